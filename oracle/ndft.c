/*
 * Direct NDFT oracle in FP64 -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load this code.  The GPU library never links or calls it, and it shares no
 * code with the GPU library.
 *
 * What it computes (paper, section "Mathematical Description", subsection NDFT):
 *
 *   forward (type 2, equation (NDFT)):
 *       fhat_j = sum_{n in I_N} f_n * exp(-2*pi*i * n . k_j),      j = 0..J-1
 *   adjoint (type 1, equation (NDFTH)):
 *       y_n    = sum_{j}        fhat_j * exp(+2*pi*i * n . k_j),   n in I_N
 *
 * I_N is the centred index set: n_d runs over -N_d/2 .. N_d/2-1 (even N_d), and
 * the coefficient array is stored row-major (last axis fastest) with storage
 * index i_d = n_d + N_d/2.  Nodes k_j are stored node-major: k[j*D + d].
 *
 * Phase factors are evaluated per dimension from the product t = n_d * k_{d,j}
 * (in turns), reduced exactly to [-1/2, 1/2] before calling cos/sin, so the phase
 * error is about one rounding of t (<= 1e-13 rad for |n_d| <= 512).  No
 * recurrences are used.  Sums are plain sequential sums.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define MAXD 6

#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the oracle's parallel loops use. */
int ndft_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* cos and sin of 2*pi*t, t in turns, with exact reduction of t to [-1/2, 1/2]. */
static void cis_turns(double t, double *c, double *s)
{
    double r = t - nearbyint(t); /* exact: |t| < 2^52 */
    double a = 2.0 * M_PI * r;
    *c = cos(a);
    *s = sin(a);
}

/*
 * Nested sum over the axes d..D-1 of one node's row factors times f
 * (interleaved re/im).  rows[d] holds N_d complex factors for axis d.
 */
static void nested_sum(int d, int D, const int64_t *N, const int64_t *stride,
                       const double *f, double *const *rows, double *re, double *im)
{
    double ar = 0.0, ai = 0.0;
    const double *row = rows[d];
    if (d == D - 1) {
        for (int64_t i = 0; i < N[d]; ++i) {
            double fr = f[2 * i], fi = f[2 * i + 1];
            double wr = row[2 * i], wi = row[2 * i + 1];
            ar += wr * fr - wi * fi;
            ai += wr * fi + wi * fr;
        }
    } else {
        for (int64_t i = 0; i < N[d]; ++i) {
            double sr, si;
            nested_sum(d + 1, D, N, stride, f + 2 * i * stride[d], rows, &sr, &si);
            double wr = row[2 * i], wi = row[2 * i + 1];
            ar += wr * sr - wi * si;
            ai += wr * si + wi * sr;
        }
    }
    *re = ar;
    *im = ai;
}

/*
 * Forward NDFT at J nodes.  f: prod(N) complex (interleaved), fhat: J complex.
 * Returns 0 on success, -1 on bad arguments.
 */
int ndft_forward(int D, const int64_t *N, int64_t J, const double *k,
                 const double *f, double *fhat)
{
    if (D < 1 || D > MAXD || J < 0) return -1;
    int64_t stride[MAXD];
    int64_t total = 1;
    for (int d = D - 1; d >= 0; --d) {
        if (N[d] < 1) return -1;
        stride[d] = total;
        total *= N[d];
    }
    int64_t rowlen = 0;
    for (int d = 0; d < D; ++d) rowlen += N[d];

#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 2 * (size_t)rowlen);
        double *rows[MAXD];
        int64_t off = 0;
        for (int d = 0; d < D; ++d) {
            rows[d] = buf + 2 * off;
            off += N[d];
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < J; ++j) {
            for (int d = 0; d < D; ++d) {
                double kd = k[j * D + d];
                int64_t half = N[d] / 2;
                for (int64_t i = 0; i < N[d]; ++i) {
                    double n = (double)(i - half);
                    double c, s;
                    cis_turns(n * kd, &c, &s);
                    rows[d][2 * i] = c;       /* exp(-2 pi i n k) = cos - i sin */
                    rows[d][2 * i + 1] = -s;
                }
            }
            nested_sum(0, D, N, stride, f, rows, &fhat[2 * j], &fhat[2 * j + 1]);
        }
        free(buf);
    }
    return 0;
}

/*
 * Adjoint NDFT at K selected coefficient positions idx[0..K-1] (flat storage
 * indices into the prod(N) array).  y: K complex.  For the full adjoint pass
 * idx = 0..prod(N)-1.
 */
int ndft_adjoint_subset(int D, const int64_t *N, int64_t J, const double *k,
                        const double *fhat, int64_t K, const int64_t *idx, double *y)
{
    if (D < 1 || D > MAXD || J < 0 || K < 0) return -1;
    int64_t stride[MAXD];
    int64_t total = 1;
    for (int d = D - 1; d >= 0; --d) {
        if (N[d] < 1) return -1;
        stride[d] = total;
        total *= N[d];
    }
    for (int64_t q = 0; q < K; ++q)
        if (idx[q] < 0 || idx[q] >= total) return -1;

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < K; ++q) {
        double n[MAXD];
        int64_t rem = idx[q];
        for (int d = 0; d < D; ++d) {
            int64_t i = rem / stride[d];
            rem -= i * stride[d];
            n[d] = (double)(i - N[d] / 2);
        }
        double ar = 0.0, ai = 0.0;
        for (int64_t j = 0; j < J; ++j) {
            /* exp(+2 pi i n.k) as the product of per-axis factors */
            double pr = 1.0, pi = 0.0;
            for (int d = 0; d < D; ++d) {
                double c, s;
                cis_turns(n[d] * k[j * D + d], &c, &s);
                double tr = pr * c - pi * s;
                double ti = pr * s + pi * c;
                pr = tr;
                pi = ti;
            }
            double fr = fhat[2 * j], fi = fhat[2 * j + 1];
            ar += pr * fr - pi * fi;
            ai += pr * fi + pi * fr;
        }
        y[2 * q] = ar;
        y[2 * q + 1] = ai;
    }
    return 0;
}
