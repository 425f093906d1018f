// Plain multi-threaded CPU NFFT (a timing baseline for bench.py; not the oracle and
// not part of the GPU library).
//
// The steps of the paper's Algorithms 1 and 2 apart from the FFT, which the Python
// side does with scipy.fft over all host cores:
//   * plan: oversampled size, per-axis resampling-correction factors
//     1 / (m I0(sqrt(beta^2 - (2 pi m n / Nt)^2))), the node cells, and per node and
//     axis the 2m window values psi_hat_Base((frac + m - 1 - t)/m) (the paper's
//     TENSOR precomputation), with beta = pi m (2 - 1/sigma); nodes counted into
//     their stencil's first axis-0 plane (a counting sort);
//   * forward: correction + zero padding into the grid (fftshift folded in), then
//     after the FFT the interpolation, in parallel over the sorted nodes;
//   * adjoint: spreading, each thread owning a range of axis-0 planes and adding
//     the taps of every node whose stencil reaches them (no atomics), then after
//     the FFT the crop + correction.
// T = double (complex128) or float (complex64: FP32 arithmetic and grid).
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace {

int64_t smooth_even(double target) {
    int64_t c = (int64_t)std::ceil(target - 1e-9 * target);
    if (c % 2) ++c;
    for (;; c += 2) {
        int64_t v = c;
        for (int p : {2, 3, 5})
            while (v % p == 0) v /= p;
        if (v == 1) return c;
    }
}

template <typename T> struct Plan {
    int D, m, taps;
    int64_t N[3], Nt[3], M, G, NN;
    std::vector<T> dec[3];       // N_d correction factors per axis
    std::vector<int> order;      // sorted position -> node index
    std::vector<int> org;        // per sorted node and axis: stencil origin (mod Nt)
    std::vector<T> wt;           // per sorted node, axis, tap: window value
    std::vector<int64_t> start;  // Nt_0 + 1: first sorted node of each origin plane
};

double kb_hat(double u, double beta) {  // sinh(beta sqrt(1-u^2)) / (pi sqrt(1-u^2)), |u| <= 1
    const double s2 = 1.0 - u * u;
    if (s2 <= 0.0) return beta / M_PI;
    const double s = std::sqrt(s2);
    return std::sinh(beta * s) / (M_PI * s);
}

template <typename T>
Plan<T> *make_plan(int D, const int64_t *N, int64_t M, const double *x, int m, double sigma) {
    Plan<T> *p = new Plan<T>();
    p->D = D;
    p->m = m;
    p->taps = 2 * m;
    p->M = M;
    p->G = p->NN = 1;
    for (int d = 0; d < 3; ++d) {
        p->N[d] = d < D ? N[d] : 1;
        p->Nt[d] = d < D ? smooth_even(sigma * (double)N[d]) : 1;
        p->G *= p->Nt[d];
        p->NN *= p->N[d];
    }
    for (int d = 0; d < D; ++d) {
        const double beta = M_PI * m * (2.0 - (double)p->N[d] / (double)p->Nt[d]);
        p->dec[d].resize(p->N[d]);
        for (int64_t i = 0; i < p->N[d]; ++i) {
            const double n = (double)(i - p->N[d] / 2);
            const double a = 2.0 * M_PI * m * n / (double)p->Nt[d];
            p->dec[d][i] = (T)(1.0 / (m * std::cyl_bessel_i(0.0, std::sqrt(beta * beta - a * a))));
        }
    }
    // cells and the counting sort by the first axis-0 plane of the stencil
    const int taps = p->taps;
    std::vector<int> o((size_t)M * D);
    std::vector<double> fr((size_t)M * D);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < M; ++j)
        for (int d = 0; d < D; ++d) {
            const double xv = x[j * D + d] - std::floor(x[j * D + d] + 0.5);
            const double y = xv * (double)p->Nt[d];
            const double c = std::floor(y);
            int64_t oo = ((int64_t)c - (m - 1)) % p->Nt[d];
            if (oo < 0) oo += p->Nt[d];
            o[j * D + d] = (int)oo;
            fr[j * D + d] = y - c;
        }
    p->start.assign(p->Nt[0] + 1, 0);
    for (int64_t j = 0; j < M; ++j) ++p->start[o[j * D] + 1];
    for (int64_t i = 0; i < p->Nt[0]; ++i) p->start[i + 1] += p->start[i];
    std::vector<int64_t> cur(p->start.begin(), p->start.end() - 1);
    p->order.resize(M);
    for (int64_t j = 0; j < M; ++j) p->order[cur[o[j * D]]++] = (int)j;
    p->org.resize((size_t)M * D);
    p->wt.resize((size_t)M * D * taps);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < M; ++s) {
        const int64_t j = p->order[s];
        for (int d = 0; d < D; ++d) {
            const double beta = M_PI * m * (2.0 - (double)p->N[d] / (double)p->Nt[d]);
            p->org[s * D + d] = o[j * D + d];
            for (int t = 0; t < taps; ++t)
                p->wt[(s * D + d) * taps + t] = (T)kb_hat((fr[j * D + d] + m - 1 - t) / m, beta);
        }
    }
    return p;
}

template <typename T> using cx = std::complex<T>;

// grid (Nt, zeroed here) <- f * correction at (n mod Nt)
template <typename T> void pad(const Plan<T> &p, const cx<T> *f, cx<T> *g) {
    memset((void *)g, 0, sizeof(cx<T>) * p.G);
    const int64_t N1 = p.N[1], N2 = p.N[2];
#pragma omp parallel for schedule(static)
    for (int64_t i0 = 0; i0 < p.N[0]; ++i0) {
        const int64_t l0 = (i0 - p.N[0] / 2 + p.Nt[0]) % p.Nt[0];
        for (int64_t i1 = 0; i1 < N1; ++i1) {
            const int64_t l1 = p.D > 1 ? (i1 - N1 / 2 + p.Nt[1]) % p.Nt[1] : 0;
            const T c01 = p.dec[0][i0] * (p.D > 1 ? p.dec[1][i1] : (T)1);
            for (int64_t i2 = 0; i2 < N2; ++i2) {
                const int64_t l2 = p.D > 2 ? (i2 - N2 / 2 + p.Nt[2]) % p.Nt[2] : 0;
                const T c = c01 * (p.D > 2 ? p.dec[2][i2] : (T)1);
                g[(l0 * p.Nt[1] + l1) * p.Nt[2] + l2] = f[(i0 * N1 + i1) * N2 + i2] * c;
            }
        }
    }
}

// y <- grid at (n mod Nt) * correction
template <typename T> void crop(const Plan<T> &p, const cx<T> *g, cx<T> *y) {
    const int64_t N1 = p.N[1], N2 = p.N[2];
#pragma omp parallel for schedule(static)
    for (int64_t i0 = 0; i0 < p.N[0]; ++i0) {
        const int64_t l0 = (i0 - p.N[0] / 2 + p.Nt[0]) % p.Nt[0];
        for (int64_t i1 = 0; i1 < N1; ++i1) {
            const int64_t l1 = p.D > 1 ? (i1 - N1 / 2 + p.Nt[1]) % p.Nt[1] : 0;
            const T c01 = p.dec[0][i0] * (p.D > 1 ? p.dec[1][i1] : (T)1);
            for (int64_t i2 = 0; i2 < N2; ++i2) {
                const int64_t l2 = p.D > 2 ? (i2 - N2 / 2 + p.Nt[2]) % p.Nt[2] : 0;
                const T c = c01 * (p.D > 2 ? p.dec[2][i2] : (T)1);
                y[(i0 * N1 + i1) * N2 + i2] = g[(l0 * p.Nt[1] + l1) * p.Nt[2] + l2] * c;
            }
        }
    }
}

template <typename T> void interp(const Plan<T> &p, const cx<T> *g, cx<T> *fhat) {
    const int D = p.D, taps = p.taps;
    const int64_t Nt0 = p.Nt[0], Nt1 = p.Nt[1], Nt2 = p.Nt[2];
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < p.M; ++s) {
        const int *o = &p.org[s * D];
        const T *w = &p.wt[s * D * taps];
        cx<T> acc = 0;
        for (int a = 0; a < taps; ++a) {
            const int64_t l0 = (o[0] + a) % Nt0;
            if (D == 1) {
                acc += w[a] * g[l0];
                continue;
            }
            cx<T> acc1 = 0;
            for (int b = 0; b < taps; ++b) {
                const int64_t l1 = (o[1] + b) % Nt1;
                if (D == 2) {
                    acc1 += w[taps + b] * g[l0 * Nt1 + l1];
                    continue;
                }
                const cx<T> *row = g + (l0 * Nt1 + l1) * Nt2;
                cx<T> acc2 = 0;
                for (int c = 0; c < taps; ++c) acc2 += w[2 * taps + c] * row[(o[2] + c) % Nt2];
                acc1 += w[taps + b] * acc2;
            }
            acc += w[a] * acc1;
        }
        fhat[p.order[s]] = acc;
    }
}

template <typename T> void spread(const Plan<T> &p, const cx<T> *fhat, cx<T> *g) {
    memset((void *)g, 0, sizeof(cx<T>) * p.G);
    const int D = p.D, taps = p.taps;
    const int64_t Nt0 = p.Nt[0], Nt1 = p.Nt[1], Nt2 = p.Nt[2];
#pragma omp parallel
    {
        // this thread owns axis-0 planes [lo, hi) and visits the nodes whose first
        // plane lies in [lo - taps + 1, hi) (cyclically)
        const int nth = omp_get_num_threads(), th = omp_get_thread_num();
        const int64_t lo = Nt0 * th / nth, hi = Nt0 * (th + 1) / nth;
        if (hi > lo) {
            for (int64_t q = lo - taps + 1; q < hi; ++q) {
                const int64_t pl = ((q % Nt0) + Nt0) % Nt0;
                for (int64_t s = p.start[pl]; s < p.start[pl + 1]; ++s) {
                    const int *o = &p.org[s * D];
                    const T *w = &p.wt[s * D * taps];
                    const cx<T> v = fhat[p.order[s]];
                    for (int a = 0; a < taps; ++a) {
                        const int64_t u = q + a;  // unwrapped plane
                        if (u < lo || u >= hi) continue;
                        const int64_t l0 = ((u % Nt0) + Nt0) % Nt0;
                        const cx<T> va = v * w[a];
                        if (D == 1) {
                            g[l0] += va;
                            continue;
                        }
                        for (int b = 0; b < taps; ++b) {
                            const int64_t l1 = (o[1] + b) % Nt1;
                            const cx<T> vb = va * w[taps + b];
                            if (D == 2) {
                                g[l0 * Nt1 + l1] += vb;
                                continue;
                            }
                            cx<T> *row = g + (l0 * Nt1 + l1) * Nt2;
                            for (int c = 0; c < taps; ++c) row[(o[2] + c) % Nt2] += vb * w[2 * taps + c];
                        }
                    }
                }
            }
        }
    }
}

}  // namespace

extern "C" {

// dtype 0: complex64 (float), 1: complex128 (double).  Returns an opaque plan or NULL.
void *cpu_nfft_plan(int dtype, int D, const int64_t *N, int64_t M, const double *x, int m,
                    double sigma) {
    if (D < 1 || D > 3 || M < 0 || m < 1) return nullptr;
    if (dtype == 1) return make_plan<double>(D, N, M, x, m, sigma);
    return make_plan<float>(D, N, M, x, m, sigma);
}

void cpu_nfft_free(int dtype, void *p) {
    if (dtype == 1) delete (Plan<double> *)p;
    else delete (Plan<float> *)p;
}

void cpu_nfft_ntilde(int dtype, void *p, int64_t *Nt) {
    for (int d = 0; d < 3; ++d) Nt[d] = dtype == 1 ? ((Plan<double> *)p)->Nt[d] : ((Plan<float> *)p)->Nt[d];
}

// step 1 of Algorithm 1: f (N, complex) -> grid (Nt, complex)
void cpu_nfft_pad(int dtype, void *p, const void *f, void *g) {
    if (dtype == 1) pad(*(Plan<double> *)p, (const cx<double> *)f, (cx<double> *)g);
    else pad(*(Plan<float> *)p, (const cx<float> *)f, (cx<float> *)g);
}
// step 3 of Algorithm 1: grid -> fhat (M, caller's node order)
void cpu_nfft_interp(int dtype, void *p, const void *g, void *fhat) {
    if (dtype == 1) interp(*(Plan<double> *)p, (const cx<double> *)g, (cx<double> *)fhat);
    else interp(*(Plan<float> *)p, (const cx<float> *)g, (cx<float> *)fhat);
}
// step 1 of Algorithm 2: fhat -> grid
void cpu_nfft_spread(int dtype, void *p, const void *fhat, void *g) {
    if (dtype == 1) spread(*(Plan<double> *)p, (const cx<double> *)fhat, (cx<double> *)g);
    else spread(*(Plan<float> *)p, (const cx<float> *)fhat, (cx<float> *)g);
}
// step 3 of Algorithm 2: grid -> y (N)
void cpu_nfft_crop(int dtype, void *p, const void *g, void *y) {
    if (dtype == 1) crop(*(Plan<double> *)p, (const cx<double> *)g, (cx<double> *)y);
    else crop(*(Plan<float> *)p, (const cx<float> *)g, (cx<float> *)y);
}

int cpu_nfft_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
