/* The C part of the oracle (oracle/ndft.c) and of the CPU timing baseline
 * (baseline/cpu_nfft.cpp, its C ABI) under AddressSanitizer / UndefinedBehaviorSanitizer
 * (built by tests/test_host_sanitize.py): small random problems through every entry
 * point, checked by the adjoint identities <A f, y> = <f, A^H y> of the NDFT and
 * <B g, y> = <g, B^T y> of the baseline's resampling pair. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int ndft_forward(int D, const int64_t *N, int64_t J, const double *x, const double *f,
                 double *out);
int ndft_adjoint_subset(int D, const int64_t *N, int64_t J, const double *x, const double *fhat,
                        int64_t K, const int64_t *idx, double *y);
void *cpu_nfft_plan(int dtype, int D, const int64_t *N, int64_t M, const double *x, int m,
                    double sigma);
void cpu_nfft_free(int dtype, void *p);
void cpu_nfft_ntilde(int dtype, void *p, int64_t *Nt);
void cpu_nfft_pad(int dtype, void *p, const void *f, void *g);
void cpu_nfft_interp(int dtype, void *p, const void *g, void *fhat);
void cpu_nfft_spread(int dtype, void *p, const void *fhat, void *g);
void cpu_nfft_crop(int dtype, void *p, const void *g, void *y);

static double rnd(void) { return rand() / (double)RAND_MAX - 0.5; }

/* Re <a, b> for interleaved complex arrays */
static double dot(const double *a, const double *b, int64_t n) {
    double s = 0;
    for (int64_t i = 0; i < n; ++i) s += a[2 * i] * b[2 * i] + a[2 * i + 1] * b[2 * i + 1];
    return s;
}

int main(void) {
    int fails = 0;
    for (int D = 1; D <= 3; ++D) {
        int64_t N[3] = {6, 4, 5}, J = 37, nn = 1;
        for (int d = 0; d < D; ++d) nn *= N[d];
        double *x = malloc(sizeof(double) * J * D), *f = malloc(16 * nn), *y = malloc(16 * J);
        double *af = malloc(16 * J), *ahy = malloc(16 * nn);
        int64_t *all = malloc(sizeof(int64_t) * nn);
        for (int64_t i = 0; i < nn; ++i) all[i] = i;
        for (int64_t i = 0; i < J * D; ++i) x[i] = rnd();
        for (int64_t i = 0; i < 2 * nn; ++i) f[i] = rnd();
        for (int64_t i = 0; i < 2 * J; ++i) y[i] = rnd();
        if (ndft_forward(D, N, J, x, f, af) || ndft_adjoint_subset(D, N, J, x, y, nn, all, ahy)) ++fails;
        const double l = dot(af, y, J), r = dot(f, ahy, nn);
        if (fabs(l - r) > 1e-10 * (fabs(l) + 1)) {
            printf("NDFT adjoint identity D=%d: %g vs %g\n", D, l, r);
            ++fails;
        }
        /* the baseline's resampling pair, both types */
        int64_t NB[3] = {8, 8, 8};
        for (int dt = 0; dt < 2; ++dt) {
            void *p = cpu_nfft_plan(dt, D, NB, J, x, 3, 2.0);
            int64_t Nt[3], G = 1;
            cpu_nfft_ntilde(dt, p, Nt);
            for (int d = 0; d < D; ++d) G *= Nt[d];
            const size_t cs = dt ? 16 : 8;
            char *g = malloc(cs * G), *g2 = malloc(cs * G), *v = malloc(cs * J), *w = malloc(cs * J);
            char *fb = malloc(cs * 512), *yb = malloc(cs * 512);
            for (int64_t i = 0; i < G; ++i) {
                if (dt) { ((double *)g)[2 * i] = rnd(); ((double *)g)[2 * i + 1] = rnd(); }
                else { ((float *)g)[2 * i] = (float)rnd(); ((float *)g)[2 * i + 1] = (float)rnd(); }
            }
            for (int64_t i = 0; i < J; ++i) {
                if (dt) { ((double *)v)[2 * i] = rnd(); ((double *)v)[2 * i + 1] = rnd(); }
                else { ((float *)v)[2 * i] = (float)rnd(); ((float *)v)[2 * i + 1] = (float)rnd(); }
            }
            for (int64_t i = 0; i < 512; ++i) {
                if (dt) { ((double *)fb)[2 * i] = rnd(); ((double *)fb)[2 * i + 1] = 0; }
                else { ((float *)fb)[2 * i] = (float)rnd(); ((float *)fb)[2 * i + 1] = 0; }
            }
            cpu_nfft_interp(dt, p, g, w);     /* w = B g */
            cpu_nfft_spread(dt, p, v, g2);    /* g2 = B^T v */
            cpu_nfft_pad(dt, p, fb, g2 + 0);  /* exercise pad and crop (values unchecked) */
            cpu_nfft_crop(dt, p, g2, yb);
            cpu_nfft_spread(dt, p, v, g2);
            double l2 = 0, r2 = 0, sc = 0;
            for (int64_t i = 0; i < J; ++i) {
                const double wr = dt ? ((double *)w)[2 * i] : ((float *)w)[2 * i];
                const double wi = dt ? ((double *)w)[2 * i + 1] : ((float *)w)[2 * i + 1];
                const double vr = dt ? ((double *)v)[2 * i] : ((float *)v)[2 * i];
                const double vi = dt ? ((double *)v)[2 * i + 1] : ((float *)v)[2 * i + 1];
                l2 += wr * vr + wi * vi;
                sc += fabs(wr * vr) + fabs(wi * vi);
            }
            for (int64_t i = 0; i < G; ++i) {
                const double gr = dt ? ((double *)g)[2 * i] : ((float *)g)[2 * i];
                const double gi = dt ? ((double *)g)[2 * i + 1] : ((float *)g)[2 * i + 1];
                const double hr = dt ? ((double *)g2)[2 * i] : ((float *)g2)[2 * i];
                const double hi = dt ? ((double *)g2)[2 * i + 1] : ((float *)g2)[2 * i + 1];
                r2 += gr * hr + gi * hi;
            }
            if (fabs(l2 - r2) > (dt ? 1e-10 : 1e-4) * (sc + 1)) {
                printf("baseline resampling adjointness D=%d dt=%d: %g vs %g\n", D, dt, l2, r2);
                ++fails;
            }
            free(g); free(g2); free(v); free(w); free(fb); free(yb);
            cpu_nfft_free(dt, p);
        }
        free(x); free(f); free(y); free(af); free(ahy); free(all);
    }
    printf("fails %d\n", fails);
    return fails;
}
