// Plan-time FP64 precomputation on the GPU: Kaiser-Bessel deconvolution factors,
// the piecewise-polynomial window table, and FFT twiddles.
#include <math.h>

#include "common.hpp"
#include "nfft_internal.hpp"

namespace nfft {

// I0 by its ascending power series sum_k ((z/2)^2)^k / (k!)^2 (Abramowitz and
// Stegun 9.6.10).  All terms are positive, so there is no cancellation; the
// series is summed until a term no longer changes the sum.
__device__ double bessel_i0_series(double z) {
    const double q = 0.25 * z * z;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 1000; ++k) {
        term *= q / ((double)k * (double)k);
        const double next = sum + term;
        if (next == sum) break;
        sum = next;
    }
    return sum;
}

// Kaiser-Bessel window on the convolution side, psi_hat_Base(u) =
// sinh(beta sqrt(1-u^2)) / (pi sqrt(1-u^2)); its value where sqrt(1-u^2) = 0 is
// the limit beta/pi.
__device__ double window_hat_fp64(double u, double beta) {
    const double s2 = 1.0 - u * u;
    const double s = s2 > 0.0 ? sqrt(s2) : 0.0;
    return s > 0.0 ? sinh(beta * s) / (M_PI * s) : beta / M_PI;
}

// The same Fourier transform on the whole line: for |u| > 1 its continuation
// sin(beta sqrt(u^2-1)) / (pi sqrt(u^2-1)), sampled by the wide stencil.
__device__ double window_hat_full_fp64(double u, double beta) {
    const double q = 1.0 - u * u;
    const double r = sqrt(fabs(q));
    if (r == 0.0) return beta / M_PI;
    return q > 0.0 ? sinh(beta * r) / (M_PI * r) : sin(beta * r) / (M_PI * r);
}

// Resampling-correction factors of one axis (paper, subsection "Resampling
// Correction"): beta_tensor[n] = 1 / (m phi_Base(m n / Nt)), n in I_N, with
// phi_Base(xi) = I0(sqrt(beta^2 - (2 pi xi)^2)), times the window peak
// sinh(beta)/pi that the stored window is divided by.  Computed in FP64, stored in T.
template <typename T>
__global__ void k_deconv_factors(int N, int Nt, int m, double beta, double peak, T *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double n = (double)(i - N / 2);
    const double a = 2.0 * M_PI * (double)m * n / (double)Nt;
    const double arg = beta * beta - a * a;  // >= 0 because sigma >= 1
    const double phi = bessel_i0_series(sqrt(arg > 0.0 ? arg : 0.0));
    out[i] = (T)(peak / ((double)m * phi));
}

// Polynomial window table (paper, POLYNOMIAL item of subsection "Window
// precomputation"): for tap t = 0..2m-1 fit P_t(zeta) = sum_z mu[t][z] zeta^z,
// zeta = frac - 1/2, to Theta equispaced samples of psi_hat_Base((zeta + m -
// 1/2 - t)/m) by least squares.  The fit is done in the variable s = 2 zeta in
// [-1, 1] with the thin QR factors of its Vandermonde matrix (qt = Q^T, Z x
// Theta; r = R, Z x Z upper), then rescaled exactly by 2^z.  One thread per
// (axis, tap); FP64 throughout, stored in T.  With the wide stencil (taps =
// 2m + 2, lo = m) tap t samples the untruncated window at (zeta + m + 1/2 - t)/m.
// The samples are divided by the window peak inv_peaks[axis]^-1 = sinh(beta)/pi.
template <typename T>
__global__ void k_window_poly(int m, int taps, int Z, int Theta, const double *betas,
                              const double *inv_peaks, const double *qt, const double *r, T *mu) {
    const int t = threadIdx.x;
    const int axis = blockIdx.x;
    if (t >= taps) return;
    const int lo = taps / 2 - 1;
    const bool wide = taps > 2 * m;
    const double beta = betas[axis];
    const double inv_peak = inv_peaks[axis];
    double c[32];
    for (int z = 0; z < Z; ++z) c[z] = 0.0;
    for (int v = 0; v < Theta; ++v) {
        const double zeta = -0.5 + (double)v / (double)(Theta - 1);
        const double u = (zeta + (double)lo + 0.5 - (double)t) / (double)m;
        const double b =
            (wide ? window_hat_full_fp64(u, beta) : window_hat_fp64(u, beta)) * inv_peak;
        for (int z = 0; z < Z; ++z) c[z] += qt[z * Theta + v] * b;
    }
    double sol[32];
    for (int z = Z - 1; z >= 0; --z) {
        double acc = c[z];
        for (int k = z + 1; k < Z; ++k) acc -= r[z * Z + k] * sol[k];
        sol[z] = acc / r[z * Z + z];
    }
    double scale = 1.0;
    for (int z = 0; z < Z; ++z) {
        mu[((size_t)axis * taps + t) * Z + z] = (T)(sol[z] * scale);
        scale *= 2.0;
    }
}

// LINEAR window table (paper, LINEAR item of subsection "Window
// precomputation"): psi_s = psi_hat_Base(s / (S - 2)) for s <= S - 2 (the sinh
// form, whose value at |u| = 1 is the limit beta/pi, the half-open support's
// value at u = -1) and psi_{S-1} = 0, outside the support; divided by the window
// peak (times inv_peak).  FP64, stored in T.
template <typename T>
__global__ void k_window_linear(long long S, double beta, double inv_peak, T *table) {
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    table[s] = s == S - 1
                   ? (T)0
                   : (T)(window_hat_fp64((double)s / (double)(S - 2), beta) * inv_peak);
}

// Polynomial window weight of tap t at offset frac, evaluated like the
// resampling kernels do (Horner in T on zeta = frac - 1/2).
template <typename T>
__device__ inline T poly_weight(const T *mu, int Z, T frac) {
    const T z = frac - (T)0.5;
    T acc = mu[Z - 1];
    for (int k = Z - 2; k >= 0; --k) acc = fma(acc, z, mu[k]);
    return acc;
}

// TENSOR precomputation: per sorted node k, axis d, tap t, the window weight
// (polynomial window, as the paper combines TENSOR with it):
// out[(k D + d) 2m + t].  FULL (D <= 2): per sorted node the (2m)^D products
// out[k (2m)^D + a 2m + b] = w_0[a] w_1[b] (1-D: the 2m weights).
template <typename T, int D>
__global__ void k_window_nodes(const NodeRec<T, D> *nodes, long long M, int m, int taps,
                               const T *mu, int full, T *out) {
    const int M2 = taps, Z = 2 * m + 1;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (!full) {
        if (i >= M * D * M2) return;
        const long long k = i / (D * M2);
        const int r = (int)(i - k * D * M2), d = r / M2, t = r - d * M2;
        out[i] = poly_weight(mu + ((size_t)d * M2 + t) * Z, Z, nodes[k].fr[d]);
    } else if (D == 1) {
        if (i >= M * M2) return;
        const long long k = i / M2;
        const int t = (int)(i - k * M2);
        out[i] = poly_weight(mu + (size_t)t * Z, Z, nodes[k].fr[0]);
    } else {
        if (i >= M * M2 * M2) return;
        const long long k = i / (M2 * M2);
        const int r = (int)(i - k * M2 * M2), a = r / M2, b = r - a * M2;
        out[i] = poly_weight(mu + (size_t)a * Z, Z, nodes[k].fr[0]) *
                 poly_weight(mu + ((size_t)M2 + b) * Z, Z, nodes[k].fr[D - 1]);
    }
}

// Twiddle table exp(-2 pi i t / L), t = 0..L-1, evaluated in FP64.
template <typename T>
__global__ void k_twiddles(int L, cplx<T> *tw) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= L) return;
    double s, c;
    sincospi(2.0 * (double)t / (double)L, &s, &c);
    tw[t] = cmake<cplx<T>>((T)c, (T)(-s));
}

hipError_t launch_deconv_factors(const nfft_plan_s &p, hipStream_t s) {
    for (int d = 0; d < p.D; ++d) {
        const int N = (int)p.N[d];
        const int blocks = (N + 255) / 256;
        if (p.dtype == NFFT_C64)
            hipLaunchKernelGGL(k_deconv_factors<float>, dim3(blocks), dim3(256), 0, s, N,
                               (int)p.Nt[d], p.m, kb_beta(p, d), window_peak(p, d),
                               (float *)p.deconv[d]);
        else
            hipLaunchKernelGGL(k_deconv_factors<double>, dim3(blocks), dim3(256), 0, s, N,
                               (int)p.Nt[d], p.m, kb_beta(p, d), window_peak(p, d),
                               (double *)p.deconv[d]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_window_poly(const nfft_plan_s &p, const double *qt, const double *r, int Z,
                              int Theta, hipStream_t s) {
    // betas, the reciprocal window peaks, qt and r live in one device scratch
    // allocation owned by the caller
    const double *betas = r + Z * Z;
    const double *inv_peaks = betas + kMaxD;
    if (p.dtype == NFFT_C64)
        hipLaunchKernelGGL(k_window_poly<float>, dim3(p.D), dim3(64), 0, s, p.m, p.geom.taps, Z,
                           Theta, betas, inv_peaks, qt, r, (float *)p.coef);
    else
        hipLaunchKernelGGL(k_window_poly<double>, dim3(p.D), dim3(64), 0, s, p.m, p.geom.taps, Z,
                           Theta, betas, inv_peaks, qt, r, (double *)p.coef);
    return hipGetLastError();
}

hipError_t launch_window_tables(const nfft_plan_s &p, hipStream_t s) {
    if (p.window == NFFT_WINDOW_LINEAR) {
        // one table per axis: beta depends on sigma_d
        for (int d = 0; d < p.D; ++d) {
            const unsigned blocks = (unsigned)((p.lin_S + 255) / 256);
            if (p.dtype == NFFT_C64)
                hipLaunchKernelGGL(k_window_linear<float>, dim3(blocks), dim3(256), 0, s, p.lin_S,
                                   kb_beta(p, d), 1.0 / window_peak(p, d),
                                   (float *)p.wtab + (size_t)d * p.lin_S);
            else
                hipLaunchKernelGGL(k_window_linear<double>, dim3(blocks), dim3(256), 0, s, p.lin_S,
                                   kb_beta(p, d), 1.0 / window_peak(p, d),
                                   (double *)p.wtab + (size_t)d * p.lin_S);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (p.window != NFFT_WINDOW_TENSOR && p.window != NFFT_WINDOW_FULL) return hipSuccess;
    if (p.M == 0) return hipSuccess;
    const int full = p.window == NFFT_WINDOW_FULL;
    const long long tp = p.geom.taps;
    const long long per = full ? (p.D == 1 ? tp : tp * tp) : (long long)p.D * tp;
    const long long n = p.M * per;
    const dim3 g((unsigned)((n + 255) / 256));
#define NFFT_WT(T, DD)                                                                            \
    hipLaunchKernelGGL((k_window_nodes<T, DD>), g, dim3(256), 0, s,                               \
                       (const NodeRec<T, DD> *)p.nodes, (long long)p.M, p.m, p.geom.taps,       \
                       (const T *)p.coef,                                                         \
                       full, (T *)p.wtab)
    if (p.dtype == NFFT_C64) {
        if (p.D == 1) NFFT_WT(float, 1);
        else if (p.D == 2) NFFT_WT(float, 2);
        else if (p.D == 3) NFFT_WT(float, 3);
        else if (p.D == 4) NFFT_WT(float, 4);
        else if (p.D == 5) NFFT_WT(float, 5);
        else NFFT_WT(float, 6);
    } else {
        if (p.D == 1) NFFT_WT(double, 1);
        else if (p.D == 2) NFFT_WT(double, 2);
        else if (p.D == 3) NFFT_WT(double, 3);
        else if (p.D == 4) NFFT_WT(double, 4);
        else if (p.D == 5) NFFT_WT(double, 5);
        else NFFT_WT(double, 6);
    }
#undef NFFT_WT
    return hipGetLastError();
}

hipError_t launch_twiddles(const nfft_plan_s &p, int axis, hipStream_t s) {
    const int L = (int)p.Nt[axis];
    const int blocks = (L + 255) / 256;
    if (p.dtype == NFFT_C64)
        hipLaunchKernelGGL(k_twiddles<float>, dim3(blocks), dim3(256), 0, s, L,
                           (float2 *)p.twiddle[axis]);
    else
        hipLaunchKernelGGL(k_twiddles<double>, dim3(blocks), dim3(256), 0, s, L,
                           (double2 *)p.twiddle[axis]);
    return hipGetLastError();
}

}  // namespace nfft
