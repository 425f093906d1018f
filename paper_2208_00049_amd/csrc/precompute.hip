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

// Resampling-correction factors of one axis (paper, subsection "Resampling
// Correction"): beta_tensor[n] = 1 / (m phi_Base(m n / Nt)), n in I_N, with
// phi_Base(xi) = I0(sqrt(beta^2 - (2 pi xi)^2)).  Computed in FP64, stored in T.
template <typename T>
__global__ void k_deconv_factors(int N, int Nt, int m, double beta, T *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double n = (double)(i - N / 2);
    const double a = 2.0 * M_PI * (double)m * n / (double)Nt;
    const double arg = beta * beta - a * a;  // >= 0 because sigma >= 1
    const double phi = bessel_i0_series(sqrt(arg > 0.0 ? arg : 0.0));
    out[i] = (T)(1.0 / ((double)m * phi));
}

// Polynomial window table (paper, POLYNOMIAL item of subsection "Window
// precomputation"): for tap t = 0..2m-1 fit P_t(zeta) = sum_z mu[t][z] zeta^z,
// zeta = frac - 1/2, to Theta equispaced samples of psi_hat_Base((zeta + m -
// 1/2 - t)/m) by least squares.  The fit is done in the variable s = 2 zeta in
// [-1, 1] with the thin QR factors of its Vandermonde matrix (qt = Q^T, Z x
// Theta; r = R, Z x Z upper), then rescaled exactly by 2^z.  One thread per
// (axis, tap); FP64 throughout, stored in T.
template <typename T>
__global__ void k_window_poly(int m, int Z, int Theta, const double *betas, const double *qt,
                              const double *r, T *mu) {
    const int t = threadIdx.x;
    const int axis = blockIdx.x;
    if (t >= 2 * m) return;
    const double beta = betas[axis];
    double c[32];
    for (int z = 0; z < Z; ++z) c[z] = 0.0;
    for (int v = 0; v < Theta; ++v) {
        const double zeta = -0.5 + (double)v / (double)(Theta - 1);
        const double b = window_hat_fp64((zeta + (double)m - 0.5 - (double)t) / (double)m, beta);
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
        mu[((size_t)axis * 2 * m + t) * Z + z] = (T)(sol[z] * scale);
        scale *= 2.0;
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

static double kb_beta(const nfft_plan_s &p, int d) {
    return M_PI * p.m * (2.0 - (double)p.N[d] / (double)p.Nt[d]);
}

hipError_t launch_deconv_factors(const nfft_plan_s &p, hipStream_t s) {
    for (int d = 0; d < p.D; ++d) {
        const int N = (int)p.N[d];
        const int blocks = (N + 255) / 256;
        if (p.dtype == NFFT_C64)
            hipLaunchKernelGGL(k_deconv_factors<float>, dim3(blocks), dim3(256), 0, s, N,
                               (int)p.Nt[d], p.m, kb_beta(p, d), (float *)p.deconv[d]);
        else
            hipLaunchKernelGGL(k_deconv_factors<double>, dim3(blocks), dim3(256), 0, s, N,
                               (int)p.Nt[d], p.m, kb_beta(p, d), (double *)p.deconv[d]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_window_poly(const nfft_plan_s &p, const double *qt, const double *r, int Z,
                              int Theta, hipStream_t s) {
    // betas, qt and r live in one device scratch allocation owned by the caller
    const double *betas = r + Z * Z;
    if (p.dtype == NFFT_C64)
        hipLaunchKernelGGL(k_window_poly<float>, dim3(p.D), dim3(64), 0, s, p.m, Z, Theta, betas,
                           qt, r, (float *)p.coef);
    else
        hipLaunchKernelGGL(k_window_poly<double>, dim3(p.D), dim3(64), 0, s, p.m, Z, Theta, betas,
                           qt, r, (double *)p.coef);
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
