// Instantiation and dispatch of the resampling kernels over (type, D, 2m).
#include "resample_impl.hpp"

namespace nfft {

// over the stencil points per axis (2m, or 2m + 2 with the wide stencil)
#define NFFT_DISPATCH_M(FN, T, D, ...)                     \
    switch (p.geom.taps / 2) {                             \
        case 1: return FN<T, D, 2>(__VA_ARGS__);           \
        case 2: return FN<T, D, 4>(__VA_ARGS__);           \
        case 3: return FN<T, D, 6>(__VA_ARGS__);           \
        case 4: return FN<T, D, 8>(__VA_ARGS__);           \
        case 5: return FN<T, D, 10>(__VA_ARGS__);          \
        case 6: return FN<T, D, 12>(__VA_ARGS__);          \
        case 7: return FN<T, D, 14>(__VA_ARGS__);          \
        case 8: return FN<T, D, 16>(__VA_ARGS__);          \
        case 9: return FN<T, D, 18>(__VA_ARGS__);          \
        case 10: return FN<T, D, 20>(__VA_ARGS__);         \
        case 11: return FN<T, D, 22>(__VA_ARGS__);         \
        default: return hipErrorInvalidValue;              \
    }

template <typename T>
static hipError_t interp_t(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s,
                           int K) {
    switch (p.D) {
        case 1: NFFT_DISPATCH_M(run_interp, T, 1, p, grid, fhat, s, K)
        case 2: NFFT_DISPATCH_M(run_interp, T, 2, p, grid, fhat, s, K)
        case 3: NFFT_DISPATCH_M(run_interp, T, 3, p, grid, fhat, s, K)
        case 4:
        case 5:
        case 6: return launch_interp_nd(p, grid, fhat, s, K);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t interp_deriv_t(const nfft_plan_s &p, const void *grid, void *dfhat,
                                 hipStream_t s) {
    switch (p.D) {
        case 1: NFFT_DISPATCH_M(run_interp_deriv, T, 1, p, grid, dfhat, s)
        case 2: NFFT_DISPATCH_M(run_interp_deriv, T, 2, p, grid, dfhat, s)
        case 3: NFFT_DISPATCH_M(run_interp_deriv, T, 3, p, grid, dfhat, s)
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t spread_t(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s,
                           bool merge, int K, void *pad) {
    switch (p.D) {
        case 1: NFFT_DISPATCH_M(run_spread, T, 1, p, fhat, grid, s, merge, K, pad)
        case 2: NFFT_DISPATCH_M(run_spread, T, 2, p, fhat, grid, s, merge, K, pad)
        case 3: NFFT_DISPATCH_M(run_spread, T, 3, p, fhat, grid, s, merge, K, pad)
        case 4:
        case 5:
        case 6: return launch_spread_nd(p, fhat, grid, s, K);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_interp(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s, int K) {
    if (p.nsub == 0) return hipSuccess;
    if (p.sweep.on && p.dtype == NFFT_C128) return launch_interp_sweep(p, grid, fhat, s, K);
    return p.dtype == NFFT_C64 ? interp_t<float>(p, grid, fhat, s, K)
                               : interp_t<double>(p, grid, fhat, s, K);
}

hipError_t launch_interp_deriv(const nfft_plan_s &p, const void *grid, void *dfhat, hipStream_t s) {
    if (p.nsub == 0) return hipSuccess;
    if (p.window != NFFT_WINDOW_POLY || p.D > 3) return hipErrorInvalidValue;
    return p.dtype == NFFT_C64 ? interp_deriv_t<float>(p, grid, dfhat, s)
                               : interp_deriv_t<double>(p, grid, dfhat, s);
}

hipError_t launch_spread(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s,
                         bool merge, int K, void *pad) {
    if (!pad) pad = p.pad;
    if (p.sweep.on) return launch_spread_sweep(p, fhat, grid, s, K, pad, merge);
    return p.dtype == NFFT_C64 ? spread_t<float>(p, fhat, grid, s, merge, K, pad)
                               : spread_t<double>(p, fhat, grid, s, merge, K, pad);
}

// Node gradient: out[j*D + d] = Re(conj(a_j) v[d*M + j]) = a.x v.x + a.y v.y.
template <typename T>
__global__ void k_node_grad(const cplx<T> *__restrict__ a, const cplx<T> *__restrict__ v,
                            T *__restrict__ out, long long M, int D) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * D) return;
    const long long j = i / D;
    const int d = (int)(i - j * D);
    const cplx<T> x = a[j], y = v[(long long)d * M + j];
    out[i] = x.x * y.x + x.y * y.y;
}

hipError_t launch_node_grad(const nfft_plan_s &p, const void *a, const void *v, void *out,
                            hipStream_t s) {
    const long long n = (long long)p.M * p.D;
    if (n == 0) return hipSuccess;
    const dim3 g((unsigned)((n + 255) / 256));
    if (p.dtype == NFFT_C64)
        hipLaunchKernelGGL(k_node_grad<float>, g, dim3(256), 0, s, (const cplx<float> *)a,
                           (const cplx<float> *)v, (float *)out, (long long)p.M, p.D);
    else
        hipLaunchKernelGGL(k_node_grad<double>, g, dim3(256), 0, s, (const cplx<double> *)a,
                           (const cplx<double> *)v, (double *)out, (long long)p.M, p.D);
    return hipGetLastError();
}

}  // namespace nfft
