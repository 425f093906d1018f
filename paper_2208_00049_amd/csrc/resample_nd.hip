// Instantiation and dispatch of the resampling kernels of D = 4, 5 and 6 (the
// tile-owner spreading and the wavefront-per-node interpolation of resample_4d.hpp)
// over (type, D, 2m), in a compilation unit of their own.
#include "resample_4d.hpp"

namespace nfft {

#define NFFT_ND_M(FN, T, D, ...)                           \
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
static hipError_t interp_nd_t(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s,
                              int K) {
    switch (p.D) {
        case 4: NFFT_ND_M(run_interp_node, T, 4, p, grid, fhat, s, K)
        case 5: NFFT_ND_M(run_interp_node, T, 5, p, grid, fhat, s, K)
        case 6: NFFT_ND_M(run_interp_node, T, 6, p, grid, fhat, s, K)
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t spread_nd_t(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s,
                              int K) {
    switch (p.D) {
        case 4: NFFT_ND_M(run_spread_owner, T, 4, p, fhat, grid, s, K)
        case 5: NFFT_ND_M(run_spread_owner, T, 5, p, fhat, grid, s, K)
        case 6: NFFT_ND_M(run_spread_owner, T, 6, p, fhat, grid, s, K)
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_interp_nd(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s,
                            int K) {
    return p.dtype == NFFT_C64 ? interp_nd_t<float>(p, grid, fhat, s, K)
                               : interp_nd_t<double>(p, grid, fhat, s, K);
}

hipError_t launch_spread_nd(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s,
                            int K) {
    return p.dtype == NFFT_C64 ? spread_nd_t<float>(p, fhat, grid, s, K)
                               : spread_nd_t<double>(p, fhat, grid, s, K);
}

}  // namespace nfft
