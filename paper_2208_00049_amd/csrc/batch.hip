// Fused batches (runtime.cpp): the resampling stages of many transforms in one
// launch each.  A workgroup looks up its transform's entry and runs the body of
// the single transform's kernel (interpolation, spreading into padded tiles, or
// their halo merge) with that transform's parameters and its own block index,
// so that every transform's results equal those of its own calls bit for bit.
#include "resample_impl.hpp"

namespace nfft {

// ---- fused batches: one launch per resampling stage for the transforms of a batch ----

template <typename T> __device__ inline WinParams<T> bx_win_params(const BxResample &x) {
    WinParams<T> wp;
#pragma unroll
    for (int d = 0; d < kMaxD; ++d) {
        wp.beta[d] = (T)x.beta[d];
        wp.inv_peak[d] = (T)x.inv_peak[d];
    }
    wp.tab = (const T *)x.tab;
    wp.S = x.S;
    wp.m = x.m;
    return wp;
}

template <typename T, int D, int M2, bool GW, int NT>
__global__ void __launch_bounds__(NT)
    k_interp_batch(const BxResample *__restrict__ tab, const int *__restrict__ b2e,
                   void *const *__restrict__ out) {
    const int e = b2e[blockIdx.x];
    if (e < 0) return;
    const BxResample &x = tab[e];
    interp_body<T, D, M2, GW, false, NT>((const cplx<T> *)x.buf, x.g, (const NodeRec<T, D> *)x.nodes,
                                         x.perm, x.subs, (const T *)x.coef, x.window,
                                         bx_win_params<T>(x), (cplx<T> *)out[x.t], 0,
                                         blockIdx.x - x.start);
}

template <typename T, int D, int M2, bool GW, int NT>
__global__ void __launch_bounds__(NT)
    k_spread_batch(const BxResample *__restrict__ tab, const int *__restrict__ b2e,
                   const void *const *__restrict__ in) {
    const int e = b2e[blockIdx.x];
    if (e < 0) return;
    const BxResample &x = tab[e];
    spread_body<T, D, M2, GW, NT>((cplx<T> *)x.buf, x.g, (const NodeRec<T, D> *)x.nodes, x.perm,
                                  x.subs, (const T *)x.coef, x.window, bx_win_params<T>(x),
                                  (T)x.wmax_prod, (const cplx<T> *)in[x.t], blockIdx.x - x.start);
}

template <typename T, int D>
__global__ void __launch_bounds__(kResampleThreads)
    k_spread_merge_batch(const BxResample *__restrict__ tab, const int *__restrict__ b2e) {
    const int e = b2e[blockIdx.x];
    if (e < 0) return;
    const BxResample &x = tab[e];
    spread_merge_body<T, D>((cplx<T> *)x.grid, x.g, (const cplx<T> *)x.buf, x.tile_sub, x.g.taps,
                            blockIdx.x - x.start, x.nblk);
}

int resample_block_threads(int D) { return D == 3 ? 512 : kResampleThreads; }

template <typename T, int D, int M2>
static hipError_t resample_batch_t(int kind, bool gw, const BxResample *tab, const int *b2e,
                                   const void *const *in, void *const *out, int nblocks, size_t shm,
                                   hipStream_t s) {
    constexpr int NT = resample_threads<T, D>();
    if (gw) return hipErrorInvalidValue;  // fused batches take the polynomial window only
    hipError_t e = hipSuccess;
    if (kind == kBxInterp) {
        auto kern = k_interp_batch<T, D, M2, false, NT>;
        e = allow_lds(kern, shm, interp_static_lds_t<T, D>());
        if (e == hipSuccess) hipLaunchKernelGGL(kern, dim3(nblocks), dim3(NT), shm, s, tab, b2e, out);
    } else if (kind == kBxSpread) {
        auto kern = k_spread_batch<T, D, M2, false, NT>;
        e = allow_lds(kern, shm, static_lds<T, D>());
        if (e == hipSuccess) hipLaunchKernelGGL(kern, dim3(nblocks), dim3(NT), shm, s, tab, b2e, in);
    } else {
        hipLaunchKernelGGL((k_spread_merge_batch<T, D>), dim3(nblocks), dim3(kResampleThreads), 0, s,
                           tab, b2e);
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <typename T>
static hipError_t resample_batch_d(int kind, int D, int taps, bool gw, const BxResample *tab,
                                   const int *b2e, const void *const *in, void *const *out,
                                   int nblocks, size_t shm, hipStream_t s) {
#define NFFT_BATCH_M(D_)                                                                                \
    switch (taps / 2) {                                                                                 \
        case 1: return resample_batch_t<T, D_, 2>(kind, gw, tab, b2e, in, out, nblocks, shm, s);       \
        case 2: return resample_batch_t<T, D_, 4>(kind, gw, tab, b2e, in, out, nblocks, shm, s);       \
        case 3: return resample_batch_t<T, D_, 6>(kind, gw, tab, b2e, in, out, nblocks, shm, s);       \
        case 4: return resample_batch_t<T, D_, 8>(kind, gw, tab, b2e, in, out, nblocks, shm, s);       \
        case 5: return resample_batch_t<T, D_, 10>(kind, gw, tab, b2e, in, out, nblocks, shm, s);      \
        case 6: return resample_batch_t<T, D_, 12>(kind, gw, tab, b2e, in, out, nblocks, shm, s);      \
        case 7: return resample_batch_t<T, D_, 14>(kind, gw, tab, b2e, in, out, nblocks, shm, s);      \
        case 8: return resample_batch_t<T, D_, 16>(kind, gw, tab, b2e, in, out, nblocks, shm, s);      \
        case 9: return resample_batch_t<T, D_, 18>(kind, gw, tab, b2e, in, out, nblocks, shm, s);      \
        case 10: return resample_batch_t<T, D_, 20>(kind, gw, tab, b2e, in, out, nblocks, shm, s);     \
        case 11: return resample_batch_t<T, D_, 22>(kind, gw, tab, b2e, in, out, nblocks, shm, s);     \
        default: return hipErrorInvalidValue;                                                           \
    }
    switch (D) {
        case 1: NFFT_BATCH_M(1)
        case 2: NFFT_BATCH_M(2)
        case 3: NFFT_BATCH_M(3)
        default: return hipErrorInvalidValue;
    }
#undef NFFT_BATCH_M
}

hipError_t launch_resample_batch(int kind, int dtype, int D, int taps, bool gw, const BxResample *tab,
                                 const int *b2e, const void *const *in, void *const *out,
                                 int nblocks, size_t shm, hipStream_t s) {
    if (nblocks == 0) return hipSuccess;
    return dtype == NFFT_C64 ? resample_batch_d<float>(kind, D, taps, gw, tab, b2e, in, out, nblocks, shm, s)
                             : resample_batch_d<double>(kind, D, taps, gw, tab, b2e, in, out, nblocks, shm, s);
}

}  // namespace nfft
