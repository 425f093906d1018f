// Resampling kernels for D = 4 (paper, step 3 of Algorithm 1 and step 1 of
// Algorithm 2, with the dimension-agnostic tensor-product window of subsection
// "Direct NFFT").
//
// The LDS-tiled kernels keep a tile plus its (taps-1)-wide trailing halo on
// chip.  In four dimensions that box has (Q + taps - 1)^4 cells, which for
// useful tiles is beyond the LDS of a workgroup, so these kernels read and
// write the grid in HBM (through L2) instead:
//
// Interpolation: one wavefront per node.  Lane i of the wavefront computes the
// weight of entry i (and i + 64) of the node's [axis][tap] weight table; the
// wavefront then walks the taps^D stencil points with the last axis fastest
// (consecutive lanes read consecutive grid points), taking the axis weights
// from the lanes that hold them, and reduces its partial sums in a fixed order.
//
// Spreading, output-driven: every grid point of a tile has one owner thread,
// which sums the contributions of all nodes whose stencil covers it.  The
// candidates are the nodes binned in the tile and in the r_d - 1 tiles before
// it along each axis, r_d = 2 + floor((taps - 2) / Q_d) (at most T_d; a node of
// a tile further back cannot reach this one).  They are staged through LDS in
// chunks together with their axis weights.  Each grid value is written once, by
// one thread, with no atomics and no halo merge.  The sum runs over the nodes in
// the plan's sorted order, so a plan reproduces its results bit for bit (two
// plans of the same nodes may order the nodes of one bin differently).
#pragma once

#include "resample_impl.hpp"

namespace nfft {

constexpr int kGatherChunk = 64;  // nodes staged per round of the spreading kernel

template <int B, int E> struct IPow {
    static constexpr int value = B * IPow<B, E - 1>::value;
};
template <int B> struct IPow<B, 0> {
    static constexpr int value = 1;
};

// Weight of tap t along axis d for the node at sorted position gk with offset frac.
template <typename T, int M2>
__device__ inline T axis_weight(const T *__restrict__ coef, int window, const WinParams<T> &wp,
                                int D, long long gk, int d, int t, T frac) {
    if (window == NFFT_WINDOW_TENSOR) return wp.tab[(gk * D + d) * M2 + t];
    T cf[M2 + 1];
    const int Z = 2 * wp.m + 1;
#pragma unroll
    for (int z = 0; z <= M2; ++z)
        cf[z] = (window == NFFT_WINDOW_POLY && z < Z) ? coef[((size_t)d * M2 + t) * Z + z] : (T)0;
    return tap_weight<T, M2>(cf, frac, t, window, wp.beta[d], wp.tab + (size_t)d * wp.S, wp.S,
                             wp.m);
}

template <typename T, int D> __device__ inline T pick(const T (&v)[D], int d) {
    T r = v[0];
#pragma unroll
    for (int e = 1; e < D; ++e) r = e == d ? v[e] : r;
    return r;
}

template <typename T, int D, int M2>
__global__ void __launch_bounds__(kResampleThreads)
    k_interp_gather(const cplx<T> *__restrict__ grid, Geom g,
                    const NodeRec<T, D> *__restrict__ nodes, const int *__restrict__ perm,
                    const int4 *__restrict__ subs, const T *__restrict__ coef, int window,
                    WinParams<T> wp, cplx<T> *__restrict__ fhat, long long gstride,
                    long long fstride) {
    using C = cplx<T>;
    grid += blockIdx.y * gstride;  // channel
    fhat += blockIdx.y * fstride;
    constexpr int NW = kResampleThreads / 64;
    constexpr int NWT = D * M2;                  // axis weights of a node
    constexpr int NT = IPow<M2, D>::value;       // stencil points
    constexpr int NK = (NT + 63) / 64;           // stencil points per lane
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int4 sp = subs[blockIdx.x];
    // the loop bound is uniform over the wavefront: all lanes stay active for the shuffles
    for (int j = sp.y + wave; j < sp.z; j += NW) {
        const NodeRec<T, D> rec = nodes[j];
        T wa = (T)0, wb = (T)0;
        {
            const int ia = lane < NWT ? lane : 0;
            const int da = ia / M2;
            wa = axis_weight<T, M2>(coef, window, wp, D, j, da, ia - da * M2, pick<T, D>(rec.fr, da));
            if constexpr (NWT > 64) {
                const int ib = lane + 64 < NWT ? lane + 64 : 0;
                const int db = ib / M2;
                wb = axis_weight<T, M2>(coef, window, wp, D, j, db, ib - db * M2,
                                        pick<T, D>(rec.fr, db));
            }
        }
        T ar = (T)0, ai = (T)0;
        for (int k = 0; k < NK; ++k) {
            const int f = k * 64 + lane;
            const bool ok = f < NT;
            int rem = ok ? f : 0;
            int t[D];
#pragma unroll
            for (int d = D - 1; d >= 0; --d) {
                t[d] = rem % M2;
                rem /= M2;
            }
            long long idx = 0;
            T w = (T)1;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                int pos = rec.o[d] + t[d];
                if (pos >= g.Nt[d]) pos -= g.Nt[d];
                idx = idx * g.Nt[d] + pos;
                const int wi = d * M2 + t[d];
                T wv = __shfl(wa, wi & 63, 64);
                if constexpr (NWT > 64) {
                    const T wv2 = __shfl(wb, wi & 63, 64);
                    wv = wi < 64 ? wv : wv2;
                }
                w *= wv;
            }
            const C v = grid[idx];
            if (ok) {
                ar = fma(w, v.x, ar);
                ai = fma(w, v.y, ai);
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            ar += __shfl_xor(ar, off, 64);
            ai += __shfl_xor(ai, off, 64);
        }
        if (lane == 0) fhat[perm[j]] = cmake<C>(ar, ai);
    }
}

// One workgroup per (tile, block of kResampleThreads cells of the tile, channel).
template <typename T, int D, int M2>
__global__ void __launch_bounds__(kResampleThreads)
    k_spread_gather(cplx<T> *__restrict__ grid, Geom g, const NodeRec<T, D> *__restrict__ nodes,
                    const int *__restrict__ perm, const int *__restrict__ key_start,
                    const T *__restrict__ coef, int window, WinParams<T> wp,
                    const cplx<T> *__restrict__ fhat, int cblocks, long long gstride,
                    long long fstride) {
    using C = cplx<T>;
    constexpr int CH = kGatherChunk;
    constexpr int NWT = D * M2;
    __shared__ T sw[CH][NWT];
    __shared__ T sfr[D][CH];
    __shared__ int srel[D][CH];
    __shared__ int snode[CH];
    __shared__ T svr[CH], svi[CH];
    __shared__ int nb_begin[kGatherMaxTiles], nb_pre[kGatherMaxTiles + 1];

    grid += blockIdx.y * gstride;  // channel
    fhat += blockIdx.y * fstride;
    const int tile = blockIdx.x / cblocks;
    const int cb = blockIdx.x - tile * cblocks;
    const int tid = threadIdx.x;
    int tc[D], t0[D], r[D];
    int cells = 1, nb = 1;
    {
        int rem = tile;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            tc[d] = rem % g.T[d];
            rem /= g.T[d];
            t0[d] = tc[d] * g.Q[d];
            r[d] = gather_reach(g, d);
            cells *= g.Q[d];
            nb *= r[d];
        }
    }
    // node ranges of the candidate tiles (tile - b, b_d = 0..r_d-1, cyclic)
    if (tid < nb) {
        int rem = tid, ti = 0;
        int bd[D];
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            bd[d] = rem % r[d];
            rem /= r[d];
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            int p = tc[d] - bd[d];
            if (p < 0) p += g.T[d];
            ti = ti * g.T[d] + p;
        }
        const int a = key_start[(long long)ti << D];
        nb_begin[tid] = a;
        nb_pre[tid + 1] = key_start[(long long)(ti + 1) << D] - a;  // size, summed below
    }
    __syncthreads();
    if (tid == 0) {
        nb_pre[0] = 0;
        for (int i = 0; i < nb; ++i) nb_pre[i + 1] += nb_pre[i];
    }
    __syncthreads();
    const int total = nb_pre[nb];

    // this thread's grid point: local coordinates and global index
    const int cell = cb * kResampleThreads + tid;
    const bool own = cell < cells;
    int lc[D];
    long long gidx = 0;
    {
        int rem = own ? cell : 0;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            lc[d] = rem % g.Q[d];
            rem /= g.Q[d];
        }
#pragma unroll
        for (int d = 0; d < D; ++d) gidx = gidx * g.Nt[d] + (t0[d] + lc[d]);
    }

    T ar = (T)0, ai = (T)0;
    for (int c0 = 0; c0 < total; c0 += CH) {
        const int n = min(CH, total - c0);
        if (tid < n) {
            const int q = c0 + tid;
            int i = 0;
            while (nb_pre[i + 1] <= q) ++i;
            const int gk = nb_begin[i] + (q - nb_pre[i]);
            const NodeRec<T, D> rec = nodes[gk];
            const C v = fhat[perm[gk]];
            snode[tid] = gk;
            svr[tid] = v.x;
            svi[tid] = v.y;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                // origin relative to the tile start, in [Q - Nt, Q)
                int rel = rec.o[d] - t0[d];
                if (rel < 0) rel += g.Nt[d];
                if (rel >= g.Q[d]) rel -= g.Nt[d];
                srel[d][tid] = rel;
                sfr[d][tid] = rec.fr[d];
            }
        }
        __syncthreads();
        for (int e = tid; e < n * NWT; e += kResampleThreads) {
            const int k = e / NWT;
            const int rest = e - k * NWT;
            const int d = rest / M2;
            const int t = rest - d * M2;
            sw[k][rest] = axis_weight<T, M2>(coef, window, wp, D, snode[k], d, t, sfr[d][k]);
        }
        __syncthreads();
        if (own) {
            for (int k = 0; k < n; ++k) {
                T w = (T)1;
                bool hit = true;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    int off = lc[d] - srel[d][k];
                    if (off < 0) off += g.Nt[d];
                    hit = hit && off < M2;
                    w *= sw[k][d * M2 + (off < M2 ? off : 0)];
                }
                if (hit) {
                    ar = fma(w, svr[k], ar);
                    ai = fma(w, svi[k], ai);
                }
            }
        }
        __syncthreads();
    }
    if (own) grid[gidx] = cmake<C>(ar, ai);
}

template <typename T, int D, int M2>
hipError_t run_interp_gather(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s,
                             int K) {
    if (p.nsub == 0) return hipSuccess;
    hipLaunchKernelGGL((k_interp_gather<T, D, M2>), dim3(p.nsub, K), dim3(kResampleThreads), 0, s,
                       (const cplx<T> *)grid, p.geom, (const NodeRec<T, D> *)p.nodes, p.perm,
                       p.subs, (const T *)p.coef, p.window, win_params<T>(p), (cplx<T> *)fhat,
                       (long long)p.G, (long long)p.M);
    return hipGetLastError();
}

// Spreading writes every grid point (zeros where no node reaches), so the
// grid needs no clearing first.
template <typename T, int D, int M2>
hipError_t run_spread_gather(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s,
                             int K) {
    int cells = 1;
    for (int d = 0; d < D; ++d) cells *= p.geom.Q[d];
    const int cblocks = (cells + kResampleThreads - 1) / kResampleThreads;
    const long long nblk = (long long)p.geom.ntiles * cblocks;
    if (nblk >= (1LL << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_spread_gather<T, D, M2>), dim3((unsigned)nblk, K),
                       dim3(kResampleThreads), 0, s, (cplx<T> *)grid, p.geom,
                       (const NodeRec<T, D> *)p.nodes, p.perm, p.key_start, (const T *)p.coef,
                       p.window, win_params<T>(p), (const cplx<T> *)fhat, cblocks, (long long)p.G,
                       (long long)p.M);
    return hipGetLastError();
}

}  // namespace nfft
