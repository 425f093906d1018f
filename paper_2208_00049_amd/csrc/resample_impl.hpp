// Window resampling kernels (paper, step 3 of Algorithm 1 and step 1 of
// Algorithm 2; subsection "Resampling").
//
// A node with Nt*x = c + frac has, per axis, 2m taps at grid points
// o + t (t = 0..2m-1, o = c - m + 1) with window values
// psi_hat_Base((frac + m - 1 - t)/m); the D-variate weight is the product over
// the axes (tensor-product window, nested sum of equation (InnerTensorStructure)).
//
// Lane mapping: a group of 2m consecutive lanes of a wavefront serves one
// node; lane t of the group owns tap t of the last (contiguous) axis and loops
// over the taps of the other axes, fetching their weights from the lanes that
// computed them with wavefront shuffles.
//
// Interpolation (forward): the workgroup of a work item (tile, node range) copies
// the tile plus a (2m-1)-wide trailing halo of the grid into LDS, wrapping the
// indices at the copy (the paper's blocked Algorithm "Block-Partitioned
// Resampling" with the copy-in of its local cache), then sums over the stencil
// of every node and reduces the group's partial sums with shuffles.
//
// Spreading (adjoint): the workgroup owns one tile of the output grid.  It
// accumulates, with LDS atomics, the taps of every node whose stencil reaches
// into the tile -- its own nodes and those of the preceding tiles whose class
// bit says that their stencil crosses the tile border -- and writes the tile
// once.  This replaces the locked addition into the global grid of the paper's
// "Block-Partitioned Adjoint Resampling": each grid value has exactly one
// writer and no global atomics are used.
#pragma once

#include <math.h>

#include "common.hpp"
#include "nfft_internal.hpp"

namespace nfft {

template <typename T> struct WinParams {
    T beta[kMaxD];
};

// Window value of tap t for a node with offset frac (lane-owned coefficients cf).
template <typename T, int M2>
__device__ inline T tap_weight(const T *cf, T frac, int t, int window, T beta) {
    if (window == NFFT_WINDOW_POLY) {
        const T z = frac - (T)0.5;
        T acc = cf[M2];
#pragma unroll
        for (int k = M2 - 1; k >= 0; --k) acc = fma(acc, z, cf[k]);
        return acc;
    }
    constexpr int m = M2 / 2;
    const T u = (frac + (T)(m - 1 - t)) / (T)m;
    const T s2 = (T)1 - u * u;
    const T s = s2 > (T)0 ? sqrt(s2) : (T)0;
    return s > (T)0 ? sinh(beta * s) / ((T)M_PI * s) : beta / (T)M_PI;
}

template <typename C> __device__ inline C shfl_c(C v, int src) {
    return cmake<C>(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}
template <typename C> __device__ inline C shfl_down_c(C v, int off) {
    return cmake<C>(__shfl_down(v.x, off, 64), __shfl_down(v.y, off, 64));
}

template <int N> struct Pow2Ceil {
    static constexpr int value = N <= 1 ? 1 : 2 * Pow2Ceil<(N + 1) / 2>::value;
};
template <> struct Pow2Ceil<1> { static constexpr int value = 1; };

template <typename T, int D, int M2>
__global__ void __launch_bounds__(256)
    k_interp(const cplx<T> *__restrict__ grid, Geom g, const NodeRec<T, D> *__restrict__ nodes,
             const int *__restrict__ perm, const int4 *__restrict__ subs,
             const T *__restrict__ coef, int window, WinParams<T> wp, cplx<T> *__restrict__ fhat) {
    using C = cplx<T>;
    constexpr int Z = M2 + 1;
    constexpr int NPW = 64 / M2;
    extern __shared__ unsigned char smem_raw[];
    C *tile = reinterpret_cast<C *>(smem_raw);

    const int4 sp = subs[blockIdx.x];
    int t0[D], P[D];
    {
        int rem = sp.x;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            const int tc = rem % g.T[d];
            rem /= g.T[d];
            t0[d] = tc * g.Q[d];
            P[d] = g.Q[d] + M2 - 1;
        }
    }
    // copy the tile and its trailing halo into LDS, wrapping at the grid edge
    int total = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) total *= P[d];
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        int rem = idx;
        long long gi = 0;
        int a[D];
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            a[d] = rem % P[d];
            rem /= P[d];
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            int c = t0[d] + a[d];
            if (c >= g.Nt[d]) c -= g.Nt[d];
            gi = gi * g.Nt[d] + c;
        }
        tile[idx] = grid[gi];
    }

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / M2, li = lane - grp * M2, gbase = grp * M2;
    T cf[D][Z];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int z = 0; z < Z; ++z) cf[d][z] = coef[((size_t)d * M2 + li) * Z + z];
    __syncthreads();

    const int begin = sp.y, end = sp.z;
    const int nwaves = blockDim.x >> 6;
    for (int base = begin + wave * NPW; base < end; base += nwaves * NPW) {
        int node = base + grp;
        const bool valid = grp < NPW && node < end;
        if (!valid) node = begin;
        const NodeRec<T, D> rec = nodes[node];
        T w[D];
        int l[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            w[d] = tap_weight<T, M2>(cf[d], rec.fr[d], li, window, wp.beta[d]);
            l[d] = rec.o[d] - t0[d];
        }
        C acc = cmake<C>((T)0, (T)0);
        if constexpr (D == 1) {
            acc = cscale(tile[l[0] + li], w[0]);
        } else if constexpr (D == 2) {
            const C *row = tile + (size_t)l[0] * P[D - 1] + l[D - 1] + li;
#pragma unroll
            for (int a = 0; a < M2; ++a) {
                const T wa = __shfl(w[0], gbase + a, 64);
                const C v = row[(size_t)a * P[D - 1]];
                acc.x = fma(wa, v.x, acc.x);
                acc.y = fma(wa, v.y, acc.y);
            }
            acc = cscale(acc, w[D - 1]);
        } else {
            const int P1 = P[1 % D], P2 = P[D - 1];
            const C *base3 = tile + ((size_t)l[0] * P1 + l[1 % D]) * P2 + l[D - 1] + li;
#pragma unroll 2
            for (int a = 0; a < M2; ++a) {
                const T wa = __shfl(w[0], gbase + a, 64);
                C s2 = cmake<C>((T)0, (T)0);
#pragma unroll
                for (int b = 0; b < M2; ++b) {
                    const T wb = __shfl(w[1 % D], gbase + b, 64);
                    const C v = base3[((size_t)a * P1 + b) * P2];
                    s2.x = fma(wb, v.x, s2.x);
                    s2.y = fma(wb, v.y, s2.y);
                }
                acc.x = fma(wa, s2.x, acc.x);
                acc.y = fma(wa, s2.y, acc.y);
            }
            acc = cscale(acc, w[D - 1]);
        }
        // reduce the group's partial sums into its first lane
#pragma unroll
        for (int off = Pow2Ceil<M2>::value / 2; off >= 1; off >>= 1) {
            const C o = shfl_down_c(acc, off);
            if (li + off < M2) acc = cadd(acc, o);
        }
        if (valid && li == 0) fhat[perm[node]] = acc;
    }
}

template <typename T, int D, int M2>
__global__ void __launch_bounds__(256)
    k_spread(cplx<T> *__restrict__ grid, Geom g, const NodeRec<T, D> *__restrict__ nodes,
             const int *__restrict__ perm, const int *__restrict__ key_start,
             const T *__restrict__ coef, int window, WinParams<T> wp,
             const cplx<T> *__restrict__ fhat) {
    using C = cplx<T>;
    constexpr int Z = M2 + 1;
    constexpr int NPW = 64 / M2;
    constexpr int NR = 1 << (2 * D);  // (shift e, class) pairs
    extern __shared__ unsigned char smem_raw[];
    T *acc = reinterpret_cast<T *>(smem_raw);  // interleaved re, im of the owned tile
    __shared__ int rbeg[NR];
    __shared__ int rpre[NR + 1];

    const int p = blockIdx.x;
    int tc[D], t0[D];
    {
        int rem = p;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            tc[d] = rem % g.T[d];
            rem /= g.T[d];
            t0[d] = tc[d] * g.Q[d];
        }
    }
    int qtot = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) qtot *= g.Q[d];
    for (int i = threadIdx.x; i < 2 * qtot; i += blockDim.x) acc[i] = (T)0;

    // node ranges: entry r = e << D | cls, e = set of axes along which the
    // source tile precedes this one; a preceding tile contributes only the
    // classes whose stencils cross into this tile (cls contains e)
    if (threadIdx.x < NR) {
        const int r = threadIdx.x;
        const int e = r >> D, cls = r & ((1 << D) - 1);
        int len = 0, b = 0;
        if ((cls & e) == e) {
            int q = 0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                int qd = tc[d] - ((e >> d) & 1);
                if (qd < 0) qd += g.T[d];
                q = q * g.T[d] + qd;
            }
            const int key = (q << D) | cls;
            b = key_start[key];
            len = key_start[key + 1] - b;
        }
        rbeg[r] = b;
        rpre[r + 1] = len;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        rpre[0] = 0;
        for (int r = 0; r < NR; ++r) rpre[r + 1] += rpre[r];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / M2, li = lane - grp * M2, gbase = grp * M2;
    T cf[D][Z];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int z = 0; z < Z; ++z) cf[d][z] = coef[((size_t)d * M2 + li) * Z + z];
    __syncthreads();

    const int total = rpre[NR];
    const int nwaves = blockDim.x >> 6;
    for (int base = wave * NPW; base < total; base += nwaves * NPW) {
        int v = base + grp;
        const bool valid = grp < NPW && v < total;
        if (!valid) v = 0;
        // largest r with rpre[r] <= v (it is a non-empty range)
        int lo = 0, hi = NR;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (rpre[mid] <= v) lo = mid;
            else hi = mid;
        }
        const int e = lo >> D;
        const int node = valid ? rbeg[lo] + (v - rpre[lo]) : 0;
        const NodeRec<T, D> rec = nodes[node];
        const C val = valid ? fhat[perm[node]] : cmake<C>((T)0, (T)0);
        T w[D];
        int l[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            w[d] = tap_weight<T, M2>(cf[d], rec.fr[d], li, window, wp.beta[d]);
            int ld = rec.o[d] - t0[d];
            if (((e >> d) & 1) && ld >= 0) ld -= g.Nt[d];
            l[d] = ld;
        }
        const int cl = l[D - 1] + li;
        const bool okl = valid && cl >= 0 && cl < g.Q[D - 1];
        const C wv = cscale(val, w[D - 1]);
        if constexpr (D == 1) {
            if (okl) {
                atomicAdd(&acc[2 * cl], wv.x);
                atomicAdd(&acc[2 * cl + 1], wv.y);
            }
        } else if constexpr (D == 2) {
#pragma unroll
            for (int a = 0; a < M2; ++a) {
                const T wa = __shfl(w[0], gbase + a, 64);
                const int r0 = l[0] + a;
                if (okl && r0 >= 0 && r0 < g.Q[0]) {
                    const int idx = r0 * g.Q[D - 1] + cl;
                    atomicAdd(&acc[2 * idx], wa * wv.x);
                    atomicAdd(&acc[2 * idx + 1], wa * wv.y);
                }
            }
        } else {
            const int Q1 = g.Q[1 % D], Q2 = g.Q[D - 1];
#pragma unroll 2
            for (int a = 0; a < M2; ++a) {
                const T wa = __shfl(w[0], gbase + a, 64);
                const int r0 = l[0] + a;
                const bool ok0 = okl && r0 >= 0 && r0 < g.Q[0];
#pragma unroll
                for (int b = 0; b < M2; ++b) {
                    const T wb = __shfl(w[1 % D], gbase + b, 64);
                    const int r1 = l[1 % D] + b;
                    if (ok0 && r1 >= 0 && r1 < Q1) {
                        const int idx = (r0 * Q1 + r1) * Q2 + cl;
                        const T ww = wa * wb;
                        atomicAdd(&acc[2 * idx], ww * wv.x);
                        atomicAdd(&acc[2 * idx + 1], ww * wv.y);
                    }
                }
            }
        }
    }
    __syncthreads();

    // write the owned tile: every grid value has exactly this one writer
    for (int idx = threadIdx.x; idx < qtot; idx += blockDim.x) {
        int rem = idx;
        int a[D];
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            a[d] = rem % g.Q[d];
            rem /= g.Q[d];
        }
        long long gi = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) gi = gi * g.Nt[d] + t0[d] + a[d];
        grid[gi] = cmake<C>(acc[2 * idx], acc[2 * idx + 1]);
    }
}

// Dynamic LDS above 64 KiB has to be allowed per kernel before its launch.
template <typename K> inline hipError_t allow_lds(K kernel, size_t shm) {
    if (shm <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

template <typename T, int D, int M2>
hipError_t run_interp(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s) {
    int tot = 1;
    for (int d = 0; d < D; ++d) tot *= p.geom.Q[d] + M2 - 1;
    const size_t shm = (size_t)tot * sizeof(cplx<T>);
    WinParams<T> wp;
    for (int d = 0; d < kMaxD; ++d)
        wp.beta[d] = d < D ? (T)(M_PI * p.m * (2.0 - (double)p.N[d] / (double)p.Nt[d])) : (T)0;
    hipError_t e = allow_lds(k_interp<T, D, M2>, shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_interp<T, D, M2>), dim3(p.nsub), dim3(256), shm, s,
                       (const cplx<T> *)grid, p.geom, (const NodeRec<T, D> *)p.nodes, p.perm,
                       p.subs, (const T *)p.coef, p.window, wp, (cplx<T> *)fhat);
    return hipGetLastError();
}

template <typename T, int D, int M2>
hipError_t run_spread(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s) {
    int tot = 1;
    for (int d = 0; d < D; ++d) tot *= p.geom.Q[d];
    const size_t shm = (size_t)tot * 2 * sizeof(T);
    WinParams<T> wp;
    for (int d = 0; d < kMaxD; ++d)
        wp.beta[d] = d < D ? (T)(M_PI * p.m * (2.0 - (double)p.N[d] / (double)p.Nt[d])) : (T)0;
    hipError_t e = allow_lds(k_spread<T, D, M2>, shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_spread<T, D, M2>), dim3(p.geom.ntiles), dim3(256), shm, s,
                       (cplx<T> *)grid, p.geom, (const NodeRec<T, D> *)p.nodes, p.perm,
                       p.key_start, (const T *)p.coef, p.window, wp, (const cplx<T> *)fhat);
    return hipGetLastError();
}

}  // namespace nfft
