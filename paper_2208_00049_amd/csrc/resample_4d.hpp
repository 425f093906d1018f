// Resampling kernels for D >= 4 (paper, step 3 of Algorithm 1 and step 1 of
// Algorithm 2, with the dimension-agnostic tensor-product window of subsection
// "Direct NFFT"); instantiated for D = 4, 5 and 6.
//
// The tiled kernels of D <= 3 give a work item its tile plus the (taps-1)-wide
// trailing halo.  In four dimensions that box has (Q + taps - 1)^4 cells, which
// for useful tiles is beyond a workgroup's LDS, and a node's stencil has taps^4
// points (4096 at m = 4), 64 times its 2-D count.
//
// Interpolation: one wavefront per node reads the node's stencil from the grid
// in device memory (through L1/L2).  Lane i computes the weight of entry i (and
// i + 64) of the node's [axis][tap] table -- a fixed tap for the lane, so its
// polynomial coefficients stay in registers; the wavefront walks the stencil
// points with the last axis fastest (consecutive lanes read consecutive grid
// points), takes the axis weights from the lanes holding them and reduces its
// partial sums in a fixed order.
//
// Spreading turns the ownership round: a workgroup owns one tile of the grid,
// exactly (no halo), and visits every node whose stencil reaches into it -- the
// nodes binned in the tile and in the r_d - 1 tiles before it along each axis,
// r_d = min(T_d, 2 + (taps - 2) / Q_d) (a node of a tile further back cannot
// reach it).  Per node it walks only the box where the stencil and the tile
// intersect (one interval per axis, since taps + Q_d <= Nt_d when T_d >= 2; the
// whole stencil, wrapped, when the tile spans the axis): lanes take the box
// points of the axes 1..D-1 and loop over axis 0, and a wavefront takes its
// next node from a per-round counter when it is done with a box.
// Contributions go into the tile in LDS with 64-bit fixed-point atomics (the
// scheme of the tiled kernels: a power-of-two scale from the largest |value| of
// the tile's candidates; exact, order-independent sums), and the tile is
// written to the grid once.  No global atomics, no scratch, no halo merge;
// bitwise reproducible.
#pragma once

#include "resample_impl.hpp"

namespace nfft {

// Polynomial coefficients of tap t along axis d (zero-padded to degree M2).
template <typename T, int M2> struct TapCoef {
    T cf[M2 + 1];
    __device__ void load(const T *__restrict__ coef, int window, int m, int d, int t) {
        const int Z = 2 * m + 1;
#pragma unroll
        for (int z = 0; z <= M2; ++z)
            cf[z] = (window == NFFT_WINDOW_POLY && z < Z) ? coef[((size_t)d * M2 + t) * Z + z] : (T)0;
    }
};

// Weight of tap t along axis d for the node at sorted position gk with offset
// frac (tc: that tap's polynomial coefficients).
template <typename T, int M2>
__device__ inline T axis_weight(const TapCoef<T, M2> &tc, int window, const WinParams<T> &wp, int D,
                                long long gk, int d, int t, T frac) {
    if (window == NFFT_WINDOW_TENSOR) return wp.tab[(gk * D + d) * M2 + t];
    return tap_weight<T, M2>(tc.cf, frac, t, window, wp.beta[d], wp.inv_peak[d],
                             wp.tab + (size_t)d * wp.S, wp.S, wp.m);
}

// Candidates staged per round (owner_chunk_n).
template <typename T, int D, int M2> constexpr int owner_chunk() {
    return owner_chunk_n(D, M2, (int)sizeof(T));
}

// Staged candidate nodes of one round.
template <typename T, int D, int M2> struct OwnerStage {
    static constexpr int CH = owner_chunk<T, D, M2>();
    int gk[CH];       // sorted node position
    int loc0[D][CH];  // tile-local coordinate of the first box point
    int tap0[D][CH];  // stencil tap of the first box point
    int n[D][CH];     // box extent (0: the stencil misses the tile)
    T fr[D][CH];
    T vr[CH], vi[CH];  // the node's value
    T w[CH][D * M2];   // axis weights of the box taps
};

template <int D> struct OwnerTile {
    int tc[D], t0[D], r[D];
    int cells, nb;
};

template <int D> __device__ inline OwnerTile<D> owner_tile(const Geom &g, int tile) {
    OwnerTile<D> ot;
    ot.cells = 1;
    ot.nb = 1;
    int rem = tile;
#pragma unroll
    for (int d = D - 1; d >= 0; --d) {
        ot.tc[d] = rem % g.T[d];
        rem /= g.T[d];
        ot.t0[d] = ot.tc[d] * g.Q[d];
        ot.r[d] = owner_reach(g, d);
        ot.cells *= g.Q[d];
        ot.nb *= ot.r[d];
    }
    return ot;
}

// Node ranges of the candidate tiles, tile - b for b_d = 0..r_d-1 (cyclic), in
// mixed-radix order of b (last axis fastest); nb_pre becomes the prefix sums.
template <int D>
__device__ inline void owner_ranges(const OwnerTile<D> &ot, const Geom &g,
                                    const int *__restrict__ key_start, int *nb_begin,
                                    int *nb_pre) {
    const int tid = threadIdx.x;
    if (tid < ot.nb) {
        int rem = tid, ti = 0, bd[D];
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            bd[d] = rem % ot.r[d];
            rem /= ot.r[d];
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            int p = ot.tc[d] - bd[d];
            if (p < 0) p += g.T[d];
            ti = ti * g.T[d] + p;
        }
        const int a = key_start[(long long)ti << D];
        nb_begin[tid] = a;
        nb_pre[tid + 1] = key_start[(long long)(ti + 1) << D] - a;
    }
    __syncthreads();
    if (tid == 0) {
        nb_pre[0] = 0;
        for (int i = 0; i < ot.nb; ++i) nb_pre[i + 1] += nb_pre[i];
    }
    __syncthreads();
}

// Stage candidates [c0, c0 + n) of the concatenated ranges: box per axis, then
// the weights of the box taps -- thread tid computes tap (tid mod D*M2) of the
// candidates tid / (D*M2), + nper, ... (tc: its coefficients).  Ends with a barrier.
template <typename T, int D, int M2>
__device__ inline void owner_stage(OwnerStage<T, D, M2> &st, int c0, int n, const OwnerTile<D> &ot,
                                   const Geom &g, const int *nb_begin, const int *nb_pre,
                                   const NodeRec<T, D> *__restrict__ nodes,
                                   const int *__restrict__ perm, const cplx<T> *__restrict__ fhat,
                                   const TapCoef<T, M2> &tc, int window, const WinParams<T> &wp) {
    const int tid = threadIdx.x;
    if (tid < n) {
        const int q = c0 + tid;
        // candidate-tile range holding q: the last i with nb_pre[i] <= q
        int lo = 0, hi = ot.nb - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (nb_pre[mid] <= q) lo = mid;
            else hi = mid - 1;
        }
        const int i = lo;
        const int gk = nb_begin[i] + (q - nb_pre[i]);
        const NodeRec<T, D> rec = nodes[gk];
        st.gk[tid] = gk;
        const cplx<T> v = fhat[perm[gk]];
        st.vr[tid] = v.x;
        st.vi[tid] = v.y;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            int loc0, tap0, cnt;
            if (g.T[d] == 1) {  // the tile spans the axis: the whole stencil, wrapped
                loc0 = rec.o[d];
                tap0 = 0;
                cnt = g.taps;
            } else {
                // origin relative to the tile start, in [Q - Nt, Q)
                int rel = rec.o[d] - ot.t0[d];
                if (rel < 0) rel += g.Nt[d];
                if (rel >= g.Q[d]) rel -= g.Nt[d];
                tap0 = rel < 0 ? -rel : 0;
                const int hi2 = min(g.taps, g.Q[d] - rel);
                cnt = max(0, hi2 - tap0);
                loc0 = rel + tap0;
            }
            st.loc0[d][tid] = loc0;
            st.tap0[d][tid] = tap0;
            st.n[d][tid] = cnt;
            st.fr[d][tid] = rec.fr[d];
        }
    }
    __syncthreads();
    constexpr int NWT = D * M2;
    const int nper = blockDim.x / NWT;
    if (tid < nper * NWT) {
        const int rest = tid % NWT;
        const int d = rest / M2;
        const int t = rest - d * M2;
        for (int k = tid / NWT; k < n; k += nper) {
            const int rel = t - st.tap0[d][k];
            if (rel >= 0 && rel < st.n[d][k])
                st.w[k][rest] = axis_weight<T, M2>(tc, window, wp, D, st.gk[k], d, t, st.fr[d][k]);
        }
    }
    __syncthreads();
}

// The coefficients of the tap this thread evaluates in owner_stage.
template <typename T, int D, int M2>
__device__ inline TapCoef<T, M2> owner_coef(const T *__restrict__ coef, int window, int m) {
    constexpr int NWT = D * M2;
    TapCoef<T, M2> tc;
    const int rest = threadIdx.x % NWT;
    tc.load(coef, window, m, rest / M2, rest % M2);
    return tc;
}

// Walk the box of candidate k: lanes over the points of axes 1..D-1, an
// unrolled loop over axis 0; f(live, cell, w) per point.  Lanes past the box get
// live = false, w = 0 and an in-range cell.  The candidate's box parameters are
// uniform over the wavefront (scalar registers), the walk has no branches.
template <typename T, int D, int M2, typename F>
__device__ inline void owner_box(const OwnerStage<T, D, M2> &st, int k, const Geom &g,
                                 const OwnerLayout &lay, int lane, F &&f) {
    int n[D], loc0[D], tap0[D];
    int npl = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        n[d] = __builtin_amdgcn_readfirstlane(st.n[d][k]);
        loc0[d] = __builtin_amdgcn_readfirstlane(st.loc0[d][k]);
        tap0[d] = __builtin_amdgcn_readfirstlane(st.tap0[d][k]);
        if (d > 0) npl *= n[d];
    }
    if (n[0] == 0 || npl == 0) return;
    float rc[D];
#pragma unroll
    for (int d = 1; d < D; ++d) rc[d] = 1.0f / (float)n[d];
    const T *wk = st.w[k];
    T w0[M2];  // axis-0 weights of the box, zero past it
#pragma unroll
    for (int u0 = 0; u0 < M2; ++u0) w0[u0] = u0 < n[0] ? wk[tap0[0] + u0] : (T)0;
    for (int base = 0; base < npl; base += 64) {
        const int q = base + lane;
        const bool ok = q < npl;
        int u[D];
        int rem = ok ? q : 0;
#pragma unroll
        for (int d = D - 1; d >= 2; --d) rem = small_divmod(rem, n[d], rc[d], u[d]);
        u[1] = rem;
        int c1 = 0;
        T w1 = (T)1;
#pragma unroll
        for (int d = 1; d < D; ++d) {
            int loc = loc0[d] + u[d];
            if (loc >= g.Q[d]) loc -= g.Q[d];  // wraps only when the tile spans the axis
            c1 += loc * lay.S[d];
            w1 *= wk[d * M2 + tap0[d] + u[d]];
        }
        w1 = ok ? w1 : (T)0;
#pragma unroll
        for (int u0 = 0; u0 < M2; ++u0) {
            const bool in = u0 < n[0];
            const int uc = in ? u0 : n[0] - 1;
            int l0 = loc0[0] + uc;
            if (l0 >= g.Q[0]) l0 -= g.Q[0];
            f(ok && in, l0 * lay.S[0] + c1, w0[u0] * w1);
        }
    }
}

// Global grid index of tile-local cell c (row-major over the tile) and, in
// *lds, its accumulator index in the layout lay.
template <int D>
__device__ inline long long owner_global(const OwnerTile<D> &ot, const Geom &g,
                                         const OwnerLayout &lay, int c, int *lds) {
    int l[D];
    int rem = c;
#pragma unroll
    for (int d = D - 1; d >= 0; --d) {
        l[d] = rem % g.Q[d];
        rem /= g.Q[d];
    }
    long long idx = 0;
    int li = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        idx = idx * g.Nt[d] + (ot.t0[d] + l[d]);
        li += l[d] * lay.S[d];
    }
    *lds = li;
    return idx;
}

template <typename T, int D> __device__ inline T pick(const T (&v)[D], int d) {
    T r = v[0];
#pragma unroll
    for (int e = 1; e < D; ++e) r = e == d ? v[e] : r;
    return r;
}

template <int B, int E> struct IPow {
    static constexpr int value = B * IPow<B, E - 1>::value;
};
template <int B> struct IPow<B, 0> {
    static constexpr int value = 1;
};

// Interpolation, one wavefront per node of the work items (channel blockIdx.y).
template <typename T, int D, int M2>
__global__ void __launch_bounds__(kResampleThreads)
    k_interp_node(const cplx<T> *__restrict__ grid, Geom g,
                  const NodeRec<T, D> *__restrict__ nodes, const int *__restrict__ perm,
                  const int4 *__restrict__ subs, const T *__restrict__ coef, int window,
                  WinParams<T> wp, cplx<T> *__restrict__ fhat, long long gstride,
                  long long fstride) {
    using C = cplx<T>;
    grid += blockIdx.y * gstride;  // channel
    fhat += blockIdx.y * fstride;
    constexpr int NW = kResampleThreads / 64;
    constexpr int NWT = D * M2;             // axis weights of a node
    constexpr int NT = IPow<M2, D>::value;  // stencil points
    constexpr int NK = (NT + 63) / 64;      // stencil points per lane
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the lane's taps of the weight table: entry ia and (if the table is longer) ib
    const int ia = lane < NWT ? lane : 0, da = ia / M2, ta = ia - da * M2;
    const int ib = lane + 64 < NWT ? lane + 64 : 0, db = ib / M2, tb = ib - db * M2;
    TapCoef<T, M2> ca, cb;
    ca.load(coef, window, wp.m, da, ta);
    if constexpr (NWT > 64) cb.load(coef, window, wp.m, db, tb);
    const int4 sp = subs[xcd_block(blockIdx.x, gridDim.x)];  // neighbouring tiles share an L2
    // the loop bound is uniform over the wavefront: all lanes stay active for the shuffles
    for (int j = sp.y + wave; j < sp.z; j += NW) {
        const NodeRec<T, D> rec = nodes[j];
        const T wa = axis_weight<T, M2>(ca, window, wp, D, j, da, ta, pick<T, D>(rec.fr, da));
        T wb = (T)0;
        if constexpr (NWT > 64)
            wb = axis_weight<T, M2>(cb, window, wp, D, j, db, tb, pick<T, D>(rec.fr, db));
        T ar = (T)0, ai = (T)0;
        // unrolled so that eight grid loads are in flight per wavefront (rolled, the
        // loop waited for each load before issuing the next)
#pragma unroll 8
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

// Spreading, tile-owner: fhat (channel blockIdx.y) -> every grid point of the
// tile.  Dynamic LDS: the tile's fixed-point accumulator planes.
template <typename T, int D, int M2>
__global__ void __launch_bounds__(kOwnerThreads)
    k_spread_owner(cplx<T> *__restrict__ grid, Geom g, const NodeRec<T, D> *__restrict__ nodes,
                   const int *__restrict__ perm, const int *__restrict__ key_start,
                   const T *__restrict__ coef, int window, WinParams<T> wp, T wmax_prod,
                   const cplx<T> *__restrict__ fhat, long long gstride, long long fstride,
                   OwnerLayout lay) {
    using C = cplx<T>;
    using FP = typename OwnerAcc<T>::type;
    constexpr int SL = 2 * FP::kSlots;  // accumulator slots per grid point
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ OwnerStage<T, D, M2> st;
    __shared__ int nb_begin[owner_max_tiles(D)], nb_pre[owner_max_tiles(D) + 1];
    __shared__ unsigned long long amax_bits;  // bits of a non-negative double
    __shared__ int next_k[2];                 // candidate counters of even and odd rounds
    static_assert(sizeof(OwnerStage<T, D, M2>) + sizeof(int) * (2 * owner_max_tiles(D) + 3) + 8 <=
                      owner_static_lds(D, M2, (int)sizeof(T)),
                  "staged candidates larger than the LDS the plan reserves for them");
    grid += blockIdx.y * gstride;
    fhat += blockIdx.y * fstride;
    const OwnerTile<D> ot = owner_tile<D>(g, xcd_block(blockIdx.x, gridDim.x));
    const int lane = threadIdx.x & 63;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem_raw);
    for (int c = threadIdx.x; c < SL * lay.cells; c += blockDim.x) acc[c] = 0ull;
    if (threadIdx.x == 0) {
        amax_bits = 0ull;
        next_k[0] = next_k[1] = 0;
    }
    owner_ranges<D>(ot, g, key_start, nb_begin, nb_pre);  // (its barriers cover the clearing)
    const int total = nb_pre[ot.nb];

    // scale: the largest |Re|, |Im| over the tile's candidates
    T amax = (T)0;
    {
        int i = 0;
        for (int q = threadIdx.x; q < total; q += blockDim.x) {
            while (nb_pre[i + 1] <= q) ++i;
            const C v = fhat[perm[nb_begin[i] + (q - nb_pre[i])]];
            amax = fmax(amax, scale_mag(v.x, v.y));
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    if (lane == 0) atomicMax(&amax_bits, (unsigned long long)__double_as_longlong((double)amax));
    __syncthreads();
    const double amax_d = __longlong_as_double((long long)amax_bits);
    const bool poisoned = isinf(amax_d);  // a non-finite candidate value (same in every thread)
    const double bound = amax_d * (double)wmax_prod;
    const T scale = bound > 0.0 && !poisoned ? FP::scale(bound, total) : (T)1;

    const TapCoef<T, M2> tc = owner_coef<T, D, M2>(coef, window, wp.m);
    constexpr int CH = OwnerStage<T, D, M2>::CH;
    int parity = 0;
    for (int c0 = 0; c0 < (poisoned ? 0 : total); c0 += CH, parity ^= 1) {
        const int n = min(CH, total - c0);
        owner_stage<T, D, M2>(st, c0, n, ot, g, nb_begin, nb_pre, nodes, perm, fhat, tc, window,
                              wp);
        if (threadIdx.x == 0) next_k[parity ^ 1] = 0;  // the next round's counter (unused now)
        // Candidates go to the wavefronts on demand: boxes range from one point to
        // taps^D, and a fixed assignment left wavefronts idle at the round's barrier.
        // The next index is requested before the current box is walked.
        int kn = 0;
        if (lane == 0) kn = atomicAdd(&next_k[parity], 1);
        kn = __builtin_amdgcn_readfirstlane(kn);
        while (kn < n) {
            const int k = kn;
            int req = 0;
            if (lane == 0) req = atomicAdd(&next_k[parity], 1);
            const T pr = st.vr[k] * scale, pi = st.vi[k] * scale;
            owner_box<T, D, M2>(st, k, g, lay, lane, [&](bool live, int cell, T w) {
                if (live) FP::add(acc + cell, lay.cells, w * pr, w * pi);
            });
            kn = __builtin_amdgcn_readfirstlane(req);
        }
        __syncthreads();
    }
    const T inv = (T)(1.0 / (double)scale);
    const T nan = (T)__builtin_nan("");
    for (int c = threadIdx.x; c < ot.cells; c += blockDim.x) {
        int li;
        const long long gi = owner_global<D>(ot, g, lay, c, &li);
        grid[gi] = poisoned ? cmake<C>(nan, nan)
                            : cmake<C>((T)FP::read(acc + li, lay.cells, 0) * inv,
                                       (T)FP::read(acc + li, lay.cells, 1) * inv);
    }
}

template <typename T, int D, int M2>
hipError_t run_interp_node(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s, int K) {
    if (p.nsub == 0) return hipSuccess;
    // the node's weight table is held by the lanes of a wavefront, two entries each
    if constexpr (D * M2 > 128) {
        return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_interp_node<T, D, M2>), dim3(p.nsub, K), dim3(kResampleThreads), 0, s,
                           (const cplx<T> *)grid, p.geom, (const NodeRec<T, D> *)p.nodes, p.perm,
                           p.subs, (const T *)p.coef, p.window, win_params<T>(p), (cplx<T> *)fhat,
                           (long long)p.G, (long long)p.M);
        return hipGetLastError();
    }
}

// Every grid point is written (zeros where no node reaches), so the grid needs
// no clearing first.
template <typename T, int D, int M2>
hipError_t run_spread_owner(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s,
                            int K) {
    // padded accumulator layout where it fits beside the staged candidates
    const size_t stat = owner_static_lds(D, M2, (int)sizeof(T));
    const size_t cell_bytes = 2 * OwnerAcc<T>::type::kSlots * sizeof(unsigned long long);
    OwnerLayout lay = owner_layout(p.geom, D, true);
    if ((size_t)lay.cells * cell_bytes + stat > (size_t)p.lds_limit) lay = owner_layout(p.geom, D, false);
    const size_t shm = (size_t)lay.cells * cell_bytes;
    const double wprod = window_bound(D);
    auto kern = k_spread_owner<T, D, M2>;
    hipError_t e = allow_lds(kern, shm, stat);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(p.geom.ntiles, K), dim3(kOwnerThreads), shm, s,
                       (cplx<T> *)grid, p.geom, (const NodeRec<T, D> *)p.nodes, p.perm,
                       p.key_start, (const T *)p.coef, p.window, win_params<T>(p), (T)wprod,
                       (const cplx<T> *)fhat, (long long)p.G, (long long)p.M, lay);
    return hipGetLastError();
}

}  // namespace nfft
