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
// over the taps of the other axes, taking their weights from the lanes that
// computed them (DPP moves for 8-lane groups, shuffles otherwise).
//
// Both kernels work through their nodes in chunks of one node per thread: the
// chunk's node data (and, for spreading, the gathered fhat values) are first
// loaded by all threads at once into LDS, so the dependent global loads are
// paid once per chunk instead of once per node.
//
// Interpolation (forward): the workgroup of a work item (tile, node range) copies
// the tile plus a (2m-1)-wide trailing halo of the grid into LDS, wrapping the
// indices at the copy (the paper's blocked Algorithm "Block-Partitioned
// Resampling" with the copy-in of its local cache), then sums over the stencil
// of every node and reduces the group's partial sums.
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

constexpr int kResampleThreads = 256;  // workgroup size = nodes staged per chunk

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

// ---- lane exchange within a group of G lanes -------------------------------

// DPP control words (GFX9): quad_perm(p0,p1,p2,p3), row_shl:n, row_shr:n.
constexpr int dpp_quad(int a, int b, int c, int d) { return a | (b << 2) | (c << 4) | (d << 6); }
constexpr int kRowShl = 0x100, kRowShr = 0x110;

template <int CTRL> __device__ inline float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ inline double dpp(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// dst = src moved by CTRL in the lanes of the enabled banks (4-lane groups of a
// 16-lane row), old elsewhere.  The move always runs with the whole wavefront
// active; a bank mask instead of a select keeps the compiler from turning the
// choice into a branch that would run the move with its source lanes disabled.
template <int CTRL, int BANKS> __device__ inline float dpp_banks(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), CTRL,
                                                      0xF, BANKS, false));
}
template <int CTRL, int BANKS> __device__ inline double dpp_banks(double old, double src) {
    const long long o = __double_as_longlong(old), b = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffff), (int)(b & 0xffffffff), CTRL,
                                               0xF, BANKS, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, 0xF, BANKS,
                                               false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Value of lane A of this lane's group (groups are G consecutive lanes).  For
// G = 8 a group is two quads (banks) of one 16-lane DPP row: broadcast lane
// A & 3 inside every quad, then copy the source quad's value four lanes over
// into the other quad (banks 1 and 3 receive from below, banks 0 and 2 from above).
template <int G, int A, typename T> __device__ inline T group_bcast(T v, int gbase) {
    if constexpr (G == 8) {
        constexpr int q = A & 3;
        const T t = dpp<dpp_quad(q, q, q, q)>(v);
        if constexpr (A < 4) return dpp_banks<kRowShr + 4, 0xA>(t, t);
        else return dpp_banks<kRowShl + 4, 0x5>(t, t);
    } else {
        return __shfl(v, gbase + A, 64);
    }
}

// Sum over the group; the result is valid in the group's first lane.
template <int G, typename T> __device__ inline T group_sum(T v, int li) {
    if constexpr (G == 8 || G == 16) {
        v += dpp<dpp_quad(1, 0, 3, 2)>(v);
        v += dpp<dpp_quad(2, 3, 0, 1)>(v);
        v += dpp<kRowShl + 4>(v);
        if constexpr (G == 16) v += dpp<kRowShl + 8>(v);
        return v;
    } else {
        constexpr int P = G <= 1 ? 1 : G <= 2 ? 2 : G <= 4 ? 4 : G <= 8 ? 8 : G <= 16 ? 16 : 32;
#pragma unroll
        for (int off = P / 2; off >= 1; off >>= 1) {
            const T o = __shfl_down(v, off, 64);
            if (li + off < G) v += o;
        }
        return v;
    }
}

// out[a] = value of lane a of the group, a = 0..G-1.
template <int G, int A, typename T> struct BcastAll {
    __device__ static inline void run(T *out, T v, int gbase) {
        out[A] = group_bcast<G, A>(v, gbase);
        BcastAll<G, A + 1, T>::run(out, v, gbase);
    }
};
template <int G, typename T> struct BcastAll<G, G, T> {
    __device__ static inline void run(T *, T, int) {}
};

// ---- staged node data -------------------------------------------------------

template <typename T, int D> struct Stage {
    int l[D][kResampleThreads];   // stencil origin relative to the workgroup's tile
    T fr[D][kResampleThreads];
    int idx[kResampleThreads];    // caller's node index
};

template <typename T, int D, int M2>
__global__ void __launch_bounds__(kResampleThreads)
    k_interp(const cplx<T> *__restrict__ grid, Geom g, const NodeRec<T, D> *__restrict__ nodes,
             const int *__restrict__ perm, const int4 *__restrict__ subs,
             const T *__restrict__ coef, int window, WinParams<T> wp, cplx<T> *__restrict__ fhat) {
    using C = cplx<T>;
    constexpr int Z = M2 + 1;
    constexpr int NPW = 64 / M2;
    extern __shared__ unsigned char smem_raw[];
    __shared__ Stage<T, D> st;
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
    for (int idx = threadIdx.x; idx < total; idx += kResampleThreads) {
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

    for (int c0 = sp.y; c0 < sp.z; c0 += kResampleThreads) {
        const int n = min(kResampleThreads, sp.z - c0);
        if (threadIdx.x < n) {
            const int node = c0 + threadIdx.x;
            const NodeRec<T, D> rec = nodes[node];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                st.l[d][threadIdx.x] = rec.o[d] - t0[d];
                st.fr[d][threadIdx.x] = rec.fr[d];
            }
            st.idx[threadIdx.x] = perm[node];
        }
        __syncthreads();  // also completes the tile copy on the first chunk
        for (int base = wave * NPW; base < n; base += (kResampleThreads / 64) * NPW) {
            const int k = base + grp;
            const bool valid = grp < NPW && k < n;
            const int ks = valid ? k : 0;
            T w[D];
            int l[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                l[d] = st.l[d][ks];
                w[d] = tap_weight<T, M2>(cf[d], st.fr[d][ks], li, window, wp.beta[d]);
            }
            T ar = (T)0, ai = (T)0;
            if constexpr (D == 1) {
                const C v = tile[l[0] + li];
                ar = w[0] * v.x;
                ai = w[0] * v.y;
            } else if constexpr (D == 2) {
                T w0[M2];
                BcastAll<M2, 0, T>::run(w0, w[0], gbase);
                const C *row = tile + l[0] * P[1] + l[1] + li;
#pragma unroll
                for (int a = 0; a < M2; ++a) {
                    const C v = row[a * P[1]];
                    ar = fma(w0[a], v.x, ar);
                    ai = fma(w0[a], v.y, ai);
                }
                ar *= w[1];
                ai *= w[1];
            } else {
                T w0[M2], w1[M2];
                BcastAll<M2, 0, T>::run(w0, w[0], gbase);
                BcastAll<M2, 0, T>::run(w1, w[1], gbase);
                const C *base3 = tile + (l[0] * P[1] + l[1]) * P[2] + l[2] + li;
#pragma unroll 2
                for (int a = 0; a < M2; ++a) {
                    T sr = (T)0, si = (T)0;
                    const C *rowp = base3 + a * P[1] * P[2];
#pragma unroll
                    for (int b = 0; b < M2; ++b) {
                        const C v = rowp[b * P[2]];
                        sr = fma(w1[b], v.x, sr);
                        si = fma(w1[b], v.y, si);
                    }
                    ar = fma(w0[a], sr, ar);
                    ai = fma(w0[a], si, ai);
                }
                ar *= w[2];
                ai *= w[2];
            }
            ar = group_sum<M2>(ar, li);
            ai = group_sum<M2>(ai, li);
            if (valid && li == 0) fhat[st.idx[ks]] = cmake<C>(ar, ai);
        }
        __syncthreads();
    }
}

// ---- spreading accumulators --------------------------------------------------
//
// LDS float atomics are slow on this hardware, so the tile is accumulated in
// fixed point with 64-bit integer LDS atomics, which also makes the sum exact
// and independent of the order of the additions.  Each workgroup picks a
// power-of-two scale s from the largest |Re|, |Im| of its nodes' fhat and the
// window maximum, so that every scaled contribution c*s is below 2^30 (c64) or
// 2^62 (c128) in magnitude.
//   c64:  c*s is rounded to an int32 and added to one int64 per component
//         (resolution 2^-30 of the largest possible contribution; no
//         overflow below 2^33 contributions per grid point).
//   c128: c*s is split into hi = floor(c*s / 2^32) and lo = c*s - hi*2^32 in
//         [0, 2^32), added to an int64 and a uint64 per component (96 bits).
template <typename T> struct FixedPoint;

template <> struct FixedPoint<float> {
    static constexpr int kSlots = 1;  // int64 slots per component
    static constexpr double kLimit = 1073741824.0;  // 2^30
    __device__ static inline void add(unsigned long long *acc, int idx, int qtot, float c, float s) {
        const long long v = (long long)__float2int_rn(c * s);
        atomicAdd(acc + idx, (unsigned long long)v);
        (void)qtot;
    }
    __device__ static inline double read(const unsigned long long *acc, int idx, int qtot) {
        (void)qtot;
        return (double)(long long)acc[idx];
    }
};

template <> struct FixedPoint<double> {
    static constexpr int kSlots = 2;
    static constexpr double kLimit = 4611686018427387904.0;  // 2^62
    __device__ static inline void add(unsigned long long *acc, int idx, int qtot, double c, double s) {
        const double v = c * s;
        const int hi = __double2int_rd(v * 2.3283064365386963e-10);  // floor(v / 2^32)
        const double rest = v - (double)hi * 4294967296.0;               // in [0, 2^32)
        const unsigned lo = __double2uint_rd(rest);
        atomicAdd(acc + idx, (unsigned long long)(long long)hi);
        atomicAdd(acc + qtot + idx, (unsigned long long)lo);
    }
    __device__ static inline double read(const unsigned long long *acc, int idx, int qtot) {
        return (double)(long long)acc[idx] * 4294967296.0 + (double)acc[qtot + idx];
    }
};

template <typename T, int D> struct SpreadStage {
    static constexpr int kChunk = 2 * kResampleThreads;
    int l[D][kChunk];  // stencil origin relative to the workgroup's tile
    T fr[D][kChunk];
    T vr[kChunk];      // fhat value
    T vi[kChunk];
};

template <typename T, int D, int M2>
__global__ void __launch_bounds__(kResampleThreads)
    k_spread(cplx<T> *__restrict__ grid, Geom g, const NodeRec<T, D> *__restrict__ nodes,
             const int *__restrict__ perm, const int *__restrict__ key_start,
             const T *__restrict__ coef, int window, WinParams<T> wp, T wmax_prod,
             const cplx<T> *__restrict__ fhat) {
    using C = cplx<T>;
    using FP = FixedPoint<T>;
    constexpr int Z = M2 + 1;
    constexpr int NPW = 64 / M2;
    constexpr int NR = 1 << (2 * D);  // (shift e, class) pairs
    constexpr int CH = SpreadStage<T, D>::kChunk;
    extern __shared__ unsigned char smem_raw[];
    __shared__ SpreadStage<T, D> st;
    __shared__ int rbeg[NR];
    __shared__ int rpre[NR + 1];
    __shared__ unsigned long long amax_bits;  // bits of a non-negative double

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
    // fixed-point accumulators of the owned tile: [re slots][im slots], qtot each
    unsigned long long *acc_re = reinterpret_cast<unsigned long long *>(smem_raw);
    unsigned long long *acc_im = acc_re + FP::kSlots * qtot;
    for (int i = threadIdx.x; i < 2 * FP::kSlots * qtot; i += kResampleThreads) acc_re[i] = 0ull;
    if (threadIdx.x == 0) amax_bits = 0ull;

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

    // stage node v of the workgroup's list into slot s; returns max(|Re|, |Im|)
    auto stage = [&](int v, int slot) -> T {
        int lo = 0, hi = NR;  // largest r with rpre[r] <= v (a non-empty range)
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (rpre[mid] <= v) lo = mid;
            else hi = mid;
        }
        const int e = lo >> D;
        const int node = rbeg[lo] + (v - rpre[lo]);
        const NodeRec<T, D> rec = nodes[node];
        const C val = fhat[perm[node]];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            int ld = rec.o[d] - t0[d];
            if (((e >> d) & 1) && ld >= 0) ld -= g.Nt[d];
            st.l[d][slot] = ld;
            st.fr[d][slot] = rec.fr[d];
        }
        st.vr[slot] = val.x;
        st.vi[slot] = val.y;
        return fmax(fabs(val.x), fabs(val.y));
    };

    // pass over all nodes for the scale; the first chunk is staged on the way
    T amax = (T)0;
    for (int v = threadIdx.x; v < total; v += kResampleThreads) {
        if (v < CH) {
            amax = fmax(amax, stage(v, v));
        } else {
            int lo = 0, hi = NR;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (rpre[mid] <= v) lo = mid;
                else hi = mid;
            }
            const C val = fhat[perm[rbeg[lo] + (v - rpre[lo])]];
            amax = fmax(amax, fmax(fabs(val.x), fabs(val.y)));
        }
    }
    atomicMax(&amax_bits, (unsigned long long)__double_as_longlong((double)amax));
    __syncthreads();
    // power-of-two scale: every |contribution| * scale stays below the limit
    const double bound = __longlong_as_double((long long)amax_bits) * (double)wmax_prod;
    const T scale = bound > 0.0 ? (T)exp2(floor(log2(FP::kLimit / bound))) : (T)1;

    for (int c0 = 0; c0 < total; c0 += CH) {
        const int n = min(CH, total - c0);
        if (c0 > 0) {
            for (int k = threadIdx.x; k < n; k += kResampleThreads) stage(c0 + k, k);
            __syncthreads();
        }
        for (int base = wave * NPW; base < n; base += (kResampleThreads / 64) * NPW) {
            const int k = base + grp;
            const bool valid = grp < NPW && k < n;
            const int ks = valid ? k : 0;
            T w[D];
            int l[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                l[d] = st.l[d][ks];
                w[d] = tap_weight<T, M2>(cf[d], st.fr[d][ks], li, window, wp.beta[d]);
            }
            const int cl = l[D - 1] + li;
            const bool okl = valid && cl >= 0 && cl < g.Q[D - 1];
            const T wr = st.vr[ks] * w[D - 1], wi = st.vi[ks] * w[D - 1];
            if constexpr (D == 1) {
                if (okl) {
                    FP::add(acc_re, cl, qtot, wr, scale);
                    FP::add(acc_im, cl, qtot, wi, scale);
                }
            } else if constexpr (D == 2) {
                T w0[M2];
                BcastAll<M2, 0, T>::run(w0, w[0], gbase);
                const int Q1 = g.Q[1];
#pragma unroll
                for (int a = 0; a < M2; ++a) {
                    const int r0 = l[0] + a;
                    if (okl && r0 >= 0 && r0 < g.Q[0]) {
                        const int idx = r0 * Q1 + cl;
                        FP::add(acc_re, idx, qtot, w0[a] * wr, scale);
                        FP::add(acc_im, idx, qtot, w0[a] * wi, scale);
                    }
                }
            } else {
                T w0[M2], w1[M2];
                BcastAll<M2, 0, T>::run(w0, w[0], gbase);
                BcastAll<M2, 0, T>::run(w1, w[1], gbase);
                const int Q1 = g.Q[1], Q2 = g.Q[2];
#pragma unroll 2
                for (int a = 0; a < M2; ++a) {
                    const int r0 = l[0] + a;
                    const bool ok0 = okl && r0 >= 0 && r0 < g.Q[0];
                    const T ar = w0[a] * wr, ai = w0[a] * wi;
#pragma unroll
                    for (int b = 0; b < M2; ++b) {
                        const int r1 = l[1] + b;
                        if (ok0 && r1 >= 0 && r1 < Q1) {
                            const int idx = (r0 * Q1 + r1) * Q2 + cl;
                            FP::add(acc_re, idx, qtot, w1[b] * ar, scale);
                            FP::add(acc_im, idx, qtot, w1[b] * ai, scale);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }

    // write the owned tile: every grid value has exactly this one writer
    const double inv = 1.0 / (double)scale;
    for (int idx = threadIdx.x; idx < qtot; idx += kResampleThreads) {
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
        grid[gi] = cmake<C>((T)(FP::read(acc_re, idx, qtot) * inv),
                            (T)(FP::read(acc_im, idx, qtot) * inv));
    }
}

// Static LDS of the resampling kernels (staged node chunk and range table).
template <typename T, int D> constexpr size_t static_lds() {
    return sizeof(Stage<T, D>) + sizeof(SpreadStage<T, D>) + sizeof(int) * (2 * (1 << (2 * D)) + 2);
}

// Dynamic LDS beyond 64 KiB (static included) has to be allowed per kernel.
template <typename K> inline hipError_t allow_lds(K kernel, size_t dyn, size_t stat) {
    if (dyn + stat <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
}

template <typename T, int D, int M2>
hipError_t run_interp(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s) {
    int tot = 1;
    for (int d = 0; d < D; ++d) tot *= p.geom.Q[d] + M2 - 1;
    const size_t shm = (size_t)tot * sizeof(cplx<T>);
    WinParams<T> wp;
    for (int d = 0; d < kMaxD; ++d)
        wp.beta[d] = d < D ? (T)(M_PI * p.m * (2.0 - (double)p.N[d] / (double)p.Nt[d])) : (T)0;
    hipError_t e = allow_lds(k_interp<T, D, M2>, shm, static_lds<T, D>());
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_interp<T, D, M2>), dim3(p.nsub), dim3(kResampleThreads), shm, s,
                       (const cplx<T> *)grid, p.geom, (const NodeRec<T, D> *)p.nodes, p.perm,
                       p.subs, (const T *)p.coef, p.window, wp, (cplx<T> *)fhat);
    return hipGetLastError();
}

template <typename T, int D, int M2>
hipError_t run_spread(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s) {
    int tot = 1;
    for (int d = 0; d < D; ++d) tot *= p.geom.Q[d];
    const size_t shm = (size_t)tot * 2 * FixedPoint<T>::kSlots * sizeof(unsigned long long);
    WinParams<T> wp;
    double wprod = 1.0;
    for (int d = 0; d < kMaxD; ++d) {
        const double beta = d < D ? M_PI * p.m * (2.0 - (double)p.N[d] / (double)p.Nt[d]) : 0.0;
        wp.beta[d] = (T)beta;
        // window maximum psi_hat_Base(0) = sinh(beta)/pi, with margin for the polynomial fit
        if (d < D) wprod *= 1.5 * sinh(beta) / M_PI;
    }
    hipError_t e = allow_lds(k_spread<T, D, M2>, shm, static_lds<T, D>());
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_spread<T, D, M2>), dim3(p.geom.ntiles), dim3(kResampleThreads), shm, s,
                       (cplx<T> *)grid, p.geom, (const NodeRec<T, D> *)p.nodes, p.perm,
                       p.key_start, (const T *)p.coef, p.window, wp, (T)wprod,
                       (const cplx<T> *)fhat);
    return hipGetLastError();
}

}  // namespace nfft
