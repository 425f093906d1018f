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
// Work items: the nodes of a tile (binned by the tile of their stencil origin)
// are cut into items of bounded size, so that a dense tile is shared by several
// workgroups.  Node data are staged through LDS in chunks of one node per
// thread, so the dependent global loads are paid once per chunk.
//
// Interpolation (forward): the workgroup of an item copies the tile plus a
// (2m-1)-wide trailing halo of the grid into LDS, wrapping the indices at the
// copy (the paper's blocked Algorithm "Block-Partitioned Resampling" with the
// copy-in of its local cache), then sums over the stencil of every node and
// reduces the group's partial sums.
//
// Spreading (adjoint): the workgroup of an item accumulates its nodes' taps
// into the padded tile (tile + trailing halo) with LDS atomics and writes the
// padded tile to a scratch slot of its own; a merge kernel then sums, for every
// grid point, the padded tiles that cover it.  This replaces the locked
// addition into the global grid of the paper's "Block-Partitioned Adjoint
// Resampling": each grid value has exactly one writer and no global atomics
// are used.
#pragma once

#include <math.h>

#include "common.hpp"
#include "nfft_internal.hpp"

namespace nfft {

// Channels per interpolation workgroup of a multi-channel call: two where both
// channels' tiles fit 64 KiB beside the staged nodes (polynomial window, D <= 2), so
// that each node's weights serve both.  Measured on the 32-channel radial workload
// (2-D 256^2, M = 65536): interpolation 59 us with one channel per workgroup, 58 us
// with two, 73 us with four (one workgroup per CU fewer than the latency needs).
template <typename T, int D> inline int interp_channel_block(int K, bool gw, size_t tile) {
    if (D > 2 || gw || K < 2) return 1;
    return 2 * tile + interp_static_lds(D, (int)sizeof(T)) <= 65536 ? 2 : 1;
}

template <typename T> struct WinParams {
    T beta[kMaxD];
    T inv_peak[kMaxD];  // direct evaluation: pi / sinh(beta), the stored window's normalisation
    const T *tab;  // TENSOR / FULL: weights per sorted node; LINEAR: S samples per axis
    long long S;   // LINEAR table entries per axis
    int m;         // window half-width (M2 = 2m, or 2m + 2 with the wide stencil)
};

// Window value of tap t for a node with offset frac (lane-owned coefficients cf;
// lin: the axis's LINEAR table of S entries).  Tap t sits at u = (frac + M2/2 -
// 1 - t) / m; with the wide stencil (M2 = 2m + 2) the outer taps lie beyond
// |u| = 1, where the untruncated window continues as sin(beta sqrt(u^2-1)) /
// (pi sqrt(u^2-1)).  Every mode returns the window divided by its peak
// sinh(beta)/pi (the polynomial and the tables are fitted and filled that way; the
// direct evaluation multiplies by inv_peak).
template <typename T, int M2>
__device__ inline T tap_weight(const T *cf, T frac, int t, int window, T beta, T inv_peak,
                               const T *lin, long long S, int m) {
    if (window == NFFT_WINDOW_POLY) {
        // degree 2m; coefficients above it are zero (wide stencil: M2 = 2m + 2)
        const T z = frac - (T)0.5;
        T acc = cf[M2];
#pragma unroll
        for (int k = M2 - 1; k >= 0; --k) acc = fma(acc, z, cf[k]);
        return acc;
    }
    constexpr int lo = M2 / 2 - 1;
    if (window == NFFT_WINDOW_LINEAR) {
        // kappa = |u| (S - 2), s = floor(kappa), alpha = kappa - s; |u| <= 1, so s + 1 < S
        const double u = ((double)frac + (double)(lo - t)) / (double)m;
        const double kappa = fabs(u) * (double)(S - 2);
        long long i = (long long)kappa;
        if (i > S - 2) i = S - 2;
        const T alpha = (T)(kappa - (double)i);
        const T a = lin[i], b = lin[i + 1];
        return a + alpha * (b - a);
    }
    const T u = (frac + (T)(lo - t)) / (T)m;
    const T s2 = (T)1 - u * u;
    if (s2 < (T)0) {  // wide stencil only: beyond the truncation interval
        const T r = sqrt(-s2);
        return sin(beta * r) / ((T)M_PI * r) * inv_peak;
    }
    const T s = s2 > (T)0 ? sqrt(s2) : (T)0;
    return (s > (T)0 ? sinh(beta * s) / ((T)M_PI * s) : beta / (T)M_PI) * inv_peak;
}

// Polynomial window weight of a tap and its derivative in frac (one Horner pass
// for both: P(z) and P'(z) at z = frac - 1/2).
template <typename T, int M2>
__device__ inline T poly_weight_d(const T *cf, T frac, T &dw) {
    const T z = frac - (T)0.5;
    T p = cf[M2], dp = (T)0;
#pragma unroll
    for (int k = M2 - 1; k >= 0; --k) {
        dp = fma(dp, z, p);
        p = fma(p, z, cf[k]);
    }
    dw = dp;
    return p;
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

// ---- box traversal ------------------------------------------------------------

// Row-wise traversal of a box whose last (contiguous) axis has n cells: each
// wavefront takes 64/lpr rows at a time, lpr lanes per row (lpr = the smallest
// power of two >= n, at most 64), so that no index needs a division per cell.
struct BoxRows {
    int lpr, rpw;
    __device__ explicit BoxRows(int n) {
        lpr = 64;
        while (lpr >= 2 * n && lpr > 1) lpr >>= 1;
        rpw = 64 / lpr;
    }
    __device__ int first_row() const { return (threadIdx.x >> 6) * rpw + (threadIdx.x & 63) / lpr; }
    __device__ int row_step() const { return (kResampleThreads / 64) * rpw; }
    __device__ int first_col() const { return (threadIdx.x & 63) % lpr; }
};

// ---- staged node data -------------------------------------------------------

template <typename T, int D, int CH_ = stage_chunk(D, (int)sizeof(T))> struct Stage {
    static constexpr int kChunk = CH_;
    int l[D][kChunk];  // stencil origin relative to the workgroup's tile, in [0, Q)
    T fr[D][kChunk];
    T vr[kChunk];      // spreading: fhat value
    T vi[kChunk];
    int idx[kChunk];   // interpolation: caller's node index
};

// Lane li of a group computes the weight of tap li along every axis; cf holds
// the polynomial coefficients of that tap per axis.
template <typename T, int D, int M2> struct LaneWindow {
    T cf[D][M2 + 1];
    // m: window half-width; the table holds 2m + 1 coefficients per (axis, tap)
    __device__ void load(const T *__restrict__ coef, int li, int m) {
        const int Z = 2 * m + 1;
#pragma unroll
        for (int d = 0; d < D; ++d)
#pragma unroll
            for (int z = 0; z <= M2; ++z)
                cf[d][z] = z < Z ? coef[((size_t)d * M2 + li) * Z + z] : (T)0;
    }
};

// Weights of this lane's tap li along every axis for the node at sorted
// position gk (TENSOR and FULL read the plan's per-node tables; FULL keeps the
// last axis's factor at 1 because its row weights are whole products).
//
// GW = false instantiates the polynomial window alone (the default mode, kept
// free of the other modes' branches and registers); GW = true handles all modes.
template <bool GW, typename T, int D, int M2>
__device__ inline void node_weights(T *w, const LaneWindow<T, D, M2> &lw, const T *fr, long long gk,
                                    int li, int window, const WinParams<T> &wp) {
    if constexpr (!GW) {
#pragma unroll
        for (int d = 0; d < D; ++d)
            w[d] = tap_weight<T, M2>(lw.cf[d], fr[d], li, NFFT_WINDOW_POLY, wp.beta[d],
                                     wp.inv_peak[d], nullptr, 0, wp.m);
        return;
    }
    if (window == NFFT_WINDOW_TENSOR) {
#pragma unroll
        for (int d = 0; d < D; ++d) w[d] = wp.tab[(gk * D + d) * M2 + li];
    } else if (window == NFFT_WINDOW_FULL) {
#pragma unroll
        for (int d = 0; d < D; ++d) w[d] = (T)1;
        if (D == 1) w[0] = wp.tab[gk * M2 + li];
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d)
            w[d] = tap_weight<T, M2>(lw.cf[d], fr[d], li, window, wp.beta[d], wp.inv_peak[d],
                                     wp.tab + d * wp.S, wp.S, wp.m);
    }
}

// Row weights of a 2-D node: the weights of axis 0 broadcast from the group's
// lanes, or, with FULL, the lane's own column of the node's (2m)^2 products.
template <bool GW, typename T, int M2>
__device__ inline void row_weights_2d(T *w0, T w_axis0, long long gk, int li, int gbase, int window,
                                      const WinParams<T> &wp) {
    if (GW && window == NFFT_WINDOW_FULL) {
#pragma unroll
        for (int a = 0; a < M2; ++a) w0[a] = wp.tab[(gk * M2 + a) * M2 + li];
    } else {
        BcastAll<M2, 0, T>::run(w0, w_axis0, gbase);
    }
}

// DV = true (polynomial window only): instead of fhat, the D partial derivatives
// of the interpolated value with respect to the node's coordinates -- the
// derivative-of-window interpolation d fhat_j / d x_jd = sum over the stencil of
// Nt_d P'_{t_d}(frac_d - 1/2) prod_{e != d} P_{t_e} times the grid value -- written
// to fhat[d * fstride + j].
// item: the work item (index into subs) of the workgroup; kb: the channels it serves
// (grids at stride gstride, fhat at stride fstride; the derivative mode takes one).
// Every channel's tile is in LDS at once, so each node's weights are evaluated once
// and serve all kb channels.
template <typename T, int D, int M2, bool GW, bool DV, int NT, int KB = 1>
__device__ inline void interp_body(const cplx<T> *__restrict__ grid, const Geom &g,
                                   const NodeRec<T, D> *__restrict__ nodes,
                                   const int *__restrict__ perm, const int4 *__restrict__ subs,
                                   const T *__restrict__ coef, int window, const WinParams<T> &wp,
                                   cplx<T> *__restrict__ fhat, long long fstride, int item,
                                   int kb = 1, long long gstride = 0) {
    using C = cplx<T>;
    constexpr int NPW = 64 / M2;
    using StageT = Stage<T, D, interp_chunk(D, (int)sizeof(T))>;
    constexpr int CH = StageT::kChunk;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ StageT st;
    C *tile = reinterpret_cast<C *>(smem_raw);

    const int4 sp = subs[item];
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
    // the first chunk's node loads go out before the tile copy, so that both
    // latencies overlap (the chunk is written to LDS after the copy)
    constexpr int SJ = (CH + NT - 1) / NT;
    NodeRec<T, D> rec[SJ];
    int pm[SJ];
    auto load_chunk = [&](int c0, int n) {
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
            const int node = c0 + min((int)threadIdx.x + j * NT, n - 1);
            rec[j] = nodes[node];
            pm[j] = perm[node];
        }
    };
    auto store_chunk = [&](int n) {
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
            const int k = threadIdx.x + j * NT;
            if (k < n) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    st.l[d][k] = rec[j].o[d] - t0[d];
                    st.fr[d][k] = rec[j].fr[d];
                }
                st.idx[k] = pm[j];
            }
        }
    };
    load_chunk(sp.y, min(CH, sp.z - sp.y));

    // copy the tile and its trailing halo into LDS, wrapping at the grid edge;
    // eight loads per thread are in flight before the first LDS write
    int ptot = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) ptot *= P[d];
    for (int ch = 0; ch < kb; ++ch) {
        const int total = ptot;
        const cplx<T> *gsrc = grid + ch * gstride;
        C *tdst = tile + ch * ptot;
        const float rl = 1.0f / (float)P[D - 1];
        const float r1 = D == 3 ? 1.0f / (float)P[1] : 1.0f;
        constexpr int U = 8;
        for (int base = 0; base < total; base += U * NT) {
            C v[U];
            int dst[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = base + u * NT + threadIdx.x;
                dst[u] = idx < total ? idx : -1;
                int col;
                const int row = small_divmod(idx < total ? idx : 0, P[D - 1], rl, col);
                long long gb = 0;
                if constexpr (D >= 2) {
                    int a1 = 0;
                    const int a0 = D == 3 ? small_divmod(row, P[1], r1, a1) : row;
                    int c0 = t0[0] + a0;
                    if (c0 >= g.Nt[0]) c0 -= g.Nt[0];
                    gb = c0;
                    if constexpr (D == 3) {
                        int c1 = t0[1] + a1;
                        if (c1 >= g.Nt[1]) c1 -= g.Nt[1];
                        gb = gb * g.Nt[1] + c1;
                    }
                    gb *= g.Nt[D - 1];
                }
                int c = t0[D - 1] + col;
                if (c >= g.Nt[D - 1]) c -= g.Nt[D - 1];
                v[u] = gsrc[gb + c];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (dst[u] >= 0) tdst[dst[u]] = v[u];
        }
    }

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / M2, li = lane - grp * M2, gbase = grp * M2;
    LaneWindow<T, D, M2> lw;
    lw.load(coef, li, wp.m);

    for (int c0 = sp.y; c0 < sp.z; c0 += CH) {
        const int n = min(CH, sp.z - c0);
        // all loads first (indices clamped into the item), then the LDS writes
        if (c0 > sp.y) load_chunk(c0, n);
        store_chunk(n);
        __syncthreads();  // also completes the tile copy on the first chunk
        for (int base = wave * NPW; base < n; base += (NT / 64) * NPW) {
            const int k = base + grp;
            const bool valid = grp < NPW && k < n;
            const int ks = valid ? k : 0;
            T w[D], fr[D];
            int l[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                l[d] = st.l[d][ks];
                fr[d] = st.fr[d][ks];
            }
            const long long gk = c0 + ks;  // sorted position of the node
            if constexpr (DV) {
                T dw[D];
#pragma unroll
                for (int d = 0; d < D; ++d) w[d] = poly_weight_d<T, M2>(lw.cf[d], fr[d], dw[d]);
                T orr[D], oi[D];  // d/dx_d, real and imaginary parts
                if constexpr (D == 1) {
                    const C v = tile[l[0] + li];
                    orr[0] = dw[0] * v.x;
                    oi[0] = dw[0] * v.y;
                } else if constexpr (D == 2) {
                    T w0[M2], dw0[M2];
                    BcastAll<M2, 0, T>::run(w0, w[0], gbase);
                    BcastAll<M2, 0, T>::run(dw0, dw[0], gbase);
                    const C *row = tile + l[0] * P[1] + l[1] + li;
                    T sr = (T)0, si = (T)0, dr = (T)0, di = (T)0;
#pragma unroll
                    for (int a = 0; a < M2; ++a) {
                        const C v = row[a * P[1]];
                        sr = fma(w0[a], v.x, sr);
                        si = fma(w0[a], v.y, si);
                        dr = fma(dw0[a], v.x, dr);
                        di = fma(dw0[a], v.y, di);
                    }
                    orr[0] = dr * w[1];
                    oi[0] = di * w[1];
                    orr[1] = sr * dw[1];
                    oi[1] = si * dw[1];
                } else {
                    T w0[M2], dw0[M2], w1[M2], dw1[M2];
                    BcastAll<M2, 0, T>::run(w0, w[0], gbase);
                    BcastAll<M2, 0, T>::run(dw0, dw[0], gbase);
                    BcastAll<M2, 0, T>::run(w1, w[1], gbase);
                    BcastAll<M2, 0, T>::run(dw1, dw[1], gbase);
                    const C *base3 = tile + (l[0] * P[1] + l[1]) * P[2] + l[2] + li;
                    T a0r = (T)0, a0i = (T)0, a1r = (T)0, a1i = (T)0, a2r = (T)0, a2i = (T)0;
#pragma unroll
                    for (int a = 0; a < M2; ++a) {
                        T rr = (T)0, ri = (T)0, qr = (T)0, qi = (T)0;
                        const C *rowp = base3 + a * P[1] * P[2];
#pragma unroll
                        for (int b = 0; b < M2; ++b) {
                            const C v = rowp[b * P[2]];
                            rr = fma(w1[b], v.x, rr);
                            ri = fma(w1[b], v.y, ri);
                            qr = fma(dw1[b], v.x, qr);
                            qi = fma(dw1[b], v.y, qi);
                        }
                        a0r = fma(dw0[a], rr, a0r);
                        a0i = fma(dw0[a], ri, a0i);
                        a1r = fma(w0[a], qr, a1r);
                        a1i = fma(w0[a], qi, a1i);
                        a2r = fma(w0[a], rr, a2r);
                        a2i = fma(w0[a], ri, a2i);
                    }
                    orr[0] = a0r * w[2];
                    oi[0] = a0i * w[2];
                    orr[1] = a1r * w[2];
                    oi[1] = a1i * w[2];
                    orr[2] = a2r * dw[2];
                    oi[2] = a2i * dw[2];
                }
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    orr[d] = group_sum<M2>(orr[d], li);
                    oi[d] = group_sum<M2>(oi[d], li);
                }
                if (valid && li == 0)
#pragma unroll
                    for (int d = 0; d < D; ++d)
                        fhat[(long long)d * fstride + st.idx[ks]] =
                            cmake<C>(orr[d] * (T)g.Nt[d], oi[d] * (T)g.Nt[d]);
                continue;
            }
            node_weights<GW, T, D, M2>(w, lw, fr, gk, li, window, wp);
            // the broadcast row weights of the node, for every channel
            T w0[D >= 2 ? M2 : 1], w1[D == 3 ? M2 : 1];
            if constexpr (D == 2) row_weights_2d<GW, T, M2>(w0, w[0], gk, li, gbase, window, wp);
            if constexpr (D == 3) {
                BcastAll<M2, 0, T>::run(w0, w[0], gbase);
                BcastAll<M2, 0, T>::run(w1, w[1], gbase);
            }
            const int dst = st.idx[ks];
#pragma unroll
            for (int ch = 0; ch < KB; ++ch) {
                if (ch >= kb) break;
                const C *tc = tile + ch * ptot;
                T ar = (T)0, ai = (T)0;
                if constexpr (D == 1) {
                    const C v = tc[l[0] + li];
                    ar = w[0] * v.x;
                    ai = w[0] * v.y;
                } else if constexpr (D == 2) {
                    const C *row = tc + l[0] * P[1] + l[1] + li;
#pragma unroll
                    for (int a = 0; a < M2; ++a) {
                        const C v = row[a * P[1]];
                        ar = fma(w0[a], v.x, ar);
                        ai = fma(w0[a], v.y, ai);
                    }
                    ar *= w[1];
                    ai *= w[1];
                } else {
                    const C *base3 = tc + (l[0] * P[1] + l[1]) * P[2] + l[2] + li;
#pragma unroll
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
                if (valid && li == 0) fhat[ch * fstride + dst] = cmake<C>(ar, ai);
            }
        }
        __syncthreads();
    }
}

template <typename T, int D, int M2, bool GW, bool DV = false, int NT = kResampleThreads, int KB = 1>
__global__ void __launch_bounds__(NT)
    k_interp(const cplx<T> *__restrict__ grid, Geom g, const NodeRec<T, D> *__restrict__ nodes,
             const int *__restrict__ perm, const int4 *__restrict__ subs,
             const T *__restrict__ coef, int window, WinParams<T> wp, cplx<T> *__restrict__ fhat,
             long long gstride, long long fstride, int K) {
    // channel block blockIdx.y: channels KB * blockIdx.y .. (at most KB of the K)
    const int c0 = blockIdx.y * KB;
    interp_body<T, D, M2, GW, DV, NT, KB>(grid + c0 * gstride, g, nodes, perm, subs, coef, window,
                                          wp, fhat + c0 * fstride, fstride, blockIdx.x,
                                          min(KB, K - c0), gstride);
}

// ---- spreading accumulators --------------------------------------------------
//
// LDS float atomics are slow on this hardware (measured about 30 times slower
// than integer ones), so the tile is accumulated in fixed point with 64-bit
// integer LDS atomics, which also makes the sum exact and independent of the
// order of the additions.  Each workgroup scales its contributions c by s, from
// the largest |Re|, |Im| of its nodes' fhat times the bound of the window product
// (window_bound), so that every |c*s| is below a limit; one int64 per component and
// grid point:
//   c64:  s is a power of two, |c*s| < 2^30, truncated to an int32 (resolution
//         2^-30 of the largest possible contribution; no overflow below 2^33
//         contributions per point; s and 1/s exact).
//   c128: s = limit(n) / bound, limit(n) = min(2^51 (1 - 2^-10), 2^62 / n') for a
//         workgroup of n nodes (n' = n rounded up to a power of two): a node adds to
//         a grid point at most once, so n contributions stay below 2^62, and below
//         2^51 the rounding to the nearest integer is exact by adding 1.5 * 2^52 and
//         reading the integer off the mantissa.  Resolution 2^-51 of the largest
//         possible contribution for n <= 2048 (FP64 rounds each value to 2^-53 of
//         itself); s is not a power of two, so the read-out's 1/s adds one FP64
//         rounding.
// The accumulators are planes of the padded tile (structure of arrays): plane
// s holds slot s of every cell, so one atomic instruction of a wavefront (eight
// nodes' rows of 2m consecutive cells) touches consecutive 8-byte words of one
// plane and spreads over all LDS banks.  Planes: [Re][Im].
template <typename T> struct FixedPoint;

// Magnitude a value contributes to the fixed-point scale: max(|Re|, |Im|), or +infinity
// when either part is NaN or infinite (fmax alone would skip a NaN).  A work item whose
// maximum is infinite holds a non-finite value: it skips the accumulation (whose integer
// conversion would drop a NaN and saturate on an infinity) and writes NaN instead, which
// the halo merge and the FFT carry to every output of the adjoint.
template <typename T> __device__ inline T scale_mag(T re, T im) {
    return (isfinite(re) && isfinite(im)) ? fmax(fabs(re), fabs(im)) : (T)INFINITY;
}

// The nearest integer to v, |v| < 2^51: v + 1.5 * 2^52 lies in (2^52, 2^53), where
// the spacing of doubles is 1, and the integer is its mantissa less the shift's
// (the addition is kept separate from the product that forms v, so that every
// instantiation rounds the same way).
__device__ inline long long round_to_ll(double v) {
    return __double_as_longlong(__dadd_rn(v, 6755399441055744.0)) - 0x4338000000000000LL;
}

template <> struct FixedPoint<float> {
    static constexpr int kSlots = 1;  // int64 slots per component
    // scale for contributions bounded by `bound` (> 0) in a workgroup of n nodes
    __device__ static inline float scale(double bound, int) {
        int e;
        (void)frexp(1073741824.0 / bound, &e);  // 2^30 / bound = f 2^e, f in [0.5, 1)
        return (float)ldexp(1.0, e - 1);
    }
    // a: the cell's word in plane 0; ps: plane size (cells); cr, ci: scaled, |c| < 2^30
    __device__ static inline void add(unsigned long long *a, int ps, float cr, float ci) {
        atomicAdd(a, (unsigned long long)(long long)(int)cr);
        atomicAdd(a + ps, (unsigned long long)(long long)(int)ci);
    }
    // the contributions w * pr, w * pi
    __device__ static inline void add_prod(unsigned long long *a, int ps, float w, float pr, float pi) {
        add(a, ps, w * pr, w * pi);
    }
    __device__ static inline double read(const unsigned long long *a, int ps, int comp) {
        return (double)(long long)a[(size_t)comp * ps];
    }
};

template <> struct FixedPoint<double> {
    static constexpr int kSlots = 1;
    // n: the most contributions one grid point can receive (the workgroup's nodes)
    __device__ static inline double scale(double bound, int n) {
        double l = 4611686018427387904.0;  // 2^62
        for (int c = 1; c < n; c *= 2) l *= 0.5;
        const double lmax = 2251799813685248.0 * (1.0 - 1.0 / 1024.0);  // 2^51 (1 - 2^-10)
        return (l < lmax ? l : lmax) / bound;
    }
    __device__ static inline void add(unsigned long long *a, int ps, double cr, double ci) {
        atomicAdd(a, (unsigned long long)round_to_ll(cr));
        atomicAdd(a + ps, (unsigned long long)round_to_ll(ci));
    }
    // the contributions w * pr, w * pi, each rounded to the nearest integer in one fused
    // multiply-add with the shift (one instruction fewer per component than product then
    // shift; the exact product is rounded once)
    __device__ static inline void add_prod(unsigned long long *a, int ps, double w, double pr,
                                           double pi) {
        const double shift = 6755399441055744.0;  // 1.5 * 2^52
        atomicAdd(a, (unsigned long long)(__double_as_longlong(fma(w, pr, shift)) - 0x4338000000000000LL));
        atomicAdd(a + ps, (unsigned long long)(__double_as_longlong(fma(w, pi, shift)) - 0x4338000000000000LL));
    }
    __device__ static inline double read(const unsigned long long *a, int ps, int comp) {
        return (double)(long long)a[(size_t)comp * ps];
    }
};

// The exact 96-bit complex128 accumulator of the tile-owner spreading (D = 4), whose
// workgroups take contributions from every node of up to 81 tiles, too many for a
// 64-bit sum at full resolution: c*s below 2^62 is split into hi = floor(c*s / 2^32)
// and lo = c*s - hi*2^32 in [0, 2^32), added to an int64 and a uint64 (two slots per
// component: planes [Re hi][Re lo][Im hi][Im lo]).
struct FixedPoint96 {
    static constexpr int kSlots = 2;
    __device__ static inline double scale(double bound, int) {
        int e;
        (void)frexp(4611686018427387904.0 / bound, &e);  // 2^62 / bound = f 2^e
        return ldexp(1.0, e - 1);
    }
    __device__ static inline void add1(unsigned long long *a, int ps, double v) {
        const int hi = __double2int_rd(v * 2.3283064365386963e-10);  // floor(v / 2^32)
        const double rest = v - (double)hi * 4294967296.0;               // in [0, 2^32)
        const unsigned lo = __double2uint_rd(rest);
        atomicAdd(a, (unsigned long long)(long long)hi);
        atomicAdd(a + ps, (unsigned long long)lo);
    }
    __device__ static inline void add(unsigned long long *a, int ps, double cr, double ci) {
        add1(a, ps, cr);
        add1(a + 2 * (size_t)ps, ps, ci);
    }
    __device__ static inline double read(const unsigned long long *a, int ps, int comp) {
        const unsigned long long *c = a + (size_t)2 * comp * ps;
        return (double)(long long)c[0] * 4294967296.0 + (double)c[ps];
    }
};
// Accumulator of the tile-owner spreading per type.
template <typename T> struct OwnerAcc { using type = FixedPoint<T>; };
template <> struct OwnerAcc<double> { using type = FixedPoint96; };

// Spreading of one work item (a tile's node range, at most a few hundred to a
// thousand nodes).  The workgroup accumulates the item's contributions into
// the tile extended by the (2m-1)-wide trailing halo, in LDS, and writes that
// padded tile to its own slot of the scratch buffer.  Every node's stencil lies
// inside the padded tile, so the tap loops carry no bounds tests.
// item: the work item (index into subs, and the padded tile's slot in pad).
template <typename T, int D, int M2, bool GW, int NT>
__device__ inline void spread_body(cplx<T> *__restrict__ pad, const Geom &g,
                                   const NodeRec<T, D> *__restrict__ nodes,
                                   const int *__restrict__ perm, const int4 *__restrict__ subs,
                                   const T *__restrict__ coef, int window, const WinParams<T> &wp,
                                   T wmax_prod, const cplx<T> *__restrict__ fhat, int item) {
    using C = cplx<T>;
    using FP = FixedPoint<T>;
    constexpr int NPW = 64 / M2;
    constexpr int CH = Stage<T, D>::kChunk;
    constexpr int SL = 2 * FP::kSlots;  // accumulator slots per grid point
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ Stage<T, D> st;
    __shared__ unsigned long long amax_bits;  // bits of a non-negative double

    const int4 sp = subs[item];
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
    int ptot = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) ptot *= P[d];
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem_raw);
    for (int i = threadIdx.x; i < SL * ptot; i += NT) acc[i] = 0ull;
    if (threadIdx.x == 0) amax_bits = 0ull;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / M2, li = lane - grp * M2, gbase = grp * M2;
    LaneWindow<T, D, M2> lw;
    lw.load(coef, li, wp.m);

    // Stage the chunk of nodes [c0, c0 + n) into LDS: all global loads of the
    // thread's nodes are issued before the first one is waited for (indices are
    // clamped into the item, so the loads need no guard); returns max |Re|, |Im|.
    constexpr int SJ = (CH + NT - 1) / NT;
    auto stage_chunk_nodes = [&](int c0, int n) -> T {
        NodeRec<T, D> rec[SJ];
        int pm[SJ];
        C val[SJ];
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
            const int node = c0 + min(threadIdx.x + j * NT, n - 1);
            rec[j] = nodes[node];
            pm[j] = perm[node];
        }
#pragma unroll
        for (int j = 0; j < SJ; ++j) val[j] = fhat[pm[j]];
        T mx = (T)0;
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
            const int k = threadIdx.x + j * NT;
            if (k < n) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    st.l[d][k] = rec[j].o[d] - t0[d];
                    st.fr[d][k] = rec[j].fr[d];
                }
                st.vr[k] = val[j].x;
                st.vi[k] = val[j].y;
                mx = fmax(mx, scale_mag(val[j].x, val[j].y));
            }
        }
        return mx;
    };

    // pass over the item's nodes for the scale; the first chunk is staged on the way
    const int nitem = sp.z - sp.y;
    T amax = stage_chunk_nodes(sp.y, min(CH, nitem));
    for (int v = CH + threadIdx.x; v < nitem; v += NT) {
        const C val = fhat[perm[sp.y + v]];
        amax = fmax(amax, scale_mag(val.x, val.y));
    }
    // wavefront maximum, then one LDS atomic per wavefront (non-negative values
    // order like their bit patterns)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    __syncthreads();  // amax_bits is initialised
    if (lane == 0) atomicMax(&amax_bits, (unsigned long long)__double_as_longlong((double)amax));
    __syncthreads();
    // power-of-two scale: every |contribution| * scale stays below the limit;
    // with limit/bound = f 2^e, f in [0.5, 1): scale = 2^(e-1)
    const double amax_d = __longlong_as_double((long long)amax_bits);
    const bool poisoned = isinf(amax_d);  // a non-finite value in the item (same in every thread)
    const double bound = amax_d * (double)wmax_prod;
    const T scale = bound > 0.0 && !poisoned ? FP::scale(bound, nitem) : (T)1;

    for (int c0 = sp.y; c0 < (poisoned ? sp.y : sp.z); c0 += CH) {
        const int n = min(CH, sp.z - c0);
        if (c0 > sp.y) {
            (void)stage_chunk_nodes(c0, n);
            __syncthreads();
        }
        for (int base = wave * NPW; base < n; base += (NT / 64) * NPW) {
            const int k = base + grp;
            const bool valid = grp < NPW && k < n;
            const int ks = valid ? k : 0;
            T w[D], fr[D];
            int l[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                l[d] = st.l[d][ks];
                fr[d] = st.fr[d][ks];
            }
            const long long gk = c0 + ks;  // sorted position of the node
            node_weights<GW, T, D, M2>(w, lw, fr, gk, li, window, wp);
            // the lane's tap along the last axis, with the value and the scale folded in
            const T ws = valid ? w[D - 1] * scale : (T)0;
            const T pr = st.vr[ks] * ws, pi = st.vi[ks] * ws;
            if constexpr (D == 1) {
                FP::add(acc + (l[0] + li), ptot, pr, pi);
            } else if constexpr (D == 2) {
                T w0[M2];
                row_weights_2d<GW, T, M2>(w0, w[0], gk, li, gbase, window, wp);
                unsigned long long *ap = acc + (l[0] * P[1] + l[1] + li);
                const int rs = P[1];
#pragma unroll
                for (int a = 0; a < M2; ++a) FP::add_prod(ap + a * rs, ptot, w0[a], pr, pi);
            } else {
                T w0[M2], w1[M2];
                BcastAll<M2, 0, T>::run(w0, w[0], gbase);
                BcastAll<M2, 0, T>::run(w1, w[1], gbase);
                unsigned long long *ap = acc + ((l[0] * P[1] + l[1]) * P[2] + l[2] + li);
                const int rs1 = P[2], rs0 = P[1] * P[2];
#pragma unroll
                for (int a = 0; a < M2; ++a) {
                    const T ar = w0[a] * pr, ai = w0[a] * pi;
                    unsigned long long *rp = ap + a * rs0;
#pragma unroll
                    for (int b = 0; b < M2; ++b) FP::add_prod(rp + b * rs1, ptot, w1[b], ar, ai);
                }
            }
        }
        __syncthreads();
    }

    // the padded tile goes to the item's scratch slot, unscaled (NaN for a non-finite item)
    const T inv = (T)(1.0 / (double)scale);
    const T nan = (T)__builtin_nan("");
    C *out = pad + (size_t)item * ptot;
    for (int idx = threadIdx.x; idx < ptot; idx += NT) {
        const unsigned long long *ap = acc + idx;
        out[idx] = poisoned ? cmake<C>(nan, nan)
                            : cmake<C>((T)FP::read(ap, ptot, 0) * inv, (T)FP::read(ap, ptot, 1) * inv);
    }
}

template <typename T, int D, int M2, bool GW, int NT = kResampleThreads>
__global__ void __launch_bounds__(NT)
    k_spread(cplx<T> *__restrict__ pad, Geom g, const NodeRec<T, D> *__restrict__ nodes,
             const int *__restrict__ perm, const int4 *__restrict__ subs,
             const T *__restrict__ coef, int window, WinParams<T> wp, T wmax_prod,
             const cplx<T> *__restrict__ fhat, long long pstride, long long fstride) {
    spread_body<T, D, M2, GW, NT>(pad + blockIdx.y * pstride, g, nodes, perm, subs, coef, window, wp,
                                  wmax_prod, fhat + blockIdx.y * fstride, blockIdx.x);
}

// Halo merge: grid point l of tile p is the sum of the padded tiles that cover
// it -- those of the work items of p and, within 2m-1 of p's leading edge along
// a set e of axes, those of the tile preceding p along e (cyclically).  Each
// grid value is written once, by one thread, in a fixed order of summation.
// bx: the workgroup's block among the nbx (one per tile) of this grid's merge.
template <typename T, int D>
__device__ inline void spread_merge_body(cplx<T> *__restrict__ grid, const Geom &g,
                                         const cplx<T> *__restrict__ pad,
                                         const int *__restrict__ tile_sub, int M2, int bx, int nbx) {
    using C = cplx<T>;
    // consecutive tiles on one XCD: a tile's own rows and the halo rows its
    // neighbour reads share cache lines (3-D 128^3: merge 15-65 us faster)
    const int p = xcd_block(bx, nbx);
    int tc[D], P[D];
    int ptot = 1;
    {
        int rem = p;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            tc[d] = rem % g.T[d];
            rem /= g.T[d];
            P[d] = g.Q[d] + M2 - 1;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) ptot *= P[d];
    }
    // item ranges of the 2^D source tiles: e = set of axes along which the
    // source precedes this tile
    __shared__ int rng[2 << D];
    if (threadIdx.x < (1 << D)) {
        const int e = threadIdx.x;
        int q = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            int qd = tc[d] - ((e >> d) & 1);
            if (qd < 0) qd += g.T[d];
            q = q * g.T[d] + qd;
        }
        rng[2 * e] = tile_sub[q];
        rng[2 * e + 1] = tile_sub[q + 1];
    }
    __syncthreads();
    int qtot = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) qtot *= g.Q[d];
    const float rl = 1.0f / (float)g.Q[D - 1];
    const float r1 = D == 3 ? 1.0f / (float)g.Q[1] : 1.0f;
    constexpr int U = 2;  // cells per thread and batch (4: 151 VGPRs, 20 % slower in 3-D)
    constexpr int NE = 1 << D;
    for (int base = 0; base < qtot; base += U * kResampleThreads) {
        int a[U][D], off[U][NE];
        bool in[U][NE];
        // cell coordinates and, per source tile, the offset in its padded tile
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * kResampleThreads + threadIdx.x;
            int rest;
            const int row = small_divmod(idx < qtot ? idx : 0, g.Q[D - 1], rl, rest);
            a[u][D - 1] = rest;
            if constexpr (D == 2) a[u][0] = row;
            if constexpr (D == 3) a[u][0] = small_divmod(row, g.Q[1], r1, a[u][1]);
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                bool ok = idx < qtot && rng[2 * e + 1] > rng[2 * e];
                int o = 0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const int ed = (e >> d) & 1;
                    if (ed && a[u][d] >= M2 - 1) ok = false;
                    o = o * P[d] + a[u][d] + (ed ? g.Q[d] : 0);
                }
                in[u][e] = ok;
                off[u][e] = o;
            }
        }
        // first item of every source tile: all loads independent
        C v[U][NE];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < NE; ++e)
                v[u][e] = in[u][e] ? pad[(size_t)rng[2 * e] * ptot + off[u][e]]
                                            : cmake<C>((T)0, (T)0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * kResampleThreads + threadIdx.x;
            if (idx >= qtot) continue;
            T sr = (T)0, si = (T)0;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                sr += v[u][e].x;
                si += v[u][e].y;
                if (in[u][e])  // further items of a split tile
                    add_split_items(sr, si, pad, ptot, off[u][e], rng[2 * e] + 1, rng[2 * e + 1]);
            }
            long long gi = 0;
#pragma unroll
            for (int d = 0; d < D; ++d) gi = gi * g.Nt[d] + tc[d] * g.Q[d] + a[u][d];
            grid[gi] = cmake<C>(sr, si);
        }
    }
}

template <typename T, int D>
__global__ void __launch_bounds__(kResampleThreads)
    k_spread_merge(cplx<T> *__restrict__ grid, Geom g, const cplx<T> *__restrict__ pad,
                   const int *__restrict__ tile_sub, int M2, long long gstride, long long pstride) {
    spread_merge_body<T, D>(grid + blockIdx.y * gstride, g, pad + blockIdx.y * pstride, tile_sub, M2,
                            blockIdx.x, gridDim.x);
}

// Static LDS of the interpolation kernel (its staged node chunk).
template <typename T, int D> constexpr size_t interp_static_lds_t() {
    static_assert(sizeof(Stage<T, D, interp_chunk(D, (int)sizeof(T))>) <=
                      interp_static_lds(D, (int)sizeof(T)),
                  "staged chunk larger than the LDS the plan reserves for it");
    return interp_static_lds(D, (int)sizeof(T));
}

// Static LDS of the resampling kernels (staged node chunk and the scale).
template <typename T, int D> constexpr size_t static_lds() {
    static_assert(sizeof(Stage<T, D>) <= stage_bytes(D, (int)sizeof(T)),
                  "staged chunk larger than the LDS the plan reserves for it");
    return resample_static_lds(D, (int)sizeof(T));
}

// Dynamic LDS beyond 64 KiB (static included) has to be allowed per kernel.
template <typename K> inline hipError_t allow_lds(K kernel, size_t dyn, size_t stat) {
    if (dyn + stat <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
}

template <typename T> inline WinParams<T> win_params(const nfft_plan_s &p) {
    WinParams<T> wp;
    for (int d = 0; d < kMaxD; ++d) {
        wp.beta[d] = d < p.D ? (T)kb_beta(p, d) : (T)0;
        wp.inv_peak[d] = d < p.D ? (T)(1.0 / window_peak(p, d)) : (T)0;
    }
    wp.tab = (const T *)p.wtab;
    wp.S = p.lin_S;
    wp.m = p.m;
    return wp;
}

// Workgroup size of the tiled resampling kernels: 256 threads, 512 in 3-D,
// whose large LDS tiles (the fixed-point accumulators of a 15 x 23 x 23 padded
// tile take 127 KB in c64, a 15^3 one 108 KB in c128) leave room for one or two
// workgroups per CU -- twice the wavefronts then hide more of the load latency
// (measured on the 3-D 128^3 workload: c128 interpolation 1.02 -> 0.76 ms and
// spreading 3.11 -> 2.72 ms; c64 with 8 x 16 x 16 tiles 1.65 -> 1.43 ms per
// pair).  In 2-D, where four or more workgroups fit, 512 threads were slower.
template <typename T, int D> constexpr int resample_threads() {
    return D == 3 ? 512 : kResampleThreads;
}

template <typename T, int D, int M2>
hipError_t run_interp(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s, int K) {
    if (p.nsub == 0) return hipSuccess;
    constexpr int NT = resample_threads<T, D>();
    const size_t tile = padded_cells(p.geom, D) * sizeof(cplx<T>);
    const bool gw = p.window != NFFT_WINDOW_POLY;
    const int kb = interp_channel_block<T, D>(K, gw, tile);
    auto kern = gw ? k_interp<T, D, M2, true, false, NT, 1> : k_interp<T, D, M2, false, false, NT, 1>;
    if constexpr (D <= 2)
        if (kb == 2) kern = k_interp<T, D, M2, false, false, NT, 2>;
    const size_t shm = kb * tile;
    hipError_t e = allow_lds(kern, shm, interp_static_lds_t<T, D>());
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(p.nsub, (K + kb - 1) / kb), dim3(NT), shm, s,
                       (const cplx<T> *)grid, p.geom, (const NodeRec<T, D> *)p.nodes, p.perm,
                       p.subs, (const T *)p.coef, p.window, win_params<T>(p), (cplx<T> *)fhat,
                       (long long)p.G, (long long)p.M, K);
    return hipGetLastError();
}

// Derivative-of-window interpolation (polynomial window): dfhat is D x M complex.
template <typename T, int D, int M2>
hipError_t run_interp_deriv(const nfft_plan_s &p, const void *grid, void *dfhat, hipStream_t s) {
    if (p.nsub == 0) return hipSuccess;
    constexpr int NT = resample_threads<T, D>();
    const size_t shm = padded_cells(p.geom, D) * sizeof(cplx<T>);
    auto kern = k_interp<T, D, M2, false, true, NT>;
    hipError_t e = allow_lds(kern, shm, interp_static_lds_t<T, D>());
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(p.nsub, 1), dim3(NT), shm, s,
                       (const cplx<T> *)grid, p.geom, (const NodeRec<T, D> *)p.nodes, p.perm,
                       p.subs, (const T *)p.coef, p.window, win_params<T>(p), (cplx<T> *)dfhat,
                       (long long)p.G, (long long)p.M, 1);
    return hipGetLastError();
}

template <typename T, int D, int M2>
hipError_t run_spread(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s, bool merge,
                      int K, void *pad) {
    const long long pstride = (long long)p.nsub * (long long)padded_cells(p.geom, D);
    if (p.nsub > 0) {
        const size_t shm = padded_cells(p.geom, D) * 2 * FixedPoint<T>::kSlots *
                           sizeof(unsigned long long);
        const double wprod = window_bound(D);
        constexpr int NT = resample_threads<T, D>();
        const bool gw = p.window != NFFT_WINDOW_POLY;
        auto kern = gw ? k_spread<T, D, M2, true, NT> : k_spread<T, D, M2, false, NT>;
        hipError_t e = allow_lds(kern, shm, static_lds<T, D>());
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(p.nsub, K), dim3(NT), shm, s,
                           (cplx<T> *)pad, p.geom, (const NodeRec<T, D> *)p.nodes, p.perm,
                           p.subs, (const T *)p.coef, p.window, win_params<T>(p), (T)wprod,
                           (const cplx<T> *)fhat, pstride, (long long)p.M);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!merge) return hipSuccess;
    hipLaunchKernelGGL((k_spread_merge<T, D>), dim3(p.geom.ntiles, K), dim3(kResampleThreads), 0, s,
                       (cplx<T> *)grid, p.geom, (const cplx<T> *)pad, p.tile_sub, M2, (long long)p.G,
                       pstride);
    return hipGetLastError();
}

}  // namespace nfft
