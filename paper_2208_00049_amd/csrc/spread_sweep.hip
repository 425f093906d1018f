// Three-dimensional spreading by column sweeps (paper, step 1 of Algorithm 2;
// subsection "Block-Partitioned Adjoint Resampling").
//
// The oversampled grid is cut into columns of 16 x 16 points along axes 1 and
// 2 that run through axis 0, and each column into segments of consecutive
// tiles along axis 0.  One workgroup sweeps one segment tile by tile, in
// increasing axis-0 order.  It keeps a ring of R = Q_0 + 2m - 1 padded planes
// in LDS, each (16 + 2m - 1)^2 points: a node binned in tile t_0 adds its
// stencil to planes o_0 .. o_0 + 2m - 1, all of which are in the ring, and after
// the tile's nodes the tile's Q_0 planes receive nothing more from this segment.
// Those planes go to the scratch once (axis-1/2 halo included) and their ring
// slots are cleared for the next planes.  The axis-0 halo thus stays in LDS;
// only the segment's last 2m - 1 planes (which belong to the next segment) go
// to a small halo slot of their own.
//
// A merge then sums, for every grid point, the scratch planes of the columns
// that cover it (its own column and, within 2m - 1 of its leading edges along
// axes 1 and 2, the columns before it) and, within 2m - 1 planes of a segment
// start, the halo slots of the segments before.  Every grid value has one
// writer, in a fixed order of summation; no global atomics are used.  In the
// adjoint transform the merge is done by the first (axis-0) FFT pass as it
// loads its lines (fft.hip); the merge kernel here serves the single
// resampling step.
//
// Before the sweep, a reduction records per block of fhat the largest |Re|, |Im|,
// from which every sweep workgroup takes the transform's fixed-point scale.  The
// sweep reads node records as consecutive runs and their values through the sort's
// permutation, and loads the next chunk of nodes while it accumulates the current
// one (the permutation one chunk further ahead, so that no load waits for another).
//
// Accumulation in LDS: 64-bit fixed point per component (the tiled kernels'
// scheme, resample_impl.hpp) with a scale from the transform's largest |Re|, |Im|:
// exact, independent of the order of the additions, so the adjoint is bitwise
// reproducible.  complex64 adds truncated int32 contributions below 2^30;
// complex128 rounds contributions to integers, scaled for the most nodes that reach
// one grid plane of the segment (no grid point receives more contributions), where
// that count leaves the full 2^-51 resolution (at most kSweepFixedNodes).  A denser
// complex128 segment (a cluster) accumulates with FP64 LDS atomics instead in the
// same 8-byte words: correct to FP64 rounding, whose order -- and so the last bits
// of such a segment's sums -- can differ between calls.
#include <type_traits>

#include "resample_impl.hpp"

namespace nfft {

constexpr int kSweepFixedNodes = 2048;

// a: the point's Re word; the Im word is `im` words further; fixed: the segment's
// words are fixed-point sums (always in complex64), else FP64 sums
template <typename T> struct SweepAcc {
    using W = unsigned long long;
    // the contributions w * pr, w * pi
    __device__ static inline void add_prod(W *a, int im, T w, T pr, T pi, bool fixed) {
        if constexpr (sizeof(T) == 8) {
            if (!fixed) {
                atomicAdd(reinterpret_cast<double *>(a), (double)(w * pr));
                atomicAdd(reinterpret_cast<double *>(a + im), (double)(w * pi));
                return;
            }
        }
        FixedPoint<T>::add_prod(a, im, w, pr, pi);
    }
    __device__ static inline T get(const W *a, double inv, bool fixed) {
        if constexpr (sizeof(T) == 8)
            if (!fixed) return (T)__longlong_as_double((long long)*a);
        return (T)((double)(long long)*a * inv);
    }
};

// Staged nodes of one chunk: ring slot and in-column offsets packed into one
// word (slot | l1 << 8 | l2 << 16), the fractions and the value.
template <typename T, int CH> struct SweepStage {
    int pk[CH];
    T fr[3][CH];
    T vr[CH];
    T vi[CH];
};

// Value of lane `l` (uniform across the wavefront).
__device__ inline double lane_value(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float lane_value(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <typename T> constexpr int sweep_chunk() { return sizeof(T) == 4 ? 1024 : 512; }
template <typename T> constexpr int sweep_threads() { return 1024; }

// part[b] = the largest max(|Re|, |Im|) of fhat over block b's range of positions
// (+infinity if one is not finite).
template <typename T>
__global__ void __launch_bounds__(256)
    k_sweep_amax(const cplx<T> *__restrict__ fhat, int M, cplx<T> *__restrict__ scr,
                 long long part_off, long long fstride, long long sstride) {
    using C = cplx<T>;
    fhat += blockIdx.y * fstride;  // channel
    scr += blockIdx.y * sstride;
    double *part = reinterpret_cast<double *>(scr + part_off);
    __shared__ double wmax[4];
    const int per = (M + gridDim.x - 1) / gridDim.x;
    const int b0 = blockIdx.x * per, b1 = min(M, b0 + per);
    T mx = (T)0;
    for (int s0 = b0; s0 < b1; s0 += 4 * 256) {
        C v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * 256 + threadIdx.x;
            v[u] = fhat[s < b1 ? s : b0];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) mx = fmax(mx, scale_mag(v[u].x, v[u].y));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = (double)mx;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
}

template <typename T, int M2, bool GW>
__global__ void __launch_bounds__(sweep_threads<T>())
    k_spread_sweep(const cplx<T> *__restrict__ fhat, const int *__restrict__ perm,
                   cplx<T> *__restrict__ scr, Geom g, SweepGeom sg,
                   const NodeRec<T, 3> *__restrict__ nodes, const int *__restrict__ key_start,
                   const T *__restrict__ coef, int window, WinParams<T> wp, T wmax_prod,
                   long long fstride, long long sstride) {
    using C = cplx<T>;
    using A = SweepAcc<T>;
    using W = typename A::W;
    constexpr int NT = sweep_threads<T>();
    constexpr int CH = sweep_chunk<T>();
    constexpr int P = kSweepQ + M2 - 1, PP = P * P;
    constexpr int NPW = 64 / M2;
    constexpr bool WN = sweep_wave_node(M2, !GW);  // one node per wavefront
    constexpr int SP = sweep_plane_stride(M2, WN);                   // words per ring plane
    scr += blockIdx.y * sstride;              // channel
    fhat += blockIdx.y * fstride;
    const double *part = reinterpret_cast<const double *>(scr + sg.part_off);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    W *acc = reinterpret_cast<W *>(smem_raw);  // [R][Re, Im][PP]
    __shared__ SweepStage<T, CH> st;
    __shared__ int seg_beg[kSweepMaxSegTiles + 1];  // node range of each tile of the segment
    __shared__ int seg_end[kSweepMaxSegTiles + 1];
    __shared__ unsigned long long amax_bits;

    const int seg = blockIdx.x;
    const int col = seg / sg.nsc, kseg = seg - col * sg.nsc;
    const int t1 = col / g.T[2], t2 = col - t1 * g.T[2];
    const int tb = kseg * sg.L, nt = sg.L;  // segments are L tiles long (L divides T_0)
    const int R = sg.R, Q0 = g.Q[0];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // the most contributions a grid plane of the segment receives: a plane takes nodes
    // of at most W = 1 + ceil((taps - 1) / Q_0) consecutive tiles of the column
    __shared__ int seg_nodes;
    if (tid == 0) {
        amax_bits = 0ull;
        seg_nodes = 0;
    }
    if (tid < nt) {
        const int tile = ((tb + tid) * g.T[1] + t1) * g.T[2] + t2;
        seg_beg[tid] = key_start[tile << g.kbits];
        seg_end[tid] = key_start[(tile + 1) << g.kbits];
    }
    __syncthreads();
    if (tid < nt) {
        const int W = 1 + (M2 - 1 + Q0 - 1) / Q0;
        int sum = 0;
        for (int j = max(0, tid - W + 1); j <= tid; ++j) sum += seg_end[j] - seg_beg[j];
        atomicMax(&seg_nodes, sum);
    }
    // the transform's largest |Re|, |Im| from the gather's block maxima
    double pm = 0.0;
    for (int i = tid; i < kSweepParts; i += NT) pm = fmax(pm, part[i]);
    for (int i = tid; i < R * SP; i += NT) acc[i] = (W)0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) pm = fmax(pm, __shfl_xor(pm, off, 64));
    __syncthreads();
    if (lane == 0) atomicMax(&amax_bits, (unsigned long long)__double_as_longlong(pm));
    __syncthreads();
    const double amax_d = __longlong_as_double((long long)amax_bits);
    const bool poisoned = isinf(amax_d);  // a non-finite value in fhat
    const bool fixed = sizeof(T) == 4 || seg_nodes <= kSweepFixedNodes;
    const T scale = amax_d > 0.0 && !poisoned && fixed
                        ? FixedPoint<T>::scale(amax_d * (double)wmax_prod, seg_nodes) : (T)1;
    const double inv = 1.0 / (double)scale;

    const int grp = lane / M2, li = lane - grp * M2, gbase = grp * M2;
    LaneWindow<T, 3, M2> lw;
    if constexpr (WN) {
        // axis 0: tap grp (the lane's plane); axes 1 and 2: tap li
        const int Z = 2 * wp.m + 1;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int z = 0; z <= M2; ++z)
                lw.cf[d][z] = z < Z ? coef[((size_t)d * M2 + (d == 0 ? grp : li)) * Z + z] : (T)0;
    } else {
        lw.load(coef, li, wp.m);
    }
    // the coefficients in registers before any node load is issued (vmcnt(0)): otherwise
    // the compiler waits for every load in flight, the prefetch of the next chunk
    // included, at each pass through the node loop
    __builtin_amdgcn_s_waitcnt(0x0f70);
    const T nan = (T)__builtin_nan("");

    // the chunk after (t, c0): the rest of tile t, else the first chunk of the next
    // tile that has nodes (t = nt: none)
    auto next_chunk = [&](int &t, int &c0) {
        c0 += CH;
        if (c0 < seg_end[t]) return;
        for (++t; t < nt && seg_beg[t] == seg_end[t]; ++t) {
        }
        c0 = t < nt ? seg_beg[t] : 0;
    };
    // one node per staging thread in registers: all loads issued at once; the value
    // through the permutation entry loaded with the chunk before
    NodeRec<T, 3> rec;
    C val;
    int pmn = 0;  // permutation entry of the chunk after the one in registers
    auto load_perm = [&](int t, int c0) {
        const int n = min(CH, seg_end[t] - c0);
        pmn = perm[c0 + (tid < n ? tid : n - 1)];
    };
    auto load_chunk = [&](int t, int c0) {
        const int n = min(CH, seg_end[t] - c0);
        rec = nodes[c0 + (tid < n ? tid : n - 1)];
        val = fhat[pmn];
    };
    int ct = -1, cc0 = 0;  // the chunk held in registers
    int bt = -1, bc0 = 0;  // the chunk after it
    {
        int t = 0;
        for (; t < nt && seg_beg[t] == seg_end[t]; ++t) {
        }
        if (t < nt && !poisoned) {
            ct = t;
            cc0 = seg_beg[t];
            load_perm(ct, cc0);
            load_chunk(ct, cc0);
            bt = ct;
            bc0 = cc0;
            next_chunk(bt, bc0);
            if (bt < nt) load_perm(bt, bc0);
        }
    }

    for (int t = 0; t < nt; ++t) {
        while (ct == t) {
            const int c0 = cc0, n = min(CH, seg_end[t] - c0);
            if (tid < n) {
                st.pk[tid] = (rec.o[0] % R) | ((rec.o[1] - t1 * kSweepQ) << 8) |
                             ((rec.o[2] - t2 * kSweepQ) << 16);
#pragma unroll
                for (int d = 0; d < 3; ++d) st.fr[d][tid] = rec.fr[d];
                st.vr[tid] = val.x;
                st.vi[tid] = val.y;
            }
            __syncthreads();
            // the next chunk's loads overlap the accumulation of this one
            ct = bt;
            cc0 = bc0;
            if (ct < nt) {
                load_chunk(ct, cc0);
                next_chunk(bt, bc0);
                if (bt < nt) load_perm(bt, bc0);
            } else {
                ct = -1;
            }
            // the accumulation, with the segment's kind of sum fixed at compile time
            auto accumulate = [&](auto fixed_tag) {
                constexpr bool kFixed = decltype(fixed_tag)::value;
                if constexpr (WN) {
                    // one node per wavefront: lane (grp, li) adds the taps (grp, b, li), b = 0..7.
                    // The next node's staged fields are read before this node's atomics are
                    // issued: LDS operations of a wavefront complete in order, so read after
                    // them they would wait for all of its atomics to drain.
                    constexpr int NW = NT / 64;
                    int pk_n = 0;
                    T z0_n = (T)0, z1_n = (T)0, z2_n = (T)0, vr_n = (T)0, vi_n = (T)0;
                    auto fetch = [&](int k) {
                        pk_n = st.pk[k];
                        z0_n = st.fr[0][k];
                        z1_n = st.fr[1][k];
                        z2_n = st.fr[2][k];
                        vr_n = st.vr[k];
                        vi_n = st.vi[k];
                    };
                    if (wave < n) fetch(wave);
                    // wait for the first reads here (lgkmcnt(0)): a read still in flight at
                    // the loop entry would make every iteration wait for its atomics
                    __builtin_amdgcn_s_waitcnt(0xc07f);
                    for (int k = wave; k < n; k += NW) {
                        const int pk = pk_n;
                        const T z0 = z0_n - (T)0.5, z1 = z1_n - (T)0.5, z2 = z2_n - (T)0.5;
                        const T vr = vr_n, vi = vi_n;
                        fetch(min(k + NW, n - 1));  // (the last node re-reads itself)
                        __builtin_amdgcn_sched_barrier(0);  // the reads stay ahead of the atomics
                        const int r0 = pk & 0xff, l1 = (pk >> 8) & 0xff, l2 = pk >> 16;
                        T h0 = lw.cf[0][M2], h1 = lw.cf[1][M2], h2 = lw.cf[2][M2];
    #pragma unroll
                        for (int z = M2 - 1; z >= 0; --z) {
                            h0 = fma(h0, z0, lw.cf[0][z]);
                            h1 = fma(h1, z1, lw.cf[1][z]);
                            h2 = fma(h2, z2, lw.cf[2][z]);
                        }
                        // the products in the order of the other mapping (bit-identical terms)
                        const T ws = h2 * scale;
                        const T pr = vr * ws, pi = vi * ws;
                        const T ar = h0 * pr, ai = h0 * pi;
                        int r = r0 + grp;
                        if (r >= R) r -= R;
                        W *pl = acc + r * SP + (l1 * P + l2 + li);
    #pragma unroll
                        for (int b = 0; b < M2; ++b) {
                            const T wb = lane_value(h1, b);  // lane b holds axis-1 tap b
                            A::add_prod(pl + b * P, PP, wb, ar, ai, kFixed);
                        }
                    }
                } else {
                for (int base = wave * NPW; base < n; base += (NT / 64) * NPW) {
                    const int k = base + grp;
                    const bool valid = grp < NPW && k < n;
                    const int ks = valid ? k : 0;
                    const int pk = st.pk[ks];
                    const int r0 = pk & 0xff, l1 = (pk >> 8) & 0xff, l2 = pk >> 16;
                    T fr[3], w[3];
    #pragma unroll
                    for (int d = 0; d < 3; ++d) fr[d] = st.fr[d][ks];
                    node_weights<GW, T, 3, M2>(w, lw, fr, (long long)(c0 + ks), li, window, wp);
                    const T ws = valid ? w[2] * scale : (T)0;
                    const T pr = st.vr[ks] * ws, pi = st.vi[ks] * ws;
                    T w0[M2], w1[M2];
                    BcastAll<M2, 0, T>::run(w0, w[0], gbase);
                    BcastAll<M2, 0, T>::run(w1, w[1], gbase);
                    W *cell = acc + (l1 * P + l2 + li);
    #pragma unroll
                    for (int a = 0; a < M2; ++a) {
                        int r = r0 + a;
                        if (r >= R) r -= R;
                        W *pl = cell + r * SP;
                        const T ar = w0[a] * pr, ai = w0[a] * pi;
    #pragma unroll
                        for (int b = 0; b < M2; ++b) A::add_prod(pl + b * P, PP, w1[b], ar, ai, kFixed);
                    }
                }
                }
            };
            if (sizeof(T) == 4 || fixed) accumulate(std::true_type{});
            else if constexpr (sizeof(T) == 8) accumulate(std::false_type{});
            __syncthreads();
        }
        // the tile's Q_0 planes are complete: write them out, clear their slots
        const int p0 = (tb + t) * Q0;
        const int rb = p0 % R;
        for (int idx = tid; idx < Q0 * PP; idx += NT) {
            const int kk = idx / PP, cell = idx - kk * PP;
            int r = rb + kk;
            if (r >= R) r -= R;
            W *a = acc + r * SP + cell;
            const C v = poisoned ? cmake<C>(nan, nan) : cmake<C>(A::get(a, inv, fixed), A::get(a + PP, inv, fixed));
            a[0] = (W)0;
            a[PP] = (W)0;
            scr[((size_t)(p0 + kk) * sg.ncols + col) * PP + cell] = v;
        }
        __syncthreads();
    }
    // the last 2m - 1 planes (the next segment's first ones) go to the halo slot
    const int ph = (tb + nt) * Q0;
    const int rh = ph % R;
    C *halo = scr + sg.main_cells + (size_t)seg * (M2 - 1) * PP;
    for (int idx = tid; idx < (M2 - 1) * PP; idx += NT) {
        const int kk = idx / PP, cell = idx - kk * PP;
        int r = rh + kk;
        if (r >= R) r -= R;
        const W *a = acc + r * SP + cell;
        halo[idx] = poisoned ? cmake<C>(nan, nan) : cmake<C>(A::get(a, inv, fixed), A::get(a + PP, inv, fixed));
    }
}

// Merge of the column sweeps: one workgroup per (plane, column), one thread per
// grid point of the column's 16 x 16 cross-section.
template <typename T, int M2>
__global__ void __launch_bounds__(256)
    k_sweep_merge(cplx<T> *__restrict__ grid, Geom g, SweepGeom sg, const cplx<T> *__restrict__ scr,
                  long long gstride, long long sstride) {
    using C = cplx<T>;
    constexpr int P = kSweepQ + M2 - 1, PP = P * P;
    grid += blockIdx.y * gstride;  // channel
    scr += blockIdx.y * sstride;
    // neighbouring columns on one XCD: they read each other's halo rows
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int p = b / sg.ncols, col = b - p * sg.ncols;
    const int t1 = col / g.T[2], t2 = col - t1 * g.T[2];
    const int a1 = threadIdx.x >> 4, a2 = threadIdx.x & 15;
    const int t0 = p / g.Q[0];
    const int kseg = t0 / sg.L;
    const int j = p - kseg * sg.L * g.Q[0];  // plane within its segment
    const int kpred = kseg == 0 ? sg.nsc - 1 : kseg - 1;
    const C *halo = scr + sg.main_cells;
    // the four column planes, then the four halo planes (the order of the fused pass)
    int cc[4], off[4];
    bool ok[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int e1 = e >> 1, e2 = e & 1;  // the source column precedes along axis 1 / 2
        ok[e] = !((e1 && a1 >= M2 - 1) || (e2 && a2 >= M2 - 1));
        int c1 = t1 - e1, c2 = t2 - e2;
        if (c1 < 0) c1 += g.T[1];
        if (c2 < 0) c2 += g.T[2];
        cc[e] = c1 * g.T[2] + c2;
        off[e] = (a1 + (e1 ? kSweepQ : 0)) * P + a2 + (e2 ? kSweepQ : 0);
    }
    T sr = (T)0, si = (T)0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const C v = ok[e] ? scr[((size_t)p * sg.ncols + cc[e]) * PP + off[e]] : cmake<C>((T)0, (T)0);
        sr += v.x;
        si += v.y;
    }
    if (j < M2 - 1) {
        T hr = (T)0, hi = (T)0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const C h = ok[e] ? halo[((size_t)(cc[e] * sg.nsc + kpred) * (M2 - 1) + j) * PP + off[e]]
                              : cmake<C>((T)0, (T)0);
            hr += h.x;
            hi += h.y;
        }
        sr += hr;
        si += hi;
    }
    const long long gi = ((long long)p * g.Nt[1] + t1 * kSweepQ + a1) * g.Nt[2] + t2 * kSweepQ + a2;
    grid[gi] = cmake<C>(sr, si);
}

// ---- interpolation by column sweeps (step 3 of Algorithm 1) --------------------
//
// Used for complex128 plans that spread by column sweeps (3-D 128^3: 0.66 ms
// against 0.71 ms for the tiled kernel, which reloads every tile's halo; for
// complex64 the tiled kernel, two workgroups per compute unit, is faster: 0.26
// against 0.33 ms).  The same columns, segments and tiles as spreading.  The workgroup of a segment
// keeps the grid planes its tile's nodes read -- planes t_0 Q_0 .. t_0 Q_0 + Q_0 +
// 2m - 2 of the column's padded cross-section, (16 + 2m - 1)^2 values each, wrapped
// at the grid's edges -- in a ring in LDS.  While it interpolates tile t_0, the Q_0
// planes tile t_0 + 1 adds are loaded into registers; afterwards they replace the
// tile's first Q_0 planes.  Every grid plane of a segment is read from memory once,
// with its axis-1/2 halo, and the loads overlap the interpolation.

// 512 threads: the complex128 tap loop needs more than the 128 registers a
// 1024-thread workgroup leaves a thread (complex64, whose tiled kernel is faster
// and which therefore does not use the sweep, measured 0.33 ms at 512 and 0.36 ms
// at 1024 threads on the 3-D 128^3 workload).
template <typename T> constexpr int interp_sweep_threads() { return 512; }
template <typename T> constexpr int interp_sweep_chunk() { return interp_sweep_threads<T>(); }

// Whether the tap loop double-buffers its LDS reads: where the second buffer's
// registers are free (the configurations that would otherwise spill keep one buffer).
template <typename T, int M2, bool GW, bool ISO>
constexpr bool kInterpPipe = sizeof(T) == 4 ? M2 <= 8 : ISO ? M2 <= 8 : GW ? M2 <= 4 : M2 <= 6;

template <typename T, int CH> struct InterpStage {
    int pk[CH];
    T fr[3][CH];
    int idx[CH];  // caller's node index
};

// ISO: every axis has the same window (the same shape parameter), so a lane keeps one
// axis's tap coefficients instead of three (complex128: 221 instead of 255 VGPRs, the
// most two waves per SIMD allow).  The next tile's prefetched planes are held as arrays
// of reals: as an array of complex values the compiler placed them in scratch memory
// (0.6 GB of writes per call on the 3-D 128^3 workload).
template <typename T, int M2, bool GW, bool ISO>
__global__ void __launch_bounds__(interp_sweep_threads<T>())
    k_interp_sweep(const cplx<T> *__restrict__ grid, Geom g, SweepGeom sg,
                   const NodeRec<T, 3> *__restrict__ nodes, const int *__restrict__ perm,
                   const int *__restrict__ key_start, const T *__restrict__ coef, int window,
                   WinParams<T> wp, cplx<T> *__restrict__ fhat, long long gstride, long long fstride) {
    using C = cplx<T>;
    constexpr int NT = interp_sweep_threads<T>();
    constexpr int CH = interp_sweep_chunk<T>();
    constexpr int P = kSweepQ + M2 - 1, PP = P * P;
    constexpr int NPW = 64 / M2;
    constexpr int PF = (8 * PP + NT - 1) / NT;  // prefetched values per thread (Q_0 <= 8)
    grid += blockIdx.y * gstride;              // channel
    fhat += blockIdx.y * fstride;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *ring = reinterpret_cast<C *>(smem_raw);  // [R][PP]
    __shared__ InterpStage<T, CH> st;
    __shared__ int seg_beg[kSweepMaxSegTiles + 1];
    __shared__ int seg_end[kSweepMaxSegTiles + 1];

    const int seg = blockIdx.x;
    const int col = seg / sg.nsc, kseg = seg - col * sg.nsc;
    const int t1 = col / g.T[2], t2 = col - t1 * g.T[2];
    const int tb = kseg * sg.L, nt = sg.L;
    const int R = sg.R, Q0 = g.Q[0];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int N0 = g.Nt[0], N1 = g.Nt[1], N2 = g.Nt[2];

    // grid offset of point q of the padded cross-section in plane p (unwrapped)
    auto src = [&](int p, int q) -> long long {
        const int i = q / P, j = q - i * P;
        int pp = p >= N0 ? p - N0 : p;
        int r1 = t1 * kSweepQ + i, r2 = t2 * kSweepQ + j;
        if (r1 >= N1) r1 -= N1;
        if (r2 >= N2) r2 -= N2;
        return ((long long)pp * N1 + r1) * N2 + r2;
    };

    if (tid < nt) {
        const int tile = ((tb + tid) * g.T[1] + t1) * g.T[2] + t2;
        seg_beg[tid] = key_start[tile << g.kbits];
        seg_end[tid] = key_start[(tile + 1) << g.kbits];
    }
    // the first R planes, eight loads per thread in flight
    {
        const int p0 = tb * Q0;
        const int total = R * PP;
        for (int base = 0; base < total; base += 8 * NT) {
            C v[8];
            int dst[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * NT + tid;
                const int ic = idx < total ? idx : 0;
                const int kk = ic / PP, q = ic - kk * PP;
                v[u] = grid[src(p0 + kk, q)];
                dst[u] = idx < total ? ((p0 + kk) % R) * PP + q : -1;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (dst[u] >= 0) ring[dst[u]] = v[u];
        }
    }
    __syncthreads();

    const int grp = lane / M2, li = lane - grp * M2, gbase = grp * M2;
    LaneWindow<T, ISO ? 1 : 3, M2> lw;
    lw.load(coef, li, wp.m);
    // (in registers before the node and plane loads are issued, as in spreading)
    __builtin_amdgcn_s_waitcnt(0x0f70);

    auto next_chunk = [&](int &t, int &c0) {
        c0 += CH;
        if (c0 < seg_end[t]) return;
        for (++t; t < nt && seg_beg[t] == seg_end[t]; ++t) {
        }
        c0 = t < nt ? seg_beg[t] : 0;
    };
    NodeRec<T, 3> rec;
    int pm = 0;
    auto load_chunk = [&](int t, int c0) {
        const int n = min(CH, seg_end[t] - c0);
        const int k = c0 + (tid < n ? tid : n - 1);
        rec = nodes[k];
        pm = perm[k];
    };
    int ct = -1, cc0 = 0;
    {
        int t = 0;
        for (; t < nt && seg_beg[t] == seg_end[t]; ++t) {
        }
        if (t < nt) {
            ct = t;
            cc0 = seg_beg[t];
            load_chunk(ct, cc0);
        }
    }

    for (int t = 0; t < nt; ++t) {
        // the planes the next tile adds, into registers
        const int pn = (tb + t) * Q0 + R;
        const bool more = t + 1 < nt;
        T pre_x[PF], pre_y[PF];  // (real and imaginary parts: kept in registers)
        // The first chunk is staged before the planes are requested: loads complete in
        // order, so a staging that waits for its chunk's loads would otherwise wait for
        // the planes too.
        auto stage = [&](int c0, int n) {
            if (tid < n) {
                st.pk[tid] = (rec.o[0] % R) | ((rec.o[1] - t1 * kSweepQ) << 8) |
                             ((rec.o[2] - t2 * kSweepQ) << 16);
#pragma unroll
                for (int d = 0; d < 3; ++d) st.fr[d][tid] = rec.fr[d];
                st.idx[tid] = pm;
            }
            __syncthreads();
        };
        auto run = [&](int c0, int n) {
            next_chunk(ct, cc0);
            if (ct < nt) load_chunk(ct, cc0);
            else ct = -1;
            // Groups 4p .. 4p + 3 of a wavefront share an LDS pass over their 16-byte
            // reads (32 lanes, a 512-byte row of banks); complex128 plans order a tile's
            // nodes so that four consecutive ones have bank slots 8 apart (mod 32), and
            // their rows of eight values then fall on disjoint banks.
            for (int base = wave * NPW; base < n; base += (NT / 64) * NPW) {
                const int v = base + grp;
                const int k = v;
                const bool valid = grp < NPW && v < n;
                const int ks = valid ? k : 0;
                const int pk = st.pk[ks];
                const int r0 = pk & 0xff, l1 = (pk >> 8) & 0xff, l2 = pk >> 16;
                T fr[3], w[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) fr[d] = st.fr[d][ks];
                if constexpr (ISO) {
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        w[d] = tap_weight<T, M2>(lw.cf[0], fr[d], li, NFFT_WINDOW_POLY, wp.beta[d],
                                                 wp.inv_peak[d], nullptr, 0, wp.m);
                } else {
                    node_weights<GW, T, 3, M2>(w, lw, fr, (long long)(c0 + ks), li, window, wp);
                }
                T w0[M2], w1[M2];
                BcastAll<M2, 0, T>::run(w0, w[0], gbase);
                BcastAll<M2, 0, T>::run(w1, w[1], gbase);
                // the offsets of the node's M2 ring planes first, so that the tap loop's
                // reads need no address arithmetic between them
                const int cell = l1 * P + l2 + li;
                int po[M2];
#pragma unroll
                for (int a = 0; a < M2; ++a) {
                    const int r = r0 + a;
                    po[a] = (r >= R ? r - R : r) * PP + cell;
                }
                T ar = (T)0, ai = (T)0;
                if constexpr (kInterpPipe<T, M2, GW, ISO>) {
                    // plane a + 1's rows are read while plane a's are summed (two buffers),
                    // so the LDS latency is not exposed once per plane
                    C v[2][M2];
#pragma unroll
                    for (int b = 0; b < M2; ++b) v[0][b] = ring[po[0] + b * P];
#pragma unroll
                    for (int a = 0; a < M2; ++a) {
                        if (a + 1 < M2) {
#pragma unroll
                            for (int b = 0; b < M2; ++b) v[(a + 1) & 1][b] = ring[po[a + 1] + b * P];
                        }
                        __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the sums
                        T sr = (T)0, si = (T)0;
#pragma unroll
                        for (int b = 0; b < M2; ++b) {
                            sr = fma(w1[b], v[a & 1][b].x, sr);
                            si = fma(w1[b], v[a & 1][b].y, si);
                        }
                        ar = fma(w0[a], sr, ar);
                        ai = fma(w0[a], si, ai);
                    }
                } else {
#pragma unroll
                    for (int a = 0; a < M2; ++a) {
                        C v[M2];
#pragma unroll
                        for (int b = 0; b < M2; ++b) v[b] = ring[po[a] + b * P];
                        T sr = (T)0, si = (T)0;
#pragma unroll
                        for (int b = 0; b < M2; ++b) {
                            sr = fma(w1[b], v[b].x, sr);
                            si = fma(w1[b], v[b].y, si);
                        }
                        ar = fma(w0[a], sr, ar);
                        ai = fma(w0[a], si, ai);
                    }
                }
                ar *= w[2];
                ai *= w[2];
                ar = group_sum<M2>(ar, li);
                ai = group_sum<M2>(ai, li);
                if (valid && li == 0) fhat[st.idx[ks]] = cmake<C>(ar, ai);
            }
            __syncthreads();
        };
        const bool have = ct == t;
        int c0 = cc0, n = have ? min(CH, seg_end[t] - c0) : 0;
        if (have) stage(c0, n);
        if (more) {
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int idx = u * NT + tid;
                const int ic = idx < Q0 * PP ? idx : 0;
                const int kk = ic / PP, q = ic - kk * PP;
                const C v = grid[src(pn + kk, q)];
                pre_x[u] = v.x;
                pre_y[u] = v.y;
            }
        }
        if (have) {
            run(c0, n);
            while (ct == t) {
                c0 = cc0;
                n = min(CH, seg_end[t] - c0);
                stage(c0, n);
                run(c0, n);
            }
        }
        if (more) {
            // the tile's first Q_0 planes are no longer needed: the next tile's take their slots
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int idx = u * NT + tid;
                if (idx < Q0 * PP) {
                    const int kk = idx / PP, q = idx - kk * PP;
                    ring[((pn + kk) % R) * PP + q] = cmake<C>(pre_x[u], pre_y[u]);
                }
            }
            __syncthreads();
        }
    }
}

template <typename T, int M2>
hipError_t run_interp_sweep(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s,
                            int K) {
    const SweepGeom &sg = p.sweep;
    const size_t shm = (size_t)sg.R * sweep_plane_cells(p.geom.taps) * sizeof(cplx<T>);
    const bool gw = p.window != NFFT_WINDOW_POLY;
    const bool iso = !gw && kb_beta(p, 1) == kb_beta(p, 0) && kb_beta(p, 2) == kb_beta(p, 0);
    auto kern = gw ? k_interp_sweep<T, M2, true, false>
                   : iso ? k_interp_sweep<T, M2, false, true> : k_interp_sweep<T, M2, false, false>;
    hipError_t e = allow_lds(kern, shm, sizeof(InterpStage<T, interp_sweep_chunk<T>()>) + 1024);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(sg.ncols * sg.nsc, K), dim3(interp_sweep_threads<T>()), shm, s,
                       (const cplx<T> *)grid,
                       p.geom, sg, (const NodeRec<T, 3> *)p.nodes, p.perm, p.key_start,
                       (const T *)p.coef, p.window, win_params<T>(p), (cplx<T> *)fhat,
                       (long long)p.G, (long long)p.M);
    return hipGetLastError();
}

template <typename T, int M2>
hipError_t run_spread_sweep(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s,
                            int K, void *pad, bool merge) {
    const long long sstride = (long long)sweep_scratch_cells(p);
    const SweepGeom &sg = p.sweep;
    if (p.M == 0) return launch_fill_zero_complex(grid, (int64_t)K * p.G, sizeof(T) == 8, s);
    hipLaunchKernelGGL(k_sweep_amax<T>, dim3(kSweepParts, K), dim3(256), 0, s,
                       (const cplx<T> *)fhat, (int)p.M, (cplx<T> *)pad, sg.part_off,
                       (long long)p.M, sstride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t shm = sweep_ring_bytes(p);
    const bool gw = p.window != NFFT_WINDOW_POLY;
    auto kern = gw ? k_spread_sweep<T, M2, true> : k_spread_sweep<T, M2, false>;
    e = allow_lds(kern, shm, sizeof(SweepStage<T, sweep_chunk<T>()>) + 1024);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(sg.ncols * sg.nsc, K), dim3(sweep_threads<T>()), shm, s,
                       (const cplx<T> *)fhat, p.perm, (cplx<T> *)pad, p.geom, sg,
                       (const NodeRec<T, 3> *)p.nodes, p.key_start, (const T *)p.coef, p.window,
                       win_params<T>(p), (T)window_bound(3), (long long)p.M, sstride);
    e = hipGetLastError();
    if (e != hipSuccess || !merge) return e;
    hipLaunchKernelGGL((k_sweep_merge<T, M2>), dim3(p.geom.Nt[0] * sg.ncols, K), dim3(256), 0, s,
                       (cplx<T> *)grid, p.geom, sg, (const cplx<T> *)pad, (long long)p.G, sstride);
    return hipGetLastError();
}

template <typename T>
static hipError_t sweep_t(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s, int K,
                          void *pad, bool merge) {
    switch (p.geom.taps) {
        case 2: return run_spread_sweep<T, 2>(p, fhat, grid, s, K, pad, merge);
        case 4: return run_spread_sweep<T, 4>(p, fhat, grid, s, K, pad, merge);
        case 6: return run_spread_sweep<T, 6>(p, fhat, grid, s, K, pad, merge);
        case 8: return run_spread_sweep<T, 8>(p, fhat, grid, s, K, pad, merge);
        case 10: return run_spread_sweep<T, 10>(p, fhat, grid, s, K, pad, merge);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spread_sweep(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s,
                               int K, void *pad, bool merge) {
    return p.dtype == NFFT_C64 ? sweep_t<float>(p, fhat, grid, s, K, pad, merge)
                               : sweep_t<double>(p, fhat, grid, s, K, pad, merge);
}

template <typename T>
static hipError_t interp_sweep_t(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s,
                                 int K) {
    switch (p.geom.taps) {
        case 2: return run_interp_sweep<T, 2>(p, grid, fhat, s, K);
        case 4: return run_interp_sweep<T, 4>(p, grid, fhat, s, K);
        case 6: return run_interp_sweep<T, 6>(p, grid, fhat, s, K);
        case 8: return run_interp_sweep<T, 8>(p, grid, fhat, s, K);
        case 10: return run_interp_sweep<T, 10>(p, grid, fhat, s, K);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_interp_sweep(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s,
                               int K) {
    if (p.M == 0) return hipSuccess;
    return p.dtype == NFFT_C64 ? interp_sweep_t<float>(p, grid, fhat, s, K)
                               : interp_sweep_t<double>(p, grid, fhat, s, K);
}

size_t sweep_static_lds(int dtype) {
    return dtype == NFFT_C64 ? sizeof(SweepStage<float, sweep_chunk<float>()>) + 1024
                             : sizeof(SweepStage<double, sweep_chunk<double>()>) + 1024;
}

size_t interp_sweep_lds(int dtype, int R, int taps) {
    const size_t ring = (size_t)R * sweep_plane_cells(taps) * (dtype == NFFT_C64 ? 8 : 16);
    return ring + (dtype == NFFT_C64 ? sizeof(InterpStage<float, interp_sweep_chunk<float>()>)
                                     : sizeof(InterpStage<double, interp_sweep_chunk<double>()>)) +
           1024;
}

}  // namespace nfft
