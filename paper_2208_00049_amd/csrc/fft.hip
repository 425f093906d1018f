// Oversampled FFT (paper, step 2 of Algorithms 1 and 2): unnormalised mixed-radix
// Stockham FFT, one axis per pass, each line resident in LDS.
//
// Radix-R Stockham pass over a line of length L (p = product of the radices of
// the previous passes): butterfly i (0 <= i < L/R), k = i mod p, reads
// x_r = line[i + r L/R], multiplies x_r by W^(r k L/(p R)) (W = exp(-+2 pi i/L)),
// applies a length-R DFT and writes y_r to line[(i - k) R + k + r p].  After
// the last pass the line holds the DFT in natural order.
//
// Zero-pad pruning: in the forward transform only the rows of I_N (stored at
// n mod Nt) are non-zero before an axis is transformed, so those passes load
// only that band; in the adjoint only the band is needed after an axis is
// transformed, so those passes store only the band.  The first forward pass
// (last axis) reads f directly and applies the resampling correction and the
// index shift; the last adjoint pass crops, corrects and writes y.
#include "common.hpp"
#include "nfft_internal.hpp"

namespace nfft {


// Copy the twiddle table (L values) into LDS: every thread issues its loads,
// up to eight at a time, before it writes any of them.
template <typename C>
__device__ inline void copy_table(C *dst, const C *__restrict__ src, int L, int tid, int nthr) {
    constexpr int U = 8;
    for (int base = 0; base < L; base += U * nthr) {
        C v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * nthr + tid;
            v[u] = src[j < L ? j : 0];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * nthr + tid;
            if (j < L) dst[j] = v[u];
        }
    }
}

template <typename C, int R> struct Dft;

template <typename C> struct Dft<C, 2> {
    __device__ static inline void run(C *x, int) {
        const C a = x[0];
        x[0] = cadd(a, x[1]);
        x[1] = csub(a, x[1]);
    }
};

template <typename C> struct Dft<C, 4> {
    // y_k = sum_n x_n w^{nk}, w = s i
    __device__ static inline void run(C *x, int s) {
        const C a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
        const C c = cadd(x[1], x[3]), d = cmul_si(csub(x[1], x[3]), s);
        x[0] = cadd(a, c);
        x[2] = csub(a, c);
        x[1] = cadd(b, d);
        x[3] = csub(b, d);
    }
};

template <typename C> struct Dft<C, 8> {
    // split into even and odd halves, two length-4 DFTs, combine with w8^k
    __device__ static inline void run(C *x, int s) {
        using T = decltype(C::x);
        const T r2 = (T)0.70710678118654752440;
        C e[4] = {x[0], x[2], x[4], x[6]};
        C o[4] = {x[1], x[3], x[5], x[7]};
        Dft<C, 4>::run(e, s);
        Dft<C, 4>::run(o, s);
        const C o1 = cscale(cadd(o[1], cmul_si(o[1], s)), r2);
        const C o2 = cmul_si(o[2], s);
        const C o3 = cscale(csub(cmul_si(o[3], s), o[3]), r2);
        x[0] = cadd(e[0], o[0]);
        x[4] = csub(e[0], o[0]);
        x[1] = cadd(e[1], o1);
        x[5] = csub(e[1], o1);
        x[2] = cadd(e[2], o2);
        x[6] = csub(e[2], o2);
        x[3] = cadd(e[3], o3);
        x[7] = csub(e[3], o3);
    }
};

template <typename C> struct Dft<C, 3> {
    // w = -1/2 + s i sqrt(3)/2
    __device__ static inline void run(C *x, int s) {
        using T = decltype(C::x);
        const T h = (T)0.86602540378443864676;
        const C t1 = cadd(x[1], x[2]);
        const C t2 = cscale(cmul_si(csub(x[1], x[2]), s), h);
        const C base = csub(x[0], cscale(t1, (T)0.5));
        x[0] = cadd(x[0], t1);
        x[1] = cadd(base, t2);
        x[2] = csub(base, t2);
    }
};

template <typename C> struct Dft<C, 5> {
    // w^k = cos(2 pi k/5) + s i sin(2 pi k/5)
    __device__ static inline void run(C *x, int s) {
        using T = decltype(C::x);
        const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
        const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
        const C a1 = cadd(x[1], x[4]), a2 = cadd(x[2], x[3]);
        const C b1 = csub(x[1], x[4]), b2 = csub(x[2], x[3]);
        const C x0 = x[0];
        const C p1 = cadd(x0, cadd(cscale(a1, c1), cscale(a2, c2)));
        const C p2 = cadd(x0, cadd(cscale(a1, c2), cscale(a2, c1)));
        const C q1 = cmul_si(cadd(cscale(b1, s1), cscale(b2, s2)), s);
        const C q2 = cmul_si(csub(cscale(b1, s2), cscale(b2, s1)), s);
        x[0] = cadd(x0, cadd(a1, a2));
        x[1] = cadd(p1, q1);
        x[4] = csub(p1, q1);
        x[2] = cadd(p2, q2);
        x[3] = csub(p2, q2);
    }
};

// One Stockham pass on an LDS line; every thread of the workgroup calls it
// (the barriers are workgroup-wide), `active` says whether this thread owns a line.
// One Stockham pass on an LDS line; every thread of the workgroup calls it
// (the barriers are workgroup-wide), `active` says whether this thread owns a
// line.  DIR (-1 forward, +1 adjoint) is a compile-time constant, so the
// butterflies' multiplications by +-i fold; POW2 (L a power of two, so p is one
// too) turns the index arithmetic into masks.
template <typename C, int R, int DIR, bool POW2>
__device__ inline void stockham_pass(C *line, bool active, int L, int p, int twstep, int t, int tpl,
                                     const C *tw) {
    constexpr int NB = (8 + R - 1) / R;  // butterflies per thread when tpl = L / 8
    const int nbf = L / R;
    C x[NB][R];
    int kk[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = t + q * tpl;
        kk[q] = 0;
        if (active && i < nbf) {
            const int k = POW2 ? (i & (p - 1)) : i % p;
            kk[q] = k;
#pragma unroll
            for (int r = 0; r < R; ++r) x[q][r] = line[i + r * nbf];
            if (p > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const C w = tw[r * k * twstep];
                    x[q][r] = DIR < 0 ? cmul(x[q][r], w) : cmulc(x[q][r], w);
                }
            }
            Dft<C, R>::run(x[q], DIR);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = t + q * tpl;
        if (active && i < nbf) {
            const int j = (i - kk[q]) * R + kk[q];
#pragma unroll
            for (int r = 0; r < R; ++r) line[j + r * p] = x[q][r];
        }
    }
    __syncthreads();
}

// tw: the line's twiddle table W^j, j < L (LDS or global)
template <typename C, int DIR, bool POW2>
__device__ inline void line_fft(C *line, bool active, int t, const FftLine &fl, const C *tw) {
    int p = 1;
    for (int s = 0; s < fl.npass; ++s) {
        const int R = fl.rad[s];
        const int twstep = fl.L / (p * R);  // uniform
        switch (R) {
            case 8: stockham_pass<C, 8, DIR, POW2>(line, active, fl.L, p, twstep, t, fl.tpl, tw); break;
            case 4: stockham_pass<C, 4, DIR, POW2>(line, active, fl.L, p, twstep, t, fl.tpl, tw); break;
            case 2: stockham_pass<C, 2, DIR, POW2>(line, active, fl.L, p, twstep, t, fl.tpl, tw); break;
            case 5:
                if constexpr (!POW2) stockham_pass<C, 5, DIR, POW2>(line, active, fl.L, p, twstep, t, fl.tpl, tw);
                break;
            default:
                if constexpr (!POW2) stockham_pass<C, 3, DIR, POW2>(line, active, fl.L, p, twstep, t, fl.tpl, tw);
                break;
        }
        p *= R;
    }
}

// First Stockham pass (p = 1: no twiddles) of a line whose values come from memory:
// butterfly i takes rows i + r L/R from ld(row) and writes y_r to line[i R + r].  No
// barrier before: the line is not read until the caller's barrier after it.
template <typename C, int R, int DIR, typename LD>
__device__ inline void first_pass_in(C *line, bool active, int L, int t, int tpl, LD &ld) {
    constexpr int NB = (8 + R - 1) / R;
    const int nbf = L / R;
    C x[NB][R];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = t + q * tpl;
        if (active && i < nbf) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[q][r] = ld(i + r * nbf);
        }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = t + q * tpl;
        if (active && i < nbf) {
            Dft<C, R>::run(x[q], DIR);
#pragma unroll
            for (int r = 0; r < R; ++r) line[i * R + r] = x[q][r];
        }
    }
}

// Last Stockham pass (p = L/R, so k = i) of a line in LDS whose outputs go to
// memory: butterfly i reads line[i + r p], applies W^(r i), and hands y_r for row
// i + r p to st(row, slot, value), slot = q + r NB numbering a thread's outputs.
template <typename C, int R, int DIR, typename ST>
__device__ inline void last_pass_out(const C *line, bool active, int L, int t, int tpl, const C *tw,
                                     ST &st) {
    constexpr int NB = (8 + R - 1) / R;
    const int p = L / R;
    C x[NB][R];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = t + q * tpl;
        if (active && i < p) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[q][r] = line[i + r * p];
        }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = t + q * tpl;
        if (active && i < p) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const C w = tw[r * i];
                x[q][r] = DIR < 0 ? cmul(x[q][r], w) : cmulc(x[q][r], w);
            }
            Dft<C, R>::run(x[q], DIR);
#pragma unroll
            for (int r = 0; r < R; ++r) st(i + r * p, q + r * NB, x[q][r]);
        }
    }
}

// A line FFT (at least two passes) whose first pass loads from memory and whose last
// pass stores to memory, the passes between them in LDS: half the LDS traffic and
// three fewer barriers than loading the line into LDS first and storing it from there.
// The line must not be in use (the caller's barrier); the table tw must be ready
// by the first pass's barrier.
template <typename C, int DIR, bool POW2, typename LD, typename ST>
__device__ __attribute__((always_inline)) inline void line_fft_io(C *line, bool active, int t, const FftLine &fl, const C *tw, LD &ld,
                                   ST &st) {
    const int L = fl.L, tpl = fl.tpl;
    switch (fl.rad[0]) {
        case 8: first_pass_in<C, 8, DIR>(line, active, L, t, tpl, ld); break;
        case 4: first_pass_in<C, 4, DIR>(line, active, L, t, tpl, ld); break;
        case 2: first_pass_in<C, 2, DIR>(line, active, L, t, tpl, ld); break;
        case 5:
            if constexpr (!POW2) first_pass_in<C, 5, DIR>(line, active, L, t, tpl, ld);
            break;
        default:
            if constexpr (!POW2) first_pass_in<C, 3, DIR>(line, active, L, t, tpl, ld);
            break;
    }
    __syncthreads();
    int p = fl.rad[0];
    for (int s = 1; s + 1 < fl.npass; ++s) {
        const int R = fl.rad[s];
        const int twstep = L / (p * R);
        switch (R) {
            case 8: stockham_pass<C, 8, DIR, POW2>(line, active, L, p, twstep, t, tpl, tw); break;
            case 4: stockham_pass<C, 4, DIR, POW2>(line, active, L, p, twstep, t, tpl, tw); break;
            case 2: stockham_pass<C, 2, DIR, POW2>(line, active, L, p, twstep, t, tpl, tw); break;
            case 5:
                if constexpr (!POW2) stockham_pass<C, 5, DIR, POW2>(line, active, L, p, twstep, t, tpl, tw);
                break;
            default:
                if constexpr (!POW2) stockham_pass<C, 3, DIR, POW2>(line, active, L, p, twstep, t, tpl, tw);
                break;
        }
        p *= R;
    }
    switch (fl.rad[fl.npass - 1]) {
        case 8: last_pass_out<C, 8, DIR>(line, active, L, t, tpl, tw, st); break;
        case 4: last_pass_out<C, 4, DIR>(line, active, L, t, tpl, tw, st); break;
        case 2: last_pass_out<C, 2, DIR>(line, active, L, t, tpl, tw, st); break;
        case 5:
            if constexpr (!POW2) last_pass_out<C, 5, DIR>(line, active, L, t, tpl, tw, st);
            break;
        default:
            if constexpr (!POW2) last_pass_out<C, 3, DIR>(line, active, L, t, tpl, tw, st);
            break;
    }
}

// Strided axis pass: the workgroup owns B consecutive inner columns of one outer
// position; rows are read and written B complex values at a time.
// bx: the workgroup's block among the nbx blocks of this grid's pass.
template <typename T, int DIR, bool POW2>
__device__ __attribute__((always_inline)) inline void fft_strided_body(cplx<T> *grid, const FftLine &fl, const AxisPass &a, int bx,
                                        int nbx) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const int L = fl.L, LP = L + kLinePad;
    const int B = a.lines_per_block;  // a power of two
    const int lgB = __ffs(B) - 1;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int nchunk = (int)((a.inner + B - 1) / B);
    const int blk = xcd_block(bx, nbx);
    const int o = blk / nchunk;
    long long obase = 0;
    {
        int rem = o;
        for (int d = a.axis - 1; d >= 0; --d) {
            const int id = rem % a.outer_n[d];
            rem /= a.outer_n[d];
            const int pos = a.outer_band[d] ? band_pos(id, a.outer_n[d], a.outer_Nt[d]) : id;
            obase += (long long)pos * a.outer_stride[d];
        }
    }
    const long long inner = a.inner;
    const long long i0 = (long long)(blk - o * nchunk) * B;
    const C zero = cmake<C>((T)0, (T)0);

    // twiddle table after the B lines (when it fits)
    C *twl = lds + B * LP;
    if (fl.tw_lds) copy_table(twl, (const C *)fl.tw, L, tid, nthr);
    // Power-of-two lengths, decided per line: a batch of mixed lengths then runs the
    // same code for them as their own plans, and the radix-3 and radix-5 passes stay
    // out of this path's registers.
    if ((L & (L - 1)) == 0 && fl.npass >= 2) {
        // thread (b, t), b the faster: the B columns of a row are B consecutive values
        const int b = tid & (B - 1), t = tid >> lgB;
        const bool active = t < fl.tpl;
        const bool col_ok = i0 + b < inner;
        const long long cb = obase + (col_ok ? i0 + b : i0);
        const int bi = a.in_band_N, bo = a.out_band_N;
        // rows of the band of I_N: 0 .. ceil(N/2) - 1 and L - floor(N/2) .. L - 1
        auto ld = [&](int row) -> C {
            const bool in = col_ok && (!bi || row < bi - bi / 2 || row >= L - bi / 2);
            return in ? grid[cb + (long long)row * inner] : cmake<C>((T)0, (T)0);
        };
        auto st = [&](int row, int, C v) {
            if (col_ok && (!bo || row < bo - bo / 2 || row >= L - bo / 2))
                grid[cb + (long long)row * inner] = v;
        };
        C *line = lds + b * LP;
        if (fl.tw_lds) line_fft_io<C, DIR, true>(line, active, t, fl, twl, ld, st);
        else line_fft_io<C, DIR, true>(line, active, t, fl, (const C *)fl.tw, ld, st);
        return;
    }
    // load the band (or the whole lines): U loads per thread in flight at once
    const int nin = a.in_band_N ? a.in_band_N : L;
    {
        constexpr int U = 8;
        const int ntot = nin * B;
        for (int base = 0; base < ntot; base += U * nthr) {
            C v[U];
            int dst[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = base + u * nthr + tid;
                const int ic = idx < ntot ? idx : 0;
                const int bb = ic & (B - 1), r = ic >> lgB;
                const int row = a.in_band_N ? band_pos(r, a.in_band_N, L) : r;
                const bool col_ok = i0 + bb < inner;
                const long long col = col_ok ? i0 + bb : i0;  // i0 < inner always
                v[u] = grid[obase + (long long)row * inner + col];
                if (!col_ok) v[u] = zero;
                dst[u] = idx < ntot ? bb * LP + row : -1;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (dst[u] >= 0) lds[dst[u]] = v[u];
        }
    }
    if (a.in_band_N) {  // rows ceil(N/2) .. L - floor(N/2) - 1 hold no n of I_N
        const int nz = L - nin;
        for (int idx = tid; idx < nz * B; idx += nthr) {
            const int bb = idx & (B - 1), r = idx >> lgB;
            lds[bb * LP + (nin - nin / 2) + r] = zero;
        }
    }
    __syncthreads();

    const int b = tid / fl.tpl, t = tid % fl.tpl;
    const bool active = b < B;
    if (fl.tw_lds) line_fft<C, DIR, POW2>(lds + (active ? b : 0) * LP, active, t, fl, twl);
    else line_fft<C, DIR, POW2>(lds + (active ? b : 0) * LP, active, t, fl, (const C *)fl.tw);

    const int nout = a.out_band_N ? a.out_band_N : L;
    for (int idx = tid; idx < nout * B; idx += nthr) {
        const int bb = idx & (B - 1), r = idx >> lgB;
        const int row = a.out_band_N ? band_pos(r, a.out_band_N, L) : r;
        if (i0 + bb < inner) grid[obase + (long long)row * inner + i0 + bb] = lds[bb * LP + row];
    }
}

template <typename T, int DIR, bool POW2>
__global__ void __launch_bounds__(1024) k_fft_strided(cplx<T> *grid, FftLine fl, AxisPass a) {
    fft_strided_body<T, DIR, POW2>(grid + blockIdx.y * a.cstride, fl, a, blockIdx.x, gridDim.x);
}

// Axis-0 pass of the adjoint (D >= 2, all Nt_0 rows in, the band of I_N out)
// whose input is not the grid but the padded tiles of spreading: grid point
// (c_0, c') is the sum, over the source tiles that cover it, of their work
// items' padded-tile values (the halo merge, with the same summation order as
// the merge kernel).  The B columns of a workgroup lie in one tile column, so
// the item ranges of the tiles along axis 0 are read into LDS once.
template <typename T, int D, bool POW2>
__device__ inline void fft_axis0_from_pad_body(cplx<T> *grid, const FftLine &fl, const AxisPass &a,
                                               const PadSource &ps, const cplx<T> *pad, int bx,
                                               int nbx) {
    constexpr int DIR = +1;  // the adjoint's first pass
    using C = cplx<T>;
    constexpr int ER = 1 << (D - 1);  // shifts along the axes after axis 0
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const int L = fl.L, LP = L + kLinePad;
    const int B = a.lines_per_block;  // a power of two dividing Q_{D-1}
    const int lgB = __ffs(B) - 1;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int blk = xcd_block(bx, nbx);
    const long long inner = a.inner;
    const int i0 = blk * B;
    const Geom &g = ps.g;
    const int M2 = ps.M2;
    C *twl = lds + B * LP;
    int *rng = reinterpret_cast<int *>(twl + (fl.tw_lds ? L : 0));  // [T0][ER][2]

    // tile column of the workgroup and the columns' offsets inside it
    int tcr[D], ar[D];  // entries 1..D-1 used
    if constexpr (D == 2) {
        tcr[1] = i0 / g.Q[1];
        ar[1] = i0 - tcr[1] * g.Q[1];
    } else {
        const int c1 = i0 / g.Nt[2], c2 = i0 - c1 * g.Nt[2];
        tcr[1] = c1 / g.Q[1];
        ar[1] = c1 - tcr[1] * g.Q[1];
        tcr[2] = c2 / g.Q[2];
        ar[2] = c2 - tcr[2] * g.Q[2];
    }
    int P[D], ptot = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        P[d] = g.Q[d] + M2 - 1;
        ptot *= P[d];
    }
    const int T0 = g.T[0];
    for (int idx = tid; idx < T0 * ER; idx += nthr) {
        const int tr = idx / ER, er = idx % ER;
        int q = tr;
#pragma unroll
        for (int d = 1; d < D; ++d) {
            int qd = tcr[d] - ((er >> (d - 1)) & 1);
            if (qd < 0) qd += g.T[d];
            q = q * g.T[d] + qd;
        }
        rng[2 * idx] = ps.tile_sub[q];
        rng[2 * idx + 1] = ps.tile_sub[q + 1];
    }
    if (fl.tw_lds) copy_table(twl, (const C *)fl.tw, L, tid, nthr);
    __syncthreads();

    const float rq0 = 1.0f / (float)g.Q[0];
    const int bb = tid & (B - 1);  // fixed per thread: nthr is a multiple of B
    int al[D];                     // offsets of this thread's column, axes 1..D-1
#pragma unroll
    for (int d = 1; d < D; ++d) al[d] = ar[d];
    al[D - 1] += bb;
    constexpr int U = 4;
    constexpr int NE = 2 * ER;
    for (int base = 0; base < L * B; base += U * nthr) {
        int off[U][NE], src[U][NE], r_of[U];
        // per element and source tile: its first item (or -1) and the offset
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * nthr + tid;
            const int r = (idx < L * B ? idx : bb) >> lgB;
            r_of[u] = idx < L * B ? r : -1;
            int a0;
            const int tr = small_divmod(r, g.Q[0], rq0, a0);
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int e0 = e & 1, er = e >> 1;
                bool ok = !(e0 && a0 >= M2 - 1);
                int o = a0 + (e0 ? g.Q[0] : 0);
#pragma unroll
                for (int d = 1; d < D; ++d) {
                    const int ed = (er >> (d - 1)) & 1;
                    if (ed && al[d] >= M2 - 1) ok = false;
                    o = o * P[d] + al[d] + (ed ? g.Q[d] : 0);
                }
                int trs = tr - e0;
                if (trs < 0) trs += T0;
                const int* rr = rng + 2 * (trs * ER + er);
                src[u][e] = ok && rr[1] > rr[0] ? trs * ER + er : -1;
                off[u][e] = o;
            }
        }
        C v[U][NE];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < NE; ++e)
                v[u][e] = src[u][e] >= 0 ? pad[(size_t)rng[2 * src[u][e]] * ptot + off[u][e]]
                                         : cmake<C>((T)0, (T)0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (r_of[u] < 0) continue;
            // bit d of e: the source precedes along axis d (the merge kernel's order)
            T sr = (T)0, si = (T)0;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                sr += v[u][e].x;
                si += v[u][e].y;
                if (src[u][e] >= 0)
                    add_split_items(sr, si, pad, ptot, off[u][e], rng[2 * src[u][e]] + 1,
                                    rng[2 * src[u][e] + 1]);
            }
            lds[bb * LP + r_of[u]] = cmake<C>(sr, si);
        }
    }
    __syncthreads();

    const int b = tid / fl.tpl, t = tid % fl.tpl;
    const bool active = b < B;
    if (fl.tw_lds) line_fft<C, DIR, POW2>(lds + (active ? b : 0) * LP, active, t, fl, twl);
    else line_fft<C, DIR, POW2>(lds + (active ? b : 0) * LP, active, t, fl, (const C *)fl.tw);

    const int nout = a.out_band_N ? a.out_band_N : L;
    for (int idx = tid; idx < nout * B; idx += nthr) {
        const int cb = idx & (B - 1), r = idx >> lgB;
        const int row = a.out_band_N ? band_pos(r, a.out_band_N, L) : r;
        if (i0 + cb < inner) grid[(long long)row * inner + i0 + cb] = lds[cb * LP + row];
    }
}

template <typename T, int D, bool POW2>
__global__ void __launch_bounds__(1024) k_fft_axis0_from_pad(cplx<T> *grid, FftLine fl, AxisPass a,
                                                             PadSource ps) {
    fft_axis0_from_pad_body<T, D, POW2>(grid + blockIdx.y * a.cstride, fl, a, ps,
                                        (const cplx<T> *)ps.pad + blockIdx.y * ps.cstride,
                                        blockIdx.x, gridDim.x);
}

// Axis-0 pass of the 3-D adjoint whose input is the scratch of the column
// sweeps: grid point (p, i1, i2) is the sum of the scratch planes p of the up to
// four columns that cover (i1, i2) and, for the first 2m - 1 planes of a segment,
// of the preceding segments' halo planes -- the sweep's merge, in the same order
// of summation (the four column planes, then the four halo planes).  The B columns of a workgroup lie in one row of one 16 x 16
// column (B divides 16), so every source read is a run of B consecutive values.
template <typename T, bool POW2>
__global__ void __launch_bounds__(1024) k_fft_axis0_from_sweep(cplx<T> *grid, FftLine fl, AxisPass a,
                                                               SweepSource ss) {
    constexpr int DIR = +1;  // the adjoint's first pass
    using C = cplx<T>;
    grid += blockIdx.y * a.cstride;  // channel
    const C *scr = (const C *)ss.scr + blockIdx.y * ss.cstride;
    const C *halo = scr + ss.sg.main_cells;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const int L = fl.L, LP = L + kLinePad;
    const int B = a.lines_per_block;  // a power of two dividing 16
    const int lgB = __ffs(B) - 1;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const long long inner = a.inner;
    const int i0 = blk * B;
    const Geom &g = ss.g;
    const int taps = g.taps, P = kSweepQ + taps - 1, PP = P * P;
    const int ncols = ss.sg.ncols, nsc = ss.sg.nsc, Ls = ss.sg.L * g.Q[0];  // planes per segment
    C *twl = lds + B * LP;
    if (fl.tw_lds) copy_table(twl, (const C *)fl.tw, L, tid, nthr);

    // this thread's column and its up to four sources (column, offset in its padded plane)
    const int bb = tid & (B - 1);  // fixed per thread: nthr is a multiple of B
    const int i1 = i0 / g.Nt[2], i2 = i0 - i1 * g.Nt[2] + bb;
    const int t1 = i1 / kSweepQ, a1 = i1 - t1 * kSweepQ;
    const int t2 = i2 / kSweepQ, a2 = i2 - t2 * kSweepQ;
    int src_col[4], src_off[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int e1 = e >> 1, e2 = e & 1;  // the source column precedes along axis 1 / 2
        int c1 = t1 - e1, c2 = t2 - e2;
        if (c1 < 0) c1 += g.T[1];
        if (c2 < 0) c2 += g.T[2];
        const bool ok = !((e1 && a1 >= taps - 1) || (e2 && a2 >= taps - 1));
        src_col[e] = ok ? c1 * g.T[2] + c2 : -1;
        src_off[e] = (a1 + (e1 ? kSweepQ : 0)) * P + a2 + (e2 ? kSweepQ : 0);
    }
    // the columns' planes (all four sources' loads of U elements in flight) ...
    constexpr int U = 4;
    for (int base = 0; base < L * B; base += U * nthr) {
        C v[U][4];
        int r_of[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * nthr + tid;
            const int r = (idx < L * B ? idx : bb) >> lgB;  // plane
            r_of[u] = idx < L * B ? r : -1;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool ok = src_col[e] >= 0;
                v[u][e] = ok ? scr[((size_t)r * ncols + src_col[e]) * PP + src_off[e]]
                             : cmake<C>((T)0, (T)0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (r_of[u] < 0) continue;
            T sr = (T)0, si = (T)0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sr += v[u][e].x;
                si += v[u][e].y;
            }
            lds[bb * LP + r_of[u]] = cmake<C>(sr, si);
        }
    }
    __syncthreads();
    // ... then the preceding segments' halo planes on the first taps - 1 planes of
    // every segment (each element has one writer in both loops)
    const int nh = nsc * (taps - 1);
    for (int idx = tid; idx < nh * B; idx += nthr) {
        const int hb = idx & (B - 1), h = idx >> lgB;
        const int kseg = h / (taps - 1), j = h - kseg * (taps - 1);
        const int kpred = kseg == 0 ? nsc - 1 : kseg - 1;
        const int r = kseg * Ls + j;
        // the source columns of column hb (recomputed: hb differs from this thread's bb)
        const int hi2 = i0 - i1 * g.Nt[2] + hb;
        const int ht2 = hi2 / kSweepQ, ha2 = hi2 - ht2 * kSweepQ;
        C hv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int e1 = e >> 1, e2 = e & 1;
            int c1 = t1 - e1, c2 = ht2 - e2;
            if (c1 < 0) c1 += g.T[1];
            if (c2 < 0) c2 += g.T[2];
            const bool ok = !((e1 && a1 >= taps - 1) || (e2 && ha2 >= taps - 1));
            const int off = (a1 + (e1 ? kSweepQ : 0)) * P + ha2 + (e2 ? kSweepQ : 0);
            const int cc = c1 * g.T[2] + c2;
            hv[e] = ok ? halo[((size_t)(cc * nsc + kpred) * (taps - 1) + j) * PP + off]
                       : cmake<C>((T)0, (T)0);
        }
        T hr = (T)0, hi = (T)0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            hr += hv[e].x;
            hi += hv[e].y;
        }
        C acc = lds[hb * LP + r];
        acc.x += hr;
        acc.y += hi;
        lds[hb * LP + r] = acc;
    }
    __syncthreads();

    const int b = tid / fl.tpl, t = tid % fl.tpl;
    const bool active = b < B;
    if (fl.tw_lds) line_fft<C, DIR, POW2>(lds + (active ? b : 0) * LP, active, t, fl, twl);
    else line_fft<C, DIR, POW2>(lds + (active ? b : 0) * LP, active, t, fl, (const C *)fl.tw);

    const int nout = a.out_band_N ? a.out_band_N : L;
    for (int idx = tid; idx < nout * B; idx += nthr) {
        const int cb = idx & (B - 1), r = idx >> lgB;
        const int row = a.out_band_N ? band_pos(r, a.out_band_N, L) : r;
        if (i0 + cb < inner) grid[(long long)row * inner + i0 + cb] = lds[cb * LP + row];
    }
}

// Last-axis pass on contiguous lines.  mode 0: grid -> grid over all lines.
// mode 1: f -> grid; the line of outer position (i_0, .., i_{D-2}) in I_N gets
// f[i_0]..[r] * beta_0[i_0] .. beta_last[r] at (r - floor(N/2)) mod Nt, zeros
// elsewhere.  mode 2: grid -> y, y[i_0]..[r] = line[(r - floor(N/2)) mod Nt] * factors.
template <typename T> struct DecPtrs {
    const T *d[kMaxD];  // resampling-correction factors per axis
};

// bx: the workgroup's block; ch: its channel (the derivative channels use it).
template <typename T, int DIR, bool POW2>
__device__ __attribute__((always_inline)) inline void fft_contig_body(const cplx<T> *src, cplx<T> *dst, const FftLine &fl,
                                       const ContigPass &c, const DecPtrs<T> &dec, int bx, int ch) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const int L = fl.L, LP = L + kLinePad;
    const int tid = threadIdx.x;
    const int b = tid / fl.tpl, t = tid % fl.tpl;
    const int line_id = bx * c.lines_per_block + b;
    const bool active = b < c.lines_per_block && line_id < c.nlines;
    C *line = lds + (b < c.lines_per_block ? b : 0) * LP;
    C *twl = lds + c.lines_per_block * LP;  // twiddle table after the lines (when it fits)
    if (fl.tw_lds) copy_table(twl, (const C *)fl.tw, L, tid, (int)blockDim.x);
    const int D = c.D;
    const T *declast = dec.d[D - 1];

    // outer indices i_0..i_{D-2} of the line (the last fastest), its grid row and f row
    int iv[kMaxD] = {};
    {
        int rem = line_id;
        for (int d = D - 2; d >= 0; --d) {
            iv[d] = rem % c.outer_len[d];
            rem /= c.outer_len[d];
        }
    }
    long long grow = 0, frow = 0;
    T fac = (T)1;
    for (int d = 0; d < D - 1; ++d) {
        const int pd = c.outer_band[d] ? band_pos(iv[d], c.N[d], c.Nt[d]) : iv[d];
        grow = grow * c.Nt[d] + pd;
        frow = frow * c.N[d] + iv[d];
        if (c.mode != 0 && active) fac *= dec.d[d][iv[d]];
    }
    grow *= L;
    frow *= c.N[D - 1];
    // derivative channels (mode 1): channel d multiplies f by -2 pi i n_d
    const T twopi = (T)6.283185307179586476925;
    if (c.deriv && ch < D - 1) {
        const int d = ch;
        fac *= (T)(iv[d] - c.N[d] / 2) * twopi;
    }
    const int Nl = c.N[D - 1];

    // Power-of-two lengths decided per line (as in the strided pass) and modes 0 and 1:
    // the first pass loads the line (with the correction and the zero padding in mode
    // 1), the last pass stores it.  (Mode 2's cropping store measured slower from
    // registers: 34.4 against 31.5 us on the 3-D 128^3 complex128 workload.)
    if ((L & (L - 1)) == 0 && fl.npass >= 2 && c.mode != 2) {
        auto ld = [&](int k) -> C {
            if (c.mode == 1) {
                // n = r - floor(N/2) sits at k = n mod L: n >= 0 for k < ceil(N/2)
                int r = -1;
                if (k < Nl - Nl / 2) r = k + Nl / 2;
                else if (k >= L - Nl / 2) r = k - (L - Nl / 2);
                if (r < 0) return cmake<C>((T)0, (T)0);
                const C x = src[frow + r];
                T sc = fac * declast[r];
                if (c.deriv && ch == D - 1) sc *= (T)(r - Nl / 2) * twopi;
                const C y = cscale(x, sc);
                return c.deriv ? cmake<C>(y.y, -y.x) : y;  // (times -i)
            }
            return src[grow + k];
        };
        auto st = [&](int k, int, C v) { dst[grow + k] = v; };
        if (fl.tw_lds) line_fft_io<C, DIR, true>(line, active, t, fl, twl, ld, st);
        else line_fft_io<C, DIR, true>(line, active, t, fl, (const C *)fl.tw, ld, st);
        return;
    }

    // each thread owns k = t + j tpl, j < L / tpl <= 8 (the largest radix): all
    // its loads are issued before the first LDS write
    constexpr int KM = 8;
    if (active) {
        C v[KM];
        if (c.mode == 1) {
#pragma unroll
            for (int j = 0; j < KM; ++j) {
                const int k = t + j * fl.tpl;
                // n = r - floor(N/2) sits at k = n mod L: n >= 0 for k < ceil(N/2)
                int r = -1;
                if (k < Nl - Nl / 2) r = k + Nl / 2;
                else if (k >= L - Nl / 2 && k < L) r = k - (L - Nl / 2);
                const int rr = r >= 0 ? r : 0;
                const C x = src[frow + rr];
                T s = fac * declast[rr];
                if (c.deriv && ch == D - 1) s *= (T)(rr - Nl / 2) * twopi;
                C y = cscale(x, s);
                if (c.deriv) y = cmake<C>(y.y, -y.x);  // times -i
                v[j] = r >= 0 ? y : cmake<C>((T)0, (T)0);
            }
        } else {
#pragma unroll
            for (int j = 0; j < KM; ++j) {
                const int k = t + j * fl.tpl;
                v[j] = src[grow + (k < L ? k : 0)];
            }
        }
#pragma unroll
        for (int j = 0; j < KM; ++j) {
            const int k = t + j * fl.tpl;
            if (k < L) line[k] = v[j];
        }
    }
    __syncthreads();

    if (fl.tw_lds) line_fft<C, DIR, POW2>(line, active, t, fl, twl);
    else line_fft<C, DIR, POW2>(line, active, t, fl, (const C *)fl.tw);

    if (active) {
        if (c.mode == 2) {
            T dl[KM];
#pragma unroll
            for (int j = 0; j < KM; ++j) {
                const int r = t + j * fl.tpl;
                dl[j] = declast[r < Nl ? r : 0];
            }
#pragma unroll
            for (int j = 0; j < KM; ++j) {
                const int r = t + j * fl.tpl;
                if (r < Nl) dst[frow + r] = cscale(line[band_pos(r, Nl, L)], fac * dl[j]);
            }
        } else {
            for (int k = t; k < L; k += fl.tpl) dst[grow + k] = line[k];
        }
    }
}

template <typename T, int DIR, bool POW2>
__global__ void __launch_bounds__(1024) k_fft_contig(const cplx<T> *src, cplx<T> *dst, FftLine fl,
                                                     ContigPass c, DecPtrs<T> dec) {
    fft_contig_body<T, DIR, POW2>(src + blockIdx.y * c.src_cstride, dst + blockIdx.y * c.dst_cstride,
                                  fl, c, dec, blockIdx.x, blockIdx.y);
}

template <typename T>
static hipError_t fft_axis_t(const nfft_plan_s &p, void *grid, const AxisPass &a, hipStream_t s) {
    const int B = a.lines_per_block;
    size_t shm = 0;
    const FftLine fl = with_lds_table(p, p.line[a.axis], B, sizeof(cplx<T>), shm);
    const dim3 g((unsigned)(((a.inner + B - 1) / B) * a.outer_len), (unsigned)a.K);
    const bool pow2 = (fl.L & (fl.L - 1)) == 0;
    auto kern = a.dir < 0 ? (pow2 ? k_fft_strided<T, -1, true> : k_fft_strided<T, -1, false>)
                          : (pow2 ? k_fft_strided<T, 1, true> : k_fft_strided<T, 1, false>);
    if (shm > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, g, dim3(B * fl.tpl), shm, s, (cplx<T> *)grid, fl, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t fft_contig_t(const nfft_plan_s &p, const void *src, void *dst,
                               const ContigPass &c, hipStream_t s) {
    const int B = c.lines_per_block;
    size_t shm = 0;
    const FftLine fl = with_lds_table(p, p.line[p.D - 1], B, sizeof(cplx<T>), shm);
    const dim3 g((unsigned)((c.nlines + B - 1) / B), (unsigned)c.K);
    const bool pow2 = (fl.L & (fl.L - 1)) == 0;
    auto kern = c.dir < 0 ? (pow2 ? k_fft_contig<T, -1, true> : k_fft_contig<T, -1, false>)
                          : (pow2 ? k_fft_contig<T, 1, true> : k_fft_contig<T, 1, false>);
    if (shm > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    DecPtrs<T> dec;
    for (int d = 0; d < kMaxD; ++d) dec.d[d] = (const T *)p.deconv[d];
    hipLaunchKernelGGL(kern, g, dim3(B * fl.tpl), shm, s, (const cplx<T> *)src,
                       (cplx<T> *)dst, fl, c, dec);
    return hipGetLastError();
}

// ---- fused batches: one launch per pass for the transforms of a batch ----------

template <typename T, int DIR, bool POW2>
__global__ void __launch_bounds__(1024)
    k_fft_contig_batch(const BxFft *__restrict__ tab, const int *__restrict__ b2e,
                       const void *const *__restrict__ in, void *const *__restrict__ out) {
    const int e = b2e[blockIdx.x];
    if (e < 0) return;
    const BxFft &x = tab[e];
    DecPtrs<T> dec;
#pragma unroll
    for (int d = 0; d < kMaxD; ++d) dec.d[d] = (const T *)x.dec[d];
    const cplx<T> *src = (const cplx<T> *)(x.src_user ? in[x.t] : x.src);
    cplx<T> *dst = (cplx<T> *)(x.dst_user ? out[x.t] : x.grid);
    fft_contig_body<T, DIR, POW2>(src, dst, x.fl, x.c, dec, blockIdx.x - x.start, 0);
}

template <typename T, int DIR, bool POW2>
__global__ void __launch_bounds__(1024)
    k_fft_strided_batch(const BxFft *__restrict__ tab, const int *__restrict__ b2e) {
    const int e = b2e[blockIdx.x];
    if (e < 0) return;
    const BxFft &x = tab[e];
    fft_strided_body<T, DIR, POW2>((cplx<T> *)x.grid, x.fl, x.a, blockIdx.x - x.start, x.nblk);
}

template <typename T, int D, bool POW2>
__global__ void __launch_bounds__(1024)
    k_fft_axis0_from_pad_batch(const BxFft *__restrict__ tab, const int *__restrict__ b2e) {
    const int e = b2e[blockIdx.x];
    if (e < 0) return;
    const BxFft &x = tab[e];
    fft_axis0_from_pad_body<T, D, POW2>((cplx<T> *)x.grid, x.fl, x.a, x.ps,
                                        (const cplx<T> *)x.ps.pad, blockIdx.x - x.start, x.nblk);
}

template <typename K> static hipError_t allow_shm(K kern, size_t shm) {
    if (shm <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

template <typename T, int DIR, bool POW2>
static hipError_t fft_batch_t(int kind, int D, const BxFft *tab, const int *b2e,
                              const void *const *in, void *const *out, int nblocks, int nthreads,
                              size_t shm, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (kind == kBxContig) {
        auto kern = k_fft_contig_batch<T, DIR, POW2>;
        e = allow_shm(kern, shm);
        if (e == hipSuccess)
            hipLaunchKernelGGL(kern, dim3(nblocks), dim3(nthreads), shm, s, tab, b2e, in, out);
    } else if (kind == kBxStrided) {
        auto kern = k_fft_strided_batch<T, DIR, POW2>;
        e = allow_shm(kern, shm);
        if (e == hipSuccess) hipLaunchKernelGGL(kern, dim3(nblocks), dim3(nthreads), shm, s, tab, b2e);
    } else if (DIR > 0 && (D == 2 || D == 3)) {
        auto kern = D == 2 ? k_fft_axis0_from_pad_batch<T, 2, POW2> : k_fft_axis0_from_pad_batch<T, 3, POW2>;
        e = allow_shm(kern, shm);
        if (e == hipSuccess) hipLaunchKernelGGL(kern, dim3(nblocks), dim3(nthreads), shm, s, tab, b2e);
    } else {
        return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <typename T>
static hipError_t fft_batch_dir(int kind, int D, int dir, bool pow2, const BxFft *tab,
                                const int *b2e, const void *const *in, void *const *out,
                                int nblocks, int nthreads, size_t shm, hipStream_t s) {
    if (dir < 0)
        return pow2 ? fft_batch_t<T, -1, true>(kind, D, tab, b2e, in, out, nblocks, nthreads, shm, s)
                    : fft_batch_t<T, -1, false>(kind, D, tab, b2e, in, out, nblocks, nthreads, shm, s);
    return pow2 ? fft_batch_t<T, 1, true>(kind, D, tab, b2e, in, out, nblocks, nthreads, shm, s)
                : fft_batch_t<T, 1, false>(kind, D, tab, b2e, in, out, nblocks, nthreads, shm, s);
}

hipError_t launch_fft_batch(int kind, int dtype, int D, int dir, bool pow2, const BxFft *tab,
                            const int *b2e, const void *const *in, void *const *out, int nblocks,
                            int nthreads, size_t shm, hipStream_t s) {
    if (nblocks == 0) return hipSuccess;
    if (nthreads < 1 || nthreads > 1024) return hipErrorInvalidValue;
    return dtype == NFFT_C64
               ? fft_batch_dir<float>(kind, D, dir, pow2, tab, b2e, in, out, nblocks, nthreads, shm, s)
               : fft_batch_dir<double>(kind, D, dir, pow2, tab, b2e, in, out, nblocks, nthreads, shm, s);
}

hipError_t launch_fft_axis(const nfft_plan_s &p, void *grid, const AxisPass &a, hipStream_t s) {
    if (a.outer_len == 0 || a.inner == 0) return hipSuccess;
    return p.dtype == NFFT_C64 ? fft_axis_t<float>(p, grid, a, s) : fft_axis_t<double>(p, grid, a, s);
}

hipError_t launch_fft_axis0_from_pad(const nfft_plan_s &p, void *grid, const AxisPass &a,
                                     const void *pad, hipStream_t s) {
    const int B = a.lines_per_block;
    const size_t cs = p.dtype == NFFT_C64 ? sizeof(cplx<float>) : sizeof(cplx<double>);
    size_t shm = 0;
    const FftLine fl = with_lds_table(p, p.line[0], B, cs, shm);
    const int ER = 1 << (p.D - 1);
    shm += (size_t)p.geom.T[0] * ER * 2 * sizeof(int);
    PadSource ps{pad, p.tile_sub, p.geom, p.geom.taps,
                 (long long)p.nsub * (long long)padded_cells(p.geom, p.D)};
    const dim3 g((unsigned)(a.inner / B), (unsigned)a.K);
    const bool pow2 = (fl.L & (fl.L - 1)) == 0;
#define NFFT_PAD_LAUNCH(T, DD)                                                                     \
    {                                                                                              \
        auto kern = pow2 ? k_fft_axis0_from_pad<T, DD, true> : k_fft_axis0_from_pad<T, DD, false>; \
        if (shm > 65536) {                                                                         \
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),              \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm); \
            if (e != hipSuccess) return e;                                                         \
        }                                                                                          \
        hipLaunchKernelGGL(kern, g, dim3(B * fl.tpl), shm, s, (cplx<T> *)grid, fl, a, ps);         \
    }
    if (p.dtype == NFFT_C64) {
        if (p.D == 2) NFFT_PAD_LAUNCH(float, 2) else NFFT_PAD_LAUNCH(float, 3)
    } else {
        if (p.D == 2) NFFT_PAD_LAUNCH(double, 2) else NFFT_PAD_LAUNCH(double, 3)
    }
#undef NFFT_PAD_LAUNCH
    return hipGetLastError();
}

hipError_t launch_fft_axis0_from_sweep(const nfft_plan_s &p, void *grid, const AxisPass &a,
                                       const void *scr, hipStream_t s) {
    const int B = a.lines_per_block;
    const size_t cs = p.dtype == NFFT_C64 ? sizeof(cplx<float>) : sizeof(cplx<double>);
    size_t shm = 0;
    const FftLine fl = with_lds_table(p, p.line[0], B, cs, shm);
    SweepSource ss{scr, p.sweep, p.geom, (long long)sweep_scratch_cells(p)};
    const dim3 g((unsigned)(a.inner / B), (unsigned)a.K);
    const bool pow2 = (fl.L & (fl.L - 1)) == 0;
#define NFFT_SWEEP_LAUNCH(T)                                                                       \
    {                                                                                              \
        auto kern = pow2 ? k_fft_axis0_from_sweep<T, true> : k_fft_axis0_from_sweep<T, false>;     \
        if (shm > 65536) {                                                                         \
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),              \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm); \
            if (e != hipSuccess) return e;                                                         \
        }                                                                                          \
        hipLaunchKernelGGL(kern, g, dim3(B * fl.tpl), shm, s, (cplx<T> *)grid, fl, a, ss);         \
    }
    if (p.dtype == NFFT_C64) NFFT_SWEEP_LAUNCH(float) else NFFT_SWEEP_LAUNCH(double)
#undef NFFT_SWEEP_LAUNCH
    return hipGetLastError();
}

hipError_t launch_fft_contig(const nfft_plan_s &p, const void *src, void *dst, const ContigPass &c,
                             hipStream_t s) {
    if (c.nlines == 0) return hipSuccess;
    return p.dtype == NFFT_C64 ? fft_contig_t<float>(p, src, dst, c, s)
                               : fft_contig_t<double>(p, src, dst, c, s);
}

}  // namespace nfft
