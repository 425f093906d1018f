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

constexpr int kLinePad = 1;  // complex values of padding after each LDS line
constexpr int kNumXcd = 8;   // MI355X: 8 accelerator dies, each with its own L2

// Workgroups are dispatched round robin over the XCDs (block b runs on XCD b mod 8).
// Renumber them so that each XCD gets a contiguous run of logical blocks: blocks
// that share cache lines (neighbouring columns, neighbouring tiles) then share an L2.
__device__ inline int xcd_block(int b, int nblocks) {
    const int full = nblocks - nblocks % kNumXcd;
    if (b >= full) return b;
    return (b % kNumXcd) * (full / kNumXcd) + b / kNumXcd;
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
template <typename C, int R>
__device__ inline void stockham_pass(C *line, bool active, int L, int p, int t, int tpl,
                                     const C *tw, int dir) {
    constexpr int NB = (8 + R - 1) / R;  // butterflies per thread when tpl = L / 8
    const int nbf = L / R;
    const int twstep = L / (p * R);
    C x[NB][R];
    int kk[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = t + q * tpl;
        kk[q] = 0;
        if (active && i < nbf) {
            const int k = i % p;
            kk[q] = k;
#pragma unroll
            for (int r = 0; r < R; ++r) x[q][r] = line[i + r * nbf];
            if (p > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const C w = tw[r * k * twstep];
                    x[q][r] = dir < 0 ? cmul(x[q][r], w) : cmulc(x[q][r], w);
                }
            }
            Dft<C, R>::run(x[q], dir);
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

template <typename C>
__device__ inline void line_fft(C *line, bool active, int t, const FftLine &fl, int dir) {
    const C *tw = (const C *)fl.tw;
    int p = 1;
    for (int s = 0; s < fl.npass; ++s) {
        const int R = fl.rad[s];
        switch (R) {
            case 8: stockham_pass<C, 8>(line, active, fl.L, p, t, fl.tpl, tw, dir); break;
            case 4: stockham_pass<C, 4>(line, active, fl.L, p, t, fl.tpl, tw, dir); break;
            case 2: stockham_pass<C, 2>(line, active, fl.L, p, t, fl.tpl, tw, dir); break;
            case 5: stockham_pass<C, 5>(line, active, fl.L, p, t, fl.tpl, tw, dir); break;
            default: stockham_pass<C, 3>(line, active, fl.L, p, t, fl.tpl, tw, dir); break;
        }
        p *= R;
    }
}

// Strided axis pass: the workgroup owns B consecutive inner columns of one outer
// position; rows are read and written B complex values at a time.
template <typename T>
__global__ void __launch_bounds__(1024) k_fft_strided(cplx<T> *grid, FftLine fl, AxisPass a) {
    using C = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const int L = fl.L, LP = L + kLinePad;
    const int B = a.lines_per_block;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int nchunk = (int)((a.inner + B - 1) / B);
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int o = blk / nchunk;
    const long long obase =
        (long long)(a.outer_band_N ? band_pos(o, a.outer_band_N, a.outer_Nt) : o) * a.outer_stride;
    const long long inner = a.inner;
    const long long i0 = (long long)(blk - o * nchunk) * B;
    const C zero = cmake<C>((T)0, (T)0);

    const int nin = a.in_band_N ? a.in_band_N : L;
    for (int idx = tid; idx < nin * B; idx += nthr) {
        const int bb = idx % B, r = idx / B;
        const int row = a.in_band_N ? band_pos(r, a.in_band_N, L) : r;
        C v = zero;
        if (i0 + bb < inner) v = grid[obase + (long long)row * inner + i0 + bb];
        lds[bb * LP + row] = v;
    }
    if (a.in_band_N) {
        const int nz = L - nin;
        for (int idx = tid; idx < nz * B; idx += nthr) {
            const int bb = idx % B, r = idx / B;
            lds[bb * LP + nin / 2 + r] = zero;
        }
    }
    __syncthreads();

    const int b = tid / fl.tpl, t = tid % fl.tpl;
    const bool active = b < B;
    line_fft<C>(lds + (active ? b : 0) * LP, active, t, fl, a.dir);

    const int nout = a.out_band_N ? a.out_band_N : L;
    for (int idx = tid; idx < nout * B; idx += nthr) {
        const int bb = idx % B, r = idx / B;
        const int row = a.out_band_N ? band_pos(r, a.out_band_N, L) : r;
        if (i0 + bb < inner) grid[obase + (long long)row * inner + i0 + bb] = lds[bb * LP + row];
    }
}

// Last-axis pass on contiguous lines.  mode 0: grid -> grid over all lines.
// mode 1: f -> grid; the line of outer position (i0, i1) in I_N gets
// f[i0][i1][r] * beta_0[i0] beta_1[i1] beta_last[r] at (r - N/2) mod Nt, zeros
// elsewhere.  mode 2: grid -> y, y[i0][i1][r] = line[(r - N/2) mod Nt] * factors.
template <typename T>
__global__ void __launch_bounds__(1024) k_fft_contig(const cplx<T> *src, cplx<T> *dst, FftLine fl,
                                                     ContigPass c, const T *dec0, const T *dec1,
                                                     const T *dec2) {
    using C = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const int L = fl.L, LP = L + kLinePad;
    const int tid = threadIdx.x;
    const int b = tid / fl.tpl, t = tid % fl.tpl;
    const int line_id = blockIdx.x * c.lines_per_block + b;
    const bool active = b < c.lines_per_block && line_id < c.nlines;
    C *line = lds + (b < c.lines_per_block ? b : 0) * LP;
    const int D = c.D;
    const T *declast = D == 1 ? dec0 : (D == 2 ? dec1 : dec2);

    int i0 = 0, i1 = 0;
    if (D == 2) {
        i0 = line_id;
    } else if (D == 3) {
        i0 = line_id / c.outer_len[1];
        i1 = line_id - i0 * c.outer_len[1];
    }
    long long grow = 0, frow = 0;
    T fac = (T)1;
    if (D >= 2) {
        const int p0 = c.outer_band[0] ? band_pos(i0, c.N[0], c.Nt[0]) : i0;
        if (D == 2) {
            grow = (long long)p0 * L;
            frow = (long long)i0 * c.N[1];
        } else {
            const int p1 = c.outer_band[1] ? band_pos(i1, c.N[1], c.Nt[1]) : i1;
            grow = ((long long)p0 * c.Nt[1] + p1) * L;
            frow = ((long long)i0 * c.N[1] + i1) * c.N[2];
        }
        if (c.mode != 0 && active) {
            fac = dec0[i0];
            if (D == 3) fac *= dec1[i1];
        }
    }
    const int Nl = c.N[D - 1];

    if (active) {
        if (c.mode == 1) {
            for (int k = t; k < L; k += fl.tpl) {
                C v = cmake<C>((T)0, (T)0);
                int r = -1;
                if (k < Nl / 2) r = k + Nl / 2;
                else if (k >= L - Nl / 2) r = k - (L - Nl / 2);
                if (r >= 0) v = cscale(src[frow + r], fac * declast[r]);
                line[k] = v;
            }
        } else {
            for (int k = t; k < L; k += fl.tpl) line[k] = src[grow + k];
        }
    }
    __syncthreads();

    line_fft<C>(line, active, t, fl, c.dir);

    if (active) {
        if (c.mode == 2) {
            for (int r = t; r < Nl; r += fl.tpl)
                dst[frow + r] = cscale(line[band_pos(r, Nl, L)], fac * declast[r]);
        } else {
            for (int k = t; k < L; k += fl.tpl) dst[grow + k] = line[k];
        }
    }
}

template <typename T>
static hipError_t fft_axis_t(const nfft_plan_s &p, void *grid, const AxisPass &a, hipStream_t s) {
    const FftLine &fl = p.line[a.axis];
    const int B = a.lines_per_block;
    const size_t shm = (size_t)B * (fl.L + kLinePad) * sizeof(cplx<T>);
    const dim3 g((unsigned)(((a.inner + B - 1) / B) * a.outer_len));
    if (shm > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_fft_strided<T>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_fft_strided<T>, g, dim3(B * fl.tpl), shm, s, (cplx<T> *)grid, fl, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t fft_contig_t(const nfft_plan_s &p, const void *src, void *dst,
                               const ContigPass &c, hipStream_t s) {
    const FftLine &fl = p.line[p.D - 1];
    const int B = c.lines_per_block;
    const size_t shm = (size_t)B * (fl.L + kLinePad) * sizeof(cplx<T>);
    const dim3 g((unsigned)((c.nlines + B - 1) / B));
    hipLaunchKernelGGL(k_fft_contig<T>, g, dim3(B * fl.tpl), shm, s, (const cplx<T> *)src,
                       (cplx<T> *)dst, fl, c, (const T *)p.deconv[0], (const T *)p.deconv[1],
                       (const T *)p.deconv[2]);
    return hipGetLastError();
}

hipError_t launch_fft_axis(const nfft_plan_s &p, void *grid, const AxisPass &a, hipStream_t s) {
    if (a.outer_len == 0 || a.inner == 0) return hipSuccess;
    return p.dtype == NFFT_C64 ? fft_axis_t<float>(p, grid, a, s) : fft_axis_t<double>(p, grid, a, s);
}

hipError_t launch_fft_contig(const nfft_plan_s &p, const void *src, void *dst, const ContigPass &c,
                             hipStream_t s) {
    if (c.nlines == 0) return hipSuccess;
    return p.dtype == NFFT_C64 ? fft_contig_t<float>(p, src, dst, c, s)
                               : fft_contig_t<double>(p, src, dst, c, s);
}

}  // namespace nfft
