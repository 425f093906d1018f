// Plan-time node preparation and GPU bin sort of the nodes into grid tiles.
//
// Per node and axis (in FP64): wrap x into [-1/2, 1/2), y = Nt*x, c = floor(y),
// frac = y - c, stencil origin o = (c - lo) mod Nt with lo = m - 1 (2m points)
// or m (the wide stencil of 2m + 2 points).  The stencil of the node covers grid
// points o .. o+taps-1 (mod Nt) on that axis.  The node is binned by
// the tile that holds its origin and, inside the tile, by a sub-key: for D <= 3 the
// LDS bank slot of the node's first value in the interpolation's LDS (the plans
// then interleave the slots by a second sort, see launch_node_sort), for D >= 4 a
// class bit per axis that says whether its stencil runs past the end of that tile
// into the next one.  Sort key = tile << kbits | sub-key (Geom::kbits).  The bin
// boundaries come from a histogram and an exclusive scan; the order is a stable
// sort of (key, node index) pairs -- least-significant
// digit first, 8 bits per pass, each pass a stable counting sort -- so nodes of
// one bin keep the caller's order and a plan is a deterministic function of its
// nodes (its work items, and with them every summation order, do not depend on
// the scheduling of the plan-time kernels).
#include <math.h>

#include <algorithm>

#include <string.h>

#include "common.hpp"
#include "nfft_internal.hpp"

namespace nfft {

__global__ void k_fill_int(int *a, int64_t n, int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// Zero n complex values (n*2 reals of 4 or 8 bytes) with 16-byte stores where possible.
__global__ void k_zero_bytes16(uint4 *a, int64_t n16) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) a[i] = make_uint4(0, 0, 0, 0);
}
__global__ void k_zero_bytes8(uint2 *a, int64_t n8) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n8) a[i] = make_uint2(0, 0);
}

struct Cell {
    int o;        // stencil origin mod Nt
    double frac;  // fractional offset in [0, 1)
};

__device__ inline Cell node_cell(double xv, int Nt, int lo) {
    const double xw = xv - floor(xv + 0.5);
    const double y = xw * (double)Nt;
    const double c = floor(y);
    long long o = (long long)c - lo;
    o %= Nt;
    if (o < 0) o += Nt;
    Cell cell;
    cell.o = (int)o;
    cell.frac = y - c;
    return cell;
}

template <typename T, int D>
__global__ void k_node_keys(const T *x, int M, Geom g, int *keys, int *counts, int *bad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    int tile = 0, cls = 0, slot = 0;
    bool ok = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double xv = (double)x[(size_t)j * D + d];
        if (!isfinite(xv)) {
            ok = false;
            continue;
        }
        const Cell c = node_cell(xv, g.Nt[d], g.lo);
        const int p = c.o / g.Q[d];
        const int loc = c.o - p * g.Q[d];
        tile = tile * g.T[d] + p;
        cls |= (loc >= g.Q[d] - (g.taps - 1)) ? (1 << d) : 0;
        if (g.ring_R > 0 && D == 3) {
            // the bank slot in the sweep's ring: (o_0 mod R) P^2 + (o_1 mod 16) P + o_2 mod 16
            const int P = kSweepQ + g.taps - 1;
            slot += d == 0 ? (c.o % g.ring_R) * P * P : d == 1 ? (c.o % kSweepQ) * P : c.o % kSweepQ;
        } else {
            // in the tile with its trailing halo: the row-major offset of the local cell
            slot = slot * (g.Q[d] + g.taps - 1) + loc;
        }
    }
    if (g.slot_mod > 0) cls = slot & (g.slot_mod - 1);
    if (!ok) {
        *bad = 1;
        tile = 0;
        cls = 0;
    }
    const int key = (tile << g.kbits) | cls;
    keys[j] = key;
    atomicAdd(&counts[key], 1);
}

__global__ void k_iota(int *a, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = i;
}

// Sorted position pos holds node perm[pos]: its stencil origin and fraction per axis.
template <typename T, int D>
__global__ void k_node_gather(const T *x, int M, Geom g, const int *perm, NodeRec<T, D> *nodes) {
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= M) return;
    const int j = perm[pos];
    NodeRec<T, D> rec;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double xv = (double)x[(size_t)j * D + d];
        if (!isfinite(xv)) xv = 0.0;  // the plan is rejected; keep the record in range
        const Cell c = node_cell(xv, g.Nt[d], g.lo);
        rec.o[d] = c.o;
        rec.fr[d] = (T)c.frac;
    }
    nodes[pos] = rec;
}

// Exclusive scan of n ints by one workgroup of 1024 threads: out[0..n], out[n] = total.
__global__ void __launch_bounds__(1024) k_exclusive_scan(const int *in, int *out, int n) {
    __shared__ int part[1024];
    const int tid = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int b = tid * chunk;
    const int e = min(n, b + chunk);
    int s = 0;
    for (int i = b; i < e; ++i) s += in[i];
    part[tid] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = tid > 0 ? part[tid - 1] : 0;
    for (int i = b; i < e; ++i) {
        out[i] = run;
        run += in[i];
    }
    if (tid == 1023) out[n] = part[1023];
}

// Interpolation work items: tile p is cut into ceil(count / maxn) items of <= maxn nodes.
__global__ void k_subprob_count(const int *key_start, int ntiles, int kbits, int maxn, int *counts) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ntiles) return;
    const int n = key_start[(p + 1) << kbits] - key_start[p << kbits];
    counts[p] = (n + maxn - 1) / maxn;
}

__global__ void k_subprob_fill(const int *key_start, const int *sub_start, int ntiles, int kbits,
                               int maxn, int4 *subs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ntiles) return;
    const int b = key_start[p << kbits];
    const int e = key_start[(p + 1) << kbits];
    int w = sub_start[p];
    for (int s = b; s < e; s += maxn) subs[w++] = make_int4(p, s, min(e, s + maxn), 0);
}

static inline dim3 grid1d(int64_t n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

hipError_t launch_fill_int(int *a, int64_t n, int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, grid1d(n, 256), dim3(256), 0, s, a, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_zero_complex(void *a, int64_t n, bool dbl, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (dbl)
        hipLaunchKernelGGL(k_zero_bytes16, grid1d(n, 256), dim3(256), 0, s, (uint4 *)a, n);
    else
        hipLaunchKernelGGL(k_zero_bytes8, grid1d(n, 256), dim3(256), 0, s, (uint2 *)a, n);
    return hipGetLastError();
}

template <typename T, int D>
static void keys_t(const nfft_plan_s &p, const void *x, int *keys, int *counts, int *bad,
                   hipStream_t s) {
    hipLaunchKernelGGL((k_node_keys<T, D>), grid1d(p.M, 256), dim3(256), 0, s, (const T *)x,
                       (int)p.M, p.geom, keys, counts, bad);
}

template <typename T, int D>
static void gather_t(nfft_plan_s &p, const void *x, hipStream_t s) {
    hipLaunchKernelGGL((k_node_gather<T, D>), grid1d(p.M, 256), dim3(256), 0, s, (const T *)x,
                       (int)p.M, p.geom, p.perm, (NodeRec<T, D> *)p.nodes);
}

hipError_t launch_node_keys(const nfft_plan_s &p, const void *x, int *keys, int *counts, int *bad,
                            hipStream_t s) {
    if (p.M == 0) return hipSuccess;
    const bool f = p.dtype == NFFT_C64;
    switch (p.D) {
        case 1: f ? keys_t<float, 1>(p, x, keys, counts, bad, s) : keys_t<double, 1>(p, x, keys, counts, bad, s); break;
        case 2: f ? keys_t<float, 2>(p, x, keys, counts, bad, s) : keys_t<double, 2>(p, x, keys, counts, bad, s); break;
        case 3: f ? keys_t<float, 3>(p, x, keys, counts, bad, s) : keys_t<double, 3>(p, x, keys, counts, bad, s); break;
        case 4: f ? keys_t<float, 4>(p, x, keys, counts, bad, s) : keys_t<double, 4>(p, x, keys, counts, bad, s); break;
        case 5: f ? keys_t<float, 5>(p, x, keys, counts, bad, s) : keys_t<double, 5>(p, x, keys, counts, bad, s); break;
        case 6: f ? keys_t<float, 6>(p, x, keys, counts, bad, s) : keys_t<double, 6>(p, x, keys, counts, bad, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Exclusive scan of large n in three launches, without scratch: the sum of every block
// of kScanBlock inputs goes to the block's first output slot, one workgroup scans
// those slots in place (and writes the total to out[n]), and every block then scans
// its inputs from the offset it finds there.
constexpr int kScanBlock = 2048;  // 256 threads x 8 consecutive inputs

__global__ void __launch_bounds__(256) k_scan_sums(const int *__restrict__ in, int n, int *out) {
    __shared__ int ws[4];
    const int base = blockIdx.x * kScanBlock, end = min(n, base + kScanBlock);
    int v = 0;
    for (int i = base + threadIdx.x; i < end; i += 256) v += in[i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) out[base] = ws[0] + ws[1] + ws[2] + ws[3];
}

// out[b * stride] for b < nb: block sums -> their exclusive prefix sums; out[n] = total.
__global__ void __launch_bounds__(1024) k_scan_offsets(int *out, int nb, int stride, int n) {
    __shared__ int part[1024];
    const int tid = threadIdx.x;
    const int chunk = (nb + 1023) / 1024;
    const int b = tid * chunk, e = min(nb, b + chunk);
    int s = 0;
    for (int i = b; i < e; ++i) s += out[(size_t)i * stride];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = tid > 0 ? part[tid - 1] : 0;
    for (int i = b; i < e; ++i) {
        const int v = out[(size_t)i * stride];
        out[(size_t)i * stride] = run;
        run += v;
    }
    if (tid == 1023) out[n] = part[1023];
}

__global__ void __launch_bounds__(256) k_scan_apply(const int *__restrict__ in, int n, int *out) {
    __shared__ int ws[4];
    __shared__ int offset;
    const int base = blockIdx.x * kScanBlock;
    if (threadIdx.x == 0) offset = out[base];  // (read before the block overwrites it)
    const int i0 = base + threadIdx.x * 8;
    int v[8];
    int tsum = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        v[u] = i0 + u < n ? in[i0 + u] : 0;
        tsum += v[u];
    }
    // exclusive prefix of the thread sums: wavefront scan, then the wavefronts' totals
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = tsum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) ws[wave] = incl;
    __syncthreads();
    int run = offset + incl - tsum;
    for (int w = 0; w < wave; ++w) run += ws[w];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if (i0 + u < n) out[i0 + u] = run;
        run += v[u];
    }
}

hipError_t launch_exclusive_scan(const int *in, int *out, int n, hipStream_t s) {
    if (n <= 4 * kScanBlock) {
        hipLaunchKernelGGL(k_exclusive_scan, dim3(1), dim3(1024), 0, s, in, out, n);
        return hipGetLastError();
    }
    const int nb = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(256), 0, s, in, n, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, s, out, nb, kScanBlock, n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

// ---- stable sort of (key, node index) pairs ----------------------------------
//
// Least-significant-digit radix sort, 8 bits per pass; each pass is a stable
// counting sort of the current sequence by one digit:
//   k_digit_hist    block b counts the digits of its run of kSortRun consecutive
//                   items: hist[digit * nblocks + b];
//   exclusive scan  of hist in (digit, block) order: the first output position of
//                   every (digit, block) pair;
//   k_digit_scatter block b walks its run again in order, 256 items at a time, and
//                   sends each item to its pair's first position plus the number of
//                   items of its digit before it in the run (a wavefront finds the
//                   lanes with its digit by ballots over the digit's bits; per-wave
//                   and running per-digit counts sit in LDS).
// Items of equal digit keep their order, so after the passes over all key bits the
// pairs are ordered by key and, within a key, by node index.

constexpr int kSortThreads = 256;
constexpr int kSortBins = 256;

// Items per block: a multiple of kSortThreads that keeps the histogram (and its
// single-workgroup scan) at most 2^24 entries.
static int sort_run(int64_t M) {
    int64_t chunks = 16;
    while ((M + chunks * kSortThreads - 1) / (chunks * kSortThreads) * kSortBins > (1 << 24))
        chunks *= 2;
    return (int)(chunks * kSortThreads);
}

__global__ void __launch_bounds__(kSortThreads)
    k_digit_hist(const int *__restrict__ keys, int M, int shift, int run, int *__restrict__ hist) {
    __shared__ int cnt[kSortBins];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int b = blockIdx.x;
    const int end = min(M, (b + 1) * run);
    for (int i = b * run + threadIdx.x; i < end; i += kSortThreads)
        atomicAdd(&cnt[(keys[i] >> shift) & (kSortBins - 1)], 1);
    __syncthreads();
    hist[threadIdx.x * gridDim.x + b] = cnt[threadIdx.x];
}

// kout may be NULL (the last pass needs only the permutation).
__global__ void __launch_bounds__(kSortThreads)
    k_digit_scatter(const int *__restrict__ kin, const int *__restrict__ iin, int M, int shift,
                    int run, const int *__restrict__ start, int *__restrict__ kout,
                    int *__restrict__ iout) {
    constexpr int W = kSortThreads / 64;
    __shared__ int base[kSortBins];       // next output position of each digit in this run
    __shared__ int wcnt[W][kSortBins];    // items of each digit in each wavefront of the round
    const int b = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    base[threadIdx.x] = start[threadIdx.x * gridDim.x + b];
    const int end = min(M, (b + 1) * run);
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int r0 = b * run; r0 < end; r0 += kSortThreads) {
        for (int w = 0; w < W; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();  // also orders the base update of the previous round
        const int i = r0 + threadIdx.x;
        const bool live = i < end;
        const int key = live ? kin[i] : 0;
        const int val = live ? iin[i] : 0;
        // digit, with bit 8 set for lanes past the end so that they match no item
        const int dig = live ? (key >> shift) & (kSortBins - 1) : kSortBins;
        unsigned long long peers = ~0ull;
#pragma unroll
        for (int bit = 0; bit < 9; ++bit) {
            const unsigned long long bal = __ballot((dig >> bit) & 1);
            peers &= ((dig >> bit) & 1) ? bal : ~bal;
        }
        const int rank = __popcll(peers & below);
        // the lowest lane of each digit group records the group's size
        if (live && rank == 0) wcnt[wave][dig] = __popcll(peers);
        __syncthreads();
        if (live) {
            int pos = base[dig] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][dig];
            if (kout) kout[pos] = key;
            iout[pos] = val;
        }
        __syncthreads();  // every position of the round is taken before base moves on
        int tot = 0;
        for (int w = 0; w < W; ++w) tot += wcnt[w][threadIdx.x];
        base[threadIdx.x] += tot;
    }
}

static unsigned key_bits(int nkeys) {
    unsigned b = 1;
    while (b < 31 && (1u << b) < (unsigned)nkeys) ++b;
    return b;
}

// Scratch of the sort: a second key and index sequence, and the histogram with its scan.
hipError_t node_sort_bytes(const nfft_plan_s &p, size_t *bytes) {
    *bytes = 0;
    if (p.M == 0) return hipSuccess;
    const int64_t nb = (p.M + sort_run(p.M) - 1) / sort_run(p.M);
    *bytes = sizeof(int) * (2 * (size_t)p.M + 2 * ((size_t)kSortBins * nb + 1));
    return hipSuccess;
}

// Radix passes over `bits` key bits of (kin, iin): intermediate sequences alternate
// between (kb, ib) and (k2, i2); the last pass writes the indices to iout and, when
// kout is not NULL, the keys to kout (neither aliasing that pass's input).
static hipError_t radix_passes(const int *kin, const int *iin, int M, unsigned bits, int *kb, int *ib,
                               int *k2, int *i2, int *hist, int *start, int *kout, int *iout,
                               hipStream_t s) {
    const int run = sort_run(M);
    const int nb = (M + run - 1) / run;
    const int nh = kSortBins * nb;
    const int passes = (int)(bits + 7) / 8;
    hipError_t e = hipSuccess;
    for (int pass = 0; pass < passes; ++pass) {
        const bool last = pass == passes - 1;
        int *ko = last ? kout : (pass % 2 == 0 ? kb : k2);
        int *io = last ? iout : (pass % 2 == 0 ? ib : i2);
        hipLaunchKernelGGL(k_digit_hist, dim3(nb), dim3(kSortThreads), 0, s, kin, M, 8 * pass, run,
                           hist);
        e = hipGetLastError();
        if (e == hipSuccess) e = launch_exclusive_scan(hist, start, nh, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_digit_scatter, dim3(nb), dim3(kSortThreads), 0, s, kin, iin, M,
                           8 * pass, run, start, ko, io);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        kin = ko;
        iin = io;
    }
    return e;
}

// Second sort key of the bank-slot plans, per sorted position: (tile, bank slot mod 8,
// rank of the node among the tile's nodes of its slot, slot / 8), so that after the
// second stable sort 2^(kbits - 3) consecutive nodes of a tile -- four (complex128,
// slots mod 32) or eight (complex64, mod 64) -- have slots 8 apart wherever those
// slots have a node of that rank.
__global__ void k_slot_group_keys(const int *__restrict__ ks, const int *__restrict__ key_start, int M,
                            int kbits, int rbits, int *__restrict__ key2) {
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= M) return;
    const int key = ks[pos];
    const int tile = key >> kbits, slot = key & ((1 << kbits) - 1);
    const int rank = min(pos - key_start[key], (1 << rbits) - 1);
    key2[pos] = (((((tile << 3) | (slot & 7)) << rbits) | rank) << (kbits - 3)) | (slot >> 3);
}

hipError_t launch_node_sort(nfft_plan_s &p, const void *x, int *keys, int *keys_sorted, int *idx,
                            void *tmp, size_t tmp_bytes, hipStream_t s) {
    if (p.M == 0) return hipSuccess;
    const int M = (int)p.M;
    const int run = sort_run(M);
    const int nb = (M + run - 1) / run;
    const int nh = kSortBins * nb;
    size_t need = 0;
    (void)node_sort_bytes(p, &need);
    if (tmp_bytes < need) return hipErrorInvalidValue;
    int *kb = (int *)tmp, *ib = kb + M, *hist = ib + M, *start = hist + nh + 1;
    hipLaunchKernelGGL(k_iota, grid1d(M, 256), dim3(256), 0, s, idx, M);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned bits = key_bits(p.nkeys);
    if (p.geom.slot_mod == 0) {
        e = radix_passes(keys, idx, M, bits, kb, ib, keys_sorted, idx, hist, start, nullptr, p.perm, s);
        if (e != hipSuccess) return e;
    } else {
        // (tile, slot) first, keeping the sorted keys: pass i reads (keys, idx) for i = 0,
        // else (kb, ib) for odd i and (keys_sorted, idx) for even i, so the last pass
        // writes its keys to the pair it does not read
        const int passes1 = (int)(bits + 7) / 8;
        int *ks = passes1 % 2 == 0 ? keys_sorted : kb;
        e = radix_passes(keys, idx, M, bits, kb, ib, keys_sorted, idx, hist, start, ks, p.perm, s);
        if (e != hipSuccess) return e;
        unsigned tbits = 1;
        while (tbits < 31 && (1u << tbits) < (unsigned)p.geom.ntiles) ++tbits;
        // ranks from 2^rbits - 1 on (31 at most) keep their order (a bin holds a handful
        // of nodes unless the nodes cluster); the fewer key bits, the fewer passes
        const int jbits = p.geom.kbits - 3;
        const int rbits = std::min(5, 31 - (int)tbits - 3 - jbits);
        if (rbits >= 1) {  // (else, with more tiles than the key holds, the first order stays)
            // then the grouping key (into keys, free now), carrying the permutation
            hipLaunchKernelGGL(k_slot_group_keys, grid1d(M, 256), dim3(256), 0, s, ks, p.key_start, M,
                               p.geom.kbits, rbits, keys);
            e = hipGetLastError();
            if (e == hipSuccess)
                e = hipMemcpyAsync(idx, p.perm, (size_t)M * sizeof(int), hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
                e = radix_passes(keys, idx, M, tbits + 3 + (unsigned)(rbits + jbits), kb, ib,
                                 keys_sorted, idx, hist, start, nullptr, p.perm, s);
            if (e != hipSuccess) return e;
        }
    }
    const bool f = p.dtype == NFFT_C64;
    switch (p.D) {
        case 1: f ? gather_t<float, 1>(p, x, s) : gather_t<double, 1>(p, x, s); break;
        case 2: f ? gather_t<float, 2>(p, x, s) : gather_t<double, 2>(p, x, s); break;
        case 3: f ? gather_t<float, 3>(p, x, s) : gather_t<double, 3>(p, x, s); break;
        case 4: f ? gather_t<float, 4>(p, x, s) : gather_t<double, 4>(p, x, s); break;
        case 5: f ? gather_t<float, 5>(p, x, s) : gather_t<double, 5>(p, x, s); break;
        case 6: f ? gather_t<float, 6>(p, x, s) : gather_t<double, 6>(p, x, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_subprob_count(const nfft_plan_s &p, int *counts, hipStream_t s) {
    hipLaunchKernelGGL(k_subprob_count, grid1d(p.geom.ntiles, 256), dim3(256), 0, s, p.key_start,
                       p.geom.ntiles, p.geom.kbits, p.max_block_nodes, counts);
    return hipGetLastError();
}

hipError_t launch_subprob_fill(nfft_plan_s &p, const int *sub_start, hipStream_t s) {
    hipLaunchKernelGGL(k_subprob_fill, grid1d(p.geom.ntiles, 256), dim3(256), 0, s, p.key_start,
                       sub_start, p.geom.ntiles, p.geom.kbits, p.max_block_nodes, p.subs);
    return hipGetLastError();
}

}  // namespace nfft
