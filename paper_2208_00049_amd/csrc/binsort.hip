// Plan-time node preparation and GPU bin sort of the nodes into grid tiles.
//
// Per node and axis (in FP64): wrap x into [-1/2, 1/2), y = Nt*x, c = floor(y),
// frac = y - c, stencil origin o = (c - lo) mod Nt with lo = m - 1 (2m points)
// or m (the wide stencil of 2m + 2 points).  The stencil of the node covers grid
// points o .. o+taps-1 (mod Nt) on that axis.  The node is binned by
// the tile that holds its origin, and by a class bit per axis that says whether
// its stencil runs past the end of that tile into the next one.  Sort key =
// tile << D | class.  The bin boundaries come from a histogram and an exclusive
// scan; the order is a stable radix sort of (key, node index) pairs (rocPRIM),
// so nodes of one bin keep the caller's order and a plan is a deterministic
// function of its nodes (its work items, and with them every summation order,
// do not depend on the scheduling of the plan-time kernels).
#include <math.h>

#include <string.h>

#include <rocprim/device/device_radix_sort.hpp>

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
    int tile = 0, cls = 0;
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
    }
    if (!ok) {
        *bad = 1;
        tile = 0;
        cls = 0;
    }
    const int key = (tile << D) | cls;
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
__global__ void k_subprob_count(const int *key_start, int ntiles, int D, int maxn, int *counts) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ntiles) return;
    const int n = key_start[(p + 1) << D] - key_start[p << D];
    counts[p] = (n + maxn - 1) / maxn;
}

__global__ void k_subprob_fill(const int *key_start, const int *sub_start, int ntiles, int D,
                               int maxn, int4 *subs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ntiles) return;
    const int b = key_start[p << D];
    const int e = key_start[(p + 1) << D];
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
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(const int *in, int *out, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_exclusive_scan, dim3(1), dim3(1024), 0, s, in, out, n);
    return hipGetLastError();
}

static unsigned key_bits(int nkeys) {
    unsigned b = 1;
    while (b < 31 && (1u << b) < (unsigned)nkeys) ++b;
    return b;
}

hipError_t node_sort_bytes(const nfft_plan_s &p, size_t *bytes) {
    *bytes = 0;
    if (p.M == 0) return hipSuccess;
    return rocprim::radix_sort_pairs(nullptr, *bytes, (const int *)nullptr, (int *)nullptr,
                                     (const int *)nullptr, (int *)nullptr, (int)p.M, 0,
                                     key_bits(p.nkeys), (hipStream_t)0);
}

hipError_t launch_node_sort(nfft_plan_s &p, const void *x, const int *keys, int *keys_sorted,
                            int *idx, void *tmp, size_t tmp_bytes, hipStream_t s) {
    if (p.M == 0) return hipSuccess;
    const int M = (int)p.M;
    hipLaunchKernelGGL(k_iota, grid1d(M, 256), dim3(256), 0, s, idx, M);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = tmp_bytes;
    e = rocprim::radix_sort_pairs(tmp, bytes, keys, keys_sorted, (const int *)idx, p.perm, M, 0,
                                  key_bits(p.nkeys), s);
    if (e != hipSuccess) return e;
    const bool f = p.dtype == NFFT_C64;
    switch (p.D) {
        case 1: f ? gather_t<float, 1>(p, x, s) : gather_t<double, 1>(p, x, s); break;
        case 2: f ? gather_t<float, 2>(p, x, s) : gather_t<double, 2>(p, x, s); break;
        case 3: f ? gather_t<float, 3>(p, x, s) : gather_t<double, 3>(p, x, s); break;
        case 4: f ? gather_t<float, 4>(p, x, s) : gather_t<double, 4>(p, x, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_subprob_count(const nfft_plan_s &p, int *counts, hipStream_t s) {
    hipLaunchKernelGGL(k_subprob_count, grid1d(p.geom.ntiles, 256), dim3(256), 0, s, p.key_start,
                       p.geom.ntiles, p.D, p.max_block_nodes, counts);
    return hipGetLastError();
}

hipError_t launch_subprob_fill(nfft_plan_s &p, const int *sub_start, hipStream_t s) {
    hipLaunchKernelGGL(k_subprob_fill, grid1d(p.geom.ntiles, 256), dim3(256), 0, s, p.key_start,
                       sub_start, p.geom.ntiles, p.D, p.max_block_nodes, p.subs);
    return hipGetLastError();
}

}  // namespace nfft
