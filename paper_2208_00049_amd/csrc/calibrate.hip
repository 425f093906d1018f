// LDS operation rates of the device (a measurement aid behind
// nfft_calibrate_lds): the roof against which the spreading kernels'
// LDS atomics are reported.
//
// Each thread of a 256-thread workgroup performs `iters` operations on a
// 16 KiB LDS buffer at addresses given by the pattern (small enough that eight
// workgroups, 32 wavefronts, are resident per compute unit); the rate is the lane
// operations of all workgroups over the launch time.  Address arithmetic is a
// few VALU instructions per operation, far below the VALU issue rate, so the
// LDS unit bounds the loop.
#include <hip/hip_runtime.h>

#include "nfft_internal.hpp"

namespace nfft {
namespace {

constexpr int kCalThreads = 256;
constexpr int kCalBytes = 16384;

__device__ inline unsigned hash32(unsigned v) {
    v ^= v >> 16;
    v *= 0x7feb352dU;
    v ^= v >> 15;
    v *= 0x846ca68bU;
    v ^= v >> 16;
    return v;
}

// Word offset of this lane in its first operation (W words in the buffer).
//   pattern 0: consecutive words across the workgroup's lanes
//   pattern 1: an independent random word per lane
//   pattern 2: groups of 8 lanes on 8 consecutive words from a random start
//              (the access of one spreading instruction: eight nodes, each a
//              row of 2m = 8 consecutive cells)
__device__ inline unsigned first_word(int pattern, unsigned W, unsigned salt) {
    const unsigned t = threadIdx.x;
    if (pattern == 0) return t;
    if (pattern == 1) return hash32(t * 2654435761U + salt) & (W - 1);
    return ((hash32((t >> 3) * 2246822519U + salt) & (W - 1)) & ~7U) + (t & 7);
}

// OP 0: atomic add; 1: store; 2: load, add, store; 3: load (summed in registers, V a
// vector of 64-bit words for the wide loads)
template <typename V, int OP>
__global__ void __launch_bounds__(kCalThreads)
    k_lds_rate(int pattern, int iters, unsigned long long *sink) {
    __shared__ V buf[kCalBytes / sizeof(V)];
    constexpr unsigned W = kCalBytes / sizeof(V);
    if constexpr (OP == 3) {
        for (unsigned i = threadIdx.x; i < W; i += kCalThreads) buf[i] = V{i, i};
        __syncthreads();
        const unsigned off = first_word(pattern, W, blockIdx.x * 0x9e3779b9U);
        const unsigned step = pattern == 0 ? kCalThreads : 8u * 97u;
        unsigned long long s = 0;
        for (int k = 0; k < iters; k += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const V v = buf[(off + (unsigned)(k + u) * step) & (W - 1)];
                s += v.x + v.y;
            }
        }
        sink[(size_t)blockIdx.x * kCalThreads + threadIdx.x] = s;
        return;
    } else {
    for (unsigned i = threadIdx.x; i < W; i += kCalThreads) buf[i] = (V)0;
    __syncthreads();
    const unsigned off = first_word(pattern, W, blockIdx.x * 0x9e3779b9U);
    // successive operations of a lane move by one workgroup's width (pattern 0)
    // or by an odd stride (random patterns), wrapping in the buffer
    const unsigned step = pattern == 0 ? kCalThreads : 8u * 97u;
    for (int k = 0; k < iters; k += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const unsigned a = (off + (unsigned)(k + u) * step) & (W - 1);
            if constexpr (OP == 0) atomicAdd(&buf[a], (V)1);          // ds_add (integer / float)
            if constexpr (OP == 1) buf[a] = (V)(k + u);                // ds_write
            if constexpr (OP == 2) buf[a] = buf[a] + (V)1;             // read-modify-write
        }
    }
    __syncthreads();
    sink[(size_t)blockIdx.x * kCalThreads + threadIdx.x] =
        (unsigned long long)buf[(threadIdx.x * 37u) & (W - 1)];
    }
}

// an 8-byte load: one 64-bit word (the .y half reads as 0)
struct Word1 {
    unsigned long long x;
    static constexpr unsigned long long y = 0;
    __device__ Word1() = default;
    __device__ Word1(unsigned long long a, unsigned long long) : x(a) {}
};

template <typename V, int OP>
hipError_t time_rate(int pattern, int iters, int blocks, int reps, unsigned long long *sink,
                     hipStream_t s, float *ms) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    // one untimed launch (module load, clocks), then the timed ones
    if (e == hipSuccess) {
        hipLaunchKernelGGL((k_lds_rate<V, OP>), dim3(blocks), dim3(kCalThreads), 0, s, pattern,
                           iters, sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        hipLaunchKernelGGL((k_lds_rate<V, OP>), dim3(blocks), dim3(kCalThreads), 0, s, pattern,
                           iters, sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return e;
}

}  // namespace
}  // namespace nfft

extern "C" int nfft_calibrate_lds(int op, int pattern, int reps, void *stream,
                                  double *lane_ops_per_s) {
    using namespace nfft;
    if (op < 0 || op >= NFFT_LDS_OPS || pattern < 0 || pattern > 2 || reps < 1 ||
        !lane_ops_per_s)
        return NFFT_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return NFFT_ERR_HIP;
    const int blocks = 8 * (cus > 0 ? cus : 256);
    const int iters = 2048;
    unsigned long long *sink = nullptr;
    e = hipMalloc(&sink, (size_t)blocks * kCalThreads * sizeof(unsigned long long));
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? NFFT_ERR_NOMEM : NFFT_ERR_HIP;
    float ms = 0.f;
    switch (op) {
        case NFFT_LDS_ADD_U32: e = time_rate<unsigned, 0>(pattern, iters, blocks, reps, sink, s, &ms); break;
        case NFFT_LDS_ADD_U64: e = time_rate<unsigned long long, 0>(pattern, iters, blocks, reps, sink, s, &ms); break;
        case NFFT_LDS_ADD_F32: e = time_rate<float, 0>(pattern, iters, blocks, reps, sink, s, &ms); break;
        case NFFT_LDS_ADD_F64: e = time_rate<double, 0>(pattern, iters, blocks, reps, sink, s, &ms); break;
        case NFFT_LDS_WRITE_B64: e = time_rate<unsigned long long, 1>(pattern, iters, blocks, reps, sink, s, &ms); break;
        case NFFT_LDS_RMW_B64: e = time_rate<unsigned long long, 2>(pattern, iters, blocks, reps, sink, s, &ms); break;
        case NFFT_LDS_READ_B64: e = time_rate<Word1, 3>(pattern, iters, blocks, reps, sink, s, &ms); break;
        default: e = time_rate<ulonglong2, 3>(pattern, iters, blocks, reps, sink, s, &ms); break;
    }
    (void)hipFree(sink);
    if (e != hipSuccess) return NFFT_ERR_HIP;
    const double ops = (double)blocks * kCalThreads * iters * reps;
    *lane_ops_per_s = ms > 0.f ? ops / ((double)ms * 1e-3) : 0.0;
    return NFFT_OK;
}
