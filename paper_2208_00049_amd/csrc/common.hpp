// Device-side helpers shared by the libnfft kernels: complex arithmetic on
// float2/double2 and the per-type traits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nfft {

template <typename T> struct ctype;
template <> struct ctype<float> { using type = float2; };
template <> struct ctype<double> { using type = double2; };
template <typename T> using cplx = typename ctype<T>::type;

template <typename C> __host__ __device__ inline C cmake(decltype(C::x) re, decltype(C::x) im) {
    C v;
    v.x = re;
    v.y = im;
    return v;
}
template <typename C> __device__ inline C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ inline C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ inline C cmul(C a, C b) {
    return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __device__ inline C cmulc(C a, C b) {
    return cmake<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C, typename T> __device__ inline C cscale(C a, T s) { return cmake<C>(a.x * s, a.y * s); }
// multiply by s*i, s = +1 or -1
template <typename C> __device__ inline C cmul_si(C a, int s) {
    return s > 0 ? cmake<C>(-a.y, a.x) : cmake<C>(a.y, -a.x);
}

// Position on the oversampled axis of the r-th entry of the centred index set
// I_N (n = r - floor(N/2), also for odd N), i.e. (n mod Nt):
// r < floor(N/2) -> Nt - floor(N/2) + r, else r - floor(N/2).
__host__ __device__ inline int band_pos(int r, int N, int Nt) {
    return r < N / 2 ? Nt - N / 2 + r : r - N / 2;
}

constexpr int kNumXcd = 8;  // MI355X: 8 accelerator dies, each with its own L2

// Workgroups are dispatched round robin over the XCDs (block b runs on XCD b mod 8).
// Renumber them so that each XCD gets a contiguous run of logical blocks: blocks
// that share cache lines (neighbouring columns, neighbouring tiles) then share an L2.
__device__ inline int xcd_block(int b, int nblocks) {
    const int full = nblocks - nblocks % kNumXcd;
    if (b >= full) return b;
    return (b % kNumXcd) * (full / kNumXcd) + b / kNumXcd;
}

// q = n / d and r = n % d for 0 <= n < 2^22 and d >= 1, given rcp = 1/d in
// float: the float quotient is off by at most one, which one step corrects.
__device__ inline int small_divmod(int n, int d, float rcp, int &r) {
    int q = (int)((float)n * rcp);
    r = n - q * d;
    if (r < 0) {
        --q;
        r += d;
    } else if (r >= d) {
        ++q;
        r -= d;
    }
    return q;
}

// Add the value at offset off of padded tiles s0 .. s1-1 (the further work items
// of a split tile) to (sr, si), in item order.  Eight loads are issued before
// their additions: a dense tile has tens of items, and one load per round trip
// left the merge latency-bound (64-transform batch: merge pass 749 -> ? us).
template <typename T>
__device__ inline void add_split_items(T &sr, T &si, const cplx<T> *__restrict__ pad, int ptot,
                                       int off, int s0, int s1) {
    using C = cplx<T>;
    constexpr int U = 8;
    int s = s0;
    for (; s + U <= s1; s += U) {
        C w[U];
#pragma unroll
        for (int k = 0; k < U; ++k) w[k] = pad[(size_t)(s + k) * ptot + off];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            sr += w[k].x;
            si += w[k].y;
        }
    }
    for (; s < s1; ++s) {
        const C w = pad[(size_t)s * ptot + off];
        sr += w.x;
        si += w.y;
    }
}

}  // namespace nfft
