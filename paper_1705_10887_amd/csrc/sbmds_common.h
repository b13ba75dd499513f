// Device-side helpers shared by the kernel sources: storage types, packed
// loads, per-mode type traits and the cross-block "last block reduces"
// completion protocol.
#pragma once

#include "sbmds_internal.h"

namespace sbmds {

// bfloat16 storage: the upper 16 bits of an IEEE float32.
struct bf16_t {
    uint16_t u;
};

__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h.u << 16); }

// float32 -> bfloat16, round to nearest even; NaN stays NaN.
__device__ __forceinline__ bf16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return bf16_t{(uint16_t)((u >> 16) | 0x40u)};
    u += 0x7fffu + ((u >> 16) & 1u);
    return bf16_t{(uint16_t)(u >> 16)};
}

template <typename TA, typename T>
__device__ __forceinline__ TA up(T x) { return (TA)x; }
template <>
__device__ __forceinline__ float up<float, bf16_t>(bf16_t x) { return bf2f(x); }
template <>
__device__ __forceinline__ double up<double, bf16_t>(bf16_t x) { return (double)bf2f(x); }

template <typename T, typename TA>
__device__ __forceinline__ T down(TA x) { return (T)x; }
template <>
__device__ __forceinline__ bf16_t down<bf16_t, float>(float x) { return f2bf(x); }

template <typename T, int N>
struct alignas(sizeof(T) * N) Pack {
    T v[N];
};

template <typename T, int N>
__device__ __forceinline__ Pack<T, N> ldp(const T *p) {
    return *reinterpret_cast<const Pack<T, N> *>(p);
}
template <typename T, int N>
__device__ __forceinline__ void stp(T *p, const Pack<T, N> &x) {
    *reinterpret_cast<Pack<T, N> *>(p) = x;
}

template <int M>
struct Traits;
template <>
struct Traits<MODE_BF16> {
    using TP = bf16_t; using TW = bf16_t; using TY = bf16_t; using TT = bf16_t;
    using TU = float;  using TA = float;
};
template <>
struct Traits<MODE_FP32> {
    using TP = float; using TW = float; using TY = float; using TT = float;
    using TU = float; using TA = float;
};
template <>
struct Traits<MODE_F64ACC> {
    using TP = float;  using TW = float;  using TY = double; using TT = double;
    using TU = double; using TA = double;
};
template <>
struct Traits<MODE_FP64> {
    using TP = double; using TW = double; using TY = double; using TT = double;
    using TU = double; using TA = double;
};

// Elements a lane moves per access: 16 bytes, but never more than the block.
template <typename T, int B>
struct VecOf {
    static constexpr int v = (16 / (int)sizeof(T)) < B ? (16 / (int)sizeof(T)) : B;
};

// Completion protocol for two-phase reductions: every block publishes its
// partial, then counts itself in; the block that arrives last reads all
// partials (in block order, so the result is deterministic) and resets the
// counter for the next launch.  Returns true in every thread of the last
// block.
__device__ __forceinline__ bool arrive_last(unsigned *counter, unsigned total) {
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = atomicAdd(counter, 1u);
        s_last = (prev == total - 1u);
    }
    __syncthreads();
    if (s_last) __threadfence();
    return s_last != 0;
}

__device__ __forceinline__ void tri_index(int ent, int B, int &a, int &b) {
    int r = ent, i = 0;
    while (r >= B - i) {
        r -= B - i;
        ++i;
    }
    a = i;
    b = i + r;
}

}  // namespace sbmds
