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

// Loads and stores through a pointer read out of device memory compile to
// flat instructions (the pointer is generic), which also count against the
// LDS wait counter; these access it as global memory.
template <int S>
struct UintOf;
template <>
struct UintOf<2> {
    using type = uint16_t;
};
template <>
struct UintOf<4> {
    using type = uint32_t;
};
template <>
struct UintOf<8> {
    using type = uint64_t;
};
template <typename T>
__device__ __forceinline__ T gld(const T *p) {
    using U = typename UintOf<(int)sizeof(T)>::type;
    const U u = *(const __attribute__((address_space(1))) U *)p;
    T r;
    __builtin_memcpy(&r, &u, sizeof(r));
    return r;
}

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
// Global-memory forms of ldp / stp (moved as whole dwords).
template <int W>
struct DwordVec {
    typedef uint32_t type __attribute__((ext_vector_type(W)));
};
template <>
struct DwordVec<1> {
    typedef uint32_t type;
};
template <typename T, int N>
__device__ __forceinline__ Pack<T, N> ldpg(const T *p) {
    static_assert(sizeof(T) * N % 4 == 0, "whole dwords");
    using V = typename DwordVec<(int)(sizeof(T) * N / 4)>::type;
    const V v = *(const __attribute__((address_space(1))) V *)p;
    Pack<T, N> r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}
template <typename T, int N>
__device__ __forceinline__ void stpg(T *p, const Pack<T, N> &x) {
    static_assert(sizeof(T) * N % 4 == 0, "whole dwords");
    using V = typename DwordVec<(int)(sizeof(T) * N / 4)>::type;
    V v;
    __builtin_memcpy(&v, &x, sizeof(v));
    *(__attribute__((address_space(1))) V *)p = v;
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

// Cross-block data inside one kernel.  gfx950 has one L2 per XCD and the L2s
// are not coherent with each other for ordinary device memory; a device-wide
// fence (__threadfence) therefore writes back and invalidates the whole L2,
// which is ruinous when hundreds of blocks do it.  Partial results that
// another block of the same launch reads are instead written and read with
// agent-scope atomic accesses (write-through / coherent loads, no cache
// maintenance), and completion is signalled with a relaxed counter atomic
// after the writer's stores have been acknowledged.
template <typename T>
__device__ __forceinline__ void st_coherent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_coherent(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Completion protocol for two-phase reductions: every block publishes its
// partial (st_coherent), then counts itself in; the block that arrives last
// reads all partials (ld_coherent, in block order, so the result is
// deterministic) and resets the counter for the next launch.  Returns true
// in every thread of the last block.
__device__ __forceinline__ bool arrive_last(unsigned *counter, unsigned total) {
    __shared__ int s_last;
    __builtin_amdgcn_s_waitcnt(0);  // this thread's coherent stores are acknowledged
    __syncthreads();                // ... and those of every thread in the block
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == total - 1u);
    }
    __syncthreads();
    return s_last != 0;
}

// Counter reset by the last block (the next launch starts from zero).
__device__ __forceinline__ void counter_reset(unsigned *counter) {
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Deterministic tree reduction across blocks.  `scratch` holds level 0 (the
// producers' partial vectors, [nparts][E], written with st_coherent)
// followed by the levels above it;
// `counters` holds one arrival counter per group of every level (all zero
// between launches).  A producer calls this after writing partial `p`; the
// last producer of each group of FAN partials sums that group (in index
// order) into the next level, and so on until a single group remains, whose
// sum goes to `out`.  Returns true in the block that wrote `out`.
template <int FAN>
__device__ bool tree_reduce(double *__restrict__ scratch, int E, int p, int nparts,
                            unsigned *__restrict__ counters, double *__restrict__ out) {
    double *src = scratch;
    unsigned *cnt = counters;
    int count = nparts, idx = p;
    for (;;) {
        const int ngroups = (count + FAN - 1) / FAN;
        const int g = idx / FAN;
        const int g0 = g * FAN;
        const int gs = min(FAN, count - g0);
        if (!arrive_last(cnt + g, (unsigned)gs)) return false;
        double *dst = (ngroups == 1) ? out : src + (size_t)count * E;
        for (int e = threadIdx.x; e < E; e += blockDim.x) {
            double acc[FAN];
#pragma unroll
            for (int q = 0; q < FAN; ++q) acc[q] = q < gs ? ld_coherent(src + (size_t)(g0 + q) * E + e) : 0.0;
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < FAN; ++q) s += acc[q];
            st_coherent(dst + (size_t)g * E + e, s);
        }
        if (threadIdx.x == 0) counter_reset(cnt + g);
        if (ngroups == 1) return true;
        src += (size_t)count * E;
        cnt += ngroups;
        count = ngroups;
        idx = g;
    }
}

// Sizes of the scratch / counter areas tree_reduce needs for nparts partials.
__host__ __device__ inline size_t tree_scratch_elems(int nparts, int E, int fan) {
    size_t tot = 0;
    int count = nparts;
    for (;;) {
        tot += (size_t)count * E;
        const int ng = (count + fan - 1) / fan;
        if (ng == 1) break;
        count = ng;
    }
    return tot;
}
__host__ __device__ inline int tree_counter_count(int nparts, int fan) {
    int tot = 0, count = nparts;
    for (;;) {
        const int ng = (count + fan - 1) / fan;
        tot += ng;
        if (ng == 1) break;
        count = ng;
    }
    return tot;
}

constexpr int kFan = 16;

// Problem that owns block `bid` of a batched launch: the largest p with
// off[p] <= bid (off is ascending, off[0] = 0).  Uniform across the block.
__device__ __forceinline__ int find_problem(const int *__restrict__ off, int nprob, int bid) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= bid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Workgroups are handed to the 8 XCDs of the device in turn (id mod 8).
// For the G blocks [a, a + G) of one problem, returns a local index in
// [0, G) such that each XCD gets a contiguous range of local indices (and so
// of the rows they stand for), in launch order within the XCD.
__device__ __forceinline__ int xcd_local_index(int g, int a, int G) {
    const int x = g & 7;
    int start = 0, first_x = 0;
#pragma unroll
    for (int xx = 0; xx < 8; ++xx) {
        const int first = a + ((xx - (a & 7)) + 8) % 8;  // first id >= a on XCD xx
        const int cnt = first >= a + G ? 0 : (a + G - 1 - first) / 8 + 1;
        if (xx < x) start += cnt;
        if (xx == x) first_x = first;
    }
    return start + (g - first_x) / 8;
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
