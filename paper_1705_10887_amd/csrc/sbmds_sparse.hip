// Sparse products with the interpolation operator and the n-space block
// kernels.
//
// The operator of Section 3.3 is applied as B X = -1/2 J P W P^T J X.  The
// two sparse factors are
//   k_spmm_t : T = (P^T Y - c e_x^T / n) C      (inner centering, basis rotation)
//   k_spmm   : Y' = P U - 1 s^T / n              (outer centering)
// where X = J Y C is the current orthonormal basis, c = P^T 1, e_x = 1^T Y and
// s = c^T U.  J = I - 1 1^T / n is never formed: both centerings are rank-one
// corrections (the paper notes J is identity plus rank one, Section 3.3).
//
// k_spmm additionally reduces the Gram matrix Y'^T Y' and the column sums
// 1^T Y' of the values it stores (after rounding to the storage type), so the
// next orthonormalisation needs no extra pass over Y'.
#include "sbmds_common.h"

namespace sbmds {

// ---------------------------------------------------------------------------
// Row-split SpMM with fused outer centering and Gram/column-sum epilogue.
// A row is handled by LPR lanes, each owning VEC consecutive columns of the
// block; a 256-thread block covers RPB rows per step and strides over rows.
// ---------------------------------------------------------------------------
template <int M, int B>
struct SpmmShape {
    using TY = typename Traits<M>::TY;
    static constexpr int VEC = VecOf<TY, B>::v;
    static constexpr int LPR = B / VEC;
    static constexpr int RPB = 256 / LPR;
    static constexpr int E = B * (B + 1) / 2;
    static constexpr int NQ = (E + 255) / 256;
};

template <int B>
__device__ __forceinline__ void gram_tile_accumulate(const double (*tile)[B], int rows, int tid,
                                                     const int *ea, const int *eb, int nq,
                                                     double *gacc, double &eacc) {
    for (int q = 0; q < nq; ++q) {
        if (ea[q] >= 0) {
            double s = 0.0;
            for (int r = 0; r < rows; ++r) s += tile[r][ea[q]] * tile[r][eb[q]];
            gacc[q] += s;
        }
    }
    if (tid < B) {
        double s = 0.0;
        for (int r = 0; r < rows; ++r) s += tile[r][tid];
        eacc += s;
    }
}

// Publish this block's Gram / column-sum partial and join the tree
// reduction whose result lands in st->Ge (packed triangle, then sums).
template <int B, int NQ>
__device__ __forceinline__ void gram_publish(const int *ea, const double *gacc, double eacc,
                                             double *__restrict__ red, unsigned *__restrict__ cnt,
                                             SolveState *__restrict__ st) {
    constexpr int E = B * (B + 1) / 2;
    constexpr int EG = E + B;
    const int tid = threadIdx.x;
    double *mine = red + (size_t)blockIdx.x * EG;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (ea[q] >= 0) st_coherent(mine + tid + q * 256, gacc[q]);
    if (tid < B) st_coherent(mine + E + tid, eacc);
    tree_reduce<kFan>(red, EG, blockIdx.x, gridDim.x, cnt, st->Ge);
}

template <int M, int B>
__global__ __launch_bounds__(256) void k_spmm(int n, const int32_t *__restrict__ rp,
                                              const int32_t *__restrict__ ci,
                                              const typename Traits<M>::TP *__restrict__ val,
                                              const typename Traits<M>::TU *__restrict__ U,
                                              SolveState *__restrict__ st, void *Y0, void *Y1, int phase,
                                              double *__restrict__ red, unsigned *__restrict__ cnt) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TY = typename Tr::TY;
    using TU = typename Tr::TU;
    using S = SpmmShape<M, B>;
    constexpr int VEC = S::VEC, LPR = S::LPR, RPB = S::RPB, E = S::E, NQ = S::NQ;
    __shared__ double tile[RPB][B];
    if (st->done || st->phase != phase) return;  // uniform: the schedule moved on
    TY *__restrict__ Y = (TY *)(st->ycur ? Y0 : Y1);  // writes the other buffer

    const int tid = threadIdx.x;
    const int g = tid % LPR;
    const int slot = tid / LPR;
    const double inv_n = 1.0 / (double)n;
    TA sc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) sc[v] = (TA)(st->Hs[B * B + g * VEC + v] * inv_n);

    int ea[NQ], eb[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        int ent = tid + q * 256;
        if (ent < E) tri_index(ent, B, ea[q], eb[q]);
        else ea[q] = eb[q] = -1;
    }
    double gacc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) gacc[q] = 0.0;
    double eacc = 0.0;

    for (int64_t base = (int64_t)blockIdx.x * RPB; base < n; base += (int64_t)gridDim.x * RPB) {
        const int64_t row = base + slot;
        if (row < n) {
            TA acc[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] = (TA)0;
            const int beg = rp[row], end = rp[row + 1];
            int e = beg;
            // two independent gathers in flight per lane
            for (; e + 1 < end; e += 2) {
                const int c0 = ci[e], c1 = ci[e + 1];
                const TA p0 = up<TA>(val[e]), p1 = up<TA>(val[e + 1]);
                Pack<TU, VEC> u0 = ldp<TU, VEC>(U + (size_t)c0 * B + g * VEC);
                Pack<TU, VEC> u1 = ldp<TU, VEC>(U + (size_t)c1 * B + g * VEC);
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[v] += p0 * up<TA>(u0.v[v]) + p1 * up<TA>(u1.v[v]);
            }
            if (e < end) {
                const int c0 = ci[e];
                const TA p0 = up<TA>(val[e]);
                Pack<TU, VEC> u0 = ldp<TU, VEC>(U + (size_t)c0 * B + g * VEC);
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[v] += p0 * up<TA>(u0.v[v]);
            }
            Pack<TY, VEC> o;
#pragma unroll
            for (int v = 0; v < VEC; ++v) o.v[v] = down<TY>(acc[v] - sc[v]);
            stp<TY, VEC>(Y + (size_t)row * B + g * VEC, o);
#pragma unroll
            for (int v = 0; v < VEC; ++v) tile[slot][g * VEC + v] = (double)up<TA>(o.v[v]);
        } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) tile[slot][g * VEC + v] = 0.0;
        }
        __syncthreads();
        gram_tile_accumulate<B>(tile, RPB, tid, ea, eb, NQ, gacc, eacc);
        __syncthreads();
    }
    gram_publish<B, NQ>(ea, gacc, eacc, red, cnt, st);
}

// Gram matrix and column sums of a stored block (start blocks).
template <int M, int B>
__global__ __launch_bounds__(256) void k_gram(int n, const typename Traits<M>::TY *__restrict__ Y,
                                              SolveState *__restrict__ st, double *__restrict__ red,
                                              unsigned *__restrict__ cnt) {
    using Tr = Traits<M>;
    using TY = typename Tr::TY;
    using S = SpmmShape<M, B>;
    constexpr int VEC = S::VEC, LPR = S::LPR, RPB = S::RPB, E = S::E, NQ = S::NQ;
    __shared__ double tile[RPB][B];
    const int tid = threadIdx.x;
    const int g = tid % LPR;
    const int slot = tid / LPR;
    int ea[NQ], eb[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        int ent = tid + q * 256;
        if (ent < E) tri_index(ent, B, ea[q], eb[q]);
        else ea[q] = eb[q] = -1;
    }
    double gacc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) gacc[q] = 0.0;
    double eacc = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * RPB; base < n; base += (int64_t)gridDim.x * RPB) {
        const int64_t row = base + slot;
        if (row < n) {
            Pack<TY, VEC> y = ldp<TY, VEC>(Y + (size_t)row * B + g * VEC);
#pragma unroll
            for (int v = 0; v < VEC; ++v) tile[slot][g * VEC + v] = (double)up<typename Tr::TA>(y.v[v]);
        } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) tile[slot][g * VEC + v] = 0.0;
        }
        __syncthreads();
        gram_tile_accumulate<B>(tile, RPB, tid, ea, eb, NQ, gacc, eacc);
        __syncthreads();
    }
    gram_publish<B, NQ>(ea, gacc, eacc, red, cnt, st);
}

// ---------------------------------------------------------------------------
// SpMM with the transposed operator (CSR of P^T), inner centering and the
// b x b basis rotation C.  WPR waves share one landmark row (its p + 1
// entries are split over them); a 256-thread block covers 4 / WPR rows.
// ---------------------------------------------------------------------------
template <int M, int B, int WPR>
__global__ __launch_bounds__(256) void k_spmm_t(int l, int n, const int32_t *__restrict__ rpT,
                                                const int32_t *__restrict__ ciT,
                                                const typename Traits<M>::TP *__restrict__ valT,
                                                const void *Y0, const void *Y1,
                                                const double *__restrict__ c,
                                                const SolveState *__restrict__ st, int phase,
                                                typename Traits<M>::TT *__restrict__ T) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TY = typename Tr::TY;
    using TT = typename Tr::TT;
    constexpr int VEC = VecOf<TY, B>::v;
    constexpr int LPR = B / VEC;
    constexpr int EPW = 64 / LPR;       // entries per wave step
    constexpr int RPBLK = 4 / WPR;      // landmark rows per block
    __shared__ double Cl[B * B];
    __shared__ double ex[B];
    __shared__ double part[4][B];       // per-wave partial sums
    __shared__ double rowbuf[RPBLK][B];
    if (st->done || st->phase != phase) return;
    const TY *__restrict__ Y = (const TY *)(st->ycur ? Y1 : Y0);

    const int tid = threadIdx.x;
    for (int i = tid; i < B * B; i += 256) Cl[i] = st->C[i];
    if (tid < B) ex[tid] = st->e_x[tid];

    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int g = lane % LPR;
    const int slot = lane / LPR;
    const int rloc = wave / WPR;        // row within the block
    const int wsub = wave % WPR;        // wave within the row
    const int64_t j = (int64_t)blockIdx.x * RPBLK + rloc;

    TA acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = (TA)0;
    if (j < l) {
        const int beg = rpT[j], end = rpT[j + 1];
        constexpr int STEP = EPW * WPR;
        int e = beg + wsub * EPW + slot;
        for (; e + STEP < end; e += 2 * STEP) {
            const TA p0 = up<TA>(valT[e]), p1 = up<TA>(valT[e + STEP]);
            const int v0 = ciT[e], v1 = ciT[e + STEP];
            Pack<TY, VEC> y0 = ldp<TY, VEC>(Y + (size_t)v0 * B + g * VEC);
            Pack<TY, VEC> y1 = ldp<TY, VEC>(Y + (size_t)v1 * B + g * VEC);
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] += p0 * up<TA>(y0.v[v]) + p1 * up<TA>(y1.v[v]);
        }
        if (e < end) {
            const TA p0 = up<TA>(valT[e]);
            const int v0 = ciT[e];
            Pack<TY, VEC> y0 = ldp<TY, VEC>(Y + (size_t)v0 * B + g * VEC);
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] += p0 * up<TA>(y0.v[v]);
        }
    }
#pragma unroll
    for (int m = LPR; m < 64; m <<= 1) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] += __shfl_xor(acc[v], m);
    }
    if (slot == 0) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) part[wave][g * VEC + v] = (double)acc[v];
    }
    __syncthreads();  // Cl, ex and the wave partials
    if (wsub == 0 && lane < B && j < l) {
        double r = 0.0;
#pragma unroll
        for (int q = 0; q < WPR; ++q) r += part[wave + q][lane];
        rowbuf[rloc][lane] = r - (c[j] / (double)n) * ex[lane];
    }
    __syncthreads();
    if (wsub == 0 && lane < B && j < l) {
        double t = 0.0;
#pragma unroll 8
        for (int i = 0; i < B; ++i) t += rowbuf[rloc][i] * Cl[i * B + lane];
        T[(size_t)j * B + lane] = down<TT>((TA)t);
    }
}

// ---------------------------------------------------------------------------
// Start blocks, precision changes and outputs.
// ---------------------------------------------------------------------------

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): counter = (row, column, 0, 0), key = seed.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * c[0];
        uint64_t p1 = (uint64_t)M1 * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

// Standard normal from two uniforms in (0, 1] (Box-Muller, float32: the
// start block needs no precision).
__device__ __forceinline__ float gauss_from(uint32_t a, uint32_t b) {
    const float u1 = ((float)(a >> 8) + 1.0f) * (1.0f / 16777216.0f);
    const float u2 = (float)(b >> 8) * (1.0f / 16777216.0f);
    return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

// Start block into buffer 0; columns >= b are zero.  Counter (row, column).
template <int M, int B>
__global__ __launch_bounds__(256) void k_random_block(int n, int b, uint64_t seed,
                                                      typename Traits<M>::TY *__restrict__ Y) {
    using TY = typename Traits<M>::TY;
    using TA = typename Traits<M>::TA;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n * B) return;
    const int64_t row = idx / B;
    const int col = (int)(idx % B);
    float z = 0.0f;
    if (col < b) {
        uint32_t ctr[4] = {(uint32_t)row, (uint32_t)col, (uint32_t)(row >> 32), 0u};
        philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
        z = gauss_from(ctr[0], ctr[1]);
    }
    Y[idx] = down<TY>((TA)z);
}

template <typename TS, int M, int B>
__global__ __launch_bounds__(256) void k_load_block(int n, int b, const TS *__restrict__ X0,
                                                    typename Traits<M>::TY *__restrict__ Y) {
    using TY = typename Traits<M>::TY;
    using TA = typename Traits<M>::TA;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n * B) return;
    const int64_t row = idx / B;
    const int col = (int)(idx % B);
    TA v = col < b ? (TA)X0[row * b + col] : (TA)0;
    Y[idx] = down<TY>(v);
}

// Precision change at the start of phase `phase`: the current block is
// copied into the other buffer in the new storage type (widening, so
// exact).  Runs only when the previous phase has just ended.
template <int MF, int MT>
__global__ __launch_bounds__(256) void k_convert(int64_t count, const void *Y0, const void *Y1, void *W0, void *W1,
                                                 const SolveState *__restrict__ st, int phase) {
    if (st->done || st->phase != phase || !st->pending_convert) return;
    using TAt = typename Traits<MT>::TA;
    using TYt = typename Traits<MT>::TY;
    const typename Traits<MF>::TY *src = (const typename Traits<MF>::TY *)(st->ycur ? Y1 : Y0);
    TYt *dst = (TYt *)(st->ycur ? W0 : W1);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) dst[i] = down<TYt>((TAt)up<double>(src[i]));
}

// After the conversion: the other buffer is now current.
__global__ void k_phase_begin(SolveState *__restrict__ st, int phase, int mode) {
    if (threadIdx.x == 0 && !st->done && st->phase == phase && st->pending_convert) {
        st->ycur ^= 1;
        st->ymode = mode;
        st->pending_convert = 0;
    }
}

// Z = J Y Zmap restricted to the first k columns: Z_ij = sum_a Y_ia Zmap_aj - zshift_j.
template <int M, int B, typename TZ>
__global__ __launch_bounds__(256) void k_embedding(int n, int k, const typename Traits<M>::TY *__restrict__ Y,
                                                   const SolveState *__restrict__ st, TZ *__restrict__ Z) {
    __shared__ double Zm[B * B];
    __shared__ double zs[B];
    for (int i = threadIdx.x; i < B * B; i += 256) Zm[i] = st->Zmap[i];
    if (threadIdx.x < B) zs[threadIdx.x] = st->zshift[threadIdx.x];
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= n) return;
    double y[B];
#pragma unroll
    for (int a = 0; a < B; ++a) y[a] = up<double>(Y[row * B + a]);
    for (int j = 0; j < k; ++j) {
        double z = -zs[j];
#pragma unroll
        for (int a = 0; a < B; ++a) z += y[a] * Zm[a * B + j];
        Z[row * k + j] = (TZ)z;
    }
}

// X = J Y C (the current orthonormal basis), first b columns.
template <int M, int B, typename TX>
__global__ __launch_bounds__(256) void k_block_out(int n, int b, const typename Traits<M>::TY *__restrict__ Y,
                                                   const SolveState *__restrict__ st, TX *__restrict__ X) {
    __shared__ double Cl[B * B];
    __shared__ double sh[B];
    for (int i = threadIdx.x; i < B * B; i += 256) Cl[i] = st->C[i];
    __syncthreads();
    if (threadIdx.x < B) {
        double s = 0.0;
        for (int a = 0; a < B; ++a) s += st->e_x[a] * Cl[a * B + threadIdx.x];
        sh[threadIdx.x] = s / (double)n;
    }
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= n) return;
    double y[B];
#pragma unroll
    for (int a = 0; a < B; ++a) y[a] = up<double>(Y[row * B + a]);
    for (int j = 0; j < b; ++j) {
        double x = -sh[j];
#pragma unroll
        for (int a = 0; a < B; ++a) x += y[a] * Cl[a * B + j];
        X[row * b + j] = (TX)x;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int M>
static size_t val_bytes() { return sizeof(typename Traits<M>::TP); }

#define SBMDS_DISPATCH_B(B_, CALL)                      \
    switch (B_) {                                       \
        case 4: { constexpr int BB = 4; CALL; } break;   \
        case 8: { constexpr int BB = 8; CALL; } break;   \
        case 16: { constexpr int BB = 16; CALL; } break; \
        case 32: { constexpr int BB = 32; CALL; } break; \
        case 64: { constexpr int BB = 64; CALL; } break; \
        default: return hipErrorInvalidValue;           \
    }

#define SBMDS_DISPATCH_M(M_, CALL)                                 \
    switch (M_) {                                                  \
        case MODE_BF16: { constexpr int MM = MODE_BF16; CALL; } break;     \
        case MODE_FP32: { constexpr int MM = MODE_FP32; CALL; } break;     \
        case MODE_F64ACC: { constexpr int MM = MODE_F64ACC; CALL; } break; \
        case MODE_FP64: { constexpr int MM = MODE_FP64; CALL; } break;     \
        default: return hipErrorInvalidValue;                      \
    }

template <int MM, int BB>
static hipError_t spmm_impl(const DevProblem &p, const LaunchCfg &cfg, int phase, hipStream_t s) {
    using Tr = Traits<MM>;
    const int grid = cfg.spmm_blocks;
    if (grid <= 0 || grid > p.max_spmm_blocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_spmm<MM, BB>), dim3(grid), dim3(256), 0, s, (int)p.n, p.rp, p.ci,
                       (const typename Tr::TP *)p.val[MM], (const typename Tr::TU *)p.U, p.st, p.Y[0], p.Y[1],
                       phase, p.red_spmm, p.spmm_cnt);
    return hipGetLastError();
}

hipError_t launch_spmm(Mode m, const DevProblem &p, const LaunchCfg &cfg, int phase, hipStream_t s) {
    SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(p.B, return (spmm_impl<MM, BB>(p, cfg, phase, s))));
    return hipErrorInvalidValue;
}

template <int MM, int BB, int WPR>
static hipError_t spmm_t_impl(const DevProblem &p, int phase, hipStream_t s) {
    using Tr = Traits<MM>;
    constexpr int RPBLK = 4 / WPR;
    const int grid = (int)((p.l + RPBLK - 1) / RPBLK);
    hipLaunchKernelGGL((k_spmm_t<MM, BB, WPR>), dim3(grid), dim3(256), 0, s, (int)p.l, (int)p.n, p.rpT, p.ciT,
                       (const typename Tr::TP *)p.valT[MM], (const void *)p.Y[0], (const void *)p.Y[1], p.c[MM],
                       p.st, phase, (typename Tr::TT *)p.T);
    return hipGetLastError();
}

hipError_t launch_spmm_t(Mode m, const DevProblem &p, const LaunchCfg &cfg, int phase, hipStream_t s) {
    switch (cfg.spmmt_wpr) {
        case 1: SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(p.B, return (spmm_t_impl<MM, BB, 1>(p, phase, s)))); break;
        case 2: SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(p.B, return (spmm_t_impl<MM, BB, 2>(p, phase, s)))); break;
        case 4: SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(p.B, return (spmm_t_impl<MM, BB, 4>(p, phase, s)))); break;
        default: return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

template <int MM, int BB>
static hipError_t start_impl(const DevProblem &p, const LaunchCfg &cfg, uint64_t seed, const void *X0,
                             hipStream_t s) {
    using Tr = Traits<MM>;
    const int64_t count = p.n * (int64_t)BB;
    const int g1 = (int)((count + 255) / 256);
    if (X0 == nullptr) {
        hipLaunchKernelGGL((k_random_block<MM, BB>), dim3(g1), dim3(256), 0, s, (int)p.n, p.b, seed,
                           (typename Tr::TY *)p.Y[0]);
    } else if (MM == MODE_FP64) {
        hipLaunchKernelGGL((k_load_block<double, MM, BB>), dim3(g1), dim3(256), 0, s, (int)p.n, p.b,
                           (const double *)X0, (typename Tr::TY *)p.Y[0]);
    } else {
        hipLaunchKernelGGL((k_load_block<float, MM, BB>), dim3(g1), dim3(256), 0, s, (int)p.n, p.b,
                           (const float *)X0, (typename Tr::TY *)p.Y[0]);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int grid = cfg.spmm_blocks;
    if (grid <= 0 || grid > p.max_spmm_blocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_gram<MM, BB>), dim3(grid), dim3(256), 0, s, (int)p.n,
                       (const typename Tr::TY *)p.Y[0], p.st, p.red_spmm, p.spmm_cnt);
    return hipGetLastError();
}

hipError_t launch_random_start(Mode m, const DevProblem &p, const LaunchCfg &cfg, uint64_t seed, hipStream_t s) {
    SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(p.B, return (start_impl<MM, BB>(p, cfg, seed, nullptr, s))));
    return hipErrorInvalidValue;
}

hipError_t launch_user_start(Mode m, const DevProblem &p, const LaunchCfg &cfg, const void *X0, hipStream_t s) {
    if (X0 == nullptr) return hipErrorInvalidValue;
    SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(p.B, return (start_impl<MM, BB>(p, cfg, 0, X0, s))));
    return hipErrorInvalidValue;
}

template <int MF, int MT>
static hipError_t convert_impl(const DevProblem &p, int phase, hipStream_t s) {
    const int64_t count = p.n * (int64_t)p.B;
    hipLaunchKernelGGL((k_convert<MF, MT>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count,
                       (const void *)p.Y[0], (const void *)p.Y[1], p.Y[0], p.Y[1], (const SolveState *)p.st,
                       phase);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_phase_begin, dim3(1), dim3(64), 0, s, p.st, phase, MT);
    return hipGetLastError();
}

hipError_t launch_convert_y(Mode from, Mode to, const DevProblem &p, int phase, hipStream_t s) {
    switch (from) {
        case MODE_BF16: {
            constexpr int MF = MODE_BF16;
            SBMDS_DISPATCH_M(to, return (convert_impl<MF, MM>(p, phase, s)));
        } break;
        case MODE_FP32: {
            constexpr int MF = MODE_FP32;
            SBMDS_DISPATCH_M(to, return (convert_impl<MF, MM>(p, phase, s)));
        } break;
        case MODE_F64ACC: {
            constexpr int MF = MODE_F64ACC;
            SBMDS_DISPATCH_M(to, return (convert_impl<MF, MM>(p, phase, s)));
        } break;
        case MODE_FP64: {
            constexpr int MF = MODE_FP64;
            SBMDS_DISPATCH_M(to, return (convert_impl<MF, MM>(p, phase, s)));
        } break;
        default: return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

template <int MM, int BB>
static hipError_t embedding_impl(const DevProblem &p, int ybuf, void *Z, int z_double, hipStream_t s) {
    using Tr = Traits<MM>;
    const unsigned grid = (unsigned)((p.n + 255) / 256);
    if (z_double)
        hipLaunchKernelGGL((k_embedding<MM, BB, double>), dim3(grid), dim3(256), 0, s, (int)p.n, p.k,
                           (const typename Tr::TY *)p.Y[ybuf], p.st, (double *)Z);
    else
        hipLaunchKernelGGL((k_embedding<MM, BB, float>), dim3(grid), dim3(256), 0, s, (int)p.n, p.k,
                           (const typename Tr::TY *)p.Y[ybuf], p.st, (float *)Z);
    return hipGetLastError();
}

hipError_t launch_embedding(Mode m, const DevProblem &p, int ybuf, void *Z, int z_double, hipStream_t s) {
    SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(p.B, return (embedding_impl<MM, BB>(p, ybuf, Z, z_double, s))));
    return hipErrorInvalidValue;
}

template <int MM, int BB>
static hipError_t block_out_impl(const DevProblem &p, int ybuf, void *X, int x_double, hipStream_t s) {
    using Tr = Traits<MM>;
    const unsigned grid = (unsigned)((p.n + 255) / 256);
    if (x_double)
        hipLaunchKernelGGL((k_block_out<MM, BB, double>), dim3(grid), dim3(256), 0, s, (int)p.n, p.b,
                           (const typename Tr::TY *)p.Y[ybuf], p.st, (double *)X);
    else
        hipLaunchKernelGGL((k_block_out<MM, BB, float>), dim3(grid), dim3(256), 0, s, (int)p.n, p.b,
                           (const typename Tr::TY *)p.Y[ybuf], p.st, (float *)X);
    return hipGetLastError();
}

hipError_t launch_block_out(Mode m, const DevProblem &p, int ybuf, void *X, int x_double, hipStream_t s) {
    SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(p.B, return (block_out_impl<MM, BB>(p, ybuf, X, x_double, s))));
    return hipErrorInvalidValue;
}

static double idx_val_bytes(Mode m) {
    return 4.0 + (m == MODE_BF16 ? 2.0 : (m == MODE_FP64 ? 8.0 : 4.0));
}
static double u_bytes(Mode m) { return m == MODE_F64ACC || m == MODE_FP64 ? 8.0 : 4.0; }

double spmm_bytes(Mode m, const DevProblem &p) {
    // CSR stream + row pointers + one write of Y' + one read of U
    return (double)p.nnz * idx_val_bytes(m) + 4.0 * (p.n + 1) + (double)p.n * p.B * y_elem_bytes(m) +
           (double)p.l * p.B * u_bytes(m);
}
double spmm_t_bytes(Mode m, const DevProblem &p) {
    // CSR(P^T) stream + row pointers + one read of Y + one write of T
    return (double)p.nnz * idx_val_bytes(m) + 4.0 * (p.l + 1) + (double)p.n * p.B * y_elem_bytes(m) +
           (double)p.l * p.B * y_elem_bytes(m);
}

}  // namespace sbmds

namespace sbmds {

__global__ __launch_bounds__(256) void k_f32_to_bf16(int64_t count, const float *__restrict__ src,
                                                     bf16_t *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) dst[i] = f2bf(src[i]);
}

hipError_t launch_f32_to_bf16(const float *src, void *dst, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, src,
                       (bf16_t *)dst);
    return hipGetLastError();
}

}  // namespace sbmds
