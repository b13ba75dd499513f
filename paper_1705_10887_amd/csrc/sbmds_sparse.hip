// Sparse products with the interpolation operator and the n-space block
// kernels, batched over every problem of a context.
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
//
// Every launch covers all problems of a batch: block b belongs to the
// problem p with off[p] <= b < off[p+1] and works on that problem's local
// block b - off[p] of off[p+1] - off[p].  A problem whose schedule is not in
// the launch's phase returns at once.
#include <type_traits>

#include "sbmds_common.h"
#include "sbmds_prep.h"
#include "sbmds_rr.h"

namespace sbmds {

template <int M, int B>
struct SpmmShape {
    using TY = typename Traits<M>::TY;
    static constexpr int VEC = VecOf<TY, B>::v;
    static constexpr int LPR = B / VEC;
    static constexpr int RPB = 256 / LPR;
    static constexpr int E = B * (B + 1) / 2;
    static constexpr int NQ = (E + 255) / 256;
};

// Widths served by the 1024-thread SpMM with the matrix-core Gram (B = 8 as
// one 16 x 16 tile with zero padding).
constexpr bool wide_width(int B) { return B == 8 || B == 16 || B == 32; }

int spmm_rows_per_block(Mode m, int B) {
    const int ysz = y_elem_bytes(m);
    int vec = 16 / ysz;
    if (vec > B) vec = B;
    const int lpr = B / vec;
    return (wide_width(B) ? 1024 : 256) / lpr;
}

int spmm_block_cap(Mode, int B) { return wide_width(B) ? 256 : 1024; }

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
                                             SolveState *__restrict__ st, int vb, int vg) {
    constexpr int E = B * (B + 1) / 2;
    constexpr int EG = E + B;
    const int tid = threadIdx.x;
    double *mine = red + (size_t)vb * EG;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (ea[q] >= 0) st_coherent(mine + tid + q * 256, gacc[q]);
    if (tid < B) st_coherent(mine + E + tid, eacc);
    tree_reduce<kFan>(red, EG, vb, vg, cnt, st->Ge);
}

// ---------------------------------------------------------------------------
// Row-split SpMM with fused outer centering and Gram/column-sum epilogue.
// A row is handled by LPR lanes, each owning VEC consecutive columns of the
// block; a 256-thread block covers RPB rows per step and strides over rows.
// ---------------------------------------------------------------------------
template <int M, int B>
__global__ __launch_bounds__(256) void k_spmm(const ProbView *__restrict__ views, const int *__restrict__ off,
                                              int nprob, int phase) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TY = typename Tr::TY;
    using TU = typename Tr::TU;
    using TP = typename Tr::TP;
    using S = SpmmShape<M, B>;
    constexpr int VEC = S::VEC, LPR = S::LPR, RPB = S::RPB, E = S::E, NQ = S::NQ;
    __shared__ double tile[RPB][B];

    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    SolveState *__restrict__ st = v.st;
    if (st->done || st->phase != phase) return;  // uniform: the schedule moved on
    const int vb = blockIdx.x - off[p], vg = off[p + 1] - off[p];
    const int n = v.n;
    const int32_t *__restrict__ rp = v.rp;
    const int32_t *__restrict__ ci = v.ci;
    const TP *__restrict__ val = (const TP *)v.val[M];
    const TU *__restrict__ U = (const TU *)v.U;
    TY *__restrict__ Y = (TY *)(st->ycur ? v.Y0 : v.Y1);  // writes the other buffer

    const int tid = threadIdx.x;
    const int g = tid % LPR;
    const int slot = tid / LPR;
    const double inv_n = 1.0 / (double)n;
    TA sc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) sc[q] = (TA)(st->Hs[B * B + g * VEC + q] * inv_n);

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

    // row bounds one step ahead; a row's entries CH at a time with all
    // their index, value and U loads in flight (as in k_spmm_wide)
    constexpr int CH = (M == MODE_FP32 || M == MODE_BF16) ? 16 : 8;
    const int64_t stride = (int64_t)vg * RPB;
    int beg_next = 0, end_next = 0;
    if ((int64_t)vb * RPB + slot < n) {
        beg_next = rp[(int64_t)vb * RPB + slot];
        end_next = rp[(int64_t)vb * RPB + slot + 1];
    }
    for (int64_t base = (int64_t)vb * RPB; base < n; base += stride) {
        const int64_t row = base + slot;
        const int beg = beg_next, end = end_next;
        if (row + stride < n) {
            beg_next = rp[row + stride];
            end_next = rp[row + stride + 1];
        }
        if (row < n) {
            TA acc[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = (TA)0;
            for (int e0 = beg; e0 < end; e0 += CH) {
                int c[CH];
                TA pv[CH];
#pragma unroll
                for (int j = 0; j < CH; ++j) {
                    const bool ok = e0 + j < end;
                    c[j] = ok ? ci[e0 + j] : 0;  // row 0 of U stands in for missing entries
                    pv[j] = ok ? up<TA>(val[e0 + j]) : (TA)0;
                }
                Pack<TU, VEC> u[CH];
#pragma unroll
                for (int j = 0; j < CH; ++j) u[j] = ldp<TU, VEC>(U + (size_t)c[j] * B + g * VEC);
#pragma unroll
                for (int j = 0; j < CH; ++j) {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) acc[q] += pv[j] * up<TA>(u[j].v[q]);
                }
            }
            Pack<TY, VEC> o;
#pragma unroll
            for (int q = 0; q < VEC; ++q) o.v[q] = down<TY>(acc[q] - sc[q]);
            stp<TY, VEC>(Y + (size_t)row * B + g * VEC, o);
#pragma unroll
            for (int q = 0; q < VEC; ++q) tile[slot][g * VEC + q] = (double)up<TA>(o.v[q]);
        } else {
#pragma unroll
            for (int q = 0; q < VEC; ++q) tile[slot][g * VEC + q] = 0.0;
        }
        __syncthreads();
        gram_tile_accumulate<B>(tile, RPB, tid, ea, eb, NQ, gacc, eacc);
        __syncthreads();
    }
    gram_publish<B, NQ>(ea, gacc, eacc, v.red_spmm, v.spmm_cnt, st, vb, vg);
}

// Gram matrix and column sums of a block already written to buffer 0 (the
// start block), same tiling as k_spmm.
template <int M, int B>
__global__ __launch_bounds__(256) void k_gram(const ProbView *__restrict__ views, const int *__restrict__ off,
                                              int nprob, int only_refill) {
    using Tr = Traits<M>;
    using TY = typename Tr::TY;
    using S = SpmmShape<M, B>;
    constexpr int VEC = S::VEC, LPR = S::LPR, RPB = S::RPB, E = S::E, NQ = S::NQ;
    __shared__ double tile[RPB][B];
    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    if (only_refill && !v.st->refill) return;  // uniform per problem
    const int vb = blockIdx.x - off[p], vg = off[p + 1] - off[p];
    const int n = v.n;
    const TY *__restrict__ Y = (const TY *)v.Y0;
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
    for (int64_t base = (int64_t)vb * RPB; base < n; base += (int64_t)vg * RPB) {
        const int64_t row = base + slot;
        if (row < n) {
            Pack<TY, VEC> y = ldp<TY, VEC>(Y + (size_t)row * B + g * VEC);
#pragma unroll
            for (int q = 0; q < VEC; ++q) tile[slot][g * VEC + q] = (double)up<typename Tr::TA>(y.v[q]);
        } else {
#pragma unroll
            for (int q = 0; q < VEC; ++q) tile[slot][g * VEC + q] = 0.0;
        }
        __syncthreads();
        gram_tile_accumulate<B>(tile, RPB, tid, ea, eb, NQ, gacc, eacc);
        __syncthreads();
    }
    gram_publish<B, NQ>(ea, gacc, eacc, v.red_spmm, v.spmm_cnt, v.st, vb, vg);
}

// ---------------------------------------------------------------------------
// Wide-block variant for B in {16, 32}: 1024-thread blocks (so the Gram
// partials of a launch are few and their tree shallow), the CSR entries of
// a block step staged in LDS with coalesced loads, and the float64 Gram
// Y'^T Y' accumulated with v_mfma_f64_16x16x4f64 on 16 x 16 tiles of it.
//
// MFMA operand layout (16 x 16 x 4, float64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and holds D[l/16 + 4r][l%16] in element r.  With both
// A^T and B the same 4 x 16 row block of Y', lane l supplies
// Y'[4 k + l/16][16 t + l%16] for tile column t.
// ---------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kWideThreads = 1024;
constexpr int kWideChunk = 16;   // CSR entries of a row whose loads are in flight together
constexpr int kSpmmTChunk = 4;   // entries per lane of a landmark row loaded together (SpMM^T)

template <int M, int B>
struct WideShape {
    using TY = typename Traits<M>::TY;
    using TP = typename Traits<M>::TP;
    static constexpr int VEC = VecOf<TY, B>::v;
    static constexpr int LPR = B / VEC;
    static constexpr int RPB = kWideThreads / LPR;  // rows per block step
    static constexpr int RW = 64 / LPR;             // rows per wave step
    static constexpr int NTB = (B + 15) / 16;  // 16 x 16 Gram tiles per side (B = 8: one, padded)
    static constexpr int TILES = NTB * (NTB + 1) / 2;
    static constexpr int E = B * (B + 1) / 2;
    static constexpr int EG = E + B;
    static constexpr int NW = kWideThreads / 64;
    static constexpr int WREG = 512;                                     // LDS doubles per wave (4 KB)
    static constexpr int CAPW = (int)(WREG * 8 / (4 + sizeof(TP)));      // CSR entries a wave stages
    static_assert(RW * B <= WREG, "a wave's tile rows fit its region");
    static constexpr int TILE_D = NW * WREG;
    static constexpr int RED_D = NW * EG;
    static constexpr int RR_D = (int)((sizeof(RRLds<B>) + 7) / 8);  // the Rayleigh-Ritz step's LDS
    static constexpr int SMEM_D0 = TILE_D > RED_D ? TILE_D : RED_D;
    static constexpr int SMEM_D = SMEM_D0 > RR_D ? SMEM_D0 : RR_D;
};

// Gram and column sums of the wave's RW rows of the tile.
template <int B, int RW, int TILES>
__device__ __forceinline__ void gram_mfma_rows(const double *__restrict__ tile, int r0, dbl4 (&acc)[TILES],
                                               double (&esum)[(B + 15) / 16]) {
    constexpr int NTB = (B + 15) / 16;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kr = lane >> 4;
#pragma unroll
    for (int ks = 0; ks < RW / 4; ++ks) {
        const double *row = tile + (size_t)(r0 + 4 * ks + kr) * B;
        double v[NTB];
#pragma unroll
        for (int ti = 0; ti < NTB; ++ti) v[ti] = (16 * ti + col < B) ? row[16 * ti + col] : 0.0;
        int t = 0;
#pragma unroll
        for (int ti = 0; ti < NTB; ++ti) {
#pragma unroll
            for (int tj = ti; tj < NTB; ++tj) {
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[ti], v[tj], acc[t], 0, 0, 0);
                ++t;
            }
        }
#pragma unroll
        for (int ti = 0; ti < NTB; ++ti) esum[ti] += v[ti];
    }
}

// Sum the waves' Gram tiles (fixed order) into this block's partial and
// join the tree reduction into st->Ge.  `smem` must be free (all waves past
// their last use of it).
template <int M, int B, int TILES>
__device__ __forceinline__ bool gram_mfma_finish(dbl4 (&acc)[TILES], double (&esum)[(B + 15) / 16],
                                                 double *__restrict__ smem, double *__restrict__ red,
                                                 unsigned *__restrict__ cnt, SolveState *__restrict__ st, int vb,
                                                 int vg) {
    using S = WideShape<M, B>;
    constexpr int NTB = S::NTB, E = S::E, EG = S::EG, NW = S::NW;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int ti = 0; ti < NTB; ++ti) {
        esum[ti] += __shfl_xor(esum[ti], 16);
        esum[ti] += __shfl_xor(esum[ti], 32);
    }
    double *mine = smem + (size_t)w * EG;
    int t = 0;
#pragma unroll
    for (int ti = 0; ti < NTB; ++ti) {
#pragma unroll
        for (int tj = ti; tj < NTB; ++tj) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * ti + (lane >> 4) + 4 * r, j = 16 * tj + (lane & 15);
                if (i <= j && j < B) mine[i * B - (i * (i - 1)) / 2 + (j - i)] = acc[t][r];
            }
            ++t;
        }
    }
    if (lane < 16) {
#pragma unroll
        for (int ti = 0; ti < NTB; ++ti)
            if (16 * ti + lane < B) mine[E + 16 * ti + lane] = esum[ti];
    }
    __syncthreads();
    double *part = red + (size_t)vb * EG;
    for (int e = tid; e < EG; e += kWideThreads) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) s += smem[(size_t)q * EG + e];
        st_coherent(part + e, s);
    }
    return tree_reduce<kFan>(red, EG, vb, vg, cnt, st->Ge);
}

// rr: 0 = no Rayleigh-Ritz step, 1 = the iteration's step, 2 = the start's
// CholQR (init mode); it runs in the block that completes the Gram
// reduction of its problem.
// ULDS: the whole l x B block U is first copied to LDS (every 16-byte piece
// load in flight at once) and the row gathers read it there, one global
// round trip less per row step; for launches where l B sizeof(U) fits
// kUldsBytes.
constexpr int kUldsBytes = 64 * 1024;

// WPE: waves per SIMD the register budget is sized for.  4 (one block per
// CU) leaves room for the fused Rayleigh-Ritz step; 8 (two blocks per CU,
// 64 registers, no U copy and no fused step) keeps twice the row steps in
// flight, for launches that move enough bytes to be bandwidth bound.
template <int M, int B, bool ULDS, int WPE = 4>
__global__ __launch_bounds__(kWideThreads, WPE) void k_spmm_wide(const ProbView *__restrict__ views,
                                                            const int *__restrict__ off, int nprob, int phase, int rr,
                                                            int b, int k, int max_sweeps, PhaseRule rule) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TY = typename Tr::TY;
    using TU = typename Tr::TU;
    using TP = typename Tr::TP;
    using S = WideShape<M, B>;
    constexpr int VEC = S::VEC, LPR = S::LPR, RPB = S::RPB, RW = S::RW, TILES = S::TILES, NTB = S::NTB;
    // entries in flight per lane: as many as the register budget of the
    // mode and width allows without spilling
    // (gathers from LDS need fewer in flight)
    static_assert(WPE == 4 || (WPE == 8 && !ULDS), "the two-block form keeps U in global memory");
    constexpr int CH = WPE == 8 ? kWideChunk / 4
                     : ULDS   ? kWideChunk / 2
                            : ((M == MODE_FP32 && B <= 16) ? kWideChunk
                                                           : ((M == MODE_BF16 && B >= 32) ? kWideChunk / 4
                                                                                          : kWideChunk / 2));
    __shared__ __attribute__((aligned(16))) double smem[S::SMEM_D];

    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    SolveState *__restrict__ st = v.st;
    if (st->done || st->phase != phase) return;  // uniform: the schedule moved on
    const int vb = blockIdx.x - off[p], vg = off[p + 1] - off[p];
    const int n = v.n;
    const int32_t *__restrict__ rp = v.rp;
    const int32_t *__restrict__ ci = v.ci;
    const TP *__restrict__ val = (const TP *)v.val[M];
    const TU *__restrict__ U = (const TU *)v.U;
    TY *__restrict__ Y = (TY *)(st->ycur ? v.Y0 : v.Y1);  // writes the other buffer

    const int tid = threadIdx.x;
    const TU *__restrict__ Ug = U;  // where the gathers read: global U, or its copy in LDS
    if constexpr (ULDS) {
        static_assert(16 % sizeof(TU) == 0 && (B * sizeof(TU)) % 16 == 0, "whole 16-byte pieces per row");
        constexpr int NPC = kUldsBytes / 16 / kWideThreads;  // pieces per thread
        __shared__ __attribute__((aligned(16))) Pack<TU, 16 / sizeof(TU)> Us[kUldsBytes / 16];
        const int pieces = (int)((size_t)v.l * B * sizeof(TU) / 16);  // <= kUldsBytes / 16 (checked at launch)
        using PU = Pack<TU, 16 / sizeof(TU)>;
        PU tmp[NPC];
#pragma unroll
        for (int q = 0; q < NPC; ++q) {
            const int i = tid + q * kWideThreads;
            if (i < pieces) tmp[q] = ldpg<TU, 16 / sizeof(TU)>(U + (size_t)i * (16 / sizeof(TU)));
        }
#pragma unroll
        for (int q = 0; q < NPC; ++q) {
            const int i = tid + q * kWideThreads;
            if (i < pieces) Us[i] = tmp[q];
        }
        __syncthreads();
        Ug = reinterpret_cast<const TU *>(Us);
    }
    const int g = tid % LPR;
    const int slot = tid / LPR;  // row of the block step; wave w owns slots [w RW, (w + 1) RW)
    const int w = tid >> 6;
    const double inv_n = 1.0 / (double)n;
    TA sc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) sc[q] = (TA)(st->Hs[B * B + g * VEC + q] * inv_n);
    dbl4 acc[TILES];
#pragma unroll
    for (int t = 0; t < TILES; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    double esum[NTB];
#pragma unroll
    for (int ti = 0; ti < NTB; ++ti) esum[ti] = 0.0;

    // Each wave works through its own rows with no block barrier: the row's
    // bounds, then the wave's whole CSR slice (its rows' entries are
    // contiguous) copied to its LDS region with coalesced loads, then each
    // row's entries CH at a time (all U loads of a chunk in flight
    // together), the output row, and the Gram of the wave's rows from its
    // own LDS rows (the same region: the slice is consumed by then).
    constexpr int WREG = S::WREG, CAPW = S::CAPW, NQ = (CAPW + 63) / 64;
    const int lane = tid & 63;
    double *__restrict__ wreg = smem + (size_t)w * WREG;
    int32_t *__restrict__ sci = reinterpret_cast<int32_t *>(wreg);
    TP *__restrict__ sval = reinterpret_cast<TP *>(sci + CAPW);
    const int rw = slot - w * RW;  // row within the wave
    const int64_t stride = (int64_t)vg * RPB;
    int beg_next = 0, end_next = 0;
    if ((int64_t)vb * RPB + slot < n) {
        beg_next = gld(rp + (int64_t)vb * RPB + slot);
        end_next = gld(rp + (int64_t)vb * RPB + slot + 1);
    }
    for (int64_t base = (int64_t)vb * RPB; base < n; base += stride) {
        const int64_t row = base + slot;
        const int beg = beg_next, end = end_next;
        // the next step's row bounds are loaded with this step's entries
        if (row + stride < n) {
            beg_next = gld(rp + row + stride);
            end_next = gld(rp + row + stride + 1);
        }
        // the wave's slice [E0, E1): rows past n have empty bounds
        const int E0 = __shfl(beg, 0);
        int E1 = end;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) E1 = max(E1, __shfl_xor(E1, m));
        const bool staged = E1 - E0 <= CAPW;  // uniform in the wave
        if (staged) {
            const int cnt = E1 - E0;
            int ct[NQ];
            TP vt[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int i = lane + 64 * q;
                ct[q] = i < cnt ? gld(ci + E0 + i) : 0;
                vt[q] = i < cnt ? gld(val + E0 + i) : TP{};
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int i = lane + 64 * q;
                if (i < cnt) {
                    sci[i] = ct[q];
                    sval[i] = vt[q];
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        TA a[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) a[q] = (TA)0;
        if (row < n) {
            for (int e0 = beg; e0 < end; e0 += CH) {
                int c[CH];
                TA pv[CH];
#pragma unroll
                for (int j = 0; j < CH; ++j) {
                    const bool ok = e0 + j < end;
                    // row 0 of U stands in for missing entries
                    if (staged) {
                        c[j] = ok ? sci[e0 - E0 + j] : 0;
                        pv[j] = ok ? up<TA>(sval[e0 - E0 + j]) : (TA)0;
                    } else {
                        c[j] = ok ? gld(ci + e0 + j) : 0;
                        pv[j] = ok ? up<TA>(gld(val + e0 + j)) : (TA)0;
                    }
                }
                Pack<TU, VEC> u[CH];
#pragma unroll
                for (int j = 0; j < CH; ++j) {
                    if constexpr (ULDS) u[j] = ldp<TU, VEC>(Ug + (size_t)c[j] * B + g * VEC);
                    else u[j] = ldpg<TU, VEC>(U + (size_t)c[j] * B + g * VEC);
                }
#pragma unroll
                for (int j = 0; j < CH; ++j) {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) a[q] += pv[j] * up<TA>(u[j].v[q]);
                }
            }
        }
        // every read of the slice is issued before the tile rows overwrite it
        __builtin_amdgcn_wave_barrier();
        if (row < n) {
            Pack<TY, VEC> o;
#pragma unroll
            for (int q = 0; q < VEC; ++q) o.v[q] = down<TY>(a[q] - sc[q]);
            stpg<TY, VEC>(Y + (size_t)row * B + g * VEC, o);
#pragma unroll
            for (int q = 0; q < VEC; ++q) wreg[rw * B + g * VEC + q] = (double)up<TA>(o.v[q]);
        } else {
#pragma unroll
            for (int q = 0; q < VEC; ++q) wreg[rw * B + g * VEC + q] = 0.0;
        }
        // the wave's rows are complete in LDS (one wave: in-order LDS, no
        // block barrier), and are read back only by this wave
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        gram_mfma_rows<B, RW, TILES>(wreg, 0, acc, esum);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();  // every wave is done with its tile rows before the reduction reuses smem
    const bool last = gram_mfma_finish<M, B, TILES>(acc, esum, smem, v.red_spmm, v.spmm_cnt, st, vb, vg);
    if constexpr (WPE != 4) return;  // no fused step (rejected at launch)
    if (rr && last) {  // uniform
        __syncthreads();  // smem is free again
        // waves past the step's own threads end here (whole waves: a
        // barrier waits only for the waves that have not ended), so the
        // step's barriers involve only its threads
        constexpr int NTR = RRShape<B>::NT;
        static_assert(NTR % 64 == 0 && NTR <= kWideThreads, "whole waves");
        if (threadIdx.x >= NTR) return;
        rr_step<B, NTR>(v, *reinterpret_cast<RRLds<B> *>(smem), b, k, kPivTol, rr == 2, max_sweeps, rule);
    }
}

// Gram matrix and column sums of the start block in buffer 0 (same
// geometry as k_spmm_wide).
template <int M, int B>
__global__ __launch_bounds__(kWideThreads) void k_gram_wide(const ProbView *__restrict__ views,
                                                            const int *__restrict__ off, int nprob,
                                                            int only_refill) {
    using Tr = Traits<M>;
    using TY = typename Tr::TY;
    using S = WideShape<M, B>;
    constexpr int VEC = S::VEC, LPR = S::LPR, RPB = S::RPB, RW = S::RW, TILES = S::TILES, NTB = S::NTB;
    __shared__ double smem[S::SMEM_D];
    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    if (only_refill && !v.st->refill) return;  // uniform per problem
    const int vb = blockIdx.x - off[p], vg = off[p + 1] - off[p];
    const int n = v.n;
    const TY *__restrict__ Y = (const TY *)v.Y0;
    double *tile = smem;
    const int tid = threadIdx.x;
    const int g = tid % LPR;
    const int slot = tid / LPR;
    const int w = tid >> 6;
    dbl4 acc[TILES];
#pragma unroll
    for (int t = 0; t < TILES; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    double esum[NTB];
#pragma unroll
    for (int ti = 0; ti < NTB; ++ti) esum[ti] = 0.0;
    for (int64_t base = (int64_t)vb * RPB; base < n; base += (int64_t)vg * RPB) {
        const int64_t row = base + slot;
        if (row < n) {
            Pack<TY, VEC> y = ldp<TY, VEC>(Y + (size_t)row * B + g * VEC);
#pragma unroll
            for (int q = 0; q < VEC; ++q) tile[slot * B + g * VEC + q] = (double)up<typename Tr::TA>(y.v[q]);
        } else {
#pragma unroll
            for (int q = 0; q < VEC; ++q) tile[slot * B + g * VEC + q] = 0.0;
        }
        __syncthreads();
        gram_mfma_rows<B, RW, TILES>(tile, w * RW, acc, esum);
        __syncthreads();
    }
    gram_mfma_finish<M, B, TILES>(acc, esum, smem, v.red_spmm, v.spmm_cnt, v.st, vb, vg);
}

// ---------------------------------------------------------------------------
// SpMM with the transposed operator (CSR of P^T), inner centering and the
// b x b basis rotation C.  WPR waves share one landmark row (its p + 1
// entries are split over them); a 256-thread block covers 4 / WPR rows.
// ---------------------------------------------------------------------------
template <int M, int B, int WPR, typename TY>
__device__ __forceinline__ void spmm_t_body(const ProbView *__restrict__ views, const int *__restrict__ off,
                                            int nprob, int phase) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TT = typename Tr::TT;
    using TP = typename Tr::TP;
    constexpr int VEC = VecOf<TY, B>::v;
    constexpr int LPR = B / VEC;
    constexpr int EPW = 64 / LPR;       // entries per wave step
    constexpr int RPBLK = 4 / WPR;      // landmark rows per block
    __shared__ double Cl[B * B];
    __shared__ double ex[B];
    __shared__ double part[4][B];       // per-wave partial sums
    __shared__ double rowbuf[RPBLK][B];

    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    const SolveState *__restrict__ st = v.st;
    if (st->done || st->phase != phase) return;
    // neighbouring landmark rows (the internal landmark order is spatial)
    // stay on one XCD, so the rows of Y they gather are shared in its L2
    const int vb = xcd_local_index(blockIdx.x, off[p], off[p + 1] - off[p]);
    const int l = v.l, n = v.n;
    const int32_t *__restrict__ rpT = v.rpT;
    const int32_t *__restrict__ ciT = v.ciT;
    const TP *__restrict__ valT = (const TP *)v.valT[M];
    const double *__restrict__ c = v.c[M];
    const TY *__restrict__ Y = (const TY *)(st->ycur ? v.Y1 : v.Y0);
    TT *__restrict__ T = (TT *)v.T;

    const int tid = threadIdx.x;
    for (int i = tid; i < B * B; i += 256) Cl[i] = st->C[i];
    if (tid < B) ex[tid] = st->e_x[tid];

    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int g = lane % LPR;
    const int slot = lane / LPR;
    const int rloc = wave / WPR;        // row within the block
    const int wsub = wave % WPR;        // wave within the row
    const int64_t j = (int64_t)vb * RPBLK + rloc;

    TA acc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) acc[q] = (TA)0;
    if (j < l) {
        const int beg = rpT[j], end = rpT[j + 1];
        constexpr int STEP = EPW * WPR;
        // CHT entries per lane at a time: all their Y loads in flight
        // together (missing entries read row 0 with weight 0), and the next
        // chunk's indices and values loaded while they are
        constexpr int CHT = kSpmmTChunk;
        int vi[CHT];
        TA pv[CHT];
        auto load_chunk = [&](int e) {
#pragma unroll
            for (int q = 0; q < CHT; ++q) {
                const int idx = e + q * STEP;
                const bool ok = idx < end;
                vi[q] = ok ? gld(ciT + idx) : 0;
                pv[q] = ok ? up<TA>(gld(valT + idx)) : (TA)0;
            }
        };
        int e = beg + wsub * EPW + slot;
        load_chunk(e);
        for (; e < end; e += CHT * STEP) {
            Pack<TY, VEC> y[CHT];
            TA pc[CHT];
#pragma unroll
            for (int q = 0; q < CHT; ++q) {
                y[q] = ldpg<TY, VEC>(Y + (size_t)vi[q] * B + g * VEC);
                pc[q] = pv[q];
            }
            load_chunk(e + CHT * STEP);
#pragma unroll
            for (int q = 0; q < CHT; ++q) {
#pragma unroll
                for (int r = 0; r < VEC; ++r) acc[r] += pc[q] * up<TA>(y[q].v[r]);
            }
        }
    }
#pragma unroll
    for (int m = LPR; m < 64; m <<= 1) {
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] += __shfl_xor(acc[q], m);
    }
    if (slot == 0) {
#pragma unroll
        for (int q = 0; q < VEC; ++q) part[wave][g * VEC + q] = (double)acc[q];
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

// The block Y is read in the storage type of this arithmetic, or -- on the
// first iteration after a precision change -- in the narrower type of the
// previous phase (widening is exact), which saves a conversion pass over Y.
template <int M>
struct PrevY {
    using T = typename Traits<M>::TY;
};
template <>
struct PrevY<MODE_FP32> {
    using T = bf16_t;
};
template <>
struct PrevY<MODE_F64ACC> {
    using T = float;
};

template <int M, int B, int WPR>
__global__ __launch_bounds__(256) void k_spmm_t(const ProbView *__restrict__ views, const int *__restrict__ off,
                                                int nprob, int phase) {
    const int p = find_problem(off, nprob, blockIdx.x);
    const int ymode = views[p].st->ymode;  // uniform in the block
    if (ymode == M || std::is_same<typename PrevY<M>::T, typename Traits<M>::TY>::value)
        spmm_t_body<M, B, WPR, typename Traits<M>::TY>(views, off, nprob, phase);
    else
        spmm_t_body<M, B, WPR, typename PrevY<M>::T>(views, off, nprob, phase);
}

// ---------------------------------------------------------------------------
// Transposed product, push form (see prep_push_*): block vb stages its
// kPushVB rows of Y in LDS (read once, contiguous), then every (block,
// landmark) pair q it owns gets the partial row sum_e val_e Y[v_e] over the
// pair's entries (in vertex order), one group of B / VEC lanes per pair.
// The reduction adds a landmark's partial rows in block order, applies the
// inner centering and the basis rotation C, and writes its row of T.

bool spmmt_push_width(int B) { return B == 8 || B == 16 || B == 32; }

constexpr int kPushChunk = 8;

template <typename TA, int B>
struct PushRed {
    static constexpr int VA = (16 / (int)sizeof(TA)) < B ? (16 / (int)sizeof(TA)) : B;
    static constexpr int G = B / VA;       // lanes per landmark
    static constexpr int ROWS = 256 / G;   // landmarks per block
};

int spmmt_push_rows(Mode m, int B) {
    const bool f64 = m == MODE_F64ACC || m == MODE_FP64;
    const int va = std::min(f64 ? 2 : 4, B);
    return 256 / (B / va);
}

template <int M, int B, typename TY>
__device__ __forceinline__ void spmmt_push_body(const ProbView *__restrict__ views, const int *__restrict__ off,
                                                int nprob, int phase) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TP = typename Tr::TP;
    constexpr int VEC = VecOf<TY, B>::v;
    constexpr int G = B / VEC;  // lanes per pair
    constexpr int GROUPS = 256 / G;
    __shared__ Pack<TY, VEC> ys[kPushVB * G];

    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    const SolveState *__restrict__ st = v.st;
    if (st->done || st->phase != phase) return;
    const int vb = blockIdx.x - off[p];
    const int64_t v0 = (int64_t)vb * kPushVB;
    const int nv = (int)((int64_t)v.n - v0 < kPushVB ? (int64_t)v.n - v0 : kPushVB);
    const TY *__restrict__ Y = (const TY *)(st->ycur ? v.Y1 : v.Y0) + v0 * B;
    for (int i = threadIdx.x; i < nv * G; i += 256) ys[i] = ldpg<TY, VEC>(Y + (size_t)i * VEC);
    __syncthreads();
    const TP *__restrict__ pv = (const TP *)v.pval[M];
    const uint8_t *__restrict__ pvl = v.pvl;
    const int32_t *__restrict__ pe = v.pe;
    TA *__restrict__ part = (TA *)v.ppart;
    const int grp = threadIdx.x / G, g = threadIdx.x % G;
    const int q1 = v.pb[vb + 1];
    constexpr int CH = kPushChunk;  // entries whose loads are in flight together
    for (int q = v.pb[vb] + grp; q < q1; q += GROUPS) {
        Pack<TA, VEC> acc;
#pragma unroll
        for (int r = 0; r < VEC; ++r) acc.v[r] = (TA)0;
        const int e1 = pe[q + 1];
        for (int e0 = pe[q]; e0 < e1; e0 += CH) {
            TA w[CH];
            int vl[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const bool ok = e0 + u < e1;  // missing entries read row 0 with weight 0
                w[u] = ok ? up<TA>(pv[e0 + u]) : (TA)0;
                vl[u] = ok ? (int)pvl[e0 + u] : 0;
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const Pack<TY, VEC> y = ys[vl[u] * G + g];
#pragma unroll
                for (int r = 0; r < VEC; ++r) acc.v[r] += w[u] * up<TA>(y.v[r]);
            }
        }
        stpg<TA, VEC>(part + (size_t)q * B + g * VEC, acc);
    }
}

template <int M, int B>
__global__ __launch_bounds__(256) void k_spmmt_push(const ProbView *__restrict__ views, const int *__restrict__ off,
                                                    int nprob, int phase) {
    const int p = find_problem(off, nprob, blockIdx.x);
    const int ymode = views[p].st->ymode;  // uniform in the block
    if (ymode == M || std::is_same<typename PrevY<M>::T, typename Traits<M>::TY>::value)
        spmmt_push_body<M, B, typename Traits<M>::TY>(views, off, nprob, phase);
    else
        spmmt_push_body<M, B, typename PrevY<M>::T>(views, off, nprob, phase);
}

template <int M, int B>
__global__ __launch_bounds__(256) void k_spmmt_reduce(const ProbView *__restrict__ views,
                                                      const int *__restrict__ off, int nprob, int phase) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TT = typename Tr::TT;
    constexpr int VA = PushRed<TA, B>::VA, G = PushRed<TA, B>::G, ROWS = PushRed<TA, B>::ROWS;
    __shared__ double Cl[B * B];
    __shared__ double ex[B];
    __shared__ double rowbuf[ROWS][B];

    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    const SolveState *__restrict__ st = v.st;
    if (st->done || st->phase != phase) return;
    const int tid = threadIdx.x;
    for (int i = tid; i < B * B; i += 256) Cl[i] = st->C[i];
    if (tid < B) ex[tid] = st->e_x[tid];
    const int grp = tid / G, g = tid % G;
    const int64_t j = (int64_t)(blockIdx.x - off[p]) * ROWS + grp;
    const bool live = j < v.l;
    Pack<TA, VA> acc;
#pragma unroll
    for (int r = 0; r < VA; ++r) acc.v[r] = (TA)0;
    if (live) {
        // kPushChunk partial rows in flight together, added in order
        constexpr int CH = kPushChunk;
        const TA *__restrict__ part = (const TA *)v.ppart;
        const int q1 = v.qp[j + 1];
        for (int q0 = v.qp[j]; q0 < q1; q0 += CH) {
            int idx[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) idx[u] = q0 + u < q1 ? v.ql[q0 + u] : -1;
            Pack<TA, VA> x[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (idx[u] >= 0) x[u] = ldpg<TA, VA>(part + (size_t)idx[u] * B + g * VA);
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (idx[u] >= 0) {
#pragma unroll
                    for (int r = 0; r < VA; ++r) acc.v[r] += x[u].v[r];
                }
        }
    }
    __syncthreads();  // Cl and ex
    if (live) {
        const double cj = v.c[M][j] / (double)v.n;
#pragma unroll
        for (int r = 0; r < VA; ++r) rowbuf[grp][g * VA + r] = (double)acc.v[r] - cj * ex[g * VA + r];
    }
    __syncthreads();
    if (live) {
        TT *__restrict__ T = (TT *)v.T;
#pragma unroll
        for (int r = 0; r < VA; ++r) {
            const int col = g * VA + r;
            double t = 0.0;
#pragma unroll 8
            for (int i = 0; i < B; ++i) t += rowbuf[grp][i] * Cl[i * B + col];
            T[(size_t)j * B + col] = down<TT>((TA)t);
        }
    }
}

// ---------------------------------------------------------------------------
// Start blocks, precision changes and outputs.
// ---------------------------------------------------------------------------

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): four 32-bit words of counter (each use below
// states its layout), key = seed.
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

// Two standard normals from two uniforms (Box-Muller: the radius from the
// first, the angle from the second, both its cosine and its sine).
__device__ __forceinline__ void gauss_pair(uint32_t a, uint32_t b, float &z0, float &z1) {
    const float u1 = ((float)(a >> 8) + 1.0f) * (1.0f / 16777216.0f);
    const float u2 = (float)(b >> 8) * (1.0f / 16777216.0f);
    const float r = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincospif(2.0f * u2, &sn, &cs);
    z0 = r * cs;
    z1 = r * sn;
}

// Start block into buffer 0 (random, or the caller's block); columns >= b
// are zero.  One thread per four consecutive columns of a row: a random
// block takes the four outputs of one Philox call (counter = row, column
// quad, row >> 32, problem) as two Box-Muller pairs, so the integer
// multiplies of the generator, which bound this kernel, are a quarter of
// one call per element.  The launch has one thread per element; the last
// three quarters of a problem's blocks have no work.
template <int M, int B, int USER, typename TS>
__global__ __launch_bounds__(256) void k_start_block(const ProbView *__restrict__ views, const int *__restrict__ off,
                                                     int nprob, int b, uint64_t seed) {
    using TY = typename Traits<M>::TY;
    using TA = typename Traits<M>::TA;
    static_assert(B % 4 == 0, "whole column quads");
    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    const int64_t q = (int64_t)(blockIdx.x - off[p]) * 256 + threadIdx.x;
    if (q >= (int64_t)v.n * (B / 4)) return;
    const int64_t row = q / (B / 4);
    const int c0 = (int)(q % (B / 4)) * 4;
    float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    TA zu[4] = {(TA)0, (TA)0, (TA)0, (TA)0};
    if (USER) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (c0 + t < b) zu[t] = (TA)((const TS *)v.X0)[row * b + c0 + t];
    } else if (c0 < b) {
        uint32_t ctr[4] = {(uint32_t)row, (uint32_t)(c0 >> 2), (uint32_t)(row >> 32), (uint32_t)p};
        philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
        gauss_pair(ctr[0], ctr[1], z[0], z[1]);
        gauss_pair(ctr[2], ctr[3], z[2], z[3]);
#pragma unroll
        for (int t = 0; t < 4; ++t) zu[t] = c0 + t < b ? (TA)z[t] : (TA)0;
    }
    TY *dst = (TY *)v.Y0 + row * B + c0;
#pragma unroll
    for (int t = 0; t < 4; ++t) dst[t] = down<TY>(zu[t]);
}

// Precision change at the start of phase `phase`: the current block is
// copied into the other buffer in the new storage type (widening, so
// exact).  Runs only for problems whose previous phase has just ended.
template <int MF, int MT, int B>
__global__ __launch_bounds__(256) void k_convert(const ProbView *__restrict__ views, const int *__restrict__ off,
                                                 int nprob, int phase) {
    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    const SolveState *st = v.st;
    if (st->done || st->phase != phase || !st->pending_convert) return;
    using TAt = typename Traits<MT>::TA;
    using TYt = typename Traits<MT>::TY;
    const typename Traits<MF>::TY *src = (const typename Traits<MF>::TY *)(st->ycur ? v.Y1 : v.Y0);
    TYt *dst = (TYt *)(st->ycur ? v.Y0 : v.Y1);
    const int64_t i = (int64_t)(blockIdx.x - off[p]) * 256 + threadIdx.x;
    if (i < (int64_t)v.n * B) dst[i] = down<TYt>((TAt)up<double>(src[i]));
}

// After the conversion: the other buffer is now current (one block per problem).
__global__ void k_phase_begin(const ProbView *__restrict__ views, int phase, int mode) {
    SolveState *st = views[blockIdx.x].st;
    if (threadIdx.x == 0 && !st->done && st->phase == phase && st->pending_convert) {
        const int ycur = st->ycur ^ 1;
        st->ycur = ycur;
        st->ymode = mode;
        st->pending_convert = 0;
        // the host copy of the state follows
        char *h = (char *)views[blockIdx.x].host_sum;
        if (h) {
            *(int *)(h + offsetof(SolveState, ycur) - kSummaryOffset) = ycur;
            *(int *)(h + offsetof(SolveState, ymode) - kSummaryOffset) = mode;
            *(int *)(h + offsetof(SolveState, pending_convert) - kSummaryOffset) = 0;
        }
    }
}

bool reads_previous_block(Mode from, Mode to) {
    return (from == MODE_BF16 && to == MODE_FP32) || (from == MODE_FP32 && to == MODE_F64ACC);
}


__device__ __forceinline__ double load_y(const void *Y, int64_t i, int mode) {
    if (mode == MODE_BF16) return (double)bf2f(((const bf16_t *)Y)[i]);
    if (mode == MODE_FP32) return (double)((const float *)Y)[i];
    return ((const double *)Y)[i];
}

__device__ __forceinline__ double to_double(bf16_t x) { return (double)bf2f(x); }
__device__ __forceinline__ double to_double(float x) { return (double)x; }
__device__ __forceinline__ double to_double(double x) { return x; }

// Row `row` of a block stored as TY, with 16-byte (or whole-row) loads.
template <int B, typename TY>
__device__ __forceinline__ void load_row(const void *Y, int64_t row, double (&y)[B]) {
    constexpr int V = (16 / (int)sizeof(TY)) < B ? 16 / (int)sizeof(TY) : B;
    static_assert(B % V == 0 && (sizeof(TY) * V) % 4 == 0, "whole dwords per load");
    const TY *base = (const TY *)Y + row * B;
#pragma unroll
    for (int a0 = 0; a0 < B; a0 += V) {
        const Pack<TY, V> pk = ldpg<TY, V>(base + a0);
#pragma unroll
        for (int q = 0; q < V; ++q) y[a0 + q] = to_double(pk.v[q]);
    }
}

// Z = J Y Zmap restricted to the first k columns: Z_ij = sum_a Y_ia Zmap_aj - zshift_j,
// with Y the buffer (and storage type) the last Ritz basis was built from.
template <int B, typename TZ>
__global__ __launch_bounds__(256) void k_embedding(const ProbView *__restrict__ views, const int *__restrict__ off,
                                                   int nprob, int k, TZ *__restrict__ Z) {
    __shared__ double Zm[B * B];
    __shared__ double zs[B];
    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    const SolveState *st = v.st;
    for (int i = threadIdx.x; i < B * B; i += 256) Zm[i] = st->Zmap[i];
    if (threadIdx.x < B) zs[threadIdx.x] = st->zshift[threadIdx.x];
    __syncthreads();
    const int64_t row = (int64_t)(blockIdx.x - off[p]) * 256 + threadIdx.x;
    if (row >= v.n) return;
    const void *Y = st->zbuf ? v.Y1 : v.Y0;
    const int mode = st->zmode;  // uniform
    double y[B];
    if (mode == MODE_BF16) load_row<B, bf16_t>(Y, row, y);
    else if (mode == MODE_FP32) load_row<B, float>(Y, row, y);
    else load_row<B, double>(Y, row, y);
    TZ *zp = Z + v.zoff + row * k;
    for (int j = 0; j < k; ++j) {
        double z = -zs[j];
#pragma unroll
        for (int a = 0; a < B; ++a) z += y[a] * Zm[a * B + j];
        zp[j] = (TZ)z;
    }
}

// Rank repair (see launch_refill).  One thread per row: the row of the basis
// X = J Y C of a problem whose last CholQR dropped columns, with every dropped
// column (an all-zero column of C below b) replaced by a fresh Gaussian
// value, written over row `row` of buffer 0 in the block's storage type.  The
// whole row is read before it is written, so buffer 0 may be the source.
template <int M, int B>
__global__ __launch_bounds__(256) void k_refill(const ProbView *__restrict__ views, const int *__restrict__ off,
                                                int nprob, int b, uint64_t seed, uint32_t salt) {
    using TY = typename Traits<M>::TY;
    using TA = typename Traits<M>::TA;
    __shared__ double Cm[B * B];
    __shared__ double ex[B];
    __shared__ int dropped[B];
    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    SolveState *st = v.st;
    if (st->done || st->dead <= 0 || st->ymode != M) return;  // uniform per problem
    for (int i = threadIdx.x; i < B * B; i += 256) Cm[i] = st->C[i];
    if (threadIdx.x < B) ex[threadIdx.x] = st->e_x[threadIdx.x];
    __syncthreads();
    if (threadIdx.x < B) {
        bool zero = true;
        for (int r = 0; r < B; ++r) zero = zero && Cm[r * B + threadIdx.x] == 0.0;
        dropped[threadIdx.x] = (threadIdx.x < b && zero) ? 1 : 0;
    }
    __syncthreads();
    if (blockIdx.x == off[p] && threadIdx.x == 0) st->refill = 1;
    const int64_t row = (int64_t)(blockIdx.x - off[p]) * 256 + threadIdx.x;
    if (row >= v.n) return;
    double y[B];
    load_row<B, TY>(st->ycur ? v.Y1 : v.Y0, row, y);
    const double inv_n = 1.0 / (double)v.n;
#pragma unroll
    for (int a = 0; a < B; ++a) y[a] -= ex[a] * inv_n;
    TY *dst = (TY *)v.Y0 + row * B;
    for (int j = 0; j < B; ++j) {
        double x = 0.0;
        if (dropped[j]) {
            uint32_t ctr[4] = {(uint32_t)row, (uint32_t)j | (salt << 8), (uint32_t)(row >> 32), (uint32_t)p};
            philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
            x = (double)gauss_from(ctr[0], ctr[1]);
        } else {
#pragma unroll
            for (int a = 0; a < B; ++a) x += y[a] * Cm[a * B + j];
        }
        dst[j] = down<TY>((TA)x);
    }
}

// Landmark-block start (see launch_lift_prep).  One thread per element of
// the l x B block U of problem p.
template <int M, int B, int LMDS>
__global__ __launch_bounds__(256) void k_lift_prep(const ProbView *__restrict__ views, const int *__restrict__ off,
                                                   int nprob, int b, int k, const ProbView *__restrict__ lviews,
                                                   const float *__restrict__ learned, uint64_t seed) {
    using TU = typename Traits<M>::TU;
    const int p = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[p];
    const int64_t idx = (int64_t)(blockIdx.x - off[p]) * 256 + threadIdx.x;
    if (idx == 0) {
        SolveState *st = v.st;
        for (int a = 0; a < B; ++a) st->Hs[B * B + a] = 0.0;  // no outer centering term
        st->ycur = 1;  // the SpMM writes the other buffer: buffer 0
        st->phase = 0;
        st->done = 0;
    }
    if (idx >= (int64_t)v.l * B) return;
    const int64_t j = idx / B;
    const int a = (int)(idx % B);
    double u = 0.0;
    if (a < b) {
        if (LMDS) {
            // column a of the landmark problem's current basis J Y C
            const ProbView &lv = lviews[p];
            const SolveState *ls = lv.st;
            const void *Y = ls->ycur ? lv.Y1 : lv.Y0;
            const int mode = ls->ymode;
            double x = 0.0, sh = 0.0;
            for (int c = 0; c < B; ++c) {
                const double cc = ls->C[c * B + a];
                x += load_y(Y, j * B + c, mode) * cc;
                sh += ls->e_x[c] * cc;
            }
            u = x - sh / (double)lv.n;
        } else if (a < k) {
            u = (double)learned[(v.loff + j) * k + a];
        } else {
            // counter (landmark, column, tag, problem): disjoint from the n-space start block
            uint32_t ctr[4] = {(uint32_t)j, (uint32_t)a, 0x4c69667du, (uint32_t)p};
            philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
            u = (double)gauss_from(ctr[0], ctr[1]);
        }
    }
    ((TU *)v.U)[j * B + a] = (TU)u;
}

// X = J Y C (the current orthonormal basis), first b columns, one problem.
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

__global__ __launch_bounds__(256) void k_f32_to_bf16(int64_t count, const float *__restrict__ src,
                                                     bf16_t *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) dst[i] = f2bf(src[i]);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define SBMDS_DISPATCH_B(B_, CALL)                      \
    switch (B_) {                                       \
        case 4: { constexpr int BB = 4; CALL; } break;   \
        case 8: { constexpr int BB = 8; CALL; } break;   \
        case 16: { constexpr int BB = 16; CALL; } break; \
        case 32: { constexpr int BB = 32; CALL; } break; \
        case 64: { constexpr int BB = 64; CALL; } break; \
        default: return hipErrorInvalidValue;           \
    }

#define SBMDS_DISPATCH_M(M_, CALL)                                         \
    switch (M_) {                                                          \
        case MODE_BF16: { constexpr int MM = MODE_BF16; CALL; } break;     \
        case MODE_FP32: { constexpr int MM = MODE_FP32; CALL; } break;     \
        case MODE_F64ACC: { constexpr int MM = MODE_F64ACC; CALL; } break; \
        case MODE_FP64: { constexpr int MM = MODE_FP64; CALL; } break;     \
        default: return hipErrorInvalidValue;                              \
    }

bool spmm_runs_rr(const Batch &bt, Mode m) { return wide_width(bt.B) && !bt.spmm_wpe8[m]; }
bool spmm_has_two_block_form(int B) { return wide_width(B); }

hipError_t launch_spmm(Mode m, const Batch &bt, int phase, hipStream_t s, int rr, int max_sweeps,
                       const PhaseRule &rule) {
    const int grid = bt.total[BK_SPMM][m];
    if (grid <= 0) return hipErrorInvalidValue;
    const int *off = bt.off(BK_SPMM, m);
    SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(bt.B, {
        if constexpr (wide_width(BB)) {
            using TUU = typename Traits<MM>::TU;
            if (bt.spmm_wpe8[MM]) {
                if (rr) return hipErrorInvalidValue;  // this form leaves the step to its own launch
                hipLaunchKernelGGL((k_spmm_wide<MM, BB, false, 8>), dim3(grid), dim3(kWideThreads), 0, s, bt.views,
                                   off, bt.nprob, phase, 0, bt.b, bt.k, 0, rule);
                return hipGetLastError();
            }
            if constexpr ((BB * sizeof(TUU)) % 16 == 0 && BB * sizeof(TUU) <= 64) {
                if ((size_t)bt.max_l * BB * sizeof(TUU) <= (size_t)kUldsBytes) {
                    hipLaunchKernelGGL((k_spmm_wide<MM, BB, true>), dim3(grid), dim3(kWideThreads), 0, s, bt.views,
                                       off, bt.nprob, phase, rr, bt.b, bt.k, max_sweeps, rule);
                    return hipGetLastError();
                }
            }
            hipLaunchKernelGGL((k_spmm_wide<MM, BB, false>), dim3(grid), dim3(kWideThreads), 0, s, bt.views, off,
                               bt.nprob, phase, rr, bt.b, bt.k, max_sweeps, rule);
        }
        else if (rr)
            return hipErrorInvalidValue;  // the narrow kernel leaves the step to its own launch
        else
            hipLaunchKernelGGL((k_spmm<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
        return hipGetLastError();
    }));
    return hipErrorInvalidValue;
}

template <int MM, int BB, int WPR>
static hipError_t spmm_t_impl(const Batch &bt, int phase, hipStream_t s) {
    const int grid = bt.total[BK_SPMMT][MM];
    if (grid <= 0) return bt.spmmt_push[MM] ? hipSuccess : hipErrorInvalidValue;  // all in the push form
    hipLaunchKernelGGL((k_spmm_t<MM, BB, WPR>), dim3(grid), dim3(256), 0, s, bt.views, bt.off(BK_SPMMT, (Mode)MM),
                       bt.nprob, phase);
    return hipGetLastError();
}

template <int MM, int BB>
static hipError_t spmmt_push_impl(const Batch &bt, int phase, hipStream_t s) {
    const int g1 = bt.total[BK_PUSH][MM], g2 = bt.total[BK_PUSHR][MM];
    if (g1 <= 0 || g2 <= 0) return hipSuccess;  // no problem of the batch takes the push form
    hipLaunchKernelGGL((k_spmmt_push<MM, BB>), dim3(g1), dim3(256), 0, s, bt.views, bt.off(BK_PUSH, (Mode)MM),
                       bt.nprob, phase);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_spmmt_reduce<MM, BB>), dim3(g2), dim3(256), 0, s, bt.views, bt.off(BK_PUSHR, (Mode)MM),
                       bt.nprob, phase);
    return hipGetLastError();
}

static hipError_t launch_spmm_t_push(Mode m, const Batch &bt, int phase, hipStream_t s) {
    switch (bt.B) {
        case 8: SBMDS_DISPATCH_M(m, return (spmmt_push_impl<MM, 8>(bt, phase, s))); break;
        case 16: SBMDS_DISPATCH_M(m, return (spmmt_push_impl<MM, 16>(bt, phase, s))); break;
        case 32: SBMDS_DISPATCH_M(m, return (spmmt_push_impl<MM, 32>(bt, phase, s))); break;
        default: return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

// Problems in the push form run its two kernels, the others the row-gather
// kernel (each launch skips the problems of the other form: they own no
// blocks of it).
hipError_t launch_spmm_t(Mode m, const Batch &bt, int phase, hipStream_t s) {
    if (bt.spmmt_push[m]) {
        hipError_t e = launch_spmm_t_push(m, bt, phase, s);
        if (e != hipSuccess || bt.total[BK_SPMMT][m] <= 0) return e;
    }
    switch (bt.spmmt_wpr[m]) {
        case 1: SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(bt.B, return (spmm_t_impl<MM, BB, 1>(bt, phase, s)))); break;
        case 2: SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(bt.B, return (spmm_t_impl<MM, BB, 2>(bt, phase, s)))); break;
        case 4: SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(bt.B, return (spmm_t_impl<MM, BB, 4>(bt, phase, s)))); break;
        default: return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

template <int MM, int BB, int USER>
static hipError_t start_impl(const Batch &bt, uint64_t seed, hipStream_t s) {
    const int g1 = bt.total[BK_ELEM_NB][MM];
    if (g1 <= 0) return hipErrorInvalidValue;
    if (MM == MODE_FP64)
        hipLaunchKernelGGL((k_start_block<MM, BB, USER, double>), dim3(g1), dim3(256), 0, s, bt.views,
                           bt.off(BK_ELEM_NB, (Mode)MM), bt.nprob, bt.b, seed);
    else
        hipLaunchKernelGGL((k_start_block<MM, BB, USER, float>), dim3(g1), dim3(256), 0, s, bt.views,
                           bt.off(BK_ELEM_NB, (Mode)MM), bt.nprob, bt.b, seed);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int grid = bt.total[BK_SPMM][MM];
    if (grid <= 0) return hipErrorInvalidValue;
    if constexpr (wide_width(BB))
        hipLaunchKernelGGL((k_gram_wide<MM, BB>), dim3(grid), dim3(kWideThreads), 0, s, bt.views,
                           bt.off(BK_SPMM, (Mode)MM), bt.nprob, 0);
    else
        hipLaunchKernelGGL((k_gram<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, bt.off(BK_SPMM, (Mode)MM),
                           bt.nprob, 0);
    return hipGetLastError();
}

template <int MM, int BB>
static hipError_t refill_impl(const Batch &bt, uint64_t seed, uint32_t salt, hipStream_t s) {
    const int g1 = bt.total[BK_ELEM_N][0];
    const int grid = bt.total[BK_SPMM][MM];
    if (g1 <= 0 || grid <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_refill<MM, BB>), dim3(g1), dim3(256), 0, s, bt.views, bt.off(BK_ELEM_N, MODE_BF16),
                       bt.nprob, bt.b, seed, salt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (wide_width(BB))
        hipLaunchKernelGGL((k_gram_wide<MM, BB>), dim3(grid), dim3(kWideThreads), 0, s, bt.views,
                           bt.off(BK_SPMM, (Mode)MM), bt.nprob, 1);
    else
        hipLaunchKernelGGL((k_gram<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, bt.off(BK_SPMM, (Mode)MM),
                           bt.nprob, 1);
    return hipGetLastError();
}

hipError_t launch_refill(Mode m, const Batch &bt, uint64_t seed, uint32_t salt, hipStream_t s) {
    SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(bt.B, return (refill_impl<MM, BB>(bt, seed, salt, s))));
    return hipErrorInvalidValue;
}

hipError_t launch_random_start(Mode m, const Batch &bt, uint64_t seed, hipStream_t s) {
    SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(bt.B, return (start_impl<MM, BB, 0>(bt, seed, s))));
    return hipErrorInvalidValue;
}

hipError_t launch_user_start(Mode m, const Batch &bt, hipStream_t s) {
    SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(bt.B, return (start_impl<MM, BB, 1>(bt, 0, s))));
    return hipErrorInvalidValue;
}

template <int MF, int MT, int BB>
static hipError_t convert_impl(const Batch &bt, int phase, hipStream_t s) {
    const int grid = bt.total[BK_ELEM_NB][MT];
    if (grid <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_convert<MF, MT, BB>), dim3(grid), dim3(256), 0, s, bt.views, bt.off(BK_ELEM_NB, (Mode)MT),
                       bt.nprob, phase);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_phase_begin, dim3(bt.nprob), dim3(64), 0, s, bt.views, phase, MT);
    return hipGetLastError();
}

hipError_t launch_convert_y(Mode from, Mode to, const Batch &bt, int phase, hipStream_t s) {
    switch (from) {
        case MODE_BF16: {
            constexpr int MF = MODE_BF16;
            SBMDS_DISPATCH_M(to, SBMDS_DISPATCH_B(bt.B, return (convert_impl<MF, MM, BB>(bt, phase, s))));
        } break;
        case MODE_FP32: {
            constexpr int MF = MODE_FP32;
            SBMDS_DISPATCH_M(to, SBMDS_DISPATCH_B(bt.B, return (convert_impl<MF, MM, BB>(bt, phase, s))));
        } break;
        case MODE_F64ACC: {
            constexpr int MF = MODE_F64ACC;
            SBMDS_DISPATCH_M(to, SBMDS_DISPATCH_B(bt.B, return (convert_impl<MF, MM, BB>(bt, phase, s))));
        } break;
        case MODE_FP64: {
            constexpr int MF = MODE_FP64;
            SBMDS_DISPATCH_M(to, SBMDS_DISPATCH_B(bt.B, return (convert_impl<MF, MM, BB>(bt, phase, s))));
        } break;
        default: return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_embedding(const Batch &bt, void *Z, int z_double, hipStream_t s) {
    const int grid = bt.total[BK_ELEM_N][0];
    if (grid <= 0) return hipErrorInvalidValue;
    const int *off = bt.off(BK_ELEM_N, MODE_BF16);
    SBMDS_DISPATCH_B(bt.B, {
        if (z_double)
            hipLaunchKernelGGL((k_embedding<BB, double>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, bt.k,
                               (double *)Z);
        else
            hipLaunchKernelGGL((k_embedding<BB, float>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, bt.k,
                               (float *)Z);
        return hipGetLastError();
    });
    return hipErrorInvalidValue;
}

template <int MM, int BB>
static hipError_t lift_impl(const Batch &bt, const Batch *lmk, const float *learned, uint64_t seed, hipStream_t s) {
    const int grid = bt.total[BK_ELEM_LB][0];
    if (grid <= 0) return hipErrorInvalidValue;
    const int *off = bt.off(BK_ELEM_LB, MODE_BF16);
    if (lmk)
        hipLaunchKernelGGL((k_lift_prep<MM, BB, 1>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, bt.b, bt.k,
                           (const ProbView *)lmk->views, (const float *)nullptr, seed);
    else
        hipLaunchKernelGGL((k_lift_prep<MM, BB, 0>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, bt.b, bt.k,
                           (const ProbView *)nullptr, learned, seed);
    return hipGetLastError();
}

hipError_t launch_lift_prep(Mode m, const Batch &bt, const Batch *lmk, const float *learned, uint64_t seed,
                            hipStream_t s) {
    if (lmk && (lmk->nprob != bt.nprob || lmk->B != bt.B)) return hipErrorInvalidValue;
    if (!lmk && !learned) return hipErrorInvalidValue;
    SBMDS_DISPATCH_M(m, SBMDS_DISPATCH_B(bt.B, return (lift_impl<MM, BB>(bt, lmk, learned, seed, s))));
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

hipError_t launch_f32_to_bf16(const float *src, void *dst, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, src,
                       (bf16_t *)dst);
    return hipGetLastError();
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
