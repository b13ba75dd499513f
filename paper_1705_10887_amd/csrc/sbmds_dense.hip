// Dense landmark product U = -1/2 W T (l x l times l x b), Section 3.3.
//
// W is streamed from HBM exactly once per launch; it dominates the bytes of
// an iteration once l^2 exceeds n * p_row.  The product is tall and skinny
// (b = 4..64 columns), so its arithmetic intensity is 2b flops per element of
// W and the kernel is bandwidth bound.
//
// Work split: a grid of (row tiles) x (K splits).  Each block accumulates a
// partial U tile over its K range; the last block to finish a row tile sums
// the K partials in fixed order, applies the -1/2, stores U and reduces the
// tile's contributions to H = T^T U (the Rayleigh quotient X^T B X, float64)
// and s = c^T U (the outer centering term).  The last tile reduces those over
// all tiles.  Every reduction runs in a fixed order, so results are bitwise
// reproducible.
#include <type_traits>

#include "sbmds_common.h"
#include "sbmds_dense_sym.h"

namespace sbmds {

template <typename TA, int B>
struct GemmShape {
    // rows per wave: keep RW * B accumulators at 64 (float) / 32..64 (double)
    static constexpr int NVMAX = sizeof(TA) == 4 ? 64 : (B >= 64 ? 64 : 32);
    static constexpr int RW = (NVMAX / B) > 0 ? (NVMAX / B) : 1;
    static constexpr int NV = RW * B;
    static constexpr int RT = 4 * RW;  // rows per block (4 waves)
};

bool gemm_mfma(Mode m, int B);

int gemm_rows_per_tile(Mode m, int B, int mfma) {
    if (mfma && gemm_mfma(m, B)) return 64;
    const bool dbl = (m == MODE_F64ACC || m == MODE_FP64);
    const int nvmax = dbl ? (B >= 64 ? 64 : 32) : 64;
    const int rw = nvmax / B > 0 ? nvmax / B : 1;
    return 4 * rw;
}

// Butterfly reduce-scatter of CNT values over the 64 lanes of a wave.  Each
// step with mask M keeps half of the values (the upper half on lanes with bit
// M set) and adds the partner's copy of them, so all indices stay
// compile-time constants.  On return a[0] holds the full sum of value index
// `off` (lanes that share `off` hold the same sum).
template <typename TA, int CNT, int M>
struct ReduceScatter {
    static __device__ __forceinline__ void run(TA *a, int lane, int &off) {
        if constexpr (M > 0) {
            if constexpr (CNT > 1) {
                constexpr int H = CNT / 2;
                const bool hi = (lane & M) != 0;
#pragma unroll
                for (int i = 0; i < H; ++i) {
                    const TA mine = hi ? a[i + H] : a[i];
                    const TA other = hi ? a[i] : a[i + H];
                    a[i] = mine + __shfl_xor(other, M);
                }
                off += hi ? H : 0;
                ReduceScatter<TA, H, M / 2>::run(a, lane, off);
            } else {
                a[0] += __shfl_xor(a[0], M);
                ReduceScatter<TA, 1, M / 2>::run(a, lane, off);
            }
        }
    }
};

// Per-tile finish of the split-K product (shared by both kernels): the
// last of the ksplit blocks of row tile rt sums the K partials in fixed
// order, stores U = -1/2 sum, and reduces the tile's contributions to
// H = T^T U and s = c^T U; the last tile reduces those into st->Hs.
template <int M, int B, int RT>
__device__ __forceinline__ void gemm_tile_finish(const ProbView &v, SolveState *__restrict__ st, int rt, int rowtiles,
                                                 int ksplit, const typename Traits<M>::TA (*own)[B] = nullptr) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TT = typename Tr::TT;
    using TU = typename Tr::TU;
    const int l = v.l, lda = v.lda;
    const TT *__restrict__ T = (const TT *)v.T;
    const TA *__restrict__ part = (const TA *)v.gpart;
    TU *__restrict__ U = (TU *)v.U;
    const double *__restrict__ c = v.c[M];
    double *__restrict__ red = v.red_gemm;
    unsigned *__restrict__ tile_cnt = v.tile_cnt;
    unsigned *__restrict__ tree_cnt = v.gemm_cnt;
    const int tid = threadIdx.x;
    // own: the whole K range was this block's (ksplit == 1), its sums are in
    // LDS and no other block takes part in the tile
    if (!own && !arrive_last(tile_cnt + rt, (unsigned)ksplit)) return;
    __shared__ double ul[RT][B];
    __shared__ double tl[RT][B];
    __shared__ double cl[RT];
    const int tile0 = rt * RT;
    for (int e = tid; e < RT * B; e += 256) {
        const int r = e / B, j = e % B;
        const int row = tile0 + r;
        if (row < l) {
            // fixed summation order; the loads of 8 partials are in flight together
            TA sum = own ? own[r][j] : (TA)0;
            for (int q0 = 0; !own && q0 < ksplit; q0 += 8) {
                TA pv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    pv[q] = (q0 + q < ksplit) ? ld_coherent(part + ((size_t)(q0 + q) * lda + row) * B + j) : (TA)0;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (q0 + q < ksplit) sum += pv[q];
            }
            const TU u = down<TU>((TA)(-0.5) * sum);
            U[(size_t)row * B + j] = u;
            ul[r][j] = (double)up<TA>(u);
            tl[r][j] = (double)up<TA>(T[(size_t)row * B + j]);
        } else {
            ul[r][j] = 0.0;
            tl[r][j] = 0.0;
        }
    }
    for (int r = tid; r < RT; r += 256) cl[r] = (tile0 + r) < l ? c[tile0 + r] : 0.0;
    if (tid == 0 && !own) counter_reset(tile_cnt + rt);
    __syncthreads();
    // this tile's contribution to H = T^T U and s = c^T U
    constexpr int EH = B * B + B;
    double *mine = red + (size_t)rt * EH;
    for (int e = tid; e < B * B; e += 256) {
        const int a = e / B, bb = e % B;
        double s = 0.0;
        for (int r = 0; r < RT; ++r) s += tl[r][a] * ul[r][bb];
        st_coherent(mine + e, s);
    }
    for (int j = tid; j < B; j += 256) {
        double s = 0.0;
        for (int r = 0; r < RT; ++r) s += cl[r] * ul[r][j];
        st_coherent(mine + B * B + j, s);
    }
    tree_reduce<kFan>(red, EH, rt, rowtiles, tree_cnt, st->Hs);
}

template <int M, int B>
__global__ __launch_bounds__(256) void k_gemm_vec(const ProbView *__restrict__ views, const int *__restrict__ off,
                                                  int nprob, int phase) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TT = typename Tr::TT;
    using TU = typename Tr::TU;
    using TW = typename Tr::TW;
    using Sh = GemmShape<TA, B>;
    constexpr int RW = Sh::RW, NV = Sh::NV, RT = Sh::RT;
    constexpr int TV = VecOf<TT, B>::v;

    const int pidx = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[pidx];
    SolveState *__restrict__ st = v.st;
    if (st->done || st->phase != phase) return;  // uniform: the schedule moved on
    const int vb = blockIdx.x - off[pidx];
    const int l = v.l, lda = v.lda;
    const int rowtiles = v.gemm_rowtiles[M];
    const int ksplit = v.gemm_ksplit[M];
    const int kchunk = v.gemm_kchunk[M];
    const TW *__restrict__ W = (const TW *)v.W[M];
    const TT *__restrict__ T = (const TT *)v.T;
    TA *__restrict__ part = (TA *)v.gpart;
    TU *__restrict__ U = (TU *)v.U;
    const double *__restrict__ c = v.c[M];
    double *__restrict__ red = v.red_gemm;
    unsigned *__restrict__ tile_cnt = v.tile_cnt;
    unsigned *__restrict__ tree_cnt = v.gemm_cnt;

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int rt = vb % rowtiles;
    const int ks = vb / rowtiles;
    const int r0 = rt * RT + wave * RW;
    const int kbeg = ks * kchunk;
    const int kend = min(lda, kbeg + kchunk);

    TA acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = (TA)0;

    // the loads of step k0 + 64 are issued before the arithmetic of step k0
    // (registers), so a step's W rows and T row are in flight while the
    // previous one is multiplied
    TA w[RW];
    Pack<TT, TV> tv[B / TV];
    auto load_step = [&](int k0) {
        const int k = k0 + lane;  // < lda while k0 < kend (kend <= lda, lda % 64 == 0)
        const bool live = k0 < kend;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int row = r0 + r;
            w[r] = (live && row < l) ? up<TA>(W[(size_t)row * lda + k]) : (TA)0;
        }
        // rows of T past l are padding and never read (W's padding columns
        // are zero, but the stale bytes there need not be finite)
        const bool trow = live && k < l;
#pragma unroll
        for (int j0 = 0; j0 < B; j0 += TV) {
            if (trow) tv[j0 / TV] = ldp<TT, TV>(T + (size_t)k * B + j0);
            else {
#pragma unroll
                for (int jj = 0; jj < TV; ++jj) tv[j0 / TV].v[jj] = TT{};
            }
        }
    };
    load_step(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += 64) {
        TA wc[RW];
        Pack<TT, TV> tc[B / TV];
#pragma unroll
        for (int r = 0; r < RW; ++r) wc[r] = w[r];
#pragma unroll
        for (int q = 0; q < B / TV; ++q) tc[q] = tv[q];
        load_step(k0 + 64);
#pragma unroll
        for (int j0 = 0; j0 < B; j0 += TV) {
#pragma unroll
            for (int jj = 0; jj < TV; ++jj) {
                const TA t = up<TA>(tc[j0 / TV].v[jj]);
#pragma unroll
                for (int r = 0; r < RW; ++r) acc[r * B + j0 + jj] += wc[r] * t;
            }
        }
    }
    int idx = 0;
    ReduceScatter<TA, NV, 32>::run(acc, lane, idx);
    constexpr int GROUP = 64 / NV;  // lanes sharing one value index
    if (ksplit == 1) {
        // uniform: the block holds the whole K range of its rows
        __shared__ TA own[RT][B];
        if ((lane % GROUP) == 0) own[wave * RW + idx / B][idx % B] = acc[0];
        __syncthreads();
        gemm_tile_finish<M, B, RT>(v, st, rt, rowtiles, ksplit, own);
        return;
    }
    if ((lane % GROUP) == 0) {
        const int row = r0 + idx / B;
        const int j = idx % B;
        if (row < l) st_coherent(part + ((size_t)ks * lda + row) * B + j, acc[0]);
    }

    gemm_tile_finish<M, B, RT>(v, st, rt, rowtiles, ksplit);
}

// ---------------------------------------------------------------------------
// Matrix-core variant (bf16 and float32 arithmetic, widths 16 and 32).  A
// block owns 64 rows of U (16 per wave) and a K range; each step stages a
// 64 x 64 slice of W (coalesced 16-byte loads) and the matching 64 x B slice
// of T (transposed, so that both MFMA operands are contiguous) in LDS, then
// every wave runs 16 x 16 tiles on the matrix cores:
//   float32: v_mfma_f32_16x16x4f32, lane l supplies A[l%16][l/16], B[l/16][l%16]
//   bf16:    v_mfma_f32_16x16x32_bf16, lane l supplies 8 consecutive k of
//            row l%16 of A and of column l%16 of B (k offset 8 (l/16))
// and holds D[4 (l/16) + r][l%16] in element r (both instructions);
//   float64 accumulation (the certification phase, float32 or float64 W
//   widened on load): v_mfma_f64_16x16x4f64, operands as for float32, D
//   element r of lane l is D[l/16 + 4 r][l%16].
// The split-K partials and the tile finish are those of k_gemm_vec.
// ---------------------------------------------------------------------------
typedef float gm_f4 __attribute__((ext_vector_type(4)));
typedef double gm_d4 __attribute__((ext_vector_type(4)));
typedef __bf16 gm_bf8 __attribute__((ext_vector_type(8)));

constexpr int kMfmaRows = 64;  // rows of U per block
constexpr int kMfmaK = 64;     // K per staged step

bool gemm_mfma(Mode, int B) { return B == 16 || B == 32; }

template <int M, int B>
__global__ __launch_bounds__(256) void k_gemm_mfma(const ProbView *__restrict__ views, const int *__restrict__ off,
                                                   int nprob, int phase) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TT = typename Tr::TT;
    using TW = typename Tr::TW;
    constexpr bool BF = (M == MODE_BF16);
    constexpr bool F64 = sizeof(TA) == 8;
    using AccV = typename std::conditional<F64, gm_d4, gm_f4>::type;
    constexpr int KS = kMfmaK, RT = kMfmaRows, NT = B / 16;
    constexpr int EPV = 16 / (int)sizeof(TW);  // elements per 16-byte load
    constexpr int PAD = EPV;                   // keeps 16-byte alignment of rows
    __shared__ __attribute__((aligned(16))) TW Ws[RT][KS + PAD];
    __shared__ __attribute__((aligned(16))) TT Ts[B][KS + PAD];  // transposed: Ts[j][k]

    const int pidx = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[pidx];
    SolveState *__restrict__ st = v.st;
    if (st->done || st->phase != phase) return;  // uniform: the schedule moved on
    const int vb = blockIdx.x - off[pidx];
    const int l = v.l, lda = v.lda;
    const int rowtiles = v.gemm_rowtiles[M];
    const int ksplit = v.gemm_ksplit[M];
    const int kchunk = v.gemm_kchunk[M];
    const TW *__restrict__ W = (const TW *)v.W[M];
    const TT *__restrict__ T = (const TT *)v.T;
    TA *__restrict__ part = (TA *)v.gpart;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int rt = vb % rowtiles, ks = vb / rowtiles;
    const int r0 = rt * RT;
    const int kbeg = ks * kchunk, kend = min(lda, kbeg + kchunk);

    AccV acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = AccV{0, 0, 0, 0};

    // W slices are loaded one step ahead (registers), so the next slice is in
    // flight while the matrix cores work on the current one
    constexpr int PPR = KS / EPV;                 // 16-byte pieces per row
    constexpr int NPC = RT * PPR / 256;           // pieces per thread
    static_assert(RT * PPR % 256 == 0, "whole pieces per thread");
    Pack<TW, EPV> wnext[NPC];
    auto load_w = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NPC; ++q) {
            const int idx = tid + 256 * q;
            const int r = idx / PPR, pc = idx % PPR;
            const int row = r0 + r;
            if (row < l && k0 < kend) {
                wnext[q] = ldp<TW, EPV>(W + (size_t)row * lda + k0 + pc * EPV);  // k0 + KS <= lda
            } else {
#pragma unroll
                for (int e = 0; e < EPV; ++e) wnext[q].v[e] = TW{};
            }
        }
    };
    // the T slice (KS x B, read transposed into LDS) travels with its W
    // slice, so a step waits on no load of its own (a second slice in
    // flight measured no faster)
    constexpr int NTP = KS * B / 256;  // T elements per thread
    static_assert(KS * B % 256 == 0, "whole T elements per thread");
    TT tnext[NTP];
    auto load_t = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NTP; ++q) {
            const int idx = tid + 256 * q;
            const int k = k0 + idx / B;
            // rows of T past l are padding and read as zero
            tnext[q] = (k0 < kend && k < l) ? T[(size_t)k * B + idx % B] : TT{};
        }
    };
    load_w(kbeg);
    load_t(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += KS) {
#pragma unroll
        for (int q = 0; q < NPC; ++q) {
            const int idx = tid + 256 * q;
            stp<TW, EPV>(&Ws[idx / PPR][(idx % PPR) * EPV], wnext[q]);
        }
#pragma unroll
        for (int q = 0; q < NTP; ++q) {
            const int idx = tid + 256 * q;
            Ts[idx % B][idx / B] = tnext[q];
        }
        load_w(k0 + KS);
        load_t(k0 + KS);
        __syncthreads();
        const int arow = 16 * w + (lane & 15);
        if constexpr (BF) {
#pragma unroll
            for (int s = 0; s < KS / 32; ++s) {
                const int kk = 32 * s + 8 * (lane >> 4);
                const gm_bf8 a = *reinterpret_cast<const gm_bf8 *>(&Ws[arow][kk]);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const gm_bf8 b = *reinterpret_cast<const gm_bf8 *>(&Ts[16 * t + (lane & 15)][kk]);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
                }
            }
        } else if constexpr (F64) {
#pragma unroll
            for (int s = 0; s < KS / 4; ++s) {
                const int kk = 4 * s + (lane >> 4);
                const double a = (double)Ws[arow][kk];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, (double)Ts[16 * t + (lane & 15)][kk], acc[t], 0, 0,
                                                                  0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < KS / 4; ++s) {
                const int kk = 4 * s + (lane >> 4);
                const float a = Ws[arow][kk];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, (float)Ts[16 * t + (lane & 15)][kk], acc[t], 0, 0,
                                                                  0);
            }
        }
        __syncthreads();
    }
    // partial U tile of this K range
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = r0 + 16 * w + (F64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
            const int j = 16 * t + (lane & 15);
            if (row < l) st_coherent(part + ((size_t)ks * lda + row) * B + j, (TA)acc[t][r]);
        }
    }
    gemm_tile_finish<M, B, RT>(v, st, rt, rowtiles, ksplit);
}

#define SBMDS_DISPATCH_B2(B_, CALL)                      \
    switch (B_) {                                        \
        case 4: { constexpr int BB = 4; CALL; } break;    \
        case 8: { constexpr int BB = 8; CALL; } break;    \
        case 16: { constexpr int BB = 16; CALL; } break;  \
        case 32: { constexpr int BB = 32; CALL; } break;  \
        case 64: { constexpr int BB = 64; CALL; } break;  \
        default: return hipErrorInvalidValue;            \
    }

hipError_t launch_gemm(Mode m, const Batch &bt, int phase, hipStream_t s) {
    if (bt.gemm_sym[m]) return launch_gemm_sym(m, bt, phase, s);
    const int grid = bt.total[BK_GEMM][m];
    if (grid <= 0) return hipErrorInvalidValue;
    const int *off = bt.off(BK_GEMM, m);
    switch (m) {
        case MODE_BF16: { constexpr int MM = MODE_BF16; SBMDS_DISPATCH_B2(bt.B, {
            if constexpr (BB == 16 || BB == 32) {
                if (bt.gemm_mfma[MM]) hipLaunchKernelGGL((k_gemm_mfma<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
                else hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
            } else {
                hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
            }
            return hipGetLastError(); }); } break;
        case MODE_FP32: { constexpr int MM = MODE_FP32; SBMDS_DISPATCH_B2(bt.B, {
            if constexpr (BB == 16 || BB == 32) {
                if (bt.gemm_mfma[MM]) hipLaunchKernelGGL((k_gemm_mfma<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
                else hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
            } else {
                hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
            }
            return hipGetLastError(); }); } break;
        case MODE_F64ACC: { constexpr int MM = MODE_F64ACC; SBMDS_DISPATCH_B2(bt.B, {
            if constexpr (BB == 16 || BB == 32) {
                if (bt.gemm_mfma[MM]) hipLaunchKernelGGL((k_gemm_mfma<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
                else hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
            } else {
                hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
            }
            return hipGetLastError(); }); } break;
        case MODE_FP64: { constexpr int MM = MODE_FP64; SBMDS_DISPATCH_B2(bt.B, {
            if constexpr (BB == 16 || BB == 32) {
                if (bt.gemm_mfma[MM]) hipLaunchKernelGGL((k_gemm_mfma<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
                else hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
            } else {
                hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase);
            }
            return hipGetLastError(); }); } break;
        default: break;
    }
    return hipErrorInvalidValue;
}

double gemm_bytes(Mode m, const DevProblem &p, bool packed) {
    const double sw = m == MODE_BF16 ? 2.0 : (m == MODE_FP64 ? 8.0 : 4.0);
    const double st = m == MODE_BF16 ? 2.0 : (m == MODE_FP32 ? 4.0 : 8.0);
    const double su = (m == MODE_F64ACC || m == MODE_FP64) ? 8.0 : 4.0;
    // the packed product reads the upper triangle: l (l + 1) / 2 elements
    const double welems = packed ? 0.5 * (double)p.l * (p.l + 1) : (double)p.l * p.l;
    return welems * sw + (double)p.l * p.B * (st + su);
}

}  // namespace sbmds
