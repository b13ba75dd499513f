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
#include "sbmds_common.h"

namespace sbmds {

template <typename TA, int B>
struct GemmShape {
    // rows per wave: keep RW * B accumulators at 64 (float) / 32..64 (double)
    static constexpr int NVMAX = sizeof(TA) == 4 ? 64 : (B >= 64 ? 64 : 32);
    static constexpr int RW = (NVMAX / B) > 0 ? (NVMAX / B) : 1;
    static constexpr int NV = RW * B;
    static constexpr int RT = 4 * RW;  // rows per block (4 waves)
};

int gemm_rows_per_tile(Mode m, int B) {
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

    for (int k0 = kbeg; k0 < kend; k0 += 64) {
        const int k = k0 + lane;  // < lda always (kend <= lda, lda % 64 == 0)
        TA w[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int row = r0 + r;
            w[r] = row < l ? up<TA>(W[(size_t)row * lda + k]) : (TA)0;
        }
        // rows of T past l are padding; they are never read (W's padding
        // columns are zero, but the stale bytes there need not be finite)
        if (k < l) {
            const TT *trow = T + (size_t)k * B;
#pragma unroll
            for (int j0 = 0; j0 < B; j0 += TV) {
                Pack<TT, TV> tv = ldp<TT, TV>(trow + j0);
#pragma unroll
                for (int jj = 0; jj < TV; ++jj) {
                    const TA t = up<TA>(tv.v[jj]);
#pragma unroll
                    for (int r = 0; r < RW; ++r) acc[r * B + j0 + jj] += w[r] * t;
                }
            }
        }
    }
    int idx = 0;
    ReduceScatter<TA, NV, 32>::run(acc, lane, idx);
    constexpr int GROUP = 64 / NV;  // lanes sharing one value index
    if ((lane % GROUP) == 0) {
        const int row = r0 + idx / B;
        const int j = idx % B;
        if (row < l) st_coherent(part + ((size_t)ks * lda + row) * B + j, acc[0]);
    }

    // ---- per-tile finish: the last of the ksplit blocks of this row tile
    if (!arrive_last(tile_cnt + rt, (unsigned)ksplit)) return;
    __shared__ double ul[RT][B];
    __shared__ double tl[RT][B];
    __shared__ double cl[RT];
    const int tile0 = rt * RT;
    for (int e = tid; e < RT * B; e += 256) {
        const int r = e / B, j = e % B;
        const int row = tile0 + r;
        if (row < l) {
            TA sum = (TA)0;
            for (int q = 0; q < ksplit; ++q) sum += ld_coherent(part + ((size_t)q * lda + row) * B + j);
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
    if (tid == 0) counter_reset(tile_cnt + rt);
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
    const int grid = bt.total[BK_GEMM][m];
    if (grid <= 0) return hipErrorInvalidValue;
    const int *off = bt.off(BK_GEMM, m);
    switch (m) {
        case MODE_BF16: { constexpr int MM = MODE_BF16; SBMDS_DISPATCH_B2(bt.B, hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase); return hipGetLastError()); } break;
        case MODE_FP32: { constexpr int MM = MODE_FP32; SBMDS_DISPATCH_B2(bt.B, hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase); return hipGetLastError()); } break;
        case MODE_F64ACC: { constexpr int MM = MODE_F64ACC; SBMDS_DISPATCH_B2(bt.B, hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase); return hipGetLastError()); } break;
        case MODE_FP64: { constexpr int MM = MODE_FP64; SBMDS_DISPATCH_B2(bt.B, hipLaunchKernelGGL((k_gemm_vec<MM, BB>), dim3(grid), dim3(256), 0, s, bt.views, off, bt.nprob, phase); return hipGetLastError()); } break;
        default: break;
    }
    return hipErrorInvalidValue;
}

double gemm_bytes(Mode m, const DevProblem &p) {
    const double sw = m == MODE_BF16 ? 2.0 : (m == MODE_FP64 ? 8.0 : 4.0);
    const double st = m == MODE_BF16 ? 2.0 : (m == MODE_FP32 ? 4.0 : 8.0);
    const double su = (m == MODE_F64ACC || m == MODE_FP64) ? 8.0 : 4.0;
    return (double)p.l * p.l * sw + (double)p.l * p.B * (st + su);
}

}  // namespace sbmds
