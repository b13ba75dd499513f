// Dense landmark product U = -1/2 W T read from the upper triangle of W
// (Section 3.3's dense l x l factor; W holds squared distances, which are
// symmetric, and the input contract requires a symmetric W).
//
// Only the upper triangle is stored and streamed, so the dominant stream of
// an iteration at large l is half the bytes of the full matrix: a 64 x 64
// tile W_ij (i <= j) is read from HBM once and applied twice, U_i += W_ij T_j
// and, off the diagonal, U_j += W_ij^T T_i.
//
// Packed layout ("strips"): strip i holds rows 64i .. 64i+63 of W and their
// columns 64i .. lda-1, row-major with row length lda - 64i, starting at
// element 64 i lda - 2048 i (i - 1) (sym_strip_base).  Rows and columns past
// l are zero.
//
// Work split: the tiles of the upper triangle are grouped into regions of R
// tile rows x C tile columns (region (gr, gc) exists when it holds a tile
// with i <= j, i.e. gc >= floor(gr R / C); regions are numbered row by row).
// A block walks its region column by column, staging each W tile and the
// matching T slices in LDS and running both products on the matrix cores
// (float32: v_mfma_f32_16x16x4f32; float64 accumulation of the float32
// operator: v_mfma_f64_16x16x4f64, W widened on the fly).  The partial U_i
// of each of its R tile rows is kept (in LDS) across the region's columns;
// the transposed partial of each column is complete after that
// column's R tiles.  Both go to slots of the partial buffer (R + C slots of
// 64 x B per region).  A second launch sums, for every 64-row tile of U, its
// slots in a fixed order (bitwise reproducible), applies -1/2, stores U and
// reduces its contributions to H = T^T U and s = c^T U over all tiles.
#include <type_traits>

#include "sbmds_common.h"
#include "sbmds_dense_sym.h"

namespace sbmds {

namespace {

typedef float gs_f4 __attribute__((ext_vector_type(4)));
typedef double gs_d4 __attribute__((ext_vector_type(4)));
typedef float gs_f4v __attribute__((ext_vector_type(4)));

// Region rows per mode and width (the row partials of a block take
// R x 64 x B accumulators of LDS).
template <int M, int B>
struct SymShape {
    static constexpr bool F64 = (M == MODE_F64ACC);
    static constexpr int BP = B < 16 ? 16 : B;  // matrix-core width (B = 8 padded with zero columns)
    static constexpr int NTC = BP / 16;
    static constexpr int R = 4;
};

}  // namespace

int sym_region_rows(Mode, int) { return 4; }

bool sym_supported(Mode m, int B) { return (m == MODE_FP32 || m == MODE_F64ACC) && (B == 8 || B == 16 || B == 32); }

// LDS layout of a staged 64 x 64 W tile: rows of 64 floats, the sixteen
// 16-byte chunks of row r permuted by chunk ^ swz(r).  Each lane feeds the
// matrix cores 16 consecutive k (lanes 16q .. 16q+15 take k = 16q .. 16q+15;
// the summation over k is the same in any order), so the row product reads
// its W operand and both products their T operand as 16-byte pieces, eight
// lanes of distinct chunks per LDS cycle; the transposed product reads W by
// columns, 4 bytes per lane, rows k and k + 16 falling into opposite halves
// of the banks.  No LDS bank is hit twice in one cycle by either pattern.
__device__ __forceinline__ int swz(int r) { return (((r & 1) << 2) | ((r >> 1) & 3)) ^ (((r >> 4) & 1) << 2); }
__device__ __forceinline__ int wpos(int r, int c) { return r * 64 + ((((c >> 2) ^ swz(r)) & 15) << 2) + (c & 3); }

template <int M, int B>
__global__ __launch_bounds__(256) void k_gemm_sym(const ProbView *__restrict__ views, const int *__restrict__ off,
                                                  int nprob, int phase) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TT = typename Tr::TT;
    using Sh = SymShape<M, B>;
    constexpr bool F64 = Sh::F64;
    constexpr int BP = Sh::BP, NTC = Sh::NTC, R = Sh::R;
    using AccV = typename std::conditional<F64, gs_d4, gs_f4>::type;
    constexpr int TSP = 64 + (F64 ? 2 : 4);  // LDS row stride of a transposed T slice
    __shared__ __attribute__((aligned(16))) float Ws[64 * 64];
    __shared__ __attribute__((aligned(16))) TT Tjs[BP * TSP];  // T_j transposed: [column][k]
    __shared__ __attribute__((aligned(16))) TT Tis[BP * TSP];  // T_i transposed
    // row partials: R tiles x (this wave's 16 rows) x NTC accumulator tiles,
    // kept between the columns of the walk (each lane its own values)
    __shared__ __attribute__((aligned(16))) AccV accs[R][4][NTC][64];

    const int pidx = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[pidx];
    const SolveState *__restrict__ st = v.st;
    if (st->done || st->phase != phase) return;  // uniform: the schedule moved on
    const int vb = blockIdx.x - off[pidx];
    const int l = v.l, lda = v.lda, nt = lda / 64;
    const int C = v.sym_c[M];
    const int ngc = (nt + C - 1) / C;
    int gr = 0, q0 = vb;
    for (;;) {
        const int cnt = ngc - sym_gcmin(gr, R, C);
        if (q0 < cnt) break;
        q0 -= cnt;
        ++gr;
    }
    const int gc = sym_gcmin(gr, R, C) + q0;
    const int i0 = gr * R;
    const int nrow = min(R, nt - i0);
    const int jbeg = gc * C, jend = min(jbeg + C, nt);
    const int jfirst = max(jbeg, i0);
    const float *__restrict__ Wp = v.Wp;
    const TT *__restrict__ T = (const TT *)v.T;
    TA *__restrict__ part = (TA *)v.gpart;
    const size_t slot0 = (size_t)vb * (R + C);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

    auto put = [&](size_t slot, const AccV *acc) {
        TA *dst = part + slot * 64 * B;
#pragma unroll
        for (int t = 0; t < NTC; ++t) {
            const int col = 16 * t + (lane & 15);
            if (col < B) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * w + (F64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
                    dst[row * B + col] = (TA)acc[t][r];
                }
            }
        }
    };
    AccV zero[NTC];
#pragma unroll
    for (int t = 0; t < NTC; ++t) zero[t] = AccV{0, 0, 0, 0};
    // columns of the region left of the diagonal hold no stored tile
    for (int j = jbeg; j < jfirst && j < jend; ++j) put(slot0 + R + (j - jbeg), zero);
    if (B < BP) {
        // zero padding columns of the matrix-core operand (never restaged)
        for (int e = tid; e < (BP - B) * TSP; e += 256) {
            Tjs[B * TSP + e] = TT{};
            Tis[B * TSP + e] = TT{};
        }
    }
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int t = 0; t < NTC; ++t) accs[q][w][t][lane] = AccV{0, 0, 0, 0};

    // ---- the walk: columns j of the region, in each the rows i0 + q with
    // i0 + q <= j; tiles are prefetched (registers) two steps ahead
    auto nq_of = [&](int j) { return min(nrow, j - i0 + 1); };
    auto advance = [&](int &j, int &q) {
        if (++q >= nq_of(j)) {
            q = 0;
            ++j;
        }
    };
    constexpr int NWP = 64 * 64 / 4 / 256;  // 16-byte pieces of the W tile per thread
    constexpr int NTE = 64 * B / 256 > 0 ? 64 * B / 256 : 1;  // T elements per thread
    static_assert(64 * B % 256 == 0, "whole T elements per thread");
    struct Set {
        gs_f4v w[NWP];
        TT ti[NTE], tj[NTE];
    };
    auto load_t = [&](TT *dst, int tile) {
#pragma unroll
        for (int p = 0; p < NTE; ++p) {
            const int idx = tid + 256 * p;
            const int k = 64 * tile + idx / B;
            // rows of T past l are padding (possibly stale): read as zero
            dst[p] = k < l ? T[(size_t)k * B + idx % B] : TT{};
        }
    };
    auto load = [&](Set &st_, int j, int q) {
        const int i = i0 + q;
        const int64_t base = sym_strip_base(i, lda) + (int64_t)(j - i) * 64;
        const int64_t len = lda - 64 * i;
#pragma unroll
        for (int p = 0; p < NWP; ++p) {
            const int idx = tid + 256 * p;
            st_.w[p] = *reinterpret_cast<const gs_f4v *>(Wp + base + (idx >> 4) * len + 4 * (idx & 15));
        }
        load_t(st_.ti, i);
        if (q == 0) load_t(st_.tj, j);
    };
    auto stage_t = [&](TT *lds, const TT *src) {
#pragma unroll
        for (int p = 0; p < NTE; ++p) {
            const int idx = tid + 256 * p;
            lds[(idx % B) * TSP + idx / B] = src[p];
        }
    };

    const int arow = 16 * w + (lane & 15);  // row of W (row product) / column of W (transposed product)
    const int sw_row = swz(arow);
    const int qk = lane >> 4;               // this lane feeds k = 16 qk .. 16 qk + 15
    AccV accc[NTC];
#pragma unroll
    for (int t = 0; t < NTC; ++t) accc[t] = AccV{0, 0, 0, 0};
    int cj = jfirst, cq = 0;  // tile being multiplied
    int pj = jfirst, pq = 0;  // next tile to prefetch
    Set s0, s1;
    if (pj < jend) {
        load(s0, pj, pq);
        advance(pj, pq);
    }
    if (pj < jend) {
        load(s1, pj, pq);
        advance(pj, pq);
    }
    // 16 consecutive k of one row of a transposed T slice in LDS (16-byte pieces)
    auto t16 = [&](const TT *lds, int col, TT (&out)[16]) {
        constexpr int PER = 16 / (int)sizeof(TT);
        typedef TT V __attribute__((ext_vector_type(PER)));
        const V *src = reinterpret_cast<const V *>(lds + col * TSP + 16 * qk);
#pragma unroll
        for (int u = 0; u < 16 / PER; ++u) {
            const V x = src[u];
#pragma unroll
            for (int v = 0; v < PER; ++v) out[u * PER + v] = x[v];
        }
    };
    auto step = [&](Set &cur) {
        // stage the tile (the previous step's reads are done)
#pragma unroll
        for (int p = 0; p < NWP; ++p) {
            const int idx = tid + 256 * p;
            const int r = idx >> 4, c4 = idx & 15;
            *reinterpret_cast<gs_f4v *>(&Ws[r * 64 + ((c4 ^ swz(r)) << 2)]) = cur.w[p];
        }
        stage_t(Tis, cur.ti);
        if (cq == 0) stage_t(Tjs, cur.tj);
        // this set's registers now take the tile two steps ahead
        if (pj < jend) {
            load(cur, pj, pq);
            advance(pj, pq);
        }
        __syncthreads();
        AccV acc[NTC];
#pragma unroll
        for (int t = 0; t < NTC; ++t) acc[t] = accs[cq][w][t][lane];
        // this lane's 16 W values of the row product (row arow, k = 16 qk ..)
        float ar[16];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const gs_f4v x = *reinterpret_cast<const gs_f4v *>(&Ws[arow * 64 + ((((4 * qk + u) ^ sw_row) & 15) << 2)]);
#pragma unroll
            for (int v = 0; v < 4; ++v) ar[4 * u + v] = x[v];
        }
        const bool offdiag = i0 + cq < cj;
#pragma unroll
        for (int t = 0; t < NTC; ++t) {
            TT bj[16];
            t16(Tjs, 16 * t + (lane & 15), bj);
#pragma unroll
            for (int s_ = 0; s_ < 16; ++s_) {
                if constexpr (F64)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ar[s_], bj[s_], acc[t], 0, 0, 0);
                else
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[s_], bj[s_], acc[t], 0, 0, 0);
            }
        }
        if (offdiag) {
            // U_j += W_ij^T T_i: W read by columns (column arow, rows 16 qk ..)
            float ac[16];
#pragma unroll
            for (int s_ = 0; s_ < 16; ++s_) ac[s_] = Ws[wpos(16 * qk + s_, arow)];
#pragma unroll
            for (int t = 0; t < NTC; ++t) {
                TT bi[16];
                t16(Tis, 16 * t + (lane & 15), bi);
#pragma unroll
                for (int s_ = 0; s_ < 16; ++s_) {
                    if constexpr (F64)
                        accc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ac[s_], bi[s_], accc[t], 0, 0, 0);
                    else
                        accc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[s_], bi[s_], accc[t], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NTC; ++t) accs[cq][w][t][lane] = acc[t];
        __syncthreads();
        if (cq == nq_of(cj) - 1) {
            // the column's transposed partial is complete
            put(slot0 + R + (cj - jbeg), accc);
#pragma unroll
            for (int t = 0; t < NTC; ++t) accc[t] = AccV{0, 0, 0, 0};
        }
        advance(cj, cq);
    };
    while (cj < jend) {
        step(s0);
        if (cj >= jend) break;
        step(s1);
    }
    for (int q = 0; q < nrow; ++q) {
        AccV acc[NTC];
#pragma unroll
        for (int t = 0; t < NTC; ++t) acc[t] = accs[q][w][t][lane];
        put(slot0 + q, acc);
    }
}

// Per 64-row tile t of U: the sum of its slots (row side: regions (t / R,
// gc) for every gc of that region row; column side: regions (gr, t / C) for
// every gr of that region column), in that fixed order; then U = -1/2 sum,
// and the tile's contributions to H and s, reduced over tiles.
// Threads of the finish launch: one per element of a 64 x B tile (at most
// 1024), each summing its element over the slot list with 16 loads in flight.
template <int B>
struct SymFinish {
    static constexpr int NT = 64 * B < 1024 ? 64 * B : 1024;
    static constexpr int EPT = 64 * B / NT;
};

template <int M, int B>
__global__ __launch_bounds__(SymFinish<B>::NT) void k_gemm_sym_finish(const ProbView *__restrict__ views,
                                                                      const int *__restrict__ off, int nprob,
                                                                      int phase) {
    using Tr = Traits<M>;
    using TA = typename Tr::TA;
    using TT = typename Tr::TT;
    using TU = typename Tr::TU;
    constexpr int R = SymShape<M, B>::R;
    constexpr int NT = SymFinish<B>::NT, EPT = SymFinish<B>::EPT;
    constexpr int QF = 16;  // slot loads in flight per element
    __shared__ int slots[2 * kSymMaxGroups];
    __shared__ int base[kSymMaxGroups + 1];
    __shared__ int nslot;
    __shared__ double ul[64][B];
    __shared__ double tl[64][B];
    __shared__ double cl[64];

    const int pidx = find_problem(off, nprob, blockIdx.x);
    const ProbView &v = views[pidx];
    SolveState *__restrict__ st = v.st;
    if (st->done || st->phase != phase) return;  // uniform
    const int t = blockIdx.x - off[pidx];
    const int l = v.l, lda = v.lda, nt = lda / 64;
    const int C = v.sym_c[M];
    const int ngr = (nt + R - 1) / R, ngc = (nt + C - 1) / C;
    const int tid = threadIdx.x;
    // region numbering: base[g] = first region of region row g
    for (int g = tid; g < ngr; g += NT) base[g + 1] = ngc - sym_gcmin(g, R, C);
    __syncthreads();
    if (tid == 0) {
        base[0] = 0;
        for (int g = 0; g < ngr; ++g) base[g + 1] += base[g];
        const int gr = t / R, gcol = t / C;
        int n = 0;
        const int gm = sym_gcmin(gr, R, C);
        for (int gc = gm; gc < ngc; ++gc) slots[n++] = (base[gr] + gc - gm) * (R + C) + (t - gr * R);
        for (int g = 0; g < ngr; ++g) {
            const int gmg = sym_gcmin(g, R, C);
            if (gmg <= gcol) slots[n++] = (base[g] + gcol - gmg) * (R + C) + R + (t - gcol * C);
        }
        nslot = n;
    }
    __syncthreads();
    const int ns = nslot;
    const TA *__restrict__ part = (const TA *)v.gpart;
    const TT *__restrict__ T = (const TT *)v.T;
    TU *__restrict__ U = (TU *)v.U;
    const double *__restrict__ c = v.c[M];
    const int tile0 = 64 * t;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * NT;
        const int r = e / B, j = e % B;
        const int row = tile0 + r;
        TA sum = (TA)0;
        for (int q0 = 0; q0 < ns; q0 += QF) {
            TA pv[QF];
#pragma unroll
            for (int u = 0; u < QF; ++u) pv[u] = (q0 + u < ns) ? part[(size_t)slots[q0 + u] * 64 * B + e] : (TA)0;
#pragma unroll
            for (int u = 0; u < QF; ++u)
                if (q0 + u < ns) sum += pv[u];
        }
        if (row < l) {
            const TU u = down<TU>((TA)(-0.5) * sum);
            U[(size_t)row * B + j] = u;
            ul[r][j] = (double)up<TA>(u);
            tl[r][j] = (double)up<TA>(T[(size_t)row * B + j]);
        } else {
            ul[r][j] = 0.0;
            tl[r][j] = 0.0;
        }
    }
    for (int r = tid; r < 64; r += NT) cl[r] = (tile0 + r) < l ? c[tile0 + r] : 0.0;
    __syncthreads();
    constexpr int EH = B * B + B;
    double *red = v.red_gemm;
    double *mine = red + (size_t)t * EH;
    for (int e = tid; e < B * B; e += NT) {
        const int a = e / B, bb = e % B;
        double s = 0.0;
        for (int r = 0; r < 64; ++r) s += tl[r][a] * ul[r][bb];
        st_coherent(mine + e, s);
    }
    for (int j = tid; j < B; j += NT) {
        double s = 0.0;
        for (int r = 0; r < 64; ++r) s += cl[r] * ul[r][j];
        st_coherent(mine + B * B + j, s);
    }
    tree_reduce<kFan>(red, EH, t, nt, v.gemm_cnt, st->Hs);
}

// Packs the upper triangle of a row-major l x lda float matrix into strips.
// Block (i, r): row r of strip i, columns 64i .. lda-1.
__global__ __launch_bounds__(256) void k_pack_sym(const float *__restrict__ W, int l, int lda,
                                                  float *__restrict__ Wp) {
    const int i = blockIdx.x, r = blockIdx.y;
    const int row = 64 * i + r;
    const int64_t len = lda - 64 * i;
    float *dst = Wp + sym_strip_base(i, lda) + (int64_t)r * len;
    const float *src = W + (size_t)row * lda + 64 * i;
    for (int64_t c4 = threadIdx.x; c4 < len / 4; c4 += 256) {
        gs_f4v x = gs_f4v{0.f, 0.f, 0.f, 0.f};
        if (row < l) x = *reinterpret_cast<const gs_f4v *>(src + 4 * c4);
        *reinterpret_cast<gs_f4v *>(dst + 4 * c4) = x;
    }
}

hipError_t launch_pack_sym(const float *W, int64_t l, int lda, float *Wp, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_sym, dim3(lda / 64, 64), dim3(256), 0, s, W, (int)l, lda, Wp);
    return hipGetLastError();
}

hipError_t launch_gemm_sym(Mode m, const Batch &bt, int phase, hipStream_t s) {
    const int g1 = bt.total[BK_GEMM][m], g2 = bt.total[BK_GEMMF][m];
    if (g1 <= 0 || g2 <= 0) return hipErrorInvalidValue;
    const int *o1 = bt.off(BK_GEMM, m), *o2 = bt.off(BK_GEMMF, m);
#define SBMDS_SYM_LAUNCH(MM, BB)                                                                              \
    do {                                                                                                      \
        hipLaunchKernelGGL((k_gemm_sym<MM, BB>), dim3(g1), dim3(256), 0, s, bt.views, o1, bt.nprob, phase);   \
        hipError_t e_ = hipGetLastError();                                                                    \
        if (e_ != hipSuccess) return e_;                                                                      \
        hipLaunchKernelGGL((k_gemm_sym_finish<MM, BB>), dim3(g2), dim3(SymFinish<BB>::NT), 0, s, bt.views, o2, \
                           bt.nprob, phase);                                                                  \
        return hipGetLastError();                                                                             \
    } while (0)
    if (m == MODE_FP32) {
        switch (bt.B) {
            case 8: SBMDS_SYM_LAUNCH(MODE_FP32, 8);
            case 16: SBMDS_SYM_LAUNCH(MODE_FP32, 16);
            case 32: SBMDS_SYM_LAUNCH(MODE_FP32, 32);
            default: break;
        }
    } else if (m == MODE_F64ACC) {
        switch (bt.B) {
            case 8: SBMDS_SYM_LAUNCH(MODE_F64ACC, 8);
            case 16: SBMDS_SYM_LAUNCH(MODE_F64ACC, 16);
            case 32: SBMDS_SYM_LAUNCH(MODE_F64ACC, 32);
            default: break;
        }
    }
#undef SBMDS_SYM_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace sbmds
