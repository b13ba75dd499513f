// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace sbmds {

// Arithmetic of one iteration.  Each mode fixes the storage type of the P
// values and of W, of the n x b block Y, of the l x b blocks T and U, and the
// accumulation type:
//   BF16   : P bf16, W bf16, Y bf16,  T bf16,  U f32, accumulate f32
//   FP32   : P f32,  W f32,  Y f32,   T f32,   U f32, accumulate f32
//   F64ACC : P f32,  W f32,  Y f64,   T f64,   U f64, accumulate f64
//            (float32 operator, float64 arithmetic: the certification pass)
//   FP64   : everything f64
enum Mode { MODE_BF16 = 0, MODE_FP32 = 1, MODE_F64ACC = 2, MODE_FP64 = 3, NUM_MODES = 4 };

inline int y_elem_bytes(Mode m) { return m == MODE_BF16 ? 2 : (m == MODE_FP32 ? 4 : 8); }

constexpr int kMaxB = 64;

// Device-resident state of the block solver for one problem.  Every array is
// sized for the widest block and indexed with the problem's kernel width B.
struct SolveState {
    double Hs[kMaxB * kMaxB + kMaxB];           // H = X^T B X (B x B row-major), then s = c^T U
    double Ge[kMaxB * (kMaxB + 1) / 2 + kMaxB]; // Y'^T Y' (packed upper triangle), then 1^T Y'
    double e_x[kMaxB];           // 1^T Y of the block the basis is built from
    double C[kMaxB * kMaxB];     // basis X = J Y C (row-major B x B)
    double Zmap[kMaxB * kMaxB];  // embedding Z = J Y Zmap (B x B, first k columns used)
    double zshift[kMaxB];        // e_x^T Zmap / n
    double theta[kMaxB];         // Ritz values, descending
    double res[kMaxB];           // ||B x_i - theta_i x_i||
    double bound[kMaxB];         // relative eigenvalue error bound per Ritz value
    double maxbound;             // max over the k wanted values
    double maxres;               // max over the k wanted values of res_i / |theta_i|
    int iter;
    int flags;                   // bit 0: Cholesky pivot repaired; bit 1: non-finite value
    int dead;                    // columns dropped after rank loss
    int nonpos;                  // wanted Ritz values <= 0
    int sweeps;                  // Jacobi sweeps of the last Rayleigh-Ritz step
    // ---- device-side control of the precision schedule (see PhaseRule)
    int ycur;                    // Y buffer holding the current block
    int zbuf;                    // Y buffer the last Rayleigh-Ritz basis came from
    int zmode;                   // Mode of that buffer
    int phase;                   // running phase of the schedule
    int done;                    // 1 once the stopping rule is met
    int pending_convert;         // a phase just ended; the next one converts Y first
    int phase_iters;             // iterations run in the current phase
    int total_iters;             // iterations run in this solve
    int iters[4];                // iterations run per phase
    int sweeps_total;            // Jacobi sweeps in this solve
    int ymode;                   // Mode of the current block Y[ycur]
    int refill;                  // dead columns were just refilled: Y0 awaits its Gram and CholQR
    double hist[4];              // maxres of the latest iterations of the phase
};

// What the Rayleigh-Ritz step decides after an iteration of phase `phase`.
// A final phase ends the solve once maxbound <= tol; other phases hand over
// to the next one once maxres <= floor_res, once the residual stalls
// (no 30% gain over three iterations) or after `cap` iterations.
struct PhaseRule {
    int phase;
    int is_final;
    int cap;
    int mode;
    double floor_res;
    double tol;
};

enum SolveFlags { SF_REPAIRED = 1, SF_NONFINITE = 2 };

// `init` argument of the Rayleigh-Ritz kernels: an iteration's step, the
// CholQR of a new start block (resets the solve's control state), or the
// CholQR of a block whose dead columns were refilled (keeps it).
enum RRInit { RR_STEP = 0, RR_START = 1, RR_REFILL = 2 };

// Bytes of SolveState from `theta` to the end: what the host reads after
// each round (the Rayleigh-Ritz kernels write it to pinned host memory).
constexpr size_t kSummaryOffset = offsetof(SolveState, theta);
constexpr size_t kSummaryBytes = sizeof(SolveState) - offsetof(SolveState, theta);

// Buffers and sizes of one problem on the device (host-side bookkeeping).
struct DevProblem {
    int64_t n = 0, l = 0, nnz = 0;
    int lda = 0;          // padded row stride of W (multiple of 64), also rows of T/U
    int b = 0, B = 0, k = 0;
    // CSR of P and of P^T
    int32_t *rp = nullptr, *ci = nullptr, *rpT = nullptr, *ciT = nullptr;
    void *val[NUM_MODES] = {};   // P values per mode (aliases where modes share)
    void *valT[NUM_MODES] = {};
    void *W[NUM_MODES] = {};     // padded l x lda
    float *Wp = nullptr;         // packed upper triangle of the float32 W (large l), or NULL
    double *c[NUM_MODES] = {};   // P^T 1 in float64 from that mode's values
    void *Y[2] = {};             // n x B, sized for 8-byte elements
    void *T = nullptr, *U = nullptr;  // lda x B, 8-byte elements
    // reduction scratch (see tree_reduce): split-K partials of the dense
    // product, tree levels and arrival counters
    void *gpart = nullptr;       // [ksplit][lda][B] (8-byte elements)
    double *red_gemm = nullptr;  // H/s partials per row tile and tree levels
    double *red_spmm = nullptr;  // Gram/column-sum partials per block and tree levels
    unsigned *tile_cnt = nullptr, *gemm_cnt = nullptr, *spmm_cnt = nullptr;
    int max_rowtiles = 0, max_ksplit = 0, max_spmm_blocks = 0;
    // push form of the transposed product (see prep_push_*), or pb == NULL
    int32_t *pb = nullptr, *pe = nullptr, *qp = nullptr, *ql = nullptr;
    uint8_t *pvl = nullptr;
    void *pval[NUM_MODES] = {};  // values in pair order per mode
    void *ppart = nullptr;       // [npairs][B] partial rows (8-byte elements)
    int64_t npairs = 0;
    int nvb = 0;                 // vertex blocks
    SolveState *st = nullptr;
    const void *X0 = nullptr;    // device copy of a user start block
    std::vector<int32_t> lperm;  // internal landmark order: internal j is caller's landmark lperm[j]
};

// Tunable launch choices of a batch in one mode (chosen by the autotuner or
// by the defaults): SpMM block cap, dense-product kernel (matrix cores or
// vector ALU) and its target block count, and waves per landmark row of the
// transposed SpMM.
struct Tune {
    int spmm_cap = 256;
    int gemm_mfma = 0;
    int gemm_target = 1024;
    int gemm_sym = 0;   // dense product from the packed upper triangle of W
    int sym_c = 16;     // its region width in 64-column tiles
    int spmmt_wpr = 4;
    int spmm_wpe = 4;  // row-split SpMM (widths 8-32): 4 = fused Rayleigh-Ritz form, 8 = two blocks per CU
};

// Launch geometry of one problem in one mode (derived from a Tune).
struct LaunchCfg {
    int spmm_blocks = 0;   // grid of the row-split SpMM (grid-stride)
    int gemm_rt = 0;       // rows per dense-product tile (fixed by mode and B)
    int gemm_ksplit = 1;   // K splits of the dense product
    int gemm_kchunk = 64;  // K range per split (multiple of 64)
};

// What one launch sees of one problem (device array, one entry per problem).
struct ProbView {
    int n, l, nnz, lda;
    const int32_t *rp, *ci, *rpT, *ciT;
    const void *val[NUM_MODES];
    const void *valT[NUM_MODES];
    const void *W[NUM_MODES];
    const float *Wp;       // packed upper triangle of W (float32), or NULL
    const double *c[NUM_MODES];
    void *Y0, *Y1, *T, *U, *gpart;
    double *red_gemm, *red_spmm;
    unsigned *tile_cnt, *gemm_cnt, *spmm_cnt;
    SolveState *st;
    const void *X0;
    int64_t zoff;          // element offset of this problem's rows in the output Z
    int64_t loff;          // row offset of this problem's landmarks in per-landmark arrays
    void *host_sum;        // pinned host copy of the SolveState tail from `theta` on (device pointer)
    int spmm_blocks[NUM_MODES];
    int gemm_rowtiles[NUM_MODES];
    int gemm_ksplit[NUM_MODES];
    int gemm_kchunk[NUM_MODES];
    int sym_c[NUM_MODES];  // region width (tiles) of the packed dense product
    // push form of the transposed product
    const int32_t *pb, *pe, *qp, *ql;
    const uint8_t *pvl;
    const void *pval[NUM_MODES];
    void *ppart;
};

// Block-to-problem tables: for each kind of launch and mode, off[p] is the
// first block of problem p and off[nprob] the grid size.
enum BlockKind {
    BK_SPMM = 0, BK_SPMMT = 1, BK_GEMM = 2, BK_ELEM_NB = 3, BK_ELEM_N = 4, BK_ELEM_LB = 5,
    BK_GEMMF = 6,  // 64-row tiles of U (finish launch of the packed dense product)
    BK_PUSH = 7,   // vertex blocks of the push-form transposed product
    BK_PUSHR = 8,  // landmark groups of its reduction
    NUM_BK = 9
};

// Host handle of a batch: every launch covers all problems of a context.
struct Batch {
    int nprob = 0;
    int B = 0, b = 0, k = 0;
    int64_t max_l = 0;                         // largest landmark count of the batch
    int spmmt_wpr[NUM_MODES] = {4, 4, 4, 4};  // waves per landmark row in the transposed SpMM
    int gemm_mfma[NUM_MODES] = {};             // dense product on the matrix cores
    int gemm_sym[NUM_MODES] = {};              // dense product from the packed upper triangle of W
    int spmm_wpe8[NUM_MODES] = {};             // row-split SpMM in its two-blocks-per-CU form
    int spmmt_push[NUM_MODES] = {};            // transposed SpMM in its push form
    ProbView *views = nullptr;   // device [nprob]
    int *offs = nullptr;         // device [NUM_BK][NUM_MODES][nprob + 1]
    int total[NUM_BK][NUM_MODES] = {};
    const int *off(BlockKind kd, Mode m) const { return offs + ((size_t)kd * NUM_MODES + m) * (nprob + 1); }
};

// Kernel launchers (defined in the .hip files).  All are asynchronous on
// `stream`, cover every problem of the batch, and return the hipError_t of
// the launch.  Kernels of an iteration skip problems whose schedule is not
// in `phase`.
hipError_t launch_spmm_t(Mode m, const Batch &bt, int phase, hipStream_t stream);
// The push form applies to widths 8, 16 and 32; landmarks per block of its
// reduction in mode m.
bool spmmt_push_width(int B);
int spmmt_push_rows(Mode m, int B);
hipError_t launch_gemm(Mode m, const Batch &bt, int phase, hipStream_t stream);
// rr = 1 (2): the SpMM also runs the iteration's Rayleigh-Ritz step (the
// start's CholQR) in the block that completes its Gram reduction; only for
// batches where spmm_runs_rr(bt, m).
bool spmm_runs_rr(const Batch &bt, Mode m);
// Widths whose row-split SpMM also has the two-blocks-per-CU form.
bool spmm_has_two_block_form(int B);
hipError_t launch_spmm(Mode m, const Batch &bt, int phase, hipStream_t stream, int rr = 0, int max_sweeps = 0,
                       const PhaseRule &rule = PhaseRule{});
hipError_t launch_rr_solve(const Batch &bt, int init, int max_sweeps, const PhaseRule &rule,
                           hipStream_t stream);
hipError_t launch_random_start(Mode m, const Batch &bt, uint64_t seed, hipStream_t stream);
hipError_t launch_user_start(Mode m, const Batch &bt, hipStream_t stream);
// Rank repair: for every problem of `bt` whose last CholQR dropped columns
// (SolveState::dead > 0, not done) and whose current block is stored in mode
// m, writes its basis X = J Y C into buffer 0 with the dropped columns
// replaced by fresh Gaussian ones (`salt` keeps them apart from the start
// block's), then its Gram; a following launch_rr_solve(bt, RR_REFILL, ...)
// orthonormalises it without touching the schedule.
hipError_t launch_refill(Mode m, const Batch &bt, uint64_t seed, uint32_t salt, hipStream_t stream);
hipError_t launch_convert_y(Mode from, Mode to, const Batch &bt, int phase, hipStream_t stream);
// Phase changes the transposed SpMM bridges by reading the previous phase's
// (narrower) block directly; they need no launch of their own.
bool reads_previous_block(Mode from, Mode to);
hipError_t launch_embedding(const Batch &bt, void *Z, int z_double, hipStream_t stream);
// Landmark-block start: fills U of every problem of `bt` with an l x b block
// (in the transposed-product type of mode m) and arms the state so that the
// next SpMM launch of phase 0 writes P U into buffer 0 with its Gram.  The
// block is the current basis of the matching problem of `lmk` (landmark MDS)
// when `lmk` is non-NULL, else the first k columns come from `learned`
// ([sum l] x k floats, rows at ProbView::loff) and the rest are Gaussian.
hipError_t launch_lift_prep(Mode m, const Batch &bt, const Batch *lmk, const float *learned, uint64_t seed,
                            hipStream_t stream);
hipError_t launch_block_out(Mode m, const DevProblem &p, int ybuf, void *X, int x_double,
                            hipStream_t stream);

hipError_t launch_f32_to_bf16(const float *src, void *dst, int64_t count, hipStream_t stream);
int gemm_rows_per_tile(Mode m, int B, int mfma);
bool gemm_mfma(Mode m, int B);  // the dense product runs on the matrix cores
int spmm_rows_per_block(Mode m, int B);
int spmm_block_cap(Mode m, int B);  // most blocks worth launching for one problem

// Algorithmic bytes / flops of one launch of each hot kernel (one problem).
double spmm_bytes(Mode m, const DevProblem &p);
double spmm_t_bytes(Mode m, const DevProblem &p);
double gemm_bytes(Mode m, const DevProblem &p, bool packed);

}  // namespace sbmds
