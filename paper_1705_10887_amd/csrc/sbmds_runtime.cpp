// Host runtime behind the C ABI of include/sbmds.h: validation, the device
// memory plan of a context, the precision schedule and the stopping rule.
//
// Iteration (block subspace iteration with Rayleigh-Ritz on
// B = -1/2 J P W P^T J, the classical scaling matrix of Section 3.3):
//   T  = (P^T Y - c e^T/n) C         k_spmm_t   (inner centering, rotation)
//   U  = -1/2 W T, H = T^T U, s=c^T U k_gemm     (dense landmark product)
//   Y' = P U - 1 s^T / n, G, e        k_spmm     (outer centering, Gram)
//   Ritz pairs, bounds, next C        k_rr_solve (float64, one workgroup)
//
// Precision schedule: bf16 bulk iterations (BF16_FP32 only) until the Ritz
// residuals reach the bf16 floor, float32 iterations until they reach the
// float32 floor, then iterations on the same float32 operator with float64
// vectors and accumulation until the float64 error bound certifies the
// requested tolerance.  FP64 precision runs float64 throughout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/sbmds.h"
#include "../../include/sbmds_mlp.h"
#include "sbmds_common.h"
#include "sbmds_compare.h"
#include "sbmds_internal.h"
#include "sbmds_dense_sym.h"
#include "sbmds_prep.h"
#include "sbmds_mlp_internal.h"

using namespace sbmds;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

}  // namespace

namespace sbmds {
int api_fail(int code, const std::string &msg) { return fail(code, msg); }
void api_clear_error() { g_err.clear(); }
}  // namespace sbmds

namespace {

struct Summary {  // tail of SolveState read back after each iteration
    double theta[kMaxB];
    double res[kMaxB];
    double bound[kMaxB];
    double maxbound;
    double maxres;
    int iter;
    int flags;
    int dead;
    int nonpos;
    int sweeps;
    int ycur, zbuf, zmode, phase, done, pending_convert, phase_iters, total_iters;
    int iters[4];
    int sweeps_total, ymode, refill;
    double hist[4];
};
static_assert(sizeof(Summary) == kSummaryBytes, "summary layout");

inline uint16_t host_f2bf(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
inline float host_bf2f(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

int kernel_width(int block) {
    for (int w : {4, 8, 16, 32, 64})
        if (block <= w) return w;
    return -1;
}

struct KStat {
    std::string name;
    int64_t launches = 0;
    double ms = 0, bytes = 0, flops = 0;
};

struct PendingEv {
    int stat;
    hipEvent_t a, b;
    double bytes, flops;
};

}  // namespace

// A batch of problems solved together: device buffers, launch tables and
// the host's view of their solver state.
struct SolveSet {
    std::vector<DevProblem> probs;
    std::vector<std::vector<LaunchCfg>> cfg;  // [problem][mode]
    Tune tune[NUM_MODES];                      // launch choices per mode
    Batch bt;                                  // launch tables over all problems
    SolveState *st_all = nullptr;              // device, one per problem (contiguous)
    Summary *host_sum = nullptr;               // pinned, one per problem (written by the kernels)
    void *host_sum_dev = nullptr;              // the same memory as the device sees it
    std::vector<int> expect;                   // iterations per phase seen in the last solve
    std::vector<int> cur_ybuf, cur_mode;       // current block per problem
    size_t zstage_bytes = 0;
    // captured rounds of iterations, keyed by their launch sequence
    std::map<std::string, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
};

struct sbmds_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;          // created when the options give no stream
    sbmds_options opt{};
    std::vector<void *> allocs;
    size_t bytes = 0;
    SolveSet main;                             // the problems of the context
    SolveSet lmk;                              // their landmark problems (landmark MDS start)
    // learned start: network, per-problem vertex positions and landmark
    // ids, and per-landmark features / predictions (rows at ProbView::loff)
    sbmds_mlp *net = nullptr;
    std::vector<float *> xyz;
    std::vector<int32_t *> lmv;
    float *feat = nullptr, *learned = nullptr;
    double *rowmax = nullptr;
    int64_t total_l = 0;
    bool timing = false;
    std::vector<KStat> stats;
    std::vector<PendingEv> pending;
    std::vector<hipEvent_t> ev_pool;
    void *zstage = nullptr;                    // device staging of Z for host outputs
    bool packed = false;                       // W also kept as its packed upper triangle
};

namespace {

int dalloc(sbmds_ctx *ctx, void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    if (ctx->opt.mem_cap && ctx->bytes + bytes > ctx->opt.mem_cap)
        return fail(SBMDS_ENOMEM, "mem_cap exceeded (" + std::to_string(ctx->bytes + bytes) + " bytes needed)");
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(SBMDS_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    ctx->allocs.push_back(*p);
    ctx->bytes += bytes;
    return SBMDS_OK;
}

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t _e = (expr);                                                                        \
        if (_e != hipSuccess) return fail(SBMDS_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

#define OKCHK(expr)                 \
    do {                            \
        int _r = (expr);            \
        if (_r < 0) return _r;      \
    } while (0)

int check_options(const sbmds_options &o) {
    if (o.k < 1) return fail(SBMDS_EINVAL, "k must be >= 1");
    if (o.block < o.k) return fail(SBMDS_EINVAL, "block must be >= k");
    if (o.block > SBMDS_MAX_BLOCK) return fail(SBMDS_EINVAL, "block must be <= 64");
    if (o.prec < SBMDS_FP64 || o.prec > SBMDS_BF16_FP32) return fail(SBMDS_EINVAL, "unknown precision");
    if (o.start < SBMDS_START_RANDOM || o.start > SBMDS_START_USER) return fail(SBMDS_EINVAL, "unknown start");
    if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return fail(SBMDS_EINVAL, "tol must be positive and finite");
    if (o.max_iter < 1) return fail(SBMDS_EINVAL, "max_iter must be >= 1");
    if (o.start == SBMDS_START_LEARNED && o.mlp_weights == nullptr)
        return fail(SBMDS_EINVAL, "SBMDS_START_LEARNED needs mlp_weights");
    return SBMDS_OK;
}

int check_shape(const sbmds_problem &p, const sbmds_options &o, int idx) {
    const std::string pre = "problem " + std::to_string(idx) + ": ";
    if (p.mem != SBMDS_MEM_HOST && p.mem != SBMDS_MEM_DEVICE) return fail(SBMDS_EINVAL, pre + "mem must be 0 or 1");
    if (p.l < 2) return fail(SBMDS_EINVAL, pre + "l must be >= 2");
    if (p.n < p.l) return fail(SBMDS_EINVAL, pre + "l must be <= n");
    if (p.n >= (int64_t)1 << 31) return fail(SBMDS_EINVAL, pre + "n must be < 2^31");
    if (p.l > (int64_t)1 << 20) return fail(SBMDS_EINVAL, pre + "l must be <= 2^20");
    if (p.nnz < 0 || p.nnz >= (int64_t)1 << 31) return fail(SBMDS_EINVAL, pre + "nnz out of range");
    if (o.block > p.l - 1) return fail(SBMDS_EINVAL, pre + "block must be <= l - 1");
    if (!p.P_rowptr) return fail(SBMDS_EINVAL, pre + "P_rowptr is NULL");
    if (p.nnz > 0 && (!p.P_col || !p.P_val)) return fail(SBMDS_EINVAL, pre + "P_col/P_val is NULL");
    if (!p.W) return fail(SBMDS_EINVAL, pre + "W is NULL");
    if (o.start == SBMDS_START_USER && !p.X0) return fail(SBMDS_EINVAL, pre + "X0 is NULL");
    if (o.start == SBMDS_START_LEARNED && (!p.xyz || !p.landmark_vertex))
        return fail(SBMDS_EINVAL, pre + "xyz/landmark_vertex needed for the learned start");
    return SBMDS_OK;
}

template <typename T>
int check_contents(const sbmds_problem &p, const int32_t *rp, const int32_t *ci, const T *val, const T *W,
                   int idx) {
    const std::string pre = "problem " + std::to_string(idx) + ": ";
    const int64_t n = p.n, l = p.l;
    if (rp[0] != 0) return fail(SBMDS_EINVAL, pre + "P_rowptr[0] != 0");
    if ((int64_t)rp[n] != p.nnz) return fail(SBMDS_EINVAL, pre + "P_rowptr[n] != nnz");
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i] || (int64_t)rp[i + 1] > p.nnz)
            return fail(SBMDS_EINVAL, pre + "P_rowptr not non-decreasing within [0, nnz] at row " + std::to_string(i));
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= l)
                return fail(SBMDS_EINVAL, pre + "P_col out of range in row " + std::to_string(i));
            if (e > rp[i] && ci[e] <= ci[e - 1])
                return fail(SBMDS_EINVAL, pre + "P_col not strictly increasing in row " + std::to_string(i));
            if (!std::isfinite((double)val[e])) return fail(SBMDS_EINVAL, pre + "non-finite P value");
        }
    }
    for (int64_t i = 0; i < l; ++i) {
        for (int64_t j = 0; j <= i; ++j) {
            const T a = W[i * l + j], b = W[j * l + i];
            if (!std::isfinite((double)a)) return fail(SBMDS_EINVAL, pre + "non-finite W entry");
            if (a != b) return fail(SBMDS_EINVAL, pre + "W is not symmetric");
        }
    }
    return SBMDS_OK;
}

// The precision schedule: one phase per arithmetic.  Non-final phases hand
// over at the residual floor of their storage precision (or when the
// residual stalls); the final phase stops at the certified tolerance.
std::vector<PhaseRule> schedule(const sbmds_options &o) {
    std::vector<Mode> modes;
    switch (o.prec) {
        case SBMDS_FP64: modes = {MODE_FP64}; break;
        case SBMDS_FP32: modes = {MODE_FP32, MODE_F64ACC}; break;
        default: modes = {MODE_BF16, MODE_FP32, MODE_F64ACC}; break;
    }
    if ((o.flags & SBMDS_FLAG_NO_CERTIFY) && modes.size() > 1) modes.pop_back();
    std::vector<PhaseRule> out;
    for (size_t i = 0; i < modes.size(); ++i) {
        PhaseRule r{};
        r.phase = (int)i;
        r.mode = modes[i];
        r.is_final = (i + 1 == modes.size()) ? 1 : 0;
        r.cap = 60;
        r.floor_res = modes[i] == MODE_BF16 ? 5e-2 : 1e-3;
        r.tol = o.tol;
        out.push_back(r);
    }
    return out;
}

constexpr int kMaxGemmSplit = 64;   // K splits of the dense product (bounds its scratch)
constexpr size_t kFusedRrMaxProblems = 16;  // batches above this size run the Rayleigh-Ritz step on its own
constexpr double kPackMinBytes = 256e6;  // float32 W of a batch above which its upper triangle is packed
constexpr int kMaxSpmmBlocks = 1024;

LaunchCfg make_cfg(Mode m, const DevProblem &p, const Tune &t) {
    LaunchCfg c;
    const int rpb = spmm_rows_per_block(m, p.B);
    int64_t want = (p.n + rpb - 1) / rpb;
    const int cap = std::min(t.spmm_cap, kMaxSpmmBlocks);
    c.spmm_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, cap));
    c.gemm_rt = gemm_rows_per_tile(m, p.B, t.gemm_mfma);
    const int rowtiles = (int)((p.l + c.gemm_rt - 1) / c.gemm_rt);
    int ks = (t.gemm_target + rowtiles - 1) / rowtiles;
    const int kblocks = p.lda / 64;
    ks = std::max(1, std::min(std::min(ks, kblocks), kMaxGemmSplit));
    c.gemm_kchunk = ((kblocks + ks - 1) / ks) * 64;
    c.gemm_ksplit = (p.lda + c.gemm_kchunk - 1) / c.gemm_kchunk;
    return c;
}

// Defaults: matrix cores for the dense product once W no longer fits the
// caches (there its bandwidth is higher; below, launch latency dominates
// and the vector kernel is as fast), waves per landmark row of P^T by the
// mean column length of P.
Tune default_tune(Mode m, const std::vector<DevProblem> &probs) {
    Tune t;
    double nnz = 0, l = 0, l2 = 0;
    for (const DevProblem &p : probs) {
        nnz += (double)p.nnz;
        l += (double)p.l;
        l2 += (double)p.l * p.l;
    }
    const int B = probs[0].B;
    t.spmm_cap = spmm_block_cap(m, B);
    // (float64-accumulating modes: the vector kernel carries half the rows
    // per wave, so the matrix cores win at every size)
    const bool f64 = m == MODE_F64ACC || m == MODE_FP64;
    t.gemm_mfma = (gemm_mfma(m, B) && (f64 || l2 * 4.0 > 64e6)) ? 1 : 0;
    t.gemm_target = t.gemm_mfma ? 512 : 1024;
    // the packed upper triangle of W (half the dense product's bytes) where
    // it was built, i.e. where W is too large for the caches
    bool all_packed = !probs.empty();
    for (const DevProblem &p : probs) all_packed = all_packed && p.Wp != nullptr;
    t.gemm_sym = (all_packed && sym_supported(m, B)) ? 1 : 0;
    t.sym_c = 16;
    // the two-blocks-per-CU SpMM once a launch streams enough bytes that
    // bandwidth, not the latency of the separate Rayleigh-Ritz launch, counts
    double sp_bytes = 0;
    for (const DevProblem &p : probs) sp_bytes += spmm_bytes(m, p);
    t.spmm_wpe = (sp_bytes > 48e6 || probs.size() > kFusedRrMaxProblems) ? 8 : 4;
    const double per_row = nnz / l;  // mean entries per landmark column of P
    // (351 entries per landmark row at 50,000 landmarks: one wave per row
    // measured fastest, 108 against 183 us with four)
    t.spmmt_wpr = per_row >= 1024 ? 4 : (per_row >= 384 ? 2 : 1);
    return t;
}

void apply_tune(SolveSet &set) {
    for (size_t i = 0; i < set.probs.size(); ++i) {
        set.cfg[i].resize(NUM_MODES);
        for (int m = 0; m < NUM_MODES; ++m) set.cfg[i][m] = make_cfg((Mode)m, set.probs[i], set.tune[m]);
    }
}

hipEvent_t ev_get(sbmds_ctx *ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int stat_index(sbmds_ctx *ctx, const char *name) {
    for (size_t i = 0; i < ctx->stats.size(); ++i)
        if (ctx->stats[i].name == name) return (int)i;
    ctx->stats.push_back(KStat{name});
    return (int)ctx->stats.size() - 1;
}

// Runs `launch` on the context stream, bracketed by events when timing.
template <typename F>
int timed(sbmds_ctx *ctx, const char *name, double bytes, double flops, F &&launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (ctx->timing) {
        a = ev_get(ctx);
        b = ev_get(ctx);
        if (a && b) HIPCHK(hipEventRecord(a, ctx->stream));
    }
    hipError_t e = launch();
    if (e != hipSuccess) return fail(SBMDS_EHIP, std::string("launch of ") + name + " failed: " + hipGetErrorString(e));
    if (ctx->timing && a && b) {
        HIPCHK(hipEventRecord(b, ctx->stream));
        ctx->pending.push_back(PendingEv{stat_index(ctx, name), a, b, bytes, flops});
    }
    return SBMDS_OK;
}

void collect_timing(sbmds_ctx *ctx) {
    for (auto &pe : ctx->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
            KStat &s = ctx->stats[pe.stat];
            s.launches += 1;
            s.ms += ms;
            s.bytes += pe.bytes;
            s.flops += pe.flops;
        }
        ctx->ev_pool.push_back(pe.a);
        ctx->ev_pool.push_back(pe.b);
    }
    ctx->pending.clear();
}

// The Rayleigh-Ritz kernels write each problem's summary into the pinned
// host array themselves; the host only waits for the stream.
int read_summaries(sbmds_ctx *ctx, SolveSet &set) {
    (void)set;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return SBMDS_OK;
}

// Jacobi sweeps allowed per Rayleigh-Ritz step.  Inexact diagonalisation
// keeps every reported bound valid (each Ritz value is the exact Rayleigh
// quotient of the vector it belongs to, and its residual is measured), and
// the next iteration continues the diagonalisation in the rotated basis.
// The final phase starts from a nearly diagonal H (the previous phase
// rotated the basis to its Ritz vectors), where three sweeps reach the
// convergence test; non-final phases take one.
int sweep_cap(const PhaseRule &r) {
    static int env = -1;
    if (env < 0) {
        const char *e = std::getenv("SBMDS_MAX_SWEEPS");
        env = e ? std::max(1, std::atoi(e)) : 0;
    }
    if (r.is_final) return 3;
    return env > 0 ? env : 1;
}

// One iteration of phase `r` for every problem, enqueued without
// synchronising: each kernel checks on the device, per problem, that the
// solve is still in this phase.
int enqueue_iteration(sbmds_ctx *ctx, SolveSet &set, const PhaseRule &r) {
    const Mode m = (Mode)r.mode;
    const Batch &bt = set.bt;
    double b_spmm = 0, b_spmmt = 0, b_gemm = 0, f_sp = 0, f_ge = 0;
    for (const DevProblem &p : set.probs) {
        b_spmm += spmm_bytes(m, p);
        b_spmmt += spmm_t_bytes(m, p);
        b_gemm += gemm_bytes(m, p, bt.gemm_sym[m] != 0);
        f_sp += 2.0 * p.nnz * p.B;
        f_ge += 2.0 * (double)p.l * p.l * p.B;
    }
    static const char *const mname[NUM_MODES] = {"bf16", "fp32", "f64acc", "fp64"};
    const std::string sfx = std::string(".") + mname[m];
    OKCHK(timed(ctx, ("spmm_t" + sfx).c_str(), b_spmmt, f_sp, [&] { return launch_spmm_t(m, bt, r.phase, ctx->stream); }));
    OKCHK(timed(ctx, ("gemm" + sfx).c_str(), b_gemm, f_ge, [&] { return launch_gemm(m, bt, r.phase, ctx->stream); }));
    if (spmm_runs_rr(bt, m)) {
        // the Rayleigh-Ritz step runs in the SpMM's reducing block
        OKCHK(timed(ctx, ("spmm_rr" + sfx).c_str(), b_spmm, f_sp,
                    [&] { return launch_spmm(m, bt, r.phase, ctx->stream, 1, sweep_cap(r), r); }));
    } else {
        OKCHK(timed(ctx, ("spmm" + sfx).c_str(), b_spmm, f_sp, [&] { return launch_spmm(m, bt, r.phase, ctx->stream); }));
        OKCHK(timed(ctx, ("rr_solve" + sfx).c_str(), 0.0, 0.0,
                    [&] { return launch_rr_solve(bt, 0, sweep_cap(r), r, ctx->stream); }));
    }
    return SBMDS_OK;
}

double ms_between(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return ms;
}

// Enqueue one round of launches (phase conversions and iterations).  Unless
// kernel timing is on or graphs are disabled, the round is captured once
// into a hipGraph and replayed on later calls with the same sequence; the
// kernels read every per-call value (phase, block buffer, state) from the
// device, so a replay is the same work as the eager launches.
int enqueue_round(sbmds_ctx *ctx, SolveSet &set, const std::vector<PhaseRule> &rules,
                  const std::vector<std::pair<int, int>> &ops) {
    auto run_ops = [&]() -> int {
        for (const auto &op : ops) {
            const int ph = op.second;
            if (op.first) {
                const Mode mf = (Mode)rules[ph - 1].mode, mt = (Mode)rules[ph].mode;
                // a phase whose kernels read the previous phase's narrower
                // block needs no launch of its own (its first Rayleigh-Ritz
                // step clears the pending flag)
                if (!reads_previous_block(mf, mt))
                    OKCHK(timed(ctx, "convert", 0.0, 0.0,
                                [&] { return launch_convert_y(mf, mt, set.bt, ph, ctx->stream); }));
            } else {
                OKCHK(enqueue_iteration(ctx, set, rules[ph]));
            }
        }
        return SBMDS_OK;
    };
    const bool use_graph = !ctx->timing && !(ctx->opt.flags & SBMDS_FLAG_NO_GRAPH) && ctx->stream != nullptr;
    if (!use_graph || ops.empty()) return run_ops();
    std::string key;
    for (const auto &op : ops) key += (op.first ? 'c' : 'i') + std::to_string(op.second) + ",";
    auto it = set.graphs.find(key);
    if (it == set.graphs.end()) {
        HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        const int rc = run_ops();
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->stream, &g);
        if (rc < 0) {
            if (e == hipSuccess && g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(SBMDS_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(SBMDS_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
        }
        it = set.graphs.emplace(key, std::make_pair(g, ex)).first;
    }
    HIPCHK(hipGraphLaunch(it->second.second, ctx->stream));
    return SBMDS_OK;
}

// Solve every problem of `set` together: one launch per kernel and
// iteration covers all of them; each follows the schedule `rules` on its own
// and drops out of the launches once it is done.  `start` enqueues the start
// block and its orthonormalisation; `after_round` (may be empty) enqueues
// work that reads the state a round leaves, ahead of the host's look at it,
// so that after the last round it is already on the device.  Returns 1 if
// every problem finished.
template <typename StartFn>
int run_set(sbmds_ctx *ctx, SolveSet &set, const std::vector<PhaseRule> &rules, int max_iter, StartFn &&start,
            const std::function<int()> &after_round = {}) {
    const int np = (int)set.probs.size();
    const int nph = (int)rules.size();
    std::vector<int> &expect = set.expect;
    if ((int)expect.size() != nph) {
        expect.assign(nph, 3);
        expect[nph - 1] = 1;
    }
    OKCHK(start());
    // Enqueue whole phases without waiting; the device decides when each
    // phase ends and when a problem is done, and later launches skip it.
    // The host looks at the state once per round.
    int launched = 0, from = 0, pending = 0;
    bool first = true, all_done = false;
    const Summary *S = set.host_sum;
    for (;;) {
        std::vector<std::pair<int, int>> ops;  // (is_convert, phase)
        for (int ph = from; ph < nph && launched < max_iter; ++ph) {
            if (ph > from || pending) ops.push_back({1, ph});
            int n_it = (first || ph > from) ? std::max(1, expect[ph]) : 2;
            n_it = std::min(n_it, max_iter - launched);
            for (int i = 0; i < n_it; ++i) ops.push_back({0, ph});
            launched += n_it;
        }
        OKCHK(enqueue_round(ctx, set, rules, ops));
        if (after_round) OKCHK(after_round());
        OKCHK(read_summaries(ctx, set));
        all_done = true;
        from = nph;
        pending = 0;
        for (int i = 0; i < np; ++i) {
            if (S[i].flags & SF_NONFINITE) return fail(SBMDS_EBREAKDOWN, "non-finite values in the block solver");
            if (!S[i].done) {
                all_done = false;
                // the slowest problem sets where the next round starts
                if (S[i].phase < from || (S[i].phase == from && S[i].pending_convert)) {
                    from = S[i].phase;
                    pending = S[i].pending_convert;
                }
            }
        }
        if (all_done || launched >= max_iter || from >= nph) break;
        // rank repair: a block that lost rank (its CholQR dropped columns,
        // e.g. a start block with a zero or repeated column) gets fresh
        // Gaussian columns in place of the dropped ones before the next round
        unsigned refill_modes = 0;
        for (int i = 0; i < np; ++i)
            if (!S[i].done && S[i].dead > 0) refill_modes |= 1u << S[i].ymode;
        if (refill_modes) {
            for (int m = 0; m < NUM_MODES; ++m)
                if (refill_modes & (1u << m))
                    OKCHK(timed(ctx, "refill", 0.0, 0.0, [&] {
                        return launch_refill((Mode)m, set.bt, ctx->opt.seed, (uint32_t)launched + 1u, ctx->stream);
                    }));
            OKCHK(timed(ctx, "rr_refill", 0.0, 0.0,
                        [&] { return launch_rr_solve(set.bt, RR_REFILL, 0, rules[0], ctx->stream); }));
        }
        first = false;
    }
    if (all_done) {
        for (int ph = 0; ph < nph; ++ph) {
            int mx = 0;
            for (int i = 0; i < np; ++i) mx = std::max(mx, S[i].iters[ph]);
            expect[ph] = mx;
        }
    }
    for (int i = 0; i < np; ++i) {
        set.cur_ybuf[i] = S[i].ycur;
        set.cur_mode[i] = S[i].ymode;
    }
    return all_done ? 1 : 0;
}

// The landmark problems are solved to a loose tolerance: their basis only
// seeds the main iteration.
constexpr double kLmdsTol = 1e-5;
constexpr int kLmdsMaxIter = 12;

std::vector<PhaseRule> lmds_rules(const sbmds_options &o) {
    PhaseRule r{};
    r.phase = 0;
    r.is_final = 1;
    r.cap = kLmdsMaxIter;
    r.mode = o.prec == SBMDS_FP64 ? MODE_FP64 : MODE_FP32;
    r.floor_res = 0.0;
    r.tol = kLmdsTol;
    return {r};
}

int solve_all(sbmds_ctx *ctx, sbmds_report *reps, const std::function<int()> &output = {}) {
    const sbmds_options &o = ctx->opt;
    SolveSet &set = ctx->main;
    const int np = (int)set.probs.size();
    const std::vector<PhaseRule> rules = schedule(o);
    const int nph = (int)rules.size();
    hipEvent_t e0 = ev_get(ctx), e1 = ev_get(ctx), e2 = ev_get(ctx);
    HIPCHK(hipEventRecord(e0, ctx->stream));
    const Mode m0 = (Mode)rules[0].mode;
    bool init_fused = false;
    // the lift Y0 = P X_l: one SpMM, which also runs the first CholQR where
    // the width allows
    auto lift = [&]() -> int {
        init_fused = spmm_runs_rr(set.bt, m0);
        if (init_fused)
            return timed(ctx, "lift_rr_init", 0.0, 0.0,
                         [&] { return launch_spmm(m0, set.bt, 0, ctx->stream, 2, 0, rules[0]); });
        return timed(ctx, "lift", 0.0, 0.0, [&] { return launch_spmm(m0, set.bt, 0, ctx->stream); });
    };
    auto start = [&]() -> int {
        init_fused = false;
        if (o.start == SBMDS_START_USER) {
            OKCHK(timed(ctx, "start", 0.0, 0.0, [&] { return launch_user_start(m0, set.bt, ctx->stream); }));
        } else if (o.start == SBMDS_START_LMDS) {
            // landmark MDS: top eigenvectors of -1/2 J W J on the landmarks
            // (the same iteration with P = I), lifted through P
            const std::vector<PhaseRule> lr = lmds_rules(o);
            const int rc = run_set(ctx, ctx->lmk, lr, kLmdsMaxIter, [&]() -> int {
                const Mode lm = (Mode)lr[0].mode;
                OKCHK(timed(ctx, "start", 0.0, 0.0,
                            [&] { return launch_random_start(lm, ctx->lmk.bt, o.seed, ctx->stream); }));
                OKCHK(timed(ctx, "rr_init", 0.0, 0.0,
                            [&] { return launch_rr_solve(ctx->lmk.bt, 1, 0, lr[0], ctx->stream); }));
                return SBMDS_OK;
            });
            if (rc < 0) return rc;
            OKCHK(timed(ctx, "lift", 0.0, 0.0,
                        [&] { return launch_lift_prep(m0, set.bt, &ctx->lmk.bt, nullptr, o.seed, ctx->stream); }));
            OKCHK(lift());
        } else if (o.start == SBMDS_START_LEARNED) {
            // the network's landmark prediction (forward pass on the features
            // made at create) as the first k columns, the rest Gaussian,
            // lifted through P
            OKCHK(mlp::forward_device(ctx->net, ctx->feat, ctx->total_l, ctx->learned));
            OKCHK(timed(ctx, "lift", 0.0, 0.0,
                        [&] { return launch_lift_prep(m0, set.bt, nullptr, ctx->learned, o.seed, ctx->stream); }));
            OKCHK(lift());
        } else {
            OKCHK(timed(ctx, "start", 0.0, 0.0, [&] { return launch_random_start(m0, set.bt, o.seed, ctx->stream); }));
        }
        if (!init_fused)
            OKCHK(timed(ctx, "rr_init", 0.0, 0.0, [&] { return launch_rr_solve(set.bt, 1, 0, rules[0], ctx->stream); }));
        HIPCHK(hipEventRecord(e1, ctx->stream));
        return SBMDS_OK;
    };
    // the outputs follow every round (the state a round leaves is complete
    // on the device): after the last one they need no further host round trip
    std::function<int()> after_round;
    if (output)
        after_round = [&]() -> int {
            HIPCHK(hipEventRecord(e2, ctx->stream));
            return output();
        };
    const int rc = run_set(ctx, set, rules, o.max_iter, start, after_round);
    if (rc < 0) return rc;
    const bool all_done = rc == 1;
    if (!output) HIPCHK(hipEventRecord(e2, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const Summary *S = set.host_sum;
    for (int i = 0; i < np && reps; ++i) {
        sbmds_report *rep = &reps[i];
        const DevProblem &p = set.probs[i];
        std::memset(rep, 0, sizeof(*rep));
        const bool done = S[i].done != 0;
        rep->status = done ? SBMDS_OK : SBMDS_ENOCONV;
        for (int ph = 0; ph < nph; ++ph) {
            const int it = S[i].iters[ph];
            if (rules[ph].mode == MODE_BF16) rep->iters_bf16 += it;
            else if (rules[ph].mode == MODE_FP32) rep->iters_fp32 += it;
            else rep->iters_fp64 += it;
        }
        rep->nonpositive = S[i].nonpos;
        rep->certified = (done && (rules[nph - 1].mode == MODE_F64ACC || rules[nph - 1].mode == MODE_FP64)) ? 1 : 0;
        rep->jacobi_sweeps = S[i].sweeps_total;
        rep->start_iters = o.start == SBMDS_START_LMDS ? ctx->lmk.host_sum[i].total_iters : 0;
        rep->ms_start = ms_between(e0, e1);
        rep->ms_iter = ms_between(e1, e2);
        rep->ms_total = ms_between(e0, e2);
        for (int j = 0; j < p.b; ++j) {
            rep->eig[j] = S[i].theta[j];
            rep->err_bound[j] = S[i].bound[j];
            rep->resid[j] = std::fabs(S[i].theta[j]) > 0 ? S[i].res[j] / std::fabs(S[i].theta[j]) : S[i].res[j];
        }
    }
    ctx->ev_pool.push_back(e0);
    ctx->ev_pool.push_back(e1);
    ctx->ev_pool.push_back(e2);
    return all_done ? SBMDS_OK : SBMDS_ENOCONV;
}

// ---------------------------------------------------------------------------
// Autotuner.  For every arithmetic of the schedule it times, on the device
// and on the problems of the context, the candidates of each launch choice
// (one choice at a time, the others held at their current values): the SpMM
// block cap and (widths 8-32) its form, the dense-product kernel and its
// block target, and the waves per landmark row of the transposed SpMM.  The
// iteration state it leaves behind is discarded: every solve starts from its
// start block.  Results are kept in a text cache, one line per (batch
// shape, arithmetic):
//   <key> <spmm_cap> <gemm_mfma> <gemm_target> <spmmt_wpr> <spmm_wpe>
// Different choices change the summation order, so results are bitwise
// reproducible for a fixed configuration only.
// ---------------------------------------------------------------------------
int build_batch(sbmds_ctx *ctx, SolveSet &set);

std::string tune_key(const SolveSet &set, Mode m) {
    std::string k = "v1;B=" + std::to_string(set.probs[0].B) + ";m=" + std::to_string((int)m);
    for (const DevProblem &p : set.probs)
        k += ";" + std::to_string(p.n) + "," + std::to_string(p.l) + "," + std::to_string(p.nnz);
    // keep keys short for large batches
    if (k.size() > 200) {
        uint64_t h = 1469598103934665603ull;  // FNV-1a
        for (char ch : k) h = (h ^ (uint8_t)ch) * 1099511628211ull;
        k = "v1;B=" + std::to_string(set.probs[0].B) + ";m=" + std::to_string((int)m) + ";np=" +
            std::to_string(set.probs.size()) + ";h=" + std::to_string(h);
    }
    return k;
}

std::vector<std::pair<std::string, std::string>> read_cache(const char *path) {
    std::vector<std::pair<std::string, std::string>> out;
    FILE *f = std::fopen(path, "r");
    if (!f) return out;
    char line[4096];
    while (std::fgets(line, sizeof(line), f)) {
        std::string ln(line);
        while (!ln.empty() && (ln.back() == '\n' || ln.back() == '\r')) ln.pop_back();
        const size_t sp = ln.find(' ');
        if (sp == std::string::npos) continue;
        out.push_back({ln.substr(0, sp), ln.substr(sp + 1)});
    }
    std::fclose(f);
    return out;
}

int write_cache(const char *path, const std::vector<std::pair<std::string, std::string>> &entries) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return fail(SBMDS_EINVAL, std::string("cannot write the tuning cache ") + path);
    for (const auto &e : entries) std::fprintf(f, "%s %s\n", e.first.c_str(), e.second.c_str());
    if (std::fclose(f) != 0 || std::rename(tmp.c_str(), path) != 0)
        return fail(SBMDS_EINVAL, std::string("cannot write the tuning cache ") + path);
    return SBMDS_OK;
}

template <typename F>
int time_launch(sbmds_ctx *ctx, F &&launch, double *ms_out) {
    for (int i = 0; i < 2; ++i) HIPCHK(launch());
    hipEvent_t a = ev_get(ctx), b = ev_get(ctx);
    if (!a || !b) return fail(SBMDS_EHIP, "hipEventCreate failed");
    constexpr int reps = 8;
    HIPCHK(hipEventRecord(a, ctx->stream));
    for (int i = 0; i < reps; ++i) HIPCHK(launch());
    HIPCHK(hipEventRecord(b, ctx->stream));
    HIPCHK(hipEventSynchronize(b));
    *ms_out = ms_between(a, b) / reps;
    ctx->ev_pool.push_back(a);
    ctx->ev_pool.push_back(b);
    return SBMDS_OK;
}

// Time of a standalone Rayleigh-Ritz launch (b <= 32, measured on the
// device), charged to the SpMM form that does not run the step itself.
constexpr double kRrLaunchMs = 0.010;

int autotune(sbmds_ctx *ctx, SolveSet &set) {
    const char *path = ctx->opt.tune_cache;
    auto cache = read_cache(path);
    bool dirty = false;
    std::vector<Mode> modes;
    for (const PhaseRule &r : schedule(ctx->opt))
        if (std::find(modes.begin(), modes.end(), (Mode)r.mode) == modes.end()) modes.push_back((Mode)r.mode);
    for (Mode m : modes) {
        const std::string key = tune_key(set, m);
        bool found = false;
        for (const auto &e : cache) {
            if (e.first != key) continue;
            Tune t = set.tune[m];  // fields the entry does not carry keep their defaults
            const int got = std::sscanf(e.second.c_str(), "%d %d %d %d %d %d %d", &t.spmm_cap, &t.gemm_mfma,
                                        &t.gemm_target, &t.spmmt_wpr, &t.spmm_wpe, &t.gemm_sym, &t.sym_c);
            if (t.gemm_sym && (set.probs[0].Wp == nullptr || !sym_supported(m, set.probs[0].B))) t.gemm_sym = 0;
            if (got >= 4 && t.spmm_cap >= 1 && t.gemm_target >= 1 &&
                (t.sym_c == 8 || t.sym_c == 16 || t.sym_c == 32) &&
                (t.spmmt_wpr == 1 || t.spmmt_wpr == 2 || t.spmmt_wpr == 4) && (t.spmm_wpe == 4 || t.spmm_wpe == 8)) {
                set.tune[m] = t;
                found = true;
            }
        }
        if (found) continue;
        // a valid state in this arithmetic: start block and its orthonormal basis
        PhaseRule r{};
        r.phase = 0;
        r.is_final = 1;
        r.cap = 1;
        r.mode = m;
        r.tol = 0.0;
        apply_tune(set);
        OKCHK(build_batch(ctx, set));
        HIPCHK(launch_random_start(m, set.bt, ctx->opt.seed, ctx->stream));
        HIPCHK(launch_rr_solve(set.bt, 1, 0, r, ctx->stream));
        auto try_all = [&](auto &&field_values, auto &&set_field, auto &&launch) -> int {
            double best = 1e30;
            Tune keep = set.tune[m];
            for (int val : field_values) {
                set_field(set.tune[m], val);
                apply_tune(set);
                OKCHK(build_batch(ctx, set));
                double ms = 0.0;
                OKCHK(time_launch(ctx, launch, &ms));
                if (ms < best) {
                    best = ms;
                    keep = set.tune[m];
                }
            }
            set.tune[m] = keep;
            return SBMDS_OK;
        };
        // block counts: powers of two and the counts that give every block
        // the same number of row steps (for the largest problem)
        std::vector<int> spmm_cands{64, 128, 256, 512, 1024};
        {
            int64_t maxn = 0;
            for (const DevProblem &q : set.probs) maxn = std::max<int64_t>(maxn, q.n);
            const int rpb = spmm_rows_per_block(m, set.probs[0].B);
            const int64_t steps = (maxn + rpb - 1) / rpb;
            for (int64_t d = 1; d <= 4; ++d) {
                const int64_t c = (steps + d - 1) / d;
                if (c >= 32 && c <= kMaxSpmmBlocks &&
                    std::find(spmm_cands.begin(), spmm_cands.end(), (int)c) == spmm_cands.end())
                    spmm_cands.push_back((int)c);
            }
        }
        {
            // both forms of the row-split SpMM where the width has them; the
            // two-block form leaves the Rayleigh-Ritz step to a launch of
            // its own, which its time is charged with.  The fused form runs
            // each problem's Rayleigh-Ritz step in that problem's last block,
            // which the timing here (no step) does not see; with many
            // problems those steps pile up at the end of the launch (256
            // meshes: 4.4 against 1.6 ms), so large batches take the
            // two-block form.
            std::vector<int> wpes;
            if (!spmm_has_two_block_form(set.probs[0].B) || set.probs.size() <= kFusedRrMaxProblems) wpes.push_back(4);
            if (spmm_has_two_block_form(set.probs[0].B)) wpes.push_back(8);
            double best = 1e30;
            Tune keep = set.tune[m];
            for (int wpe : wpes) {
                for (int cap : spmm_cands) {
                    set.tune[m].spmm_wpe = wpe;
                    set.tune[m].spmm_cap = cap;
                    apply_tune(set);
                    OKCHK(build_batch(ctx, set));
                    double ms = 0.0;
                    OKCHK(time_launch(ctx, [&] { return launch_spmm(m, set.bt, 0, ctx->stream); }, &ms));
                    if (wpe == 8) ms += kRrLaunchMs;
                    if (ms < best) {
                        best = ms;
                        keep = set.tune[m];
                    }
                }
            }
            set.tune[m] = keep;
        }
        // dense product: full W on the matrix cores or vector ALUs with a
        // K split (target block counts), or the packed upper triangle with
        // regions of 8, 16 or 32 tile columns
        std::vector<int> gemm_cands;
        for (int mf = 0; mf < (gemm_mfma(m, set.probs[0].B) ? 2 : 1); ++mf)
            for (int tg : {1, 128, 256, 512, 1024, 2048}) gemm_cands.push_back(mf * 100000 + tg);  // 1: no K split
        bool packed = sym_supported(m, set.probs[0].B);
        for (const DevProblem &q : set.probs) packed = packed && q.Wp != nullptr;
        if (packed)
            for (int cw : {8, 16, 32}) gemm_cands.push_back(1000000 + cw);
        const int keep_mfma = set.tune[m].gemm_mfma, keep_target = set.tune[m].gemm_target;
        OKCHK(try_all(gemm_cands,
                      [&](Tune &t, int v) {
                          if (v >= 1000000) {
                              t.gemm_sym = 1;
                              t.sym_c = v - 1000000;
                              t.gemm_mfma = keep_mfma;
                              t.gemm_target = keep_target;
                          } else {
                              t.gemm_sym = 0;
                              t.gemm_mfma = v / 100000;
                              t.gemm_target = v % 100000;
                          }
                      },
                      [&] { return launch_gemm(m, set.bt, 0, ctx->stream); }));
        OKCHK(try_all(std::vector<int>{1, 2, 4}, [](Tune &t, int v) { t.spmmt_wpr = v; },
                      [&] { return launch_spmm_t(m, set.bt, 0, ctx->stream); }));
        const Tune &t = set.tune[m];
        char val[96];
        std::snprintf(val, sizeof(val), "%d %d %d %d %d %d %d", t.spmm_cap, t.gemm_mfma, t.gemm_target, t.spmmt_wpr,
                      t.spmm_wpe, t.gemm_sym, t.sym_c);
        cache.push_back({key, val});
        dirty = true;
    }
    apply_tune(set);
    OKCHK(build_batch(ctx, set));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (dirty) OKCHK(write_cache(path, cache));
    return SBMDS_OK;
}

// Create-time scratch on the device, released when it goes out of scope.
struct DevTmp {
    void *p = nullptr;
    DevTmp() = default;
    DevTmp(const DevTmp &) = delete;
    DevTmp &operator=(const DevTmp &) = delete;
    ~DevTmp() {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t bytes) {
        if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
            p = nullptr;
            return fail(SBMDS_ENOMEM, "hipMalloc of create-time scratch failed (" + std::to_string(bytes) + " bytes)");
        }
        return SBMDS_OK;
    }
};

std::string prep_error_text(unsigned long long key) {
    const int code = (int)(key >> 40);
    const std::string row = std::to_string(key & ((1ull << 40) - 1));
    switch (code) {
        case PREP_ROWPTR0: return "P_rowptr[0] != 0";
        case PREP_ROWPTRN: return "P_rowptr[n] != nnz";
        case PREP_ROWPTR_ORDER: return "P_rowptr not non-decreasing within [0, nnz] at row " + row;
        case PREP_COL_RANGE: return "P_col out of range in row " + row;
        case PREP_COL_ORDER: return "P_col not strictly increasing in row " + row;
        case PREP_VAL: return "non-finite P value in row " + row;
        case PREP_W_FINITE: return "non-finite W entry in row " + row;
        case PREP_W_SYM: return "W is not symmetric (row " + row + ")";
        default: return "invalid input";
    }
}

// Internal landmark order: a recursive partition of the landmarks into the
// cells of up to 8 pivots (the first members of the cell in the caller's
// farthest-point order, so spread out), each landmark joining the cell of
// its nearest pivot by W; cells of at most 64 landmarks (or 12 levels deep)
// keep their order.  Neighbouring internal indices are then spatially close,
// which the transposed SpMM exploits.  The order is invisible outside: P's
// columns and W are permuted together, which leaves B unchanged.  Run level
// by level: the nearest pivots of all landmarks of a level come from one
// kernel on the device-resident W; the host splits every cell, in place and
// stably, in pivot order (the same arrangement as a depth-first recursion).
template <typename T>
int landmark_order(sbmds_ctx *ctx, const T *dW, int64_t l, std::vector<int32_t> &order) {
    hipStream_t s = ctx->stream;
    order.resize(l);
    for (int64_t j = 0; j < l; ++j) order[j] = (int32_t)j;
    struct Cell {
        int64_t start, len;
        int depth;
    };
    std::vector<Cell> cells{{0, l, 0}};
    DevTmp tbuf;
    OKCHK(tbuf.alloc((size_t)l * 4 * 3 + (size_t)(l / 64 + 2) * 8 * 4));
    int32_t *d_order = (int32_t *)tbuf.p, *d_seg = d_order + l, *d_label = d_seg + l, *d_piv = d_label + l;
    std::vector<int32_t> seg(l), label(l), piv, tmp;
    for (;;) {
        std::vector<Cell> active, next;
        std::fill(seg.begin(), seg.end(), -1);
        piv.clear();
        for (const Cell &c : cells) {
            if (c.len <= 64 || c.depth >= 12) {
                next.push_back(c);  // final
                continue;
            }
            const int id = (int)active.size();
            active.push_back(c);
            for (int q = 0; q < 8; ++q) piv.push_back(order[c.start + q]);
            for (int64_t x = c.start; x < c.start + c.len; ++x) seg[x] = id;
        }
        if (active.empty()) break;
        HIPCHK(hipMemcpyAsync(d_order, order.data(), (size_t)l * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_seg, seg.data(), (size_t)l * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_piv, piv.data(), piv.size() * 4, hipMemcpyHostToDevice, s));
        HIPCHK(prep_labels<T>(dW, l, d_order, d_seg, d_piv, d_label, s));
        HIPCHK(hipMemcpyAsync(label.data(), d_label, (size_t)l * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        // split every active cell stably by its pivot label, children in pivot order
        std::vector<Cell> split;
        for (const Cell &c : active) {
            tmp.clear();
            int64_t off = c.start;
            for (int q = 0; q < 8; ++q) {
                const size_t before = tmp.size();
                for (int64_t x = c.start; x < c.start + c.len; ++x)
                    if (label[x] == q) tmp.push_back(order[x]);
                const int64_t cnt = (int64_t)(tmp.size() - before);
                if (cnt) split.push_back({off, cnt, c.depth + 1});
                off += cnt;
            }
            std::copy(tmp.begin(), tmp.end(), order.begin() + c.start);
        }
        next.insert(next.end(), split.begin(), split.end());
        std::sort(next.begin(), next.end(), [](const Cell &a, const Cell &b) { return a.start < b.start; });
        cells.swap(next);
    }
    return SBMDS_OK;
}

// One problem on the device: its operator in the internal landmark order
// (P's columns relabelled and rows re-sorted, CSR of P^T, c = P^T 1, W
// permuted and padded), the per-precision copies.  Host inputs were
// validated on the host and are uploaded first; device inputs are validated
// by kernels and never leave the device.
// The push form of the transposed product (SBMDS_FLAG_PUSH_T: vertex blocks
// scatter partial rows per landmark, a reduction adds them in block order)
// where the blocks touch few landmarks each: at least kPushMinEntries entries
// per (block, landmark) pair on average, else the row-gather form stays.
constexpr double kPushMinEntries = 4.0;

int build_push(sbmds_ctx *ctx, DevProblem &p, bool fp64, bool bf) {
    hipStream_t s = ctx->stream;
    const int64_t n = p.n, l = p.l, nnz = p.nnz;
    if (nnz <= 0 || nnz >= ((int64_t)1 << 31)) return SBMDS_OK;
    DevTmp tmp;
    const size_t tb = prep_push_tmp_bytes(nnz);
    OKCHK(tmp.alloc(tb));
    int64_t npairs = 0;
    HIPCHK(prep_push_pairs(p.rp, p.ci, n, l, nnz, tmp.p, tb, &npairs, s));
    if (npairs <= 0 || (double)nnz < kPushMinEntries * (double)npairs) return SBMDS_OK;
    const int64_t nvb = (n + kPushVB - 1) / kPushVB;
    PushOut po{};
    const int esz = fp64 ? 8 : 4;
    OKCHK(dalloc(ctx, (void **)&po.pb, (nvb + 1) * 4));
    OKCHK(dalloc(ctx, (void **)&po.pe, (npairs + 1) * 4));
    OKCHK(dalloc(ctx, (void **)&po.pvl, nnz));
    OKCHK(dalloc(ctx, (void **)&po.qp, (l + 1) * 4));
    OKCHK(dalloc(ctx, (void **)&po.ql, npairs * 4));
    OKCHK(dalloc(ctx, &po.pv, nnz * esz));
    if (bf) OKCHK(dalloc(ctx, &po.pv16, nnz * 2));
    OKCHK(dalloc(ctx, &p.ppart, (size_t)npairs * p.B * 8));
    const void *val = fp64 ? p.val[MODE_FP64] : p.val[MODE_FP32];
    HIPCHK(prep_push_fill(n, l, nnz, npairs, val, esz, bf ? p.val[MODE_BF16] : nullptr, po, tmp.p, tb, s));
    HIPCHK(hipStreamSynchronize(s));  // the scratch goes when this returns
    p.pb = po.pb;
    p.pe = po.pe;
    p.pvl = po.pvl;
    p.qp = po.qp;
    p.ql = po.ql;
    p.npairs = npairs;
    p.nvb = (int)nvb;
    if (fp64) {
        p.pval[MODE_FP64] = po.pv;
    } else {
        p.pval[MODE_FP32] = po.pv;
        p.pval[MODE_F64ACC] = po.pv;
        if (bf) p.pval[MODE_BF16] = po.pv16;
    }
    return SBMDS_OK;
}

template <typename T>
int prepare_problem(sbmds_ctx *ctx, const sbmds_problem &in, DevProblem &p, bool fp64, int idx) {
    const int64_t n = p.n, l = p.l, nnz = p.nnz;
    hipStream_t s = ctx->stream;
    const int32_t *drp = in.P_rowptr, *dci = in.P_col;
    const T *dval = (const T *)in.P_val, *dW = (const T *)in.W;
    DevTmp raw;
    if (in.mem == SBMDS_MEM_HOST) {
        // raw inputs in the caller's order, uploaded as they are
        const size_t b_rp = (size_t)(n + 1) * 4, b_ci = (size_t)nnz * 4, b_v = (size_t)nnz * sizeof(T);
        const size_t b_w = (size_t)l * l * sizeof(T);
        OKCHK(raw.alloc(b_rp + b_ci + b_v + b_w + 64));
        char *q = (char *)raw.p;
        int32_t *rrp = (int32_t *)q;
        int32_t *rci = (int32_t *)(q + ((b_rp + 15) & ~(size_t)15));
        T *rval = (T *)((char *)rci + ((b_ci + 15) & ~(size_t)15));
        T *rW = (T *)((char *)rval + ((b_v + 15) & ~(size_t)15));
        HIPCHK(hipMemcpyAsync(rrp, in.P_rowptr, b_rp, hipMemcpyHostToDevice, s));
        if (nnz) HIPCHK(hipMemcpyAsync(rci, in.P_col, b_ci, hipMemcpyHostToDevice, s));
        if (nnz) HIPCHK(hipMemcpyAsync(rval, in.P_val, b_v, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(rW, in.W, b_w, hipMemcpyHostToDevice, s));
        drp = rrp;
        dci = rci;
        dval = rval;
        dW = rW;
    } else {
        DevTmp terr;
        OKCHK(terr.alloc(8));
        unsigned long long *derr = (unsigned long long *)terr.p;
        unsigned long long herr = kPrepNoError;
        HIPCHK(hipMemcpyAsync(derr, &herr, 8, hipMemcpyHostToDevice, s));
        HIPCHK(prep_validate<T>(drp, dci, dval, dW, n, l, nnz, derr, s));
        HIPCHK(hipMemcpyAsync(&herr, derr, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (herr != kPrepNoError)
            return fail(SBMDS_EINVAL, "problem " + std::to_string(idx) + ": " + prep_error_text(herr));
    }
    std::vector<int32_t> order;
    OKCHK(landmark_order<T>(ctx, dW, l, order));
    p.lperm = order;
    std::vector<int32_t> inv(l);
    for (int64_t j = 0; j < l; ++j) inv[order[j]] = (int32_t)j;

    OKCHK(dalloc(ctx, (void **)&p.rp, (n + 1) * 4));
    OKCHK(dalloc(ctx, (void **)&p.ci, nnz * 4));
    OKCHK(dalloc(ctx, (void **)&p.rpT, (l + 1) * 4));
    OKCHK(dalloc(ctx, (void **)&p.ciT, nnz * 4));
    void *Wd = nullptr, *vd = nullptr, *vTd = nullptr, *cd = nullptr, *c16 = nullptr;
    const bool bf = !fp64 && ctx->opt.prec == SBMDS_BF16_FP32;
    OKCHK(dalloc(ctx, &vd, nnz * sizeof(T)));
    OKCHK(dalloc(ctx, &vTd, nnz * sizeof(T)));
    OKCHK(dalloc(ctx, &Wd, (size_t)l * p.lda * sizeof(T)));
    OKCHK(dalloc(ctx, &cd, l * 8));
    if (bf) OKCHK(dalloc(ctx, &c16, l * 8));
    HIPCHK(hipMemcpyAsync(p.rp, drp, (n + 1) * 4, hipMemcpyDeviceToDevice, s));
    DevTmp tperm, twork;
    OKCHK(tperm.alloc((size_t)l * 8));
    int32_t *dperm = (int32_t *)tperm.p, *dinv = dperm + l;
    HIPCHK(hipMemcpyAsync(dperm, order.data(), (size_t)l * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dinv, inv.data(), (size_t)l * 4, hipMemcpyHostToDevice, s));
    const size_t wb = prep_tmp_bytes(nnz, fp64);
    OKCHK(twork.alloc(wb));
    PrepIn pi{n, l, nnz, drp, dci, dval, dW, dperm, dinv};
    PrepOut po{p.lda, p.ci, p.rpT, p.ciT, vd, vTd, Wd, (double *)cd, (double *)c16};
    HIPCHK(prep_operator<T>(pi, po, twork.p, wb, s));
    if (fp64) {
        p.val[MODE_FP64] = vd;
        p.valT[MODE_FP64] = vTd;
        p.W[MODE_FP64] = Wd;
        p.c[MODE_FP64] = (double *)cd;
    } else {
        for (Mode m : {MODE_FP32, MODE_F64ACC}) {
            p.val[m] = vd;
            p.valT[m] = vTd;
            p.W[m] = Wd;
            p.c[m] = (double *)cd;
        }
        if (bf) {
            void *v16 = nullptr, *vT16 = nullptr, *W16 = nullptr;
            OKCHK(dalloc(ctx, &v16, nnz * 2));
            OKCHK(dalloc(ctx, &vT16, nnz * 2));
            OKCHK(dalloc(ctx, &W16, (size_t)l * p.lda * 2));
            HIPCHK(launch_f32_to_bf16((const float *)vd, v16, nnz, s));
            HIPCHK(launch_f32_to_bf16((const float *)vTd, vT16, nnz, s));
            HIPCHK(launch_f32_to_bf16((const float *)Wd, W16, (int64_t)l * p.lda, s));
            p.val[MODE_BF16] = v16;
            p.valT[MODE_BF16] = vT16;
            p.W[MODE_BF16] = W16;
            p.c[MODE_BF16] = (double *)c16;
        }
    }
    if ((ctx->opt.flags & SBMDS_FLAG_PUSH_T) && spmmt_push_width(p.B)) OKCHK(build_push(ctx, p, fp64, bf));
    // the scratch is released when this returns: the stream must be done with it
    HIPCHK(hipStreamSynchronize(s));
    return SBMDS_OK;
}

// Whether problem p runs the transposed product of mode m in its push form.
bool push_form(const Batch &bt, const DevProblem &p, int m) {
    return bt.spmmt_push[m] && p.pb != nullptr && p.pval[m] != nullptr;
}

// Launch tables of the context: one view per problem and, per kind of
// launch and mode, the prefix sums of the blocks each problem takes.
int build_batch(sbmds_ctx *ctx, SolveSet &set) {
    const int np = (int)set.probs.size();
    Batch &bt = set.bt;
    bt.nprob = np;
    bt.B = set.probs[0].B;
    bt.b = set.probs[0].b;
    bt.k = set.probs[0].k;
    bt.max_l = 0;
    for (const DevProblem &q : set.probs) bt.max_l = std::max<int64_t>(bt.max_l, q.l);
    for (int m = 0; m < NUM_MODES; ++m) {
        bt.spmmt_wpr[m] = set.tune[m].spmmt_wpr;
        bt.gemm_mfma[m] = set.tune[m].gemm_mfma && gemm_mfma((Mode)m, bt.B) ? 1 : 0;
        bool packed = sym_supported((Mode)m, bt.B);
        for (const DevProblem &q : set.probs) packed = packed && q.Wp != nullptr;
        bt.gemm_sym[m] = set.tune[m].gemm_sym && packed ? 1 : 0;
        bt.spmm_wpe8[m] = set.tune[m].spmm_wpe == 8 ? 1 : 0;  // read by the widths that have the form
        // each problem takes its own form of the transposed product, so a
        // problem solves the same alone or beside others
        bool push = false;
        for (const DevProblem &q : set.probs) push = push || (q.pb != nullptr && q.pval[m] != nullptr);
        bt.spmmt_push[m] = push && spmmt_push_width(bt.B) ? 1 : 0;
    }

    std::vector<ProbView> views(np);
    std::vector<int> offs((size_t)NUM_BK * NUM_MODES * (np + 1), 0);
    int64_t zoff = 0, loff = 0;
    for (int i = 0; i < np; ++i) {
        const DevProblem &p = set.probs[i];
        ProbView &v = views[i];
        std::memset(&v, 0, sizeof(v));
        v.n = (int)p.n;
        v.l = (int)p.l;
        v.nnz = (int)p.nnz;
        v.lda = p.lda;
        v.rp = p.rp;
        v.ci = p.ci;
        v.rpT = p.rpT;
        v.ciT = p.ciT;
        for (int m = 0; m < NUM_MODES; ++m) {
            v.val[m] = p.val[m];
            v.valT[m] = p.valT[m];
            v.W[m] = p.W[m];
            v.c[m] = p.c[m];
            const LaunchCfg &c = set.cfg[i][m];
            v.spmm_blocks[m] = c.spmm_blocks;
            v.gemm_rowtiles[m] = (int)((p.l + c.gemm_rt - 1) / c.gemm_rt);
            v.gemm_ksplit[m] = c.gemm_ksplit;
            v.gemm_kchunk[m] = c.gemm_kchunk;
            v.sym_c[m] = set.tune[m].sym_c;
            if (bt.gemm_sym[m]) v.gemm_rowtiles[m] = p.lda / 64;  // H / s partials per 64-row tile
        }
        v.Wp = p.Wp;
        v.Y0 = p.Y[0];
        v.Y1 = p.Y[1];
        v.T = p.T;
        v.U = p.U;
        v.gpart = p.gpart;
        v.red_gemm = p.red_gemm;
        v.red_spmm = p.red_spmm;
        v.tile_cnt = p.tile_cnt;
        v.gemm_cnt = p.gemm_cnt;
        v.spmm_cnt = p.spmm_cnt;
        v.st = p.st;
        v.X0 = p.X0;
        v.pb = p.pb;
        v.pe = p.pe;
        v.qp = p.qp;
        v.ql = p.ql;
        v.pvl = p.pvl;
        for (int m = 0; m < NUM_MODES; ++m) v.pval[m] = p.pval[m];
        v.ppart = p.ppart;
        v.zoff = zoff;
        v.loff = loff;
        v.host_sum = (char *)set.host_sum_dev + (size_t)i * sizeof(Summary);
        zoff += p.n * p.k;
        loff += p.l;
    }
    for (int kd = 0; kd < NUM_BK; ++kd) {
        for (int m = 0; m < NUM_MODES; ++m) {
            int *o = offs.data() + ((size_t)kd * NUM_MODES + m) * (np + 1);
            int64_t acc = 0;
            for (int i = 0; i < np; ++i) {
                o[i] = (int)acc;
                const DevProblem &p = set.probs[i];
                const ProbView &v = views[i];
                int64_t nb = 0;
                switch (kd) {
                    case BK_SPMM: nb = v.spmm_blocks[m]; break;
                    case BK_SPMMT:
                        nb = push_form(bt, p, m) ? 0 : (p.l + 4 / bt.spmmt_wpr[m] - 1) / (4 / bt.spmmt_wpr[m]);
                        break;
                    case BK_GEMM:
                        nb = bt.gemm_sym[m] ? sym_regions(p.lda / 64, sym_region_rows((Mode)m, bt.B), v.sym_c[m])
                                            : (int64_t)v.gemm_rowtiles[m] * v.gemm_ksplit[m];
                        break;
                    case BK_GEMMF: nb = bt.gemm_sym[m] ? p.lda / 64 : 0; break;
                    case BK_ELEM_NB: nb = (p.n * p.B + 255) / 256; break;
                    case BK_ELEM_LB: nb = (p.l * p.B + 255) / 256; break;
                    case BK_PUSH: nb = push_form(bt, p, m) ? p.nvb : 0; break;
                    case BK_PUSHR: {
                        const int rows = spmmt_push_rows((Mode)m, bt.B);
                        nb = push_form(bt, p, m) ? (p.l + rows - 1) / rows : 0;
                        break;
                    }
                    default: nb = (p.n + 255) / 256; break;
                }
                acc += nb;
            }
            if (acc >= ((int64_t)1 << 31)) return fail(SBMDS_EINVAL, "too many blocks for one launch");
            o[np] = (int)acc;
            bt.total[kd][m] = (int)acc;
        }
    }
    if (!bt.views) OKCHK(dalloc(ctx, (void **)&bt.views, sizeof(ProbView) * np));
    if (!bt.offs) OKCHK(dalloc(ctx, (void **)&bt.offs, sizeof(int) * offs.size()));
    HIPCHK(hipMemcpyAsync(bt.views, views.data(), sizeof(ProbView) * np, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(bt.offs, offs.data(), sizeof(int) * offs.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));  // host tables go out of scope
    size_t zmax = 0;
    for (const DevProblem &p : set.probs) zmax += (size_t)p.n * p.k;
    set.zstage_bytes = zmax * (ctx->opt.prec == SBMDS_FP64 ? 8 : 4);
    return SBMDS_OK;
}

// Pinned summaries and the contiguous solver states of a set.
int alloc_set(sbmds_ctx *ctx, SolveSet &set, int nprob) {
    set.probs.resize(nprob);
    set.cfg.resize(nprob);
    set.cur_ybuf.assign(nprob, 0);
    set.cur_mode.assign(nprob, schedule(ctx->opt).back().mode);
    if (hipHostMalloc((void **)&set.host_sum, sizeof(Summary) * nprob, hipHostMallocMapped) != hipSuccess)
        return fail(SBMDS_ENOMEM, "pinned host allocation failed");
    std::memset(set.host_sum, 0, sizeof(Summary) * nprob);
    HIPCHK(hipHostGetDevicePointer(&set.host_sum_dev, set.host_sum, 0));
    OKCHK(dalloc(ctx, (void **)&set.st_all, sizeof(SolveState) * nprob));
    HIPCHK(hipMemsetAsync(set.st_all, 0, sizeof(SolveState) * nprob, ctx->stream));
    return SBMDS_OK;
}

// Launch configurations and the iteration buffers of problem i of a set
// (its operator is already on the device).
int alloc_work(sbmds_ctx *ctx, SolveSet &set, int i) {
    DevProblem &p = set.probs[i];
    // scratch for every launch shape the tuner may pick
    for (int m = 0; m < NUM_MODES; ++m) {
        const int rpb = spmm_rows_per_block((Mode)m, p.B);
        p.max_spmm_blocks = std::max<int>(p.max_spmm_blocks,
                                          (int)std::min<int64_t>((p.n + rpb - 1) / rpb, kMaxSpmmBlocks));
        for (int mf = 0; mf < 2; ++mf) {
            const int rt = gemm_rows_per_tile((Mode)m, p.B, mf);
            p.max_rowtiles = std::max(p.max_rowtiles, (int)((p.l + rt - 1) / rt));
        }
    }
    p.max_spmm_blocks = std::max(p.max_spmm_blocks, 1);
    p.max_ksplit = std::max(1, std::min(p.lda / 64, kMaxGemmSplit));
    const int B = p.B;
    size_t gpart_elems = (size_t)p.max_ksplit * p.lda * B;
    if (p.Wp) {
        // slots of the packed product: R + C per region, 64 x B each, for
        // every region shape the tuner may pick
        const int nt = p.lda / 64;
        for (int R : {4, 8})
            for (int cw : {8, 16, 32})
                gpart_elems = std::max(gpart_elems, (size_t)sym_regions(nt, R, cw) * (R + cw) * 64 * B);
    }
    const int EG = B * (B + 1) / 2 + B;   // Gram triangle + column sums
    const int EH = B * B + B;             // H + s
    const int nspmm_cnt = tree_counter_count(p.max_spmm_blocks, kFan);
    const int ngemm_cnt = tree_counter_count(p.max_rowtiles, kFan);
    const size_t ncnt = (size_t)p.max_rowtiles + nspmm_cnt + ngemm_cnt;
    unsigned *cnt = nullptr;
    OKCHK(dalloc(ctx, &p.Y[0], (size_t)p.n * B * 8));
    OKCHK(dalloc(ctx, &p.Y[1], (size_t)p.n * B * 8));
    OKCHK(dalloc(ctx, &p.T, (size_t)p.lda * B * 8));
    OKCHK(dalloc(ctx, &p.U, (size_t)p.lda * B * 8));
    OKCHK(dalloc(ctx, &p.gpart, gpart_elems * 8));
    OKCHK(dalloc(ctx, (void **)&p.red_gemm, tree_scratch_elems(p.max_rowtiles, EH, kFan) * 8));
    OKCHK(dalloc(ctx, (void **)&p.red_spmm, tree_scratch_elems(p.max_spmm_blocks, EG, kFan) * 8));
    OKCHK(dalloc(ctx, (void **)&cnt, ncnt * 4));
    p.st = set.st_all + i;
    p.tile_cnt = cnt;
    p.spmm_cnt = cnt + p.max_rowtiles;
    p.gemm_cnt = p.spmm_cnt + nspmm_cnt;
    HIPCHK(hipMemsetAsync(p.T, 0, (size_t)p.lda * B * 8, ctx->stream));
    HIPCHK(hipMemsetAsync(p.U, 0, (size_t)p.lda * B * 8, ctx->stream));
    HIPCHK(hipMemsetAsync(cnt, 0, ncnt * 4, ctx->stream));
    return SBMDS_OK;
}

// The landmark problem of main problem i for the landmark MDS start: P = I
// (l x l), the same W, so its operator is -1/2 J W J on the landmarks.
int make_landmark_problem(sbmds_ctx *ctx, int i) {
    const DevProblem &mp = ctx->main.probs[i];
    DevProblem &p = ctx->lmk.probs[i];
    const int64_t l = mp.l;
    p.n = l;
    p.l = l;
    p.nnz = l;
    p.lda = mp.lda;
    p.b = mp.b;
    p.B = mp.B;
    p.k = mp.k;
    std::vector<int32_t> iota(l + 1);
    for (int64_t j = 0; j <= l; ++j) iota[j] = (int32_t)j;
    const bool fp64 = ctx->opt.prec == SBMDS_FP64;
    const size_t esz = fp64 ? 8 : 4;
    std::vector<char> ones(l * esz);
    for (int64_t j = 0; j < l; ++j) {
        if (fp64) reinterpret_cast<double *>(ones.data())[j] = 1.0;
        else reinterpret_cast<float *>(ones.data())[j] = 1.0f;
    }
    std::vector<double> c(l, 1.0);
    void *vals = nullptr, *cd = nullptr;
    OKCHK(dalloc(ctx, (void **)&p.rp, (l + 1) * 4));
    OKCHK(dalloc(ctx, (void **)&p.ci, l * 4));
    OKCHK(dalloc(ctx, &vals, l * esz));
    OKCHK(dalloc(ctx, &cd, l * 8));
    HIPCHK(hipMemcpyAsync(p.rp, iota.data(), (l + 1) * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(p.ci, iota.data(), l * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(vals, ones.data(), l * esz, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(cd, c.data(), l * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));  // host vectors go out of scope
    p.rpT = p.rp;
    p.ciT = p.ci;
    for (Mode m : {MODE_FP32, MODE_F64ACC, MODE_FP64}) {
        if ((m == MODE_FP64) != fp64) continue;
        p.val[m] = vals;
        p.valT[m] = vals;
        p.W[m] = mp.W[m];
        p.c[m] = (double *)cd;
    }
    p.Wp = mp.Wp;
    return alloc_work(ctx, ctx->lmk, i);
}

// Learned start: load the network and keep device copies of the vertex
// positions and landmark ids of every problem.
int setup_learned(sbmds_ctx *ctx, const sbmds_problem *probs, int nprob) {
    OKCHK(sbmds_mlp_load(ctx->opt.mlp_weights, ctx->stream, &ctx->net));
    if (mlp::out_width(ctx->net) != ctx->opt.k)
        return fail(SBMDS_EINVAL, "the network predicts " + std::to_string(mlp::out_width(ctx->net)) +
                                      " coordinates but k = " + std::to_string(ctx->opt.k));
    ctx->xyz.assign(nprob, nullptr);
    ctx->lmv.assign(nprob, nullptr);
    int64_t maxl = 0;
    ctx->total_l = 0;
    for (int i = 0; i < nprob; ++i) {
        const sbmds_problem &in = probs[i];
        const hipMemcpyKind kind = in.mem == SBMDS_MEM_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
        std::vector<int32_t> hl(in.l);
        HIPCHK(hipMemcpy(hl.data(), in.landmark_vertex, in.l * 4, kind));
        for (int64_t j = 0; j < in.l; ++j)
            if (hl[j] < 0 || hl[j] >= in.n)
                return fail(SBMDS_EINVAL, "problem " + std::to_string(i) + ": landmark_vertex out of range");
        OKCHK(dalloc(ctx, (void **)&ctx->xyz[i], (size_t)in.n * 12));
        OKCHK(dalloc(ctx, (void **)&ctx->lmv[i], (size_t)in.l * 4));
        HIPCHK(hipMemcpyAsync(ctx->xyz[i], in.xyz, (size_t)in.n * 12,
                              in.mem == SBMDS_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              ctx->stream));
        std::vector<int32_t> hlp(in.l);  // in the internal landmark order
        for (int64_t j = 0; j < in.l; ++j) hlp[j] = hl[ctx->main.probs[i].lperm[j]];
        HIPCHK(hipMemcpyAsync(ctx->lmv[i], hlp.data(), (size_t)in.l * 4, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));  // hl goes out of scope
        maxl = std::max<int64_t>(maxl, in.l);
        ctx->total_l += in.l;
    }
    OKCHK(dalloc(ctx, (void **)&ctx->feat, (size_t)ctx->total_l * mlp::kIn * 4));
    OKCHK(dalloc(ctx, (void **)&ctx->learned, (size_t)ctx->total_l * ctx->opt.k * 4));
    OKCHK(dalloc(ctx, (void **)&ctx->rowmax, (size_t)maxl * 8));
    // features of each problem's landmarks (they depend on the inputs only);
    // the forward pass over all of them runs in every sbmds_embed, as part of
    // the start block, on work buffers reserved here
    const Mode wm = ctx->opt.prec == SBMDS_FP64 ? MODE_FP64 : MODE_FP32;
    int64_t loff = 0;
    for (int i = 0; i < nprob; ++i) {
        const DevProblem &p = ctx->main.probs[i];
        OKCHK(mlp::launch_features(p.W[wm], wm == MODE_FP64 ? 1 : 0, p.l, p.lda, ctx->xyz[i], ctx->lmv[i],
                                   ctx->feat + loff * mlp::kIn, ctx->rowmax, ctx->stream));
        loff += p.l;
    }
    OKCHK(mlp::reserve_rows(ctx->net, ctx->total_l));
    return SBMDS_OK;
}

int device_ok(int *dev) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(SBMDS_ENODEV, "no HIP device available");
    HIPCHK(hipGetDevice(dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, *dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SBMDS_ENODEV, std::string("device is ") + prop.gcnArchName + ", this library targets gfx950");
    return SBMDS_OK;
}

int create_impl(const sbmds_problem *probs, int nprob, const sbmds_options *opt_in, sbmds_ctx **out) {
    if (!out) return fail(SBMDS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!probs || nprob < 1) return fail(SBMDS_EINVAL, "need at least one problem");
    sbmds_options o;
    sbmds_default_options(&o);
    if (opt_in) o = *opt_in;
    OKCHK(check_options(o));
    for (int i = 0; i < nprob; ++i) OKCHK(check_shape(probs[i], o, i));
    const bool fp64 = o.prec == SBMDS_FP64;
    for (int i = 0; i < nprob; ++i) {
        const sbmds_problem &p = probs[i];
        if (p.mem != SBMDS_MEM_HOST) continue;
        if (fp64)
            OKCHK(check_contents<double>(p, p.P_rowptr, p.P_col, (const double *)p.P_val, (const double *)p.W, i));
        else
            OKCHK(check_contents<float>(p, p.P_rowptr, p.P_col, (const float *)p.P_val, (const float *)p.W, i));
    }
    int dev = 0;
    OKCHK(device_ok(&dev));

    sbmds_ctx *ctx = new sbmds_ctx();
    ctx->device = dev;
    ctx->opt = o;
    ctx->stream = (hipStream_t)o.stream;
    if (!ctx->stream) {
        // a stream of our own (it synchronises with the null stream), so
        // that rounds of iterations can be captured as graphs
        if (hipStreamCreate(&ctx->own_stream) != hipSuccess) {
            delete ctx;
            return fail(SBMDS_EHIP, "hipStreamCreate failed");
        }
        ctx->stream = ctx->own_stream;
    }
    ctx->timing = (o.flags & SBMDS_FLAG_KERNEL_TIMING) != 0;
    auto cleanup = [&](int rc) {
        sbmds_destroy(ctx);
        return rc;
    };
    if (int rc = alloc_set(ctx, ctx->main, nprob); rc < 0) return cleanup(rc);

    const size_t esz = fp64 ? 8 : 4;
    {
        // W is also kept as its packed upper triangle once the batch's float32
        // W no longer fits the caches (the dense product then streams half)
        double wbytes = 0.0;
        bool fits = !fp64;
        for (int i = 0; i < nprob; ++i) {
            const int64_t lda = (probs[i].l + 63) / 64 * 64;
            wbytes += 4.0 * (double)probs[i].l * (double)probs[i].l;
            fits = fits && lda / 64 <= kSymMaxTiles;
        }
        ctx->packed = fits && !(o.flags & SBMDS_FLAG_FULL_W) &&
                      (wbytes > kPackMinBytes || (o.flags & SBMDS_FLAG_PACK_W));
    }
    for (int i = 0; i < nprob; ++i) {
        const sbmds_problem &in = probs[i];
        DevProblem &p = ctx->main.probs[i];
        p.n = in.n;
        p.l = in.l;
        p.nnz = in.nnz;
        p.lda = (int)((in.l + 63) / 64) * 64;
        p.b = o.block;
        p.B = kernel_width(o.block);
        p.k = o.k;
        // host inputs were validated above; device inputs are validated on the device
        int rc = fp64 ? prepare_problem<double>(ctx, in, p, true, i) : prepare_problem<float>(ctx, in, p, false, i);
        if (rc < 0) return cleanup(rc);
        if (ctx->packed) {
            const size_t pk = (size_t)sym_strip_base(p.lda / 64, p.lda) * 4;
            if ((rc = dalloc(ctx, (void **)&p.Wp, pk)) < 0) return cleanup(rc);
            if (launch_pack_sym((const float *)p.W[MODE_FP32], p.l, p.lda, p.Wp, ctx->stream) != hipSuccess)
                return cleanup(fail(SBMDS_EHIP, "packing W failed"));
        }

        if ((rc = alloc_work(ctx, ctx->main, i)) < 0) return cleanup(rc);
        if (o.start == SBMDS_START_USER) {
            void *x0 = nullptr;
            const size_t xb = (size_t)p.n * p.b * esz;
            if ((rc = dalloc(ctx, &x0, xb)) < 0) return cleanup(rc);
            if (hipMemcpyAsync(x0, in.X0, xb,
                               in.mem == SBMDS_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                               ctx->stream) != hipSuccess)
                return cleanup(fail(SBMDS_EHIP, "copying X0 failed"));
            p.X0 = x0;
        }
    }
    for (int m = 0; m < NUM_MODES; ++m) ctx->main.tune[m] = default_tune((Mode)m, ctx->main.probs);
    apply_tune(ctx->main);
    if (int rc = build_batch(ctx, ctx->main); rc < 0) return cleanup(rc);
    if (o.tune_cache)
        if (int rc = autotune(ctx, ctx->main); rc < 0) return cleanup(rc);
    if (o.start == SBMDS_START_LEARNED)
        if (int rc = setup_learned(ctx, probs, nprob); rc < 0) return cleanup(rc);
    if (o.start == SBMDS_START_LMDS) {
        if (int rc = alloc_set(ctx, ctx->lmk, nprob); rc < 0) return cleanup(rc);
        for (int i = 0; i < nprob; ++i)
            if (int rc = make_landmark_problem(ctx, i); rc < 0) return cleanup(rc);
        for (int m = 0; m < NUM_MODES; ++m) ctx->lmk.tune[m] = default_tune((Mode)m, ctx->lmk.probs);
        apply_tune(ctx->lmk);
        if (int rc = build_batch(ctx, ctx->lmk); rc < 0) return cleanup(rc);
    }
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return cleanup(fail(SBMDS_EHIP, "create: stream sync failed"));
    *out = ctx;
    return SBMDS_OK;
}

}  // namespace

extern "C" {

void sbmds_default_options(sbmds_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->k = 3;
    o->block = 16;
    o->prec = SBMDS_FP32;
    o->start = SBMDS_START_RANDOM;
    o->tol = 1e-6;
    o->max_iter = 500;
    o->seed = 12345;
    o->stream = nullptr;
}

int sbmds_create(const sbmds_problem *probs, int nprob, const sbmds_options *opt, sbmds_ctx **out) {
    g_err.clear();
    try {
        return create_impl(probs, nprob, opt, out);
    } catch (const std::exception &e) {
        return fail(SBMDS_ENOMEM, std::string("host exception: ") + e.what());
    } catch (...) {
        return fail(SBMDS_ENOMEM, "unknown host exception");
    }
}

int sbmds_embed(sbmds_ctx *ctx, double *eigvals, void *Z, int Z_mem, sbmds_report *reports) {
    g_err.clear();
    if (!ctx) return fail(SBMDS_EINVAL, "ctx is NULL");
    if (Z && Z_mem != SBMDS_MEM_HOST && Z_mem != SBMDS_MEM_DEVICE) return fail(SBMDS_EINVAL, "Z_mem must be 0 or 1");
    try {
        HIPCHK(hipSetDevice(ctx->device));
        const SolveSet &set = ctx->main;
        const int np = (int)set.probs.size();
        const bool zdouble = ctx->opt.prec == SBMDS_FP64;
        void *dz = Z;
        if (Z && Z_mem == SBMDS_MEM_HOST) {
            if (!ctx->zstage) OKCHK(dalloc(ctx, &ctx->zstage, set.zstage_bytes));
            dz = ctx->zstage;
        }
        // the embedding (and its copy to the host) is enqueued after each
        // round of the solve; the one after the last round is the result
        std::function<int()> output;
        if (Z)
            output = [&]() -> int {
                OKCHK(timed(ctx, "embedding", 0.0, 0.0,
                            [&] { return launch_embedding(set.bt, dz, zdouble ? 1 : 0, ctx->stream); }));
                if (Z_mem == SBMDS_MEM_HOST)
                    HIPCHK(hipMemcpyAsync(Z, dz, set.zstage_bytes, hipMemcpyDeviceToHost, ctx->stream));
                return SBMDS_OK;
            };
        int worst = solve_all(ctx, reports, output);
        if (worst < 0) return worst;
        if (eigvals)
            for (int i = 0; i < np; ++i)
                for (int j = 0; j < set.probs[i].k; ++j)
                    eigvals[(size_t)i * set.probs[i].k + j] = set.host_sum[i].theta[j];
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (ctx->timing) collect_timing(ctx);
        return worst;
    } catch (const std::exception &e) {
        return fail(SBMDS_ENOMEM, std::string("host exception: ") + e.what());
    }
}

// The comparison solvers on every problem of a context, one after the other:
// operator views in the context's top precision, Z in the layout of
// sbmds_embed.
static int run_compare(sbmds_ctx *ctx, const char *what, void *Z, int Z_mem, double *eigvals,
                       sbmds_solver_report *reports,
                       const std::function<int(const CmpOp &, void *, CmpResult *)> &solve) {
    g_err.clear();
    if (!ctx) return fail(SBMDS_EINVAL, "ctx is NULL");
    if (Z && Z_mem != SBMDS_MEM_HOST && Z_mem != SBMDS_MEM_DEVICE) return fail(SBMDS_EINVAL, "Z_mem must be 0 or 1");
    if (ctx->opt.k > kCmpMaxK) return fail(SBMDS_EINVAL, std::string(what) + " returns at most 16 eigenpairs");
    try {
        HIPCHK(hipSetDevice(ctx->device));
        const SolveSet &set = ctx->main;
        const bool zd = ctx->opt.prec == SBMDS_FP64;
        const Mode mode = zd ? MODE_FP64 : MODE_FP32;
        const size_t esz = zd ? 8 : 4;
        void *zbuf = nullptr;  // device output of one problem
        size_t zcap = 0;
        for (const DevProblem &p : set.probs) zcap = std::max(zcap, (size_t)p.n * p.k * esz);
        if (!ctx->zstage) OKCHK(dalloc(ctx, &ctx->zstage, set.zstage_bytes));
        zbuf = ctx->zstage;
        (void)zcap;
        int worst = SBMDS_OK;
        size_t zoff = 0;
        for (size_t i = 0; i < set.probs.size(); ++i) {
            const DevProblem &p = set.probs[i];
            CmpOp op;
            op.n = p.n;
            op.l = p.l;
            op.nnz = p.nnz;
            op.lda = p.lda;
            op.rp = p.rp;
            op.ci = p.ci;
            op.rpT = p.rpT;
            op.ciT = p.ciT;
            op.val = p.val[mode];
            op.valT = p.valT[mode];
            op.W = p.W[mode];
            op.c = p.c[mode];
            op.f64 = zd;
            if (!op.val || !op.valT || !op.W || !op.c)
                return fail(SBMDS_EINVAL, std::string(what) + ": the context holds no operator in its top precision");
            void *dz = Z_mem == SBMDS_MEM_DEVICE && Z ? (void *)((char *)Z + zoff) : (void *)((char *)zbuf + zoff);
            CmpResult r;
            const auto t0 = std::chrono::steady_clock::now();
            const int rc = solve(op, dz, &r);
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (rc < 0) return rc;
            worst = std::max(worst, rc);
            if (eigvals)
                for (int j = 0; j < p.k; ++j) eigvals[i * p.k + j] = r.eig[j];
            if (reports) {
                sbmds_solver_report &o = reports[i];
                std::memset(&o, 0, sizeof(o));
                o.status = rc;
                o.steps = r.steps;
                o.basis = r.basis;
                o.nonpositive = r.nonpositive;
                o.ms_total = ms;
                for (int j = 0; j < p.k; ++j) {
                    o.eig[j] = r.eig[j];
                    o.err_bound[j] = r.bound[j];
                    o.resid[j] = r.resid[j];
                }
            }
            zoff += (size_t)p.n * p.k * esz;
        }
        if (Z && Z_mem == SBMDS_MEM_HOST) {
            HIPCHK(hipMemcpyAsync(Z, zbuf, zoff, hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
        }
        return worst;
    } catch (const std::exception &e) {
        return fail(SBMDS_ENOMEM, std::string("host exception: ") + e.what());
    }
}

int sbmds_embed_lanczos(sbmds_ctx *ctx, int block, int max_steps, double *eigvals, void *Z, int Z_mem,
                        sbmds_solver_report *reports) {
    if (ctx && (block != 1 && block != 2 && block != 4 && block != 8))
        return fail(SBMDS_EINVAL, "Lanczos block must be 1, 2, 4 or 8");
    if (ctx && max_steps < 1) return fail(SBMDS_EINVAL, "max_steps must be >= 1");
    return run_compare(ctx, "sbmds_embed_lanczos", Z, Z_mem, eigvals, reports,
                       [&](const CmpOp &op, void *dz, CmpResult *r) {
                           return lanczos_solve(op, ctx->opt.k, block, max_steps, ctx->opt.tol, ctx->opt.seed, dz,
                                                ctx->opt.prec == SBMDS_FP64 ? 1 : 0, r, ctx->stream);
                       });
}

int sbmds_embed_bmds(sbmds_ctx *ctx, double *eigvals, void *Z, int Z_mem, sbmds_solver_report *reports) {
    return run_compare(ctx, "sbmds_embed_bmds", Z, Z_mem, eigvals, reports,
                       [&](const CmpOp &op, void *dz, CmpResult *r) {
                           return bmds_solve(op, ctx->opt.k, dz, ctx->opt.prec == SBMDS_FP64 ? 1 : 0, r,
                                             ctx->stream);
                       });
}

int sbmds_get_block(sbmds_ctx *ctx, int prob, void *X, int X_mem) {
    g_err.clear();
    if (!ctx || !X) return fail(SBMDS_EINVAL, "ctx and X must be non-NULL");
    if (prob < 0 || prob >= (int)ctx->main.probs.size()) return fail(SBMDS_EINVAL, "problem index out of range");
    if (X_mem != SBMDS_MEM_HOST && X_mem != SBMDS_MEM_DEVICE) return fail(SBMDS_EINVAL, "X_mem must be 0 or 1");
    const DevProblem &p = ctx->main.probs[prob];
    const bool xd = ctx->opt.prec == SBMDS_FP64;
    const size_t bytes = (size_t)p.n * p.b * (xd ? 8 : 4);
    void *dx = X;
    HIPCHK(hipSetDevice(ctx->device));
    if (X_mem == SBMDS_MEM_HOST) HIPCHK(hipMalloc(&dx, bytes));
    hipError_t e = launch_block_out((Mode)ctx->main.cur_mode[prob], p, ctx->main.cur_ybuf[prob], dx, xd ? 1 : 0, ctx->stream);
    if (e == hipSuccess && X_mem == SBMDS_MEM_HOST) e = hipMemcpyAsync(X, dx, bytes, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (X_mem == SBMDS_MEM_HOST) (void)hipFree(dx);
    if (e != hipSuccess) return fail(SBMDS_EHIP, std::string("sbmds_get_block: ") + hipGetErrorString(e));
    return SBMDS_OK;
}

int sbmds_kernel_stats(sbmds_ctx *ctx, sbmds_kernel_stat *out, int max) {
    if (!ctx) return fail(SBMDS_EINVAL, "ctx is NULL");
    const int nst = (int)ctx->stats.size();
    for (int i = 0; i < nst && out && i < max; ++i) {
        std::memset(&out[i], 0, sizeof(out[i]));
        std::snprintf(out[i].name, sizeof(out[i].name), "%s", ctx->stats[i].name.c_str());
        out[i].launches = ctx->stats[i].launches;
        out[i].ms_total = ctx->stats[i].ms;
        out[i].bytes_total = ctx->stats[i].bytes;
        out[i].flops_total = ctx->stats[i].flops;
    }
    return nst;
}

void sbmds_reset_kernel_stats(sbmds_ctx *ctx) {
    if (ctx) ctx->stats.clear();
}

void sbmds_destroy(sbmds_ctx *ctx) {
    if (!ctx) return;
    if (ctx->stream || !ctx->allocs.empty()) (void)hipStreamSynchronize(ctx->stream);
    for (SolveSet *set : {&ctx->main, &ctx->lmk})
        for (auto &g : set->graphs) {
            (void)hipGraphExecDestroy(g.second.second);
            (void)hipGraphDestroy(g.second.first);
        }
    if (ctx->net) sbmds_mlp_destroy(ctx->net);
    for (void *p : ctx->allocs) (void)hipFree(p);
    for (auto &pe : ctx->pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->main.host_sum) (void)hipHostFree(ctx->main.host_sum);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    if (ctx->lmk.host_sum) (void)hipHostFree(ctx->lmk.host_sum);
    delete ctx;
}

const char *sbmds_last_error(void) { return g_err.c_str(); }

int sbmds_version(void) { return (SBMDS_VERSION_MAJOR << 16) | SBMDS_VERSION_MINOR; }

}  // extern "C"
