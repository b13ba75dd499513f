/*
 * sbmds.h -- C ABI of the sparse biharmonic MDS (sBMDS) embedding path on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (Turek & Huth, "Efficient, sparse representation of manifold
 * distance matrices for classical scaling", Section 3.3, with classical MDS
 * from Section 2.3): given the sparse interpolation operator P (n x l, the
 * thresholded biharmonic operator of Section 3.1 / Eq. (PDefinition)) and
 * the landmark block W (l x l; here the SQUARED landmark geodesic
 * distances, the matrix classical scaling needs), compute the k
 * algebraically largest eigenpairs (lambda_i, v_i) of
 *
 *        B = -1/2 * J * P * W * P^T * J,      J = I - 1 1^T / n,
 *
 * and the embedding Z = V_k * Lambda_k^{1/2}, without forming any n x n
 * matrix.  The paper names a Lanczos method on matrix-vector products for
 * this step; this library runs block subspace iteration with a
 * Rayleigh-Ritz step on the same implicit operator, which reaches the same
 * eigenpairs.  Coordinates whose eigenvalue is not positive are returned
 * as zero and flagged in the report.
 *
 * Conventions for every function:
 *   - All functions have C linkage; no exception crosses the boundary.
 *   - Negative return values are errors: no output was written and
 *     sbmds_last_error() returns a message (thread-local, valid until the
 *     next call on the same thread).
 *   - SBMDS_ENOCONV (positive) means the iteration limit was reached; the
 *     outputs hold the best estimate and the report holds its error bounds.
 *   - The caller owns every array it passes.  sbmds_create copies what it
 *     needs, so inputs may be freed or reused once it returns.
 *   - A context owns all device memory it allocated until sbmds_destroy.
 *     It is bound to the HIP device that was current at sbmds_create and to
 *     the stream given in the options; it is not thread-safe, but any number
 *     of contexts may coexist.
 */
#ifndef SBMDS_H
#define SBMDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBMDS_VERSION_MAJOR 0
#define SBMDS_VERSION_MINOR 1
#define SBMDS_MAX_BLOCK 64 /* largest subspace block the kernels carry */

typedef struct sbmds_ctx sbmds_ctx; /* opaque */

typedef enum {
    SBMDS_OK = 0,
    SBMDS_ENOCONV = 1,     /* warning: max_iter reached, outputs are best effort */
    SBMDS_EINVAL = -1,     /* invalid argument or malformed input */
    SBMDS_ENOMEM = -2,     /* device allocation failed or mem_cap exceeded */
    SBMDS_EHIP = -3,       /* a HIP runtime call failed */
    SBMDS_ENODEV = -4,     /* no usable gfx950 device */
    SBMDS_EBREAKDOWN = -5  /* non-finite values appeared in the block solver */
} sbmds_status;

typedef enum {
    SBMDS_FP64 = 0,      /* P, W, vectors and accumulation in float64 */
    SBMDS_FP32 = 1,      /* float32 storage and accumulation, float64 block algebra */
    SBMDS_BF16_FP32 = 2  /* bfloat16 bulk iterations, then float32 refinement */
} sbmds_precision;

typedef enum {
    SBMDS_START_RANDOM = 0, /* seeded Gaussian block (counter-based generator) */
    SBMDS_START_LMDS = 1,   /* landmark MDS of W lifted through P */
    SBMDS_START_LEARNED = 2,/* MLP prediction from landmark features, lifted through P;
                               the features are made once, in sbmds_create, and
                               the network's forward pass runs in every sbmds_embed */
    SBMDS_START_USER = 3    /* caller-supplied block (sbmds_problem.X0), e.g. to resume */
} sbmds_start;

typedef enum { SBMDS_MEM_HOST = 0, SBMDS_MEM_DEVICE = 1 } sbmds_mem;

/* Option flags */
#define SBMDS_FLAG_KERNEL_TIMING 0x1u /* time every kernel launch with HIP events */
#define SBMDS_FLAG_NO_GRAPH 0x2u      /* launch iterations eagerly, no hipGraph replay */
#define SBMDS_FLAG_NO_CERTIFY 0x4u    /* skip the float64 certification pass */
/* W is symmetric, so the dense product can stream only its upper triangle
 * (packed once at sbmds_create; half the bytes of the full matrix).  By
 * default this is done when the batch's float32 W exceeds 256 MB; these
 * flags force it on or off (float32 / bf16 precisions; FP64 keeps the full
 * matrix). */
#define SBMDS_FLAG_PACK_W 0x8u        /* pack W whatever its size */
#define SBMDS_FLAG_FULL_W 0x10u       /* never pack W */
/* The transposed product P^T Y gathers, for each landmark row, the rows of
 * Y of its vertices.  With this flag it runs in its push form instead where
 * that applies (block widths 8, 16 and 32, and vertex blocks that touch few
 * landmarks: at least 4 entries per block-landmark pair): blocks of 256
 * vertices read their rows of Y once and write one partial row per landmark
 * they touch, and a second pass adds those per landmark in block order.  It
 * costs a second copy of P's values at sbmds_create and moves 2 B words per
 * block-landmark pair; it is slower than the gathering form on meshes whose
 * vertex order is not blocked in two dimensions. */
#define SBMDS_FLAG_PUSH_T 0x20u

/*
 * One problem (mesh).  Arrays live in host or device memory according to
 * `mem`; all of one problem's arrays must be in the same place.
 *
 *   n, l      vertices and landmarks, 2 <= l <= n < 2^31.
 *   nnz       number of stored entries of P, 0 <= nnz < 2^31.
 *   P_rowptr  [n+1] int32, P_rowptr[0] = 0, non-decreasing, P_rowptr[n] = nnz.
 *   P_col     [nnz] int32 landmark index of each entry, in [0, l), strictly
 *             increasing within a row.
 *   P_val     [nnz] entries of P: double for SBMDS_FP64, float otherwise.
 *             Rows need not sum to one (the thresholded operator does not).
 *   W         [l*l] row-major landmark block, same element type as P_val;
 *             must be symmetric with finite entries.
 *   xyz       [n*3] float vertex positions; read only for SBMDS_START_LEARNED
 *             (may be NULL otherwise).
 *   landmark_vertex [l] int32 vertex id of landmark j; read only for
 *             SBMDS_START_LEARNED (may be NULL otherwise).
 *   X0        [n*block] row-major start block, element type as P_val; read
 *             only for SBMDS_START_USER.
 */
typedef struct {
    int64_t n, l, nnz;
    const int32_t *P_rowptr;
    const int32_t *P_col;
    const void *P_val;
    const void *W;
    const float *xyz;
    const int32_t *landmark_vertex;
    const void *X0;
    int mem; /* sbmds_mem */
} sbmds_problem;

/*
 * Solver options.  Call sbmds_default_options first, then override.
 *   k          wanted eigenpairs / embedding dimension, 1 <= k <= block.
 *   block      subspace width, k <= block <= min(l - 1, SBMDS_MAX_BLOCK).
 *              Geodesic classical scaling has negative eigenvalues larger in
 *              magnitude than the wanted ones; the block must be wide enough
 *              to hold them as well (default 16).
 *   prec       sbmds_precision (default SBMDS_FP32).
 *   start      sbmds_start (default SBMDS_START_RANDOM).
 *   tol        target bound on the relative eigenvalue error of each of the
 *              k eigenvalues (default 1e-6).
 *   max_iter   iteration cap over all phases (default 500).
 *   seed       seed of the random start block.
 *   stream     hipStream_t to run on (NULL = the null stream).
 *   mlp_weights  path of a weights file for SBMDS_START_LEARNED (or NULL).
 *   tune_cache   path of the autotuner's text cache.  When set, sbmds_create
 *                times the launch choices on the device for every arithmetic
 *                of the schedule (unless the file already holds them for this
 *                batch shape) and stores them there; NULL = default choices,
 *                no timing.
 *   mem_cap    upper bound on device bytes the context may allocate (0 = none).
 *   flags      SBMDS_FLAG_* bits.
 */
typedef struct {
    int k;
    int block;
    int prec;
    int start;
    double tol;
    int max_iter;
    uint64_t seed;
    void *stream;
    const char *mlp_weights;
    const char *tune_cache;
    size_t mem_cap;
    unsigned flags;
} sbmds_options;

/*
 * Per-problem report filled by sbmds_embed.
 *   status      per-problem sbmds_status.
 *   iters_*     iterations run in each arithmetic (bf16 bulk, fp32,
 *               fp64-accumulated certification / fp64 mode).
 *   eig[i]      Ritz value i (i < k), descending.
 *   err_bound[i] bound on |eig[i] - lambda_i| / |eig[i]| from the final
 *               residuals (quadratic residual bound over gap-separated
 *               clusters, or the plain residual norm when smaller).
 *   resid[i]    ||B x_i - eig[i] x_i|| / |eig[i]|.
 *   nonpositive number of the k eigenvalues <= 0 (their coordinates are 0).
 *   jacobi_sweeps total Jacobi sweeps spent in the Rayleigh-Ritz steps.
 *   start_iters iterations spent building the start block (the landmark
 *               problem's iterations for SBMDS_START_LMDS, else 0).
 *   ms_*        wall time of the start block, of the iterations, and of the
 *               whole call, measured with HIP events on the context's stream.
 */
typedef struct {
    int status;
    int iters_bf16, iters_fp32, iters_fp64;
    int nonpositive;
    int certified;
    int jacobi_sweeps;
    int start_iters;
    double ms_start, ms_iter, ms_total;
    double eig[SBMDS_MAX_BLOCK];
    double err_bound[SBMDS_MAX_BLOCK];
    double resid[SBMDS_MAX_BLOCK];
} sbmds_report;

/* Per-kernel timing (SBMDS_FLAG_KERNEL_TIMING): launches, summed event time
 * and the algorithmic bytes and flops per launch summed over launches. */
typedef struct {
    char name[48];
    int64_t launches;
    double ms_total;
    double bytes_total;
    double flops_total;
} sbmds_kernel_stat;

/* Fill `opt` with the defaults listed above.  NULL is ignored. */
void sbmds_default_options(sbmds_options *opt);

/*
 * Validate and upload `nprob` problems, build the transposed operator and
 * the per-precision copies, and allocate every buffer the solve needs.
 * Validation of host-resident inputs happens before any device call, so
 * malformed input returns SBMDS_EINVAL even on a machine without a GPU.
 * On success *out owns the new context; on error *out is set to NULL.
 */
int sbmds_create(const sbmds_problem *probs, int nprob, const sbmds_options *opt, sbmds_ctx **out);

/*
 * Run the eigensolve for every problem of the context.
 *   eigvals  [nprob*k] host doubles (may be NULL): the k eigenvalues of each
 *            problem, descending.
 *   Z        [sum_p n_p * k] row-major embedding (may be NULL), problems
 *            concatenated in order; double for SBMDS_FP64, float otherwise.
 *   Z_mem    sbmds_mem of Z.
 *   reports  [nprob] (may be NULL).
 * Returns the worst per-problem status.  May be called repeatedly; each
 * call starts again from the start block chosen in the options.  A block
 * that loses rank during the solve (its CholQR drops a column, e.g. a start
 * block with a zero or repeated column) has the dropped columns replaced by
 * fresh Gaussian ones before the next round of iterations.
 */
int sbmds_embed(sbmds_ctx *ctx, double *eigvals, void *Z, int Z_mem, sbmds_report *reports);

/*
 * The interpolation operator P of Eq. (PDefinition) built on the device from
 * a triangle mesh (Sections 2.2 and 3.1): cotangent weights and lumped mass
 * (or, with SBMDS_INTERP_GRAPH, the generic-graph variant D = I, A = 0/1
 * edge adjacency), M = L^T D^-1 L with L = diag(A 1) - A, P_u = -M_uu^-1 M_ub
 * by a Cholesky factorisation of M_uu (Section 3.2 names a sparse Cholesky
 * decomposition), then per column the p entries of largest magnitude (ties
 * at the cut to the lower vertex id, exact zeros dropped; p <= 0 keeps
 * every nonzero), and the identity rows of the landmarks.  Two routes:
 *   dense    M_uu as a dense matrix: 8 n^2 bytes, O(n^3); n <= 46340.
 *   blocked  the mesh's breadth-first levels order the non-landmarks so
 *            that M_uu is block tridiagonal with blocks of two levels; its
 *            factor keeps that shape and is applied to batches of the
 *            right-hand sides.  About 16 n w bytes and O(n w (w + l))
 *            flops for blocks of w vertices; n < 2^30.
 *   V          [n*3] double vertex positions.
 *   F          [nf*3] int32 triangles (distinct vertices in [0, n)).
 *   landmarks  [l] int32 distinct vertex ids, 1 <= l < n; column j of P
 *              belongs to landmarks[j].
 *   flags      SBMDS_INTERP_* bits: GRAPH for the generic-graph variant;
 *              DENSE or BLOCKED picks the route (neither: dense up to 4096
 *              vertices, blocked above).  Both routes compute the same
 *              sums for M; their solutions differ by rounding.
 *   rowptr, col, val  output CSR of P (n x l): [n+1] int32, [cap] int32,
 *              [cap] double, columns ascending within a row.
 *   cap        capacity of col and val; *nnz receives the entry count (also
 *              when cap is too small, which returns SBMDS_EINVAL).  l + l p
 *              (l + l (n - l) without thresholding) always suffices.
 *   mem        sbmds_mem of every array; stream as for the other calls (the
 *              call synchronises it).
 * Invalid meshes, landmarks or flags return SBMDS_EINVAL before any use of
 * them as an index; a matrix M_uu that is not positive definite (a
 * component of the mesh without a landmark) SBMDS_EBREAKDOWN; a route that
 * does not fit the free device memory SBMDS_ENOMEM.
 */
#define SBMDS_INTERP_GRAPH 0x1   /* generic-graph variant: D = I, A = edge adjacency */
#define SBMDS_INTERP_DENSE 0x2   /* dense route */
#define SBMDS_INTERP_BLOCKED 0x4 /* level-blocked route */
int sbmds_interpolation(const double *V, int64_t n, const int32_t *F, int64_t nf, const int32_t *landmarks, int64_t l,
                        int64_t p, int flags, int32_t *rowptr, int32_t *col, double *val, int64_t cap, int64_t *nnz,
                        int mem, void *stream);

/*
 * Landmarks and the landmark block W on the device (Section 3): farthest-
 * point sampling, Eq. (FarthestPoint) -- landmarks[0] = first, then each
 * further landmark is the vertex whose smallest geodesic distance to the
 * landmarks chosen so far is largest (lowest vertex id on ties) -- and
 * W = D_ll o D_ll, the squared geodesic distances between the landmarks in
 * that order, W_ij = (d_ij^2 + d_ji^2) / 2 with d_ij the distance from
 * landmark i to landmark j, zero diagonal (the input sbmds_create takes).
 * Geodesic distances are shortest paths over the weighted graph (for a mesh:
 * its edges weighted by their lengths), in float64, equal bit for bit to a
 * textbook Dijkstra's.
 *   rowptr, col, w  CSR of the graph: [n+1] int32, [nnz] int32, [nnz]
 *             double; every edge stored in both directions, weights finite
 *             and > 0, no self loops (checked on the device: SBMDS_EINVAL).
 *   l         landmarks, 1 <= l <= min(n, 65535); first in [0, n).
 *   landmarks [l] int32 output.
 *   W         [l*l] row-major double output, or NULL for the landmarks only.
 *             Entries between disconnected parts are +inf.
 *   mem       sbmds_mem of every array.
 *   batch     sources searched at once for W (1..256; 64 is a good default).
 *   stream    hipStream_t (NULL = the null stream); the call synchronises it.
 * Device memory: about 32 n bytes, plus 24 n batch + 16 l^2 bytes for W,
 * allocated and freed by the call.
 */
int sbmds_landmarks_geodesic(const int32_t *rowptr, const int32_t *col, const double *w, int64_t n, int64_t l,
                             int32_t first, int32_t *landmarks, double *W, int mem, int batch, void *stream);

/*
 * The paper's other two routes to the same eigenpairs (Section 3.3), run on
 * the operator a context holds (its top precision: float64 for SBMDS_FP64,
 * float32 otherwise; vectors and products in float64), as comparison
 * solvers beside sbmds_embed.  Both use the context's k, tol and seed and
 * write eigvals and Z exactly as sbmds_embed does (k <= 16).
 *
 * sbmds_embed_lanczos: (block) Lanczos on the implicit operator
 * B = -1/2 J P W P^T J, using only products with B (the paper's sBMDS;
 * block = 1 is the single-vector method, block 2, 4 or 8 resolves
 * eigenvalues of that multiplicity), with full reorthogonalisation.  It
 * stops when the k largest Ritz values meet the same error bound as
 * sbmds_embed's certification (tol), or after max_steps block steps
 * (SBMDS_ENOCONV, best Ritz pairs written).  The basis, n x block x
 * max_steps doubles (at most 2048 columns), is allocated per call.
 *
 * sbmds_embed_bmds: BMDS.  Q R = J P by a Householder QR of the dense
 * n x l matrix J P, the eigendecomposition of -1/2 R W R^T, and
 * Z = Q V_k Lambda_k^{1/2}.  It needs 8 n l bytes of device memory (and
 * l <= 65535); SBMDS_ENOMEM when that does not fit.  err_bound and resid
 * are the measured relative residuals ||B x - theta x|| / |theta|.
 */
typedef struct {
    int status;      /* SBMDS_OK, SBMDS_ENOCONV */
    int steps;       /* block Lanczos steps (0 for BMDS) */
    int basis;       /* columns of the Krylov basis used (0 for BMDS) */
    int nonpositive; /* of the k eigenvalues, those <= 0 (their coordinates are 0) */
    double ms_total; /* host wall time of the problem's solve */
    double eig[SBMDS_MAX_BLOCK];
    double err_bound[SBMDS_MAX_BLOCK];
    double resid[SBMDS_MAX_BLOCK];
} sbmds_solver_report;

int sbmds_embed_lanczos(sbmds_ctx *ctx, int block, int max_steps, double *eigvals, void *Z, int Z_mem,
                        sbmds_solver_report *reports);
int sbmds_embed_bmds(sbmds_ctx *ctx, double *eigvals, void *Z, int Z_mem, sbmds_solver_report *reports);

/* Copy the current basis block (the iteration's state) of problem `prob`
 * into `X` ([n*block] row-major, element type as P_val, host or device per
 * X_mem), so that a later solve can resume from it via SBMDS_START_USER. */
int sbmds_get_block(sbmds_ctx *ctx, int prob, void *X, int X_mem);

/* Copy at most `max` kernel statistics into `out`; returns the number
 * available (or a negative status).  Statistics accumulate over calls until
 * sbmds_reset_kernel_stats. */
int sbmds_kernel_stats(sbmds_ctx *ctx, sbmds_kernel_stat *out, int max);
void sbmds_reset_kernel_stats(sbmds_ctx *ctx);

/*
 * Rows of the sparse biharmonic approximation K~ = P L P^T of a symmetric
 * matrix whose landmark block is L (Section 3.1: the landmark block
 * interpolated to every vertex by P on both sides), and their relative
 * error against the exact rows (Section 4.1's eps(K~) on a row subset S):
 * sum_S ||K~_s - K_s||^2 / sum_S ||K_s||^2.  L is the landmark distances
 * for the geodesic distance approximation that section measures, or
 * W = D^2_ll for the squared distances classical scaling uses.
 *   prob     P (n x l CSR) in host or device memory (prob->mem); W, xyz,
 *            landmark_vertex and X0 are not read.  P is checked on the
 *            device like sbmds_create's device inputs.
 *   fp64     element type of P_val, L and K_rows: double if non-zero, else
 *            float.
 *   L        [l*l] row-major, symmetric, finite; same memory as P.
 *   rows     [nrows] vertex ids in [0, n), same memory as P; 1 <= nrows <= 4096.
 *   K_rows   [nrows*n] row-major exact rows (NULL if err is NULL), same
 *            memory as P.
 *   err      [2] host doubles (may be NULL): sum_S ||K~_s - K_s||^2 and
 *            sum_S ||K_s||^2, accumulated in float64 in a fixed order.
 *   out      [nrows*n] row-major doubles (may be NULL): the rows of K~,
 *            host or device memory per out_mem.
 *   stream   hipStream_t (NULL = the null stream); the call synchronises it.
 * The products run on the device in float64 from the given values; the
 * call allocates (and frees) its own device scratch, S x l doubles.
 */
int sbmds_approx_rows(const sbmds_problem *prob, int fp64, const void *L, const int32_t *rows, int64_t nrows,
                      const void *K_rows, double *err, double *out, int out_mem, void *stream);

/*
 * Stress of an embedding, the objective of Eq. (MDS_problem) (Section 2.3;
 * Section 4.2 compares solutions by it): ||Z Z^T + 1/2 J E J||_F with
 * E = K o K the squared distances and J the centering matrix.
 *   Z       [n*m] row-major embedding (1 <= m <= 16), e.g. sbmds_embed's Z.
 *   K       [n*n] row-major exact distances, symmetric (only its column
 *           sums are formed; they stand for the row sums too); same element
 *           type and memory as Z.
 *   fp64    element type of Z and K: double if non-zero, else float.
 *   mem     sbmds_mem of Z and K (host arrays are uploaded first).
 *   out     [2] host doubles: the stress and ||1/2 J E J||_F (the stress of
 *           Z = 0, its natural scale).
 *   stream  hipStream_t (NULL = the null stream); the call synchronises it.
 * K is read once, in float64 arithmetic with fixed-order sums (bitwise
 * reproducible); the call allocates (and frees) its device scratch, 24 n
 * bytes per split of the rows (at most about 2048 / ceil(n / 256) splits),
 * plus copies of host inputs.  Non-finite inputs give non-finite output.
 */
int sbmds_stress(const void *Z, int64_t n, int m, const void *K, int fp64, int mem, double *out, void *stream);

/* Release the context and all device memory it owns.  NULL is a no-op. */
void sbmds_destroy(sbmds_ctx *ctx);

/* Message of the last error on this thread ("" if none). */
const char *sbmds_last_error(void);

/* (major << 16) | minor */
int sbmds_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SBMDS_H */
