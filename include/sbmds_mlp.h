/*
 * sbmds_mlp.h -- C ABI of the learned warm start of the sBMDS embedding
 * path on AMD Instinct MI355X (gfx950).
 *
 * The paper has no learned component.  This network only seeds the block
 * subspace iteration that computes the classical scaling of Section 3.3
 * (see sbmds.h): from 19 features per landmark it predicts an l x k block
 * whose span approximates the landmark rows of the top-k eigenvectors; the
 * solver lifts it through P (the interpolation operator of Section 3.1,
 * whose landmark rows are identity rows) and iterates from there, so a poor
 * prediction costs iterations, never accuracy.
 *
 * Features of landmark j (float32):
 *   0..2   landmark position minus the centroid of all landmark positions,
 *          over their root-mean-square distance to it
 *   3..6   mean of u, u^2, u^3, u^4 over landmarks i != j, where
 *          u_i = sqrt(W_ji) / max_i sqrt(W_ji) (W: squared distances)
 *   7      standard deviation of u
 *   8..17  fraction of u in each of 10 equal bins of [0, 1] (u = 1: last)
 *   18     max_i sqrt(W_ji) over its maximum over all landmarks
 * Network: y = W3^T g(W2^T g(W1^T x + b1) + b2) + b3 with g the GELU
 * z Phi(z), x the features standardised by a stored mean and deviation,
 * 19 -> 128 -> 128 -> k, float32.  Flat parameter order: W1 [19][128],
 * b1 [128], W2 [128][128], b2 [128], W3 [128][k], b3 [k].
 * Loss (training): mean over meshes m of
 *   min_A ( ||Y_m A - T_m||_F^2 + 1e-4 rows_m ||A||_F^2 ) / ||T_m||_F^2
 * with T_m the landmark rows of a converged embedding of mesh m.
 *
 * Conventions as in sbmds.h: negative returns are errors with a message in
 * sbmds_last_error(); the caller owns its arrays; a network handle owns its
 * device memory until sbmds_mlp_destroy and runs on the stream it was
 * created with; it is not thread-safe.
 */
#ifndef SBMDS_MLP_H
#define SBMDS_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBMDS_MLP_FEATURES 19
#define SBMDS_MLP_HIDDEN 128
#define SBMDS_MLP_MAX_OUT 8 /* largest k the network supports */

typedef struct sbmds_mlp sbmds_mlp; /* opaque */

/* New network with k outputs (1 <= k <= 8): He-initialised weights drawn from
 * a seeded generator, zero biases, identity standardisation, fresh Adam
 * state.  stream: hipStream_t (NULL = null stream). */
int sbmds_mlp_create(int k, uint64_t seed, void *stream, sbmds_mlp **out);

/* Load / save a weights file: the standardisation and the parameters
 * (little-endian: 8-byte magic "SBMDSMLP", int32 version 1, int32 inputs,
 * int32 hidden, int32 k, float32 mean[19], float32 std[19], float32
 * params[]).  Adam state is not stored. */
int sbmds_mlp_load(const char *path, void *stream, sbmds_mlp **out);
int sbmds_mlp_save(const sbmds_mlp *net, const char *path);

/* Number of parameters, and host copies of them ([count] floats). */
int64_t sbmds_mlp_num_params(const sbmds_mlp *net);
int sbmds_mlp_get_params(const sbmds_mlp *net, float *theta);
int sbmds_mlp_set_params(sbmds_mlp *net, const float *theta);

/* Standardisation applied to the features: x = (f - mean) / std (host
 * arrays of 19 floats, std > 0). */
int sbmds_mlp_set_norm(sbmds_mlp *net, const float *mean, const float *std);

/* Features of one mesh: xyz [n*3] vertex positions, landmark_vertex [l]
 * vertex of each landmark (in [0, n)), W [l*l] row-major squared landmark
 * distances (double if w_double, else float), feat [l*19] output.  All
 * arrays in host (mem 0) or device (mem 1) memory. */
int sbmds_mlp_features(const float *xyz, int64_t n, const int32_t *landmark_vertex, const void *W, int64_t l,
                       int w_double, float *feat, int mem, void *stream);

/* Forward pass on `rows` feature rows (rows <= 4,000,000): Y [rows*k]. */
int sbmds_mlp_forward(sbmds_mlp *net, const float *feat, int64_t rows, float *Y, int mem);

/* The forward pass of sbmds_mlp_forward for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): feat [rows*19] and Y [rows*k] are
 * device arrays; 1 <= rows <= 4,000,000, larger counts return SBMDS_EINVAL.
 * Nothing is allocated: the hidden layers go through a fixed work buffer of
 * 8,192 rows (about 9 MB of device memory per GPU, held until the process
 * ends), chunk after chunk, with the same kernels as sbmds_mlp_forward, so
 * Y matches its output bit for bit.  Asynchronous on the network's stream
 * (no synchronisation); call it with the network's device current.  Calls
 * that overlap on one GPU share that buffer and race: serialise them. */
int sbmds_mlp_forward_noalloc(sbmds_mlp *net, const float *feat, int64_t rows, float *Y);

/* Loss and gradient over meshes whose rows are seg[m] .. seg[m+1]-1 of feat
 * [rows*19] and of the targets T [rows*k] (seg: nseg+1 int64 offsets,
 * seg[0] = 0, non-decreasing, each mesh at least one row).  The gradient
 * stays in the handle for sbmds_mlp_adam_step; `loss` (host double) and
 * `grad` (host [num_params] floats) receive copies when non-NULL. */
int sbmds_mlp_loss_grad(sbmds_mlp *net, const float *feat, const float *T, const int64_t *seg, int nseg,
                        double *loss, float *grad, int mem);

/* One Adam update (beta 0.9 / 0.999, eps 1e-8, bias-corrected) with the
 * gradient of the last sbmds_mlp_loss_grad call. */
int sbmds_mlp_adam_step(sbmds_mlp *net, float lr);

void sbmds_mlp_destroy(sbmds_mlp *net);

#ifdef __cplusplus
}
#endif

#endif /* SBMDS_MLP_H */
