// Internal declarations of the learned warm start (network kernels and the
// handle shared by the C ABI and the solver runtime).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace sbmds {
namespace mlp {

constexpr int kIn = 19;     // features per landmark
constexpr int kHid = 128;   // width of both hidden layers
constexpr int kHist = 10;   // histogram bins among the features
constexpr int kMaxOut = 8;  // largest output width (k) the kernels carry
constexpr double kRidge = 1e-4;  // alignment ridge per row of a mesh

hipError_t launch_features(const void *W, int w_double, int64_t l, int64_t ldw, const float *xyz,
                           const int32_t *lmv, float *feat, double *rowmax, hipStream_t s);
hipError_t launch_standardise(const float *F, int64_t rows, const float *mean, const float *inv_std, float *X,
                              hipStream_t s);
hipError_t launch_gemm(int epi, const float *A, int64_t M, int K, int64_t sam, int64_t sak, const float *B, int N,
                       int64_t sbk, int64_t sbn, const float *bias, float *C, float *Zout, const float *Zin,
                       hipStream_t s);
int wgrad_chunks(int64_t M);
hipError_t launch_wgrad(const float *A, int64_t M, int K, const float *D, int N, float *part, float *gW, float *gb,
                        hipStream_t s);
hipError_t launch_loss(int k, const float *Y, const float *T, const int64_t *seg, int nseg, int64_t rows,
                       double ridge, double *stats, double *A, double *loss_seg, double *gscale, float *dY,
                       double *loss_out, hipStream_t s);
hipError_t launch_adam(float *theta, const float *g, float *m, float *v, int64_t count, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t s);

}  // namespace mlp
}  // namespace sbmds

// Defined in sbmds_mlp_api.cpp; used by the solver runtime for the learned
// start (forward pass on device-resident features).
struct sbmds_mlp;
namespace sbmds {
namespace mlp {
int forward_device(sbmds_mlp *net, const float *feat, int64_t rows, float *Y);
// Grow the handle's work buffers to `rows` now, so that later forward passes
// of at most that many rows allocate nothing.
int reserve_rows(sbmds_mlp *net, int64_t rows);
int out_width(const sbmds_mlp *net);
}  // namespace mlp
// Error reporting of the C ABI (defined with sbmds_last_error).
int api_fail(int code, const std::string &msg);
void api_clear_error();
}  // namespace sbmds
