// Kernels of the learned warm start: landmark features, the 19-128-128-k
// GELU network (forward and backward), the span-aligned loss and Adam.
//
// The network predicts, from per-landmark features, an l x k block whose
// span approximates the landmark rows of the top-k eigenvectors of the
// classical scaling matrix of Section 3.3; lifted through P it seeds the
// block subspace iteration.  All arithmetic is float32 except the loss
// statistics and the k x k alignment solve, which are float64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sbmds_mlp_internal.h"

namespace sbmds {
namespace mlp {

namespace {

__device__ __forceinline__ double block_reduce_sum(double v, double *lds) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += lds[i];
    return s;
}

__device__ __forceinline__ double block_reduce_max(double v, double *lds) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = lds[0];
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 1; i < nw; ++i) s = fmax(s, lds[i]);
    return s;
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

}  // namespace

// ---------------------------------------------------------------------------
// Features.  One block per landmark row j of W (squared distances):
// u_i = sqrt(W_ji) / max_i sqrt(W_ji) over i != j; moments of u, its
// standard deviation and a 10-bin histogram.  Distances, u and the bin
// decisions are float64.  The row maximum is kept for the last feature.
// ---------------------------------------------------------------------------
template <typename TW>
__global__ __launch_bounds__(256) void k_feat_rows(const TW *__restrict__ W, int64_t l, int64_t ldw,
                                                   float *__restrict__ feat, double *__restrict__ rowmax) {
    __shared__ double lds[8];
    const int64_t j = blockIdx.x;
    const TW *row = W + j * ldw;
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < l; i += blockDim.x)
        if (i != j) mx = fmax(mx, (double)row[i]);
    mx = block_reduce_max(mx, lds);
    const double m = sqrt(mx);
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
    int h[kHist];
#pragma unroll
    for (int q = 0; q < kHist; ++q) h[q] = 0;
    for (int64_t i = threadIdx.x; i < l; i += blockDim.x) {
        if (i == j) continue;
        const double d = sqrt(fmax((double)row[i], 0.0));
        const double u = m > 0.0 ? d / m : 0.0;
        const double u2 = u * u;
        s1 += u;
        s2 += u2;
        s3 += u2 * u;
        s4 += u2 * u2;
        const int bin = min((int)floor(u * kHist), kHist - 1);
#pragma unroll
        for (int q = 0; q < kHist; ++q) h[q] += (bin == q) ? 1 : 0;
    }
    const double cnt = (double)(l > 1 ? l - 1 : 1);
    s1 = block_reduce_sum(s1, lds) / cnt;
    s2 = block_reduce_sum(s2, lds) / cnt;
    s3 = block_reduce_sum(s3, lds) / cnt;
    s4 = block_reduce_sum(s4, lds) / cnt;
    double hf[kHist];
#pragma unroll
    for (int q = 0; q < kHist; ++q) hf[q] = block_reduce_sum((double)h[q], lds) / cnt;
    if (threadIdx.x == 0) {
        float *f = feat + j * kIn;
        f[3] = (float)s1;
        f[4] = (float)s2;
        f[5] = (float)s3;
        f[6] = (float)s4;
        f[7] = (float)sqrt(fmax(s2 - s1 * s1, 0.0));
#pragma unroll
        for (int q = 0; q < kHist; ++q) f[8 + q] = (float)hf[q];
        rowmax[j] = m;
    }
}

// Positions of the landmarks relative to their centroid and RMS radius, and
// the row maxima relative to the largest (one block).
__global__ __launch_bounds__(256) void k_feat_finish(const float *__restrict__ xyz, const int32_t *__restrict__ lmv,
                                                     int64_t l, float *__restrict__ feat,
                                                     const double *__restrict__ rowmax) {
    __shared__ double lds[8];
    double c[3] = {0.0, 0.0, 0.0}, mx = 0.0;
    for (int64_t j = threadIdx.x; j < l; j += blockDim.x) {
        const int64_t v = lmv[j];
#pragma unroll
        for (int a = 0; a < 3; ++a) c[a] += (double)xyz[v * 3 + a];
        mx = fmax(mx, rowmax[j]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = block_reduce_sum(c[a], lds) / (double)l;
    mx = block_reduce_max(mx, lds);
    double r2 = 0.0;
    for (int64_t j = threadIdx.x; j < l; j += blockDim.x) {
        const int64_t v = lmv[j];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double d = (double)xyz[v * 3 + a] - c[a];
            r2 += d * d;
        }
    }
    const double r = sqrt(block_reduce_sum(r2, lds) / (double)l);
    const double inv_r = r > 0.0 ? 1.0 / r : 1.0;
    for (int64_t j = threadIdx.x; j < l; j += blockDim.x) {
        const int64_t v = lmv[j];
        float *f = feat + j * kIn;
#pragma unroll
        for (int a = 0; a < 3; ++a) f[a] = (float)(((double)xyz[v * 3 + a] - c[a]) * inv_r);
        f[18] = mx > 0.0 ? (float)(rowmax[j] / mx) : 0.0f;
    }
}

__global__ __launch_bounds__(256) void k_standardise(const float *__restrict__ F, int64_t count,
                                                     const float *__restrict__ mean,
                                                     const float *__restrict__ inv_std, float *__restrict__ X) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const int c = (int)(i % kIn);
        X[i] = (F[i] - mean[c]) * inv_std[c];
    }
}

// ---------------------------------------------------------------------------
// C = A B with a fused epilogue; A(m, q) = A[m sam + q sak], B(q, n) =
// B[q sbk + n sbn] (so transposed operands need no copy), C row-major M x N.
// 64 x 64 output tile per 256-thread block, 4 x 4 per thread, K staged
// through LDS in steps of 16.
// ---------------------------------------------------------------------------
enum Epi { EPI_BIAS = 0, EPI_BIAS_GELU = 1, EPI_GELU_BWD = 2 };

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(const float *__restrict__ A, int64_t M, int K, int64_t sam,
                                              int64_t sak, const float *__restrict__ Bm, int N, int64_t sbk,
                                              int64_t sbn, const float *__restrict__ bias, float *__restrict__ C,
                                              float *__restrict__ Zout, const float *__restrict__ Zin) {
    constexpr int BM = 64, BN = 64, BK = 16;
    __shared__ float As[BK][BM + 1];
    __shared__ float Bs[BK][BN + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * BM;
    const int n0 = blockIdx.x * BN;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jx = 0; jx < 4; ++jx) acc[i][jx] = 0.0f;
    for (int k0 = 0; k0 < K; k0 += BK) {
        for (int e = threadIdx.x; e < BK * BM; e += 256) {
            const int kk = e / BM, mm = e % BM;
            const int64_t m = m0 + mm;
            const int q = k0 + kk;
            As[kk][mm] = (m < M && q < K) ? A[m * sam + (int64_t)q * sak] : 0.0f;
        }
        for (int e = threadIdx.x; e < BK * BN; e += 256) {
            const int kk = e / BN, nn = e % BN;
            const int n = n0 + nn;
            const int q = k0 + kk;
            Bs[kk][nn] = (n < N && q < K) ? Bm[(int64_t)q * sbk + (int64_t)n * sbn] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int jx = 0; jx < 4; ++jx) b[jx] = Bs[kk][tx * 4 + jx];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jx = 0; jx < 4; ++jx) acc[i][jx] += a[i] * b[jx];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t m = m0 + ty * 4 + i;
        if (m >= M) continue;
#pragma unroll
        for (int jx = 0; jx < 4; ++jx) {
            const int n = n0 + tx * 4 + jx;
            if (n >= N) continue;
            const int64_t o = m * N + n;
            if (EPI == EPI_BIAS) {
                C[o] = acc[i][jx] + bias[n];
            } else if (EPI == EPI_BIAS_GELU) {
                const float z = acc[i][jx] + bias[n];
                if (Zout) Zout[o] = z;  // pre-activations are kept for the backward pass only
                C[o] = gelu(z);
            } else {
                C[o] = acc[i][jx] * gelu_grad(Zin[o]);
            }
        }
    }
}

// Weight gradient partials: G[q][n] = sum_m A[m][q] D[m][n] over the row
// chunk of this block, with an extra row q = K holding sum_m D[m][n] (the
// bias gradient).  part[chunk][(K + 1) N]; reduced by k_sum_chunks in a
// fixed order, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_wgrad(const float *__restrict__ A, int64_t M, int K,
                                               const float *__restrict__ D, int N, int64_t rows_per_chunk,
                                               float *__restrict__ part) {
    constexpr int TQ = 64, TN = 64, RB = 32;
    __shared__ float As[RB][TQ + 1];
    __shared__ float Ds[RB][TN + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int n0 = blockIdx.x * TN;
    const int q0 = blockIdx.y * TQ;
    const int64_t r0 = (int64_t)blockIdx.z * rows_per_chunk;
    const int64_t r1 = min(M, r0 + rows_per_chunk);
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jx = 0; jx < 4; ++jx) acc[i][jx] = 0.0f;
    for (int64_t rb = r0; rb < r1; rb += RB) {
        for (int e = threadIdx.x; e < RB * TQ; e += 256) {
            const int rr = e / TQ, qq = e % TQ;
            const int64_t r = rb + rr;
            const int q = q0 + qq;
            float v = 0.0f;
            if (r < r1) v = (q < K) ? A[r * K + q] : (q == K ? 1.0f : 0.0f);
            As[rr][qq] = v;
        }
        for (int e = threadIdx.x; e < RB * TN; e += 256) {
            const int rr = e / TN, nn = e % TN;
            const int64_t r = rb + rr;
            const int n = n0 + nn;
            Ds[rr][nn] = (r < r1 && n < N) ? D[r * N + n] : 0.0f;
        }
        __syncthreads();
#pragma unroll 8
        for (int rr = 0; rr < RB; ++rr) {
            float a[4], d[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[rr][ty * 4 + i];
#pragma unroll
            for (int jx = 0; jx < 4; ++jx) d[jx] = Ds[rr][tx * 4 + jx];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jx = 0; jx < 4; ++jx) acc[i][jx] += a[i] * d[jx];
        }
        __syncthreads();
    }
    float *out = part + (size_t)blockIdx.z * (size_t)(K + 1) * N;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = q0 + ty * 4 + i;
        if (q > K) continue;
#pragma unroll
        for (int jx = 0; jx < 4; ++jx) {
            const int n = n0 + tx * 4 + jx;
            if (n < N) out[(size_t)q * N + n] = acc[i][jx];
        }
    }
}

// Sum the chunk partials (in chunk order) into the flat gradient: rows
// 0..K-1 to the weight matrix, row K to the bias.
__global__ __launch_bounds__(256) void k_sum_chunks(const float *__restrict__ part, int nchunk, int K, int N,
                                                    float *__restrict__ gW, float *__restrict__ gb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = (K + 1) * N;
    if (i >= total) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * total + i];
    if (i < K * N) gW[i] = s;
    else gb[i - K * N] = s;
}

// ---------------------------------------------------------------------------
// Loss.  Per mesh (segment of rows): Y^T Y, Y^T T and ||T||^2 in float64.
// ---------------------------------------------------------------------------
template <int KO>
__global__ __launch_bounds__(256) void k_seg_stats(const float *__restrict__ Y, const float *__restrict__ T,
                                                   const int64_t *__restrict__ seg, double *__restrict__ stats) {
    constexpr int NS = 2 * KO * KO + 1;
    __shared__ double lds[8];
    const int s = blockIdx.x;
    const int64_t a = seg[s], b = seg[s + 1];
    double acc[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) acc[i] = 0.0;
    for (int64_t r = a + threadIdx.x; r < b; r += blockDim.x) {
        double y[KO], t[KO];
#pragma unroll
        for (int c = 0; c < KO; ++c) {
            y[c] = (double)Y[r * KO + c];
            t[c] = (double)T[r * KO + c];
        }
#pragma unroll
        for (int p = 0; p < KO; ++p)
#pragma unroll
            for (int q = 0; q < KO; ++q) {
                acc[p * KO + q] += y[p] * y[q];
                acc[KO * KO + p * KO + q] += y[p] * t[q];
            }
#pragma unroll
        for (int c = 0; c < KO; ++c) acc[NS - 1] += t[c] * t[c];
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const double v = block_reduce_sum(acc[i], lds);
        if (threadIdx.x == 0) stats[(size_t)s * NS + i] = v;
    }
}

// One thread per mesh: A = (Y^T Y + delta I)^{-1} Y^T T by Cholesky, the
// mesh loss (||Y A - T||^2 + delta ||A||^2) / ||T||^2 from the statistics,
// and the scale of the gradient rows.
template <int KO>
__global__ void k_seg_solve(const double *__restrict__ stats, const int64_t *__restrict__ seg, int nseg,
                            double ridge, double *__restrict__ Aout, double *__restrict__ loss_seg,
                            double *__restrict__ gscale) {
    constexpr int NS = 2 * KO * KO + 1;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const double *S = stats + (size_t)s * NS;
    const double delta = ridge * (double)(seg[s + 1] - seg[s]);
    double L[KO][KO], A[KO][KO];
    for (int i = 0; i < KO; ++i)
        for (int j = 0; j < KO; ++j) L[i][j] = S[i * KO + j] + (i == j ? delta : 0.0);
    // Cholesky in place (lower)
    for (int j = 0; j < KO; ++j) {
        double d = L[j][j];
        for (int t = 0; t < j; ++t) d -= L[j][t] * L[j][t];
        d = sqrt(fmax(d, 1e-300));
        L[j][j] = d;
        for (int i = j + 1; i < KO; ++i) {
            double v = L[i][j];
            for (int t = 0; t < j; ++t) v -= L[i][t] * L[j][t];
            L[i][j] = v / d;
        }
    }
    for (int c = 0; c < KO; ++c) {
        double z[KO];
        for (int i = 0; i < KO; ++i) {
            double v = S[KO * KO + i * KO + c];
            for (int t = 0; t < i; ++t) v -= L[i][t] * z[t];
            z[i] = v / L[i][i];
        }
        for (int i = KO - 1; i >= 0; --i) {
            double v = z[i];
            for (int t = i + 1; t < KO; ++t) v -= L[t][i] * A[t][c];
            A[i][c] = v / L[i][i];
        }
    }
    // ||Y A - T||^2 = tr(A^T YtY A) - 2 tr(A^T YtT) + ||T||^2
    double q = 0.0, lin = 0.0, aa = 0.0;
    for (int c = 0; c < KO; ++c)
        for (int i = 0; i < KO; ++i) {
            double m = 0.0;
            for (int j = 0; j < KO; ++j) m += S[i * KO + j] * A[j][c];
            q += A[i][c] * m;
            lin += A[i][c] * S[KO * KO + i * KO + c];
            aa += A[i][c] * A[i][c];
        }
    const double tt = S[NS - 1];
    const double inv_tt = tt > 0.0 ? 1.0 / tt : 0.0;
    loss_seg[s] = (q - 2.0 * lin + tt + delta * aa) * inv_tt;
    gscale[s] = 2.0 * inv_tt / (double)nseg;
    for (int i = 0; i < KO; ++i)
        for (int c = 0; c < KO; ++c) Aout[(size_t)s * KO * KO + i * KO + c] = A[i][c];
}

// dY = gscale_m (Y A - T) A^T for the rows of mesh m; the mean loss lands in
// loss_out[0] (written by the first thread).
template <int KO>
__global__ __launch_bounds__(256) void k_loss_grad(const float *__restrict__ Y, const float *__restrict__ T,
                                                   const int64_t *__restrict__ seg, int nseg,
                                                   const double *__restrict__ Am, const double *__restrict__ gscale,
                                                   const double *__restrict__ loss_seg, float *__restrict__ dY,
                                                   double *__restrict__ loss_out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) {
        double s = 0.0;
        for (int i = 0; i < nseg; ++i) s += loss_seg[i];
        loss_out[0] = s / (double)nseg;
    }
    if (r >= seg[nseg]) return;
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {  // segment m with seg[m] <= r < seg[m + 1]
        const int mid = (lo + hi + 1) >> 1;
        if (seg[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    const double *A = Am + (size_t)lo * KO * KO;
    double res[KO];
#pragma unroll
    for (int c = 0; c < KO; ++c) {
        double v = -(double)T[r * KO + c];
#pragma unroll
        for (int b = 0; b < KO; ++b) v += (double)Y[r * KO + b] * A[b * KO + c];
        res[c] = v;
    }
#pragma unroll
    for (int p = 0; p < KO; ++p) {
        double g = 0.0;
#pragma unroll
        for (int c = 0; c < KO; ++c) g += res[c] * A[p * KO + c];
        dY[r * KO + p] = (float)(gscale[lo] * g);
    }
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ theta, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, int64_t count, float lr,
                                              float b1, float b2, float eps, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_features(const void *W, int w_double, int64_t l, int64_t ldw, const float *xyz,
                           const int32_t *lmv, float *feat, double *rowmax, hipStream_t s) {
    if (l < 1) return hipErrorInvalidValue;
    if (w_double)
        hipLaunchKernelGGL((k_feat_rows<double>), dim3((unsigned)l), dim3(256), 0, s, (const double *)W, l, ldw, feat,
                           rowmax);
    else
        hipLaunchKernelGGL((k_feat_rows<float>), dim3((unsigned)l), dim3(256), 0, s, (const float *)W, l, ldw, feat,
                           rowmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_feat_finish, dim3(1), dim3(256), 0, s, xyz, lmv, l, feat, (const double *)rowmax);
    return hipGetLastError();
}

hipError_t launch_standardise(const float *F, int64_t rows, const float *mean, const float *inv_std, float *X,
                              hipStream_t s) {
    const int64_t count = rows * kIn;
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_standardise, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, F, count, mean, inv_std,
                       X);
    return hipGetLastError();
}

hipError_t launch_gemm(int epi, const float *A, int64_t M, int K, int64_t sam, int64_t sak, const float *B, int N,
                       int64_t sbk, int64_t sbn, const float *bias, float *C, float *Zout, const float *Zin,
                       hipStream_t s) {
    if (M <= 0) return hipSuccess;
    const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
    switch (epi) {
        case EPI_BIAS:
            hipLaunchKernelGGL((k_gemm<EPI_BIAS>), grid, dim3(256), 0, s, A, M, K, sam, sak, B, N, sbk, sbn, bias, C,
                               Zout, Zin);
            break;
        case EPI_BIAS_GELU:
            hipLaunchKernelGGL((k_gemm<EPI_BIAS_GELU>), grid, dim3(256), 0, s, A, M, K, sam, sak, B, N, sbk, sbn,
                               bias, C, Zout, Zin);
            break;
        case EPI_GELU_BWD:
            hipLaunchKernelGGL((k_gemm<EPI_GELU_BWD>), grid, dim3(256), 0, s, A, M, K, sam, sak, B, N, sbk, sbn, bias,
                               C, Zout, Zin);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Row chunks of the weight gradient: ~64 rows each (enough blocks to fill
// the device at a few thousand rows), at most 256 partials to sum.
int wgrad_chunks(int64_t M) { return (int)std::min<int64_t>(256, std::max<int64_t>(1, (M + 63) / 64)); }

hipError_t launch_wgrad(const float *A, int64_t M, int K, const float *D, int N, float *part, float *gW, float *gb,
                        hipStream_t s) {
    const int nchunk = wgrad_chunks(M);
    const int64_t rpc = (M + nchunk - 1) / nchunk;
    const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((K + 1 + 63) / 64), (unsigned)nchunk);
    hipLaunchKernelGGL(k_wgrad, grid, dim3(256), 0, s, A, M, K, D, N, rpc, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int total = (K + 1) * N;
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const float *)part,
                       nchunk, K, N, gW, gb);
    return hipGetLastError();
}

#define SBMDS_MLP_K(KO_, CALL)                           \
    switch (KO_) {                                       \
        case 1: { constexpr int KO = 1; CALL; } break;   \
        case 2: { constexpr int KO = 2; CALL; } break;   \
        case 3: { constexpr int KO = 3; CALL; } break;   \
        case 4: { constexpr int KO = 4; CALL; } break;   \
        case 5: { constexpr int KO = 5; CALL; } break;   \
        case 6: { constexpr int KO = 6; CALL; } break;   \
        case 7: { constexpr int KO = 7; CALL; } break;   \
        case 8: { constexpr int KO = 8; CALL; } break;   \
        default: return hipErrorInvalidValue;            \
    }

hipError_t launch_loss(int k, const float *Y, const float *T, const int64_t *seg, int nseg, int64_t rows,
                       double ridge, double *stats, double *A, double *loss_seg, double *gscale, float *dY,
                       double *loss_out, hipStream_t s) {
    if (nseg < 1) return hipErrorInvalidValue;
    SBMDS_MLP_K(k, {
        hipLaunchKernelGGL((k_seg_stats<KO>), dim3((unsigned)nseg), dim3(256), 0, s, Y, T, seg, stats);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_seg_solve<KO>), dim3((unsigned)((nseg + 63) / 64)), dim3(64), 0, s,
                           (const double *)stats, seg, nseg, ridge, A, loss_seg, gscale);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int64_t nthr = std::max<int64_t>(rows, 1);
        hipLaunchKernelGGL((k_loss_grad<KO>), dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, Y, T, seg,
                           nseg, (const double *)A, (const double *)gscale, (const double *)loss_seg, dY, loss_out);
        return hipGetLastError();
    });
    return hipErrorInvalidValue;
}

hipError_t launch_adam(float *theta, const float *g, float *m, float *v, int64_t count, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, theta, g, m, v, count, lr, b1,
                       b2, eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace sbmds
