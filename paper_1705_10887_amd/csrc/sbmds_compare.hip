// Comparison eigensolvers of Section 3.3 on the device: block Lanczos on
// the implicit operator B = -1/2 J P W P^T J (width 1 is the paper's sBMDS)
// and BMDS through a dense QR of J P.  Vectors are float64; P and W are read
// in the precision the context holds them.
//
// Block Lanczos with full reorthogonalisation: the basis V (n x m, column
// blocks of width p) is extended by X = B V_j made orthogonal to the
// constant vector (that is J) and to every basis column, twice (classical
// Gram-Schmidt applied twice), then orthonormalised by Cholesky QR, twice.
// The coefficients of both passes and the Cholesky factors are the entries
// of H = V^T B V (block tridiagonal up to rounding); the Ritz pairs of H
// give the eigenvalue estimates, and ||R s_last|| (R the last Cholesky
// factor, s_last the last p entries of a Ritz vector of H) is the residual
// norm of its Ritz vector.  The same error bound as the block subspace
// iteration decides convergence: over clusters of Ritz values (relative
// distance 1e-3) min(||r||, ||R_cluster||^2 / gap) / |theta|.
//
// BMDS: A = J P formed densely (n x l, column-major), A = Q R by Householder
// QR (rocSOLVER), M = -1/2 R W R^T by two GEMMs (rocBLAS), M = V Lambda V^T
// (rocSOLVER), Z = Q V_k Lambda_k^{1/2} by applying the reflectors to
// [V_k; 0].  The residual of every returned pair is then measured with the
// operator products of the Lanczos solver.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/sbmds.h"
#include "sbmds_compare.h"
#include "sbmds_mlp_internal.h"  // api_fail

namespace sbmds {
namespace {

constexpr int kDotCols = 4;      // basis columns per block of the projection kernel
constexpr int kDotChunks = 128;  // row chunks of the projection kernel

// ---------------------------------------------------------------------------
// Gaussian start block: splitmix64 of (seed, index) gives two uniforms, the
// Box-Muller transform one normal deviate.
__device__ inline uint64_t cmp_mix(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_cmp_rand(double *X, int64_t count, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const uint64_t a = cmp_mix(seed ^ cmp_mix(2 * (uint64_t)i));
    const uint64_t b = cmp_mix(seed ^ cmp_mix(2 * (uint64_t)i + 1));
    const double u1 = (double)((a >> 11) + 1) * 0x1.0p-53;  // (0, 1]
    const double u2 = (double)(b >> 11) * 0x1.0p-53;        // [0, 1)
    X[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) v += __shfl_xor(v, sh);
    return v;
}

// ---------------------------------------------------------------------------
// Products with B.  X, Y: n x p column blocks (column q at q * n); t, u:
// column blocks of stride lda.

// t = P^T J X: one wave per landmark row of P^T, its entries strided over the
// lanes; J enters as -c_j * mean(x_q).
template <typename T, int P>
__global__ __launch_bounds__(256) void k_cmp_spmmt(const int32_t *__restrict__ rpT, const int32_t *__restrict__ ciT,
                                                   const T *__restrict__ valT, const double *__restrict__ c,
                                                   int64_t l, int lda, int64_t n, const double *__restrict__ X,
                                                   const double *__restrict__ xsum, double *__restrict__ t) {
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= l) return;  // the whole wave leaves together
    double acc[P];
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = 0.0;
    for (int32_t e = rpT[j] + lane; e < rpT[j + 1]; e += 64) {
        const double w = (double)valT[e];
        const int64_t v = ciT[e];
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q] += w * X[q * n + v];
    }
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = wave_sum(acc[q]);
    if (lane == 0) {
        const double cj = c[j];
#pragma unroll
        for (int q = 0; q < P; ++q) t[q * lda + j] = acc[q] - cj * (xsum[q] / (double)n);
    }
}

// u = W t: R rows of W per block (R * P = 8 accumulators per thread), four
// consecutive columns per thread and step; each block sum in a fixed order.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_cmp_gemm(const T *__restrict__ W, int lda, int64_t l,
                                                  const double *__restrict__ t, double *__restrict__ u) {
    constexpr int R = 8 / P;
    __shared__ double red[R * P][4];
    const int64_t i0 = (int64_t)blockIdx.x * R;
    double acc[R][P];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < P; ++q) acc[r][q] = 0.0;
    for (int64_t j = (int64_t)threadIdx.x * 4; j < l; j += 1024) {
        double tv[P][4];
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
            for (int a = 0; a < 4; ++a) tv[q][a] = (j + a < l) ? t[q * lda + j + a] : 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = i0 + r < l ? i0 + r : l - 1;  // rows past l repeat row l-1, unused
            const T *row = (const T *)__builtin_assume_aligned(W + i * lda + j, 4 * sizeof(T) >= 16 ? 16 : 8);
            T w[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) w[a] = row[a];  // j + 3 < lda: lda is a multiple of 64
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const double wa = (j + a < l) ? (double)w[a] : 0.0;
#pragma unroll
                for (int q = 0; q < P; ++q) acc[r][q] += wa * tv[q][a];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const double v = wave_sum(acc[r][q]);
            if ((threadIdx.x & 63) == 0) red[r * P + q][threadIdx.x >> 6] = v;
        }
    __syncthreads();
    if (threadIdx.x < R * P) {
        const int r = threadIdx.x / P, q = threadIdx.x % P;
        if (i0 + r < l) {
            const double *x = red[threadIdx.x];
            u[q * lda + i0 + r] = ((x[0] + x[1]) + x[2]) + x[3];
        }
    }
}

// Y = -1/2 P u (not yet centred): one thread per vertex.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_cmp_spmm(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                  const T *__restrict__ val, int64_t n, int lda,
                                                  const double *__restrict__ u, double *__restrict__ Y) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    double acc[P];
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = 0.0;
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
        const double w = (double)val[e];
        const int64_t col = ci[e];
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q] += w * u[q * lda + col];
    }
#pragma unroll
    for (int q = 0; q < P; ++q) Y[q * n + v] = -0.5 * acc[q];
}

// ---------------------------------------------------------------------------
// Projections.  Columns 0..ncols-1 are basis columns V_i; with with_const
// column ncols is the constant vector of ones.  Block (c, g) takes row
// chunk c and columns kDotCols g .. kDotCols g + 3 and writes
// part[(i p + q) kDotChunks + c] = sum over its rows of col_i[v] X_q[v].
template <int P>
__global__ __launch_bounds__(256) void k_cmp_dots(const double *__restrict__ V, int ncols, int with_const, int64_t n,
                                                  const double *__restrict__ X, double *__restrict__ part) {
    __shared__ double red[kDotCols * P][4];
    const int c = blockIdx.x;
    const int i0 = blockIdx.y * kDotCols;
    const int tot = ncols + with_const;
    const int64_t csz = (n + kDotChunks - 1) / kDotChunks;
    const int64_t rb = (int64_t)c * csz;
    const int64_t re = rb + csz < n ? rb + csz : n;
    double acc[kDotCols][P];
#pragma unroll
    for (int a = 0; a < kDotCols; ++a)
#pragma unroll
        for (int q = 0; q < P; ++q) acc[a][q] = 0.0;
    for (int64_t v = rb + threadIdx.x; v < re; v += 256) {
        double xv[P];
#pragma unroll
        for (int q = 0; q < P; ++q) xv[q] = X[q * n + v];
#pragma unroll
        for (int a = 0; a < kDotCols; ++a) {
            const int i = i0 + a;
            const double ci = i < ncols ? V[(int64_t)i * n + v] : (i < tot ? 1.0 : 0.0);
#pragma unroll
            for (int q = 0; q < P; ++q) acc[a][q] += ci * xv[q];
        }
    }
#pragma unroll
    for (int a = 0; a < kDotCols; ++a)
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const double s = wave_sum(acc[a][q]);
            if ((threadIdx.x & 63) == 0) red[a * P + q][threadIdx.x >> 6] = s;
        }
    __syncthreads();
    if (threadIdx.x < kDotCols * P) {
        const int a = threadIdx.x / P, q = threadIdx.x % P;
        const int i = i0 + a;
        if (i < tot) {
            const double *x = red[threadIdx.x];
            part[((int64_t)i * P + q) * kDotChunks + c] = ((x[0] + x[1]) + x[2]) + x[3];
        }
    }
}

// h[idx] = sum of the kDotChunks partials of idx, in chunk order.
__global__ __launch_bounds__(256) void k_cmp_dots_reduce(const double *__restrict__ part, int count,
                                                         double *__restrict__ h) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= count) return;
    const double *p = part + (int64_t)idx * kDotChunks;
    double s = 0.0;
    for (int c = 0; c < kDotChunks; ++c) s += p[c];
    h[idx] = s;
}

// X_q -= sum_i h[i p + q] V_i (+ h[ncols p + q] / n times the ones).
template <int P>
__global__ __launch_bounds__(256) void k_cmp_update(const double *__restrict__ V, int ncols, int with_const,
                                                    int64_t n, const double *__restrict__ h, double *__restrict__ X) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    double x[P];
#pragma unroll
    for (int q = 0; q < P; ++q) x[q] = X[q * n + v];
    if (with_const) {
#pragma unroll
        for (int q = 0; q < P; ++q) x[q] -= h[ncols * P + q] / (double)n;
    }
    for (int i = 0; i < ncols; ++i) {
        const double vi = V[(int64_t)i * n + v];
#pragma unroll
        for (int q = 0; q < P; ++q) x[q] -= h[i * P + q] * vi;
    }
#pragma unroll
    for (int q = 0; q < P; ++q) X[q * n + v] = x[q];
}

// Y = X Rinv (Rinv p x p row-major, upper triangular); Y may alias X.
template <int P>
__global__ __launch_bounds__(256) void k_cmp_mulr(const double *X, int64_t n, const double *__restrict__ Rinv,
                                                  double *Y) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    double x[P];
#pragma unroll
    for (int q = 0; q < P; ++q) x[q] = X[q * n + v];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        double y = 0.0;
#pragma unroll
        for (int r = 0; r <= q; ++r) y += x[r] * Rinv[r * P + q];
        Y[q * n + v] = y;
    }
}

// Z[v k + q] = scale_q sum_i V_i[v] S[i k + q] (row-major output).
template <typename TZ>
__global__ __launch_bounds__(256) void k_cmp_ritz(const double *__restrict__ V, int m, int64_t n,
                                                  const double *__restrict__ S, int k,
                                                  const double *__restrict__ scale, TZ *__restrict__ Z) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    double z[kCmpMaxK];
#pragma unroll
    for (int q = 0; q < kCmpMaxK; ++q) z[q] = 0.0;
    for (int i = 0; i < m; ++i) {
        const double vi = V[(int64_t)i * n + v];
#pragma unroll
        for (int q = 0; q < kCmpMaxK; ++q)
            if (q < k) z[q] += vi * S[i * k + q];
    }
#pragma unroll
    for (int q = 0; q < kCmpMaxK; ++q)
        if (q < k) Z[v * k + q] = (TZ)(z[q] * scale[q]);
}

// ---------------------------------------------------------------------------
// BMDS helpers (column-major dense arrays).
template <typename T>
__global__ __launch_bounds__(256) void k_bm_scatter(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                    const T *__restrict__ val, int64_t n, double *__restrict__ A) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) A[(int64_t)ci[e] * n + v] = (double)val[e];
}

// A = J A: column j loses its mean c_j / n.
__global__ __launch_bounds__(256) void k_bm_center(double *__restrict__ A, int64_t n, int64_t l,
                                                   const double *__restrict__ c) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (v >= n || j >= l) return;
    A[j * n + v] -= c[j] / (double)n;
}

// R (l x l, column-major): the upper triangle of the QR output, zero below.
__global__ __launch_bounds__(256) void k_bm_upper(const double *__restrict__ A, int64_t n, int64_t l,
                                                  double *__restrict__ R) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i >= l || j >= l) return;
    R[j * l + i] = i <= j ? A[j * n + i] : 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_bm_w64(const T *__restrict__ W, int lda, int64_t l, double *__restrict__ Wd) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i >= l || j >= l) return;
    Wd[j * l + i] = (double)W[j * lda + i];  // W symmetric: row j = column j
}

// C (n x k, column-major) = [V_k; 0] with V_k the eigenvectors of the k
// largest eigenvalues (columns l-1, l-2, ... of Mv), and the float64
// eigenvalues of those columns.
__global__ __launch_bounds__(256) void k_bm_fill(const double *__restrict__ Mv, int64_t l, int k, int64_t n,
                                                 double *__restrict__ C) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int q = blockIdx.y;
    if (i >= n || q >= k) return;
    C[(int64_t)q * n + i] = i < l ? Mv[(l - 1 - q) * l + i] : 0.0;
}

// Z[v k + q] = C[q n + v] scale_q.
template <typename TZ>
__global__ __launch_bounds__(256) void k_bm_out(const double *__restrict__ C, int64_t n, int k,
                                                const double *__restrict__ scale, TZ *__restrict__ Z) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    for (int q = 0; q < k; ++q) Z[v * k + q] = (TZ)(C[(int64_t)q * n + v] * scale[q]);
}

// ---------------------------------------------------------------------------
// Host side.

#define CCHK(expr)                                                                                          \
    do {                                                                                                    \
        hipError_t _e = (expr);                                                                             \
        if (_e != hipSuccess) return api_fail(SBMDS_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

#define RBCHK(expr)                                                                                         \
    do {                                                                                                    \
        rocblas_status _e = (expr);                                                                         \
        if (_e != rocblas_status_success)                                                                   \
            return api_fail(SBMDS_EHIP, std::string(#expr) + ": " + rocblas_status_to_string(_e));          \
    } while (0)

struct DevMem {
    void *p = nullptr;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
};

unsigned blocks_of(int64_t count) { return (unsigned)((count + 255) / 256); }

struct Handle {
    rocblas_handle h = nullptr;
    ~Handle() {
        if (h) (void)rocblas_destroy_handle(h);
    }
};

// Eigenpairs of the m x m symmetric row-major A on the device (rocSOLVER):
// eigenvalues w descending, eigenvectors as the columns of Vr (row-major).
int dense_eig(rocblas_handle hd, const std::vector<double> &A, int m, double *Ad, double *Dd, double *Ed, int *info,
              hipStream_t s, std::vector<double> &w, std::vector<double> &Vr) {
    CCHK(hipMemcpyAsync(Ad, A.data(), (size_t)m * m * 8, hipMemcpyHostToDevice, s));
    RBCHK(rocsolver_dsyevd(hd, rocblas_evect_original, rocblas_fill_upper, m, Ad, m, Dd, Ed, info));
    std::vector<double> col((size_t)m * m), d(m);
    int hinfo = 0;
    CCHK(hipMemcpyAsync(col.data(), Ad, (size_t)m * m * 8, hipMemcpyDeviceToHost, s));
    CCHK(hipMemcpyAsync(d.data(), Dd, (size_t)m * 8, hipMemcpyDeviceToHost, s));
    CCHK(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
    CCHK(hipStreamSynchronize(s));
    if (hinfo != 0) return api_fail(SBMDS_EBREAKDOWN, "the projected eigenproblem did not converge");
    // A is symmetric, so the row-major copy reads as column-major: column c of
    // the result (ascending) is eigenvector c
    w.resize(m);
    Vr.resize((size_t)m * m);
    for (int c = 0; c < m; ++c) {
        const int src = m - 1 - c;
        w[c] = d[src];
        for (int r = 0; r < m; ++r) Vr[(size_t)r * m + c] = col[(size_t)src * m + r];
    }
    return SBMDS_OK;
}

// Cholesky factor (upper, row-major p x p) of the Gram G and the inverse of
// that factor.  False when G is not numerically positive definite.
bool chol_upper(const std::vector<double> &G, int p, std::vector<double> &R, std::vector<double> &Rinv) {
    R.assign((size_t)p * p, 0.0);
    double gmax = 0.0;
    for (int i = 0; i < p; ++i) gmax = std::max(gmax, G[(size_t)i * p + i]);
    for (int i = 0; i < p; ++i) {
        double d = G[(size_t)i * p + i];
        for (int r = 0; r < i; ++r) d -= R[(size_t)r * p + i] * R[(size_t)r * p + i];
        if (!(d > 1e-24 * gmax) || !(gmax > 0.0)) return false;
        const double rii = sqrt(d);
        R[(size_t)i * p + i] = rii;
        for (int j = i + 1; j < p; ++j) {
            double s = G[(size_t)i * p + j];
            for (int r = 0; r < i; ++r) s -= R[(size_t)r * p + i] * R[(size_t)r * p + j];
            R[(size_t)i * p + j] = s / rii;
        }
    }
    Rinv.assign((size_t)p * p, 0.0);  // back substitution, column by column
    for (int j = 0; j < p; ++j) {
        for (int i = j; i >= 0; --i) {
            double s = i == j ? 1.0 : 0.0;
            for (int r = i + 1; r <= j; ++r) s -= R[(size_t)i * p + r] * Rinv[(size_t)r * p + j];
            Rinv[(size_t)i * p + j] = s / R[(size_t)i * p + i];
        }
    }
    return true;
}

// Error bounds of the k wanted Ritz values among all m (descending) by the
// cluster rule; returns the largest.
double ritz_bounds(const std::vector<double> &th, const std::vector<double> &res, int m, int k, double *bound) {
    double maxb = 0.0;
    int i = 0;
    while (i < m && i < k) {
        int j = i;
        while (j + 1 < m && fabs(th[j] - th[j + 1]) <= 1e-3 * std::max(fabs(th[j]), fabs(th[j + 1]))) ++j;
        double r2 = 0.0;
        for (int q = i; q <= j; ++q) r2 += res[q] * res[q];
        double gap = INFINITY;
        if (i > 0) gap = std::min(gap, th[i - 1] - th[i]);
        if (j + 1 < m) gap = std::min(gap, th[j] - th[j + 1]);
        for (int q = i; q <= j && q < k; ++q) {
            double b = res[q];
            if (gap > 0.0 && std::isfinite(gap)) b = std::min(b, r2 / gap);
            const double a = fabs(th[q]);
            bound[q] = a > 0.0 ? b / a : INFINITY;
            maxb = std::max(maxb, bound[q]);
        }
        i = j + 1;
    }
    return maxb;
}

template <typename T>
struct Lz {
    const CmpOp &op;
    int p;
    hipStream_t s;
    double *part, *h;

    template <int P>
    hipError_t apply_p(const double *X, const double *xsum, double *t, double *u, double *Y) {
        const T *valT = (const T *)op.valT, *val = (const T *)op.val, *W = (const T *)op.W;
        hipLaunchKernelGGL((k_cmp_spmmt<T, P>), dim3((unsigned)((op.l + 3) / 4)), dim3(256), 0, s, op.rpT, op.ciT,
                           valT, op.c, op.l, op.lda, op.n, X, xsum, t);
        constexpr int R = 8 / P;
        hipLaunchKernelGGL((k_cmp_gemm<T, P>), dim3((unsigned)((op.l + R - 1) / R)), dim3(256), 0, s, W, op.lda, op.l,
                           (const double *)t, u);
        hipLaunchKernelGGL((k_cmp_spmm<T, P>), dim3(blocks_of(op.n)), dim3(256), 0, s, op.rp, op.ci, val, op.n, op.lda,
                           (const double *)u, Y);
        return hipGetLastError();
    }
    // Y = -1/2 P W P^T J X (the outer J is left to the projections)
    hipError_t apply(const double *X, const double *xsum, double *t, double *u, double *Y) {
        switch (p) {
            case 1: return apply_p<1>(X, xsum, t, u, Y);
            case 2: return apply_p<2>(X, xsum, t, u, Y);
            case 4: return apply_p<4>(X, xsum, t, u, Y);
            default: return apply_p<8>(X, xsum, t, u, Y);
        }
    }
    template <int P>
    hipError_t dots_p(const double *V, int ncols, int wc, const double *X) {
        const int tot = ncols + wc;
        hipLaunchKernelGGL((k_cmp_dots<P>), dim3(kDotChunks, (unsigned)((tot + kDotCols - 1) / kDotCols)), dim3(256),
                           0, s, V, ncols, wc, op.n, X, part);
        hipLaunchKernelGGL(k_cmp_dots_reduce, dim3(blocks_of((int64_t)tot * P)), dim3(256), 0, s,
                           (const double *)part, tot * P, h);
        return hipGetLastError();
    }
    // h = [V_0 .. V_{ncols-1} (ones)]^T X, (ncols + wc) x p row-major
    hipError_t dots(const double *V, int ncols, int wc, const double *X) {
        switch (p) {
            case 1: return dots_p<1>(V, ncols, wc, X);
            case 2: return dots_p<2>(V, ncols, wc, X);
            case 4: return dots_p<4>(V, ncols, wc, X);
            default: return dots_p<8>(V, ncols, wc, X);
        }
    }
    hipError_t update(const double *V, int ncols, int wc, double *X) {
        switch (p) {
            case 1: hipLaunchKernelGGL((k_cmp_update<1>), dim3(blocks_of(op.n)), dim3(256), 0, s, V, ncols, wc, op.n,
                                       (const double *)h, X); break;
            case 2: hipLaunchKernelGGL((k_cmp_update<2>), dim3(blocks_of(op.n)), dim3(256), 0, s, V, ncols, wc, op.n,
                                       (const double *)h, X); break;
            case 4: hipLaunchKernelGGL((k_cmp_update<4>), dim3(blocks_of(op.n)), dim3(256), 0, s, V, ncols, wc, op.n,
                                       (const double *)h, X); break;
            default: hipLaunchKernelGGL((k_cmp_update<8>), dim3(blocks_of(op.n)), dim3(256), 0, s, V, ncols, wc,
                                        op.n, (const double *)h, X); break;
        }
        return hipGetLastError();
    }
    hipError_t mulr(double *X, const double *Rinv_dev, double *Y) {
        switch (p) {
            case 1: hipLaunchKernelGGL((k_cmp_mulr<1>), dim3(blocks_of(op.n)), dim3(256), 0, s, X, op.n, Rinv_dev, Y); break;
            case 2: hipLaunchKernelGGL((k_cmp_mulr<2>), dim3(blocks_of(op.n)), dim3(256), 0, s, X, op.n, Rinv_dev, Y); break;
            case 4: hipLaunchKernelGGL((k_cmp_mulr<4>), dim3(blocks_of(op.n)), dim3(256), 0, s, X, op.n, Rinv_dev, Y); break;
            default: hipLaunchKernelGGL((k_cmp_mulr<8>), dim3(blocks_of(op.n)), dim3(256), 0, s, X, op.n, Rinv_dev, Y); break;
        }
        return hipGetLastError();
    }
};

// One projection pass: h = [V, ones]^T X, X -= [V, ones/n] h; the host copy
// of h is returned in hh ((ncols + 1) x p).
template <typename T>
int project(Lz<T> &lz, const double *V, int ncols, double *X, std::vector<double> &hh) {
    CCHK(lz.dots(V, ncols, 1, X));
    CCHK(lz.update(V, ncols, 1, X));
    hh.resize((size_t)(ncols + 1) * lz.p);
    CCHK(hipMemcpyAsync(hh.data(), lz.h, hh.size() * 8, hipMemcpyDeviceToHost, lz.s));
    CCHK(hipStreamSynchronize(lz.s));
    return SBMDS_OK;
}

// Cholesky QR of the n x p block X into Y (may alias X); R receives the factor.
// Returns 1 when X is numerically rank deficient.
template <typename T>
int cholqr(Lz<T> &lz, double *X, double *Y, double *Rinv_dev, std::vector<double> &R, double *trace = nullptr) {
    const int p = lz.p;
    CCHK(lz.dots(X, p, 0, X));
    std::vector<double> G((size_t)p * p), Rinv;
    CCHK(hipMemcpyAsync(G.data(), lz.h, G.size() * 8, hipMemcpyDeviceToHost, lz.s));
    CCHK(hipStreamSynchronize(lz.s));
    for (int i = 0; i < p; ++i)  // symmetrise the Gram
        for (int j = i + 1; j < p; ++j) G[(size_t)i * p + j] = G[(size_t)j * p + i] =
            0.5 * (G[(size_t)i * p + j] + G[(size_t)j * p + i]);
    if (trace) {
        *trace = 0.0;
        for (int i = 0; i < p; ++i) *trace += G[(size_t)i * p + i];
    }
    if (!chol_upper(G, p, R, Rinv)) return 1;
    CCHK(hipMemcpyAsync(Rinv_dev, Rinv.data(), Rinv.size() * 8, hipMemcpyHostToDevice, lz.s));
    CCHK(lz.mulr(X, Rinv_dev, Y));
    return 0;
}

template <typename T>
int lanczos_impl(const CmpOp &op, int k, int p, int max_steps, double tol, uint64_t seed, void *Z, int z_double,
                 CmpResult *res, hipStream_t s) {
    const int64_t n = op.n;
    int mmax = max_steps * p;
    if (mmax > (int)std::min<int64_t>(n - 1, 2048)) mmax = (int)std::min<int64_t>(n - 1, 2048) / p * p;
    if (mmax < p + k) return api_fail(SBMDS_EINVAL, "max_steps * block too small for k");
    // device memory: basis (mmax + p columns), working block, t/u, projection
    // partials and coefficients, small matrices
    const int maxcols = mmax + p + 1;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bV = (size_t)(mmax + p) * n * 8, bX = (size_t)p * n * 8, bt = (size_t)p * op.lda * 8;
    const size_t bpart = (size_t)maxcols * p * kDotChunks * 8, bh = (size_t)maxcols * p * 8;
    const size_t bS = (size_t)mmax * kCmpMaxK * 8, bH = (size_t)mmax * mmax * 8, bD = (size_t)mmax * 8;
    const size_t total = al(bV) + al(bX) + 2 * al(bt) + al(bpart) + al(bh) + al(bS) + al(bH) + 2 * al(bD) + 4096;
    DevMem mem;
    if (hipMalloc(&mem.p, total) != hipSuccess) {
        mem.p = nullptr;
        return api_fail(SBMDS_ENOMEM, "hipMalloc of " + std::to_string(total) + " bytes failed");
    }
    char *q = (char *)mem.p;
    auto take = [&](size_t b) {
        char *r = q;
        q += al(b);
        return (double *)r;
    };
    double *V = take(bV), *X = take(bX), *t = take(bt), *u = take(bt);
    double *part = take(bpart), *h = take(bh), *Sd = take(bS), *Hd = take(bH), *Dd = take(bD), *Ed = take(bD);
    double *Rinv_dev = take(512), *xsum = take(512);
    int *info = (int *)take(256);
    Lz<T> lz{op, p, s, part, h};
    Handle hd;
    RBCHK(rocblas_create_handle(&hd.h));
    RBCHK(rocblas_set_stream(hd.h, s));

    // start block: Gaussian, centred, orthonormal
    hipLaunchKernelGGL(k_cmp_rand, dim3(blocks_of((int64_t)p * n)), dim3(256), 0, s, X, (int64_t)p * n, seed);
    CCHK(hipGetLastError());
    std::vector<double> hh, R;
    for (int pass = 0; pass < 2; ++pass)
        if (int rc = project(lz, V, 0, X, hh); rc < 0) return rc;
    for (int pass = 0; pass < 2; ++pass) {
        const int rc = cholqr(lz, X, V, Rinv_dev, R);
        if (rc < 0) return rc;
        if (rc == 1) return api_fail(SBMDS_EBREAKDOWN, "the start block is rank deficient");
        if (pass == 0) CCHK(hipMemcpyAsync(X, V, bX, hipMemcpyDeviceToDevice, s));
    }
    int m = p;  // basis columns
    std::vector<double> H((size_t)(mmax + p) * (mmax + p), 0.0);
    auto Hat = [&](int i, int j) -> double & { return H[(size_t)i * (mmax + p) + j]; };
    std::vector<double> th, Sv, resv, best_th, best_S;
    int best_m = 0, steps = 0;
    bool converged = false;
    double best_bound = INFINITY;
    std::vector<double> bnd(kCmpMaxK, INFINITY);
    while (true) {
        const double *Vj = V + (size_t)(m - p) * n;
        // mean of each column of V_j (the J on the right of B)
        CCHK(lz.dots(nullptr, 0, 1, Vj));
        CCHK(hipMemcpyAsync(xsum, h, (size_t)p * 8, hipMemcpyDeviceToDevice, s));
        CCHK(lz.apply(Vj, xsum, t, u, X));
        std::vector<double> h1, h2;
        if (int rc = project(lz, V, m, X, h1); rc < 0) return rc;
        if (int rc = project(lz, V, m, X, h2); rc < 0) return rc;
        ++steps;
        for (int i = 0; i < m; ++i)
            for (int c = 0; c < p; ++c) {
                const double v = h1[(size_t)i * p + c] + h2[(size_t)i * p + c];
                if (i < m - p) {
                    Hat(i, m - p + c) = v;
                    Hat(m - p + c, i) = v;
                } else {
                    Hat(i, m - p + c) = v;
                }
            }
        for (int a = 0; a < p; ++a)  // symmetrise the diagonal block
            for (int b = a + 1; b < p; ++b) {
                const double v = 0.5 * (Hat(m - p + a, m - p + b) + Hat(m - p + b, m - p + a));
                Hat(m - p + a, m - p + b) = Hat(m - p + b, m - p + a) = v;
            }
        // next block: X = V_{j+1} R, Cholesky QR twice
        double *Vn = V + (size_t)m * n;
        std::vector<double> R1, R2;
        double xtrace = 0.0;
        int rk = cholqr(lz, X, Vn, Rinv_dev, R1, &xtrace);
        if (rk < 0) return rk;
        if (rk == 0) {
            CCHK(hipMemcpyAsync(X, Vn, bX, hipMemcpyDeviceToDevice, s));
            rk = cholqr(lz, X, Vn, Rinv_dev, R2);
            if (rk < 0) return rk;
        }
        std::vector<double> Rt((size_t)p * p, 0.0);  // R = R2 R1 (upper)
        if (rk == 0)
            for (int a = 0; a < p; ++a)
                for (int b = a; b < p; ++b) {
                    double v = 0.0;
                    for (int r = a; r <= b; ++r) v += R2[(size_t)a * p + r] * R1[(size_t)r * p + b];
                    Rt[(size_t)a * p + b] = v;
                }
        // a rank-deficient new block: the basis cannot grow; residual norms are
        // then bounded by ||X||_F ||s_last|| instead of ||R s_last||
        const bool stuck = rk == 1;
        // Ritz pairs of H_m and their residual norms ||R s_last||
        const int every = std::max(1, m / 64);
        const bool last = m + p > mmax;
        if (m >= k && (steps % every == 0 || stuck || last)) {
            std::vector<double> A((size_t)m * m);
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) A[(size_t)i * m + j] = Hat(i, j);
            if (int rc = dense_eig(hd.h, A, m, Hd, Dd, Ed, info, s, th, Sv); rc < 0) return rc;
            resv.assign(m, 0.0);
            for (int i = 0; i < m; ++i) {
                double r2 = 0.0;
                if (stuck) {
                    for (int b = 0; b < p; ++b) r2 += Sv[(size_t)(m - p + b) * m + i] * Sv[(size_t)(m - p + b) * m + i];
                    r2 *= xtrace;
                } else {
                    for (int a = 0; a < p; ++a) {
                        double v = 0.0;
                        for (int b = a; b < p; ++b) v += Rt[(size_t)a * p + b] * Sv[(size_t)(m - p + b) * m + i];
                        r2 += v * v;
                    }
                }
                resv[i] = sqrt(r2);
            }
            std::vector<double> bq(kCmpMaxK, INFINITY);
            const double mb = ritz_bounds(th, resv, m, k, bq.data());
            if (mb <= best_bound || best_m == 0) {
                best_bound = mb;
                best_m = m;
                best_th = th;
                best_S = Sv;
                bnd = bq;
                for (int i = 0; i < k; ++i) res->resid[i] = fabs(th[i]) > 0.0 ? resv[i] / fabs(th[i]) : INFINITY;
            }
            if (mb <= tol) {
                converged = true;
                break;
            }
        }
        if (stuck || last) break;
        for (int a = 0; a < p; ++a)  // H[j+1 block, j block] = R
            for (int b = a; b < p; ++b) {
                Hat(m + a, m - p + b) = Rt[(size_t)a * p + b];
                Hat(m - p + b, m + a) = Rt[(size_t)a * p + b];
            }
        m += p;
    }
    if (best_m == 0) return api_fail(SBMDS_ENOCONV, "no Ritz values were formed");
    // Ritz vectors of the best basis, scaled by sqrt(theta)
    const int mb = best_m;
    std::vector<double> Sk((size_t)mb * k), sc(k);
    int nonpos = 0;
    for (int q2 = 0; q2 < k; ++q2) {
        for (int i = 0; i < mb; ++i) Sk[(size_t)i * k + q2] = best_S[(size_t)i * mb + q2];
        sc[q2] = best_th[q2] > 0.0 ? sqrt(best_th[q2]) : 0.0;
        if (best_th[q2] <= 0.0) ++nonpos;
        res->eig[q2] = best_th[q2];
        res->bound[q2] = bnd[q2];
    }
    CCHK(hipMemcpyAsync(Sd, Sk.data(), Sk.size() * 8, hipMemcpyHostToDevice, s));
    CCHK(hipMemcpyAsync(Rinv_dev, sc.data(), sc.size() * 8, hipMemcpyHostToDevice, s));
    if (z_double)
        hipLaunchKernelGGL((k_cmp_ritz<double>), dim3(blocks_of(n)), dim3(256), 0, s, (const double *)V, mb, n,
                           (const double *)Sd, k, (const double *)Rinv_dev, (double *)Z);
    else
        hipLaunchKernelGGL((k_cmp_ritz<float>), dim3(blocks_of(n)), dim3(256), 0, s, (const double *)V, mb, n,
                           (const double *)Sd, k, (const double *)Rinv_dev, (float *)Z);
    CCHK(hipGetLastError());
    CCHK(hipStreamSynchronize(s));
    res->steps = steps;
    res->basis = mb;
    res->nonpositive = nonpos;
    res->status = converged ? SBMDS_OK : SBMDS_ENOCONV;
    return res->status;
}

template <typename T>
int bmds_impl(const CmpOp &op, int k, void *Z, int z_double, CmpResult *res, hipStream_t s) {
    const int64_t n = op.n, l = op.l;
    if (n >= ((int64_t)1 << 31) || l > 65535) return api_fail(SBMDS_EINVAL, "BMDS needs n < 2^31 and l <= 65535");
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bA = (size_t)n * l * 8, bLL = (size_t)l * l * 8, bC = (size_t)n * k * 8;
    const size_t bt = (size_t)op.lda * 8;
    const size_t total = al(bA) + 3 * al(bLL) + al(bC) + 2 * al((size_t)l * 8) + 2 * al(bt) + al(2 * (size_t)n * 8) +
                         al((size_t)2 * kDotChunks * 8) + 4096;
    size_t free_b = 0, tot_b = 0;
    CCHK(hipMemGetInfo(&free_b, &tot_b));
    if ((double)total > 0.9 * (double)free_b)
        return api_fail(SBMDS_ENOMEM, "BMDS needs the dense n x l matrix J P: " + std::to_string(total) +
                                          " bytes, " + std::to_string(free_b) + " free");
    DevMem mem;
    if (hipMalloc(&mem.p, total) != hipSuccess) {
        mem.p = nullptr;
        return api_fail(SBMDS_ENOMEM, "hipMalloc of " + std::to_string(total) + " bytes failed");
    }
    char *q = (char *)mem.p;
    auto take = [&](size_t b) {
        char *r = q;
        q += al(b);
        return (double *)r;
    };
    double *A = take(bA), *Rm = take(bLL), *Wd = take(bLL), *M = take(bLL), *C = take(bC);
    double *tau = take((size_t)l * 8), *D = take((size_t)l * 8), *t = take(bt), *u = take(bt);
    double *Y = take(2 * (size_t)n * 8), *part = take((size_t)2 * kDotChunks * 8), *small = take(4096 - 256);
    double *E = Y;  // off-diagonal workspace of the eigensolver (l <= 2 n)
    int *info = (int *)(small + 64);
    Handle hd;
    RBCHK(rocblas_create_handle(&hd.h));
    RBCHK(rocblas_set_stream(hd.h, s));
    const int ni = (int)n, li = (int)l;
    // A = J P (dense, column-major)
    CCHK(hipMemsetAsync(A, 0, bA, s));
    hipLaunchKernelGGL((k_bm_scatter<T>), dim3(blocks_of(n)), dim3(256), 0, s, op.rp, op.ci, (const T *)op.val, n, A);
    hipLaunchKernelGGL(k_bm_center, dim3(blocks_of(n), (unsigned)l), dim3(256), 0, s, A, n, l, op.c);
    CCHK(hipGetLastError());
    RBCHK(rocsolver_dgeqrf(hd.h, ni, li, A, ni, tau));
    hipLaunchKernelGGL(k_bm_upper, dim3(blocks_of(l), (unsigned)l), dim3(256), 0, s, (const double *)A, n, l, Rm);
    hipLaunchKernelGGL((k_bm_w64<T>), dim3(blocks_of(l), (unsigned)l), dim3(256), 0, s, (const T *)op.W, op.lda, l, Wd);
    CCHK(hipGetLastError());
    // M = -1/2 R W R^T
    const double one = 1.0, zero = 0.0, mhalf = -0.5;
    RBCHK(rocblas_dgemm(hd.h, rocblas_operation_none, rocblas_operation_none, li, li, li, &one, Rm, li, Wd, li, &zero,
                        M, li));
    RBCHK(rocblas_dgemm(hd.h, rocblas_operation_none, rocblas_operation_transpose, li, li, li, &mhalf, M, li, Rm, li,
                        &zero, Wd, li));
    RBCHK(rocsolver_dsyevd(hd.h, rocblas_evect_original, rocblas_fill_upper, li, Wd, li, D, E, info));
    int hinfo = 0;
    std::vector<double> hD(l);
    CCHK(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
    CCHK(hipMemcpyAsync(hD.data(), D, (size_t)l * 8, hipMemcpyDeviceToHost, s));
    CCHK(hipStreamSynchronize(s));
    if (hinfo != 0) return api_fail(SBMDS_EBREAKDOWN, "the dense eigensolver did not converge (info " +
                                                          std::to_string(hinfo) + ")");
    // C = Q [V_k; 0]
    hipLaunchKernelGGL(k_bm_fill, dim3(blocks_of(n), (unsigned)k), dim3(256), 0, s, (const double *)Wd, l, k, n, C);
    CCHK(hipGetLastError());
    RBCHK(rocsolver_dormqr(hd.h, rocblas_side_left, rocblas_operation_none, ni, k, li, A, ni, tau, C, ni));
    // residuals ||J B x_q - theta_q x_q|| with the Lanczos operator products (width 1)
    Lz<T> lz{op, 1, s, part, small};
    std::vector<double> sc(k);
    int nonpos = 0;
    for (int q2 = 0; q2 < k; ++q2) {
        const double th = hD[l - 1 - q2];
        res->eig[q2] = th;
        sc[q2] = th > 0.0 ? sqrt(th) : 0.0;
        if (th <= 0.0) ++nonpos;
        double *x = C + (size_t)q2 * n;
        CCHK(lz.dots(nullptr, 0, 1, x));
        CCHK(hipMemcpyAsync(small + 32, small, 8, hipMemcpyDeviceToDevice, s));
        CCHK(lz.apply(x, small + 32, t, u, Y));
        std::vector<double> hh;
        if (int rc = project(lz, nullptr, 0, Y, hh); rc < 0) return rc;  // Y = J Y
        // r = Y - theta x formed explicitly (its norm from <Y,Y>, <x,Y> and
        // <x,x> would cancel down to 1e-8 of theta)
        CCHK(hipMemcpyAsync(small, &th, 8, hipMemcpyHostToDevice, s));
        CCHK(lz.update(x, 1, 0, Y));
        CCHK(lz.dots(Y, 1, 0, Y));
        double r2 = 0.0;
        CCHK(hipMemcpyAsync(&r2, small, 8, hipMemcpyDeviceToHost, s));
        CCHK(hipStreamSynchronize(s));
        const double r = sqrt(r2 > 0.0 ? r2 : 0.0);
        res->resid[q2] = fabs(th) > 0.0 ? r / fabs(th) : INFINITY;
        res->bound[q2] = res->resid[q2];
    }
    CCHK(hipMemcpyAsync(small, sc.data(), (size_t)k * 8, hipMemcpyHostToDevice, s));
    if (z_double)
        hipLaunchKernelGGL((k_bm_out<double>), dim3(blocks_of(n)), dim3(256), 0, s, (const double *)C, n, k,
                           (const double *)small, (double *)Z);
    else
        hipLaunchKernelGGL((k_bm_out<float>), dim3(blocks_of(n)), dim3(256), 0, s, (const double *)C, n, k,
                           (const double *)small, (float *)Z);
    CCHK(hipGetLastError());
    CCHK(hipStreamSynchronize(s));
    res->nonpositive = nonpos;
    res->status = SBMDS_OK;
    return SBMDS_OK;
}

}  // namespace

int lanczos_solve(const CmpOp &op, int k, int p, int max_steps, double tol, uint64_t seed, void *Z, int z_double,
                  CmpResult *res, hipStream_t s) {
    if (k < 1 || k > kCmpMaxK) return api_fail(SBMDS_EINVAL, "k must be in [1, 16] for the comparison solvers");
    if (p != 1 && p != 2 && p != 4 && p != 8) return api_fail(SBMDS_EINVAL, "Lanczos block must be 1, 2, 4 or 8");
    if (max_steps < 1) return api_fail(SBMDS_EINVAL, "max_steps must be >= 1");
    return op.f64 ? lanczos_impl<double>(op, k, p, max_steps, tol, seed, Z, z_double, res, s)
                  : lanczos_impl<float>(op, k, p, max_steps, tol, seed, Z, z_double, res, s);
}

int bmds_solve(const CmpOp &op, int k, void *Z, int z_double, CmpResult *res, hipStream_t s) {
    if (k < 1 || k > kCmpMaxK) return api_fail(SBMDS_EINVAL, "k must be in [1, 16] for the comparison solvers");
    if (k > op.l) return api_fail(SBMDS_EINVAL, "k must be <= l");
    return op.f64 ? bmds_impl<double>(op, k, Z, z_double, res, s) : bmds_impl<float>(op, k, Z, z_double, res, s);
}

}  // namespace sbmds
