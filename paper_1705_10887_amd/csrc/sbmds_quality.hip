// Rows of the sparse biharmonic approximation K~ = P L P^T (Section 3.1:
// the landmark block L interpolated to every vertex by P on both sides) and
// their relative error against exact rows, eps = ||K~_S - K_S||^2 /
// ||K_S||^2 (Section 4.1, on the row subset S).  Two passes, float64
// arithmetic from the given values:
//   1. X = P_S L  (|S| x l): row i is the combination of the rows of L that
//      row s_i of P names (L symmetric, so its rows are its columns);
//   2. K~[i, v] = sum_e P[v, e] X[i, col_e] for every vertex v, with the
//      error sums of each block of vertices written as partials and summed
//      by one block in a fixed order (bitwise reproducible).
#include <string>
#include <vector>

#include "../../include/sbmds.h"
#include "sbmds_common.h"
#include "sbmds_mlp_internal.h"  // api_fail / api_clear_error
#include "sbmds_prep.h"

namespace sbmds {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_q_landmark_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                         const T *__restrict__ val, const T *__restrict__ L, int64_t l,
                                                         const int32_t *__restrict__ rows, double *__restrict__ X) {
    const int i = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= l) return;
    const int32_t s = rows[i];
    double x = 0.0;
    for (int32_t e = rp[s]; e < rp[s + 1]; ++e) x += (double)val[e] * (double)L[(int64_t)ci[e] * l + j];
    X[(int64_t)i * l + j] = x;
}

template <typename T>
__global__ __launch_bounds__(256) void k_q_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                const T *__restrict__ val, int64_t n, int64_t l,
                                                const double *__restrict__ X, const T *__restrict__ K,
                                                double *__restrict__ out, double *__restrict__ part) {
    const int i = blockIdx.y;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double num = 0.0, den = 0.0;
    if (v < n) {
        const double *xi = X + (int64_t)i * l;
        double kt = 0.0;
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) kt += (double)val[e] * xi[ci[e]];
        if (out) out[(int64_t)i * n + v] = kt;
        if (K) {
            const double k = (double)K[(int64_t)i * n + v];
            num = (kt - k) * (kt - k);
            den = k * k;
        }
    }
    if (!part) return;
    __shared__ double red[2][4];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        num += __shfl_xor(num, m);
        den += __shfl_xor(den, m);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = num;
        red[1][threadIdx.x >> 6] = den;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const size_t b = (size_t)i * gridDim.x + blockIdx.x;
        part[2 * b] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        part[2 * b + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// Sum of the partials in a fixed order (each thread a fixed stride, then the
// threads in order).
__global__ __launch_bounds__(256) void k_q_reduce(const double *__restrict__ part, int64_t count,
                                                  double *__restrict__ out) {
    __shared__ double s[2][256];
    double a = 0.0, b = 0.0;
    for (int64_t q = threadIdx.x; q < count; q += 256) {
        a += part[2 * q];
        b += part[2 * q + 1];
    }
    s[0][threadIdx.x] = a;
    s[1][threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int t = 0; t < 256; ++t) {
            x += s[0][t];
            y += s[1][t];
        }
        out[0] = x;
        out[1] = y;
    }
}

struct Tmp {
    void *p = nullptr;
    ~Tmp() {
        if (p) (void)hipFree(p);
    }
};

#define QCHK(expr)                                                                                          \
    do {                                                                                                    \
        hipError_t _e = (expr);                                                                             \
        if (_e != hipSuccess) return api_fail(SBMDS_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

template <typename T>
int approx_rows_impl(const sbmds_problem &pr, const T *L, const int32_t *rows, int64_t S, const T *K, double *err,
                     double *out, int out_mem, hipStream_t s) {
    const int64_t n = pr.n, l = pr.l, nnz = pr.nnz;
    const size_t b_rp = (size_t)(n + 1) * 4, b_ci = (size_t)nnz * 4, b_v = (size_t)nnz * sizeof(T);
    const size_t b_L = (size_t)l * l * sizeof(T), b_rows = (size_t)S * 4;
    const size_t b_K = K ? (size_t)S * n * sizeof(T) : 0;
    const int64_t nb = (n + 255) / 256;
    const size_t b_X = (size_t)S * l * 8, b_part = (size_t)S * nb * 16;
    const size_t b_out = (out && out_mem == SBMDS_MEM_HOST) ? (size_t)S * n * 8 : 0;
    const bool host = pr.mem == SBMDS_MEM_HOST;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t total = al(b_X) + al(b_part) + 256 + al(b_out) + 8;
    if (host) total += al(b_rp) + al(b_ci) + al(b_v) + al(b_L) + al(b_rows) + al(b_K);
    Tmp tmp;
    if (hipMalloc(&tmp.p, total) != hipSuccess) {
        tmp.p = nullptr;
        return api_fail(SBMDS_ENOMEM, "hipMalloc of " + std::to_string(total) + " bytes failed");
    }
    char *q = (char *)tmp.p;
    auto take = [&](size_t b) {
        char *r = q;
        q += al(b);
        return r;
    };
    double *X = (double *)take(b_X);
    double *part = (double *)take(b_part);
    double *derr = (double *)take(256);
    double *dout = b_out ? (double *)take(b_out) : out;
    const int32_t *drp = pr.P_rowptr, *dci = pr.P_col, *drows = rows;
    const T *dval = (const T *)pr.P_val, *dL = L, *dK = K;
    if (host) {
        int32_t *a = (int32_t *)take(b_rp);
        int32_t *b = (int32_t *)take(b_ci);
        T *c = (T *)take(b_v);
        T *d = (T *)take(b_L);
        int32_t *e = (int32_t *)take(b_rows);
        T *f = b_K ? (T *)take(b_K) : nullptr;
        QCHK(hipMemcpyAsync(a, drp, b_rp, hipMemcpyHostToDevice, s));
        if (nnz) QCHK(hipMemcpyAsync(b, dci, b_ci, hipMemcpyHostToDevice, s));
        if (nnz) QCHK(hipMemcpyAsync(c, dval, b_v, hipMemcpyHostToDevice, s));
        QCHK(hipMemcpyAsync(d, dL, b_L, hipMemcpyHostToDevice, s));
        QCHK(hipMemcpyAsync(e, drows, b_rows, hipMemcpyHostToDevice, s));
        if (f) QCHK(hipMemcpyAsync(f, dK, b_K, hipMemcpyHostToDevice, s));
        drp = a;
        dci = b;
        dval = c;
        dL = d;
        drows = e;
        dK = f;
    }
    // the operator and L are checked on the device before any of it is used
    // as an index (the same checks as for sbmds_create's device inputs)
    unsigned long long *dchk = (unsigned long long *)(derr + 4);
    unsigned long long hchk = kPrepNoError;
    QCHK(hipMemcpyAsync(dchk, &hchk, 8, hipMemcpyHostToDevice, s));
    QCHK(prep_validate<T>(drp, dci, dval, dL, n, l, nnz, dchk, s));
    QCHK(hipMemcpyAsync(&hchk, dchk, 8, hipMemcpyDeviceToHost, s));
    std::vector<int32_t> hrows(S);
    QCHK(hipMemcpyAsync(hrows.data(), drows, b_rows, hipMemcpyDeviceToHost, s));
    QCHK(hipStreamSynchronize(s));
    if (hchk != kPrepNoError) return api_fail(SBMDS_EINVAL, "the operator or L failed validation (code " +
                                                               std::to_string(hchk >> 40) + ")");
    for (int64_t i = 0; i < S; ++i)
        if (hrows[i] < 0 || hrows[i] >= n) return api_fail(SBMDS_EINVAL, "rows[" + std::to_string(i) + "] out of range");
    hipLaunchKernelGGL((k_q_landmark_rows<T>), dim3((unsigned)((l + 255) / 256), (unsigned)S), dim3(256), 0, s, drp,
                       dci, dval, dL, l, drows, X);
    QCHK(hipGetLastError());
    hipLaunchKernelGGL((k_q_rows<T>), dim3((unsigned)nb, (unsigned)S), dim3(256), 0, s, drp, dci, dval, n, l, X, dK,
                       dout, dK ? part : nullptr);
    QCHK(hipGetLastError());
    if (dK) {
        hipLaunchKernelGGL(k_q_reduce, dim3(1), dim3(256), 0, s, part, S * nb, derr);
        QCHK(hipGetLastError());
    }
    if (b_out) QCHK(hipMemcpyAsync(out, dout, b_out, hipMemcpyDeviceToHost, s));
    double herr[2] = {0.0, 0.0};
    if (dK) QCHK(hipMemcpyAsync(herr, derr, 16, hipMemcpyDeviceToHost, s));
    QCHK(hipStreamSynchronize(s));
    if (err) {
        err[0] = herr[0];
        err[1] = herr[1];
    }
    return SBMDS_OK;
}

}  // namespace
}  // namespace sbmds

extern "C" int sbmds_approx_rows(const sbmds_problem *prob, int fp64, const void *L, const int32_t *rows,
                                 int64_t nrows, const void *K_rows, double *err, double *out, int out_mem,
                                 void *stream) {
    using namespace sbmds;
    api_clear_error();
    if (!prob || !L || !rows) return api_fail(SBMDS_EINVAL, "prob, L and rows must be non-NULL");
    const sbmds_problem &p = *prob;
    if (p.mem != SBMDS_MEM_HOST && p.mem != SBMDS_MEM_DEVICE) return api_fail(SBMDS_EINVAL, "mem must be 0 or 1");
    if (out && out_mem != SBMDS_MEM_HOST && out_mem != SBMDS_MEM_DEVICE)
        return api_fail(SBMDS_EINVAL, "out_mem must be 0 or 1");
    if (p.l < 1 || p.n < p.l || p.n >= ((int64_t)1 << 31) || p.l > ((int64_t)1 << 20))
        return api_fail(SBMDS_EINVAL, "need 1 <= l <= n < 2^31 and l <= 2^20");
    if (p.nnz < 0 || p.nnz >= ((int64_t)1 << 31)) return api_fail(SBMDS_EINVAL, "nnz out of range");
    if (!p.P_rowptr || (p.nnz > 0 && (!p.P_col || !p.P_val))) return api_fail(SBMDS_EINVAL, "P arrays are NULL");
    if (nrows < 1 || nrows > 4096) return api_fail(SBMDS_EINVAL, "nrows must be in [1, 4096]");
    if (!err && !out) return api_fail(SBMDS_EINVAL, "nothing to compute: err and out are both NULL");
    if (err && !K_rows) return api_fail(SBMDS_EINVAL, "err needs K_rows");
    try {
        return fp64 ? approx_rows_impl<double>(p, (const double *)L, rows, nrows, (const double *)K_rows, err, out,
                                               out_mem, (hipStream_t)stream)
                    : approx_rows_impl<float>(p, (const float *)L, rows, nrows, (const float *)K_rows, err, out,
                                              out_mem, (hipStream_t)stream);
    } catch (const std::exception &e) {
        return api_fail(SBMDS_ENOMEM, std::string("host exception: ") + e.what());
    }
}
