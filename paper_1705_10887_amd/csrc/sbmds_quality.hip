// Quality measures of the approximation and of the embedding, float64
// arithmetic from the given values, every sum in a fixed order (bitwise
// reproducible).
//
// Rows of the sparse biharmonic approximation K~ = P L P^T (Section 3.1:
// the landmark block L interpolated to every vertex by P on both sides) and
// their relative error against exact rows, eps = ||K~_S - K_S||^2 /
// ||K_S||^2 (Section 4.1, on the row subset S).  Two passes:
//   1. X = P_S L  (|S| x l): row i is the combination of the rows of L that
//      row s_i of P names (L symmetric, so its rows are its columns);
//   2. K~[i, v] = sum_e P[v, e] X[i, col_e] for every vertex v, with the
//      error sums of each block of vertices written as partials and summed
//      by one block.
//
// Stress of an embedding Z (n x m) against a dense symmetric distance
// matrix K (the objective of Eq. (MDS_problem), Section 2.3):
// ||Z Z^T + 1/2 J E J||_F with E = K o K.  K is read once.  With r_i the
// row means of E, g their mean and u_i = g/4 - r_i/2, the entry (i, j) of
// the matrix inside the norm is c_ij + u_i + u_j where c_ij = z_i.z_j +
// E_ij/2, so its squared norm is
//   sum c_ij^2 + 4 sum_i u_i C_i + 2 n sum u_i^2 + 2 (sum u_i)^2,
// C_i = sum_j c_ij = z_i.s + n r_i / 2 and s = sum_j z_j (E and c are
// symmetric, so column sums stand for row sums).  Expanding u_i, every term
// is a plain sum over rows of sum_j c_ij^2, sum_j E_ij, sum_j E_ij^2, r_i^2,
// z_i and r_i z_i.  The pass over K forms the first three per column (each
// thread one column, down a range of rows); the rest are block sums.  The
// same expansion with Z = 0 gives ||1/2 J E J||_F, the scale of the stress.
#include <string>
#include <type_traits>
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

// K~ rows for kQRows rows of S per block: each thread takes one vertex v,
// reads its row of P once and applies it to the kQRows rows of X (staged in
// LDS when l is small enough, else read through the cache).
constexpr int kQRows = 8;
constexpr int64_t kQLdsMaxL = 1000;  // kQRows x l doubles and the reduction buffer within 64 KB

template <typename T, bool LDS>
__global__ __launch_bounds__(256) void k_q_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                const T *__restrict__ val, int64_t n, int64_t l, int64_t S,
                                                const double *__restrict__ X, const T *__restrict__ K,
                                                double *__restrict__ out, double *__restrict__ part) {
    extern __shared__ unsigned char q_smem[];
    double *xs = (double *)q_smem;  // [kQRows][l] when LDS
    const int64_t i0 = (int64_t)blockIdx.y * kQRows;
    const int nr = (int)(S - i0 < kQRows ? S - i0 : kQRows);
    const double *xb = X + i0 * l;
    if (LDS) {
        for (int64_t t = threadIdx.x; t < nr * l; t += 256) xs[t] = xb[t];
        __syncthreads();
        xb = xs;
    }
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double kt[kQRows];
#pragma unroll
    for (int r = 0; r < kQRows; ++r) kt[r] = 0.0;
    if (v < n) {
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            const double pv = (double)val[e];
            const int64_t c = ci[e];
#pragma unroll
            for (int r = 0; r < kQRows; ++r)
                if (r < nr) kt[r] += pv * xb[r * l + c];
        }
    }
    __shared__ double red[kQRows][2][4];
#pragma unroll
    for (int r = 0; r < kQRows; ++r) {
        if (r >= nr) break;
        const int64_t i = i0 + r;
        double num = 0.0, den = 0.0;
        if (v < n) {
            if (out) out[i * n + v] = kt[r];
            if (K) {
                const double k = (double)K[i * n + v];
                num = (kt[r] - k) * (kt[r] - k);
                den = k * k;
            }
        }
        if (part) {
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) {
                num += __shfl_xor(num, m);
                den += __shfl_xor(den, m);
            }
            if ((threadIdx.x & 63) == 0) {
                red[r][0][threadIdx.x >> 6] = num;
                red[r][1][threadIdx.x >> 6] = den;
            }
        }
    }
    if (!part) return;
    __syncthreads();
    if (threadIdx.x < 2 * nr) {
        const int r = threadIdx.x >> 1, h = threadIdx.x & 1;
        const size_t b = (size_t)(i0 + r) * gridDim.x + blockIdx.x;
        const double *x = red[r][h];
        part[2 * b + h] = x[0] + x[1] + x[2] + x[3];
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

constexpr int kStressMaxM = 16;   // embedding dimensions supported
constexpr int kStressUnroll = 8;  // rows of K in flight per thread
constexpr int kStressVals = 4 + 2 * kStressMaxM;

// Block-wide sum in a fixed order (a butterfly within each wave, then the
// four wave sums in order); every thread gets the result.
__device__ double block_sum_fixed(double v, double *buf) {
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) v += __shfl_xor(v, sh);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((buf[0] + buf[1]) + buf[2]) + buf[3];
}

// One pass over K: thread t of block (x, y) takes V consecutive columns
// j = V (256 x + t) + c and walks them down the rows of split y with
// kStressUnroll (V = 1) or half as many (V = 4) coalesced row loads in
// flight.  V = 4 (16-byte loads of float32 rows) needs m <= 4, n % 4 == 0
// and K 16-byte aligned.  It writes part[(3 y + s) n + j] for s = 0, 1, 2:
// the split's sums of c_ij^2, E_ij and E_ij^2.  z_j stays in registers; z_i
// is the same for the whole block.  Threads past the last columns read the
// last V columns and store nothing.
template <typename T, int V, int MM>
__global__ __launch_bounds__(256) void k_q_stress_part(const T *__restrict__ Z, int64_t n, int m,
                                                       int64_t rows_per_split, const T *__restrict__ K,
                                                       double *__restrict__ part) {
    const int64_t j = ((int64_t)blockIdx.x * 256 + threadIdx.x) * V;
    const int64_t jc = j < n ? j : n - V;
    const int64_t ib = (int64_t)blockIdx.y * rows_per_split;
    const int64_t ie = (ib + rows_per_split < n ? ib + rows_per_split : n);
    double zj[V][MM];
#pragma unroll
    for (int c = 0; c < V; ++c)
#pragma unroll
        for (int q = 0; q < MM; ++q) zj[c][q] = q < m ? (double)Z[(jc + c) * m + q] : 0.0;
    double c2[V], se[V], se2[V];
#pragma unroll
    for (int c = 0; c < V; ++c) c2[c] = se[c] = se2[c] = 0.0;
    auto add = [&](int64_t i, const T *kv) {
#pragma unroll
        for (int c = 0; c < V; ++c) {
            double a = 0.0;
#pragma unroll
            for (int q = 0; q < MM; ++q)
                if (q < m) a += (double)Z[i * m + q] * zj[c][q];
            const double e = (double)kv[c] * (double)kv[c];
            const double h = a + 0.5 * e;
            c2[c] += h * h;
            se[c] += e;
            se2[c] += e * e;
        }
    };
    auto load = [&](int64_t i, T *kv) {
        const T *src = (const T *)__builtin_assume_aligned(K + i * n + jc, V * sizeof(T) >= 16 ? 16 : sizeof(T));
#pragma unroll
        for (int c = 0; c < V; ++c) kv[c] = src[c];
    };
    int64_t i = ib;
    constexpr int U = V == 1 ? kStressUnroll : kStressUnroll / 2;
    for (; i + U <= ie; i += U) {
        T kv[U][V];
#pragma unroll
        for (int t = 0; t < U; ++t) load(i + t, kv[t]);
#pragma unroll
        for (int t = 0; t < U; ++t) add(i + t, kv[t]);
    }
    for (; i < ie; ++i) {
        T kv[V];
        load(i, kv);
        add(i, kv);
    }
    if (j < n) {
        double *p = part + (int64_t)blockIdx.y * 3 * n + j;
#pragma unroll
        for (int c = 0; c < V; ++c) {
            p[c] = c2[c];
            p[n + c] = se[c];
            p[2 * n + c] = se2[c];
        }
    }
}

// Per column j: the split sums added in split order, then this block's sums
// of sum_j c^2, sum_j E, sum_j E^2, r_j^2, z_j (m) and r_j z_j (m), written
// to blk[blockIdx.x][0 .. 4 + 2m).
template <typename T>
__global__ __launch_bounds__(256) void k_q_stress_cols(const T *__restrict__ Z, int64_t n, int m, int splits,
                                                       const double *__restrict__ part, double *__restrict__ blk) {
    __shared__ double buf[4];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double c2 = 0.0, se = 0.0, se2 = 0.0;
    if (j < n) {
        int y = 0;
        for (; y + 8 <= splits; y += 8) {  // 24 loads in flight, added in split order
            double v[8][3];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const double *p = part + (int64_t)(y + t) * 3 * n + j;
                v[t][0] = p[0];
                v[t][1] = p[n];
                v[t][2] = p[2 * n];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                c2 += v[t][0];
                se += v[t][1];
                se2 += v[t][2];
            }
        }
        for (; y < splits; ++y) {
            const double *p = part + (int64_t)y * 3 * n + j;
            c2 += p[0];
            se += p[n];
            se2 += p[2 * n];
        }
    }
    const double r = se / (double)n;
    double *o = blk + (int64_t)blockIdx.x * kStressVals;
    const double v4[4] = {c2, se, se2, r * r};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double x = block_sum_fixed(v4[t], buf);
        if (threadIdx.x == 0) o[t] = x;
    }
#pragma unroll
    for (int q = 0; q < kStressMaxM; ++q) {
        if (q < m) {  // m is the same for every thread
            const double z = j < n ? (double)Z[j * m + q] : 0.0;
            const double a = block_sum_fixed(z, buf);
            const double b = block_sum_fixed(r * z, buf);
            if (threadIdx.x == 0) {
                o[4 + q] = a;
                o[4 + kStressMaxM + q] = b;
            }
        }
    }
}

// out[0] = stress, out[1] = ||1/2 J E J||_F from the block sums (added in
// block order).
__global__ __launch_bounds__(256) void k_q_stress_finish(int64_t n, int m, int64_t nblk,
                                                         const double *__restrict__ blk, double *__restrict__ out) {
    __shared__ double buf[4];
    __shared__ double tot[kStressVals];
    for (int v = 0; v < kStressVals; ++v) {
        double x = 0.0;
        for (int64_t b = threadIdx.x; b < nblk; b += 256) x += blk[b * kStressVals + v];
        x = block_sum_fixed(x, buf);
        if (threadIdx.x == 0) tot[v] = x;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double dn = (double)n;
    const double A = tot[0], Se = tot[1], Se2 = tot[2], R2 = tot[3];
    const double g = Se / (dn * dn), R1 = Se / dn;
    double ss = 0.0, ts = 0.0;
    for (int q = 0; q < m; ++q) {
        ss += tot[4 + q] * tot[4 + q];
        ts += tot[4 + kStressMaxM + q] * tot[4 + q];
    }
    const double su = 0.25 * dn * g - 0.5 * R1;
    const double su2 = dn * g * g / 16.0 - 0.25 * g * R1 + 0.25 * R2;
    const double uc0 = 0.125 * g * dn * R1 - 0.25 * dn * R2;  // sum u_i C_i at Z = 0
    const double uc = 0.25 * g * ss - 0.5 * ts + uc0;
    const double tail = 2.0 * dn * su2 + 2.0 * su * su;
    const double s2 = A + 4.0 * uc + tail;
    const double n2 = 0.25 * Se2 + 4.0 * uc0 + tail;
    out[0] = sqrt(s2 > 0.0 ? s2 : 0.0);
    out[1] = sqrt(n2 > 0.0 ? n2 : 0.0);
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
    const dim3 qg((unsigned)nb, (unsigned)((S + kQRows - 1) / kQRows));
    if (l <= kQLdsMaxL)
        hipLaunchKernelGGL((k_q_rows<T, true>), qg, dim3(256), (size_t)kQRows * l * 8, s, drp, dci, dval, n, l, S, X,
                           dK, dout, dK ? part : nullptr);
    else
        hipLaunchKernelGGL((k_q_rows<T, false>), qg, dim3(256), 0, s, drp, dci, dval, n, l, S, X, dK, dout,
                           dK ? part : nullptr);
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

template <typename T>
int stress_impl(const T *Z, int64_t n, int m, const T *K, int mem, double *out, hipStream_t s) {
    // splits of the rows: at least about 2048 blocks over the columns and
    // rows, each split at least 64 rows
    const int64_t ncb = (n + 255) / 256;
    // host inputs are copied to 256-byte aligned scratch
    const bool vec = std::is_same<T, float>::value && m <= 4 && n % 4 == 0 &&
                     (mem == SBMDS_MEM_HOST || ((uintptr_t)K & 15) == 0);
    const int64_t nxb = vec ? (n + 1023) / 1024 : ncb;  // blocks across the columns of the pass over K
    int64_t splits = (2048 + nxb - 1) / nxb;
    const int64_t max_splits = (n + 63) / 64;
    if (splits > max_splits) splits = max_splits;
    if (splits < 1) splits = 1;
    const int64_t rows_per_split = (n + splits - 1) / splits;
    splits = (n + rows_per_split - 1) / rows_per_split;
    const size_t b_part = (size_t)splits * 3 * n * 8, b_blk = (size_t)ncb * kStressVals * 8;
    const size_t b_Z = (size_t)n * m * sizeof(T), b_K = (size_t)n * n * sizeof(T);
    const bool host = mem == SBMDS_MEM_HOST;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t total = al(b_part) + al(b_blk) + 256 + (host ? al(b_Z) + al(b_K) : 0);
    Tmp tmp;
    if (hipMalloc(&tmp.p, total) != hipSuccess) {
        tmp.p = nullptr;
        return api_fail(SBMDS_ENOMEM, "hipMalloc of " + std::to_string(total) + " bytes failed");
    }
    char *q = (char *)tmp.p;
    double *part = (double *)q;
    double *blk = (double *)(q + al(b_part));
    double *dout = (double *)(q + al(b_part) + al(b_blk));
    const T *dZ = Z, *dK = K;
    if (host) {
        T *a = (T *)(q + al(b_part) + al(b_blk) + 256);
        T *b = (T *)((char *)a + al(b_Z));
        QCHK(hipMemcpyAsync(a, Z, b_Z, hipMemcpyHostToDevice, s));
        QCHK(hipMemcpyAsync(b, K, b_K, hipMemcpyHostToDevice, s));
        dZ = a;
        dK = b;
    }
    if (vec)
        hipLaunchKernelGGL((k_q_stress_part<T, 4, 4>), dim3((unsigned)nxb, (unsigned)splits), dim3(256), 0, s, dZ, n,
                           m, rows_per_split, dK, part);
    else
        hipLaunchKernelGGL((k_q_stress_part<T, 1, kStressMaxM>), dim3((unsigned)ncb, (unsigned)splits), dim3(256), 0,
                           s, dZ, n, m, rows_per_split, dK, part);
    QCHK(hipGetLastError());
    hipLaunchKernelGGL((k_q_stress_cols<T>), dim3((unsigned)ncb), dim3(256), 0, s, dZ, n, m, (int)splits, part,
                       blk);
    QCHK(hipGetLastError());
    hipLaunchKernelGGL(k_q_stress_finish, dim3(1), dim3(256), 0, s, n, m, ncb, blk, dout);
    QCHK(hipGetLastError());
    double h[2];
    QCHK(hipMemcpyAsync(h, dout, 16, hipMemcpyDeviceToHost, s));
    QCHK(hipStreamSynchronize(s));
    out[0] = h[0];
    out[1] = h[1];
    return SBMDS_OK;
}

}  // namespace
}  // namespace sbmds

extern "C" int sbmds_stress(const void *Z, int64_t n, int m, const void *K, int fp64, int mem, double *out,
                            void *stream) {
    using namespace sbmds;
    api_clear_error();
    if (!Z || !K || !out) return api_fail(SBMDS_EINVAL, "Z, K and out must be non-NULL");
    if (mem != SBMDS_MEM_HOST && mem != SBMDS_MEM_DEVICE) return api_fail(SBMDS_EINVAL, "mem must be 0 or 1");
    if (n < 1 || n >= ((int64_t)1 << 31)) return api_fail(SBMDS_EINVAL, "need 1 <= n < 2^31");
    if (m < 1 || m > kStressMaxM) return api_fail(SBMDS_EINVAL, "need 1 <= m <= 16");
    try {
        return fp64 ? stress_impl<double>((const double *)Z, n, m, (const double *)K, mem, out, (hipStream_t)stream)
                    : stress_impl<float>((const float *)Z, n, m, (const float *)K, mem, out, (hipStream_t)stream);
    } catch (const std::exception &e) {
        return api_fail(SBMDS_ENOMEM, std::string("host exception: ") + e.what());
    }
}

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
