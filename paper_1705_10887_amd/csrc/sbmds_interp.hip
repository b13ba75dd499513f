// The interpolation operator P of Eq. (PDefinition) built on the device
// from a triangle mesh and its landmarks (Sections 2.2, 3.1):
//   1. the cotangent weights A_ij = (cot alpha_ij + cot beta_ij) / 2 of every
//      edge and the lumped mass d_i (a third of the area of the triangles at
//      i), or, for the generic-graph variant, A the 0/1 edge adjacency and
//      D = I;  L = diag(A 1) - A;
//   2. M = L^T D^-1 L, written densely in the order [non-landmarks,
//      landmarks]: M_uu and M_ub are then its two leading blocks;
//   3. P_u = -M_uu^-1 M_ub by a dense Cholesky factorisation and two
//      triangular solves (rocSOLVER), the l right-hand sides at once;
//   4. the thresholding of Section 3.1: in every column the p entries of
//      largest magnitude (ties at the cut to the lower vertex, exact zeros
//      never kept), by a segmented radix sort of the magnitudes;
//   5. the CSR of P with the identity rows of the landmarks.
// Edges and per-vertex sums come from radix sorts and segmented sums in a
// fixed order, so the result is bitwise reproducible.  The dense route costs
// 8 n^2 bytes and O(n^3) flops: it serves meshes up to a few ten thousand
// vertices.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/sbmds.h"
#include "sbmds_mlp_internal.h"  // api_fail

namespace sbmds {
namespace {

constexpr int64_t kInterpMaxN = 46340;  // n^2 < 2^31 elements in the dense M

unsigned nb(int64_t c) { return (unsigned)((c + 255) / 256); }

// Input checks: face entries in range and distinct, landmarks in range and
// distinct (mark[v] counts them), coordinates finite.  err = smallest code.
__global__ __launch_bounds__(256) void k_in_check(const double *__restrict__ V, int64_t n,
                                                  const int32_t *__restrict__ F, int64_t nf,
                                                  const int32_t *__restrict__ lm, int64_t l, int32_t *__restrict__ mark,
                                                  int *__restrict__ err) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < nf) {
        const int32_t a = F[3 * t], b = F[3 * t + 1], c = F[3 * t + 2];
        if (a < 0 || b < 0 || c < 0 || a >= n || b >= n || c >= n || a == b || b == c || a == c) atomicMin(err, 1);
    }
    if (t < l) {
        const int32_t v = lm[t];
        if (v < 0 || v >= n) atomicMin(err, 2);
        else if (atomicAdd(&mark[v], 1) != 0) atomicMin(err, 3);
    }
    if (t < n) {
        for (int q = 0; q < 3; ++q)
            if (!(fabs(V[3 * t + q]) < INFINITY)) atomicMin(err, 4);
    }
}

// Per triangle corner k (opposite edge {i, j}): the edge key and half the
// cotangent of the angle at the corner; per (vertex, corner) a mass key and
// a third of the triangle's area.  Products are rounded one at a time.
__global__ __launch_bounds__(256) void k_corners(const double *__restrict__ V, const int32_t *__restrict__ F,
                                                 int64_t nf, int64_t n, int graph, int64_t *__restrict__ ekey,
                                                 double *__restrict__ ehalf, int64_t *__restrict__ mkey,
                                                 double *__restrict__ marea) {
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nf) return;
    const int32_t f[3] = {F[3 * t], F[3 * t + 1], F[3 * t + 2]};
    double p[3][3];
    for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 3; ++q) p[a][q] = V[3 * (int64_t)f[a] + q];
    // area from the cross product of the edges at corner 0
    double e1[3], e2[3], cr[3];
    for (int q = 0; q < 3; ++q) {
        e1[q] = p[1][q] - p[0][q];
        e2[q] = p[2][q] - p[0][q];
    }
    cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double area = 0.5 * sqrt((cr[0] * cr[0] + cr[1] * cr[1]) + cr[2] * cr[2]);
    const double third = area / 3.0;
    for (int k = 0; k < 3; ++k) {
        const int32_t o = f[k], i = f[(k + 1) % 3], j = f[(k + 2) % 3];
        double a[3], b[3], c[3];
        for (int q = 0; q < 3; ++q) {
            a[q] = p[(k + 1) % 3][q] - p[k][q];
            b[q] = p[(k + 2) % 3][q] - p[k][q];
        }
        c[0] = a[1] * b[2] - a[2] * b[1];
        c[1] = a[2] * b[0] - a[0] * b[2];
        c[2] = a[0] * b[1] - a[1] * b[0];
        const double dot = (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
        const double crs = sqrt((c[0] * c[0] + c[1] * c[1]) + c[2] * c[2]);
        const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
        ekey[3 * t + k] = lo * n + hi;
        ehalf[3 * t + k] = graph ? 1.0 : 0.5 * (dot / crs);
        // mass records ordered by (vertex, corner, triangle)
        mkey[3 * t + k] = ((int64_t)o * 3 + k) * nf + t;
        marea[3 * t + k] = graph ? 1.0 : third;
    }
}

// Segment heads of a sorted key array: head[i] = 1 where key changes.
__global__ __launch_bounds__(256) void k_heads(const int64_t *__restrict__ key, int64_t count, int64_t div,
                                               int32_t *__restrict__ head) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    head[i] = (i == 0 || key[i] / div != key[i - 1] / div) ? 1 : 0;
}

// Unique edges: edge e = the segment starting at a head (segment id from the
// inclusive scan of heads); its weight the sum of its records in sorted
// order (the generic-graph variant keeps 1).  Writes both directions.
__global__ __launch_bounds__(256) void k_edges(const int64_t *__restrict__ key, const double *__restrict__ val,
                                               const int32_t *__restrict__ head, const int32_t *__restrict__ segid,
                                               int64_t count, int64_t n, int graph, int64_t *__restrict__ dkey,
                                               double *__restrict__ dval) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count || !head[i]) return;
    double s = 0.0;
    int64_t q = i;
    do {
        s += val[q];
        ++q;
    } while (q < count && !head[q]);
    if (graph) s = 1.0;
    const int64_t e = segid[i] - 1;
    const int64_t a = key[i] / n, b = key[i] % n;
    dkey[2 * e] = a * n + b;
    dkey[2 * e + 1] = b * n + a;
    dval[2 * e] = s;
    dval[2 * e + 1] = s;
}

// Lumped mass: d[v] = sum of its records in (corner, triangle) order.
__global__ __launch_bounds__(256) void k_mass(const int64_t *__restrict__ key, const double *__restrict__ val,
                                              const int32_t *__restrict__ head, int64_t count, int64_t per_vertex,
                                              int graph, double *__restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count || !head[i]) return;
    double s = 0.0;
    int64_t q = i;
    do {
        s += val[q];
        ++q;
    } while (q < count && !head[q]);
    d[key[i] / per_vertex] = graph ? 1.0 : s;
}

// Row pointers (nrows + 1) of entries sorted by key, row = key / div.
__global__ __launch_bounds__(256) void k_rowptr(const int64_t *__restrict__ key, int64_t count, int64_t div,
                                                int64_t nrows, int32_t *__restrict__ rp) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i > count) return;
    const int64_t r = i < count ? key[i] / div : nrows;
    const int64_t rprev = i > 0 ? key[i - 1] / div : -1;
    for (int64_t q = rprev + 1; q <= r; ++q) rp[q] = (int32_t)i;
}

// Vertex positions in the dense order: non-landmarks first (ascending id),
// then the landmarks in their order.  uflag[v] = 1 for non-landmarks.
__global__ __launch_bounds__(256) void k_uflag(const int32_t *__restrict__ mark, int64_t n, int32_t *__restrict__ uflag) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v < n) uflag[v] = mark[v] ? 0 : 1;
}

__global__ __launch_bounds__(256) void k_positions(const int32_t *__restrict__ uflag, const int32_t *__restrict__ urank,
                                                   const int32_t *__restrict__ lm, int64_t n, int64_t l, int64_t m,
                                                   int32_t *__restrict__ pos, int32_t *__restrict__ uvert) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v < n && uflag[v]) {
        pos[v] = urank[v];
        uvert[urank[v]] = (int32_t)v;
    }
    if (v < l) pos[lm[v]] = (int32_t)(m + v);
}

// M = L^T D^-1 L into the dense column-major Md (n x n) in position order:
// thread i owns row i, M_ij = sum over k of (L_ki / d_k) L_kj in ascending
// k (L symmetric, so row k of L is its column k).  L's row i is the diagonal
// deg_i and -A_ij off it.
__global__ __launch_bounds__(256) void k_dense_m(const int32_t *__restrict__ rp, const int64_t *__restrict__ dkey,
                                                 const double *__restrict__ dval, const double *__restrict__ d,
                                                 const int32_t *__restrict__ pos, int64_t n, double *__restrict__ Md) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double *row = Md + pos[i];  // element (pos i, pos j) at pos j * n + pos i
    auto degree = [&](int64_t k) {
        double s = 0.0;
        for (int32_t e = rp[k]; e < rp[k + 1]; ++e) s += dval[e];
        return s;
    };
    // entries of L's row i in ascending column order: the diagonal goes
    // between the neighbours below and above i
    auto for_row = [&](int64_t r, auto &&fn) {
        const double dg = degree(r);
        bool diag_done = false;
        for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int64_t c = dkey[e] % n;
            if (!diag_done && c > r) {
                fn(r, dg);
                diag_done = true;
            }
            fn(c, -dval[e]);
        }
        if (!diag_done) fn(r, dg);
    };
    for_row(i, [&](int64_t k, double lik) {
        const double coef = lik * (1.0 / d[k]);
        for_row(k, [&](int64_t j, double lkj) {
            double *x = row + (int64_t)pos[j] * n;
            *x = *x + coef * lkj;
        });
    });
}

// B = -M_ub (m x l, column-major) from the dense M.
__global__ __launch_bounds__(256) void k_rhs(const double *__restrict__ Md, int64_t n, int64_t m, int64_t l,
                                             double *__restrict__ B) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (r >= m || c >= l) return;
    B[c * m + r] = -Md[(m + c) * n + r];
}

// Sort keys for the thresholding: magnitude bits complemented (largest
// first), the row as the value; exact zeros get the largest key.
__global__ __launch_bounds__(256) void k_mag_keys(const double *__restrict__ X, int64_t count,
                                                  uint64_t *__restrict__ key, int32_t *__restrict__ idx, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const double a = fabs(X[i]);
    key[i] = ~(uint64_t)__double_as_longlong(a);
    idx[i] = (int32_t)(i % m);
}

// Kept entries of column c: the first min(p, nonzeros) of its sorted
// segment; flag[c * m + r] = 1 for a kept row r.
__global__ __launch_bounds__(256) void k_keep(const uint64_t *__restrict__ key, const int32_t *__restrict__ idx,
                                              int64_t m, int64_t l, int64_t p, int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m * l) return;
    const int64_t c = i / m, rank = i % m;
    const bool nonzero = key[i] != ~(uint64_t)0;  // |x| > 0
    if (nonzero && (p <= 0 || rank < p)) flag[c * m + idx[i]] = 1;
}

// Entries of P as (row * l + col) keys and values: kept entries of P_u, then
// the landmark identity rows.
__global__ __launch_bounds__(256) void k_entries(const double *__restrict__ X, const int32_t *__restrict__ flag,
                                                 const int32_t *__restrict__ slot, const int32_t *__restrict__ uvert,
                                                 const int32_t *__restrict__ lm, int64_t m, int64_t l,
                                                 int64_t nkept, int64_t *__restrict__ key,
                                                 double *__restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m * l && flag[i]) {
        const int64_t c = i / m, r = i % m;
        const int64_t s = slot[i];
        key[s] = (int64_t)uvert[r] * l + c;
        val[s] = X[i];
    }
    if (i < l) {
        key[nkept + i] = (int64_t)lm[i] * l + i;
        val[nkept + i] = 1.0;
    }
}

__global__ __launch_bounds__(256) void k_csr_out(const int64_t *__restrict__ key, const double *__restrict__ val,
                                                 const int32_t *__restrict__ perm, int64_t count, int64_t l,
                                                 int32_t *__restrict__ col, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    col[i] = (int32_t)(key[i] % l);
    out[i] = val[perm[i]];
}

#define ICHK(expr)                                                                                          \
    do {                                                                                                    \
        hipError_t _e = (expr);                                                                             \
        if (_e != hipSuccess) return api_fail(SBMDS_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

#define IRB(expr)                                                                                           \
    do {                                                                                                    \
        rocblas_status _e = (expr);                                                                         \
        if (_e != rocblas_status_success)                                                                   \
            return api_fail(SBMDS_EHIP, std::string(#expr) + ": " + rocblas_status_to_string(_e));          \
    } while (0)

// Device memory of the call, freed in one place.
struct Pool {
    std::vector<void *> ptrs;
    ~Pool() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    T *get(size_t count, int *rc) {
        void *p = nullptr;
        if (*rc < 0) return nullptr;
        if (hipMalloc(&p, std::max<size_t>(count * sizeof(T), 16)) != hipSuccess) {
            *rc = api_fail(SBMDS_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
            return nullptr;
        }
        ptrs.push_back(p);
        return (T *)p;
    }
};

struct Handle {
    rocblas_handle h = nullptr;
    ~Handle() {
        if (h) (void)rocblas_destroy_handle(h);
    }
};

// Radix sort of (key, value) pairs with hipCUB (temporary storage from the pool).
template <typename K, typename Vv>
int sort_pairs(Pool &pool, const K *kin, K *kout, const Vv *vin, Vv *vout, int64_t count, int bits, hipStream_t s) {
    size_t bytes = 0;
    ICHK(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, kin, kout, vin, vout, (int)count, 0, bits, s));
    int rc = 0;
    void *tmp = pool.get<char>(bytes, &rc);
    if (rc < 0) return rc;
    ICHK(hipcub::DeviceRadixSort::SortPairs(tmp, bytes, kin, kout, vin, vout, (int)count, 0, bits, s));
    return SBMDS_OK;
}

int inclusive_sum(Pool &pool, const int32_t *in, int32_t *out, int64_t count, hipStream_t s) {
    size_t bytes = 0;
    ICHK(hipcub::DeviceScan::InclusiveSum(nullptr, bytes, in, out, (int)count, s));
    int rc = 0;
    void *tmp = pool.get<char>(bytes, &rc);
    if (rc < 0) return rc;
    ICHK(hipcub::DeviceScan::InclusiveSum(tmp, bytes, in, out, (int)count, s));
    return SBMDS_OK;
}

__global__ void k_iota(int32_t *p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = (int32_t)i;
}

__global__ void k_gather(const double *a, const int32_t *q, double *b, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) b[i] = a[q[i]];
}

__global__ void k_fill_d(double *x, int64_t count, double v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) x[i] = v;
}

__global__ void k_dec(int32_t *x, int64_t count) {  // inclusive -> exclusive counts of flagged items
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) x[i] -= 1;
}

__global__ void k_seg_offsets(int32_t *o, int64_t segs, int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i <= segs) o[i] = (int32_t)(i * len);
}

int bits_for(int64_t maxval) {
    int b = 1;
    while (b < 63 && (((int64_t)1 << b) <= maxval)) ++b;
    return b;
}

int interp_impl(const double *V_in, int64_t n, const int32_t *F_in, int64_t nf, const int32_t *lm_in, int64_t l,
                int64_t p, int graph, int32_t *rowptr, int32_t *col, double *val, int64_t cap, int64_t *nnz_out,
                int mem, hipStream_t s) {
    const bool host = mem == SBMDS_MEM_HOST;
    const int64_t m = n - l;
    {
        size_t free_b = 0, tot_b = 0;
        ICHK(hipMemGetInfo(&free_b, &tot_b));
        const double need = 8.0 * (double)n * (double)n + 16.0 * (double)m * (double)l + 64.0 * (double)nf;
        if (need > 0.8 * (double)free_b)
            return api_fail(SBMDS_ENOMEM, "the dense route needs about " + std::to_string((int64_t)need) + " bytes");
    }
    Pool pool;
    int rc = 0;
    const double *V = V_in;
    const int32_t *F = F_in, *lm = lm_in;
    if (host) {
        double *a = pool.get<double>(3 * n, &rc);
        int32_t *b = pool.get<int32_t>(3 * nf, &rc);
        int32_t *c = pool.get<int32_t>(l, &rc);
        if (rc < 0) return rc;
        ICHK(hipMemcpyAsync(a, V_in, 3 * n * 8, hipMemcpyHostToDevice, s));
        ICHK(hipMemcpyAsync(b, F_in, 3 * nf * 4, hipMemcpyHostToDevice, s));
        ICHK(hipMemcpyAsync(c, lm_in, l * 4, hipMemcpyHostToDevice, s));
        V = a;
        F = b;
        lm = c;
    }
    int32_t *mark = pool.get<int32_t>(n, &rc);
    int *derr = pool.get<int>(1, &rc);
    if (rc < 0) return rc;
    ICHK(hipMemsetAsync(mark, 0, n * 4, s));
    int herr = 1 << 30;
    ICHK(hipMemcpyAsync(derr, &herr, 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_in_check, dim3(nb(std::max({n, nf, l}))), dim3(256), 0, s, V, n, F, nf, lm, l, mark, derr);
    ICHK(hipGetLastError());
    ICHK(hipMemcpyAsync(&herr, derr, 4, hipMemcpyDeviceToHost, s));
    ICHK(hipStreamSynchronize(s));
    static const char *what[] = {"", "a face has an index out of range or a repeated vertex",
                                 "a landmark is out of range", "a landmark is repeated", "a coordinate is not finite"};
    if (herr != (1 << 30)) return api_fail(SBMDS_EINVAL, what[herr]);

    // 1. corners -> edges and masses
    const int64_t nc = 3 * nf;
    int64_t *ekey = pool.get<int64_t>(nc, &rc), *ekey2 = pool.get<int64_t>(nc, &rc);
    int64_t *mkey = pool.get<int64_t>(nc, &rc), *mkey2 = pool.get<int64_t>(nc, &rc);
    double *ehalf = pool.get<double>(nc, &rc), *marea = pool.get<double>(nc, &rc);
    double *sval = pool.get<double>(nc, &rc);
    int32_t *ids = pool.get<int32_t>(nc, &rc), *ids2 = pool.get<int32_t>(nc, &rc);
    int32_t *head = pool.get<int32_t>(nc, &rc), *segid = pool.get<int32_t>(nc, &rc);
    double *d = pool.get<double>(n, &rc);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(k_corners, dim3(nb(nf)), dim3(256), 0, s, V, F, nf, n, graph, ekey, ehalf, mkey, marea);
    hipLaunchKernelGGL(k_iota, dim3(nb(nc)), dim3(256), 0, s, ids, nc);
    ICHK(hipGetLastError());
    // edge records sorted by key, stable (corner order within an edge)
    if ((rc = sort_pairs(pool, ekey, ekey2, ids, ids2, nc, bits_for(n * n), s)) < 0) return rc;
    // gather the values in sorted order
    auto gather = [&](const double *src, const int32_t *perm, double *dst, int64_t count) {
        hipLaunchKernelGGL(k_gather, dim3(nb(count)), dim3(256), 0, s, src, perm, dst, count);
    };
    gather(ehalf, ids2, sval, nc);
    hipLaunchKernelGGL(k_heads, dim3(nb(nc)), dim3(256), 0, s, (const int64_t *)ekey2, nc, (int64_t)1, head);
    ICHK(hipGetLastError());
    if ((rc = inclusive_sum(pool, head, segid, nc, s)) < 0) return rc;
    int32_t hne = 0;
    ICHK(hipMemcpyAsync(&hne, segid + nc - 1, 4, hipMemcpyDeviceToHost, s));
    ICHK(hipStreamSynchronize(s));
    const int64_t ne = hne, nd = 2 * ne;  // unique edges, directed entries
    int64_t *dkey = pool.get<int64_t>(nd, &rc), *dkey2 = pool.get<int64_t>(nd, &rc);
    double *dval = pool.get<double>(nd, &rc), *dval2 = pool.get<double>(nd, &rc);
    int32_t *did = pool.get<int32_t>(nd, &rc), *did2 = pool.get<int32_t>(nd, &rc);
    int32_t *rp = pool.get<int32_t>(n + 1, &rc);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(k_edges, dim3(nb(nc)), dim3(256), 0, s, (const int64_t *)ekey2, (const double *)sval,
                       (const int32_t *)head, (const int32_t *)segid, nc, n, graph, dkey, dval);
    hipLaunchKernelGGL(k_iota, dim3(nb(nd)), dim3(256), 0, s, did, nd);
    ICHK(hipGetLastError());
    if ((rc = sort_pairs(pool, dkey, dkey2, did, did2, nd, bits_for(n * n), s)) < 0) return rc;
    gather(dval, did2, dval2, nd);
    hipLaunchKernelGGL(k_rowptr, dim3(nb(nd + 1)), dim3(256), 0, s, (const int64_t *)dkey2, nd, n, n, rp);
    // masses
    hipLaunchKernelGGL(k_iota, dim3(nb(nc)), dim3(256), 0, s, ids, nc);
    ICHK(hipGetLastError());
    if ((rc = sort_pairs(pool, mkey, mkey2, ids, ids2, nc, bits_for(3 * n * nf), s)) < 0) return rc;
    gather(marea, ids2, sval, nc);
    hipLaunchKernelGGL(k_heads, dim3(nb(nc)), dim3(256), 0, s, (const int64_t *)mkey2, nc, 3 * nf, head);
    ICHK(hipMemsetAsync(d, 0, n * 8, s));
    hipLaunchKernelGGL(k_mass, dim3(nb(nc)), dim3(256), 0, s, (const int64_t *)mkey2, (const double *)sval,
                       (const int32_t *)head, nc, 3 * nf, graph, d);
    ICHK(hipGetLastError());
    if (graph)  // D = I, also for vertices on no triangle
        hipLaunchKernelGGL(k_fill_d, dim3(nb(n)), dim3(256), 0, s, d, n, 1.0);

    // 2. dense M in the order [non-landmarks, landmarks]
    int32_t *uflag = pool.get<int32_t>(n, &rc), *urank = pool.get<int32_t>(n, &rc);
    int32_t *pos = pool.get<int32_t>(n, &rc), *uvert = pool.get<int32_t>(std::max<int64_t>(m, 1), &rc);
    double *Md = pool.get<double>((size_t)n * n, &rc);
    double *X = pool.get<double>((size_t)m * l, &rc);
    int *info = pool.get<int>(1, &rc);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(k_uflag, dim3(nb(n)), dim3(256), 0, s, (const int32_t *)mark, n, uflag);
    ICHK(hipGetLastError());
    if ((rc = inclusive_sum(pool, uflag, urank, n, s)) < 0) return rc;
    hipLaunchKernelGGL(k_dec, dim3(nb(n)), dim3(256), 0, s, urank, n);
    hipLaunchKernelGGL(k_positions, dim3(nb(n)), dim3(256), 0, s, (const int32_t *)uflag, (const int32_t *)urank,
                       lm, n, l, m, pos, uvert);
    ICHK(hipMemsetAsync(Md, 0, (size_t)n * n * 8, s));
    hipLaunchKernelGGL(k_dense_m, dim3(nb(n)), dim3(256), 0, s, (const int32_t *)rp, (const int64_t *)dkey2,
                       (const double *)dval2, (const double *)d, (const int32_t *)pos, n, Md);
    ICHK(hipGetLastError());

    // 3. P_u = -M_uu^-1 M_ub
    hipLaunchKernelGGL(k_rhs, dim3(nb(m), (unsigned)l), dim3(256), 0, s, (const double *)Md, n, m, l, X);
    ICHK(hipGetLastError());
    Handle hd;
    IRB(rocblas_create_handle(&hd.h));
    IRB(rocblas_set_stream(hd.h, s));
    IRB(rocsolver_dpotrf(hd.h, rocblas_fill_lower, (int)m, Md, (int)n, info));
    int hinfo = 0;
    ICHK(hipMemcpyAsync(&hinfo, info, 4, hipMemcpyDeviceToHost, s));
    ICHK(hipStreamSynchronize(s));
    if (hinfo != 0) return api_fail(SBMDS_EBREAKDOWN, "M_uu is not positive definite (Cholesky pivot " +
                                                          std::to_string(hinfo) + ")");
    IRB(rocsolver_dpotrs(hd.h, rocblas_fill_lower, (int)m, (int)l, Md, (int)n, X, (int)m));

    // 4. thresholding: per column the p largest magnitudes (segmented sort)
    const int64_t mlc = m * l;
    uint64_t *mk = pool.get<uint64_t>(mlc, &rc), *mk2 = pool.get<uint64_t>(mlc, &rc);
    int32_t *mi = pool.get<int32_t>(mlc, &rc), *mi2 = pool.get<int32_t>(mlc, &rc);
    int32_t *flag = pool.get<int32_t>(mlc, &rc), *slot = pool.get<int32_t>(mlc, &rc);
    int32_t *offs = pool.get<int32_t>(l + 1, &rc);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(k_mag_keys, dim3(nb(mlc)), dim3(256), 0, s, (const double *)X, mlc, mk, mi, m);
    hipLaunchKernelGGL(k_seg_offsets, dim3(nb(l + 1)), dim3(256), 0, s, offs, l, m);
    ICHK(hipGetLastError());
    {
        size_t bytes = 0;
        ICHK(hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, bytes, mk, mk2, mi, mi2, (int)mlc, (int)l, offs,
                                                         offs + 1, 0, 64, s));
        void *tmp = pool.get<char>(bytes, &rc);
        if (rc < 0) return rc;
        ICHK(hipcub::DeviceSegmentedRadixSort::SortPairs(tmp, bytes, mk, mk2, mi, mi2, (int)mlc, (int)l, offs,
                                                         offs + 1, 0, 64, s));
    }
    ICHK(hipMemsetAsync(flag, 0, mlc * 4, s));
    const int64_t pk = (p <= 0 || p >= m) ? 0 : p;  // 0: keep every nonzero
    hipLaunchKernelGGL(k_keep, dim3(nb(mlc)), dim3(256), 0, s, (const uint64_t *)mk2, (const int32_t *)mi2, m, l, pk,
                       flag);
    ICHK(hipGetLastError());
    if ((rc = inclusive_sum(pool, flag, slot, mlc, s)) < 0) return rc;
    int32_t hk = 0;
    ICHK(hipMemcpyAsync(&hk, slot + mlc - 1, 4, hipMemcpyDeviceToHost, s));
    ICHK(hipStreamSynchronize(s));
    const int64_t nkept = hk, total = nkept + l;
    *nnz_out = total;
    if (total > cap) return api_fail(SBMDS_EINVAL, "cap is below the number of entries of P (" +
                                                       std::to_string(total) + ", returned in *nnz)");
    hipLaunchKernelGGL(k_dec, dim3(nb(mlc)), dim3(256), 0, s, slot, mlc);

    // 5. CSR of P
    int64_t *pkey = pool.get<int64_t>(total, &rc), *pkey2 = pool.get<int64_t>(total, &rc);
    double *pval = pool.get<double>(total, &rc);
    int32_t *pid = pool.get<int32_t>(total, &rc), *pid2 = pool.get<int32_t>(total, &rc);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(k_entries, dim3(nb(std::max(mlc, l))), dim3(256), 0, s, (const double *)X,
                       (const int32_t *)flag, (const int32_t *)slot, (const int32_t *)uvert, lm, m, l, nkept, pkey,
                       pval);
    hipLaunchKernelGGL(k_iota, dim3(nb(total)), dim3(256), 0, s, pid, total);
    ICHK(hipGetLastError());
    if ((rc = sort_pairs(pool, pkey, pkey2, pid, pid2, total, bits_for(n * l), s)) < 0) return rc;
    int32_t *drp = rowptr, *dcol = col;
    double *dv = val;
    if (host) {
        drp = pool.get<int32_t>(n + 1, &rc);
        dcol = pool.get<int32_t>(total, &rc);
        dv = pool.get<double>(total, &rc);
        if (rc < 0) return rc;
    }
    hipLaunchKernelGGL(k_rowptr, dim3(nb(total + 1)), dim3(256), 0, s, (const int64_t *)pkey2, total, l, n, drp);
    hipLaunchKernelGGL(k_csr_out, dim3(nb(total)), dim3(256), 0, s, (const int64_t *)pkey2, (const double *)pval,
                       (const int32_t *)pid2, total, l, dcol, dv);
    ICHK(hipGetLastError());
    if (host) {
        ICHK(hipMemcpyAsync(rowptr, drp, (n + 1) * 4, hipMemcpyDeviceToHost, s));
        ICHK(hipMemcpyAsync(col, dcol, total * 4, hipMemcpyDeviceToHost, s));
        ICHK(hipMemcpyAsync(val, dv, total * 8, hipMemcpyDeviceToHost, s));
    }
    ICHK(hipStreamSynchronize(s));
    return SBMDS_OK;
}

}  // namespace
}  // namespace sbmds

extern "C" int sbmds_interpolation(const double *V, int64_t n, const int32_t *F, int64_t nf,
                                   const int32_t *landmarks, int64_t l, int64_t p, int graph, int32_t *rowptr,
                                   int32_t *col, double *val, int64_t cap, int64_t *nnz, int mem, void *stream) {
    using namespace sbmds;
    api_clear_error();
    if (!V || !F || !landmarks || !rowptr || !col || !val || !nnz)
        return api_fail(SBMDS_EINVAL, "V, F, landmarks, rowptr, col, val and nnz must be non-NULL");
    if (mem != SBMDS_MEM_HOST && mem != SBMDS_MEM_DEVICE) return api_fail(SBMDS_EINVAL, "mem must be 0 or 1");
    if (n < 2 || n > kInterpMaxN) return api_fail(SBMDS_EINVAL, "need 2 <= n <= 46340 for the dense route");
    if (nf < 1 || nf > ((int64_t)1 << 28)) return api_fail(SBMDS_EINVAL, "need 1 <= nf <= 2^28");
    if (l < 1 || l >= n) return api_fail(SBMDS_EINVAL, "need 1 <= l < n");
    *nnz = 0;
    try {
        return interp_impl(V, n, F, nf, landmarks, l, p, graph ? 1 : 0, rowptr, col, val, cap, nnz, mem,
                           (hipStream_t)stream);
    } catch (const std::exception &e) {
        return api_fail(SBMDS_ENOMEM, std::string("host exception: ") + e.what());
    }
}
