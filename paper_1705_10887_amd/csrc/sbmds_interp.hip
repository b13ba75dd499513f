// The interpolation operator P of Eq. (PDefinition) built on the device
// from a triangle mesh and its landmarks (Sections 2.2, 3.1):
//   1. the cotangent weights A_ij = (cot alpha_ij + cot beta_ij) / 2 of every
//      edge and the lumped mass d_i (a third of the area of the triangles at
//      i), or, for the generic-graph variant, A the 0/1 edge adjacency and
//      D = I;  L = diag(A 1) - A;
//   2. M = L^T D^-1 L, written densely in the order [non-landmarks,
//      landmarks]: M_uu and M_ub are then its two leading blocks;
//   3. P_u = -M_uu^-1 M_ub by a Cholesky factorisation and two triangular
//      solves: either dense (rocSOLVER, the l right-hand sides at once), or
//      blocked: breadth-first levels of the mesh make M_uu block
//      tridiagonal, whose factor is computed block by block and applied
//      to batches of right-hand sides (rocSOLVER / rocBLAS on the blocks);
//   4. the thresholding of Section 3.1: in every column the p entries of
//      largest magnitude (ties at the cut to the lower vertex, exact zeros
//      never kept), by a segmented radix sort of the magnitudes (dense
//      route) or a radix selection per column (blocked route);
//   5. the CSR of P with the identity rows of the landmarks.
// Edges and per-vertex sums come from radix sorts and segmented sums in a
// fixed order, so the result is bitwise reproducible.  The dense route costs
// 8 n^2 bytes and O(n^3) flops: it serves meshes up to a few ten thousand
// vertices.  The blocked route costs 8 n w bytes and O(n w^2 + n w l) flops
// for blocks of about w vertices (two breadth-first levels): on a mesh
// shaped like a torus or a sphere w grows like the square root of n.
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

constexpr int64_t kInterpMaxN = 46340;     // n^2 < 2^31 elements in the dense M
constexpr int64_t kInterpDenseAuto = 4096;  // larger meshes take the blocked route by default

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

// ---- the level-blocked route ----
// Breadth-first levels of the edge graph order the non-landmarks so that
// M_uu is block tridiagonal: M couples vertices at most two edges apart, so
// with blocks made of whole pairs of consecutive levels only neighbouring
// blocks couple.  Its Cholesky factor keeps that shape (fill stays inside
// the diagonal blocks and the blocks below them), which is what the
// factorisation and the triangular solves below work on.

// One breadth-first level: every vertex of the frontier labels its unlabelled
// neighbours with `label` and appends them to the next frontier.  Levels are
// unique, so the labels do not depend on the order of the appends.
__global__ __launch_bounds__(256) void k_bfs_step(const int32_t *__restrict__ rp, const int64_t *__restrict__ dkey,
                                                  int64_t n, int32_t *__restrict__ lev,
                                                  const int32_t *__restrict__ fin, const int32_t *__restrict__ cin,
                                                  int32_t *__restrict__ fout, int32_t *__restrict__ cout,
                                                  int32_t label) {
    const int64_t count = *cin;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < count; t += (int64_t)gridDim.x * 256) {
        const int32_t v = fin[t];
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int32_t u = (int32_t)(dkey[e] % n);
            if (__hip_atomic_load(&lev[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != -1) continue;
            if (atomicCAS(&lev[u], -1, label) == -1) fout[atomicAdd(cout, 1)] = u;
        }
    }
}

__global__ void k_bfs_seed(int32_t *lev, int32_t *front, int32_t *cnt, int32_t v, int32_t label) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        lev[v] = label;
        front[0] = v;
        cnt[0] = 1;
    }
}

// Smallest vertex of a frontier, and smallest vertex not yet labelled.
__global__ __launch_bounds__(256) void k_front_min(const int32_t *__restrict__ front, const int32_t *__restrict__ cnt,
                                                   int32_t *__restrict__ out) {
    const int64_t count = *cnt;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < count; t += (int64_t)gridDim.x * 256)
        atomicMin(out, front[t]);
}

__global__ __launch_bounds__(256) void k_unlabelled_min(const int32_t *__restrict__ lev, int64_t n,
                                                        int32_t *__restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v < n && lev[v] == -1) atomicMin(out, (int32_t)v);
}

__global__ void k_fill_i(int32_t *x, int64_t count, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) x[i] = v;
}

__global__ void k_fill_l(int64_t *x, int64_t count, int64_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) x[i] = v;
}

// Non-landmarks per group of two consecutive levels.
__global__ __launch_bounds__(256) void k_group_count(const int32_t *__restrict__ lev, const int32_t *__restrict__ uflag,
                                                     int64_t n, int32_t *__restrict__ gcnt) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v < n && uflag[v]) atomicAdd(&gcnt[lev[v] >> 1], 1);
}

// Sort key of the position order: (block, vertex) for non-landmarks, the
// landmarks after every block.  blk[v] is the block of a non-landmark.
__global__ __launch_bounds__(256) void k_block_keys(const int32_t *__restrict__ lev, const int32_t *__restrict__ uflag,
                                                    const int32_t *__restrict__ gblk, int64_t n, int64_t nblk,
                                                    int64_t *__restrict__ key, int32_t *__restrict__ ids,
                                                    int32_t *__restrict__ blk) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const int64_t b = uflag[v] ? gblk[lev[v] >> 1] : nblk;
    blk[v] = (int32_t)b;
    key[v] = b * n + v;
    ids[v] = (int32_t)v;
}

__global__ __launch_bounds__(256) void k_block_pos(const int32_t *__restrict__ order, int64_t m,
                                                   int32_t *__restrict__ bpos) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) bpos[order[i]] = (int32_t)i;
}

// Landmarks in the order of their level groups' blocks (key = block * l +
// landmark): a batch of consecutive landmarks in this order has right-hand
// sides that vanish above its first block, where the forward solve starts.
__global__ __launch_bounds__(256) void k_lm_keys(const int32_t *__restrict__ lm, const int32_t *__restrict__ lev,
                                                 const int32_t *__restrict__ gblk, int64_t l, int64_t nblk,
                                                 int64_t *__restrict__ key, int32_t *__restrict__ ids) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= l) return;
    const int64_t b = std::min<int64_t>(gblk[lev[lm[c]] >> 1], nblk - 1);
    key[c] = b * l + c;
    ids[c] = (int32_t)c;
}

// lmidx[v] = rank of landmark vertex v in the processing order (-1 else).
__global__ __launch_bounds__(256) void k_lm_index(const int32_t *__restrict__ lm, const int32_t *__restrict__ lmorder,
                                                  int64_t l, int32_t *__restrict__ lmidx) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q < l) lmidx[lm[lmorder[q]]] = (int32_t)q;
}

// Layout of the blocked M_uu: block b holds positions [boff[b], boff[b+1]);
// its diagonal block D_b (s_b x s_b, column-major) starts at doff[b], the
// block E_b below it (s_{b+1} x s_b, rows of block b+1) at eoff[b].
struct BlockMap {
    const int32_t *blk, *bpos, *uflag, *lmidx;
    const int32_t *boff;
    const int64_t *doff, *eoff;
};

// Entries of L's row r in ascending column order, as (column, value) to fn:
// the diagonal deg_r (the sum of the row's weights) goes between the
// neighbours below and above r.
template <typename Fn>
__device__ inline void l_row(const int32_t *__restrict__ rp, const int64_t *__restrict__ dkey,
                             const double *__restrict__ dval, int64_t n, int64_t r, Fn &&fn) {
    double dg = 0.0;
    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) dg += dval[e];
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
}

// M_uu into its blocks (lower part: D_b and E_{b-1}): thread i owns row i of
// M, M_ij = sum over k of (L_ki / d_k) L_kj in ascending k, the same sums in
// the same order as the dense route.
__global__ __launch_bounds__(256) void k_block_m(const int32_t *__restrict__ rp, const int64_t *__restrict__ dkey,
                                                 const double *__restrict__ dval, const double *__restrict__ d,
                                                 BlockMap bm, int64_t n, double *__restrict__ Mb,
                                                 int *__restrict__ err) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n || !bm.uflag[i]) return;
    const int32_t b = bm.blk[i];
    const int64_t s = bm.boff[b + 1] - bm.boff[b];
    const int64_t li = bm.bpos[i] - bm.boff[b];
    l_row(rp, dkey, dval, n, i, [&](int64_t k, double lik) {
        const double coef = lik * (1.0 / d[k]);
        l_row(rp, dkey, dval, n, k, [&](int64_t j, double lkj) {
            if (!bm.uflag[j]) return;
            const int32_t bj = bm.blk[j];
            const int64_t lj = bm.bpos[j] - bm.boff[bj];
            double *x;
            if (bj == b) x = Mb + bm.doff[b] + li + lj * s;
            else if (bj == b - 1) x = Mb + bm.eoff[bj] + li + lj * s;  // E_{b-1} has s_b rows
            else {
                if (bj != b + 1) atomicOr(err, 1);  // not block tridiagonal
                return;
            }
            *x = *x + coef * lkj;
        });
    });
}

// Right-hand sides -M_ub for the landmarks of ranks [c0, c0 + r) in the
// processing order, column-major (m x r) in position order; the same sums
// as the dense route, negated.
__global__ __launch_bounds__(256) void k_block_rhs(const int32_t *__restrict__ rp, const int64_t *__restrict__ dkey,
                                                   const double *__restrict__ dval, const double *__restrict__ d,
                                                   BlockMap bm, int64_t n, int64_t m, int64_t c0, int64_t r,
                                                   double *__restrict__ X) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n || !bm.uflag[i]) return;
    double *row = X + bm.bpos[i];
    l_row(rp, dkey, dval, n, i, [&](int64_t k, double lik) {
        const double coef = lik * (1.0 / d[k]);
        l_row(rp, dkey, dval, n, k, [&](int64_t j, double lkj) {
            const int64_t c = bm.lmidx[j] - c0;
            if (bm.lmidx[j] < 0 || c < 0 || c >= r) return;
            double *x = row + c * m;
            *x = *x - coef * lkj;
        });
    });
}

// Solution columns from position order to ascending vertex order of the
// non-landmarks (uvert[q] is the q-th non-landmark).
__global__ __launch_bounds__(256) void k_unpermute(const double *__restrict__ X, const int32_t *__restrict__ uvert,
                                                   const int32_t *__restrict__ bpos, int64_t m,
                                                   double *__restrict__ Xv) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (q < m) Xv[c * m + q] = X[c * m + bpos[uvert[q]]];
}

__device__ inline uint64_t mag_bits(double v) { return (uint64_t)__double_as_longlong(fabs(v)); }

// Sum over the 256 threads of a workgroup (4 waves).
__device__ inline int64_t wg_sum(int64_t v, int64_t *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

// Thresholding of Section 3.1 for one column per workgroup (column
// lmorder[c0 + c] of P, m values in ascending vertex order): the pk entries of largest
// magnitude, ties at the cut to the lower vertex, zeros never kept.  The
// cut is found by a radix selection over the magnitude bits (8 passes of 8
// bits); kept entries of column j go to slots [j pk, (j + 1) pk) in any
// order, with key = vertex * l + j, and cnt[j] their number.
__global__ __launch_bounds__(256) void k_topp(const double *__restrict__ Xv, int64_t m, int64_t pk, int64_t c0,
                                              int64_t l, const int32_t *__restrict__ uvert,
                                              const int32_t *__restrict__ lmorder, int64_t *__restrict__ okey,
                                              double *__restrict__ oval, int32_t *__restrict__ ocnt) {
    __shared__ uint32_t hist[256];
    __shared__ int64_t sh[4];
    __shared__ uint64_t sh_prefix;
    __shared__ int64_t sh_need, sh_eq;
    __shared__ uint32_t slot;
    __shared__ uint32_t wtot[4];
    const int64_t c = blockIdx.x, col = lmorder[c0 + c];
    const double *x = Xv + c * m;
    const int tid = threadIdx.x;
    int64_t nzl = 0;
    for (int64_t i = tid; i < m; i += 256) nzl += x[i] != 0.0;
    const int64_t nz = wg_sum(nzl, sh);
    uint64_t t = 0;
    int64_t need = 0, eq = 0;
    const bool all_nz = nz <= pk;
    if (!all_nz) {
        uint64_t prefix = 0;
        int64_t k = pk;  // rank of the cut among the entries matching prefix
        for (int shift = 56; shift >= 0; shift -= 8) {
            hist[tid] = 0;
            __syncthreads();
            const uint64_t hmask = shift == 56 ? 0ull : (~0ull << (shift + 8));
            for (int64_t i = tid; i < m; i += 256) {
                const uint64_t bits = mag_bits(x[i]);
                if ((bits & hmask) == prefix) atomicAdd(&hist[(bits >> shift) & 255], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                int64_t cum = 0;
                int dgt = 255;
                for (; dgt > 0; --dgt) {
                    if (cum + (int64_t)hist[dgt] >= k) break;
                    cum += hist[dgt];
                }
                sh_need = k - cum;
                sh_prefix = prefix | ((uint64_t)dgt << shift);
                sh_eq = hist[dgt];
            }
            __syncthreads();
            prefix = sh_prefix;
            k = sh_need;
            eq = sh_eq;
            __syncthreads();
        }
        t = prefix;  // magnitude bits of the pk-th largest entry
        need = k;    // how many entries equal to it are kept
    }
    if (tid == 0) slot = 0;
    __syncthreads();
    const bool take_all_eq = !all_nz && eq == need;
    auto emit = [&](int64_t i) {
        const uint32_t s = atomicAdd(&slot, 1u);
        okey[col * pk + s] = (int64_t)uvert[i] * l + col;
        oval[col * pk + s] = x[i];
    };
    for (int64_t i = tid; i < m; i += 256) {
        const uint64_t bits = mag_bits(x[i]);
        const bool keep = all_nz ? bits != 0 : (bits > t || (take_all_eq && bits == t));
        if (keep) emit(i);
    }
    if (!all_nz && !take_all_eq) {
        // the first `need` entries equal to the cut, in ascending vertex order
        int64_t taken = 0;
        for (int64_t base = 0; base < m && taken < need; base += 256) {
            const int64_t i = base + tid;
            const bool e = i < m && mag_bits(x[i]) == t;
            const unsigned long long bal = __ballot(e);
            const int lane = tid & 63, w = tid >> 6;
            const uint32_t below = (uint32_t)__popcll(bal & ((1ull << lane) - 1));
            __syncthreads();
            if (lane == 0) wtot[w] = (uint32_t)__popcll(bal);
            __syncthreads();
            uint32_t off = 0;
            for (int q = 0; q < w; ++q) off += wtot[q];
            if (e && taken + off + below < need) emit(i);
            taken += wtot[0] + wtot[1] + wtot[2] + wtot[3];
        }
    }
    __syncthreads();
    if (tid == 0) ocnt[col] = (int32_t)slot;
}

// The landmark identity rows after the l * pk slots.
__global__ __launch_bounds__(256) void k_identity_rows(const int32_t *__restrict__ lm, int64_t l, int64_t at,
                                                       int64_t *__restrict__ okey, double *__restrict__ oval) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= l) return;
    okey[at + c] = (int64_t)lm[c] * l + c;
    oval[at + c] = 1.0;
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

constexpr int64_t kGroupMin = 64;      // non-landmarks per block at least (blocks merge level groups)
constexpr int64_t kBatchMax = 2048;    // right-hand sides per batch of the blocked route
constexpr int kBfsChunk = 8;           // breadth-first levels launched per host check

struct EdgeData {
    const int32_t *rp;
    const int64_t *dkey;
    const double *dval, *d;
};

// Entries of P (thresholded columns of P_u plus the identity rows) by the
// level-blocked route: slots = l * pk + l keys/values, of which *total are
// entries and the rest hold the key n * l (they sort last).
int blocked_entries(Pool &pool, const EdgeData &ed, int64_t n, int64_t l, int64_t m, int64_t p, const int32_t *lm,
                    const int32_t *uflag, const int32_t *uvert, int64_t *slots_out, int64_t *total_out,
                    int64_t **pkey_out, double **pval_out, hipStream_t s) {
    int rc = 0;
    const int64_t pk = (p <= 0 || p >= m) ? m : p;
    const int64_t slots = l * pk + l;
    int32_t *lev = pool.get<int32_t>(n, &rc), *fr[2] = {pool.get<int32_t>(n, &rc), pool.get<int32_t>(n, &rc)};
    int32_t *cnt = pool.get<int32_t>(n + 2 + kBfsChunk, &rc), *dmin = pool.get<int32_t>(1, &rc);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(k_fill_i, dim3(nb(n)), dim3(256), 0, s, lev, n, -1);
    ICHK(hipMemsetAsync(cnt, 0, (n + 2 + kBfsChunk) * 4, s));
    const unsigned grid = (unsigned)std::min<int64_t>(nb(n), 2048);
    // one breadth-first search from `start` labelling its component with
    // base, base + 1, ...; returns the last level (relative to base) and the
    // smallest vertex on it
    auto bfs = [&](int32_t start, int32_t base, int64_t *last, int32_t *vmin) -> int {
        hipLaunchKernelGGL(k_bfs_seed, dim3(1), dim3(64), 0, s, lev, fr[0], cnt, start, base);
        int64_t L = 0;
        for (;;) {
            for (int q = 0; q < kBfsChunk; ++q) {
                const int64_t lq = L + q;
                hipLaunchKernelGGL(k_bfs_step, dim3(grid), dim3(256), 0, s, ed.rp, ed.dkey, n, lev,
                                   (const int32_t *)fr[lq & 1], (const int32_t *)(cnt + lq), fr[(lq + 1) & 1],
                                   cnt + lq + 1, (int32_t)(base + lq + 1));
            }
            ICHK(hipGetLastError());
            int32_t h[kBfsChunk];
            ICHK(hipMemcpyAsync(h, cnt + L + 1, sizeof(h), hipMemcpyDeviceToHost, s));
            ICHK(hipStreamSynchronize(s));
            int z = 0;
            while (z < kBfsChunk && h[z] != 0) ++z;
            if (z < kBfsChunk) {
                *last = L + z;
                break;
            }
            L += kBfsChunk;
            if (L > n) return api_fail(SBMDS_EHIP, "breadth-first search did not end");
        }
        int32_t big = INT32_MAX;
        ICHK(hipMemcpyAsync(dmin, &big, 4, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_front_min, dim3(grid), dim3(256), 0, s, (const int32_t *)fr[*last & 1],
                           (const int32_t *)(cnt + *last), dmin);
        ICHK(hipMemcpyAsync(vmin, dmin, 4, hipMemcpyDeviceToHost, s));
        ICHK(hipMemsetAsync(cnt, 0, (*last + 2) * 4, s));
        ICHK(hipStreamSynchronize(s));
        return SBMDS_OK;
    };
    // levels: a second search from the far end of the first one (a
    // pseudo-peripheral start), then one search per further component
    int64_t last = 0;
    int32_t far = 0;
    if ((rc = bfs(0, 0, &last, &far)) < 0) return rc;
    hipLaunchKernelGGL(k_fill_i, dim3(nb(n)), dim3(256), 0, s, lev, n, -1);
    int32_t unused = 0;
    if ((rc = bfs(far, 0, &last, &unused)) < 0) return rc;
    int64_t maxlev = last;
    for (;;) {
        int32_t big = INT32_MAX, v = 0;
        ICHK(hipMemcpyAsync(dmin, &big, 4, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_unlabelled_min, dim3(nb(n)), dim3(256), 0, s, (const int32_t *)lev, n, dmin);
        ICHK(hipMemcpyAsync(&v, dmin, 4, hipMemcpyDeviceToHost, s));
        ICHK(hipStreamSynchronize(s));
        if (v == INT32_MAX) break;
        const int64_t base = maxlev + 2;
        if (base + n > INT32_MAX) return api_fail(SBMDS_EINVAL, "too many components for the blocked route");
        if ((rc = bfs(v, (int32_t)base, &last, &unused)) < 0) return rc;
        maxlev = base + last;
    }

    // blocks: consecutive pairs of levels, merged until a block holds at
    // least kGroupMin non-landmarks
    const int64_t ngroups = (maxlev >> 1) + 1;
    int32_t *gcnt = pool.get<int32_t>(ngroups, &rc), *gblk_d = pool.get<int32_t>(ngroups, &rc);
    if (rc < 0) return rc;
    ICHK(hipMemsetAsync(gcnt, 0, ngroups * 4, s));
    hipLaunchKernelGGL(k_group_count, dim3(nb(n)), dim3(256), 0, s, (const int32_t *)lev, uflag, n, gcnt);
    ICHK(hipGetLastError());
    std::vector<int32_t> hg(ngroups), gblk(ngroups);
    ICHK(hipMemcpyAsync(hg.data(), gcnt, ngroups * 4, hipMemcpyDeviceToHost, s));
    ICHK(hipStreamSynchronize(s));
    std::vector<int64_t> bs;
    int64_t acc = 0;
    for (int64_t g = 0; g < ngroups; ++g) {
        gblk[g] = (int32_t)bs.size();
        acc += hg[g];
        if (acc >= kGroupMin) {
            bs.push_back(acc);
            acc = 0;
        }
    }
    if (acc > 0) bs.push_back(acc);
    const int64_t nblk = (int64_t)bs.size();
    std::vector<int32_t> boff(nblk + 1, 0);
    std::vector<int64_t> doff(nblk), eoff(nblk);
    int64_t nmb = 0;  // doubles of the blocked M_uu
    for (int64_t b = 0; b < nblk; ++b) {
        boff[b + 1] = (int32_t)(boff[b] + bs[b]);
        doff[b] = nmb;
        nmb += bs[b] * bs[b];
        eoff[b] = nmb;
        if (b + 1 < nblk) nmb += bs[b + 1] * bs[b];
    }
    if (boff[nblk] != m) return api_fail(SBMDS_EHIP, "blocked route: block sizes do not add up to n - l");

    // memory: the blocked M_uu, the entry slots, two m x r batches
    int64_t r = 0;
    {
        size_t free_b = 0, tot_b = 0;
        ICHK(hipMemGetInfo(&free_b, &tot_b));
        const double fixed = 8.0 * (double)nmb + 44.0 * (double)slots + 40.0 * (double)n;
        const double avail = 0.8 * (double)free_b - fixed;
        r = std::min<int64_t>({l, kBatchMax, avail > 0 ? (int64_t)(avail / (16.0 * (double)m)) : 0});
        if (r < 1)
            return api_fail(SBMDS_ENOMEM, "the blocked route needs more than " + std::to_string((int64_t)fixed) +
                                              " bytes (largest block " +
                                              std::to_string(*std::max_element(bs.begin(), bs.end())) + ")");
    }

    // positions: (block, vertex) order of the non-landmarks
    int64_t *key = pool.get<int64_t>(n, &rc), *key2 = pool.get<int64_t>(n, &rc);
    int32_t *ids = pool.get<int32_t>(n, &rc), *order = pool.get<int32_t>(n, &rc);
    int32_t *blk = pool.get<int32_t>(n, &rc), *bpos = pool.get<int32_t>(n, &rc), *lmidx = pool.get<int32_t>(n, &rc);
    int32_t *boff_d = pool.get<int32_t>(nblk + 1, &rc);
    int64_t *doff_d = pool.get<int64_t>(nblk, &rc), *eoff_d = pool.get<int64_t>(nblk, &rc);
    int *err = pool.get<int>(1, &rc), *info = pool.get<int>(nblk, &rc);
    double *Mb = pool.get<double>(nmb, &rc);
    if (rc < 0) return rc;
    ICHK(hipMemcpyAsync(gblk_d, gblk.data(), ngroups * 4, hipMemcpyHostToDevice, s));
    ICHK(hipMemcpyAsync(boff_d, boff.data(), (nblk + 1) * 4, hipMemcpyHostToDevice, s));
    ICHK(hipMemcpyAsync(doff_d, doff.data(), nblk * 8, hipMemcpyHostToDevice, s));
    ICHK(hipMemcpyAsync(eoff_d, eoff.data(), nblk * 8, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_block_keys, dim3(nb(n)), dim3(256), 0, s, (const int32_t *)lev, uflag,
                       (const int32_t *)gblk_d, n, nblk, key, ids, blk);
    ICHK(hipGetLastError());
    if ((rc = sort_pairs(pool, key, key2, ids, order, n, bits_for((nblk + 1) * n), s)) < 0) return rc;
    hipLaunchKernelGGL(k_block_pos, dim3(nb(m)), dim3(256), 0, s, (const int32_t *)order, m, bpos);
    // landmarks in block order (ranks in lmidx, first block of each batch)
    int64_t *lkey = pool.get<int64_t>(l, &rc), *lkey2 = pool.get<int64_t>(l, &rc);
    int32_t *lids = pool.get<int32_t>(l, &rc), *lmorder = pool.get<int32_t>(l, &rc);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(k_lm_keys, dim3(nb(l)), dim3(256), 0, s, lm, (const int32_t *)lev, (const int32_t *)gblk_d, l,
                       nblk, lkey, lids);
    ICHK(hipGetLastError());
    if ((rc = sort_pairs(pool, lkey, lkey2, lids, lmorder, l, bits_for(nblk * l), s)) < 0) return rc;
    hipLaunchKernelGGL(k_fill_i, dim3(nb(n)), dim3(256), 0, s, lmidx, n, -1);
    hipLaunchKernelGGL(k_lm_index, dim3(nb(l)), dim3(256), 0, s, lm, (const int32_t *)lmorder, l, lmidx);
    ICHK(hipGetLastError());
    std::vector<int64_t> hlkey(l);
    ICHK(hipMemcpyAsync(hlkey.data(), lkey2, l * 8, hipMemcpyDeviceToHost, s));
    const BlockMap bm{blk, bpos, uflag, lmidx, boff_d, doff_d, eoff_d};

    // M_uu in blocks
    ICHK(hipMemsetAsync(Mb, 0, (size_t)nmb * 8, s));
    ICHK(hipMemsetAsync(err, 0, 4, s));
    hipLaunchKernelGGL(k_block_m, dim3(nb(n)), dim3(256), 0, s, ed.rp, ed.dkey, ed.dval, ed.d, bm, n, Mb, err);
    ICHK(hipGetLastError());
    int herr = 0;
    ICHK(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s));
    ICHK(hipStreamSynchronize(s));
    if (herr) return api_fail(SBMDS_EHIP, "blocked route: M_uu is not block tridiagonal in the level order");

    // Block Cholesky from both ends ("twisted"): the blocks above the
    // meeting block k are eliminated downwards and the blocks below it
    // upwards; block k takes the Schur complements of both and is
    // eliminated last.
    //   top, b < k:     D_b -= E_{b-1} E_{b-1}^T, D_b = L_bb L_bb^T,
    //                   E_b <- E_b L_bb^-T
    //   bottom, b > k:  D_b -= H_b^T H_b, D_b = L_bb L_bb^T,
    //                   E_{b-1} <- H_{b-1} = L_bb^-1 E_{b-1}
    //   k:              D_k -= E_{k-1} E_{k-1}^T + H_k^T H_k, D_k = L_kk L_kk^T
    // (E_b, rows of block b+1 by columns of block b, holds its top or bottom
    // form in place.)  k splits sum s_b^2 in halves.  Eliminating from both
    // ends lets a batch's forward solve cover only the blocks between its
    // first and last landmark: the right-hand sides, and so the forward
    // solution, vanish on both chain ends outside them.  The two chains are
    // independent; they run one after the other on the caller's stream.
    int64_t kmid = 0;
    {
        double tot = 0.0, run = 0.0;
        for (int64_t b = 0; b < nblk; ++b) tot += (double)bs[b] * (double)bs[b];
        while (kmid + 1 < nblk && run + (double)bs[kmid] * (double)bs[kmid] < 0.5 * tot)
            run += (double)bs[kmid] * (double)bs[kmid], ++kmid;
    }
    Handle hd;
    IRB(rocblas_create_handle(&hd.h));
    IRB(rocblas_set_stream(hd.h, s));
    const double one = 1.0, mone = -1.0;
    auto sz = [&](int64_t b) { return (int)bs[b]; };
    auto Dp = [&](int64_t b) { return Mb + doff[b]; };
    auto Ep = [&](int64_t b) { return Mb + eoff[b]; };
    // D -= A^T A for A (k x n, lda k): the lower triangle of D is what the
    // factorisation reads
    auto sub_ata = [&](rocblas_handle h, double *D, int nn, const double *A, int kk) {
        return rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_transpose, nn, kk, &mone, A, kk, &one, D, nn);
    };
    ICHK(hipMemsetAsync(info, 0, nblk * 4, s));
    for (int64_t b = 0; b < kmid; ++b) {
        if (b > 0)
            IRB(rocblas_dsyrk(hd.h, rocblas_fill_lower, rocblas_operation_none, sz(b), sz(b - 1), &mone, Ep(b - 1),
                              sz(b), &one, Dp(b), sz(b)));
        IRB(rocsolver_dpotrf(hd.h, rocblas_fill_lower, sz(b), Dp(b), sz(b), info + b));
        IRB(rocblas_dtrsm(hd.h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                          rocblas_diagonal_non_unit, sz(b + 1), sz(b), &one, Dp(b), sz(b), Ep(b), sz(b + 1)));
    }
    for (int64_t b = nblk - 1; b > kmid; --b) {
        if (b + 1 < nblk) IRB(sub_ata(hd.h, Dp(b), sz(b), Ep(b), sz(b + 1)));
        IRB(rocsolver_dpotrf(hd.h, rocblas_fill_lower, sz(b), Dp(b), sz(b), info + b));
        IRB(rocblas_dtrsm(hd.h, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                          rocblas_diagonal_non_unit, sz(b), sz(b - 1), &one, Dp(b), sz(b), Ep(b - 1), sz(b)));
    }
    if (kmid > 0)
        IRB(rocblas_dsyrk(hd.h, rocblas_fill_lower, rocblas_operation_none, sz(kmid), sz(kmid - 1), &mone,
                          Ep(kmid - 1), sz(kmid), &one, Dp(kmid), sz(kmid)));
    if (kmid + 1 < nblk) IRB(sub_ata(hd.h, Dp(kmid), sz(kmid), Ep(kmid), sz(kmid + 1)));
    IRB(rocsolver_dpotrf(hd.h, rocblas_fill_lower, sz(kmid), Dp(kmid), sz(kmid), info + kmid));
    {
        std::vector<int> hi(nblk);
        ICHK(hipMemcpyAsync(hi.data(), info, nblk * 4, hipMemcpyDeviceToHost, s));
        ICHK(hipStreamSynchronize(s));
        for (int64_t b = 0; b < nblk; ++b)
            if (hi[b] != 0)
                return api_fail(SBMDS_EBREAKDOWN, "M_uu is not positive definite (block " + std::to_string(b) +
                                                      ", pivot " + std::to_string(hi[b]) + ")");
    }

    // right-hand sides in batches: solve, back to vertex order, threshold
    double *X = pool.get<double>((size_t)m * r, &rc), *Xv = pool.get<double>((size_t)m * r, &rc);
    int64_t *okey = pool.get<int64_t>(slots, &rc);
    double *oval = pool.get<double>(slots, &rc);
    int32_t *ocnt = pool.get<int32_t>(l, &rc);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(k_fill_l, dim3(nb(slots)), dim3(256), 0, s, okey, slots, n * l);
    ICHK(hipGetLastError());
    for (int64_t c0 = 0; c0 < l; c0 += r) {
        const int64_t rr = std::min(r, l - c0);
        const int ri = (int)rr, mi = (int)m;
        ICHK(hipMemsetAsync(X, 0, (size_t)m * rr * 8, s));
        hipLaunchKernelGGL(k_block_rhs, dim3(nb(n)), dim3(256), 0, s, ed.rp, ed.dkey, ed.dval, ed.d, bm, n, m, c0, rr,
                           X);
        ICHK(hipGetLastError());
        auto Xp = [&](int64_t b) { return X + boff[b]; };
        auto gemm = [&](rocblas_handle h, rocblas_operation ta, int64_t b, const double *A, int lda, int64_t bsrc) {
            return rocblas_dgemm(h, ta, rocblas_operation_none, sz(b), ri, sz(bsrc), &mone, A, lda, Xp(bsrc), mi,
                                 &one, Xp(b), mi);
        };
        auto trsm = [&](rocblas_handle h, rocblas_operation ta, int64_t b) {
            return rocblas_dtrsm(h, rocblas_side_left, rocblas_fill_lower, ta, rocblas_diagonal_non_unit, sz(b), ri,
                                 &one, Dp(b), sz(b), Xp(b), mi);
        };
        // L y = rhs.  The batch's landmarks lie in blocks [first, last] of
        // the level order, so its right-hand sides vanish outside
        // [first - 1, last + 1], and so does y on the chain ends before them.
        const int64_t bfirst = std::max<int64_t>(0, hlkey[c0] / l - 1);
        const int64_t blast = std::min<int64_t>(nblk - 1, hlkey[c0 + rr - 1] / l + 1);
        for (int64_t b = bfirst; b < kmid; ++b) {
            if (b > bfirst) IRB(gemm(hd.h, rocblas_operation_none, b, Ep(b - 1), sz(b), b - 1));
            IRB(trsm(hd.h, rocblas_operation_none, b));
        }
        for (int64_t b = blast; b > kmid; --b) {
            if (b < blast) IRB(gemm(hd.h, rocblas_operation_transpose, b, Ep(b), sz(b + 1), b + 1));
            IRB(trsm(hd.h, rocblas_operation_none, b));
        }
        if (kmid > 0) IRB(gemm(hd.h, rocblas_operation_none, kmid, Ep(kmid - 1), sz(kmid), kmid - 1));
        if (kmid + 1 < nblk) IRB(gemm(hd.h, rocblas_operation_transpose, kmid, Ep(kmid), sz(kmid + 1), kmid + 1));
        IRB(trsm(hd.h, rocblas_operation_none, kmid));
        // L^T x = y: block k, then both chains outwards
        IRB(trsm(hd.h, rocblas_operation_transpose, kmid));
        for (int64_t b = kmid - 1; b >= 0; --b) {
            IRB(gemm(hd.h, rocblas_operation_transpose, b, Ep(b), sz(b + 1), b + 1));
            IRB(trsm(hd.h, rocblas_operation_transpose, b));
        }
        for (int64_t b = kmid + 1; b < nblk; ++b) {
            IRB(gemm(hd.h, rocblas_operation_none, b, Ep(b - 1), sz(b), b - 1));
            IRB(trsm(hd.h, rocblas_operation_transpose, b));
        }
        hipLaunchKernelGGL(k_unpermute, dim3(nb(m), (unsigned)rr), dim3(256), 0, s, (const double *)X, uvert,
                           (const int32_t *)bpos, m, Xv);
        hipLaunchKernelGGL(k_topp, dim3((unsigned)rr), dim3(256), 0, s, (const double *)Xv, m, pk, c0, l, uvert,
                           (const int32_t *)lmorder, okey, oval, ocnt);
        ICHK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_identity_rows, dim3(nb(l)), dim3(256), 0, s, lm, l, l * pk, okey, oval);
    ICHK(hipGetLastError());
    std::vector<int32_t> hc(l);
    ICHK(hipMemcpyAsync(hc.data(), ocnt, l * 4, hipMemcpyDeviceToHost, s));
    ICHK(hipStreamSynchronize(s));
    int64_t kept = 0;
    for (int64_t c = 0; c < l; ++c) kept += hc[c];
    *slots_out = slots;
    *total_out = kept + l;
    *pkey_out = okey;
    *pval_out = oval;
    return SBMDS_OK;
}

// The CSR of P from `slots` (key = row * l + column, value) records of which
// the `total` smallest keys are its entries.
int csr_from_entries(Pool &pool, const int64_t *pkey, const double *pval, int64_t slots, int64_t total, int64_t n,
                     int64_t l, bool host, int32_t *rowptr, int32_t *col, double *val, hipStream_t s) {
    int rc = 0;
    int64_t *pkey2 = pool.get<int64_t>(slots, &rc);
    int32_t *pid = pool.get<int32_t>(slots, &rc), *pid2 = pool.get<int32_t>(slots, &rc);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(k_iota, dim3(nb(slots)), dim3(256), 0, s, pid, slots);
    ICHK(hipGetLastError());
    if ((rc = sort_pairs(pool, pkey, pkey2, (const int32_t *)pid, pid2, slots, bits_for(n * l), s)) < 0) return rc;
    int32_t *drp = rowptr, *dcol = col;
    double *dv = val;
    if (host) {
        drp = pool.get<int32_t>(n + 1, &rc);
        dcol = pool.get<int32_t>(total, &rc);
        dv = pool.get<double>(total, &rc);
        if (rc < 0) return rc;
    }
    hipLaunchKernelGGL(k_rowptr, dim3(nb(total + 1)), dim3(256), 0, s, (const int64_t *)pkey2, total, l, n, drp);
    hipLaunchKernelGGL(k_csr_out, dim3(nb(total)), dim3(256), 0, s, (const int64_t *)pkey2, pval,
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

int interp_impl(const double *V_in, int64_t n, const int32_t *F_in, int64_t nf, const int32_t *lm_in, int64_t l,
                int64_t p, int graph, bool blocked, int32_t *rowptr, int32_t *col, double *val, int64_t cap,
                int64_t *nnz_out, int mem, hipStream_t s) {
    const bool host = mem == SBMDS_MEM_HOST;
    const int64_t m = n - l;
    if (!blocked) {
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

    // non-landmarks in ascending vertex order (uvert), positions of the dense
    // order [non-landmarks, landmarks] (pos)
    int32_t *uflag = pool.get<int32_t>(n, &rc), *urank = pool.get<int32_t>(n, &rc);
    int32_t *pos = pool.get<int32_t>(n, &rc), *uvert = pool.get<int32_t>(std::max<int64_t>(m, 1), &rc);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(k_uflag, dim3(nb(n)), dim3(256), 0, s, (const int32_t *)mark, n, uflag);
    ICHK(hipGetLastError());
    if ((rc = inclusive_sum(pool, uflag, urank, n, s)) < 0) return rc;
    hipLaunchKernelGGL(k_dec, dim3(nb(n)), dim3(256), 0, s, urank, n);
    hipLaunchKernelGGL(k_positions, dim3(nb(n)), dim3(256), 0, s, (const int32_t *)uflag, (const int32_t *)urank,
                       lm, n, l, m, pos, uvert);
    ICHK(hipGetLastError());

    if (blocked) {
        const EdgeData ed{rp, dkey2, dval2, d};
        int64_t slots = 0, total = 0;
        int64_t *okey = nullptr;
        double *oval = nullptr;
        if ((rc = blocked_entries(pool, ed, n, l, m, p, lm, uflag, uvert, &slots, &total, &okey, &oval, s)) < 0)
            return rc;
        *nnz_out = total;
        if (total > cap) return api_fail(SBMDS_EINVAL, "cap is below the number of entries of P (" +
                                                           std::to_string(total) + ", returned in *nnz)");
        return csr_from_entries(pool, okey, oval, slots, total, n, l, host, rowptr, col, val, s);
    }

    // 2. dense M in the order [non-landmarks, landmarks]
    double *Md = pool.get<double>((size_t)n * n, &rc);
    double *X = pool.get<double>((size_t)m * l, &rc);
    int *info = pool.get<int>(1, &rc);
    if (rc < 0) return rc;
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
    int64_t *pkey = pool.get<int64_t>(total, &rc);
    double *pval = pool.get<double>(total, &rc);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(k_entries, dim3(nb(std::max(mlc, l))), dim3(256), 0, s, (const double *)X,
                       (const int32_t *)flag, (const int32_t *)slot, (const int32_t *)uvert, lm, m, l, nkept, pkey,
                       pval);
    ICHK(hipGetLastError());
    return csr_from_entries(pool, pkey, pval, total, total, n, l, host, rowptr, col, val, s);
}

}  // namespace
}  // namespace sbmds

extern "C" int sbmds_interpolation(const double *V, int64_t n, const int32_t *F, int64_t nf,
                                   const int32_t *landmarks, int64_t l, int64_t p, int flags, int32_t *rowptr,
                                   int32_t *col, double *val, int64_t cap, int64_t *nnz, int mem, void *stream) {
    using namespace sbmds;
    api_clear_error();
    if (!V || !F || !landmarks || !rowptr || !col || !val || !nnz)
        return api_fail(SBMDS_EINVAL, "V, F, landmarks, rowptr, col, val and nnz must be non-NULL");
    if (mem != SBMDS_MEM_HOST && mem != SBMDS_MEM_DEVICE) return api_fail(SBMDS_EINVAL, "mem must be 0 or 1");
    const unsigned known = SBMDS_INTERP_GRAPH | SBMDS_INTERP_DENSE | SBMDS_INTERP_BLOCKED;
    if ((unsigned)flags & ~known) return api_fail(SBMDS_EINVAL, "unknown bits in flags");
    if ((flags & SBMDS_INTERP_DENSE) && (flags & SBMDS_INTERP_BLOCKED))
        return api_fail(SBMDS_EINVAL, "SBMDS_INTERP_DENSE and SBMDS_INTERP_BLOCKED exclude each other");
    const bool blocked = (flags & SBMDS_INTERP_BLOCKED) || (!(flags & SBMDS_INTERP_DENSE) && n > kInterpDenseAuto);
    if (n < 2 || n > (blocked ? (int64_t)INT32_MAX / 2 : kInterpMaxN))
        return api_fail(SBMDS_EINVAL, blocked ? "need 2 <= n < 2^30 for the blocked route"
                                              : "need 2 <= n <= 46340 for the dense route");
    if (nf < 1 || nf > ((int64_t)1 << 28)) return api_fail(SBMDS_EINVAL, "need 1 <= nf <= 2^28");
    if (l < 1 || l >= n) return api_fail(SBMDS_EINVAL, "need 1 <= l < n");
    *nnz = 0;
    try {
        return interp_impl(V, n, F, nf, landmarks, l, p, (flags & SBMDS_INTERP_GRAPH) ? 1 : 0, blocked, rowptr, col,
                           val, cap, nnz, mem, (hipStream_t)stream);
    } catch (const std::exception &e) {
        return api_fail(SBMDS_ENOMEM, std::string("host exception: ") + e.what());
    }
}
