// Create-time preparation of one problem on the device: validation of
// device-resident inputs, the labels of the internal landmark order, P's
// columns relabelled into that order, the CSR of P^T, the column sums
// c = P^T 1 (the inner centering term of Section 3.3's J P W P^T J, J being
// identity minus rank one) and W permuted into that order.  Inputs never
// leave the device; only per-level landmark labels travel to the host.
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "sbmds_common.h"
#include "sbmds_prep.h"

namespace sbmds {

namespace {

// First failing check: the smallest (code, row) key wins.
__device__ __forceinline__ void flag(unsigned long long *err, int code, int64_t row) {
    const unsigned long long key = ((unsigned long long)code << 40) | (unsigned long long)(row & ((1ll << 40) - 1));
    atomicMin(err, key);
}

template <typename T>
__device__ __forceinline__ bool finite_val(T x) {
    return isfinite((double)x);
}

__global__ __launch_bounds__(256) void k_check_rowptr(const int32_t *__restrict__ rp, int64_t n, int64_t nnz,
                                                      unsigned long long *err) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0) {
        if (rp[0] != 0) flag(err, PREP_ROWPTR0, 0);
        if ((int64_t)rp[n] != nnz) flag(err, PREP_ROWPTRN, 0);
    }
    if (i < n && (rp[i + 1] < rp[i] || (int64_t)rp[i + 1] > nnz)) flag(err, PREP_ROWPTR_ORDER, i);
}

// Row entries: columns in range and strictly increasing, values finite.
// Entry ranges are clamped to [0, nnz), so malformed row pointers (reported
// by k_check_rowptr) never lead to reads out of bounds.
template <typename T>
__global__ __launch_bounds__(256) void k_check_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                    const T *__restrict__ val, int64_t n, int64_t l, int64_t nnz,
                                                    unsigned long long *err) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t e0 = max((int64_t)0, min(nnz, (int64_t)rp[i]));
    const int64_t e1 = max(e0, min(nnz, (int64_t)rp[i + 1]));
    for (int64_t e = e0; e < e1; ++e) {
        const int32_t c = ci[e];
        if (c < 0 || c >= l) {
            flag(err, PREP_COL_RANGE, i);
            return;
        }
        if (e > e0 && c <= ci[e - 1]) {
            flag(err, PREP_COL_ORDER, i);
            return;
        }
        if (!finite_val(val[e])) {
            flag(err, PREP_VAL, i);
            return;
        }
    }
}

// W finite and symmetric: block (bi, bj), bj <= bi, compares the 32 x 32
// tile (bi, bj) with the transpose of tile (bj, bi) through LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_check_w(const T *__restrict__ W, int64_t l, unsigned long long *err) {
    const int bi = blockIdx.y, bj = blockIdx.x;
    if (bj > bi) return;
    __shared__ T tt[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows per pass
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = (int64_t)bj * 32 + r, j = (int64_t)bi * 32 + tx;
        tt[r][tx] = (i < l && j < l) ? W[i * l + j] : T{};
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = (int64_t)bi * 32 + r, j = (int64_t)bj * 32 + tx;
        if (i < l && j < l) {
            const T a = W[i * l + j];
            if (!finite_val(a)) flag(err, PREP_W_FINITE, i);
            else if (a != tt[tx][r]) flag(err, PREP_W_SYM, i);
        }
    }
}

// Nearest of its cell's pivots for every landmark at position pos of the
// current order (cells listed by seg[pos] >= 0, pivots 8 per cell; landmarks
// in cells that are final get -1).  Distances compared in float64 with the
// first minimum kept.
template <typename T>
__global__ __launch_bounds__(256) void k_lmk_labels(const T *__restrict__ W, int64_t l,
                                                    const int32_t *__restrict__ order, const int32_t *__restrict__ seg,
                                                    const int32_t *__restrict__ piv, int32_t *__restrict__ label) {
    const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (pos >= l) return;
    const int s = seg[pos];
    if (s < 0) {
        label[pos] = -1;
        return;
    }
    const int64_t m = order[pos];
    int best = 0;
    double bd = (double)W[m * l + piv[8 * s]];
    for (int c = 1; c < 8; ++c) {
        const double d = (double)W[m * l + piv[8 * s + c]];
        if (d < bd) {
            bd = d;
            best = c;
        }
    }
    label[pos] = best;
}

// Sort keys of the entries: (row, internal column) for P, (internal
// column, row) for P^T; 31 + 20 bits.
__global__ __launch_bounds__(256) void k_entry_keys(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                    const int32_t *__restrict__ inv, int64_t n,
                                                    unsigned long long *__restrict__ krow,
                                                    unsigned long long *__restrict__ kcol,
                                                    int32_t *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const unsigned long long c = (unsigned long long)inv[ci[e]];
        krow[e] = ((unsigned long long)i << 20) | c;
        kcol[e] = (c << 31) | (unsigned long long)i;
        idx[e] = e;
    }
}

// Entry arrays from a sorted (key, entry index) list: the minor field of the
// key and the value of the entry.
template <typename T>
__global__ __launch_bounds__(256) void k_gather_entries(const unsigned long long *__restrict__ key,
                                                        const int32_t *__restrict__ idx, int64_t nnz,
                                                        unsigned long long mask, const T *__restrict__ val,
                                                        int32_t *__restrict__ minor, T *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nnz) return;
    minor[e] = (int32_t)(key[e] & mask);
    out[e] = val[idx[e]];
}

// Row pointers of P^T from the column-major keys: rpT[j] = first entry of
// column j (columns without entries point at the next one).
__global__ __launch_bounds__(256) void k_rowptr_t(const unsigned long long *__restrict__ kcol, int64_t nnz, int64_t l,
                                                  int32_t *__restrict__ rpT) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e > nnz) return;
    const int64_t c = e < nnz ? (int64_t)(kcol[e] >> 31) : l;
    const int64_t cp = e > 0 ? (int64_t)(kcol[e - 1] >> 31) : -1;
    for (int64_t j = cp + 1; j <= c; ++j) rpT[j] = (int32_t)e;
}

// c_j = sum of column j of P in float64, in increasing vertex order (the
// order of P^T's rows); with `bf` the values are first rounded to bfloat16.
template <typename T, bool BF>
__global__ __launch_bounds__(256) void k_colsums(const int32_t *__restrict__ rpT, const T *__restrict__ valT, int64_t l,
                                                 double *__restrict__ c) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= l) return;
    double s = 0.0;
    for (int32_t e = rpT[j]; e < rpT[j + 1]; ++e) {
        if constexpr (BF) s += (double)bf2f(f2bf((float)valT[e]));
        else s += (double)valT[e];
    }
    c[j] = s;
}

// W in the internal landmark order, rows padded to lda with zeros: block
// per internal row.
template <typename T>
__global__ __launch_bounds__(256) void k_permute_w(const T *__restrict__ W, int64_t l, int lda,
                                                   const int32_t *__restrict__ perm, T *__restrict__ out) {
    const int64_t i = blockIdx.x;
    const T *src = W + (int64_t)perm[i] * l;
    T *dst = out + i * lda;
    for (int j = threadIdx.x; j < lda; j += 256) dst[j] = j < l ? src[perm[j]] : T{};
}

inline unsigned blocks(int64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

template <typename T>
hipError_t prep_validate(const int32_t *rp, const int32_t *ci, const void *val, const void *W, int64_t n, int64_t l,
                         int64_t nnz, unsigned long long *err, hipStream_t s) {
    hipLaunchKernelGGL(k_check_rowptr, dim3(blocks(n)), dim3(256), 0, s, rp, n, nnz, err);
    hipLaunchKernelGGL((k_check_rows<T>), dim3(blocks(n)), dim3(256), 0, s, rp, ci, (const T *)val, n, l, nnz, err);
    const unsigned nt = (unsigned)((l + 31) / 32);
    hipLaunchKernelGGL((k_check_w<T>), dim3(nt, nt), dim3(256), 0, s, (const T *)W, l, err);
    return hipGetLastError();
}

template <typename T>
hipError_t prep_labels(const void *W, int64_t l, const int32_t *order, const int32_t *seg, const int32_t *piv,
                       int32_t *label, hipStream_t s) {
    hipLaunchKernelGGL((k_lmk_labels<T>), dim3(blocks(l)), dim3(256), 0, s, (const T *)W, l, order, seg, piv, label);
    return hipGetLastError();
}

template <typename T>
hipError_t prep_operator(const PrepIn &in, const PrepOut &out, void *tmp, size_t tmp_bytes, hipStream_t s) {
    const int64_t n = in.n, l = in.l, nnz = in.nnz;
    // scratch: two key arrays, two index arrays, the sort's work area
    char *t = (char *)tmp;
    unsigned long long *krow = (unsigned long long *)t;
    t += 8 * (size_t)nnz;
    unsigned long long *kcol = (unsigned long long *)t;
    t += 8 * (size_t)nnz;
    unsigned long long *ksort = (unsigned long long *)t;
    t += 8 * (size_t)nnz;
    int32_t *idx = (int32_t *)t;
    t += 4 * (size_t)nnz;
    int32_t *idx_sorted = (int32_t *)t;
    t += 4 * (size_t)nnz;
    t = (char *)(((uintptr_t)t + 255) & ~(uintptr_t)255);
    const size_t used = (size_t)(t - (char *)tmp);
    if (used > tmp_bytes) return hipErrorInvalidValue;
    size_t sort_bytes = tmp_bytes - used;
    hipError_t e = hipSuccess;
    if (nnz > 0) {
        hipLaunchKernelGGL(k_entry_keys, dim3(blocks(n)), dim3(256), 0, s, in.rp, in.ci, in.inv, n, krow, kcol, idx);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // P: entries by (row, internal column); P^T: by (internal column, row)
        e = hipcub::DeviceRadixSort::SortPairs(t, sort_bytes, krow, ksort, idx, idx_sorted, (int)nnz, 0, 51, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_gather_entries<T>), dim3(blocks(nnz)), dim3(256), 0, s, ksort, idx_sorted, nnz,
                           (1ull << 20) - 1, (const T *)in.val, out.ci, (T *)out.val);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        sort_bytes = tmp_bytes - used;
        e = hipcub::DeviceRadixSort::SortPairs(t, sort_bytes, kcol, ksort, idx, idx_sorted, (int)nnz, 0, 51, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_gather_entries<T>), dim3(blocks(nnz)), dim3(256), 0, s, ksort, idx_sorted, nnz,
                           (1ull << 31) - 1, (const T *)in.val, out.ciT, (T *)out.valT);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_rowptr_t, dim3(blocks(nnz + 1)), dim3(256), 0, s, ksort, nnz, l, out.rpT);
    hipLaunchKernelGGL((k_colsums<T, false>), dim3(blocks(l)), dim3(256), 0, s, out.rpT, (const T *)out.valT, l, out.c);
    if (out.c_bf16)
        hipLaunchKernelGGL((k_colsums<T, true>), dim3(blocks(l)), dim3(256), 0, s, out.rpT, (const T *)out.valT, l,
                           out.c_bf16);
    hipLaunchKernelGGL((k_permute_w<T>), dim3((unsigned)l), dim3(256), 0, s, (const T *)in.W, l, out.lda, in.perm,
                       (T *)out.W);
    return hipGetLastError();
}

size_t prep_tmp_bytes(int64_t nnz, bool fp64) {
    size_t sort_bytes = 0;
    if (nnz > 0) {
        unsigned long long *k = nullptr;
        int32_t *v = nullptr;
        (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, k, k, v, v, (int)nnz, 0, 51, (hipStream_t)0);
    }
    (void)fp64;
    return 32 * (size_t)nnz + 256 + sort_bytes + 256;  // three key arrays, two index arrays, the sort
}

// ---------------------------------------------------------------------------
// Push form of the transposed product.  Scratch layout: key, sorted key,
// index, sorted index (nnz each), head / pair id (nnz each), the sort's work
// area; a second key array for the reduction lists reuses the first two.

namespace {

struct PushTmp {
    unsigned long long *key, *key2;
    int32_t *idx, *idx2, *head, *pid;
    char *sort;
    size_t sort_bytes;
};

PushTmp push_tmp(void *tmp, size_t tmp_bytes, int64_t nnz) {
    PushTmp t{};
    char *q = (char *)tmp;
    auto take = [&](size_t b) {
        char *r = q;
        q += (b + 255) & ~(size_t)255;
        return r;
    };
    t.key = (unsigned long long *)take(8 * (size_t)nnz);
    t.key2 = (unsigned long long *)take(8 * (size_t)nnz);
    t.idx = (int32_t *)take(4 * (size_t)nnz);
    t.idx2 = (int32_t *)take(4 * (size_t)nnz);
    t.head = (int32_t *)take(4 * (size_t)nnz);
    t.pid = (int32_t *)take(4 * (size_t)nnz);
    t.sort = q;
    const size_t used = (size_t)(q - (char *)tmp);
    t.sort_bytes = used <= tmp_bytes ? tmp_bytes - used : 0;
    return t;
}

int key_bits(unsigned long long maxkey) {
    int b = 1;
    while (b < 64 && (maxkey >> b) != 0) ++b;
    return b;
}

// key = (block * l + column) * kPushVB + vertex within block, per entry.
__global__ __launch_bounds__(256) void k_push_keys(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   int64_t n, int64_t l, unsigned long long *__restrict__ key,
                                                   int32_t *__restrict__ idx) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const unsigned long long blk = (unsigned long long)(v / kPushVB), w = (unsigned long long)(v % kPushVB);
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
        key[e] = (blk * (unsigned long long)l + (unsigned long long)ci[e]) * kPushVB + w;
        idx[e] = e;
    }
}

__global__ __launch_bounds__(256) void k_push_heads(const unsigned long long *__restrict__ key, int64_t nnz,
                                                    int32_t *__restrict__ head) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nnz) return;
    head[i] = (i == 0 || key[i] / kPushVB != key[i - 1] / kPushVB) ? 1 : 0;
}

// Per entry in pair order: vertex within block and value(s); per pair its
// first entry; the reduction key (column * nvb + block) and pair id.
template <typename T>
__global__ __launch_bounds__(256) void k_push_fill(const unsigned long long *__restrict__ key,
                                                   const int32_t *__restrict__ idx, const int32_t *__restrict__ head,
                                                   const int32_t *__restrict__ pid, int64_t nnz, int64_t l,
                                                   int64_t nvb, const T *__restrict__ val,
                                                   const bf16_t *__restrict__ val16, uint8_t *__restrict__ pvl,
                                                   T *__restrict__ pv, bf16_t *__restrict__ pv16,
                                                   int32_t *__restrict__ pe, unsigned long long *__restrict__ rkey,
                                                   int32_t *__restrict__ rval) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nnz) return;
    const unsigned long long k = key[i];
    pvl[i] = (uint8_t)(k % kPushVB);
    pv[i] = val[idx[i]];
    if (pv16) pv16[i] = val16[idx[i]];
    if (head[i]) {
        const int64_t q = pid[i] - 1;
        const unsigned long long bc = k / kPushVB;  // block * l + column
        pe[q] = (int32_t)i;
        rkey[q] = (bc % (unsigned long long)l) * (unsigned long long)nvb + bc / (unsigned long long)l;
        rval[q] = (int32_t)q;
    }
    if (i == nnz - 1) pe[pid[i]] = (int32_t)nnz;
}

// Row pointers (nrows + 1) of sorted keys, row = key / div.
__global__ __launch_bounds__(256) void k_push_rowptr(const unsigned long long *__restrict__ key, int64_t count,
                                                     unsigned long long div, int64_t nrows, int32_t *__restrict__ rp) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i > count) return;
    const int64_t r = i < count ? (int64_t)(key[i] / div) : nrows;
    const int64_t rprev = i > 0 ? (int64_t)(key[i - 1] / div) : -1;
    for (int64_t q = rprev + 1; q <= r; ++q) rp[q] = (int32_t)i;
}

// Pair p's vertex block: pb from the pair keys block * l + column.
__global__ __launch_bounds__(256) void k_push_pair_keys(const unsigned long long *__restrict__ rkey, int64_t npairs,
                                                        int64_t nvb, unsigned long long *__restrict__ bkey) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= npairs) return;
    bkey[q] = rkey[q] % (unsigned long long)nvb;  // pairs are already in (block, column) order
}

}  // namespace

size_t prep_push_tmp_bytes(int64_t nnz) {
    size_t sort_bytes = 0;
    if (nnz > 0) {
        unsigned long long *k = nullptr;
        int32_t *v = nullptr;
        (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, k, k, v, v, (int)nnz, 0, 64, (hipStream_t)0);
    }
    size_t inclusive = 0;
    if (nnz > 0) {
        int32_t *a = nullptr;
        (void)hipcub::DeviceScan::InclusiveSum(nullptr, inclusive, a, a, (int)nnz, (hipStream_t)0);
    }
    return 32 * (size_t)nnz + 6 * 256 + std::max(sort_bytes, inclusive) + 256;
}

hipError_t prep_push_pairs(const int32_t *rp, const int32_t *ci, int64_t n, int64_t l, int64_t nnz, void *tmp,
                           size_t tmp_bytes, int64_t *npairs, hipStream_t s) {
    *npairs = 0;
    if (nnz <= 0) return hipSuccess;
    PushTmp t = push_tmp(tmp, tmp_bytes, nnz);
    const int64_t nvb = (n + kPushVB - 1) / kPushVB;
    hipLaunchKernelGGL(k_push_keys, dim3(blocks(n)), dim3(256), 0, s, rp, ci, n, l, t.key, t.idx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int bits = key_bits((unsigned long long)nvb * (unsigned long long)l * kPushVB);
    size_t sb = t.sort_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(t.sort, sb, t.key, t.key2, t.idx, t.idx2, (int)nnz, 0, bits, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_push_heads, dim3(blocks(nnz)), dim3(256), 0, s, (const unsigned long long *)t.key2, nnz,
                       t.head);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    sb = t.sort_bytes;
    e = hipcub::DeviceScan::InclusiveSum(t.sort, sb, t.head, t.pid, (int)nnz, s);
    if (e != hipSuccess) return e;
    int32_t h = 0;
    if ((e = hipMemcpyAsync(&h, t.pid + nnz - 1, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *npairs = h;
    return hipSuccess;
}

hipError_t prep_push_fill(int64_t n, int64_t l, int64_t nnz, int64_t npairs, const void *val, int esz,
                          const void *val16, const PushOut &out, void *tmp, size_t tmp_bytes, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    PushTmp t = push_tmp(tmp, tmp_bytes, nnz);
    const int64_t nvb = (n + kPushVB - 1) / kPushVB;
    // the reduction keys and pair ids reuse key / idx (free after the sort)
    unsigned long long *rkey = t.key;
    int32_t *rval = t.idx;
    if (esz == 8)
        hipLaunchKernelGGL((k_push_fill<double>), dim3(blocks(nnz)), dim3(256), 0, s,
                           (const unsigned long long *)t.key2, (const int32_t *)t.idx2, (const int32_t *)t.head,
                           (const int32_t *)t.pid, nnz, l, nvb, (const double *)val, (const bf16_t *)val16, out.pvl,
                           (double *)out.pv, (bf16_t *)out.pv16, out.pe, rkey, rval);
    else
        hipLaunchKernelGGL((k_push_fill<float>), dim3(blocks(nnz)), dim3(256), 0, s,
                           (const unsigned long long *)t.key2, (const int32_t *)t.idx2, (const int32_t *)t.head,
                           (const int32_t *)t.pid, nnz, l, nvb, (const float *)val, (const bf16_t *)val16, out.pvl,
                           (float *)out.pv, (bf16_t *)out.pv16, out.pe, rkey, rval);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // vertex-block ranges of the pairs: the block of pair q is rkey[q] % nvb
    unsigned long long *bkey = t.key2;  // sorted entry keys are no longer needed
    hipLaunchKernelGGL(k_push_pair_keys, dim3(blocks(npairs)), dim3(256), 0, s, (const unsigned long long *)rkey,
                       npairs, nvb, bkey);
    hipLaunchKernelGGL(k_push_rowptr, dim3(blocks(npairs + 1)), dim3(256), 0, s, (const unsigned long long *)bkey,
                       npairs, 1ull, nvb, out.pb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // reduction lists: pairs by (column, block)
    unsigned long long *rkey2 = (unsigned long long *)t.head;  // head + pid: 8 nnz bytes >= 8 npairs
    const int bits = key_bits((unsigned long long)l * (unsigned long long)nvb);
    size_t sb = t.sort_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(t.sort, sb, rkey, rkey2, rval, out.ql, (int)npairs, 0, bits, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_push_rowptr, dim3(blocks(npairs + 1)), dim3(256), 0, s, (const unsigned long long *)rkey2,
                       npairs, (unsigned long long)nvb, l, out.qp);
    return hipGetLastError();
}

template hipError_t prep_validate<float>(const int32_t *, const int32_t *, const void *, const void *, int64_t,
                                         int64_t, int64_t, unsigned long long *, hipStream_t);
template hipError_t prep_validate<double>(const int32_t *, const int32_t *, const void *, const void *, int64_t,
                                          int64_t, int64_t, unsigned long long *, hipStream_t);
template hipError_t prep_labels<float>(const void *, int64_t, const int32_t *, const int32_t *, const int32_t *,
                                       int32_t *, hipStream_t);
template hipError_t prep_labels<double>(const void *, int64_t, const int32_t *, const int32_t *, const int32_t *,
                                        int32_t *, hipStream_t);
template hipError_t prep_operator<float>(const PrepIn &, const PrepOut &, void *, size_t, hipStream_t);
template hipError_t prep_operator<double>(const PrepIn &, const PrepOut &, void *, size_t, hipStream_t);

}  // namespace sbmds
