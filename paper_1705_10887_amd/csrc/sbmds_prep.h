// Create-time preparation of one problem on the device (see sbmds_prep.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sbmds {

// Failed checks of device-resident inputs, in the order they are reported
// (the smallest code, then the smallest row, wins).
enum PrepError {
    PREP_ROWPTR0 = 1,       // P_rowptr[0] != 0
    PREP_ROWPTRN = 2,       // P_rowptr[n] != nnz
    PREP_ROWPTR_ORDER = 3,  // P_rowptr decreasing or past nnz (row)
    PREP_COL_RANGE = 4,     // P_col outside [0, l) (row)
    PREP_COL_ORDER = 5,     // P_col not strictly increasing (row)
    PREP_VAL = 6,           // non-finite P value (row)
    PREP_W_FINITE = 7,      // non-finite W entry (row)
    PREP_W_SYM = 8          // W not symmetric (row)
};
constexpr unsigned long long kPrepNoError = ~0ull;

// Device inputs of the operator preparation (caller's vertex and landmark
// order) and the internal landmark order: perm[j] = caller landmark of
// internal landmark j, inv its inverse.
struct PrepIn {
    int64_t n, l, nnz;
    const int32_t *rp, *ci;
    const void *val, *W;
    const int32_t *perm, *inv;
};
// Device outputs: P with internal column ids (rows re-sorted; row pointers
// are unchanged), P^T (rows in increasing vertex order), c = P^T 1 in
// float64 (and from bfloat16-rounded values when c_bf16 is set), W in the
// internal order with rows of lda elements, zero-padded.
struct PrepOut {
    int lda;
    int32_t *ci, *rpT, *ciT;
    void *val, *valT, *W;
    double *c, *c_bf16;
};

template <typename T>
hipError_t prep_validate(const int32_t *rp, const int32_t *ci, const void *val, const void *W, int64_t n, int64_t l,
                         int64_t nnz, unsigned long long *err, hipStream_t s);
template <typename T>
hipError_t prep_labels(const void *W, int64_t l, const int32_t *order, const int32_t *seg, const int32_t *piv,
                       int32_t *label, hipStream_t s);
template <typename T>
hipError_t prep_operator(const PrepIn &in, const PrepOut &out, void *tmp, size_t tmp_bytes, hipStream_t s);
// Scratch bytes prep_operator needs for nnz entries.
size_t prep_tmp_bytes(int64_t nnz, bool fp64);

// The push form of the transposed product (T = P^T Y by vertex blocks of
// kPushVB rows): entries of P grouped by (vertex block, column, vertex);
// each distinct (block, column) is a "pair" whose partial row one block
// writes and the reduction sums per column in block order.
constexpr int kPushVB = 256;
struct PushOut {
    int32_t *pb;    // [nvb + 1] first pair of each vertex block
    int32_t *pe;    // [npairs + 1] first entry of each pair
    uint8_t *pvl;   // [nnz] vertex within its block, per entry in pair order
    int32_t *qp;    // [l + 1] first reduction item of each column
    int32_t *ql;    // [npairs] pairs of each column, in block order
    void *pv;       // [nnz] values in pair order (element size esz)
    void *pv16;     // [nnz] bfloat16 values in pair order, or NULL
};
// Scratch bytes of the push-form preparation; its first phase sorts the
// entries and returns the pair count (the stream is synchronised), the
// second fills PushOut from the same scratch.
size_t prep_push_tmp_bytes(int64_t nnz);
hipError_t prep_push_pairs(const int32_t *rp, const int32_t *ci, int64_t n, int64_t l, int64_t nnz, void *tmp,
                           size_t tmp_bytes, int64_t *npairs, hipStream_t s);
hipError_t prep_push_fill(int64_t n, int64_t l, int64_t nnz, int64_t npairs, const void *val, int esz,
                          const void *val16, const PushOut &out, void *tmp, size_t tmp_bytes, hipStream_t s);

}  // namespace sbmds
