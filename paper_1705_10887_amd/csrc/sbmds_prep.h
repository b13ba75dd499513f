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

}  // namespace sbmds
