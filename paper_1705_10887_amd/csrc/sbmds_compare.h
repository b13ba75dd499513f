// The paper's other two routes to the top-k eigenpairs of
// B = -1/2 J P W P^T J (Section 3.3), on one problem of a context, as
// comparison solvers beside the block subspace iteration:
//   * (block) Lanczos on the implicit operator: only products with B, each
//     one transposed sparse product, one dense product with W and one sparse
//     product (block width 1 is the paper's sBMDS);
//   * BMDS: the QR factorisation J P = Q R, the eigendecomposition of
//     -1/2 R W R^T and Z = Q V_k Lambda_k^{1/2} (O(n l) memory).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sbmds {

// One problem's operator as the comparison solvers read it: CSR of P and of
// P^T in the internal landmark order, W (l x lda row-major, symmetric), the
// column sums c = P^T 1 in float64; values float or double (f64).
struct CmpOp {
    int64_t n = 0, l = 0, nnz = 0;
    int lda = 0;
    const int32_t *rp = nullptr, *ci = nullptr, *rpT = nullptr, *ciT = nullptr;
    const void *val = nullptr, *valT = nullptr, *W = nullptr;
    const double *c = nullptr;
    bool f64 = false;
};

constexpr int kCmpMaxK = 16;  // eigenpairs the comparison solvers return

struct CmpResult {
    int status = 0;       // SBMDS_OK or SBMDS_ENOCONV
    int steps = 0;        // block Lanczos steps (0 for BMDS)
    int basis = 0;        // columns of the Krylov basis (0 for BMDS)
    int nonpositive = 0;  // wanted eigenvalues <= 0 (their coordinates are 0)
    double eig[kCmpMaxK] = {}, bound[kCmpMaxK] = {}, resid[kCmpMaxK] = {};
};

// Both write Z (device, row-major n x k, double if z_double else float) and
// return SBMDS_OK, SBMDS_ENOCONV (Lanczos step cap reached; best Ritz pairs
// written) or a negative status with the message set.  They synchronise s.
int lanczos_solve(const CmpOp &op, int k, int p, int max_steps, double tol, uint64_t seed, void *Z, int z_double,
                  CmpResult *res, hipStream_t s);
int bmds_solve(const CmpOp &op, int k, void *Z, int z_double, CmpResult *res, hipStream_t s);

}  // namespace sbmds
