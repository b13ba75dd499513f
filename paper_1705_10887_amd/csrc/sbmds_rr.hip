// Launcher of the standalone Rayleigh-Ritz kernel (B <= 32); the step itself
// is in sbmds_rr.h.
#include "sbmds_rr.h"

namespace sbmds {

hipError_t launch_rr_solve2(const Batch &bt, int init, int max_sweeps, const PhaseRule &rule, hipStream_t s) {
    const double piv_tol = kPivTol;
    const dim3 grid(bt.nprob);
    switch (bt.B) {
        case 4:
            hipLaunchKernelGGL((k_rr_solve2<4>), grid, dim3(RRShape<4>::NT), 0, s, bt.views, bt.b, bt.k, piv_tol, init,
                               max_sweeps, rule);
            break;
        case 8:
            hipLaunchKernelGGL((k_rr_solve2<8>), grid, dim3(RRShape<8>::NT), 0, s, bt.views, bt.b, bt.k, piv_tol, init,
                               max_sweeps, rule);
            break;
        case 16:
            hipLaunchKernelGGL((k_rr_solve2<16>), grid, dim3(RRShape<16>::NT), 0, s, bt.views, bt.b, bt.k, piv_tol,
                               init, max_sweeps, rule);
            break;
        case 32:
            hipLaunchKernelGGL((k_rr_solve2<32>), grid, dim3(RRShape<32>::NT), 0, s, bt.views, bt.b, bt.k, piv_tol,
                               init, max_sweeps, rule);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sbmds
