// Packed upper triangle of W and the dense product that streams it (see
// sbmds_dense_sym.hip): layout helpers shared by the kernels and the host.
#pragma once

#include "sbmds_internal.h"

namespace sbmds {

// First element of strip i (rows 64i .. 64i+63, columns 64i .. lda-1) of the
// packed upper triangle of an lda x lda matrix; sym_strip_base(lda / 64, lda)
// is the packed size.
__host__ __device__ inline int64_t sym_strip_base(int i, int lda) {
    return (int64_t)64 * i * lda - (int64_t)2048 * i * (i - 1);
}

// First region column of region row gr (regions of R x C tiles that hold a
// tile of the upper triangle).
__host__ __device__ inline int sym_gcmin(int gr, int R, int C) { return (gr * R) / C; }

// Number of regions of R x C tiles over nt x nt tiles.
__host__ __device__ inline int sym_regions(int nt, int R, int C) {
    const int ngr = (nt + R - 1) / R, ngc = (nt + C - 1) / C;
    int n = 0;
    for (int g = 0; g < ngr; ++g) n += ngc - sym_gcmin(g, R, C);
    return n;
}

// Limits of the packed path: region rows/columns per side (the finish
// kernel's slot list), so lda / 64 <= kSymMaxTiles and C >= kSymMinC.
constexpr int kSymMaxGroups = 256;
constexpr int kSymMaxTiles = 1024;
constexpr int kSymMinC = 8;

int sym_region_rows(Mode m, int B);   // R of the packed kernel for this mode and width
bool sym_supported(Mode m, int B);
hipError_t launch_pack_sym(const float *W, int64_t l, int lda, float *Wp, hipStream_t s);
hipError_t launch_gemm_sym(Mode m, const Batch &bt, int phase, hipStream_t s);

}  // namespace sbmds
