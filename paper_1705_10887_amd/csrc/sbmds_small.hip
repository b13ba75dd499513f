// The b x b float64 step of block subspace iteration: Rayleigh-Ritz, residual
// norms, error bounds and the next orthonormal basis (CholQR), all on the
// device in one workgroup.
//
// Iteration state: X = J Y C is an orthonormal, centred basis (J the
// centering matrix), Y' = B X was just produced by the sparse/dense kernels,
// and the kernels also left
//   H  = X^T B X            (from T^T U, Section 3.3 operator)
//   G  = Y'^T Y',  e = 1^T Y'
// This step computes
//   1. H = S Theta S^T       (cyclic Jacobi, Ritz values sorted descending;
//                             classical MDS keeps the largest eigenvalues,
//                             Section 2.3)
//   2. Zmap = C S_k Theta_k^{1/2}, so that Z = J Y Zmap = X S_k Theta_k^{1/2}
//   3. ||B x_i - theta_i x_i||^2 = s_i^T Gc s_i - theta_i^2 with
//      Gc = G - e e^T / n (the Gram of J Y'), since X^T X = I and X^T B X = H
//   4. error bounds (see bounds())
//   5. Sc^T Gc S = L L^T (Cholesky) and C' = S L^{-T}, so X' = J Y' C' is
//      orthonormal again and its leading columns follow the Ritz order.
// In `init` mode only step 5 runs, with S = I, on a fresh start block.
#include "sbmds_common.h"

namespace sbmds {

template <int B>
struct SmallLds {
    double A[B][B + 1];
    double V[B][B + 1];
    double Gc[B][B + 1];
    double th[B];
    double red[256];
    int perm[B];
    int dead[B];
    int rot_p[B / 2 + 1], rot_q[B / 2 + 1];
    double rot_c[B / 2 + 1], rot_s[B / 2 + 1];
};

__device__ __forceinline__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// Cyclic Jacobi with round-robin pair ordering; A (b x b, symmetric) is
// diagonalised in place and V accumulates the rotations (V starts as I).
template <int B>
__device__ void jacobi(SmallLds<B> &L, int b) {
    const int tid = threadIdx.x;
    const int bb = (b & 1) ? b + 1 : b;  // odd sizes get a dummy index
    const int npair = bb / 2;
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int e = tid; e < b * b; e += 256) {
            const int i = e / b, j = e % b;
            const double v = L.A[i][j];
            if (i != j) off += v * v;
            else dia += v * v;
        }
        off = block_sum(off, L.red);
        dia = block_sum(dia, L.red);
        if (!(off > 1e-32 * dia) || dia == 0.0) break;
        for (int round = 0; round < bb - 1; ++round) {
            if (tid < npair) {
                int p, q;
                if (tid == 0) {
                    p = round;
                    q = bb - 1;
                } else {
                    p = (round + tid) % (bb - 1);
                    q = (round - tid + (bb - 1)) % (bb - 1);
                }
                double c = 1.0, s = 0.0;
                if (p < b && q < b) {
                    const double apq = L.A[p][q];
                    const double app = L.A[p][p], aqq = L.A[q][q];
                    if (fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * (fabs(app) + fabs(aqq))) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                L.rot_p[tid] = p;
                L.rot_q[tid] = q;
                L.rot_c[tid] = c;
                L.rot_s[tid] = s;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int e = tid; e < npair * b; e += 256) {
                const int k = e / b, col = e % b;
                const int p = L.rot_p[k], q = L.rot_q[k];
                const double s = L.rot_s[k];
                if (s != 0.0) {
                    const double c = L.rot_c[k];
                    const double ap = L.A[p][col], aq = L.A[q][col];
                    L.A[p][col] = c * ap - s * aq;
                    L.A[q][col] = s * ap + c * aq;
                }
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (int e = tid; e < npair * b; e += 256) {
                const int k = e / b, row = e % b;
                const int p = L.rot_p[k], q = L.rot_q[k];
                const double s = L.rot_s[k];
                if (s != 0.0) {
                    const double c = L.rot_c[k];
                    const double ap = L.A[row][p], aq = L.A[row][q];
                    L.A[row][p] = c * ap - s * aq;
                    L.A[row][q] = s * ap + c * aq;
                    const double vp = L.V[row][p], vq = L.V[row][q];
                    L.V[row][p] = c * vp - s * vq;
                    L.V[row][q] = s * vp + c * vq;
                }
            }
            __syncthreads();
        }
    }
}

// Error bounds for the k wanted Ritz values (thread 0).  Ritz values closer
// than 1e-3 (relative) form a cluster; a cluster's gap is its distance to the
// nearest other Ritz value or to the magnitude of the smallest Ritz value of
// the block (which stands for the spectrum the block does not hold).  For
// each wanted value the bound is min(||r_i||, ||R_cluster||^2 / gap) / |theta_i|.
__device__ void bounds(SolveState *st, const double *th, const double *res, int b, int k) {
    double floor_mag = INFINITY;
    for (int i = 0; i < b; ++i) floor_mag = fmin(floor_mag, fabs(th[i]));
    double maxb = 0.0, maxr = 0.0;
    int nonpos = 0;
    int i = 0;
    while (i < b) {
        int j = i;
        while (j + 1 < b && fabs(th[j] - th[j + 1]) <= 1e-3 * fmax(fabs(th[j]), fabs(th[j + 1]))) ++j;
        // cluster [i, j]
        double r2 = 0.0;
        for (int q = i; q <= j; ++q) r2 += res[q] * res[q];
        double gap = INFINITY;
        if (i > 0) gap = fmin(gap, th[i - 1] - th[i]);
        if (j + 1 < b) gap = fmin(gap, th[j] - th[j + 1]);
        const double lo = th[j];
        const double out_gap = lo > 0.0 ? lo - floor_mag : (-lo) - floor_mag;
        gap = fmin(gap, out_gap);
        for (int q = i; q <= j; ++q) {
            const double a = fabs(th[q]);
            double bnd = res[q];
            if (gap > 0.0) bnd = fmin(bnd, r2 / gap);
            const double rel = a > 0.0 ? bnd / a : INFINITY;
            st->bound[q] = rel;
            st->res[q] = res[q];
            if (q < k) {
                maxb = fmax(maxb, rel);
                maxr = fmax(maxr, a > 0.0 ? res[q] / a : INFINITY);
                if (th[q] <= 0.0) ++nonpos;
            }
        }
        i = j + 1;
    }
    st->maxbound = maxb;
    st->maxres = maxr;
    st->nonpos = nonpos;
}

template <int B>
__global__ __launch_bounds__(256) void k_rr_solve(SolveState *__restrict__ st, int b, int k, double n,
                                                  double piv_tol, int init) {
    __shared__ SmallLds<B> L;
    const int tid = threadIdx.x;
    const double inv_n = 1.0 / n;

    // Gc = G - e e^T / n
    for (int e = tid; e < b * b; e += 256) {
        const int i = e / b, j = e % b;
        L.Gc[i][j] = st->G[i * B + j] - st->e_new[i] * st->e_new[j] * inv_n;
    }
    if (tid < B) L.dead[tid] = 0;
    __syncthreads();

    if (init) {
        for (int e = tid; e < b * b; e += 256) {
            const int i = e / b, j = e % b;
            L.A[i][j] = (i == j) ? 1.0 : 0.0;  // S = I
        }
        __syncthreads();
    } else {
        for (int e = tid; e < b * b; e += 256) {
            const int i = e / b, j = e % b;
            L.A[i][j] = 0.5 * (st->H[i * B + j] + st->H[j * B + i]);
            L.V[i][j] = (i == j) ? 1.0 : 0.0;
        }
        __syncthreads();
        jacobi<B>(L, b);
        // sort Ritz values descending (ties by index)
        if (tid < b) {
            const double t = L.A[tid][tid];
            int rank = 0;
            for (int j = 0; j < b; ++j) {
                const double u = L.A[j][j];
                rank += (u > t) || (u == t && j < tid);
            }
            L.perm[rank] = tid;
        }
        __syncthreads();
        if (tid < b) L.th[tid] = L.A[L.perm[tid]][L.perm[tid]];
        __syncthreads();
        // S (sorted eigenvectors) into A
        for (int e = tid; e < b * b; e += 256) {
            const int r = e / b, i = e % b;
            L.A[r][i] = L.V[r][L.perm[i]];
        }
        __syncthreads();
        // Zmap = C S_k sqrt(max(theta, 0)), zshift = e_x^T Zmap / n
        for (int e = tid; e < B * B; e += 256) {
            const int r = e / B, i = e % B;
            double z = 0.0;
            if (r < b && i < k) {
                for (int m = 0; m < b; ++m) z += st->C[r * B + m] * L.A[m][i];
                z *= sqrt(fmax(L.th[i], 0.0));
            }
            st->Zmap[e] = z;
        }
        __syncthreads();
        if (tid < B) {
            double z = 0.0;
            if (tid < k)
                for (int r = 0; r < b; ++r) z += st->e_x[r] * st->Zmap[r * B + tid];
            st->zshift[tid] = z * inv_n;
        }
        // GS = Gc S into V
        for (int e = tid; e < b * b; e += 256) {
            const int r = e / b, i = e % b;
            double v = 0.0;
            for (int m = 0; m < b; ++m) v += L.Gc[r][m] * L.A[m][i];
            L.V[r][i] = v;
        }
        __syncthreads();
        // residuals, Ritz values out
        if (tid < b) {
            double d = 0.0;
            for (int r = 0; r < b; ++r) d += L.A[r][tid] * L.V[r][tid];
            const double t = L.th[tid];
            L.red[tid] = sqrt(fmax(d - t * t, 0.0));
            st->theta[tid] = t;
        }
        __syncthreads();
        if (tid == 0) bounds(st, L.th, L.red, b, k);
        __syncthreads();
        // Gc <- S^T Gc S
        for (int e = tid; e < b * b; e += 256) {
            const int i = e / b, j = e % b;
            double v = 0.0;
            for (int r = 0; r < b; ++r) v += L.A[r][i] * L.V[r][j];
            L.Gc[i][j] = v;
        }
        __syncthreads();
        // symmetrise
        for (int e = tid; e < b * b; e += 256) {
            const int i = e / b, j = e % b;
            if (i < j) {
                const double v = 0.5 * (L.Gc[i][j] + L.Gc[j][i]);
                L.Gc[i][j] = v;
                L.Gc[j][i] = v;
            }
        }
        __syncthreads();
    }

    // Left-looking Cholesky Gc = Lc Lc^T, Lc stored in the lower triangle.
    // A pivot that kept no more than piv_tol of its original size marks a
    // column whose direction is already spanned by earlier ones; it is
    // dropped from the next basis (its column of C' is zero).
    for (int j = 0; j < b; ++j) {
        if (tid == 0) {
            const double orig = L.Gc[j][j];
            double d = orig;
            for (int m = 0; m < j; ++m) d -= L.Gc[j][m] * L.Gc[j][m];
            if (!(d > piv_tol * orig) || !(orig > 0.0) || !isfinite(d)) {
                L.dead[j] = 1;
                L.Gc[j][j] = 1.0;
            } else {
                L.Gc[j][j] = sqrt(d);
            }
        }
        __syncthreads();
        const int isdead = L.dead[j];
        const double ljj = L.Gc[j][j];
        for (int i = j + 1 + tid; i < b; i += 256) {
            if (isdead) {
                L.Gc[i][j] = 0.0;
            } else {
                double v = L.Gc[i][j];
                for (int m = 0; m < j; ++m) v -= L.Gc[i][m] * L.Gc[j][m];
                L.Gc[i][j] = v / ljj;
            }
        }
        __syncthreads();
    }
    // Linv = Lc^{-1} into V (column j per thread, forward substitution)
    if (tid < b) {
        const int j = tid;
        for (int i = 0; i < b; ++i) L.V[i][j] = 0.0;
        L.V[j][j] = 1.0 / L.Gc[j][j];
        for (int i = j + 1; i < b; ++i) {
            double v = 0.0;
            for (int m = j; m < i; ++m) v -= L.Gc[i][m] * L.V[m][j];
            L.V[i][j] = v / L.Gc[i][i];
        }
    }
    __syncthreads();
    // C' = S Linv^T ; dropped columns are zeroed
    for (int e = tid; e < B * B; e += 256) {
        const int r = e / B, j = e % B;
        double v = 0.0;
        if (r < b && j < b && !L.dead[j]) {
            for (int m = 0; m <= j; ++m) v += L.A[r][m] * L.V[j][m];
        }
        st->C[e] = v;
    }
    if (tid < B) st->e_x[tid] = st->e_new[tid];
    __syncthreads();
    if (tid == 0) {
        int nd = 0;
        for (int j = 0; j < b; ++j) nd += L.dead[j];
        st->dead = nd;
        if (nd) st->flags |= SF_REPAIRED;
        bool fin = true;
        for (int j = 0; j < b; ++j) fin = fin && isfinite(st->C[j * B + j]);
        if (!fin) st->flags |= SF_NONFINITE;
        if (init) {
            st->iter = 0;
            st->maxbound = INFINITY;
            st->maxres = INFINITY;
        } else {
            st->iter += 1;
        }
    }
}

hipError_t launch_rr_solve(const DevProblem &p, int init, hipStream_t s) {
    const double piv_tol = 1e-10;
    switch (p.B) {
        case 4: hipLaunchKernelGGL((k_rr_solve<4>), dim3(1), dim3(256), 0, s, p.st, p.b, p.k, (double)p.n, piv_tol, init); break;
        case 8: hipLaunchKernelGGL((k_rr_solve<8>), dim3(1), dim3(256), 0, s, p.st, p.b, p.k, (double)p.n, piv_tol, init); break;
        case 16: hipLaunchKernelGGL((k_rr_solve<16>), dim3(1), dim3(256), 0, s, p.st, p.b, p.k, (double)p.n, piv_tol, init); break;
        case 32: hipLaunchKernelGGL((k_rr_solve<32>), dim3(1), dim3(256), 0, s, p.st, p.b, p.k, (double)p.n, piv_tol, init); break;
        case 64: hipLaunchKernelGGL((k_rr_solve<64>), dim3(1), dim3(256), 0, s, p.st, p.b, p.k, (double)p.n, piv_tol, init); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sbmds
