// The b x b float64 step of block subspace iteration: Rayleigh-Ritz, residual
// norms, error bounds and the next orthonormal basis (CholQR), all on the
// device in one workgroup.
//
// Iteration state: X = J Y C is an orthonormal, centred basis (J the
// centering matrix), Y' = B X was just produced by the sparse/dense kernels,
// and the kernels also left (SolveState::Hs and ::Ge)
//   H  = X^T B X            (from T^T U, Section 3.3 operator)
//   G  = Y'^T Y',  e = 1^T Y'
// All inputs are staged into LDS first; the step runs in a single wave.
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
#include "sbmds_bounds.h"

namespace sbmds {

constexpr int kSolveThreads = 64;  // one wave: barriers are nearly free

template <int B>
struct SmallLds {
    double A[B][B + 1];     // H, then the sorted eigenvectors S
    double V[B][B + 1];     // Jacobi rotations; later scratch (Zmap, Gc S, L^-1)
    double Gc[B][B + 1];    // centred Gram; later S^T Gc S and its Cholesky factor
    double Cold[B][B + 1];  // basis transform the current H was computed with
    double e_new[B], e_x[B];
    double th[B], res[B];
    int perm[B], dead[B];
    int rot_p[B / 2 + 1], rot_q[B / 2 + 1];
    double rot_c[B / 2 + 1], rot_s[B / 2 + 1];
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// Cyclic Jacobi with round-robin pair ordering; A (b x b, symmetric) is
// diagonalised in place and V accumulates the rotations (V starts as I).
// The b/2 rotations of one round act on disjoint index pairs, so A <- J^T A J
// splits into independent 2x2 blocks (pair k rows, pair l columns) and
// V <- V J into independent row pieces: one barrier-separated phase each.
template <int B>
__device__ int jacobi(SmallLds<B> &L, int b, int max_sweeps) {
    const int tid = threadIdx.x;
    constexpr int NT = kSolveThreads;
    const int bb = (b & 1) ? b + 1 : b;  // odd sizes get a dummy index (a zero padding row)
    const int npair = bb / 2;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int e = tid; e < b * b; e += NT) {
            const int i = e / b, j = e % b;
            const double v = L.A[i][j];
            if (i != j) off += v * v;
            else dia += v * v;
        }
        off = wave_sum(off);
        dia = wave_sum(dia);
        if (!(off > 1e-24 * dia) || dia == 0.0) break;
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
            // A <- J^T A J on the 2x2 block (rows of pair k, columns of pair l)
            for (int e = tid; e < npair * npair; e += NT) {
                const int k = e / npair, l2 = e % npair;
                const int pk = L.rot_p[k], qk = L.rot_q[k], pl = L.rot_p[l2], ql = L.rot_q[l2];
                const double ck = L.rot_c[k], sk = L.rot_s[k], cl = L.rot_c[l2], sl = L.rot_s[l2];
                if (sk == 0.0 && sl == 0.0) continue;
                const double a00 = L.A[pk][pl], a01 = L.A[pk][ql], a10 = L.A[qk][pl], a11 = L.A[qk][ql];
                // rows
                const double r00 = ck * a00 - sk * a10, r01 = ck * a01 - sk * a11;
                const double r10 = sk * a00 + ck * a10, r11 = sk * a01 + ck * a11;
                // columns
                L.A[pk][pl] = cl * r00 - sl * r01;
                L.A[pk][ql] = sl * r00 + cl * r01;
                L.A[qk][pl] = cl * r10 - sl * r11;
                L.A[qk][ql] = sl * r10 + cl * r11;
            }
            // V <- V J
            for (int e = tid; e < npair * b; e += NT) {
                const int l2 = e / b, row = e % b;
                const double sl = L.rot_s[l2];
                if (sl == 0.0) continue;
                const int pl = L.rot_p[l2], ql = L.rot_q[l2];
                const double cl = L.rot_c[l2];
                const double vp = L.V[row][pl], vq = L.V[row][ql];
                L.V[row][pl] = cl * vp - sl * vq;
                L.V[row][ql] = sl * vp + cl * vq;
            }
            __syncthreads();
        }
    }
    return sweep;
}

template <int B>
__global__ __launch_bounds__(kSolveThreads) void k_rr_solve(const ProbView *__restrict__ views, int b, int k,
                                                            double piv_tol, int init, int max_sweeps,
                                                            PhaseRule rule) {
    __shared__ SmallLds<B> L;
    SolveState *__restrict__ st = views[blockIdx.x].st;
    const double n = (double)views[blockIdx.x].n;
    if (!init && (st->done || st->phase != rule.phase)) return;
    if (init == RR_REFILL && !st->refill) return;
    constexpr int NT = kSolveThreads;
    constexpr int E = B * (B + 1) / 2;
    const int tid = threadIdx.x;
    const double inv_n = 1.0 / n;

    // ---- stage every input in LDS
    for (int j = tid; j < B; j += NT) {
        L.e_new[j] = st->Ge[E + j];
        L.e_x[j] = st->e_x[j];
        L.dead[j] = 0;
    }
    for (int e = tid; e < B * B; e += NT) {
        const int i = e / B, j = e % B;
        L.Cold[i][j] = st->C[e];
        if (init) {
            L.A[i][j] = (i == j) ? 1.0 : 0.0;  // S = I
        } else {
            L.A[i][j] = 0.5 * (st->Hs[i * B + j] + st->Hs[j * B + i]);
            L.V[i][j] = (i == j) ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    // Gc = G - e e^T / n from the packed upper triangle
    for (int e = tid; e < B * B; e += NT) {
        const int a = e / B, c = e % B;
        const int lo = a < c ? a : c, hi = a < c ? c : a;
        const int pk = lo * B - (lo * (lo - 1)) / 2 + (hi - lo);
        L.Gc[a][c] = st->Ge[pk] - L.e_new[a] * L.e_new[c] * inv_n;
    }
    __syncthreads();

    if (!init) {
        const int nsw = jacobi<B>(L, b, max_sweeps);
        if (tid == 0) st->sweeps = nsw;
        // sort Ritz values descending (ties by index)
        for (int t = tid; t < b; t += NT) {
            const double th = L.A[t][t];
            int rank = 0;
            for (int j = 0; j < b; ++j) {
                const double u = L.A[j][j];
                rank += (u > th) || (u == th && j < t);
            }
            L.perm[rank] = t;
        }
        __syncthreads();
        for (int t = tid; t < b; t += NT) L.th[t] = L.A[L.perm[t]][L.perm[t]];
        __syncthreads();
        for (int e = tid; e < b * b; e += NT) {
            const int r = e / b, i = e % b;
            L.A[r][i] = L.V[r][L.perm[i]];  // S, columns in Ritz order
        }
        __syncthreads();
        // Zmap = Cold S_k sqrt(max(theta, 0)) into V, zshift = e_x^T Zmap / n
        for (int e = tid; e < B * B; e += NT) {
            const int r = e / B, i = e % B;
            double z = 0.0;
            if (r < b && i < k) {
                for (int m = 0; m < b; ++m) z += L.Cold[r][m] * L.A[m][i];
                z *= sqrt(fmax(L.th[i], 0.0));
            }
            L.V[r][i] = z;
        }
        __syncthreads();
        for (int e = tid; e < B * B; e += NT) st->Zmap[e] = L.V[e / B][e % B];
        for (int i = tid; i < B; i += NT) {
            double z = 0.0;
            if (i < k)
                for (int r = 0; r < b; ++r) z += L.e_x[r] * L.V[r][i];
            st->zshift[i] = z * inv_n;
        }
        __syncthreads();
        // Gc S into V
        for (int e = tid; e < b * b; e += NT) {
            const int r = e / b, i = e % b;
            double v = 0.0;
            for (int m = 0; m < b; ++m) v += L.Gc[r][m] * L.A[m][i];
            L.V[r][i] = v;
        }
        __syncthreads();
        // ||B x_i - theta_i x_i||^2 = s_i^T Gc s_i - theta_i^2
        for (int i = tid; i < b; i += NT) {
            double d = 0.0;
            for (int r = 0; r < b; ++r) d += L.A[r][i] * L.V[r][i];
            const double t = L.th[i];
            L.res[i] = sqrt(fmax(d - t * t, 0.0));
            st->theta[i] = t;
        }
        __syncthreads();
        if (tid == 0) bounds(st, L.th, L.res, b, k);
        // S^T Gc S into Gc (reads only A and V), then symmetrise
        for (int e = tid; e < b * b; e += NT) {
            const int i = e / b, j = e % b;
            double v = 0.0;
            for (int r = 0; r < b; ++r) v += L.A[r][i] * L.V[r][j];
            L.Gc[i][j] = v;
        }
        __syncthreads();
        for (int e = tid; e < b * b; e += NT) {
            const int i = e / b, j = e % b;
            if (i < j) {
                const double v = 0.5 * (L.Gc[i][j] + L.Gc[j][i]);
                L.Gc[i][j] = v;
                L.Gc[j][i] = v;
            }
        }
        __syncthreads();
    }

    // Left-looking Cholesky Gc = Lc Lc^T, Lc in the lower triangle.  A pivot
    // that kept no more than piv_tol of its original size marks a column whose
    // direction is already spanned by earlier ones; it is dropped from the
    // next basis (its column of C' is zero).
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
        for (int i = j + 1 + tid; i < b; i += NT) {
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
    // Lc^{-1} into V, one column per thread (forward substitution)
    for (int j = tid; j < b; j += NT) {
        for (int i = 0; i < b; ++i) L.V[i][j] = 0.0;
        L.V[j][j] = 1.0 / L.Gc[j][j];
        for (int i = j + 1; i < b; ++i) {
            double v = 0.0;
            for (int m = j; m < i; ++m) v -= L.Gc[i][m] * L.V[m][j];
            L.V[i][j] = v / L.Gc[i][i];
        }
    }
    __syncthreads();
    // C' = S Lc^{-T}; dropped columns are zero
    int nonfinite = 0;
    for (int e = tid; e < B * B; e += NT) {
        const int r = e / B, j = e % B;
        double v = 0.0;
        if (r < b && j < b && !L.dead[j]) {
            for (int m = 0; m <= j; ++m) v += L.A[r][m] * L.V[j][m];
        }
        nonfinite |= !isfinite(v);
        st->C[e] = v;
    }
    for (int j = tid; j < B; j += NT) st->e_x[j] = L.e_new[j];
    nonfinite = (int)wave_sum((double)nonfinite);
    if (tid == 0) {
        int nd = 0;
        for (int j = 0; j < b; ++j) nd += L.dead[j];
        st->dead = nd;
        int fl = init == RR_START ? 0 : st->flags;  // a new solve starts with clean flags
        if (nd) fl |= SF_REPAIRED;
        if (nonfinite) fl |= SF_NONFINITE;
        st->flags = fl;
        if (init == RR_REFILL) {
            // the refilled block sits in buffer 0; the schedule goes on
            st->ycur = 0;
            st->maxbound = INFINITY;
            st->sweeps = 0;
            st->refill = 0;
        } else {
            if (init) {
                st->iter = 0;
                st->maxbound = INFINITY;
                st->maxres = INFINITY;
                st->sweeps = 0;
                st->refill = 0;
            } else {
                st->iter += 1;
            }
            phase_control(st, rule, init);
        }
    }
    __syncthreads();
    publish_summary(st, views[blockIdx.x].host_sum, blockDim.x);
}

hipError_t launch_rr_solve2(const Batch &bt, int init, int max_sweeps, const PhaseRule &rule, hipStream_t s);

// Widths up to 32 run the element-parallel kernel of sbmds_rr.hip; 64 runs
// the kernel above.
hipError_t launch_rr_solve(const Batch &bt, int init, int max_sweeps, const PhaseRule &rule, hipStream_t s) {
    if (bt.B <= 32) return launch_rr_solve2(bt, init, max_sweeps, rule, s);
    const double piv_tol = 1e-10;
    const dim3 blk(kSolveThreads), grid(bt.nprob);
    switch (bt.B) {
        case 32: hipLaunchKernelGGL((k_rr_solve<32>), grid, blk, 0, s, bt.views, bt.b, bt.k, piv_tol, init, max_sweeps, rule); break;
        case 64: hipLaunchKernelGGL((k_rr_solve<64>), grid, blk, 0, s, bt.views, bt.b, bt.k, piv_tol, init, max_sweeps, rule); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sbmds
