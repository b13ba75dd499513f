// The b x b float64 step of block subspace iteration for kernel widths
// B <= 32: one workgroup per problem, one LDS-resident matrix element per
// thread (or a few), every step parallel over elements.  It runs either as
// its own kernel or inside the SpMM, in the block that completes the Gram
// reduction.
//
// Mathematics as in sbmds_small.hip (Rayleigh-Ritz on H = X^T B X, residual
// norms from the Gram of B X, error bounds, CholQR of the next block):
//   1. H = S Theta S^T by cyclic Jacobi.  A sweep is B - 1 rounds; round m
//      rotates every index pair {i, i ^ m} at once (for B a power of two the
//      pairs of one round are disjoint and the B - 1 rounds cover every pair
//      once).  A rotation leaves a 2 x 2 block of H (rows of one pair,
//      columns of another) depending only on that block, so each thread
//      computes its element(s) from four values of the previous round's
//      matrix (ping-pong buffers).  The rotations of round m + 1 need only
//      three entries per pair of the matrix round m produces; the element
//      threads compute those entries from the same old values and the next
//      rotations in the same step, so a round costs one barrier and one
//      rotation latency.
//   2. Ritz values sorted descending (padding columns last), Zmap = C S_k
//      Theta_k^{1/2}, residuals ||B x_i - theta_i x_i||^2 = s_i^T Gc s_i -
//      theta_i^2, error bounds per gap-separated cluster (one thread per
//      Ritz value).
//   3. S^T Gc S = L L^T (right-looking, in place, one element per thread and
//      one barrier per pivot) and C' = S L^{-T} (one row per thread).
// In `init` mode only step 3 runs, with S = I.
#pragma once

#include "sbmds_bounds.h"

namespace sbmds {

// A CholQR pivot that fell below this fraction of its starting value drops
// its column (the block lost rank there).
constexpr double kPivTol = 1e-10;

template <int B>
struct RRShape {
    static constexpr int NT = (B * B < 64) ? 64 : (B * B > 256 ? 256 : B * B);
    static constexpr int EPT = (B * B + NT - 1) / NT;  // matrix elements per thread
};

template <int B>
struct RRLds {
    double A[2][B][B + 1];  // H during Jacobi (ping-pong)
    double V[2][B][B + 1];  // accumulated rotations (ping-pong)
    double G[B][B + 1];     // centred Gram Gc, then S^T Gc S
    double Cold[B][B + 1];  // basis transform H was computed with
    double S[B][B + 1];     // sorted Ritz vectors
    double GS[B][B + 1];    // Gc S, then the Cholesky factor
    double2 rot[2][B];      // rotation of a round per index i: (c, -s) if i is the lower index of its pair, else (c, s)
    double e_new[B], e_x[B], th[B], res[B], linv[B], w[B], gd[B];
    double bnd[B], rres[B];
    double red[2][16];  // one slot per wave of a block of up to 1024 threads
    int perm[B], dead[B], nonpos[B];
};

template <int NT>
__device__ __forceinline__ double rr_block_sum(double v, double (&red)[16]) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    constexpr int NW = (NT + 63) / 64;
    if (NW == 1) return v;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += red[i];
    return s;
}

template <int NT>
__device__ __forceinline__ void rr_block_sum2(double &a, double &c, double (&red)[2][16]) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        a += __shfl_xor(a, m);
        c += __shfl_xor(c, m);
    }
    constexpr int NW = (NT + 63) / 64;
    if (NW == 1) return;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    a = 0.0;
    c = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        a += red[0][i];
        c += red[1][i];
    }
}

// 1/sqrt(x) for normal positive x: hardware estimate and two Newton steps
// (a few ulp).
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - 0.5 * x * y * y);
    y = y * (1.5 - 0.5 * x * y * y);
    return y;
}

// Rotation (c, s) of an index pair (p < q) that annihilates A_pq (the
// classical symmetric Schur rotation, smaller-angle root), branch-free.  The
// tangent t only needs to be close (hardware reciprocal estimates on
// operands scaled by a power of two): a rough t leaves a small off-diagonal
// entry for later rounds.  c = 1/sqrt(1 + t^2) and s = t c are accurate to
// a few ulp, so the rotation is orthogonal to rounding -- the residual
// formula s^T Gc s - theta^2 relies on unit Ritz vectors.
__device__ __forceinline__ void pair_rotation(double app, double aqq, double apq, double &c, double &s) {
    const bool rot = fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * (fabs(app) + fabs(aqq));
    const double th0 = aqq - app, ph0 = 2.0 * apq;
    const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(th0), fabs(ph0)));
    const double th = __builtin_amdgcn_ldexp(th0, -ex), ph = __builtin_amdgcn_ldexp(ph0, -ex);
    const double q = th * th + ph * ph;  // in [1/4, 2) when rot
    const double r = q * __builtin_amdgcn_rsq(q);
    const double t = (th >= 0.0 ? ph : -ph) * __builtin_amdgcn_rcp(fabs(th) + r);
    const double cc = rsqrt_nr(1.0 + t * t);
    c = rot ? cc : 1.0;
    s = rot ? t * cc : 0.0;
}

// Entry (i, j) after one round of rotations.  Row i of the rotated matrix is
// c_i row_i + t_i row_{i^m} with (c_i, t_i) the rotation stored for index i
// (t_i = -s for the lower index of the pair, +s for the upper), and the same
// for columns; a_ij = A[i][j], a_pj = A[i^m][j], a_ip = A[i][j^m], a_pp =
// A[i^m][j^m].
__device__ __forceinline__ double rotate_entry(double2 ri, double2 rj, double a_ij, double a_pj, double a_ip,
                                               double a_pp) {
    return rj.x * (ri.x * a_ij + ri.y * a_pj) + rj.y * (ri.x * a_ip + ri.y * a_pp);
}

// Lower index of pair t of round m (m in [1, B)): pairs {p, p ^ m} with the
// highest set bit of m clear in p.
__device__ __forceinline__ int round_pair_low(int t, int m) {
    const int hb = 31 - __builtin_clz(m);
    return ((t >> hb) << (hb + 1)) | (t & ((1 << hb) - 1));
}

// One Jacobi round m on the buffers of parity CUR (a compile-time constant,
// so every LDS address is a register plus an immediate).  Every thread
// rotates its element(s) of H and of the accumulated rotations.  With NEXT
// (every round of a sweep but the last) each thread also forms the entries
// (p, p), (q, q), (p, q) of the rotated H for pair tp = {p, q} of round
// m + 1 and that pair's rotation, from the same old values, and the first
// B / 2 threads store it: a round needs one barrier.
template <int B, int NT, int EPT, int CUR, bool NEXT>
__device__ __forceinline__ void jacobi_round(RRLds<B> &L, int tid, int m, int tp) {
    const bool act = tid < NT;  // element thread (the block may be larger)
    const double(*Ac)[B + 1] = L.A[CUR];
    const double(*Vc)[B + 1] = L.V[CUR];
    const double2 *rot = L.rot[CUR];
    // all reads of the round come before its writes (the compiler cannot
    // tell the two parities apart through the row pointers)
    int p = 0, q = 0;
    double2 rp{}, rq{};
    double pp[4], qq[4], pq[4];
    if (NEXT && act) {
        p = round_pair_low(tp, m + 1);
        q = p ^ (m + 1);
        const int pm = p ^ m, qm = q ^ m;
        rp = rot[p];
        rq = rot[q];
        pp[0] = Ac[p][p], pp[1] = Ac[pm][p], pp[2] = Ac[p][pm], pp[3] = Ac[pm][pm];
        qq[0] = Ac[q][q], qq[1] = Ac[qm][q], qq[2] = Ac[q][qm], qq[3] = Ac[qm][qm];
        pq[0] = Ac[p][q], pq[1] = Ac[pm][q], pq[2] = Ac[p][qm], pq[3] = Ac[pm][qm];
    }
    double an[EPT], vn[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = tid + k * NT;
        an[k] = vn[k] = 0.0;
        if (act && e < B * B) {
            const int i = e / B, j = e % B, im = i ^ m, jm = j ^ m;
            const double2 ri = rot[i], rj = rot[j];
            an[k] = rotate_entry(ri, rj, Ac[i][j], Ac[im][j], Ac[i][jm], Ac[im][jm]);
            vn[k] = rj.x * Vc[i][j] + rj.y * Vc[i][jm];
        }
    }
    double c = 1.0, sn = 0.0;
    if (NEXT && act) {
        const double app = rotate_entry(rp, rp, pp[0], pp[1], pp[2], pp[3]);
        const double aqq = rotate_entry(rq, rq, qq[0], qq[1], qq[2], qq[3]);
        const double apq = rotate_entry(rp, rq, pq[0], pq[1], pq[2], pq[3]);
        pair_rotation(app, aqq, apq, c, sn);
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = tid + k * NT;
        if (act && e < B * B) {
            L.A[CUR ^ 1][e / B][e % B] = an[k];
            L.V[CUR ^ 1][e / B][e % B] = vn[k];
        }
    }
    if (NEXT && tid < B / 2) {
        L.rot[CUR ^ 1][p] = double2{c, -sn};
        L.rot[CUR ^ 1][q] = double2{c, sn};
    }
    __syncthreads();
}

// One Rayleigh-Ritz / CholQR step of the problem `view` by a whole
// workgroup of NBLK threads (the standalone kernel, NBLK = RRShape::NT, or
// the block of another kernel that finished the Gram reduction, NBLK =
// 1024): the first RRShape::NT threads own the matrix elements, the others
// only take part in the barriers.  The caller has checked that the problem
// is in this phase (or `init`).  The Gram sums are read with coherent loads:
// the calling kernel may have just written them from this block.
template <int B, int NBLK>
__device__ __forceinline__ void rr_step(const ProbView &view, RRLds<B> &L, int b, int k, double piv_tol, int init,
                                        int max_sweeps, const PhaseRule &rule) {
    constexpr int NT = RRShape<B>::NT, EPT = RRShape<B>::EPT;
    constexpr int E = B * (B + 1) / 2;
    static_assert(NBLK >= NT && NBLK % 64 == 0, "whole waves, at least the element threads");
    SolveState *__restrict__ st = view.st;
    const double n = (double)view.n;
    const int tid = threadIdx.x;
    const bool act = tid < NT;  // element thread
    const double inv_n = 1.0 / n;
    static_assert(NT % B == 0, "column index of a thread is the same for all its elements");
    Ctl ctl;
    if (tid == 0) ctl = load_ctl(st);

    // ---- stage the inputs (independent loads)
    if (tid < B) {
        L.e_new[tid] = ld_coherent(st->Ge + E + tid);
        L.e_x[tid] = st->e_x[tid];
    }
    double graw[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * NT;
        graw[q] = 0.0;
        if (act && e < B * B) {
            const int i = e / B, j = e % B;
            const int lo = i < j ? i : j, hi = i < j ? j : i;
            graw[q] = ld_coherent(st->Ge + lo * B - (lo * (lo - 1)) / 2 + (hi - lo));
            L.Cold[i][j] = st->C[e];
            if (!init) {
                L.A[0][i][j] = 0.5 * (st->Hs[i * B + j] + st->Hs[j * B + i]);
                L.V[0][i][j] = (i == j) ? 1.0 : 0.0;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * NT;
        if (act && e < B * B) {
            const int i = e / B, j = e % B;
            const double g = graw[q] - L.e_new[i] * L.e_new[j] * inv_n;
            L.G[i][j] = g;
            if (i == j) L.gd[i] = g;  // pivot reference of the init factorisation
        }
    }

    int cur = 0;
    if (!init) {
        // ---- 1. Jacobi
        const int tp = tid % (B / 2);  // pair whose next rotation this thread forms
        int sweep = 0;
        for (; sweep < max_sweeps; ++sweep) {
            double off = 0.0, dia = 0.0;
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                const int e = tid + q * NT;
                if (act && e < B * B) {
                    const int i = e / B, j = e % B;
                    const double a = L.A[cur][i][j];
                    if (i == j) dia += a * a;
                    else off += a * a;
                }
            }
            if (tid < B / 2) {
                // rotations of round 1
                const int p = round_pair_low(tp, 1), qq = p ^ 1;
                double c, sn;
                pair_rotation(L.A[cur][p][p], L.A[cur][qq][qq], L.A[cur][p][qq], c, sn);
                L.rot[cur][p] = double2{c, -sn};
                L.rot[cur][qq] = double2{c, sn};
            }
            rr_block_sum2<NBLK>(off, dia, L.red);
            __syncthreads();  // rotations of round 1 visible (the sum has no barrier for one wave)
            if (!(off > 1e-24 * dia) || dia == 0.0) break;
            for (int m = 1; m < B - 1; ++m) {
                if (cur == 0) jacobi_round<B, NT, EPT, 0, true>(L, tid, m, tp);
                else jacobi_round<B, NT, EPT, 1, true>(L, tid, m, tp);
                cur ^= 1;
            }
            if (cur == 0) jacobi_round<B, NT, EPT, 0, false>(L, tid, B - 1, tp);
            else jacobi_round<B, NT, EPT, 1, false>(L, tid, B - 1, tp);
            cur ^= 1;
        }
        if (tid == 0) ctl.sweeps = sweep;
        // ---- 2. sort (padding columns last), Ritz vectors
        if (tid < B) {
            const double mine = tid < b ? L.A[cur][tid][tid] : -INFINITY;
            int rank = 0;
            for (int o = 0; o < B; ++o) {
                const double other = o < b ? L.A[cur][o][o] : -INFINITY;
                rank += (other > mine) || (other == mine && o < tid);
            }
            L.perm[rank] = tid;
        }
        __syncthreads();
        if (tid < B) L.th[tid] = L.A[cur][L.perm[tid]][L.perm[tid]];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * NT;
            if (act && e < B * B) {
                const int i = e / B, j = e % B;
                L.S[i][j] = L.V[cur][i][L.perm[j]];
            }
        }
        __syncthreads();
        // Zmap = C S_k Theta^{1/2} (first k columns), Gc S, and the weights
        // w = C^T e_x for the shift of the embedding
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * NT;
            if (act && e < B * B) {
                const int i = e / B, j = e % B;
                double z = 0.0, g = 0.0;
#pragma unroll 8
                for (int a = 0; a < B; ++a) {
                    z += L.Cold[i][a] * L.S[a][j];
                    g += L.G[i][a] * L.S[a][j];
                }
                const double scale = (j < k && j < b) ? sqrt(fmax(L.th[j], 0.0)) : 0.0;
                st->Zmap[i * B + j] = z * scale;
                L.GS[i][j] = g;
            }
        }
        if (tid < B) {
            double w = 0.0;
            for (int r = 0; r < B; ++r) w += L.e_x[r] * L.Cold[r][tid];
            L.w[tid] = w;
        }
        __syncthreads();
        if (tid < B) {
            const int j = tid;
            double d = 0.0, zs = 0.0;
            for (int r = 0; r < B; ++r) {
                d += L.S[r][j] * L.GS[r][j];
                zs += L.w[r] * L.S[r][j];
            }
            const double scale = (j < k && j < b) ? sqrt(fmax(L.th[j], 0.0)) : 0.0;
            st->zshift[j] = zs * scale * inv_n;
            L.res[j] = sqrt(fmax(d - L.th[j] * L.th[j], 0.0));
            if (j < b) st->theta[j] = L.th[j];
        }
        __syncthreads();
        // error bounds: one thread per Ritz value, clusters found by scanning
        // neighbours (same clusters as the sequential rule)
        if (tid < b) {
            const double *th = L.th;
            double floor_mag = INFINITY;
            for (int i = 0; i < b; ++i) floor_mag = fmin(floor_mag, fabs(th[i]));
            auto close = [&](int x, int y) { return fabs(th[x] - th[y]) <= 1e-3 * fmax(fabs(th[x]), fabs(th[y])); };
            int i0 = tid, j0 = tid;
            while (i0 > 0 && close(i0 - 1, i0)) --i0;
            while (j0 + 1 < b && close(j0, j0 + 1)) ++j0;
            double r2 = 0.0;
            for (int x = i0; x <= j0; ++x) r2 += L.res[x] * L.res[x];
            double gap = INFINITY;
            if (i0 > 0) gap = fmin(gap, th[i0 - 1] - th[i0]);
            if (j0 + 1 < b) gap = fmin(gap, th[j0] - th[j0 + 1]);
            const double lo = th[j0];
            gap = fmin(gap, lo > 0.0 ? lo - floor_mag : (-lo) - floor_mag);
            const double a = fabs(th[tid]);
            double bnd = L.res[tid];
            if (gap > 0.0) bnd = fmin(bnd, r2 / gap);
            const double rel = a > 0.0 ? bnd / a : INFINITY;
            st->bound[tid] = rel;
            st->res[tid] = L.res[tid];
            L.bnd[tid] = rel;
            L.rres[tid] = a > 0.0 ? L.res[tid] / a : INFINITY;
            L.nonpos[tid] = th[tid] <= 0.0 ? 1 : 0;
        }
        __syncthreads();
        if (tid == 0) {
            double mb = 0.0, mr = 0.0;
            int np_ = 0;
            for (int i = 0; i < k && i < b; ++i) {
                mb = fmax(mb, L.bnd[i]);
                mr = fmax(mr, L.rres[i]);
                np_ += L.nonpos[i];
            }
            ctl.maxbound = mb;
            ctl.maxres = mr;
            ctl.nonpos = np_;
        }
        // S^T Gc S into G (Gc is no longer needed)
        double sg[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * NT;
            sg[q] = 0.0;
            if (act && e < B * B) {
                const int i = e / B, j = e % B;
                double g = 0.0;
#pragma unroll 8
                for (int r = 0; r < B; ++r) g += L.S[r][i] * L.GS[r][j];
                sg[q] = g;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * NT;
            if (act && e < B * B) {
                L.G[e / B][e % B] = sg[q];
                if (e / B == e % B) L.gd[e / B] = sg[q];
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * NT;
            if (act && e < B * B) {
                const int i = e / B, j = e % B;
                L.S[i][j] = (i == j) ? 1.0 : 0.0;
            }
        }
    }
    __syncthreads();

    // ---- 3. right-looking Cholesky of G, in place: at pivot m every thread
    // forms column m of the factor from the updated column m of G (into GS)
    // and downdates its own trailing element(s); one barrier per pivot.
    // Pivot m is dead (its column dropped) for padding columns or when it
    // lost its relative size against the diagonal it started from.
    int ndead = 0;
#pragma unroll
    for (int m = 0; m < B; ++m) {
        // every read first, then branch-free arithmetic, then the writes
        const double d = L.G[m][m];
        const double om = L.gd[m];
        double gim[EPT], gjm[EPT], gij[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * NT;
            const int i = (e / B) % B, j = e % B;  // in range for every thread
            gim[q] = L.G[i][m];
            gjm[q] = L.G[j][m];
            gij[q] = L.G[i][j];
        }
        const bool isdead = (m >= b) || !(d > piv_tol * om) || !(om > 0.0) || !isfinite(d);
        const double inv = rsqrt_nr(isdead ? 1.0 : d);
        const double sc = isdead ? 0.0 : inv;
        const double lmm = isdead ? 1.0 : d * inv;
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = tid + q * NT;
            if (act && e < B * B) {
                const int i = e / B, j = e % B;
                const double lim = gim[q] * sc;
                // column m of the factor (rows >= m) and the trailing block:
                // neither is read at this pivot
                if (j == m && i >= m) L.GS[i][m] = (i == m) ? lmm : lim;
                if (i > m && j > m) L.G[i][j] = gij[q] - lim * (gjm[q] * sc);
            }
        }
        if (tid == 0) {
            L.dead[m] = isdead ? 1 : 0;
            L.linv[m] = inv;
            ndead += isdead ? 1 : 0;
        }
        __syncthreads();
    }
    // C' = S L^{-T}: row r solves L c = S[r, :]^T
    int nonfinite = 0;
    if (tid < B) {
        double c[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            double acc = L.S[tid][j];
#pragma unroll
            for (int t = 0; t < j; ++t) acc -= L.GS[j][t] * c[t];
            c[j] = acc * L.linv[j];
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const double out = L.dead[j] ? 0.0 : c[j];
            nonfinite |= !isfinite(out);
            st->C[tid * B + j] = out;
        }
        st->e_x[tid] = L.e_new[tid];
    }
    nonfinite = (int)rr_block_sum<NBLK>((double)nonfinite, L.red[0]);
    if (tid == 0) {
        if (init == RR_START) ctl.flags = 0;  // a new solve starts with clean flags
        ctl.dead = ndead - (B - b);
        if (ndead > B - b) ctl.flags |= SF_REPAIRED;
        if (nonfinite) ctl.flags |= SF_NONFINITE;
        if (init == RR_REFILL) {
            // the refilled block sits in buffer 0; the schedule goes on
            ctl.ycur = 0;
            ctl.maxbound = INFINITY;
            ctl.sweeps = 0;
            st->refill = 0;
        } else {
            if (init) {
                ctl.iter = 0;
                ctl.maxbound = INFINITY;
                ctl.maxres = INFINITY;
                ctl.sweeps = 0;
                st->refill = 0;
            } else {
                ctl.iter += 1;
            }
            phase_control(ctl, rule, init);
        }
        store_ctl(st, ctl);
    }
    __syncthreads();
    publish_summary(st, view.host_sum, NBLK);
}

template <int B>
__global__ __launch_bounds__(RRShape<B>::NT) void k_rr_solve2(const ProbView *__restrict__ views, int b, int k,
                                                              double piv_tol, int init, int max_sweeps,
                                                              PhaseRule rule) {
    __shared__ RRLds<B> L;
    const ProbView &v = views[blockIdx.x];
    if (!init && (v.st->done || v.st->phase != rule.phase)) return;  // uniform
    if (init == RR_REFILL && !v.st->refill) return;
    rr_step<B, RRShape<B>::NT>(v, L, b, k, piv_tol, init, max_sweeps, rule);
}


}  // namespace sbmds
