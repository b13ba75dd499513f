// Register-resident b x b float64 step for block widths B <= 16 (one wave).
//
// Same mathematics as k_rr_solve (Rayleigh-Ritz on H = X^T B X, residual
// norms from the Gram of B X, bounds, CholQR of the next block; see
// sbmds_small.hip), laid out so that the serial parts run on registers and
// cross-lane operations instead of LDS round trips:
//
//   * lane j owns column j of H in an XOR-permuted layout, a[r] = H[j^r][j];
//     Jacobi round M (M = 1..B-1) rotates every index pair {i, i^M} at once,
//     so a lane's partner column is lane j^M and every register index used
//     is a compile-time constant (r, r^M); the exchanges are DPP moves;
//   * the Ritz vectors, the Gram products and the triangular solve use
//     LDS with lane-uniform addresses (broadcast reads, no dependent chains);
//   * the Cholesky factorisation is left-looking with the pivot row
//     broadcast from its owning lane.
// Lanes >= B hold replicas of lanes j mod B so that every lane takes part in
// the shuffles with well-defined data.
#include "sbmds_bounds.h"

namespace sbmds {

namespace {

template <int M>
constexpr int high_bit() {
    int h = 1;
    while ((h << 1) <= M) h <<= 1;
    return h;
}

__device__ __forceinline__ double bcast(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// x from lane (lane ^ M), M < 16, with DPP moves (ALU path, no LDS round
// trip).  Within a row of 16 lanes: quad_perm gives xor 1..3, row_half_mirror
// is xor 7 and row_mirror is xor 15; any M < 16 is a product of at most one
// of each.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int M>
__device__ __forceinline__ int xor_i(int x) {
    static_assert(M > 0 && M < 16, "xor mask within a DPP row");
    constexpr int A = (M & 8) ? 15 : 0;
    constexpr int M1 = M ^ A;
    constexpr int Bm = (M1 & 4) ? 7 : 0;
    constexpr int C = M1 ^ Bm;  // 0..3
    if constexpr (A) x = dpp_i<0x140>(x);   // row_mirror
    if constexpr (Bm) x = dpp_i<0x141>(x);  // row_half_mirror
    if constexpr (C == 1) x = dpp_i<0xB1>(x);  // quad_perm [1,0,3,2]
    if constexpr (C == 2) x = dpp_i<0x4E>(x);  // quad_perm [2,3,0,1]
    if constexpr (C == 3) x = dpp_i<0x1B>(x);  // quad_perm [3,2,1,0]
    return x;
}
template <int M>
__device__ __forceinline__ double xor_d(double x) {
    if constexpr (M == 0) {
        return x;
    } else {
        const int lo = xor_i<M>(__double2loint(x));
        const int hi = xor_i<M>(__double2hiint(x));
        return __hiloint2double(hi, lo);
    }
}

// Register-pair loop of one round, unrolled with compile-time indices.
template <int B, int M, int R>
struct PairLoop;

// One Jacobi round: rotate all pairs {i, i ^ M} of indices.
template <int B, int M, int R>
struct PairLoop {
    static __device__ __forceinline__ void run(double (&a)[B], int jj, double c, double s) {
        constexpr int HB = high_bit<M>();
        if constexpr ((R & HB) == 0) {
            constexpr int R2 = R ^ M;
            const bool jlo = (jj & HB) == 0;
            // rows i = jj ^ R and i ^ M form one rotated pair; its parameters
            // were computed by lane jj ^ R
            const double cr = xor_d<R>(c);
            const double sr = xor_d<R>(s);
            const bool ilo = ((jj ^ R) & HB) == 0;
            const double x00 = a[R];           // (row i,   col jj)
            const double x10 = a[R2];          // (row i^M, col jj)
            const double x01 = xor_d<M>(a[R2]); // (row i,   col jj^M)
            const double x11 = xor_d<M>(a[R]);  // (row i^M, col jj^M)
            const double lo0 = ilo ? x00 : x10, hi0 = ilo ? x10 : x00;
            const double lo1 = ilo ? x01 : x11, hi1 = ilo ? x11 : x01;
            const double nlo0 = cr * lo0 - sr * hi0, nhi0 = sr * lo0 + cr * hi0;
            const double nlo1 = cr * lo1 - sr * hi1, nhi1 = sr * lo1 + cr * hi1;
            const double t00 = ilo ? nlo0 : nhi0, t10 = ilo ? nhi0 : nlo0;  // col jj
            const double t01 = ilo ? nlo1 : nhi1, t11 = ilo ? nhi1 : nlo1;  // col jj^M
            a[R] = jlo ? (c * t00 - s * t01) : (s * t01 + c * t00);
            a[R2] = jlo ? (c * t10 - s * t11) : (s * t11 + c * t10);
        }
        if constexpr (R + 1 < B) PairLoop<B, M, R + 1>::run(a, jj, c, s);
    }
};

template <int B, int M>
__device__ __forceinline__ void jround(double (&a)[B], double (&v)[B], int jj) {
    constexpr int HB = high_bit<M>();
    const bool jlo = (jj & HB) == 0;  // column jj is the lower index of its pair
    const double pa0 = xor_d<M>(a[0]);
    const double pam = xor_d<M>(a[M]);
    const double app = jlo ? a[0] : pa0;
    const double aqq = jlo ? pa0 : a[0];
    const double apq = jlo ? a[M] : pam;  // both lanes use the lower lane's copy
    // branch-free (branches here make the unrolled rounds very slow to
    // compile): a negligible off-diagonal gives the identity rotation
    const bool rot = fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * (fabs(app) + fabs(aqq));
    const double tau = (aqq - app) / (2.0 * (rot ? apq : 1.0));
    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    const double c0 = 1.0 / sqrt(1.0 + t * t);
    const double c = rot ? c0 : 1.0;
    const double s = rot ? t * c0 : 0.0;
    PairLoop<B, M, 0>::run(a, jj, c, s);
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const double pv = xor_d<M>(v[i]);
        v[i] = jlo ? (c * v[i] - s * pv) : (s * pv + c * v[i]);
    }
}

template <int B, int M>
struct Rounds {
    static __device__ __forceinline__ void run(double (&a)[B], double (&v)[B], int jj) {
        jround<B, M>(a, v, jj);
        Rounds<B, M + 1>::run(a, v, jj);
    }
};
template <int B>
struct Rounds<B, B> {
    static __device__ __forceinline__ void run(double (&)[B], double (&)[B], int) {}
};

}  // namespace

template <int B>
__global__ __launch_bounds__(64) void k_rr_solve_reg(const ProbView *__restrict__ views, int b, int k,
                                                     double piv_tol, int init, int max_sweeps,
                                                     PhaseRule rule) {
    SolveState *__restrict__ st = views[blockIdx.x].st;
    const double n = (double)views[blockIdx.x].n;
    constexpr int E = B * (B + 1) / 2;
    if (!init && (st->done || st->phase != rule.phase)) return;
    __shared__ double Cold[B][B + 1];
    __shared__ double Gc[B][B + 1];
    __shared__ double Sm[B][B + 1];   // Ritz vectors, Sm[m][i] = S[m][i]
    __shared__ double Lf[B][B + 1];   // Cholesky factor, rows
    __shared__ double GSm[B][B + 1];  // Gc S
    __shared__ double e_new[B], e_x[B], th[B], res[B], linv[B];
    __shared__ int dead[B];
    const int lane = threadIdx.x;
    const int jj = lane & (B - 1);
    const double inv_n = 1.0 / n;

    for (int e = lane; e < B * B; e += 64) Cold[e / B][e % B] = st->C[e];
    for (int e = lane; e < B; e += 64) {
        e_new[e] = st->Ge[E + e];
        e_x[e] = st->e_x[e];
    }
    __syncthreads();
    for (int e = lane; e < B * B; e += 64) {
        const int a = e / B, c = e % B;
        const int lo = a < c ? a : c, hi = a < c ? c : a;
        const int pk = lo * B - (lo * (lo - 1)) / 2 + (hi - lo);
        Gc[a][c] = st->Ge[pk] - e_new[a] * e_new[c] * inv_n;
    }

    // ---- Ritz vectors (column jj of S) and values
    double s[B];
    double theta = 0.0;
    if (init) {
#pragma unroll
        for (int m = 0; m < B; ++m) s[m] = (m == jj) ? 1.0 : 0.0;
    } else {
        double a[B], v[B];
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int i = jj ^ r;
            a[r] = 0.5 * (st->Hs[i * B + jj] + st->Hs[jj * B + i]);
            v[r] = (r == jj) ? 1.0 : 0.0;
        }
        int sweep = 0;
        for (; sweep < max_sweeps; ++sweep) {
            double off = 0.0;
#pragma unroll
            for (int r = 1; r < B; ++r) off += a[r] * a[r];
            const bool own = lane < B;
            off = wsum(own ? off : 0.0);
            const double dia = wsum(own ? a[0] * a[0] : 0.0);
            if (!(off > 1e-24 * dia) || dia == 0.0) break;
            Rounds<B, 1>::run(a, v, jj);
        }
        if (lane == 0) st->sweeps = sweep;
        // rank of my Ritz value (padding columns jj >= b sort last)
        const double mine = jj < b ? a[0] : -INFINITY;
        int rank = 0;
#pragma unroll
        for (int r = 1; r < B; ++r) {
            const double o = __shfl_xor(mine, r);
            const int oj = jj ^ r;
            rank += (o > mine) || (o == mine && oj < jj);
        }
        // lane i takes the column whose rank is i
        int src = jj;
#pragma unroll
        for (int r = 1; r < B; ++r) {
            const int orank = __shfl_xor(rank, r);
            if (orank == jj) src = jj ^ r;
        }
        if (rank == jj) src = jj;
        const int src_lane = (lane & ~(B - 1)) | src;
#pragma unroll
        for (int m = 0; m < B; ++m) s[m] = __shfl(v[m], src_lane);
        theta = __shfl(a[0], src_lane);
    }
    if (lane < B) {
#pragma unroll
        for (int m = 0; m < B; ++m) Sm[m][jj] = s[m];
    }
    __syncthreads();

    // GSm column jj = Gc s (runtime loops over rows; s[] is indexed by the
    // unrolled inner loop only)
    double gs[B];  // column jj of S^T Gc S (or of Gc in init mode)
    if (!init) {
        const double scale = (jj < k && jj < b) ? sqrt(fmax(theta, 0.0)) : 0.0;
        double zs = 0.0;
        for (int r = 0; r < B; ++r) {
            double z = 0.0, g = 0.0;
#pragma unroll
            for (int m = 0; m < B; ++m) {
                z += Cold[r][m] * s[m];
                g += Gc[r][m] * s[m];
            }
            z *= scale;
            zs += e_x[r] * z;
            if (lane < B) {
                st->Zmap[r * B + jj] = z;
                GSm[r][jj] = g;
            }
        }
        if (lane < B) st->zshift[jj] = zs * inv_n;
        __syncthreads();
        double d = 0.0;
#pragma unroll
        for (int r = 0; r < B; ++r) d += s[r] * GSm[r][jj];
        if (lane < B) {
            th[jj] = theta;
            res[jj] = sqrt(fmax(d - theta * theta, 0.0));
            if (jj < b) st->theta[jj] = theta;
        }
        __syncthreads();
        if (lane == 0) bounds(st, th, res, b, k);
        // column jj of S^T Gc S
#pragma unroll
        for (int i = 0; i < B; ++i) {
            double g = 0.0;
            for (int r = 0; r < B; ++r) g += Sm[r][i] * GSm[r][jj];
            gs[i] = g;
        }
    } else {
#pragma unroll
        for (int i = 0; i < B; ++i) gs[i] = Gc[i][jj];
    }

    // ---- left-looking Cholesky of Gs: lane j owns row j (= column j)
    double l[B];
#pragma unroll
    for (int t = 0; t < B; ++t) l[t] = 0.0;
    int ndead = 0;
#pragma unroll
    for (int m = 0; m < B; ++m) {
        double d = gs[m];
#pragma unroll
        for (int t = 0; t < m; ++t) d -= l[t] * l[t];
        const double dm = bcast(d, m);
        const double om = bcast(gs[m], m);
        const bool isdead = (m >= b) || !(dm > piv_tol * om) || !(om > 0.0) || !isfinite(dm);
        ndead += isdead ? 1 : 0;
        const double lmm = isdead ? 1.0 : sqrt(dm);
        const double inv = 1.0 / lmm;
        double acc = gs[m];
#pragma unroll
        for (int t = 0; t < m; ++t) acc -= l[t] * bcast(l[t], m);
        if (jj == m) l[m] = lmm;
        else if (jj > m) l[m] = isdead ? 0.0 : acc * inv;
        if (lane == 0) {
            dead[m] = isdead ? 1 : 0;
            linv[m] = inv;
        }
    }
    if (lane < B) {
#pragma unroll
        for (int t = 0; t < B; ++t) Lf[jj][t] = l[t];
    }
    __syncthreads();
    // ---- C' = S L^{-T}: row r solves L c^T = S[r, :]^T (forward substitution)
    int nonfinite = 0;
    {
        double c[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            double acc = Sm[jj][j];
#pragma unroll
            for (int t = 0; t < j; ++t) acc -= Lf[j][t] * c[t];
            c[j] = acc * linv[j];
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const double out = dead[j] ? 0.0 : c[j];
            nonfinite |= !isfinite(out);
            if (lane < B) st->C[jj * B + j] = out;
        }
    }
    if (lane < B) st->e_x[jj] = e_new[jj];
    nonfinite = (int)wsum((double)(lane < B ? nonfinite : 0));
    if (lane == 0) {
        st->dead = ndead - (B - b);
        int fl = st->flags;
        if (ndead > B - b) fl |= SF_REPAIRED;
        if (nonfinite) fl |= SF_NONFINITE;
        st->flags = fl;
        if (init) {
            st->iter = 0;
            st->maxbound = INFINITY;
            st->maxres = INFINITY;
            st->sweeps = 0;
        } else {
            st->iter += 1;
        }
        phase_control(st, rule, init);
    }
}

hipError_t launch_rr_solve_reg(const Batch &bt, int init, int max_sweeps, const PhaseRule &rule, hipStream_t s) {
    const double piv_tol = 1e-10;
    const dim3 grid(bt.nprob), blk(64);
    switch (bt.B) {
        case 4: hipLaunchKernelGGL((k_rr_solve_reg<4>), grid, blk, 0, s, bt.views, bt.b, bt.k, piv_tol, init, max_sweeps, rule); break;
        case 8: hipLaunchKernelGGL((k_rr_solve_reg<8>), grid, blk, 0, s, bt.views, bt.b, bt.k, piv_tol, init, max_sweeps, rule); break;
        case 16: hipLaunchKernelGGL((k_rr_solve_reg<16>), grid, blk, 0, s, bt.views, bt.b, bt.k, piv_tol, init, max_sweeps, rule); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sbmds
