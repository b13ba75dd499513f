// Error bounds of the Ritz values (shared by both small-solver variants).
#pragma once

#include "sbmds_common.h"

namespace sbmds {

// Error bounds for the k wanted Ritz values (one thread).  Ritz values closer
// than 1e-3 (relative) form a cluster; a cluster's gap is its distance to the
// nearest other Ritz value or to the magnitude of the smallest Ritz value of
// the block (which stands for the spectrum the block does not hold).  For
// each wanted value the bound is min(||r_i||, ||R_cluster||^2 / gap) / |theta_i|.
__device__ inline void bounds(SolveState *st, const double *th, const double *res, int b, int k) {
    double floor_mag = INFINITY;
    for (int i = 0; i < b; ++i) floor_mag = fmin(floor_mag, fabs(th[i]));
    double maxb = 0.0, maxr = 0.0;
    int nonpos = 0;
    int i = 0;
    while (i < b) {
        int j = i;
        while (j + 1 < b && fabs(th[j] - th[j + 1]) <= 1e-3 * fmax(fabs(th[j]), fabs(th[j + 1]))) ++j;
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

// Control fields of SolveState, held in registers by the thread that
// updates them (loaded together at kernel start, stored together at the
// end, so their global-memory latency is paid once).
struct Ctl {
    double maxbound, maxres;
    int iter, flags, dead, nonpos, sweeps;
    int ycur, zbuf, zmode, phase, done, pending_convert, phase_iters, total_iters;
    int iters[4];
    int sweeps_total, ymode;
    double hist[4];
};

__device__ inline Ctl load_ctl(const SolveState *st) {
    Ctl c;
    c.maxbound = st->maxbound;
    c.maxres = st->maxres;
    c.iter = st->iter;
    c.flags = st->flags;
    c.dead = st->dead;
    c.nonpos = st->nonpos;
    c.sweeps = st->sweeps;
    c.ycur = st->ycur;
    c.zbuf = st->zbuf;
    c.zmode = st->zmode;
    c.phase = st->phase;
    c.done = st->done;
    c.pending_convert = st->pending_convert;
    c.phase_iters = st->phase_iters;
    c.total_iters = st->total_iters;
    for (int i = 0; i < 4; ++i) c.iters[i] = st->iters[i];
    c.sweeps_total = st->sweeps_total;
    c.ymode = st->ymode;
    for (int i = 0; i < 4; ++i) c.hist[i] = st->hist[i];
    return c;
}

__device__ inline void store_ctl(SolveState *st, const Ctl &c) {
    st->maxbound = c.maxbound;
    st->maxres = c.maxres;
    st->iter = c.iter;
    st->flags = c.flags;
    st->dead = c.dead;
    st->nonpos = c.nonpos;
    st->sweeps = c.sweeps;
    st->ycur = c.ycur;
    st->zbuf = c.zbuf;
    st->zmode = c.zmode;
    st->phase = c.phase;
    st->done = c.done;
    st->pending_convert = c.pending_convert;
    st->phase_iters = c.phase_iters;
    st->total_iters = c.total_iters;
    for (int i = 0; i < 4; ++i) st->iters[i] = c.iters[i];
    st->sweeps_total = c.sweeps_total;
    st->ymode = c.ymode;
    for (int i = 0; i < 4; ++i) st->hist[i] = c.hist[i];
}

// Schedule bookkeeping after a Rayleigh-Ritz step.  In `init` mode it
// resets the control state for a new solve.
__device__ inline void phase_control(Ctl &st, const PhaseRule &rule, int init) {
    if (init) {
        st.ycur = 0;
        st.zbuf = 0;
        st.zmode = rule.mode;
        st.phase = 0;
        st.done = 0;
        st.pending_convert = 0;
        st.phase_iters = 0;
        st.total_iters = 0;
        for (int i = 0; i < 4; ++i) st.iters[i] = 0;
        st.sweeps_total = 0;
        st.ymode = rule.mode;
        for (int i = 0; i < 4; ++i) st.hist[i] = INFINITY;
        return;
    }
    // an iteration of this phase has run: nothing is pending from the phase
    // change that led here
    st.pending_convert = 0;
    // the block just produced (Y') becomes current; the basis the Ritz
    // vectors were taken from stays readable until the next SpMM overwrites it
    st.zbuf = st.ycur;
    st.zmode = st.ymode;  // the storage type of that block (a phase may start on the narrower one)
    st.ymode = rule.mode;
    st.ycur ^= 1;
    st.total_iters += 1;
    for (int i = 0; i < 4; ++i) st.iters[i] += (i == rule.phase) ? 1 : 0;
    st.sweeps_total += st.sweeps;
    st.hist[3] = st.hist[2];
    st.hist[2] = st.hist[1];
    st.hist[1] = st.hist[0];
    st.hist[0] = st.maxres;
    st.phase_iters += 1;
    if (st.flags & SF_NONFINITE) {
        st.done = 1;
        return;
    }
    if (rule.is_final) {
        if (st.maxbound <= rule.tol) st.done = 1;
        return;
    }
    const bool plateau = st.phase_iters >= 4 && st.hist[0] > 0.7 * st.hist[2] && st.hist[0] > 0.7 * st.hist[3];
    if (st.maxres <= rule.floor_res || plateau || st.phase_iters >= rule.cap) {
        st.phase += 1;
        st.pending_convert = 1;
        st.phase_iters = 0;
        for (int i = 0; i < 4; ++i) st.hist[i] = INFINITY;
    }
}

__device__ inline void phase_control(SolveState *st, const PhaseRule &rule, int init) {
    Ctl c = load_ctl(st);
    phase_control(c, rule, init);
    store_ctl(st, c);
}

// Copy the SolveState tail (Ritz values, bounds, control) to the pinned host
// summary of the problem, threads 0 .. nthreads - 1 of the block taking
// part.  Their global writes to st must be complete and visible (after a
// barrier).
__device__ inline void publish_summary(const SolveState *st, void *host, int nthreads) {
    static_assert(kSummaryOffset % 8 == 0 && kSummaryBytes % 8 == 0, "whole 8-byte words");
    if (!host) return;
    const uint64_t *src = reinterpret_cast<const uint64_t *>(reinterpret_cast<const char *>(st) + kSummaryOffset);
    uint64_t *dst = reinterpret_cast<uint64_t *>(host);
    for (int i = threadIdx.x; i < (int)(kSummaryBytes / 8); i += nthreads) dst[i] = src[i];
}

}  // namespace sbmds
