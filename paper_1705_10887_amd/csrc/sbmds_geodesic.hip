// Landmarks and the landmark block of the geodesic distance matrix on the
// device (Section 3): farthest-point sampling, Eq. (FarthestPoint) -- the
// first landmark is given, each further one is the vertex whose smallest
// distance to the landmarks chosen so far is largest (lowest vertex id on
// ties) -- and W = D_ll o D_ll, the squared distances between landmarks,
// averaged with its transpose, zero diagonal.
//
// Distances are shortest paths over the weighted graph (mesh edges with
// their lengths), in float64.  Every search is a frontier relaxation
// (Bellman-Ford restricted to the vertices whose distance just dropped)
// with atomicMin on the bit patterns of non-negative doubles, which order
// like the values.  Its result is the least fixed point of
// d[v] = min_u fl(d[u] + w_uv), d[src] = 0, which is also what Dijkstra
// computes (fl(x + w) is monotone in x and never below x), so the distances
// are those of a textbook Dijkstra bit for bit.
//
// Farthest-point step j searches from b_j only where it lowers the running
// minimum m[v] = min_t d(b_t, v): a relaxation whose candidate is not below
// m[v] is dropped.  m is 1-Lipschitz along edges (m[v] <= fl(m[u] + w_uv)),
// so a path through a vertex at or above its minimum never lowers the
// minimum beyond it, and the kept vertices get their exact distance.  The
// landmark block then comes from full searches, many sources at once, each
// keeping its distances at the landmark vertices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sbmds.h"
#include "sbmds_mlp_internal.h"  // api_fail

namespace sbmds {
namespace {

constexpr unsigned long long kInfBits = 0x7ff0000000000000ull;  // +inf
constexpr int kRoundGrid = 2048;                                 // blocks of a many-source round (grid-stride)
constexpr int kRoundsPerCheck = 4;                               // rounds launched between frontier checks

__device__ inline double as_d(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ inline unsigned long long as_b(double d) { return (unsigned long long)__double_as_longlong(d); }

// Appends x for every active lane with pred set: one atomicAdd per wave on
// the counter, each lane at the base plus its rank among the set lanes.
template <typename T>
__device__ inline void wave_append(T *list, int *cnt, bool pred, T x) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(cnt, __popcll(m));
    base = __shfl(base, leader);
    if (pred) list[base + __popcll(m & ((1ull << lane) - 1ull))] = x;
}

__global__ __launch_bounds__(256) void k_geo_fill_u64(unsigned long long *p, int64_t count, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ __launch_bounds__(256) void k_geo_fill_i32(int32_t *p, int64_t count, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = v;
}

// ---------------------------------------------------------------------------
// Farthest-point sampling.  State: mind[n] (bits), dist[n] (bits, +inf
// between steps), inq[n] (round stamp of the last queueing, 0 between
// steps), the touched list and two frontiers (global), the landmarks.
struct FpsState {
    unsigned long long *mind, *dist;
    int32_t *inq, *front[2], *touched;
    int32_t *lm;    // [l] landmarks (device)
    int *err;       // [1] set when a search exceeds its round limit
    // largest mind per chunk of kChunk vertices (value bits, lowest index of
    // it), a dirty flag per chunk and the list of dirty chunks
    unsigned long long *cval;
    int64_t *cidx;
    int32_t *cflag, *clist;
    int64_t nchunks;
};

constexpr int kSearchThreads = 1024;
constexpr int kSub = 8;  // threads per frontier vertex in a farthest-point search
constexpr int kChunk = 1024;

// (value, index) of the larger value, the lower index on ties (idx < 0: none)
__device__ inline void better(unsigned long long &bv, int64_t &bi, unsigned long long v, int64_t i) {
    if (i >= 0 && (bi < 0 || v > bv || (v == bv && i < bi))) {
        bv = v;
        bi = i;
    }
}

__device__ inline void wave_best(unsigned long long &bv, int64_t &bi) {
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) {
        const unsigned long long ov = __shfl_xor(bv, sh);
        const int64_t oi = __shfl_xor(bi, sh);
        better(bv, bi, ov, oi);
    }
}

// Initial chunk maxima: every mind is +inf, so each chunk's first vertex.
__global__ __launch_bounds__(256) void k_fps_chunks_init(FpsState s, int64_t n) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= s.nchunks) return;
    s.cval[c] = kInfBits;
    s.cidx[c] = c * kChunk;
    s.cflag[c] = 0;
}

template <typename T>
__device__ inline T ld_l2(const T *p) {  // bypasses the L1 cache
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One farthest-point step in one workgroup, with no host round trip: the
// pruned search from lm[j] in rounds over frontiers kept in global memory
// (their sizes in LDS), then mind takes the new distances and the state of
// the touched vertices is reset.  Data written during the search (frontier
// entries, distances, the touched list) is read back with L1-bypassing
// loads.
__global__ __launch_bounds__(kSearchThreads) void k_fps_search(FpsState s, const int32_t *__restrict__ rp,
                                                               const int32_t *__restrict__ ci,
                                                               const double *__restrict__ w, int64_t n, int j,
                                                               int last, int64_t max_rounds) {
    __shared__ int cnt[2];
    __shared__ int tcount;
    const int tid = threadIdx.x;
    const int32_t src = s.lm[j];
    if (tid == 0) {
        s.dist[src] = 0ull;
        s.inq[src] = 1;
        s.front[0][0] = src;
        s.touched[0] = src;
        cnt[0] = 1;
        cnt[1] = 0;
        tcount = 1;
    }
    __syncthreads();
    for (int64_t round = 0;; ++round) {
        const int in = (int)(round & 1);
        const int count = cnt[in];
        if (count == 0) break;  // the same for every thread (read after a barrier)
        if (round >= max_rounds) {
            if (tid == 0) s.err[0] = 1;
            break;
        }
        const int32_t *fin = s.front[in];
        int32_t *fout = s.front[in ^ 1];
        const int stamp = (int)round + 2;
        // kSub threads per frontier vertex, its edges strided over them
        for (int base = 0; base < count; base += kSearchThreads / kSub) {
            const int i = base + tid / kSub;
            if (i >= count) break;
            const int32_t u = ld_l2(fin + i);
            const double du = as_d(ld_l2(s.dist + u));
            for (int32_t e = rp[u] + tid % kSub; e < rp[u + 1]; e += kSub) {
                const int32_t v = ci[e];
                const unsigned long long cb = as_b(du + w[e]);
                bool first = false, queue = false;
                if (cb < s.mind[v] && cb < s.dist[v]) {
                    const unsigned long long old = atomicMin(&s.dist[v], cb);
                    if (cb < old) {
                        first = old == kInfBits;
                        queue = atomicExch(&s.inq[v], stamp) != stamp;
                    }
                }
                wave_append(s.touched, &tcount, first, v);
                wave_append(fout, &cnt[in ^ 1], queue, v);
            }
        }
        __syncthreads();  // every thread has read cnt[in]: it becomes the next output count
        if (tid == 0) cnt[in] = 0;
        __syncthreads();
    }
    __shared__ int ndirty;
    if (tid == 0) ndirty = 0;
    __syncthreads();
    const int tc = tcount;
    for (int i = tid; i < tc; i += kSearchThreads) {
        const int32_t v = ld_l2(s.touched + i);
        const unsigned long long d = ld_l2(s.dist + v);
        if (d < s.mind[v]) s.mind[v] = d;
        s.dist[v] = kInfBits;
        s.inq[v] = 0;
        const int32_t c = v / kChunk;
        const bool fresh = atomicExch(&s.cflag[c], 1) == 0;
        wave_append(s.clist, &ndirty, fresh, c);
    }
    __syncthreads();
    // the maxima of the chunks whose minima dropped: one wave per chunk
    const int lane = tid & 63, wave = tid >> 6, nd = ndirty;
    for (int q = wave; q < nd; q += kSearchThreads / 64) {
        const int32_t c = ld_l2(s.clist + q);
        unsigned long long bv = 0ull;
        int64_t bi = -1;
        for (int t = lane; t < kChunk; t += 64) {
            const int64_t v = (int64_t)c * kChunk + t;
            if (v < n) better(bv, bi, ld_l2(s.mind + v), v);
        }
        wave_best(bv, bi);
        if (lane == 0) {
            s.cval[c] = bv;
            s.cidx[c] = bi;
            s.cflag[c] = 0;
        }
    }
    __syncthreads();
    // the next landmark: the largest chunk maximum
    if (!last) {
        __shared__ unsigned long long wv[kSearchThreads / 64];
        __shared__ int64_t wi[kSearchThreads / 64];
        unsigned long long bv = 0ull;
        int64_t bi = -1;
        for (int64_t c = tid; c < s.nchunks; c += kSearchThreads) better(bv, bi, ld_l2(s.cval + c), ld_l2(s.cidx + c));
        wave_best(bv, bi);
        if (lane == 0) {
            wv[wave] = bv;
            wi[wave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long v0 = 0ull;
            int64_t i0 = -1;
            for (int q = 0; q < kSearchThreads / 64; ++q) better(v0, i0, wv[q], wi[q]);
            s.lm[j + 1] = (int32_t)i0;
        }
    }
}

// ---------------------------------------------------------------------------
// Full searches from S sources at once (the landmark block).  The frontier
// holds (source slot, vertex) pairs as slot << 32 | vertex.  Relaxations go
// in distance buckets (near-far): a pair whose new distance is below the
// current threshold joins the next round's frontier, one at or above it
// waits (once) on a far list; when the frontier runs empty the threshold
// moves past the smallest waiting distance and the far pairs below it
// return.  Rounds in hop order alone relax a vertex again each time a path
// with more hops but a smaller length reaches it (six to nine times per
// vertex on the meshes here); buckets a few edges wide keep that near one.
struct MultiState {
    unsigned long long *dist;  // [S][n]
    int32_t *inq;              // [S][n] round stamp of the last queueing
    int32_t *farf;             // [S][n] 1 while the pair waits on a far list
    int64_t *front[2];
    int64_t *far[2];           // far lists: one gets this bucket's pairs, the other the pairs kept at a refill
    int *cnt;                  // [3]
    int *fcnt;                 // [2]
    int *last;                 // [1] last round that had a non-empty frontier
    unsigned long long *fmin;  // [1] smallest distance on a far list (bits)
    double *thr;               // [1] the current bucket's threshold
};

__global__ __launch_bounds__(256) void k_ms_begin(MultiState s, const int32_t *__restrict__ lm, int first, int S,
                                                  int64_t n, double delta) {
    const int q = threadIdx.x;
    if (blockIdx.x != 0) return;
    if (q < S) {
        const int32_t src = lm[first + q];
        s.dist[(int64_t)q * n + src] = 0ull;
        s.inq[(int64_t)q * n + src] = 1;
        s.front[0][q] = ((int64_t)q << 32) | src;
    }
    if (q == 0) {
        s.cnt[0] = S;
        s.cnt[1] = 0;
        s.cnt[2] = 0;
        s.fcnt[0] = 0;
        s.fcnt[1] = 0;
        s.thr[0] = delta;
        s.fmin[0] = kInfBits;
    }
}

__global__ __launch_bounds__(256) void k_ms_round(MultiState s, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const double *__restrict__ w,
                                                  int64_t n, int round, int fsel) {
    const double thr = s.thr[0];
    const int in = round % 3, out = (round + 1) % 3, clr = (round + 2) % 3;
    const int64_t *fin = s.front[round & 1];
    int64_t *fout = s.front[(round + 1) & 1];
    const int count = s.cnt[in];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.cnt[clr] = 0;
        if (count > 0) s.last[0] = round;
    }
    for (int i = blockIdx.x * 256 + threadIdx.x; i < count; i += gridDim.x * 256) {
        const int64_t key = fin[i];
        const int64_t q = key >> 32;
        const int32_t u = (int32_t)(key & 0xffffffffll);
        unsigned long long *dq = s.dist + q * n;
        const double du = as_d(dq[u]);
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            const int32_t v = ci[e];
            const double cd = du + w[e];
            const unsigned long long cb = as_b(cd);
            bool queue = false, defer = false;
            if (cb < dq[v]) {
                const unsigned long long old = atomicMin(&dq[v], cb);
                if (cb < old) {
                    if (cd < thr) queue = atomicExch(&s.inq[q * n + v], round + 2) != round + 2;
                    else defer = atomicExch(&s.farf[q * n + v], 1) == 0;
                }
            }
            wave_append(fout, &s.cnt[out], queue, (q << 32) | v);
            wave_append(s.far[fsel], &s.fcnt[fsel], defer, (q << 32) | v);
        }
    }
}

// Smallest distance among the pairs on far list fsel.
__global__ __launch_bounds__(256) void k_ms_farmin(MultiState s, int fsel, int64_t n) {
    const int count = s.fcnt[fsel];
    const int64_t *lst = s.far[fsel];
    for (int i = blockIdx.x * 256 + threadIdx.x; i < count; i += gridDim.x * 256) {
        const int64_t key = lst[i];
        atomicMin(s.fmin, s.dist[(key >> 32) * n + (key & 0xffffffffll)]);
    }
}

// The next bucket's threshold: past the smallest waiting distance (k_ms_farmin
// wrote it), by delta; the minimum is reset for the next bucket.
__global__ void k_ms_next_thr(MultiState s, double delta) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    s.thr[0] = fmax(s.thr[0], as_d(s.fmin[0])) + delta;
    s.fmin[0] = kInfBits;
}

// Next bucket: the pairs of far list fsel below thr join the frontier of
// round `round` (stamped as queued for it), the others move to the other far
// list.  (A pair lowered below an earlier threshold after it was deferred
// was processed then; processing it again changes nothing.)
__global__ __launch_bounds__(256) void k_ms_refill(MultiState s, int fsel, int round, int64_t n) {
    const double thr = s.thr[0];
    const int count = s.fcnt[fsel];
    const int64_t *lst = s.far[fsel];
    for (int i = blockIdx.x * 256 + threadIdx.x; i < count; i += gridDim.x * 256) {
        const int64_t key = lst[i];
        const int64_t at = (key >> 32) * n + (key & 0xffffffffll);
        const bool below = as_d(s.dist[at]) < thr;
        bool to_near = false;
        if (below) {
            s.farf[at] = 0;
            to_near = atomicExch(&s.inq[at], round + 1) != round + 1;
        }
        wave_append(s.front[round & 1], &s.cnt[round % 3], to_near, key);
        wave_append(s.far[fsel ^ 1], &s.fcnt[fsel ^ 1], !below, key);
    }
}

// Largest edge weight (bits of a positive double), for the bucket width.
__global__ __launch_bounds__(256) void k_geo_wmax(const double *__restrict__ w, int64_t nnz,
                                                  unsigned long long *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < nnz) atomicMax(out, as_b(w[e]));
}

// D[(first + q) l + t] = distance from source first + q to landmark t.
__global__ __launch_bounds__(256) void k_ms_gather(const unsigned long long *__restrict__ dist,
                                                   const int32_t *__restrict__ lm, int64_t n, int64_t l, int first,
                                                   int S, double *__restrict__ D) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int q = blockIdx.y;
    if (t >= l || q >= S) return;
    D[(int64_t)(first + q) * l + t] = as_d(dist[(int64_t)q * n + lm[t]]);
}

// W = 1/2 (D o D + (D o D)^T), zero diagonal; each square rounded on its
// own (no fused multiply-add), as when the squares are formed first and then
// averaged.
__global__ __launch_bounds__(256) void k_geo_square_sym(const double *__restrict__ D, int64_t l,
                                                        double *__restrict__ W) {
#pragma clang fp contract(off)
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (j >= l || i >= l) return;
    const double a = D[i * l + j], b = D[j * l + i];
    const double a2 = a * a, b2 = b * b;
    W[i * l + j] = i == j ? 0.0 : 0.5 * (a2 + b2);
}

// Graph checks: rowptr monotone from 0, columns in range and not the row
// itself, weights finite and positive.  err = smallest failing row (or n).
__global__ __launch_bounds__(256) void k_geo_check(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   const double *__restrict__ w, int64_t n, int64_t nnz,
                                                   unsigned long long *__restrict__ err) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    bool bad = rp[v] > rp[v + 1] || rp[v] < 0 || rp[v + 1] > nnz || (v == 0 && rp[0] != 0) ||
               (v == n - 1 && rp[n] != nnz);
    if (!bad)
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            const double x = w[e];
            if (ci[e] < 0 || ci[e] >= n || ci[e] == v || !(x > 0.0) || !(x < INFINITY)) {
                bad = true;
                break;
            }
        }
    if (bad) atomicMin(err, (unsigned long long)v);
}

#define GCHK(expr)                                                                                          \
    do {                                                                                                    \
        hipError_t _e = (expr);                                                                             \
        if (_e != hipSuccess) return api_fail(SBMDS_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

struct DevMem {
    void *p = nullptr;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
};

unsigned nblk(int64_t c) { return (unsigned)((c + 255) / 256); }

int geodesic_impl(const int32_t *rp_in, const int32_t *ci_in, const double *w_in, int64_t n, int64_t nnz, int64_t l,
                  int32_t first, int32_t *landmarks, double *W, int mem, int batch, hipStream_t s) {
    const bool host = mem == SBMDS_MEM_HOST;
    const int S = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)batch, l, 256}));
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bn8 = (size_t)n * 8, bn4 = (size_t)n * 4;
    const size_t bS8 = (size_t)S * n * 8, bS4 = (size_t)S * n * 4;
    const size_t bL = (size_t)l * l * 8;
    const bool want_w = W != nullptr;
    const int64_t nch = (n + kChunk - 1) / kChunk;
    size_t total = 2 * al(bn8) + 4 * al(bn4) + al((size_t)l * 4) + 2 * al((size_t)nch * 8) + 2 * al((size_t)nch * 4) +
                   4096;
    if (want_w) total += al(bS8) + 2 * al(bS4) + 4 * al(bS8) + 2 * al(bL);
    if (host) total += al((size_t)(n + 1) * 4) + al((size_t)nnz * 4) + al((size_t)nnz * 8);
    DevMem mem_;
    if (hipMalloc(&mem_.p, total) != hipSuccess) {
        mem_.p = nullptr;
        return api_fail(SBMDS_ENOMEM, "hipMalloc of " + std::to_string(total) + " bytes failed");
    }
    char *q = (char *)mem_.p;
    auto take = [&](size_t b) {
        char *r = q;
        q += al(b);
        return (void *)r;
    };
    FpsState fs;
    fs.mind = (unsigned long long *)take(bn8);
    fs.dist = (unsigned long long *)take(bn8);
    fs.inq = (int32_t *)take(bn4);
    fs.front[0] = (int32_t *)take(bn4);
    fs.front[1] = (int32_t *)take(bn4);
    fs.touched = (int32_t *)take(bn4);
    fs.lm = (int32_t *)take((size_t)l * 4);
    MultiState ms{};
    double *D = nullptr, *Wd = nullptr;
    if (want_w) {
        ms.dist = (unsigned long long *)take(bS8);
        ms.inq = (int32_t *)take(bS4);
        ms.farf = (int32_t *)take(bS4);
        ms.front[0] = (int64_t *)take(bS8);
        ms.front[1] = (int64_t *)take(bS8);
        ms.far[0] = (int64_t *)take(bS8);
        ms.far[1] = (int64_t *)take(bS8);
        D = (double *)take(bL);
        Wd = (double *)take(bL);
    }
    fs.nchunks = (n + kChunk - 1) / kChunk;
    fs.cval = (unsigned long long *)take((size_t)fs.nchunks * 8);
    fs.cidx = (int64_t *)take((size_t)fs.nchunks * 8);
    fs.cflag = (int32_t *)take((size_t)fs.nchunks * 4);
    fs.clist = (int32_t *)take((size_t)fs.nchunks * 4);
    int *small = (int *)take(4096);
    fs.err = small;
    ms.cnt = small + 8;
    ms.last = small + 12;
    ms.fcnt = small + 20;
    ms.fmin = (unsigned long long *)(small + 24);
    unsigned long long *dwmax = (unsigned long long *)(small + 26);
    ms.thr = (double *)(small + 28);
    unsigned long long *derr = (unsigned long long *)(small + 16);
    const int32_t *rp = rp_in, *ci = ci_in;
    const double *w = w_in;
    if (host) {
        int32_t *a = (int32_t *)take((size_t)(n + 1) * 4);
        int32_t *b = (int32_t *)take((size_t)nnz * 4);
        double *c = (double *)take((size_t)nnz * 8);
        GCHK(hipMemcpyAsync(a, rp_in, (size_t)(n + 1) * 4, hipMemcpyHostToDevice, s));
        if (nnz) GCHK(hipMemcpyAsync(b, ci_in, (size_t)nnz * 4, hipMemcpyHostToDevice, s));
        if (nnz) GCHK(hipMemcpyAsync(c, w_in, (size_t)nnz * 8, hipMemcpyHostToDevice, s));
        rp = a;
        ci = b;
        w = c;
    }
    // the graph is checked before it is used as an index
    unsigned long long herr = (unsigned long long)n;
    GCHK(hipMemcpyAsync(derr, &herr, 8, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_geo_check, dim3(nblk(n)), dim3(256), 0, s, rp, ci, w, n, nnz, derr);
    GCHK(hipGetLastError());
    GCHK(hipMemcpyAsync(&herr, derr, 8, hipMemcpyDeviceToHost, s));
    GCHK(hipStreamSynchronize(s));
    if (herr != (unsigned long long)n)
        return api_fail(SBMDS_EINVAL, "graph row " + std::to_string(herr) +
                                          ": bad row pointers, a column out of range or on the diagonal, or a "
                                          "weight that is not finite and positive");

    hipLaunchKernelGGL(k_geo_fill_u64, dim3(nblk(n)), dim3(256), 0, s, fs.mind, n, kInfBits);
    hipLaunchKernelGGL(k_geo_fill_u64, dim3(nblk(n)), dim3(256), 0, s, fs.dist, n, kInfBits);
    hipLaunchKernelGGL(k_geo_fill_i32, dim3(nblk(n)), dim3(256), 0, s, fs.inq, n, 0);
    GCHK(hipMemcpyAsync(fs.lm, &first, 4, hipMemcpyHostToDevice, s));
    GCHK(hipGetLastError());
    const int64_t max_rounds = 4 * n + 64;  // a search settles within n rounds
    GCHK(hipMemsetAsync(fs.err, 0, sizeof(int), s));
    // the steps are enqueued back to back: step j + 1 reads the landmark
    // that step j's argmax wrote on the device
    hipLaunchKernelGGL(k_fps_chunks_init, dim3(nblk(fs.nchunks)), dim3(256), 0, s, fs, n);
    for (int64_t j = 0; j < l; ++j) {
        hipLaunchKernelGGL(k_fps_search, dim3(1), dim3(kSearchThreads), 0, s, fs, rp, ci, w, n, (int)j,
                           (int)(j + 1 == l), max_rounds);
        GCHK(hipGetLastError());
    }
    int herr_fps = 0;
    GCHK(hipMemcpyAsync(&herr_fps, fs.err, sizeof(int), hipMemcpyDeviceToHost, s));
    GCHK(hipStreamSynchronize(s));
    if (herr_fps) return api_fail(SBMDS_EHIP, "a farthest-point search did not settle");
    // the landmark block: full searches, S sources at a time, in distance
    // buckets twice the largest edge weight wide
    if (want_w) {
        hipLaunchKernelGGL(k_geo_fill_u64, dim3(nblk((int64_t)S * n)), dim3(256), 0, s, ms.dist, (int64_t)S * n,
                           kInfBits);
        hipLaunchKernelGGL(k_geo_fill_i32, dim3(nblk((int64_t)S * n)), dim3(256), 0, s, ms.inq, (int64_t)S * n, 0);
        hipLaunchKernelGGL(k_geo_fill_i32, dim3(nblk((int64_t)S * n)), dim3(256), 0, s, ms.farf, (int64_t)S * n, 0);
        GCHK(hipMemsetAsync(dwmax, 0, 8, s));
        if (nnz > 0) hipLaunchKernelGGL(k_geo_wmax, dim3(nblk(nnz)), dim3(256), 0, s, w, nnz, dwmax);
        GCHK(hipGetLastError());
        unsigned long long hwmax = 0;
        GCHK(hipMemcpyAsync(&hwmax, dwmax, 8, hipMemcpyDeviceToHost, s));
        GCHK(hipStreamSynchronize(s));
        double wmax = 0.0;
        std::memcpy(&wmax, &hwmax, 8);
        const double delta = wmax > 0.0 ? 2.0 * wmax : 1.0;
        for (int64_t f0 = 0; f0 < l; f0 += S) {
            const int Sb = (int)std::min<int64_t>(S, l - f0);
            hipLaunchKernelGGL(k_ms_begin, dim3(1), dim3(256), 0, s, ms, (const int32_t *)fs.lm, (int)f0, Sb, n,
                               delta);
            GCHK(hipGetLastError());
            int r = 0, fsel = 0;
            for (;;) {
                // rounds until the frontier runs empty; one host check per
                // kRoundsPerCheck rounds, the threshold stays on the device
                for (int q = 0; q < kRoundsPerCheck; ++q, ++r)
                    hipLaunchKernelGGL(k_ms_round, dim3(kRoundGrid), dim3(256), 0, s, ms, rp, ci, w, n, r, fsel);
                GCHK(hipGetLastError());
                int hc[2] = {0, 0};
                GCHK(hipMemcpyAsync(&hc[0], ms.cnt + (r % 3), sizeof(int), hipMemcpyDeviceToHost, s));
                GCHK(hipMemcpyAsync(&hc[1], ms.fcnt + fsel, sizeof(int), hipMemcpyDeviceToHost, s));
                GCHK(hipStreamSynchronize(s));
                if (r > max_rounds) return api_fail(SBMDS_EHIP, "a shortest-path search did not settle");
                if (hc[0] != 0) continue;
                if (hc[1] == 0) break;  // nothing waits: the search has settled
                // next bucket: past the smallest waiting distance
                hipLaunchKernelGGL(k_ms_farmin, dim3(kRoundGrid), dim3(256), 0, s, ms, fsel, n);
                hipLaunchKernelGGL(k_ms_next_thr, dim3(1), dim3(64), 0, s, ms, delta);
                GCHK(hipMemsetAsync(ms.fcnt + (fsel ^ 1), 0, sizeof(int), s));
                hipLaunchKernelGGL(k_ms_refill, dim3(kRoundGrid), dim3(256), 0, s, ms, fsel, r, n);
                GCHK(hipGetLastError());
                fsel ^= 1;
            }
            hipLaunchKernelGGL(k_ms_gather, dim3(nblk(l), (unsigned)Sb), dim3(256), 0, s,
                               (const unsigned long long *)ms.dist, (const int32_t *)fs.lm, n, l, (int)f0, Sb, D);
            hipLaunchKernelGGL(k_geo_fill_u64, dim3(nblk((int64_t)Sb * n)), dim3(256), 0, s, ms.dist,
                               (int64_t)Sb * n, kInfBits);
            hipLaunchKernelGGL(k_geo_fill_i32, dim3(nblk((int64_t)Sb * n)), dim3(256), 0, s, ms.inq,
                               (int64_t)Sb * n, 0);
            hipLaunchKernelGGL(k_geo_fill_i32, dim3(nblk((int64_t)Sb * n)), dim3(256), 0, s, ms.farf,
                               (int64_t)Sb * n, 0);
            GCHK(hipGetLastError());
        }
        hipLaunchKernelGGL(k_geo_square_sym, dim3(nblk(l), (unsigned)l), dim3(256), 0, s, (const double *)D, l, Wd);
        GCHK(hipGetLastError());
        GCHK(hipMemcpyAsync(W, Wd, bL, host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
    }
    GCHK(hipMemcpyAsync(landmarks, fs.lm, (size_t)l * 4, host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
    GCHK(hipStreamSynchronize(s));
    return SBMDS_OK;
}

}  // namespace
}  // namespace sbmds

extern "C" int sbmds_landmarks_geodesic(const int32_t *rowptr, const int32_t *col, const double *w, int64_t n,
                                        int64_t l, int32_t first, int32_t *landmarks, double *W, int mem, int batch,
                                        void *stream) {
    using namespace sbmds;
    api_clear_error();
    if (!rowptr || !landmarks) return api_fail(SBMDS_EINVAL, "rowptr and landmarks must be non-NULL");
    if (mem != SBMDS_MEM_HOST && mem != SBMDS_MEM_DEVICE) return api_fail(SBMDS_EINVAL, "mem must be 0 or 1");
    if (n < 1 || n >= ((int64_t)1 << 31)) return api_fail(SBMDS_EINVAL, "need 1 <= n < 2^31");
    if (l < 1 || l > n || l > 65535) return api_fail(SBMDS_EINVAL, "need 1 <= l <= min(n, 65535)");
    if (first < 0 || first >= n) return api_fail(SBMDS_EINVAL, "first landmark out of range");
    if (batch < 1) return api_fail(SBMDS_EINVAL, "batch must be >= 1");
    int64_t nnz = 0;
    if (mem == SBMDS_MEM_HOST) {
        nnz = rowptr[n];
    } else {
        int32_t t = 0;
        if (hipMemcpy(&t, rowptr + n, 4, hipMemcpyDeviceToHost) != hipSuccess)
            return api_fail(SBMDS_EHIP, "reading rowptr[n] failed");
        nnz = t;
    }
    if (nnz < 0) return api_fail(SBMDS_EINVAL, "rowptr[n] < 0");
    if (nnz > 0 && (!col || !w)) return api_fail(SBMDS_EINVAL, "col and w must be non-NULL");
    try {
        return geodesic_impl(rowptr, col, w, n, nnz, l, first, landmarks, W, mem, batch, (hipStream_t)stream);
    } catch (const std::exception &e) {
        return api_fail(SBMDS_ENOMEM, std::string("host exception: ") + e.what());
    }
}
