/*
 * Shortest-path helpers for the synthetic input generator (CPU only).
 *
 * Geodesic distances are taken as Dijkstra shortest paths over the mesh
 * edge graph (edge weight = Euclidean edge length).  Two entry points:
 *
 *   sbgen_fps        farthest-point landmark selection, Eq. (FarthestPoint):
 *                    the first landmark is given, each further one is the
 *                    vertex of largest minimum distance to those already
 *                    chosen (lowest vertex id on ties).  Each search only
 *                    expands vertices whose minimum it lowers, which cannot
 *                    change the result.
 *   sbgen_sssp_to    for every source, the full single-source distances,
 *                    kept only at a list of target vertices; sources are
 *                    spread over OpenMP threads.
 *
 * The graph is symmetric CSR: indptr[n+1] (int64), indices[nnz] (int32),
 * weights[nnz] (double, > 0).  Return value 0 on success, -1 on bad input,
 * -2 on allocation failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double key;
    int32_t v;
} hnode;

typedef struct {
    hnode *a;
    int64_t size, cap;
} heap;

static int heap_push(heap *h, double key, int32_t v) {
    if (h->size == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        hnode *na = (hnode *)realloc(h->a, (size_t)nc * sizeof(hnode));
        if (!na) return -2;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->size++;
    while (i > 0) {
        int64_t p = (i - 1) >> 1;
        /* order by key, then by vertex id so that pops are deterministic */
        if (h->a[p].key < key || (h->a[p].key == key && h->a[p].v <= v)) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].key = key;
    h->a[i].v = v;
    return 0;
}

static hnode heap_pop(heap *h) {
    hnode top = h->a[0];
    hnode last = h->a[--h->size];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= h->size) break;
        if (c + 1 < h->size &&
            (h->a[c + 1].key < h->a[c].key ||
             (h->a[c + 1].key == h->a[c].key && h->a[c + 1].v < h->a[c].v)))
            c++;
        if (last.key < h->a[c].key || (last.key == h->a[c].key && last.v <= h->a[c].v)) break;
        h->a[i] = h->a[c];
        i = c;
    }
    h->a[i] = last;
    return top;
}

/* Dijkstra from src; dist[] must be +inf on entry for every vertex.  With a
 * per-vertex `bound` (may be NULL), a vertex u is only relaxed to distances
 * strictly below bound[u].  Every vertex whose dist[] was written is appended
 * to touched[] (if non-NULL). */
static int dijkstra(int64_t n, const int64_t *indptr, const int32_t *indices, const double *w,
                    int32_t src, const double *bound, double *dist, int32_t *touched,
                    int64_t *ntouched, heap *h) {
    (void)n;
    h->size = 0;
    dist[src] = 0.0;
    if (touched) touched[(*ntouched)++] = src;
    if (heap_push(h, 0.0, src)) return -2;
    while (h->size) {
        hnode t = heap_pop(h);
        if (t.key > dist[t.v]) continue; /* stale entry */
        for (int64_t e = indptr[t.v]; e < indptr[t.v + 1]; ++e) {
            int32_t u = indices[e];
            double nd = t.key + w[e];
            if (nd < dist[u] && (!bound || nd < bound[u])) {
                if (touched && isinf(dist[u])) touched[(*ntouched)++] = u;
                dist[u] = nd;
                if (heap_push(h, nd, u)) return -2;
            }
        }
    }
    return 0;
}

int sbgen_fps(int64_t n, const int64_t *indptr, const int32_t *indices, const double *w,
              int64_t l, int64_t first, int64_t *landmarks, double *mind_out) {
    if (n <= 0 || l <= 0 || l > n || first < 0 || first >= n) return -1;
    double *mind = (double *)malloc((size_t)n * sizeof(double));
    double *dist = (double *)malloc((size_t)n * sizeof(double));
    int32_t *touched = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    heap h = {0, 0, 0};
    int rc = 0;
    if (!mind || !dist || !touched) { rc = -2; goto done; }
    for (int64_t i = 0; i < n; ++i) { mind[i] = INFINITY; dist[i] = INFINITY; }
    int64_t cur = first;
    for (int64_t j = 0; j < l; ++j) {
        landmarks[j] = cur;
        int64_t nt = 0;
        /* A path through a vertex v already at or above mind[v] cannot lower
         * the minimum of anything beyond it (mind is 1-Lipschitz along
         * edges), so the search is pruned against mind itself. */
        rc = dijkstra(n, indptr, indices, w, (int32_t)cur, mind, dist, touched, &nt, &h);
        if (rc) goto done;
        dist[cur] = 0.0;
        mind[cur] = 0.0;
        for (int64_t t = 0; t < nt; ++t) {
            int32_t v = touched[t];
            if (dist[v] < mind[v]) mind[v] = dist[v];
            dist[v] = INFINITY;
        }
        if (j + 1 < l) {
            int64_t best = 0;
            double bv = mind[0];
            for (int64_t i = 1; i < n; ++i)
                if (mind[i] > bv) { bv = mind[i]; best = i; }
            cur = best;
        }
    }
    if (mind_out) memcpy(mind_out, mind, (size_t)n * sizeof(double));
done:
    free(mind);
    free(dist);
    free(touched);
    free(h.a);
    return rc;
}

int sbgen_sssp_to(int64_t n, const int64_t *indptr, const int32_t *indices, const double *w,
                  int64_t nsrc, const int64_t *src, int64_t ntgt, const int64_t *tgt, double *out,
                  int nthreads) {
    if (n <= 0 || nsrc < 0 || ntgt < 0) return -1;
    for (int64_t s = 0; s < nsrc; ++s)
        if (src[s] < 0 || src[s] >= n) return -1;
    for (int64_t t = 0; t < ntgt; ++t)
        if (tgt[t] < 0 || tgt[t] >= n) return -1;
    int rc = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        double *dist = (double *)malloc((size_t)n * sizeof(double));
        int32_t *touched = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        heap h = {0, 0, 0};
        int myrc = (dist && touched) ? 0 : -2;
        if (!myrc)
            for (int64_t i = 0; i < n; ++i) dist[i] = INFINITY;
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < nsrc; ++s) {
            if (myrc) continue;
            int64_t nt = 0;
            myrc = dijkstra(n, indptr, indices, w, (int32_t)src[s], NULL, dist, touched, &nt, &h);
            for (int64_t t = 0; t < ntgt; ++t) out[s * ntgt + t] = dist[tgt[t]];
            for (int64_t t = 0; t < nt; ++t) dist[touched[t]] = INFINITY;
        }
        if (myrc) {
#pragma omp critical
            rc = myrc;
        }
        free(dist);
        free(touched);
        free(h.a);
    }
    return rc;
}
