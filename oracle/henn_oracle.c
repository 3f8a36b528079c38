/*
 * henn_oracle.c -- plain, slow, FP64 CPU oracle for HENN (arXiv 2505.17368).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * What it computes, step by step, in the paper's order:
 *   - Philox4x64-10 counter-based stream (Salmon et al., SC'11), used for the
 *     with-replacement samples of Alg. 2 (BuildEpsNetSampling) and for the
 *     ring ranges that the practical IsEpsNet check samples (App. B.1,
 *     "Practical Implementation"; App. G.2).
 *   - distances of the data model (Sec. 2): squared L2 or negative inner
 *     product, summed in FP64 in coordinate order.
 *   - ring members (Def. "Ring Ranges", Sec. 2.1) by a full sort.
 *   - the exact kNN navigable graph of one layer (App. B.2, App. G.4 "knn").
 *   - HNSW-style beam search with a candidate min-heap and a result max-heap
 *     (Sec. 2.2, k>1 by a candidate set; Alg. 4 GreedySearch when ef=1),
 *     descending from the root layer to layer 0 (Alg. 4 Query).
 *   - brute-force exact k-NN (Sec. 2, problem setting) as quality reference.
 *
 * Every comparison uses the lexicographic key (distance, global id).
 * Parallelism: none inside; the Python driver calls row/query ranges from
 * several threads (the functions are re-entrant).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).                  */
/* ------------------------------------------------------------------ */
static void mul_hilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void ho_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t hi0, lo0, hi1, lo1;
    mul_hilo64(M0, x0, &hi0, &lo0);
    mul_hilo64(M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0; k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Word q of the stream (tag, layer, attempt): output word q mod 4 of the
 * block with counter (q/4, layer, attempt, tag) and key (seed, 0). */
uint64_t ho_stream_word(uint64_t seed, uint64_t tag, uint64_t layer, uint64_t attempt,
                        uint64_t q) {
  uint64_t ctr[4] = {q / 4, layer, attempt, tag};
  uint64_t key[2] = {seed, 0};
  uint64_t out[4];
  ho_philox4x64_10(ctr, key, out);
  return out[q % 4];
}

/* Uniform index in [0, s): the high half of the 128-bit product w*s. */
uint64_t ho_uniform_index(uint64_t w, uint64_t s) {
  unsigned __int128 p = (unsigned __int128)w * (unsigned __int128)s;
  return (uint64_t)(p >> 64);
}

/* Fill out[q] = u(word q of stream (tag, layer, attempt), s) for q < count. */
void ho_draw_indices(uint64_t seed, uint64_t tag, uint64_t layer, uint64_t attempt,
                     int64_t s, int64_t count, int64_t *out) {
  for (int64_t q = 0; q < count; ++q)
    out[q] = (int64_t)ho_uniform_index(ho_stream_word(seed, tag, layer, attempt, (uint64_t)q),
                                       (uint64_t)s);
}

/* ------------------------------------------------------------------ */
/* Distances (Sec. 2 data model).  metric 0: squared L2; 1: -<a,b>.    */
/* ------------------------------------------------------------------ */
static double dist64(const float *a, const float *b, int d, int metric) {
  double acc = 0.0;
  if (metric == 0) {
    for (int j = 0; j < d; ++j) {
      double t = (double)a[j] - (double)b[j];
      acc += t * t;
    }
    return acc;
  }
  for (int j = 0; j < d; ++j) acc += (double)a[j] * (double)b[j];
  return -acc;
}

double ho_distance(const float *a, const float *b, int d, int metric) {
  return dist64(a, b, d, metric);
}

static double norm64(const float *a, int d) {
  double acc = 0.0;
  for (int j = 0; j < d; ++j) acc += (double)a[j] * (double)a[j];
  return sqrt(acc);
}

typedef struct {
  double d;
  int64_t id;
} dkey;

/* strict total order on (distance, id) */
static int key_less(dkey a, dkey b) { return a.d < b.d || (a.d == b.d && a.id < b.id); }

static int key_cmp(const void *pa, const void *pb) {
  dkey a = *(const dkey *)pa, b = *(const dkey *)pb;
  if (key_less(a, b)) return -1;
  if (key_less(b, a)) return 1;
  return 0;
}

/* relative decision margin between two distances */
static double margin_l2(double a, double b) {
  double m = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
  if (m < 1e-30) m = 1e-30;
  return fabs(a - b) / m;
}

/* ------------------------------------------------------------------ */
/* Ring ranges (Def. Ring Ranges; App. B.1 practical IsEpsNet).         */
/* The members of L_{i-1} (global ids, ascending) are ranked by         */
/* (dist(centre, x), x); the ring is ranks [a, a+w-1].                  */
/* out_local receives the w local indices (positions in `members`) in   */
/* rank order; out_margin the relative gaps at the two window ends.     */
/* ------------------------------------------------------------------ */
int ho_ring_members(const float *X, int d, int metric, const int32_t *members, int64_t s,
                    int64_t centre_local, int64_t a, int64_t w, int64_t *out_local,
                    double *out_margin) {
  if (a < 0 || w < 1 || a + w > s) return -1;
  dkey *keys = (dkey *)malloc(sizeof(dkey) * (size_t)s);
  if (!keys) return -2;
  const float *c = X + (size_t)members[centre_local] * (size_t)d;
  for (int64_t j = 0; j < s; ++j) {
    keys[j].d = dist64(c, X + (size_t)members[j] * (size_t)d, d, metric);
    keys[j].id = members[j];
  }
  /* remember which local index each key came from: ids are ascending, so a
   * binary search over members recovers it after the sort */
  qsort(keys, (size_t)s, sizeof(dkey), key_cmp);
  double mg = INFINITY;
  if (a > 0) mg = fmin(mg, margin_l2(keys[a - 1].d, keys[a].d));
  if (a + w < s) mg = fmin(mg, margin_l2(keys[a + w - 1].d, keys[a + w].d));
  for (int64_t r = 0; r < w; ++r) {
    int64_t id = keys[a + r].id;
    int64_t lo = 0, hi = s - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if (members[mid] < id) lo = mid + 1; else hi = mid;
    }
    out_local[r] = lo;
  }
  if (out_margin) *out_margin = mg;
  free(keys);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Exact kNN graph of one layer (App. B.2; App. G.4 "knn").            */
/* For rows [row_begin, row_end) of the layer: the first R members     */
/* u != v in ascending (dist(v,u), u) order, as local indices; -1 pad.  */
/* cut_margin[row]: relative gap between the R-th and (R+1)-th sorted   */
/* neighbour (a near tie there can change which nodes are neighbours).  */
/* order_margin[row]: smallest relative gap between consecutive entries */
/* of the first R+1 (a near tie there can also reorder the list).       */
/* ------------------------------------------------------------------ */
int ho_knn_graph(const float *X, int d, int metric, const int32_t *members, int64_t s,
                 int64_t row_begin, int64_t row_end, int R, int32_t *adj, double *adj_dist,
                 double *cut_margin, double *order_margin) {
  dkey *keys = (dkey *)malloc(sizeof(dkey) * (size_t)(s > 0 ? s : 1));
  if (!keys) return -2;
  for (int64_t v = row_begin; v < row_end; ++v) {
    const float *xv = X + (size_t)members[v] * (size_t)d;
    int64_t cnt = 0;
    for (int64_t u = 0; u < s; ++u) {
      if (u == v) continue;
      keys[cnt].d = dist64(xv, X + (size_t)members[u] * (size_t)d, d, metric);
      keys[cnt].id = u; /* local index; same order as the global id */
      ++cnt;
    }
    qsort(keys, (size_t)cnt, sizeof(dkey), key_cmp);
    double mg = INFINITY;
    int64_t lim = cnt < (int64_t)R + 1 ? cnt : (int64_t)R + 1;
    for (int64_t r = 1; r < lim; ++r) mg = fmin(mg, margin_l2(keys[r - 1].d, keys[r].d));
    for (int r = 0; r < R; ++r) {
      adj[(size_t)v * R + r] = r < cnt ? (int32_t)keys[r].id : -1;
      if (adj_dist) adj_dist[(size_t)v * R + r] = r < cnt ? keys[r].d : INFINITY;
    }
    if (cut_margin) cut_margin[v] = cnt > R ? margin_l2(keys[R - 1].d, keys[R].d) : INFINITY;
    if (order_margin) order_margin[v] = mg;
  }
  free(keys);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Diversity pruning (App. B.2 navigable graphs: the neighbour selection  */
/* of NSW/HNSW-style graphs).  Row v of adj_in holds C candidates in      */
/* ascending (dist(v,.), id) order, -1 padded.  They are taken in that    */
/* order; a candidate c is dropped when some already kept r is closer to  */
/* c than v is, d(c, r) < d(c, v); otherwise it is kept, until R_keep are */
/* kept.  Rows are -1 padded.  prune_margin[v] = the smallest relative    */
/* margin |d(c,r) - d(c,v)| / max(|.|) over every comparison made.        */
/* ------------------------------------------------------------------ */
int ho_prune(const float *X, int d, int metric, const int32_t *members, int64_t s,
             const int32_t *adj_in, int C, int R_keep, int32_t *adj_out, double *prune_margin) {
  int32_t *kept = (int32_t *)malloc(sizeof(int32_t) * (size_t)(R_keep > 0 ? R_keep : 1));
  if (!kept) return -2;
  for (int64_t v = 0; v < s; ++v) {
    const float *xv = X + (size_t)members[v] * (size_t)d;
    int nk = 0;
    double mg = INFINITY;
    for (int j = 0; j < C && nk < R_keep; ++j) {
      const int32_t c = adj_in[(size_t)v * C + j];
      if (c < 0) break;
      const float *xc = X + (size_t)members[c] * (size_t)d;
      const double dcv = dist64(xc, xv, d, metric);
      int drop = 0;
      for (int r = 0; r < nk; ++r) {
        const double dcr = dist64(xc, X + (size_t)members[kept[r]] * (size_t)d, d, metric);
        mg = fmin(mg, margin_l2(dcr, dcv));
        if (dcr < dcv) drop = 1;
      }
      if (!drop) kept[nk++] = c;
    }
    for (int r = 0; r < R_keep; ++r) adj_out[(size_t)v * R_keep + r] = r < nk ? kept[r] : -1;
    if (prune_margin) prune_margin[v] = mg;
  }
  free(kept);
  return 0;
}

/* ------------------------------------------------------------------ */
/* kNN graph plus reverse edges (the kNN_SYM navigable graph): row v is   */
/* the first max_deg of the deduplicated union of v's out-neighbours and  */
/* the nodes that list v, in ascending (dist(v,u), u) order.  adj_knn is  */
/* the layer's kNN adjacency (local indices, R per row, -1 padded).       */
/* cut/order margins as in ho_knn_graph, over the union's sorted list.    */
/* ------------------------------------------------------------------ */
int ho_knn_sym(const float *X, int d, int metric, const int32_t *members, int64_t s,
               const int32_t *adj_knn, int R, int max_deg, int32_t *adj, double *cut_margin,
               double *order_margin) {
  int64_t *indeg = (int64_t *)calloc((size_t)s + 1, sizeof(int64_t));
  if (!indeg) return -2;
  for (int64_t v = 0; v < s; ++v)
    for (int r = 0; r < R; ++r) {
      int32_t u = adj_knn[(size_t)v * R + r];
      if (u >= 0) indeg[u + 1]++;
    }
  for (int64_t v = 0; v < s; ++v) indeg[v + 1] += indeg[v];
  int64_t total = indeg[s];
  int32_t *inl = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(s > 0 ? s : 1));
  if (!inl || !cur) { free(indeg); free(inl); free(cur); return -2; }
  for (int64_t v = 0; v < s; ++v) cur[v] = indeg[v];
  for (int64_t v = 0; v < s; ++v)
    for (int r = 0; r < R; ++r) {
      int32_t u = adj_knn[(size_t)v * R + r];
      if (u >= 0) inl[cur[u]++] = (int32_t)v;
    }
  int64_t maxc = 0;
  for (int64_t v = 0; v < s; ++v)
    if (indeg[v + 1] - indeg[v] > maxc) maxc = indeg[v + 1] - indeg[v];
  dkey *keys = (dkey *)malloc(sizeof(dkey) * (size_t)(maxc + R + 1));
  if (!keys) { free(indeg); free(inl); free(cur); return -2; }
  for (int64_t v = 0; v < s; ++v) {
    const float *xv = X + (size_t)members[v] * (size_t)d;
    int64_t cnt = 0;
    for (int r = 0; r < R; ++r) {
      int32_t u = adj_knn[(size_t)v * R + r];
      if (u < 0) continue;
      keys[cnt].d = dist64(xv, X + (size_t)members[u] * (size_t)d, d, metric);
      keys[cnt].id = u;
      ++cnt;
    }
    for (int64_t j = indeg[v]; j < indeg[v + 1]; ++j) {
      int32_t u = inl[j];
      int dup = 0;
      for (int r = 0; r < R; ++r)
        if (adj_knn[(size_t)v * R + r] == u) dup = 1;
      if (dup) continue;
      keys[cnt].d = dist64(xv, X + (size_t)members[u] * (size_t)d, d, metric);
      keys[cnt].id = u;
      ++cnt;
    }
    qsort(keys, (size_t)cnt, sizeof(dkey), key_cmp);
    double mg = INFINITY;
    int64_t lim = cnt < (int64_t)max_deg + 1 ? cnt : (int64_t)max_deg + 1;
    for (int64_t r = 1; r < lim; ++r) mg = fmin(mg, margin_l2(keys[r - 1].d, keys[r].d));
    for (int r = 0; r < max_deg; ++r) adj[(size_t)v * max_deg + r] = r < cnt ? (int32_t)keys[r].id : -1;
    if (cut_margin)
      cut_margin[v] = cnt > max_deg ? margin_l2(keys[max_deg - 1].d, keys[max_deg].d) : INFINITY;
    if (order_margin) order_margin[v] = mg;
  }
  free(keys); free(indeg); free(inl); free(cur);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Binary heaps over dkey.                                              */
/* ------------------------------------------------------------------ */
typedef struct {
  dkey *a;
  int64_t n, cap;
  int max_heap; /* 1: largest on top */
} heap;

static int heap_above(const heap *h, dkey x, dkey y) {
  return h->max_heap ? key_less(y, x) : key_less(x, y);
}

static int heap_push(heap *h, dkey x) {
  if (h->n == h->cap) {
    int64_t nc = h->cap ? h->cap * 2 : 64;
    dkey *na = (dkey *)realloc(h->a, sizeof(dkey) * (size_t)nc);
    if (!na) return -1;
    h->a = na;
    h->cap = nc;
  }
  int64_t i = h->n++;
  h->a[i] = x;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (!heap_above(h, h->a[i], h->a[p])) break;
    dkey t = h->a[i]; h->a[i] = h->a[p]; h->a[p] = t;
    i = p;
  }
  return 0;
}

static dkey heap_pop(heap *h) {
  dkey top = h->a[0];
  h->a[0] = h->a[--h->n];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, b = i;
    if (l < h->n && heap_above(h, h->a[l], h->a[b])) b = l;
    if (r < h->n && heap_above(h, h->a[r], h->a[b])) b = r;
    if (b == i) break;
    dkey t = h->a[i]; h->a[i] = h->a[b]; h->a[b] = t;
    i = b;
  }
  return top;
}

/* ------------------------------------------------------------------ */
/* One layer of the search: HNSW's SEARCH-LAYER under the total order.   */
/* Sec. 2.2 (k>1 through a candidate set), Alg. 4 GreedySearch when      */
/* ef = 1.  Works on one layer given as member ids + local adjacency.    */
/* ------------------------------------------------------------------ */
typedef struct {
  const float *X;
  int d, metric;
  const float *q;
  double qnorm;
  double min_margin;       /* min relative margin over decisive comparisons */
  double min_adj_margin;   /* min adjacency margin over expanded nodes */
  int64_t expansions, evals;
} trace;

static double pair_margin(const trace *t, dkey a, dkey b) {
  if (a.id == b.id) return INFINITY;
  if (t->metric == 0) return margin_l2(a.d, b.d);
  double na = norm64(t->X + (size_t)a.id * (size_t)t->d, t->d);
  double nb = norm64(t->X + (size_t)b.id * (size_t)t->d, t->d);
  double den = t->qnorm * (na > nb ? na : nb);
  if (den < 1e-30) den = 1e-30;
  return fabs(a.d - b.d) / den;
}

static void note(trace *t, dkey a, dkey b) {
  double m = pair_margin(t, a, b);
  if (m < t->min_margin) t->min_margin = m;
}

/* Result W is written ascending into out (up to ef entries, global ids);
 * returns |W|.  `stamp` is a per-call visited array of the layer size with
 * values < `gen` meaning "not visited". */
static int64_t search_layer(trace *t, const int32_t *members, int64_t size, const int32_t *adj,
                            int deg, const double *adj_margin, int64_t entry_local, int ef,
                            int32_t *stamp, int32_t gen, dkey *out) {
  heap C = {0, 0, 0, 0}, W = {0, 0, 0, 1};
  /* keys in the heaps carry the GLOBAL id in .id; the local index is
   * recovered through the ascending member list */
  dkey e = {dist64(t->q, t->X + (size_t)members[entry_local] * (size_t)t->d, t->d, t->metric),
            members[entry_local]};
  t->evals++;
  stamp[entry_local] = gen;
  heap_push(&C, e);
  heap_push(&W, e);
  while (C.n > 0) {
    dkey c = heap_pop(&C);
    /* which candidate is expanded next: c against the one that follows it,
     * now the top of C */
    if (C.n > 0) note(t, c, C.a[0]);
    dkey wmax = W.a[0];
    note(t, c, wmax); /* the stop test */
    if (key_less(wmax, c)) break;
    /* local index of c */
    int64_t lo = 0, hi = size - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if (members[mid] < c.id) lo = mid + 1; else hi = mid;
    }
    int64_t cl = lo;
    t->expansions++;
    if (adj_margin && adj_margin[cl] < t->min_adj_margin) t->min_adj_margin = adj_margin[cl];
    for (int j = 0; j < deg; ++j) {
      int32_t ul = adj[(size_t)cl * deg + j];
      if (ul < 0) continue;
      if (stamp[ul] == gen) continue;
      stamp[ul] = gen;
      dkey u = {dist64(t->q, t->X + (size_t)members[ul] * (size_t)t->d, t->d, t->metric),
                members[ul]};
      t->evals++;
      if (W.n >= ef) note(t, u, W.a[0]); /* admission against the worst kept */
      if (W.n < ef || key_less(u, W.a[0])) {
        heap_push(&C, u);
        heap_push(&W, u);
        if (W.n > ef) {
          dkey worst = heap_pop(&W);
          note(t, worst, W.a[0]); /* eviction */
        }
      }
    }
  }
  int64_t m = W.n;
  for (int64_t i = m - 1; i >= 0; --i) out[i] = heap_pop(&W);
  free(C.a);
  free(W.a);
  return m;
}

/* ------------------------------------------------------------------ */
/* Query (Alg. 4 Query with the Sec. 2.2 candidate set at layer 0).      */
/* Layers are 0..num_layers-1 (0 = all points).  members[i]: ascending   */
/* global ids of layer i; adj[i]: local adjacency, deg[i] per row.       */
/* Entry: the smallest id of the root layer.  Upper layers use ef_upper, */
/* layer 0 uses max(ef, k).  Outputs k ids/dists per query (padded with  */
/* -1 / +inf), the minimum decision margin over the trace, the minimum   */
/* adjacency margin over expanded nodes, and per-query counters          */
/* [expansions, evaluations] summed over layers (plus layer-0 only).     */
/* ------------------------------------------------------------------ */
int ho_search(const float *X, int d, int metric, int num_layers, const int64_t *sizes,
              const int32_t *const *members, const int32_t *const *adj, const int32_t *deg,
              const double *const *adj_margin, const float *Q, int64_t q_begin, int64_t q_end,
              int k, int ef, int ef_upper, int root_complete, int32_t *out_ids, double *out_dist,
              double *out_margin, double *out_adj_margin, int64_t *counters) {
  if (num_layers < 1 || k < 1 || ef < 1 || ef_upper < 1) return -1;
  int ef0 = ef > k ? ef : k;
  int64_t maxsize = 0;
  for (int i = 0; i < num_layers; ++i) maxsize = sizes[i] > maxsize ? sizes[i] : maxsize;
  int32_t *stamp = (int32_t *)calloc((size_t)maxsize, sizeof(int32_t));
  int efmax = ef0 > ef_upper ? ef0 : ef_upper;
  dkey *res = (dkey *)malloc(sizeof(dkey) * (size_t)efmax);
  if (!stamp || !res) { free(stamp); free(res); return -2; }
  int32_t gen = 0;
  for (int64_t qi = q_begin; qi < q_end; ++qi) {
    trace t;
    t.X = X; t.d = d; t.metric = metric; t.q = Q + (size_t)qi * (size_t)d;
    t.qnorm = norm64(t.q, d);
    t.min_margin = INFINITY; t.min_adj_margin = INFINITY;
    t.expansions = 0; t.evals = 0;
    int top = num_layers - 1;
    int64_t entry_local = 0; /* smallest id of the root layer */
    int64_t m = 0;
    int64_t e0 = 0, v0 = 0;
    if (root_complete && top >= 1) {
      /* complete graph on the root (App. B.2: trivially navigable): greedy
       * search from any node reaches the exact nearest root member */
      dkey best = {INFINITY, -1}, second = {INFINITY, -1};
      for (int64_t j = 0; j < sizes[top]; ++j) {
        dkey u = {dist64(t.q, X + (size_t)members[top][j] * (size_t)d, d, metric),
                  members[top][j]};
        t.evals++;
        if (best.id < 0 || key_less(u, best)) { second = best; best = u; }
        else if (second.id < 0 || key_less(u, second)) second = u;
      }
      if (second.id >= 0) note(&t, best, second);
      const int32_t *mb = members[top - 1];
      int64_t lo = 0, hi = sizes[top - 1] - 1;
      while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (mb[mid] < best.id) lo = mid + 1; else hi = mid;
      }
      entry_local = lo;
      top = top - 1;
    }
    for (int i = top; i >= 0; --i) {
      ++gen;
      if (gen == INT32_MAX) { memset(stamp, 0, sizeof(int32_t) * (size_t)maxsize); gen = 1; }
      int efl = i == 0 ? ef0 : ef_upper;
      if (i == 0) { e0 = t.expansions; v0 = t.evals; }
      m = search_layer(&t, members[i], sizes[i], adj[i], deg[i], adj_margin ? adj_margin[i] : 0,
                       entry_local, efl, stamp, gen, res);
      if (i > 0) {
        /* hand the best node to the layer below (inter-layer edge: same point) */
        int64_t id = res[0].id;
        const int32_t *mb = members[i - 1];
        int64_t lo = 0, hi = sizes[i - 1] - 1;
        while (lo < hi) {
          int64_t mid = (lo + hi) / 2;
          if (mb[mid] < id) lo = mid + 1; else hi = mid;
        }
        entry_local = lo;
      }
    }
    /* the returned top-k: adjacent pairs and the k / k+1 cut are decisive */
    int64_t kk = m < k ? m : k;
    for (int64_t j = 1; j < kk + (m > k ? 1 : 0); ++j) note(&t, res[j - 1], res[j]);
    for (int j = 0; j < k; ++j) {
      out_ids[(size_t)qi * k + j] = j < m ? (int32_t)res[j].id : -1;
      out_dist[(size_t)qi * k + j] = j < m ? res[j].d : INFINITY;
    }
    if (out_margin) out_margin[qi] = t.min_margin;
    if (out_adj_margin) out_adj_margin[qi] = t.min_adj_margin;
    if (counters) {
      counters[qi * 4 + 0] = t.expansions;
      counters[qi * 4 + 1] = t.evals;
      counters[qi * 4 + 2] = t.expansions - e0;
      counters[qi * 4 + 3] = t.evals - v0;
    }
  }
  free(stamp);
  free(res);
  return 0;
}

/* ------------------------------------------------------------------ */
/* NSW graph of one layer (App. B.2: points are inserted one after the   */
/* other and joined to their nearest neighbours found in the graph built */
/* so far), one batch of the insertion.  The layer's members are given   */
/* by ascending global id; positions [0, lo) already form the graph in   */
/* adj (local positions, M per row, -1 padded) and the positions         */
/* [lo, hi) join it together:                                            */
/*  1. each new point p runs SEARCH-LAYER with a beam of max(ef, R) over  */
/*     the graph on [0, lo) from position 0, and its row becomes the R    */
/*     best results (none when lo = 0);                                  */
/*  2. every old point v chosen by some new points gets, as its row, the */
/*     first M of (its row plus those new points) in (distance, id)      */
/*     order.                                                            */
/* Points of one batch do not see each other (batched insertion); a      */
/* batch of one point is the plain sequential insertion.  margin[] is    */
/* min-folded with each row's decision margins: the search trace of a    */
/* new row, the adjacent keys and the M / M+1 cut of a merged row.       */
/* ------------------------------------------------------------------ */
static int64_t local_of(const int32_t *members, int64_t size, int64_t id) {
  int64_t lo = 0, hi = size - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (members[mid] < id) lo = mid + 1; else hi = mid;
  }
  return lo;
}

int ho_nsw_insert(const float *X, int d, int metric, const int32_t *members, int64_t s,
                  int32_t *adj, int M, int64_t lo, int64_t hi, int R, int ef, double *margin) {
  if (lo < 0 || hi > s || lo > hi || R < 1 || M < R || ef < 1) return -1;
  if (hi == lo) return 0;
  const int64_t nb = hi - lo;
  const int efl = ef > R ? ef : R;
  int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nb * R));
  int32_t *stamp = (int32_t *)calloc((size_t)(lo > 0 ? lo : 1), sizeof(int32_t));
  dkey *res = (dkey *)malloc(sizeof(dkey) * (size_t)efl);
  if (!rows || !stamp || !res) { free(rows); free(stamp); free(res); return -2; }
  /* 1. searches over the graph on [0, lo) */
  int32_t gen = 0;
  for (int64_t p = lo; p < hi; ++p) {
    int32_t *row = rows + (size_t)(p - lo) * (size_t)R;
    for (int j = 0; j < R; ++j) row[j] = -1;
    if (lo == 0) continue;
    trace t;
    t.X = X; t.d = d; t.metric = metric;
    t.q = X + (size_t)members[p] * (size_t)d;
    t.qnorm = norm64(t.q, d);
    t.min_margin = INFINITY; t.min_adj_margin = INFINITY;
    t.expansions = 0; t.evals = 0;
    ++gen;
    int64_t m = search_layer(&t, members, lo, adj, M, 0, 0, efl, stamp, gen, res);
    int64_t kk = m < R ? m : R;
    for (int64_t j = 1; j < kk + (m > R ? 1 : 0); ++j) note(&t, res[j - 1], res[j]);
    for (int64_t j = 0; j < kk; ++j) row[j] = (int32_t)local_of(members, lo, res[j].id);
    if (t.min_margin < margin[p]) margin[p] = t.min_margin;
  }
  for (int64_t p = lo; p < hi; ++p)
    for (int j = 0; j < M; ++j)
      adj[(size_t)p * M + j] = j < R ? rows[(size_t)(p - lo) * R + j] : -1;
  /* 2. reverse edges: the new points that chose v, grouped per v */
  int64_t *start = (int64_t *)calloc((size_t)lo + 1, sizeof(int64_t));
  int32_t *chosen = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nb * R + 1));
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(lo + 1));
  dkey *keys = (dkey *)malloc(sizeof(dkey) * (size_t)(M + nb + 1));
  if (!start || !chosen || !cur || !keys) {
    free(rows); free(stamp); free(res); free(start); free(chosen); free(cur); free(keys);
    return -2;
  }
  for (int64_t i = 0; i < nb * R; ++i)
    if (rows[i] >= 0) start[rows[i] + 1]++;
  for (int64_t v = 0; v < lo; ++v) start[v + 1] += start[v];
  for (int64_t v = 0; v < lo; ++v) cur[v] = start[v];
  for (int64_t p = lo; p < hi; ++p)
    for (int j = 0; j < R; ++j) {
      int32_t v = rows[(size_t)(p - lo) * R + j];
      if (v >= 0) chosen[cur[v]++] = (int32_t)p;
    }
  for (int64_t v = 0; v < lo; ++v) {
    if (start[v + 1] == start[v]) continue;
    trace t;
    t.X = X; t.d = d; t.metric = metric;
    t.q = X + (size_t)members[v] * (size_t)d;
    t.qnorm = norm64(t.q, d);
    t.min_margin = INFINITY;
    int64_t cnt = 0;
    for (int j = 0; j < M; ++j) {
      int32_t u = adj[(size_t)v * M + j];
      if (u < 0) continue;
      keys[cnt].d = dist64(t.q, X + (size_t)members[u] * (size_t)d, d, metric);
      keys[cnt].id = members[u];
      ++cnt;
    }
    for (int64_t i = start[v]; i < start[v + 1]; ++i) {
      int32_t u = chosen[i];
      keys[cnt].d = dist64(t.q, X + (size_t)members[u] * (size_t)d, d, metric);
      keys[cnt].id = members[u];
      ++cnt;
    }
    qsort(keys, (size_t)cnt, sizeof(dkey), key_cmp);
    int64_t lim = cnt < (int64_t)M + 1 ? cnt : (int64_t)M + 1;
    for (int64_t r = 1; r < lim; ++r) note(&t, keys[r - 1], keys[r]);
    for (int j = 0; j < M; ++j)
      adj[(size_t)v * M + j] = j < cnt ? (int32_t)local_of(members, s, keys[j].id) : -1;
    if (t.min_margin < margin[v]) margin[v] = t.min_margin;
  }
  free(rows); free(stamp); free(res); free(start); free(chosen); free(cur); free(keys);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Delete(x) (App. C): repair of one layer graph before its deleted      */
/* members are dropped.  Every live row v that links to a deleted member */
/* becomes the first M of the live points among its own row and the rows */
/* of its deleted neighbours (v itself and repeats left out), in         */
/* (distance, id) order.  Deleted rows are left as they are.  margin[] is */
/* min-folded with the repaired rows' adjacent-key and cut margins.      */
/* ------------------------------------------------------------------ */
int ho_nsw_repair(const float *X, int d, int metric, const int32_t *members, int64_t s,
                  int32_t *adj, int M, const uint8_t *del, double *margin) {
  int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M + M * M + 1));
  dkey *keys = (dkey *)malloc(sizeof(dkey) * (size_t)(M + M * M + 1));
  int32_t *row = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
  if (!cand || !keys || !row) { free(cand); free(keys); free(row); return -2; }
  for (int64_t v = 0; v < s; ++v) {
    if (del[v]) continue;
    int touched = 0;
    for (int j = 0; j < M; ++j) {
      row[j] = adj[(size_t)v * M + j];
      if (row[j] >= 0 && del[row[j]]) touched = 1;
    }
    if (!touched) continue;
    int64_t nc = 0;
    for (int j = 0; j < M; ++j) {
      int32_t u = row[j];
      if (u < 0) continue;
      if (!del[u]) { cand[nc++] = u; continue; }
      for (int r = 0; r < M; ++r) {
        int32_t w = adj[(size_t)u * M + r];
        if (w >= 0 && !del[w] && w != v) cand[nc++] = w;
      }
    }
    trace t;
    t.X = X; t.d = d; t.metric = metric;
    t.q = X + (size_t)members[v] * (size_t)d;
    t.qnorm = norm64(t.q, d);
    t.min_margin = INFINITY;
    int64_t nk = 0;
    for (int64_t i = 0; i < nc; ++i) {
      int dup = 0;
      for (int64_t j = 0; j < nk && !dup; ++j) dup = keys[j].id == members[cand[i]];
      if (dup) continue;
      keys[nk].d = dist64(t.q, X + (size_t)members[cand[i]] * (size_t)d, d, metric);
      keys[nk].id = members[cand[i]];
      ++nk;
    }
    qsort(keys, (size_t)nk, sizeof(dkey), key_cmp);
    int64_t lim = nk < (int64_t)M + 1 ? nk : (int64_t)M + 1;
    for (int64_t r = 1; r < lim; ++r) note(&t, keys[r - 1], keys[r]);
    for (int j = 0; j < M; ++j)
      adj[(size_t)v * M + j] = j < nk ? (int32_t)local_of(members, s, keys[j].id) : -1;
    if (t.min_margin < margin[v]) margin[v] = t.min_margin;
  }
  free(cand); free(keys); free(row);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Brute-force exact k-NN (Sec. 2 problem setting): quality reference.  */
/* ------------------------------------------------------------------ */
int ho_brute_knn(const float *X, int64_t n, int d, int metric, const float *Q, int64_t q_begin,
                 int64_t q_end, int k, int32_t *out_ids, double *out_dist) {
  heap W = {0, 0, 0, 1};
  for (int64_t qi = q_begin; qi < q_end; ++qi) {
    const float *q = Q + (size_t)qi * (size_t)d;
    W.n = 0;
    for (int64_t j = 0; j < n; ++j) {
      dkey u = {dist64(q, X + (size_t)j * (size_t)d, d, metric), j};
      if (W.n < k) {
        if (heap_push(&W, u)) { free(W.a); return -2; }
      } else if (key_less(u, W.a[0])) {
        heap_pop(&W);
        heap_push(&W, u);
      }
    }
    int64_t m = W.n;
    for (int64_t j = k - 1; j >= 0; --j) {
      if (j >= m) {
        out_ids[(size_t)qi * k + j] = -1;
        out_dist[(size_t)qi * k + j] = INFINITY;
      } else {
        dkey x = heap_pop(&W);
        out_ids[(size_t)qi * k + j] = (int32_t)x.id;
        out_dist[(size_t)qi * k + j] = x.d;
      }
    }
  }
  free(W.a);
  return 0;
}
