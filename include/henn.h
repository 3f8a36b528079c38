/*
 * henn.h -- C ABI of the MI355X (gfx950) HENN library.
 *
 * HENN (arXiv 2505.17368) answers k-nearest-neighbour queries over points
 * X in R^d (Sec. 2, "Data Model" and "Problem setting") with a hierarchy of
 * layers L_0 = X, L_1, ..., L_L where each L_i is an eps-net of L_{i-1} for
 * ring ranges (Def. HENN, Def. Ring Ranges, Alg. 1), each layer carries a
 * navigable graph (App. B.2; here the exact kNN graph of App. G.4), and a
 * query descends greedily from the root to layer 0 (Alg. 4, Sec. 2.2).
 *
 * Conventions for every entry point:
 *  - C linkage; no exception crosses the boundary.
 *  - Every call returns a henn_status.  On error the outputs are untouched
 *    and henn_last_error() (thread-local) describes the failure.
 *  - Device pointers are HIP device addresses (e.g. a torch tensor's
 *    data_ptr()); host pointers are ordinary process memory.  Each argument
 *    below says which one it is.
 *  - hip_stream is a hipStream_t (0 = the null stream).  Work is enqueued on
 *    it; henn_search_batch returns without waiting.
 *  - Distances returned are squared L2 (the paper's l2 norm with the
 *    monotone square root dropped) or -<q, x> for inner product (the angular
 *    metric of App. G.4 on unit vectors).  Every ordering is by the
 *    lexicographic key (distance, point id), so ties go to the lower id.
 */
#ifndef HENN_H
#define HENN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct henn_index henn_index; /* opaque; owned by the library */

typedef enum {
  HENN_OK = 0,
  HENN_E_INVAL = 1,       /* bad argument: sizes, null pointers, struct_size */
  HENN_E_NOMEM = 2,       /* device or host allocation failed */
  HENN_E_DEVICE = 3,      /* a HIP runtime call failed */
  HENN_E_UNSUPPORTED = 4, /* valid but not supported by the library */
  HENN_W_NOT_VERIFIED = 100 /* warning: index usable, some layer kept its best
                               unverified sample (Alg. 2 attempt cap reached) */
} henn_status;

typedef enum { HENN_L2 = 0, HENN_IP = 1 } henn_metric;

/* Storage of the vectors the search traverses.  F32 is the plain path.
 * BF16 and FP8_E4M3 (OCP, max 448) keep one FP32 scale per vector and an
 * FP32 copy for the final re-rank.  BF16 traversal distances are FP32 sums;
 * FP8 traversal forms q - s*c in f16 (query rounded to f16, codes scaled by
 * the converter) and accumulates the squares (or q*c for inner product) in
 * FP32. */
typedef enum { HENN_F32 = 0, HENN_BF16 = 1, HENN_FP8_E4M3 = 2 } henn_storage;

/* Navigable graph per layer (App. B.2): exact kNN, or kNN plus reverse
 * edges (deduplicated, kept in (distance, id) order, capped at max_degree). */
/* Navigable graph of each layer (App. B.2):
 *   KNN:        the exact R nearest other members, (distance, id) order;
 *   KNN_SYM:    KNN plus reverse edges: the first max_degree of the
 *               deduplicated union of out- and in-neighbours in that order;
 *   PRUNED:     diversity pruning of the exact top min(2R, 32) (the NSW/HNSW
 *               neighbour selection): candidates in order, each dropped when an
 *               already kept one is closer to it than the row is; <= R kept;
 *   PRUNED_SYM: PRUNED plus reverse edges, as KNN_SYM;
 *   NSW:        the incremental-insertion graph of App. B.2: members join in
 *               ascending id order, each linked to the R best results of a
 *               beam search (width max(ef_construction, R), from the first
 *               member) over the graph built so far, and every point it
 *               links to keeps the first max_degree of its row plus the new
 *               point, in (distance, id) order.  Insertion runs in batches
 *               [lo, lo + max(1, lo >> insert_shift)) whose points search
 *               the graph on [0, lo) together (henn_nsw_insert). */
typedef enum {
  HENN_GRAPH_KNN = 0,
  HENN_GRAPH_KNN_SYM = 1,
  HENN_GRAPH_PRUNED = 2,
  HENN_GRAPH_PRUNED_SYM = 3,
  HENN_GRAPH_NSW = 4
} henn_graph;

/* How layer i is drawn from layer i-1 (App. B.1):
 *   DRAWS:   Alg. 2 (BuildEpsNetSampling): ceil(|L_{i-1}| / 2^m) draws with
 *            replacement, duplicates merged;
 *   HALVING: Alg. 3 (BuildEpsNetDiscV2): m halving steps.  Each step pairs
 *            the current members in ascending id order (the matching the paper
 *            leaves arbitrary), keeps one member of every pair by a coin, and
 *            keeps an odd last member; the layer then holds exactly
 *            ceil(|L_{i-1}| / 2^m) distinct points.  The coin of pair p in
 *            step j (0-based) of attempt t is u(word p of stream
 *            (tag 4 + j, layer i, attempt t), 2): 0 keeps the lower id.
 * Either sample goes through the same ring check and Las-Vegas repeat
 * (max_attempts 1 gives the plain one-shot construction). */
typedef enum { HENN_SAMPLER_DRAWS = 0, HENN_SAMPLER_HALVING = 1 } henn_sampler;

#define HENN_MAX_LAYERS 16

typedef struct {
  uint32_t struct_size;   /* = sizeof(henn_build_params) */
  int32_t metric;         /* henn_metric */
  int32_t max_layers;     /* L of Alg. 1: upper layers allowed; < 0: build until
                             ceil(|L_{i-1}| / 2^m) < degree + 1 */
  int32_t m;              /* exponential decay of Eq. (1) / Lemma "layer-size";
                             each layer draws ceil(|L_{i-1}| / 2^m) samples */
  double c0;              /* constant of Eq. (1), natural logarithm */
  double eps_override;    /* > 0: use this eps on every layer instead of Eq. (1) */
  int32_t num_rings;      /* r: ring ranges checked per layer (App. G.2) */
  int32_t max_attempts;   /* Las-Vegas cap of Alg. 2's repeat loop; 0: derived from phi */
  int32_t degree;         /* R: kNN graph degree (kept neighbours for PRUNED) */
  int32_t max_degree;     /* row capacity of the graphs with reverse edges and NSW
                             (>= degree, <= 64) */
  int32_t graph;          /* henn_graph */
  int32_t storage;        /* henn_storage */
  uint64_t seed;          /* key word 0 of the Philox4x64-10 stream (word 1 = 0) */
  int32_t root_complete_max; /* > 0: stop adding layers once a layer holds at most this
                                many points, and search that root with the complete graph
                                (App. B.2: trivially navigable), i.e. an exhaustive scan
                                for the root member nearest to q; 0: off */
  int32_t sampler;        /* henn_sampler */
  int32_t ef_construction;/* NSW: beam width of the insertion searches, [1, 2048] */
  int32_t insert_shift;   /* NSW: batch after lo inserted members = max(1, lo >> shift);
                             large values give the one-by-one insertion */
  double phi;             /* Alg. 2: probability that one sample is not an eps-net
                             (Eq. (3)); the repeat loop then runs 1 / (1 - phi) times
                             in expectation.  With max_attempts = 0 the attempt cap is
                             the smallest t with phi^t <= 1e-9 (phi in (0, 1));
                             otherwise only reported */
  int32_t gram;           /* kNN graph kinds, d <= 128: 0 = Gram tiles on BF16 matrix
                             cores with split operands (hi + lo, three exact products
                             per coordinate), 1 = FP32 matrix-core tiles.  Both feed the
                             exact FP32 re-rank and its proven fallback, so the graph is
                             the same exact kNN graph; 0 does 3/16 of the matrix work.
                             Rows wider than 128 always take FP32 tiles */
} henn_build_params;

/* Search flags (bits 4..32 are taken by the test-only flags of
 * henn_testing.h) */
#define HENN_SEARCH_COUNTERS 1u   /* fill counters[] */
#define HENN_SEARCH_PERSISTENT 2u /* one persistent launch pulling queries from a
                                     device work counter (batched form) */
#define HENN_SEARCH_EXACT_VISITED 64u /* remember every evaluated node exactly (a bit
                                     per member of the largest layer and query,
                                     nq * ceil(n / 32) * 4 bytes of workspace)
                                     instead of the LDS table that may forget:
                                     same results, slower; the evaluation
                                     counters then count each node once per
                                     layer, as the method does */

typedef struct {
  uint32_t struct_size;   /* = sizeof(henn_search_params) */
  uint32_t flags;         /* HENN_SEARCH_* */
  const int32_t *k;       /* device [nq] per-query k, or NULL -> k_all */
  const int32_t *ef;      /* device [nq] per-query beam width, or NULL -> ef_all */
  int32_t k_all;          /* k when k == NULL */
  int32_t ef_all;         /* beam width when ef == NULL */
  int32_t k_max;          /* output row stride; >= every k */
  int32_t ef_max;         /* upper bound of every ef (sizes on-chip lists) */
  int32_t ef_upper;       /* beam width on layers L..1 (1 = Alg. 4 greedy) */
  int32_t rerank_factor;  /* precision forms: re-rank min(|W|, factor*k) in FP32 */
  int32_t *counters;      /* device [nq][4] or NULL: expansions, distance
                             evaluations, layer-0 expansions, layer-0 evaluations
                             (summed over layers; a complete root counts all its
                             members; without EXACT_VISITED a node the visited
                             table forgot and met again is evaluated and counted
                             again) */
  int32_t lanes_per_vec;  /* 0 = autotuned; else 1, 2, 4, 8 or 16 lanes
                             cooperate on one neighbour vector (those whose
                             chunks per lane, 1 to 8, times lanes equal the
                             row's 8-coordinate chunks rounded up to a power
                             of two; HENN_E_INVAL otherwise) */
  int32_t waves_per_block;/* 0 = autotuned; else 1, 2, 4 or 8 */
  void *ev_begin;         /* hipEvent_t or NULL: recorded on hip_stream right before */
  void *ev_end;           /* and right after the main search kernel (timing only) */
  int32_t vis_bits;       /* 0 = autotuned; else log2 of the per-query visited-table
                             entries in LDS, 8..13 (results do not depend on it).
                             An entry takes 1 byte while n < 2^vis_bits * 255, 2
                             while n < 2^vis_bits * 65535, else 4 */
  int32_t reserved;
  void *workspace;        /* device scratch or NULL; when it holds at least
                             henn_search_workspace_size() bytes the call allocates
                             nothing (needed under hipGraph capture) */
  int64_t workspace_bytes;
  int64_t *query_ns;      /* device [nq] or NULL: each query's time inside the main
                             search kernel, from its wave's first instruction for
                             the query to its last (all layers, the FP32 re-rank
                             and the output rows), on the device's constant-rate
                             clock (10 ns steps on MI355X), in ns.  It counts the
                             time the wave waits on memory and shares its SIMD
                             with other waves; the complete-root scan kernels that
                             run before the search are not included */
} henn_search_params;

typedef struct {
  int64_t size;           /* |L_i| */
  int64_t draws;          /* samples drawn (with replacement), or the halved
                             size ceil(|L_{i-1}| / 2^m) */
  double eps;             /* eps_i used (Eq. (1) or override) */
  int64_t window;         /* minimal heavy ring size floor(eps*s)+1 */
  int32_t attempts;       /* Las-Vegas attempts made */
  int32_t hits;           /* rings hit by the kept attempt */
  int32_t status;         /* 0 base, 1 vacuous (window > s), 2 verified,
                             3 not verified (best attempt kept) */
  int32_t degree;         /* adjacency row stride of the layer */
  int32_t fallback_rows;  /* rows whose shortlist was re-solved exactly */
  int32_t reserved;
} henn_layer_info;

/* Fills *p with the defaults: L2, max_layers -1, m 4, c0 1, no override,
 * 64 rings, 64 attempts, degree 16, max_degree 32, kNN graph, F32, seed 0,
 * root_complete_max 0, DRAWS sampler, ef_construction 256, insert_shift 3,
 * phi 0.5, gram 0 (split BF16). */
henn_status henn_default_build_params(henn_build_params *p);

/* Defaults: no per-query arrays, k_all 10, ef_all 32, k_max 10, ef_max 32,
 * ef_upper 1, rerank_factor 4, no counters, autotuned launch shape. */
henn_status henn_default_search_params(henn_search_params *p);

/* Alg. 1 (BuildHENN) on the GPU.
 *   X: device, FP32 row-major [n][d]; copied into library memory, so the
 *      caller may free it on return.
 *   n in [1, 2^31 - 1]; d in [1, 1024].
 *   *out: receives a new index owned by the library (free with henn_free).
 * Blocks: the Las-Vegas decisions of Alg. 2 are taken on the host, so the
 * call synchronises hip_stream.  Returns HENN_W_NOT_VERIFIED (index usable)
 * when a layer kept its best unverified attempt. */
henn_status henn_build(const float *X, int64_t n, int32_t d, const henn_build_params *p,
                       void *hip_stream, henn_index **out);

/* Batched k-NN search (Alg. 4 Query; beam of max(ef, k) on layer 0, Sec. 2.2).
 *   Q: device, FP32 row-major [nq][d] (d of the index).
 *   out_ids: device int32 [nq][k_max]; out_dist: device float [nq][k_max].
 *   Row i holds the first k_i results in ascending (distance, id) order,
 *   padded with id -1 and distance +inf (also when fewer than k_i points are
 *   reachable).  HENN_E_UNSUPPORTED when n * ceil(d / 8) >= 2^32 (rows are
 *   addressed by a 32-bit chunk index).  nq = 0 is a no-op.  Enqueued on hip_stream; results are
 *   valid once the stream has reached this point.  The index is read-only;
 *   concurrent searches on several streams are safe. */
henn_status henn_search_batch(const henn_index *idx, const float *Q, int64_t nq,
                              const henn_search_params *sp, int32_t *out_ids, float *out_dist,
                              void *hip_stream);

/* henn_search_batch for callers that cannot allocate device memory: code
 * under hipGraph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, results and stream semantics as
 * henn_search_batch (sp->workspace is ignored); the scratch the search
 * needs (the persistent work counter and the complete-root scan's keys,
 * henn_search_workspace_size bytes) comes from a fixed 32 MiB device array
 * that the library holds once per GPU until the process ends, so the call
 * makes no allocation at all.  HENN_E_INVAL when the search needs more
 * scratch than that (e.g. more than ~240,000 queries on a complete root of
 * a few thousand points).  Every call on one GPU shares its array: calls
 * whose work overlaps on that GPU (several streams, or host threads) race
 * and must be serialised by the caller; calls in one stream are safe. */
henn_status henn_search_batch_noalloc(const henn_index *idx, const float *Q, int64_t nq,
                                      const henn_search_params *sp, int32_t *out_ids,
                                      float *out_dist, void *hip_stream);

/* Autotuner for the batched search.  Times candidate launch shapes (lanes
 * cooperating on one neighbour vector, waves per workgroup, visited-table
 * size in LDS, one-shot vs persistent launch) on the given queries with the
 * given search parameters, writes *sp with the tuned fields set into
 * *tuned (may be NULL), and caches the choice in the index for later calls
 * whose tuned fields are 0 and whose storage, beam-width bucket and k_max
 * bucket match.  Results never depend on the shape (every shape computes the
 * same canonical distances), only the speed does.
 *   Q: device FP32 [nq][d] calibration queries (nq >= 1); outputs are
 *   scratch allocated inside.  Synchronous on hip_stream.
 *   The cache write is guarded by a mutex; concurrent searches may run. */
henn_status henn_autotune(henn_index *idx, const float *Q, int64_t nq,
                          const henn_search_params *sp, void *hip_stream,
                          henn_search_params *tuned);

/* Scratch bytes henn_search_batch needs for nq queries with these params
 * (root-scan partial results and the persistent work counter); 0 when it
 * needs none.  Host-only. */
henn_status henn_search_workspace_size(const henn_index *idx, int64_t nq,
                                       const henn_search_params *sp, int64_t *bytes);

/* Batched form captured once in a hipGraph: the launches of one
 * henn_search_batch(idx, Q, nq, sp, out_ids, out_dist) call (root scan,
 * counter reset, persistent search) are recorded on a private stream and
 * instantiated; henn_search_graph_launch replays them on hip_stream.  Q and
 * the outputs are bound at creation: refill Q in place between replays.
 * The graph owns its workspace; it holds no memset nodes.  The index and the
 * bound buffers must outlive the graph. */
typedef struct henn_search_graph henn_search_graph;
henn_status henn_search_graph_create(const henn_index *idx, const float *Q, int64_t nq,
                                     const henn_search_params *sp, int32_t *out_ids,
                                     float *out_dist, henn_search_graph **out);
/* Replays the graph on hip_stream.  HENN_E_INVAL for a null graph, or once the
 * index has been changed by henn_insert / henn_delete since the capture (the
 * graph holds the old layer arrays). */
henn_status henn_search_graph_launch(henn_search_graph *g, void *hip_stream);
void henn_search_graph_free(henn_search_graph *g);

/* ---------------------------------------------------------------------
 * Serving form: a continuous-batching request loop on one index.
 * Requests wait in a host FIFO and are admitted at a tick when a slot is
 * free and the device state pool has room for the request's traversal
 * state (list of next_pow2(max(ef, k, ef_upper)) 8-byte keys + the visited
 * table, rounded to 256 B): admission is by memory (a finished request's
 * block is reused by later requests whose state has the same size; the rest
 * comes from the unused part of the pool).  Each tick advances every
 * admitted request by at most steps_per_tick expansions in one launch, so
 * new requests join while others are in flight.  Results equal those of
 * henn_search_batch with the same shape (the traversal code is shared and
 * each request's state is private), whatever else is in flight.
 * The server uses its own non-blocking stream; the index must outlive it.
 * Not thread-safe: one host thread drives a server.
 * --------------------------------------------------------------------- */
typedef struct henn_server henn_server;

typedef struct {
  uint32_t struct_size;   /* = sizeof(henn_server_params) */
  int32_t max_slots;      /* requests in flight at most */
  int64_t pool_bytes;     /* device bytes for per-request traversal state */
  int32_t steps_per_tick; /* expansions per request per tick */
  int32_t k_max;          /* largest k; result row width */
  int32_t ef_max;         /* largest beam width */
  int32_t ef_upper;       /* beam width above layer 0 */
  int32_t rerank_factor;  /* precision forms */
  int32_t lanes_per_vec;  /* 0 = the shape henn_autotune chose for this index and
                             storage (its beam bucket first), else the default */
  int32_t waves_per_block;
  int32_t vis_bits;       /* 0 = by beam width, as henn_search_batch chooses */
} henn_server_params;

typedef struct {
  int64_t pending, active, completed, admitted, ticks, pool_bytes_used, max_active,
      done_queued, cancelled;
} henn_server_stats_t;

/* Defaults: 4096 slots, 64 MiB pool, 16 steps per tick, k_max 10,
 * ef_max 128, ef_upper 1, rerank_factor 4. */
henn_status henn_default_server_params(henn_server_params *p);
henn_status henn_server_create(const henn_index *idx, const henn_server_params *p,
                               henn_server **out);
/* q_host: host FP32 [d], copied.  1 <= k <= k_max, max(ef, k) <= ef_max. */
henn_status henn_server_submit(henn_server *s, const float *q_host, int32_t k, int32_t ef,
                               int64_t tag);
/* n requests at once: q_host FP32 [n][d], k[n], ef[n], tags[n] (host). */
henn_status henn_server_submit_batch(henn_server *s, const float *q_host, const int32_t *k,
                                     const int32_t *ef, const int64_t *tags, int64_t n);
/* Retires the requests the previous tick's step finished to the completion
 * queue, admits what fits into the freed slots, and launches one step of
 * every active request.  The queries of the requests that may be admitted
 * are copied while the previous step still runs, and the tick returns
 * without waiting for its own step, so the caller's work between ticks
 * overlaps the device: a request's result reaches the completion queue in
 * the tick after the one whose step finished it, and its slot is taken by a
 * waiting request in that same tick (call tick until every result has been
 * polled).
 * *n_active (may be NULL): requests in this tick's step.
 * HENN_E_INVAL once the index has been changed by henn_insert / henn_delete
 * since the server was created. */
henn_status henn_server_tick(henn_server *s, int32_t *n_active);
/* Drains up to max_results completions: tags[n], ids[n][k_max],
 * dist[n][k_max] (host; any may be NULL), *n_out. */
henn_status henn_server_poll(henn_server *s, int32_t max_results, int64_t *tags, int32_t *ids,
                             float *dist, int32_t *n_out);
henn_status henn_server_stats(const henn_server *s, henn_server_stats_t *out);
/* Cancels the request submitted with this tag (tags are meant to be unique;
 * with repeated tags, a waiting request is taken before an admitted one).
 * *state (may be NULL):
 *   0 no such request;
 *   1 it was waiting for admission: removed, it will not run;
 *   2 it was admitted: it returns no result, and its slot and state bytes
 *     are freed by the next tick (the step in flight may still advance it);
 *   3 it had already finished: its result stays in the completion queue.
 * Searching a waiting request is linear in the queue length (and removing
 * one moves the requests behind it), so cancellation is for the occasional
 * request, not the common path. */
henn_status henn_server_cancel(henn_server *s, int64_t tag, int32_t *state);
void henn_server_destroy(henn_server *s);

/* Releases the index.  No enqueued work may still use it.  NULL is a no-op. */
void henn_free(henn_index *idx);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *henn_last_error(void);

/* Number of layers (L + 1, layer 0 included) and the point dimension. */
henn_status henn_index_shape(const henn_index *idx, int32_t *num_layers, int64_t *n,
                             int32_t *d);

/* Build record of layer i (host struct). */
henn_status henn_layer_info_get(const henn_index *idx, int32_t layer, henn_layer_info *info);

/* Copies layer i to host memory:
 *   ids_host: int32 [|L_i|] ascending point ids (may be NULL);
 *   adj_host: int32 [|L_i|][degree] neighbour positions within the layer's
 *             id list, in (distance, id) order, -1 padded (may be NULL).
 * Synchronous. */
henn_status henn_export_layer(const henn_index *idx, int32_t layer, int32_t *ids_host,
                              int32_t *adj_host);

/* Builds an index from given layers instead of sampling them (for parity
 * runs on a hierarchy produced elsewhere).
 *   X: device FP32 [n][d] (copied).  p: metric, storage and degree are used.
 *   sizes[i], ids_host[i] (int32 [sizes[i]], ascending, ids_host[0] may be
 *   NULL meaning 0..n-1), adj_host[i] (int32 [sizes[i]][adj_stride], local
 *   positions, -1 padded): host arrays for i < num_layers.
 * Synchronous. */
henn_status henn_import(const float *X, int64_t n, int32_t d, const henn_build_params *p,
                        int32_t num_layers, const int64_t *sizes,
                        const int32_t *const *ids_host, const int32_t *const *adj_host,
                        int32_t adj_stride, void *hip_stream, henn_index **out);

/* Insert(x) of the dynamic setting (App. C) for an index built with the NSW
 * graph: appends count points with ids N, N+1, ..., N+count-1, where N is one
 * past the largest id the index ever held (n for a fresh index).
 *   X_new: device FP32 [count][d] (copied).
 * Every new point joins layer 0; a new member g of layer i-1 also joins layer
 * i when u(word g of stream (tag 5, layer i, attempt 0), 2^m) = 0, i.e. with
 * probability 2^-m, which keeps each layer a random sample of the one below
 * (no new layers are added).  Each layer graph takes its new members by NSW
 * insertion (HENN_GRAPH_NSW rule, continuing the build's batch schedule from
 * the layer's old size); the precision-form copies and a complete root's scan
 * data are rebuilt.  The eps-net check is not re-run: layer_info keeps the
 * build's verification record.
 * Errors: HENN_E_UNSUPPORTED for other graph kinds; HENN_E_INVAL for a null
 * index or X_new, count < 0 or N + count >= 2^31.  On HENN_E_DEVICE /
 * HENN_E_NOMEM the index may be partly grown and should be freed.
 * Blocking; no search may use the index meanwhile, and captured search graphs
 * and servers of the index must be created again afterwards
 * (henn_search_graph_launch and henn_server_tick return HENN_E_INVAL for
 * ones made before). */
henn_status henn_insert(henn_index *idx, const float *X_new, int64_t count, void *hip_stream);

/* Delete(x) of the dynamic setting (App. C) for an index built with the NSW
 * graph.
 *   ids_host: host int32 [count] point ids to delete (repeats are ignored);
 *   each must be in the index, and at least one point must remain.
 * Every deleted point leaves every layer.  In each layer, every remaining
 * row that linked to a deleted member is replaced by the first max_degree of
 * the remaining points among its row and the rows of its deleted neighbours
 * (itself and repeats left out), in (distance, id) order; then the layer is
 * compacted (positions stay in id order).  A layer i >= 1 left with fewer
 * than half of ceil(|L_{i-1}| / 2^m) members is drawn again from L_{i-1}
 * with the build's sampler, ring check and streams, together with every
 * layer above it, and those layers get new NSW graphs.  Ids of the remaining
 * points do not change, and ids are never reused by henn_insert (which
 * continues after the largest id ever given).
 * Errors: HENN_E_UNSUPPORTED for other graph kinds; HENN_E_INVAL for a null
 * index or ids_host, count < 0, an id not in the index, or deleting every
 * point (nothing is changed then).  On HENN_E_DEVICE / HENN_E_NOMEM the index
 * may be partly changed and should be freed.
 * Blocking; no search may use the index meanwhile, and captured search graphs
 * and servers of the index must be created again afterwards
 * (henn_search_graph_launch and henn_server_tick return HENN_E_INVAL for
 * ones made before). */
henn_status henn_delete(henn_index *idx, const int32_t *ids_host, int64_t count,
                        void *hip_stream);

/* One batch of the NSW insertion (App. B.2; the HENN_GRAPH_NSW rule) on a
 * graph the caller holds, e.g. to grow a layer graph or to check a batch.
 *   V:   device FP32 [s][d] row-major, the layer's points in insertion order
 *        (only rows < hi are read); d in [1, 1024]; metric a henn_metric.
 *   adj: device int32 [s][max_degree] positions, -1 padded at the end of a
 *        row; rows < lo hold the graph on [0, lo), rows [lo, hi) are
 *        overwritten with the new points' rows, rows < lo that some new
 *        point links to are replaced by their merged rows, rows >= hi are
 *        not touched.
 *   0 <= lo <= hi <= s < 2^31; degree (R) in [1, 32]; max_degree in
 *   [degree, 64]; ef_construction in [1, 2048].
 * Blocking: returns after the batch is complete on hip_stream.  On error
 * adj may be partly updated only when the error is HENN_E_DEVICE. */
henn_status henn_nsw_insert(const float *V, int64_t s, int32_t d, int32_t metric, int32_t *adj,
                            int32_t max_degree, int64_t lo, int64_t hi, int32_t degree,
                            int32_t ef_construction, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* HENN_H */
