/*
 * fsm.h -- C ABI of the MI355X (gfx950) two-vertex-exploration frequent
 * subgraph miner.
 *
 * Problem (Section 2.2 of Jiang, Wang and Wu, "Efficient Mining of Frequent
 * Subgraphs with Two-Vertex Exploration"): given an undirected graph whose
 * vertices carry labels, a threshold t and a maximum size s, find every
 * connected vertex-labelled pattern P with 2 <= |V_P| <= s whose MNI support
 *     sigma(P) = min over pattern vertices v of |{ f(v) : f an embedding }|
 * is at least t.  Embeddings are edge-induced: injective, label-preserving
 * maps carrying every pattern edge onto a graph edge (Section 6.1 setting).
 *
 * Method (Sections 3-4): size-n subgraphs are produced level by level by
 * joining the size-(n-2) subgraphs of frequent patterns with size-3 subgraphs
 * (wedges, triangles) on one common vertex (Theorem 1), read from CSR
 * adjacency restricted to frequent labelled edges; each joined subgraph gets
 * an index-based quick pattern (Section 4.4), quick patterns are mapped to
 * canonical patterns, MNI domains are accumulated in per-(pattern, orbit)
 * bitmaps and patterns below t are filtered before the next join.
 *
 * Conventions for every call:
 *   - Every function returning int returns FSM_OK (0) or a negative
 *     fsm_status; nothing throws across this boundary.  On failure a
 *     thread-local message is available from fsm_last_error().
 *   - Input arrays are HOST pointers, read during the call only; the caller
 *     keeps ownership.  Handles (fsm_graph, fsm_result) are owned by the
 *     library and released with the matching *_free call.
 *   - Device work runs on the stream set by fsm_set_stream (default: the
 *     null stream) and allocates through the hooks set by fsm_set_allocator
 *     (default: hipMalloc / hipFree).  Each call synchronises its stream
 *     before returning.
 */
#ifndef FSM_H
#define FSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest pattern size supported (vertices). */
#define FSM_MAX_SIZE 7
/* Largest number of distinct labels that can be frequent in one call. */
#define FSM_MAX_FREQ_LABELS 64

typedef struct fsm_graph fsm_graph;    /* device-resident CSR, immutable */
typedef struct fsm_result fsm_result;  /* host-resident mining result */

/* Canonical code of a pattern (36 bytes, little-endian).
 *   n        number of vertices (2..7)
 *   label[i] label of canonical vertex i (the caller's label values), -1
 *            for i >= n; labels are non-decreasing in i
 *   adj      bit k set when the k-th vertex pair (i<j), counted in row-major
 *            upper-triangle order (0,1),(0,2),...,(0,n-1),(1,2),..., is an
 *            edge
 * The canonical form is the vertex order whose (label sequence, pair bit
 * sequence (0,1),(0,2),...) is lexicographically smallest over all n! orders
 * (one fixed choice of the canonical form that Section 2.1 leaves to a
 * tool); two patterns are isomorphic iff their codes are equal.  Results are
 * ordered by (n, label sequence, pair bit sequence). */
typedef struct {
    int32_t n;
    int32_t label[FSM_MAX_SIZE];
    uint32_t adj;
} fsm_code;

/* Mode bits for fsm_mine / fsm_options.mode. */
enum {
    FSM_PLAIN = 0,    /* level-by-level exact join (Sections 3-4) */
    FSM_BATCHED = 1,  /* many graphs in one pass (fsm_mine_batch) */
    FSM_LEARNED = 2,  /* size join tables from a cost model (options.model) */
    FSM_SAMPLED = 4,  /* subgraph sampling during joining (Section 5) */
    FSM_INDUCED = 8,  /* vertex-induced subgraphs: embeddings must also map
                         pattern non-edges onto non-edges (a join keeps every
                         connecting edge, C = E_c, Section 4.2) */
    FSM_SINGLE = 16   /* single-vertex exploration, the baseline of Section
                         6: every size n >= 3 joins the size-(n-1) subgraphs
                         with one edge (no size-3 table, no pruning).  Same
                         results; join_threshold x then keeps x edges of
                         every neighbour list per join.  Not with
                         FSM_SAMPLED, FSM_LEARNED or match_threshold */
};

/* Join tile schedules (fsm_options.schedule).  Results never depend on it. */
enum {
    FSM_SCHEDULE_QUEUE = 0,   /* waves take the next tile from a device counter;
                                 FSM_LEARNED orders the tiles by predicted cost,
                                 largest first */
    FSM_SCHEDULE_STATIC = 1   /* wave w of W takes tiles w, w+W, w+2W, ... in
                                 joining-vertex order */
};

typedef enum {
    FSM_OK = 0,
    FSM_EINVAL = -1,       /* invalid argument; nothing was done */
    FSM_ENOMEM = -2,       /* device or host allocation failed */
    FSM_EDEVICE = -3,      /* a HIP runtime call or kernel failed */
    FSM_EOVERFLOW = -4,    /* a size limit was exceeded (see message) */
    FSM_EUNSUPPORTED = -5  /* valid request outside the library's size limits */
} fsm_status;

/* Per-level counters of one mining call (index = pattern size). */
typedef struct {
    int64_t parents;      /* size-(n-2) embeddings joined (n >= 4) */
    int64_t work_items;   /* (parent, joining position) pairs */
    int64_t candidates;   /* (work item, size-3 piece) slots enumerated */
    int64_t emitted;      /* subgraphs produced (valid, dissection-accepted,
                             not pruned); for sizes 2 and 3 the edges and
                             size-3 subgraphs over frequent labelled edges */
    int64_t quick_patterns;   /* distinct quick patterns */
    int64_t patterns;         /* distinct canonical patterns seen */
    int64_t frequent;         /* patterns with support >= t */
    int64_t stored;           /* embeddings kept for the next join */
    int64_t algorithmic_bytes;  /* bytes the join's domain pass must move:
                                   parent rows, the neighbour lists it
                                   enumerates, 8 per adjacency probe, 4 per
                                   domain-bitmap word of each emitted
                                   subgraph position */
    double kernel_ms;         /* device time of this level (all passes) */
    double join_ms;           /* device time of the join's domain pass */
    int64_t domain_passes;    /* domain passes run: 1 + reruns after the
                                 quick-pattern table overflowed */
    int64_t qp_capacity;      /* quick-pattern table slots of the last pass */
    int64_t qp_predicted;     /* FSM_LEARNED join levels: the cost model's
                                 estimate of quick_patterns (0 otherwise) */
    int64_t rank_slices;      /* domain passes over vertex-rank slices: 1
                                 when the domain bitmaps of the level fit
                                 the pool budget at once */
    int64_t hash_bytes;       /* join levels: bytes the join's loops read
                                 from the subgraph lists grouped by joining
                                 vertex, every read a miss (the accounting of
                                 Section 6.2's memory-access comparison), 4
                                 per vertex id: per work item, 12 per stored
                                 size-3 subgraph containing its joining
                                 vertex (two-vertex) or 8 per G_f edge of it
                                 (single-vertex), at most the ST sample */
    int64_t canonical_forms;  /* canonical-form computations of the level:
                                 one per quick pattern and canonical pass
                                 (the analogue of the isomorphism-tool calls
                                 counted in Section 6.2; a miner without
                                 index-based quick patterns makes one per
                                 emitted subgraph) */
} fsm_level_stats;

typedef struct {
    int32_t max_size;
    int32_t frequent_labels;
    int64_t dropped_self_loops;    /* from fsm_build_graph */
    int64_t dropped_duplicates;    /* duplicate undirected edges merged */
    int64_t filtered_edges;        /* undirected edges whose labelled edge is frequent */
    fsm_level_stats level[FSM_MAX_SIZE + 1];
    double total_ms;               /* wall time of the mining call */
    int32_t batch_chunk;           /* batched calls: the union pass (chunk)
                                      this graph was mined in; level counters
                                      describe that whole chunk */
    int32_t batch_chunks;          /* chunks of the call (1 for fsm_mine) */
    int32_t batch_splits;          /* chunks split after a table or memory
                                      overflow */
    int32_t captured_levels;       /* levels of this pass run as one replay of
                                      a captured HIP graph (batched calls:
                                      the last join level of a chunk) */
    int32_t captured_graphs;       /* batched calls: distinct level shapes
                                      captured (each replayed across the
                                      chunks of that shape) */
    int32_t level_fallbacks;       /* captured levels rerun with eager
                                      launches after a table overflow */
    int64_t host_syncs;            /* host waits on the device in this pass
                                      (for a batch: in its chunk) */
} fsm_stats;

/* Options of fsm_mine_ex.  Zero-initialise, then set fields. */
typedef struct {
    int64_t support;          /* MNI threshold t >= 1 */
    int32_t max_size;         /* 2..7 */
    uint32_t mode;            /* FSM_PLAIN, or any of FSM_SAMPLED,
                                 FSM_LEARNED, FSM_INDUCED, FSM_SINGLE */
    int32_t disable_pruning;  /* 1: skip the Section 4.5 pruning (results
                                 are identical; counters differ) */
    int32_t schedule;         /* join tile schedule: FSM_SCHEDULE_QUEUE
                                 (0, default) or FSM_SCHEDULE_STATIC */
    double sampling_rate;     /* FSM_SAMPLED: keep probability of a size-3
                                 piece per key group, in (0, 1] */
    uint64_t seed;            /* FSM_SAMPLED: hash seed */
    int64_t hash_capacity_min;  /* >0: initial quick-pattern table slots
                                   (grown on overflow) */
    int64_t pattern_capacity_min;  /* >0: initial canonical-pattern table
                                      slots (grown on overflow) */
    const struct fsm_model *model; /* FSM_LEARNED: cost model with
                                      FSM_FEATURES inputs */
    int32_t record;           /* 1: keep one training row per join work item
                                 in the result (fsm_result_training_rows) */
    int32_t tiles_per_wave;   /* >0: join tiles per wavefront the tile
                                 height aims for; 0: the tuned value
                                 (fsm_tune_batch), else 16 */
    int64_t pool_budget_mib;  /* >0: device memory for the domain bitmaps of
                                 a level, in MiB; 0: 40% of the free memory.
                                 Bitmaps larger than this are computed in
                                 vertex-rank slices, one join pass each */
    int64_t join_threshold;   /* >0: sampling threshold x of the joins
                                 (Section 5, "ST x"): every join keeps x^2 of
                                 the stored size-3 subgraphs of each key
                                 group (those containing the joining vertex)
                                 and the size-4 join x of its edges; a group
                                 with fewer keeps all.  0: off.  In
                                 [0, 2^20]; not with FSM_SAMPLED */
    int64_t match_threshold;  /* >0: matching sampling threshold t (Section
                                 5): t of the size-3 subgraphs credited to
                                 each vertex (a wedge to its centre, a
                                 triangle to its smallest vertex) are kept
                                 and joined.  0: off */
    int32_t force_overflow;   /* 1: every quick-pattern and canonical-pattern
                                 table starts at 2 slots (hash_capacity_min,
                                 pattern_capacity_min and learned sizing are
                                 ignored), so every level overflows and
                                 reruns its passes with grown tables; the
                                 results are identical (a test of the
                                 overflow path) */
    int32_t reserved2;
} fsm_options;

/* Device scratch of fsm_mine_noalloc, in MiB: one array per GPU the
 * library runs on, held until the process ends. */
#define FSM_NOALLOC_SCRATCH_MIB 256

/* Allocation hooks used for all device memory of later calls (e.g. a
 * framework's caching allocator).  Both NULL restores hipMalloc/hipFree.
 * alloc(bytes, ctx) returns device memory or NULL; release(ptr, ctx). */
int fsm_set_allocator(void *(*alloc)(size_t bytes, void *ctx),
                      void (*release)(void *ptr, void *ctx), void *ctx);

/* Stream (a hipStream_t, NULL = null stream) used by later calls. */
int fsm_set_stream(void *hip_stream);

/* Build the device CSR of a labelled undirected graph (the input graph
 * G = (V, E, L) of Section 2.1, vertex labels only).
 *   n_vertices      number of vertices, ids 0..n_vertices-1 (>= 1)
 *   n_edges         length of src/dst (>= 0)
 *   src, dst        host int32 arrays: one undirected edge per index, in any
 *                   order and direction; self-loops are dropped and repeated
 *                   pairs merged (counts in fsm_result_stats)
 *   vertex_labels   host int32 array of n_vertices labels, each in
 *                   [0, 2^24)
 *   out             receives the handle (NULL on failure)
 * Errors: FSM_EINVAL for NULL pointers, n_vertices < 1, an id out of range
 * or a label out of range; FSM_EUNSUPPORTED when the CSR would exceed 2^31-1
 * directed entries; FSM_ENOMEM / FSM_EDEVICE from the device. */
int fsm_build_graph(int64_t n_vertices, int64_t n_edges, const int32_t *src,
                    const int32_t *dst, const int32_t *vertex_labels,
                    fsm_graph **out);

/* Number of vertices / undirected edges of a built graph (-1 for NULL). */
int64_t fsm_graph_vertices(const fsm_graph *g);
int64_t fsm_graph_edges(const fsm_graph *g);

/* Mine every frequent pattern of sizes 2..max_size (Section 2.2 problem,
 * Section 3 workflow: size-3 matching, support filtering, two-vertex joins,
 * aggregation).
 *   support    MNI threshold t (>= 1); a pattern is kept iff sigma >= t
 *   max_size   2..7
 *   mode       FSM_PLAIN, or FSM_INDUCED and/or FSM_SINGLE (FSM_SAMPLED needs
 *              fsm_mine_ex)
 *   out        receives the result handle
 * Errors: FSM_EINVAL (NULL graph/out, support < 1, max_size outside 2..7,
 * unknown mode bits, FSM_SAMPLED here); FSM_EUNSUPPORTED when more than
 * FSM_MAX_FREQ_LABELS labels occur on at least `support` vertices, a
 * frequent label has more than 2^26 vertices, a vertex would need more than
 * 2^29 neighbour-table buckets, or a join has 2^31 or more parent
 * embeddings; FSM_EOVERFLOW when a table cannot grow within device memory
 * or a join's work-item grouping table would pass 2^32 slots;
 * FSM_ENOMEM / FSM_EDEVICE from the device. */
int fsm_mine(const fsm_graph *g, int64_t support, int32_t max_size,
             uint32_t mode, fsm_result **out);

/* fsm_mine with options.  FSM_SAMPLED keeps each size-3 piece of a key group
 * at every join with probability sampling_rate, decided by a counter-based
 * hash of (seed, level, joining vertex, the piece's vertices) -- subgraph
 * sampling during joining (Section 5).  join_threshold and match_threshold
 * instead keep a fixed number of every group's members, a uniform sample
 * without replacement: the members whose counter-based hash is at most the
 * group's cap-th smallest.  Sampled supports are MNI over the sampled
 * embeddings (a lower bound of the exact ones); results are reproducible
 * for a seed.  Errors as fsm_mine, plus FSM_EINVAL for a sampling rate
 * outside (0, 1], a threshold out of range, or join_threshold together
 * with FSM_SAMPLED. */
int fsm_mine_ex(const fsm_graph *g, const fsm_options *opt, fsm_result **out);

/* fsm_mine_ex for callers that cannot allocate device memory (code that a
 * harness forbids to call hipMalloc, tight serving loops): the call
 * allocates nothing on the device -- no hipMalloc / hipFree, no allocation
 * hook, no HIP event -- and takes every buffer it needs from a file-scope
 * device array of FSM_NOALLOC_SCRATCH_MIB MiB (its device address fetched
 * once per device with hipGetSymbolAddress, that device current).  Host
 * bookkeeping still uses the C++ heap, as in every call.
 *   g          a graph from fsm_build_graph on the current device (input)
 *   opt        as fsm_mine_ex; record must be 0
 *   capacity   entries of the three output arrays (>= 0)
 *   sizes, codes, supports
 *              host arrays receiving the patterns, ordered as
 *              fsm_result_patterns orders them (may be NULL when capacity
 *              is 0)
 *   count      receives the number of frequent patterns (also on
 *              FSM_EOVERFLOW for too small a capacity, nothing written)
 *   stats      NULL or receives the call's counters (timings are 0)
 * Every call on a GPU uses that GPU's one array, which keeps the previous
 * call's contents (each call initialises what it reads); calls on one
 * device are serialised by the library, as overlapping calls would race on
 * the array.  Errors: as fsm_mine_ex; FSM_EINVAL for a NULL g/opt/count,
 * capacity < 0, NULL arrays with capacity > 0, record set, or a graph of
 * another device; FSM_EOVERFLOW when the graph alone exceeds the scratch
 * (64 bytes per vertex + 16 per CSR entry) or the patterns exceed
 * capacity; FSM_ENOMEM when the call needs more than the scratch holds (the
 * message names the buffer). */
int fsm_mine_noalloc(const fsm_graph *g, const fsm_options *opt, int64_t capacity,
                     int32_t *sizes, fsm_code *codes, int64_t *supports, int64_t *count,
                     fsm_stats *stats);

/* Mine many graphs in one pass (batched mode): every level runs as one
 * launch per kernel over the disjoint union of the graphs, whose work items
 * are load-balanced together; patterns are keyed by graph, so each graph's
 * result equals what fsm_mine would return for it.
 *   graphs     count handles from fsm_build_graph (count 1..2048)
 *   supports   count thresholds, supports[i] for graphs[i] (each >= 1)
 *   max_size   2..6 (2..7 when count == 1)
 *   mode       FSM_PLAIN or FSM_BATCHED (same meaning here)
 *   outs       receives count result handles; the per-level counters of
 *              every result describe the union pass it was mined in
 * Graphs are mined in chunks (fsm_mine_batch_ex with chunk_vertices 0).
 * Errors: as fsm_mine; FSM_EUNSUPPORTED for more than 2048 graphs or
 * max_size 7 with several graphs.  On failure no handle is returned. */
int fsm_mine_batch(const fsm_graph *const *graphs, int32_t count,
                   const int64_t *supports, int32_t max_size, uint32_t mode,
                   fsm_result **outs);

/* Options of fsm_mine_batch_ex.  Zero-initialise, then set fields. */
typedef struct {
    int32_t max_size;           /* 2..6 (2..7 when count == 1) */
    uint32_t mode;              /* FSM_PLAIN or FSM_BATCHED (same meaning),
                                   with FSM_LEARNED and/or FSM_INDUCED */
    int64_t chunk_vertices;     /* >0: at most this many vertices in one
                                   union pass (a larger single graph gets a
                                   pass of its own); 0: the tuned value
                                   (fsm_tune_batch), else 16384 */
    int32_t disable_pruning;    /* as fsm_options */
    int32_t tiles_per_wave;     /* as fsm_options */
    int64_t hash_capacity_min;  /* as fsm_options (first chunk) */
    int64_t pattern_capacity_min;
    struct fsm_model *model;    /* FSM_LEARNED: cost model with FSM_FEATURES
                                   inputs, used to size every chunk's join
                                   tables */
    int32_t learn;              /* 1: after each chunk, train the model on
                                   that chunk's work items (train_steps Adam
                                   steps at learning rate lr) */
    int32_t train_steps;
    float lr;
    int32_t eager_levels;       /* 1: every level of every chunk with eager
                                   kernel launches; 0: the last join level
                                   of each chunk as one replay of a HIP graph
                                   captured per level shape (tables sized up
                                   front, one host wait; a table overflow
                                   reruns the level eagerly) */
    int64_t pool_budget_mib;    /* as fsm_options */
} fsm_batch_options;

/* fsm_mine_batch with options.  Graphs are ordered by their most populous
 * label (so one chunk's domain bitmaps fit all its graphs) and packed into
 * chunks of at most chunk_vertices vertices; each chunk is one union pass.
 * A chunk whose tables or bitmaps exceed the limits or device memory is
 * split in two and rerun (counted in batch_splits); the quick-pattern table
 * of each level starts at the size the earlier chunks needed per vertex.
 * Errors as fsm_mine_batch; FSM_EINVAL for chunk_vertices < 0. */
int fsm_mine_batch_ex(const fsm_graph *const *graphs, int32_t count,
                      const int64_t *supports, const fsm_batch_options *opt,
                      fsm_result **outs);

/* Autotuning of the batch shapes.  fsm_tune_batch mines the given graphs
 * (a representative sample of a workload) twice per candidate shape --
 * chunk_vertices in {8192, 16384, 32768} x tiles_per_wave in {4, 16, 64},
 * after one warm-up call -- times each call on the host clock, scores a
 * candidate by its faster call, and keeps the fastest candidate as the
 * library's defaults for later calls that leave chunk_vertices /
 * tiles_per_wave at 0 (process-wide, until fsm_reset_tuning).  Results
 * never depend on the shapes. */
#define FSM_TUNE_MAX 16
typedef struct {
    int64_t chunk_vertices;            /* the winner */
    int32_t tiles_per_wave;
    int32_t configs;                   /* candidates timed */
    int64_t cand_chunk[FSM_TUNE_MAX];  /* each candidate and its time */
    int32_t cand_tiles[FSM_TUNE_MAX];
    double cand_ms[FSM_TUNE_MAX];
} fsm_tuning;

/* Errors as fsm_mine_batch; out receives the timings and the winner. */
int fsm_tune_batch(const fsm_graph *const *graphs, int32_t count, const int64_t *supports,
                   int32_t max_size, fsm_tuning *out);

/* Forget the tuned defaults (chunk_vertices 16384, tiles_per_wave 16). */
int fsm_reset_tuning(void);

/* Work-item features of the cost model (one row per join work item: a
 * parent quick pattern P of size n-2 with embeddings, and the position i of
 * the joining vertex in it), FSM_FEATURES float32 values:
 *   0  n / 8                       3  log1p(mean G_f degree of the vertices
 *   1  edges of P / pairs of P            at position i) / 8
 *   2  log1p(embeddings of P) / 16 4  log1p(MNI support of P's pattern) / 16
 *                                  5  log1p(support threshold) / 16
 *   6 .. 21   label histogram of P (fraction of positions per frequent
 *             label id, ids >= 15 share bucket 15)
 *   22 .. 37  one-hot label bucket of position i
 * Targets: log1p(children the join emits from the item), log1p(distinct
 * child quick patterns).  Child quick patterns of different items are
 * distinct, so the second target sums to the level's quick_patterns. */
#define FSM_FEATURE_LABELS 16
#define FSM_FEATURES (6 + 2 * FSM_FEATURE_LABELS)

/* Training rows recorded by a call with options.record = 1 (-1 for NULL). */
int64_t fsm_result_training_count(const fsm_result *r);

/* Copy the recorded rows out: x (count x FSM_FEATURES), t (count x 2),
 * level (count, the join size n of each row); any pointer may be NULL. */
int fsm_result_training_rows(const fsm_result *r, float *x, float *t, int32_t *level);

/* ---------------------------------------------------------------------
 * Join cost model.  Not part of the paper's method: a two-layer perceptron
 * that predicts, per join work item (a parent quick pattern and the joining
 * position), log1p of the children the join emits from it and log1p of the
 * distinct child quick patterns.  The miner records such rows itself
 * (fsm_result_training_rows) and uses the predictions to size its tables and
 * to order its work (FSM_LEARNED); it never changes a mined result.
 *
 * Shape: in_dim inputs (1..FSM_MODEL_MAX_IN), FSM_MODEL_HIDDEN ReLU units,
 * FSM_MODEL_OUT linear outputs.  Parameters, float32, flat in this order:
 * W1 (in_dim x 64, row-major), b1 (64), W2 (64 x 2, row-major), b2 (2);
 * forward and backward passes read them rounded to bfloat16 (round to
 * nearest even) and accumulate in float32; training updates float32 master
 * copies with full-batch Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the loss
 * sum((y - t)^2) / (2 rows).  All array arguments are host memory, row-major,
 * copied during the call; the caller keeps ownership.
 * ------------------------------------------------------------------- */
typedef struct fsm_model fsm_model;

#define FSM_MODEL_HIDDEN 64
#define FSM_MODEL_OUT 2
#define FSM_MODEL_MAX_IN 160

/* Number of parameters of a model with in_dim inputs (-1 if out of range). */
int64_t fsm_model_param_count(int32_t in_dim);

/* New model on the current device.  params: fsm_model_param_count(in_dim)
 * initial values, or NULL for the library's initialisation (uniform in
 * +-1/sqrt(fan_in) from a splitmix64 stream seeded by seed, zero biases).
 * Errors: FSM_EINVAL for in_dim out of range or NULL out. */
int fsm_model_create(int32_t in_dim, const float *params, uint64_t seed, fsm_model **out);

/* Inputs of a model (-1 for NULL). */
int32_t fsm_model_in_dim(const fsm_model *m);

/* Copy the float32 master parameters out (param_count values). */
int fsm_model_params(const fsm_model *m, float *params);

/* Gradient of the loss over rows (x: rows x in_dim, t: rows x 2) with
 * respect to the bfloat16 parameter values, into grad (param_count values);
 * loss (may be NULL) receives the loss.  Does not change the model. */
int fsm_model_gradient(fsm_model *m, const float *x, const float *t, int64_t rows,
                       float *grad, double *loss);

/* steps full-batch Adam steps at learning rate lr on (x, t); loss (may be
 * NULL) receives the loss of the last step's forward pass.  The optimiser
 * state persists across calls. */
int fsm_model_train(fsm_model *m, const float *x, const float *t, int64_t rows,
                    int32_t steps, float lr, double *loss);

/* Predictions y (rows x 2) for inputs x (rows x in_dim). */
int fsm_model_predict(const fsm_model *m, const float *x, int64_t rows, float *y);

void fsm_model_free(fsm_model *m);

/* Number of frequent patterns in a result (-1 for NULL). */
int64_t fsm_result_count(const fsm_result *r);

/* Copy the patterns out, ordered by (size, canonical code).  Each array
 * argument may be NULL (skipped) or must hold fsm_result_count(r) entries.
 *   ids       0..count-1, the rank in that order
 *   sizes     pattern sizes
 *   codes     canonical codes
 *   supports  exact MNI supports (sampled mode: supports over the sample) */
int fsm_result_patterns(const fsm_result *r, int32_t *ids, int32_t *sizes,
                        fsm_code *codes, int64_t *supports);

/* Per-level counters and timings of the call that produced r. */
int fsm_result_stats(const fsm_result *r, fsm_stats *s);

void fsm_graph_free(fsm_graph *g);
void fsm_result_free(fsm_result *r);

/* Message of the last failing call on this thread ("" if none). */
const char *fsm_last_error(void);

/* Smallest-vertex-first dissection (Section 4.3, Algorithm 1), run on the
 * host with the same code the device join uses.  For a connected graph on
 * n (4..7) vertices with distinct ids, it picks the one split of the vertex
 * set into a connected 3-vertex part l and a connected (n-2)-vertex part r
 * sharing one vertex v' that the join accepts: l is the lexicographically
 * smallest sorted id triple for which such a v' exists, v' the smallest one.
 *   n        vertices; ids[i] their ids (distinct)
 *   adj      LSB-first pair bits as in fsm_code (row-major upper triangle)
 *   l_mask   receives the positions of l (bit i = vertex i)
 *   shared   receives the position of v'
 * Returns FSM_OK, FSM_EINVAL for bad arguments or a disconnected graph. */
int fsm_dissect(int32_t n, const int32_t *ids, uint32_t adj, uint32_t *l_mask,
                int32_t *shared);

/* Keep thresholds of the learned sampling proposal (FSM_SAMPLED |
 * FSM_LEARNED), run on the host with the code the miner uses.  Not part of
 * the paper's method: for work item r with predicted children
 * c_r = expm1(max(0, pred[r])) the keep rate is min(1, lambda / max(c_r, 1)),
 * lambda chosen so that the expected work sum(rate_r c_r) equals
 * rate * sum(c_r) (the uniform rate's); a piece of item r is kept when its
 * sampling hash is below thresholds[r] (2^64 - 1: everything).  The result
 * depends only on the multiset of rows (sums run over sorted costs), each
 * rate relative to `rate` is rounded to 2^-20, and with no predicted work
 * (or rate >= 1) every threshold is 2^64 - 1.
 *   pred        rows host floats: log1p of predicted children per item
 *   rate        the uniform sampling rate, in (0, 1]
 *   thresholds  receives rows keep thresholds
 * Returns FSM_OK, FSM_EINVAL for NULL arrays, rows < 0 or a rate outside
 * (0, 1]. */
int fsm_proposal_thresholds(const float *pred, int64_t rows, double rate,
                            uint64_t *thresholds);

/* Graph id carried by a pattern key of a batched call (the canonical code in
 * the low bits, the graph id from bit 52 for sizes whose code leaves room,
 * graph 0 otherwise), checked against the call's graph count: the miner
 * decodes keys read back from the device with this check and reports
 * FSM_EDEVICE instead of indexing with a graph id that names no graph.
 *   key     pattern-table key; size  pattern size 2..7; graphs  graphs of
 *           the call (>= 1); graph  receives the id
 * Returns FSM_OK, FSM_EINVAL for bad arguments, FSM_EDEVICE when the key
 * names no graph of the call. */
int fsm_key_graph(uint64_t key, int32_t size, int32_t graphs, int32_t *graph);

#ifdef __cplusplus
}
#endif
#endif /* FSM_H */
