/*
 * arb.h — C ABI of the MI355X (gfx950) exact k-clique counting library, libarb.so.
 *
 * The library computes the hot path of arb-count / arb-count-v from Shi, Dhulipala
 * and Shun, "Parallel Clique Counting and Peeling Algorithms" (arXiv 2002.10047):
 *   1. orient an undirected simple graph by peeling low-degree vertices in rounds
 *      (Sec. 3.1; appendix Alg. 4 with the threshold (2+eps) x the average degree of
 *      the vertices still present), then direct every edge from the earlier-peeled
 *      endpoint to the later one (Sec. 3.1, last paragraph);
 *   2. for every vertex, recursively intersect directed out-neighbour sets k-1 levels
 *      deep to count k-cliques (Alg. 1), optionally per vertex (Sec. 3.2, the -v
 *      variant), using the induced subgraph of N+(v) relabelled to local ids
 *      (Sec. 3.4).
 *
 * Conventions shared by every entry point
 *   - Pointers to graph arrays, outputs and workspaces are DEVICE pointers owned by
 *     the caller; the library never allocates or frees device memory (hipMalloc-free,
 *     so every *_async call may be captured into a HIP graph).  Host pointers are
 *     marked "host".
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.  Work
 *     is enqueued on it in order.  Functions documented as "synchronises" wait for
 *     the stream before returning.
 *   - Integer return codes are ARB_* below.  On an error the outputs are unspecified;
 *     nothing else is touched.  arb_last_error() returns the code of the most recent
 *     failing call on the calling host thread.
 *   - Graph layout: CSR with int64 row offsets (n+1 entries, offsets[0] = 0) and int32
 *     column indices.  An undirected graph lists each edge in both rows (nnz = 2m);
 *     rows sorted strictly ascending, no self-loops (the paper's simple undirected
 *     graphs, Sec. 2).  A directed ("oriented") graph lists each edge once, every arc
 *     i -> j has i < j, rows sorted strictly ascending.
 *   - Counts are uint64 modulo 2^64.
 */
#ifndef ARB_H
#define ARB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ARB_OK = 0,
    ARB_EINVAL = 1,      /* bad argument: null pointer, k / eps / n / option out of range */
    ARB_EGRAPH = 2,      /* input graph violates the layout above */
    ARB_EWORKSPACE = 3,  /* workspace smaller than the matching *_workspace() size */
    ARB_EHIP = 4,        /* a HIP runtime call failed */
    ARB_ELIMIT = 5,      /* an implementation limit was exceeded (see ARB_MAX_*) */
    ARB_EMISMATCH = 6    /* two schedules gave different totals (a library defect) */
};

#define ARB_MAX_K 32            /* largest clique size the counting kernels take */
#define ARB_MAX_LOCAL 768       /* largest candidate set held in LDS per work item */
#define ARB_MAX_ROUNDS 64       /* peel rounds recorded in the round statistics */
#define ARB_MAX_ROW_SORT 16384  /* longest directed row the orientation can sort */

typedef struct {
    int64_t n;                 /* vertices */
    int64_t nnz;               /* stored entries = 2 x undirected edges */
    const int64_t *offsets;    /* device, n+1 */
    const int32_t *indices;    /* device, nnz */
} arb_csr;

typedef struct {
    int64_t n;                 /* vertices */
    int64_t m;                 /* arcs = undirected edges */
    int64_t *offsets;          /* device, n+1 */
    int32_t *indices;          /* device, m */
} arb_ocsr;

/* ---------------------------------------------------------------- orientation */

/* Bytes of workspace arb_orient needs for a graph with n vertices and nnz entries
 * (O(n) plus 4 bytes per entry). */
size_t arb_orient_workspace(int64_t n, int64_t nnz);

/*
 * Low out-degree orientation (Sec. 3.1, appendix Alg. 4) and directing (Sec. 3.1).
 *
 * Rounds r = 0, 1, ... over the vertices still present: S_r = sum of their current
 * degrees (int64), c_r = their number, T_r = floor(((2+eps) * S_r) / c_r) evaluated in
 * IEEE double in that order; every present vertex of degree <= T_r is removed in
 * round r, and its degree at the start of the round is recorded; afterwards each
 * removed vertex lowers the degree of every neighbour still present by one.  The
 * ordering sorts vertices by (round, degree at removal, id); rank[v] is v's position.
 * The output is the directed graph in rank space: out->offsets[rank(u)] .. lists
 * rank(w) for every neighbour w with rank(w) > rank(u), ascending.  Since at most
 * c_r/(2+eps) vertices exceed T_r, there are at most ceil(log_{2+eps} n) rounds.
 *
 *   g            undirected input (device arrays)
 *   eps          0 <= eps <= 64
 *   validate     nonzero: check g first (O(n + m log d)); on failure return ARB_EGRAPH.
 *                This synchronises the stream.
 *   out          out->n = g->n, out->m = g->nnz/2; caller allocates offsets (n+1) and
 *                indices (m) on the device
 *   rank         device int32[n] (original id -> rank)
 *   round        device int32[n] (original id -> peel round), nullable
 *   deg_at_peel  device int32[n] (original id -> degree at removal), nullable
 *   stats        device int64[2 + ARB_MAX_ROUNDS], nullable:
 *                [0] rounds used, [1] largest out-degree, [2 + r] = T_r
 *   ws, ws_bytes device workspace of at least arb_orient_workspace(n, nnz) bytes
 * Errors: ARB_EINVAL, ARB_EGRAPH (validate), ARB_EWORKSPACE, ARB_ELIMIT (n >= 2^31,
 * a degree >= 2^26, or a directed row longer than ARB_MAX_ROW_SORT), ARB_EHIP.
 * Without `validate` the call does not synchronise (capture-safe); the ARB_ELIMIT
 * row-length check then only reports through stats[1].
 */
int arb_orient(const arb_csr *g, double eps, int validate, arb_ocsr *out,
               int32_t *rank, int32_t *round, int32_t *deg_at_peel, int64_t *stats,
               void *ws, size_t ws_bytes, void *stream);

/* Orderings for arb_orient_method (Sec. 3.1 and the experiments of Sec. 5):
 *   ARB_ORIENT_PEEL  the peel of arb_orient (degree <= (2+eps) x average remaining);
 *   ARB_ORIENT_DEGREE  by degree (ties by id): one round, round = 0, degree at removal = degree;
 *   ARB_ORIENT_GOODRICH_PSZONA  Alg. 3: each round removes the ceil(eps c / (2 + eps))
 *     present vertices of lowest (degree, id), c = number present (eps > 0);
 *   ARB_ORIENT_KCORE  round r removes every present vertex of degree <= T_r,
 *     T_r = max(T_{r-1}, least degree present) (T_{-1} = 0): a degeneracy ordering,
 *     out-degree <= degeneracy.
 * All rank by (round, degree at removal, id). */
enum { ARB_ORIENT_PEEL = 0, ARB_ORIENT_DEGREE = 1, ARB_ORIENT_GOODRICH_PSZONA = 2, ARB_ORIENT_KCORE = 3 };

/* arb_orient with the ordering `method`; arguments, workspace and errors as arb_orient.
 * stats[0] = rounds (thresholds stats[2..] only for ARB_ORIENT_PEEL).  The Goodrich-
 * Pszona and k-core orderings synchronise the stream (a host check per round / per 64
 * rounds) and cannot be captured. */
int arb_orient_method(const arb_csr *g, int method, double eps, int validate, arb_ocsr *out, int32_t *rank,
                      int32_t *round_out, int32_t *dap_out, int64_t *stats, void *ws, size_t ws_bytes,
                      void *stream);

/* Workspace of arb_orient_batch for a union of G graphs. */
size_t arb_orient_batch_workspace(int64_t n, int64_t nnz, int64_t G);

/* arb_orient for a batch: g is the disjoint union of G graphs, graph i on the vertex
 * range graph_vtx_offsets[i] .. graph_vtx_offsets[i+1]-1 (device int64[G+1], 0 = first,
 * n = last, non-decreasing; no edge between graphs).  Each graph is peeled with its own
 * remaining count, degree sum and threshold per round (Alg. 4 applied to every graph),
 * so every graph gets exactly the orientation, rounds and degrees at removal that
 * arb_orient gives it alone, shifted by its first vertex; its ranks stay inside its own
 * range, so per-graph results of arb_count are contiguous in rank space.  max_graph_n
 * (host) is the largest graph's vertex count and bounds the number of rounds.
 * validate = 1 also checks the ranges and that no edge crosses graphs (ARB_EGRAPH);
 * without it, malformed ranges give wrong results but no access outside the buffers.
 * stats (nullable): stats[0] = rounds used, stats[1] = largest out-degree.  Other
 * arguments and errors as arb_orient. */
int arb_orient_batch(const arb_csr *g, const int64_t *graph_vtx_offsets, int64_t G, int64_t max_graph_n,
                     double eps, int validate, arb_ocsr *out, int32_t *rank, int32_t *round_out,
                     int32_t *dap_out, int64_t *stats, void *ws, size_t ws_bytes, void *stream);

/* Check an undirected CSR: returns ARB_OK or ARB_EGRAPH (synchronises). */
int arb_validate(const arb_csr *g, void *ws, size_t ws_bytes, void *stream);

/* Check a directed CSR: every arc ascends, rows strictly ascending, indices in range.
 * Returns ARB_OK or ARB_EGRAPH (synchronises).  Workspace: arb_count_workspace(). */
int arb_check_oriented(const arb_ocsr *dg, void *ws, size_t ws_bytes, void *stream);

/* out[v] = in_rank_space[rank[v]] for v < n: maps per-vertex results of the rank-space
 * graph back to original ids. */
int arb_permute_u64(const int32_t *rank, const uint64_t *in_rank_space, uint64_t *out,
                    int64_t n, void *stream);

/* ---------------------------------------------------------------- counting */

enum {
    ARB_SCHED_PLAIN = 0,       /* one launch per tier, one team per root, degree-descending */
    ARB_SCHED_PERSISTENT = 1,  /* persistent teams popping a device queue, degree cost */
    ARB_SCHED_LEARNED = 2      /* persistent, queue ordered and split by the MLP cost */
};

typedef struct {
    int schedule;          /* ARB_SCHED_* */
    int split_min_degree;  /* degree schedules: a root with d+ >= this becomes
                              P = ceil(d+ / split_min_degree) parts (at most 64), each
                              building the root's induced subgraph and taking every
                              P-th row of its work; 0 = never split */
    float split_min_cost;  /* learned schedule: a root whose predicted log2(1+work) y is
                              >= this becomes P = ceil(2^(y - split_min_cost)) parts;
                              0 = never split */
    int persist_blocks_per_cu;  /* persistent grid: up to this many blocks per CU (1..8) */
    int chunk_small;       /* items popped at once by single-wave teams (1..256) */
    int bitmap_max_span;   /* membership test of the second level: an id-range bitmap when
                              the members' ids span fewer than this (and the tier's
                              capacity), else a hash; 0 = always hash */
    int concurrent_tiers;  /* nonzero: the tier kernels of a call run side by side on
                              library streams forked from and joined back into `stream`
                              by events (persistent schedules, profiling off) */
    int tier_fill;         /* LDS tile per item, 10..100 (%): an item goes to the first tier
                              (64, 128, 256, 384, 512, 768 local vertices) whose capacity
                              times tier_fill / 100 holds its set, so lower values give
                              items larger tiles and teams of more waves; 100 = the
                              smallest tier that fits */
    int big_max_degree;    /* roots with ARB_MAX_LOCAL < d+ <= big_max_degree are counted
                              whole by the global-scratch kernel (bit rows in the
                              workspace), larger ones as one (root, child) item per
                              out-neighbour; -1 = as large as the workspace allows */
    const uint16_t *mlp_weights; /* device bf16 weights for ARB_SCHED_LEARNED (8641) */
    const float *features;       /* device float[n][3] from arb_features, ARB_SCHED_LEARNED */
} arb_count_opts;

/* Fills opts with the defaults (persistent degree schedule). */
void arb_count_default_opts(arb_count_opts *opts);

/* Bytes of workspace arb_count / arb_count_async need (n vertices, m arcs). */
size_t arb_count_workspace(int64_t n, int64_t m, int k);

/*
 * Exact k-clique count of the undirected graph whose orientation is dg (Alg. 1,
 * arb-count), and optionally per-vertex counts (the -v variant, Sec. 3.2):
 * per_vertex[x] = number of k-cliques that contain vertex x (rank space).
 * Every k-clique is found once, from its lowest-ranked vertex: for each root v the
 * candidate set N+(v) is relabelled 0..d-1 and its induced subgraph is kept as bit
 * rows in LDS (Sec. 3.4); the recursion intersects those rows.
 *
 *   dg          directed graph; arcs must ascend (arb_check_oriented)
 *   k           1 <= k <= ARB_MAX_K (k = 1 gives n, k = 2 gives m)
 *   total_dev   device uint64[1], overwritten with the total
 *   per_vertex  device uint64[n], nullable; overwritten
 *   per_root    device uint64[n], nullable; overwritten with the number of k-cliques
 *               whose lowest-ranked vertex is v (the root's share of the total)
 *   work_out    device uint64[n], nullable; overwritten with the per-root work measure
 *               w(v) = sum_{u in N+(v)} d+(u) + ceil(d+(v)/32) * sum_{j=1}^{k-2} c_j(v)
 *               where c_j(v) is the number of j-cliques in G[N+(v)]  (roots with
 *               d+(v) < k-1 and k <= 2 get 0); forces the unsplit schedule
 *   opts        nullable (defaults)
 * Does not synchronise and is capture-safe, except ARB_SCHED_PLAIN, which synchronises
 * once to size its grids.  Errors: ARB_EINVAL, ARB_EWORKSPACE.  A work item whose
 * candidate set exceeds ARB_MAX_LOCAL cannot be reported here: the call then leaves
 * total_dev = UINT64_MAX (arb_count turns that into ARB_ELIMIT).
 */
int arb_count_async(const arb_ocsr *dg, int k, uint64_t *total_dev, uint64_t *per_vertex,
                    uint64_t *per_root, uint64_t *work_out, const arb_count_opts *opts,
                    void *ws, size_t ws_bytes, void *stream);

/* The per-root work measure of the learned schedule (its training label): work_out[v]
 * (device uint64[n], overwritten) = w(v) as for arb_count_async's work_out; cycles_out
 * (device uint64[n], nullable, overwritten) = shader clock cycles (s_memtime) the team
 * spent on root v's items, a timing and not reproducible.  Runs the unsplit schedule
 * given by opts (nullable: defaults).  Workspace: arb_count_workspace(n, m, k).
 * Asynchronous; errors as arb_count_async. */
int arb_count_instrumented(const arb_ocsr *dg, int k, uint64_t *work_out, uint64_t *cycles_out,
                           const arb_count_opts *opts, void *ws, size_t ws_bytes, void *stream);

/* out[g] = sum of in[offsets[g] .. offsets[g+1]) for g < G (device arrays; offsets has
 * G+1 entries).  With per_root counts mapped to original ids (arb_permute_u64) and a
 * disjoint union of G graphs, this yields the per-graph totals of a batch. */
int arb_segment_sum_u64(const uint64_t *in, const int64_t *offsets, int64_t G, uint64_t *out,
                        void *stream);

/* Workspace of arb_count_batch_async. */
size_t arb_count_batch_workspace(int64_t n, int64_t m, int k, int64_t G);

/* Per-graph k-clique totals of a batch oriented by arb_orient_batch (its rank ranges are
 * the graphs' vertex ranges): totals_dev[i] (device uint64[G]) = k-cliques of graph i,
 * total_dev (device, nullable) = their sum, per_vertex (nullable, rank space) as in
 * arb_count_async.  graph_vtx_offsets: device int64[G+1] as given to arb_orient_batch.
 * Asynchronous and capture-safe in the persistent schedules; errors as arb_count_async. */
int arb_count_batch_async(const arb_ocsr *dg, const int64_t *graph_vtx_offsets, int64_t G, int k,
                          uint64_t *per_vertex, uint64_t *totals_dev, uint64_t *total_dev,
                          const arb_count_opts *opts, void *ws, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): arb_count_async without a caller
 * workspace.  Its scratch is a file-scope device array of ARB_NOALLOC_SCRATCH_BYTES that
 * each GPU the library runs on holds until the process ends; the call makes no
 * allocation of its own.  Graphs whose arb_count_workspace(n, m, k) exceeds that size are
 * rejected with ARB_ELIMIT before any work is enqueued.  The tier kernels run on `stream`
 * only (concurrent_tiers is ignored) and launch timing is not recorded.  Every call on a
 * GPU shares that GPU's array and clears what must start at zero, so calls that overlap
 * on one GPU (different streams or host threads) race: serialise them.  Arguments,
 * outputs and other errors as arb_count_async with per_root = work_out = NULL.
 */
#define ARB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int arb_count_noalloc(const arb_ocsr *dg, int k, uint64_t *total_dev, uint64_t *per_vertex,
                      const arb_count_opts *opts, void *stream);

/* Synchronous arb_count_async that also checks dg first; returns the total, or 0 with
 * arb_last_error() != ARB_OK on failure.  Synchronises the stream. */
uint64_t arb_count(const arb_ocsr *dg, int k, uint64_t *per_vertex,
                   const arb_count_opts *opts, void *ws, size_t ws_bytes, void *stream);

/* Launch timing of the counting kernels.  While enabled, each tier-kernel launch of
 * arb_count / arb_count_async / arb_autotune is bracketed by two HIP events on the
 * stream it runs on (tier t holds items whose candidate set fits 64, 128, 256, 384,
 * 512, 768 local vertices; tier ARB_NUM_TIERS is the global-scratch kernel's launch for
 * the larger roots, tier ARB_NUM_TIERS + 1 its launch for the pair items the tier
 * kernels overflowed, when it runs apart).  arb_profile_enable(1) clears the totals.  arb_profile_read
 * waits for pending events and fills, for each (tier, k, per-vertex, instrumented)
 * seen, the number of launches and their summed duration in ms (host arrays of
 * max_entries); it returns the number of entries (which may exceed max_entries), or
 * -1 on error.  Not thread-safe; synchronises. */
#define ARB_NUM_TIERS 6
int arb_profile_enable(int on);
int arb_profile_read(int max_entries, int32_t *tier, int32_t *k, int32_t *per_vertex,
                     int32_t *instrumented, int64_t *launches, double *total_ms);

/*
 * Autotuner: coordinate descent (two passes) over the split threshold
 * (split_min_degree, or split_min_cost for ARB_SCHED_LEARNED), persist_blocks_per_cu,
 * chunk_small, bitmap_max_span (id-range bitmap vs hash membership), concurrent_tiers,
 * tier_fill (LDS tile and waves per item) and big_max_degree (whole big roots in global
 * scratch vs per-out-neighbour items) for this graph and k.  Each candidate runs once to
 * warm up and then `trials` times; its time is the fastest run (HIP events on the
 * stream).  Every candidate's total must equal the first one's, else ARB_EMISMATCH.
 * opts: in, the schedule (and weights/features when learned) and starting values;
 * out, the fastest configuration found.  best_ms (host, nullable): its time.
 * Synchronises; workspace as arb_count.
 */
int arb_autotune(const arb_ocsr *dg, int k, arb_count_opts *opts, int trials, float *best_ms,
                 void *ws, size_t ws_bytes, void *stream);

/* The autotuner's search space: the candidate values of dimension `dim` (ARB_TUNE_*)
 * are written to values (host, up to max_values entries, as doubles); returns how many
 * candidates the dimension has, or -1 for an unknown dim. */
enum { ARB_TUNE_SPLIT_MIN_DEGREE = 0, ARB_TUNE_SPLIT_MIN_COST = 1, ARB_TUNE_BLOCKS_PER_CU = 2,
       ARB_TUNE_CHUNK_SMALL = 3, ARB_TUNE_BITMAP_MAX_SPAN = 4, ARB_TUNE_CONCURRENT_TIERS = 5,
       ARB_TUNE_TIER_FILL = 6, ARB_TUNE_BIG_MAX_DEGREE = 7 };
int arb_autotune_space(int dim, int max_values, double *values);

/* ---------------------------------------------------------------- learned schedule */

#define ARB_MLP_PARAMS 8641     /* 3->64->64->64->1, ReLU, weights then bias per layer */

/* Workspace of arb_sparsify. */
size_t arb_sparsify_workspace(int64_t n, int64_t nnz);

/* Colorful sparsification (Sec. 3.3; estimator and its variance in the appendix's
 * sampling theorem): keeps the edges {u, v} of g with colors[u] == colors[v] (colors:
 * device int32[n], drawn by the caller, e.g. uniformly from c colours).  out_offsets
 * (device, n+1) and out_indices (device, capacity g->nnz) receive the sparsified CSR,
 * rows still sorted; *out_nnz (host) its entry count.  Synchronises the stream. */
int arb_sparsify(const arb_csr *g, const int32_t *colors, int64_t *out_offsets, int32_t *out_indices,
                 int64_t *out_nnz, void *ws, size_t ws_bytes, void *stream);

/* count * colors^(k-1): the unbiased estimate of the k-clique count of the original
 * graph from the count of the graph sparsified with that many colours. */
double arb_colorful_estimate(uint64_t count, int colors, int k);

/* Workspace of arb_approx_peel. */
size_t arb_approx_peel_workspace(int64_t n, int64_t m, int k);

/* arb-approx-peel (Sec. 4.2): a 1/(k(1+eps))-approximation of the k-clique densest
 * subgraph of the graph oriented as dg (rank space).  Rounds on the present set S (all
 * vertices at first): count per-vertex k-cliques of G[S] (dg restricted to S), density
 * d(S) = cliques(S) / |S|, then remove every present vertex whose count c satisfies
 * (double)c <= ((double)k * (1 + eps) * (double)cliques(S)) / (double)|S|.
 * *best_density = the largest d(S) met, *rounds (nullable) the rounds, best_mask
 * (nullable, device int32[n], rank space) 1 on the S that gave it.  eps in (0, 64],
 * 1 <= k <= ARB_MAX_K; opts as arb_count_async.  Synchronises every round. */
int arb_approx_peel(const arb_ocsr *dg, int k, double eps, const arb_count_opts *opts, double *best_density,
                    int64_t *rounds, int32_t *best_mask, void *ws, size_t ws_bytes, void *stream);

/* Workspace of arb_peel. */
size_t arb_peel_workspace(int64_t n, int64_t m, int k);

/* arb-peel (Alg. 2, Sec. 4.1): k-clique vertex peeling of the graph oriented as dg, a
 * 1/k-approximation of the k-clique densest subgraph.  From the per-vertex k-clique
 * counts, round r removes every present vertex whose count is the least present count
 * (round_out[v] = r, device int32[n], rank space) and lowers the others' counts by the
 * k-cliques removed with them (counted around each removed vertex on its present
 * neighbourhood).  *best_density = max over the vertex sets met (the whole graph first,
 * then after every round while vertices remain) of cliques(S) / |S| (double);
 * *rounds (nullable) = rounds.  3 <= k <= ARB_MAX_K.  Synchronises every round. */
int arb_peel(const arb_ocsr *dg, int k, double *best_density, int64_t *rounds, int32_t *round_out, void *ws,
             size_t ws_bytes, void *stream);

/* Per-root features in rank space: feat[3v..3v+2] = (log2(1+d+(v)),
 * log2(1 + sum_{u in N+(v)} d+(u)), round(v)); round_orig/rank as from arb_orient. */
int arb_features(const arb_ocsr *dg, const int32_t *round_orig, const int32_t *rank,
                 float *feat, void *stream);

/* The rows of arb_features for the roots with at least min_degree out-neighbours only;
 * the other rows of feat are left as they were (min_degree = 0: every row, the same as
 * arb_features).  The learned schedule reads the cost of roots with at least
 * ARB_LEARNED_MIN_DEGREE out-neighbours only (the smaller roots share the 64-tier, where
 * the order of the light roots does not matter), so features computed with that bound
 * give it all it reads.  ARB_EINVAL on a negative min_degree or the arb_features errors. */
#define ARB_LEARNED_MIN_DEGREE 65
int arb_features_min_degree(const arb_ocsr *dg, const int32_t *round_orig, const int32_t *rank,
                            int64_t min_degree, float *feat, void *stream);

/* y[r] = MLP(x[r]) for rows r < rows; x float[rows][3]; weights bf16 (ARB_MLP_PARAMS,
 * layout W1[64][3] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[1][64] b4[1]);
 * act (nullable) float[rows][192] receives the three hidden pre-activations for
 * arb_mlp_backward. FP32 accumulation.  With act == NULL (inference, as the learned
 * schedule runs it) the hidden layers run on the matrix cores with each activation split
 * into two bf16 terms; y then agrees with the act != NULL path to about 1e-5 relative. */
int arb_mlp_forward(const uint16_t *w_bf16, const float *x, int64_t rows, float *y,
                    float *act, void *stream);

/* Workspace of arb_mlp_backward for `rows` rows. */
size_t arb_mlp_workspace(int64_t rows);

/* Gradient of sum_r dy[r] * y[r] with respect to the parameters (overwrites grad,
 * float[ARB_MLP_PARAMS]); act from arb_mlp_forward on the same x and weights.  The
 * per-row deltas and per-256-row partial sums go to ws; partials are summed in a fixed
 * order, so the result is deterministic. */
int arb_mlp_backward(const uint16_t *w_bf16, const float *x, const float *act,
                     const float *dy, int64_t rows, float *grad, void *ws, size_t ws_bytes,
                     void *stream);

/* Mean squared error: dy[r] = (y[r] - target[r]) / rows and, if loss != NULL,
 * *loss = sum_r (y[r] - target[r])^2 / (2 rows) (device float). */
int arb_mse_grad(const float *y, const float *target, int64_t rows, float *dy, float *loss,
                 void *stream);

/* fp32 -> bf16, round to nearest even. */
int arb_to_bf16(const float *w, uint16_t *w_bf16, int64_t count, void *stream);

/* One Adam step (Kingma & Ba 2015, bias-corrected, beta1 0.9, beta2 0.999, eps 1e-8)
 * on fp32 master weights w, moments m and v; writes the bf16 copy (round to nearest
 * even).  step counts from 1. */
int arb_adam_step(float *w, uint16_t *w_bf16, const float *grad, float *m, float *v,
                  float lr, int step, void *stream);

/* ---------------------------------------------------------------- errors */

int arb_last_error(void);
const char *arb_error_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* ARB_H */
