/*
 * dm.h — C ABI of libdumato_mi: exact k-clique and induced k-motif counting by
 * DFS-wide subgraph enumeration on one AMD Instinct MI355X (gfx950).
 *
 * Method: DuMato (Ferraz, Dias, Teixeira, Teodoro, Meira Jr., arXiv 2212.04551).
 *   - Enumeration function E(G, tr, k) with property P and output A:
 *     Section II, Eq. (1).
 *   - Filter-process workflow (Control, Extend, Filter, Compact, Aggregate,
 *     Move): Section IV-A; DFS-wide exploration: Section IV-B, Alg. 1 (Move);
 *     Extend: Section IV-C, Alg. 2; Filter: Alg. 3; Compact and Aggregate:
 *     Section IV-C.
 *   - Clique and motif counting: Section IV-E, Alg. 4.
 *   - Warp-level load balancing: Section IV-D (realised here inside the kernel,
 *     the asynchronous form named as future work in Section VI).
 *
 * Conventions for every entry point:
 *   - Graphs are simple and undirected (Section II): CSR with int64 row
 *     offsets `row_ptr[n+1]` and int32 column ids `col[nnz]`, every adjacency
 *     list sorted strictly ascending, no self-loops, both directions present.
 *     Row offsets are 64-bit so that nnz may exceed 2^31 - 1 (graphs of more
 *     than about 1.07e9 edges); vertex ids stay 32-bit.
 *   - Counts are exact uint64.  Any uint64 wrap, in a per-wave accumulator or
 *     in a global sum, returns DM_E_OVERFLOW; outputs are then unspecified.
 *   - Output arrays are caller-owned HOST memory unless stated otherwise.
 *     Calls return after the results are in host memory.
 *   - GPU work is enqueued on `opt->stream` (a hipStream_t, e.g.
 *     torch.cuda.current_stream().cuda_stream); NULL means the library's
 *     own stream.  The call synchronises that stream before returning.
 *   - On DM_E_ARG, DM_E_CSR, DM_E_K or DM_E_BUFSZ no output is written.
 *   - A graph handle serves one call at a time; distinct handles may be used
 *     from different threads.
 *   - Nothing here throws; failures are reported by status code, and
 *     dm_strerror / dm_last_error give text.
 */
#ifndef DM_H
#define DM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dm_graph dm_graph; /* opaque, owned by the library, freed by dm_free */

typedef enum {
    DM_OK = 0,
    DM_E_ARG = 1,      /* null pointer, negative size, bad flag or option */
    DM_E_CSR = 2,      /* CSR rejected: unsorted/duplicate, self-loop, asymmetric, out of range */
    DM_E_K = 3,        /* k outside the supported range for the operation */
    DM_E_OVERFLOW = 4, /* a uint64 count wrapped */
    DM_E_NOMEM = 5,    /* device or host allocation failed, or workspace cap exceeded */
    DM_E_HIP = 6,      /* a HIP runtime call failed (text in dm_last_error) */
    DM_E_BUFSZ = 7,    /* output buffer shorter than required */
    DM_E_MODEL = 8     /* learned scheduling requested without valid parameters */
} dm_status;

/* dm_load_csr flags */
enum {
    DM_CSR_HOST = 0,    /* row_ptr / col are host pointers */
    DM_CSR_DEVICE = 1,  /* row_ptr / col are device pointers (copied device-to-device) */
    DM_CSR_TRUSTED = 2, /* skip validation (caller guarantees the conventions above) */
    DM_CSR_ORIENT = 4,  /* also build the (degree, id) orientation used by clique counting
                           now, instead of at the first clique call */
    DM_CSR_RANK = 8     /* also build the orientation and the rank-renamed graph used by
                           motif counting now (dm_count_motifs_static needs it) */
};

/* dm_options.sched bits */
enum {
    DM_SCHED_PLAIN = 0,    /* roots in (degree, id) rank order */
    DM_SCHED_LEARNED = 1,  /* order and chunk roots by the MLP's predicted subtree size */
    DM_SCHED_AUTOTUNE = 2, /* pick chunk / rebalance / waves-per-CU from the tuner cache */
    DM_RECORD_ROOTS = 4,   /* write per-root {tree nodes, leaves, adjacency reads} */
    DM_NO_DONATION = 8,    /* disable in-kernel work donation (ablation: static schedule) */
    DM_SCHED_COST = 16,    /* order and chunk roots like DM_SCHED_LEARNED, by the caller's
                              per-vertex costs `root_cost` instead of the MLP's predictions
                              (e.g. recorded tree sizes: the ordering a perfect predictor gives) */
    DM_IMPL_DFS = 32,      /* ablation (Section V-A, the DFS implementation of Table III): one
                              lane per traversal instead of one wave, each lane taking roots from
                              a global counter; same counts.  Plain root order over every root
                              only (with DM_NO_DONATION or nothing else), clique k <= 16, motif k <= 7. */
    DM_SCHED_HOST_BALANCE = 64 /* the paper's own load balancing (Section IV-D): no in-kernel
                              donation; once the queue is drained and fewer than a fraction
                              `rebalance` of the waves are still busy (default 0.4 for cliques,
                              0.1 for motifs, the paper's Section V-A thresholds) the launch
                              stops, busy waves write their untried extensions as tasks, and the
                              host splits those tasks and relaunches with them as the queue, until
                              no work is left (at most 64 stopped launches; the last runs to the
                              end).  Same counts.  Single-graph calls only; excludes
                              DM_NO_DONATION. */
};

enum { DM_OP_CLIQUE = 0, DM_OP_MOTIF = 1 };

/*
 * Options.  opt == NULL means all defaults (plain schedule).  `size` must be
 * sizeof(dm_options) so the struct can grow.  Besides the schedule, stream,
 * chunk, rebalance threshold, model and per-root records, it carries the knobs
 * the measurements need: resident waves per CU, explicit root lists (sampled
 * parity), per-wave idle / busy statistics, an accumulator bias (overflow
 * tests), the bound on idle waits, and caller-given root costs.
 */
typedef struct {
    uint32_t size;
    uint32_t sched;          /* DM_SCHED_* | DM_RECORD_ROOTS | DM_NO_DONATION */
    void* stream;            /* hipStream_t or NULL */
    uint32_t chunk;          /* plain queue: roots per grab (0 = 1; the queue's blocks of
                                `chunk` roots are dealt round-robin to 8 counters, so the roots
                                of one launch leave in about, not exactly, rank order);
                                learned queue: chunks of equal predicted cost per wave (0 = 8) */
    float rebalance;         /* donate once at least this fraction of waves is idle; 0 = default */
    uint32_t waves_per_cu;   /* resident waves per CU for the persistent grid; 0 = occupancy maximum */
    const float* mlp;        /* DM_SCHED_LEARNED: device pointer to DM_MLP_NPARAMS floats */
    const int32_t* roots;    /* host pointer: explicit root order/subset (original vertex ids),
                                NULL = every vertex */
    int64_t num_roots;       /* length of `roots` */
    uint64_t* root_stats;    /* DM_RECORD_ROOTS: device pointer, 3 uint64 per root, indexed by
                                vertex id (or by position in `roots` when given):
                                {tree nodes, leaves, adjacency entries read} */
    uint64_t* wave_stats;    /* optional device pointer, 4 uint64 per wave:
                                {busy ticks, idle ticks, tree nodes, tasks taken} */
    uint32_t wave_stats_len; /* number of waves wave_stats can hold */
    uint64_t counter_bias;   /* test hook: global accumulators start at this value (0 normally) */
    uint32_t wait_limit_us;  /* longest time (microseconds) an idle wave of the persistent grid
                                waits for donated work before it gives up (0 = 600 s).  A wave that gives up
                                makes the call fail with DM_E_HIP (every wave still exits
                                normally), so a scheduler fault cannot keep the GPU busy. */
    const float* root_cost;  /* DM_SCHED_COST: device pointer, n floats indexed by vertex id,
                                log(1 + expected tree nodes) of each root (the MLP's scale) */
} dm_options;

/*
 * Load a graph.  Arrays are borrowed for the call only and copied to the
 * device; validated on the GPU unless DM_CSR_TRUSTED.  `stream` may be NULL.
 * Errors: DM_E_ARG (n < 0, null pointers), DM_E_CSR (validation), DM_E_NOMEM,
 * DM_E_HIP.  On error *out is NULL.
 */
dm_status dm_load_csr(int32_t n, const int64_t* row_ptr, const int32_t* col, uint32_t flags,
                      void* stream, dm_graph** out);

/* Free a handle (NULL is a no-op). */
void dm_free(dm_graph* g);

/* Vertex and adjacency-entry counts of a loaded graph. */
dm_status dm_graph_info(const dm_graph* g, int32_t* n, int64_t* nnz);

/*
 * Number of k-cliques (Section IV-E, clique counting; Alg. 4 left).  The graph
 * is oriented once by (degree, id) rank and cached on the handle; each clique
 * is found from its lowest-rank vertex.  k in 1..32 (k=1 gives n, k=2 gives m).
 * A wave keeps a root's out-list and its k+1 candidate bitsets in LDS, so the
 * oriented graph's largest out-degree D must satisfy
 * (8 + (k+1)/8) D + 5.4 KB <= 160 KB (D up to about 17,000 at k = 8 and
 * 13,000 at k = 32; always met when m <= 8.5e7, since D <= sqrt(2m)), else
 * DM_E_NOMEM.
 * Errors: DM_E_ARG, DM_E_K, DM_E_OVERFLOW, DM_E_NOMEM, DM_E_HIP, DM_E_MODEL.
 */
dm_status dm_count_cliques(dm_graph* g, int k, uint64_t* out_count, const dm_options* opt);

/* Number of connected k-vertex classes: 2, 6, 21, 112, 853, 11117 for k = 3..8; -1 otherwise.
 * (The first call for a k builds that k's dictionary on the host: for k = 8,
 * 2^27 entries from an orbit labelling of all 2^28 labelled graphs, using all
 * host threads and about 1.3 GiB of host memory for a few seconds.) */
int dm_motif_num_classes(int k);

/*
 * Canonical adjacency of class `cls`: bit i(i-1)/2 + t set iff vertices t < i
 * are adjacent, the minimum such bitmap over all relabellings.  Classes are
 * numbered by (edge count, canonical bitmap) ascending.
 * Errors: DM_E_K, DM_E_ARG (cls out of range or null pointer).
 */
dm_status dm_motif_class_mask(int k, int cls, uint32_t* upper_tri_mask);

/*
 * The canonical-relabeling dictionary of Section IV-C (Aggregate): entry c, for
 * a traversal code c of 2^(k(k-1)/2 - 1) values (edge v0-v1 implied; vertex
 * v_i, i >= 2, stores its edges to v_0..v_{i-1} in bits i(i-1)/2 - 1 + t),
 * is the class id, or 0xFF when some v_i has no edge to its predecessors.
 * `len` must be at least 2^(k(k-1)/2 - 1).  k in 3..6 (class ids fit a byte).
 * Host-only; needs no GPU.  Errors: DM_E_K, DM_E_ARG, DM_E_BUFSZ.
 */
dm_status dm_motif_class_table(int k, uint8_t* out, size_t len);

/*
 * The same dictionary with 16-bit class ids, for k in 3..8 (k = 7: 2^20
 * entries, 853 classes; k = 8: 2^27 entries, 11,117 classes); unreachable
 * codes hold 0xFFFF.  This is the table the motif kernels read (Section IV-C
 * gives its size for a pattern of k vertices as 2^(k(k-1)/2 - 1) codes).
 * Host-only; needs no GPU.  Errors: DM_E_K, DM_E_ARG, DM_E_BUFSZ.
 */
dm_status dm_motif_class_table16(int k, uint16_t* out, size_t len);

/*
 * Per-class counts of connected induced k-vertex subgraphs (Section IV-E,
 * motif counting; Alg. 4 right).  out_counts[cls] for cls < ncls(k); k in 3..8
 * (k = 8 keeps each wave's 11,117 class counters in global memory instead of
 * LDS, and its dictionary takes 256 MiB of device memory).
 * Each subgraph is enumerated once, from its lowest (degree, id) vertex (the
 * same root rule as cliques; per-root records and root lists use it).
 * Errors: DM_E_ARG, DM_E_K, DM_E_BUFSZ (out_len < ncls), DM_E_OVERFLOW,
 * DM_E_NOMEM, DM_E_HIP, DM_E_MODEL.
 */
dm_status dm_count_motifs(dm_graph* g, int k, uint64_t* out_counts, size_t out_len,
                          const dm_options* opt);

/*
 * dm_count_motifs (k in 3..7) without device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same counts and errors as
 * dm_count_motifs; the graph must carry its rank-renamed copy
 * (dm_load_csr with DM_CSR_RANK, or an earlier dm_count_motifs call).
 * Every device buffer of the launch (dictionary, scheduler words, class
 * counters, per-wave extension stacks) lives in one library-owned static
 * device array of 64 MiB per GPU, held until the process ends; the persistent
 * grid shrinks to the waves whose stacks fit in it, and a graph whose single
 * wave needs more (about 5 (k-1)(k-2)/2 + 4 bytes per unit of maximum degree,
 * i.e. a maximum degree above about 1.1 million at k = 5) is rejected with
 * DM_E_NOMEM.  Plain root queue over every root only: DM_SCHED_LEARNED,
 * DM_SCHED_COST, DM_IMPL_DFS and root lists give DM_E_ARG; root_stats,
 * wave_stats, chunk, rebalance, waves_per_cu, DM_NO_DONATION and
 * DM_SCHED_AUTOTUNE knobs work as in dm_count_motifs.  NULL stream = the
 * handle's own stream.  Calls share the device's array: the library
 * serialises its own calls, but calls that overlap on one GPU from other
 * processes or loaded copies of the library race.
 */
dm_status dm_count_motifs_static(dm_graph* g, int k, uint64_t* out_counts, size_t out_len,
                                 const dm_options* opt);

/*
 * Property filters (Section II: E(G, tr, k, P) keeps the subgraphs with
 * property P; cliques and connected induced patterns are two such P).
 *
 * dm_induced_subgraph: a vertex property.  Makes a new handle holding the
 * subgraph induced by the vertices with keep[v] != 0 (keep: host array of n
 * bytes, e.g. "carries an allowed label"), vertices renumbered in id order
 * (v becomes the number of kept vertices below it).  Every count or listing
 * on it is the count or listing, on g, of the subgraphs all of whose
 * vertices are kept.  The new handle is independent of g (free both).
 * Errors: DM_E_ARG, DM_E_NOMEM, DM_E_HIP.
 */
dm_status dm_induced_subgraph(dm_graph* g, const uint8_t* keep, void* stream, dm_graph** out);

/*
 * dm_count_quasi_cliques: a pattern property.  The number of connected
 * induced k-subgraphs with at least min_edges edges (k in 3..8, min_edges in
 * 0..k(k-1)/2): the density-gamma quasi-cliques for min_edges =
 * ceil(gamma k(k-1)/2); min_edges = k(k-1)/2 gives the k-cliques, min_edges
 * <= k-1 every connected k-subgraph.  Computed by the motif kernel, summing the
 * classes whose pattern has enough edges; options as dm_count_motifs.
 * Errors: as dm_count_motifs, and DM_E_ARG for min_edges out of range.
 */
dm_status dm_count_quasi_cliques(dm_graph* g, int k, int min_edges, uint64_t* out_count, const dm_options* opt);

/*
 * Directed graphs (Section II: the method is stated for undirected graphs and
 * carries over to directed ones; Section IV-C: a subgraph's pattern is the
 * bitmap of its pairs, here two bits per pair).
 *
 * dm_load_digraph: like dm_load_csr, but row_ptr / col are the arcs as sorted
 * out-lists (arc v -> col[i] for i in [row_ptr[v], row_ptr[v+1])): strictly
 * ascending per vertex, no self-arc; an opposite pair u -> w, w -> u is two
 * arcs.  row_ptr[n] is the number of arcs (any value >= 0).  Flags as
 * dm_load_csr (DM_CSR_DEVICE: device pointers; DM_CSR_TRUSTED skips the
 * checks; DM_CSR_ORIENT / DM_CSR_RANK prepare the underlying graph).  The
 * handle holds the underlying undirected graph (edge {u, w} for every arc),
 * which every other call sees: cliques, undirected motifs, listings and
 * filters count subgraphs of the underlying graph.  It also holds two arc bits
 * per adjacency entry for dm_count_motifs_directed.  The caller's arrays are
 * copied.  Errors: DM_E_ARG (null pointers, n < 0, unknown flag), DM_E_CSR
 * (conventions violated), DM_E_NOMEM / DM_E_HIP.
 */
dm_status dm_load_digraph(int32_t n, const int64_t* row_ptr, const int32_t* col, uint32_t flags, void* stream,
                          dm_graph** out);

/* *is_directed = 1 for a dm_load_digraph handle (and *arcs its arc count), else 0 (arcs 0). */
dm_status dm_digraph_info(const dm_graph* g, int32_t* is_directed, int64_t* arcs);

/*
 * Directed classes on k vertices (k in 1..5).  A k-vertex digraph in a vertex
 * order has the code with, for each pair t < i (p = i(i-1)/2 + t), bit 2p set
 * for the arc t -> i and bit 2p+1 for the arc i -> t.  Its class is the
 * smallest code over all k! vertex orders; the classes of the weakly connected
 * digraphs are numbered 0, 1, ... by increasing smallest code (13, 199 and
 * 9,364 classes at k = 3, 4, 5).
 *   dm_motif_directed_num_classes: the number of classes, or -1 for k outside 1..5.
 *   dm_motif_directed_class_code: the smallest code of class cls.
 *   dm_motif_directed_class_table: the class of every code, out[code] for all
 *     2^(k(k-1)) codes (0xFFFF: not weakly connected); len >= 2^(k(k-1)).
 * Host-only; no GPU needed.  Errors: DM_E_K, DM_E_ARG, DM_E_BUFSZ.
 */
int32_t dm_motif_directed_num_classes(int k);
dm_status dm_motif_directed_class_code(int k, int32_t cls, uint32_t* code);
dm_status dm_motif_directed_class_table(int k, uint16_t* out, size_t len);

/*
 * dm_count_motifs_directed: for k in 3..5, out_counts[c] (host, out_len >=
 * dm_motif_directed_num_classes(k)) = the number of vertex sets S, |S| = k,
 * whose induced subdigraph is weakly connected and in class c.  Enumeration
 * over the underlying undirected graph renamed by (degree, id) rank (every
 * connected k-subset once, from its lowest-rank vertex, by Section IV-E's
 * canonical-candidate rule; the renaming is built at the first call and kept
 * on the handle), one wave per root, no donation; classification by the
 * dictionary above.  Options: stream, chunk, waves_per_cu (a cap on the
 * resident waves per CU the launch is planned for), wait_limit_us and
 * DM_NO_DONATION (no effect); anything else gives DM_E_ARG.  Errors: DM_E_ARG
 * (null pointers, a handle not made by dm_load_digraph, a degree of 2^26 or
 * more), DM_E_K, DM_E_BUFSZ, DM_E_OVERFLOW, DM_E_NOMEM / DM_E_HIP.
 */
dm_status dm_count_motifs_directed(dm_graph* g, int k, uint64_t* out_counts, size_t out_len,
                                   const dm_options* opt);

/*
 * Subgraph matching (Section IV-E: Filter admits subgraph-matching
 * properties; Section IV-C: patterns as pair bitmaps).  *out_count = the
 * number of copies of the connected pattern P in g:
 *   DM_PATTERN_INDUCED: vertex sets S, |S| = k, whose induced subgraph is
 *     isomorphic to P (the count of P's class);
 *   otherwise: subgraphs of g (vertex set and edge subset) isomorphic to P,
 *     i.e. monomorphisms of P into g divided by |Aut(P)|, computed as
 *     sum over classes H of count(H) x (copies of P spanning H).
 * pattern: P's code on k vertices in any vertex order: one bit per pair
 * (bit i(i-1)/2 + t = edge t-i, k in 3..8), or with DM_PATTERN_DIRECTED two
 * bits per pair as in the directed dictionary (k in 3..5; g from
 * dm_load_digraph).  Runs dm_count_motifs / dm_count_motifs_directed with opt.
 * Errors: DM_E_ARG (null pointers, unknown flag, bits beyond k vertices, a
 * pattern that is not (weakly) connected), DM_E_K, DM_E_OVERFLOW, and those of
 * the counting call.
 */
enum { DM_PATTERN_INDUCED = 1, DM_PATTERN_DIRECTED = 2 };
dm_status dm_count_pattern(dm_graph* g, int k, uint32_t pattern, uint32_t flags, uint64_t* out_count,
                           const dm_options* opt);

/*
 * Count many graphs in one persistent launch.  op is DM_OP_CLIQUE (one count
 * per graph) or DM_OP_MOTIF (ncls(k) counts per graph).  out_counts is
 * row-major [num_graphs][per-graph width].  The graphs are concatenated as a
 * disjoint union (no traversal crosses graphs), so each row equals the count
 * of the corresponding single-graph call.  The union, its orientation and the
 * launch (clears, persistent kernel, copy-back) are built on the first call
 * for a given list of handles and options, captured into a hipGraph, and
 * replayed by later calls (batch calls are serialised by a library lock; the
 * cached union of a list of handles lives until the process ends).
 * Errors: as the single-graph calls, plus DM_E_BUFSZ.
 */
dm_status dm_batch(dm_graph* const* gs, int32_t num_graphs, int op, int k, uint64_t* out_counts,
                   size_t out_len, const dm_options* opt);

/*
 * Receives one batch of listed subgraphs: `rows` holds `nrows` rows of
 * `width` int32 in host memory, valid only during the call.
 */
typedef void (*dm_sink_fn)(const int32_t* rows, uint64_t nrows, int width, void* user);

/*
 * aggregate_store (Section IV-C, Aggregate; Table II): list the subgraphs
 * themselves instead of counting them.  op = DM_OP_CLIQUE: every k-clique
 * (k in 1..32), a row of k original vertex ids in (degree, id) rank order.
 * op = DM_OP_MOTIF: every connected induced k-subgraph (k in 3..8), a row of
 * its k original vertex ids in canonical traversal order (Section IV-E: the
 * lowest-(degree, id) vertex first, then each time the lowest vertex adjacent
 * to those before it) followed by its class id (dm_motif_class_mask's
 * numbering; row width k + 1).  Each subgraph appears exactly once; the order
 * of rows is unspecified.  The kernel writes rows into a ring of pinned host
 * memory (8 blocks of 65,536 rows) and `sink` is called on the calling thread
 * with consecutive rows of one block while the kernel runs; a block is reused
 * only after the sink has returned for all its rows, so a slow sink stalls
 * the kernel (an idle wait longer than opt->wait_limit_us fails the call with
 * DM_E_HIP).  *out_total = rows delivered.  Options: stream, waves-per-CU and
 * wait limit; plain root queue over every root only (other sched bits, root
 * lists and records give DM_E_ARG).
 * Errors: DM_E_ARG, DM_E_K, DM_E_NOMEM, DM_E_HIP.
 */
dm_status dm_list(dm_graph* g, int op, int k, dm_sink_fn sink, void* user, uint64_t* out_total,
                  const dm_options* opt);

/* ---------------------------------------------------------------------------
 * Learned root ordering (an addition to the paper's method; it only orders and
 * chunks the initial root queue and never changes a count).  The model is a
 * 4 -> 64 -> 64 -> 1 FP32 MLP with ReLU that maps the standardised log1p of
 * four per-vertex features (degree, 2-hop degree sum, core number, triangle
 * count) to log(1 + enumeration-tree nodes of the root).  Parameter blob
 * (device, DM_MLP_NPARAMS floats): W1[64][4], b1[64], W2[64][64], b2[64],
 * w3[64], b3, then feature mean[4] and std[4] of log1p(feature).
 * With DM_SCHED_LEARNED the queue is sorted by predicted size, longest
 * first, and cut into chunks of about equal predicted cost (exp of the
 * prediction per root).  The queue is cached on the graph handle and rebuilt
 * when a 64-bit fingerprint of the parameter blob (computed on the device at
 * every call), the grid or the chunk count changes.
 * All pointers below are device pointers unless stated; calls synchronise
 * `stream` before returning.
 * ------------------------------------------------------------------------- */
#define DM_MLP_NET 4545
#define DM_MLP_NPARAMS 4553

/* Per-vertex features as int64 [n][4]: degree, sum of neighbour degrees, core
 * number (k-core decomposition), number of triangles containing the vertex. */
dm_status dm_features(dm_graph* g, int64_t* out, void* stream);

/* He-uniform weights from `seed`, zero biases, identity normaliser. */
dm_status dm_mlp_init(float* params, uint64_t seed, void* stream);

/* Set the normaliser slots to the mean / std of log1p(feats) over n rows. */
dm_status dm_mlp_fit_normalizer(float* params, const int64_t* feats, int64_t n, void* stream);

/* out[r] = network(feats[r]) for r < n. */
dm_status dm_mlp_forward(const float* params, const int64_t* feats, int64_t n, float* out, void* stream);

/* out[r] = log1p(root_stats[r][0]) (tree nodes recorded by DM_RECORD_ROOTS). */
dm_status dm_mlp_targets(const uint64_t* root_stats, int64_t n, float* out, void* stream);

/* Mean squared error over the n rows and its gradient (DM_MLP_NET floats);
 * *loss is host memory. */
dm_status dm_mlp_loss_grad(const float* params, const int64_t* feats, const float* targets, int64_t n,
                           float* grad, float* loss, void* stream);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected, step t >= 1) on
 * the DM_MLP_NET network weights; m and v are caller-owned moment buffers. */
dm_status dm_mlp_adam_step(float* params, const float* grad, float* m, float* v, int64_t t, float lr,
                           void* stream);

/* Minibatch Adam training: every epoch shuffles the rows (seeded) and takes
 * one step per batch.  loss_history (host, `epochs` floats, nullable) gets the
 * mean batch loss of each epoch. */
dm_status dm_mlp_train(float* params, const int64_t* feats, const float* targets, int64_t n, int epochs,
                       int batch, float lr, uint64_t seed, float* loss_history, void* stream);

/* ---------------------------------------------------------------------------
 * Autotuning of the scheduling knobs (never changes a count).  The load
 * balancer's threshold was picked by a sensitivity analysis in the paper
 * (Section V-A2); here a coordinate search times one launch per candidate of
 * roots per queue grab (1..128), donation threshold (idle-wave fraction 0 ..
 * 0.4) and resident waves per CU, on the given graph (num_graphs == 1) or batch,
 * and remembers the best setting per (op, k).  Later calls with
 * DM_SCHED_AUTOTUNE use it for every knob they leave at 0.
 * ------------------------------------------------------------------------- */
typedef struct {
    uint32_t chunk;
    float rebalance;
    uint32_t waves_per_cu;  /* 0 = occupancy maximum */
    float ms;               /* best measured launch time */
} dm_tuning;

dm_status dm_autotune(dm_graph* const* gs, int32_t num_graphs, int op, int k, const dm_options* opt,
                      dm_tuning* out);

/* Static text for a status code. */
const char* dm_strerror(dm_status s);

/* Text of the last error raised on the calling thread ("" if none). */
const char* dm_last_error(void);

/* Kernel launches made by the calling thread's last dm_count_cliques /
 * dm_count_motifs call: 1, or more when DM_SCHED_HOST_BALANCE stopped and
 * relaunched it. */
int dm_last_launch_count(void);

#ifdef __cplusplus
}
#endif

#endif /* DM_H */
