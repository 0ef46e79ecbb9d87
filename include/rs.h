/*
 * librestless_sieve: GF(2^64) multilinear sieve for k-RestlessPath and
 * k-RestlessMotif queries on one MI355X (gfx950) GPU.
 *
 * Method: Thejaswi, Lauri, Gionis, "Restless reachability problems in
 * temporal graphs" (arXiv 2010.08423).
 *   - Restless walk / path: Sec. 2 (consecutive edges (u,v,j), (v,w,j') with
 *     0 <= j' - j <= delta(v); a path repeats no vertex).
 *   - k-RestlessPath (a restless path with k vertices) and k-RestlessMotif
 *     (k vertices whose colours equal the multiset M): Sec. 3. The queries
 *     here ask whether such a path exists anywhere in the graph.
 *   - Evaluation: the restless-walk generating function, Eq. (poly-enc:1),
 *     sieved over all subsets L of [k], Eq. (multilinear:1); motif queries use
 *     colour shades, Eq. (multilinear:3) and Eq. (multilinear:2); the sum over
 *     L is the loop of Alg. 1. All arithmetic is in GF(2^64) (Sec. 5.1, b = 64)
 *     with modulus x^64 + x^4 + x^3 + x + 1.
 *
 * Result: fingerprint F = XOR over L of f_L, where f_L sums the level-k
 * evaluation over every end vertex and end time. F equals, over the same field,
 *     XOR over restless paths P (motif: colour-agreeing) of
 *     (prod_{p=1}^{k-1} y_{e_p,p}) * det [z_{v_p,j}]_{p,j},
 * so F != 0 implies such a path exists (no false positives). If one exists,
 * F == 0 with probability at most (3k-1)/2^64 (Schwartz-Zippel).
 *
 * The random values are a deterministic function of the query seed:
 *   mix64 = SplitMix64 output finalizer; G = 0x9E3779B97F4A7C15;
 *   H(seed, tag, w_1..w_r): h = mix64(seed + tag*G); h = mix64(h ^ (w_i + G)).
 *   z_{u,j}   = H(seed, 'Z', u | j<<32)           j = 1..k   (path queries)
 *   gamma_{u,d} = H(seed, 'G', u | d<<32)         d = shade 0..k-1
 *   omega_{d,j} = H(seed, 'W', d | j<<32)
 *   motif: z_{u,j} = sum over shades d of colour c(u) of gamma_{u,d} * omega_{d,j};
 *          shades are numbered contiguously per colour, colours ascending.
 *   y_{e,p}   = H(seed, 'Y', src | dst<<32, t | p<<32)   p = 1..k-1
 *   iteration i in [0, 2^k) <-> L(i) = { j : bit j-1 of i is set }.
 *
 * Conventions for every call:
 *   - Returns RS_OK (0) or a negative rs_status. No C++ exception crosses
 *     this boundary. Errors leave outputs untouched unless stated.
 *   - "host" pointers are read during the call only and never retained;
 *     "device" pointers are device (HBM) addresses, e.g. a torch tensor's
 *     data_ptr(), read during the call only.
 *   - hip_stream is a hipStream_t (NULL = the null stream). Calls that return
 *     a result synchronise that stream before returning.
 *   - Graph objects are immutable after creation. Query calls on one graph
 *     are serialised internally (they share a cached device workspace).
 */
#ifndef RESTLESS_SIEVE_RS_H
#define RESTLESS_SIEVE_RS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rs_status;
#define RS_OK 0
#define RS_EINVAL (-1)     /* invalid argument (sizes, ids, k, motif) */
#define RS_ENOMEM (-2)     /* device or host allocation failed / over budget */
#define RS_EDEVICE (-3)    /* HIP runtime error or a kernel-side failure flag */
#define RS_EBUSY (-4)      /* server: not admitted yet / queue full */
#define RS_ECANCELED (-5)  /* server: query cancelled */
#define RS_ENOTFOUND (-6)  /* server: unknown ticket or graph id */
#define RS_ETIMEOUT (-7)   /* server: poll wait expired before completion */
#define RS_ERETRY (-8)     /* extraction: a query missed a path that exists (a
                              zero of a non-zero polynomial, probability about
                              2^-57 per slot); run again with another seed */

#define RS_MAX_K 16
#define RS_MAX_COLOURS 256

/* Human-readable name of a status code (static storage). */
const char* rs_status_str(rs_status s);

/* Library version string, including the GPU target it was built for. */
const char* rs_version(void);

/* Text of the last error seen by the calling thread (HIP call and message),
 * or "" (static thread-local storage, valid until the next call). */
const char* rs_last_error(void);

/* ------------------------------------------------------------------------
 * Graphs (Sec. 2: a directed temporal graph is a SET of triples (u, v, j)
 * with j >= 1; N_j(v) is the set of in-neighbours of v at time j).
 * ---------------------------------------------------------------------- */
typedef struct rs_graph rs_graph;

typedef struct {
  uint32_t n;               /* vertices */
  uint64_t m_input;         /* edges passed in */
  uint64_t m;               /* distinct non-loop edges kept */
  uint64_t self_loops;      /* removed (a self-loop lies on no path) */
  uint64_t duplicates;      /* removed (E is a set) */
  uint32_t t_min, t_max;    /* timestamp range of the input edges (0,0 if none kept) */
  uint32_t n_colours;       /* 0 = uncoloured graph */
  uint32_t max_in_degree;
  uint64_t device_bytes;    /* HBM held by the graph (excluding workspaces) */
} rs_graph_info;

/* Upload a temporal graph. src, dst, t: host arrays of m entries; vertex ids
 * < n, timestamps >= 1 (else RS_EINVAL). colour: host array of n entries with
 * values < n_colours, or NULL (then n_colours must be 0). Duplicated triples
 * and self-loops are dropped. The edges are deduplicated, sorted by
 * (dst, t, src) and indexed on the device. On success *out owns device memory
 * until rs_graph_destroy. Requires n < 2^31 and m + n < 2^32. */
rs_status rs_graph_create(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                          const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                          void* hip_stream, rs_graph** out);

/* As rs_graph_create, with src/dst/t/colour given as DEVICE pointers. */
rs_status rs_graph_create_device(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                                 const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                                 void* hip_stream, rs_graph** out);

rs_status rs_graph_get_info(const rs_graph* g, rs_graph_info* out);

/* Copy the canonical (deduplicated, (dst,t,src)-sorted) edge list to host
 * arrays of info.m entries each (any may be NULL). */
rs_status rs_graph_edges(const rs_graph* g, uint32_t* src, uint32_t* dst, uint32_t* t);

/* Frees the graph and its workspaces. NULL is accepted. */
rs_status rs_graph_destroy(rs_graph* g);

/* ------------------------------------------------------------------------
 * Queries.
 * ---------------------------------------------------------------------- */
typedef struct {
  uint32_t k;                 /* vertices on the path, 2..RS_MAX_K */
  uint32_t delta;             /* resting time delta(v), the same at every vertex */
  const uint8_t* motif_count; /* NULL = k-RestlessPath; else host array of
                                 n_colours multiplicities mu(s) summing to k
                                 (k-RestlessMotif). Copied during the call. */
  uint64_t seed;              /* selects the random substitution */
  uint64_t it_begin, it_end;  /* sieve iterations [it_begin, it_end) of the
                                 2^k; (0, 0) = all. A range yields the partial
                                 fingerprint; partials XOR to the whole. */
} rs_query;

typedef struct {
  uint64_t fingerprint;  /* F over the requested iteration range */
  uint32_t yes;          /* F != 0 (meaningful for the full range) */
  rs_status status;      /* per-query status (batched and served calls) */
  float device_ms;       /* device time of the query (hipEvents), or of the
                            whole batch for rs_run_batch */
} rs_result;

/* Launch-shape knobs; zero fields mean "choose automatically". */
typedef struct {
  uint32_t edges_per_tile;     /* edges per wavefront tile in the scan levels: 8 or 16 */
  uint32_t top_edges_per_tile; /* edges per wavefront in the last level: 1..4096 */
  uint32_t chunks_per_launch;  /* plain path: 64-iteration chunks per launch
                                  (the batched path ignores it) */
  uint32_t waves_per_block;    /* 1, 2 or 4 */
  uint32_t max_slots;          /* batched path: at most this many chunks
                                  resident per round; 0 = as many as the
                                  HBM budget allows */
  uint32_t no_graph;           /* batched path: 1 = enqueue the launches
                                  directly instead of replaying a captured
                                  hipGraph */
  uint32_t chunks_per_wave;    /* plain path: 1 or 2 chunks per wavefront
                                  in the last level (2: one wavefront sums 128
                                  iterations and forms each entry's indices and
                                  row sums once for both chunks). It applies to
                                  queries with k >= 7 whose iteration range
                                  covers an even number of chunks from an even
                                  chunk and whose launches take an even number
                                  of chunks (min(chunks_per_launch, chunks));
                                  the fine-grained last level and any other
                                  query run with 1. 0 = automatic (2 where it
                                  applies). Results are identical. */
} rs_tuning;

/* HBM bytes rs_run needs for this query on this graph beyond the graph
 * itself: window indices 4m, substitution table 8nk, per-level products
 * 8m*kq*(k-1) (kq = k rounded up to a multiple of 4), store and product
 * flags (k-2)*m plus about 5(m+n) bytes of scratch, two prefix-state buffers
 * 2*8*(m+n)*64 per concurrent chunk, look-back state and 8*2^k of
 * per-iteration sums. */
rs_status rs_query_footprint(const rs_graph* g, const rs_query* q, uint64_t* bytes);

/* Plain path: one query, kernels launched one level at a time on hip_stream.
 * Validation (RS_EINVAL): q != NULL; 2 <= k <= RS_MAX_K; motif only on a
 * coloured graph, counts sum to k; it_begin <= it_end <= 2^k. k > n is not an
 * error (F = 0). */
rs_status rs_run(const rs_graph* g, const rs_query* q, rs_result* r, void* hip_stream);

/* As rs_run with explicit launch knobs (NULL = automatic) and, if
 * per_iteration != NULL, the per-iteration values f_L for every iteration of
 * the range copied to that host array (it_end - it_begin entries; 2^k for the
 * full range). */
rs_status rs_run_ex(const rs_graph* g, const rs_query* q, const rs_tuning* tune,
                    uint64_t* per_iteration, rs_result* r, void* hip_stream);

/* ------------------------------------------------------------------------
 * Constraints of the problems of Sec. 3 and the fine-grained oracle of
 * Alg. 1 (Sec. 4.5).
 * ---------------------------------------------------------------------- */
typedef struct {
  const uint32_t* delta_per_vertex; /* host array of n resting times delta(v)
                                       (Sec. 2: delta is a function of the
                                       vertex), or NULL for rs_query.delta at
                                       every vertex. Read during the call. */
  const uint32_t* sources;          /* host array of n_sources vertex ids: only
                                       paths whose first vertex is one of them
                                       count (the source s of the problems of
                                       Sec. 3; several sources as in Sec. 4.6).
                                       NULL / 0 = any first vertex. */
  uint32_t n_sources;
  const uint32_t* targets;          /* host array of n_targets vertex ids: only
                                       paths whose last vertex is one of them
                                       count (the destination d). NULL / 0 =
                                       any last vertex. */
  uint32_t n_targets;
  const uint32_t* removed;          /* host array of n_removed vertex ids that
                                       no path may pass through (the deleted
                                       vertices of the extraction queries of
                                       Sec. 4.7). NULL / 0 = none. */
  uint32_t n_removed;
  uint32_t t_max;                   /* only edges with timestamp <= t_max
                                       (the time-truncated graph of Sec. 4.7);
                                       0 = every edge. */
} rs_constraints;

/* rs_run_ex (automatic launch shape) under constraints c (NULL = none): F is
 * the XOR over the restless paths that start at a source and end at a target
 * of (prod y) det Z_P, so F != 0 decides k-RestlessPath / k-RestlessMotif
 * from s to d. The start restriction keeps the level-1 terms of Eq.
 * (poly-enc:1) of the source vertices only; walks that start elsewhere are
 * never formed. Vertex ids >= n -> RS_EINVAL. */
rs_status rs_run_constrained(const rs_graph* g, const rs_query* q, const rs_constraints* c, uint64_t* per_iteration,
                             rs_result* r, void* hip_stream);

/* Fine-grained oracle (Alg. 1, FineGrainedOracle): the last level's values
 * are summed over the iterations per slot (u, i), giving zeta_{u,k,i}, which
 * is non-zero only if a restless path (motif: colour-agreeing) with k
 * vertices ends at u at time i (and, with constraints, starts at a source).
 * reach_time: host array of n entries, receives R_u = the least i with
 * zeta_{u,k,i} != 0, or 0xFFFFFFFF (D = the vertices with a finite R_u).
 * slot_zeta: host array of info.m entries or NULL; receives, for every edge
 * of the canonical list (rs_graph_edges order), the zeta of its slot
 * (dst, t). r->fingerprint is the XOR of all zeta (the rs_run_constrained
 * fingerprint), r->yes says D is not empty. The iteration range of q selects
 * the iterations summed. */
rs_status rs_run_fine(const rs_graph* g, const rs_query* q, const rs_constraints* c, uint32_t* reach_time,
                      uint64_t* slot_zeta, rs_result* r, void* hip_stream);

/* At most k vertices (Sec. 4.6, at-most-k restless reachability): one
 * fine-grained sieve for each k' = 2..q->k with q's seed and constraints
 * (typically a source). reach_time[u] (n entries) = the least R_u over the
 * k', 0xFFFFFFFF if none; reach_vertices (n entries or NULL) = the least k'
 * with a path ending at u, 0 if none. Path queries over the whole iteration
 * range only (a motif or an iteration range -> RS_EINVAL). r->fingerprint is
 * the XOR of the k' fingerprints; r->yes says some vertex is reached. */
rs_status rs_reach_at_most(const rs_graph* g, const rs_query* q, const rs_constraints* c, uint32_t* reach_time,
                           uint32_t* reach_vertices, rs_result* r, void* hip_stream);

/* Extraction of an optimal solution with k fine-grained queries (Sec. 4.7):
 * a restless path with q->k vertices (colour-agreeing with q->motif_count
 * when given; from a source and to a target under c) whose largest
 * timestamp is least. Query j = k, k-1, .., 2 runs the fine-grained sieve
 * with j vertices on the graph without the vertices found so far and
 * without the edges later than the last timestamp found, with the motif
 * less their colours; the next vertex is the least in-neighbour v (through
 * an edge at that timestamp) with a non-zero slot (v, i) in its waiting
 * window [t - delta(v), t], and i the least such time; the first vertex is
 * the least such in-neighbour that is a source of the remaining colour.
 * On YES (r->yes = 1): path_vertices (host, k entries) receives u_1..u_k and
 * path_times (host, k-1 entries) the timestamps of the edges u_j -> u_{j+1}.
 * On NO (r->yes = 0) neither array is written. r->fingerprint is the first
 * (k-vertex) query's, device_ms the sum over the queries. c->removed and
 * c->t_max must be unset (RS_EINVAL), as must an iteration range. RS_ERETRY
 * if a later query misses the path the earlier ones proved. */
rs_status rs_extract(const rs_graph* g, const rs_query* q, const rs_constraints* c, uint32_t* path_vertices,
                     uint32_t* path_times, rs_result* r, void* hip_stream);

/* Fine-grained sieve under the literal reading of Eq. (poly-enc:1): the y
 * variable of each window term is keyed by the edge's end points, the level
 * and the predecessor's arrival time i - j (y_{uv,l-1,i-j}), and level 1 is
 * x_u at every time, so an edge-update costs one product per window term (up
 * to delta(v) + 1; the evaluation-cost lemma of Sec. 4.3). Paths that differ
 * only in their last edge's time share every variable and cancel in a sum over
 * end times, so each slot is tested on its own (Alg. 1). Outputs as
 * rs_run_fine: reach_time (host, n entries) = least i with zeta_{u,k,i} != 0
 * or 0xFFFFFFFF; slot_zeta (host, info.m entries, or NULL) = the zeta of each
 * canonical edge's slot; r->yes = some slot is non-zero; r->fingerprint = the
 * XOR of the slot values (a checksum, not a decision value). delta_per_vertex:
 * host array of n resting times or NULL for q->delta. The iteration range of
 * q selects the iterations summed. The graph's slot structure is built on the
 * first call (4 bytes per edge and per slot, kept with the graph). */
rs_status rs_run_literal(const rs_graph* g, const rs_query* q, const uint32_t* delta_per_vertex,
                         uint32_t* reach_time, uint64_t* slot_zeta, rs_result* r, void* hip_stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): rs_run_ex without
 * tuning knobs, whose query workspace (window indices, substitution and
 * product rows, flags, prefix states, look-back records, partial sums) is
 * carved from one 256 MiB array in device memory that the library holds per
 * GPU from the first such call until the process ends. The call allocates and
 * frees no device memory and records no events (device_ms = 0; kernel timing
 * and the launch trace skip it); it runs one 64-iteration chunk per launch.
 * A query whose workspace exceeds the array (its footprint at one chunk per
 * launch; about 1 KiB per edge-and-vertex slot plus 8 kq (k-1) bytes per edge)
 * fails with RS_ENOMEM and rs_last_error() says by how much. All calls on one
 * GPU share the array: the library serialises them (each returns after its
 * kernels finish), and the array keeps the last call's contents, which the
 * next call clears where it must (the look-back records). per_iteration as in
 * rs_run_ex. */
rs_status rs_run_noalloc(const rs_graph* g, const rs_query* q, uint64_t* per_iteration, rs_result* r,
                         void* hip_stream);

/* Batched path: nq queries, each on its own graph (graphs[i]; graphs may
 * repeat), evaluated together. Every (query, 64-iteration chunk) is a unit
 * with its own prefix-state buffers; units are packed into rounds, and four
 * stream lanes run one round each at a time. A round holds at most max_slots
 * units and at most a quarter of the HBM budget (a third of free device
 * memory) in prefix state, and never more than 20 GiB, so the lanes together
 * stay within the budget. A round runs level l of all its units in shared launches (one per product-row
 * width), each walking a device table of unit descriptors. The launch
 * sequence is captured once per batch shape into a hipGraph and replayed with
 * new descriptors (tune->no_graph = 1 enqueues it directly).
 * results[i].status holds each query's status (RS_EINVAL for an invalid
 * query, which is skipped); the call returns the first error, or RS_OK.
 * tune == NULL uses the shape rs_autotune chose for graphs[0] (or a default).
 * Results are bit-identical to rs_run. Calls are serialised internally. */
rs_status rs_run_batch(const rs_graph* const* graphs, const rs_query* queries, uint32_t nq,
                       rs_result* results, const rs_tuning* tune, void* hip_stream);

/* Times candidate launch shapes on the sample queries and returns the
 * fastest; the choice is cached per (graph, k class) for later NULL-tuning
 * calls. */
rs_status rs_autotune(const rs_graph* g, const rs_query* sample, uint32_t ns, rs_tuning* out);

/* Batched path only: times candidate batched launch shapes (edges per tile,
 * waves per block, last-level range) on the sample run as one batch, caches
 * the fastest on g for later rs_run_batch calls with tune == NULL whose first
 * graph is g, and returns it in *out (may be NULL). Use a sample shaped like
 * the batches to come (several rounds of chunks exercise the stream lanes);
 * the plain-path choices of rs_autotune are kept. RS_EINVAL for an invalid
 * query or ns == 0. */
rs_status rs_autotune_batch(const rs_graph* g, const rs_query* sample, uint32_t ns, rs_tuning* out);

/* ------------------------------------------------------------------------
 * Kernel timing (hipEvents recorded around the launches of each kernel
 * class on the launch stream while enabled). Classes: "level_scan" (prefix
 * levels 3..k-1), "level_first" (level 2), "level_top" (level k), "qtable",
 * "ztable", "window" (plain path), "batch" (one whole rs_run_batch launch
 * sequence). algorithmic_bytes sums, per launch, the HBM bytes the exact
 * computation has to move: per 64-iteration chunk 1024 bytes of window
 * gathers per edge whose window is non-empty and whose product reaches a read
 * slot (all non-empty windows at level k), and 512 bytes per prefix slot that
 * some window reads; per launch the indices and flags of every edge (8 to 13
 * bytes) and the 8*kq-byte rows of the edges that form a product (twice that
 * at level 2). The window counts are measured once per (graph, delta) while
 * timing is on; that first query synchronises once to read them back.
 * ---------------------------------------------------------------------- */
rs_status rs_profile_enable(int on);
/* Launch trace of the plain path (rs_run, rs_run_ex): while on, every launch
 * is followed by a synchronisation of the query's stream and one line on
 * stderr naming the step (workspace, setup, product rows, prefix level l,
 * last level) with the host wall time since the previous line; prefix levels
 * add the look-back counters: predecessor tiles recomputed after the bounded
 * wait, and probe rounds that found no published record. Initially on when
 * the environment variable RS_TRACE is set to anything but "0". For
 * diagnosing large queries: it serialises the launches with the host and so
 * changes timings. Results are unchanged. Never fails. */
rs_status rs_trace_enable(int on);
/* Look-back counters of the prefix levels (both paths). A level launch
 * carries a segment's running XOR across runs of tiles through published
 * per-run records; a run whose predecessor has not published within a
 * bounded wait recomputes that predecessor's part itself. While counting is
 * on (rs_lookback_count(1), which also zeroes the totals), every query and
 * batch adds its numbers of recomputed predecessor runs and of probe rounds
 * that found no record to process-wide totals, read by rs_lookback_get.
 * Counting adds one device-side atomic per event and a small copy per call;
 * results are unchanged. Never fails (rs_lookback_get: RS_EINVAL for NULL). */
rs_status rs_lookback_count(int on);
rs_status rs_lookback_get(uint64_t* recomputes, uint64_t* unanswered_rounds);
rs_status rs_profile_reset(void);
/* launches and summed milliseconds of a kernel class since the last reset. */
rs_status rs_profile_get(const char* kernel_class, uint64_t* launches, double* total_ms,
                         double* algorithmic_bytes);

/* Measurement aid, not part of the sieve: the bandwidth of the prefix
 * state's access pattern (whole 512-byte rows at random rows of a large
 * array), the practical ceiling for the level kernels' HBM traffic.
 * rows: device array of n_rows rows of 64 uint64 (n_rows a power of two);
 * out: device array of waves rows of 64 uint64 (each wave's XOR of what it
 * read). waves (a multiple of 4) wavefronts each take `steps` steps; a step
 * moves 16 rows read (mode 0), 16 rows written (mode 1, rows is
 * overwritten) or 16 rows read and 8 written (mode 2), at row indices hashed
 * from (wave, step). Bytes moved: waves x steps x rows per step x 512.
 * Enqueued on hip_stream; the caller times it. RS_EINVAL for null pointers,
 * waves not a positive multiple of 4, n_rows not a power of two, or mode > 2;
 * RS_EDEVICE if the launch fails. */
rs_status rs_probe_rows(uint64_t* rows, uint64_t n_rows, uint64_t* out, uint32_t waves, uint32_t steps,
                        uint32_t mode, void* hip_stream);

/* ------------------------------------------------------------------------
 * Server: continuous batching over resident graphs.
 * Worker threads, each with its own HIP stream, take queued queries in
 * arrival order. A query on a large graph runs alone through the plain
 * kernels in a workspace kept resident per graph; queries on small graphs
 * (at most group_max_edges edges) that wait together run as one group
 * through the batched path (shared level launches). Workers run
 * concurrently, so queries overlap on the device. Admission is by HBM: the
 * resident workspaces plus what a job adds stay within the budget, and idle
 * workspaces are freed when a job needs their room. Every result equals the
 * query's rs_run result. All server calls are thread-safe.
 * ---------------------------------------------------------------------- */
typedef struct rs_server rs_server;

typedef struct {
  uint32_t max_inflight;       /* queries running at once (0 = 256) */
  uint64_t group_edge_updates; /* work cap of one group, in edge-updates
                                  (iterations * (k-1) * m summed over its
                                  queries; 0 = 4e9). A query whose remaining
                                  work exceeds what is left of the cap joins
                                  with a slice of whole 64-iteration chunks
                                  (alone, through the plain kernels, when no
                                  other query waits) and its rest rejoins the
                                  queue in arrival order, so queries enter and
                                  leave groups at chunk boundaries; a query
                                  none of whose chunks fits runs alone, whole
                                  (1 turns grouping off). Graphs above
                                  group_max_edges always run whole and alone. */
  uint32_t streams;            /* worker threads and streams (0 = 2, at most 16);
                                  level kernels size their grids to fill the
                                  GPU, so more than two concurrent jobs mostly
                                  compete for the same CUs */
  uint64_t group_max_edges;    /* graphs with at most this many edges are
                                  grouped (0 = 262144) */
} rs_server_opts;

typedef struct {
  uint64_t submitted, completed, admitted, deferred, cancelled, rejected;
  uint64_t queued, inflight;   /* at the time of the call */
  double qps;                  /* completed / seconds since creation */
  double p50_ms, p99_ms;       /* latency submit -> completion of completed queries */
  double busy_ms;              /* wall time of jobs, summed over workers */
  uint64_t jobs;               /* jobs run (a group or a single query) */
  uint64_t held_bytes;         /* device bytes held by resident workspaces */
  uint64_t slices;             /* pieces run of queries that ran in more than
                                  one (work above the group cap) */
} rs_server_stats;

/* hbm_budget: bytes of HBM the server may hold for query workspaces. */
rs_status rs_server_create(uint64_t hbm_budget, const rs_server_opts* opts, rs_server** out);
/* The graph must outlive the server. */
rs_status rs_server_add_graph(rs_server* s, const rs_graph* g, uint32_t* graph_id);
/* Non-blocking. Copies the query (and its motif). RS_EINVAL for invalid
 * queries, RS_ENOMEM if its plain workspace (rs_query_footprint) can never
 * fit the budget. */
rs_status rs_server_submit(rs_server* s, uint32_t graph_id, const rs_query* q, uint64_t* ticket);
/* Wait up to wait_ms (0 = don't wait, <0 = forever). RS_OK with the result,
 * RS_ETIMEOUT if not yet complete, RS_ENOTFOUND for unknown or already
 * collected tickets. */
rs_status rs_server_poll(rs_server* s, uint64_t ticket, rs_result* r, int32_t wait_ms);
rs_status rs_server_cancel(rs_server* s, uint64_t ticket);
rs_status rs_server_stats_get(rs_server* s, rs_server_stats* out);
/* Stops the workers after running jobs finish; queued queries are
 * cancelled; frees the server's workspaces. */
rs_status rs_server_destroy(rs_server* s);

#ifdef __cplusplus
}
#endif
#endif
