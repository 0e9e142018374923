/*
 * libldd -- exponential-shift low-diameter decomposition on AMD Instinct MI355X (gfx950).
 *
 * The operation (Miller, Peng, Xu, "Parallel Graph Decompositions Using Random Shifts"):
 * given an undirected unweighted graph G = (V, E) and one shift delta_u >= 0 per vertex
 * (drawn from Exp(beta) by the caller: Algorithm 1 step 1, Sec. 2), every vertex v joins the
 * centre u that minimises the shifted distance dist(u,v) - delta_u of Eq. (1) (Sec. 3),
 * ties broken by the smaller vertex id (Algorithm 2, Sec. 4).  The pieces {v : c(v) = u}
 * form the partition of Def. 1.1 (Sec. 1); the library also returns the number of edges
 * whose endpoints lie in different pieces.
 *
 * Shifts are passed in fixed point, shift_fix[u] = floor(delta_u * 2^20), so the result is
 * exact and reproducible: c(v) = lexicographic argmin over u of (2^20 dist(u,v) - shift_fix[u], u).
 * It depends only on the graph and shift_fix (beta is a hint and never changes it).
 *
 * The computation follows the breadth-first formulation of Sec. 5: a super source with an
 * arc of length Delta - shift_fix[u] to every u (Delta = max shift), processed one integer
 * distance ("round") at a time; u enters the search at round floor((Delta - shift_fix[u]) / 2^20)
 * unless already reached, and the fractional parts break ties inside a round.
 *
 * Conventions for every entry point
 *   - Device pointers point to memory of the current HIP device; the caller owns them and
 *     must keep them alive until the call returns (single graph) or the request is polled
 *     done (server).  Host pointers are ordinary host memory.
 *   - Graphs are CSR with int32 indices: row_ptr[n+1] (row_ptr[0] = 0, non-decreasing,
 *     row_ptr[n] = nnz) and col_idx[nnz] with 0 <= col_idx[a] < n.  The graph must be
 *     symmetric (each edge stored as two arcs).  Self-loops are never cut; repeated arcs
 *     count with multiplicity in the cut.
 *   - Calls never abort and never throw; they return an ldd_status.  Argument errors are
 *     detected before any device work where the check is O(1); malformed CSR content is
 *     reported as LDD_ERR_INVALID_ARG by bounds checks inside the kernels (no out-of-range
 *     access is made).  ldd_last_error() gives a thread-local detail string.
 *   - hip_stream is a hipStream_t (NULL = default stream).  Work is ordered on that stream;
 *     the single-graph and batch calls return once their outputs are complete.  Round steps
 *     enqueued ahead of the end may still be queued on the stream then; they return at once,
 *     and later work on the stream is ordered after them and after the outputs; a later call
 *     on another stream of the same device starts after them too (the workspace is shared).
 */
#ifndef LDD_H
#define LDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LDD_OK = 0,
  LDD_ERR_INVALID_ARG = 1, /* bad pointer, size, CSR content or negative shift            */
  LDD_ERR_OOM = 2,         /* device workspace allocation failed                           */
  LDD_ERR_OVERFLOW = 3,    /* (Delta + 2^20) << ceil(log2 n) does not fit 64 bits, or the */
                           /* shifts span more rounds than the engine takes                */
  LDD_ERR_HIP = 4,         /* a HIP runtime call failed (text in ldd_last_error)           */
  LDD_ERR_BUDGET = 5,      /* server: request larger than the whole memory budget          */
  LDD_ERR_CANCELLED = 6,   /* server: request cancelled before it ran                      */
  LDD_ERR_INTERNAL = 7,    /* round watchdog or barrier time-out fired (a library bug)     */
  LDD_ERR_PENDING = 8,     /* server: request not finished yet                             */
  LDD_ERR_RETRIES = 9      /* verified decomposition: no draw met the bounds               */
} ldd_status;

/* One CSR graph in device memory (see conventions above). */
typedef struct {
  int32_t n;              /* vertices, >= 0                                               */
  int64_t nnz;            /* arcs (twice the undirected edges), 0 <= nnz < 2^31            */
  const int32_t* row_ptr; /* device [n+1]                                                 */
  const int32_t* col_idx; /* device [nnz]                                                 */
} ldd_csr;

/* Traversal direction policy of a round (the result never depends on it). */
enum { LDD_DIR_AUTO = 0, LDD_DIR_TOP_DOWN = 1, LDD_DIR_BOTTOM_UP = 2 };
/* Round engine: one persistent kernel with grid barriers, one launch per round step over the
 * whole GPU, one workgroup running every round of the graph (workgroup barriers only), or a team
 * of workgroups (blocks of them, default one per CU, at most the workgroups that can be resident
 * at once) running every round with one barrier in device memory per round (top-down only: for
 * large graphs of low degree and many rounds, such as grids).  AUTO: a graph of more than 7 arcs
 * per vertex on average, or a call with direction LDD_DIR_BOTTOM_UP, takes the launch engine; a
 * sparser graph takes one workgroup when it has at most 2^15 arcs, else a team, unless a vertex
 * has more than 4096 arcs (the team finds it in its preparation and the call continues on the
 * launch engine).  ldd_tune may pick any of them. */
enum {
  LDD_ENGINE_AUTO = 0,
  LDD_ENGINE_PERSISTENT = 1,
  LDD_ENGINE_LAUNCH = 2,
  LDD_ENGINE_WORKGROUP = 3,
  LDD_ENGINE_TEAM = 4
};

typedef struct {
  int32_t direction;      /* LDD_DIR_*                                                    */
  int32_t engine;         /* LDD_ENGINE_*                                                 */
  int32_t validate;       /* 1: check CSR monotonicity on the device before running       */
  int32_t blocks;         /* workgroups of the round kernel (0 = 2 per CU; the workgroup batch engine
                             and a team: 1 per CU, a team at most the workgroups that can be resident
                             at once, one per CU; at most 1024)                                               */
  int32_t td_to_bu;       /* switch to bottom-up when frontier arcs * td_to_bu > unsettled arcs (0 = default 14) */
  int32_t bu_to_td;       /* switch back when frontier vertices * bu_to_td < n (0 = default 24)                 */
  int32_t tail_vertices;  /* finish by label correction once unsettled vertices * this <= active vertices
                             (0 = default 32, -1 = never)                                                      */
  int32_t batch_mode;     /* ldd_decompose_batch: LDD_BATCH_* (below)                                    */
  int32_t team_arcs;      /* workgroup batch engine: arcs per workgroup of a team (0 = default: all arcs over
                             the grid, at least 2^14; -1 = no teams: one workgroup per graph)                 */
  int32_t reserved[7];
} ldd_options;

/* Batch engines: AUTO = WORKGROUP (one workgroup per graph, the largest graphs first, every
 * graph's rounds with workgroup barriers only; a graph with many more arcs than a workgroup's
 * share of the batch runs on a team of up to 16 workgroups that meet at a barrier in device
 * memory once per round; a graph whose shifts span 4096 or more units of distance runs alone on
 * the launch engine); SEQUENTIAL = one ldd_decompose per graph (the plain
 * path, for comparison); UNION = the disjoint union of all graphs on the launch engine, one
 * launch per round for all graphs. */
enum { LDD_BATCH_AUTO = 0, LDD_BATCH_SEQUENTIAL = 1, LDD_BATCH_UNION = 2, LDD_BATCH_WORKGROUP = 3 };

/* Counters of the last call (filled when a non-NULL pointer is passed). */
typedef struct {
  int32_t rounds;          /* rounds executed (empty rounds skipped are not counted)      */
  int32_t rounds_bound;    /* floor(Delta / 2^20) + 1                                     */
  int32_t td_rounds;       /* rounds expanded top-down                                    */
  int32_t bu_rounds;       /* rounds expanded bottom-up                                   */
  int32_t tail_iters;      /* label-correction sweeps after switching to the tail         */
  int32_t tail_round;      /* first round the tail replaced (-1: rounds ran to the end)   */
  int32_t blocks;          /* workgroups used by the round kernel                         */
  int64_t delta;           /* max shift_fix                                               */
  int64_t pieces;          /* number of centres                                           */
  int64_t max_frontier;    /* largest frontier (vertices)                                 */
  int64_t arcs_examined;   /* arcs read by the traversal (all of F's arcs top-down; the   */
                           /* arcs scanned before the early exit bottom-up)               */
  int64_t n_active;        /* vertices with at least one arc                              */
  float ms_prep;           /* device time: init, Delta, wake-round sort (HIP events)      */
  float ms_rounds;         /* device time: all round steps enqueued, idle ones included   */
  float ms_finalize;       /* device time: centre extraction                              */
  float ms_cut;            /* device time: cut count                                      */
  int32_t steps;           /* round-kernel launches (steps) enqueued, done ones included  */
  int64_t max_radius;      /* largest distance from a vertex to its centre                */
} ldd_stats;

/*
 * Decompose one graph (Algorithm 2 via the search of Sec. 5).
 *   g          graph in device memory.
 *   shift_fix  device int64[n], 0 <= shift_fix[u] <= 2^52, units of 2^-20.
 *   beta       the Exp rate the shifts were drawn with (0 < beta); a hint only.
 *   centre     device int32[n], OUT: centre id of every vertex.
 *   cut_edges  host int64*, OUT (may be NULL): edges whose endpoints have different centres.
 *   opt        NULL for defaults.
 *   stats      host, OUT (may be NULL).
 * Returns once centre and the cut are complete (see the stream convention above).
 */
ldd_status ldd_decompose(const ldd_csr* g, const int64_t* shift_fix, double beta, int32_t* centre,
                         int64_t* cut_edges, const ldd_options* opt, ldd_stats* stats, void* hip_stream);

/* Device bytes the library's workspace needs for one graph of this size (upper bound). */
size_t ldd_workspace_bytes(int32_t n, int64_t nnz);

/*
 * Decompose many independent graphs in one pass (same operation per graph).
 * The graphs are packed into one offset CSR with LOCAL vertex ids:
 *   vtx_off   host int64[num_graphs+1], graph g owns vertices [vtx_off[g], vtx_off[g+1]).
 *   arc_off   host int64[num_graphs+1], graph g owns arcs [arc_off[g], arc_off[g+1]).
 *   row_ptr   device int32[vtx_off[G] + num_graphs]: graph g's row offsets (n_g+1 entries,
 *             starting at 0) stored at row_ptr[vtx_off[g] + g].
 *   col_idx   device int32[arc_off[G]]: local ids 0 <= col < n_g.
 *   shift_fix device int64[vtx_off[G]]; centre device int32[vtx_off[G]] OUT (local ids).
 *   cut_edges host int64[num_graphs] OUT (may be NULL).
 * Each graph's result equals ldd_decompose on that graph alone, bit for bit.
 */
ldd_status ldd_decompose_batch(int32_t num_graphs, const int64_t* vtx_off, const int64_t* arc_off,
                               const int32_t* row_ptr, const int32_t* col_idx, const int64_t* shift_fix,
                               int32_t* centre, int64_t* cut_edges, const ldd_options* opt, void* hip_stream);

/*
 * Tune the engine and its mapping for a workload: the engine (one graph: engine = LAUNCH,
 * PERSISTENT, TEAM, or WORKGROUP when nnz <= 2^22; a batch: batch_mode = WORKGROUP or UNION), grid
 * size (blocks: a quarter of the CU count up to four per CU), the top-down / bottom-up switching thresholds (td_to_bu, bu_to_td; not for the
 * workgroup engine and its teams, which run top-down only), the tail threshold (tail_vertices) and, for the
 * workgroup batch engine, the arcs per team member (team_arcs), searched one knob at a time by
 * timing whole decompositions of the given inputs (median of three, HIP events on hip_stream).  The inputs are those of ldd_decompose_batch (num_graphs = 1: one graph,
 * run through ldd_decompose); centre is scratch output of the right size.  Every candidate gives
 * the same result, so only time is traded.  The winner is cached per workload signature (device,
 * CU count, number of graphs, vertices, arcs) in the process and, if cache_path is not NULL, in
 * that text file (appended; a later line for a signature wins).  base (may be NULL) supplies the
 * other options.  *best receives base with the tuned knobs; *report (may be NULL) the timings.
 */
typedef struct {
  float default_ms;   /* the starting point (the base options' knobs, or the defaults)       */
  float best_ms;      /* the winner (from the cache if from_cache)                            */
  int32_t runs;       /* decompositions timed                                                 */
  int32_t from_cache; /* 1: no run, the cached winner was returned                            */
} ldd_tune_report;

ldd_status ldd_tune(int32_t num_graphs, const int64_t* vtx_off, const int64_t* arc_off, const int32_t* row_ptr,
                    const int32_t* col_idx, const int64_t* shift_fix, int32_t* centre, const ldd_options* base,
                    const char* cache_path, ldd_options* best, ldd_tune_report* report, void* hip_stream);

/*
 * Serving: a long-lived engine that decomposes a stream of independent requests (the same
 * operation as ldd_decompose per request, bit for bit) with continuous batching.  Admitted
 * requests share one device-resident arena of per-vertex state and advance together, one
 * launch per round over all of them; a request joins at the next round boundary and leaves as
 * soon as its own labels are final, while others keep going.  The arena is sized once, from
 * the memory budget; requests wait in a first-come-first-served queue until their vertices and
 * a slot fit.  A request whose round 0 runs at global round r0 is the search of Sec. 5 with
 * every source arc lengthened by r0 units, which changes no comparison inside its component.
 *
 * Threads: one engine thread per server owns its device stream.  submit / poll / wait / cancel
 * / query may be called from any thread.  All calls return an ldd_status.
 */
typedef struct ldd_server ldd_server;

typedef struct {
  int64_t hbm_budget_bytes; /* arena size in device bytes, 33 B per arena vertex (labels, queues, */
                            /* wake order, stamps); requests' CSR and shifts stay in the callers' */
                            /* buffers and take no arena space                                    */
  int64_t max_vertices;     /* arena vertices (a request takes n + 1 rounded up to 64);           */
                            /* 0 = from the budget (at most 2^30)                                 */
  int64_t max_arcs;         /* unused (0)                                                         */
  int32_t max_slots;        /* requests on the device at once, 1..256 (0 = 256)                   */
  int32_t chunk_steps;      /* rounds per replayed launch graph, 1..64 (0 = 4)                    */
  int32_t blocks;           /* workgroups of the round kernel (0 = 2 per CU)                      */
  int32_t direction;        /* LDD_DIR_* policy of every round                                     */
  int32_t max_rounds;       /* testing: key range in rounds before keys are rebased (0 = the      */
                            /* largest the label width allows); requests may need at most half   */
  int32_t tail_vertices;    /* a request finishes by label correction once its unreached         */
                            /* vertices * this <= its vertices with arcs (0 = 32, -1 = never)     */
  int32_t reserved[6];
} ldd_server_config;

/* One request.  All buffers are device memory of the server's device, owned by the caller,
 * and must stay alive and unchanged until the request is reported done (poll / wait). */
typedef struct {
  int32_t n;                /* vertices, >= 0                                                 */
  int64_t nnz;              /* arcs, 0 <= nnz < 2^31, stored symmetric as for ldd_decompose   */
  const int32_t* row_ptr;   /* device [n+1]                                                   */
  const int32_t* col_idx;   /* device [nnz]                                                   */
  const int64_t* shift_fix; /* device [n], in [0, 2^52], units of 2^-20                        */
  int32_t* centre;          /* device [n], OUT: centre of every vertex (request-local ids)     */
  void* hip_stream;         /* stream whose queued work produces the inputs (NULL = default)  */
} ldd_request;

typedef struct {
  ldd_status status;        /* LDD_OK, LDD_ERR_INVALID_ARG / LDD_ERR_OVERFLOW (content),       */
                            /* LDD_ERR_CANCELLED, or the engine's failure                      */
  int32_t rounds;           /* floor(Delta / 2^20) + 1 of the request                          */
  int64_t cut_edges;        /* edges whose endpoints have different centres                    */
  int64_t first_round;      /* global round its round 0 ran at (numbering at admission)        */
  double t_submit;          /* seconds since the server was created                            */
  double t_admit;
  double t_done;
  double latency_ms;        /* t_done - t_submit                                               */
} ldd_result;

typedef struct {
  int64_t arena_vertices;
  int64_t arena_arcs;       /* 0: arcs are read from the callers' buffers                          */
  int32_t max_rounds;       /* largest floor(Delta / 2^20) + 1 a request may have              */
  int32_t max_slots;
  int64_t admitted;
  int64_t completed;
  int64_t queued;
  int64_t max_active;       /* most requests on the device at once so far                      */
  int64_t steps;            /* rounds launched so far                                          */
  int64_t rebases;
} ldd_server_info;

/* Create a server on the current HIP device.  LDD_ERR_BUDGET if the budget gives no usable
 * arena, LDD_ERR_OOM if the arena cannot be allocated. */
ldd_status ldd_server_create(const ldd_server_config* cfg, ldd_server** out);

/* Queue a request.  Only O(1) checks happen here: LDD_ERR_INVALID_ARG for bad sizes or NULL
 * pointers, LDD_ERR_BUDGET if its vertices can never fit the arena.  On LDD_OK *ticket names the request
 * until its result is collected.  An event recorded on req->hip_stream orders the request's
 * admission after the work that stream has queued so far.  The content is checked on the
 * device at admission: row offsets not non-decreasing from 0 to nnz, a shift outside
 * [0, 2^52] or a column id outside [0, n) make the result's status LDD_ERR_INVALID_ARG, more
 * rounds than the server takes (ldd_server_info.max_rounds) LDD_ERR_OVERFLOW; such a request
 * never disturbs the others. */
ldd_status ldd_server_submit(ldd_server* srv, const ldd_request* req, uint64_t* ticket);

/* LDD_ERR_PENDING while the request runs; otherwise fills *out, forgets the ticket and returns
 * the request's status.  After a result is collected, req->centre holds the decomposition. */
ldd_status ldd_server_poll(ldd_server* srv, uint64_t ticket, ldd_result* out);

/* As poll, blocking until the request is done. */
ldd_status ldd_server_wait(ldd_server* srv, uint64_t ticket, ldd_result* out);

/* Cancel a request still in the queue (its result then has status LDD_ERR_CANCELLED and must
 * still be collected); LDD_ERR_PENDING if it is already on the device. */
ldd_status ldd_server_cancel(ldd_server* srv, uint64_t ticket);

/* Counters and limits; returns the engine's failure status, if any. */
ldd_status ldd_server_query(ldd_server* srv, ldd_server_info* out);

/* Finish every queued and running request, then free the server (tickets not collected are
 * dropped).  Returns the engine's failure status, if any. */
ldd_status ldd_server_destroy(ldd_server* srv);

/*
 * Decompose one graph without allocating: for callers that cannot allocate device or pinned
 * host memory (code that must not call hipMalloc / hipFree, tight serving loops, harnesses
 * that forbid allocation).  Same operation, arguments and result as ldd_decompose (bit for
 * bit), with these differences:
 *   - every device buffer beyond the caller's inputs and outputs comes from one file-scope
 *     device array of LDD_STATIC_SCRATCH_BYTES (34.4 MiB) per device, held from the first
 *     call on that device until the process ends; the call makes no hipMalloc / hipFree, no
 *     pinned host allocation and creates no event, stream or graph;
 *   - n <= LDD_STATIC_MAX_VERTICES, else LDD_ERR_BUDGET before any device work; shifts whose
 *     range spans 8192 or more units of distance (floor(max shift / 2^20) >= 8192) also give
 *     LDD_ERR_BUDGET (ldd_decompose handles them);
 *   - work runs on hip_stream only, and the call synchronises that stream (after every eight
 *     round steps and at the end), so it cannot be captured into a graph;
 *   - no statistics; opt->engine must not be LDD_ENGINE_PERSISTENT.
 * All calls on one device share its array and the array keeps the last call's contents (what
 * must start at zero is cleared at the start of each call): calls that overlap on one device,
 * from several threads or streams, race and must be serialised by the caller.
 */
#define LDD_STATIC_MAX_VERTICES (1 << 20)
#define LDD_STATIC_SCRATCH_BYTES 36040704
ldd_status ldd_decompose_static(const ldd_csr* g, const int64_t* shift_fix, double beta, int32_t* centre,
                                int64_t* cut_edges, const ldd_options* opt, void* hip_stream);

/*
 * Shifts delta_u ~ Exp(beta) for u < n in fixed point (Algorithm 1 step 1, Sec. 2; the
 * exponential density beta exp(-beta x) of Sec. 3), shift_fix[u] = floor(2^20 delta_u), drawn by
 * inverting the CDF at a uniform U_u from a counter-based generator: draw u of seed s depends
 * only on (s, u) (O(n) work, O(1) depth, as the proof of Theorem 1.1 in Sec. 5 uses).  The recipe
 * (SplitMix64 draws, U = (x >> 11) 2^-53, -ln(1 - U) by an integer-only base-2 logarithm to 47
 * bits, then floor((T * ln2 * 2^-27) / beta) in correctly rounded double arithmetic) gives the same
 * bits on the host and on the device.
 *   ldd_make_shifts         host:   out_host int64[n] (caller's host memory).
 *   ldd_make_shifts_device  device: out_device int64[n] (caller's device memory), enqueued on
 *                           hip_stream; returns once enqueued.
 * LDD_ERR_INVALID_ARG for n < 0, a NULL buffer with n > 0, or beta not finite and > 0.
 */
ldd_status ldd_make_shifts(int32_t n, double beta, uint64_t seed, int64_t* out_host);

/*
 * Shift variants of the closing remarks of Sec. 5, which note that the fractional parts of the
 * shifts act only as a random ordering for ties, and that shifts may be assigned from positions
 * in a random permutation instead of being sampled.  A seeded random ranking orders the vertices
 * (by a 64-bit counter-based draw of the seed's permutation stream, ties by id).
 *   LDD_SHIFTS_EXP         ldd_make_shifts.
 *   LDD_SHIFTS_INT_PERM    the integer parts of the Exp(beta) shifts of the same seed, plus the
 *                          fraction floor((n - 1 - rank) 2^20 / n): rank 0 wins every tie.  The
 *                          fractions are distinct while n <= 2^20 (beyond, nearby ranks share one
 *                          and the smaller id wins).
 *   LDD_SHIFTS_PERM_ORDER  the vertex of rank i takes the expected i-th largest of n Exp(beta)
 *                          draws, (H_n - H_i) / beta (H_i = sum_{j<=i} 1/j, the order statistics'
 *                          expectations), as floor(2^20 (S_i / beta)) with S_i accumulated from
 *                          S_n = 0 down to S_i = S_{i+1} + 1/(i+1) in double.
 * Host only (the ranking is a sort); out_host int64[n].  LDD_ERR_INVALID_ARG as ldd_make_shifts,
 * or for an unknown kind.
 */
enum { LDD_SHIFTS_EXP = 0, LDD_SHIFTS_INT_PERM = 1, LDD_SHIFTS_PERM_ORDER = 2 };
ldd_status ldd_make_shifts_variant(int32_t n, double beta, uint64_t seed, int32_t kind, int64_t* out_host);
ldd_status ldd_make_shifts_device(int32_t n, double beta, uint64_t seed, int64_t* out_device, void* hip_stream);

/*
 * Las Vegas decomposition (the proof of Theorem 1.1, Sec. 5): draw the shifts on the device
 * (ldd_make_shifts_device with seed, seed + 1, ...), decompose, verify the partition, and draw
 * again until it meets both bounds of a (beta, O(log n / beta)) decomposition:
 *   cut_edges  <= cut_factor * beta * m                  (m = nnz / 2; Cor. 4.5 bounds the
 *                                                          expected cut by (1 - e^-beta) m)
 *   max_v dist(c(v), v) <= radius_factor * ln(n) / beta  (Lemma 4.2: every shift is below
 *                                                          (d+1) ln n / beta w.h.p., and a
 *                                                          vertex's distance to its centre is
 *                                                          at most the centre's shift)
 * Verification is O(m) work on the device: the cut of the output pass and the largest distance
 * to a centre, read off the exact labels.  Defaults: cut_factor 2 (by Markov's inequality a
 * draw fails the cut bound with probability below 1/2), radius_factor 3 (d = 2), 16 attempts.
 *   g          graph in device memory (as ldd_decompose).
 *   shift_fix  device int64[n], OUT: the shifts of the last draw (caller's memory).
 *   centre     device int32[n], OUT: the decomposition of the last draw.
 *   vopt, opt  NULL for defaults.
 *   report     host, OUT (may be NULL): attempts, acceptance, the last draw's seed, cut and radius.
 * Returns LDD_OK when the last draw was accepted, LDD_ERR_RETRIES when max_attempts draws all
 * failed (the outputs then hold the last draw), or the decomposition's own errors.
 */
typedef struct {
  double cut_factor;     /* accept when cut_edges <= cut_factor * beta * m (0 = 2)            */
  double radius_factor;  /* accept when every distance to a centre <= radius_factor ln n / beta (0 = 3) */
  int32_t max_attempts;  /* draws before giving up (0 = 16)                                    */
  int32_t reserved[7];
} ldd_verify_options;

typedef struct {
  int32_t attempts;      /* draws made; the outputs hold the last one                         */
  int32_t accepted;      /* 1: the last draw met both bounds                                  */
  uint64_t seed;         /* seed of the last draw                                             */
  int64_t cut_edges;     /* cut of the last draw                                              */
  int64_t max_radius;    /* largest dist(c(v), v) of the last draw                            */
  double cut_bound;      /* cut_factor * beta * m                                             */
  double radius_bound;   /* radius_factor * ln(n) / beta                                      */
} ldd_verify_report;

ldd_status ldd_decompose_verified(const ldd_csr* g, double beta, uint64_t seed, int64_t* shift_fix, int32_t* centre,
                                  const ldd_verify_options* vopt, const ldd_options* opt, ldd_verify_report* report,
                                  void* hip_stream);

/*
 * Block decomposition (the Linial-Saks decomposition of Sec. 2, obtained by iterating the
 * decomposition): level 0 decomposes the whole graph with shifts drawn as ldd_make_shifts_device
 * (beta, seed); the edges inside a piece take level 0 and the cut edges form the graph of level
 * 1, decomposed with seed + 1, and so on.  Each level cuts an edge with probability below beta
 * (Cor. 4.5), so the edges left shrink geometrically; the edges of one level join only vertices
 * of one piece of that level, within O(log n / beta) of its centre (Lemma 4.2).
 *   g            graph in device memory (as ldd_decompose).
 *   beta         the decomposition's parameter per level, in (0, 1); 0 = 1/2.
 *   max_levels   levels at most (>= 1).
 *   arc_level    device int32[nnz], OUT: the level of every arc (both arcs of an edge share it);
 *                -1 for arcs left after max_levels levels.
 *   levels       host, OUT: levels run.
 *   level_edges  host int64[max_levels] (may be NULL), OUT: edges placed in each level run.
 *   opt          options of the per-level decompositions (NULL = defaults).
 * Returns LDD_ERR_RETRIES when arcs are left after max_levels levels (outputs as described),
 * else as ldd_decompose.  Allocates its own device buffers (a few arrays of n and nnz ints).
 */
ldd_status ldd_block_decompose(const ldd_csr* g, double beta, uint64_t seed, int32_t max_levels, int32_t* arc_level,
                               int32_t* levels, int64_t* level_edges, const ldd_options* opt, void* hip_stream);

/* Human-readable name of a status code (static string). */
const char* ldd_status_string(ldd_status s);
/* Detail of the last error on this thread (static thread-local buffer). */
const char* ldd_last_error(void);
/* Release cached device workspaces of the calling thread's current device. */
void ldd_release_workspace(void);

#ifdef __cplusplus
}
#endif
#endif /* LDD_H */
