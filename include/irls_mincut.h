/*
 * irls_mincut.h -- C ABI of the MI355X (gfx950) IRLS undirected s-t min-cut
 * library (libirls_mincut.so).
 *
 * Method: Zhu & Gleich, "A Parallel Min-Cut Algorithm using Iteratively
 * Reweighted Least Squares".
 *   - problem (Section 2): G = (V, E) undirected, capacities c({u,v}) > 0,
 *     source s, sink t, G connected; find the s-t cut of least capacity;
 *   - IRLS (Section 2.1): round 0 solves the weighted least-squares problem
 *     (eq. constrained-wls) with W = C; each later round recomputes the edge
 *     conductances from the current potentials (Step 1, eq.
 *     define-reweight-vector with eq. reweighted-laplacian) and solves the
 *     reduced Laplacian system L~ v = b (eq. reduced-laplacian-system) on the
 *     non-terminal nodes with x_s = 1, x_t = 0;
 *   - solver (Section 3.1): Jacobi-preconditioned CG, warm-started from the
 *     previous round;
 *   - rounding (Section 3.4): sweep cut over the sorted final potentials.
 *
 * Every call returns an irls_status; no exception or signal crosses the ABI.
 * Argument validation finishes before any HIP call, so error paths can be
 * exercised without a GPU.  Handles are not thread safe; distinct handles are
 * independent.  All device work of a handle is ordered on the HIP stream given
 * at creation; calls that return host-visible results synchronise it.
 */
#ifndef IRLS_MINCUT_H
#define IRLS_MINCUT_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct irls_mincut_s *irls_mincut_t;   /* opaque, owned by the library */

typedef enum {
  IRLS_OK = 0,
  IRLS_ERR_NULL = 1,          /* a required pointer is NULL */
  IRLS_ERR_RANGE = 2,         /* n < 2, m < 0, an endpoint or s/t outside [0,n), s == t,
                                 a non-finite potential, or a graph too large for 32-bit
                                 device indices */
  IRLS_ERR_CAPACITY = 3,      /* a capacity <= 0, NaN or infinite (Section 2: c > 0) */
  IRLS_ERR_DISCONNECTED = 4,  /* G is not connected (Section 2; Proposition 1) */
  IRLS_ERR_OPTIONS = 5,       /* an option out of range or struct_size mismatch */
  IRLS_ERR_NOT_SOLVED = 6,    /* cut/potentials requested before a successful solve */
  IRLS_ERR_CG_BREAKDOWN = 7,  /* p^T q <= 0 or a non-finite CG scalar */
  IRLS_ERR_DEVICE = 8,        /* HIP runtime error; text in irls_mincut_last_error */
  IRLS_ERR_OOM = 9,           /* device or host allocation failed */
  IRLS_WARN_CG_MAXIT = 100    /* finished, but some round stopped at cg_maxit */
} irls_status;

/* Options.  Fill with irls_options_default() and change fields. */
typedef struct {
  int32_t struct_size;        /* must equal sizeof(irls_options) */
  int32_t rounds;             /* T, reweighted rounds after round 0 (>= 0), default 30 */
  double  eps0;               /* smoothing of round 1 (> 0), default 0.1 */
  double  eps_factor;         /* eps_{l+1} = eps_l * eps_factor, in (0,1], default 0.5 */
  int32_t weight_form;        /* 0: g = c/sqrt(d^2+eps) (default);
                                 1: g = c^2/sqrt((c d)^2+eps), the paper's w with eps^2 -> eps */
  int32_t init;               /* 0: round 0 solves with W = C (paper, default);
                                 1: x = 1/2 on every non-terminal, no round-0 solve;
                                 2: caller potentials x0 passed to irls_mincut_solve */
  int32_t warm_start;         /* 1: CG starts from the previous round (default); 0: from 0 */
  double  cg_rtol;            /* stop when ||r||_2 <= cg_rtol * ||b||_2, default 1e-10 */
  int64_t cg_maxit;           /* per round, >= 1, default 100000 */
  int32_t precision;          /* 0: FP64 everywhere (default);
                                 1: FP32 conductances, SpMV and CG vectors, FP64 potentials,
                                    FP64 dot products, FP64 residual replacement */
  int32_t refine_every;       /* precision 1: true FP64 residual every this many CG steps */
  double  fp64_weights_below_eps; /* precision 1: conductances computed in FP64 once eps is
                                     below this value, in FP32 before (default 1e-4) */
  int32_t format;             /* 0 auto; 1 CSR; 2 diagonal (few constant index offsets) */
  int32_t solver;             /* 0 auto; 1 multi-workgroup kernels; 2 one resident workgroup */
  int32_t chunk;              /* CG iterations launched between host checks, 0 = auto */
  int32_t inputs_on_device;   /* 1: edge arrays and x0 are device pointers */
  int32_t rows_per_wave;      /* CSR SpMV rows per 64-lane wavefront: 0 auto (from the
                                 average row length), else 1,2,4,...,64 */
  int32_t precond;            /* 0: Jacobi, M = diag(L~) (default);
                                 1: block-Jacobi (Section 3.1), M = the principal submatrices
                                    of L~ over blocks of block_size consecutive rows, each
                                    solved exactly.  Needs a grid (diagonal format, offsets
                                    1 < off[1] < ...), FP64 and the multi-workgroup solver;
                                    a block then lies inside one line of offset-1 edges, so
                                    it is tridiagonal;
                                 2: block-Jacobi with every block solved by ILU(0) in
                                    ascending row order (Section 3.1's second strategy: L
                                    unit lower and U upper triangular on the block's
                                    pattern, (LU)_ij = L~_ij there), factored once per
                                    round; the multi-workgroup solver, FP64 (the precision
                                    form only with tiles of edge 4: FP32 pivots, residual
                                    and substitutions; the FP64 residual replacement is
                                    followed by the application).  In the
                                    diagonal format the blocks are cubic tiles of a 3-D grid
                                    (block_size^3 rows: block_size consecutive rows of
                                    block_size lines of block_size planes; offsets 1, N, P
                                    with N and the P / N lines of a plane multiples of
                                    block_size, whole planes; tiles past the last plane are
                                    cut short).  In CSR (any graph; format 1 forces it) a
                                    block is block_size consecutive positions of a
                                    breadth-first ordering of the non-terminal rows (from
                                    the smallest unvisited row, neighbours in ascending
                                    order) */
  int32_t block_size;         /* precond 1: rows per block, even, 2..128 and at most
                                 off[1]; 0 = min(off[1], 128) rounded down to even.
                                 precond 2: tiles: the tile edge, 2, 4 or 8 (0 = 4); CSR:
                                 rows per block, even, 2..128 (0 = 32) */
  int32_t unscaled_cg;        /* 0 (default): where the marching SpMV runs (3-D grids) with
                                 point Jacobi, CG runs on the symmetrically scaled system
                                 D^-1/2 L~ D^-1/2 -- in exact arithmetic the same iterates as
                                 Jacobi PCG (Section 3.1), but the SpMV reads no diagonal;
                                 1: always the z = D^-1 r form */
  double  stop_gap;           /* 0 (default): run every round.  > 0: stop after the first
                                 round whose certified gap l1 - lower_bound (see
                                 irls_round_stats) is at most stop_gap * l1; then
                                 mu* <= sweep cut <= l1 <= lower_bound / (1 - stop_gap).
                                 Rounds after the stop are not run: their records hold
                                 eps = 0 and cg_iters = 0 */
} irls_options;

/* Per-round record (round 0 first). */
typedef struct {
  double  eps;                /* smoothing of this round (0 for round 0) */
  int64_t cg_iters;           /* CG iterations of this round */
  double  rel_res;            /* recursive ||r||/||b|| at exit */
  double  true_rel_res;       /* ||b - L~ v||/||b|| recomputed in FP64 at exit */
  double  s_eps;              /* smoothed objective (eq. l1-min-smooth-version) at this
                                 round's x, with the next round's eps */
  double  l1;                 /* ||C B x||_1 (eq. l1-min) */
  double  flow;               /* x^T L x, the electrical flow value (Proposition 3) */
  double  flow_s, flow_t;     /* flow leaving s / entering t */
  double  vmin, vmax;         /* range of the non-terminal potentials (Proposition 2) */
  int32_t status;             /* irls_status of this round's CG */
  double  lower_bound;        /* a lower bound on the minimum cut mu* from this round's
                                 electrical flow f_e = g_e (x_u - x_v) (Proposition 3).
                                 Node u's imbalance is the residual r_u, so f's net flow
                                 across any s-t cut is at least
                                 F = max(flow_s, flow_t) - ||b - L~ x||_1.  By max-flow /
                                 min-cut duality both F / max(1, rho), with rho = the
                                 largest |f_e| / c_e (f scaled to respect every capacity),
                                 and F - sum_e max(0, |f_e| - c_e) (a cut carries at most
                                 its capacity plus its edges' overload) are at most mu*;
                                 this is the larger.  With l1 >= mu* the pair brackets
                                 the minimum cut.  In round 0 (g = c, |x_u - x_v| <= 1)
                                 it is the flow value E0 of the Cheeger-type bracket,
                                 less the residual. */
} irls_round_stats;

/* Fills *o with the defaults given beside each field, struct_size included
 * (NULL is a no-op). */
void irls_options_default(irls_options *o);

/* Build a handle for graph G.
 *   n        nodes, ids 0..n-1 (n >= 2)
 *   m        edges; edge e joins edge_u[e] and edge_v[e] with capacity cap[e] > 0.
 *            Edges are undirected; self loops are dropped; parallel edges are merged
 *            by summing their capacities in ascending e.  The s-t edge counts in the
 *            cut value but not in the linear systems.
 *   s, t     source and sink
 *   opt      NULL = defaults; copied
 *   hip_stream  hipStream_t to order all work on, NULL = the default stream
 * Arrays are read during the call only (host memory, or device memory when
 * opt->inputs_on_device); the caller keeps ownership.  On error *out = NULL and
 * nothing is leaked. */
irls_status irls_mincut_create(irls_mincut_t *out, int64_t n, int64_t m,
                               const int64_t *edge_u, const int64_t *edge_v,
                               const double *cap, int64_t s, int64_t t,
                               const irls_options *opt, void *hip_stream);

/* Run round 0 (or the chosen start) and rounds 1..T on the device.
 *   x0      n potentials (entries of s and t ignored) when init == 2, else NULL
 *   stats   NULL, or an array of T+1 records (host memory) filled on return
 * Returns IRLS_OK, IRLS_WARN_CG_MAXIT or an error. */
irls_status irls_mincut_solve(irls_mincut_t h, const double *x0, irls_round_stats *stats);

/* Run `rounds` reweighted rounds from a chosen start (checkpoint/resume, the
 * paper's warm start carried across calls, and sequences of related problems
 * in the spirit of Section 6):
 *   start 0: round 0 as the options say (init 0/1/2; x0 used for init 2)
 *   start 1: continue from the potentials the handle holds (after a solve or
 *            irls_mincut_set_potentials); no round-0 solve
 *   start 2: start from x0 (n doubles); no round-0 solve
 * Round l >= 1 uses eps_first * eps_factor^(l-1) (eps_first <= 0 with start 0:
 * the options' eps0).  stats: NULL or rounds+1 records (record 0 describes the
 * start).  Options stay as created. */
irls_status irls_mincut_solve_range(irls_mincut_t h, int32_t start, const double *x0,
                                    double eps_first, int32_t rounds, irls_round_stats *stats);

/* Sweep cut of the current potentials (Section 3.4): non-terminals in
 * descending potential, ties by ascending id; S_k = {s} + first k; the
 * smallest k with the least cut value wins.  Cut values are exact integer
 * sums of round-half-even(c * 2^k) at one 128-bit scale per graph; the value
 * returned is the exact minimum rounded once to double.
 *   in_source_side  NULL or n bytes (host): 1 for nodes in S (s included)
 *   cut_value       NULL or 1 double (host)
 *   k_star          NULL or 1 int64 (host): number of non-terminals in S */
irls_status irls_mincut_cut(irls_mincut_t h, uint8_t *in_source_side, double *cut_value,
                            int64_t *k_star);

/* irls_mincut_cut for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same sweep cut, bit for bit, with its work buffers (sort keys and ids,
 * ranks, 128-bit deltas, scan partials, the mask) carved from one static
 * device array of the library, which each GPU holds (about 12 MB) until the
 * process ends.  It calls no hipMalloc, hipFree or other allocating routine.
 * Graphs of up to IRLS_NOALLOC_MAX_NONTERMINAL non-terminal nodes; larger
 * ones get IRLS_ERR_OPTIONS.  Every call on one GPU uses that GPU's array,
 * whatever the handle or stream: calls that overlap on one GPU race, and the
 * caller must order them (each call returns after its stream has finished
 * with the array).  Arguments, results and other errors as irls_mincut_cut;
 * IRLS_ERR_DEVICE when the array's address cannot be obtained. */
#define IRLS_NOALLOC_MAX_NONTERMINAL 262144
irls_status irls_mincut_cut_noalloc(irls_mincut_t h, uint8_t *in_source_side, double *cut_value,
                                    int64_t *k_star);

/* Two-level rounding of the current potentials (Section 3.4, the two-level
 * rounding procedure, and its proposition):
 *   1. K-means with two centres on all n potentials (x_s = 1, x_t = 0
 *      included), started at 0.1 and 0.9: a value joins the upper cluster
 *      when it lies strictly above the midpoint of the centres, a centre is
 *      its cluster's mean (kept if the cluster is empty), and the iteration
 *      stops when an assignment repeats (at most 100 updates);
 *   2. gamma0 = c0 + 0.05, gamma1 = c1 - 0.05; S0 = {x <= gamma0} is
 *      coalesced with t, S1 = {x >= gamma1} with s, Sc is the rest;
 *   3. the coarse graph on {s_c, t_c} and Sc: edges inside Sc, {s_c, u} with
 *      u's summed capacity to S1, {t_c, u} to S0, {s_c, t_c} between S1 and
 *      S0, all as exact fixed-point sums (the sweep's scale);
 *   4. an exact minimum s_c-t_c cut of the coarse graph (on the host; its
 *      source side is the largest one: the nodes that cannot reach t_c in
 *      the residual graph of a maximum flow), lifted to S = S1 + its Sc part.
 * If some minimum cut of G keeps S1 on the source side and S0 on the sink
 * side, the result is a minimum cut of G.
 *   in_source_side  NULL or n bytes (host): 1 for nodes in S (s included)
 *   cut_value       NULL or 1 double (host): the exact cut value rounded once
 *   info            NULL or the centres, thresholds and coarse graph size
 * Errors: IRLS_ERR_NOT_SOLVED before a solve; IRLS_ERR_OPTIONS for a batch
 * handle; IRLS_ERR_RANGE if the potentials leave s or t out of S1 / S0
 * (potentials far outside [0, 1]). */
typedef struct {
  double  c0, c1;             /* K-means centres */
  double  gamma0, gamma1;     /* split thresholds */
  int32_t kmeans_updates;     /* centre updates before an assignment repeated */
  int64_t n_s0, n_s1, n_sc;   /* class sizes over all n nodes (t in S0, s in S1) */
  int64_t coarse_edges;       /* edges of the coarse graph (parallel edges merged) */
  double  coarse_value;       /* minimum cut value of the coarse graph (= cut_value) */
} irls_two_level_info;

irls_status irls_mincut_cut_two_level(irls_mincut_t h, uint8_t *in_source_side, double *cut_value,
                                      irls_two_level_info *info);

/* New capacities for the graph of a single-graph handle, for sequences of
 * related min-cut problems (the paper's stated application and future work,
 * Section 6: FlowImprove and graph-cut loops).  The edge list follows
 * irls_mincut_create's rules and must merge to the handle's structure (the
 * same nodes, s, t and neighbour pairs); only capacities change.  The
 * potentials are kept: irls_mincut_solve_range with start 1 continues from
 * them, irls_mincut_solve starts over per the options.  Arrays are read
 * during the call (device arrays when inputs_on_device).
 * Errors: as irls_mincut_create for the arrays; IRLS_ERR_OPTIONS when the
 * structure differs or for a batch handle. */
irls_status irls_mincut_update_capacities(irls_mincut_t h, int64_t m, const int64_t *edge_u,
                                          const int64_t *edge_v, const double *cap);

/* Cheeger-type bracket of the minimum cut value (Section 2.3, the
 * Cheeger-type inequality phi^2/2 <= lambda_2 <= 2 phi of the pencil (L, D)
 * with D = C at s and t).  With C = 2 * (sum of all capacities) and E01 the
 * energy x^T L x of round 0 (W = C, x_s = 1, x_t = 0), lambda_2 = 2 E01 / C
 * and phi = mu* / C, so
 *   E01 <= mu* <= 2 sqrt(C E01):  *lower = E01, *upper = 2 sqrt(C E01).
 * E01 comes from the round-0 CG solve (to cg_rtol) of the last
 * irls_mincut_solve (or solve_range with start 0) with init == 0; it depends
 * on the graph only, so it stays valid until irls_mincut_update_capacities.
 * Errors: IRLS_ERR_NOT_SOLVED without such a solve; IRLS_ERR_OPTIONS for a
 * batch handle. */
irls_status irls_mincut_cheeger_bracket(irls_mincut_t h, double *lower, double *upper);

/* Copy the current potentials (host; x_s = 1, x_t = 0): n doubles, or for a
 * batch handle sum(n_g) doubles laid out like node_off. */
irls_status irls_mincut_potentials(irls_mincut_t h, double *x);

/* Replace the current potentials (n doubles, host or device per
 * inputs_on_device; s and t entries ignored) and mark the handle solved, so
 * that irls_mincut_cut rounds them and a later solve with init == 2 may
 * resume from them.  Non-finite entries give IRLS_ERR_RANGE. */
irls_status irls_mincut_set_potentials(irls_mincut_t h, const double *x);

/* Sizes chosen at creation: non-terminal count, stored off-diagonal entries,
 * storage format (1 CSR, 2 diagonal), number of diagonals, solver (1 or 2),
 * CSR rows per wavefront. */
irls_status irls_mincut_info(irls_mincut_t h, int64_t *n_nonterminal, int64_t *nnz_offdiag,
                             int32_t *format, int32_t *n_diagonals, int32_t *solver,
                             int32_t *rows_per_wave);

/* The SpMV kernel the CG loop of a multi-workgroup handle launches and its
 * workgroup count.  variant: 0 CSR (rows_per_wave rows per wavefront),
 * 1 diagonal format with a row per thread, 2 diagonal with 16-byte row
 * vectors, 3 diagonal marching along the largest offset (the plane of a 3-D
 * grid, the row of a 2-D one), 4 the marching kernel on the symmetrically
 * scaled system (no diagonal read; see unscaled_cg).  IRLS_ERR_OPTIONS for
 * the resident solver or a batch. */
irls_status irls_mincut_spmv_kernel(irls_mincut_t h, int32_t *variant, int32_t *grid);

/* Tile shape of the marching SpMV (variant 3 or 4 above; Section 3.1's PCG
 * product on grids).  A workgroup of `threads` threads (256 or 512) owns a
 * tile of one plane and walks a chunk of planes:
 *   lines 0:   `threads` consecutive groups of rows of the plane (any grid);
 *   lines >= 1 (3-D grids): that many consecutive grid lines (offset off[1])
 *              by threads / lines row groups of each line.
 * The tile's two boundary lines are re-read by the neighbouring tiles, so
 * taller tiles move fewer bytes.  threads = lines = 0 restores the default
 * (256, 0).  The shape changes no result beyond the rounding order of the
 * SpMV's partial dot products.  Errors: IRLS_ERR_OPTIONS when the handle does
 * not march (batch, resident solver, CSR) or cannot take the shape (lines
 * must divide threads; a tile no wider or taller than a plane).
 * irls_mincut_march_tile reports the shape in use and the planes per
 * workgroup (all 0 without the marching SpMV); pointers may be NULL. */
irls_status irls_mincut_set_march_tile(irls_mincut_t h, int32_t threads, int32_t lines);
irls_status irls_mincut_march_tile(irls_mincut_t h, int32_t *threads, int32_t *lines, int32_t *planes);

/* Streaming ceiling of the GPU for a mix of memory streams: the bandwidth a
 * kernel that only reads `reads` arrays and writes `writes` arrays of `rows`
 * doubles each (two rows per thread, 16-byte accesses, rows in XCD slabs, no
 * other work) sustains, with plain accesses and with the streaming
 * (non-temporal) hint on every access; the faster of the two counts.  The CG kernels (Section 3.1's PCG: the SpMV streams
 * five arrays in and two out per row) are read against it.  Allocates
 * (reads + writes) * rows doubles on the current device for the call, runs
 * one warm-up and `reps` timed launches of each form on hip_stream (NULL:
 * the default stream) with `workgroups` workgroups, and writes the smaller
 * of the two mean launch times (ms).  Bytes moved per launch: (reads + writes) * rows * 8.
 * Errors: IRLS_ERR_OPTIONS unless rows is even and >= 2, reads in 1..6,
 * writes in 1..2, workgroups a multiple of 8 in 8..1024, reps in 1..1000;
 * IRLS_ERR_OOM / IRLS_ERR_DEVICE from HIP (text via
 * irls_mincut_last_error(NULL)). */
irls_status irls_stream_probe(int64_t rows, int32_t reads, int32_t writes, int32_t workgroups,
                              int32_t reps, void *hip_stream, double *avg_ms);

/* Time one hot kernel of the CG loop on the handle's stream with HIP events:
 * `which` 0 = SpMV (with its fused direction update), 1 = the CG vector
 * update of an odd iteration, 2 = of an even one (they differ only on the
 * scaled system, where the potentials move every second iteration: the odd
 * update adds both steps).  `reps` back-to-back launches after one warm-up launch; *avg_ms is
 * the mean duration.  Needs a prior solve; overwrites the CG work vectors
 * (p, q; potentials untouched) -- call solve again before resuming. */
irls_status irls_mincut_time_kernel(irls_mincut_t h, int32_t which, int32_t reps,
                                    double *avg_ms);

/* In-solve timing of one kernel of the CG iteration (Section 3.1's PCG; the
 * SpMV is its dominant cost).  From this call on, every solve of the handle
 * brackets the launches of that kernel for CG iterations 0, every,
 * 2 * every, ... of each round with a HIP event pair on the handle's stream,
 * and the totals are reset:
 *   which  -1 off, 0 the SpMV (with its fused direction update), 1 the vector
 *          update, 2 the FP64 residual replacement of the precision form (with
 *          ILU(0) of 4x4x4 tiles, and the application to the new residual), 3 the
 *          block-Jacobi application z = M^-1 r (precond 1 or 2; with ILU(0) of
 *          4x4x4 tiles the application runs inside the vector update, so
 *          which = 1 times both and which = 3 is refused)
 *   every  >= 1: the sampling stride (each event pair adds a marker before and
 *          after its launch, a few microseconds; a stride keeps that small)
 * Needs a single-graph handle on the multi-workgroup solver (solver 1),
 * precision 1 for which = 2 and a block-Jacobi preconditioner for which = 3;
 * IRLS_ERR_OPTIONS otherwise.  The solve's results are unchanged. */
irls_status irls_mincut_set_kernel_timing(irls_mincut_t h, int32_t which, int32_t every);

/* Totals of the in-solve timing since irls_mincut_set_kernel_timing: the
 * summed duration (ms) and count of the timed launches that did work (in
 * each round, the launches of CG iterations below its converged count) and of
 * all timed launches (launches queued past convergence return at once).  Any
 * pointer may be NULL (host memory). */
irls_status irls_mincut_kernel_timing(irls_mincut_t h, double *ms_working, int64_t *n_working,
                                      double *ms_all, int64_t *n_all);

/* Free the handle and all its device memory (NULL is a no-op). */
void irls_mincut_destroy(irls_mincut_t h);

/* Text of the last error of h, or of the calling thread's last failed create
 * when h == NULL.  Valid until the next call on the same handle/thread. */
const char *irls_mincut_last_error(irls_mincut_t h);

/* ----------------------------------------------------------------------------
 * Batched form (the paper's setting of many related min-cut problems, Section
 * 6, run as independent instances): G graphs solved together in FP64, one
 * 1024-thread workgroup per graph running every round of its graph inside one
 * persistent kernel launch; workgroups take graphs from a queue, largest
 * first.  Each solve replays a HIP graph captured at the first solve (queue
 * reset + the persistent launch).  Options: precision 0, solver 0 or 2, init
 * 0 or 1.  G <= 65536; node ids local to each graph.
 *   node_off[G+1], edge_off[G+1]   graph g owns nodes node_off[g]..node_off[g+1]-1
 *                                   and edges edge_off[g]..edge_off[g+1]-1
 *   edge_u, edge_v                 LOCAL node ids (0..n_g-1) of each graph
 *   s[G], t[G]                     local source and sink of each graph
 * Each graph obeys the single-graph rules above. */
irls_status irls_mincut_create_batch(irls_mincut_t *out, int32_t G, const int64_t *node_off,
                                     const int64_t *edge_off, const int64_t *edge_u,
                                     const int64_t *edge_v, const double *cap,
                                     const int64_t *s, const int64_t *t,
                                     const irls_options *opt, void *hip_stream);

/* Solve every graph of a batch handle.  stats: NULL or G*(T+1) records,
 * graph-major (host). */
irls_status irls_mincut_solve_batch(irls_mincut_t h, irls_round_stats *stats);

/* Sweep cut of every graph: in_source_side NULL or sum(n_g) bytes laid out like
 * node_off; cut_values NULL or G doubles. */
irls_status irls_mincut_cut_batch(irls_mincut_t h, uint8_t *in_source_side, double *cut_values);

/* Rows per wavefront of the resident solver (a batch handle, or a single
 * graph with solver 2).  Not in the paper, which has no GPU kernels: a tuning
 * knob of how the solver's per-row sums and SpMV map rows to lanes.  Rows of
 * at most 128 entries are binned by length: bin b (0..5) holds rows of at
 * most 2^(b+1) entries (bin 5: 33 to 128).  lanes[b] lanes walk each row of
 * bin b, each lane taking every lanes[b]-th entry; 64 / lanes[b] rows share
 * a wavefront.  The default is lanes[b] = min(2^(b+1), 64), one entry per
 * lane (bin 5: two).  Longer rows are always cut into 64-entry chunks.
 * The lanes change the order of each row's summation, not the arithmetic:
 * results agree to rounding, and are bit-identical across runs for one table.
 *
 * irls_mincut_set_row_lanes sets the table:
 *   lanes   6 int32 (host): each a power of two from 1 to min(2^(b+1), 64).
 * irls_mincut_autotune measures it: one sweep of coordinate descent over the
 * bins that hold rows, each trying its default and a half, a quarter and an
 * eighth of it (not below 1), timing `reps` resident solves of rounds
 * 0..`rounds` per candidate (the minimum counts) with HIP events; a bin
 * changes only for a gain of at least 2 % over its current choice.  The
 * timing solves start as irls_mincut_solve would; the potentials in place
 * before the call are restored after it, so the handle's state is unchanged
 * but for the table.  The next solve runs (and a batch re-captures its HIP
 * graph) with the chosen table.
 *   rounds  0 .. the handle's rounds; reps 1 .. 100
 *   lanes   NULL or 6 int32 (host): the table chosen
 * For a single-graph handle on the multi-workgroup solver in the CSR format,
 * irls_mincut_autotune instead tunes that path's rows per wavefront (its
 * SpMV and per-round CSR kernels): it times 20 * reps SpMV launches
 * (irls_mincut_time_kernel, which 0) on the last solve's system at each of
 * 1, 2, 4, ..., 64 rows per wavefront, keeps the fastest (again by at least
 * 2 %), and writes lanes[0] = 64 / rows per wavefront, lanes[1..5] = 0.
 * On the marching SpMV (diagonal format) it tunes the tile shape the same
 * way over every shape irls_mincut_set_march_tile accepts here (256 or 512
 * threads; 0, 1, 2, 4, ..., 32 lines) and writes lanes[0] = threads,
 * lanes[1] = lines, lanes[2..5] = 0.  For both, rounds is ignored; a solved
 * handle is needed (else IRLS_ERR_NOT_SOLVED); a diagonal format without
 * the marching SpMV has nothing to tune (IRLS_ERR_OPTIONS).
 * Errors (all): IRLS_ERR_OPTIONS for a handle that does not use the
 * resident solver, the CSR format or the marching SpMV, or for values out of
 * range; autotune with init 2 before the potentials are set:
 * IRLS_ERR_NOT_SOLVED.  A device error during the timing solves leaves the
 * potentials undefined and the handle unsolved. */
irls_status irls_mincut_set_row_lanes(irls_mincut_t h, const int32_t *lanes);
irls_status irls_mincut_autotune(irls_mincut_t h, int32_t rounds, int32_t reps, int32_t *lanes);

#ifdef __cplusplus
}
#endif
#endif
