/*
 * ustd.h -- C ABI of the MI355X (gfx950) library for the uniform-spanning-tree (UST)
 * estimator of diag(L^+), the diagonal of the pseudoinverse of a graph Laplacian
 * (Angriman, Predari, van der Grinten, Meyerhenke, "Approximation of the Diagonal of a
 * Laplacian's Pseudoinverse for Complex Network Analysis", ESA 2020).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named d_* are DEVICE pointers (HIP global memory of the current device);
 *    the caller allocates and owns them.  Pointers without the prefix are host pointers.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All device
 *    work is enqueued on it in order; an entry point returns after enqueueing unless it
 *    says it synchronises (those that must read a scalar back, e.g. ecc to size tau,
 *    synchronise `stream` once per phase).
 *  - The library never allocates device memory: every call takes a caller-owned
 *    workspace of at least ustd_workspace_bytes() bytes (256-byte aligned), which it
 *    may overwrite freely.  Calls sharing one workspace must not overlap in time.
 *  - Graph input (Section "Problem Description and Notation"): simple, connected,
 *    undirected, CSR with row_ptr int64[n+1] (row_ptr[0] = 0, row_ptr[n] = nnz = 2m),
 *    col int32[nnz], every row strictly ascending, every edge present in both rows, no
 *    self-loops; unit weights, or conductances d_weight (Section "Generalizations").
 *    With `validate` set the library checks all of this on the device (weights too) and
 *    returns USTD_EGRAPH if it fails.
 *  - Return value: USTD_OK or an error code; ustd_last_error() gives a thread-local
 *    message.  No C++ exception crosses this boundary.
 *  - Determinism: for a fixed (graph, weights, pivot, seed, tree range) the sampled
 *    trees, the walk-step counts and the integer (or, weighted, fixed-point) flow counts
 *    are bit-identical across runs, batch sizes and devices, and equal those of the
 *    sequential definition (ascending Wilson start order, minimum-ID BFS parents,
 *    Philox4x32-10 walk words keyed by (seed; step/4, walk start, tree)).
 */
#ifndef USTD_H
#define USTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    USTD_OK = 0,
    USTD_EINVAL = 1,   /* bad argument (pivot out of range, eps <= 0, delta/kappa not in (0,1), ...) */
    USTD_EGRAPH = 2,   /* graph fails validation (asymmetric, self-loop, unsorted, disconnected) */
    USTD_ENOMEM = 3,   /* workspace smaller than ustd_workspace_bytes() */
    USTD_EHIP = 4,     /* a HIP runtime call failed */
    USTD_ENOTCONV = 5  /* the pivot-column solve ended above its residual target; outputs are still written */
};

enum {
    USTD_SOLVE_FP64 = 0,  /* FP64 Jacobi-preconditioned CG */
    USTD_SOLVE_MIXED = 1  /* FP32 Jacobi-PCG iterations, FP64 solution and reliable updates (true residuals) */
};

/* Where the pivot-column solve's iterations run.  Both engines run the same algorithm (Jacobi
 * PCG with reliable updates) and differ only in the order of their FP64 partial sums, so a
 * solve is bit-reproducible for a fixed engine. */
enum {
    USTD_ENGINE_AUTO = 0,      /* single calls: WORKGROUP up to 16384 vertices, else MULTI;
                                  ustd_batch_diag_lpinv: WORKGROUP for every member */
    USTD_ENGINE_WORKGROUP = 1, /* the whole solve in one workgroup, no host round trip (batches run
                                  all members' solves side by side in one launch) */
    USTD_ENGINE_MULTI = 2      /* eight kernels per iteration over the whole GPU, enqueued ahead of a
                                  device-side done flag */
};

/* How each tree is sampled.  Both draw uniform spanning trees rooted at the pivot; they consume
 * the random words differently, so the trees (and counts) of one seed differ between them.
 *  - PLAIN: Wilson's algorithm on G rooted at u, starts in ascending vertex order, the walk from
 *    s keyed by (step / 4, s, tree);
 *  - BLOCKS (engineering appendix, after Hayashi et al.): Wilson's algorithm in each biconnected
 *    component B of G, rooted at B's vertex of largest degree inside B (smallest ID on ties),
 *    starts in ascending vertex order, the walk confined to B's edges and keyed by
 *    (step / 4, e(v, B), tree) with e(v, B) the CSR position of v's first edge inside B; the
 *    block trees are re-rooted at each block's vertex closest to u and joined.  Weighted
 *    problems and batches take PLAIN only. */
enum {
    USTD_WILSON_PLAIN = 0,
    USTD_WILSON_BLOCKS = 1
};

/* One problem instance: the inputs of ApproxDiagLpinv(G, u, eps, delta) (Algorithm 1)
 * plus the solver split kappa and the random seed. */
typedef struct ustd_problem {
    int64_t n;                /* vertices, 2 .. 2^30 (a connected graph with nnz < 2^31) */
    int64_t nnz;              /* row_ptr[n] = 2m; must be < 2^31 */
    const int64_t *d_row_ptr; /* device, n+1 */
    const int32_t *d_col;     /* device, nnz */
    int32_t pivot;            /* u in [0, n); -1 selects the maximum-degree vertex (smallest ID on ties);
                                 -2 the vertex with the smallest eccentricity lower bound after 10 BFS
                                 sweeps (engineering appendix): first source the maximum-degree vertex,
                                 each next one the farthest from the last, ties to the smallest ID */
    int32_t solve_mode;       /* USTD_SOLVE_FP64 or USTD_SOLVE_MIXED */
    double eps;               /* absolute error bound, > 0 */
    double delta;             /* failure probability in (0,1); <= 0 selects 1/n */
    double kappa;             /* error split between solve and sampling in (0,1); <= 0 selects 0.3 */
    uint64_t seed;            /* Philox key */
    int64_t tau_override;     /* > 0 replaces the sample-size formula */
    double solve_tol;         /* relative residual target; <= 0 selects min(eta, 1e-12) */
    int32_t solve_maxit;      /* iteration cap of the solve; <= 0 selects 20000 */
    int32_t validate;         /* 1 = validate the CSR on the device first */
    int32_t trees_per_batch;  /* trees resident in the workspace at once; <= 0 = automatic */
    int32_t tau_cap;          /* > 0: tau = min(formula, tau_cap) (ignored with tau_override) */
    /* Conductances (Section "Generalizations", weighted graphs): device double[nnz], w[e] > 0
     * and finite, equal at both entries of an edge; NULL = unit weights.  With weights:
     *  - a walk at x with word w32 moves to the first neighbour j (ascending adjacency) with
     *    t < C_x[j], where C_x[j] is the running sum of the row's conductances taken left to
     *    right in FP64 and t = (w32 * 2^-32) * C_x[deg-1]; trees are then drawn with
     *    probability proportional to the product of their conductances, and all-ones weights
     *    give the unweighted trees exactly;
     *  - Algorithm 2 counts the edge (parB(b), b) of P(v) as +-F[b] instead of +-1, with
     *    F[b] = llround(2^k / w(b, parB(b))) (the Ohm's-law factor in int64 fixed point);
     *    the counts R are then sum_T c_T(v) in units of 2^-k and diag[v] = R[v] / (tau 2^k)
     *    - x[u] + 2 x[v];
     *  - rho(v) = sum of 1/w over P(v)'s edges, added from v towards u; rho_max = max_v
     *    rho(v) replaces ecc(u) in the sample size: tau = ceil(rho_max^2 * ceil(ln(2m/delta)
     *    / (2 (1-kappa)^2 eps^2))) (then tau_cap / tau_override as above);
     *  - k = 62 - e, where tau * rho_max = f 2^e with f in [0.5, 1), so sums over up to 2 tau
     *    trees fit int64 (count calls on tree ranges use the problem's tau to fix k);
     *  - the pivot-column solve uses the weighted Laplacian (Jacobi on weighted degrees).
     * ustd_batch_diag_lpinv takes weighted and unweighted members together. */
    const double *d_weight;
    int32_t solve_engine;     /* USTD_ENGINE_AUTO, USTD_ENGINE_WORKGROUP or USTD_ENGINE_MULTI (below) */
    int32_t wilson_variant;   /* USTD_WILSON_PLAIN or USTD_WILSON_BLOCKS (below) */
} ustd_problem;

/* Filled by the calls that take it (nullable); times from HIP events on `stream`. */
typedef struct ustd_report {
    int64_t tau;          /* number of sampled trees */
    int64_t walk_steps;   /* steps of the sequential definition (equals the CPU oracle's) */
    int64_t walk_draws;   /* random-walk steps actually executed (includes speculative ones) */
    int32_t pivot;        /* pivot used */
    int32_t ecc;          /* eccentricity of the pivot */
    int32_t solve_iters;  /* total (inner) CG iterations */
    int32_t solve_outer;  /* FP64 refinement steps (mixed mode), 1 in FP64 mode */
    int32_t n_batches;    /* tree batches */
    int32_t trees_per_batch;
    double solve_relres;  /* ||b - L x||_2 / ||b||_2 of the returned column, in FP64 */
    /* phase times; ms_sample and ms_aggregate sum the launches of every tree batch, which on
     * graphs above 131072 vertices run on two streams at once (ms_total is wall time) */
    double ms_setup, ms_bfs, ms_sample, ms_intervals, ms_aggregate, ms_solve, ms_combine, ms_total;
    double rho_max;       /* largest B-path resistance (= ecc for unit weights) */
    int32_t fixed_shift;  /* k of the fixed-point counts of a weighted problem (0 unweighted) */
    int32_t weighted;     /* 1 if d_weight was given */
    /* eta = kappa eps / (3 sqrt(m n ln n) diam(G)) of Algorithm 1 (solver accuracy), with
     * diam(G) <= 2 ecc(u); natural log */
    double eta;
    double solve_tol;        /* relative residual target of the solve: prob->solve_tol, or min(eta, 1e-12) */
    int32_t solve_converged; /* 1 if solve_relres <= solve_tol (else the call returned USTD_ENOTCONV) */
    int32_t pad_;
} ustd_report;

/* Minimum workspace size for every call below on this problem (host only, no device work).
 * Depends on n, nnz and trees_per_batch. */
int ustd_workspace_bytes(const ustd_problem *prob, size_t *bytes);

/* BFS tree B_u of the pivot (Section "Effective Resistance Approximation by UST
 * Sampling": one shortest path P(v) per vertex, kept as parent pointers).  The parent of
 * v is the smallest-ID neighbour one level closer to u; d_parB[u] = -1.  d_dist (int32[n])
 * and d_parB (int32[n]) are nullable outputs; *ecc_out and *pivot_out are host outputs
 * (nullable).  Synchronises `stream`. */
int ustd_bfs(const ustd_problem *prob, void *d_ws, size_t ws_bytes, int32_t *d_dist,
             int32_t *d_parB, int32_t *ecc_out, int32_t *pivot_out, void *stream);

/* Sample trees tree_begin .. tree_begin+tree_count-1 with Wilson's algorithm rooted at the
 * pivot (Appendix "Wilson's UST Algorithm").  d_parents: int32[tree_count][n], row i is
 * the parent array of tree tree_begin+i (parent[u] = -1).  d_steps: int64[tree_count]
 * walk steps of each tree under the sequential definition (nullable).  tree_count <=
 * trees per batch of the workspace; with tree_count = 0 nothing is written (d_parents may
 * then be NULL).  Synchronises `stream` (pivot selection). */
int ustd_sample_trees(const ustd_problem *prob, int64_t tree_begin, int64_t tree_count,
                      void *d_ws, size_t ws_bytes, int32_t *d_parents, int64_t *d_steps,
                      void *stream);

/* Flow counts of trees tree_begin .. +tree_count-1 (Algorithm 2, summed over the trees; a
 * weighted problem takes at most 2 tau trees per call, else USTD_EINVAL):
 * d_counts[v] += sum_T c_T(v), where c_T(v) adds +1 for every edge (a,b) of P(v) that T
 * traverses from a to b on its path from u to v and -1 for every one it traverses from b
 * to a (Kirchhoff's theorem; Eq. N-values-in-path); for a weighted problem +-F[b] in fixed
 * point (see d_weight).  d_counts is int64[n], accumulated (the caller zeroes it).  Any
 * split of a tree range gives the same final counts.
 * rep (nullable) receives walk_steps/draws and phase times.  Synchronises `stream`. */
int ustd_flow_counts(const ustd_problem *prob, int64_t tree_begin, int64_t tree_count,
                     void *d_ws, size_t ws_bytes, int64_t *d_counts, ustd_report *rep,
                     void *stream);

/* Flow counts of caller-supplied spanning trees (Algorithm 2 only): d_parents is
 * int32[tree_count][n] of parent arrays rooted at the pivot (parent[u] = -1); d_counts
 * (int64[n]) is accumulated (fixed point for a weighted problem, k from the problem's
 * tau).  d_parents may be NULL when tree_count = 0.  A parent array that is not a spanning
 * tree rooted at the pivot (a parent out of range, a cycle, a vertex that does not reach the
 * pivot) returns USTD_EINVAL and leaves d_counts unchanged: every array is checked before
 * Algorithm 2 reads it, and the counts are added to d_counts only at the end.  A weighted
 * problem takes at most 2 tau trees per call (the fixed-point range), else USTD_EINVAL.
 * Synchronises `stream`. */
int ustd_tree_counts(const ustd_problem *prob, const int32_t *d_parents, int64_t tree_count,
                     void *d_ws, size_t ws_bytes, int64_t *d_counts, void *stream);

/* Column u of L^+ (Section "Overview", step 1): solves L x = e_u - (1/n) 1 with x
 * orthogonal to 1 to relative residual solve_tol (default min(eta, 1e-12), Algorithm 1's
 * solver accuracy), by FP64 Jacobi-PCG or by FP32 PCG with FP64 residuals and refinement
 * (solve_mode).  d_x is double[n].  Returns USTD_ENOTCONV (with d_x written and
 * rep->solve_converged = 0) whenever the final relative residual ||b - L x|| / ||b|| of the
 * projected solution exceeds the target.  Synchronises `stream`. */
int ustd_solve_pivot_column(const ustd_problem *prob, void *d_ws, size_t ws_bytes, double *d_x,
                            ustd_report *rep, void *stream);

/* ApproxDiagLpinv (Algorithm 1) end to end: BFS, tau, tau trees sampled and aggregated,
 * the pivot-column solve, and the combination of Eq. diag-comp,
 *   diag[u] = x[u],  diag[v] = R[v]/tau - x[u] + 2 x[v].
 * d_diag is double[n]; d_counts (int64[n], nullable) receives R (overwritten, not
 * accumulated; fixed point with shift rep->fixed_shift for a weighted problem).  The
 * pivot-column solve runs on a second stream of the library's own, during sampling.
 * Synchronises `stream`. */
int ustd_diag_lpinv(const ustd_problem *prob, void *d_ws, size_t ws_bytes, double *d_diag,
                    int64_t *d_counts, ustd_report *rep, void *stream);

/* ustd_diag_lpinv for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same computation,
 * with no workspace argument.  Its workspace is a 64 MiB array of device memory inside the
 * library (USTD_NOALLOC_SCRATCH_BYTES), which every GPU the library runs on holds from the
 * library's load until the process ends; the call allocates nothing (no hipMalloc or
 * hipFree, no HIP streams or events, no pinned host memory).  It runs every phase on
 * `stream` (no side stream), solves with the one-workgroup engine, and takes as many trees
 * per batch as fit the array (prob->trees_per_batch > 0 must fit as given).  A problem whose
 * workspace does not fit even at one tree per batch returns USTD_ENOMEM.  Counts, walk
 * steps and the diagonal equal those of ustd_diag_lpinv with solve_engine =
 * USTD_ENGINE_WORKGROUP; rep->trees_per_batch gives the batch size used; phase times are
 * not measured (0).  Every call on a GPU shares that GPU's array: calls that overlap in time
 * on one GPU race and must not be made (the array is re-initialised by each call).
 * Synchronises `stream`. */
#define USTD_NOALLOC_SCRATCH_BYTES (64u << 20)
int ustd_diag_lpinv_noalloc(const ustd_problem *prob, double *d_diag, int64_t *d_counts, ustd_report *rep,
                            void *stream);

/* Workspace size for ustd_batch_diag_lpinv over probs[0 .. count-1] (host only). */
int ustd_batch_workspace_bytes(const ustd_problem *probs, int32_t count, size_t *bytes);

/* ApproxDiagLpinv (Algorithm 1) for `count` independent problems (different graphs,
 * pivots, seeds, tau_cap ...) in one call.  d_diags: host array of `count` device
 * pointers, d_diags[i] double[n_i].  d_counts: nullable host array of nullable device
 * pointers (int64[n_i], overwritten with R of problem i).  reps: nullable, `count`
 * entries; ms_sample, ms_aggregate and ms_total there are those of the whole batch
 * (members share launches), the other fields are per member.  FP64 members of up to 16384
 * vertices solve side by side in one launch (a workgroup each); each reports an equal share of
 * that launch's time as ms_solve.  Each member's trees,
 * counts and diagonal are bit-identical to those of ustd_diag_lpinv on that problem alone.
 * The members' trees share one pool of records in the workspace and are sampled by
 * persistent launches that take (member, tree) tiles, larger graphs first.
 * A member's trees_per_batch (> 0) bounds its trees per pool fill.  A member error returns its code with "problem i: ..." in
 * ustd_last_error(); USTD_ENOTCONV of a member solve is returned after all members are
 * written.  Synchronises `stream`. */
int ustd_batch_diag_lpinv(const ustd_problem *probs, int32_t count, void *d_ws, size_t ws_bytes,
                          double *const *d_diags, int64_t *const *d_counts, ustd_report *reps,
                          void *stream);

/* ---- planned batches: set up once, execute many times, capture in a HIP graph ----
 *
 * ustd_batch_diag_lpinv above runs a plan once.  A plan splits the call in two: creation does
 * everything that needs the host (argument and graph checks, pivots, the BFS trees' depths and
 * so tau, the schedule of (member, tree) tiles over pool fills), and execution only enqueues
 * kernels on the stream and the library's side streams: no host wait, copy or memory set, so
 * an execution can be captured in a HIP graph and replayed.  Every execution recomputes the
 * whole estimator from the graphs (CSR views, BFS trees, sampling, Algorithm 2, solves,
 * combination) and gives results bit-identical to ustd_batch_diag_lpinv and to single calls;
 * the graphs' CSR arrays (and weights) must not change while the plan lives.  Trees are keyed
 * by (seed, tree, start), so no schedule changes any result. */

/* Schedule of a planned batch's launches (zero-initialised = the defaults). */
typedef struct {
    int32_t group_fills;  /* sampler group (one persistent launch) of about this many GPU-fills of trees
                             (resident sampler waves); 0 = 2; -1 = the whole pool fill in one launch */
    int32_t agg_chunk;    /* trees per Algorithm 2 thread, walked in lockstep: 0 = by eccentricity (4 from
                             ecc 8 on, else 8), or 4 or 8 */
    int32_t layout;       /* USTD_LAYOUT_AUTO or USTD_LAYOUT_RECORDS (below) */
    int32_t branches;     /* 0 or 1: sampler groups alternate between two streams and Algorithm 2 runs on a
                             third; 2 .. 4: the members are split into this many independent chains (by
                             estimated work), each one persistent sampler launch on its share of the
                             GPU's resident waves followed by its Algorithm 2 on the same stream
                             (group_fills is then unused) */
    int64_t fill_trees;   /* trees resident at once (one pool fill) at most; 0 = as many as the
                             workspace's record pool holds, up to 2^20 */
} ustd_batch_schedule;

enum {
    USTD_LAYOUT_AUTO = 0,    /* sampler tree state in an LDS bitmap when every member fits it */
    USTD_LAYOUT_RECORDS = 1  /* tree state in the tree records and per-edge entries, for every member */
};

typedef struct ustd_batch_plan ustd_batch_plan; /* opaque */

/* Creates a plan for probs[0 .. count-1] on the workspace d_ws (ustd_batch_workspace_bytes
 * bytes, kept by the plan until it is destroyed) with schedule `sched` (nullable: defaults).
 * Runs the members' set-up on `stream` (synchronises it) and allocates the plan's own device
 * memory for the tile schedule (24 bytes per tree plus a few hundred bytes per member).  The
 * problems are copied; their device arrays must stay valid.  Errors as ustd_batch_diag_lpinv
 * ("problem i: ..."); *plan is NULL on error. */
int ustd_batch_plan_create(const ustd_problem *probs, int32_t count, void *d_ws, size_t ws_bytes,
                           const ustd_batch_schedule *sched, ustd_batch_plan **plan, void *stream);

/* Enqueues one execution of the plan on `stream`: diag of member i into d_diags[i]
 * (double[n_i]); d_counts as in ustd_batch_diag_lpinv.  Returns without waiting.  Executions of
 * one plan must not overlap (they share the workspace).  When `stream` is capturing, phase
 * timers are left out and members that asked for USTD_ENGINE_MULTI are refused (that engine
 * is driven from the host); otherwise ustd_batch_plan_reports gives the phase times. */
int ustd_batch_plan_execute(ustd_batch_plan *plan, double *const *d_diags, int64_t *const *d_counts,
                            void *stream);

/* Per-member reports of the plan's last execution (or graph launch): synchronises `stream`
 * (the one it ran on) and reads walk totals and solve results from the device; ms_sample,
 * ms_aggregate, ms_solve, ms_combine and ms_total are those of the last eager execution (0
 * after a graph launch), ms_bfs is the set-up at creation.  `reps`: `count` entries.
 * Returns USTD_ENOTCONV (after filling every report) when a member's solve ended above its
 * target. */
int ustd_batch_plan_reports(ustd_batch_plan *plan, ustd_report *reps, void *stream);

/* The schedule a plan runs with (defaults filled in). */
int ustd_batch_plan_schedule(const ustd_batch_plan *plan, ustd_batch_schedule *out);

/* Frees the plan's device memory (synchronises the device).  USTD_EINVAL (nothing freed) while a
 * graph captured from the plan is alive: destroy the graphs first. */
int ustd_batch_plan_destroy(ustd_batch_plan *plan);

/* Captures one execution of the plan (ustd_batch_plan_execute with these outputs) into an
 * instantiated HIP graph; *graph = an opaque handle.  Capture runs on a stream of the library's.
 * The graph uses the plan's device memory, the workspace and the outputs, which must outlive
 * it.  USTD_EINVAL when a member uses USTD_ENGINE_MULTI. */
int ustd_batch_graph_create(ustd_batch_plan *plan, double *const *d_diags, int64_t *const *d_counts, void **graph);
/* Launches a captured execution on `stream` (returns without waiting).  Launches of graphs of
 * one plan, and its executions, must not overlap. */
int ustd_batch_graph_launch(void *graph, void *stream);
/* Destroys a captured graph (synchronises the device). */
int ustd_batch_graph_destroy(void *graph);

/* Autotuner of a batch's schedule (dynamic load balancing, parallel implementation appendix):
 * times executions of plans over branches {alternating groups, 2, 3, 4 chains}, group_fills
 * {1, 2, 4, whole fill}, agg_chunk {by eccentricity, 4, 8}, layout {auto, records} and fill_trees
 * {all, half}, one dimension at a time from the defaults, and returns the fastest in *best (its
 * time per execution in *best_ms, nullable).  graph != 0 times replays of each plan's captured
 * HIP graph (the way a repeated batch runs), else eager executions.
 * cache_path (nullable: the environment variable USTD_TUNE_CACHE, none when unset) names a JSON
 * file of tuned schedules keyed by the batch's shape (members' n, nnz, tau, eccentricity,
 * weightedness), the timing mode and the device (architecture, compute units): a hit returns the stored
 * schedule without timing (*from_cache = 1, nullable), a miss adds the result to the file.
 * Synchronises `stream`; the workspace as for ustd_batch_plan_create. */
int ustd_batch_autotune(const ustd_problem *probs, int32_t count, void *d_ws, size_t ws_bytes,
                        const char *cache_path, int32_t graph, ustd_batch_schedule *best, double *best_ms,
                        int32_t *from_cache, void *stream);

/* Spanning-edge counts (Kirchhoff index appendix: counting, for each edge, the sampled USTs
 * it appears in; count / #trees estimates the edge's effective resistance r(e), which is
 * also the probability that a uniform spanning tree contains e).  Trees tree_begin ..
 * +tree_count-1 are the ones ustd_sample_trees returns.  For each tree and each v != u the
 * edge {v, parent_T(v)} adds 1 at the CSR position of the entry (a, b), a = min and b = max
 * of its endpoints (row a); entries with a > b end at 0 (a value there is moved to the
 * entry (b, a)).  d_counts is int64[nnz], accumulated (the caller zeroes it); any split of a
 * tree range gives the same counts.
 * rep (nullable): walk steps/draws and times (the counting in ms_aggregate).  Synchronises
 * `stream`. */
int ustd_edge_counts(const ustd_problem *prob, int64_t tree_begin, int64_t tree_count,
                     void *d_ws, size_t ws_bytes, int64_t *d_counts, ustd_report *rep, void *stream);

/* Number of trees for every edge's effective resistance within +-eps with probability
 * 1 - delta (Kirchhoff index appendix, after Hayashi et al.): *q = ceil(2 eps^-2 ln(2m/delta)),
 * delta <= 0 selecting 1/n.  Host only. */
int ustd_edge_sample_size(int64_t n, int64_t m, double eps, double delta, int64_t *q);

/* Edge measures from spanning-edge counts (Kirchhoff index appendix, denominator of the
 * Sherman-Morrison form of the Kirchhoff edge centrality C^Delta_theta(e)): with
 * lev(e) = c(e) / q, the fraction of the q sampled trees that contain e (an estimate of the
 * leverage w(e) r(e), the probability that a tree drawn with probability proportional to its
 * weight contains e), d_r[e] = lev(e) / w(e) estimates the effective resistance r(e) and
 * d_denom[e] = 1 - (1 - theta) lev(e) the denominator 1 - (1 - theta) w(e) r(e), both in FP64
 * in that order of operations.  d_counts is the int64[nnz] output of ustd_edge_counts
 * (counts at the entries (a, b), a < b); both outputs (double[nnz], nullable) get the edge's
 * value at both of its entries.  d_row_ptr int64[n+1], d_col int32[nnz] as in ustd_problem,
 * d_weight nullable (unit weights).  q >= 1; theta in (0, 1).  Enqueued on `stream`; does not
 * synchronise. */
int ustd_edge_resistances(int64_t n, int64_t nnz, const int64_t *d_row_ptr, const int32_t *d_col,
                          const double *d_weight, const int64_t *d_counts, int64_t q, double theta, double *d_r,
                          double *d_denom, void *stream);

/* Vertex measures that depend only on the diagonal d = diag(L^+) (section on electrical
 * closeness, Eq. elec-farness; Lemma on normalized random-walk betweenness; Kirchhoff
 * index appendix): tr = sum_v d[v]; farness[v] = n d[v] + tr; closeness[v] = (n-1) /
 * farness[v]; nrwb[v] = 1/n + tr / ((n-1) farness[v]); Kirchhoff index n tr.  d_diag
 * double[n] (device, e.g. from ustd_diag_lpinv); d_farness, d_closeness, d_nrwb double[n]
 * (device, nullable); d_scalars double[2] (device) receives {tr, Kirchhoff index}.  The
 * trace is summed in a fixed order.  Enqueued on `stream`; does not synchronise. */
int ustd_centralities(int64_t n, const double *d_diag, double *d_farness, double *d_closeness,
                      double *d_nrwb, double *d_scalars, void *stream);

/* Test hook for the walk generator: d_out[i] = word ((k0+i) mod 4) of Philox4x32-10 with
 * key (seed lo, seed hi) and counter ((k0+i)/4, s, t lo, t hi), i < count; uint32[count]. */
int ustd_philox_words(uint64_t seed, int64_t t, int32_t s, int64_t k0, int64_t count,
                      uint32_t *d_out, void *stream);

/* Static name of a status code. */
const char *ustd_status_string(int status);

/* Detail of the last error raised on the calling thread ("" if none). */
const char *ustd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* USTD_H */
