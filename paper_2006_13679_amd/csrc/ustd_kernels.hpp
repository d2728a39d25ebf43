// ustd_kernels.hpp -- argument blocks and launchers of the gfx950 kernels (library-internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ustd_device.hpp"

namespace ustd {

// instantiate a launch for the row-group size G (lanes per light row) of a graph
#define USTD_DISPATCH_G(G, ...)                            \
    switch (G) {                                           \
        case 4: { constexpr int GG = 4; __VA_ARGS__; break; }   \
        case 8: { constexpr int GG = 8; __VA_ARGS__; break; }   \
        case 16: { constexpr int GG = 16; __VA_ARGS__; break; } \
        default: { constexpr int GG = 32; __VA_ARGS__; break; } \
    }


// One graph as the sampler sees it (read-only while sampling).
struct WilsonGraph {
    int n, u, nwords, rob;
    const int *rp;
    const void *colv;       // column indices: int32, or uint16 when the launch says so
    const int *bflag;       // [n] (parB + 1) | (internal in B_u) << 31
    // graphs whose tree state is in global memory (past the LDS bitmap):
    const int4 *vrow;       // [n] {rp[v], rp[v+1], bflag[v], 0}
    const int4 *edge;       // [nnz] entry (x, y): {y, rp[y], rp[y+1], bflag[y]}: a walk step's loads
    const double *cw;       // [nnz] running conductance sums of each row (weighted launches)
    const int *guide;       // [nnz] start of the weighted step search per (row, bucket)
    uint32_t key0, key1;    // Philox key (seed)
};

// One unit of sampler work in a batched launch: tree `tree` of graph `graph`, whose
// records go to rec + rec_off.
struct WilsonTile {
    long long tree, rec_off;
    int graph, pad;
};

// Persistent sampler launch: every block repeatedly takes the next tile index from
// *queue until all `ntiles` are taken.  Tile i is tree tree_begin + i of `g` with
// records at rec + i * rec_stride, or tiles[i] of the graph table when `tiles` is set.
struct WilsonArgs {
    WilsonGraph g;
    const WilsonGraph *graphs;  // batched launches: graph table (device)
    const WilsonTile *tiles;    // batched launches: tile table (device); null = single graph
    int ntiles;
    long long tree_begin;
    int2 *rec;                  // records {parent_T, nba | marked << 31}
    long long rec_stride;
    int *path;                  // [blocks][kSamplerPathSlot] recorded steps beyond the LDS part
    int *queue;                 // tile counter, zero at launch
    long long *steps;           // [ntiles], nullable
    long long *draws;           // [ntiles], nullable
    // single-graph launches on the block-split graph (Wilson per biconnected component): every
    // block's root starts in the tree (roots[0..nroots), in place of the single root g.u), and
    // the walk from s is keyed by skey[s] in place of s
    const int *roots;
    const int *skey;
    int nroots;
};

struct IntervalArgs {
    int n, u;
    const int *par;         // [ntrees][par_stride]
    long long par_stride;
    int *scratch;           // [ntrees][scratch_stride], scratch_stride >= 7n + 3
    long long scratch_stride;
    int2 *rec;              // [ntrees][rec_stride] {parent, nba | flags} records out
    long long rec_stride;
    const int *bflag;       // [n] B_u flag words
    int *err;
};

// trees one aggregation thread walks together: 8, or 4 where the marked-ancestor chains are
// long (fewer registers, more threads to cover the chain loads)
constexpr int kAggChunk = 8;
constexpr int kAggChunkLarge = 4;

struct AggregateArgs {
    int n, u, ntrees;
    const int *parB;        // [n] B_u parents
    const int2 *bint;       // [n] {pre_B, size_B} subtree intervals of B_u
    const int2 *rec;
    long long rec_stride;
    long long *counts;
    const long long *F;     // [n] fixed-point 1/w of each vertex's B_u edge; null = unit weights
    int chunk;              // trees per thread: kAggChunk or kAggChunkLarge (0 = kAggChunk)
};

struct EdgeCountArgs {
    int n, u, ntrees, trees_per_chunk;
    const int *rp, *col;        // int32 row pointers, ascending rows
    const int2 *rec;            // [ntrees][rec_stride] tree records
    long long rec_stride;
    long long *counts;          // [nnz], accumulated
};

constexpr int kSamplerRobMax = 128;      // reorder-buffer entries of the sampler (tree state in the records)
constexpr int kSamplerRobLds = 64;       // reorder-buffer entries with the tree bitmap in LDS
constexpr int kSamplerPathGlobal = 250;  // recorded steps per entry kept in global memory
constexpr long long kSamplerPathSlot = (long long)kSamplerRobMax * kSamplerPathGlobal;  // ints per block
constexpr int kSamplerMaxBlocks = 8192;  // resident sampler blocks (path slots)
constexpr int kMaxSolveGrid = 8192;  // blocks of the solve's row and vector kernels

// degree-balanced row mapping (see the BFS / SpMV kernels)
struct RowMap {
    const int *rp, *col;
    int n;
    int heavy_thresh;
    const int *heavy;   // ascending IDs of rows with degree > heavy_thresh
    const int *nheavy;  // device count
    const double *w;    // [nnz] conductances; null = unit weights
    const double *wdeg; // [n] conductance sum of each row (with w)
};

// Scalars of one pivot-column solve on the device: preconditioned CG with reliable updates.
// The solution x is kept in FP64; the iteration runs on vectors of type T (FP64, or FP32 in
// the mixed mode) holding the correction xs since the last reliable update and the iterated
// residual rs.  A reliable update folds xs into x and replaces rs by the true FP64 residual
// b - L x; it is taken when |rs|^2 drops below delta2 times the largest |r|^2 since the
// last one, when |rs|^2 reaches the target, or at the iteration cap.  The solve ends at an
// update whose true residual meets the target (or at the cap, or on stagnation).
struct SolveScalars {
    double rz;       // z.r of the iterated residual
    double alpha, beta;
    double rr;       // |rs|^2
    double rr_max;   // largest |r|^2 since the last reliable update
    double rr_true;  // |b - L x|^2 at the last reliable update
    double bb;       // |b|^2
    double tol2;     // target |b - L x|^2 <= tol2 bb
    double delta2;
    int iter, maxit;
    int done;        // later kernels of the solve are no-ops
    int upd;         // a reliable update is due in this iteration
    int updates;     // reliable updates taken
    int stalls;      // consecutive updates whose true residual fell by less than 2x
    int broke;       // p.q was not positive (breakdown): the next update ends the solve
};

template <typename T>
struct SolveArgs {
    int n, u;
    double *x;                // FP64 solution (the pivot column)
    T *xs, *rs, *z, *p, *q;   // correction, iterated residual, preconditioned residual, direction, L p
    double *part;             // per-block partials, 6 * kMaxSolveGrid
    int grid_spmv, grid_vec;
    SolveScalars *sc;
    const int *rp;            // row pointers (degrees as the Jacobi diagonal)
    const double *wdeg;       // Jacobi diagonal of a weighted Laplacian; null = degrees
};

// One pivot-column solve of a batched one-workgroup launch: right-hand side e_u - 1/n.
template <typename T>
struct SolveJob {
    SolveArgs<T> a;
    RowMap m;
    double tol2, delta2;
    int maxit;
};

inline long long interval_scratch_ints(long long n) { return 7 * n + 3; }

hipError_t launch_rp_to_i32(int n, const long long *rp64, int *rp32, hipStream_t st);
hipError_t launch_validate(int n, long long nnz, const long long *rp64, const int *col, int *err, hipStream_t st);
hipError_t launch_argmax_degree(int n, const int *rp, unsigned long long *best, hipStream_t st);
hipError_t launch_bfs_init(int n, int u, int *dist, int *parB, hipStream_t st);
hipError_t launch_sweep_update(int n, const int *dist, int *bound, int first, unsigned long long *far, hipStream_t st);
hipError_t launch_argmin_bound(int n, const int *bound, unsigned long long *best, hipStream_t st);
// the whole sweep-pivot choice in one workgroup (n <= kSmallSolveMaxN); *pivot = the pivot
hipError_t launch_sweep_small(const RowMap &m, int G, int sweeps, int *dist, int *bound, int *pivot, hipStream_t st);
// one BFS level; with prev (the previous level's found flag) set, it returns at once if that is 0
hipError_t launch_bfs_level(const RowMap &m, int G, int d, int *dist, int *parB, int *found, const int *prev,
                            hipStream_t st);
hipError_t launch_heavy_list(int n, const int *rp, int thresh, int *bcount, int *heavy, int *nheavy, hipStream_t st);
int solve_grid(const RowMap &m, int G);
int vec_grid(int n);
hipError_t launch_count_unreached(int n, const int *dist, int *err, hipStream_t st);
// resident blocks of one sampler launch on the current device (occupancy x compute units)
int wilson_resident_blocks(bool lds_bits, bool col16, bool weighted, int nwords, bool block_split = false);
// Small unweighted graphs (16-bit columns, LDS tree bitmap) may keep the graph in LDS as well:
// its bytes there (row pointers, B_u flags, columns), and the resident blocks of such a
// launch by the LDS residency measured on gfx950 (two 80 KB halves, 256-byte units).
long long wilson_graph_lds_bytes(int n, long long nnz);
int wilson_resident_blocks_graph_lds(int nwords, long long graph_bytes);
// graph_lds_bytes > 0 (single-graph launches only): the graph-in-LDS variant
// block_split: the block-split graph of the per-block variant (several roots, keyed starts)
hipError_t launch_wilson(const WilsonArgs &a, int blocks, bool lds_bits, bool col16, bool weighted, int nwords,
                         hipStream_t st, long long graph_lds_bytes = 0, bool block_split = false);
// per-member walk totals of a batch: totals[2 g] += steps[i], totals[2 g + 1] += draws[i], g = tiles[i].graph
hipError_t launch_tile_walks(int cnt, const WilsonTile *tiles, const long long *steps, const long long *draws,
                             unsigned long long *totals, hipStream_t st);
// weighted graphs: running row sums and row totals; weight checks; B_u edge conductances,
// B-path resistances (max into *rmax_bits, as the bits of a non-negative double); F
hipError_t launch_sum_walks(int cnt, const long long *steps, const long long *draws, unsigned long long *totals,
                            hipStream_t st);
hipError_t launch_row_cumsum(int n, int nnz, const int *rp, const double *w, int heavy_thresh, const int *heavy,
                             const int *nheavy, double *cw, double *wdeg, int *guide, hipStream_t st);
hipError_t launch_check_weights(int n, const int *rp, const int *col, const double *w, int *err, hipStream_t st);
hipError_t launch_vertex_rows(int n, const int *rp, const int *bflag, int4 *vrow, hipStream_t st);
hipError_t launch_edge_rows(long long nnz, const int *col, const int4 *vrow, int4 *edge, hipStream_t st);
hipError_t launch_bpath(int n, int u, const int *rp, const int *col, const double *w, const int *parB, double *wB,
                        unsigned long long *rmax_bits, hipStream_t st);
hipError_t launch_fixed_weights(int n, int u, const double *wB, int shift, long long *F, hipStream_t st);
hipError_t launch_col_to_u16(long long nnz, const int *col, unsigned short *col16, hipStream_t st);
hipError_t launch_tree_records(const IntervalArgs &a, int ntrees, hipStream_t st);
hipError_t launch_aggregate(const AggregateArgs &a, hipStream_t st);
hipError_t launch_extract_parents(int n, int ntrees, const int2 *rec, long long rec_stride, int *out, hipStream_t st);
hipError_t launch_centralities(long long n, const double *diag, double *farness, double *closeness, double *nrwb,
                               double *scalars, hipStream_t st);
hipError_t launch_edge_counts(const EdgeCountArgs &a, hipStream_t st);
hipError_t launch_edge_fold(int n, long long nnz, const int *rp, const int *col, long long *counts, hipStream_t st);
// BFS tree, connectivity check and B_u intervals of a small graph (n <= kSmallSolveMaxN) in
// one workgroup; out[0] = ecc, out[1] = 1 if a vertex is unreached; scratch holds 3n ints
hipError_t launch_setup_small(const RowMap &m, int G, int u, int *dist, int *parB, int *scratch, int2 *bint,
                              int *bflag, int *out, hipStream_t st);
hipError_t launch_b_intervals(int n, int u, int ecc, const int *dist, const int *parB, int *scratch, int2 *bint,
                              int *bflag, hipStream_t st);
// Pivot-column solve (SolveScalars): start (x = 0, r = b) and iterations of the multi-kernel
// engine; the whole solve in one workgroup (one-workgroup engine); many one-workgroup solves in
// one launch (one workgroup each).
constexpr int kSmallSolveMaxN = 16384;
template <typename T>
hipError_t launch_solve_start(const SolveArgs<T> &a, double tol2, double delta2, int maxit, hipStream_t st);
template <typename T>
hipError_t launch_solve_iteration(const SolveArgs<T> &a, const RowMap &m, int G, hipStream_t st);
template <typename T>
hipError_t launch_solve_small(const SolveArgs<T> &a, const RowMap &m, int G, double tol2, double delta2, int maxit,
                              hipStream_t st);
template <typename T>
hipError_t launch_solve_small_batch(const SolveJob<T> *jobs, int count, int G, hipStream_t st);
// res = b - L x (nullable), sums of [res, res^2, x] into out[0..3)
hipError_t launch_residual64(const RowMap &m, int G, int u, const double *x, double *res, double *part, double *out,
                             hipStream_t st);
// x -= mean_src[0] / n
hipError_t launch_project(int n, double *x, const double *mean_src, int grid, hipStream_t st);
// Wilson per biconnected component (ustd_blocks.hip): exclusive scan of int counts (out[n] =
// total, also written to *total; sums holds (n / 1024 + 2) ints); the blocks of G from B_u
// (lo, hi, uf: int[n]); per entry its block and the first entries of each (vertex, block);
// the slots of G*; G*'s columns; block roots and tops; and, per batch of trees, the join of the
// block trees (records of G* in recs) into records of spanning trees of G (rec)
hipError_t launch_scan_excl(const int *in, int *out, long long n, int *sums, int *total, hipStream_t st);
hipError_t launch_fill_i32(long long n, int *a, int v, hipStream_t st);
hipError_t launch_bc_blocks(const RowMap &m, int G, int u, int ecc, const int *dist, const int *parB,
                            const int2 *bint, int *lo, int *hi, int *uf, hipStream_t st);
hipError_t launch_bc_entries(int n, long long nnz, int u, const int *rp, const int *col, const int *parB,
                             const int2 *bint, const int *uf, int *eblk, int *firstPar, int *firstTop, int *flag,
                             hipStream_t st);
hipError_t launch_bc_slots(int n, long long nnz, int u, const int *rp, const int *flag, const int *sid,
                           const int *eblk, const int *uf, int *vtx, int *skey, int *sblk, int *slotPar, int *slotTop,
                           int *deg, hipStream_t st);
hipError_t launch_bc_columns(int n, int u, const int *rp, const int *col, const int *eblk, const int *uf,
                             const int *slotPar, const int *slotTop, const int *rps, int *cursor, int *cols,
                             hipStream_t st);
hipError_t launch_bc_roots(int nslots, const int *rps, const int *vtx, const int *sblk, unsigned long long *key,
                           int *flag, hipStream_t st);
hipError_t launch_bc_top_flags(int nslots, const int *sblk, const int *slotTop, int *flag, hipStream_t st);
hipError_t launch_bc_compact(int nslots, const int *flag, const int *pos, int *list, hipStream_t st);
hipError_t launch_bc_join(int n, int u, int ntrees, int ntop, int nslots, const int *tops, const int *slotPar,
                          const int *vtx, int2 *recs, long long sstride, int2 *rec, long long stride,
                          const int *bflag, hipStream_t st);
// a[0..n) = v; b[0..n) += a[0..n) (int64)
hipError_t launch_fill_i64(long long n, long long *a, long long v, hipStream_t st);
hipError_t launch_add_i64(long long n, const long long *a, long long *b, hipStream_t st);
hipError_t launch_edge_resistance(int n, long long nnz, const long long *rp, const int *col, const double *w,
                                  const long long *counts, double q, double theta, double *r, double *denom,
                                  hipStream_t st);
hipError_t launch_combine(int n, int u, double den, const long long *counts, const double *x, double *diag,
                          hipStream_t st);
hipError_t launch_philox_words(uint32_t key0, uint32_t key1, long long t, int s, long long k0, long long count,
                               uint32_t *out, hipStream_t st);

}  // namespace ustd
