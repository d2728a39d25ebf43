// ustd_api.hip -- C ABI (include/ustd.h): argument checks, workspace planning and the
// stream-ordered orchestration of the estimator's phases (Algorithm 1 of Angriman et
// al., ESA 2020: BFS tree and sample size, tau trees sampled and aggregated, the pivot
// column solve, and the final combination).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ustd.h"
#include "ustd_kernels.hpp"

using namespace ustd;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(...)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (__VA_ARGS__);                                                             \
        if (e_ != hipSuccess) return fail(USTD_EHIP, "%s: %s", #__VA_ARGS__, hipGetErrorString(e_)); \
    } while (0)

#define USTD_TRY(...)                   \
    do {                                \
        int rc_ = (__VA_ARGS__);        \
        if (rc_ != USTD_OK) return rc_; \
    } while (0)

constexpr long long kAlign = 256;
constexpr int kLdsBitsMaxWords = 4096;      // tree bitmap in LDS up to 131072 vertices (16 KB)
constexpr long long kGraphLdsMaxBytes = 40960;  // graph copy in the sampler's LDS (small graphs)
constexpr long long kDefaultBudget = 96ll << 30;  // tree records + sampler scratch, a third of 288 GB HBM
constexpr int kMaxTreesPerBatch = 8192;
constexpr long long kPoolMinTrees = 4096;  // a pool that fills the GPU's sampler slots
constexpr int kBatchGroupFills = 2;        // sampler group of a batch fill, in GPU-fills of trees
constexpr int kEdgeTreesPerChunk = 8;  // trees one edge-counting thread goes through

inline long long align_up(long long v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Misc {                      // small zero-initialised block at the front of the workspace
    int err_validate;
    int bfs_found[64];             // found flags of a group of queued BFS levels (kBfsGroupMax)
    int err_interval;
    int nheavy;
    int queue[2];                  // sampler tile counters, one per tree pool
    int setup_out[2];              // small-graph set-up: ecc, unreached flag
    int pad_[3];
    unsigned long long best_degree;
    unsigned long long rho_max_bits;  // weighted: the largest B-path resistance, as double bits
    unsigned long long walk_totals[2];  // walk steps and draws of a run of batches
    int nslots, nroots, ntops, scan_total;  // per-block variant: slots of G*, block roots and tops
    SolveScalars sc;
    double sums[4];
};

struct Plan {
    int n, nnz, K, Kiv, slots, pools, rob, nwords, G, heavy_thresh;
    bool lds_bits, col16, weighted;
    bool edges;  // edge entries for the sampler (tree state in global memory)
    long long rec_stride, scr_stride;
    long long off_misc, off_rp32, off_col16, off_dist, off_parB, off_bint, off_bflag, off_vrow, off_edge, off_heavy, off_bcount, off_counts, off_steps,
        off_draws, off_rec, off_path, off_scr, off_part, off_x64, off_r64, off_z64, off_p64, off_q64,
        off_res64, off_x32, off_r32, off_z32, off_p32, off_q32, off_cw, off_guide, off_wdeg, off_wB, off_F;
    // Wilson per biconnected component: the block-split graph G* (at most 2n slots) and its
    // sampler layout, decided for the upper bound of slots
    bool bv, s_lds, s_col16, s_edges;
    int s_nmax, s_nwords;
    long long s_rec_stride;
    long long off_bc_lo, off_bc_hi, off_uf, off_fpar, off_ftop, off_spar, off_stop, off_rkey, off_eblk, off_flag,
        off_sid, off_svtx, off_skey, off_sblk, off_sdeg, off_rps, off_cur, off_scol, off_scol16, off_sbflag,
        off_rflag, off_rpos, off_roots, off_tops, off_tiles, off_svrow, off_sedge, off_srec;
    long long total;
};

int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

int check_problem(const ustd_problem *p) {
    if (!p) return fail(USTD_EINVAL, "problem is NULL");
    if (p->n < 2 || p->n >= (1ll << 30) - 1) return fail(USTD_EINVAL, "n = %lld out of range [2, 2^30 - 1)", (long long)p->n);
    if (p->nnz < 2 || p->nnz >= (1ll << 31)) return fail(USTD_EINVAL, "nnz = %lld out of range [2, 2^31)", (long long)p->nnz);
    if (!p->d_row_ptr || !p->d_col) return fail(USTD_EINVAL, "row_ptr / col is NULL");
    if (p->pivot < -2 || p->pivot >= p->n) return fail(USTD_EINVAL, "pivot %d out of range", p->pivot);
    if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return fail(USTD_EINVAL, "eps must be > 0");
    if (p->delta > 0.0 && !(p->delta < 1.0)) return fail(USTD_EINVAL, "delta must lie in (0,1)");
    if (p->kappa > 0.0 && !(p->kappa < 1.0)) return fail(USTD_EINVAL, "kappa must lie in (0,1)");
    if (p->solve_mode != USTD_SOLVE_FP64 && p->solve_mode != USTD_SOLVE_MIXED)
        return fail(USTD_EINVAL, "unknown solve_mode %d", p->solve_mode);
    if (p->solve_engine < USTD_ENGINE_AUTO || p->solve_engine > USTD_ENGINE_MULTI)
        return fail(USTD_EINVAL, "unknown solve_engine %d", p->solve_engine);
    if (p->wilson_variant != USTD_WILSON_PLAIN && p->wilson_variant != USTD_WILSON_BLOCKS)
        return fail(USTD_EINVAL, "unknown wilson_variant %d", p->wilson_variant);
    if (p->wilson_variant == USTD_WILSON_BLOCKS && p->d_weight)
        return fail(USTD_EINVAL, "the per-block Wilson variant takes unit weights only");
    if (p->trees_per_batch > kMaxTreesPerBatch)
        return fail(USTD_EINVAL, "trees_per_batch %d exceeds %d", p->trees_per_batch, kMaxTreesPerBatch);
    return USTD_OK;
}

// Workspace layout of one problem.  Without trees (a batch member's own region) the tree
// records and sampler slots are left out: a batch keeps them in a shared pool.
Plan make_plan(const ustd_problem *p, bool with_trees = true, bool force_edges = false) {
    Plan L{};
    L.n = (int)p->n;
    L.nnz = (int)p->nnz;
    L.nwords = (L.n + 31) / 32;
    L.lds_bits = L.nwords <= kLdsBitsMaxWords;
    L.col16 = L.n <= 65536;  // 16-bit column copy for the sampler (half the cache footprint)
    L.edges = !L.lds_bits || force_edges;
    L.weighted = p->d_weight != nullptr;
    L.rob = std::min(L.lds_bits && !force_edges ? kSamplerRobLds : kSamplerRobMax, next_pow2(std::max(L.n, 2)));
    const double avg = (double)L.nnz / (double)L.n;
    L.G = avg <= 6.0 ? 4 : (avg <= 16.0 ? 8 : (avg <= 48.0 ? 16 : 32));
    L.heavy_thresh = 32 * L.G;
    L.rec_stride = align_up((long long)L.n * 8) / 8;  // int2 records
    L.scr_stride = align_up(interval_scratch_ints(L.n) * 4) / 4;
    // trees resident at once (records), and sampler blocks resident at once (scratch slots).
    // Graphs past the LDS bitmap run several batches.  When the budget holds two pools that
    // can each fill the GPU (kPoolMinTrees trees), they are sampled on two streams, so one
    // batch's tail and its Algorithm 2 overlap the next batch; smaller pools would leave
    // every batch short of the resident sampler slots, so the budget stays one pool.
    L.bv = p->wilson_variant == USTD_WILSON_BLOCKS;
    if (L.bv) {
        L.s_nmax = 2 * L.n;
        L.s_nwords = (L.s_nmax + 31) / 32;
        L.s_lds = L.s_nwords <= kLdsBitsMaxWords;
        L.s_col16 = L.s_nmax <= 65536;
        L.s_edges = !L.s_lds;
        L.s_rec_stride = align_up((long long)L.s_nmax * 8) / 8;
        L.edges = false;  // the sampler runs on G*, not on G
    }
    const long long per_tree = L.rec_stride * 8 + 16 + (L.bv ? L.s_rec_stride * 8 : 0);
    const long long per_slot = kSamplerPathSlot * 4;
    L.pools = (with_trees && !L.bv && !L.lds_bits && p->trees_per_batch <= 0 &&
               kDefaultBudget / (per_tree + per_slot) >= 2 * kPoolMinTrees)
                  ? 2
                  : 1;
    long long K = p->trees_per_batch > 0 ? p->trees_per_batch
                                         : std::max(1ll, kDefaultBudget / L.pools / (per_tree + per_slot));
    K = std::min<long long>(K, kMaxTreesPerBatch);
    if (p->tau_override > 0) K = std::min<long long>(K, p->tau_override);
    if (p->tau_cap > 0) K = std::min<long long>(K, p->tau_cap);
    L.K = with_trees ? (int)std::max(1ll, K) : 0;
    L.Kiv = std::min(L.K, 16);
    L.slots = std::min(L.K, kSamplerMaxBlocks);
    long long o = 0;
    auto take = [&](long long bytes) {
        long long at = o;
        o += align_up(bytes);
        return at;
    };
    const long long n = L.n;
    L.off_misc = take(sizeof(Misc));
    L.off_rp32 = take((n + 1) * 4);
    L.off_col16 = take(L.col16 ? (long long)L.nnz * 2 : 0);
    L.off_dist = take(n * 4);
    L.off_parB = take(n * 4);
    L.off_bint = take(n * 8);
    L.off_bflag = take(n * 4);
    L.off_vrow = take(L.edges ? n * 16 : 0);
    L.off_edge = take(L.edges ? (long long)L.nnz * 16 : 0);
    L.off_heavy = take(n * 4);
    L.off_bcount = take((n / 256 + 2) * 4);
    L.off_counts = take(n * 8);
    L.off_steps = take((long long)L.pools * L.K * 8);
    L.off_draws = take((long long)L.pools * L.K * 8);
    L.off_rec = take((long long)L.pools * L.K * L.rec_stride * 8);
    L.off_path = take((long long)L.pools * L.slots * kSamplerPathSlot * 4);
    L.off_scr = take(std::max((long long)L.Kiv * L.scr_stride, 3 * n) * 4);
    L.off_part = take((long long)kMaxSolveGrid * 6 * 8);
    L.off_x64 = take(n * 8);
    L.off_r64 = take(n * 8);
    L.off_z64 = take(n * 8);
    L.off_p64 = take(n * 8);
    L.off_q64 = take(n * 8);
    L.off_res64 = take(n * 8);
    L.off_x32 = take(n * 4);
    L.off_r32 = take(n * 4);
    L.off_z32 = take(n * 4);
    L.off_p32 = take(n * 4);
    L.off_q32 = take(n * 4);
    // weighted graphs: running row sums of the conductances, row totals, B_u edge weights,
    // fixed-point edge factors
    L.off_cw = take(L.weighted ? (long long)L.nnz * 8 : 0);
    L.off_guide = take(L.weighted ? (long long)L.nnz * 4 : 0);
    L.off_wdeg = take(L.weighted ? n * 8 : 0);
    L.off_wB = take(L.weighted ? n * 8 : 0);
    L.off_F = take(L.weighted ? n * 8 : 0);
    // the per-block variant: blocks of G, the slots of G* and its CSR, roots and tops, the
    // sampler's view of G*, and G*'s tree records (the joined trees go to the records above)
    const long long bn = L.bv ? n : 0, bnnz = L.bv ? (long long)L.nnz : 0, bs = L.bv ? L.s_nmax : 0;
    L.off_bc_lo = take(bn * 4);
    L.off_bc_hi = take(bn * 4);
    L.off_uf = take(bn * 4);
    L.off_fpar = take(bn * 4);
    L.off_ftop = take(bn * 4);
    L.off_spar = take(bn * 4);
    L.off_stop = take(bn * 4);
    L.off_rkey = take(bn * 8);
    L.off_eblk = take(bnnz * 4);
    L.off_flag = take(bnnz * 4);
    L.off_sid = take(L.bv ? (bnnz + 1) * 4 : 0);
    L.off_svtx = take(bs * 4);
    L.off_skey = take(bs * 4);
    L.off_sblk = take(bs * 4);
    L.off_sdeg = take(bs * 4);
    L.off_rps = take(L.bv ? (bs + 1) * 4 : 0);
    L.off_cur = take(bs * 4);
    L.off_scol = take(bnnz * 4);
    L.off_scol16 = take(L.bv && L.s_col16 ? bnnz * 2 : 0);
    L.off_sbflag = take(bs * 4);
    L.off_rflag = take(bs * 4);
    L.off_rpos = take(L.bv ? (bs + 1) * 4 : 0);
    L.off_roots = take(bn * 4);
    L.off_tops = take(bn * 4);
    L.off_tiles = take(L.bv ? (std::max(bnnz, bs) / 1024 + 2) * 4 : 0);
    L.off_svrow = take(L.bv && L.s_edges ? bs * 16 : 0);
    L.off_sedge = take(L.bv && L.s_edges ? bnnz * 16 : 0);
    L.off_srec = take(L.bv ? (long long)L.pools * L.K * L.s_rec_stride * 8 : 0);
    L.total = o;
    return L;
}

template <typename T>
T *at(void *ws, long long off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// tau = ecc^2 * ceil( ln(2m/delta) / (2 (1-kappa)^2 eps^2) ) (Algorithm 1, initialisation),
// then at most tau_cap when one is set; tau_override replaces the formula
long long sample_size(const ustd_problem *p, int ecc) {
    if (p->tau_override > 0) return p->tau_override;
    const double n = (double)p->n, m = (double)(p->nnz / 2);
    const double delta = p->delta > 0.0 ? p->delta : 1.0 / n;
    const double kappa = p->kappa > 0.0 ? p->kappa : 0.3;
    const double om = 1.0 - kappa;
    const double q = std::log(2.0 * m / delta) / (2.0 * om * om * p->eps * p->eps);
    const long long tau = (long long)ecc * (long long)ecc * (long long)std::ceil(q);
    return p->tau_cap > 0 ? std::min<long long>(tau, p->tau_cap) : tau;
}

// Weighted graphs (Section "Generalizations"): rho_max, the largest resistance of a B_u
// path, takes the place of ecc(u): tau = ceil(rho_max^2 ceil(ln(2m/delta) / (2 (1-kappa)^2
// eps^2))), then tau_cap; tau_override replaces the formula.
long long sample_size_weighted(const ustd_problem *p, double rho_max) {
    if (p->tau_override > 0) return p->tau_override;
    const double n = (double)p->n, m = (double)(p->nnz / 2);
    const double delta = p->delta > 0.0 ? p->delta : 1.0 / n;
    const double kappa = p->kappa > 0.0 ? p->kappa : 0.3;
    const double om = 1.0 - kappa;
    const double q = std::ceil(std::log(2.0 * m / delta) / (2.0 * om * om * p->eps * p->eps));
    const double r2 = rho_max * rho_max;
    const long long tau = (long long)std::ceil(r2 * q);
    return p->tau_cap > 0 ? std::min<long long>(tau, p->tau_cap) : tau;
}
// Fixed-point shift of a weighted problem's counts: tau rho_max 2^k <= 2^62.
int fixed_shift(long long tau, double rho_max) {
    int e = 0;
    std::frexp((double)tau * rho_max, &e);
    return 62 - e;
}

// eta = kappa eps / (3 sqrt(m n ln n) diam), diam <= 2 ecc (Algorithm 1, solver accuracy)
double solver_eta(const ustd_problem *p, int ecc) {
    const double n = (double)p->n, m = (double)(p->nnz / 2);
    const double kappa = p->kappa > 0.0 ? p->kappa : 0.3;
    return kappa * p->eps / (3.0 * std::sqrt(m * n * std::log(n)) * (2.0 * std::max(ecc, 1)));
}

// Calls of the allocation-free entry point create no HIP events (and no streams): timers then
// read 0 and synchronise with the stream instead.
thread_local bool g_no_events = false;
struct NoEventsScope {
    NoEventsScope() { g_no_events = true; }
    ~NoEventsScope() { g_no_events = false; }
};

// start/stop events around queued work, read once the stream has been synchronised
struct SpanTimer {
    hipEvent_t a = nullptr, b = nullptr;
    SpanTimer() {
        if (g_no_events) return;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    void start(hipStream_t st) {
        if (a) (void)hipEventRecord(a, st);
    }
    void stop(hipStream_t st) {
        if (b) (void)hipEventRecord(b, st);
    }
    double ms() const {
        float m = 0.f;
        if (a && b) (void)hipEventElapsedTime(&m, a, b);
        return (double)m;
    }
    ~SpanTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// elapsed time of the work queued on a stream between construction and stop_ms(), which
// synchronises the stream
struct Timer {
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    explicit Timer(hipStream_t s) : st(s) {
        if (g_no_events) return;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, st);
    }
    double stop_ms() {
        if (!a || !b) {
            (void)hipStreamSynchronize(st);
            return 0.0;
        }
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        return (double)ms;
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Extra streams per device (default priority, not blocking on the null stream): stream 0
// runs the pivot-column solve (and a weighted graph's row sums) while the trees are sampled
// on the caller's stream; stream 1 runs the second tree pool of a large graph (and every
// other sampler group of a batch); stream 2 runs a batch's Algorithm 2; streams 1 to 3 run
// the chains of a batch split into branches.  Created on first use and kept until the
// process ends.
constexpr int kSideStreams = 4;
int side_stream(hipStream_t *out, int which = 0) {
    static std::mutex mu;
    static std::vector<hipStream_t> streams;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    const size_t need = (size_t)(dev + 1) * kSideStreams;
    if (streams.size() < need) streams.resize(need, nullptr);
    hipStream_t &s = streams[(size_t)dev * kSideStreams + which];
    if (!s) HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    *out = s;
    return USTD_OK;
}

// an event without timing, destroyed with its scope
struct SyncEvent {
    hipEvent_t e = nullptr;
    SyncEvent() {
        if (!g_no_events) (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    }
    ~SyncEvent() {
        if (e) (void)hipEventDestroy(e);
    }
};

struct Ctx {
    const ustd_problem *p;
    Plan L;
    void *ws;
    hipStream_t st;
    Misc *misc;
    int *rp32;
    RowMap rows;
    int pivot = -1, ecc = 0;
    double rho_max = 0.0;  // weighted: largest B-path resistance
    long long tau = 0;     // weighted: the problem's tau (fixes the shift)
    int shift = 0;         // weighted: fixed-point shift k of the counts
    int nslots = 0, nblocks = 0;  // per-block variant: slots of G*, blocks of G
};

// tau of the problem set up in c
long long problem_tau(const Ctx &c) { return c.L.weighted ? c.tau : sample_size(c.p, c.ecc); }
// denominator of Eq. diag-comp for the counts: tau, or tau 2^k (fixed point)
double count_scale(const Ctx &c, long long tau) { return std::ldexp((double)tau, c.L.weighted ? c.shift : 0); }

// Weighted problems sum fixed-point contributions scaled so that the sums of up to 2 tau trees
// fit int64 (the shift comes from the problem's tau): a single call on more trees is refused.
int check_fixed_point_range(const Ctx &c, long long tree_count) {
    if (c.L.weighted && tree_count > 2 * c.tau)
        return fail(USTD_EINVAL, "a weighted count call covers at most 2 tau = %lld trees (got %lld)", 2 * c.tau,
                    tree_count);
    return USTD_OK;
}

int check_ws(void *ws, size_t ws_bytes, long long need) {
    if (!ws) return fail(USTD_EINVAL, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) return fail(USTD_EINVAL, "workspace must be 256-byte aligned");
    if ((long long)ws_bytes < need) return fail(USTD_ENOMEM, "workspace %zu bytes < required %lld", ws_bytes, need);
    return USTD_OK;
}

// per-problem preparation on the stream: 32-bit row pointers, the 16-bit column copy and
// the list of heavy rows, in the workspace region `ws` laid out by `L`
int begin_with(Ctx &c, const ustd_problem *p, const Plan &L, void *ws, void *stream) {
    c.p = p;
    c.L = L;
    c.ws = ws;
    c.st = (hipStream_t)stream;
    c.misc = at<Misc>(ws, c.L.off_misc);
    c.rp32 = at<int>(ws, c.L.off_rp32);
    HIP_TRY(hipMemsetAsync(c.misc, 0, sizeof(Misc), c.st));
    HIP_TRY(launch_rp_to_i32(c.L.n, (const long long *)p->d_row_ptr, c.rp32, c.st));
    if (c.L.col16) HIP_TRY(launch_col_to_u16(c.L.nnz, p->d_col, at<unsigned short>(ws, c.L.off_col16), c.st));
    c.rows.rp = c.rp32;
    c.rows.col = p->d_col;
    c.rows.n = c.L.n;
    c.rows.heavy_thresh = c.L.heavy_thresh;
    c.rows.heavy = at<int>(ws, c.L.off_heavy);
    c.rows.nheavy = &c.misc->nheavy;
    c.rows.w = nullptr;
    c.rows.wdeg = nullptr;
    HIP_TRY(launch_heavy_list(c.L.n, c.rp32, c.L.heavy_thresh, at<int>(ws, c.L.off_bcount), at<int>(ws, c.L.off_heavy),
                              &c.misc->nheavy, c.st));
    if (c.L.weighted) {  // the running row sums are queued by setup(), beside the BFS
        c.rows.w = p->d_weight;
        c.rows.wdeg = at<double>(ws, c.L.off_wdeg);
    }
    return USTD_OK;
}

int begin(Ctx &c, const ustd_problem *p, void *ws, size_t ws_bytes, void *stream) {
    USTD_TRY(check_problem(p));
    const Plan L = make_plan(p);
    USTD_TRY(check_ws(ws, ws_bytes, L.total));
    return begin_with(c, p, L, ws, stream);
}

// level-synchronous BFS from src into dist / parB, one readback per level; *ecc = levels - 1
// Levels are queued in groups with one readback per group, of 4, 4, then doubling to 64 (few
// round trips on deep graphs; small-world graphs, eccentricity below 8, queue two groups of 4
// and no idle launch beyond the second): a level after one
// that reached nothing returns at once (the group's first level runs: the previous group's
// last level reached something, or the loop would have ended).
constexpr int kBfsGroupFirst = 4, kBfsGroupMax = 64;
int bfs_levels(Ctx &c, int src, int *dist, int *parB, int *ecc) {
    static_assert(sizeof(c.misc->bfs_found) == kBfsGroupMax * sizeof(int), "one flag per queued level");
    HIP_TRY(launch_bfs_init(c.L.n, src, dist, parB, c.st));
    int *fl = c.misc->bfs_found;
    for (int d0 = 0, group = kBfsGroupFirst;;) {
        HIP_TRY(hipMemsetAsync(fl, 0, sizeof(int) * group, c.st));
        for (int j = 0; j < group; ++j)
            HIP_TRY(launch_bfs_level(c.rows, c.L.G, d0 + j, dist, parB, fl + j, j ? fl + j - 1 : nullptr, c.st));
        int found[kBfsGroupMax] = {};
        HIP_TRY(hipMemcpyAsync(found, fl, sizeof(int) * group, hipMemcpyDeviceToHost, c.st));
        HIP_TRY(hipStreamSynchronize(c.st));
        for (int j = 0; j < group; ++j)
            if (!found[j]) {
                *ecc = d0 + j;
                return USTD_OK;
            }
        d0 += group;
        group = d0 < 2 * kBfsGroupFirst ? kBfsGroupFirst : std::min(2 * group, kBfsGroupMax);
    }
}

unsigned packed_id(unsigned long long key) { return 0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull); }

// the packed key a reduction kernel left in misc->best_degree (then cleared for the next)
int read_key(Ctx &c, unsigned long long *key) {
    HIP_TRY(hipMemcpyAsync(key, &c.misc->best_degree, sizeof(*key), hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipMemsetAsync(&c.misc->best_degree, 0, sizeof(*key), c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    return USTD_OK;
}

// Pivot of low eccentricity by repeated BFS sweeps (engineering appendix): BFS from the
// maximum-degree vertex, then from the vertex farthest from the last source (smallest ID
// among the farthest), kPivotSweeps BFS in all; each raises every vertex's lower bound on
// its eccentricity to its distance; the pivot has the smallest bound (then smallest ID).
constexpr int kPivotSweeps = 10;
int sweep_pivot(Ctx &c, int *pivot) {
    const int n = c.L.n;
    int *dist = at<int>(c.ws, c.L.off_dist);
    int *parB = at<int>(c.ws, c.L.off_parB);
    int *bound = at<int>(c.ws, c.L.off_scr);
    if (n <= kSmallSolveMaxN) {  // all sweeps in one workgroup, one readback
        HIP_TRY(launch_sweep_small(c.rows, c.L.G, kPivotSweeps, dist, bound, c.misc->setup_out, c.st));
        int piv = -1;
        HIP_TRY(hipMemcpyAsync(&piv, c.misc->setup_out, sizeof(int), hipMemcpyDeviceToHost, c.st));
        HIP_TRY(hipStreamSynchronize(c.st));
        if (piv < 0 || piv >= n) return fail(USTD_EHIP, "sweep pivot out of range");
        *pivot = piv;
        return USTD_OK;
    }
    unsigned long long key = 0;
    HIP_TRY(hipMemsetAsync(&c.misc->best_degree, 0, sizeof(key), c.st));
    HIP_TRY(launch_argmax_degree(n, c.rp32, &c.misc->best_degree, c.st));
    USTD_TRY(read_key(c, &key));
    int src = (int)packed_id(key);
    for (int i = 0; i < kPivotSweeps; ++i) {
        int ecc = 0;
        USTD_TRY(bfs_levels(c, src, dist, parB, &ecc));
        HIP_TRY(launch_sweep_update(n, dist, bound, i == 0 ? 1 : 0, &c.misc->best_degree, c.st));
        USTD_TRY(read_key(c, &key));
        src = (int)packed_id(key);
    }
    HIP_TRY(launch_argmin_bound(n, bound, &c.misc->best_degree, c.st));
    USTD_TRY(read_key(c, &key));
    *pivot = (int)packed_id(key);
    return USTD_OK;
}

// Weighted graphs, after B_u: (with validate) the weight checks, then the B_u edge
// conductances, rho_max (read back), tau, the fixed-point shift and the edge factors F.
int setup_weighted(Ctx &c) {
    if (!c.L.weighted) return USTD_OK;
    const ustd_problem *p = c.p;
    const int n = c.L.n;
    if (p->validate) HIP_TRY(launch_check_weights(n, c.rp32, p->d_col, p->d_weight, &c.misc->err_validate, c.st));
    double *wB = at<double>(c.ws, c.L.off_wB);
    HIP_TRY(hipMemsetAsync(&c.misc->rho_max_bits, 0, sizeof(unsigned long long), c.st));
    HIP_TRY(launch_bpath(n, c.pivot, c.rp32, p->d_col, p->d_weight, at<int>(c.ws, c.L.off_parB), wB,
                         &c.misc->rho_max_bits, c.st));
    unsigned long long bits = 0;
    int err = 0;
    HIP_TRY(hipMemcpyAsync(&bits, &c.misc->rho_max_bits, sizeof(bits), hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipMemcpyAsync(&err, &c.misc->err_validate, sizeof(err), hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    if (err) return fail(USTD_EGRAPH, "weight validation failed (a conductance is not positive and finite, or "
                                      "differs between the two entries of its edge)");
    std::memcpy(&c.rho_max, &bits, sizeof(bits));
    if (!(c.rho_max > 0.0) || !std::isfinite(c.rho_max))
        return fail(USTD_EGRAPH, "largest B-path resistance %g is not positive and finite", c.rho_max);
    c.tau = sample_size_weighted(p, c.rho_max);
    c.shift = fixed_shift(c.tau, c.rho_max);
    if (c.shift < 0) return fail(USTD_EINVAL, "tau * rho_max = %g leaves no fixed-point range", (double)c.tau * c.rho_max);
    HIP_TRY(launch_fixed_weights(n, c.pivot, wB, c.shift, at<long long>(c.ws, c.L.off_F), c.st));
    return USTD_OK;
}

// relative residual target of the pivot-column solve: the caller's, else min(eta, 1e-12)
double solve_target(const ustd_problem *p, int ecc) {
    return p->solve_tol > 0.0 ? p->solve_tol : std::min(solver_eta(p, ecc), 1e-12);
}

// what set-up fixed: pivot, ecc, rho_max, the fixed-point shift, eta and the solve target
void setup_report(const Ctx &c, ustd_report *rep) {
    rep->pivot = c.pivot;
    rep->ecc = c.ecc;
    rep->rho_max = c.L.weighted ? c.rho_max : (double)c.ecc;
    rep->fixed_shift = c.shift;
    rep->weighted = c.L.weighted ? 1 : 0;
    rep->eta = solver_eta(c.p, c.ecc);
    rep->solve_tol = solve_target(c.p, c.ecc);
}

int setup_graph(Ctx &c, ustd_report *rep);

// pivot choice, optional validation and the BFS tree B_u; synchronises the stream.  For a
// weighted graph the running row sums and the step guide (needed from sampling on) are
// computed on the side stream meanwhile; the caller's stream waits for them on success, and
// on an error the host waits, so nothing is left writing the workspace.
int setup_blocks(Ctx &c);

int setup(Ctx &c, ustd_report *rep) {
    if (!c.L.weighted) {
        USTD_TRY(setup_graph(c, rep));
        return c.L.bv ? setup_blocks(c) : USTD_OK;
    }
    if (g_no_events) {  // everything on the caller's stream
        const ustd_problem *p = c.p;
        HIP_TRY(launch_row_cumsum(c.L.n, c.L.nnz, c.rp32, p->d_weight, c.L.heavy_thresh, c.rows.heavy, c.rows.nheavy,
                                  at<double>(c.ws, c.L.off_cw), at<double>(c.ws, c.L.off_wdeg),
                                  at<int>(c.ws, c.L.off_guide), c.st));
        return setup_graph(c, rep);
    }
    hipStream_t side = nullptr;
    USTD_TRY(side_stream(&side));
    SyncEvent fork, join;
    if (!fork.e || !join.e) return fail(USTD_EHIP, "hipEventCreateWithFlags failed");
    HIP_TRY(hipEventRecord(fork.e, c.st));
    HIP_TRY(hipStreamWaitEvent(side, fork.e, 0));
    const ustd_problem *p = c.p;
    int rc = hipSuccess == launch_row_cumsum(c.L.n, c.L.nnz, c.rp32, p->d_weight, c.L.heavy_thresh, c.rows.heavy,
                                             c.rows.nheavy, at<double>(c.ws, c.L.off_cw),
                                             at<double>(c.ws, c.L.off_wdeg), at<int>(c.ws, c.L.off_guide), side)
                 ? USTD_OK
                 : fail(USTD_EHIP, "row sums launch failed");
    if (rc == USTD_OK && hipEventRecord(join.e, side) != hipSuccess) rc = fail(USTD_EHIP, "hipEventRecord failed");
    if (rc != USTD_OK) {
        (void)hipStreamSynchronize(side);
        return rc;
    }
    rc = setup_graph(c, rep);
    if (rc != USTD_OK) {
        (void)hipEventSynchronize(join.e);
        return rc;
    }
    HIP_TRY(hipStreamWaitEvent(c.st, join.e, 0));
    return USTD_OK;
}

int setup_graph(Ctx &c, ustd_report *rep) {
    const ustd_problem *p = c.p;
    const int n = c.L.n;
    Timer tm(c.st);
    if (p->validate) HIP_TRY(launch_validate(n, p->nnz, (const long long *)p->d_row_ptr, p->d_col, &c.misc->err_validate, c.st));
    if (p->pivot >= 0) {
        c.pivot = p->pivot;
    } else if (p->pivot == -2) {
        USTD_TRY(sweep_pivot(c, &c.pivot));
    } else {
        HIP_TRY(launch_argmax_degree(n, c.rp32, &c.misc->best_degree, c.st));
        unsigned long long best = 0;
        HIP_TRY(hipMemcpyAsync(&best, &c.misc->best_degree, sizeof(best), hipMemcpyDeviceToHost, c.st));
        HIP_TRY(hipStreamSynchronize(c.st));
        c.pivot = (int)(0xFFFFFFFFu - (unsigned)(best & 0xFFFFFFFFull));
    }
    if (p->validate) {
        int err = 0;
        HIP_TRY(hipMemcpyAsync(&err, &c.misc->err_validate, sizeof(int), hipMemcpyDeviceToHost, c.st));
        HIP_TRY(hipStreamSynchronize(c.st));
        if (err) return fail(USTD_EGRAPH, "graph validation failed (code %d: 1 bounds, 2 unsorted/range, 4 self-loop, 8 asymmetric, 16 isolated)", err);
    }
    int *dist = at<int>(c.ws, c.L.off_dist);
    int *parB = at<int>(c.ws, c.L.off_parB);
    if (n <= kSmallSolveMaxN) {
        // BFS tree, connectivity and B_u intervals in one workgroup, one readback
        HIP_TRY(launch_setup_small(c.rows, c.L.G, c.pivot, dist, parB, at<int>(c.ws, c.L.off_scr),
                                   at<int2>(c.ws, c.L.off_bint), at<int>(c.ws, c.L.off_bflag), c.misc->setup_out,
                                   c.st));
        int out[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(out, c.misc->setup_out, sizeof(out), hipMemcpyDeviceToHost, c.st));
        HIP_TRY(hipStreamSynchronize(c.st));
        if (out[1]) return fail(USTD_EGRAPH, "graph is not connected");
        c.ecc = out[0];
        if (c.L.edges) {
            HIP_TRY(launch_vertex_rows(n, c.rp32, at<int>(c.ws, c.L.off_bflag), at<int4>(c.ws, c.L.off_vrow), c.st));
            HIP_TRY(launch_edge_rows(c.L.nnz, c.p->d_col, at<int4>(c.ws, c.L.off_vrow), at<int4>(c.ws, c.L.off_edge), c.st));
        }
        USTD_TRY(setup_weighted(c));
        if (rep) {
            setup_report(c, rep);
            rep->ms_bfs += tm.stop_ms();
        }
        return USTD_OK;
    }
    USTD_TRY(bfs_levels(c, c.pivot, dist, parB, &c.ecc));
    HIP_TRY(launch_count_unreached(n, dist, &c.misc->err_validate, c.st));
    int err = 0;
    HIP_TRY(hipMemcpyAsync(&err, &c.misc->err_validate, sizeof(int), hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    if (err) return fail(USTD_EGRAPH, "graph is not connected");
    // subtree intervals of B_u (fixed for every tree): bint[x] = {pre_B, size_B}
    HIP_TRY(launch_b_intervals(n, c.pivot, c.ecc, dist, parB, at<int>(c.ws, c.L.off_scr), at<int2>(c.ws, c.L.off_bint),
                               at<int>(c.ws, c.L.off_bflag), c.st));
    if (c.L.edges) {  // the sampler's vertex and edge entries
        HIP_TRY(launch_vertex_rows(n, c.rp32, at<int>(c.ws, c.L.off_bflag), at<int4>(c.ws, c.L.off_vrow), c.st));
        HIP_TRY(launch_edge_rows(c.L.nnz, c.p->d_col, at<int4>(c.ws, c.L.off_vrow), at<int4>(c.ws, c.L.off_edge), c.st));
    }
    USTD_TRY(setup_weighted(c));
    if (rep) {
        setup_report(c, rep);
        rep->ms_bfs += tm.stop_ms();
    }
    return USTD_OK;
}

// The per-block variant's set-up, after B_u: blocks, the slots and CSR of G*, the block roots
// and tops, and the sampler's view of G*.  Two readbacks (the slot count, then the root and top
// counts); synchronises the stream.
int setup_blocks(Ctx &c) {
    const Plan &L = c.L;
    const int n = L.n, u = c.pivot;
    const long long nnz = L.nnz;
    void *ws = c.ws;
    hipStream_t st = c.st;
    int *lo = at<int>(ws, L.off_bc_lo), *hi = at<int>(ws, L.off_bc_hi), *uf = at<int>(ws, L.off_uf);
    int *fpar = at<int>(ws, L.off_fpar), *ftop = at<int>(ws, L.off_ftop);
    int *spar = at<int>(ws, L.off_spar), *stop = at<int>(ws, L.off_stop);
    int *eblk = at<int>(ws, L.off_eblk), *flag = at<int>(ws, L.off_flag), *sid = at<int>(ws, L.off_sid);
    int *vtx = at<int>(ws, L.off_svtx), *skey = at<int>(ws, L.off_skey), *sblk = at<int>(ws, L.off_sblk);
    int *sdeg = at<int>(ws, L.off_sdeg), *rps = at<int>(ws, L.off_rps), *cur = at<int>(ws, L.off_cur);
    int *scol = at<int>(ws, L.off_scol), *rflag = at<int>(ws, L.off_rflag), *rpos = at<int>(ws, L.off_rpos);
    int *roots = at<int>(ws, L.off_roots), *tops = at<int>(ws, L.off_tops), *tiles = at<int>(ws, L.off_tiles);
    const int *parB = at<int>(ws, L.off_parB), *dist = at<int>(ws, L.off_dist);
    const int2 *bint = at<int2>(ws, L.off_bint);
    HIP_TRY(launch_bc_blocks(c.rows, L.G, u, c.ecc, dist, parB, bint, lo, hi, uf, st));
    HIP_TRY(launch_fill_i32(n, fpar, INT32_MAX, st));
    HIP_TRY(launch_fill_i32(n, ftop, INT32_MAX, st));
    HIP_TRY(launch_bc_entries(n, nnz, u, c.rp32, c.p->d_col, parB, bint, uf, eblk, fpar, ftop, flag, st));
    HIP_TRY(launch_scan_excl(flag, sid, nnz, tiles, &c.misc->nslots, st));
    HIP_TRY(launch_fill_i32(L.s_nmax, sdeg, 0, st));
    HIP_TRY(launch_fill_i32(L.s_nmax, cur, 0, st));
    HIP_TRY(hipMemsetAsync(at<void>(ws, L.off_rkey), 0, (size_t)n * 8, st));
    HIP_TRY(launch_bc_slots(n, nnz, u, c.rp32, flag, sid, eblk, uf, vtx, skey, sblk, spar, stop, sdeg, st));
    int ns = 0;
    HIP_TRY(hipMemcpyAsync(&ns, &c.misc->nslots, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (ns < n || ns > L.s_nmax) return fail(USTD_EHIP, "block split: %d slots for %d vertices", ns, n);
    HIP_TRY(launch_scan_excl(sdeg, rps, ns, tiles, &c.misc->scan_total, st));
    HIP_TRY(launch_bc_columns(n, u, c.rp32, c.p->d_col, eblk, uf, spar, stop, rps, cur, scol, st));
    HIP_TRY(launch_bc_roots(ns, rps, vtx, sblk, at<unsigned long long>(ws, L.off_rkey), rflag, st));
    HIP_TRY(launch_scan_excl(rflag, rpos, ns, tiles, &c.misc->nroots, st));
    HIP_TRY(launch_bc_compact(ns, rflag, rpos, roots, st));
    HIP_TRY(launch_bc_top_flags(ns, sblk, stop, rflag, st));
    HIP_TRY(launch_scan_excl(rflag, rpos, ns, tiles, &c.misc->ntops, st));
    HIP_TRY(launch_bc_compact(ns, rflag, rpos, tops, st));
    // the sampler's view of G*: no B_u flags (no marks), 16-bit columns or edge entries
    int *sbflag = at<int>(ws, L.off_sbflag);
    HIP_TRY(launch_fill_i32(ns, sbflag, 0, st));
    if (L.s_col16) HIP_TRY(launch_col_to_u16(nnz, scol, at<unsigned short>(ws, L.off_scol16), st));
    if (L.s_edges) {
        HIP_TRY(launch_vertex_rows(ns, rps, sbflag, at<int4>(ws, L.off_svrow), st));
        HIP_TRY(launch_edge_rows(nnz, scol, at<int4>(ws, L.off_svrow), at<int4>(ws, L.off_sedge), st));
    }
    int cnt[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&cnt[0], &c.misc->nroots, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&cnt[1], &c.misc->ntops, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (cnt[0] != cnt[1] || cnt[0] < 1 || ns != n + cnt[0] - 1)
        return fail(USTD_EHIP, "block split: %d roots, %d tops, %d slots for %d vertices", cnt[0], cnt[1], ns, n);
    c.nslots = ns;
    c.nblocks = cnt[0];
    return USTD_OK;
}

WilsonGraph wilson_graph(const Ctx &c) {
    WilsonGraph g{};
    g.n = c.L.n;
    g.u = c.pivot;
    g.nwords = c.L.nwords;
    g.rob = c.L.rob;
    g.rp = c.rp32;
    g.colv = c.L.col16 ? (const void *)at<unsigned short>(c.ws, c.L.off_col16) : (const void *)c.p->d_col;
    g.bflag = at<int>(c.ws, c.L.off_bflag);
    g.vrow = c.L.edges ? at<int4>(c.ws, c.L.off_vrow) : nullptr;
    g.edge = c.L.edges ? at<int4>(c.ws, c.L.off_edge) : nullptr;
    g.cw = c.L.weighted ? at<double>(c.ws, c.L.off_cw) : nullptr;
    g.guide = c.L.weighted ? at<int>(c.ws, c.L.off_guide) : nullptr;
    g.key0 = (uint32_t)(c.p->seed & 0xFFFFFFFFull);
    g.key1 = (uint32_t)(c.p->seed >> 32);
    return g;
}

// records, sampler slots, step and draw counts of tree pool `pool`
int2 *pool_rec(const Ctx &c, int pool) { return at<int2>(c.ws, c.L.off_rec) + (long long)pool * c.L.K * c.L.rec_stride; }
long long *pool_steps(const Ctx &c, int pool) { return at<long long>(c.ws, c.L.off_steps) + (long long)pool * c.L.K; }
long long *pool_draws(const Ctx &c, int pool) { return at<long long>(c.ws, c.L.off_draws) + (long long)pool * c.L.K; }

// trees tree_begin .. +ntrees-1 into the record slots 0 .. ntrees-1 of a pool (ntrees <= K),
// on stream st
// the per-block variant: trees on G* (several roots, keyed starts) into G*'s records, then the
// block trees joined into records of spanning trees of G in the pool's records
int sample_batch_blocks(Ctx &c, long long tree_begin, int ntrees, long long *steps, long long *draws, int pool,
                        hipStream_t st) {
    const Plan &L = c.L;
    const int ns = c.nslots;
    WilsonArgs a{};
    WilsonGraph &g = a.g;
    g.n = ns;
    g.u = -1;
    g.nwords = (ns + 31) / 32;
    g.rob = std::min(L.s_lds ? kSamplerRobLds : kSamplerRobMax, next_pow2(std::max(ns, 2)));
    g.rp = at<int>(c.ws, L.off_rps);
    g.colv = L.s_col16 ? (const void *)at<unsigned short>(c.ws, L.off_scol16) : (const void *)at<int>(c.ws, L.off_scol);
    g.bflag = at<int>(c.ws, L.off_sbflag);
    g.vrow = L.s_edges ? at<int4>(c.ws, L.off_svrow) : nullptr;
    g.edge = L.s_edges ? at<int4>(c.ws, L.off_sedge) : nullptr;
    g.key0 = (uint32_t)(c.p->seed & 0xFFFFFFFFull);
    g.key1 = (uint32_t)(c.p->seed >> 32);
    a.ntiles = ntrees;
    a.tree_begin = tree_begin;
    int2 *srec = at<int2>(c.ws, L.off_srec) + (long long)pool * L.K * L.s_rec_stride;
    a.rec = srec;
    a.rec_stride = L.s_rec_stride;
    a.path = at<int>(c.ws, L.off_path) + (long long)pool * L.slots * kSamplerPathSlot;
    a.queue = &c.misc->queue[pool];
    a.steps = steps;
    a.draws = draws;
    a.roots = at<int>(c.ws, L.off_roots);
    a.nroots = c.nblocks;
    a.skey = at<int>(c.ws, L.off_skey);
    int blocks = std::min(ntrees, L.slots);
    const int resident = wilson_resident_blocks(L.s_lds, L.s_col16, false, g.nwords, true);
    if (resident > 0) blocks = std::min(blocks, resident);
    HIP_TRY(hipMemsetAsync(&c.misc->queue[pool], 0, sizeof(int), st));
    HIP_TRY(launch_wilson(a, blocks, L.s_lds, L.s_col16, false, g.nwords, st, 0, true));
    HIP_TRY(launch_bc_join(L.n, c.pivot, ntrees, c.nblocks, ns, at<int>(c.ws, L.off_tops), at<int>(c.ws, L.off_spar),
                           at<int>(c.ws, L.off_svtx), srec, L.s_rec_stride, pool_rec(c, pool), L.rec_stride,
                           at<int>(c.ws, L.off_bflag), st));
    return USTD_OK;
}

int sample_batch(Ctx &c, long long tree_begin, int ntrees, long long *steps, long long *draws, int pool = 0,
                 hipStream_t st = nullptr) {
    if (!st) st = c.st;
    if (c.L.bv) return sample_batch_blocks(c, tree_begin, ntrees, steps, draws, pool, st);
    WilsonArgs a{};
    a.g = wilson_graph(c);
    a.ntiles = ntrees;
    a.tree_begin = tree_begin;
    a.rec = pool_rec(c, pool);
    a.rec_stride = c.L.rec_stride;
    a.path = at<int>(c.ws, c.L.off_path) + (long long)pool * c.L.slots * kSamplerPathSlot;
    a.queue = &c.misc->queue[pool];
    a.steps = steps;
    a.draws = draws;
    int blocks = std::min(ntrees, c.L.slots);
    const int resident = wilson_resident_blocks(c.L.lds_bits, c.L.col16, c.L.weighted, c.L.nwords);
    if (resident > 0) blocks = std::min(blocks, resident);
    // a small unweighted graph also goes into LDS when that leaves as many trees running at once
    long long gl = 0;
    if (c.L.lds_bits && c.L.col16 && !c.L.weighted) {
        const long long gb = wilson_graph_lds_bytes(c.L.n, c.L.nnz);
        if (gb <= kGraphLdsMaxBytes && wilson_resident_blocks_graph_lds(c.L.nwords, gb) >= blocks) gl = gb;
    }
    HIP_TRY(hipMemsetAsync(&c.misc->queue[pool], 0, sizeof(int), st));
    HIP_TRY(launch_wilson(a, blocks, c.L.lds_bits, c.L.col16, c.L.weighted, c.L.nwords, st, gl));
    return USTD_OK;
}

// Trees per Algorithm 2 thread: deep B_u (long marked-ancestor chains: grids, hyperbolic
// graphs) walks 4 trees per thread, which leaves registers for more threads to cover the chain
// loads; shallow small-world B_u walks 8 (measured: RHG 1M and the 64-graph batch gain 15-18%
// of Algorithm 2 time with 4, R-MAT 16 loses 6%).
constexpr int kAggDeepEcc = 8;
int agg_chunk(int ecc) { return ecc >= kAggDeepEcc ? kAggChunkLarge : kAggChunk; }
// the form of Algorithm 2: a schedule's fixed chunk, else by eccentricity
void agg_form(AggregateArgs &aa, int ecc, int sched_chunk) { aa.chunk = sched_chunk > 0 ? sched_chunk : agg_chunk(ecc); }

// Algorithm 2 over `cnt` resident trees (records of a pool), on stream st
int aggregate_trees(Ctx &c, int cnt, long long *counts, double *ms_ag, int pool = 0, hipStream_t st = nullptr) {
    if (!st) st = c.st;
    AggregateArgs aa{};
    aa.n = c.L.n;
    aa.u = c.pivot;
    aa.ntrees = cnt;
    aa.parB = at<int>(c.ws, c.L.off_parB);
    aa.bint = at<int2>(c.ws, c.L.off_bint);
    aa.rec = pool_rec(c, pool);
    aa.rec_stride = c.L.rec_stride;
    aa.counts = counts;
    aa.F = c.L.weighted ? at<long long>(c.ws, c.L.off_F) : nullptr;
    agg_form(aa, c.ecc, 0);
    Timer tm(st);
    HIP_TRY(launch_aggregate(aa, st));
    if (ms_ag) *ms_ag += tm.stop_ms();
    return USTD_OK;
}

// Spanning-edge counts over `cnt` resident trees (records of a pool), on stream st
int edge_count_trees(Ctx &c, int cnt, long long *edge_counts, double *ms, int pool = 0, hipStream_t st = nullptr) {
    if (!st) st = c.st;
    EdgeCountArgs ea{};
    ea.n = c.L.n;
    ea.u = c.pivot;
    ea.ntrees = cnt;
    ea.trees_per_chunk = kEdgeTreesPerChunk;
    ea.rp = c.rp32;
    ea.col = c.p->d_col;
    ea.rec = pool_rec(c, pool);
    ea.rec_stride = c.L.rec_stride;
    ea.counts = edge_counts;
    Timer tm(st);
    HIP_TRY(launch_edge_counts(ea, st));
    if (ms) *ms += tm.stop_ms();
    return USTD_OK;
}

// Samples trees tree_begin .. +tree_count-1 in batches of at most K; after each batch,
// Algorithm 2 adds into `counts` and/or the spanning-edge counts into `edge_counts`.  With
// two tree pools, batches alternate between the caller's stream and side stream 1, so a
// batch's tail and its Algorithm 2 overlap the next batch (integer counts make the order
// irrelevant).  Walk totals are summed on the device and read once.  `overlap`, if given,
// runs on the host once all batches are queued, before anything waits for them (work for
// other streams).
int run_trees(Ctx &c, long long tree_begin, long long tree_count, long long *counts, ustd_report *rep,
              long long *edge_counts = nullptr, const std::function<void()> &overlap = nullptr,
              hipEvent_t last_sampled = nullptr) {
    // equal batches: ceil(count / K) of them, none larger than K
    const long long nb = (tree_count + c.L.K - 1) / c.L.K;
    const long long per = nb > 0 ? (tree_count + nb - 1) / nb : 0;
    const int npools = (c.L.pools == 2 && nb > 1) ? 2 : 1;
    hipStream_t st[2] = {c.st, c.st};
    unsigned long long *totals = c.misc->walk_totals;
    HIP_TRY(hipMemsetAsync(totals, 0, 2 * sizeof(unsigned long long), c.st));
    SyncEvent fork, join;
    if (npools == 2) {
        USTD_TRY(side_stream(&st[1], 1));
        if (!fork.e || !join.e) return fail(USTD_EHIP, "hipEventCreateWithFlags failed");
        HIP_TRY(hipEventRecord(fork.e, c.st));
        HIP_TRY(hipStreamWaitEvent(st[1], fork.e, 0));
    }
    std::vector<std::unique_ptr<SpanTimer>> ts, ta;
    int batches = 0;
    int rc = USTD_OK;
    for (long long b0 = 0; b0 < tree_count && rc == USTD_OK; b0 += per) {
        const int cnt = (int)std::min<long long>(per, tree_count - b0);
        const int pool = batches % npools;
        hipStream_t s = st[pool];
        ts.emplace_back(new SpanTimer());
        ta.emplace_back(new SpanTimer());
        ts.back()->start(s);
        rc = sample_batch(c, tree_begin + b0, cnt, pool_steps(c, pool), pool_draws(c, pool), pool, s);
        if (rc != USTD_OK) break;
        ts.back()->stop(s);
        if (last_sampled && b0 + per >= tree_count && hipEventRecord(last_sampled, s) != hipSuccess) {
            rc = fail(USTD_EHIP, "hipEventRecord failed");
            break;
        }
        if (launch_sum_walks(cnt, pool_steps(c, pool), pool_draws(c, pool), totals, s) != hipSuccess) {
            rc = fail(USTD_EHIP, "walk totals launch failed");
            break;
        }
        ta.back()->start(s);
        if (counts) rc = aggregate_trees(c, cnt, counts, nullptr, pool, s);
        if (rc == USTD_OK && edge_counts) rc = edge_count_trees(c, cnt, edge_counts, nullptr, pool, s);
        ta.back()->stop(s);
        ++batches;
    }
    // every batch is queued; the host is free for the other streams' work meanwhile
    if (rc == USTD_OK && overlap) overlap();
    if (npools == 2) {
        // the caller's stream takes up after both pools' work; on an error the host waits
        if (rc == USTD_OK && hipEventRecord(join.e, st[1]) == hipSuccess &&
            hipStreamWaitEvent(c.st, join.e, 0) == hipSuccess) {
        } else {
            (void)hipStreamSynchronize(st[1]);
            if (rc == USTD_OK) rc = fail(USTD_EHIP, "joining the tree pools failed");
        }
    }
    if (rc != USTD_OK) {
        (void)hipStreamSynchronize(c.st);
        return rc;
    }
    unsigned long long tot[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(tot, totals, sizeof(tot), hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    double ms_s = 0, ms_a = 0;
    for (size_t i = 0; i < ts.size(); ++i) {
        ms_s += ts[i]->ms();
        ms_a += ta[i]->ms();
    }
    if (rep) {
        rep->walk_steps += (long long)tot[0];
        rep->walk_draws += (long long)tot[1];
        rep->n_batches += batches;
        rep->trees_per_batch = c.L.K;
        rep->ms_sample += ms_s;
        rep->ms_aggregate += ms_a;
    }
    return USTD_OK;
}

// ---------------------------------------------------------------------------------------
// pivot-column solve
// ---------------------------------------------------------------------------------------
// Reliable-update threshold of the pivot-column solve: an update when |r_s| has fallen by delta
// since the largest residual after the last one.  FP32 iterations drift from the true residual
// after a few orders of magnitude, FP64 ones only near the rounding floor.  Measured on the
// hyperbolic 1M graph (FP32 iterations / time against FP64's 2377 / 614 ms): delta 0.1 2442 /
// 470 ms, 0.01 2463 / 473 ms, 0.001 4257 / 811 ms; on R-MAT scale 22 (35 iterations either way)
// 0.1 costs 9 updates (51 ms), 0.01 six (48 ms, FP64 47 ms).
constexpr double kDeltaMixed = 1e-2, kDeltaFp64 = 1e-6;

template <typename T>
SolveArgs<T> solve_args(const Ctx &c, void *ws, const Plan &L, double *x) {
    SolveArgs<T> a{};
    a.n = L.n;
    a.u = c.pivot;
    a.x = x;
    if constexpr (sizeof(T) == 8) {
        a.xs = (T *)at<double>(ws, L.off_res64);
        a.rs = (T *)at<double>(ws, L.off_r64);
        a.z = (T *)at<double>(ws, L.off_z64);
        a.p = (T *)at<double>(ws, L.off_p64);
        a.q = (T *)at<double>(ws, L.off_q64);
    } else {
        a.xs = (T *)at<float>(ws, L.off_x32);
        a.rs = (T *)at<float>(ws, L.off_r32);
        a.z = (T *)at<float>(ws, L.off_z32);
        a.p = (T *)at<float>(ws, L.off_p32);
        a.q = (T *)at<float>(ws, L.off_q32);
    }
    a.part = at<double>(ws, L.off_part);
    a.grid_spmv = solve_grid(c.rows, L.G);
    a.grid_vec = vec_grid(L.n);
    a.sc = &c.misc->sc;
    a.rp = c.rp32;
    a.wdeg = c.rows.wdeg;
    return a;
}

double solve_delta2(const ustd_problem *p) {
    const double d = p->solve_mode == USTD_SOLVE_MIXED ? kDeltaMixed : kDeltaFp64;
    return d * d;
}

// A small pinned host buffer per thread and device for the solve's scalars, so that reading
// them back does not stall the stream (allocated on first use, kept until the process ends).
SolveScalars *pinned_scalars(int slots) {
    thread_local std::vector<SolveScalars *> bufs;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    if ((int)bufs.size() <= dev) bufs.resize(dev + 1, nullptr);
    if (!bufs[dev]) {
        void *h = nullptr;
        if (hipHostMalloc(&h, sizeof(SolveScalars) * 4, hipHostMallocDefault) != hipSuccess) return nullptr;
        bufs[dev] = static_cast<SolveScalars *>(h);
    }
    return slots <= 4 ? bufs[dev] : nullptr;
}

// the engine of a solve: `batch` for a member of ustd_batch_diag_lpinv
bool one_workgroup(const ustd_problem *p, int n, bool batch) {
    if (p->solve_engine == USTD_ENGINE_WORKGROUP) return true;
    if (p->solve_engine == USTD_ENGINE_MULTI) return false;
    return batch || n <= kSmallSolveMaxN;
}

// PCG with reliable updates on the vectors of type T, in one workgroup or by iteration kernels.
// The iteration kernels are enqueued in chunks of 8, 16, ... 256 iterations, each followed by an
// asynchronous copy of the scalars into pinned memory; the host stays one chunk ahead and stops
// enqueueing once a copied `done` is set, so the device never waits for the host.  Leaves x
// (not yet projected) and the final scalars in *out.
template <typename T>
int solve_iterate(Ctx &c, double *x, double tol2, int maxit, SolveScalars *out) {
    const SolveArgs<T> a = solve_args<T>(c, c.ws, c.L, x);
    const double delta2 = solve_delta2(c.p);
    if (one_workgroup(c.p, c.L.n, false)) {
        HIP_TRY(launch_solve_small<T>(a, c.rows, c.L.G, tol2, delta2, maxit, c.st));
    } else {
        SolveScalars *hs = pinned_scalars(2);
        if (!hs) return fail(USTD_EHIP, "pinned host buffer for the solve scalars");
        SyncEvent ev[2];
        if (!ev[0].e || !ev[1].e) return fail(USTD_EHIP, "hipEventCreateWithFlags failed");
        HIP_TRY(launch_solve_start<T>(a, tol2, delta2, maxit, c.st));
        int launched = 0, chunk = 8, k = 0;
        for (;;) {
            const int todo = std::min(chunk, maxit - launched);
            for (int i = 0; i < todo; ++i) HIP_TRY(launch_solve_iteration<T>(a, c.rows, c.L.G, c.st));
            launched += todo;
            chunk = std::min(2 * chunk, 256);
            HIP_TRY(hipMemcpyAsync(&hs[k & 1], a.sc, sizeof(SolveScalars), hipMemcpyDeviceToHost, c.st));
            HIP_TRY(hipEventRecord(ev[k & 1].e, c.st));
            if (launched >= maxit) break;
            if (k > 0) {  // the chunk before the one just queued
                HIP_TRY(hipEventSynchronize(ev[(k - 1) & 1].e));
                if (hs[(k - 1) & 1].done) break;
            }
            ++k;
        }
    }
    HIP_TRY(hipMemcpyAsync(out, a.sc, sizeof(*out), hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    return USTD_OK;
}

// x <- x - mean(x), then the true relative residual ||b - L x|| / ||b|| of the projected x
int project_and_residual(Ctx &c, double *x, double *relres) {
    double *part = at<double>(c.ws, c.L.off_part) + 3 * kMaxSolveGrid;  // residual partials
    double *sums = c.misc->sums;
    HIP_TRY(launch_residual64(c.rows, c.L.G, c.pivot, x, nullptr, part, sums, c.st));
    HIP_TRY(launch_project(c.L.n, x, sums + 2, vec_grid(c.L.n), c.st));
    HIP_TRY(launch_residual64(c.rows, c.L.G, c.pivot, x, nullptr, part, sums, c.st));
    double hs[4];
    HIP_TRY(hipMemcpyAsync(hs, sums, sizeof(hs), hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    const double bnorm = std::sqrt((double)(c.L.n - 1) / (double)c.L.n);
    *relres = std::sqrt(std::max(hs[1], 0.0)) / bnorm;
    return USTD_OK;
}

// Column u of L^+ into x_out: FP64 PCG, or FP32 PCG with FP64 reliable updates (mixed).
// Success is judged on the true FP64 residual of the projected solution alone.
int solve_column(Ctx &c, double *x_out, ustd_report *rep) {
    const ustd_problem *p = c.p;
    const double tol = solve_target(p, c.ecc);
    const int maxit = p->solve_maxit > 0 ? p->solve_maxit : 20000;
    Timer tm(c.st);
    SolveScalars sc{};
    if (p->solve_mode == USTD_SOLVE_FP64) USTD_TRY(solve_iterate<double>(c, x_out, tol * tol, maxit, &sc));
    else USTD_TRY(solve_iterate<float>(c, x_out, tol * tol, maxit, &sc));
    double relres = 0.0;
    USTD_TRY(project_and_residual(c, x_out, &relres));
    const bool conv = relres <= tol;
    if (rep) {
        rep->solve_iters += sc.iter;
        rep->solve_outer += sc.updates;
        rep->solve_relres = relres;
        rep->solve_tol = tol;
        rep->solve_converged = conv ? 1 : 0;
        rep->ms_solve += tm.stop_ms();
    }
    if (!conv) return fail(USTD_ENOTCONV, "solve stopped at relative residual %.3e (target %.3e)", relres, tol);
    return USTD_OK;
}

// ---------------------------------------------------------------------------------------
// batches of problems: every member keeps its own region (CSR copies, B_u, counts, solve
// vectors); the trees of all members share one pool of records and sampler slots, filled
// with (graph, tree) tiles, larger graphs first, and sampled by one persistent launch per
// pool fill.
// ---------------------------------------------------------------------------------------
constexpr long long kMaxBatchTiles = 1ll << 20;
constexpr int kMaxBranches = 4;

struct BatchPlan {
    std::vector<Plan> g;
    std::vector<long long> base;  // byte offset of each member's region
    bool lds_bits = true, col16 = true;
    int nwords_max = 0, slots = 0;
    long long rec_pool = 0, max_tiles = 0;
    long long path_slots = 0;  // sampler path slots per launch stream (blocks of one launch at most)
    long long off_queue = 0, off_rec = 0, off_path = 0, off_steps = 0, off_draws = 0, total = 0;
};

// the schedule with its defaults filled in, and its checks
ustd_batch_schedule schedule_of(const ustd_batch_schedule *s) {
    ustd_batch_schedule r{};
    if (s) r = *s;
    if (r.group_fills == 0) r.group_fills = kBatchGroupFills;
    if (r.branches == 1) r.branches = 0;
    return r;
}
int check_schedule(const ustd_batch_schedule &s) {
    if (s.group_fills < -1) return fail(USTD_EINVAL, "group_fills %d (> 0, 0 or -1)", s.group_fills);
    if (s.agg_chunk != 0 && s.agg_chunk != kAggChunk && s.agg_chunk != kAggChunkLarge)
        return fail(USTD_EINVAL, "agg_chunk %d (0, %d or %d)", s.agg_chunk, kAggChunkLarge, kAggChunk);
    if (s.layout != USTD_LAYOUT_AUTO && s.layout != USTD_LAYOUT_RECORDS)
        return fail(USTD_EINVAL, "layout %d", s.layout);
    if (s.fill_trees < 0) return fail(USTD_EINVAL, "fill_trees %lld < 0", (long long)s.fill_trees);
    if (s.branches < 0 || s.branches > kMaxBranches) return fail(USTD_EINVAL, "branches %d (0 .. %d)", s.branches, kMaxBranches);
    return USTD_OK;
}

int make_batch_plan(const ustd_problem *probs, int count, BatchPlan &B, const ustd_batch_schedule &S) {
    if (!probs || count <= 0) return fail(USTD_EINVAL, "empty batch");
    long long o = 0, want_rec = 0, min_rec = 0, want_tiles = 0;
    bool bounded = true;
    B.lds_bits = S.layout == USTD_LAYOUT_AUTO;
    for (int i = 0; i < count; ++i) {
        const int rc = check_problem(&probs[i]);
        if (rc != USTD_OK) {
            const std::string m = g_err;
            return fail(rc, "problem %d: %s", i, m.c_str());
        }
        if (probs[i].wilson_variant != USTD_WILSON_PLAIN)
            return fail(USTD_EINVAL, "problem %d: a batch samples with the plain Wilson variant only", i);
        B.lds_bits = B.lds_bits && make_plan(&probs[i], false).lds_bits;
    }
    // one sampler variant serves every member: without the LDS bitmap all need edge entries
    for (int i = 0; i < count; ++i) {
        const Plan L = make_plan(&probs[i], false, !B.lds_bits);
        B.g.push_back(L);
        B.base.push_back(o);
        o += align_up(L.total);
        B.col16 = B.col16 && L.col16;
        B.nwords_max = std::max(B.nwords_max, L.nwords);
        const long long rb = L.rec_stride * 8;
        min_rec = std::max(min_rec, rb);
        long long cap = probs[i].tau_override > 0 ? probs[i].tau_override : probs[i].tau_cap;
        if (probs[i].trees_per_batch > 0) cap = cap > 0 ? std::min<long long>(cap, probs[i].trees_per_batch)
                                                        : probs[i].trees_per_batch;
        if (cap > 0) {
            want_rec += cap * rb;
            want_tiles += cap;
        } else {
            bounded = false;
        }
    }
    B.max_tiles = std::max(1ll, std::min(bounded ? want_tiles : kMaxBatchTiles, kMaxBatchTiles));
    if (S.fill_trees > 0) B.max_tiles = std::min<long long>(B.max_tiles, S.fill_trees);
    B.slots = (int)std::min<long long>(kSamplerMaxBlocks, B.max_tiles);
    // path slots per launch stream, for any schedule: a launch never has more blocks than the
    // batch has tiles, and each of up to kMaxBranches chains gets at least one slot
    const long long tile_bound = std::min(bounded ? want_tiles : kMaxBatchTiles, kMaxBatchTiles);
    B.path_slots = std::max<long long>(std::min<long long>(kSamplerMaxBlocks, tile_bound), kMaxBranches);
    const long long slot_bytes = 2 * B.path_slots * kSamplerPathSlot * 4;
    long long pool = std::max(kDefaultBudget - slot_bytes, min_rec);
    if (bounded) pool = std::min(pool, std::max(want_rec, min_rec));
    B.rec_pool = align_up(pool);
    auto take = [&](long long bytes) {
        const long long at = o;
        o += align_up(bytes);
        return at;
    };
    B.off_queue = take(kMaxBranches * sizeof(int));
    B.off_rec = take(B.rec_pool);
    B.off_path = take(2 * B.path_slots * kSamplerPathSlot * 4);  // two launch streams
    B.off_steps = take(std::min(bounded ? want_tiles : kMaxBatchTiles, kMaxBatchTiles) * 8);
    B.off_draws = take(std::min(bounded ? want_tiles : kMaxBatchTiles, kMaxBatchTiles) * 8);
    B.total = o;
    return USTD_OK;
}

// the workspace of a batch: enough for every schedule (the records layout needs edge entries)
int batch_workspace(const ustd_problem *probs, int count, long long *bytes) {
    BatchPlan a, b;
    ustd_batch_schedule s = schedule_of(nullptr);
    USTD_TRY(make_batch_plan(probs, count, a, s));
    s.layout = USTD_LAYOUT_RECORDS;
    USTD_TRY(make_batch_plan(probs, count, b, s));
    *bytes = std::max(a.total, b.total);
    return USTD_OK;
}

int member(int i, int rc) {
    if (rc == USTD_OK) return rc;
    const std::string m = g_err;
    return fail(rc, "problem %d: %s", i, m.c_str());
}

// the pieces of a planned batch: a run of tiles of one pool fill sampled by one persistent
// launch (a group), the members' trees in it (segments, for Algorithm 2), and the fills
struct BatchSeg {
    int graph;
    long long ntrees, rec_off;
};
struct BatchGroup {
    int t0, cnt;  // tiles of the fill
    bool weighted;
    int branch;  // chain of a batch split into branches, else -1
    std::vector<BatchSeg> segs;
};
struct BatchFill {
    long long tile0;  // first tile in the plan's tile table
    int ntiles;
    std::vector<BatchGroup> groups;
};

// Re-enqueues a member's set-up with the pivot and eccentricity its plan found (no host round
// trip): the CSR views and heavy-row list, the BFS tree B_u (ecc levels), its intervals and
// marks, the sampler's edge entries, and a weighted graph's row sums, B-path resistances and
// edge factors at the planned fixed-point shift.  The kernels are deterministic, so the
// workspace ends as the plan's set-up left it.
int setup_replay(Ctx &c) {
    const ustd_problem *p = c.p;
    const Plan &L = c.L;
    const int n = L.n;
    hipStream_t st = c.st;
    void *ws = c.ws;
    HIP_TRY(launch_rp_to_i32(n, (const long long *)p->d_row_ptr, c.rp32, st));
    if (L.col16) HIP_TRY(launch_col_to_u16(L.nnz, p->d_col, at<unsigned short>(ws, L.off_col16), st));
    HIP_TRY(launch_heavy_list(n, c.rp32, L.heavy_thresh, at<int>(ws, L.off_bcount), at<int>(ws, L.off_heavy),
                              &c.misc->nheavy, st));
    if (L.weighted)
        HIP_TRY(launch_row_cumsum(n, L.nnz, c.rp32, p->d_weight, L.heavy_thresh, c.rows.heavy, c.rows.nheavy,
                                  at<double>(ws, L.off_cw), at<double>(ws, L.off_wdeg), at<int>(ws, L.off_guide), st));
    int *dist = at<int>(ws, L.off_dist), *parB = at<int>(ws, L.off_parB);
    if (n <= kSmallSolveMaxN) {
        HIP_TRY(launch_setup_small(c.rows, L.G, c.pivot, dist, parB, at<int>(ws, L.off_scr), at<int2>(ws, L.off_bint),
                                   at<int>(ws, L.off_bflag), c.misc->setup_out, st));
    } else {
        HIP_TRY(launch_bfs_init(n, c.pivot, dist, parB, st));
        for (int d = 0; d < c.ecc; ++d)
            HIP_TRY(launch_bfs_level(c.rows, L.G, d, dist, parB, &c.misc->bfs_found[0], nullptr, st));
        HIP_TRY(launch_b_intervals(n, c.pivot, c.ecc, dist, parB, at<int>(ws, L.off_scr), at<int2>(ws, L.off_bint),
                                   at<int>(ws, L.off_bflag), st));
    }
    if (L.edges) {
        HIP_TRY(launch_vertex_rows(n, c.rp32, at<int>(ws, L.off_bflag), at<int4>(ws, L.off_vrow), st));
        HIP_TRY(launch_edge_rows(L.nnz, p->d_col, at<int4>(ws, L.off_vrow), at<int4>(ws, L.off_edge), st));
    }
    if (L.weighted) {
        double *wB = at<double>(ws, L.off_wB);
        HIP_TRY(launch_fill_i64(1, reinterpret_cast<long long *>(&c.misc->rho_max_bits), 0, st));
        HIP_TRY(launch_bpath(n, c.pivot, c.rp32, p->d_col, p->d_weight, parB, wB, &c.misc->rho_max_bits, st));
        HIP_TRY(launch_fixed_weights(n, c.pivot, wB, c.shift, at<long long>(ws, L.off_F), st));
    }
    return USTD_OK;
}

}  // namespace

// A batch set up once and executed by kernel launches only.
struct ustd_batch_plan {
    int count = 0, device = 0;
    std::vector<ustd_problem> probs;  // copies; the contexts point here
    BatchPlan B;
    ustd_batch_schedule sched{};
    void *ws = nullptr;
    std::vector<Ctx> cs;
    std::vector<long long> tau;
    std::vector<ustd_report> setup_rep;  // what the set-up fixed, per member
    std::vector<BatchFill> fills;
    long long largest = 0;  // tiles of the largest fill
    int resident = 0, resident_w = 0;
    // pivot-column solves: one-workgroup members by (precision, row-group size) runs, the
    // others (multi-kernel engine, host-driven)
    std::vector<int> small, big;
    std::vector<std::pair<int, int>> runs64, runs32;  // (row-group size, jobs), in launch order
    std::vector<double> tols;
    std::vector<ustd_report> big_rep;  // solve fields of the host-driven members, last execution
    std::vector<int> big_rc;
    // the plan's device memory: tiles of every fill, graph table, solve jobs, walk totals
    char *dmem = nullptr;
    WilsonTile *d_tiles = nullptr;
    WilsonGraph *d_graphs = nullptr;
    SolveJob<double> *d_j64 = nullptr;
    SolveJob<float> *d_j32 = nullptr;
    unsigned long long *d_totals = nullptr;
    // captured graphs of this plan still alive (they use the plan's device memory)
    int live_graphs = 0;
    // timers of the last eager execution
    bool timed = false;
    std::vector<std::unique_ptr<SpanTimer>> ts, ta;
    std::unique_ptr<SpanTimer> t_solve, t_combine, t_total;
    ~ustd_batch_plan() {
        if (dmem) (void)hipFree(dmem);
    }
};

namespace {

// an instantiated capture of one execution, and the plan whose memory it uses
struct BatchGraph {
    hipGraphExec_t ex;
    ustd_batch_plan *plan;
};

// Set-up of every member (with host readbacks: validation, pivot, eccentricity, tau), the
// schedule of tiles over pool fills and sampler groups, the solve jobs, and the plan's device
// memory.  A pool fill takes members in order (unweighted before weighted, then decreasing
// eccentricity: the longest B-paths, so the costliest Algorithm 2, first) as far as the
// record pool and fill_trees allow; a fill is split into groups of whole members of about
// group_fills GPU-fills of trees (one persistent launch each, one kind per launch), each
// group's tiles by decreasing graph size (the longest trees start first), a member's trees in
// order.
int batch_plan_create(const ustd_problem *probs, int count, void *d_ws, size_t ws_bytes,
                      const ustd_batch_schedule *sched, std::unique_ptr<ustd_batch_plan> &out, hipStream_t st) {
    auto P = std::make_unique<ustd_batch_plan>();
    P->sched = schedule_of(sched);
    USTD_TRY(check_schedule(P->sched));
    BatchPlan &B = P->B;
    USTD_TRY(make_batch_plan(probs, count, B, P->sched));
    USTD_TRY(check_ws(d_ws, ws_bytes, B.total));
    HIP_TRY(hipGetDevice(&P->device));
    P->count = count;
    P->probs.assign(probs, probs + count);
    P->ws = d_ws;
    P->cs.resize(count);
    P->tau.assign(count, 0);
    P->setup_rep.assign(count, ustd_report{});
    P->big_rep.assign(count, ustd_report{});
    P->big_rc.assign(count, USTD_OK);
    P->tols.assign(count, 0.0);
    std::vector<WilsonGraph> gt(count);
    for (int i = 0; i < count; ++i) {
        void *wsi = static_cast<char *>(d_ws) + B.base[i];
        Ctx &c = P->cs[i];
        USTD_TRY(member(i, begin_with(c, &P->probs[i], B.g[i], wsi, st)));
        Timer tm(st);
        USTD_TRY(member(i, setup(c, &P->setup_rep[i])));
        P->setup_rep[i].ms_bfs = tm.stop_ms();
        P->tau[i] = problem_tau(c);
        P->setup_rep[i].tau = P->tau[i];
        gt[i] = wilson_graph(c);
        gt[i].colv = B.col16 ? (const void *)at<unsigned short>(wsi, B.g[i].off_col16) : (const void *)probs[i].d_col;
    }
    HIP_TRY(hipStreamSynchronize(st));  // a weighted member's side-stream set-up is joined into st

    // fills and groups
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (B.g[a].weighted != B.g[b].weighted) return !B.g[a].weighted;
        const Ctx &ca = P->cs[a], &cb = P->cs[b];
        return ca.ecc != cb.ecc ? ca.ecc > cb.ecc : B.g[a].n > B.g[b].n;
    });
    P->resident = wilson_resident_blocks(B.lds_bits, B.col16, false, B.nwords_max);
    P->resident_w = wilson_resident_blocks(B.lds_bits, B.col16, true, B.nwords_max);
    const long long group_trees =
        P->sched.group_fills > 0 ? (long long)P->sched.group_fills * std::max(P->resident, 1) : LLONG_MAX;
    std::vector<WilsonTile> tiles;
    std::vector<long long> next(count, 0);
    for (;;) {
        std::vector<std::pair<int, long long>> part;  // members of this fill, with their tree counts
        long long used = 0, ntiles = 0;
        for (int gi : order) {
            const long long left = P->tau[gi] - next[gi];
            if (left <= 0) continue;
            const long long rb = B.g[gi].rec_stride * 8;
            const long long fit = std::min((B.rec_pool - used) / rb, B.max_tiles - ntiles);
            const long long lim = probs[gi].trees_per_batch > 0 ? probs[gi].trees_per_batch : left;
            const long long take = std::min(std::min(left, fit), lim);
            if (take <= 0) break;
            part.emplace_back(gi, take);
            used += take * rb;
            ntiles += take;
        }
        if (part.empty()) break;
        BatchFill F{(long long)tiles.size(), 0, {}};
        long long rec_used = 0;
        // the fill's members in launch groups: runs of `order` (alternating groups), or each
        // branch's members of one kind (branches; members to the least loaded branch, largest
        // estimated work first: tau (n ecc + nnz), walks and Algorithm 2)
        std::vector<std::pair<int, std::vector<std::pair<int, long long>>>> runs;  // (branch, members)
        if (P->sched.branches >= 2) {
            const int nb = P->sched.branches;
            std::vector<std::pair<double, size_t>> work;
            for (size_t k = 0; k < part.size(); ++k) {
                const Plan &L = B.g[part[k].first];
                work.emplace_back((double)part[k].second *
                                      ((double)L.n * (double)std::max(P->cs[part[k].first].ecc, 1) + (double)L.nnz),
                                  k);
            }
            std::stable_sort(work.begin(), work.end(),
                             [](const std::pair<double, size_t> &a, const std::pair<double, size_t> &b) {
                                 return a.first > b.first;
                             });
            std::vector<double> load(nb, 0.0);
            std::vector<std::vector<std::pair<int, long long>>> br(2 * nb);  // (branch, kind)
            for (auto &wk : work) {
                const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                load[b] += wk.first;
                br[2 * b + (B.g[part[wk.second].first].weighted ? 1 : 0)].push_back(part[wk.second]);
            }
            for (int b = 0; b < 2 * nb; ++b)
                if (!br[b].empty()) runs.emplace_back(b / 2, br[b]);
        } else {
            for (size_t k = 0; k < part.size();) {
                size_t e = k;
                long long cnt = 0;
                const bool wk = B.g[part[k].first].weighted;
                while (e < part.size() && (e == k || cnt < group_trees) && B.g[part[e].first].weighted == wk)
                    cnt += part[e++].second;
                runs.emplace_back(-1, std::vector<std::pair<int, long long>>(part.begin() + k, part.begin() + e));
                k = e;
            }
        }
        for (auto &run : runs) {
            std::vector<std::pair<int, long long>> &mem = run.second;
            std::stable_sort(mem.begin(), mem.end(), [&](const std::pair<int, long long> &x,
                                                         const std::pair<int, long long> &y) {
                return B.g[x.first].n > B.g[y.first].n;
            });
            BatchGroup G{(int)(tiles.size() - F.tile0), 0, B.g[mem[0].first].weighted, run.first, {}};
            for (auto &pr : mem) {
                const int gi = pr.first;
                const long long take = pr.second;
                G.segs.push_back(BatchSeg{gi, take, rec_used / 8});
                for (long long j = 0; j < take; ++j)
                    tiles.push_back(WilsonTile{next[gi] + j, rec_used / 8 + j * B.g[gi].rec_stride, gi, 0});
                rec_used += take * B.g[gi].rec_stride * 8;
                next[gi] += take;
            }
            G.cnt = (int)(tiles.size() - F.tile0) - G.t0;
            F.groups.push_back(std::move(G));
        }
        F.ntiles = (int)(tiles.size() - F.tile0);
        P->largest = std::max<long long>(P->largest, F.ntiles);
        P->fills.push_back(std::move(F));
    }

    // solves: members on the one-workgroup engine (all by default) in one launch per precision
    // and row-group size, a workgroup each; the others by the host-driven multi-kernel loop
    std::vector<SolveJob<double>> j64;
    std::vector<SolveJob<float>> j32;
    for (int i = 0; i < count; ++i) {
        P->tols[i] = solve_target(&P->probs[i], P->cs[i].ecc);
        (one_workgroup(&P->probs[i], B.g[i].n, true) ? P->small : P->big).push_back(i);
    }
    for (int mixed = 0; mixed < 2; ++mixed)
        for (int G : {4, 8, 16, 32}) {
            int cnt = 0;
            for (int i : P->small) {
                Ctx &c = P->cs[i];
                const bool mx = c.p->solve_mode == USTD_SOLVE_MIXED;
                if (c.L.G != G || (int)mx != mixed) continue;
                const double tol = P->tols[i];
                const int maxit = c.p->solve_maxit > 0 ? c.p->solve_maxit : 20000;
                double *x = at<double>(c.ws, B.g[i].off_x64);
                if (mx) j32.push_back(SolveJob<float>{solve_args<float>(c, c.ws, c.L, x), c.rows, tol * tol,
                                                      solve_delta2(c.p), maxit});
                else j64.push_back(SolveJob<double>{solve_args<double>(c, c.ws, c.L, x), c.rows, tol * tol,
                                                    solve_delta2(c.p), maxit});
                ++cnt;
            }
            if (cnt) (mixed ? P->runs32 : P->runs64).emplace_back(G, cnt);
        }
    if (j64.size() + j32.size() != P->small.size())
        return fail(USTD_EINVAL, "unexpected row-group size in a batched solve");

    // device memory of the plan
    const long long b_tiles = align_up((long long)std::max<size_t>(tiles.size(), 1) * sizeof(WilsonTile));
    const long long b_graphs = align_up((long long)count * sizeof(WilsonGraph));
    const long long b_j64 = align_up((long long)std::max<size_t>(j64.size(), 1) * sizeof(SolveJob<double>));
    const long long b_j32 = align_up((long long)std::max<size_t>(j32.size(), 1) * sizeof(SolveJob<float>));
    const long long b_tot = align_up((long long)count * 2 * sizeof(unsigned long long));
    if (hipMalloc((void **)&P->dmem, (size_t)(b_tiles + b_graphs + b_j64 + b_j32 + b_tot)) != hipSuccess) {
        (void)hipGetLastError();
        P->dmem = nullptr;
        return fail(USTD_ENOMEM, "plan memory of %lld bytes", b_tiles + b_graphs + b_j64 + b_j32 + b_tot);
    }
    P->d_tiles = reinterpret_cast<WilsonTile *>(P->dmem);
    P->d_graphs = reinterpret_cast<WilsonGraph *>(P->dmem + b_tiles);
    P->d_j64 = reinterpret_cast<SolveJob<double> *>(P->dmem + b_tiles + b_graphs);
    P->d_j32 = reinterpret_cast<SolveJob<float> *>(P->dmem + b_tiles + b_graphs + b_j64);
    P->d_totals = reinterpret_cast<unsigned long long *>(P->dmem + b_tiles + b_graphs + b_j64 + b_j32);
    if (!tiles.empty())
        HIP_TRY(hipMemcpy(P->d_tiles, tiles.data(), sizeof(WilsonTile) * tiles.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(P->d_graphs, gt.data(), sizeof(WilsonGraph) * (size_t)count, hipMemcpyHostToDevice));
    if (!j64.empty())
        HIP_TRY(hipMemcpy(P->d_j64, j64.data(), sizeof(SolveJob<double>) * j64.size(), hipMemcpyHostToDevice));
    if (!j32.empty())
        HIP_TRY(hipMemcpy(P->d_j32, j32.data(), sizeof(SolveJob<float>) * j32.size(), hipMemcpyHostToDevice));
    out = std::move(P);
    return USTD_OK;
}

// the one-workgroup solves, then every such member's projection and final residual, on st
int enqueue_small_solves(ustd_batch_plan &P, std::vector<Ctx> &cs, hipStream_t st) {
    int off = 0;
    for (auto &r : P.runs64) {
        HIP_TRY(launch_solve_small_batch<double>(P.d_j64 + off, r.second, r.first, st));
        off += r.second;
    }
    off = 0;
    for (auto &r : P.runs32) {
        HIP_TRY(launch_solve_small_batch<float>(P.d_j32 + off, r.second, r.first, st));
        off += r.second;
    }
    for (int i : P.small) {
        Ctx &c = cs[i];
        double *x64 = at<double>(c.ws, P.B.g[i].off_x64);
        double *part = at<double>(c.ws, c.L.off_part) + 3 * kMaxSolveGrid;
        double *sums = c.misc->sums;
        HIP_TRY(launch_residual64(c.rows, c.L.G, c.pivot, x64, nullptr, part, sums, st));
        HIP_TRY(launch_project(c.L.n, x64, sums + 2, vec_grid(c.L.n), st));
        HIP_TRY(launch_residual64(c.rows, c.L.G, c.pivot, x64, nullptr, part, sums, st));
    }
    return USTD_OK;
}

// One execution: the members' set-up replayed on st; then, beside each other, the solves on
// side stream 0, the sampler groups alternating between st and side stream 1 and each
// group's Algorithm 2 on side stream 2; a pool fill starts once the previous one's groups
// and Algorithm 2 are done (they share the record pool); all streams join st before the
// combination.  No host wait unless a member uses the host-driven solve engine (eager only).
int batch_plan_execute(ustd_batch_plan &P, double *const *d_diags, int64_t *const *d_counts, hipStream_t st) {
    if (!d_diags) return fail(USTD_EINVAL, "d_diags is NULL");
    for (int i = 0; i < P.count; ++i)
        if (!d_diags[i]) return fail(USTD_EINVAL, "d_diags[%d] is NULL", i);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != P.device) return fail(USTD_EINVAL, "plan made on device %d, current device %d", P.device, dev);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cap));
    const bool capturing = cap != hipStreamCaptureStatusNone;
    if (capturing && !P.big.empty())
        return fail(USTD_EINVAL, "problem %d uses the multi-kernel solve engine, which the host drives: it cannot be "
                                 "captured", P.big[0]);
    const bool timed = !capturing && !g_no_events;
    P.timed = timed;
    P.ts.clear();
    P.ta.clear();
    P.t_solve.reset();
    P.t_combine.reset();
    P.t_total.reset();
    if (timed) {
        P.t_solve.reset(new SpanTimer());
        P.t_combine.reset(new SpanTimer());
        P.t_total.reset(new SpanTimer());
        P.t_total->start(st);
    }
    const BatchPlan &B = P.B;
    std::vector<Ctx> cs = P.cs;
    std::vector<long long *> counts(P.count);
    for (int i = 0; i < P.count; ++i) {
        Ctx &c = cs[i];
        c.st = st;
        counts[i] = (d_counts && d_counts[i]) ? (long long *)d_counts[i] : at<long long>(c.ws, B.g[i].off_counts);
        USTD_TRY(member(i, setup_replay(c)));
        HIP_TRY(launch_fill_i64(B.g[i].n, counts[i], 0, st));
    }
    HIP_TRY(launch_fill_i64(2ll * P.count, reinterpret_cast<long long *>(P.d_totals), 0, st));

    hipStream_t side = nullptr, samp1 = nullptr, aggq = nullptr, br3 = nullptr;
    USTD_TRY(side_stream(&side, 0));
    USTD_TRY(side_stream(&samp1, 1));
    USTD_TRY(side_stream(&aggq, 2));
    USTD_TRY(side_stream(&br3, 3));
    const int nbr = P.sched.branches;
    const hipStream_t br[kMaxBranches] = {st, samp1, aggq, br3};  // the chains of branch mode
    std::vector<std::unique_ptr<SyncEvent>> evs;  // kept until every wait on them is queued
    auto event = [&](hipStream_t s) -> hipEvent_t {
        evs.emplace_back(new SyncEvent());
        hipEvent_t e = evs.back()->e;
        if (e && hipEventRecord(e, s) != hipSuccess) return nullptr;
        return e;
    };
    auto wait = [&](hipStream_t s, hipEvent_t e) { return e && hipStreamWaitEvent(s, e, 0) == hipSuccess; };
    hipEvent_t fork = event(st);
    if (!wait(side, fork) || !wait(samp1, fork) || !wait(aggq, fork) || (nbr >= 4 && !wait(br3, fork)))
        return fail(USTD_EHIP, "forking the batch streams failed");
    if (timed) P.t_solve->start(side);
    USTD_TRY(enqueue_small_solves(P, cs, side));

    int2 *pool = at<int2>(P.ws, B.off_rec);
    long long *steps = at<long long>(P.ws, B.off_steps), *draws = at<long long>(P.ws, B.off_draws);
    int *queue = at<int>(P.ws, B.off_queue);
    for (size_t f = 0; f < P.fills.size(); ++f) {
        const BatchFill &F = P.fills[f];
        if (f > 0) {  // the previous fill's groups and Algorithm 2 are done with the record pool
            if (!wait(st, event(samp1)) || !wait(st, event(aggq)) || (nbr >= 4 && !wait(st, event(br3))))
                return fail(USTD_EHIP, "joining a pool fill failed");
            hipEvent_t ready = event(st);
            if (!wait(samp1, ready) || !wait(aggq, ready) || (nbr >= 4 && !wait(br3, ready)))
                return fail(USTD_EHIP, "starting a pool fill failed");
        }
        for (size_t gidx = 0; gidx < F.groups.size(); ++gidx) {
            const BatchGroup &G = F.groups[gidx];
            // alternating groups: streams st / 1, sampler scratch and tile counter by parity;
            // branches: the branch's stream, scratch and counter (Algorithm 2 on that stream)
            const int pool2 = G.branch >= 0 ? G.branch : (int)(gidx & 1);
            hipStream_t s = G.branch >= 0 ? br[G.branch] : (pool2 ? samp1 : st);
            hipStream_t sa = G.branch >= 0 ? s : aggq;
            WilsonArgs a{};
            a.graphs = P.d_graphs;
            a.tiles = P.d_tiles + F.tile0 + G.t0;
            a.ntiles = G.cnt;
            a.rec = pool;
            // sampler path slots: path_slots per stream of alternating groups; a branch's launch
            // has at most path_slots / branches blocks and takes that share of the first stream's
            const long long share = G.branch >= 0 ? B.path_slots / nbr : B.path_slots;
            const long long slot0 = G.branch >= 0 ? (long long)G.branch * share : (long long)pool2 * B.path_slots;
            a.path = at<int>(P.ws, B.off_path) + slot0 * kSamplerPathSlot;
            a.queue = queue + pool2;
            a.steps = steps + G.t0;
            a.draws = draws + G.t0;
            const int res = G.weighted ? P.resident_w : P.resident;
            int blocks = std::min(G.cnt, B.slots);
            if (res > 0) blocks = std::min(blocks, res);
            if (G.branch >= 0) blocks = std::max(1, std::min(blocks, std::min(res > 0 ? res : kSamplerMaxBlocks,
                                                                                  kSamplerMaxBlocks) / nbr));
            blocks = (int)std::min<long long>(blocks, share);  // within the launch's path slots
            if (timed) {
                P.ts.emplace_back(new SpanTimer());
                P.ts.back()->start(s);
            }
            HIP_TRY(launch_fill_i32(1, queue + pool2, 0, s));
            HIP_TRY(launch_wilson(a, blocks, B.lds_bits, B.col16, G.weighted, B.nwords_max, s));
            if (timed) P.ts.back()->stop(s);
            HIP_TRY(launch_tile_walks(G.cnt, a.tiles, a.steps, a.draws, P.d_totals, s));
            if (sa != s && !wait(sa, event(s)))
                return fail(USTD_EHIP, "ordering Algorithm 2 after a sampler group failed");
            if (timed) {
                P.ta.emplace_back(new SpanTimer());
                P.ta.back()->start(sa);
            }
            for (const BatchSeg &sg : G.segs) {
                const Ctx &c = cs[sg.graph];
                const Plan &L = B.g[sg.graph];
                AggregateArgs aa{};
                aa.n = L.n;
                aa.u = c.pivot;
                aa.ntrees = (int)sg.ntrees;
                aa.parB = at<int>(c.ws, L.off_parB);
                aa.bint = at<int2>(c.ws, L.off_bint);
                aa.rec = pool + sg.rec_off;
                aa.rec_stride = L.rec_stride;
                aa.counts = counts[sg.graph];
                aa.F = L.weighted ? at<long long>(c.ws, L.off_F) : nullptr;
                agg_form(aa, c.ecc, P.sched.agg_chunk);
                HIP_TRY(launch_aggregate(aa, sa));
            }
            if (timed) P.ta.back()->stop(sa);
        }
    }
    // members on the host-driven engine: every fill is queued, the GPU samples meanwhile
    for (int i : P.big) {
        Ctx ci = cs[i];
        ci.st = side;
        ustd_report r{};
        const int rc = solve_column(ci, at<double>(ci.ws, B.g[i].off_x64), &r);
        if (rc != USTD_OK && rc != USTD_ENOTCONV) {
            (void)hipStreamSynchronize(side);
            return member(i, rc);
        }
        P.big_rep[i] = r;
        P.big_rc[i] = rc;
    }
    if (timed) P.t_solve->stop(side);
    if (!wait(st, event(side)) || !wait(st, event(samp1)) || !wait(st, event(aggq)) ||
        (nbr >= 4 && !wait(st, event(br3))))
        return fail(USTD_EHIP, "joining the batch streams failed");
    if (timed) P.t_combine->start(st);
    for (int i = 0; i < P.count; ++i)
        HIP_TRY(launch_combine(B.g[i].n, cs[i].pivot, count_scale(cs[i], P.tau[i]), counts[i],
                               at<double>(cs[i].ws, B.g[i].off_x64), d_diags[i], st));
    if (timed) {
        P.t_combine->stop(st);
        P.t_total->stop(st);
    }
    return USTD_OK;
}

// reports of the last execution; synchronises st
int batch_plan_reports(ustd_batch_plan &P, ustd_report *R, hipStream_t st) {
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<unsigned long long> tot(2 * (size_t)P.count);
    HIP_TRY(hipMemcpy(tot.data(), P.d_totals, sizeof(unsigned long long) * tot.size(), hipMemcpyDeviceToHost));
    double ms_s = 0, ms_a = 0;
    for (auto &t : P.ts) ms_s += t->ms();
    for (auto &t : P.ta) ms_a += t->ms();
    const double ms_solve = P.timed && P.t_solve ? P.t_solve->ms() : 0.0;
    const double ms_comb = P.timed && P.t_combine ? P.t_combine->ms() : 0.0;
    const double ms_tot = P.timed && P.t_total ? P.t_total->ms() : 0.0;
    int status = USTD_OK;
    for (int i = 0; i < P.count; ++i) {
        ustd_report &r = R[i];
        r = P.setup_rep[i];
        r.walk_steps = (long long)tot[2 * i];
        r.walk_draws = (long long)tot[2 * i + 1];
        r.n_batches = (int32_t)P.fills.size();
        r.trees_per_batch = (int32_t)P.largest;
        r.ms_sample = ms_s;
        r.ms_aggregate = ms_a;
        r.ms_combine = ms_comb / (double)P.count;
        r.ms_total = ms_tot;
        r.solve_tol = P.tols[i];
        if (std::find(P.big.begin(), P.big.end(), i) != P.big.end()) {
            const ustd_report &b = P.big_rep[i];
            r.solve_iters = b.solve_iters;
            r.solve_outer = b.solve_outer;
            r.solve_relres = b.solve_relres;
            r.solve_converged = b.solve_converged;
            r.ms_solve = b.ms_solve;
            if (P.big_rc[i] != USTD_OK && status == USTD_OK)
                status = member(i, fail(P.big_rc[i], "solve stopped at relative residual %.3e (target %.3e)",
                                        b.solve_relres, P.tols[i]));
            continue;
        }
        const Ctx &c = P.cs[i];
        SolveScalars sc{};
        double hs[4];
        HIP_TRY(hipMemcpy(&sc, &c.misc->sc, sizeof(sc), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(hs, c.misc->sums, sizeof(hs), hipMemcpyDeviceToHost));
        const double bnorm = std::sqrt((double)(c.L.n - 1) / (double)c.L.n);
        const double relres = std::sqrt(std::max(hs[1], 0.0)) / bnorm;
        const bool conv = relres <= P.tols[i];
        r.solve_iters = sc.iter;
        r.solve_outer = sc.updates;
        r.solve_relres = relres;
        r.solve_converged = conv ? 1 : 0;
        r.ms_solve = P.small.empty() ? 0.0 : ms_solve / (double)P.small.size();
        if (!conv && status == USTD_OK)
            status = member(i, fail(USTD_ENOTCONV, "solve stopped at relative residual %.3e (target %.3e)", relres,
                                    P.tols[i]));
    }
    return status;
}

// ---------------------------------------------------------------------------------------
// autotuner cache: a JSON object of schedules keyed by the batch's shape and the device,
// one entry per line, {"key": {"group_fills": g, "agg_chunk": c, "layout": l, "branches": b, "fill_trees": f,
// "ms": t}}
// ---------------------------------------------------------------------------------------
struct TuneEntry {
    ustd_batch_schedule s{};
    double ms = 0.0;
};

bool json_number(const std::string &obj, const char *name, double *v) {
    const std::string k = std::string("\"") + name + "\"";
    const size_t at_ = obj.find(k);
    if (at_ == std::string::npos) return false;
    size_t c = obj.find(':', at_ + k.size());
    if (c == std::string::npos) return false;
    char *end = nullptr;
    const double x = std::strtod(obj.c_str() + c + 1, &end);
    if (end == obj.c_str() + c + 1) return false;
    *v = x;
    return true;
}

// entries of the cache file (missing or unreadable: none); malformed entries are skipped
std::vector<std::pair<std::string, TuneEntry>> read_tune_cache(const std::string &path) {
    std::vector<std::pair<std::string, TuneEntry>> out;
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return out;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
    std::fclose(f);
    size_t pos = 0;
    for (;;) {
        const size_t q0 = text.find('"', pos);
        if (q0 == std::string::npos) break;
        const size_t q1 = text.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        const size_t b0 = text.find('{', q1);
        const size_t b1 = b0 == std::string::npos ? b0 : text.find('}', b0);
        if (b1 == std::string::npos) break;
        const std::string key = text.substr(q0 + 1, q1 - q0 - 1), obj = text.substr(b0, b1 - b0 + 1);
        pos = b1 + 1;
        double g = 0, c = 0, l = 0, ft = 0, ms = 0, nb = 0;
        if (!json_number(obj, "group_fills", &g) || !json_number(obj, "agg_chunk", &c) ||
            !json_number(obj, "layout", &l) || !json_number(obj, "fill_trees", &ft))
            continue;
        json_number(obj, "ms", &ms);
        json_number(obj, "branches", &nb);
        TuneEntry e;
        e.s.branches = (int32_t)nb;
        e.s.group_fills = (int32_t)g;
        e.s.agg_chunk = (int32_t)c;
        e.s.layout = (int32_t)l;
        e.s.fill_trees = (int64_t)ft;
        e.ms = ms;
        out.emplace_back(key, e);
    }
    return out;
}

int write_tune_cache(const std::string &path, const std::vector<std::pair<std::string, TuneEntry>> &entries) {
    const std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(USTD_EINVAL, "cannot write the tuning cache %s", tmp.c_str());
    std::fprintf(f, "{\n");
    for (size_t i = 0; i < entries.size(); ++i) {
        const TuneEntry &e = entries[i].second;
        std::fprintf(f, "  \"%s\": {\"group_fills\": %d, \"agg_chunk\": %d, \"layout\": %d, \"branches\": %d, "
                        "\"fill_trees\": %lld, \"ms\": %.3f}%s\n",
                     entries[i].first.c_str(), e.s.group_fills, e.s.agg_chunk, e.s.layout, e.s.branches,
                     (long long)e.s.fill_trees, e.ms, i + 1 < entries.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0)
        return fail(USTD_EINVAL, "cannot write the tuning cache %s", path.c_str());
    return USTD_OK;
}

// the cache key: device architecture and compute units, then each member's n, nnz, tau, ecc
// and weightedness, hashed (FNV-1a, 64 bits)
int tune_key(const ustd_batch_plan &P, std::string *key) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    std::string d;
    char buf[128];
    for (int i = 0; i < P.count; ++i) {
        std::snprintf(buf, sizeof(buf), "%lld,%lld,%lld,%d,%d;", (long long)P.probs[i].n, (long long)P.probs[i].nnz,
                      P.tau[i], P.cs[i].ecc, P.B.g[i].weighted ? 1 : 0);
        d += buf;
    }
    unsigned long long h = 1469598103934665603ull;
    for (unsigned char ch : d) {
        h ^= ch;
        h *= 1099511628211ull;
    }
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    std::snprintf(buf, sizeof(buf), "%s-cu%d-m%d-%016llx", arch.c_str(), prop.multiProcessorCount, P.count, h);
    *key = buf;
    return USTD_OK;
}

// ---------------------------------------------------------------------------------------
// the allocation-free entry point's scratch: a file-scope device array that each GPU holds
// from the library's load until the process ends.  Host code never uses the array's name
// as an address: its device address is taken once per device with hipGetSymbolAddress.
// ---------------------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = USTD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

int static_scratch(void **out) {
    static std::mutex mu;
    static std::vector<void *> ptrs;  // per device
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
    if (!ptrs[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(USTD_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        if ((reinterpret_cast<uintptr_t>(ptr) & (kAlign - 1)) != 0)
            return fail(USTD_EHIP, "static scratch is not 256-byte aligned");
        ptrs[dev] = ptr;
    }
    *out = ptrs[dev];
    return USTD_OK;
}

// the problem as the allocation-free entry point runs it: the one-workgroup solve engine and
// the most trees per batch (at most kMaxTreesPerBatch) whose workspace fits the static scratch
int fit_static(const ustd_problem *prob, ustd_problem *q, Plan *L) {
    *q = *prob;
    q->solve_engine = USTD_ENGINE_WORKGROUP;
    if (prob->trees_per_batch > 0) {
        *L = make_plan(q);
        if ((size_t)L->total > kStaticScratchBytes)
            return fail(USTD_ENOMEM, "the problem needs %lld bytes of scratch at %d trees per batch; the static "
                                     "scratch holds %zu", L->total, prob->trees_per_batch, kStaticScratchBytes);
        return USTD_OK;
    }
    q->trees_per_batch = 1;
    *L = make_plan(q);
    if ((size_t)L->total > kStaticScratchBytes)
        return fail(USTD_ENOMEM, "the problem needs %lld bytes of scratch even at one tree per batch; the static "
                                 "scratch holds %zu", L->total, kStaticScratchBytes);
    int lo = 1, hi = kMaxTreesPerBatch;  // largest K whose plan fits
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        q->trees_per_batch = mid;
        if ((size_t)make_plan(q).total <= kStaticScratchBytes) lo = mid;
        else hi = mid - 1;
    }
    q->trees_per_batch = lo;
    *L = make_plan(q);
    return USTD_OK;
}

}  // namespace

// =========================================================================================
// C ABI
// =========================================================================================
extern "C" {

int ustd_workspace_bytes(const ustd_problem *prob, size_t *bytes) {
    g_err.clear();
    USTD_TRY(check_problem(prob));
    if (!bytes) return fail(USTD_EINVAL, "bytes is NULL");
    *bytes = (size_t)make_plan(prob).total;
    return USTD_OK;
}

int ustd_bfs(const ustd_problem *prob, void *d_ws, size_t ws_bytes, int32_t *d_dist, int32_t *d_parB,
             int32_t *ecc_out, int32_t *pivot_out, void *stream) {
    g_err.clear();
    Ctx c;
    USTD_TRY(begin(c, prob, d_ws, ws_bytes, stream));
    USTD_TRY(setup(c, nullptr));
    const size_t nb = (size_t)c.L.n * 4;
    if (d_dist) HIP_TRY(hipMemcpyAsync(d_dist, at<int>(c.ws, c.L.off_dist), nb, hipMemcpyDeviceToDevice, c.st));
    if (d_parB) HIP_TRY(hipMemcpyAsync(d_parB, at<int>(c.ws, c.L.off_parB), nb, hipMemcpyDeviceToDevice, c.st));
    if (ecc_out) *ecc_out = c.ecc;
    if (pivot_out) *pivot_out = c.pivot;
    HIP_TRY(hipStreamSynchronize(c.st));
    return USTD_OK;
}

int ustd_sample_trees(const ustd_problem *prob, int64_t tree_begin, int64_t tree_count, void *d_ws,
                      size_t ws_bytes, int32_t *d_parents, int64_t *d_steps, void *stream) {
    g_err.clear();
    Ctx c;
    USTD_TRY(begin(c, prob, d_ws, ws_bytes, stream));
    if (tree_begin < 0 || tree_count < 0) return fail(USTD_EINVAL, "negative tree range");
    if (tree_count > c.L.K) return fail(USTD_EINVAL, "tree_count %lld exceeds trees per batch %d", (long long)tree_count, c.L.K);
    if (!d_parents && tree_count > 0) return fail(USTD_EINVAL, "d_parents is NULL");
    USTD_TRY(setup(c, nullptr));
    if (tree_count == 0) return USTD_OK;
    long long *steps = d_steps ? (long long *)d_steps : at<long long>(c.ws, c.L.off_steps);
    USTD_TRY(sample_batch(c, tree_begin, (int)tree_count, steps, at<long long>(c.ws, c.L.off_draws)));
    HIP_TRY(launch_extract_parents(c.L.n, (int)tree_count, at<int2>(c.ws, c.L.off_rec), c.L.rec_stride, d_parents, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    return USTD_OK;
}

int ustd_flow_counts(const ustd_problem *prob, int64_t tree_begin, int64_t tree_count, void *d_ws,
                     size_t ws_bytes, int64_t *d_counts, ustd_report *rep, void *stream) {
    g_err.clear();
    Ctx c;
    USTD_TRY(begin(c, prob, d_ws, ws_bytes, stream));
    if (tree_begin < 0 || tree_count < 0) return fail(USTD_EINVAL, "negative tree range");
    if (!d_counts) return fail(USTD_EINVAL, "d_counts is NULL");
    if (rep) memset(rep, 0, sizeof(*rep));
    Timer total(c.st);
    USTD_TRY(setup(c, rep));
    USTD_TRY(check_fixed_point_range(c, tree_count));
    USTD_TRY(run_trees(c, tree_begin, tree_count, (long long *)d_counts, rep));
    if (rep) {
        rep->tau = tree_count;
        rep->ms_total = total.stop_ms();
    }
    return USTD_OK;
}

int ustd_tree_counts(const ustd_problem *prob, const int32_t *d_parents, int64_t tree_count, void *d_ws,
                     size_t ws_bytes, int64_t *d_counts, void *stream) {
    g_err.clear();
    Ctx c;
    USTD_TRY(begin(c, prob, d_ws, ws_bytes, stream));
    if (tree_count < 0) return fail(USTD_EINVAL, "negative tree count");
    if ((!d_parents && tree_count > 0) || !d_counts) return fail(USTD_EINVAL, "NULL parents / counts");
    USTD_TRY(setup(c, nullptr));
    USTD_TRY(check_fixed_point_range(c, tree_count));
    // Every batch's parent arrays are checked (tree_records_kernel) before Algorithm 2 reads the
    // records built from them, and the counts go to the workspace first: a parent array that is
    // not a spanning tree rooted at the pivot returns USTD_EINVAL with d_counts unchanged.
    long long *acc = at<long long>(c.ws, c.L.off_counts);
    HIP_TRY(launch_fill_i64(c.L.n, acc, 0, c.st));
    for (long long b0 = 0; b0 < tree_count; b0 += c.L.Kiv) {
        const int cnt = (int)std::min<long long>(c.L.Kiv, tree_count - b0);
        IntervalArgs ia{};
        ia.n = c.L.n;
        ia.u = c.pivot;
        ia.par = d_parents + b0 * c.L.n;
        ia.par_stride = c.L.n;
        ia.scratch = at<int>(c.ws, c.L.off_scr);
        ia.scratch_stride = c.L.scr_stride;
        ia.rec = at<int2>(c.ws, c.L.off_rec);
        ia.rec_stride = c.L.rec_stride;
        ia.bflag = at<int>(c.ws, c.L.off_bflag);
        ia.err = &c.misc->err_interval;
        HIP_TRY(launch_tree_records(ia, cnt, c.st));
        int err = 0;
        HIP_TRY(hipMemcpyAsync(&err, &c.misc->err_interval, sizeof(int), hipMemcpyDeviceToHost, c.st));
        HIP_TRY(hipStreamSynchronize(c.st));
        if (err) return fail(USTD_EINVAL, "parent array of tree %lld..%lld is not a spanning tree rooted at the pivot",
                             b0, b0 + cnt - 1);
        USTD_TRY(aggregate_trees(c, cnt, acc, nullptr));
    }
    HIP_TRY(launch_add_i64(c.L.n, acc, (long long *)d_counts, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    return USTD_OK;
}

int ustd_solve_pivot_column(const ustd_problem *prob, void *d_ws, size_t ws_bytes, double *d_x, ustd_report *rep,
                            void *stream) {
    g_err.clear();
    Ctx c;
    USTD_TRY(begin(c, prob, d_ws, ws_bytes, stream));
    if (!d_x) return fail(USTD_EINVAL, "d_x is NULL");
    if (rep) memset(rep, 0, sizeof(*rep));
    USTD_TRY(setup(c, rep));
    return solve_column(c, d_x, rep);
}

int ustd_diag_lpinv(const ustd_problem *prob, void *d_ws, size_t ws_bytes, double *d_diag, int64_t *d_counts,
                    ustd_report *rep, void *stream) {
    g_err.clear();
    Ctx c;
    USTD_TRY(begin(c, prob, d_ws, ws_bytes, stream));
    if (!d_diag) return fail(USTD_EINVAL, "d_diag is NULL");
    ustd_report local{};
    ustd_report *r = rep ? rep : &local;
    memset(r, 0, sizeof(*r));
    Timer total(c.st);
    USTD_TRY(setup(c, r));
    const long long tau = problem_tau(c);
    r->tau = tau;
    long long *counts = d_counts ? (long long *)d_counts : at<long long>(c.ws, c.L.off_counts);
    HIP_TRY(hipMemsetAsync(counts, 0, (size_t)c.L.n * 8, c.st));
    // The pivot column needs only the graph and the pivot: it is solved on the side stream
    // while the first batch of trees is sampled (the two touch disjoint workspace).
    double *x = at<double>(c.ws, c.L.off_x64);
    hipStream_t side = nullptr;
    USTD_TRY(side_stream(&side));
    SyncEvent fork, join;
    if (!fork.e || !join.e) return fail(USTD_EHIP, "hipEventCreateWithFlags failed");
    HIP_TRY(hipEventRecord(fork.e, c.st));
    HIP_TRY(hipStreamWaitEvent(side, fork.e, 0));
    Ctx cs = c;
    cs.st = side;
    int src = USTD_EHIP;
    bool solved = false;
    // Where the solve overlaps.  The LDS-bitmap sampler leaves registers for the solve's kernels
    // beside it, so the solve runs during sampling.  The records sampler fills every SIMD's
    // registers (96 x 5 waves): solve kernels issued beside it only get slots as its launches
    // drain.  With two tree pools the launches of the two streams overlap and the solve fills
    // their drain gaps, so it still starts at once.  With one pool the batches run back to back
    // on one stream, and which of the solve and the first launch reached the CUs first changed
    // the run time by 13% from call to call (R-MAT scale 22, 19 MB of records per tree): there
    // the solve waits for the last sampler launch and runs beside the last batch's Algorithm 2.
    SyncEvent sampled;
    const bool after_sampling = !c.L.lds_bits && c.L.pools == 1 && sampled.e;
    const int trc = run_trees(c, 0, tau, counts, r, nullptr, [&]() {
        if (after_sampling && hipStreamWaitEvent(side, sampled.e, 0) != hipSuccess) {
            src = fail(USTD_EHIP, "hipStreamWaitEvent failed");
            solved = true;
            return;
        }
        src = solve_column(cs, x, r);
        solved = true;
    }, after_sampling ? sampled.e : nullptr);
    if (!solved) {
        if (trc != USTD_OK) return trc;  // failed before the first sampler launch
        src = solve_column(cs, x, r);
    }
    // the side stream is idle on every return below: solve_column ends with a synchronisation
    // of it, and an early error return is followed by one here
    if (src != USTD_OK && src != USTD_ENOTCONV) {
        (void)hipStreamSynchronize(side);
        return trc != USTD_OK ? trc : src;
    }
    if (trc != USTD_OK) return trc;
    HIP_TRY(hipEventRecord(join.e, side));
    HIP_TRY(hipStreamWaitEvent(c.st, join.e, 0));
    {
        Timer tm(c.st);
        HIP_TRY(launch_combine(c.L.n, c.pivot, count_scale(c, tau), counts, x, d_diag, c.st));
        r->ms_combine += tm.stop_ms();
    }
    r->ms_total = total.stop_ms();
    return src;
}

int ustd_diag_lpinv_noalloc(const ustd_problem *prob, double *d_diag, int64_t *d_counts, ustd_report *rep,
                            void *stream) {
    g_err.clear();
    USTD_TRY(check_problem(prob));
    if (!d_diag) return fail(USTD_EINVAL, "d_diag is NULL");
    ustd_problem q;
    Plan L;
    USTD_TRY(fit_static(prob, &q, &L));
    void *ws = nullptr;
    USTD_TRY(static_scratch(&ws));
    NoEventsScope no_events;  // no HIP events or streams are created during this call
    Ctx c;
    USTD_TRY(begin_with(c, &q, L, ws, stream));
    ustd_report local{};
    ustd_report *r = rep ? rep : &local;
    memset(r, 0, sizeof(*r));
    USTD_TRY(setup(c, r));
    const long long tau = problem_tau(c);
    r->tau = tau;
    long long *counts = d_counts ? (long long *)d_counts : at<long long>(c.ws, c.L.off_counts);
    HIP_TRY(hipMemsetAsync(counts, 0, (size_t)c.L.n * 8, c.st));
    // everything on the caller's stream: the trees, then the pivot column, then the combination
    USTD_TRY(run_trees(c, 0, tau, counts, r));
    double *x = at<double>(c.ws, c.L.off_x64);
    const int src = solve_column(c, x, r);
    if (src != USTD_OK && src != USTD_ENOTCONV) return src;
    HIP_TRY(launch_combine(c.L.n, c.pivot, count_scale(c, tau), counts, x, d_diag, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    return src;
}

int ustd_batch_workspace_bytes(const ustd_problem *probs, int32_t count, size_t *bytes) {
    g_err.clear();
    if (!bytes) return fail(USTD_EINVAL, "bytes is NULL");
    long long b = 0;
    USTD_TRY(batch_workspace(probs, count, &b));
    *bytes = (size_t)b;
    return USTD_OK;
}

int ustd_batch_diag_lpinv(const ustd_problem *probs, int32_t count, void *d_ws, size_t ws_bytes,
                          double *const *d_diags, int64_t *const *d_counts, ustd_report *reps, void *stream) {
    g_err.clear();
    if (!d_diags) return fail(USTD_EINVAL, "d_diags is NULL");
    for (int i = 0; i < count; ++i)
        if (!d_diags[i]) return fail(USTD_EINVAL, "d_diags[%d] is NULL", i);
    hipStream_t st = (hipStream_t)stream;
    std::unique_ptr<ustd_batch_plan> P;
    Timer total(st);
    USTD_TRY(batch_plan_create(probs, count, d_ws, ws_bytes, nullptr, P, st));
    const int rc = batch_plan_execute(*P, d_diags, d_counts, st);
    if (rc != USTD_OK) {
        (void)hipStreamSynchronize(st);
        return rc;
    }
    std::vector<ustd_report> local(count);
    ustd_report *R = reps ? reps : local.data();
    const int status = batch_plan_reports(*P, R, st);
    const double ms = total.stop_ms();
    for (int i = 0; i < count; ++i) R[i].ms_total = ms;
    return status;
}

int ustd_batch_plan_create(const ustd_problem *probs, int32_t count, void *d_ws, size_t ws_bytes,
                           const ustd_batch_schedule *sched, ustd_batch_plan **plan, void *stream) {
    g_err.clear();
    if (!plan) return fail(USTD_EINVAL, "plan is NULL");
    *plan = nullptr;
    std::unique_ptr<ustd_batch_plan> P;
    const int rc = batch_plan_create(probs, count, d_ws, ws_bytes, sched, P, (hipStream_t)stream);
    if (rc != USTD_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        return rc;
    }
    *plan = P.release();
    return USTD_OK;
}

int ustd_batch_plan_execute(ustd_batch_plan *plan, double *const *d_diags, int64_t *const *d_counts, void *stream) {
    g_err.clear();
    if (!plan) return fail(USTD_EINVAL, "plan is NULL");
    return batch_plan_execute(*plan, d_diags, d_counts, (hipStream_t)stream);
}

int ustd_batch_plan_reports(ustd_batch_plan *plan, ustd_report *reps, void *stream) {
    g_err.clear();
    if (!plan || !reps) return fail(USTD_EINVAL, "plan or reps is NULL");
    return batch_plan_reports(*plan, reps, (hipStream_t)stream);
}

int ustd_batch_plan_schedule(const ustd_batch_plan *plan, ustd_batch_schedule *out) {
    g_err.clear();
    if (!plan || !out) return fail(USTD_EINVAL, "plan or out is NULL");
    *out = plan->sched;
    return USTD_OK;
}

int ustd_batch_plan_destroy(ustd_batch_plan *plan) {
    g_err.clear();
    if (plan && plan->live_graphs > 0)
        return fail(USTD_EINVAL, "%d captured graph(s) of this plan are still alive: destroy them first",
                    plan->live_graphs);
    if (plan) (void)hipDeviceSynchronize();  // no execution still reads the plan's memory
    delete plan;
    return USTD_OK;
}

int ustd_batch_graph_create(ustd_batch_plan *plan, double *const *d_diags, int64_t *const *d_counts, void **graph) {
    g_err.clear();
    if (!plan || !graph) return fail(USTD_EINVAL, "plan or graph is NULL");
    *graph = nullptr;
    if (!plan->big.empty())
        return fail(USTD_EINVAL, "problem %d uses the multi-kernel solve engine, which the host drives: it cannot be "
                                 "captured", plan->big[0]);
    hipStream_t s = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return fail(USTD_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    const int rc = batch_plan_execute(*plan, d_diags, d_counts, s);
    const std::string err = g_err;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    (void)hipStreamDestroy(s);
    if (rc != USTD_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        if (rc != USTD_OK) return fail(rc, "%s", err.c_str());
        return fail(USTD_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(USTD_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    *graph = new BatchGraph{ex, plan};
    ++plan->live_graphs;
    return USTD_OK;
}

int ustd_batch_graph_launch(void *graph, void *stream) {
    g_err.clear();
    if (!graph) return fail(USTD_EINVAL, "graph is NULL");
    HIP_TRY(hipGraphLaunch(static_cast<BatchGraph *>(graph)->ex, (hipStream_t)stream));
    return USTD_OK;
}

int ustd_batch_graph_destroy(void *graph) {
    g_err.clear();
    if (!graph) return USTD_OK;
    BatchGraph *bg = static_cast<BatchGraph *>(graph);
    (void)hipDeviceSynchronize();  // no launch of it still running
    const hipError_t e = hipGraphExecDestroy(bg->ex);
    --bg->plan->live_graphs;
    delete bg;
    if (e != hipSuccess) return fail(USTD_EHIP, "hipGraphExecDestroy: %s", hipGetErrorString(e));
    return USTD_OK;
}

int ustd_batch_autotune(const ustd_problem *probs, int32_t count, void *d_ws, size_t ws_bytes, const char *cache_path,
                        int32_t graph, ustd_batch_schedule *best, double *best_ms, int32_t *from_cache, void *stream) {
    g_err.clear();
    if (!best) return fail(USTD_EINVAL, "best is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (from_cache) *from_cache = 0;
    std::unique_ptr<ustd_batch_plan> P;
    USTD_TRY(batch_plan_create(probs, count, d_ws, ws_bytes, nullptr, P, st));
    if (graph && !P->big.empty())
        return fail(USTD_EINVAL, "problem %d uses the multi-kernel solve engine: its batches cannot be captured",
                    P->big[0]);
    std::string key;
    USTD_TRY(tune_key(*P, &key));
    key += graph ? "-graph" : "-eager";
    const char *env = std::getenv("USTD_TUNE_CACHE");
    const std::string path = cache_path ? cache_path : (env ? env : "");
    std::vector<std::pair<std::string, TuneEntry>> cache;
    if (!path.empty()) {
        cache = read_tune_cache(path);
        for (auto &kv : cache)
            if (kv.first == key && check_schedule(kv.second.s) == USTD_OK) {
                *best = schedule_of(&kv.second.s);
                if (best_ms) *best_ms = kv.second.ms;
                if (from_cache) *from_cache = 1;
                g_err.clear();
                return USTD_OK;
            }
        g_err.clear();
    }
    // outputs for the timed executions
    long long ntot = 0;
    for (int i = 0; i < count; ++i) ntot += probs[i].n;
    double *dd = nullptr;
    if (hipMalloc((void **)&dd, (size_t)ntot * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(USTD_ENOMEM, "tuning outputs of %lld doubles", ntot);
    }
    std::unique_ptr<double, void (*)(double *)> hold(dd, [](double *p) { (void)hipFree(p); });
    std::vector<double *> diags(count);
    for (int i = 0, o = 0; i < count; o += (int)probs[i].n, ++i) diags[i] = dd + o;
    std::vector<ustd_report> reps(count);
    // one execution of the plan (eager, or a replay of its captured graph), timed by events
    auto time_plan = [&](ustd_batch_plan &Q, double *ms) -> int {
        void *gx = nullptr;
        hipGraphExec_t ex = nullptr;
        if (graph) {
            USTD_TRY(ustd_batch_graph_create(&Q, diags.data(), nullptr, &gx));
            ex = static_cast<BatchGraph *>(gx)->ex;
        }
        hipEvent_t a = nullptr, b = nullptr;
        int rc = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess
                     ? USTD_OK
                     : fail(USTD_EHIP, "hipEventCreate failed");
        if (rc == USTD_OK && hipEventRecord(a, st) != hipSuccess) rc = fail(USTD_EHIP, "hipEventRecord failed");
        if (rc == USTD_OK)
            rc = ex ? (hipGraphLaunch(ex, st) == hipSuccess ? USTD_OK : fail(USTD_EHIP, "hipGraphLaunch failed"))
                    : batch_plan_execute(Q, diags.data(), nullptr, st);
        if (rc == USTD_OK && hipEventRecord(b, st) != hipSuccess) rc = fail(USTD_EHIP, "hipEventRecord failed");
        (void)hipStreamSynchronize(st);
        float m = 0.f;
        if (rc == USTD_OK && hipEventElapsedTime(&m, a, b) != hipSuccess) rc = fail(USTD_EHIP, "hipEventElapsedTime failed");
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        if (gx) (void)ustd_batch_graph_destroy(gx);
        if (rc != USTD_OK) return rc;
        rc = batch_plan_reports(Q, reps.data(), st);
        if (rc != USTD_OK && rc != USTD_ENOTCONV) return rc;
        *ms = (double)m;
        return USTD_OK;
    };
    double ms0 = 0.0;
    USTD_TRY(time_plan(*P, &ms0));  // warm-up: code objects and caches
    USTD_TRY(time_plan(*P, &ms0));
    P.reset();
    ustd_batch_schedule cur = schedule_of(nullptr);
    double cur_ms = ms0;
    auto try_one = [&](ustd_batch_schedule cand) -> int {
        std::unique_ptr<ustd_batch_plan> Q;
        USTD_TRY(batch_plan_create(probs, count, d_ws, ws_bytes, &cand, Q, st));
        double ms = 0.0;
        USTD_TRY(time_plan(*Q, &ms));
        if (ms < cur_ms) {
            cur_ms = ms;
            cur = Q->sched;
        }
        return USTD_OK;
    };
    // one dimension at a time, from the defaults, each value against the best so far
    for (int b : {2, 3, 4}) {
        ustd_batch_schedule c = cur;
        c.branches = b;
        USTD_TRY(try_one(c));
    }
    for (int g : {1, 4, -1}) {
        if (cur.branches >= 2) break;  // the chains of branch mode have no groups
        ustd_batch_schedule c = cur;
        c.group_fills = g;
        if (c.group_fills != cur.group_fills) USTD_TRY(try_one(c));
    }
    for (int ch : {kAggChunkLarge, kAggChunk}) {
        ustd_batch_schedule c = cur;
        c.agg_chunk = ch;
        USTD_TRY(try_one(c));
    }
    {
        ustd_batch_schedule c = cur;
        c.layout = USTD_LAYOUT_RECORDS;
        USTD_TRY(try_one(c));
    }
    {  // half the largest pool fill: more fills, less of the record pool
        std::unique_ptr<ustd_batch_plan> Q;
        USTD_TRY(batch_plan_create(probs, count, d_ws, ws_bytes, &cur, Q, st));
        const long long largest = Q->largest;
        Q.reset();
        if (largest > 1) {
            ustd_batch_schedule c = cur;
            c.fill_trees = (largest + 1) / 2;
            USTD_TRY(try_one(c));
        }
    }
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    if (!path.empty()) {
        TuneEntry e;
        e.s = cur;
        e.ms = cur_ms;
        bool found = false;
        for (auto &kv : cache)
            if (kv.first == key) {
                kv.second = e;
                found = true;
            }
        if (!found) cache.emplace_back(key, e);
        USTD_TRY(write_tune_cache(path, cache));
    }
    return USTD_OK;
}

int ustd_edge_counts(const ustd_problem *prob, int64_t tree_begin, int64_t tree_count, void *d_ws, size_t ws_bytes,
                     int64_t *d_counts, ustd_report *rep, void *stream) {
    g_err.clear();
    Ctx c;
    USTD_TRY(begin(c, prob, d_ws, ws_bytes, stream));
    if (tree_begin < 0 || tree_count < 0) return fail(USTD_EINVAL, "negative tree range");
    if (!d_counts) return fail(USTD_EINVAL, "d_counts is NULL");
    if (rep) memset(rep, 0, sizeof(*rep));
    Timer total(c.st);
    USTD_TRY(setup(c, rep));
    USTD_TRY(run_trees(c, tree_begin, tree_count, nullptr, rep, (long long *)d_counts));
    {
        Timer tm(c.st);
        HIP_TRY(launch_edge_fold(c.L.n, c.L.nnz, c.rp32, prob->d_col, (long long *)d_counts, c.st));
        if (rep) rep->ms_aggregate += tm.stop_ms();
    }
    if (rep) {
        rep->tau = tree_count;
        rep->ms_total = total.stop_ms();
    }
    return USTD_OK;
}

int ustd_edge_sample_size(int64_t n, int64_t m, double eps, double delta, int64_t *q) {
    g_err.clear();
    if (!q) return fail(USTD_EINVAL, "q is NULL");
    if (n < 2 || m < 1) return fail(USTD_EINVAL, "n = %lld, m = %lld out of range", (long long)n, (long long)m);
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(USTD_EINVAL, "eps must be > 0");
    if (delta > 0.0 && !(delta < 1.0)) return fail(USTD_EINVAL, "delta must lie in (0,1)");
    const double d = delta > 0.0 ? delta : 1.0 / (double)n;
    *q = (int64_t)std::ceil(2.0 * std::log(2.0 * (double)m / d) / (eps * eps));
    return USTD_OK;
}

int ustd_edge_resistances(int64_t n, int64_t nnz, const int64_t *d_row_ptr, const int32_t *d_col,
                          const double *d_weight, const int64_t *d_counts, int64_t q, double theta, double *d_r,
                          double *d_denom, void *stream) {
    g_err.clear();
    if (n < 2 || n >= (1ll << 30) - 1 || nnz < 2 || nnz >= (1ll << 31))
        return fail(USTD_EINVAL, "n = %lld, nnz = %lld out of range", (long long)n, (long long)nnz);
    if (!d_row_ptr || !d_col || !d_counts) return fail(USTD_EINVAL, "row_ptr / col / counts is NULL");
    if (q < 1) return fail(USTD_EINVAL, "q must be >= 1");
    if (!(theta > 0.0 && theta < 1.0)) return fail(USTD_EINVAL, "theta must lie in (0,1)");
    HIP_TRY(launch_edge_resistance((int)n, nnz, (const long long *)d_row_ptr, d_col, d_weight,
                                   (const long long *)d_counts, (double)q, theta, d_r, d_denom,
                                   (hipStream_t)stream));
    return USTD_OK;
}

int ustd_centralities(int64_t n, const double *d_diag, double *d_farness, double *d_closeness, double *d_nrwb,
                      double *d_scalars, void *stream) {
    g_err.clear();
    if (n < 2) return fail(USTD_EINVAL, "n = %lld out of range", (long long)n);
    if (!d_diag || !d_scalars) return fail(USTD_EINVAL, "d_diag / d_scalars is NULL");
    HIP_TRY(launch_centralities(n, d_diag, d_farness, d_closeness, d_nrwb, d_scalars, (hipStream_t)stream));
    return USTD_OK;
}

int ustd_philox_words(uint64_t seed, int64_t t, int32_t s, int64_t k0, int64_t count, uint32_t *d_out, void *stream) {
    g_err.clear();
    if (count < 0 || k0 < 0 || !d_out) return fail(USTD_EINVAL, "bad arguments");
    if (count == 0) return USTD_OK;
    HIP_TRY(launch_philox_words((uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32), t, s, k0, count, d_out,
                                (hipStream_t)stream));
    return USTD_OK;
}

const char *ustd_status_string(int status) {
    switch (status) {
        case USTD_OK: return "USTD_OK";
        case USTD_EINVAL: return "USTD_EINVAL";
        case USTD_EGRAPH: return "USTD_EGRAPH";
        case USTD_ENOMEM: return "USTD_ENOMEM";
        case USTD_EHIP: return "USTD_EHIP";
        case USTD_ENOTCONV: return "USTD_ENOTCONV";
        default: return "USTD_UNKNOWN";
    }
}

const char *ustd_last_error(void) { return g_err.c_str(); }

}  // extern "C"
