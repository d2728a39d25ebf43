// ustd_kernels.hip -- gfx950 kernels of the UST estimator of diag(L^+)
// (Angriman, Predari, van der Grinten, Meyerhenke, ESA 2020).
//
//   graph set-up   : int32 row pointers, device CSR validation, max-degree pivot,
//                    level-synchronous BFS with the minimum-ID parent rule (tree B_u)
//   sampling       : Wilson's algorithm, one wavefront per tree, speculative walks with
//                    an in-order commit that reproduces the sequential algorithm exactly
//   tree intervals : subtree intervals of each sampled tree (replacing the DFS
//                    timestamps of Algorithm 2) from a child CSR and a BFS order
//   aggregation    : Algorithm 2, thread per vertex over a chunk of resident trees
//   solve          : Jacobi-PCG on the pivot column (FP64, or FP32 inner + FP64 outer)
//   combine        : Eq. diag-comp in FP64
#include "ustd_kernels.hpp"

#include <algorithm>
#include <climits>
#include <type_traits>

namespace ustd {

// ======================================================================================
// graph set-up
// ======================================================================================
__global__ void col_to_u16_kernel(long long nnz, const int *__restrict__ col, unsigned short *__restrict__ col16) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) col16[e] = (unsigned short)col[e];
}

__global__ void rp_to_i32_kernel(int n, const long long *__restrict__ rp64, int *__restrict__ rp32) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v <= n) rp32[v] = (int)rp64[v];
}

// Structural checks of the input CSR (Section "Problem Description and Notation": simple,
// undirected): row bounds, ascending rows (no duplicates), no self-loops, symmetry.
// Connectivity is checked after the BFS.  err receives a bit per failure class.
__global__ void validate_kernel(int n, long long nnz, const long long *__restrict__ rp64,
                                const int *__restrict__ col, int *__restrict__ err) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0 && (rp64[0] != 0 || rp64[n] != nnz)) atomicOr(err, 1);
    if (v >= n) return;
    const long long lo = rp64[v], hi = rp64[v + 1];
    if (hi < lo || lo < 0 || hi > nnz) { atomicOr(err, 1); return; }
    if (hi == lo) { atomicOr(err, 16); return; }  // isolated vertex
    for (long long e = lo; e < hi; ++e) {
        const int w = col[e];
        if (w < 0 || w >= n) { atomicOr(err, 2); return; }
        if (w == v) { atomicOr(err, 4); return; }
        if (e > lo && col[e - 1] >= w) { atomicOr(err, 2); return; }
        long long a = rp64[w], b = rp64[w + 1];
        bool found = false;
        while (a < b) {
            const long long mid = a + (b - a) / 2;
            const int c = col[mid];
            if (c == v) { found = true; break; }
            if (c < v) a = mid + 1; else b = mid;
        }
        if (!found) { atomicOr(err, 8); return; }
    }
}

// Maximum-degree vertex, smallest ID on ties: max of (deg << 32 | ~id).
__global__ void argmax_degree_kernel(int n, const int *__restrict__ rp, unsigned long long *__restrict__ best) {
    unsigned long long key = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const unsigned long long deg = (unsigned long long)(rp[v + 1] - rp[v]);
        const unsigned long long k = (deg << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)v);
        key = k > key ? k : key;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const unsigned long long o = __shfl_xor(key, d, 64);
        key = o > key ? o : key;
    }
    if (lane_id() == 0) atomicMax(best, key);
}

// Pivot by repeated BFS sweeps (engineering appendix): after each BFS, bound[v] = max(bound[v],
// dist[v]) (bound = dist after the first) and the farthest vertex, largest distance then
// smallest ID, as a packed key; at the end the vertex of smallest bound, then smallest ID.
__global__ void sweep_update_kernel(int n, const int *__restrict__ dist, int *__restrict__ bound, int first,
                                    unsigned long long *__restrict__ far) {
    unsigned long long key = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int d = dist[v];
        bound[v] = first ? d : max(bound[v], d);
        const unsigned long long k = ((unsigned long long)(unsigned)d << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)v);
        key = k > key ? k : key;
    }
#pragma unroll
    for (int dd = 32; dd > 0; dd >>= 1) {
        const unsigned long long o = __shfl_xor(key, dd, 64);
        key = o > key ? o : key;
    }
    if (lane_id() == 0) atomicMax(far, key);
}
__global__ void argmin_bound_kernel(int n, const int *__restrict__ bound, unsigned long long *__restrict__ best) {
    unsigned long long key = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const unsigned long long k = ((unsigned long long)(0x7FFFFFFFu - (unsigned)bound[v]) << 32) |
                                     (unsigned long long)(0xFFFFFFFFu - (unsigned)v);
        key = k > key ? k : key;
    }
#pragma unroll
    for (int dd = 32; dd > 0; dd >>= 1) {
        const unsigned long long o = __shfl_xor(key, dd, 64);
        key = o > key ? o : key;
    }
    if (lane_id() == 0) atomicMax(best, key);
}

__global__ void bfs_init_kernel(int n, int u, int *__restrict__ dist, int *__restrict__ parB) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) {
        dist[v] = (v == u) ? 0 : INT_MAX;
        parB[v] = (v == u) ? -1 : INT_MAX;
    }
}

// Rows are processed in a degree-balanced way: rows of degree <= heavy_thresh by groups of
// G lanes (one row per group), heavier rows (listed once per graph in ascending order) by a
// whole 256-thread block each.  Grid-stride over a fixed grid, so every reduction order
// depends only on the graph.

// One BFS level: every vertex at distance d offers itself as parent to its unvisited
// neighbours; atomicMin keeps the smallest-ID one among all of them, which is the
// minimum-ID neighbour one level closer to u.  `found` is set if any vertex is reached.
// Levels are queued several at a time: a level whose predecessor reached nothing (*prev == 0)
// has no vertex at distance d and returns at once.
template <int G>
__global__ __launch_bounds__(256) void bfs_level_kernel(RowMap m, int d, int *__restrict__ dist,
                                                        int *__restrict__ parB, int *__restrict__ found,
                                                        const int *__restrict__ prev) {
    if (prev && *prev == 0) return;  // uniform over the grid
    int any = 0;
    const int nh = *m.nheavy;
    for (int h = blockIdx.x; h < nh; h += gridDim.x) {
        const int v = m.heavy[h];
        if (dist[v] != d) continue;  // uniform in the block
        for (int e = m.rp[v] + threadIdx.x; e < m.rp[v + 1]; e += blockDim.x) {
            const int y = m.col[e];
            const int dy = dist[y];
            if (dy > d) {
                atomicMin(&parB[y], v);
                if (dy != d + 1) dist[y] = d + 1;
                any = 1;
            }
        }
    }
    const int rows_per_tile = 256 / G;
    const int g = threadIdx.x / G, l = threadIdx.x % G;
    for (int tile = blockIdx.x; tile * rows_per_tile < m.n; tile += gridDim.x) {
        const int v = tile * rows_per_tile + g;
        if (v >= m.n || dist[v] != d) continue;
        const int lo = m.rp[v], hi = m.rp[v + 1];
        if (hi - lo > m.heavy_thresh) continue;
        for (int e = lo + l; e < hi; e += G) {
            const int y = m.col[e];
            const int dy = dist[y];
            if (dy > d) {
                atomicMin(&parB[y], v);
                if (dy != d + 1) dist[y] = d + 1;
                any = 1;
            }
        }
    }
    if (__any(any) && lane_id() == 0) atomicOr(found, 1);
}

// heavy-row list, deterministic: per-block counts, one-block scan, ordered writes
__global__ __launch_bounds__(256) void heavy_count_kernel(int n, const int *__restrict__ rp, int thresh,
                                                          int *__restrict__ bcount) {
    __shared__ int sh[5];
    const int v = blockIdx.x * 256 + threadIdx.x;
    const int hv = (v < n && rp[v + 1] - rp[v] > thresh) ? 1 : 0;
    int tot;
    block_incl_scan(hv, &tot, sh);
    if (threadIdx.x == 0) bcount[blockIdx.x] = tot;
}
__global__ __launch_bounds__(256) void heavy_scan_kernel(int nb, int *__restrict__ bcount, int *__restrict__ nheavy) {
    __shared__ int sh[5];
    int carry = 0;
    for (int base = 0; base < nb; base += 256) {
        const int i = base + threadIdx.x;
        const int c = i < nb ? bcount[i] : 0;
        int tot;
        const int incl = block_incl_scan(c, &tot, sh);
        if (i < nb) bcount[i] = carry + incl - c;
        carry += tot;
    }
    if (threadIdx.x == 0) *nheavy = carry;
}
__global__ __launch_bounds__(256) void heavy_write_kernel(int n, const int *__restrict__ rp, int thresh,
                                                          const int *__restrict__ boff, int *__restrict__ heavy) {
    __shared__ int sh[5];
    const int v = blockIdx.x * 256 + threadIdx.x;
    const int hv = (v < n && rp[v + 1] - rp[v] > thresh) ? 1 : 0;
    int tot;
    const int incl = block_incl_scan(hv, &tot, sh);
    if (hv) heavy[boff[blockIdx.x] + incl - 1] = v;
}

__global__ void count_unreached_kernel(int n, const int *__restrict__ dist, int *__restrict__ err) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && dist[v] == INT_MAX) atomicOr(err, 32);
}

// ======================================================================================
// Wilson sampler (Appendix "Wilson's UST Algorithm"), one 64-lane wavefront per tree.
//
// The sequential definition takes start vertices s = 0..n-1 in ascending order; from each
// s not yet in T it walks until it reaches T and adds the loop erasure of the walk.  Step
// k of the walk from s uses its own Philox word (counter (k/4, s, t)), so the whole walk
// from s is a fixed sequence x_0 = s, x_1, x_2, ... that does not depend on T; T only
// decides where it stops (the first x_i in T) and whether s walks at all.
//
// Lanes therefore run the walks of the next not-in-tree starts speculatively, against the
// tree committed so far, and record their vertices.  Walks are committed strictly in
// start order from a reorder buffer (ROB).  Every commit sees exactly the tree the
// sequential algorithm would see at that start (all earlier starts committed, no later
// one), so it truncates the recorded walk at its first vertex now in T, skips s if s has
// been absorbed meanwhile, and adds the loop erasure (each vertex's successor after its
// last visit).  A recorded walk is always long enough: it stopped at a vertex of an older
// tree, which is still in T.  Three commit paths:
//   - runs of short walks (at most kPathLds steps, kept in LDS) commit as one batch, one
//     lane each, up to the first entry that reads a vertex an earlier entry of the batch
//     writes (detected through two minimum-writer tables under independent hashes);
//   - longer recorded walks (up to 255 steps) commit cooperatively with ballots (one ballot per
//     64-step chunk finds the truncation point, one per chunk and branch vertex finds the
//     vertex's last visit).  A walk that filled its 255-step record without reaching the
//     tree it saw takes this path too: the tree has usually grown since, so the record
//     mostly does reach it;
//   - if no recorded vertex is in the tree, one lane turns the record into Next pointers (in
//     the parent field of the record array) and continues the walk from its last vertex in
//     a tight loop (the sequential algorithm for that start).
// Everything a commit needs is prefetched into LDS while walking (the B_u flag word of
// every recorded vertex, the chain value of the vertex a walk ends on), so the in-order
// commit path does no dependent global loads in the common cases.
//
// Output per vertex x: rec[x] = {parent_T(x), nba(x) | marked(x) << 31} (see "Marked
// vertices").  Launches are persistent: each block takes tree after tree from a queue.
// ======================================================================================
namespace {

// reorder-buffer entries (LDS): with the tree bitmap in LDS the sampler's occupancy is bound by
// LDS (64 entries); with the tree state in the records it is bound by registers, and 128 entries
// let the lanes run further ahead of a long walk at the head
template <bool LDS>
constexpr int rob_cap() { return LDS ? kSamplerRobLds : kSamplerRobMax; }
constexpr int kPathLds = 5;              // recorded steps kept in LDS per entry (x_1..x_5)
constexpr int kPath = 255;               // recorded steps per speculative walk (x_1..x_255)
static_assert(kPath - kPathLds == kSamplerPathGlobal, "path split");
// reorder-buffer entry states besides a finished walk's step count (>= 0):
//   kWalking  - still walking
//   kOverflow - recorded kPath steps without reaching the tree it saw
//   kContinue - an overflowed walk none of whose recorded vertices is in the tree at commit
//   kRewalk   - re-walk from the start (never expected; keeps the commit exact regardless)
constexpr int kWalking = -1, kOverflow = -2, kContinue = -3, kRewalk = -4;

// Membership of the tree being built.  Graphs of up to 131072 vertices keep an n-bit
// bitmap in LDS (allocation words of 32 vertices).  Larger graphs use the vertex's own
// record: its nba field holds kFree until the vertex joins the tree (the records are
// cleared when the tree starts), so a membership test reads the line a walk that ends
// there needs anyway, and joining is the record write itself (set() does nothing).
// Records are read for membership with agent-scope loads (past the per-CU L1).
constexpr int kFree = 0x3FFFFFFF;  // nba of a vertex not in the tree; vertex IDs are below it

// the {nba | flags} word of a record another lane of the wave may have written
__device__ __forceinline__ int load_nbx(const int *recw, int v) {
    return __hip_atomic_load(recw + 2 * v + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool LDS>
struct TreeState;

template <>
struct TreeState<true> {
    uint32_t *w;
    static constexpr int kShift = 5;  // allocation word: 32 vertices
    __device__ __forceinline__ uint32_t word(int i, int /*n*/) const { return w[i]; }
    __device__ __forceinline__ bool test(int v) const { return (w[v >> 5] >> (v & 31)) & 1u; }
    __device__ __forceinline__ void set(int v) const { atomicOr(w + (v >> 5), 1u << (v & 31)); }
};

template <>
struct TreeState<false> {
    int *recw;                        // int pairs {parent, nba | flags}
    static constexpr int kShift = 3;  // allocation word: 8 vertices
    __device__ __forceinline__ int nbx(int v) const { return load_nbx(recw, v); }
    __device__ __forceinline__ uint32_t word(int i, int n) const {
        uint32_t m = 0u;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int v = (i << 3) + b;
            if (v < n && nbx(v) != kFree) m |= 1u << b;
        }
        return m;
    }
    __device__ __forceinline__ bool test(int v) const { return nbx(v) != kFree; }
    __device__ __forceinline__ void set(int) const {}
};

// Marked vertices.  Algorithm 2 adds, for v and each edge (a, b) of P(v), +1 when T
// contains a -> b above v and -1 when it contains b -> a above v.  Written per T-ancestor x
// of v (x != u), x contributes only if x lies on P(v) and its tree edge x -> parent_T(x) is
// a B_u edge: +1 when parent_T(x) = parB(x) (that edge of P(v) is traversed forward), -1
// when parB(parent_T(x)) = x and parent_T(x) is on P(v) too (traversed backward).  A
// strict T-ancestor of v on P(v) has a child in B_u, so only vertices that are internal in
// B_u and whose tree edge is a B_u edge ("marked") can contribute.  Each vertex x stores
// nba(x) = nearest marked strict T-ancestor (u if none) and its flags (marked; forward or
// backward edge); cv(x) = x if x is marked, else nba(x), is the nba value of x's children.
// Algorithm 2 then follows the nba chain and decides "on P(v)" with the fixed subtree
// intervals of B_u: a forward x counts if x is on P(v), a backward x if parent_T(x) is.
//
// bflag[x] = (parB(x) + 1) | (1 << 31 if x is internal in B_u), so parB(u) = -1.
__device__ __forceinline__ int bf_parent(int f) { return (int)((unsigned)f & 0x7FFFFFFFu) - 1; }
__device__ __forceinline__ bool bf_internal(int f) { return (unsigned)f >> 31; }
// A record is {parent_T(x), nba(x) | flags}: bit 31 = x is marked, bit 30 = its tree edge
// is a forward B_u edge (parent_T(x) = parB(x)), else it is a backward one
// (parB(parent_T(x)) = x).  Vertex IDs are < 2^30 (a connected graph with nnz < 2^31).
// cv(x) follows from the record.
constexpr int kMarkBit = (int)0x80000000u;
constexpr int kFwdBit = 0x40000000;
__device__ __forceinline__ int cv_of(int x, int nbx) { return (nbx & kMarkBit) ? x : nbx; }
__device__ __forceinline__ int nba_of(int nbx) { return nbx & 0x3FFFFFFF; }
// the flag bits of vertex x (B_u flag word fx) whose tree parent is px (flag word fpx)
__device__ __forceinline__ int mark_bits(int x, int fx, int px, int fpx) {
    const unsigned fwd = px == bf_parent(fx), bwd = bf_parent(fpx) == x;
    const unsigned m = (unsigned)bf_internal(fx) & (fwd | bwd);
    return (int)((m << 31) | ((m & fwd) << 30));
}
// The same two bits in the low bits, for a walk step x -> y: the walk records them with y,
// since a vertex kept by the loop erasure has as its tree edge the step after its last visit.
__device__ __forceinline__ int edge_bits(int x, int fx, int y, int fy) {
    return (int)((unsigned)mark_bits(x, fx, y, fy) >> 30);
}
constexpr int kVertexMask = 0x3FFFFFFF;  // a recorded global step is y | edge bits << 30

// The sampler's block is one wavefront.  Its LDS operations execute in issue order, so
// lanes exchange data through LDS with compiler ordering only; a workgroup barrier would
// also wait for every outstanding global load and store.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
// Force loaded values into registers here.  A load still in flight when its register is
// reused later makes the compiler wait for the whole in-order memory counter, i.e. for
// every store issued since (the commit phase's record stores).
__device__ __forceinline__ void consume(int a, int b, int c, int d) {
    asm volatile("" ::"v"(a), "v"(b), "v"(c), "v"(d));
}
// wait until all of this wavefront's global loads and stores have completed
__device__ __forceinline__ void wait_global() {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt/lgkmcnt unconstrained
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Batch-commit conflict tables: two tables of minimum-writer lanes under independent
// hashes; a read conflicts only if both of its slots hold a smaller lane, so collisions
// rarely cut a batch short and a real conflict is never missed.  240 slots each rather than
// 256 keep the sampler's LDS at R-MAT scale 16 within 8960 bytes, the size at which a CU
// holds 18 blocks (16 above it).
constexpr int kHashSlots = 240;

// inclusive prefix sum over the 64 lanes with DPP row shifts and row broadcasts
__device__ __forceinline__ int wave_scan_dpp(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}
// Multiplicative hashes scaled to [0, kHashSlots).  Any hash keeps the commit exact: a
// collision only ends a batch early.  With the tree bitmap in LDS (vertex IDs below 2^17) they
// take bits 16..23 of a 24 x 24-bit product (odd multipliers near 2^24 times the golden ratio
// and another irrational, so consecutive IDs spread over the table), then x 240 / 256: two
// full-rate v_mul_u32_u24 instead of a quarter-rate 32-bit multiply and high multiply, as that
// sampler is bound by instruction issue.  The large-graph sampler keeps the 32-bit hashes (the
// other form costs it a register and one wave per SIMD).
template <bool LDS>
__device__ __forceinline__ int hash_slot(int v) {
    if constexpr (LDS)
        return (int)(__umul24((__umul24((unsigned)v, 0x9E3779u) >> 16) & 0xFFu, (unsigned)kHashSlots) >> 8);
    else
        return (int)__umulhi((unsigned)v * 2654435761u, kHashSlots);
}
template <bool LDS>
__device__ __forceinline__ int hash_slot2(int v) {
    if constexpr (LDS)
        return (int)(__umul24(((__umul24((unsigned)v, 0xC2B2AFu) + 0x5BD1E9u) >> 16) & 0xFFu, (unsigned)kHashSlots) >>
                     8);
    else
        return (int)__umulhi((unsigned)v * 2246822519u + 3266489917u, kHashSlots);
}

// position of the k-th set bit of x (k < popc(x)), by halving
__device__ __forceinline__ int select_bit(uint32_t x, int k) {
    int pos = 0, c = __popc(x & 0xFFFFu);
    if (k >= c) { k -= c; pos += 16; x >>= 16; }
    c = __popc(x & 0xFFu);
    if (k >= c) { k -= c; pos += 8; x >>= 8; }
    c = __popc(x & 0xFu);
    if (k >= c) { k -= c; pos += 4; x >>= 4; }
    c = __popc(x & 0x3u);
    if (k >= c) { k -= c; pos += 2; x >>= 2; }
    return pos + (k >= (int)(x & 1u) ? 1 : 0);
}
__device__ __forceinline__ int select_bit64(uint64_t x, int k) {
    const int c = __popc((uint32_t)x);
    return k >= c ? 32 + select_bit((uint32_t)(x >> 32), k - c) : select_bit((uint32_t)x, k);
}

// Neighbour index (0 .. deg-1) of a walk step with word w from the row [r0, r1).  Unit
// weights: floor(w deg / 2^32).  Weighted (Section "Generalizations"): the first j with
// t < C[j], C the row's running conductance sums (cw, taken left to right in FP64) and
// t = (w 2^-32) C[deg-1]; both products are exact or rounded once, so the choice is the
// same on every device, and all-ones weights give floor(w deg / 2^32).
//
// The weighted search starts from a guide entry: bucket i = floor(w deg / 2^32) holds the
// first j with C[j] > t(w_i), w_i the bucket's smallest word.  t is non-decreasing in w, so
// that j never passes the answer, and a forward scan ends on it; buckets are equally wide
// in t, so the scan takes one probe on average for any weights (deg boundaries, deg buckets).
template <bool WT>
__device__ __forceinline__ int step_index(uint32_t w, int r0, int r1, const double *__restrict__ cw,
                                          const int *__restrict__ guide) {
    const int bucket = (int)__umulhi(w, (uint32_t)(r1 - r0));
    if constexpr (!WT) {
        return bucket;
    } else {
        const double t = ((double)w * 0x1p-32) * cw[r1 - 1];
        const int last = r1 - r0 - 1;
        int j = guide[r0 + bucket];
        while (j < last && !(t < cw[r0 + j])) ++j;  // t < C[deg-1] for any normal row total
        return j;
    }
}

// The sequential algorithm for one start s0 against the current tree, in two parts: a walk
// that writes Next pointers (in the parent field) until it reaches the tree, then the retrace
// of the loop erasure that writes the branch's records {parent, nba | marked << 31}.  The walk
// resumes at step k0 from vertex x0 (k0 = 0, x0 = s0 for a whole walk; otherwise the Next
// pointers of steps 0..k0-1 are already written).

// Retrace from s0 to the tree vertex the walk reached.  One lane.
template <bool LDS>
__device__ void retrace_commit(const TreeState<LDS> &bits, int *recw, const int *__restrict__ bflag, int s0) {
    int z = s0;
    while (!bits.test(z)) {
        bits.set(z);
        z = recw[2 * z];
    }
    const int ya = z;
    const int cva = cv_of(ya, load_nbx(recw, ya));
    // nba: the nearest marked vertex strictly closer to ya on the branch, else cv(ya)
    int run = s0;
    z = s0;
    while (z != ya) {
        const int nz = recw[2 * z];
        if (mark_bits(z, bflag[z], nz, bflag[nz])) {
            for (int w2 = run; w2 != z; w2 = recw[2 * w2]) recw[2 * w2 + 1] = z;
            run = z;
        }
        z = nz;
    }
    for (int w2 = run; w2 != ya; w2 = recw[2 * w2]) recw[2 * w2 + 1] = cva;
    for (z = s0; z != ya; z = recw[2 * z]) {
        const int nz = recw[2 * z];
        recw[2 * z + 1] |= mark_bits(z, bflag[z], nz, bflag[nz]);
    }
}

// The walk on graphs held in LDS (the graph-in-LDS sampler).  Every lane calls it; lane 0 walks.  The
// wave computes the walk's Philox words 256 at a time (lane i the block of steps 4(b0+i) ..
// 4(b0+i)+3) into wbuf (LDS), so the walking lane reads a word per step instead of running a
// ten-round Philox block on one lane every fourth step.  Returns the walk's total step count
// on every lane.
template <typename CT, bool WT>
__device__ long long walk_next_wave(const TreeState<true> &bits, int *recw, const int *__restrict__ rp,
                                    const CT *__restrict__ col, const double *__restrict__ cw,
                                    const int *__restrict__ guide, uint32_t wkey, int x0, long long k0, uint32_t tlo,
                                    uint32_t thi, uint32_t key0, uint32_t key1, uint32_t *wbuf) {
    const int lane = threadIdx.x;
    long long k = k0;  // wave-uniform between word blocks
    int xw = x0, r0 = 0, r1 = 0;
    if (lane == 0) {
        r0 = rp[x0];
        r1 = rp[x0 + 1];
    }
    for (;;) {
        const long long b0 = k >> 2;
        const uint4 ph = philox4x32_10(make_uint4((uint32_t)(b0 + lane), wkey, tlo, thi), key0, key1);
        wbuf[4 * lane] = ph.x;
        wbuf[4 * lane + 1] = ph.y;
        wbuf[4 * lane + 2] = ph.z;
        wbuf[4 * lane + 3] = ph.w;
        wave_sync();
        int fin = 0;
        if (lane == 0) {
            const long long kend = (b0 + kWave) * 4;
            while (k < kend) {
                const uint32_t w = wbuf[(int)(k - b0 * 4)];
                const int y = (int)col[r0 + step_index<WT>(w, r0, r1, cw, guide)];
                const int ny0 = rp[y], ny1 = rp[y + 1];
                ++k;
                recw[2 * xw] = y;  // Next pointer; becomes the parent when xw joins T
                if (bits.test(y)) {
                    fin = 1;
                    break;
                }
                xw = y;
                r0 = ny0;
                r1 = ny1;
            }
        }
        wave_sync();  // the words are read before they are overwritten
        fin = __shfl(fin, 0, kWave);
        const int klo = __shfl((int)(unsigned long long)k, 0, kWave);
        const int khi = __shfl((int)((unsigned long long)k >> 32), 0, kWave);
        k = (long long)(((unsigned long long)(unsigned)khi << 32) | (unsigned)klo);
        if (fin) return k;
    }
}

// The walk and retrace by one lane.  Graphs past the LDS bitmap read the edge entries {y,
// row of y, B_u flag of y}: the entry of step k gives everything step k + 1 needs, so step
// k + 1's entry is loaded together with the tree test of y (before its answer is known) and
// each step waits for one load, not two in a row.  Graphs within it read the compact column
// and row arrays, which stay in the L1.  Returns the walk's total step count.
template <bool LDS, typename CT, bool WT>
__device__ long long rewalk_commit(const TreeState<LDS> &bits, int *recw, const int *__restrict__ rp,
                                   const CT *__restrict__ col, const int4 *__restrict__ edge,
                                   const int4 *__restrict__ vrow, const double *__restrict__ cw,
                                   const int *__restrict__ guide, const int *__restrict__ bflag, int s0, uint32_t wkey,
                                   int x0, long long k0, uint32_t tlo, uint32_t thi, uint32_t key0, uint32_t key1) {
    int xw = x0;
    long long k = k0;
    uint4 ph = philox4x32_10(make_uint4((uint32_t)(k >> 2), wkey, tlo, thi), key0, key1);
    if constexpr (LDS) {
        int r0 = rp[x0], r1 = rp[x0 + 1];
        for (;;) {
            if ((k & 3) == 0) ph = philox4x32_10(make_uint4((uint32_t)(k >> 2), wkey, tlo, thi), key0, key1);
            const int q = (int)(k & 3);
            const uint32_t w = q == 0 ? ph.x : (q == 1 ? ph.y : (q == 2 ? ph.z : ph.w));
            const int y = (int)col[r0 + step_index<WT>(w, r0, r1, cw, guide)];
            const int ny0 = rp[y], ny1 = rp[y + 1];
            ++k;
            recw[2 * xw] = y;  // Next pointer; becomes the parent when xw joins T
            if (bits.test(y)) break;
            xw = y;
            r0 = ny0;
            r1 = ny1;
        }
        retrace_commit<true>(bits, recw, bflag, s0);
        return k;
    } else {
    int4 e;  // entry of step k: the step from xw
    {
        const int4 v0 = vrow[x0];
        const int q = (int)(k & 3);
        const uint32_t w = q == 0 ? ph.x : (q == 1 ? ph.y : (q == 2 ? ph.z : ph.w));
        e = edge[v0.x + step_index<WT>(w, v0.x, v0.y, cw, guide)];
    }
    for (;;) {
        const int y = e.x;
        ++k;
        if ((k & 3) == 0) ph = philox4x32_10(make_uint4((uint32_t)(k >> 2), wkey, tlo, thi), key0, key1);
        const int q = (int)(k & 3);
        const uint32_t w = q == 0 ? ph.x : (q == 1 ? ph.y : (q == 2 ? ph.z : ph.w));
        const int4 en = edge[e.y + step_index<WT>(w, e.y, e.z, cw, guide)];  // step k from y
        recw[2 * xw] = y;  // Next pointer; becomes the parent when xw joins T
        if (bits.test(y)) break;
        xw = y;
        e = en;
    }
    retrace_commit<false>(bits, recw, bflag, s0);
    return k;
    }
}

template <typename T>
__device__ __forceinline__ T sel4(int c, T a0, T a1, T a2, T a3) {
    return c == 0 ? a0 : (c == 1 ? a1 : (c == 2 ? a2 : a3));
}

}  // namespace

template <bool LDS, typename CT, bool WT, bool GL = false, bool BV = false>
__global__ __launch_bounds__(64) void wilson_kernel(WilsonArgs a) {
    // Reorder buffer.  Vertex IDs take the column type (16 bits when n <= 65536), so that
    // with the tree bitmap a block of R-MAT scale 16 fits 18 to a CU.  A recorded step
    // keeps the vertex and the step's edge bits (below), not the vertex's B_u flag word.
    constexpr int kRobMax = rob_cap<LDS>();
    extern __shared__ uint32_t lds_bits[];
    __shared__ CT rob_s[kRobMax], rob_cv[kRobMax];
    __shared__ short rob_k[kRobMax];
    __shared__ unsigned short rob_pb[kRobMax];  // edge bits of steps 1..kPathLds, 2 bits each
    __shared__ CT rob_p[kRobMax][kPathLds];
    __shared__ int htab[2 * kHashSlots];
    // tree state in the records: the free-vertex words of the last scanned window (a window of
    // 64 allocation words is read once, not once per allocation round)
    __shared__ uint32_t win_fb[LDS ? 1 : kWave];
    __shared__ int win_base;  // first word of that window, -1 before the first read
    int *const hslot = htab;                     // first conflict table
    int *const hslot2 = htab + kHashSlots;       // second conflict table
    int *const br = htab;  // a long walk's branch (vertex | edge bits << 30) shares the tables'
                           // storage; the slots are cleared again afterwards
    static_assert(kPath + 1 <= 2 * kHashSlots, "the branch buffer fits the conflict tables");
    static_assert(4 * kWave <= 2 * kHashSlots, "a re-walk's Philox words fit the conflict tables");
    static_assert(kPathLds * 2 <= 16, "edge bits fit rob_pb");

    const int lane = threadIdx.x;
    int *__restrict__ gpath = a.path + (long long)blockIdx.x * kSamplerPathSlot;

    // GL (small graphs, single-graph launches): the row pointers, B_u flags and 16-bit columns
    // are copied into LDS after the tree bitmap, once per block, so that walk steps (above all
    // the one-lane re-walk of long walks) read LDS instead of the L1/L2.
    const int *lrp = nullptr, *lbf = nullptr;
    const CT *lcol = nullptr;
    if constexpr (GL) {
        static_assert(LDS && !WT && sizeof(CT) == 2, "graph in LDS: small unweighted graphs");
        const int n0 = a.g.n;
        int *srp = reinterpret_cast<int *>(lds_bits + a.g.nwords);
        int *sbf = srp + n0 + 1;
        CT *scol = reinterpret_cast<CT *>(sbf + n0);
        const int nnz0 = a.g.rp[n0];
        const CT *gcol = reinterpret_cast<const CT *>(a.g.colv);
        for (int i = lane; i <= n0; i += kWave) srp[i] = a.g.rp[i];
        for (int i = lane; i < n0; i += kWave) sbf[i] = a.g.bflag[i];
        for (int i = lane; i < nnz0; i += kWave) scol[i] = gcol[i];
        wave_sync();
        lrp = srp;
        lbf = sbf;
        lcol = scol;
    }

    for (;;) {
    // ---------------------------------------------------------------- next tile
    int tile = 0;
    if (lane == 0) tile = atomicAdd(a.queue, 1);
    tile = __builtin_amdgcn_readfirstlane(tile);
    if (tile >= a.ntiles) break;
    WilsonGraph g;
    long long t;
    int2 *rec;
    if (a.tiles) {
        const WilsonTile tl = a.tiles[tile];
        g = a.graphs[tl.graph];
        t = tl.tree;
        rec = a.rec + tl.rec_off;
    } else {
        g = a.g;
        t = a.tree_begin + tile;
        rec = a.rec + (long long)tile * a.rec_stride;
    }
    const int n = g.n;
    const int nwords = g.nwords;
    const int rob = min(g.rob, kRobMax);  // power of two
    const int robm = rob - 1;
    const uint32_t tlo = (uint32_t)(unsigned long long)t, thi = (uint32_t)((unsigned long long)t >> 32);
    int *recw = reinterpret_cast<int *>(rec);  // recw[2x] = parent (Next while walking)
    TreeState<LDS> bits;
    if constexpr (LDS) bits.w = lds_bits;
    else bits.recw = recw;
    constexpr int kWShift = TreeState<LDS>::kShift, kW = 1 << kWShift;
    const int nw = (n + kW - 1) >> kWShift;  // allocation words
    const int *__restrict__ bflag = GL ? lbf : g.bflag;
    const int4 *__restrict__ vrow = g.vrow;
    const int4 *__restrict__ edge = g.edge;  // set when the tree state is in global memory
    const int u = g.u;
    const int *__restrict__ rp = GL ? lrp : g.rp;
    const CT *__restrict__ col = GL ? lcol : reinterpret_cast<const CT *>(g.colv);  // int32, or uint16 when n <= 65536
    const double *__restrict__ cw = g.cw;
    const int *__restrict__ guide = g.guide;

    wait_global();  // the previous tree's record writes have landed
    if constexpr (LDS) {
        for (int i = lane; i < nwords; i += kWave) bits.w[i] = 0u;
    } else {
        for (int i = lane; i < n; i += kWave) rec[i] = make_int2(-1, kFree);
        wait_global();
    }
    for (int i = lane; i < 2 * kHashSlots; i += kWave) htab[i] = kWave;
    if (lane == 0) __hip_atomic_store(&win_base, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    wave_sync();
    if constexpr (BV) {  // several roots (one per block of the block-split graph)
        for (int i = lane; i < a.nroots; i += kWave) {
            const int r = a.roots[i];
            bits.set(r);
            rec[r] = make_int2(-1, r);
        }
    } else if (lane == 0) {
        bits.set(u);
        rec[u] = make_int2(-1, u);
    }
    wave_sync();

    int head = 0, tail = 0, cursor = 0;  // wave-uniform
    int mode = 0;                        // 0 idle, 1 speculative walk
    int my_e = 0, x = 0, s = 0, sk = 0, k = 0, r0 = 0, r1 = 0, fx = 0, pbits = 0;
    uint4 ph = make_uint4(0, 0, 0, 0);
    long long steps = 0, draws = 0;

    for (;;) {
        // ---------------------------------------------------------------- allocate
        // The idle lane of rank r takes the r-th not-in-tree vertex at or after `cursor`
        // (ascending start order).  A window of 64 bitmap words is scanned at once: every
        // lane finds its own start by a binary search over the lanes' prefix counts and a
        // select of the bit within that word, with no per-bit loop.
        const uint64_t idle = __ballot(mode == 0);
        const int want = min(__popcll(idle), rob - (tail - head));
        const int rank = __popcll(idle & lanemask_lt());
        int got = 0, mys = 0;
        while (got < want && cursor < n) {
            // With the tree state in the records, the window's words are read once and kept in
            // LDS while the cursor stays inside it.  A vertex that joined the tree since the
            // read still shows as free: it is allocated, and its walk finds it in the tree after
            // one step and ends without a commit (as the sequential algorithm skips it).
            int wbase = cursor >> kWShift;
            uint32_t fb = 0u;
            if constexpr (LDS) {
                if (wbase + lane < nw) fb = ~bits.word(wbase + lane, n);
            } else {
                // win_base is written by lane 0 and read by every lane: atomic accesses
                const int wb = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(&win_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT));
                if (wb >= 0 && wbase < wb + kWave) {
                    wbase = wb;
                } else {
                    win_fb[lane] = wbase + lane < nw ? ~bits.word(wbase + lane, n) : 0u;
                    if (lane == 0) __hip_atomic_store(&win_base, wbase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    wave_sync();
                }
                fb = win_fb[lane];  // this lane's own word
            }
            const int wi = wbase + lane;
            if (wi < nw) {
                fb &= (kW == 32 ? ~0u : (1u << kW) - 1u);
                const int d = cursor - (wi << kWShift);  // vertices of this word before the cursor
                if (d > 0) fb = d >= kW ? 0u : fb & (~0u << d);
                if (wi == nw - 1 && (n & (kW - 1))) fb &= (1u << (n & (kW - 1))) - 1u;
            } else {
                fb = 0u;
            }
            const int c = __popc(fb);
            const int incl = wave_scan_dpp(c);
            const int excl = incl - c;
            const int total = __shfl(incl, kWave - 1, kWave);
            const int need = want - got;
            const int j = rank - got;  // this lane's index among the window's free vertices
            int L = 0;                 // the lane whose word holds free vertex j
#pragma unroll
            for (int st = kWave / 2; st >= 1; st >>= 1)
                if (__shfl(excl, L + st, kWave) <= j) L += st;
            const uint32_t wL = (uint32_t)__shfl((int)fb, L, kWave);
            const int eL = __shfl(excl, L, kWave);
            if (mode == 0 && j >= 0 && j < min(total, need)) mys = ((wbase + L) << kWShift) + select_bit(wL, j - eL);
            if (total >= need) {
                got = want;
                cursor = __builtin_amdgcn_readfirstlane(__shfl(mys, select_bit64(idle, want - 1), kWave) + 1);
            } else {
                got += total;
                cursor = (wbase + kWave) << kWShift;
            }
        }
        if (got > 0) {
            if (mode == 0 && rank < got) {
                my_e = tail + rank;
                s = mys;
                if constexpr (BV) sk = a.skey[s];
                x = s;
                k = 0;
                mode = 1;
                if constexpr (LDS) {
                    r0 = rp[s];
                    r1 = rp[s + 1];
                    fx = bflag[s];
                } else {  // the vertex entry {row begin, row end, B_u flag}: one load
                    const int4 vr = vrow[s];
                    r0 = vr.x;
                    r1 = vr.y;
                    fx = vr.z;
                }
                pbits = 0;
                const int sl = my_e & robm;
                rob_s[sl] = (CT)s;
                rob_k[sl] = (short)kWalking;
            }
            tail += got;
        }
        if (head == tail && cursor >= n) break;
        wave_sync();

        // ---------------------------------------------------------------- one walk step
        if (mode == 1) {
            if ((k & 3) == 0)
                ph = philox4x32_10(make_uint4((uint32_t)(k >> 2), (uint32_t)(BV ? sk : s), tlo, thi), g.key0, g.key1);
            const int q = k & 3;
            const uint32_t w = q == 0 ? ph.x : (q == 1 ? ph.y : (q == 2 ? ph.z : ph.w));
            // y, its B_u flag and its row bounds.  With the tree bitmap in LDS (small graphs,
            // whose compact column and row arrays stay in cache): a column load, then the
            // flag, and the row bounds only if the walk goes on.  Otherwise one edge-entry load.
            const int e = r0 + step_index<WT>(w, r0, r1, cw, guide);
            int y, fy, ny0 = 0, ny1 = 0;
            if constexpr (LDS) {
                y = (int)col[e];
                fy = bflag[y];
            } else {
                const int4 ey = edge[e];
                y = ey.x;
                fy = ey.w;
                ny0 = ey.y;
                ny1 = ey.z;
            }
            // y's tree membership, with the chain value when the walk ends here
            bool in;
            int cvy = 0;
            if constexpr (LDS) {
                in = bits.test(y);
                if (in) {
                    cvy = recw[2 * y + 1];
                } else {
                    ny0 = rp[y];
                    ny1 = rp[y + 1];
                }
            } else {
                cvy = bits.nbx(y);  // membership and chain value in one load
                in = cvy != kFree;
            }
            consume(fy, cvy, ny0, ny1);  // no load may stay in flight into the commit phase
            if (in) cvy = cv_of(y, cvy);
            ++k;
            ++draws;
            const int sl = my_e & robm;
            const int eb = edge_bits(x, fx, y, fy);
            if (k <= kPathLds) {
                rob_p[sl][k - 1] = (CT)y;
                pbits |= eb << (2 * (k - 1));
                rob_pb[sl] = (unsigned short)pbits;
            } else {
                gpath[sl * (kPath - kPathLds) + (k - 1 - kPathLds)] = y | (eb << 30);
            }
            if (in) { rob_k[sl] = (short)k; rob_cv[sl] = (CT)cvy; mode = 0; }
            else if (k == kPath) { rob_k[sl] = (short)kOverflow; mode = 0; }
            else if (bits.test(s)) { rob_k[sl] = 0; mode = 0; }  // s absorbed: never walks
            else { x = y; fx = fy; r0 = ny0; r1 = ny1; }
        }
        wave_sync();

        // ---------------------------------------------------------------- in-order commit
        while (head < tail) {
            const int hs = rob_k[head & robm];
            if (hs == kWalking) break;
            if (hs == kContinue || hs == kRewalk) {
                // lane 0 runs the sequential algorithm for this start against the current tree
                // (all earlier starts are committed).  An overflowed walk whose record misses
                // the tree resumes after its record: the recorded steps become Next pointers.
                const int sl = head & robm;
                const int s0 = (int)rob_s[sl];
                if (!bits.test(s0)) {
                    uint32_t wk0 = (uint32_t)s0;  // the walk's Philox key
                    if constexpr (BV) wk0 = (uint32_t)a.skey[s0];
                    if (hs == kContinue) wait_global();  // recorded steps stored by another lane
                    int xs = s0;
                    const long long k0 = hs == kContinue ? kPath : 0;
                    if (lane == 0 && hs == kContinue) {
#pragma unroll 8
                        for (int j = 1; j <= kPath; ++j) {
                            const int xj = j <= kPathLds ? (int)rob_p[sl][j - 1]
                                                         : gpath[sl * (kPath - kPathLds) + (j - 1 - kPathLds)] & kVertexMask;
                            recw[2 * xs] = xj;
                            xs = xj;
                        }
                    }
                    long long kk = 0;
                    if constexpr (GL) {
                        // the conflict tables (all free now) hold the walk's Philox words meanwhile
                        xs = __shfl(xs, 0, kWave);
                        kk = walk_next_wave<CT, WT>(bits, recw, rp, col, cw, guide, wk0, xs, k0, tlo, thi, g.key0,
                                                    g.key1, reinterpret_cast<uint32_t *>(htab));
                        for (int i = lane; i < 4 * kWave; i += kWave) htab[i] = kWave;
                        wave_sync();
                        if (lane == 0) retrace_commit<true>(bits, recw, bflag, s0);
                    } else {
                        if (lane == 0)
                            kk = rewalk_commit<LDS, CT, WT>(bits, recw, rp, col, edge, vrow, cw, guide, bflag, s0, wk0,
                                                            xs, k0, tlo, thi, g.key0, g.key1);
                    }
                    if (lane == 0) {
                        steps += kk;
                        draws += kk - k0;
                    }
                }
                ++head;
                wave_sync();
                continue;
            }
            const int idx = head + lane;
            const int sk = idx < tail ? (int)rob_k[idx & robm] : kWalking;
            const uint64_t okm = __ballot(sk >= 0 && sk <= kPathLds);
            const int r = (~okm == 0ull) ? kWave : __builtin_ctzll(~okm);
            if (r > 0) {
                // Batch commit of the done entries head .. head+r-1 (walks of <= kPathLds steps), one
                // lane each, all planned against the current tree T0.  Entry j's plan is what
                // the sequential algorithm does unless an earlier entry of the batch adds a
                // vertex j has read (its start or a vertex before its truncation point); the
                // plan's written vertices go into the two minimum-writer tables, and the batch
                // commits up to the first lane that reads a vertex whose two slots both hold a
                // smaller lane (collisions only shorten the batch).  The head never conflicts.
                const bool act = lane < r;
                const int sl = idx & robm;
                const int K = act ? sk : 0;
                // xv[j] = x_j; bits j = edge bits of the step x_{j-1} -> x_j
                int xv[kPathLds + 1];
                xv[0] = act ? (int)rob_s[sl] : -1;
                const int pb = act ? (int)rob_pb[sl] : 0;
#pragma unroll
                for (int j = 1; j <= kPathLds; ++j) xv[j] = (j <= K) ? (int)rob_p[sl][j - 1] : -1;
                const bool live = K > 0 && !bits.test(act ? xv[0] : 0);
                int istar = kPathLds + 1;
#pragma unroll
                for (int j = kPathLds; j >= 1; --j)
                    if (live && j <= K && bits.test(xv[j])) istar = j;
                const bool bad = live && istar > K;  // cannot happen for a recorded walk
                // loop erasure in registers: keep = positions on the erased branch
                unsigned keep = 0u;
                if (live && !bad) {
                    int b = xv[0];
#pragma unroll
                    for (int step = 0; step <= kPathLds; ++step) {
                        int q = -1;
#pragma unroll
                        for (int j = 0; j <= kPathLds; ++j)
                            if (j < istar && xv[j] == b) q = j;
                        if (q < 0) break;
                        keep |= 1u << q;
                        if (q + 1 >= istar) break;
                        int nb = -1;
#pragma unroll
                        for (int j = 1; j <= kPathLds; ++j)
                            if (j == q + 1) nb = xv[j];
                        b = nb;
                    }
                }
                const uint64_t badm = __ballot(bad);
                if (badm & 1ull) {  // never expected: fall back to the exact re-walk
                    rob_k[head & robm] = (short)kRewalk;
                    wave_sync();
                    continue;
                }
                if (live && !bad) {
#pragma unroll
                    for (int j = 0; j <= kPathLds; ++j)
                        if ((keep >> j) & 1u) {
                            atomicMin(&hslot[hash_slot<LDS>(xv[j])], lane);
                            atomicMin(&hslot2[hash_slot2<LDS>(xv[j])], lane);
                        }
                }
                wave_sync();
                bool conflict = bad;
                if (live && !bad) {
#pragma unroll
                    for (int j = 0; j <= kPathLds; ++j)
                        if (j < istar && hslot[hash_slot<LDS>(xv[j])] < lane && hslot2[hash_slot2<LDS>(xv[j])] < lane)
                            conflict = true;
                }
                wave_sync();
                if (live && !bad) {
#pragma unroll
                    for (int j = 0; j <= kPathLds; ++j)
                        if ((keep >> j) & 1u) {
                            hslot[hash_slot<LDS>(xv[j])] = kWave;
                            hslot2[hash_slot2<LDS>(xv[j])] = kWave;
                        }
                }
                const uint64_t cm = __ballot(conflict);
                const int jstar = cm ? __builtin_ctzll(cm) : r;
                const bool commit = live && !bad && lane < jstar;
                int ya = -1;
#pragma unroll
                for (int j = 1; j <= kPathLds; ++j)
                    if (j == istar) ya = xv[j];
                int carry = commit ? (int)rob_cv[sl] : 0;
                const bool need = commit && istar < K;  // ya joined T after the walk passed it
                if (__ballot(need)) {
                    wait_global();
                    if (need) carry = cv_of(ya, load_nbx(recw, ya));
                }
                if (commit) {
                    // a kept x_j is the last visit of its vertex, so its tree edge is the
                    // recorded step x_j -> x_{j+1}, whose edge bits are step j+1's
                    int pv = ya;
#pragma unroll
                    for (int j = kPathLds; j >= 0; --j) {
                        if ((keep >> j) & 1u) {
                            const int v = xv[j];
                            const int mb = (int)((unsigned)(pb >> (2 * j)) << 30);  // j + 1 <= kPathLds
                            const int cv = mb ? v : carry;
                            rec[v] = make_int2(pv, carry | mb);
                            bits.set(v);
                            carry = cv;
                            pv = v;
                        }
                    }
                    steps += istar;
                }
                head += jstar;
                wave_sync();
                continue;
            }
            // head: recorded walk x_0..x_K, kPathLds < K <= 255 (an overflowed walk: its whole
            // record, K = 255), committed cooperatively; lane j holds x_{j+64c} and the edge bits
            // of the step into it, c = 0..3
            const int sl = head & robm;
            const int s0 = (int)rob_s[sl];
            if (!bits.test(s0)) {
                const bool ended = hs >= 0;  // the walk reached the tree it saw
                const int K = ended ? hs : kPath;
                int xv[4] = {-1, -1, -1, -1}, xb[4] = {0, 0, 0, 0};
                if (lane == 0) {
                    xv[0] = s0;
                } else if (lane <= min(K, kPathLds)) {
                    xv[0] = (int)rob_p[sl][lane - 1];
                    xb[0] = ((int)rob_pb[sl] >> (2 * (lane - 1))) & 3;
                }
                if (K > kPathLds) {
                    wait_global();  // steps beyond the LDS part were stored by other lanes
                    int e[4] = {0, 0, 0, 0};
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int j = c * kWave + lane;
                        if (j > kPathLds && j <= K) e[c] = gpath[sl * (kPath - kPathLds) + (j - 1 - kPathLds)];
                    }
                    consume(e[0], e[1], e[2], e[3]);
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int j = c * kWave + lane;
                        if (j > kPathLds && j <= K) {
                            xv[c] = e[c] & kVertexMask;
                            xb[c] = (int)((unsigned)e[c] >> 30);
                        }
                    }
                }
                int istar = -1;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (istar < 0 && c * kWave <= K) {
                        const int j = c * kWave + lane;
                        const bool valid = j >= 1 && j <= K;
                        const uint64_t im = __ballot(valid && bits.test(valid ? xv[c] : 0));
                        if (im) istar = c * kWave + __builtin_ctzll(im);
                    }
                }
                if (istar < 0) {
                    // an overflowed walk that still misses the tree resumes after its record; for
                    // a finished walk this cannot happen, and the re-walk keeps the commit exact
                    rob_k[sl] = (short)(ended ? kRewalk : kContinue);
                    wave_sync();
                    continue;
                }
                // loop erasure: from b, jump past b's last visit before istar
                int b = s0, blen = 0, ya = -1;
                for (;;) {
                    int qlast = -1;
#pragma unroll
                    for (int c = 3; c >= 0; --c) {
                        if (qlast < 0 && c * kWave < istar) {
                            const uint64_t mm = __ballot(c * kWave + lane < istar && xv[c] == b);
                            if (mm) qlast = c * kWave + 63 - __builtin_clzll(mm);
                        }
                    }
                    if (qlast < 0) break;  // unreachable for a recorded walk; never spin
                    const int nq = qlast + 1, cq = nq >> 6, lq = nq & 63;
                    const int nx = __shfl(sel4(cq, xv[0], xv[1], xv[2], xv[3]), lq, kWave);
                    const int nb = __shfl(sel4(cq, xb[0], xb[1], xb[2], xb[3]), lq, kWave);  // edge b -> nx
                    if (lane == 0) {
                        br[blen] = b | (nb << 30);
                        bits.set(b);
                    }
                    ++blen;
                    if (nq == istar) {
                        ya = nx;
                        break;
                    }
                    b = nx;
                }
                wave_sync();
                if (ya >= 0) {
                    // records of the branch b_0 = s .. b_{blen-1}, attached to ya
                    int carry;
                    if (ended && istar == K) {
                        carry = (int)rob_cv[sl];
                    } else {  // ya joined T after the walk passed it: its record was written since
                        wait_global();
                        carry = cv_of(ya, load_nbx(recw, ya));
                    }
                    for (int c = (blen - 1) >> 6; c >= 0; --c) {
                        const int i = c * kWave + lane;
                        const bool mine = i < blen;
                        const int be = mine ? br[i] : 0;
                        const int bi = be & kVertexMask;
                        const int nexti = mine ? (i + 1 < blen ? br[i + 1] & kVertexMask : ya) : 0;
                        const int mb = be & ~kVertexMask;  // the edge bits, in the record's flag position
                        const bool mk = mb != 0;
                        const uint64_t m = __ballot(mk);
                        const uint64_t above = lane < kWave - 1 ? (m & (~0ull << (lane + 1))) : 0ull;
                        const int nba = above ? br[c * kWave + __builtin_ctzll(above)] & kVertexMask : carry;
                        if (mine) rec[bi] = make_int2(nexti, nba | mb);
                        carry = m ? br[c * kWave + __builtin_ctzll(m)] & kVertexMask : carry;
                    }
                    if (lane == 0) steps += istar;
                }
            }
            wave_sync();
            for (int i = lane; i < kPath + 1; i += kWave) htab[i] = kWave;
            ++head;
            wave_sync();
        }
    }

    steps = wave_sum(steps);
    draws = wave_sum(draws);
    if (lane == 0) {
        if (a.steps) a.steps[tile] = steps;
        if (a.draws) a.draws[tile] = draws;
    }
    }  // next tile
}

// ======================================================================================
// Records of caller-supplied trees.  The sampler writes each vertex's record {parent,
// nba | flags} as it commits; for trees given as parent arrays the same records are built
// here.  One block per tree checks the parents, builds a child CSR (counting sort by
// parent), expands a BFS order of T level by level (children of one vertex contiguous),
// and writes the records top-down along that order, so a vertex's parent is done first.
// A parent array that is not a spanning tree rooted at u sets err |= 64.
// ======================================================================================
constexpr int kIvThreads = 256;

__global__ __launch_bounds__(kIvThreads) void tree_records_kernel(IntervalArgs a) {
    __shared__ int sh[kIvThreads / kWave + 1];
    __shared__ int bigq[kIvThreads];
    __shared__ int nbig;
    const int tid = threadIdx.x;
    const int n = a.n, u = a.u;
    const int *__restrict__ par = a.par + (long long)blockIdx.x * a.par_stride;
    int *__restrict__ scr = a.scratch + (long long)blockIdx.x * a.scratch_stride;
    int *__restrict__ cnt = scr;            // n
    int *__restrict__ cst = cnt + n;        // n + 1
    int *__restrict__ child = cst + n + 1;  // n
    int *__restrict__ ord = child + n;      // n
    int *__restrict__ fc = ord + n;         // n   first-child position of each position
    int *__restrict__ ppos = fc + n;        // n   parent position of each position
    int *__restrict__ lv = ppos + n;        // n + 2 level starts

    for (int v = tid; v < n; v += kIvThreads) cnt[v] = 0;
    __syncthreads();
    int bad = 0;
    for (int v = tid; v < n; v += kIvThreads) {
        if (v == u) continue;
        const int pv = par[v];
        if (pv < 0 || pv >= n || pv == v) bad = 1;
        else atomicAdd(&cnt[pv], 1);
    }
    if (__syncthreads_or(bad)) {
        if (tid == 0) atomicOr(a.err, 64);
        return;
    }
    int carry = 0;
    for (int base = 0; base < n; base += kIvThreads) {
        const int v = base + tid;
        const int c = v < n ? cnt[v] : 0;
        int tot;
        const int incl = block_incl_scan(c, &tot, sh);
        if (v < n) cst[v] = carry + incl - c;
        carry += tot;
    }
    if (tid == 0) cst[n] = carry;
    __syncthreads();
    for (int v = tid; v < n; v += kIvThreads) cnt[v] = cst[v];
    __syncthreads();
    for (int v = tid; v < n; v += kIvThreads)
        if (v != u) child[atomicAdd(&cnt[par[v]], 1)] = v;
    __syncthreads();

    // BFS order of T from u
    if (tid == 0) {
        ord[0] = u;
        ppos[0] = -1;
        lv[0] = 0;
    }
    __syncthreads();
    int ls = 0, le = 1, nlev = 0;
    while (ls < le) {
        carry = 0;
        for (int base = ls; base < le; base += kIvThreads) {
            const int i = base + tid;
            int c = 0;
            if (i < le) {
                const int xv = ord[i];
                c = cst[xv + 1] - cst[xv];
            }
            int tot;
            const int incl = block_incl_scan(c, &tot, sh);
            if (i < le) fc[i] = le + carry + incl - c;
            carry += tot;
        }
        __syncthreads();
        for (int base = ls; base < le; base += kIvThreads) {
            if (tid == 0) nbig = 0;
            __syncthreads();
            const int i = base + tid;
            if (i < le) {
                const int xv = ord[i];
                const int c0 = cst[xv], c = cst[xv + 1] - c0, f = fc[i];
                if (c <= 32) {
                    for (int j = 0; j < c; ++j) {
                        ord[f + j] = child[c0 + j];
                        ppos[f + j] = i;
                    }
                } else {
                    bigq[atomicAdd(&nbig, 1)] = i;
                }
            }
            __syncthreads();
            const int nb = nbig;
            for (int q = 0; q < nb; ++q) {
                const int i2 = bigq[q];
                const int xv = ord[i2];
                const int c0 = cst[xv], c = cst[xv + 1] - c0, f = fc[i2];
                for (int j = tid; j < c; j += kIvThreads) {
                    ord[f + j] = child[c0 + j];
                    ppos[f + j] = i2;
                }
            }
            __syncthreads();
        }
        ++nlev;
        if (tid == 0) lv[nlev] = le;
        ls = le;
        le += carry;
        __syncthreads();
    }
    if (tid == 0 && ls != n) atomicOr(a.err, 64);  // not a spanning tree rooted at u
    if (ls != n) return;

    // {parent, nba | marked << 31} top-down along the BFS order of T
    int2 *rec = a.rec + (long long)blockIdx.x * a.rec_stride;
    if (tid == 0) rec[u] = make_int2(-1, u);
    __syncthreads();
    for (int L = 1; L < nlev; ++L) {
        for (int j = lv[L] + tid; j < lv[L + 1]; j += kIvThreads) {
            const int xv = ord[j];
            const int pv = par[xv];
            const int nba = cv_of(pv, rec[pv].y);
            rec[xv] = make_int2(pv, nba | mark_bits(xv, a.bflag[xv], pv, a.bflag[pv]));
        }
        __syncthreads();
    }
}

// ======================================================================================
// Aggregation (Algorithm 2), on the {parent, chain} records: for v != u,
//   c_T(v) = [parent_T(v) = parB(v)]
//          + sum over marked strict T-ancestors x of v lying on P(v) of
//              +1 if parent_T(x) = parB(x),  -1 if parB(parent_T(x)) = x and parent_T(x) on P(v),
// which equals Algorithm 2's signed count term by term.  "On P(v)" is the B_u subtree test
// pre_B(x) <= pre_B(v) < pre_B(x) + size_B(x).  Thread per vertex over a chunk of resident
// trees; one int64 atomic per vertex and chunk, skipped when the sum is zero.
// ======================================================================================
// WT: weighted graph, the edge (parB(b), b) of P(v) counts +-F[b] (Ohm's-law factor in fixed
// point) instead of +-1.
template <bool WT, int CH>
__global__ __launch_bounds__(256) void aggregate_kernel(AggregateArgs a) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.n || v == a.u) return;
    const int t0 = blockIdx.y * CH;
    const int nt = min(a.ntrees - t0, CH);
    const int u = a.u;
    const int2 *__restrict__ bint = a.bint;
    const int pbv = a.parB[v];
    const int pv = bint[v].x;
    const int2 *__restrict__ rec0 = a.rec + (long long)t0 * a.rec_stride;
    // The chains of the chunk's trees are walked in lockstep, one step of every unfinished
    // chain per round, so their independent loads are in flight together.
    using Acc = typename std::conditional<WT, long long, int>::type;
    const long long *__restrict__ F = a.F;
    const Acc fv = WT ? (Acc)F[v] : (Acc)1;
    int x[CH];
    Acc sum = 0;
#pragma unroll
    for (int i = 0; i < CH; ++i) {
        x[i] = u;
        if (i < nt) {
            const int2 rv = rec0[(long long)i * a.rec_stride + v];
            sum += (rv.x == pbv) ? fv : (Acc)0;
            x[i] = nba_of(rv.y);
            if (x[i] >= a.n) x[i] = u;
        }
    }
    // a chain visits each T-ancestor at most once: n rounds bound it even on broken records
    for (int round = 0; round < a.n; ++round) {
        int2 rx[CH], bx[CH];
        bool act = false;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (x[i] != u) {
                act = true;
                rx[i] = rec0[(long long)i * a.rec_stride + x[i]];
                bx[i] = bint[x[i]];
            }
        }
        if (!act) break;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (x[i] != u) {
                // a forward x counts +1 if x is on P(v); a backward x counts -1 if parent_T(x),
                // a B_u child of x, is on P(v), which needs x on P(v) first
                if (bx[i].x <= pv && pv < bx[i].x + bx[i].y) {
                    if (rx[i].y & kFwdBit) {
                        if constexpr (WT) sum += F[x[i]];
                        else ++sum;
                    } else {
                        const int2 bp = bint[rx[i].x];
                        if (bp.x <= pv && pv < bp.x + bp.y) {
                            if constexpr (WT) sum -= F[rx[i].x];
                            else --sum;
                        }
                    }
                }
                x[i] = nba_of(rx[i].y);
                if (x[i] >= a.n) x[i] = u;  // never for sampled trees; keeps reads in bounds
            }
        }
    }
    if (sum != 0) atomicAdd((unsigned long long *)&a.counts[v], (unsigned long long)(long long)sum);
}

// Subtree intervals of B_u, level by level over the whole grid (B_u has ecc(u) + 1 levels):
// sizes bottom-up (each vertex adds its finished size to its parent), then pre-order
// numbers top-down (each vertex takes the next free range under its parent; the order of
// siblings is whatever the atomics give, and any order is a valid nesting).
__global__ void bsub_init_kernel(int n, int u, int *__restrict__ sz, int *__restrict__ cur, int *__restrict__ pre) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    sz[v] = 1;
    if (v == u) {
        pre[v] = 0;
        cur[v] = 1;
    }
}
// Children of one hub make up most of a level in small-world graphs; the lanes of a wave
// that share the parent of the wave's first active lane combine into one atomic.
__global__ __launch_bounds__(256) void bsub_size_kernel(int n, int d, const int *__restrict__ dist,
                                                        const int *__restrict__ parB, int *__restrict__ sz) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = v < n && dist[v] == d;
    const int p = act ? parB[v] : -1, val = act ? sz[v] : 0;
    const uint64_t am = __ballot(act);
    if (!am) return;
    const int leader = __builtin_ctzll(am);
    const int lp = __shfl(p, leader, kWave);
    const bool same = act && p == lp;
    const int tot = wave_sum(same ? val : 0);
    if (lane_id() == leader) atomicAdd(&sz[lp], tot);
    if (act && !same) atomicAdd(&sz[p], val);
}
__global__ __launch_bounds__(256) void bsub_pre_kernel(int n, int d, const int *__restrict__ dist,
                                                       const int *__restrict__ parB, const int *__restrict__ sz,
                                                       int *__restrict__ cur, int *__restrict__ pre) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = v < n && dist[v] == d;
    const int p = act ? parB[v] : -1, val = act ? sz[v] : 0;
    const uint64_t am = __ballot(act);
    if (!am) return;
    const int leader = __builtin_ctzll(am);
    const int lp = __shfl(p, leader, kWave);
    const bool same = act && p == lp;
    const int incl = wave_incl_scan(same ? val : 0);
    const int tot = __shfl(incl, kWave - 1, kWave);
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(&cur[lp], tot);
    base = __shfl(base, leader, kWave);
    int pv = 0;
    if (same) pv = base + incl - val;
    else if (act) pv = atomicAdd(&cur[p], val);
    if (act) {
        pre[v] = pv;
        cur[v] = pv + 1;
    }
}
__global__ void bsub_pack_kernel(int n, const int *__restrict__ parB, const int *__restrict__ pre,
                                 const int *__restrict__ sz, int2 *__restrict__ bint, int *__restrict__ bflag) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int pb = parB[v], z = sz[v];
    bint[v] = make_int2(pre[v], z);
    bflag[v] = (int)((unsigned)(pb + 1) | (z > 1 ? 0x80000000u : 0u));
}

// The pivot by BFS sweeps for a small graph, in one workgroup and with no host round trip:
// the same first source (largest degree, then smallest ID), the same level-synchronous BFS, the
// same bounds (the distances of the first sweep, then their running maximum) and next source
// (the farthest vertex, then smallest ID) as sweep_update_kernel, and the same choice (smallest
// bound, then smallest ID) as argmin_bound_kernel.  *pivot receives the choice.
constexpr int kSweepThreads = 1024;

__device__ __forceinline__ unsigned long long block_max_key(unsigned long long key, unsigned long long *sh) {
#pragma unroll
    for (int dd = 32; dd > 0; dd >>= 1) {
        const unsigned long long o = __shfl_xor(key, dd, 64);
        key = o > key ? o : key;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = key;
    __syncthreads();
    unsigned long long r = 0;
    for (int i = 0; i < kSweepThreads / kWave; ++i) r = sh[i] > r ? sh[i] : r;
    __syncthreads();  // every thread has read sh before it is written again
    return r;
}

template <int G>
__global__ __launch_bounds__(kSweepThreads) void sweep_small_kernel(RowMap m, int sweeps, int *__restrict__ dist,
                                                                    int *__restrict__ bound, int *__restrict__ pivot) {
    __shared__ unsigned long long shk[kSweepThreads / kWave];
    __shared__ int found;
    const int n = m.n, tid = threadIdx.x;
    const int nh = *m.nheavy;
    unsigned long long key = 0;
    for (int v = tid; v < n; v += kSweepThreads) {
        const unsigned long long k = ((unsigned long long)(unsigned)(m.rp[v + 1] - m.rp[v]) << 32) |
                                     (unsigned long long)(0xFFFFFFFFu - (unsigned)v);
        key = k > key ? k : key;
    }
    int src = (int)(0xFFFFFFFFu - (unsigned)(block_max_key(key, shk) & 0xFFFFFFFFull));
    for (int it = 0; it < sweeps; ++it) {
        for (int v = tid; v < n; v += kSweepThreads) dist[v] = (v == src) ? 0 : INT_MAX;
        for (int d = 0;; ++d) {
            if (tid == 0) found = 0;
            __syncthreads();
            int any = 0;
            for (int h = 0; h < nh; ++h) {
                const int v = m.heavy[h];
                if (dist[v] != d) continue;  // uniform in the block
                for (int e = m.rp[v] + tid; e < m.rp[v + 1]; e += kSweepThreads) {
                    const int y = m.col[e];
                    if (dist[y] > d + 1) {
                        dist[y] = d + 1;
                        any = 1;
                    }
                }
            }
            constexpr int rows_per_tile = kSweepThreads / G;
            const int g = tid / G, l = tid % G;
            for (int base = 0; base < n; base += rows_per_tile) {
                const int v = base + g;
                if (v >= n || dist[v] != d) continue;
                const int lo = m.rp[v], hi = m.rp[v + 1];
                if (hi - lo > m.heavy_thresh) continue;
                for (int e = lo + l; e < hi; e += G) {
                    const int y = m.col[e];
                    if (dist[y] > d + 1) {
                        dist[y] = d + 1;
                        any = 1;
                    }
                }
            }
            if (any) found = 1;
            __syncthreads();
            const int f = found;
            __syncthreads();  // every thread has read `found` before it is reset
            if (!f) break;
        }
        key = 0;
        for (int v = tid; v < n; v += kSweepThreads) {
            const int d = dist[v];
            bound[v] = it == 0 ? d : max(bound[v], d);
            const unsigned long long k = ((unsigned long long)(unsigned)d << 32) |
                                         (unsigned long long)(0xFFFFFFFFu - (unsigned)v);
            key = k > key ? k : key;
        }
        src = (int)(0xFFFFFFFFu - (unsigned)(block_max_key(key, shk) & 0xFFFFFFFFull));
    }
    key = 0;
    for (int v = tid; v < n; v += kSweepThreads) {
        const unsigned long long k = ((unsigned long long)(0x7FFFFFFFu - (unsigned)bound[v]) << 32) |
                                     (unsigned long long)(0xFFFFFFFFu - (unsigned)v);
        key = k > key ? k : key;
    }
    key = block_max_key(key, shk);
    if (tid == 0) *pivot = (int)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
}

// Set-up of a small graph in one workgroup: the BFS levels (the same minimum-ID parent
// rule as bfs_level_kernel), the connectivity check, and the subtree intervals and flag
// words of B_u (as the bsub_* kernels).  out[0] = ecc(u), out[1] = 1 if a vertex is
// unreached.  scratch holds 3n ints.
constexpr int kSetupThreads = 1024;

template <int G>
__global__ __launch_bounds__(kSetupThreads) void setup_small_kernel(RowMap m, int u, int *__restrict__ dist,
                                                                    int *__restrict__ parB, int *__restrict__ scratch,
                                                                    int2 *__restrict__ bint, int *__restrict__ bflag,
                                                                    int *__restrict__ out) {
    __shared__ int found, unreached;
    const int n = m.n, tid = threadIdx.x;
    int *__restrict__ sz = scratch;
    int *__restrict__ cur = scratch + n;
    int *__restrict__ pre = scratch + 2 * n;
    for (int v = tid; v < n; v += kSetupThreads) {
        dist[v] = (v == u) ? 0 : INT_MAX;
        parB[v] = (v == u) ? -1 : INT_MAX;
        sz[v] = 1;
    }
    if (tid == 0) unreached = 0;
    const int nh = *m.nheavy;
    int d = 0;
    for (;; ++d) {
        if (tid == 0) found = 0;
        __syncthreads();
        int any = 0;
        for (int h = 0; h < nh; ++h) {
            const int v = m.heavy[h];
            if (dist[v] != d) continue;  // uniform in the block
            for (int e = m.rp[v] + tid; e < m.rp[v + 1]; e += kSetupThreads) {
                const int y = m.col[e];
                const int dy = dist[y];
                if (dy > d) {
                    atomicMin(&parB[y], v);
                    if (dy != d + 1) dist[y] = d + 1;
                    any = 1;
                }
            }
        }
        constexpr int rows_per_tile = kSetupThreads / G;
        const int g = tid / G, l = tid % G;
        for (int base = 0; base < n; base += rows_per_tile) {
            const int v = base + g;
            if (v >= n || dist[v] != d) continue;
            const int lo = m.rp[v], hi = m.rp[v + 1];
            if (hi - lo > m.heavy_thresh) continue;
            for (int e = lo + l; e < hi; e += G) {
                const int y = m.col[e];
                const int dy = dist[y];
                if (dy > d) {
                    atomicMin(&parB[y], v);
                    if (dy != d + 1) dist[y] = d + 1;
                    any = 1;
                }
            }
        }
        if (any) found = 1;
        __syncthreads();
        const int f = found;
        __syncthreads();  // every thread has read `found` before it is reset
        if (!f) break;
    }
    const int ecc = d;
    for (int v = tid; v < n; v += kSetupThreads)
        if (dist[v] == INT_MAX) unreached = 1;
    __syncthreads();
    if (unreached) {
        if (tid == 0) {
            out[0] = ecc;
            out[1] = 1;
        }
        return;
    }
    // subtree sizes bottom-up, then pre-order ranges top-down, level by level
    for (int dd = ecc; dd >= 1; --dd) {
        for (int v = tid; v < n; v += kSetupThreads)
            if (dist[v] == dd) atomicAdd(&sz[parB[v]], sz[v]);
        __syncthreads();
    }
    if (tid == 0) {
        pre[u] = 0;
        cur[u] = 1;
    }
    __syncthreads();
    for (int dd = 1; dd <= ecc; ++dd) {
        for (int v = tid; v < n; v += kSetupThreads) {
            if (dist[v] == dd) {
                const int pv = atomicAdd(&cur[parB[v]], sz[v]);
                pre[v] = pv;
                cur[v] = pv + 1;
            }
        }
        __syncthreads();
    }
    for (int v = tid; v < n; v += kSetupThreads) {
        const int pb = parB[v], z = sz[v];
        bint[v] = make_int2(pre[v], z);
        bflag[v] = (int)((unsigned)(pb + 1) | (z > 1 ? 0x80000000u : 0u));
    }
    if (tid == 0) {
        out[0] = ecc;
        out[1] = 0;
    }
}


// parents[i][v] = rec_i[v].parent
__global__ void extract_parents_kernel(int n, int ntrees, const int2 *__restrict__ rec, long long rec_stride,
                                       int *__restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * ntrees) return;
    const long long t = i / n, v = i - t * n;
    out[i] = rec[t * rec_stride + v].x;
}

// ======================================================================================
// Measures that depend only on diag(L^+) (section on electrical closeness, Eq. elec-farness;
// Lemma on normalized random-walk betweenness; Kirchhoff index appendix):
//   tr = sum_v diag[v], farness[v] = n diag[v] + tr, closeness[v] = (n-1) / farness[v],
//   nrwb[v] = 1/n + tr / ((n-1) farness[v]), Kirchhoff index = n tr.
// The trace is summed by one workgroup in a fixed order (deterministic).
// ======================================================================================
constexpr int kTraceThreads = 1024;

__global__ __launch_bounds__(kTraceThreads) void trace_kernel(long long n, const double *__restrict__ diag,
                                                              double *__restrict__ scalars) {
    __shared__ double sh[kTraceThreads / kWave];
    double acc = 0.0;
    for (long long v = threadIdx.x; v < n; v += kTraceThreads) acc += diag[v];
    acc = block_sum_t<double>(acc, sh);
    if (threadIdx.x == 0) {
        scalars[0] = acc;
        scalars[1] = (double)n * acc;
    }
}

__global__ __launch_bounds__(256) void centrality_kernel(long long n, const double *__restrict__ diag,
                                                         const double *__restrict__ scalars,
                                                         double *__restrict__ farness, double *__restrict__ closeness,
                                                         double *__restrict__ nrwb) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const double tr = scalars[0];
    const double f = (double)n * diag[v] + tr;
    if (farness) farness[v] = f;
    if (closeness) closeness[v] = (double)(n - 1) / f;
    if (nrwb) nrwb[v] = 1.0 / (double)n + tr / ((double)(n - 1) * f);
}

// ======================================================================================
// Spanning-edge counts (Kirchhoff index appendix: for each edge, the number of sampled
// USTs it appears in).  Thread per vertex v != u over a chunk of resident trees: the edge
// v -> parent_T(v) is found by binary search in v's own ascending row (short for the
// children of hubs) and counted at that position; equal positions in a row of trees add
// with one atomic.  edge_fold_kernel then moves every count at an entry (a, b), a > b, to
// the entry (b, a), so each undirected edge is counted at (min, max).
// ======================================================================================
__global__ __launch_bounds__(256) void edge_count_kernel(EdgeCountArgs a) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.n || v == a.u) return;
    const int t0 = blockIdx.y * a.trees_per_chunk;
    const int t1 = min(a.ntrees, t0 + a.trees_per_chunk);
    long long cur = -1;
    int c = 0;
    for (int t = t0; t < t1; ++t) {
        const int p = a.rec[(long long)t * a.rec_stride + v].x;
        int lo = a.rp[v], hi = a.rp[v + 1];
        const int end = hi;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (a.col[mid] < p) lo = mid + 1;
            else hi = mid;
        }
        if (lo == end || a.col[lo] != p) continue;  // not a neighbour: never for a sampled tree
        if (lo == cur) {
            ++c;
        } else {
            if (c) atomicAdd((unsigned long long *)&a.counts[cur], (unsigned long long)c);
            cur = lo;
            c = 1;
        }
    }
    if (c) atomicAdd((unsigned long long *)&a.counts[cur], (unsigned long long)c);
}

// Thread per entry e = (a, b) with a > b and a nonzero count: add it to the entry (b, a)
// (binary search in row b) and clear it.  Entries (b, a) with b < a are never cleared, so
// each receives from exactly one entry.  The row a of entry e comes from a binary search
// over the row pointers.
__global__ __launch_bounds__(256) void edge_fold_kernel(int n, long long nnz, const int *__restrict__ rp,
                                                        const int *__restrict__ col, long long *__restrict__ counts) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const long long c = counts[e];
    if (c == 0) return;
    int lo = 0, hi = n;  // largest a with rp[a] <= e
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rp[mid] <= e) lo = mid;
        else hi = mid;
    }
    const int a = lo, b = col[e];
    if (b >= a) return;
    int l = rp[b], h = rp[b + 1];
    const int end = h;
    while (l < h) {
        const int mid = (l + h) >> 1;
        if (col[mid] < a) l = mid + 1;
        else h = mid;
    }
    if (l == end || col[l] != a) return;  // asymmetric input: left where it is
    atomicAdd((unsigned long long *)&counts[l], (unsigned long long)c);
    counts[e] = 0;
}

// Edge measures from spanning-edge counts (Kirchhoff index appendix): thread per CSR entry
// e = (a, b); the count sits at the entry (min, max) of the edge (the mirror entry (b, a) is
// found by binary search in row b); lev = c / q, r = lev / w(e), denom = 1 - (1 - theta) lev.
__global__ __launch_bounds__(256) void edge_resistance_kernel(int n, long long nnz, const long long *__restrict__ rp,
                                                              const int *__restrict__ col,
                                                              const double *__restrict__ w,
                                                              const long long *__restrict__ counts, double q,
                                                              double theta, double *__restrict__ r,
                                                              double *__restrict__ denom) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int lo = 0, hi = n;  // the row a: the largest a with rp[a] <= e
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rp[mid] <= e) lo = mid;
        else hi = mid;
    }
    const int a = lo, b = col[e];
    long long c = counts[e];
    if (b < a) {  // the count is at the mirror entry (b, a)
        long long l = rp[b], h = rp[b + 1];
        c = 0;
        while (l < h) {
            const long long mid = (l + h) >> 1;
            const int cm = col[mid];
            if (cm == a) {
                c = counts[mid];
                break;
            }
            if (cm < a) l = mid + 1;
            else h = mid;
        }
    }
    {
        // each operation rounded on its own, as the definition reads: no contraction into a fused
        // multiply-add
#pragma clang fp contract(off)
        const double lev = (double)c / q;
        if (r) r[e] = lev / (w ? w[e] : 1.0);
        if (denom) denom[e] = 1.0 - (1.0 - theta) * lev;
    }
}

// Final fill (Algorithm 1; Eq. diag-comp): diag[u] = x[u], diag[v] = R[v]/tau - x[u] + 2 x[v]
// ======================================================================================
// Weighted graphs (Section "Generalizations").  Set-up only: the running conductance sums
// of every row (the sampler's step table and the Laplacian's diagonal), the weight checks,
// the B-path resistances and the fixed-point edge factors of Algorithm 2.
// ======================================================================================
// Running sums taken left to right, so every device (and the CPU oracle) gets the same FP64
// sums: cw[e] = w[row start] + ... + w[e], wdeg[v] = the row total.  One thread per light
// row; rows above `heavy_thresh` entries are left to row_cumsum_heavy_kernel.
__global__ __launch_bounds__(256) void row_cumsum_kernel(int n, const int *__restrict__ rp, const double *__restrict__ w,
                                                         int heavy_thresh, double *__restrict__ cw,
                                                         double *__restrict__ wdeg) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        double run = 0.0;
        int e = rp[v];
        const int end = rp[v + 1];
        if (end - e > heavy_thresh) continue;
        for (; e + 8 <= end; e += 8) {  // eight loads in flight, the additions still in order
            double wv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) wv[k] = w[e + k];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                run += wv[k];
                cw[e + k] = run;
            }
        }
        for (; e < end; ++e) {
            run += w[e];
            cw[e] = run;
        }
        wdeg[v] = run;
    }
}

// A heavy row per wavefront: each 64-entry chunk is loaded at once (the next one while the
// current is summed), and the running sum passes through the lanes in order, one addition
// per entry as in the sequential loop; lane k keeps the sum up to its own entry.
__global__ __launch_bounds__(64) void row_cumsum_heavy_kernel(const int *__restrict__ rp, const double *__restrict__ w,
                                                              const int *__restrict__ heavy, const int *__restrict__ nheavy,
                                                              double *__restrict__ cw, double *__restrict__ wdeg) {
    const int nh = *nheavy;
    const int lane = threadIdx.x;
    for (int h = blockIdx.x; h < nh; h += gridDim.x) {
        const int v = heavy[h];
        const int r0 = rp[v], end = rp[v + 1];
        double run = 0.0;
        double wn = r0 + lane < end ? w[r0 + lane] : 0.0;
        for (int base = r0; base < end; base += kWave) {
            const double wc = wn;
            wn = base + kWave + lane < end ? w[base + kWave + lane] : 0.0;
            const int cnt = min(kWave, end - base);
            const long long bits = __double_as_longlong(wc);
            const int lo = (int)(bits & 0xFFFFFFFFll), hi = (int)(bits >> 32);
            double mine = 0.0;
            for (int k = 0; k < cnt; ++k) {
                const long long bk = ((long long)(unsigned)__builtin_amdgcn_readlane(hi, k) << 32) |
                                     (long long)(unsigned)__builtin_amdgcn_readlane(lo, k);
                run += __longlong_as_double(bk);
                if (lane == k) mine = run;
            }
            if (lane < cnt) cw[base + lane] = mine;
        }
        if (lane == 0) wdeg[v] = run;
    }
}

// Guide of the weighted step search, one thread per CSR entry e = (row v, bucket i):
// guide[e] = the first j (at most deg-1) with C[j] > t(w_i), w_i = ceil(i 2^32 / deg) the
// smallest word of bucket i.  The row is found by a binary search over the row pointers.
__global__ __launch_bounds__(256) void step_guide_kernel(int n, int nnz, const int *__restrict__ rp,
                                                         const double *__restrict__ cw, int *__restrict__ guide) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x) {
        int lo = 0, hi = n - 1;  // the last v with rp[v] <= e
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rp[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int r0 = rp[lo], deg = rp[lo + 1] - r0, i = e - r0;
        const unsigned long long wi = (((unsigned long long)i << 32) + (unsigned long long)(deg - 1)) / (unsigned)deg;
        const double ti = ((double)wi * 0x1p-32) * cw[r0 + deg - 1];
        int a = 0, b = deg - 1;  // the first j with ti < C[j], or deg-1
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (ti < cw[r0 + mid]) b = mid;
            else a = mid + 1;
        }
        guide[e] = a;
    }
}

// position of x in the ascending row [lo, hi), or -1
__device__ __forceinline__ int find_in_row(const int *__restrict__ col, int lo, int hi, int x) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int c = col[mid];
        if (c == x) return mid;
        if (c < x) lo = mid + 1;
        else hi = mid;
    }
    return -1;
}

// err |= 64 if a conductance is not positive and finite or differs from its mirror entry
__global__ __launch_bounds__(256) void check_weights_kernel(int n, const int *__restrict__ rp, const int *__restrict__ col,
                                                            const double *__restrict__ w, int *__restrict__ err) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        bool bad = false;
        for (int e = rp[v]; e < rp[v + 1]; ++e) {
            const double we = w[e];
            const int x = col[e];
            if (!(we > 0.0) || !isfinite(we) || x < 0 || x >= n) { bad = true; break; }
            const int f = find_in_row(col, rp[x], rp[x + 1], v);
            if (f < 0 || w[f] != we) { bad = true; break; }
        }
        if (bad) atomicOr(err, 64);
    }
}

// wB[v] = w(v, parB(v)) (0 at u), then rho(v) = sum of 1 / wB over P(v) from v towards u;
// the largest rho into *rmax_bits (bits of a non-negative double order like the values)
__global__ __launch_bounds__(256) void b_edge_weight_kernel(int n, int u, const int *__restrict__ rp,
                                                            const int *__restrict__ col, const double *__restrict__ w,
                                                            const int *__restrict__ parB, double *__restrict__ wB) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double wb = 0.0;
    if (v != u) {
        const int f = find_in_row(col, rp[v], rp[v + 1], parB[v]);
        wb = f >= 0 ? w[f] : 0.0;  // parB(v) is a neighbour of v
    }
    wB[v] = wb;
}
__global__ __launch_bounds__(256) void bpath_resist_kernel(int n, int u, const int *__restrict__ parB,
                                                           const double *__restrict__ wB,
                                                           unsigned long long *__restrict__ rmax_bits) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    double r = 0.0;
    if (v < n)
        for (int b = v; b != u; b = parB[b]) r += 1.0 / wB[b];
    unsigned long long bits = (unsigned long long)__double_as_longlong(r);
    for (int d = kWave / 2; d > 0; d >>= 1) bits = max(bits, (unsigned long long)__shfl_xor((long long)bits, d, kWave));
    if (lane_id() == 0 && bits) atomicMax(rmax_bits, bits);
}

// F[v] = llround(2^shift / wB[v]), F[u] = 0
__global__ void fixed_weights_kernel(int n, int u, const double *__restrict__ wB, double scale, long long *__restrict__ F) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    F[v] = v == u ? 0ll : llround(scale / wB[v]);
}

// walk steps and draws of `cnt` trees added to totals[0], totals[1] (one block)
__global__ __launch_bounds__(256) void sum_walks_kernel(int cnt, const long long *__restrict__ steps,
                                                        const long long *__restrict__ draws,
                                                        unsigned long long *__restrict__ totals) {
    long long a = 0, b = 0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        a += steps[i];
        b += draws[i];
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
        a += __shfl_xor(a, d, kWave);
        b += __shfl_xor(b, d, kWave);
    }
    if (lane_id() == 0) {
        atomicAdd(&totals[0], (unsigned long long)a);
        atomicAdd(&totals[1], (unsigned long long)b);
    }
}

// walk steps and draws of a batch's tiles added to their member's totals (totals[2 g], totals[2 g + 1])
__global__ __launch_bounds__(256) void tile_walks_kernel(int cnt, const WilsonTile *__restrict__ tiles,
                                                         const long long *__restrict__ steps,
                                                         const long long *__restrict__ draws,
                                                         unsigned long long *__restrict__ totals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const int g = tiles[i].graph;
    atomicAdd(&totals[2 * g], (unsigned long long)steps[i]);
    atomicAdd(&totals[2 * g + 1], (unsigned long long)draws[i]);
}

// den = tau, or tau 2^k for the fixed-point counts of a weighted graph
__global__ void combine_kernel(int n, int u, double den, const long long *__restrict__ counts,
                               const double *__restrict__ x, double *__restrict__ diag) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const double xu = x[u];
    diag[v] = (v == u) ? xu : (double)counts[v] / den - xu + 2.0 * x[v];
}

__global__ void philox_words_kernel(uint32_t key0, uint32_t key1, long long t, int s, long long k0, long long count,
                                    uint32_t *__restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const long long k = k0 + i;
    const uint4 o = philox4x32_10(make_uint4((uint32_t)(k >> 2), (uint32_t)s, (uint32_t)(unsigned long long)t,
                                             (uint32_t)((unsigned long long)t >> 32)), key0, key1);
    const int q = (int)(k & 3);
    out[i] = q == 0 ? o.x : (q == 1 ? o.y : (q == 2 ? o.z : o.w));
}

// ======================================================================================
// launchers
// ======================================================================================
static inline int blocks_for(long long n, int bs) { return (int)((n + bs - 1) / bs); }

hipError_t launch_col_to_u16(long long nnz, const int *col, unsigned short *col16, hipStream_t st) {
    col_to_u16_kernel<<<blocks_for(nnz, 256), 256, 0, st>>>(nnz, col, col16);
    return hipGetLastError();
}
hipError_t launch_rp_to_i32(int n, const long long *rp64, int *rp32, hipStream_t st) {
    rp_to_i32_kernel<<<blocks_for(n + 1, 256), 256, 0, st>>>(n, rp64, rp32);
    return hipGetLastError();
}
hipError_t launch_validate(int n, long long nnz, const long long *rp64, const int *col, int *err, hipStream_t st) {
    validate_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, nnz, rp64, col, err);
    return hipGetLastError();
}
hipError_t launch_argmax_degree(int n, const int *rp, unsigned long long *best, hipStream_t st) {
    argmax_degree_kernel<<<min(blocks_for(n, 256), 1024), 256, 0, st>>>(n, rp, best);
    return hipGetLastError();
}
hipError_t launch_sweep_update(int n, const int *dist, int *bound, int first, unsigned long long *far, hipStream_t st) {
    sweep_update_kernel<<<min(blocks_for(n, 256), 1024), 256, 0, st>>>(n, dist, bound, first, far);
    return hipGetLastError();
}
hipError_t launch_argmin_bound(int n, const int *bound, unsigned long long *best, hipStream_t st) {
    argmin_bound_kernel<<<min(blocks_for(n, 256), 1024), 256, 0, st>>>(n, bound, best);
    return hipGetLastError();
}
hipError_t launch_bfs_init(int n, int u, int *dist, int *parB, hipStream_t st) {
    bfs_init_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, u, dist, parB);
    return hipGetLastError();
}
static inline int row_grid(const RowMap &m, int G) {
    const long long tiles = ((long long)m.n + (256 / G) - 1) / (256 / G);
    return (int)std::min<long long>(std::max<long long>(tiles, 1), 4096);
}

hipError_t launch_bfs_level(const RowMap &m, int G, int d, int *dist, int *parB, int *found, const int *prev,
                            hipStream_t st) {
    const int grid = row_grid(m, G);
    USTD_DISPATCH_G(G, bfs_level_kernel<GG><<<grid, 256, 0, st>>>(m, d, dist, parB, found, prev));
    return hipGetLastError();
}
hipError_t launch_heavy_list(int n, const int *rp, int thresh, int *bcount, int *heavy, int *nheavy, hipStream_t st) {
    const int nb = blocks_for(n, 256);
    heavy_count_kernel<<<nb, 256, 0, st>>>(n, rp, thresh, bcount);
    heavy_scan_kernel<<<1, 256, 0, st>>>(nb, bcount, nheavy);
    heavy_write_kernel<<<nb, 256, 0, st>>>(n, rp, thresh, bcount, heavy);
    return hipGetLastError();
}
hipError_t launch_count_unreached(int n, const int *dist, int *err, hipStream_t st) {
    count_unreached_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, dist, err);
    return hipGetLastError();
}
template <bool LDS, typename CT, bool WT, bool BV = false>
int resident_of(size_t dyn, int *per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, wilson_kernel<LDS, CT, WT, false, BV>, 64, dyn) ==
           hipSuccess;
}
int wilson_resident_blocks(bool lds_bits, bool col16, bool weighted, int nwords, bool block_split) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const size_t dyn = lds_bits ? (size_t)nwords * 4 : 0;
    int ok;
    if (block_split) {
        if (lds_bits) ok = col16 ? resident_of<true, unsigned short, false, true>(dyn, &per_cu)
                                 : resident_of<true, int, false, true>(dyn, &per_cu);
        else ok = col16 ? resident_of<false, unsigned short, false, true>(0, &per_cu)
                        : resident_of<false, int, false, true>(0, &per_cu);
    } else if (lds_bits) {
        if (col16) ok = weighted ? resident_of<true, unsigned short, true>(dyn, &per_cu)
                                 : resident_of<true, unsigned short, false>(dyn, &per_cu);
        else ok = weighted ? resident_of<true, int, true>(dyn, &per_cu) : resident_of<true, int, false>(dyn, &per_cu);
    } else {
        if (col16) ok = weighted ? resident_of<false, unsigned short, true>(0, &per_cu)
                                 : resident_of<false, unsigned short, false>(0, &per_cu);
        else ok = weighted ? resident_of<false, int, true>(0, &per_cu) : resident_of<false, int, false>(0, &per_cu);
    }
    if (!ok) return 0;
    return std::max(1, per_cu) * std::max(1, cus);
}
long long wilson_graph_lds_bytes(int n, long long nnz) {
    return ((long long)(n + 1) * 4 + (long long)n * 4 + nnz * 2 + 3) / 4 * 4;
}
int wilson_resident_blocks_graph_lds(int nwords, long long graph_bytes) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(wilson_kernel<true, unsigned short, false, true>)) !=
        hipSuccess)
        return 0;
    const long long dyn = (long long)nwords * 4 + graph_bytes;
    const long long bytes = ((long long)fa.sharedSizeBytes + dyn + 255) / 256 * 256;
    if (bytes > 65536) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, wilson_kernel<true, unsigned short, false, true>, 64,
                                                     (size_t)dyn) != hipSuccess)
        return 0;
    const int by_lds = 2 * (int)(81920 / bytes);  // two 80 KB halves, whole blocks in each
    return std::max(0, std::min(per_cu, by_lds)) * std::max(1, cus);
}
template <bool LDS, typename CT>
void launch_wilson_t(const WilsonArgs &a, int blocks, bool weighted, bool bv, size_t dyn, hipStream_t st) {
    if (bv) wilson_kernel<LDS, CT, false, false, true><<<blocks, 64, dyn, st>>>(a);
    else if (weighted) wilson_kernel<LDS, CT, true><<<blocks, 64, dyn, st>>>(a);
    else wilson_kernel<LDS, CT, false><<<blocks, 64, dyn, st>>>(a);
}
hipError_t launch_wilson(const WilsonArgs &a, int blocks, bool lds_bits, bool col16, bool weighted, int nwords,
                         hipStream_t st, long long graph_lds_bytes, bool block_split) {
    if (block_split && (weighted || a.tiles || graph_lds_bytes > 0)) return hipErrorInvalidValue;
    if (graph_lds_bytes > 0) {
        if (!lds_bits || !col16 || weighted || a.tiles) return hipErrorInvalidValue;
        wilson_kernel<true, unsigned short, false, true>
            <<<blocks, 64, (size_t)nwords * 4 + (size_t)graph_lds_bytes, st>>>(a);
        return hipGetLastError();
    }
    if (lds_bits) {
        const size_t dyn = (size_t)nwords * 4;
        if (col16) launch_wilson_t<true, unsigned short>(a, blocks, weighted, block_split, dyn, st);
        else launch_wilson_t<true, int>(a, blocks, weighted, block_split, dyn, st);
    } else {
        if (col16) launch_wilson_t<false, unsigned short>(a, blocks, weighted, block_split, 0, st);
        else launch_wilson_t<false, int>(a, blocks, weighted, block_split, 0, st);
    }
    return hipGetLastError();
}
hipError_t launch_tree_records(const IntervalArgs &a, int ntrees, hipStream_t st) {
    tree_records_kernel<<<ntrees, kIvThreads, 0, st>>>(a);
    return hipGetLastError();
}
hipError_t launch_extract_parents(int n, int ntrees, const int2 *rec, long long rec_stride, int *out, hipStream_t st) {
    // a dispatch counts its work-items in 32 bits: at most 2^31 (vertex, tree) items per launch
    const int chunk = (int)std::max(1ll, std::min<long long>(ntrees, (1ll << 31) / std::max(n, 1)));
    for (int t0 = 0; t0 < ntrees; t0 += chunk) {
        const int nt = std::min(chunk, ntrees - t0);
        extract_parents_kernel<<<blocks_for((long long)n * nt, 256), 256, 0, st>>>(
            n, nt, rec + (long long)t0 * rec_stride, rec_stride, out + (long long)t0 * n);
    }
    return hipGetLastError();
}
hipError_t launch_b_intervals(int n, int u, int ecc, const int *dist, const int *parB, int *scratch, int2 *bint,
                              int *bflag, hipStream_t st) {
    int *sz = scratch, *cur = scratch + n, *pre = scratch + 2 * n;
    const int nb = blocks_for(n, 256);
    bsub_init_kernel<<<nb, 256, 0, st>>>(n, u, sz, cur, pre);
    for (int d = ecc; d >= 1; --d) bsub_size_kernel<<<nb, 256, 0, st>>>(n, d, dist, parB, sz);
    for (int d = 1; d <= ecc; ++d) bsub_pre_kernel<<<nb, 256, 0, st>>>(n, d, dist, parB, sz, cur, pre);
    bsub_pack_kernel<<<nb, 256, 0, st>>>(n, parB, pre, sz, bint, bflag);
    return hipGetLastError();
}
hipError_t launch_sweep_small(const RowMap &m, int G, int sweeps, int *dist, int *bound, int *pivot, hipStream_t st) {
    USTD_DISPATCH_G(G, (sweep_small_kernel<GG><<<1, kSweepThreads, 0, st>>>(m, sweeps, dist, bound, pivot)));
    return hipGetLastError();
}
hipError_t launch_setup_small(const RowMap &m, int G, int u, int *dist, int *parB, int *scratch, int2 *bint,
                              int *bflag, int *out, hipStream_t st) {
    USTD_DISPATCH_G(G, (setup_small_kernel<GG><<<1, kSetupThreads, 0, st>>>(m, u, dist, parB, scratch, bint, bflag,
                                                                             out)));
    return hipGetLastError();
}
hipError_t launch_centralities(long long n, const double *diag, double *farness, double *closeness, double *nrwb,
                               double *scalars, hipStream_t st) {
    trace_kernel<<<1, kTraceThreads, 0, st>>>(n, diag, scalars);
    if (farness || closeness || nrwb)
        centrality_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, diag, scalars, farness, closeness, nrwb);
    return hipGetLastError();
}
hipError_t launch_edge_counts(const EdgeCountArgs &a, hipStream_t st) {
    dim3 grid(blocks_for(a.n, 256), (a.ntrees + a.trees_per_chunk - 1) / a.trees_per_chunk);
    edge_count_kernel<<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}
hipError_t launch_edge_fold(int n, long long nnz, const int *rp, const int *col, long long *counts, hipStream_t st) {
    edge_fold_kernel<<<blocks_for(nnz, 256), 256, 0, st>>>(n, nnz, rp, col, counts);
    return hipGetLastError();
}
hipError_t launch_aggregate(const AggregateArgs &a, hipStream_t st) {
    const int ch = a.chunk == kAggChunkLarge ? kAggChunkLarge : kAggChunk;
    dim3 grid(blocks_for(a.n, 256), (a.ntrees + ch - 1) / ch);
    if (ch == kAggChunkLarge) {
        if (a.F) aggregate_kernel<true, kAggChunkLarge><<<grid, 256, 0, st>>>(a);
        else aggregate_kernel<false, kAggChunkLarge><<<grid, 256, 0, st>>>(a);
    } else {
        if (a.F) aggregate_kernel<true, kAggChunk><<<grid, 256, 0, st>>>(a);
        else aggregate_kernel<false, kAggChunk><<<grid, 256, 0, st>>>(a);
    }
    return hipGetLastError();
}
__global__ void fill_i64_kernel(long long n, long long *__restrict__ a, long long v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}
__global__ void add_i64_kernel(long long n, const long long *__restrict__ a, long long *__restrict__ b) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] += a[i];
}
hipError_t launch_fill_i64(long long n, long long *a, long long v, hipStream_t st) {
    if (n > 0) fill_i64_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, a, v);
    return hipGetLastError();
}
hipError_t launch_add_i64(long long n, const long long *a, long long *b, hipStream_t st) {
    if (n > 0) add_i64_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, a, b);
    return hipGetLastError();
}
hipError_t launch_edge_resistance(int n, long long nnz, const long long *rp, const int *col, const double *w,
                                  const long long *counts, double q, double theta, double *r, double *denom,
                                  hipStream_t st) {
    if (nnz > 0)
        edge_resistance_kernel<<<blocks_for(nnz, 256), 256, 0, st>>>(n, nnz, rp, col, w, counts, q, theta, r, denom);
    return hipGetLastError();
}
hipError_t launch_combine(int n, int u, double den, const long long *counts, const double *x, double *diag,
                          hipStream_t st) {
    combine_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, u, den, counts, x, diag);
    return hipGetLastError();
}
hipError_t launch_sum_walks(int cnt, const long long *steps, const long long *draws, unsigned long long *totals,
                            hipStream_t st) {
    sum_walks_kernel<<<1, 256, 0, st>>>(cnt, steps, draws, totals);
    return hipGetLastError();
}
hipError_t launch_tile_walks(int cnt, const WilsonTile *tiles, const long long *steps, const long long *draws,
                             unsigned long long *totals, hipStream_t st) {
    if (cnt > 0) tile_walks_kernel<<<blocks_for(cnt, 256), 256, 0, st>>>(cnt, tiles, steps, draws, totals);
    return hipGetLastError();
}
hipError_t launch_row_cumsum(int n, int nnz, const int *rp, const double *w, int heavy_thresh, const int *heavy,
                             const int *nheavy, double *cw, double *wdeg, int *guide, hipStream_t st) {
    row_cumsum_kernel<<<std::min(blocks_for(n, 256), 4096), 256, 0, st>>>(n, rp, w, heavy_thresh, cw, wdeg);
    row_cumsum_heavy_kernel<<<1024, kWave, 0, st>>>(rp, w, heavy, nheavy, cw, wdeg);
    step_guide_kernel<<<std::min(blocks_for(nnz, 256), 8192), 256, 0, st>>>(n, nnz, rp, cw, guide);
    return hipGetLastError();
}
__global__ void vertex_rows_kernel(int n, const int *__restrict__ rp, const int *__restrict__ bflag,
                                   int4 *__restrict__ vrow) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) vrow[v] = make_int4(rp[v], rp[v + 1], bflag[v], 0);
}
hipError_t launch_vertex_rows(int n, const int *rp, const int *bflag, int4 *vrow, hipStream_t st) {
    vertex_rows_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, rp, bflag, vrow);
    return hipGetLastError();
}
__global__ void edge_rows_kernel(long long nnz, const int *__restrict__ col, const int4 *__restrict__ vrow,
                                 int4 *__restrict__ edge) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nnz; i += (long long)gridDim.x * blockDim.x) {
        const int y = col[i];
        const int4 r = vrow[y];
        edge[i] = make_int4(y, r.x, r.y, r.z);
    }
}
hipError_t launch_edge_rows(long long nnz, const int *col, const int4 *vrow, int4 *edge, hipStream_t st) {
    edge_rows_kernel<<<(int)std::min<long long>(blocks_for(nnz, 256), 16384), 256, 0, st>>>(nnz, col, vrow, edge);
    return hipGetLastError();
}
hipError_t launch_check_weights(int n, const int *rp, const int *col, const double *w, int *err, hipStream_t st) {
    check_weights_kernel<<<std::min(blocks_for(n, 256), 4096), 256, 0, st>>>(n, rp, col, w, err);
    return hipGetLastError();
}
hipError_t launch_bpath(int n, int u, const int *rp, const int *col, const double *w, const int *parB, double *wB,
                        unsigned long long *rmax_bits, hipStream_t st) {
    b_edge_weight_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, u, rp, col, w, parB, wB);
    bpath_resist_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, u, parB, wB, rmax_bits);
    return hipGetLastError();
}
hipError_t launch_fixed_weights(int n, int u, const double *wB, int shift, long long *F, hipStream_t st) {
    fixed_weights_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, u, wB, ldexp(1.0, shift), F);
    return hipGetLastError();
}
hipError_t launch_philox_words(uint32_t key0, uint32_t key1, long long t, int s, long long k0, long long count,
                               uint32_t *out, hipStream_t st) {
    philox_words_kernel<<<blocks_for(count, 256), 256, 0, st>>>(key0, key1, t, s, k0, count, out);
    return hipGetLastError();
}

}  // namespace ustd
