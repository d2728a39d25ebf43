// ustd_blocks.hip -- Wilson's algorithm per biconnected component (engineering appendix of
// Angriman et al., after Hayashi et al.): the set-up that splits the graph into its blocks and
// lays out the block-split graph G* the sampler runs on, and the per-batch kernels that join
// the block trees into spanning trees of G rooted at the pivot.
//
// Blocks (Tarjan and Vishkin's construction on the BFS tree B_u, with its preorder numbers and
// subtree sizes): tree edges are named by their child vertex; two tree edges are joined when a
// non-tree edge connects their unrelated subtrees, and a tree edge (v, w) is joined with v's
// own tree edge when w's subtree reaches outside v's (its low / high preorder numbers); a
// non-tree edge belongs to the block of the tree edge above its later endpoint.  The joins run
// through a lock-free union-find whose representatives (vertex IDs) name the blocks.
//
// G* has one vertex ("slot") per pair (v, B) with v in block B, numbered in the order of e(v, B),
// the CSR position of v's first edge inside B; its edges are G's edges, each between the slots
// of its endpoints in its block, in the order of the CSR rows.  G* is a disjoint union of the
// blocks, so Wilson's algorithm on G* with every block's root in the tree at the start is
// Wilson's algorithm in each block.  A slot's walk is keyed by e(v, B).
#include "ustd_kernels.hpp"

#include <algorithm>
#include <climits>

namespace ustd {

// ======================================================================================
// exclusive scan of int counts (multi-block): out[i] = in[0] + ... + in[i-1], out[n] = total
// ======================================================================================
constexpr int kScanThreads = 256, kScanItems = 4, kScanTile = kScanThreads * kScanItems;

__global__ __launch_bounds__(kScanThreads) void scan_tile_sums_kernel(const int *__restrict__ in, long long n,
                                                                      int *__restrict__ sums) {
    __shared__ int sh[kScanThreads / kWave + 1];
    const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    int tot;
    block_incl_scan(s, &tot, sh);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// one block: exclusive scan of the tile sums in place; *total = their sum
__global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(int *__restrict__ sums, int ntiles,
                                                                 int *__restrict__ total) {
    __shared__ int sh[kScanThreads / kWave + 1];
    int carry = 0;
    for (int base = 0; base < ntiles; base += kScanThreads) {
        const int i = base + threadIdx.x;
        const int c = i < ntiles ? sums[i] : 0;
        int tot;
        const int incl = block_incl_scan(c, &tot, sh);
        if (i < ntiles) sums[i] = carry + incl - c;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const int *__restrict__ in, long long n,
                                                                  const int *__restrict__ sums,
                                                                  const int *__restrict__ total,
                                                                  int *__restrict__ out) {
    __shared__ int sh[kScanThreads / kWave + 1];
    const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    const int incl = block_incl_scan(s, &tot, sh);
    int run = sums[blockIdx.x] + incl - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) {
            out[base + k] = run;
            run += v[k];
        }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = *total;
}

long long scan_tiles(long long n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t launch_scan_excl(const int *in, int *out, long long n, int *sums, int *total, hipStream_t st) {
    const long long tiles = std::max(1ll, scan_tiles(n));
    scan_tile_sums_kernel<<<(unsigned)tiles, kScanThreads, 0, st>>>(in, n, sums);
    scan_sums_kernel<<<1, kScanThreads, 0, st>>>(sums, (int)tiles, total);
    scan_apply_kernel<<<(unsigned)tiles, kScanThreads, 0, st>>>(in, n, sums, total, out);
    return hipGetLastError();
}

// ======================================================================================
// blocks
// ======================================================================================
// low / high of each vertex's own row: the smallest and largest preorder number among v and its
// neighbours (rows by G lanes, heavy rows by a whole block, as the BFS)
template <int G>
__global__ __launch_bounds__(256) void bc_local_kernel(RowMap m, const int2 *__restrict__ bint, int *__restrict__ lo,
                                                       int *__restrict__ hi) {
    __shared__ int shl[256 / kWave], shh[256 / kWave];
    const int nh = *m.nheavy;
    for (int h = blockIdx.x; h < nh; h += gridDim.x) {
        const int v = m.heavy[h];
        int a = INT_MAX, b = INT_MIN;
        for (int e = m.rp[v] + threadIdx.x; e < m.rp[v + 1]; e += blockDim.x) {
            const int p = bint[m.col[e]].x;
            a = min(a, p);
            b = max(b, p);
        }
        for (int d = kWave / 2; d > 0; d >>= 1) {
            a = min(a, __shfl_xor(a, d, kWave));
            b = max(b, __shfl_xor(b, d, kWave));
        }
        if (lane_id() == 0) {
            shl[threadIdx.x / kWave] = a;
            shh[threadIdx.x / kWave] = b;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int pv = bint[v].x;
            int ra = pv, rb = pv;
            for (int i = 0; i < (int)blockDim.x / kWave; ++i) {
                ra = min(ra, shl[i]);
                rb = max(rb, shh[i]);
            }
            lo[v] = ra;
            hi[v] = rb;
        }
        __syncthreads();
    }
    const int rows_per_tile = 256 / G;
    const int g = threadIdx.x / G, l = threadIdx.x % G;
    for (int tile = blockIdx.x; tile * rows_per_tile < m.n; tile += gridDim.x) {
        const int v = tile * rows_per_tile + g;
        const bool ok = v < m.n;
        const int r0 = ok ? m.rp[v] : 0, r1 = ok ? m.rp[v + 1] : 0;
        const bool light = ok && (r1 - r0 <= m.heavy_thresh);
        int a = INT_MAX, b = INT_MIN;
        if (light)
            for (int e = r0 + l; e < r1; e += G) {
                const int p = bint[m.col[e]].x;
                a = min(a, p);
                b = max(b, p);
            }
#pragma unroll
        for (int d = G / 2; d > 0; d >>= 1) {
            a = min(a, __shfl_xor(a, d, G));
            b = max(b, __shfl_xor(b, d, G));
        }
        if (light && l == 0) {
            const int pv = bint[v].x;
            lo[v] = min(a, pv);
            hi[v] = max(b, pv);
        }
    }
}

// subtree minimum / maximum, one BFS level at a time from the deepest
__global__ void bc_subtree_kernel(int n, int d, const int *__restrict__ dist, const int *__restrict__ parB,
                                  int *__restrict__ lo, int *__restrict__ hi) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || dist[v] != d) return;
    const int p = parB[v];
    atomicMin(&lo[p], lo[v]);
    atomicMax(&hi[p], hi[v]);
}

__global__ void bc_uf_init_kernel(int n, int *__restrict__ uf) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) uf[v] = v;
}

// Union-find with agent-scope atomics (the parents are read and written by every workgroup);
// the smaller representative wins, so every set's representative is its smallest vertex.
__device__ __forceinline__ int uf_get(const int *uf, int x) {
    return __hip_atomic_load(uf + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int uf_find(int *uf, int x) {
    for (;;) {
        const int p = uf_get(uf, x);
        if (p == x) return x;
        const int gp = uf_get(uf, p);
        if (gp != p) atomicCAS(uf + x, p, gp);  // path halving; losing the race is harmless
        x = p;
    }
}
__device__ __forceinline__ void uf_unite(int *uf, int a, int b) {
    for (;;) {
        a = uf_find(uf, a);
        b = uf_find(uf, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(uf + b, b, a) == b) return;  // b was still a representative: hooked under a
    }
}

__device__ __forceinline__ bool in_subtree(int2 anc, int pre) { return anc.x <= pre && pre < anc.x + anc.y; }

// The joins: (i) a tree edge (v, w), v = parB(w) != u, with v's own tree edge when w's subtree
// has a neighbour outside v's subtree; (ii) for every non-tree edge {a, b} (a < b) whose
// endpoints are unrelated in B_u, the tree edges of a and b.  Thread per vertex and its row's
// entries (rows by G lanes, heavy rows by a block).
template <int G>
__global__ __launch_bounds__(256) void bc_union_kernel(RowMap m, int u, const int *__restrict__ parB,
                                                       const int2 *__restrict__ bint, const int *__restrict__ lo,
                                                       const int *__restrict__ hi, int *__restrict__ uf) {
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < m.n; w += gridDim.x * blockDim.x) {
        if (w == u) continue;
        const int v = parB[w];
        if (v == u) continue;
        const int2 bv = bint[v];
        if (lo[w] < bv.x || hi[w] >= bv.x + bv.y) uf_unite(uf, w, v);
    }
    auto entry = [&](int a, int b) {
        if (b <= a || parB[a] == b || parB[b] == a) return;
        const int2 ba = bint[a], bb = bint[b];
        if (in_subtree(ba, bb.x) || in_subtree(bb, ba.x)) return;
        uf_unite(uf, a, b);
    };
    const int nh = *m.nheavy;
    for (int h = blockIdx.x; h < nh; h += gridDim.x) {
        const int a = m.heavy[h];
        for (int e = m.rp[a] + threadIdx.x; e < m.rp[a + 1]; e += blockDim.x) entry(a, m.col[e]);
    }
    const int rows_per_tile = 256 / G;
    const int g = threadIdx.x / G, l = threadIdx.x % G;
    for (int tile = blockIdx.x; tile * rows_per_tile < m.n; tile += gridDim.x) {
        const int a = tile * rows_per_tile + g;
        if (a >= m.n) continue;
        const int r0 = m.rp[a], r1 = m.rp[a + 1];
        if (r1 - r0 > m.heavy_thresh) continue;
        for (int e = r0 + l; e < r1; e += G) entry(a, m.col[e]);
    }
}

__global__ void bc_flatten_kernel(int n, int *__restrict__ uf) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) uf[v] = uf_find(uf, v);
}

// the row a of CSR entry e (the largest a with rp[a] <= e)
__device__ __forceinline__ int row_of(const int *__restrict__ rp, int n, long long e) {
    int lo2 = 0, hi2 = n;
    while (hi2 - lo2 > 1) {
        const int mid = (lo2 + hi2) >> 1;
        if (rp[mid] <= e) lo2 = mid;
        else hi2 = mid;
    }
    return lo2;
}

// block of every entry; the first entry of each (vertex, block): firstPar[a] for a's own block
// (the block of its tree edge), firstTop[b] for the block b whose top vertex a is
__global__ void bc_entry_kernel(int n, long long nnz, int u, const int *__restrict__ rp, const int *__restrict__ col,
                                const int *__restrict__ parB, const int2 *__restrict__ bint,
                                const int *__restrict__ uf, int *__restrict__ eblk, int *__restrict__ firstPar,
                                int *__restrict__ firstTop) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int a = row_of(rp, n, e), b = col[e];
    int blk;
    if (parB[b] == a) blk = uf[b];
    else if (parB[a] == b) blk = uf[a];
    else blk = bint[a].x < bint[b].x ? uf[b] : uf[a];
    eblk[e] = blk;
    if (a != u && blk == uf[a]) atomicMin(&firstPar[a], (int)e);
    else atomicMin(&firstTop[blk], (int)e);
}

// slot flag of every entry: the first entry of its row inside its block
__global__ void bc_slot_flag_kernel(int n, long long nnz, int u, const int *__restrict__ rp,
                                    const int *__restrict__ eblk, const int *__restrict__ uf,
                                    const int *__restrict__ firstPar, const int *__restrict__ firstTop,
                                    int *__restrict__ flag) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int a = row_of(rp, n, e), blk = eblk[e];
    const int first = (a != u && blk == uf[a]) ? firstPar[a] : firstTop[blk];
    flag[e] = first == (int)e ? 1 : 0;
}

// slot arrays from the scanned flags: vertex, key e(v, B) and block of each slot; the slot of
// each vertex in its own block (slotPar) and of each block's top vertex (slotTop)
__global__ void bc_slot_kernel(int n, long long nnz, int u, const int *__restrict__ rp, const int *__restrict__ flag,
                               const int *__restrict__ sid, const int *__restrict__ eblk, const int *__restrict__ uf,
                               int *__restrict__ vtx, int *__restrict__ skey, int *__restrict__ sblk,
                               int *__restrict__ slotPar, int *__restrict__ slotTop) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz || !flag[e]) return;
    const int a = row_of(rp, n, e), blk = eblk[e], s = sid[e];
    vtx[s] = a;
    skey[s] = (int)e;
    sblk[s] = blk;
    if (a != u && blk == uf[a]) slotPar[a] = s;
    else slotTop[blk] = s;
}

__device__ __forceinline__ int slot_of(int v, int blk, int u, const int *__restrict__ uf,
                                       const int *__restrict__ slotPar, const int *__restrict__ slotTop) {
    return (v != u && blk == uf[v]) ? slotPar[v] : slotTop[blk];
}

// degree of every slot (its row's entries inside its block)
__global__ void bc_slot_degree_kernel(int n, long long nnz, int u, const int *__restrict__ rp,
                                      const int *__restrict__ eblk, const int *__restrict__ uf,
                                      const int *__restrict__ slotPar, const int *__restrict__ slotTop,
                                      int *__restrict__ deg) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int a = row_of(rp, n, e);
    atomicAdd(&deg[slot_of(a, eblk[e], u, uf, slotPar, slotTop)], 1);
}

// Columns of G*: one wavefront per row of G.  A row whose entries all lie in one block keeps
// its order; a cut vertex's row is split by block, stably: each 64-entry chunk ranks every lane
// among the earlier lanes of its slot, and the first lane of each slot advances that slot's
// cursor by the slot's entries in the chunk.
__global__ __launch_bounds__(64) void bc_columns_kernel(int n, int u, const int *__restrict__ rp,
                                                        const int *__restrict__ col, const int *__restrict__ eblk,
                                                        const int *__restrict__ uf,
                                                        const int *__restrict__ slotPar,
                                                        const int *__restrict__ slotTop,
                                                        const int *__restrict__ rps, int *__restrict__ cursor,
                                                        int *__restrict__ cols) {
    const int lane = threadIdx.x;
    for (int a = blockIdx.x; a < n; a += gridDim.x) {
        const int r0 = rp[a], r1 = rp[a + 1];
        for (int base = r0; base < r1; base += kWave) {
            const int e = base + lane;
            const bool act = e < r1;
            int key = -1, target = 0;
            if (act) {
                const int blk = eblk[e], b = col[e];
                key = slot_of(a, blk, u, uf, slotPar, slotTop);
                target = slot_of(b, blk, u, uf, slotPar, slotTop);
            }
            int rank = 0, cnt = 0, leader = lane;
            for (int j = 0; j < kWave; ++j) {
                const int kj = __shfl(key, j, kWave);
                if (act && kj == key) {
                    if (j < lane) ++rank;
                    if (j < leader) leader = j;
                    ++cnt;
                }
            }
            int start = 0;
            if (act && leader == lane) start = atomicAdd(&cursor[key], cnt);
            start = __shfl(start, leader, kWave);
            if (act) cols[rps[key] + start + rank] = target;
        }
    }
}

// root of each block: the slot of largest degree inside it, the smallest vertex ID on ties,
// as the maximum of (degree << 32 | ~vertex)
__global__ void bc_root_key_kernel(int nslots, const int *__restrict__ rps, const int *__restrict__ vtx,
                                   const int *__restrict__ sblk, unsigned long long *__restrict__ key) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    const unsigned long long k = ((unsigned long long)(unsigned)(rps[s + 1] - rps[s]) << 32) |
                                 (unsigned long long)(0xFFFFFFFFu - (unsigned)vtx[s]);
    atomicMax(&key[sblk[s]], k);
}

__global__ void bc_root_flag_kernel(int nslots, const int *__restrict__ vtx, const int *__restrict__ sblk,
                                    const unsigned long long *__restrict__ key, int *__restrict__ flag) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    flag[s] = (unsigned)(key[sblk[s]] & 0xFFFFFFFFull) == 0xFFFFFFFFu - (unsigned)vtx[s] ? 1 : 0;
}

// the slot of each block's top vertex (the vertex of the block closest to u)
__global__ void bc_top_flag_kernel(int nslots, const int *__restrict__ sblk, const int *__restrict__ slotTop,
                                   int *__restrict__ flag) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nslots) flag[s] = slotTop[sblk[s]] == s ? 1 : 0;
}

// list of the flagged slots, in slot order (pos: the exclusive scan of the flags)
__global__ void bc_compact_kernel(int nslots, const int *__restrict__ flag, const int *__restrict__ pos,
                                  int *__restrict__ list) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nslots && flag[s]) list[pos[s]] = s;
}

__global__ void fill_i32_kernel(long long n, int *__restrict__ a, int v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// ======================================================================================
// per batch: join the block trees
// ======================================================================================
// Re-root every block's tree at its top vertex's slot: thread per (tree, block); the path from
// the top slot up to the block's root is reversed (at most the block's size steps).
__global__ void bc_reroot_kernel(int ntop, const int *__restrict__ tops, int ntrees, int nslots,
                                 int2 *__restrict__ recs, long long stride) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)ntop * ntrees) return;
    const long long t = i / ntop;
    int *par = reinterpret_cast<int *>(recs + t * stride);  // par[2 s] = parent slot of s
    int x = tops[i - t * ntop], prev = -1;
    for (int steps = 0; x >= 0 && x < nslots && steps < nslots; ++steps) {  // a path of a tree: bounded
        const int up = par[2 * x];
        par[2 * x] = prev;
        prev = x;
        x = up;
    }
}

// parent in G of every vertex v != u: the vertex of the parent slot of v's slot in its own block
__global__ void bc_map_parents_kernel(int n, int u, int ntrees, const int *__restrict__ slotPar,
                                      const int *__restrict__ vtx, const int2 *__restrict__ recs, long long sstride,
                                      int2 *__restrict__ rec, long long stride) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * ntrees) return;
    const long long t = i / n;
    const int v = (int)(i - t * n);
    int *out = reinterpret_cast<int *>(rec + t * stride);
    const int ps = v == u ? -1 : recs[t * sstride + slotPar[v]].x;
    out[2 * v] = ps >= 0 ? vtx[ps] : -1;
}

// the {nba | marks} half of each vertex's record for Algorithm 2, from the parents: the marks
// of v and its tree edge, and the nearest marked strict ancestor nba(v) (u if none).  A vertex
// y is marked when its own tree edge (y, parent(y)) is an edge of B_u.
__device__ __forceinline__ int bf_parent_b(int f) { return (int)((unsigned)f & 0x7FFFFFFFu) - 1; }
__device__ __forceinline__ int marks_of(int x, int fx, int px, int fpx) {
    const unsigned fwd = px == bf_parent_b(fx), bwd = bf_parent_b(fpx) == x;
    const unsigned m = ((unsigned)fx >> 31) & (fwd | bwd);
    return (int)((m << 31) | ((m & fwd) << 30));
}

// nba by pointer jumping, in place in the record's second word: jw(v) = J | done << 31, where J
// is an ancestor of v such that every vertex from parent(v) up to J is unmarked and not u
// (not done), or J = nba(v) (done).  Start: J = parent(v), done when parent(v) is u or marked.
// A step replaces jw(v) by jw(J): nba(v) = nba(J) when J is unmarked, and the path covered
// doubles.  Any value of jw(J) that another thread has stored keeps the invariant, so the
// steps run concurrently without ordering; the words are single 32-bit loads and stores.
constexpr unsigned kJumpDone = 0x80000000u;

__global__ void bc_nba_init_kernel(int n, int u, int ntrees, const int *__restrict__ bflag, int2 *__restrict__ rec,
                                   long long stride) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * ntrees) return;
    const long long t = i / n;
    const int v = (int)(i - t * n);
    int *r = reinterpret_cast<int *>(rec + t * stride);
    const int pv = v == u ? -1 : r[2 * v];
    unsigned jw;
    if (pv < 0 || pv >= n || pv == u) {  // out-of-range never for a joined tree; keeps accesses in bounds
        jw = (unsigned)u | kJumpDone;
    } else {
        const int ppv = r[2 * pv];
        const bool marked = ppv >= 0 && ppv < n && marks_of(pv, bflag[pv], ppv, bflag[ppv]) != 0;
        jw = (unsigned)pv | (marked ? kJumpDone : 0u);
    }
    r[2 * v + 1] = (int)jw;
}

__global__ void bc_nba_jump_kernel(int n, int ntrees, int2 *__restrict__ rec, long long stride) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * ntrees) return;
    const long long t = i / n;
    const int v = (int)(i - t * n);
    int *r = reinterpret_cast<int *>(rec + t * stride);
    unsigned jw = __hip_atomic_load(r + 2 * v + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // each step moves J at least one vertex up the tree: at most n steps
    for (int steps = 0; !(jw & kJumpDone) && steps < n; ++steps) {
        const int x = (int)(jw & ~kJumpDone);
        if (x >= n) {
            jw = kJumpDone;  // never for a joined tree
            break;
        }
        jw = __hip_atomic_load(r + 2 * x + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(r + 2 * v + 1, (int)jw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// the final record word: nba(v) | marks of v
__global__ void bc_records_kernel(int n, int u, int ntrees, const int *__restrict__ bflag, int2 *__restrict__ rec,
                                  long long stride) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * ntrees) return;
    const long long t = i / n;
    const int v = (int)(i - t * n);
    int *r = reinterpret_cast<int *>(rec + t * stride);
    if (v == u) {
        r[2 * v + 1] = u;
        return;
    }
    const int pv = r[2 * v];
    const unsigned jw = (unsigned)r[2 * v + 1];
    int y = (int)(jw & ~kJumpDone);
    if (!(jw & kJumpDone) || y >= n) y = u;  // never for a joined tree
    const int mv = pv >= 0 && pv < n ? marks_of(v, bflag[v], pv, bflag[pv]) : 0;
    r[2 * v + 1] = y | mv;
}

// ======================================================================================
// launchers
// ======================================================================================
static inline unsigned bgrid(long long n, int bs) { return (unsigned)std::max(1ll, (n + bs - 1) / bs); }

hipError_t launch_bc_blocks(const RowMap &m, int G, int u, int ecc, const int *dist, const int *parB,
                            const int2 *bint, int *lo, int *hi, int *uf, hipStream_t st) {
    const int n = m.n;
    int grid = (int)std::min<long long>(std::max<long long>(((long long)n + (256 / G) - 1) / (256 / G), 1), 4096);
    USTD_DISPATCH_G(G, (bc_local_kernel<GG><<<grid, 256, 0, st>>>(m, bint, lo, hi)));
    for (int d = ecc; d >= 1; --d) bc_subtree_kernel<<<bgrid(n, 256), 256, 0, st>>>(n, d, dist, parB, lo, hi);
    bc_uf_init_kernel<<<bgrid(n, 256), 256, 0, st>>>(n, uf);
    USTD_DISPATCH_G(G, (bc_union_kernel<GG><<<grid, 256, 0, st>>>(m, u, parB, bint, lo, hi, uf)));
    bc_flatten_kernel<<<bgrid(n, 256), 256, 0, st>>>(n, uf);
    return hipGetLastError();
}

hipError_t launch_bc_entries(int n, long long nnz, int u, const int *rp, const int *col, const int *parB,
                             const int2 *bint, const int *uf, int *eblk, int *firstPar, int *firstTop, int *flag,
                             hipStream_t st) {
    bc_entry_kernel<<<bgrid(nnz, 256), 256, 0, st>>>(n, nnz, u, rp, col, parB, bint, uf, eblk, firstPar, firstTop);
    bc_slot_flag_kernel<<<bgrid(nnz, 256), 256, 0, st>>>(n, nnz, u, rp, eblk, uf, firstPar, firstTop, flag);
    return hipGetLastError();
}

hipError_t launch_bc_slots(int n, long long nnz, int u, const int *rp, const int *flag, const int *sid,
                           const int *eblk, const int *uf, int *vtx, int *skey, int *sblk, int *slotPar, int *slotTop,
                           int *deg, hipStream_t st) {
    bc_slot_kernel<<<bgrid(nnz, 256), 256, 0, st>>>(n, nnz, u, rp, flag, sid, eblk, uf, vtx, skey, sblk, slotPar,
                                                     slotTop);
    bc_slot_degree_kernel<<<bgrid(nnz, 256), 256, 0, st>>>(n, nnz, u, rp, eblk, uf, slotPar, slotTop, deg);
    return hipGetLastError();
}

hipError_t launch_bc_columns(int n, int u, const int *rp, const int *col, const int *eblk, const int *uf,
                             const int *slotPar, const int *slotTop, const int *rps, int *cursor, int *cols,
                             hipStream_t st) {
    bc_columns_kernel<<<(unsigned)std::min(n, 65536), 64, 0, st>>>(n, u, rp, col, eblk, uf, slotPar, slotTop, rps,
                                                                    cursor, cols);
    return hipGetLastError();
}

hipError_t launch_bc_roots(int nslots, const int *rps, const int *vtx, const int *sblk, unsigned long long *key,
                           int *flag, hipStream_t st) {
    bc_root_key_kernel<<<bgrid(nslots, 256), 256, 0, st>>>(nslots, rps, vtx, sblk, key);
    bc_root_flag_kernel<<<bgrid(nslots, 256), 256, 0, st>>>(nslots, vtx, sblk, key, flag);
    return hipGetLastError();
}

hipError_t launch_bc_top_flags(int nslots, const int *sblk, const int *slotTop, int *flag, hipStream_t st) {
    bc_top_flag_kernel<<<bgrid(nslots, 256), 256, 0, st>>>(nslots, sblk, slotTop, flag);
    return hipGetLastError();
}

hipError_t launch_bc_compact(int nslots, const int *flag, const int *pos, int *list, hipStream_t st) {
    bc_compact_kernel<<<bgrid(nslots, 256), 256, 0, st>>>(nslots, flag, pos, list);
    return hipGetLastError();
}

hipError_t launch_fill_i32(long long n, int *a, int v, hipStream_t st) {
    if (n > 0) fill_i32_kernel<<<bgrid(n, 256), 256, 0, st>>>(n, a, v);
    return hipGetLastError();
}

hipError_t launch_bc_join(int n, int u, int ntrees, int ntop, int nslots, const int *tops, const int *slotPar,
                          const int *vtx, int2 *recs, long long sstride, int2 *rec, long long stride,
                          const int *bflag, hipStream_t st) {
    if (ntrees <= 0) return hipSuccess;
    // One work-item per (vertex, tree), and a dispatch counts its work-items in 32 bits: the
    // trees go in chunks of at most 2^31 work-items per launch (each tree is independent).
    const long long per = std::max<long long>({(long long)n, (long long)ntop, 1ll});
    const int chunk = (int)std::max(1ll, std::min<long long>(ntrees, (1ll << 31) / per));
    for (int t0 = 0; t0 < ntrees; t0 += chunk) {
        const int nt = std::min(chunk, ntrees - t0);
        int2 *rs = recs + (long long)t0 * sstride;
        int2 *rr = rec + (long long)t0 * stride;
        bc_reroot_kernel<<<bgrid((long long)ntop * nt, 256), 256, 0, st>>>(ntop, tops, nt, nslots, rs, sstride);
        bc_map_parents_kernel<<<bgrid((long long)n * nt, 256), 256, 0, st>>>(n, u, nt, slotPar, vtx, rs, sstride,
                                                                             rr, stride);
        bc_nba_init_kernel<<<bgrid((long long)n * nt, 256), 256, 0, st>>>(n, u, nt, bflag, rr, stride);
        bc_nba_jump_kernel<<<bgrid((long long)n * nt, 256), 256, 0, st>>>(n, nt, rr, stride);
        bc_records_kernel<<<bgrid((long long)n * nt, 256), 256, 0, st>>>(n, u, nt, bflag, rr, stride);
    }
    return hipGetLastError();
}

}  // namespace ustd
