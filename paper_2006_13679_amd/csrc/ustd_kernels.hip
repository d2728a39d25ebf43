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

#include <climits>

namespace ustd {

// ======================================================================================
// graph set-up
// ======================================================================================
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

__global__ void bfs_init_kernel(int n, int u, int *__restrict__ dist, int *__restrict__ parB) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) {
        dist[v] = (v == u) ? 0 : INT_MAX;
        parB[v] = (v == u) ? -1 : INT_MAX;
    }
}

// One BFS level: every vertex at distance d offers itself as parent to its unvisited
// neighbours; atomicMin keeps the smallest-ID one among all of them, which is the
// minimum-ID neighbour one level closer to u.  `found` counts vertices reached.
__global__ void bfs_level_kernel(int n, const int *__restrict__ rp, const int *__restrict__ col, int d,
                                 int *__restrict__ dist, int *__restrict__ parB, int *__restrict__ found) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || dist[v] != d) return;
    int any = 0;
    for (int e = rp[v]; e < rp[v + 1]; ++e) {
        const int y = col[e];
        const int dy = dist[y];
        if (dy > d) {
            atomicMin(&parB[y], v);
            if (dy != d + 1) dist[y] = d + 1;
            any = 1;
        }
    }
    if (any) atomicOr(found, 1);
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
//   - runs of one-step walks (s -> y) commit in parallel, one lane each;
//   - recorded walks of 2..63 steps commit cooperatively with ballots (one ballot finds
//     the truncation point, one per branch vertex finds its last visit);
//   - walks longer than the record are re-walked from s by one lane against the current
//     tree (the sequential algorithm for that start, Next pointers in the parent array).
// ======================================================================================
namespace {

constexpr int kRobMax = 256;   // reorder-buffer entries (LDS)
constexpr int kPath = 63;      // recorded steps per speculative walk (x_1..x_63)
constexpr int kWalking = -1, kOverflow = -2;

template <bool LDS>
struct TreeBits {
    uint32_t *w;
    __device__ __forceinline__ uint32_t word(int i) const {
        if (LDS) return w[i];
        return __hip_atomic_load(w + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ bool test(int v) const { return (word(v >> 5) >> (v & 31)) & 1u; }
    __device__ __forceinline__ void set(int v) const { atomicOr(w + (v >> 5), 1u << (v & 31)); }
};

}  // namespace

template <bool LDS>
__global__ __launch_bounds__(64) void wilson_kernel(WilsonArgs a) {
    extern __shared__ uint32_t lds_bits[];
    __shared__ int rob_s[kRobMax], rob_k[kRobMax], rob_y[kRobMax];
    __shared__ int cand[kWave];

    const int lane = threadIdx.x;
    const int n = a.n;
    const int rob = a.rob;  // power of two <= kRobMax
    const int robm = rob - 1;
    const long long t = a.tree_begin + blockIdx.x;
    const uint32_t tlo = (uint32_t)(unsigned long long)t, thi = (uint32_t)((unsigned long long)t >> 32);
    int *__restrict__ par = a.par + (long long)blockIdx.x * a.par_stride;
    int *__restrict__ path = a.path + (long long)blockIdx.x * ((long long)rob * kPath);
    TreeBits<LDS> bits{LDS ? lds_bits : a.bits + (long long)blockIdx.x * a.nwords};
    const int *__restrict__ rp = a.rp;
    const int *__restrict__ col = a.col;

    for (int i = lane; i < a.nwords; i += kWave) {
        if (LDS) bits.w[i] = 0u;
        else __hip_atomic_store(bits.w + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (lane == 0) {
        bits.set(a.u);
        par[a.u] = -1;
    }
    __syncthreads();

    int head = 0, tail = 0, cursor = 0;  // wave-uniform
    int seq_lane = -1;                   // wave-uniform: lane re-walking the head entry
    int mode = 0;                        // 0 idle, 1 speculative walk, 2 re-walk, 3 re-walk done
    int my_e = 0, x = 0, s = 0, k = 0;
    uint4 ph = make_uint4(0, 0, 0, 0);
    long long steps = 0, draws = 0;

    for (;;) {
        // ---------------------------------------------------------------- allocate
        const uint64_t idle = __ballot(mode == 0);
        const int want = min(__popcll(idle), rob - (tail - head));
        int got = 0;
        while (got < want && cursor < n) {
            const int wbase = cursor >> 5;
            const int wi = wbase + lane;
            uint32_t fb = 0u;
            if (wi < a.nwords) {
                fb = ~bits.word(wi);
                if (lane == 0) fb &= ~0u << (cursor & 31);
                if (wi == a.nwords - 1 && (n & 31)) fb &= (1u << (n & 31)) - 1u;
            }
            const int c = __popc(fb);
            const int incl = wave_incl_scan(c);
            const int total = __shfl(incl, kWave - 1, kWave);
            const int need = want - got;
            int r = incl - c;
            while (fb && r < need) {
                cand[got + r] = wi * 32 + (__ffs(fb) - 1);
                ++r;
                fb &= fb - 1u;
            }
            __syncthreads();
            if (total >= need) {
                got = want;
                cursor = cand[want - 1] + 1;
            } else {
                got += total;
                cursor = (wbase + kWave) * 32;
            }
        }
        if (got > 0) {
            const int rank = __popcll(idle & lanemask_lt());
            if (mode == 0 && rank < got) {
                my_e = tail + rank;
                s = cand[rank];
                x = s;
                k = 0;
                mode = 1;
                rob_s[my_e & robm] = s;
                rob_k[my_e & robm] = kWalking;
            }
            tail += got;
        }
        if (head == tail && cursor >= n) break;
        __syncthreads();

        // ---------------------------------------------------------------- one walk step
        if (mode == 1 || mode == 2) {
            if ((k & 3) == 0) ph = philox4x32_10(make_uint4((uint32_t)(k >> 2), (uint32_t)s, tlo, thi), a.key0, a.key1);
            const int q = k & 3;
            const uint32_t w = q == 0 ? ph.x : (q == 1 ? ph.y : (q == 2 ? ph.z : ph.w));
            const int rs = rp[x];
            const int deg = rp[x + 1] - rs;
            const int y = col[rs + (int)__umulhi(w, (uint32_t)deg)];
            ++k;
            ++draws;
            const bool in = bits.test(y);
            if (mode == 1) {
                const int sl = my_e & robm;
                if (k == 1) rob_y[sl] = y;
                path[sl * kPath + k - 1] = y;
                if (in) { rob_k[sl] = k; mode = 0; }
                else if (k == kPath) { rob_k[sl] = kOverflow; mode = 0; }
                else if (bits.test(s)) { rob_k[sl] = 0; mode = 0; }  // s absorbed: never walks
                else x = y;
            } else {
                par[x] = y;  // Next pointer; becomes the parent when x joins T
                if (in) {
                    int z = s;
                    while (!bits.test(z)) {
                        bits.set(z);
                        z = par[z];
                    }
                    mode = 3;
                } else {
                    x = y;
                }
            }
        }
        __syncthreads();
        if (seq_lane >= 0) {
            if (__shfl(mode, seq_lane, kWave) == 3) {
                if (lane == seq_lane) {
                    steps += k;
                    mode = 0;
                }
                ++head;
                seq_lane = -1;
            }
        }

        // ---------------------------------------------------------------- in-order commit
        while (head < tail && seq_lane < 0) {
            const int hs = rob_k[head & robm];
            if (hs == kWalking) break;
            if (hs == kOverflow) {
                const int s0 = rob_s[head & robm];
                if (bits.test(s0)) { ++head; continue; }
                const uint64_t idl = __ballot(mode == 0);
                if (idl == 0) break;
                const int L = __ffsll((unsigned long long)idl) - 1;
                if (lane == L) { mode = 2; s = s0; x = s0; k = 0; }
                seq_lane = L;
                break;
            }
            const int idx = head + lane;
            const int sk = idx < tail ? rob_k[idx & robm] : kWalking;
            const uint64_t fm = __ballot(sk == 0 || sk == 1);
            const int r = (~fm == 0ull) ? kWave : __builtin_ctzll(~fm);
            if (r > 0) {
                if (lane < r && sk == 1) {
                    const int sl = idx & robm;
                    const int ss = rob_s[sl];
                    if (!bits.test(ss)) {
                        bits.set(ss);
                        par[ss] = rob_y[sl];
                        steps += 1;
                    }
                }
                head += r;
                __syncthreads();
                continue;
            }
            // recorded walk x_0..x_K, 2 <= K <= 63: truncate at the first vertex in T, then
            // follow successors after last visits
            const int sl = head & robm;
            const int s0 = rob_s[sl];
            if (!bits.test(s0)) {
                const bool valid = lane >= 1 && lane <= hs;
                const int xj = lane == 0 ? s0 : (valid ? path[sl * kPath + lane - 1] : -1);
                const uint64_t im = __ballot(valid && bits.test(valid ? xj : 0));
                if (im == 0ull) {
                    // cannot happen for a correctly recorded walk; re-walk to stay exact
                    rob_k[sl] = kOverflow;
                    __syncthreads();
                    continue;
                }
                const int istar = __builtin_ctzll(im);
                int b = s0;
                for (;;) {
                    const uint64_t mm = __ballot(lane < istar && xj == b);
                    if (mm == 0ull) break;  // unreachable for a recorded walk; never spin
                    const int qlast = 63 - __builtin_clzll(mm);
                    const int nx = __shfl(xj, qlast + 1, kWave);
                    if (lane == 0) {
                        par[b] = nx;
                        bits.set(b);
                    }
                    if (qlast + 1 == istar) break;
                    b = nx;
                }
                if (lane == 0) steps += istar;
            }
            ++head;
            __syncthreads();
        }
    }

    steps = wave_sum(steps);
    draws = wave_sum(draws);
    if (lane == 0) {
        if (a.steps) a.steps[blockIdx.x] = steps;
        if (a.draws) a.draws[blockIdx.x] = draws;
    }
}

// ======================================================================================
// Tree intervals.  Algorithm 2 asks whether v lies below an edge of T, which the paper
// answers with DFS discovery/finish times.  Any subtree-interval labelling answers it the
// same way: v is in the subtree of b  <=>  pre[b] <= pre[v] < pre[b] + size[b].  One block
// per tree builds a child CSR (counting sort by parent), expands a BFS order of T level
// by level (children of one vertex are contiguous), sums subtree sizes bottom-up with
// per-level prefix sums, and assigns pre-order numbers top-down as parent's number + 1 +
// sizes of the earlier siblings.  Output: {parent, pre, size, 0} per vertex.
// ======================================================================================
constexpr int kIvThreads = 256;

__global__ __launch_bounds__(kIvThreads) void intervals_kernel(IntervalArgs a) {
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
    int *__restrict__ sz = ppos + n;        // n
    int *__restrict__ ps = sz + n;          // n   per-level inclusive prefix sums of sz
    int *__restrict__ pre = ps + n;         // n
    int *__restrict__ lv = pre + n;         // n + 2 level starts
    int4 *__restrict__ pk = a.pk + (long long)blockIdx.x * a.pk_stride;

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

    // subtree sizes, deepest level first; ps holds the inclusive prefix of the level below
    for (int L = nlev - 1; L >= 0; --L) {
        const int lb = lv[L], le2 = lv[L + 1];
        for (int i = lb + tid; i < le2; i += kIvThreads) {
            const int xv = ord[i];
            const int c = cst[xv + 1] - cst[xv];
            int sv = 1;
            if (c > 0) {
                const int f = fc[i];
                sv += ps[f + c - 1] - (f > le2 ? ps[f - 1] : 0);
            }
            sz[i] = sv;
        }
        __syncthreads();
        carry = 0;
        for (int base = lb; base < le2; base += kIvThreads) {
            const int i = base + tid;
            const int sv = i < le2 ? sz[i] : 0;
            int tot;
            const int incl = block_incl_scan(sv, &tot, sh);
            if (i < le2) ps[i] = carry + incl;
            carry += tot;
        }
        __syncthreads();
    }
    // pre-order numbers, top level first
    if (tid == 0) pre[0] = 0;
    __syncthreads();
    for (int L = 1; L < nlev; ++L) {
        const int lb = lv[L], le2 = lv[L + 1];
        for (int j = lb + tid; j < le2; j += kIvThreads) {
            const int i = ppos[j];
            const int f = fc[i];
            const int before = j > f ? ps[j - 1] - (f > lb ? ps[f - 1] : 0) : 0;
            pre[j] = pre[i] + 1 + before;
        }
        __syncthreads();
    }
    for (int j = tid; j < n; j += kIvThreads) {
        const int xv = ord[j];
        pk[xv] = make_int4(par[xv], pre[j], sz[j], 0);
    }
}

// ======================================================================================
// Aggregation (Algorithm 2).  For v != u and each edge (a, b) of P(v), a = parB(b):
//   +1 if parent_T(b) = a and v lies in the subtree of b (b = v included),
//   -1 if parent_T(a) = b and v lies in the subtree of a.
// Thread per vertex, looping over a chunk of resident trees; one int64 atomic per vertex
// and chunk, skipped when the chunk's sum is zero.
// ======================================================================================
__global__ __launch_bounds__(256) void aggregate_kernel(AggregateArgs a) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.n || v == a.u) return;
    const int t0 = blockIdx.y * a.trees_per_chunk;
    const int t1 = min(a.ntrees, t0 + a.trees_per_chunk);
    const int u = a.u;
    const int *__restrict__ parB = a.parB;
    int sum = 0;
    for (int t = t0; t < t1; ++t) {
        const int4 *__restrict__ pk = a.pk + (long long)t * a.pk_stride;
        int4 pb = pk[v];
        const int pv = pb.y;
        int b = v;
        while (b != u) {
            const int av = parB[b];
            const int4 pa = pk[av];
            if (pb.x == av) sum += (pb.y <= pv && pv < pb.y + pb.z) ? 1 : 0;
            else if (pa.x == b) sum -= (pa.y <= pv && pv < pa.y + pa.z) ? 1 : 0;
            b = av;
            pb = pa;
        }
    }
    if (sum != 0) atomicAdd((unsigned long long *)&a.counts[v], (unsigned long long)(long long)sum);
}

// ======================================================================================
// Pivot-column solve: L x = e_u - (1/n) 1, x orthogonal to 1 (Section "Overview", step 1),
// with conjugate gradients and the diagonal (Jacobi) preconditioner the paper uses.
// Reductions are deterministic: fixed grid, per-block partials, and the last block to
// finish sums the partials in index order.
// ======================================================================================
template <typename T>
__device__ __forceinline__ T lap_row(int v, const int *__restrict__ rp, const int *__restrict__ col,
                                     const T *__restrict__ p) {
    const int lo = rp[v], hi = rp[v + 1];
    T s = (T)(hi - lo) * p[v];
    for (int e = lo; e < hi; ++e) s -= p[col[e]];
    return s;
}

// last block of the grid sums `nparts` partials of width `w` into out[0..w)
__device__ __forceinline__ bool last_block(unsigned int *counter) {
    __shared__ bool am_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int prev = atomicAdd(counter, 1u);
        am_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (am_last) {
        __threadfence();
        if (threadIdx.x == 0) *counter = 0u;
    }
    return am_last;
}

__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int nparts, int stride,
                                               double *sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) v += __hip_atomic_load(part + (long long)i * stride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return block_sum(v, sh);
}

// q = L p and alpha = rz / (p . q)
template <typename T>
__global__ __launch_bounds__(256) void cg_spmv_kernel(CgArgs<T> a) {
    __shared__ double sh[4];
    if (a.sc->done) return;  // uniform: written by an earlier kernel
    double acc = 0.0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        const T qv = lap_row<T>(v, a.rp, a.col, a.p);
        a.q[v] = qv;
        acc += (double)a.p[v] * (double)qv;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) __hip_atomic_store(a.part + blockIdx.x * 2, acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (last_block(a.counter)) {
        const double pq = sum_partials(a.part, gridDim.x, 2, sh);
        if (threadIdx.x == 0) {
            CgScalars *S = a.sc;
            S->pq = pq;
            if (pq > 0.0 && pq == pq) {
                S->alpha = S->rz / pq;
            } else {  // breakdown (p = 0 or non-finite): stop with the current x
                S->alpha = 0.0;
                S->done = 1;
            }
        }
    }
}

// x += alpha p; r -= alpha q; z = r / deg; beta = (r . z) / rz_old; rr = r . r
template <typename T>
__global__ __launch_bounds__(256) void cg_update_kernel(CgArgs<T> a) {
    __shared__ double sh[4];
    if (a.sc->done) return;
    const double alpha = a.sc->alpha;
    const T al = (T)alpha;
    double rz = 0.0, rr = 0.0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        a.x[v] += al * a.p[v];
        const T rv = a.r[v] - al * a.q[v];
        a.r[v] = rv;
        const T zv = rv / (T)(a.rp[v + 1] - a.rp[v]);
        a.z[v] = zv;
        rz += (double)rv * (double)zv;
        rr += (double)rv * (double)rv;
    }
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        __hip_atomic_store(a.part + blockIdx.x * 2, rz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.part + blockIdx.x * 2 + 1, rr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (last_block(a.counter)) {
        const double rzn = sum_partials(a.part, gridDim.x, 2, sh);
        const double rrn = sum_partials(a.part + 1, gridDim.x, 2, sh);
        if (threadIdx.x == 0) {
            CgScalars *S = a.sc;
            S->beta = (S->rz != 0.0) ? rzn / S->rz : 0.0;
            S->rz = rzn;
            S->rr = rrn;
            a.rr_hist[S->iter & (kRrHist - 1)] = rrn;
            S->iter += 1;
            if (!(rrn > S->tol2 * S->rr0)) S->done = 1;  // converged (or NaN)
        }
    }
}

// p = z + beta p
template <typename T>
__global__ __launch_bounds__(256) void cg_pdir_kernel(CgArgs<T> a) {
    if (a.sc->done) return;
    const T be = (T)a.sc->beta;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x)
        a.p[v] = a.z[v] + be * a.p[v];
}

// start of a CG solve of L d = rhs: d = 0, r = rhs (optionally scaled and shifted to mean
// zero), z = r/deg, p = z, rz = r . z
template <typename Tin, typename T>
__global__ __launch_bounds__(256) void cg_start_kernel(CgArgs<T> a, const Tin *__restrict__ rhs, int rhs_is_pivot,
                                                      int u, const double *__restrict__ shift_scale, double tol2) {
    __shared__ double sh[4];
    double rz = 0.0, rr = 0.0;
    const double shift = shift_scale ? shift_scale[0] : 0.0;
    const double scale = shift_scale ? shift_scale[1] : 1.0;
    const double inv_n = 1.0 / (double)a.n;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        double b;
        if (rhs_is_pivot) b = (v == u ? 1.0 : 0.0) - inv_n;
        else b = ((double)rhs[v] - shift) * scale;
        const T rv = (T)b;
        const T zv = rv / (T)(a.rp[v + 1] - a.rp[v]);
        a.x[v] = (T)0;
        a.r[v] = rv;
        a.z[v] = zv;
        a.p[v] = zv;
        rz += (double)rv * (double)zv;
        rr += (double)rv * (double)rv;
    }
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        __hip_atomic_store(a.part + blockIdx.x * 2, rz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.part + blockIdx.x * 2 + 1, rr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (last_block(a.counter)) {
        const double rzn = sum_partials(a.part, gridDim.x, 2, sh);
        const double rrn = sum_partials(a.part + 1, gridDim.x, 2, sh);
        if (threadIdx.x == 0) {
            CgScalars *S = a.sc;
            S->rz = rzn;
            S->rr = rrn;
            S->rr0 = rrn;
            S->beta = 0.0;
            S->alpha = 0.0;
            S->iter = 0;
            S->tol2 = tol2;
            S->done = (rrn > 0.0) ? 0 : 1;
            a.rr_hist[kRrHist - 1] = rrn;
        }
    }
}

// FP64 residual of the current x64: res = b - L x, sums (res, res.res, x) for the outer
// loop of the mixed solve and for the final relative residual.  out: [sum res, |res|^2, sum x]
__global__ __launch_bounds__(256) void residual64_kernel(int n, const int *__restrict__ rp, const int *__restrict__ col,
                                                         int u, const double *__restrict__ x, double *__restrict__ res,
                                                         double *__restrict__ part, unsigned int *counter,
                                                         double *__restrict__ out) {
    __shared__ double sh[4];
    const double inv_n = 1.0 / (double)n;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const double b = (v == u ? 1.0 : 0.0) - inv_n;
        const double rv = b - lap_row<double>(v, rp, col, x);
        if (res) res[v] = rv;
        s0 += rv;
        s1 += rv * rv;
        s2 += x[v];
    }
    s0 = block_sum(s0, sh);
    s1 = block_sum(s1, sh);
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) {
        __hip_atomic_store(part + blockIdx.x * 3, s0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(part + blockIdx.x * 3 + 1, s1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(part + blockIdx.x * 3 + 2, s2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (last_block(counter)) {
        const double a0 = sum_partials(part, gridDim.x, 3, sh);
        const double a1 = sum_partials(part + 1, gridDim.x, 3, sh);
        const double a2 = sum_partials(part + 2, gridDim.x, 3, sh);
        if (threadIdx.x == 0) {
            out[0] = a0;
            out[1] = a1;
            out[2] = a2;
        }
    }
}

// x64 += scale * d (FP32 or FP64 correction) and optionally subtract mean_src[0] / n
template <typename T>
__global__ __launch_bounds__(256) void axpy_project_kernel(int n, double *__restrict__ x, const T *__restrict__ d,
                                                           const double *__restrict__ scale_src, int scale_idx,
                                                           const double *__restrict__ mean_src) {
    const double sc = scale_src ? scale_src[scale_idx] : 1.0;
    const double mean = mean_src ? mean_src[0] / (double)n : 0.0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        double xv = x[v];
        if (d) xv += sc * (double)d[v];
        x[v] = xv - mean;
    }
}

// [shift, scale] for the next inner solve: shift = mean(res), scale = 1 / ||res - shift||
__global__ void outer_scalars_kernel(int n, const double *__restrict__ sums, double *__restrict__ ss) {
    const double mean = sums[0] / (double)n;
    const double nrm2 = sums[1] - (double)n * mean * mean;
    const double nrm = nrm2 > 0.0 ? sqrt(nrm2) : 0.0;
    ss[0] = mean;
    ss[1] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    ss[2] = nrm;
}

// Final fill (Algorithm 1; Eq. diag-comp): diag[u] = x[u], diag[v] = R[v]/tau - x[u] + 2 x[v]
__global__ void combine_kernel(int n, int u, long long tau, const long long *__restrict__ counts,
                               const double *__restrict__ x, double *__restrict__ diag) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const double xu = x[u];
    diag[v] = (v == u) ? xu : (double)counts[v] / (double)tau - xu + 2.0 * x[v];
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
hipError_t launch_bfs_init(int n, int u, int *dist, int *parB, hipStream_t st) {
    bfs_init_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, u, dist, parB);
    return hipGetLastError();
}
hipError_t launch_bfs_level(int n, const int *rp, const int *col, int d, int *dist, int *parB, int *found,
                            hipStream_t st) {
    bfs_level_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, rp, col, d, dist, parB, found);
    return hipGetLastError();
}
hipError_t launch_count_unreached(int n, const int *dist, int *err, hipStream_t st) {
    count_unreached_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, dist, err);
    return hipGetLastError();
}
hipError_t launch_wilson(const WilsonArgs &a, int ntrees, bool lds_bits, hipStream_t st) {
    if (lds_bits) {
        wilson_kernel<true><<<ntrees, 64, (size_t)a.nwords * 4, st>>>(a);
    } else {
        wilson_kernel<false><<<ntrees, 64, 0, st>>>(a);
    }
    return hipGetLastError();
}
hipError_t launch_intervals(const IntervalArgs &a, int ntrees, hipStream_t st) {
    intervals_kernel<<<ntrees, kIvThreads, 0, st>>>(a);
    return hipGetLastError();
}
hipError_t launch_aggregate(const AggregateArgs &a, hipStream_t st) {
    dim3 grid(blocks_for(a.n, 256), (a.ntrees + a.trees_per_chunk - 1) / a.trees_per_chunk);
    aggregate_kernel<<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_cg_iteration(const CgArgs<T> &a, int grid, hipStream_t st) {
    cg_spmv_kernel<T><<<grid, 256, 0, st>>>(a);
    cg_update_kernel<T><<<grid, 256, 0, st>>>(a);
    cg_pdir_kernel<T><<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}
template hipError_t launch_cg_iteration<double>(const CgArgs<double> &, int, hipStream_t);
template hipError_t launch_cg_iteration<float>(const CgArgs<float> &, int, hipStream_t);

template <typename Tin, typename T>
hipError_t launch_cg_start(const CgArgs<T> &a, int grid, const Tin *rhs, int rhs_is_pivot, int u,
                           const double *shift_scale, double tol2, hipStream_t st) {
    cg_start_kernel<Tin, T><<<grid, 256, 0, st>>>(a, rhs, rhs_is_pivot, u, shift_scale, tol2);
    return hipGetLastError();
}
template hipError_t launch_cg_start<double, double>(const CgArgs<double> &, int, const double *, int, int,
                                                    const double *, double, hipStream_t);
template hipError_t launch_cg_start<double, float>(const CgArgs<float> &, int, const double *, int, int,
                                                   const double *, double, hipStream_t);

hipError_t launch_residual64(int n, const int *rp, const int *col, int u, const double *x, double *res,
                             double *part, unsigned int *counter, double *out, int grid, hipStream_t st) {
    residual64_kernel<<<grid, 256, 0, st>>>(n, rp, col, u, x, res, part, counter, out);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_axpy_project(int n, double *x, const T *d, const double *scale_src, int scale_idx,
                               const double *mean_src, int grid, hipStream_t st) {
    axpy_project_kernel<T><<<grid, 256, 0, st>>>(n, x, d, scale_src, scale_idx, mean_src);
    return hipGetLastError();
}
template hipError_t launch_axpy_project<double>(int, double *, const double *, const double *, int, const double *,
                                                int, hipStream_t);
template hipError_t launch_axpy_project<float>(int, double *, const float *, const double *, int, const double *,
                                               int, hipStream_t);
hipError_t launch_outer_scalars(int n, const double *sums, double *ss, hipStream_t st) {
    outer_scalars_kernel<<<1, 1, 0, st>>>(n, sums, ss);
    return hipGetLastError();
}
hipError_t launch_combine(int n, int u, long long tau, const long long *counts, const double *x, double *diag,
                          hipStream_t st) {
    combine_kernel<<<blocks_for(n, 256), 256, 0, st>>>(n, u, tau, counts, x, diag);
    return hipGetLastError();
}
hipError_t launch_philox_words(uint32_t key0, uint32_t key1, long long t, int s, long long k0, long long count,
                               uint32_t *out, hipStream_t st) {
    philox_words_kernel<<<blocks_for(count, 256), 256, 0, st>>>(key0, key1, t, s, k0, count, out);
    return hipGetLastError();
}

}  // namespace ustd
