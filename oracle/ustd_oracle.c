/*
 * ustd_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, FP64 CPU implementation of the uniform-spanning-tree (UST)
 * estimator for diag(L^+) of Angriman, Predari, van der Grinten and Meyerhenke,
 * "Approximation of the Diagonal of a Laplacian's Pseudoinverse for Complex Network
 * Analysis" (ESA 2020).  It exists to check the GPU library against; it is slow on
 * purpose and takes every step in the paper's order.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code, header
 * or table with the GPU library.
 *
 * Every free choice the paper leaves open is pinned the same way the GPU library pins
 * it (ascending start order for Wilson, minimum-ID BFS predecessor, a Philox4x32-10
 * counter per (seed, tree, walk start, step)); with those pins the sampled trees and
 * the integer flow counts are unique, so a correct GPU path must reproduce them bit for
 * bit.
 *
 * Parity pins (all in the CPU test suite): Philox known-answer vectors and an
 * independent numpy Philox; exhaustive spanning-tree enumeration on tiny graphs
 * (Kirchhoff's theorem: mean tree flow = effective resistance, matrix-tree counts,
 * chi-square uniformity); dense pseudoinverse columns and diagonals; closed forms for
 * complete graphs, cycles and trees.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_EGRAPH 2
#define ORC_ENOMEM 3
#define ORC_ENOTCONV 5

/* ------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy as
 * 1, 2, 3", SC 2011).  One round multiplies the even counter words by two fixed odd
 * constants, keeps both halves of each 64-bit product, and mixes the high halves with
 * the odd words and the key; the key is bumped by the Weyl constants between rounds.
 * The paper itself uses PCG32 (Appendix "UST Generation, Pivot Selection, and the
 * Linear System"); a counter-based generator is used here so that every random walk
 * step has its own address.
 * ---------------------------------------------------------------------------------- */
void ustd_oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The 32-bit random word that drives step k of the walk that tree t starts at
 * vertex s: word (k mod 4) of Philox4x32-10 with key (seed lo, seed hi) and counter
 * (k / 4, s, t lo, t hi). */
uint32_t ustd_oracle_walk_word(uint64_t seed, int64_t t, int32_t s, int64_t k)
{
    uint32_t ctr[4] = {(uint32_t)((uint64_t)k >> 2), (uint32_t)s,
                       (uint32_t)((uint64_t)t & 0xffffffffu), (uint32_t)((uint64_t)t >> 32)};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    ustd_oracle_philox4x32_10(ctr, key, out);
    return out[k & 3];
}

/* ------------------------------------------------------------------------------------
 * Input graph (Section "Problem Description and Notation"): simple, finite, connected,
 * undirected.  CSR with ascending rows; every edge stored in both directions.
 * ---------------------------------------------------------------------------------- */
static int row_has(const int64_t *rp, const int32_t *col, int32_t v, int32_t w)
{
    int64_t lo = rp[v], hi = rp[v + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] == w) return 1;
        if (col[mid] < w) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* Plain BFS distances from src (-1 = unreached).  Returns the number reached. */
static int64_t bfs_dist(int64_t n, const int64_t *rp, const int32_t *col, int32_t src,
                        int32_t *dist, int32_t *queue)
{
    for (int64_t i = 0; i < n; ++i) dist[i] = -1;
    int64_t head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int32_t v = queue[head++];
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            int32_t w = col[e];
            if (dist[w] < 0) {
                dist[w] = dist[v] + 1;
                queue[tail++] = w;
            }
        }
    }
    return tail;
}

int ustd_oracle_validate(int64_t n, const int64_t *rp, const int32_t *col)
{
    if (n < 2 || rp == NULL || col == NULL) return ORC_EINVAL;
    if (rp[0] != 0) return ORC_EGRAPH;
    for (int64_t v = 0; v < n; ++v)
        if (rp[v + 1] < rp[v]) return ORC_EGRAPH;
    if (rp[n] % 2 != 0) return ORC_EGRAPH;
    for (int64_t v = 0; v < n; ++v) {
        if (rp[v + 1] == rp[v]) return ORC_EGRAPH; /* isolated vertex: not connected */
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            int32_t w = col[e];
            if (w < 0 || w >= n) return ORC_EGRAPH;
            if (w == v) return ORC_EGRAPH;                           /* self-loop */
            if (e > rp[v] && col[e - 1] >= w) return ORC_EGRAPH;    /* unsorted/dup */
            if (!row_has(rp, col, w, (int32_t)v)) return ORC_EGRAPH; /* asymmetric */
        }
    }
    int32_t *dist = malloc(sizeof(int32_t) * n), *q = malloc(sizeof(int32_t) * n);
    if (!dist || !q) { free(dist); free(q); return ORC_ENOMEM; }
    int64_t reached = bfs_dist(n, rp, col, 0, dist, q);
    free(dist); free(q);
    return reached == n ? ORC_OK : ORC_EGRAPH;
}

/* ------------------------------------------------------------------------------------
 * BFS tree B_u (Section "Effective Resistance Approximation by UST Sampling"): one
 * shortest path P(v) per vertex, stored as parent pointers.  The paper does not say
 * which shortest-path parent to keep; the pinned choice is the smallest-ID neighbour
 * one level closer to u.  Returns ecc(u); parB[u] = -1.
 * ---------------------------------------------------------------------------------- */
int32_t ustd_oracle_bfs(int64_t n, const int64_t *rp, const int32_t *col, int32_t u,
                        int32_t *dist, int32_t *parB)
{
    int32_t *q = malloc(sizeof(int32_t) * n);
    if (!q) return -1;
    bfs_dist(n, rp, col, u, dist, q);
    free(q);
    int32_t ecc = 0;
    for (int64_t v = 0; v < n; ++v) {
        parB[v] = -1;
        if (dist[v] > ecc) ecc = dist[v];
        if (v == u || dist[v] < 0) continue;
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {      /* rows ascend: first hit = min ID */
            if (dist[col[e]] == dist[v] - 1) { parB[v] = col[e]; break; }
        }
    }
    return ecc;
}

/* ------------------------------------------------------------------------------------
 * Pivot by degree.  The paper picks a pivot of low eccentricity (engineering appendix,
 * "Pivot Selection"); the degree rule taken for graphs whose workload names no pivot is the
 * vertex of largest degree, and among several of equal degree the one with the smallest ID.
 * ---------------------------------------------------------------------------------- */
int32_t ustd_oracle_max_degree_pivot(int64_t n, const int64_t *rp)
{
    int32_t best = 0;
    for (int64_t v = 1; v < n; ++v)
        if (rp[v + 1] - rp[v] > rp[best + 1] - rp[best]) best = (int32_t)v;
    return best;
}

/* ------------------------------------------------------------------------------------
 * Sample size (Algorithm 1, initialisation; Appendix proof of the main theorem):
 * tau = ecc(u)^2 * ceil( log(2m/delta) / (2 (1-kappa)^2 eps^2) ), natural log.
 * Solver accuracy eta = kappa eps / (3 sqrt(m n log n) diam(G)), diam(G) <= 2 ecc(u).
 * ---------------------------------------------------------------------------------- */
int64_t ustd_oracle_tau(int64_t n, int64_t m, int32_t ecc, double eps, double delta, double kappa)
{
    if (delta <= 0.0) delta = 1.0 / (double)n;
    if (kappa <= 0.0) kappa = 0.3;
    double one_minus = 1.0 - kappa;
    double q = log(2.0 * (double)m / delta) / (2.0 * one_minus * one_minus * eps * eps);
    return (int64_t)ecc * (int64_t)ecc * (int64_t)ceil(q);
}

double ustd_oracle_eta(int64_t n, int64_t m, int32_t ecc, double eps, double kappa)
{
    if (kappa <= 0.0) kappa = 0.3;
    double diam = 2.0 * (double)ecc;
    return kappa * eps / (3.0 * sqrt((double)m * (double)n * log((double)n)) * diam);
}

/* ------------------------------------------------------------------------------------
 * Wilson's algorithm rooted at u (Appendix "Wilson's UST Algorithm"), Next-pointer
 * form.  Start vertices are taken in ascending ID order; from each start not yet in
 * the tree a random walk runs until it reaches the tree, overwriting Next[x] at every
 * visit (so the retrace follows the successor after the last visit: the loop erasure),
 * and the retrace from the start adds the erased path.  Step k of the walk from s
 * moves to neighbour floor(w * deg(x) / 2^32) of x's ascending adjacency, where w is
 * the walk word above.  parent[u] = -1.  Returns the number of walk steps.
 * ---------------------------------------------------------------------------------- */
int64_t ustd_oracle_wilson(int64_t n, const int64_t *rp, const int32_t *col, int32_t u,
                           uint64_t seed, int64_t t, int32_t *parent, int32_t *next,
                           uint8_t *in_tree)
{
    int64_t steps = 0;
    for (int64_t v = 0; v < n; ++v) { in_tree[v] = 0; parent[v] = -1; next[v] = -1; }
    in_tree[u] = 1;
    parent[u] = -1;
    for (int32_t s = 0; s < n; ++s) {
        if (in_tree[s]) continue;
        int32_t x = s;
        int64_t k = 0;
        while (!in_tree[x]) {
            uint32_t w = ustd_oracle_walk_word(seed, t, s, k);
            uint64_t deg = (uint64_t)(rp[x + 1] - rp[x]);
            uint64_t j = ((uint64_t)w * deg) >> 32;
            next[x] = col[rp[x] + (int64_t)j];
            x = next[x];
            ++k;
        }
        steps += k;
        x = s;
        while (!in_tree[x]) {
            in_tree[x] = 1;
            parent[x] = next[x];
            x = next[x];
        }
    }
    return steps;
}

/* ------------------------------------------------------------------------------------
 * Aggregation of one tree (Algorithm 2).  DFS discovery/finish times alpha/Omega of T
 * rooted at u, then for every v != u and every edge (a, b) of P(v), a = parB(b):
 *   +1 if T has parent(b) = a and v lies in the subtree of b (b = v included),
 *   -1 if T has parent(a) = b and v lies in the subtree of a.
 * The printed test for the +1 case is strict, which would never count the last edge
 * of P(v); the subtree test is read as inclusive (v below or equal to b), the only
 * reading under which a tree graph gives c_T(v) = dist(u, v) = r(u, v).
 * counts[v] += c_T(v).
 * ---------------------------------------------------------------------------------- */
int ustd_oracle_tree_flow(int64_t n, int32_t u, const int32_t *parB, const int32_t *parent,
                          int64_t *counts)
{
    int32_t *first_child = malloc(sizeof(int32_t) * n);
    int32_t *sibling = malloc(sizeof(int32_t) * n);
    int64_t *alpha = malloc(sizeof(int64_t) * n);
    int64_t *omega = malloc(sizeof(int64_t) * n);
    int32_t *stack = malloc(sizeof(int32_t) * n);
    int32_t *cursor = malloc(sizeof(int32_t) * n);
    if (!first_child || !sibling || !alpha || !omega || !stack || !cursor) {
        free(first_child); free(sibling); free(alpha); free(omega); free(stack); free(cursor);
        return ORC_ENOMEM;
    }
    /* child/sibling representation of T (Section "Data structures") */
    for (int64_t v = 0; v < n; ++v) { first_child[v] = -1; sibling[v] = -1; }
    for (int64_t v = n - 1; v >= 0; --v) {
        if (v == u) continue;
        int32_t p = parent[v];
        sibling[v] = first_child[p];
        first_child[p] = (int32_t)v;
    }
    /* iterative DFS from u: one clock for discovery and finish events */
    int64_t clock = 0, top = 0;
    stack[top++] = u;
    alpha[u] = clock++;
    cursor[u] = first_child[u];
    while (top > 0) {
        int32_t v = stack[top - 1];
        int32_t c = cursor[v];
        if (c >= 0) {
            cursor[v] = sibling[c];
            alpha[c] = clock++;
            cursor[c] = first_child[c];
            stack[top++] = c;
        } else {
            omega[v] = clock++;
            --top;
        }
    }
    for (int64_t v = 0; v < n; ++v) {
        if (v == u) continue;
        int64_t c = 0;
        int32_t b = (int32_t)v;
        while (b != u) {
            int32_t a = parB[b];
            if (parent[b] == a) {
                if (alpha[b] <= alpha[v] && omega[v] <= omega[b]) c += 1;
            } else if (parent[a] == b) {
                if (alpha[a] < alpha[v] && omega[v] < omega[a]) c -= 1;
            }
            b = a;
        }
        counts[v] += c;
    }
    free(first_child); free(sibling); free(alpha); free(omega); free(stack); free(cursor);
    return ORC_OK;
}

/* Trees tree_begin .. tree_begin+tree_count-1: parents (tree_count x n, nullable),
 * walk steps per tree (nullable), and flow counts accumulated into counts (nullable). */
int ustd_oracle_trees(int64_t n, const int64_t *rp, const int32_t *col, int32_t u,
                      const int32_t *parB, uint64_t seed, int64_t tree_begin, int64_t tree_count,
                      int32_t *parents, int64_t *steps, int64_t *counts)
{
    int32_t *parent = malloc(sizeof(int32_t) * n);
    int32_t *next = malloc(sizeof(int32_t) * n);
    uint8_t *in_tree = malloc(n);
    if (!parent || !next || !in_tree) { free(parent); free(next); free(in_tree); return ORC_ENOMEM; }
    int rc = ORC_OK;
    for (int64_t i = 0; i < tree_count && rc == ORC_OK; ++i) {
        int64_t s = ustd_oracle_wilson(n, rp, col, u, seed, tree_begin + i, parent, next, in_tree);
        if (steps) steps[i] = s;
        if (parents) memcpy(parents + i * n, parent, sizeof(int32_t) * n);
        if (counts) rc = ustd_oracle_tree_flow(n, u, parB, parent, counts);
    }
    free(parent); free(next); free(in_tree);
    return rc;
}

/* ------------------------------------------------------------------------------------
 * Wilson's algorithm per biconnected component (engineering appendix, after Hayashi et al.):
 * compute the biconnected components (blocks) of G, run Wilson's algorithm in each block
 * with a vertex of maximal degree as its root, and join the block trees into a spanning tree
 * of G.  Every spanning tree of G is one spanning tree per block and vice versa, so drawing
 * each block's tree uniformly and independently draws a uniform spanning tree of G.
 *
 * Readings (the appendix gives the idea only):
 *  - a block's root is the vertex of largest degree inside the block (the graph the block's
 *    walks run on), the smallest ID among equal degrees;
 *  - inside a block, starts are taken in ascending vertex order and the walk at x moves to
 *    neighbour floor(w * deg_B(x) / 2^32) of x's ascending adjacency inside the block;
 *  - a cut vertex starts one walk in each block it is not the root of, so walks are keyed by
 *    the CSR position e(v, B) of v's first edge inside B (unique per vertex and block) in
 *    place of the vertex: step k of that walk takes word (k mod 4) of Philox4x32-10 with
 *    counter (k / 4, e(v, B), tree lo, tree hi), so the blocks' draws are independent;
 *  - joined rooted at u: each block's tree is re-rooted at the block's vertex closest to u
 *    (u itself, or the cut vertex through which every path from the block to u passes), and
 *    every vertex v != u takes its parent from the one block in which it is not that vertex.
 * ---------------------------------------------------------------------------------- */

/* position of w in the ascending row of v, or -1 */
static int64_t row_find(const int64_t *rp, const int32_t *col, int32_t v, int32_t w)
{
    int64_t lo = rp[v], hi = rp[v + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] == w) return mid;
        if (col[mid] < w) lo = mid + 1; else hi = mid;
    }
    return -1;
}

/* Blocks of the edges by Tarjan's depth-first search with an edge stack (iterative).  Two
 * edges share a block iff some simple cycle contains both; an edge on no cycle (a bridge) is a
 * block of its own.  eblock[e] (per CSR entry, the same at both entries of an edge) gets ids
 * 0 .. nb-1 in the order the blocks are completed.  Returns nb (-1 if out of memory). */
int64_t ustd_oracle_blocks(int64_t n, const int64_t *rp, const int32_t *col, int32_t *eblock)
{
    int64_t nnz = rp[n];
    int64_t *disc = malloc(sizeof(int64_t) * n), *low = malloc(sizeof(int64_t) * n);
    int64_t *cur = malloc(sizeof(int64_t) * n), *pe = malloc(sizeof(int64_t) * n);
    int32_t *vst = malloc(sizeof(int32_t) * n);
    int64_t *est = malloc(sizeof(int64_t) * (nnz / 2 + 1));
    if (!disc || !low || !cur || !pe || !vst || !est) {
        free(disc); free(low); free(cur); free(pe); free(vst); free(est);
        return -1;
    }
    for (int64_t v = 0; v < n; ++v) disc[v] = -1;
    for (int64_t e = 0; e < nnz; ++e) eblock[e] = -1;
    int64_t clock = 0, nb = 0, vtop = 0, etop = 0;
    for (int32_t r = 0; r < n; ++r) {
        if (disc[r] >= 0) continue;
        disc[r] = low[r] = clock++;
        cur[r] = rp[r];
        pe[r] = -1;
        vst[vtop++] = r;
        while (vtop > 0) {
            int32_t v = vst[vtop - 1];
            if (cur[v] < rp[v + 1]) {
                int64_t e = cur[v]++;
                int32_t w = col[e];
                if (disc[w] < 0) {               /* tree edge */
                    disc[w] = low[w] = clock++;
                    cur[w] = rp[w];
                    pe[w] = e;
                    est[etop++] = e;
                    vst[vtop++] = w;
                } else if (disc[w] < disc[v] && (vtop < 2 || w != vst[vtop - 2])) {
                    /* an edge back to an ancestor other than the tree parent (the vertex below v
                     * on the stack; the graph is simple) */
                    est[etop++] = e;
                    if (disc[w] < low[v]) low[v] = disc[w];
                }
            } else {
                --vtop;
                if (vtop == 0) break;
                int32_t p = vst[vtop - 1];
                if (low[v] < low[p]) low[p] = low[v];
                if (low[v] >= disc[p]) {         /* p separates v's subtree: one block */
                    int64_t f;
                    do {
                        f = est[--etop];
                        int64_t lo2 = 0, hi2 = n;  /* the row a of entry f */
                        while (hi2 - lo2 > 1) {
                            int64_t mid = (lo2 + hi2) / 2;
                            if (rp[mid] <= f) lo2 = mid; else hi2 = mid;
                        }
                        int32_t a = (int32_t)lo2;
                        eblock[f] = (int32_t)nb;
                        eblock[row_find(rp, col, col[f], a)] = (int32_t)nb;
                    } while (f != pe[v]);
                    ++nb;
                }
            }
        }
    }
    free(disc); free(low); free(cur); free(pe); free(vst); free(est);
    return nb;
}

/* One spanning tree by Wilson's algorithm per block (readings above).  eblock and nb from
 * ustd_oracle_blocks, dist from the BFS of u.  parent[u] = -1.  Returns the walk steps (the
 * sum over the blocks), -1 if out of memory. */
int64_t ustd_oracle_wilson_blocks(int64_t n, const int64_t *rp, const int32_t *col, int32_t u,
                                  const int32_t *eblock, int64_t nb, const int32_t *dist, uint64_t seed,
                                  int64_t t, int32_t *parent)
{
    int64_t nnz = rp[n];
    /* entries grouped by block, each block's in CSR order (so by row, then neighbour) */
    int64_t *bstart = calloc((size_t)(nb + 1), sizeof(int64_t));
    int64_t *ent = malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (nb > 0 ? nb : 1));
    int32_t *loc = malloc(sizeof(int32_t) * n);          /* vertex -> index inside the block */
    int32_t *vx = malloc(sizeof(int32_t) * n);           /* block vertices, ascending */
    int64_t *ad0 = malloc(sizeof(int64_t) * n);          /* first of the vertex's entries in ent */
    int32_t *dg = malloc(sizeof(int32_t) * n);           /* its degree inside the block */
    int32_t *nxt = malloc(sizeof(int32_t) * n), *bpar = malloc(sizeof(int32_t) * n);
    uint8_t *in = malloc(n);
    if (!bstart || !ent || !fill || !loc || !vx || !ad0 || !dg || !nxt || !bpar || !in) {
        free(bstart); free(ent); free(fill); free(loc); free(vx); free(ad0); free(dg); free(nxt); free(bpar);
        free(in);
        return -1;
    }
    for (int64_t e = 0; e < nnz; ++e) bstart[eblock[e] + 1]++;
    for (int64_t b = 0; b < nb; ++b) bstart[b + 1] += bstart[b];
    for (int64_t b = 0; b < nb; ++b) fill[b] = bstart[b];
    for (int64_t e = 0; e < nnz; ++e) ent[fill[eblock[e]]++] = e;
    for (int64_t v = 0; v < n; ++v) { loc[v] = -1; parent[v] = -1; }
    int64_t steps = 0;
    for (int64_t b = 0; b < nb; ++b) {
        /* the block's vertices (ascending), their first entries and degrees inside it */
        int32_t nv = 0;
        for (int64_t i = bstart[b]; i < bstart[b + 1]; ++i) {
            int64_t e = ent[i];
            int64_t lo2 = 0, hi2 = n;               /* the row of entry e */
            while (hi2 - lo2 > 1) {
                int64_t mid = (lo2 + hi2) / 2;
                if (rp[mid] <= e) lo2 = mid; else hi2 = mid;
            }
            int32_t v = (int32_t)lo2;
            if (nv == 0 || vx[nv - 1] != v) {
                vx[nv] = v;
                ad0[nv] = i;
                dg[nv] = 0;
                loc[v] = nv;
                ++nv;
            }
            dg[nv - 1]++;
        }
        /* root: largest degree inside the block, smallest ID among equal ones */
        int32_t root = 0;
        for (int32_t i = 1; i < nv; ++i)
            if (dg[i] > dg[root]) root = i;
        for (int32_t i = 0; i < nv; ++i) { in[i] = 0; bpar[i] = -1; }
        in[root] = 1;
        for (int32_t i = 0; i < nv; ++i) {      /* starts in ascending vertex order */
            if (in[i]) continue;
            int32_t key = (int32_t)ent[ad0[i]];   /* e(v, B): v's first edge inside the block */
            int32_t x = i;
            int64_t k = 0;
            while (!in[x]) {
                uint32_t w = ustd_oracle_walk_word(seed, t, key, k);
                uint64_t j = ((uint64_t)w * (uint64_t)dg[x]) >> 32;
                nxt[x] = loc[col[ent[ad0[x] + (int64_t)j]]];
                x = nxt[x];
                ++k;
            }
            steps += k;
            for (x = i; !in[x]; x = nxt[x]) {
                in[x] = 1;
                bpar[x] = nxt[x];
            }
        }
        /* re-root at the block's vertex closest to u, then each vertex but that one takes its
         * parent from this block */
        int32_t c = 0;
        for (int32_t i = 1; i < nv; ++i)
            if (dist[vx[i]] < dist[vx[c]]) c = i;
        int32_t prev = -1, x = c;
        while (x >= 0) {
            int32_t up = bpar[x];
            bpar[x] = prev;
            prev = x;
            x = up;
        }
        for (int32_t i = 0; i < nv; ++i) {
            if (i != c) parent[vx[i]] = vx[bpar[i]];
            loc[vx[i]] = -1;
        }
    }
    parent[u] = -1;
    free(bstart); free(ent); free(fill); free(loc); free(vx); free(ad0); free(dg); free(nxt); free(bpar); free(in);
    return steps;
}

/* Trees tree_begin .. +tree_count-1 of the per-block variant: parents (tree_count x n,
 * nullable), steps (nullable), flow counts accumulated into counts (nullable; Algorithm 2 on
 * the joined tree). */
int ustd_oracle_trees_blocks(int64_t n, const int64_t *rp, const int32_t *col, int32_t u, const int32_t *parB,
                             uint64_t seed, int64_t tree_begin, int64_t tree_count, int32_t *parents,
                             int64_t *steps, int64_t *counts)
{
    int32_t *eblock = malloc(sizeof(int32_t) * (rp[n] > 0 ? rp[n] : 1));
    int32_t *dist = malloc(sizeof(int32_t) * n), *pb = malloc(sizeof(int32_t) * n);
    int32_t *parent = malloc(sizeof(int32_t) * n);
    if (!eblock || !dist || !pb || !parent) { free(eblock); free(dist); free(pb); free(parent); return ORC_ENOMEM; }
    int64_t nb = ustd_oracle_blocks(n, rp, col, eblock);
    ustd_oracle_bfs(n, rp, col, u, dist, pb);
    int rc = nb < 0 ? ORC_ENOMEM : ORC_OK;
    for (int64_t i = 0; i < tree_count && rc == ORC_OK; ++i) {
        int64_t s = ustd_oracle_wilson_blocks(n, rp, col, u, eblock, nb, dist, seed, tree_begin + i, parent);
        if (s < 0) { rc = ORC_ENOMEM; break; }
        if (steps) steps[i] = s;
        if (parents) memcpy(parents + i * n, parent, sizeof(int32_t) * n);
        if (counts) rc = ustd_oracle_tree_flow(n, u, parB, parent, counts);
    }
    free(eblock); free(dist); free(pb); free(parent);
    return rc;
}

/* ------------------------------------------------------------------------------------
 * Pivot column of L^+ (Section "Overview", step 1; Algorithm 1, linear system):
 * solve L x = e_u - (1/n) 1 with x orthogonal to 1, which is column u of L^+.  The
 * paper uses conjugate gradients with a diagonal preconditioner.  Plain FP64 Jacobi-PCG
 * from x = 0 on the consistent singular system, stopped when the updated residual
 * satisfies ||r||_2 <= tol ||b||_2, followed by projection onto the mean-zero subspace.
 * Returns the iteration count (negative if maxit was reached).
 * ---------------------------------------------------------------------------------- */
static void lap_apply(int64_t n, const int64_t *rp, const int32_t *col, const double *p, double *q)
{
    for (int64_t v = 0; v < n; ++v) {
        double acc = (double)(rp[v + 1] - rp[v]) * p[v];
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) acc -= p[col[e]];
        q[v] = acc;
    }
}

int64_t ustd_oracle_solve(int64_t n, const int64_t *rp, const int32_t *col, int32_t u,
                          double tol, int64_t maxit, double *x, double *relres_out)
{
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    if (!r || !z || !p || !q) { free(r); free(z); free(p); free(q); return -1; }
    double bnorm2 = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        double b = (v == u ? 1.0 : 0.0) - 1.0 / (double)n;
        x[v] = 0.0;
        r[v] = b;
        bnorm2 += b * b;
    }
    double bnorm = sqrt(bnorm2);
    double rz = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        z[v] = r[v] / (double)(rp[v + 1] - rp[v]);
        p[v] = z[v];
        rz += r[v] * z[v];
    }
    int64_t it = 0;
    double rnorm = bnorm;
    int converged = rnorm <= tol * bnorm;
    while (!converged && it < maxit) {
        lap_apply(n, rp, col, p, q);
        double pq = 0.0;
        for (int64_t v = 0; v < n; ++v) pq += p[v] * q[v];
        double alpha = rz / pq;
        double rr = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            x[v] += alpha * p[v];
            r[v] -= alpha * q[v];
            rr += r[v] * r[v];
        }
        ++it;
        rnorm = sqrt(rr);
        if (rnorm <= tol * bnorm) { converged = 1; break; }
        double rz_new = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            z[v] = r[v] / (double)(rp[v + 1] - rp[v]);
            rz_new += r[v] * z[v];
        }
        double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t v = 0; v < n; ++v) p[v] = z[v] + beta * p[v];
    }
    double mean = 0.0;
    for (int64_t v = 0; v < n; ++v) mean += x[v];
    mean /= (double)n;
    for (int64_t v = 0; v < n; ++v) x[v] -= mean;
    /* true residual of the projected solution */
    lap_apply(n, rp, col, x, q);
    double tr = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        double b = (v == u ? 1.0 : 0.0) - 1.0 / (double)n;
        tr += (b - q[v]) * (b - q[v]);
    }
    if (relres_out) *relres_out = sqrt(tr) / bnorm;
    free(r); free(z); free(p); free(q);
    return converged ? it : -it - 1;
}

/* Final fill (Algorithm 1; Eq. diag-comp): L^+_uu = x[u] and, for v != u,
 * L^+_vv = R[v]/tau - x[u] + 2 x[v]. */
void ustd_oracle_combine(int64_t n, int32_t u, int64_t tau, const int64_t *counts,
                         const double *x, double *diag)
{
    for (int64_t v = 0; v < n; ++v) {
        if (v == u) diag[v] = x[u];
        else diag[v] = (double)counts[v] / (double)tau - x[u] + 2.0 * x[v];
    }
}

/* ------------------------------------------------------------------------------------
 * ApproxDiagLpinv (Algorithm 1) end to end.  tau_override > 0 replaces the formula.
 * Outputs diag (n), counts (n, nullable), and tau / ecc / steps through pointers.
 * ---------------------------------------------------------------------------------- */
int ustd_oracle_diag_lpinv(int64_t n, const int64_t *rp, const int32_t *col, int32_t u,
                           double eps, double delta, double kappa, uint64_t seed,
                           int64_t tau_override, double solve_tol, int64_t solve_maxit,
                           double *diag, int64_t *counts_out, int64_t *tau_out,
                           int32_t *ecc_out, int64_t *steps_out, double *relres_out)
{
    if (u < 0 || u >= n || !(eps > 0.0)) return ORC_EINVAL;
    int32_t *dist = malloc(sizeof(int32_t) * n), *parB = malloc(sizeof(int32_t) * n);
    int64_t *counts = calloc((size_t)n, sizeof(int64_t));
    double *x = malloc(sizeof(double) * n);
    if (!dist || !parB || !counts || !x) {
        free(dist); free(parB); free(counts); free(x);
        return ORC_ENOMEM;
    }
    int32_t ecc = ustd_oracle_bfs(n, rp, col, u, dist, parB);
    int64_t m = rp[n] / 2;
    int64_t tau = tau_override > 0 ? tau_override : ustd_oracle_tau(n, m, ecc, eps, delta, kappa);
    int64_t total_steps = 0;
    int32_t *parent = malloc(sizeof(int32_t) * n), *next = malloc(sizeof(int32_t) * n);
    uint8_t *in_tree = malloc(n);
    int rc = (parent && next && in_tree) ? ORC_OK : ORC_ENOMEM;
    for (int64_t t = 0; t < tau && rc == ORC_OK; ++t) {
        total_steps += ustd_oracle_wilson(n, rp, col, u, seed, t, parent, next, in_tree);
        rc = ustd_oracle_tree_flow(n, u, parB, parent, counts);
    }
    free(parent); free(next); free(in_tree);
    if (rc == ORC_OK) {
        double tol = solve_tol;
        if (!(tol > 0.0)) {
            double eta = ustd_oracle_eta(n, m, ecc, eps, kappa);
            tol = eta < 1e-12 ? eta : 1e-12;
        }
        int64_t it = ustd_oracle_solve(n, rp, col, u, tol, solve_maxit > 0 ? solve_maxit : 100000,
                                       x, relres_out);
        ustd_oracle_combine(n, u, tau, counts, x, diag);
        if (it < 0) rc = ORC_ENOTCONV;
    }
    if (counts_out) memcpy(counts_out, counts, sizeof(int64_t) * n);
    if (tau_out) *tau_out = tau;
    if (ecc_out) *ecc_out = ecc;
    if (steps_out) *steps_out = total_steps;
    free(dist); free(parB); free(counts); free(x);
    return rc;
}

/* ====================================================================================
 * Weighted graphs (Section "Generalizations", extension to weighted graphs).
 *
 * w[e] > 0 is the conductance of CSR entry e, the same in both directions of an edge.
 * The paper's text leaves three points open; the readings taken here are:
 *  1. Wilson's walk moves to a neighbour with probability proportional to the
 *     conductance, so trees come out with probability proportional to their weight (the
 *     product of their conductances).  Under that distribution the weighted Kirchhoff
 *     theorem makes the current on an edge the mean signed traversal count, so every tree
 *     contributes +-1 per traversed edge and the sum is divided by tau, the number of
 *     trees.  (Adding each tree's weight as well, as the printed text says, would weight
 *     the trees twice.)
 *  2. The potential difference along P(v) is the current times the edge's resistance
 *     1/w(e) (Ohm's law), a factor the unweighted Eq. N-values-in-path does not show.
 *  3. The sample size replaces ecc(u), the largest range of a tree's contribution in the
 *     unweighted bound, by rho_max = max_v of the resistance of P(v).  For unit weights
 *     rho_max = ecc(u) and every definition below reduces to the unweighted one.
 * To stay exact and order-independent, a tree's contributions are integers: the edge
 * (b, parB(b)) of P(v) contributes +-F[b], F[b] = llround(2^k / w(b, parB(b))), with k
 * the largest shift that keeps every sum below 2^62.
 * ---------------------------------------------------------------------------------- */

/* 0 if every weight is positive and finite and w(v, x) = w(x, v) for every edge. */
int ustd_oracle_validate_weights(int64_t n, const int64_t *rp, const int32_t *col, const double *w)
{
    for (int64_t v = 0; v < n; ++v) {
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            if (!(w[e] > 0.0) || !isfinite(w[e])) return ORC_EGRAPH;
            int32_t x = col[e];
            int64_t lo = rp[x], hi = rp[x + 1], f = -1;
            while (lo < hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (col[mid] == (int32_t)v) { f = mid; break; }
                if (col[mid] < (int32_t)v) lo = mid + 1; else hi = mid;
            }
            if (f < 0 || w[f] != w[e]) return ORC_EGRAPH;
        }
    }
    return ORC_OK;
}

/* Resistance of P(v): the sum of 1/w over its edges, added from v towards u; wB[v] is
 * the conductance of v's own B_u edge (wB[u] = 0).  Returns rho_max. */
double ustd_oracle_bpath_resistance(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
                                    int32_t u, const int32_t *parB, double *wB, double *rho)
{
    for (int64_t v = 0; v < n; ++v) {
        wB[v] = 0.0;
        if (v == u) continue;
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
            if (col[e] == parB[v]) { wB[v] = w[e]; break; }
    }
    double rmax = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        double r = 0.0;
        for (int32_t b = (int32_t)v; b != u; b = parB[b]) r += 1.0 / wB[b];
        rho[v] = r;
        if (r > rmax) rmax = r;
    }
    return rmax;
}

/* tau = ceil(rho_max^2 * ceil(log(2m/delta) / (2 (1-kappa)^2 eps^2))) (reading 3). */
int64_t ustd_oracle_tau_weighted(int64_t n, int64_t m, double rho_max, double eps, double delta, double kappa)
{
    if (delta <= 0.0) delta = 1.0 / (double)n;
    if (kappa <= 0.0) kappa = 0.3;
    double one_minus = 1.0 - kappa;
    double q = ceil(log(2.0 * (double)m / delta) / (2.0 * one_minus * one_minus * eps * eps));
    double r2 = rho_max * rho_max;
    return (int64_t)ceil(r2 * q);
}

/* Fixed-point shift k: tau * rho_max * 2^k <= 2^62, so no sum of tau trees' contributions
 * (each at most 2^k rho(v) plus rounding) leaves int64. */
int32_t ustd_oracle_fixed_shift(int64_t tau, double rho_max)
{
    int e = 0;
    frexp((double)tau * rho_max, &e);
    return (int32_t)(62 - e);
}

/* F[b] = llround(2^k / wB[b]) for b != u; F[u] = 0. */
void ustd_oracle_fixed_weights(int64_t n, int32_t u, const double *wB, int32_t k, int64_t *F)
{
    double S = ldexp(1.0, k);
    for (int64_t v = 0; v < n; ++v) F[v] = v == u ? 0 : llround(S / wB[v]);
}

/* Wilson's algorithm with conductance-weighted steps.  The walk at x with word w32 goes to
 * the first neighbour j (ascending adjacency) whose running conductance sum exceeds
 * t = (w32 * 2^-32) * W_x, W_x the row total; sums are taken left to right in FP64.  With
 * all conductances 1, t = w32 deg / 2^32 exactly and j = floor(t): the unweighted step. */
int64_t ustd_oracle_wilson_weighted(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
                                    int32_t u, uint64_t seed, int64_t t, int32_t *parent, int32_t *next,
                                    uint8_t *in_tree)
{
    int64_t steps = 0;
    for (int64_t v = 0; v < n; ++v) { in_tree[v] = 0; parent[v] = -1; next[v] = -1; }
    in_tree[u] = 1;
    for (int32_t s = 0; s < n; ++s) {
        if (in_tree[s]) continue;
        int32_t x = s;
        int64_t k = 0;
        while (!in_tree[x]) {
            uint32_t word = ustd_oracle_walk_word(seed, t, s, k);
            double total = 0.0;
            for (int64_t e = rp[x]; e < rp[x + 1]; ++e) total += w[e];
            double target = ((double)word * 0x1p-32) * total;
            double run = 0.0;
            int64_t pick = rp[x + 1] - 1;
            for (int64_t e = rp[x]; e < rp[x + 1]; ++e) {
                run += w[e];
                if (target < run) { pick = e; break; }
            }
            next[x] = col[pick];
            x = next[x];
            ++k;
        }
        steps += k;
        x = s;
        while (!in_tree[x]) {
            in_tree[x] = 1;
            parent[x] = next[x];
            x = next[x];
        }
    }
    return steps;
}

/* Algorithm 2 with the edge factor: as ustd_oracle_tree_flow, adding +-F[b] for the edge
 * (parB(b), b) instead of +-1 (reading 2); acc[v] += c_T(v). */
int ustd_oracle_tree_flow_weighted(int64_t n, int32_t u, const int32_t *parB, const int32_t *parent,
                                   const int64_t *F, int64_t *acc)
{
    int32_t *first_child = malloc(sizeof(int32_t) * n);
    int32_t *sibling = malloc(sizeof(int32_t) * n);
    int64_t *alpha = malloc(sizeof(int64_t) * n);
    int64_t *omega = malloc(sizeof(int64_t) * n);
    int32_t *stack = malloc(sizeof(int32_t) * n);
    int32_t *cursor = malloc(sizeof(int32_t) * n);
    if (!first_child || !sibling || !alpha || !omega || !stack || !cursor) {
        free(first_child); free(sibling); free(alpha); free(omega); free(stack); free(cursor);
        return ORC_ENOMEM;
    }
    for (int64_t v = 0; v < n; ++v) { first_child[v] = -1; sibling[v] = -1; }
    for (int64_t v = n - 1; v >= 0; --v) {
        if (v == u) continue;
        int32_t p = parent[v];
        sibling[v] = first_child[p];
        first_child[p] = (int32_t)v;
    }
    int64_t clock = 0, top = 0;
    stack[top++] = u;
    alpha[u] = clock++;
    cursor[u] = first_child[u];
    while (top > 0) {
        int32_t v = stack[top - 1];
        int32_t c = cursor[v];
        if (c >= 0) {
            cursor[v] = sibling[c];
            alpha[c] = clock++;
            cursor[c] = first_child[c];
            stack[top++] = c;
        } else {
            omega[v] = clock++;
            --top;
        }
    }
    for (int64_t v = 0; v < n; ++v) {
        if (v == u) continue;
        int64_t c = 0;
        int32_t b = (int32_t)v;
        while (b != u) {
            int32_t a = parB[b];
            if (parent[b] == a) {
                if (alpha[b] <= alpha[v] && omega[v] <= omega[b]) c += F[b];
            } else if (parent[a] == b) {
                if (alpha[a] < alpha[v] && omega[v] < omega[a]) c -= F[b];
            }
            b = a;
        }
        acc[v] += c;
    }
    free(first_child); free(sibling); free(alpha); free(omega); free(stack); free(cursor);
    return ORC_OK;
}

/* Weighted trees tree_begin .. +tree_count-1: parents (nullable), steps (nullable) and the
 * fixed-point flow sums accumulated into acc (nullable; needs F). */
int ustd_oracle_trees_weighted(int64_t n, const int64_t *rp, const int32_t *col, const double *w, int32_t u,
                               const int32_t *parB, const int64_t *F, uint64_t seed, int64_t tree_begin,
                               int64_t tree_count, int32_t *parents, int64_t *steps, int64_t *acc)
{
    int32_t *parent = malloc(sizeof(int32_t) * n);
    int32_t *next = malloc(sizeof(int32_t) * n);
    uint8_t *in_tree = malloc(n);
    if (!parent || !next || !in_tree) { free(parent); free(next); free(in_tree); return ORC_ENOMEM; }
    int rc = ORC_OK;
    for (int64_t i = 0; i < tree_count && rc == ORC_OK; ++i) {
        int64_t s = ustd_oracle_wilson_weighted(n, rp, col, w, u, seed, tree_begin + i, parent, next, in_tree);
        if (steps) steps[i] = s;
        if (parents) memcpy(parents + i * n, parent, sizeof(int32_t) * n);
        if (acc) rc = ustd_oracle_tree_flow_weighted(n, u, parB, parent, F, acc);
    }
    free(parent); free(next); free(in_tree);
    return rc;
}

/* Weighted Laplacian: (L p)_v = wdeg(v) p_v - sum_e w[e] p[col[e]], wdeg(v) the row's
 * conductance sum (left to right).  Jacobi-PCG as ustd_oracle_solve, preconditioned by
 * wdeg. */
static void lap_apply_weighted(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
                               const double *wdeg, const double *p, double *q)
{
    for (int64_t v = 0; v < n; ++v) {
        double acc = wdeg[v] * p[v];
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) acc -= w[e] * p[col[e]];
        q[v] = acc;
    }
}

int64_t ustd_oracle_solve_weighted(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
                                   int32_t u, double tol, int64_t maxit, double *x, double *relres_out)
{
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    double *wdeg = malloc(sizeof(double) * n);
    if (!r || !z || !p || !q || !wdeg) { free(r); free(z); free(p); free(q); free(wdeg); return -1; }
    for (int64_t v = 0; v < n; ++v) {
        double s = 0.0;
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) s += w[e];
        wdeg[v] = s;
    }
    double bnorm2 = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        double b = (v == u ? 1.0 : 0.0) - 1.0 / (double)n;
        x[v] = 0.0;
        r[v] = b;
        bnorm2 += b * b;
    }
    double bnorm = sqrt(bnorm2);
    double rz = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        z[v] = r[v] / wdeg[v];
        p[v] = z[v];
        rz += r[v] * z[v];
    }
    int64_t it = 0;
    int converged = bnorm <= tol * bnorm;
    while (!converged && it < maxit) {
        lap_apply_weighted(n, rp, col, w, wdeg, p, q);
        double pq = 0.0;
        for (int64_t v = 0; v < n; ++v) pq += p[v] * q[v];
        double alpha = rz / pq;
        double rr = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            x[v] += alpha * p[v];
            r[v] -= alpha * q[v];
            rr += r[v] * r[v];
        }
        ++it;
        if (sqrt(rr) <= tol * bnorm) { converged = 1; break; }
        double rz_new = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            z[v] = r[v] / wdeg[v];
            rz_new += r[v] * z[v];
        }
        double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t v = 0; v < n; ++v) p[v] = z[v] + beta * p[v];
    }
    double mean = 0.0;
    for (int64_t v = 0; v < n; ++v) mean += x[v];
    mean /= (double)n;
    for (int64_t v = 0; v < n; ++v) x[v] -= mean;
    lap_apply_weighted(n, rp, col, w, wdeg, x, q);
    double tr = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        double b = (v == u ? 1.0 : 0.0) - 1.0 / (double)n;
        tr += (b - q[v]) * (b - q[v]);
    }
    if (relres_out) *relres_out = sqrt(tr) / bnorm;
    free(r); free(z); free(p); free(q); free(wdeg);
    return converged ? it : -it - 1;
}

/* Eq. diag-comp with fixed-point sums: L^+_vv = acc[v] / (tau 2^k) - x[u] + 2 x[v]. */
void ustd_oracle_combine_weighted(int64_t n, int32_t u, int64_t tau, int32_t k, const int64_t *acc,
                                  const double *x, double *diag)
{
    double den = ldexp((double)tau, k);
    for (int64_t v = 0; v < n; ++v) {
        if (v == u) diag[v] = x[u];
        else diag[v] = (double)acc[v] / den - x[u] + 2.0 * x[v];
    }
}

/* ApproxDiagLpinv on a weighted graph, end to end (tau_override > 0 replaces the formula).
 * Outputs diag, acc (nullable), tau, the fixed-point shift, rho_max, steps and the relative
 * residual of the solve. */
int ustd_oracle_diag_lpinv_weighted(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
                                    int32_t u, double eps, double delta, double kappa, uint64_t seed,
                                    int64_t tau_override, double solve_tol, int64_t solve_maxit,
                                    double *diag, int64_t *acc_out, int64_t *tau_out, int32_t *shift_out,
                                    double *rho_out, int64_t *steps_out, double *relres_out)
{
    if (u < 0 || u >= n || !(eps > 0.0)) return ORC_EINVAL;
    int32_t *dist = malloc(sizeof(int32_t) * n), *parB = malloc(sizeof(int32_t) * n);
    double *wB = malloc(sizeof(double) * n), *rho = malloc(sizeof(double) * n);
    int64_t *F = malloc(sizeof(int64_t) * n), *acc = calloc((size_t)n, sizeof(int64_t));
    double *x = malloc(sizeof(double) * n);
    if (!dist || !parB || !wB || !rho || !F || !acc || !x) {
        free(dist); free(parB); free(wB); free(rho); free(F); free(acc); free(x);
        return ORC_ENOMEM;
    }
    int32_t ecc = ustd_oracle_bfs(n, rp, col, u, dist, parB);
    int64_t m = rp[n] / 2;
    double rho_max = ustd_oracle_bpath_resistance(n, rp, col, w, u, parB, wB, rho);
    int64_t tau = tau_override > 0 ? tau_override : ustd_oracle_tau_weighted(n, m, rho_max, eps, delta, kappa);
    int32_t k = ustd_oracle_fixed_shift(tau, rho_max);
    ustd_oracle_fixed_weights(n, u, wB, k, F);
    int64_t total_steps = 0;
    int64_t *st = malloc(sizeof(int64_t) * (size_t)tau);
    int rc = st ? ustd_oracle_trees_weighted(n, rp, col, w, u, parB, F, seed, 0, tau, NULL, st, acc) : ORC_ENOMEM;
    if (st) {
        for (int64_t i = 0; i < tau && rc == ORC_OK; ++i) total_steps += st[i];
        free(st);
    }
    if (rc == ORC_OK) {
        double tol = solve_tol;
        if (!(tol > 0.0)) {
            double eta = ustd_oracle_eta(n, m, ecc, eps, kappa);
            tol = eta < 1e-12 ? eta : 1e-12;
        }
        int64_t it = ustd_oracle_solve_weighted(n, rp, col, w, u, tol, solve_maxit > 0 ? solve_maxit : 100000,
                                                x, relres_out);
        ustd_oracle_combine_weighted(n, u, tau, k, acc, x, diag);
        if (it < 0) rc = ORC_ENOTCONV;
    }
    if (acc_out) memcpy(acc_out, acc, sizeof(int64_t) * n);
    if (tau_out) *tau_out = tau;
    if (shift_out) *shift_out = k;
    if (rho_out) *rho_out = rho_max;
    if (steps_out) *steps_out = total_steps;
    free(dist); free(parB); free(wB); free(rho); free(F); free(acc); free(x);
    return rc;
}
