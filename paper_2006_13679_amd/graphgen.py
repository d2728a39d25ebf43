"""Seeded synthetic input graphs (CSR) for the UST estimator of diag(L^+).

This module only builds inputs: it holds none of the estimator's arithmetic, so the GPU
library and the CPU oracle can both be fed from it.  Every graph is returned in the
canonical form the estimator takes (Section "Problem Description and Notation" of the
paper: simple, finite, connected, undirected, unit weights): symmetrised, self-loops
dropped, duplicates removed, restricted to the largest connected component, relabelled
in increasing original ID order, and stored as CSR with ascending rows
(``row_ptr`` int64[n+1], ``col`` int32[2m]).

Families (the paper's synthetic families, Section "Experiments" and its appendix):
  * 2-D grids (row-major IDs),
  * R-MAT with the Graph500 parameters (a, b, c, d) = (0.57, 0.19, 0.19, 0.05),
  * random hyperbolic graphs (threshold model, power-law exponent 3, average degree 20),
  * small closed-form graphs (complete, cycle, path, star, complete bipartite) for tests.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Graph:
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[2m]
    name: str = ""

    @property
    def n(self) -> int:
        return len(self.row_ptr) - 1

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1]) // 2

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.int32).tobytes())
        return h.hexdigest()[:16]


# ----------------------------------------------------------------------------------------
# canonicalisation
# ----------------------------------------------------------------------------------------
def canonical_csr(n: int, src: np.ndarray, dst: np.ndarray, name: str = "", lcc: bool = True) -> Graph:
    """Symmetrise, drop self-loops, deduplicate, keep the largest connected component,
    relabel keeping the original order, and build CSR with ascending rows."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    a = np.concatenate([src, dst])
    b = np.concatenate([dst, src])
    key = np.unique(a * n + b)
    a = key // n
    b = key % n
    if lcc:
        import scipy.sparse as sp
        from scipy.sparse.csgraph import connected_components

        A = sp.csr_matrix((np.ones(len(a), dtype=np.int8), (a, b)), shape=(n, n))
        ncomp, lab = connected_components(A, directed=False)
        if ncomp > 1:
            sizes = np.bincount(lab)
            big = int(np.argmax(sizes))  # lowest label among the largest
            alive = lab == big
        else:
            alive = np.ones(n, dtype=bool)
        # isolated vertices never appear in edges but are separate components
        newid = np.full(n, -1, dtype=np.int64)
        newid[alive] = np.arange(int(alive.sum()))
        sel = alive[a]
        a, b = newid[a[sel]], newid[b[sel]]
        n = int(alive.sum())
    # key order is (a, b) ascending: rows grouped and columns ascending
    counts = np.bincount(a, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(row_ptr=row_ptr, col=b.astype(np.int32), name=name)


def from_edges(n: int, edges, name: str = "") -> Graph:
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    return canonical_csr(n, e[:, 0], e[:, 1], name=name)


# ----------------------------------------------------------------------------------------
# families
# ----------------------------------------------------------------------------------------
def grid2d(rows: int, cols: int | None = None) -> Graph:
    """rows x cols grid, vertex (i, j) has ID i*cols + j."""
    cols = rows if cols is None else cols
    ids = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    h = np.stack([ids[:, :-1].ravel(), ids[:, 1:].ravel()], axis=1)
    v = np.stack([ids[:-1, :].ravel(), ids[1:, :].ravel()], axis=1)
    e = np.concatenate([h, v])
    return canonical_csr(rows * cols, e[:, 0], e[:, 1], name="grid%dx%d" % (rows, cols), lcc=False)


def grid_center_pivot(rows: int, cols: int | None = None) -> int:
    """Minimum-eccentricity vertex of a grid with the smallest ID: ecc(i, j) =
    max(i, rows-1-i) + max(j, cols-1-j) is minimised at i = (rows-1)//2, j = (cols-1)//2."""
    cols = rows if cols is None else cols
    return ((rows - 1) // 2) * cols + (cols - 1) // 2


def _even_bits(x: np.ndarray) -> np.ndarray:
    """Bits 0, 2, 4, ... of each uint64, packed into bits 0, 1, 2, ..."""
    x = x & np.uint64(0x5555555555555555)
    x = (x | (x >> np.uint64(1))) & np.uint64(0x3333333333333333)
    x = (x | (x >> np.uint64(2))) & np.uint64(0x0F0F0F0F0F0F0F0F)
    x = (x | (x >> np.uint64(4))) & np.uint64(0x00FF00FF00FF00FF)
    x = (x | (x >> np.uint64(8))) & np.uint64(0x0000FFFF0000FFFF)
    x = (x | (x >> np.uint64(16))) & np.uint64(0x00000000FFFFFFFF)
    return x


def rmat_edges(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19,
               chunk: int = 1 << 22):
    """Raw R-MAT edge list: edge_factor * 2^scale edges; at every one of the `scale`
    levels each edge draws r uniform in [0,1) and picks quadrant q = [r >= a] + [r >= a+b]
    + [r >= a+b+c] (probabilities a, b, c, d); bit `level` of the source is q >> 1 and of
    the destination q & 1.  Draws are consumed chunk by chunk, level by level."""
    rng = np.random.default_rng(seed)
    M = edge_factor << scale
    src = np.empty(M, dtype=np.int64)
    dst = np.empty(M, dtype=np.int64)
    ab, abc = a + b, a + b + c
    r = np.empty(min(chunk, M), dtype=np.float64)
    q = np.empty(len(r), dtype=np.uint8)
    t = np.empty(len(r), dtype=np.uint8)
    for lo in range(0, M, chunk):
        L = min(M, lo + chunk) - lo
        code = np.zeros(L, dtype=np.uint64)  # quadrant of level l in bits 2l, 2l+1
        rr, qq, tt = r[:L], q[:L], t[:L]
        for level in range(scale):
            rng.random(out=rr)
            np.greater_equal(rr, a, out=qq.view(bool))
            np.greater_equal(rr, ab, out=tt.view(bool))
            qq += tt
            np.greater_equal(rr, abc, out=tt.view(bool))
            qq += tt
            code |= qq.astype(np.uint64) << np.uint64(2 * level)
        dst[lo:lo + L] = _even_bits(code).astype(np.int64)
        src[lo:lo + L] = _even_bits(code >> np.uint64(1)).astype(np.int64)
    return src, dst


def rmat(scale: int, edge_factor: int = 16, seed: int = 1) -> Graph:
    src, dst = rmat_edges(scale, edge_factor, seed)
    return canonical_csr(1 << scale, src, dst, name="rmat-s%d-ef%d-seed%d" % (scale, edge_factor, seed))


def hyperbolic(n: int, avg_degree: float = 20.0, gamma: float = 3.0, seed: int = 1,
               tol: float = 0.01, max_bisect: int = 40) -> Graph:
    """Random hyperbolic graph, threshold model (temperature 0): n points in a hyperbolic
    disk of radius R, radial density alpha sinh(alpha r) / (cosh(alpha R) - 1) with
    alpha = (gamma - 1)/2, uniform angle; an edge joins two points at hyperbolic distance
    < R.  R is tuned by bisection so that the average degree is within `tol` of the
    target (the points are drawn once; only R moves)."""
    alpha = (gamma - 1.0) / 2.0
    rng = np.random.default_rng(seed)
    theta = rng.random(n) * 2.0 * np.pi
    u01 = rng.random(n)
    # a first guess from the asymptotic degree formula, then bisection on R
    xi = alpha / (alpha - 0.5)
    R0 = 2.0 * math.log(2.0 * xi * xi * n / (math.pi * avg_degree))

    def radii(R):
        # inverse CDF of the radial density on [0, R]
        return np.arccosh(1.0 + u01 * (math.cosh(alpha * R) - 1.0)) / alpha

    def edges_for(R):
        r = radii(R)
        return _rhg_edges(r, theta, R)

    lo, hi = R0 - 2.0, R0 + 2.0
    best = None
    for _ in range(max_bisect):
        R = 0.5 * (lo + hi)
        s, d = edges_for(R)
        deg = 2.0 * len(s) / n
        best = (R, s, d)
        if abs(deg - avg_degree) <= tol * avg_degree:
            break
        if deg > avg_degree:
            lo = R
        else:
            hi = R
    R, s, d = best
    return canonical_csr(n, s, d, name="rhg-n%d-deg%g-gamma%g-seed%d" % (n, avg_degree, gamma, seed))


def _rhg_edges(r: np.ndarray, theta: np.ndarray, R: float, bands: int | None = None):
    """All pairs at hyperbolic distance < R, by radial bands and angular windows:
    cosh d = cosh r1 cosh r2 - sinh r1 sinh r2 cos(dtheta) < cosh R  <=>
    cos(dtheta) > (cosh r1 cosh r2 - cosh R) / (sinh r1 sinh r2).  For a point at r1 and a
    band with inner radius b, the largest admissible angular gap is bounded by the gap at
    r2 = b, so candidates come from one sorted-angle window per band."""
    n = len(r)
    if bands is None:
        bands = max(4, int(math.ceil(math.log2(max(n, 2)))) * 2)
    edges_s, edges_d = [], []
    order = np.argsort(theta, kind="stable")
    # band boundaries, geometric towards the rim
    bounds = np.linspace(0.0, R, bands + 1)
    band_of = np.minimum(np.searchsorted(bounds, r, side="right") - 1, bands - 1)
    coshR = math.cosh(R)
    ch, sh = np.cosh(r), np.sinh(r)
    for bi in range(bands):
        members = order[band_of[order] == bi]  # angle-sorted members of band bi
        if len(members) == 0:
            continue
        mth = theta[members]
        b_in = bounds[bi]
        # maximal angular gap for each query point against the band's inner radius
        ch_b, sh_b = math.cosh(b_in), math.sinh(b_in)
        with np.errstate(divide="ignore", invalid="ignore"):
            cosg = (ch * ch_b - coshR) / (sh * sh_b)
        cosg = np.where(np.isfinite(cosg), cosg, -1.0)
        # the admissible gap shrinks as r2 grows, so the one at the inner radius bounds the
        # band; an argument below -1 admits every angle
        gap = np.arccos(np.clip(cosg, -1.0, 1.0))
        # query only points with band >= bi to count each pair once (then filter by id)
        q = np.nonzero(band_of >= bi)[0]
        if len(q) == 0:
            continue
        lo_ang = theta[q] - gap[q]
        hi_ang = theta[q] + gap[q]
        ext = np.concatenate([mth - 2 * np.pi, mth, mth + 2 * np.pi])
        extm = np.concatenate([members, members, members])
        lo_i = np.searchsorted(ext, lo_ang, side="left")
        hi_i = np.searchsorted(ext, hi_ang, side="right")
        cnt = np.minimum(hi_i - lo_i, len(members))
        tot = int(cnt.sum())
        if tot == 0:
            continue
        qi = np.repeat(q, cnt)
        starts = np.repeat(lo_i, cnt)
        offs = np.arange(tot) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        cj = extm[starts + offs]
        keep = (qi != cj) & ((band_of[qi] > bi) | (qi < cj))
        qi, cj = qi[keep], cj[keep]
        dth = np.abs(theta[qi] - theta[cj])
        dth = np.minimum(dth, 2 * np.pi - dth)
        coshd = ch[qi] * ch[cj] - sh[qi] * sh[cj] * np.cos(dth)
        ok = coshd < coshR
        edges_s.append(qi[ok])
        edges_d.append(cj[ok])
    if not edges_s:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64)
    return np.concatenate(edges_s), np.concatenate(edges_d)


def complete(n: int) -> Graph:
    i, j = np.triu_indices(n, 1)
    return canonical_csr(n, i, j, name="K%d" % n, lcc=False)


def cycle(n: int) -> Graph:
    i = np.arange(n)
    return canonical_csr(n, i, (i + 1) % n, name="C%d" % n, lcc=False)


def path(n: int) -> Graph:
    i = np.arange(n - 1)
    return canonical_csr(n, i, i + 1, name="P%d" % n, lcc=False)


def star(n: int) -> Graph:
    i = np.arange(1, n)
    return canonical_csr(n, np.zeros(n - 1, dtype=np.int64), i, name="S%d" % n, lcc=False)


def complete_bipartite(p: int, q: int) -> Graph:
    i, j = np.meshgrid(np.arange(p), np.arange(p, p + q), indexing="ij")
    return canonical_csr(p + q, i.ravel(), j.ravel(), name="K%d,%d" % (p, q), lcc=False)


def random_tree(n: int, seed: int) -> Graph:
    rng = np.random.default_rng(seed)
    par = np.array([rng.integers(0, v) for v in range(1, n)], dtype=np.int64)
    return canonical_csr(n, par, np.arange(1, n), name="tree%d-%d" % (n, seed), lcc=False)


def random_connected(n: int, p: float, seed: int) -> Graph:
    """Erdos-Renyi G(n, p) reduced to its largest component."""
    rng = np.random.default_rng(seed)
    i, j = np.triu_indices(n, 1)
    keep = rng.random(len(i)) < p
    return canonical_csr(n, i[keep], j[keep], name="gnp%d-%g-%d" % (n, p, seed))


# ----------------------------------------------------------------------------------------
# edge weights (conductances)
# ----------------------------------------------------------------------------------------
def edge_weights(g: Graph, seed: int, kind: str = "uniform", lo: float = 1.0, hi: float = 4.0) -> np.ndarray:
    """One positive conductance per undirected edge, stored at both CSR entries (float64[2m]).
    Edges are drawn in the order of their (a < b) CSR entries with default_rng(seed):
    "uniform" in [lo, hi); "lognormal" exp(N(0, 1)); "pow2" 2^j for an integer j in
    [log2(lo), log2(hi)] (exactly representable sums); "ones" all 1."""
    n = g.n
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    upper = rows < col
    rng = np.random.default_rng(seed)
    k = int(upper.sum())
    if kind == "uniform":
        wu = rng.uniform(lo, hi, size=k)
    elif kind == "lognormal":
        wu = np.exp(rng.standard_normal(k))
    elif kind == "pow2":
        wu = np.exp2(rng.integers(int(round(math.log2(lo))), int(round(math.log2(hi))) + 1, size=k)).astype(np.float64)
    elif kind == "ones":
        wu = np.ones(k)
    else:
        raise ValueError(kind)
    w = np.zeros(len(col), dtype=np.float64)
    w[upper] = wu
    key = rows * n + col                      # ascending over the CSR
    lower = ~upper
    mirror = np.searchsorted(key, col[lower] * n + rows[lower])
    w[lower] = w[mirror]
    return w


# ----------------------------------------------------------------------------------------
# pivots
# ----------------------------------------------------------------------------------------
def max_degree_pivot(g: Graph) -> int:
    """Vertex of maximum degree, smallest ID on ties."""
    return int(np.argmax(g.degrees))


# ----------------------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------------------
def batch_members(count: int = 64, tau_cap: int = 4096):
    """The mixed batch: for g < count/2 an R-MAT graph with scale in [10, 16] and edge factor
    in [8, 16], for g >= count/2 a square grid with side in [16, 256], each drawn uniformly
    with default_rng(g); Philox seed g; pivot = max degree (R-MAT) or grid centre."""
    out = []
    half = count // 2
    for g in range(count):
        rng = np.random.default_rng(g)
        if g < half:
            scale = int(rng.integers(10, 17))
            ef = int(rng.integers(8, 17))
            G = rmat(scale, ef, seed=g)
            out.append(dict(graph=G, pivot=max_degree_pivot(G), seed=g, tau_cap=tau_cap))
        else:
            side = int(rng.integers(16, 257))
            G = grid2d(side)
            out.append(dict(graph=G, pivot=grid_center_pivot(side), seed=g, tau_cap=tau_cap))
    return out
