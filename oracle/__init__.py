"""CPU oracle for the UST estimator of diag(L^+) -- TEST INFRASTRUCTURE ONLY.

A thin ctypes loader around ``ustd_oracle.c`` (plain sequential FP64 C, built with gcc).
Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg
may import this package; the GPU library never does, and the two share no code.

Every function follows the paper (Angriman et al., ESA 2020) step by step; see the C
file for the section each one follows and for the readings of ambiguous passages.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ustd_oracle.c")
_LIB = os.path.join(_HERE, "libustd_oracle.so")

_lib = None

OK, EINVAL, EGRAPH, ENOMEM, ENOTCONV = 0, 1, 2, 3, 5


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no HIP involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        P = ctypes.c_void_p
        L.ustd_oracle_philox4x32_10.argtypes = [P, P, P]
        L.ustd_oracle_philox4x32_10.restype = None
        L.ustd_oracle_walk_word.argtypes = [u64, i64, i32, i64]
        L.ustd_oracle_walk_word.restype = ctypes.c_uint32
        L.ustd_oracle_validate.argtypes = [i64, P, P]
        L.ustd_oracle_validate.restype = ctypes.c_int
        L.ustd_oracle_bfs.argtypes = [i64, P, P, i32, P, P]
        L.ustd_oracle_bfs.restype = i32
        L.ustd_oracle_max_degree_pivot.argtypes = [i64, P]
        L.ustd_oracle_max_degree_pivot.restype = i32
        L.ustd_oracle_tau.argtypes = [i64, i64, i32, dbl, dbl, dbl]
        L.ustd_oracle_tau.restype = i64
        L.ustd_oracle_eta.argtypes = [i64, i64, i32, dbl, dbl]
        L.ustd_oracle_eta.restype = dbl
        L.ustd_oracle_wilson.argtypes = [i64, P, P, i32, u64, i64, P, P, P]
        L.ustd_oracle_wilson.restype = i64
        L.ustd_oracle_tree_flow.argtypes = [i64, i32, P, P, P]
        L.ustd_oracle_tree_flow.restype = ctypes.c_int
        L.ustd_oracle_trees.argtypes = [i64, P, P, i32, P, u64, i64, i64, P, P, P]
        L.ustd_oracle_trees.restype = ctypes.c_int
        L.ustd_oracle_solve.argtypes = [i64, P, P, i32, dbl, i64, P, P]
        L.ustd_oracle_solve.restype = i64
        L.ustd_oracle_combine.argtypes = [i64, i32, i64, P, P, P]
        L.ustd_oracle_combine.restype = None
        L.ustd_oracle_diag_lpinv.argtypes = [i64, P, P, i32, dbl, dbl, dbl, u64, i64, dbl, i64,
                                             P, P, P, P, P, P]
        L.ustd_oracle_diag_lpinv.restype = ctypes.c_int
        L.ustd_oracle_validate_weights.argtypes = [i64, P, P, P]
        L.ustd_oracle_validate_weights.restype = ctypes.c_int
        L.ustd_oracle_bpath_resistance.argtypes = [i64, P, P, P, i32, P, P, P]
        L.ustd_oracle_bpath_resistance.restype = dbl
        L.ustd_oracle_tau_weighted.argtypes = [i64, i64, dbl, dbl, dbl, dbl]
        L.ustd_oracle_tau_weighted.restype = i64
        L.ustd_oracle_fixed_shift.argtypes = [i64, dbl]
        L.ustd_oracle_fixed_shift.restype = i32
        L.ustd_oracle_fixed_weights.argtypes = [i64, i32, P, i32, P]
        L.ustd_oracle_fixed_weights.restype = None
        L.ustd_oracle_wilson_weighted.argtypes = [i64, P, P, P, i32, u64, i64, P, P, P]
        L.ustd_oracle_wilson_weighted.restype = i64
        L.ustd_oracle_tree_flow_weighted.argtypes = [i64, i32, P, P, P, P]
        L.ustd_oracle_tree_flow_weighted.restype = ctypes.c_int
        L.ustd_oracle_trees_weighted.argtypes = [i64, P, P, P, i32, P, P, u64, i64, i64, P, P, P]
        L.ustd_oracle_trees_weighted.restype = ctypes.c_int
        L.ustd_oracle_solve_weighted.argtypes = [i64, P, P, P, i32, dbl, i64, P, P]
        L.ustd_oracle_solve_weighted.restype = i64
        L.ustd_oracle_combine_weighted.argtypes = [i64, i32, i64, i32, P, P, P]
        L.ustd_oracle_combine_weighted.restype = None
        L.ustd_oracle_diag_lpinv_weighted.argtypes = [i64, P, P, P, i32, dbl, dbl, dbl, u64, i64, dbl, i64,
                                                      P, P, P, P, P, P, P]
        L.ustd_oracle_diag_lpinv_weighted.restype = ctypes.c_int
        L.ustd_oracle_blocks.argtypes = [i64, P, P, P]
        L.ustd_oracle_blocks.restype = i64
        L.ustd_oracle_wilson_blocks.argtypes = [i64, P, P, i32, P, i64, P, u64, i64, P]
        L.ustd_oracle_wilson_blocks.restype = i64
        L.ustd_oracle_trees_blocks.argtypes = [i64, P, P, i32, P, u64, i64, i64, P, P, P]
        L.ustd_oracle_trees_blocks.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    return rp, c


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ustd_oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def walk_word(seed: int, t: int, s: int, k: int) -> int:
    return int(lib().ustd_oracle_walk_word(seed, t, s, k))


def validate(row_ptr, col) -> int:
    rp, c = _csr(row_ptr, col)
    return int(lib().ustd_oracle_validate(len(rp) - 1, _p(rp), _p(c)))


def bfs(row_ptr, col, u: int):
    """Returns (dist int32[n], parB int32[n], ecc)."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    dist = np.zeros(n, dtype=np.int32)
    parB = np.zeros(n, dtype=np.int32)
    ecc = int(lib().ustd_oracle_bfs(n, _p(rp), _p(c), u, _p(dist), _p(parB)))
    return dist, parB, ecc


def max_degree_pivot(row_ptr) -> int:
    """Vertex of largest degree, smallest ID among equal degrees (the pivot rule of pivot = -1)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    return int(lib().ustd_oracle_max_degree_pivot(len(rp) - 1, _p(rp)))


def tau(n: int, m: int, ecc: int, eps: float, delta: float = 0.0, kappa: float = 0.0) -> int:
    return int(lib().ustd_oracle_tau(n, m, ecc, eps, delta, kappa))


def eta(n: int, m: int, ecc: int, eps: float, kappa: float = 0.0) -> float:
    return float(lib().ustd_oracle_eta(n, m, ecc, eps, kappa))


def wilson(row_ptr, col, u: int, seed: int, t: int):
    """One UST rooted at u.  Returns (parent int32[n], walk steps)."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    parent = np.zeros(n, dtype=np.int32)
    nxt = np.zeros(n, dtype=np.int32)
    intree = np.zeros(n, dtype=np.uint8)
    steps = int(lib().ustd_oracle_wilson(n, _p(rp), _p(c), u, seed, t, _p(parent), _p(nxt), _p(intree)))
    return parent, steps


def tree_flow(u: int, parB, parent) -> np.ndarray:
    """c_T(v) of one given tree (Algorithm 2), as int64[n]."""
    pb = np.ascontiguousarray(parB, dtype=np.int32)
    pt = np.ascontiguousarray(parent, dtype=np.int32)
    counts = np.zeros(len(pb), dtype=np.int64)
    rc = lib().ustd_oracle_tree_flow(len(pb), u, _p(pb), _p(pt), _p(counts))
    if rc != OK:
        raise RuntimeError("oracle tree_flow failed: %d" % rc)
    return counts


def trees(row_ptr, col, u: int, seed: int, tree_begin: int, tree_count: int,
          want_parents: bool = True, want_counts: bool = True, parB=None):
    """Trees [tree_begin, tree_begin + tree_count).  Returns (parents or None, steps, counts or None).
    parB: the BFS parents of u if already computed (else the BFS runs here)."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    if parB is None:
        _, parB, _ = bfs(rp, c, u)
    parB = np.ascontiguousarray(parB, dtype=np.int32)
    parents = np.zeros((tree_count, n), dtype=np.int32) if want_parents else None
    steps = np.zeros(tree_count, dtype=np.int64)
    counts = np.zeros(n, dtype=np.int64) if want_counts else None
    rc = lib().ustd_oracle_trees(n, _p(rp), _p(c), u, _p(parB), seed, tree_begin, tree_count,
                                 _p(parents) if parents is not None else None, _p(steps),
                                 _p(counts) if counts is not None else None)
    if rc != OK:
        raise RuntimeError("oracle trees failed: %d" % rc)
    return parents, steps, counts


def trees_threads(row_ptr, col, u: int, seed: int, tree_begin: int, tree_count: int, threads: int, parB=None):
    """The trees of `trees` (steps and flow counts, no parents) split into `threads` contiguous
    ranges, each run by the sequential C code on its own host thread (the foreign call releases
    the interpreter lock).  Trees are independent and counts are integers, so the result is the
    same as one sequential call.  Returns (steps, counts)."""
    import threading

    rp, c = _csr(row_ptr, col)
    if parB is None:
        _, parB, _ = bfs(rp, c, u)
    threads = max(1, min(int(threads), int(tree_count))) if tree_count > 0 else 1
    bounds = [tree_begin + (tree_count * i) // threads for i in range(threads + 1)]
    out = [None] * threads

    def run(i):
        out[i] = trees(rp, c, u, seed, bounds[i], bounds[i + 1] - bounds[i], want_parents=False, parB=parB)

    ts = [threading.Thread(target=run, args=(i,)) for i in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    steps = np.concatenate([o[1] for o in out])
    counts = np.sum([o[2] for o in out], axis=0).astype(np.int64)
    return steps, counts


def blocks(row_ptr, col):
    """Biconnected components of the edges (Tarjan): (eblock int32[nnz], the same id at both
    entries of an edge, and the number of blocks)."""
    rp, c = _csr(row_ptr, col)
    eb = np.zeros(len(c), dtype=np.int32)
    nb = int(lib().ustd_oracle_blocks(len(rp) - 1, _p(rp), _p(c), _p(eb)))
    if nb < 0:
        raise RuntimeError("oracle blocks: out of memory")
    return eb, nb


def wilson_blocks(row_ptr, col, u: int, seed: int, t: int):
    """One UST rooted at u by Wilson's algorithm per biconnected component (the engineering
    appendix's variant).  Returns (parent int32[n], walk steps)."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    eb, nb = blocks(rp, c)
    dist, _, _ = bfs(rp, c, u)
    parent = np.zeros(n, dtype=np.int32)
    steps = int(lib().ustd_oracle_wilson_blocks(n, _p(rp), _p(c), u, _p(eb), nb, _p(dist), seed, t, _p(parent)))
    if steps < 0:
        raise RuntimeError("oracle wilson_blocks: out of memory")
    return parent, steps


def trees_blocks(row_ptr, col, u: int, seed: int, tree_begin: int, tree_count: int,
                 want_parents: bool = True, want_counts: bool = True):
    """Trees [tree_begin, +tree_count) of the per-block variant.  Returns (parents or None, steps,
    counts or None); counts by Algorithm 2 on the joined trees."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    _, parB, _ = bfs(rp, c, u)
    parents = np.zeros((tree_count, n), dtype=np.int32) if want_parents else None
    steps = np.zeros(tree_count, dtype=np.int64)
    counts = np.zeros(n, dtype=np.int64) if want_counts else None
    rc = lib().ustd_oracle_trees_blocks(n, _p(rp), _p(c), u, _p(parB), seed, tree_begin, tree_count,
                                        _p(parents) if parents is not None else None, _p(steps),
                                        _p(counts) if counts is not None else None)
    if rc != OK:
        raise RuntimeError("oracle trees_blocks failed: %d" % rc)
    return parents, steps, counts


def solve(row_ptr, col, u: int, tol: float = 1e-12, maxit: int = 100000):
    """Column u of L^+ by FP64 Jacobi-PCG + mean-zero projection.  Returns (x, iters, relres)."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    x = np.zeros(n, dtype=np.float64)
    rr = ctypes.c_double(0.0)
    it = int(lib().ustd_oracle_solve(n, _p(rp), _p(c), u, tol, maxit, _p(x), ctypes.byref(rr)))
    return x, it, rr.value


def combine(u: int, tau_: int, counts, x) -> np.ndarray:
    cnt = np.ascontiguousarray(counts, dtype=np.int64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    diag = np.zeros(len(cnt), dtype=np.float64)
    lib().ustd_oracle_combine(len(cnt), u, tau_, _p(cnt), _p(xx), _p(diag))
    return diag


def diag_lpinv(row_ptr, col, u: int, eps: float, seed: int, delta: float = 0.0, kappa: float = 0.0,
               tau_override: int = 0, solve_tol: float = 0.0, solve_maxit: int = 0):
    """Algorithm 1 end to end.  Returns dict(diag, counts, tau, ecc, steps, relres, status)."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    diag = np.zeros(n, dtype=np.float64)
    counts = np.zeros(n, dtype=np.int64)
    t = ctypes.c_int64(0)
    e = ctypes.c_int32(0)
    s = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    rc = lib().ustd_oracle_diag_lpinv(n, _p(rp), _p(c), u, eps, delta, kappa, seed, tau_override,
                                      solve_tol, solve_maxit, _p(diag), _p(counts), ctypes.byref(t),
                                      ctypes.byref(e), ctypes.byref(s), ctypes.byref(rr))
    return dict(diag=diag, counts=counts, tau=t.value, ecc=e.value, steps=s.value,
                relres=rr.value, status=rc)


# ---------------------------------------------------------------------------------------
# Weighted graphs (Section "Generalizations"; readings in the C file): conductance-weighted
# Wilson steps, Algorithm 2 with the Ohm's-law factor 1/w(e) in fixed point (F = 2^k / w of
# each vertex's B_u edge), tau from the largest B-path resistance, weighted Laplacian solve.
# ---------------------------------------------------------------------------------------
def _w(w):
    return np.ascontiguousarray(w, dtype=np.float64)


def validate_weights(row_ptr, col, w) -> int:
    rp, c = _csr(row_ptr, col)
    return int(lib().ustd_oracle_validate_weights(len(rp) - 1, _p(rp), _p(c), _p(_w(w))))


def bpath_resistance(row_ptr, col, w, u: int):
    """Returns (wB float64[n], rho float64[n], rho_max): the conductance of each vertex's B_u
    edge and the resistance of P(v), summed from v towards u."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    _, parB, _ = bfs(rp, c, u)
    wB = np.zeros(n)
    rho = np.zeros(n)
    rmax = float(lib().ustd_oracle_bpath_resistance(n, _p(rp), _p(c), _p(_w(w)), u, _p(parB), _p(wB), _p(rho)))
    return wB, rho, rmax


def tau_weighted(n: int, m: int, rho_max: float, eps: float, delta: float = 0.0, kappa: float = 0.0) -> int:
    return int(lib().ustd_oracle_tau_weighted(n, m, rho_max, eps, delta, kappa))


def fixed_shift(tau_: int, rho_max: float) -> int:
    return int(lib().ustd_oracle_fixed_shift(tau_, rho_max))


def fixed_weights(u: int, wB, k: int) -> np.ndarray:
    wb = _w(wB)
    F = np.zeros(len(wb), dtype=np.int64)
    lib().ustd_oracle_fixed_weights(len(wb), u, _p(wb), k, _p(F))
    return F


def wilson_weighted(row_ptr, col, w, u: int, seed: int, t: int):
    """One tree drawn with probability proportional to its weight.  Returns (parent, steps)."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    parent = np.zeros(n, dtype=np.int32)
    nxt = np.zeros(n, dtype=np.int32)
    intree = np.zeros(n, dtype=np.uint8)
    steps = int(lib().ustd_oracle_wilson_weighted(n, _p(rp), _p(c), _p(_w(w)), u, seed, t, _p(parent), _p(nxt),
                                                  _p(intree)))
    return parent, steps


def tree_flow_weighted(u: int, parB, parent, F) -> np.ndarray:
    """Fixed-point c_T(v) of one given tree (Algorithm 2 with +-F[b] per edge), int64[n]."""
    pb = np.ascontiguousarray(parB, dtype=np.int32)
    pt = np.ascontiguousarray(parent, dtype=np.int32)
    f = np.ascontiguousarray(F, dtype=np.int64)
    acc = np.zeros(len(pb), dtype=np.int64)
    rc = lib().ustd_oracle_tree_flow_weighted(len(pb), u, _p(pb), _p(pt), _p(f), _p(acc))
    if rc != OK:
        raise RuntimeError("oracle tree_flow_weighted failed: %d" % rc)
    return acc


def trees_weighted(row_ptr, col, w, u: int, seed: int, tree_begin: int, tree_count: int, k: int,
                   want_parents: bool = True, want_acc: bool = True):
    """Weighted trees [tree_begin, +tree_count) with fixed-point shift k.
    Returns (parents or None, steps, acc or None)."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    ww = _w(w)
    _, parB, _ = bfs(rp, c, u)
    wB, _, _ = bpath_resistance(rp, c, ww, u)
    F = fixed_weights(u, wB, k)
    parents = np.zeros((tree_count, n), dtype=np.int32) if want_parents else None
    steps = np.zeros(tree_count, dtype=np.int64)
    acc = np.zeros(n, dtype=np.int64) if want_acc else None
    rc = lib().ustd_oracle_trees_weighted(n, _p(rp), _p(c), _p(ww), u, _p(parB), _p(F), seed, tree_begin,
                                          tree_count, _p(parents) if parents is not None else None, _p(steps),
                                          _p(acc) if acc is not None else None)
    if rc != OK:
        raise RuntimeError("oracle trees_weighted failed: %d" % rc)
    return parents, steps, acc


def solve_weighted(row_ptr, col, w, u: int, tol: float = 1e-12, maxit: int = 100000):
    """Column u of the weighted L^+ (FP64 Jacobi-PCG + projection).  Returns (x, iters, relres)."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    x = np.zeros(n, dtype=np.float64)
    rr = ctypes.c_double(0.0)
    it = int(lib().ustd_oracle_solve_weighted(n, _p(rp), _p(c), _p(_w(w)), u, tol, maxit, _p(x), ctypes.byref(rr)))
    return x, it, rr.value


def combine_weighted(u: int, tau_: int, k: int, acc, x) -> np.ndarray:
    a = np.ascontiguousarray(acc, dtype=np.int64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    diag = np.zeros(len(a), dtype=np.float64)
    lib().ustd_oracle_combine_weighted(len(a), u, tau_, k, _p(a), _p(xx), _p(diag))
    return diag


def diag_lpinv_weighted(row_ptr, col, w, u: int, eps: float, seed: int, delta: float = 0.0, kappa: float = 0.0,
                        tau_override: int = 0, solve_tol: float = 0.0, solve_maxit: int = 0):
    """Algorithm 1 on a weighted graph.  Returns dict(diag, acc, tau, shift, rho_max, steps, relres, status)."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    diag = np.zeros(n, dtype=np.float64)
    acc = np.zeros(n, dtype=np.int64)
    t = ctypes.c_int64(0)
    k = ctypes.c_int32(0)
    rmax = ctypes.c_double(0.0)
    s = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    rc = lib().ustd_oracle_diag_lpinv_weighted(n, _p(rp), _p(c), _p(_w(w)), u, eps, delta, kappa, seed,
                                               tau_override, solve_tol, solve_maxit, _p(diag), _p(acc),
                                               ctypes.byref(t), ctypes.byref(k), ctypes.byref(rmax),
                                               ctypes.byref(s), ctypes.byref(rr))
    return dict(diag=diag, acc=acc, tau=t.value, shift=k.value, rho_max=rmax.value, steps=s.value,
                relres=rr.value, status=rc)


# ---------------------------------------------------------------------------------------
# Measures derived from the estimator's outputs (plain numpy; the paper's formulas)
# ---------------------------------------------------------------------------------------
def centralities(diag) -> dict:
    """Vertex measures that depend only on diag(L^+):
    trace tr(L^+); electrical farness n L^+_vv + tr (Eq. elec-farness, section on electrical
    closeness); electrical closeness (n-1)/farness; normalized random-walk betweenness
    1/n + tr/((n-1) farness) (Lemma on NRWB); Kirchhoff index n tr (Kirchhoff appendix)."""
    d = np.asarray(diag, dtype=np.float64)
    n = len(d)
    tr = float(np.sum(d))
    far = n * d + tr
    return dict(trace=tr, kirchhoff=n * tr, farness=far, closeness=(n - 1) / far,
                nrwb=1.0 / n + tr / ((n - 1) * far))


def edge_sample_size(n: int, m: int, eps: float, delta: float = 0.0) -> int:
    """q = ceil(2 eps^-2 ln(2m/delta)) trees for every edge's effective resistance within eps
    (Kirchhoff appendix, after Hayashi et al.); delta <= 0 selects 1/n."""
    import math

    d = delta if delta > 0 else 1.0 / n
    return int(math.ceil(2.0 * math.log(2.0 * m / d) / (eps * eps)))


def edge_counts(row_ptr, col, parents, u: int) -> np.ndarray:
    """Spanning-edge counts (Kirchhoff appendix: for each edge the number of sampled USTs it
    appears in) of the given parent arrays.  The edge {v, parent(v)} is counted at the CSR
    position of (min, max) of its endpoints; entries (a, b) with a > b stay 0."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    key = rows * n + c  # ascending: rows in order, each row ascending
    counts = np.zeros(len(c), dtype=np.int64)
    par = np.asarray(parents, dtype=np.int64).reshape(-1, n)
    v = np.arange(n, dtype=np.int64)
    for p in par:
        keep = v != u
        a = np.minimum(v[keep], p[keep])
        b = np.maximum(v[keep], p[keep])
        slot = np.searchsorted(key, a * n + b)
        assert (key[slot] == a * n + b).all(), "a parent is not a neighbour"
        np.add.at(counts, slot, 1)
    return counts


def edge_resistances(row_ptr, col, counts, q, theta: float, w=None):
    """Edge measures from spanning-edge counts (Kirchhoff index appendix): lev(e) = c(e) / q, the
    fraction of the q trees containing e, estimates the leverage w(e) r(e); r(e) = lev / w(e);
    the denominator of the Sherman-Morrison form of C^Delta_theta(e) is 1 - (1 - theta) w(e) r(e)
    = 1 - (1 - theta) lev.  counts is per CSR entry, at the entries (a, b) with a < b (as
    edge_counts returns them; a float array of exact leverages times q is accepted too).
    Returns (r, denom) per CSR entry, the edge's value at both of its entries."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    cols = c.astype(np.int64)
    key = rows * n + cols
    cnt = np.asarray(counts)
    upper_slot = np.where(rows < cols, np.arange(len(cols)), np.searchsorted(key, cols * n + rows))
    lev = cnt[upper_slot].astype(np.float64) / float(q)
    ww = np.ones(len(cols)) if w is None else np.asarray(w, dtype=np.float64)
    return lev / ww, 1.0 - (1.0 - theta) * lev


def sweep_pivot(row_ptr, col, sweeps: int = 10) -> tuple:
    """Pivot of low eccentricity by repeated BFS sweeps (engineering appendix, after Magnien et
    al.'s double sweep): BFS from a first source, then from the vertex farthest from it, and
    so on, `sweeps` BFS in all; every BFS raises each vertex's lower bound on its
    eccentricity to its distance from the source; the pivot is the vertex with the lowest
    bound.  Readings: the first source is the maximum-degree vertex (the paper draws it at
    random); ties everywhere go to the smallest vertex ID.  Returns (pivot, bounds)."""
    rp, c = _csr(row_ptr, col)
    n = len(rp) - 1
    deg = np.diff(rp)
    src = int(np.flatnonzero(deg == deg.max())[0])
    bound = np.zeros(n, dtype=np.int64)
    for _ in range(sweeps):
        dist, _, ecc = bfs(rp, c, src)
        bound = np.maximum(bound, dist)
        src = int(np.flatnonzero(dist == ecc)[0])
    piv = int(np.flatnonzero(bound == bound.min())[0])
    return piv, bound
