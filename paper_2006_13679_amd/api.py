"""Python binding of libustd.so (include/ustd.h): argument marshalling only.

Every step of the estimator runs in the library's HIP kernels; torch provides device
memory (inputs, outputs, the workspace) and the stream.  If the built library is missing
the calls raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libustd.so")

OK, EINVAL, EGRAPH, ENOMEM, EHIP, ENOTCONV = 0, 1, 2, 3, 4, 5
SOLVE_FP64, SOLVE_MIXED = 0, 1
ENGINE_AUTO, ENGINE_WORKGROUP, ENGINE_MULTI = 0, 1, 2
WILSON_PLAIN, WILSON_BLOCKS = 0, 1
LAYOUT_AUTO, LAYOUT_RECORDS = 0, 1


class UstdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


_STATUS = {0: "USTD_OK", 1: "USTD_EINVAL", 2: "USTD_EGRAPH", 3: "USTD_ENOMEM", 4: "USTD_EHIP", 5: "USTD_ENOTCONV"}


class Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("d_row_ptr", ctypes.c_void_p), ("d_col", ctypes.c_void_p),
        ("pivot", ctypes.c_int32), ("solve_mode", ctypes.c_int32),
        ("eps", ctypes.c_double), ("delta", ctypes.c_double), ("kappa", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("tau_override", ctypes.c_int64),
        ("solve_tol", ctypes.c_double), ("solve_maxit", ctypes.c_int32),
        ("validate", ctypes.c_int32), ("trees_per_batch", ctypes.c_int32), ("tau_cap", ctypes.c_int32),
        ("d_weight", ctypes.c_void_p), ("solve_engine", ctypes.c_int32), ("wilson_variant", ctypes.c_int32),
    ]


class Report(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_int64), ("walk_steps", ctypes.c_int64), ("walk_draws", ctypes.c_int64),
        ("pivot", ctypes.c_int32), ("ecc", ctypes.c_int32), ("solve_iters", ctypes.c_int32),
        ("solve_outer", ctypes.c_int32), ("n_batches", ctypes.c_int32), ("trees_per_batch", ctypes.c_int32),
        ("solve_relres", ctypes.c_double),
        ("ms_setup", ctypes.c_double), ("ms_bfs", ctypes.c_double), ("ms_sample", ctypes.c_double),
        ("ms_intervals", ctypes.c_double), ("ms_aggregate", ctypes.c_double), ("ms_solve", ctypes.c_double),
        ("ms_combine", ctypes.c_double), ("ms_total", ctypes.c_double),
        ("rho_max", ctypes.c_double), ("fixed_shift", ctypes.c_int32), ("weighted", ctypes.c_int32),
        ("eta", ctypes.c_double), ("solve_tol", ctypes.c_double), ("solve_converged", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Schedule(ctypes.Structure):
    """ustd_batch_schedule: launch schedule of a planned batch (zeros = defaults)."""
    _fields_ = [
        ("group_fills", ctypes.c_int32), ("agg_chunk", ctypes.c_int32), ("layout", ctypes.c_int32),
        ("branches", ctypes.c_int32), ("fill_trees", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


EXPORTS = ["ustd_workspace_bytes", "ustd_bfs", "ustd_sample_trees", "ustd_flow_counts", "ustd_tree_counts",
           "ustd_solve_pivot_column", "ustd_diag_lpinv", "ustd_diag_lpinv_noalloc", "ustd_batch_workspace_bytes",
           "ustd_batch_diag_lpinv", "ustd_batch_plan_create", "ustd_batch_plan_execute", "ustd_batch_plan_reports",
           "ustd_batch_plan_schedule", "ustd_batch_plan_destroy", "ustd_batch_graph_create", "ustd_batch_graph_launch",
           "ustd_batch_graph_destroy", "ustd_batch_autotune",
           "ustd_edge_counts", "ustd_edge_sample_size", "ustd_edge_resistances", "ustd_centralities",
           "ustd_philox_words", "ustd_status_string", "ustd_last_error"]

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libustd.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        PP = ctypes.POINTER(Problem)
        PR = ctypes.POINTER(Report)
        L.ustd_workspace_bytes.argtypes = [PP, ctypes.POINTER(ctypes.c_size_t)]
        L.ustd_bfs.argtypes = [PP, P, ctypes.c_size_t, P, P, ctypes.POINTER(i32), ctypes.POINTER(i32), P]
        L.ustd_sample_trees.argtypes = [PP, i64, i64, P, ctypes.c_size_t, P, P, P]
        L.ustd_flow_counts.argtypes = [PP, i64, i64, P, ctypes.c_size_t, P, PR, P]
        L.ustd_tree_counts.argtypes = [PP, P, i64, P, ctypes.c_size_t, P, P]
        L.ustd_solve_pivot_column.argtypes = [PP, P, ctypes.c_size_t, P, PR, P]
        L.ustd_diag_lpinv.argtypes = [PP, P, ctypes.c_size_t, P, P, PR, P]
        L.ustd_diag_lpinv_noalloc.argtypes = [PP, P, P, PR, P]
        L.ustd_batch_workspace_bytes.argtypes = [PP, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.ustd_batch_diag_lpinv.argtypes = [PP, i32, P, ctypes.c_size_t, P, P, PR, P]
        PS = ctypes.POINTER(Schedule)
        L.ustd_batch_plan_create.argtypes = [PP, i32, P, ctypes.c_size_t, PS, ctypes.POINTER(P), P]
        L.ustd_batch_plan_execute.argtypes = [P, P, P, P]
        L.ustd_batch_plan_reports.argtypes = [P, PR, P]
        L.ustd_batch_plan_schedule.argtypes = [P, PS]
        L.ustd_batch_plan_destroy.argtypes = [P]
        L.ustd_batch_graph_create.argtypes = [P, P, P, ctypes.POINTER(P)]
        L.ustd_batch_graph_launch.argtypes = [P, P]
        L.ustd_batch_graph_destroy.argtypes = [P]
        L.ustd_batch_autotune.argtypes = [PP, i32, P, ctypes.c_size_t, ctypes.c_char_p, i32, PS,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32), P]
        L.ustd_edge_counts.argtypes = [PP, i64, i64, P, ctypes.c_size_t, P, PR, P]
        L.ustd_edge_sample_size.argtypes = [i64, i64, ctypes.c_double, ctypes.c_double, ctypes.POINTER(i64)]
        L.ustd_edge_resistances.argtypes = [i64, i64, P, P, P, P, i64, ctypes.c_double, P, P, P]
        L.ustd_centralities.argtypes = [i64, P, P, P, P, P, P]
        L.ustd_philox_words.argtypes = [u64, i64, i32, i64, i64, P, P]
        for name in EXPORTS[:-2]:
            getattr(L, name).restype = ctypes.c_int
        L.ustd_status_string.argtypes = [ctypes.c_int]
        L.ustd_status_string.restype = ctypes.c_char_p
        L.ustd_last_error.argtypes = []
        L.ustd_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int, allow=(OK,)):
    if rc not in allow:
        raise UstdError(rc, lib().ustd_last_error().decode())
    return rc


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


@dataclass
class Graph:
    """A CSR graph resident on the device (int64 row pointers, int32 columns, optional
    float64 conductances per CSR entry)."""
    row_ptr: torch.Tensor
    col: torch.Tensor
    weight: torch.Tensor | None = None

    @property
    def n(self) -> int:
        return self.row_ptr.numel() - 1

    @property
    def nnz(self) -> int:
        return self.col.numel()

    @staticmethod
    def from_host(row_ptr, col, device="cuda", weight=None) -> "Graph":
        rp = torch.as_tensor(row_ptr, dtype=torch.int64).to(device).contiguous()
        c = torch.as_tensor(col, dtype=torch.int32).to(device).contiguous()
        w = None if weight is None else torch.as_tensor(weight, dtype=torch.float64).to(device).contiguous()
        return Graph(rp, c, w)


def problem(g: Graph, pivot: int = -1, eps: float = 0.3, seed: int = 1, delta: float = 0.0, kappa: float = 0.0,
            tau_override: int = 0, solve_mode: int = SOLVE_FP64, solve_tol: float = 0.0, solve_maxit: int = 0,
            validate: bool = False, trees_per_batch: int = 0, tau_cap: int = 0,
            solve_engine: int = ENGINE_AUTO, wilson_variant: int = WILSON_PLAIN) -> Problem:
    assert g.row_ptr.dtype == torch.int64 and g.col.dtype == torch.int32
    assert g.row_ptr.is_cuda and g.col.is_cuda and g.row_ptr.is_contiguous() and g.col.is_contiguous()
    w = g.weight
    if w is not None:
        assert w.dtype == torch.float64 and w.is_cuda and w.is_contiguous() and w.numel() == g.nnz
    return Problem(n=g.n, nnz=g.nnz, d_row_ptr=g.row_ptr.data_ptr(), d_col=g.col.data_ptr(), pivot=pivot,
                   solve_mode=solve_mode, eps=eps, delta=delta, kappa=kappa, seed=seed & 0xFFFFFFFFFFFFFFFF,
                   tau_override=tau_override, solve_tol=solve_tol, solve_maxit=solve_maxit,
                   validate=1 if validate else 0, trees_per_batch=trees_per_batch, tau_cap=tau_cap,
                   d_weight=w.data_ptr() if w is not None else None, solve_engine=solve_engine,
                   wilson_variant=wilson_variant)


def with_engine(p: Problem, engine: int) -> Problem:
    """A copy of the problem with another solve engine (ENGINE_*)."""
    q = Problem.from_buffer_copy(p)
    q.solve_engine = engine
    return q


def workspace_bytes(p: Problem) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().ustd_workspace_bytes(ctypes.byref(p), ctypes.byref(b)))
    return int(b.value)


class Workspace:
    """A reusable device workspace (grown on demand, 256-byte aligned by torch's allocator)."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws: dict = {}


def _ws(p: Problem, g: Graph, ws: Workspace | None):
    if ws is None:
        key = g.row_ptr.device
        ws = _default_ws.setdefault(key, Workspace(key))
    nbytes = workspace_bytes(p)
    buf = ws.get(nbytes)
    return buf, buf.numel()


def bfs(g: Graph, p: Problem, ws: Workspace | None = None):
    buf, nb = _ws(p, g, ws)
    dist = torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
    parB = torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
    ecc, piv = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().ustd_bfs(ctypes.byref(p), _ptr(buf), nb, _ptr(dist), _ptr(parB), ctypes.byref(ecc),
                          ctypes.byref(piv), _stream(g.row_ptr.device)))
    return dist, parB, int(ecc.value), int(piv.value)


def sample_trees(g: Graph, p: Problem, tree_begin: int, tree_count: int, ws: Workspace | None = None):
    buf, nb = _ws(p, g, ws)
    dev = g.row_ptr.device
    parents = torch.empty((tree_count, g.n), dtype=torch.int32, device=dev)
    steps = torch.empty(tree_count, dtype=torch.int64, device=dev)
    _check(lib().ustd_sample_trees(ctypes.byref(p), tree_begin, tree_count, _ptr(buf), nb, _ptr(parents),
                                   _ptr(steps), _stream(dev)))
    return parents, steps


def flow_counts(g: Graph, p: Problem, tree_begin: int, tree_count: int, counts: torch.Tensor | None = None,
                ws: Workspace | None = None):
    buf, nb = _ws(p, g, ws)
    dev = g.row_ptr.device
    if counts is None:
        counts = torch.zeros(g.n, dtype=torch.int64, device=dev)
    rep = Report()
    _check(lib().ustd_flow_counts(ctypes.byref(p), tree_begin, tree_count, _ptr(buf), nb, _ptr(counts),
                                  ctypes.byref(rep), _stream(dev)))
    return counts, rep.as_dict()


def tree_counts(g: Graph, p: Problem, parents: torch.Tensor, counts: torch.Tensor | None = None,
                ws: Workspace | None = None):
    buf, nb = _ws(p, g, ws)
    dev = g.row_ptr.device
    parents = parents.to(device=dev, dtype=torch.int32).contiguous()
    assert parents.dim() == 2 and parents.shape[1] == g.n
    if counts is None:
        counts = torch.zeros(g.n, dtype=torch.int64, device=dev)
    _check(lib().ustd_tree_counts(ctypes.byref(p), _ptr(parents), parents.shape[0], _ptr(buf), nb, _ptr(counts),
                                  _stream(dev)))
    return counts


def solve_pivot_column(g: Graph, p: Problem, ws: Workspace | None = None, allow_notconv: bool = False):
    buf, nb = _ws(p, g, ws)
    dev = g.row_ptr.device
    x = torch.empty(g.n, dtype=torch.float64, device=dev)
    rep = Report()
    rc = lib().ustd_solve_pivot_column(ctypes.byref(p), _ptr(buf), nb, _ptr(x), ctypes.byref(rep), _stream(dev))
    _check(rc, (OK, ENOTCONV) if allow_notconv else (OK,))
    return x, rep.as_dict()


def diag_lpinv_p(g: Graph, p: Problem, ws: Workspace | None = None, want_counts: bool = True,
                 allow_notconv: bool = False):
    """ApproxDiagLpinv on a prepared problem.  Returns (diag float64[n], counts int64[n] or None, report)."""
    buf, nb = _ws(p, g, ws)
    dev = g.row_ptr.device
    diag = torch.empty(g.n, dtype=torch.float64, device=dev)
    counts = torch.empty(g.n, dtype=torch.int64, device=dev) if want_counts else None
    rep = Report()
    rc = lib().ustd_diag_lpinv(ctypes.byref(p), _ptr(buf), nb, _ptr(diag), _ptr(counts), ctypes.byref(rep),
                               _stream(dev))
    _check(rc, (OK, ENOTCONV) if allow_notconv else (OK,))
    out = rep.as_dict()
    out["status"] = rc
    return diag, counts, out


NOALLOC_SCRATCH_BYTES = 64 << 20


def diag_lpinv_noalloc_p(g: Graph, p: Problem, diag: torch.Tensor, counts: torch.Tensor | None = None,
                         allow_notconv: bool = False):
    """ApproxDiagLpinv through the allocation-free entry point (the library's own static device
    scratch, no workspace): the caller passes the outputs.  Returns the report."""
    dev = g.row_ptr.device
    assert diag.dtype == torch.float64 and diag.numel() == g.n and diag.is_contiguous()
    rep = Report()
    rc = lib().ustd_diag_lpinv_noalloc(ctypes.byref(p), _ptr(diag), _ptr(counts), ctypes.byref(rep), _stream(dev))
    _check(rc, (OK, ENOTCONV) if allow_notconv else (OK,))
    out = rep.as_dict()
    out["status"] = rc
    return out


def diag_lpinv(row_ptr, col, pivot: int = -1, eps: float = 0.3, seed: int = 1, weight=None, **kw):
    """diag(L^+) of a CSR graph (host or device arrays; optional conductances per CSR entry)
    by the UST estimator."""
    g = Graph.from_host(row_ptr, col, weight=weight)
    p = problem(g, pivot=pivot, eps=eps, seed=seed, **kw)
    return diag_lpinv_p(g, p)


def batch_diag_lpinv(graphs: list, probs: list, ws: Workspace | None = None, want_counts: bool = True,
                     allow_notconv: bool = False):
    """ApproxDiagLpinv for several prepared problems in one call (ustd_batch_diag_lpinv).
    Returns (list of diag float64[n_i], list of counts int64[n_i] or None, list of reports)."""
    count = len(probs)
    assert count == len(graphs) and count > 0
    dev = graphs[0].row_ptr.device
    arr = (Problem * count)(*probs)
    b = ctypes.c_size_t(0)
    _check(lib().ustd_batch_workspace_bytes(arr, count, ctypes.byref(b)))
    if ws is None:
        ws = _default_ws.setdefault(dev, Workspace(dev))
    buf = ws.get(int(b.value))
    diags = [torch.empty(g.n, dtype=torch.float64, device=dev) for g in graphs]
    counts = [torch.empty(g.n, dtype=torch.int64, device=dev) for g in graphs] if want_counts else None
    dptr = (ctypes.c_void_p * count)(*[d.data_ptr() for d in diags])
    cptr = (ctypes.c_void_p * count)(*[c.data_ptr() for c in counts]) if want_counts else None
    reps = (Report * count)()
    rc = lib().ustd_batch_diag_lpinv(arr, count, _ptr(buf), buf.numel(), dptr, cptr, reps, _stream(dev))
    _check(rc, (OK, ENOTCONV) if allow_notconv else (OK,))
    return diags, counts, [r.as_dict() for r in reps]


def _batch_ws(graphs: list, probs: list, ws: Workspace | None):
    count = len(probs)
    assert count == len(graphs) and count > 0
    dev = graphs[0].row_ptr.device
    arr = (Problem * count)(*probs)
    b = ctypes.c_size_t(0)
    _check(lib().ustd_batch_workspace_bytes(arr, count, ctypes.byref(b)))
    if ws is None:
        ws = _default_ws.setdefault(dev, Workspace(dev))
    return arr, ws.get(int(b.value)), dev


class BatchPlan:
    """A planned batch (ustd_batch_plan_*): set up once, then executed eagerly or through a
    captured HIP graph.  Owns its output tensors; the workspace buffer is held until close()."""

    def __init__(self, graphs: list, probs: list, ws: Workspace | None = None, schedule: Schedule | None = None,
                 want_counts: bool = True):
        arr, buf, dev = _batch_ws(graphs, probs, ws)
        self.count, self.dev, self._buf, self._graphs = len(probs), dev, buf, list(graphs)
        self.diags = [torch.empty(g.n, dtype=torch.float64, device=dev) for g in graphs]
        self.counts = [torch.empty(g.n, dtype=torch.int64, device=dev) for g in graphs] if want_counts else None
        self._dptr = (ctypes.c_void_p * self.count)(*[d.data_ptr() for d in self.diags])
        self._cptr = (ctypes.c_void_p * self.count)(*[c.data_ptr() for c in self.counts]) if want_counts else None
        h = ctypes.c_void_p(None)
        _check(lib().ustd_batch_plan_create(arr, self.count, _ptr(buf), buf.numel(),
                                            ctypes.byref(schedule) if schedule is not None else None,
                                            ctypes.byref(h), _stream(dev)))
        self._h = h
        self._graph = None

    def schedule(self) -> dict:
        s = Schedule()
        _check(lib().ustd_batch_plan_schedule(self._h, ctypes.byref(s)))
        return s.as_dict()

    def execute(self):
        _check(lib().ustd_batch_plan_execute(self._h, self._dptr, self._cptr, _stream(self.dev)))

    def capture(self):
        """Captures one execution into a HIP graph (replaced if one exists)."""
        if self._graph is not None:
            _check(lib().ustd_batch_graph_destroy(self._graph))
            self._graph = None
        g = ctypes.c_void_p(None)
        _check(lib().ustd_batch_graph_create(self._h, self._dptr, self._cptr, ctypes.byref(g)))
        self._graph = g

    def replay(self):
        assert self._graph is not None, "capture() first"
        _check(lib().ustd_batch_graph_launch(self._graph, _stream(self.dev)))

    def reports(self, allow_notconv: bool = False) -> list:
        reps = (Report * self.count)()
        rc = lib().ustd_batch_plan_reports(self._h, reps, _stream(self.dev))
        _check(rc, (OK, ENOTCONV) if allow_notconv else (OK,))
        return [r.as_dict() for r in reps]

    def close(self):
        if self._graph is not None:
            lib().ustd_batch_graph_destroy(self._graph)
            self._graph = None
        if self._h:
            torch.cuda.synchronize(self.dev)
            lib().ustd_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_autotune(graphs: list, probs: list, ws: Workspace | None = None, cache_path: str | None = None,
                   graph: bool = True):
    """Tuned schedule of a batch (ustd_batch_autotune), timing graph replays (graph=True) or eager
    executions.  Returns (Schedule, ms per execution, whether it came from the cache)."""
    arr, buf, dev = _batch_ws(graphs, probs, ws)
    best = Schedule()
    ms = ctypes.c_double(0.0)
    hit = ctypes.c_int32(0)
    _check(lib().ustd_batch_autotune(arr, len(probs), _ptr(buf), buf.numel(),
                                     cache_path.encode() if cache_path else None, 1 if graph else 0, ctypes.byref(best),
                                     ctypes.byref(ms), ctypes.byref(hit), _stream(dev)))
    return best, float(ms.value), bool(hit.value)


def edge_counts(g: Graph, p: Problem, tree_begin: int, tree_count: int, counts: torch.Tensor | None = None,
                ws: Workspace | None = None):
    """Spanning-edge counts of trees [tree_begin, tree_begin + tree_count) at the CSR entries
    (a, b), a < b (ustd_edge_counts).  Returns (counts int64[nnz], report)."""
    buf, nb = _ws(p, g, ws)
    dev = g.row_ptr.device
    if counts is None:
        counts = torch.zeros(g.nnz, dtype=torch.int64, device=dev)
    rep = Report()
    _check(lib().ustd_edge_counts(ctypes.byref(p), tree_begin, tree_count, _ptr(buf), nb, _ptr(counts),
                                  ctypes.byref(rep), _stream(dev)))
    return counts, rep.as_dict()


def edge_sample_size(n: int, m: int, eps: float, delta: float = 0.0) -> int:
    q = ctypes.c_int64(0)
    _check(lib().ustd_edge_sample_size(n, m, eps, delta, ctypes.byref(q)))
    return int(q.value)


def edge_resistances(g: Graph, counts: torch.Tensor, q: int, theta: float = 0.5):
    """Effective resistance and Kirchhoff-edge denominator 1 - (1 - theta) w(e) r(e) of every
    edge from spanning-edge counts of q trees (ustd_edge_resistances).  Returns (r, denom),
    float64[nnz] each, the edge's value at both of its CSR entries."""
    dev = g.row_ptr.device
    assert counts.dtype == torch.int64 and counts.numel() == g.nnz and counts.is_contiguous()
    r = torch.empty(g.nnz, dtype=torch.float64, device=dev)
    den = torch.empty_like(r)
    _check(lib().ustd_edge_resistances(g.n, g.nnz, _ptr(g.row_ptr), _ptr(g.col), _ptr(g.weight), _ptr(counts), q,
                                       theta, _ptr(r), _ptr(den), _stream(dev)))
    return r, den


def centralities(diag: torch.Tensor) -> dict:
    """Electrical farness and closeness, normalized random-walk betweenness and the Kirchhoff
    index from diag(L^+) (ustd_centralities)."""
    assert diag.dtype == torch.float64 and diag.is_cuda and diag.is_contiguous()
    n = diag.numel()
    dev = diag.device
    far = torch.empty(n, dtype=torch.float64, device=dev)
    clo = torch.empty_like(far)
    nrwb = torch.empty_like(far)
    sc = torch.empty(2, dtype=torch.float64, device=dev)
    _check(lib().ustd_centralities(n, _ptr(diag), _ptr(far), _ptr(clo), _ptr(nrwb), _ptr(sc), _stream(dev)))
    h = sc.cpu()
    return dict(farness=far, closeness=clo, nrwb=nrwb, trace=float(h[0]), kirchhoff=float(h[1]))


def philox_words(seed: int, t: int, s: int, k0: int, count: int, device="cuda") -> torch.Tensor:
    out = torch.empty(count, dtype=torch.int32, device=device)
    _check(lib().ustd_philox_words(seed & 0xFFFFFFFFFFFFFFFF, t, s, k0, count, _ptr(out), _stream(torch.device(device))))
    return out
