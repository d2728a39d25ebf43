"""Host-only checks of the C-ABI library: it loads, exports every entry point that
include/ustd.h declares, and its argument checks and workspace planner work without a GPU."""
import ctypes
import os
import re

import pytest

from paper_2006_13679_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ustd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ustd_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    assert declared_symbols() == sorted(api.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = api.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def _prob(**kw):
    base = dict(n=1024, nnz=3968, d_row_ptr=0x1000, d_col=0x2000, pivot=495, solve_mode=0, eps=0.3, delta=0.0,
                kappa=0.0, seed=1, tau_override=0, solve_tol=0.0, solve_maxit=0, validate=0, trees_per_batch=0,
                tau_cap=0)
    base.update(kw)
    return api.Problem(**base)


def test_workspace_bytes_host_only():
    b = api.workspace_bytes(_prob())
    assert b > 1024 * 16
    b2 = api.workspace_bytes(_prob(trees_per_batch=10))
    b3 = api.workspace_bytes(_prob(trees_per_batch=20))
    assert b2 < b3


@pytest.mark.parametrize("kw", [dict(pivot=1024), dict(pivot=-3), dict(eps=0.0), dict(eps=-1.0), dict(delta=1.5),
                                dict(kappa=1.0), dict(solve_mode=7), dict(n=1), dict(nnz=1), dict(d_col=0),
                                dict(trees_per_batch=100000)])
def test_invalid_arguments_rejected(kw):
    with pytest.raises(api.UstdError) as e:
        api.workspace_bytes(_prob(**kw))
    assert e.value.status == api.EINVAL


def test_status_strings():
    L = api.lib()
    assert L.ustd_status_string(0) == b"USTD_OK"
    assert L.ustd_status_string(5) == b"USTD_ENOTCONV"
    assert L.ustd_status_string(99) == b"USTD_UNKNOWN"


def test_weighted_workspace_single_and_batch():
    """Weights add the running row sums (nnz doubles) and three n-vectors, to a single problem's
    workspace and to that member's share of a batch workspace."""
    b0 = api.workspace_bytes(_prob())
    b1 = api.workspace_bytes(_prob(d_weight=0x3000))
    assert b1 - b0 >= 3968 * 8 + 3 * 1024 * 8

    def batch_bytes(*ps):
        arr = (api.Problem * len(ps))(*ps)
        size = ctypes.c_size_t(0)
        assert api.lib().ustd_batch_workspace_bytes(arr, len(ps), ctypes.byref(size)) == api.OK
        return size.value

    plain = batch_bytes(_prob(), _prob(seed=2))
    mixed = batch_bytes(_prob(), _prob(seed=2, d_weight=0x3000))
    assert mixed - plain >= 3968 * 8 + 3 * 1024 * 8


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the C structs' sizes and field offsets (a C program built from
    include/ustd.h prints them)."""
    import subprocess

    fields = {"ustd_problem": api.Problem, "ustd_report": api.Report, "ustd_batch_schedule": api.Schedule}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "ustd.h"', "int main(void) {"]
    for cname, cls in fields.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, cls in fields.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


@pytest.mark.parametrize("kw", [dict(group_fills=-2), dict(agg_chunk=5), dict(layout=2), dict(branches=5),
                                dict(branches=-1), dict(fill_trees=-3)])
def test_batch_plan_rejects_bad_schedules(kw):
    """The schedule is checked before anything touches a device: USTD_EINVAL and no plan."""
    arr = (api.Problem * 2)(_prob(), _prob(seed=2))
    plan = ctypes.c_void_p(None)
    rc = api.lib().ustd_batch_plan_create(arr, 2, ctypes.c_void_p(0x100000), 1 << 40,
                                          ctypes.byref(api.Schedule(**kw)), ctypes.byref(plan), None)
    assert rc == api.EINVAL and not plan.value
    assert api.lib().ustd_last_error()


def test_batch_plan_null_arguments():
    L = api.lib()
    assert L.ustd_batch_plan_create(None, 0, None, 0, None, None, None) == api.EINVAL
    assert L.ustd_batch_plan_destroy(None) == api.OK
    assert L.ustd_batch_graph_destroy(None) == api.OK
    assert L.ustd_batch_graph_launch(None, None) == api.EINVAL
    assert L.ustd_batch_plan_execute(None, None, None, None) == api.EINVAL
    assert L.ustd_batch_plan_reports(None, None, None) == api.EINVAL
    s = api.Schedule()
    assert L.ustd_batch_plan_schedule(None, ctypes.byref(s)) == api.EINVAL
    arr = (api.Problem * 1)(_prob())
    assert L.ustd_batch_autotune(arr, 1, None, 0, None, 1, None, None, None, None) == api.EINVAL


def test_batch_workspace_covers_every_layout():
    """One workspace size serves every schedule: the records layout (edge entries for every
    member) needs more than the LDS-bitmap layout for members that fit the bitmap."""
    arr = (api.Problem * 2)(_prob(tau_cap=64), _prob(seed=2, tau_cap=64))
    size = ctypes.c_size_t(0)
    assert api.lib().ustd_batch_workspace_bytes(arr, 2, ctypes.byref(size)) == api.OK
    single = api.workspace_bytes(_prob())
    assert size.value > 2 * 3968 * 16  # edge entries of both members
    assert size.value < 64 * single + (1 << 30)
