"""The C-ABI library loads on the CPU and exports every entry point
include/nmf.h declares; argument errors are caught on the host before any
device call (so they can be checked without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1506_08938_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"NMF_API\s+[\w\s\*]*?\b((?:nmf|nnls)_\w+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_entry_point():
    L = native.lib()
    declared = declared_entry_points()
    assert declared, "no NMF_API declarations found"
    for name in declared:
        assert hasattr(L, name), f"{name} declared in include/ but not exported"
    assert sorted(native.EXPORTS) == declared


def test_default_opts():
    o = native.opts()
    assert (o.max_outer, o.max_inner, o.eps, o.ls_guard, o.precision) == (50, 100, 1e-3, 1, 0)


@pytest.mark.parametrize("r", [0, -1, 129])
def test_rank_out_of_range_is_rejected_on_host(r):
    L = native.lib()
    o = native.opts()
    st = L.nnls_solve_batch(r, 10, None, None, None, ctypes.byref(o), None, None)
    assert st == native.NMF_E_INVAL
    assert "r must be in" in native.last_error()


def test_bad_options_are_rejected_on_host():
    L = native.lib()
    for kw in [dict(max_inner=0), dict(eps=-1.0), dict(eps=float("nan")), dict(precision=7)]:
        o = native.opts(**kw)
        st = L.nnls_solve_batch(10, 10, None, None, None, ctypes.byref(o), None, None)
        assert st == native.NMF_E_INVAL, kw


def test_null_pointers_are_rejected_and_empty_batch_is_a_noop():
    L = native.lib()
    o = native.opts()
    assert L.nnls_solve_batch(10, 5, None, None, None, ctypes.byref(o), None, None) == native.NMF_E_INVAL
    assert L.nnls_solve_batch(10, 0, None, None, None, ctypes.byref(o), None, None) == native.NMF_OK
