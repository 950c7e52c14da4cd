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


def test_bad_lanes_option_is_rejected_on_host():
    L = native.lib()
    for lanes in [3, 32, -1]:
        o = native.opts(lanes=lanes)
        st = L.nnls_solve_batch(10, 10, None, None, None, ctypes.byref(o), None, None)
        assert st == native.NMF_E_INVAL, lanes
    # one lane per column holds at most rank 32, two at most 64
    o = native.opts(lanes=1)
    assert L.nnls_solve_batch(33, 10, None, None, None, ctypes.byref(o), None, None) == native.NMF_E_INVAL
    with pytest.raises(native.NmfError):
        native.layout(65, 100, lanes=2)


def tuned_table():
    src = open(os.path.join(ROOT, "paper_1506_08938_amd", "csrc", "nqp_tuned.h")).read()
    ranks = [int(x) for x in re.search(r"kTunedRanks\[\] = \{([^}]*)\}", src).group(1).split(",")]
    cols = [int(x) for x in re.search(r"kTunedCols\[\] = \{([^}]*)\}", src).group(1).split(",")]
    body = re.search(r"kTunedLanes\[\d+\]\[\d+\] = \{(.*?)\};", src, re.S).group(1)
    rows = [[int(x) for x in row.split(",")] for row in re.findall(r"\{([^}]*)\}", body)]
    return ranks, cols, rows


@pytest.mark.parametrize("r", list(range(1, 129)))
def test_layout_covers_every_rank(r):
    # forced layouts: E * L covers r with the least padding the compiled table allows
    for lanes, emax in [(1, 32), (2, 32), (4, 32), (8, 16), (16, 8)]:
        if r > lanes * emax:
            continue
        E, L = native.layout(r, 1000, lanes)
        assert L == lanes and E * L >= r
        assert E * L - r < max(4 * L, 0.25 * r + L), (r, lanes, E)
    # automatic: a valid layout, never more lanes than coordinates
    for ncols in [0, 1, 300, 5000, 70000, 10 ** 6]:
        E, L = native.layout(r, ncols)
        assert L in (1, 2, 4, 8, 16) and E * L >= r
        assert L == 1 or L // 2 < r


def test_automatic_layout_follows_the_tuned_table():
    ranks, cols, rows = tuned_table()
    assert len(rows) == len(ranks) and all(len(x) == len(cols) for x in rows)
    def capped(L, r):  # never more lanes than coordinates
        while L > 1 and L // 2 >= r:
            L //= 2
        return L

    for i, r in enumerate(ranks):
        for j, c in enumerate(cols):
            E, L = native.layout(r, c)
            assert L == capped(rows[i][j], r), (r, c)
            # a launch size between two grid points takes the lower one's layout
            assert native.layout(r, c + 1) == (E, L)
            if j:
                assert native.layout(r, c - 1)[1] == capped(rows[i][j - 1], r)


def test_gather_probe_arguments_are_checked_on_host():
    L = native.lib()
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below fails its host checks
    assert L.nmf_probe_gather(None, 10, 16, fake, 4, fake, None) == native.NMF_E_INVAL
    assert L.nmf_probe_gather(fake, 10, 24, fake, 4, fake, None) == native.NMF_E_INVAL  # not a multiple of 16
    assert "multiple of 16" in native.last_error()
    assert L.nmf_probe_gather(fake, 0, 16, fake, 4, fake, None) == native.NMF_E_INVAL
    assert L.nmf_probe_gather(fake, 10, 16, fake, -1, fake, None) == native.NMF_E_INVAL
    assert L.nmf_probe_gather(fake, 10, 400, fake, 1 << 30, fake, None) == native.NMF_E_INVAL  # too much work


def test_dense_product_time_arguments_are_checked_on_host():
    L = native.lib()
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below fails its host checks
    ms = ctypes.c_double()
    ok = dict(m=64, n=64, ld=64, trans=1, r=32, prec=0, ns=0, reps=1)

    def call(**kw):
        a = dict(ok, **kw)
        return L.nmf_dense_product_time(fake, a["m"], a["n"], a["ld"], a["trans"], a["r"], fake, a["prec"], a["ns"],
                                        a["reps"], ctypes.byref(ms), None)
    assert L.nmf_dense_product_time(None, 64, 64, 64, 1, 32, fake, 0, 0, 1, ctypes.byref(ms), None) == native.NMF_E_INVAL
    for bad in [dict(trans=2), dict(r=0), dict(r=129), dict(prec=5), dict(ns=-1), dict(ns=513), dict(reps=0),
                dict(ld=10), dict(m=0)]:
        assert call(**bad) == native.NMF_E_INVAL, bad
