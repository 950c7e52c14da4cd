"""The limited-internal-memory fit (V in host memory, streamed in panels of
instances) against the FP64 oracle and against the resident fit, through
the C ABI."""
import numpy as np
import pytest

import fp32_sensitivity
import oracle
from paper_1506_08938_amd import synth

pytestmark = pytest.mark.gpu


def T(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def H(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def host(a, pinned=True):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    return t.pin_memory() if pinned else t


def f32(reg):
    return tuple(float(np.float32(x)) for x in reg)


def rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def streamed(V, r, reg, W0, Ht0, Tn, panel, pinned=True, want_trace=True, **kw):
    from paper_1506_08938_amd import native as nat
    Wd, Hd = T(W0), T(Ht0)
    tr, st = nat.fit_streamed(host(V, pinned), r, nat.reg(*reg), nat.opts(max_outer=Tn, **kw), Wd, Hd,
                              panel, want_trace=want_trace)
    return H(Wd), H(Hd), tr, st


FIXED = dict(max_inner=10, eps=0.0)


def problem():
    V = synth.dense_lowrank(400, 300, 16, 77, "gamma", 0.05)
    W0, Ht0 = synth.start_point(400, 300, 16, 78)
    return V, W0, Ht0


# One outer iteration from a common state (the oracle's after t_before
# iterations) against the oracle, for panels of one column, a ragged split,
# exactly n and more than n columns.  As for the resident fit, the objective
# and the factors are held to twice the oracle's own spread under
# float32-sized disturbances of the same step (fp32_sensitivity.py); from the
# converging state also to the 1e-6 of a float32 computation.
@pytest.mark.parametrize("panel", [1, 37, 300, 1000])
@pytest.mark.parametrize("t_before", [0, 10])
def test_streamed_step_matches_oracle(panel, t_before):
    V, W0, Ht0 = problem()
    reg = f32((0.05, 0.0, 0.1, 0.02))
    if t_before:
        o = oracle.nmf_fit(V, 16, reg, W0, Ht0, T=t_before, want_trace=False, **FIXED)
        W0, Ht0 = o["W"].astype(np.float32), o["Ht"].astype(np.float32)
    Wg, Hg, tr, _ = streamed(V, 16, reg, W0, Ht0, 1, panel, **FIXED)
    check_step_against_oracle(f"streamed panel={panel} after {t_before}", V, reg, W0, Ht0, Wg, Hg, tr, t_before)


def check_step_against_oracle(label, V, reg, W0, Ht0, Wg, Hg, tr, t_before):
    o = oracle.nmf_fit(V, 16, reg, W0, Ht0, T=1, **FIXED)
    S = fp32_sensitivity.spread(V, 16, reg, W0, Ht0, 1, **FIXED)
    Jg = oracle.objective(V, Wg, Hg, reg)
    Jo = oracle.objective(V, o["W"], o["Ht"], reg)
    J = abs(Jg - Jo) / Jo
    w, h = rel_fro(Wg, o["W"]), rel_fro(Hg, o["Ht"])
    lr = np.abs(tr - o["loss"]) / o["loss"]
    print(f"{label}: J rel {J:.2e} (spread {S['dJ']:.2e}) W {w:.2e} ({S['dW']:.2e}) Ht {h:.2e} "
          f"({S['dH']:.2e}) loss rel {lr.max():.2e}")
    assert lr[0] < 1e-12  # the start point's loss, summed panel by panel in FP64
    assert J <= 2 * S["dJ"] and w <= 2 * S["dW"] and h <= 2 * S["dH"]
    if t_before:
        assert J < 1e-6 and lr[1] < 1e-6


def test_streamed_follows_the_resident_fit():
    """Same iteration as nmf_fit; only the products' sums are grouped by
    panel.  From a converging state (the oracle's after 10 iterations) the
    two agree to the FP32 floor after one iteration and stay close over a
    few; from the random start the non-converged first solves amplify
    rounding, as between the GPU and the oracle (compared at 1e-2 there)."""
    from paper_1506_08938_amd import native as nat
    wl = synth.workload1()
    V, r, reg = wl["V"], wl["r"], wl["reg"]
    o = oracle.nmf_fit(V, r, reg, wl["W0"], wl["Ht0"], T=10, want_trace=False, **FIXED)
    W0, Ht0 = o["W"].astype(np.float32), o["Ht"].astype(np.float32)
    for Tn, tol_loss, tol_f in ((1, 2e-6, 1e-4), (4, 1e-4, 1e-3)):
        Wr, Hr = T(W0), T(Ht0)
        tr_r, st_r = nat.fit(nat.DeviceMatrix(T(V)), r, nat.reg(*reg), nat.opts(max_outer=Tn, **FIXED), Wr, Hr)
        Wg, Hg, tr, st = streamed(V, r, reg, W0, Ht0, Tn, 64, **FIXED)
        lr = np.abs(tr - tr_r) / tr_r
        w, h = rel_fro(Wg, H(Wr)), rel_fro(Hg, H(Hr))
        print(f"streamed vs resident, {Tn} iterations: loss max rel {lr.max():.2e}, W {w:.2e}, Ht {h:.2e}; "
              f"inner {st['inner_total']} vs {st_r['inner_total']}")
        assert lr[0] < 1e-12
        assert lr.max() < tol_loss and w < tol_f and h < tol_f
        assert st["inner_total"] == st_r["inner_total"]  # fixed-K: every column runs K iterations
    # from the random start, 5 iterations
    Wr, Hr = T(wl["W0"]), T(wl["Ht0"])
    tr_r, _ = nat.fit(nat.DeviceMatrix(T(V)), r, nat.reg(*reg), nat.opts(max_outer=5, **FIXED), Wr, Hr)
    _, _, tr, _ = streamed(V, r, reg, wl["W0"], wl["Ht0"], 5, 64, **FIXED)
    lr = np.abs(tr - tr_r) / tr_r
    print(f"streamed vs resident from the random start: loss rel {lr}")
    assert lr[1] < 1e-5 and lr.max() < 1e-2


def test_streamed_trace_stats_and_zero_iterations():
    wl = synth.workload1()
    V, r, reg = wl["V"], wl["r"], f32((0.01, 0.02, 0.03, 0.04))
    Wg, Hg, tr, st = streamed(V, r, reg, wl["W0"], wl["Ht0"], 6, 40, objective_every=3)
    assert np.isfinite(tr[[0, 3, 6]]).all() and np.isnan(tr[[1, 2, 4, 5]]).all()
    assert tr[0] == pytest.approx(oracle.loss(V, wl["W0"], wl["Ht0"]), rel=1e-12)
    assert st["loss"] == pytest.approx(oracle.loss(V, Wg, Hg), rel=1e-12)
    assert st["objective"] == pytest.approx(oracle.objective(V, Wg, Hg, reg), rel=1e-12)
    assert st["kkt_h"] >= 0 and st["kkt_w"] >= 0 and st["outer_done"] == 6
    # the three KKT conditions of the last half-iterations (the E-step's
    # gathered over the panels): the solve never leaves x >= 0, and on a zero
    # entry |min(x, g)| = max(0, -g), so the min-map residual bounds the third
    for k, mm in (("kkt_h_cond", "kkt_h"), ("kkt_w_cond", "kkt_w")):
        c = st[k]
        assert c[0] == 0.0 and c[1] >= 0.0 and c[2] >= 0.0 and np.isfinite(c).all()
        assert st[mm] >= c[2]
    assert st["kbar"] >= 1.0 and st["inner_total"] >= 6 * 350
    # no iterations: the start point's objective, factors untouched
    W0, Ht0 = wl["W0"], wl["Ht0"]
    Wz, Hz, trz, stz = streamed(V, r, reg, W0, Ht0, 0, 40)
    assert np.array_equal(Wz, W0.astype(np.float64)) and np.array_equal(Hz, Ht0.astype(np.float64))
    assert trz[0] == pytest.approx(oracle.loss(V, W0, Ht0), rel=1e-12)
    assert stz["loss"] == trz[0] and stz["outer_done"] == 0


def test_streamed_is_deterministic_pinned_or_not_and_with_a_leading_dimension():
    V, W0, Ht0 = problem()
    reg = (0.0, 0.01, 0.0, 0.01)
    a = streamed(V, 16, reg, W0, Ht0, 3, 64)
    b = streamed(V, 16, reg, W0, Ht0, 3, 64)
    c = streamed(V, 16, reg, W0, Ht0, 3, 64, pinned=False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    assert np.array_equal(a[2], c[2])
    # V as a column slice of a wider host array (leading dimension > n)
    from paper_1506_08938_amd import native as nat
    import torch
    wide = np.zeros((V.shape[0], V.shape[1] + 13), dtype=np.float32)
    wide[:, :V.shape[1]] = V
    Vw = torch.from_numpy(wide).pin_memory()[:, :V.shape[1]]
    Wd, Hd = T(W0), T(Ht0)
    tr, _ = nat.fit_streamed(Vw, 16, nat.reg(*reg), nat.opts(max_outer=3), Wd, Hd, 64)
    assert np.array_equal(H(Wd), a[0]) and np.array_equal(H(Hd), a[1]) and np.array_equal(tr, a[2])


def test_streamed_fast_break_runs_within_panels():
    """The fast-break over runs that never cross a panel: with panels a
    multiple of the run length the runs are those of the resident fit.
    Compared from a converging state, where the adaptive stopping rule is
    least sensitive to rounding (a flipped iteration count moves a column by
    O(sqrt(eps)))."""
    from paper_1506_08938_amd import native as nat
    V, W0, Ht0 = problem()
    reg = f32((0.0, 0.0, 0.05, 0.0))
    o = oracle.nmf_fit(V, 16, reg, W0, Ht0, T=10, want_trace=False, **FIXED)
    W0, Ht0 = o["W"].astype(np.float32), o["Ht"].astype(np.float32)
    fb = dict(max_inner=50, eps=1e-3, fast_break_cols=8, lanes=4)
    Wr, Hr = T(W0), T(Ht0)
    tr_r, st_r = nat.fit(nat.DeviceMatrix(T(V)), 16, nat.reg(*reg), nat.opts(max_outer=2, **fb), Wr, Hr)
    Wg, Hg, tr, st = streamed(V, 16, reg, W0, Ht0, 2, 64, **fb)
    _, _, _, st_plain = streamed(V, 16, reg, W0, Ht0, 2, 64, max_inner=50, eps=1e-3, lanes=4)
    lr = np.abs(tr - tr_r) / tr_r
    print(f"streamed fast-break: loss max rel {lr.max():.2e}; inner {st['inner_total']} vs resident "
          f"{st_r['inner_total']} (no fast-break {st_plain['inner_total']})")
    assert lr.max() < 1e-4
    assert abs(st["inner_total"] - st_r["inner_total"]) <= 0.02 * st_r["inner_total"]
    assert st["inner_total"] <= st_plain["inner_total"]


def test_streamed_rejects_bad_arguments():
    from paper_1506_08938_amd import native as nat
    V, W0, Ht0 = problem()
    reg = nat.reg()
    with pytest.raises(nat.NmfError) as ei:
        nat.fit_streamed(host(V), 16, reg, nat.opts(precision=nat.NMF_BF16), T(W0), T(Ht0), 64)
    assert ei.value.status == nat.NMF_E_UNSUPPORTED
    with pytest.raises(nat.NmfError) as ei:
        nat.fit_streamed(host(V), 16, reg, nat.opts(), T(W0), T(Ht0), 0)
    assert ei.value.status == nat.NMF_E_INVAL
    bad = V.copy()
    bad[123, 45] = -1.0
    with pytest.raises(nat.NmfError) as ei:
        nat.fit_streamed(host(bad), 16, reg, nat.opts(max_outer=1, check_finite=1), T(W0), T(Ht0), 64)
    assert ei.value.status == nat.NMF_E_NONFINITE
    bad[123, 45] = np.nan
    with pytest.raises(nat.NmfError) as ei:
        nat.fit_streamed(host(bad), 16, reg, nat.opts(max_outer=1, check_finite=1), T(W0), T(Ht0), 64)
    assert ei.value.status == nat.NMF_E_NONFINITE


# --------------------------------------------------------------------------- single pass, resident V
def single_pass(Vd, r, reg, W0, Ht0, Tn, panel, **kw):
    from paper_1506_08938_amd import native as nat
    Wd, Hd = T(W0), T(Ht0)
    tr, st = nat.fit_single_pass(Vd, r, nat.reg(*reg), nat.opts(max_outer=Tn, **kw), Wd, Hd, panel)
    return H(Wd), H(Hd), tr, st


# The same panels as the streamed fit, read in place from device memory: the
# same kernels on the same panels (the products do not depend on the leading
# dimension), so the results equal the streamed fit's bitwise.
@pytest.mark.parametrize("panel", [1, 37, 300, 1000])
@pytest.mark.parametrize("adaptive", [False, True])
def test_single_pass_equals_streamed(panel, adaptive):
    from paper_1506_08938_amd import native as nat
    V, W0, Ht0 = problem()
    reg = f32((0.05, 0.01, 0.1, 0.02))
    kw = dict(max_inner=100, eps=1e-3) if adaptive else FIXED
    a = streamed(V, 16, reg, W0, Ht0, 3, panel, **kw)
    b = single_pass(nat.DeviceMatrix(T(V)), 16, reg, W0, Ht0, 3, panel, **kw)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
    assert a[3]["inner_total"] == b[3]["inner_total"] and a[3]["loss"] == b[3]["loss"]
    assert a[3]["kkt_h_cond"] == b[3]["kkt_h_cond"] and a[3]["kkt_w"] == b[3]["kkt_w"]


@pytest.mark.parametrize("t_before", [0, 10])
def test_single_pass_step_matches_oracle(t_before):
    from paper_1506_08938_amd import native as nat
    V, W0, Ht0 = problem()
    reg = f32((0.05, 0.0, 0.1, 0.02))
    if t_before:
        o = oracle.nmf_fit(V, 16, reg, W0, Ht0, T=t_before, want_trace=False, **FIXED)
        W0, Ht0 = o["W"].astype(np.float32), o["Ht"].astype(np.float32)
    Wg, Hg, tr, _ = single_pass(nat.DeviceMatrix(T(V)), 16, reg, W0, Ht0, 1, 37, **FIXED)
    check_step_against_oracle(f"single pass after {t_before}", V, reg, W0, Ht0, Wg, Hg, tr, t_before)


def test_single_pass_leading_dimension_and_arguments():
    from paper_1506_08938_amd import native as nat
    V, W0, Ht0 = problem()
    reg = (0.0, 0.01, 0.0, 0.01)
    a = single_pass(nat.DeviceMatrix(T(V)), 16, reg, W0, Ht0, 3, 64)
    wide = np.zeros((V.shape[0], V.shape[1] + 13), dtype=np.float32)
    wide[:, :V.shape[1]] = V
    b = single_pass(nat.DeviceMatrix(T(wide)[:, :V.shape[1]]), 16, reg, W0, Ht0, 3, 64)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    Vd = nat.DeviceMatrix(T(V))
    with pytest.raises(nat.NmfError) as ei:
        single_pass(Vd, 16, reg, W0, Ht0, 1, 64, precision=nat.NMF_BF16)
    assert ei.value.status == nat.NMF_E_UNSUPPORTED
    with pytest.raises(nat.NmfError) as ei:
        single_pass(Vd, 16, reg, W0, Ht0, 1, 0)
    assert ei.value.status == nat.NMF_E_INVAL
    import scipy.sparse as sp
    with pytest.raises(nat.NmfError) as ei:
        single_pass(nat.DeviceMatrix(sp.csr_matrix(V)), 16, reg, W0, Ht0, 1, 64)
    assert ei.value.status == nat.NMF_E_UNSUPPORTED
