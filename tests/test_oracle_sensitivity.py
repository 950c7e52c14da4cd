"""The yardstick the GPU parity bounds are taken from (fp32_sensitivity.py):
the FP64 oracle's own spread under float32-sized disturbances.  These CPU
tests pin the helper (an undisturbed run is the oracle's fit bit for bit; the
disturbances have the stated sizes) and record the facts the bounds rest on."""
import numpy as np
import pytest
import scipy.sparse as sp

import fp32_sensitivity as fs
import oracle
from paper_1506_08938_amd import synth

FIXED = dict(max_inner=10, eps=0.0)


@pytest.mark.parametrize("sparse", [False, True])
def test_undisturbed_stepwise_fit_is_the_oracle_fit(sparse):
    g = np.random.default_rng(4)
    V = g.random((60, 45)) * (g.random((60, 45)) < (0.3 if sparse else 1.1))
    Vin = sp.csr_matrix(V) if sparse else V
    W0 = g.random((60, 6)); Ht0 = g.random((45, 6))
    reg = (0.01, 0.02, 0.05, 0.0)
    W, Ht = fs.stepwise_fit(Vin, 6, reg, W0, Ht0, 3, None, max_inner=20, eps=1e-3)
    o = oracle.nmf_fit(Vin, 6, reg, W0, Ht0, T=3, max_inner=20, eps=1e-3, want_trace=False)
    assert np.array_equal(W, o["W"]) and np.array_equal(Ht, o["Ht"])


def test_disturbances_have_the_stated_sizes():
    g = np.random.default_rng(0)
    a = g.random(200000) + 0.5
    # rounding to float32: relative change at most 2^-24
    d = np.abs(fs._round32(a) - a) / a
    assert d.max() <= 2.0 ** -24 and d.max() > 2.0 ** -26
    # the accumulation-error model: relative change u sqrt(k) z, z ~ N(0, 1),
    # then rounding
    k = 400
    j = (fs._jitter(a, k, np.random.default_rng(1)) - a) / a
    sd = 2.0 ** -24 * np.sqrt(k)
    assert abs(j.std() / sd - 1.0) < 0.02 and abs(j.mean()) < 0.02 * sd
    # one ulp up
    a32 = a.astype(np.float32)
    up = np.nextafter(a32, np.float32(np.inf))
    assert (up > a32).all() and np.all((up - a32) / a32 <= 2.0 ** -23)


def test_spread_facts_the_gpu_bounds_rest_on():
    """Workload 1 (dense 200 x 150, r = 10): from the random start and in
    adaptive mode float32-sized disturbances move the oracle's own objective
    by more than 1e-6, so no float32 computation can be held to 1e-6 there;
    the spread after 50 outer iterations is of order 1e-3 on the loss."""
    wl = synth.workload1()
    args = (wl["V"], wl["r"], wl["reg"])
    s0 = fs.spread(*args, wl["W0"], wl["Ht0"], 1, **FIXED)
    st = oracle.nmf_fit(*args, wl["W0"], wl["Ht0"], T=10, want_trace=False, max_inner=100, eps=1e-3)
    sa = fs.spread(*args, st["W"].astype(np.float32), st["Ht"].astype(np.float32), 1, max_inner=100, eps=1e-3)
    sl = fs.spread(*args, wl["W0"], wl["Ht0"], 50, seeds=range(1, 9), max_inner=100, eps=1e-3)
    print(f"workload 1 spread: one step from the start dJ {s0['dJ']:.2e}; adaptive step dJ {sa['dJ']:.2e}; "
          f"50 iterations loss {sl['dloss']:.2e}, kbar {sl['dkbar']:.2e}")
    for s in (s0, sa):
        assert s["dJ"] > 1e-6
    assert 1e-4 < sl["dloss"] < 1e-1 and sl["dkbar"] > 0
    # every disturbance leaves the objective finite and the factors nonnegative
    for mode in ("round", "ulp", "jitter"):
        W, Ht = fs.stepwise_fit(*args, wl["W0"], wl["Ht0"], 2, mode, seed=3, **FIXED)
        assert (W >= 0).all() and (Ht >= 0).all() and np.isfinite(oracle.objective(wl["V"], W, Ht, wl["reg"]))
