"""Pins for the FP64 oracle, each against something other than the oracle:
the paper's worked example, closed forms, brute force, Lawson-Hanson NNLS
(scipy), numpy/scipy products, and invariants the paper states.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import scipy.sparse as sp

import oracle
from paper_1506_08938_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def f_val(H, h, x):
    return 0.5 * x @ H @ x + h @ x


def random_nqp(r, seed, k=None, l1=0.0, l2=0.0):
    g = np.random.default_rng(seed)
    k = k or 3 * r
    A = g.random((k, r))
    b = g.random(k) * r * 0.3
    H = A.T @ A + 2 * l2 * np.eye(r)
    h = -A.T @ b + l1
    return A, b, H, h


def brute_force_nqp(H, h):
    """Enumerate every passive set S: solve H_SS x_S = -h_S and keep the
    point that satisfies x >= 0 and grad >= 0 off S (the KKT conditions)."""
    r = len(h)
    best, bx = np.inf, None
    for mask in itertools.product([0, 1], repeat=r):
        S = np.array(mask, dtype=bool)
        x = np.zeros(r)
        if S.any():
            x[S] = np.linalg.solve(H[np.ix_(S, S)], -h[S])
        if (x < -1e-12).any():
            continue
        gr = H @ x + h
        if (gr[~S] < -1e-9).any():
            continue
        fv = f_val(H, h, x)
        if fv < best:
            best, bx = fv, x
    return bx


def lawson_hanson_nqp(H, h):
    """min 0.5x'Hx + h'x, x >= 0, as NNLS: H = LL' gives
    0.5||L'x + L^-1 h||^2 + const, solved by scipy's Lawson-Hanson."""
    L = np.linalg.cholesky(H)
    c = scipy.linalg.solve_triangular(L, -h, lower=True)
    x, _ = scipy.optimize.nnls(L.T, c, maxiter=50 * len(h))
    return x


# --------------------------------------------------------------------------- worked example
def test_worked_example_rescale_matches_eq_nqpi():
    ex = json.load(open(os.path.join(GOLD, "worked_example.json")))
    Q, d, fr = oracle.rescale(ex["H"])
    assert not fr.any()
    assert Q[0, 1] == pytest.approx(ex["rescaled_Q_offdiag"], rel=1e-15)
    assert np.allclose(np.diag(Q), 1.0)
    q = np.array(ex["h"]) / d
    assert np.allclose(q, ex["rescaled_q"], rtol=1e-15)


def test_worked_example_unscaled_line_search_takes_59_steps():
    ex = json.load(open(os.path.join(GOLD, "worked_example.json")))
    H = np.array(ex["H"]); h = np.array(ex["h"])
    first = None
    for K in range(1, 80):
        x, k = oracle.nqp(H, h, ex["x0"], max_inner=K, eps=0.0, ls_guard=0,
                          flags=oracle.NO_RESCALE | oracle.NO_CD)
        assert k == K
        if np.linalg.norm(H @ x + h) < 1e-3:
            first = K
            break
    assert first == ex["unscaled_line_search_iterations"]


def test_worked_example_rescaled_method_needs_one_iteration():
    ex = json.load(open(os.path.join(GOLD, "worked_example.json")))
    H = np.array(ex["H"]); h = np.array(ex["h"]); xs = np.array(ex["x_star"])
    # the closed-form optimum of the fixture is the interior stationary point
    assert np.allclose(np.linalg.solve(H, -h), xs, rtol=1e-14)
    assert f_val(H, h, xs) == pytest.approx(ex["f_star"], rel=1e-14)
    x, k = oracle.nqp(H, h, ex["x0"], max_inner=100, eps=1e-7)
    assert k == ex["rescaled_iterations"]
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 2e-4
    assert f_val(H, h, x) - ex["f_star"] < 1e-3
    # and it converges to the optimum with more iterations
    x, k = oracle.nqp(H, h, ex["x0"], max_inner=10, eps=0.0)
    assert np.allclose(x, xs, rtol=1e-12)


def _first_iteration_2d_decimal(H, h, x0):
    """The first iteration of Algorithm 3 on a 2-variable NQP, written out for
    two variables in 50-digit decimal arithmetic (independent of the oracle's
    code): rescale to unit diagonal, the exact projected line search with the
    guard, two greedy coordinate steps (lowest index on ties), the projected
    gradient norms before and after, and the unscaled point."""
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 50
        Hd = [[Decimal(repr(float(v))) for v in row] for row in H]
        hd = [Decimal(repr(float(v))) for v in h]
        sq = [Hd[0][0].sqrt(), Hd[1][1].sqrt()]
        off = Hd[0][1] / (sq[0] * sq[1])
        Q = [[Decimal(1), off], [off, Decimal(1)]]
        q = [hd[0] / sq[0], hd[1] / sq[1]]
        y = [Decimal(repr(float(x0[0]))) * sq[0], Decimal(repr(float(x0[1]))) * sq[1]]

        def mv(v):
            return [Q[0][0] * v[0] + Q[0][1] * v[1], Q[1][0] * v[0] + Q[1][1] * v[1]]

        def pgrad(y, g):
            return [gi if (yi > 0 or gi < 0) else Decimal(0) for yi, gi in zip(y, g)]

        g = [a + b for a, b in zip(mv(y), q)]
        pg = pgrad(y, g)
        n0 = pg[0] ** 2 + pg[1] ** 2
        u = mv(pg)
        alpha = n0 / (pg[0] * u[0] + pg[1] * u[1])
        step = [max(Decimal(0), yi - alpha * gi) - yi for yi, gi in zip(y, pg)]
        w = mv(step)
        if g[0] * step[0] + g[1] * step[1] + (step[0] * w[0] + step[1] * w[1]) / 2 <= 0:
            y = [a + b for a, b in zip(y, step)]
            g = [a + b for a, b in zip(g, w)]
        for _ in range(2):
            cand = []
            for i in range(2):
                delta = max(Decimal(0), y[i] - g[i]) - y[i]
                cand.append((abs(g[i] * delta + delta * delta / 2), i, delta))
            dec, p, delta = max(cand, key=lambda c: (c[0], -c[1]))
            if not dec > 0:
                break
            g = [g[0] + Q[0][p] * delta, g[1] + Q[1][p] * delta]
            y[p] += delta
        pg = pgrad(y, g)
        n1 = pg[0] ** 2 + pg[1] ** 2
        return [float(y[0] / sq[0]), float(y[1] / sq[1])], float(n1 / n0)


def test_worked_example_first_iteration_point():
    # Section 3.4's example: one iteration of Algorithm 3 (under the readings
    # of the stopping quantity, the CD count and the tie rule) reaches
    # x = (79.08014973, 9.19850272) with f - f* = 5.73e-4 and
    # ||f~_1||^2 / ||f~_0||^2 = 7.0e-8, so it stops after one iteration for any
    # eps >= 7.01e-8 -- the paper's "only one iteration".
    ex = json.load(open(os.path.join(GOLD, "worked_example.json")))
    H = np.array(ex["H"]); h = np.array(ex["h"])
    xd, ratio_d = _first_iteration_2d_decimal(H, h, ex["x0"])
    assert xd == pytest.approx([79.08014973, 9.19850272], rel=1e-9)
    assert ratio_d == pytest.approx(7.008e-8, rel=1e-3)
    x, k = oracle.nqp(H, h, ex["x0"], max_inner=1, eps=0.0)
    assert k == 1
    assert np.allclose(x, xd, rtol=1e-12)
    assert np.allclose(x, [79.08014973, 9.19850272], rtol=1e-8)
    assert f_val(H, h, x) - ex["f_star"] == pytest.approx(5.73e-4, rel=2e-3)
    _, _, nk = oracle.nqp_trace(H, h, ex["x0"], max_inner=1, eps=0.0)
    assert nk[1] / nk[0] == pytest.approx(ratio_d, rel=1e-9)
    # the accelerated stopping rule: one iteration for eps just above the
    # ratio, two just below it
    assert oracle.nqp(H, h, ex["x0"], max_inner=100, eps=7.01e-8)[1] == 1
    assert oracle.nqp(H, h, ex["x0"], max_inner=100, eps=6.99e-8)[1] == 2


# --------------------------------------------------------------------------- closed forms
@pytest.mark.parametrize("seed", range(6))
def test_r1_closed_form_in_one_iteration(seed):
    g = np.random.default_rng(seed)
    a = g.random(20); b = g.random(20) * (2.0 if seed % 2 else -1.0)
    l1 = [0.0, 0.3][seed % 2]; l2 = [0.0, 0.1][(seed // 2) % 2]
    H = np.array([[a @ a + 2 * l2]]); h = np.array([-a @ b + l1])
    x, k = oracle.nqp(H, h, [g.random() * 3], max_inner=50, eps=1e-12)
    assert k == 1
    assert x[0] == pytest.approx(max(0.0, (a @ b - l1) / (a @ a + 2 * l2)), rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("r", [3, 17, 128])
def test_orthogonal_columns_closed_form(r):
    inst = synth.nqp_instance(r, 4, seed=r, kind="orthogonal")
    A = inst["A"].astype(np.float64); B = inst["B"].astype(np.float64)
    H = A.T @ A
    assert np.count_nonzero(H - np.diag(np.diag(H))) == 0
    for j in range(4):
        h = -A.T @ B[:, j] + 0.05
        x, k = oracle.nqp(H, h, inst["x0"][j], max_inner=5, eps=1e-12)
        assert k == 1
        assert np.allclose(x, np.maximum(0.0, -h) / np.diag(H), rtol=1e-13, atol=1e-300)


# --------------------------------------------------------------------------- brute force / library
@pytest.mark.parametrize("r", [2, 3, 5, 8])
@pytest.mark.parametrize("seed", range(4))
def test_converged_matches_brute_force(r, seed):
    A, b, H, h = random_nqp(r, 100 * r + seed, l1=0.2 * (seed % 2), l2=0.05 * (seed // 2))
    xs = brute_force_nqp(H, h)
    x, _ = oracle.nqp(H, h, np.random.default_rng(seed).random(r), max_inner=2000, eps=0.0)
    assert np.allclose(x, xs, rtol=1e-9, atol=1e-9 * np.abs(xs).max())


@pytest.mark.parametrize("r", [16, 64, 100])
def test_converged_matches_lawson_hanson(r):
    A, b, H, h = random_nqp(r, 7 + r, l1=0.01, l2=0.01)
    xs = lawson_hanson_nqp(H, h)
    x, _ = oracle.nqp(H, h, np.zeros(r), max_inner=20000, eps=0.0)
    assert np.allclose(x, xs, rtol=1e-7, atol=1e-8 * np.abs(xs).max())
    assert f_val(H, h, x) <= f_val(H, h, xs) + 1e-10 * abs(f_val(H, h, xs))


def test_kkt_residual_vanishes_at_convergence():
    A, b, H, h = random_nqp(40, 3, l1=0.05)
    x, _ = oracle.nqp(H, h, np.ones(40), max_inner=5000, eps=0.0)
    gr = H @ x + h
    assert (x >= 0).all()
    assert np.abs(np.minimum(x, gr)).max() < 1e-10 * max(1.0, np.abs(h).max())
    res = oracle.kkt(H, (-h)[None, :], 0.0, x[None, :])
    assert res[0] == pytest.approx(np.abs(np.minimum(x, gr)).max(), abs=1e-12)


def test_kkt_reports_each_condition_separately():
    # With Gamma = I the gradient of column j is g = x - P_j + l1, so choosing
    # P = x + l1 - g plants any gradient.  Values are dyadic (exact in FP64).
    G = np.eye(3)
    l1 = 0.25
    X = np.array([[1.5, 0.0, -0.375],     # a negative entry (nonnegativity)
                  [2.0, 0.0, 0.0],        # g = 0.5 on a positive entry (complementarity)
                  [0.0, 0.0, 0.5]])       # g = -0.75 on a zero entry
    g = np.array([[0.0, 0.125, 0.0],
                  [0.5, 1.0, 0.0],
                  [-0.75, 0.0, 0.0]])
    P = X + l1 - g
    res = oracle.kkt(G, P, l1, X)
    assert res[0] == 0.75                  # max |min(x, g)|: the zero entry with g = -0.75
    assert res[1] == 0.375                 # max(0, -min x)
    assert res[2] == 1.0                   # max x |g| = 2.0 * 0.5
    assert res[3] == 0.75                  # max(0, -min g over x == 0)
    # at a converged solution every condition holds to rounding
    A, b, H, h = random_nqp(30, 11, l1=0.05)
    xs = lawson_hanson_nqp(H, h)
    xs = np.maximum(xs, 0.0)
    xo, _ = oracle.nqp(H, h, np.ones(30), max_inner=5000, eps=0.0)
    for x in (xs, xo):
        res = oracle.kkt(H, (-h)[None, :], 0.0, x[None, :])
        scale = max(1.0, np.abs(h).max())
        assert res[1] == 0.0
        assert res[2] < 1e-9 * scale * max(1.0, x.max())
        assert res[3] < 1e-9 * scale


# --------------------------------------------------------------------------- invariants
@pytest.mark.parametrize("seed", range(5))
def test_rescale_invariants(seed):
    r = 5 + 7 * seed
    A, b, H, h = random_nqp(r, seed)
    Q, d, fr = oracle.rescale(H)
    assert np.array_equal(np.diag(Q), np.ones(r))
    assert np.abs(Q).max() <= 1.0 + 1e-15
    nf = np.linalg.norm(Q)
    assert np.sqrt(r) - 1e-12 <= nf <= r + 1e-12
    # f(x) = f_hat(y) with y = x * sqrt(diag H), q = h / sqrt(diag H)
    x = np.random.default_rng(seed).random(r)
    y = x * d; q = h / d
    assert f_val(H, h, x) == pytest.approx(f_val(Q, q, y), rel=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_objective_non_increasing_with_guard(seed):
    r = [2, 3, 4, 6, 10, 20, 40, 64][seed]
    A, b, H, h = random_nqp(r, 50 + seed, l1=0.1 * (seed % 3))
    Q, d, fr = oracle.rescale(H)
    x0 = np.random.default_rng(seed).random(r) * 3
    x, k, fk = oracle.nqp(H, h, x0, max_inner=30, eps=0.0, trace=True)
    assert np.all(np.diff(fk) <= 1e-12 * np.abs(fk).max())
    # coordinate-descent steps alone are exact coordinate minimisations
    x, k, fk = oracle.nqp(H, h, x0, max_inner=30, eps=0.0, flags=oracle.NO_LS, trace=True)
    assert np.all(np.diff(fk) <= 1e-12 * np.abs(fk).max())
    # the traced objective is f of the returned point
    assert fk[-1] == pytest.approx(f_val(H, h, x), rel=1e-10, abs=1e-10)


def test_literal_line_search_can_raise_f_and_guard_rejects_it():
    # Q has unit diagonal, so y = x; y = (0.01, 1), grad = (1, -1)
    H = np.array([[1.0, 0.9], [0.9, 1.0]]); h = np.array([0.09, -2.009]); x0 = np.array([0.01, 1.0])
    assert np.allclose(H @ x0 + h, [1.0, -1.0])
    f0 = f_val(H, h, x0)
    x, k = oracle.nqp(H, h, x0, max_inner=1, eps=0.0, ls_guard=0, flags=oracle.NO_CD)
    assert f_val(H, h, x) > f0 + 30.0  # -1.499 -> 38.40
    assert f0 == pytest.approx(-1.49905, abs=1e-5)
    assert f_val(H, h, x) == pytest.approx(38.40, abs=5e-3)
    x, k = oracle.nqp(H, h, x0, max_inner=1, eps=0.0, ls_guard=1, flags=oracle.NO_CD)
    assert np.array_equal(x, x0)


def test_zero_column_is_frozen_at_zero():
    inst = synth.nqp_instance(6, 3, seed=9, kind="zerocol")
    A = inst["A"].astype(np.float64); B = inst["B"].astype(np.float64)
    H = A.T @ A
    for j in range(3):
        h = -A.T @ B[:, j] + 0.1
        x, _ = oracle.nqp(H, h, inst["x0"][j], max_inner=3000, eps=0.0)
        assert x[0] == 0.0
        xs = brute_force_nqp(H[1:, 1:], h[1:])
        assert np.allclose(x[1:], xs, rtol=1e-9, atol=1e-12)


def test_singular_gram_reaches_optimal_value():
    inst = synth.nqp_instance(5, 2, seed=4, kind="dupcol")
    A = inst["A"].astype(np.float64); B = inst["B"].astype(np.float64)
    H = A.T @ A
    h = -A.T @ B[:, 0]
    x, _ = oracle.nqp(H, h, inst["x0"][0], max_inner=5000, eps=0.0)
    xs, _ = scipy.optimize.nnls(A, B[:, 0])
    assert f_val(H, h, x) == pytest.approx(f_val(H, h, xs), rel=1e-9)


def test_stopping_rule_and_repeat_until():
    A, b, H, h = random_nqp(12, 1)
    # the accelerated condition with a loose eps stops early, tight eps later
    _, k_loose = oracle.nqp(H, h, np.ones(12), max_inner=500, eps=1e-1)
    _, k_tight = oracle.nqp(H, h, np.ones(12), max_inner=500, eps=1e-12)
    assert 1 <= k_loose < k_tight
    # an exactly optimal start (x0 = 0 with h >= 0: zero projected gradient)
    # still runs one iteration and stays put
    x, k = oracle.nqp(H, np.abs(h), np.zeros(12), max_inner=50, eps=1e-3)
    assert k == 1 and np.array_equal(x, np.zeros(12))
    # eps = 0 runs exactly max_inner iterations
    _, k = oracle.nqp(H, h, np.ones(12), max_inner=7, eps=0.0)
    assert k == 7


# --------------------------------------------------------------------------- products / losses
def test_gram_and_products_match_numpy_and_scipy():
    g = np.random.default_rng(0)
    V = g.random((37, 23)); W = g.random((37, 5)); Ht = g.random((23, 5))
    assert np.allclose(oracle.gram(W, 0.25), W.T @ W + 0.5 * np.eye(5), rtol=1e-14)
    assert np.allclose(oracle.product_dense(V, W, 0), (W.T @ V).T, rtol=1e-14)
    assert np.allclose(oracle.product_dense(V, Ht, 1), V @ Ht, rtol=1e-14)
    S = sp.random(37, 23, density=0.2, random_state=1, format="csr")
    assert np.allclose(oracle.product_csr(S, W, 0), S.T @ W, rtol=1e-14)
    assert np.allclose(oracle.product_csr(S, Ht, 1), S @ Ht, rtol=1e-14)


def test_losses_and_objective():
    g = np.random.default_rng(1)
    S = sp.random(40, 30, density=0.3, random_state=2, format="csr")
    W = g.random((40, 4)); Ht = g.random((30, 4))
    direct = 0.5 * np.sum((S.toarray() - W @ Ht.T) ** 2)
    assert oracle.loss(S.toarray(), W, Ht) == pytest.approx(direct, rel=1e-13)
    assert oracle.loss(S, W, Ht) == pytest.approx(direct, rel=1e-11)
    reg = (0.1, 0.2, 0.3, 0.4)
    J = direct + 0.3 * Ht.sum() + 0.4 * (Ht ** 2).sum() + 0.1 * W.sum() + 0.2 * (W ** 2).sum()
    assert oracle.objective(S, W, Ht, reg) == pytest.approx(J, rel=1e-11)


# --------------------------------------------------------------------------- NMF loop
def _exact_half(A, Bcols, l1, l2):
    """Every column's NQP solved exactly by Lawson-Hanson (independent path)."""
    H = A.T @ A + 2 * l2 * np.eye(A.shape[1])
    return np.stack([lawson_hanson_nqp(H, -A.T @ Bcols[:, j] + l1) for j in range(Bcols.shape[1])])


@pytest.mark.parametrize("sparse", [False, True])
def test_one_outer_iteration_with_exact_inner_solves_matches_lawson_hanson(sparse):
    g = np.random.default_rng(5)
    m, n, r = 30, 22, 4
    V = g.random((m, n)) * (g.random((m, n)) < (0.5 if sparse else 1.1))
    reg = (0.02, 0.03, 0.05, 0.01)  # l1_w, l2_w, l1_h, l2_h
    W0 = g.random((m, r)); Ht0 = g.random((n, r))
    Vin = sp.csr_matrix(V) if sparse else V
    out = oracle.nmf_fit(Vin, r, reg, W0, Ht0, T=1, max_inner=20000, eps=0.0)
    # E-step first (W fixed, columns of V), then the M-step with the new H
    Ht1 = _exact_half(W0, V, reg[2], reg[3])
    W1 = _exact_half(Ht1, V.T, reg[0], reg[1])
    assert np.allclose(out["Ht"], Ht1, rtol=1e-7, atol=1e-9)
    assert np.allclose(out["W"], W1, rtol=1e-7, atol=1e-9)


def test_rank_one_nmf_closed_form():
    g = np.random.default_rng(6)
    V = g.random((15, 12)); w = g.random((15, 1)); ht = g.random((12, 1))
    reg = (0.1, 0.05, 0.2, 0.0)
    out = oracle.nmf_fit(V, 1, reg, w, ht, T=1, max_inner=10, eps=0.0)
    h1 = np.maximum(0.0, (V.T @ w[:, 0] - reg[2]) / (w[:, 0] @ w[:, 0] + 2 * reg[3]))
    w1 = np.maximum(0.0, (V @ h1 - reg[0]) / (h1 @ h1 + 2 * reg[1]))
    assert np.allclose(out["Ht"][:, 0], h1, rtol=1e-13)
    assert np.allclose(out["W"][:, 0], w1, rtol=1e-13)


def test_regularised_objective_non_increasing_per_half():
    wl = synth.workload1()
    reg = (0.01, 0.02, 0.05, 0.01)
    out = oracle.nmf_fit(wl["V"], wl["r"], reg, wl["W0"], wl["Ht0"], T=8, max_inner=100, eps=1e-3)
    jh = out["jhalf"]
    assert np.all(np.diff(jh) <= 1e-12 * jh[0])
    assert out["inner"].min() >= wl["V"].shape[1]  # at least one iteration per column


def test_dense_and_csr_fits_agree():
    g = np.random.default_rng(8)
    V = g.random((40, 30)) * (g.random((40, 30)) < 0.3)
    W0 = g.random((40, 5)); Ht0 = g.random((30, 5))
    reg = (0.0, 0.01, 0.1, 0.0)
    a = oracle.nmf_fit(V, 5, reg, W0, Ht0, T=5, max_inner=50, eps=1e-3)
    b = oracle.nmf_fit(sp.csr_matrix(V), 5, reg, W0, Ht0, T=5, max_inner=50, eps=1e-3)
    assert np.allclose(a["W"], b["W"], rtol=1e-9, atol=1e-12)
    assert np.allclose(a["Ht"], b["Ht"], rtol=1e-9, atol=1e-12)
    assert np.allclose(a["loss"], b["loss"], rtol=1e-9)


def test_workload1_fit_converges_and_is_deterministic():
    wl = synth.workload1()
    a = oracle.nmf_fit(wl["V"], wl["r"], wl["reg"], wl["W0"], wl["Ht0"], T=wl["T"])
    b = oracle.nmf_fit(wl["V"], wl["r"], wl["reg"], wl["W0"], wl["Ht0"], T=wl["T"])
    assert np.array_equal(a["W"], b["W"]) and np.array_equal(a["loss"], b["loss"])
    vv = 0.5 * np.sum(wl["V"].astype(np.float64) ** 2)
    assert a["loss"][-1] < 1e-3 * vv
    assert np.all(np.diff(a["loss"]) <= 1e-12 * vv)
    kbar = a["inner"].sum() / (wl["T"] * sum(wl["V"].shape))
    assert 1.0 <= kbar < 20.0


# ---------------------------------------------------------------------------
# Fast-break of Algorithm 3 (the maxStop condition), over fixed chunks of
# consecutive columns ("threads of computation"; maxStop reset per half).

def _faststop_instance(r=12, ncols=61, seed=41):
    inst = synth.nqp_instance(r, ncols, seed=seed, l1=0.02)
    A = inst["A"].astype(np.float64); B = inst["B"].astype(np.float64)
    return A.T @ A, -(B.T @ A) + 0.02, inst["x0"].astype(np.float64)


def test_faststop_with_one_column_chunks_is_the_plain_solver():
    # maxStop starts at 0 in every chunk, so a one-column chunk never fast-breaks
    G, h, x0 = _faststop_instance()
    xa, ia = oracle.nqp_batch(G, h, x0, max_inner=40, eps=1e-5)
    xb, ib, _ = oracle.nqp_batch_faststop(G, h, x0, chunk=1, max_inner=40, eps=1e-5)
    assert np.array_equal(xa, xb) and np.array_equal(ia, ib)


@pytest.mark.parametrize("chunk", [4, 16, 61])
def test_faststop_follows_the_rule_on_each_columns_own_trace(chunk):
    # The fast-break only truncates a column's iterations.  From each column's
    # plain trace of ||f~_k||^2 the stopping iteration is the first k >= 1 with
    # ||f~_k||^2 <= eps ||f~_0||^2 or <= the largest final ||f~||^2 of the
    # earlier columns of its chunk (0 for the first one), else max_inner.
    G, h, x0 = _faststop_instance()
    K, eps = 40, 1e-5
    x, it, nk = oracle.nqp_batch_faststop(G, h, x0, chunk=chunk, max_inner=K, eps=eps)
    ncols = h.shape[0]
    saw_break = False
    for c0 in range(0, ncols, chunk):
        m = 0.0
        for j in range(c0, min(ncols, c0 + chunk)):
            _, kt, tr = oracle.nqp_trace(G, h[j], x0[j], max_inner=K, eps=0.0)
            want = K
            for k in range(1, len(tr)):
                if tr[k] <= eps * tr[0] or tr[k] <= m:
                    want = k
                    break
            plain = next((k for k in range(1, len(tr)) if tr[k] <= eps * tr[0]), K)
            saw_break |= want < plain
            assert it[j] == want, (chunk, j, it[j], want)
            assert nk[j] == tr[want]
            m = max(m, tr[want])
            xt, _ = oracle.nqp(G, h[j], x0[j], max_inner=want, eps=0.0)
            assert np.array_equal(x[j], xt)
    if chunk > 1:
        assert saw_break  # the instance does exercise the fast-break


# ---------------------------------------------------------------------------
# The stopping quantity of Algorithm 3 recorded per iteration: ||f~_k||^2, the
# squared norm of the projected gradient in the rescaled variables y = x sqrt(d)
# (Q = D^-1/2 H D^-1/2, q = h / sqrt(d): g = Q y + q, and g_i counts where
# y_i > 0 or g_i < 0), checked against that definition at the iterate the
# solver reaches after k iterations.

@pytest.mark.parametrize("seed,r,l1", [(3, 6, 0.0), (8, 10, 0.05), (21, 16, 0.2)])
def test_trace_is_the_projected_gradient_norm_of_each_iterate(seed, r, l1):
    _, _, H, h = random_nqp(r, seed, l1=l1)
    x0 = np.random.default_rng(seed + 100).random(r)
    K = 12
    _, kt, tr = oracle.nqp_trace(H, h, x0, max_inner=K, eps=0.0)
    assert kt == K and len(tr) == K + 1
    s = np.sqrt(np.diag(H))
    Q = H / np.outer(s, s)
    q = h / s
    for k in range(K + 1):
        xk = x0 if k == 0 else oracle.nqp(H, h, x0, max_inner=k, eps=0.0)[0]
        y = xk * s
        g = Q @ y + q
        p = np.where((y > 0) | (g < 0), g, 0.0)
        want = float(p @ p)
        assert tr[k] == pytest.approx(want, rel=1e-9, abs=1e-300), (k, tr[k], want)
    assert tr[K] < tr[0]  # the iterations make progress on these instances
