"""How far the FP64 oracle's own alternating fit moves under perturbations of
float32 size: the yardstick for comparing a float32 GPU run with it.

The GPU path stores the factors, the Gram matrices and the data products in
float32 and solves every NQP in float32.  The oracle does all of it in float64.
So a GPU result may legitimately differ from the oracle's by as much as the
oracle's own result moves when its intermediate quantities are disturbed at
float32 resolution.  This module measures that spread with the oracle alone
(it calls nothing of the GPU library), by running the same outer iterations as
``oracle.nmf_fit`` step by step -- Gram, product, half-update, for the H-update
then the W-update -- with one of these disturbances:

  "round":   the Gram matrix, the product and the factor after every half are
             rounded to float32 (what the GPU stores between its kernels);
  "ulp":     the start point W0 nudged up by one float32 ulp in every entry
             (a perturbation the trajectory may amplify);
  "jitter":  as "round", and every computed entry x additionally multiplied by
             (1 + u sqrt(k) z), z ~ N(0, 1), u = 2^-24, k the number of terms
             summed or updated to form it (the rows of A for the Gram and the
             product; r times the inner iterations its NQP ran for a solved
             factor entry, each iteration updating the gradient with r-term
             sums): the usual random-walk model of the rounding error of a
             k-term float32 sum.  The solve's own gradient, an r-term sum
             Gamma x, carries an error of about u sqrt(r) sum_b |Gamma_ab x_b|;
             that much is added to the product at random, so that the oracle's
             greedy choices meet near-ties as a float32 solve does.  A few
             seeds.

The quantity reported is the relative change of the regularised objective J
and of the factors against the undisturbed float64 run.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

import oracle


def _round32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


U32 = 2.0 ** -24


def _jitter(a, k, g):
    """a rounded to float32 after a relative error u sqrt(k) z, z ~ N(0, 1)."""
    a = np.asarray(a, dtype=np.float64)
    return _round32(a * (1.0 + U32 * np.sqrt(k) * g.standard_normal(a.shape)))


def _product(V, A, trans):
    return oracle.product_csr(V, A, trans) if sp.issparse(V) else oracle.product_dense(V, A, trans)


def stepwise_fit(V, r, reg, W0, Ht0, T, mode=None, seed=0, max_inner=10, eps=0.0, ls_guard=1,
                 losses=None, inner=None):
    """T outer iterations of Algorithm 2 through the oracle's building blocks,
    with the disturbance `mode` (None: none; then the result equals
    oracle.nmf_fit's).  `losses` (a list) gets 0.5||V - WH||^2 after each
    outer iteration, `inner` (a list) the inner iterations of each half."""
    l1w, l2w, l1h, l2h = reg
    g = np.random.default_rng(seed)
    W = np.asarray(W0, dtype=np.float64).copy()
    Ht = np.asarray(Ht0, dtype=np.float64).copy()
    if mode == "ulp":
        W = np.nextafter(np.asarray(W0, dtype=np.float32), np.float32(np.inf)).astype(np.float64)
    if mode == "jitter":
        post = lambda a, k: _jitter(a, k, g)  # noqa: E731
    elif mode == "round":
        post = lambda a, k: _round32(a)  # noqa: E731
    else:
        post = lambda a, k: a  # noqa: E731
    def grad_noise(P, G, X):
        """The solve's own gradient rounding, charged to the linear term: an
        r-term float32 sum Gamma x carries an error of about u sqrt(r) times
        sum_b |Gamma_ab x_b|, so P gets that much extra, at random."""
        if mode != "jitter":
            return P
        scale = U32 * np.sqrt(r) * (np.abs(X) @ np.abs(G))
        return _round32(P + scale * g.standard_normal(P.shape))

    m, n = V.shape
    for _ in range(T):
        G = post(oracle.gram(W, l2h), m)
        P = grad_noise(post(_product(V, W, 0), m), G, Ht)
        Ht, ih = oracle.half_update(G, P, l1h, Ht, max_inner=max_inner, eps=eps, ls_guard=ls_guard)
        Ht = post(Ht, r * ih[:, None])
        G = post(oracle.gram(Ht, l2w), n)
        P = grad_noise(post(_product(V, Ht, 1), n), G, W)
        W, iw = oracle.half_update(G, P, l1w, W, max_inner=max_inner, eps=eps, ls_guard=ls_guard)
        W = post(W, r * iw[:, None])
        if inner is not None:
            inner += [int(ih.sum()), int(iw.sum())]
        if losses is not None:
            losses.append(oracle.loss(V, W, Ht))
    return W, Ht


def rel_fro(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


MODES = ("round", "ulp", "jitter")


# Jitter seeds of a spread: the largest change over the seeds estimates the
# top of the oracle's own FP32 variability, and three under-sample it -- on
# the dense regularised test problem the one-step |dJ|/J over 40 seeds has
# median 2.5e-5, 90th percentile 8.1e-5, maximum 1.6e-4, while seeds 1-3 give
# at most 2.4e-5.
SEEDS = tuple(range(1, 21))


def spread(V, r, reg, W0, Ht0, T, seeds=SEEDS, modes=MODES, **opts):
    """Largest relative change of J, of W and Ht, and (over the T outer
    iterations) of the loss, under the disturbances, against the undisturbed
    float64 run, and of the mean inner iterations per solved column (kbar).
    Returns a dict with the per-run values ("modes": name -> (dJ, dW, dH,
    dloss, dkbar)) and their maxima "dJ", "dW", "dH", "dloss", "dkbar"."""
    lr, ir = [], []
    Wr, Hr = stepwise_fit(V, r, reg, W0, Ht0, T, None, losses=lr, inner=ir, **opts)
    Jr = oracle.objective(V, Wr, Hr, reg)
    lr = np.array(lr)
    kr = sum(ir)
    res = {"J": Jr, "modes": {}}
    runs = [(m, 0) for m in modes if m != "jitter"]
    if "jitter" in modes:
        runs += [("jitter", s) for s in seeds]
    for mode, s in runs:
        ls, it = [], []
        W, Ht = stepwise_fit(V, r, reg, W0, Ht0, T, mode, seed=s, losses=ls, inner=it, **opts)
        J = oracle.objective(V, W, Ht, reg)
        res["modes"][f"{mode}{s if mode == 'jitter' else ''}"] = (
            abs(J - Jr) / Jr, rel_fro(W, Wr), rel_fro(Ht, Hr),
            float(np.max(np.abs(np.array(ls) - lr) / lr)), abs(sum(it) - kr) / kr)
    vals = np.array(list(res["modes"].values()))
    res["dJ"], res["dW"], res["dH"], res["dloss"], res["dkbar"] = (float(v) for v in vals.max(axis=0))
    return res
