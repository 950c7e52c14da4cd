"""Serving (continuously batched fold-in requests and small fits) on the GPU:
a request's result is the same alone and in a mix of other requests
(bitwise: a column's arithmetic does not depend on its batch), equals the
direct nmf_foldin / nmf_fit result, and matches the FP64 oracle."""
import numpy as np
import pytest

import oracle
from near_ties import near_tied
from paper_1506_08938_amd import synth

pytestmark = pytest.mark.gpu


def T(a, dt=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()


def H(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def basis():
    from paper_1506_08938_amd import native as nat
    m, r = 4000, 48
    W = np.random.default_rng(5).gamma(2.0, 0.5, (m, r)).astype(np.float32)
    B = nat.Basis(T(W), l1=0.05, l2=0.0, opt=nat.opts(max_inner=100, eps=1e-3))
    yield B, W
    B.close()


def test_alone_equals_mix_equals_direct(basis):
    import torch
    from paper_1506_08938_amd import native as nat
    B, W = basis
    m, r = W.shape
    req = synth.foldin_columns(m, 300, 60, seed=1)
    R = nat.sparse_request(req, m)
    # direct call
    direct = H(B.foldin(R))
    # alone through the server
    S = nat.Server(B, hbm_budget=1 << 30, max_slots=2, max_batch_cols=4096)
    out_alone = torch.empty((300, r), device="cuda")
    S.wait(S.submit_foldin(R, out_alone))
    # in a mix: many requests of other sizes (sparse and dense), a fit, and R again
    mix_out = []
    tickets = []
    sizes = synth.request_sizes(40, seed=9, cmax=2000)
    for i, c in enumerate(sizes):
        q = synth.foldin_columns(m, int(c), 60, seed=100 + i)
        if i % 7 == 3:
            Rq = nat.DeviceMatrix(T(q.toarray().T))  # dense request
        else:
            Rq = nat.sparse_request(q, m)
        o = torch.empty((int(c), r), device="cuda")
        tickets.append(S.submit_foldin(Rq, o))
        if i == 20:
            out_mix = torch.empty((300, r), device="cuda")
            t_r = S.submit_foldin(R, out_mix)
            fitp = synth.workload4(count=1024, first=1)[0]
            Wf, Hf = T(fitp["W0"]), T(fitp["Ht0"])
            t_fit = S.submit_fit(T(fitp["V"]), fitp["r"], nat.reg(), nat.opts(max_outer=3), Wf, Hf)
    S.wait()
    assert np.array_equal(H(out_alone), direct)
    assert np.array_equal(H(out_mix), direct)
    # the fit request equals nmf_fit
    W2, H2 = T(fitp["W0"]), T(fitp["Ht0"])
    nat.fit(nat.DeviceMatrix(T(fitp["V"])), fitp["r"], nat.reg(), nat.opts(max_outer=3), W2, H2,
            want_trace=False)
    assert np.array_equal(H(Wf), H(W2)) and np.array_equal(H(Hf), H(H2))
    st = S.stats()
    assert st["completed"] == 43 and st["batches"] <= 43
    S.close()
    # and the fold-in matches the FP64 oracle (cold start, same stopping rule)
    G = oracle.gram(W, 0.0)
    P = oracle.product_csr(req, W, 1)
    xo, ito, cd = oracle.nqp_batch_cdtrace(G.astype(np.float32), (-P + np.float32(0.05)).astype(np.float32),
                                           np.zeros((300, r)), max_inner=100, eps=1e-3, trace_iters=10)
    e = np.linalg.norm(direct - xo, axis=1) / np.maximum(np.linalg.norm(xo, axis=1), 1e-30)
    tie = near_tied(cd) | (ito > 10)
    print(f"served fold-in vs oracle: median {np.median(e):.2e} p99 {np.quantile(e, .99):.2e} "
          f"max {e.max():.2e}; near-tied {tie.mean():.3f}")
    assert np.median(e) < 1e-5 and np.quantile(e, 0.99) < 2e-5
    assert not ((e > 1e-4) & ~tie).any()


def test_bf16_basis_alone_equals_mix_equals_direct():
    """A BF16 basis (Gram in BF16, sparse requests gathered from a BF16 copy
    of W): the batched server path gives the direct nmf_foldin result
    bitwise, alone and in a mix, and matches the oracle fed the rounded W."""
    import torch
    from paper_1506_08938_amd import native as nat
    m, r = 3000, 40
    W = np.random.default_rng(6).gamma(2.0, 0.5, (m, r)).astype(np.float32)
    B = nat.Basis(T(W), l1=0.05, l2=0.0, opt=nat.opts(max_inner=100, eps=1e-3, precision=nat.NMF_BF16))
    req = synth.foldin_columns(m, 200, 60, seed=2)
    R = nat.sparse_request(req, m)
    direct = H(B.foldin(R))
    S = nat.Server(B, hbm_budget=1 << 30, max_slots=2, max_batch_cols=4096)
    out_alone = torch.empty((200, r), device="cuda")
    S.wait(S.submit_foldin(R, out_alone))
    outs = []
    for i, c in enumerate(synth.request_sizes(12, seed=19, cmax=1500)):
        o = torch.empty((int(c), r), device="cuda")
        S.submit_foldin(nat.sparse_request(synth.foldin_columns(m, int(c), 60, seed=300 + i), m), o)
        if i == 6:
            out_mix = torch.empty((200, r), device="cuda")
            S.submit_foldin(R, out_mix)
    S.wait()
    S.close()
    assert np.array_equal(H(out_alone), direct) and np.array_equal(H(out_mix), direct)
    u = W.view(np.uint32)
    Wb = ((u + np.uint32(0x7FFF) + ((u >> 16) & np.uint32(1))) & np.uint32(0xFFFF0000)).view(np.float32)
    xo, _ = oracle.nqp_batch(oracle.gram(Wb, 0.0).astype(np.float32),
                             (-oracle.product_csr(req, Wb, 1) + np.float32(0.05)).astype(np.float32),
                             np.zeros((200, r)), max_inner=100, eps=1e-3)
    e = np.linalg.norm(direct - xo, axis=1) / np.maximum(np.linalg.norm(xo, axis=1), 1e-30)
    print(f"bf16 basis fold-in vs rounded-W oracle: median {np.median(e):.2e} p99 {np.quantile(e, .99):.2e} "
          f"max {e.max():.2e}")
    assert np.median(e) < 1e-5 and np.quantile(e, 0.99) < 1e-4
    B.close()


def test_budget_refusal_and_latency(basis):
    import torch
    from paper_1506_08938_amd import native as nat
    B, W = basis
    m, r = W.shape
    S = nat.Server(B, hbm_budget=200000, max_slots=1, max_batch_cols=1024)
    small = nat.sparse_request(synth.foldin_columns(m, 50, 20, seed=2), m)
    big = nat.sparse_request(synth.foldin_columns(m, 3000, 20, seed=3), m)
    o = torch.empty((50, r), device="cuda")
    lat = S.wait(S.submit_foldin(small, o))
    assert lat > 0
    with pytest.raises(nat.NmfError) as ei:
        S.submit_foldin(big, torch.empty((3000, r), device="cuda"))
    assert ei.value.status == nat.NMF_E_BUSY
    S.close()


def test_fast_break_results_do_not_depend_on_the_batch():
    import torch
    from paper_1506_08938_amd import native as nat
    m, r = 3000, 40
    W = np.random.default_rng(8).gamma(2.0, 0.5, (m, r)).astype(np.float32)
    B = nat.Basis(T(W), l1=0.05, l2=0.0, opt=nat.opts(max_inner=100, eps=1e-3, fast_break_cols=24))
    req = nat.sparse_request(synth.foldin_columns(m, 333, 40, seed=11), m)
    direct = H(B.foldin(req))
    S = nat.Server(B, hbm_budget=1 << 30, max_slots=3, max_batch_cols=4096)
    outs, tickets = [], []
    for i, c in enumerate([5, 333, 100, 17]):
        q = req if c == 333 else nat.sparse_request(synth.foldin_columns(m, c, 40, seed=50 + i), m)
        o = torch.empty((c, r), device="cuda")
        outs.append(o)
        tickets.append(S.submit_foldin(q, o))
    S.wait()
    assert np.array_equal(H(outs[1]), direct)
    S.close()
    B.close()


def test_fit_requests_batched_together_equal_nmf_fit(basis):
    """Fit requests waiting together run as one batch through the batched
    kernels (each with its nmf_fit solve layout): every result equals its
    nmf_fit bitwise, regularised problems and options included; a request
    with other options, or one that asks for the input scan, runs alone."""
    import torch
    from paper_1506_08938_amd import native as nat
    B, W = basis
    fits = synth.workload5_fits(10, seed=7007)
    regs = [nat.reg(0.01 * (i % 2), 0.02 * (i % 3 == 0), 0.05 * (i % 4 == 1), 0.01 * (i % 5 == 2))
            for i in range(len(fits))]
    opts = [nat.opts(max_outer=4) if i != 7 else nat.opts(max_outer=3, eps=1e-4) for i in range(len(fits))]
    opts[8] = nat.opts(max_outer=4, check_finite=1)
    # one slot for fits (max_slots 2): every fit submitted before the first
    # can start waits in the queue and is taken with the next batch
    S = nat.Server(B, hbm_budget=4 << 30, max_slots=2, max_batch_cols=4096)
    outs, tickets = [], []
    for f, rg, o in zip(fits, regs, opts):
        Wd, Hd = T(f["W0"]), T(f["Ht0"])
        outs.append((Wd, Hd))
        tickets.append(S.submit_fit(T(f["V"]), f["r"], rg, o, Wd, Hd))
    S.wait()
    batches = S.stats()["batches"]
    S.close()
    for (Wd, Hd), f, rg, o in zip(outs, fits, regs, opts):
        W2, H2 = T(f["W0"]), T(f["Ht0"])
        nat.fit(nat.DeviceMatrix(T(f["V"])), f["r"], rg, o, W2, H2, want_trace=False)
        assert np.array_equal(H(Wd), H(W2)) and np.array_equal(H(Hd), H(H2))
    print(f"{len(fits)} fit requests in {batches} batches")
    assert batches < len(fits)


def test_stream_of_small_requests_all_succeed_and_match_direct(basis):
    """Thousands of small fold-in requests submitted at once keep every slot
    at its limit of batches in flight, each batch in a reused workspace:
    every request completes without error and equals the direct fold-in."""
    import torch
    from paper_1506_08938_amd import native as nat
    B, W = basis
    m, r = W.shape
    reqs = [nat.sparse_request(synth.foldin_columns(m, c, 30, seed=900 + c), m) for c in (1, 3, 7, 20, 64)]
    direct = [H(B.foldin(q)) for q in reqs]
    S = nat.Server(B, hbm_budget=1 << 30, max_slots=3, max_batch_cols=256)
    outs, tickets = [], []
    for i in range(3000):
        k = i % len(reqs)
        o = torch.empty((reqs[k].m.cols, r), device="cuda")
        outs.append((k, o))
        tickets.append(S.submit_foldin(reqs[k], o))
    for t in tickets:
        S.wait(t)  # raises on a failed request
    st = S.stats()
    S.close()
    assert st["completed"] == 3000
    for k, o in outs[::37]:
        assert np.array_equal(H(o), direct[k])
