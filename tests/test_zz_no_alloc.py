"""nmf_foldin_noalloc (the fold-in with no device allocation, its scratch a
fixed device array) against nmf_foldin through the C ABI: two calls in a row,
the second smaller, bitwise equal results and iteration counts; sizes beyond
its scratch and dense requests are refused on the host."""
import numpy as np
import pytest

from paper_1506_08938_amd import synth

pytestmark = pytest.mark.gpu


def T(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


@pytest.mark.parametrize("r,precision", [(128, 0), (16, 0), (100, 1)])
def test_noalloc_foldin_equals_foldin(r, precision):
    import torch
    from paper_1506_08938_amd import native as nat
    m = 5000
    W = np.random.default_rng(r).gamma(2.0, 0.5, (m, r)).astype(np.float32)
    B = nat.Basis(T(W), l1=0.05, l2=0.01, opt=nat.opts(max_inner=100, eps=1e-3, precision=precision))
    for c, seed in ((3000, 1), (700, 2)):  # the second call smaller than the first
        req = nat.sparse_request(synth.foldin_columns(m, c, 40, seed=seed + 10 * r), m)
        it_ref = torch.zeros(c, dtype=torch.int32, device="cuda")
        ref = B.foldin(req, iters=it_ref)
        out = torch.full((c, r), -1.0, device="cuda")
        it = torch.full((c,), -1, dtype=torch.int32, device="cuda")
        B.foldin_noalloc(req, out, iters=it)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (r, c)
        assert torch.equal(it, it_ref), (r, c)
        assert (it >= 1).all()
    B.close()


def test_noalloc_foldin_refuses_what_its_scratch_cannot_hold():
    import torch
    from paper_1506_08938_amd import native as nat
    m, r = 600, 128
    W = np.random.default_rng(3).random((m, r), dtype=np.float32)
    B = nat.Basis(T(W), l1=0.05)
    cap = ((16 << 20) - 256) // (4 * r)
    big = nat.sparse_request(synth.foldin_columns(m, cap + 1, 2, seed=4), m)
    out = torch.empty((cap + 1, r), device="cuda")
    with pytest.raises(nat.NmfError) as ei:
        B.foldin_noalloc(big, out)
    assert ei.value.status == nat.NMF_E_INVAL and "at most" in str(ei.value)
    dense = nat.DeviceMatrix(T(np.ones((m, 3))))
    with pytest.raises(nat.NmfError) as ei:
        B.foldin_noalloc(dense, torch.empty((3, r), device="cuda"))
    assert ei.value.status == nat.NMF_E_UNSUPPORTED
    # at the limit it runs and equals nmf_foldin
    edge = nat.sparse_request(synth.foldin_columns(m, cap, 2, seed=5), m)
    out = torch.empty((cap, r), device="cuda")
    B.foldin_noalloc(edge, out)
    assert torch.equal(out, B.foldin(edge))
    B.close()
