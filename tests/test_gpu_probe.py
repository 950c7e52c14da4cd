"""The gather probe (a measurement aid, not a step of the method) reads the
rows it is given: the sum of its output equals the sum of the gathered rows
(float32 running sums: checked to a bound on their rounding), for uneven
counts, out-of-range indices (read as the nearest row) and an empty list."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rows,width,n", [(1000, 100, 12345), (77, 52, 1), (5000, 4, 300001), (10, 8, 0)])
def test_probe_reads_the_named_rows(rows, width, n):
    import torch
    from paper_1506_08938_amd import native as nat
    g = np.random.default_rng(rows + n)
    table = g.random((rows, width)).astype(np.float32)
    idx = g.integers(-3, rows + 3, n).astype(np.int32)
    out = nat.probe_gather(torch.from_numpy(table).cuda(), torch.from_numpy(idx).cuda())
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64).sum()
    want = table.astype(np.float64)[np.clip(idx, 0, rows - 1)].sum()
    # each float32 running sum adds at most n*width/(4*lanes) terms of [0, 1)
    bound = 1e-6 * max(want, 1.0) * max(1.0, n * width / 4 / (2048 * 256)) + 1e-3
    assert abs(got - want) <= bound, (got, want)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("trans", [0, 1])
def test_dense_product_time_runs_every_split(precision, trans):
    """The autotuner's timing entry runs the product with any slice count
    (0: the library's choice; counts above k/64 are clamped) and reports a
    positive time per launch."""
    import torch
    from paper_1506_08938_amd import native as nat
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    V = torch.rand((700, 300), device="cuda", generator=g)
    K = 700 if trans == 0 else 300
    A = torch.rand((K, 40), device="cuda", generator=g)
    for ns in (0, 1, 3, 512):
        ms = nat.dense_product_time(V, A, trans, precision, ns, reps=2)
        assert 0.0 < ms < 1e3, (ns, ms)
