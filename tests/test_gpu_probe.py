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
