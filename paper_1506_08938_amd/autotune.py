"""Lanes-per-column autotuner for the solve kernel.

For a grid of ranks r and launch sizes ncols it times nnls_solve_batch with
every lanes-per-column value the compiled table allows (1, 2, 4, 8, 16) and
records the fastest.  The result is written as a C table (``nqp_tuned.h``)
that the library compiles in: the automatic layout choice then follows the
measurement, and stays a fixed function of (r, ncols), so results are
reproducible run to run.

The instances are shaped like the alternating fit's subproblems: Gamma =
A'A + 2*l2*I with A ~ U[0,1) of 4r rows, h = -A'B + l1, max_inner 100, eps
1e-3, from two start points: near the solution (1% off, as late in a fit:
about one iteration per column) and mid-fit (each entry scaled by U[0.5,
1.5) plus 10% of the mean, several iterations per column and a longer tail
of slow columns).  A layout's score is the sum of its two times.

Usage (on the GPU):  python -m paper_1506_08938_amd.autotune OUT_DIR
writes OUT_DIR/nqp_tuned.h and OUT_DIR/nqp_tuned.json;
python -m paper_1506_08938_amd.autotune --from-json JSON OUT_DIR re-derives
the header from a saved sweep.  The library compiles csrc/nqp_tuned.h (and
csrc/nqp_tuned.json keeps the sweep it came from).
"""
from __future__ import annotations

import json
import os
import sys
import time

RANKS = [4, 8, 12, 16, 20, 24, 32, 40, 48, 56, 64, 72, 80, 90, 100, 112, 128]
COLS = [256, 1024, 4096, 16384, 32768, 65536, 131072, 262144]
LANES = [1, 2, 4, 8, 16]
REPS = 5


def _instance(r, ncols, torch, native, synth):
    import numpy as np
    inst = synth.nqp_instance(r, 2048, seed=1234 + r, l1=0.05, l2=0.01, k=4 * r)
    A = inst["A"].astype(np.float64)
    B = inst["B"].astype(np.float64)
    G = torch.from_numpy((A.T @ A + 0.02 * np.eye(r)).astype(np.float32)).cuda()
    h0 = torch.from_numpy((0.05 - B.T @ A).astype(np.float32)).cuda()
    h = h0.repeat((ncols + 2047) // 2048, 1)[:ncols].contiguous()
    X = torch.rand((ncols, r), device="cuda")
    native.nnls_solve_batch(G, h, X, native.opts(max_inner=100, eps=1e-3, lanes=0))
    g = torch.Generator(device="cuda")
    g.manual_seed(r * 7919 + ncols)
    Xw = (X + 0.01 * torch.rand(X.shape, device="cuda", generator=g)).contiguous()
    scale = torch.rand(X.shape, device="cuda", generator=g) + 0.5
    Xm = (X * scale + 0.1 * X.mean() * torch.rand(X.shape, device="cuda", generator=g)).contiguous()
    torch.cuda.synchronize()
    return G, h, Xw, Xm


def _time(G, h, X0, lanes, torch, native):
    o = native.opts(max_inner=100, eps=1e-3, lanes=lanes)
    s = torch.cuda.current_stream()
    ts = []
    for _ in range(REPS):
        X = X0.clone()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        native.nnls_solve_batch(G, h, X, o)
        b.record(s)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


# A wider layout must win by this margin: differences below it are launch
# noise at the small sizes, and narrower groups waste fewer lanes on padding.
MARGIN = 1.03


def choose(times):
    """The narrowest layout within MARGIN of the fastest."""
    best = min(times.values())
    return min(L for L, t in times.items() if t <= MARGIN * best)


def sweep(log=print):
    import torch
    from . import native, synth
    table = {}
    for r in RANKS:
        for c in COLS:
            G, h, Xw, Xm = _instance(r, c, torch, native, synth)
            times, parts = {}, {}
            for L in LANES:
                try:
                    native.layout(r, c, L)
                except native.NmfError:
                    continue
                tn = _time(G, h, Xw, L, torch, native)
                tm = _time(G, h, Xm, L, torch, native)
                times[L] = tn + tm
                parts[L] = (tn, tm)
            best = choose(times)
            table[(r, c)] = (best, times, parts)
            log(f"r={r:4d} ncols={c:7d} " +
                " ".join(f"L{L}={a:.3f}+{b:.3f}ms" for L, (a, b) in parts.items()) + f"  -> L={best}")
    return table


def write(table, out_dir, command):
    lines = [
        "// Lanes per column of the solve kernel, measured by autotune.py on an",
        "// MI355X: the fastest value for each (rank, launch size) grid point.",
        f"// Command: {command}",
        "#pragma once",
        "",
        "namespace nmfi {",
        "",
        f"constexpr int kTunedRanks[] = {{{', '.join(str(r) for r in RANKS)}}};",
        f"constexpr long long kTunedCols[] = {{{', '.join(str(c) for c in COLS)}}};",
        "// [rank index][column index]",
        f"constexpr int kTunedLanes[{len(RANKS)}][{len(COLS)}] = {{",
    ]
    for r in RANKS:
        lines.append("    {" + ", ".join(str(table[(r, c)][0]) for c in COLS) + "},")
    lines += ["};", "", "}  // namespace nmfi", ""]
    with open(os.path.join(out_dir, "nqp_tuned.h"), "w") as f:
        f.write("\n".join(lines))
    with open(os.path.join(out_dir, "nqp_tuned.json"), "w") as f:
        json.dump({f"{r},{c}": {"best": v[0], "ms": {str(L): t for L, t in v[1].items()},
                                "ms_near_mid": {str(L): list(p) for L, p in (v[2] if len(v) > 2 else {}).items()}}
                   for (r, c), v in table.items()}, f, indent=1)


def from_json(path):
    """The table of an earlier sweep (its nqp_tuned.json), re-chosen."""
    with open(path) as f:
        raw = json.load(f)
    table = {}
    for key, v in raw.items():
        r, c = (int(x) for x in key.split(","))
        times = {int(L): t for L, t in v["ms"].items()}
        parts = {int(L): tuple(p) for L, p in v.get("ms_near_mid", {}).items()}
        table[(r, c)] = (choose(times), times, parts)
    return table


def main():
    if len(sys.argv) > 3 and sys.argv[1] == "--from-json":
        src, out = sys.argv[2], sys.argv[3]
        write(from_json(src), out,
              f"python -m paper_1506_08938_amd.autotune (sweep on the GPU), then "
              f"--from-json {os.path.basename(src)}")
        return
    out = sys.argv[1] if len(sys.argv) > 1 else "."
    os.makedirs(out, exist_ok=True)
    t0 = time.perf_counter()
    table = sweep(lambda s: print(s, flush=True))
    write(table, out, "python -m paper_1506_08938_amd.autotune " + out)
    print(f"autotune done in {time.perf_counter() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main()
