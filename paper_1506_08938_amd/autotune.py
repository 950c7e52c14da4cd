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
python -m paper_1506_08938_amd.autotune --dense OUT_DIR writes the dense
product's split-K table OUT_DIR/dense_tuned.h (and dense_tuned.json), and
--dense-from-json JSON OUT_DIR re-derives it from a saved sweep;
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


# ---------------------------------------------------------------------------- dense split-K
# The dense product's one free tile parameter per shape is its split-K slice
# count (a block computes 128 rows of P by 32 x NT columns over one slice of
# k; the slices' partial products are summed in slice order).  For a grid of
# shapes (rows of P, k) and column tiles NT = 1..4 it times every candidate
# count for each of the three kernel instantiations -- FP32 reading V (the
# W-update), FP32 reading V' k-major (the H-update), BF16 -- and records the
# fastest; the library's rule competes as candidate 0 and is kept (0 in the
# table) unless a count beats it by more than DENSE_RULE_MARGIN (then, of the
# counts within DENSE_MARGIN of the fastest, the fewest slices: less partial
# traffic).  A table entry is applied to shapes around its grid point, where
# an optimum a few percent deep does not carry over (measured at 20000 x 10000,
# r = 64, BF16: the neighbouring grid points' 3-4% better counts were 7-10%
# slower there), so only clear wins replace the rule.  Shapes beyond
# DENSE_MAX_ELEMS entries of V keep the rule.
DENSE_C = [128, 512, 2048, 8192, 32768]
DENSE_K = [256, 1024, 4096, 16384, 65536, 262144]
DENSE_NT = [1, 2, 3, 4]
DENSE_KERNELS = [("fp32", 0, 1), ("fp32_vt", 0, 0), ("bf16", 1, 1)]  # (name, precision, trans)
DENSE_MAX_ELEMS = 1 << 30
DENSE_MARGIN = 1.02
DENSE_RULE_MARGIN = 1.10
DENSE_REPS = 5


def dense_candidates(K):
    most = min(512, (K + 63) // 64)
    return sorted({1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512} & set(range(1, most + 1)))


def dense_choose(times):
    """0 (the rule) unless a slice count beats it by more than
    DENSE_RULE_MARGIN; else the fewest slices within DENSE_MARGIN of the
    fastest."""
    best_t = min(times.values())
    if times[0] <= DENSE_RULE_MARGIN * best_t:
        return 0
    return min(ns for ns, t in times.items() if ns > 0 and t <= DENSE_MARGIN * best_t)


def dense_from_json(path):
    """The table of an earlier sweep (its dense_tuned.json), re-chosen."""
    with open(path) as f:
        raw = json.load(f)
    table = {}
    for key, v in raw.items():
        k, nt, C, K = key.split(",")
        times = {int(ns): t for ns, t in v["ms"].items()}
        table[(k, int(nt), int(C), int(K))] = (dense_choose(times), times)
    return table


def dense_sweep(log=print):
    import torch
    from . import native
    table = {}
    g = torch.Generator(device="cuda")
    g.manual_seed(4242)
    for C in DENSE_C:
        for K in DENSE_K:
            if C * K > DENSE_MAX_ELEMS:
                continue
            for kname, prec, trans in DENSE_KERNELS:
                # trans = 1: P (m x r) = V A, C = m, K = n; trans = 0: P (n x r) = V' A, C = n, K = m
                m, n = (C, K) if trans else (K, C)
                V = torch.rand((m, n), device="cuda", generator=g)
                for nt in DENSE_NT:
                    r = 32 * nt
                    A = torch.rand((K, r), device="cuda", generator=g)
                    times = {}
                    for ns in [0] + dense_candidates(K):
                        ts = sorted(native.dense_product_time(V, A, trans, prec, ns, DENSE_REPS) for _ in range(3))
                        times[ns] = ts[1]
                    best = dense_choose(times)
                    table[(kname, nt, C, K)] = (best, times)
                    log(f"{kname:8s} NT={nt} C={C:6d} K={K:6d}: best {best:3d} slices {times[best]:.4f} ms "
                        f"(1 slice {times[1]:.4f} ms, rule {times[0]:.4f} ms)")
                    del A
                del V
                torch.cuda.empty_cache()
    return table


def dense_write(table, out_dir, command):
    kn = [k for k, _, _ in DENSE_KERNELS]
    lines = [
        "// Split-K slices of the dense product, measured by autotune.py --dense on an",
        "// MI355X at each grid point: 0 keeps the rule in k_dense.hip (not measured, or",
        "// no count beat it by more than 10%); k_dense.hip reads an entry as the block",
        "// count it gave at its grid point.",
        f"// Command: {command}",
        "#pragma once",
        "",
        "namespace nmfi {",
        "",
        f"constexpr long long kDenseTunedC[] = {{{', '.join(str(c) for c in DENSE_C)}}};",
        f"constexpr long long kDenseTunedK[] = {{{', '.join(str(k) for k in DENSE_K)}}};",
        "// [kernel: 0 FP32 V, 1 FP32 V' (k-major), 2 BF16][column tiles - 1][C index][K index]",
        f"constexpr int kDenseTunedSplit[3][{len(DENSE_NT)}][{len(DENSE_C)}][{len(DENSE_K)}] = {{",
    ]
    for k in kn:
        lines.append("    {")
        for nt in DENSE_NT:
            rows = []
            for C in DENSE_C:
                rows.append("{" + ", ".join(str(table.get((k, nt, C, K), (0,))[0]) for K in DENSE_K) + "}")
            lines.append("        {" + ", ".join(rows) + "},")
        lines.append("    },")
    lines += ["};", "", "}  // namespace nmfi", ""]
    with open(os.path.join(out_dir, "dense_tuned.h"), "w") as f:
        f.write("\n".join(lines))
    with open(os.path.join(out_dir, "dense_tuned.json"), "w") as f:
        json.dump({f"{k},{nt},{C},{K}": {"best": v[0], "ms": {str(ns): t for ns, t in v[1].items()}}
                   for (k, nt, C, K), v in table.items()}, f, indent=1)


def main():
    if len(sys.argv) > 3 and sys.argv[1] == "--dense-from-json":
        src, out = sys.argv[2], sys.argv[3]
        dense_write(dense_from_json(src), out,
                    f"python -m paper_1506_08938_amd.autotune --dense OUT_DIR (sweep on the GPU), then "
                    f"--dense-from-json {os.path.basename(src)}")
        return
    if len(sys.argv) > 2 and sys.argv[1] == "--dense":
        out = sys.argv[2]
        os.makedirs(out, exist_ok=True)
        t0 = time.perf_counter()
        table = dense_sweep(lambda s: print(s, flush=True))
        dense_write(table, out, "python -m paper_1506_08938_amd.autotune --dense " + out)
        print(f"dense autotune done in {time.perf_counter() - t0:.1f}s", flush=True)
        return
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
