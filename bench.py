"""Throughput of the alternating anti-lopsided NNLS hot path on one MI355X.

One step = one outer iteration of Algorithm 2 on the sparse text-like
workload (CSR V 200000 x 100000, 0.1% density, Zipf(1.1) column ranks,
values log(1 + Poisson(3)), r = 100, L1 = 0.1 on H, L2 = 0.01 on W): the
H-update (Gram of W, rescale, CSR(V') W product, 100000 column NQPs) and the
W-update (Gram of H, rescale, CSR(V) Ht product, 200000 row NQPs), all in the
library's HIP kernels, with inputs resident in HBM.

value = column NNLS solves per second = (m + n) x steps / elapsed.  The
roofline entry is for the dominant kernel (the NQP solve), timed with HIP
events recorded on its stream during the timed steps; its algorithmic work
is counted per solved column as  init(r) = r^2 + 5r  plus, per inner
iteration,  iter(r) = 7r^2 + 13r  lane operations, against
the VALU issue rate of 256 CUs x 64 lanes x 2.4 GHz.  The CPU baseline is
the FP64 oracle timed on the host cores for one outer iteration of the same
workload from the same start point (its first --cpu-iters outer
iterations).

The "serving" entry covers the fold-in side of the metric: a basis W
(100000 x 128) fitted on the device to Gamma-factor data stays resident;
fold-in requests of c ~ logU[1, 8192] sparse columns (0.5% density) and 5%
small full fits go through nmf_server_*.  First every request is submitted at
once (saturated: fold-in columns solved per second), then the same mix
arrives as a Poisson stream at --serve-load times the saturated request rate
and the per-request latencies (submission to completion) give p50/p99.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--cpu-iters T]
                       [--no-serve] [--serve-requests N] [--serve-load F]
       python bench.py --calibrate-copy   (1 GiB device copy, for counter scaling)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_LANE_OPS = 256 * 64 * 2.4e9  # VALU lane operations / s (no packed math)
METRIC = "column NNLS solves/s at r=100 vs roofline; p50/p99 fold-in latency at 1 GPU"


def init_ops(r):
    return r * r + 5 * r


def iter_ops(r):
    return 7 * r * r + 13 * r


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash(L):
    """SHA-256 of the sources that define the solve kernel with L lanes per
    column (its template, its instantiation file and the build flags)."""
    import hashlib
    h = hashlib.sha256()
    for rel in ["paper_1506_08938_amd/csrc/nqp_kernel.h", f"paper_1506_08938_amd/csrc/k_nqp_l{L}.hip",
                "paper_1506_08938_amd/build.py"]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, L):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when there is none or the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", "k_nqp_sparse_r100_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel") != kernel or fields.get("source_sha256") != kernel_source_hash(L):
        return None
    return float(fields["traffic_bytes_per_launch"])


def serving_leg(native, synth, torch, n_req, load, seed=5005):
    """Saturated throughput and Poisson-arrival latency of nmf_server_*."""
    import numpy as np
    t_setup = time.perf_counter()
    wb = synth.workload5_basis()
    m, r = wb["V"].shape[0], wb["r"]
    Vb = native.DeviceMatrix(torch.from_numpy(wb["V"]).cuda())
    W = torch.from_numpy(wb["W0"]).cuda()
    Ht = torch.from_numpy(wb["Ht0"]).cuda()
    native.fit(Vb, r, native.reg(), native.opts(max_outer=10), W, Ht, want_trace=False)
    del Vb, Ht
    basis = native.Basis(W, l1=0.05, l2=0.0, opt=native.opts(max_inner=100, eps=1e-3))
    # a pool of distinct requests, reused by the arrivals (each arrival has its own output)
    n_pool = 96
    sizes = synth.request_sizes(n_pool, seed, cmax=8192)
    pool = [native.sparse_request(synth.foldin_columns_many(m, int(c), 500, seed + 1 + i), m)
            for i, c in enumerate(sizes)]
    fits = synth.workload5_fits(8)
    fit_V = [torch.from_numpy(f["V"]).cuda() for f in fits]
    g = synth.rng(seed + 999)
    is_fit = g.random(n_req) < 0.05
    pick = g.integers(0, n_pool, n_req)
    fpick = g.integers(0, len(fits), n_req)
    fit_opt = native.opts(max_outer=30)

    def make_outputs():
        outs = []
        for i in range(n_req):
            if is_fit[i]:
                f = fits[fpick[i]]
                outs.append((torch.from_numpy(f["W0"]).cuda(), torch.from_numpy(f["Ht0"]).cuda()))
            else:
                outs.append(torch.empty((int(sizes[pick[i]]), r), device="cuda"))
        torch.cuda.synchronize()
        return outs

    def submit(S, i, outs):
        if is_fit[i]:
            f = fits[fpick[i]]
            return S.submit_fit(fit_V[fpick[i]], f["r"], native.reg(), fit_opt, *outs[i])
        return S.submit_foldin(pool[pick[i]], outs[i])

    def run(arrivals):
        outs = make_outputs()
        S = native.Server(basis, hbm_budget=8 << 30, max_slots=4, max_batch_cols=16384)
        tickets = []
        t0 = time.perf_counter()
        for i in range(n_req):
            if arrivals is not None:
                while time.perf_counter() - t0 < arrivals[i]:
                    pass
            tickets.append(submit(S, i, outs))
        S.wait()
        elapsed = time.perf_counter() - t0
        lat = np.array([S.poll(t)[1] for t in tickets])
        st = S.stats()
        S.close()
        return elapsed, lat, st

    cols = int(sum(int(sizes[pick[i]]) for i in range(n_req) if not is_fit[i]))
    log(f"[bench] serving set up in {time.perf_counter() - t_setup:.1f}s; {n_req} requests, "
        f"{cols} fold-in columns, {int(is_fit.sum())} fits")
    run(None)  # warm-up pass
    el_sat, lat_sat, st_sat = run(None)
    rate = load * n_req / el_sat
    log(f"[bench] serving saturated {el_sat * 1e3:.1f} ms; Poisson arrivals at {rate:.0f} req/s")
    arrivals = synth.poisson_arrivals(n_req, rate, seed + 7)
    el, lat, st = run(arrivals)
    fold = lat[~is_fit]
    fitl = lat[is_fit]
    basis.close()
    return {
        "workload": "resident basis W 100000x128 (10 outer iterations fitted on the device to "
                    "Gamma(2,0.5)-factor data), L1=0.05, eps=1e-3; fold-in requests of "
                    "c~logU[1,8192] columns at 0.5% density, values log(1+Poisson(3)); 5% small "
                    "full fits (m,n~logU[64,2048], r~U{4..32}, 30 outer iterations); 4 slots",
        "requests": n_req,
        "fold_in_columns": cols,
        "saturated_solves_per_s": cols / el_sat,
        "saturated_ms": el_sat * 1e3,
        "saturated_batches": st_sat["batches"],
        "arrival_rate_req_per_s": rate,
        "load": load,
        "poisson_solves_per_s": cols / el,
        "fold_in_p50_ms": float(np.percentile(fold, 50)),
        "fold_in_p99_ms": float(np.percentile(fold, 99)),
        "fit_p50_ms": float(np.percentile(fitl, 50)) if fitl.size else None,
        "poisson_batches": st["batches"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=8,
                    help="outer iterations of the CPU-oracle sample")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.5,
                    help="Poisson arrival rate as a fraction of the saturated request rate")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB device buffer (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)

    log("[bench] importing torch")
    import numpy as np
    import torch

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copied 1 GiB (read 1 GiB, write 1 GiB)")
        return

    from paper_1506_08938_amd import native, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log("[bench] generating the sparse workload")
    t_gen = time.perf_counter()
    wl = synth.workload3()
    V = wl["V"]
    m, n = V.shape
    r = wl["r"]
    log(f"[bench] generated {m}x{n} nnz={V.nnz} in {time.perf_counter() - t_gen:.1f}s")

    Vd = native.DeviceMatrix(V, with_transpose=False)  # CSR(V') is built on the device
    reg = native.reg(*wl["reg"])
    opt = native.opts(max_inner=100, eps=1e-3, ls_guard=1)
    plan = native.Plan(Vd, r, reg, opt)
    W = torch.from_numpy(wl["W0"]).cuda()
    Ht = torch.from_numpy(wl["Ht0"]).cuda()
    torch.cuda.synchronize()
    log("[bench] plan ready")

    for _ in range(args.warmup):
        plan.run(W, Ht, 1)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done")

    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = plan.run(W, Ht, args.steps, want_stats=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timers = plan.timers()
    plan.profile(False)
    elapsed = t1 - t0
    K = args.steps
    log(f"[bench] timed {K} steps in {elapsed:.3f}s")

    E_h, L_h = native.layout(r, n)
    E_w, L_w = native.layout(r, m)
    kernel = f"k_nqp<{E_h}, {L_h}>" + ("" if (E_h, L_h) == (E_w, L_w) else f" / k_nqp<{E_w}, {L_w}>")
    traffic = measured_traffic(kernel, L_h) if (E_h, L_h) == (E_w, L_w) else None
    solves = (m + n) * K
    value = solves / elapsed
    solve_ms, solve_calls = timers["solve"]
    inner_total = st["inner_total"]
    ops = solves * init_ops(r) + inner_total * iter_ops(r)
    avg_launch_s = solve_ms / 1e3 / solve_calls
    achieved = ops / solve_calls / avg_launch_s
    kbar = st["kbar"]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "column NNLS solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "sparse text-like CSR V 200000x100000, 100 Zipf(1.1) columns per row "
                        "(0.1% density), values log(1+Poisson(3)), r=100, L1=0.1 on H, L2=0.01 "
                        "on W, eps=1e-3, max_inner=100; one step = one outer iteration",
            "m": m, "n": n, "nnz": int(V.nnz), "r": r,
        },
        "roofline": {
            "bound": "alu",
            "kernel": kernel + " (Algorithm 3 solve)",
            "achieved": achieved,
            "peak": PEAK_LANE_OPS,
            "unit": "lane-ops/s",
            "frac": achieved / PEAK_LANE_OPS,
            "traffic": traffic,
            "avg_launch_ms": solve_ms / solve_calls,
            "ops_per_launch": ops / solve_calls,
        },
        "kbar": kbar,
        "phases_ms_per_step": {k: v[0] / K for k, v in timers.items()},
        "loss_after": st["loss"],
    }

    plan.close()
    if not args.no_serve:
        out["serving"] = serving_leg(native, synth, torch, args.serve_requests, args.serve_load)

    if not args.no_cpu:
        import oracle
        cores = oracle.num_threads()
        T_cpu = args.cpu_iters
        log(f"[bench] CPU oracle: {T_cpu} outer iterations on {cores} threads")
        tc = time.perf_counter()
        res = oracle.nmf_fit(V, r, wl["reg"], wl["W0"], wl["Ht0"], T=T_cpu, max_inner=100,
                             eps=1e-3, ls_guard=1, want_trace=False)
        tcpu = time.perf_counter() - tc
        kbar_cpu = res["inner"].sum() / (T_cpu * (m + n))
        out["cpu_baseline"] = {
            "value": T_cpu * (m + n) / tcpu,
            "unit": "column NNLS solves/s",
            "cores": cores,
            "kind": "oracle",
            "sample": f"the first {T_cpu} outer iterations ({T_cpu * (m + n)} column NQP solves "
                      f"plus the Gram and CSR products, FP64) of the same workload from the same "
                      f"start point; {tcpu:.1f}s; kbar {kbar_cpu:.3f}",
        }
        log(f"[bench] CPU oracle {tcpu:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
