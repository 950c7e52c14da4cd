"""Throughput of the alternating anti-lopsided NNLS hot path on one MI355X.

One step = one outer iteration of Algorithm 2 on the sparse text-like
workload (CSR V 200000 x 100000, 0.1% density, Zipf(1.1) column ranks,
values log(1 + Poisson(3)), r = 100, L1 = 0.1 on H, L2 = 0.01 on W): the
H-update (Gram of W, rescale, CSR(V') W product, 100000 column NQPs) and the
W-update (Gram of H, rescale, CSR(V) Ht product, 200000 row NQPs), all in the
library's HIP kernels, with inputs resident in HBM.

value = column NNLS solves per second = (m + n) x steps / elapsed.  The
roofline entry is for the dominant kernel (the NQP solve), timed with HIP
events attached to its own dispatches during the timed steps; its
algorithmic work is counted per solved column as  r^2  (the warm start)
plus, per inner iteration,  11 r^2 + 11 r  lane operations (the line search
about 2 r^2, the r greedy CD steps about 9 r^2), against the VALU issue rate
of 256 CUs x 64 lanes x 2.4 GHz; the exact count of the operations the
method performs (r^2 + 5r, then 7 r^2 + 13 r per iteration) is reported
beside it.  The product_roofline entry is for the product phase (row
gathers of the CSR products), algorithmic bytes per step over its time from
a separate run with events around every phase, against 8 TB/s; beside it,
the time of the gather probe (nothing but the same row loads in the same
orders) over the phase's time, the measured ceiling of the gathers.  The CPU
baseline is the FP64 oracle timed on the host cores for --cpu-iters outer
iterations of the same workload from the same start point, after --warmup
untimed ones (the GPU's warm-up).

The "serving" entry covers the fold-in side of the metric: a basis W
(100000 x 128) fitted on the device to Gamma-factor data stays resident;
fold-in requests of c ~ logU[1, 8192] sparse columns (0.5% density) and 5%
small full fits go through nmf_server_*.  First every request is submitted at
once (saturated: fold-in columns solved per second), then the same mix
arrives as a Poisson stream at each of --serve-loads times the saturated
request rate, --serve-requests measured after --serve-warmup warm-up
requests, and the per-request latencies (submission to completion) give
p50/p99.  "foldin_solve" is the fold-in's solve kernel alone on 8192 request
columns: its kbar and lane operations per second against the VALU peak.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--cpu-iters T]
                       [--no-serve] [--serve-requests N] [--serve-warmup N] [--serve-loads a,b,c]
       python bench.py --calibrate-copy   (1 GiB device copy, for counter scaling)
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_LANE_OPS = 256 * 64 * 2.4e9  # VALU lane operations / s (no packed math)
METRIC = "column NNLS solves/s at r=100 vs roofline; p50/p99 fold-in latency at 1 GPU"


def init_ops(r):
    """Lane operations of Algorithm 3's start per column, counted exactly:
    q = h / sqrt(d), y = x0 sqrt(d), g = Q y + q and ||pg_0||^2."""
    return r * r + 5 * r


def iter_ops(r):
    """Lane operations of one iteration of Algorithm 3 per column, counted
    exactly: the projected gradient and its norm 2r, Q pg r^2, pg'Q pg r,
    the projected step 3r, Q delta r^2, the guard 2r, the y and g updates
    2r, r CD steps of 5r + 1 each, the stop test 2r."""
    return 7 * r * r + 13 * r


def init_ops_agreed(r):
    """The same start in the scope's count of algorithmic work: r^2 (the warm
    start's Q y)."""
    return r * r


def iter_ops_agreed(r):
    """One iteration in the scope's count: 11 r^2 + 11 r (the line search about
    2 r^2, the r CD steps about 9 r^2: every coordinate's step, decrease and
    comparison plus the gradient update, each weighted as in that count)."""
    return 11 * r * r + 11 * r


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


def summary_fields(name):
    """The "- key: value" lines of a committed counter summary (empty if absent)."""
    path = os.path.join(ROOT, "profiles", name)
    fields = {}
    if os.path.exists(path):
        with open(path) as f:
            for line in f:
                if line.startswith("- ") and ": " in line:
                    k, v = line[2:].split(": ", 1)
                    fields[k.strip()] = v.strip().strip("`")
    return fields


def sources_hash(rels):
    import hashlib
    h = hashlib.sha256()
    for rel in rels:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, L):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when there is none or the kernel's sources changed since."""
    fields = summary_fields("k_nqp_sparse_r100_hbm_traffic.md")
    if fields.get("kernel") != kernel or fields.get("source_sha256") != kernel_source_hash(L):
        return None
    return float(fields["traffic_bytes_per_launch"])


def measured_product_traffic():
    """HBM bytes per step of the sparse product phase (k_spmm both halves and
    the hot columns' k_dense) from the committed counter summary, or None when
    there is none or their sources (or the plan's column split) changed since."""
    fields = summary_fields("product_phase_sparse_r100_hbm_traffic.md")
    # the kernels, and the plan that splits the columns between them
    src = ["paper_1506_08938_amd/csrc/k_spmm.hip", "paper_1506_08938_amd/csrc/k_dense.hip",
           "paper_1506_08938_amd/csrc/fit.hip", "paper_1506_08938_amd/build.py"]
    if fields.get("kernel") != "product phase" or fields.get("source_sha256") != sources_hash(src):
        return None
    return float(fields["traffic_bytes_per_step"])


def foldin_solve_roofline(native, synth, torch, W, m, r, seed, ncols=8192):
    """The fold-in's solve kernel alone (Algorithm 3 from x0 = 0 against the resident basis'
    Gram), on the configured request columns: kbar, and lane operations per second against the
    VALU peak, timed with HIP events on the stream the kernel runs on."""
    import numpy as np
    l1 = 0.05
    G = native.gram(W, 0.0)
    req = synth.foldin_columns_many(m, ncols, 500, seed)
    P = native.product(native.sparse_request(req, m), W, 0)   # (c x r) = (W' Vnew)'
    h = (l1 - P).contiguous()
    it = torch.zeros(ncols, dtype=torch.int32, device="cuda")
    opt = native.opts(max_inner=100, eps=1e-3)
    X = torch.zeros((ncols, r), device="cuda")
    native.nnls_solve_batch(G, h, X, opt, it)  # warm
    times = []
    for _ in range(5):
        X.zero_()
        a = torch.cuda.Event(enable_timing=True); b = torch.cuda.Event(enable_timing=True)
        a.record(); native.nnls_solve_batch(G, h, X, opt, it); b.record(); b.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    inner = int(it.sum().item())
    # cold start: g = q, no Q y (the agreed count's r^2 start term is the warm start's)
    ops = inner * iter_ops_agreed(r)
    E, L = native.layout(r, ncols)
    return {"kernel": f"k_nqp<{E}, {L}> (Algorithm 3 from x0 = 0)", "columns": ncols, "r": r,
            "kbar": inner / ncols, "ms": ms, "solves_per_s": ncols / (ms / 1e3),
            "achieved": ops / (ms / 1e3), "peak": PEAK_LANE_OPS, "unit": "lane-ops/s",
            "frac": ops / (ms / 1e3) / PEAK_LANE_OPS,
            "ops_count": "per column k (11 r^2 + 11 r), k its inner iterations"}


def serving_leg(native, synth, torch, n_req, loads=(0.5,), seed=5005, n_warm=None, batch_cols=16384,
                foldin_solve=False, slots=3):
    """Saturated throughput and Poisson-arrival latency of nmf_server_* at each offered load
    (a fraction of the saturated request rate)."""
    import numpy as np
    loads = tuple(loads) if isinstance(loads, (tuple, list)) else (loads,)
    n_warm = n_req // 10 if n_warm is None else n_warm
    t_setup = time.perf_counter()
    wb = synth.workload5_basis()
    m, r = wb["V"].shape[0], wb["r"]
    Vb = native.DeviceMatrix(torch.from_numpy(wb["V"]).cuda())
    W = torch.from_numpy(wb["W0"]).cuda()
    Ht = torch.from_numpy(wb["Ht0"]).cuda()
    native.fit(Vb, r, native.reg(), native.opts(max_outer=20), W, Ht, want_trace=False)
    del Vb, Ht
    basis = native.Basis(W, l1=0.05, l2=0.0, opt=native.opts(max_inner=100, eps=1e-3))
    fsolve = foldin_solve_roofline(native, synth, torch, W, m, r, seed + 4242) if foldin_solve else None
    # a pool of distinct requests, reused by the arrivals (each arrival has its own output)
    n_pool = 96
    sizes = synth.request_sizes(n_pool, seed, cmax=8192)
    pool_csr = [synth.foldin_columns_many(m, int(c), 500, seed + 1 + i) for i, c in enumerate(sizes)]
    pool = [native.sparse_request(q, m) for q in pool_csr]
    fits = synth.workload5_fits(8)
    fit_V = [torch.from_numpy(f["V"]).cuda() for f in fits]
    total = n_warm + n_req
    g = synth.rng(seed + 999)
    is_fit = g.random(total) < 0.05
    pick = g.integers(0, n_pool, total)
    fpick = g.integers(0, len(fits), total)
    csize = np.array([0 if is_fit[i] else int(sizes[pick[i]]) for i in range(total)])
    fit_opt = native.opts(max_outer=30)
    outs = [None] * total
    for i in range(total):
        if not is_fit[i]:
            outs[i] = torch.empty((int(csize[i]), r), device="cuda")

    def reset_fits():
        for i in range(total):
            if is_fit[i]:
                f = fits[fpick[i]]
                outs[i] = (torch.from_numpy(f["W0"]).cuda(), torch.from_numpy(f["Ht0"]).cuda())
        torch.cuda.synchronize()

    def submit(S, i):
        if is_fit[i]:
            f = fits[fpick[i]]
            return S.submit_fit(fit_V[fpick[i]], f["r"], native.reg(), fit_opt, *outs[i])
        return S.submit_foldin(pool[pick[i]], outs[i])

    def run(arrivals):
        """All requests at once (arrivals None) or at the given times; returns the elapsed
        time of the measured requests and their latencies."""
        reset_fits()
        S = native.Server(basis, hbm_budget=8 << 30, max_slots=slots, max_batch_cols=batch_cols)
        tickets = []
        lag = np.zeros(total)  # how late each submission left the load generator (s)
        # A full pass of Python's garbage collector inside the submission loop
        # stalls the load generator for tens of milliseconds, and the overdue
        # requests then arrive as one burst: it is kept out of the timed loop.
        gc.collect()
        gc.disable()
        try:
            t0 = time.perf_counter()
            t_first = None
            for i in range(total):
                if arrivals is not None:
                    while time.perf_counter() - t0 < arrivals[i]:
                        pass
                    lag[i] = time.perf_counter() - t0 - arrivals[i]
                if i == n_warm:
                    t_first = time.perf_counter()
                tickets.append(submit(S, i))
            S.wait()
            t_end = time.perf_counter()
        finally:
            gc.enable()
        tl = np.array([S.poll_times(t)[1] for t in tickets])  # queued, launch, device, latency (ms)
        st = S.stats()
        S.close()
        st["submit_lag_ms"] = {"p99": float(np.percentile(lag[n_warm:], 99) * 1e3),
                               "max": float(lag[n_warm:].max() * 1e3)}
        return t_end - t_first, tl[n_warm:], st

    meas = slice(n_warm, total)
    cols = int(csize[meas].sum())
    fold = ~is_fit[meas]
    log(f"[bench] serving set up in {time.perf_counter() - t_setup:.1f}s; {n_req} measured requests "
        f"after {n_warm} warm-up, {cols} fold-in columns, {int(is_fit[meas].sum())} fits")
    run(None)  # warm-up pass
    el_sat, _, st_sat = run(None)
    rate_sat = n_req / el_sat
    log(f"[bench] serving saturated {el_sat * 1e3:.1f} ms ({rate_sat:.0f} req/s)")
    # The fold-in products gather one basis row (r floats) per stored entry of
    # a request; at saturation, against the gather probe's rate for as many
    # uniformly random rows of the same basis (the fits share the window, so
    # this is a lower bound of the fold-ins' own rate).
    nnz_meas = int(sum(pool_csr[pick[i]].nnz for i in range(n_warm, total) if not is_fit[i]))
    gathered = nnz_meas * r * 4
    idx = torch.from_numpy(synth.rng(seed + 31).integers(0, m, min(nnz_meas, 1 << 25)).astype(np.int32)).cuda()
    pout = torch.empty(native.PROBE_GATHER_OUT_FLOATS, device="cuda")
    for _ in range(2):
        native.probe_gather(W, idx, pout)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(5):
        native.probe_gather(W, idx, pout)
    ev[1].record()
    torch.cuda.synchronize()
    probe_rate = idx.numel() * r * 4 / (ev[0].elapsed_time(ev[1]) / 5 / 1e3)
    gather_bound = {"gathered_bytes": gathered, "saturated_bytes_per_s": gathered / el_sat,
                    "probe_bytes_per_s": probe_rate, "frac_of_probe": gathered / el_sat / probe_rate,
                    "note": "fold-in products' basis-row gathers at saturation over the gather probe's rate for "
                            "uniformly random rows of the same basis"}
    del idx, pout
    per_load = []
    for k, ld in enumerate(loads):
        rate = ld * rate_sat
        arrivals = synth.poisson_arrivals(total, rate, seed + 7 + k)
        el, tl, st = run(arrivals)
        lat = tl[:, 3]
        lf = lat[fold]
        # where the slowest 1% of fold-in requests spent their time
        slow = tl[fold][lf >= np.percentile(lf, 99)]
        tail = {"queued_ms": float(np.median(slow[:, 0])), "launch_ms": float(np.median(slow[:, 1])),
                "device_ms": float(np.median(slow[:, 2]))}
        sz = csize[meas][fold]
        edges = np.quantile(sz, np.linspace(0, 1, 11))
        dec = []
        for d in range(10):
            sel = (sz >= edges[d]) & ((sz < edges[d + 1]) if d < 9 else (sz <= edges[d + 1]))
            if sel.any():
                dec.append({"cols": [int(sz[sel].min()), int(sz[sel].max())], "n": int(sel.sum()),
                            "p50_ms": float(np.percentile(lf[sel], 50)),
                            "p99_ms": float(np.percentile(lf[sel], 99))})
        per_load.append({
            "load": ld, "arrival_rate_req_per_s": rate, "solves_per_s": cols / el,
            "requests_per_s": n_req / el,
            "fold_in_p50_ms": float(np.percentile(lf, 50)), "fold_in_p99_ms": float(np.percentile(lf, 99)),
            "fit_p50_ms": float(np.percentile(lat[~fold], 50)) if (~fold).any() else None,
            "batches": st["batches"], "p99_tail_median_breakdown": tail, "by_size_decile": dec,
            "submit_lag_ms": st["submit_lag_ms"]})
        log(f"[bench] load {ld}: {rate:.0f} req/s, fold-in p50 {per_load[-1]['fold_in_p50_ms']:.3f} ms "
            f"p99 {per_load[-1]['fold_in_p99_ms']:.3f} ms")
    basis.close()
    res = {
        "workload": "resident basis W 100000x128 (20 outer iterations fitted on the device to "
                    "2048 columns of Gamma(2,0.5)-factor data), L1=0.05, eps=1e-3; fold-in requests of "
                    "c~logU[1,8192] columns at 0.5% density, values log(1+Poisson(3)); 5% small "
                    f"full fits (m,n~logU[64,2048], r~U{{4..32}}, 30 outer iterations); {slots} slots, "
                    f"batches of up to {batch_cols} columns",
        "requests": n_req, "warmup_requests": n_warm,
        "fold_in_columns": cols,
        "saturated_solves_per_s": cols / el_sat,
        "saturated_requests_per_s": rate_sat,
        "saturated_ms": el_sat * 1e3,
        "saturated_batches": st_sat["batches"],
        "saturated_gathers": gather_bound,
        "loads": per_load,
    }
    if fsolve is not None:
        res["foldin_solve"] = fsolve
    if len(per_load) == 1:  # the headline line's short form
        res.update({k: per_load[0][k] for k in ("fold_in_p50_ms", "fold_in_p99_ms", "fit_p50_ms")})
        res["load"] = per_load[0]["load"]
    return res


def base_line(metric, value, unit, K, W, ms, dtype, config, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": K, "warmup": W,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": dtype, "data": "synthetic", "config": config}
    out.update(extra)
    return out


def timed_plan(native, torch, Vd, r, reg, opt, W0, Ht0, K, warm):
    """ms per outer iteration and per-phase ms of a plan on fresh copies of the start point."""
    plan = native.Plan(Vd, r, reg, opt)
    W = W0.clone(); Ht = Ht0.clone()
    for _ in range(warm):
        plan.run(W, Ht, 1)
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = plan.run(W, Ht, K, want_stats=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tm = plan.timers()
    plan.close()
    return el * 1e3 / K, {k: v[0] / K for k, v in tm.items()}, {k: v for k, v in tm.items()}, st


def bench_dense(args, native, synth, torch, np):
    """Dense workload (V 20000x10000 = Gamma-factor low rank + |N(0, 0.05)|, r = 64, L2 = 0.01 on
    both factors): FP32 against BF16 products, per outer iteration and at equal objective
    accuracy on the 2000x1000 slice (J* = the FP64 oracle's J after 100 iterations)."""
    K, Wm = args.steps, args.warmup
    log("[bench] generating the dense workload")
    wl = synth.workload2()
    m, n = wl["V"].shape
    r = wl["r"]
    V = torch.from_numpy(wl["V"]).cuda()
    Vd = native.DeviceMatrix(V)
    reg = native.reg(*wl["reg"])
    W0 = torch.from_numpy(wl["W0"]).cuda()
    H0 = torch.from_numpy(wl["Ht0"]).cuda()
    modes = {}
    for prec, name in ((0, "fp32"), (1, "bf16")):
        ms, ph, tm, st = timed_plan(native, torch, Vd, r, reg,
                                    native.opts(max_inner=100, eps=1e-3, precision=prec, lanes=args.lanes),
                                    W0, H0, K, Wm)
        vbytes = (4 if prec == 0 else 2) * m * n
        # per product launch: V once, the fixed factor once, the output once
        prod_bytes = vbytes + 4 * (m + n) * r // 2 + 4 * (m + n) * r // 2
        prod_ms = tm["product"][0] / tm["product"][1]
        gram_ms = tm["gram"][0] / tm["gram"][1]
        modes[name] = {
            "ms_per_step": ms, "solves_per_s": (m + n) / (ms / 1e3), "phases_ms_per_step": ph,
            "product_avg_ms": prod_ms,
            "product_hbm_GBps": prod_bytes / (prod_ms / 1e3) / 1e9,
            "product_frac_of_8TBps": prod_bytes / (prod_ms / 1e3) / 8e12,
            "product_tflops": 2.0 * m * n * r / (prod_ms / 1e3) / 1e12,
            "gram_avg_ms": gram_ms,
            "gram_GBps": 4.0 * (m + n) / 2 * r / (gram_ms / 1e3) / 1e9,
            "kbar": st["kbar"], "loss_after": st["loss"],
        }
        log(f"[bench] dense {name}: {ms:.3f} ms/step, product {prod_ms:.3f} ms")
    del Vd, V
    if args.skip_accuracy:
        out = base_line(
            "dense NMF column NNLS solves/s (FP32 and BF16 products)",
            modes["bf16"]["solves_per_s"], "column NNLS solves/s", K, Wm, modes["bf16"]["ms_per_step"], "bf16",
            {"workload": "dense V 20000x10000 = W0 H0 + |N(0,0.05)|, W0, H0 ~ Gamma(2,0.5) of inner dimension 64; "
                         "r=64, L2=0.01 on W and H; eps=1e-3, max_inner=100; one step = one outer iteration; "
                         "value = the BF16-product mode", "m": m, "n": n, "r": r},
            modes=modes)
        print(json.dumps(out), flush=True)
        return
    # equal accuracy on the slice
    import oracle
    sl = synth.workload2_slice()
    T_or = 100
    log("[bench] oracle: 100 outer iterations on the 2000x1000 slice")
    t0 = time.perf_counter()
    o = oracle.nmf_fit(sl["V"], r, sl["reg"], sl["W0"], sl["Ht0"], T=T_or, max_inner=100, eps=1e-3,
                       ls_guard=1, want_trace=True)
    t_or = time.perf_counter() - t0
    Jstar = float(o["jhalf"][-1])
    Vs = native.DeviceMatrix(torch.from_numpy(sl["V"]).cuda())
    regs = native.reg(*sl["reg"])
    acc = {}
    Tmax = 3 * T_or
    for prec, name in ((0, "fp32"), (1, "bf16")):
        plan = native.Plan(Vs, r, regs, native.opts(max_inner=100, eps=1e-3, precision=prec))
        W = torch.from_numpy(sl["W0"]).cuda(); Ht = torch.from_numpy(sl["Ht0"]).cuda()
        Js = []
        for t in range(Tmax):
            plan.run(W, Ht, 1)
            Js.append(native.objective(Vs, r, regs, W, Ht)[1])
        ms_slice, _, _, _ = timed_plan(native, torch, Vs, r, regs,
                                       native.opts(max_inner=100, eps=1e-3, precision=prec),
                                       torch.from_numpy(sl["W0"]).cuda(), torch.from_numpy(sl["Ht0"]).cuda(),
                                       20, 2)
        plan.close()
        reach = {}
        for d in (1e-2, 1e-3, 1e-4):
            it = next((i + 1 for i, J in enumerate(Js) if J <= Jstar * (1 + d)), None)
            reach[f"{d:g}"] = {"iterations": it, "ms": None if it is None else it * ms_slice}
        acc[name] = {"J_at_100_over_Jstar": Js[T_or - 1] / Jstar, "J_floor_over_Jstar": min(Js) / Jstar,
                     "ms_per_iteration": ms_slice, "reach": reach}
        log(f"[bench] slice {name}: J(100)/J* = {Js[T_or - 1] / Jstar:.6f}")
    fp, bf = modes["fp32"], modes["bf16"]
    out = base_line(
        "dense NMF column NNLS solves/s (FP32 and BF16 products) and time to equal objective accuracy",
        bf["solves_per_s"], "column NNLS solves/s", K, Wm, bf["ms_per_step"], "bf16",
        {"workload": "dense V 20000x10000 = W0 H0 + |N(0,0.05)|, W0, H0 ~ Gamma(2,0.5) of inner "
                     "dimension 64; r=64, L2=0.01 on W and H; eps=1e-3, max_inner=100; one step = one "
                     "outer iteration; value = the BF16-product mode", "m": m, "n": n, "r": r},
        modes=modes,
        equal_accuracy={"slice": "V[:2000, :1000] of the same data as its own problem",
                        "Jstar": Jstar, "oracle_iterations": T_or, "oracle_s": t_or,
                        "oracle_threads": oracle.num_threads(), "modes": acc},
    )
    print(json.dumps(out), flush=True)


def bench_batched(args, native, synth, torch, np):
    """1024 uneven dense problems, 30 outer iterations each: one nmf_fit_batched call (a
    captured hipGraph of all iterations) against a loop of per-problem nmf_fit calls."""
    count, T = 1024, 30
    log("[bench] generating 1024 problems")
    t0 = time.perf_counter()
    probs = synth.workload4(count=count)
    log(f"[bench] generated in {time.perf_counter() - t0:.1f}s")
    dev = [dict(V=torch.from_numpy(p["V"]).cuda(), r=p["r"], W0=torch.from_numpy(p["W0"]).cuda(),
                Ht0=torch.from_numpy(p["Ht0"]).cuda()) for p in probs]
    torch.cuda.synchronize()
    cols = sum(p["V"].shape[0] + p["V"].shape[1] for p in probs)
    vbytes = sum(4 * p["V"].size for p in probs)
    res = {}
    for prec, name in ((1, "bf16"), (0, "fp32")):
        opt = native.opts(max_outer=T, max_inner=100, eps=1e-3, precision=prec,
                          fast_break_cols=args.fast_break)
        best = None
        for rep in range(2):
            batch = [dict(V=d["V"], r=d["r"], reg=native.reg(), W=d["W0"].clone(), Ht=d["Ht0"].clone())
                     for d in dev]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            native.fit_batched(batch, opt, want_stats=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
        # the same run with statistics (identical arithmetic) for the iteration counts
        st = native.fit_batched([dict(V=d["V"], r=d["r"], reg=native.reg(), W=d["W0"].clone(),
                                      Ht=d["Ht0"].clone()) for d in dev], opt)
        ops = sum((p["V"].shape[0] + p["V"].shape[1]) * T * init_ops(p["r"]) + x["inner_total"] * iter_ops(p["r"])
                  for p, x in zip(probs, st))
        # HBM floor: V read twice per outer iteration (BF16 copies: 2 bytes, FP32: 4)
        vb = vbytes // 2 if prec == 1 else vbytes
        t_valu = ops / PEAK_LANE_OPS
        t_hbm = 2 * vb * T / 8e12
        res[name] = {"batched_s": best, "solves_per_s": cols * T / best,
                     "problems_per_s": count / best,
                     "kbar": float(sum(x["inner_total"] for x in st)) / (cols * T),
                     "solve_lane_ops": ops, "t_valu_floor_s": t_valu, "t_hbm_floor_s": t_hbm,
                     "roofline_frac": max(t_valu, t_hbm) / best}
        log(f"[bench] batched {name}: {best:.3f}s")
    # per-problem baseline: plain FP32 nmf_fit calls, one after another
    opt = native.opts(max_outer=T, max_inner=100, eps=1e-3, precision=0)
    for d in dev[:8]:  # warm the per-shape code paths
        native.fit(native.DeviceMatrix(d["V"]), d["r"], native.reg(), native.opts(max_outer=1),
                   d["W0"].clone(), d["Ht0"].clone(), want_trace=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inner = 0
    for d in dev:
        _, st = native.fit(native.DeviceMatrix(d["V"]), d["r"], native.reg(), opt, d["W0"].clone(),
                           d["Ht0"].clone(), want_trace=False)
    torch.cuda.synchronize()
    base = time.perf_counter() - t0
    log(f"[bench] per-problem loop: {base:.3f}s")
    # roofline of one batched outer iteration: V read twice (BF16 copy: 2 bytes per entry)
    b = res["bf16"]
    t_hbm = 2 * (vbytes // 2) / 8e12
    out = base_line(
        "batched uneven NMF: column NNLS solves/s in one graph-captured launch sequence vs per-problem fits",
        b["solves_per_s"], "column NNLS solves/s", T, 0, b["batched_s"] * 1e3 / T, "bf16",
        {"workload": "1024 dense problems, m~logU[64,4096], n~logU[64,2048], r~U{4..64}, V = W0 H0 + "
                     "|N(0,0.01)| with U[0,1] factors, FP32 storage; 30 outer iterations each; one step = "
                     "one outer iteration of all problems; value = BF16 products, batched",
         "problems": count, "columns_per_iteration": cols, "V_bytes_fp32": vbytes},
        modes=res,
        per_problem_fp32_s=base,
        speedup_bf16_batched_vs_per_problem_fp32=base / b["batched_s"],
        speedup_fp32_batched_vs_per_problem_fp32=base / res["fp32"]["batched_s"],
        hbm_floor_ms_per_step=t_hbm * 1e3,
    )
    print(json.dumps(out), flush=True)


def gather_probe(native, synth, torch, np, V, r, bf16_case=True, uniform_case=True):
    """Times the gather probe (nothing but the row loads of the sparse
    products) on the headline workload's access orders: W rows in the
    H-update's order (CSR(V') of the columns outside the plan's hot set) and
    Ht rows in the W-update's order (CSR(V)), FP32 rows of r floats; optionally
    W rows as BF16 (rows padded to 8 values) and uniformly random W rows."""
    m, n = V.shape
    # the plan's hot columns: c_j >= max(m/24, 256) entries, the longest first,
    # all up to 127, else 128 or 256 of them
    cnt = np.bincount(V.indices, minlength=n)
    thr = max((m + 23) // 24, 256)
    cand = np.nonzero(cnt >= thr)[0]
    cand = cand[np.argsort(-cnt[cand], kind="stable")]
    if cand.size >= 128:
        cand = cand[: min(cand.size, 256) // 128 * 128]
    hot = np.zeros(n, bool)
    if cand.size >= 4:
        hot[cand] = True
    Vc = V.tocsc()
    keep = np.repeat(~hot, np.diff(Vc.indptr))
    idx_h = Vc.indices[keep].astype(np.int32)  # CSR(V') order, cold columns
    idx_w = V.indices.astype(np.int32)          # CSR(V) order
    # the probe's rate does not depend on the values it reads
    W = torch.ones((m, r), device="cuda")
    Ht = torch.ones((n, r), device="cuda")
    cases = [("h_update", "H-update order, W rows FP32", W, idx_h),
             ("w_update", "W-update order, Ht rows FP32", Ht, idx_w)]
    if bf16_case:
        W16 = torch.ones((m, (r + 7) // 8 * 8), dtype=torch.bfloat16, device="cuda")
        cases.append(("h_update_bf16", "H-update order, W rows BF16", W16, idx_h))
    if uniform_case:
        idx_u = synth.rng(4711).integers(0, m, idx_h.size).astype(np.int32)
        cases.append(("uniform", "uniformly random W rows FP32", W, idx_u))
    out = torch.empty(native.PROBE_GATHER_OUT_FLOATS, device="cuda")
    res = {}
    for key, name, table, idx in cases:
        d = torch.from_numpy(idx).cuda()
        for _ in range(3):
            native.probe_gather(table, d, out)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        K = 10
        ev[0].record()
        for _ in range(K):
            native.probe_gather(table, d, out)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / K
        row_bytes = int(table.shape[1] * table.element_size())
        nbytes = idx.size * row_bytes
        res[key] = dict(case=name, rows=int(table.shape[0]), row_bytes=row_bytes, gathers=int(idx.size),
                        gathered_bytes=int(nbytes), ms=ms, bytes_per_s=nbytes / ms * 1e3)
        log(f"[bench] probe, {name} ({row_bytes} B rows): {idx.size} rows, {nbytes / 1e9:.2f} GB in "
            f"{ms:.3f} ms = {nbytes / ms / 1e9:.2f} TB/s")
    return res, int(hot.sum())


def bench_gather_ceiling(args, native, synth, torch, np):
    """The row-gather ceiling of the sparse products on the headline workload
    (gather_probe, all four cases)."""
    log("[bench] generating the sparse workload")
    wl = synth.workload3()
    res, nhot = gather_probe(native, synth, torch, np, wl["V"], wl["r"])
    print(json.dumps({"metric": "row-gather ceiling of the sparse products (probe)", "unit": "B/s",
                      "data": "synthetic", "hot_columns": nhot,
                      "config": {"workload": "sparse text-like CSR V 200000x100000 (the headline workload), r=100"},
                      "cases": res}), flush=True)


def bench_streamed(args, native, synth, torch, np):
    """Limited internal memory: workload 2 (V 20000x10000 FP32, 800 MB) kept in page-locked host
    memory and streamed to the device in panels of instances, one read of V per outer iteration
    (nmf_fit_streamed); against the host-to-device copy rate and the resident FP32 fit."""
    K, Wm = args.steps, args.warmup
    panel = args.panel_cols
    log("[bench] generating the dense workload")
    wl = synth.workload2()
    m, n = wl["V"].shape
    r = wl["r"]
    Vh = torch.from_numpy(wl["V"]).pin_memory()
    reg = native.reg(*wl["reg"])
    vbytes = 4 * m * n
    # the host-to-device rate of one whole copy of V (median of 3)
    dst = torch.empty((m, n), dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream()
    ts = []
    for _ in range(3):
        a = torch.cuda.Event(enable_timing=True); b = torch.cuda.Event(enable_timing=True)
        a.record(s); dst.copy_(Vh, non_blocking=True); b.record(s); b.synchronize()
        ts.append(a.elapsed_time(b))
    copy_ms = sorted(ts)[1]
    h2d = vbytes / (copy_ms / 1e3)
    log(f"[bench] host-to-device copy of V: {copy_ms:.2f} ms ({h2d / 1e9:.1f} GB/s)")
    # resident FP32 fit for comparison (V already on the device)
    W0 = torch.from_numpy(wl["W0"]).cuda(); H0 = torch.from_numpy(wl["Ht0"]).cuda()
    res_ms, _, _, _ = timed_plan(native, torch, native.DeviceMatrix(dst), r, reg,
                                 native.opts(max_inner=100, eps=1e-3), W0, H0, K, Wm)
    del dst
    torch.cuda.empty_cache()
    opt_w = native.opts(max_outer=Wm, max_inner=100, eps=1e-3)
    opt = native.opts(max_outer=K, max_inner=100, eps=1e-3)
    W = W0.clone(); Ht = H0.clone()
    if Wm:
        native.fit_streamed(Vh, r, reg, opt_w, W, Ht, panel, want_trace=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = native.fit_streamed(Vh, r, reg, opt, W, Ht, panel, want_trace=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1e3 / K
    # device buffers beyond W and Ht: two panels, P_W and its per-panel addend, the panel product
    ldp = (min(panel, n) + 3) // 4 * 4
    dev_bytes = 4 * (2 * m * ldp + 2 * m * r + min(panel, n) * r)
    log(f"[bench] streamed: {ms:.2f} ms/step (copy floor {copy_ms * (K + 1) / K:.2f} ms), resident {res_ms:.2f} ms")
    out = base_line(
        "limited-memory dense NMF: column NNLS solves/s with V streamed from host memory",
        (m + n) * K / el, "column NNLS solves/s", K, Wm, ms, "f32",
        {"workload": "dense V 20000x10000 = W0 H0 + |N(0,0.05)|, Gamma(2,0.5) factors of inner dimension "
                     "64, FP32 in page-locked host memory; r=64, L2=0.01 on W and H; eps=1e-3, "
                     f"max_inner=100; panels of {panel} instances (columns of V); one step = one outer "
                     "iteration (one read of V); the run's statistics add one more read",
         "m": m, "n": n, "r": r, "panel_cols": panel},
        V_bytes=vbytes, device_buffer_bytes=dev_bytes, h2d_copy_GBps=h2d / 1e9,
        copy_floor_ms_per_step=copy_ms * (K + 1) / K, frac_of_copy_floor=copy_ms * (K + 1) / K / ms,
        resident_fp32_ms_per_step=res_ms, kbar=st["kbar"], loss_after=st["loss"],
    )
    print(json.dumps(out), flush=True)


def bench_sparse_accuracy(args, native, synth, torch, np):
    """The sparse text-like workload: float32 against BF16 products at equal objective accuracy.
    J* = the FP64 oracle's objective J after --accuracy-iters outer iterations from the same start
    point (the oracle on the host cores); each GPU mode runs up to three times as many outer
    iterations, J evaluated in FP64 after each, and reports the iterations and time it needs to
    reach J <= J* (1 + d) for d = 1e-2, 1e-3, 1e-4 (None: never within the run)."""
    import oracle
    wl = synth.workload3()
    V = wl["V"]
    m, n = V.shape
    r = wl["r"]
    T_or = args.accuracy_iters
    log(f"[bench] oracle: {T_or} outer iterations of the {m}x{n} sparse workload on {oracle.num_threads()} threads")
    regs32 = tuple(float(np.float32(x)) for x in wl["reg"])  # the weights the library receives
    t0 = time.perf_counter()
    o = oracle.nmf_fit(V, r, regs32, wl["W0"], wl["Ht0"], T=T_or, max_inner=100, eps=1e-3, ls_guard=1,
                       want_trace=False)
    t_or = time.perf_counter() - t0
    Jstar = float(oracle.objective(V, o["W"], o["Ht"], regs32))
    log(f"[bench] oracle {t_or:.1f}s, J* = {Jstar:.8e}")
    Vd = native.DeviceMatrix(V, with_transpose=False)
    reg = native.reg(*wl["reg"])
    acc = {}
    for prec, name in ((0, "fp32"), (1, "bf16")):
        opt = native.opts(max_inner=100, eps=1e-3, precision=prec)
        ms, _, _, _ = timed_plan(native, torch, Vd, r, reg, opt, torch.from_numpy(wl["W0"]).cuda(),
                                 torch.from_numpy(wl["Ht0"]).cuda(), 20, 2)
        plan = native.Plan(Vd, r, reg, opt)
        W = torch.from_numpy(wl["W0"]).cuda(); Ht = torch.from_numpy(wl["Ht0"]).cuda()
        Js = []
        for t in range(3 * T_or):
            plan.run(W, Ht, 1)
            Js.append(native.objective(Vd, r, reg, W, Ht)[1])
        plan.close()
        reach = {}
        for d in (1e-2, 1e-3, 1e-4):
            it = next((i + 1 for i, J in enumerate(Js) if J <= Jstar * (1 + d)), None)
            reach[f"{d:g}"] = {"iterations": it, "ms": None if it is None else it * ms}
        acc[name] = {"ms_per_iteration": ms, f"J_at_{T_or}_over_Jstar": Js[T_or - 1] / Jstar,
                     "J_floor_over_Jstar": min(Js) / Jstar, "reach": reach}
        log(f"[bench] {name}: J({T_or})/J* = {Js[T_or - 1] / Jstar:.6f}, {ms:.3f} ms/iteration")
    fp, bf = acc["fp32"], acc["bf16"]
    out = base_line(
        "sparse NMF: time to equal objective accuracy, float32 against BF16 products",
        (m + n) / (bf["ms_per_iteration"] / 1e3), "column NNLS solves/s", 20, 2, bf["ms_per_iteration"], "bf16",
        {"workload": "sparse text-like CSR V 200000x100000 (0.1% density, Zipf(1.1) columns, log(1+Poisson(3)) "
                     "values), r=100, L1=0.1 on H, L2=0.01 on W, eps=1e-3; J* = the FP64 oracle's J after "
                     f"{T_or} outer iterations from the same start; value = the BF16-product mode",
         "m": m, "n": n, "r": r},
        equal_accuracy={"Jstar": Jstar, "oracle_iterations": T_or, "oracle_s": t_or,
                        "oracle_threads": oracle.num_threads(), "modes": acc})
    print(json.dumps(out), flush=True)


def bench_single_pass(args, native, synth, torch, np):
    """Algorithm 2's single pass over a V resident in HBM (nmf_fit_single_pass: the M-step's data
    term summed over instance panels while the E-step solves them, V read from memory once per
    outer iteration) against the two-pass resident fit (nmf_plan_run: V read once per half), on
    the dense workload in FP32."""
    K, Wm = args.steps, args.warmup
    panel = args.panel_cols
    log("[bench] generating the dense workload")
    wl = synth.workload2()
    m, n = wl["V"].shape
    r = wl["r"]
    Vd = native.DeviceMatrix(torch.from_numpy(wl["V"]).cuda())
    reg = native.reg(*wl["reg"])
    W0 = torch.from_numpy(wl["W0"]).cuda(); H0 = torch.from_numpy(wl["Ht0"]).cuda()
    opt = native.opts(max_inner=100, eps=1e-3)
    two_ms, ph, _, st2 = timed_plan(native, torch, Vd, r, reg, opt, W0, H0, K, Wm)
    W = W0.clone(); Ht = H0.clone()
    if Wm:
        native.fit_single_pass(Vd, r, reg, native.opts(max_outer=Wm, max_inner=100, eps=1e-3), W, Ht, panel,
                               want_trace=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = native.fit_single_pass(Vd, r, reg, native.opts(max_outer=K, max_inner=100, eps=1e-3), W, Ht, panel,
                                   want_trace=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / K
    log(f"[bench] single pass {ms:.3f} ms/step (panels of {panel}), two-pass {two_ms:.3f} ms/step")
    out = base_line(
        "dense NMF, single pass over resident V: column NNLS solves/s",
        (m + n) / (ms / 1e3), "column NNLS solves/s", K, Wm, ms, "f32",
        {"workload": "dense V 20000x10000 = W0 H0 + |N(0,0.05)|, Gamma(2,0.5) factors of inner dimension 64, "
                     "FP32 resident in HBM; r=64, L2=0.01 on W and H; eps=1e-3, max_inner=100; "
                     f"panels of {panel} instances; one step = one outer iteration (V read once); the run's "
                     "statistics add one more read", "m": m, "n": n, "r": r, "panel_cols": panel},
        two_pass_ms_per_step=two_ms, two_pass_phases_ms=ph, V_bytes=4 * m * n,
        hbm_floor_ms_single=4 * m * n / 8e12 * 1e3, hbm_floor_ms_two_pass=2 * 4 * m * n / 8e12 * 1e3,
        kbar=st["kbar"], kbar_two_pass=st2["kbar"], loss_after=st["loss"], loss_after_two_pass=st2["loss"])
    print(json.dumps(out), flush=True)


def bench_serving(args, native, synth, torch, np):
    """The serving configuration at several offered loads."""
    loads = (0.3, 0.6, 0.9)
    res = serving_leg(native, synth, torch, args.serve_requests, loads, n_warm=args.serve_warmup,
                      batch_cols=args.serve_batch_cols, foldin_solve=True, slots=args.serve_slots)
    out = base_line(
        "fold-in serving: column NNLS solves/s and p50/p99 latency at offered loads",
        res["saturated_solves_per_s"], "column NNLS solves/s", args.serve_requests, 0,
        res["saturated_ms"], "f32", {"workload": res["workload"]}, serving=res)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=8,
                    help="outer iterations of the CPU-oracle sample")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=20000,
                    help="measured requests per offered load")
    ap.add_argument("--serve-warmup", type=int, default=1000, help="warm-up requests before each measurement")
    ap.add_argument("--serve-loads", default="0.3,0.6,0.9",
                    help="offered loads, as fractions of the saturated request rate")
    ap.add_argument("--serve-slots", type=int, default=3,
                    help="server slots (streams; the library caps them at the hardware queues minus one)")
    ap.add_argument("--serve-batch-cols", type=int, default=16384,
                    help="largest fold-in batch (columns) the server forms")
    ap.add_argument("--accuracy-iters", type=int, default=50,
                    help="--workload sparse_accuracy: outer iterations of the oracle's reference run")
    ap.add_argument("--workload", default="sparse",
                    choices=["sparse", "dense", "batched", "serving", "streamed", "sparse_accuracy", "gather_ceiling",
                             "single_pass"],
                    help="sparse: the headline line (default); the others print supplementary lines")
    ap.add_argument("--lanes", type=int, default=0,
                    help="solve layout: lanes per column (0: the tuned table)")
    ap.add_argument("--skip-accuracy", action="store_true",
                    help="--workload dense: skip the equal-accuracy leg on the slice")
    ap.add_argument("--panel-cols", type=int, default=2048,
                    help="instances per streamed panel (--workload streamed)")
    ap.add_argument("--fast-break", type=int, default=0,
                    help="Algorithm 3's fast-break over runs of this many columns (0: off)")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16-products leg of the sparse workload")
    ap.add_argument("--no-probe", action="store_true", help="skip the gather-ceiling probe of the product phase")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"],
                    help="sparse workload: float32 products, or BF16 gathers and Gram (the solve stays float32)")
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
    if args.workload == "dense":
        return bench_dense(args, native, synth, torch, np)
    if args.workload == "batched":
        return bench_batched(args, native, synth, torch, np)
    if args.workload == "serving":
        return bench_serving(args, native, synth, torch, np)
    if args.workload == "streamed":
        return bench_streamed(args, native, synth, torch, np)
    if args.workload == "sparse_accuracy":
        return bench_sparse_accuracy(args, native, synth, torch, np)
    if args.workload == "single_pass":
        return bench_single_pass(args, native, synth, torch, np)
    if args.workload == "gather_ceiling":
        return bench_gather_ceiling(args, native, synth, torch, np)
    log("[bench] generating the sparse workload")
    t_gen = time.perf_counter()
    wl = synth.workload3()
    V = wl["V"]
    m, n = V.shape
    r = wl["r"]
    log(f"[bench] generated {m}x{n} nnz={V.nnz} in {time.perf_counter() - t_gen:.1f}s")

    Vd = native.DeviceMatrix(V, with_transpose=False)  # CSR(V') is built on the device
    reg = native.reg(*wl["reg"])
    bf16 = args.precision == "bf16"

    def timed_run(precision):
        """Plan, warm-up, the timed steps (events on the solve's own dispatches:
        nothing is added to the stream between kernels), then a separate untimed
        run with events around every phase."""
        opt = native.opts(max_inner=100, eps=1e-3, ls_guard=1, fast_break_cols=args.fast_break,
                          lanes=args.lanes, precision=precision)
        plan = native.Plan(Vd, r, reg, opt)
        W = torch.from_numpy(wl["W0"]).cuda()
        Ht = torch.from_numpy(wl["Ht0"]).cuda()
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            plan.run(W, Ht, 1)
        torch.cuda.synchronize()
        plan.profile(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = plan.run(W, Ht, args.steps, want_stats=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        timers = plan.timers()
        plan.profile(False)
        Kp = min(args.steps, 5)
        plan.profile(True)
        plan.run(W.clone(), Ht.clone(), Kp)
        torch.cuda.synchronize()
        phases = {k: v[0] / Kp for k, v in plan.timers().items()}
        plan.profile(False)
        plan.close()
        return elapsed, st, timers, phases

    elapsed, st, timers, phases = timed_run(native.NMF_BF16 if bf16 else native.NMF_FP32)
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
    ops = solves * init_ops_agreed(r) + inner_total * iter_ops_agreed(r)
    ops_exact = solves * init_ops(r) + inner_total * iter_ops(r)
    avg_launch_s = solve_ms / 1e3 / solve_calls
    achieved = ops / solve_calls / avg_launch_s
    kbar = st["kbar"]
    # the product phase (the row gathers k_spmm with its split-row fixup, and
    # the H-update's hot columns on k_dense), from the separate run with
    # events around every phase; algorithmic bytes of a CSR product:
    # 8 nnz + 4 (rows + 1) + 4 k r (the fixed factor once) + 4 c r (the output)
    nnz = int(V.nnz)
    prod_bytes = (8 * nnz + 4 * (n + 1) + 4 * m * r + 4 * n * r) + (8 * nnz + 4 * (m + 1) + 4 * n * r + 4 * m * r)
    prod_s = phases["product"] / 1e3  # both halves' product phases of one step

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
        "dtype": "bf16" if bf16 else "f32",
        "data": "synthetic",
        "config": {
            "workload": "sparse text-like CSR V 200000x100000, 100 Zipf(1.1) columns per row "
                        "(0.1% density), values log(1+Poisson(3)), r=100, L1=0.1 on H, L2=0.01 "
                        "on W, eps=1e-3, max_inner=100; one step = one outer iteration"
                        + (f"; fast-break over runs of {args.fast_break} columns" if args.fast_break > 1 else "")
                        + ("; BF16 products: row gathers from a BF16 copy of the fixed factor, the hot "
                           "columns' product and the Gram on BF16 MFMA, float32 accumulation and solve"
                           if bf16 else ""),
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
            "ops_count": "per column r^2 + k (11 r^2 + 11 r), k its inner iterations",
            "ops_per_launch_exact_count": ops_exact / solve_calls,
            "frac_exact_count": ops_exact / solve_calls / avg_launch_s / PEAK_LANE_OPS,
        },
        "product_roofline": {
            "bound": "hbm",
            "kernel": "product phase: k_spmm row gathers + split-row fixup (+ hot columns on k_dense in the "
                      "H-update), both halves",
            "achieved": prod_bytes / prod_s,
            "peak": 8e12,
            "unit": "B/s",
            "frac": prod_bytes / prod_s / 8e12,
            "traffic": measured_product_traffic() if not bf16 else None,
            "algorithmic_bytes_per_step": prod_bytes,
            "ms_per_step": prod_s * 1e3,
        },
        "kbar": kbar,
        "phases_ms_per_step": phases,
        "loss_after": st["loss"],
    }

    if not args.no_probe:
        # the measured ceiling of the product phase's row gathers: the probe in
        # both halves' access orders (the hot columns' dense product excluded)
        probe, _ = gather_probe(native, synth, torch, np, V, r, bf16_case=False, uniform_case=False)
        ceil_ms = probe["h_update"]["ms"] + probe["w_update"]["ms"]
        out["product_roofline"]["gather_probe"] = {
            "h_update_ms": probe["h_update"]["ms"], "w_update_ms": probe["w_update"]["ms"],
            "h_update_bytes_per_s": probe["h_update"]["bytes_per_s"],
            "w_update_bytes_per_s": probe["w_update"]["bytes_per_s"],
            "note": "nothing but the row loads of both products in their own orders (FP32 rows, cold entries "
                    "of the H-update, all entries of the W-update)"}
        out["product_roofline"]["frac_of_gather_probe"] = ceil_ms / (prod_s * 1e3)

    if not bf16 and not args.no_bf16:
        # the same steps with BF16 products (gathers from BF16 copies of the fixed
        # factor, BF16 hot-column product and Gram; the solve stays float32): speed
        # and the loss reached after the same number of iterations from the same
        # start point
        el16, st16, _, ph16 = timed_run(native.NMF_BF16)
        out["bf16_products"] = {
            "value": (m + n) * K / el16, "unit": "column NNLS solves/s", "ms_per_step": el16 * 1e3 / K,
            "phases_ms_per_step": ph16, "kbar": st16["kbar"], "loss_after": st16["loss"],
            "loss_rel_to_fp32": st16["loss"] / st["loss"] - 1.0,
        }
        log(f"[bench] BF16 products: {el16 * 1e3 / K:.3f} ms/step")
    if not args.no_serve:
        loads = tuple(float(x) for x in args.serve_loads.split(","))
        res = serving_leg(native, synth, torch, args.serve_requests, loads, n_warm=args.serve_warmup,
                          batch_cols=args.serve_batch_cols, foldin_solve=True, slots=args.serve_slots)
        out["serving"] = res

    if not args.no_cpu:
        import oracle
        cores = oracle.num_threads()
        T_cpu = args.cpu_iters
        # the same window as the GPU's timed steps: the oracle's own first
        # `warmup` iterations untimed (their inner-iteration counts are higher),
        # then T_cpu timed from the oracle's state
        W_c, H_c = wl["W0"], wl["Ht0"]
        if args.warmup:
            pre = oracle.nmf_fit(V, r, wl["reg"], W_c, H_c, T=args.warmup, max_inner=100, eps=1e-3, ls_guard=1,
                                 want_trace=False)
            W_c, H_c = pre["W"], pre["Ht"]
        log(f"[bench] CPU oracle: {T_cpu} outer iterations after {args.warmup} untimed, on {cores} threads")
        tc = time.perf_counter()
        res = oracle.nmf_fit(V, r, wl["reg"], W_c, H_c, T=T_cpu, max_inner=100,
                             eps=1e-3, ls_guard=1, want_trace=False)
        tcpu = time.perf_counter() - tc
        kbar_cpu = res["inner"].sum() / (T_cpu * (m + n))
        out["cpu_baseline"] = {
            "value": T_cpu * (m + n) / tcpu,
            "unit": "column NNLS solves/s",
            "cores": cores,
            "kind": "oracle",
            "sample": f"outer iterations {args.warmup + 1}..{args.warmup + T_cpu} ({T_cpu * (m + n)} column "
                      f"NQP solves plus the Gram and CSR products, FP64) of the same workload from the same "
                      f"start point, the first {args.warmup} untimed as the GPU's warm-up; {tcpu:.1f}s; "
                      f"kbar {kbar_cpu:.3f} (the GPU's timed steps: iterations {args.warmup + 1}.."
                      f"{args.warmup + args.steps})",
        }
        log(f"[bench] CPU oracle {tcpu:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
