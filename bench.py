"""Throughput of lattice-spline evaluation on one MI355X.

Workload: BCC lattice 2 x 64^3 coefficients (a smooth field plus N(0,0.01)
noise), the 8-direction box spline, 2^22 uniform random query points held in
HBM.  One step = one forward pass over all points (locate + symmetry
transform, stencil gather, Horner evaluation, store).  `value` is forward
points/s with FP32 coefficients; the same line reports BF16-coefficient
forward, forward+backward (dL/dc and dL/dx) when the workload allows, the
error against the FP64 CPU checker, the roofline of the forward kernel and
the checker's own throughput on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "query points/s fwd and fwd+bwd, BCC 8-dir box spline, FP32 vs BF16 coeffs @ stated err"
PEAK_FP32_VECTOR_TFLOPS = 157.3   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
PEAK_FP32_NONPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of every kernel source and generated table the library builds from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2102_08518_amd", "csrc")
    for dirpath, _, files in sorted(os.walk(csrc)):
        for f in sorted(files):
            if f.endswith((".h", ".hip")):
                with open(os.path.join(dirpath, f), "rb") as fh:
                    h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_path: str):
    """HBM bytes per launch of the forward kernel from the committed counter
    summary (profiles/traffic.json: FETCH_SIZE and WRITE_SIZE scaled by a
    device copy of known size), or None when the kernel sources changed
    since the counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = t.get(kernel_path)
    if not entry or t.get("source_hash") != kernel_source_hash():
        return None
    return entry["bytes_per_launch"]


def write_traffic(fetch_dir: str, write_dir: str) -> dict:
    """profiles/traffic.json from two rocprofv3 counter runs of this script
    (--pmc FETCH_SIZE and --pmc WRITE_SIZE, each with --copy-probe): every
    kernel's average counter value scaled by what the same counter reads for
    the 256 MiB device copy, as HBM bytes per launch (per step for the binned
    path: its binning kernels plus the evaluation)."""
    import collections
    import csv

    def load(d, counter):
        agg = collections.defaultdict(list)
        copy = 0.0
        with open(os.path.join(d, "run_counter_collection.csv")) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"])
                if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer"):
                    copy = max(copy, v)   # the probe is the largest copy
                else:
                    agg[r["Kernel_Name"]].append(v)
        return {k: sum(v) / len(v) for k, v in agg.items()}, copy

    fe, cf = load(fetch_dir, "FETCH_SIZE")
    wr, cw = load(write_dir, "WRITE_SIZE")
    probe_kib = 262144.0
    sf, sw = probe_kib / cf, probe_kib / cw

    def per_launch(prefix):
        def one(d):
            ks = [k for k in d if k.startswith(prefix)]
            if len(ks) != 1:
                raise RuntimeError("kernel %r: %d matches" % (prefix, len(ks)))
            return d[ks[0]]
        return one(fe) * sf * 1024.0, one(wr) * sw * 1024.0

    direct = per_launch("void lsp::k_eval<1, float, float, 0, false>")
    prep = ["lsp::(anonymous namespace)::k_zero", "void lsp::(anonymous namespace)::k_bin_count<1, float>",
            "lsp::(anonymous namespace)::k_bin_scan", "void lsp::(anonymous namespace)::k_bin_scatter<float>"]
    bf = bw = 0.0
    for k in prep:
        f, w = per_launch(k)
        bf += f
        bw += w
    ef, ew = per_launch("void lsp::(anonymous namespace)::k_eval_binned<1, float, float, 0>")
    out = {"source_hash": kernel_source_hash(),
           "note": "HBM bytes per launch (per step for the binned path: binning kernels + evaluation) "
                   "of the BCC 2x64^3 / 2^22-point forward, FP32 coefficients; FETCH_SIZE x %.3f, "
                   "WRITE_SIZE x %.3f (the 256 MiB device copy reads %.0f / %.0f KiB)" % (sf, sw, cf, cw),
           "bcc8_f32_direct": {"bytes_per_launch": round(direct[0] + direct[1]),
                               "fetch": round(direct[0]), "write": round(direct[1])},
           "bcc8_f32_binned": {"bytes_per_launch": round(bf + bw + ef + ew), "fetch": round(bf + ef),
                               "write": round(bw + ew), "eval_kernel_fetch": round(ef),
                               "eval_kernel_write": round(ew)}}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def time_fn(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms per call


def run_orders(args, dev, stream):
    """Each spline of the order-2, -3 and -4 comparisons on its equal-memory
    lattice (about 2.1 M sites): forward (direct and binned order) and
    value + gradient over 10^6 uniform random points, FP32 coefficients."""
    import torch
    from paper_2102_08518_amd import api, inputs

    out_all = {}
    for order, names in inputs.ORDERS.items():
        row = {}
        for name in names:
            w = inputs.orders_workload(name)
            E, x = w["E"], w["points"]
            n = x.shape[0]
            sp = api.Spline.named(name)
            vol = api.Volume(sp, (E, E, E), "f32")
            vol.set(torch.tensor(w["coeffs"], device=dev))
            xt = torch.tensor(x, device=dev)
            out = torch.empty(n, dtype=torch.float32, device=dev)
            ws, _, _ = vol._binned_ws(xt, None)
            ms_d = time_fn(lambda: vol.eval(xt, out), args.steps, args.warmup, stream)
            ms_b = time_fn(lambda: vol.eval(xt, out, binned=True, workspace=ws), args.steps,
                           args.warmup, stream)
            ms_g = time_fn(lambda: vol.eval_grad(xt), args.steps, args.warmup, stream)
            fma = sp.info.fma_eval
            extra = {}
            if sp.info.n_reference > 1:
                # the paper's "branchless" variant: both reference polynomials, then a select
                api.use_predication(True)
                ms_p = time_fn(lambda: vol.eval(xt, out), args.steps, args.warmup, stream)
                api.use_predication(False)
                extra = {"fwd_direct_branch_free_pts_s": round(n / (ms_p * 1e-3))}
                log("order %d %-12s branch-free direct %.3e points/s" % (order, name, n / (ms_p * 1e-3)))
            row[name] = {"sites": int(sp.n_cosets * E ** 3), "taps": sp.info.taps,
                         "fma_per_point": fma,
                         "fwd_direct_pts_s": round(n / (ms_d * 1e-3)),
                         "fwd_binned_pts_s": round(n / (ms_b * 1e-3)),
                         "value_grad_pts_s": round(n / (ms_g * 1e-3)),
                         "fwd_direct_tflops": round(2 * fma * n / (ms_d * 1e-3) / 1e12, 2), **extra}
            log("order %d %-12s taps %2d  direct %.3e  binned %.3e  value+grad %.3e points/s"
                % (order, name, sp.info.taps, n / (ms_d * 1e-3), n / (ms_b * 1e-3), n / (ms_g * 1e-3)))
            del vol, xt, out, ws
        out_all[str(order)] = row
    print(json.dumps({"mode": "orders", "unit": "points/s", "points": 10 ** 6, "storage": "f32",
                      "steps": args.steps, "warmup": args.warmup, "data": "synthetic",
                      "lattice_extent": inputs.ORDERS_E, "results": out_all}), flush=True)


def sampled_errors(name, E, c, x, outs, m, seed=12):
    """Max |f - f_ref| / max|c| over a seeded sample of m points, against the
    FP64 checker run on the coefficients as stored (per storage type in outs)
    and on the unrounded FP64 coefficients."""
    import torch
    import oracle
    orc = {"tricubic": oracle.TRICUBIC, "bcc8": oracle.BCC8, "fcc6": oracle.FCC6}[name]
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
    idx = np.random.default_rng(seed).choice(x.shape[0], min(m, x.shape[0]), replace=False)
    xs = x[idx].astype(np.float64)
    cmax = float(np.abs(c).max())
    ref64 = oracle.evaluate(orc, (E, E, E), list(np.asarray(c, dtype=np.float64)), xs)
    err = {}
    for st, f in outs.items():
        cs = torch.tensor(c, dtype=torch.float32).to(tdt[st]).double().numpy()
        ref = oracle.evaluate(orc, (E, E, E), list(cs), xs)
        err[st] = dict(max_rel_vs_stored=float(np.abs(f[idx] - ref).max() / cmax),
                       max_rel_vs_fp64=float(np.abs(f[idx] - ref64).max() / cmax))
    return err


def run_configs(args, dev, stream):
    """The other workloads, one JSON line: tricubic Z^3 32^3 with 10^5 points
    (eager launches and a one-volume batch plan replayed as a graph); FCC6 on
    4 x 128^3 along 2^24 coherent ray samples, FP32 / BF16 / FP16 storage;
    BCC8 on 2 x 96^3 with 2^23 points, one forward + backward step and one
    Adam step of the fit; 64 volumes of uneven size (tricubic and BCC8,
    2.06e7 points) through one batch plan, value and value + gradient.
    Sampled errors against the FP64 checker unless --no-cpu."""
    import torch
    from paper_2102_08518_amd import api, inputs

    res = {}
    # tricubic, 10^5 points: launch-bound
    w = inputs.workload1()
    E, c, x = w["E"], w["coeffs"], w["points"]
    vol = api.Volume(api.Spline.tricubic(), (E,) * 3, "f32")
    vol.set(torch.tensor(c, dtype=torch.float32, device=dev))
    xt = torch.tensor(x, device=dev)
    o = torch.empty(x.shape[0], device=dev)
    ms = time_fn(lambda: vol.eval(xt, o), 10 * args.steps, args.warmup, stream)
    plan = api.BatchPlan([vol], [xt], [False], autotune=True)
    ms_g = time_fn(plan.run, 10 * args.steps, args.warmup, stream)
    vol.eval(xt, o)
    r = dict(points=x.shape[0], ms=round(ms, 5), pts_per_s=round(x.shape[0] / (ms * 1e-3)),
             ms_graph=round(ms_g, 5), pts_per_s_graph=round(x.shape[0] / (ms_g * 1e-3)))
    if not args.no_cpu:
        r["err"] = sampled_errors("tricubic", E, c, x, {"f32": o.double().cpu().numpy()}, m=400)["f32"]
    res["tricubic_cc32_1e5"] = r
    log("tricubic 32^3, 1e5 points: %.4f ms per call, %.4f ms per graph replay" % (ms, ms_g))
    del plan, vol, xt, o

    # FCC6 rays, three storage types
    w = inputs.workload3()
    E, c, x = w["E"], w["coeffs"], w["points"]
    xt = torch.tensor(x, device=dev)
    o = torch.empty(x.shape[0], device=dev)
    for st in ("f32", "bf16", "f16"):
        vol = api.Volume(api.Spline.fcc6(), (E,) * 3, st)
        vol.set(torch.tensor(c, dtype=torch.float32, device=dev))
        ms = time_fn(lambda: vol.eval(xt, o), args.steps, args.warmup, stream)
        vol.eval(xt, o)
        r = dict(points=x.shape[0], ms=round(ms, 5), pts_per_s=round(x.shape[0] / (ms * 1e-3)))
        if not args.no_cpu:
            r["err"] = sampled_errors("fcc6", E, c, x, {st: o.double().cpu().numpy()}, m=400)[st]
        res["fcc6_fcc128_rays_" + st] = r
        log("fcc6 rays %s: %.4f ms, %.3e points/s" % (st, ms, x.shape[0] / (ms * 1e-3)))
        del vol
    del xt, o

    # BCC8 2 x 96^3 fit: forward + backward step and Adam step
    w = inputs.workload4()
    E, x, y = w["E"], w["points"], w["targets"]
    vol = api.Volume(api.Spline.bcc8(), (E,) * 3, "f32")
    ct = torch.zeros(2, E, E, E, device=dev, requires_grad=True)
    opt = torch.optim.Adam([ct], lr=0.05)
    xt = torch.tensor(x, device=dev)
    yt = torch.tensor(y, device=dev)

    def fit_step():
        opt.zero_grad()
        f = api.LatticeSplineFn.apply(xt, ct, vol)
        loss = ((f - yt) ** 2).mean()
        loss.backward()
        opt.step()
        return loss

    losses = [float(fit_step().detach()) for _ in range(5)]
    ms_adam = time_fn(fit_step, max(args.steps // 5, 3), 1, stream)
    g = torch.empty(x.shape[0], device=dev).uniform_(-1e-6, 1e-6)
    ws = torch.empty(vol.workspace_bytes(x.shape[0]) + 256, dtype=torch.uint8, device=dev)

    def fwd_bwd():
        _, gr = vol.eval_grad(xt)
        vol.backward(xt, g, workspace=ws, grad_f=gr)

    ms_fb = time_fn(fwd_bwd, max(args.steps // 5, 3), 2, stream)
    res["bcc8_bcc96_fit_8M"] = dict(points=x.shape[0], ms_fwd_bwd=round(ms_fb, 5),
                                    pts_per_s_fwd_bwd=round(x.shape[0] / (ms_fb * 1e-3)),
                                    ms_adam_step=round(ms_adam, 5),
                                    first_losses=[round(v, 6) for v in losses])
    log("bcc8 2x96^3 fit: fwd+bwd %.4f ms, Adam step %.4f ms" % (ms_fb, ms_adam))
    del vol, ct, opt, xt, yt, g, ws

    # 64 volumes through one batch plan
    wl = inputs.workload5()
    vols, pts = [], []
    for d in wl:
        v = api.Volume(api.Spline.named(d["spline"]), (d["E"],) * 3, "f32")
        v.set(torch.tensor(d["coeffs"], device=dev))
        vols.append(v)
        pts.append(torch.tensor(d["points"], device=dev))
    ntot = sum(d["n"] for d in wl)
    for mode in ("value", "value+grad"):
        plan = api.BatchPlan(vols, pts, [mode != "value"] * len(vols), autotune=True)
        ms = time_fn(plan.run, args.steps, args.warmup, stream)
        res["batch64_" + mode] = dict(points=ntot, volumes=len(vols), ms=round(ms, 5),
                                      pts_per_s=round(ntot / (ms * 1e-3)), tile=plan.tile,
                                      blocks=plan.blocks)
        log("batch of %d volumes, %s: %.4f ms, %.3e points/s" % (len(vols), mode, ms, ntot / (ms * 1e-3)))
    print(json.dumps({"mode": "configs", "unit": "points/s", "storage": "f32 unless named",
                      "steps": args.steps, "warmup": args.warmup, "data": "synthetic",
                      "results": res}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=1 << 15)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device-to-device copy (a kernel of known traffic "
                         "that calibrates hardware byte counters)")
    ap.add_argument("--orders", action="store_true",
                    help="instead of the headline line: the order-2/3/4 spline comparisons of the "
                         "paper's experiments (equal-memory lattices, 10^6 random points), one JSON "
                         "line with points/s per spline")
    ap.add_argument("--configs", action="store_true",
                    help="instead of the headline line: the other workloads (tricubic 32^3 with "
                         "10^5 points, FCC6 rays on 4x128^3, the BCC8 2x96^3 fit, a batch of 64 "
                         "volumes), one JSON line")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json from the rocprofv3 output directories of a "
                         "--pmc FETCH_SIZE and a --pmc WRITE_SIZE run of this script (no GPU)")
    args = ap.parse_args()
    if args.traffic_from:
        print(json.dumps(write_traffic(*args.traffic_from), indent=1))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the evaluation runs on a single device "
              "(--gpus %d requested)." % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2102_08518_amd import api, inputs

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.orders:
        run_orders(args, dev, stream)
        return
    if args.configs:
        run_configs(args, dev, stream)
        return
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = inputs.workload2()
    E, c, x = w["E"], w["coeffs"], w["points"]
    n = x.shape[0]
    log("workload 2: BCC 2x%d^3, %d points" % (E, n))
    sp = api.Spline.bcc8()
    fma = sp.info.fma_eval
    xt = torch.tensor(x, device=dev)
    ct = torch.tensor(c, dtype=torch.float32, device=dev)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    res = {}
    vols = {}
    paths = {}
    for storage in ("f32", "bf16"):
        vol = api.Volume(sp, (E, E, E), storage)
        vol.set(ct)
        vols[storage] = vol
        ws, _, _ = vol._binned_ws(xt, None)
        for path in ("direct", "binned"):
            if path == "direct":
                fn = lambda: vol.eval(xt, out)
            else:
                fn = lambda: vol.eval(xt, out, binned=True, workspace=ws)
            ms = time_fn(fn, args.steps, args.warmup, stream)
            paths[(storage, path)] = ms
            log("%s %s forward: %.4f ms/step, %.3e points/s" % (storage, path, ms, n / (ms * 1e-3)))
        best = min(("direct", "binned"), key=lambda pth: paths[(storage, pth)])
        ms = paths[(storage, best)]
        if best == "direct":
            vol.eval(xt, out)
        else:
            vol.eval(xt, out, binned=True, workspace=ws)
        f = out.double().cpu().numpy()
        res[storage] = dict(ms=ms, pts_per_s=n / (ms * 1e-3), f=f, path=best)

    # forward + backward (dL/dc, dL/dx) of a loss with a given dL/df
    fb = None
    try:
        g = torch.empty(n, dtype=torch.float32, device=dev).uniform_(-1e-6, 1e-6)
        vol = vols["f32"]
        wsb = vol.workspace_bytes(n)
        ws = torch.empty(wsb + 256, dtype=torch.uint8, device=dev)

        fwd_binned = res["f32"]["path"] == "binned"
        wsf, _, _ = vol._binned_ws(xt, None)

        def step_fb():
            # forward: value and point gradient; backward: dL/dc, and dL/dx
            # from the saved gradient
            _, grad = vol.eval_grad(xt, binned=fwd_binned, workspace=wsf)
            vol.backward(xt, g, want_dc=True, want_dx=True, workspace=ws, grad_f=grad)

        ms_fb = time_fn(step_fb, max(args.steps // 5, 3), 2, stream)
        fb = dict(ms=ms_fb, pts_per_s=n / (ms_fb * 1e-3))
        log("fwd+bwd: %.4f ms/step" % ms_fb)
    except Exception as e:  # the backward coefficient pass may be unavailable
        log("fwd+bwd not measured: %s" % e)

    # the CPU leg (skipped with --no-cpu): accuracy against the FP64 checker
    # on a seeded sample, then the checker's own throughput
    err = {"f32": None, "bf16": {"max_rel_vs_stored": None, "max_rel_vs_fp64": None}}
    if not args.no_cpu:
        err = sampled_errors("bcc8", E, c, x, {st: res[st]["f"] for st in ("f32", "bf16")}, m=512)

    ms = res["f32"]["ms"]
    t_k = ms * 1e-3
    flops = 2.0 * fma * n
    achieved = flops / t_k / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
            "traffic": measured_traffic("bcc8_f32_" + res["f32"]["path"]),
            "kernel": ("k_eval<bcc8,f32,f32,value>" if res["f32"]["path"] == "direct"
                       else "k_eval_binned<bcc8,f32,f32,value> (+ binning kernels, whole step timed)"),
            "algorithmic_flops_per_point": 2 * fma,
            "frac_of_nonpacked_peak": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
            "hbm_compulsory_GBs": round(16.0 * n / t_k / 1e9, 1),
            "hbm_compulsory_frac": round(16.0 * n / t_k / 1e9 / PEAK_HBM_GBS, 4),
            # the bytes a fetch of every tap would move (point, value and 4 B
            # per tap), against the HBM peak; served mostly by L1/L2, not HBM
            "effective_gather_bytes_per_point": 16 + 4 * sp.info.taps,
            "effective_gather_GBs": round((16 + 4 * sp.info.taps) * n / t_k / 1e9, 1),
            "effective_gather_frac_of_hbm_peak": round((16 + 4 * sp.info.taps) * n / t_k / 1e9 / PEAK_HBM_GBS, 4),
            # what the counters show binds this kernel (profiles/): the
            # L1-to-L2 requests of the random stencil gathers, not the VALU
            "measured_limit": "L1->L2 gather requests (about 9.5 per point); VALU about 38% busy"}

    cpu = None
    if not args.no_cpu:
        import oracle
        m = args.cpu_sample
        sub = x[:m].astype(np.float64)
        t0 = time.time()
        oracle.evaluate(oracle.BCC8, (E, E, E), list(c), sub)
        dt = time.time() - t0
        cpu = {"value": round(m / dt, 1), "unit": "points/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "first %d of the %d workload points, FP64 naive convolution sum" % (m, n)}
        log("cpu oracle: %.1f points/s on %d threads (%.1f s)" % (m / dt, oracle.num_threads(), dt))

    line = {
        "metric": METRIC,
        "value": round(res["f32"]["pts_per_s"], 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "BCC 2x64^3 (L rows [-1,1,1],[1,-1,1],[1,1,-1]), 8-direction box "
                               "spline, smooth field + N(0,0.01) coefficients, 2^22 uniform "
                               "interior points, forward",
                   "points": n, "coeffs": int(c.size), "storage": "f32",
                   "path": res["f32"]["path"]},
        "paths_ms": {"%s_%s" % k: round(v, 5) for k, v in paths.items()},
        "bf16": {"value": round(res["bf16"]["pts_per_s"], 1), "ms_per_step": round(res["bf16"]["ms"], 5),
                 "path": res["bf16"]["path"],
                 "speedup_vs_f32": round(res["f32"]["ms"] / res["bf16"]["ms"], 3),
                 "max_rel_err_vs_fp64": err["bf16"]["max_rel_vs_fp64"],
                 "max_rel_err_vs_stored": err["bf16"]["max_rel_vs_stored"]},
        "f32_err": err["f32"],
        "fwd_bwd": None if fb is None else {"value": round(fb["pts_per_s"], 1),
                                            "ms_per_step": round(fb["ms"], 5)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
