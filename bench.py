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

    # accuracy against the FP64 checker on a seeded sample
    import oracle
    rng = np.random.default_rng(12)
    idx = rng.choice(n, 512, replace=False)
    cmax = float(np.abs(c).max())
    err = {}
    for storage, tdt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        cs = torch.tensor(c, dtype=torch.float32).to(tdt).double().numpy()
        ref = oracle.evaluate(oracle.BCC8, (E, E, E), list(cs), x[idx].astype(np.float64))
        ref64 = oracle.evaluate(oracle.BCC8, (E, E, E), list(c), x[idx].astype(np.float64))
        f = res[storage]["f"][idx]
        err[storage] = dict(max_rel_vs_stored=float(np.abs(f - ref).max() / cmax),
                            max_rel_vs_fp64=float(np.abs(f - ref64).max() / cmax))

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
