"""GPU parity of the batched persistent launch (one graph replay evaluates
many volumes of uneven size): every volume's outputs equal the single-volume
per-lane FMA kernels' (the batch runs the same per-point body) and match
the FP64 checker on samples; graph replays see the current contents of the
bound buffers."""
import numpy as np
import pytest
import torch

import oracle
from paper_2102_08518_amd import api, inputs

pytestmark = pytest.mark.gpu

ORC = {"tricubic": oracle.TRICUBIC, "bcc8": oracle.BCC8, "fcc6": oracle.FCC6,
       "trilinear": oracle.TRILINEAR, "bcc4": oracle.BCC4, "triquadratic": oracle.TRIQUADRATIC,
       "cc7": oracle.CC7, "bcc7": oracle.BCC7, "cc6": oracle.CC6}
MIXED = [("tricubic", "f32", 9, 1000, False), ("bcc8", "f32", 12, 40000, True),
         ("fcc6", "bf16", 8, 7000, False), ("bcc8", "f16", 7, 0, False),
         ("tricubic", "f32", 20, 70001, True), ("bcc8", "f32", 10, 513, False),
         ("fcc6", "f32", 9, 25000, True), ("tricubic", "bf16", 6, 3000, False)]
OTHER_KINDS = [("cc7", "f32", 10, 20000, True), ("bcc7", "bf16", 9, 9000, False),
               ("trilinear", "f32", 11, 5000, True), ("bcc4", "f16", 8, 4097, False),
               ("triquadratic", "f32", 9, 12000, False), ("bcc7", "f32", 7, 333, True),
               ("cc7", "bf16", 6, 64, False), ("cc6", "f32", 9, 7001, True)]


def _mixed(device, seed=41, specs=MIXED):
    rng = np.random.default_rng(seed)
    vols, pts, grads, cs = [], [], [], []
    for name, st, E, n, g in specs:
        nc = ORC[name].n_cosets
        c = rng.uniform(-1, 1, (nc, E, E, E)).astype(np.float32)
        v = api.Volume(getattr(api.Spline, name)(), (E, E, E), st)
        v.set(torch.tensor(c, device=device))
        D = inputs.LATTICE[name]["D"]
        x = rng.uniform(-2, D * (E - 1) + 3, (n, 3)).astype(np.float32)
        vols.append(v)
        pts.append(torch.tensor(x, device=device).reshape(n, 3))
        grads.append(g)
        cs.append((name, st, E, c))
    return vols, pts, grads, cs


def _check_against_single(vols, pts, grads, val, grad):
    # the batch runs the per-point body the single-volume entry points use
    # for each volume's size (four lanes per point for the separable splines
    # up to their limit), without matrix cores
    api.use_mfma(False)
    try:
        for v, p, g, a, b in zip(vols, pts, grads, val, grad):
            if g:
                rv, rg = v.eval_grad(p)
                assert torch.equal(a, rv) and torch.equal(b, rg)
            else:
                assert torch.equal(a, v.eval(p))
    finally:
        api.use_mfma(False)


@pytest.mark.parametrize("which", ["mixed", "other_kinds", "one_lane"])
def test_batch_matches_single_volume_and_oracle(device, which):
    """one_lane: with four lanes per point switched off the plan follows."""
    print("case batch", which, flush=True)
    if which == "one_lane":
        api.set_split_maxn(0)
    try:
        _batch_vs_single(device, which)
    finally:
        api.set_split_maxn(-1)


def _batch_vs_single(device, which):
    vols, pts, grads, cs = _mixed(device, specs=OTHER_KINDS if which == "other_kinds" else MIXED)
    plan = api.BatchPlan(vols, pts, grads, autotune=True)
    assert plan.tile in (256, 1024, 4096, 16384) and plan.blocks >= 1
    val, grad = plan.run()
    torch.cuda.synchronize()
    _check_against_single(vols, pts, grads, val, grad)
    rng = np.random.default_rng(0)
    for (name, st, E, c), p, a in zip(cs, pts, val):
        n = p.shape[0]
        if n == 0:
            continue
        idx = rng.choice(n, min(n, 300), replace=False)
        x = p.cpu().numpy()[idx].astype(np.float64)
        tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[st]
        cq = torch.tensor(c).to(tdt).double().numpy()
        ref = oracle.evaluate(ORC[name], (E, E, E), list(cq), x)
        assert np.abs(a.cpu().numpy()[idx] - ref).max() <= 2e-6


def test_graph_replays_read_current_buffers(device):
    """Replay three times with eager work in between and the bound point
    buffers rewritten in place; every replay equals the eager result."""
    print("case batch replays", flush=True)
    vols, pts, grads, cs = _mixed(device, seed=42)
    plan = api.BatchPlan(vols, pts, grads, autotune=False)
    for r in range(3):
        for p in pts:
            if p.shape[0]:
                p.add_(0.25 * (r + 1)).remainder_(7.0)   # eager work on the same stream
        torch.cuda.synchronize()
        val, grad = plan.run()
        torch.cuda.synchronize()
        _check_against_single(vols, pts, grads, val, grad)


def test_full_batched_workload_sampled(device):
    """64 uneven volumes (tricubic and BCC 8-direction, E in 16..128,
    N_v log-uniform in [1e3, 2^21]) with value+gradient, one replay; a sample
    of every volume checked against the checker."""
    print("case batch full size", flush=True)
    wl = inputs.workload5()
    vols, pts = [], []
    for d in wl:
        v = api.Volume(getattr(api.Spline, d["spline"])(), (d["E"],) * 3, "f32")
        v.set(torch.tensor(d["coeffs"], device=device))
        vols.append(v)
        pts.append(torch.tensor(d["points"], device=device))
    plan = api.BatchPlan(vols, pts, [True] * len(vols), autotune=True)
    val, grad = plan.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for d, a, g in zip(wl, val, grad):
        n = d["n"]
        idx = rng.choice(n, min(n, 48), replace=False)
        x = d["points"][idx].astype(np.float64)
        f, gr = oracle.evaluate(ORC[d["spline"]], (d["E"],) * 3, list(d["coeffs"].astype(np.float64)), x,
                                grad=True)
        assert np.abs(a.cpu().numpy()[idx] - f).max() <= 2e-6
        assert np.abs(g.cpu().numpy()[idx] - gr).max() <= 2e-5
