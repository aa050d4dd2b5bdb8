"""The matrix-core evaluation of the one-sub-region BCC splines (8-direction
and quartic; monomial coefficients A = Wq c / Q on the MFMA units) against the FP64 checker and
against the per-lane FMA path, for every coefficient storage, value and
gradient, direct and binned order, and wavefront-ragged point counts
(lanes without a point still take part in the matrix products).

Tolerances as in the forward tests: 2e-6 max|c| for values, 2e-5 max|c| for
gradients, against the checker run on the coefficients as stored."""
import numpy as np
import pytest
import torch

import oracle
from paper_2102_08518_amd import api, inputs

pytestmark = pytest.mark.gpu

TORCH_DT = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


def _stored(c, storage):
    return torch.tensor(c, dtype=torch.float32).to(TORCH_DT[storage]).to(torch.float64).numpy()


@pytest.fixture
def restore_mfma():
    yield
    api.use_mfma(False)


ORC = {"bcc8": oracle.BCC8, "bcc7": oracle.BCC7}


@pytest.mark.parametrize("name", list(ORC))
@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 3001])
def test_mfma_matches_oracle_and_fma_path(device, restore_mfma, name, storage, n):
    print("case mfma", name, storage, n, flush=True)
    rng = np.random.default_rng(300 + n)
    E = 12
    c = rng.uniform(-1, 1, (2, E, E, E))
    vol = api.Volume(api.Spline.named(name), (E, E, E), storage)
    vol.set(torch.tensor(c, dtype=torch.float32, device=device))
    x = rng.uniform(-3, 2 * (E - 1) + 3, (n, 3)).astype(np.float32)
    xt = torch.tensor(x, device=device)
    cs = _stored(c, storage)
    fref, gref = oracle.evaluate(ORC[name], (E, E, E), list(cs), x.astype(np.float64), grad=True)
    out = {}
    for on in (True, False):
        api.use_mfma(on)
        f = vol.eval(xt).double().cpu().numpy()
        v, g = vol.eval_grad(xt)
        fb = vol.eval(xt, binned=True).double().cpu().numpy()
        out[on] = f
        tol = 2e-6 * np.abs(cs).max()
        assert np.abs(f - fref).max() <= tol, (on, np.abs(f - fref).max())
        assert np.abs(fb - fref).max() <= tol
        assert np.abs(v.double().cpu().numpy() - fref).max() <= tol
        assert np.abs(g.double().cpu().numpy() - gref).max() <= 10 * tol
    assert np.abs(out[True] - out[False]).max() <= 4e-6 * np.abs(cs).max()


@pytest.mark.parametrize("name", list(ORC))
def test_mfma_special_points(device, restore_mfma, name):
    """NaN -> NaN, far and infinite points -> 0, mixed into full wavefronts
    with ordinary points, on the matrix-core path."""
    print("case mfma special", name, flush=True)
    api.use_mfma(True)
    rng = np.random.default_rng(8)
    E = 8
    c = rng.uniform(-1, 1, (2, E, E, E))
    vol = api.Volume(api.Spline.named(name), (E, E, E), "f32")
    vol.set(torch.tensor(c, dtype=torch.float32, device=device))
    x = rng.uniform(0, 2 * (E - 1), (128, 3)).astype(np.float32)
    x[3] = np.nan
    x[40] = [np.inf, 1, 1]
    x[70] = [1e30, 2, 2]
    x[100] = [-50, 3, 3]
    f = vol.eval(torch.tensor(x, device=device)).cpu().numpy().astype(np.float64)
    assert np.isnan(f[3]) and f[40] == 0 and f[70] == 0 and f[100] == 0
    ok = np.ones(128, bool)
    ok[[3, 40, 70, 100]] = False
    ref = oracle.evaluate(ORC[name], (E, E, E), list(_stored(c, "f32")), x[ok].astype(np.float64))
    assert np.abs(f[ok] - ref).max() <= 2e-6 * np.abs(c).max()


def test_mfma_full_size_against_fma_path(device, restore_mfma):
    """Bench workload (BCC 2x64^3, 2^22 points): matrix-core and per-lane FMA
    evaluation agree everywhere within the FP32 tolerance, and a sample
    matches the checker."""
    print("case mfma full size", flush=True)
    w = inputs.workload2()
    E, c, x = w["E"], w["coeffs"], w["points"]
    vol = api.Volume(api.Spline.bcc8(), (E, E, E), "f32")
    vol.set(torch.tensor(c, dtype=torch.float32, device=device))
    xt = torch.tensor(x, device=device)
    api.use_mfma(True)
    a = vol.eval(xt)
    ab = vol.eval(xt, binned=True)
    api.use_mfma(False)
    b = vol.eval(xt)
    cm = float(np.abs(c).max())
    assert torch.equal(a, ab)
    assert float((a - b).abs().max()) <= 4e-6 * cm
    idx = np.random.default_rng(11).choice(x.shape[0], 1000, replace=False)
    ref = oracle.evaluate(oracle.BCC8, (E, E, E), list(_stored(c, "f32")), x[idx].astype(np.float64))
    assert np.abs(a.cpu().numpy()[idx] - ref).max() <= 2e-6 * cm
