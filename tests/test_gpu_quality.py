"""GPU: the quality functions of Sec. 3.1, Eq. (1) (hpez_quality_eval) and the
quality-target bound search (hpez_fit_eb) through the C ABI, against the
oracle (oracle/oracle_quality.py) on the same seeded inputs.

Metric tolerances: the maximum error and the value range are order-free and
must be equal; n_windows equal; MSE and each window's moments are float64 sums
taken in another order than the oracle's, so MSE and SSIM must agree to a
relative 1e-12 and PSNR to 1e-9 dB (n <= 2^32 terms, each sum's rounding is
below n * 2^-53 relative).  The search decides on integer grid indices, so its
bounds and iteration counts must be equal to the oracle's."""
from __future__ import annotations

import math

import numpy as np
import pytest

from cfgs import make_cfg
from oracle import oracle as O
from oracle import oracle_quality as Q
from paper_2311_12133_amd import fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_12133_amd import binding
    binding.lib()
    return torch


def _field(shape, seed=5, dtype=np.float32):
    rng = np.random.default_rng(seed)
    return fields.gaussian_field(shape, -5.0 / 3.0, rng).astype(dtype)


def check_metrics(got, want, label):
    print(f"[case] {label}", flush=True)
    assert got["n"] == want["n"], label
    assert got["n_windows"] == want["n_windows"], label
    assert got["value_range"] == want["value_range"], label
    assert got["max_abs_err"] == want["max_abs_err"], label
    assert got["mse"] == pytest.approx(want["mse"], rel=1e-12, abs=0), label
    if math.isinf(want["psnr"]):
        assert got["psnr"] == want["psnr"], label
    else:
        assert got["psnr"] == pytest.approx(want["psnr"], rel=0, abs=1e-9), label
    assert got["ssim"] == pytest.approx(want["ssim"], rel=1e-12, abs=0), label


CASES = [((40, 36, 34), "f32", 8), ((64, 64, 64), "f32", 8), ((33, 17, 70), "f64", 8),
         ((301, 211), "f32", 8), ((5000,), "f64", 7), ((9, 10, 12, 14), "f32", 4),
         ((24, 5, 40), "f32", 8), ((70, 66, 97), "f32", 16)]


@pytest.mark.parametrize("shape,dt,w", CASES)
def test_quality_matches_oracle(torch_cuda, shape, dt, w):
    torch = torch_cuda
    from paper_2311_12133_amd import binding
    npdt = np.float32 if dt == "f32" else np.float64
    x = _field(shape, dtype=npdt)
    # a real reconstruction (the oracle's) and a noisy one
    cfg = make_cfg(shape, dtype=dt, eb=1e-3, kind="nat")
    xr1 = O.decompress(O.compress(x, cfg)).reshape(shape)
    rng = np.random.default_rng(9)
    xr2 = (x + rng.normal(0, 0.01, size=shape)).astype(npdt)
    xt = torch.from_numpy(x).cuda()
    for i, xr in enumerate((xr1, xr2)):
        got = binding.quality(xt, torch.from_numpy(np.ascontiguousarray(xr)).cuda(), window=w)
        check_metrics(got, Q.metrics(x, xr, w), f"{shape} {dt} w={w} rec{i}")


def test_quality_special_cases(torch_cuda):
    torch = torch_cuda
    from paper_2311_12133_amd import binding
    x = _field((30, 31, 32))
    xt = torch.from_numpy(x).cuda()
    q = binding.quality(xt, xt)
    assert q["psnr"] == math.inf and q["ssim"] == 1.0 and q["mse"] == 0.0
    z = torch.full((17, 19), 2.5, dtype=torch.float32, device="cuda")
    q = binding.quality(z, z + 1)
    assert q["value_range"] == 0.0 and q["psnr"] == -math.inf
    check_metrics(q, Q.metrics(np.full((17, 19), 2.5, np.float32),
                               np.full((17, 19), 3.5, np.float32)), "constant")
    # repeated evaluations give the same bits
    y = xt + 0.001
    a, b = binding.quality(xt, y), binding.quality(xt, y)
    assert a == b
    # non-finite values and oversized windows are rejected
    bad = xt.clone()
    bad[3, 4, 5] = float("nan")
    with pytest.raises(binding.HpezError):
        binding.quality(bad, xt)
    with pytest.raises(binding.HpezError):
        binding.quality(xt, xt, window=65)


FITS = [((40, 36, 34), "f32", "nat", "psnr", 60.0), ((40, 36, 34), "f32", "lin", "psnr", 85.0),
        ((48, 40, 33), "f64", "nak", "psnr", 100.0), ((64, 64, 64), "f32", "nat", "ssim", 0.9995),
        ((200, 150), "f32", "lin", "ssim", 0.99)]


@pytest.mark.parametrize("shape,dt,kind,metric,target", FITS)
def test_fit_eb_matches_oracle(torch_cuda, shape, dt, kind, metric, target):
    torch = torch_cuda
    from paper_2311_12133_amd import binding
    npdt = np.float32 if dt == "f32" else np.float64
    x = _field(shape, seed=7, dtype=npdt)
    cfg = make_cfg(shape, dtype=dt, kind=kind)
    print(f"[case] fit {shape} {dt} {kind} {metric}>={target}", flush=True)
    got = binding.fit_eb(torch.from_numpy(x).cuda(), cfg, metric, target, max_iter=16)
    e, q, it, hi = Q.fit_eb(x, cfg, metric, target, max_iter=16)
    assert got["e"] == e and got["e_hi"] == hi and got["iterations"] == it
    assert e > 0 and q[metric] >= target
    check_metrics(got["quality"], q, "fit quality")
    ref = O.compress(x, dict(cfg, eb_mode="abs", eb=e))
    assert got["bytes"] == len(ref)


def test_fit_eb_constant_field(torch_cuda):
    torch = torch_cuda
    from paper_2311_12133_amd import binding
    z = torch.full((20, 21, 22), -1.25, dtype=torch.float32, device="cuda")
    r = binding.fit_eb(z, make_cfg((20, 21, 22)), "psnr", 90.0)
    assert r["e"] == 0.0 and r["iterations"] == 0 and r["quality"]["psnr"] == math.inf


def test_quality_fronts_field_c2(torch_cuda):
    """The 256 x 384 x 384 fronts field at rel 1e-3 (the tuned full method):
    metrics of the library's own reconstruction against the oracle's metrics
    of the same arrays."""
    torch = torch_cuda
    from paper_2311_12133_amd import binding
    x = fields.fronts_field()
    xt = torch.from_numpy(x).cuda()
    cfg0 = make_cfg(x.shape, eb=1e-3, block_log2=5)
    cfg = binding.tune(xt, cfg0, dict(block_log2=5))
    y = binding.decompress(binding.compress(xt, cfg))
    got = binding.quality(xt, y)
    check_metrics(got, Q.metrics(x, y.cpu().numpy()), "fronts 256x384x384")
    assert got["max_abs_err"] <= 1e-3 * got["value_range"]
