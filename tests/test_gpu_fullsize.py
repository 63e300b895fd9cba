"""GPU parity at the benchmark's full sizes, in the configuration bench.py
times: the auto-tuned block-wise configuration, compressed by the library and
by the oracle (whole streams compared byte for byte), and the library's
reconstruction compared bit for bit with the oracle's.  The oracle handles these
sizes in seconds per call, so every output is checked, not a sample.

  * 512^3 float32, exp(1.5 g) with g a -5/3 Gaussian field, relative bound 1e-3
    (the benchmark workload), and its float64 copy (computed in float64);
  * 256 x 384 x 384 float32, -5/3 field plus three tanh fronts, relative bounds
    1e-2 ... 1e-5 (the swept full-method workload);
  * the tuner's whole output (Sec. 6) against the oracle's at 512^3 and on the
    fronts field at 1e-4.
"""
from __future__ import annotations

import numpy as np
import pytest

from cfgs import make_cfg
from oracle import oracle as O
from paper_2311_12133_amd import fields

pytestmark = pytest.mark.gpu

TUNE = dict(global_rate=0.01, sub_rate=0.04, lorenzo_coef=1.0, block_log2=5, allow_freeze=1,
            allow_lorenzo=1, block_wise=1, tune_ab=1)  # the options bench.py times


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_12133_amd import binding
    binding.lib()
    return torch


def check(torch, x, eb, label):
    from paper_2311_12133_amd import binding
    print(f"[case] {label} shape={x.shape} eb={eb}", flush=True)
    f64 = x.dtype == np.float64
    cfg = make_cfg(x.shape, dtype="f64" if f64 else "f32", eb=eb)
    xt = torch.from_numpy(x).cuda()
    tuned = binding.tune(xt, cfg, TUNE)
    s = binding.compress(xt, tuned)
    torch.cuda.synchronize()
    got = s.cpu().numpy().tobytes()
    ref = O.compress(x, tuned)
    assert got == ref, f"{label}: stream differs (gpu {len(got)} B, oracle {len(ref)} B)"
    rec = binding.decompress(s)
    torch.cuda.synchronize()
    r = rec.cpu().numpy()
    r_ref = O.decompress(ref)
    assert np.array_equal(r.view(np.uint8), r_ref.view(np.uint8)), f"{label}: values differ"
    e = eb * (float(x.max()) - float(x.min()))
    assert np.max(np.abs(r.astype(np.float64) - x.astype(np.float64))) <= e


@pytest.fixture(scope="module")
def lognormal():
    return fields.lognormal_field((512, 512, 512))


def test_lognormal_512(torch_cuda, lognormal):
    check(torch_cuda, lognormal, 1e-3, "lognormal 512^3")


def tune_matches(torch, x, eb, label):
    """The library's tuned configuration equals the oracle's, field by field
    (every decision is made from integer scores and histograms)."""
    from paper_2311_12133_amd import binding
    print(f"[case] tune {label} shape={x.shape} eb={eb}", flush=True)
    cfg = make_cfg(x.shape, dtype="f64" if x.dtype == np.float64 else "f32", eb=eb)
    got = binding.tune(torch.from_numpy(x).cuda(), cfg, TUNE)
    ref, _ = O.tune(x, cfg, TUNE)
    for k in ("predictor", "anchor_log2", "frozen_dim", "block_log2", "md_w", "levels", "cand"):
        assert got[k] == ref[k], (label, k)
    assert np.array_equal(np.asarray(got["block_cfg"]), np.asarray(ref["block_cfg"])), label


def test_tune_lognormal_512(torch_cuda, lognormal):
    tune_matches(torch_cuda, lognormal, 1e-3, "lognormal 512^3")


def test_lognormal_512_f64(torch_cuda):
    # the float64 field is computed in float64 (the float32 benchmark field is its cast)
    x = fields.lognormal_field((512, 512, 512), dtype=np.float64)
    assert x.dtype == np.float64
    tune_matches(torch_cuda, x, 1e-3, "lognormal 512^3 float64")
    check(torch_cuda, x, 1e-3, "lognormal 512^3 float64")


@pytest.fixture(scope="module")
def fronts():
    return fields.fronts_field((256, 384, 384))


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4, 1e-5])
def test_fronts_256x384x384(torch_cuda, fronts, eb):
    check(torch_cuda, fronts, eb, "fronts 256x384x384")


def test_tune_fronts_256x384x384(torch_cuda, fronts):
    tune_matches(torch_cuda, fronts, 1e-4, "fronts 256x384x384")
