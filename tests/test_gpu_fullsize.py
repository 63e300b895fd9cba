"""GPU parity at the benchmark's full sizes, in the configuration bench.py
times: the auto-tuned block-wise configuration, compressed by the library and
by the oracle (whole streams compared byte for byte), and the library's
reconstruction compared bit for bit with the oracle's.  The oracle handles these
sizes in seconds per call, so every output is checked, not a sample.

  * 512^3 float32, exp(1.5 g) with g a -5/3 Gaussian field, relative bound 1e-3
    (the benchmark workload);
  * 256 x 384 x 384 float32, -5/3 field plus three tanh fronts, relative bounds
    1e-2 ... 1e-5 (the swept full-method workload).
"""
from __future__ import annotations

import numpy as np
import pytest

from cfgs import make_cfg
from oracle import oracle as O
from paper_2311_12133_amd import fields

pytestmark = pytest.mark.gpu

TUNE = dict(global_rate=0.01, sub_rate=0.04, lorenzo_coef=1.0, block_log2=5, allow_freeze=1,
            allow_lorenzo=1, block_wise=1)


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
    cfg = make_cfg(x.shape, dtype="f32", eb=eb)
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
    assert np.array_equal(r.view(np.uint32), r_ref.view(np.uint32)), f"{label}: values differ"
    e = eb * (float(x.max()) - float(x.min()))
    assert np.max(np.abs(r.astype(np.float64) - x.astype(np.float64))) <= e


def test_lognormal_512(torch_cuda):
    x = fields.lognormal_field((512, 512, 512))
    check(torch_cuda, x, 1e-3, "lognormal 512^3")


@pytest.fixture(scope="module")
def fronts():
    return fields.fronts_field((256, 384, 384))


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4, 1e-5])
def test_fronts_256x384x384(torch_cuda, fronts, eb):
    check(torch_cuda, fronts, eb, "fronts 256x384x384")
