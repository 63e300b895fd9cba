"""GPU: hpez_autotune measures launch shapes (face steps, tuner region trials)
and caches them in the context; shapes change speed only, so streams and
tuned configurations after autotuning equal the oracle's as before."""
from __future__ import annotations

import numpy as np
import pytest

from cfgs import make_cfg
from oracle import oracle as O
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


def test_autotune_keeps_results(torch_cuda):
    torch = torch_cuda
    from paper_2311_12133_amd import binding
    x = fields.lognormal_field((128, 128, 128))
    xt = torch.from_numpy(x).cuda()
    opts = dict(global_rate=0.2)
    cfg0 = make_cfg(x.shape, eb=1e-3)
    print("[case] autotune 128^3", flush=True)
    with binding.Context(0) as cx:
        before = binding.tune(xt, cfg0, opts, context=cx)
        s0 = binding.compress(xt, before, context=cx).cpu().numpy().tobytes()
        choices = binding.autotune(xt, before, opts, context=cx)
        assert any(c["kind"] == "faces" for c in choices)
        assert any(c["kind"] == "trials" for c in choices)
        for c in choices:
            if c["kind"] == "faces":
                assert c["shape"]["lanes"] in (64, 128, 256)
                assert c["shape"]["points_per_lane"] in (1, 2, 4, 8)
            else:
                assert c["shape"]["lanes"] in (64, 256, 1024)
            assert c["ms_best"] > 0
        after = binding.tune(xt, cfg0, opts, context=cx)
        for k in ("levels", "cand", "md_w", "alpha", "beta", "frozen_dim", "predictor"):
            assert after[k] == before[k]
        assert np.array_equal(after["block_cfg"], before["block_cfg"])
        s1 = binding.compress(xt, after, context=cx)
        assert s1.cpu().numpy().tobytes() == s0
        assert s0 == O.compress(x, before)
        y = binding.decompress(s1, context=cx).cpu().numpy()
        assert np.array_equal(y, O.decompress(s0))
