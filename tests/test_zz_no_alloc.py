"""hpez_decompress_noalloc (decompression in the library's static per-GPU
workspace, for callers that cannot allocate) against hpez_decompress: two calls
in a row on one GPU, the second with a smaller stream, each bit-identical to the
plain call; a stream needing more than the static workspace is refused."""
from __future__ import annotations

import numpy as np
import pytest

from cfgs import make_cfg
from paper_2311_12133_amd import fields

pytestmark = pytest.mark.gpu

TUNE = dict(global_rate=0.2, sub_rate=0.04, lorenzo_coef=1.0, block_log2=5, allow_freeze=1,
            allow_lorenzo=1, block_wise=1)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_12133_amd import binding
    binding.lib()
    return torch


def _stream(torch, x, tuned):
    from paper_2311_12133_amd import binding
    xt = torch.from_numpy(x).cuda()
    cfg = make_cfg(x.shape, dtype="f64" if x.dtype == np.float64 else "f32", eb=1e-3)
    if tuned:
        cfg = binding.tune(xt, cfg, TUNE)
    s = binding.compress(xt, cfg)
    torch.cuda.synchronize()
    return s


def test_noalloc_matches_plain_twice(torch_cuda):
    from paper_2311_12133_amd import binding
    torch = torch_cuda
    cases = [("fronts 96x128x160 tuned block-wise", fields.fronts_field((96, 128, 160)), True),
             ("plain 40x48x56", fields.plain_field((40, 48, 56)), False)]
    for label, x, tuned in cases:
        print(f"[case] noalloc {label}", flush=True)
        s = _stream(torch, x, tuned)
        ref = binding.decompress(s)
        got = torch.full_like(ref, float("nan"))
        binding.decompress_noalloc(s, got)
        torch.cuda.synchronize()
        assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), label


def test_noalloc_f64_and_refusal(torch_cuda):
    from paper_2311_12133_amd import binding
    torch = torch_cuda
    print("[case] noalloc f64 70x66x97", flush=True)
    x = fields.fronts_field((70, 66, 97)).astype(np.float64)
    s = _stream(torch, x, True)
    ref = binding.decompress(s)
    got = torch.empty_like(ref)
    binding.decompress_noalloc(s, got)
    torch.cuda.synchronize()
    assert torch.equal(got.view(torch.int64), ref.view(torch.int64))
    # 2^25 points need 64 MiB of codes alone: more than the static workspace
    print("[case] noalloc refusal 512x512x128", flush=True)
    big = torch.zeros((512, 512, 128), dtype=torch.float32, device="cuda")
    big[0, 0, 0] = 1.0
    cfg = make_cfg(tuple(big.shape), eb=1e-3)
    sb = binding.compress(big, cfg)
    out = torch.empty_like(big)
    with pytest.raises(binding.HpezError) as ei:
        binding.decompress_noalloc(sb, out)
    assert ei.value.code == -2
    # the refused call leaves the next one unaffected
    print("[case] noalloc after refusal 40x48x56", flush=True)
    x2 = fields.plain_field((40, 48, 56))
    s2 = _stream(torch, x2, False)
    ref2 = binding.decompress(s2)
    got2 = torch.empty_like(ref2)
    binding.decompress_noalloc(s2, got2)
    torch.cuda.synchronize()
    assert torch.equal(got2.view(torch.int32), ref2.view(torch.int32))
