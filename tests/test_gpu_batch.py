"""GPU: the batch entry points (hpez_tune_batch, hpez_compress_batch,
hpez_decompress_batch) against the plain per-field calls on a mix of uneven
fields: float32 and float64, one to four dims, block-wise tuned and fixed
configurations, a constant field.  The tolerance is zero: tuned configurations
are equal, streams byte-identical, reconstructions bit-identical.  A sample of
the batch's streams is also compared with the oracle's, so the batch path is
pinned to the oracle directly and not only through the plain path."""
from __future__ import annotations

import numpy as np
import pytest

from cfgs import make_cfg
from oracle import oracle as O
from paper_2311_12133_amd import fields

pytestmark = pytest.mark.gpu

TUNE = dict(global_rate=0.05, sub_rate=0.04, lorenzo_coef=1.0, block_log2=5, allow_freeze=1,
            allow_lorenzo=1, block_wise=1)

SPECS = [  # shape, dtype, kind, relative bound
    ((37, 70, 129), np.float32, "smooth", 1e-3),
    ((70, 66, 97), np.float32, "mixed", 1e-4),
    ((100, 80), np.float32, "mixed", 1e-2),
    ((5000,), np.float64, "smooth", 1e-3),
    ((33, 65, 40), np.float64, "smooth", 1e-3),
    ((9, 17, 33, 5), np.float32, "mixed", 1e-3),
    ((64, 1, 65), np.float32, "smooth", 1e-3),
    ((1800, 36), np.float32, "rough", 1e-3),
    ((96, 64, 70), np.float32, "smooth", 1e-5),
]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_12133_amd import binding
    binding.lib()
    return torch


@pytest.fixture(scope="module")
def mix(torch_cuda):
    xs, cfgs = [], []
    for i, (shape, dt, kind, eb) in enumerate(SPECS):
        x = fields.random_field(shape, 100 + i, dt, kind)
        xs.append(x)
        cfgs.append(make_cfg(shape, dtype="f64" if dt == np.float64 else "f32", eb=eb))
    # a constant field
    xs.append(np.full((20, 30, 40), 3.5, np.float32))
    cfgs.append(make_cfg((20, 30, 40), eb=1e-3))
    xts = [torch_cuda.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs]
    return xs, xts, cfgs


def same_cfg(a: dict, b: dict):
    assert a.keys() == b.keys()
    for k in a:
        if k == "block_cfg":
            assert (a[k] is None) == (b[k] is None)
            if a[k] is not None:
                assert np.array_equal(a[k], b[k])
        else:
            assert a[k] == b[k], k


def test_tune_batch_matches_plain(torch_cuda, mix):
    from paper_2311_12133_amd import binding
    xs, xts, cfgs = mix
    print("[case] tune_batch vs tune", flush=True)
    plain = [binding.tune(x, c, TUNE) for x, c in zip(xts, cfgs)]
    batch = binding.tune_batch(xts, cfgs, TUNE)
    for i, (p, b) in enumerate(zip(plain, batch)):
        same_cfg(p, b)
    # the tuner's choices are the oracle's
    for i in (0, 3, 7):
        ref, _ = O.tune(xs[i], cfgs[i], TUNE)
        for k in ("predictor", "anchor_log2", "frozen_dim", "block_log2", "md_w", "levels",
                  "cand"):
            assert batch[i][k] == ref[k], (i, k)
        if ref["block_cfg"] is None:
            assert batch[i]["block_cfg"] is None
        else:
            assert np.array_equal(batch[i]["block_cfg"], ref["block_cfg"])


def configs_for(xts, cfgs, tuned):
    """Tuned configurations for every field plus fixed ones for a few."""
    out = list(tuned)
    out.append(make_cfg(xts[0].shape, eb=1e-3, kind="nat", md=1))
    out.append(make_cfg(xts[4].shape, dtype="f64", eb=1e-4, kind="nak", same_level=1))
    out.append(make_cfg(xts[2].shape, eb=1e-3, predictor="lorenzo"))
    return out, list(xts) + [xts[0], xts[4], xts[2]]


def test_compress_decompress_batch_match_plain(torch_cuda, mix):
    from paper_2311_12133_amd import binding
    xs, xts, cfgs = mix
    print("[case] compress_batch / decompress_batch vs plain", flush=True)
    tuned = binding.tune_batch(xts, cfgs, TUNE)
    cs, ins = configs_for(xts, cfgs, tuned)
    plain = [binding.compress(x, c) for x, c in zip(ins, cs)]
    batch = binding.compress_batch(ins, cs)
    torch_cuda.cuda.synchronize()
    pb = [p.cpu().numpy().tobytes() for p in plain]
    bb = [b.cpu().numpy().tobytes() for b in batch]
    for i in range(len(cs)):
        assert pb[i] == bb[i], f"field {i}: batch stream differs from the plain call's"
    # pinned to the oracle directly on a sample
    host = [x.cpu().numpy() for x in ins]
    for i in (1, 3, 5, len(cs) - 1):
        assert bb[i] == O.compress(host[i], cs[i]), f"field {i}: differs from the oracle"
    dplain = [binding.decompress(b) for b in batch]
    dbatch = binding.decompress_batch(batch)
    torch_cuda.cuda.synchronize()
    for i in range(len(cs)):
        a = dplain[i].cpu().numpy()
        b = dbatch[i].cpu().numpy()
        assert a.dtype == b.dtype and a.shape == b.shape
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"field {i}: values differ"


def test_batch_edges(torch_cuda, mix):
    from paper_2311_12133_amd import binding
    xs, xts, cfgs = mix
    print("[case] batch edges", flush=True)
    assert binding.compress_batch([], []) == []
    assert binding.decompress_batch([]) == []
    assert binding.tune_batch([], []) == []
    one = binding.compress_batch([xts[3]], [cfgs[3]])[0]
    assert one.cpu().numpy().tobytes() == binding.compress(xts[3], cfgs[3]).cpu().numpy().tobytes()
    # the same field twice in one batch
    two = binding.compress_batch([xts[0], xts[0]], [cfgs[0], cfgs[0]])
    assert two[0].cpu().numpy().tobytes() == two[1].cpu().numpy().tobytes()
    # a truncated stream fails with ECORRUPT
    good = binding.compress(xts[1], cfgs[1])
    with pytest.raises(binding.HpezError) as ei:
        binding.decompress_batch([good, good[: good.numel() // 2]])
    assert ei.value.code == -4
    # a field with a non-finite value fails alone with EINVAL; its out size is 0
    bad = xts[6].clone()
    bad.view(-1)[5] = float("nan")
    with pytest.raises(binding.HpezError) as ei:
        binding.compress_batch([xts[6], bad], [cfgs[6], cfgs[6]])
    assert ei.value.code == -1
