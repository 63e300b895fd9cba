"""GPU parity for integer fields (uint8, uint16, int16, int32): the method in
float64 on the integer values with every rebuilt value rounded to an integer,
output in the field's type.  Streams must be byte-identical to the oracle's,
reconstructions equal, and the bound must hold on every point; the tuner's
configuration must equal the oracle's; a batch mixing integer and float
fields must give each field's plain stream."""
from __future__ import annotations

import numpy as np
import pytest

from cfgs import candidates, make_cfg
from oracle import oracle as O
from oracle import oracle_quality as Q
from paper_2311_12133_amd import fields

pytestmark = pytest.mark.gpu

INT_TYPES = [("u8", np.uint8), ("u16", np.uint16), ("i16", np.int16), ("i32", np.int32)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_12133_amd import binding
    binding.lib()
    return torch


def int_field(shape, npdt, seed=4, span=None):
    rng = np.random.default_rng(seed)
    g = fields.gaussian_field(shape, -5.0 / 3.0, rng)
    g = (g - g.min()) / (g.max() - g.min())
    lim = np.iinfo(npdt)
    lo = float(lim.min) if span is None else 0.0
    hi = float(lim.max) if span is None else float(span)
    return np.round(lo + g * (hi - lo)).astype(npdt)


def roundtrip(torch, x, cfg, label):
    from paper_2311_12133_amd import binding
    print(f"[case] {label} shape={x.shape} dtype={cfg['dtype']}", flush=True)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    s = binding.compress(xt, cfg)
    torch.cuda.synchronize()
    got = s.cpu().numpy().tobytes()
    ref = O.compress(x, cfg)
    assert got == ref, f"{label}: stream differs ({len(got)} vs {len(ref)} bytes)"
    y = binding.decompress(s).cpu().numpy()
    yo = O.decompress(ref)
    assert y.dtype == x.dtype and np.array_equal(y, yo), f"{label}: reconstruction differs"
    e = cfg["eb"] if cfg["eb_mode"] == "abs" else O.error_bound(x, cfg)[0]
    assert np.abs(x.astype(np.int64) - y.astype(np.int64)).max() <= e
    return s


@pytest.mark.parametrize("name,npdt", INT_TYPES, ids=[n for n, _ in INT_TYPES])
def test_int_configs(torch_cuda, name, npdt):
    x = int_field((37, 70, 129), npdt, span=None if name != "i32" else 1 << 22)
    for eb, kw in ((0.4, dict(kind="nat")), (2.0, dict(kind="nat", md=1)),
                   (7.0, dict(kind="nak", same_level=1)), (1e-3, dict(kind="lin", eb_mode="rel"))):
        mode = kw.pop("eb_mode", "abs")
        cfg = make_cfg(x.shape, dtype=name, eb=eb, eb_mode=mode, **kw)
        roundtrip(torch_cuda, x, cfg, f"{name} eb={eb} {kw}")


@pytest.mark.parametrize("shape", [(5000,), (300, 211), (9, 17, 33, 5)])
def test_int_shapes(torch_cuda, shape):
    x = int_field(shape, np.int16, seed=len(shape))
    roundtrip(torch_cuda, x, make_cfg(shape, dtype="i16", eb=3.0, eb_mode="abs", kind="nat"),
              f"i16 {shape}")


@pytest.mark.parametrize("B,al", [(32, 6), (8, 4)])
def test_int_block_wise(torch_cuda, B, al):
    x = int_field((70, 66, 97), np.uint16, seed=9)
    cand = candidates(3)
    nb = int(np.prod([(s + B - 1) // B for s in x.shape]))
    bc = (np.arange(nb) * 5 % 11).astype(np.uint8)
    cfg = make_cfg(x.shape, dtype="u16", eb=5.0, eb_mode="abs", kind="nat", anchor_log2=al,
                   block_log2=int(np.log2(B)), cand=cand, block_cfg=bc)
    roundtrip(torch_cuda, x, cfg, f"u16 block-wise B={B}")


def test_int_clamp(torch_cuda):
    rng = np.random.default_rng(2)
    x = np.where(rng.uniform(size=(40, 40, 20)) < 0.5, 0, 255).astype(np.uint8)
    x[:, :20] = 255
    roundtrip(torch_cuda, x, make_cfg(x.shape, dtype="u8", eb=6.0, eb_mode="abs", kind="nak"),
              "u8 clamp")


@pytest.mark.parametrize("name,npdt", [("u8", np.uint8), ("i32", np.int32)])
def test_int_tune(torch_cuda, name, npdt):
    from paper_2311_12133_amd import binding
    x = int_field((64, 96, 80), npdt, span=None if name != "i32" else 1 << 20)
    cfg = make_cfg(x.shape, dtype=name, eb=1e-3)
    opts = dict(global_rate=0.2, tune_ab=1)
    print(f"[case] tune {name}", flush=True)
    ref, rep = O.tune(x, cfg, opts)
    xt = torch_cuda.from_numpy(x).cuda()
    got = binding.tune(xt, cfg, opts)
    for k in ("predictor", "anchor_log2", "frozen_dim", "block_log2", "md_w", "levels", "cand",
              "alpha", "beta"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.array_equal(got["block_cfg"], ref["block_cfg"])
    assert got["predictor"] == "interp"
    s = binding.compress(xt, got)
    assert s.cpu().numpy().tobytes() == O.compress(x, ref)


def test_int_batch_and_quality(torch_cuda):
    torch = torch_cuda
    from paper_2311_12133_amd import binding
    xs = [int_field((40, 36, 34), np.uint8), fields.fronts_field((40, 36, 34)),
          int_field((50, 61), np.int32, span=1 << 18)]
    cfgs = [make_cfg(xs[0].shape, dtype="u8", eb=1.5, eb_mode="abs", kind="nat"),
            make_cfg(xs[1].shape, dtype="f32", eb=1e-3, kind="nat"),
            make_cfg(xs[2].shape, dtype="i32", eb=10.0, eb_mode="abs", kind="nak", md=1)]
    ts = [torch.from_numpy(x).cuda() for x in xs]
    outs = binding.compress_batch(ts, cfgs)
    for x, c, s in zip(xs, cfgs, outs):
        assert s.cpu().numpy().tobytes() == O.compress(x, c)
    recs = binding.decompress_batch(outs)
    for x, c, y in zip(xs, cfgs, recs):
        assert np.array_equal(y.cpu().numpy(), O.decompress(O.compress(x, c)))
    # quality of an integer reconstruction (read in its own type)
    q = binding.quality(ts[0], recs[0])
    want = Q.metrics(xs[0], recs[0].cpu().numpy())
    assert q["max_abs_err"] == want["max_abs_err"] and q["value_range"] == want["value_range"]
    assert q["mse"] == pytest.approx(want["mse"], rel=1e-12)
    assert q["ssim"] == pytest.approx(want["ssim"], rel=1e-12)


def test_int_rejects_lorenzo(torch_cuda):
    from paper_2311_12133_amd import binding
    x = int_field((30, 30, 30), np.int16)
    with pytest.raises(binding.HpezError) as ei:
        binding.compress(torch_cuda.from_numpy(x).cuda(),
                         make_cfg(x.shape, dtype="i16", eb=2.0, eb_mode="abs",
                                  predictor="lorenzo"))
    assert ei.value.code == -6
