"""Pins of the Lorenzo alternative (Sec. 6.5) and of the tuner (Sec. 6) in the
CPU oracle.  Tuner decisions have no printed values in the paper to compare
with (parity with the paper is unpinned there); these tests pin the pieces
that mathematics fixes and the decisions that are forced by construction."""
from __future__ import annotations

import numpy as np
import pytest

from cfgs import candidates, make_cfg
from oracle import oracle as O
from paper_2311_12133_amd import fields


def brick_order(shape, S=32):
    """Stream order: bricks of S points per dim in row-major order, points of a
    brick in row-major order (re-derived with numpy index arithmetic)."""
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    nb = [(n + S - 1) // S for n in shape]
    out = []
    for b in np.ndindex(*nb):
        sl = tuple(slice(bi * S, min((bi + 1) * S, n)) for bi, n in zip(b, shape))
        out.append(idx[sl].reshape(-1))
    return np.concatenate(out)


@pytest.mark.parametrize("shape", [(70,), (33, 65), (40, 31, 70), (5, 33, 2, 40)])
def test_stream_order(shape):
    o = O.stream_order(shape)
    assert np.array_equal(o, brick_order(shape))
    assert np.array_equal(np.sort(o), np.arange(o.size))


def mixed_difference(v):
    """First-order Lorenzo residual: backward difference along every axis with
    zero outside the grid."""
    d = v.copy()
    for ax in range(v.ndim):
        if v.shape[ax] > 1:
            d = np.diff(d, axis=ax, prepend=0)
    return d


@pytest.mark.parametrize("shape", [(200,), (31, 45), (12, 17, 23)])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_lorenzo_residuals_and_bound(shape, dtype):
    T = np.float32 if dtype == "f32" else np.float64
    x = fields.random_field(shape, 3, T, "mixed")
    cfg = make_cfg(shape, dtype=dtype, eb=1e-3, predictor="lorenzo")
    e, _ = O.error_bound(x, cfg)
    r = O.lorenzo_codes(x, cfg, e)
    t = x.astype(np.float64) * (1.0 / (2.0 * e))
    v = (np.sign(t) * np.floor(np.abs(t) + 0.5)).astype(np.int64)
    delta = mixed_difference(v)
    R = 32768
    inr = np.abs(delta) < R
    assert np.array_equal(r["code"][inr].astype(np.int64), delta[inr] + R)
    assert (r["code"][~inr] == 0).all()
    # outliers are listed in stream (brick) order
    flat = delta.reshape(-1)[brick_order(shape)]
    assert np.array_equal(r["outliers"], flat[np.abs(flat) >= R])
    s = O.compress(x, cfg)
    y = O.decompress(s)
    assert np.abs(x.astype(np.float64) - y).max() <= e
    assert np.array_equal(y, r["W"])


def test_lorenzo_exact_on_bilinear():
    """A 2D field a*i + b*j on the quantization lattice has zero residual
    everywhere except the first row and column."""
    e = 0.5
    i, j = np.meshgrid(np.arange(20), np.arange(30), indexing="ij")
    x = (3 * i - 2 * j + 7).astype(np.float64)  # multiples of 2e = 1
    cfg = make_cfg(x.shape, dtype="f64", eb=e, eb_mode="abs", predictor="lorenzo")
    r = O.lorenzo_codes(x, cfg, e)
    assert (r["code"][1:, 1:] == 32768).all()
    assert np.array_equal(O.decompress(O.compress(x, cfg)), x)


def test_candidates():
    c = O.candidates(3)
    assert c == [dict(kind=k["kind"], md=k["md"], same_level=k["same_level"],
                      order=tuple(k["order"])) for k in candidates(3)]
    assert len(c) == 11 and len({str(v) for v in c}) == 11


def test_tune_freezes_rough_dim():
    """Sec. 6.3: smooth along dims 1, 2 but white noise along dim 0 -> the least
    smooth dim is 0 and freezing it wins."""
    rng = np.random.default_rng(1)
    n = 64
    base = fields.gaussian_field((n, n), -3.0, rng)
    x = (base[None, :, :] + 0.5 * rng.standard_normal((n, 1, 1))).astype(np.float32)
    cfg = make_cfg(x.shape, eb=1e-3)
    out, rep = O.tune(x, cfg, dict(global_rate=0.25, block_wise=0, allow_lorenzo=0))
    assert rep["freeze_candidate"] == 0
    assert rep["sigma2"][0][0] > 10 * rep["sigma2"][0][1]
    assert out["frozen_dim"] == 0
    e, _ = O.error_bound(x, out)
    y = O.decompress(O.compress(x, out))
    assert np.abs(x.astype(np.float64) - y).max() <= e


def test_tune_smooth_prefers_cubic_and_weights():
    """Smooth data: a cubic candidate wins every level that has interior
    stencils (at s = 16 a 33^3 trial box only has end stencils, where all
    candidates tie and the lowest index wins), and the MD weights are
    1/sigma^2 of the statistics (Eq. 12)."""
    x = fields.plain_field((64, 64, 64))
    cfg = make_cfg(x.shape, eb=1e-4)
    out, rep = O.tune(x, cfg, dict(global_rate=0.1, block_wise=0, allow_lorenzo=1,
                                   allow_freeze=1))
    assert out["predictor"] == "interp"
    for l in range(1, 5):
        assert out["levels"][l - 1]["kind"] in (1, 2)
    assert out["levels"][4]["kind"] == 0
    s2 = rep["sigma2"]
    for k in range(3):
        for d in range(3):
            assert out["md_w"][k][d] == 1.0 / max(s2[k][d], 1.0)


def test_tune_noise_prefers_lorenzo():
    """Sec. 6.5: on white noise at a tight bound the Lorenzo residual entropy is
    not worse than interpolation's, so with a coefficient below one Lorenzo is
    chosen; with a large coefficient it is not."""
    x = fields.random_field((64, 64, 64), 9, np.float32, "rough")
    cfg = make_cfg(x.shape, eb=1e-4)
    out, rep = O.tune(x, cfg, dict(global_rate=0.1, block_wise=0, lorenzo_coef=0.5))
    assert out["predictor"] == "lorenzo"
    out2, _ = O.tune(x, cfg, dict(global_rate=0.1, block_wise=0, lorenzo_coef=4.0))
    assert out2["predictor"] == "interp"


def test_tune_block_wise_roundtrip():
    """Sec. 6.6: block-wise tuning fills one candidate per 32^3 block; the tuned
    configuration compresses within the bound."""
    x = fields.fronts_field((64, 96, 80))
    cfg = make_cfg(x.shape, eb=1e-3)
    out, rep = O.tune(x, cfg, dict(global_rate=0.2, sub_rate=0.04, block_wise=1,
                                   allow_lorenzo=0))
    assert out["block_log2"] == 5
    nb = 2 * 3 * 3
    assert out["block_cfg"].shape == (nb,)
    assert out["block_cfg"].max() < 11
    e, _ = O.error_bound(x, out)
    s = O.compress(x, out)
    y = O.decompress(s)
    assert np.abs(x.astype(np.float64) - y).max() <= e
