"""Pins of the oracle's quality metrics and quality-target search (Sec. 3.1,
Eq. 1: M(X, X') >= m0 with M = PSNR or SSIM).

The metrics are checked against closed forms that do not share the oracle's
per-window loop (a constant shift, affine maps, equal inputs), against a
summed-area-table brute force of the windowed moments, and against the
window placement rule on ragged shapes.  The search is checked by what its
result must satisfy: the returned bound meets the target, the bracketing
bound above it misses it, and the two are adjacent bounds of the search grid."""
from __future__ import annotations

import math

import numpy as np
import pytest

from cfgs import make_cfg
from oracle import oracle_quality as Q
from paper_2311_12133_amd import fields


def _field(shape, seed=3):
    rng = np.random.default_rng(seed)
    return fields.gaussian_field(shape, -5.0 / 3.0, rng).astype(np.float32)


def _block_view(a, win):
    """Windows of a as an array [windows..., window cells...] by reshaping
    (independent of the oracle's slicing loop)."""
    sl = tuple(slice(0, s * n) for s, n in win)
    b = a[sl]
    shp = []
    for s, n in win:
        shp += [n, s]
    b = b.reshape(shp)
    nd = len(win)
    perm = [2 * i for i in range(nd)] + [2 * i + 1 for i in range(nd)]
    return b.transpose(perm).reshape([n for _, n in win] + [-1])


def _win(shape, w):
    return [(1, 1) if n <= 1 else (n, 1) if n < w else (w, n // w) for n in shape]


def test_psnr_constant_shift_closed_form():
    x = _field((20, 24, 17)).astype(np.float64)
    c = 2.0 ** -10
    q = Q.metrics(x, x + c)
    L = float(x.max() - x.min())
    assert q["mse"] == c * c
    assert q["max_abs_err"] == c
    assert q["psnr"] == pytest.approx(20 * math.log10(L) - 20 * math.log10(c), rel=0, abs=1e-12)


def test_psnr_two_level_error_pattern():
    # errors +d on half the points and -2d on the other half: MSE = 2.5 d^2
    x = _field((16, 16, 16)).astype(np.float64)
    d = 2.0 ** -12
    err = np.where(np.arange(x.size).reshape(x.shape) % 2 == 0, d, -2 * d)
    q = Q.metrics(x, x + err)
    assert q["mse"] == pytest.approx(2.5 * d * d, rel=1e-14)
    assert q["max_abs_err"] == 2 * d


def test_psnr_exact_and_constant_cases():
    x = _field((9, 11))
    assert Q.metrics(x, x)["psnr"] == math.inf
    z = np.full((7, 5), 3.0, np.float32)
    assert Q.metrics(z, z)["psnr"] == math.inf
    assert Q.metrics(z, z + 1)["psnr"] == -math.inf


def test_ssim_equal_inputs_is_one():
    x = _field((24, 17, 33))
    s, nw = Q.ssim(x, x)
    assert s == 1.0
    assert nw == 3 * 2 * 4


@pytest.mark.parametrize("shape", [(32, 24, 16), (40, 19), (300,), (9, 16, 5, 8)])
def test_ssim_shift_closed_form(shape):
    x = _field(shape).astype(np.float64)
    c = 0.125
    L = float(x.max() - x.min())
    C1 = (0.01 * L) ** 2
    m = _block_view(x, _win(shape, 8)).mean(axis=-1)
    want = np.mean((2 * m * (m + c) + C1) / (m * m + (m + c) ** 2 + C1))
    got, nw = Q.ssim(x, x + c)
    assert nw == m.size
    assert got == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("a,b", [(0.5, 0.0), (-1.0, 0.25), (1.5, -0.75)])
def test_ssim_affine_closed_form(a, b):
    shape = (24, 32, 16)
    x = _field(shape).astype(np.float64)
    L = float(x.max() - x.min())
    C1, C2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    v = _block_view(x, _win(shape, 8))
    m = v.mean(axis=-1)
    s2 = v.var(axis=-1)
    my = a * m + b
    want = np.mean(((2 * m * my + C1) * (2 * a * s2 + C2)) /
                   ((m * m + my * my + C1) * (s2 + a * a * s2 + C2)))
    got, _ = Q.ssim(x, a * x + b)
    assert got == pytest.approx(want, rel=1e-11)


def _sat_ssim(x, y, w):
    """Windowed SSIM from summed-area tables of x, y, x^2, y^2, xy (one-pass
    moments), windows at multiples of w along every dim >= w."""
    L = float(x.max() - x.min())
    C1, C2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    win = _win(x.shape, w)
    tabs = []
    for f in (x, y, x * x, y * y, x * y):
        t = np.pad(f, [(1, 0)] * f.ndim)
        for ax in range(f.ndim):
            t = np.cumsum(t, axis=ax)
        tabs.append(t)
    n = int(np.prod([s for s, _ in win]))
    total, cnt = 0.0, 0
    import itertools
    for idx in itertools.product(*[range(k) for _, k in win]):
        lo = [i * s for i, (s, _) in zip(idx, win)]
        hi = [l + s for l, (s, _) in zip(lo, win)]
        sums = []
        for t in tabs:
            acc = 0.0
            for corner in itertools.product((0, 1), repeat=x.ndim):
                pos = tuple(hi[k] if corner[k] else lo[k] for k in range(x.ndim))
                sign = (-1) ** (x.ndim - sum(corner))
                acc += sign * t[pos]
            sums.append(acc)
        mx, my = sums[0] / n, sums[1] / n
        sxx = sums[2] / n - mx * mx
        syy = sums[3] / n - my * my
        sxy = sums[4] / n - mx * my
        total += ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
        cnt += 1
    return total / cnt, cnt


@pytest.mark.parametrize("shape,w", [((21, 18, 12), 8), ((30, 13), 8), ((17, 9, 10), 4),
                                     ((50,), 7)])
def test_ssim_brute_force_windows(shape, w):
    rng = np.random.default_rng(11)
    x = _field(shape).astype(np.float64)
    y = x + rng.normal(0, 0.05, size=shape)
    got, nw = Q.ssim(x, y, w)
    want, nw2 = _sat_ssim(x, y, w)
    assert nw == nw2
    assert got == pytest.approx(want, rel=1e-9)


def test_ssim_window_rule_ragged():
    # dims 5 (< w: one window of 5), 19 (two windows of 8, 3 left out), 8 (one)
    x = _field((5, 19, 8)).astype(np.float64)
    y = x * 0.9
    _, nw = Q.ssim(x, y)
    assert nw == 2
    # the points outside the windows do not matter
    y2 = y.copy()
    y2[:, 16:, :] += 100.0
    assert Q.ssim(x, y2)[0] == Q.ssim(x, y)[0]


@pytest.mark.parametrize("metric,target", [("psnr", 70.0), ("psnr", 45.0), ("ssim", 0.999)])
def test_fit_eb_brackets_target(metric, target):
    shape = (24, 20, 18)
    x = _field(shape)
    cfg = make_cfg(shape, kind="nat")
    e, q, it, hi = Q.fit_eb(x, cfg, metric, target, max_iter=24)
    assert e > 0
    assert q[metric] >= target
    assert it < 24
    from oracle import oracle as O
    # the reported metrics are those of the compression at e
    xr = O.decompress(O.compress(x, dict(cfg, eb_mode="abs", eb=e)))
    assert Q.metrics(x, xr)[metric] == q[metric]
    assert q["max_abs_err"] <= e
    # the ceiling of the bracket is the next grid bound and misses the target
    L = Q.value_range(x)
    k = round(Q.STEPS * math.log2(e / L))
    assert e == Q.grid_eb(L, k)
    assert hi == Q.grid_eb(L, k + 1)
    xr2 = O.decompress(O.compress(x, dict(cfg, eb_mode="abs", eb=hi)))
    assert Q.metrics(x, xr2)[metric] < target


def test_fit_eb_psnr_model_start():
    # the first PSNR bound follows the uniform-error model e = L sqrt(3) 10^(-t/20)
    for t in (40.0, 63.5, 100.0):
        k = Q.initial_k("psnr", t)
        r = Q.grid_eb(1.0, k)
        assert abs(math.log2(r / (math.sqrt(3) * 10 ** (-t / 20)))) <= 0.5 / Q.STEPS + 1e-12


def test_fit_eb_model_steps():
    # a PSNR 6.0206 dB above the target is one octave (G steps) of e
    assert Q.model_step("psnr", 60.0, 60.0 + 20 * math.log10(2)) == Q.STEPS
    assert Q.model_step("psnr", 60.0, 60.0 - 20 * math.log10(2)) == -Q.STEPS
    assert Q.model_step("psnr", 60.0, 60.0) == 1
    assert Q.model_step("psnr", 60.0, 59.9999999) == -1
    assert Q.model_step("psnr", 60.0, math.inf) == 4 * Q.STEPS
    # SSIM deficit four times too small: e may double
    assert Q.model_step("ssim", 0.99, 1 - 0.01 / 4) == Q.STEPS
    assert Q.model_step("ssim", 0.99, 1.0) == 4 * Q.STEPS


def test_fit_eb_constant_field():
    x = np.full((8, 9, 10), 2.5, np.float32)
    e, q, it, hi = Q.fit_eb(x, make_cfg(x.shape), "psnr", 80.0)
    assert e == 0.0 and it == 0 and q["psnr"] == math.inf
