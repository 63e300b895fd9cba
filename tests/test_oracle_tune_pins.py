"""Pins of the tuner's decisions in the CPU oracle against an independent
brute force.

Sec. 6.2 picks, per level, the candidate with the lowest prediction error on
sampled regions; Sec. 6.3 and 6.5 compare estimated sizes; Sec. 6.6 tunes one
configuration per block on a centred sub-block.  The paper prints no per-block
decisions, so these tests recompute each decision from its definition with the
pure-Python twin (`oracle/tiny.py`, written separately from the C oracle) and
numpy, and require the oracle's decisions and estimates to equal them:

  * the size estimate is the zeroth-order entropy in bits (hand-computed
    histograms, and the Lorenzo trial's estimate recomputed with numpy);
  * the global per-level scores, the per-level argmin and the unfrozen size
    estimate (entropy of the tuned trial's codes plus the anchors' verbatim
    bits) recomputed from trial compressions of the sampled boxes;
  * every block's configuration is the argmin (ties to the lowest index) of the
    candidates' total scores on the centred sub-block.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from cfgs import make_cfg
from oracle import oracle as O
from oracle.tiny import Tiny
from paper_2311_12133_amd import fields


# ---------------------------------------------------------------------------
# the size estimate (Sec. 6.3 / 6.5), hand-computed values

def test_entropy_bits_hand_values():
    # four equally likely symbols: 2 bits each
    assert O.entropy_bits([0, 5, 5, 0, 5, 5]) == 2.0
    # a 1:3 split: H = 1/4 log2 4 + 3/4 log2 (4/3) = 2 - (3/4) log2 3
    h = O.entropy_bits([1, 0, 3])
    assert abs(h - 0.8112781244591328) < 1e-15
    assert abs(h - (2.0 - 0.75 * math.log2(3.0))) < 1e-15
    # one symbol: no information; empty histogram: zero by convention
    assert O.entropy_bits([0, 0, 9, 0]) == 0.0
    assert O.entropy_bits(np.zeros(65536, np.uint64)) == 0.0
    # eight equal symbols spread over a 65536-bin alphabet: 3 bits
    hist = np.zeros(65536, np.uint64)
    hist[[0, 7, 100, 32767, 32768, 40000, 65000, 65535]] = 11
    assert O.entropy_bits(hist) == 3.0


def np_entropy(hist):
    hist = np.asarray(hist, dtype=np.float64)
    n = hist.sum()
    nz = hist[hist > 0]
    return float((nz * np.log2(n / nz)).sum() / n) if n else 0.0


# ---------------------------------------------------------------------------
# sampled regions of the global trials (Sec. 6.2): (B+1)^D boxes at the origins
# of every k-th block, k = round(1 / rate), starting at block k // 2

def sampled_boxes(shape, B, rate):
    nb = [(n + B - 1) // B for n in shape]
    nbt = int(np.prod(nb))
    k = max(1, int(math.floor(1.0 / rate + 0.5)))
    first = k // 2
    if first >= nbt:
        first = nbt // 2
    out = []
    for bi in range(first, nbt, k):
        b = np.unravel_index(bi, nb)
        sl = tuple(slice(bd * B, min(bd * B + B + 1, n)) for bd, n in zip(b, shape))
        out.append(sl)
    return out


def round_half_away(t):
    return np.sign(t) * np.floor(np.abs(t) + 0.5)


@pytest.mark.parametrize("shape,rate", [((48, 40, 70), 0.25), ((70, 100), 0.3)])
def test_lorenzo_estimate_recomputed(shape, rate):
    """The Lorenzo trial's estimate (Sec. 6.5) is the entropy, in bits, of the
    first-order Lorenzo codes of the sampled boxes, recomputed here with numpy:
    dual quantization v = round(x / 2e), the backward mixed difference, codes
    delta + R inside the radius and 0 outside."""
    x = fields.fronts_field(shape)
    cfg = make_cfg(shape, eb=1e-3)
    e, _ = O.error_bound(x, cfg)
    _, rep = O.tune(x, cfg, dict(global_rate=rate, block_wise=0, allow_freeze=0,
                                 allow_lorenzo=1))
    R = 32768
    hist = np.zeros(2 * R, np.int64)
    for sl in sampled_boxes(shape, 32, rate):
        box = x[sl].astype(np.float64)
        v = round_half_away(box * (1.0 / (2.0 * e))).astype(np.int64)
        d = v.copy()
        for ax in range(d.ndim):
            if d.shape[ax] > 1:
                d = np.diff(d, axis=ax, prepend=0)
        codes = np.where(np.abs(d) < R, d + R, 0)
        hist += np.bincount(codes.reshape(-1), minlength=2 * R)
    want = np_entropy(hist)
    assert abs(rep["H_lorenzo"] - want) <= 1e-12 * max(1.0, want)
    assert rep["H_lorenzo"] > 0.5  # a real estimate, not a degenerate one


# ---------------------------------------------------------------------------
# global tuning (Sec. 6.2) and the unfrozen size estimate (Sec. 6.3)

def tiny_trial(box, cfg, e, levels, anchor_log2, frozen=-1):
    """One closed-loop trial compression of a small region with the twin;
    returns (per-level scores, codes of the predicted points)."""
    tc = dict(cfg)
    tc.update(dims=tuple(box.shape), anchor_log2=anchor_log2, levels=levels, block_log2=0,
              frozen_dim=frozen, alpha=1.0, beta=1.0)
    t = Tiny(box, tc, e)
    t.score = {}
    code, _ = t.compress()
    anc = np.zeros(box.size, bool)
    anc[t.anchors()] = True
    return t.score, code[~anc]


def test_global_scores_argmin_and_estimate_recomputed():
    """2-D field, four sampled boxes (33x33, clipped at the grid end): every candidate's per-level score,
    the per-level winner (lowest score, ties to the lowest index; levels above
    the block size reuse the block-size level's winner) and the unfrozen size
    estimate H = entropy(tuned trial codes) + anchors * 32 / N."""
    shape = (70, 100)
    rate = 0.3
    x = fields.fronts_field(shape)
    cfg = make_cfg(shape, eb=1e-3)
    e, _ = O.error_bound(x, cfg)
    out, rep = O.tune(x, cfg, dict(global_rate=rate, block_wise=0, allow_freeze=0,
                                   allow_lorenzo=0))
    cands = O.candidates(2)
    tcfg = dict(cfg, md_w=out["md_w"])
    boxes = [x[sl] for sl in sampled_boxes(shape, 32, rate)]
    assert len(boxes) == 4  # k = 3 of 12 blocks, from block 1
    Lb = 5
    score = np.zeros((11, 17), np.uint64)
    for ci, c in enumerate(cands):
        for box in boxes:
            sc, _ = tiny_trial(box, tcfg, e, [c] * 16, Lb)
            for lvl, v in sc.items():
                score[ci, lvl] += np.uint64(v)
    assert np.array_equal(score[:, :16], rep["global_score"][0][:, :16])
    best = {l: int(np.argmin(score[:, l])) for l in range(1, Lb + 1)}  # argmin: first minimum
    L = out["anchor_log2"]
    for l in range(1, L + 1):
        assert out["levels"][l - 1] == cands[best[min(l, Lb)]], l
    # the level winners differ from the worst candidates (the test has power)
    assert any(best[l] != int(np.argmax(score[:, l])) for l in best)
    hist = np.zeros(65536, np.int64)
    levels = [cands[best[min(l, Lb)]] for l in range(1, 17)]
    for box in boxes:
        _, codes = tiny_trial(box, tcfg, e, levels, Lb)
        hist += np.bincount(codes.astype(np.int64), minlength=65536)
    A = 1 << L
    anchors = np.prod([(n - 1) // A + 1 for n in shape])
    want = np_entropy(hist) + anchors * 4 * 8.0 / np.prod(shape)
    assert abs(rep["H"][0] - want) <= 1e-12 * want


# ---------------------------------------------------------------------------
# block-wise tuning (Sec. 6.6)

def sub_block(shape, b, B, side):
    """Centred sub-block of block b: side `side` clipped to the block's extent,
    offset (extent - side) // 2 inside the block."""
    sl = []
    for bd, n in zip(b, shape):
        ext = min(B, n - bd * B)
        m = min(side, ext) if n > 1 else 1
        o = bd * B + (ext - m) // 2
        sl.append(slice(o, o + m))
    return tuple(sl)


def corner_block(shape, b, B, side):
    sl = []
    for bd, n in zip(b, shape):
        ext = min(B, n - bd * B)
        m = min(side, ext) if n > 1 else 1
        sl.append(slice(bd * B, bd * B + m))
    return tuple(sl)


def brute_block_choice(x, cfg, e, md_w, sub_rate, region, B=32):
    shape = x.shape
    D = sum(1 for n in shape if n > 1)
    side = int(math.floor(B * sub_rate ** (1.0 / D) + 0.5))
    side = min(max(side, 3), B)
    al = 0
    while (1 << (al + 1)) <= side - 1:
        al += 1
    cands = O.candidates(len(shape))
    tcfg = dict(cfg, md_w=md_w)
    nb = [(n + B - 1) // B for n in shape]
    choice, worst = [], []
    for b in np.ndindex(*nb):
        box = x[region(shape, b, B, side)]
        tot = []
        for c in cands:
            sc, _ = tiny_trial(box, tcfg, e, [c] * 16, al)
            tot.append(sum(sc.values()))
        choice.append(int(np.argmin(tot)))  # first minimum: ties to the lowest index
        worst.append(int(np.argmax(tot)))
    return np.array(choice, np.uint8), np.array(worst, np.uint8)


def block_pattern_field(shape, seed):
    """Blocks whose centre and corner differ in character: a smooth background,
    a per-block quadratic ramp along a per-block dimension in each block's
    centre, and a period-2 ripple in each block's low corner."""
    rng = np.random.default_rng(seed)
    x = fields.gaussian_field(shape, -3.0, rng) * 0.3
    nb = [(n + 31) // 32 for n in shape]
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    for b in np.ndindex(*nb):
        lo = [bd * 32 for bd in b]
        cen = tuple(slice(l + 8, min(l + 24, n)) for l, n in zip(lo, shape))
        cor = tuple(slice(l, min(l + 10, n)) for l, n in zip(lo, shape))
        d = int(rng.integers(len(shape)))
        u = grids[d][cen] - lo[d]
        x[cen] += rng.uniform(0.5, 2.0) * (u / 16.0) ** 2 * rng.choice([-1.0, 1.0])
        par = sum(g[cor] for g in grids) % 2
        x[cor] += rng.uniform(0.2, 0.6) * (2.0 * par - 1.0)
    return x.astype(np.float32)


@pytest.mark.parametrize("shape,sub_rate", [((64, 64, 50), 0.04), ((96, 77), 0.04),
                                            ((40, 70, 36), 0.02)])
def test_block_choice_brute_force(shape, sub_rate):
    """Every block's configuration (Sec. 6.6) equals the brute-force argmin of
    the candidates' total scores on the block's centred sub-block, blocks
    clipped at the grid end included; the same choice made on the block's low
    corner, or by argmax, differs somewhere, so the pin sees both mistakes."""
    x = block_pattern_field(shape, 7 + len(shape))
    cfg = make_cfg(shape, eb=1e-3)
    e, _ = O.error_bound(x, cfg)
    out, _ = O.tune(x, cfg, dict(global_rate=0.5, sub_rate=sub_rate, block_wise=1,
                                 allow_freeze=0, allow_lorenzo=0))
    assert out["frozen_dim"] == -1 and out["predictor"] == "interp"
    want, worst = brute_block_choice(x, cfg, e, out["md_w"], sub_rate, sub_block)
    assert np.array_equal(out["block_cfg"], want)
    corner, _ = brute_block_choice(x, cfg, e, out["md_w"], sub_rate, corner_block)
    assert not np.array_equal(corner, want)
    assert not np.array_equal(worst, want)
    # more than one candidate is chosen across the blocks
    assert len(set(want.tolist())) > 1


# ---------------------------------------------------------------------------
# level-wise error bounds (Sec. 6.4, Eq. 15): (alpha, beta) tuning

AB_GRID = [(1.0, 1.0)] + [(a, b) for a in (1.25, 1.5, 1.75, 2.0) for b in (1.5, 2.0, 3.0, 4.0)]


def lognormal_2d(shape, seed):
    g = fields.gaussian_field(shape, -5.0 / 3.0, np.random.default_rng(seed))
    return np.exp(1.5 * g).astype(np.float32)


@pytest.mark.parametrize("make,eb,radius,nontrivial", [
    (lambda: lognormal_2d((70, 100), 0), 1e-4, 32768, True),
    (lambda: fields.fronts_field((70, 100)), 1e-3, 64, False),
])
def test_alpha_beta_brute_force(make, eb, radius, nontrivial):
    """Every (alpha, beta) pair's rate, distortion and score, recomputed from
    trial compressions of the sampled boxes with the twin under the tuned
    per-level configuration and the pair's level bounds (Eq. 15): rate =
    entropy of the codes + verbatim bits of the unpredictable points per
    predicted point, D = sum floor(((x - x') / e)^2 2^32), score =
    -10 log10((D + 1) / (n 2^32)) - 20 log10(2) rate; the chosen pair is the
    first maximum.  One field picks a pair other than (1, 1), the other has
    unpredictable points (radius 64), so the rate's verbatim term counts."""
    x = make()
    shape = x.shape
    rate = 0.3
    cfg = make_cfg(shape, eb=eb, radius=radius)
    e, _ = O.error_bound(x, cfg)
    out, rep = O.tune(x, cfg, dict(global_rate=rate, block_wise=0, allow_freeze=0,
                                   allow_lorenzo=0, tune_ab=1))
    assert [(a, b) for a, b in zip(rep["ab_alpha"], rep["ab_beta"])] == AB_GRID
    Lb = 5
    boxes = [x[sl] for sl in sampled_boxes(shape, 32, rate)]
    scores, unpred = [], 0
    for c, (a, b) in enumerate(AB_GRID):
        hist = np.zeros(2 * radius, np.int64)
        sq = 0
        for box in boxes:
            tc = dict(cfg, dims=tuple(box.shape), anchor_log2=Lb, levels=out["levels"],
                      block_log2=0, frozen_dim=-1, alpha=a, beta=b, md_w=out["md_w"])
            t = Tiny(box, tc, e)
            code, W = t.compress()
            pred = np.ones(box.size, bool)
            pred[t.anchors()] = False
            hist += np.bincount(code[pred].astype(np.int64), minlength=2 * radius)
            inv_e = 1.0 / e
            for xv, wv in zip(box.reshape(-1)[pred], W[pred]):
                u = (float(xv) - float(wv)) * inv_e
                sq += math.floor(u * u * 4294967296.0)
        n = int(hist.sum())
        r = np_entropy(hist) + hist[0] * 4 * 8.0 / n
        score = -10.0 * math.log10((sq + 1.0) / (n * 4294967296.0)) - 20.0 * math.log10(2.0) * r
        assert rep["ab_sq"][c] == sq, (c, rep["ab_sq"][c], sq)
        assert abs(rep["ab_rate"][c] - r) <= 1e-12 * max(1.0, r), c
        assert abs(rep["ab_score"][c] - score) <= 1e-9 * max(1.0, abs(score)), c
        scores.append(score)
        unpred += int(hist[0])
    best = int(np.argmax(scores))  # first maximum: ties to the earlier pair
    assert rep["ab_choice"] == best
    assert (out["alpha"], out["beta"]) == AB_GRID[best]
    assert (best != 0) == nontrivial
    if radius < 1000:
        assert unpred > 0


def test_alpha_beta_off_keeps_caller_values():
    """Without tune_ab the caller's alpha and beta pass through unchanged."""
    x = fields.fronts_field((40, 50, 36))
    cfg = make_cfg(x.shape, eb=1e-3, alpha=1.5, beta=3.0)
    out, rep = O.tune(x, cfg, dict(global_rate=0.3, block_wise=0))
    assert (out["alpha"], out["beta"]) == (1.5, 3.0) and rep["ab_choice"] == -1
