"""Huffman pins (Sec. 4 step 4) and the brute-force tiny-grid cross-check of
the oracle's interpolation schedule (Sec. 5.1, 5.3, 5.4, 6.3, 6.6)."""
from __future__ import annotations

import heapq
import itertools

import numpy as np
import pytest

from cfgs import candidates, make_cfg
from oracle import oracle as O
from oracle.tiny import Tiny
from paper_2311_12133_amd import fields


def heap_huffman_cost(counts):
    """Textbook Huffman (heap of subtree weights): the optimal total bit count
    sum(count * length) is the same for every valid tie-break."""
    w = [int(c) for c in counts if c > 0]
    if len(w) == 1:
        return w[0]
    heapq.heapify(w)
    cost = 0
    while len(w) > 1:
        a, b = heapq.heappop(w), heapq.heappop(w)
        cost += a + b
        heapq.heappush(w, a + b)
    return cost


@pytest.mark.parametrize("seed", range(8))
def test_huffman_optimal_and_prefix_free(seed):
    rng = np.random.default_rng(seed)
    nsym = 300
    counts = np.zeros(nsym, dtype=np.uint64)
    used = rng.choice(nsym, rng.integers(2, 200), replace=False)
    counts[used] = rng.geometric(0.05, used.size)
    lens = O.huff_lengths(counts)
    assert ((lens > 0) == (counts > 0)).all()
    assert int((counts * lens.astype(np.uint64)).sum()) == heap_huffman_cost(counts)
    # Kraft equality: a complete prefix code
    assert sum(2.0 ** -int(l) for l in lens if l) == 1.0
    cw = O.huff_canonical(lens)
    codes = {(int(lens[s]), int(cw[s])) for s in range(nsym) if lens[s]}
    words = [format(c, f"0{l}b") for l, c in codes]
    for a, b in itertools.permutations(words, 2):
        assert not b.startswith(a)
    # canonical: ordering by (length, symbol) gives increasing codewords
    order = sorted((int(lens[s]), s) for s in range(nsym) if lens[s])
    vals = [int(cw[s]) << (32 - l) for l, s in order]
    assert vals == sorted(vals) and len(set(vals)) == len(vals)


def test_huffman_roundtrip_and_chunks():
    rng = np.random.default_rng(1)
    sym = (32768 + np.round(rng.standard_normal(5000) * 3)).astype(np.uint16)
    counts = np.bincount(sym, minlength=65536).astype(np.uint64)
    lens = O.huff_lengths(counts)
    cw = O.huff_canonical(lens)
    for chunk in (64, 1024):
        words, bits, cb = O.huff_encode(sym, lens, cw, chunk)
        assert int(cb.sum()) == bits
        assert bits == int((counts * lens.astype(np.uint64)).sum())
        out = O.huff_decode(words, bits, lens, chunk, cb, sym.size)
        assert np.array_equal(out, sym)


def test_huffman_single_symbol_and_length_limit():
    counts = np.zeros(10, dtype=np.uint64)
    counts[3] = 7
    lens = O.huff_lengths(counts)
    assert lens[3] == 1 and lens.sum() == 1
    # Fibonacci counts force a degenerate tree deeper than 32 levels
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    counts = np.array(fib, dtype=np.uint64)
    lens = O.huff_lengths(counts)
    assert lens.max() <= 32
    assert sum(2.0 ** -int(l) for l in lens) == 1.0


def tiny_cases():
    c3 = candidates(3)
    c2 = candidates(2)
    cases = []
    for shape in ((9,), (13, 11), (17, 9, 6), (5, 12, 7)):
        nd = len(shape)
        for kind, md, sl in itertools.product(("lin", "nak", "nat"), (0, 1), (0, 1)):
            if kind == "lin" and sl:
                continue
            cases.append((shape, dict(kind=kind, md=md, same_level=sl, anchor_log2=3)))
        if nd >= 2:
            cases.append((shape, dict(kind="nak", order=tuple(reversed(range(nd))), anchor_log2=2)))
            cases.append((shape, dict(kind="nat", frozen_dim=1, anchor_log2=3)))
            cases.append((shape, dict(kind="nat", md=1, frozen_dim=0, anchor_log2=2)))
    # block-wise: B = 4 with faces and clipped interiors
    for shape, cand in (((13, 11), c2), ((10, 9, 7), c3)):
        nb = int(np.prod([(s + 3) // 4 for s in shape]))
        bc = (np.arange(nb) * 7 % 11).astype(np.uint8)
        cases.append((shape, dict(kind="nak", anchor_log2=3, block_log2=2, cand=cand,
                                  block_cfg=bc)))
        cases.append((shape, dict(kind="lin", md=1, anchor_log2=4, block_log2=2, cand=cand,
                                  block_cfg=bc[::-1].copy())))
    return cases


@pytest.mark.parametrize("shape,kw", tiny_cases())
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_tiny_twin_matches_oracle(shape, kw, dtype):
    """Brute force: every point predicted exactly once, no read of an
    unreconstructed point, any in-pass order gives the same codes (Sec. 5.4.1),
    and the C oracle agrees bit for bit."""
    T = np.float32 if dtype == "f32" else np.float64
    x = fields.random_field(shape, sum(shape), T, "mixed")
    cfg = make_cfg(shape, dtype=dtype, eb=2e-3, **kw)
    e, _ = O.error_bound(x, cfg)
    r = O.interp_codes(x, cfg, e)
    for seed in (0, 1):
        tw = Tiny(x, cfg, e, seed=seed)
        code, W = tw.compress()
        assert np.array_equal(code, r["code"].reshape(-1))
        assert np.array_equal(W, r["W"].reshape(-1))
    y = Tiny(x, cfg, e, seed=2).decompress(code, r["anchors"], r["unpred"])
    assert np.array_equal(y, W)
