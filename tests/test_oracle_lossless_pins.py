"""Pins of the lossless-stage oracle (Sec. 4, step 5): the token definition on
hand-worked inputs, the inverse on brute-force inputs, optimality of the token
code against an independent heap-built Huffman code, the stored fallback, the
container layout, and round trips of real compressed streams."""
from __future__ import annotations

import heapq

import numpy as np
import pytest

from cfgs import make_cfg
from oracle import oracle as O
from oracle import oracle_lossless as L
from paper_2311_12133_amd import fields

R = L.RUN_MAX


@pytest.mark.parametrize("data,want", [
    (b"", []),
    (b"\x05", [5]),
    (b"\xff\x01", [255, 1]),
    (b"\x00", [256]),
    (b"\x00\x00\x00", [258]),
    (b"\x07\x00\x00\x09", [7, 257, 9]),
    (b"\x07\x00\x00", [7, 257]),
    (b"\x00\x00\x07", [257, 7]),
    (bytes(R), [255 + R]),
    (bytes(R + 1), [255 + R, 256]),
    (bytes(2 * R + 3) + b"\x02", [255 + R, 255 + R, 258, 2]),
])
def test_tokens_hand_worked(data, want):
    assert L.tokens(data).tolist() == want


def test_tokens_brute_force_inverse():
    rng = np.random.default_rng(3)
    for trial in range(40):
        n = int(rng.integers(0, 3 * R))
        p0 = rng.choice([0.0, 0.5, 0.95, 0.999, 1.0])
        b = np.where(rng.uniform(size=n) < p0, 0, rng.integers(1, 256, n)).astype(np.uint8)
        t = L.tokens(b)
        assert L.expand(t) == b.tobytes()
        # every token in range; zero bytes only ever as runs, never as literals
        assert t.size == 0 or (t.min() >= 1 and t.max() <= 255 + R)
        # runs are maximal: no two short-run tokens in a row, and a short run
        # never follows a full one except as the tail of the same run
        for a, c in zip(t[:-1].tolist(), t[1:].tolist()):
            assert not (255 < a < 255 + R and c > 255)


def heap_huffman_cost(counts):
    """Total bits of an optimal prefix code (independent construction)."""
    h = [int(c) for c in counts if c > 0]
    if len(h) == 1:
        return h[0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


def test_coded_bits_are_optimal_and_layout():
    rng = np.random.default_rng(9)
    b = np.where(rng.uniform(size=200_000) < 0.8, 0, rng.integers(1, 40, 200_000)).astype(np.uint8)
    z = L.encode(b.tobytes())
    h = L.parse(z)
    assert h["mode"] == 1 and h["n"] == b.size
    tok = L.tokens(b)
    assert h["n_tokens"] == tok.size
    counts = np.bincount(tok, minlength=L.NSYM)
    assert h["payload_bits"] == heap_huffman_cost(counts)
    used = np.flatnonzero(counts)
    assert (h["sym_min"], h["sym_max"]) == (used[0], used[-1])
    nch = -(-tok.size // L.CHUNK)
    off_chunks = (48 + used[-1] - used[0] + 1 + 7) // 8 * 8
    off_payload = (off_chunks + 2 * nch + 7) // 8 * 8
    assert len(z) == off_payload + 4 * ((h["payload_bits"] + 31) // 32)
    assert L.decode(z) == b.tobytes()


def test_stored_when_incompressible():
    rng = np.random.default_rng(1)
    b = rng.integers(1, 256, 50_000).astype(np.uint8).tobytes()
    z = L.encode(b)
    assert len(z) == L.HDR + len(b) and L.parse(z)["mode"] == 0
    assert L.decode(z) == b
    assert L.decode(L.encode(b"")) == b"" and len(L.encode(b"")) == L.HDR


def test_all_zero_input():
    n = 1_000_000
    z = L.encode(bytes(n))
    h = L.parse(z)
    full, r = divmod(n, R)
    assert h["mode"] == 1 and h["n_tokens"] == full + 1
    # two symbols: one bit each
    assert h["payload_bits"] == full + 1
    assert (h["sym_min"], h["sym_max"]) == (255 + r, 255 + R)
    assert L.decode(z) == bytes(n)


def test_single_byte_inputs():
    for v in (0, 1, 200):
        z = L.encode(bytes([v]))
        assert L.decode(z) == bytes([v])


def test_corrupt_containers_rejected():
    z = bytearray(L.encode(bytes(5000) + b"\x01" * 10))
    with pytest.raises(L.LosslessError):
        L.decode(bytes(z[:-1]))
    z2 = bytearray(z)
    z2[0] ^= 1
    with pytest.raises(L.LosslessError):
        L.decode(bytes(z2))
    z3 = bytearray(z)
    z3[8] ^= 1  # the byte count no longer matches the tokens
    with pytest.raises((L.LosslessError, O.OracleError)):
        L.decode(bytes(z3))


@pytest.mark.parametrize("eb", [1e-2, 1e-3])
def test_real_streams(eb):
    x = fields.lognormal_field((64, 64, 64))
    s = O.compress(x, make_cfg(x.shape, eb=eb, kind="nak"))
    z = L.encode(s)
    assert L.decode(z) == s
    assert L.parse(z)["mode"] == 1
    # the one-bit code of the exactly predicted points leaves zero runs to remove
    assert len(z) < len(s) * (0.6 if eb == 1e-2 else 0.98)
