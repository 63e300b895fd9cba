"""GPU parity of the lossless stage after Huffman coding (Sec. 4, step 5):
hpez_lossless_encode's container must be byte-identical to the oracle's, and
hpez_lossless_decode must give back the input exactly, on real compressed
streams at three bounds, incompressible bytes (stored), zero runs at and
around the 4096-byte token limit, all-zero input, empty and one-byte inputs,
an unaligned input; malformed containers are rejected."""
from __future__ import annotations

import numpy as np
import pytest

from cfgs import make_cfg
from oracle import oracle as O
from oracle import oracle_lossless as L
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


def roundtrip(torch, data: bytes, label: str, offset: int = 0):
    from paper_2311_12133_amd import binding
    print(f"[case] lossless {label} n={len(data)}", flush=True)
    buf = torch.zeros(len(data) + offset, dtype=torch.uint8, device="cuda")
    if data:
        buf[offset:] = torch.from_numpy(np.frombuffer(data, np.uint8).copy()).cuda()
    t = buf[offset:]
    z = binding.lossless_encode(t)
    torch.cuda.synchronize()
    got = z.cpu().numpy().tobytes()
    want = L.encode(data)
    assert got == want, f"{label}: container differs ({len(got)} vs {len(want)} bytes)"
    back = binding.lossless_decode(z)
    assert back.cpu().numpy().tobytes() == data, f"{label}: decoded bytes differ"
    return got


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4])
def test_real_streams(torch_cuda, eb):
    from paper_2311_12133_amd import binding
    x = fields.lognormal_field((128, 96, 80))
    xt = torch_cuda.from_numpy(x).cuda()
    s = binding.compress(xt, make_cfg(x.shape, eb=eb, kind="nak")).cpu().numpy().tobytes()
    z = roundtrip(torch_cuda, s, f"stream eb={eb}")
    if eb >= 1e-3:
        assert L.parse(z)["mode"] == 1 and len(z) < len(s)


def test_runs_around_token_limit(torch_cuda):
    R = L.RUN_MAX
    parts = [b"\x01", bytes(R), b"\x02", bytes(R + 1), b"\x03", bytes(R - 1), b"\x04",
             bytes(3 * R), b"\x05\x00\x06", bytes(2 * R + 17)]
    data = b"".join(parts) * 20
    z = roundtrip(torch_cuda, data, "token limit runs")
    assert L.parse(z)["mode"] == 1


def test_stored_and_tiny(torch_cuda):
    rng = np.random.default_rng(5)
    roundtrip(torch_cuda, rng.integers(1, 256, 100_003).astype(np.uint8).tobytes(), "random")
    roundtrip(torch_cuda, b"", "empty")
    roundtrip(torch_cuda, b"\x00", "one zero")
    roundtrip(torch_cuda, b"\x07", "one byte")
    roundtrip(torch_cuda, bytes(1_000_001), "all zero")


def test_unaligned_and_ragged(torch_cuda):
    rng = np.random.default_rng(6)
    b = np.where(rng.uniform(size=300_007) < 0.9, 0, rng.integers(1, 9, 300_007)).astype(np.uint8)
    roundtrip(torch_cuda, b.tobytes(), "unaligned", offset=3)
    roundtrip(torch_cuda, b[:4095].tobytes(), "one partial tile")


def test_corrupt_containers(torch_cuda):
    from paper_2311_12133_amd import binding
    torch = torch_cuda
    data = bytes(5000) + b"\x01" * 10 + bytes(300)
    z = bytearray(L.encode(data))
    for label, bad in (("magic", lambda v: v.__setitem__(0, v[0] ^ 1)),
                       ("byte count", lambda v: v.__setitem__(8, v[8] ^ 1)),
                       ("truncated", None)):
        v = bytearray(z)
        if bad is None:
            v = v[:-4]
        else:
            bad(v)
        print(f"[case] corrupt {label}", flush=True)
        t = torch.from_numpy(np.frombuffer(bytes(v), np.uint8).copy()).cuda()
        with pytest.raises(binding.HpezError) as ei:
            binding.lossless_decode(t)
        assert ei.value.code == -4
