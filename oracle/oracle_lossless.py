"""Oracle of the lossless stage after Huffman coding (Sec. 4, step 5) -- test
infrastructure only: the test suite, ``__graft_entry__.smoke()`` and the CPU
baseline of ``bench.py`` use it; the product library never does.

The paper passes the Huffman-coded stream through a general-purpose lossless
compressor.  What that stage finds in such a stream is mostly runs of zero
bytes: the most frequent quantization code gets the one-bit codeword 0, so
stretches of exactly predicted points become runs of zero bits.  This stage
codes those runs explicitly and entropy-codes the result:

1. Tokens.  The bytes are read left to right.  A nonzero byte v is the token
   v (1..255).  A maximal run of k zero bytes becomes floor(k / RUN_MAX)
   tokens 255 + RUN_MAX, then, if r = k mod RUN_MAX is not 0, the token
   255 + r.  So tokens lie in [1, 255 + RUN_MAX].
2. Huffman coding of the tokens with the same code construction, canonical
   codewords, chunking and bit order as the stream's own quantization codes
   (the oracle's Huffman functions).
3. A container: if the coded form is not smaller than the bytes themselves,
   the bytes are stored instead.

Container (little-endian):
    0 u32 magic 0x4C5A5048   4 u16 version 1   6 u16 mode (0 stored, 1 coded)
    8 u64 n (bytes of the input)   16 u64 n_tokens   24 u64 payload_bits
   32 u32 chunk   36 u32 sym_min   40 u32 sym_max   44 u32 RUN_MAX
   48 mode 0: the n input bytes.
      mode 1: code lengths u8[sym_max - sym_min + 1], padded to 8 bytes; chunk
      bit counts u16[ceil(n_tokens / chunk)], padded to 8; payload
      u32[ceil(payload_bits / 32)] (codewords most significant bit first).
"""
from __future__ import annotations

import struct

import numpy as np

from . import oracle as O

MAGIC = 0x4C5A5048
VERSION = 1
RUN_MAX = 4096
NSYM = 256 + RUN_MAX
CHUNK = 1024
HDR = 48


class LosslessError(ValueError):
    pass


def _align8(v: int) -> int:
    return (v + 7) & ~7


def tokens(b) -> np.ndarray:
    """The token sequence of the bytes b (step 1), by a plain walk over the
    zero runs between nonzero bytes."""
    b = np.frombuffer(bytes(b), dtype=np.uint8) if not isinstance(b, np.ndarray) else b
    nz = np.flatnonzero(b)
    out = []
    prev = -1
    for j in range(len(nz) + 1):
        nxt = int(nz[j]) if j < len(nz) else len(b)
        k = nxt - prev - 1  # zero bytes between the previous nonzero byte and this one
        full, r = divmod(k, RUN_MAX)
        out.extend([255 + RUN_MAX] * full)
        if r:
            out.append(255 + r)
        if j < len(nz):
            out.append(int(b[nxt]))
        prev = nxt
    return np.array(out, dtype=np.uint16)


def expand(tok: np.ndarray) -> bytes:
    """The bytes of a token sequence (the inverse of step 1)."""
    parts = []
    for t in tok.tolist():
        if t < 1 or t > 255 + RUN_MAX:
            raise LosslessError(f"token {t} out of range")
        parts.append(bytes([t]) if t <= 255 else bytes(t - 255))
    return b"".join(parts)


def layout(sym_min: int, sym_max: int, n_tokens: int, payload_bits: int) -> dict:
    off_len = HDR
    off_chunks = _align8(off_len + sym_max - sym_min + 1)
    nch = (n_tokens + CHUNK - 1) // CHUNK
    off_payload = _align8(off_chunks + 2 * nch)
    total = off_payload + 4 * ((payload_bits + 31) // 32)
    return dict(off_len=off_len, off_chunks=off_chunks, off_payload=off_payload, n_chunks=nch,
                total=total)


def _header(mode, n, n_tokens, bits, sym_min, sym_max) -> bytes:
    return struct.pack("<IHHQQQIIII", MAGIC, VERSION, mode, n, n_tokens, bits, CHUNK, sym_min,
                       sym_max, RUN_MAX)


def encode(data) -> bytes:
    """The container of `data` (bytes-like)."""
    raw = bytes(data)
    n = len(raw)
    stored = _header(0, n, 0, 0, 0, 0) + raw
    tok = tokens(np.frombuffer(raw, dtype=np.uint8))
    if tok.size == 0:
        return stored
    hist = np.bincount(tok, minlength=NSYM).astype(np.uint64)
    lens = O.huff_lengths(hist)
    cw = O.huff_canonical(lens)
    words, bits, cb = O.huff_encode(tok, lens, cw, CHUNK)
    used = np.flatnonzero(lens)
    smin, smax = int(used[0]), int(used[-1])
    L = layout(smin, smax, tok.size, bits)
    if L["total"] >= len(stored):
        return stored
    out = bytearray(L["total"])
    out[:HDR] = _header(1, n, int(tok.size), int(bits), smin, smax)
    out[L["off_len"]:L["off_len"] + smax - smin + 1] = lens[smin:smax + 1].tobytes()
    out[L["off_chunks"]:L["off_chunks"] + 2 * cb.size] = cb.astype(np.uint16).tobytes()
    w = np.asarray(words, dtype=np.uint32)
    out[L["off_payload"]:L["off_payload"] + 4 * w.size] = w.astype("<u4").tobytes()
    return bytes(out)


def parse(z: bytes) -> dict:
    if len(z) < HDR:
        raise LosslessError("short container")
    magic, ver, mode, n, ntok, bits, chunk, smin, smax, rmax = struct.unpack("<IHHQQQIIII",
                                                                             z[:HDR])
    if magic != MAGIC or ver != VERSION or mode not in (0, 1) or chunk != CHUNK or rmax != RUN_MAX:
        raise LosslessError("bad header")
    h = dict(mode=mode, n=n, n_tokens=ntok, payload_bits=bits, sym_min=smin, sym_max=smax)
    if mode == 0:
        h["total"] = HDR + n
    else:
        if not (1 <= smin <= smax < NSYM) or ntok == 0:
            raise LosslessError("bad symbol range")
        h.update(layout(smin, smax, ntok, bits))
    if len(z) != h["total"]:
        raise LosslessError("size mismatch")
    return h


def decode(z: bytes) -> bytes:
    """The bytes a container holds."""
    z = bytes(z)
    h = parse(z)
    if h["mode"] == 0:
        return z[HDR:]
    lens = np.zeros(NSYM, dtype=np.uint8)
    lens[h["sym_min"]:h["sym_max"] + 1] = np.frombuffer(
        z[h["off_len"]:h["off_len"] + h["sym_max"] - h["sym_min"] + 1], dtype=np.uint8)
    cb = np.frombuffer(z[h["off_chunks"]:h["off_chunks"] + 2 * h["n_chunks"]], dtype="<u2")
    nw = (h["payload_bits"] + 31) // 32
    words = np.frombuffer(z[h["off_payload"]:h["off_payload"] + 4 * nw], dtype="<u4")
    tok = O.huff_decode(words, h["payload_bits"], lens, CHUNK, cb.astype(np.uint32),
                        h["n_tokens"])
    out = expand(tok)
    if len(out) != h["n"]:
        raise LosslessError("length mismatch")
    return out
