"""ctypes binding of the CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this module.  The product library never does.

Configurations are passed as plain dicts (see ``tests/cfgs.py``) and are
converted here into the oracle's own parameter block.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
SOURCES = ["hpez_oracle.c", "oracle_core.inc", "oracle_huffman.inc", "oracle_stream.inc",
           "oracle_tune.inc"]

ORC_OK, ORC_EINVAL, ORC_ENOMEM, ORC_ECORRUPT, ORC_ENOSPC, ORC_EUNSUPPORTED, ORC_ESCHEDULE = (
    0, -1, -2, -4, -5, -6, -7)

# dtype codes; integer fields run the method in float64 on their values, with
# reconstructions rounded to integers, and are returned in their own type
DTYPES = {"f32": 0, "f64": 1, "u8": 2, "u16": 3, "i16": 4, "i32": 5}
INT_NP = {"u8": np.uint8, "u16": np.uint16, "i16": np.int16, "i32": np.int32}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: scalar C11, no FP contraction, no fast-math."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall",
               "-fPIC", "-shared", "-o", LIB_PATH + ".tmp", os.path.join(HERE, "hpez_oracle.c"),
               "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _stale() -> bool:
    t = os.path.getmtime(LIB_PATH)
    return any(os.path.getmtime(os.path.join(HERE, f)) > t for f in SOURCES)


class Interp(C.Structure):
    _fields_ = [("kind", C.c_uint8), ("md", C.c_uint8), ("same_level", C.c_uint8),
                ("order", C.c_uint8 * 4), ("pad", C.c_uint8)]


class Params(C.Structure):
    _fields_ = [("dtype", C.c_uint8), ("ndims", C.c_uint8), ("eb_mode", C.c_uint8),
                ("predictor", C.c_uint8), ("anchor_log2", C.c_uint8), ("block_log2", C.c_uint8),
                ("frozen_dim", C.c_int8), ("pad0", C.c_uint8), ("radius", C.c_uint32),
                ("chunk", C.c_uint32), ("dims", C.c_uint64 * 4), ("eb", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("md_w", (C.c_double * 4) * 3),
                ("level", Interp * 16), ("cand", Interp * 16), ("n_cand", C.c_uint32),
                ("pad1", C.c_uint32), ("block_cfg", C.c_void_p)]


class TuneOpts(C.Structure):
    _fields_ = [("global_rate", C.c_double), ("sub_rate", C.c_double),
                ("lorenzo_coef", C.c_double), ("block_log2", C.c_uint8),
                ("allow_freeze", C.c_uint8), ("allow_lorenzo", C.c_uint8),
                ("block_wise", C.c_uint8), ("anchor_log2", C.c_uint8), ("tune_ab", C.c_uint8),
                ("pad", C.c_uint8 * 2)]


class TuneReport(C.Structure):
    _fields_ = [("sigma2", (C.c_double * 4) * 3), ("count", C.c_int64),
                ("freeze_candidate", C.c_int), ("global_score", ((C.c_uint64 * 16) * 11) * 2),
                ("H", C.c_double * 2), ("H_lorenzo", C.c_double), ("frozen", C.c_int),
                ("lorenzo", C.c_int), ("ab_alpha", C.c_double * 17), ("ab_beta", C.c_double * 17),
                ("ab_score", C.c_double * 17), ("ab_sq", C.c_uint64 * 17),
                ("ab_rate", C.c_double * 17), ("ab_choice", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or _stale():
            build()
        L = C.CDLL(LIB_PATH)
        vp, u64, i64 = C.c_void_p, C.c_uint64, C.c_int64
        P = C.POINTER
        L.orc_compress.argtypes = [vp, P(Params), vp, u64, P(u64)]
        L.orc_decompress.argtypes = [vp, u64, vp, u64]
        L.orc_compress_bound.argtypes = [P(Params)]
        L.orc_compress_bound.restype = u64
        L.orc_interp_codes.argtypes = [vp, P(Params), C.c_double, vp, vp, vp, P(i64), vp, P(i64)]
        L.orc_lorenzo_codes.argtypes = [vp, P(Params), C.c_double, vp, vp, P(i64), vp, vp,
                                        P(i64), vp]
        L.orc_error_bound.argtypes = [vp, P(Params), P(C.c_double), P(C.c_int)]
        L.orc_stream_codes.argtypes = [vp, u64, vp]
        L.orc_inspect.argtypes = [vp, u64, P(u64), P(C.c_int), P(C.c_int), P(u64)]
        L.orc_huff_lengths.argtypes = [vp, C.c_uint32, vp]
        L.orc_huff_canonical.argtypes = [vp, C.c_uint32, vp]
        L.orc_huff_encode.argtypes = [vp, u64, vp, vp, C.c_uint32, vp, vp]
        L.orc_huff_encode.restype = u64
        L.orc_huff_decode.argtypes = [vp, u64, vp, C.c_uint32, C.c_uint32, vp, u64, vp]
        L.orc_stats.argtypes = [vp, P(Params), C.c_double, vp, P(i64)]
        L.orc_tune.argtypes = [vp, P(Params), P(TuneOpts), P(Params), vp, P(TuneReport)]
        L.orc_candidates.argtypes = [C.c_int, vp]
        L.orc_entropy_bits.argtypes = [vp, C.c_uint32]
        L.orc_entropy_bits.restype = C.c_double
        L.orc_stream_order.argtypes = [P(u64), C.c_int, vp]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def params_from_cfg(cfg: dict, keep=None) -> Params:
    """Neutral config dict -> oracle parameter block.  ``keep`` collects arrays
    whose memory the block points into."""
    p = Params()
    p.dtype = DTYPES[cfg["dtype"]]
    dims = list(cfg["dims"])
    p.ndims = len(dims)
    for d in range(4):
        p.dims[d] = dims[d] if d < len(dims) else 1
    p.eb_mode = {"abs": 0, "rel": 1}[cfg["eb_mode"]]
    p.predictor = {"interp": 0, "lorenzo": 1}[cfg.get("predictor", "interp")]
    p.anchor_log2 = cfg["anchor_log2"]
    p.block_log2 = cfg.get("block_log2", 0)
    p.frozen_dim = cfg.get("frozen_dim", -1)
    p.radius = cfg.get("radius", 32768)
    p.chunk = cfg.get("chunk", 1024)
    p.eb = cfg["eb"]
    p.alpha = cfg.get("alpha", 1.0)
    p.beta = cfg.get("beta", 1.0)
    mw = cfg.get("md_w", [[1.0] * 4] * 3)
    for k in range(3):
        for d in range(4):
            p.md_w[k][d] = mw[k][d]
    levels = cfg["levels"]
    for i in range(16):
        _fill_interp(p.level[i], levels[i] if i < len(levels) else levels[-1])
    cand = cfg.get("cand", [])
    p.n_cand = len(cand)
    for i in range(16):
        _fill_interp(p.cand[i], cand[i] if i < len(cand) else None)
    bc = cfg.get("block_cfg")
    if bc is not None:
        arr = np.ascontiguousarray(np.asarray(bc, dtype=np.uint8))
        if keep is not None:
            keep.append(arr)
        p.block_cfg = arr.ctypes.data
    return p


def _fill_interp(dst: Interp, src):
    if src is None:
        dst.kind = dst.md = dst.same_level = 0
        for j in range(4):
            dst.order[j] = j
        return
    dst.kind = src["kind"]
    dst.md = src.get("md", 0)
    dst.same_level = src.get("same_level", 0)
    order = list(src.get("order", (0, 1, 2, 3)))
    order = order + [j for j in range(4) if j not in order]
    for j in range(4):
        dst.order[j] = order[j]
    dst.pad = 0


def interp_from_struct(s: Interp) -> dict:
    return dict(kind=int(s.kind), md=int(s.md), same_level=int(s.same_level),
                order=tuple(int(v) for v in s.order))


def _np_dtype(cfg):
    """The type the method computes in (integers: float64)."""
    return np.float32 if cfg["dtype"] == "f32" else np.float64


def compress(x: np.ndarray, cfg: dict) -> bytes:
    keep = []
    p = params_from_cfg(cfg, keep)
    x = np.ascontiguousarray(x, dtype=_np_dtype(cfg))
    cap = lib().orc_compress_bound(C.byref(p))
    out = np.zeros(cap, dtype=np.uint8)
    n = C.c_uint64(0)
    rc = lib().orc_compress(_ptr(x), C.byref(p), _ptr(out), cap, C.byref(n))
    if rc:
        raise OracleError(rc, "compress")
    return out[: n.value].tobytes()


def inspect(stream: bytes):
    buf = np.frombuffer(stream, dtype=np.uint8)
    dims = (C.c_uint64 * 4)()
    dt, nd, tot = C.c_int(), C.c_int(), C.c_uint64()
    rc = lib().orc_inspect(_ptr(buf), len(stream), dims, C.byref(dt), C.byref(nd), C.byref(tot))
    if rc:
        raise OracleError(rc, "inspect")
    name = {v: k for k, v in DTYPES.items()}[dt.value]
    return dict(dims=tuple(int(dims[d]) for d in range(nd.value)), dtype=name,
                total=int(tot.value))


def decompress(stream: bytes) -> np.ndarray:
    """The reconstruction, in the field's own dtype (integer fields: the
    integer-valued float64 reconstruction clamped to the type's range)."""
    info = inspect(stream)
    dt = np.float32 if info["dtype"] == "f32" else np.float64
    out = np.zeros(int(np.prod(info["dims"])), dtype=dt)
    buf = np.frombuffer(stream, dtype=np.uint8)
    rc = lib().orc_decompress(_ptr(buf), len(stream), _ptr(out), out.nbytes)
    if rc:
        raise OracleError(rc, "decompress")
    it = INT_NP.get(info["dtype"])
    if it is not None:
        lim = np.iinfo(it)
        out = np.clip(out, lim.min, lim.max).astype(it)
    return out.reshape(info["dims"])


def stream_codes(stream: bytes) -> np.ndarray:
    info = inspect(stream)
    code = np.zeros(int(np.prod(info["dims"])), dtype=np.uint16)
    buf = np.frombuffer(stream, dtype=np.uint8)
    rc = lib().orc_stream_codes(_ptr(buf), len(stream), _ptr(code))
    if rc:
        raise OracleError(rc, "stream_codes")
    return code.reshape(info["dims"])


def error_bound(x: np.ndarray, cfg: dict):
    p = params_from_cfg(cfg)
    x = np.ascontiguousarray(x, dtype=_np_dtype(cfg))
    e, const = C.c_double(), C.c_int()
    rc = lib().orc_error_bound(_ptr(x), C.byref(p), C.byref(e), C.byref(const))
    if rc:
        raise OracleError(rc, "error_bound")
    return e.value, bool(const.value)


def interp_codes(x: np.ndarray, cfg: dict, e: float):
    """Codes, reconstruction, anchors and verbatim values of the interpolation
    predictor (before Huffman coding)."""
    keep = []
    p = params_from_cfg(cfg, keep)
    dt = _np_dtype(cfg)
    x = np.ascontiguousarray(x, dtype=dt)
    N = x.size
    code = np.zeros(N, dtype=np.uint16)
    W = np.zeros(N, dtype=dt)
    anchors = np.zeros(N, dtype=dt)
    unpred = np.zeros(N, dtype=dt)
    na, nu = C.c_int64(), C.c_int64()
    rc = lib().orc_interp_codes(_ptr(x), C.byref(p), e, _ptr(code), _ptr(W), _ptr(anchors),
                                C.byref(na), _ptr(unpred), C.byref(nu))
    if rc:
        raise OracleError(rc, "interp_codes")
    return dict(code=code.reshape(x.shape), W=W.reshape(x.shape), anchors=anchors[: na.value],
                unpred=unpred[: nu.value])


def lorenzo_codes(x: np.ndarray, cfg: dict, e: float):
    p = params_from_cfg(cfg)
    dt = _np_dtype(cfg)
    x = np.ascontiguousarray(x, dtype=dt)
    N = x.size
    code = np.zeros(N, dtype=np.uint16)
    outl = np.zeros(N, dtype=np.int64)
    pidx = np.zeros(N, dtype=np.uint64)
    pval = np.zeros(N, dtype=dt)
    W = np.zeros(N, dtype=dt)
    no, npch = C.c_int64(), C.c_int64()
    rc = lib().orc_lorenzo_codes(_ptr(x), C.byref(p), e, _ptr(code), _ptr(outl), C.byref(no),
                                 _ptr(pidx), _ptr(pval), C.byref(npch), _ptr(W))
    if rc:
        raise OracleError(rc, "lorenzo_codes")
    return dict(code=code.reshape(x.shape), outliers=outl[: no.value],
                patch_idx=pidx[: npch.value], patch_val=pval[: npch.value], W=W.reshape(x.shape))


def huff_lengths(counts: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(counts, dtype=np.uint64)
    out = np.zeros(c.size, dtype=np.uint8)
    rc = lib().orc_huff_lengths(_ptr(c), c.size, _ptr(out))
    if rc:
        raise OracleError(rc, "huff_lengths")
    return out


def huff_canonical(lens: np.ndarray) -> np.ndarray:
    l = np.ascontiguousarray(lens, dtype=np.uint8)
    out = np.zeros(l.size, dtype=np.uint32)
    lib().orc_huff_canonical(_ptr(l), l.size, _ptr(out))
    return out


def huff_encode(sym: np.ndarray, lens: np.ndarray, cw: np.ndarray, chunk: int):
    s = np.ascontiguousarray(sym, dtype=np.uint16)
    words = np.zeros(s.size + 1, dtype=np.uint32)
    nch = (s.size + chunk - 1) // chunk
    cb = np.zeros(max(nch, 1), dtype=np.uint32)
    bits = lib().orc_huff_encode(_ptr(s), s.size, _ptr(np.ascontiguousarray(lens, np.uint8)),
                                 _ptr(np.ascontiguousarray(cw, np.uint32)), chunk, _ptr(words),
                                 _ptr(cb))
    return words[: (bits + 31) // 32], int(bits), cb[:nch]


def huff_decode(words, bits, lens, chunk, chunk_bits, n):
    out = np.zeros(n, dtype=np.uint16)
    w = np.ascontiguousarray(words, dtype=np.uint32)
    if w.size == 0:
        w = np.zeros(1, np.uint32)
    l = np.ascontiguousarray(lens, dtype=np.uint8)
    cb = np.ascontiguousarray(chunk_bits, dtype=np.uint32)
    if cb.size == 0:
        cb = np.zeros(1, np.uint32)
    rc = lib().orc_huff_decode(_ptr(w), bits, _ptr(l), l.size, chunk, _ptr(cb), n, _ptr(out))
    if rc:
        raise OracleError(rc, "huff_decode")
    return out


def stats(x: np.ndarray, cfg: dict, e: float):
    p = params_from_cfg(cfg)
    x = np.ascontiguousarray(x, dtype=_np_dtype(cfg))
    sums = np.zeros((3, 4), dtype=np.uint64)
    cnt = C.c_int64()
    lib().orc_stats(_ptr(x), C.byref(p), e, _ptr(sums), C.byref(cnt))
    return sums, cnt.value


def candidates(ndims: int):
    arr = (Interp * 11)()
    lib().orc_candidates(ndims, C.cast(arr, C.c_void_p))
    return [interp_from_struct(arr[i]) for i in range(11)]


def tune(x: np.ndarray, cfg: dict, opts: dict):
    """Run the tuner; returns (tuned config dict, report dict)."""
    p = params_from_cfg(cfg)
    x = np.ascontiguousarray(x, dtype=_np_dtype(cfg))
    o = TuneOpts()
    o.global_rate = opts.get("global_rate", 0.01)
    o.sub_rate = opts.get("sub_rate", 0.04)
    o.lorenzo_coef = opts.get("lorenzo_coef", 1.0)
    o.block_log2 = opts.get("block_log2", 5)
    o.allow_freeze = opts.get("allow_freeze", 1)
    o.allow_lorenzo = opts.get("allow_lorenzo", 1)
    o.block_wise = opts.get("block_wise", 1)
    o.anchor_log2 = opts.get("anchor_log2", 0)
    o.tune_ab = opts.get("tune_ab", 0)
    outp = Params()
    B = 1 << o.block_log2
    nb = 1
    for n in cfg["dims"]:
        nb *= (n + B - 1) // B
    bc = np.zeros(max(nb, 1), dtype=np.uint8)
    rep = TuneReport()
    rc = lib().orc_tune(_ptr(x), C.byref(p), C.byref(o), C.byref(outp), _ptr(bc), C.byref(rep))
    if rc:
        raise OracleError(rc, "tune")
    out = dict(cfg)
    out["predictor"] = "lorenzo" if outp.predictor == 1 else "interp"
    out["anchor_log2"] = int(outp.anchor_log2)
    out["frozen_dim"] = int(outp.frozen_dim)
    out["block_log2"] = int(outp.block_log2)
    out["md_w"] = [[float(outp.md_w[k][d]) for d in range(4)] for k in range(3)]
    out["levels"] = [interp_from_struct(outp.level[i]) for i in range(16)]
    out["cand"] = [interp_from_struct(outp.cand[i]) for i in range(outp.n_cand)]
    out["block_cfg"] = bc[:nb].copy() if outp.block_log2 else None
    out["alpha"] = float(outp.alpha)
    out["beta"] = float(outp.beta)
    report = dict(sigma2=np.array([[rep.sigma2[k][d] for d in range(4)] for k in range(3)]),
                  count=rep.count, freeze_candidate=rep.freeze_candidate,
                  global_score=np.array([[[rep.global_score[f][c][l] for l in range(16)]
                                          for c in range(11)] for f in range(2)],
                                        dtype=np.uint64),
                  H=(rep.H[0], rep.H[1]), H_lorenzo=rep.H_lorenzo, frozen=rep.frozen,
                  lorenzo=rep.lorenzo, ab_alpha=list(rep.ab_alpha), ab_beta=list(rep.ab_beta),
                  ab_score=list(rep.ab_score), ab_sq=list(rep.ab_sq), ab_rate=list(rep.ab_rate),
                  ab_choice=rep.ab_choice)
    return out, report


def entropy_bits(hist) -> float:
    """The tuner's size estimate (Sec. 6.3 / 6.5): bits per symbol of a code
    histogram."""
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    return float(lib().orc_entropy_bits(_ptr(h), h.size))


def stream_order(dims) -> np.ndarray:
    """Row-major index of each code in stream order (brick order)."""
    dims = list(dims)
    d = (C.c_uint64 * 4)(*(dims + [1] * (4 - len(dims))))
    out = np.zeros(int(np.prod(dims)), dtype=np.int64)
    lib().orc_stream_order(d, len(dims), _ptr(out))
    return out
