"""ctypes binding of libhpez.so: argument marshalling only.

Every step of compression, decompression and tuning runs in the library's HIP
kernels; this module converts Python configuration dicts into the C structs of
``include/hpez.h``, passes torch device pointers and the current HIP stream,
and turns error codes into exceptions.  There is no fallback: if the library
is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import struct
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhpez.so")

HPEZ_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ECORRUPT", -5: "ENOSPC",
          -6: "EUNSUPPORTED"}


class HpezError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str = ""):
        super().__init__(f"{what}: {ERRORS.get(code, code)} ({msg})")
        self.code = code


class Interp(C.Structure):
    _fields_ = [("kind", C.c_uint8), ("md", C.c_uint8), ("same_level", C.c_uint8),
                ("order", C.c_uint8 * 4), ("pad", C.c_uint8)]


class FieldDesc(C.Structure):
    _fields_ = [("dtype", C.c_uint8), ("ndims", C.c_uint8), ("eb_mode", C.c_uint8),
                ("pad", C.c_uint8 * 5), ("dims", C.c_uint64 * 4), ("eb", C.c_double)]


class Config(C.Structure):
    _fields_ = [("predictor", C.c_uint8), ("anchor_log2", C.c_uint8), ("block_log2", C.c_uint8),
                ("frozen_dim", C.c_int8), ("radius", C.c_uint32), ("chunk", C.c_uint32),
                ("n_cand", C.c_uint32), ("alpha", C.c_double), ("beta", C.c_double),
                ("md_w", (C.c_double * 4) * 3), ("level", Interp * 16), ("cand", Interp * 16),
                ("block_cfg", C.c_void_p)]


class TuneOpts(C.Structure):
    _fields_ = [("global_rate", C.c_double), ("sub_rate", C.c_double),
                ("lorenzo_coef", C.c_double), ("block_log2", C.c_uint8),
                ("allow_freeze", C.c_uint8), ("allow_lorenzo", C.c_uint8),
                ("block_wise", C.c_uint8), ("anchor_log2", C.c_uint8), ("tune_ab", C.c_uint8),
                ("pad", C.c_uint8 * 2)]


class Quality(C.Structure):
    _fields_ = [("n", C.c_uint64), ("n_windows", C.c_uint64), ("value_range", C.c_double),
                ("max_abs_err", C.c_double), ("mse", C.c_double), ("psnr", C.c_double),
                ("ssim", C.c_double)]


class FitOpts(C.Structure):
    _fields_ = [("metric", C.c_int32), ("steps_per_octave", C.c_uint32), ("target", C.c_double),
                ("max_iter", C.c_uint32), ("ssim_window", C.c_uint32)]


class FitResult(C.Structure):
    _fields_ = [("e", C.c_double), ("e_hi", C.c_double), ("quality", Quality),
                ("bytes", C.c_uint64), ("iterations", C.c_uint32), ("pad", C.c_uint32)]


class TileChoice(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("size_class", C.c_int32),
                ("value", C.c_uint32), ("ms_before", C.c_double), ("ms_best", C.c_double)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_uint64), ("bytes", C.c_uint64),
                ("total_ms", C.c_double)]


EXPORTS = ["hpez_strerror", "hpez_ctx_create", "hpez_ctx_destroy", "hpez_config_default",
           "hpez_compress_bound", "hpez_compress", "hpez_inspect", "hpez_decompress",
           "hpez_tune", "hpez_footprint", "hpez_profile_enable", "hpez_profile_read",
           "hpez_compress_batch", "hpez_decompress_batch", "hpez_tune_batch",
           "hpez_ctx_trim", "hpez_ctx_set_limit", "hpez_ctx_workspace", "hpez_decompress_noalloc",
           "hpez_quality_eval", "hpez_fit_eb", "hpez_autotune", "hpez_decompress_plan",
           "hpez_plan_launch", "hpez_plan_status", "hpez_plan_destroy", "hpez_lossless_bound",
           "hpez_lossless_encode", "hpez_lossless_decode", "hpez_profile_only"]

_lib = None
_lock = threading.Lock()
_ctx = {}


def lib():
    """Load libhpez.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
            L = C.CDLL(LIB_PATH)
            vp, u64, P = C.c_void_p, C.c_uint64, C.POINTER
            L.hpez_strerror.argtypes = [C.c_int]
            L.hpez_strerror.restype = C.c_char_p
            L.hpez_ctx_create.argtypes = [P(vp), C.c_int]
            L.hpez_ctx_destroy.argtypes = [vp]
            L.hpez_ctx_destroy.restype = None
            L.hpez_config_default.argtypes = [P(FieldDesc), P(Config)]
            L.hpez_compress_bound.argtypes = [P(FieldDesc), P(Config), P(u64)]
            L.hpez_compress.argtypes = [vp, P(FieldDesc), vp, P(Config), vp, u64, P(u64), vp]
            L.hpez_inspect.argtypes = [vp, u64, P(FieldDesc), P(u64), P(u64)]
            L.hpez_decompress.argtypes = [vp, vp, u64, vp, u64, vp]
            L.hpez_decompress_noalloc.argtypes = [C.c_int, vp, u64, vp, u64, vp]
            L.hpez_tune.argtypes = [vp, P(FieldDesc), vp, P(TuneOpts), P(Config), vp, u64, vp]
            L.hpez_footprint.argtypes = [P(FieldDesc), P(Config), C.c_int, P(u64)]
            L.hpez_profile_enable.argtypes = [vp, C.c_int]
            L.hpez_profile_read.argtypes = [vp, P(KernelStat), C.c_int, P(C.c_int)]
            L.hpez_compress_batch.argtypes = [vp, C.c_int, P(FieldDesc), P(vp), P(Config), P(vp),
                                              P(u64), P(u64), vp]
            L.hpez_decompress_batch.argtypes = [vp, C.c_int, P(vp), P(u64), P(vp), P(u64),
                                                P(C.c_int), vp]
            L.hpez_tune_batch.argtypes = [vp, C.c_int, P(FieldDesc), P(vp), P(TuneOpts),
                                          P(Config), P(vp), P(u64), P(C.c_int), vp]
            L.hpez_ctx_trim.argtypes = [vp, u64]
            L.hpez_ctx_set_limit.argtypes = [vp, u64]
            L.hpez_ctx_workspace.argtypes = [vp, P(u64)]
            L.hpez_quality_eval.argtypes = [vp, P(FieldDesc), vp, vp, C.c_uint32, P(Quality), vp]
            L.hpez_fit_eb.argtypes = [vp, P(FieldDesc), vp, P(Config), P(FitOpts), P(FitResult),
                                      vp]
            L.hpez_autotune.argtypes = [vp, P(FieldDesc), vp, P(Config), P(TuneOpts),
                                        P(TileChoice), C.c_int, P(C.c_int), vp]
            L.hpez_decompress_plan.argtypes = [vp, C.c_int, P(vp), P(u64), P(vp), P(u64),
                                               P(C.c_int), vp, P(vp)]
            L.hpez_plan_launch.argtypes = [vp, vp]
            L.hpez_plan_status.argtypes = [vp, vp, P(C.c_int)]
            L.hpez_plan_destroy.argtypes = [vp]
            L.hpez_plan_destroy.restype = None
            L.hpez_profile_only.argtypes = [vp, C.c_char_p]
            L.hpez_lossless_bound.argtypes = [u64, P(u64)]
            L.hpez_lossless_encode.argtypes = [vp, vp, u64, vp, u64, P(u64), vp]
            L.hpez_lossless_decode.argtypes = [vp, vp, u64, vp, u64, P(u64), vp]
            _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != HPEZ_OK:
        raise HpezError(rc, what, lib().hpez_strerror(rc).decode())


def ctx(device: int):
    with _lock:
        c = _ctx.get(device)
    if c is None:
        p = C.c_void_p()
        _check(lib().hpez_ctx_create(C.byref(p), device), "hpez_ctx_create")
        with _lock:
            _ctx[device] = p
        c = p
    return c


class Context:
    """A library context of its own (workspace, pinned staging), for callers
    that drive several streams from several threads: one context per thread.
    The calls below use a shared per-device context unless given one."""

    def __init__(self, device: int = 0):
        self.device = device
        self.ptr = C.c_void_p()
        _check(lib().hpez_ctx_create(C.byref(self.ptr), device), "hpez_ctx_create")

    def trim(self, keep_bytes: int = 0):
        _check(lib().hpez_ctx_trim(self.ptr, int(keep_bytes)), "hpez_ctx_trim")

    def set_limit(self, max_workspace_bytes: int):
        _check(lib().hpez_ctx_set_limit(self.ptr, int(max_workspace_bytes)), "hpez_ctx_set_limit")

    def workspace(self) -> int:
        n = C.c_uint64()
        _check(lib().hpez_ctx_workspace(self.ptr, C.byref(n)), "hpez_ctx_workspace")
        return n.value

    def close(self):
        if self.ptr:
            lib().hpez_ctx_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cx(context, device: int):
    return context.ptr if context is not None else ctx(device)


def footprint(dims, dtype: str, cfg: dict, op: str) -> int:
    """Device bytes of the library's workspace for op ("compress",
    "decompress", "tune") on such a field (hpez_footprint)."""
    keep = []
    d = desc_from(dims, dtype, cfg.get("eb", 1e-3), cfg.get("eb_mode", "rel"))
    c = config_from(cfg, keep)
    n = C.c_uint64()
    _check(lib().hpez_footprint(C.byref(d), C.byref(c), {"compress": 0, "decompress": 1,
                                                         "tune": 2}[op], C.byref(n)),
           "hpez_footprint")
    return n.value


# ---------------------------------------------------------------------------
# config dict <-> structs

def desc_from(dims, dtype: str, eb: float, eb_mode: str) -> FieldDesc:
    d = FieldDesc()
    d.dtype = DTYPES[dtype]
    d.ndims = len(dims)
    for i in range(4):
        d.dims[i] = int(dims[i]) if i < len(dims) else 1
    d.eb_mode = {"abs": 0, "rel": 1}[eb_mode]
    d.eb = float(eb)
    return d


_NO_INTERP = bytes((0, 0, 0, 0, 1, 2, 3, 0))


def _interp_bytes(src) -> bytes:
    """The 8 bytes of an hpez_interp (kind, md, same_level, order[4], pad)."""
    if src is None:
        return _NO_INTERP
    order = src.get("order", (0, 1, 2, 3))
    if len(order) != 4:
        order = list(order)
        order = order + [j for j in range(4) if j not in order]
    try:  # integer-valued entries (the usual case): no conversions
        return bytes((src["kind"], src.get("md", 0), src.get("same_level", 0), order[0], order[1],
                      order[2], order[3], 0))
    except TypeError:
        return bytes((int(src["kind"]), int(src.get("md", 0)), int(src.get("same_level", 0)),
                      *(int(v) for v in order), 0))


def _fill_interp(dst: Interp, src):
    C.memmove(C.addressof(dst), _interp_bytes(src), 8)


_LEVEL_OFF = Config.level.offset
_CAND_OFF = Config.cand.offset
_MDW_OFF = Config.md_w.offset


def config_from(cfg: dict, keep: list) -> Config:
    c = Config()
    c.predictor = {"interp": 0, "lorenzo": 1}[cfg.get("predictor", "interp")]
    c.anchor_log2 = int(cfg["anchor_log2"])
    c.block_log2 = int(cfg.get("block_log2", 0))
    c.frozen_dim = int(cfg.get("frozen_dim", -1))
    c.radius = int(cfg.get("radius", 32768))
    c.chunk = int(cfg.get("chunk", 1024))
    c.alpha = float(cfg.get("alpha", 1.0))
    c.beta = float(cfg.get("beta", 1.0))
    mw = cfg.get("md_w")
    if mw is not None:
        C.memmove(C.addressof(c) + _MDW_OFF,
                  struct.pack("12d", *(float(mw[k][d]) for k in range(3) for d in range(4))), 96)
    else:
        C.memmove(C.addressof(c) + _MDW_OFF, struct.pack("12d", *([1.0] * 12)), 96)
    # the level and candidate tables are written as bytes (one copy each)
    levels = cfg["levels"]
    lv = [_interp_bytes(x) for x in levels[:16]]
    lv += [lv[-1]] * (16 - len(lv))
    C.memmove(C.addressof(c) + _LEVEL_OFF, b"".join(lv), 128)
    cand = cfg.get("cand", [])
    c.n_cand = len(cand)
    cb = [_interp_bytes(x) for x in cand[:16]]
    cb += [_NO_INTERP] * (16 - len(cb))
    C.memmove(C.addressof(c) + _CAND_OFF, b"".join(cb), 128)
    bc = cfg.get("block_cfg")
    if bc is not None:
        arr = np.ascontiguousarray(np.asarray(bc, dtype=np.uint8))
        keep.append(arr)
        c.block_cfg = arr.ctypes.data
    return c


def interp_dict(s: Interp) -> dict:
    b = bytes(s)
    return dict(kind=b[0], md=b[1], same_level=b[2], order=tuple(b[3:7]))


def _interp_dicts(c: Config, off: int, n: int) -> list:
    b = C.string_at(C.addressof(c) + off, 8 * n)
    return [dict(kind=b[8 * i], md=b[8 * i + 1], same_level=b[8 * i + 2],
                 order=tuple(b[8 * i + 3:8 * i + 7])) for i in range(n)]


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# field types (integer fields: the method runs in float64 on their values)
DTYPES = {"f32": 0, "f64": 1, "u8": 2, "u16": 3, "i16": 4, "i32": 5}
DTYPE_NAMES = {v: k for k, v in DTYPES.items()}


def _torch_dtype(name: str):
    torch = _torch()
    return {"f32": torch.float32, "f64": torch.float64, "u8": torch.uint8, "u16": torch.uint16,
            "i16": torch.int16, "i32": torch.int32}[name]


def _dtype_of(t) -> str:
    torch = _torch()
    for name in DTYPES:
        if t.dtype == _torch_dtype(name):
            return name
    raise TypeError("hpez compresses float32, float64, uint8, uint16, int16 or int32 tensors")


# ---------------------------------------------------------------------------
# public calls

def compress_bound(dims, dtype: str, cfg: dict) -> int:
    keep = []
    d = desc_from(dims, dtype, cfg.get("eb", 1e-3), cfg.get("eb_mode", "rel"))
    c = config_from(cfg, keep)
    n = C.c_uint64()
    _check(lib().hpez_compress_bound(C.byref(d), C.byref(c), C.byref(n)), "hpez_compress_bound")
    return n.value


def compress(x, cfg: dict, stream=None, out=None, context=None):
    """Compress a CUDA tensor (float32/float64, contiguous).  Returns a uint8 CUDA
    tensor holding the stream (a view of `out` when given)."""
    torch = _torch()
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous device tensor")
    dtype = _dtype_of(x)
    keep = []
    d = desc_from(tuple(x.shape) if x.dim() else (1,), dtype, cfg["eb"], cfg["eb_mode"])
    c = config_from(cfg, keep)
    cap = C.c_uint64()
    _check(lib().hpez_compress_bound(C.byref(d), C.byref(c), C.byref(cap)), "hpez_compress_bound")
    if out is None:
        out = torch.empty(cap.value, dtype=torch.uint8, device=x.device)
    n = C.c_uint64()
    rc = lib().hpez_compress(_cx(context, x.device.index or 0), C.byref(d), C.c_void_p(x.data_ptr()),
                             C.byref(c), C.c_void_p(out.data_ptr()), out.numel(), C.byref(n),
                             _stream_ptr(stream))
    _check(rc, "hpez_compress")
    return out[: n.value]


def inspect(header_bytes: bytes):
    d = FieldDesc()
    npts, tot = C.c_uint64(), C.c_uint64()
    buf = np.frombuffer(header_bytes, dtype=np.uint8)
    _check(lib().hpez_inspect(buf.ctypes.data_as(C.c_void_p), buf.size, C.byref(d), C.byref(npts),
                              C.byref(tot)), "hpez_inspect")
    return dict(dims=tuple(int(d.dims[i]) for i in range(d.ndims)),
                dtype=DTYPE_NAMES[d.dtype], points=npts.value, total=tot.value)


def decompress(stream_t, stream=None, out=None, context=None):
    """Decompress a uint8 CUDA tensor holding a stream; returns the field."""
    torch = _torch()
    if out is None:
        # the field's shape and dtype from the header (the library checks out's size)
        hdr = stream_t[:512].cpu().numpy().tobytes()
        info = inspect(hdr + b"\0" * max(0, 512 - len(hdr)))
        dt = _torch_dtype(info["dtype"])
        out = torch.empty(info["dims"], dtype=dt, device=stream_t.device)
    rc = lib().hpez_decompress(_cx(context, stream_t.device.index or 0),
                               C.c_void_p(stream_t.data_ptr()),
                               stream_t.numel(), C.c_void_p(out.data_ptr()),
                               out.numel() * out.element_size(), _stream_ptr(stream))
    _check(rc, "hpez_decompress")
    return out


def decompress_noalloc(stream_t, out, stream=None):
    """hpez_decompress_noalloc: decompress into the caller's `out` with the
    library's static per-GPU workspace (no allocation in the call)."""
    rc = lib().hpez_decompress_noalloc(stream_t.device.index or 0, C.c_void_p(stream_t.data_ptr()),
                                       stream_t.numel(), C.c_void_p(out.data_ptr()),
                                       out.numel() * out.element_size(), _stream_ptr(stream))
    _check(rc, "hpez_decompress_noalloc")
    return out


def _tune_opts(opts: dict | None) -> TuneOpts:
    opts = opts or {}
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
    return o


def _n_blocks(shape, block_log2: int) -> int:
    B = 1 << block_log2
    nb = 1
    for n in shape:
        nb *= (n + B - 1) // B
    return nb


def _tuned_dict(cfg: dict, c: Config, bc, nb: int) -> dict:
    res = dict(cfg)
    res["predictor"] = "lorenzo" if c.predictor == 1 else "interp"
    res["anchor_log2"] = int(c.anchor_log2)
    res["frozen_dim"] = int(c.frozen_dim)
    res["block_log2"] = int(c.block_log2)
    w = struct.unpack("12d", C.string_at(C.addressof(c) + _MDW_OFF, 96))
    res["md_w"] = [list(w[4 * k:4 * k + 4]) for k in range(3)]
    res["levels"] = _interp_dicts(c, _LEVEL_OFF, 16)
    res["cand"] = _interp_dicts(c, _CAND_OFF, c.n_cand)
    res["block_cfg"] = bc[:nb].copy() if c.block_log2 else None
    res["alpha"] = float(c.alpha)
    res["beta"] = float(c.beta)
    return res


def tune(x, cfg: dict, opts: dict | None = None, stream=None, context=None) -> dict:
    """Run the auto-tuner on a CUDA tensor; returns a complete config dict."""
    dtype = _dtype_of(x)
    keep = []
    d = desc_from(tuple(x.shape), dtype, cfg["eb"], cfg["eb_mode"])
    c = config_from(cfg, keep)
    o = _tune_opts(opts)
    nb = _n_blocks(x.shape, o.block_log2)
    bc = np.zeros(max(nb, 1), dtype=np.uint8)
    rc = lib().hpez_tune(_cx(context, x.device.index or 0), C.byref(d), C.c_void_p(x.data_ptr()),
                         C.byref(o), C.byref(c), bc.ctypes.data_as(C.c_void_p), bc.size,
                         _stream_ptr(stream))
    _check(rc, "hpez_tune")
    return _tuned_dict(cfg, c, bc, nb)


def tune_batch(xs, cfgs, opts=None, stream=None, context=None) -> list:
    """Tune many CUDA tensors in one call (trials of all fields in fused
    launches).  opts: one dict for all fields or a list of dicts."""
    n = len(xs)
    if n == 0:
        return []
    dev = xs[0].device.index or 0
    keep = []
    D = (FieldDesc * n)()
    Cs = (Config * n)()
    O = (TuneOpts * n)()
    ins = (C.c_void_p * n)()
    bcs, bptr, bcap = [], (C.c_void_p * n)(), (C.c_uint64 * n)()
    rcs = (C.c_int * n)()
    nbs = []
    for i, (x, cfg) in enumerate(zip(xs, cfgs)):
        if not x.is_cuda or not x.is_contiguous() or (x.device.index or 0) != dev:
            raise ValueError("fields must be contiguous tensors on one device")
        D[i] = desc_from(tuple(x.shape), _dtype_of(x), cfg["eb"], cfg["eb_mode"])
        Cs[i] = config_from(cfg, keep)
        O[i] = _tune_opts(opts[i] if isinstance(opts, (list, tuple)) else opts)
        ins[i] = x.data_ptr()
        nb = _n_blocks(x.shape, O[i].block_log2)
        nbs.append(nb)
        bc = np.zeros(max(nb, 1), dtype=np.uint8)
        bcs.append(bc)
        bptr[i] = bc.ctypes.data
        bcap[i] = bc.size
    rc = lib().hpez_tune_batch(_cx(context, dev), n, D, ins, O, Cs, bptr, bcap, rcs,
                               _stream_ptr(stream))
    _check(rc, "hpez_tune_batch")
    return [_tuned_dict(cfgs[i], Cs[i], bcs[i], nbs[i]) for i in range(n)]


def compress_batch(xs, cfgs, stream=None, outs=None, context=None, sizes_out=None) -> list:
    """Compress many CUDA tensors in one call; returns one uint8 CUDA tensor
    per field (views of `outs` when given), each byte-identical to compress()."""
    torch = _torch()
    n = len(xs)
    if n == 0:
        return []
    dev = xs[0].device.index or 0
    keep = []
    D = (FieldDesc * n)()
    Cs = (Config * n)()
    ins, optr = (C.c_void_p * n)(), (C.c_void_p * n)()
    caps, sizes = (C.c_uint64 * n)(), (C.c_uint64 * n)()
    bufs = []
    for i, (x, cfg) in enumerate(zip(xs, cfgs)):
        if not x.is_cuda or not x.is_contiguous() or (x.device.index or 0) != dev:
            raise ValueError("fields must be contiguous tensors on one device")
        D[i] = desc_from(tuple(x.shape) if x.dim() else (1,), _dtype_of(x), cfg["eb"],
                         cfg["eb_mode"])
        Cs[i] = config_from(cfg, keep)
        cap = C.c_uint64()
        _check(lib().hpez_compress_bound(C.byref(D[i]), C.byref(Cs[i]), C.byref(cap)),
               "hpez_compress_bound")
        o = outs[i] if outs is not None else torch.empty(cap.value, dtype=torch.uint8,
                                                          device=x.device)
        bufs.append(o)
        ins[i] = x.data_ptr()
        optr[i] = o.data_ptr()
        caps[i] = o.numel()
    rc = lib().hpez_compress_batch(_cx(context, dev), n, D, ins, Cs, optr, caps, sizes,
                                   _stream_ptr(stream))
    if sizes_out is not None:
        sizes_out[:] = [int(sizes[i]) for i in range(n)]
    _check(rc, "hpez_compress_batch")
    return [bufs[i][: sizes[i]] for i in range(n)]


def decompress_batch(streams, stream=None, outs=None, context=None, rcs_out=None) -> list:
    """Decompress many uint8 CUDA tensors (streams) in one call."""
    torch = _torch()
    n = len(streams)
    if n == 0:
        return []
    dev = streams[0].device.index or 0
    heads = None
    if outs is None:
        # every header in one device-to-host copy, for the output shapes
        heads = torch.stack([torch.nn.functional.pad(s[:512], (0, max(0, 512 - min(512, s.numel()))))
                             for s in streams]).cpu().numpy()
    ins, optr = (C.c_void_p * n)(), (C.c_void_p * n)()
    isz, caps = (C.c_uint64 * n)(), (C.c_uint64 * n)()
    rcs = (C.c_int * n)()
    res = []
    for i, s in enumerate(streams):
        if outs is not None:
            o = outs[i]
        else:
            info = inspect(heads[i].tobytes())
            dt = _torch_dtype(info["dtype"])
            o = torch.empty(info["dims"], dtype=dt, device=s.device)
        res.append(o)
        ins[i] = s.data_ptr()
        isz[i] = s.numel()
        optr[i] = o.data_ptr()
        caps[i] = o.numel() * o.element_size()
    rc = lib().hpez_decompress_batch(_cx(context, dev), n, ins, isz, optr, caps, rcs,
                                     _stream_ptr(stream))
    if rcs_out is not None:
        rcs_out[:] = [int(rcs[i]) for i in range(n)]
    _check(rc, "hpez_decompress_batch")
    return res


def lossless_encode(data, stream=None, context=None):
    """hpez_lossless_encode: the lossless-stage container (uint8 device tensor)
    of the bytes of the contiguous device tensor `data` (Sec. 4 step 5)."""
    torch = _torch()
    b = data.reshape(-1).view(torch.uint8)
    n = b.numel()
    cap = C.c_uint64()
    _check(lib().hpez_lossless_bound(n, C.byref(cap)), "hpez_lossless_bound")
    out = torch.empty(cap.value, dtype=torch.uint8, device=b.device)
    size = C.c_uint64()
    _check(lib().hpez_lossless_encode(_cx(context, b.device.index or 0),
                                      C.c_void_p(b.data_ptr() if n else 0), n,
                                      C.c_void_p(out.data_ptr()), cap.value, C.byref(size),
                                      _stream_ptr(stream)), "hpez_lossless_encode")
    return out[: size.value]


def lossless_decode(z, out=None, stream=None, context=None):
    """hpez_lossless_decode: the bytes (uint8 device tensor) a container holds."""
    torch = _torch()
    size = C.c_uint64()
    dev = z.device.index or 0
    if out is None:
        hdr = z[:48].cpu().numpy().tobytes()
        if len(hdr) < 48:
            raise HpezError(-4, "hpez_lossless_decode", "short container")
        n = struct.unpack_from("<Q", hdr, 8)[0]
        out = torch.empty(n, dtype=torch.uint8, device=z.device)
    _check(lib().hpez_lossless_decode(_cx(context, dev), C.c_void_p(z.data_ptr()), z.numel(),
                                      C.c_void_p(out.data_ptr() if out.numel() else 0),
                                      out.numel(), C.byref(size), _stream_ptr(stream)),
           "hpez_lossless_decode")
    return out[: size.value]


class DecompressPlan:
    """hpez_decompress_plan: the decompression of fixed device streams into
    fixed device outputs, run once (checked, outputs filled) and recorded as a
    HIP graph; launch() replays it on a stream with no host work, status()
    synchronises and returns the per-stream codes of the last replay.  The
    streams and outputs (kept referenced here) must not change meanwhile."""

    def __init__(self, streams, outs=None, stream=None, context=None):
        torch = _torch()
        n = len(streams)
        if n == 0:
            raise ValueError("a plan needs at least one stream")
        dev = streams[0].device.index or 0
        if outs is None:
            heads = torch.stack([torch.nn.functional.pad(s[:512], (0, max(0, 512 - min(512, s.numel()))))
                                 for s in streams]).cpu().numpy()
            outs = []
            for i, s in enumerate(streams):
                info = inspect(heads[i].tobytes())
                outs.append(torch.empty(info["dims"], dtype=_torch_dtype(info["dtype"]),
                                        device=s.device))
        self.streams, self.outs, self.n, self.device = list(streams), list(outs), n, dev
        ins, optr = (C.c_void_p * n)(), (C.c_void_p * n)()
        isz, caps = (C.c_uint64 * n)(), (C.c_uint64 * n)()
        rcs = (C.c_int * n)()
        for i, (s, o) in enumerate(zip(self.streams, self.outs)):
            ins[i], isz[i] = s.data_ptr(), s.numel()
            optr[i], caps[i] = o.data_ptr(), o.numel() * o.element_size()
        self.ptr = C.c_void_p()
        rc = lib().hpez_decompress_plan(_cx(context, dev), n, ins, isz, optr, caps, rcs,
                                        _stream_ptr(stream), C.byref(self.ptr))
        self.rcs = [int(rcs[i]) for i in range(n)]
        _check(rc, "hpez_decompress_plan")

    def launch(self, stream=None):
        _check(lib().hpez_plan_launch(self.ptr, _stream_ptr(stream)), "hpez_plan_launch")
        return self.outs

    def status(self, stream=None) -> list:
        rcs = (C.c_int * self.n)()
        lib().hpez_plan_status(self.ptr, _stream_ptr(stream), rcs)
        return [int(rcs[i]) for i in range(self.n)]

    def close(self):
        if self.ptr:
            lib().hpez_plan_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _quality_dict(q: Quality) -> dict:
    return dict(n=q.n, value_range=q.value_range, max_abs_err=q.max_abs_err, mse=q.mse,
                psnr=q.psnr, ssim=q.ssim, n_windows=q.n_windows)


def quality(x, xr, window: int = 8, stream=None, context=None) -> dict:
    """hpez_quality_eval: value range, max error, MSE, PSNR and windowed SSIM of
    the device reconstruction xr of the device field x (Sec. 3.1, Eq. 1)."""
    if not (x.is_cuda and xr.is_cuda and x.is_contiguous() and xr.is_contiguous()):
        raise ValueError("x and xr must be contiguous device tensors")
    if x.shape != xr.shape or x.dtype != xr.dtype:
        raise ValueError("x and xr differ in shape or dtype")
    d = desc_from(tuple(x.shape) if x.dim() else (1,), _dtype_of(x), 1.0, "abs")
    q = Quality()
    _check(lib().hpez_quality_eval(_cx(context, x.device.index or 0), C.byref(d),
                                   C.c_void_p(x.data_ptr()), C.c_void_p(xr.data_ptr()), window,
                                   C.byref(q), _stream_ptr(stream)), "hpez_quality_eval")
    return _quality_dict(q)


def fit_eb(x, cfg: dict, metric: str, target: float, steps_per_octave: int = 64,
           max_iter: int = 12, window: int = 8, stream=None, context=None) -> dict:
    """hpez_fit_eb: the largest bound e = L 2^(k / G) found whose compression of
    x under cfg reaches metric ("psnr" or "ssim") >= target.  Returns e, e_hi,
    the quality and stream size at e, and the number of compressions."""
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous device tensor")
    keep = []
    d = desc_from(tuple(x.shape) if x.dim() else (1,), _dtype_of(x), 1.0, "abs")
    c = config_from(cfg, keep)
    o = FitOpts()
    o.metric = {"psnr": 0, "ssim": 1}[metric]
    o.steps_per_octave = steps_per_octave
    o.target = target
    o.max_iter = max_iter
    o.ssim_window = window
    r = FitResult()
    _check(lib().hpez_fit_eb(_cx(context, x.device.index or 0), C.byref(d),
                             C.c_void_p(x.data_ptr()), C.byref(c), C.byref(o), C.byref(r),
                             _stream_ptr(stream)), "hpez_fit_eb")
    return dict(e=r.e, e_hi=r.e_hi, quality=_quality_dict(r.quality), bytes=r.bytes,
                iterations=r.iterations)


def autotune(x, cfg: dict, tune_opts: dict | None = None, stream=None, context=None) -> list:
    """hpez_autotune: measure launch shapes for this field's compress /
    decompress (and tune, with tune_opts) and cache the fastest in the
    context.  Returns the choices (kind "faces" or "trials", size class, shape,
    and the group times before and after)."""
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous device tensor")
    keep = []
    d = desc_from(tuple(x.shape) if x.dim() else (1,), _dtype_of(x), cfg["eb"], cfg["eb_mode"])
    c = config_from(cfg, keep)
    to = _tune_opts(tune_opts) if tune_opts is not None else None
    out = (TileChoice * 64)()
    n = C.c_int()
    _check(lib().hpez_autotune(_cx(context, x.device.index or 0), C.byref(d),
                               C.c_void_p(x.data_ptr()), C.byref(c),
                               C.byref(to) if to is not None else None, out, 64, C.byref(n),
                               _stream_ptr(stream)), "hpez_autotune")
    res = []
    for i in range(min(n.value, 64)):
        t = out[i]
        shape = (dict(lanes=t.value & 0xFFFF, points_per_lane=t.value >> 16) if t.kind == 0
                 else dict(lanes=t.value))
        res.append(dict(kind="faces" if t.kind == 0 else "trials", dtype_class=t.dtype,
                        size_class=t.size_class, shape=shape, ms_before=round(t.ms_before, 4),
                        ms_best=round(t.ms_best, 4)))
    return res


def profile_enable(device: int = 0, on: bool = True):
    """Start (clearing totals) or stop per-kernel event timing in the library."""
    _check(lib().hpez_profile_enable(ctx(device), int(on)), "hpez_profile_enable")


def profile_only(group: str | None, device: int = 0):
    """Record only one kernel group's spans while profiling (None: all)."""
    _check(lib().hpez_profile_only(ctx(device), group.encode() if group else None),
           "hpez_profile_only")


def profile_read(device: int = 0):
    """Per-kernel-group totals: {name: dict(launches, bytes, ms)}."""
    n = C.c_int()
    _check(lib().hpez_profile_read(ctx(device), None, 0, C.byref(n)), "hpez_profile_read")
    arr = (KernelStat * max(n.value, 1))()
    _check(lib().hpez_profile_read(ctx(device), arr, n.value, C.byref(n)), "hpez_profile_read")
    return {arr[i].name.decode(): dict(launches=int(arr[i].launches), bytes=int(arr[i].bytes),
                                       ms=float(arr[i].total_ms)) for i in range(n.value)}
