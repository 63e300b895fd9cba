"""Continuous-batching request server over the library's batch entry points.

Requests (compress a device field, optionally auto-tuned first; decompress a
device stream) arrive over time.  The server keeps a FIFO of waiting requests
and a set of slots; each slot owns one HIP stream (default priority), one
library context and one worker thread.  Whenever a slot is free, the
dispatcher admits the longest FIFO prefix of waiting requests of the head's
kind whose device bytes fit in the free HBM budget (at most `max_batch` of
them) and hands them to that slot as one batch (hpez_tune_batch +
hpez_compress_batch, or hpez_decompress_batch).  Requests that arrive while
batches run join later batches as slots and memory free up, and the batches
of different slots overlap on the device.  Fields, streams and results stay on
the device.

Admission counts, per request, the library's workspace for the call
(hpez_footprint, plus the tuner's when tuning) and the output buffer.  A slot
context keeps its workspace between batches up to `keep_bytes` and trims it
above; that much per slot is reserved from the budget when the server starts.
A completed request's result stays on the device and stays charged against
the budget (its own size: compressed streams are copied out of their
worst-case buffers) until the caller calls `Server.release(r)`; the rest of
its admitted bytes return on completion.  A request larger than the whole
budget, or one the library rejects, completes with its error code; the others
are unaffected.

Every request's result is the same as the plain call's on the same input: the
batch entry points take the same steps per field as the plain ones (checked in
the GPU tests)."""
from __future__ import annotations

import math
import queue
import threading
import time
from collections import deque
from dataclasses import dataclass

from . import binding


@dataclass
class Request:
    rid: int
    op: str                      # "compress" or "decompress"
    arrival: float               # seconds after the start of the run
    data: object                 # device tensor: the field, or the stream
    cfg: dict | None = None      # compress: the configuration (the base one when tuning)
    tune: bool = False           # compress: auto-tune first (Sec. 6)
    tune_opts: dict | None = None
    # filled in by the server
    result: object = None
    config: dict | None = None   # the configuration used (tuned or given)
    error: int = 0
    admitted: float = math.nan
    done: float = math.nan
    slot: int = -1
    batch_size: int = 0
    mem: int = 0

    @property
    def nbytes(self) -> int:
        """Uncompressed bytes of the request (its field, or its output)."""
        return self.in_bytes if self.op == "compress" else self.out_bytes

    in_bytes: int = 0            # compress: bytes of the field (set at admission)
    out_bytes: int = 0           # decompress: bytes of the reconstruction
    out_shape: tuple = ()        # decompress: shape and dtype of the field, when known
    out_dtype: object = None
    ready: object = None         # optional device event after which `data` is complete


def _dtype_name(t) -> str:
    return "f64" if t.element_size() == 8 else "f32"


class LibraryBackend:
    """Runs batches through the library: per slot one HIP stream (default
    priority) and one context."""

    def __init__(self, device: int = 0, keep_bytes: int = 512 << 20):
        import torch
        self.torch = torch
        self.device = device
        self.keep = int(keep_bytes)

    def make_slot(self, i: int) -> dict:
        return dict(id=i, stream=self.torch.cuda.Stream(device=self.device),
                    ctx=binding.Context(self.device))

    def reserved_bytes(self, slots: int) -> int:
        """Device bytes held outside any request: each slot's kept workspace."""
        return slots * self.keep

    def result_bytes(self, r) -> int:
        """Device bytes a completed request's result holds."""
        if r.result is None:
            return 0
        return int(r.result.numel() * r.result.element_size())

    def close_slot(self, slot: dict):
        slot["ctx"].close()

    def prepare(self, r: Request):
        """Device bytes the request needs while it runs."""
        torch = self.torch
        if r.op == "compress":
            x = r.data
            dims = tuple(x.shape) if x.dim() else (1,)
            cfg = dict(r.cfg)
            cfg["dims"] = dims
            dt = _dtype_name(x)
            need = binding.footprint(dims, dt, cfg, "compress")
            if r.tune:
                need = max(need, binding.footprint(dims, dt, cfg, "tune"))
            need += binding.compress_bound(dims, dt, cfg)
            r.mem = need
            r.in_bytes = x.numel() * x.element_size()
        else:
            if not r.out_shape:
                # a stream of unknown origin: read its header
                s = r.data
                hdr = s[:512].cpu().numpy().tobytes()
                info = binding.inspect(hdr + b"\0" * max(0, 512 - len(hdr)))
                r.out_shape = tuple(info["dims"])
                r.out_dtype = torch.float64 if info["dtype"] == "f64" else torch.float32
            esz = 8 if r.out_dtype == torch.float64 else 4
            npts = 1
            for v in r.out_shape:
                npts *= int(v)
            r.out_bytes = npts * esz
            # the producing configuration when known, else the block-wise upper bound
            cfg = r.cfg or dict(eb=1e-3, eb_mode="rel", anchor_log2=6, block_log2=5,
                                levels=[dict(kind=0)])
            r.mem = r.out_bytes + binding.footprint(tuple(r.out_shape),
                                                    "f64" if esz == 8 else "f32", cfg,
                                                    "decompress")

    def run(self, batch, slot):
        torch = self.torch
        for r in batch:
            if r.ready is not None:
                slot["stream"].wait_event(r.ready)
        with torch.cuda.stream(slot["stream"]):
            if batch[0].op == "compress":
                self._compress(batch, slot)
            else:
                self._decompress(batch, slot)
        if slot["ctx"].workspace() > self.keep:
            slot["ctx"].trim(self.keep)

    def _compress(self, batch, slot):
        torch = self.torch
        st, cx = slot["stream"], slot["ctx"]
        cfgs = [dict(r.cfg, dims=tuple(r.data.shape)) for r in batch]
        tuned = [i for i, r in enumerate(batch) if r.tune]
        if tuned:
            try:
                res = binding.tune_batch([batch[i].data for i in tuned], [cfgs[i] for i in tuned],
                                         [batch[i].tune_opts for i in tuned], stream=st, context=cx)
                for i, c in zip(tuned, res):
                    cfgs[i] = c
            except binding.HpezError:
                # one field failed: tune the rest alone so only it fails
                for i in tuned:
                    try:
                        cfgs[i] = binding.tune(batch[i].data, cfgs[i], batch[i].tune_opts,
                                               stream=st, context=cx)
                    except binding.HpezError as e:
                        batch[i].error = e.code
        live = [i for i, r in enumerate(batch) if not r.error]
        if not live:
            return
        outs = []
        for i in live:
            x = batch[i].data
            cap = binding.compress_bound(tuple(x.shape), _dtype_name(x), cfgs[i])
            outs.append(torch.empty(cap, dtype=torch.uint8, device=x.device))
        sizes = [0] * len(live)
        try:
            binding.compress_batch([batch[i].data for i in live], [cfgs[i] for i in live],
                                   stream=st, outs=outs, context=cx, sizes_out=sizes)
        except binding.HpezError as e:
            if all(sz == 0 for sz in sizes):
                for i in live:
                    batch[i].error = e.code
                return
        for k, i in enumerate(live):
            r = batch[i]
            r.config = cfgs[i]
            if sizes[k]:
                # a right-sized copy: the worst-case buffer is freed here
                r.result = outs[k][: sizes[k]].clone()
            else:
                r.error = r.error or -1

    def _decompress(self, batch, slot):
        torch = self.torch
        st, cx = slot["stream"], slot["ctx"]
        outs = [torch.empty(r.out_shape, dtype=r.out_dtype, device=r.data.device) for r in batch]
        rcs = [0] * len(batch)
        try:
            binding.decompress_batch([r.data for r in batch], stream=st, outs=outs, context=cx,
                                     rcs_out=rcs)
        except binding.HpezError as e:
            if not any(rcs):
                for r in batch:
                    r.error = e.code
                return
        for r, o, rc in zip(batch, outs, rcs):
            if rc:
                r.error = rc
            else:
                r.result = o


class Server:
    def __init__(self, device: int = 0, slots: int = 4, hbm_budget: int = 64 << 30,
                 max_batch: int = 16, keep_bytes: int = 512 << 20, backend=None):
        self.backend = backend if backend is not None else LibraryBackend(device, keep_bytes)
        self.budget = int(hbm_budget)
        reserve = getattr(self.backend, "reserved_bytes", None)
        self.reserved = int(reserve(slots)) if reserve else 0
        if self.reserved > self.budget:
            raise ValueError("the slots' kept workspace exceeds the HBM budget")
        self._used = self.reserved  # reserved + admitted work + held results
        self._held = {}  # rid -> result bytes still charged
        self.max_batch = int(max_batch)
        self.slots = []
        for i in range(slots):
            sl = self.backend.make_slot(i)
            sl.update(inbox=queue.Queue(), thread=None)
            self.slots.append(sl)
        self._done = queue.Queue()
        self._t0 = time.perf_counter()

    # -- slot workers -----------------------------------------------------------
    def _worker(self, slot):
        while True:
            item = slot["inbox"].get()
            if item is None:
                return
            batch, mem = item
            t0 = self._t0
            for r in batch:
                r.admitted = time.perf_counter() - t0
                r.slot = slot["id"]
                r.batch_size = len(batch)
            try:
                self.backend.run(batch, slot)
            except Exception as e:  # a device error: every request of the batch fails
                for r in batch:
                    if not r.error and r.result is None:
                        r.error = getattr(e, "code", -3)
            t = time.perf_counter() - t0
            for r in batch:
                r.done = t
            self._done.put((slot, mem, batch))

    def _result_bytes(self, r) -> int:
        f = getattr(self.backend, "result_bytes", None)
        return int(f(r)) if f else 0

    def _complete(self, mem, batch):
        """Return a finished batch's admitted bytes except its results' (which
        stay charged until release)."""
        held = 0
        for r in batch:
            b = self._result_bytes(r) if not r.error else 0
            if b:
                self._held[r.rid] = b
                held += b
        self._used -= mem - held

    def release(self, r):
        """The caller no longer keeps r's result on the device: its bytes
        return to the budget."""
        self._used -= self._held.pop(r.rid, 0)

    @property
    def charged(self) -> int:
        """Bytes charged now: reserved slot workspace, admitted work, held results."""
        return self._used

    # -- dispatcher -------------------------------------------------------------
    def run(self, requests, on_arrival=None, on_done=None):
        """Serve `requests` (arrival times relative to the start).  on_arrival(r),
        if given, is called when r arrives (before it is queued): a producer hook
        that may create r.data.  on_done(r) is called on the dispatcher thread
        when r has completed.  Returns when every request has completed."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        n = len(reqs)
        pending = deque()
        free = deque(self.slots)
        nxt = 0
        finished = 0
        self._t0 = time.perf_counter()
        for s in self.slots:
            s["thread"] = threading.Thread(target=self._worker, args=(s,), daemon=True)
            s["thread"].start()
        try:
            while finished < n:
                now = time.perf_counter() - self._t0
                while nxt < n and reqs[nxt].arrival <= now:
                    r = reqs[nxt]
                    nxt += 1
                    if on_arrival is not None:
                        on_arrival(r)
                    self.backend.prepare(r)
                    if r.mem > self.budget - self.reserved:
                        r.error = -2  # larger than the whole budget
                        r.admitted = r.done = time.perf_counter() - self._t0
                        finished += 1
                        if on_done is not None:
                            on_done(r)
                    else:
                        pending.append(r)
                # completions
                while True:
                    try:
                        slot, mem, batch = self._done.get_nowait()
                    except queue.Empty:
                        break
                    free.append(slot)
                    self._complete(mem, batch)
                    finished += len(batch)
                    if on_done is not None:
                        for r in batch:
                            on_done(r)
                # admission: FIFO prefix of the head's kind that fits
                while pending and free:
                    op = pending[0].op
                    take, mem = [], 0
                    for r in pending:
                        if r.op != op:
                            continue
                        if self._used + mem + r.mem > self.budget or len(take) == self.max_batch:
                            break
                        take.append(r)
                        mem += r.mem
                    if not take:
                        if len(free) == len(self.slots):
                            # nothing runs, yet the head does not fit: results the
                            # caller still holds fill the budget; it fails (-2)
                            # rather than waiting for a release that may not come
                            r = pending.popleft()
                            r.error = -2
                            r.admitted = r.done = time.perf_counter() - self._t0
                            finished += 1
                            if on_done is not None:
                                on_done(r)
                            continue
                        break
                    for r in take:
                        pending.remove(r)
                    self._used += mem
                    free.popleft()["inbox"].put((take, mem))
                    # the slot object moves with the batch; it comes back on completion
                if finished >= n:
                    break
                # wait for a completion or the next arrival
                wait = None
                if nxt < n:
                    wait = max(0.0, reqs[nxt].arrival - (time.perf_counter() - self._t0))
                try:
                    slot, mem, batch = self._done.get(timeout=wait)
                    free.append(slot)
                    self._complete(mem, batch)
                    finished += len(batch)
                    if on_done is not None:
                        for r in batch:
                            on_done(r)
                except queue.Empty:
                    pass
        finally:
            for s in self.slots:
                s["inbox"].put(None)
            for s in self.slots:
                if s["thread"] is not None:
                    s["thread"].join()
                    s["thread"] = None
        return summarize(reqs)

    def close(self):
        for s in self.slots:
            self.backend.close_slot(s)


def _pct(v, q):
    if not v:
        return None
    v = sorted(v)
    k = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[k]


def summarize(reqs) -> dict:
    """p50/p99 latency (arrival to completion) and aggregate GB/s (uncompressed
    bytes of the completed requests over first arrival to last completion)."""
    ok = [r for r in reqs if not r.error]
    lat = [(r.done - r.arrival) * 1e3 for r in ok]
    out = dict(requests=len(reqs), completed=len(ok), failed=len(reqs) - len(ok))
    if ok:
        span = max(r.done for r in ok) - min(r.arrival for r in reqs)
        tot = sum(r.nbytes for r in ok)
        out.update(p50_ms=round(_pct(lat, 50), 3), p99_ms=round(_pct(lat, 99), 3),
                   mean_ms=round(sum(lat) / len(lat), 3), span_s=round(span, 4),
                   bytes=tot, GBps=round(tot / span / 1e9, 3) if span > 0 else None,
                   mean_batch=round(sum(r.batch_size for r in ok) / len(ok), 2))
        for op in ("compress", "decompress"):
            lo = [(r.done - r.arrival) * 1e3 for r in ok if r.op == op]
            if lo:
                out[op] = dict(n=len(lo), p50_ms=round(_pct(lo, 50), 3),
                               p99_ms=round(_pct(lo, 99), 3))
    return out
