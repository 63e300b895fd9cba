"""Pure-Python brute-force twin of the oracle's interpolation schedule, for tiny
grids only (test infrastructure).

It restates the level-wise interpolation of Sec. 5.1 point by point, in
Python, with float32/float64 arithmetic done through numpy scalars so each
operation rounds exactly once.  Unlike the C oracle it

  * visits the points of each pass in a shuffled order (Sec. 5.4.1 says the
    in-pass traversal order changes speed, not results),
  * records how many times every point is predicted (each must be predicted
    exactly once) and refuses to read a point before it is reconstructed.

It is independent of the C oracle (written separately from the same reading)
and is used to cross-check it on tiny grids.
"""
from __future__ import annotations

import itertools
import math
import random

import numpy as np


class ScheduleError(AssertionError):
    pass


def _consts(T):
    if T is np.float32:
        return (np.float32(float.fromhex("0x1.555556p-3")), np.float32(float.fromhex("0x1.99999ap-6")),
                np.float32(float.fromhex("0x1.084210p-6")))
    return (np.float64(float.fromhex("0x1.5555555555555p-3")),
            np.float64(float.fromhex("0x1.999999999999ap-6")),
            np.float64(float.fromhex("0x1.0842108421084p-6")))


def level_eb(e, alpha, beta, l):
    pw = 1.0
    for _ in range(1, l):
        pw = pw * alpha
    m = min(pw, beta) if l > 1 else 1.0
    return e / m


class Tiny:
    def __init__(self, x, cfg, e, seed=0):
        self.T = np.float32 if cfg["dtype"] == "f32" else np.float64
        self.x = np.asarray(x, dtype=self.T).reshape(-1)
        self.shape = tuple(cfg["dims"]) + (1,) * (4 - len(cfg["dims"]))
        self.cfg = cfg
        self.e = e
        self.R = cfg.get("radius", 32768)
        f = cfg.get("frozen_dim", -1)
        self.act = [self.shape[d] > 1 and d != f for d in range(4)]
        self.strides = [int(np.prod(self.shape[d + 1:])) for d in range(4)]
        self.rng = random.Random(seed)
        self.K6, self.K40, self.K62 = _consts(self.T)
        # optional tuner score (Sec. 6.2): per level, the sum of
        # floor(|x - p| * 4096 / e) over the predicted points, capped at 2^32
        self.score = None
        self.level = 0

    def idx(self, c):
        return sum(c[d] * self.strides[d] for d in range(4))

    # -- stencils ---------------------------------------------------------
    def rd(self, i):
        if not self.known[i]:
            raise ScheduleError(f"read of point {i} before it is known")
        return self.W[i]

    def stencil(self, i, sd, xc, s, lo, hi, kind, sl):
        T = self.T
        ha, hc, hd = xc - 3 * s >= lo, xc + s <= hi, xc + 3 * s <= hi
        b = self.rd(i - sd)
        if kind == 0:
            if hc:
                return (b + self.rd(i + sd)) * T(0.5)
            if ha:
                return (b * T(3) - self.rd(i - 3 * sd)) * T(0.5)
            return b
        if sl:
            ha2, hd2 = xc - 2 * s >= lo, xc + 2 * s <= hi
            if kind == 1 and ha2 and hc and hd2:
                return ((b + self.rd(i + sd)) * T(4) - (self.rd(i - 2 * sd) + self.rd(i + 2 * sd))) * self.K6
            if kind == 2 and ha and ha2 and hc and hd2 and hd:
                return ((b + self.rd(i + sd)) * T(46) - (self.rd(i - 2 * sd) + self.rd(i + 2 * sd)) * T(18)
                        + (self.rd(i - 3 * sd) + self.rd(i + 3 * sd)) * T(3)) * self.K62
        if ha and hc and hd:
            a, c, d = self.rd(i - 3 * sd), self.rd(i + sd), self.rd(i + 3 * sd)
            if kind == 1:
                return ((b + c) * T(9) - (a + d)) * T(0.0625)
            return ((b + c) * T(23) - (a + d) * T(3)) * self.K40
        if hc and hd:
            return (b * T(3) + self.rd(i + sd) * T(6) - self.rd(i + 3 * sd)) * T(0.125)
        if ha and hc:
            return (b * T(6) + self.rd(i + sd) * T(3) - self.rd(i - 3 * sd)) * T(0.125)
        if hc:
            return (b + self.rd(i + sd)) * T(0.5)
        if ha:
            return (b * T(3) - self.rd(i - 3 * sd)) * T(0.5)
        return b

    def weights(self, kind, odd):
        mw = self.cfg.get("md_w", [[1.0] * 4] * 3)[kind]
        s = 0.0
        for d in range(4):
            if odd >> d & 1:
                s = s + mw[d]
        return {d: self.T(mw[d] / s) for d in range(4) if odd >> d & 1}

    # -- one point --------------------------------------------------------
    def visit(self, c, ip, pd, odd, sl, s, lo, hi, mode):
        i = self.idx(c)
        self.count[i] += 1
        if ip["md"]:
            wt = self.weights(ip["kind"], odd)
            acc = None
            for d in range(4):
                if odd >> d & 1:
                    t = wt[d] * self.stencil(i, s * self.strides[d], c[d], s, lo[d], hi[d], ip["kind"], sl)
                    acc = t if acc is None else acc + t
            p = acc
        else:
            p = self.stencil(i, s * self.strides[pd], c[pd], s, lo[pd], hi[pd], ip["kind"], sl)
        if mode == "d":
            q = int(self.code[i])
            if q != 0:
                self.W[i] = self.T(float(p) + float(q - self.R) * self.twoe)
        else:
            xv = self.x[i]
            if self.score is not None:
                u = abs(float(xv) - float(p)) * (4096.0 / self.e)
                self.score[self.level] = self.score.get(self.level, 0) + (
                    math.floor(u) if u < 4294967296.0 else 4294967296)
            t = (float(xv) - float(p)) * self.inv2e
            qf = math.floor(abs(t) + 0.5) if math.isfinite(t) else math.inf
            ok = qf < self.R
            if ok:
                q = -qf if t < 0 else qf
                xr = self.T(float(p) + q * self.twoe)
                ok = abs(float(xr) - float(xv)) <= self.el
            if ok:
                self.code[i] = int(q) + self.R
                self.W[i] = xr
            else:
                self.code[i] = 0
                self.W[i] = xv
        self.known[i] = True

    def lattice(self, r, m, rlo, rhi, filt, B):
        ranges = []
        for d in range(4):
            v = rlo[d] + ((r[d] - rlo[d]) % m[d])
            ranges.append(range(v, rhi[d] + 1, m[d]))
        pts = []
        for c in itertools.product(*ranges):
            if filt:
                face = any(self.act[d] and c[d] % B == 0 for d in range(4))
                if (filt == 1) != face:
                    continue
            pts.append(c)
        self.rng.shuffle(pts)
        return pts

    def run_config(self, ip, s, rlo, rhi, lo, hi, filt, B, mode):
        act = self.act
        if ip["md"]:
            nact = sum(act)
            for cnt in range(1, nact + 1):
                for odd in range(1, 16):
                    dims = [d for d in range(4) if odd >> d & 1]
                    if len(dims) != cnt or any(not act[d] for d in dims):
                        continue
                    r = [0] * 4
                    m = [1] * 4
                    for d in range(4):
                        if act[d]:
                            r[d], m[d] = (s, 2 * s) if odd >> d & 1 else (0, 2 * s)
                    pts = self.lattice(r, m, rlo, rhi, filt, B)
                    if ip["kind"] != 0 and ip["same_level"]:
                        # same-level halves (Sec. 5.4.2 extended to MD): the
                        # checkerboard of sum (x_d - s) / 2s over the odd dims;
                        # colour 0 first, regular stencils, then colour 1 with
                        # the same-level stencils
                        colour = lambda c: sum((c[d] - s) // (2 * s) for d in dims) % 2
                        for half in (0, 1):
                            for c in pts:
                                if colour(c) == half:
                                    self.visit(c, ip, -1, odd, half, s, lo, hi, mode)
                    else:
                        for c in pts:
                            self.visit(c, ip, -1, odd, 0, s, lo, hi, mode)
            return
        order = [d for d in ip["order"] if d < 4 and act[d]]
        seen = []
        for d in order:
            if d not in seen:
                seen.append(d)
        for k, pd in enumerate(seen):
            r = [0] * 4
            m = [1] * 4
            for d in range(4):
                if not act[d]:
                    continue
                if d == pd:
                    r[d], m[d] = s, 2 * s
                elif d in seen[:k]:
                    r[d], m[d] = 0, s
                else:
                    r[d], m[d] = 0, 2 * s
            if ip["kind"] != 0 and ip["same_level"]:
                m[pd] = 4 * s
                for half, rr in ((0, s), (1, 3 * s)):
                    r[pd] = rr
                    for c in self.lattice(r, m, rlo, rhi, filt, B):
                        self.visit(c, ip, pd, 0, half, s, lo, hi, mode)
            else:
                for c in self.lattice(r, m, rlo, rhi, filt, B):
                    self.visit(c, ip, pd, 0, 0, s, lo, hi, mode)

    def schedule(self, mode):
        cfg = self.cfg
        L = cfg["anchor_log2"]
        B = (1 << cfg["block_log2"]) if cfg.get("block_log2", 0) else 0
        n = self.shape
        glo = [0] * 4
        ghi = [n[d] - 1 for d in range(4)]
        for l in range(L, 0, -1):
            s = 1 << (l - 1)
            self.level = l
            self.el = level_eb(self.e, cfg.get("alpha", 1.0), cfg.get("beta", 1.0), l)
            self.inv2e = 1.0 / (2.0 * self.el)
            self.twoe = 2.0 * self.el
            ip = cfg["levels"][l - 1]
            if B and s < B:
                self.run_config(ip, s, glo, ghi, glo, ghi, 1, B, mode)
                nb = [(n[d] + B - 1) // B for d in range(4)]
                for bi, b in enumerate(itertools.product(*[range(v) for v in nb])):
                    bp = cfg["cand"][int(cfg["block_cfg"][bi])]
                    rlo = [b[d] * B for d in range(4)]
                    rhi = [min(rlo[d] + B - 1, n[d] - 1) for d in range(4)]
                    chi = [min(rlo[d] + B, n[d] - 1) for d in range(4)]
                    self.run_config(bp, s, rlo, rhi, rlo, chi, 2, B, mode)
            else:
                self.run_config(ip, s, glo, ghi, glo, ghi, 0, B, mode)

    def anchors(self):
        A = 1 << self.cfg["anchor_log2"]
        out = []
        for c in itertools.product(*[range(v) for v in self.shape]):
            if all((not self.act[d]) or c[d] % A == 0 for d in range(4)):
                out.append(self.idx(c))
        return out

    def compress(self):
        N = self.x.size
        self.W = np.zeros(N, dtype=self.T)
        self.code = np.zeros(N, dtype=np.int64)
        self.known = np.zeros(N, dtype=bool)
        self.count = np.zeros(N, dtype=np.int64)
        for i in self.anchors():
            self.W[i] = self.x[i]
            self.code[i] = self.R
            self.known[i] = True
            self.count[i] += 1
        self.schedule("c")
        if not (self.count == 1).all():
            bad = np.nonzero(self.count != 1)[0][:5]
            raise ScheduleError(f"points predicted {self.count[bad]} times: {bad}")
        return self.code.astype(np.uint16), self.W.copy()

    def decompress(self, code, anchor_vals, unpred_vals):
        N = code.size
        self.code = np.asarray(code, dtype=np.int64).reshape(-1)
        self.W = np.zeros(N, dtype=self.T)
        self.known = np.zeros(N, dtype=bool)
        self.count = np.zeros(N, dtype=np.int64)
        anc = self.anchors()
        aset = set(anc)
        for k, i in enumerate(anc):
            self.W[i] = anchor_vals[k]
            self.known[i] = True
        u = 0
        for i in range(N):
            if i not in aset and self.code[i] == 0:
                self.W[i] = unpred_vals[u]
                u += 1
        self.schedule("d")
        return self.W.copy()
