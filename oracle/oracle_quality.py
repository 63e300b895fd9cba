"""Quality metrics and quality-target error bounds of the oracle (test
infrastructure only: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it; the product library never does).

Sec. 3.1, Eq. (1): the compressor meets the point-wise bound e and, among such
configurations, maximises the compression ratio subject to a user quality
requirement M(X, X') >= m0, M being PSNR, SSIM, or a constant (ratio only).
The paper uses PSNR with the data's value range and SSIM (Wang et al. 2004)
without restating either; the definitions below are the usual ones, made
exact where the paper leaves a choice open:

* value range L = max(X) - min(X) in float64;
* MSE = mean((x - x')^2) in float64, PSNR = 20 log10(L) - 10 log10(MSE)
  (+inf when MSE = 0; with L = 0 and MSE > 0, -inf);
* SSIM = mean over windows of ((2 mx my + C1)(2 sxy + C2)) /
  ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2)), with C1 = (0.01 L)^2,
  C2 = (0.03 L)^2 (L = 1 when the range is 0), uniform weights and
  population moments (1/n).  Windows are boxes of side w (8 by default) along
  every dimension of size > 1 (a dimension shorter than w is one window
  wide), laid without overlap from the origin; a partial window at the far
  end of a dimension is left out.

The quality-target search (`fit_eb`) looks for the largest absolute bound e
whose full compression meets M >= m0 (the ratio grows with e), by the steps
written out in `fit_eb` itself.

parity pinned: metrics by closed forms (constant shift, affine maps, equal
inputs) and an independent sliding-window brute force on small grids
(tests/test_oracle_quality_pins.py); the search by feasibility and
bracketing properties of its result.
"""
from __future__ import annotations

import math

import numpy as np

K1, K2 = 0.01, 0.03
DEFAULT_WINDOW = 8


def value_range(x: np.ndarray) -> float:
    x = np.asarray(x)
    return float(np.float64(x.max()) - np.float64(x.min())) if x.size else 0.0


def _windows(shape, w):
    """Per dimension: (window side, number of windows) under the rule above."""
    out = []
    for n in shape:
        if n <= 1:
            out.append((1, 1))
        elif n < w:
            out.append((n, 1))
        else:
            out.append((w, n // w))
    return out


def ssim(x: np.ndarray, xr: np.ndarray, window: int = DEFAULT_WINDOW, L: float | None = None):
    """Mean SSIM over the non-overlapping windows (definition in the module
    docstring); returns (ssim, number of windows)."""
    x = np.asarray(x, dtype=np.float64)
    xr = np.asarray(xr, dtype=np.float64)
    if L is None:
        L = value_range(x)
    if L == 0.0:
        L = 1.0
    C1 = (K1 * L) ** 2
    C2 = (K2 * L) ** 2
    win = _windows(x.shape, window)
    total = 0.0
    count = 0
    for idx in np.ndindex(*[nw for _, nw in win]):
        sl = tuple(slice(i * s, i * s + s) for i, (s, _) in zip(idx, win))
        a = x[sl].ravel()
        b = xr[sl].ravel()
        n = a.size
        mx = a.sum() / n
        my = b.sum() / n
        da = a - mx
        db = b - my
        sxx = (da * da).sum() / n
        syy = (db * db).sum() / n
        sxy = (da * db).sum() / n
        total += ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
        count += 1
    return total / count, count


def metrics(x: np.ndarray, xr: np.ndarray, window: int = DEFAULT_WINDOW) -> dict:
    """Eq. (1)'s quality functions M of a reconstruction xr of x."""
    x64 = np.asarray(x, dtype=np.float64)
    r64 = np.asarray(xr, dtype=np.float64)
    if x64.shape != r64.shape:
        raise ValueError("shapes differ")
    L = value_range(x64)
    d = x64 - r64
    mse = float(np.mean(d * d)) if d.size else 0.0
    maxerr = float(np.max(np.abs(d))) if d.size else 0.0
    if mse == 0.0:
        psnr = math.inf
    elif L == 0.0:
        psnr = -math.inf
    else:
        psnr = 20.0 * math.log10(L) - 10.0 * math.log10(mse)
    s, nw = ssim(x64, r64, window, L)
    return dict(n=int(x64.size), value_range=L, max_abs_err=maxerr, mse=mse, psnr=psnr,
                ssim=float(s), n_windows=int(nw))


METRICS = ("psnr", "ssim")
STEPS = 64  # bound grid: G steps per octave


def grid_eb(L: float, k: int, G: int = STEPS) -> float:
    """Bound k of the search grid: e_k = L 2^(k / G) (L the value range)."""
    return L * math.pow(2.0, k / G)


def _round(v: float) -> int:
    return int(math.floor(v + 0.5))


def initial_k(metric: str, target: float, G: int = STEPS) -> int:
    """First grid index of the search: for PSNR the uniform-quantizer model
    (errors uniform on [-e, e] have MSE e^2 / 3, so e / L = sqrt(3)
    10^(-PSNR / 20)), for SSIM e / L = 10^-3."""
    if metric == "psnr":
        r = math.sqrt(3.0) * math.pow(10.0, -target / 20.0)
    else:
        r = 1e-3
    return _round(G * math.log2(r))


def model_step(metric: str, target: float, m: float, G: int = STEPS) -> int:
    """Grid steps suggested by a measured metric m: PSNR moves by 20 dB per
    decade of e; SSIM's deficit 1 - SSIM grows as e^2.  At least one step
    away from a met target (up) or a missed one (down), at most 4 octaves."""
    if metric == "psnr":
        dk = 4 * G if math.isinf(m) else _round(G * (m - target) / 20.0 * math.log2(10.0))
    else:
        dk = 4 * G if m >= 1.0 else _round(G * math.log2((1.0 - target) / (1.0 - m)) / 2.0)
    if m >= target:
        return min(4 * G, max(1, dk))
    return max(-4 * G, min(-1, dk))


def fit_eb(x: np.ndarray, cfg: dict, metric: str, target: float, max_iter: int = 12,
           window: int = DEFAULT_WINDOW, G: int = STEPS, compress=None, decompress=None):
    """Largest absolute bound on the grid e_k = L 2^(k / G) found whose
    compression of x under cfg meets metric >= target (Eq. 1).  Steps:
    k = initial_k; each iteration compresses and decompresses at e_k and
    measures the metric; a bound that meets the target raises the feasible
    floor k_lo, one that misses lowers the infeasible ceiling k_hi; the next
    index is k + model_step until both k_lo and k_hi exist, then
    floor((k_lo + k_hi) / 2); the search ends when k_hi - k_lo <= 1 or after
    max_iter compressions.  Returns (e_lo, its metrics, iterations, e_hi);
    e_lo = 0 when no tried bound met the target, e_hi = inf when none missed
    it.  A field of range 0 is reproduced exactly at any bound: (0, metrics of
    x itself, 0, inf).  (The grid makes the result a function of integer
    decisions, so implementations whose metric sums round differently still
    agree unless a metric lands within rounding of the target.)"""
    from . import oracle as O  # the oracle's own compressor

    if metric not in METRICS:
        raise ValueError(metric)
    compress = compress or O.compress
    decompress = decompress or O.decompress
    L = value_range(x)
    if L == 0.0:
        return 0.0, metrics(x, x, window), 0, math.inf
    k = initial_k(metric, target, G)
    k_lo = k_hi = None
    best = None
    it = 0
    while it < max_iter:
        e = grid_eb(L, k, G)
        c = dict(cfg, eb_mode="abs", eb=e)
        xr = decompress(compress(x, c)).reshape(x.shape)
        q = metrics(x, xr, window)
        it += 1
        m = q[metric]
        if m >= target:
            if k_lo is None or k > k_lo:
                k_lo, best = k, q
        elif k_hi is None or k < k_hi:
            k_hi = k
        if k_lo is not None and k_hi is not None:
            if k_hi - k_lo <= 1:
                break
            k = k_lo + (k_hi - k_lo) // 2
        else:
            k = k + model_step(metric, target, m, G)
    e_lo = grid_eb(L, k_lo, G) if k_lo is not None else 0.0
    e_hi = grid_eb(L, k_hi, G) if k_hi is not None else math.inf
    return e_lo, best, it, e_hi
