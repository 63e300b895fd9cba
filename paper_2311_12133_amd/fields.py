"""Seeded synthetic input fields.

This module only draws random numbers and shapes them into test fields; it
holds none of the compressor's arithmetic, and both the oracle side and the
GPU side read the very same bytes from it.

The paper evaluates on real simulation datasets (Miranda 256x384x384, JHTDB
512^3, CESM-ATM 1800x3600 slices, RTM 449^3-class volumes; see the dataset
table of Sec. 7.1.1).  They are not available here, so these fields stand in
for them with the same shapes and with turbulence-like power-law spectra.

Spectrum convention: ``slope`` is the exponent of the shell-integrated energy
spectrum E(k) ~ k^slope.  In D dimensions the spectral density is then
~ k^(slope - (D - 1)), so the Fourier amplitudes are scaled by |k|^gamma with
gamma = (slope - (D - 1)) / 2 (the k = 0 mode is zeroed).  Fields are
normalised to zero mean and unit variance, generated in float64.
"""
from __future__ import annotations

import os

import numpy as np

SEED_BASE = 2311121330


def rng_for(config: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * config + index))


def gaussian_field(shape, slope: float, rng: np.random.Generator) -> np.ndarray:
    """Zero-mean unit-variance Gaussian random field with E(k) ~ k^slope (float64)."""
    shape = tuple(int(s) for s in shape)
    D = len(shape)
    noise = rng.standard_normal(shape)
    spec = np.fft.rfftn(noise)
    del noise
    k2 = None
    for ax, n in enumerate(shape):
        if ax == D - 1:
            f = np.fft.rfftfreq(n) * n
        else:
            f = np.fft.fftfreq(n) * n
        sh = [1] * D
        sh[ax] = f.size
        term = (f.reshape(sh)) ** 2
        k2 = term if k2 is None else k2 + term
    gamma = (slope - (D - 1)) / 2.0
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (gamma / 2.0), 0.0)
    del k2
    spec *= amp
    del amp
    g = np.fft.irfftn(spec, s=shape, axes=tuple(range(D)))
    del spec
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    return g


def _pow2_size(n: int) -> int:
    """Smallest power of two >= n."""
    m = 1
    while m < n:
        m *= 2
    return m


def gaussian_field_device(shape, slope: float, seed: int, device, dtype=None):
    """The same construction as gaussian_field, on a torch device (float64 FFTs)
    with torch's seeded normal generator: for workloads too large to synthesise
    on the host within a benchmark run.  The field is synthesised on the
    smallest enclosing grid with power-of-two sides (transform sizes with
    precompiled kernels) and cropped; the crop of a stationary field has the
    same spectrum.  Deterministic
    for a given seed and device type; its values differ from gaussian_field's."""
    import torch
    want = tuple(int(s) for s in shape)
    shape = tuple(_pow2_size(s) for s in want)
    D = len(shape)
    gen = torch.Generator(device=device)
    gen.manual_seed(SEED_BASE + int(seed))
    noise = torch.randn(shape, generator=gen, dtype=torch.float64, device=device)
    spec = torch.fft.rfftn(noise)
    del noise
    k2 = None
    for ax, n in enumerate(shape):
        if ax == D - 1:
            f = torch.fft.rfftfreq(n, dtype=torch.float64, device=device) * n
        else:
            f = torch.fft.fftfreq(n, dtype=torch.float64, device=device) * n
        sh = [1] * D
        sh[ax] = f.numel()
        term = f.reshape(sh) ** 2
        k2 = term if k2 is None else k2 + term
    gamma = (slope - (D - 1)) / 2.0
    amp = torch.where(k2 > 0, k2.clamp_min(1e-300) ** (gamma / 2.0), torch.zeros_like(k2))
    del k2
    spec *= amp
    del amp
    g = torch.fft.irfftn(spec, s=shape, dim=tuple(range(D)))
    del spec
    g = g[tuple(slice(0, n) for n in want)].contiguous()
    g -= g.mean()
    sd = g.std(unbiased=False)
    if sd > 0:
        g /= sd
    return g if dtype is None else g.to(dtype)


def fronts(shape, count: int, width: float, amp: float, rng: np.random.Generator) -> np.ndarray:
    """Sum of `count` tanh fronts amp * tanh(n.(x - c) / width) with random unit
    normals n and centres c uniform in the box (float64)."""
    shape = tuple(int(s) for s in shape)
    D = len(shape)
    out = np.zeros(shape, dtype=np.float64)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij",
                        sparse=True)
    for _ in range(count):
        nv = rng.standard_normal(D)
        nv /= np.linalg.norm(nv)
        c = rng.uniform(0, 1, D) * np.array(shape, dtype=np.float64)
        arg = sum(nv[d] * (grids[d] - c[d]) for d in range(D))
        out += amp * np.tanh(arg / width)
    return out


def _cache_path(name: str):
    root = os.environ.get("HPEZ_FIELD_CACHE")
    if not root:
        return None
    os.makedirs(root, exist_ok=True)
    return os.path.join(root, name + ".npy")


def _cached(name: str, make):
    p = _cache_path(name)
    if p and os.path.exists(p):
        return np.load(p, allow_pickle=False)
    a = make()
    if p:
        np.save(p + ".tmp.npy", a)
        os.replace(p + ".tmp.npy", p)
    return a


def plain_field(shape=(64, 64, 64), slope=-3.0, seed_index=0, dtype=np.float32):
    """Plain-method workload: Gaussian field with E(k) ~ k^-3 (smooth)."""
    name = f"plain_{'x'.join(map(str, shape))}_{slope}_{seed_index}_{np.dtype(dtype).name}"
    return _cached(name, lambda: gaussian_field(shape, slope, rng_for(1, seed_index))
                   .astype(dtype))


def fronts_field(shape=(256, 384, 384), seed_index=0, dtype=np.float32):
    """Turbulence-like field (E ~ k^-5/3) plus three tanh fronts of width 2
    cells, standing in for the Miranda volume."""
    name = f"fronts_{'x'.join(map(str, shape))}_{seed_index}_{np.dtype(dtype).name}"

    def make():
        rng = rng_for(2, seed_index)
        g = gaussian_field(shape, -5.0 / 3.0, rng)
        g += fronts(shape, 3, 2.0, 1.0, rng)
        return g.astype(dtype)
    return _cached(name, make)


def lognormal_field(shape=(512, 512, 512), seed_index=0, dtype=np.float32):
    """Heavy-tailed density-like field exp(1.5 g), g a unit-variance E ~ k^-5/3
    Gaussian field, standing in for the JHTDB volume.  The float32 copy is the
    cast of the float64 one."""
    name = f"lognormal_{'x'.join(map(str, shape))}_{seed_index}_{np.dtype(dtype).name}"

    def make():
        g = gaussian_field(shape, -5.0 / 3.0, rng_for(3, seed_index))
        np.multiply(g, 1.5, out=g)
        np.exp(g, out=g)
        return g.astype(dtype)
    return _cached(name, make)


def turbulence_field(shape, seed_index=0, config=4, dtype=np.float32):
    """E ~ k^-5/3 Gaussian field of any shape (batched workloads)."""
    name = f"turb_{config}_{'x'.join(map(str, shape))}_{seed_index}_{np.dtype(dtype).name}"
    return _cached(name, lambda: gaussian_field(shape, -5.0 / 3.0, rng_for(config, seed_index))
                   .astype(dtype))


def random_field(shape, seed: int, dtype=np.float32, kind: str = "smooth"):
    """Small seeded fields for tests: 'smooth' (k^-3 spectrum), 'rough'
    (white noise), 'mixed' (smooth plus noise plus a few spikes)."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 7 + seed))
    if kind == "rough":
        a = rng.standard_normal(shape)
    elif kind == "mixed":
        a = gaussian_field(shape, -3.0, rng) + 0.05 * rng.standard_normal(shape)
        flat = a.reshape(-1)
        idx = rng.integers(0, flat.size, max(1, flat.size // 500))
        flat[idx] += rng.standard_normal(idx.size) * 50.0
    else:
        a = gaussian_field(shape, -3.0, rng)
    return np.ascontiguousarray(a.astype(dtype))


def batch_shapes(seed_index: int = 0):
    """Shapes of the uneven batched workload: 16 x (100,500,500), 16 x (1800,3600),
    16 3D fields with each dim uniform in [64, 449]; per-field relative bounds
    drawn from {1e-2, 1e-3, 1e-4}."""
    rng = rng_for(4, 10_000 + seed_index)
    shapes = [(100, 500, 500)] * 16 + [(1800, 3600)] * 16
    for _ in range(16):
        shapes.append(tuple(int(v) for v in rng.integers(64, 450, 3)))
    ebs = [float(v) for v in rng.choice([1e-2, 1e-3, 1e-4], len(shapes))]
    return shapes, ebs
