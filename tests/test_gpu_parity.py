"""GPU parity: the HIP library through the C ABI against the CPU oracle on the
same seeded inputs.  Integer outputs (codes, Huffman bitstream, the whole
stream) must be byte-identical; decompressed values bit-identical (the method
is deterministic: FP contraction is off on both sides and every stencil and
quantizer operation is written in the same order).  Every case also checks
|x - x'| <= e on every point."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from cfgs import candidates, interp, make_cfg
from oracle import oracle as O
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


def roundtrip(torch, x, cfg, label):
    from paper_2311_12133_amd import binding
    print(f"[case] {label} shape={x.shape} dtype={cfg['dtype']}", flush=True)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    s = binding.compress(xt, cfg)
    torch.cuda.synchronize()
    got = s.cpu().numpy().tobytes()
    ref = O.compress(x, cfg)
    if got != ref:
        a = np.frombuffer(got, np.uint8)
        b = np.frombuffer(ref, np.uint8)
        n = min(a.size, b.size)
        first = int(np.nonzero(a[:n] != b[:n])[0][0]) if (a[:n] != b[:n]).any() else n
        raise AssertionError(f"{label}: stream differs (gpu {a.size} B, oracle {b.size} B, "
                             f"first diff at byte {first})")
    y = binding.decompress(s).cpu().numpy()
    yo = O.decompress(ref)
    assert np.array_equal(y.view(np.uint8), yo.view(np.uint8)), f"{label}: decompressed differs"
    if cfg["eb_mode"] == "rel":
        e, const = O.error_bound(x, cfg)
    else:
        e, const = cfg["eb"], False
    if not const:
        assert np.abs(x.astype(np.float64) - y.astype(np.float64)).max() <= e
    return got


KW = [
    dict(kind="lin"), dict(kind="nak"), dict(kind="nat"),
    dict(kind="lin", md=1), dict(kind="nak", md=1), dict(kind="nat", md=1),
    dict(kind="nak", same_level=1), dict(kind="nat", same_level=1),
    dict(kind="nak", order=(2, 0, 1)), dict(kind="nat", order=(1, 2, 0), same_level=1),
    dict(kind="nak", md=1, same_level=1), dict(kind="nat", md=1, same_level=1),
]


@pytest.mark.parametrize("kw", KW, ids=[str(i) for i in range(len(KW))])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_configs_3d(torch_cuda, kw, dtype):
    x = fields.random_field((37, 70, 129), 3, np.float32 if dtype == "f32" else np.float64,
                            "smooth")
    roundtrip(torch_cuda, x, make_cfg(x.shape, dtype=dtype, eb=1e-3, **kw), f"3d {kw}")


@pytest.mark.parametrize("shape", [(1,), (2,), (7,), (1000,), (5000,), (3, 1),
                                   (1, 300), (257, 129), (1800, 36), (2, 3, 4),
                                   (64, 1, 65), (9, 17, 33, 5)])
def test_shapes(torch_cuda, shape):
    x = fields.random_field(shape, len(shape) + shape[0], np.float32, "mixed")
    for kw in (dict(kind="nak"), dict(kind="nat", md=1)):
        roundtrip(torch_cuda, x, make_cfg(shape, eb=1e-3, **kw), f"shape {shape} {kw}")


def test_plain_64cube(torch_cuda):
    """The plain-method workload: 64^3 k^-3 field, linear, natural order."""
    x = fields.plain_field((64, 64, 64))
    roundtrip(torch_cuda, x, make_cfg(x.shape, eb=1e-3), "plain 64^3")


def test_unpredictable_and_radius(torch_cuda):
    """Spikes with a tiny radius force out-of-range codes (verbatim values)."""
    x = fields.random_field((40, 50, 60), 5, np.float32, "mixed")
    cfg = make_cfg(x.shape, eb=1e-4, kind="nak", radius=64)
    s = roundtrip(torch_cuda, x, cfg, "radius 64")
    n_unpred = int(np.frombuffer(s[456:464], np.uint64)[0])
    assert n_unpred > 100


def test_abs_bound_alpha_beta_frozen(torch_cuda):
    x = fields.random_field((30, 64, 70), 8, np.float64, "rough")
    for kw in (dict(kind="nak", alpha=1.5, beta=4.0), dict(kind="lin", frozen_dim=1),
               dict(kind="nat", md=1, frozen_dim=2, alpha=2.0, beta=2.0)):
        roundtrip(torch_cuda, x, make_cfg(x.shape, dtype="f64", eb=0.01, eb_mode="abs", **kw),
                  f"abs {kw}")


def test_constant_field(torch_cuda):
    x = np.full((33, 17, 5), -2.5, dtype=np.float32)
    roundtrip(torch_cuda, x, make_cfg(x.shape, eb=1e-3), "constant")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_block_wise(torch_cuda, dtype):
    x = fields.random_field((70, 66, 97), 9, np.float32 if dtype == "f32" else np.float64,
                            "mixed")
    cand = candidates(3)
    for B, al in ((8, 4), (32, 6)):
        nb = int(np.prod([(s + B - 1) // B for s in x.shape]))
        bc = (np.arange(nb) * 5 % 11).astype(np.uint8)
        cfg = make_cfg(x.shape, dtype=dtype, eb=1e-3, kind="nat", anchor_log2=al,
                       block_log2=int(np.log2(B)), cand=cand, block_cfg=bc)
        roundtrip(torch_cuda, x, cfg, f"block-wise B={B}")


@pytest.mark.parametrize("use", ["none", "one", "all"])
def test_block_wise_same_level_use(torch_cuda, use):
    """Generic block steps (float64) with same-level candidates offered: no
    block on them (the second-half steps are skipped), exactly one block on
    one, every block on one."""
    x = fields.random_field((45, 40, 52), 21, np.float64, "mixed")
    cand = candidates(3)
    B = 8
    nb = int(np.prod([(s + B - 1) // B for s in x.shape]))
    bc = (np.arange(nb) * 5 % 9).astype(np.uint8)
    if use == "one":
        bc[nb // 2] = 9
    elif use == "all":
        bc[:] = 9 + np.arange(nb) % 2
    cfg = make_cfg(x.shape, dtype="f64", eb=1e-3, kind="nat", anchor_log2=4, block_log2=3,
                   cand=cand, block_cfg=bc)
    roundtrip(torch_cuda, x, cfg, f"same-level use {use}")


GENERIC_BLOCK = [((30, 64, 70), "f64", 1, 8), ((9, 17, 33, 5), "f32", -1, 4),
                 ((11, 6, 20, 13), "f64", 2, 4)]


@pytest.mark.parametrize("shape,dt,frozen,B", GENERIC_BLOCK,
                         ids=["x".join(map(str, s)) + f"-{d}-fz{f}-B{b}"
                              for s, d, f, b in GENERIC_BLOCK])
def test_block_wise_generic_frozen_4d(torch_cuda, shape, dt, frozen, B):
    """Generic block steps where a dim takes every coordinate of a block (a
    frozen dim) and in four dims, every candidate in use."""
    nd = len(shape)
    cand = candidates(nd)
    nb = int(np.prod([(s + B - 1) // B for s in shape]))
    bc = (np.arange(nb) * 7 % len(cand)).astype(np.uint8)
    x = fields.random_field(shape, nb + nd, np.float32 if dt == "f32" else np.float64, "mixed")
    cfg = make_cfg(shape, dtype=dt, eb=1e-3, kind="nat", md=1, frozen_dim=frozen,
                   anchor_log2=3 if B == 4 else 4, block_log2=int(np.log2(B)), cand=cand,
                   block_cfg=bc)
    roundtrip(torch_cuda, x, cfg, f"generic blocks {shape} {dt} frozen {frozen} B={B}")


@pytest.mark.parametrize("pred", ["interp", "lorenzo"])
@pytest.mark.parametrize("radius", [1, 2, 3])
def test_smallest_radii(torch_cuda, pred, radius):
    """Radius 1-3 on the paths with a separate code histogram: the bins next to
    the zero-error code reach the ends of the code range (radius 1 has only the
    verbatim code and the zero-error code)."""
    x = fields.random_field((23, 31, 40), radius, np.float64, "mixed")
    cfg = make_cfg(x.shape, dtype="f64", eb=1e-3, kind="nak", radius=radius, predictor=pred)
    roundtrip(torch_cuda, x, cfg, f"radius {radius} {pred}")


def test_chunk_sizes(torch_cuda):
    x = fields.random_field((50, 61, 33), 2, np.float32, "smooth")
    for chunk in (64, 256, 1024):
        roundtrip(torch_cuda, x, make_cfg(x.shape, eb=1e-4, kind="nak", chunk=chunk),
                  f"chunk {chunk}")


def test_corrupt_stream_rejected(torch_cuda):
    from paper_2311_12133_amd import binding
    x = fields.random_field((20, 20, 20), 2, np.float32, "smooth")
    cfg = make_cfg(x.shape)
    s = binding.compress(torch_cuda.from_numpy(x).cuda(), cfg)
    bad = s.clone()
    bad[0] ^= 0xFF
    with pytest.raises(binding.HpezError):
        binding.decompress(bad)
    with pytest.raises(binding.HpezError):
        binding.decompress(s[: s.numel() - 8])


def test_nonfinite_rejected(torch_cuda):
    from paper_2311_12133_amd import binding
    x = fields.random_field((10, 10, 10), 2, np.float32, "smooth")
    x[3, 4, 5] = np.nan
    with pytest.raises(binding.HpezError):
        binding.compress(torch_cuda.from_numpy(x).cuda(), make_cfg(x.shape))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_lorenzo(torch_cuda, dtype):
    """Lorenzo alternative (Sec. 6.5): residual codes, outliers and patches."""
    T = np.float32 if dtype == "f32" else np.float64
    for shape in ((3000,), (70, 90), (33, 40, 29), (6, 7, 8, 9)):
        x = fields.random_field(shape, 4, T, "mixed")
        roundtrip(torch_cuda, x, make_cfg(shape, dtype=dtype, eb=1e-3, predictor="lorenzo"),
                  f"lorenzo {shape}")
    # small radius forces outliers
    x = fields.random_field((40, 50, 60), 6, T, "rough")
    s = roundtrip(torch_cuda, x, make_cfg(x.shape, dtype=dtype, eb=1e-4, predictor="lorenzo",
                                          radius=16), "lorenzo outliers")
    assert int(np.frombuffer(s[464:472], np.uint64)[0]) > 100
    if dtype == "f32":
        # values far above the bound: (float)(v * 2e) often misses -> patches
        x = (fields.random_field((30, 40, 50), 7, np.float64, "smooth") * 1e3 + 3e6).astype(T)
        s = roundtrip(torch_cuda, x, make_cfg(x.shape, dtype=dtype, eb=0.13, eb_mode="abs",
                                              predictor="lorenzo"), "lorenzo patches")
        assert int(np.frombuffer(s[472:480], np.uint64)[0]) > 10


def fibonacci_walk(nsym: int, seed: int) -> np.ndarray:
    """A 1-D walk whose first-order differences take nsym values with
    Fibonacci counts F_1..F_nsym (the most frequent difference 0, then +1, -1,
    +2, ...), shuffled with a seeded generator.  With the Lorenzo predictor at
    an absolute bound of 1/2 (bins of width 1) the codes are exactly the
    differences, so their Huffman tree is a chain as deep as the alphabet."""
    f = [1, 1]
    while len(f) < nsym:
        f.append(f[-1] + f[-2])
    counts = np.array(f[:nsym][::-1], dtype=np.int64)
    vals = np.array([0] + [(k + 1) // 2 * (1 if k % 2 else -1) for k in range(1, nsym)])
    d = np.repeat(vals, counts)
    np.random.Generator(np.random.PCG64(2311121330 + 77 + nsym)).shuffle(d)
    x = np.cumsum(d)
    assert np.abs(x).max() < 2 ** 24  # exact in float32
    return x.astype(np.float32)


@pytest.mark.parametrize("nsym,maxlen", [(33, 32), (34, 17)])
def test_huffman_long_codes(torch_cuda, nsym, maxlen):
    """Huffman edge cases of Sec. 4 step 4: 33 Fibonacci-distributed symbols give
    codewords of the full 32 bits (the decoder's path beyond its lookup tables);
    34 exceed the 32-bit limit and force the halving rebuild, which leaves 17."""
    x = fibonacci_walk(nsym, 0)
    f = [1, 1]
    while len(f) < nsym:
        f.append(f[-1] + f[-2])
    assert int(O.huff_lengths(np.array(f[:nsym], np.uint32)).max()) == maxlen
    roundtrip(torch_cuda, x, make_cfg(x.shape, eb=0.5, eb_mode="abs", predictor="lorenzo"),
              f"huffman {nsym} Fibonacci symbols ({x.size} points)")


# the last four sit at the split between the block kernel's 1024-lane launch
# (any box) and its 256-lane one (at most two active dims, at most 33 x 33
# points): a tiny box with three active dims, a thin one with three, and two
# with one or two active dims
FAST_SHAPES = [(64, 64, 64), (65, 33, 97), (96, 31, 130), (33, 64, 1), (200, 161), (1, 77, 64),
               (40, 40, 40), (10, 12, 9), (3, 50, 40), (17, 1, 33), (1, 1, 3000)]


@pytest.mark.parametrize("shape", FAST_SHAPES, ids=["x".join(map(str, s)) for s in FAST_SHAPES])
def test_block_fast_path(torch_cuda, shape):
    """Block-wise configurations with B = 32 (faces + per-block LDS kernel)."""
    x = fields.random_field(shape, sum(shape), np.float32, "mixed")
    nd = len(shape)
    cand = candidates(nd)
    nb = int(np.prod([(s + 31) // 32 for s in shape]))
    rng = np.random.default_rng(nb)
    for trial, kw in enumerate((dict(kind="nak"), dict(kind="nat", md=1),
                                dict(kind="lin", same_level=1, alpha=1.5, beta=3.0),
                                dict(kind="nak", same_level=1, frozen_dim=0, radius=512))):
        bc = rng.integers(0, len(cand), nb).astype(np.uint8)
        cfg = make_cfg(shape, eb=1e-3 if trial != 3 else 2e-5, anchor_log2=6 if nd >= 3 else 7,
                       block_log2=5, cand=cand, block_cfg=bc, **kw)
        roundtrip(torch_cuda, x, cfg, f"fast {shape} {kw}")


@pytest.mark.parametrize("shape", [(36, 600, 600), (3, 40000)], ids=["36x600x600", "3x40000"])
def test_block_fast_path_planes_too_large(torch_cuda, shape):
    """Block-wise B = 32 on fields whose face planes are too large for the
    plane kernel (600 x 600 planes; a face line of 10^4 lattice cells): the
    coarse face levels run as face steps, which the coarse block levels read.
    Three compressions of each configuration must equal the oracle's stream."""
    from paper_2311_12133_amd import binding
    nd = len(shape)
    x = fields.random_field(shape, 600, np.float32, "mixed")
    cand = candidates(nd)
    nb = int(np.prod([(s + 31) // 32 for s in shape]))
    bc = np.random.default_rng(nb).integers(0, len(cand), nb).astype(np.uint8)
    xt = torch_cuda.from_numpy(x).cuda()
    for kw in (dict(kind="nak"), dict(kind="nat", md=1)):
        cfg = make_cfg(shape, eb=1e-3, anchor_log2=6 if nd == 3 else 7, block_log2=5, cand=cand,
                       block_cfg=bc, **kw)
        got = roundtrip(torch_cuda, x, cfg, f"large planes {kw}")
        for _ in range(2):
            again = binding.compress(xt, cfg).cpu().numpy().tobytes()
            assert again == got, f"large planes {kw}: repeated compression differs"


def test_block_fast_2d_f64(torch_cuda):
    x = fields.random_field((150, 230), 3, np.float64, "mixed")
    cand = candidates(2)
    nb = 5 * 8
    bc = (np.arange(nb) * 3 % 11).astype(np.uint8)
    roundtrip(torch_cuda, x, make_cfg(x.shape, dtype="f64", eb=1e-4, anchor_log2=7, block_log2=5,
                                      cand=cand, block_cfg=bc, kind="nat", md=1), "fast 2d f64")


def test_caller_stream(torch_cuda):
    """Every call on a caller-created stream (not the current one): the work the
    library queues on its own second stream (coarse block levels, block-wise
    tuner trials) is ordered by that stream; results equal the oracle's."""
    torch = torch_cuda
    from paper_2311_12133_amd import binding
    shape = (96, 64, 128)
    x = fields.fronts_field(shape)
    print(f"[case] caller stream shape={shape}", flush=True)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    opts = dict(global_rate=0.2, allow_freeze=0)
    cfg = make_cfg(shape, eb=1e-3)
    ref_cfg, _ = O.tune(x, cfg, opts)
    with torch.cuda.stream(st):
        got_cfg = binding.tune(xt, cfg, opts, stream=st)
        s = binding.compress(xt, got_cfg, stream=st)
        y = binding.decompress(s, stream=st)
    st.synchronize()
    for k in ("predictor", "frozen_dim", "levels", "cand"):
        assert got_cfg[k] == ref_cfg[k], k
    assert np.array_equal(got_cfg["block_cfg"], ref_cfg["block_cfg"])
    ref = O.compress(x, ref_cfg)
    assert s.cpu().numpy().tobytes() == ref
    assert np.array_equal(y.cpu().numpy().view(np.uint8), O.decompress(ref).view(np.uint8))


MDSL_SHAPES = [(1000,), (257, 129), (37, 70, 129), (9, 17, 33, 5)]


@pytest.mark.parametrize("shape", MDSL_SHAPES, ids=["x".join(map(str, s)) for s in MDSL_SHAPES])
def test_md_same_level_global(torch_cuda, shape):
    """Same-level cubic inside multi-dimensional sub-steps (Sec. 5.4.2): the
    global step kernels on 1-4-D ragged grids."""
    x = fields.random_field(shape, len(shape) * 3 + 1, np.float32, "mixed")
    for kind in ("nak", "nat"):
        cfg = make_cfg(shape, eb=1e-3, kind=kind, md=1, same_level=1)
        roundtrip(torch_cuda, x, cfg, f"md+sl {shape} {kind}")


MDSL_BLOCK = [((64, 64, 64), "f32", 32), ((70, 66, 97), "f32", 32), ((70, 66, 97), "f64", 32),
              ((45, 38, 41), "f32", 8), ((200, 161), "f32", 32)]


@pytest.mark.parametrize("shape,dt,B", MDSL_BLOCK,
                         ids=["x".join(map(str, s)) + f"-{d}-B{b}" for s, d, b in MDSL_BLOCK])
def test_md_same_level_blocks(torch_cuda, shape, dt, B):
    """Same-level MD on every block path: the face steps and planes (global
    level configuration), the coarse block lattice, the full-block schedule
    (float32 32^3 bricks), the row-major box (float64, partial bricks) and the
    generic per-level block steps (B = 8)."""
    nd = len(shape)
    cand = candidates(nd) + [interp("nak", 1, 1, ndims=nd), interp("nat", 1, 1, ndims=nd)]
    nb = int(np.prod([(s + B - 1) // B for s in shape]))
    bc = np.random.default_rng(nb).integers(0, len(cand), nb).astype(np.uint8)
    x = fields.random_field(shape, nb, np.float32 if dt == "f32" else np.float64, "mixed")
    al = 6 if nd >= 3 else 7
    if B == 8:
        al = 4
    cfg = make_cfg(shape, dtype=dt, eb=1e-3, kind="nat", md=1, same_level=1, anchor_log2=al,
                   block_log2=int(np.log2(B)), cand=cand, block_cfg=bc)
    roundtrip(torch_cuda, x, cfg, f"md+sl blocks {shape} {dt} B={B}")
