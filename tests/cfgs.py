"""Neutral configuration dicts shared by the oracle binding and the library
binding in the tests (plain data, no arithmetic of the method)."""
from __future__ import annotations

KINDS = {"lin": 0, "nak": 1, "nat": 2}


def interp(kind="lin", md=False, same_level=False, order=None, ndims=3):
    if order is None:
        order = tuple(range(ndims))
    order = tuple(j for j in order if j < ndims)
    order = order + tuple(j for j in range(4) if j not in order)
    return dict(kind=KINDS[kind] if isinstance(kind, str) else int(kind), md=int(bool(md)),
                same_level=int(bool(same_level)), order=order)


def default_anchor_log2(shape):
    big = sum(1 for s in shape if s > 1)
    return 6 if big >= 3 else 7 if big == 2 else 8


def make_cfg(shape, dtype="f32", eb=1e-3, eb_mode="rel", kind="lin", md=False,
             same_level=False, order=None, anchor_log2=None, frozen_dim=-1, block_log2=0,
             radius=32768, chunk=1024, alpha=1.0, beta=1.0, md_w=None, levels=None,
             cand=None, block_cfg=None, predictor="interp"):
    nd = len(shape)
    if levels is None:
        levels = [interp(kind, md, same_level, order, nd)] * 16
    return dict(dtype=dtype, dims=tuple(int(s) for s in shape), eb=eb, eb_mode=eb_mode,
                predictor=predictor,
                anchor_log2=default_anchor_log2(shape) if anchor_log2 is None else anchor_log2,
                frozen_dim=frozen_dim, block_log2=block_log2, radius=radius, chunk=chunk,
                alpha=alpha, beta=beta, md_w=md_w or [[1.0] * 4 for _ in range(3)],
                levels=list(levels), cand=list(cand or []), block_cfg=block_cfg)


def candidates(ndims):
    """The eleven interpolation candidates, in index order (see the tuner)."""
    out = []
    for i in range(11):
        if i < 9:
            kind, par = i // 3, i % 3
            sl = 0
        else:
            kind, par, sl = (1 if i == 9 else 2), 0, 1
        order = tuple(range(ndims)) if par != 1 else tuple(reversed(range(ndims)))
        out.append(interp(kind, par == 2, sl, order, ndims))
    return out
