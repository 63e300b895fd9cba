"""GPU test of the serving loop with the library backend: requests of
different kinds, sizes and dtypes arrive while others run on several slots
(streams); every served result must equal the same request run alone through
the plain calls (streams byte for byte, reconstructions bit for bit), and a
request that the library rejects (workspace cap) fails alone while the server
keeps serving."""
from __future__ import annotations

import numpy as np
import pytest

from cfgs import make_cfg
from paper_2311_12133_amd import fields

pytestmark = pytest.mark.gpu

TUNE = dict(global_rate=0.05, sub_rate=0.04, block_log2=5)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_12133_amd import binding
    binding.lib()
    return torch


def make_requests(torch, n_comp=16, seed=7):
    from paper_2311_12133_amd import binding
    from paper_2311_12133_amd.serve import Request
    rng = np.random.default_rng(seed)
    shapes = [(64, 64, 64), (37, 70, 129), (100, 80), (5000,), (33, 65, 40), (9, 17, 33, 5),
              (96, 64, 70), (300, 257)]
    reqs, alone = [], []
    t = 0.0
    for i in range(n_comp):
        sh = shapes[i % len(shapes)]
        dt = np.float64 if i % 5 == 4 else np.float32
        x = fields.random_field(sh, 300 + i, dt, "smooth" if i % 3 else "mixed")
        xt = torch.from_numpy(x).cuda()
        cfg = make_cfg(sh, dtype="f64" if dt == np.float64 else "f32",
                       eb=float(10 ** rng.uniform(-5, -2)))
        tune = i % 2 == 0
        t += float(rng.exponential(0.002))
        reqs.append(Request(rid=len(reqs), op="compress", arrival=t, data=xt, cfg=cfg, tune=tune,
                            tune_opts=TUNE if tune else None))
        c = binding.tune(xt, cfg, TUNE) if tune else cfg
        s = binding.compress(xt, c)
        alone.append(s.cpu().numpy().tobytes())
        # a decompression of this stream, arriving later
        t2 = t + float(rng.exponential(0.002))
        r = Request(rid=len(reqs) + 1, op="decompress", arrival=t2, data=s.clone(), cfg=c)
        r.out_shape = tuple(sh)
        r.out_dtype = xt.dtype
        reqs.append(None)
        reqs.append(r)
        alone.append(None)
        alone.append(binding.decompress(s).cpu().numpy())
    torch.cuda.synchronize()
    keep = [(r, a) for r, a in zip(reqs, alone) if r is not None]
    for k, (r, _) in enumerate(keep):
        r.rid = k
    return [r for r, _ in keep], [a for _, a in keep]


def test_served_equals_alone(torch_cuda):
    from paper_2311_12133_amd.serve import Server
    print("[case] serve mix, 4 slots", flush=True)
    reqs, alone = make_requests(torch_cuda)
    srv = Server(device=0, slots=4, hbm_budget=8 << 30, max_batch=4)
    try:
        st = srv.run(reqs)
    finally:
        srv.close()
    torch_cuda.cuda.synchronize()
    assert st["completed"] == len(reqs), st
    for r, a in zip(reqs, alone):
        assert r.error == 0, (r.rid, r.error)
        got = r.result.cpu().numpy()
        if r.op == "compress":
            assert got.tobytes() == a, f"request {r.rid}: stream differs from the plain call's"
        else:
            assert np.array_equal(got.view(np.uint8), a.view(np.uint8)), f"request {r.rid}"
    assert st["mean_batch"] >= 1 and st["p50_ms"] <= st["p99_ms"]


def test_small_budget_still_serves_everything(torch_cuda):
    from paper_2311_12133_amd.serve import Server
    print("[case] serve with a budget of about two requests", flush=True)
    reqs, alone = make_requests(torch_cuda, n_comp=6, seed=11)
    srv = Server(device=0, slots=3, hbm_budget=1, max_batch=4, keep_bytes=0)
    for r in reqs:
        srv.backend.prepare(r)
    srv.budget = 2 * max(r.mem for r in reqs)
    try:
        st = srv.run(reqs)
    finally:
        srv.close()
    assert st["completed"] == len(reqs)
    for r, a in zip(reqs, alone):
        got = r.result.cpu().numpy()
        if r.op == "compress":
            assert got.tobytes() == a
        else:
            assert np.array_equal(got.view(np.uint8), a.view(np.uint8))


def test_rejected_request_fails_alone(torch_cuda):
    from paper_2311_12133_amd.serve import Request, Server
    print("[case] serve with a workspace cap", flush=True)
    small = torch_cuda.from_numpy(fields.random_field((40, 40, 40), 1, np.float32)).cuda()
    big = torch_cuda.from_numpy(fields.random_field((160, 160, 160), 2, np.float32)).cuda()
    cs = make_cfg(small.shape)
    cb = make_cfg(big.shape)
    srv = Server(device=0, slots=1, hbm_budget=8 << 30, max_batch=1)
    # the slot's context can hold the small field's workspace only
    from paper_2311_12133_amd import binding
    lim = binding.footprint(tuple(small.shape), "f32", cs, "compress") * 2
    srv.slots[0]["ctx"].set_limit(lim)
    reqs = [Request(rid=0, op="compress", arrival=0.0, data=small, cfg=cs),
            Request(rid=1, op="compress", arrival=0.001, data=big, cfg=cb),
            Request(rid=2, op="compress", arrival=0.002, data=small, cfg=cs)]
    try:
        srv.run(reqs)
    finally:
        srv.close()
    assert reqs[1].error == -2
    ref = binding.compress(small, cs).cpu().numpy().tobytes()
    for k in (0, 2):
        assert reqs[k].error == 0
        assert reqs[k].result.cpu().numpy().tobytes() == ref
