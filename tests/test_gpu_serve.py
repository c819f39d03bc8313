"""Served form on the GPU: continuous batching admits requests as slots and
arena bytes free up, never exceeds the arena, and every result equals the
same request projected alone."""
import numpy as np
import pytest

from paper_1902_09699_amd import serve, sip

pytestmark = pytest.mark.gpu


def _small_mix(n):
    return serve.make_requests(n, rate=1e9, frac3d=0.25, seed0=5000, max2d=96, side3d=(12, 20))


@pytest.mark.parametrize("chunk,lanes", [(5, 1), (10, 1), (7, 1), (5, 2), (10, 2)])
def test_served_results_equal_alone_and_respect_the_arena(chunk, lanes):
    """With two lanes the small requests (at most 5000 points here) and the
    large ones run in two resident batches on two streams."""
    import torch
    opts = serve.serving_opts(max_iter=60)
    reqs = _small_mix(14)
    need = [sip.workspace_bytes(r.m.shape, r.sets, opts) for r in reqs]
    arena = 3 * max(need) * lanes  # forces queueing: at most a few fit at once (per lane)
    srv = serve.Server(opts, arena, max_slots=4, chunk=chunk, lanes=lanes, split_points=5000)
    info = srv.run(reqs, realtime=False)
    srv.close()
    if lanes == 2:
        assert any(r.m.size <= 5000 for r in reqs) and any(r.m.size > 5000 for r in reqs)
    print(f"\n[serve] chunk {chunk}, lanes {lanes}: peak arena {info['peak_arena_bytes']} of {arena}, "
          f"chunks {info['chunks']}", flush=True)
    assert info["rejected"] == 0
    assert info["peak_arena_bytes"] <= arena
    assert all(r.result is not None and r.result["status"] == 0 for r in reqs)
    assert any(r.result["converged"] for r in reqs)
    for r in reqs:
        md = torch.tensor(r.m, dtype=torch.float32, device="cuda")
        x, res = sip.project(md, r.sets, opts)
        assert np.array_equal(x.cpu().numpy(), r.x), r.rid
        assert res["iters"] == r.result["iters"]


def test_oversized_request_is_rejected_not_hung():
    opts = serve.serving_opts(max_iter=10)
    reqs = _small_mix(3)
    need = max(sip.workspace_bytes(r.m.shape, r.sets, opts) for r in reqs)
    srv = serve.Server(opts, need // 4, max_slots=2, chunk=5)
    info = srv.run(reqs, realtime=False)
    srv.close()
    assert info["rejected"] >= 1


@pytest.mark.parametrize("tiles", [(1024, 512, 1024, 512, 256, 2), (1024, 512, 1024, 512, 512, 1)])
def test_served_results_under_other_tiles_equal_a_plan(tiles):
    """Lanes under fixed tiles (the LDS-staged CG form, whose 2D requests run
    the one-launch steps and 3D ones the textbook steps beside them, and the
    one-reduction form): every result equals a plan of the same tiles run
    alone."""
    import torch
    opts = serve.serving_opts(max_iter=60)
    reqs = _small_mix(10)
    need = [sip.workspace_bytes(r.m.shape, r.sets, opts) for r in reqs]
    srv = serve.Server(opts, 4 * max(need) * 2, max_slots=4, chunk=5, lanes=2, split_points=5000, tiles=tiles)
    info = srv.run(reqs, realtime=False)
    srv.close()
    print(f"\n[serve] tiles {tiles}: chunks {info['chunks']}", flush=True)
    assert info["rejected"] == 0
    assert any(r.m.ndim == 3 for r in reqs) and any(r.m.ndim == 2 for r in reqs)
    for r in reqs:
        assert r.result is not None and r.result["status"] == 0
        md = torch.tensor(r.m, dtype=torch.float32, device="cuda")
        plan = sip.Plan(r.m.shape, r.sets, opts, tiles=tiles)
        x, res = plan.project(md)
        plan.close()
        assert np.array_equal(x.cpu().numpy(), r.x), r.rid
        assert res["iters"] == r.result["iters"]
