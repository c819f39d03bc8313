"""Parity at the benchmark sizes (341x1361 float32 with four sets, 200x200x100
float32 with three sets, the 256-instance uneven batch): lockstep iterations
against the FP64 oracle in the tile configurations the benchmark uses,
covering an adapt iteration (k = 3, the first with a snapshot) and every
state array; plus properties of a complete benchmark-length run that hold at
any size."""
import numpy as np
import pytest

from oracle import parsdmm as orc
from paper_1902_09699_amd import sip
from paper_1902_09699_amd import workloads as wl
from tests.gpu_util import Slot, SlotView, compare_step, rounding_spread, sync_oracle

pytestmark = pytest.mark.gpu

TILES = {"default": (2048, 512, 2048, 512, 512), "tuned": (1024, 256, 2048, 256, 512),
         "small_blocks": (2048, 1024, 4096, 512, 256), "one_reduction": (1024, 512, 2048, 512, 512, 1),
         "one_reduction_256": (1024, 1024, 2048, 512, 256, 1),
         "thr_items_1024": (2048, 512, 2048, 1024, 512)}


def _load(name):
    if name == "layered2d":
        m, sets, field, iters = wl.layered2d_four_sets()
    else:
        m, sets, field, iters = wl.smooth3d_box_tv_lat()
    m = wl.rounded(m, field)
    return m, wl.finalize(m, sets), field, iters


@pytest.mark.parametrize("name,tiles", [("layered2d", "default"), ("layered2d", "tuned"), ("layered2d", "small_blocks"),
                                        ("layered2d", "one_reduction"), ("layered2d", "one_reduction_256"),
                                        ("smooth3d", "tuned"), ("smooth3d", "small_blocks"),
                                        ("smooth3d", "one_reduction"), ("smooth3d", "thr_items_1024")])
def test_fullsize_lockstep(name, tiles):
    m, sets, field, iters = _load(name)
    print(f"\n[fullsize] {name} {m.shape} tiles={TILES[tiles]}", flush=True)
    sl = Slot(m, sets, field, dict(max_iter=iters, cg_max=10, cg_fixed=1), tiles=TILES[tiles])
    prob = orc.Problem(m, m.shape, sets)
    oo = orc.Options(max_iter=iters, cg_max=10, cg_fixed=True)
    st = orc.initial_state(prob, oo)
    for it in range(3):
        sync_oracle(sl, prob, st)
        spread = rounding_spread(prob, st, oo, field)
        orc.iterate(prob, st, oo)
        sl.batch.run(1)
        worst, ratio = compare_step(sl, prob, st, spread, 1e-5, label=(name, it + 1))
        print(f"[fullsize] {name} iteration {it + 1}: worst rel err {worst:.2e}, worst err / x-rounding spread "
              f"{ratio:.1f}", flush=True)


def test_fullsize_run_properties():
    """A complete 341x1361 run: status, iteration and CG-step counts, and the
    final y of every set lies in its set (the projections are exact)."""
    m, sets, field, iters = _load("layered2d")
    sl = Slot(m, sets, field, dict(max_iter=iters, cg_max=10, cg_fixed=1), tiles=TILES["tuned"])
    sl.batch.run(iters)
    res = sl.batch.result(sl.slot)
    assert res["status"] == 0 and res["iters"] == iters and 10 * (iters - 1) <= res["cg_steps"] <= 10 * iters
    y_box = sl.arr(sip.FIELD_Y, 0)
    assert y_box.min() >= 1.5 and y_box.max() <= 4.5
    y_mono = sl.arr(sip.FIELD_Y, 1)
    assert y_mono.min() >= 0.0
    y_l1 = sl.arr(sip.FIELD_Y, 2)
    assert np.abs(y_l1).sum() <= sets[2]["tau"] * (1 + 1e-5)
    y_card = sl.arr(sip.FIELD_Y, 3)
    assert (y_card != 0).sum() <= sets[3]["k"]
    # x approaches the intersection: transform-domain infeasibility is small
    x = sl.x()
    prob = orc.Problem(m, m.shape, sets)
    print(f"\n[fullsize] rho {np.round(res['rho'], 3)}, box violation "
          f"{max(0.0, 1.5 - x.min(), x.max() - 4.5):.2e}", flush=True)
    assert np.abs(prob.A[2] @ x).sum() <= 1.05 * sets[2]["tau"]


# The tiles the autotuner picks for the 256-instance batch on an MI355X: 2048-
# point CG items (at most 1024 per instance), 4096-point threshold items (at
# most 512), 256-thread blocks, the LDS-staged CG form.
BATCH_TILES = (2048, 1024, 4096, 512, 256, 2)


def _kind(sets):
    ks = set()
    for s in sets:
        if s["kind"] == "l1":
            ks.add("tv" if s["op"] == "GRAD" else "l1")
        elif s["kind"] == "card":
            ks.add("card")
    return ks


def test_full_batch_lockstep():
    """The whole 256-instance batch in the benchmark's launch configuration:
    sampled instances (a TV ball, another l1 ball, a cardinality set, the
    largest instance) in lockstep with the oracle for three iterations."""
    import torch
    insts = []
    for m, sets in wl.batched_instances(256):
        m = wl.rounded(m, "f32")
        insts.append((m, wl.finalize(m, sets)))
    picks = []
    for want in ("tv", "l1", "card"):
        picks.append(next(j for j, (_, s) in enumerate(insts) if want in _kind(s) and j not in picks))
    picks.append(max((j for j in range(len(insts)) if j not in picks), key=lambda j: insts[j][0].size))
    opts = sip.make_opts("f32", max_iter=200, cg_max=10, cg_fixed=1)
    arena = sum(sip.workspace_bytes(m.shape, s, opts) for m, s in insts)
    b = sip.Batch(len(insts), arena, opts)
    b.set_tiles(*BATCH_TILES)
    views = {}
    for j, (m, s) in enumerate(insts):
        md = torch.tensor(m, dtype=torch.float32, device="cuda")
        xd = torch.empty_like(md)
        sl = b.add(md, s, xd)
        if j in picks:
            views[j] = SlotView(b, sl, m, s, "f32", md, xd)
    print(f"\n[fullsize] batch of {len(insts)} ({sum(m.size for m, _ in insts)} points), tiles {BATCH_TILES}, "
          f"checked {[(j, insts[j][0].shape) for j in picks]}", flush=True)
    oo = orc.Options(max_iter=200, cg_max=10, cg_fixed=True)
    probs = {j: orc.Problem(insts[j][0], insts[j][0].shape, insts[j][1]) for j in picks}
    states = {j: orc.initial_state(probs[j], oo) for j in picks}
    for it in range(3):
        spreads = {}
        for j in picks:
            sync_oracle(views[j], probs[j], states[j])
            spreads[j] = rounding_spread(probs[j], states[j], oo, "f32")
            orc.iterate(probs[j], states[j], oo)
        b.run(1)
        torch.cuda.synchronize()
        for j in picks:
            worst, ratio = compare_step(views[j], probs[j], states[j], spreads[j], 1e-5, label=(j, it + 1))
            print(f"[fullsize] batch instance {j} iteration {it + 1}: worst rel err {worst:.2e}, "
                  f"worst err / x-rounding spread {ratio:.1f}", flush=True)
    b.close()
