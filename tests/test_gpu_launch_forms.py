"""The launch structure of an iteration depends on the batch: the
projection and w passes share a launch up to 8M grid points, and a batch
whose threshold pipelines all have at most 2^19 entries runs one refine pass
instead of two.  Neither changes any arithmetic, so an instance's iterates
are bit-identical whatever batch it runs in."""
import numpy as np
import pytest

from paper_1902_09699_amd import sip
from paper_1902_09699_amd import workloads as wl
from tests.gpu_util import make_case

pytestmark = pytest.mark.gpu


def _run(instances, opts, iters, tiles):
    import torch
    ws = sum(sip.workspace_bytes(m.shape, s, opts) for m, s in instances)
    b = sip.Batch(len(instances), ws, opts)
    b.set_tiles(*tiles)
    xs = []
    for m, s in instances:
        md = torch.tensor(m, dtype=torch.float32, device="cuda")
        x = torch.empty_like(md)
        b.add(md, s, x)
        xs.append((md, x))
    b.run(iters)
    out = xs[0][1].cpu().numpy().copy()
    b.close()
    return out


@pytest.mark.parametrize("form", [0, 1, 2])
def test_same_iterates_in_small_and_large_batches(form):
    m, sets = make_case("four_sets_2d", 3)
    m = wl.rounded(m, "f32")
    sets = wl.finalize(m, sets)
    # a 3000 x 3000 filler: 9M points (passes launched apart) and a
    # cardinality pipeline of ~9M entries (two refine passes)
    rng = wl.rng_for(77)
    big = wl.rounded(wl.grf((3000, 3000), 6.0, rng), "f32")
    big_sets = wl.finalize(big, [wl.bounds("I", -1.0, 1.0), wl.card("DX", 0.05)])
    opts = sip.make_opts("f32", max_iter=6, cg_max=10, cg_fixed=1)
    tiles = (1024, 1024, 2048, 512, 256, form)
    print(f"\n[launch forms] cg_form={form}: {m.shape} alone and beside {big.shape}", flush=True)
    alone = _run([(m, sets)], opts, 6, tiles)
    mixed = _run([(m, sets), (big, big_sets)], opts, 6, tiles)
    assert np.array_equal(alone, mixed)


@pytest.mark.parametrize("kind", ["3d", "wide_rows"])
def test_lds_staged_form_falls_back_to_the_textbook_steps(kind):
    """Under cg_form 2, an instance the LDS-staged step cannot take (a 3D
    grid, or rows too long for a block's LDS with three halo rows) runs the
    two-launch textbook steps: its iterates equal those under cg_form 0 bit
    for bit, and differ from the one-reduction form's."""
    rng = wl.rng_for(91)
    if kind == "3d":
        m = wl.grf((24, 20, 18), 4.0, rng)
        sets = [wl.bounds("I", -1.0, 1.0), wl.l1("GRAD", 0.5)]
    else:
        m = wl.grf((8, 6000), 8.0, rng)
        sets = [wl.bounds("I", -1.0, 1.0), wl.card("DX", 0.2)]
    m = wl.rounded(m, "f32")
    sets = wl.finalize(m, sets)
    opts = sip.make_opts("f32", max_iter=5, cg_max=10, cg_fixed=1)
    print(f"\n[launch forms] {kind} {m.shape}: cg_form 2 against 0", flush=True)
    f2 = _run([(m, sets)], opts, 5, (2048, 512, 2048, 512, 256, 2))
    f0 = _run([(m, sets)], opts, 5, (2048, 512, 2048, 512, 256, 0))
    f1 = _run([(m, sets)], opts, 5, (2048, 512, 2048, 512, 256, 1))
    assert np.array_equal(f2, f0)
    assert not np.array_equal(f1, f0)
