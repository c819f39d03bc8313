"""Plans through the C ABI (the paper's set-up-once / project-many sequence):
a plan gives the projection of sip_project (bitwise for float fields), is
reused across models without new set-up, runs from a caller workspace, and
its exported state, imported into another plan, continues exactly as the
uninterrupted run."""
import numpy as np
import pytest

from paper_1902_09699_amd import sip
from paper_1902_09699_amd import workloads as wl
from tests.gpu_util import make_case

pytestmark = pytest.mark.gpu


def _case(kind, field, seed=0):
    m, sets = make_case(kind, seed)
    m = wl.rounded(m, field)
    return m, wl.finalize(m, sets)


def _dev(m, field):
    import torch
    return torch.tensor(m, dtype=torch.float64 if field == "f64" else torch.float32, device="cuda")


# Float fields are bit-reproducible; double fields sum the l1 radix buckets
# with double atomics, whose order (so the last bits) varies run to run.
F64_TOL = 1e-10


def _eq(a, b, field):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    if field == "f32":
        assert np.array_equal(a, b)
    else:
        assert np.linalg.norm(a - b) <= F64_TOL * max(np.linalg.norm(b), 1e-300)


def _same(ra, rb, field="f32"):
    for key in ("status", "iters", "cg_steps", "converged"):
        assert ra[key] == rb[key], (key, ra[key], rb[key])
    for key in ("r_evol", "r_feas", "rho", "gamma"):
        if field == "f32":
            assert ra[key] == rb[key], (key, ra[key], rb[key])
        else:
            np.testing.assert_allclose(ra[key], rb[key], rtol=1e-7, atol=0)


CASES = [("box_tv_2d", "f64", {}), ("four_sets_2d", "f32", {}), ("mixed_3d", "f32", {}),
         ("mixed_2d", "f32", dict(stop_every=5, cg_fixed=0))]


@pytest.mark.parametrize("kind,field,extra", CASES)
def test_plan_equals_sip_project(kind, field, extra):
    m, sets = _case(kind, field)
    opts = sip.make_opts(field, max_iter=40, cg_max=10, cg_fixed=extra.get("cg_fixed", 1),
                         stop_every=extra.get("stop_every", 0))
    print(f"\n[plan] {kind} {field} {m.shape} {extra}", flush=True)
    md = _dev(m, field)
    xr, rr = sip.project(md, sets, opts)
    plan = sip.Plan(m.shape, sets, opts)
    xp, rp = plan.project(md)
    _eq(xp.cpu().numpy(), xr.cpu().numpy(), field)
    _same(rp, rr, field)
    plan.close()


def test_plan_reused_across_models():
    """One plan, three models of the same grid: each result equals a fresh
    sip_project; x may alias m."""
    field = "f32"
    shape = (41, 67)
    opts = sip.make_opts(field, max_iter=30, cg_max=10, cg_fixed=1)
    base = None
    plan = None
    for seed in (0, 1, 2):
        m, sets, _, _ = wl.layered2d_four_sets(n=shape, seed=100 + seed)
        m = wl.rounded(m, field)
        if base is None:
            base = wl.finalize(m, sets)
            plan = sip.Plan(shape, base, opts)
        md = _dev(m, field)
        xr, rr = sip.project(md, base, opts)
        xp, rp = plan.project(md)
        assert np.array_equal(xp.cpu().numpy(), xr.cpu().numpy()), seed
        _same(rp, rr)
        # in place: x is m's own buffer
        mi = _dev(m, field)
        xi, ri = plan.project(mi, x=mi)
        assert np.array_equal(xi.cpu().numpy(), xr.cpu().numpy()), seed
    plan.close()


def test_plan_in_caller_workspace():
    import torch
    m, sets = _case("mixed_2d", "f32")
    opts = sip.make_opts("f32", max_iter=30, cg_max=10, cg_fixed=1)
    tiles = (1024, 512, 1024, 512, 256, 1)
    need = sip.plan_bytes(m.shape, sets, opts, tiles)
    assert need >= sip.workspace_bytes(m.shape, sets, opts)
    ws = torch.full((need + 4096,), 0xAB, dtype=torch.uint8, device="cuda")  # stale contents
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(sip.SipError) as e:
        sip.Plan(m.shape, sets, opts, tiles, workspace=small)
    assert e.value.status == sip.EBUDGET
    with pytest.raises(sip.SipError) as e:
        sip.Plan(m.shape, sets, opts, tiles, workspace=ws[16:])
    assert e.value.status == sip.EINVAL
    md = _dev(m, "f32")
    own = sip.Plan(m.shape, sets, opts, tiles)
    xo, ro = own.project(md)
    borrowed = sip.Plan(m.shape, sets, opts, tiles, workspace=ws)
    for _ in range(2):
        xb, rb = borrowed.project(md)
        assert np.array_equal(xb.cpu().numpy(), xo.cpu().numpy())
        _same(rb, ro)
    # the plan wrote nothing past its workspace size
    assert bool((ws[need:] == 0xAB).all())
    own.close()
    borrowed.close()


@pytest.mark.parametrize("kind,field,extra", [
    ("four_sets_2d", "f32", {}), ("box_tv_lat_3d", "f64", {}),
    ("mixed_2d", "f32", dict(stop_every=5, cg_fixed=0)), ("mixed_3d", "f32", dict(stop_every=5, cg_fixed=0)),
])
def test_state_export_import_continues_exactly(kind, field, extra):
    """Run 7 iterations, export, run 16 more; a second plan started from a
    different model imports the blob and runs 16: the same x and result
    (bitwise for float fields).  The first plan, re-imported, repeats them
    too."""
    m, sets = _case(kind, field)
    kw = dict(max_iter=60, cg_max=10, cg_fixed=extra.get("cg_fixed", 1), stop_every=extra.get("stop_every", 0),
              log_schedule=1)
    opts = sip.make_opts(field, **kw)
    print(f"\n[state] {kind} {field} {extra}", flush=True)
    a = sip.Plan(m.shape, sets, opts)
    xa = a.start(_dev(m, field))
    a.iterate(7)
    blob = a.export_state()
    assert blob.numel() == a.state_bytes()
    a.iterate(16)
    ra = a.result()
    xa_end = xa.cpu().numpy().copy()
    m2, _ = _case(kind, field, seed=5)
    b = sip.Plan(m.shape, sets, opts)
    xb = b.start(_dev(m2, field))
    b.iterate(3)
    b.import_state(blob)
    b.iterate(16)
    rb = b.result()
    _eq(xb.cpu().numpy(), xa_end, field)
    _same(rb, ra, field)
    a.import_state(blob)
    a.iterate(16)
    _eq(xa.cpu().numpy(), xa_end, field)
    _same(a.result(), ra, field)
    a.close()
    b.close()


def test_state_import_rejects_another_layout():
    m, sets = _case("four_sets_2d", "f32")
    opts = sip.make_opts("f32", max_iter=10, cg_max=10, cg_fixed=1)
    a = sip.Plan(m.shape, sets, opts)
    a.start(_dev(m, "f32"))
    blob = a.export_state()
    m3, sets3 = _case("mixed_2d", "f32")
    c = sip.Plan(m3.shape, sets3, opts)
    c.start(_dev(m3, "f32"))
    with pytest.raises(sip.SipError) as e:
        c.import_state(blob)
    assert e.value.status == sip.EINVAL
    a.close()
    c.close()
