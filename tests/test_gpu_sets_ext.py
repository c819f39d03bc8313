"""The l2 ball, the annulus and per-pixel bound vectors on the device against
the oracle, through the C ABI: step parity (lockstep), schedule-locked end to
end, the annulus at w = 0, and the multilevel transfer of an l2 radius."""
import numpy as np
import pytest

from oracle import multilevel as ml
from oracle import parsdmm as orc
from paper_1902_09699_amd import sip
from paper_1902_09699_amd import workloads as wl
from tests.gpu_util import Slot, pad, rel, sync_oracle

pytestmark = pytest.mark.gpu


def _case(kind, field):
    """(m, sets for the device, sets for the oracle)."""
    import torch
    rng = np.random.default_rng({"l2_grad": 1, "annulus_i": 2, "vec_bounds": 3, "mixed3d": 4}[kind])
    if kind == "l2_grad":
        m = wl.grf((33, 47), 5.0, rng)
        g = np.linalg.norm(orc.operator("GRAD", m.shape, (1.0, 1.0)) @ m.ravel())
        sets = [{"kind": "l2", "op": "GRAD", "tau": 0.4 * g}, {"kind": "bounds", "op": "I", "lo": -1.5, "hi": 1.5}]
        return m, sets, sets
    if kind == "annulus_i":
        m = wl.grf((29, 35), 4.0, rng)
        nm = np.linalg.norm(m)
        sets = [{"kind": "annulus", "op": "I", "lo": 1.3 * nm, "hi": 1.6 * nm},
                {"kind": "l1", "op": "DX", "tau": 0.5 * np.abs(orc.operator("DX", m.shape, (1.0, 1.0)) @ m.ravel()).sum()}]
        return m, sets, sets
    if kind == "vec_bounds":
        shape = (31, 44)
        m = wl.grf(shape, 4.0, rng)
        dt = torch.float64 if field == "f64" else torch.float32
        nz = shape[0]
        # depth-varying lower bound on D_z (a graded monotonicity) and a
        # box whose width varies along x
        lo_dz = np.repeat(np.linspace(-0.2, 0.05, nz - 1)[:, None], shape[1], axis=1).ravel()
        box_hi = np.tile(np.linspace(0.5, 1.5, shape[1]), shape[0])
        box_lo = -box_hi
        if field == "f32":
            lo_dz, box_lo, box_hi = (wl.rounded(a, "f32") for a in (lo_dz, box_lo, box_hi))
        dev = [{"kind": "bounds", "op": "DZ", "lo": 0.0, "hi": np.inf,
                "lo_vec": torch.tensor(pad(shape, "DZ", lo_dz), dtype=dt, device="cuda")},
               {"kind": "bounds", "op": "I", "lo": 0.0, "hi": 0.0,
                "lo_vec": torch.tensor(box_lo, dtype=dt, device="cuda"),
                "hi_vec": torch.tensor(box_hi, dtype=dt, device="cuda")}]
        orcs = [{"kind": "bounds", "op": "DZ", "lo": lo_dz, "hi": np.full(lo_dz.size, np.inf)},
                {"kind": "bounds", "op": "I", "lo": box_lo, "hi": box_hi}]
        return m, dev, orcs
    m = wl.grf((9, 12, 14), 3.0, rng)
    a = orc.operator("LAT", m.shape, (1.0, 1.0, 1.0)) @ m.ravel()
    sets = [{"kind": "l2", "op": "LAT", "tau": 0.5 * np.linalg.norm(a)},
            {"kind": "annulus", "op": "DZ", "lo": 0.0,
             "hi": 0.7 * np.linalg.norm(orc.operator("DZ", m.shape, (1.0, 1.0, 1.0)) @ m.ravel())},
            {"kind": "bounds", "op": "I", "lo": -1.0, "hi": 1.0}]
    return m, sets, sets


CASES = [("l2_grad", "f64"), ("l2_grad", "f32"), ("annulus_i", "f64"), ("annulus_i", "f32"),
         ("vec_bounds", "f64"), ("vec_bounds", "f32"), ("mixed3d", "f64"), ("mixed3d", "f32")]


@pytest.mark.parametrize("kind,field", CASES)
def test_step_parity_new_sets(kind, field):
    m, dev, orcs = _case(kind, field)
    m = wl.rounded(m, field)
    print(f"\n[sets ext step] {kind} {field} {m.shape}", flush=True)
    sl = Slot(m, dev, field, dict(max_iter=50, cg_max=10, cg_fixed=1), tiles=(1024, 1024, 1024, 512, 256))
    prob = orc.Problem(m, m.shape, orcs)
    oo = orc.Options(max_iter=50, cg_max=10, cg_fixed=True)
    st = orc.initial_state(prob, oo)
    tol = 1e-10 if field == "f64" else 1e-5
    worst = 0.0
    for it in range(9):
        sync_oracle(sl, prob, st)
        orc.iterate(prob, st, oo)
        sl.batch.run(1)
        worst = max(worst, rel(sl.x(), st.x))
        for i in range(len(dev) + 1):
            yo, vo = st.y[i], st.v[i]
            op = "I" if i == len(dev) else dev[i]["op"]
            anorm = 1.0 if op == "I" else 2.0 * np.sqrt(2.0)
            scale = max(np.linalg.norm(yo), np.linalg.norm(st.w_last[i]), anorm * np.linalg.norm(st.x))
            ey = np.linalg.norm(sl.arr(sip.FIELD_Y, i) - yo) / scale
            ev = np.linalg.norm(sl.arr(sip.FIELD_V, i) - vo) / max(np.linalg.norm(vo), scale)
            worst = max(worst, ey, ev)
            assert ey <= tol and ev <= 10 * tol, (it, i, ey, ev)
        rho, gam, kg, _ = sl.batch.get_params(sl.slot)
        assert kg == st.k
        if field == "f64":  # float32 spectral estimates (ratios of dots of differences) carry ~1e-6..1e-5
            np.testing.assert_allclose(rho, st.rho, rtol=1e-8)
            np.testing.assert_allclose(gam, st.gamma, rtol=1e-8)
    print(f"[sets ext step] {kind} {field}: worst {worst:.2e}", flush=True)


@pytest.mark.parametrize("kind", ["l2_grad", "annulus_i", "vec_bounds", "mixed3d"])
def test_schedule_locked_f64_new_sets(kind):
    m, dev, orcs = _case(kind, "f64")
    iters = 40
    sl = Slot(m, dev, "f64", dict(max_iter=iters, cg_max=10, cg_fixed=1, log_schedule=1))
    sl.batch.run(iters)
    assert sl.batch.result(sl.slot)["status"] == 0
    rho, gam = sl.batch.schedule(sl.slot, iters)
    xo, _ = orc.parsdmm(m, m.shape, orcs, orc.Options(max_iter=iters, cg_max=10, cg_fixed=True),
                        schedule={k + 1: (rho[k], gam[k]) for k in range(iters)})
    err = rel(sl.x(), xo)
    print(f"\n[sets ext locked] {kind}: rel err {err:.2e}", flush=True)
    assert err <= 1e-9


def test_annulus_at_zero_takes_the_first_row():
    """m = 0 and an annulus on I with lo > 0: w = 0 on the first iteration,
    so y = lo e_0; device and oracle agree over the run."""
    shape = (6, 7)
    m = np.zeros(shape)
    sets = [{"kind": "annulus", "op": "I", "lo": 0.8, "hi": 1.2}]
    sl = Slot(m, sets, "f64", dict(max_iter=15, cg_max=10, cg_fixed=1, log_schedule=1))
    sl.batch.run(1)
    y = sl.arr(sip.FIELD_Y, 0)
    assert y[0] == 0.8 and np.count_nonzero(y) == 1
    sl.batch.run(14)
    rho, gam = sl.batch.schedule(sl.slot, 15)
    xo, _ = orc.parsdmm(m, shape, sets, orc.Options(max_iter=15, cg_max=10, cg_fixed=True),
                        schedule={k + 1: (rho[k], gam[k]) for k in range(15)})
    assert rel(sl.x(), xo) <= 1e-10


def test_multilevel_l2_radius_transfer():
    import torch
    m, sets, _ = _case("l2_grad", "f64")
    iters = [20, 12, 8]
    opts = sip.make_opts("f64", max_iter=20, cg_max=10, cg_fixed=1, adapt_every=0)
    x, res, run = sip.project_multilevel(torch.tensor(m, device="cuda"), sets, opts, 3, iters, False)
    xo, _ = ml.parsdmm_multilevel(m, m.shape, sets, 3, iters,
                                  orc.Options(max_iter=20, cg_max=10, cg_fixed=True, adapt_every=0))
    err = rel(x.cpu().numpy(), xo)
    print(f"\n[sets ext multilevel] l2 on GRAD: rel err {err:.2e}", flush=True)
    assert err <= 1e-10


def test_multilevel_rejects_bound_vectors():
    import torch
    m, dev, _ = _case("vec_bounds", "f64")
    opts = sip.make_opts("f64", max_iter=5)
    with pytest.raises(sip.SipError) as e:
        sip.project_multilevel(torch.tensor(m, device="cuda"), dev, opts, 2, [5, 5])
    assert e.value.status == sip.EUNSUPPORTED
