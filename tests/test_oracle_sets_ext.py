"""Pins of the oracle's l2-ball, annulus and per-pixel (vector) bound
projections (Table set-overview) against an independent solver, dense
sampling and closed forms, and of PARSDMM on them."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import parsdmm as orc
from tests import refs


def _slsqp_ball(w, tau):
    cons = [{"type": "ineq", "fun": lambda y: tau * tau - y @ y, "jac": lambda y: -2.0 * y}]
    r = minimize(lambda y: 0.5 * (y - w) @ (y - w), np.zeros_like(w), jac=lambda y: y - w,
                 constraints=cons, method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
    return r.x


@pytest.mark.parametrize("seed", range(4))
def test_l2_projection_vs_slsqp(seed):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(6) * 2.0
    tau = 0.3 + seed
    y = orc.project_l2(w, tau)
    np.testing.assert_allclose(y, _slsqp_ball(w, tau), atol=1e-6)
    # inside the ball: unchanged
    np.testing.assert_array_equal(orc.project_l2(w * 1e-3, tau), w * 1e-3)


@pytest.mark.parametrize("seed", range(3))
def test_annulus_projection_by_sampling(seed):
    rng = np.random.default_rng(10 + seed)
    lo, hi = 1.0, 2.0
    pts = rng.standard_normal((40000, 3))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    pts *= rng.uniform(lo, hi, (40000, 1))          # samples of the shell
    for scale in (0.2, 1.5, 4.0):                      # inside the hole, in the shell, outside
        w = rng.standard_normal(3)
        w *= scale / np.linalg.norm(w)
        y = orc.project_annulus(w, lo, hi)
        assert lo - 1e-12 <= np.linalg.norm(y) <= hi + 1e-12
        d = np.linalg.norm(y - w)
        assert np.min(np.linalg.norm(pts - w, axis=1)) >= d - 1e-9
        if lo <= scale <= hi:
            np.testing.assert_array_equal(y, w)
    # w = 0: the reading picks lo e_0
    np.testing.assert_array_equal(orc.project_annulus(np.zeros(4), lo, hi), [lo, 0, 0, 0])


def test_vector_bounds_projection_is_clip():
    rng = np.random.default_rng(3)
    w = rng.standard_normal(50)
    lo = rng.uniform(-1.0, 0.0, 50)
    hi = lo + rng.uniform(0.0, 1.0, 50)
    y = orc.project_set({"kind": "bounds", "op": "I", "lo": lo, "hi": hi}, w)
    np.testing.assert_array_equal(y, np.clip(w, lo, hi))


def test_parsdmm_single_l2_ball_converges_to_closed_form():
    m = np.random.default_rng(5).standard_normal((7, 9))
    tau = 0.4 * np.linalg.norm(m)
    x, st = orc.parsdmm(m, m.shape, [{"kind": "l2", "op": "I", "tau": tau}],
                        orc.Options(max_iter=400, cg_max=30, cg_fixed=False, cg_rel=1e-8))
    np.testing.assert_allclose(x.ravel(), orc.project_l2(m.ravel(), tau), atol=1e-6)


def test_parsdmm_vector_bounds_vs_qp():
    """Per-row lower bounds on D_z (a depth-varying monotonicity) with a box:
    the PARSDMM result equals the SLSQP projection on the explicit rows."""
    rng = np.random.default_rng(6)
    shape = (5, 6)
    m = rng.standard_normal(shape)
    Dz = orc.operator("DZ", shape, (1.0, 1.0)).toarray()
    lo = rng.uniform(-0.2, 0.3, Dz.shape[0])
    sets = [{"kind": "bounds", "op": "DZ", "lo": lo, "hi": np.full(Dz.shape[0], np.inf)},
            {"kind": "bounds", "op": "I", "lo": -1.0, "hi": 1.0}]
    x, _ = orc.parsdmm(m, shape, sets, orc.Options(max_iter=3000, cg_max=50, cg_fixed=False, cg_rel=1e-8))
    ref = refs.qp_projection(m.ravel(), lin_ineq=[(-Dz, -lo)], bounds=(-1.0, 1.0))
    assert np.linalg.norm(x.ravel() - ref) <= 1e-5 * np.linalg.norm(ref)
