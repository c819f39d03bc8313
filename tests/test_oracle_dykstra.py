"""Pins of the parallel Dykstra oracle (Appendix A listing, inner projections
by single-set PARSDMM): the first iterate in closed form, and convergence to
the projection onto the intersection computed by a general QP solver."""
import numpy as np

from oracle import dykstra as dk
from oracle import parsdmm as orc
from tests import refs

TIGHT = orc.Options(max_iter=3000, cg_max=50, cg_fixed=False, cg_rel=1e-10, stop_every=5, eps_evol=1e-11,
                    eps_feas=1e-11)


def test_first_iterate_is_mean_of_projections():
    """Two boxes on the identity: y_i = clip_i(m) exactly, x^1 = their mean,
    v_i^1 = x^1 + m - y_i."""
    rng = np.random.default_rng(0)
    shape = (3, 4)
    m = rng.standard_normal(shape) * 2.0
    sets = [{"kind": "bounds", "op": "I", "lo": -1.0, "hi": 0.5}, {"kind": "bounds", "op": "I", "lo": -0.2, "hi": 2.0}]
    x1, log, xs = dk.parallel_dykstra(m, shape, sets, 1, TIGHT)
    c1, c2 = np.clip(m, -1.0, 0.5), np.clip(m, -0.2, 2.0)
    np.testing.assert_allclose(x1, 0.5 * (c1 + c2), atol=1e-9)
    x2, _, _ = dk.parallel_dykstra(m, shape, sets, 2, TIGHT)
    # second iterate by hand from v_i^1
    v1 = [0.5 * (c1 + c2) + m - c1, 0.5 * (c1 + c2) + m - c2]
    ref2 = 0.5 * (np.clip(v1[0], -1.0, 0.5) + np.clip(v1[1], -0.2, 2.0))
    np.testing.assert_allclose(x2, ref2, atol=1e-9)
    assert len(log) == 1 and len(log[0].iters) == 2


def test_converges_to_projection_onto_intersection():
    """Box, TV ball and vertical monotonicity (the paper's first comparison
    sets) on a 4x5 grid: the Dykstra iterate reaches the QP solution."""
    rng = np.random.default_rng(0)
    shape = (4, 5)
    m = np.cumsum(rng.standard_normal(shape) * 0.5, axis=0)[::-1].copy()
    D = orc.operator("GRAD", shape).toarray()
    Dz = orc.operator("DZ", shape).toarray()
    tau = 0.5 * np.abs(D @ m.ravel()).sum()
    sets = [{"kind": "bounds", "op": "I", "lo": -1.0, "hi": 1.0}, {"kind": "l1", "op": "GRAD", "tau": tau},
            {"kind": "bounds", "op": "DZ", "lo": 0.0, "hi": np.inf}]
    xq = refs.qp_projection(m.ravel(), lin_ineq=[(-Dz, np.zeros(Dz.shape[0]))], l1_blocks=[(D, tau)],
                            bounds=(-1.0, 1.0))
    x, log, xs = dk.parallel_dykstra(m, shape, sets, 60, TIGHT)
    np.testing.assert_allclose(x.ravel(), xq, atol=1e-6)
    # the error shrinks along the way
    e = [np.abs(xi - xq).max() for xi in xs]
    assert e[-1] < 1e-3 * e[0]
