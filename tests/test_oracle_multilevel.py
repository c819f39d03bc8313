"""Pins of the multilevel oracle (ML-PARSDMM listing) against facts that do
not come from the oracle itself: the filter and interpolation rules on
fields they must reproduce exactly, the parameter transfer's closed form,
one level being exactly PARSDMM, and convergence of the multilevel scheme to
the unique projection computed by an independent QP solver."""
import numpy as np
import pytest

from oracle import multilevel as ml
from oracle import parsdmm as orc
from tests import refs


def test_coarse_shapes():
    assert ml.level_shapes((341, 1361), 3) == [(341, 1361), (171, 681), (86, 341)]
    assert ml.level_shapes((200, 200, 100), 2) == [(200, 200, 100), (100, 100, 50)]
    assert ml.coarse_shape((1, 9)) == (1, 5)


def test_restrict_constant_and_linear():
    c = np.full((9, 11), 2.5)
    np.testing.assert_allclose(ml.restrict(c), np.full((5, 6), 2.5), rtol=0, atol=0)
    z, x = np.meshgrid(np.arange(9.0), np.arange(11.0), indexing="ij")
    f = 0.7 * z - 1.3 * x + 4.0
    r = ml.restrict(f)
    assert r.shape == (5, 6)
    # the [1,2,1]/4 filter keeps linear functions where the stencil fits
    for jz in range(1, 4):
        for jx in range(1, 5):
            assert abs(r[jz, jx] - f[2 * jz, 2 * jx]) < 1e-13
    # at a replicated edge: (f0 + 2 f0 + f1)/4 = f0 + slope/4 along that axis
    assert abs(r[0, 2] - (f[0, 4] + 0.7 / 4)) < 1e-13


def test_restrict_3d_filter_weights():
    d = np.zeros((5, 5, 5))
    d[2, 2, 2] = 64.0
    r = ml.restrict(d)
    # the coarse sample at fine (2,2,2) sees the full centre weight (1/2)^3
    assert r.shape == (3, 3, 3) and abs(r[1, 1, 1] - 8.0) < 1e-13
    assert abs(r.sum() - 8.0) < 1e-13


def test_prolong_points_reproduces_linear():
    z, x = np.meshgrid(np.arange(9.0), np.arange(13.0), indexing="ij")
    f = 0.3 * z + 2.0 * x - 1.0
    coarse = f[::2, ::2]
    np.testing.assert_allclose(ml.prolong_image(coarse, f.shape), f, atol=1e-12)


def test_prolong_staggered_rows_reproduce_linear():
    # m = z^2: coarse D_z (spacing 2) sampled at z = 2 jc + 1 is 2z; fine
    # rows j sit at z = j + 1/2, where the value is 2 j + 1
    nf = 13
    zc = np.arange(0, nf, 2.0)
    dc = np.diff(zc ** 2) / 2.0
    img_c = np.tile(dc[:, None], (1, 3))
    img_f = ml.prolong_image(img_c, (nf - 1, 3), stag_axis=0)
    for j in range(1, nf - 2):
        assert abs(img_f[j, 0] - (2 * j + 1)) < 1e-12, j


def test_level_sets_scaling():
    sets = [{"kind": "bounds", "op": "DZ", "lo": 0.0, "hi": np.inf},
            {"kind": "l1", "op": "GRAD", "tau": 120.0},
            {"kind": "card", "op": "DX", "k": 100}]
    out = ml.level_sets(sets, (21, 41), (11, 21))
    assert out[0] == sets[0]
    ratio = (10 * 21 + 11 * 20) / (20 * 41 + 21 * 40)
    assert abs(out[1]["tau"] - 120.0 * ratio) < 1e-12
    assert out[2]["k"] == int(np.floor(100 * (11 * 20) / (21 * 40) + 0.5))


def test_one_level_is_parsdmm():
    rng = np.random.default_rng(3)
    m = rng.standard_normal((9, 12))
    sets = [{"kind": "bounds", "op": "I", "lo": -0.5, "hi": 0.5}, {"kind": "l1", "op": "GRAD", "tau": 4.0}]
    o = orc.Options(max_iter=25, cg_max=10, cg_fixed=True)
    x1, _ = ml.parsdmm_multilevel(m, m.shape, sets, 1, [25], o)
    x0, _ = orc.parsdmm(m, m.shape, sets, o)
    np.testing.assert_array_equal(x1, x0)


def test_multilevel_reaches_the_projection():
    """Bounds, vertical monotonicity and lateral slope bounds (the sets of
    the paper's timing experiment) on a small layered model: the multilevel
    result after enough fine-level iterations equals the unique projection
    computed by SLSQP on the explicit constraints."""
    rng = np.random.default_rng(11)
    shape = (7, 8)
    m = np.repeat(rng.uniform(1.5, 4.5, (shape[0], 1)), shape[1], axis=1) + 0.3 * rng.standard_normal(shape)
    sets = [{"kind": "bounds", "op": "I", "lo": 1.5, "hi": 4.5},
            {"kind": "bounds", "op": "DZ", "lo": 0.0, "hi": np.inf},
            {"kind": "bounds", "op": "DX", "lo": -0.2, "hi": 0.2}]
    o = orc.Options(max_iter=3000, cg_max=50, cg_fixed=False, cg_rel=1e-6)
    x, states = ml.parsdmm_multilevel(m, shape, sets, 2, [3000, 400], o)
    Dz = orc.operator("DZ", shape, (1.0, 1.0)).toarray()
    Dx = orc.operator("DX", shape, (1.0, 1.0)).toarray()
    ref = refs.qp_projection(m.ravel(), lin_ineq=[(-Dz, np.zeros(Dz.shape[0])), (Dx, np.full(Dx.shape[0], 0.2)),
                                                   (-Dx, np.full(Dx.shape[0], 0.2))], bounds=(1.5, 4.5))
    assert np.linalg.norm(x.ravel() - ref) <= 1e-5 * np.linalg.norm(ref)
    assert states[1].x.shape == (4 * 4,)


@pytest.mark.parametrize("kind", ["l2", "annulus"])
@pytest.mark.parametrize("op,shape", [("I", (9, 13)), ("DX", (9, 13)), ("DZ", (11, 7)), ("DX", (5, 6, 9)),
                                      ("DY", (5, 7, 6))])
def test_l2_radius_transfer_matches_sampled_norms(kind, op, shape):
    """The l2 radius carried to a coarser level is the radius the coarse
    samples of a field sit at.  A field that is linear along the operator's
    axis (constant for the identity) has the same value in every row of A
    on every level (the spacing doubles with the sample distance), so
    ||A_l m_l||_2 = sqrt(rows_l / rows) ||A m||_2 exactly.  A field lying on
    the fine sphere must therefore lie on the transferred coarse sphere; a
    transfer by the row ratio itself (or not at all) misses it."""
    nd = len(shape)
    h = (1.0,) * nd
    ax = {"I": None, "DZ": 0, "DY": 1, "DX": nd - 1}[op]
    grids = np.meshgrid(*[np.arange(float(n)) for n in shape], indexing="ij")
    m = np.full(shape, 1.7) if ax is None else 0.35 * grids[ax] + 2.0
    shape_c = ml.coarse_shape(shape)
    m_c = m[tuple(slice(0, None, 2) for _ in shape)]
    assert m_c.shape == shape_c
    fine = np.linalg.norm(orc.operator(op, shape, h) @ m.ravel())
    coarse = np.linalg.norm(orc.operator(op, shape_c, tuple(2.0 * v for v in h)) @ m_c.ravel())
    ratio = ml.rows(shape_c, op) / ml.rows(shape, op)
    assert abs(coarse - np.sqrt(ratio) * fine) <= 1e-12 * fine
    # the alternatives a slip would produce differ measurably here
    assert abs(coarse - ratio * fine) > 1e-3 * fine and abs(coarse - fine) > 1e-3 * fine
    if kind == "l2":
        s = {"kind": "l2", "op": op, "tau": fine}
        got = ml.level_sets([s], shape, shape_c)[0]
        assert abs(got["tau"] - coarse) <= 1e-12 * coarse
    else:
        s = {"kind": "annulus", "op": op, "lo": 0.5 * fine, "hi": fine}
        got = ml.level_sets([s], shape, shape_c)[0]
        assert abs(got["hi"] - coarse) <= 1e-12 * coarse
        assert abs(got["lo"] - 0.5 * coarse) <= 1e-12 * coarse
