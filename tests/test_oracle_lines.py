"""Pins of the oracle's line-wise sets (constraints that act on every row,
column or fiber of A x on its own, the paper's section on software and its
full-waveform example): the line partition against grid coordinates, the
per-line projections against bisection, brute force and closed forms taken
row by row from a reshaped image, and a converged PARSDMM run against a
general QP solver."""
import numpy as np
import pytest

from oracle import parsdmm as orc
from tests import refs


def _image(shape, op, comp):
    """Shape of component `comp` of operator op's output."""
    axes = orc.AXIS_OPS[len(shape)][op] if op != "I" else (None,)
    sh = list(shape)
    if axes[comp] is not None:
        sh[axes[comp]] -= 1
    return tuple(sh)


@pytest.mark.parametrize("shape,op,line", [((4, 6), "DX", "x"), ((4, 6), "DZ", "z"), ((4, 6), "GRAD", "x"),
                                           ((4, 6), "GRAD", "z"), ((4, 6), "I", "z"), ((3, 4, 5), "LAT", "y"),
                                           ((3, 4, 5), "GRAD", "z"), ((3, 4, 5), "DY", "x"), ((1, 7), "DX", "x")])
def test_lines_partition_rows(shape, op, line):
    """Every row of A lies on exactly one line; along a line the grid
    coordinate on the line axis runs 0, 1, 2, ... and all other coordinates
    and the component are fixed."""
    A = orc.operator(op, shape)
    lines = orc.line_rows(op, shape, line)
    seen = np.concatenate(lines) if lines else np.zeros(0, int)
    assert np.array_equal(np.sort(seen), np.arange(A.shape[0]))
    ax = orc.LINE_AXES[len(shape)][line]
    ncomp = len(orc.AXIS_OPS[len(shape)][op]) if op != "I" else 1
    offs = np.cumsum([0] + [int(np.prod(_image(shape, op, c))) for c in range(ncomp)])
    for idx in lines:
        comp = np.searchsorted(offs, idx[0], side="right") - 1
        assert np.all((idx >= offs[comp]) & (idx < offs[comp + 1]))
        coords = np.array(np.unravel_index(idx - offs[comp], _image(shape, op, comp)))
        assert np.array_equal(coords[ax], np.arange(idx.size))
        others = np.delete(coords, ax, axis=0)
        assert np.all(others == others[:, :1])


def test_row_l1_against_bisection_per_row():
    rng = np.random.default_rng(0)
    shape = (5, 8)
    w = rng.standard_normal(5 * 7) * 2.0
    s = {"kind": "l1", "op": "DX", "tau": 1.5, "line": "x"}
    y = orc.project_lines(s, w, orc.line_rows("DX", shape, "x"))
    img = w.reshape(5, 7)
    ref = np.stack([refs.l1_bisection(img[i], 1.5) for i in range(5)])
    np.testing.assert_allclose(y.reshape(5, 7), ref, atol=1e-12)
    assert np.all(np.abs(y.reshape(5, 7)).sum(axis=1) <= 1.5 + 1e-12)


def test_column_card_against_brute_force_per_column():
    rng = np.random.default_rng(1)
    shape = (6, 5)
    w = rng.standard_normal(5 * 5)
    s = {"kind": "card", "op": "DZ", "k": 2, "line": "z"}
    y = orc.project_lines(s, w, orc.line_rows("DZ", shape, "z")).reshape(5, 5)
    img = w.reshape(5, 5)
    for j in range(5):
        ref, _ = refs.card_bruteforce(img[:, j], 2)
        np.testing.assert_array_equal(y[:, j], ref)
    assert np.all((y != 0).sum(axis=0) <= 2)


def test_fiber_l2_and_annulus_closed_form():
    rng = np.random.default_rng(2)
    shape = (3, 4, 5)
    # LAT: components D_y (image 3x3x5) then D_x (image 3x4x4); fibers along y
    w = rng.standard_normal(3 * 3 * 5 + 3 * 4 * 4)
    lines = orc.line_rows("LAT", shape, "y")
    y2 = orc.project_lines({"kind": "l2", "op": "LAT", "tau": 0.7, "line": "y"}, w, lines)
    ya = orc.project_lines({"kind": "annulus", "op": "LAT", "lo": 1.0, "hi": 1.2, "line": "y"}, w, lines)
    for blk, sh in ((slice(0, 45), (3, 3, 5)), (slice(45, None), (3, 4, 4))):
        img = w[blk].reshape(sh)
        nrm = np.linalg.norm(img, axis=1, keepdims=True)          # norm along y per (z, x)
        ref2 = img * np.minimum(1.0, 0.7 / nrm)
        refa = img * np.clip(nrm, 1.0, 1.2) / nrm
        np.testing.assert_allclose(y2[blk].reshape(sh), ref2, atol=1e-13)
        np.testing.assert_allclose(ya[blk].reshape(sh), refa, atol=1e-13)


def test_annulus_zero_line_takes_first_entry():
    shape = (3, 4)
    w = np.zeros(3 * 4)
    w[4:8] = [0.0, 3.0, 0.0, 4.0]  # second row nonzero
    y = orc.project_lines({"kind": "annulus", "op": "I", "lo": 1.0, "hi": 2.0, "line": "x"}, w,
                          orc.line_rows("I", shape, "x")).reshape(3, 4)
    np.testing.assert_allclose(y[0], [1.0, 0, 0, 0])
    np.testing.assert_allclose(y[2], [1.0, 0, 0, 0])
    np.testing.assert_allclose(y[1], [0.0, 1.2, 0.0, 1.6])


def test_single_line_equals_whole_vector():
    rng = np.random.default_rng(3)
    w = rng.standard_normal(9)
    for s in ({"kind": "l1", "tau": 1.0}, {"kind": "card", "k": 3}, {"kind": "l2", "tau": 0.5}):
        ln = orc.line_rows("DX", (1, 10), "x")
        assert len(ln) == 1
        np.testing.assert_array_equal(orc.project_lines({**s, "op": "DX", "line": "x"}, w, ln),
                                      orc.project_set(s, w))


def test_bounds_cannot_be_line_wise():
    with pytest.raises(ValueError):
        orc.Problem(np.zeros((3, 3)), (3, 3), [{"kind": "bounds", "op": "I", "lo": 0, "hi": 1, "line": "x"}])


def test_parsdmm_row_l1_matches_qp():
    """Converged PARSDMM with per-row l1 balls on D_x and bounds equals the
    QP solution with one l1 block per row."""
    rng = np.random.default_rng(4)
    shape = (4, 6)
    m = rng.standard_normal(shape)
    tau = 0.8
    sets = [{"kind": "l1", "op": "DX", "tau": tau, "line": "x"}, {"kind": "bounds", "op": "I", "lo": -1.0, "hi": 1.0}]
    opts = orc.Options(max_iter=4000, cg_max=60, cg_fixed=False, cg_rel=1e-10, stop_every=5, eps_evol=1e-9,
                       eps_feas=1e-9)
    x, st = orc.parsdmm(m, shape, sets, opts)
    D = orc.operator("DX", shape).toarray()
    blocks = [(D[idx], tau) for idx in orc.line_rows("DX", shape, "x")]
    xq = refs.qp_projection(m.ravel(), l1_blocks=blocks, bounds=(-1.0, 1.0))
    np.testing.assert_allclose(x.ravel(), xq, atol=2e-5)
    rows = np.abs((D @ x.ravel()).reshape(4, 5)).sum(axis=1)
    assert np.all(rows <= tau * (1 + 1e-6))


def test_parsdmm_column_card_is_feasible():
    """Per-column cardinality on D_z: the final y of the set has at most k
    nonzeros in every column, and x reaches it to within the stopping rule."""
    rng = np.random.default_rng(5)
    shape = (8, 6)
    blocky = np.zeros(shape)
    blocky[3:, :] += 1.0
    blocky[6:, 2:] += 0.5          # at most two jumps down every column
    m = blocky + 0.02 * rng.standard_normal(shape)
    sets = [{"kind": "card", "op": "DZ", "k": 2, "line": "z"}]
    opts = orc.Options(max_iter=3000, cg_max=30, cg_fixed=False, cg_rel=1e-8, stop_every=5, eps_evol=1e-7,
                       eps_feas=1e-7)
    x, st = orc.parsdmm(m, shape, sets, opts)
    assert st.converged
    y = st.y[0].reshape(7, 6)
    assert np.all((y != 0).sum(axis=0) <= 2)
    dz = np.diff(x, axis=0)
    assert np.linalg.norm(dz.ravel() - st.y[0]) <= 1e-6 * max(1.0, np.linalg.norm(dz))
    assert np.abs(x - blocky).max() < 0.1


def test_multilevel_rejects_line_sets():
    from oracle import multilevel as ml
    with pytest.raises(NotImplementedError):
        ml.parsdmm_multilevel(np.zeros((8, 8)), (8, 8), [{"kind": "l1", "op": "DX", "tau": 1.0, "line": "x"}], 2,
                              [5, 5])
