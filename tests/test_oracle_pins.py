"""Pins of the FP64 oracle against what the paper and mathematics fix:
closed forms, brute force on tiny inputs, independent algorithms (bisection,
pool-adjacent-violators, halfspace Dykstra, a QP solver, DCT diagonalisation)
and hand-worked cases.  CPU only."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import parsdmm as orc
from tests import refs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- operators

@pytest.mark.parametrize("shape", [(5, 7), (4, 3, 6)])
def test_difference_operators_match_axis_differences(shape):
    rng = np.random.default_rng(0)
    h = tuple(rng.uniform(0.5, 2.0, size=len(shape)))
    m = rng.standard_normal(shape)
    names = {2: ("DZ", "DX"), 3: ("DZ", "DY", "DX")}[len(shape)]
    for axis, name in enumerate(names):
        got = orc.operator(name, shape, h) @ m.ravel()
        want = np.diff(m, axis=axis).ravel() / h[axis]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


def test_difference_exact_on_linear_and_zero_on_constant():
    shape = (6, 9)
    zz, xx = np.meshgrid(np.arange(6.0), np.arange(9.0), indexing="ij")
    lin = 3.0 * zz - 2.0 * xx + 1.0
    h = (0.5, 2.0)
    np.testing.assert_allclose(orc.operator("DZ", shape, h) @ lin.ravel(), 3.0 / 0.5)
    np.testing.assert_allclose(orc.operator("DX", shape, h) @ lin.ravel(), -2.0 / 2.0)
    assert np.abs(orc.operator("GRAD", shape, h) @ np.full(54, 7.0)).max() == 0.0


def test_stacked_operators_rows_and_tv():
    rng = np.random.default_rng(1)
    m = rng.standard_normal((4, 5, 6))
    G = orc.operator("GRAD", m.shape)
    L = orc.operator("LAT", m.shape)
    assert G.shape == (3 * 5 * 6 + 4 * 4 * 6 + 4 * 5 * 5, m.size)
    assert L.shape == (4 * 4 * 6 + 4 * 5 * 5, m.size)
    tv = sum(np.abs(np.diff(m, axis=a)).sum() for a in range(3))
    assert abs(np.abs(G @ m.ravel()).sum() - tv) < 1e-11


def test_normal_matrix_is_neumann_laplacian_with_known_spectrum():
    n, h = 9, 0.7
    D = orc.fd_matrix(n, h)
    B = (D.T @ D).toarray() * h * h
    ev = np.sort(np.linalg.eigvalsh(B))
    want = np.sort(4.0 * np.sin(np.pi * np.arange(n) / (2.0 * n)) ** 2)
    np.testing.assert_allclose(ev, want, atol=1e-12)


# ------------------------------------------------------------- projections

def test_bounds_projection_elementwise():
    w = np.array([-3.0, -1.0, 0.2, 1.0, 5.0])
    np.testing.assert_array_equal(orc.project_bounds(w, -1.0, 1.0), [-1.0, -1.0, 0.2, 1.0, 1.0])
    np.testing.assert_array_equal(orc.project_bounds(w, 0.0, math.inf), [0.0, 0.0, 0.2, 1.0, 5.0])


@pytest.mark.parametrize("seed", range(6))
def test_l1_projection_vs_bisection_and_kkt(seed):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(200) * rng.uniform(0.1, 3.0)
    tau = float(np.abs(w).sum() * rng.uniform(0.05, 0.9))
    y = orc.project_l1(w, tau)
    np.testing.assert_allclose(y, refs.l1_bisection(w, tau), atol=1e-12)
    assert abs(np.abs(y).sum() - tau) < 1e-9 * max(1.0, tau)
    sup = y != 0
    assert np.all(np.sign(y[sup]) == np.sign(w[sup]))
    gap = np.abs(w[sup]) - np.abs(y[sup])
    assert np.ptp(gap) < 1e-12
    assert np.all(np.abs(w[~sup]) <= gap[0] + 1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_l1_projection_bruteforce_tiny(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 9))
    w = rng.standard_normal(n)
    tau = float(np.abs(w).sum() * rng.uniform(0.1, 1.2))
    np.testing.assert_allclose(orc.project_l1(w, tau), refs.l1_bruteforce(w, tau), atol=1e-12)


def test_l1_special_cases():
    w = np.array([0.5, -0.25, 0.0])
    np.testing.assert_array_equal(orc.project_l1(w, 10.0), w)
    np.testing.assert_array_equal(orc.project_l1(w, 0.0), np.zeros(3))
    # equal magnitudes: theta = (3a - tau)/3
    y = orc.project_l1(np.array([2.0, -2.0, 2.0]), 3.0)
    np.testing.assert_allclose(y, [1.0, -1.0, 1.0])


@pytest.mark.parametrize("seed", range(6))
def test_card_projection_bruteforce_with_ties(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(3, 10))
    w = rng.integers(-3, 4, size=n).astype(np.float64)  # many ties
    k = int(rng.integers(1, n + 1))
    want, sup = refs.card_bruteforce(w, k)
    np.testing.assert_array_equal(orc.project_card(w, k), want)
    np.testing.assert_array_equal(orc.card_support(w, k), sup)


def test_prox_sq_dist_is_minimiser():
    rng = np.random.default_rng(3)
    m, w = rng.standard_normal(50), rng.standard_normal(50)
    rho = 2.5
    z = orc.prox_sq_dist(w, m, rho)
    grad = (z - m) + rho * (z - w)
    assert np.abs(grad).max() < 1e-14


# ---------------------------------------------------------------------- CG

def _system(shape, rho, sets):
    prob = orc.Problem(np.zeros(int(np.prod(shape))), shape, sets)
    return prob, prob.system_matrix(np.asarray(rho, dtype=np.float64))


def test_converged_cg_matches_direct_and_dct_solution():
    shape = (12, 17)
    sets = [{"kind": "bounds", "op": "I", "lo": -1, "hi": 1},
            {"kind": "l1", "op": "GRAD", "tau": 1.0},
            {"kind": "bounds", "op": "DZ", "lo": 0, "hi": math.inf}]
    rho = [0.7, 2.0, 0.4, 1.3]
    prob, C = _system(shape, rho, sets)
    b = np.random.default_rng(4).standard_normal(C.shape[0])
    x, steps = orc.cg(C, b, np.zeros_like(b), cg_rel=1e-14, cg_max=2000, fixed=False)
    np.testing.assert_allclose(x, spla.spsolve(C.tocsc(), b), rtol=0, atol=1e-10)
    # C = c0 I + cz Lz + cx Lx, with c0 = rho_box + rho_{p+1}, cz = rho_tv + rho_mono, cx = rho_tv
    xd = refs.neumann_solve_dct(b.reshape(shape), rho[0] + rho[3], [rho[1] + rho[2], rho[1]])
    np.testing.assert_allclose(x, xd.ravel(), atol=1e-10)


def test_cg_relative_stop_and_warm_start():
    shape = (10, 10)
    prob, C = _system(shape, [1.0, 1.0], [{"kind": "l1", "op": "GRAD", "tau": 1.0}])
    rng = np.random.default_rng(5)
    xs = rng.standard_normal(C.shape[0])
    b = C @ xs
    x, steps = orc.cg(C, b, xs, fixed=False)
    assert steps == 0
    x0 = xs + 0.1 * rng.standard_normal(xs.size)
    r0 = np.linalg.norm(b - C @ x0)
    x, steps = orc.cg(C, b, x0, cg_rel=0.1, cg_max=100, fixed=False)
    assert np.linalg.norm(b - C @ x) < 0.1 * r0
    assert 0 < steps < 100


def test_first_x_update_returns_m():
    m = np.random.default_rng(6).standard_normal((8, 9))
    sets = [{"kind": "bounds", "op": "I", "lo": -0.5, "hi": 0.5}, {"kind": "l1", "op": "GRAD", "tau": 3.0}]
    prob = orc.Problem(m, m.shape, sets)
    opts = orc.Options()
    st = orc.initial_state(prob, opts)
    orc.x_update(prob, st, opts)
    np.testing.assert_allclose(st.x, m.ravel(), atol=1e-12)


# ----------------------------------------------------------- adapt / stop

def test_adapt_rho_gamma_hand_worked_cases():
    with open(os.path.join(GOLDEN, "adapt_rho_gamma_cases.json")) as f:
        cases = json.load(f)["cases"]
    z = np.zeros(3)
    for c in cases:
        snap = orc.Snapshot(vhat=z, v=z, s=z, y=z)
        arr = {k: np.array(c[k], dtype=np.float64) for k in ("s", "y_old", "v_old", "y_new", "v_new")}
        rho, gamma, _ = orc.adapt_rho_gamma(arr["s"], arr["y_old"], arr["y_new"], arr["v_old"],
                                            arr["v_new"], c["rho"], c["gamma"], snap)
        assert rho == pytest.approx(c["expect_rho"], rel=1e-14), c["name"]
        assert gamma == pytest.approx(c["expect_gamma"], rel=1e-14), c["name"]


def test_adapt_first_call_only_stores_snapshot():
    v = np.ones(4)
    rho, gamma, snap = orc.adapt_rho_gamma(v, v, v, v, v, 3.0, 1.2, None)
    assert (rho, gamma) == (3.0, 1.2) and snap is not None


def test_spectral_estimate_recovers_linear_curvature():
    rng = np.random.default_rng(7)
    for c in (0.1, 1.0, 42.0):
        d = rng.standard_normal(20)
        ok, est = orc._spectral(d, c * d, 0.3)
        assert ok and est == pytest.approx(c, rel=1e-12)


def test_guards():
    opts = orc.Options()
    rho, gamma = orc.guard_parameters([1e-5, 1e5, 1.0, 2.0], [2.0, 1.5, 1.0, 1.9], opts)
    np.testing.assert_allclose(rho, [0.02, 200.0, 1.0, 2.0])
    np.testing.assert_allclose(gamma, [1.999, 1.5, 1.0, 1.9])


def test_stopping_measures():
    x = np.array([3.0, 4.0])
    assert orc.relative_evolution(x, [x.copy()] * 5) == 0.0
    assert orc.relative_evolution(x, [x, 0.5 * x]) == pytest.approx(0.5)
    s = {"kind": "bounds", "lo": 0.0, "hi": 1.0}
    assert orc.feasibility_error(s, np.array([0.5, 0.5])) == 0.0
    assert orc.feasibility_error(s, np.array([2.0, 0.0])) == pytest.approx(0.5)
    assert orc.feasibility_error({"kind": "bounds", "lo": 1.0, "hi": 2.0}, np.zeros(3)) == math.inf


# ------------------------------------------------------- end-to-end, convex

def _run(m, sets, iters, **kw):
    opts = orc.Options(max_iter=iters, **kw)
    x, st = orc.parsdmm(m, m.shape, sets, opts)
    return x, st


def test_single_box_set_converges_to_clip():
    m = np.random.default_rng(8).standard_normal((9, 11)) * 2
    x, _ = _run(m, [{"kind": "bounds", "op": "I", "lo": -1.0, "hi": 1.0}], 300)
    np.testing.assert_allclose(x, np.clip(m, -1, 1), atol=1e-8)


def test_single_l1_set_converges_to_l1_projection():
    m = np.random.default_rng(9).standard_normal((6, 7))
    tau = 0.4 * np.abs(m).sum()
    x, _ = _run(m, [{"kind": "l1", "op": "I", "tau": tau}], 400)
    np.testing.assert_allclose(x.ravel(), refs.l1_bisection(m.ravel(), tau), atol=1e-7)


def test_monotonicity_set_converges_to_isotonic_regression():
    m = np.random.default_rng(10).standard_normal((10, 6))
    x, _ = _run(m, [{"kind": "bounds", "op": "DZ", "lo": 0.0, "hi": math.inf}], 1500, cg_fixed=False,
                cg_rel=1e-3, cg_max=200)
    np.testing.assert_allclose(x, refs.monotone_columns(m), atol=1e-6)


def _tiny_multiset():
    rng = np.random.default_rng(11)
    m = rng.standard_normal((2, 3)) * 1.5
    G = orc.operator("GRAD", m.shape).toarray()
    tau = 0.2 * np.abs(G @ m.ravel()).sum()
    sets = [{"kind": "bounds", "op": "I", "lo": -1.0, "hi": 1.0},
            {"kind": "l1", "op": "GRAD", "tau": tau},
            {"kind": "bounds", "op": "DZ", "lo": 0.0, "hi": math.inf}]
    return m, G, tau, sets


def test_multiset_convex_matches_dykstra_and_qp():
    m, G, tau, sets = _tiny_multiset()
    n = m.size
    Dz = orc.operator("DZ", m.shape).toarray()
    H = [np.eye(n), -np.eye(n), -Dz]
    b = [np.ones(n), np.ones(n), np.zeros(Dz.shape[0])]
    import itertools
    for signs in itertools.product((-1.0, 1.0), repeat=G.shape[0]):
        H.append((np.array(signs) @ G)[None, :])
        b.append(np.array([tau]))
    H = np.vstack(H)
    b = np.concatenate(b)
    x_dyk = refs.dykstra_halfspaces(m.ravel(), H, b)
    x_qp = refs.qp_projection(m.ravel(), lin_ineq=[(-Dz, np.zeros(Dz.shape[0]))],
                              l1_blocks=[(G, tau)], bounds=(-1.0, 1.0))
    np.testing.assert_allclose(x_dyk, x_qp, atol=1e-6)
    x, st = _run(m, sets, 3000, cg_fixed=False, cg_rel=1e-4, cg_max=100)
    np.testing.assert_allclose(x.ravel(), x_qp, atol=1e-6)


def test_convex_result_is_feasible_and_satisfies_variational_inequality():
    from paper_1902_09699_amd import workloads as wl
    m, sets, _, _ = wl.smooth2d_box_tv(n=(24, 28), seed=77)
    sets = wl.finalize(m, sets)
    x, st = _run(m, sets, 600, cg_fixed=False, cg_rel=1e-2, cg_max=50)
    xv = x.ravel()
    assert xv.min() >= -1 - 1e-6 and xv.max() <= 1 + 1e-6
    G = orc.operator("GRAD", m.shape)
    assert np.abs(G @ xv).sum() <= sets[1]["tau"] * (1 + 1e-6)
    # <m - x, z - x> <= 0 for feasible z: constants in [-1, 1] and segments toward them
    d = m.ravel() - xv
    for c in np.linspace(-1, 1, 9):
        for t in (1.0, 0.3, 0.01):
            z = xv + t * (c - xv)
            assert d @ (z - xv) <= 1e-5 * np.linalg.norm(d) * np.linalg.norm(z - xv) + 1e-12
    # idempotence: projecting the projection returns it
    x2, _ = _run(x, sets, 300, cg_fixed=False, cg_rel=1e-2, cg_max=50)
    np.testing.assert_allclose(x2, x, atol=1e-5)


def test_stopping_rule_stops_and_reports():
    m = np.random.default_rng(12).standard_normal((10, 12))
    sets = [{"kind": "bounds", "op": "I", "lo": -1.0, "hi": 1.0}]
    x, st = _run(m, sets, 500, stop_every=5)
    assert st.converged and st.k - 1 < 500 and (st.k - 1) % 5 == 0
    assert st.r_evol < 1e-2 and np.all(st.r_feas < 1e-3)


def test_schedule_replay_reproduces_free_run():
    from paper_1902_09699_amd import workloads as wl
    m, sets, _, _ = wl.smooth2d_box_tv(n=(16, 20), seed=5)
    sets = wl.finalize(m, sets)
    opts = orc.Options(max_iter=30)
    prob = orc.Problem(m, m.shape, sets)
    st = orc.initial_state(prob, opts)
    sched = {}
    while st.k <= opts.max_iter:
        sched[st.k] = (st.rho.copy(), st.gamma.copy())
        orc.iterate(prob, st, opts)
    x2, st2 = orc.parsdmm(m, m.shape, sets, opts, schedule=sched)
    np.testing.assert_array_equal(x2.ravel(), st.x)


def test_relative_evolution_window_is_last_five_iterates():
    prob = orc.Problem(np.zeros(4), (2, 2), [{"kind": "bounds", "op": "I", "lo": -1, "hi": 1}])
    opts = orc.Options()
    st = orc.initial_state(prob, opts)
    x = np.array([1.0, 2.0, 2.0, 4.0])  # ||x|| = 5
    # x^{k-5} is off by 2.5 (r_evol 0.5); x^{k-6} (outside the window) by far more
    st.x_hist = [x + 100.0, x + np.array([0, 0, 0, 2.5])] + [x.copy()] * 4 + [x.copy()]
    st.x = x.copy()
    orc.stop_test(prob, st, opts)
    assert st.r_evol == pytest.approx(0.5)


def test_adapt_runs_on_odd_iterations_only():
    from paper_1902_09699_amd import workloads as wl
    m, sets, _, _ = wl.smooth2d_box_tv(n=(10, 12), seed=9)
    sets = wl.finalize(m, sets)
    opts = orc.Options(max_iter=10)
    prob = orc.Problem(m, m.shape, sets)
    st = orc.initial_state(prob, opts)
    orc.iterate(prob, st, opts)               # k = 1: first call stores snapshots only
    snaps1 = list(st.snaps)
    assert all(s is not None for s in snaps1)
    assert np.all(st.rho == 1.0) and np.all(st.gamma == 1.0)
    orc.iterate(prob, st, opts)               # k = 2: no adapt call
    assert all(a is b for a, b in zip(st.snaps, snaps1))
    orc.iterate(prob, st, opts)               # k = 3: new snapshots
    assert all(a is not b for a, b in zip(st.snaps, snaps1))


def test_support_replay_of_own_choice_reproduces_free_run():
    """Replaying a run's own cardinality supports (and schedule) changes
    nothing: the replay only substitutes the choice of rows."""
    from paper_1902_09699_amd import workloads as wl
    m, sets, _, _ = wl.layered2d_four_sets(n=(14, 19), seed=6)
    sets = wl.finalize(m, sets)
    icard = [i for i, s in enumerate(sets) if s["kind"] == "card"]
    assert icard
    opts = orc.Options(max_iter=12)
    prob = orc.Problem(m, m.shape, sets)
    st = orc.initial_state(prob, opts)
    sched, sup = {}, {}
    while st.k <= opts.max_iter:
        k = st.k
        sched[k] = (st.rho.copy(), st.gamma.copy())
        orc.iterate(prob, st, opts)
        sup[k] = {i: np.nonzero(st.y[i])[0] for i in icard}
        for i in icard:
            assert np.array_equal(np.sort(orc.card_support(st.w_last[i], sets[i]["k"])), sup[k][i])
    x2, _ = orc.parsdmm(m, m.shape, sets, opts, schedule=sched, supports=sup)
    np.testing.assert_array_equal(x2.ravel(), st.x)


def test_support_replay_takes_the_other_tied_row():
    """At an exact tie the set has two projections; a replay of the other
    choice keeps the other row (and only the cardinality set's y changes)."""
    prob = orc.Problem(np.array([0.0, 0.0, 0.0]), (1, 3), [{"kind": "card", "op": "I", "k": 1}])
    w = np.array([2.0, -2.0, 0.5])
    np.testing.assert_array_equal(prob.prox(0, w, 1.0), [2.0, 0.0, 0.0])      # ties to the lower index
    np.testing.assert_array_equal(prob.prox(0, w, 1.0, keep=np.array([1])), [0.0, -2.0, 0.0])
    with pytest.raises(ValueError):
        orc.Problem(np.zeros(3), (1, 3), [{"kind": "l1", "op": "I", "tau": 1.0}]).prox(0, w, 1.0, keep=np.array([0]))


def test_cg_count_replay_of_own_decisions_reproduces_free_run():
    """With the relative CG stop on, replaying a run's own CG step counts
    (and schedule) reproduces it bitwise, and every count is the first step
    whose residual ratio fell below cg_rel (eq. cg_stop) or the cap."""
    from paper_1902_09699_amd import workloads as wl
    m, sets, _, _ = wl.smooth2d_box_tv(n=(18, 21), seed=8)
    sets = wl.finalize(m, sets)
    opts = orc.Options(max_iter=25, cg_max=10, cg_fixed=False, stop_every=5)
    prob = orc.Problem(m, m.shape, sets)
    st = orc.initial_state(prob, opts)
    sched = {}
    while st.k <= opts.max_iter:
        k = st.k
        rho, gam = st.rho.copy(), st.gamma.copy()
        before = st.cg_steps
        stop = orc.iterate(prob, st, opts)
        n = st.cg_steps - before
        sched[k] = (rho, gam, n)
        tr = st.cg_trace
        assert n == opts.cg_max or tr[n] < opts.cg_rel or tr[n] == 0.0
        assert all(t >= opts.cg_rel for t in tr[1:n])
        if stop:
            break
    x2, st2 = orc.parsdmm(m, m.shape, sets, opts, schedule=sched)
    np.testing.assert_array_equal(x2.ravel(), st.x)
    assert st2.k == st.k and st2.cg_steps == st.cg_steps
