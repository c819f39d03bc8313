"""GPU-vs-oracle parity of line-wise sets (the set's projection on every
row, column or fiber of A x) through the C ABI: lockstep iterations on small
grids spanning many lines with ragged lengths, exact ties in the per-line
cardinality, the feasibility numbers of the stopping test, edge cases and the
full-size layered section."""
import math
import zlib

import numpy as np
import pytest

from oracle import parsdmm as orc
from paper_1902_09699_amd import sip
from paper_1902_09699_amd import workloads as wl
from tests.gpu_util import Slot, rel, sync_oracle

pytestmark = pytest.mark.gpu

STEP_TOL = {"f64": 1e-10, "f32": 1e-5}


def _line_l1(m, op, line, frac):
    """tau of a per-line l1 set: frac times the mean l1 norm of m's lines."""
    shape = m.shape
    a = orc.operator(op, shape) @ m.ravel()
    lines = orc.line_rows(op, shape, line)
    return frac * float(np.mean([np.abs(a[i]).sum() for i in lines]))


def _line_l2(m, op, line, frac):
    shape = m.shape
    a = orc.operator(op, shape) @ m.ravel()
    lines = orc.line_rows(op, shape, line)
    return frac * float(np.mean([np.linalg.norm(a[i]) for i in lines]))


def _case(kind, field, seed=0):
    rng = wl.rng_for(7000 + seed)
    if kind == "rows_card_2d":
        m = wl.layered((23, 37), rng, n_layers=5, min_rows=3)
        sets = [wl.bounds("I", 1.5, 4.5), {"kind": "card", "op": "DX", "k": 2, "line": "x"},
                {"kind": "l1", "op": "DZ", "tau": _line_l1(m, "DZ", "z", 0.5), "line": "z"}]
    elif kind == "cols_mixed_2d":
        m = wl.grf((31, 17), 4.0, rng)
        sets = [{"kind": "card", "op": "DZ", "k": 3, "line": "z"},
                {"kind": "l2", "op": "DX", "tau": _line_l2(m, "DX", "x", 0.6), "line": "x"},
                wl.l1("GRAD", 0.5)]
    elif kind == "fibers_3d":
        m = wl.grf((7, 9, 11), 3.0, rng)
        sets = [{"kind": "l1", "op": "LAT", "tau": _line_l1(m, "LAT", "y", 0.5), "line": "y"},
                {"kind": "card", "op": "GRAD", "k": 2, "line": "z"},
                {"kind": "annulus", "op": "I", "lo": 0.5 * _line_l2(m, "I", "x", 1.0),
                 "hi": 0.8 * _line_l2(m, "I", "x", 1.0), "line": "x"},
                wl.bounds("DZ", -0.3, 0.3)]
    elif kind == "annulus_rows_2d":
        m = wl.grf((12, 40), 5.0, rng)
        nrm = _line_l2(m, "DX", "x", 1.0)
        sets = [{"kind": "annulus", "op": "DX", "lo": 0.7 * nrm, "hi": 0.9 * nrm, "line": "x"},
                wl.bounds("I", -2.0, 2.0)]
    else:
        raise KeyError(kind)
    m = wl.rounded(m, field)
    return m, wl.finalize(m, sets)


def _card_line_mask(w, k, lines, rtol):
    """Entries away from their line's k-th magnitude (the support there is
    decided by the arithmetic, not by rounding)."""
    mask = np.ones(w.size, bool)
    for idx in lines:
        a = np.abs(w[idx])
        if k >= idx.size:
            continue
        tk = np.sort(a)[::-1][k - 1]
        mask[idx] = np.abs(a - tk) > rtol * max(tk, 1e-300)
    return mask


CASES = [("rows_card_2d", "f32", 0), ("rows_card_2d", "f64", 0), ("cols_mixed_2d", "f32", 0),
         ("cols_mixed_2d", "f64", 1), ("fibers_3d", "f32", 0), ("fibers_3d", "f64", 0),
         ("annulus_rows_2d", "f64", 0), ("annulus_rows_2d", "f32", 1), ("rows_card_2d", "f32", 2),
         ("cols_mixed_2d", "f64", 2)]


@pytest.mark.parametrize("kind,field,form", CASES)
def test_line_sets_step_parity(kind, field, form):
    m, sets = _case(kind, field)
    iters = 11
    print(f"\n[lines step] {kind} {field} shape={m.shape} cg_form={form}", flush=True)
    kw = dict(max_iter=50, cg_max=10, cg_fixed=1, stop_every=5, eps_evol=1e-30, eps_feas=1e-30)
    sl = Slot(m, sets, field, kw, tiles=(1024, 1024, 1024, 512, 512, form))
    prob = orc.Problem(m, m.shape, sets)
    oo = orc.Options(max_iter=50, cg_max=10, cg_fixed=True, stop_every=5, eps_evol=1e-30, eps_feas=1e-30)
    st = orc.initial_state(prob, oo)
    tol = STEP_TOL[field]
    worst = 0.0
    for it in range(iters):
        sync_oracle(sl, prob, st)
        k_now = st.k
        orc.iterate(prob, st, oo)
        sl.batch.run(1)
        ex = rel(sl.x(), st.x)
        worst = max(worst, ex)
        assert ex <= tol, (it, "x", ex)
        for i in range(len(sets) + 1):
            yg, vg = sl.arr(sip.FIELD_Y, i), sl.arr(sip.FIELD_V, i)
            yo, vo, wo = st.y[i], st.v[i], st.w_last[i]
            if i < len(sets) and sets[i]["kind"] == "card":
                lines = prob.lines[i] if prob.lines[i] is not None else [np.arange(wo.size)]
                mask = _card_line_mask(wo, sets[i]["k"], lines, 1e-4 if field == "f32" else 1e-10)
                # the k-th entry of every line is always left out; few others
                assert (~mask).sum() <= 1.1 * len(lines) + 0.02 * mask.size
                assert np.array_equal((yg != 0)[mask], (yo != 0)[mask]), (it, i, "card support")
                for idx in lines:
                    assert (yg[idx] != 0).sum() <= sets[i]["k"]
                yg, yo, vg, vo, wo = yg[mask], yo[mask], vg[mask], vo[mask], wo[mask]
            op = "I" if i == len(sets) else sets[i]["op"]
            ncomp = {"I": 1, "DZ": 1, "DY": 1, "DX": 1, "GRAD": m.ndim, "LAT": m.ndim - 1}[op]
            anorm = 1.0 if op == "I" else 2.0 * math.sqrt(ncomp)
            scale = max(np.linalg.norm(yo), np.linalg.norm(wo), anorm * np.linalg.norm(st.x), 1e-30)
            ey = np.linalg.norm(yg - yo) / scale
            ev = np.linalg.norm(vg - vo) / max(np.linalg.norm(vo), scale)
            worst = max(worst, ey, ev)
            assert ey <= tol, (it, i, "y", ey)
            assert ev <= 10 * tol, (it, i, "v", ev)
        if k_now % 5 == 0:
            res = sl.batch.result(sl.slot)
            for i, s in enumerate(sets):
                if s["kind"] == "card":
                    continue  # support decisions near ties move single entries
                a, b = res["r_feas"][i], st.r_feas[i]
                assert abs(a - b) <= (1e-8 if field == "f64" else 2e-3) * max(abs(b), 1e-6), (it, i, a, b)
        rg, gg, kg, _ = sl.batch.get_params(sl.slot)
        assert kg == st.k
        if field == "f64":
            np.testing.assert_allclose(rg, st.rho, rtol=1e-8)
    print(f"[lines step] {kind} {field}: worst rel err {worst:.2e}", flush=True)


@pytest.mark.parametrize("field", ["f64", "f32"])
def test_line_card_exact_ties(field):
    """Integer-valued m: many entries of a line share the k-th magnitude.
    With no CG step x stays m, so the first iteration projects w = A m
    exactly; the kept supports must be those of the oracle bit for bit
    (ties to the lower index along the line)."""
    rng = np.random.default_rng(11)
    m = rng.integers(-3, 4, size=(9, 33)).astype(np.float64)
    sets = wl.finalize(m, [{"kind": "card", "op": "I", "k": 5, "line": "x"},
                           {"kind": "card", "op": "DZ", "k": 2, "line": "z"}])
    print(f"\n[lines ties] {field}", flush=True)
    sl = Slot(m, sets, field, dict(max_iter=1, cg_max=0, cg_fixed=1, adapt_every=0))
    sl.batch.run(1)
    prob = orc.Problem(m, m.shape, sets)
    for i in range(2):
        w = prob.A[i] @ m.ravel()
        yo = orc.project_lines(sets[i], w, prob.lines[i])
        np.testing.assert_array_equal(sl.arr(sip.FIELD_Y, i), yo)
        ties = sum(int((np.abs(w[idx]) == np.sort(np.abs(w[idx]))[::-1][sets[i]["k"] - 1]).sum() > 1)
                   for idx in prob.lines[i])
        print(f"[lines ties] set {i}: {ties} of {len(prob.lines[i])} lines tie at the k-th magnitude", flush=True)
        assert ties > 0


@pytest.mark.parametrize("name", ["length_one_lines", "k_above_length", "tau_zero", "zero_lines_annulus",
                                  "longest_rows_f32", "longest_rows_f64"])
def test_line_edge_cases(name):
    field = "f64"
    if name == "length_one_lines":
        shape, sets = (6, 2), [{"kind": "card", "op": "DX", "k": 1, "line": "x"}, wl.bounds("I", -1, 1)]
    elif name == "k_above_length":
        shape, sets = (7, 5), [{"kind": "card", "op": "DZ", "k": 40, "line": "z"}, wl.l1("GRAD", 0.5)]
    elif name == "tau_zero":
        shape, sets = (6, 9), [{"kind": "l1", "op": "DX", "tau": 0.0, "line": "x"}]
    elif name == "zero_lines_annulus":
        shape, sets = (5, 8), [{"kind": "annulus", "op": "DZ", "lo": 0.2, "hi": 0.5, "line": "z"}]
    elif name == "longest_rows_f32":
        field, shape, sets = "f32", (3, 4097), [{"kind": "card", "op": "DX", "k": 7, "line": "x"},
                                                 {"kind": "l1", "op": "DZ", "tau": 5.0, "line": "z"}]
    else:
        shape, sets = (3, 2049), [{"kind": "l1", "op": "DX", "tau": 3.0, "line": "x"},
                                  {"kind": "card", "op": "I", "k": 9, "line": "z"}]
    rng = np.random.default_rng(zlib.crc32(name.encode()) % 1000)
    m = rng.standard_normal(shape)
    if name == "zero_lines_annulus":
        m[:, 3] = 1.0  # D_z of column 3 is zero: its line takes lo on its first entry
    m = wl.rounded(m, field)
    sets = wl.finalize(m, sets)
    iters = 6
    print(f"\n[lines edge] {name} {field} {shape}", flush=True)
    sl = Slot(m, sets, field, dict(max_iter=iters, cg_max=10, cg_fixed=1, log_schedule=1))
    sl.batch.run(iters)
    res = sl.batch.result(sl.slot)
    assert res["status"] == 0
    rho, gam = sl.batch.schedule(sl.slot, iters)
    xo, _ = orc.parsdmm(m, shape, sets, orc.Options(max_iter=iters, cg_max=10, cg_fixed=True),
                        schedule={k + 1: (rho[k], gam[k]) for k in range(iters)})
    err = rel(sl.x(), xo)
    print(f"[lines edge] {name}: schedule-locked rel err {err:.2e}", flush=True)
    assert err <= (1e-9 if field == "f64" else 1e-4)


def test_line_sets_fullsize_lockstep():
    """The 341x1361 section under the full-waveform example's set list: two
    lockstep iterations against the oracle (supports away from ties)."""
    m, sets, field, iters = wl.layered2d_line_sets()
    m = wl.rounded(m, field)
    sets = wl.finalize(m, sets)
    print(f"\n[lines fullsize] {m.shape}", flush=True)
    sl = Slot(m, sets, field, dict(max_iter=iters, cg_max=10, cg_fixed=1), tiles=(2048, 512, 2048, 512, 512, 1))
    prob = orc.Problem(m, m.shape, sets)
    oo = orc.Options(max_iter=iters, cg_max=10, cg_fixed=True)
    st = orc.initial_state(prob, oo)
    for it in range(2):
        sync_oracle(sl, prob, st)
        orc.iterate(prob, st, oo)
        sl.batch.run(1)
        ex = rel(sl.x(), st.x)
        assert ex <= 1e-5, (it, ex)
        for i, s in enumerate(sets):
            yg, yo, wo = sl.arr(sip.FIELD_Y, i), st.y[i], st.w_last[i]
            lines = prob.lines[i] if prob.lines[i] is not None else [np.arange(wo.size)]
            if s["kind"] == "card":
                mask = _card_line_mask(wo, s["k"], lines, 1e-4)
                assert (~mask).sum() <= 1.1 * len(lines) + 0.02 * mask.size
                assert np.array_equal((yg != 0)[mask], (yo != 0)[mask]), (it, i)
                for idx in lines[:50]:
                    assert (yg[idx] != 0).sum() <= s["k"]
        print(f"[lines fullsize] iteration {it + 1}: x rel err {ex:.2e}", flush=True)
