"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and its host-only entry points (validation, sizes, option
defaults) behave.  No GPU call is made."""
import math
import os
import re

import numpy as np
import pytest

from paper_1902_09699_amd import sip

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sip.h")).read()
    pat = r"^\s*(?:const\s+char\s*\*|int32_t|int64_t)\s+(sip_[a-z_]+)\s*\("
    return sorted(set(re.findall(pat, text, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(sip.LIB_PATH):
        from paper_1902_09699_amd import build
        build.build()
    return sip.lib()


def test_every_declared_symbol_is_exported(L):
    decl = _declared()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(sip.exported_symbols()) == decl


def test_opts_defaults(L):
    o = sip.make_opts()
    assert (o.max_iter, o.cg_max, o.adapt_every, o.stop_every, o.evol_hist) == (200, 10, 2, 0, 5)
    assert (o.rho0, o.gamma0, o.eps_corr, o.gamma_max, o.cg_rel) == (1.0, 1.0, 0.3, 1.999, 0.1)
    assert (o.eps_evol, o.eps_feas, o.rho_ratio_max) == (1e-2, 1e-3, 100.0)
    assert (o.field, o.reduce, o.log_schedule) == (sip.F32, sip.F64, 0)


def test_reduce_option_validation(L):
    """FP32 reductions (the precision ablation) only with FP32 fields."""
    box = [{"kind": "bounds", "op": "I", "lo": -1, "hi": 1}]
    assert sip.validate((8, 8), box, sip.make_opts("f32", reduce="f32")) == 0
    assert sip.validate((8, 8), box, sip.make_opts("f64", reduce="f64")) == 0
    assert sip.validate((8, 8), box, sip.make_opts("f64", reduce="f32")) == sip.EINVAL
    bad = sip.make_opts("f32")
    bad.reduce = 7
    assert sip.validate((8, 8), box, bad) == sip.EINVAL


def test_rows(L):
    assert sip.set_rows((5, 7), {"kind": "bounds", "op": "DZ"}) == 4 * 7
    assert sip.set_rows((5, 7), {"kind": "bounds", "op": "DX"}) == 5 * 6
    assert sip.set_rows((5, 7), {"kind": "l1", "op": "GRAD"}) == 4 * 7 + 5 * 6
    assert sip.set_rows((4, 5, 6), {"kind": "l1", "op": "GRAD"}) == 3 * 30 + 4 * 4 * 6 + 4 * 5 * 5
    assert sip.set_rows((4, 5, 6), {"kind": "l1", "op": "LAT"}) == 4 * 4 * 6 + 4 * 5 * 5
    assert sip.set_rows((341, 1361), {"kind": "card", "op": "DX"}) == 463760


@pytest.mark.parametrize("shape,sets,ok", [
    ((8, 8), [{"kind": "bounds", "op": "I", "lo": -1, "hi": 1}], True),
    ((8, 8), [{"kind": "bounds", "op": "I", "lo": 1, "hi": -1}], False),
    ((8, 8), [{"kind": "bounds", "op": "DY", "lo": 0, "hi": 1}], False),
    ((1, 8), [{"kind": "bounds", "op": "DZ", "lo": 0, "hi": 1}], False),
    ((1, 8), [{"kind": "bounds", "op": "DX", "lo": 0, "hi": 1}], True),
    ((8, 8), [{"kind": "l1", "op": "GRAD", "tau": -1.0}], False),
    ((8, 8), [{"kind": "l1", "op": "GRAD", "tau": math.inf}], False),
    ((8, 8), [{"kind": "card", "op": "DX", "k": 0}], False),
    ((8, 8), [{"kind": "card", "op": "DX", "k": 56}], True),
    ((8, 8), [{"kind": "card", "op": "DX", "k": 57}], False),
    ((8, 8), [{"kind": "bounds", "op": "I", "lo": -1, "hi": 1}] * 17, False),
    ((8, 8, 8), [{"kind": "bounds", "op": "LAT", "lo": -1, "hi": 1}], True),
])
def test_validation(L, shape, sets, ok):
    assert (sip.validate(shape, sets, sip.make_opts()) == 0) == ok


def test_workspace_bytes_exact_and_monotone(L):
    o = sip.make_opts()
    a = sip.workspace_bytes((64, 64), [{"kind": "bounds", "op": "I", "lo": -1, "hi": 1}], o)
    b = sip.workspace_bytes((64, 64), [{"kind": "bounds", "op": "I", "lo": -1, "hi": 1},
                                       {"kind": "l1", "op": "GRAD", "tau": 1.0}], o)
    assert a > 0 and b > a and a % 256 == 0 and b % 256 == 0
    assert sip.workspace_bytes((64, 64), [{"kind": "bounds", "op": "I", "lo": 2, "hi": 1}], o) == -1
    o64 = sip.make_opts("f64")
    assert sip.workspace_bytes((64, 64), [{"kind": "bounds", "op": "I", "lo": -1, "hi": 1}], o64) > a


def test_strerror(L):
    assert sip.strerror(0) == "ok"
    assert "invalid" in sip.strerror(-1)


@pytest.mark.parametrize("shape,nlev", [((21, 41), 3), ((341, 1361), 3), ((9, 12, 14), 2), ((1, 9), 2)])
def test_level_grids_and_sets_match_oracle(L, shape, nlev):
    """sip_level (the library's multilevel grids and set parameters) against
    the multilevel oracle's definitions."""
    from oracle import multilevel as ml
    ndim = len(shape)
    sets = [{"kind": "bounds", "op": "I", "lo": -1.0, "hi": 1.0},
            {"kind": "l1", "op": "GRAD" if shape[0] > 1 else "DX", "tau": 57.0},
            {"kind": "card", "op": "DX", "k": 7}]
    if ndim == 3:
        sets.append({"kind": "bounds", "op": "LAT", "lo": -0.1, "hi": 0.1})
    shapes = ml.level_shapes(shape, nlev)
    for lev in range(nlev):
        shp, got = sip.level(shape, sets, lev)
        assert shp == shapes[lev]
        want = ml.level_sets(sets, shape, shapes[lev])
        for a, b in zip(got, want):
            assert a["kind"] == b["kind"] and a["op"] == b["op"]
            if a["kind"] == "l1":
                assert abs(a["tau"] - b["tau"]) <= 1e-12 * b["tau"]
            elif a["kind"] == "card":
                assert a["k"] == b["k"]
            else:
                assert (a["lo"], a["hi"]) == (b["lo"], b["hi"])


@pytest.mark.parametrize("s,ok", [
    ({"kind": "l2", "op": "GRAD", "tau": 1.0}, True),
    ({"kind": "l2", "op": "GRAD", "tau": -1.0}, False),
    ({"kind": "annulus", "op": "I", "lo": 0.5, "hi": 2.0}, True),
    ({"kind": "annulus", "op": "I", "lo": 2.0, "hi": 0.5}, False),
    ({"kind": "annulus", "op": "I", "lo": -0.1, "hi": 0.5}, False),
    ({"kind": "annulus", "op": "I", "lo": 0.0, "hi": np.inf}, True),
])
def test_validation_l2_and_annulus(L, s, ok):
    assert (sip.validate((8, 9), [s], sip.make_opts()) == 0) == ok


def test_bound_vectors_only_for_bounds(L):
    """A bound-vector pointer on a non-bounds set is rejected (validation
    only reads the pointer's presence)."""
    g = sip.make_grid((8, 9))
    arr = sip.make_sets([{"kind": "l1", "op": "DX", "tau": 1.0}])
    arr[0].lo_vec = 16  # any non-null address
    assert sip.lib().sip_validate(sip.C.byref(g), arr, 1, sip.C.byref(sip.make_opts())) == sip.EINVAL
    arr = sip.make_sets([{"kind": "bounds", "op": "DX", "lo": -1.0, "hi": 1.0}])
    arr[0].hi_vec = 16
    assert sip.lib().sip_validate(sip.C.byref(g), arr, 1, sip.C.byref(sip.make_opts())) == 0


@pytest.mark.parametrize("shape,s,field,rc", [
    ((8, 9), {"kind": "card", "op": "DX", "k": 2, "line": "x"}, "f32", 0),
    ((8, 9), {"kind": "card", "op": "DZ", "k": 50, "line": "z"}, "f32", 0),     # k above the line length: keep all
    ((8, 9), {"kind": "l1", "op": "GRAD", "tau": 1.0, "line": "z"}, "f64", 0),
    ((4, 5, 6), {"kind": "l2", "op": "LAT", "tau": 1.0, "line": "y"}, "f32", 0),
    ((4, 5, 6), {"kind": "annulus", "op": "I", "lo": 0.5, "hi": 1.0, "line": "x"}, "f64", 0),
    ((8, 9), {"kind": "l1", "op": "DX", "tau": 1.0, "line": "y"}, "f32", "EINVAL"),  # no y axis in 2D
    ((8, 9), {"kind": "bounds", "op": "I", "lo": 0, "hi": 1, "line": "x"}, "f32", "EINVAL"),
    ((3, 4097), {"kind": "card", "op": "I", "k": 2, "line": "x"}, "f32", "EUNSUPPORTED"),
    ((3, 4097), {"kind": "card", "op": "DX", "k": 2, "line": "x"}, "f32", 0),  # D_x rows hold 4096
    ((3, 2049), {"kind": "card", "op": "I", "k": 2, "line": "x"}, "f64", "EUNSUPPORTED"),
    ((3, 2049), {"kind": "card", "op": "I", "k": 2, "line": "z"}, "f64", 0),
])
def test_validation_line_sets(L, shape, s, field, rc):
    want = 0 if rc == 0 else getattr(sip, rc)
    assert sip.validate(shape, [s], sip.make_opts(field)) == want


def test_multilevel_rejects_line_sets_on_host(L):
    """The multilevel entry point refuses line-wise sets before touching the
    device (null device pointers are never dereferenced on this path)."""
    g = sip.make_grid((16, 16))
    arr = sip.make_sets([{"kind": "l1", "op": "DX", "tau": 1.0, "line": "x"}])
    iters = (sip.C.c_int32 * 2)(5, 5)
    res = sip.Result()
    rc = sip.lib().sip_project_multilevel(sip.C.byref(g), arr, 1, sip.C.byref(sip.make_opts()), 2, iters, 0,
                                          sip.C.c_void_p(16), sip.C.c_void_p(16), sip.C.byref(res), None, None)
    assert rc == sip.EUNSUPPORTED


def test_plan_sizes(L):
    """A plan's device bytes: the instance workspace plus its descriptor,
    scalars and work tables; the default tiles are the library's; invalid
    sets or tiles give -1."""
    box_tv = [{"kind": "bounds", "op": "I", "lo": -1, "hi": 1}, {"kind": "l1", "op": "GRAD", "tau": 3.0}]
    o = sip.make_opts("f32")
    t = sip.make_tiles()
    assert (t.pt_points, t.pt_max_items, t.thr_points, t.thr_max_items, t.pt_threads, t.cg_form) == \
        (2048, 512, 2048, 512, 512, 0)
    ws = sip.workspace_bytes((64, 80), box_tv, o)
    pb = sip.plan_bytes((64, 80), box_tv, o)
    assert ws < pb < ws + (1 << 20)
    assert pb % 256 == 0
    # finer tiles need more table entries and partial sums
    assert sip.plan_bytes((640, 800), box_tv, o, (256, 4096, 256, 4096, 256, 0)) > \
        sip.plan_bytes((640, 800), box_tv, o)
    assert sip.plan_bytes((64, 80), [{"kind": "l1", "op": "GRAD", "tau": -1.0}], o) == -1
    assert sip.plan_bytes((64, 80), box_tv, o, (100, 512, 2048, 512, 512, 0)) == -1
    assert sip.plan_bytes((64, 80), box_tv, o, (2048, 512, 2048, 512, 384, 0)) == -1
