"""The allocation-free entry point (sip_project_noalloc) through the C ABI:
two calls in a row, the second on a smaller instance, each equal to
sip_project on the same input (bitwise for float fields: the same kernels
in the same order, with every device buffer taken from the library's fixed
array instead of the allocator); an instance beyond the array is refused
before any GPU work."""
import numpy as np
import pytest

from paper_1902_09699_amd import sip
from paper_1902_09699_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _dev(m, field):
    import torch
    return torch.tensor(m, dtype=torch.float64 if field == "f64" else torch.float32, device="cuda")


def _check(m, sets, field, opts):
    """Float fields: bitwise equal.  Double fields sum the l1 radix buckets
    with double atomics, whose order (so the last bits) varies from run to
    run: equal to 1e-10."""
    md = _dev(m, field)
    xr, rr = sip.project(md, sets, opts)
    xn, rn = sip.project_noalloc(md, sets, opts)
    a, b = xn.double().cpu().numpy(), xr.double().cpu().numpy()
    for key in ("status", "iters", "cg_steps", "converged"):
        assert rn[key] == rr[key], key
    if field == "f32":
        assert np.array_equal(a, b)
        for key in ("r_evol", "r_feas", "rho", "gamma"):
            assert rn[key] == rr[key], key
    else:
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)
        for key in ("r_evol", "r_feas", "rho", "gamma"):
            np.testing.assert_allclose(rn[key], rr[key], rtol=1e-7, atol=0)
    return rn


@pytest.mark.parametrize("field", ["f32", "f64"])
def test_noalloc_equals_project_twice_second_smaller(field):
    opts = sip.make_opts(field, max_iter=40, cg_max=10, cg_fixed=1)
    big, sets, _, _ = wl.layered2d_four_sets(n=(173, 311), seed=7)
    big = wl.rounded(big, field)
    print(f"\n[noalloc] {field} first call {big.shape}", flush=True)
    _check(big, wl.finalize(big, sets), field, opts)
    small, sets2, _, _ = wl.smooth2d_box_tv(n=(37, 45), seed=8)
    small = wl.rounded(small, field)
    print(f"[noalloc] {field} second call {small.shape}", flush=True)
    _check(small, wl.finalize(small, sets2), field, opts)


def test_noalloc_stopping_rule_and_3d():
    opts = sip.make_opts("f32", max_iter=60, cg_max=10, cg_fixed=0, stop_every=5)
    m, sets, _, _ = wl.smooth3d_box_tv_lat(n=(21, 26, 31), seed=9)
    m = wl.rounded(m, "f32")
    print("\n[noalloc] 3D with the stopping rule", flush=True)
    _check(m, wl.finalize(m, sets), "f32", opts)


def test_noalloc_refuses_an_instance_beyond_its_array():
    import torch
    opts = sip.make_opts("f32", max_iter=2)
    shape = (200, 200, 100)
    sets = [{"kind": "bounds", "op": "I", "lo": -1.0, "hi": 1.0}, {"kind": "l1", "op": "GRAD", "tau": 10.0},
            {"kind": "bounds", "op": "LAT", "lo": -0.05, "hi": 0.05}]
    assert sip.plan_bytes(shape, sets, opts) > 128 << 20
    m = torch.zeros(shape, dtype=torch.float32, device="cuda")
    with pytest.raises(sip.SipError) as e:
        sip.project_noalloc(m, sets, opts)
    assert e.value.status == sip.ETOOLARGE
