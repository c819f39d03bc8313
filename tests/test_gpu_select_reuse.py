"""Reuse of the previous iteration's first selection digit (sip_opts
sel_fresh = 0, the default).  The w pass also gathers the entries of the
first-digit bucket the last selection of the pipeline chose ("list A"); a
selection whose first digit falls in that bucket, with list A holding all of
it, refines over list A instead of every value.  It selects the same entries
(the l1 soft threshold and the cardinality support are fixed by the bucket
counts and sums, not by where they are read), so with float32 fields, whose
bucket sums are exact in float64, every iterate is bit-identical to the run
that reads all of w (sel_fresh = 1); with float64 fields the l1 bucket sums
are accumulated in another order (equal to 1e-10).  The result's sel_reused
count shows that the reuse path ran.  Cases: one refine pass (pipelines up to 2^19 entries),
two refine passes with list A above the candidate cap (a 3D TV ball and a
cardinality set; the 200x200x100 workload), a bucket concentrated in one
w-pass block (more than its LDS stage holds), the stopping test's pipeline,
and a batch of uneven instances."""
import numpy as np
import pytest

from paper_1902_09699_amd import sip
from paper_1902_09699_amd import workloads as wl
from tests.gpu_util import make_case

pytestmark = pytest.mark.gpu


def _case(kind, field):
    if kind == "2d_one_pass":
        m, sets = make_case("four_sets_2d", 5)
    elif kind == "2d_one_pass_large":
        m, sets, _, _ = wl.layered2d_four_sets(n=(341, 1361), seed=1002)
    elif kind == "3d_two_pass":
        rng = wl.rng_for(4321)
        m = wl.grf((96, 96, 64), 6.0, rng)
        sets = [wl.bounds("I", -1.0, 1.0), wl.l1("GRAD", 0.4), wl.card("DX", 0.05)]
    else:
        raise KeyError(kind)
    m = wl.rounded(m, field)
    return m, wl.finalize(m, sets)


def _project(m, sets, field, fresh, **kw):
    import torch
    opts = sip.make_opts(field, sel_fresh=int(fresh), **kw)
    dt = torch.float32 if field == "f32" else torch.float64
    md = torch.tensor(m, dtype=dt, device="cuda")
    x, res = sip.project(md, sets, opts)
    return x.cpu().numpy(), res


def _compare(a, b, field):
    (xa, ra), (xb, rb) = a, b
    assert ra["status"] == rb["status"] == 0
    assert ra["iters"] == rb["iters"] and ra["cg_steps"] == rb["cg_steps"]
    if field == "f32":
        assert np.array_equal(xa, xb)
        assert ra["rho"] == rb["rho"] and ra["gamma"] == rb["gamma"]
    else:
        d = float(np.max(np.abs(xa - xb))) / max(float(np.max(np.abs(xb))), 1e-300)
        assert d <= 1e-10, d
        np.testing.assert_allclose(ra["rho"], rb["rho"], rtol=1e-10)


@pytest.mark.parametrize("field", ["f32", "f64"])
@pytest.mark.parametrize("kind", ["2d_one_pass", "2d_one_pass_large", "3d_two_pass"])
def test_reuse_matches_full_refine(kind, field):
    m, sets = _case(kind, field)
    iters = 40 if kind != "3d_two_pass" else 24
    kw = dict(max_iter=iters, cg_max=10, cg_fixed=1)
    print(f"\n[select reuse] {kind} {field} {m.shape}, {iters} iterations", flush=True)
    fresh = _project(m, sets, field, True, **kw)
    reuse = _project(m, sets, field, False, **kw)
    print(f"[select reuse] selections over list A: {reuse[1]['sel_reused']} "
          f"(of {iters * sum(s['kind'] in ('l1', 'card') for s in sets)})", flush=True)
    assert fresh[1]["sel_reused"] == 0
    assert reuse[1]["sel_reused"] > 0
    _compare(reuse, fresh, field)


def test_reuse_at_200x200x100():
    """The 200x200x100 workload (box, TV ball, lateral slopes) at its own
    size: a TV pipeline of 11.9M entries (two refine passes, list A of
    ~0.35M keys read in chunks, blocks whose stage fills); 40 iterations with
    and without reuse, bit-identical."""
    m, sets, field, _ = wl.smooth3d_box_tv_lat()
    m = wl.rounded(m, field)
    sets = wl.finalize(m, sets)
    kw = dict(max_iter=40, cg_max=10, cg_fixed=1)
    print("\n[select reuse] 200x200x100 f32, 40 iterations", flush=True)
    fresh = _project(m, sets, field, True, **kw)
    reuse = _project(m, sets, field, False, **kw)
    print(f"[select reuse] selections over list A: {reuse[1]['sel_reused']} of 40", flush=True)
    assert fresh[1]["sel_reused"] == 0
    assert reuse[1]["sel_reused"] >= 20
    _compare(reuse, fresh, field)


@pytest.mark.parametrize("field", ["f32", "f64"])
def test_reuse_with_a_full_stage(field):
    """A bucket concentrated in one w-pass block: every entry of the k-th
    magnitude's first-digit bucket lies in the first eight rows (4088
    entries, the first 4096-point item), more than a block stages in LDS
    (1024 float / 512 double keys), so that block appends the rest straight
    to list A."""
    rng = wl.rng_for(5)
    nz, nx = 256, 512
    d = np.empty((nz, nx - 1))
    d[:8] = rng.uniform(0.50, 0.56, size=(8, nx - 1))
    d[8:64] = rng.uniform(1.0, 2.0, size=(56, nx - 1))
    d[64:] = rng.uniform(0.0, 0.1, size=(192, nx - 1))
    d *= rng.choice([-1.0, 1.0], size=d.shape)
    m = np.zeros((nz, nx))
    m[:, 1:] = np.cumsum(d, axis=1)
    m = wl.rounded(m, field)
    sets = wl.finalize(m, [{"kind": "card", "op": "DX", "k": 56 * 511 + 2000}, wl.bounds("I", -1e4, 1e4)])
    kw = dict(max_iter=12, cg_max=10, cg_fixed=1)
    print(f"\n[select reuse] full stage {field} {m.shape}", flush=True)
    fresh = _project(m, sets, field, True, **kw)
    reuse = _project(m, sets, field, False, **kw)
    print(f"[select reuse] selections over list A: {reuse[1]['sel_reused']} of 12", flush=True)
    assert fresh[1]["sel_reused"] == 0
    assert reuse[1]["sel_reused"] > 0
    _compare(reuse, fresh, field)


def test_reuse_with_stopping_pipeline():
    """Stopping-test iterations run a second pipeline (s = A x) per set,
    with its own list A kept from one test to the next: the same iteration
    count, r_feas and r_evol as without reuse."""
    m, sets = _case("2d_one_pass_large", "f32")
    kw = dict(max_iter=150, cg_max=10, cg_fixed=0, stop_every=5)
    print("\n[select reuse] stopping rule on, 341x1361 f32", flush=True)
    fresh = _project(m, sets, "f32", True, **kw)
    reuse = _project(m, sets, "f32", False, **kw)
    print(f"[select reuse] iterations {reuse[1]['iters']}, selections over list A {reuse[1]['sel_reused']}",
          flush=True)
    assert reuse[1]["sel_reused"] > 0
    _compare(reuse, fresh, "f32")
    assert reuse[1]["r_feas"] == fresh[1]["r_feas"] and reuse[1]["r_evol"] == fresh[1]["r_evol"]


def test_reuse_in_a_batch():
    import torch
    insts = []
    for m, sets in wl.batched_instances(12, seed0=2400, max_side=300):
        m = wl.rounded(m, "f32")
        insts.append((m, wl.finalize(m, sets)))
    out = {}
    for fresh in (True, False):
        opts = sip.make_opts("f32", max_iter=30, cg_max=10, cg_fixed=1, sel_fresh=int(fresh))
        ms = [torch.tensor(m, dtype=torch.float32, device="cuda") for m, _ in insts]
        xs, res = sip.project_batched(ms, [s for _, s in insts], opts)
        out[fresh] = ([x.cpu().numpy() for x in xs], res)
    print(f"\n[select reuse] batch of {len(insts)}: selections over list A "
          f"{[r['sel_reused'] for r in out[False][1]]}", flush=True)
    assert sum(r["sel_reused"] for r in out[False][1]) > 0
    for i in range(len(insts)):
        assert out[True][1][i]["sel_reused"] == 0
        _compare((out[False][0][i], out[False][1][i]), (out[True][0][i], out[True][1][i]), "f32")
