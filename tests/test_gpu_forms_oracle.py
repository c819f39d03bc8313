"""The batched and served forms against the FP64 oracle (needs an MI355X).

Batched: an uneven batch of the benchmark's instance mix with autotuned
tiles; sampled instances (TV balls, l1 balls on D_z, cardinality sets) are
compared with the oracle replaying each instance's (rho, gamma) schedule and
kept cardinality rows, and the same batch advanced in captured chunks of 10
iterations is bit-identical to the one advanced an iteration at a time.
Served: a small float32 mix with the stopping rule (every 5 iterations) and
the relative CG stop, 2D and 3D requests arriving together into a resident
batch with continuous admission; each checked result is compared with the
oracle replaying the device's (rho, gamma) and CG step counts: same
iteration count and stopping decision, r_feas and r_evol, x within 1e-5."""
import numpy as np
import pytest

from oracle import parsdmm as orc
from paper_1902_09699_amd import autotune, serve, sip
from paper_1902_09699_amd import workloads as wl
from tests.gpu_util import card_sets, rel, replay_locked, slot_rows

pytestmark = pytest.mark.gpu


def _kinds(sets):
    out = set()
    for s in sets:
        if s["kind"] == "l1":
            out.add("tv" if s["op"] == "GRAD" else "l1dz")
        elif s["kind"] == "card":
            out.add("card")
    return out


def test_batched_instances_match_oracle():
    import torch
    B = 20
    iters = 16
    insts = []
    for m, sets in wl.batched_instances(B):
        m = wl.rounded(m, "f32")
        insts.append((m, wl.finalize(m, sets)))
    # sampled instances: one per kind of threshold set, and the largest
    picks = []
    for want in ("tv", "l1dz", "card"):
        j = next(j for j, (m, s) in enumerate(insts) if want in _kinds(s) and j not in picks)
        picks.append(j)
    picks.append(max((j for j in range(B) if j not in picks), key=lambda j: insts[j][0].size))
    print(f"\n[batched] {B} instances, {sum(m.size for m, _ in insts)} points; checked {picks}", flush=True)
    opts = sip.make_opts("f32", max_iter=iters, cg_max=10, cg_fixed=1, log_schedule=1)
    arena = sum(sip.workspace_bytes(m.shape, s, opts) for m, s in insts)
    ms = [torch.tensor(m, dtype=torch.float32, device="cuda") for m, _ in insts]

    def make():
        b = sip.Batch(B, arena, opts)
        xs = [torch.empty_like(md) for md in ms]
        slots = [b.add(md, s, x) for md, (_, s), x in zip(ms, insts, xs)]
        return b, xs, slots

    b1, xs1, slots1 = make()
    tiles, _ = autotune.tune(b1, slots1, ms, "f32", [m.shape for m, _ in insts], iters=3, use_cache=False,
                             cache=None)
    print(f"[batched] autotuned tiles {tiles}", flush=True)
    for sl, md in zip(slots1, ms):
        b1.reset(sl, md)
    sup = {j: {} for j in picks}
    for k in range(1, iters + 1):
        b1.run(1)
        for j in picks:
            m, sets = insts[j]
            sup[j][k] = {i: np.nonzero(slot_rows(b1, slots1[j], m.shape, sets, sip.FIELD_Y, i))[0]
                         for i in card_sets(sets)}
    torch.cuda.synchronize()
    # the same batch in captured chunks of 10 iterations: bit-identical
    b2, xs2, slots2 = make()
    b2.set_tiles(*tiles)
    b2.run(10)
    b2.run(iters - 10)
    torch.cuda.synchronize()
    for j in range(B):
        assert torch.equal(xs1[j], xs2[j]), j
    b2.close()
    oo = orc.Options(max_iter=iters, cg_max=10, cg_fixed=True)
    for j in picks:
        m, sets = insts[j]
        rho, gam = b1.schedule(slots1[j], iters)
        res = b1.result(slots1[j])
        assert res["status"] == 0 and res["iters"] == iters
        sched = {k + 1: (rho[k], gam[k]) for k in range(iters)}
        st, rep, _ = replay_locked(m, sets, oo, sched, sup[j] if card_sets(sets) else None)
        err = rel(xs1[j].double().cpu().numpy(), st.x)
        kinds = [f"{s['kind']}({s['op']})" for s in sets]
        print(f"[batched] instance {j} {m.shape} {kinds}: rel err vs oracle {err:.2e}, card entries chosen "
              f"differently {sum(r[3] for r in rep)}", flush=True)
        assert all(r[2] for r in rep)
        assert err <= 1e-5
    b1.close()


def _served_mix():
    reqs = serve.make_requests(10, rate=1e9, frac3d=0.3, seed0=5100, max2d=160, side3d=(20, 28))
    assert any(r.m.ndim == 3 for r in reqs)
    return reqs


def test_served_results_match_oracle():
    opts = sip.make_opts("f32", max_iter=80, cg_max=10, cg_fixed=0, stop_every=5, log_schedule=1)
    reqs = _served_mix()
    need = [sip.workspace_bytes(r.m.shape, r.sets, opts) for r in reqs]
    arena = 4 * max(need)                      # at most a few resident at once: admission as slots free up
    logs = {}

    def on_chunk(batch, active):
        # after every chunk (one iteration here): per request, the CG steps and
        # the cardinality rows of the iteration that just ran
        for slot, (r, _, _, _) in active.items():
            res = batch.result(slot)
            lg = logs.setdefault(r.rid, {"cg": [], "sup": {}, "n": 0})
            if res["iters"] > lg["n"]:
                lg["cg"].append(res["cg_steps"] - sum(lg["cg"]))
                lg["n"] = res["iters"]
                cs = card_sets(r.sets)
                if cs:
                    lg["sup"][res["iters"]] = {i: np.nonzero(slot_rows(batch, slot, r.m.shape, r.sets, sip.FIELD_Y,
                                                                       i))[0] for i in cs}

    def on_done(batch, slot, r):
        rho, gam = batch.schedule(slot, opts.max_iter)
        logs[r.rid]["sched"] = (rho, gam)

    srv = serve.Server(opts, arena, max_slots=6, chunk=1)
    info = srv.run(reqs, realtime=False, on_chunk=on_chunk, on_done=on_done)
    srv.close()
    print(f"\n[served] {len(reqs)} requests ({sum(r.m.ndim == 3 for r in reqs)} 3D), peak arena "
          f"{info['peak_arena_bytes']} of {arena}, chunks {info['chunks']}", flush=True)
    assert info["rejected"] == 0
    oo = orc.Options(max_iter=opts.max_iter, cg_max=10, cg_fixed=False, stop_every=5)
    checked = 0
    for r in reqs:
        res = r.result
        assert res["status"] == 0
        lg = logs[r.rid]
        rho, gam = lg["sched"]
        n = res["iters"]
        assert len(lg["cg"]) == n and rho.shape[0] == n
        sched = {k + 1: (rho[k], gam[k], lg["cg"][k]) for k in range(n)}
        st, rep, cgrep = replay_locked(r.m, r.sets, oo, sched, lg["sup"] or None)
        err = rel(r.x, st.x)
        cg_diff = sum(c[2] for c in cgrep)
        print(f"[served] request {r.rid} {r.m.shape} {[s['kind'] + '(' + s['op'] + ')' for s in r.sets]}: "
              f"device {n} iterations converged {res['converged']}, oracle {st.k - 1} converged {st.converged}; "
              f"rel err {err:.2e}; r_evol {res['r_evol']:.4e} / {st.r_evol:.4e}; CG decisions differing from "
              f"the oracle's own {cg_diff} of {len(cgrep)}", flush=True)
        assert all(c[1] for c in cgrep), [c for c in cgrep if not c[1]][:3]
        assert all(x[2] for x in rep)
        assert st.k - 1 == n and bool(st.converged) == bool(res["converged"])
        assert err <= 1e-5
        if res["converged"]:
            np.testing.assert_allclose(res["r_feas"], st.r_feas, rtol=1e-3, atol=1e-7)
            assert res["r_evol"] == pytest.approx(st.r_evol, rel=1e-3)
        checked += 1
    assert checked >= 3
