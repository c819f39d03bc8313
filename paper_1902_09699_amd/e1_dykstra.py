"""Synthetic re-run of the paper's first PARSDMM vs parallel Dykstra
comparison (section "Parallel Dykstra versus PARSDMM"): a 341x400 layered
stand-in for the geological model, projected onto bounds, an anisotropic TV
ball and vertical monotonicity.  Both methods run on this library's kernels;
the relative transform-domain feasibility of every set (eq. feas_stop) is
recorded against the paper's cost counts: CG steps (parallel Dykstra: the
slowest of its parallel sub-problems per outer iteration) and l1-ball
projections (PARSDMM: one per iteration; Dykstra: the inner iterations of the
TV sub-problem).  Prints one JSON line per method (traces and the counts at
which every set's feasibility first drops below each threshold).

    python -m paper_1902_09699_amd.e1_dykstra
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1902_09699_amd import dykstra as ddk  # noqa: E402
from paper_1902_09699_amd import sip  # noqa: E402
from paper_1902_09699_amd import workloads as wl  # noqa: E402


def e1_problem(shape=(341, 400), seed=1005, tv_frac=0.5):
    m = wl.layered(shape, wl.rng_for(seed))
    sets = [wl.bounds("I", 1.5, 4.5), wl.l1("GRAD", tv_frac), wl.bounds("DZ", 0.0, np.inf)]
    return m, wl.finalize(m, sets)


class FeasProbe:
    """r_feas of a given x for every set, computed by the library: one
    iteration with no CG step (x stays the given model) and the stopping
    test at k = 1."""

    def __init__(self, x_like, sets, field):
        import torch
        self.opts = sip.make_opts(field, max_iter=1, cg_max=0, stop_every=1, evol_hist=1, eps_feas=0.0,
                                  eps_evol=0.0, adapt_every=0)
        self.buf = torch.empty_like(x_like)
        self.src = x_like.clone()
        self.b = sip.Batch(1, sip.workspace_bytes(tuple(x_like.shape), sets, self.opts), self.opts)
        self.slot = self.b.add(self.src, sets, self.buf)

    def __call__(self, x):
        self.src.copy_(x)
        self.b.reset(self.slot, self.src)
        self.b.run(1)
        return list(self.b.result(self.slot)["r_feas"])

    def close(self):
        self.b.close()


def first_reach(trace, key, t):
    for row in trace:
        if max(row["r_feas"]) <= t:
            return row[key]
    return None


def run_parsdmm(md, sets, field, iters, tiles):
    opts = sip.make_opts(field, max_iter=iters, cg_max=10, cg_fixed=1, stop_every=1, evol_hist=1,
                         eps_feas=0.0, eps_evol=0.0)
    import torch
    x = torch.empty_like(md)
    b = sip.Batch(1, sip.workspace_bytes(tuple(md.shape), sets, opts), opts)
    if tiles:
        b.set_tiles(*tiles)
    sl = b.add(md, sets, x)
    trace = []
    for k in range(1, iters + 1):
        b.run(1)
        r = b.result(sl)
        trace.append({"iter": k, "cg": r["cg_steps"], "l1": k, "r_feas": list(r["r_feas"]),
                      "rel_change": r["r_evol"]})
    b.close()
    return trace


def run_dykstra(md, sets, field, outer, inner_iters, inner_eps, tiles, probe):
    import torch
    inner = sip.make_opts(field, max_iter=inner_iters, cg_max=10, cg_fixed=1, stop_every=5 if inner_eps else 0,
                          eps_feas=inner_eps or 0.0, eps_evol=inner_eps or 0.0)
    dk = ddk.ParallelDykstra(md, sets, inner, tiles=tiles)
    tv = [i for i, s in enumerate(sets) if s["kind"] == "l1"][0]
    trace, cg, l1 = [], 0, 0
    prev = md.clone()
    for k in range(1, outer + 1):
        dk.step()
        cg += max(dk.log.cg_steps[-1])
        l1 += dk.log.iters[-1][tv]
        nx = float(torch.linalg.vector_norm(dk.x.double()))
        ch = float(torch.linalg.vector_norm((dk.x - prev).double())) / max(nx, 1e-300)
        prev.copy_(dk.x)
        trace.append({"iter": k, "cg": cg, "l1": l1, "r_feas": probe(dk.x), "rel_change": ch})
    dk.close()
    return trace


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--field", default="f32", choices=("f32", "f64"))
    ap.add_argument("--parsdmm-iters", type=int, default=400)
    ap.add_argument("--outer", type=int, default=60)
    ap.add_argument("--inner", default="50:1e-3,200:1e-3,50:1e-2,25:0",
                    help="inner settings to try, max_iter:eps (eps 0: no inner stopping test)")
    ap.add_argument("--thresholds", type=float, nargs="+", default=[1e-1, 1e-2, 1e-3])
    ap.add_argument("--tiles", default="2048,512,2048,512,512,1")
    a = ap.parse_args()
    import torch
    m, sets = e1_problem()
    m = wl.rounded(m, a.field)
    sets = wl.finalize(m, sets)
    md = torch.tensor(m, dtype=torch.float64 if a.field == "f64" else torch.float32, device="cuda")
    tiles = tuple(int(v) for v in a.tiles.split(",")) if a.tiles else None
    probe = FeasProbe(md, sets, a.field)

    def summary(name, trace, extra):
        out = {"method": name, "grid": list(m.shape), **extra,
               "reach": {f"{t:g}": {"cg": first_reach(trace, "cg", t), "l1": first_reach(trace, "l1", t)}
                         for t in a.thresholds},
               "final": {"iter": trace[-1]["iter"], "cg": trace[-1]["cg"], "l1": trace[-1]["l1"],
                         "r_feas": trace[-1]["r_feas"], "rel_change": trace[-1]["rel_change"]},
               "trace": [[r["cg"], r["l1"], max(r["r_feas"])] for r in trace]}
        print(json.dumps(out), flush=True)

    summary("PARSDMM", run_parsdmm(md, sets, a.field, a.parsdmm_iters, tiles), {"iterations": a.parsdmm_iters})
    for spec in a.inner.split(","):
        it, eps = spec.split(":")
        tr = run_dykstra(md, sets, a.field, a.outer, int(it), float(eps), tiles, probe)
        summary("parallel Dykstra", tr, {"outer": a.outer, "inner_max_iter": int(it), "inner_eps": float(eps)})
    probe.close()


if __name__ == "__main__":
    main()
