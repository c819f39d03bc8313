"""Multilevel vs single-level PARSDMM: time to a solution that passes the
stopping rule, on the set list of the paper's timing experiment (bounds,
lateral smoothness, vertical monotonicity) over a seeded layered 2D model and
a seeded smooth 3D model.  Prints one JSON line per (model, levels).

    python -m paper_1902_09699_amd.mlbench --levels 1 2 3
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1902_09699_amd import sip  # noqa: E402
from paper_1902_09699_amd import workloads as wl  # noqa: E402


def models(which):
    out = []
    if "2d" in which:
        m, _, _, _ = wl.layered2d_four_sets()
        sets = [wl.bounds("I", 1.5, 4.5), wl.bounds("DX", -0.02, 0.02), wl.bounds("DZ", 0.0, np.inf)]
        out.append(("layered 341x1361", wl.rounded(m, "f32"), sets))
    if "3d" in which:
        m, _, _, _ = wl.smooth3d_box_tv_lat()
        sets = [wl.bounds("I", -1.0, 1.0), wl.bounds("LAT", -0.02, 0.02), wl.bounds("DZ", 0.0, np.inf)]
        out.append(("smooth 200x200x100", wl.rounded(m, "f32"), sets))
    return out


def run(name, m, sets, nlev, max_iter, coarse_iter, carry, reps):
    import torch
    md = torch.tensor(m, dtype=torch.float32, device="cuda")
    opts = sip.make_opts("f32", max_iter=max_iter, cg_max=10, cg_fixed=0, stop_every=5)
    iters = [max_iter] + [coarse_iter] * (nlev - 1)
    x, res, its = sip.project_multilevel(md, sets, opts, nlev, iters, carry)  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        x, res, its = sip.project_multilevel(md, sets, opts, nlev, iters, carry)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return x, res, its, float(np.median(times))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--levels", type=int, nargs="+", default=[1, 2, 3])
    ap.add_argument("--models", default="2d,3d")
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--coarse-iters", type=int, nargs="+", default=[150],
                    help="iteration caps of the coarser levels to try")
    ap.add_argument("--carry", type=int, nargs="+", default=[0, 1],
                    help="0: levels restart (rho, gamma); 1: carry the coarser level's")
    a = ap.parse_args()
    for name, m, sets in models(a.models):
        sets = wl.finalize(m, sets)
        ref = None
        cases = [(n, c, k) for n in a.levels for c in (a.coarse_iters if n > 1 else [0])
                 for k in (a.carry if n > 1 else [0])]
        for nlev, cap, carry in cases:
            x, res, its, t = run(name, m, sets, nlev, a.max_iter, cap, bool(carry), a.reps)
            xv = x.double().cpu().numpy()
            if ref is None:
                ref = xv
            diff = float(np.linalg.norm(xv - ref) / np.linalg.norm(ref))
            print(json.dumps({"model": name, "levels": nlev, "coarse_cap": cap, "carry_params": carry,
                              "wall_ms": round(1e3 * t, 2),
                              "iterations_per_level": its, "converged": res["converged"],
                              "r_evol": res["r_evol"], "max_r_feas": max(res["r_feas"]),
                              "rel_diff_to_first": diff}), flush=True)


if __name__ == "__main__":
    main()
