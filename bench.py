"""Benchmark: PARSDMM grid-points x iterations per second on one MI355X.

One step = one complete projection (state reset from m, then every
iteration of the PARSDMM listing) of the chosen workload, inputs resident in
HBM.  Prints one JSON line with the throughput, the roofline of the dominant
kernel (algorithmic bytes per launch over its HIP-event-timed mean launch
duration, against the 8 TB/s HBM peak) and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = ("layered2d", "layered2d_lines", "smooth2d", "smooth3d", "batched")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="layered2d", choices=WORKLOADS)
    ap.add_argument("--graph-iters", type=int, default=50)
    ap.add_argument("--reps", type=int, default=30, help="launches per kernel timing")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU oracle sample budget (0: skip)")
    ap.add_argument("--batched-count", type=int, default=256)
    ap.add_argument("--copy-mb", type=int, default=1024, help="plain-copy reference size (0: skip)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tiles")
    ap.add_argument("--reduce", default="f64", choices=("f64", "f32"),
                    help="reduction type (f32: the pure-FP32 precision ablation)")
    ap.add_argument("--check-iters", type=int, default=10,
                    help="iterations of the schedule-locked error check against the oracle (0: skip)")
    ap.add_argument("--tiles", default=None,
                    help="fixed tiles pt_points,pt_max_items,thr_points,thr_max_items[,pt_threads[,cg_form]] "
                         "(no autotune)")
    return ap.parse_args()


def workload(name, args):
    from paper_1902_09699_amd import workloads as wl
    if name == "layered2d":
        m, sets, field, iters = wl.layered2d_four_sets()
        desc = "layered 341x1361 f32: box, D_z>=0, l1(D_x), card(D_x); 300 it x 10 CG"
    elif name == "smooth2d":
        m, sets, field, iters = wl.smooth2d_box_tv()
        desc = "smooth 64x64 f64: box, TV ball; 200 it x 10 CG"
    elif name == "layered2d_lines":
        m, sets, field, iters = wl.layered2d_line_sets()
        desc = ("layered 341x1361 f32: box, card(D_z) <= nx, card(D_x) <= nz, card <= 2 of D_x per row and of "
                "D_z per column; 300 it x 10 CG")
    elif name == "smooth3d":
        m, sets, field, iters = wl.smooth3d_box_tv_lat()
        desc = "smooth 200x200x100 f32: box, TV ball, lateral slopes; 200 it x 10 CG"
    else:
        raise ValueError(name)
    m = wl.rounded(m, field)
    return [(m, wl.finalize(m, sets))], field, iters, desc


def batched_workload(args):
    from paper_1902_09699_amd import workloads as wl
    out = []
    for m, sets in wl.batched_instances(args.batched_count):
        m = wl.rounded(m, "f32")
        out.append((m, wl.finalize(m, sets)))
    return out, "f32", 200, f"{args.batched_count} uneven 2D instances (sides U[32,512]), 2-5 sets; 200 it x 10 CG"


def rows(shape, s):
    from paper_1902_09699_amd import workloads as wl
    return wl.rows_of(shape, s["op"])


def algorithmic_bytes(insts, esz):
    """Compulsory bytes of one launch of each kernel (all instances):
    CG direction: read r, p, write p (3N); CG update: read x, r, p, write x, r
    (5N); one-reduction CG step: read x, p, r, w, s, write all five (10N);
    its w_0 pass: read r, write w (2N); RHS: read x and every y_i, v_i (identity block included), write r;
    projection (non-adapt iteration): read x, m, y_i, v_i of the bounds sets
    and the identity block, write y_i, v_i; threshold w pass: read x, y_i,
    v_i, write w over y_i (N + 3 M_i per l1 / cardinality set); threshold
    apply pass: read w, write y_i, v_i (3 M_i); line-wise sets: read x, y_i, v_i,
    write y_i, v_i (N + 4 M_i)."""
    b = {"cg_dir": 0, "cg_upd": 0, "cg1_step": 0, "cg1_w0": 0, "rhs": 0, "proj": 0, "thr_w": 0, "thr_apply": 0,
         "line": 0}
    for m, sets in insts:
        N = m.size
        sum_m = N + sum(rows(m.shape, s) for s in sets)
        clip = N + sum(rows(m.shape, s) for s in sets if s["kind"] == "bounds")
        thr = [rows(m.shape, s) for s in sets if s["kind"] != "bounds" and s.get("line") is None]
        line = [rows(m.shape, s) for s in sets if s.get("line") is not None]
        b["cg_dir"] += 3 * N * esz
        b["cg_upd"] += 5 * N * esz
        b["cg1_step"] += 10 * N * esz
        b["cg1_w0"] += 2 * N * esz
        b["rhs"] += (2 * N + 2 * sum_m) * esz
        b["proj"] += (2 * N + 4 * clip) * esz
        b["thr_w"] += sum(N + 3 * mi for mi in thr) * esz
        b["thr_apply"] += sum(3 * mi for mi in thr) * esz
        b["line"] += sum(N + 4 * mi for mi in line) * esz
    return b


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("sip_kernels.hip", "sip_internal.h"):
        with open(os.path.join(ROOT, "paper_1902_09699_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, wname):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{wname}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def device_reference(inst, field, reduce, iters, tiles=None):
    """The first instance alone on the device for `iters` iterations with the
    (rho, gamma) schedule logged (tiles and CG form as timed): its x and the
    schedule."""
    import torch
    from paper_1902_09699_amd import sip
    m, sets = inst
    opts = sip.make_opts(field, reduce=reduce, max_iter=iters, cg_max=10, cg_fixed=1, log_schedule=1)
    md = torch.tensor(m, dtype=torch.float64 if field == "f64" else torch.float32, device="cuda")
    xd = torch.empty_like(md)
    b = sip.Batch(1, sip.workspace_bytes(m.shape, sets, opts), opts)
    if tiles:
        b.set_tiles(*tiles)
    slot = b.add(md, sets, xd)
    b.run(iters)
    rho, gam = b.schedule(slot, iters)
    x = xd.double().cpu().numpy()
    b.close()
    return x, {k + 1: (rho[k], gam[k]) for k in range(len(rho))}


def oracle_sensitivity(inst, iters, schedule, field):
    """How far the oracle's own x moves after `iters` iterations (same
    schedule) when m is perturbed by one unit roundoff of the field type:
    the scale an error against the oracle is to be read on."""
    from oracle import parsdmm as orc
    m, sets = inst
    u = 2.0 ** -24 if field == "f32" else 2.0 ** -53
    mp = m * (1.0 + u * np.random.default_rng(5).standard_normal(m.shape))
    oo = orc.Options(max_iter=iters, cg_max=10, cg_fixed=True)
    xa, _ = orc.parsdmm(m, m.shape, sets, oo, schedule=schedule)
    xb, _ = orc.parsdmm(mp, m.shape, sets, oo, schedule=schedule)
    return float(np.linalg.norm(xb - xa) / max(np.linalg.norm(xa), 1e-300))


def cpu_baseline(insts, iters_full, budget_s, schedule=None, check=None):
    """The FP64 oracle as it stands, on the first instance, for as many
    iterations as fit the budget (at least 2), replaying the device's (rho,
    gamma) schedule where one is given; check = (k, x_device) compares the
    oracle's x after iteration k with the device's."""
    from oracle import parsdmm as orc
    m, sets = insts[0]
    prob = orc.Problem(m, m.shape, sets)
    opts = orc.Options(max_iter=iters_full, cg_max=10, cg_fixed=True)
    st = orc.initial_state(prob, opts)
    err = None

    def step():
        nonlocal err
        orc.iterate(prob, st, opts, schedule)
        if check is not None and st.k - 1 == check[0]:
            xo = st.x.ravel()
            err = float(np.linalg.norm(check[1].ravel() - xo) / max(np.linalg.norm(xo), 1e-300))

    step()  # first iteration: warm-up, untimed
    ru0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    done = 0
    while done < 2 or (time.perf_counter() - t0 < budget_s and st.k <= iters_full) or \
            (check is not None and err is None and st.k <= check[0]):
        step()
        done += 1
    wall = time.perf_counter() - t0
    ru1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (ru1.ru_utime - ru0.ru_utime) + (ru1.ru_stime - ru0.ru_stime)
    cores = max(1, int(round(cpu / wall)))
    out = {"value": m.size * done / wall, "unit": "grid-pts*iters/s", "cores": cores, "kind": "oracle",
           "sample": f"iterations 2..{done + 1} of the first instance ({m.shape}), FP64 CSR oracle, "
                     f"{wall:.1f} s wall, {cpu:.1f} s CPU"}
    return out, err


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1902_09699_amd import sip

    if args.workload == "batched":
        insts, field, iters, desc = batched_workload(args)
    else:
        insts, field, iters, desc = workload(args.workload, args)
    esz = 8 if field == "f64" else 4
    dt = torch.float64 if field == "f64" else torch.float32
    opts = sip.make_opts(field, reduce=args.reduce, max_iter=iters, cg_max=10, cg_fixed=1)
    ms = [torch.tensor(m, dtype=dt, device="cuda") for m, _ in insts]
    xs = [torch.empty_like(m) for m in ms]
    arena = sum(sip.workspace_bytes(m.shape, s, opts) for m, s in insts)
    batch = sip.Batch(len(insts), arena, opts)
    slots = [batch.add(md, s, xd) for md, (_, s), xd in zip(ms, insts, xs)]
    assert all(s >= 0 for s in slots)
    chunk = min(args.graph_iters, iters)
    n_pts = sum(m.size for m, _ in insts)
    tiles = None
    if args.tiles:
        tiles = tuple(int(v) for v in args.tiles.split(","))
        batch.set_tiles(*tiles)
    elif not args.no_autotune:
        from paper_1902_09699_amd import autotune
        tiles, tile_ms = autotune.tune(batch, slots, ms, field, [m.shape for m, _ in insts], use_cache=False,
                                       cache=None)
        for cand, t in sorted(tile_ms.items(), key=lambda kv: kv[1])[:6]:
            print(f"autotune {cand}: {1e3 * t:.1f} us/iteration", file=sys.stderr, flush=True)

    def one_step():
        for sl, md in zip(slots, ms):
            batch.reset(sl, md)
        left = iters
        while left > 0:
            n = min(chunk, left)
            batch.run(n)
            left -= n

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    results = [batch.result(sl) for sl in slots]
    assert all(r["status"] == 0 and r["iters"] == iters for r in results), results[:3]
    value = n_pts * iters * args.steps / wall
    ms_step = 1e3 * wall / args.steps

    # roofline: time each kernel on its own (HIP events on the launch stream)
    batch.set_params(slots[0], *batch.get_params(slots[0])[:2], 2, True)
    for sl in slots[1:]:
        r_, g_, _, _ = batch.get_params(sl)
        batch.set_params(sl, r_, g_, 2, True)
    ab = algorithmic_bytes(insts, esz)
    one_red = bool(tiles) and len(tiles) > 5 and tiles[5] == 1
    if one_red:
        ids = {"cg1_step": sip.K_CG1_STEP, "cg1_w0": sip.K_CG1_W0}
    else:
        ids = {"cg_dir": sip.K_CG_DIR, "cg_upd": sip.K_CG_UPD}
    ids.update({"rhs": sip.K_RHS, "proj": sip.K_PROJ, "thr_w": sip.K_THR_W, "thr_apply": sip.K_THR_APPLY,
                "line": sip.K_LINE})
    per_iter = {"cg_dir": 10, "cg_upd": 10, "cg1_step": 10, "cg1_w0": 1, "rhs": 1, "proj": 1, "thr_w": 1,
                "thr_apply": 1, "line": 1}
    kernels = {}
    for name, kid in ids.items():
        if ab[name] == 0:
            continue
        t_ms = batch.time_kernel(kid, args.reps)
        kernels[name] = {"ms": t_ms, "GBs": ab[name] / (t_ms * 1e-3) / 1e9, "bytes": ab[name],
                         "launches_per_iter": per_iter[name]}
    dom = max(kernels, key=lambda k: kernels[k]["ms"] * kernels[k]["launches_per_iter"])
    ach = kernels[dom]["GBs"]
    traffic = traffic_from_profiles(dom, args.workload)
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "bytes_per_launch": ab[dom], "launch_ms": round(kernels[dom]["ms"], 5)}
    copy = None
    if args.copy_mb > 0:
        n = args.copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            sip.stream_copy(dst, src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        reps = 10
        for _ in range(reps):
            sip.stream_copy(dst, src)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / reps
        copy = {"bytes_moved": 2 * n * 4, "ms": round(t, 4), "GBs": round(2 * n * 4 / (t * 1e-3) / 1e9, 1)}
        del src, dst
    cpu = None
    check = None
    if args.cpu_seconds > 0:
        sched, chk = None, None
        kc = min(args.check_iters, iters)
        if kc > 0:
            xr, sched = device_reference(insts[0], field, args.reduce, kc, tiles)
            chk = (kc, xr)
        cpu, err = cpu_baseline(insts, iters, args.cpu_seconds, sched, chk)
        if chk is not None:
            check = {"iterations": kc, "rel_l2_x": err, "instance": "first",
                     "oracle": "FP64, replaying the device (rho, gamma) schedule",
                     "oracle_sensitivity": oracle_sensitivity(insts[0], kc, sched, field)}
    line = {
        "metric": "PARSDMM grid-pts*iters/s",
        "value": round(value, 1),
        "unit": "grid-pts*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": field,
        "data": "synthetic (seeded generators)",
        "config": {"workload": desc, "instances": len(insts), "grid_points": n_pts, "iterations": iters,
                   "cg_steps": 10, "reductions": args.reduce, "tiles": list(tiles) if tiles else "default"},
        "roofline": roofline,
        "kernels": {k: {"ms": round(v["ms"], 5), "GBs": round(v["GBs"], 1)} for k, v in kernels.items()},
        "cpu_baseline": cpu,
        "oracle_error": check,
        "copy_reference": copy,
    }
    if args.workload == "batched":
        line["instances_per_s"] = round(len(insts) * args.steps / wall, 2)
    print(json.dumps(line), flush=True)
    batch.close()


if __name__ == "__main__":
    main()
