"""Benchmark: PARSDMM grid-points x iterations per second on one MI355X.

One step = one complete projection of every instance of the workload (state
reset from m, then every iteration of the PARSDMM listing), inputs resident
in HBM.  The default workload is the largest single-GPU configuration: 256
uneven 2D instances in one batch.  One JSON line carries

* the throughput (grid-pts*iters/s) and instances/s of that batch;
* the roofline of its dominant kernel (algorithmic bytes per launch over the
  HIP-event mean launch duration) and of the whole iteration (the compulsory
  words of an iteration, (5 + 8 n_cg) N + 9 sum M + 2 sum M_thr + N per
  instance with an l1/cardinality set, over the measured time per iteration),
  both against the 8 TB/s HBM peak;
* the same whole-iteration figures on the 200x200x100 grid (the single
  instance that streams from HBM) and the served form's p50/p99 latency next
  to the plain one-at-a-time form on the same requests;
* the FP64 CPU oracle timed on a bounded sample of the workload on the host's
  cores, and the error against it of a sample of instances (the oracle
  replays each device run's (rho, gamma) schedule and kept cardinality rows).
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
METRIC = "PARSDMM grid-pts·iters/s, % HBM peak; served p50/p99 latency vs plain"
WORKLOADS = ("batched", "layered2d", "layered2d_lines", "smooth2d", "smooth3d")
# relative band around the k-th magnitude inside which a cardinality
# support may go either way (ties of the non-convex projection)
CARD_BAND = 1e-4
# the same band relative to the scale of w (the largest sum of the sizes of
# its terms over the rows): float32 rounding of the state w is formed from,
# accumulated over the iterations (2^-17, 128 float32 ulps of that scale)
CARD_TERM_BAND = 2.0 ** -17


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched", choices=WORKLOADS)
    ap.add_argument("--graph-iters", type=int, default=50)
    ap.add_argument("--reps", type=int, default=30, help="launches per kernel timing")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU oracle timing budget (0: skip the CPU leg)")
    ap.add_argument("--batched-count", type=int, default=256)
    ap.add_argument("--copy-mb", type=int, default=1024, help="plain-copy reference size (0: skip)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tiles")
    ap.add_argument("--sel-fresh", type=int, default=0, choices=(0, 1),
                    help="1: threshold selections read all of w (no reuse of the previous first digit)")
    ap.add_argument("--reduce", default="f64", choices=("f64", "f32"),
                    help="reduction type (f32: the pure-FP32 precision ablation)")
    ap.add_argument("--check-iters", type=int, default=40,
                    help="iterations of the locked error check against the oracle (0: skip)")
    ap.add_argument("--check-instances", type=int, default=4, help="sampled instances of the error check")
    ap.add_argument("--tiles", default=None,
                    help="fixed tiles pt_points,pt_max_items,thr_points,thr_max_items[,pt_threads[,cg_form]] "
                         "(no autotune)")
    ap.add_argument("--extras", default="auto", choices=("auto", "on", "off"),
                    help="200x200x100 and served legs (auto: with the batched workload)")
    ap.add_argument("--c3-steps", type=int, default=2)
    ap.add_argument("--c3-check-iters", type=int, default=0,
                    help="locked iterations of the 200x200x100 error check against the oracle (0: skip)")
    ap.add_argument("--served-requests", type=int, default=200)
    ap.add_argument("--served-rate", type=float, default=200.0)
    ap.add_argument("--served-check", type=int, default=3,
                    help="smallest served requests rerun alone and compared with the oracle")
    return ap.parse_args()


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- workloads

def load_workload(name, args):
    from paper_1902_09699_amd import workloads as wl
    if name == "batched":
        out = []
        for m, sets in wl.batched_instances(args.batched_count):
            m = wl.rounded(m, "f32")
            out.append((m, wl.finalize(m, sets)))
        return out, "f32", 200, (f"{args.batched_count} uneven 2D instances (sides U[32,512]), 2-5 sets from "
                                 f"{{box, TV, l1(D_z), card(D_x)}}; 200 it x 10 CG, f32 fields, f64 reductions")
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


def rows(shape, s):
    from paper_1902_09699_amd import workloads as wl
    return wl.rows_of(shape, s["op"])


def iteration_words(insts, n_cg=10):
    """Compulsory words of one PARSDMM iteration, summed over instances: each
    phase between two global reductions streams its operands once.
    RHS + CG init 2 sum M + 2N; CG 8N per step (3N direction + 5N update);
    projections 2N + 4 sum M; threshold sets' histogram pass 2 M_i (+N for x
    once); adapt-rho-gamma snapshots 3 sum M + N every second iteration
    (amortised 1.5 sum M + N/2, rounded into 9 sum M and the 5N)."""
    w = 0
    for m, sets in insts:
        N = m.size
        sum_m = N + sum(rows(m.shape, s) for s in sets)
        thr = [rows(m.shape, s) for s in sets if s["kind"] != "bounds"]
        w += (5 + 8 * n_cg) * N + 9 * sum_m + 2 * sum(thr) + (N if thr else 0)
    return w


def kernel_bytes(insts, esz):
    """Algorithmic bytes of one launch of each kernel (all instances), on the
    same per-phase accounting as iteration_words: CG direction read r, p,
    write p (3N); CG update read x, r, p, write x, r (5N); a one-reduction CG
    step counts as one CG step of the same accounting (8N, although that
    arrangement moves 10N); its w_0 pass read r, write w (2N); the
    LDS-staged form's step likewise counts 8N (it moves 6N) and its
    r_0^T C r_0 pass N; RHS read x and
    every y_i, v_i (identity block included), write r; projection read x, m
    and y_i, v_i of the bounds sets and the identity block, write y_i, v_i;
    threshold w pass read x, y_i, v_i, write w (N + 3 M_i); apply pass read
    w, write y_i, v_i (3 M_i); line-wise sets read x, y_i, v_i, write y_i,
    v_i (N + 4 M_i)."""
    b = {"cg_dir": 0, "cg_upd": 0, "cg1_step": 0, "cg1_w0": 0, "cg2_step": 0, "cg2_d0": 0, "rhs": 0, "proj": 0,
         "thr_w": 0, "thr_apply": 0, "line": 0}
    for m, sets in insts:
        N = m.size
        sum_m = N + sum(rows(m.shape, s) for s in sets)
        clip = N + sum(rows(m.shape, s) for s in sets if s["kind"] == "bounds")
        thr = [rows(m.shape, s) for s in sets if s["kind"] != "bounds" and s.get("line") is None]
        line = [rows(m.shape, s) for s in sets if s.get("line") is not None]
        b["cg_dir"] += 3 * N * esz
        b["cg_upd"] += 5 * N * esz
        b["cg1_step"] += 8 * N * esz
        b["cg1_w0"] += 2 * N * esz
        b["cg2_step"] += 8 * N * esz
        b["cg2_d0"] += N * esz
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


# ------------------------------------------------------------------ GPU legs

def run_timed(insts, field, iters, args, steps, warmup, tiles_arg=None, autotune=True):
    """Admit every instance into one batch, pick tiles, then time `steps`
    complete projections (reset from m + every iteration, chunks of
    graph_iters iterations replayed from captured graphs)."""
    import torch
    from paper_1902_09699_amd import sip
    dt = torch.float64 if field == "f64" else torch.float32
    opts = sip.make_opts(field, reduce=args.reduce, max_iter=iters, cg_max=10, cg_fixed=1, sel_fresh=args.sel_fresh)
    ms = [torch.tensor(m, dtype=dt, device="cuda") for m, _ in insts]
    xs = [torch.empty_like(m) for m in ms]
    arena = sum(sip.workspace_bytes(m.shape, s, opts) for m, s in insts)
    batch = sip.Batch(len(insts), arena, opts)
    slots = [batch.add(md, s, xd) for md, (_, s), xd in zip(ms, insts, xs)]
    assert all(s >= 0 for s in slots)
    tiles = None
    if tiles_arg:
        tiles = tuple(int(v) for v in tiles_arg.split(","))
        batch.set_tiles(*tiles)
    elif autotune:
        from paper_1902_09699_amd import autotune as at
        tiles, tile_ms = at.tune(batch, slots, ms, field, [m.shape for m, _ in insts], use_cache=False, cache=None)
        for cand, t in sorted(tile_ms.items(), key=lambda kv: kv[1])[:4]:
            say(f"autotune {cand}: {1e3 * t:.1f} us/iteration")
    chunk = min(args.graph_iters, iters)

    def one_step():
        for sl, md in zip(slots, ms):
            batch.reset(sl, md)
        left = iters
        while left > 0:
            n = min(chunk, left)
            batch.run(n)
            left -= n

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    results = [batch.result(sl) for sl in slots]
    assert all(r["status"] == 0 and r["iters"] == iters for r in results), results[:3]
    n_pts = sum(m.size for m, _ in insts)
    # threshold selections of the last step that refined over the w pass's
    # list A (the previous iteration's first-digit bucket)
    n_sel = iters * sum(sum(1 for q in s if q["kind"] in ("l1", "card") and not q.get("line")) for _, s in insts)
    reuse = {"reused": int(sum(r["sel_reused"] for r in results)), "selections": int(n_sel)}
    return {"batch": batch, "slots": slots, "ms": ms, "xs": xs, "tiles": tiles, "wall": wall,
            "ms_step": 1e3 * wall / steps, "value": n_pts * iters * steps / wall, "n_pts": n_pts,
            "selection_reuse": reuse}


def kernel_table(run, insts, field, reps):
    """Each iteration kernel timed on its own over the batch's work tables
    (HIP events on the launch stream), with its algorithmic bytes."""
    from paper_1902_09699_amd import sip
    batch, slots = run["batch"], run["slots"]
    for sl in slots:  # an adapt iteration follows: the snapshot branches run
        r_, g_, _, _ = batch.get_params(sl)
        batch.set_params(sl, r_, g_, 2, True)
    esz = 8 if field == "f64" else 4
    ab = kernel_bytes(insts, esz)
    tiles = run["tiles"]
    form = tiles[5] if tiles and len(tiles) > 5 else 0
    if form == 2 and any(m.ndim == 3 for m, _ in insts):
        form = 0  # the LDS-staged form runs the steps of 2D grids only
    ids = {0: {"cg_dir": sip.K_CG_DIR, "cg_upd": sip.K_CG_UPD},
           1: {"cg1_step": sip.K_CG1_STEP, "cg1_w0": sip.K_CG1_W0},
           2: {"cg2_step": sip.K_CG2_STEP, "cg2_d0": sip.K_CG2_D0}}[form]
    ids.update({"rhs": sip.K_RHS, "proj": sip.K_PROJ, "thr_w": sip.K_THR_W, "thr_apply": sip.K_THR_APPLY,
                "line": sip.K_LINE})
    per_iter = {"cg_dir": 10, "cg_upd": 10, "cg1_step": 10, "cg1_w0": 1, "cg2_step": 10, "cg2_d0": 1, "rhs": 1,
                "proj": 1, "thr_w": 1, "thr_apply": 1, "line": 1}
    kernels = {}
    for name, kid in ids.items():
        if ab[name] == 0:
            continue
        t_ms = batch.time_kernel(kid, reps)
        kernels[name] = {"ms": t_ms, "GBs": ab[name] / (t_ms * 1e-3) / 1e9, "bytes": ab[name],
                         "launches_per_iter": per_iter[name]}
    return kernels


def roofline_of(kernels, wname):
    dom = max(kernels, key=lambda k: kernels[k]["ms"] * kernels[k]["launches_per_iter"])
    ach = kernels[dom]["GBs"]
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_from_profiles(dom, wname), "kernel": dom,
            "bytes_per_launch": kernels[dom]["bytes"], "launch_ms": round(kernels[dom]["ms"], 5)}


def iteration_roofline(insts, field, iters, ms_step):
    esz = 8 if field == "f64" else 4
    words = iteration_words(insts)
    t = ms_step * 1e-3 / iters
    gbs = words * esz / t / 1e9
    return {"bytes": words * esz, "ms": round(1e3 * t, 5), "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}


def c3_leg(args):
    """The 200x200x100 grid (box, TV ball, lateral slopes): whole-iteration
    figures of the single instance that streams from HBM."""
    insts, field, iters, desc = load_workload("smooth3d", args)
    say("200x200x100: autotune and timing")
    run = run_timed(insts, field, iters, args, args.c3_steps, 1)
    kernels = kernel_table(run, insts, field, max(5, args.reps // 3))
    out = {"workload": desc, "grid_points": run["n_pts"], "iterations": iters, "steps": args.c3_steps,
           "ms_per_step": round(run["ms_step"], 3), "value": round(run["value"], 1),
           "tiles": list(run["tiles"]) if run["tiles"] else "default",
           "iteration": iteration_roofline(insts, field, iters, run["ms_step"]),
           "selection_reuse": run["selection_reuse"],
           "roofline": roofline_of(kernels, "smooth3d"),
           "kernels": {k: {"ms": round(v["ms"], 5), "GBs": round(v["GBs"], 1)} for k, v in kernels.items()}}
    run["batch"].close()
    return out, insts


def served_leg(args):
    """The served mix (Poisson arrivals, 5% 3D, stopping rule on, continuous
    batching in two resident batches split by size) and the plain
    one-at-a-time form on the same requests."""
    from paper_1902_09699_amd import serve
    opts = serve.serving_opts(200)
    arena = 64 << 30
    n, rate = args.served_requests, args.served_rate
    say(f"served: {n} requests at {rate:g} req/s")
    # warm both lanes (code objects, graph capture at their first sizes)
    warm = serve.make_requests(4, 1e9, 0.0, seed0=9000, max2d=128) + \
        serve.make_requests(2, 1e9, 1.0, seed0=9050, side3d=(66, 72))
    srv = serve.Server(opts, arena, 256, 5, lanes=2, split_points=1 << 18, tiles=serve.SERVED_TILES)
    srv.run(warm, realtime=False)
    reqs = serve.make_requests(n, rate)
    info = srv.run(reqs, realtime=True)
    srv.close()
    served = serve.summary(reqs, "served")
    served.update(info)
    say("plain: the same requests one at a time")
    plain_reqs = serve.make_requests(n, rate)
    pinfo = serve.serve_plain(plain_reqs, opts, arena, 10)
    plain = serve.summary(plain_reqs, "plain")
    plain.update(pinfo)
    offered = sum(r.m.size for r in reqs) / max(reqs[-1].arrival - reqs[0].arrival, 1e-9)
    return {"requests": n, "rate_per_s": rate, "frac_3d": 0.05, "offered_grid_pts_per_s": round(offered, 1),
            "server": ("two resident batches on two streams (requests up to 2^18 points / larger), chunks of 5 "
                       "(plain form: 10), "
                       f"tiles {list(serve.SERVED_TILES)} (plain form: the engine's defaults)"),
            "stopping": "eqs. feas_stop/obj_stop every 5 it, cap 200, CG cap 10 at 0.1 relative residual",
            "served": served, "plain": plain,
            "speedup_instances_per_s": round(served["instances_per_s"] / max(plain["instances_per_s"], 1e-9), 2)}


def copy_reference(mb):
    import torch
    from paper_1902_09699_amd import sip
    n = mb * (1 << 20) // 4
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
    return {"bytes_moved": 2 * n * 4, "ms": round(t, 4), "GBs": round(2 * n * 4 / (t * 1e-3) / 1e9, 1)}


def device_logged(inst, field, reduce, tiles, iters, stop_every=0):
    """One instance alone on the device (tiles and CG form as timed; results
    are bit-identical alone and in a batch), one iteration at a time: its x,
    the (rho, gamma) and CG step count of every iteration, the rows every
    whole-vector cardinality set kept (operator row order) and the result.
    stop_every > 0: the served options (stopping rule on, relative CG stop)."""
    import torch
    from paper_1902_09699_amd import sip
    m, sets = inst
    if stop_every:
        opts = sip.make_opts(field, reduce=reduce, max_iter=iters, cg_max=10, cg_fixed=0, stop_every=stop_every)
    else:
        opts = sip.make_opts(field, reduce=reduce, max_iter=iters, cg_max=10, cg_fixed=1)
    md = torch.tensor(m, dtype=torch.float64 if field == "f64" else torch.float32, device="cuda")
    xd = torch.empty_like(md)
    b = sip.Batch(1, sip.workspace_bytes(m.shape, sets, opts), opts)
    if tiles:
        b.set_tiles(*tiles)
    slot = b.add(md, sets, xd)
    card = [i for i, s in enumerate(sets) if s["kind"] == "card" and s.get("line") is None]
    sched, sup = {}, {}
    cg_before = 0
    for _ in range(iters):
        rho, gam, k, _ = b.get_params(slot)
        b.run(1)
        res = b.result(slot)
        if res["iters"] < k:
            break  # finished before this iteration
        sched[k] = (rho.copy(), gam.copy(), res["cg_steps"] - cg_before)
        cg_before = res["cg_steps"]
        if card:
            sup[k] = {i: np.nonzero(b.rows(slot, sip.FIELD_Y, i, m.shape, sets[i]["op"]))[0] for i in card}
        if b.poll()[slot] == 1:
            break
    torch.cuda.synchronize()
    res = b.result(slot)
    x = xd.double().cpu().numpy()
    b.close()
    return x, sched, sup, res


# ------------------------------------------------------------------ CPU leg

def host_info():
    info = {"logical_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"),
            "OPENBLAS_NUM_THREADS": os.environ.get("OPENBLAS_NUM_THREADS")}
    model, cores = None, set()
    try:
        phys = None
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    cores.add((phys, v))
    except OSError:
        pass
    info["model"] = model
    info["physical_cores"] = len(cores) or None
    return info


def cpu_baseline(insts, iters_full, budget_s):
    """The FP64 oracle as it stands, free-running, on instances of the
    workload in order, each from its second iteration on, until the budget
    is spent (at least two iterations)."""
    from oracle import parsdmm as orc
    pts_iters, done_desc = 0, []
    wall = cpu = 0.0
    for j, (m, sets) in enumerate(insts):
        prob = orc.Problem(m, m.shape, sets)
        opts = orc.Options(max_iter=iters_full, cg_max=10, cg_fixed=True)
        st = orc.initial_state(prob, opts)
        orc.iterate(prob, st, opts)  # first iteration untimed (x = m)
        ru0 = resource.getrusage(resource.RUSAGE_SELF)
        t0 = time.perf_counter()
        n = 0
        while st.k <= iters_full and (n < 2 or wall + time.perf_counter() - t0 < budget_s):
            orc.iterate(prob, st, opts)
            n += 1
        dt = time.perf_counter() - t0
        ru1 = resource.getrusage(resource.RUSAGE_SELF)
        wall += dt
        cpu += (ru1.ru_utime - ru0.ru_utime) + (ru1.ru_stime - ru0.ru_stime)
        pts_iters += m.size * n
        done_desc.append(f"#{j} {'x'.join(map(str, m.shape))} it 2..{n + 1}")
        if wall >= budget_s:
            break
    threads = max(1, int(round(cpu / wall)))
    return {"value": round(pts_iters / wall, 1), "unit": "grid-pts*iters/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 CSR oracle, free-running, fixed 10 CG steps: {'; '.join(done_desc)} "
                      f"({wall:.1f} s wall, {cpu:.1f} s CPU)",
            "host": host_info()}


def pick_sample(insts, count):
    """Indices of up to `count` instances covering every set kind present
    (TV ball, l1 on D_z, cardinality, box), first occurrences first."""
    want = [("l1", "GRAD"), ("l1", "DZ"), ("card", None), ("bounds", None)]
    pick = []
    for kind, op in want:
        for j, (_, sets) in enumerate(insts):
            if j in pick:
                continue
            if any(s["kind"] == kind and (op is None or s["op"] == op) for s in sets):
                pick.append(j)
                break
    for j in range(len(insts)):
        if len(pick) >= count:
            break
        if j not in pick:
            pick.append(j)
    return sorted(pick[:count])


def oracle_errors(insts, field, reduce, tiles, iters, count, picks=None, stop_every=0):
    """Relative L2 error of x after `iters` iterations for a sample of
    instances; the oracle replays each device run's (rho, gamma) schedule
    (and, with the relative CG stop, its CG step counts) and, for
    cardinality sets, its kept rows, each checked to be a valid top-k choice
    of the oracle's own w within CARD_BAND of the k-th magnitude or
    CARD_TERM_BAND of w's scale, whichever is larger (equal choices within
    the band are ties at float32 resolution).  stop_every > 0: the served options;
    the oracle then also stops by its own stopping test, and the iteration
    counts of both sides are reported."""
    from oracle import parsdmm as orc
    out = []
    for j in (picks if picks is not None else pick_sample(insts, count)):
        m, sets = insts[j]
        x, sched, sup, res = device_logged(insts[j], field, reduce, tiles, iters, stop_every)
        prob = orc.Problem(m, m.shape, sets)
        if stop_every:
            oo = orc.Options(max_iter=iters, cg_max=10, cg_fixed=False, stop_every=stop_every)
        else:
            oo = orc.Options(max_iter=iters, cg_max=10, cg_fixed=True)
        st = orc.initial_state(prob, oo)
        valid, differ, worst, worst_t = True, 0, 0.0, 0.0
        card = [i for i, s in enumerate(sets) if s["kind"] == "card" and s.get("line") is None]
        while st.k <= iters and st.k in sched:
            k = st.k
            pre = {i: (st.y[i].copy(), st.v[i].copy()) for i in card}
            stop = orc.iterate(prob, st, oo, sched, sup or None)
            for i in card:
                a = np.abs(st.w_last[i])
                kk = sets[i]["k"]
                tk = np.partition(a, a.size - kk)[a.size - kk]
                # scale of w = gamma s + (1 - gamma) y - v / rho: the largest
                # sum of its terms' sizes over the rows; the float32 state the
                # device carries differs from the oracle's by rounding relative
                # to that scale, not to a small k-th magnitude
                rho_i, gam_i = sched[k][0][i], sched[k][1][i]
                y0, v0 = pre[i]
                terms = np.abs(gam_i * (prob.A[i] @ st.x)) + np.abs((1.0 - gam_i) * y0) + np.abs(v0 / rho_i)
                scale = float(np.max(terms)) if terms.size else 0.0
                band = max(CARD_BAND * tk, CARD_TERM_BAND * scale)
                keep = sup[k][i]
                drop = np.ones(a.size, bool)
                drop[keep] = False
                valid &= keep.size <= kk and bool(np.all(a[keep] >= tk - band)) and \
                    bool(np.all(a[drop] <= tk + band))
                diff = np.setxor1d(orc.card_support(st.w_last[i], kk), keep)
                differ += int(diff.size)
                if diff.size:
                    worst = max(worst, float(np.max(np.abs(a[diff] - tk)) / max(tk, 1e-300)))
                    worst_t = max(worst_t, float(np.max(np.abs(a[diff] - tk)) / max(scale, 1e-300)))
            if stop:
                st.converged = True
                break
        xo = st.x
        err = float(np.linalg.norm(x.ravel() - xo) / max(np.linalg.norm(xo), 1e-300))
        extra = {}
        if stop_every:
            extra = {"device_iterations": res["iters"], "oracle_iterations": st.k - 1,
                     "device_converged": bool(res["converged"]), "oracle_converged": bool(st.converged)}
        out.append({"instance": j, "shape": list(m.shape), "sets": [f"{s['kind']}({s['op']})" for s in sets],
                    "iterations": res["iters"] if stop_every else iters, "rel_l2_x": err, **extra,
                    **({"card_supports_valid": bool(valid), "card_rows_differing_from_oracle_choice": differ,
                        "card_max_rel_distance_from_tk": worst,
                        "card_max_distance_over_w_scale": worst_t} if card else {})})
    return out


# -------------------------------------------------------------------- main

def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the library has no multi-GPU path; "
              f"independent instances would be routed to GPUs by free memory, which is not built",
              file=sys.stderr)
        sys.exit(2)
    import torch  # noqa: F401

    insts, field, iters, desc = load_workload(args.workload, args)
    say(f"workload {args.workload}: {len(insts)} instance(s), {sum(m.size for m, _ in insts)} points")
    run = run_timed(insts, field, iters, args, args.steps, args.warmup, args.tiles, not args.no_autotune)
    say(f"timed {args.steps} steps: {run['ms_step']:.3f} ms/step")
    kernels = kernel_table(run, insts, field, args.reps)
    roofline = roofline_of(kernels, args.workload)
    tiles = run["tiles"]
    run["batch"].close()
    copy = copy_reference(args.copy_mb) if args.copy_mb > 0 else None

    extras = args.extras == "on" or (args.extras == "auto" and args.workload == "batched")
    c3 = served = None
    if extras:
        c3, c3_insts = c3_leg(args)
        say(f"200x200x100: {c3['ms_per_step']:.3f} ms/step, iteration {c3['iteration']['frac']:.3f} of HBM peak")
        served = served_leg(args)
        say(f"served p50 {served['served']['p50_ms']} ms p99 {served['served']['p99_ms']} ms; "
            f"plain p50 {served['plain']['p50_ms']} ms p99 {served['plain']['p99_ms']} ms")

    cpu = errors = None
    if args.cpu_seconds > 0:
        say(f"CPU oracle: {args.cpu_seconds:g} s timing budget")
        cpu = cpu_baseline(insts, iters, args.cpu_seconds)
        if args.check_iters > 0:
            say(f"oracle errors: {args.check_instances} instance(s), {args.check_iters} iterations")
            errors = oracle_errors(insts, field, args.reduce, tiles, min(args.check_iters, iters),
                                   args.check_instances)
        if c3 is not None and args.c3_check_iters > 0:
            say(f"oracle error on 200x200x100: {args.c3_check_iters} iterations")
            tiles3 = tuple(c3["tiles"]) if isinstance(c3["tiles"], list) else None
            c3["oracle_error"] = oracle_errors(c3_insts, "f32", args.reduce, tiles3, args.c3_check_iters, 1,
                                               picks=[0])
        if served is not None and args.served_check > 0:
            # the served results are bit-identical to the same request alone:
            # the smallest requests rerun alone with logging, against the oracle
            from paper_1902_09699_amd import serve
            reqs = serve.make_requests(args.served_requests, args.served_rate)
            small = sorted(range(len(reqs)), key=lambda j: reqs[j].m.size)[:args.served_check]
            say(f"oracle errors of served requests {small}")
            sinst = [(r.m, r.sets) for r in reqs]
            served["oracle_error"] = oracle_errors(sinst, "f32", "f64", serve.SERVED_TILES, 200, 0, picks=small,
                                                   stop_every=5)

    line = {
        "metric": METRIC,
        "value": round(run["value"], 1),
        "unit": "grid-pts*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(run["ms_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": field,
        "data": "synthetic (seeded generators)",
        "config": {"workload": desc, "instances": len(insts), "grid_points": run["n_pts"], "iterations": iters,
                   "cg_steps": 10, "reductions": args.reduce, "tiles": list(tiles) if tiles else "default"},
        "roofline": roofline,
        "iteration": iteration_roofline(insts, field, iters, run["ms_step"]),
        "selection_reuse": run["selection_reuse"],
        "kernels": {k: {"ms": round(v["ms"], 5), "GBs": round(v["GBs"], 1)} for k, v in kernels.items()},
        "cpu_baseline": cpu,
        "oracle_error": errors,
        "copy_reference": copy,
    }
    if len(insts) > 1:
        line["instances_per_s"] = round(len(insts) * args.steps / run["wall"], 2)
    if c3 is not None:
        line["smooth3d_200x200x100"] = c3
    if served is not None:
        line["served"] = served
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
