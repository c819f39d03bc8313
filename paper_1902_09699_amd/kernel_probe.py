"""Launch each iteration kernel of a workload a few times, in the launch
configuration bench.py times, plus the plain copy kernel: a short program for
rocprofv3 counter passes (FETCH_SIZE / WRITE_SIZE need few dispatches).

    python -m paper_1902_09699_amd.kernel_probe --workload layered2d --reps 3
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="layered2d")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--copy-mb", type=int, default=256)
    ap.add_argument("--tiles", default=None, help="pt_points,pt_max_items,thr_points,thr_max_items[,pt_threads]")
    a = ap.parse_args()
    import torch

    import bench
    from paper_1902_09699_amd import sip

    args = argparse.Namespace(batched_count=256)
    insts, field, iters, _ = bench.load_workload(a.workload, args)
    dt = torch.float64 if field == "f64" else torch.float32
    opts = sip.make_opts(field, max_iter=iters, cg_max=10, cg_fixed=1)
    ms = [torch.tensor(m, dtype=dt, device="cuda") for m, _ in insts]
    xs = [torch.empty_like(m) for m in ms]
    batch = sip.Batch(len(insts), sum(sip.workspace_bytes(m.shape, s, opts) for m, s in insts), opts)
    slots = [batch.add(md, s, xd) for md, (_, s), xd in zip(ms, insts, xs)]
    tiles = [int(v) for v in a.tiles.split(",")] if a.tiles else []
    if tiles:
        batch.set_tiles(*tiles)
    form = tiles[5] if len(tiles) > 5 else 0
    batch.run(2)
    torch.cuda.synchronize()
    for sl in slots:
        r_, g_, _, _ = batch.get_params(sl)
        batch.set_params(sl, r_, g_, 2, True)
    out = {}
    cg = {0: (("cg_dir", sip.K_CG_DIR), ("cg_upd", sip.K_CG_UPD)),
          1: (("cg1_step", sip.K_CG1_STEP), ("cg1_w0", sip.K_CG1_W0)),
          2: (("cg2_step", sip.K_CG2_STEP), ("cg2_d0", sip.K_CG2_D0))}[form]
    has_line = any(s.get("line") is not None for _, sets in insts for s in sets)
    for name, kid in cg + (("rhs", sip.K_RHS), ("proj", sip.K_PROJ), ("thr_w", sip.K_THR_W),
                           ("thr_apply", sip.K_THR_APPLY)) + ((("line", sip.K_LINE),) if has_line else ()):
        out[name] = batch.time_kernel(kid, a.reps)
        print(f"{name}: {out[name] * 1e3:.2f} us", flush=True)
    n = a.copy_mb * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        sip.stream_copy(dst, src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "kernel_ms": out}), flush=True)
    batch.close()


if __name__ == "__main__":
    main()
