"""Parallel Dykstra on the device (Appendix A, the Parallel-DYKSTRA
listing), the baseline of the paper's PARSDMM comparison: each outer
iteration projects every v_i onto V_i = {x | A_i x in C_i} with single-set
PARSDMM (the p sub-problems are the instances of one batch, run together),
then sip_dykstra_update forms x = sum_i w_i y_i and v_i = x + v_i - y_i.

Counts follow the paper: per outer iteration the CG steps of the slowest
sub-problem, and the inner iterations of each thresholding set (one
projection each)."""
from __future__ import annotations

from dataclasses import dataclass, field

from paper_1902_09699_amd import sip


@dataclass
class DykstraLog:
    cg_steps: list = field(default_factory=list)   # per outer iteration: per set
    iters: list = field(default_factory=list)      # per outer iteration: inner iterations per set


class ParallelDykstra:
    """Resident state of one parallel Dykstra run: the batch of p single-set
    sub-problems, the v_i and the iterate x (device tensors)."""

    def __init__(self, m, sets, inner: sip.Opts, weights=None, h=None, tiles=None):
        import torch
        self.p = len(sets)
        self.sets = [dict(s) for s in sets]
        self.inner = inner
        self.w = [1.0 / self.p] * self.p if weights is None else [float(v) for v in weights]
        self.x = m.clone()
        self.v = [m.clone() for _ in range(self.p)]
        self.y = [torch.empty_like(m) for _ in range(self.p)]
        ws = sum(sip.workspace_bytes(tuple(m.shape), [s], inner) for s in self.sets)
        self.batch = sip.Batch(self.p, ws, inner)
        if tiles:
            self.batch.set_tiles(*tiles)
        self.slots = [self.batch.add(self.v[i], [self.sets[i]], self.y[i], h=h) for i in range(self.p)]
        self.log = DykstraLog()
        self.first = True

    def step(self):
        """One outer iteration."""
        if not self.first:
            for i in range(self.p):
                self.batch.reset(self.slots[i], self.v[i])
        self.first = False
        self.batch.run(self.inner.max_iter)
        res = [self.batch.result(sl) for sl in self.slots]
        for r in res:
            if r["status"] != 0:
                raise sip.SipError(r["status"], "parallel Dykstra sub-problem")
        self.log.cg_steps.append([r["cg_steps"] for r in res])
        self.log.iters.append([r["iters"] for r in res])
        sip.dykstra_update(self.y, self.v, self.w, self.x)

    def close(self):
        self.batch.close()
