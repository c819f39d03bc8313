"""Parallel Dykstra (Appendix A, the Parallel-DYKSTRA listing): plain FP64 CPU
reference.  Test infrastructure only: imported by tests/, never by the
library.

m is projected onto the intersection of V_i = {x | A_i x in C_i} using only
projections onto each V_i:

  x^0 = m, v_i^0 = x^0, weights w_i with sum 1;
  repeat:  y_i = P_{V_i}(v_i)            (all i, independent)
           x   = sum_i w_i y_i
           v_i = x + v_i - y_i.

For a V_i whose operator is not orthogonal, P_{V_i} has no closed form; the
paper's comparison computes it with an adaptive relaxed ADMM using the same
penalty / relaxation update as PARSDMM.  Here that inner solver is PARSDMM
itself with the single set i (the projection of v_i onto V_i is PARSDMM's
problem with p = 1), with its own iteration cap and stopping rule.

Counting (the paper's convention): per outer iteration the CG steps of the
slowest sub-problem (they run in parallel) and, for a set projected by
thresholding (the l1 ball), its number of inner iterations (one projection
each).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from oracle import parsdmm as orc


@dataclass
class OuterStats:
    cg_steps: list = field(default_factory=list)    # per set
    iters: list = field(default_factory=list)       # inner PARSDMM iterations per set


def project_onto_set(v, shape, s, inner: orc.Options, h=None):
    """P_{V_i}(v) by single-set PARSDMM; returns (y, cg steps, iterations)."""
    y, st = orc.parsdmm(np.asarray(v).reshape(shape), shape, [s], inner, h=h)
    return y.ravel(), st.cg_steps, st.k - 1


def parallel_dykstra(m, shape, sets, outer_iters, inner: orc.Options, weights=None, h=None):
    """Returns (x, per-outer-iteration OuterStats, per-outer-iteration x)."""
    p = len(sets)
    w = np.full(p, 1.0 / p) if weights is None else np.asarray(weights, dtype=np.float64)
    x = np.asarray(m, dtype=np.float64).ravel().copy()
    v = [x.copy() for _ in range(p)]
    log, xs = [], []
    for _ in range(outer_iters):
        stats = OuterStats()
        ys = []
        for i, s in enumerate(sets):
            y, cg, it = project_onto_set(v[i], shape, s, inner, h)
            ys.append(y)
            stats.cg_steps.append(cg)
            stats.iters.append(it)
        x = np.zeros_like(x)
        for i in range(p):
            x = x + w[i] * ys[i]
        v = [x + v[i] - ys[i] for i in range(p)]
        log.append(stats)
        xs.append(x.copy())
    return x.reshape(shape), log, xs
