"""Multilevel PARSDMM (the ML-PARSDMM listing, section "Multilevel PARSDMM"):
plain FP64 CPU reference.  Test infrastructure only: imported by tests/, the
smoke check and the benchmark's CPU baseline, never by the library.

Coarse-to-fine continuation without cycling: the model is coarsened level by
level (anti-alias filter, then subsampling); PARSDMM runs on the coarsest
grid; x and every y_i, v_i (i = 1..p+1) are interpolated as images to the
next finer grid and used as that level's initial guess; and so on up to the
original grid.

The paper leaves the following open; this module fixes them (readings):
  * coarsening: factor 2 per axis, keeping samples 0, 2, 4, ... so a level
    has ceil(n / 2) points per axis (an axis of one point stays one point);
    the grid spacing doubles;
  * anti-alias filter: the binomial [1, 2, 1] / 4 along each axis, edges
    replicated, applied before subsampling;
  * interpolation: linear along each axis at the geometric position of the
    fine sample: fine point i sits at coarse coordinate i / 2; a row of a
    forward difference along axis a sits half-way between its two points,
    so fine row j sits at coarse row coordinate (j + 1/2) / 2 - 1/2; the
    coordinate is clamped to the coarse image;
  * set parameters per level: bounds unchanged (difference quotients keep
    their units since h doubles with the spacing); an l1 budget tau and a
    cardinality k scale with the number of rows of the operator at that
    level (k rounded half up, at least 1, at most the rows); l2 radii (the
    l2 ball's tau, the annulus' lo and hi) with its square root;
  * the coarsest level starts like single-level PARSDMM (x = m, y_i = A_i m,
    v_i = 0), so one level is exactly PARSDMM;
  * (rho, gamma) on a finer level: either restart from (rho0, gamma0) or
    continue from the coarser level's final values (carry_params); the
    listing passes only x, y_i and v_i between levels.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import parsdmm as orc

# axes of the components of each operator (0 = z, the slowest), per ndim
COMP_AXES = {
    2: {"I": (None,), "DZ": (0,), "DX": (1,), "GRAD": (0, 1), "LAT": (1,)},
    3: {"I": (None,), "DZ": (0,), "DY": (1,), "DX": (2,), "GRAD": (0, 1, 2), "LAT": (1, 2)},
}


def coarse_shape(shape):
    """Grid of the next coarser level."""
    return tuple((int(n) + 1) // 2 for n in shape)


def level_shapes(shape, nlevels):
    out = [tuple(int(n) for n in shape)]
    for _ in range(nlevels - 1):
        out.append(coarse_shape(out[-1]))
    return out


def rows(shape, op):
    """Rows of A for an operator on a grid."""
    n = 0
    for ax in COMP_AXES[len(shape)][op]:
        sh = list(shape)
        if ax is not None:
            sh[ax] -= 1
        n += int(np.prod(sh))
    return n


def level_sets(sets, shape, shape_l):
    """The set list on a coarser grid (tau and k scaled by the row ratio)."""
    out = []
    for s in sets:
        if s.get("line") is not None:
            raise NotImplementedError("multilevel PARSDMM with line-wise sets")
        s2 = dict(s)
        ratio = rows(shape_l, s["op"]) / rows(shape, s["op"])
        if s["kind"] == "l1":
            s2["tau"] = s["tau"] * ratio
        elif s["kind"] == "l2":
            s2["tau"] = s["tau"] * math.sqrt(ratio)
        elif s["kind"] == "annulus":
            s2["lo"], s2["hi"] = s["lo"] * math.sqrt(ratio), s["hi"] * math.sqrt(ratio)
        elif s["kind"] == "card":
            s2["k"] = int(min(rows(shape_l, s["op"]), max(1, math.floor(s["k"] * ratio + 0.5))))
        out.append(s2)
    return out


def restrict(m):
    """Binomial [1, 2, 1] / 4 filter along every axis (edges replicated),
    then every other sample from 0."""
    a = np.asarray(m, dtype=np.float64)
    for ax in range(a.ndim):
        n = a.shape[ax]
        idx = np.arange(n)
        lo = np.take(a, np.maximum(idx - 1, 0), axis=ax)
        hi = np.take(a, np.minimum(idx + 1, n - 1), axis=ax)
        a = 0.25 * lo + 0.5 * a + 0.25 * hi
    sl = tuple(slice(0, None, 2) for _ in range(a.ndim))
    return a[sl]


def _interp_axis(a, ax, n_out, staggered):
    """Linear interpolation along one axis to n_out samples at the positions
    given in the module notes."""
    n_in = a.shape[ax]
    off = 0.5 if staggered else 0.0
    out_sh = list(a.shape)
    out_sh[ax] = n_out
    res = np.empty(out_sh)
    for i in range(n_out):
        c = (i + off) / 2.0 - off
        c = min(max(c, 0.0), n_in - 1.0)
        i0 = int(math.floor(c))
        i1 = min(i0 + 1, n_in - 1)
        t = c - i0
        v0 = np.take(a, i0, axis=ax)
        v1 = np.take(a, i1, axis=ax)
        idx = [slice(None)] * a.ndim
        idx[ax] = i
        res[tuple(idx)] = (1.0 - t) * v0 + t * v1
    return res


def prolong_image(img, out_shape, stag_axis=None):
    """A coarse image to the fine image shape, axis by axis."""
    a = np.asarray(img, dtype=np.float64)
    for ax in range(a.ndim):
        a = _interp_axis(a, ax, out_shape[ax], stag_axis == ax)
    return a


def prolong_rows(v, op, shape_c, shape_f):
    """An operator-row vector (A_i's row order: component blocks, each an
    image) from a coarse grid to a fine one."""
    parts, off = [], 0
    for ax in COMP_AXES[len(shape_f)][op]:
        shc, shf = list(shape_c), list(shape_f)
        if ax is not None:
            shc[ax] -= 1
            shf[ax] -= 1
        cnt = int(np.prod(shc))
        img = np.asarray(v[off:off + cnt]).reshape(shc)
        off += cnt
        parts.append(prolong_image(img, shf, ax).ravel())
    return np.concatenate(parts)


def parsdmm_multilevel(m, shape, sets, nlevels, level_iters, opts: orc.Options | None = None, h=None,
                       carry_params=False):
    """Multilevel PARSDMM.  level_iters[l] caps the iterations of level l
    (0 = the given grid).  Returns (x, per-level final states)."""
    opts = opts or orc.Options()
    shape = tuple(int(n) for n in shape)
    h0 = tuple(float(v) for v in (h if h is not None else (1.0,) * len(shape)))
    shapes = level_shapes(shape, nlevels)
    ms = [np.asarray(m, dtype=np.float64).reshape(shape)]
    for _ in range(1, nlevels):
        ms.append(restrict(ms[-1]))
    states = [None] * nlevels
    prev = None
    for lev in range(nlevels - 1, -1, -1):
        sh = shapes[lev]
        hl = tuple(v * 2.0 ** lev for v in h0)
        sets_l = level_sets(sets, shape, sh)
        prob = orc.Problem(ms[lev], sh, sets_l, hl)
        o = orc.Options(**{**opts.__dict__, "max_iter": int(level_iters[lev])})
        st = orc.initial_state(prob, o)
        if prev is not None:
            pprob, pst, psh = prev
            st.x = prolong_image(pst.x.reshape(psh), sh).ravel()
            st.x_hist = [st.x.copy()]
            ops = [s["op"] for s in sets_l] + ["I"]
            st.y = [prolong_rows(pst.y[i], ops[i], psh, sh) for i in range(len(ops))]
            st.v = [prolong_rows(pst.v[i], ops[i], psh, sh) for i in range(len(ops))]
            if carry_params:
                st.rho, st.gamma = pst.rho.copy(), pst.gamma.copy()
        _, st = orc.parsdmm(ms[lev], sh, sets_l, o, h=hl, state=st)
        states[lev] = st
        prev = (prob, st, sh)
    return states[0].x.reshape(shape), states
