"""Plain FP64 CPU oracle of PARSDMM (Peters & Herrmann, "Algorithms and
software for projections onto intersections of convex and non-convex sets
with applications to inverse problems", arXiv:1902.09699).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this module; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the HIP path.

It is written to be checked against the paper by eye: every linear operator
is an explicit sparse matrix built from its Kronecker definition, the system
matrix C is formed as a sparse matrix from eq. (sys_mat) with the current
rho at every x-update (the incremental update of eq. C_update gives the same
matrix up to rounding), the x-update is plain
conjugate gradients, the l1-ball projection sorts, and the cardinality
projection uses a stable full sort.  Everything is float64.

Readings of the paper that the text leaves open (they are stated again in the
docstrings where they act):

* grid vectors are C-ordered: axis 0 is z (vertical, slowest), the last axis
  is x; D along an axis is the forward difference of eq. (FD_mat) lifted by
  Kronecker products with identities on the other axes;
* the prox of the squared distance divides by 1 + rho_{p+1} (eq. prox_sq_dist),
  not by 1 + rho_i as the PARSDMM listing prints;
* CG stops when ||r|| < cg_rel * ||r_0||, where r_0 is the residual of the warm
  start x^k (eq. cg_stop: ||b|| cancels), or after cg_max steps; with
  cg_fixed it runs exactly cg_max steps unless the residual is exactly zero;
* adapt-rho-gamma uses the y of the current iteration before its update for
  v-hat, its first call only stores the k0 snapshot, a correlation with a zero
  norm counts as unreliable, gamma is capped at gamma_max and each rho_i
  (i <= p) is kept within [rho_{p+1}/R, R rho_{p+1}] after rho_{p+1} moves;
* the stopping test runs when k is a multiple of stop_every (k >= evol_hist);
* initial values: x = m, y_i = A_i m, v_i = 0, rho_i = rho0, gamma_i = gamma0;
* cardinality keeps exactly k entries: largest |w| first, ties to the lower
  linear index.

Parity of the adapt-rho-gamma trajectory (beyond its hand-checked single
calls) and of cardinality end-to-end runs is unpinned: the paper prints no
worked example and the non-convex set has no closed-form reference.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

AXIS_OPS = {
    2: {"I": (), "DZ": (0,), "DX": (1,), "GRAD": (0, 1), "LAT": (1,)},
    3: {"I": (), "DZ": (0,), "DY": (1,), "DX": (2,), "GRAD": (0, 1, 2), "LAT": (1, 2)},
}


# ---------------------------------------------------------------------------
# Linear operators (Sec. "Notation, assumptions, and definitions", eq. FD_mat)
# ---------------------------------------------------------------------------

def fd_matrix(n: int, h: float) -> sp.csr_matrix:
    """The (n-1) x n first-order forward difference of eq. (FD_mat): row j
    holds -1/h at column j and +1/h at column j+1."""
    rows, cols, vals = [], [], []
    for j in range(n - 1):
        rows += [j, j]
        cols += [j, j + 1]
        vals += [-1.0 / h, 1.0 / h]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n - 1, n), dtype=np.float64)


def axis_difference(shape, h, axis: int) -> sp.csr_matrix:
    """D along one grid axis, lifted with identities: for a 2D grid and
    axis z this is D_z (x) I_x, for axis x it is I_z (x) D_x (eq. FD_mat and
    the Kronecker definition that follows it)."""
    factors = [sp.identity(n, dtype=np.float64, format="csr") for n in shape]
    factors[axis] = fd_matrix(shape[axis], h[axis])
    out = factors[0]
    for f in factors[1:]:
        out = sp.kron(out, f, format="csr")
    return out.tocsr()


def operator(op: str, shape, h=None) -> sp.csr_matrix:
    """A_i for one set.  "I" is the identity; "DZ"/"DY"/"DX" one difference;
    "GRAD" stacks every axis difference (anisotropic total variation, as in
    the 341x400 example's TV set); "LAT" stacks the lateral ones (y, x)."""
    shape = tuple(int(n) for n in shape)
    h = tuple(float(v) for v in (h if h is not None else (1.0,) * len(shape)))
    n_pts = int(np.prod(shape))
    if op == "I":
        return sp.identity(n_pts, dtype=np.float64, format="csr")
    axes = AXIS_OPS[len(shape)][op]
    return sp.vstack([axis_difference(shape, h, a) for a in axes], format="csr")


# ---------------------------------------------------------------------------
# Projections onto simple sets (Table set-overview) and the distance prox
# ---------------------------------------------------------------------------

def project_bounds(w, lo, hi):
    """Element-wise bounds lo <= w[i] <= hi."""
    return np.minimum(np.maximum(w, lo), hi)


def project_l1(w, tau):
    """Euclidean projection onto {y : ||y||_1 <= tau} by sorting (the
    sort-and-threshold method the paper cites, Duchi et al. 2008): if w is
    inside the ball it is returned; otherwise with u = |w| sorted descending
    and c its running sum, rho is the largest j with u_j > (c_j - tau)/j,
    theta = (c_rho - tau)/rho and y = sign(w) max(|w| - theta, 0)."""
    w = np.asarray(w, dtype=np.float64)
    if tau <= 0.0:
        return np.zeros_like(w)
    a = np.abs(w)
    if a.sum() <= tau:
        return w.copy()
    u = np.sort(a)[::-1]
    c = np.cumsum(u)
    j = np.arange(1, u.size + 1)
    rho = int(np.nonzero(u - (c - tau) / j > 0)[0][-1]) + 1
    theta = (c[rho - 1] - tau) / rho
    return np.sign(w) * np.maximum(a - theta, 0.0)


def card_support(w, k):
    """Indices kept by the cardinality projection card(y) <= k: the k entries
    of largest |w|, ties broken toward the lower linear index (stable sort)."""
    w = np.asarray(w, dtype=np.float64)
    order = np.lexsort((np.arange(w.size), -np.abs(w)))
    return np.sort(order[: int(k)])


def project_card(w, k):
    """Projection onto {y : card(y) <= k} (a non-convex set): keep k entries."""
    w = np.asarray(w, dtype=np.float64)
    y = np.zeros_like(w)
    keep = card_support(w, k)
    y[keep] = w[keep]
    return y


def project_l2(w, tau):
    """Euclidean projection onto the l2 ball {y : ||y||_2 <= tau} (Table
    set-overview): w itself when inside, otherwise w scaled back to the
    sphere, tau w / ||w||."""
    w = np.asarray(w, dtype=np.float64)
    nrm = float(np.linalg.norm(w))
    if nrm <= tau:
        return w.copy()
    return w * (tau / nrm)


def project_annulus(w, lo, hi):
    """Projection onto the annulus {y : lo <= ||y||_2 <= hi} (Table
    set-overview; not convex when lo > 0): w itself inside, otherwise w
    scaled radially to the nearer radius.  At w = 0 with lo > 0 every point of
    the inner sphere is nearest; the reading takes lo e_0 (the first row)."""
    w = np.asarray(w, dtype=np.float64)
    nrm = float(np.linalg.norm(w))
    if lo <= nrm <= hi:
        return w.copy()
    if nrm > hi:
        return w * (hi / nrm)
    if nrm > 0.0:
        return w * (lo / nrm)
    y = np.zeros_like(w)
    y[0] = lo
    return y


def project_set(s: dict, w):
    """P_{C_i}(w).  Bounds take scalars or per-row vectors (per-pixel
    bounds l[i] <= (A x)[i] <= u[i], in A's row order)."""
    kind = s["kind"]
    if kind == "bounds":
        return project_bounds(w, np.asarray(s["lo"], dtype=np.float64), np.asarray(s["hi"], dtype=np.float64))
    if kind == "l1":
        return project_l1(w, s["tau"])
    if kind == "card":
        return project_card(w, s["k"])
    if kind == "l2":
        return project_l2(w, s["tau"])
    if kind == "annulus":
        return project_annulus(w, s["lo"], s["hi"])
    raise ValueError(f"unknown set kind {kind!r}")


# Line-wise sets (the paper's constraints "for each row / column / fiber"):
# the operator is the same; the simple set's projection acts on every line
# of A x on its own.  Readings: A x is split into its component blocks (one
# image per component, one layer shorter along the component's difference
# axis); within a block, the entries that share every grid coordinate except
# the one along the line axis form one line, in increasing order along it
# (2D: line "x" is a row X[i, :], line "z" a column X[:, j]; 3D adds "y");
# l1, cardinality, l2 and annulus sets may be line-wise (bounds act entry by
# entry anyway); the annulus at a zero line takes lo on the line's first entry.
LINE_AXES = {2: {"z": 0, "x": 1}, 3: {"z": 0, "y": 1, "x": 2}}


def line_rows(op: str, shape, line: str):
    """Row indices of A (operator op on the grid) grouped into lines, A's row
    order inside each line."""
    shape = tuple(int(n) for n in shape)
    ax_line = LINE_AXES[len(shape)][line]
    axes = AXIS_OPS[len(shape)][op] if op != "I" else (None,)
    out, off = [], 0
    for a in axes:
        sh = list(shape)
        if a is not None:
            sh[a] -= 1
        cnt = int(np.prod(sh))
        idx = (np.arange(cnt) + off).reshape(sh)
        if cnt:
            out.extend(np.moveaxis(idx, ax_line, -1).reshape(-1, sh[ax_line]))
        off += cnt
    return out


def project_lines(s: dict, w, lines):
    """The set's projection applied to every line of w independently."""
    base = {k: v for k, v in s.items() if k != "line"}
    y = np.asarray(w, dtype=np.float64).copy()
    for idx in lines:
        y[idx] = project_set(base, y[idx])
    return y


def prox_sq_dist(w, m, rho):
    """prox of f(z) = 1/2 ||z - m||^2 with penalty rho: (m + rho w)/(1 + rho),
    eq. (prox_sq_dist)."""
    return (m + rho * w) / (1.0 + rho)


# ---------------------------------------------------------------------------
# Options and state
# ---------------------------------------------------------------------------

@dataclass
class Options:
    max_iter: int = 200
    cg_max: int = 10
    cg_fixed: bool = True
    cg_rel: float = 0.1
    adapt_every: int = 2
    stop_every: int = 0          # 0: no stopping test, run max_iter iterations
    evol_hist: int = 5
    eps_evol: float = 1e-2
    eps_feas: float = 1e-3
    rho0: float = 1.0
    gamma0: float = 1.0
    eps_corr: float = 0.3
    rho_ratio_max: float = 100.0
    gamma_max: float = 1.999


@dataclass
class Snapshot:
    vhat: np.ndarray
    v: np.ndarray
    s: np.ndarray
    y: np.ndarray


@dataclass
class State:
    """Everything PARSDMM carries between iterations.  Index p (the last) is
    the extra identity block A_{p+1} = I with f_{p+1} = 1/2 ||. - m||^2."""
    x: np.ndarray
    y: list
    v: list
    rho: np.ndarray
    gamma: np.ndarray
    k: int = 1
    snaps: list = field(default_factory=list)
    x_hist: list = field(default_factory=list)
    cg_steps: int = 0
    converged: bool = False
    r_feas: np.ndarray | None = None
    r_evol: float = math.inf
    w_last: list = field(default_factory=list)   # prox arguments of the last iteration
    cg_trace: list = field(default_factory=list)  # ||r_j|| / ||r_0|| of the last x-update
    cg_r0_rel: float = 0.0                        # ||b - C x^k|| / ||b|| of the last x-update


class Problem:
    """m, the grid, the sets and everything precomputed from them: the
    operators A_1..A_p, A_{p+1} = I and B_i = A_i^T A_i (PARSDMM listing,
    initialisation)."""

    def __init__(self, m, shape, sets, h=None):
        self.shape = tuple(int(n) for n in shape)
        self.h = tuple(float(v) for v in (h if h is not None else (1.0,) * len(self.shape)))
        self.m = np.asarray(m, dtype=np.float64).reshape(-1)
        self.n = self.m.size
        self.sets = [dict(s) for s in sets]
        for s in self.sets:
            if s.get("line") is not None and s["kind"] not in ("l1", "card", "l2", "annulus"):
                raise ValueError("line-wise sets are l1, card, l2 or annulus sets")
        self.A = [operator(s["op"], self.shape, self.h) for s in self.sets]
        self.lines = [line_rows(s["op"], self.shape, s["line"]) if s.get("line") is not None else None
                      for s in self.sets]
        self.A.append(sp.identity(self.n, dtype=np.float64, format="csr"))
        self.B = [(a.T @ a).tocsr() for a in self.A]
        self.p = len(self.sets)

    def system_matrix(self, rho) -> sp.csr_matrix:
        """C = sum_{i=1}^{p+1} rho_i A_i^T A_i, eq. (sys_mat)."""
        c = self.B[0] * rho[0]
        for i in range(1, self.p + 1):
            c = c + self.B[i] * rho[i]
        return c.tocsr()

    def project(self, i, w):
        """P_{C_i}(w), line by line for a line-wise set."""
        if self.lines[i] is not None:
            return project_lines(self.sets[i], w, self.lines[i])
        return project_set(self.sets[i], w)

    def prox(self, i, w, rho_i, keep=None):
        """prox_i(w); ``keep`` (cardinality sets only) replaces the set's own
        choice of the k kept rows by the given row indices (support-locked
        replay of another run: the projection is then y = w on those rows and
        0 elsewhere)."""
        if i == self.p:
            return prox_sq_dist(w, self.m, rho_i)
        if keep is not None:
            if self.sets[i]["kind"] != "card" or self.lines[i] is not None:
                raise ValueError("a kept support is replayed only for whole-vector cardinality sets")
            y = np.zeros_like(w)
            y[keep] = w[keep]
            return y
        return self.project(i, w)


def initial_state(prob: Problem, opts: Options) -> State:
    """x = m, y_i = A_i m, v_i = 0, rho_i = rho0, gamma_i = gamma0, k = 1."""
    x = prob.m.copy()
    y = [a @ x for a in prob.A]
    v = [np.zeros(a.shape[0]) for a in prob.A]
    n = prob.p + 1
    return State(x=x, y=y, v=v, rho=np.full(n, opts.rho0), gamma=np.full(n, opts.gamma0),
                 snaps=[None] * n, x_hist=[x.copy()])


# ---------------------------------------------------------------------------
# x-update: conjugate gradients on C x = b (eqs. SDMM_adaptive, sys_mat, cg_stop)
# ---------------------------------------------------------------------------

def rhs(prob: Problem, st: State) -> np.ndarray:
    """b = sum_{i=1}^{p+1} A_i^T (rho_i y_i + v_i)."""
    b = np.zeros(prob.n)
    for i, a in enumerate(prob.A):
        b += a.T @ (st.rho[i] * st.y[i] + st.v[i])
    return b


def cg(C, b, x0, cg_rel=0.1, cg_max=10, fixed=True, steps_forced=None, trace=None):
    """Plain conjugate gradients from the warm start x0.  Returns (x, steps).
    Stops when ||r|| < cg_rel ||r_0|| (unless ``fixed``), when the residual is
    exactly zero, or after cg_max steps.  A non-positive curvature p^T C p with
    a non-zero residual raises (C is SPD in exact arithmetic).
    ``steps_forced`` (replay of another run's stopping decisions) runs exactly
    that many steps unless the residual becomes exactly zero; ``trace``, a
    list, receives ||r_j|| / ||r_0|| before every step j and after the last."""
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - C @ x
    rr = float(r @ r)
    rr0 = rr
    p = r.copy()
    steps = 0
    n = cg_max if steps_forced is None else int(steps_forced)
    for j in range(n):
        if trace is not None:
            trace.append(math.sqrt(rr / rr0) if rr0 > 0.0 else 0.0)
        if rr == 0.0:
            break
        if steps_forced is None and not fixed and j > 0 and rr < cg_rel * cg_rel * rr0:
            break
        q = C @ p
        pq = float(p @ q)
        if not pq > 0.0:
            raise FloatingPointError("CG breakdown: p^T C p <= 0")
        alpha = rr / pq
        x += alpha * p
        r -= alpha * q
        rr_new = float(r @ r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        steps += 1
    if trace is not None and steps == n:
        trace.append(math.sqrt(rr / rr0) if rr0 > 0.0 else 0.0)
    return x, steps


# ---------------------------------------------------------------------------
# Automatic penalty and relaxation (section "Solving the linear system and
# automatic parameter selection"; the adaptive relaxed ADMM of Xu et al. 2017
# that the paper adopts), one set at a time
# ---------------------------------------------------------------------------

def _spectral(d_a, d_b, eps_corr):
    """Spectral (Barzilai-Borwein type) curvature estimate of one of the two
    dual-function pieces from a pair of differences over the adaptation
    interval: the pair is trusted only when the differences are correlated,
    cos(d_a, d_b) > eps_corr, and then the estimate blends the
    minimum-gradient value d_a.d_b / d_a.d_a with the steepest-descent value
    d_b.d_b / d_a.d_b (the former when twice it exceeds the latter, else
    the latter minus half the former).  Returns (trusted, estimate)."""
    ab = float(d_a @ d_b)
    aa = float(d_a @ d_a)
    bb = float(d_b @ d_b)
    den = math.sqrt(aa) * math.sqrt(bb)
    if den == 0.0:
        return False, 0.0
    corr = ab / den
    if not corr > eps_corr:
        return False, 0.0
    mg = ab / aa
    sd = bb / ab
    est = mg if 2.0 * mg > sd else sd - 0.5 * mg
    return True, est


def _penalty_relaxation(trusted_a, a, trusted_b, b, rho):
    """The new (rho, gamma) from the two curvature estimates: with both
    trusted, rho is their geometric mean and gamma = 1 + 2 sqrt(a b)/(a + b);
    with one, rho follows it and gamma is 1.9 (from a) or 1.1 (from b); with
    neither, rho stays and gamma is 1.5."""
    if trusted_a and trusted_b:
        g = math.sqrt(a * b)
        return g, 1.0 + 2.0 * g / (a + b)
    if trusted_a:
        return a, 1.9
    if trusted_b:
        return b, 1.1
    return rho, 1.5


def adapt_rho_gamma(s, y_old, y_new, v_old, v_new, rho, gamma, snap, eps_corr=0.3):
    """One adaptation of (rho_i, gamma_i) for one set.

    The two dual pieces are probed through their iterates: the unrelaxed
    multiplier v-hat = v^k + rho (y^k - s^{k+1}) against s = A_i x^{k+1}
    (the x-side piece), and v^{k+1} against -y^{k+1} (the y-side piece), y^k
    being y before this iteration's update.  Their differences since the
    snapshot of the previous adaptation give the two curvature estimates
    (_spectral), which set the new penalty and relaxation
    (_penalty_relaxation).  The first adaptation has no snapshot and keeps
    (rho, gamma).  Returns (rho, gamma, the snapshot for the next
    adaptation)."""
    vhat = v_old + rho * (y_old - s)
    new_snap = Snapshot(vhat=vhat.copy(), v=v_new.copy(), s=s.copy(), y=y_new.copy())
    if snap is None:
        return rho, gamma, new_snap
    trusted_a, a = _spectral(s - snap.s, vhat - snap.vhat, eps_corr)
    trusted_b, b = _spectral(-(y_new - snap.y), v_new - snap.v, eps_corr)
    rho_new, gamma_new = _penalty_relaxation(trusted_a, a, trusted_b, b, rho)
    return rho_new, gamma_new, new_snap


def guard_parameters(rho, gamma, opts: Options):
    """gamma_i <= gamma_max (the relaxation must stay below 2) and
    rho_{p+1}/R <= rho_i <= R rho_{p+1} for i <= p (the paper limits the
    ratio to keep C well conditioned without giving R)."""
    rho = np.array(rho, dtype=np.float64)
    gamma = np.minimum(np.array(gamma, dtype=np.float64), opts.gamma_max)
    r_last = rho[-1]
    rho[:-1] = np.clip(rho[:-1], r_last / opts.rho_ratio_max, r_last * opts.rho_ratio_max)
    return rho, gamma


# ---------------------------------------------------------------------------
# Stopping conditions (eqs. feas_stop, obj_stop, stopping_conditions)
# ---------------------------------------------------------------------------

def feasibility_error(s: dict, ax, lines=None):
    """r_feas = ||A x - P_C(A x)|| / ||A x||; with A x = 0 it is 0 when A x is
    in C and infinity otherwise."""
    proj = project_lines(s, ax, lines) if lines is not None else project_set(s, ax)
    num = float(np.linalg.norm(ax - proj))
    den = float(np.linalg.norm(ax))
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return num / den


def relative_evolution(x, history):
    """r_evol = max_j ||x^k - x^{k-j}|| / ||x^k|| over the stored history."""
    nx = float(np.linalg.norm(x))
    worst = max(float(np.linalg.norm(x - h)) for h in history)
    if nx == 0.0:
        return 0.0 if worst == 0.0 else math.inf
    return worst / nx


# ---------------------------------------------------------------------------
# One PARSDMM iteration and the full run (the PARSDMM listing)
# ---------------------------------------------------------------------------

def x_update(prob: Problem, st: State, opts: Options, steps_forced=None) -> int:
    """x^{k+1} = C^{-1} sum_i A_i^T (rho_i y_i + v_i) by warm-started CG
    (``steps_forced``: replay another run's number of CG steps; the residual
    ratios of this x-update are left in st.cg_trace, and ||b - C x^k|| / ||b||
    in st.cg_r0_rel)."""
    C = prob.system_matrix(st.rho)
    b = rhs(prob, st)
    nb = float(np.linalg.norm(b))
    st.cg_r0_rel = float(np.linalg.norm(b - C @ st.x)) / nb if nb > 0.0 else 0.0
    st.cg_trace = []
    st.x, steps = cg(C, b, st.x, opts.cg_rel, opts.cg_max, opts.cg_fixed, steps_forced, st.cg_trace)
    st.cg_steps += steps
    return steps


def set_updates(prob: Problem, st: State, keep=None):
    """For i = 1..p+1: s_i = A_i x, x-bar_i = gamma_i s_i + (1 - gamma_i) y_i,
    y_i = prox_i(x-bar_i - v_i/rho_i), v_i += rho_i (y_i - x-bar_i).
    Returns the s_i and the pre-update y_i and v_i (adapt-rho-gamma needs them)."""
    s_all, y_old, v_old = [], [], []
    st.w_last = []
    for i, a in enumerate(prob.A):
        s = a @ st.x
        xbar = st.gamma[i] * s + (1.0 - st.gamma[i]) * st.y[i]
        w = xbar - st.v[i] / st.rho[i]
        st.w_last.append(w)
        y_old.append(st.y[i])
        v_old.append(st.v[i])
        st.y[i] = prob.prox(i, w, st.rho[i], None if keep is None else keep.get(i))
        st.v[i] = st.v[i] + st.rho[i] * (st.y[i] - xbar)
        s_all.append(s)
    return s_all, y_old, v_old


def stop_test(prob: Problem, st: State, opts: Options) -> bool:
    st.r_feas = np.array([feasibility_error(s, a @ st.x, ln) for s, a, ln in zip(prob.sets, prob.A, prob.lines)])
    st.r_evol = relative_evolution(st.x, st.x_hist[-opts.evol_hist - 1:-1])
    return bool(st.r_evol < opts.eps_evol and np.all(st.r_feas < opts.eps_feas))


def adapt(prob: Problem, st: State, s_all, y_old, v_old, opts: Options):
    """adapt-rho-gamma for every i = 1..p+1, then the guards; C follows from
    the new rho at the next x-update."""
    rho, gamma = st.rho.copy(), st.gamma.copy()
    for i in range(prob.p + 1):
        rho[i], gamma[i], st.snaps[i] = adapt_rho_gamma(
            s_all[i], y_old[i], st.y[i], v_old[i], st.v[i], st.rho[i], st.gamma[i],
            st.snaps[i], opts.eps_corr)
    st.rho, st.gamma = guard_parameters(rho, gamma, opts)


def iterate(prob: Problem, st: State, opts: Options, schedule=None, supports=None) -> bool:
    """One PARSDMM iteration.  ``schedule`` (optional) maps k to (rho, gamma)
    to use in iteration k instead of the adapted values, or to (rho, gamma,
    CG steps) to replay the number of CG steps as well (schedule-locked
    replay of another run); ``supports`` (optional) maps k to {set index:
    kept row indices} for cardinality sets (support-locked replay: a
    non-convex set has several equally valid projections where entries tie
    or nearly tie at the k-th magnitude, so a replay may take the other run's
    choice; the caller checks that choice against the oracle's own w).
    Returns True when the stopping test passed."""
    forced = None
    if schedule is not None and st.k in schedule:
        st.rho = np.array(schedule[st.k][0], dtype=np.float64)
        st.gamma = np.array(schedule[st.k][1], dtype=np.float64)
        if len(schedule[st.k]) > 2:
            forced = schedule[st.k][2]
    x_update(prob, st, opts, forced)
    s_all, y_old, v_old = set_updates(prob, st, None if supports is None else supports.get(st.k))
    st.x_hist.append(st.x.copy())
    if len(st.x_hist) > opts.evol_hist + 1:
        st.x_hist.pop(0)
    stop = False
    if opts.stop_every and st.k % opts.stop_every == 0 and st.k >= opts.evol_hist:
        stop = stop_test(prob, st, opts)
    if not stop and opts.adapt_every and st.k % opts.adapt_every == 1 % opts.adapt_every:
        adapt(prob, st, s_all, y_old, v_old, opts)
    st.k += 1
    return stop


def parsdmm(m, shape, sets, opts: Options | None = None, h=None, schedule=None,
            state: State | None = None, supports=None):
    """Project m onto the intersection of the sets.  Returns (x, state)."""
    opts = opts or Options()
    prob = Problem(m, shape, sets, h)
    st = state if state is not None else initial_state(prob, opts)
    while st.k <= opts.max_iter:
        if iterate(prob, st, opts, schedule, supports):
            st.converged = True
            break
    return st.x.reshape(prob.shape), st
