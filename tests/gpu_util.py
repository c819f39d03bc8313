"""Helpers for GPU-vs-oracle parity: layout conversion between the device
state (one N-element block per operator component, last layer along the
component's axis unused) and the oracle's stacked operator rows, and state
transfer from a device batch slot into an oracle State."""
from __future__ import annotations

import math

import numpy as np

from oracle import parsdmm as orc
from paper_1902_09699_amd import sip
from paper_1902_09699_amd import workloads as wl

_COMP_AXES = {
    2: {"I": (None,), "DZ": (0,), "DX": (1,), "GRAD": (0, 1), "LAT": (1,)},
    3: {"I": (None,), "DZ": (0,), "DY": (1,), "DX": (2,), "GRAD": (0, 1, 2), "LAT": (1, 2)},
}


def unpad(shape, op, flat, stride=None):
    """Device component blocks (block c at c * stride) -> oracle row vector
    (A_i's row order)."""
    N = int(np.prod(shape))
    stride = N if stride is None else stride
    parts = []
    for c, ax in enumerate(_COMP_AXES[len(shape)][op]):
        blk = np.asarray(flat[c * stride:c * stride + N]).reshape(shape)
        if ax is not None:
            sl = [slice(None)] * len(shape)
            sl[ax] = slice(0, shape[ax] - 1)
            blk = blk[tuple(sl)]
        parts.append(blk.ravel())
    return np.concatenate(parts)


def pad(shape, op, rows, stride=None):
    N = int(np.prod(shape))
    stride = N if stride is None else stride
    axes = _COMP_AXES[len(shape)][op]
    out = np.zeros(len(axes) * stride)
    off = 0
    for c, ax in enumerate(axes):
        sh = list(shape)
        if ax is not None:
            sh[ax] -= 1
        cnt = int(np.prod(sh))
        blk = np.zeros(shape)
        sl = tuple(slice(0, s) for s in sh)
        blk[sl] = np.asarray(rows[off:off + cnt]).reshape(sh)
        out[c * stride:c * stride + N] = blk.ravel()
        off += cnt
    return out


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    d = np.linalg.norm(a - b)
    return d / nb if nb > 0 else d


def make_case(kind, seed=0):
    """Small instances spanning several tiles with ragged tails."""
    if kind == "box_tv_2d":
        m, sets, _, _ = wl.smooth2d_box_tv(n=(37, 45), seed=seed + 11)
    elif kind == "four_sets_2d":
        m, sets, _, _ = wl.layered2d_four_sets(n=(41, 67), seed=seed + 12)
    elif kind == "box_tv_lat_3d":
        m, sets, _, _ = wl.smooth3d_box_tv_lat(n=(11, 13, 17), seed=seed + 13)
        m = m * 0.8
    elif kind == "mixed_2d":
        rng = wl.rng_for(seed + 14)
        m = wl.grf((29, 53), 5.0, rng)
        sets = [wl.l1("I", 0.5), wl.card("GRAD", 0.1), wl.bounds("DX", -0.3, 0.3), wl.bounds("DZ", -0.25, math.inf)]
    elif kind == "mixed_3d":
        rng = wl.rng_for(seed + 15)
        m = wl.grf((9, 12, 14), 3.0, rng)
        sets = [wl.bounds("DY", -0.2, 0.2), wl.l1("LAT", 0.6), wl.card("DZ", 0.2), wl.bounds("I", -1.2, 1.2)]
    else:
        raise KeyError(kind)
    return m, sets


class Slot:
    """One device instance in a fresh batch, with helpers to read its state."""

    def __init__(self, m, sets, field, opts_kw, tiles=(1024, 1024, 1024, 512)):
        import torch
        self.shape = m.shape
        self.sets = sets
        self.field = field
        self.opts = sip.make_opts(field, **opts_kw)
        dt = torch.float64 if field == "f64" else torch.float32
        self.md = torch.tensor(m, dtype=dt, device="cuda")
        self.xd = torch.empty_like(self.md)
        ws = sip.workspace_bytes(self.shape, sets, self.opts)
        self.batch = sip.Batch(1, ws, self.opts)
        self.batch.set_tiles(*tiles)
        self.slot = self.batch.add(self.md, sets, self.xd)
        assert self.slot == 0

    def x(self):
        import torch
        torch.cuda.synchronize()
        return self.xd.double().cpu().numpy().ravel()

    def arr(self, which, i):
        op = "I" if i == len(self.sets) else self.sets[i]["op"]
        t = self.batch.field_tensor(self.slot, which, i).double().cpu().numpy()
        cs = self.batch.field(self.slot, which, i)[2]
        return unpad(self.shape, op, t, cs)

    def raw(self, which, i):
        return self.batch.field_tensor(self.slot, which, i).double().cpu().numpy()


class SlotView(Slot):
    """One instance of a batch that holds others too (same helpers as Slot)."""

    def __init__(self, batch, slot, m, sets, field, md, xd):
        self.shape = m.shape
        self.sets = sets
        self.field = field
        self.batch = batch
        self.slot = slot
        self.md = md
        self.xd = xd


def sync_oracle(sl: Slot, prob: orc.Problem, st: orc.State):
    """Overwrite the oracle state with the device state (exact upcast)."""
    p = len(sl.sets)
    st.x = sl.x()
    st.y = [sl.arr(sip.FIELD_Y, i) for i in range(p + 1)]
    st.v = [sl.arr(sip.FIELD_V, i) for i in range(p + 1)]
    rho, gam, k, have = sl.batch.get_params(sl.slot)
    st.rho, st.gamma, st.k = rho.copy(), gam.copy(), k
    if have:
        # the x snapshot the next adapt call reads: call c uses buffer (c & 1) ^ 1
        kk = k if k % 2 == 1 else k + 1
        c = (kk - 1) // 2 + 1
        xs = sl.raw(sip.FIELD_XS0 if ((c & 1) ^ 1) == 0 else sip.FIELD_XS1, 0)
        st.snaps = [orc.Snapshot(vhat=sl.arr(sip.FIELD_VHAT0, i), v=sl.arr(sip.FIELD_V0, i),
                                 s=prob.A[i] @ xs, y=sl.arr(sip.FIELD_Y0, i)) for i in range(p + 1)]
    else:
        st.snaps = [None] * (p + 1)


# ------------------------------------------------- cardinality sets, replays

# Entries whose |w| lies within this fraction of the k-th magnitude t_k count
# as ties of the cardinality projection: either choice among them is a valid
# projection, so supports are compared outside the band only.
CARD_BAND = 1e-4


def card_sets(sets):
    """Indices of the whole-vector cardinality sets."""
    return [i for i, s in enumerate(sets) if s["kind"] == "card" and s.get("line") is None]


def band_mask(w, k, band=CARD_BAND):
    """Rows of w whose |w| is farther than band * t_k from the k-th largest
    magnitude t_k (outside the tie band)."""
    a = np.abs(np.asarray(w, dtype=np.float64))
    tk = np.partition(a, a.size - k)[a.size - k]
    return np.abs(a - tk) > band * max(tk, 1e-300)


def support_report(w, keep, k, band=CARD_BAND):
    """Check that the rows `keep` are a valid choice of the k largest |w|
    (ties within band * t_k may go either way): returns (valid, entries
    where keep differs from the oracle's own choice, largest relative
    distance of those from t_k)."""
    a = np.abs(np.asarray(w, dtype=np.float64))
    keep = np.asarray(keep)
    own = orc.card_support(w, k)
    tk = np.partition(a, a.size - k)[a.size - k]
    dropped = np.ones(a.size, bool)
    dropped[keep] = False
    ok = keep.size <= k and (keep.size == k or np.all(a[keep] != 0) and not np.any(a[dropped] > 0))
    lo = tk * (1.0 - band)
    hi = tk * (1.0 + band)
    ok = ok and bool(np.all(a[keep] >= lo)) and bool(np.all(a[dropped] <= hi))
    diff = np.setxor1d(own, keep)
    dist = float(np.max(np.abs(a[diff] - tk)) / max(tk, 1e-300)) if diff.size else 0.0
    return ok, int(diff.size), dist


def run_logged(sl: Slot, iters):
    """Advance a slot one iteration at a time (stopping when it finishes);
    returns {k: (rho, gamma, CG steps)} of every iteration run and the rows
    each whole-vector cardinality set kept, {k: {set: rows}} (the oracle's
    row order)."""
    sched, sup = {}, {}
    ic = card_sets(sl.sets)
    cg_before = sl.batch.result(sl.slot)["cg_steps"]
    for _ in range(iters):
        rho, gam, k, _ = sl.batch.get_params(sl.slot)
        sl.batch.run(1)
        res = sl.batch.result(sl.slot)
        if res["iters"] < k:
            break  # finished before this iteration
        sched[k] = (rho.copy(), gam.copy(), res["cg_steps"] - cg_before)
        cg_before = res["cg_steps"]
        if ic:
            sup[k] = {i: np.nonzero(sl.arr(sip.FIELD_Y, i))[0] for i in ic}
        if sl.batch.poll()[sl.slot] == 1:
            break
    return sched, sup


# A replayed CG step count is a valid stopping decision when the oracle's
# own residual ratio at that step is below cg_rel and at every earlier step
# above it, up to this relative band (eq. cg_stop is a threshold test).
CG_BAND = 1e-3
# Below this ||b - C x^k|| / ||b|| the warm start already solves the system
# to the rounding of a float32 right-hand side (the first x-update returns
# m): the residual is rounding noise and the count decided on it is not
# compared.
CG_NOISE = 1e-5


def cg_decision_ok(trace, n, cg_rel, cg_max):
    if len(trace) <= n:
        # the oracle's residual became exactly zero before step n
        return trace[-1] == 0.0
    if n < cg_max and not (trace[n] < cg_rel * (1 + CG_BAND) or trace[n] == 0.0):
        return False
    return all(t >= cg_rel * (1 - CG_BAND) for t in trace[1:n])


def replay_locked(m, sets, opts: orc.Options, sched, sup, h=None):
    """The oracle replaying another run's (rho, gamma, CG steps) schedule and
    cardinality supports.  Every replayed support is checked against the
    oracle's own w of that iteration and, with the relative CG stop on, every
    CG step count against the oracle's own residual ratios.  Returns (state,
    [(k, set, valid, differing entries, distance from t_k)], [(k, CG count
    valid, count differs from the oracle's own)]).  The replay stops where
    the oracle's own stopping test passes (or at the end of the schedule)."""
    prob = orc.Problem(m, m.shape, sets, h)
    st = orc.initial_state(prob, opts)
    ic = card_sets(sets)
    rep, cgrep = [], []
    while st.k <= opts.max_iter and st.k in sched:
        k = st.k
        stop = orc.iterate(prob, st, opts, sched, sup)
        for i in ic:
            rep.append((k, i) + support_report(st.w_last[i], sup[k][i], sets[i]["k"]))
        if len(sched[k]) > 2 and not opts.cg_fixed and st.cg_r0_rel >= CG_NOISE:
            n = sched[k][2]
            tr = st.cg_trace
            own = next((j for j in range(1, len(tr)) if tr[j] < opts.cg_rel or tr[j] == 0.0), opts.cg_max)
            own = min(own, opts.cg_max)
            cgrep.append((k, cg_decision_ok(tr, n, opts.cg_rel, opts.cg_max), own != n))
        if stop:
            st.converged = True
            break
    return st, rep, cgrep


def slot_rows(batch, slot, shape, sets, which, i):
    """A state array of any slot of a batch in the oracle's row order."""
    op = "I" if i == len(sets) else sets[i]["op"]
    t = batch.field_tensor(slot, which, i).double().cpu().numpy()
    return unpad(shape, op, t, batch.field(slot, which, i)[2])


# Multiple of the measured x-rounding spread a float32 step may differ from
# the oracle by (see rounding_spread).
SPREAD_MULT = 16.0


def rounding_spread(prob: orc.Problem, st_before: orc.State, opts: orc.Options, field: str):
    """How far one iteration's y_i and v_i move when the oracle's x, right
    after its x-update, is rounded to the field type: the part of a
    device-vs-oracle difference that fields of that precision cannot avoid
    (float32 rounding of x reaches A_i x amplified by the difference
    operators, which is large against small differences of a smooth x).
    Cardinality sets keep the unrounded run's rows in both runs.  Returns per
    unit (y spread, v spread), each relative to max(||y||, ||w||) and
    max(||v||, ||y||, ||w||) of the unrounded run."""
    import copy
    if field == "f64":
        return [(0.0, 0.0)] * (prob.p + 1)
    a = copy.deepcopy(st_before)
    orc.x_update(prob, a, opts)
    b = copy.deepcopy(a)
    b.x = b.x.astype(np.float32).astype(np.float64)
    orc.set_updates(prob, a)
    keep = {i: orc.card_support(a.w_last[i], prob.sets[i]["k"]) for i in card_sets(prob.sets)}
    orc.set_updates(prob, b, keep)
    out = []
    for i in range(prob.p + 1):
        sc = max(np.linalg.norm(a.y[i]), np.linalg.norm(a.w_last[i]), 1e-300)
        out.append((float(np.linalg.norm(b.y[i] - a.y[i]) / sc),
                    float(np.linalg.norm(b.v[i] - a.v[i]) / max(np.linalg.norm(a.v[i]), sc))))
    return out


def compare_step(sl: Slot, prob: orc.Problem, st: orc.State, spread, tol, label=""):
    """Device state after one iteration against the oracle's (both started
    from the same state): x relative to ||x||; y_i relative to
    max(||y_i||, ||w_i||) and v_i relative to max(||v_i||, ||y_i||, ||w_i||),
    each gated at max(tol, SPREAD_MULT * the measured rounding spread);
    cardinality supports identical outside the tie band.  Returns the worst
    error and the worst error / spread ratio."""
    ex = rel(sl.x(), st.x)
    assert ex <= tol, (label, "x", ex)
    worst, worst_ratio = ex, 0.0
    sets = sl.sets
    for i in range(len(sets) + 1):
        yg, vg = sl.arr(sip.FIELD_Y, i), sl.arr(sip.FIELD_V, i)
        yo, vo, wo = st.y[i], st.v[i], st.w_last[i]
        if i < len(sets) and sets[i]["kind"] == "card" and sets[i].get("line") is None:
            mask = band_mask(wo, sets[i]["k"])
            assert np.array_equal((yg != 0)[mask], (yo != 0)[mask]), (label, i, "card support")
            assert (yg != 0).sum() <= sets[i]["k"], (label, i, "card count")
            yg, yo, vg, vo = yg[mask], yo[mask], vg[mask], vo[mask]
        sc = max(np.linalg.norm(yo), np.linalg.norm(wo), 1e-300)
        ey = np.linalg.norm(yg - yo) / sc
        ev = np.linalg.norm(vg - vo) / max(np.linalg.norm(vo), sc)
        sy, sv = spread[i]
        gy, gv = max(tol, SPREAD_MULT * sy), max(tol, SPREAD_MULT * sv)
        assert ey <= gy, (label, i, "y", ey, "spread", sy)
        assert ev <= gv, (label, i, "v", ev, "spread", sv)
        worst = max(worst, ey, ev)
        if sy > 0:
            worst_ratio = max(worst_ratio, ey / sy)
        if sv > 0:
            worst_ratio = max(worst_ratio, ev / sv)
    return worst, worst_ratio
