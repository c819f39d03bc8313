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
