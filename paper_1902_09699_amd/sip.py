"""Thin ctypes binding of libsip (include/sip.h).

Argument marshalling only: every step of the projection runs in the HIP
kernels of libsip.so.  PyTorch supplies device memory and streams.  The
library must have been built in-tree (paper_1902_09699_amd/build.py); there
is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsip.so")

MAX_SETS = 16

OK, EINVAL, ENOMEM, EHIP, ENUMERIC, EUNSUPPORTED, EBUDGET, ETOOLARGE = 0, -1, -2, -3, -4, -5, -6, -7
F32, F64 = 0, 1
OPS = {"I": 0, "DZ": 1, "DY": 2, "DX": 3, "GRAD": 4, "LAT": 5}
KINDS = {"bounds": 0, "l1": 1, "card": 2, "l2": 3, "annulus": 4}
K_RHS, K_CG_DIR, K_CG_UPD, K_PROJ, K_THR_W, K_THR_APPLY, K_CG1_STEP, K_CG1_W0, K_LINE, K_CG2_STEP, K_CG2_D0 = range(11)
FIELD_Y, FIELD_V, FIELD_VHAT0, FIELD_V0, FIELD_Y0, FIELD_R, FIELD_XS0, FIELD_XS1 = range(8)


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("reserved", C.c_int32), ("n", C.c_int64 * 3), ("h", C.c_double * 3)]


class Set(C.Structure):
    _fields_ = [("kind", C.c_int32), ("op", C.c_int32), ("lo", C.c_double), ("hi", C.c_double),
                ("tau", C.c_double), ("k", C.c_int64), ("lo_vec", C.c_void_p), ("hi_vec", C.c_void_p),
                ("line", C.c_int32), ("reserved_", C.c_int32)]


# line-wise sets: the axis of the lines ("z", "y", "x"; 2D: "x" rows, "z" columns)
LINES = {None: 0, "z": 1, "y": 2, "x": 3}


class Opts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("cg_max", C.c_int32), ("cg_fixed", C.c_int32),
                ("adapt_every", C.c_int32), ("stop_every", C.c_int32), ("evol_hist", C.c_int32),
                ("rho0", C.c_double), ("gamma0", C.c_double), ("eps_corr", C.c_double),
                ("rho_ratio_max", C.c_double), ("gamma_max", C.c_double), ("eps_evol", C.c_double),
                ("eps_feas", C.c_double), ("cg_rel", C.c_double), ("field", C.c_int32),
                ("reduce", C.c_int32), ("log_schedule", C.c_int32),
                ("sel_fresh", C.c_int32)]


class Tiles(C.Structure):
    _fields_ = [("pt_points", C.c_int32), ("pt_max_items", C.c_int32), ("thr_points", C.c_int32),
                ("thr_max_items", C.c_int32), ("pt_threads", C.c_int32), ("cg_form", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("cg_steps", C.c_int32),
                ("converged", C.c_int32), ("nsets", C.c_int32), ("sel_reused", C.c_int32),
                ("r_evol", C.c_double), ("r_feas", C.c_double * MAX_SETS),
                ("rho", C.c_double * (MAX_SETS + 1)), ("gamma", C.c_double * (MAX_SETS + 1))]

    def as_dict(self):
        p = self.nsets
        return {"status": self.status, "iters": self.iters, "cg_steps": self.cg_steps,
                "converged": bool(self.converged), "sel_reused": self.sel_reused, "r_evol": self.r_evol,
                "r_feas": list(self.r_feas[:p]), "rho": list(self.rho[:p + 1]),
                "gamma": list(self.gamma[:p + 1])}


class SipError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})" if what else strerror(status))


_lib = None


def _torch_first():
    """torch (which allocates the caller's device tensors) brings its own HIP
    runtime; it failed to find the GPU when the library's runtime had opened
    it first, so torch's is initialised before the library is loaded."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def lib():
    """Load libsip.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1902_09699_amd/build.py")
    _torch_first()
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "sip_strerror": (C.c_char_p, [i32]),
        "sip_opts_default": (i32, [C.POINTER(Opts)]),
        "sip_set_rows": (i64, [C.POINTER(Grid), C.POINTER(Set)]),
        "sip_validate": (i32, [C.POINTER(Grid), C.POINTER(Set), i32, C.POINTER(Opts)]),
        "sip_workspace_bytes": (i64, [C.POINTER(Grid), C.POINTER(Set), i32, C.POINTER(Opts)]),
        "sip_project": (i32, [C.POINTER(Grid), C.POINTER(Set), i32, C.POINTER(Opts), vp, vp,
                              C.POINTER(Result), vp]),
        "sip_project_batched": (i32, [i32, C.POINTER(Grid), C.POINTER(Set), C.POINTER(i32), C.POINTER(Opts),
                                      C.POINTER(vp), C.POINTER(vp), C.POINTER(Result), i32, vp]),
        "sip_batch_create": (i32, [C.POINTER(vp), i32, i64, C.POINTER(Opts)]),
        "sip_batch_destroy": (i32, [vp]),
        "sip_batch_add": (i32, [vp, C.POINTER(Grid), C.POINTER(Set), i32, vp, vp, C.POINTER(i32), vp]),
        "sip_batch_run": (i32, [vp, i32, vp]),
        "sip_batch_poll": (i32, [vp, C.POINTER(i32), vp]),
        "sip_batch_remove": (i32, [vp, i32, C.POINTER(Result), vp]),
        "sip_batch_result": (i32, [vp, i32, C.POINTER(Result), vp]),
        "sip_batch_field": (i32, [vp, i32, i32, i32, C.POINTER(vp), C.POINTER(i64), C.POINTER(i64)]),
        "sip_batch_get_params": (i32, [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(i32), C.POINTER(i32), vp]),
        "sip_batch_set_params": (i32, [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_double), i32, i32, vp]),
        "sip_batch_schedule": (i32, [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_double), i32,
                                     C.POINTER(i32), vp]),
        "sip_batch_set_tiles": (i32, [vp, i32, i32, i32, i32, i32, i32]),
        "sip_batch_reset": (i32, [vp, i32, vp, vp]),
        "sip_batch_time_kernel": (i32, [vp, i32, i32, vp, C.POINTER(C.c_double)]),
        "sip_stream_copy": (i32, [vp, vp, i64, vp]),
        "sip_batch_items": (i32, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "sip_level": (i32, [C.POINTER(Grid), C.POINTER(Set), i32, i32, C.POINTER(Grid), C.POINTER(Set)]),
        "sip_restrict": (i32, [C.POINTER(Grid), i32, vp, vp, vp]),
        "sip_project_multilevel": (i32, [C.POINTER(Grid), C.POINTER(Set), i32, C.POINTER(Opts), i32,
                                         C.POINTER(i32), i32, vp, vp, C.POINTER(Result), C.POINTER(i32), vp]),
        "sip_dykstra_update": (i32, [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_double), vp, i64, i32, vp]),
        "sip_tiles_default": (i32, [C.POINTER(Tiles)]),
        "sip_plan_bytes": (i64, [C.POINTER(Grid), C.POINTER(Set), i32, C.POINTER(Opts), C.POINTER(Tiles)]),
        "sip_plan_create": (i32, [C.POINTER(vp), C.POINTER(Grid), C.POINTER(Set), i32, C.POINTER(Opts),
                                  C.POINTER(Tiles), vp, i64, vp]),
        "sip_plan_destroy": (i32, [vp]),
        "sip_plan_project": (i32, [vp, vp, vp, C.POINTER(Result), vp]),
        "sip_plan_start": (i32, [vp, vp, vp, vp]),
        "sip_plan_iterate": (i32, [vp, i32, vp]),
        "sip_plan_result": (i32, [vp, C.POINTER(Result), vp]),
        "sip_state_bytes": (i64, [vp]),
        "sip_state_export": (i32, [vp, vp, vp]),
        "sip_state_import": (i32, [vp, vp, vp]),
        "sip_project_noalloc": (i32, [C.POINTER(Grid), C.POINTER(Set), i32, C.POINTER(Opts), vp, vp,
                                      C.POINTER(Result), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols():
    return ["sip_strerror", "sip_opts_default", "sip_set_rows", "sip_validate", "sip_workspace_bytes",
            "sip_project", "sip_project_batched", "sip_batch_create", "sip_batch_destroy", "sip_batch_add",
            "sip_batch_run", "sip_batch_poll", "sip_batch_remove", "sip_batch_result", "sip_batch_field",
            "sip_batch_get_params", "sip_batch_set_params", "sip_batch_schedule", "sip_batch_set_tiles",
            "sip_batch_items", "sip_batch_reset", "sip_batch_time_kernel", "sip_stream_copy", "sip_level",
            "sip_restrict", "sip_project_multilevel", "sip_dykstra_update", "sip_tiles_default", "sip_plan_bytes",
            "sip_plan_create", "sip_plan_destroy", "sip_plan_project", "sip_plan_start", "sip_plan_iterate",
            "sip_plan_result", "sip_state_bytes", "sip_state_export", "sip_state_import", "sip_project_noalloc"]


def strerror(status: int) -> str:
    try:
        return lib().sip_strerror(int(status)).decode()
    except ImportError:
        return f"status {status}"


def check(status, what=""):
    if status != OK:
        raise SipError(status, what)


# ------------------------------------------------------------------ marshal

def make_grid(shape, h=None) -> Grid:
    g = Grid()
    g.ndim = len(shape)
    hh = tuple(h) if h is not None else (1.0,) * len(shape)
    for a in range(3):
        g.n[a] = int(shape[a]) if a < len(shape) else 0
        g.h[a] = float(hh[a]) if a < len(shape) else 0.0
    return g


def make_set(d: dict) -> Set:
    s = Set()
    s.kind = KINDS[d["kind"]]
    s.op = OPS[d["op"]]
    s.lo = float(d.get("lo", -math.inf))
    s.hi = float(d.get("hi", math.inf))
    s.tau = float(d.get("tau", 0.0))
    s.k = int(d.get("k", 0))
    s.line = LINES[d.get("line")]
    # per-row bound vectors: device tensors of the field type, one block of N
    # per operator component (the grid layout of the operator's rows)
    for key in ("lo_vec", "hi_vec"):
        t = d.get(key)
        if t is not None:
            if not t.is_contiguous():
                raise ValueError(f"{key}: contiguous device tensor expected")
            setattr(s, key, C.c_void_p(t.data_ptr()))
    return s


def make_sets(sets) -> C.Array:
    arr = (Set * max(1, len(sets)))()
    for i, d in enumerate(sets):
        arr[i] = make_set(d)
    return arr


def make_opts(field="f32", reduce="f64", **kw) -> Opts:
    """Options with the library defaults, the field type, the reduction type
    ("f64", or "f32" for the pure-FP32 ablation) and any sip_opts field."""
    o = Opts()
    check(lib().sip_opts_default(C.byref(o)), "sip_opts_default")
    o.field = F64 if field in ("f64", F64, "float64") else F32
    o.reduce = F32 if reduce in ("f32", F32, "float32") else F64
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, int(v) if isinstance(getattr(o, k), int) else float(v))
    return o


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dtype_of(opts: Opts):
    import torch
    return torch.float64 if opts.field == F64 else torch.float32


def _check_tensor(t, n, opts, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != _dtype_of(opts) or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{what}: need a contiguous {_dtype_of(opts)} tensor of {n} elements")


# ------------------------------------------------------------- entry points

def set_rows(shape, set_dict) -> int:
    g = make_grid(shape)
    s = make_set(set_dict)
    return int(lib().sip_set_rows(C.byref(g), C.byref(s)))


def validate(shape, sets, opts: Opts) -> int:
    g = make_grid(shape)
    arr = make_sets(sets)
    return int(lib().sip_validate(C.byref(g), arr, len(sets), C.byref(opts)))


def workspace_bytes(shape, sets, opts: Opts) -> int:
    g = make_grid(shape)
    arr = make_sets(sets)
    return int(lib().sip_workspace_bytes(C.byref(g), arr, len(sets), C.byref(opts)))


def project(m, sets, opts: Opts, x=None, h=None, stream=None):
    """x = P(m) onto the intersection of ``sets`` (blocking).  m is a device
    tensor shaped like the grid.  Returns (x, result dict)."""
    import torch
    shape = tuple(m.shape)
    n = m.numel()
    _check_tensor(m, n, opts, "m")
    if x is None:
        x = torch.empty_like(m)
    _check_tensor(x, n, opts, "x")
    g = make_grid(shape, h)
    arr = make_sets(sets)
    res = Result()
    st = lib().sip_project(C.byref(g), arr, len(sets), C.byref(opts), C.c_void_p(m.data_ptr()),
                           C.c_void_p(x.data_ptr()), C.byref(res), _stream_ptr(stream))
    check(st, "sip_project")
    return x, res.as_dict()


def project_noalloc(m, sets, opts: Opts, x=None, h=None, stream=None):
    """sip_project_noalloc: the projection of project() with every device
    buffer taken from the library's fixed array (blocking).  Raises
    SipError with ETOOLARGE when the instance does not fit it."""
    import torch
    shape = tuple(m.shape)
    n = m.numel()
    _check_tensor(m, n, opts, "m")
    if x is None:
        x = torch.empty_like(m)
    _check_tensor(x, n, opts, "x")
    g = make_grid(shape, h)
    arr = make_sets(sets)
    res = Result()
    st = lib().sip_project_noalloc(C.byref(g), arr, len(sets), C.byref(opts), C.c_void_p(m.data_ptr()),
                                   C.c_void_p(x.data_ptr()), C.byref(res), _stream_ptr(stream))
    check(st, "sip_project_noalloc")
    return x, res.as_dict()


def make_tiles(tiles=None) -> Tiles:
    """Tiles from a (pt_points, pt_max_items, thr_points, thr_max_items[,
    pt_threads[, cg_form]]) tuple; None: the library defaults."""
    t = Tiles()
    check(lib().sip_tiles_default(C.byref(t)), "sip_tiles_default")
    if tiles is not None:
        names = ["pt_points", "pt_max_items", "thr_points", "thr_max_items", "pt_threads", "cg_form"]
        for k, v in zip(names, tiles):
            setattr(t, k, int(v))
    return t


def plan_bytes(shape, sets, opts: Opts, tiles=None, h=None) -> int:
    g = make_grid(shape, h)
    arr = make_sets(sets)
    t = make_tiles(tiles)
    return int(lib().sip_plan_bytes(C.byref(g), arr, len(sets), C.byref(opts), C.byref(t)))


class Plan:
    """A plan for one grid and set list (sip_plan_*): precomputed once,
    reused for many models m.  workspace: optional device tensor (uint8) of at
    least plan_bytes() from which the plan takes all its device memory."""

    def __init__(self, shape, sets, opts: Opts, tiles=None, workspace=None, h=None, stream=None):
        self.opts = opts
        self.shape = tuple(shape)
        self.sets = list(sets)
        g = make_grid(self.shape, h)
        arr = make_sets(self.sets)
        t = make_tiles(tiles)
        hnd = C.c_void_p()
        ws_ptr = C.c_void_p(workspace.data_ptr()) if workspace is not None else None
        ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
        self.workspace = workspace
        check(lib().sip_plan_create(C.byref(hnd), C.byref(g), arr, len(self.sets), C.byref(opts), C.byref(t),
                                    ws_ptr, int(ws_bytes), _stream_ptr(stream)), "sip_plan_create")
        self.h = hnd
        self.x = None

    def close(self):
        if self.h:
            lib().sip_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _tensors(self, m, x):
        import torch
        n = m.numel()
        _check_tensor(m, n, self.opts, "m")
        if x is None:
            x = torch.empty_like(m)
        _check_tensor(x, n, self.opts, "x")
        return x

    def project(self, m, x=None, stream=None):
        x = self._tensors(m, x)
        res = Result()
        st = lib().sip_plan_project(self.h, C.c_void_p(m.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(res),
                                    _stream_ptr(stream))
        check(st, "sip_plan_project")
        self.x = x
        return x, res.as_dict()

    def start(self, m, x=None, stream=None):
        x = self._tensors(m, x)
        check(lib().sip_plan_start(self.h, C.c_void_p(m.data_ptr()), C.c_void_p(x.data_ptr()),
                                   _stream_ptr(stream)), "sip_plan_start")
        self.x = x
        return x

    def iterate(self, iters, stream=None):
        check(lib().sip_plan_iterate(self.h, int(iters), _stream_ptr(stream)), "sip_plan_iterate")

    def result(self, stream=None):
        r = Result()
        check(lib().sip_plan_result(self.h, C.byref(r), _stream_ptr(stream)), "sip_plan_result")
        return r.as_dict()

    def state_bytes(self) -> int:
        return int(lib().sip_state_bytes(self.h))

    def export_state(self, stream=None):
        """The plan's whole state as a new device tensor (uint8)."""
        import torch
        out = torch.empty(self.state_bytes(), dtype=torch.uint8, device="cuda")
        check(lib().sip_state_export(self.h, C.c_void_p(out.data_ptr()), _stream_ptr(stream)), "sip_state_export")
        return out

    def import_state(self, blob, stream=None):
        check(lib().sip_state_import(self.h, C.c_void_p(blob.data_ptr()), _stream_ptr(stream)), "sip_state_import")


def level(shape, sets, lev, h=None):
    """(shape, set dicts) of multilevel level ``lev`` (0 = the given grid)."""
    g = make_grid(shape, h)
    arr = make_sets(sets)
    go = Grid()
    out = (Set * max(1, len(sets)))()
    check(lib().sip_level(C.byref(g), arr, len(sets), int(lev), C.byref(go), out), "sip_level")
    shp = tuple(int(go.n[a]) for a in range(go.ndim))
    inv_k = {v: k for k, v in KINDS.items()}
    inv_o = {v: k for k, v in OPS.items()}
    res = []
    for i, d in enumerate(sets):
        e = dict(d)
        e.update(kind=inv_k[out[i].kind], op=inv_o[out[i].op])
        if e["kind"] in ("bounds", "annulus"):
            e.update(lo=out[i].lo, hi=out[i].hi)
        elif e["kind"] in ("l1", "l2"):
            e["tau"] = out[i].tau
        else:
            e["k"] = int(out[i].k)
        res.append(e)
    return shp, res


def restrict(m, stream=None):
    """The next level's coarse model of device tensor m (new tensor)."""
    import torch
    shape = tuple(m.shape)
    shp, _ = level(shape, [], 1)
    dt = F64 if m.dtype == torch.float64 else F32
    if m.dtype not in (torch.float32, torch.float64) or not m.is_contiguous():
        raise ValueError("m: contiguous float32/float64 device tensor expected")
    out = torch.empty(shp, dtype=m.dtype, device=m.device)
    g = make_grid(shape)
    check(lib().sip_restrict(C.byref(g), dt, C.c_void_p(m.data_ptr()), C.c_void_p(out.data_ptr()),
                             _stream_ptr(stream)), "sip_restrict")
    return out


def project_multilevel(m, sets, opts: Opts, nlevels, level_iters, carry_params=True, x=None, h=None,
                       stream=None):
    """Multilevel projection (blocking).  level_iters[l] caps level l (0 =
    the grid of m); carry_params: start each level from the coarser level's
    final (rho, gamma) instead of (rho0, gamma0).  Returns (x, result dict of
    level 0, iterations run per level)."""
    import torch
    shape = tuple(m.shape)
    n = m.numel()
    _check_tensor(m, n, opts, "m")
    if x is None:
        x = torch.empty_like(m)
    _check_tensor(x, n, opts, "x")
    g = make_grid(shape, h)
    arr = make_sets(sets)
    its = (C.c_int32 * nlevels)(*[int(v) for v in level_iters])
    run = (C.c_int32 * nlevels)()
    res = Result()
    st = lib().sip_project_multilevel(C.byref(g), arr, len(sets), C.byref(opts), int(nlevels), its,
                                      1 if carry_params else 0, C.c_void_p(m.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(res), run,
                                      _stream_ptr(stream))
    check(st, "sip_project_multilevel")
    return x, res.as_dict(), list(run)


def project_batched(ms, sets_list, opts: Opts, xs=None, graph_iters=25, stream=None):
    """Independent projections of uneven sizes in one batch (blocking)."""
    import torch
    B = len(ms)
    if xs is None:
        xs = [torch.empty_like(m) for m in ms]
    grids = (Grid * B)()
    nsets = (C.c_int32 * B)()
    flat = []
    for b, (m, sets) in enumerate(zip(ms, sets_list)):
        _check_tensor(m, m.numel(), opts, "m")
        _check_tensor(xs[b], m.numel(), opts, "x")
        grids[b] = make_grid(tuple(m.shape))
        nsets[b] = len(sets)
        flat += list(sets)
    arr = make_sets(flat)
    mp = (C.c_void_p * B)(*[m.data_ptr() for m in ms])
    xp = (C.c_void_p * B)(*[x.data_ptr() for x in xs])
    res = (Result * B)()
    st = lib().sip_project_batched(B, grids, arr, nsets, C.byref(opts), mp, xp, res, int(graph_iters),
                                   _stream_ptr(stream))
    check(st, "sip_project_batched")
    return xs, [r.as_dict() for r in res]


class Batch:
    """A resident batch (served form and step-level control)."""

    def __init__(self, max_slots: int, arena_bytes: int, opts: Opts):
        self.opts = opts
        self.max_slots = int(max_slots)
        h = C.c_void_p()
        check(lib().sip_batch_create(C.byref(h), self.max_slots, int(arena_bytes), C.byref(opts)),
              "sip_batch_create")
        self.h = h
        self.nsets = {}
        self.keep = {}

    def close(self):
        if self.h:
            lib().sip_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, m, sets, x, stream=None, h=None) -> int:
        n = m.numel()
        _check_tensor(m, n, self.opts, "m")
        _check_tensor(x, n, self.opts, "x")
        g = make_grid(tuple(m.shape), h)
        arr = make_sets(sets)
        slot = C.c_int32(-1)
        st = lib().sip_batch_add(self.h, C.byref(g), arr, len(sets), C.c_void_p(m.data_ptr()),
                                 C.c_void_p(x.data_ptr()), C.byref(slot), _stream_ptr(stream))
        if st == EBUDGET:
            return -1
        check(st, "sip_batch_add")
        self.nsets[slot.value] = len(sets)
        self.keep[slot.value] = x
        return slot.value

    def run(self, iters: int, stream=None):
        check(lib().sip_batch_run(self.h, int(iters), _stream_ptr(stream)), "sip_batch_run")

    def poll(self, stream=None):
        done = (C.c_int32 * self.max_slots)()
        check(lib().sip_batch_poll(self.h, done, _stream_ptr(stream)), "sip_batch_poll")
        return list(done)

    def result(self, slot, stream=None):
        r = Result()
        check(lib().sip_batch_result(self.h, int(slot), C.byref(r), _stream_ptr(stream)), "sip_batch_result")
        return r.as_dict()

    def remove(self, slot, stream=None):
        r = Result()
        check(lib().sip_batch_remove(self.h, int(slot), C.byref(r), _stream_ptr(stream)), "sip_batch_remove")
        self.nsets.pop(slot, None)
        self.keep.pop(slot, None)
        return r.as_dict()

    def field(self, slot, which, set_index):
        """(device pointer, element count, component stride) of a state
        array of a slot."""
        p = C.c_void_p()
        n = C.c_int64()
        cs = C.c_int64()
        check(lib().sip_batch_field(self.h, int(slot), int(which), int(set_index), C.byref(p), C.byref(n),
                                    C.byref(cs)), "sip_batch_field")
        return p.value, n.value, cs.value

    def field_tensor(self, slot, which, set_index):
        """Copy a state array of a slot into a new device tensor."""
        import torch
        ptr, n, _ = self.field(slot, which, set_index)
        dt = _dtype_of(self.opts)
        out = torch.empty(n, dtype=dt, device="cuda")
        torch.cuda.synchronize()
        _memcpy_d2d(out.data_ptr(), ptr, n * out.element_size())
        return out

    def rows(self, slot, which, set_index, shape, op):
        """A slot's set array (FIELD_Y, FIELD_V, ...) copied to the host as
        the operator's row vector (float64)."""
        t = self.field_tensor(slot, which, set_index).double().cpu().numpy()
        return component_rows(shape, op, t, self.field(slot, which, set_index)[2])

    def load_field(self, slot, which, set_index, values):
        import torch
        ptr, n, _ = self.field(slot, which, set_index)
        src = values.to(device="cuda", dtype=_dtype_of(self.opts)).contiguous()
        assert src.numel() == n
        torch.cuda.synchronize()
        _memcpy_d2d(ptr, src.data_ptr(), n * src.element_size())

    def get_params(self, slot, stream=None):
        p = self.nsets[slot]
        rho = (C.c_double * (p + 1))()
        gam = (C.c_double * (p + 1))()
        k = C.c_int32()
        have = C.c_int32()
        check(lib().sip_batch_get_params(self.h, int(slot), rho, gam, C.byref(k), C.byref(have),
                                         _stream_ptr(stream)), "sip_batch_get_params")
        return np.array(rho[:]), np.array(gam[:]), k.value, bool(have.value)

    def set_params(self, slot, rho, gamma, k, have, stream=None):
        p = self.nsets[slot]
        r = (C.c_double * (p + 1))(*[float(v) for v in rho])
        g = (C.c_double * (p + 1))(*[float(v) for v in gamma])
        check(lib().sip_batch_set_params(self.h, int(slot), r, g, int(k), int(bool(have)), _stream_ptr(stream)),
              "sip_batch_set_params")

    def schedule(self, slot, max_n, stream=None):
        p1 = self.nsets[slot] + 1
        rho = (C.c_double * (max_n * p1))()
        gam = (C.c_double * (max_n * p1))()
        n = C.c_int32()
        check(lib().sip_batch_schedule(self.h, int(slot), rho, gam, int(max_n), C.byref(n), _stream_ptr(stream)),
              "sip_batch_schedule")
        cnt = n.value
        return (np.array(rho[:cnt * p1]).reshape(cnt, p1), np.array(gam[:cnt * p1]).reshape(cnt, p1))

    def set_tiles(self, pt_points=2048, pt_max_items=512, thr_points=2048, thr_max_items=512, pt_threads=512,
                  cg_form=0):
        check(lib().sip_batch_set_tiles(self.h, int(pt_points), int(pt_max_items), int(thr_points),
                                        int(thr_max_items), int(pt_threads), int(cg_form)), "sip_batch_set_tiles")

    def reset(self, slot, m, stream=None):
        _check_tensor(m, m.numel(), self.opts, "m")
        check(lib().sip_batch_reset(self.h, int(slot), C.c_void_p(m.data_ptr()), _stream_ptr(stream)),
              "sip_batch_reset")

    def time_kernel(self, kernel, reps=20, stream=None) -> float:
        """Mean duration (ms) of one launch of an iteration kernel (HIP events)."""
        ms = C.c_double()
        check(lib().sip_batch_time_kernel(self.h, int(kernel), int(reps), _stream_ptr(stream), C.byref(ms)),
              "sip_batch_time_kernel")
        return ms.value

    def items(self):
        a, b, c, d = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().sip_batch_items(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)), "sip_batch_items")
        return a.value, b.value, c.value, d.value


# components of each operator, by grid axis (None: the identity block)
_COMP_AXES = {
    2: {"I": (None,), "DZ": (0,), "DX": (1,), "GRAD": (0, 1), "LAT": (1,)},
    3: {"I": (None,), "DZ": (0,), "DY": (1,), "DX": (2,), "GRAD": (0, 1, 2), "LAT": (1, 2)},
}


def component_rows(shape, op, flat, stride=None):
    """A set array in the device layout (one block of `stride` elements per
    operator component, each the grid image with the last layer along the
    component's axis unused) as the operator's row vector (components
    stacked, rows in C order): host-side layout conversion only."""
    N = int(np.prod(shape))
    stride = N if stride is None else int(stride)
    parts = []
    for c, ax in enumerate(_COMP_AXES[len(shape)][op]):
        blk = np.asarray(flat[c * stride:c * stride + N]).reshape(shape)
        if ax is not None:
            sl = [slice(None)] * len(shape)
            sl[ax] = slice(0, shape[ax] - 1)
            blk = blk[tuple(sl)]
        parts.append(blk.ravel())
    return np.concatenate(parts)


def dykstra_update(ys, vs, weights, x, stream=None):
    """Parallel Dykstra steps 2-3 on the device: x = sum_i w_i y_i, then
    v_i = x + v_i - y_i (device tensors of one dtype and size)."""
    import torch
    p = len(ys)
    f = F64 if x.dtype == torch.float64 else F32
    for t in list(ys) + list(vs):
        if t.dtype != x.dtype or t.numel() != x.numel() or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("dykstra_update: contiguous device tensors of one dtype and size expected")
    yp = (C.c_void_p * p)(*[t.data_ptr() for t in ys])
    vp_ = (C.c_void_p * p)(*[t.data_ptr() for t in vs])
    w = (C.c_double * p)(*[float(v) for v in weights])
    check(lib().sip_dykstra_update(p, yp, vp_, w, C.c_void_p(x.data_ptr()), x.numel(), f, _stream_ptr(stream)),
          "sip_dykstra_update")


def stream_copy(dst, src, stream=None):
    """dst <- src with the library's plain copy kernel (bandwidth reference)."""
    nbytes = src.numel() * src.element_size()
    check(lib().sip_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes,
                                _stream_ptr(stream)), "sip_stream_copy")


_hip = None


def _memcpy_d2d(dst, src, nbytes):
    """Device-to-device copy between raw pointers (via the HIP runtime)."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    rc = _hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), C.c_size_t(nbytes), 3)
    if rc != 0:
        raise SipError(EHIP, f"hipMemcpy ({rc})")
