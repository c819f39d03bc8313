"""Seeded synthetic workloads for projections onto intersections of sets.

This module only draws inputs: model fields m and set lists in plain-dict
form.  It holds none of the projection method's arithmetic, so both the HIP
path and the FP64 CPU oracle can take their inputs from here.

The paper's own test models (a 341-row geological section, aerial photos)
are not available; the fields below stand in for them with the paper's
shapes and set lists (Sec. "Parallel Dykstra versus PARSDMM", Sec. "Timings
for 2D and 3D projections").  Every array is generated in float64.  Callers
that run in float32 round it once and hand the same rounded values to both
paths; set parameters that depend on m (tau) are then derived from the
rounded field through :func:`finalize`.

A set is a dict ``{"kind", "op", "lo", "hi", "tau", "k"}`` with
kind in {"bounds", "l1", "card"} and op in {"I", "DZ", "DY", "DX", "GRAD",
"LAT"}.  Sets whose parameter is relative to m carry ``tau_frac`` (l1) or
``k_frac`` (card) until :func:`finalize` turns them into absolute values.
Axis 0 is z (vertical, slowest), the last axis is x (contiguous).
"""
from __future__ import annotations

import math

import numpy as np

_OP_AXES = {
    2: {"DZ": (0,), "DX": (1,), "GRAD": (0, 1), "LAT": (1,), "I": ()},
    3: {"DZ": (0,), "DY": (1,), "DX": (2,), "GRAD": (0, 1, 2), "LAT": (1, 2), "I": ()},
}


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def grf(shape, corr_len: float, rng: np.random.Generator) -> np.ndarray:
    """Smooth Gaussian random field: white N(0,1) noise convolved periodically
    with a Gaussian kernel of standard deviation ``corr_len`` cells (applied as
    a multiplication in the FFT domain), then shifted and scaled to zero mean
    and unit standard deviation."""
    white = rng.standard_normal(shape)
    freqs = np.meshgrid(*[np.fft.fftfreq(n) for n in shape], indexing="ij")
    f2 = sum(f * f for f in freqs)
    filt = np.exp(-2.0 * math.pi ** 2 * corr_len ** 2 * f2)
    field = np.real(np.fft.ifftn(np.fft.fftn(white) * filt))
    field -= field.mean()
    sd = field.std()
    return field / sd if sd > 0 else field


def layered(shape, rng: np.random.Generator, n_layers: int = 8, min_rows: int = 8,
            lo: float = 1.5, hi: float = 4.5, noise_sd: float = 0.2) -> np.ndarray:
    """Flat layers stacked along z with random thicknesses (each at least
    ``min_rows`` rows when the grid allows it), one value per layer drawn
    uniformly from [lo, hi] in random (unsorted) order, plus N(0, noise_sd^2)."""
    nz = shape[0]
    n_layers = max(1, min(n_layers, nz // max(min_rows, 1)))
    spare = nz - n_layers * min_rows
    if spare < 0:
        min_rows, spare = 1, nz - n_layers
    cuts = rng.uniform(size=n_layers)
    extra = np.floor(cuts / cuts.sum() * spare).astype(np.int64)
    extra[-1] += spare - extra.sum()
    thick = extra + min_rows
    values = rng.uniform(lo, hi, size=n_layers)
    prof = np.repeat(values, thick)
    field = np.broadcast_to(prof.reshape((nz,) + (1,) * (len(shape) - 1)), shape).copy()
    return field + rng.normal(0.0, noise_sd, size=shape)


def _abs_diff_sum(m: np.ndarray, axes) -> float:
    """Sum of absolute forward differences of m along the given grid axes
    (unit spacing): the set parameter recipes quote tau relative to it."""
    return float(sum(np.abs(np.diff(m, axis=a)).sum() for a in axes))


def rows_of(shape, op: str) -> int:
    """Number of rows of the operator ``op`` on ``shape`` (unit-stride grid)."""
    axes = _OP_AXES[len(shape)][op]
    if op == "I":
        return int(np.prod(shape))
    total = 0
    for a in axes:
        s = list(shape)
        s[a] -= 1
        total += int(np.prod(s))
    return total


def finalize(m: np.ndarray, sets):
    """Turn relative set parameters into absolute ones, measured on ``m``
    exactly as it will be handed to the solvers (after any rounding)."""
    m = np.asarray(m, dtype=np.float64)
    out = []
    for s in sets:
        s = dict(s)
        if "tau_frac" in s:
            s["tau"] = float(s.pop("tau_frac") * _abs_diff_sum(m, _OP_AXES[m.ndim][s["op"]])
                             if s["op"] != "I" else s.pop("tau_frac") * float(np.abs(m).sum()))
        if "k_frac" in s:
            s["k"] = max(1, int(math.floor(s.pop("k_frac") * rows_of(m.shape, s["op"]))))
        s.setdefault("lo", -math.inf)
        s.setdefault("hi", math.inf)
        s.setdefault("tau", 0.0)
        s.setdefault("k", 0)
        out.append(s)
    return out


def bounds(op, lo, hi):
    return {"kind": "bounds", "op": op, "lo": float(lo), "hi": float(hi)}


def l1(op, tau_frac):
    return {"kind": "l1", "op": op, "tau_frac": float(tau_frac)}


def card(op, k_frac):
    return {"kind": "card", "op": op, "k_frac": float(k_frac)}


# --------------------------------------------------------------------------
# Named workloads.  Each returns (m float64, sets with relative parameters,
# field dtype name, iterations).  Call finalize() after rounding m.
# --------------------------------------------------------------------------

def smooth2d_box_tv(n=(64, 64), seed=1001):
    """64x64 smooth field + N(0, 0.1^2) noise; box [-1, 1] and an anisotropic
    TV ball at half the field's own TV; 200 iterations x 10 CG steps; float64."""
    rng = rng_for(seed)
    m = grf(n, 8.0, rng) + rng.normal(0.0, 0.1, size=n)
    sets = [bounds("I", -1.0, 1.0), l1("GRAD", 0.5)]
    return m, sets, "f64", 200


def layered2d_four_sets(n=(341, 1361), seed=1002):
    """341x1361 layered section; box [1.5, 4.5], vertical monotonicity
    D_z x >= 0, l1 ball on D_x at 0.3 of ||D_x m||_1 and cardinality of D_x
    at 5% of its rows; 300 iterations x 10 CG steps; float32."""
    rng = rng_for(seed)
    m = layered(n, rng)
    sets = [bounds("I", 1.5, 4.5), bounds("DZ", 0.0, math.inf), l1("DX", 0.3), card("DX", 0.05)]
    return m, sets, "f32", 300


def layered2d_line_sets(n=(341, 1361), seed=1004):
    """The layered section under the set list of the paper's full-waveform
    example without its rank set: box [1.5, 4.5], at most n_x nonzeros of
    D_z and n_z of D_x over the whole model, at most two nonzeros of D_x in
    every row and of D_z in every column; 300 iterations x 10 CG steps;
    float32."""
    rng = rng_for(seed)
    m = layered(n, rng)
    nz, nx = n
    sets = [bounds("I", 1.5, 4.5), {"kind": "card", "op": "DZ", "k": nx}, {"kind": "card", "op": "DX", "k": nz},
            {"kind": "card", "op": "DX", "k": 2, "line": "x"}, {"kind": "card", "op": "DZ", "k": 2, "line": "z"}]
    return m, sets, "f32", 300


def smooth3d_box_tv_lat(n=(200, 200, 100), seed=1003):
    """200x200x100 smooth field; box [-1, 1], TV ball at 0.4 of the field's
    TV, lateral slope bounds |D_x x|, |D_y x| <= 0.05; 200 iterations x 10 CG
    steps; float32 fields with float64 reductions."""
    rng = rng_for(seed)
    m = grf(n, 8.0, rng)
    sets = [bounds("I", -1.0, 1.0), l1("GRAD", 0.4), bounds("LAT", -0.05, 0.05)]
    return m, sets, "f32", 200


def _random_sets(m, rng, pool_2d=True):
    choices = ("box", "tv", "l1dz", "carddx")
    p = int(rng.integers(2, 6))
    sets = []
    for _ in range(p):
        c = choices[int(rng.integers(0, len(choices)))]
        if c == "box":
            sets.append(bounds("I", float(np.quantile(m, 0.05)), float(np.quantile(m, 0.95))))
        elif c == "tv":
            sets.append(l1("GRAD", float(rng.uniform(0.3, 0.7))))
        elif c == "l1dz":
            sets.append(l1("DZ", float(rng.uniform(0.3, 0.7))))
        else:
            sets.append(card("DX", float(rng.uniform(0.02, 0.10))))
    return sets


def random_instance(seed: int, max_side: int = 512, min_side: int = 32):
    """One instance of the uneven mix: 2D sides uniform on {32..512}, half
    smooth fields with correlation length U[4, 16], half layered sections,
    2..5 sets drawn with replacement from {box at the 5/95% quantiles, TV
    ball, l1 ball on D_z, cardinality of D_x}."""
    rng = rng_for(seed)
    shape = (int(rng.integers(min_side, max_side + 1)), int(rng.integers(min_side, max_side + 1)))
    if rng.uniform() < 0.5:
        m = grf(shape, float(rng.uniform(4.0, 16.0)), rng)
    else:
        m = layered(shape, rng)
    return m, _random_sets(m, rng)


def batched_instances(count=256, seed0=2000, max_side=512, min_side=32):
    """The uneven batch: instance j uses seed seed0 + j."""
    return [random_instance(seed0 + j, max_side, min_side) for j in range(count)]


def served_request(j: int, seed0=3000, frac3d=0.05, max2d=1024, min2d=64, side3d=(64, 160)):
    """Request j of the served mix: 2D sides log-uniform on [64, 1024] per
    axis, 3D sides uniform on {64..160} per axis with probability ``frac3d``;
    fields and sets as in the uneven batch."""
    rng = rng_for(seed0 + j)
    if rng.uniform() < frac3d:
        shape = tuple(int(rng.integers(side3d[0], side3d[1] + 1)) for _ in range(3))
    else:
        shape = tuple(int(round(math.exp(rng.uniform(math.log(min2d), math.log(max2d))))) for _ in range(2))
    if rng.uniform() < 0.5:
        m = grf(shape, float(rng.uniform(4.0, 16.0)), rng)
    else:
        m = layered(shape, rng)
    return m, _random_sets(m, rng)


def poisson_arrivals(n: int, rate: float, seed: int = 3999) -> np.ndarray:
    """Arrival times (seconds) of n requests of a Poisson process."""
    rng = rng_for(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def rounded(m: np.ndarray, dtype: str) -> np.ndarray:
    """Round a float64 field once to the field type ("f32" or "f64") and
    return it as float64 holding exactly the rounded values."""
    if dtype == "f32":
        return m.astype(np.float32).astype(np.float64)
    return np.asarray(m, dtype=np.float64).copy()
