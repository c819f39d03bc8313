"""Independent references used to pin the oracle.  None of these repeats the
oracle's own code path: each solves the same mathematical problem by a
different method (bisection, brute force, pool-adjacent-violators, halfspace
Dykstra, a general QP solver, a DCT diagonalisation)."""
from __future__ import annotations

import itertools
import math

import numpy as np


def l1_bisection(w, tau, steps=200):
    """Projection onto the l1 ball by bisection on theta in
    sum max(|w| - theta, 0) = tau."""
    w = np.asarray(w, dtype=np.float64)
    a = np.abs(w)
    if a.sum() <= tau:
        return w.copy()
    lo, hi = 0.0, float(a.max())
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if np.maximum(a - mid, 0.0).sum() > tau:
            lo = mid
        else:
            hi = mid
    theta = 0.5 * (lo + hi)
    return np.sign(w) * np.maximum(a - theta, 0.0)


def l1_bruteforce(w, tau):
    """Projection onto the l1 ball for tiny n: try every support S, put
    theta = (sum_S |w| - tau)/|S|, keep candidates consistent with the KKT
    sign/threshold pattern and return the closest feasible one."""
    w = np.asarray(w, dtype=np.float64)
    a = np.abs(w)
    if a.sum() <= tau:
        return w.copy()
    best, best_d = None, math.inf
    n = w.size
    for size in range(1, n + 1):
        for S in itertools.combinations(range(n), size):
            S = list(S)
            theta = (a[S].sum() - tau) / size
            if theta < 0:
                continue
            y = np.zeros(n)
            y[S] = np.sign(w[S]) * (a[S] - theta)
            if np.any(a[S] - theta < -1e-15):
                continue
            if abs(np.abs(y).sum() - tau) > 1e-9:
                continue
            d = float(((y - w) ** 2).sum())
            if d < best_d - 1e-15:
                best, best_d = y, d
    return best


def card_bruteforce(w, k):
    """Best k-sparse approximation by enumerating every k-subset; among
    equally good subsets the lexicographically smallest index tuple."""
    w = np.asarray(w, dtype=np.float64)
    best, best_val = None, -1.0
    for S in itertools.combinations(range(w.size), k):
        val = float((w[list(S)] ** 2).sum())
        if val > best_val:
            best, best_val = S, val
    y = np.zeros_like(w)
    y[list(best)] = w[list(best)]
    return y, np.array(best)


def pava_nondecreasing(v):
    """Isotonic (nondecreasing) least-squares fit by pool-adjacent-violators."""
    blocks = []  # [sum, count]
    for val in np.asarray(v, dtype=np.float64):
        blocks.append([val, 1])
        while len(blocks) > 1 and blocks[-2][0] / blocks[-2][1] > blocks[-1][0] / blocks[-1][1]:
            s, c = blocks.pop()
            blocks[-1][0] += s
            blocks[-1][1] += c
    out = []
    for s, c in blocks:
        out += [s / c] * c
    return np.array(out)


def monotone_columns(m2d):
    """Projection of a 2D field onto {x : x[z+1, :] >= x[z, :]}: one isotonic
    regression per column."""
    return np.stack([pava_nondecreasing(m2d[:, j]) for j in range(m2d.shape[1])], axis=1)


def dykstra_halfspaces(m, H, b, iters=400000, tol=1e-14):
    """Parallel Dykstra (Appendix A listing) with every set a halfspace
    {x : H[j] x <= b[j]}, equal weights: x0 = m, v_j = x0; y_j = P_j(v_j),
    x = mean_j y_j, v_j = x + v_j - y_j."""
    H = np.asarray(H, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    hh = (H * H).sum(axis=1)
    x = np.asarray(m, dtype=np.float64).copy()
    V = np.tile(x, (H.shape[0], 1))
    for it in range(iters):
        e = (H * V).sum(axis=1) - b
        Y = V - (np.maximum(e, 0.0) / hh)[:, None] * H
        x_new = Y.mean(axis=0)
        V = x_new[None, :] + V - Y
        if it % 100 == 0 and np.linalg.norm(x_new - x) <= tol * max(1.0, np.linalg.norm(x_new)):
            return x_new
        x = x_new
    return x


def qp_projection(m, lin_ineq=(), l1_blocks=(), bounds=None):
    """min 1/2||x - m||^2 subject to G x <= g (each (G, g) in lin_ineq),
    ||A x||_1 <= tau (each (A, tau) in l1_blocks, lifted with -t <= A x <= t,
    sum t <= tau) and lo <= x <= hi, solved by SciPy's SLSQP."""
    from scipy.optimize import minimize
    m = np.asarray(m, dtype=np.float64)
    n = m.size
    l1_blocks = [(np.asarray(A, dtype=np.float64), float(t)) for A, t in l1_blocks]
    nt = sum(A.shape[0] for A, _ in l1_blocks)
    nv = n + nt
    rows, rhs = [], []
    for G, g in lin_ineq:
        G = np.asarray(G, dtype=np.float64)
        rows.append(np.hstack([G, np.zeros((G.shape[0], nt))]))
        rhs.append(np.asarray(g, dtype=np.float64))
    off = 0
    for A, tau in l1_blocks:
        r = A.shape[0]
        E = np.zeros((r, nt))
        E[:, off:off + r] = np.eye(r)
        rows.append(np.hstack([A, -E]))
        rhs.append(np.zeros(r))
        rows.append(np.hstack([-A, -E]))
        rhs.append(np.zeros(r))
        s = np.zeros((1, nv))
        s[0, n + off:n + off + r] = 1.0
        rows.append(s)
        rhs.append(np.array([tau]))
        off += r
    G = np.vstack(rows) if rows else np.zeros((0, nv))
    g = np.concatenate(rhs) if rhs else np.zeros(0)
    lo, hi = bounds if bounds is not None else (None, None)
    bnds = [(lo, hi)] * n + [(0.0, None)] * nt
    z0 = np.concatenate([m, np.zeros(nt)])
    res = minimize(lambda z: 0.5 * ((z[:n] - m) ** 2).sum(), z0,
                   jac=lambda z: np.concatenate([z[:n] - m, np.zeros(nt)]),
                   constraints=[{"type": "ineq", "fun": lambda z: g - G @ z, "jac": lambda z: -G}],
                   bounds=bnds, method="SLSQP", options={"ftol": 1e-16, "maxiter": 5000})
    return res.x[:n]


def neumann_solve_dct(rhs_grid, c0, c_axes):
    """Solve (c0 I + sum_a c_a L_a) x = rhs on a grid, where L_a is the 1D
    Neumann Laplacian (diag 1,2,...,2,1, off-diagonals -1) along axis a, by the
    separable DCT-II that diagonalises it (eigenvalues 4 sin^2(pi j / (2n)))."""
    from scipy.fft import dctn, idctn
    shape = rhs_grid.shape
    lam = np.full(shape, float(c0))
    for a, c in enumerate(c_axes):
        n = shape[a]
        ev = 4.0 * np.sin(np.pi * np.arange(n) / (2.0 * n)) ** 2
        sh = [1] * len(shape)
        sh[a] = n
        lam = lam + c * ev.reshape(sh)
    return idctn(dctn(rhs_grid, type=2, norm="ortho") / lam, type=2, norm="ortho")
