"""Independent NumPy solvers and brute-force routines that pin the oracle.

None of this code is shared with the oracle or with the HIP path. Each routine solves
a problem whose answer the paper fixes (or that a textbook method answers) by a
different algorithm than the lifted primal-dual iteration.
"""
from __future__ import annotations

import itertools

import numpy as np


# --------------------------------------------------------------------------- operators

def fd_grad(u: np.ndarray):
    """Forward differences, zero on the last row / column (np.diff based)."""
    gx = np.zeros_like(u)
    gy = np.zeros_like(u)
    gx[..., :, :-1] = np.diff(u, axis=-1)
    gy[..., :-1, :] = np.diff(u, axis=-2)
    return gx, gy


def fd_div(px: np.ndarray, py: np.ndarray):
    """Negative adjoint of fd_grad, built from the transpose of the difference matrix."""
    d = np.zeros_like(px)
    d[..., :, :-1] += px[..., :, :-1]
    d[..., :, 1:] -= px[..., :, :-1]
    d[..., :-1, :] += py[..., :-1, :]
    d[..., 1:, :] -= py[..., :-1, :]
    return d


def iso_tv(u: np.ndarray) -> float:
    gx, gy = fd_grad(u)
    return float(np.sqrt(gx * gx + gy * gy).sum())


def aniso_tv(u: np.ndarray) -> float:
    gx, gy = fd_grad(u)
    return float((np.abs(gx) + np.abs(gy)).sum())


# --------------------------------------------------------------------------- ROF (Prop. 3)

def fgp_box_rof(f: np.ndarray, lam: float, lo: float = 0.0, hi: float = 1.0,
                tol: float = 1e-11, max_iter: int = 400000, aniso: bool = False):
    """Fast gradient projection on the dual of box-constrained ROF (Beck & Teboulle
    2009):  min_{lo<=u<=hi} 1/2 |u - f|^2 + lam sum |grad u|, with the isotropic (l2) or
    the anisotropic (l1) norm of the gradient; the dual variable is then projected onto
    unit l2 discs or onto the unit l-inf box. Returns (u, primal, dual)."""
    f = f.astype(np.float64)
    px = np.zeros_like(f)
    py = np.zeros_like(f)
    rx, ry = px.copy(), py.copy()
    t = 1.0
    step = 1.0 / (8.0 * lam)

    def u_of(ax, ay):
        return np.clip(f + lam * fd_div(ax, ay), lo, hi)

    def bounds(ax, ay):
        u = u_of(ax, ay)
        primal = 0.5 * ((u - f) ** 2).sum() + lam * (aniso_tv(u) if aniso else iso_tv(u))
        dual = 0.5 * ((u - f) ** 2).sum() - lam * (fd_div(ax, ay) * u).sum()
        return u, primal, dual

    for it in range(max_iter):
        u = u_of(rx, ry)
        gx, gy = fd_grad(u)
        qx, qy = rx + step * gx, ry + step * gy
        if aniso:
            nx, ny = np.clip(qx, -1.0, 1.0), np.clip(qy, -1.0, 1.0)
        else:
            nrm = np.maximum(1.0, np.sqrt(qx * qx + qy * qy))
            nx, ny = qx / nrm, qy / nrm
        t2 = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        rx = nx + (t - 1.0) / t2 * (nx - px)
        ry = ny + (t - 1.0) / t2 * (ny - py)
        px, py, t = nx, ny, t2
        if it % 200 == 199:
            _, P, D = bounds(px, py)
            if P - D <= tol * max(abs(P), 1.0):
                break
    return bounds(px, py)


# --------------------------------------------------------------------------- Prop. 2

def iso_decreasing(y: np.ndarray) -> np.ndarray:
    """Least-squares non-increasing fit along axis 0 (min-max formula of isotonic
    regression), vectorised over the remaining axes."""
    k = y.shape[0]
    cs = np.concatenate([np.zeros((1,) + y.shape[1:]), np.cumsum(y, axis=0)], axis=0)
    out = np.empty_like(y)
    for i in range(k):
        # non-increasing fit: x_i = min_{a<=i} max_{b>=i} mean(y[a..b])
        best = None
        for a in range(i + 1):
            inner = None
            for b in range(i, k):
                m = (cs[b + 1] - cs[a]) / (b - a + 1)
                inner = m if inner is None else np.maximum(inner, m)
            best = inner if best is None else np.minimum(best, inner)
        out[i] = best
    return out


def proj_ordered_box(y: np.ndarray) -> np.ndarray:
    """Projection onto {1 >= u_1 >= ... >= u_k >= 0} along axis 0."""
    return np.clip(iso_decreasing(y), 0.0, 1.0)


def baseline_lifting(rho_at_labels: np.ndarray, gamma: np.ndarray, lam: float,
                     iters: int = 20000, tol: float = 1e-9):
    """Solve the piecewise-linear special case of Prop. 2 directly:
        min_{1>=u_1>=...>=u_k>=0} sum_x rho(x,gamma_1) + <u(x), r(x)> + lam sum_i h_i |grad u_i|
    with r_i = rho(gamma_{i+1}) - rho(gamma_i), by a plain primal-dual method with the
    ordered-box projection. Returns (primal, dual) certified bounds."""
    L, H, W = rho_at_labels.shape
    k = L - 1
    h = np.diff(gamma)
    r = np.diff(rho_at_labels, axis=0)
    base = rho_at_labels[0].sum()
    u = np.zeros((k, H, W))
    ub = u.copy()
    px = np.zeros_like(u)
    py = np.zeros_like(u)
    tau = sig = 0.99 / np.sqrt(8.0)
    rad = (lam * h)[:, None, None]

    def bounds(u, px, py):
        gx, gy = fd_grad(u)
        primal = base + (u * r).sum() + lam * (h[:, None, None] * np.sqrt(gx ** 2 + gy ** 2)).sum()
        g = r - fd_div(px, py)
        # min over the ordered box of a linear function is attained at a vertex 1_j
        cum = np.concatenate([np.zeros((1, H, W)), np.cumsum(g, axis=0)], axis=0)
        dual = base + cum.min(axis=0).sum()
        return primal, dual

    for it in range(iters):
        gx, gy = fd_grad(ub)
        qx, qy = px + sig * gx, py + sig * gy
        nrm = np.maximum(1.0, np.sqrt(qx * qx + qy * qy) / rad)
        px, py = qx / nrm, qy / nrm
        un = proj_ordered_box(u + tau * fd_div(px, py) - tau * r)
        ub = 2 * un - u
        u = un
        if it % 500 == 499:
            P, D = bounds(u, px, py)
            if P - D <= tol * max(abs(P), 1.0):
                break
    return bounds(u, px, py)


# --------------------------------------------------------------------------- brute force

def dp_chain(cost: np.ndarray, grid: np.ndarray, lam: float) -> float:
    """Exact minimum over u_c in ``grid`` of sum_c cost[c, g] + lam sum_c |u_{c+1} - u_c|
    for a 1-D chain (cost: [n, G])."""
    jump = lam * np.abs(grid[:, None] - grid[None, :])
    val = cost[0].copy()
    for c in range(1, cost.shape[0]):
        val = (val[:, None] + jump).min(axis=0) + cost[c]
    return float(val.min())


def lift(uval: np.ndarray, gamma: np.ndarray) -> np.ndarray:
    """Graph lifting 1_i^alpha of values u (Sec. 3): u_j = clip((u - gamma_j)/h_j, 0, 1)."""
    h = np.diff(gamma)
    return np.clip((uval[None] - gamma[:-1].reshape((-1,) + (1,) * uval.ndim))
                   / h.reshape((-1,) + (1,) * uval.ndim), 0.0, 1.0)


def brute_force_lifted(cost_fn, grid: np.ndarray, gamma: np.ndarray, H: int, W: int,
                       lam: float) -> float:
    """Minimum over all assignments u(x) in ``grid`` of the lifted energy of the graph
    lifting: sum_x cost_fn(x, u(x)) + lam sum_i h_i |grad (1^alpha(u))_i|_2."""
    h = np.diff(gamma)
    N = H * W
    G = len(grid)
    costs = np.array([[cost_fn(x, g) for g in grid] for x in range(N)])  # [N, G]
    best = np.inf
    combos = np.array(list(itertools.product(range(G), repeat=N)))      # [C, N]
    for chunk in np.array_split(combos, max(1, len(combos) // 200000)):
        vals = grid[chunk].reshape(-1, H, W)                            # [C, H, W]
        data = costs[np.arange(N)[None, :], chunk].sum(axis=1)
        lifted = np.clip((vals[:, None] - gamma[None, :-1, None, None]) / h[None, :, None, None],
                         0.0, 1.0)                                       # [C, k, H, W]
        gx, gy = fd_grad(lifted)
        tv = (h[None, :, None, None] * np.sqrt(gx ** 2 + gy ** 2)).sum(axis=(1, 2, 3))
        best = min(best, float((data + lam * tv).min()))
    return best


def brute_force_aniso(cost_fn, grid: np.ndarray, H: int, W: int, lam: float) -> float:
    """Minimum over all assignments u(x) in ``grid`` of the unlifted energy
    sum_x cost_fn(x, u(x)) + lam sum_x (|d_x u| + |d_y u|) (anisotropic TV)."""
    N = H * W
    G = len(grid)
    costs = np.array([[cost_fn(x, g) for g in grid] for x in range(N)])  # [N, G]
    best = np.inf
    combos = np.array(list(itertools.product(range(G), repeat=N)))      # [C, N]
    for chunk in np.array_split(combos, max(1, len(combos) // 200000)):
        vals = grid[chunk].reshape(-1, H, W)
        data = costs[np.arange(N)[None, :], chunk].sum(axis=1)
        gx, gy = fd_grad(vals)
        tv = (np.abs(gx) + np.abs(gy)).sum(axis=(1, 2))
        best = min(best, float((data + lam * tv).min()))
    return best


def simplex_bisection(x: np.ndarray, iters: int = 200) -> np.ndarray:
    """Projection onto the probability simplex by bisection on the threshold."""
    lo, hi = x.min() - 1.0, x.max()
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if np.maximum(x - mid, 0).sum() > 1.0:
            lo = mid
        else:
            hi = mid
    return np.maximum(x - 0.5 * (lo + hi), 0.0)
