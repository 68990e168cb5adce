"""Pins of the oracle's periodic quadratic data term (phase unwrapping, Sec. 5.5): the
squared distance on a circle of circumference nu, approximated on every interval by the
quadratic branch whose centre lies nearest the interval's midpoint. CPU only.

* the branch chosen per interval: its centre differs from f by a whole number of periods
  and is the nearest such centre to the midpoint;
* lambda = 0: the relaxed optimum is the sum over pixels of the smallest value the pieces
  take (each piece is convex, so its envelope keeps its minimum), in closed form;
* the relaxed optimum lower-bounds the exact minimum of the piecewise energy over a fine
  label grid on a chain (dynamic programming);
* the nonconvex energy uses the true circular distance.
"""
import numpy as np
import pytest

import workloads as W
from tests import checkers as ck
from tests.test_oracle_solver import _run_to


def _centres(orc, P, wl):
    """Branch centres of every (pixel, interval), in original label units."""
    gam, _, shift, scale = P.normalized()
    cen = np.empty((wl.k, wl.H * wl.W))
    for x in range(wl.H * wl.W):
        for i in range(wl.k):
            kind, acd, _, _ = P.piece(x, i)
            assert kind == orc.PIECE_QUAD
            cen[i, x] = shift + scale * acd[1]
    return cen


def test_branch_is_nearest_shift_of_f(orc):
    wl = W.phase_unwrapping(H=6, W=7, L=8)
    P = orc.Problem(wl)
    cen = _centres(orc, P, wl)
    f = wl.f.reshape(-1).astype(np.float64)
    per = wl.nu
    mid = 0.5 * (wl.gamma[:-1] + wl.gamma[1:])
    m = (cen - f[None]) / per
    assert np.allclose(m, np.round(m), atol=1e-9)
    # nearest: no other shift is closer to the midpoint (ties within float rounding)
    d = np.abs(cen - mid[:, None])
    assert np.all(d <= per / 2 + 1e-5)
    # on Gamma = [0, 4 pi] with f in [0, 2 pi) the branches are m = -1 .. 2
    assert set(np.unique(np.round(m)).astype(int)) <= {-1, 0, 1, 2}


def test_lambda_zero_closed_form(orc):
    wl = W.phase_unwrapping(H=5, W=6, L=4, lam=0.0)
    wl.gamma = W.equispaced(4, 1.0, 2.0)    # a narrow range: many pixels have no zero
    P = orc.Problem(wl)
    cen = _centres(orc, P, wl)
    lo, hi = wl.gamma[:-1, None], wl.gamma[1:, None]
    dist = np.maximum(0.0, np.maximum(lo - cen, cen - hi))          # distance to the interval
    exact = (0.5 * wl.a * dist ** 2).min(axis=0).sum()
    rep, _ = _run_to(P, 1e-9, 40000)
    assert rep["best_dual"] <= exact + 1e-9 <= rep["best_primal"] + 2e-9
    # the dual bound reaches the closed form, the primal bound approaches it
    assert exact - rep["best_dual"] <= 1e-9 * exact
    assert rep["best_primal"] - exact <= 2e-6 * exact


def test_relaxation_lower_bounds_chain_minimum(orc):
    rng = np.random.default_rng(17)
    n, L = 10, 6
    gamma = W.equispaced(L, 0.0, 4 * np.pi)
    f = rng.uniform(0, 2 * np.pi, size=(1, n)).astype(np.float32)
    wl = W.Workload("ph1", 1, n, gamma, W.PERIODIC_QUAD, 0.3, f=f, a=2.0, nu=2 * np.pi)
    P = orc.Problem(wl)
    cen = _centres(orc, P, wl)
    rep, hist = _run_to(P, 1e-7, 40000)
    grid = np.unique(np.concatenate([np.linspace(0, 4 * np.pi, 1601), gamma]))
    # the piecewise energy: on interval i the branch centred at cen[i]; at a label the
    # smaller of its two pieces
    cost = np.full((n, grid.size), np.inf)
    for i in range(L - 1):
        inside = (grid >= gamma[i]) & (grid <= gamma[i + 1])
        val = 0.5 * wl.a * (grid[None, inside] - cen[i][:, None]) ** 2
        cost[:, inside] = np.minimum(cost[:, inside], val)
    dp = ck.dp_chain(cost, grid, wl.lam)
    for r in hist:
        assert r["dual"] <= dp + 1e-9
    assert rep["best_dual"] >= 0.5 * dp     # the bound is not vacuous


def test_nonconvex_energy_uses_circular_distance(orc):
    wl = W.phase_unwrapping(H=12, W=14, L=8)
    P = orc.Problem(wl)
    P.run(200)
    rep = P.monitor()
    _, u = P.read_u()
    f = wl.f.astype(np.float64)
    d = np.abs(np.mod(u - f + np.pi, 2 * np.pi) - np.pi)
    e = (0.5 * wl.a * d ** 2).sum() + wl.lam * ck.iso_tv(u)
    assert rep["e_nc"] == pytest.approx(e, rel=1e-12)


def test_period_must_be_positive(orc):
    wl = W.phase_unwrapping(H=16, W=16)
    wl.nu = 0.0
    with pytest.raises(ValueError, match="nu"):
        orc.Problem(wl)
