"""Pins of the oracle's step balance and residual norms (step control of the primal-dual
method, Sec. 4; residual balancing of the adaptive variant it cites). CPU only.

* the balance c multiplies every dual step and divides every primal step, so the
  products sigma * tau (and the convergence condition) do not change;
* it is a change of metric only: for c = 1/4 and c = 4 the iteration still converges to
  the box-ROF optimum of the unlifted L = 2 problem (Prop. 3), found by an independent
  direct solver;
* the residual norms equal the textbook formulas r_p = T^-1 dx - K^T dy,
  r_d = Sigma^-1 dy - K dx with K written out densely from the Lagrangian of Sec. 4 on a
  2 x 3 image with 3 labels;
* at a saddle point both residuals vanish.
"""
import numpy as np
import pytest

import workloads as W
from tests import checkers as ck


def test_balance_scales_steps_and_keeps_products(orc):
    wl = W.truncated_quadratic(L=6, H=5, W=7, seed=3)
    s1 = orc.Problem(wl).steps()
    for c in (0.125, 3.0):
        sc = orc.Problem(wl, step_balance=c).steps()
        sp1, svz1, sq1, tu1, ts1 = s1
        spc, svzc, sqc, tuc, tsc = sc
        assert np.isclose(spc, c * sp1, rtol=1e-15) and np.isclose(sqc, c * sq1, rtol=1e-15)
        np.testing.assert_allclose(svzc, c * svz1, rtol=1e-15)
        np.testing.assert_allclose(tuc, tu1 / c, rtol=1e-15)
        np.testing.assert_allclose(tsc, ts1 / c, rtol=1e-15)


@pytest.mark.parametrize("c", [0.25, 4.0])
def test_balanced_iteration_reaches_box_rof_optimum(orc, c):
    wl = W.rof(H=24, W=24)
    P = orc.Problem(wl, step_balance=c)
    rep = None
    for _ in range(1000):
        P.run(100)
        rep = P.monitor()
        if rep["rel_gap"] <= 1e-6:
            break
    assert rep["rel_gap"] <= 1e-6          # c = 1/4: about 50k iterations, c = 4: about 3k
    _, Pf, Df = ck.fgp_box_rof(wl.f, wl.lam)
    assert rep["best_dual"] - 1e-8 <= Pf and Df <= rep["best_primal"] + 1e-8


def _dense_K(H, Wd, gam):
    """K of the Lagrangian <u,v> - sum q + <p, grad u> + sum_i s_i (z_i - h_i q +
    h_i <1_{i-1}, v> - gamma_i v_i) as a matrix from x = (u[k,N], s[k,N]) to
    y = (v[k,N], z[k,N], px[k,N], py[k,N], q[N])."""
    k = len(gam) - 1
    h = np.diff(gam)
    N = H * Wd
    nx, ny = 2 * k * N, 4 * k * N + N
    K = np.zeros((ny, nx))
    U = lambda i, x: i * N + x                     # noqa: E731
    Sx = lambda i, x: k * N + i * N + x            # noqa: E731
    V = lambda i, x: i * N + x                     # noqa: E731
    Z = lambda i, x: k * N + i * N + x             # noqa: E731
    PX = lambda i, x: 2 * k * N + i * N + x        # noqa: E731
    PY = lambda i, x: 3 * k * N + i * N + x        # noqa: E731
    Q = lambda x: 4 * k * N + x                    # noqa: E731
    for i in range(k):
        for r in range(H):
            for cc in range(Wd):
                x = r * Wd + cc
                K[V(i, x), U(i, x)] = 1.0                       # <u, v>
                K[V(i, x), Sx(i, x)] = -gam[i]                  # -gamma_i s_i v_i
                for j in range(i + 1, k):                       # h_j s_j <1_{j-1}, v>
                    K[V(i, x), Sx(j, x)] = h[j]
                K[Z(i, x), Sx(i, x)] = 1.0                      # s_i z_i
                K[Q(x), Sx(i, x)] = -h[i]                       # -h_i s_i q
                if cc < Wd - 1:                                 # <p, grad u>
                    K[PX(i, x), U(i, x + 1)] += 1.0
                    K[PX(i, x), U(i, x)] -= 1.0
                if r < H - 1:
                    K[PY(i, x), U(i, x + Wd)] += 1.0
                    K[PY(i, x), U(i, x)] -= 1.0
    return K


def test_residual_norms_match_dense_formula(orc):
    rng = np.random.default_rng(4)
    H, Wd = 2, 3
    gam = np.array([0.0, 0.35, 1.0])
    wl = W.Workload("t", H, Wd, gam, W.TRUNC_QUAD, 0.3, f=rng.uniform(0, 1, (H, Wd)).astype(np.float32),
                    a=2.0, nu=0.025)
    P = orc.Problem(wl, step_balance=0.5)
    sp, svz, sq, tu, ts = P.steps()
    k, N = 2, H * Wd
    names = ("u", "u_prev", "s", "s_prev", "v", "z", "px", "py", "qd")
    a = {n: rng.normal(size=(H, Wd) if n == "qd" else (k, H, Wd)) for n in names}
    b = {n: rng.normal(size=(H, Wd) if n == "qd" else (k, H, Wd)) for n in names}
    rp, rd = P.residual_norms(a, b)
    K = _dense_K(H, Wd, gam)
    dx = np.concatenate([(a["u"] - b["u"]).ravel(), (a["s"] - b["s"]).ravel()])
    dy = np.concatenate([(a[n] - b[n]).ravel() for n in ("v", "z", "px", "py", "qd")])
    Tinv = np.concatenate([np.tile(1.0 / tu, k), np.repeat(1.0 / ts, N)])
    Sinv = np.concatenate([np.repeat(1.0 / svz, N), np.repeat(1.0 / svz, N),
                           np.full(2 * k * N, 1.0 / sp), np.full(N, 1.0 / sq)])
    ref_p = np.abs(Tinv * dx - K.T @ dy).sum()
    ref_d = np.abs(Sinv * dy - K @ dx).sum()
    assert np.isclose(rp, ref_p, rtol=1e-12) and np.isclose(rd, ref_d, rtol=1e-12)


def test_residuals_vanish_at_saddle_point(orc):
    wl = W.rof(H=16, W=16)
    P = orc.Problem(wl)
    P.run(1)
    first = P.residual_norms(P.get_state(), (P.run(1), P.get_state())[1])
    for _ in range(200):
        P.run(100)
        if P.monitor()["rel_gap"] <= 1e-10:
            break
    a = P.get_state()
    P.run(1)
    last = P.residual_norms(a, P.get_state())
    assert last[0] <= 1e-6 * first[0] and last[1] <= 1e-6 * first[1], (first, last)
