"""Pins of the oracle's anisotropic total variation (Sec. 5.3, comparison with Zach and
Kohli: Props. 4 and 5 hold for any convex one-homogeneous norm of the gradient; for the
l1 norm the per-label dual set K is the l-inf box of half-width lambda h_i).

* the box projection: Moreau's identity against soft thresholding (the prox of the l1
  norm, whose conjugate is the box indicator), KKT conditions, idempotence;
* its adjoint against central finite differences;
* L = 2 is box-constrained anisotropic ROF (Prop. 3), and for convex data with L > 2 the
  relaxation is exact: with the l1 norm the lifted TV of a graph lifting equals the TV of
  the function, and the triangle inequality gives the reverse bound. Both are compared
  with an independent FGP solve of the unlifted problem;
* for a nonconvex data term the relaxed optimum lower-bounds the unlifted energy of
  every labelling (brute force over a grid on a 2x3 image), with no lifted-TV detour;
* the nonconvex energy reported by the monitor matches its definition;
* the reverse pass (one-step dot-product test, unrolled gradients against central
  differences).
CPU only."""
import copy

import numpy as np
import pytest

import workloads as W
from tests import checkers as ck
from tests.test_oracle_solver import _run_to, _tq_interp_cost

EPS = 1e-6


def _aniso(wl):
    wl.tv = 1
    return wl


def test_box_projection_moreau_kkt(orc):
    rng = np.random.default_rng(31)
    for _ in range(2000):
        r = rng.uniform(0.0, 2.0)
        a = rng.normal(0.0, 1.5, 2)
        p = np.array(orc.proj_box(a[0], a[1], r))
        # Moreau: a = prox_{r |.|_1}(a) + Proj_{|.|_inf <= r}(a)
        soft = np.sign(a) * np.maximum(np.abs(a) - r, 0.0)
        assert np.allclose(soft + p, a, rtol=0, atol=1e-15)
        # KKT: the residual a - p lies in the normal cone of the box at p
        res = a - p
        for j in range(2):
            if abs(a[j]) <= r:
                assert res[j] == 0.0
            else:
                assert abs(p[j]) == r and res[j] * p[j] > 0
        assert np.array_equal(np.array(orc.proj_box(p[0], p[1], r)), p)


def test_box_projection_adjoint_matches_finite_differences(orc):
    rng = np.random.default_rng(32)
    checked = 0
    for _ in range(500):
        r = rng.uniform(0.1, 2.0)
        a = rng.normal(0.0, 1.5, 2)
        if np.abs(np.abs(a) - r).min() < 1e-3:
            continue   # a face of the box: not differentiable there
        pb = rng.normal(size=2)
        ab = orc.proj_box_vjp(a[0], a[1], r, pb[0], pb[1])

        def F(x, y, rr):
            px, py = orc.proj_box(x, y, rr)
            return pb[0] * px + pb[1] * py

        fd = [(F(a[0] + EPS, a[1], r) - F(a[0] - EPS, a[1], r)) / (2 * EPS),
              (F(a[0], a[1] + EPS, r) - F(a[0], a[1] - EPS, r)) / (2 * EPS),
              (F(a[0], a[1], r + EPS) - F(a[0], a[1], r - EPS)) / (2 * EPS)]
        for got, want in zip(ab, fd):
            assert abs(got - want) <= 1e-8 * (1 + abs(want))
        checked += 1
    assert checked > 400


@pytest.mark.parametrize("L", [2, 5])
def test_convex_data_equals_direct_anisotropic_rof(orc, L):
    """Quadratic data on [0,1]: the lifted problem with the l1 norm has the optimum of
    min_{0<=u<=1} 1/2 |u - f|^2 + lambda TV_1(u), for L = 2 (Prop. 3) and for L = 5."""
    wl = _aniso(W.rof(H=20, W=22))
    wl.gamma = W.equispaced(L)
    P = orc.Problem(wl)
    # the primal bound of the lifted problem converges slowly for L > 2; its dual does not
    gap = 1e-8 if L == 2 else 2e-5
    rep, _ = _run_to(P, gap, 60000)
    u_fgp, Pf, Df = ck.fgp_box_rof(wl.f, wl.lam, aniso=True)
    assert Pf - Df <= 1e-9 * Pf
    assert rep["rel_gap"] < gap
    # the certified interval of the lifted problem contains the unlifted optimum, and its
    # lower end reaches it
    assert rep["best_dual"] - 1e-9 <= Pf and Df <= rep["best_primal"] + 1e-9
    assert Pf - rep["best_dual"] <= 1e-6 * Pf
    # and differs from the isotropic optimum by far more than both gaps
    _, Pi, _ = ck.fgp_box_rof(wl.f, wl.lam)
    assert abs(Pi - Pf) > 1e3 * (rep["best_gap"] + (Pf - Df))
    # strong convexity: the back-projected u is near the unique minimiser
    _, u = P.read_u()
    E_u = 0.5 * ((u - wl.f) ** 2).sum() + wl.lam * ck.aniso_tv(u)
    assert E_u >= Df - 1e-9
    assert np.sqrt(((u - u_fgp) ** 2).sum()) <= np.sqrt(2 * (E_u - Df)) + 1e-6
    assert rep["e_nc"] == pytest.approx(E_u, rel=1e-12)


def test_relaxation_lower_bounds_unlifted_bruteforce_2d(orc):
    """2x3 image, truncated quadratic: every dual value lower-bounds the unlifted energy
    (with TV_1) of every labelling on an 11-point grid."""
    rng = np.random.default_rng(14)
    H, Wd = 2, 3
    f = rng.uniform(0, 1, size=(H, Wd)).astype(np.float32)
    gamma = W.equispaced(3)
    wl = _aniso(W.Workload("b2", H, Wd, gamma, W.TRUNC_QUAD, 0.04, f=f, a=2.0, nu=0.025))
    P = orc.Problem(wl)
    rep, hist = _run_to(P, 1e-7, 40000)
    grid = np.linspace(0, 1, 11)
    ff = f.reshape(-1).astype(np.float64)
    bf = ck.brute_force_aniso(lambda x, g: _tq_interp_cost(ff[x], g, 2.0, 0.025, gamma),
                              grid, H, Wd, wl.lam)
    for r in hist:
        assert r["dual"] <= bf + 1e-9
    assert rep["rel_gap"] < 1e-7


def test_nonconvex_energy_matches_definition(orc):
    wl = _aniso(W.truncated_quadratic(L=6, H=12, W=14))
    P = orc.Problem(wl)
    P.run(300)
    rep = P.monitor()
    _, u = P.read_u()
    f = wl.f.astype(np.float64)
    e = np.minimum((u - f) ** 2, 0.025).sum() + wl.lam * ck.aniso_tv(u)
    assert rep["e_nc"] == pytest.approx(e, rel=1e-12)


def test_step_adjoint_dot_product(orc):
    rng = np.random.default_rng(22)
    wl = _aniso(W.truncated_quadratic(L=5, H=7, W=9, seed=3))
    wl.tau = wl.gamma.copy()
    wl.samples = rng.normal(0, 0.02, (5, 7, 9)).astype(np.float32)
    o = orc.Problem(wl)
    o.run(37)
    st = {n: v + rng.normal(0, 0.05, v.shape) for n, v in o.get_state().items()}
    adj = {n: rng.normal(size=v.shape) for n, v in st.items()}
    d = {n: rng.normal(size=v.shape) for n, v in st.items()}
    a_in, _, _, _ = o.step_vjp(st, adj)

    def F(sign):
        o.set_state({n: st[n] + sign * EPS * d[n] for n in st})
        o.run(1)
        s2 = o.get_state()
        return sum(float(np.sum(adj[n] * s2[n])) for n in adj)

    jvp = (F(1) - F(-1)) / (2 * EPS)
    vjp = sum(float(np.sum(a_in[n] * d[n])) for n in d)
    assert abs(jvp - vjp) <= 1e-7 * abs(jvp), (jvp, vjp)


def test_unrolled_gradients_match_finite_differences(orc):
    from tests.test_oracle_adjoint import _fd_f32, _loss, _tq_w, _with
    rng = np.random.default_rng(6)
    wl = _aniso(_tq_w(rng))
    K = 30
    g = rng.uniform(0, 1, (wl.H, wl.W))
    o = orc.Problem(wl)
    o.unrolled_forward(K)
    _, u = o.read_u()
    gf, gl, gw = o.unrolled_backward(2 * (u - g))
    lp = _loss(orc, _with(wl, lam=wl.lam + EPS), g, K)
    lm = _loss(orc, _with(wl, lam=wl.lam - EPS), g, K)
    fd = (lp - lm) / (2 * EPS)
    assert abs(fd - gl) <= 1e-5 * abs(fd) + 1e-9, (fd, gl)
    pick = np.random.default_rng(52)
    for field, grad in (("f", gf), ("samples", gw)):
        done = tries = 0
        while done < 16:
            tries += 1
            assert tries < 64, "too many kinks"
            idx = tuple(int(pick.integers(n)) for n in getattr(wl, field).shape)
            fd, kink = _fd_f32(orc, wl, g, K, field, idx)
            if kink:
                continue
            assert abs(fd - grad[idx]) <= 1e-5 * abs(fd) + 1e-9, (field, idx, fd, grad[idx])
            done += 1


def test_unknown_tv_kind_rejected(orc):
    wl = W.rof(H=16, W=16)
    wl.tv = 2
    with pytest.raises(ValueError, match="TV kind"):
        orc.Problem(wl)
    wl2 = copy.copy(wl)
    wl2.tv = 0
    orc.Problem(wl2)
