"""Pins of the oracle's whole iteration against results the paper fixes: Prop. 3 (L = 2
is the unlifted problem: box-constrained ROF), Prop. 2 (piecewise-linear pieces give the
baseline lifting), the relaxation lower-bounds the discrete minimum, lambda = 0 closed
form, monotone best gap, label ordering at convergence, invariance under label
normalisation. CPU only."""
import numpy as np
import pytest

import workloads as W
from tests import checkers as ck


def _run_to(P, gap, max_iters, every=100):
    hist = []
    rep = None
    while True:
        P.run(every)
        rep = P.monitor()
        hist.append(rep)
        if rep["rel_gap"] <= gap or rep["iters"] >= max_iters:
            return rep, hist


def test_rof_L2_matches_direct_solver(orc):
    """Prop. 3: for L = 2 the lifted problem is min_{u in Gamma} rho(u) + lambda TV(u),
    here box-constrained ROF, solved independently by FGP (Beck-Teboulle 2009)."""
    wl = W.rof(H=32, W=32)
    P = orc.Problem(wl)
    rep, _ = _run_to(P, 1e-7, 20000)
    u_fgp, Pf, Df = ck.fgp_box_rof(wl.f, wl.lam)
    assert Pf - Df <= 1e-9 * Pf
    # both certified intervals contain the same optimum
    assert rep["best_dual"] <= Pf + 1e-9
    assert Df <= rep["best_primal"] + 1e-9
    assert rep["best_dual"] - 1e-9 <= Pf <= rep["best_primal"] + 1e-9
    assert rep["rel_gap"] < 1e-6
    # 1-strong convexity of the data term: |u - u*|^2 <= 2 (E(u) - E*)
    _, u = P.read_u()
    E_u = 0.5 * ((u - wl.f) ** 2).sum() + wl.lam * ck.iso_tv(u)
    assert E_u >= Df - 1e-9
    assert np.sqrt(((u - u_fgp) ** 2).sum()) <= np.sqrt(2 * (E_u - Df)) + 1e-6
    assert np.abs(u - u_fgp).max() < 1e-3


def test_rof_config_2000_iterations_tracks_direct(orc):
    """The 64x64 ROF workload at its 2000 iterations."""
    wl = W.rof()
    P = orc.Problem(wl)
    P.run(wl.iters)
    rep = P.monitor()
    _, Pf, Df = ck.fgp_box_rof(wl.f, wl.lam, tol=1e-8)
    assert rep["best_dual"] <= Pf + 1e-9 and Df <= rep["best_primal"] + 1e-9
    assert rep["rel_gap"] < 1e-4


def test_lambda_zero_closed_form(orc):
    """lambda = 0: the relaxed optimum is sum_x min_{t in Gamma} rho(x,t) (the convex
    envelope keeps the minimum); for rho = a/2 (t-f)^2 that is a/2 dist(f, Gamma)^2."""
    rng = np.random.default_rng(11)
    f = rng.uniform(-0.5, 1.5, size=(6, 7)).astype(np.float32)
    wl = W.Workload("l0", 6, 7, W.equispaced(4), W.QUAD, 0.0, f=f, a=1.5)
    P = orc.Problem(wl)
    rep, _ = _run_to(P, 1e-9, 30000)
    exact = 0.75 * ((f.astype(np.float64) - np.clip(f, 0, 1)) ** 2).sum()
    assert rep["best_dual"] <= exact + 1e-9
    assert rep["best_primal"] >= exact - 1e-9
    assert rep["rel_gap"] < 1e-4


def _tq_piece_min(f, g0, g1, a, nu, n_sub=16):
    """Minimum over [g0, g1] of the convex piece the relaxation puts on that interval for
    rho = min(a/2 (t-f)^2, nu) (Sec. 5.2): the clamped quadratic inside the band
    |t-f| <= sqrt(2 nu / a), nu outside it, and on a straddling interval the least of its
    n_sub equispaced samples (a lower hull attains its minimum at a sample)."""
    d = np.sqrt(2.0 * nu / a)
    if f - d <= g0 and g1 <= f + d:
        return 0.5 * a * (min(max(f, g0), g1) - f) ** 2
    if g1 <= f - d or g0 >= f + d:
        return nu
    ts = g0 + (g1 - g0) * np.arange(n_sub) / (n_sub - 1)
    return float(np.minimum(0.5 * a * (ts - f) ** 2, nu).min())


@pytest.mark.parametrize("L,nu", [(2, 0.01), (3, 0.025), (5, 0.025), (8, 0.1)])
def test_lambda_zero_closed_form_truncated_quadratic(orc, L, nu):
    """lambda = 0 with the truncated quadratic: the relaxed problem decouples per pixel and
    its optimum is sum_x min_i min_{t in Gamma_i} rho_i(x, t), the conjugate of
    max_i rho_i^* taken at 0 (Prop. 1). Both certified bounds must close on it, so a piece
    built too low or too high (a wrong band half-width, a dropped end sample of a
    straddling interval) is caught. With lambda = 0 the dual bound sees p = 0, so it equals
    this sum at every iterate (a two-sided pin of the piece minima); the repaired primal
    bound stays above it and closes on it."""
    rng = np.random.default_rng(100 + L)
    H, Wd, a = 5, 8, 2.0
    f = rng.uniform(-0.1, 1.1, size=(H, Wd)).astype(np.float32)
    gamma = W.equispaced(L)
    d = np.sqrt(2.0 * nu / a)
    ff = f.astype(np.float64).reshape(-1)
    # no band edge within rounding of a label: the float classification is then exact
    assert np.abs(np.subtract.outer(np.concatenate([ff - d, ff + d]), gamma)).min() > 1e-5
    wl = W.Workload("l0tq", H, Wd, gamma, W.TRUNC_QUAD, 0.0, f=f, a=a, nu=nu)
    P = orc.Problem(wl)
    rep, hist = _run_to(P, 1e-10, 30000, every=1000)
    exact = sum(min(_tq_piece_min(x, gamma[i], gamma[i + 1], a, nu) for i in range(L - 1)) for x in ff)
    for r in hist:
        assert r["dual"] == pytest.approx(exact, rel=1e-12)
        assert r["primal"] >= exact - 1e-12 * abs(exact)
    assert rep["best_gap"] <= 0.25 * hist[0]["best_gap"]
    assert rep["rel_gap"] <= 0.25


def test_nonconvex_energy_sampled_matches_interpolation(orc):
    """E_nc for sampled costs (reading C12): the costs interpolated linearly between sample
    positions at the back-projected u, plus lambda times the isotropic TV, here with
    unevenly spaced samples in original label units."""
    rng = np.random.default_rng(16)
    H, Wd, M = 7, 9, 12
    tau = np.cumsum(rng.uniform(0.2, 1.0, size=M)) + 2.0
    gamma = tau[[0, 4, 7, 11]]
    costs = rng.uniform(0, 2, size=(M, H, Wd)).astype(np.float32)
    wl = W.Workload("enc", H, Wd, gamma, W.SAMPLED, 0.3, tau=tau, samples=costs)
    P = orc.Problem(wl)
    P.run(150)
    rep = P.monitor()
    _, u = P.read_u()
    data = 0.0
    for r in range(H):
        for c in range(Wd):
            data += np.interp(u[r, c], tau, costs[:, r, c].astype(np.float64))
    e = data + wl.lam * ck.iso_tv(u)
    assert rep["e_nc"] == pytest.approx(e, rel=1e-11)


def test_prop2_piecewise_linear_equals_baseline_lifting(orc):
    """Prop. 2: with pieces linear between labels the relaxation equals the baseline
    lifting rho(gamma_1) + <u, r> on 1 >= u_1 >= ... >= u_k >= 0; solved independently
    with an isotonic (ordered-box) projection."""
    rng = np.random.default_rng(12)
    H, Wd, L = 8, 9, 5
    gamma = np.array([0.0, 0.2, 0.45, 0.7, 1.0])
    costs = rng.uniform(0, 1, size=(L, H, Wd)).astype(np.float32)
    lam = 0.15
    wl = W.Workload("p2", H, Wd, gamma, W.SAMPLED, lam, tau=gamma.copy(), samples=costs)
    P = orc.Problem(wl)
    rep, _ = _run_to(P, 1e-6, 60000)
    Pb, Db = ck.baseline_lifting(costs.astype(np.float64), gamma, lam, iters=40000, tol=1e-9)
    assert Pb - Db <= 1e-7 * abs(Pb)
    assert rep["best_dual"] <= Pb + 1e-8
    assert Db <= rep["best_primal"] + 1e-8
    assert rep["best_primal"] == pytest.approx(Pb, rel=2e-6)


def _tq_interp_cost(f, t, a, nu, gamma, n_sub=16):
    """Truncated quadratic with straddling intervals replaced by the linear interpolation
    of n_sub equispaced samples: pointwise >= the per-interval convex pieces the relaxation
    uses, so the relaxed optimum is <= any energy built from it."""
    d = np.sqrt(2 * nu / a)
    i = int(np.clip(np.searchsorted(gamma, t, side="right") - 1, 0, len(gamma) - 2))
    g0, g1 = gamma[i], gamma[i + 1]
    q = lambda x: np.minimum(0.5 * a * (x - f) ** 2, nu)
    if (f - d <= g0 and g1 <= f + d) or (g1 <= f - d or g0 >= f + d):
        return float(q(t))
    ts = np.linspace(g0, g1, n_sub)
    return float(np.interp(t, ts, q(ts)))


def test_relaxation_lower_bounds_discrete_minimum_1d(orc):
    """The relaxed energy is a lower bound of the minimum over a fine label grid
    (exact dynamic programming on a chain); 1-D lifted TV of a graph lifting equals the
    TV of the function."""
    rng = np.random.default_rng(13)
    n = 10
    f = rng.uniform(0, 1, size=(1, n)).astype(np.float32)
    wl = W.Workload("c1", 1, n, W.equispaced(4), W.TRUNC_QUAD, 0.05, f=f, a=2.0, nu=0.025)
    P = orc.Problem(wl)
    rep, hist = _run_to(P, 1e-6, 20000)
    grid = np.unique(np.concatenate([np.linspace(0, 1, 1201), wl.gamma]))
    cost = np.array([[_tq_interp_cost(float(f[0, c]), g, 2.0, 0.025, wl.gamma) for g in grid]
                     for c in range(n)])
    dp = ck.dp_chain(cost, grid, wl.lam)
    for r in hist:
        assert r["dual"] <= dp + 1e-9
    assert rep["best_dual"] <= dp + 1e-9


def test_relaxation_lower_bounds_bruteforce_2d(orc):
    """2x3 image: the relaxed optimum lower-bounds the lifted energy of every graph
    lifting with values on an 11-point grid (lifted TV, see the isotropic-TV reading)."""
    rng = np.random.default_rng(14)
    H, Wd = 2, 3
    f = rng.uniform(0, 1, size=(H, Wd)).astype(np.float32)
    gamma = W.equispaced(3)
    wl = W.Workload("b2", H, Wd, gamma, W.TRUNC_QUAD, 0.04, f=f, a=2.0, nu=0.025)
    P = orc.Problem(wl)
    rep, hist = _run_to(P, 1e-6, 20000)
    grid = np.linspace(0, 1, 11)
    ff = f.reshape(-1).astype(np.float64)
    bf = ck.brute_force_lifted(lambda x, g: _tq_interp_cost(ff[x], g, 2.0, 0.025, gamma),
                               grid, gamma, H, Wd, wl.lam)
    for r in hist:
        assert r["dual"] <= bf + 1e-9
    assert rep["rel_gap"] <= 1e-6


def test_gap_monotone_ordering_and_sublabel_values(orc):
    """Convex quadratic data with L = 5: the best-so-far certified gap decreases
    monotonically towards zero, the lifted solution respects 1 >= u_1 >= ... >= u_k >= 0
    (domain of the relaxed data term, proof of Prop. 2) and back-projects to values
    between labels (sublabel accuracy)."""
    wl = W.rof(H=24, W=24)
    wl.gamma = W.equispaced(5)
    P = orc.Problem(wl)
    rep, hist = _run_to(P, 1e-4, 40000)
    gaps = [r["best_gap"] for r in hist]
    assert all(b <= a + 1e-15 for a, b in zip(gaps, gaps[1:]))
    assert rep["rel_gap"] <= 2e-4
    assert gaps[-1] < 1e-2 * gaps[0]
    ul, u = P.read_u()
    assert ul.min() >= -1e-3 and ul.max() <= 1 + 1e-3
    assert (ul[1:] - ul[:-1]).max() <= 1e-3
    on_label = np.isclose(u[..., None], wl.gamma[None, None, :], atol=1e-3).any(-1)
    assert (~on_label).mean() > 0.5


def test_label_normalisation_invariance(orc):
    """Mapping the labels affinely onto [0,1] is an exact reparametrisation: the certified
    optimum is the same."""
    rng = np.random.default_rng(15)
    H, Wd = 6, 6
    tau = np.arange(10, dtype=np.float64) * 0.25 + 0.5
    gamma = tau[[0, 3, 6, 9]]
    costs = rng.uniform(0, 1, size=(10, H, Wd)).astype(np.float32)
    wl = W.Workload("n", H, Wd, gamma, W.SAMPLED, 0.2, tau=tau, samples=costs)
    r1, _ = _run_to(orc.Problem(wl, normalize=True), 1e-8, 80000)
    r0, _ = _run_to(orc.Problem(wl, normalize=False), 1e-6, 80000)
    # the normalised optimum lies in the certified interval of the original problem
    assert r0["best_dual"] - 1e-9 <= r1["best_primal"]
    assert r1["best_dual"] <= r0["best_primal"] + 1e-9
    assert r1["rel_gap"] < 1e-8 and r0["rel_gap"] < 1e-4


def test_nonconvex_energy_matches_definition(orc):
    """E_nc of the monitor equals the energy (eq. 1, discretised) of the back-projected u."""
    wl = W.truncated_quadratic(L=6, H=12, W=14)
    P = orc.Problem(wl)
    P.run(300)
    rep = P.monitor()
    _, u = P.read_u()
    f = wl.f.astype(np.float64)
    e = np.minimum((u - f) ** 2, 0.025).sum() + wl.lam * ck.iso_tv(u)
    assert rep["e_nc"] == pytest.approx(e, rel=1e-12)


def test_invalid_arguments_rejected(orc):
    f = np.zeros((3, 3), np.float32)
    bad = [
        W.Workload("x", 3, 3, np.array([0.0, 0.0, 1.0]), W.QUAD, 0.1, f=f),
        W.Workload("x", 3, 3, np.array([0.0]), W.QUAD, 0.1, f=f),
        W.Workload("x", 3, 3, W.equispaced(3), W.QUAD, -1.0, f=f),
        W.Workload("x", 3, 3, W.equispaced(3), W.QUAD, 0.1, f=f, a=0.0),
        W.Workload("x", 3, 3, W.equispaced(3), W.TRUNC_QUAD, 0.1, f=f, a=1.0, nu=0.0),
        W.Workload("x", 3, 3, W.equispaced(3), W.QUAD, 0.1, f=np.full((3, 3), np.nan, np.float32)),
        W.Workload("x", 3, 3, np.array([0.0, 0.5, 1.0]), W.SAMPLED, 0.1,
                   tau=np.array([0.0, 0.4, 1.0]), samples=np.zeros((3, 3, 3), np.float32)),
    ]
    for wl in bad:
        with pytest.raises(ValueError):
            orc.Problem(wl)


def test_proposed_relaxation_below_baseline_lifting(orc):
    """At the same labels the proposed pieces (convex envelopes of rho on each interval)
    lie below the baseline's chords between the labels (a convex function on an interval
    lies below its chord, and the envelope meets rho at the interval ends), so the
    proposed relaxed optimum is at most the baseline's (Sec. 5, Prop. 2)."""
    for L in (3, 5):
        tq = W.truncated_quadratic(L=L, H=10, W=12, seed=44)
        rp, _ = _run_to(orc.Problem(tq), 2e-4, 80000)
        rb, _ = _run_to(orc.Problem(W.baseline_lifting(tq)), 1e-9, 80000)
        assert rp["rel_gap"] <= 2e-4 and rb["rel_gap"] <= 1e-9
        # certified: the proposed upper bound is below the baseline's lower bound
        assert rp["best_primal"] < rb["best_dual"]
