"""Pins of the oracle's building blocks against what the paper and the mathematics fix:
hand-derived worked cases (tests/golden), brute force, optimality conditions and
textbook identities. CPU only."""
import json
import os

import numpy as np
import pytest

import workloads as W
from tests import checkers as ck

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "primitives.json")))


# ------------------------------------------------------------------ golden worked cases

def test_golden_conj_quad(orc):
    g = GOLD["conj_quad"]
    p = g["piece"]
    for y, val in g["cases"]:
        assert orc.conj_quad(p["a"], p["c"], p["d"], p["g0"], p["g1"], y) == pytest.approx(val, abs=1e-14)


def test_golden_proj_epi_quad(orc):
    g = GOLD["proj_epi_quad"]
    p = g["piece"]
    for (y, w), (ey, ew) in g["cases"]:
        py_, pw = orc.proj_epi_quad(p["a"], p["c"], p["d"], p["g0"], p["g1"], y, w)
        assert (py_, pw) == pytest.approx((ey, ew), abs=1e-12)


def test_golden_conj_and_proj_pl(orc):
    g = GOLD["conj_pl"]
    for y, val in g["cases"]:
        assert orc.conj_pl(g["t"], g["r"], y) == pytest.approx(val, abs=1e-14)
    g = GOLD["proj_epi_pl"]
    for (y, w), (ey, ew) in g["cases"]:
        assert orc.proj_epi_pl(g["t"], g["r"], y, w) == pytest.approx((ey, ew), abs=1e-12)


def test_golden_ball(orc):
    for (px, py), rad, exp in GOLD["proj_ball"]["cases"]:
        assert orc.proj_ball(px, py, rad) == pytest.approx(tuple(exp), abs=1e-15)


def test_golden_tq_pieces(orc):
    """Truncated-quadratic pieces (Sec. 5.2) against hand-derived cases: an interval inside
    the band (quadratic piece), one outside it (constant), one straddling each band edge
    and one holding both edges (lower hull of the 16 samples)."""
    g = GOLD["tq_pieces"]
    for case in g["cases"]:
        f = np.full((1, 1), case["f"], np.float32)
        wl = W.Workload("tq", 1, 1, np.array(case["gamma"]), W.TRUNC_QUAD, 0.1, f=f,
                        a=case["a"], nu=case["nu"])
        kind, acd, t, r = orc.Problem(wl).piece(0, case["interval"])
        if case["kind"] == "quad":
            assert kind == 0, case["name"]
            assert acd == pytest.approx(case["acd"], abs=1e-7), case["name"]
        else:
            assert kind == 1, case["name"]
            assert len(t) == len(case["t"]), (case["name"], t)
            assert t == pytest.approx(case["t"], abs=1e-12), case["name"]
            assert r == pytest.approx(case["r"], abs=1e-8), case["name"]


def test_golden_variable_count(orc):
    """The state holds 6N(L-1)+N variables (Sec. 5) plus the 2N(L-1) primal history."""
    for H, Wd, L in GOLD["variable_count"]["cases"]:
        wl = W.Workload("vc", H, Wd, W.equispaced(L), W.QUAD, 0.1,
                        f=np.zeros((H, Wd), np.float32))
        P = orc.Problem(wl)
        N, k = H * Wd, L - 1
        st = P.get_state()
        paper_vars = sum(st[n].size for n in ("u", "s", "v", "z", "px", "py", "qd"))
        assert paper_vars == 6 * N * (L - 1) + N
        assert sum(a.size for a in st.values()) == paper_vars + 2 * N * k


# ------------------------------------------------------------------ operators

def test_grad_div_adjoint(orc):
    rng = np.random.default_rng(0)
    for H, Wd in [(1, 7), (5, 1), (6, 9), (13, 4)]:
        u = rng.normal(size=(H, Wd))
        px, py = rng.normal(size=(H, Wd)), rng.normal(size=(H, Wd))
        gx, gy = orc.grad(u)
        lhs = (gx * px + gy * py).sum()
        rhs = -(u * orc.div(px, py)).sum()
        assert lhs == pytest.approx(rhs, rel=1e-13, abs=1e-13)
        # against an independent np.diff implementation
        cx, cy = ck.fd_grad(u)
        np.testing.assert_allclose(gx, cx, atol=1e-15)
        np.testing.assert_allclose(gy, cy, atol=1e-15)
        np.testing.assert_allclose(orc.div(px, py), ck.fd_div(px, py), atol=1e-14)


def _lagrangian_bilinear(gam, H, Wd, u, s, v, q, px, py, z):
    """Bilinear part of the Lagrangian of the split saddle-point problem (Sec. 4), written
    term by term: <u,v> + <p, grad u> + sum_i s_i (z_i - h_i q + h_i <1_{i-1},v> - gamma_i v_i)."""
    k = len(gam) - 1
    h = np.diff(gam)
    total = (u * v).sum()
    gx, gy = ck.fd_grad(u)
    total += (px * gx + py * gy).sum()
    for i in range(k):
        c_i = h[i] * v[:i].sum(axis=0) - gam[i] * v[i]        # h_i * c_i(v)
        total += (s[i] * (z[i] - h[i] * q + c_i)).sum()
    return total


@pytest.mark.parametrize("gamma", [[0.0, 0.3, 0.55, 1.0], [-2.0, -0.5, 1.0, 1.5, 4.0]])
def test_operator_K_matches_lagrangian(orc, gamma):
    """Assemble K column by column from the Lagrangian and compare with the oracle's
    matrix-free K and K^T; the diagonal steps are the inverse absolute row / column sums
    (Pock-Chambolle preconditioning, alpha = 1; v_i and z_i share a step)."""
    H, Wd = 3, 4
    gam = np.array(gamma)
    L = len(gam)
    k, N = L - 1, H * Wd
    wl = W.Workload("K", H, Wd, gam, W.QUAD, 0.3, f=np.zeros((H, Wd), np.float32))
    P = orc.Problem(wl, normalize=False)
    nx = 2 * k * N
    ny_shape = [(k, H, Wd), (H, Wd), (k, H, Wd), (k, H, Wd), (k, H, Wd)]   # v q px py z
    ny = sum(int(np.prod(s)) for s in ny_shape)

    def split_y(yv):
        out, o = [], 0
        for s in ny_shape:
            n = int(np.prod(s))
            out.append(yv[o:o + n].reshape(s))
            o += n
        return out

    Kmat = np.zeros((ny, nx))
    for col in range(nx):
        xv = np.zeros(nx)
        xv[col] = 1.0
        u, s = xv[:k * N].reshape(k, H, Wd), xv[k * N:].reshape(k, H, Wd)
        for row in range(ny):
            yv = np.zeros(ny)
            yv[row] = 1.0
            Kmat[row, col] = _lagrangian_bilinear(gam, H, Wd, u, s, *split_y(yv))
    rng = np.random.default_rng(1)
    xv = rng.normal(size=nx)
    Kv, Kq, Kpx, Kpy, Kz = P.apply_K(xv[:k * N], xv[k * N:])
    np.testing.assert_allclose(np.concatenate([Kv, Kq, Kpx, Kpy, Kz]), Kmat @ xv, atol=1e-12)
    yv = rng.normal(size=ny)
    v, q, px, py, z = split_y(yv)
    Ku, Ks = P.apply_KT(v, q, px, py, z)
    np.testing.assert_allclose(np.concatenate([Ku, Ks]), Kmat.T @ yv, atol=1e-12)

    sig_p, sig_vz, sig_q, tau_u, tau_s = P.steps()
    rows = np.abs(Kmat).sum(axis=1)
    cols = np.abs(Kmat).sum(axis=0)
    r_v, r_q, r_px, r_py, r_z = split_y(rows)
    np.testing.assert_allclose(sig_vz, 1.0 / np.maximum(r_v, r_z).reshape(k, N)[:, 0])
    assert np.allclose(r_v, r_v[:, :1, :1])          # constant over pixels
    assert sig_q == pytest.approx(1.0 / r_q.ravel()[0])
    assert sig_p == pytest.approx(1.0 / max(r_px.max(), r_py.max()))
    np.testing.assert_allclose(tau_u, 1.0 / cols[:k * N].reshape(k, N)[0])
    np.testing.assert_allclose(tau_s, 1.0 / cols[k * N:].reshape(k, N)[:, 0])


# ------------------------------------------------------------------ projections

def _rand_quad_piece(rng):
    a = rng.uniform(0.2, 5.0)
    g0 = rng.uniform(-2, 2)
    g1 = g0 + rng.uniform(0.05, 2.0)
    c = rng.uniform(g0 - 1, g1 + 1)
    d = rng.uniform(-1, 1)
    return a, c, d, g0, g1


def test_conj_quad_bruteforce(orc):
    rng = np.random.default_rng(2)
    for _ in range(50):
        a, c, d, g0, g1 = _rand_quad_piece(rng)
        ts = np.linspace(g0, g1, 200001)
        rho = 0.5 * a * (ts - c) ** 2 + d
        for y in rng.normal(0, 4, size=8):
            bf = (ts * y - rho).max()
            lip = abs(y) + a * max(abs(g0 - c), abs(g1 - c))
            assert orc.conj_quad(a, c, d, g0, g1, y) == pytest.approx(bf, abs=lip * (g1 - g0) / 200000 + 1e-12)


def _bf_epigraph_proj(gfun, y0, w0, n=4001):
    """Nearest point of the graph of g to an outside point by dense search, then a
    local refinement (golden section on the y coordinate)."""
    R = abs(gfun(y0) - w0) + 1e-3
    ys = np.linspace(y0 - R, y0 + R, n)
    gs = np.array([gfun(y) for y in ys])
    d = (ys - y0) ** 2 + (gs - w0) ** 2
    j = int(np.argmin(d))
    lo, hi = ys[max(j - 1, 0)], ys[min(j + 1, n - 1)]
    phi = (np.sqrt(5) - 1) / 2
    f = lambda y: (y - y0) ** 2 + (gfun(y) - w0) ** 2
    for _ in range(100):
        m1, m2 = hi - phi * (hi - lo), lo + phi * (hi - lo)
        if f(m1) < f(m2):
            hi = m2
        else:
            lo = m1
    y = 0.5 * (lo + hi)
    return y, gfun(y)


def test_proj_epi_quad_bruteforce_and_kkt(orc):
    rng = np.random.default_rng(3)
    for trial in range(120):
        a, c, d, g0, g1 = _rand_quad_piece(rng)
        # brute-force conjugate from its definition (sup over a dense grid of t)
        ts = np.linspace(g0, g1, 4001)
        rho = 0.5 * a * (ts - c) ** 2 + d
        gbf = lambda y: float((ts * y - rho).max())
        y0 = rng.normal(0, 3)
        w0 = gbf(y0) - abs(rng.normal(0, 3)) - 1e-3          # strictly below the graph
        py_, pw = orc.proj_epi_quad(a, c, d, g0, g1, y0, w0)
        # on the graph
        gy = orc.conj_quad(a, c, d, g0, g1, py_)
        assert pw == pytest.approx(gy, abs=1e-9)
        # KKT: residual is an outward normal (g'(y), -1) * mu, mu >= 0
        slope = min(max(c + py_ / a, g0), g1)
        ry, rw = y0 - py_, w0 - pw
        assert rw <= 1e-12
        assert ry + slope * rw == pytest.approx(0.0, abs=1e-8 * (1 + abs(rw)))
        # brute force nearest point
        by, bw = _bf_epigraph_proj(gbf, y0, w0)
        dist_or = np.hypot(py_ - y0, pw - w0)
        dist_bf = np.hypot(by - y0, bw - w0)
        assert dist_or <= dist_bf + 1e-6 * (1 + dist_bf)
        assert np.hypot(py_ - by, pw - bw) <= 1e-3 * (1 + dist_bf)
        # idempotence and points inside stay
        assert orc.proj_epi_quad(a, c, d, g0, g1, py_, pw) == pytest.approx((py_, pw), abs=1e-12)
        assert orc.proj_epi_quad(a, c, d, g0, g1, y0, gbf(y0) + 0.5) == (y0, gbf(y0) + 0.5)


def test_proj_epi_quad_three_root_region(orc):
    """Points far below the parabola vertex with W0 > a make the cubic have three real
    roots; the projection must still be the nearest graph point."""
    a, c, d, g0, g1 = 1.0, 0.0, 0.0, -20.0, 20.0
    for y0, w0 in [(10.0, 40.0), (-10.0, 40.0), (3.0, 4.0), (0.5, 0.05)]:
        assert w0 < y0 * y0 / (2 * a)                     # outside the epigraph
        py_, pw = orc.proj_epi_quad(a, c, d, g0, g1, y0, w0)
        # brute force on the arc (rays are far away here)
        Y = np.linspace(-30, 30, 2000001)
        dd = (Y - y0) ** 2 + (Y * Y / 2 - w0) ** 2
        j = np.argmin(dd)
        assert np.hypot(py_ - Y[j], pw - Y[j] ** 2 / 2) < 1e-4


def _rand_convex_pl(rng, n):
    t = np.sort(rng.uniform(-2, 2, size=n))
    t = np.unique(t)
    slopes = np.sort(rng.normal(0, 2, size=len(t) - 1))
    r = rng.normal() + np.concatenate([[0.0], np.cumsum(slopes * np.diff(t))])
    return t, r


def test_conj_pl_bruteforce(orc):
    rng = np.random.default_rng(4)
    for _ in range(40):
        t, r = _rand_convex_pl(rng, rng.integers(2, 9))
        tt = np.linspace(t[0], t[-1], 100001)
        rr = np.interp(tt, t, r)
        for y in rng.normal(0, 3, size=6):
            bf = (tt * y - rr).max()
            lip = abs(y) + np.abs(np.diff(r) / np.diff(t)).max()
            assert orc.conj_pl(t, r, y) == pytest.approx(bf, abs=lip * (tt[1] - tt[0]) + 1e-12)


def test_proj_epi_pl_bruteforce_and_kkt(orc):
    rng = np.random.default_rng(5)
    for _ in range(150):
        t, r = _rand_convex_pl(rng, rng.integers(2, 9))
        gbf = lambda y: float((t * y - r).max())
        y0 = rng.normal(0, 3)
        w0 = gbf(y0) - abs(rng.normal(0, 3)) - 1e-3
        py_, pw = orc.proj_epi_pl(t, r, y0, w0)
        assert pw == pytest.approx(gbf(py_), abs=1e-9)
        # KKT: (y0-py, pw-w0) = mu (s, 1) with s in the subdifferential [t_lo, t_hi] at py
        vals = t * py_ - r
        act = np.where(vals >= vals.max() - 1e-9)[0]
        ry, rw = y0 - py_, pw - w0
        assert rw >= -1e-12
        if rw > 1e-9:
            s = ry / rw
            assert t[act].min() - 1e-6 <= s <= t[act].max() + 1e-6
        by, bw = _bf_epigraph_proj(gbf, y0, w0)
        assert np.hypot(py_ - y0, pw - w0) <= np.hypot(by - y0, bw - w0) + 1e-7
        assert orc.proj_epi_pl(t, r, py_, pw) == pytest.approx((py_, pw), abs=1e-12)


def test_lower_hull_bruteforce(orc):
    """The lower convex envelope of a point set is unique: it lies below every point,
    touches the hull vertices, and its slopes increase strictly."""
    rng = np.random.default_rng(6)
    for _ in range(200):
        n = int(rng.integers(1, 17))
        t = np.sort(rng.choice(np.linspace(0, 1, 200), size=n, replace=False))
        r = rng.normal(size=n) if rng.random() < 0.7 else (t - 0.5) ** 2
        idx = orc.lower_hull(t, r)
        assert idx[0] == 0 and idx[-1] == n - 1
        env = np.interp(t, t[idx], r[idx])
        assert np.all(env <= r + 1e-12)
        if len(idx) >= 3:
            sl = np.diff(r[idx]) / np.diff(t[idx])
            assert np.all(np.diff(sl) > 0)
        # O(n^2) check: a point is a hull vertex iff no chord between two other points lies
        # on or below it
        for j in range(n):
            below = False
            for a in range(j):
                for b in range(j + 1, n):
                    lam = (t[j] - t[a]) / (t[b] - t[a])
                    if (1 - lam) * r[a] + lam * r[b] <= r[j] + 1e-12:
                        below = True
            assert (j in idx) == (not below)


def test_proj_simplex_vs_bisection(orc):
    rng = np.random.default_rng(7)
    for n in [1, 2, 3, 7, 19]:
        for _ in range(30):
            x = rng.normal(0, 2, size=n)
            np.testing.assert_allclose(orc.proj_simplex(x), ck.simplex_bisection(x), atol=1e-10)


def test_ball_invariants(orc):
    rng = np.random.default_rng(8)
    for _ in range(100):
        px, py, rad = rng.normal(0, 3), rng.normal(0, 3), abs(rng.normal())
        a, b = orc.proj_ball(px, py, rad)
        assert np.hypot(a, b) <= rad * (1 + 1e-14)
        assert orc.proj_ball(a, b, rad) == pytest.approx((a, b), abs=1e-15)
        if np.hypot(px, py) > rad:
            assert a * py - b * px == pytest.approx(0.0, abs=1e-12)


def test_isotonic_checker_vs_sklearn():
    """The independent ordered-box projection used by the Prop. 2 checker."""
    from sklearn.isotonic import IsotonicRegression
    rng = np.random.default_rng(9)
    for _ in range(50):
        y = rng.normal(size=6)
        ref = IsotonicRegression(increasing=False).fit_transform(np.arange(6), y)
        np.testing.assert_allclose(ck.iso_decreasing(y[:, None])[:, 0], ref, atol=1e-12)
