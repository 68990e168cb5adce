"""Pins of the oracle's reverse pass (differentiation of K unrolled iterations) against
FP64 central finite differences of the oracle's own forward pass.

* projection adjoints (ball, quadratic and piecewise-linear epigraphs) against finite
  differences of the projections, at random points away from kinks;
* the adjoint of one whole iteration by the dot-product test <J d, w> = <d, J^T w> with
  J d taken by central differences of the iteration;
* gradients of a squared-error loss of the read-out u after K iterations with respect to
  the data image f, lambda and the additive values w, against central differences on 16
  random coordinates (seed 51); a coordinate whose one-sided differences disagree sits at
  a kink of the unrolled map and is replaced by another.

Inputs are stored in float32 (as the C-ABI takes them), so a perturbation is taken as the
exact float32 step x -> fl(x +- 1e-6) and divided by its true size.
"""
import copy

import numpy as np
import pytest

import workloads as W

EPS = 1e-6


def _kink(fp, fm, f0, h):
    a, b = (fp - f0) / h, (f0 - fm) / h
    return abs(a - b) > 1e-4 * (1.0 + abs(a))


def test_projection_vjps_match_finite_differences(orc):
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(600):
        a = rng.uniform(0.5, 5)
        c = rng.uniform(-0.5, 1.5)
        d = rng.uniform(-0.3, 0.3)
        g0 = rng.uniform(-0.5, 0.5)
        g1 = g0 + rng.uniform(0.05, 1)
        y0, w0 = rng.normal(0, 2, 2)
        yb, wb = rng.normal(size=2)
        got = orc.proj_epi_quad_vjp(a, c, d, g0, g1, y0, w0, yb, wb)

        def F(dy=0.0, dw=0.0, dc=0.0, dd=0.0):
            y, w = orc.proj_epi_quad(a, c + dc, d + dd, g0, g1, y0 + dy, w0 + dw)
            return yb * y + wb * w

        for j, key in enumerate(("dy", "dw", "dc", "dd")):
            fp, fm, f0 = F(**{key: EPS}), F(**{key: -EPS}), F()
            if _kink(fp, fm, f0, EPS):
                continue
            fd = (fp - fm) / (2 * EPS)
            assert abs(fd - got[j]) <= 1e-6 * (1 + abs(fd)), (key, fd, got[j])
            checked += 1
    for _ in range(400):
        n = int(rng.integers(2, 7))
        t = np.sort(rng.uniform(-1, 2, n)) + 0.01 * np.arange(n)
        slopes = np.sort(rng.normal(0, 2, n - 1))
        r = np.concatenate([[0.0], np.cumsum(slopes * np.diff(t))]) + rng.normal()
        y0, w0 = rng.normal(0, 3, 2)
        yb, wb = rng.normal(size=2)
        y0b, w0b, rb = orc.proj_epi_pl_vjp(t, r, y0, w0, yb, wb)

        def G(dy=0.0, dw=0.0, m=-1, dr=0.0):
            rr = r.copy()
            if m >= 0:
                rr[m] += dr
            y, w = orc.proj_epi_pl(t, rr, y0 + dy, w0 + dw)
            return yb * y + wb * w

        cases = [(dict(dy=EPS), dict(dy=-EPS), y0b), (dict(dw=EPS), dict(dw=-EPS), w0b)]
        cases += [(dict(m=m, dr=EPS), dict(m=m, dr=-EPS), rb[m]) for m in range(n)]
        for kp, km, val in cases:
            fp, fm, f0 = G(**kp), G(**km), G()
            if _kink(fp, fm, f0, EPS):
                continue
            fd = (fp - fm) / (2 * EPS)
            assert abs(fd - val) <= 1e-6 * (1 + abs(fd)), (kp, fd, val)
            checked += 1
    for _ in range(300):
        ax, ay = rng.normal(0, 1, 2)
        rad = rng.uniform(0.1, 2)
        pb = rng.normal(size=2)
        axb, ayb, rb = orc.proj_ball_vjp(ax, ay, rad, pb[0], pb[1])

        def B(dx=0.0, dy=0.0, dr=0.0):
            return float(np.dot(pb, orc.proj_ball(ax + dx, ay + dy, rad + dr)))

        for kp, km, val in ((dict(dx=EPS), dict(dx=-EPS), axb), (dict(dy=EPS), dict(dy=-EPS), ayb),
                            (dict(dr=EPS), dict(dr=-EPS), rb)):
            fp, fm, f0 = B(**kp), B(**km), B()
            if _kink(fp, fm, f0, EPS):
                continue
            fd = (fp - fm) / (2 * EPS)
            assert abs(fd - val) <= 1e-6 * (1 + abs(fd))
            checked += 1
    assert checked > 4000


def _quad_w(rng, H=8, Wd=9):
    gam = np.array([0.0, 0.3, 0.5, 1.0])
    return W.Workload("qw", H, Wd, gam, W.QUAD, 0.3, f=rng.uniform(0, 1, (H, Wd)).astype(np.float32),
                      a=2.0, tau=gam.copy(), samples=rng.normal(0, 0.1, (4, H, Wd)).astype(np.float32))


def _tq_w(rng, L=5, H=10, Wd=12, seed=4):
    wl = W.truncated_quadratic(L=L, H=H, W=Wd, seed=seed)
    wl.tau = wl.gamma.copy()
    wl.samples = rng.normal(0, 0.02, (L, H, Wd)).astype(np.float32)
    return wl


@pytest.mark.parametrize("kind", ["quad", "quad_w", "tq", "tq_w"])
def test_step_adjoint_dot_product(orc, kind):
    rng = np.random.default_rng(21)
    if kind.startswith("quad"):
        wl = _quad_w(rng, 6, 8)
    else:
        wl = _tq_w(rng, 5, 7, 9, 3)
    if not kind.endswith("_w"):
        wl.tau, wl.samples = None, None
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


def _loss(orc, wl, g, K):
    o = orc.Problem(wl)
    o.run(K)
    _, u = o.read_u()
    return float(np.sum((u - g) ** 2))


def _fd_f32(orc, wl, g, K, field, idx):
    x = np.float32(getattr(wl, field)[idx])
    xs = (np.float32(x + np.float32(EPS)), np.float32(x - np.float32(EPS)), x)
    vals = []
    for v in xs:
        w2 = copy.copy(wl)
        arr = getattr(wl, field).copy()
        arr[idx] = v
        setattr(w2, field, arr)
        vals.append(_loss(orc, w2, g, K))
    lp, lm, l0 = vals
    hp, hm = float(xs[0]) - float(x), float(x) - float(xs[1])
    kink = abs((lp - l0) / hp - (l0 - lm) / hm) > 1e-4 * (1.0 + abs((lp - l0) / hp))
    return (lp - lm) / (hp + hm), kink


@pytest.mark.parametrize("kind", ["quad_w", "tq_w"])
def test_unrolled_gradients_match_finite_differences(orc, kind):
    rng = np.random.default_rng(5)
    wl = _quad_w(rng) if kind == "quad_w" else _tq_w(rng)
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

    pick = np.random.default_rng(51)
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


def _with(wl, **kw):
    w2 = copy.copy(wl)
    for k, v in kw.items():
        setattr(w2, k, v)
    return w2


def test_reverse_pass_preconditions(orc):
    rng = np.random.default_rng(3)
    wl = _quad_w(rng)
    o = orc.Problem(wl)
    with pytest.raises(ValueError):
        o.unrolled_backward(np.zeros((wl.H, wl.W)))       # no forward pass yet
    o.unrolled_forward(3)
    o.run(1)
    with pytest.raises(ValueError):
        o.unrolled_backward(np.zeros((wl.H, wl.W)))       # state moved on since
    smp = W.Workload("s", 4, 5, np.array([0.0, 2.0, 4.0]), W.SAMPLED, 0.3, tau=np.arange(5.0),
                     samples=rng.uniform(0, 1, (5, 4, 5)).astype(np.float32))
    o = orc.Problem(smp)
    o.unrolled_forward(2)
    with pytest.raises(ValueError):
        o.unrolled_backward(np.zeros((4, 5)))


def test_zero_loss_adjoint_gives_zero_gradients(orc):
    rng = np.random.default_rng(8)
    wl = _tq_w(rng, 4, 6, 7, 9)
    o = orc.Problem(wl)
    o.unrolled_forward(10)
    gf, gl, gw = o.unrolled_backward(np.zeros((wl.H, wl.W)))
    assert not gf.any() and gl == 0.0 and not gw.any()
