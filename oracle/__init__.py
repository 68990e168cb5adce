"""ctypes binding of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the CPU
baseline leg of the benchmark, never by the product package. It shares no code with
the HIP path; both consume the seeded inputs of the ``workloads`` module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "oracle.c")

QUAD, TRUNC_QUAD, SAMPLED = 0, 1, 2
TV_ISO, TV_ANISO = 0, 1
PIECE_QUAD, PIECE_PL = 0, 1


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (IEEE double, no FMA contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", LIB_PATH + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Desc(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("L", C.c_int32),
                ("gamma", C.POINTER(C.c_double)), ("rho", C.c_int32),
                ("f", C.POINTER(C.c_float)), ("a", C.c_double), ("nu", C.c_double),
                ("M", C.c_int32), ("tau", C.POINTER(C.c_double)),
                ("samples", C.POINTER(C.c_float)), ("lam", C.c_double),
                ("normalize", C.c_int32), ("n_sub", C.c_int32), ("step_balance", C.c_double),
                ("tv", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("primal", C.c_double), ("dual", C.c_double), ("best_primal", C.c_double),
                ("best_dual", C.c_double), ("gap", C.c_double), ("best_gap", C.c_double),
                ("rel_gap", C.c_double), ("e_nc", C.c_double), ("iters", C.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None
_dp = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.or_last_error.restype = C.c_char_p
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.POINTER(_Desc)]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_num_threads.argtypes = [C.c_int]
        L.or_num_threads.restype = C.c_int
        L.or_run.argtypes = [C.c_void_p, C.c_int]
        L.or_monitor.argtypes = [C.c_void_p, C.POINTER(Report)]
        L.or_state_size.argtypes = [C.c_void_p]
        L.or_state_size.restype = C.c_int64
        L.or_get_state.argtypes = [C.c_void_p, _dp]
        L.or_set_state.argtypes = [C.c_void_p, _dp]
        L.or_read_u.argtypes = [C.c_void_p, _dp, _dp]
        L.or_normalized.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.or_apply_K.argtypes = [C.c_void_p] + [_dp] * 7
        L.or_apply_KT.argtypes = [C.c_void_p] + [_dp] * 7
        L.or_steps.argtypes = [C.c_void_p] + [_dp] * 5
        L.or_piece.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.POINTER(C.c_int), _dp,
                               C.POINTER(C.c_int), _dp, _dp]
        L.or_grad.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
        L.or_div.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
        L.or_conj_quad.argtypes = [C.c_double] * 6
        L.or_conj_quad.restype = C.c_double
        L.or_proj_epi_quad.argtypes = [C.c_double] * 5 + [_dp, _dp]
        L.or_conj_pl.argtypes = [C.c_int, _dp, _dp, C.c_double]
        L.or_conj_pl.restype = C.c_double
        L.or_proj_epi_pl.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
        L.or_lower_hull.argtypes = [C.c_int, _dp, _dp, C.POINTER(C.c_int)]
        L.or_lower_hull.restype = C.c_int
        L.or_proj_simplex.argtypes = [C.c_int, _dp, _dp]
        L.or_proj_ball.argtypes = [_dp, _dp, C.c_double]
        L.or_proj_box.argtypes = [_dp, _dp, C.c_double]
        L.or_stereo_costs.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_float),
                                      C.POINTER(C.c_float), C.c_double, _dp]
        L.or_residual_norms.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.or_unrolled_forward.argtypes = [C.c_void_p, C.c_int]
        L.or_unrolled_backward.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.or_step_vjp.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp]
        L.or_proj_ball_vjp.argtypes = [C.c_double] * 5 + [_dp] * 3
        L.or_proj_box_vjp.argtypes = [C.c_double] * 5 + [_dp] * 3
        L.or_proj_epi_quad_vjp.argtypes = [C.c_double] * 9 + [_dp] * 4
        L.or_proj_epi_pl_vjp.argtypes = [C.c_int, _dp, _dp] + [C.c_double] * 4 + [_dp] * 3
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> int:
    return lib().or_num_threads(int(n))


# ----------------------------------------------------------------------------- primitives

def grad(u: np.ndarray):
    u = _f64(u)
    H, W = u.shape
    gx, gy = np.empty_like(u), np.empty_like(u)
    lib().or_grad(H, W, _p(u), _p(gx), _p(gy))
    return gx, gy


def div(px: np.ndarray, py: np.ndarray):
    px, py = _f64(px), _f64(py)
    H, W = px.shape
    d = np.empty_like(px)
    lib().or_div(H, W, _p(px), _p(py), _p(d))
    return d


def conj_quad(a, c, d, g0, g1, y) -> float:
    return lib().or_conj_quad(a, c, d, g0, g1, y)


def proj_epi_quad(a, c, d, g0, g1, y, w):
    yy, ww = C.c_double(y), C.c_double(w)
    lib().or_proj_epi_quad(a, c, d, g0, g1, C.byref(yy), C.byref(ww))
    return yy.value, ww.value


def conj_pl(t, r, y) -> float:
    t, r = _f64(t), _f64(r)
    return lib().or_conj_pl(len(t), _p(t), _p(r), y)


def proj_epi_pl(t, r, y, w):
    t, r = _f64(t), _f64(r)
    yy, ww = C.c_double(y), C.c_double(w)
    lib().or_proj_epi_pl(len(t), _p(t), _p(r), C.byref(yy), C.byref(ww))
    return yy.value, ww.value


def lower_hull(t, r):
    t, r = _f64(t), _f64(r)
    idx = (C.c_int * len(t))()
    n = lib().or_lower_hull(len(t), _p(t), _p(r), idx)
    return np.array(idx[:n], dtype=np.int64)


def proj_simplex(x):
    x = _f64(x)
    out = np.empty_like(x)
    lib().or_proj_simplex(len(x), _p(x), _p(out))
    return out


def proj_ball(px, py, radius):
    a, b = C.c_double(px), C.c_double(py)
    lib().or_proj_ball(C.byref(a), C.byref(b), radius)
    return a.value, b.value


def stereo_costs(left, right, D: int, trunc: float):
    """Matching costs [D][H][W] of a rectified pair (see or_stereo_costs)."""
    left = np.ascontiguousarray(left, dtype=np.float32)
    right = np.ascontiguousarray(right, dtype=np.float32)
    H, W = left.shape
    out = np.empty((D, H, W), np.float64)
    fp = C.POINTER(C.c_float)
    lib().or_stereo_costs(H, W, D, left.ctypes.data_as(fp), right.ctypes.data_as(fp),
                          float(trunc), _p(out))
    return out


def proj_box(px, py, radius):
    a, b = C.c_double(px), C.c_double(py)
    lib().or_proj_box(C.byref(a), C.byref(b), radius)
    return a.value, b.value


def proj_box_vjp(ax, ay, radius, pxb, pyb):
    """Adjoint of the box projection: returns (axb, ayb, radius_b)."""
    a, b, r = C.c_double(), C.c_double(), C.c_double(0.0)
    lib().or_proj_box_vjp(ax, ay, radius, pxb, pyb, C.byref(a), C.byref(b), C.byref(r))
    return a.value, b.value, r.value


def proj_ball_vjp(ax, ay, radius, pxb, pyb):
    """Adjoint of the ball projection: returns (axb, ayb, radius_b)."""
    a, b, r = C.c_double(), C.c_double(), C.c_double(0.0)
    lib().or_proj_ball_vjp(ax, ay, radius, pxb, pyb, C.byref(a), C.byref(b), C.byref(r))
    return a.value, b.value, r.value


def proj_epi_quad_vjp(a, c, d, g0, g1, y0, w0, yb, wb):
    """Adjoint of proj_epi_quad at (y0, w0): returns (y0b, w0b, cb, db)."""
    o = [C.c_double(0.0) for _ in range(4)]
    lib().or_proj_epi_quad_vjp(a, c, d, g0, g1, y0, w0, yb, wb, *[C.byref(x) for x in o])
    return tuple(x.value for x in o)


def proj_epi_pl_vjp(t, r, y0, w0, yb, wb):
    """Adjoint of proj_epi_pl at (y0, w0): returns (y0b, w0b, rb[n])."""
    t, r = _f64(t), _f64(r)
    rb = np.zeros(len(t))
    y0b, w0b = C.c_double(), C.c_double()
    lib().or_proj_epi_pl_vjp(len(t), _p(t), _p(r), y0, w0, yb, wb, C.byref(y0b), C.byref(w0b), _p(rb))
    return y0b.value, w0b.value, rb


# ----------------------------------------------------------------------------- problem

STATE_ORDER = ("u", "u_prev", "s", "s_prev", "v", "z", "px", "py", "qd")


class Problem:
    """FP64 oracle instance built from a ``workloads.Workload``."""

    def __init__(self, wl, normalize: bool = True, n_sub: int = 16, step_balance: float = 1.0):
        self.wl = wl
        self.k = wl.k
        self.H, self.W = wl.H, wl.W
        self._keep = []
        d = _Desc()
        d.H, d.W, d.L = wl.H, wl.W, wl.L
        gam = _f64(wl.gamma)
        d.gamma = _p(gam)
        d.rho = wl.rho
        self._keep.append(gam)
        if wl.f is not None:
            f = np.ascontiguousarray(wl.f, dtype=np.float32).reshape(-1)
            d.f = f.ctypes.data_as(C.POINTER(C.c_float))
            self._keep.append(f)
        d.a, d.nu = float(wl.a), float(wl.nu)
        if wl.tau is not None:
            tau = _f64(wl.tau)
            smp = np.ascontiguousarray(wl.samples, dtype=np.float32).reshape(-1)
            d.M = len(tau)
            d.tau = _p(tau)
            d.samples = smp.ctypes.data_as(C.POINTER(C.c_float))
            self._keep += [tau, smp]
        d.lam = float(wl.lam)
        d.normalize = 1 if normalize else 0
        d.n_sub = n_sub
        d.step_balance = float(step_balance)
        d.tv = int(wl.tv)
        h = lib().or_create(C.byref(d))
        if not h:
            raise ValueError(lib().or_last_error().decode())
        self.h = h
        self._keep = None
        self.N = wl.H * wl.W

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().or_destroy(self.h)
                self.h = None
        except Exception:   # interpreter shutdown: module globals already cleared
            pass

    def run(self, iters: int):
        lib().or_run(self.h, int(iters))

    def monitor(self) -> dict:
        r = Report()
        lib().or_monitor(self.h, C.byref(r))
        return r.as_dict()

    def get_state(self) -> dict:
        n = lib().or_state_size(self.h)
        buf = np.empty(n, np.float64)
        lib().or_get_state(self.h, _p(buf))
        k, H, W = self.k, self.H, self.W
        kN = k * H * W
        out = {}
        for b, name in enumerate(STATE_ORDER[:-1]):
            out[name] = buf[b * kN:(b + 1) * kN].reshape(k, H, W).copy()
        out["qd"] = buf[8 * kN:].reshape(H, W).copy()
        return out

    def set_state(self, st: dict):
        parts = [_f64(st[n]).reshape(-1) for n in STATE_ORDER]
        buf = np.ascontiguousarray(np.concatenate(parts))
        assert buf.size == lib().or_state_size(self.h)
        lib().or_set_state(self.h, _p(buf))

    def read_u(self):
        ul = np.empty((self.k, self.H, self.W), np.float64)
        u = np.empty((self.H, self.W), np.float64)
        lib().or_read_u(self.h, _p(ul), _p(u))
        return ul, u

    def normalized(self):
        gam = np.empty(self.k + 1, np.float64)
        lam, sh, sc = C.c_double(), C.c_double(), C.c_double()
        lib().or_normalized(self.h, _p(gam), C.byref(lam), C.byref(sh), C.byref(sc))
        return gam, lam.value, sh.value, sc.value

    def apply_K(self, u, s):
        k, N = self.k, self.N
        u, s = _f64(u).reshape(-1), _f64(s).reshape(-1)
        Kv, Kpx, Kpy, Kz = (np.empty(k * N) for _ in range(4))
        Kq = np.empty(N)
        lib().or_apply_K(self.h, _p(u), _p(s), _p(Kv), _p(Kq), _p(Kpx), _p(Kpy), _p(Kz))
        return Kv, Kq, Kpx, Kpy, Kz

    def apply_KT(self, v, q, px, py, z):
        k, N = self.k, self.N
        v, q, px, py, z = (_f64(a).reshape(-1) for a in (v, q, px, py, z))
        Ku, Ks = np.empty(k * N), np.empty(k * N)
        lib().or_apply_KT(self.h, _p(v), _p(q), _p(px), _p(py), _p(z), _p(Ku), _p(Ks))
        return Ku, Ks

    def steps(self):
        k, N = self.k, self.N
        sp, sq = C.c_double(), C.c_double()
        svz, ts, tu = np.empty(k), np.empty(k), np.empty(N)
        lib().or_steps(self.h, C.byref(sp), _p(svz), C.byref(sq), _p(tu), _p(ts))
        return sp.value, svz, sq.value, tu, ts

    def residual_norms(self, before: dict, after: dict):
        """l1 norms (primal, dual) of the residuals between two consecutive states."""
        a = np.ascontiguousarray(np.concatenate([_f64(before[n]).reshape(-1) for n in STATE_ORDER]))
        b = np.ascontiguousarray(np.concatenate([_f64(after[n]).reshape(-1) for n in STATE_ORDER]))
        rp, rd = C.c_double(), C.c_double()
        lib().or_residual_norms(self.h, _p(a), _p(b), C.byref(rp), C.byref(rd))
        return rp.value, rd.value

    # ---- reverse pass
    def unrolled_forward(self, K: int):
        """Run K iterations from the current state, keeping every state for the reverse pass."""
        if lib().or_unrolled_forward(self.h, int(K)) != 0:
            raise ValueError(lib().or_last_error().decode())

    def unrolled_backward(self, gu):
        """Gradients (f [H,W], lambda, w [L,H,W] or None) of a function of the read-out u
        after the unrolled pass, given its adjoint gu [H,W] in original label units."""
        gu = _f64(gu).reshape(-1)
        gf = np.empty(self.N)
        gl = C.c_double()
        has_w = self.wl.tau is not None
        gw = np.empty((self.k + 1) * self.N) if has_w else None
        rc = lib().or_unrolled_backward(self.h, _p(gu), _p(gf), C.byref(gl),
                                        _p(gw) if has_w else None)
        if rc != 0:
            raise ValueError(lib().or_last_error().decode())
        return (gf.reshape(self.H, self.W), gl.value,
                gw.reshape(self.k + 1, self.H, self.W) if has_w else None)

    def step_vjp(self, state: dict, adj: dict):
        """Adjoint of one iteration at ``state`` (STATE_ORDER dict): the adjoint of the
        state before it, and the accumulated adjoints of the normalised data centre [H,W],
        the normalised lambda and the additive values [L,H,W] (or None)."""
        st = np.ascontiguousarray(np.concatenate([_f64(state[n]).reshape(-1) for n in STATE_ORDER]))
        ab = np.ascontiguousarray(np.concatenate([_f64(adj[n]).reshape(-1) for n in STATE_ORDER]))
        gc = np.zeros(self.N)
        gl = C.c_double(0.0)
        has_w = self.wl.tau is not None
        gw = np.zeros((self.k + 1) * self.N) if has_w else None
        if lib().or_step_vjp(self.h, _p(st), _p(ab), _p(gc), C.byref(gl), _p(gw) if has_w else None) != 0:
            raise ValueError(lib().or_last_error().decode())
        k, H, W = self.k, self.H, self.W
        kN = k * H * W
        out = {n: ab[b * kN:(b + 1) * kN].reshape(k, H, W).copy() for b, n in enumerate(STATE_ORDER[:-1])}
        out["qd"] = ab[8 * kN:].reshape(H, W).copy()
        return out, gc.reshape(H, W), gl.value, (gw.reshape(k + 1, H, W) if has_w else None)

    def piece(self, x: int, i: int):
        kind = C.c_int()
        acd = np.empty(3)
        n = C.c_int()
        t = np.empty(512)
        r = np.empty(512)
        lib().or_piece(self.h, x, i, C.byref(kind), _p(acd), C.byref(n), _p(t), _p(r))
        return kind.value, acd.copy(), t[:n.value].copy(), r[:n.value].copy()


def run_to_gap(prob: Problem, rel_gap: float, max_iters: int, check_every: int = 50):
    """Iterate until the certified relative gap drops below ``rel_gap``."""
    rep = None
    done = 0
    while done < max_iters:
        n = min(check_every, max_iters - done)
        prob.run(n)
        done += n
        rep = prob.monitor()
        if rep["rel_gap"] <= rel_gap:
            break
    return rep
