"""MI355X (gfx950) solver for the sublabel-accurate convex relaxation of
min_u sum_x rho(x, u(x)) + lambda TV(u) (Moellenhoff et al., CVPR 2016).

This module is a thin ctypes binding of ``libsublabel.so`` (C-ABI in
``include/sublabel.h``): it marshals arguments, allocates the workspace and the
input copies as torch device tensors, and passes torch's current HIP stream. Every step
of the iteration, the monitor and the read-out runs in the library's HIP kernels; if the
library is missing, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import ctypes as C_  # the same module; methods with a parameter named C use this name
import os
import re
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsublabel.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "sublabel.h")

RHO_QUAD, RHO_TRUNC_QUAD, RHO_SAMPLED, RHO_PERIODIC_QUAD = 0, 1, 2, 3
TV_ISO, TV_ANISO = 0, 1
STORE_FP32, STORE_BF16_DUAL = 0, 1

STATUS = {0: "SL_OK", 1: "SL_ERR_INVALID_ARG", 2: "SL_ERR_UNSUPPORTED", 3: "SL_ERR_DEVICE",
          4: "SL_ERR_WORKSPACE", 5: "SL_ERR_NUMERIC"}


class SublabelError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Desc(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("L", C.c_int32),
                ("gamma", C.POINTER(C.c_double)), ("rho", C.c_int32),
                ("f", C.c_void_p), ("a", C.c_double), ("nu", C.c_double),
                ("M", C.c_int32), ("tau", C.POINTER(C.c_double)), ("samples", C.c_void_p),
                ("lam", C.c_double), ("tv", C.c_int32), ("storage", C.c_int32),
                ("check_every", C.c_int32), ("normalize_labels", C.c_int32),
                ("adaptive_steps", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("primal_ub", C.c_double), ("dual_lb", C.c_double), ("gap", C.c_double),
                ("best_gap", C.c_double), ("rel_gap", C.c_double), ("e_nonconvex", C.c_double),
                ("iters", C.c_int64), ("best_primal", C.c_double), ("best_dual", C.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def declared_symbols():
    """Names of the functions declared in include/sublabel.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sl_[a-z_]+)\s*\(", txt)))


def lib():
    """Load libsublabel.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1512_01383_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, sz = C.c_void_p, C.c_size_t
        L.sl_status_string.restype = C.c_char_p
        L.sl_status_string.argtypes = [C.c_int]
        L.sl_last_error.restype = C.c_char_p
        L.sl_workspace_size.argtypes = [C.POINTER(Desc), C.POINTER(sz)]
        L.sl_create.argtypes = [C.POINTER(Desc), vp, sz, vp, C.POINTER(vp)]
        L.sl_run.argtypes = [vp, C.c_int32]
        L.sl_run_to_gap.argtypes = [vp, C.c_double, C.c_int32, C.POINTER(C.c_int32)]
        L.sl_read_u.argtypes = [vp, vp, vp]
        L.sl_energy.argtypes = [vp, C.POINTER(Report)]
        L.sl_state_size.argtypes = [vp, C.POINTER(sz)]
        L.sl_save_state.argtypes = [vp, vp, sz]
        L.sl_load_state.argtypes = [vp, vp, sz]
        L.sl_set_tiling.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
        L.sl_stereo_costs.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, vp, vp]
        L.sl_get_tiling.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.sl_batch_workspace_size.argtypes = [C.POINTER(Desc), C.c_int32, C.POINTER(sz)]
        L.sl_batch_create.argtypes = [C.POINTER(Desc), C.c_int32, vp, sz, vp, C.POINTER(vp)]
        L.sl_batch_energy.argtypes = [vp, C.c_int32, C.POINTER(Report)]
        L.sl_batch_read_u.argtypes = [vp, C.c_int32, vp, vp]
        L.sl_batch_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        L.sl_set_graphs.argtypes = [vp, C.c_int32]
        L.sl_autotune.argtypes = [vp, C.c_int32, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32)]
        L.sl_unrolled_workspace_size.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(sz)]
        L.sl_unrolled_forward.argtypes = [vp, C.c_int32, C.c_int32, vp, sz]
        L.sl_unrolled_backward.argtypes = [vp, vp, vp, C.POINTER(C.c_double), vp]
        L.sl_residuals.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.sl_set_balance_rule.argtypes = [vp, C.c_int32, C.c_double]
        L.sl_set_residual_target.argtypes = [vp, C.c_double]
        L.sl_set_step_balance.argtypes = [vp, C.c_double]
        L.sl_get_step_balance.argtypes = [vp, C.POINTER(C.c_double)]
        L.sl_set_storage.argtypes = [vp, C.c_int32, C.c_int32]
        L.sl_set_finishing.argtypes = [vp, C.c_int32, C.c_double, C.c_double]
        L.sl_storage_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.sl_temporal_workspace_size.argtypes = [vp, C.POINTER(sz)]
        L.sl_set_temporal.argtypes = [vp, vp, sz]
        L.sl_solve_static.argtypes = [C.POINTER(Desc), C.c_double, C.c_int32, vp, vp,
                                      C.POINTER(Report), vp]
        L.sl_destroy.argtypes = [vp]
        L.sl_destroy.restype = None
        for name in ("sl_workspace_size", "sl_create", "sl_run", "sl_run_to_gap", "sl_read_u",
                     "sl_energy", "sl_state_size", "sl_save_state", "sl_load_state",
                     "sl_set_tiling", "sl_get_tiling", "sl_batch_workspace_size", "sl_batch_create",
                     "sl_batch_energy", "sl_batch_read_u", "sl_batch_info", "sl_set_graphs",
                     "sl_autotune", "sl_unrolled_workspace_size", "sl_unrolled_forward",
                     "sl_unrolled_backward", "sl_set_step_balance", "sl_get_step_balance",
                     "sl_residuals", "sl_set_residual_target", "sl_solve_static",
                     "sl_set_storage", "sl_set_finishing", "sl_storage_info", "sl_set_balance_rule",
                     "sl_temporal_workspace_size", "sl_set_temporal"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise SublabelError(status, lib().sl_last_error().decode())


def _torch():
    import torch
    return torch


def _dev_f32(a, device):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)


def _make_desc(obj, H, W, gamma, rho, lam, f, a, nu, tau, samples, storage, normalize,
               check_every, device, adaptive=False, tv=TV_ISO):
    """Fill a Desc; device copies of the inputs are kept on ``obj._keep``."""
    obj.H, obj.W = int(H), int(W)
    obj.gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    obj.k = len(obj.gamma) - 1
    d = Desc()
    d.H, d.W, d.L = obj.H, obj.W, len(obj.gamma)
    d.gamma = obj.gamma.ctypes.data_as(C.POINTER(C.c_double))
    d.rho = int(rho)
    if f is not None:
        obj._keep["f"] = _dev_f32(f, device).reshape(-1)
        d.f = obj._keep["f"].data_ptr()
    d.a, d.nu = float(a), float(nu)
    if tau is not None:
        obj.tau = np.ascontiguousarray(tau, dtype=np.float64)
        obj._keep["samples"] = _dev_f32(samples, device).reshape(-1)
        d.M = len(obj.tau)
        d.tau = obj.tau.ctypes.data_as(C.POINTER(C.c_double))
        d.samples = obj._keep["samples"].data_ptr()
    obj.has_w = tau is not None and int(rho) != RHO_SAMPLED
    d.lam = float(lam)
    d.tv = int(tv)
    d.storage = {"fp32": STORE_FP32, "bf16": STORE_BF16_DUAL}[storage]
    d.check_every = int(check_every)
    d.normalize_labels = 1 if normalize else 0
    d.adaptive_steps = 1 if adaptive else 0
    return d


class _Inst:
    def __init__(self):
        self._keep = {}


class Problem:
    """One lifted problem on one GPU. Inputs may be numpy arrays or torch tensors."""

    def __init__(self, H: int, W: int, gamma, rho: int, lam: float, f=None, a: float = 1.0,
                 nu: float = 0.0, tau=None, samples=None, storage: str = "fp32",
                 normalize: bool = True, check_every: int = 50, device=None,
                 adaptive: bool = True, tv: int = TV_ISO):
        torch = _torch()
        self.device = torch.device(device if device is not None else "cuda:0")
        L_ = lib()
        self._keep = {}
        d = _make_desc(self, H, W, gamma, rho, lam, f, a, nu, tau, samples, storage, normalize,
                       check_every, self.device, adaptive, tv)
        self.desc = d
        nbytes = C.c_size_t()
        _check(L_.sl_workspace_size(C.byref(d), C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(L_.sl_create(C.byref(d), C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                            C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self._keep = None    # sl_create synchronised after reading the inputs

    @classmethod
    def from_workload(cls, wl, **kw):
        kw.setdefault("tv", getattr(wl, "tv", TV_ISO))
        return cls(wl.H, wl.W, wl.gamma, wl.rho, wl.lam, f=wl.f, a=wl.a, nu=wl.nu, tau=wl.tau,
                   samples=wl.samples, **kw)

    # ------------------------------------------------------------------ calls
    def run(self, iters: int):
        _check(lib().sl_run(self.h, int(iters)))

    def run_to_gap(self, rel_gap: float, max_iters: int) -> int:
        done = C.c_int32()
        _check(lib().sl_run_to_gap(self.h, float(rel_gap), int(max_iters), C.byref(done)))
        return done.value

    def read_u(self):
        torch = _torch()
        ul = torch.empty((self.k, self.H, self.W), dtype=torch.float32, device=self.device)
        u = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        _check(lib().sl_read_u(self.h, C.c_void_p(ul.data_ptr()), C.c_void_p(u.data_ptr())))
        return ul, u

    def energy(self) -> dict:
        r = Report()
        _check(lib().sl_energy(self.h, C.byref(r)))
        return r.as_dict()

    def state_size(self) -> int:
        n = C.c_size_t()
        _check(lib().sl_state_size(self.h, C.byref(n)))
        return n.value

    def save_state(self):
        torch = _torch()
        t = torch.empty(self.state_size() // 4, dtype=torch.float32, device=self.device)
        _check(lib().sl_save_state(self.h, C.c_void_p(t.data_ptr()), t.numel() * 4))
        return t

    def load_state(self, t):
        t = _dev_f32(t, self.device).reshape(-1)
        _check(lib().sl_load_state(self.h, C.c_void_p(t.data_ptr()), t.numel() * 4))
        self.stream.synchronize()

    # ---- unrolled differentiation
    def unrolled_forward(self, K: int, C: int):
        """Run K iterations with a checkpoint every C (workspace allocated here and kept
        until the next unrolled_forward or close)."""
        torch = _torch()
        n = C_.c_size_t()
        _check(lib().sl_unrolled_workspace_size(self.h, int(K), int(C), C_.byref(n)))
        self._uws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        _check(lib().sl_unrolled_forward(self.h, int(K), int(C), C_.c_void_p(self._uws.data_ptr()), n.value))

    def unrolled_backward(self, grad_u, want_f: bool = True, want_w: bool = True):
        """Gradients of a function of the read-out u after unrolled_forward, given its
        adjoint grad_u [H, W]: (grad_f [H, W] or None, grad_lambda, grad_w [L, H, W] or None)."""
        torch = _torch()
        gu = _dev_f32(grad_u, self.device).reshape(-1)
        gf = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device) if want_f else None
        gw = (torch.empty((self.k + 1, self.H, self.W), dtype=torch.float32, device=self.device)
              if (want_w and self.has_w) else None)
        gl = C_.c_double()
        _check(lib().sl_unrolled_backward(self.h, C_.c_void_p(gu.data_ptr()),
                                          C_.c_void_p(gf.data_ptr() if gf is not None else 0),
                                          C_.byref(gl),
                                          C_.c_void_p(gw.data_ptr() if gw is not None else 0)))
        return gf, gl.value, gw

    def residuals(self):
        """Run one iteration; return the l1 norms (primal, dual) of its residuals."""
        return self.residuals_full()[:2]

    def residuals_full(self):
        """Run one iteration; return (primal, dual, |K^T y|, |K x|), l1 norms."""
        rp, rd, ky, kx = C_.c_double(), C_.c_double(), C_.c_double(), C_.c_double()
        _check(lib().sl_residuals(self.h, C_.byref(rp), C_.byref(rd), C_.byref(ky), C_.byref(kx)))
        return rp.value, rd.value, ky.value, kx.value

    def set_balance_rule(self, scaled: bool, s: float):
        """Adaptive balance: raw residual norms (scaled=False) or residuals relative to
        |K^T y| and |K x| (scaled=True), compared with target ratio s."""
        _check(lib().sl_set_balance_rule(self.h, 1 if scaled else 0, float(s)))

    def set_temporal(self, on: bool = True):
        """Run groups of four iterations as two two-iteration passes (k <= 3, FP32,
        quadratic or truncated-quadratic data); the shadow workspace is allocated here and
        kept until set_temporal(False) or close."""
        if not on:
            _check(lib().sl_set_temporal(self.h, None, 0))
            self._band_ws = None
            return
        n = C.c_size_t()
        _check(lib().sl_temporal_workspace_size(self.h, C.byref(n)))
        torch = _torch()
        ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        _check(lib().sl_set_temporal(self.h, C.c_void_p(ws.data_ptr() + off), n.value))
        self._band_ws = ws

    def widen(self, i: int = -1):
        """Widen bf16 duals to float in place (problem i of a batch, -1: all)."""
        _check(lib().sl_set_storage(self.h, int(i), STORE_FP32))

    def set_finishing(self, stall_checks: int = 4, stall_progress: float = 0.1, widen_gap: float = 0.05):
        """run_to_gap widens bf16 duals after stall_checks checks in which the best gap did
        not shrink by the fraction stall_progress (0 checks: never on a stall), or once the
        certified relative gap is <= widen_gap (0: off)."""
        _check(lib().sl_set_finishing(self.h, int(stall_checks), float(stall_progress), float(widen_gap)))

    def storage_info(self, i: int = 0):
        """(storage now: 'fp32' or 'bf16', iterations run with bf16 duals) of problem i."""
        st, nb = C_.c_int32(), C_.c_int64()
        _check(lib().sl_storage_info(self.h, int(i), C_.byref(st), C_.byref(nb)))
        return ("bf16" if st.value == STORE_BF16_DUAL else "fp32"), nb.value

    def set_residual_target(self, s: float):
        """Target ratio of the adaptive balance (default 0.2, scaled rule)."""
        _check(lib().sl_set_residual_target(self.h, float(s)))

    def set_step_balance(self, c: float):
        """Scale the dual steps by c and the primal steps by 1/c (c = 1 by default)."""
        _check(lib().sl_set_step_balance(self.h, float(c)))

    def get_step_balance(self) -> float:
        c = C_.c_double()
        _check(lib().sl_get_step_balance(self.h, C_.byref(c)))
        return c.value

    def autotune(self, iters: int = 20, cache: Optional[str] = None):
        """Pick the fastest tiling (resets the iteration state); returns (groups, rows, cols)."""
        g, t, c = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().sl_autotune(self.h, int(iters), cache.encode() if cache else None,
                                 C.byref(g), C.byref(t), C.byref(c)))
        return g.value, t.value, c.value

    def set_tiling(self, label_groups: int, tile_rows: int, tile_cols: int = 64):
        """(0, 0, 0) restores the automatic choice; tile_cols 128 = two pixels per lane."""
        _check(lib().sl_set_tiling(self.h, int(label_groups), int(tile_rows), int(tile_cols)))

    def get_tiling(self):
        g, t, c = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().sl_get_tiling(self.h, C.byref(g), C.byref(t), C.byref(c)))
        return g.value, t.value, c.value

    def close(self):
        if getattr(self, "h", None):
            lib().sl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchProblem(Problem):
    """Many independent problems advanced together by one launch per
    iteration (sl_batch_create). ``instances`` are ``workloads.Workload``-like objects."""

    def __init__(self, instances, storage: str = "fp32", normalize: bool = True,
                 check_every: int = 48, device=None, adaptive: bool = True):
        torch = _torch()
        self.device = torch.device(device if device is not None else "cuda:0")
        L_ = lib()
        self._insts = []
        descs = (Desc * len(instances))()
        for j, wl in enumerate(instances):
            it = _Inst()
            descs[j] = _make_desc(it, wl.H, wl.W, wl.gamma, wl.rho, wl.lam, wl.f, wl.a, wl.nu,
                                  wl.tau, wl.samples, storage, normalize, check_every,
                                  self.device, adaptive, getattr(wl, "tv", TV_ISO))
            self._insts.append(it)
        self.n = len(instances)
        nbytes = C.c_size_t()
        _check(L_.sl_batch_workspace_size(descs, self.n, C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(L_.sl_batch_create(descs, self.n, C.c_void_p(self.workspace.data_ptr()),
                                  nbytes.value, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        for it in self._insts:
            it._keep = None

    def energy_of(self, i: int) -> dict:
        r = Report()
        _check(lib().sl_batch_energy(self.h, int(i), C.byref(r)))
        return r.as_dict()

    def read_u_of(self, i: int):
        torch = _torch()
        it = self._insts[i]
        ul = torch.empty((it.k, it.H, it.W), dtype=torch.float32, device=self.device)
        u = torch.empty((it.H, it.W), dtype=torch.float32, device=self.device)
        _check(lib().sl_batch_read_u(self.h, int(i), C.c_void_p(ul.data_ptr()),
                                     C.c_void_p(u.data_ptr())))
        return ul, u

    def info_of(self, i: int):
        n, a = C.c_int64(), C.c_int32()
        _check(lib().sl_batch_info(self.h, int(i), C.byref(n), C.byref(a)))
        return n.value, bool(a.value)

    def set_graphs(self, enable: bool):
        _check(lib().sl_set_graphs(self.h, 1 if enable else 0))


STATE_ORDER = ("u", "u_prev", "s", "s_prev", "v", "z", "px", "py", "qd")

# bytes of the library's fixed device array used by solve_static (SL_STATIC_WORKSPACE_BYTES)
STATIC_WORKSPACE_BYTES = 64 * 1024 * 1024


def solve_static(wl, rel_gap: float = 0.0, max_iters: int = 0, storage: str = "fp32",
                 normalize: bool = True, check_every: int = 50, adaptive: bool = False,
                 device=None, out=None):
    """Allocation-free solve (sl_solve_static) of a ``workloads.Workload``-like instance:
    the library keeps the iteration state in its own fixed device array, so the call itself
    allocates nothing. Runs to the certified gap ``rel_gap`` (> 0) within ``max_iters``
    iterations, or exactly ``max_iters`` iterations (``rel_gap`` = 0), on torch's current
    stream. ``out`` may give the (u_lifted [k,H,W], u [H,W]) float32 device tensors to write;
    they are allocated here otherwise. Returns (u_lifted, u, report dict)."""
    torch = _torch()
    dev = torch.device(device if device is not None else "cuda:0")
    it = _Inst()
    d = _make_desc(it, wl.H, wl.W, wl.gamma, wl.rho, wl.lam, wl.f, wl.a, wl.nu, wl.tau,
                   wl.samples, storage, normalize, check_every, dev, adaptive,
                   getattr(wl, "tv", TV_ISO))
    if out is None:
        out = (torch.empty((it.k, it.H, it.W), dtype=torch.float32, device=dev),
               torch.empty((it.H, it.W), dtype=torch.float32, device=dev))
    ul, u = out
    rep = Report()
    stream = torch.cuda.current_stream(dev)
    _check(lib().sl_solve_static(C.byref(d), float(rel_gap), int(max_iters),
                                 C.c_void_p(ul.data_ptr() if ul is not None else 0),
                                 C.c_void_p(u.data_ptr() if u is not None else 0),
                                 C.byref(rep), C.c_void_p(stream.cuda_stream)))
    return ul, u, rep.as_dict()


def stereo_costs(left, right, D: int, trunc: float, out=None, device=None):
    """Matching-cost volume [D][H][W] (float32, on the GPU) of a rectified pair: the
    truncated sum of absolute gradient differences over 4x4 patches (sl_stereo_costs), on
    torch's current stream."""
    torch = _torch()
    dev = torch.device(device if device is not None else "cuda:0")
    lt = _dev_f32(left, dev).contiguous()
    rt = _dev_f32(right, dev).contiguous()
    H, W = lt.shape
    if out is None:
        out = torch.empty((int(D), H, W), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    _check(lib().sl_stereo_costs(C.c_void_p(lt.data_ptr()), C.c_void_p(rt.data_ptr()), H, W, int(D),
                                 float(trunc), C.c_void_p(out.data_ptr()),
                                 C.c_void_p(stream.cuda_stream)))
    return out   # lt / rt may be released: the allocator orders their reuse on this stream


def unpack_state(t, k: int, H: int, W: int) -> dict:
    """Split a packed state vector into named [k][H][W] / [H][W] arrays (numpy)."""
    a = t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)
    kN = k * H * W
    out = {n: a[b * kN:(b + 1) * kN].reshape(k, H, W) for b, n in enumerate(STATE_ORDER[:-1])}
    out["qd"] = a[8 * kN:].reshape(H, W)
    return out


def pack_state(st: dict) -> np.ndarray:
    return np.concatenate([np.asarray(st[n], np.float32).reshape(-1) for n in STATE_ORDER])
