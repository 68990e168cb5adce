"""Seeded synthetic inputs shared by the oracle tests, the HIP parity tests and the
benchmark.

This module only draws and shapes input data (images, cost volumes, label sets and
model parameters). It contains none of the solver's arithmetic, so both the CPU
oracle and the HIP path can consume it without sharing any code of the method.

The paper's own inputs (the ROF / truncated-quadratic test images, Middlebury stereo
pairs, SAR phase data, the focal stack) are not available, so every workload below is
a synthetic stand-in with the shape and value distribution of the corresponding
experiment (Sec. 5.1 ROF model, Sec. 5.2 robust truncated quadratic, Sec. 5.4 stereo,
Sec. 5.5 phase unwrapping).
All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

QUAD = 0
TRUNC_QUAD = 1
SAMPLED = 2
PERIODIC_QUAD = 3       # a/2 d(t, f)^2, d the distance on a circle of circumference nu


@dataclasses.dataclass
class Workload:
    """One problem instance of the energy  sum_x rho(x, u(x)) + lambda TV(u)  (eq. 1).

    rho kinds: QUAD      rho = a/2 (t - f)^2
               TRUNC_QUAD rho = min(a/2 (t - f)^2, nu)
               SAMPLED   rho given by ``samples[m]`` at positions ``tau[m]``
    For QUAD / TRUNC_QUAD, ``samples`` (shape [L][H][W], ``tau == gamma``) optionally
    holds per-label additive values w that are interpolated linearly between labels.
    """

    name: str
    H: int
    W: int
    gamma: np.ndarray                   # [L] float64, strictly increasing
    rho: int
    lam: float
    f: Optional[np.ndarray] = None      # [H][W] float32
    a: float = 1.0
    nu: float = 0.0
    tau: Optional[np.ndarray] = None    # [M] float64
    samples: Optional[np.ndarray] = None  # [M][H][W] float32
    iters: int = 0                      # fixed iteration count of the workload (0: run to gap)
    target: Optional[np.ndarray] = None  # clean image (differentiation workload)
    tv: int = 0                         # 0: isotropic TV (l2), 1: anisotropic TV (l1)
    pair: Optional[tuple] = None        # (left, right) [H][W] float32 images (stereo)

    @property
    def L(self) -> int:
        return int(self.gamma.shape[0])

    @property
    def k(self) -> int:
        return self.L - 1

    @property
    def M(self) -> int:
        return 0 if self.tau is None else int(self.tau.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def rectangles_image(rng: np.random.Generator, H: int, W: int, n_rect: int = 8,
                     noise: float = 0.1) -> np.ndarray:
    """Background 0, ``n_rect`` axis-aligned rectangles (sides >= 4 px) with
    intensities U[0,1], later ones overwriting earlier ones, plus N(0, noise^2).
    No clipping. Needs H, W >= 5 (a rectangle of side >= 4 spans 5 pixels)."""
    if H < 5 or W < 5:
        raise ValueError(f"rectangles of side >= 4 px need an image of at least 5 x 5 pixels, not {H} x {W}")
    img = np.zeros((H, W), np.float64)
    for _ in range(n_rect):
        while True:
            r0, r1 = sorted(rng.integers(0, H, size=2))
            c0, c1 = sorted(rng.integers(0, W, size=2))
            if r1 - r0 >= 4 and c1 - c0 >= 4:
                break
        img[r0:r1 + 1, c0:c1 + 1] = rng.uniform(0.0, 1.0)
    img += rng.normal(0.0, noise, size=(H, W))
    return img.astype(np.float32)


def blobs_image(rng: np.random.Generator, H: int, W: int, n_blobs: int = 12,
                sigma_scale: float = 1.0) -> np.ndarray:
    """Min-max normalised sum of Gaussian blobs: centres U[0,W)xU[0,H),
    sigma U[12,48]*sigma_scale px, amplitude U[-1,1]."""
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    g = np.zeros((H, W), np.float64)
    for _ in range(n_blobs):
        cy = rng.uniform(0, H)
        cx = rng.uniform(0, W)
        sig = rng.uniform(12.0, 48.0) * sigma_scale
        amp = rng.uniform(-1.0, 1.0)
        g += amp * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2.0 * sig * sig))
    lo, hi = g.min(), g.max()
    g = (g - lo) / (hi - lo) if hi > lo else np.zeros_like(g)
    return g


def with_outliers(rng: np.random.Generator, g: np.ndarray, frac: float = 0.1) -> np.ndarray:
    """Replace ``frac`` of the pixels (drawn without replacement) by U[0,1]."""
    f = g.copy().reshape(-1)
    n = int(round(frac * f.size))
    idx = rng.choice(f.size, size=n, replace=False)
    f[idx] = rng.uniform(0.0, 1.0, size=n)
    return f.reshape(g.shape).astype(np.float32)


def equispaced(L: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return np.linspace(lo, hi, L, dtype=np.float64)


# ----------------------------------------------------------------------------------
# Named workloads (shapes and parameters of the paper's experiments, synthetic data)
# ----------------------------------------------------------------------------------

def rof(seed: int = 1, H: int = 64, W: int = 64, lam: float = 0.2,
        iters: int = 2000) -> Workload:
    """Convex ROF (Sec. 5.1): rho = 1/2 (t - f)^2 on Gamma = [0,1], L = 2."""
    rng = _rng(seed)
    f = rectangles_image(rng, H, W)
    return Workload("rof64", H, W, equispaced(2), QUAD, lam, f=f, a=1.0, iters=iters)


def truncated_quadratic(L: int = 10, seed: int = 2, H: int = 256, W: int = 256,
                        lam: float = 0.25, sigma_scale: float = 1.0) -> Workload:
    """Robust truncated quadratic denoising (Sec. 5.2): rho = min((t - f)^2, 0.025),
    i.e. a = 2, nu = 0.025, L equispaced labels on [0,1]."""
    rng = _rng(seed)
    g = blobs_image(rng, H, W, sigma_scale=sigma_scale)
    f = with_outliers(rng, g)
    w = Workload(f"tq{H}x{W}_L{L}", H, W, equispaced(L), TRUNC_QUAD, lam, f=f, a=2.0,
                 nu=0.025)
    w.target = g.astype(np.float32)
    return w


def _box_blur3(img: np.ndarray) -> np.ndarray:
    p = np.pad(img, 1, mode="edge")
    out = np.zeros_like(img)
    for dy in range(3):
        for dx in range(3):
            out += p[dy:dy + img.shape[0], dx:dx + img.shape[1]]
    return out / 9.0


def stereo(seed: int = 3, H: int = 288, W: int = 384, n_disp: int = 64, L: int = 8,
           lam: float = 0.5, iters: int = 1000, n_regions: int = 6) -> Workload:
    """Sampled-cost lifting (Sec. 5.4 stand-in): random-texture left image, right image
    warped by a piecewise-planar disparity map in [0, n_disp-1], absolute-difference
    costs at the integer disparities 0..n_disp-1, labels gamma_j = step*(j-1)."""
    rng = _rng(seed)
    left = _box_blur3(rng.uniform(0.0, 1.0, size=(H, W)))
    left = (left - left.min()) / (left.max() - left.min())
    # piecewise-planar disparity over Voronoi regions
    cy = rng.uniform(0, H, size=n_regions)
    cx = rng.uniform(0, W, size=n_regions)
    pa = rng.uniform(5.0, 58.0, size=n_regions)
    pb = rng.uniform(-0.05, 0.05, size=n_regions)
    pc = rng.uniform(-0.05, 0.05, size=n_regions)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    reg = np.argmin((yy[None] - cy[:, None, None]) ** 2 + (xx[None] - cx[:, None, None]) ** 2,
                    axis=0)
    disp = np.clip(pa[reg] + pb[reg] * xx + pc[reg] * yy, 0.0, n_disp - 1.0)
    # right image: I_R(x, y) = I_L(min(x + D(x, y), W - 1), y), linear interpolation
    xs = np.minimum(xx + disp, W - 1.0)
    x0 = np.floor(xs).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    fr = xs - x0
    rows = np.arange(H)[:, None]
    right = (1.0 - fr) * left[rows, x0] + fr * left[rows, x1]
    cost = np.empty((n_disp, H, W), np.float32)
    cols = np.arange(W)
    for d in range(n_disp):
        xr = np.maximum(cols - d, 0)
        cost[d] = np.abs(left - right[:, xr]).astype(np.float32)
    step = (n_disp - 1) / (L - 1)
    gamma = step * np.arange(L, dtype=np.float64)
    tau = np.arange(n_disp, dtype=np.float64)
    w = Workload(f"stereo{H}x{W}_L{L}", H, W, gamma, SAMPLED, lam, tau=tau, samples=cost,
                 iters=iters)
    w.target = disp.astype(np.float32)
    w.pair = (left.astype(np.float32), right.astype(np.float32))
    return w


def batch(seed0: int = 400, n: int = 64, lam: float = 0.25,
          sizes=(64, 128, 256, 512), labels=(2, 4, 8, 16)) -> List[Workload]:
    """Batched workload: instance j has S ~ U(sizes), L ~ U(labels), truncated-quadratic
    data as in the denoising workload with blob sigma scaled by S/256."""
    out = []
    for j in range(n):
        rng = _rng(seed0 + j)
        S = int(rng.choice(np.asarray(sizes)))
        L = int(rng.choice(np.asarray(labels)))
        g = blobs_image(rng, S, S, sigma_scale=S / 256.0)
        f = with_outliers(rng, g)
        w = Workload(f"batch{j}_S{S}_L{L}", S, S, equispaced(L), TRUNC_QUAD, lam, f=f,
                     a=2.0, nu=0.025)
        w.target = g.astype(np.float32)
        out.append(w)
    return out


def differentiation(seed: int = 5, H: int = 256, W: int = 256, L: int = 8,
                    lam: float = 0.25, K: int = 200) -> Workload:
    """Differentiation workload: truncated-quadratic instance with per-label additive
    data-term values w (zero in the forward instance) and a clean target image."""
    w = truncated_quadratic(L=L, seed=seed, H=H, W=W, lam=lam)
    w.name = f"diff{H}x{W}_L{L}"
    w.tau = w.gamma.copy()
    w.samples = np.zeros((L, H, W), np.float32)
    w.iters = K
    return w


def roofline(seed: int = 6, H: int = 2048, W: int = 2048, L: int = 16,
             lam: float = 0.25) -> Workload:
    """Large truncated-quadratic instance whose working set is far beyond the on-chip
    caches (bandwidth measurement)."""
    w = truncated_quadratic(L=L, seed=seed, H=H, W=W, lam=lam)
    w.name = f"tq{H}x{W}_L{L}"
    return w


def phase_unwrapping(seed: int = 7, H: int = 256, W: int = 256, L: int = 8,
                     lam: float = 0.005, noise: float = 0.3) -> Workload:
    """Phase unwrapping (Sec. 5.5 stand-in for the SAR data): a smooth phase surface in
    [0.3 pi, 3.7 pi] (blobs image rescaled), observed wrapped to [0, 2 pi) after adding
    N(0, noise^2); rho = d(t, f)^2 on the circle of circumference 2 pi (a = 2, nu = 2 pi),
    labels equispaced on Gamma = [0, 4 pi], lambda = 0.005 as in the paper."""
    rng = _rng(seed)
    g = blobs_image(rng, H, W)
    phase = np.pi * (0.3 + 3.4 * g)
    f = np.mod(phase + rng.normal(0.0, noise, size=(H, W)), 2.0 * np.pi)
    w = Workload(f"phase{H}x{W}_L{L}", H, W, equispaced(L, 0.0, 4.0 * np.pi), PERIODIC_QUAD, lam,
                 f=f.astype(np.float32), a=2.0, nu=2.0 * np.pi)
    w.target = phase.astype(np.float32)
    return w


def baseline_lifting(wl: Workload) -> Workload:
    """The comparison method of Sec. 5 as a special case (Prop. 2): the data term of a
    quadratic, truncated-quadratic or periodic workload given only at its labels (samples
    at tau == gamma), so every interval's convex piece is the chord between its end
    labels."""
    f = wl.f.astype(np.float64)
    dist = wl.gamma[:, None, None] - f[None]
    if wl.rho == PERIODIC_QUAD:   # distance on the circle of circumference nu
        dist = np.abs(np.mod(dist + 0.5 * wl.nu, wl.nu) - 0.5 * wl.nu)
    rho = 0.5 * wl.a * dist ** 2
    if wl.rho == TRUNC_QUAD:
        rho = np.minimum(rho, wl.nu)
    return Workload(wl.name + "_baseline", wl.H, wl.W, wl.gamma.copy(), SAMPLED, wl.lam,
                    tau=wl.gamma.copy(), samples=rho.astype(np.float32), tv=wl.tv)


def random_state(seed: int, k: int, H: int, W: int, scale: float = 1.0) -> dict:
    """Random iteration state (float32) for single-step parity tests. Plane order and
    shapes follow the documented state layout: u, u_prev, s, s_prev, v, z: [k][H][W];
    px, py: [k][H][W]; qd: [H][W]."""
    rng = _rng(seed)
    st = {}
    st["u"] = rng.uniform(-0.2, 1.2, size=(k, H, W))
    st["u_prev"] = st["u"] + rng.normal(0, 0.05, size=(k, H, W))
    st["s"] = rng.normal(0, 0.5, size=(k, H, W)) * scale
    st["s_prev"] = st["s"] + rng.normal(0, 0.05, size=(k, H, W))
    st["v"] = rng.normal(0, 1.0, size=(k, H, W)) * scale
    st["z"] = rng.normal(0, 1.0, size=(k, H, W)) * scale
    st["px"] = rng.normal(0, 0.3, size=(k, H, W)) * scale
    st["py"] = rng.normal(0, 0.3, size=(k, H, W)) * scale
    st["qd"] = rng.normal(0, 1.0, size=(H, W)) * scale
    return {n: a.astype(np.float32) for n, a in st.items()}


STATE_ORDER = ("u", "u_prev", "s", "s_prev", "v", "z", "px", "py", "qd")
