"""Pins of the oracle's stereo matching costs (Sec. 5.4: a truncated sum of absolute
gradient differences over a 4x4 patch). CPU only.

* a pair whose right image is the left one moved by d* columns: the cost at d* vanishes
  wherever the patch needs no clamping, and is positive at every other disparity, so the
  per-pixel minimum sits at d*;
* an affine image (constant gradient) matches itself at every disparity;
* identical images match at d = 0 everywhere (clamping included);
* truncation: no cost exceeds it, and with a large threshold the costs are the plain sums
  (checked against a threshold-free evaluation on a few pixels written from the
  definition).
"""
import numpy as np

import workloads as W


def _shifted_pair(seed, H, Wd, D, dstar):
    rng = np.random.default_rng(seed)
    tex = rng.uniform(0, 1, size=(H, Wd + 2 * D)).astype(np.float32)
    left = tex[:, D:D + Wd].copy()
    right = tex[:, D + dstar:D + dstar + Wd].copy()
    return left, right


def test_shifted_pair_matches_at_its_disparity(orc):
    H, Wd, D, dstar = 12, 40, 8, 5
    left, right = _shifted_pair(3, H, Wd, D, dstar)
    c = orc.stereo_costs(left, right, D, 1e9)
    # patch columns c-1 .. c+2 must satisfy p - d* >= 0 and p <= W-2; rows 1 .. H-3
    rows = slice(1, H - 2)
    cols = slice(dstar + 1, Wd - 3)
    assert np.all(c[dstar][rows, cols] == 0.0)
    others = np.delete(c[:, rows, cols], dstar, axis=0)
    assert np.all(others > 0.0)
    assert np.all(np.argmin(c[:, rows, cols], axis=0) == dstar)


def test_affine_image_matches_everywhere(orc):
    H, Wd, D = 9, 30, 6
    yy, xx = np.meshgrid(np.arange(H), np.arange(Wd), indexing="ij")
    img = (0.01 * xx + 0.02 * yy).astype(np.float32)
    c = orc.stereo_costs(img, img, D, 1e9)
    # gradients are constant wherever no forward difference meets the last row / column
    assert np.all(np.abs(c[:, 1:H - 3, D + 1:Wd - 3]) <= 1e-6)


def test_identical_images_match_at_zero(orc):
    rng = np.random.default_rng(4)
    img = rng.uniform(0, 1, size=(7, 11)).astype(np.float32)
    c = orc.stereo_costs(img, img, 4, 1e9)
    assert np.all(c[0] == 0.0)


def test_truncation_and_plain_sums(orc):
    wl = W.stereo(H=24, W=40, n_disp=10, L=4)
    left, right = wl.pair
    c_inf = orc.stereo_costs(left, right, 10, 1e9)
    T = float(np.median(c_inf))
    c_t = orc.stereo_costs(left, right, 10, T)
    assert np.all(c_t <= T) and np.array_equal(c_t, np.minimum(c_inf, T))
    # a few pixels from the definition, with explicit clamping
    L64, R64 = left.astype(np.float64), right.astype(np.float64)
    H, Wd = L64.shape

    def grads(im):
        gx = np.zeros_like(im)
        gy = np.zeros_like(im)
        gx[:, :-1] = im[:, 1:] - im[:, :-1]
        gy[:-1, :] = im[1:, :] - im[:-1, :]
        return gx, gy

    lx, ly = grads(L64)
    rx, ry = grads(R64)
    rng = np.random.default_rng(5)
    for _ in range(40):
        r, cc, d = int(rng.integers(H)), int(rng.integers(Wd)), int(rng.integers(10))
        acc = 0.0
        for i in (-1, 0, 1, 2):
            for j in (-1, 0, 1, 2):
                pr, pc = min(max(r + i, 0), H - 1), min(max(cc + j, 0), Wd - 1)
                qc = max(pc - d, 0)
                acc += abs(lx[pr, pc] - rx[pr, qc]) + abs(ly[pr, pc] - ry[pr, qc])
        assert c_inf[d, r, cc] == acc


def test_cost_minimum_tracks_the_generating_disparity(orc):
    """On the synthetic pair (right image warped by a known disparity map) the per-pixel
    cost minimum lies within 2 of the true disparity far more often than chance (5/64)."""
    wl = W.stereo()
    left, right = wl.pair
    c = orc.stereo_costs(left, right, 64, 1.0)
    hit = np.abs(np.argmin(c, axis=0) - wl.target) <= 2.0
    assert hit.mean() > 0.4
