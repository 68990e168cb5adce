"""The seeded input generators (CPU): shapes, ranges and the data they promise, so that a
change in them cannot pass unnoticed through both the oracle and the HIP path."""
import numpy as np
import pytest

import workloads as W


def test_baseline_lifting_samples_rho_at_the_labels():
    tq = W.truncated_quadratic(L=6, H=9, W=11, seed=3)
    b = W.baseline_lifting(tq)
    assert b.rho == W.SAMPLED and np.array_equal(b.tau, tq.gamma) and b.samples.shape == (6, 9, 11)
    f = tq.f.astype(np.float64)
    for j, g in enumerate(tq.gamma):
        want = np.minimum(0.5 * tq.a * (g - f) ** 2, tq.nu)
        assert np.allclose(b.samples[j], want, rtol=1e-6, atol=1e-7)


def test_baseline_lifting_of_phase_uses_circular_distance():
    ph = W.phase_unwrapping(H=7, W=8, L=5)
    b = W.baseline_lifting(ph)
    f = ph.f.astype(np.float64)
    for j, g in enumerate(ph.gamma):
        d = np.abs(np.angle(np.exp(1j * (g - f))))        # distance on the circle
        assert np.allclose(b.samples[j], 0.5 * ph.a * d ** 2, rtol=1e-5, atol=1e-6)


def test_phase_workload_ranges():
    ph = W.phase_unwrapping(H=32, W=40, L=8)
    assert ph.rho == W.PERIODIC_QUAD and ph.nu == 2 * np.pi and ph.a == 2.0
    assert np.isclose(ph.gamma[0], 0.0) and np.isclose(ph.gamma[-1], 4 * np.pi) and len(ph.gamma) == 8
    assert ph.f.min() >= 0.0 and ph.f.max() < 2 * np.pi
    assert ph.target.min() >= 0.3 * np.pi - 1e-5 and ph.target.max() <= 3.7 * np.pi + 1e-5
    # the observation is the generating phase wrapped, up to the added noise
    d = np.abs(np.angle(np.exp(1j * (ph.f.astype(np.float64) - ph.target))))
    assert np.mean(d) < 0.5


def test_stereo_pair_and_costs_consistent():
    st = W.stereo(H=20, W=48, n_disp=12, L=4)
    left, right = st.pair
    assert left.shape == right.shape == (20, 48) and st.samples.shape == (12, 20, 48)
    # the stored absolute-difference costs are those of the stored pair
    cols = np.arange(48)
    for d in (0, 5, 11):
        want = np.abs(left - right[:, np.maximum(cols - d, 0)])
        assert np.allclose(st.samples[d], want, atol=1e-6)


def test_rectangles_need_room():
    """The rectangle generator draws sides of at least 4 px: on a smaller image it raises
    instead of drawing forever."""
    with pytest.raises(ValueError):
        W.rof(H=2, W=3)
    assert W.rof(H=5, W=5).f.shape == (5, 5)
