"""Pins for the smoothed, median-damped diagonal B_0 oracle (eq. 4; CPU only)."""
import numpy as np

from oracle import precond


def test_constant_field_is_unchanged_and_closed_form():
    nx, nz, npar = 13, 7, 3
    h = np.full(npar * nz * nx, 2.5)
    hs = precond.smooth(h, nx, nz, npar, 2.0, 5)
    np.testing.assert_allclose(hs, 2.5, rtol=1e-15)
    h0, _, lam = precond.precond_diag(h, nx, nz, npar, 2.0, 5, damping=0.5)
    assert lam == 1.25
    np.testing.assert_allclose(h0, np.float32(1.0 / 3.75), rtol=0)


def test_interior_impulse_is_the_outer_product_of_the_weights():
    nx, nz, half, sigma = 31, 29, 4, 1.5
    h = np.zeros((2, nz, nx))
    h[1, 14, 15] = 1.0
    hs = precond.smooth(h.ravel(), nx, nz, 2, sigma, half).reshape(2, nz, nx)
    t = np.arange(-half, half + 1)
    w = np.exp(-t * t / (2 * sigma * sigma))
    w /= w.sum()
    want = np.zeros((nz, nx))
    want[14 - half:14 + half + 1, 15 - half:15 + half + 1] = np.outer(w, w)
    np.testing.assert_allclose(hs[1], want, atol=1e-16)
    assert np.abs(hs[0]).max() == 0.0


def test_edge_renormalisation_by_hand():
    # 1 x 3 grid, half 1, sigma such that the side weight is exactly 1/2: the edge
    # points see two taps (weights 1 and 1/2), the middle three
    sigma = 1.0 / np.sqrt(2.0 * np.log(2.0))
    h = np.array([1.0, 4.0, 7.0])
    hs = precond.smooth(h, 3, 1, 1, sigma, 1)
    np.testing.assert_allclose(hs, [(1 + 0.5 * 4) / 1.5, (0.5 * 1 + 4 + 0.5 * 7) / 2.0, (0.5 * 4 + 7) / 1.5],
                               rtol=1e-15)


def test_median_damping_by_hand():
    # no smoothing effect with half = 0; n even: mean of the two middle values
    h = np.array([5.0, 1.0, 3.0, 9.0])
    h0, hs, lam = precond.precond_diag(h, 4, 1, 1, 1.0, 0, damping=2.0)
    assert lam == 2.0 * 4.0
    np.testing.assert_allclose(h0, np.float32(1.0 / (h + 8.0)), rtol=0)
    h0, hs, lam = precond.precond_diag(np.array([5.0, 1.0, 3.0]), 3, 1, 1, 1.0, 0)
    assert lam == 3.0
