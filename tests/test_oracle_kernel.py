"""Pins of the oracle's M4 smoothing kernel (paper Sect. 2.3, F_ij of Sect. 2.6).

The polynomial is pinned to scipy's cardinal cubic B-spline (the M4 kernel is
the B-spline of degree 3 on knots -2..2, rescaled so f(0)=1), the
normalisation to a quadrature of W over 3D space, and the two derivatives to
central finite differences.
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.interpolate import BSpline

import oracle

B3 = BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)


def bspline_w(r, h):
    q = np.asarray(r, dtype=float) / h
    b = np.nan_to_num(B3(q), nan=0.0)
    return 1.5 * b / (np.pi * h ** 3)  # B3(0) = 2/3, so 1.5*B3 has f(0) = 1


@pytest.mark.parametrize("h", [0.3, 1.0, 2.7])
def test_kernel_equals_cubic_bspline(h):
    r = np.linspace(0.0, 2.5 * h, 1001)
    w, _, _ = oracle.kernel_m4(r, h)
    np.testing.assert_allclose(w, bspline_w(r, h), rtol=1e-13, atol=1e-15 / h ** 3)
    assert np.all(w[r >= 2 * h] == 0.0)


@pytest.mark.parametrize("h", [0.05, 1.0, 3.0])
def test_kernel_normalised_in_3d(h):
    def integrand(r):
        return 4.0 * np.pi * r * r * oracle.kernel_m4(np.array([r]), h)[0][0]

    total = quad(integrand, 0.0, h, epsabs=0, epsrel=1e-13)[0] + \
        quad(integrand, h, 2.0 * h, epsabs=0, epsrel=1e-13)[0]
    assert abs(total - 1.0) < 1e-12


@pytest.mark.parametrize("h", [0.5, 1.3])
def test_radial_derivative_matches_fd(h):
    r = np.linspace(0.01 * h, 1.99 * h, 397)
    eps = 1e-6 * h
    _, F, _ = oracle.kernel_m4(r, h)
    wp, _, _ = oracle.kernel_m4(r + eps, h)
    wm, _, _ = oracle.kernel_m4(r - eps, h)
    fd = (wp - wm) / (2 * eps)
    np.testing.assert_allclose(F, fd, rtol=1e-7, atol=1e-8 / h ** 4)
    assert np.all(F <= 0.0)


@pytest.mark.parametrize("h", [0.5, 1.3])
def test_h_derivative_matches_fd(h):
    r = np.linspace(0.0, 2.2 * h, 401)
    eps = 1e-6 * h
    _, _, dh = oracle.kernel_m4(r, h)
    wp, _, _ = oracle.kernel_m4(r, np.full(r.shape, h + eps))
    wm, _, _ = oracle.kernel_m4(r, np.full(r.shape, h - eps))
    fd = (wp - wm) / (2 * eps)
    # skip points where the FD stencil straddles the q=2 cut-off
    ok = np.abs(r / h - 2.0) > 1e-4
    np.testing.assert_allclose(dh[ok], fd[ok], rtol=1e-7, atol=1e-8 / h ** 4)
