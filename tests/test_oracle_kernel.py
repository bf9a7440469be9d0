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


# ---- M6 quintic spline and Wendland C6 (the other kernels of Sect. 2.3) ----
#
# M6 is pinned to scipy's cardinal quintic B-spline on knots -3..3 (f = 120 B5,
# so f(0) = 66), the Wendland C6 function to its construction by the
# dimension walk: for three dimensions and smoothness k = 3 it is I^3 applied
# to (1 - x)^5 with (I g)(x) = integral_x^1 t g(t) dt, normalised to 1 at
# x = 0 (x = r / H, compact support H = 2h).  Normalisations and derivatives
# as for M4.

B5 = BSpline.basis_element([-3.0, -2.0, -1.0, 0.0, 1.0, 2.0, 3.0], extrapolate=False)
KINDS = [oracle.M4, oracle.M6, oracle.WENDLAND_C6]


def wendland_c6_by_dimension_walk(x):
    P = np.polynomial.Polynomial
    g = P([1.0, -1.0]) ** 5  # (1 - t)^5
    t = P([0.0, 1.0])
    for _ in range(3):
        anti = (t * g).integ()  # antiderivative of t g(t)
        g = anti(1.0) - anti  # integral from x to 1
    return g(x) / g(0.0)


def test_support_radii():
    assert oracle.kernel_support(oracle.M4) == 2.0
    assert oracle.kernel_support(oracle.M6) == 3.0
    assert oracle.kernel_support(oracle.WENDLAND_C6) == 2.0


@pytest.mark.parametrize("h", [0.4, 1.0, 2.2])
def test_m6_equals_quintic_bspline(h):
    r = np.linspace(0.0, 3.5 * h, 1401)
    w, _, _ = oracle.kernel(oracle.M6, r, h)
    q = r / h
    expect = 120.0 * np.nan_to_num(B5(q), nan=0.0) / (120.0 * np.pi * h ** 3)
    np.testing.assert_allclose(w, expect, rtol=1e-12, atol=1e-15 / h ** 3)
    assert np.all(w[r >= 3 * h] == 0.0)


@pytest.mark.parametrize("h", [0.4, 1.0, 2.2])
def test_wendland_c6_equals_dimension_walk(h):
    r = np.linspace(0.0, 2.5 * h, 1251)
    w, _, _ = oracle.kernel(oracle.WENDLAND_C6, r, h)
    x = np.minimum(r / (2.0 * h), 1.0)
    w0 = oracle.kernel(oracle.WENDLAND_C6, np.array([0.0]), h)[0][0]
    # the walk's degree-11 monomial form loses ~1e-12 of W(0) to cancellation
    np.testing.assert_allclose(w, w0 * wendland_c6_by_dimension_walk(x), rtol=1e-11,
                               atol=1e-11 * w0)
    assert np.all(w[r >= 2 * h] == 0.0)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("h", [0.05, 1.0, 3.0])
def test_kernels_normalised_in_3d(kind, h):
    S = oracle.kernel_support(kind)

    def integrand(r):
        return 4.0 * np.pi * r * r * oracle.kernel(kind, np.array([r]), h)[0][0]

    edges = [0.0] + [k * h for k in range(1, int(S) + 1)]
    total = sum(quad(integrand, a, b, epsabs=0, epsrel=1e-13)[0]
                for a, b in zip(edges[:-1], edges[1:]))
    assert abs(total - 1.0) < 1e-12


@pytest.mark.parametrize("kind", KINDS)
def test_kernel_derivatives_match_fd(kind):
    h = 0.9
    S = oracle.kernel_support(kind)
    r = np.linspace(0.01 * h, (S - 0.01) * h, 600)
    eps = 1e-6 * h
    w, F, dh = oracle.kernel(kind, r, h)
    fd_r = (oracle.kernel(kind, r + eps, h)[0] - oracle.kernel(kind, r - eps, h)[0]) / (2 * eps)
    np.testing.assert_allclose(F, fd_r, rtol=1e-7, atol=1e-8 / h ** 4)
    fd_h = (oracle.kernel(kind, r, np.full(r.shape, h + eps))[0] -
            oracle.kernel(kind, r, np.full(r.shape, h - eps))[0]) / (2 * eps)
    np.testing.assert_allclose(dh, fd_h, rtol=1e-7, atol=1e-8 / h ** 4)
    assert np.all(F <= 0.0) and np.all(w >= 0.0)


@pytest.mark.parametrize("kind", [oracle.M6, oracle.WENDLAND_C6])
def test_kernels_smooth_at_breakpoints(kind):
    """f and f' are continuous across the pieces and vanish at the support."""
    h = 1.0
    S = oracle.kernel_support(kind)
    for q0 in [1.0, 2.0, S]:
        if q0 > S:
            continue
        lo, hi = np.array([q0 - 1e-9]), np.array([q0 + 1e-9])
        wl, Fl, _ = oracle.kernel(kind, lo, h)
        wr, Fr, _ = oracle.kernel(kind, hi, h)
        assert abs(wl[0] - wr[0]) < 1e-8 and abs(Fl[0] - Fr[0]) < 1e-7
    w, F, _ = oracle.kernel(kind, np.array([S * h * (1 - 1e-6)]), h)
    assert abs(w[0]) < 1e-20 and abs(F[0]) < 1e-15
