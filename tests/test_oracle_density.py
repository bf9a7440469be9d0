"""Pins of the oracle's density / smoothing-length solve (Sect. 2.2, Sect. 3.2.1).

The oracle's root h* is checked against quantities computed here by other
means: the kernel is scipy's cubic B-spline, neighbour sums run over scipy's
periodic k-d tree or an explicit infinite-lattice sum, roots come from
brentq, and Omega from a finite difference of the density sum in h.
"""
import numpy as np
import pytest
from scipy.interpolate import BSpline
from scipy.optimize import brentq
from scipy.spatial import cKDTree

import oracle
from paper_1909_07439_amd import inputs

B3 = BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)


def w_ref(r, h):
    return 1.5 * np.nan_to_num(B3(np.asarray(r) / h), nan=0.0) / (np.pi * h ** 3)


def lattice_sum(h, dx, m, reach=4):
    g = np.arange(-reach, reach + 1)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    r = dx * np.sqrt(I ** 2 + J ** 2 + K ** 2).ravel()
    return m * w_ref(r, h).sum(), r


def test_perfect_lattice_matches_infinite_lattice_root():
    c = inputs.lattice(16, jitter=0.0)
    dx, m, hf = c["dx"], c["m"][0], c["hfact"]
    f = lambda h: lattice_sum(h, dx, m)[0] - m * (hf / h) ** 3
    hs = brentq(f, 0.8 * dx, 1.6 * dx, xtol=1e-16, rtol=1e-15)
    rho = lattice_sum(hs, dx, m)[0]
    d = 1e-6 * hs
    dS = (lattice_sum(hs + d, dx, m)[0] - lattice_sum(hs - d, dx, m)[0]) / (2 * d)
    omega = 1.0 + hs * dS / (3.0 * rho)
    nn = int(np.sum(lattice_sum(hs, dx, m)[1] < 2 * hs))
    o = oracle.density(c["x"], c["y"], c["z"], c["m"], c["h"], oracle.make_params(c))
    np.testing.assert_allclose(o["h"], hs, rtol=1e-12)
    np.testing.assert_allclose(o["rho"], rho, rtol=1e-12)
    np.testing.assert_allclose(o["omega"], omega, rtol=1e-8)
    assert np.all(o["nneigh"] == nn) and nn == 57
    # the M4 lattice-sum bias: uniform lattice density is rho0 to within 1e-3
    assert abs(o["rho"].mean() - 1.0) < 1e-3
    assert o["rho"].std() < 1e-14


@pytest.mark.parametrize("jitter", [0.05, 0.3])
def test_jittered_root_and_omega_by_kdtree_sums(jitter):
    c = inputs.lattice(16, jitter=jitter)
    p = oracle.make_params(c)
    o = oracle.density(c["x"], c["y"], c["z"], c["m"], c["h"], p)
    pts = np.stack([c["x"], c["y"], c["z"]], 1)
    kd = cKDTree(pts, boxsize=1.0)

    def S0(i, h):
        nb = np.array(kd.query_ball_point(pts[i], 2.2 * h))
        d = np.linalg.norm(((pts[nb] - pts[i] + 0.5) % 1.0) - 0.5, axis=1)
        return np.sum(c["m"][nb] * w_ref(d, h))

    for i in range(0, c["n"], 97):
        h = o["h"][i]
        s0 = S0(i, h)
        target = c["m"][i] * (c["hfact"] / h) ** 3
        assert abs(s0 - target) <= 1e-12 * target
        assert abs(o["rho"][i] - s0) <= 1e-13 * s0
        d = 1e-6 * h
        om = 1.0 + h * (S0(i, h + d) - S0(i, h - d)) / (2 * d) / (3.0 * s0)
        assert abs(o["omega"][i] - om) < 1e-7


@pytest.mark.parametrize("scale", [0.55, 1.0, 1.7])
def test_root_independent_of_starting_h(scale):
    """NR from far-off starts (forcing the bracketing fallback) reaches the same root."""
    c = inputs.lattice(12, jitter=0.2)
    p = oracle.make_params(c)
    ref = oracle.density(c["x"], c["y"], c["z"], c["m"], c["h"], p)
    o = oracle.density(c["x"], c["y"], c["z"], c["m"], c["h"] * scale, p)
    np.testing.assert_allclose(o["h"], ref["h"], rtol=1e-12)
    np.testing.assert_allclose(o["rho"], ref["rho"], rtol=1e-12)


def test_sod_interiors_keep_lattice_ratio():
    """Both Sod states are perfect lattices: far from the interfaces each has
    the same lattice-sum bias, so rho/rho0 is identical on both sides."""
    c = inputs.sod(dx_left=1.0 / 64, width=0.25)
    p = oracle.make_params(c)
    o = oracle.density(c["x"], c["y"], c["z"], c["m"], c["h"], p)
    x = c["x"]
    left = (x > -0.4) & (x < -0.1)
    right = (x > 0.1) & (x < 0.4)
    rl = o["rho"][left] / 1.0
    rr = o["rho"][right] / 0.125
    np.testing.assert_allclose(rl, rl[0], rtol=1e-12)
    np.testing.assert_allclose(rr, rl[0], rtol=1e-12)
    np.testing.assert_allclose(o["h"][right], 2 * o["h"][left][0], rtol=1e-12)


# ---- the other kernels of Sect. 2.3 on a perfect lattice ----
B5 = BSpline.basis_element([-3.0, -2.0, -1.0, 0.0, 1.0, 2.0, 3.0], extrapolate=False)


def w_m6(r, h):
    return np.nan_to_num(B5(np.asarray(r) / h), nan=0.0) / (np.pi * h ** 3)  # 120 B5 / (120 pi)


def w_wc6(r, h):
    """Wendland C6 (3D, k = 3) built by the dimension walk I^3 (1 - x)^5 on
    x = r / (2h), normalised here by a radial quadrature."""
    P = np.polynomial.Polynomial
    g, t = P([1.0, -1.0]) ** 5, P([0.0, 1.0])
    for _ in range(3):
        a = (t * g).integ()
        g = a(1.0) - a
    xs = np.linspace(0.0, 1.0, 200001)
    norm = 1.0 / np.trapezoid(4.0 * np.pi * (2.0 * xs) ** 2 * g(xs), 2.0 * xs)
    x = np.minimum(np.asarray(r) / (2.0 * h), 1.0)
    return norm * g(x) / h ** 3


@pytest.mark.parametrize("kind,wfun,nn_expect", [(oracle.M6, w_m6, 112),
                                                 (oracle.WENDLAND_C6, w_wc6, 136)])
def test_perfect_lattice_root_other_kernels(kind, wfun, nn_expect):
    c = inputs.with_kernel(inputs.lattice(16, jitter=0.0), kind)
    dx, m, hf = c["dx"], c["m"][0], c["hfact"]
    S = oracle.kernel_support(kind)
    g = np.arange(-5, 6)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    r = dx * np.sqrt(I ** 2 + J ** 2 + K ** 2).ravel()
    f = lambda h: m * wfun(r, h).sum() - m * (hf / h) ** 3
    hs = brentq(f, 0.7 * hf * dx, 1.4 * hf * dx, xtol=1e-16, rtol=1e-15)
    rho = m * wfun(r, hs).sum()
    o = oracle.density(c["x"], c["y"], c["z"], c["m"], c["h"], oracle.make_params(c))
    # the C6 reference carries the quadrature error of its normalisation
    tol = 1e-12 if kind == oracle.M6 else 1e-9
    np.testing.assert_allclose(o["h"], hs, rtol=tol)
    np.testing.assert_allclose(o["rho"], rho, rtol=tol)
    assert np.all(o["nneigh"] == int(np.sum(r < S * hs)))
    assert abs(int(np.sum(r < S * hs)) - nn_expect) <= 12
    assert abs(o["rho"].mean() - 1.0) < 3e-3  # each kernel's lattice-sum bias


def dwdh_ref(r, h):
    """dW/dh of the M4 kernel, -(3 f(q) + q f'(q)) / (pi h^4) with f = 1.5 B3
    and f' from scipy's derivative of the B-spline."""
    q = np.asarray(r) / h
    f = 1.5 * np.nan_to_num(B3(q), nan=0.0)
    fp = 1.5 * np.nan_to_num(B3.derivative()(q), nan=0.0)
    return -(3.0 * f + q * fp) / (np.pi * h ** 4)


@pytest.mark.parametrize("start", [0.93, 1.45, 0.7])
def test_fixed_passes_recurrence_on_perfect_lattice(start):
    """The paper's fixed iteration (Sect. 3.2.1: the density is computed three
    times), read as two Newton updates of h clamped to [0.8 h, 1.2 h] (h kept
    where f' <= 0) from the sums at h0 and h1, then rho and Omega from the
    third sum at h2.  The recurrence is run here on the infinite-lattice sums
    with scipy's B-spline and its derivative; from 1.45 and 0.7 times the root
    the first steps hit the clamps."""
    c = inputs.lattice(16, jitter=0.0)
    dx, m, hf = c["dx"], c["m"][0], c["hfact"]
    g = np.arange(-6, 7)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    r = dx * np.sqrt(I ** 2 + J ** 2 + K ** 2).ravel()
    S0 = lambda h: m * w_ref(r, h).sum()
    S1 = lambda h: m * dwdh_ref(r, h).sum()
    root = brentq(lambda h: S0(h) - m * (hf / h) ** 3, 0.8 * dx, 1.6 * dx, xtol=1e-16,
                  rtol=1e-15)
    h = start * root
    h0 = h
    clamped = 0
    for _ in range(2):
        rh = m * (hf / h) ** 3
        f, fp = S0(h) - rh, S1(h) + 3.0 * rh / h
        hn = h - f / fp
        if not fp > 0.0:
            hn = h
        elif hn > 1.2 * h:
            hn, clamped = 1.2 * h, clamped + 1
        elif hn < 0.8 * h:
            hn, clamped = 0.8 * h, clamped + 1
        h = hn
    rho = S0(h)
    omega = 1.0 + h * S1(h) / (3.0 * rho)
    oc = dict(c)
    oc["h_tol_oracle"] = -1.0
    o = oracle.density(c["x"], c["y"], c["z"], c["m"], np.full(c["n"], h0),
                       oracle.make_params(oc))
    np.testing.assert_allclose(o["h"], h, rtol=1e-12)
    np.testing.assert_allclose(o["rho"], rho, rtol=1e-12)
    np.testing.assert_allclose(o["omega"], omega, rtol=1e-10)
    assert np.all(o["iters"] == 2)
    if start != 0.93:
        assert clamped >= 1  # the case exercises a clamp
    else:
        assert clamped == 0 and abs(h / root - 1) < 1e-3  # two free steps land near the root
