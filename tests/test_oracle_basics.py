"""Pins of the oracle's building blocks against mathematics and libraries."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

from oracle import dft, quadrature as qd, tables as tb
from paper_1903_04670_amd import workloads as wl


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 6, 6), (8, 8, 8), (16, 16, 16), (24, 8, 12)])
def test_naive_dft_matches_numpy_fft(shape):
    rng = np.random.default_rng(1)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert np.max(np.abs(dft.fft3(a) - np.fft.fftn(a))) < 1e-12 * np.max(np.abs(np.fft.fftn(a)))
    assert np.max(np.abs(dft.ifft3(a) - np.fft.ifftn(a))) < 1e-13


def test_wave_index():
    assert list(qd.wave_index(8)) == [0, 1, 2, 3, -4, -3, -2, -1]
    assert list(qd.wave_index(6)) == [0, 1, 2, -3, -2, -1]


def test_grid_matches_input_generator():
    for N, L in [(16, 7.7), (32, 8.83)]:
        c, h = qd.velocity_grid(N, L)
        assert np.allclose(c, wl.grid(N, L), atol=0, rtol=0)
        assert abs(h - 2 * L / N) < 1e-15


@pytest.mark.parametrize("n", [1, 4, 8, 16])
def test_gauss_legendre_exactness(n):
    R = 7.3
    x, w = qd.gauss_legendre(n, R)
    assert np.all(np.diff(x) > 0) and x[0] > 0 and x[-1] < R
    for k in range(2 * n):
        assert abs(np.sum(w * x ** k) - R ** (k + 1) / (k + 1)) < 1e-12 * R ** (k + 1)


def _sphere_moment(s, w, px, py, pz):
    return np.sum(w * s[:, 0] ** px * s[:, 1] ** py * s[:, 2] ** pz)


def _exact_sphere_moment(px, py, pz):
    # int_{S^2} x^a y^b z^c = 2 G(A)G(B)G(C)/G(A+B+C), A = (a+1)/2 ..., 0 if any odd
    if px % 2 or py % 2 or pz % 2:
        return 0.0
    A, B, C = (px + 1) / 2, (py + 1) / 2, (pz + 1) / 2
    return 2 * math.gamma(A) * math.gamma(B) * math.gamma(C) / math.gamma(A + B + C)


@pytest.mark.parametrize("kind,M,degree", [("octahedron", 6, 3), ("icosahedron", 12, 5)])
def test_sphere_designs(kind, M, degree):
    s, w = qd.sphere_set(kind, M)
    assert s.shape == (M, 3)
    assert np.allclose(np.sum(s * s, axis=1), 1.0, atol=1e-15)
    assert abs(np.sum(w) - 4 * math.pi) < 1e-13
    for a in range(degree + 1):
        for b in range(degree + 1 - a):
            for c in range(degree + 1 - a - b):
                assert abs(_sphere_moment(s, w, a, b, c) - _exact_sphere_moment(a, b, c)) < 1e-13
    # not a design of the next even degree
    assert abs(_sphere_moment(s, w, degree + 1, 0, 0) - _exact_sphere_moment(degree + 1, 0, 0)) > 1e-3


def test_fibonacci_converges():
    errs = []
    for M in (32, 128, 512):
        s, w = qd.sphere_set("fibonacci", M)
        assert np.allclose(np.sum(s * s, axis=1), 1.0, atol=1e-14)
        errs.append(abs(_sphere_moment(s, w, 2, 2, 0) - _exact_sphere_moment(2, 2, 0)))
    assert errs[0] > errs[1] > errs[2]


def test_truncation_radius_equal_masses_is_twice_support():
    # with m_p = m_q the rule of Sec. 2.1 gives R = 4L/(3 + sqrt 2), and with
    # L = (3 + sqrt 2) S / 2 that is 2 S, the R = 2S of the workloads
    for S in (3.5, 4.0):
        L, R = wl.box_for_support(S)
        assert abs(qd.truncation_radius(L, 1.0, 1.0) - R) < 1e-13
        assert abs(qd.truncation_radius(L, 2.0, 2.0) - R) < 1e-13
    # a heavier partner shrinks R
    assert qd.truncation_radius(12.0, 1.0, 4.0) < qd.truncation_radius(12.0, 1.0, 1.0)


def test_spherical_bessel_against_scipy():
    x = np.array([0.0, 1e-4, 0.3, math.pi, 2 * math.pi, 7.7, 41.0, 118.3, 160.0])
    J = tb.spherical_jn_all(220, x)
    for n in range(221):
        assert np.max(np.abs(J[n] - sp.spherical_jn(n, x))) < 1e-14


def test_legendre_against_scipy():
    t = np.linspace(-1, 1, 23)
    P = tb.legendre_all(40, t)
    for n in range(41):
        assert np.max(np.abs(P[n] - sp.eval_legendre(n, t))) < 1e-13


@pytest.mark.parametrize("eta", [0.0, 0.4, 0.36, -0.3])
def test_funk_hecke_coefficients_by_quadrature(eta):
    a = tb.funk_hecke_coeffs(eta, 12)
    for n in range(13):
        val, _ = si.quad(lambda t: (1 + t) ** eta * sp.eval_legendre(n, t), -1, 1,
                         limit=200, epsabs=1e-14, epsrel=1e-13)
        assert abs(a[n] - 0.5 * (2 * n + 1) * val) < 1e-11
    if eta == 0.0:
        assert a[0] == 1.0 and np.all(a[1:] == 0.0)


@pytest.mark.parametrize("eta", [0.4, -0.3, 2.0])
def test_funk_hecke_coefficients_high_orders(eta):
    """Orders up to 240 (the series at the largest |k| of an N = 48 grid needs
    about 180): against a Gauss-Jacobi rule with weight (1+t)^eta, exact for
    the polynomial P_n.  For integer eta the coefficients vanish past n = eta.
    The rule's own sum over ~120 nodes carries about 1e-12 of rounding, hence
    the 1e-10 bar; an overflow or a wrong factor misses by order one."""
    nmax = 240
    a = tb.funk_hecke_coeffs(eta, nmax)
    assert np.all(np.isfinite(a))
    t, w = sp.roots_jacobi(nmax // 2 + 2, 0.0, eta)
    for n in range(nmax + 1):
        ref = 0.5 * (2 * n + 1) * np.sum(w * sp.eval_legendre(n, t))
        assert abs(a[n] - ref) <= 1e-10 * max(1.0, abs(ref)), (n, a[n], ref)
    if eta == 2.0:
        assert np.all(a[3:] == 0.0)


def _phi_bruteforce(x, khat, sig, eta, nt=400, nphi=400):
    """int_{S^2} (1 + sig.u)^eta exp(-i x khat.u) du by a product rule:
    Gauss-Legendre in cos(theta) about sig, trapezoid in azimuth."""
    ct, wt = np.polynomial.legendre.leggauss(nt)
    ph = np.arange(nphi) * 2 * math.pi / nphi
    sig = np.asarray(sig, float)
    # orthonormal frame (e1, e2, sig)
    tmp = np.array([1.0, 0, 0]) if abs(sig[0]) < 0.9 else np.array([0, 1.0, 0])
    e1 = np.cross(sig, tmp)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(sig, e1)
    st = np.sqrt(1 - ct ** 2)
    U = (st[:, None, None] * (np.cos(ph)[None, :, None] * e1 + np.sin(ph)[None, :, None] * e2)
         + ct[:, None, None] * sig)
    integrand = (1 + ct[:, None]) ** eta * np.exp(-1j * x * (U @ np.asarray(khat, float)))
    return np.sum(wt[:, None] * integrand) * (2 * math.pi / nphi)


@pytest.mark.parametrize("eta", [0.0, 0.4])
def test_sphere_integral_closed_forms(eta):
    rng = np.random.default_rng(7)
    # x up to 94: the largest argument of the N = 48, N_rho = 24 gain table
    for x in (0.0, 0.7, 3.1, 9.5, 60.0, 94.0):
        k = rng.standard_normal(3)
        k /= np.linalg.norm(k)
        s = rng.standard_normal(3)
        s /= np.linalg.norm(s)
        got = tb.phi_vss(np.array(x), np.array(float(s @ k)), eta)
        ref = _phi_bruteforce(x, k, s, eta)
        assert abs(got - ref) < 2e-6 * max(1.0, abs(ref)), (x, got, ref)
    assert abs(tb.sphere_integral_C(eta) - _phi_bruteforce(0.0, [0, 0, 1], [1, 0, 0], eta)) < 1e-6


def test_gain_table_special_values():
    N, L = 8, 5.0
    rho, wr = qd.gauss_legendre(3, 4.0)
    s, w = qd.sphere_set("icosahedron")
    for eta, gamma in [(0.0, 1.0), (0.4, 0.6)]:
        b = tb.gain_table(N, L, rho, s, 1.0, 2.0, gamma, eta)
        # k = 0: rho^{gamma+2} C_eta
        for r in range(3):
            assert np.allclose(b[r, :, 0, 0, 0], rho[r] ** (gamma + 2) * tb.sphere_integral_C(eta), rtol=1e-13)
        # F(-k) = conj F(k) away from the Nyquist index
        for (i, j, k) in [(1, 2, 3), (3, 1, 1), (2, 0, 7)]:
            mi, mj, mk = (-i) % N, (-j) % N, (-k) % N
            assert np.allclose(b[:, :, mi, mj, mk], np.conj(b[:, :, i, j, k]), rtol=1e-12, atol=1e-14)
        if eta == 0.0:
            assert np.max(np.abs(b.imag)) == 0.0
            # VHS: sigma-independent
            assert np.max(np.abs(b - b[:, :1])) == 0.0
    c = tb.loss_table(N, L, rho, wr, 1.0, 0.0)
    assert abs(c[0, 0, 0] - np.sum(wr * rho ** 3) * 4 * math.pi * 4 * math.pi) < 1e-10


def test_beta_hard_sphere_closed_form():
    # omega = 1/2, alpha = 1, equal unit masses, Kn = 1: 1/sqrt 2 * 1/(4 Gamma(2) pi)
    assert abs(tb.beta_prefactor(1.0, 1.0, 0.5, 1.0, 1.0) - 1 / (4 * math.sqrt(2) * math.pi)) < 1e-16


def test_knudsen_numbers_of_table2():
    """Kn of Eq. (Kn) with the Case C-01 parameters of Table 2 reproduces the
    printed (Kn11, Kn22) = (0.793, 0.606) and (Kn12, Kn21) = (0.803, 0.555)."""
    m = {1: 66.3, 2: 139.1}
    d = {(1, 1): 4.11e-10, (1, 2): 4.405e-10, (2, 1): 4.405e-10, (2, 2): 4.7e-10}
    om = {(1, 1): 0.81, (1, 2): 0.805, (2, 1): 0.805, (2, 2): 0.8}
    printed = {(1, 1): 0.793, (2, 2): 0.606, (1, 2): 0.803, (2, 1): 0.555}
    for (p, q), kn in printed.items():
        got = tb.knudsen(m[p], m[q], 1.680e21, d[p, q], 273.0, 273.0, om[p, q], 1e-3)
        assert abs(got - kn) < 0.6e-3, (p, q, got)
