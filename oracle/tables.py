"""Kernel tables of the fast spectral method (oracle; test infrastructure).

The paper precomputes (Algorithm 1)
  b^{pq}_{r m}(k) = F^{pq}(k, rho_r, sigma_m)        gain table, Eq. (Fkr_vss)
  c^{pq}(k)       = G^{pq-}(k)                        loss table, Eq. (Gmm_vss)
with the inner sphere integrals done by an unspecified "pre-computation"
quadrature sigma^pre.  The oracle evaluates those sphere integrals exactly
(the M^pre -> infinity limit):

  * VHS (alpha = 1):  int_{S^2} exp(-i x khat.u) du = 4 pi sinc(x)
  * VSS (alpha != 1): Funk-Hecke,
        int_{S^2} (1 + sigma.u)^eta exp(-i x khat.u) du
            = 4 pi sum_n a_n (-i)^n j_n(x) P_n(sigma.khat),
        a_n = (2n+1)/2 int_{-1}^{1} (1+t)^eta P_n(t) dt.

The collision kernel without its prefactor is |u|^gamma (1 + cos chi)^eta
(Eq. VSSNonDim) with gamma = 2(1 - omega) and eta = alpha - 1.  Algorithm 1
prints gamma = 2(omega - 1); Eq. (VSSNonDim) and F = rho^2 B need the
exponent 2(1 - omega), which is the reading taken here.
"""
import math

import numpy as np

from .quadrature import wave_grid


def kernel_exponents(omega, alpha):
    """(gamma, eta) = (2(1 - omega), alpha - 1)."""
    return 2.0 * (1.0 - omega), alpha - 1.0


def beta_prefactor(mp, mq, omega, alpha, kn):
    """beta^{pq} of Sec. 2 (the prefactor of Eq. VSSNonDim divided by Kn_pq)."""
    mu = mp * mq / (mp + mq)
    return (1.0 / kn) / math.sqrt(1.0 + mp / mq) / mu ** (omega - 0.5) \
        * alpha / (2.0 ** (1.0 + alpha) * math.gamma(2.5 - omega) * math.pi)


def beta_reduced(mp, mq, omega, alpha):
    """beta^{pq} with unit reduced Knudsen number Kn_pq sqrt(1 + m_p/m_q) = 1.

    Kn_pq of Eq. (Kn) carries the factor 1/sqrt(1 + m_p/m_q) that also
    appears in beta^{pq}; the two cancel, leaving
    mu^{1/2 - omega} alpha / (2^{1+alpha} Gamma(5/2 - omega) pi), mu the
    reduced mass.  This is symmetric in (p, q), as conservation of total
    momentum and energy between Q^{pq} and Q^{qp} requires."""
    mu = mp * mq / (mp + mq)
    return mu ** (0.5 - omega) * alpha / (2.0 ** (1.0 + alpha) * math.gamma(2.5 - omega) * math.pi)


def knudsen(mp, mq, n0, dref, Tref, T0, omega, H0):
    """Kn_pq of Eq. (Kn)."""
    return 1.0 / (math.sqrt(1.0 + mp / mq) * math.pi * n0 * dref ** 2
                  * (Tref / T0) ** (omega - 0.5) * H0)


def sinc(x):
    x = np.asarray(x, dtype=float)
    out = np.ones_like(x)
    nz = x != 0.0
    out[nz] = np.sin(x[nz]) / x[nz]
    return out


def spherical_jn_all(nmax, x):
    """j_0..j_nmax at the points x by Miller's downward recurrence
    j_{n-1} = (2n+1)/x j_n - j_{n+1}, started well above max(nmax, x) and
    normalised by the sum rule sum_n (2n+1) j_n(x)^2 = 1, with the sign taken
    from whichever of j_0 = sin x / x and j_1 = sin x / x^2 - cos x / x is
    larger in magnitude.  Returns [nmax+1, *x.shape]; at x = 0, j_0 = 1 and
    j_n = 0 for n > 0."""
    x = np.asarray(x, dtype=float)
    flat = x.ravel()
    out = np.zeros((nmax + 1, flat.size))
    zero = flat == 0.0
    xs = np.where(zero, 1.0, flat)
    start = nmax + int(np.max(xs)) + 40
    jp1 = np.zeros_like(xs)
    jn = np.full_like(xs, 1e-200)
    norm = (2 * start + 1) * jn * jn
    for n in range(start, 0, -1):
        jm1 = (2 * n + 1) / xs * jn - jp1
        jp1, jn = jn, jm1
        norm = norm + (2 * (n - 1) + 1) * jn * jn
        if n - 1 <= nmax:
            out[n - 1] = jn
        big = np.abs(jn) > 1e100
        if np.any(big):
            s = np.where(big, 1e-100, 1.0)
            jn, jp1 = jn * s, jp1 * s
            norm = norm * s * s
            out *= s[None, :]
    scale = 1.0 / np.sqrt(norm)
    j0 = np.sin(xs) / xs
    j1 = np.sin(xs) / xs ** 2 - np.cos(xs) / xs
    use0 = np.abs(j0) >= np.abs(j1)
    ref = np.where(use0, j0, j1)
    got = np.where(use0, out[0], out[1] if nmax >= 1 else out[0])
    if nmax < 1:
        # j_1 is not stored; fall back to j_0 for the sign
        ref, got = j0, out[0]
    scale = scale * np.sign(ref * got)
    out *= scale[None, :]
    out[:, zero] = 0.0
    out[0, zero] = 1.0
    return out.reshape((nmax + 1,) + x.shape)


def legendre_all(nmax, t):
    """P_0..P_nmax at t by Bonnet's recurrence."""
    t = np.asarray(t, dtype=float)
    P = np.zeros((nmax + 1,) + t.shape)
    P[0] = 1.0
    if nmax >= 1:
        P[1] = t
    for n in range(1, nmax):
        P[n + 1] = ((2 * n + 1) * t * P[n] - n * P[n - 1]) / (n + 1)
    return P


def funk_hecke_coeffs(eta, nmax):
    """a_n = (2n+1)/2 int_{-1}^{1} (1+t)^eta P_n(t) dt, n = 0..nmax, from
    int (1+t)^eta P_n = 2^{eta+1} eta(eta-1)..(eta-n+1) / ((eta+1)..(eta+n+1)).
    The ratio of the two products is carried as one number, r_0 = 1/(eta+1),
    r_n = r_{n-1} (eta-n+1)/(eta+n+1): each product alone overflows past
    n = 170, which the series reaches at the largest |k| of an N = 48 grid."""
    a = np.zeros(nmax + 1)
    r = 1.0 / (eta + 1.0)
    for n in range(nmax + 1):
        if n > 0:
            r *= (eta - n + 1) / (eta + n + 1)
        a[n] = 0.5 * (2 * n + 1) * 2.0 ** (eta + 1.0) * r
    return a


def sphere_integral_C(eta):
    """int_{S^2} (1 + sigma.u)^eta dsigma = 2 pi 2^(eta+1)/(eta+1)."""
    return 2.0 * math.pi * 2.0 ** (eta + 1.0) / (eta + 1.0)


def _nmax_for(xmax):
    return int(xmax + 10.0 * xmax ** (1.0 / 3.0) + 40.0)


def phi_vss(x, t, eta):
    """int_{S^2} (1 + sigma.u)^eta exp(-i x khat.u) du with t = sigma.khat,
    by Funk-Hecke (x >= 0; arrays broadcast)."""
    x = np.asarray(x, dtype=float)
    t = np.asarray(t, dtype=float)
    if eta == 0.0:
        return (4.0 * math.pi * sinc(x)).astype(complex) * np.ones_like(t)
    nmax = _nmax_for(float(np.max(x)) if x.size else 0.0)
    xb, tb = np.broadcast_arrays(x, t)
    return _funk_hecke_sum(eta, spherical_jn_all(nmax, xb), tb)


def _funk_hecke_sum(eta, J, t):
    """4 pi sum_n a_n (-i)^n j_n(x) P_n(t) with J = [j_0(x) .. j_nmax(x)]."""
    nmax = J.shape[0] - 1
    a = funk_hecke_coeffs(eta, nmax)
    P = legendre_all(nmax, t)
    phase = (-1j) ** np.arange(nmax + 1)
    return 4.0 * math.pi * np.tensordot(a * phase, J * P, axes=(0, 0))


def gain_table(N, L, rho, sigma, mp, mq, gamma, eta):
    """b_{rm}(k) = F^{pq}(k, rho_r, sigma_m), Eq. (Fkr_vss), for all wave
    indices k of the N^3 grid.  F = rho^2 int B e^{-i pi/L rho m_q/(m_p+m_q) k.u} du
    with B = rho^gamma (1 + sigma.u)^eta.  Returns complex [Nr, M, N, N, N]."""
    lx, ly, lz = wave_grid(N)
    kk = np.sqrt(lx * lx + ly * ly + lz * lz).astype(float)
    aq = mq / (mp + mq)
    out = np.zeros((len(rho), len(sigma), N, N, N), dtype=complex)
    safe = np.where(kk == 0.0, 1.0, kk)
    for r, rr in enumerate(rho):
        x = math.pi / L * rr * aq * kk
        # the Bessel values depend on |k| and r only: computed once per radius
        J = None if eta == 0.0 else spherical_jn_all(_nmax_for(float(np.max(x))), x)
        for m, s in enumerate(sigma):
            t = np.where(kk == 0.0, 1.0, (s[0] * lx + s[1] * ly + s[2] * lz) / safe)
            phi = phi_vss(x, t, eta) if J is None else _funk_hecke_sum(eta, J, t)
            out[r, m] = rr ** (gamma + 2.0) * phi
    return out


def loss_table(N, L, rho, w_rho, gamma, eta):
    """c(k) = G^{pq-}(k), Eq. (Gmm_vss):
    sum_r w_r rho_r^{gamma+2} C_eta 4 pi sinc(pi/L rho_r |k|), with the sigma
    integral C_eta done exactly.  Returns real [N, N, N]."""
    lx, ly, lz = wave_grid(N)
    kk = np.sqrt(lx * lx + ly * ly + lz * lz).astype(float)
    C = sphere_integral_C(eta)
    c = np.zeros((N, N, N))
    for rr, wr in zip(rho, w_rho):
        c += wr * rr ** (gamma + 2.0) * C * 4.0 * math.pi * sinc(math.pi / L * rr * kk)
    return c
