"""Collision operator Q^{pq}(f^p, f^q) (oracle; test infrastructure).

``collide`` evaluates the Fourier-Galerkin form of the operator (Sec. 2.1):
the gain as the low-rank sum of circular convolutions of Eq.
(apndx_fs_Glm_Qk), with the (rho, sigma) quadrature of Eq. (realGG) as the
low-rank expansion of G^+, and the loss as one convolution with G^-; each
convolution goes through the oracle's own naive DFT.  ``collide_direct``
evaluates the projected operator of Eq. (apndx_Qprojected) as a direct
O(N^6) sum over wave-index pairs with the same quadrature of G^+ and G^-
(Eq. Gmm_vss), so the two can be compared at small N.  Arrays are indexed
[x, y, z].
"""
import math

import numpy as np

from . import dft
from .quadrature import gauss_legendre, sphere_set, truncation_radius, wave_grid
from .tables import beta_reduced, gain_table, kernel_exponents, loss_table


class PairPlan:
    """Everything Algorithm 2 needs for one ordered pair (p, q): the inputs
    of Algorithm 1 and its outputs b, c, plus beta.

    N, L        velocity grid points per axis and half-width of D_L
    mp, mq      species masses
    omega,alpha VSS parameters of the pair (alpha = 1 is VHS)
    R           truncation radius (None: the rule of Sec. 2.1)
    Nrho        Gauss-Legendre points on [0, R]
    sigma, w_sigma  sphere quadrature (M points, weights summing to 4 pi)
    beta        prefactor; None => unit reduced Knudsen number (beta_reduced)
    gamma, eta  override the kernel exponents (Krook-Wu uses gamma = eta = 0)
    nyquist_zero  form the gain's translates t1, t2 from fft(f^p), fft(f^q)
                with their Nyquist planes (wave index -N/2 on any axis) set
                to zero; the loss term is unchanged.  Then t1 and t2 are
                Hermitian, so u1 = ifft(t1) and u2 = ifft(t2) are real.
                This variant is not in the paper (whose Algorithm 2 keeps the
                Nyquist planes and takes Re() at the end).
    """

    def __init__(self, N, L, mp, mq, omega, alpha, Nrho, sigma, w_sigma,
                 R=None, beta=None, gamma=None, eta=None, nyquist_zero=False):
        self.N, self.L, self.mp, self.mq = N, L, float(mp), float(mq)
        self.nyquist_zero = bool(nyquist_zero)
        g, e = kernel_exponents(omega, alpha)
        self.gamma = g if gamma is None else gamma
        self.eta = e if eta is None else eta
        self.R = truncation_radius(L, mp, mq) if R is None else R
        self.rho, self.w_rho = gauss_legendre(Nrho, self.R)
        self.sigma = np.asarray(sigma, dtype=float)
        self.w_sigma = np.asarray(w_sigma, dtype=float)
        self.beta = beta_reduced(mp, mq, omega, alpha) if beta is None else beta
        self.b = gain_table(N, L, self.rho, self.sigma, mp, mq, self.gamma, self.eta)
        self.c = loss_table(N, L, self.rho, self.w_rho, self.gamma, self.eta)


def phase_argument(plan, r, m):
    """a = pi/L rho_r (l . sigma_m) on the N^3 wave grid (Algorithm 1, table a)."""
    lx, ly, lz = wave_grid(plan.N)
    s = plan.sigma[m]
    return math.pi / plan.L * plan.rho[r] * (lx * s[0] + ly * s[1] + lz * s[2])


def nyquist_mask(N):
    """1 on the N^3 wave grid except where some axis has wave index -N/2
    (storage index N/2), which is 0."""
    keep = np.ones(N)
    keep[N // 2] = 0.0
    return keep[:, None, None] * keep[None, :, None] * keep[None, None, :]


def gain_spectra(plan, FTf, FTg):
    """The transforms the gain's translates are formed from: FTf, FTg as
    they are, or with their Nyquist planes zeroed (plan.nyquist_zero)."""
    if not plan.nyquist_zero:
        return FTf, FTg
    z = nyquist_mask(plan.N)
    return z * FTf, z * FTg


def fourier_coefficients(a):
    """Coefficients a_hat of the truncated Fourier series of the samples a
    (Sec. 2.1, the series approximating f^p and f^q): the forward DFT over
    N^3, a_hat = DFT(a) / N^3."""
    return dft.fft3(a) / a.size


def synthesize(a_hat):
    """The series sum_k a_hat_k e^{2 pi i k.j/N} evaluated at every grid
    index j (the inverse of fourier_coefficients)."""
    return dft.ifft3(a_hat) * a_hat.size


def circular_convolution(A, B):
    """sum over l + m = k (mod N, per axis) of A_l B_m, for every k.

    The Galerkin sum of Eq. (apndx_Qprojected) runs over wave pairs with
    l + m = k; the modular reading is the one the FFT form of the method
    computes.  By the convolution theorem the sum equals the coefficients of
    the pointwise product of the two synthesized series."""
    return fourier_coefficients(synthesize(A) * synthesize(B))


def gain_loss_coefficients(plan, f, g):
    """(Qhat+, Qhat-): the gain and loss Fourier coefficients of Q^{pq}
    before the prefactor beta.

    Gain, Eq. (apndx_fs_Glm_Qk) with the low-rank expansion of G+ given by
    the (rho_r, sigma_m) quadrature of Eq. (realGG):
        Qhat+_k = sum_{r,m} alpha_rm(k) sum_{l+m'=k} (beta_rm(l) fhat_l)
                                                    (gamma_rm(m') ghat_m'),
        alpha_rm(k) = w_r w_m F(k, rho_r, sigma_m)   (table b, Eq. Fkr_vss),
        beta_rm(l)  = exp(+i pi/L rho_r m_q/(m_p+m_q) l.sigma_m),
        gamma_rm(m')= exp(-i pi/L rho_r m_p/(m_p+m_q) m'.sigma_m).
    Loss: Qhat-_k = sum_{l+m'=k} G-(m') fhat_l ghat_m' (table c, Eq. Gmm_vss).
    The (r, m) sum runs r outer, m inner, in increasing order.  With
    plan.nyquist_zero the gain convolves the Nyquist-zeroed coefficients
    (gain_spectra); the loss is unchanged."""
    mp, mq = plan.mp, plan.mq
    fh = fourier_coefficients(f)
    gh = fourier_coefficients(g)
    fg, gg = gain_spectra(plan, fh, gh)
    gain = np.zeros_like(fh)
    for r in range(len(plan.rho)):
        for m in range(len(plan.sigma)):
            a = phase_argument(plan, r, m)
            beta_l = np.exp(1j * mq / (mp + mq) * a)
            gamma_m = np.exp(-1j * mp / (mp + mq) * a)
            alpha_k = plan.w_rho[r] * plan.w_sigma[m] * plan.b[r, m]
            gain = gain + alpha_k * circular_convolution(beta_l * fg, gamma_m * gg)
    loss = circular_convolution(fh, plan.c * gh)
    return gain, loss


def collide_gain_loss(plan, f, g):
    """The gain and loss parts of Q^{pq}(f, g) on the grid, each with the
    prefactor beta: (beta Re gain(c_j), beta Re loss(c_j))."""
    gain, loss = gain_loss_coefficients(plan, f, g)
    return plan.beta * np.real(synthesize(gain)), plan.beta * np.real(synthesize(loss))


def collide(plan, f, g):
    """Q^{pq}(f, g) = beta Re sum_k (Qhat+_k - Qhat-_k) e^{i pi/L k.c} on the
    grid, the operator Algorithm 2 evaluates (the collision step of the
    fast spectral method, Sec. 2.1).

    f = F^p and g = F^q are real N^3 arrays indexed [x, y, z]."""
    gain, loss = gain_loss_coefficients(plan, f, g)
    return plan.beta * np.real(synthesize(gain - loss))


def kernel_mode_gain(plan, l, m):
    """G^{pq+}(l, m) of Eq. (realGG) by the (rho_r, sigma_m) quadrature:
    sum_{r,m} w_r w_m F(k, rho_r, sigma_m) exp(i pi/L rho (a_q l - a_p m).sigma)
    with k = l + m wrapped into [-N/2, N/2) (circular convolution)."""
    N = plan.N
    aq = plan.mq / (plan.mp + plan.mq)
    ap = plan.mp / (plan.mp + plan.mq)
    l = np.asarray(l)
    m = np.asarray(m)
    k = (l + m + N // 2) % N - N // 2
    kidx = tuple(k % N)  # storage index of wave k
    out = 0.0j
    for r in range(len(plan.rho)):
        for s in range(len(plan.sigma)):
            sg = plan.sigma[s]
            ph = math.pi / plan.L * plan.rho[r] * float(np.dot(aq * l - ap * m, sg))
            out += plan.w_rho[r] * plan.w_sigma[s] * plan.b[(r, s) + kidx] * np.exp(1j * ph)
    return out


def collide_direct(plan, f, g):
    """Direct O(N^6) evaluation of Eq. (apndx_Qprojected) on the discrete
    Fourier coefficients: Qhat_k = sum_{l+m = k mod N} [G+(l,m) - G-(m)]
    fhat_l ghat_m, fhat = fft3(f)/N^3, then Q = beta Re(sum_k Qhat_k e^{...}).
    With plan.nyquist_zero the G+ part runs over l and m off the Nyquist
    planes only (no component equal to -N/2); G- over all pairs.
    Vectorised over l for each m.  Only sensible for N <= 8."""
    N = plan.N
    n3 = N ** 3
    fh = dft.fft3(f) / n3
    gh = dft.fft3(g) / n3
    aq = plan.mq / (plan.mp + plan.mq)
    ap = plan.mp / (plan.mp + plan.mq)
    lx, ly, lz = wave_grid(N)
    L3 = np.stack([lx.ravel(), ly.ravel(), lz.ravel()], axis=1)  # storage order
    fh = fh.ravel()
    gh = gh.ravel()
    c = plan.c.ravel()
    b = plan.b.reshape(len(plan.rho), len(plan.sigma), n3)
    if plan.nyquist_zero:
        off_nyq = np.all(L3 != -(N // 2), axis=1).astype(float)
    else:
        off_nyq = np.ones(n3)
    Qh = np.zeros(n3, dtype=complex)
    for mi in range(n3):
        mvec = L3[mi]
        kvec = (L3 + mvec + N // 2) % N - N // 2
        kidx = ((kvec[:, 0] % N) * N + (kvec[:, 1] % N)) * N + (kvec[:, 2] % N)
        Gp = np.zeros(n3, dtype=complex)
        for r in range(len(plan.rho)):
            for s in range(len(plan.sigma)):
                sg = plan.sigma[s]
                ph = math.pi / plan.L * plan.rho[r] * ((aq * L3 - ap * mvec) @ sg)
                Gp += plan.w_rho[r] * plan.w_sigma[s] * b[r, s, kidx] * np.exp(1j * ph)
        contrib = (Gp * off_nyq * off_nyq[mi] - c[mi]) * fh * gh[mi]
        np.add.at(Qh, kidx, contrib)
    Q = dft.ifft3(Qh.reshape(N, N, N)) * n3
    return plan.beta * np.real(Q)


def default_pair_plan(N, L, masses, p, q, omega, alpha, Nrho, sphere, M=None,
                      R=None, beta=None, gamma=None, eta=None, nyquist_zero=False):
    """Convenience: PairPlan for species (p, q) with a named sphere set."""
    sigma, w = sphere_set(sphere, M)
    return PairPlan(N, L, masses[p], masses[q], omega, alpha, Nrho, sigma, w,
                    R=R, beta=beta, gamma=gamma, eta=eta, nyquist_zero=nyquist_zero)


def mixture_collision(pair_plans, F):
    """sum_q Q^{pq}(f^p, f^q) for every node and species p of
    F [nodes, ns, N, N, N]; pair_plans[p][q] is the PairPlan of (p, q)
    (Eq. bzeNonDim, with 1/Kn inside beta)."""
    out = np.zeros_like(F)
    ns = F.shape[1]
    for i in range(F.shape[0]):
        for p in range(ns):
            for q in range(ns):
                out[i, p] += collide(pair_plans[p][q], F[i, p], F[i, q])
    return out
