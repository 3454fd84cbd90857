"""Krook-Wu exact solution of the space-homogeneous binary mixture with a
constant collision kernel B_pq = lambda_qp / (4 pi n^q) (oracle; Sec. 3.2,
Eqs. bkw_pde and bkw_f and the expression for its time derivative).

Written out from the paper's closed forms.  The velocity v is measured from
the origin of the grid (the mixture is at rest).
"""
import math

import numpy as np


class KrookWu:
    def __init__(self, m1, m2, n1=1.0, n2=1.0, l11=1.0, l12=0.5, l21=0.5, l22=1.0):
        self.m = (float(m1), float(m2))
        self.n = (float(n1), float(n2))
        self.lam = {(1, 1): l11, (1, 2): l12, (2, 1): l21, (2, 2): l22}
        mu = 4.0 * m1 * m2 / (m1 + m2) ** 2
        t1 = l22 - l21 * mu * (3.0 - 2.0 * mu)
        t2 = l11 - l12 * mu * (3.0 - 2.0 * mu)
        self.mu, self.tau = mu, (t1, t2)
        self.A = (l11 + l21 * mu * (3.0 - 2.0 * mu * t2 / t1)) / 6.0
        self.B = (l11 * t1 + l21 * mu * (3.0 - 2.0 * mu) * t2) / 3.0

    def constraint(self):
        """(tau_1 - tau_2)(2 mu^2 (l21/tau_1 - l12/tau_2) - 1); must vanish."""
        t1, t2 = self.tau
        return (t1 - t2) * (2.0 * self.mu ** 2 * (self.lam[2, 1] / t1 - self.lam[1, 2] / t2) - 1.0)

    def beta(self, p, q):
        """Constant kernel value B_pq = lambda_qp / (4 pi n^q), p, q in {1, 2}."""
        return self.lam[q, p] / (4.0 * math.pi * self.n[q - 1])

    def Q(self, t):
        return self.A / (self.A * math.exp(self.A * t) - self.B)

    def dQ(self, t):
        e = math.exp(self.A * t)
        return -self.A ** 3 * e / (self.A * e - self.B) ** 2

    def K(self, t):
        n1, n2 = self.n
        t1, t2 = self.tau
        return (n1 + n2) / ((n1 + n2) + 2.0 * (n1 * t1 + n2 * t2) * self.Q(t))

    def dK(self, t):
        n1, n2 = self.n
        t1, t2 = self.tau
        s = n1 * t1 + n2 * t2
        return -2.0 * (n1 + n2) * s / ((n1 + n2) + 2.0 * s * self.Q(t)) ** 2 * self.dQ(t)

    def f(self, p, t, v2):
        """f^p(t, v) with v2 = |v|^2 (array)."""
        m, n = self.m[p - 1], self.n[p - 1]
        K = self.K(t)
        Qp = self.tau[p - 1] * self.Q(t)
        g = n * (m / (2.0 * math.pi * K)) ** 1.5 * np.exp(-m * v2 / (2.0 * K))
        return g * ((1.0 - 3.0 * Qp) + m / K * Qp * v2)

    def dfdt(self, p, t, v2):
        """The paper's closed form of d f^p / dt."""
        m, n = self.m[p - 1], self.n[p - 1]
        K, dK = self.K(t), self.dK(t)
        tau = self.tau[p - 1]
        Qp, dQp = tau * self.Q(t), tau * self.dQ(t)
        g = n * (m / (2.0 * math.pi * K)) ** 1.5 * np.exp(-m * v2 / (2.0 * K))
        f = g * ((1.0 - 3.0 * Qp) + m / K * Qp * v2)
        return f * (-1.5 * dK / K + m * v2 / (2.0 * K * K) * dK) + \
            g * (-3.0 * dQp + m / K * dQp * v2 - m / (K * K) * dK * Qp * v2)


def table1_errors(N, Nr, M, ratio, L=12.0, t=5.5, R=None):
    """(E1, E2): L-infinity errors of the mixture collision term
    sum_q Q^{pq}(f^p, f^q) against the exact d f^p/dt (the accuracy study
    of Sec. 3.2, Table 1), for m_1 = 1, m_2 = ratio, on the cell-centred
    N^3 grid over [-L, L]^3, with N_rho radii and the M-point octahedron
    (M = 6) or icosahedron (M = 12) set.  The kernel is the constant
    B_pq = lambda_qp / (4 pi n^q) (gamma = eta = 0).  R: the truncation
    radius of every pair; None applies the rule of Sec. 2.1 per pair."""
    from .collide import PairPlan, collide
    from .quadrature import sphere_set, velocity_grid
    kw = KrookWu(1.0, ratio)
    c, _ = velocity_grid(N, L)
    cx, cy, cz = np.meshgrid(c, c, c, indexing="ij")
    v2 = cx ** 2 + cy ** 2 + cz ** 2
    f = {p: kw.f(p, t, v2) for p in (1, 2)}
    s, w = sphere_set("octahedron" if M == 6 else "icosahedron")
    masses = {1: 1.0, 2: float(ratio)}
    errs = []
    for p in (1, 2):
        tot = 0.0
        for q in (1, 2):
            pl = PairPlan(N, L, masses[p], masses[q], 1.0, 1.0, Nr, s, w, R=R,
                          beta=kw.beta(p, q), gamma=0.0, eta=0.0)
            tot = tot + collide(pl, f[p], f[q])
        errs.append(float(np.max(np.abs(tot - kw.dfdt(p, t, v2)))))
    return tuple(errs)
