"""Nodal discontinuous Galerkin transport in x with upwind flux, Maxwell
diffuse walls, and SSP-RK3 time stepping (oracle; test infrastructure).

The paper uses RKDG for the transport part of Eq. (bzeNonDim) and cites its
details elsewhere.  This is the textbook nodal DG scheme on Gauss-Lobatto-
Legendre (GLL) nodes in strong form:
    d f_e/dt = -(2/h) c_x Dr f_e + (2/h) Minv [ l_R (c_x f_R - F*_R)
                                              - l_L (c_x f_L - F*_L) ]
with the upwind flux F* = c_x f(upwind side), and the third-order strong-
stability-preserving Runge-Kutta scheme of Shu and Osher.

Diffuse walls: on the inflow half of velocity space the wall emits
n_w M_w(c) with M_w = (m/(pi T_w))^{3/2} exp(-m |c - u_w|^2 / T_w) and n_w
chosen so that the discrete net mass flux through the wall is zero.

Layout of the state F: [node, species, N, N, N], node = element*(P+1) + i.
"""
import math

import numpy as np

from .quadrature import velocity_grid


def gll_nodes(P):
    """P+1 Gauss-Lobatto-Legendre nodes on [-1, 1]: the endpoints and the
    roots of P_P' (numpy supplies the polynomial roots)."""
    if P == 0:
        raise ValueError("P >= 1")
    inner = np.polynomial.legendre.Legendre.basis(P).deriv().roots()
    return np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])


def _norm_legendre(n, x):
    """Orthonormal Legendre P~_n(x) = sqrt((2n+1)/2) P_n(x) and derivative."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    p = np.polynomial.legendre.legval(x, c)
    dp = np.polynomial.legendre.legval(x, np.polynomial.legendre.legder(c))
    s = math.sqrt((2 * n + 1) / 2.0)
    return s * p, s * dp


def dg_operators(P):
    """(r, Minv, Dr): GLL nodes, inverse mass matrix (Minv = V V^T) and the
    nodal differentiation matrix Dr = Vr V^{-1}."""
    r = gll_nodes(P)
    V = np.zeros((P + 1, P + 1))
    Vr = np.zeros((P + 1, P + 1))
    for j in range(P + 1):
        V[:, j], Vr[:, j] = _norm_legendre(j, r)
    Minv = V @ V.T
    Dr = Vr @ np.linalg.inv(V)
    return r, Minv, Dr


def advect_rhs(u, cx, h, Minv, Dr, ghost_left, ghost_right):
    """DG right-hand side of u_t + cx u_x = 0.

    u: [K, P+1, ...] nodal values (trailing axes = independent velocity
    points), cx broadcastable to u[0, 0].  ghost_left / ghost_right are the
    exterior states at x = 0 and x = 1 (used only where they are upwind)."""
    K, Pp1 = u.shape[0], u.shape[1]
    du = -(2.0 / h) * cx * np.einsum("ij,kj...->ki...", Dr, u)
    # traces: left neighbour's right node and the element's left node
    uL = np.concatenate([ghost_left[None], u[:, -1]], axis=0)   # faces 0..K
    uR = np.concatenate([u[:, 0], ghost_right[None]], axis=0)
    Fstar = np.where(cx > 0, cx * uL, cx * uR)                   # [K+1, ...]
    termR = cx * u[:, -1] - Fstar[1:]
    termL = -(cx * u[:, 0] - Fstar[:-1])
    for i in range(Pp1):
        du[:, i] += (2.0 / h) * (Minv[i, -1] * termR + Minv[i, 0] * termL)
    return du


def wall_maxwellian(N, L, m, uw, Tw):
    c, _ = velocity_grid(N, L)
    cx, cy, cz = np.meshgrid(c, c, c, indexing="ij")
    d2 = (cx - uw[0]) ** 2 + (cy - uw[1]) ** 2 + (cz - uw[2]) ** 2
    return (m / (math.pi * Tw)) ** 1.5 * np.exp(-m * d2 / Tw)


def diffuse_ghost(f_trace, cx, Mw, inflow_positive):
    """Wall-emitted distribution n_w M_w on the inflow half, with n_w from
    zero discrete net mass flux.  inflow_positive: the wall emits c_x > 0
    (left wall) or c_x < 0 (right wall).  Outflow half of the ghost is the
    interior trace (it is never upwind)."""
    if inflow_positive:
        out_flux = -np.sum(np.where(cx < 0, cx * f_trace, 0.0))
        in_unit = np.sum(np.where(cx > 0, cx * Mw, 0.0))
        return np.where(cx > 0, out_flux / in_unit * Mw, f_trace)
    out_flux = np.sum(np.where(cx > 0, cx * f_trace, 0.0))
    in_unit = -np.sum(np.where(cx < 0, cx * Mw, 0.0))
    return np.where(cx < 0, out_flux / in_unit * Mw, f_trace)


class Couette1D:
    """Transport part of the 1-D-x problem of Sec. 3.3 (two diffuse walls at
    x = 0 and x = 1) plus a collision callback.

    collision(F) -> dF/dt from collisions, same layout as F, or None."""

    def __init__(self, N, L, masses, K, P, u_left, u_right, T_left=1.0, T_right=1.0):
        self.N, self.L, self.masses, self.K, self.P = N, L, list(masses), K, P
        self.h = 1.0 / K
        self.r, self.Minv, self.Dr = dg_operators(P)
        c, _ = velocity_grid(N, L)
        self.cx = np.meshgrid(c, c, c, indexing="ij")[0]
        self.Mw_left = [wall_maxwellian(N, L, m, u_left, T_left) for m in masses]
        self.Mw_right = [wall_maxwellian(N, L, m, u_right, T_right) for m in masses]

    def node_x(self):
        xe = np.arange(self.K) * self.h
        return (xe[:, None] + 0.5 * (self.r[None, :] + 1.0) * self.h).ravel()

    def transport_rhs(self, F):
        K, Pp1, N = self.K, self.P + 1, self.N
        ns = len(self.masses)
        out = np.zeros_like(F)
        U = F.reshape(K, Pp1, ns, N, N, N)
        O = out.reshape(K, Pp1, ns, N, N, N)
        for p in range(ns):
            u = U[:, :, p]
            gl = diffuse_ghost(u[0, 0], self.cx, self.Mw_left[p], True)
            gr = diffuse_ghost(u[-1, -1], self.cx, self.Mw_right[p], False)
            O[:, :, p] = advect_rhs(u, self.cx, self.h, self.Minv, self.Dr, gl, gr)
        return out

    def rhs(self, F, collision=None):
        out = self.transport_rhs(F)
        if collision is not None:
            out = out + collision(F)
        return out


def ssp_rk3(F, dt, rhs):
    """One Shu-Osher SSP-RK3 step."""
    F1 = F + dt * rhs(F)
    F2 = 0.75 * F + 0.25 * (F1 + dt * rhs(F1))
    return F / 3.0 + 2.0 / 3.0 * (F2 + dt * rhs(F2))
