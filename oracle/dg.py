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


class Box2D:
    """Transport part in two space dimensions, x and y: the extension of the
    1-D-x scheme above that Sec. 3.3 leaves to future work (its footnote on
    higher spatial dimensions).  Kx x Ky uniform rectangles on
    [x0, x1] x [y0, y1], tensor-product GLL nodes ((P+1)^2 per element),
    upwind flux on every face.  Each direction is periodic or bounded by two
    Maxwell diffuse walls (walls = {"left": (u_w, T_w), "right": ..,
    "bottom": .., "top": ..}).

    With the exact mass matrices of the tensor basis, the strong form
    separates: the right-hand side is the 1-D operator of advect_rhs along
    every x-line of nodes (fixed element row and local j) with velocity c_x,
    plus the same along every y-line with c_y.  A diffuse-wall node emits
    n_w M_w on its inflow half with n_w from zero net mass flux through that
    node.

    Layout of F: [node, species, N, N, N],
    node = ((ey Kx + ex)(P+1) + j)(P+1) + i, i along x and j along y."""

    def __init__(self, N, L, masses, Kx, Ky, P, extent=((0.0, 1.0), (0.0, 1.0)),
                 periodic=(False, True), walls=None):
        self.N, self.L, self.masses = N, L, list(masses)
        self.Kx, self.Ky, self.P = Kx, Ky, P
        (self.x0, self.x1), (self.y0, self.y1) = extent
        self.hx, self.hy = (self.x1 - self.x0) / Kx, (self.y1 - self.y0) / Ky
        self.periodic = tuple(bool(v) for v in periodic)
        self.r, self.Minv, self.Dr = dg_operators(P)
        c, _ = velocity_grid(N, L)
        cx, cy, _ = np.meshgrid(c, c, c, indexing="ij")
        self.cx, self.cy = cx, cy
        walls = walls or {}
        self.Mw = {side: [wall_maxwellian(N, L, m, uw, Tw) for m in masses]
                   for side, (uw, Tw) in walls.items()}
        for side, per in (("left", 0), ("right", 0), ("bottom", 1), ("top", 1)):
            if not self.periodic[per] and side not in self.Mw:
                raise ValueError("no wall given for the %s side" % side)

    def n_nodes(self):
        return self.Kx * self.Ky * (self.P + 1) ** 2

    def node_xy(self):
        """(x, y) of every node in node order."""
        r = self.r
        out = np.zeros((self.Ky, self.Kx, self.P + 1, self.P + 1, 2))
        for ey in range(self.Ky):
            for ex in range(self.Kx):
                xs = self.x0 + (ex + 0.5 * (r + 1.0)) * self.hx
                ys = self.y0 + (ey + 0.5 * (r + 1.0)) * self.hy
                out[ey, ex, :, :, 0] = xs[None, :]
                out[ey, ex, :, :, 1] = ys[:, None]
        return out.reshape(-1, 2)

    def _line(self, u, c, h, periodic, Mw_lo, Mw_hi):
        """advect_rhs along one line u [K, P+1, N, N, N] with velocity c;
        ghosts from periodicity or the two diffuse walls."""
        if periodic:
            gl, gr = u[-1, -1], u[0, 0]
        else:
            gl = diffuse_ghost(u[0, 0], c, Mw_lo, True)
            gr = diffuse_ghost(u[-1, -1], c, Mw_hi, False)
        return advect_rhs(u, c, h, self.Minv, self.Dr, gl, gr)

    def transport_rhs(self, F):
        Kx, Ky, Pp1, N = self.Kx, self.Ky, self.P + 1, self.N
        ns = len(self.masses)
        U = F.reshape(Ky, Kx, Pp1, Pp1, ns, N, N, N)
        out = np.zeros_like(U)
        for p in range(ns):
            ml, mr = self.Mw.get("left", [None] * ns)[p], self.Mw.get("right", [None] * ns)[p]
            mb, mt = self.Mw.get("bottom", [None] * ns)[p], self.Mw.get("top", [None] * ns)[p]
            for ey in range(Ky):
                for j in range(Pp1):
                    u = U[ey, :, j, :, p]                        # [Kx, P+1 (i), ...]
                    out[ey, :, j, :, p] += self._line(u, self.cx, self.hx, self.periodic[0], ml, mr)
            for ex in range(Kx):
                for i in range(Pp1):
                    u = U[:, ex, :, i, p]                        # [Ky, P+1 (j), ...]
                    out[:, ex, :, i, p] += self._line(u, self.cy, self.hy, self.periodic[1], mb, mt)
        return out.reshape(F.shape)

    def rhs(self, F, collision=None):
        out = self.transport_rhs(F)
        if collision is not None:
            out = out + collision(F)
        return out
