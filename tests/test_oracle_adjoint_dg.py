"""Pins of the oracle's adjoint (brute-force Jacobian, finite differences) and
of its DG transport and SSP-RK3 (exact polynomial identities, convergence on
a smooth problem, zero wall mass flux, third-order accuracy)."""
import math

import numpy as np
import pytest

from oracle import dg
from oracle.adjoint import collide_vjp
from oracle.collide import PairPlan, collide
from oracle.quadrature import sphere_set


def _plan(N, alpha=1.0, mp=1.0, mq=2.5, nyquist_zero=False):
    s, w = sphere_set("icosahedron")
    return PairPlan(N, 5.0, mp, mq, 0.7, alpha, 3, s, w, R=4.0, nyquist_zero=nyquist_zero)


@pytest.mark.parametrize("alpha,nyq", [(1.0, False), (1.4, False), (1.0, True), (1.4, True)])
def test_vjp_equals_bruteforce_jacobian(alpha, nyq):
    """Q is linear in each argument, so the Jacobian's columns are Q(e_j, g)
    and Q(f, e_j); the VJP must equal J^T wbar (also for the variant whose
    gain drops the Nyquist planes)."""
    N = 4
    rng = np.random.default_rng(3)
    pl = _plan(N, alpha, nyquist_zero=nyq)
    f, g, wb = rng.random((N,) * 3), rng.random((N,) * 3), rng.standard_normal((N,) * 3)
    n3 = N ** 3
    Jf = np.zeros((n3, n3))
    Jg = np.zeros((n3, n3))
    for j in range(n3):
        e = np.zeros(n3)
        e[j] = 1.0
        e = e.reshape((N,) * 3)
        Jf[:, j] = collide(pl, e, g).ravel()
        Jg[:, j] = collide(pl, f, e).ravel()
    gf, gg = collide_vjp(pl, f, g, wb)
    assert np.max(np.abs(gf.ravel() - Jf.T @ wb.ravel())) < 1e-12 * np.max(np.abs(gf))
    assert np.max(np.abs(gg.ravel() - Jg.T @ wb.ravel())) < 1e-12 * np.max(np.abs(gg))


def test_vjp_central_differences():
    """Bilinear map: the central difference is exact up to rounding."""
    N = 6
    rng = np.random.default_rng(5)
    pl = _plan(N)
    f, g, wb = rng.random((N,) * 3), rng.random((N,) * 3), rng.standard_normal((N,) * 3)
    gf, gg = collide_vjp(pl, f, g, wb)
    for _ in range(4):
        d = rng.standard_normal((N,) * 3)
        eps = 1e-3
        fd_f = (np.sum(wb * collide(pl, f + eps * d, g)) - np.sum(wb * collide(pl, f - eps * d, g))) / (2 * eps)
        fd_g = (np.sum(wb * collide(pl, f, g + eps * d)) - np.sum(wb * collide(pl, f, g - eps * d))) / (2 * eps)
        assert abs(fd_f - np.sum(gf * d)) < 1e-10 * max(1.0, abs(fd_f))
        assert abs(fd_g - np.sum(gg * d)) < 1e-10 * max(1.0, abs(fd_g))


def test_gll_nodes_closed_form():
    r = dg.gll_nodes(3)
    assert np.allclose(r, [-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], atol=1e-15)
    r = dg.gll_nodes(2)
    assert np.allclose(r, [-1, 0, 1], atol=1e-15)


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_dg_operators_exact_on_polynomials(P):
    r, Minv, Dr = dg.dg_operators(P)
    for k in range(P + 1):
        assert np.allclose(Dr @ r ** k, k * r ** max(k - 1, 0) if k else 0 * r, atol=1e-12)
    Mass = np.linalg.inv(Minv)
    # mass matrix integrates products of nodal polynomials exactly
    xg, wg = np.polynomial.legendre.leggauss(P + 2)
    from numpy.polynomial import polynomial as Pn
    Vg = np.zeros((len(xg), P + 1))
    for j in range(P + 1):
        e = np.zeros(P + 1)
        e[j] = 1.0
        coeff = np.polyfit(r, e, P)
        Vg[:, j] = np.polyval(coeff, xg)
    assert np.allclose(Mass, Vg.T @ (wg[:, None] * Vg), atol=1e-12)


def _advect_error(K, P, c, T=0.25):
    """u_t + c u_x = 0 on [0,1], exact u = sin(2 pi (x - c t)) + 2, inflow
    boundary values taken from the exact solution; SSP-RK3 with a small dt."""
    r, Minv, Dr = dg.dg_operators(P)
    h = 1.0 / K
    x = (np.arange(K)[:, None] * h + 0.5 * (r[None, :] + 1) * h)
    exact = lambda t: np.sin(2 * math.pi * (x - c * t)) + 2.0
    bnd = lambda xx, t: np.sin(2 * math.pi * (xx - c * t)) + 2.0
    u = exact(0.0)
    dt = 0.05 * h / abs(c) / (P + 1) ** 2
    n = int(math.ceil(T / dt))
    dt = T / n
    t = 0.0
    cx = np.array(c)
    for _ in range(n):
        tt = [t]

        def rhs(v, tt=tt):
            return dg.advect_rhs(v, cx, h, Minv, Dr, np.array(bnd(0.0, tt[0])), np.array(bnd(1.0, tt[0])))
        # SSP-RK3 with the boundary data at the stage times
        u1 = u + dt * rhs(u)
        tt[0] = t + dt
        u2 = 0.75 * u + 0.25 * (u1 + dt * rhs(u1))
        tt[0] = t + 0.5 * dt
        u = u / 3.0 + 2.0 / 3.0 * (u2 + dt * rhs(u2))
        t += dt
    return np.max(np.abs(u - exact(T)))


@pytest.mark.parametrize("c", [1.0, -0.7])
def test_dg_advection_converges(c):
    P = 2
    e = [_advect_error(K, P, c) for K in (4, 8, 16)]
    rates = [math.log2(a / b) for a, b in zip(e, e[1:])]
    assert min(rates) > P + 0.5, (e, rates)


def test_diffuse_wall_zero_net_mass_flux():
    from oracle.quadrature import velocity_grid
    N, L = 8, 5.0
    c, _ = velocity_grid(N, L)
    cx = np.meshgrid(c, c, c, indexing="ij")[0]
    rng = np.random.default_rng(2)
    f = rng.random((N, N, N))
    Mw = dg.wall_maxwellian(N, L, 2.0, (0, -0.5, 0), 1.0)
    for left in (True, False):
        gh = dg.diffuse_ghost(f, cx, Mw, left)
        # the upwind state: ghost on the inflow half, interior elsewhere
        inflow = cx > 0 if left else cx < 0
        up = np.where(inflow, gh, f)
        assert abs(np.sum(cx * up)) < 1e-13 * np.sum(np.abs(cx * f))


def test_ssp_rk3_third_order():
    lam = -1.3
    errs = []
    for n in (20, 40, 80):
        dt = 1.0 / n
        y = np.array(1.0)
        for _ in range(n):
            y = dg.ssp_rk3(y, dt, lambda v: lam * v)
        errs.append(abs(y - math.exp(lam)))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert min(rates) > 2.9, rates


@pytest.mark.parametrize("sphere,symmetric", [("icosahedron", True), ("octahedron", True), ("fibonacci", False)])
def test_gain_part_is_symmetric_for_antipodal_sets(sphere, symmetric):
    """For p == q and a sphere set closed under sigma -> -sigma (equal
    weights) the gain part of Q(f, g) is a symmetric bilinear form, so at
    f == g its derivatives along any direction d with respect to f and to g
    agree (the adjoint then needs one side's gain sums only).  Checked by
    central differences of the oracle's gain part, which is exact for a
    bilinear map up to rounding; a Fibonacci set is not antipodal and the
    two differ."""
    from oracle.collide import PairPlan, collide_gain_loss
    from oracle.quadrature import sphere_set
    N, L = 6, 4.0
    s, w = sphere_set(sphere, 7 if sphere == "fibonacci" else None)
    pl = PairPlan(N, L, 1.0, 1.0, 0.6, 1.0, 3, s, w, R=5.0)
    rng = np.random.default_rng(5)
    f = rng.random((N, N, N))
    wb = rng.standard_normal((N, N, N))
    d = rng.standard_normal((N, N, N))

    def gain(a, b):
        return collide_gain_loss(pl, a, b)[0]
    e = 1e-3
    df = float(((gain(f + e * d, f) - gain(f - e * d, f)) * wb).sum() / (2 * e))
    dg = float(((gain(f, f + e * d) - gain(f, f - e * d)) * wb).sum() / (2 * e))
    if symmetric:
        assert abs(df - dg) <= 1e-10 * abs(df)
    else:
        assert abs(df - dg) > 1e-3 * abs(df)


# ------------------------------------------------------------ 2-D box transport
def test_box2d_reduces_to_the_1d_operator():
    """Periodic in y with data independent of y: the 2-D transport equals the
    pinned 1-D-x operator with the same walls at every y-node."""
    N, L, masses, K, P = 6, 4.0, [1.0, 2.0], 5, 2
    walls = {"left": ((0, -0.5, 0), 1.0), "right": ((0, 0.5, 0), 1.3)}
    box = dg.Box2D(N, L, masses, K, 3, P, periodic=(False, True), walls=walls)
    line = dg.Couette1D(N, L, masses, K, P, (0, -0.5, 0), (0, 0.5, 0), 1.0, 1.3)
    rng = np.random.default_rng(7)
    F1 = rng.random((K * (P + 1), 2, N, N, N)) + 0.5
    # replicate along y: node ((ey Kx + ex)(P+1) + j)(P+1) + i <- 1-D node ex(P+1) + i
    U1 = F1.reshape(K, P + 1, 2, N, N, N)
    F2 = np.broadcast_to(U1[None, :, None], (3, K, P + 1, P + 1, 2, N, N, N)).reshape(-1, 2, N, N, N).copy()
    d1 = line.transport_rhs(F1).reshape(K, P + 1, 2, N, N, N)
    d2 = box.transport_rhs(F2).reshape(3, K, P + 1, P + 1, 2, N, N, N)
    ref = np.broadcast_to(d1[None, :, None], d2.shape)
    assert np.max(np.abs(d2 - ref)) <= 1e-13 * np.max(np.abs(d1))


def _box_advect_error(K, P, T=0.25):
    """f_t + c_x f_x + c_y f_y = 0 on the periodic unit square for the eight
    velocities of an N = 2 grid (c = +-0.5 per axis): the exact solution is
    the initial data translated by c t."""
    N, L = 2, 1.0
    box = dg.Box2D(N, L, [1.0], K, K, P, periodic=(True, True))
    xy = box.node_xy()
    cx, cy = box.cx, box.cy

    def exact(t):
        x = xy[:, 0][:, None, None, None] - cx[None] * t
        y = xy[:, 1][:, None, None, None] - cy[None] * t
        return (np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y) + 2.0)[:, None]
    F = exact(0.0)
    h = 1.0 / K
    dt = 0.05 * h / 0.5 / (P + 1) ** 2
    n = int(math.ceil(T / dt))
    for _ in range(n):
        F = dg.ssp_rk3(F, T / n, box.transport_rhs)
    return np.max(np.abs(F - exact(T)))


def test_box2d_advection_converges():
    P = 2
    e = [_box_advect_error(K, P) for K in (4, 8, 16)]
    rates = [math.log2(a / b) for a, b in zip(e, e[1:])]
    assert min(rates) > P + 0.5, (e, rates)


def test_box2d_closed_box_conserves_mass():
    """Four diffuse walls (each node's inflow carries its outflow): the DG
    mass of every species, sum over nodes of w_i w_j hx hy / 4 times the
    velocity sum, does not change under the transport."""
    N, L, K, P = 6, 4.0, 3, 1
    walls = {"left": ((0, -0.3, 0), 1.0), "right": ((0, 0.4, 0), 1.2),
             "bottom": ((0.2, 0, 0), 0.9), "top": ((-0.1, 0, 0.1), 1.1)}
    box = dg.Box2D(N, L, [1.0, 3.0], K, 2, P, extent=((0.0, 1.5), (0.0, 1.0)),
                   periodic=(False, False), walls=walls)
    rng = np.random.default_rng(9)
    F = rng.random((box.n_nodes(), 2, N, N, N)) + 0.1
    d = box.transport_rhs(F)
    w = np.array([1.0, 1.0])               # GLL weights for P = 1 (the trapezoid rule)
    wn = np.outer(w, w).ravel()            # weights of (j, i)
    wt = np.tile(wn, 3 * 2) * box.hx * box.hy / 4.0
    for p in range(2):
        rate = np.sum(wt[:, None] * d[:, p].reshape(box.n_nodes(), -1))
        scale = np.sum(wt[:, None] * np.abs(d[:, p]).reshape(box.n_nodes(), -1))
        assert abs(rate) < 1e-13 * scale, (p, rate, scale)
