"""Discretisation inputs of the collision operator (oracle; test infrastructure).

Velocity grid, Fourier wave index, radial Gauss-Legendre rule, sphere
quadratures and the truncation radius, as used by Algorithm 1 and Sec. 2.1
of the paper.
"""
import math

import numpy as np


def velocity_grid(N, L):
    """Cell-centred uniform grid on [-L, L] (Sec. 2.1, domain D_L).

    The paper does not state the offset; the cell-centred reading
    c_j = -L + (j + 1/2) h, h = 2L/N is used.  Returns (c, h) with c of
    length N.
    """
    h = 2.0 * L / N
    c = -L + (np.arange(N) + 0.5) * h
    return c, h


def wave_index(N):
    """v_x = x - N [x >= N/2] for x = 0..N-1 (Algorithm 1, first loop)."""
    x = np.arange(N)
    return x - N * (x >= N // 2)


def wave_grid(N):
    """l = ndgrid(v): three N^3 integer arrays (Algorithm 1)."""
    v = wave_index(N)
    return np.meshgrid(v, v, v, indexing="ij")


def gauss_legendre(n, R):
    """Gauss-Legendre nodes/weights on [0, R], nodes ascending (Algorithm 1
    input rho, w_rho).  numpy's leggauss supplies the rule on [-1, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * R * (x + 1.0), 0.5 * R * w


def sphere_set(kind, M=None):
    """Equal-weight quadratures on the full unit sphere (weights 4 pi / M).

    'octahedron'  : +-e_x, +-e_y, +-e_z (M = 6)
    'icosahedron' : cyclic permutations of (0, +-1, +-phi), normalised (M = 12)
    'fibonacci'   : z_i = 1 - (2i+1)/M, azimuth i*pi*(3 - sqrt 5)
    The paper counts M on the full sphere in Table 1; the same reading is
    used everywhere.  Returns (sigma [M,3], w [M]).
    """
    if kind == "octahedron":
        s = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0],
                      [0, 0, 1], [0, 0, -1]], dtype=float)
    elif kind == "icosahedron":
        phi = 0.5 * (1.0 + math.sqrt(5.0))
        pts = []
        for a in (1.0, -1.0):
            for b in (phi, -phi):
                pts.append((0.0, a, b))
                pts.append((a, b, 0.0))
                pts.append((b, 0.0, a))
        s = np.array(pts) / math.sqrt(1.0 + phi * phi)
    elif kind == "fibonacci":
        i = np.arange(M)
        z = 1.0 - (2.0 * i + 1.0) / M
        az = i * math.pi * (3.0 - math.sqrt(5.0))
        rxy = np.sqrt(1.0 - z * z)
        s = np.stack([rxy * np.cos(az), rxy * np.sin(az), z], axis=1)
    else:
        raise ValueError(kind)
    if M is not None and len(s) != M:
        raise ValueError("sphere set %s has %d points, asked %d" % (kind, len(s), M))
    return s, np.full(len(s), 4.0 * math.pi / len(s))


def truncation_radius(L, mp, mq):
    """R = 4L / (1 + max(4 m_q/(m_p+m_q), 2) + sqrt(1 + m_q/m_p)) (Sec. 2.1,
    truncation of the u integral to the ball B_R)."""
    return 4.0 * L / (1.0 + max(4.0 * mq / (mp + mq), 2.0) + math.sqrt(1.0 + mq / mp))
