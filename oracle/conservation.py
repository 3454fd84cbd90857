"""Moments and the conservation projection (oracle; test infrastructure).

The collision operator conserves the mass of each species and the total
momentum and energy of the mixture (Sec. 2: the post-collision velocities
conserve momentum and energy).  The discrete operator does so only to the
accuracy of its quadratures.  The projection restores the invariants exactly
by the smallest L2 change: with the constraint matrix C (rows: mass of each
species, total momentum in x, y, z, total energy, each a quadrature with
weight h^3 on the grid),
    Q_tilde = Q - C^T (C C^T)^{-1} C Q .
Arrays: Q has shape [ns, N, N, N].
"""
import numpy as np

from .quadrature import velocity_grid


def constraint_rows(N, L, masses):
    """C as an array [ns + 4, ns, N, N, N]."""
    c, h = velocity_grid(N, L)
    cx, cy, cz = np.meshgrid(c, c, c, indexing="ij")
    ns = len(masses)
    w = h ** 3
    C = np.zeros((ns + 4, ns, N, N, N))
    for p, m in enumerate(masses):
        C[p, p] = w
        C[ns + 0, p] = w * m * cx
        C[ns + 1, p] = w * m * cy
        C[ns + 2, p] = w * m * cz
        C[ns + 3, p] = w * 0.5 * m * (cx * cx + cy * cy + cz * cz)
    return C


def moments(Q, N, L, masses):
    """C Q: [mass_1..mass_ns, momentum x, y, z, energy]."""
    C = constraint_rows(N, L, masses)
    return np.tensordot(C, Q, axes=4)


def project(Q, N, L, masses, rows="all"):
    """Q - C^T (C C^T)^{-1} C Q (FP64, dense normal equations).  rows="mass"
    keeps only the mass rows of C (what a single cross-species term
    Q^{pq} conserves on its own)."""
    C = constraint_rows(N, L, masses)
    if rows == "mass":
        C = C[:len(masses)]
    elif rows != "all":
        raise ValueError(rows)
    k = C.shape[0]
    Cm = C.reshape(k, -1)
    lam = np.linalg.solve(Cm @ Cm.T, Cm @ Q.ravel())
    return Q - (Cm.T @ lam).reshape(Q.shape)
