"""Seeded synthetic inputs for the collision operator and the DG solver.

This module only draws and shapes inputs: parameter sets of the five
workloads and distribution functions built from Maxwellians on the uniform
cell-centred velocity grid c_j = -L + (j + 1/2) h, h = 2L/N.  It holds none
of the collision method's arithmetic and imports nothing from the library or
from the CPU reference, so both may be fed from it.

Maxwellian (non-dimensional, characteristic speed sqrt(2 k_B T0 / m0)):
    M(c; m, n, u, T) = n (m / (pi T))^{3/2} exp(-m |c - u|^2 / T).
"""
import math

import numpy as np

SQ2 = math.sqrt(2.0)


def box_for_support(S):
    """(L, R) = ((3 + sqrt 2) S / 2, 2 S) for a support radius S."""
    return (3.0 + SQ2) * S / 2.0, 2.0 * S


def grid(N, L):
    h = 2.0 * L / N
    return -L + (np.arange(N) + 0.5) * h


def maxwellian(N, L, m, n=1.0, u=(0.0, 0.0, 0.0), T=1.0):
    c = grid(N, L)
    cx, cy, cz = np.meshgrid(c, c, c, indexing="ij")
    d2 = (cx - u[0]) ** 2 + (cy - u[1]) ** 2 + (cz - u[2]) ** 2
    return n * (m / (math.pi * T)) ** 1.5 * np.exp(-m * d2 / T)


def _sym(ns, vals):
    """Symmetric ns x ns matrix from the upper triangle listed row-wise."""
    A = np.zeros((ns, ns))
    it = iter(vals)
    for p in range(ns):
        for q in range(p, ns):
            A[p, q] = A[q, p] = next(it)
    return A


# ---------------------------------------------------------------- workloads
def homogeneous_single():
    """Single species, one spatial point, N = 16, octahedron M = 6,
    N_rho = 8, S = 3.5 (R = 7), omega = 0.5, alpha = 1; f = half-density
    Maxwellians at bulk velocity +-e_x, T = 1; one Euler step dt = 0.01."""
    S = 3.5
    L, R = box_for_support(S)
    N = 16
    f0 = maxwellian(N, L, 1.0, 0.5, (1.0, 0.0, 0.0), 1.0) + \
        maxwellian(N, L, 1.0, 0.5, (-1.0, 0.0, 0.0), 1.0)
    return dict(name="homogeneous N=16 M=6 Nrho=8", ns=1, masses=[1.0],
                omega=np.full((1, 1), 0.5), alpha=np.ones((1, 1)), N=N, L=L,
                S=S, R=np.full((1, 1), R), sphere="octahedron", M=6, Nrho=8,
                dt=0.01, F=f0[None, None].copy(), n_nodes=1)


def couette_two_species(seed=2, K=16, P=3, N=32, Nrho=16):
    """Two-species 1-D-x Couette flow: masses (1, 2), omega (0.5, 0.6, 0.7)
    for pairs (11, 12, 22), N = 32, S = 4 (R = 8), icosahedron M = 12,
    N_rho = 16, K = 16 elements on [0, 1] with P = 3 (64 GLL nodes), diffuse
    walls at x = 0 (u = (0, -0.5, 0)) and x = 1 (u = (0, +0.5, 0)), T_w = 1;
    f^p = M_p(n=1, u=0, T=1) (1 + 0.01 U(-1, 1)) drawn i.i.d.; SSP-RK3,
    dt = 1e-3."""
    S = 4.0
    L, R = box_for_support(S)
    masses = [1.0, 2.0]
    rng = np.random.default_rng(seed)
    n_nodes = K * (P + 1)
    F = np.empty((n_nodes, 2, N, N, N))
    for p, m in enumerate(masses):
        base = maxwellian(N, L, m)
        F[:, p] = base[None] * (1.0 + 0.01 * rng.uniform(-1.0, 1.0, (n_nodes, N, N, N)))
    return dict(name="couette 2 species N=%d M=12 Nrho=%d K=%d P=%d" % (N, Nrho, K, P),
                ns=2, masses=masses, omega=_sym(2, [0.5, 0.6, 0.7]),
                alpha=np.ones((2, 2)), N=N, L=L, S=S, R=np.full((2, 2), R),
                sphere="icosahedron", M=12, Nrho=Nrho, K=K, P=P,
                u_left=(0.0, -0.5, 0.0), u_right=(0.0, 0.5, 0.0), T_wall=1.0,
                dt=1e-3, steps=100, F=F, n_nodes=n_nodes)


def differentiation(seed=4, n_nodes=256, N=32, Nrho=16):
    """256 nodes, masses (1, 2.5), omega (0.5, 0.6, 0.7), N = 32, S = 4,
    icosahedron M = 12, N_rho = 16; f^p = M_p (1 + 0.05 U(-1, 1));
    cotangent w ~ N(0, 1) per output entry."""
    S = 4.0
    L, R = box_for_support(S)
    masses = [1.0, 2.5]
    rng = np.random.default_rng(seed)
    F = np.empty((n_nodes, 2, N, N, N))
    for p, m in enumerate(masses):
        F[:, p] = maxwellian(N, L, m)[None] * (1.0 + 0.05 * rng.uniform(-1, 1, (n_nodes, N, N, N)))
    W = rng.standard_normal((n_nodes, 2, N, N, N))
    return dict(name="vjp 2 species N=%d M=12 Nrho=%d" % (N, Nrho), ns=2,
                masses=masses, omega=_sym(2, [0.5, 0.6, 0.7]), alpha=np.ones((2, 2)),
                N=N, L=L, S=S, R=np.full((2, 2), R), sphere="icosahedron", M=12,
                Nrho=Nrho, F=F, W=W, n_nodes=n_nodes)


def mixture_maxwellians(rng, N, L, m, J, n_rng=(0.2, 1.0), u_rng=(-1.0, 1.0), T_rng=(0.5, 2.0)):
    f = np.zeros((N, N, N))
    for _ in range(J):
        n = rng.uniform(*n_rng)
        u = rng.uniform(u_rng[0], u_rng[1], 3)
        T = rng.uniform(*T_rng)
        f += maxwellian(N, L, m, n, u, T)
    return f


def batched_instances(seed=3, n_inst=1024, Ns=(16, 24, 32)):
    """Space-homogeneous instances of uneven size: N in Ns, species count in
    {1, 2, 3}, masses U[1, 4], omega_pq U[0.5, 1] (symmetric), alpha = 1,
    N_rho in {8, 16}, icosahedron M = 12, S = 4; each f is a sum of J in
    {1, 2, 3} Maxwellians with n U[0.2, 1], u U[-1, 1]^3, T U[0.5, 2]."""
    rng = np.random.default_rng(seed)
    S = 4.0
    L, R = box_for_support(S)
    out = []
    for _ in range(n_inst):
        N = int(rng.choice(Ns))
        ns = int(rng.integers(1, 4))
        masses = list(rng.uniform(1.0, 4.0, ns))
        om = rng.uniform(0.5, 1.0, ns * (ns + 1) // 2)
        Nrho = int(rng.choice([8, 16]))
        F = np.stack([mixture_maxwellians(rng, N, L, masses[p], int(rng.integers(1, 4)))
                      for p in range(ns)])[None]
        out.append(dict(ns=ns, masses=masses, omega=_sym(ns, om), alpha=np.ones((ns, ns)),
                        N=N, L=L, S=S, R=np.full((ns, ns), R), sphere="icosahedron",
                        M=12, Nrho=Nrho, F=F, n_nodes=1))
    return out


def precision_vss(seed=5, n_nodes=512, N=48, M=32, Nrho=24):
    """Three species, masses (1, 2, 4), VSS alpha = 1.4, omega_pq U[0.6, 0.8],
    N = 48, Fibonacci M = 32, N_rho = 24, S = 4, 512 nodes; per node and
    species f = (sum of 2 Maxwellians, n U[0.5, 1], u U[-0.5, 0.5]^3,
    T U[0.8, 1.2]) (1 + 0.05 U(-1, 1))."""
    rng = np.random.default_rng(seed)
    S = 4.0
    L, R = box_for_support(S)
    masses = [1.0, 2.0, 4.0]
    om = _sym(3, rng.uniform(0.6, 0.8, 6))
    F = np.empty((n_nodes, 3, N, N, N))
    for i in range(n_nodes):
        for p, m in enumerate(masses):
            f = mixture_maxwellians(rng, N, L, m, 2, (0.5, 1.0), (-0.5, 0.5), (0.8, 1.2))
            F[i, p] = f * (1.0 + 0.05 * rng.uniform(-1, 1, (N, N, N)))
    return dict(name="vss 3 species N=%d M=%d Nrho=%d" % (N, M, Nrho), ns=3,
                masses=masses, omega=om, alpha=np.full((3, 3), 1.4), N=N, L=L, S=S,
                R=np.full((3, 3), R), sphere="fibonacci", M=M, Nrho=Nrho, F=F,
                n_nodes=n_nodes)
