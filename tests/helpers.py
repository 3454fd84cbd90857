"""Shared test helpers: build the oracle's and the library's plans from the
same workload parameters."""
import numpy as np

from oracle.collide import PairPlan
from oracle.quadrature import sphere_set


def oracle_pairs(cfg, gamma=None, eta=None, beta=None, nyquist_zero=False):
    ns = cfg["ns"]
    s, w = sphere_set(cfg["sphere"], cfg["M"])
    plans = [[None] * ns for _ in range(ns)]
    for p in range(ns):
        for q in range(ns):
            plans[p][q] = PairPlan(cfg["N"], cfg["L"], cfg["masses"][p], cfg["masses"][q],
                                   cfg["omega"][p][q], cfg["alpha"][p][q], cfg["Nrho"], s, w,
                                   R=cfg["R"][p][q], gamma=gamma, eta=eta,
                                   beta=None if beta is None else beta[p][q],
                                   nyquist_zero=nyquist_zero)
    return plans


def gpu_plan(cfg, precision="fp64", dg_order=0, beta=None, nyquist_zero=False):
    from paper_1903_04670_amd import dgfs
    return dgfs.Plan(cfg["masses"], cfg["omega"], cfg["alpha"], cfg["N"], cfg["L"], cfg["Nrho"],
                     sphere=cfg["sphere"], M=cfg["M"], S=cfg["S"], R=cfg["R"], beta=beta,
                     dg_order=dg_order, precision=precision, nyquist_zero=nyquist_zero)


def rel_linf(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def small_config(N, ns=2, M_kind="icosahedron", Nrho=3, seed=0, n_nodes=1, masses=None, S=2.5):
    """A small synthetic workload for parity at sizes the oracle runs in
    well under a second."""
    from paper_1903_04670_amd import workloads as wl
    rng = np.random.default_rng(seed)
    L, R = wl.box_for_support(S)
    masses = masses or [1.0, 2.5, 4.0, 1.5][:ns]
    F = np.empty((n_nodes, ns, N, N, N))
    for i in range(n_nodes):
        for p in range(ns):
            F[i, p] = wl.mixture_maxwellians(rng, N, L, masses[p], 2) * (1 + 0.05 * rng.uniform(-1, 1, (N, N, N)))
    om = rng.uniform(0.5, 1.0, (ns, ns))
    om = 0.5 * (om + om.T)
    M = {"octahedron": 6, "icosahedron": 12}.get(M_kind, 7)
    return dict(ns=ns, masses=masses, omega=om, alpha=np.ones((ns, ns)), N=N, L=L, S=S,
                R=np.full((ns, ns), R), sphere=M_kind, M=M, Nrho=Nrho, F=F, n_nodes=n_nodes)
