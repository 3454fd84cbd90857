"""GPU parity of the VSS (alpha != 1) path: the Funk-Hecke gain table and the
per-direction gain pipeline against the oracle; at the three-species N = 48
size, the FP32-mixed path against FP64 and the projected conservation."""
import numpy as np
import pytest

from helpers import gpu_plan, oracle_pairs, rel_linf, small_config
from oracle import conservation as cons
from oracle.collide import collide as oracle_collide
from oracle.collide import mixture_collision

pytestmark = pytest.mark.gpu
TOL = 1e-11


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def vss_config(N, ns=2, kind="fibonacci", M=7, Nrho=3, seed=0, n_nodes=1, alpha=1.4):
    cfg = small_config(N, ns=ns, M_kind=kind, Nrho=Nrho, seed=seed, n_nodes=n_nodes)
    cfg["alpha"] = np.full((ns, ns), alpha)
    if kind == "fibonacci":
        cfg["M"] = M
    return cfg


@pytest.mark.parametrize("N,M,alpha", [(8, 7, 1.4), (6, 5, 0.8), (8, 7, 0.8)])
def test_vss_gain_table_matches_oracle(torch_cuda, N, M, alpha):
    cfg = vss_config(N, ns=2, M=M, alpha=alpha)
    pl = gpu_plan(cfg)
    opl = oracle_pairs(cfg)
    for p, q in [(0, 1), (1, 0)]:
        b = opl[p][q].b
        re = pl.table(p, q, 3).reshape(b.shape)
        im = pl.table(p, q, 4).reshape(b.shape)
        assert np.max(np.abs(re + 1j * im - b)) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("N,kind,M,alpha", [(8, "fibonacci", 7, 1.4), (12, "octahedron", 6, 1.36),
                                            (16, "icosahedron", 12, 1.32), (6, "fibonacci", 5, 1.4),
                                            (8, "fibonacci", 7, 0.8), (6, "fibonacci", 5, 0.8),
                                            (6, "octahedron", 6, 1.4), (6, "icosahedron", 12, 1.4),
                                            (12, "fibonacci", 5, 1.4), (4, "fibonacci", 5, 1.4),
                                            (10, "fibonacci", 5, 1.4), (14, "octahedron", 6, 1.3)])
def test_vss_collide_parity(torch_cuda, N, kind, M, alpha):
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = vss_config(N, ns=2, kind=kind, M=M, Nrho=4, seed=N, n_nodes=2, alpha=alpha)
    pl = gpu_plan(cfg)
    opl = oracle_pairs(cfg)
    F = torch.from_numpy(cfg["F"]).cuda()
    for p in range(2):
        for q in range(2):
            got = dgfs.collide(pl, p, q, F[:, p], F[:, q]).cpu().numpy()
            for i in range(2):
                ref = oracle_collide(opl[p][q], cfg["F"][i, p], cfg["F"][i, q])
                assert rel_linf(got[i], ref) <= TOL, (N, p, q, i)


def test_vss_radix5_grid_N40(torch_cuda):
    """A VSS plan (alpha = 1.3) on N = 40 = 8 x 5: one node, a cross pair and
    a self pair, octahedron, N_rho = 2, against the oracle at 1e-11 (its
    direction-dependent tables take about 20 s to build at this size)."""
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = vss_config(40, ns=2, kind="octahedron", Nrho=2, seed=40, n_nodes=1, alpha=1.3)
    pl = gpu_plan(cfg)
    opl = oracle_pairs(cfg)
    F = torch.from_numpy(cfg["F"]).cuda()
    for p, q in [(0, 1), (1, 1)]:
        got = dgfs.collide(pl, p, q, F[:, p], F[:, q]).cpu().numpy()
        ref = oracle_collide(opl[p][q], cfg["F"][0, p], cfg["F"][0, q])
        assert rel_linf(got[0], ref) <= TOL, (p, q)


def test_vss_radix7_grid_N56(torch_cuda):
    """A VSS plan (alpha = 1.3) on N = 56 = 8 x 7, where the gain kernels run
    one group of 2N lanes per block: one node, a cross pair and a self pair,
    octahedron, N_rho = 2, against the oracle at 1e-11."""
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = vss_config(56, ns=2, kind="octahedron", Nrho=2, seed=56, n_nodes=1, alpha=1.3)
    pl = gpu_plan(cfg)
    opl = oracle_pairs(cfg)
    F = torch.from_numpy(cfg["F"]).cuda()
    for p, q in [(0, 1), (1, 1)]:
        got = dgfs.collide(pl, p, q, F[:, p], F[:, q]).cpu().numpy()
        ref = oracle_collide(opl[p][q], cfg["F"][0, p], cfg["F"][0, q])
        assert rel_linf(got[0], ref) <= TOL, (p, q)


def _vss_cfg5_shape(n_nodes=1, Nrho=2):
    """The precision workload's collision shape (three species, masses 1, 2,
    4, alpha = 1.4, N = 48, Fibonacci M = 32) with N_rho = 2: the kernels'
    code paths depend on N and M, not on N_rho, and the oracle's VSS tables
    then take about 15 s per pair."""
    from paper_1903_04670_amd import workloads as wl
    return wl.precision_vss(n_nodes=n_nodes, Nrho=Nrho)


def _oracle_pair(cfg, p, q):
    from oracle.collide import PairPlan
    from oracle.quadrature import sphere_set
    s, w = sphere_set(cfg["sphere"], cfg["M"])
    return PairPlan(cfg["N"], cfg["L"], cfg["masses"][p], cfg["masses"][q], cfg["omega"][p][q],
                    cfg["alpha"][p][q], cfg["Nrho"], s, w, R=cfg["R"][p][q])


def test_vss_cfg5_shape_N48_against_oracle(torch_cuda):
    """N = 48, Fibonacci M = 32, alpha = 1.4, three species: a cross pair
    (masses 1 and 4) and a self pair, one node, FP64 against the oracle at
    1e-11 (k_gain_yz_vss and k_gain_x_vss at N = 48)."""
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = _vss_cfg5_shape()
    pl = gpu_plan(cfg)
    F = torch.from_numpy(cfg["F"]).cuda()
    for p, q in [(0, 2), (1, 1)]:
        got = dgfs.collide(pl, p, q, F[:, p], F[:, q]).cpu().numpy()
        ref = oracle_collide(_oracle_pair(cfg, p, q), cfg["F"][0, p], cfg["F"][0, q])
        err = rel_linf(got[0], ref)
        print("VSS N=48 M=32 (%d,%d): rel Linf %.3e" % (p, q, err))
        assert err <= TOL, (p, q, err)


def test_vss_cfg5_shape_N48_fp32_mixed_against_oracle(torch_cuda):
    """The same shape in FP32-mixed against the FP64 oracle, within the
    FP32 bounds stated for the VHS path: 2e-6 of the loss term, 5e-4 of Q."""
    from oracle.collide import collide_gain_loss
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = _vss_cfg5_shape()
    pl = gpu_plan(cfg, precision="fp32")
    F = torch.from_numpy(cfg["F"]).cuda()
    for p, q in [(0, 2), (1, 1)]:
        got = dgfs.collide(pl, p, q, F[:, p], F[:, q]).cpu().numpy()[0]
        gain, loss = collide_gain_loss(_oracle_pair(cfg, p, q), cfg["F"][0, p], cfg["F"][0, q])
        ref = gain - loss
        err_q = rel_linf(got, ref)
        err_l = float(np.max(np.abs(got - ref)) / np.max(np.abs(loss)))
        print("VSS N=48 fp32-mixed (%d,%d): rel to |Q| %.3e, rel to |loss| %.3e" % (p, q, err_q, err_l))
        assert err_l <= 2e-6 and err_q <= 5e-4


@pytest.mark.parametrize("N", [40, 56])
def test_vss_fp32_mixed_radix5_radix7_grids(torch_cuda, N):
    """FP32-mixed VSS plans (alpha = 1.3, octahedron, N_rho = 2) on N = 40
    and 56, a cross pair and a self pair against the FP64 oracle within the
    FP32 bounds: 2e-6 of the loss term, 5e-4 of Q."""
    from oracle.collide import collide_gain_loss
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = vss_config(N, ns=2, kind="octahedron", Nrho=2, seed=N + 1, n_nodes=1, alpha=1.3)
    pl = gpu_plan(cfg, precision="fp32")
    opl = oracle_pairs(cfg)
    F = torch.from_numpy(cfg["F"]).cuda()
    for p, q in [(0, 1), (1, 1)]:
        got = dgfs.collide(pl, p, q, F[:, p], F[:, q]).cpu().numpy()[0]
        gain, loss = collide_gain_loss(opl[p][q], cfg["F"][0, p], cfg["F"][0, q])
        ref = gain - loss
        err_q = rel_linf(got, ref)
        err_l = float(np.max(np.abs(got - ref)) / np.max(np.abs(loss)))
        print("VSS N=%d fp32-mixed (%d,%d): rel to |Q| %.3e, rel to |loss| %.3e" % (N, p, q, err_q, err_l))
        assert err_l <= 2e-6 and err_q <= 5e-4


def test_vss_three_species_rhs_N16(torch_cuda):
    """Three species (masses 1, 2, 4), alpha = 1.4, Fibonacci M = 32,
    N_rho = 8 at N = 16: the mixture collision term against the oracle."""
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = vss_config(16, ns=3, kind="fibonacci", M=32, Nrho=8, seed=5, n_nodes=1)
    cfg["masses"] = [1.0, 2.0, 4.0]
    pl = gpu_plan(cfg)
    ref = mixture_collision(oracle_pairs(cfg), cfg["F"])
    got = dgfs.rhs(pl, torch.from_numpy(cfg["F"]).cuda()).cpu().numpy()
    assert rel_linf(got, ref) <= TOL


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_vss_cfg5_full_shape_all_pairs_against_stored_oracle(torch_cuda, precision):
    """The precision workload at its full shape (three species, N = 48,
    Fibonacci M = 32, N_rho = 24, alpha = 1.4): all nine ordered pairs at two
    nodes against the oracle's terms, stored by
    tests/golden/make_vss_cfg5_oracle.py as 96 sampled points, 32 points
    where |Q| >= 1% of max |Q|, the point of max |Q| and four projections of
    the whole term onto seeded normal weights.  FP64: every compared point within 1e-11 of max |Q|, and each
    projection within 1e-11 max |Q| ||W||_2 (the size an error of that bar,
    independent of the weights, takes in the projection).  FP32-mixed: the
    bounds stated for that path, 2e-6 of max |loss| and 5e-4 of max |Q|,
    and the projections within 2e-6 max |loss| ||W||_2."""
    import json
    import os
    from paper_1903_04670_amd import dgfs, workloads as wl
    torch = torch_cuda
    with open(os.path.join(os.path.dirname(__file__), "golden", "vss_cfg5_oracle.json")) as fh:
        gold = json.load(fh)
    nodes = gold["nodes"]
    cfg = wl.precision_vss(n_nodes=nodes)
    F = cfg["F"]
    # the seeded input must be the one the stored terms were computed from
    assert list(F.shape) == gold["inputs"]["shape"]
    for i in range(nodes):
        for p in range(cfg["ns"]):
            s = gold["inputs"]["sums"][i][p]
            assert abs(F[i, p].sum() - s) <= 1e-12 * abs(s)
            assert abs(F[i, p].flat[0] - gold["inputs"]["first"][i][p]) <= 1e-15 * abs(F[i, p].flat[0])
    n3 = cfg["N"] ** 3
    idx = np.asarray(gold["sample_idx"])
    W = np.random.default_rng(gold["proj_seed"]).standard_normal((gold["n_proj"], n3))
    wn = np.linalg.norm(W, axis=1)
    pl = gpu_plan(cfg, precision=precision)
    Fd = torch.from_numpy(F).cuda()
    assert len(gold["pairs"]) == cfg["ns"] ** 2
    for key, ref_nodes in gold["pairs"].items():
        p, q = map(int, key.split(","))
        got = dgfs.collide(pl, p, q, Fd[:, p], Fd[:, q]).cpu().numpy().reshape(nodes, n3)
        for i, g in enumerate(ref_nodes):
            Q = got[i]
            e_pt = max(float(np.max(np.abs(Q[idx] - np.asarray(g["samples"])))),
                       float(np.max(np.abs(Q[np.asarray(g["bulk_idx"])] - np.asarray(g["bulk"])))),
                       abs(Q[g["argmax"]] - g["at_argmax"]))
            e_proj = np.abs(W @ Q - np.asarray(g["proj"])) / wn
            print("%s pair (%d,%d) node %d: points %.3e, projections %.3e of max|Q|; %.3e of max|loss|"
                  % (precision, p, q, i, e_pt / g["qmax"], e_proj.max() / g["qmax"], e_pt / g["lossmax"]))
            if precision == "fp64":
                assert e_pt <= TOL * g["qmax"] and np.all(e_proj <= TOL * g["qmax"]), (p, q, i)
            else:
                assert e_pt <= 2e-6 * g["lossmax"] and e_pt <= 5e-4 * g["qmax"], (p, q, i)
                assert np.all(e_proj <= 2e-6 * g["lossmax"]), (p, q, i)


def test_vss_N48_fp32_mixed_vs_fp64_and_projection(torch_cuda):
    """The precision workload at full velocity size (N = 48, M = 32 Fibonacci,
    N_rho = 24, three species, alpha = 1.4) on 2 nodes: FP32-mixed with the
    FP64 projection against the FP64 path, and exact conservation."""
    from paper_1903_04670_amd import dgfs, workloads as wl
    torch = torch_cuda
    cfg = wl.precision_vss(n_nodes=2)
    F = torch.from_numpy(cfg["F"]).cuda()
    p64 = gpu_plan(cfg, precision="fp64")
    ref = dgfs.rhs(p64, F).cpu().numpy()
    del p64
    p32 = gpu_plan(cfg, precision="fp32")
    got = dgfs.rhs(p32, F, project=True).cpu().numpy()
    del p32
    ref_proj = np.stack([cons.project(ref[i], cfg["N"], cfg["L"], cfg["masses"]) for i in range(2)])
    err = rel_linf(got, ref_proj)
    print("N=48 VSS fp32-mixed+projection vs fp64+projection: rel Linf %.3e" % err)
    assert err < 1e-3
    for i in range(2):
        mom = cons.moments(got[i], cfg["N"], cfg["L"], cfg["masses"])
        scale = cons.moments(np.abs(ref[i]), cfg["N"], cfg["L"], cfg["masses"])
        res = np.max(np.abs(mom)) / np.max(np.abs(scale))
        print("node %d conservation residual after projection: %.3e" % (i, res))
        assert res < 1e-12


def test_vss_full_size_512_nodes_properties(torch_cuda):
    """The precision workload at full size (512 nodes, three species, N = 48,
    M = 32 Fibonacci, N_rho = 24, alpha = 1.4): at every node the FP32-mixed
    collision term with the FP64 projection is within the stated bound of
    the projected FP64 term, and conserves mass of each species, momentum
    and energy to round-off (checked on the GPU in FP64)."""
    from paper_1903_04670_amd import dgfs, workloads as wl
    torch = torch_cuda
    cfg = wl.precision_vss(n_nodes=512)
    n, ns, N = cfg["n_nodes"], cfg["ns"], cfg["N"]
    F = torch.from_numpy(cfg["F"]).cuda()
    del cfg["F"]
    p64 = gpu_plan(cfg, precision="fp64")
    ref = dgfs.rhs(p64, F)
    del p64
    p32 = gpu_plan(cfg, precision="fp32")
    got = dgfs.rhs(p32, F, project=True)
    del p32, F
    C = torch.from_numpy(cons.constraint_rows(N, cfg["L"], cfg["masses"]).reshape(ns + 4, -1)).cuda()
    G = C @ C.T
    refm = ref.reshape(n, -1).T                      # [ns N^3, nodes]
    lam = torch.linalg.solve(G, C @ refm)
    ref_proj = (refm - C.T @ lam).T.reshape(got.shape)
    err = float((got - ref_proj).abs().max() / ref_proj.abs().max())
    print("512 nodes, N=48 VSS fp32-mixed+projection vs fp64+projection: rel Linf %.3e" % err)
    assert err < 1e-3
    mom = C @ got.reshape(n, -1).T                   # [ns + 4, nodes]
    scale = C @ ref.abs().reshape(n, -1).T
    res = float((mom.abs() / scale.abs().max(dim=0).values).max())
    print("worst conservation residual after projection over 512 nodes: %.3e" % res)
    assert res < 1e-12
