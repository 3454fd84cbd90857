"""GPU adjoint (dgfs_collide_vjp) against the oracle's gradient, central
finite differences of the GPU forward, and the dot-product identity."""
import numpy as np
import pytest

from helpers import gpu_plan, oracle_pairs, rel_linf, small_config
from oracle.adjoint import collide_vjp as oracle_vjp
from paper_1903_04670_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("N,kind", [(8, "icosahedron"), (10, "octahedron"), (12, "octahedron"),
                                    (14, "icosahedron"), (16, "fibonacci")])
def test_vjp_matches_oracle_gradient(torch_cuda, N, kind):
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = small_config(N, ns=2, M_kind=kind, Nrho=4, seed=20 + N, n_nodes=2)
    rng = np.random.default_rng(N)
    W = rng.standard_normal((2, N, N, N))
    opl = oracle_pairs(cfg)
    pl = gpu_plan(cfg)
    F = torch.from_numpy(cfg["F"]).cuda()
    Wd = torch.from_numpy(W).cuda()
    for p, q in [(0, 1), (1, 0), (1, 1)]:
        gf, gq = dgfs.collide_vjp(pl, p, q, F[:, p], F[:, q], Wd)
        torch.cuda.synchronize()
        for i in range(2):
            rf, rq = oracle_vjp(opl[p][q], cfg["F"][i, p], cfg["F"][i, q], W[i])
            assert rel_linf(gf[i].cpu().numpy(), rf) <= 1e-11, (p, q, i)
            assert rel_linf(gq[i].cpu().numpy(), rq) <= 1e-11, (p, q, i)


@pytest.mark.parametrize("N", [40, 56])
def test_vjp_radix5_radix7_grids(torch_cuda, N):
    """The adjoint on N = 40 = 8 x 5 and N = 56 = 8 x 7 (one node, a cross
    pair and a self pair, octahedron, N_rho = 2) against the oracle's
    gradient at 1e-11."""
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = small_config(N, ns=2, M_kind="octahedron", Nrho=2, seed=70 + N, n_nodes=1)
    W = np.random.default_rng(N + 3).standard_normal((1, N, N, N))
    opl = oracle_pairs(cfg)
    pl = gpu_plan(cfg)
    F = torch.from_numpy(cfg["F"]).cuda()
    Wd = torch.from_numpy(W).cuda()
    for p, q in [(0, 1), (1, 1)]:
        gf, gq = dgfs.collide_vjp(pl, p, q, F[:, p], F[:, q], Wd)
        torch.cuda.synchronize()
        rf, rq = oracle_vjp(opl[p][q], cfg["F"][0, p], cfg["F"][0, q], W[0])
        assert rel_linf(gf[0].cpu().numpy(), rf) <= 1e-11, (N, p, q)
        assert rel_linf(gq[0].cpu().numpy(), rq) <= 1e-11, (N, p, q)


@pytest.mark.parametrize("N,kind,alpha", [(8, "fibonacci", 1.4), (10, "icosahedron", 1.2),
                                          (12, "octahedron", 1.3), (16, "fibonacci", 0.8)])
def test_vss_vjp_matches_oracle_gradient(torch_cuda, N, kind, alpha):
    """VSS plans (alpha != 1): the direction-dependent table gives one
    v_rm = F(w_r w_m b_rm u) per (r, m) term; against the oracle's gradient
    (its transposition holds for any table) at 1e-11."""
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = small_config(N, ns=2, M_kind=kind, Nrho=3, seed=30 + N, n_nodes=2)
    cfg["alpha"] = np.full((2, 2), alpha)
    rng = np.random.default_rng(N + 1)
    W = rng.standard_normal((2, N, N, N))
    opl = oracle_pairs(cfg)
    pl = gpu_plan(cfg)
    F = torch.from_numpy(cfg["F"]).cuda()
    Wd = torch.from_numpy(W).cuda()
    for p, q in [(0, 1), (1, 0), (1, 1)]:
        gf, gq = dgfs.collide_vjp(pl, p, q, F[:, p], F[:, q], Wd)
        torch.cuda.synchronize()
        for i in range(2):
            rf, rq = oracle_vjp(opl[p][q], cfg["F"][i, p], cfg["F"][i, q], W[i])
            assert rel_linf(gf[i].cpu().numpy(), rf) <= 1e-11, (N, p, q, i)
            assert rel_linf(gq[i].cpu().numpy(), rq) <= 1e-11, (N, p, q, i)


def test_fp32_mixed_vjp_error_bound(torch_cuda):
    """An FP32-mixed plan's adjoint (FP32 transforms, FP64 inputs and
    outputs) against the FP64 oracle's gradient on the two-species N = 32
    node, within 1e-5 of the gradient's largest entry.  With a random
    cotangent there is none of the forward operator's gain/loss
    cancellation, so the error is that of the FP32 transform chain: about
    five 3-D transforms of 3 log2(32) = 15 rounding stages each, 75 x 6e-8
    = 4.5e-6."""
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = wl.couette_two_species(K=1, P=0)
    N = cfg["N"]
    W = np.random.default_rng(7).standard_normal((1, N, N, N))
    opl = oracle_pairs(cfg)
    pl = gpu_plan(cfg, precision="fp32")
    F = torch.from_numpy(cfg["F"]).cuda()
    Wd = torch.from_numpy(W).cuda()
    for p, q in [(0, 1), (1, 1)]:
        gf, gq = dgfs.collide_vjp(pl, p, q, F[:, p], F[:, q], Wd)
        torch.cuda.synchronize()
        rf, rq = oracle_vjp(opl[p][q], cfg["F"][0, p], cfg["F"][0, q], W[0])
        ef, eq = rel_linf(gf[0].cpu().numpy(), rf), rel_linf(gq[0].cpu().numpy(), rq)
        print("fp32-mixed vjp (%d,%d): rel Linf %.3e %.3e" % (p, q, ef, eq))
        assert ef <= 1e-5 and eq <= 1e-5, (p, q, ef, eq)


def test_fp32_mixed_vss_vjp_error_bound(torch_cuda):
    """The VSS adjoint of an FP32-mixed plan (complex direction tables in
    FP32) against the FP64 oracle's gradient at N = 12, Fibonacci M = 7,
    alpha = 1.3: within 1e-5 of the largest gradient entry, as for the VHS
    FP32-mixed adjoint (a shorter transform chain at N = 12)."""
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = small_config(12, ns=2, M_kind="fibonacci", Nrho=3, seed=44, n_nodes=1)
    cfg["alpha"] = np.full((2, 2), 1.3)
    W = np.random.default_rng(9).standard_normal((1, 12, 12, 12))
    opl = oracle_pairs(cfg)
    pl = gpu_plan(cfg, precision="fp32")
    F = torch.from_numpy(cfg["F"]).cuda()
    Wd = torch.from_numpy(W).cuda()
    for p, q in [(0, 1), (1, 1)]:
        gf, gq = dgfs.collide_vjp(pl, p, q, F[:, p], F[:, q], Wd)
        torch.cuda.synchronize()
        rf, rq = oracle_vjp(opl[p][q], cfg["F"][0, p], cfg["F"][0, q], W[0])
        ef, eq = rel_linf(gf[0].cpu().numpy(), rf), rel_linf(gq[0].cpu().numpy(), rq)
        print("fp32-mixed vss vjp (%d,%d): rel Linf %.3e %.3e" % (p, q, ef, eq))
        assert ef <= 1e-5 and eq <= 1e-5, (p, q, ef, eq)


@pytest.mark.parametrize("n_nodes,n_dirs", [(4, 16), (256, 64)])
def test_vjp_central_differences_N32(torch_cuda, n_nodes, n_dirs):
    """Two species (masses 1, 2.5), N = 32, icosahedron, N_rho = 16, on 4
    nodes and on the differentiation workload's full 256 nodes: <wbar, dQ>
    by central differences (eps = 1e-6, relative to |f|_inf) along random
    directions equals <grad, d>.  Q is bilinear, so the difference quotient
    is exact up to rounding."""
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = wl.differentiation(n_nodes=n_nodes)
    pl = gpu_plan(cfg)
    F = torch.from_numpy(cfg["F"]).cuda()
    W = torch.from_numpy(cfg["W"][:, 0]).cuda()
    gen = torch.Generator(device="cpu").manual_seed(44)
    p, q = 0, 1
    gf, gq = dgfs.collide_vjp(pl, p, q, F[:, p].contiguous(), F[:, q].contiguous(), W)
    worst = 0.0
    for k in range(n_dirs):
        d = torch.randn(F[:, p].shape, generator=gen, dtype=torch.float64).cuda()
        d = d * (F.abs().max() / d.abs().max())
        eps = 1e-6
        side = k % 2
        base = [F[:, p].contiguous(), F[:, q].contiguous()]
        plus = list(base)
        minus = list(base)
        plus[side] = base[side] + eps * d
        minus[side] = base[side] - eps * d
        qp = dgfs.collide(pl, p, q, plus[0], plus[1])
        qm = dgfs.collide(pl, p, q, minus[0], minus[1])
        fd = float(((qp - qm) * W).sum() / (2 * eps))
        an = float(((gf if side == 0 else gq) * d).sum())
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-30))
    print("VJP vs central differences: worst relative gap %.3e" % worst)
    assert worst < 1e-6


def test_autograd_function(torch_cuda):
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = small_config(8, ns=2, Nrho=3, seed=31, n_nodes=2)
    pl = gpu_plan(cfg)
    F = torch.from_numpy(cfg["F"]).cuda()
    fp = F[:, 0].clone().requires_grad_(True)
    fq = F[:, 1].clone().requires_grad_(True)
    Q = dgfs.collide_autograd(pl, 0, 1, fp, fq)
    W = torch.randn_like(Q)
    (Q * W).sum().backward()
    gf, gq = dgfs.collide_vjp(pl, 0, 1, F[:, 0].contiguous(), F[:, 1].contiguous(), W)
    assert torch.allclose(fp.grad, gf, rtol=0, atol=0)
    assert torch.allclose(fq.grad, gq, rtol=0, atol=0)


def test_vjp_accumulate_and_one_sided_calls(torch_cuda):
    """DGFS_ACCUMULATE adds the gradients into the given arrays, and with
    grad_fp or grad_fq NULL the other side alone is formed, bit-identical to
    the two-sided call (through the C ABI directly for the NULL cases)."""
    import ctypes as ct
    from paper_1903_04670_amd import dgfs
    torch = torch_cuda
    cfg = small_config(8, ns=2, Nrho=3, seed=51, n_nodes=3)
    pl = gpu_plan(cfg)
    F = torch.from_numpy(cfg["F"]).cuda()
    fp, fq = F[:, 0].contiguous(), F[:, 1].contiguous()
    W = torch.randn(3, 8, 8, 8, dtype=torch.float64, device="cuda")
    gf, gq = dgfs.collide_vjp(pl, 0, 1, fp, fq, W)
    A, B = torch.randn_like(gf), torch.randn_like(gq)
    a2, b2 = dgfs.collide_vjp(pl, 0, 1, fp, fq, W, grad_fp=A.clone(), grad_fq=B.clone(), accumulate=True)
    torch.cuda.synchronize()
    assert torch.allclose(a2, A + gf, rtol=0, atol=1e-14 * float(gf.abs().max()))
    assert torch.allclose(b2, B + gq, rtol=0, atol=1e-14 * float(gq.abs().max()))
    n3 = 8 ** 3
    ws = dgfs.workspace(pl, 3, dgfs.OP_VJP)
    for side in (0, 1):
        out = torch.full_like(gf, 7.0)
        pg = ct.c_void_p(out.data_ptr())
        st = dgfs.lib.dgfs_collide_vjp(pl.handle, 3, 0, 1, ct.c_void_p(fp.data_ptr()), ct.c_void_p(fq.data_ptr()),
                                       n3, ct.c_void_p(W.data_ptr()), n3,
                                       pg if side == 0 else None, pg if side == 1 else None, n3, 0,
                                       ct.c_void_p(ws.data_ptr()), ws.numel(), None)
        torch.cuda.synchronize()
        assert st == 0
        assert torch.equal(out, gf if side == 0 else gq)
