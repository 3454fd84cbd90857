"""Table 1 on the GPU: the error of the library's mixture collision term
against the Krook-Wu exact solution (Sec. 3.2) for all 72 printed cells,
N = 16 ... 56 (radix-5 and radix-7 transforms at N = 40 and 56).

The exact solution, its time derivative and the kernel constants come from
the oracle's Krook-Wu module; the collision term is dgfs_rhs (FP64) on one
space-homogeneous node with the truncation radius R = L/2 = 6 for every pair.
Two bars per species error:
  * it equals the oracle's error of the same cell
    (table1_krook_wu_oracle.txt, written from the oracle) to 1e-6 relative,
    so the library reproduces the oracle on every cell, misses included;
  * it lies within x0.8 ... x1.25 of the printed error, except the named
    misses (helpers.TABLE1_MISSES).
"""
import numpy as np
import pytest

from helpers import TABLE1_L, TABLE1_R, TABLE1_T, table1_check, table1_oracle, table1_printed
from oracle.krook_wu import KrookWu
from oracle.quadrature import velocity_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("cell", sorted(table1_printed()), ids=lambda c: "N%d_Nr%d_M%d_r%g" % c)
def test_table1_krook_wu_on_gpu(torch_cuda, cell):
    from paper_1903_04670_amd import dgfs
    N, Nr, M, ratio = cell
    L, T = TABLE1_L, TABLE1_T
    kw = KrookWu(1.0, ratio)
    c, _ = velocity_grid(N, L)
    cx, cy, cz = np.meshgrid(c, c, c, indexing="ij")
    v2 = cx ** 2 + cy ** 2 + cz ** 2
    F = np.stack([kw.f(1, T, v2), kw.f(2, T, v2)])[None]
    beta = [[kw.beta(p, q) for q in (1, 2)] for p in (1, 2)]
    pl = dgfs.Plan([1.0, ratio], np.ones((2, 2)), np.ones((2, 2)), N, L, Nr,
                   sphere="octahedron" if M == 6 else "icosahedron", beta=beta,
                   R=np.full((2, 2), TABLE1_R))
    d = dgfs.rhs(pl, torch_cuda.from_numpy(F).cuda()).cpu().numpy()[0]
    got = [float(np.max(np.abs(d[p - 1] - kw.dfdt(p, T, v2)))) for p in (1, 2)]
    ref = table1_oracle()[cell]
    printed = table1_printed()[cell]
    print("N=%d Nr=%d M=%d ratio=%g: E1 %.3e (x%.3f), E2 %.3e (x%.3f)"
          % (N, Nr, M, ratio, got[0], got[0] / printed[0], got[1], got[1] / printed[1]))
    for g, r in zip(got, ref):
        assert abs(g - r) <= 1e-6 * r, (got, ref)
    bad = table1_check(cell, got)
    assert not bad, bad
