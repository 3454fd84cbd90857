"""FP64 CPU oracle for the multi-species fast spectral collision operator.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised NumPy implementation of what the GPU path computes, written from
the paper (Jaiswal, Hu, Brillon, Alexeenko, "A discontinuous Galerkin fast
spectral method for multi-species full Boltzmann on streaming
multi-processors", PASC'19, arXiv:1903.04670).  It exists to check the HIP
library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product package never
does, and this package never imports the product package.

Modules
-------
quadrature    velocity grid, wave index, Gauss-Legendre radii, sphere sets,
              truncation radius (Sec. 2.1; Algorithm 1 inputs)
dft           the oracle's own naive per-axis DFT (dense N x N matrices)
tables        gain table b, loss table c, prefactor beta (Eqs. VSSNonDim,
              Fkr_vss, Gmm_vss; Algorithm 1) evaluated by closed forms
collide       Algorithm 2 step by step, and the direct O(N^6) Galerkin sum
              of Eq. apndx_Qprojected
krook_wu      Krook-Wu exact solution and its time derivative (Sec. 3.2)
conservation  moments and the Lagrange-multiplier conservation projection
adjoint       vector-Jacobian product of Algorithm 2 by transposition
dg            nodal DG upwind transport, diffuse walls, SSP-RK3 (Sec. 3.3)

Functions whose result is not pinned by an independent check say
"parity unpinned" in their docstring.
"""
