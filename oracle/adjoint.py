"""Vector-Jacobian product of Algorithm 2 (oracle; test infrastructure).

Q = beta Re( iF( sum_{rm} W_rm * F(u1_rm * u2_rm) ) - f * iF(c * F g) ),
u1 = iF(P1 * F f), u2 = iF(P2 * F g), W = w_r w_m b_rm,
P1 = exp(+i m_q/(m_p+m_q) a), P2 = exp(-i m_p/(m_p+m_q) a), a = pi/L rho (l.sigma).
F (forward DFT) and iF (inverse) are symmetric matrices, and for real inputs
the gradient of <wbar, Re(A x)> is Re(A^T wbar).  Transposing each factor:
  dQ/df^T wbar = beta Re F( sum_rm P1 * iF(u2 * F(W * iF wbar)) )
                 - beta wbar * Re iF(c * F g)
  dQ/dg^T wbar = beta Re F( sum_rm P2 * iF(u1 * F(W * iF wbar)) )
                 - beta Re F(c * iF(f * wbar))
u1, u2 are recomputed per (r, m).  When p = q and one array feeds both
arguments, its gradient is the sum of the two.  With plan.nyquist_zero the
gain's translates are formed from Z F f and Z F g, Z the (diagonal,
symmetric) Nyquist-plane mask, so Z joins P1 and P2.
"""
import numpy as np

from . import dft
from .collide import nyquist_mask, phase_argument


def collide_vjp(plan, f, g, wbar):
    mp, mq = plan.mp, plan.mq
    FTf, FTg = dft.fft3(f), dft.fft3(g)
    u = dft.ifft3(wbar)
    acc_f = np.zeros_like(FTf)
    acc_g = np.zeros_like(FTg)
    z = nyquist_mask(plan.N) if plan.nyquist_zero else 1.0
    for r in range(len(plan.rho)):
        for m in range(len(plan.sigma)):
            a = phase_argument(plan, r, m)
            P1 = np.exp(1j * mq / (mp + mq) * a) * z
            P2 = np.exp(-1j * mp / (mp + mq) * a) * z
            u1 = dft.ifft3(P1 * FTf)
            u2 = dft.ifft3(P2 * FTg)
            v = dft.fft3(plan.w_rho[r] * plan.w_sigma[m] * plan.b[r, m] * u)
            acc_f = acc_f + P1 * dft.ifft3(u2 * v)
            acc_g = acc_g + P2 * dft.ifft3(u1 * v)
    gf = plan.beta * (np.real(dft.fft3(acc_f)) - wbar * np.real(dft.ifft3(plan.c * FTg)))
    gg = plan.beta * (np.real(dft.fft3(acc_g)) - np.real(dft.fft3(plan.c * dft.ifft3(f * wbar))))
    return gf, gg
