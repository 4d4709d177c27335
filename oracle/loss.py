"""Scalar objectives of EV-FDLB runs (test infrastructure), evaluated with
the oracle so that their derivatives can be taken by complex step.

slab_loss: time-integrated mass flux through one node plus the L2 misfit of
the final density profile to a target,
    L = dt sum_{n=1}^{N} J(f^n) + 1/2 sum_i dx (n_i^N - n*_i)^2,
    J(f) = sum_k p_k F_k at the flux node,
starting from the reduced Maxwellian of (n0, u = 0, T0).  Every input may be
complex (phi_sigma, sigma, n0) for complex-step differentiation.
"""
import numpy as np

from . import step1d
from .model import Params


def slab_loss(n0, T0, Q, dx, dt, nsteps, flux_node, target, phi=1.0, sigma=1.0, **kw):
    p = Params(Q=Q, dx=dx, dt=dt, phi=phi, sigma=sigma, sigma_ref=float(np.real(sigma)), **kw)
    tb = step1d.Tables(p)
    n0 = np.asarray(n0)
    F, G = step1d.initial_state(n0, np.zeros(n0.shape), np.full(n0.shape, T0), tb)
    total = 0.0
    for _ in range(nsteps):
        F, G = step1d.rk3_step(F, G, tb)
        total = total + dt * np.sum(tb.v * F[:, flux_node])
    nN = F.sum(0)
    return total + 0.5 * dx * np.sum((nN - target) ** 2)
