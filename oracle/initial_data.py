"""Initial data and static gauge source (oracle; test infrastructure only).

App. A.3: the first-order variables follow from a given 4-metric g_ab by their
definitions (eq. defPiPhi), with the spatial derivatives taken numerically
(here: the oracle's spectral Cartesian derivatives) and d_t g_ab = 0, so
Pi_ab = beta^i Phi_iab / alpha.  The gauge source is H_a = -Gamma_a at t = 0
and held fixed (eq. gauge); its spatial derivatives are again spectral.
"""
import numpy as np

from .derivs import cartesian_derivs
from .ghg import dependent, unpack, pack


def first_order_data(g10, shell, extra=None):
    """u = {g, Pi, Phi} (+ extra gauge fields for the 58-field form) from the
    10 metric components g10 [10, N_phi, N_theta, N_r]."""
    dg = np.array(cartesian_derivs(g10, shell))          # [3, 10, ...]
    u = np.zeros((50,) + g10.shape[1:])
    u[0:10] = g10
    for i in range(3):
        u[20 + 10 * i:30 + 10 * i] = dg[i]
    g, _, Phi, _ = unpack(u)
    q = dependent(g, np.zeros_like(g), Phi)
    Pi = np.einsum('i...,iab...->ab...', q['beta_up'], Phi) / q['alpha']
    u = pack(g, Pi, Phi)
    if extra is not None:
        u = np.concatenate([u, extra], axis=0)
    return u


def static_gauge(u, shell):
    """H_a = -Gamma_a (eq. gauge) and dH[a, b] = d_a H_b with d_t H_b = 0 and the
    spatial derivatives spectral."""
    g, Pi, Phi, _ = unpack(u)
    H = -dependent(g, Pi, Phi)['Gam_c']
    dHi = np.array(cartesian_derivs(H, shell))           # [3, 4, ...] = d_i H_b
    dH = np.concatenate([np.zeros_like(H)[None], dHi], axis=0)
    return H, dH
