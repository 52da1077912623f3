"""First-order generalized-harmonic (GHG) right-hand side and outer boundary
condition (oracle; test infrastructure only).

Equations as printed in App. A.1 (eqs. gdot, Phidot, Pidot with gamma_0 =
gamma_2 = 1, gamma_1 = -1, gamma_3 = gamma_1 gamma_2), dependent quantities
from eqs. normal, abgfromgab and Gamma, and the closed-form
freezing-incoming boundary operator B of App. A.3.  All tensors are handled as
full 4x4 (or 3x4x4) arrays with the point axes trailing.

Index conventions: a, b, c, d, e, f run over (t, x, y, z) = 0..3; i, j, k over
the spatial (x, y, z), which are 4-indices 1..3.
"""
import numpy as np


def _es(spec, *ops):
    return np.einsum(spec, *ops, optimize=True)

from .tensor_filter import PAIRS


def unpack(u):
    """State vector [50 or 58, ...] -> (g[4,4], Pi[4,4], Phi[3,4,4], extra)."""
    def sym(block):
        full = np.empty((4, 4) + block.shape[1:], dtype=block.dtype)
        for p, (a, b) in enumerate(PAIRS):
            full[a, b] = block[p]
            full[b, a] = block[p]
        return full
    g = sym(u[0:10])
    Pi = sym(u[10:20])
    Phi = np.array([sym(u[20 + 10 * i:30 + 10 * i]) for i in range(3)])
    extra = u[50:] if u.shape[0] > 50 else None
    return g, Pi, Phi, extra


def pack(gdot, Pidot, Phidot, extra=None):
    out = [gdot[a, b] for (a, b) in PAIRS] + [Pidot[a, b] for (a, b) in PAIRS]
    for i in range(3):
        out += [Phidot[i, a, b] for (a, b) in PAIRS]
    if extra is not None:
        out += list(extra)
    return np.array(out)


def _inv(m):
    """Inverse of [n, n, ...] matrices along the leading axes."""
    mt = np.moveaxis(np.moveaxis(m, 0, -1), 0, -1)
    inv = np.linalg.inv(mt)
    return np.moveaxis(np.moveaxis(inv, -1, 0), -1, 0)


def dependent(g, Pi, Phi):
    """3+1 quantities and Christoffel symbols from the undifferentiated
    variables: gamma_ij = g_ij, beta_j = g_tj, beta^i = gamma^ij beta_j,
    alpha = sqrt(beta_i beta^i - g_tt) (eq. abgfromgab); n_a = (-alpha, 0),
    n^a = (1/alpha, -beta^i/alpha) (eq. normal); inverse metrics by matrix
    inversion; d_t g_ab = -alpha Pi_ab + beta^i Phi_iab, d_i g_ab = Phi_iab and
    Gamma_cab = (d_a g_bc + d_b g_ac - d_c g_ab)/2, Gamma_c = g^ab Gamma_cab
    (eq. Gamma and App. A.1)."""
    gam = g[1:, 1:]
    beta_low = g[0, 1:]
    gam_inv = _inv(gam)
    beta_up = _es('ij...,j...->i...', gam_inv, beta_low)
    alpha = np.sqrt(_es('i...,i...->...', beta_low, beta_up) - g[0, 0])
    g_inv = _inv(g)
    zero = np.zeros_like(alpha)
    n_up = np.array([1.0 / alpha] + [-beta_up[i] / alpha for i in range(3)])
    n_low = np.array([-alpha, zero, zero, zero])
    dtg = -alpha * Pi + _es('i...,iab...->ab...', beta_up, Phi)
    dg = np.concatenate([dtg[None], Phi], axis=0)          # dg[c,a,b] = d_c g_ab
    Gam = 0.5 * (_es('abc...->cab...', dg) + _es('bac...->cab...', dg) - dg)
    Gam_c = _es('ab...,cab...->c...', g_inv, Gam)
    return dict(gam_inv=gam_inv, beta_up=beta_up, alpha=alpha, g_inv=g_inv,
                n_up=n_up, n_low=n_low, Gam=Gam, Gam_c=Gam_c)


def rhs(u, du, H=None, dH=None):
    """Right-hand side d_t u of the first-order GHG system, App. A.1.

    u: state [n_v, ...] (n_v = 50, or 58 with H_a and Q_a = d_t H_a appended).
    du: Cartesian derivatives [3, n_v, ...], du[k, mu] = d_k u^mu.
    H, dH: gauge source H_a [4, ...] and dH[a, b] = d_a H_b [4, 4, ...] for
    the 50-field system (static gauge, eq. gauge: d_t H = 0).  For 58 fields
    they are taken from the state: d_t H_b = Q_b, d_i H_b = du[i, 50 + b].

    The 58-field extension evolves d_t H_a = Q_a, d_t Q_a = 0; the paper gives
    no evolution equation for H_a (App. A.1 mentions the extended state only),
    so this part is parity unpinned."""
    g, Pi, Phi, extra = unpack(u)
    dgi = np.array([unpack(du[k])[0] for k in range(3)])     # d_k g_ab
    dPi = np.array([unpack(du[k])[1] for k in range(3)])     # d_k Pi_ab
    dPhi = np.array([unpack(du[k])[2] for k in range(3)])    # d_k Phi_iab  [k,i,a,b]
    if u.shape[0] == 58:
        H = u[50:54]
        Q = u[54:58]
        dH = np.concatenate([Q[None], du[:, 50:54]], axis=0)
    q = dependent(g, Pi, Phi)
    al, bu, gi, gI = q['alpha'], q['beta_up'], q['gam_inv'], q['g_inv']
    nu, nl, Gam, Gc = q['n_up'], q['n_low'], q['Gam'], q['Gam_c']

    # eq. gdot
    gdot = -al * Pi + _es('i...,iab...->ab...', bu, Phi)

    # eq. Phidot
    nnPhi = _es('c...,d...,icd...->i...', nu, nu, Phi)
    Phidot = (_es('k...,kiab...->iab...', bu, dPhi)
              - al * dPi + al * dgi
              + 0.5 * al * nnPhi[:, None, None] * Pi[None]
              + al * _es('jk...,c...,ijc...,kab...->iab...', gi, nu, Phi[:, 1:], Phi)
              - al * Phi)

    # eq. Pidot
    Phi4 = np.concatenate([np.zeros_like(Phi[:1]), Phi], axis=0)  # spatial index padded
    t_adv = _es('k...,kab...->ab...', bu, dPi)
    t_pp = -al * _es('ik...,kiab...->ab...', gi, dPhi)
    t_cg = -_es('k...,kab...->ab...', bu, dgi)
    quad = (_es('cd...,ij...,iac...,jbd...->ab...', gI, gi, Phi, Phi)
            - _es('cd...,ac...,bd...->ab...', gI, Pi, Pi)
            - _es('cd...,ef...,ace...,bdf...->ab...', gI, gI, Gam, Gam))
    nablaH = dH - _es('cd...,cab...,d...->ab...', gI, Gam, H)
    symH = 0.5 * (nablaH + _es('ab...->ba...', nablaH))
    nnPi = _es('c...,d...,cd...->...', nu, nu, Pi)
    t_npp = -al * _es('c...,ci...,ij...,jab...->ab...', nu, Pi[:, 1:], gi, Phi)
    C = H + Gc
    nC = _es('c...,c...->...', nu, C)
    t_damp = al * (_es('a...,b...->ab...', C, nl) + _es('b...,a...->ab...', C, nl)
                   - g * nC)
    Pidot = (t_adv + t_pp + t_cg + 2.0 * al * quad - 2.0 * al * symH
             - 0.5 * al * nnPi * Pi + t_npp + t_damp
             + _es('i...,iab...->ab...', bu, Phi))
    del Phi4

    extra_dot = None
    if u.shape[0] == 58:
        extra_dot = np.concatenate([Q, np.zeros_like(Q)], axis=0)
    return pack(gdot, Pidot, Phidot, extra_dot)


def constraints(u, du, H=None):
    """Constraint fields of the first-order GHG system (App. A.1): the gauge
    constraint C_a = H_a + Gamma_a and the first-order constraint
    C_iab = d_i g_ab - Phi_iab.

    u: state [n_v, ...]; du: Cartesian derivatives [3, n_v, ...] (only the
    g_ab rows are used); H: gauge source [4, ...] for 50 fields (58 fields take
    H_a from the state).  Returns (C_a [4, ...], C_iab [3, 10, ...]) with the
    symmetric pairs in storage order."""
    g, Pi, Phi, _ = unpack(u)
    if u.shape[0] == 58:
        H = u[50:54]
    Gc = dependent(g, Pi, Phi)['Gam_c']
    C_a = H + Gc
    C_iab = du[:, 0:10] - u[20:50].reshape((3, 10) + u.shape[1:])
    return C_a, C_iab


def constraint_norms(C_a, C_iab):
    """(max |C_a|, rms C_a, max |C_iab|, rms C_iab); rms over every component
    and grid point."""
    return (float(np.abs(C_a).max()), float(np.sqrt(np.mean(C_a ** 2))),
            float(np.abs(C_iab).max()), float(np.sqrt(np.mean(C_iab ** 2))))


def boundary_normal(u, xhat):
    """Outward unit normal of a sphere, s_i = xhat_i / sqrt(gamma^jk xhat_j xhat_k)
    and s^i = gamma^ij s_j (App. A.2 / A.3)."""
    g, Pi, Phi, _ = unpack(u)
    gi = _inv(g[1:, 1:])
    norm = np.sqrt(_es('jk...,j...,k...->...', gi, xhat, xhat))
    s_low = xhat / norm
    s_up = _es('ij...,j...->i...', gi, s_low)
    return s_low, s_up


def freeze_incoming(rhs_pt, u_pt, xhat):
    """Boundary operator B = E^-1 Z E freezing the incoming characteristic
    fields, closed form of App. A.3: B(dg) = dg, B(dPi) = (dg + dPi + s^k dPhi_k)/2,
    B(dPhi_i) = s_i (-dg + dPi + s^k dPhi_k)/2.  Applied to every symmetric
    pair ab; extra gauge fields (58-field form) pass unchanged."""
    s_low, s_up = boundary_normal(u_pt, xhat)
    out = rhs_pt.copy()
    dg = rhs_pt[0:10]
    dPi = rhs_pt[10:20]
    dPhi = np.array([rhs_pt[20 + 10 * i:30 + 10 * i] for i in range(3)])
    sPhi = _es('k...,kp...->p...', s_up, dPhi)
    out[10:20] = 0.5 * (dg + dPi + sPhi)
    w = 0.5 * (-dg + dPi + sPhi)
    for i in range(3):
        out[20 + 10 * i:30 + 10 * i] = s_low[i] * w
    return out


def characteristic_matrix(s_low, s_up, alpha, b):
    """s_k A^k for one symmetric pair as printed in App. A.2 eq.
    characteristics: rows/cols ordered (g, Pi, Phi_1, Phi_2, Phi_3)."""
    M = np.zeros((5, 5))
    M[1, 0], M[1, 1] = b, -b
    M[1, 2:5] = alpha * np.asarray(s_up)
    M[2:5, 0] = -alpha * np.asarray(s_low)
    M[2:5, 1] = alpha * np.asarray(s_low)
    M[2:5, 2:5] = -b * np.eye(3)
    return M
