"""Nested shells coupled at shared spheres (oracle; test infrastructure only).

The paper's outlook (Sec. 1, Sec. 5) decomposes the domain into nested
spherical shells but gives no interface conditions.  Reading used here: two
shells A (inside) and B (outside) that share the sphere r = r_max(A) =
r_min(B) on the same angular grid each carry a copy of that sphere.  At every
point of it, each copy's right-hand side is taken apart into the
characteristic fields of App. A.2 (eq. characteristics) with the unit normal
s_i pointing from A into B,

  u^0 = g (speed 0),  u^1+ = -g + Pi + s^k Phi_k (speed alpha - b),
  u^1- = -g + Pi - s^k Phi_k (speed -alpha - b),
  u^2_i = P^k_i Phi_k (speed -b),  b = s_k beta^k,  P^k_i = delta^k_i - s^k s_i,

(for every symmetric pair ab), and both copies receive the same right-hand
side: every characteristic field from the side it comes from (speed > 0: it
travels from A into B, so A's value; speed < 0: B's; speed 0: the mean of
both), transformed back to d_t g, d_t Pi, d_t Phi_k.  This is the freezing
boundary operator of App. A.3 with the frozen incoming fields replaced by
the neighbour's values.  The copies therefore stay equal if they start
equal (the filter acts on each sphere by itself).  Fields without spatial
derivatives in their evolution (the gauge fields of the 58-field form) have
speed 0.  The outermost sphere keeps the freezing condition; the innermost
sphere has none (inside the horizon).  All shells take the same time step.
"""
import numpy as np

from .derivs import cartesian_derivs
from .ghg import rhs as ghg_rhs, freeze_incoming, boundary_normal, unpack, dependent, _es


def patch_interface(rA, rB, u_pt, xhat):
    """Common right-hand side of the two copies of an interface point.
    rA, rB: right-hand sides [n_v, ...] of shell A (inside) and B (outside);
    u_pt: the state there (the copies are equal); xhat: unit radial vector."""
    s_low, s_up = boundary_normal(u_pt, xhat)
    g, Pi, Phi, _ = unpack(u_pt)
    d = dependent(g, Pi, Phi)
    b = _es('i...,i...->...', s_low, d['beta_up'])
    alpha = d['alpha']

    def chars(r):
        dg, dPi = r[0:10], r[10:20]
        dPhi = np.array([r[20 + 10 * i:30 + 10 * i] for i in range(3)])
        sdPhi = _es('k...,kp...->p...', s_up, dPhi)
        tang = dPhi - s_low[:, None] * sdPhi[None]          # P^k_i dPhi_k
        return dg, -dg + dPi + sdPhi, -dg + dPi - sdPhi, tang

    gA, pA, mA, tA = chars(rA)
    gB, pB, mB, tB = chars(rB)

    def upwind(v, a, bb):
        return np.where(v > 0, a, np.where(v < 0, bb, 0.5 * (a + bb)))

    dg = 0.5 * (gA + gB)
    dp = upwind(alpha - b, pA, pB)
    dm = upwind(-alpha - b, mA, mB)
    dt = upwind(-b, tA, tB)
    out = rA.copy()
    out[0:10] = dg
    out[10:20] = dg + 0.5 * (dp + dm)
    for i in range(3):
        out[20 + 10 * i:30 + 10 * i] = s_low[i] * (0.5 * (dp - dm)) + dt[i]
    if rA.shape[0] > 50:
        out[50:] = 0.5 * (rA[50:] + rB[50:])
    return out


class NestedEvolution:
    """Shells in order of radius, each an (Shell, H, dH) triple, coupled at
    every shared sphere; the state is a list of per-shell arrays."""

    def __init__(self, shells, n_v=50, Hs=None, dHs=None, filter_kind='Yn', n_f=4):
        from .evolve import Evolution
        self.shells = shells
        self.n_v = n_v
        self.ev = [Evolution(sh, n_v, None if Hs is None else Hs[k], None if dHs is None else dHs[k],
                             filter_kind, n_f) for k, sh in enumerate(shells)]
        for a, b in zip(shells[:-1], shells[1:]):
            if not (a.r_max == b.r_min and a.n_theta == b.n_theta and a.n_phi == b.n_phi):
                raise ValueError("nested shells must share a sphere and its angular grid")

    def rhs(self, us):
        out = []
        for k, (ev, u) in enumerate(zip(self.ev, us)):
            du = np.array(cartesian_derivs(u, ev.shell))
            out.append(ghg_rhs(u, du, ev.H, ev.dH))
        last = len(us) - 1
        x, y, z = self.shells[last].cartesian()
        xhat = np.array([x, y, z]) / np.sqrt(x * x + y * y + z * z)
        kb = self.shells[last].n_r - 1
        out[last][..., kb] = freeze_incoming(out[last][..., kb], us[last][..., kb], xhat[..., kb])
        for k in range(last):
            x, y, z = self.shells[k].cartesian()
            xhat = np.array([x, y, z]) / np.sqrt(x * x + y * y + z * z)
            kb = self.shells[k].n_r - 1
            r = patch_interface(out[k][..., kb], out[k + 1][..., 0], us[k][..., kb], xhat[..., kb])
            out[k][..., kb] = r
            out[k + 1][..., 0] = r
        return out

    def rk4_step(self, us, dt):
        """Classical RK4 (Sec. 2.5) of all shells together, then each shell's filter."""
        def axpy(a, xs, ys):
            return [x + a * y for x, y in zip(xs, ys)]
        k1 = self.rhs(us)
        k2 = self.rhs(axpy(0.5 * dt, us, k1))
        k3 = self.rhs(axpy(0.5 * dt, us, k2))
        k4 = self.rhs(axpy(dt, us, k3))
        new = [u + dt / 6.0 * (a + 2.0 * b + 2.0 * c + d) for u, a, b, c, d in zip(us, k1, k2, k3, k4)]
        return [ev.filter(u) for ev, u in zip(self.ev, new)]
