"""Method of lines with classical RK4 and a filter after every full step
(oracle; test infrastructure only), Sec. 2.5.

One right-hand-side evaluation: coordinate derivatives of all fields, the
Cartesian chain rule (Sec. 2.2), the GHG right-hand side (App. A.1), and the
freezing-incoming boundary operator on the outermost sphere k = N_r - 1
(App. A.3; no condition at r_min, which lies inside the horizon).
"""
import numpy as np

from .derivs import cartesian_derivs
from .ghg import rhs as ghg_rhs, freeze_incoming
from .tensor_filter import yn_filter, y_filter, yg_filter


class Evolution:
    def __init__(self, shell, n_v=50, H=None, dH=None, filter_kind='Yn', n_f=4):
        self.shell, self.n_v = shell, n_v
        self.H, self.dH = H, dH
        self.filter_kind, self.n_f = filter_kind, n_f

    def cart_derivs(self, u):
        return np.array(cartesian_derivs(u, self.shell))

    def rhs(self, u, du=None):
        """S(u) - A^k(u) d_k u with the outer boundary condition applied."""
        if du is None:
            du = self.cart_derivs(u)
        r = ghg_rhs(u, du, self.H, self.dH)
        x, y, z = self.shell.cartesian()
        rad = np.sqrt(x * x + y * y + z * z)
        xhat = np.array([x, y, z]) / rad
        kb = self.shell.n_r - 1
        r[..., kb] = freeze_incoming(r[..., kb], u[..., kb], xhat[..., kb])
        return r

    def filter(self, u):
        if self.filter_kind == 'Yn':
            return yn_filter(u, self.shell, self.n_f)
        if self.filter_kind == 'Y':
            return y_filter(u, self.shell, self.n_f)
        if self.filter_kind == 'Yg':
            return yg_filter(u, self.shell, self.n_f)
        if self.filter_kind == 'none':
            return u
        raise ValueError(self.filter_kind)

    def rk4_step(self, u, dt, rhs_fn=None):
        """Classical RK4 (Sec. 2.5): k1..k4 at u, u+dt/2 k1, u+dt/2 k2, u+dt k3;
        u + dt (k1 + 2 k2 + 2 k3 + k4)/6, followed by the filter."""
        f = rhs_fn or self.rhs
        k1 = f(u)
        k2 = f(u + 0.5 * dt * k1)
        k3 = f(u + 0.5 * dt * k2)
        k4 = f(u + dt * k3)
        unew = u + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        return self.filter(unew)
