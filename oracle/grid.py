"""Shell collocation grid and 1-d differentiation matrices (oracle; test
infrastructure only).

Follows Sec. 2.1 (eqs. rk, thetai, phij), Sec. 2.3 (Fourier matrix FD and the
Chebyshev matrix of eq. CDhat) and Sec. 4.1 (Courant factor, Tab. dtfac).
"""
import numpy as np


class Shell:
    """One spherical shell r in [r_min, r_max] with N_r x N_theta x N_phi points."""

    def __init__(self, n_r, n_theta, n_phi, r_min, r_max):
        if n_phi % 2:
            raise ValueError("N_phi must be even (Sec. 2.1)")
        self.n_r, self.n_theta, self.n_phi = int(n_r), int(n_theta), int(n_phi)
        self.r_min, self.r_max = float(r_min), float(r_max)
        self.r = radial_points(n_r, r_min, r_max)
        self.theta = theta_points(n_theta)
        self.phi = phi_points(n_phi)

    @property
    def shape(self):
        """Array shape of one field: [phi j][theta i][r k] (r fastest)."""
        return (self.n_phi, self.n_theta, self.n_r)

    @property
    def npts(self):
        return self.n_r * self.n_theta * self.n_phi

    def coords(self):
        """Spherical (r, theta, phi) broadcast to the field shape."""
        r = self.r[None, None, :]
        th = self.theta[None, :, None]
        ph = self.phi[:, None, None]
        return np.broadcast_arrays(r, th, ph)

    def cartesian(self):
        """Cartesian (x, y, z) of every collocation point, field shape."""
        r, th, ph = self.coords()
        return (r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph),
                r * np.cos(th))


def radial_points(n_r, r_min, r_max):
    """r_k = (r_max+r_min)/2 - (r_max-r_min)/2 cos(pi k/(N_r-1)), Sec. 2.1 eq. rk."""
    k = np.arange(n_r)
    return 0.5 * (r_max + r_min) - 0.5 * (r_max - r_min) * np.cos(np.pi * k / (n_r - 1))


def theta_points(n_theta):
    """theta_i = pi (i + 1/2)/N_theta, staggered off the poles, Sec. 2.1 eq. thetai."""
    return np.pi * (np.arange(n_theta) + 0.5) / n_theta


def phi_points(n_phi):
    """phi_j = 2 pi j / N_phi, Sec. 2.1 eq. phij."""
    return 2.0 * np.pi * np.arange(n_phi) / n_phi


def fourier_diff_matrix(n):
    """Periodic Fourier differentiation matrix for n (even) equally spaced
    points of spacing 2 pi/n: FD_ij = (-1)^(i+j) / (2 tan((x_i-x_j)/2)),
    FD_ii = 0 (Sec. 2.3).  On this grid (x_i - x_j)/2 = pi (i - j)/n exactly,
    so the half-difference is formed from the integer i - j rather than from
    two rounded coordinates."""
    if n % 2:
        raise ValueError("Fourier differentiation needs an even number of points")
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (-1.0) ** (i + j) / (2.0 * np.tan(np.pi * (i - j) / n))
    return D


def cheb_diff_matrix(n, r_min, r_max):
    """Chebyshev extrema-grid differentiation matrix rescaled to [r_min, r_max]:
    x_i = -cos(pi i/(N-1)), CD_ij = (c_i/c_j) (-1)^(i+j)/(x_i - x_j),
    CD_ii = -sum_{j != i} CD_ij, c_0 = c_{N-1} = 2 (Sec. 2.3 eq. CDhat),
    then multiplied by 2/(r_max - r_min)."""
    x = -np.cos(np.pi * np.arange(n) / (n - 1))
    c = np.ones(n)
    c[0] = c[-1] = 2.0
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (c[i] / c[j]) * (-1.0) ** (i + j) / (x[i] - x[j])
        D[i, i] = -sum(D[i, j] for j in range(n) if j != i)
    return 2.0 * D / (r_max - r_min)


def min_spacing(shell):
    """Smallest grid distance, Sec. 4.1: the smaller of the first radial step
    r_1 - r_0 and the chord 2 r_0 sin(theta_0) sin(dphi/2) next to the pole on
    the innermost sphere."""
    dr = shell.r[1] - shell.r[0]
    dphi = 2.0 * np.pi / shell.n_phi
    chord = 2.0 * shell.r[0] * np.sin(shell.theta[0]) * np.sin(0.5 * dphi)
    return min(dr, chord), dr, chord


def courant_dt(shell, lam=4.0):
    """Delta t = lambda * min(Delta x), Sec. 4.1 (default lambda = 4)."""
    return lam * min_spacing(shell)[0]
