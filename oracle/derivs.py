"""3-d spectral derivatives on the shell (oracle; test infrastructure only).

Fields are numpy arrays shaped [..., N_phi, N_theta, N_r] (r fastest), one
leading axis per variable.  Derivatives are taken along coordinate lines
(Sec. 2.2, 2.4) with the 1-d matrices of Sec. 2.3; the theta derivative uses
the explicit double cover of Sec. 2.1.  The Cartesian derivatives follow from
the chain rule of Sec. 2.2 eq. dvdx with the analytic Jacobian.
"""
import numpy as np

from .grid import cheb_diff_matrix, fourier_diff_matrix


def d_r(u, shell):
    """d/dr along each radial line: (D_1 u) with D_1 the rescaled Chebyshev
    matrix (Sec. 2.4 eq. D1)."""
    D = cheb_diff_matrix(shell.n_r, shell.r_min, shell.r_max)
    return np.einsum('kl,...l->...k', D, u)


def meridian_circle(u, j, shell):
    """Values on the full 2 N_theta-point theta circle through phi_j: for
    i < N_theta the stored f(theta_i, phi_j); for i >= N_theta the identity
    f(theta, phi) = f(2 pi - theta, pi + phi) gives
    f(theta_{2N-1-i}, phi_j + pi) (Sec. 2.1, double cover).  Returns an array
    shaped [..., 2 N_theta, N_r]."""
    n_phi = shell.n_phi
    jp = (j + n_phi // 2) % n_phi
    upper = u[..., j, :, :]
    lower = u[..., jp, ::-1, :]
    return np.concatenate([upper, lower], axis=-2)


def d_theta(u, shell):
    """d/dtheta with the Fourier matrix on the double-covered theta circle,
    keeping only the single-cover rows (Sec. 2.1, Sec. 2.4 eq. D2).  As in
    d_phi, the mean over each circle is subtracted first (same result up to
    rounding)."""
    n_th = shell.n_theta
    FD = fourier_diff_matrix(2 * n_th)
    out = np.empty_like(u)
    for j in range(shell.n_phi):
        circle = meridian_circle(u, j, shell)
        circle = circle - circle.mean(axis=-2, keepdims=True)   # FD annihilates constants
        dcircle = np.einsum('ab,...bk->...ak', FD, circle)
        out[..., j, :, :] = dcircle[..., :n_th, :]
    return out


def d_phi(u, shell):
    """d/dphi with the Fourier matrix on the N_phi-point circle (Sec. 2.4 eq. D3).

    The mean over the circle is subtracted first.  The derivative of a
    constant vanishes, so the rows of FD sum to zero (Sec. 2.3) and the result
    is the same up to rounding; the rounding is then proportional to the
    variation of u along the circle instead of to its size, which matters
    where the chain rule divides by r sin(theta)."""
    FD = fourier_diff_matrix(shell.n_phi)
    v = u - u.mean(axis=-3, keepdims=True)
    return np.einsum('jl,...lik->...jik', FD, v)


def coordinate_derivs(u, shell):
    """(d_r u, d_theta u, d_phi u)."""
    return d_r(u, shell), d_theta(u, shell), d_phi(u, shell)


def jacobian(shell):
    """Analytic d(r, theta, phi)/d(x, y, z) at the collocation points, as a
    [3 (x,y,z)][3 (r,theta,phi)] nested list of field-shaped arrays (Sec. 2.2).
    The 1/sin(theta) pole is never sampled because theta is staggered."""
    r, th, ph = shell.coords()
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    zero = np.zeros_like(r)
    return [[st * cp, ct * cp / r, -sp / (r * st)],
            [st * sp, ct * sp / r, cp / (r * st)],
            [ct, -st / r, zero]]


def cartesian_derivs(u, shell):
    """Cartesian partial derivatives (d_x u, d_y u, d_z u) by the chain rule
    d_i = (d xtilde^j/d x^i) d_{xtilde^j}, Sec. 2.2 eq. dvdx."""
    dr, dth, dph = coordinate_derivs(u, shell)
    J = jacobian(shell)
    return tuple(J[i][0] * dr + J[i][1] * dth + J[i][2] * dph for i in range(3))
