"""Seeded synthetic inputs for the shell evolution.

This module only draws random numbers and evaluates closed-form input fields
at coordinates handed in by the caller.  It holds no spectral derivative,
filter, right-hand-side or time-stepping arithmetic, so it can feed both the
HIP library and an independent checker with identical inputs.

Field order of a state vector: g_ab (10), Pi_ab (10), Phi_xab, Phi_yab,
Phi_zab (10 each) [, H_a (4), d_t H_a (4)], symmetric pairs ordered
tt tx ty tz xx xy xz yy yz zz.  Arrays are shaped [field, phi, theta, r].
"""
import itertools
import math

import numpy as np

PAIRS = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]


def spatial_degree(n_v):
    """Number of spatial indices of every Cartesian component."""
    d2 = [sum(1 for x in ab if x > 0) for ab in PAIRS]
    d = d2 + d2 + [1 + x for x in d2] * 3
    if n_v == 58:
        d += [0, 1, 1, 1] * 2
    return np.array(d[:n_v])


def _monomials(deg):
    return [e for e in itertools.product(range(deg + 1), repeat=3) if sum(e) <= deg]


def _cheb(k, x):
    return np.cos(k * np.arccos(np.clip(x, -1.0, 1.0)))


def spherical_to_cartesian(r, theta, phi):
    """Broadcast 1-d coordinate lists (r fastest) to [phi, theta, r] arrays."""
    r = np.asarray(r)[None, None, :]
    th = np.asarray(theta)[None, :, None]
    ph = np.asarray(phi)[:, None, None]
    return (r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph),
            r * np.cos(th) + 0 * ph)


def band_limited_fields(seed, r, theta, phi, r_min, r_max, n_v=50, l_max=8, n_cheb=None):
    """Band-limited Cartesian tensor fields.

    Component mu is sum_k a_k e^{-k} T_k(x(r)) * P_mu(xhat) with a_k ~ N(0,1),
    T_k the Chebyshev polynomials in x = (2r - r_max - r_min)/(r_max - r_min),
    k < n_cheb (default: len(r)), and P_mu a polynomial of degree
    l_max - d(mu) in the unit vector xhat with N(0,1)/sqrt(#terms)
    coefficients; d(mu) is the number of spatial indices.  Every tetrad
    component of such a tensor contains spin-weighted harmonics with
    l <= l_max only, and every Cartesian component is a trigonometric
    polynomial of degree <= l_max in theta and phi."""
    rng = np.random.default_rng(seed)
    n_r = len(r)
    n_cheb = n_r if n_cheb is None else n_cheb
    x, y, z = spherical_to_cartesian(r, theta, phi)
    rad = np.sqrt(x * x + y * y + z * z)
    xh, yh, zh = x / rad, y / rad, z / rad
    xr = (2.0 * np.asarray(r) - r_max - r_min) / (r_max - r_min)
    deg = spatial_degree(n_v)
    out = np.zeros((n_v,) + x.shape)
    for mu in range(n_v):
        a = rng.standard_normal(n_cheb)
        radial = sum(a[k] * math.exp(-k) * _cheb(k, xr) for k in range(n_cheb))
        mons = _monomials(l_max - deg[mu])
        b = rng.standard_normal(len(mons)) / math.sqrt(len(mons))
        ang = sum(c * xh ** e[0] * yh ** e[1] * zh ** e[2] for c, e in zip(b, mons))
        out[mu] = radial[None, None, :] * ang
    return out


def kerr_schild_metric(x, y, z, mass=1.0):
    """Schwarzschild in Kerr-Schild form g_ab = eta_ab + (2M/r) l_a l_b,
    l_a = (1, x_i/r), as 10 stored components."""
    rad = np.sqrt(x * x + y * y + z * z)
    f = 2.0 * mass / rad
    l = [np.ones_like(rad), x / rad, y / rad, z / rad]
    eta = np.diag([-1.0, 1.0, 1.0, 1.0])
    return np.array([eta[a, b] + f * l[a] * l[b] for (a, b) in PAIRS])


def smooth_perturbation(seed, x, y, z, n_comp, amp=1e-6, r0=6.0, width=1.0, l_max=4):
    """n_comp fields amp * exp(-(r - r0)^2/width^2) * P_c(xhat) with P_c a
    polynomial of degree l_max in xhat (angular content l <= l_max) and
    N(0,1)/sqrt(#terms) coefficients."""
    rng = np.random.default_rng(seed)
    rad = np.sqrt(x * x + y * y + z * z)
    xh, yh, zh = x / rad, y / rad, z / rad
    prof = amp * np.exp(-((rad - r0) / width) ** 2)
    mons = _monomials(l_max)
    out = np.zeros((n_comp,) + rad.shape)
    for c in range(n_comp):
        b = rng.standard_normal(len(mons)) / math.sqrt(len(mons))
        out[c] = prof * sum(cc * xh ** e[0] * yh ** e[1] * zh ** e[2] for cc, e in zip(b, mons))
    return out


def perturbed_kerr_schild(seed, r, theta, phi, mass=1.0, amp=1e-6, r0=6.0, width=1.0):
    """Kerr-Schild metric plus a seeded smooth perturbation (10 components)."""
    x, y, z = spherical_to_cartesian(r, theta, phi)
    return kerr_schild_metric(x, y, z, mass) + smooth_perturbation(seed, x, y, z, 10, amp, r0, width)


def gauge_perturbation(seed, r, theta, phi, amp=1e-6, r0=6.0, width=1.0):
    """Seeded smooth values for the 8 extra gauge fields of the 58-field form:
    returns (dH [4, ...] added to H_a = -Gamma_a, Q [4, ...] = d_t H_a)."""
    x, y, z = spherical_to_cartesian(r, theta, phi)
    p = smooth_perturbation(seed, x, y, z, 8, amp, r0, width)
    return p[:4], p[4:]


# Shell lists of the benchmark workloads: (N_r, N_theta, N_phi, r_min, r_max),
# identical shells adjacent so that they run as one batch.  Shell k draws its
# perturbation with seed base + k (gauge fields: base + 1000 + k).
WORKLOAD_SEED = {"ks33": 2, "ks49": 3, "batch64": 4000, "large8": 5000}


def workload_shells(name):
    """(shells, n_fields) of a named workload."""
    if name == "ks33":
        return [(33, 32, 64, 1.8, 11.8)], 50
    if name == "ks49":
        return [(49, 48, 96, 1.8, 11.8)], 50
    if name == "batch64":
        sizes = [(17, 16), (25, 24), (33, 32), (49, 48)]
        return [(a, b, 2 * b, 1.8, 11.8) for (a, b) in sizes for _ in range(16)], 50
    if name == "large8":
        return [(65, 64, 128, 1.8, 21.8)] * 8, 58
    raise ValueError(name)

