"""Spin-weighted spherical harmonics and projection-filter matrices (oracle;
test infrastructure only).

Sec. 3.3 relates the spin-n associated Legendre functions to Wigner d
functions: Phat^n_{lm}(theta) = (-1)^n sqrt((2l+1)/(4 pi)) d^l_{m,-n}(theta),
with Y^n_{lm} = Phat^n_{lm} e^{i m phi}.  The oracle evaluates d from its
textbook definition, the matrix element <l m'| exp(-i beta J_y) |l m> of the
rotation operator in the spin-l representation (ladder operators with the
Condon-Shortley phase), through the eigen-decomposition of the Hermitian
J_y.  This route is independent of the recursion in l and n (Sec. 3.3 eqs.
Yninc, Yndec) that the HIP library uses, and it is numerically stable.

The filter matrices follow Sec. 3.2 (pseudo-inverse of the Legendre synthesis
matrix via the SVD) and Sec. 3.5 eq. FasPfQ: F = P diag(1..1, 0..0) P^+.
"""
from functools import lru_cache

import numpy as np


@lru_cache(maxsize=None)
def _jy_eig(two_l):
    """Eigen-decomposition of J_y in the basis |l, m>, m = l, l-1, ..., -l."""
    l = two_l / 2.0
    ms = l - np.arange(two_l + 1)                 # descending m
    dim = two_l + 1
    jplus = np.zeros((dim, dim))
    for col in range(1, dim):                     # J_+ |l m> = sqrt(l(l+1)-m(m+1)) |l m+1>
        m = ms[col]
        jplus[col - 1, col] = np.sqrt(l * (l + 1) - m * (m + 1))
    jminus = jplus.T
    jy = (jplus - jminus) / 2j
    w, v = np.linalg.eigh(jy)
    return ms, w, v


def wigner_d(l, beta):
    """Wigner small-d matrix d^l_{m'm}(beta) = <l m'| exp(-i beta J_y) |l m>.

    Returns (ms, d) with d[a, b] = d^l_{ms[a], ms[b]}(beta) for the descending
    list ms = l, ..., -l (integer l only here)."""
    ms, w, v = _jy_eig(int(round(2 * l)))
    rot = (v * np.exp(-1j * beta * w)) @ v.conj().T
    if np.max(np.abs(rot.imag)) > 1e-10:
        raise RuntimeError("Wigner d should be real")
    return ms, rot.real


def spin_legendre(n, l, m, theta):
    """Phat^n_{lm}(theta) = (-1)^n sqrt((2l+1)/(4 pi)) d^l_{m,-n}(theta) (Sec. 3.3);
    zero when l < max(|m|, |n|)."""
    theta = np.atleast_1d(np.asarray(theta, dtype=float))
    if l < max(abs(m), abs(n)):
        return np.zeros_like(theta)
    out = np.empty_like(theta)
    for t, th in enumerate(theta):
        ms, d = wigner_d(l, th)
        a = int(l - m)                 # row of m' = m
        b = int(l + n)                 # column of m = -n  (ms[b] = l - (l + n) = -n)
        out[t] = d[a, b]
    return (-1.0) ** n * np.sqrt((2 * l + 1) / (4 * np.pi)) * out


@lru_cache(maxsize=None)
def _d_columns(l, theta_key, n_max=3):
    """d^l_{m', -n}(theta) for all m' (descending, rows) and n = -n_max..n_max
    (columns, only |n| <= l), at the angles in theta_key; shape
    [len(theta), 2l+1, 2 n_max + 1] (absent columns zero)."""
    theta = np.array(theta_key)
    ms, w, v = _jy_eig(2 * l)
    out = np.zeros((theta.size, 2 * l + 1, 2 * n_max + 1))
    for c, n in enumerate(range(-n_max, n_max + 1)):
        if abs(n) > l:
            continue
        vrow = v[l + n].conj()                     # <m| for m = -n is row l + n
        for t, th in enumerate(theta):
            col = (v * np.exp(-1j * th * w)) @ vrow
            out[t, :, c] = col.real
    return out


def spin_legendre_table(n, m, l_max, theta):
    """All Phat^n_{lm}(theta_i) for l = 0..l_max, shape [len(theta), l_max+1]
    (same definition as spin_legendre, cached per degree)."""
    theta = np.atleast_1d(np.asarray(theta, dtype=float))
    key = tuple(float(t) for t in theta)
    tab = np.zeros((theta.size, l_max + 1))
    for l in range(max(abs(m), abs(n)), l_max + 1):
        d = _d_columns(l, key)
        tab[:, l] = d[:, int(l - m), n + 3] * np.sqrt((2 * l + 1) / (4 * np.pi))
    return (-1.0) ** n * tab


def swsh(n, l, m, theta, phi):
    """Y^n_{lm}(theta, phi) = Phat^n_{lm}(theta) e^{i m phi} (Sec. 3.3)."""
    return spin_legendre(n, l, m, theta) * np.exp(1j * m * np.asarray(phi, dtype=float))


def synthesis_matrix(n, m, n_theta):
    """Legendre synthesis matrix (P^n_m)_{ik} = Phat^n_{(k+|m|) m}(theta_i)
    (Sec. 3.2 eq. Pmatrix, Sec. 3.3), for l = |m|..L with L = N_theta - 1.
    Returns (P, ls) with the identically zero columns l < |n| dropped, so P
    has full column rank."""
    theta = np.pi * (np.arange(n_theta) + 0.5) / n_theta
    L = n_theta - 1
    l0 = max(abs(m), abs(n))
    ls = np.arange(l0, L + 1)
    tab = spin_legendre_table(n, m, L, theta)
    return tab[:, ls], ls


def filter_matrix(n, m, n_theta, n_f):
    """Projection filter for spin n and Fourier order m removing the top n_f
    degrees: F = P diag(f) P^+ with f_l = 1 for l <= L - n_f and 0 otherwise,
    P^+ the Moore-Penrose pseudo-inverse from the SVD (Sec. 3.2 eq. forwardL,
    Sec. 3.5 eq. FasPfQ).  Shape N_theta x N_theta; zero when no degree
    survives."""
    L = n_theta - 1
    if abs(m) > L:
        return np.zeros((n_theta, n_theta))
    P, ls = synthesis_matrix(n, m, n_theta)
    if P.shape[1] == 0:
        return np.zeros((n_theta, n_theta))
    Pplus = np.linalg.pinv(P)
    keep = (ls <= L - n_f).astype(float)
    return P @ np.diag(keep) @ Pplus
