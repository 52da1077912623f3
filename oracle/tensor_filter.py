"""Scalar Y, graded Yg and tensor Yn projection filters (oracle; test
infrastructure only).

A filter F_n of spin n acts on a complex function on every sphere of the
shell: Fourier analysis in phi (Sec. 3.1, complex form of eqs. Fanalysis /
Fsynthesis with J = N_phi and the Nyquist mode dropped), the theta filter
matrix F^n_m = P diag P^+ for every Fourier order m (Sec. 3.5 eq. FasPfQ), and
Fourier synthesis.

The Yn filter (Sec. 3.5) decomposes each tensor on the complex tetrad
(t, r, m, mbar) of Sec. 3.4 eq. tetrad, filters each component with the spin
filter of its weight, and recombines (eq. tensorexpansion).  Spin label used
here: a component obtained by contracting k_m slots with m and k_mbar slots
with mbar is filtered with F_n, n = k_m - k_mbar, in the basis Y^n of Sec. 3.3
(so m . x-hat is expanded in Y^{+1}, as in App. B eq. mxfinite).

Field order of a state vector (also used by the GHG module):
  g_ab (10), Pi_ab (10), Phi_xab (10), Phi_yab (10), Phi_zab (10)
  [, H_a (4), dH_a/dt (4)] with pairs ab = tt tx ty tz xx xy xz yy yz zz.
"""
from functools import lru_cache
import itertools

import numpy as np

from .swsh import filter_matrix

PAIRS = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]


def pair_index(a, b):
    return PAIRS.index((min(a, b), max(a, b)))


@lru_cache(maxsize=None)
def _fmat(n, m, n_theta, n_f):
    return filter_matrix(n, m, n_theta, n_f)


@lru_cache(maxsize=None)
def _fstack(n, n_theta, n_phi, n_f):
    M = n_phi // 2
    ms = np.arange(-(M - 1), M)
    return ms, np.array([_fmat(n, int(m), n_theta, n_f) for m in ms])


def spin_filter(f, n, shell, n_f):
    """F_n(f) for a (complex) function f shaped [N_phi, N_theta, N_r]:
    forward Fourier transform in phi for the orders |m| <= N_phi/2 - 1
    (Nyquist dropped), theta filter F^n_m for every order m, backward Fourier
    transform (Sec. 3.3 last paragraph, Sec. 3.5)."""
    n_phi, n_th, n_r = f.shape
    ms, Fs = _fstack(n, n_th, n_phi, n_f)
    E = np.exp(-1j * np.outer(ms, shell.phi))                 # [m, j]
    fm = (E @ f.reshape(n_phi, -1)).reshape(len(ms), n_th, n_r) / n_phi
    gm = np.matmul(Fs, fm)                                    # per m: F^n_m f_m
    return (E.conj().T @ gm.reshape(len(ms), -1)).reshape(f.shape)


def tetrad(shell):
    """Complex tetrad of Sec. 3.4 eq. tetrad with Cartesian 4-components:
    returns dict label -> array [4 (t,x,y,z), N_phi, N_theta, N_r] for the
    basis vectors E_A (A = t, r, m, mbar), the dual vectors used to
    recombine (t->t, r->r, m->mbar, mbar->m: mbar . m = 1), and spin labels."""
    _, th, ph = shell.coords()
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    zero = np.zeros_like(st)
    one = np.ones_like(st)
    t_vec = np.array([one, zero, zero, zero], dtype=complex)
    r_vec = np.array([zero, st * cp, st * sp, ct], dtype=complex)
    th_vec = np.array([zero, ct * cp, ct * sp, -st], dtype=complex)
    ph_vec = np.array([zero, -sp, cp, zero], dtype=complex)
    m_vec = (th_vec + 1j * ph_vec) / np.sqrt(2.0)
    mb_vec = (th_vec - 1j * ph_vec) / np.sqrt(2.0)
    basis = {'t': t_vec, 'r': r_vec, 'm': m_vec, 'mb': mb_vec}
    dual = {'t': t_vec, 'r': r_vec, 'm': mb_vec, 'mb': m_vec}
    spin = {'t': 0, 'r': 0, 'm': 1, 'mb': -1}
    return basis, dual, spin


def yn_filter_tensor(T, slots, shell, n_f):
    """Yn filter of one real tensor field T with Cartesian covariant indices.

    T: array [d_1, ..., d_k, N_phi, N_theta, N_r]; slots: list of '4' (index
    t,x,y,z) or '3' (spatial x,y,z).  Every tetrad component
    c_A = E_{A1}^{a1} ... E_{Ak}^{ak} T_{a1..ak} is filtered with F_{n(A)},
    n(A) = #m - #mbar, then T' = sum_A F(c_A) Edual^{A1} ... (Sec. 3.5).
    Returns the real part and the largest imaginary part (which must vanish,
    Sec. 3.3 eq. ccFn)."""
    basis, dual, spin = tetrad(shell)

    def restrict(vec, kind):
        return vec if kind == '4' else vec[1:]

    labels = []
    for kind in slots:
        labels.append(['t', 'r', 'm', 'mb'] if kind == '4' else ['r', 'm', 'mb'])
    out = np.zeros(T.shape, dtype=complex)
    k = len(slots)
    letters = 'abcd'[:k]
    for A in itertools.product(*labels):
        comp = T.astype(complex)
        # contract slot by slot (leading axis each time)
        for s, lab in enumerate(A):
            comp = np.einsum('a...,a...->...', restrict(basis[lab], slots[s]), comp)
        n = sum(spin[lab] for lab in A)
        fc = spin_filter(comp, n, shell, n_f)
        term = fc
        for s in reversed(range(k)):
            vec = restrict(dual[A[s]], slots[s])
            extra = term.ndim - fc.ndim
            vec = vec.reshape(vec.shape[:1] + (1,) * extra + vec.shape[1:])
            term = vec * term[None]
        out += term
    return out.real, np.max(np.abs(out.imag))


def _sym2(u10):
    """10 stored components -> full symmetric 4x4 array."""
    full = np.empty((4, 4) + u10.shape[1:], dtype=u10.dtype)
    for p, (a, b) in enumerate(PAIRS):
        full[a, b] = u10[p]
        full[b, a] = u10[p]
    return full


def _pack2(full):
    return np.array([full[a, b] for (a, b) in PAIRS])


def yn_filter(u, shell, n_f, return_imag=False):
    """Tensor Yn filter of a full state vector (50 or 58 fields), Sec. 3.5."""
    n_v = u.shape[0]
    out = np.empty_like(u)
    imag = 0.0
    for base in (0, 10):                       # g_ab, Pi_ab
        T = _sym2(u[base:base + 10])
        Tf, im = yn_filter_tensor(T, ['4', '4'], shell, n_f)
        out[base:base + 10] = _pack2(Tf)
        imag = max(imag, im)
    Phi = np.array([_sym2(u[20 + 10 * i:30 + 10 * i]) for i in range(3)])
    Pf, im = yn_filter_tensor(Phi, ['3', '4', '4'], shell, n_f)
    for i in range(3):
        out[20 + 10 * i:30 + 10 * i] = _pack2(Pf[i])
    imag = max(imag, im)
    if n_v == 58:
        for base in (50, 54):                  # H_a and its time derivative
            Vf, im = yn_filter_tensor(u[base:base + 4], ['4'], shell, n_f)
            out[base:base + 4] = Vf
            imag = max(imag, im)
    return (out, imag) if return_imag else out


def spatial_degree(n_v):
    """Number of spatial indices d(u^mu) of every Cartesian component (Sec. 3.5)."""
    d2 = [sum(1 for x in ab if x > 0) for ab in PAIRS]
    d = d2 + d2 + [1 + x for x in d2] * 3
    if n_v == 58:
        d += [0, 1, 1, 1] * 2
    return np.array(d[:n_v])


def y_filter(u, shell, n_f):
    """Scalar Y filter: F_0 on every Cartesian component (Sec. 3.5)."""
    return np.array([spin_filter(u[mu], 0, shell, n_f).real for mu in range(u.shape[0])])


def yg_filter(u, shell, n_f):
    """Graded Yg filter: F_0 with n_f(mu) = n_f - d(u^mu) (Sec. 3.5 eq. nfofmu)."""
    d = spatial_degree(u.shape[0])
    return np.array([spin_filter(u[mu], 0, shell, n_f - d[mu]).real
                     for mu in range(u.shape[0])])
