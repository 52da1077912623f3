"""Pins of the oracle's spin-weighted Legendre functions (Sec. 3.3, App. B)."""
import numpy as np
import pytest
from numpy import sin, cos, sqrt, pi  # noqa: F401  (used by the golden expressions)
from scipy.special import sph_harm_y

from conftest import read_golden
from oracle.swsh import spin_legendre, swsh, wigner_d, spin_legendre_table

THETA = np.array([0.05, 0.4, 1.0, 1.5707963, 2.2, 3.0])


@pytest.mark.parametrize("row", read_golden("swsh_appB.txt"), ids=lambda r: "n%s_l%s_m%s" % tuple(r[:3]))
def test_appendix_b_closed_forms(row):
    """Every closed form printed in App. B for n >= 0, l <= 2."""
    n, l, m = map(int, row[:3])
    expr = " ".join(row[3:])
    t = THETA
    expect = eval(expr) * np.ones_like(t)
    assert np.abs(spin_legendre(n, l, m, t) - expect).max() < 1e-13


@pytest.mark.parametrize("n,l,m", [(n, l, m) for n in (1, 2, 3) for l in range(0, 7) for m in range(-l, l + 1)])
def test_negative_spin_symmetry(n, l, m):
    """Phat^{-n}_{lm} = (-1)^{n+m} Phat^n_{l,-m} (Sec. 3.3, App. B)."""
    a = spin_legendre(-n, l, m, THETA)
    b = (-1) ** (n + m) * spin_legendre(n, l, -m, THETA)
    assert np.abs(a - b).max() < 1e-13


def _alpha(n, l):
    return np.sqrt((l - n + 1) / (l + n))


def _beta(n, l, m):
    return np.sqrt((2 * l + 1) / (2 * l - 1) * (l + n - 1) * (l * l - m * m) / (l + n)) / l


@pytest.mark.parametrize("n", [1, 2, 3])
def test_recursion_in_n_holds(n):
    """The printed two-term recursions (Sec. 3.3 eqs. Yninc, Yndec, Yncoeffs)
    hold for the Wigner-d based functions: raising n from n-1 and lowering
    -n from -n+1."""
    t = THETA
    for l in range(n, 9):
        for m in range(-l, l + 1):
            up = (_alpha(n, l) * (m / l - cos(t)) / sin(t) * spin_legendre(n - 1, l, m, t)
                  + _beta(n, l, m) / sin(t) * spin_legendre(n - 1, l - 1, m, t))
            assert np.abs(up - spin_legendre(n, l, m, t)).max() < 1e-12
            k = -n
            dn = (_alpha(-k, l) * (m / l + cos(t)) / sin(t) * spin_legendre(k + 1, l, m, t)
                  - _beta(-k, l, m) / sin(t) * spin_legendre(k + 1, l - 1, m, t))
            assert np.abs(dn - spin_legendre(k, l, m, t)).max() < 1e-12


def _inner(n1, l1, m1, n2, l2, m2, nq=200):
    """(Y^{n1}_{l1 m1}, Y^{n2}_{l2 m2}) by Gauss-Legendre quadrature in theta."""
    if m1 != m2:
        return 0.0
    x, w = np.polynomial.legendre.leggauss(nq)
    th = 0.5 * np.pi * (x + 1)
    f = spin_legendre(n1, l1, m1, th) * spin_legendre(n2, l2, m2, th) * np.sin(th)
    return 2 * np.pi * 0.5 * np.pi * np.sum(w * f)


@pytest.mark.parametrize("row", read_golden("swsh_inner_products.txt"))
def test_appendix_b_inner_products(row):
    n1, l1, m1, n2, l2, m2 = map(int, row[:6])
    val = eval(row[6])
    assert _inner(n1, l1, m1, n2, l2, m2) == pytest.approx(val, abs=1e-12)


@pytest.mark.parametrize("n", [-3, -1, 0, 2, 3])
def test_orthonormal_for_fixed_spin(n):
    for m in (-2, 0, 1):
        for l1 in range(max(abs(n), abs(m)), 7):
            for l2 in range(max(abs(n), abs(m)), 7):
                assert _inner(n, l1, m, n, l2, m) == pytest.approx(float(l1 == l2), abs=1e-12)


def test_mx_expansion():
    """m_x = (cos th cos ph - i sin ph)/sqrt2 = sqrt(2 pi/3)(Y^1_{1,1} - Y^1_{1,-1})
    (App. B eq. mxfinite)."""
    rng = np.random.default_rng(5)
    th = rng.uniform(0.01, np.pi - 0.01, 20)
    ph = rng.uniform(0, 2 * np.pi, 20)
    lhs = (cos(th) * cos(ph) - 1j * sin(ph)) / sqrt(2)
    rhs = np.sqrt(2 * np.pi / 3) * (swsh(1, 1, 1, th, ph) - swsh(1, 1, -1, th, ph))
    assert np.abs(lhs - rhs).max() < 1e-14


@pytest.mark.parametrize("l", [0, 1, 3, 7, 12])
def test_spin_zero_is_scipy_spherical_harmonic(l):
    """Y^0_{lm} is the ordinary orthonormal spherical harmonic with the
    Condon-Shortley phase (Sec. 3.3): compare with scipy's sph_harm_y."""
    rng = np.random.default_rng(l)
    th = rng.uniform(0, np.pi, 9)
    ph = rng.uniform(0, 2 * np.pi, 9)
    for m in range(-l, l + 1):
        assert np.abs(swsh(0, l, m, th, ph) - sph_harm_y(l, m, th, ph)).max() < 1e-12


def test_wigner_d_is_rotation():
    """d^l(0) = 1, d^l(b1) d^l(b2) = d^l(b1 + b2), d^l orthogonal; d^1_{1,0} = -sin/sqrt2."""
    for l in (1, 4, 9):
        _, d0 = wigner_d(l, 0.0)
        assert np.allclose(d0, np.eye(2 * l + 1), atol=1e-14)
        _, d1 = wigner_d(l, 0.3)
        _, d2 = wigner_d(l, 0.9)
        _, d12 = wigner_d(l, 1.2)
        assert np.allclose(d1 @ d2, d12, atol=1e-13)
        assert np.allclose(d1 @ d1.T, np.eye(2 * l + 1), atol=1e-13)
    ms, d = wigner_d(1, 0.7)
    assert d[0, 1] == pytest.approx(-np.sin(0.7) / np.sqrt(2), abs=1e-15)


def test_table_matches_pointwise():
    th = np.pi * (np.arange(16) + 0.5) / 16
    for n in (-3, 0, 2):
        for m in (-4, 0, 5):
            tab = spin_legendre_table(n, m, 15, th)
            for l in range(16):
                assert np.abs(tab[:, l] - spin_legendre(n, l, m, th)).max() < 1e-13


def test_high_degree_stable():
    """Stable at the largest degrees used (l = 63): orthonormality by
    quadrature stays at round-off."""
    for n, m in ((3, 0), (-2, 40), (1, 63)):
        for l in (max(abs(m), abs(n)), 63):
            assert _inner(n, l, m, n, l, m, nq=300) == pytest.approx(1.0, abs=1e-11)
