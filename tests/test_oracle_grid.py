"""Pins of the oracle's grid, differentiation matrices and time-step rule."""
import numpy as np
import pytest

from conftest import read_golden
from oracle.grid import (Shell, cheb_diff_matrix, fourier_diff_matrix, min_spacing,
                         courant_dt, radial_points, theta_points)


def test_grid_endpoints_and_symmetry():
    r = radial_points(17, 1.8, 11.8)
    assert r[0] == pytest.approx(1.8, abs=1e-15) and r[-1] == pytest.approx(11.8, abs=1e-14)
    th = theta_points(9)
    assert np.allclose(th + th[::-1], np.pi, atol=1e-15)   # staggered, pole-free
    assert th.min() > 0 and th.max() < np.pi


@pytest.mark.parametrize("row", read_golden("dtfac.txt"))
def test_dtfac_table(row):
    """Tab. dtfac: the two printed ratios dt_stab/min(dr) and
    dt_stab/min(r dphi) follow from the grid (chord form of the pole spacing),
    and lambda_max is the larger ratio floored to one decimal."""
    n_r, n_th, n_ph = map(int, row[:3])
    dt_stab, _, ratio_r, ratio_phi, lam_max = map(float, row[3:])
    sh = Shell(n_r, n_th, n_ph, 1.8, 11.8)
    dx, dr, chord = min_spacing(sh)
    assert dt_stab / dr == pytest.approx(ratio_r, abs=1.5e-3)
    assert dt_stab / chord == pytest.approx(ratio_phi, abs=1.5e-3)
    assert np.floor(10 * dt_stab / dx) / 10 == pytest.approx(lam_max, abs=1e-9)


def test_courant_default():
    sh = Shell(33, 32, 64, 1.8, 11.8)
    assert courant_dt(sh, 4.0) == pytest.approx(4 * min_spacing(sh)[0])
    assert courant_dt(sh) == pytest.approx(0.03467, abs=5e-6)


@pytest.mark.parametrize("n", [5, 12, 17, 33])
def test_chebyshev_exact_on_polynomials(n):
    """D_r differentiates polynomials of degree <= N-1 exactly; row sums vanish."""
    a, b = 1.8, 11.8
    D = cheb_diff_matrix(n, a, b)
    r = radial_points(n, a, b)
    assert np.abs(D.sum(axis=1)).max() < 1e-12 * np.abs(D).max()
    rng = np.random.default_rng(n)
    c = rng.standard_normal(n)
    x = (2 * r - a - b) / (b - a)
    p = np.polynomial.chebyshev.Chebyshev(c)
    exact = p.deriv()(x) * 2 / (b - a)
    assert np.abs(D @ p(x) - exact).max() < 1e-12 * max(1, np.abs(exact).max()) * n


def test_chebyshev_plain_n3():
    """Brute force for N = 3 on [-1, 1]: x = (-1, 0, 1), derivative of a
    quadratic through the points."""
    D = cheb_diff_matrix(3, -1.0, 1.0)
    expect = np.array([[-1.5, 2.0, -0.5], [-0.5, 0.0, 0.5], [0.5, -2.0, 1.5]])
    assert np.allclose(D, expect, atol=1e-14)


@pytest.mark.parametrize("n", [6, 18, 24, 64])
def test_fourier_exact_on_trig_polynomials(n):
    """FD is exact on trigonometric polynomials below Nyquist and maps the
    Nyquist mode cos(N x/2) to zero."""
    D = fourier_diff_matrix(n)
    x = 2 * np.pi * np.arange(n) / n
    rng = np.random.default_rng(n)
    f = np.zeros(n)
    df = np.zeros(n)
    for m in range(n // 2):
        a, b = rng.standard_normal(2)
        f += a * np.cos(m * x) + b * np.sin(m * x)
        df += -a * m * np.sin(m * x) + b * m * np.cos(m * x)
    assert np.abs(D @ f - df).max() < 1e-12 * n
    assert np.abs(D @ np.cos(n // 2 * x)).max() < 1e-12 * n
    assert np.allclose(D, -D.T)
