"""Pins of the oracle's projection filters (Sec. 3.2, 3.5)."""
import numpy as np
import pytest
from scipy.special import sph_harm_y

from oracle.grid import Shell
from oracle.swsh import filter_matrix, synthesis_matrix, spin_legendre
from oracle import tensor_filter as tf
from paper_1104_3408_amd import inputs


@pytest.mark.parametrize("N,n_f", [(9, 0), (12, 1), (16, 4), (32, 4)])
def test_filter_matrix_algebra(N, n_f):
    """Idempotent; F^n_{-m} = F^{-n}_m; F^{-n}_m = J F^n_m J (theta reversal);
    band-limited columns pass, the removed degrees are annihilated."""
    J = np.eye(N)[::-1]
    th = np.pi * (np.arange(N) + 0.5) / N
    L = N - 1
    for n in range(-3, 4):
        for m in range(0, N):
            F = filter_matrix(n, m, N, n_f)
            assert np.abs(F @ F - F).max() < 1e-12
            assert np.abs(filter_matrix(n, -m, N, n_f) - filter_matrix(-n, m, N, n_f)).max() < 1e-12
            assert np.abs(filter_matrix(-n, m, N, n_f) - J @ F @ J).max() < 1e-12
            for l in range(max(abs(n), m), L + 1):
                col = spin_legendre(n, l, m, th)
                target = col if l <= L - n_f else 0 * col
                assert np.abs(F @ col - target).max() < 1e-12


def test_unfiltered_projection_is_orthogonal():
    """With n_f = 0, F = P P^+ is the orthogonal projector onto the span of
    the columns of P (Sec. 3.2): symmetric with trace = rank."""
    for n, m in ((0, 0), (2, 3), (-1, 5)):
        F = filter_matrix(n, m, 16, 0)
        P, ls = synthesis_matrix(n, m, 16)
        assert np.abs(F - F.T).max() < 1e-12
        assert np.trace(F) == pytest.approx(len(ls), abs=1e-10)


def test_spin_zero_equals_scipy_least_squares():
    """Spin 0 reduces to the scalar spherical-harmonic transform of Sec. 3.2
    built from scipy's sph_harm_y: analysis by the pseudo-inverse of the full
    synthesis matrix (l = m..L), top n_f degrees zeroed, synthesis (eq. FasPfQ).
    This is not the orthogonal projector onto the truncated basis."""
    N = 10
    th = np.pi * (np.arange(N) + 0.5) / N
    for m in (0, 2, 7):
        ls = np.arange(m, N)
        P = np.array([[sph_harm_y(l, m, t, 0.0).real for l in ls] for t in th])
        F = filter_matrix(0, m, N, 1)
        assert np.abs(P @ np.diag((ls <= N - 2).astype(float)) @ np.linalg.pinv(P) - F).max() < 1e-12
        Pt = P[:, ls <= N - 2]
        if Pt.shape[1] < P.shape[1] and Pt.shape[1] > 0:
            assert np.abs(Pt @ np.linalg.pinv(Pt) - F).max() > 1e-3


def _rand_state(sh, seed, n_v=50):
    return np.random.default_rng(seed).standard_normal((n_v,) + sh.shape)


def test_constant_tensors_pass_yn():
    """Constant Cartesian tensors of rank <= 3 are band-limited at l <= 3 in
    every spin component, so the Yn filter leaves them unchanged when
    L - n_f >= 3; the recombined imaginary part vanishes (eq. ccFn)."""
    sh = Shell(3, 8, 16, 2.0, 4.0)
    u = np.zeros((58,) + sh.shape) + np.random.default_rng(1).standard_normal(58)[:, None, None, None]
    out, imag = tf.yn_filter(u, sh, 4, return_imag=True)
    assert np.abs(out - u).max() < 1e-13
    assert imag < 1e-13


def test_constant_tensor_pin_catches_flipped_spin(monkeypatch):
    """Planted mistake: filtering m-contractions with F_{-1} instead of F_{+1}
    breaks the constant-tensor pin (so the pin fixes the spin convention)."""
    sh = Shell(2, 8, 16, 2.0, 4.0)
    orig = tf.tetrad

    def flipped(shell):
        b, d, s = orig(shell)
        return b, d, {k: -v for k, v in s.items()}
    monkeypatch.setattr(tf, "tetrad", flipped)
    u = np.zeros((50,) + sh.shape) + np.random.default_rng(2).standard_normal(50)[:, None, None, None]
    out = tf.yn_filter(u, sh, 4)
    assert np.abs(out - u).max() > 1e-2


def test_band_limited_fields_pass_yn():
    """Seeded band-limited tensor fields of the 12x12x24 linear-operator case
    (every spin component has l <= 8) pass a filter that keeps l <= 10
    unchanged."""
    sh = Shell(12, 12, 24, 2.0, 12.0)
    u = inputs.band_limited_fields(1, sh.r, sh.theta, sh.phi, 2.0, 12.0)
    out, imag = tf.yn_filter(u, sh, 1, return_imag=True)
    assert np.abs(out - u).max() < 1e-12 * np.abs(u).max()
    assert imag < 1e-12 * np.abs(u).max()


def test_yn_idempotent_and_real_on_random_data():
    sh = Shell(4, 10, 20, 2.0, 5.0)
    u = _rand_state(sh, 3)
    f1, im = tf.yn_filter(u, sh, 2, return_imag=True)
    f2 = tf.yn_filter(f1, sh, 2)
    assert np.abs(f2 - f1).max() < 1e-12
    assert im < 1e-12
    assert np.abs(f1 - u).max() > 0.1


def _rotate_state(u, R):
    """Cartesian components of R.T for every tensor in the state (t passes)."""
    R4 = np.eye(4)
    R4[1:, 1:] = R
    g, Pi, Phi, extra = [np.asarray(x) if x is not None else None for x in _unpack(u)]
    g2 = np.einsum('ac,bd,cd...->ab...', R4, R4, g)
    Pi2 = np.einsum('ac,bd,cd...->ab...', R4, R4, Pi)
    Phi2 = np.einsum('ij,ac,bd,jcd...->iab...', R, R4, R4, Phi)
    out = [g2[a, b] for (a, b) in tf.PAIRS] + [Pi2[a, b] for (a, b) in tf.PAIRS]
    for i in range(3):
        out += [Phi2[i, a, b] for (a, b) in tf.PAIRS]
    return np.array(out)


def _unpack(u):
    from oracle.ghg import unpack
    return unpack(u)


@pytest.mark.parametrize("which", ["z_shift", "x_pi"])
def test_yn_covariant_under_grid_rotations(which):
    """Rotations that map the collocation grid onto itself (about z by one
    phi step; by pi about x: (theta, phi) -> (pi - theta, -phi)) commute with
    the Yn filter exactly, for arbitrary (not band-limited) data, since the
    tetrad rotates with the sphere and rotations preserve the degree l."""
    sh = Shell(3, 9, 18, 2.0, 5.0)
    u = _rand_state(sh, 7)
    if which == "z_shift":
        psi = 2 * np.pi / sh.n_phi
        R = np.array([[np.cos(psi), -np.sin(psi), 0], [np.sin(psi), np.cos(psi), 0], [0, 0, 1]])

        def move(v):                # value at phi_j comes from phi_{j-1}
            return np.roll(v, 1, axis=1)
    else:
        R = np.diag([1.0, -1.0, -1.0])

        def move(v):
            return v[:, (-np.arange(sh.n_phi)) % sh.n_phi][:, :, ::-1]
    rot = lambda v: _rotate_state(move(v), R)
    a = tf.yn_filter(rot(u), sh, 3)
    b = rot(tf.yn_filter(u, sh, 3))
    assert np.abs(a - b).max() < 1e-12


def test_y_and_yg_filters():
    """Y filter: F_0 per component; Yg: n_f(mu) = n_f - d(u^mu) (eq. nfofmu).
    A scalar field with l <= L - n_f passes Y; a vector component x/r (l = 1)
    passes Yg only when n_f - 1 >= ... is honoured per component."""
    sh = Shell(2, 8, 16, 2.0, 4.0)
    x, y, z = sh.cartesian()
    rad = np.sqrt(x * x + y * y + z * z)
    u = np.zeros((50,) + sh.shape)
    u[0] = (z / rad) ** 3                       # g_tt, l <= 3
    u[1] = (x / rad) ** 4                       # g_tx, l <= 4
    L = sh.n_theta - 1
    uy = tf.y_filter(u, sh, L - 4)              # keeps l <= 4 everywhere
    assert np.abs(uy[:2] - u[:2]).max() < 1e-13
    ug = tf.yg_filter(u, sh, L - 4)             # keeps l <= 4 for g_tt, l <= 5 for g_tx
    assert np.abs(ug[:2] - u[:2]).max() < 1e-13
    ug2 = tf.yg_filter(u, sh, L - 3)            # g_tt keeps l <= 3, g_tx keeps l <= 4
    assert np.abs(ug2[:2] - u[:2]).max() < 1e-13
    uy2 = tf.y_filter(u, sh, L - 3)             # keeps l <= 3 only: g_tx (l = 4, 2, 0) changes
    assert np.abs(uy2[1] - u[1]).max() > 1e-3
    assert list(tf.spatial_degree(50)[:10]) == [0, 1, 1, 1, 2, 2, 2, 2, 2, 2]
    assert list(tf.spatial_degree(50)[20:30]) == [1, 2, 2, 2, 3, 3, 3, 3, 3, 3]
