"""Pins of the oracle's GHG right-hand side, boundary operator and RK4."""
import numpy as np
import pytest
import sympy as sp

from conftest import read_golden
from oracle import ghg
from oracle.ghg import unpack, pack, dependent, freeze_incoming, characteristic_matrix
from oracle.grid import Shell, courant_dt
from oracle.evolve import Evolution
from oracle import initial_data
from paper_1104_3408_amd import inputs

PAIRS = ghg.PAIRS


def _ks_fields(x, M=1.0):
    """Kerr-Schild state at points x[3, P] (complex-safe closed forms of
    App. A.3): g = eta + f l l, Phi_iab = d_i g_ab analytically,
    alpha = (1+f)^-1/2, beta^i = l^i f/(1+f), Pi = beta^i Phi_i / alpha."""
    r = np.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
    f = 2 * M / r
    l = [np.ones_like(r), x[0] / r, x[1] / r, x[2] / r]
    eta = np.diag([-1.0, 1, 1, 1])
    g = np.array([[eta[a, b] + f * l[a] * l[b] for b in range(4)] for a in range(4)])
    df = [-2 * M * x[i] / r ** 3 for i in range(3)]
    dl = [[np.zeros_like(r)] + [((i == j) / r - x[i] * x[j] / r ** 3) for j in range(3)] for i in range(3)]
    Phi = np.array([[[df[i] * l[a] * l[b] + f * (dl[i][a] * l[b] + l[a] * dl[i][b])
                      for b in range(4)] for a in range(4)] for i in range(3)])
    alpha = 1 / np.sqrt(1 + f)
    beta = [l[i + 1] * f / (1 + f) for i in range(3)]
    Pi = sum(beta[i] * Phi[i] for i in range(3)) / alpha
    return g, Pi, Phi


def _ks_state(x):
    g, Pi, Phi = _ks_fields(x)
    return pack(g, Pi, Phi)


def _ks_gauge(x):
    """H_a = -Gamma_a of the static metric (eq. gauge), complex-safe: with
    d_t g = 0, Gamma_cab = (Phi_abc + Phi_bac - Phi_cab)/2 (spatial a, b, c),
    Gamma_c = g^ab Gamma_cab, g^ab = eta^ab - f l^a l^b."""
    g, Pi, Phi = _ks_fields(x)
    r = np.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
    f = 2 / r
    lu = [-np.ones_like(r), x[0] / r, x[1] / r, x[2] / r]
    etai = np.diag([-1.0, 1, 1, 1])
    gi = np.array([[etai[a, b] - f * lu[a] * lu[b] for b in range(4)] for a in range(4)])
    D = np.concatenate([np.zeros_like(Phi[:1]), Phi])       # D[c,a,b] = d_c g_ab
    Gam = 0.5 * (np.einsum('abc...->cab...', D) + np.einsum('bac...->cab...', D) - D)
    return -np.einsum('ab...,cab...->c...', gi, Gam)


def _cstep(fun, x, h=1e-30):
    """Exact first derivatives d_k fun(x) by the complex step."""
    out = []
    for k in range(3):
        xc = x.astype(complex)
        xc[k] += 1j * h
        out.append(fun(xc).imag / h)
    return np.array(out)


def _points(n=16, seed=0, rmin=1.8, rmax=11.8):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3, n))
    v /= np.linalg.norm(v, axis=0)
    return v * rng.uniform(rmin, rmax, n)


def test_kerr_schild_rhs_vanishes_with_exact_derivatives():
    """Kerr-Schild is static (App. A.3): with exact derivatives every
    component of the GHG right-hand side vanishes to round-off, which
    exercises every term of eqs. gdot, Phidot, Pidot that is non-zero on the
    solution."""
    x = _points()
    u = _ks_state(x)
    du = _cstep(_ks_state, x)
    H = _ks_gauge(x)
    dH = np.concatenate([np.zeros_like(H)[None], _cstep(_ks_gauge, x)])
    r = ghg.rhs(u, du, H, dH)
    assert np.abs(r).max() < 1e-12
    # the pieces are not individually small
    assert np.abs(du).max() > 0.1 and np.abs(dH).max() > 0.1


def test_kerr_schild_rhs_pin_catches_dropped_term(monkeypatch):
    """Planted mistake: dropping the quadratic Gamma-Gamma contraction in
    eq. Pidot makes the static-solution pin fail."""
    x = _points(4, 1)
    u = _ks_state(x)
    du = _cstep(_ks_state, x)
    H = _ks_gauge(x)
    dH = np.concatenate([np.zeros_like(H)[None], _cstep(_ks_gauge, x)])
    orig = ghg._es

    def broken(spec, *ops):
        if spec == 'cd...,ef...,ace...,bdf...->ab...':
            return 0 * orig(spec, *ops)
        return orig(spec, *ops)
    monkeypatch.setattr(ghg, "_es", broken)
    assert np.abs(ghg.rhs(u, du, H, dH)).max() > 1e-3


def test_christoffel_contraction_against_sympy():
    """Gamma_a of the Kerr-Schild metric with the metric derivatives taken
    symbolically (sympy) and d_t g = 0 equals the oracle's route through
    the first-order variables (eq. Gamma with d_t g from eq. gdot)."""
    X = sp.symbols('x y z', real=True)
    r = sp.sqrt(sum(c ** 2 for c in X))
    l = [1] + [c / r for c in X]
    eta = sp.diag(-1, 1, 1, 1)
    g = sp.Matrix(4, 4, lambda a, b: eta[a, b] + 2 / r * l[a] * l[b])
    dgs = [[[sp.diff(g[a, b], X[c]) for b in range(4)] for a in range(4)] for c in range(3)]
    pts = _points(3, 2)
    u = _ks_state(pts)
    gg, Pi, Phi, _ = unpack(u)
    got = dependent(gg, Pi, Phi)['Gam_c']
    for p in range(3):
        sub = dict(zip(X, pts[:, p]))
        gnum = np.array(g.evalf(subs=sub), dtype=float)
        D = np.zeros((4, 4, 4))
        for c in range(3):
            D[c + 1] = np.array([[float(dgs[c][a][b].evalf(subs=sub)) for b in range(4)] for a in range(4)])
        Gam = 0.5 * (np.einsum('abc->cab', D) + np.einsum('bac->cab', D) - D)
        expect = np.einsum('ab,cab->c', np.linalg.inv(gnum), Gam)
        assert np.allclose(got[:, p], expect, atol=1e-13)


def test_inverse_metric_matches_3p1_closed_form():
    """g^ab by inversion equals the 3+1 form g^tt = -1/alpha^2,
    g^ti = beta^i/alpha^2, g^ij = gamma^ij - beta^i beta^j/alpha^2 (App. A.1)."""
    x = _points(8, 3)
    u = _ks_state(x) + 0.05 * np.random.default_rng(3).standard_normal((50, 8))
    g, Pi, Phi, _ = unpack(u)
    q = dependent(g, Pi, Phi)
    a2 = q['alpha'] ** 2
    b = q['beta_up']
    assert np.allclose(q['g_inv'][0, 0], -1 / a2)
    assert np.allclose(q['g_inv'][0, 1:], b / a2)
    assert np.allclose(q['g_inv'][1:, 1:], q['gam_inv'] - b[:, None] * b[None] / a2)
    n_low, n_up = q['n_low'], q['n_up']
    assert np.allclose(np.einsum('a...,a...->...', n_low, n_up), -1)


def _principal_symbol(u, s_low):
    """-(d rhs / d(d_k u)) contracted with s_k, from the implemented rhs,
    which is linear in the derivative inputs."""
    n = u.shape[0]
    H = np.zeros((4, 1))
    dH = np.zeros((4, 4, 1))
    base = ghg.rhs(u[:, None], np.zeros((3, n, 1)), H, dH)[:, 0]
    A = np.zeros((n, n))
    for k in range(3):
        for nu in range(n):
            du = np.zeros((3, n, 1))
            du[k, nu, 0] = 1.0
            A[:, nu] -= s_low[k] * (ghg.rhs(u[:, None], du, H, dH)[:, 0] - base)
    return A


def test_principal_symbol_is_the_printed_characteristic_matrix():
    """s_k A^k of the implemented rhs equals the matrix printed in App. A.2
    (eq. characteristics) for every symmetric pair, with no coupling between
    pairs, on a generic (non-Kerr-Schild) state."""
    x = _points(1, 4)
    u = _ks_state(x)[:, 0] + 0.03 * np.random.default_rng(4).standard_normal(50)
    s = np.array([0.3, -0.5, 0.8])
    A = _principal_symbol(u, s)
    g, Pi, Phi, _ = unpack(u[:, None])
    q = dependent(g, Pi, Phi)
    s_up = q['gam_inv'][..., 0] @ s
    alpha = q['alpha'][0]
    b = s @ q['beta_up'][:, 0]
    M = characteristic_matrix(s, s_up, alpha, b)
    expect = np.zeros((50, 50))
    for p in range(10):
        idx = [p, 10 + p, 20 + p, 30 + p, 40 + p]
        expect[np.ix_(idx, idx)] = M
    assert np.abs(A - expect).max() < 1e-12


@pytest.mark.parametrize("row", read_golden("ks_speeds.txt"))
def test_fastest_speed_on_kerr_schild(row):
    """The most negative characteristic speed at the inner boundary radius is
    -1.45 / -sqrt(2) / -1.53 at r = 1.8 / 2 / 1.5 (App. A.3)."""
    rad, speed, digits = float(row[0]), float(row[1]), int(row[2])
    x = np.array([[rad], [0.0], [0.0]])
    u = _ks_state(x)[:, 0]
    g, Pi, Phi, _ = unpack(u[:, None])
    q = dependent(g, Pi, Phi)
    s_low = np.array([1.0, 0, 0]) / np.sqrt(q['gam_inv'][0, 0, 0])
    A = _principal_symbol(u, s_low)
    ev = np.linalg.eigvals(A).real
    assert round(ev.min(), digits) == pytest.approx(speed, abs=0.5 * 10 ** -digits + 1e-12)


def test_boundary_operator_is_characteristic_projector():
    """B = E^-1 Z E (App. A.2, A.3): B^2 = B; after B the incoming
    characteristic combinations -g + Pi - s^k Phi_k and the tangential Phi
    vanish, while g and -g + Pi + s^k Phi_k are unchanged."""
    rng = np.random.default_rng(6)
    x = _points(5, 6, 11.8, 11.8)
    u = _ks_state(x) + 1e-2 * rng.standard_normal((50, 5))
    xhat = x / np.linalg.norm(x, axis=0)
    rhs = rng.standard_normal((50, 5))
    b1 = freeze_incoming(rhs, u, xhat)
    b2 = freeze_incoming(b1, u, xhat)
    assert np.abs(b2 - b1).max() < 1e-14
    s_low, s_up = ghg.boundary_normal(u, xhat)

    def chars(v):
        g_, P_, F_ = v[0:10], v[10:20], np.array([v[20 + 10 * i:30 + 10 * i] for i in range(3)])
        sF = np.einsum('k...,kp...->p...', s_up, F_)
        tang = F_ - s_low[:, None] * sF[None]
        return g_, -g_ + P_ + sF, -g_ + P_ - sF, tang
    c0, c1 = chars(rhs), chars(b1)
    assert np.allclose(c1[0], c0[0]) and np.allclose(c1[1], c0[1])
    assert np.abs(c1[2]).max() < 1e-14 and np.abs(c1[3]).max() < 1e-14
    assert np.allclose(np.einsum('i...,i...->...', s_low, s_up), 1.0)


def test_rk4_amplification_polynomial():
    """Classical RK4 (Sec. 2.5) multiplies y' = A y by
    1 + hA + (hA)^2/2 + (hA)^3/6 + (hA)^4/24 per step."""
    sh = Shell(3, 4, 8, 2.0, 3.0)
    ev = Evolution(sh, filter_kind='none')
    A = np.array([[-0.3, -1.1], [0.9, 0.2]])
    y = np.array([0.7, -0.4])
    h = 0.37
    got = ev.rk4_step(y, h, rhs_fn=lambda v: A @ v)
    hA = h * A
    P = np.eye(2) + hA + hA @ hA / 2 + hA @ hA @ hA / 6 + hA @ hA @ hA @ hA / 24
    assert np.abs(got - P @ y).max() < 1e-15


def test_constraints_vanish_initially():
    """With H_a = -Gamma_a (eq. gauge) the gauge constraint C_a = H_a + Gamma_a
    is zero at t = 0, and d_t g_ab = 0 (rhs of g vanishes) for the paper's
    data with numerical Phi."""
    sh = Shell(13, 8, 16, 1.8, 11.8)
    g10 = inputs.perturbed_kerr_schild(2, sh.r, sh.theta, sh.phi)
    u = initial_data.first_order_data(g10, sh)
    H, dH = initial_data.static_gauge(u, sh)
    g, Pi, Phi, _ = unpack(u)
    assert np.abs(H + dependent(g, Pi, Phi)['Gam_c']).max() < 1e-14
    r = Evolution(sh, 50, H, dH).rhs(u)
    assert np.abs(r[0:10]).max() < 1e-14


def test_radial_convergence_on_innermost_sphere():
    """Fig. r10_rconv behaviour: at 9 x 18 angular points the initial rhs on
    the innermost sphere decays exponentially with N_r (Sec. 4.1)."""
    errs = []
    for n_r in (13, 19, 25, 31):
        sh = Shell(n_r, 9, 18, 1.8, 11.8)
        g10 = inputs.perturbed_kerr_schild(2, sh.r, sh.theta, sh.phi, amp=0.0)
        u = initial_data.first_order_data(g10, sh)
        H, dH = initial_data.static_gauge(u, sh)
        errs.append(np.abs(Evolution(sh, 50, H, dH).rhs(u)[..., 0]).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 20), errs


def test_short_evolution_stays_near_static():
    """Three filtered RK4 steps of perturbed Kerr-Schild at lambda = 4 stay at
    the perturbation level (Sec. 4.1 default configuration)."""
    sh = Shell(13, 8, 16, 1.8, 11.8)
    g10 = inputs.perturbed_kerr_schild(2, sh.r, sh.theta, sh.phi)
    u0 = initial_data.first_order_data(g10, sh)
    H, dH = initial_data.static_gauge(u0, sh)
    ev = Evolution(sh, 50, H, dH)
    u = u0
    for _ in range(3):
        u = ev.rk4_step(u, courant_dt(sh))
    assert np.abs(u - u0).max() < 1e-2
    assert np.all(np.isfinite(u))


def test_constraint_fields_vanish_for_exact_kerr_schild():
    """C_a = H_a + Gamma_a and C_iab = d_i g_ab - Phi_iab (App. A.1) are zero
    for the Kerr-Schild state with closed-form Phi, H_a = -Gamma_a from the
    independent closed form, and d_i g from the complex step."""
    x = _points(12, 5)
    u = _ks_state(x)
    du = np.zeros((3,) + u.shape)
    du[:, 0:10] = _cstep(lambda xc: _ks_state(xc)[0:10], x)
    C_a, C_iab = ghg.constraints(u, du, _ks_gauge(x))
    assert np.abs(C_a).max() < 1e-14
    assert np.abs(C_iab).max() < 1e-14


def test_constraint_fields_report_planted_violations():
    """A planted change of Phi_iab shows up as -delta in C_iab, of H_a as
    +h in C_a; the 58-field state supplies H_a itself."""
    rng = np.random.default_rng(9)
    x = _points(10, 6)
    u = _ks_state(x)
    du = np.zeros((3,) + u.shape)
    du[:, 0:10] = _cstep(lambda xc: _ks_state(xc)[0:10], x)
    H = _ks_gauge(x)
    delta = 1e-3 * rng.standard_normal((30, x.shape[1]))
    h = 1e-3 * rng.standard_normal((4, x.shape[1]))
    up = u.copy()
    up[20:50] += delta
    C_a, C_iab = ghg.constraints(up, du, H + h)
    assert np.abs(C_iab + delta.reshape(3, 10, -1)).max() < 1e-14
    # the Phi change also moves Gamma_a; the H change enters one to one
    C_a0, _ = ghg.constraints(up, du, H)
    assert np.abs(C_a - C_a0 - h).max() < 1e-15
    u58 = np.concatenate([u, H + h, np.zeros_like(H)])
    du58 = np.concatenate([du, np.zeros((3, 8) + u.shape[1:])], axis=1)
    C58, _ = ghg.constraints(u58, du58)
    assert np.abs(C58 - h).max() < 1e-14


def test_constraint_norms_definition():
    C_a = np.zeros((4, 5))
    C_a[2, 3] = -2.0
    C_iab = np.ones((3, 10, 5))
    mx_a, rms_a, mx_i, rms_i = ghg.constraint_norms(C_a, C_iab)
    assert (mx_a, mx_i, rms_i) == (2.0, 1.0, 1.0)
    assert rms_a == pytest.approx(np.sqrt(4.0 / 20.0), rel=1e-15)


def _damping_case(seed=13):
    """Kerr-Schild at three points with |x| = 3 (so that n_a = (-alpha, 0) and
    n^a = (1/alpha, -beta^i/alpha) differ), exact complex-step derivatives,
    and a gauge source H = -Gamma + h with h a constant (in space and time)
    offset.  Returns the points, the oracle's rhs and the hand value of the
    Pi rows, built with sympy from the metric alone."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3, 3))
    x = 3.0 * v / np.linalg.norm(v, axis=0)
    h = rng.standard_normal((4, 3))
    u = _ks_state(x)
    du = _cstep(_ks_state, x)
    H = _ks_gauge(x) + h
    dH = np.concatenate([np.zeros_like(H)[None], _cstep(_ks_gauge, x)])   # d_a h = 0
    got = ghg.rhs(u, du, H, dH)
    # hand value from the printed terms of eq. Pidot.  On the static solution
    # with exact derivatives every term vanishes except the two that contain
    # the offset: the damping term alpha (2 delta^c_(a n_b) - g_ab n^c) C_c with
    # C_c = H_c + Gamma_c = h_c, and -2 alpha nabla_(a H_b), whose change is
    # +2 alpha g^cd Gamma_cab h_d (nabla_a H_b = d_a H_b - g^cd Gamma_cab H_d).
    X = sp.symbols('x y z', real=True)
    r = sp.sqrt(sum(c ** 2 for c in X))
    l = [1] + [c / r for c in X]
    eta = sp.diag(-1, 1, 1, 1)
    gs = sp.Matrix(4, 4, lambda a, b: eta[a, b] + 2 / r * l[a] * l[b])
    dgs = [[[sp.diff(gs[a, b], X[c]) for b in range(4)] for a in range(4)] for c in range(3)]
    expect = np.zeros((4, 4, 3))
    for p in range(3):
        sub = dict(zip(X, x[:, p]))
        g = np.array(gs.evalf(subs=sub), dtype=float)
        D = np.zeros((4, 4, 4))                       # D[c, a, b] = d_c g_ab, d_t g = 0
        for c in range(3):
            D[c + 1] = np.array([[float(dgs[c][a][b].evalf(subs=sub)) for b in range(4)] for a in range(4)])
        gi = np.linalg.inv(g)
        alpha = 1.0 / np.sqrt(-gi[0, 0])              # g^tt = -1/alpha^2
        n_low = np.array([-alpha, 0.0, 0.0, 0.0])
        n_up = gi @ n_low
        hp = h[:, p]
        for a in range(4):
            for b in range(4):
                Gam_ab = [0.5 * (D[a, b, c] + D[b, a, c] - D[c, a, b]) for c in range(4)]   # Gamma_cab
                damp = alpha * (hp[a] * n_low[b] + hp[b] * n_low[a] - g[a, b] * (n_up @ hp))
                nab = 2.0 * alpha * sum(gi[c, d] * Gam_ab[c] * hp[d] for c in range(4) for d in range(4))
                expect[a, b, p] = damp + nab
    return x, got, expect, h


def test_constraint_damping_term_against_hand_value():
    """Eq. Pidot's gauge-constraint damping alpha (2 delta^c_(a n_b) - g_ab n^c) C_c,
    pinned at C_a != 0 (every other pin has C_a = 0): the oracle's Pi rows equal
    the hand value, and the g and Phi rows stay zero (the offset enters eq. Pidot
    only)."""
    x, got, expect, h = _damping_case()
    g, Pi, Phi, _ = unpack(got)
    assert np.abs(expect).max() > 0.1
    assert np.abs(Pi - expect).max() < 1e-12, np.abs(Pi - expect).max()
    assert np.abs(g).max() < 1e-12 and np.abs(Phi).max() < 1e-12


@pytest.mark.parametrize("mistake", ["sign of C_a n_b", "dropped g_ab n^c C_c", "n^b for n_b"])
def test_constraint_damping_pin_catches_planted_mistakes(monkeypatch, mistake):
    """Planted mistakes in the damping term (a flipped sign of the
    delta^c_(a n_b) part, a dropped trace part, the contravariant normal in
    place of the covariant one) make the hand-value pin fail."""
    orig = ghg._es
    orig_dep = ghg.dependent

    def broken(spec, *ops):
        if mistake == "sign of C_a n_b" and spec == 'a...,b...->ab...':
            return -orig(spec, *ops)
        if mistake == "dropped g_ab n^c C_c" and spec == 'c...,c...->...':
            return 0 * orig(spec, *ops)
        return orig(spec, *ops)

    def dep_up_for_low(g, Pi, Phi):
        q = orig_dep(g, Pi, Phi)
        q = dict(q)
        q['n_low'] = q['n_up']
        return q
    monkeypatch.setattr(ghg, "_es", broken)
    if mistake == "n^b for n_b":
        monkeypatch.setattr(ghg, "dependent", dep_up_for_low)
    x, got, expect, h = _damping_case()
    Pi = unpack(got)[1]
    assert np.abs(Pi - expect).max() > 1e-3
