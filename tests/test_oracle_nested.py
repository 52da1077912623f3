"""Pins of the nested-shell interface coupling of the oracle (oracle.nested,
reading of the paper's outlook Sec. 1 / Sec. 5 with the characteristic
fields of App. A.2): the patch is a change of basis into characteristic
fields and back (equal inputs pass unchanged), it takes every field from its
upwind side, and a shell split in two at a shared sphere converges to the
single shell's evolution with resolution (a patch that ignores the upwind
direction does not), and a static black hole split in two stays static to
truncation error."""
import numpy as np
import pytest

from oracle import nested
from oracle.grid import Shell, courant_dt
from oracle import initial_data as oid
from oracle.ghg import boundary_normal, unpack, dependent
from paper_1104_3408_amd import inputs


def _point_state(seed, r=(6.8, 4.0, 9.0), n=40):
    """Perturbed Kerr-Schild states at n points on spheres of radius r (each
    point's metric from the closed form, with O(1e-2) noise in Pi and Phi)."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.1, np.pi - 0.1, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    rr = np.array(r)[rng.integers(0, len(r), n)]
    x, y, z = rr * np.sin(th) * np.cos(ph), rr * np.sin(th) * np.sin(ph), rr * np.cos(th)
    g10 = inputs.kerr_schild_metric(x, y, z)
    u = np.zeros((50, n))
    u[0:10] = g10
    u[10:50] = 1e-2 * rng.standard_normal((40, n))
    xhat = np.array([x, y, z]) / rr
    return u, xhat


def _chars(r, u, xhat):
    s_low, s_up = boundary_normal(u, xhat)
    dg, dPi = r[0:10], r[10:20]
    dPhi = np.array([r[20 + 10 * i:30 + 10 * i] for i in range(3)])
    sdPhi = np.einsum('k...,kp...->p...', s_up, dPhi)
    tang = dPhi - s_low[:, None] * sdPhi[None]
    return dg, -dg + dPi + sdPhi, -dg + dPi - sdPhi, tang


def test_patch_of_equal_inputs_is_identity():
    u, xhat = _point_state(1)
    r = np.random.default_rng(2).standard_normal(u.shape)
    out = nested.patch_interface(r, r.copy(), u, xhat)
    assert np.abs(out - r).max() < 1e-13 * np.abs(r).max()


def test_patch_takes_each_characteristic_field_from_its_upwind_side():
    """Speeds alpha - b > 0 (u^1+ from A, the inside), -alpha - b < 0 and
    -b < 0 (u^1- and u^2 from B) at these radii; u^0 (speed 0) is the mean."""
    u, xhat = _point_state(3)
    rng = np.random.default_rng(4)
    rA, rB = rng.standard_normal(u.shape), rng.standard_normal(u.shape)
    out = nested.patch_interface(rA, rB, u, xhat)
    g, Pi, Phi, _ = unpack(u)
    d = dependent(g, Pi, Phi)
    s_low, _ = boundary_normal(u, xhat)
    b = np.einsum('i...,i...->...', s_low, d['beta_up'])
    assert np.all(d['alpha'] - b > 0) and np.all(b > 0)
    co, ca, cb = _chars(out, u, xhat), _chars(rA, u, xhat), _chars(rB, u, xhat)
    tol = 1e-12
    assert np.abs(co[0] - 0.5 * (ca[0] + cb[0])).max() < tol
    assert np.abs(co[1] - ca[1]).max() < tol
    assert np.abs(co[2] - cb[2]).max() < tol
    assert np.abs(co[3] - cb[3]).max() < tol


def test_patch_follows_the_sign_of_the_speed():
    """Inside the horizon (r = 1.85 < 2M) the shift exceeds the lapse, alpha - b < 0:
    u^1+ then travels inward and is taken from B as well."""
    u, xhat = _point_state(5, r=(1.85,))
    rng = np.random.default_rng(6)
    rA, rB = rng.standard_normal(u.shape), rng.standard_normal(u.shape)
    g, Pi, Phi, _ = unpack(u)
    d = dependent(g, Pi, Phi)
    s_low, _ = boundary_normal(u, xhat)
    b = np.einsum('i...,i...->...', s_low, d['beta_up'])
    assert np.all(d['alpha'] - b < 0)
    out = nested.patch_interface(rA, rB, u, xhat)
    assert np.abs(_chars(out, u, xhat)[1] - _chars(rB, u, xhat)[1]).max() < 1e-12


def _evolve_split(n, T, patch=None, amp=1e-3, drift=False):
    """Perturbed Kerr-Schild on [1.8, 11.8]: two shells [1.8, 6.8] + [6.8, 11.8]
    with n radial points each, and one shell with 2n - 1 (whose middle point
    is r = 6.8); both to time T with the same steps.  Returns the state on
    the sphere r = 6.8 of each (drift: the largest change of the state since
    t = 0 on the single shell and on the split pair instead)."""
    n_th, n_ph = 6, 12
    outer = Shell(2 * n - 1, n_th, n_ph, 1.8, 11.8)
    parts = [Shell(n, n_th, n_ph, 1.8, 6.8), Shell(n, n_th, n_ph, 6.8, 11.8)]
    dt = min(courant_dt(outer), *(courant_dt(s) for s in parts))
    steps = int(np.ceil(T / dt))
    dt = T / steps

    def init(sh):
        g10 = inputs.perturbed_kerr_schild(7, sh.r, sh.theta, sh.phi, amp=amp)
        u = oid.first_order_data(g10, sh)
        return (u,) + oid.static_gauge(u, sh)

    from oracle.evolve import Evolution
    u1, H1, dH1 = init(outer)
    ev1 = Evolution(outer, 50, H1, dH1, "Yn", 2)
    ps = [init(s) for s in parts]
    nev = nested.NestedEvolution(parts, 50, [p[1] for p in ps], [p[2] for p in ps], "Yn", 2)
    us = [p[0] for p in ps]
    u10, us0 = u1.copy(), [u.copy() for u in us]
    if patch is not None:
        nested.patch_interface, saved = patch, nested.patch_interface
    try:
        for _ in range(steps):
            u1 = ev1.rk4_step(u1, dt)
            us = nev.rk4_step(us, dt)
    finally:
        if patch is not None:
            nested.patch_interface = saved
    if drift:
        return np.abs(u1 - u10).max(), max(np.abs(u - u0).max() for u, u0 in zip(us, us0))
    return u1[..., n - 1], us[0][..., -1], us[1][..., 0], us[0][..., 0] - u1[..., 0]


@pytest.mark.slow
def test_two_shells_converge_to_one_shell():
    """The split evolution and the single shell approach the same solution:
    their difference on the shared sphere falls with the radial resolution
    (the perturbation, amplitude 1e-3 centred at r = 6, crosses the sphere)."""
    diffs = []
    for n in (7, 11, 15):
        single, a, b, _ = _evolve_split(n, 1.0)
        diffs.append(np.abs(a - single).max() / 1e-3)
        # the two copies of the sphere differ by what their initial Phi (each
        # shell's own spectral derivative) did: truncation error as well
        assert np.abs(a - b).max() <= 2 * np.abs(a - single).max()
    # measured 2.5, 0.066, 0.0028 of the perturbation
    assert diffs[1] < 0.1 * diffs[0] and diffs[2] < 0.1 * diffs[1], diffs


@pytest.mark.slow
@pytest.mark.parametrize("mistake", ["from_inside", "downwind"])
def test_convergence_pin_catches_a_wrong_patch(mistake):
    """Taking every field from the inside shell (no upwinding), or every
    field from its downwind side (A and B exchanged), breaks the agreement:
    measured 0.11 and 0.29 against 6.6e-5 at n = 11."""
    correct = nested.patch_interface

    def wrong(rA, rB, u_pt, xhat):
        return rA.copy() if mistake == "from_inside" else correct(rB, rA, u_pt, xhat)
    single, a, _, _ = _evolve_split(11, 1.0, patch=wrong)
    good_single, good_a, _, _ = _evolve_split(11, 1.0)
    assert np.abs(a - single).max() > 100 * np.abs(good_a - good_single).max()


@pytest.mark.slow
def test_static_black_hole_stays_static_across_the_interface():
    """Unperturbed Kerr-Schild is a static solution: split at r = 6.8 it
    drifts only by truncation error, which falls exponentially with the
    radial points (measured 3.2e-2 at 7, 1.5e-3 at 11 points per shell by
    t = 1; the single shell with 13 and 21 points: 5.0e-3, 2.5e-5, its
    points clustering twice as densely at the horizon), while a patch that
    takes every field from the inside shell or from its downwind side drives
    the interface (9.2e-2 and 0.24 at 11 points)."""
    single7, split7 = _evolve_split(7, 1.0, amp=0.0, drift=True)
    single11, split11 = _evolve_split(11, 1.0, amp=0.0, drift=True)
    assert split11 < 0.1 * split7 and single11 < 0.1 * single7
    correct = nested.patch_interface
    for wrong in (lambda rA, rB, u_pt, xhat: rA.copy(), lambda rA, rB, u_pt, xhat: correct(rB, rA, u_pt, xhat)):
        _, bad = _evolve_split(11, 1.0, patch=wrong, amp=0.0, drift=True)
        assert bad > 30 * split11, (bad, split11)
