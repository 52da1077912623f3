"""The large 58-field form (8 shells of 65x64x128 on [1.8, 21.8], gauge source
H_a and its rate Q_a evolved with the state, Yn filter n_f = 4, Courant factor
4) over many steps, monitored by the constraint norms of App. A.1 (max and RMS
of C_a = H_a + Gamma_a and of C_iab = d_i g_ab - Phi_iab), in the launch
configuration bench.py times (one grid for the batch, captured step graphs).

* Against the oracle: the first shell's FP64 oracle evolution stored by
  tests/golden/make_oracle_evolutions.py (case large8_shell0, from the oracle
  alone: constraint norms after every step, the state on a seeded sample
  after the stored step counts).  FP64: the state and the C_a norms within the
  parity bar (1e-12 of the state's scale); C_iab = d_i g_ab - Phi_iab is a
  difference of FP64 spectral derivatives that is exactly zero at t = 0, so
  over these steps it is FP64 rounding, different on each side: both are held
  to a rounding rate of 2e-12 per step and the GPU's to at most twice the
  oracle's.  FP32 and
  BF16x3 angular forms: their distance from the oracle's state is printed
  and held below 50 units of their angular products (2^-24, 2^-16) per step.
* 1000 steps of the whole batch in FP64 and both mixed forms, norms of every
  shell every 10 steps, printed every 100.  Measured (max over shells):
  FP64 max |C_a| decays from the seeded gauge offset 1.2e-6 to 1.9e-7 (the
  damping terms of eq. Pidot), max |C_iab| levels off near 2.6e-10; FP32
  angular: C_a 5.6e-7, C_iab 1.7e-6; BF16x3 angular: C_a and C_iab near
  1.4e-4, each level reached within the first few hundred steps and then
  flat.  Asserted: every norm finite; FP64's C_a lower after 1000 steps than
  at t = 0 and its C_iab below 1e-9; no norm of any form more than doubles
  over the last 500 steps (no growing mode over this span; the paper expects
  eventual growth through the outer boundary at r_max ~ 22, Sec. 4.1, over
  far longer times); and each mixed form's C_iab, and its C_a distance from
  FP64's, below 100 units of its angular products times max |u| (FP32 2^-24,
  BF16x3 2^-16: the constraint violation a mode adds is its rounding carried
  into Phi and H; measured 14 and 5 units).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1104_3408_amd import shellspec as ss
from paper_1104_3408_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PRECS = {"fp64": ss.SG_PREC_FP64, "fp32": ss.SG_PREC_FP32, "bf16x3": ss.SG_PREC_BF16X3}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ss.lib()


def _batch(precision):
    """The 8-shell grid and its seeded initial state (bench.py's recipe)."""
    shells, n_v = inputs.workload_shells("large8")
    seed0 = inputs.WORKLOAD_SEED["large8"]
    g = ss.ShellGrid(shells, n_fields=n_v, filter="Yn", n_f=4, courant=4.0, precision=precision)
    g10, extra = [], []
    for k in range(len(shells)):
        r, th, ph = g.coords(k)
        g10.append(inputs.perturbed_kerr_schild(seed0 + k, r, th, ph).ravel())
        dH, Q = inputs.gauge_perturbation(seed0 + 1000 + k, r, th, ph)
        extra.append(np.concatenate([dH, Q]).ravel())
    u = torch.zeros(g.state_size, dtype=torch.float64, device="cuda")
    g.kerr_schild_data(torch.from_numpy(np.concatenate(g10)).cuda(), u,
                       extra8=torch.from_numpy(np.concatenate(extra)).cuda())
    return g, shells, u


def _norms(g, u, n_shells):
    out = torch.zeros(4 * n_shells, dtype=torch.float64, device="cuda")
    g.ghg_constraints(u, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(n_shells, 4)


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x3"])
def test_first_shell_against_stored_oracle(form):
    path = os.path.join(GOLDEN, "oracle_large8_shell0.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle evolution large8_shell0 not generated")
    ref = dict(np.load(path))
    cn = ref["constraint_norms"]                      # [step][max C_a, rms C_a, max C_iab, rms C_iab]
    g, shells, u = _batch(PRECS[form])
    off, cnt, dt = g.info(0)
    assert dt == pytest.approx(float(ref["dt"]), rel=1e-15)
    idx = torch.from_numpy(ref["idx"]).cuda()
    scale = float(ref["max_u0"])
    saves = set(int(n) for n in ref["steps"])
    unit = {"fp64": 0.0, "fp32": 2.0 ** -24, "bf16x3": 2.0 ** -16}[form]
    for n in range(0, cn.shape[0]):
        if n > 0:
            g.rk_step(u, 1)
        got = _norms(g, u, len(shells))[0]
        d = np.abs(got - cn[n])
        print("%s step %d: norms gpu %s oracle %s" % (form, n, got, cn[n]), flush=True)
        if form == "fp64":
            # C_a = H_a + Gamma_a from the state: the parity bar
            assert d[:2].max() <= TOL * scale, (n, got, cn[n])
            # C_iab = d_i g_ab - Phi_iab is zero at t = 0 and then grows from
            # FP64 rounding, each side in its own summation order: held to a
            # rounding rate of 2e-12 per step (measured: the oracle's max grows
            # by 1.4e-12 per step, the GPU's by half that) and the GPU's to at
            # most twice the oracle's
            assert got[2] <= 2.0 * cn[n][2] + TOL * scale and max(got[2], cn[n][2]) <= 2e-12 * n, (n, got, cn[n])
        if n in saves:
            v = u[off:off + cnt][idx].cpu().numpy()
            e = np.abs(v - ref["vals_%d" % n]).max() / ref["max_u_%d" % n]
            print("%s step %d: max rel state error vs oracle %.2e" % (form, n, e), flush=True)
            if form == "fp64":
                assert e <= TOL, (n, e)
            else:
                assert e <= 50 * unit * n, (n, e)     # within the mode's rounding unit per step
    g.close()


TRAJ = {}   # form -> (norms [sample][shell][4] every 10 steps, max |u| at the end)


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x3"])
def test_thousand_steps(form):
    """1000 steps of the batch in one form: finite norms, none growing over
    the last 500 steps; FP64's C_a damped and its C_iab below 1e-9."""
    g, shells, u = _batch(PRECS[form])
    rows = [_norms(g, u, len(shells))]
    for _ in range(100):
        g.rk_step(u, 10)
        rows.append(_norms(g, u, len(shells)))
    assert torch.isfinite(u).all(), form
    u_max = float(u.abs().max())
    g.close()
    del u
    torch.cuda.empty_cache()
    traj = np.array(rows)
    TRAJ[form] = (traj, u_max)
    assert np.isfinite(traj).all(), form
    t = traj.max(axis=1)                                # max over shells
    print("%s: max over shells every 100 steps, (max C_a, rms C_a, max C_iab, rms C_iab):" % form, flush=True)
    for k in range(0, t.shape[0], 10):
        print("  step %4d: %s" % (10 * k, " ".join("%.3e" % x for x in t[k])), flush=True)
    for c in (0, 2):
        assert t[-1, c] <= 2.0 * t[50, c], (form, c, t[50, c], t[-1, c])
    if form == "fp64":
        assert t[-1, 0] < t[0, 0] and t[:, 2].max() < 1e-9


def test_thousand_steps_mixed_against_fp64():
    if any(f not in TRAJ for f in PRECS):
        pytest.skip("needs the three 1000-step runs of this module")
    f64, _ = TRAJ["fp64"]
    for form in ("fp32", "bf16x3"):
        m, u_max = TRAJ[form]
        unit = {"fp32": 2.0 ** -24, "bf16x3": 2.0 ** -16}[form]
        d_ca = np.abs(m[..., 0] - f64[..., 0]).max()
        c_iab = m[..., 2].max()
        print("%s: max |C_a - C_a(FP64)| %.2e, max C_iab %.2e (FP64 %.2e): %.1f and %.1f units of max|u|" % (
            form, d_ca, c_iab, f64[..., 2].max(), d_ca / (unit * u_max), c_iab / (unit * u_max)), flush=True)
        assert d_ca <= 100 * unit * u_max, (form, d_ca)
        assert c_iab <= 100 * unit * u_max, (form, c_iab)
