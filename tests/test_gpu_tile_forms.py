"""GPU parity of the alternative tile forms the tuning table can select, each
forced through a temporary table (SG_TUNING_FILE) and compared with the
oracle (FP64 bar 1e-12) and with the default form:

* d_theta on whole meridian plane pairs (th_plane 1) against the 64-column
  tile: the same arithmetic in the same order, so the derivatives and whole
  filtered steps agree bit for bit, in the one-launch form of the three
  derivative contractions and in the separate launches of the timing mode;
  shapes with odd N_theta, N_r above one 64-lane chunk and the 58-field form;
* d_phi in the parity form (dph_par 1) in FP64 against the oracle;
* the FP64 circulant d_phi on the matrix cores (dph_mfma 1; N_phi = 16 ...
  128, ragged column tiles) against the oracle, and whole filtered steps with
  it (captured and eager) equal to each other bit for bit.
"""
import os
import tempfile

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1104_3408_amd import shellspec as ss
from paper_1104_3408_amd import inputs
from oracle.grid import Shell
from oracle import derivs as od

pytestmark = pytest.mark.gpu
TOL = 1e-12
# dr_rows th_rows dph_rows ana_rows syn_rows filt_waves: the library defaults
DEFAULT_ROWS = "9 4 8 8 8 8"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ss.lib()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _grid(shells, n_v, dph_par=-1, th_plane=0, rows=DEFAULT_ROWS, fuse=1, dph_mfma=0, **kw):
    """A grid whose shells take the given forms (one table line per size)."""
    fd, path = tempfile.mkstemp(suffix=".txt", prefix="sg_forms_")
    prec = kw.get("precision", ss.SG_PREC_FP64)
    with os.fdopen(fd, "w") as f:
        for (n_r, n_th) in sorted({(s[0], s[1]) for s in shells}):
            f.write("%d %d %d %d %s %d %d %d %d\n" % (n_r, n_th, n_v, prec, rows, dph_par, th_plane, fuse, dph_mfma))
    old = os.environ.get("SG_TUNING_FILE")
    os.environ["SG_TUNING_FILE"] = path
    try:
        return ss.ShellGrid(shells, n_fields=n_v, **kw)
    finally:
        if old is None:
            del os.environ["SG_TUNING_FILE"]
        else:
            os.environ["SG_TUNING_FILE"] = old
        os.unlink(path)


def _derivs(g, u, timing):
    du = torch.zeros(3 * u.numel(), dtype=torch.float64, device="cuda")
    g.enable_timing(timing)
    g.spec_derivs(u, du, ss.SG_COORD)
    g.enable_timing(False)
    torch.cuda.synchronize()
    return du


# (N_r, N_theta, fields, rows): odd N_theta, N_r > 64, the 58-field form, a
# shape whose row targets keep the three derivative workgroups apart (separate
# launches even outside the timing mode)
PLANE_CASES = [(13, 10, 50, DEFAULT_ROWS), (37, 7, 50, DEFAULT_ROWS), (77, 9, 50, DEFAULT_ROWS),
               (33, 32, 50, "9 3 8 8 8 8"), (49, 48, 50, "8 3 13 6 8 8"), (25, 24, 58, DEFAULT_ROWS),
               (17, 16, 50, "3 3 4 3 3 8")]


@pytest.mark.parametrize("n_r,n_th,n_v,rows", PLANE_CASES)
def test_theta_plane_tile(n_r, n_th, n_v, rows):
    desc = (n_r, n_th, 2 * n_th, 1.8, 11.8)
    sh = Shell(*desc)
    u = np.random.default_rng(n_r + n_th).standard_normal((n_v,) + sh.shape)
    ut = dev(u)
    gc = _grid([desc], n_v, rows=rows)
    gp = _grid([desc], n_v, th_plane=1, rows=rows)
    ref = od.coordinate_derivs(u, sh)
    for timing in (False, True):
        dc = _derivs(gc, ut, timing)
        dp = _derivs(gp, ut, timing)
        assert torch.equal(dc, dp), timing
        got = dp.cpu().numpy().reshape((3,) + u.shape)
        for d in range(3):
            assert rel(got[d], ref[d]) < TOL, (timing, d, rel(got[d], ref[d]))
    gc.close()
    gp.close()


@pytest.mark.parametrize("prec", [ss.SG_PREC_FP64, ss.SG_PREC_FP32])
@pytest.mark.parametrize("shells", [[(33, 32, 64, 1.8, 11.8)],
                                    [(17, 16, 32, 1.8, 11.8), (13, 9, 18, 2.0, 9.0), (17, 16, 32, 1.8, 11.8)]])
def test_step_forms(shells, prec):
    """Filtered RK4 steps (captured and eager) are the same bit for bit with
    the plane or the column d_theta tile and with the three derivative
    contractions of a stage in one launch or in three on forked streams."""
    out = []
    for th_plane, fuse in ((0, 1), (1, 1), (0, 0), (1, 0)):
        g = _grid(shells, 50, th_plane=th_plane, fuse=fuse, precision=prec)
        u = torch.zeros(g.state_size, dtype=torch.float64, device="cuda")
        parts = []
        for s in range(len(shells)):
            r, th, ph = g.coords(s)
            parts.append(inputs.perturbed_kerr_schild(11 + s, r, th, ph).ravel())
        g.kerr_schild_data(dev(np.concatenate(parts)), u)
        ua, ub = u.clone(), u.clone()
        g.rk_step(ua, 3)
        g.enable_timing(True)
        g.rk_step(ub, 3)
        g.enable_timing(False)
        torch.cuda.synchronize()
        assert torch.isfinite(ua).all() and torch.equal(ua, ub)
        out.append(ua)
        g.close()
    for k in range(1, len(out)):
        assert torch.equal(out[0], out[k]), k


@pytest.mark.parametrize("n_r,n_th", [(13, 10), (37, 7), (33, 32)])
def test_phi_parity_form_fp64(n_r, n_th):
    desc = (n_r, n_th, 2 * n_th, 1.8, 11.8)
    sh = Shell(*desc)
    u = np.random.default_rng(3 * n_r).standard_normal((50,) + sh.shape)
    g = _grid([desc], 50, dph_par=1)
    ref = od.coordinate_derivs(u, sh)
    for timing in (False, True):
        got = _derivs(g, dev(u), timing).cpu().numpy().reshape((3,) + u.shape)
        for d in range(3):
            assert rel(got[d], ref[d]) < TOL, (timing, d, rel(got[d], ref[d]))
    g.close()


@pytest.mark.parametrize("n_r,n_th", [(13, 8), (37, 24), (33, 32), (49, 48), (21, 64)])
def test_phi_matrix_cores_fp64(n_r, n_th):
    desc = (n_r, n_th, 2 * n_th, 1.8, 11.8)
    sh = Shell(*desc)
    u = np.random.default_rng(5 * n_r + n_th).standard_normal((50,) + sh.shape)
    g = _grid([desc], 50, dph_par=0, dph_mfma=1, fuse=0)
    ref = od.coordinate_derivs(u, sh)
    for timing in (False, True):
        got = _derivs(g, dev(u), timing).cpu().numpy().reshape((3,) + u.shape)
        for d in range(3):
            assert rel(got[d], ref[d]) < TOL, (timing, d, rel(got[d], ref[d]))
    g.close()


def test_steps_with_phi_on_matrix_cores():
    shells = [(33, 32, 64, 1.8, 11.8), (17, 16, 32, 1.8, 11.8)]
    g = _grid(shells, 50, dph_par=0, dph_mfma=1, fuse=1)   # the one-launch form steps aside for it
    u = torch.zeros(g.state_size, dtype=torch.float64, device="cuda")
    parts = []
    for s in range(len(shells)):
        r, th, ph = g.coords(s)
        parts.append(inputs.perturbed_kerr_schild(21 + s, r, th, ph).ravel())
    g.kerr_schild_data(dev(np.concatenate(parts)), u)
    ua, ub = u.clone(), u.clone()
    g.rk_step(ua, 3)
    g.enable_timing(True)
    g.rk_step(ub, 3)
    g.enable_timing(False)
    torch.cuda.synchronize()
    assert torch.isfinite(ua).all() and torch.equal(ua, ub)
    g.close()
