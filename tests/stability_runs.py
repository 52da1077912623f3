"""Long single-black-hole runs of the filtered evolution on the GPU (the
paper's Sec. 4.1 stability study, Figs. r10_f0, r10_f1, r10_f2, r10_long).

Unperturbed Kerr-Schild (M = 1) on r in [1.8, 11.8], Courant factor 4, the
chosen filter with n_f = 4 after every step.  Every `--every` time units the
library's right-hand side is evaluated and the paper's monitor quantities
are printed: max |rhs(g_tt)| over the shell, and the coefficients a_lm, b_lm
(l <= 2) of rhs(g_tt) on the innermost sphere in real, non-weighted
spherical harmonics (eq. realYexp), by least squares on the collocation
points.  The run stops when max |rhs(g_tt)| exceeds 1e-2 or is not finite.
Qualitative (no oracle): the paper reports no exponential growth to
t = 200,000 with the Yn filter, failure near t = 70,000 with Yg.

Usage: python tests/stability_runs.py N_r N_theta FILTER T_END [--every 500]
"""
import argparse
import math
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def real_harmonics(theta, phi, l_max=2):
    """Columns (name, values) of the real spherical harmonics up to l_max on
    the (theta, phi) grid (unnormalised Legendre form: a_lm cos(m phi),
    b_lm sin(m phi) times P_l^m(cos theta))."""
    from scipy.special import lpmv
    T, P = np.meshgrid(theta, phi, indexing="ij")
    cols = []
    for l in range(l_max + 1):
        for m in range(l + 1):
            p = lpmv(m, l, np.cos(T))
            cols.append(("a%d%d" % (l, m), (p * np.cos(m * P)).ravel()))
            if m > 0:
                cols.append(("b%d%d" % (l, m), (p * np.sin(m * P)).ravel()))
    return cols


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("n_r", type=int)
    ap.add_argument("n_theta", type=int)
    ap.add_argument("filter", choices=["Yn", "Yg", "Y"])
    ap.add_argument("t_end", type=float)
    ap.add_argument("--every", type=float, default=500.0)
    ap.add_argument("--n_f", type=int, default=4)
    a = ap.parse_args()
    import torch
    from paper_1104_3408_amd import shellspec as ss
    from paper_1104_3408_amd import inputs
    shape = (a.n_r, a.n_theta, 2 * a.n_theta)
    g = ss.ShellGrid([shape + (1.8, 11.8)], filter=a.filter, n_f=a.n_f, courant=4.0)
    r, th, ph = g.coords(0)
    g10 = inputs.perturbed_kerr_schild(2, r, th, ph, amp=0.0)
    u = torch.zeros(g.state_size, dtype=torch.float64, device="cuda")
    g.kerr_schild_data(torch.from_numpy(g10.ravel()).cuda(), u)
    dt = g.info(0)[2]
    npts = int(np.prod(shape))
    names, cols = zip(*real_harmonics(th, ph))
    A = np.array(cols).T                       # (N_theta N_phi) x modes, layout [phi][theta] transposed below
    rt = torch.zeros_like(u)
    every = max(1, int(round(a.every / dt)))
    t, t0 = 0.0, time.perf_counter()
    print("# %dx%dx%d %s n_f=%d dt=%.5f, sample every %d steps; columns: t max|rhs(g_tt)| %s"
          % (shape + (a.filter, a.n_f, dt, every, " ".join(names))), flush=True)
    while True:
        g.ghg_rhs(u, rt)
        gtt = rt[:npts].view(shape[2], shape[1], shape[0])       # [phi][theta][r]
        mx = float(gtt.abs().max())
        inner = gtt[:, :, 0].cpu().numpy().T.ravel()             # [theta][phi] at r_min
        coef = np.linalg.lstsq(A, inner, rcond=None)[0]
        print("%.1f %.4e %s   (%.0f s)" % (t, mx, " ".join("%.3e" % c for c in coef), time.perf_counter() - t0),
              flush=True)
        if not math.isfinite(mx) or mx > 1e-2 or t >= a.t_end:
            break
        g.rk_step(u, every)
        t += every * dt


if __name__ == "__main__":
    main()
