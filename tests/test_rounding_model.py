"""Pins of the oracle's reduced-precision products (oracle.rounding), used by
the mixed-precision parity tests (CPU only)."""
import numpy as np
import pytest
import torch

from oracle.rounding import bf16, split, product, RoundedEvolution
from oracle.grid import Shell, courant_dt, fourier_diff_matrix
from oracle import initial_data as oid
from paper_1104_3408_amd import inputs


def test_bf16_rounding_matches_torch():
    """Round to nearest even into bfloat16, checked against torch's own
    conversion on values that include exact ties."""
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    ties = (np.arange(1, 2000, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, -ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(bf16(x), ref)


def test_split_residual_within_two_bfloat16_units():
    """x - x_hi - x_lo is at most 2^-16 |x| (two levels of the bfloat16 unit
    roundoff 2^-8), and x_hi alone misses by up to 2^-8 |x|."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal(100000).astype(np.float32)
    hi, lo = split(x)
    r2 = np.abs(x.astype(np.float64) - hi - lo) / np.abs(x)
    r1 = np.abs(x.astype(np.float64) - hi) / np.abs(x)
    assert r2.max() <= 2.0 ** -16 and r1.max() <= 2.0 ** -8
    assert r1.max() > 2.0 ** -9 and r2.max() > 2.0 ** -18      # the units are attained


def test_product_errors_scale_with_the_units():
    """On a Fourier derivative of random columns the three modes err in the
    order of their units: plain bf16 (2^-8) far above bf16x3, whose split
    residuals (2^-16) stay above the FP32 accumulation and storage (2^-24)
    that both FP32-accumulating modes share."""
    rng = np.random.default_rng(2)
    W = fourier_diff_matrix(64)
    x = rng.standard_normal((64, 500))
    exact = W @ x
    err = {m: np.abs(product(W, x, m) - exact).max() for m in ("fp32", "bf16x3", "bf16")}
    assert err["bf16"] > 100 * err["bf16x3"], err
    assert err["bf16x3"] > 5 * err["fp32"], err


@pytest.mark.slow
def test_model_separates_the_modes_on_an_evolution():
    """Five filtered RK4 steps of perturbed Kerr-Schild (13 x 12 x 24): the
    model's state errors are ordered fp32 << bf16x3 << bf16, so a GPU result
    held to within a factor 3 of the bf16x3 prediction cannot be a plain
    bfloat16 or an FP32 computation."""
    sh = Shell(13, 12, 24, 1.8, 11.8)
    g10 = inputs.perturbed_kerr_schild(3, sh.r, sh.theta, sh.phi)
    u0 = oid.first_order_data(g10, sh)
    H, dH = oid.static_gauge(u0, sh)
    dt = courant_dt(sh)
    res = {}
    for mode in ("fp64", "fp32", "bf16x3", "bf16"):
        ev = RoundedEvolution(sh, 50, H, dH, "Yn", 4, mode=mode)
        u = u0
        for _ in range(5):
            u = ev.rk4_step(u, dt)
        res[mode] = u
    e = {m: np.abs(res[m] - res["fp64"]).max() for m in ("fp32", "bf16x3", "bf16")}
    assert e["bf16"] > 100 * e["bf16x3"] and e["bf16x3"] > 30 * e["fp32"], e
    assert e["fp32"] > 1e-10      # the model really rounds
