"""Reduced-precision forms of the oracle's angular derivative products
(oracle; test infrastructure only).

The exact FP64 steps are the oracle's own; this module replaces only the two
angular derivative products of the right-hand side (Sec. 2.4 eqs. D2, D3) by
the same products carried out in the rounding each precision mode defines,
so that the error a mode must show is predicted on the CPU:

  fp32   operator and (mean-removed) input rounded to FP32, products
         accumulated in FP32, result stored in FP32;
  bf16x3 operator W and input x rounded to FP32 and split into two bfloat16
         parts, x = x_hi + x_lo (x_hi = bf16(x), x_lo = bf16(x - x_hi), round
         to nearest even), W x ~ W_hi x_hi + W_hi x_lo + W_lo x_hi accumulated
         in FP32 (each bfloat16 product is exact in FP32), stored in FP32;
  bf16   plain bfloat16 operands (x_hi, W_hi only), FP32 accumulation.

The theta product acts on the oracle's explicit 2 N_theta-point meridian
circle (Sec. 2.1), the phi product on the N_phi-point circle (Sec. 2.4), both
after subtracting the circle mean in FP64 (the Fourier rows annihilate
constants, Sec. 2.3).  The radial derivative, the rhs, the filter and the RK4
update stay the oracle's FP64 code.

The per-product error of each mode follows from its unit roundoff: FP32
operands carry 2^-24 each; for bf16x3 the dropped W_lo x_lo and the two split
residuals are each at most 2^-8 * 2^-8 of |W||x| (the bfloat16 unit roundoff
is 2^-8), and plain bfloat16 operands carry 2^-8 each.  Worst-case sums of
these over K terms and RK4 stages overestimate the observed error by two to
three orders of magnitude (random signs, typical rather than maximal
residuals), so the stated error of a mode is this model's prediction on the
same input, and the GPU is held to it within a factor (the model then tells
the modes apart: their predictions differ by factors of 100 and more).
"""
import numpy as np

from . import derivs as od
from .evolve import Evolution
from .grid import fourier_diff_matrix


def bf16(x):
    """bfloat16 value of FP32 input (round to nearest even), returned as FP32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32)


def split(x):
    xf = np.ascontiguousarray(x, dtype=np.float32)
    hi = bf16(xf)
    return hi, bf16(xf - hi)


def product(W, x, mode):
    """W (n x n, FP64) times x (n x cols, FP64) in the arithmetic of mode,
    returned as FP64."""
    if mode == "fp64":
        return W @ x
    if mode == "fp32":
        return (W.astype(np.float32) @ x.astype(np.float32)).astype(np.float64)
    if mode == "bf16x3":
        wh, wl = split(W)
        xh, xl = split(x)
        return (wh @ xh + wh @ xl + wl @ xh).astype(np.float64)
    if mode == "bf16":
        return (bf16(W) @ bf16(x)).astype(np.float64)
    raise ValueError(mode)


def d_theta(u, shell, mode):
    """Double-cover theta derivative (meridian circle, mean removed) with the
    product in the arithmetic of mode."""
    n = shell.n_theta
    FD = fourier_diff_matrix(2 * n)
    out = np.empty_like(u)
    for j in range(shell.n_phi):
        c = od.meridian_circle(u, j, shell)
        c = np.moveaxis(c - c.mean(axis=-2, keepdims=True), -2, 0)
        d = product(FD, c.reshape(2 * n, -1), mode).reshape(c.shape)
        out[..., j, :, :] = np.moveaxis(d, 0, -2)[..., :n, :]
    return out


def d_phi(u, shell, mode):
    FD = fourier_diff_matrix(shell.n_phi)
    v = np.moveaxis(u - u.mean(axis=-3, keepdims=True), -3, 0)
    d = product(FD, v.reshape(shell.n_phi, -1), mode).reshape(v.shape)
    return np.moveaxis(d, 0, -3)


class RoundedEvolution(Evolution):
    """The oracle's evolution with the angular products in reduced precision."""

    def __init__(self, *args, mode="fp64", **kw):
        super().__init__(*args, **kw)
        self.mode = mode

    def cart_derivs(self, u):
        sh = self.shell
        dr, dth, dph = od.d_r(u, sh), d_theta(u, sh, self.mode), d_phi(u, sh, self.mode)
        J = od.jacobian(sh)
        return np.array([J[i][0] * dr + J[i][1] * dth + J[i][2] * dph for i in range(3)])
