"""Library checks that need no GPU: the shared object loads and exports every
function the C header declares, argument validation, and the host-built
operator matrices against the oracle's independent constructions."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1104_3408_amd import shellspec as ss
from oracle.grid import cheb_diff_matrix, fourier_diff_matrix
from oracle.swsh import filter_matrix

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shellspec.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)
    skip = {"if", "sizeof", "defined"}
    return sorted({n for n in names if n not in skip and (n.startswith(("sg_", "shell_", "ghg_"))
                                                          or n in ("spec_derivs", "swsh_filter", "rk_step"))})


def test_library_exports_every_declared_symbol():
    assert os.path.exists(ss.LIB_PATH), "build the library first (python -m paper_1104_3408_amd.build)"
    out = subprocess.run(["nm", "-D", "--defined-only", ss.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(\S+)", out))
    declared = _declared()
    assert len(declared) >= 18 and "ghg_constraints_static" in declared
    missing = [n for n in declared if n not in exported]
    assert not missing, missing
    assert set(ss.EXPORTED) == set(declared)
    ss.lib()                       # loads through ctypes


def test_shape_validation_is_host_side():
    with pytest.raises(ss.ShellSpecError) as e:
        ss.ShellGrid([(12, 12, 20, 2.0, 12.0)])       # N_phi != 2 N_theta
    assert e.value.status == ss.SG_ESHAPE
    with pytest.raises(ss.ShellSpecError) as e:
        ss.ShellGrid([(12, 12, 24, 2.0, 12.0)], n_fields=52)
    assert e.value.status == ss.SG_EINVAL
    with pytest.raises(ss.ShellSpecError) as e:
        ss.ShellGrid([(12, 12, 24, 12.0, 2.0)])
    assert e.value.status == ss.SG_EINVAL
    with pytest.raises(ss.ShellSpecError) as e:
        ss.ShellGrid([(81, 12, 24, 2.0, 12.0)])
    assert e.value.status == ss.SG_ESHAPE
    with pytest.raises(ss.ShellSpecError) as e:
        ss.ShellGrid([(12, 12, 24, 2.0, 12.0)], precision=ss.SG_PREC_BF16X3 + 7)
    assert e.value.status == ss.SG_EUNSUPPORTED


@pytest.mark.parametrize("N,n_f", [(9, 0), (12, 1), (32, 4), (48, 4), (64, 4)])
def test_host_filter_matrices_match_oracle(N, n_f):
    """The library's F^n_m (Legendre + spin recursion, Householder QR) equals
    the oracle's (Wigner d by rotation operator, SVD pseudo-inverse)."""
    worst = 0.0
    ms = range(0, N) if N <= 32 else (0, 1, 2, 3, 7, N // 2, N - 6, N - 5, N - 1)
    for n in range(-3, 4):
        for m in ms:
            a = ss.host_filter_matrix(n, m, N, n_f)
            b = filter_matrix(n, m, N, n_f)
            worst = max(worst, np.abs(a - b).max())
    assert worst < 1e-12, worst


@pytest.mark.parametrize("n", [4, 12, 33, 65, 80])
def test_host_chebyshev_matches_oracle(n):
    a = ss.host_cheb_matrix(n, 1.8, 11.8)
    b = cheb_diff_matrix(n, 1.8, 11.8)
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("n", [5, 12, 32, 48])
def test_host_theta_matrix_is_double_cover(n):
    """The folded N x 2N matrix equals the Fourier matrix on the explicit
    2N-point circle with the lower half read from phi + pi in reverse
    (Sec. 2.1)."""
    H = ss.host_theta_matrix(n)
    FD = fourier_diff_matrix(2 * n)
    expect = np.concatenate([FD[:n, :n], FD[:n, n:][:, ::-1]], axis=1)
    assert np.abs(H - expect).max() < 1e-13 * np.abs(FD).max()


def test_binding_rejects_wrong_sizes_before_any_call():
    """The binding checks tensor kinds and sizes on the host (CPU tensors are
    refused before the library is reached; no GPU is needed)."""
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        ss._ptr(torch.zeros(4, dtype=torch.float64))          # not a CUDA tensor
    with pytest.raises(TypeError):
        ss._ptr(torch.zeros(4, dtype=torch.float32))
    assert ss._ptr(None) is None and ss._ptr(1234) == 1234
