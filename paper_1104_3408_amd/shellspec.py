"""ctypes binding of libshellspec (include/shellspec.h).

Argument marshalling only: every computation runs in the HIP library.  Device
arrays are passed as torch CUDA tensors (float64, contiguous) or raw integer
device addresses; streams as torch streams, raw handles, or None for the
current torch stream.  The library is loaded from this package directory and
a missing or unbuildable library raises at import of the first call.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshellspec.so")

SG_OK, SG_EINVAL, SG_ESHAPE, SG_ENOMEM, SG_EHIP, SG_ENONFINITE, SG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
SG_FILTER_YN, SG_FILTER_Y, SG_FILTER_YG, SG_FILTER_NONE = 0, 1, 2, 3
SG_PREC_FP64, SG_PREC_FP32, SG_PREC_BF16X3 = 0, 1, 2
SG_COORD, SG_CART = 0, 1
SG_CHECK_FINITE = 1
SG_NO_GRAPH = 2
SG_NESTED = 4

KERNEL_CLASSES = ["d_r", "d_theta", "d_phi", "rhs_stage", "filter_decompose", "filter_phi_analysis",
                  "filter_theta", "filter_phi_synthesis", "filter_recompose"]

FILTERS = {"Yn": SG_FILTER_YN, "Y": SG_FILTER_Y, "Yg": SG_FILTER_YG, "none": SG_FILTER_NONE}


class ShellDesc(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int), ("n_theta", ctypes.c_int), ("n_phi", ctypes.c_int),
                ("r_min", ctypes.c_double), ("r_max", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("n_fields", ctypes.c_int), ("filter_kind", ctypes.c_int), ("n_f", ctypes.c_int),
                ("precision", ctypes.c_int), ("courant", ctypes.c_double), ("mass", ctypes.c_double),
                ("flags", ctypes.c_uint)]


class ShellSpecError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("shellspec status %d: %s" % (status, msg))
        self.status = status


_lib = None

_P = ctypes.c_void_p
_SIGS = {
    "shell_grid_create": (ctypes.c_int, [ctypes.POINTER(ShellDesc), ctypes.c_int, ctypes.POINTER(Options), _P,
                                         ctypes.POINTER(_P)]),
    "shell_grid_destroy": (None, [_P]),
    "shell_grid_info": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_double)]),
    "shell_grid_coords": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P]),
    "sg_set_gauge": (ctypes.c_int, [_P, _P, _P]),
    "spec_derivs": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P]),
    "swsh_filter": (ctypes.c_int, [_P, _P, _P]),
    "ghg_rhs": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "ghg_constraints": (ctypes.c_int, [_P, _P, _P, _P]),
    "ghg_constraints_static": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "rk_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P]),
    "sg_kerr_schild_data": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "sg_enable_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "sg_kernel_times": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "sg_last_error": (ctypes.c_char_p, []),
    "sg_host_filter_matrix": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P]),
    "sg_host_cheb_matrix": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, _P]),
    "sg_host_theta_matrix": (ctypes.c_int, [ctypes.c_int, _P]),
}

EXPORTED = sorted(_SIGS)


def lib():
    """Load libshellspec.so from the package directory (raises if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libshellspec.so is not built: run python -m paper_1104_3408_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != SG_OK:
        raise ShellSpecError(status, lib().sg_last_error().decode())


def _ptr(x, n=None):
    """Device pointer of a contiguous float64 CUDA tensor holding at least n
    values (raw integer addresses pass through unchecked)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    import torch
    if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    if n is not None and x.numel() < n:
        raise ValueError("tensor holds %d values, the call needs %d" % (x.numel(), n))
    return x.data_ptr()


def _stream(s):
    if isinstance(s, int):
        return s
    import torch
    if s is None:
        s = torch.cuda.current_stream()
    return s.cuda_stream


def host_filter_matrix(n, m, n_theta, n_f):
    import numpy as np
    out = np.zeros((n_theta, n_theta))
    _check(lib().sg_host_filter_matrix(n, m, n_theta, n_f, out.ctypes.data))
    return out


def host_cheb_matrix(n_r, r_min, r_max):
    import numpy as np
    out = np.zeros((n_r, n_r))
    _check(lib().sg_host_cheb_matrix(n_r, r_min, r_max, out.ctypes.data))
    return out


def host_theta_matrix(n_theta):
    import numpy as np
    out = np.zeros((n_theta, 2 * n_theta))
    _check(lib().sg_host_theta_matrix(n_theta, out.ctypes.data))
    return out


class ShellGrid:
    """Owner of one sg_grid.  Methods map one-to-one onto the C-ABI."""

    def __init__(self, shells, n_fields=50, filter="Yn", n_f=4, courant=4.0, mass=1.0,
                 precision=SG_PREC_FP64, flags=0, gauge_H=None):
        descs = (ShellDesc * len(shells))(*[ShellDesc(int(a), int(b), int(c), float(d), float(e))
                                            for (a, b, c, d, e) in shells])
        opt = Options(n_fields, FILTERS[filter] if isinstance(filter, str) else int(filter), n_f, precision,
                      courant, mass, flags)
        h = _P()
        _check(lib().shell_grid_create(descs, len(shells), ctypes.byref(opt), _ptr(gauge_H), ctypes.byref(h)))
        self.h = h
        self.shells = [tuple(s) for s in shells]
        self.n_fields = n_fields
        self.n_points = sum(int(a) * int(b) * int(c) for (a, b, c, _, _) in self.shells)

    def close(self):
        if getattr(self, "h", None):
            lib().shell_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self, shell=-1):
        off, cnt, dt = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_double()
        _check(lib().shell_grid_info(self.h, shell, ctypes.byref(off), ctypes.byref(cnt), ctypes.byref(dt)))
        return off.value, cnt.value, dt.value

    def coords(self, shell):
        import numpy as np
        n_r, n_th, n_ph = self.shells[shell][:3]
        r, th, ph = np.zeros(n_r), np.zeros(n_th), np.zeros(n_ph)
        _check(lib().shell_grid_coords(self.h, shell, r.ctypes.data, th.ctypes.data, ph.ctypes.data))
        return r, th, ph

    @property
    def state_size(self):
        return self.info(-1)[1]

    def set_gauge(self, H, stream=None):
        _check(lib().sg_set_gauge(self.h, _ptr(H, 4 * self.n_points), _stream(stream)))

    def spec_derivs(self, u, du, mode=SG_COORD, stream=None):
        n = self.state_size
        _check(lib().spec_derivs(self.h, _ptr(u, n), _ptr(du, 3 * n), mode, _stream(stream)))

    def swsh_filter(self, u, stream=None):
        _check(lib().swsh_filter(self.h, _ptr(u, self.state_size), _stream(stream)))

    def ghg_rhs(self, u, rhs, du_cart=None, stream=None):
        n = self.state_size
        _check(lib().ghg_rhs(self.h, _ptr(u, n), _ptr(du_cart, 3 * n), _ptr(rhs, n), _stream(stream)))

    def ghg_constraints(self, u, norms, stream=None):
        """norms: device float64 tensor of 4 * n_shells, per shell
        (max |C_a|, rms C_a, max |C_iab|, rms C_iab)."""
        _check(lib().ghg_constraints(self.h, _ptr(u, self.state_size), _ptr(norms, 4 * len(self.shells)),
                                     _stream(stream)))

    def ghg_constraints_static(self, u, du_cart, norms, stream=None):
        """ghg_constraints from caller-given Cartesian derivatives (spec_derivs
        SG_CART layout), with no allocation in the library."""
        n = self.state_size
        _check(lib().ghg_constraints_static(self.h, _ptr(u, n), _ptr(du_cart, 3 * n),
                                            _ptr(norms, 4 * len(self.shells)), _stream(stream)))

    def rk_step(self, u, n_steps=1, dt=None, stream=None):
        arr = None
        if dt is not None:
            if len(dt) != len(self.shells):
                raise ValueError("dt needs one time step per shell")
            arr = (ctypes.c_double * len(dt))(*[float(x) for x in dt])
        _check(lib().rk_step(self.h, _ptr(u, self.state_size), arr, int(n_steps), _stream(stream)))

    def kerr_schild_data(self, g10, u, extra8=None, H_out=None, stream=None):
        n = self.n_points
        _check(lib().sg_kerr_schild_data(self.h, _ptr(g10, 10 * n), _ptr(extra8, 8 * n), _ptr(u, self.state_size),
                                         _ptr(H_out, 4 * n), _stream(stream)))

    def enable_timing(self, on=True):
        _check(lib().sg_enable_timing(self.h, 1 if on else 0))

    def kernel_times(self):
        """(ms, counts) per kernel class, in the order of KERNEL_CLASSES."""
        n = len(KERNEL_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int * n)()
        _check(lib().sg_kernel_times(self.h, ms, cnt, n))
        return list(ms), list(cnt)
