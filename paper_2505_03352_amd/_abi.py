"""ctypes declarations of the yeeopt C ABI (include/yeeopt.h).

Argument marshalling only.  Loading fails loudly when the HIP library has
not been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libyeeopt.so")

YO_OK = 0
YO_EINVAL = -1
YO_EUNSUPPORTED = -2
YO_EHIP = -3
YO_EWORKSPACE = -4
YO_EUNSTABLE = -5
YO_ESTATE = -6

YO_FORWARD, YO_ADJOINT, YO_BOTH = 1, 2, 3

STATUS_NAMES = {0: "YO_OK", -1: "YO_EINVAL", -2: "YO_EUNSUPPORTED", -3: "YO_EHIP",
                -4: "YO_EWORKSPACE", -5: "YO_EUNSTABLE", -6: "YO_ESTATE"}


class YeeOptError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class yo_grid(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int),
                ("dx", ct.c_double), ("dy", ct.c_double), ("dz", ct.c_double),
                ("courant", ct.c_double), ("npml", ct.c_int * 6),
                ("pml_m", ct.c_double), ("pml_sigma_scale", ct.c_double),
                ("pml_kappa_max", ct.c_double), ("pml_a_max", ct.c_double)]


class yo_design(ct.Structure):
    _fields_ = [("i0", ct.c_int), ("j0", ct.c_int), ("md", ct.c_int), ("nd", ct.c_int),
                ("k_lo", ct.c_int), ("k_hi", ct.c_int), ("mc", ct.c_int), ("nc", ct.c_int),
                ("filter_r", ct.c_double), ("supersample", ct.c_int),
                ("eps_core", ct.c_double), ("eps_clad", ct.c_double),
                ("sobel_delta", ct.c_double)]


class yo_plane(ct.Structure):
    _fields_ = [("axis", ct.c_int), ("index", ct.c_int), ("lo0", ct.c_int), ("lo1", ct.c_int),
                ("n0", ct.c_int), ("n1", ct.c_int)]


class yo_freq(ct.Structure):
    _fields_ = [("omega", ct.c_double), ("ramp_steps", ct.c_double),
                ("win_start", ct.c_int), ("win_len", ct.c_int)]


_P = ct.c_void_p
_S = ct.c_void_p   # hipStream_t
_I = ct.c_int

_SIGS = {
    "yo_plan_create": [ct.POINTER(yo_grid), ct.POINTER(yo_design), _I, _I, ct.POINTER(yo_freq),
                       _I, ct.POINTER(yo_plane), _I, ct.POINTER(yo_plane), ct.POINTER(_P)],
    "yo_set_morphology": [_P, ct.c_char_p, ct.c_double, ct.c_double],
    "yo_set_pulse": [_P, ct.c_double, ct.c_double, ct.c_double],
    "yo_set_dft_stride": [_P, _I],
    "yo_set_time_blocking": [_P, _I],
    "yo_set_alpha_terms": [_P, _I],
    "yo_workspace_bytes": [_P, ct.POINTER(ct.c_size_t)],
    "yo_bind_workspace": [_P, _P, ct.c_size_t, _S],
    "yo_bind_static_workspace": [_P, _S],
    "yo_set_background": [_P, _P, _P, _S],
    "yo_set_source_mode": [_P, _I, _P, _S],
    "yo_set_port_mode": [_P, _I, _P, _P, _S],
    "yo_set_design": [_P, _P, ct.c_double, _S],
    "yo_run": [_P, _I, _I, _I, _S],
    "yo_reset": [_P, _I, _S],
    "yo_advance": [_P, _I, _I, _S],
    "yo_finalize": [_P, _I, _S],
    "yo_advance_many": [ct.POINTER(_P), ct.POINTER(_I), _I, _I, _I, _I, _S],
    "yo_steps_done": [_P, ct.POINTER(_I)],
    "yo_set_tiling": [_P, _I, _I, _I],
    "yo_set_timing": [_P, _I, _I],
    "yo_unbinarity": [_P, ct.c_double, ct.c_double, _P, _P],
    "yo_adam_step": [_P, _P, _P, _P, _I, _I, ct.c_double, ct.c_double, ct.c_double, ct.c_double, _P],
    "yo_get_timing": [_P, _I, ct.POINTER(ct.c_float), ct.POINTER(ct.c_int)],
    "yo_alpha": [_P, _P, _S],
    "yo_gradient": [_P, _P, _P, _S],
    "yo_gradient_kappa": [_P, _P, _P, _S],
    "yo_chain_vjp": [_P, _P, _P, _S],
    "yo_rhs_count": [_P, ct.POINTER(_I)],
    "yo_get_dft": [_P, _I, _I, _P, _S],
    "yo_set_fields": [_P, _I, _P, _P, _S],
    "yo_get_fields": [_P, _I, _P, _P, _S],
    "yo_get_kappa": [_P, _P, _S],
    "yo_tile_table": [_P, _I, ct.POINTER(ct.c_int), _I, ct.POINTER(ct.c_int)],
    "yo_time_kernel": [_P, _I, _I, ct.POINTER(ct.c_float), ct.POINTER(ct.c_double),
                       ct.POINTER(ct.c_double), _S],
    "yo_model_bytes": [_P, _I, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)],
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libyeeopt.so not found at {LIB_PATH}: run "
                              "`python -c 'import __graft_entry__ as g; g.build()'` first")
        L = ct.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ct.c_int
        L.yo_plan_destroy.argtypes = [_P]
        L.yo_plan_destroy.restype = None
        L.yo_last_error.restype = ct.c_char_p
        L.yo_version.restype = ct.c_char_p
        _lib = L
    return _lib


def check(status: int):
    if status != YO_OK:
        msg = lib().yo_last_error().decode(errors="replace")
        raise YeeOptError(status, msg)
    return status


def call(name: str, *args):
    return check(getattr(lib(), name)(*args))
