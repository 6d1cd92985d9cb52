"""ctypes binding of libdcf.so (include/dcf.h).  Argument marshalling only.

The binding exposes the C entry points under the same names.  Loading fails
loudly when the HIP library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdcf.so")

DCF_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENONPHYS", -5: "EBUDGET",
          -6: "EUNSUPPORTED"}

BC = {"periodic": 0, "wall": 1, "porous": 2, "zerograd": 3, "dirichlet": 4, "disturb": 5}
VISC = {"none": 0, "power": 1, "sutherland": 2}
STRETCH = {"uniform": 0, "tanh2": 1, "tanh1": 2}
SOURCE = {"none": 0, "massflux": 1}
SCHEME = {"weno5": 0, "teno6a": 1}


class DcfError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: DCF_{ERRORS.get(code, code)}: {msg}")
        self.code = code


class dcf_grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("stretch", C.c_int * 3), ("beta", C.c_double * 3)]


class dcf_gas(C.Structure):
    _fields_ = [("gamma", C.c_double), ("R", C.c_double), ("Pr", C.c_double),
                ("visc_law", C.c_int), ("mu_ref", C.c_double), ("T_ref", C.c_double),
                ("visc_param", C.c_double)]


class dcf_bc(C.Structure):
    _fields_ = [("kind", C.c_int), ("T_wall", C.c_double), ("dirichlet", C.c_void_p),
                ("porous_begin", C.c_int), ("porous_end", C.c_int), ("p_inf", C.c_double)]


_vp = C.c_void_p
_SIGS = {
    "dcf_create": [C.POINTER(dcf_grid), C.POINTER(dcf_gas), C.POINTER(C.c_void_p)],
    "dcf_destroy": [_vp],
    "dcf_state_info": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_long), C.POINTER(C.c_size_t)],
    "dcf_workspace_size": [_vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)],
    "dcf_set_workspace": [_vp, C.c_int, C.c_int, C.c_int, _vp, C.c_size_t],
    "dcf_workspace_size_for": [C.POINTER(dcf_grid), C.POINTER(dcf_gas), C.c_int, C.c_int,
                               C.c_int, C.POINTER(C.c_size_t)],
    "dcf_set_bc": [_vp, C.c_int, C.POINTER(dcf_bc)],
    "dcf_set_params": [_vp, _vp, C.c_int],
    "dcf_set_source": [_vp, C.c_int],
    "dcf_set_scheme": [_vp, C.c_int],
    "dcf_set_cost": [_vp, C.c_int, C.c_double],
    "dcf_init_state": [_vp, _vp, _vp, _vp],
    "dcf_rhs": [_vp, _vp, _vp, _vp],
    "dcf_compute_dt": [_vp, _vp, C.c_double, C.c_double, _vp, _vp],
    "dcf_rk3_step": [_vp, _vp, _vp, _vp],
    "dcf_rk3_step_noalloc": [_vp, _vp, _vp, _vp, _vp],
    "dcf_diagnostics": [_vp, _vp, _vp, _vp],
    "dcf_vjp_step": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "dcf_rk3_step_keep": [_vp, _vp, _vp, _vp, _vp],
    "dcf_cost_term": [_vp, _vp, C.c_double, _vp, _vp, _vp],
    "dcf_gradient": [_vp, _vp, C.c_int, _vp, C.c_int, _vp, _vp, _vp, _vp],
    "dcf_gradient_begin": [_vp, _vp, C.c_int, _vp, C.c_int, _vp, _vp, _vp],
    "dcf_gradient_advance": [_vp, C.c_int, C.POINTER(C.c_int), _vp],
    "dcf_gradient_finish": [_vp, _vp, _vp],
    "dcf_flags": [_vp, C.POINTER(C.c_uint), _vp],
    "dcf_time_kernel": [_vp, _vp, C.c_int, C.c_int, C.POINTER(C.c_double), _vp],
    "dcf_probe_begin": [_vp, C.c_int, C.c_int],
    "dcf_probe_end": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_double)],
    "dcf_batch_table_bytes": [C.c_int, C.POINTER(C.c_size_t)],
    "dcf_rk3_step_cfl": [_vp, _vp, _vp, C.c_double, C.c_double, _vp, _vp],
    "dcf_rk3_steps_cfl": [_vp, _vp, _vp, C.c_int, C.c_double, C.c_double, _vp],
    "dcf_batch_rk3_step": [C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.c_int, C.c_double,
                           _vp, C.c_size_t, _vp],
    "dcf_batch_table_fill": [C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.c_int, _vp,
                             C.c_size_t],
    "dcf_batch_rk3_step_table": [_vp, _vp, C.c_int, C.c_double, _vp],
}

_lib = None


def lib():
    """Load libdcf.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.dcf_last_error.restype = C.c_char_p
        L.dcf_last_error.argtypes = []
        L.dcf_num_params.restype = C.c_int
        L.dcf_num_params.argtypes = [_vp]
        _lib = L
    return _lib


def declared_symbols():
    """Function names declared in include/dcf.h."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "dcf.h")
    with open(hdr) as fh:
        text = fh.read()
    decl = re.compile(r"^(?:dcf_status|int|const char \*)\s*(dcf_[a-z_0-9]+)\s*\(", re.M)
    return sorted(set(decl.findall(text)))


def check(code, where):
    if code != DCF_OK:
        msg = lib().dcf_last_error().decode(errors="replace")
        raise DcfError(code, where, msg)


def call(name, *args):
    """Call a dcf_* entry point and raise DcfError on a non-zero status."""
    check(getattr(lib(), name)(*args), name)
