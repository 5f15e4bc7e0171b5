"""ctypes declarations of the C ABI in ``include/hemelb_hip.h``.

Argument marshalling only: every step of the lattice update runs in the HIP
library.  Loading fails loudly when the library has not been built; there is
no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhemelb_hip.so")

HL_OK = 0
HL_E_INVAL = -1
HL_E_RANGE = -2
HL_E_STATE = -3
HL_E_NOMEM = -4
HL_E_DEVICE = -5
HL_E_DIVERGED = -6
HL_W_MACH = 1
HL_W_TAU = 2

HL_F64 = 0
HL_F32_OFFSET = 1
HL_F16_OFFSET = 2
HL_F16_SCALED = 3
HL_F16_STOCHASTIC = 4
HL_WALL_SBB = 0
HL_WALL_BOUZIDI = 1
HL_INLET_VEL = 0
HL_OUTLET_P = 1
HL_ALTERNATE = 0
HL_BOTH_EACH_STEP = 1
HL_COUPLE_VELOCITY = 2
HL_DRIVE_LAUNCH = 0
HL_DRIVE_GRAPH = 1
HL_SCHED_XCD_REMAP = 1
HL_ORDER_BULK_MORTON = 1
HL_ORDER_BOUNDARY_MORTON = 2
HL_ORDER_INTERLEAVE = 4
HL_ORDER_BRICK = 8
HL_SCHED_FUSED = 2
HL_SCHED_PAIRS = 4
HL_SCHED_XCD_RUNS = 8
HL_SCHEME_AA = 16
HL_ORDER_BRICK_32 = 32
HL_DEBUG_CHECKS = 64
HL_SCHED_XCD_BRICKS = 16


class hl_info(ct.Structure):
    _fields_ = [
        ("n_sites", ct.c_int64),
        ("n_bulk", ct.c_int64),
        ("n_boundary", ct.c_int64),
        ("n_iolet_sites", ct.c_int64),
        ("n_domains", ct.c_int32),
        ("n_iolets", ct.c_int32),
        ("n_blocks_bulk", ct.c_int32),
        ("n_blocks_bnd", ct.c_int32),
        ("precision", ct.c_int32),
        ("block_size", ct.c_int32),
        ("sched_flags", ct.c_int32),
        ("drive", ct.c_int32),
        ("device_bytes", ct.c_int64),
        ("bytes_per_site", ct.c_double),
        ("n_near", ct.c_int64),
    ]


_P = ct.c_void_p
_I = ct.c_int
_I32 = ct.c_int32
_I64 = ct.c_int64
_D = ct.c_double
_pD = ct.POINTER(ct.c_double)
_pI32 = ct.POINTER(ct.c_int32)
_pI64 = ct.POINTER(ct.c_int64)

SIGNATURES = {
    "hl_create": (_I, [ct.POINTER(_P), _I, _I, ct.c_uint64]),
    "hl_destroy": (None, [_P]),
    "hl_last_error": (ct.c_char_p, [_P]),
    "hl_status_string": (ct.c_char_p, [_I]),
    "hl_set_stream": (_I, [_P, _P]),
    "hl_add_domain": (_I, [_P, _pI32]),
    "hl_validate_sites": (_I, [_I64, _pI32, _I64]),
    "hl_load_sites": (_I, [_P, _I32, _I64, _pI32, _pI32, _I32, _I64, _pI64, ct.POINTER(ct.c_int8),
                           ct.POINTER(ct.c_float)]),
    "hl_set_wall_normals": (_I, [_P, _I32, _I64, _pI64, _pD]),
    "hl_set_wall_mode": (_I, [_P, _I32, _I]),
    "hl_set_tau": (_I, [_P, _I32, _D]),
    "hl_set_iolet": (_I, [_P, _I32, _I32, _I, _pD, _pD, _D]),
    "hl_set_inlet_velocity": (_I, [_P, _I32, _I32, _D, _I, _pD, _pD, _D]),
    "hl_set_outlet_density": (_I, [_P, _I32, _I32, _D, _I, _pD, _pD, _D]),
    "hl_set_body_force": (_I, [_P, _I32, _pD, _D]),
    "hl_couple": (_I, [_P, _I32, _I32, _I32, _I32, _D, _D]),
    "hl_set_coupling_mode": (_I, [_P, _I]),
    "hl_commit": (_I, [_P]),
    "hl_step": (_I, [_P, _I64]),
    "hl_sync": (_I, [_P]),
    "hl_get_time": (_I, [_P, _pI64]),
    "hl_set_drive": (_I, [_P, _I, _I32]),
    "hl_read_density": (_I, [_P, _I32, _pD]),
    "hl_read_velocity": (_I, [_P, _I32, _pD]),
    "hl_read_wss": (_I, [_P, _I32, _pD]),
    "hl_read_populations": (_I, [_P, _I32, _pD]),
    "hl_set_populations": (_I, [_P, _I32, _pD]),
    "hl_read_iolet_stats": (_I, [_P, _I32, _pD, _pD]),
    "hl_read_iolet_bc": (_I, [_P, _I32, _I, _pD]),
    "hl_read_density_device": (_I, [_P, _I32, _P]),
    "hl_read_velocity_device": (_I, [_P, _I32, _P]),
    "hl_read_wss_device": (_I, [_P, _I32, _P]),
    "hl_read_observables_device_noalloc": (_I, [_P, _I32, _P, _P, _P]),
    "hl_get_state": (_I, [_P, _P, ct.POINTER(ct.c_size_t)]),
    "hl_set_state": (_I, [_P, _P, ct.c_size_t]),
    "hl_autotune": (_I, [_P, _I]),
    "hl_get_schedule": (_I, [_P, _pI32, _pI32]),
    "hl_set_schedule": (_I, [_P, _I32, _I32]),
    "hl_get_info": (_I, [_P, ct.POINTER(hl_info)]),
    "hl_time_kernels": (_I, [_P, _I64, _pD, _pD]),
    "hl_copy_bandwidth": (_I, [_P, _P, _I64, _I32, _P, _pD]),
    "hl_autotune_report": (_I, [_P, _pI32, _pD, _pD, _pD]),
    "hl_coupling_map": (_I, [_I32, _pD, _I32, _pD, _pI32, _pD]),
    "hl_velocity_factors": (_I, [_I32, _pD, _pD, _pD, _D, _pD]),
}

_lib = None


def load():
    """Load the built library (raises when it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "(the HIP library is the only implementation of this package)")
    lib = ct.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
