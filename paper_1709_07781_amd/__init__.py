"""Python binding of the kernel-actor C ABI (``include/ka.h``).

Argument marshalling only: every function below calls the function of the
same name in ``libka.so``; all work runs in the library's HIP kernels.  The
library must have been built (``paper_1709_07781_amd/build.py``); importing
the binding without it raises ``ImportError``.

PyTorch is optional and only used by callers for device memory and streams
(``tensor.data_ptr()`` into ``ka_ref_wrap``, ``torch.cuda.current_stream()``
into ``ka_system_config.stream``).
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libka.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "ka.h")

# ---- constants (ka.h) -----------------------------------------------------------------
KA_OK = 0
KA_E_ARG, KA_E_TYPE, KA_E_ARITY, KA_E_NOKERNEL, KA_E_DEVICE, KA_E_OOM = -1, -2, -3, -4, -5, -6
KA_E_BUDGET, KA_E_TIMEOUT, KA_E_NOT_SERIALIZABLE, KA_E_LAUNCH, KA_E_CANCELLED, KA_E_STATE = -7, -8, -9, -10, -11, -12
KA_U32, KA_I32, KA_U64, KA_F32, KA_U8 = 1, 2, 3, 4, 5
KA_IN, KA_OUT, KA_IN_OUT, KA_LOCAL, KA_PRIV = 1, 2, 3, 4, 5
KA_VAL, KA_REF = 0, 1
KA_ACCESS_READ, KA_ACCESS_WRITE, KA_ACCESS_RW = 1, 2, 3
KA_SYS_PROFILE = 1
KA_WAH_INPUT_DEVICE, KA_WAH_OUTPUT_REFS = 1, 2


def KA_WAH_VALUE_BITS(b: int) -> int:
    return (b & 0x3F) << 8


KA_WAH_PAPER, KA_WAH_CANONICAL, KA_WAH_PLWAH = 0, 1, 2


def KA_WAH_FORMAT(f: int) -> int:
    return (f & 0xFF) << 16


# ---- structs (ka.h) -----------------------------------------------------------------
class ka_system_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("n_streams", ctypes.c_uint32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("stream", ctypes.c_void_p),
                ("flags", ctypes.c_uint32)]


class ka_nd_range(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_uint32), ("global_", ctypes.c_uint64 * 3),
                ("offset", ctypes.c_uint64 * 3), ("local", ctypes.c_uint32 * 3)]


class ka_nd_range_dev(ctypes.Structure):
    _fields_ = [("global_", ctypes.c_uint64 * 3), ("offset", ctypes.c_uint64 * 3)]


class ka_value(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("dtype", ctypes.c_uint32), ("ptr", ctypes.c_void_p),
                ("count", ctypes.c_uint64), ("ref", ctypes.c_void_p)]


ka_size_fn = ctypes.CFUNCTYPE(ctypes.c_uint64, ctypes.POINTER(ka_value), ctypes.c_uint32, ctypes.c_void_p)
ka_map_fn = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.POINTER(ka_value), ctypes.c_uint32, ctypes.POINTER(ka_value),
                             ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32, ctypes.c_void_p)


class ka_arg(ctypes.Structure):
    _fields_ = [("dir", ctypes.c_uint32), ("dtype", ctypes.c_uint32), ("in_mode", ctypes.c_uint32),
                ("out_mode", ctypes.c_uint32), ("count", ctypes.c_uint64), ("size_fn", ka_size_fn),
                ("size_ud", ctypes.c_void_p), ("init", ctypes.c_void_p)]


class ka_wah_result(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("D", ctypes.c_uint64), ("W", ctypes.c_uint64),
                ("keys", ctypes.POINTER(ctypes.c_uint32)), ("offsets", ctypes.POINTER(ctypes.c_uint32)),
                ("words", ctypes.POINTER(ctypes.c_uint32)), ("keys_ref", ctypes.c_void_p),
                ("offsets_ref", ctypes.c_void_p), ("words_ref", ctypes.c_void_p)]


_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_U32, _U64, _I64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64
_U32P, _U64P = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)
_DBLP = ctypes.POINTER(ctypes.c_double)

# name -> argtypes; every function returns int except the two string functions.
class ka_wah_batch_result(ctypes.Structure):
    _fields_ = [("nreq", ctypes.c_uint32), ("n", ctypes.c_uint64), ("D", ctypes.c_uint64), ("W", ctypes.c_uint64),
                ("keys", ctypes.POINTER(ctypes.c_uint32)), ("offsets", ctypes.POINTER(ctypes.c_uint32)),
                ("words", ctypes.POINTER(ctypes.c_uint32)), ("key_start", ctypes.POINTER(ctypes.c_uint32)),
                ("word_start", ctypes.POINTER(ctypes.c_uint32)), ("keys_ref", ctypes.c_void_p),
                ("offsets_ref", ctypes.c_void_p), ("words_ref", ctypes.c_void_p), ("key_start_ref", ctypes.c_void_p),
                ("word_start_ref", ctypes.c_void_p)]


class ka_server_config(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_uint32), ("max_batch", ctypes.c_uint32), ("max_batch_bytes", ctypes.c_uint64),
                ("hbm_budget_bytes", ctypes.c_uint64),
                ("value_bits", ctypes.c_uint32), ("chain_len", ctypes.c_uint32),
                ("chain_a", ctypes.POINTER(ctypes.c_uint32)), ("chain_b", ctypes.POINTER(ctypes.c_uint32)),
                ("copy_threads", ctypes.c_uint32)]


class ka_request(ctypes.Structure):
    _fields_ = [("args", ctypes.POINTER(ka_value)), ("nargs", ctypes.c_uint32)]


class ka_server_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64), ("elements", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("mean_batch", ctypes.c_double), ("p50_us", ctypes.c_double),
                ("p99_us", ctypes.c_double), ("max_us", ctypes.c_double), ("mean_us", ctypes.c_double),
                ("queued", ctypes.c_uint64), ("budget_in_use", ctypes.c_uint64), ("budget_peak", ctypes.c_uint64)]


KA_REQ_WAH, KA_REQ_SCAN, KA_REQ_CHAIN = 0, 1, 2
KA_SRV_OUTPUT_REFS = 1
KA_PLAN_AUTOTUNE = 1


SIGNATURES = {
    "ka_system_create": [ctypes.POINTER(ka_system_config), _PP],
    "ka_system_destroy": [_P],
    "ka_system_synchronize": [_P],
    "ka_system_stream": [_P, _U32, _PP],
    "ka_system_memory": [_P, _U64P, _U64P],
    "ka_system_length_reads": [_P, _U64P],
    "ka_program_builtin": [_P, _PP],
    "ka_program_load": [_P, ctypes.c_char_p, _PP],
    "ka_program_release": [_P],
    "ka_spawn": [_P, _P, ctypes.c_char_p, ctypes.POINTER(ka_nd_range), ctypes.POINTER(ka_arg), _U32, _PP],
    "ka_actor_set_mapping": [_P, ka_map_fn, ka_map_fn, _P],
    "ka_compose": [_P, _P, _PP],
    "ka_actor_set_stream": [_P, _U32],
    "ka_actor_retain": [_P],
    "ka_actor_release": [_P],
    "ka_send": [_P, ctypes.POINTER(ka_value), _U32, _PP],
    "ka_send_as": [_P, _P, ctypes.POINTER(ka_value), _U32, _PP],
    "ka_receive": [_P, ctypes.POINTER(ka_value), _U32, _I64],
    "ka_ticket_arity": [_P, _U32P],
    "ka_batch_run": [_P, _P, _U32, _P],
    "ka_ticket_release": [_P],
    "ka_ref_info": [_P, _U32P, _U64P, _U32P],
    "ka_ref_capacity": [_P, _U64P],
    "ka_ref_read": [_P, _P, _U64],
    "ka_ref_device_ptr": [_P, _PP],
    "ka_ref_wrap": [_P, _P, _U32, _U64, _U32, _PP],
    "ka_ref_alloc": [_P, _U32, _U64, _PP],
    "ka_ref_retain": [_P],
    "ka_ref_release": [_P],
    "ka_ref_serialize": [_P, _P, _U64, _U64P],
    "ka_wah_index": [_P, _P, _U64, _U32, ctypes.POINTER(ka_wah_result)],
    "ka_wah_result_free": [ctypes.POINTER(ka_wah_result)],
    "ka_wah_batch": [_P, _P, _U64, _P, _U32, _U32, _U32, ctypes.POINTER(ka_wah_batch_result)],
    "ka_wah_batch_result_free": [ctypes.POINTER(ka_wah_batch_result)],
    "ka_affine_chain_raw": [_P, _P, _U64, _P, _P, _U32],
    "ka_wah_index_noalloc": [_P, _U64, _P, _P, _P, _P, _P],
    "ka_batch_plan_create": [_P, _P, _U32, _U32, _U32, _PP],
    "ka_batch_plan_shape": [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float), _U32],
    "ka_batch_plan_input": [_P, _PP],
    "ka_batch_plan_stream": [_P, _PP],
    "ka_batch_plan_run": [_P, _P, _U32],
    "ka_batch_plan_create_any": [_P, _U64, _U32, _U32, _U32, _U32, _PP],
    "ka_batch_plan_run_batch": [_P, _P, _P, _U32, _U32],
    "ka_batch_plan_result": [_P, ctypes.POINTER(ka_wah_batch_result)],
    "ka_batch_plan_destroy": [_P],
    "ka_server_create": [_P, ctypes.POINTER(ka_server_config), _PP],
    "ka_server_submit": [_P, _U32, _P, _U64, ctypes.c_double, _PP],
    "ka_server_send": [_P, _U32, ctypes.POINTER(ka_value), _U32, _U32, ctypes.c_double, _PP],
    "ka_server_wait": [_P, _I64],
    "ka_server_result": [_P, _U32, _P, _U64, _U64P],
    "ka_server_request_release": [_P],
    "ka_server_get_stats": [_P, ctypes.POINTER(ka_server_stats)],
    "ka_server_reset_stats": [_P],
    "ka_server_clock_us": [_DBLP],
    "ka_server_destroy": [_P],
    "ka_profile_get": [_P, ctypes.c_char_p, _U64P, _DBLP],
    "ka_profile_reset": [_P],
    "ka_profile_enable": [_P, ctypes.c_int],
}


def header_functions(path: str = HEADER_PATH) -> list[str]:
    """Names of every function ka.h declares."""
    with open(path) as f:
        text = f.read()
    return re.findall(r"KA_API\s+[\w\s\*]+?\b(ka_\w+)\s*\(", text)


def _load():
    # torch ships its own HIP runtime under another file name; loading it first
    # lets libka.so bind to that same runtime (matched by soname) instead of
    # bringing a second HIP/HSA runtime into the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run paper_1709_07781_amd/build.py (or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, argt in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = argt
        fn.restype = ctypes.c_int
    lib.ka_error_string.argtypes = [ctypes.c_int]
    lib.ka_error_string.restype = ctypes.c_char_p
    lib.ka_last_error.argtypes = []
    lib.ka_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()

# Module-level functions with the C names.
for _name in list(SIGNATURES) + ["ka_error_string", "ka_last_error"]:
    globals()[_name] = getattr(lib, _name)


class KaError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = lib.ka_last_error().decode(errors="replace")
        super().__init__(f"{what}: {lib.ka_error_string(code).decode()} ({code}): {msg}")
        self.code = code


def check(rc: int, what: str = "ka call") -> int:
    """Raises KaError for a negative status code."""
    if rc != KA_OK:
        raise KaError(rc, what)
    return rc


# ---- small marshalling helpers -----------------------------------------------------------
def arg(dir: int, dtype: int = KA_U32, in_mode: int = KA_REF, out_mode: int = KA_REF, count: int = 0,
        init=None) -> ka_arg:
    """One ka_arg; `init` (PRIV) is a ctypes array kept alive by the caller until ka_spawn returns."""
    a = ka_arg()
    a.dir, a.dtype, a.in_mode, a.out_mode, a.count = dir, dtype, in_mode, out_mode, count
    if init is not None:
        a.init = ctypes.cast(init, ctypes.c_void_p)
    return a


def sig(*args: ka_arg):
    return (ka_arg * len(args))(*args)


def nd_range(global0: int = 0, offset0: int = 0, local0: int = 0, dims: int = 1,
             global_=(0, 0, 0), offset=(0, 0, 0), local=(0, 0, 0)) -> ka_nd_range:
    r = ka_nd_range()
    r.dims = dims
    g = list(global_)
    o = list(offset)
    lo = list(local)
    g[0] = global0 or g[0]
    o[0] = offset0 or o[0]
    lo[0] = local0 or lo[0]
    for i in range(3):
        r.global_[i], r.offset[i], r.local[i] = g[i], o[i], lo[i]
    return r


def val(ptr: int, count: int, dtype: int = KA_U32) -> ka_value:
    """A VAL message element over host memory at address `ptr`."""
    v = ka_value()
    v.mode, v.dtype, v.ptr, v.count = KA_VAL, dtype, ptr, count
    return v


def ref(r) -> ka_value:
    v = ka_value()
    v.mode, v.ref = KA_REF, r
    return v


def values(*vs: ka_value):
    return (ka_value * len(vs))(*vs)
