"""The C-ABI library on the host: it loads, exports every function ka.h
declares, and validates signatures, messages and compositions before any
device work (no GPU needed)."""
import ctypes
import os
import subprocess
from ctypes import byref, c_void_p

import numpy as np
import pytest

import paper_1709_07781_amd as ka


def test_exports_every_declared_function():
    names = ka.header_functions()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(ka.lib, n)]
    assert not missing, missing
    # and nothing undeclared is exported under the ka_ prefix
    out = subprocess.run(["nm", "-D", "--defined-only", ka.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T ka_" in line}
    assert exported == set(names), exported ^ set(names)


def test_binding_covers_header():
    assert set(ka.header_functions()) == set(ka.SIGNATURES) | {"ka_error_string", "ka_last_error"}


@pytest.fixture
def host_system():
    s = c_void_p()
    ka.check(ka.ka_system_create(None, byref(s)))
    p = c_void_p()
    ka.check(ka.ka_program_builtin(s, byref(p)))
    yield s, p
    ka.ka_program_release(p)
    ka.check(ka.ka_system_destroy(s))


def _spawn(s, p, name, args, rng=None):
    a = c_void_p()
    r = rng or ka.nd_range()
    rc = ka.ka_spawn(s, p, name.encode(), byref(r), ka.sig(*args), len(args), byref(a))
    return rc, a


def test_error_strings():
    for code in range(0, -13, -1):
        assert ka.ka_error_string(code)
    assert ka.ka_error_string(-999) == b"unknown error"


def test_unknown_kernel(host_system):
    s, p = host_system
    rc, _ = _spawn(s, p, "no_such_kernel", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT)])
    assert rc == ka.KA_E_NOKERNEL


def test_signature_arity_and_type(host_system):
    s, p = host_system
    rc, _ = _spawn(s, p, "exclusive_scan_u32", [ka.arg(ka.KA_IN)])
    assert rc == ka.KA_E_ARITY
    rc, _ = _spawn(s, p, "exclusive_scan_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_IN)])
    assert rc == ka.KA_E_TYPE
    rc, _ = _spawn(s, p, "exclusive_scan_u32", [ka.arg(ka.KA_IN, dtype=ka.KA_F32), ka.arg(ka.KA_OUT)])
    assert rc == ka.KA_E_TYPE
    # a local argument where the kernel has none
    rc, _ = _spawn(s, p, "exclusive_scan_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_LOCAL, count=128)])
    assert rc == ka.KA_E_TYPE
    # priv without a value
    rc, _ = _spawn(s, p, "affine_u32", [ka.arg(ka.KA_IN_OUT), ka.arg(ka.KA_PRIV), ka.arg(ka.KA_PRIV)])
    assert rc == ka.KA_E_ARG


def test_range_rules(host_system):
    s, p = host_system
    rc, _ = _spawn(s, p, "exclusive_scan_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT)], ka.nd_range(local0=128))
    assert rc == ka.KA_E_ARG
    rc, _ = _spawn(s, p, "exclusive_scan_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT)], ka.nd_range(offset0=4))
    assert rc == ka.KA_E_ARG
    bad = ka.nd_range()
    bad.dims = 4
    rc, _ = _spawn(s, p, "exclusive_scan_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT)], bad)
    assert rc == ka.KA_E_ARG


def test_message_matching(host_system):
    s, p = host_system
    rc, a = _spawn(s, p, "exclusive_scan_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_REF), ka.arg(ka.KA_OUT)])
    assert rc == 0
    x = np.arange(16, dtype=np.uint32)
    t = c_void_p()
    # a value where a device reference is expected
    assert ka.ka_send(a, ka.values(ka.val(x.ctypes.data, 16)), 1, byref(t)) == ka.KA_E_TYPE
    # wrong arity
    assert ka.ka_send(a, ka.values(ka.val(x.ctypes.data, 16), ka.val(x.ctypes.data, 16)), 2, byref(t)) == ka.KA_E_ARITY
    assert ka.ka_send(a, None, 0, byref(t)) == ka.KA_E_ARITY
    # a REF element without a reference
    assert ka.ka_send(a, ka.values(ka.ref(None)), 1, byref(t)) == ka.KA_E_ARG
    ka.ka_actor_release(a)
    rc, a = _spawn(s, p, "exclusive_scan_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT)])
    # right dtype check on values
    assert ka.ka_send(a, ka.values(ka.val(x.ctypes.data, 16, dtype=ka.KA_F32)), 1, byref(t)) == ka.KA_E_TYPE
    # a well-formed request reaches the device check: no GPU here
    rc = ka.ka_send(a, ka.values(ka.val(x.ctypes.data, 16)), 1, byref(t))
    assert rc == ka.KA_E_DEVICE
    assert b"device" in ka.ka_last_error()
    ka.ka_actor_release(a)


def test_compose_type_checks(host_system):
    s, p = host_system
    _, sort = _spawn(s, p, "radix_sort_rows_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT), ka.arg(ka.KA_OUT)])
    _, enc = _spawn(s, p, "wah_encode_sorted", [ka.arg(ka.KA_IN), ka.arg(ka.KA_IN)] + [ka.arg(ka.KA_OUT)] * 3)
    _, scan = _spawn(s, p, "exclusive_scan_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT)])
    _, enc_val = _spawn(s, p, "wah_encode_sorted", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL)] * 2 + [ka.arg(ka.KA_OUT)] * 3)
    c = c_void_p()
    assert ka.ka_compose(enc, sort, byref(c)) == 0          # 2 refs -> 2 refs
    ka.ka_actor_release(c)
    assert ka.ka_compose(scan, sort, byref(c)) == ka.KA_E_TYPE   # 2 outputs -> 1 input
    assert ka.ka_compose(enc_val, sort, byref(c)) == ka.KA_E_TYPE  # ref -> value
    assert ka.ka_compose(sort, enc, byref(c)) == ka.KA_E_TYPE    # 3 outputs -> 1 input
    # with a mapping function the shapes are checked per message instead
    keep = ka.ka_map_fn(lambda i, ni, o, no, cap, ud: 0)
    ka.check(ka.ka_actor_set_mapping(scan, keep, ka.ka_map_fn(), None))
    assert ka.ka_compose(scan, sort, byref(c)) == 0
    ka.ka_actor_release(c)
    for a in (sort, enc, scan, enc_val):
        ka.ka_actor_release(a)


def test_refs_are_not_serializable(host_system):
    s, _ = host_system
    r = c_void_p()
    ka.check(ka.ka_ref_wrap(s, c_void_p(0x1000), ka.KA_U32, 4, ka.KA_ACCESS_READ, byref(r)))
    n = ctypes.c_uint64()
    assert ka.ka_ref_serialize(r, None, 0, byref(n)) == ka.KA_E_NOT_SERIALIZABLE
    cap = ctypes.c_uint64()
    ka.check(ka.ka_ref_capacity(r, byref(cap)))
    assert cap.value == 4
    dt, cnt, acc = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint32()
    ka.check(ka.ka_ref_info(r, byref(dt), byref(cnt), byref(acc)))
    assert (dt.value, cnt.value, acc.value) == (ka.KA_U32, 4, ka.KA_ACCESS_READ)
    ka.check(ka.ka_ref_retain(r))
    ka.check(ka.ka_ref_release(r))
    ka.check(ka.ka_ref_release(r))


def test_destroyed_system_rejects_use():
    s = c_void_p()
    ka.check(ka.ka_system_create(None, byref(s)))
    p = c_void_p()
    ka.check(ka.ka_program_builtin(s, byref(p)))
    ka.check(ka.ka_system_destroy(s))
    a = c_void_p()
    r = ka.nd_range()
    sg = ka.sig(ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT))
    assert ka.ka_spawn(s, p, b"exclusive_scan_u32", byref(r), sg, 2, byref(a)) == ka.KA_E_STATE
    assert ka.ka_system_destroy(s) == ka.KA_E_STATE
    ka.check(ka.ka_program_release(p))  # the last reference frees the system


def test_bad_arguments():
    assert ka.ka_system_create(None, None) == ka.KA_E_ARG
    cfg = ka.ka_system_config()
    cfg.n_streams = 65
    s = c_void_p()
    assert ka.ka_system_create(byref(cfg), byref(s)) == ka.KA_E_ARG
    assert ka.ka_send(None, None, 0, None) == ka.KA_E_ARG
    assert ka.ka_receive(None, None, 0, 0) == ka.KA_E_ARG
    assert ka.ka_ref_release(None) == ka.KA_E_ARG
    res = ka.ka_wah_result()
    assert ka.ka_wah_index(None, None, 0, 0, byref(res)) == ka.KA_E_ARG
