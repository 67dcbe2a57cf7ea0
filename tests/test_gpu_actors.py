"""GPU tests of the actor machinery around the kernels: user kernels from a
gfx950 code object (Sec. 3.2: programs built explicitly), the empty-stage
actor of the messaging-cost probe (Sec. 3.6), local and private arguments,
pre/post mapping functions (Sec. 3.4, Listing 3; Sec. 3.5) and reference
lifetimes.  Expected values are computed on the host from the definitions."""
import ctypes
import os
from ctypes import byref, c_void_p

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

HSACO = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kernels", "user_kernels.hsaco")


@pytest.fixture(scope="module")
def sess():
    from paper_1709_07781_amd.session import Session
    s = Session()
    yield s
    s.close()


@pytest.fixture(scope="module")
def prog(sess):
    import paper_1709_07781_amd as ka
    if not os.path.exists(HSACO):
        from paper_1709_07781_amd import build
        build.build_code_object(HSACO[:-len(".hsaco")] + ".hip")
    p = c_void_p()
    ka.check(ka.lib.ka_program_load(sess.sys, HSACO.encode(), byref(p)))
    yield p
    ka.lib.ka_program_release(p)


def _ka():
    import paper_1709_07781_amd as ka
    return ka


def test_unknown_module_kernel(sess, prog):
    ka = _ka()
    a = c_void_p()
    r = ka.nd_range(global0=16)
    rc = ka.lib.ka_spawn(sess.sys, prog, b"no_such_kernel", byref(r), ka.sig(ka.arg(ka.KA_IN)), 1, byref(a))
    assert rc == ka.KA_E_NOKERNEL


@pytest.mark.parametrize("n", [1, 255, 256, 257, 100_000])
def test_module_add(sess, prog, n):
    ka = _ka()
    a = workloads.u32(1, n)
    b = workloads.u32(2, n)
    act = sess.spawn("add_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_IN, in_mode=ka.KA_VAL),
                                 ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)], rng=ka.nd_range(global0=n), prog=prog)
    (c,) = sess.request(act, ka.val(a.ctypes.data, n), ka.val(b.ctypes.data, n), n_out=1)
    sess.release_actor(act)
    np.testing.assert_array_equal(c, a + b)


def test_module_local_and_priv(sess, prog):
    ka = _ka()
    n, wg, factor = 1000, 256, 7
    x = workloads.u32(3, n)
    f = (ctypes.c_uint32 * 1)(factor)
    act = sess.spawn("reverse_scale_local",
                     [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL),
                      ka.arg(ka.KA_LOCAL, count=wg), ka.arg(ka.KA_PRIV, count=1, init=f)],
                     rng=ka.nd_range(global0=n, local0=wg), prog=prog)
    (y,) = sess.request(act, ka.val(x.ctypes.data, n), n_out=1)
    sess.release_actor(act)
    exp = np.empty(n, dtype=np.uint32)
    for i in range(n):
        base, t = (i // wg) * wg, i % wg
        src = base + wg - 1 - t
        exp[i] = (x[src] * np.uint32(factor)) if src < n else 0xFFFFFFFF
    np.testing.assert_array_equal(y, exp)


def test_empty_stage_actor(sess, prog):
    """An actor with an empty kernel that receives a device reference and
    answers with nothing once the kernel ran."""
    ka = _ka()
    t = sess.upload(workloads.u32(4, 4096))
    r = sess.wrap(t)
    act = sess.spawn("empty_stage", [ka.arg(ka.KA_IN)], rng=ka.nd_range(global0=4096), prog=prog)
    for _ in range(3):
        tk = sess.send(act, ka.ref(r))
        n = ctypes.c_uint32()
        ka.check(ka.lib.ka_ticket_arity(tk, byref(n)))
        assert n.value == 0
        ka.check(ka.lib.ka_receive(tk, None, 0, -1))
        sess.release_ticket(tk)
    sess.release_actor(act)
    sess.release_ref(r)


def test_pre_and_post_mapping(sess):
    """pre drops the first message element; post keeps only the rows of the
    sort's response (dropping the keys ref releases it)."""
    ka = _ka()

    @ka.ka_map_fn
    def pre(inp, n_in, out, n_out, cap, ud):
        if n_in != 2 or cap < 1:
            return ka.KA_E_ARITY
        out[0] = inp[1]
        n_out[0] = 1
        return 0

    @ka.ka_map_fn
    def post(inp, n_in, out, n_out, cap, ud):
        out[0] = inp[1]
        n_out[0] = 1
        return 0

    act = sess.spawn("radix_sort_rows_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT),
                                             ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)])
    ka.check(ka.lib.ka_actor_set_mapping(act, pre, post, None))
    junk = np.arange(5, dtype=np.uint32)
    v = workloads.uniform_values(5, 20_000, 300)
    (rows,) = sess.request(act, ka.val(junk.ctypes.data, 5), ka.val(v.ctypes.data, v.size), n_out=1)
    # a mapping function's error fails the request
    t = c_void_p()
    rc = ka.lib.ka_send(act, ka.values(ka.val(v.ctypes.data, v.size)), 1, byref(t))
    assert rc == ka.KA_E_ARITY
    sess.release_actor(act)
    _, exp_rows = oracle.default().sort_pairs(v)
    np.testing.assert_array_equal(rows, exp_rows)


def test_refs_survive_their_producer(sess):
    """A ref received from an actor stays valid after the actor and the
    ticket are gone; releasing it returns the memory to the pool."""
    ka = _ka()
    v = workloads.u32(6, 50_000)
    act = sess.spawn("exclusive_scan_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT)])
    t = sess.send(act, ka.val(v.ctypes.data, v.size))
    sess.release_actor(act)
    (r,) = sess.receive(t, 1)
    sess.release_ticket(t)
    used0, _ = sess.memory()
    y = sess.read(r)
    sess.release_ref(r)
    used1, _ = sess.memory()
    assert used1 < used0
    np.testing.assert_array_equal(y, oracle.default().exclusive_scan(v))


def test_receive_buffer_too_small_and_timeout(sess):
    ka = _ka()
    v = workloads.u32(7, 1000)
    act = sess.spawn("exclusive_scan_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)])
    t = sess.send(act, ka.val(v.ctypes.data, v.size))
    small = np.empty(10, dtype=np.uint32)
    outs = (ka.ka_value * 1)()
    outs[0].ptr = small.ctypes.data
    outs[0].count = 10
    assert ka.lib.ka_receive(t, outs, 1, -1) == ka.KA_E_ARG
    assert outs[0].count == 1000
    # the ticket stays valid: receive again with a large enough buffer
    big = np.empty(1000, dtype=np.uint32)
    outs[0].ptr = big.ctypes.data
    outs[0].count = 1000
    ka.check(ka.lib.ka_receive(t, outs, 1, 0))
    np.testing.assert_array_equal(big, oracle.default().exclusive_scan(v))
    sess.release_ticket(t)
    sess.release_actor(act)


def test_budget_exceeded():
    """A system with a tiny HBM budget refuses allocations beyond it."""
    ka = _ka()
    from paper_1709_07781_amd.session import Session
    s = Session(budget_bytes=1 << 20)
    try:
        v = workloads.u32(8, 1 << 20)  # 4 MiB input > 1 MiB budget
        act = s.spawn("exclusive_scan_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT)])
        t = c_void_p()
        rc = ka.lib.ka_send(act, ka.values(ka.val(v.ctypes.data, v.size)), 1, byref(t))
        assert rc == ka.KA_E_BUDGET
        # a small request still fits
        w = workloads.u32(9, 1000)
        (r,) = s.request(act, ka.val(w.ctypes.data, w.size), n_out=1)
        np.testing.assert_array_equal(s.read(r), oracle.default().exclusive_scan(w))
        s.release_ref(r)
        s.release_actor(act)
    finally:
        s.close()


def test_in_place_write_waits_for_reads_on_other_streams():
    """A ref read by an actor on stream 1 and then written in place by an actor
    on stream 0: the write must not start before the read has finished
    (Sec. 3.5: refs are shared between stages).  The scan on stream 1 must see
    the original values."""
    import torch
    from paper_1709_07781_amd.session import Session
    ka = _ka()
    s = Session(n_streams=2)
    try:
        n = 1 << 24
        x = workloads.u32(61, n)
        dx = s.upload(x)
        rx = s.wrap(dx)
        scan = s.spawn("exclusive_scan_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT)])
        ka.check(ka.lib.ka_actor_set_stream(scan, 1))
        aff = s.affine_actor(3, 5)
        for _ in range(3):
            torch.cuda.synchronize()
            t = s.send(scan, ka.ref(rx))
            (r,) = s.request(aff, ka.ref(rx), n_out=1)
            (y,) = s.receive(t, 1)
            s.release_ticket(t)
            np.testing.assert_array_equal(s.read(y), oracle.default().exclusive_scan(x))
            s.release_ref(y)
            s.release_ref(r)
            x = (x * np.uint32(3) + np.uint32(5)).astype(np.uint32)
            np.testing.assert_array_equal(s.read(rx), x)
        s.release_actor(scan)
        s.release_actor(aff)
        s.release_ref(rx)
    finally:
        s.close()


def test_send_as_routes_the_response(sess):
    """ka_send_as: the scan actor's response goes to the affine actor, whose
    response answers the ticket (Sec. 3.4: send_as)."""
    ka = _ka()
    a, b = 0x01000193, 77
    v = workloads.u32(40, 70_001)
    scan = sess.spawn("exclusive_scan_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT)])
    aff = sess.affine_actor(a, b, in_mode=ka.KA_REF, out_mode=ka.KA_VAL)
    t = c_void_p()
    try:
        ka.check(ka.lib.ka_send_as(scan, aff, ka.values(ka.val(v.ctypes.data, v.size)), 1, byref(t)))
        (y,) = sess.receive(t, 1)
        sess.release_ticket(t)
    finally:
        sess.release_actor(scan)
        sess.release_actor(aff)
    o = oracle.default()
    exp = o.affine_chain(o.exclusive_scan(v), np.array([a], np.uint32), np.array([b], np.uint32))
    np.testing.assert_array_equal(y, exp)


def test_post_redirects_and_suppresses_the_response(sess):
    """A post-processing function sends the kernel's result on to another
    actor (ka_send from inside the mapping) and returns nothing: the original
    request's response is suppressed (arity 0), the redirected one carries the
    result (Sec. 3.4)."""
    ka = _ka()
    a, b = 5, 11
    aff = sess.affine_actor(a, b, in_mode=ka.KA_REF, out_mode=ka.KA_VAL)
    sent = []

    @ka.ka_map_fn
    def post(inp, n_in, out, n_out, cap, ud):
        t = c_void_p()
        rc = ka.lib.ka_send(aff, inp, n_in, byref(t))
        if rc:
            return rc
        sent.append(t)
        n_out[0] = 0
        return 0

    scan = sess.spawn("exclusive_scan_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT)])
    ka.check(ka.lib.ka_actor_set_mapping(scan, ka.ka_map_fn(), post, None))  # no pre-processing
    v = workloads.u32(41, 9_999)
    try:
        t = sess.send(scan, ka.val(v.ctypes.data, v.size))
        n = ctypes.c_uint32()
        ka.check(ka.lib.ka_ticket_arity(t, byref(n)))
        assert n.value == 0
        assert sess.receive(t, 0) == []
        sess.release_ticket(t)
        assert len(sent) == 1
        (y,) = sess.receive(sent[0], 1)
        sess.release_ticket(sent[0])
    finally:
        sess.release_actor(scan)
        sess.release_actor(aff)
    o = oracle.default()
    exp = o.affine_chain(o.exclusive_scan(v), np.array([a], np.uint32), np.array([b], np.uint32))
    np.testing.assert_array_equal(y, exp)
