"""GPU tests of ka_batch_run: independent requests to one actor as one batch.
For the built-in actors with a batched form (wah_index with a value-bits
hint, exclusive_scan_u32, affine_u32) every request's response must equal the
oracle's, whatever mix of host values and device references goes in and
whichever output mode the actor has; a value beyond the hint fails only its own
request; any other actor answers through ka_send in turn."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sess():
    from paper_1709_07781_amd.session import Session
    s = Session(n_streams=2)
    yield s
    s.close()


def _requests(sess, arrays, device: bool):
    """Messages for the arrays: host values, or device references."""
    import paper_1709_07781_amd as ka
    msgs, held = [], []
    for i, x in enumerate(arrays):
        if device:
            if x.size:
                t = sess.upload(x)
                r = sess.wrap(t)
            else:  # an empty device buffer of the library's own
                t, r = None, ctypes.c_void_p()
                ka.check(ka.lib.ka_ref_alloc(sess.sys, ka.KA_U32, 0, ctypes.byref(r)))
            held.append((r, t))
            msgs.append([ka.ref(r)])
        else:
            msgs.append([ka.val(x.ctypes.data if x.size else None, x.size)])
    return msgs, held


def _collect(sess, tickets, n_out, refs):
    out = []
    for t in tickets:
        got = sess.receive(t, n_out)
        if refs:
            arrs = [sess.read(r) for r in got]
            for r in got:
                sess.release_ref(r)
            got = arrs
        sess.release_ticket(t)
        out.append(got)
    return out


def _wah_actor(sess, bits, mode, in_mode):
    import paper_1709_07781_amd as ka
    b = (ctypes.c_uint32 * 1)(bits)
    return sess.spawn("wah_index", [ka.arg(ka.KA_IN, in_mode=in_mode),
                                    ka.arg(ka.KA_PRIV, count=1, init=b)]
                      + [ka.arg(ka.KA_OUT, out_mode=mode) for _ in range(3)])


@pytest.mark.parametrize("device_in", [False, True])
@pytest.mark.parametrize("refs_out", [False, True])
@pytest.mark.parametrize("sizes", ["small", "mixed"])
def test_wah_index_batch(sess, device_in, refs_out, sizes):
    import paper_1709_07781_amd as ka
    ora = oracle.default()
    if sizes == "small":  # every request fits one work-group
        lens = workloads.log_uniform_sizes(31, 40, 0, 10)
    else:  # the tagged sort, tiles spanning requests, empty requests
        lens = np.concatenate([workloads.log_uniform_sizes(32, 30, 4, 17), [0, 1, 0]]).astype(np.int64)
    arrays = [workloads.uniform_values(500 + i, int(m), 1 << 12) for i, m in enumerate(lens)]
    act = _wah_actor(sess, 12, ka.KA_REF if refs_out else ka.KA_VAL, ka.KA_REF if device_in else ka.KA_VAL)
    msgs, held = _requests(sess, arrays, device_in)
    try:
        got = _collect(sess, sess.batch_run(act, msgs), 3, refs_out)
    finally:
        sess.release_actor(act)
        for r, _ in held:
            sess.release_ref(r)
    for x, g in zip(arrays, got):
        for a, b in zip(g, ora.wah_index(x)):
            np.testing.assert_array_equal(a, b, err_msg=f"n={x.size}")


@pytest.mark.parametrize("device_in", [False, True])
@pytest.mark.parametrize("base", [200, 5000])
def test_wah_index_batch_rejects_one_request(sess, base, device_in):
    import paper_1709_07781_amd as ka
    ora = oracle.default()
    arrays = [workloads.uniform_values(600 + i, base + 37 * i, 1 << 12) for i in range(7)]
    arrays[3] = arrays[3].copy()
    arrays[3][5] = 0xFFFFFFFF
    act = _wah_actor(sess, 12, ka.KA_VAL, ka.KA_REF if device_in else ka.KA_VAL)
    msgs, held = _requests(sess, arrays, device_in)
    try:
        tickets = sess.batch_run(act, msgs)
        for i, (x, t) in enumerate(zip(arrays, tickets)):
            if i == 3:
                with pytest.raises(ka.KaError) as e:
                    sess.receive(t, 3)
                assert e.value.code == ka.KA_E_ARG
            else:
                for a, b in zip(sess.receive(t, 3), ora.wah_index(x)):
                    np.testing.assert_array_equal(a, b)
            sess.release_ticket(t)
    finally:
        sess.release_actor(act)
        for r, _ in held:
            sess.release_ref(r)


@pytest.mark.parametrize("device_in", [False, True])
@pytest.mark.parametrize("refs_out", [False, True])
def test_scan_batch(sess, refs_out, device_in):
    import paper_1709_07781_amd as ka
    ora = oracle.default()
    lens = np.concatenate([workloads.log_uniform_sizes(41, 25, 0, 18), [0, 8192, 8193]]).astype(np.int64)
    arrays = [workloads.u32(700 + i, int(m)) for i, m in enumerate(lens)]
    act = sess.spawn("exclusive_scan_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_REF if device_in else ka.KA_VAL),
                                            ka.arg(ka.KA_OUT, out_mode=ka.KA_REF if refs_out else ka.KA_VAL)])
    msgs, held = _requests(sess, arrays, device_in)
    try:
        got = _collect(sess, sess.batch_run(act, msgs), 1, refs_out)
    finally:
        sess.release_actor(act)
        for r, _ in held:
            sess.release_ref(r)
    for x, (g,) in zip(arrays, got):
        np.testing.assert_array_equal(g, ora.exclusive_scan(x), err_msg=f"n={x.size}")


@pytest.mark.parametrize("refs_out", [False, True])
def test_affine_batch_updates_refs_in_place(sess, refs_out):
    import paper_1709_07781_amd as ka
    ora = oracle.default()
    a, b = 0x9E3779B1, 12345
    lens = workloads.log_uniform_sizes(51, 20, 0, 16)
    arrays = [workloads.u32(800 + i, int(m)) for i, m in enumerate(lens)]
    act = sess.affine_actor(a, b, in_mode=ka.KA_REF, out_mode=ka.KA_REF if refs_out else ka.KA_VAL)
    msgs, held = _requests(sess, arrays, True)
    try:
        got = _collect(sess, sess.batch_run(act, msgs), 1, refs_out)
        for (r, _), x, (g,) in zip(held, [x for x in arrays if x.size], [g for x, g in zip(arrays, got) if x.size]):
            exp = ora.affine_chain(x, np.array([a], np.uint32), np.array([b], np.uint32))
            np.testing.assert_array_equal(g, exp)
            np.testing.assert_array_equal(sess.read(r), exp)  # the caller's reference, updated in place
    finally:
        sess.release_actor(act)
        for r, _ in held:
            sess.release_ref(r)


def test_composed_actor_answers_in_turn(sess):
    """An actor without a batched form: the requests go through ka_send."""
    import paper_1709_07781_amd as ka
    ora = oracle.default()
    sort = sess.spawn("radix_sort_rows_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT),
                                              ka.arg(ka.KA_OUT)])
    enc = sess.spawn("wah_encode_sorted", [ka.arg(ka.KA_IN), ka.arg(ka.KA_IN)]
                     + [ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL) for _ in range(3)])
    pipe = sess.compose(enc, sort)
    arrays = [workloads.uniform_values(900 + i, 3000 + 1000 * i, 1 << 10) for i in range(4)]
    msgs = [[ka.val(x.ctypes.data, x.size)] for x in arrays]
    try:
        got = _collect(sess, sess.batch_run(pipe, msgs), 3, False)
    finally:
        for x in (pipe, sort, enc):
            sess.release_actor(x)
    for x, g in zip(arrays, got):
        for a, b in zip(g, ora.wah_index(x)):
            np.testing.assert_array_equal(a, b)
