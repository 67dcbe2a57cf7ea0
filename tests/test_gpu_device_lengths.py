"""Stages after a compaction: the compaction's count stays on the device, and
the sort, the encoders and the lookup read it there (grids sized by the
capacity, tiles past the count leave at once).  A composition compact -> sort
-> encode is sent without any host read of a length (ka_system_length_reads
does not move), and its results equal the oracle's on the compacted values."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SORT_TILE, ENC_TILE = 8192, 8192


@pytest.fixture(scope="module")
def sess():
    from paper_1709_07781_amd.session import Session
    s = Session()
    yield s
    s.close()


@pytest.fixture(scope="module")
def ora():
    return oracle.default()


def _ka():
    import paper_1709_07781_amd as ka
    return ka


def _values(n, zero_frac, seed, bits=16):
    """Zipf values below 2^bits with a fraction zero_frac of zeros."""
    v = workloads.structured("zipf", n, seed=seed) & np.uint32((1 << bits) - 1)
    rng = np.random.default_rng(seed + 100)
    v[rng.random(n) < zero_frac] = 0
    return v


def _send_refs(sess, actor, v, n_out):
    """Sends v (host value) and receives n_out REF outputs; returns the refs
    and the number of host length reads the send and the receive made."""
    ka = _ka()
    before = sess.length_reads()
    t = sess.send(actor, ka.val(v.ctypes.data, v.size))
    sent = sess.length_reads()
    try:
        refs = sess.receive(t, n_out)
    finally:
        sess.release_ticket(t)
    return refs, sent - before, sess.length_reads() - before


def _read_all(sess, refs):
    out = [sess.read(r) for r in refs]
    for r in refs:
        sess.release_ref(r)
    return out


def _compact_actor(sess):
    ka = _ka()
    return sess.spawn("compact_nonzero_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT)])


SIZES = [1, 7, 4097, ENC_TILE + 1, ENC_TILE + 31, 3 * SORT_TILE + 7, 70_001]
FRACS = [0.0, 0.3, 0.9, 1.0]


@pytest.mark.parametrize("frac", FRACS)
@pytest.mark.parametrize("n", SIZES)
def test_compact_sort_encode_without_host_reads(sess, ora, n, frac):
    ka = _ka()
    v = _values(n, frac, seed=n % 97 + int(frac * 10))
    comp = _compact_actor(sess)
    sort = sess.spawn("radix_sort_rows_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT), ka.arg(ka.KA_OUT)])
    enc = sess.spawn("wah_encode_sorted", [ka.arg(ka.KA_IN), ka.arg(ka.KA_IN)] + [ka.arg(ka.KA_OUT) for _ in range(3)])
    s1 = sess.compose(sort, comp)
    pipe = sess.compose(enc, s1)
    try:
        refs, at_send, at_receive = _send_refs(sess, pipe, v, 3)
        got = _read_all(sess, refs)
    finally:
        for a in (pipe, s1, enc, sort, comp):
            sess.release_actor(a)
    assert at_send == 0 and at_receive == 0, "a length was read back on the host inside the composition"
    exp = ora.wah_index(v[v != 0])
    for g, e, name in zip(got, exp, ("keys", "offsets", "words")):
        np.testing.assert_array_equal(g, e, err_msg=f"{name} n={n} zero fraction={frac}")


@pytest.mark.parametrize("frac", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("n", [5, SORT_TILE + 3, 3 * SORT_TILE + 7])
def test_compact_then_sort_rows(sess, ora, n, frac):
    """The sort's outputs get the compaction's count as their length."""
    ka = _ka()
    v = _values(n, frac, seed=7 + n % 13)
    comp = _compact_actor(sess)
    sort = sess.spawn("radix_sort_rows_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT), ka.arg(ka.KA_OUT)])
    pipe = sess.compose(sort, comp)
    try:
        refs, at_send, at_receive = _send_refs(sess, pipe, v, 2)
        sk, sr = _read_all(sess, refs)
    finally:
        for a in (pipe, sort, comp):
            sess.release_actor(a)
    assert at_send == 0 and at_receive == 0
    ek, er = ora.sort_pairs(v[v != 0])
    np.testing.assert_array_equal(sk, ek)
    np.testing.assert_array_equal(sr, er)


@pytest.mark.parametrize("bits,fmt", [(16, 0), (0, 0), (20, 0), (12, 1), (16, 2), (0, 1)])
@pytest.mark.parametrize("n", [9, SORT_TILE + 3, 3 * SORT_TILE + 7])
def test_compact_then_wah_index(sess, ora, n, bits, fmt):
    """The composed index actor (every value-bits path and word format) after a
    compaction."""
    ka = _ka()
    v = _values(n, 0.4, seed=3 + n % 11, bits=bits if 0 < bits <= 16 else 16)
    priv = (ctypes.c_uint32 * 2)(bits, fmt)
    comp = _compact_actor(sess)
    idx = sess.spawn("wah_index", [ka.arg(ka.KA_IN), ka.arg(ka.KA_PRIV, count=2, init=priv)]
                     + [ka.arg(ka.KA_OUT) for _ in range(3)])
    pipe = sess.compose(idx, comp)
    try:
        refs, at_send, at_receive = _send_refs(sess, pipe, v, 3)
        got = _read_all(sess, refs)
    finally:
        for a in (pipe, idx, comp):
            sess.release_actor(a)
    assert at_send == 0 and at_receive == 0
    c = v[v != 0]
    exp = ora.wah_index(c) if fmt == 0 else ora.wah_index_format(c, fmt)
    for g, e, name in zip(got, exp, ("keys", "offsets", "words")):
        np.testing.assert_array_equal(g, e, err_msg=f"{name} n={n} bits={bits} format={fmt}")


def test_compact_then_wah_index_rejects(sess):
    """A value at or above 2^value_bits among the compacted values still voids
    the result (every length 0), with the count on the device."""
    ka = _ka()
    n = 2 * SORT_TILE + 5
    v = _values(n, 0.5, seed=21, bits=12)
    v[n - 3] = 1 << 12
    priv = (ctypes.c_uint32 * 2)(12, 0)
    comp = _compact_actor(sess)
    idx = sess.spawn("wah_index", [ka.arg(ka.KA_IN), ka.arg(ka.KA_PRIV, count=2, init=priv)]
                     + [ka.arg(ka.KA_OUT) for _ in range(3)])
    pipe = sess.compose(idx, comp)
    try:
        refs, at_send, _ = _send_refs(sess, pipe, v, 3)
        lens = [sess.length(r) for r in refs]
        for r in refs:
            sess.release_ref(r)
    finally:
        for a in (pipe, idx, comp):
            sess.release_actor(a)
    assert at_send == 0
    assert lens == [0, 0, 0]


@pytest.mark.parametrize("frac", [0.0, 0.5, 1.0])
def test_compact_then_lookup(sess, ora, frac):
    """Queries counted on the device: the lookup answers exactly the compacted
    queries."""
    ka = _ka()
    n = 3 * 4096 + 11
    base = _values(20_000, 0.0, seed=31, bits=12)
    keys, _, _ = ora.wah_index(base)
    q = _values(n, frac, seed=32, bits=13)
    kref = sess.wrap(kt := sess.upload(keys))
    comp = _compact_actor(sess)
    look = sess.spawn("wah_lookup", [ka.arg(ka.KA_IN), ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT)])
    try:
        before = sess.length_reads()
        t1 = sess.send(comp, ka.val(q.ctypes.data, q.size))
        (cq,) = sess.receive(t1, 1)
        sess.release_ticket(t1)
        t2 = sess.send(look, ka.ref(cq), ka.ref(kref))
        assert sess.length_reads() == before
        (slots,) = sess.receive(t2, 1)
        sess.release_ticket(t2)
        got = sess.read(slots)
        sess.release_ref(slots)
        sess.release_ref(cq)
    finally:
        sess.release_actor(look)
        sess.release_actor(comp)
        sess.release_ref(kref)
    del kt
    np.testing.assert_array_equal(got, ora.wah_lookup(keys, q[q != 0]))
