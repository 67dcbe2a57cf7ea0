"""GPU parity of the batched index build on batches whose requests all hold at
most 1024 values (one persistent launch: each work-group takes requests in
turn, sorts one in LDS, encodes it and writes it after the earlier requests).
Every request must equal the oracle's index of that request alone, and the
same batch through the tagged-sort path (value_bits above 22, where the
small-request path does not apply) must give the same bytes."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SMALL_SIZES = [0, 1, 2, 30, 31, 32, 61, 62, 63, 64, 93, 500, 1000, 1023, 1024, 0, 7]


@pytest.fixture(scope="module")
def sess():
    from paper_1709_07781_amd.session import Session
    s = Session()
    yield s
    s.close()


def _offsets(sizes):
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def _check(results, off, values):
    ora = oracle.default()
    assert len(results) == len(off) - 1
    for j in range(len(off) - 1):
        v = values[off[j]:off[j + 1]]
        ek, eo, ew = ora.wah_index(v)
        k, o, w = results[j]
        np.testing.assert_array_equal(k, ek, err_msg=f"request {j} keys (n={v.size})")
        np.testing.assert_array_equal(o, eo, err_msg=f"request {j} offsets (n={v.size})")
        np.testing.assert_array_equal(w, ew, err_msg=f"request {j} words (n={v.size})")


@pytest.mark.parametrize("kind", ["uniform", "all_equal", "alternating_chunks", "sparse_hot", "presorted", "reverse"])
@pytest.mark.parametrize("value_bits", [12, 22])
def test_small_requests_match_oracle(sess, kind, value_bits):
    off = _offsets(SMALL_SIZES)
    parts = []
    for i, n in enumerate(SMALL_SIZES):
        if kind == "uniform":
            parts.append(workloads.uniform_values(500 + i, n, 1 << value_bits))
        else:
            parts.append(workloads.structured(kind, n, seed=600 + i) & np.uint32((1 << value_bits) - 1))
    v = np.concatenate(parts).astype(np.uint32)
    _check(sess.wah_batch(v, off, value_bits), off, v)


def test_small_path_equals_tagged_sort_path(sess):
    off, v = workloads.batched_requests(seed=71, count=400, lo_log2=0, hi_log2=10)
    v = v & np.uint32((1 << 20) - 1)
    small = sess.wah_batch(v, off, 22)  # every request <= 1024 values, value_bits <= 22
    tagged = sess.wah_batch(v, off, 23)  # value_bits 23: the tagged radix sort path
    assert len(small) == len(tagged)
    for a, b in zip(small, tagged):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
    _check(small, off, v)


def test_small_requests_reject_values_beyond_value_bits(sess):
    import paper_1709_07781_amd as ka
    off = np.array([0, 100, 300, 301], dtype=np.uint32)
    v = workloads.uniform_values(81, 301, 1 << 10)
    v[250] = 1 << 10
    res = ka.ka_wah_batch_result()
    rc = ka.lib.ka_wah_batch(sess.sys, v.ctypes.data, v.size, off.ctypes.data, 3, 10, 0, ctypes.byref(res))
    assert rc == ka.KA_E_ARG
    v[250] = 5
    _check(sess.wah_batch(v, off, 10), off, v)


def test_small_requests_plan_replays(sess):
    from paper_1709_07781_amd.session import BatchPlan
    off, v1 = workloads.batched_requests(seed=91, count=256, lo_log2=0, hi_log2=10)
    n = int(off[-1])
    v2 = workloads.uniform_values(92, n, 1 << 12)
    plan = BatchPlan(sess, off, 12)
    try:
        for v in (v1, v2, v1):
            plan.run(v)
            _check(plan.result(), off, v)
    finally:
        plan.close()


def test_actor_size_hint(sess):
    """The builtin actor with its optional second private value (largest
    request + 1): a hint of at most 1024 takes the small-request path, no hint
    the tagged sort (same bytes); a request above 1024 values under such a
    hint fails the batch (every output length 0) instead of being truncated."""
    import paper_1709_07781_amd as ka
    off = np.array([0, 10, 110, 110, 140], dtype=np.uint32)
    v = workloads.uniform_values(61, 140, 1 << 8)

    def run(hint):
        priv = (ctypes.c_uint32 * 2)(8, hint)
        act = sess.spawn("wah_index_batch", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_IN, in_mode=ka.KA_VAL),
                                             ka.arg(ka.KA_PRIV, count=2, init=priv)] + [ka.arg(ka.KA_OUT)] * 5)
        try:
            refs = sess.request(act, ka.val(v.ctypes.data, v.size), ka.val(off.ctypes.data, off.size), n_out=5)
        finally:
            sess.release_actor(act)
        try:
            return [sess.length(r) for r in refs], [sess.read(r) for r in refs]
        finally:
            for r in refs:
                sess.release_ref(r)

    lens, outs = run(101)  # right: the largest request holds 100 values
    lens0, outs0 = run(0)  # no hint
    assert lens == lens0 and lens[0] > 0
    for a, b in zip(outs, outs0):
        np.testing.assert_array_equal(a, b)
    words = outs[2]
    ws = outs[4]
    ora = oracle.default()
    for j in range(len(off) - 1):
        np.testing.assert_array_equal(words[ws[j]:ws[j + 1]], ora.wah_index(v[off[j]:off[j + 1]])[2])
    lens_small, outs_small = run(11)  # below the largest request but within 1024: still exact
    assert lens_small == lens
    for a, b in zip(outs_small, outs):
        np.testing.assert_array_equal(a, b)
    big_off = np.array([0, 10, 2010], dtype=np.uint32)  # a 2000-value request
    big_v = workloads.uniform_values(62, 2010, 1 << 8)
    priv = (ctypes.c_uint32 * 2)(8, 11)
    act = sess.spawn("wah_index_batch", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_IN, in_mode=ka.KA_VAL),
                                         ka.arg(ka.KA_PRIV, count=2, init=priv)] + [ka.arg(ka.KA_OUT)] * 5)
    try:
        refs = sess.request(act, ka.val(big_v.ctypes.data, big_v.size), ka.val(big_off.ctypes.data, big_off.size),
                            n_out=5)
    finally:
        sess.release_actor(act)
    try:
        assert [sess.length(r) for r in refs] == [0] * 5
    finally:
        for r in refs:
            sess.release_ref(r)


@pytest.mark.parametrize("count", [1, 2047, 2048, 2049, 5000])
def test_small_requests_many_tickets(sess, count):
    """Both forms of the small-request path: the three-launch form (ka_wah_batch)
    and the persistent fused launch (a plan of sort variant 1), which has fewer
    work-groups than requests, so each takes several in turn from the ticket
    counter and writes a request's words and keys after all earlier requests'
    (the look-back over requests).  A value out of range in a late request
    rejects the batch in both."""
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import BatchPlan
    off, v = workloads.batched_requests(seed=120 + count % 7, count=count, lo_log2=0, hi_log2=10)
    _check(sess.wah_batch(v, off, 12), off, v)
    j = count - 1 - count // 7  # a late request that is not empty
    while off[j + 1] == off[j]:
        j -= 1
    bad = v.copy()
    bad[off[j]] = 1 << 12
    offu = off.astype(np.uint32)
    res = ka.ka_wah_batch_result()
    rc = ka.lib.ka_wah_batch(sess.sys, bad.ctypes.data, bad.size, offu.ctypes.data, count, 12, 0, ctypes.byref(res))
    assert rc == ka.KA_E_ARG
    plan = BatchPlan(sess, off, 12, shape=1)
    try:
        for x, ok in ((v, True), (bad, False), (v, True)):
            plan.run(x)
            if ok:
                _check(plan.result(), off, x)
            else:
                with pytest.raises(ka.KaError) as e:
                    plan.result()
                assert e.value.code == ka.KA_E_ARG
    finally:
        plan.close()
    _check(sess.wah_batch(v, off, 12), off, v)  # and the next batch is exact again


@pytest.mark.parametrize("kind", ["uniform", "all_equal", "alternating_chunks", "sparse_hot"])
def test_fused_launch_structured(sess, kind):
    """The persistent fused launch on the structured layouts and every size
    class of SMALL_SIZES, replayed."""
    from paper_1709_07781_amd.session import BatchPlan
    off = _offsets(SMALL_SIZES * 3)
    parts = []
    for i, n in enumerate(SMALL_SIZES * 3):
        if kind == "uniform":
            parts.append(workloads.uniform_values(700 + i, n, 1 << 12))
        else:
            parts.append(workloads.structured(kind, n, seed=800 + i) & np.uint32((1 << 12) - 1))
    v = np.concatenate(parts).astype(np.uint32)
    plan = BatchPlan(sess, off, 12, shape=1)
    try:
        for _ in range(3):
            plan.run(v)
            _check(plan.result(), off, v)
    finally:
        plan.close()
