"""GPU parity of the batched index build (ka_wah_batch, built-in actor
wah_index_batch): every request's (keys, offsets, words) must equal the
oracle's index of that request alone (rows restart at 0 in each request),
bit for bit.  Inputs: workloads.batched_requests (log-uniform sizes, values
uniform below 2^12) and hand-made layouts with empty and one-element requests."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sess():
    from paper_1709_07781_amd.session import Session
    s = Session()
    yield s
    s.close()


def _check(results, offsets, values, ora, sample=None):
    nreq = len(offsets) - 1
    assert len(results) == nreq
    idx = range(nreq) if sample is None else sample
    for j in idx:
        v = values[offsets[j]:offsets[j + 1]]
        ek, eo, ew = ora.wah_index(v)
        k, o, w = results[j]
        np.testing.assert_array_equal(k, ek, err_msg=f"request {j} keys (n={v.size})")
        np.testing.assert_array_equal(o, eo, err_msg=f"request {j} offsets (n={v.size})")
        np.testing.assert_array_equal(w, ew, err_msg=f"request {j} words (n={v.size})")


@pytest.mark.parametrize("seed,count,lo,hi", [(11, 64, 4, 12), (12, 300, 0, 10), (13, 17, 10, 16)])
def test_batch_matches_each_request(sess, seed, count, lo, hi):
    off, v = workloads.batched_requests(seed=seed, count=count, lo_log2=lo, hi_log2=hi)
    res = sess.wah_batch(v, off, 12)
    _check(res, off, v, oracle.default())


def test_batch_device_input_and_empty_requests(sess):
    import torch
    sizes = [0, 5, 0, 0, 31, 1, 62, 0, 4096, 4097, 0, 1000, 0]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    v = workloads.uniform_values(21, int(off[-1]), 1 << 12)
    dv = torch.from_numpy(v.view(np.int32)).to("cuda")
    res = sess.wah_batch(dv, off, 12)
    _check(res, off, v, oracle.default())
    for j, s in enumerate(sizes):
        if s == 0:
            k, o, w = res[j]
            assert k.size == 0 and w.size == 0 and list(o) == [0]


@pytest.mark.parametrize("kind", ["all_equal", "all_zero", "alternating_chunks", "sparse_hot", "presorted", "reverse"])
def test_batch_structured(sess, kind):
    parts = [workloads.structured(kind, n, seed=30 + i) & np.uint32(0xFFFF) for i, n in enumerate([1, 31, 32, 700,
                                                                                                   5000, 65])]
    off = np.zeros(len(parts) + 1, dtype=np.int64)
    np.cumsum([p.size for p in parts], out=off[1:])
    v = np.concatenate(parts).astype(np.uint32)
    res = sess.wah_batch(v, off, 16)
    _check(res, off, v, oracle.default())


def test_single_request_batch_equals_plain_index(sess):
    v = workloads.u32(41, 50_000)  # full 32-bit values: value_bits 32, one request
    res = sess.wah_batch(v, [0, v.size], 32)
    k, o, w = sess.wah_index(v)
    np.testing.assert_array_equal(res[0][0], k)
    np.testing.assert_array_equal(res[0][1], o)
    np.testing.assert_array_equal(res[0][2], w)


def test_all_requests_empty(sess):
    res = sess.wah_batch(np.zeros(0, dtype=np.uint32), [0, 0, 0, 0], 8)
    assert [(r[0].size, list(r[1]), r[2].size) for r in res] == [(0, [0], 0)] * 3


def test_batch_rejects_values_beyond_value_bits(sess):
    import paper_1709_07781_amd as ka
    v = workloads.uniform_values(51, 3000, 1 << 12)
    v[1234] = 1 << 12  # one value needs 13 bits
    off = np.array([0, 1000, 3000], dtype=np.uint32)
    res = ka.ka_wah_batch_result()
    rc = ka.lib.ka_wah_batch(sess.sys, v.ctypes.data, v.size, off.ctypes.data, 2, 12, 0, ctypes.byref(res))
    assert rc == ka.KA_E_ARG
    # the system stays usable
    ok = sess.wah_batch(v[:1000] & np.uint32(0xFFF), [0, 1000], 12)
    np.testing.assert_array_equal(ok[0][2], oracle.default().wah_index(v[:1000] & np.uint32(0xFFF))[2])


def test_batch_argument_errors(sess):
    import paper_1709_07781_amd as ka
    v = np.arange(10, dtype=np.uint32)
    res = ka.ka_wah_batch_result()
    bad = [
        (np.array([0, 5, 10], dtype=np.uint32), 2, 31),   # 31 value bits + 1 request bit is fine ...
        (np.array([0, 5, 10], dtype=np.uint32), 2, 0),    # value_bits 0
        (np.array([0, 5, 9], dtype=np.uint32), 2, 8),     # does not end at n
        (np.array([0, 6, 5, 10], dtype=np.uint32), 3, 8),  # decreasing
        (np.array([0, 2, 4, 6, 10], dtype=np.uint32), 4, 31),  # 31 + 2 bits > 32
    ]
    for i, (off, nreq, vb) in enumerate(bad):
        rc = ka.lib.ka_wah_batch(sess.sys, v.ctypes.data, v.size, off.ctypes.data, nreq, vb, 0, ctypes.byref(res))
        if i == 0:
            assert rc == 0
            ka.check(ka.lib.ka_wah_batch_result_free(ctypes.byref(res)))
        else:
            assert rc == ka.KA_E_ARG, (i, rc)


def test_batch_full_config_every_request(sess):
    """The batched configuration at full size (4096 requests, sizes 2^10..2^20,
    values below 2^12, about 6.2e8 elements) in the launch bench.py times:
    every request's keys, offsets and words against the oracle's index of that
    request alone.  This is the case that reaches the encoder's multi-group
    tile offsets (more than 1024 encoder tiles) together with request-relative
    rows.  The oracle runs on a pool of host threads."""
    import torch
    from parallel_oracle import map_requests
    off, v = workloads.batched_requests()
    dv = torch.from_numpy(v.view(np.int32)).to("cuda")
    res = sess.wah_batch(dv, off, 12)
    del dv
    torch.cuda.empty_cache()
    nreq = len(off) - 1
    assert len(res) == nreq
    exp = map_requests("wah_index", [v[off[j]:off[j + 1]] for j in range(nreq)])
    for j in range(nreq):
        for got, e, what in zip(res[j], exp[j], ("keys", "offsets", "words")):
            if not np.array_equal(got, e):
                raise AssertionError(f"request {j} (n={off[j + 1] - off[j]}): {what} differ from the oracle")


def test_batch_tagged_path_rejects_wide_values(sess):
    """A batch on the tagged-sort path (a request above 1024 values) holding
    values far above 2^value_bits (0xFFFFFFFF, 2^15 with value_bits 12) is
    rejected with KA_E_ARG, every request tag stays in range while it is
    rejected, and the system stays usable afterwards."""
    import paper_1709_07781_amd as ka
    v = workloads.uniform_values(52, 6000, 1 << 12)
    v[17] = 0xFFFFFFFF
    v[4321] = 1 << 15
    off = np.array([0, 1500, 1500, 6000], dtype=np.uint32)
    res = ka.ka_wah_batch_result()
    rc = ka.lib.ka_wah_batch(sess.sys, v.ctypes.data, v.size, off.ctypes.data, 3, 12, 0, ctypes.byref(res))
    assert rc == ka.KA_E_ARG
    good = v & np.uint32(0xFFF)
    got = sess.wah_batch(good, off, 12)
    _check(got, off, good, oracle.default())


@pytest.mark.parametrize("bits", [1, 2, 3, 4, 7, 8, 9, 10, 12, 13, 15, 16, 17, 20])
def test_batch_value_widths_and_tile_edges(sess, bits):
    """Values of 1..16 bits take the segmented sort (tiles cut at request
    boundaries and at the multiples of 8192, one or two passes over 16-bit
    keys); wider values the tagged sort.  Requests straddle tile edges, hold
    exactly a tile, are empty or hold one value."""
    sizes = [0, 1, 8191, 8192, 8193, 3, 0, 20000, 16384 + 5, 7, 0, 40000, 1, 8192 * 3 - 2]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    v = workloads.uniform_values(30 + bits, int(off[-1]), 1 << bits)
    v[:: 97] = (1 << bits) - 1  # the largest value appears in most requests
    res = sess.wah_batch(v, off, bits)
    _check(res, off, v, oracle.default())


@pytest.mark.parametrize("bits", [1, 3, 5, 9, 12, 13, 16])
def test_byte_digit_split(sess, bits):
    """The segmented sort with the byte digit split (batch variant 3: 8 bits,
    then the rest rounded up to even; variant 0, which ka_wah_batch takes,
    splits value_bits evenly) against the oracle, on the same request layout;
    and a value out of range rejects the batch."""
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import BatchPlan
    sizes = [0, 1, 8191, 8192, 8193, 3, 0, 20000, 16384 + 5, 7, 0, 40000, 1, 8192 * 3 - 2]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    v = workloads.uniform_values(50 + bits, int(off[-1]), 1 << bits)
    v[:: 89] = (1 << bits) - 1
    plan = BatchPlan(sess, off, bits, shape=3)
    try:
        plan.run(v)
        _check(plan.result(), off, v, oracle.default())
        bad = v.copy()
        bad[int(off[8]) + 11] = 1 << bits
        plan.run(bad)
        with pytest.raises(ka.KaError) as e:
            plan.result()
        assert e.value.code == ka.KA_E_ARG
        plan.run(v)
        _check(plan.result(), off, v, oracle.default())
    finally:
        plan.close()
