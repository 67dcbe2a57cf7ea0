"""GPU parity of the look-back kernels with their fallback forced: a system
created with KA_LOOKBACK_SPIN=1 never waits for a predecessor tile that has
not published its total, but computes that total from the predecessor's
input at once.  Scans (both tile sizes), compactions, the sort (whose
digit-table scans are look-back scans) and the composed index must still
match the oracle exactly."""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SCAN_TILE, LARGE_SCAN, LARGE_SCAN_TILE = 8192, 1 << 23, 16384


@pytest.fixture(scope="module")
def sess():
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import Session
    old = os.environ.get("KA_LOOKBACK_SPIN")
    os.environ["KA_LOOKBACK_SPIN"] = "1"
    try:
        s = Session()
        # the variable is read when the system first uses the device
        act = s.spawn("exclusive_scan_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)])
        x = np.arange(5, dtype=np.uint32)
        (y,) = s.request(act, ka.val(x.ctypes.data, 5), n_out=1)
        s.release_actor(act)
        assert list(y) == [0, 0, 1, 3, 6]
    finally:
        if old is None:
            del os.environ["KA_LOOKBACK_SPIN"]
        else:
            os.environ["KA_LOOKBACK_SPIN"] = old
    yield s
    s.close()


@pytest.mark.parametrize("n", [SCAN_TILE + 1, 300 * SCAN_TILE + 17, LARGE_SCAN + 40 * LARGE_SCAN_TILE + 3])
def test_scan_with_fallback(sess, n):
    import paper_1709_07781_amd as ka
    x = workloads.u32(4000 + n % 997, n)
    act = sess.spawn("exclusive_scan_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)])
    try:
        for _ in range(2):
            (y,) = sess.request(act, ka.val(x.ctypes.data, n), n_out=1)
            np.testing.assert_array_equal(y, oracle.default().exclusive_scan(x))
    finally:
        sess.release_actor(act)


@pytest.mark.parametrize("zeros", ["third", "most"])
def test_compaction_with_fallback(sess, zeros):
    import paper_1709_07781_amd as ka
    n = 257 * SCAN_TILE + 5
    x = workloads.u32(4100, n)
    r = workloads.u32(4101, n)
    if zeros == "third":
        x[r % 3 == 0] = 0
    else:
        x[r % 50 != 0] = 0
    act = sess.spawn("compact_nonzero_u32", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)])
    try:
        (y,) = sess.request(act, ka.val(x.ctypes.data, n), n_out=1)
    finally:
        sess.release_actor(act)
    np.testing.assert_array_equal(y, oracle.default().compact_nonzero(x))


def test_index_with_fallback(sess):
    v = workloads.plain_request(seed=4200, n=(1 << 21) + 333, bound=1 << 16)
    got = sess.wah_index(sess.upload(v))
    exp = oracle.default().wah_index(v)
    for g, e in zip(got, exp):
        np.testing.assert_array_equal(g, e)


@pytest.mark.parametrize("bits", [0, 16, 10])
def test_index_hint_with_fallback(sess, bits):
    """The encoder's two look-back chains (words, values) and the narrow-key
    sort's table scans, every stall taking the fallback."""
    n = (1 << 20) + 4096 * 7 + 13
    v = workloads.zipf_values(4300 + bits, n)
    if bits:
        v = (v & np.uint32((1 << bits) - 1)).astype(np.uint32)
    got = sess.wah_index(sess.upload(v), value_bits=bits)
    exp = oracle.default().wah_index(v)
    for g, e in zip(got, exp):
        np.testing.assert_array_equal(g, e)
