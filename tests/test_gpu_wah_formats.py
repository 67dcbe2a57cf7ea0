"""GPU parity of the index in the other word formats (canonical WAH with
1-fills, PLWAH) and of the query path on the index: lookup of values in the
table, decoding of one bitmap, AND / OR of two bitmaps re-encoded in any
format.  Every result must equal the oracle's (oracle.wah_index_format,
wah_lookup, wah_decode, wah_combine), word for word."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

FMTS = [0, 1, 2]


@pytest.fixture(scope="module")
def sess():
    from paper_1709_07781_amd.session import Session
    s = Session()
    yield s
    s.close()


@pytest.fixture(scope="module")
def ora():
    return oracle.default()


def _layout(kind, n, seed):
    """Layouts whose bitmaps hold long runs of full groups, groups of 30 rows
    after such runs and single rows after gaps (the cases the formats treat
    differently), besides the usual ones."""
    r = np.arange(n, dtype=np.int64)
    if kind == "full_runs":  # values change every 5 chunks: runs of 5 full groups
        return ((r // (31 * 5)) % 3).astype(np.uint32)
    if kind == "runs_then_30":  # value 1 holds 4 full chunks, then a chunk missing one row, repeatedly
        v = np.zeros(n, np.uint32)
        block = r // (31 * 6)
        pos = r % (31 * 6)
        v[(pos < 31 * 5) & (block % 2 == 0)] = 1
        v[(pos == 31 * 4 + 7) & (block % 2 == 0)] = 2  # chunk 4 of the block misses one row of value 1
        return v
    if kind == "single_rows":  # value 9 at one row every few chunks, otherwise uniform small values
        v = workloads.uniform_values(seed, n, 4)
        v[(r % 97) == 13] = 9
        return v
    return workloads.structured(kind, n, seed=seed)


KINDS = ["full_runs", "runs_then_30", "single_rows", "all_equal", "alternating_chunks", "zipf", "distinct",
         "uniform1024", "sparse_hot"]
SIZES = [0, 1, 30, 31, 62, 155, 4096 + 31, 3 * 8192 + 5, 70_001]


@pytest.mark.parametrize("fmt", [1, 2])
@pytest.mark.parametrize("bits", [0, 16])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", SIZES)
def test_index_formats(sess, ora, fmt, bits, kind, n):
    v = _layout(kind, n, seed=n + 5)
    if bits:
        v = (v & np.uint32((1 << bits) - 1)).astype(np.uint32)
    got = sess.wah_index(v, value_bits=bits, fmt=fmt)
    for g, e, what in zip(got, ora.wah_index_format(v, fmt), ("keys", "offsets", "words")):
        np.testing.assert_array_equal(g, e, err_msg=f"{what} fmt={fmt} bits={bits} {kind} n={n}")


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_index_formats_large(sess, ora, fmt):
    v = _layout("runs_then_30", (1 << 21) + 77, seed=3)
    got = sess.wah_index(v, value_bits=12, fmt=fmt)
    for g, e in zip(got, ora.wah_index_format(v, fmt)):
        np.testing.assert_array_equal(g, e)


def _run(sess, kernel, args, n_out, ins):
    act = sess.spawn(kernel, args)
    try:
        return sess.request(act, *ins, n_out=n_out)
    finally:
        sess.release_actor(act)


@pytest.mark.parametrize("n", [1, 5000, 100_000])
def test_lookup(sess, ora, n):
    import paper_1709_07781_amd as ka
    v = workloads.zipf_values(n, n, 1.1, 1 << 12)
    keys, _, _ = ora.wah_index(v)
    q = np.concatenate([workloads.uniform_values(n + 1, 3000, 1 << 13), keys[:50], [0, 0xFFFFFFFF]]).astype(np.uint32)
    (slots,) = _run(sess, "wah_lookup", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_IN, in_mode=ka.KA_VAL),
                                         ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)], 1,
                    [ka.val(q.ctypes.data, q.size), ka.val(keys.ctypes.data, keys.size)])
    np.testing.assert_array_equal(slots, ora.wah_lookup(keys, q))


def test_lookup_on_index_refs(sess, ora):
    """Lookup against the device-resident table of an index built on the GPU."""
    import paper_1709_07781_amd as ka
    v = workloads.plain_request(seed=8, n=50_000, bound=700)
    res = sess.wah_index(sess.upload(v), refs=True, value_bits=10)
    q = np.arange(0, 1024, dtype=np.uint32)
    act = sess.spawn("wah_lookup", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_IN),
                                    ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)])
    try:
        (slots,) = sess.request(act, ka.val(q.ctypes.data, q.size), ka.ref(res.keys_ref), n_out=1)
    finally:
        sess.release_actor(act)
        for r in (res.keys_ref, res.offsets_ref, res.words_ref):
            sess.release_ref(r)
    keys, _, _ = ora.wah_index(v)
    np.testing.assert_array_equal(slots, ora.wah_lookup(keys, q))


def _bitmaps(ora, v, fmt):
    keys, offs, words = ora.wah_index_format(v, fmt)
    return keys, [words[offs[d]:offs[d + 1]] for d in range(keys.size)]


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("kind", ["runs_then_30", "single_rows", "full_runs", "zipf"])
def test_decode(sess, ora, fmt, kind):
    import paper_1709_07781_amd as ka
    n = 31 * 700 + 11
    v = _layout(kind, n, seed=21)
    ng = (n + 30) // 31
    keys, bms = _bitmaps(ora, v, fmt)
    for d in list(range(min(keys.size, 6))) + [keys.size - 1]:
        w = np.ascontiguousarray(bms[d])
        priv = (ctypes.c_uint32 * 2)(fmt, ng)
        (groups,) = _run(sess, "wah_decode", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_PRIV, count=2, init=priv),
                                              ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)], 1, [ka.val(w.ctypes.data, w.size)])
        np.testing.assert_array_equal(groups, ora.wah_decode(w, fmt, ng), err_msg=f"fmt={fmt} {kind} d={d}")
        # the decoded groups are the value's rows
        bits = np.unpackbits(groups.view(np.uint8), bitorder="little").reshape(-1, 32)[:, :31].reshape(-1)[:n]
        np.testing.assert_array_equal(bits.astype(bool), v == keys[d])


def test_decode_rejects_too_few_groups(sess, ora):
    import paper_1709_07781_amd as ka
    v = _layout("full_runs", 31 * 40, seed=1)
    _, bms = _bitmaps(ora, v, 1)
    w = np.ascontiguousarray(bms[0])
    priv = (ctypes.c_uint32 * 2)(1, 10)  # the bitmap covers more than 10 groups
    (groups,) = _run(sess, "wah_decode", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_PRIV, count=2, init=priv),
                                          ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)], 1, [ka.val(w.ctypes.data, w.size)])
    assert groups.size == 0


@pytest.mark.parametrize("fin", FMTS)
@pytest.mark.parametrize("fout", FMTS)
@pytest.mark.parametrize("op", [0, 1])
def test_combine(sess, ora, fin, fout, op):
    import paper_1709_07781_amd as ka
    n = 31 * 900 + 17
    ng = (n + 30) // 31
    v = _layout("runs_then_30", n, seed=2)
    w = _layout("single_rows", n, seed=4)
    _, bv = _bitmaps(ora, v, fin)
    _, bw = _bitmaps(ora, w, fin)
    pairs = [(bv[0], bv[1]), (bv[1], bv[2]), (bv[1], bw[0]), (bw[3], bv[0]), (bw[0], bw[1]), (bv[0], bv[0])]
    for a, b in pairs:
        a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
        priv = (ctypes.c_uint32 * 4)(op, fin, fout, ng)
        (out,) = _run(sess, "wah_combine", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_IN, in_mode=ka.KA_VAL),
                                            ka.arg(ka.KA_PRIV, count=4, init=priv),
                                            ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)], 1,
                      [ka.val(a.ctypes.data, a.size), ka.val(b.ctypes.data, b.size)])
        np.testing.assert_array_equal(out, ora.wah_combine(a, b, fin, ng, op, fout),
                                      err_msg=f"fin={fin} fout={fout} op={op}")


def test_combine_large_device(sess, ora):
    """AND and OR of two bitmaps of an index built on the GPU, as device refs."""
    import paper_1709_07781_amd as ka
    n = (1 << 20) + 5
    ng = (n + 30) // 31
    v = _layout("runs_then_30", n, seed=6)
    keys, offs, words = ora.wah_index_format(v, 1)
    a = np.ascontiguousarray(words[offs[0]:offs[1]])
    b = np.ascontiguousarray(words[offs[1]:offs[2]])
    ta, tb = sess.upload(a), sess.upload(b)
    ra, rb = sess.wrap(ta), sess.wrap(tb)
    try:
        for op in (0, 1):
            priv = (ctypes.c_uint32 * 4)(op, 1, 2, ng)
            (out,) = _run(sess, "wah_combine", [ka.arg(ka.KA_IN), ka.arg(ka.KA_IN), ka.arg(ka.KA_PRIV, count=4, init=priv),
                                                ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL)], 1, [ka.ref(ra), ka.ref(rb)])
            np.testing.assert_array_equal(out, ora.wah_combine(a, b, 1, ng, op, 2))
    finally:
        sess.release_ref(ra)
        sess.release_ref(rb)
