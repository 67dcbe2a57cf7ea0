"""GPU parity of the built-in wah_index actor (the sort and the encoder queued
by one actor) under each value-bits hint: 1..16 sorts 16-bit keys in
ceil(bits / 8) fixed passes, 17..31 and 0 sort uint32 keys with the plan.  Every
result must equal the oracle's index word for word; a value at or above the
hint must fail the request and leave the system usable."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SORT_TILE, ENC_TILE = 8192, 8192
SIZES = [0, 1, 30, 31, 32, 4095, 4097, ENC_TILE - 1, ENC_TILE, ENC_TILE + 1, ENC_TILE + 31, 2 * ENC_TILE + 29,
         3 * SORT_TILE + 5, 40_000, (1 << 20) + 17]
KINDS = ["uniform4096", "u32", "all_equal", "all_max", "distinct", "reverse", "zipf", "alternating_chunks",
         "sparse_hot"]


@pytest.fixture(scope="module")
def sess():
    from paper_1709_07781_amd.session import Session
    s = Session()
    yield s
    s.close()


@pytest.fixture(scope="module")
def ora():
    return oracle.default()


def _values(kind, n, bits, seed):
    v = workloads.structured(kind, n, seed=seed)
    if bits < 32:
        v = (v & np.uint32((1 << bits) - 1)).astype(np.uint32)
    return v


def _check(got, exp, what):
    for g, e, name in zip(got, exp, ("keys", "offsets", "words")):
        np.testing.assert_array_equal(g, e, err_msg=f"{name} {what}")


@pytest.mark.parametrize("bits", [16, 12, 8])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", SIZES)
def test_narrow_keys(sess, ora, bits, kind, n):
    v = _values(kind, n, bits, seed=11 * n + bits)
    _check(sess.wah_index(v, value_bits=bits), ora.wah_index(v), f"bits={bits} {kind} n={n}")


@pytest.mark.parametrize("bits", [1, 2, 3, 5, 7, 9, 10, 11, 13, 14, 15])
@pytest.mark.parametrize("n", [ENC_TILE + 31, 5 * SORT_TILE + 3, 70_001])
def test_narrow_keys_other_widths(sess, ora, bits, n):
    v = _values("u32", n, bits, seed=n + bits)
    _check(sess.wah_index(v, value_bits=bits), ora.wah_index(v), f"bits={bits} n={n}")


@pytest.mark.parametrize("bits", [0, 17, 24, 31, 32])
@pytest.mark.parametrize("kind", ["u32", "zipf", "high_bits", "distinct"])
@pytest.mark.parametrize("n", [1, ENC_TILE + 1, 3 * SORT_TILE + 5, 70_001])
def test_wide_keys(sess, ora, bits, kind, n):
    v = _values(kind, n, bits if bits else 32, seed=5 * n + bits)
    _check(sess.wah_index(v, value_bits=bits), ora.wah_index(v), f"bits={bits} {kind} n={n}")


def test_device_input_refs_out(sess, ora):
    v = workloads.plain_request()
    t = sess.upload(v)
    res = sess.wah_index(t, refs=True, value_bits=10)
    got = tuple(sess.read(r) for r in (res.keys_ref, res.offsets_ref, res.words_ref))
    for r in (res.keys_ref, res.offsets_ref, res.words_ref):
        sess.release_ref(r)
    _check(got, ora.wah_index(v), "plain request, refs out")


@pytest.mark.parametrize("bits,bad", [(12, 1 << 12), (16, 0xFFFFFFFF), (8, 256), (20, 1 << 20), (31, 0x80000000)])
@pytest.mark.parametrize("where", [0, "middle", "last"])
def test_value_beyond_hint_is_rejected(sess, ora, bits, bad, where):
    import paper_1709_07781_amd as ka
    n = 3 * SORT_TILE + 77
    v = _values("u32", n, bits, seed=bits)
    pos = {0: 0, "middle": n // 2, "last": n - 1}[where]
    v[pos] = bad
    with pytest.raises(ka.KaError) as e:
        sess.wah_index(v, value_bits=bits)
    assert e.value.code == ka.KA_E_ARG
    # the system stays usable, and the same values below the hint pass
    v[pos] = 0
    _check(sess.wah_index(v, value_bits=bits), ora.wah_index(v), f"after rejection bits={bits}")


def test_hint_actor_directly(sess, ora):
    """The wah_index built-in spawned by name with its private value_bits."""
    import paper_1709_07781_amd as ka
    v = workloads.structured("zipf", 3 * SORT_TILE + 9, seed=3)
    bits = (ctypes.c_uint32 * 1)(16)
    act = sess.spawn("wah_index", [ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_PRIV, count=1, init=bits)]
                     + [ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL) for _ in range(3)])
    try:
        got = sess.request(act, ka.val(v.ctypes.data, v.size), n_out=3)
    finally:
        sess.release_actor(act)
    _check(got, ora.wah_index(v), "spawned wah_index")
