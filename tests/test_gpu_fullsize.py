"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times: the 2^26-value Zipf(1.1) index through the composed actor
(every word checked against the oracle), the 8-stage affine chain at 2^24,
the exclusive scan at 2^26, and a sort beyond them (2^28 + 3 keys) checked by
properties that hold at any size (keys non-decreasing, rows a permutation,
equal keys in row order, each output pair an input pair)."""
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


def test_large_zipf_request_composed(sess):
    import paper_1709_07781_amd as ka
    v = workloads.large_request()
    dv = sess.upload(v)
    sort = sess.spawn("radix_sort_rows_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT), ka.arg(ka.KA_OUT)])
    enc = sess.spawn("wah_encode_sorted", [ka.arg(ka.KA_IN), ka.arg(ka.KA_IN)] + [ka.arg(ka.KA_OUT)] * 3)
    pipe = sess.compose(enc, sort)
    vin = sess.wrap(dv)
    outs = sess.request(pipe, ka.ref(vin), n_out=3)
    keys, offs, words = (sess.read(r) for r in outs)
    for r in outs:
        sess.release_ref(r)
    for a in (pipe, sort, enc):
        sess.release_actor(a)
    sess.release_ref(vin)
    ek, eo, ew = oracle.default().wah_index(v)
    np.testing.assert_array_equal(keys, ek)
    np.testing.assert_array_equal(offs, eo)
    np.testing.assert_array_equal(words, ew)


def test_large_zipf_request_wah_index_actor(sess):
    """The benchmark's configuration: the built-in wah_index actor with the
    16-bit hint (two passes over uint16 sort keys), device input, refs out."""
    v = workloads.large_request()
    dv = sess.upload(v)
    res = sess.wah_index(dv, refs=True, value_bits=16)
    got = tuple(sess.read(r) for r in (res.keys_ref, res.offsets_ref, res.words_ref))
    for r in (res.keys_ref, res.offsets_ref, res.words_ref):
        sess.release_ref(r)
    ek, eo, ew = oracle.default().wah_index(v)
    np.testing.assert_array_equal(got[0], ek)
    np.testing.assert_array_equal(got[1], eo)
    np.testing.assert_array_equal(got[2], ew)


def test_affine_chain_2p24(sess):
    import paper_1709_07781_amd as ka
    a, b = workloads.chain_params()
    x = workloads.chain_input(m=1 << 24)
    acts = [sess.affine_actor(int(a[i]), int(b[i])) for i in range(8)]
    chain = acts[0]
    comps = []
    for i in range(1, 8):
        chain = sess.compose(acts[i], chain)
        comps.append(chain)
    dv = sess.upload(x)
    vin = sess.wrap(dv)
    (r,) = sess.request(chain, ka.ref(vin), n_out=1)
    got = sess.read(r)
    sess.release_ref(r)
    sess.release_ref(vin)
    for c in comps + acts:
        sess.release_actor(c)
    np.testing.assert_array_equal(got, oracle.default().affine_chain(x, a, b))


def test_exclusive_scan_2p26(sess):
    import paper_1709_07781_amd as ka
    x = workloads.u32(7, (1 << 26) + 5)
    act = sess.spawn("exclusive_scan_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT)])
    dv = sess.upload(x)
    vin = sess.wrap(dv)
    (r,) = sess.request(act, ka.ref(vin), n_out=1)
    got = sess.read(r)
    sess.release_ref(r)
    sess.release_ref(vin)
    sess.release_actor(act)
    np.testing.assert_array_equal(got, oracle.default().exclusive_scan(x))


def test_sort_2p28_properties(sess):
    import paper_1709_07781_amd as ka
    n = (1 << 28) + 3
    k = workloads.u32(11, n) & np.uint32(0x00FFFFFF)  # 3 active passes, many equal keys
    act = sess.spawn("radix_sort_rows_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT), ka.arg(ka.KA_OUT)])
    dv = sess.upload(k)
    vin = sess.wrap(dv)
    outs = sess.request(act, ka.ref(vin), n_out=2)
    sk, sr = (sess.read(r) for r in outs)
    for r in outs:
        sess.release_ref(r)
    sess.release_ref(vin)
    sess.release_actor(act)
    del dv
    assert sk.size == n and sr.size == n
    assert np.all(sk[1:] >= sk[:-1])
    eq = sk[1:] == sk[:-1]
    assert np.all(sr[1:][eq] > sr[:-1][eq])  # stable: equal keys in row order
    assert np.array_equal(k[sr], sk)          # each output pair is an input pair
    seen = np.zeros(n, dtype=bool)
    seen[sr] = True
    assert seen.all()                          # rows are a permutation


@pytest.mark.parametrize("lg", [10, 14, 18, 22, 24])
def test_affine_chain_raw_launches(sess, lg):
    """The raw launch sequence of the actor-overhead comparison
    (ka_affine_chain_raw: 8 launches of the affine kernel, no actors) at the
    chain workload's sizes, against the oracle's chain."""
    import ctypes
    import torch
    import paper_1709_07781_amd as ka
    a, b = workloads.chain_params()
    ca = np.ascontiguousarray(a, dtype=np.uint32)
    cb = np.ascontiguousarray(b, dtype=np.uint32)
    x = workloads.chain_input(m=1 << lg)
    dv = sess.upload(x)
    torch.cuda.synchronize()
    ka.check(ka.lib.ka_affine_chain_raw(sess.sys, ctypes.c_void_p(dv.data_ptr()), x.size, ca.ctypes.data,
                                        cb.ctypes.data, 8))
    sess.synchronize()
    got = dv.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got, oracle.default().affine_chain(x, a, b))
