"""GPU test of the allocation-free index build (ka_wah_index_noalloc) through
the C ABI: its keys, offsets and words equal those of ka_wah_index (the entry
point it is a variant of) and the oracle's, bit for bit, on two calls in a row
with the second input smaller than the first (the static scratch keeps the
first call's contents); sizes beyond the static limit are refused."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _noalloc(ka, torch, v):
    n = v.size
    dv = torch.from_numpy(np.ascontiguousarray(v).view(np.int32)).to("cuda")
    keys = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    offs = torch.full((n + 1,), -1, dtype=torch.int32, device="cuda")
    words = torch.full((max(2 * n, 1),), -1, dtype=torch.int32, device="cuda")
    lens = torch.full((3,), -1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    ka.check(ka.lib.ka_wah_index_noalloc(ctypes.c_void_p(dv.data_ptr()), n, ctypes.c_void_p(keys.data_ptr()),
                                         ctypes.c_void_p(offs.data_ptr()), ctypes.c_void_p(words.data_ptr()),
                                         ctypes.c_void_p(lens.data_ptr()), ctypes.c_void_p(stream.cuda_stream)),
             "ka_wah_index_noalloc")
    torch.cuda.synchronize()
    D, D1, W = (int(x) for x in lens.cpu().numpy())
    assert D1 == D + 1
    return (keys.cpu().numpy().view(np.uint32)[:D], offs.cpu().numpy().view(np.uint32)[:D + 1],
            words.cpu().numpy().view(np.uint32)[:W])


@pytest.mark.parametrize("sizes", [((1 << 22), (1 << 16) + 7), (100_003, 31), (4097, 0)])
def test_noalloc_two_calls_match_ka_wah_index(sizes):
    import torch
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import Session
    torch.cuda.set_device(0)
    s = Session()
    try:
        for i, n in enumerate(sizes):
            v = (workloads.large_request(seed=70 + i, n=n) if n >= (1 << 20)
                 else workloads.plain_request(seed=70 + i, n=n, bound=4096))
            got = _noalloc(ka, torch, v)
            exp = s.wah_index(v)
            ora = oracle.default().wah_index(v)
            for g, e, o, what in zip(got, exp, ora, ("keys", "offsets", "words")):
                np.testing.assert_array_equal(g, e, err_msg=f"call {i} (n={n}): {what} vs ka_wah_index")
                np.testing.assert_array_equal(g, o, err_msg=f"call {i} (n={n}): {what} vs the oracle")
    finally:
        s.close()


def test_noalloc_refuses_sizes_beyond_the_limit():
    import torch
    import paper_1709_07781_amd as ka
    torch.cuda.set_device(0)
    n = (1 << 22) + 1
    buf = torch.zeros(8, dtype=torch.int64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    rc = ka.lib.ka_wah_index_noalloc(p, n, p, p, p, p, None)
    assert rc == ka.KA_E_ARG
    assert b"KA_NOALLOC_MAX_N" in ka.lib.ka_last_error()
