"""GPU tests of batch plans (ka_batch_plan_*): the batched index build
recorded into a HIP graph and replayed.  Every replay is checked against the
oracle and against the eager batched build (ka_wah_batch) of the same values,
with the program's own eager work and synchronisations between replays."""
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


def _same(a, b):
    assert len(a) == len(b)
    for (k1, o1, w1), (k2, o2, w2) in zip(a, b):
        np.testing.assert_array_equal(k1, k2)
        np.testing.assert_array_equal(o1, o2)
        np.testing.assert_array_equal(w1, w2)


def _oracle(off, v):
    o = oracle.default()
    return [o.wah_index(v[off[j]:off[j + 1]]) for j in range(len(off) - 1)]


def test_plan_replays_match_eager_and_oracle(sess):
    import torch
    from paper_1709_07781_amd.session import BatchPlan
    off, v1 = workloads.batched_requests(seed=81, count=50, lo_log2=0, hi_log2=13)
    n = int(off[-1])
    v2 = workloads.uniform_values(82, n, 1 << 12)
    v3 = workloads.structured("alternating_chunks", n, seed=83) & np.uint32(0xFFF)
    plan = BatchPlan(sess, off, 12)
    try:
        for rep, v in enumerate([v1, v2, v1, v3, v2, v1]):
            plan.run(v)
            got = plan.result()
            # eager work between replays: the same batch without the graph, a torch op, a sync
            eager = sess.wah_batch(v, off, 12)
            t = torch.arange(1000, device="cuda").sum().item()
            assert t == 499500
            torch.cuda.synchronize()
            _same(got, eager)
            _same(got, _oracle(off, v))
    finally:
        plan.close()


def test_plan_device_input_and_prefilled_buffer(sess):
    import torch
    from paper_1709_07781_amd.session import BatchPlan
    sizes = [0, 1, 31, 0, 4097, 5000, 0]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    v = workloads.uniform_values(91, int(off[-1]), 1 << 10)
    plan = BatchPlan(sess, off, 10)
    try:
        dv = torch.from_numpy(v.view(np.int32)).to("cuda")
        for _ in range(3):
            plan.run(dv)  # device-to-device copy into the plan's input, then the graph
            _same(plan.result(), _oracle(off, v))
        assert plan.input_ptr() != 0
        for _ in range(2):
            plan.run(None)  # the input buffer still holds v
            _same(plan.result(), _oracle(off, v))
    finally:
        plan.close()


def test_plan_rejects_out_of_range_values(sess):
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import BatchPlan
    off = np.array([0, 100, 300], dtype=np.uint32)
    v = workloads.uniform_values(95, 300, 1 << 8)
    plan = BatchPlan(sess, off, 8)
    try:
        v[150] = 256
        plan.run(v)
        with pytest.raises(ka.KaError) as e:
            plan.result()
        assert e.value.code == ka.KA_E_ARG
        v[150] = 255  # the next replay is fine again
        plan.run(v)
        _same(plan.result(), _oracle(off, v))
    finally:
        plan.close()


def test_plan_argument_errors(sess):
    import ctypes
    import paper_1709_07781_amd as ka
    p = ctypes.c_void_p()
    for off, nreq, vb in [([0, 5, 3], 2, 8), ([1, 5], 1, 8), ([0, 5, 10, 12, 20], 4, 31), ([0, 4], 1, 0)]:
        a = np.array(off, dtype=np.uint32)
        assert ka.lib.ka_batch_plan_create(sess.sys, a.ctypes.data, nreq, vb, 0, ctypes.byref(p)) == ka.KA_E_ARG


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
def test_each_tile_shape_matches_oracle(sess, shape):
    """Every sort tile shape the autotuner chooses from gives the same, correct
    result (sizes span several tiles of each shape and ragged ends)."""
    from paper_1709_07781_amd.session import BatchPlan
    off, v = workloads.batched_requests(seed=100 + shape, count=40, lo_log2=8, hi_log2=15)
    plan = BatchPlan(sess, off, 12, shape=shape)
    try:
        assert plan.shape()[0] == shape
        for _ in range(2):
            plan.run(v)
            _same(plan.result(), _oracle(off, v))
    finally:
        plan.close()


def test_autotuned_plan(sess):
    from paper_1709_07781_amd.session import BatchPlan
    off, v = workloads.batched_requests(seed=110, count=64, lo_log2=10, hi_log2=16)
    plan = BatchPlan(sess, off, 12, autotune=True)
    try:
        assert plan.shape()[0] == -1
        plan.run(v)  # times every shape
        chosen, ms = plan.shape()
        assert chosen in (0, 1, 2, 3) and all(t > 0 for t in ms[:4]) and ms[chosen] == min(ms[:4])
        _same(plan.result(), _oracle(off, v))
        v2 = workloads.uniform_values(111, int(off[-1]), 1 << 12)
        plan.run(v2)
        assert plan.shape()[0] == chosen
        _same(plan.result(), _oracle(off, v2))
    finally:
        plan.close()



# ---- plans for any batch -----------------------------------------------------------------
def _batches(seed, cap_values, cap_requests, bits, lo, hi):
    """A sequence of different batches within the capacities: varied request
    counts and sizes, an empty batch, a batch of empty requests, and one filling
    both capacities exactly (last request takes the remaining values)."""
    out = []
    for i, count in enumerate([cap_requests // 3, 1, cap_requests, 7, cap_requests // 2]):
        off, v = workloads.batched_requests(seed=seed + i, count=max(count, 1), lo_log2=lo, hi_log2=hi,
                                            bound=1 << bits, max_total=cap_values)
        out.append((off, v))
    out.append((np.zeros(1, np.int64), np.zeros(0, np.uint32)))               # no requests
    out.append((np.zeros(4, np.int64), np.zeros(0, np.uint32)))               # three empty requests
    sizes = np.full(cap_requests, cap_values // cap_requests, np.int64)
    sizes[-1] += cap_values - sizes.sum()
    off = np.zeros(cap_requests + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    out.append((off, workloads.uniform_values(seed + 99, cap_values, 1 << bits)))  # both capacities full
    return out


@pytest.mark.parametrize("bits,shape", [(12, 0), (12, 1), (20, 0), (16, 2)])
def test_any_batch_plan_serves_every_batch(sess, bits, shape):
    """One recorded graph serves a sequence of different batches (request
    counts, sizes, empty batches, both capacities full): every result equals
    the oracle's, with eager work between the runs."""
    import torch
    from paper_1709_07781_amd.session import BatchPlan
    cap_values, cap_requests = 3 * 8192 * 8 + 5, 96
    plan = BatchPlan(sess, None, bits, shape=shape, any_batch=(cap_values, cap_requests, 0))
    try:
        for off, v in _batches(200 + bits, cap_values, cap_requests, bits, 4, 14):
            plan.run_batch(v, off)
            got = plan.result()
            assert torch.arange(100, device="cuda").sum().item() == 4950
            _same(got, _oracle(off, v))
            plan.run(v)  # the same batch again through ka_batch_plan_run
            _same(plan.result(), _oracle(off, v))
    finally:
        plan.close()


def test_any_batch_plan_small_requests_and_device_input(sess):
    """Requests bounded by 1024 values take the one-work-group-per-request
    path; values from a device tensor; autotuning on the first batch."""
    import torch
    from paper_1709_07781_amd.session import BatchPlan
    cap_values, cap_requests = 300_000, 1024
    plan = BatchPlan(sess, None, 12, autotune=True, any_batch=(cap_values, cap_requests, 1024))
    try:
        for i, count in enumerate([1024, 10, 500]):
            off, v = workloads.batched_requests(seed=300 + i, count=count, lo_log2=0, hi_log2=10)
            dv = torch.from_numpy(v.view(np.int32)).to("cuda")
            torch.cuda.synchronize()
            plan.run_batch(dv, off)
            _same(plan.result(), _oracle(off, v))  # waits for the plan's stream
            del dv
    finally:
        plan.close()


def test_any_batch_plan_rejections_and_errors(sess):
    import ctypes
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import BatchPlan
    plan = BatchPlan(sess, None, 8, any_batch=(10_000, 8, 2000))
    fixed = BatchPlan(sess, np.array([0, 10], np.uint32), 8)
    try:
        off = np.array([0, 100, 300], np.uint32)
        v = workloads.uniform_values(95, 300, 1 << 8)
        v[150] = 256
        plan.run_batch(v, off)
        with pytest.raises(ka.KaError) as e:
            plan.result()
        assert e.value.code == ka.KA_E_ARG
        v[150] = 3
        plan.run_batch(v, off)
        _same(plan.result(), _oracle(off, v))
        bad = [np.arange(10, dtype=np.uint32) * 1000,                # 9 requests > 8
               np.array([0, 2001], np.uint32),                        # a request above 2000 values
               np.array([0, 2000, 4000, 6000, 8000, 10000, 10001], np.uint32),  # more than 10000 values
               np.array([0, 5, 3], np.uint32), np.array([1, 5], np.uint32)]
        for o in bad:
            x = np.zeros(int(o.max()), np.uint32)
            with pytest.raises(ka.KaError) as e:
                plan.run_batch(x, o)
            assert e.value.code == ka.KA_E_ARG
        with pytest.raises(ka.KaError) as e:
            fixed.run_batch(np.zeros(10, np.uint32), np.array([0, 10], np.uint32))
        assert e.value.code == ka.KA_E_STATE
        p = ctypes.c_void_p()
        assert ka.lib.ka_batch_plan_create_any(sess.sys, 100, 0, 0, 8, 0, ctypes.byref(p)) == ka.KA_E_ARG
        assert ka.lib.ka_batch_plan_create_any(sess.sys, 100, 1 << 20, 0, 16, 0, ctypes.byref(p)) == ka.KA_E_ARG
    finally:
        plan.close()
        fixed.close()
