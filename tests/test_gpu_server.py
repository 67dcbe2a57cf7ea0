"""GPU tests of the served form (ka_server_*): a mix of index, scan and
affine-chain requests submitted together is batched, and every result equals
both the oracle's and the result of the same request served alone (a server
with batching off), bit for bit.  Inputs: workloads.served_requests /
served_payload (the served mix) at sizes small enough for the oracle."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sess():
    from paper_1709_07781_amd.session import Session
    s = Session(n_streams=4)
    yield s
    s.close()


def _chain():
    return workloads.chain_params()


def _expected(ora, kind, x, a, b):
    if kind == workloads.KIND_WAH:
        return ora.wah_index(x)
    if kind == workloads.KIND_SCAN:
        return (ora.exclusive_scan(x),)
    return (ora.affine_chain(x, a, b),)


def _results(srv, req, kind):
    return tuple(srv.result(req, i) for i in range(3 if kind == workloads.KIND_WAH else 1))


def _mix(count, seed, lo=4, hi=14):
    _, sizes, kinds, dseeds = workloads.served_requests(seed=seed, count=count, lo_log2=lo, hi_log2=hi)
    return [(int(k), workloads.served_payload(int(k), int(s), int(d))) for k, s, d in zip(kinds, sizes, dseeds)]


def test_mix_equals_alone_and_oracle(sess):
    from paper_1709_07781_amd.session import Server
    a, b = _chain()
    ora = oracle.default()
    reqs = _mix(120, seed=61)
    reqs += [(workloads.KIND_WAH, np.zeros(0, np.uint32)), (workloads.KIND_SCAN, np.zeros(0, np.uint32)),
             (workloads.KIND_CHAIN, np.zeros(0, np.uint32)), (workloads.KIND_WAH, np.array([4095], np.uint32))]
    mixed = Server(sess, streams=3, max_batch=64, chain_a=a, chain_b=b)
    alone = Server(sess, streams=1, max_batch=1, chain_a=a, chain_b=b)
    try:
        hm = [mixed.submit(k, x) for k, x in reqs]  # all queued at once: batched
        for k, x in reqs:  # the same requests one at a time
            h = alone.submit(k, x)
            assert alone.wait(h) == 0
            r_alone = _results(alone, h, k)
            alone.release(h)
            exp = _expected(ora, k, x, a, b)
            for got, e in zip(r_alone, exp):
                np.testing.assert_array_equal(got, e)
        for (k, x), h in zip(reqs, hm):
            assert mixed.wait(h) == 0
            got = _results(mixed, h, k)
            mixed.release(h)
            for g, e in zip(got, _expected(ora, k, x, a, b)):
                np.testing.assert_array_equal(g, e)
        st = mixed.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["mean_batch"] > 1.0  # requests were merged
        assert 0 < st["p50_us"] <= st["p99_us"] <= st["max_us"]
        assert alone.stats()["mean_batch"] == 1.0
    finally:
        mixed.close()
        alone.close()


def test_budget_admission_and_rejection(sess):
    """A budget that holds about one request at a time still serves them all;
    a request larger than the budget is refused at submission."""
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import Server
    a, b = _chain()
    srv = Server(sess, streams=2, max_batch=32, budget_bytes=48 * 20_000, chain_a=a, chain_b=b)
    ora = oracle.default()
    try:
        reqs = [(workloads.KIND_WAH, workloads.uniform_values(70 + i, 15_000, 4096)) for i in range(6)]
        hs = [srv.submit(k, x) for k, x in reqs]
        for (k, x), h in zip(reqs, hs):
            assert srv.wait(h) == 0
            got = _results(srv, h, k)
            srv.release(h)
            for g, e in zip(got, ora.wah_index(x)):
                np.testing.assert_array_equal(g, e)
        st = srv.stats()
        assert st["budget_peak"] <= 48 * 20_000 and st["mean_batch"] <= 1.5
        with pytest.raises(ka.KaError) as e:
            srv.submit(workloads.KIND_WAH, workloads.uniform_values(79, 30_000, 4096))
        assert e.value.code == ka.KA_E_BUDGET
    finally:
        srv.close()


def test_value_bits_checked_at_submit(sess):
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import Server
    srv = Server(sess)
    try:
        with pytest.raises(ka.KaError) as e:
            srv.submit(workloads.KIND_WAH, np.array([1, 2, 4096], np.uint32))
        assert e.value.code == ka.KA_E_ARG
    finally:
        srv.close()


@pytest.mark.parametrize("copy_threads", [1, 0, 8])
def test_large_payload_copied_and_checked_in_chunks(sess, copy_threads):
    """A payload of 1 MiB or more is copied in 2^16-value chunks by several
    threads, its values checked in the same pass: a value at or above
    2^value_bits in the first chunk, at a chunk edge or in the ragged last
    chunk fails the submission; valid payloads of the same size give the
    oracle's index (1 copy thread: the submitting thread copies alone)."""
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import Server
    chunk = 1 << 16
    n = 3 * chunk + 5
    ora = oracle.default()
    srv = Server(sess, copy_threads=copy_threads)
    try:
        for pos in (0, chunk - 1, chunk, 2 * chunk + 1, n - 1):
            x = workloads.uniform_values(70 + pos % 7, n, 4096)
            x[pos] = 4096 + pos
            with pytest.raises(ka.KaError) as e:
                srv.submit(workloads.KIND_WAH, x)
            assert e.value.code == ka.KA_E_ARG, f"bad value at {pos}"
        xs = [workloads.uniform_values(80 + i, n + i * 977, 4096) for i in range(3)]
        hs = [srv.submit(workloads.KIND_WAH, x) for x in xs]
        for x, h in zip(xs, hs):
            assert srv.wait(h) == 0
            for g, e in zip(_results(srv, h, workloads.KIND_WAH), ora.wah_index(x)):
                np.testing.assert_array_equal(g, e)
            srv.release(h)
        y = workloads.u32(90, n)
        h = srv.submit(workloads.KIND_SCAN, y)
        assert srv.wait(h) == 0
        np.testing.assert_array_equal(srv.result(h, 0), ora.exclusive_scan(y))
        srv.release(h)
    finally:
        srv.close()


def test_destroy_cancels_or_finishes_everything(sess):
    """Destroying a server with a full mailbox ends every request: finished
    (with the right result) or cancelled."""
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd import lib
    from paper_1709_07781_amd.session import Server
    a, b = _chain()
    srv = Server(sess, streams=1, max_batch=2, chain_a=a, chain_b=b)
    reqs = [(workloads.KIND_SCAN, workloads.u32(90 + i, 50_000)) for i in range(40)]
    hs = [srv.submit(k, x) for k, x in reqs]
    srv.close()
    ora = oracle.default()
    done = 0
    for (k, x), h in zip(reqs, hs):
        rc = lib.ka_server_wait(h, 10_000_000)
        assert rc in (0, ka.KA_E_CANCELLED)
        if rc == 0:
            np.testing.assert_array_equal(srv.result(h, 0), ora.exclusive_scan(x))
            done += 1
        lib.ka_server_request_release(h)
    assert done >= 1


def test_served_mix_at_full_sizes(sess):
    """The served configuration's sizes (log-uniform in [2^8, 2^22]) under its
    16 MiB batch limit: 40 requests of the mix, one index request of 2^22
    values (16 MiB: a batch of its own), and three index requests whose inputs
    add up to 4 bytes under 16 MiB (one batch filled to the limit), all queued
    at once.  Every result equals the oracle's and the one the same request
    gets from a server that runs one request at a time."""
    import concurrent.futures as cf
    from parallel_oracle import host_threads
    from paper_1709_07781_amd.session import Server
    a, b = _chain()
    ora = oracle.default()
    reqs = _mix(40, seed=62, lo=8, hi=22)
    reqs.append((workloads.KIND_WAH, workloads.uniform_values(63, 1 << 22, 4096)))
    third = (16 << 20) // 4 // 3
    reqs += [(workloads.KIND_WAH, workloads.uniform_values(64 + i, third, 4096)) for i in range(3)]
    assert sum(x.size for _, x in reqs[-3:]) * 4 == (16 << 20) - 4
    with cf.ThreadPoolExecutor(max_workers=host_threads()) as ex:
        exp = list(ex.map(lambda kx: _expected(ora, kx[0], kx[1], a, b), reqs))
    mixed = Server(sess, streams=2, max_batch=1024, max_batch_bytes=16 << 20, chain_a=a, chain_b=b)
    alone = Server(sess, streams=1, max_batch=1, chain_a=a, chain_b=b)
    try:
        hm = [mixed.submit(k, x) for k, x in reqs]
        for (k, x), e in zip(reqs, exp):
            h = alone.submit(k, x)
            assert alone.wait(h) == 0
            for g, ee in zip(_results(alone, h, k), e):
                np.testing.assert_array_equal(g, ee, err_msg=f"alone: kind {k}, n={x.size}")
            alone.release(h)
        for (k, x), h, e in zip(reqs, hm, exp):
            assert mixed.wait(h) == 0
            for g, ee in zip(_results(mixed, h, k), e):
                np.testing.assert_array_equal(g, ee, err_msg=f"mixed: kind {k}, n={x.size}")
            mixed.release(h)
        st = mixed.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["mean_batch"] > 1.0
    finally:
        mixed.close()
        alone.close()


def test_send_values_and_refs_through_tickets(sess):
    """ka_server_send: host values and device references in, host values or
    device references out through tickets (ka_receive); every result equals
    the oracle's, batched with the others, in either form."""
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import Server
    a, b = _chain()
    ora = oracle.default()
    reqs = _mix(60, seed=71, lo=4, hi=15)
    reqs += [(workloads.KIND_WAH, np.zeros(0, np.uint32)), (workloads.KIND_CHAIN, np.zeros(0, np.uint32))]
    srv = Server(sess, streams=2, max_batch=32, chain_a=a, chain_b=b)
    held = []
    try:
        tickets = []
        for i, (k, x) in enumerate(reqs):
            dev_in = i % 2 == 1 and x.size > 0
            data = sess.upload(x) if dev_in else x
            if dev_in:
                r = sess.wrap(data)
                held.append((r, data))
                data = r
            tickets.append((srv.send(k, data, refs=(i % 3 == 0)), i % 3 == 0))
        for (k, x), (t, refs) in zip(reqs, tickets):
            n_out = 3 if k == workloads.KIND_WAH else 1
            got = sess.receive(t, n_out)
            if refs:
                arrs = []
                for r in got:
                    arrs.append(sess.read(r))
                    sess.release_ref(r)
                got = arrs
            sess.release_ticket(t)
            for g, e in zip(got, _expected(ora, k, x, a, b)):
                np.testing.assert_array_equal(g, e, err_msg=f"kind={k} n={x.size} refs={refs}")
    finally:
        srv.close()
        for r, _ in held:
            sess.release_ref(r)


@pytest.mark.parametrize("base", [300, 3000])  # the one-work-group path, the tagged sort
def test_send_device_value_beyond_bits_fails_alone(sess, base):
    """A device-resident index request holding a value at or above
    2^value_bits fails at ka_receive with KA_E_ARG; the requests batched with
    it are unaffected."""
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import Server
    ora = oracle.default()
    good = [workloads.served_payload(workloads.KIND_WAH, base + base // 6 * i, 90 + i) for i in range(6)]
    bad = good[2].copy()
    bad[17] = 1 << 12
    bad_dev = sess.upload(bad)
    rbad = sess.wrap(bad_dev)
    srv = Server(sess, streams=1, max_batch=16)
    try:
        ts = [srv.send(workloads.KIND_WAH, g) for g in good[:3]]
        tb = srv.send(workloads.KIND_WAH, rbad)
        ts += [srv.send(workloads.KIND_WAH, g) for g in good[3:]]
        with pytest.raises(ka.KaError) as e:
            sess.receive(tb, 3)
        assert e.value.code == ka.KA_E_ARG
        sess.release_ticket(tb)
        for g, t in zip(good, ts):
            got = sess.receive(t, 3)
            sess.release_ticket(t)
            for x, y in zip(got, ora.wah_index(g)):
                np.testing.assert_array_equal(x, y)
    finally:
        srv.close()
        sess.release_ref(rbad)


@pytest.mark.parametrize("stages", [1, 16, 17, 40])
def test_long_chains_in_one_pass(sess, stages):
    """Chain requests run as one fused pass per 16 stages: chains of 1, 16, 17
    and 40 stages over a batch of uneven requests equal the oracle's chain."""
    from paper_1709_07781_amd.session import Server
    a, b = workloads.chain_params(seed=9, stages=stages)
    ora = oracle.default()
    xs = [workloads.u32(900 + i, n) for i, n in enumerate([0, 1, 5, 4096, 4099, 100_003])]
    srv = Server(sess, streams=2, max_batch=64, chain_a=a, chain_b=b)
    try:
        hs = [srv.submit(workloads.KIND_CHAIN, x) for x in xs]
        for x, h in zip(xs, hs):
            assert srv.wait(h) == 0
            np.testing.assert_array_equal(srv.result(h, 0), ora.affine_chain(x, a, b), err_msg=f"n={x.size}")
            srv.release(h)
    finally:
        srv.close()
