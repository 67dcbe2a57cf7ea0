"""Oracle calls over many independent requests, run on several host threads.

The oracle is a C library called through ctypes, which releases the GIL for
the duration of each call, so a thread pool runs requests in parallel without
starting processes.  Test infrastructure only."""
from __future__ import annotations

import concurrent.futures as cf
import os

import oracle


def host_threads(limit: int = 16) -> int:
    """Threads to use: the CPUs this process may run on, at most `limit`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(limit, n))


def map_requests(fn_name: str, inputs, threads: int | None = None):
    """[getattr(oracle, fn_name)(x) for x in inputs], computed on a thread pool,
    in input order."""
    ora = oracle.default()
    fn = getattr(ora, fn_name)
    with cf.ThreadPoolExecutor(max_workers=threads or host_threads()) as ex:
        return list(ex.map(fn, inputs))
