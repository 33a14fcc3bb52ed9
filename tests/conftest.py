import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)

_POOL = None
_FUTURES = {}


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (runs the HIP library through the C ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")
    config.addinivalue_line(
        "markers", "oracle_jobs(*names): oracle histories (tests/oracle_jobs.py) "
        "the test compares against; they start in worker processes when "
        "collection ends")


def _pool():
    global _POOL
    import concurrent.futures as cf
    import multiprocessing as mp
    import oracle_jobs
    if _POOL is None:
        _POOL = cf.ProcessPoolExecutor(
            max_workers=oracle_jobs.WORKERS,
            mp_context=mp.get_context("spawn"),
            initializer=oracle_jobs.worker_init)
    return _POOL


def _submit(names):
    import oracle_jobs
    order = list(oracle_jobs.JOBS)
    todo = sorted((n for n in set(names) if n not in _FUTURES), key=order.index)
    if not todo:
        return
    _pool()
    for n in todo:
        _FUTURES[n] = _POOL.submit(oracle_jobs.run, n)


def pytest_collection_finish(session):
    names = []
    for item in session.items:
        m = item.get_closest_marker("oracle_jobs")
        if m is not None:
            names.extend(a for a in m.args if a not in names)
    if names:
        _submit(names)


def pytest_sessionfinish(session, exitstatus):
    # oracle runs still going (a test failed early) are not waited for
    if _POOL is not None:
        procs = list(getattr(_POOL, "_processes", {}).values())
        _POOL.shutdown(wait=False, cancel_futures=True)
        for p in procs:
            if p.is_alive():
                p.terminate()


@pytest.fixture(scope="session")
def oracle_map():
    """oracle_map(fn, items) -> [fn(x) for x in items], in the worker
    processes (fn: a module-level function of tests/oracle_jobs.py)."""
    def pmap(fn, items):
        return list(_pool().map(fn, items))
    return pmap


@pytest.fixture(scope="session")
def oracle_run():
    """oracle_run(name) -> the result of tests/oracle_jobs.py job `name`."""
    def get(name):
        _submit([name])
        return _FUTURES[name].result()
    return get
