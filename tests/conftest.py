import os
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running oracle check")


# ---------------------------------------------------------------------------
# Oracle references that take minutes on one core (full-size parity cases)
# are started in background threads as soon as collection ends, so they run
# on the host while the GPU tests before them execute.  The oracle's ctypes
# calls release the GIL, so the threads really run in parallel.  A test
# module lists its references in a module-level dict BACKGROUND_REFS
# {name: zero-argument callable}; only references of selected tests start.
# Names in a module's BACKGROUND_LONG (the longest jobs) are submitted first.
# ---------------------------------------------------------------------------
_pool = None
_futures = {}


def _workers():
    n = os.cpu_count() or 4
    return max(1, min(15, n - 1))


@pytest.hookimpl(trylast=True)
def pytest_collection_modifyitems(session, config, items):
    global _pool
    mods = {}
    for it in items:
        mod = getattr(it, "module", None)
        refs = getattr(mod, "BACKGROUND_REFS", None)
        if refs and it.get_closest_marker("gpu") is not None:
            mods[mod.__name__] = (refs, getattr(mod, "BACKGROUND_LONG", ()))
    if not mods:
        return
    try:
        import torch
        if not torch.cuda.is_available():
            return
    except Exception:
        return
    _pool = ThreadPoolExecutor(max_workers=_workers())
    jobs = [(name, fn, name in long) for refs, long in mods.values() for name, fn in refs.items()]
    for name, fn, _ in sorted(jobs, key=lambda j: not j[2]):
        if name not in _futures:
            _futures[name] = _pool.submit(fn)


def background_ref(name, fn):
    """Result of the background reference `name` (computed now with fn if it
    was not started at collection)."""
    f = _futures.get(name)
    return f.result() if f is not None else fn()


def pytest_sessionfinish(session, exitstatus):
    if _pool is not None:
        _pool.shutdown(wait=False, cancel_futures=True)
