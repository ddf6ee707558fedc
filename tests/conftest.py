import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def gpu_available() -> bool:
    # counting devices does not initialise the GPU runtime in this process,
    # so background processes can still be started after this check
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


def pytest_collection_finish(session):
    """Start the background oracle runs of the full-length GPU tests as soon
    as they are collected on a machine with a GPU, so that they overlap the
    GPU tests that run before them."""
    if not any(item.nodeid.startswith("tests/test_gpu_full_length.py") and "gpu" in item.keywords
               for item in session.items):
        return
    if not gpu_available():
        return
    from tests import full_length_jobs
    full_length_jobs.start()


def pytest_sessionfinish(session, exitstatus):
    import sys
    mod = sys.modules.get("tests.full_length_jobs")
    if mod is not None:
        mod.stop()
