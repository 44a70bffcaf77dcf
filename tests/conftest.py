import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_sessionstart(session):
    """Build the HIP library once, before collection, when it is missing or
    stale (a fresh checkout has none).  A failed build is reported here; the
    tests that load the library then fail on their own, the oracle tests still
    run."""
    try:
        # build.py by path: importing the package here would load the library
        # before the tests import torch
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "_afqmc_build", os.path.join(ROOT, "paper_1804_03310_amd", "build.py"))
        _build = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(_build)
        _build.ensure_built()
    except Exception as e:  # no hipcc, compile error
        print(f"[conftest] libafqmc.so not built: {e}", file=sys.stderr, flush=True)
