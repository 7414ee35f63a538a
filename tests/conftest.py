"""Shared pytest configuration.

Markers
-------
gpu   needs an MI355X (gfx950) and the built HIP library; these are the parity
      tests proper and always call through the C ABI.
slow  CPU tests that take more than a few seconds (still part of the default run).
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def pytest_collection_modifyitems(config, items):
    # GPU tests run only when a GPU is actually present; on a CPU-only host they
    # are skipped (the CPU suite is selected with -m "not gpu" anyway).
    have_gpu = None
    for item in items:
        if "gpu" in item.keywords:
            if have_gpu is None:
                try:
                    import torch
                    have_gpu = bool(torch.cuda.is_available())
                except Exception:  # pragma: no cover
                    have_gpu = False
            if not have_gpu:
                item.add_marker(pytest.mark.skip(reason="no GPU on this host"))
