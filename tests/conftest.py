import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
    # Full-size parity runs the tiles that bench.py launches: start from the
    # same shipped autotuner choices (a copy, since the library appends to it).
    if "GCP_TILE_CACHE" not in os.environ:
        import shutil
        import tempfile
        src = os.path.join(ROOT, "paper_2208_05740_amd", "tuned_tiles_gfx950.txt")
        if os.path.exists(src):
            fd, dst = tempfile.mkstemp(prefix="gcp_tiles_test_", suffix=".txt")
            os.close(fd)
            shutil.copyfile(src, dst)
            os.environ["GCP_TILE_CACHE"] = dst


def pytest_collection_modifyitems(config, items):
    # GPU tests need a device; skip them cleanly on CPU-only machines.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
