import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-only oracle runs")


def _lib_built():
    return os.path.exists(os.path.join(ROOT, "paper_1909_07439_amd", "libsph.so"))


def pytest_collection_modifyitems(config, items):
    import pytest

    gpu_items = [it for it in items if "gpu" in it.keywords]
    if not gpu_items:
        return
    try:
        import torch

        ok = torch.cuda.is_available()
    except Exception:
        ok = False
    if not ok:
        skip = pytest.mark.skip(reason="no GPU visible")
        for it in gpu_items:
            it.add_marker(skip)
