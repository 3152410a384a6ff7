import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (HIP device) and the built library")


def _ensure_built():
    lib = os.path.join(ROOT, "paper_2503_11213_amd", "libsdirt.so")
    if not os.path.exists(lib):
        from paper_2503_11213_amd import build
        build.build()


_ensure_built()
