import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


_CONFIG = None


def pytest_configure(config):
    global _CONFIG
    _CONFIG = config
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large CPU-side case")


def say(*a):
    """A progress line straight to the terminal, past pytest's output capture,
    so that a long GPU test (the full-size meshes take minutes to generate,
    load and compare) shows that it is still running."""
    capman = _CONFIG.pluginmanager.getplugin("capturemanager") if _CONFIG is not None else None
    if capman is not None:
        with capman.global_and_fixture_disabled():
            print(*a, flush=True)
    else:
        print(*a, flush=True)
