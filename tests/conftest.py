import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

# Tests load the libraries that are built; they build them only when none exists.
if not (os.path.exists(os.path.join(ROOT, "paper_2403_16438_amd", "libseg.so"))
        and os.path.exists(os.path.join(ROOT, "synth", "libsynth.so"))):
    sys.path.insert(0, ROOT)
    import __graft_entry__
    __graft_entry__.build()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")
