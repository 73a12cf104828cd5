import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle():
    from oracle import build as obuild
    from oracle import oracle as O
    src = os.path.join(ROOT, "oracle", "ode_oracle.c")
    if any(not os.path.exists(f) or os.path.getmtime(f) < os.path.getmtime(src)
           for f in (O.LIB_PATH, O.LIB_FMA_PATH)):
        obuild.build()
    O.lib()
    O.lib("fma")
    return O


@pytest.fixture(scope="session")
def ode():
    """The HIP library binding on cuda:0 (GPU tests only)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_03931_amd import ensemble
    ensemble.load_library()
    return ensemble
