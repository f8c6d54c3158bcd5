import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests must not silently run without a GPU: skip them only when no GPU is present.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session", autouse=True)
def _built_libs():
    # The oracle and the generator are plain C libraries; build them if absent.
    from oracle import oracle as O
    O.build(force=False)
    gen = os.path.join(ROOT, "paper_1402_4466_amd", "datagen", "libewahgen.so")
    if not os.path.exists(gen):
        import subprocess
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", gen,
                               os.path.join(ROOT, "paper_1402_4466_amd", "datagen", "ewahgen.c"), "-lm"])
    yield
