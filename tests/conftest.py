import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_collection_modifyitems(config, items):
    # GPU tests run last so that a GPU failure cannot hide the CPU results.
    items.sort(key=lambda it: 1 if it.get_closest_marker("gpu") else 0)


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library binding; GPU tests fail loudly if it is not built."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    from paper_2208_04448_amd import nvdb
    return nvdb


@pytest.fixture(scope="session")
def record():
    """record(name, **values): appends measured errors of a test as one JSON line to
    $NVDB_RECORD (if set), so that tolerances can be set from observed values."""
    import json
    path = os.environ.get("NVDB_RECORD")

    def _rec(name, **vals):
        if path:
            with open(path, "a") as f:
                f.write(json.dumps(dict(test=name, **{k: float(v) for k, v in vals.items()})) + "\n")
    return _rec
