import json
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def load_golden(name):
    """Golden fixtures store +-inf and NaN as strings."""
    def fix(v):
        if isinstance(v, list):
            return [fix(x) for x in v]
        if isinstance(v, str) and v in ("inf", "-inf", "nan"):
            return float(v)
        return v
    with open(os.path.join(GOLDEN, name)) as f:
        d = json.load(f)
    return {k: fix(v) for k, v in d.items()}


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle


def has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
