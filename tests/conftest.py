import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle.build(force=False)
    return oracle


def rel_err_max(y, ref):
    """max_i |y_i - ref_i| / max_i |ref_i| over complex components (infinity-norm relative error)."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(y - ref)) / den) if den > 0 else float(np.max(np.abs(y)))


def rel_err_2(y, ref):
    """|y - ref|_2 / |ref|_2."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    return float(np.linalg.norm((y - ref).ravel()) / np.linalg.norm(ref.ravel()))
