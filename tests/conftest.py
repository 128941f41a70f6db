import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def hip_lib():
    """The HIP library through its Python binding; fails loudly if not built."""
    import paper_1607_00909_amd as cdmt
    cdmt.load()
    return cdmt


def allow_short_overlap(plan, dms) -> bool:
    """Parity tests also cover DM trials whose Eq. 2 sweep is longer than the
    plan's overlap: the method is then a circular convolution with
    wrap-around in the kept samples, which the oracle computes the same way.
    The library rejects such DMs by default (CDMT_OPT_DM_CHECK); turn the
    check off for this plan only when the test's DMs need it.  Returns
    whether it did."""
    import paper_1607_00909_amd as cdmt
    if max(abs(float(d)) for d in dms) <= plan.dm_limit():
        return False
    cdmt.cdmt_plan_set(plan.handle, cdmt.CDMT_OPT_DM_CHECK, 0)
    return True
