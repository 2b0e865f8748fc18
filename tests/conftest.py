import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def hjrlib():
    """The HIP library, built in-tree if it is not there yet (hipcc cross-compiles on a CPU host).
    A library built from other sources than the ones in the tree is rejected: its results would
    not be those of the code under test."""
    from paper_1903_07715_amd import build, hjr

    if not os.path.exists(hjr.LIB_PATH):
        build.build()
    hjr.load()
    want = build.source_hash()
    if hjr.build_id() != want:
        pytest.fail(f"{hjr.LIB_PATH} was built from other sources (build id {hjr.build_id()}, sources "
                    f"{want}); rebuild it with `python -m paper_1903_07715_amd.build`")
    return hjr


@pytest.fixture(scope="session")
def gpu(hjrlib):
    import torch

    if not torch.cuda.is_available() or hjrlib.device_count() < 1:
        pytest.fail("GPU test selected but no GPU is visible")
    return torch.device("cuda:0")
