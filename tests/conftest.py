"""Shared pytest configuration.

Tests marked ``gpu`` need an MI355X (they call the HIP library through its
C ABI); everything else runs on the CPU.  Native libraries are built on
demand only when missing (``__graft_entry__.build()`` rebuilds them).
"""
import os
import sys

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if REPO not in sys.path:
    sys.path.insert(0, REPO)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD MI355X GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def inputs_mod():
    from paper_2112_03229_amd import inputs
    return inputs


@pytest.fixture(scope="session")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_03229_amd import binding
    binding.lib()  # raises if the HIP library is missing
    return torch.device("cuda:0")
