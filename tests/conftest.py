"""Shared fixtures.  Tests marked ``gpu`` need an MI355X and the built
``libcmlb.so``; everything else runs on the CPU (oracle pins, host logic,
the ABI's symbol table)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and libcmlb.so")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library; fails loudly when it is missing or no GPU is visible."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("gpu test run without a visible GPU")
    from paper_2504_09024_amd import cmlb
    return cmlb.load()
