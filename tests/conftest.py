import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def gpu_ctx():
    """A librpfit context on cuda:0 (GPU tests only)."""
    import torch
    from paper_1906_00142_amd import rp
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.init()
    return rp.Context(0)


def planted_in_order(orc, pl):
    """Planted coefficients in the library's monomial order, matched by tuple."""
    import numpy as np
    num, den = pl.coef_by_tuple()
    En = orc.monomials(pl.nvars, pl.deg_num)
    Ed = orc.monomials(pl.nvars, pl.deg_den)
    return np.array([num[tuple(int(t) for t in e)] for e in En]
                    + [den[tuple(int(t) for t in e)] for e in Ed[1:]])
