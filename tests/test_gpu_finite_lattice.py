"""The finite-lattice series end to end (Sec. 4.1 with the coefficient form
on the GPU, Sec. 3.5): the square-lattice bulk, surface and corner series
equal the paper's Table 1, at odd k one order further with the polygon
term of Sec. 4.2."""
import pytest

from mapinterp import table1
from paper_1005_3609_amd import finite_lattice as FL
from paper_1005_3609_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    yield


@pytest.mark.parametrize("k,mode,extra", [(14, "batched", False), (24, "graph", False), (13, "graph", True),
                                          (37, "graph", True)])
def test_square_series_match_table1(k, mode, extra):
    # extra: alpha and beta one order further (z^{2k-3}) with the polygon term
    res = FL.square_series(k, W.seeded_primes(5, 2024), mode=mode, extra=extra)
    assert res["stable"]
    N = 2 * k - 4 + extra
    t = table1()
    assert res["alpha"] == [t[i][0] for i in range(N + 1)]
    assert res["beta"] == [t[i][1] for i in range(N + 1)]
    assert res["gamma"] == [t[i][2] for i in range(2 * k - 3)]
