"""Host side of the coefficient form (normalised weights, polynomials in
x = 1/q, Sec. 3.5): the normalised factor maps and read-out maps, run by a
small numpy interpreter on truncated coefficient arrays mod p (test code,
not a product path), reproduce the oracle's truncated P~ exactly; the maps
have the same sparsity as the evaluation-form maps; the CRT helpers lift
residues back to the integers."""
import numpy as np
import pytest

from oracle import transfer as OT
from mapinterp import run_series as _run_series
from paper_1005_3609_amd import api, host

SQ, TRI = "square", "triangular"
P31 = 2 ** 31 - 1


def _oracle_series(lat, m, n_max, d, p):
    res = OT.projected_strip(lat, m, n_max, OT.ExactX(dmax=d))
    out = np.zeros((n_max, d + 1), dtype=np.int64)
    for r, z in enumerate(res):
        z = list(z)[: d + 1]
        out[r, : len(z)] = [c % p for c in z]
    return out


@pytest.mark.parametrize("lat", [SQ, TRI])
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("d,p", [(5, P31), (30, 998244353)])
def test_normalised_maps_reproduce_oracle(lat, m, d, p):
    np.testing.assert_array_equal(_run_series(lat, m, 4, d, p), _oracle_series(lat, m, 4, d, p))


SHARE = r"""
import sys
import numpy as np
from paper_1005_3609_amd import api
lat, m, out = sys.argv[1], int(sys.argv[2]), sys.argv[3]
arrs = {}
for i in range(m):
    for which in (0, 4):
        rp, cols, codes, nc = api.map_export(lat, m, which, i)
        arrs[f"{which}_{i}_rp"], arrs[f"{which}_{i}_cols"], arrs[f"{which}_{i}_codes"] = rp, cols, codes
np.savez(out, **arrs)
"""


@pytest.mark.parametrize("lat", [SQ, TRI])
def test_normalised_maps_share_the_sparsity(lat, tmp_path):
    # both forms in one numbering (the paper's order; by default the
    # evaluation form takes the site order and the normalised one the reader
    # order)
    import os
    import subprocess
    import sys
    m = 6
    out = str(tmp_path / "maps.npz")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, PYTHONPATH=root, CHROMSTRIP_STATE_ORDER="paper")
    r = subprocess.run([sys.executable, "-c", SHARE, lat, str(m), out], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr
    z = np.load(out)
    for i in range(m):
        a = tuple(z[f"0_{i}_{k}"] for k in ("rp", "cols", "codes"))
        b = tuple(z[f"4_{i}_{k}"] for k in ("rp", "cols", "codes"))
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
        # entry by entry the two coefficients agree up to a power of q:
        # c_norm(1/q) q^k = c(q) for some k in 0..3
        un = api.code_table(lat, m, normalised=False)[a[2]]
        no = api.code_table(lat, m, normalised=True)[b[2]]
        for u, n in zip(un, no):
            ok = any(all(n[i] == (u[k - i] if 0 <= k - i < 4 else 0) for i in range(4)) and
                     all(u[j] == (n[k - j] if 0 <= k - j < 4 else 0) for j in range(4)) for k in range(4))
            assert ok, (u, n)


def test_series_crt_lifts_to_the_exact_polynomial():
    # 3 x 4 square: P~ has degree 11, coefficients well below the product of 3 primes
    ps = [P31, 998244353, 1000000007]
    d = 14
    res = np.stack([_run_series(SQ, 3, 4, d, p)[3] for p in ps])
    coef, _ = host.series_exact(res, ps)
    exact = OT.chromatic_exact(SQ, 3, 4)[3]                 # P(q), ascending powers of q
    V = 12
    want = [exact[V - k] if 0 <= V - k < len(exact) else 0 for k in range(d + 1)]
    assert coef == want
    stab, used = host.series_stabilised(res, ps)
    assert stab == want and used <= 3


@pytest.mark.parametrize("lat", [SQ, TRI])
@pytest.mark.parametrize("m", [1, 2, 3, 5, 8, 11, 13])
def test_device_expansion_reproduces_host_maps(lat, m):
    # the per-state expansion that builds the coefficient form's maps on the
    # device, run on the host: every forward and read-out factor equal to
    # the host builder's (paper order), and the evaluation form's forward
    # factors too
    api.check_expansion(lat, m, normalised=True)
    api.check_expansion(lat, m, normalised=False)


def test_exact_polynomials_host_side(monkeypatch):
    # polynomial.chromatic_polynomials with the strips run by the map
    # interpreter: the prime loop, the CRT and the x^k -> q^{|V|-k} reversal
    from paper_1005_3609_amd import polynomial as PL

    def cpu_series(lat, m, n, d, primes, mode="graph", tuning=None):
        return np.stack([_run_series(lat, m, n, d, int(p)) for p in primes], axis=1)
    monkeypatch.setattr(PL.api, "series", cpu_series)
    polys, used = PL.chromatic_polynomials(SQ, 3, 4, batch=1)
    want = OT.chromatic_exact(SQ, 3, 4)
    assert [p[: len(w)] for p, w in zip(polys, want)] == want and all(not any(p[len(w):]) for p, w in zip(polys, want))
    assert used >= 2
    with pytest.raises(ValueError):
        PL.chromatic_polynomials(SQ, 23, 23)                      # |V| = 529 > 512 slots
