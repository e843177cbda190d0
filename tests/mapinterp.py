"""Test helpers (not a product path): a numpy interpreter of the exported
normalised factor maps on truncated coefficient arrays mod p, and the
paper's Table 1 fixture."""
import os

import numpy as np

from paper_1005_3609_amd import api

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def apply_poly(csr, polys, X, p):
    """out[t] = sum over entries (t, s, c) of polys[c](x) * X[s], truncated
    to X's number of coefficients, mod p."""
    rp, cols, codes, _ = csr
    nrows = rp.size - 1
    D1 = X.shape[1]
    out = np.zeros((nrows, D1), dtype=np.int64)
    if cols.size:
        rows = np.repeat(np.arange(nrows), np.diff(rp))
        src = X[cols]
        for k in range(polys.shape[1]):
            ck = polys[codes, k] % p
            if not ck.any() or k >= D1:
                continue
            contrib = np.zeros_like(src)
            contrib[:, k:] = (ck[:, None] * src[:, : D1 - k]) % p
            np.add.at(out, rows, contrib)
    return out % p


def run_series(lat, m, n_max, d, p):
    """P~ of the m x r rectangles, r = 1..n_max, coefficients of x^0..x^d
    mod p, by the normalised maps: int64 [n_max][d+1]."""
    polys = api.code_table(lat, m, normalised=True)
    fwd = [api.map_export(lat, m, 4, i) for i in range(m)]
    last = [api.map_export(lat, m, 5, i) for i in range(m)]
    x = np.zeros((fwd[0][3], d + 1), dtype=np.int64)
    x[0, 0] = 1                                          # e_0: all singletons, weight 1
    rows = []
    for r in range(n_max):
        y = x
        for i in range(m):
            y = apply_poly(last[i], polys, y, p)
        assert y.shape[0] == 1
        rows.append(y[0])
        if r + 1 < n_max:
            for i in range(m):
                x = apply_poly(fwd[i], polys, x, p)
    return np.stack(rows)


def table1():
    """The paper's Table 1 (square lattice): {k: (alpha_k, beta_k, gamma_k)}."""
    rows = {}
    with open(os.path.join(GOLDEN, "table1_square.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            k, a, b, c = ln.split()
            rows[int(k)] = (int(a), int(b), None if c == "-" else int(c))
    return rows
