"""Proper 3-colourings of the square-lattice rectangles, counted directly.

Test infrastructure only (see the package docstring).

P_G(3) is, by the definition of Sec. 1, the number of proper 3-colourings of G.
This module counts them for the m x n square-lattice rectangles with a
transfer matrix over colours, which shares nothing with the partition
transfer matrix of Sec. 3. It gives an exact value of P(3) at sizes that
backtracking cannot reach, such as the 20 x 21 rectangle.

Colours are residues mod 3. A proper colouring of a row of m sites is fixed by
its first colour and the differences d_j = c_j - c_{j-1}, each 1 or 2 mod 3.
A next row b differs from row a site by site exactly when b_j = a_j + e_j with
e_j in {1, 2}. Its differences are then d'_j = d_j + e_j - e_{j-1}, and b is
proper exactly when none of them is 0. Adding 1 to every colour maps proper
colourings to proper colourings, so the count is 3 times the count with the
first colour of the first row fixed, and the first colours never need to be
tracked.

A row is added one site at a time. Between sites the state is the m - 1
differences (the new ones left of the site, the old ones from it on) together
with the last e chosen. The counts are kept mod a few 31-bit primes, and the
exact value is recovered by the Chinese remainder theorem. A proper colouring
has at most 3 * 2^(mn - 1) members (every site after the first avoids the
colour of a neighbour already coloured), so primes are added until their
product exceeds twice that bound.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np


def _is_prime(n: int) -> bool:
    if n < 2:
        return False
    k = 2
    while k * k <= n:
        if n % k == 0:
            return False
        k += 1
    return True


@lru_cache(maxsize=None)
def _primes_below(limit: int, count: int) -> tuple:
    out, n = [], limit - 1
    while len(out) < count:
        if _is_prime(n):
            out.append(n)
        n -= 1
    return tuple(out)


def _counts_mod(m: int, n_max: int, p: int) -> list[int]:
    """[number of proper 3-colourings of the m x r rectangle with the first
    colour fixed, mod p, for r = 1..n_max]."""
    nb = m - 1                      # difference bits; bit j-1 holds d_j - 1
    size = 1 << nb
    x = np.ones(size, dtype=np.int64) % p          # row 1: any differences
    out = [int(x.sum() % p)]
    idx = np.arange(2 * size, dtype=np.int64)      # state: differences | (e - 1) << nb
    ebit = (idx >> nb) & 1
    for _ in range(1, n_max):
        # site 0: any e_0, differences unchanged
        y = np.concatenate([x, x])
        for j in range(1, m):
            dj = ((idx >> (j - 1)) & 1) + 1
            ep = ebit + 1
            z = np.zeros(2 * size, dtype=np.float64)
            base = idx & ~((1 << (j - 1)) | (1 << nb))
            for e in (1, 2):
                dn = (dj + e - ep) % 3
                ok = dn != 0
                tgt = base | ((dn - 1) << (j - 1)) | ((e - 1) << nb)
                z += np.bincount(tgt[ok], weights=y[ok].astype(np.float64), minlength=2 * size)
            y = z.astype(np.int64) % p
        x = (y[:size] + y[size:]) % p              # forget the last e
        out.append(int(x.sum() % p))
    return out


def square_three_colourings(m: int, n_max: int) -> list[int]:
    """[P(3) of the square m x r rectangle, r = 1..n_max]: the exact numbers of
    proper 3-colourings (m >= 1)."""
    if m < 1 or n_max < 1:
        raise ValueError("need m >= 1 and n_max >= 1")
    bound = 2 * 3 * 2 ** (m * n_max - 1)
    primes, prod = [], 1
    for p in _primes_below(2 ** 31, 64):
        primes.append(p)
        prod *= p
        if prod > bound:
            break
    residues = [_counts_mod(m, n_max, p) for p in primes]
    out = []
    for r in range(n_max):
        v, mod = 0, 1
        for p, res in zip(primes, residues):
            # v := the value mod mod * p that is v mod mod and res[r] mod p
            t = ((res[r] - v) * pow(mod, -1, p)) % p
            v, mod = v + mod * t, mod * p
        out.append(3 * v)
    return out
