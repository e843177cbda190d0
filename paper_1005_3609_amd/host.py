"""Host finish: from residues of P at integer q modulo primes to exact
integer polynomials.

The paper combines residues modulo several primes by the Chinese remainder
theorem and stops adding primes once the result stabilises (Sec. 3.5).  Here
the residues are values at integer points q, so each prime first gives the
polynomial's coefficients mod p by interpolation; CRT then combines the
coefficient residues and a symmetric lift recovers the signed integers.
"""
from __future__ import annotations

from math import prod


def crt(residues, primes) -> tuple[int, int]:
    """x mod M with M = prod(primes) and x = r_k mod p_k for every k."""
    x, M = 0, 1
    for r, p in zip(residues, primes):
        r, p = int(r) % int(p), int(p)
        # x + M t = r (mod p)
        t = ((r - x) * pow(M, -1, p)) % p
        x += M * t
        M *= p
    return x % M, M


def symmetric(x: int, M: int) -> int:
    """Representative of x mod M in (-M/2, M/2]."""
    x %= M
    return x - M if x > M // 2 else x


def interp_mod_p(xs, ys, p: int) -> list[int]:
    """Coefficients (ascending powers, mod p) of the unique polynomial of
    degree < len(xs) through (xs[k], ys[k]) modulo p: Newton divided
    differences, then expansion of the Newton form.  The xs must be
    distinct mod p."""
    xs = [int(x) % p for x in xs]
    coef = [int(y) % p for y in ys]
    n = len(xs)
    for j in range(1, n):
        for k in range(n - 1, j - 1, -1):
            coef[k] = (coef[k] - coef[k - 1]) * pow((xs[k] - xs[k - j]) % p, -1, p) % p
    poly = [0] * n
    for k in range(n - 1, -1, -1):
        # poly = poly * (x - xs[k]) + coef[k]
        new = [0] * n
        for d in range(n - 1):
            new[d + 1] = (new[d + 1] + poly[d]) % p
            new[d] = (new[d] - xs[k] * poly[d]) % p
        new[0] = (new[0] + coef[k]) % p
        poly = new
    return poly


def exact_polynomial(q_points, residues, primes) -> tuple[list[int], int]:
    """Integer coefficients of P from residues[a][b] = P(q_a) mod p_b.

    Needs len(q_points) > deg P.  Returns (coefficients, modulus): the
    coefficients are exact when every |coefficient| < modulus / 2."""
    per_prime = []
    for b, p in enumerate(primes):
        per_prime.append(interp_mod_p(q_points, [residues[a][b] for a in range(len(q_points))], int(p)))
    M = prod(int(p) for p in primes)
    coeffs = []
    for d in range(len(q_points)):
        x, _ = crt([pp[d] for pp in per_prime], primes)
        coeffs.append(symmetric(x, M))
    while len(coeffs) > 1 and coeffs[-1] == 0:
        coeffs.pop()
    return coeffs, M


def stabilised(q_points, residues, primes) -> tuple[list[int], int]:
    """Adds primes one at a time until the lifted coefficients stop changing
    (the stopping rule of Sec. 3.5); returns (coefficients, primes used)."""
    prev = None
    for k in range(1, len(primes) + 1):
        cur, _ = exact_polynomial(q_points, [row[:k] for row in residues], primes[:k])
        if cur == prev:
            return cur, k
        prev = cur
    return prev, len(primes)


def series_exact(residues, primes) -> tuple[list[int], int]:
    """Integer coefficients of the normalised polynomial P~ (powers of x =
    1/q) from the coefficient form: residues[b][k] = coefficient k mod
    primes[b].  Returns (coefficients, modulus); exact while every
    |coefficient| < modulus / 2 (Sec. 3.5: CRT over the primes)."""
    M = prod(int(p) for p in primes)
    out = []
    for k in range(len(residues[0])):
        x, _ = crt([residues[b][k] for b in range(len(primes))], primes)
        out.append(symmetric(x, M))
    return out, M


def series_stabilised(residues, primes) -> tuple[list[int], int]:
    """Adds primes one at a time until the lifted coefficients of P~ stop
    changing (the stopping rule of Sec. 3.5); returns (coefficients, primes
    used)."""
    prev = None
    for k in range(1, len(primes) + 1):
        cur, _ = series_exact([row for row in residues[:k]], primes[:k])
        if cur == prev:
            return cur, k
        prev = cur
    return prev, len(primes)
