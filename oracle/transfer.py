"""The FK transfer matrix, as the paper builds it, on a dictionary of partitions.

Test infrastructure only (see the package docstring).

A vector is a dict {partition tuple: weight}.  Partitions are canonical label
tuples (``oracle.partitions``); points are 1-based in every function
argument, as in the paper.  No ranking, no index maps, no fusion: each
single-edge operator of Sec. 3.1 is its own pass over the dictionary, and
the per-site factors are the products the paper writes, applied right to
left.

Two bookkeepings of the factor q^{k(A)} of eq. Z2 are supported:

* normalised (the paper's, eq. Z_modified): weights are polynomials in
  x = 1/q, a join of two distinct components costs x, the vertical edge is
  V_i = v x + D_i, and the read-out is P-tilde = q^{-|V|} P.
* un-normalised: weights are polynomials in q (or residues of them at an
  integer q), joins cost 1, and a component pays its factor q once, when it
  leaves the layer: the detach D_i multiplies by q when point i was alone in
  its block.  Then V_i = v + D_i and the read-out is P itself.  This is the
  same sum over edge subsets counted differently (each component of G_A
  leaves the top layer exactly once); it is what allows integer q = 0.
"""
from __future__ import annotations

import numpy as np

from .partitions import canonical, singletons

SQUARE = "square"
TRIANGULAR = "triangular"


# --------------------------------------------------------------------------
# Weight algebras
# --------------------------------------------------------------------------
class ExactQ:
    """Un-normalised weights: exact integer polynomials in q (index = power)."""
    normalised = False

    def one(self):
        return (1,)

    def is_zero(self, w):
        return not any(w)

    def add(self, a, b):
        n = max(len(a), len(b))
        return tuple((a[k] if k < len(a) else 0) + (b[k] if k < len(b) else 0)
                     for k in range(n))

    def scale(self, w, k: int):
        return tuple(k * c for c in w)

    def times_q(self, w):
        return (0,) + tuple(w)

    def times_x(self, w):                          # never used un-normalised
        raise AssertionError("x = 1/q only appears in the normalised form")


class ExactX:
    """Normalised weights (eq. Z_modified): exact polynomials in x = 1/q,
    optionally truncated above degree ``dmax`` (Sec. 3.5)."""
    normalised = True

    def __init__(self, dmax: int | None = None):
        self.dmax = dmax

    def one(self):
        return (1,)

    def is_zero(self, w):
        return not any(w)

    def add(self, a, b):
        return ExactQ.add(self, a, b)

    def scale(self, w, k: int):
        return tuple(k * c for c in w)

    def times_q(self, w):                          # never used normalised
        raise AssertionError("the normalised form has no closure factor")

    def times_x(self, w):
        out = (0,) + tuple(w)
        if self.dmax is not None:
            out = out[: self.dmax + 1]
        return out


class Residues:
    """Un-normalised weights as residues: one int64 entry per instance
    (q_j, p_j), every result reduced into [0, p_j) (Sec. 3.5 uses residues
    modulo primes below 2^31 so that no intermediate overflows)."""
    normalised = False

    def __init__(self, qs, ps):
        self.p = np.asarray(ps, dtype=np.int64)
        self.q = np.asarray(qs, dtype=np.int64) % self.p
        assert (self.p > 2).all() and (self.p < 2 ** 31).all()

    def one(self):
        return np.ones_like(self.p)

    def is_zero(self, w):
        return not w.any()

    def add(self, a, b):
        return (a + b) % self.p

    def scale(self, w, k: int):
        return (w * k) % self.p

    def times_q(self, w):
        return (w * self.q) % self.p

    def times_x(self, w):
        raise AssertionError("residues use the un-normalised form")


def _acc(out: dict, key, w, alg):
    if key in out:
        out[key] = alg.add(out[key], w)
    else:
        out[key] = w


def _drop_zeros(vec: dict, alg) -> dict:
    return {s: w for s, w in vec.items() if not alg.is_zero(w)}


# --------------------------------------------------------------------------
# Operations on one partition (Sec. 3.1)
# --------------------------------------------------------------------------
def join(s: tuple, i: int, j: int) -> tuple:
    """The blocks of points i and j merged into one."""
    a, b = s[i - 1], s[j - 1]
    return canonical([a if x == b else x for x in s])


def detach(s: tuple, i: int) -> tuple:
    """Point i removed from its block and made a singleton."""
    fresh = max(s) + 1
    lab = list(s)
    lab[i - 1] = fresh
    return canonical(lab)


def alone(s: tuple, i: int) -> bool:
    return sum(1 for x in s if x == s[i - 1]) == 1


# --------------------------------------------------------------------------
# Single-edge operators on a whole vector (Sec. 3.1)
# --------------------------------------------------------------------------
def op_J(vec: dict, i: int, j: int, alg) -> dict:
    """Join operator: identity when i, j already share a block; otherwise
    merges the two blocks, at a cost x in the normalised form."""
    out: dict = {}
    for s, w in vec.items():
        if s[i - 1] == s[j - 1]:
            _acc(out, s, w, alg)
        else:
            _acc(out, join(s, i, j), alg.times_x(w) if alg.normalised else w, alg)
    return out


def op_H(vec: dict, i: int, j: int, v: int, alg) -> dict:
    """Edge between points i and j of the layer: H = 1 + v J."""
    out = dict(vec)
    for s, w in op_J(vec, i, j, alg).items():
        _acc(out, s, alg.scale(w, v), alg)
    return _drop_zeros(out, alg)


def op_D(vec: dict, i: int, alg) -> dict:
    """Detach operator D_i: point i becomes a singleton (the new vertex i'
    relabelled as i).  Un-normalised: if i was alone, its component leaves
    the layer for good and pays q."""
    out: dict = {}
    for s, w in vec.items():
        if alone(s, i):
            _acc(out, s, w if alg.normalised else alg.times_q(w), alg)
        else:
            _acc(out, detach(s, i), w, alg)
    return out


def op_V(vec: dict, i: int, v: int, alg) -> dict:
    """Vertical edge from point i to the next layer: V_i = v x + D_i
    (normalised) or v + D_i (un-normalised).  With the edge present the new
    vertex takes i's place in i's block, so the partition is unchanged."""
    out: dict = {}
    for s, w in vec.items():
        present = alg.scale(w, v)
        if alg.normalised:
            present = alg.times_x(present)
        _acc(out, s, present, alg)
    for s, w in op_D(vec, i, alg).items():
        _acc(out, s, w, alg)
    return _drop_zeros(out, alg)


def op_P(vec: dict, pairs) -> dict:
    """Product of projectors P_{j,j+1} over the given j: a state survives
    only if no listed pair (j, j+1) shares a block (eq. projector)."""
    return {s: w for s, w in vec.items()
            if all(s[j - 1] != s[j] for j in pairs)}


# --------------------------------------------------------------------------
# Generic transfer matrix, any v (Sec. 3.2, first displayed T)
# --------------------------------------------------------------------------
def generic_row(vec: dict, lattice: str, m: int, v: int, alg) -> dict:
    """One layer for any v: all horizontal edges H_{i,i+1}, then the vertical
    edges V_1..V_m; on the triangular lattice the diagonal H_{i-1,i} is laid
    after V_{i-1} and before V_i (Sec. 3.3)."""
    for i in range(1, m):
        vec = op_H(vec, i, i + 1, v, alg)
    for i in range(1, m + 1):
        if lattice == TRIANGULAR and i >= 2:
            vec = op_H(vec, i - 1, i, v, alg)
        vec = op_V(vec, i, v, alg)
    return vec


def generic_readout(vec: dict, m: int, v: int, alg):
    """Last layer's horizontal edges, then every block still open closes
    (un-normalised: a factor q per block; normalised: nothing further)."""
    for i in range(1, m):
        vec = op_H(vec, i, i + 1, v, alg)
    total = None
    for s, w in vec.items():
        if not alg.normalised:
            for _ in range(len(set(s))):
                w = alg.times_q(w)
        total = w if total is None else alg.add(total, w)
    return total


def generic_strip(lattice: str, m: int, n_max: int, v: int, alg) -> list:
    """Z of the m x r rectangle for r = 1..n_max, any v, over all
    non-crossing partitions (Catalan C_m states)."""
    vec = {singletons(m): alg.one()}
    out = []
    for r in range(1, n_max + 1):
        out.append(generic_readout(dict(vec), m, v, alg))
        if r < n_max:
            vec = generic_row(vec, lattice, m, v, alg)
    return out


# --------------------------------------------------------------------------
# Projected sparse factorisation at v = -1 (Sec. 3.2 - 3.3)
# --------------------------------------------------------------------------
V_CHROMATIC = -1


def factor_square(vec: dict, i: int, m: int, alg) -> dict:
    """eq. T_sq_proj: T_i = (prod_{j != i} P_{j,j+1}) V_i H_{i,i+1} for
    i < m, and T_m = (prod_j P_{j,j+1}) V_m."""
    if i < m:
        vec = op_H(vec, i, i + 1, V_CHROMATIC, alg)
    vec = op_V(vec, i, V_CHROMATIC, alg)
    return op_P(vec, [j for j in range(1, m) if j != i])


def factor_triangular(vec: dict, i: int, m: int, alg) -> dict:
    """Triangular factors (Sec. 3.3): T_1 = P V_1 H_{1,2},
    T_i = P V_i H_{i-1,i} H_{i,i+1}, T_m = P V_m H_{m-1,m}, with P the
    product of all nearest-neighbour projectors.  m = 1 has no edge in a
    layer, so T_1 = V_1."""
    if i < m:
        vec = op_H(vec, i, i + 1, V_CHROMATIC, alg)
    if i > 1:
        vec = op_H(vec, i - 1, i, V_CHROMATIC, alg)
    vec = op_V(vec, i, V_CHROMATIC, alg)
    return op_P(vec, list(range(1, m)))


def projected_row(vec: dict, lattice: str, m: int, alg) -> dict:
    """eq. T_sq_decomp: T = T_m ... T_2 T_1 (T_1 applied first)."""
    factor = factor_square if lattice == SQUARE else factor_triangular
    for i in range(1, m + 1):
        vec = factor(vec, i, m, alg)
    return vec


def last_factor(vec: dict, i: int, m: int, alg) -> dict:
    """eq. T_last_i: T_i^last = (prod_{j=i+1}^{m-1} P_{j,j+1}) D_i H_{i,i+1};
    for i = m there is no edge H_{m,m+1}, so T_m^last = D_m."""
    if i < m:
        vec = op_H(vec, i, i + 1, V_CHROMATIC, alg)
    vec = op_D(vec, i, alg)
    return op_P(vec, list(range(i + 1, m)))


def projected_readout(vec: dict, m: int, alg):
    """eq. T_last then eq. Z_from_T: the coefficient of e_0 after
    T_last = T_m^last ... T_1^last (only e_0 survives)."""
    for i in range(1, m + 1):
        vec = last_factor(vec, i, m, alg)
    e0 = singletons(m)
    assert set(vec) <= {e0}, "only the all-singleton state survives T_last"
    return vec.get(e0)


def projected_strip(lattice: str, m: int, n_max: int, alg, trace=None) -> list:
    """P of the m x r rectangle for r = 1..n_max by eq. Z_from_T with the
    sparse factorisation: start from e_0, read out with T_last after every
    row.  ``trace`` (a list) receives the state vector after every factor."""
    vec = {singletons(m): alg.one()}
    out = []
    for r in range(1, n_max + 1):
        z = projected_readout(dict(vec), m, alg)
        out.append(z)
        if r < n_max:
            factor = factor_square if lattice == SQUARE else factor_triangular
            for i in range(1, m + 1):
                vec = factor(vec, i, m, alg)
                if trace is not None:
                    trace.append((r, i, dict(vec)))
    return out


# --------------------------------------------------------------------------
# Convenience front ends
# --------------------------------------------------------------------------
def chromatic_exact(lattice: str, m: int, n_max: int) -> list[list[int]]:
    """Exact integer polynomials P_{m x r}(q), r = 1..n_max (un-normalised)."""
    res = projected_strip(lattice, m, n_max, ExactQ())
    out = []
    for z in res:
        z = list(z) if z is not None else [0]
        while len(z) > 1 and z[-1] == 0:
            z.pop()
        out.append(z)
    return out


def chromatic_residues(lattice: str, m: int, n_max: int, qs, ps) -> np.ndarray:
    """Residues of P_{m x r}(q) for r = 1..n_max at every instance
    (qs[j], ps[j]); returns int64 [n_max][len(qs)]."""
    alg = Residues(qs, ps)
    res = projected_strip(lattice, m, n_max, alg)
    return np.stack([z if z is not None else np.zeros_like(alg.p) for z in res])


def chromatic_grid(lattice: str, m: int, n_max: int, q_points, primes) -> np.ndarray:
    """Residues laid out [n_max][nq][np], instance (q, p) = (q_points[a],
    primes[b]) -- the layout of the library's output."""
    qs = [q for q in q_points for _ in primes]
    ps = [p for _ in q_points for p in primes]
    flat = chromatic_residues(lattice, m, n_max, qs, ps)
    return flat.reshape(n_max, len(q_points), len(primes))
