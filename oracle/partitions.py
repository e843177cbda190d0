"""Set partitions of one layer and the paper's NCNNN ordering.

Test infrastructure only (see the package docstring).

A partition of the points 1..m is stored as a tuple ``lab`` of length m with
``lab[i-1]`` the block label of point i, labels numbered in order of first
appearance (so equal partitions have equal tuples).  The paper writes them
as e.g. (13)(2)(4); ``to_paper``/``from_paper`` convert.
"""
from __future__ import annotations

from math import comb, factorial


def canonical(labels) -> tuple:
    seen: dict = {}
    return tuple(seen.setdefault(x, len(seen)) for x in labels)


def blocks(lab) -> list[list[int]]:
    """Blocks as sorted lists of 1-based points, ordered by smallest point."""
    out: dict = {}
    for i, x in enumerate(lab, start=1):
        out.setdefault(x, []).append(i)
    return list(out.values())


def to_paper(lab) -> str:
    """Write as the paper does: blocks by smallest element, e.g. '(13)(2)(4)'.
    Points above 9 are written in braces to stay unambiguous."""
    def pt(i):
        return str(i) if i < 10 else "{%d}" % i
    return "".join("(" + "".join(pt(i) for i in b) + ")" for b in blocks(lab))


def from_paper(text: str, m: int) -> tuple:
    lab = [None] * m
    for k, part in enumerate(text.strip("()").split(")(")):
        for ch in part:
            lab[int(ch) - 1] = k
    return canonical(lab)


def singletons(m: int) -> tuple:
    """The all-singleton partition (1)(2)...(m), written e_0 in eq. Z_from_T."""
    return tuple(range(m))


# --------------------------------------------------------------------------
# Predicates (Sec. 3.2)
# --------------------------------------------------------------------------
def is_noncrossing(lab) -> bool:
    """No a < b < c < d with a~c, b~d in different blocks (planarity)."""
    m = len(lab)
    for a in range(m):
        for b in range(a + 1, m):
            for c in range(b + 1, m):
                if lab[a] != lab[c] or lab[b] == lab[a]:
                    continue
                for d in range(c + 1, m):
                    if lab[b] == lab[d]:
                        return False
    return True


def is_nnn(lab, allowed=None) -> bool:
    """No two neighbouring points in one block, except the pair (allowed,
    allowed+1) when given (1-based)."""
    for i in range(1, len(lab)):
        if lab[i - 1] == lab[i] and i != allowed:
            return False
    return True


def all_partitions(m: int):
    """Every set partition of 1..m (restricted growth strings)."""
    def rec(prefix, top):
        if len(prefix) == m:
            yield tuple(prefix)
            return
        for x in range(top + 1):
            yield from rec(prefix + [x], max(top, x + 1))
    if m == 0:
        yield ()
        return
    yield from rec([0], 1)


def noncrossing_partitions(m: int) -> list[tuple]:
    return [p for p in all_partitions(m) if is_noncrossing(p)]


def ncnnn_partitions_by_filter(m: int) -> list[tuple]:
    """NCNNN partitions found by filtering all partitions (order unspecified)."""
    return [p for p in noncrossing_partitions(m) if is_nnn(p)]


# --------------------------------------------------------------------------
# Counts (Sec. 3.2, Catalan and Motzkin numbers; Sec. 3.4, eq. M_recurs)
# --------------------------------------------------------------------------
def catalan(m: int) -> int:
    """C_m = (2m)! / (m! (m+1)!)."""
    return factorial(2 * m) // (factorial(m) * factorial(m + 1))


def motzkin(k: int) -> int:
    """M_k = sum_j binom(k, 2j) C_j."""
    return sum(comb(k, 2 * j) * catalan(j) for j in range(k // 2 + 1))


def motzkin_by_recursion(p: int) -> int:
    """eq. M_recurs: M_p = M_{p-1} + sum_{k=0}^{p-2} M_k M_{p-k-2}, M_0 = M_1 = 1."""
    M = [1, 1]
    for q in range(2, p + 1):
        M.append(M[q - 1] + sum(M[k] * M[q - k - 2] for k in range(q - 1)))
    return M[p]


# --------------------------------------------------------------------------
# The NCNNN ordering of Sec. 3.4
# --------------------------------------------------------------------------
def ncnnn_in_paper_order(m: int) -> list[tuple]:
    """All NCNNN partitions of 1..m in the order defined in Sec. 3.4.

    First those where point 1 is a singleton, ordered as the partitions of
    2..m.  Then those where point 1 shares its block; with 3+k the smallest
    other point of that block (k = 0..m-3), in increasing k, and for fixed k
    ordered with the partition of 2..2+k as the more significant and the
    partition of 3+k..m as the less significant digit.  Sets of one or two
    points have a single NCNNN partition.
    """
    def rec(points: list[int]) -> list[dict]:
        # returns list of {point: block id}, block ids are fresh objects
        n = len(points)
        if n == 0:
            return [{}]
        if n <= 2:
            return [{pt: ("s", pt) for pt in points}]
        first, rest = points[0], points[1:]
        out = []
        for sub in rec(rest):                       # point 1 a singleton
            d = dict(sub)
            d[first] = ("s", first)
            out.append(d)
        for k in range(0, n - 2):                   # point 1 joined to 3+k
            inner = points[1:2 + k]                 # points 2 .. 2+k
            outer = points[2 + k:]                  # points 3+k .. m
            for a in rec(inner):
                for b in rec(outer):
                    d = dict(a)
                    d.update(b)
                    d[first] = b[outer[0]]          # 1 joins the block of 3+k
                    out.append(d)
        return out

    result = []
    for d in rec(list(range(1, m + 1))):
        result.append(canonical([d[i] for i in range(1, m + 1)]))
    return result


def ncnnn_rank_table(m: int) -> dict:
    """0-based rank of each NCNNN partition in the paper's order."""
    return {p: r for r, p in enumerate(ncnnn_in_paper_order(m))}


def square_intermediate_in_paper_order(m: int, i: int) -> list[tuple]:
    """States after the square-lattice factor T_i (Sec. 3.4, last paragraph):
    first the M_{m-1} NCNNN partitions, then the M_{m-2} partitions where i
    and i+1 share a block, ordered as the NCNNN partitions of the m-1 points
    obtained by contracting i and i+1 into one point."""
    first = ncnnn_in_paper_order(m)
    second = []
    for c in ncnnn_in_paper_order(m - 1):
        # expand point i of the contracted partition into points i and i+1
        lab = list(c[:i]) + [c[i - 1]] + list(c[i:])
        second.append(canonical(lab))
    return first + second
