"""Graphs, the definition of the chromatic polynomial, and direct ways to get it.

Test infrastructure only (see the package docstring).

Polynomials in q are lists of Python ints, index k holding the coefficient of
q**k.  Everything is exact.
"""
from __future__ import annotations

import itertools

SQUARE = "square"
TRIANGULAR = "triangular"


# --------------------------------------------------------------------------
# The lattice rectangles
# --------------------------------------------------------------------------
def lattice_graph(lattice: str, m: int, n: int):
    """Vertices and edges of the m x n rectangle, free boundaries.

    Sec. 3 (the text around eq. Z_from_T): a layer holds m vertices; each
    transfer step adds m-1 horizontal edges in the layer and m vertical edges
    to the next layer, and on the triangular lattice also m-1 diagonals.  The
    triangular lattice is the square lattice with one diagonal per face
    (Sec. 3.3).  Which diagonal: the triangular factors apply H_{i-1,i}
    after V_{i-1} has moved site i-1 to the new layer but before V_i has
    moved site i, so the diagonal joins new-layer vertex i-1 to old-layer
    vertex i, i.e. (r+1, c) -- (r, c+1) on every face.

    Vertices are (r, c) with r = 1..n (rows, the transfer direction) and
    c = 1..m (across the strip).  Returns (vertices, edges) with edges as
    pairs of vertex indices into ``vertices``.
    """
    if lattice not in (SQUARE, TRIANGULAR):
        raise ValueError(lattice)
    vertices = [(r, c) for r in range(1, n + 1) for c in range(1, m + 1)]
    index = {v: k for k, v in enumerate(vertices)}
    edges = []
    for r in range(1, n + 1):
        for c in range(1, m):
            edges.append((index[(r, c)], index[(r, c + 1)]))           # horizontal
    for r in range(1, n):
        for c in range(1, m + 1):
            edges.append((index[(r, c)], index[(r + 1, c)]))           # vertical
    if lattice == TRIANGULAR:
        for r in range(1, n):
            for c in range(1, m):
                edges.append((index[(r + 1, c)], index[(r, c + 1)]))   # diagonal
    return vertices, edges


def path_graph(k: int):
    return list(range(k)), [(i, i + 1) for i in range(k - 1)]


def cycle_graph(k: int):
    return list(range(k)), [(i, (i + 1) % k) for i in range(k)]


def complete_graph(k: int):
    return list(range(k)), [(i, j) for i in range(k) for j in range(i + 1, k)]


# --------------------------------------------------------------------------
# Definition: number of proper q-colourings (Sec. 1)
# --------------------------------------------------------------------------
def count_colourings(vertices, edges, q: int) -> int:
    """Number of assignments of q colours to the vertices such that the two
    ends of every edge differ (Sec. 1).  Plain backtracking in vertex order."""
    nv = len(vertices)
    earlier = [[] for _ in range(nv)]
    for a, b in edges:
        if a == b:
            return 0                      # a loop can never be properly coloured
        lo, hi = min(a, b), max(a, b)
        earlier[hi].append(lo)
    colour = [0] * nv

    def place(v: int) -> int:
        if v == nv:
            return 1
        total = 0
        for c in range(q):
            if all(colour[u] != c for u in earlier[v]):
                colour[v] = c
                total += place(v + 1)
        return total

    return place(0)


def count_colourings_product(vertices, edges, q: int) -> int:
    """The same count by listing every one of the q**|V| assignments
    (itertools.product); only for the smallest graphs."""
    total = 0
    for col in itertools.product(range(q), repeat=len(vertices)):
        if all(col[a] != col[b] for a, b in edges):
            total += 1
    return total


# --------------------------------------------------------------------------
# FK subset expansion (Sec. 2, eq. Z2) and its chromatic specialisation
# --------------------------------------------------------------------------
def _components(nv: int, edge_subset) -> int:
    parent = list(range(nv))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    k = nv
    for a, b in edge_subset:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
            k -= 1
    return k


def potts_by_subsets(vertices, edges, v: int) -> list[int]:
    """Z_G(q, v) = sum over edge subsets A of q^{k(A)} v^{|A|} (eq. Z2), as an
    exact polynomial in q for an integer v.  2^|E| terms."""
    nv = len(vertices)
    poly = [0] * (nv + 1)
    for size in range(len(edges) + 1):
        for subset in itertools.combinations(edges, size):
            poly[_components(nv, subset)] += v ** size
    return poly


def chromatic_by_subsets(vertices, edges) -> list[int]:
    """P_G(q) = Z_G(q, -1) (Sec. 2, the specialisation v = -1)."""
    return potts_by_subsets(vertices, edges, -1)


def potts_by_spins(vertices, edges, q: int, v: int) -> int:
    """Z_G(q, v) as the spin sum of eq. Z1: sum over all q^{|V|} spin
    configurations of the product over edges of (1 + v * delta)."""
    total = 0
    for sig in itertools.product(range(q), repeat=len(vertices)):
        w = 1
        for a, b in edges:
            if sig[a] == sig[b]:
                w *= 1 + v
        total += w
    return total


# --------------------------------------------------------------------------
# Colour-class dynamic programme over a rectangle (an independent method)
# --------------------------------------------------------------------------
def chromatic_by_colour_classes(lattice: str, m: int, n: int) -> list[int]:
    """P_G(q) of the m x n rectangle as an exact polynomial, by counting proper
    colourings vertex by vertex in row-major order.

    This is not the paper's transfer matrix: it tracks which of the last m
    placed vertices (the frontier) carry equal colours.  A new vertex either
    reuses the colour of a frontier colour class that contains none of its
    neighbours, or takes a colour absent from the frontier: (q - #classes)
    choices, the polynomial factor.  Neighbours of vertex (r, c) already
    placed: (r, c-1), (r-1, c) and, on the triangular lattice, (r-1, c+1)
    (the diagonal of ``lattice_graph``).  Exact for any q because the number
    of colourings depends only on the equality pattern.
    """
    # state: tuple of class labels of the frontier, oldest first, canonical.
    def canon(labels):
        seen = {}
        return tuple(seen.setdefault(x, len(seen)) for x in labels)

    states = {(): [1]}                      # polynomial weight per state
    order = [(r, c) for r in range(1, n + 1) for c in range(1, m + 1)]
    placed = []                             # the frontier's vertices, oldest first
    for (r, c) in order:
        nbrs = []
        if c > 1:
            nbrs.append((r, c - 1))
        if r > 1:
            nbrs.append((r - 1, c))
            if lattice == TRIANGULAR and c < m:
                nbrs.append((r - 1, c + 1))
        new_states: dict = {}
        for lab, w in states.items():
            classes = sorted(set(lab))
            banned = {lab[placed.index(u)] for u in nbrs}
            options = []
            for cl in classes:
                if cl not in banned:
                    options.append((cl, [1]))
            # a colour not present in the frontier: q - #classes choices
            options.append((len(classes), [-len(classes), 1]))
            for cl, factor in options:
                nl = lab + (cl,)
                if len(nl) > m:
                    nl = nl[1:]
                key = canon(nl)
                prod = _poly_mul(w, factor)
                new_states[key] = _poly_add(new_states.get(key, [0]), prod)
        placed.append((r, c))
        if len(placed) > m:
            placed.pop(0)
        states = new_states
    total = [0]
    for w in states.values():
        total = _poly_add(total, w)
    return _trim(total)


# --------------------------------------------------------------------------
# Small exact polynomial helpers (coefficient lists, index = power)
# --------------------------------------------------------------------------
def _trim(p):
    p = list(p)
    while len(p) > 1 and p[-1] == 0:
        p.pop()
    return p


def _poly_add(a, b):
    n = max(len(a), len(b))
    return [(a[k] if k < len(a) else 0) + (b[k] if k < len(b) else 0) for k in range(n)]


def _poly_mul(a, b):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x:
            for j, y in enumerate(b):
                out[i + j] += x * y
    return out


def poly_eval(p, q: int) -> int:
    acc = 0
    for coef in reversed(p):
        acc = acc * q + coef
    return acc


def poly_trim(p):
    return _trim(p)


def poly_mul(a, b):
    return _poly_mul(a, b)


def poly_pow(a, k: int):
    out = [1]
    for _ in range(k):
        out = _poly_mul(out, a)
    return out


# Closed forms used as pins -------------------------------------------------
def closed_form_path(k: int):
    """q (q-1)^{k-1}: a tree on k vertices."""
    return _trim(_poly_mul([0, 1], poly_pow([-1, 1], k - 1)))


def closed_form_cycle(k: int):
    """(q-1)^k + (-1)^k (q-1) for the k-cycle, k >= 3 (k = 2 gives the double
    edge, which as a simple graph is the path)."""
    return _trim(_poly_add(poly_pow([-1, 1], k), [(-1) ** k * -1, (-1) ** k]))


def closed_form_square_ladder(n: int):
    """2 x n square strip: q (q-1) (q^2 - 3q + 3)^{n-1}."""
    return _trim(_poly_mul([0, -1, 1], poly_pow([3, -3, 1], n - 1)))


def closed_form_triangular_ladder(n: int):
    """2 x n triangular strip (a 2-tree: each new vertex joins an edge):
    q (q-1) (q-2)^{2(n-1)}."""
    return _trim(_poly_mul([0, -1, 1], poly_pow([-2, 1], 2 * (n - 1))))


def closed_form_complete(k: int):
    """q (q-1) ... (q-k+1)."""
    out = [1]
    for j in range(k):
        out = _poly_mul(out, [-j, 1])
    return out
