"""Seeded synthetic workloads: q points, 31-bit primes, rectangle sets and
job streams.

This module generates inputs only.  It holds none of the transfer-matrix
arithmetic and imports nothing else from the package, so the CPU oracle's
fixture script and the GPU path can both draw the same inputs from it.

The paper fixes no primes (it says only that up to 16 primes below 2^31
were needed, Sec. 3.5), so they are drawn here: uniform in [2^30, 2^31-1)
from ``numpy.random.default_rng(seed)``, moved up to the next prime
(deterministic Miller-Rabin with bases 2, 7, 61, exact below 4 759 123 141),
redrawn if that passes 2^31-1 or repeats an earlier prime.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 10053609          # the arXiv number, plus the workload index
P_MERSENNE31 = 2 ** 31 - 1


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    for sp in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61):
        if n % sp == 0:
            return n == sp
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 7, 61):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def next_prime(n: int) -> int:
    while not is_prime(n):
        n += 1
    return n


def seeded_primes(count: int, seed: int) -> list[int]:
    rng = np.random.default_rng(seed)
    out: list[int] = []
    while len(out) < count:
        p = next_prime(int(rng.integers(2 ** 30, 2 ** 31 - 1)))
        if p < 2 ** 31 and p not in out:
            out.append(p)
    return out


def instances(q_points, primes):
    """Instance list in the library's order: q-major, prime-minor."""
    return [(int(q), int(p)) for q in q_points for p in primes]


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------
def workload(name: str) -> dict:
    """Named workloads.  Each entry lists rectangles as (lattice, m, n_max)
    strips, with the q points and primes shared by all of them."""
    if name == "square_4x5":
        return dict(strips=[("square", 4, 5)], q_points=list(range(21)),
                    primes=[P_MERSENNE31])
    if name == "square_m10":
        return dict(strips=[("square", 10, 11)], q_points=list(range(1, 81)),
                    primes=seeded_primes(4, SEED_BASE + 2))
    if name == "triangular_m12":
        return dict(strips=[("triangular", 12, 13)], q_points=list(range(1, 49)),
                    primes=seeded_primes(6, SEED_BASE + 3))
    if name == "square_sweep_2_14":
        return dict(strips=[("square", m, m + 1) for m in range(2, 15)],
                    q_points=list(range(1, 81)), primes=seeded_primes(8, SEED_BASE + 4))
    if name == "square_14x15":
        w = workload("square_sweep_2_14")
        return dict(strips=[("square", 14, 15)], q_points=w["q_points"], primes=w["primes"])
    if name == "square_18x19":
        w = workload("square_sweep_2_14")
        return dict(strips=[("square", 18, 19)], q_points=w["q_points"], primes=w["primes"])
    raise KeyError(name)


def sample_instances(n_inst: int, count: int, seed: int) -> list[int]:
    """A seeded sorted sample of instance indices."""
    rng = np.random.default_rng(seed)
    if count >= n_inst:
        return list(range(n_inst))
    return sorted(int(x) for x in rng.choice(n_inst, size=count, replace=False))


def serving_stream(n_jobs: int, rate: float = 20.0, seed: int = SEED_BASE + 5) -> list[dict]:
    """Poisson arrivals (mean ``rate`` jobs/s) of rectangle jobs: lattice
    uniform in {square, triangular}, m uniform in 6..16, n = m+1, q = 1..Q
    with Q uniform in 16..80, and 1..4 primes drawn from a seeded pool of 8."""
    rng = np.random.default_rng(seed)
    pool = seeded_primes(8, seed + 1000)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        lat = "square" if rng.integers(0, 2) == 0 else "triangular"
        m = int(rng.integers(6, 17))
        nq = int(rng.integers(16, 81))
        npr = int(rng.integers(1, 5))
        primes = [pool[k] for k in sorted(rng.choice(8, size=npr, replace=False))]
        jobs.append(dict(id=j, arrival=t, lattice=lat, m=m, n_max=m + 1,
                         q_points=list(range(1, nq + 1)), primes=primes))
    return jobs
