"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module only draws random numbers and picks box shapes; it holds none of
the method's arithmetic (no GLL points, geometry, numbering, operator or
solver).  Every draw uses numpy's PCG64 with an explicit seed, so both sides
receive the same arrays.

Recipes (the workloads of the paper's kind: Nekbone on a box of hexahedra,
degree 9 in Sec. V, 1024-4096 elements in Sec. VI-B):

* geometry displacement coefficients ``a`` (3 values, U[-1,1]) for a bump of
  amplitude 0.05 that vanishes on the boundary;
* nodal values ``u`` uniform in [-1, 1] per local point;
* right-hand sides uniform in [-1, 1] per lattice node of the box (the
  caller scatters them through its own numbering and masks them);
* Poisson arrival traces of (E, N) solve requests for the served form.
"""
from __future__ import annotations

import numpy as np

SEED_GEOM = 2005
SEED_RHS = 13425
SEED_U = 1
AMP = 0.05

# Box shapes for the element counts the workloads use (Ex, Ey, Ez).
BOXES = {
    8: (2, 2, 2),
    27: (3, 3, 3),
    64: (4, 4, 4),
    512: (8, 8, 8),
    1024: (16, 8, 8),
    2048: (16, 16, 8),
    4096: (16, 16, 16),
    8192: (32, 16, 16),
}

# Degree sweep: boxes holding about 32.8 million local points each.
SWEEP_BOXES = {
    5: (48, 48, 64),
    7: (40, 40, 40),
    9: (32, 32, 32),
    11: (24, 24, 32),
    13: (16, 24, 32),
    15: (20, 20, 20),
}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def box_for(E: int):
    """(Ex, Ey, Ez) for an element count in BOXES, else the most cubic split."""
    if E in BOXES:
        return BOXES[E]
    best = None
    for ex in range(1, E + 1):
        if E % ex:
            continue
        for ey in range(1, E // ex + 1):
            if (E // ex) % ey:
                continue
            ez = E // ex // ey
            s = max(ex, ey, ez) - min(ex, ey, ez)
            if best is None or s < best[0]:
                best = (s, (ex, ey, ez))
    return best[1]


def geom_coeffs(seed: int = SEED_GEOM) -> np.ndarray:
    """Three displacement coefficients a_d ~ U[-1, 1]."""
    return rng(seed).uniform(-1.0, 1.0, size=3)


def local_uniform(P: int, seed: int = SEED_U) -> np.ndarray:
    """P values uniform in [-1, 1] (nodal values u, one per local point)."""
    return rng(seed).uniform(-1.0, 1.0, size=P)


def lattice_uniform(Ex: int, Ey: int, Ez: int, N: int, seed: int = SEED_RHS) -> np.ndarray:
    """One U[-1, 1] value per lattice node of the box, (Ex N+1)(Ey N+1)(Ez N+1) values
    in x-fastest lattice order."""
    U = (Ex * N + 1) * (Ey * N + 1) * (Ez * N + 1)
    return rng(seed).uniform(-1.0, 1.0, size=U)


def arrival_trace(n_requests: int, rate: float, seed: int = 7,
                  Es=(64, 512, 1024, 4096, 8192), Ns=(5, 7, 9, 11)):
    """Poisson arrivals: exponential gaps of mean 1/rate seconds; E and N drawn
    uniformly from the given sets; one geometry and one rhs seed per request."""
    r = rng(seed)
    gaps = r.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    Esel = r.choice(np.asarray(Es), size=n_requests)
    Nsel = r.choice(np.asarray(Ns), size=n_requests)
    seeds = r.integers(0, 2**31 - 1, size=(n_requests, 2))
    return [dict(t=float(t[i]), E=int(Esel[i]), N=int(Nsel[i]),
                 geom_seed=int(seeds[i, 0]), rhs_seed=int(seeds[i, 1]))
            for i in range(n_requests)]
