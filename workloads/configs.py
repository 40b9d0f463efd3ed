"""The synthetic workloads, built from formulas and seeds.

The paper benchmarks closed antiferromagnetic Heisenberg chains with U(1),
spin inversion, translation and reflection symmetry (Section 6, "Test
Hamiltonians"); the workloads below are of that shape, extended to J1-J2
couplings and the square lattice.  Nothing is read from disk.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import lattice, rng, terms


@dataclass
class Sector:
    name: str
    n_sites: int
    weight: int
    group: lattice.Group
    terms: np.ndarray
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def is_real(self) -> bool:
        return bool(np.all(self.group.chi[:, 1] == 0.0) and np.all(self.terms["im"] == 0.0))


def ring16_u1(seed: int = 1) -> Sector:
    """Heisenberg ring N=16, J=1, Sz=0, no lattice symmetry (dim 12870)."""
    n = 16
    return Sector("ring16_sz0_nosym", n, n // 2, lattice.trivial_group(n),
                  terms.heisenberg_terms(lattice.ring_bonds(n, 1.0)), seed)


def ring_symmetric(n: int, k: int = 0, reflection: int = 1, inversion: int = 1,
                   j2: float = 0.0, seed: int = 2) -> Sector:
    g = lattice.ring_group(n, k, reflection, inversion)
    return Sector(f"ring{n}_k{k}_r{reflection}_z{inversion}" + (f"_j2{j2:g}" if j2 else ""),
                  n, n // 2, g, terms.heisenberg_terms(lattice.ring_bonds(n, 1.0, j2)), seed)


def ring32_symmetric(seed: int = 2) -> Sector:
    """Ring N=32, Sz=0, k=0, R=+1, Z=+1 (nG=128, dim 4,707,969)."""
    return ring_symmetric(32, 0, 1, 1, 0.0, seed)


def square_j1j2(lx: int = 6, ly: int = 6, j2: float = 0.5, seed: int = 3,
                inversion: int = 1, point_group: str = "full") -> Sector:
    """Square-lattice J1-J2 torus, Sz=0, k=(0,0), fully symmetric characters."""
    g = lattice.torus_group(lx, ly, 0, 0, point_group, None, inversion)
    n = lx * ly
    return Sector(f"square{lx}x{ly}_j2{j2:g}", n, n // 2, g,
                  terms.heisenberg_terms(lattice.torus_bonds(lx, ly, 1.0, j2)), seed)


def batched_rings(count: int = 64, seed: int = 4, sizes=(20, 22, 24, 26, 28, 30, 32),
                  j2_max: float = 0.6) -> List[Sector]:
    """Independent ring sectors: N uniform over even sizes, J2 ~ U[0, j2_max],
    momentum k uniform in [0, N), translations only (complex characters)."""
    st = rng.Stream(seed)
    out = []
    for q in range(count):
        n = int(sizes[st.randint(0, len(sizes))])
        j2 = st.uniform(0.0, j2_max)
        k = st.randint(0, n)
        g = lattice.ring_group(n, k, 0, 0)
        out.append(Sector(f"ring{n}_k{k}_j2{j2:.3f}", n, n // 2, g,
                          terms.heisenberg_terms(lattice.ring_bonds(n, 1.0, j2)),
                          seed=seed * 1000 + q, meta={"k": k, "j2": j2}))
    return out


@dataclass
class Request:
    rid: int
    arrival: float
    sector: Sector


def serving_trace(count: int = 200, rate: float = 20.0, seed: int = 5,
                  ring_sizes=(24, 26, 28, 30, 32, 34, 36), squares=((4, 6), (6, 6)),
                  j2_max: float = 0.6) -> List[Request]:
    """Poisson arrivals of ground-state requests on fully symmetric sectors."""
    st = rng.Stream(seed)
    t = 0.0
    kinds = [("ring", n) for n in ring_sizes] + [("square", s) for s in squares]
    out = []
    for q in range(count):
        t += st.exponential(rate)
        kind, p = kinds[st.randint(0, len(kinds))]
        j2 = st.uniform(0.0, j2_max)
        if kind == "ring":
            sec = ring_symmetric(p, 0, 1, 1, j2, seed=seed * 1000 + q)
        else:
            lx, ly = p
            sec = square_j1j2(lx, ly, j2, seed=seed * 1000 + q)
        out.append(Request(q, t, sec))
    return out


def sector_from_arrays(name, n_sites, weight, perm, flip, chi, term_table, seed=0) -> Sector:
    g = lattice.Group(n_sites, np.asarray(perm, np.uint16), np.asarray(flip, np.uint8),
                      np.asarray(chi, np.float64))
    return Sector(name, n_sites, weight, g, np.asarray(term_table), seed)
