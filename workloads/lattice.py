"""Lattices, their bonds, and their symmetry groups with characters.

Conventions (the paper leaves them open; these are fixed here and used by
every consumer):

* Bit i of a basis state is site i; a set bit is an up spin, so the Hamming
  weight counts up spins (Section 2.1, the U(1) example).
* A group element g = (perm, flip) sends bit i of s to bit perm[i] of g.s,
  then inverts all N bits if flip is set.  Composition (g h).s = g.(h.s).
* Ring: site i, translation T: i -> i+1 (mod N).  Torus Lx x Ly: site
  x + Lx*y, translations (x, y) -> (x+a, y+b).
* Momentum character: chi(T^t) = exp(2 pi i k t / N).
* Reflection R: i -> -i (mod N); together with translations it gives all
  N maps i -> t - i.
* The group is returned as three arrays: perm uint16 [nG][N], flip uint8
  [nG], chi float64 [nG][2] (re, im).  Element 0 is the identity.

This module only *describes* the inputs (which permutations, which
characters); it does not act on basis states.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Sequence, Tuple

import numpy as np


@dataclass
class Group:
    n_sites: int
    perm: np.ndarray   # uint16 [nG][N]
    flip: np.ndarray   # uint8 [nG]
    chi: np.ndarray    # float64 [nG][2]

    @property
    def size(self) -> int:
        return int(self.perm.shape[0])

    @property
    def chi_complex(self) -> np.ndarray:
        return self.chi[:, 0] + 1j * self.chi[:, 1]


def _compose(p: Tuple[int, ...], q: Tuple[int, ...]) -> Tuple[int, ...]:
    """perm of (p o q): first q then p; site i goes to p[q[i]]."""
    return tuple(p[q[i]] for i in range(len(q)))


def close_group(n: int, generators: Sequence[Tuple[Sequence[int], int, complex]]) -> Group:
    """Close a set of generators (perm, flip, character) into a group.

    Breadth-first over products g*h with h a generator; the character of a
    new element is the product along the path that first reached it.  The
    result is not checked for consistency here (the consumers validate that
    the characters form a one-dimensional representation).
    """
    ident = tuple(range(n))
    elems: List[Tuple[Tuple[int, ...], int]] = [(ident, 0)]
    chis: List[complex] = [1.0 + 0.0j]
    seen: Dict[Tuple[Tuple[int, ...], int], int] = {(ident, 0): 0}
    gens = [(tuple(int(v) for v in p), int(f), complex(c)) for p, f, c in generators]
    head = 0
    while head < len(elems):
        p, f = elems[head]
        c = chis[head]
        head += 1
        for gp, gf, gc in gens:
            key = (_compose(gp, p), f ^ gf)
            if key not in seen:
                seen[key] = len(elems)
                elems.append(key)
                chis.append(gc * c)
    perm = np.array([e[0] for e in elems], dtype=np.uint16)
    flip = np.array([e[1] for e in elems], dtype=np.uint8)
    chi = np.array([[c.real, c.imag] for c in chis], dtype=np.float64)
    # Components within rounding of 0 or +-1 are set exactly, so characters
    # that are fourth roots of unity (k = 0, N/4, N/2, ...) are exact.
    for target in (-1.0, 0.0, 1.0):
        chi[np.abs(chi - target) < 1e-12] = target
    return Group(n, perm, flip, chi)


def trivial_group(n: int) -> Group:
    return Group(n, np.arange(n, dtype=np.uint16)[None, :], np.zeros(1, np.uint8),
                 np.array([[1.0, 0.0]]))


def _ring_generators(n: int, k: int, reflection: int, inversion: int):
    gens = []
    t = [(i + 1) % n for i in range(n)]
    gens.append((t, 0, np.exp(2j * np.pi * k / n)))
    if reflection:
        r = [(-i) % n for i in range(n)]
        gens.append((r, 0, complex(reflection)))
    if inversion:
        gens.append((list(range(n)), 1, complex(inversion)))
    return gens


def ring_group(n: int, k: int = 0, reflection: int = 0, inversion: int = 0) -> Group:
    """Translations of an N-site ring with momentum k (integer units of 2pi/N).

    ``reflection`` = 0 (not used) or the character +1/-1 of R: i -> -i,
    only meaningful for k in {0, N/2}.  ``inversion`` = 0 or the character
    of the global spin flip.  Elements are listed translation-major so that
    index = t + N * (reflection part + 2 * flip part) when all are present.
    """
    gens = _ring_generators(n, k, reflection, inversion)
    g = close_group(n, gens)
    # Re-list in a canonical order: (flip, refl, t).
    order = []
    for f in ([0, 1] if inversion else [0]):
        for rho in ([0, 1] if reflection else [0]):
            for t in range(n):
                if rho == 0:
                    p = tuple((i + t) % n for i in range(n))
                else:
                    p = tuple((t - i) % n for i in range(n))
                order.append((p, f))
    index = {(tuple(int(v) for v in g.perm[i]), int(g.flip[i])): i for i in range(g.size)}
    idx = [index[o] for o in order]
    assert len(idx) == g.size, "ring group closure mismatch"
    return Group(n, g.perm[idx].copy(), g.flip[idx].copy(), g.chi[idx].copy())


def torus_site(x: int, y: int, lx: int, ly: int) -> int:
    return (x % lx) + lx * (y % ly)


def torus_group(lx: int, ly: int, kx: int = 0, ky: int = 0, point_group: str = "full",
                point_chars: Dict[str, int] | None = None, inversion: int = 0) -> Group:
    """Translations x point group (x spin inversion) of an Lx x Ly torus.

    ``point_group``: "none", "c2v" (x and y mirrors) or "full" (D4 = C4v
    when Lx == Ly, C2v otherwise).  ``point_chars`` maps generator names
    ("mx", "my", "rot") to +-1; default all +1.  Momentum (kx, ky) in units
    of 2pi/Lx, 2pi/Ly; point-group generators are only combined with
    momenta they commute with (the caller's responsibility; inconsistent
    choices are rejected by the consumers' homomorphism check).
    """
    n = lx * ly
    pc = {"mx": 1, "my": 1, "rot": 1}
    if point_chars:
        pc.update(point_chars)
    def perm_of(fn):
        p = [0] * n
        for y in range(ly):
            for x in range(lx):
                p[torus_site(x, y, lx, ly)] = fn(x, y)
        return p
    tx = perm_of(lambda x, y: torus_site(x + 1, y, lx, ly))
    ty = perm_of(lambda x, y: torus_site(x, y + 1, lx, ly))
    gens = [(tx, 0, np.exp(2j * np.pi * kx / lx)), (ty, 0, np.exp(2j * np.pi * ky / ly))]
    if point_group in ("c2v", "full"):
        gens.append((perm_of(lambda x, y: torus_site(-x, y, lx, ly)), 0, complex(pc["mx"])))
        gens.append((perm_of(lambda x, y: torus_site(x, -y, lx, ly)), 0, complex(pc["my"])))
    if point_group == "full" and lx == ly:
        gens.append((perm_of(lambda x, y: torus_site(-y, x, lx, ly)), 0, complex(pc["rot"])))
    if inversion:
        gens.append((list(range(n)), 1, complex(inversion)))
    return close_group(n, gens)


def relabel_group(g: Group, new_of_old: Sequence[int]) -> Group:
    """The same abstract group after renaming site i to new_of_old[i].

    Useful to produce groups with no rotation structure (a scrambled site
    order) that must still give identical physics.
    """
    n = g.n_sites
    m = np.asarray(new_of_old, dtype=np.int64)
    assert sorted(m.tolist()) == list(range(n))
    # new perm: new site a = m[i] -> m[perm[i]]
    perm = np.empty_like(g.perm)
    for e in range(g.size):
        p = g.perm[e].astype(np.int64)
        perm[e, m] = m[p]
    return Group(n, perm, g.flip.copy(), g.chi.copy())


def hypercube_group(dim: int, sign: bool = False) -> Group:
    """Automorphisms of the dim-dimensional hypercube graph on 2^dim sites
    (site = a dim-bit index): XOR translations and permutations of the index
    bits, 2^dim * dim! elements.  sign: the character is the sign of the bit
    permutation (trivial on the translations), else 1."""
    n = 1 << dim

    def bitperm(dest):   # bit b of the index moves to bit dest[b]
        return [sum(((s >> b) & 1) << dest[b] for b in range(dim)) for s in range(n)]

    gens = [([s ^ (1 << k) for s in range(n)], 0, 1.0) for k in range(dim)]
    swap = list(range(dim))
    swap[0], swap[1] = 1, 0
    gens.append((bitperm(swap), 0, -1.0 if sign else 1.0))
    cycle = [(b + 1) % dim for b in range(dim)]
    gens.append((bitperm(cycle), 0, 1.0 if dim % 2 == 1 else (-1.0 if sign else 1.0)))
    return close_group(n, gens)


def hypercube_bonds(dim: int, j1: float = 1.0, j2: float = 0.0) -> List[Tuple[int, int, float]]:
    """Pairs of sites at Hamming distance 1 (j1) and 2 (j2) of their indices."""
    n = 1 << dim
    out = []
    for a in range(n):
        for b in range(a + 1, n):
            d = bin(a ^ b).count("1")
            if d == 1:
                out.append((a, b, j1))
            elif d == 2 and j2 != 0.0:
                out.append((a, b, j2))
    return out


def ring_bonds(n: int, j1: float = 1.0, j2: float = 0.0) -> List[Tuple[int, int, float]]:
    bonds = [(i, (i + 1) % n, j1) for i in range(n)]
    if j2 != 0.0:
        bonds += [(i, (i + 2) % n, j2) for i in range(n)]
    return bonds


def torus_bonds(lx: int, ly: int, j1: float = 1.0, j2: float = 0.0) -> List[Tuple[int, int, float]]:
    bonds = []
    for y in range(ly):
        for x in range(lx):
            i = torus_site(x, y, lx, ly)
            bonds.append((i, torus_site(x + 1, y, lx, ly), j1))
            bonds.append((i, torus_site(x, y + 1, lx, ly), j1))
    if j2 != 0.0:
        for y in range(ly):
            for x in range(lx):
                i = torus_site(x, y, lx, ly)
                bonds.append((i, torus_site(x + 1, y + 1, lx, ly), j2))
                bonds.append((i, torus_site(x + 1, y - 1, lx, ly), j2))
    return bonds


def relabel_bonds(bonds, new_of_old):
    return [(int(new_of_old[i]), int(new_of_old[j]), J) for i, j, J in bonds]
