"""Spin-1/2 Hamiltonians written as a table of elementary terms.

A term (re, im, sel_mask, sel_value, flip, sign_mask) is the operator

    c * sum over s with (s & sel_mask) == sel_value of
        (-1)^popcount(s & sign_mask) |s ^ flip><s|

with c = re + i*im.  A diagonal term has flip == 0.  This is the "sum of
bit-flip and diagonal spin terms" form of the problem statement; the table
is the Hamiltonian input of both the GPU path and the oracle.

Heisenberg exchange J S_i.S_j with S = sigma/2 (fixed by the 4-site ring
ground energy -2J) is three terms:

* diagonal   J/4 * sigma^z_i sigma^z_j: c = J/4, sign = bit i | bit j;
* exchange   J/2 * (S+_i S-_j + S-_i S+_j): two terms with
  c = J/2, sel = flip = bit i | bit j, and sel_value = bit i or bit j
  (the two antiparallel configurations).
"""
from __future__ import annotations

from typing import Iterable, Tuple

import numpy as np

TERM_DTYPE = np.dtype([
    ("re", "<f8"), ("im", "<f8"),
    ("sel_mask", "<u8"), ("sel_value", "<u8"),
    ("flip", "<u8"), ("sign_mask", "<u8"),
], align=True)
assert TERM_DTYPE.itemsize == 48


def make_terms(rows: Iterable[Tuple[complex, int, int, int, int]]) -> np.ndarray:
    rows = list(rows)
    t = np.zeros(len(rows), dtype=TERM_DTYPE)
    for k, (c, sel, val, flip, sign) in enumerate(rows):
        c = complex(c)
        t[k] = (c.real, c.imag, sel, val, flip, sign)
    return t


def heisenberg_terms(bonds: Iterable[Tuple[int, int, float]]) -> np.ndarray:
    rows = []
    for i, j, J in bonds:
        if i == j:
            raise ValueError("a bond needs two distinct sites")
        bi, bj = 1 << int(i), 1 << int(j)
        rows.append((J / 4.0, 0, 0, 0, bi | bj))
    for i, j, J in bonds:
        bi, bj = 1 << int(i), 1 << int(j)
        rows.append((J / 2.0, bi | bj, bi, bi | bj, 0))
        rows.append((J / 2.0, bi | bj, bj, bi | bj, 0))
    return make_terms(rows)


def field_terms(n: int, hx: float = 0.0, hz: float = 0.0) -> np.ndarray:
    """Transverse/longitudinal fields (no U(1)): -hx sigma^x_i - hz sigma^z_i."""
    rows = []
    for i in range(n):
        b = 1 << i
        if hz:
            # sigma^z = -(-1)^bit (bit 1 = up), so -hz sigma^z = hz (-1)^bit.
            rows.append((hz, 0, 0, 0, b))
        if hx:
            rows.append((-hx, 0, 0, b, 0))
    return make_terms(rows)
