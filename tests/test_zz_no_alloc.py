"""ls_sector_count_noalloc (no device allocation; the group's tables and the
accumulator live in a static device array) against ls_sector_count, through
the C ABI: several calls in a row, each smaller than the one before, on
sectors that use every table the count reads (pair table of a torus,
complex characters, a rank sub-range), and the refusal of a group whose
tables exceed the array."""
import ctypes
import sys

import numpy as np
import pytest

import physics_ref as ref
from workloads import configs, lattice, terms

pytestmark = pytest.mark.gpu

from paper_2308_16712_amd import _lib  # noqa: E402


def _desc(sec):
    g = sec.group
    keep = (np.ascontiguousarray(g.perm, np.uint16), np.ascontiguousarray(g.flip, np.uint8),
            np.ascontiguousarray(g.chi, np.float64))
    d = _lib.SectorDesc(sec.n_sites, sec.weight, keep[0].shape[0], keep[0].ctypes.data, keep[1].ctypes.data,
                        keep[2].ctypes.data)
    return d, keep


def _count(fn, sec, lo=0, hi=2 ** 64 - 1):
    d, keep = _desc(sec)
    m, c = ctypes.c_uint64(), ctypes.c_uint64()
    st = fn(ctypes.byref(d), lo, hi, ctypes.byref(m), ctypes.byref(c), None)
    return st, m.value, c.value


def _sector(name, n, w, g, bonds):
    return configs.sector_from_arrays(name, n, w, g.perm, g.flip, g.chi, terms.heisenberg_terms(bonds))


def test_noalloc_count_equals_allocating_count():
    import torch
    torch.cuda.init()
    L = _lib.load()
    cases = [
        # the 4x6 torus with its full group: pair table, 8 coset representatives
        (_sector("torus4x6_full", 24, 12, lattice.torus_group(6, 4, 0, 0, "full", None, 1),
                 lattice.torus_bonds(6, 4, 1.0, 0.35)), None),
        # smaller: a 20-site ring at momentum 3 (complex characters)
        (_sector("ringT20_k3", 20, 10, lattice.ring_group(20, 3), lattice.ring_bonds(20, 1.0, 0.45)), None),
        # smaller again: a rank slice of the 32-site symmetric ring
        (configs.ring32_symmetric(), (123456789, 123456789 + 4000000)),
        # and a slice of the 6x6 torus (pair table again, 64-bit words)
        (configs.square_j1j2(), (10 ** 9, 10 ** 9 + 3000000)),
    ]
    for sec, rng_ in cases:
        lo, hi = rng_ if rng_ else (0, 2 ** 64 - 1)
        print(f"[gpu] noalloc count {sec.name} ranks [{lo}, {min(hi, 2**63)})", flush=True)
        sys.stdout.flush()
        st0, m0, c0 = _count(L.ls_sector_count, sec, lo, hi)
        st1, m1, c1 = _count(L.ls_sector_count_noalloc, sec, lo, hi)
        assert st0 == 0 and st1 == 0, L.ls_last_error()
        assert (m1, c1) == (m0, c0)
        if rng_ is None:
            assert m1 == ref.character_dimension(sec.group, sec.weight)
    # the same call again after the others: the array is rewritten and the
    # accumulator cleared
    sec = cases[1][0]
    assert _count(L.ls_sector_count_noalloc, sec)[1] == ref.character_dimension(sec.group, sec.weight)


def test_noalloc_count_refuses_tables_above_the_array():
    """(Z2)^12 of independent pair swaps on 24 sites: 4096 elements and no
    lattice translations, so 4096 coset representatives (393 KB of tables),
    above the 256 KiB array.  The allocating count handles it."""
    import torch
    torch.cuda.init()
    L = _lib.load()
    n = 24
    perms = []
    for m in range(1 << 12):
        p = list(range(n))
        for i in range(12):
            if (m >> i) & 1:
                p[2 * i], p[2 * i + 1] = 2 * i + 1, 2 * i
        perms.append(p)
    g = lattice.Group(n, np.array(perms, dtype=np.uint16), np.zeros(len(perms), np.uint8),
                      np.tile([1.0, 0.0], (len(perms), 1)))
    sec = configs.sector_from_arrays("pairswaps24", n, 12, g.perm, g.flip, g.chi, terms.heisenberg_terms([]))
    st, m, c = _count(L.ls_sector_count_noalloc, sec)
    assert st == _lib.LS_EINVAL
    assert b"scratch" in L.ls_last_error()
    st0, m0, c0 = _count(L.ls_sector_count, sec)
    assert st0 == 0 and m0 == ref.character_dimension(g, 12)
