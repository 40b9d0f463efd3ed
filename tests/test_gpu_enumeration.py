"""Count-only enumeration (ls_sector_count) through the C ABI.

Bit-exact integers throughout: against the oracle's enumeration on small
sectors (whole range and split ranges, where the count below a split rank
is read off the oracle's representatives), against the character formula on
the full-size ring and torus sectors, and against the printed sector
dimensions of the paper's Table 2 for closed chains of 40-44 spins.
"""
import sys
import time
from math import comb

import numpy as np
import pytest

import oracle
import physics_ref as ref
from workloads import configs, lattice, terms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2308_16712_amd as ls  # noqa: E402
from test_gpu_parity import SMALL  # noqa: E402

U64_MAX = 2**64 - 1


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _candidates(sec):
    return comb(sec.n_sites, sec.weight) if sec.weight >= 0 else 2**sec.n_sites


def _rank(sec, s):
    return ref.colex_rank(int(s)) if sec.weight >= 0 else int(s)


@pytest.mark.parametrize("sec", SMALL, ids=lambda s: s.name)
def test_count_matches_oracle(sec):
    _say(f"[count] {sec.name}")
    want = oracle.count_basis(oracle.Problem(sec))
    got, cand = ls.ls_sector_count(sec)
    assert cand == _candidates(sec)
    assert got == want


@pytest.mark.parametrize("sec", [s for s in SMALL if s.name in
                                 ("ringD20_0pp", "ringT20_k3", "torus4x6_full", "ring40_w3_D",
                                  "torus6x6_w4_k10", "ringT10_noU1_k1", "ring32_w4_D")],
                         ids=lambda s: s.name)
def test_count_ranges(sec):
    """Counts over [0, r) equal the oracle's representatives of rank < r, and
    consecutive ranges add up; empty and out-of-range ranges count 0."""
    _say(f"[count ranges] {sec.name}")
    reps, _ = oracle.enumerate_basis(oracle.Problem(sec))
    ranks = np.sort(np.array([_rank(sec, s) for s in reps], dtype=np.uint64))
    total = _candidates(sec)
    rs = np.random.default_rng(11)
    cuts = sorted({0, total, 1, total - 1, *(int(c) for c in rs.integers(0, total, 6))})
    parts = 0
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        got, _ = ls.ls_sector_count(sec, lo, hi)
        want = int(np.searchsorted(ranks, hi, "left") - np.searchsorted(ranks, lo, "left"))
        assert got == want, (lo, hi)
        parts += got
    assert parts == len(reps)
    assert ls.ls_sector_count(sec, 5, 5)[0] == 0
    assert ls.ls_sector_count(sec, total, U64_MAX)[0] == 0
    assert ls.ls_sector_count(sec, 0, total + 12345)[0] == len(reps)


def test_count_bad_range():
    sec = SMALL[0]
    with pytest.raises(ls.LSError):
        ls.ls_sector_count(sec, 10, 9)


@pytest.mark.parametrize("sec", [configs.ring32_symmetric(), configs.square_j1j2()], ids=lambda s: s.name)
def test_count_full_size_matches_formula_and_build(sec):
    want = ref.character_dimension(sec.group, sec.weight)
    _say(f"[count full] {sec.name} want {want}")
    got, _ = ls.ls_sector_count(sec)
    assert got == want
    b = ls.ls_basis_build(sec)
    try:
        assert b.dim == want
    finally:
        b.close()


def _table2(golden_dir):
    out = {}
    for line in open(f"{golden_dir}/table2_chain_dims.txt"):
        line = line.strip()
        if line and not line.startswith("#"):
            n, d = line.split()
            out[int(n)] = int(d)
    return out


def _chain(n):
    return configs.sector_from_arrays(f"chain{n}", n, n // 2, *_chain_group(n), terms.heisenberg_terms([]))


def _chain_group(n):
    g = lattice.ring_group(n, 0, 1, 1)
    return g.perm, g.flip, g.chi


@pytest.mark.timeout(900)
@pytest.mark.parametrize("n", [40, 42, 44, 46, 48])
def test_table2_counts(golden_dir, n):
    """Closed chains, Sz = 0, D_N x Z2 fully symmetric sector: all five
    dimensions printed in Table 2, counted over every candidate (N = 48:
    C(48, 24) = 3.2e13 candidates, about three minutes, in rank slices that
    report progress)."""
    want = _table2(golden_dir)[n]
    sec = _chain(n)
    total = comb(n, n // 2)
    slices = 1 if n <= 42 else 1 << (n - 42)
    t = time.perf_counter()
    got = 0
    for k in range(slices):
        m, cand = ls.ls_sector_count(sec, total * k // slices, total * (k + 1) // slices)
        assert cand == total
        got += m
        if slices > 1:
            _say(f"[table2] N={n} slice {k + 1}/{slices} t={time.perf_counter() - t:.1f}s")
    _say(f"[table2] N={n} members={got} candidates={total} s={time.perf_counter() - t:.2f}")
    assert got == want


def test_table2_build_n40(golden_dir):
    """The stored basis of the 40-spin chain: its dimension, strictly
    increasing representatives, and the first and last few checked by the
    oracle's state_info (each is its own orbit minimum)."""
    sec = _chain(40)
    b = ls.ls_basis_build(sec)
    try:
        assert b.dim == _table2(golden_dir)[40]
        d_reps, _ = b.copy()
        # values are below 2^40: the int64 view orders them as uint64
        assert bool((d_reps[1:] > d_reps[:-1]).all())
        step = max(1, b.dim // 256)
        sample = torch.cat([d_reps[:64], d_reps[-64:], d_reps[::step]]).cpu().numpy().view(np.uint64)
        del d_reps
        r, _, norm = oracle.state_info(oracle.Problem(sec), sample)
        assert np.array_equal(r, sample) and np.all(norm > 0)
    finally:
        b.close()
