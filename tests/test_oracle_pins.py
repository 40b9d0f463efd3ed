"""Pins of the oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (Table 2, the four-spin example of Section 2.1), closed forms,
invariants, full-space constructions built independently in
``physics_ref.py``, or a published generator test vector.
"""
import math
from math import comb

import numpy as np
import pytest

import oracle
import physics_ref as ref
from workloads import configs, lattice, rng, terms


def _sector(n, w, group, bonds=None, term_table=None, name="t"):
    tt = term_table if term_table is not None else terms.heisenberg_terms(bonds or [])
    return configs.sector_from_arrays(name, n, w, group.perm, group.flip, group.chi, tt)


def _read_golden(path):
    rows = []
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


# ---------------------------------------------------------------- Section 2.1, Fig. 1

def test_fig1_four_spins(golden_dir):
    rows = {r[0]: [int(v) for v in r[1:]] for r in _read_golden(f"{golden_dir}/fig1_four_spins.txt")}
    g = lattice.ring_group(4, 0)
    P = oracle.Problem(_sector(4, -1, g, lattice.ring_bonds(4)))
    reps, _ = oracle.enumerate_basis(P)
    assert len(reps) == 6                      # "from 16 to 6"
    assert reps.tolist() == rows["translations"]
    P = oracle.Problem(_sector(4, 2, lattice.trivial_group(4), lattice.ring_bonds(4)))
    reps, stab = oracle.enumerate_basis(P)
    assert len(reps) == comb(4, 2) == 6        # C(4,2)
    assert reps.tolist() == rows["u1_weight2"]
    assert np.all(stab == 1)


# ---------------------------------------------------------------- Table 2

def test_table2_dimensions_by_character_formula(golden_dir):
    """The closed-form sector dimension reproduces the paper's printed
    integers; this pins the formula used below to pin the oracle's counts."""
    for n_s, d_s in _read_golden(f"{golden_dir}/table2_chain_dims.txt"):
        n, d = int(n_s), int(d_s)
        g = lattice.ring_group(n, 0, 1, 1)
        assert g.size == 4 * n
        assert ref.character_dimension(g, n // 2) == d


@pytest.mark.parametrize("n", [8, 10, 12, 14, 16, 18])
def test_enumeration_count_matches_character_formula(n):
    ks = [0, n // 2, 1] if n <= 12 else [0, 1]
    for k in ks:
        for r in ([1, -1] if k in (0, n // 2) else [0]):
            for z in (1, -1):
                g = lattice.ring_group(n, k, r, z)
                P = oracle.Problem(_sector(n, n // 2, g, lattice.ring_bonds(n)))
                assert oracle.count_basis(P) == ref.character_dimension(g, n // 2), (n, k, r, z)


@pytest.mark.parametrize("dim,w", [(3, 4), (4, 6), (4, 8), (5, 5)])
def test_enumeration_count_hypercube(dim, w):
    """A non-abelian group with many stabilizer sizes: the hypercube's
    automorphisms (2^dim * dim! elements), trivial and sign characters."""
    n = 1 << dim
    for sign in (False, True):
        g = lattice.hypercube_group(dim, sign)
        assert g.size == n * math.factorial(dim)
        P = oracle.Problem(_sector(n, w, g, lattice.hypercube_bonds(dim, 1.0, 0.3)))
        reps, stab = oracle.enumerate_basis(P)
        assert len(reps) == ref.character_dimension(g, w), (dim, w, sign)
        assert all(g.size % int(st) == 0 for st in stab)


@pytest.mark.parametrize("lx,ly,w", [(3, 3, 4), (4, 3, 6), (4, 4, 8), (2, 4, 4), (4, 4, 7)])
def test_enumeration_count_torus(lx, ly, w):
    n = lx * ly
    for inv in ([0, 1] if 2 * w == n else [0]):
        g = lattice.torus_group(lx, ly, 0, 0, "full", None, inv)
        P = oracle.Problem(_sector(n, w, g, lattice.torus_bonds(lx, ly)))
        assert oracle.count_basis(P) == ref.character_dimension(g, w)


@pytest.mark.parametrize("n", [6, 8, 9, 10])
def test_dimensions_sum_to_binomial_abelian(n):
    """Translations (x inversion): the sectors of all characters partition
    the weight-w space."""
    for w in range(n + 1):
        tot = 0
        for k in range(n):
            tot += oracle.count_basis(oracle.Problem(_sector(n, w, lattice.ring_group(n, k),
                                                             lattice.ring_bonds(n))))
        assert tot == comb(n, w)
    if n % 2 == 0:
        tot = 0
        for k in range(n):
            for z in (1, -1):
                tot += oracle.count_basis(oracle.Problem(
                    _sector(n, n // 2, lattice.ring_group(n, k, 0, z), lattice.ring_bonds(n))))
        assert tot == comb(n, n // 2)


# ---------------------------------------------------------------- term table

@pytest.mark.parametrize("n", [3, 4, 5])
def test_heisenberg_terms_match_pauli_construction(n):
    """The term encoding reproduces J S_i.S_j built from Pauli matrices."""
    bonds = [(0, 1, 1.0), (1, 2, 0.7)] + ([(0, n - 1, -0.3)] if n > 3 else [])
    tt = terms.heisenberg_terms(bonds)
    H = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    for t in tt:
        c = t["re"] + 1j * t["im"]
        for s in range(2 ** n):
            if (s & int(t["sel_mask"])) != int(t["sel_value"]):
                continue
            sign = -1.0 if bin(s & int(t["sign_mask"])).count("1") % 2 else 1.0
            H[s ^ int(t["flip"]), s] += c * sign
    assert np.allclose(H, ref.heisenberg_full(n, bonds), atol=1e-14)


# ---------------------------------------------------------------- dense checks

def _dense_cases():
    cases = []
    for n in (6, 8):
        for k in range(n):
            cases.append((f"ringT{n}_k{k}", n, n // 2, lattice.ring_group(n, k), lattice.ring_bonds(n, 1.0, 0.3)))
        for k in (0, n // 2):
            for r in (1, -1):
                for z in (1, -1):
                    cases.append((f"ringD{n}_{k}{r}{z}", n, n // 2, lattice.ring_group(n, k, r, z),
                                  lattice.ring_bonds(n, 1.0, 0.4)))
    cases.append(("ring7_w3_k2", 7, 3, lattice.ring_group(7, 2), lattice.ring_bonds(7, 1.0, 0.25)))
    cases.append(("ring9_w4_k3", 9, 4, lattice.ring_group(9, 3), lattice.ring_bonds(9, 1.0, 0.1)))
    cases.append(("torus3x3_w4", 9, 4, lattice.torus_group(3, 3), lattice.torus_bonds(3, 3, 1.0, 0.5)))
    g = lattice.torus_group(2, 4, 0, 0, "full", None, 1)
    cases.append(("torus2x4_z", 8, 4, g, lattice.torus_bonds(2, 4, 1.0, 0.5)))
    g = lattice.torus_group(3, 3, 1, 2, "none")
    cases.append(("torus3x3_k12", 9, 4, g, lattice.torus_bonds(3, 3, 1.0, 0.5)))
    perm = [3, 7, 0, 5, 1, 6, 2, 4]
    g = lattice.relabel_group(lattice.ring_group(8, 2), perm)
    cases.append(("scrambled8_k2", 8, 4, g, lattice.relabel_bonds(lattice.ring_bonds(8, 1.0, 0.3), perm)))
    return cases


@pytest.mark.parametrize("case", _dense_cases(), ids=lambda c: c[0])
def test_sector_matrix_equals_projected_full_hamiltonian(case):
    """Oracle column-form matrix == B^dagger H_full B with B from the projector."""
    name, n, w, g, bonds = case
    sec = _sector(n, w, g, bonds)
    P = oracle.Problem(sec)
    reps, stab = oracle.enumerate_basis(P)
    if len(reps) == 0:
        return
    Hs = oracle.dense(P, reps, stab)
    B = ref.sector_basis(n, w, g, reps)
    Hf = ref.heisenberg_full(n, bonds)
    Href = B.conj().T @ Hf @ B
    assert np.allclose(Hs, Href, atol=1e-12), np.abs(Hs - Href).max()
    assert np.allclose(Hs, Hs.conj().T, atol=1e-13)
    # the columns of B are orthonormal and in the sector
    assert np.allclose(B.conj().T @ B, np.eye(len(reps)), atol=1e-12)
    # stabilizer sizes match the norm of P|r>: ||P|r>||^2 = stab/|G|, and
    # each is the order of a subgroup, so it divides |G| (Lagrange)
    Pm = ref.projector(n, g)
    for r, st in zip(reps, stab):
        assert abs(np.linalg.norm(Pm[:, int(r)]) ** 2 - st / g.size) < 1e-12
        assert g.size % int(st) == 0


@pytest.mark.parametrize("case", _dense_cases()[:12], ids=lambda c: c[0])
def test_get_row_equals_column_form(case):
    """Pull form (getRow, Section 5.3 first listing) equals push form."""
    name, n, w, g, bonds = case
    P = oracle.Problem(_sector(n, w, g, bonds))
    reps, stab = oracle.enumerate_basis(P)
    Hs = oracle.dense(P, reps, stab)
    idx = {int(r): i for i, r in enumerate(reps)}
    Hr = np.zeros_like(Hs)
    for i, r in enumerate(reps):
        rr, cc = oracle.get_row(P, int(r))
        for a, c in zip(rr, cc):
            Hr[i, idx[int(a)]] += c
    assert np.allclose(Hr, Hs, atol=1e-13)


@pytest.mark.parametrize("n", [6, 8, 10])
def test_union_of_sector_spectra_is_full_spectrum(n):
    """Abelian groups T and T x Z2: the sector spectra together are the
    spectrum of H on the whole weight-n/2 space."""
    bonds = lattice.ring_bonds(n, 1.0, 0.35)
    states = ref.weight_states(n, n // 2)
    Hf = ref.heisenberg_full(n, bonds)[np.ix_(states, states)]
    full = np.sort(np.linalg.eigvalsh(Hf))
    for with_z in (False, True):
        ev = []
        for k in range(n):
            for z in ((1, -1) if with_z else (0,)):
                P = oracle.Problem(_sector(n, n // 2, lattice.ring_group(n, k, 0, z), bonds))
                reps, stab = oracle.enumerate_basis(P)
                if len(reps):
                    ev.extend(np.linalg.eigvalsh(oracle.dense(P, reps, stab)))
        assert np.allclose(np.sort(ev), full, atol=1e-11)


def test_nonabelian_sector_spectrum_contained_in_full():
    n = 10
    bonds = lattice.ring_bonds(n, 1.0, 0.2)
    states = ref.weight_states(n, n // 2)
    full = np.linalg.eigvalsh(ref.heisenberg_full(n, bonds)[np.ix_(states, states)])
    for k in (0, n // 2):
        for r in (1, -1):
            for z in (1, -1):
                P = oracle.Problem(_sector(n, n // 2, lattice.ring_group(n, k, r, z), bonds))
                reps, stab = oracle.enumerate_basis(P)
                for e in np.linalg.eigvalsh(oracle.dense(P, reps, stab)):
                    assert np.min(np.abs(full - e)) < 1e-10


# ---------------------------------------------------------------- closed forms

def _e0(n, w, g, bonds):
    P = oracle.Problem(_sector(n, w, g, bonds))
    reps, stab = oracle.enumerate_basis(P)
    if len(reps) == 0:
        return np.inf
    return np.linalg.eigvalsh(oracle.dense(P, reps, stab))[0]


@pytest.mark.parametrize("J", [1.0, 2.5])
def test_closed_form_energies(J):
    # four-site ring: E0 = -2J (with and without symmetries)
    assert abs(_e0(4, 2, lattice.trivial_group(4), lattice.ring_bonds(4, J)) + 2 * J) < 1e-12
    assert abs(_e0(4, 2, lattice.ring_group(4, 0, 1, 1), lattice.ring_bonds(4, J)) + 2 * J) < 1e-12
    # one bond: singlet at -3J/4
    assert abs(_e0(2, 1, lattice.trivial_group(2), [(0, 1, J)]) + 0.75 * J) < 1e-12
    # triangle at weight 1: J/2 (S(S+1) - 9/4) with S = 1/2
    tri = [(0, 1, J), (1, 2, J), (0, 2, J)]
    assert abs(_e0(3, 1, lattice.trivial_group(3), tri) + 0.75 * J) < 1e-12


@pytest.mark.parametrize("n", [8, 10, 12])
def test_majumdar_ghosh_point(n):
    """J2 = J1/2 on an even ring: E0 = -3 N J1 / 8 (dimer product), both on
    the whole Sz=0 space and as the lowest of the D_N x Z2 sector energies."""
    bonds = lattice.ring_bonds(n, 1.0, 0.5)
    e_all = _e0(n, n // 2, lattice.trivial_group(n), bonds)
    e_sym = min(_e0(n, n // 2, lattice.ring_group(n, k, r, z), bonds)
                for k in (0, n // 2) for r in (1, -1) for z in (1, -1))
    assert abs(e_all + 3 * n / 8) < 1e-10
    assert abs(e_sym + 3 * n / 8) < 1e-10


@pytest.mark.parametrize("n", [6, 8, 10])
def test_bethe_ansatz_matches_full_space_ground_energy(n):
    """The Bethe-ansatz ground energy of the closed chain equals the lowest
    eigenvalue of the Sz=0 block of the full 2^n Hamiltonian built from Pauli
    matrices (no oracle code involved)."""
    H = ref.heisenberg_full(n, lattice.ring_bonds(n, 1.0))
    idx = ref.weight_states(n, n // 2)
    e_full = np.linalg.eigvalsh(H[np.ix_(idx, idx)])[0]
    assert abs(ref.bethe_ground_energy(n) - e_full) < 1e-11


def test_bethe_ansatz_closed_form_and_oracle_sector():
    """n = 4: E0 = -2J.  n = 8, 12 (n divisible by 4, ground state at k = 0,
    even under reflection and spin inversion): the oracle's (k=0, R=+1,
    Z=+1) sector has the Bethe-ansatz energy as its lowest eigenvalue."""
    assert abs(ref.bethe_ground_energy(4) + 2.0) < 1e-14
    assert abs(ref.bethe_ground_energy(4, 2.5) + 5.0) < 1e-13
    for n in (8, 12):
        e = _e0(n, n // 2, lattice.ring_group(n, 0, 1, 1), lattice.ring_bonds(n, 1.0))
        assert abs(e - ref.bethe_ground_energy(n)) < 1e-11


def test_hermiticity_random_vectors():
    for g, n, bonds in [(lattice.ring_group(10, 3), 10, lattice.ring_bonds(10, 1.0, 0.3)),
                        (lattice.torus_group(4, 3), 12, lattice.torus_bonds(4, 3, 1.0, 0.5))]:
        P = oracle.Problem(_sector(n, n // 2, g, bonds))
        reps, stab = oracle.enumerate_basis(P)
        u = rng.uniform_pm1_complex(11, len(reps))
        v = rng.uniform_pm1_complex(12, len(reps))
        lhs = np.vdot(u, oracle.matvec(P, reps, stab, v))
        rhs = np.vdot(oracle.matvec(P, reps, stab, u), v)
        assert abs(lhs - rhs) < 1e-11 * max(1, abs(lhs))


# ---------------------------------------------------------------- state info / index

@pytest.mark.parametrize("case", _dense_cases()[::5], ids=lambda c: c[0])
def test_state_info_brute_force(case):
    """rep = min over the orbit, norm = ||P|s>||-consistent, chi = character
    of the element bringing s to its representative (from U_g matrices)."""
    name, n, w, g, bonds = case
    P = oracle.Problem(_sector(n, w, g, bonds))
    states = np.arange(2 ** n, dtype=np.uint64)
    reps, chi, norm = oracle.state_info(P, states)
    ch = g.chi[:, 0] + 1j * g.chi[:, 1]
    s_all = np.arange(2 ** n, dtype=np.int64)
    images = []
    for e in range(g.size):
        t = np.zeros_like(s_all)
        for i in range(n):
            t |= ((s_all >> i) & 1) << int(g.perm[e, i])
        if g.flip[e]:
            t ^= (1 << n) - 1
        images.append(t)
    images = np.stack(images)                       # [nG][2^n]
    rmin = images.min(axis=0)
    assert np.array_equal(reps.astype(np.int64), rmin)
    Pm = ref.projector(n, g)
    for s in range(2 ** n):
        wt = bin(s).count("1")
        r = int(rmin[s])
        nr = np.linalg.norm(Pm[:, r])
        in_sector = (w < 0 or wt == w) and nr > 1e-9
        if not in_sector:
            assert norm[s] == 0.0 and chi[s] == 0
            continue
        assert abs(norm[s] - nr) < 1e-14
        # U_g* |s> = |r> and P U_g = chi(g) P give P|s> = conj(chi(g*)) P|r>
        assert np.allclose(Pm[:, s], np.conj(chi[s]) * Pm[:, r], atol=1e-12)


def test_index_is_colex_rank_for_u1_only_basis():
    for n, w in [(10, 5), (12, 4), (16, 8)]:
        P = oracle.Problem(_sector(n, w, lattice.trivial_group(n), lattice.ring_bonds(n)))
        reps, _ = oracle.enumerate_basis(P)
        assert len(reps) == comb(n, w)
        sample = reps[:: max(1, len(reps) // 500)]
        got = oracle.index_lookup(reps, sample)
        assert [ref.colex_rank(int(s)) for s in sample] == got.tolist()
        absent = np.array([(1 << w) - 1 << 1 | 1, 0], dtype=np.uint64)  # wrong weight
        assert oracle.index_lookup(reps, absent).tolist() == [-1, -1]


def test_threaded_state_info_and_rows_match_serial():
    """Splitting the oracle's state_info and getRow over host threads changes
    nothing: the same representatives, characters, norms and rows."""
    sec = _sector(14, 7, lattice.ring_group(14, 3, 0, 0), lattice.ring_bonds(14, 1.0, 0.3))
    P = oracle.Problem(sec)
    st = rng.counter_u64(5, np.arange(20000, dtype=np.uint64)) & np.uint64((1 << 14) - 1)
    a = oracle.state_info(P, st)
    b = oracle.state_info(P, st, workers=4)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    reps, _ = oracle.enumerate_basis(P)
    rows1 = [oracle.get_row(P, int(r)) for r in reps[:300]]
    rows4 = oracle.get_rows(P, reps[:300], workers=4)
    for (n1, c1), (n4, c4) in zip(rows1, rows4):
        assert np.array_equal(n1, n4) and np.array_equal(c1, c4)


@pytest.mark.parametrize("case", ["ring12_D", "ring12_k5", "torus4x3"])
def test_sparse_matrix_equals_column_product(case):
    """The sparse matrix assembled from getRow applies H like the
    column-by-column product (real and complex sectors)."""
    g, n, bonds = {
        "ring12_D": (lattice.ring_group(12, 0, 1, 1), 12, lattice.ring_bonds(12, 1.0, 0.4)),
        "ring12_k5": (lattice.ring_group(12, 5), 12, lattice.ring_bonds(12, 1.0, 0.2)),
        "torus4x3": (lattice.torus_group(4, 3), 12, lattice.torus_bonds(4, 3, 1.0, 0.5)),
    }[case]
    P = oracle.Problem(_sector(n, n // 2, g, bonds))
    reps, stab = oracle.enumerate_basis(P)
    H = oracle.sparse_matrix(P, reps, workers=2)
    x = rng.vector(4, len(reps), 3, complex_=not P.is_real)
    y = oracle.matvec(P, reps, stab, x)
    assert np.linalg.norm(H @ x - y) <= 1e-13 * np.linalg.norm(y)
    assert (H - H.conj().T).count_nonzero() == 0 or abs(H - H.conj().T).max() < 1e-14


# ---------------------------------------------------------------- Lanczos

def test_lanczos_converges_to_dense_ground_energy():
    n = 12
    sec = _sector(n, n // 2, lattice.ring_group(n, 0, 1, 1), lattice.ring_bonds(n, 1.0, 0.3))
    P = oracle.Problem(sec)
    reps, stab = oracle.enumerate_basis(P)
    e_dense = np.linalg.eigvalsh(oracle.dense(P, reps, stab))[0]
    v0 = rng.vector(7, len(reps))
    res = oracle.lanczos(lambda v: oracle.matvec(P, reps, stab, v), v0, min(60, len(reps)))
    assert abs(res["e0"] - e_dense) < 1e-10


def test_lanczos_ring16_against_full_space_sparse():
    """N=16 ring, Sz=0, no lattice symmetry: the oracle's Lanczos ground
    energy equals the lowest eigenvalue of the full 2^16-dimensional sparse
    Hamiltonian built independently (scipy eigsh)."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import eigsh
    n = 16
    s = np.arange(2 ** n, dtype=np.int64)
    rows, cols, vals = [], [], []
    diag = np.zeros(2 ** n)
    for i, j, J in lattice.ring_bonds(n):
        bi, bj = (s >> i) & 1, (s >> j) & 1
        diag += J / 4.0 * np.where(bi == bj, 1.0, -1.0)
        m = bi != bj
        rows.append(s[m] ^ ((1 << i) | (1 << j)))
        cols.append(s[m])
        vals.append(np.full(m.sum(), J / 2.0))
    H = sp.csr_matrix((np.concatenate(vals + [diag]),
                       (np.concatenate(rows + [s]), np.concatenate(cols + [s]))),
                      shape=(2 ** n, 2 ** n))
    e_full = eigsh(H, k=1, which="SA", tol=1e-14)[0][0]
    sec = configs.ring16_u1()
    P = oracle.Problem(sec)
    reps, stab = oracle.enumerate_basis(P)
    res = oracle.lanczos(lambda v: oracle.matvec(P, reps, stab, v), rng.vector(1, len(reps)), 80)
    assert abs(res["e0"] - e_full) < 1e-10
    # and the Bethe-ansatz value for the 16-site chain
    assert abs(ref.bethe_ground_energy(16) - e_full) < 1e-10



def test_cgs_selective_decision_and_result():
    """The selective pass (DGKS, eta^2 = 1/2): a vector far from span(V) gets
    one pass and is orthogonal to V afterwards; a vector almost inside span(V)
    loses most of its norm in the first pass and gets the second one."""
    g = np.random.default_rng(11)
    Vm = np.linalg.qr(g.standard_normal((40, 6)))[0].T          # 6 orthonormal rows
    far = g.standard_normal(40)
    w, passes = oracle.cgs_selective(Vm, far)
    assert passes == 1 and np.abs(Vm @ w).max() < 1e-13
    near = Vm.T @ g.standard_normal(6) + 1e-3 * g.standard_normal(40)
    w, passes = oracle.cgs_selective(Vm, near)
    assert passes == 2 and np.abs(Vm @ w).max() < 1e-16 * 40
    # the result is the component of w outside span(V), as projecting by hand gives
    ref = near - Vm.T @ (Vm @ near)
    assert np.allclose(w, ref, rtol=0, atol=1e-15)


def test_lanczos_selective_matches_dense_and_full_cgs2():
    n = 12
    sec = _sector(n, n // 2, lattice.ring_group(n, 0, 1, 1), lattice.ring_bonds(n, 1.0, 0.3))
    P = oracle.Problem(sec)
    reps, stab = oracle.enumerate_basis(P)
    e_dense = np.linalg.eigvalsh(oracle.dense(P, reps, stab))[0]
    v0 = rng.vector(7, len(reps))
    apply_h = lambda v: oracle.matvec(P, reps, stab, v)
    sel = oracle.lanczos(apply_h, v0, min(60, len(reps)), reorth="selective")
    full = oracle.lanczos(apply_h, v0, min(60, len(reps)))
    assert abs(sel["e0"] - e_dense) < 1e-10
    k = min(len(sel["alpha"]), 20)
    assert np.allclose(sel["alpha"][:k], full["alpha"][:k], rtol=0, atol=1e-11)

# ---------------------------------------------------------------- generator

def test_counter_generator_matches_published_splitmix64(golden_dir):
    want = [int(r[0]) for r in _read_golden(f"{golden_dir}/splitmix64_seed1234567.txt")]
    st = rng.Stream(1234567)
    assert [st.u64() for _ in range(5)] == want
    got = rng.counter_u64(1234567, np.arange(5, dtype=np.uint64))
    assert got.tolist() == want


def test_state_values_torch_matches_numpy():
    """The tensor form of the state-keyed generator (used to fill full-size
    vectors on the device) draws the same numbers as the numpy form."""
    import torch
    st = rng.counter_u64(77, np.arange(5000, dtype=np.uint64))
    st = np.concatenate([st, st >> np.uint64(20), np.array([0, 1, (1 << 63), (1 << 64) - 1], dtype=np.uint64)])
    want = rng.state_values(11, st)
    got = rng.state_values_torch(11, torch.from_numpy(st.view(np.int64))).numpy()
    assert np.array_equal(got, want)
