"""A large non-abelian group on the generic orbit walk (C ABI: ls_basis_build,
ls_matvec, ls_operator_store).

The hypercube's automorphisms (XOR translations and permutations of the
site-index bits) have no ring or torus structure, so the products take the
generic walk over coset representatives.  On 32 sites the group has 3840
elements, whose order has 36 divisors: the element normalisation
sqrt(stab_j / stab_i) is divided out per element (no stabilizer-ratio
table); on 16 sites (384 elements) it comes from the table.  Trivial and
sign characters; many distinct stabilizer sizes.  Basis bit-exact, products
to the tolerance against the oracle (Section 5.3's row form), and the stored
product equal to the generated one.
"""
import sys

import numpy as np
import pytest

from workloads import configs, lattice, rng, terms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2308_16712_amd as ls  # noqa: E402

MATVEC_TOL = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sectors():
    out = []
    for dim, w, sign in ((4, 8, False), (4, 8, True), (5, 5, False), (5, 6, True)):
        g = lattice.hypercube_group(dim, sign)
        name = f"hypercube{dim}_w{w}_{'sign' if sign else 'trivial'}"
        out.append(configs.sector_from_arrays(name, 1 << dim, w, g.perm, g.flip, g.chi,
                                              terms.heisenberg_terms(lattice.hypercube_bonds(dim, 1.0, 0.3))))
    return out


SECTORS = _sectors()


@pytest.mark.parametrize("sec", SECTORS, ids=lambda s: s.name)
def test_hypercube_group_parity(sec):
    _say(f"[gpu] hypercube sector {sec.name} (|G| = {sec.group.size})")
    P = oracle.Problem(sec)
    reps, stab = oracle.enumerate_basis(P)
    b = ls.ls_basis_build(sec)
    assert b.dim == len(reps) > 0
    g_reps, g_stab = b.copy()
    assert np.array_equal(g_reps.cpu().numpy().view(np.uint64), reps)
    assert np.array_equal(g_stab.cpu().numpy().view(np.uint16), stab)
    if np.all(sec.group.chi[:, 0] == 1.0):
        assert len(set(stab.tolist())) >= 8      # many stabilizer sizes meet in the products
    op = ls.ls_operator_create(b, sec.terms)
    for nrhs in (1, 4):
        x = rng.vector(sec.seed + 31 + nrhs, len(reps), nrhs, complex_=op.is_complex)
        y_ref = oracle.matvec(P, reps, stab, x)
        y = op.matvec(torch.from_numpy(np.ascontiguousarray(x)).cuda()).cpu().numpy()
        rel = np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)
        assert rel <= MATVEC_TOL, (nrhs, rel)
        assert np.max(np.abs(y - y_ref)) <= MATVEC_TOL * np.max(np.abs(y_ref))
    op.check()
    x = torch.from_numpy(rng.vector(sec.seed + 5, len(reps), complex_=op.is_complex)).cuda()
    y = op.matvec(x)
    st = ls.ls_operator_create(b, sec.terms)
    ls.ls_operator_store(st)
    assert torch.equal(st.matvec(x), y)
    st.close()
    op.close()
    b.close()
