"""Push (transposed, atomic) form of the product (ls_matvec_push) against
the oracle and the pull form.  Atomic adds land in a run-dependent order, so
the comparison is to rounding: relative L2 and max-abs within 1e-12."""
import sys

import numpy as np
import pytest

import oracle
from workloads import configs, rng

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2308_16712_amd as ls  # noqa: E402
from test_gpu_parity import SMALL, MATVEC_TOL  # noqa: E402


def _close(got, want):
    scale = max(np.max(np.abs(want)), 1e-300)
    assert np.linalg.norm(got - want) <= MATVEC_TOL * max(np.linalg.norm(want), 1e-300)
    assert np.max(np.abs(got - want)) <= MATVEC_TOL * scale


@pytest.mark.parametrize("sec", SMALL, ids=lambda s: s.name)
def test_push_matches_oracle_and_pull(sec):
    print(f"[push] {sec.name}", flush=True)
    sys.stdout.flush()
    P = oracle.Problem(sec)
    reps, stab = oracle.enumerate_basis(P)
    b = ls.ls_basis_build(sec)
    op = ls.ls_operator_create(b, sec.terms)
    try:
        for nrhs in (1, 3):
            x = rng.vector(sec.seed + 60 + nrhs, len(reps), nrhs, complex_=op.is_complex)
            xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
            if len(reps) == 0:
                continue
            y_push = op.matvec_push(xt).cpu().numpy()
            y_pull = op.matvec(xt).cpu().numpy()
            _close(y_push, oracle.matvec(P, reps, stab, x))
            _close(y_push, y_pull)
    finally:
        op.close()
        b.close()


def test_push_full_square6x6():
    sec = configs.square_j1j2()
    b = ls.ls_basis_build(sec)
    op = ls.ls_operator_create(b, sec.terms)
    try:
        x = torch.from_numpy(rng.vector(13, b.dim, 1)).cuda().reshape(-1)
        _close(op.matvec_push(x).cpu().numpy(), op.matvec(x).cpu().numpy())
    finally:
        op.close()
        b.close()
