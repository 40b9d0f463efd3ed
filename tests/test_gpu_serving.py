"""Lanczos stepper and the continuous-batching serving loop on the GPU."""
import numpy as np
import pytest

import oracle
from workloads import configs, lattice, rng, terms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2308_16712_amd as ls  # noqa: E402
from paper_2308_16712_amd import serve  # noqa: E402


def _small_trace(count=8, rate=200.0, seed=9):
    st = rng.Stream(seed)
    t = 0.0
    out = []
    for q in range(count):
        t += st.exponential(rate)
        kind = st.randint(0, 4)
        j2 = st.uniform(0.0, 0.6)
        if kind == 0:
            sec = configs.ring_symmetric(16, 0, 1, 1, j2, seed=500 + q)
        elif kind == 1:
            sec = configs.ring_symmetric(20, 0, 1, 1, j2, seed=500 + q)
        elif kind == 2:
            sec = configs.square_j1j2(4, 4, j2, seed=500 + q)
        else:
            sec = configs.ring_symmetric(18, 0, 1, 1, j2, seed=500 + q)
        out.append(configs.Request(q, t, sec))
    return out


def test_stepper_matches_lanczos_alone_and_in_a_mix():
    secs = [configs.ring16_u1(), configs.ring_symmetric(20, 0, 1, 1, 0.3, seed=7),
            configs.ring_symmetric(18, 3, 0, 0, 0.2, seed=8)]          # complex sector
    ops = [ls.ls_operator_create(ls.ls_basis_build(s), s.terms) for s in secs]
    alone = [op.lanczos(40, seed=s.seed) for op, s in zip(ops, secs)]
    solvers = [ls.Solver(op, 40, seed=s.seed) for op, s in zip(ops, secs)]
    while not all(s.result()["done"] for s in solvers):
        ls.Solver.step_all(solvers)
    for a, s in zip(alone, solvers):
        r = s.result()
        assert r["iters"] == a["iters"]
        assert r["e0"] == a["e0"]                 # same arithmetic: identical
    # a solver stepped alone gives the same as in the mix
    one = ls.Solver(ops[1], 40, seed=secs[1].seed)
    while not one.result()["done"]:
        ls.Solver.step_all([one])
    assert one.result()["e0"] == solvers[1].result()["e0"]



def test_stepper_selective_matches_lanczos_alone():
    secs = [configs.ring_symmetric(20, 0, 1, 1, 0.3, seed=7),
            configs.ring_symmetric(18, 3, 0, 0, 0.2, seed=8)]          # complex sector
    ops = [ls.ls_operator_create(ls.ls_basis_build(s), s.terms) for s in secs]
    alone = [op.lanczos(40, seed=s.seed, reorth="selective") for op, s in zip(ops, secs)]
    solvers = [ls.Solver(op, 40, seed=s.seed, reorth="selective") for op, s in zip(ops, secs)]
    while not all(s.result()["done"] for s in solvers):
        ls.Solver.step_all(solvers)
    for a, s in zip(alone, solvers):
        r = s.result()
        assert r["iters"] == a["iters"]
        assert r["e0"] == a["e0"]

def test_stepper_against_oracle_lanczos():
    sec = configs.ring_symmetric(16, 0, 1, 1, 0.4, seed=3)
    P = oracle.Problem(sec)
    reps, stab = oracle.enumerate_basis(P)
    want = oracle.lanczos(lambda v: oracle.matvec(P, reps, stab, v), rng.vector(3, len(reps)), 30)
    op = ls.ls_operator_create(ls.ls_basis_build(sec), sec.terms)
    s = ls.Solver(op, 30, seed=3)
    while not s.result()["done"]:
        ls.Solver.step_all([s])
    assert abs(s.result()["e0"] - want["e0"]) < 1e-10 * max(1, abs(want["e0"]))


def test_serving_loop_admits_by_footprint_and_matches_alone():
    trace = _small_trace()
    budget = sorted(serve.footprint_bytes(r.sector, 120) for r in trace)[-1] * 2   # forces queueing
    served = serve.serve(trace, budget, max_iter=120, tol=1e-10)
    alone = serve.serve_one_at_a_time(trace, max_iter=120, tol=1e-10)
    assert len(served.records) == len(trace) == len(alone.records)
    assert served.peak_bytes <= budget
    assert served.max_active >= 2                  # requests overlapped on the device
    for a, b in zip(served.records, alone.records):
        assert a.rid == b.rid and a.converged and b.converged
        assert abs(a.e0 - b.e0) <= 1e-10 * max(1.0, abs(b.e0)), (a.name, a.e0, b.e0)
        assert a.latency > 0


def test_serving_rejects_request_larger_than_budget():
    trace = _small_trace(count=2)
    with pytest.raises(ValueError):
        serve.serve(trace, hbm_budget=1 << 20, max_iter=50)


def test_serve_with_stored_elements_matches_alone():
    """Stored products are bit-identical to generated ones, so a trace served
    with element storage returns the energies of the plain solves exactly."""
    trace = configs.serving_trace(count=12, rate=50.0, seed=9)
    trace = [r for r in trace if serve.sector_dimension(r.sector) < 2_000_000][:4]
    assert len(trace) == 4
    a = serve.serve(trace, 64 << 30, max_iter=80, tol=1e-9, store_elements=True)
    b = serve.serve_one_at_a_time(trace, max_iter=80, tol=1e-9)
    assert a.stored_bytes > 0
    for x, y in zip(a.records, b.records):
        assert x.e0 == y.e0 and x.iters == y.iters
