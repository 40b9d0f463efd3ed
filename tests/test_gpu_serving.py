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


_EXACT = {}


def _exact_e0(sec):
    """Lowest eigenvalue of the oracle's sector Hamiltonian (its getRow
    matrix, diagonalised densely)."""
    if sec.name not in _EXACT:
        P = oracle.Problem(sec)
        reps, _ = oracle.enumerate_basis(P)
        H = oracle.sparse_matrix(P, reps, workers=0).toarray()
        _EXACT[sec.name] = float(np.linalg.eigvalsh(H)[0])
    return _EXACT[sec.name]


def test_serving_loop_admits_by_footprint_and_matches_alone():
    trace = _small_trace()
    budget = sorted(serve.footprint_bytes(r.sector, 120) for r in trace)[-1] * 2   # forces queueing
    served = serve.serve(trace, budget, max_iter=120, tol=1e-10)
    alone = serve.serve_one_at_a_time(trace, max_iter=120, tol=1e-10)
    assert len(served.records) == len(trace) == len(alone.records)
    assert served.peak_bytes <= budget
    assert served.max_active >= 2                  # requests overlapped on the device
    for req, a, b in zip(sorted(trace, key=lambda r: r.rid), served.records, alone.records):
        assert a.rid == b.rid == req.rid and a.status == b.status == "ok"
        assert a.converged and b.converged
        assert abs(a.e0 - b.e0) <= 1e-10 * max(1.0, abs(b.e0)), (a.name, a.e0, b.e0)
        # the converged solve reaches the sector's ground energy (oracle, dense)
        e = _exact_e0(req.sector)
        assert abs(a.e0 - e) <= 1e-9 * max(1.0, abs(e)), (a.name, a.e0, e)
        assert a.latency > 0


def test_serving_rejects_request_larger_than_budget():
    """A request that can never fit is rejected on arrival and recorded; the
    loop does not raise."""
    trace = _small_trace(count=2)
    st = serve.serve(trace, hbm_budget=1 << 20, max_iter=50)
    assert [r.status for r in st.records] == ["rejected", "rejected"]
    assert all("budget" in r.error for r in st.records)


def test_serving_isolates_failures_and_cancellation():
    """A mixed trace: one request whose basis loses a key after its build
    (its solve is stopped with LS_EINTERNAL), one that can never fit the
    budget, one withdrawn while it runs.  Only those three end without a
    result; every other request converges to the oracle's ground energy and
    to the energy it has alone."""
    trace = _small_trace(count=10, rate=400.0, seed=13)
    big = configs.Request(len(trace), trace[-1].arrival, configs.ring_symmetric(32, 0, 1, 1, 0.1, seed=77))
    trace.append(big)
    budget = max(serve.footprint_bytes(r.sector, 120) for r in trace[:-1]) * 3
    assert serve.footprint_bytes(big.sector, 120) > budget
    bad, gone = trace[2].rid, trace[5].rid

    def corrupt(req, basis, op):
        if req.rid == bad:
            basis.test_drop_key(basis.dim // 3)

    st = serve.serve(trace, budget, max_iter=120, tol=1e-10, cancel={gone: trace[5].arrival + 0.02},
                     on_built=corrupt)
    by = {r.rid: r for r in st.records}
    assert len(by) == len(trace)
    assert by[bad].status == "failed" and "LS_EINTERNAL" in by[bad].error
    assert by[big.rid].status == "rejected"
    assert by[gone].status in ("cancelled", "ok")       # a fast solve may finish first
    alone = {r.rid: r for r in serve.serve_one_at_a_time(trace[:-1], max_iter=120, tol=1e-10).records}
    done = [r for r in st.records if r.status == "ok"]
    assert len(done) >= len(trace) - 3
    for r in done:
        req = trace[r.rid]
        assert r.converged and r.e0 == alone[r.rid].e0
        e = _exact_e0(req.sector)
        assert abs(r.e0 - e) <= 1e-9 * max(1.0, abs(e))
    assert st.summary()["status"]["failed"] == 1


def test_serve_with_stored_elements_matches_alone():
    """Stored products are bit-identical to generated ones, so a trace served
    with element storage returns the energies of the plain solves exactly,
    and so does the one-at-a-time baseline that stores as well."""
    trace = configs.serving_trace(count=12, rate=50.0, seed=9)
    trace = [r for r in trace if serve.sector_dimension(r.sector) < 2_000_000][:4]
    assert len(trace) == 4
    a = serve.serve(trace, 64 << 30, max_iter=80, tol=1e-9, store_elements=True)
    b = serve.serve_one_at_a_time(trace, max_iter=80, tol=1e-9)
    c = serve.serve_one_at_a_time(trace, max_iter=80, tol=1e-9, store_elements=True, hbm_budget=64 << 30)
    assert a.stored_bytes > 0 and c.stored_bytes > 0
    for x, y, z in zip(a.records, b.records, c.records):
        assert x.e0 == y.e0 == z.e0 and x.iters == y.iters == z.iters


def test_stepper_mixes_stored_and_generated_products():
    """In one step, a solve with stored elements takes its stored product and
    the others the fused launch: the numbers are those of each solve alone."""
    secs = [configs.ring_symmetric(20, 0, 1, 1, 0.3, seed=7), configs.ring_symmetric(18, 3, 0, 0, 0.2, seed=8),
            configs.square_j1j2(4, 4, 0.4, seed=9)]
    ops = [ls.ls_operator_create(ls.ls_basis_build(s), s.terms) for s in secs]
    alone = [op.lanczos(40, seed=s.seed) for op, s in zip(ops, secs)]
    ops[0].store()
    ops[2].store()
    solvers = [ls.Solver(op, 40, seed=s.seed) for op, s in zip(ops, secs)]
    while not all(s.result()["done"] for s in solvers):
        ls.Solver.step_all(solvers)
    for a, s in zip(alone, solvers):
        assert s.result()["e0"] == a["e0"] and s.result()["iters"] == a["iters"]


def test_batched_step_all_modes_match_lanczos_alone():
    """Several solves in one step run their Lanczos work batched (one launch
    per kernel for all of them): real and complex solves, with full,
    selective and no reorthogonalisation, each give exactly the numbers of
    ls_lanczos alone."""
    secs = [configs.ring_symmetric(20, 0, 1, 1, 0.3, seed=7), configs.ring_symmetric(18, 3, 0, 0, 0.2, seed=8),
            configs.square_j1j2(4, 4, 0.4, seed=9), configs.ring_symmetric(22, 0, 1, 1, 0.1, seed=10),
            configs.ring_symmetric(16, 5, 0, 0, 0.4, seed=11)]
    modes = ["full", "selective", "none", "full", "none"]
    ops = [ls.ls_operator_create(ls.ls_basis_build(s), s.terms) for s in secs]
    alone = [op.lanczos(45, seed=s.seed, reorth=m) for op, s, m in zip(ops, secs, modes)]
    solvers = [ls.Solver(op, 45, seed=s.seed, reorth=m) for op, s, m in zip(ops, secs, modes)]
    while not all(s.result()["done"] for s in solvers):
        ls.Solver.step_all(solvers)
    for a, s, m in zip(alone, solvers, modes):
        r = s.result()
        assert r["iters"] == a["iters"], m
        assert r["e0"] == a["e0"], (m, r["e0"], a["e0"])
        assert r["resid"] == a["resid"], m


@pytest.mark.parametrize("steps", [3, 8])
def test_chunked_steps_match_single_steps(steps):
    """ls_solver_step_n: several solves (real and complex, full and
    selective reorthogonalisation, different tolerances and step limits,
    one that converges inside a chunk) advanced `steps` iterations per
    synchronisation end exactly where single steps end, with the same
    numbers, and agree with ls_lanczos alone."""
    secs = [configs.ring16_u1(), configs.ring_symmetric(20, 0, 1, 1, 0.3, seed=7),
            configs.ring_symmetric(18, 3, 0, 0, 0.2, seed=8), configs.square_j1j2(4, 4, 0.4, seed=9)]
    ops = [ls.ls_operator_create(ls.ls_basis_build(s), s.terms) for s in secs]
    kw = [dict(max_iter=60, tol=1e-10, reorth=True), dict(max_iter=37, tol=0.0, reorth="selective"),
          dict(max_iter=50, tol=1e-8, reorth=True), dict(max_iter=45, tol=1e-10, reorth="selective")]

    def make():
        return [ls.Solver(op, k["max_iter"], tol=k["tol"], seed=s.seed, reorth=k["reorth"])
                for op, s, k in zip(ops, secs, kw)]

    single, chunked = make(), make()
    while not all(s.result()["done"] for s in single):
        ls.Solver.step_all(single)
    rounds = 0
    while not all(s.result()["done"] for s in chunked):
        ls.Solver.step_all(chunked, steps=steps)
        rounds += 1
    for op, s, k, a, c in zip(ops, secs, kw, single, chunked):
        ra, rc = a.result(), c.result()
        assert ra == rc, (s.name, ra, rc)
        alone = op.lanczos(k["max_iter"], tol=k["tol"], seed=s.seed, reorth=k["reorth"])
        assert rc["e0"] == alone["e0"] and rc["iters"] == alone["iters"], s.name
    assert rounds < max(r.result()["iters"] for r in single)
    for h in single + chunked + ops:
        h.close()


def test_breakdown_inside_a_chunk_stops_where_single_steps_stop():
    """A start vector that spans an invariant subspace: a basis state under a
    diagonal (Ising) Hamiltonian, so w = H v - alpha v is exactly zero and
    beta_1 = 0.  ls_lanczos (chunks of 32 steps), ls_solver_step_n and single
    steps all stop after one step with alpha_1 = the state's diagonal
    element (the oracle's), although the chunks compute further steps on a
    0/0 vector and discard them."""
    n = 12
    bonds = lattice.ring_bonds(n, 1.0, 0.4)
    zz = terms.make_terms([(0.25 * J, 0, 0, 0, (1 << i) | (1 << j)) for i, j, J in bonds])
    sec = configs.sector_from_arrays("ring12_ising", n, n // 2, lattice.trivial_group(n).perm,
                                     lattice.trivial_group(n).flip, lattice.trivial_group(n).chi, zz)
    b = ls.ls_basis_build(sec)
    op = ls.ls_operator_create(b, sec.terms)
    P = oracle.Problem(sec)
    reps, stab = oracle.enumerate_basis(P)
    e = np.zeros(len(reps))
    e[5] = 1.0
    d5 = float(oracle.matvec(P, reps, stab, e)[5])
    v0 = torch.from_numpy(e).cuda()
    res = op.lanczos(50, tol=0.0, v0=v0)
    assert res["iters"] == 1 and res["alpha"].tolist() == [d5] and res["e0"] == d5
    for steps in (1, 8):
        s = ls.Solver(op, 50, v0=v0)
        while not s.result()["done"]:
            ls.Solver.step_all([s], steps=steps)
        r = s.result()
        assert r["iters"] == 1 and r["e0"] == d5 and not r["converged"], (steps, r)
        s.close()
    op.close()
    b.close()
