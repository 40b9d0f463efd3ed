"""Handle destruction is stream-ordered (C ABI: the *_destroy calls).

A handle's destroy waits for the streams the handle was used on and for no
other.  The test queues a long run of products of one operator on stream B,
then builds, uses and destroys a second, small set of handles on stream A,
and checks that B is still busy afterwards: none of those calls waited for
the whole device.  The small handles' results are checked against the same
computation made before B's work was queued.
"""
import sys
import time

import pytest

from workloads import configs, lattice, rng, terms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2308_16712_amd as ls  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _small():
    g = lattice.ring_group(16, 0, 1, 1)
    return configs.sector_from_arrays("ringD16_0pp", 16, 8, g.perm, g.flip, g.chi,
                                      terms.heisenberg_terms(lattice.ring_bonds(16, 1.0, 0.3)))


def _small_cycle(sec, stream):
    """Build, product, Lanczos steps, batch product, destroy: all on `stream`."""
    b = ls.ls_basis_build(sec, stream=stream)
    op = ls.ls_operator_create(b, sec.terms)
    with torch.cuda.stream(stream):
        x = torch.from_numpy(rng.vector(7, b.dim)).cuda()
        y = op.matvec(x, stream=stream)
        s = ls.Solver(op, 20, seed=3)
        for _ in range(20):
            ls.Solver.step_all([s], stream=stream)
        e0 = s.result()["e0"]
        bt = ls.Batch([op], [1])
        yb = torch.empty_like(x)
        bt.matvec([x], [yb], stream=stream)
    stream.synchronize()
    out = (y.cpu(), yb.cpu(), e0)
    bt.close()
    s.close()
    op.close()
    b.close()
    return out


def test_destroy_waits_only_for_its_own_streams():
    big = configs.ring32_symmetric()
    _say("[gpu] streams: building the 32-site sector")
    bb = ls.ls_basis_build(big)
    bop = ls.ls_operator_create(bb, big.terms)
    bx = torch.from_numpy(rng.vector(11, bb.dim, complex_=bop.is_complex)).cuda()
    by = torch.empty_like(bx)
    sa = torch.cuda.Stream()
    sb = torch.cuda.Stream()
    sec = _small()
    # first cycle: loads every code object the small cycle needs, reference results
    want = _small_cycle(sec, sa)
    # time one product of the big operator to size B's queue (about 1.5 s)
    for _ in range(3):
        bop.matvec(bx, by, stream=sb)
    sb.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        bop.matvec(bx, by, stream=sb)
    sb.synchronize()
    per = (time.perf_counter() - t0) / 10
    reps = int(min(4000, max(50, 1.5 / max(per, 1e-6))))
    _say(f"[gpu] streams: {per * 1e3:.3f} ms per product, queueing {reps} on stream B")
    for _ in range(reps):
        bop.matvec(bx, by, stream=sb)
    t1 = time.perf_counter()
    got = _small_cycle(sec, sa)
    busy = not sb.query()
    t_small = time.perf_counter() - t1
    sb.synchronize()
    t_b = time.perf_counter() - t1
    _say(f"[gpu] streams: small cycle {t_small * 1e3:.1f} ms, B drained after {t_b * 1e3:.1f} ms, busy={busy}")
    assert busy, "a call on stream A waited for stream B's queued products"
    assert torch.equal(got[0], want[0]) and torch.equal(got[1], want[1]) and got[2] == want[2]
    bop.close()
    bb.close()


def test_destroy_waits_for_its_own_work_not_later_work_on_its_stream():
    """A basis built and used on stream A is destroyed while products of
    another operator, enqueued on A after that use, are still running: the
    destroy waits for the basis's own work only."""
    big = configs.ring32_symmetric()
    bb = ls.ls_basis_build(big)
    bop = ls.ls_operator_create(bb, big.terms)
    bx = torch.from_numpy(rng.vector(11, bb.dim, complex_=bop.is_complex)).cuda()
    by = torch.empty_like(bx)
    sa = torch.cuda.Stream()
    sec = _small()
    want = _small_cycle(sec, sa)          # warm; reference results
    b = ls.ls_basis_build(sec, stream=sa)
    op = ls.ls_operator_create(b, sec.terms)
    with torch.cuda.stream(sa):
        x = torch.from_numpy(rng.vector(7, b.dim)).cuda()
        y = op.matvec(x, stream=sa)
    for _ in range(3):
        bop.matvec(bx, by, stream=sa)
    sa.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        bop.matvec(bx, by, stream=sa)
    sa.synchronize()
    per = (time.perf_counter() - t0) / 10
    reps = int(min(4000, max(50, 1.5 / max(per, 1e-6))))
    for _ in range(reps):
        bop.matvec(bx, by, stream=sa)     # later work on the same stream
    t1 = time.perf_counter()
    op.close()
    b.close()
    busy = not sa.query()
    t_close = time.perf_counter() - t1
    sa.synchronize()
    _say(f"[gpu] streams: destroy {t_close * 1e3:.1f} ms with {reps} later products queued, busy={busy}")
    assert busy, "the destroy waited for work enqueued after the basis's own"
    assert torch.equal(y.cpu(), want[0])
    bop.close()
    bb.close()
