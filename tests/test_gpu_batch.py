"""Batched products (one persistent launch per kernel variant, HIP graph
replay) against single products and the oracle."""
import numpy as np
import pytest

import oracle
from workloads import configs, lattice, rng, terms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2308_16712_amd as ls  # noqa: E402


def _sector(name, n, w, g, bonds):
    return configs.sector_from_arrays(name, n, w, g.perm, g.flip, g.chi, terms.heisenberg_terms(bonds))


def _mixed_sectors():
    return [
        _sector("ringT20_k3", 20, 10, lattice.ring_group(20, 3), lattice.ring_bonds(20, 1.0, 0.4)),
        _sector("ringT22_k0", 22, 11, lattice.ring_group(22, 0), lattice.ring_bonds(22, 1.0, 0.1)),
        _sector("ringT18_k7", 18, 9, lattice.ring_group(18, 7), lattice.ring_bonds(18, 1.0, 0.55)),
        _sector("ringD20_0pp", 20, 10, lattice.ring_group(20, 0, 1, 1), lattice.ring_bonds(20, 1.0, 0.3)),
        _sector("torus4x4_full", 16, 8, lattice.torus_group(4, 4, 0, 0, "full", None, 1),
                lattice.torus_bonds(4, 4, 1.0, 0.5)),
        _sector("torus4x6_full", 24, 12, lattice.torus_group(6, 4, 0, 0, "full", None, 1),
                lattice.torus_bonds(6, 4, 1.0, 0.25)),
        _sector("torus6x6_w4_k10", 36, 4, lattice.torus_group(6, 6, 1, 0, "none"),
                lattice.torus_bonds(6, 6, 1.0, 0.5)),
        configs.ring16_u1(),
    ]


def _setup(sectors, nrhs):
    ops, xs, ys, refs = [], [], [], []
    for k, (sec, r) in enumerate(zip(sectors, nrhs)):
        b = ls.ls_basis_build(sec)
        op = ls.ls_operator_create(b, sec.terms)
        x = rng.vector(100 + k, b.dim, r, complex_=op.is_complex)
        ops.append(op)
        xs.append(torch.from_numpy(np.ascontiguousarray(x)).cuda())
        ys.append(torch.zeros_like(xs[-1]))
        refs.append((sec, b, x))
    return ops, xs, ys, refs


def test_batch_equals_single_products_and_oracle():
    sectors = _mixed_sectors()
    nrhs = [4, 1, 3, 2, 5, 1, 4, 8]
    ops, xs, ys, refs = _setup(sectors, nrhs)
    batch = ls.Batch(ops, nrhs)
    for rep in range(3):                      # first call tunes and captures; then replays
        for y in ys:
            y.zero_()
        batch.matvec(xs, ys)
        torch.cuda.synchronize()
        for op, x, y in zip(ops, xs, ys):
            single = op.matvec(x)
            assert torch.equal(single, y), rep     # same arithmetic per row: bit-identical
        # eager work between replays
        _ = (xs[0] * 2).sum().item()
    info = batch.info()
    assert info["graph"] and info["launches"] >= 3
    for op in ops:
        op.check()      # annihilated orbits (k != 0) are not reported as misses
    # oracle on a few of them
    for (sec, b, x), y in list(zip(refs, ys))[:4]:
        P = oracle.Problem(sec)
        reps, stab = oracle.enumerate_basis(P)
        want = oracle.matvec(P, reps, stab, x)
        got = y.cpu().numpy()
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert err < 1e-12, (sec.name, err)


def test_batch_pointer_change_and_direct_launch():
    sectors = _mixed_sectors()[:3]
    nrhs = [2, 2, 1]
    ops, xs, ys, refs = _setup(sectors, nrhs)
    for graph in (True, False):
        batch = ls.Batch(ops, nrhs, graph=graph)
        batch.matvec(xs, ys)
        xs2 = [torch.flip(x, dims=[0]).contiguous() for x in xs]
        ys2 = [torch.empty_like(y) for y in ys]
        batch.matvec(xs2, ys2)                    # new buffers: job tables rewritten
        torch.cuda.synchronize()
        for op, x, y in zip(ops, xs2, ys2):
            assert torch.equal(op.matvec(x), y)
        assert batch.info()["graph"] == graph


def test_operator_count_matches_host_count():
    for sec in _mixed_sectors()[:5]:
        b = ls.ls_basis_build(sec)
        op = ls.ls_operator_create(b, sec.terms)
        reps = b.copy()[0].cpu().numpy().view(np.uint64)
        off = sec.terms[sec.terms["flip"] != 0]
        want = sum(int(np.count_nonzero((reps & np.uint64(t["sel_mask"])) == np.uint64(t["sel_value"])))
                   for t in off)
        assert op.count_elements() == want


def test_batch_rejects_bad_input():
    sectors = _mixed_sectors()[:2]
    ops, xs, ys, refs = _setup(sectors, [1, 1])
    batch = ls.Batch(ops, [1, 1])
    with pytest.raises(ls.LSError):
        batch.matvec([xs[0], xs[1]], [xs[0], ys[1]])   # y overlaps x
    with pytest.raises(ValueError):
        ls.Batch(ops, [1])


@pytest.mark.parametrize("search", [("buckets", 6), ("buckets", 12), ("staged", 5), ("staged", 8), ("staged", 11),
                                    "own"], ids=lambda s: s if isinstance(s, str) else f"{s[0]}{s[1]}")
def test_batch_forced_search_layouts_equal_single_products(search):
    """Every search layout the batch can use (bucket tables in global memory,
    bucket tables staged in LDS, each basis's own) gives the single
    products' bits: the layout changes how an index is found, not which."""
    sectors = _mixed_sectors()
    nrhs = [4, 1, 3, 2, 5, 1, 4, 8]
    ops, xs, ys, refs = _setup(sectors, nrhs)
    batch = ls.Batch(ops, nrhs, search=search)
    batch.matvec(xs, ys)
    torch.cuda.synchronize()
    want_mode = search if isinstance(search, str) else search[0]
    for k, (op, x, y, (sec, b, _)) in enumerate(zip(ops, xs, ys, refs)):
        assert torch.equal(op.matvec(x), y), (sec.name, search)
        got = batch.search(k)
        own = op.search_kind()
        if sec.name == "ring16_sz0_nosym":
            assert got["mode"] == "rank"
        elif want_mode == "own":
            assert got["mode"] == "hash"
        else:
            assert got["mode"] == want_mode and got["bits"] == search[1], (sec.name, got, own)
    for op in ops:
        op.check()


def test_batch_staged_table_too_large_for_lds_is_refused():
    """A staged bucket table that does not fit beside the 6x6 torus jobs'
    LDS tables (pair table, flip images, terms) is refused with LS_EINVAL."""
    sec = _mixed_sectors()[6]
    ops, xs, ys, _ = _setup([sec], [1])
    batch = ls.Batch(ops, [1], search=("staged", 13))
    with pytest.raises(ls.LSError) as e:
        batch.matvec(xs, ys)
    assert e.value.status == ls._lib.LS_EINVAL
    with pytest.raises(ls.LSError):
        ls.Batch(ops, [1], search=("staged", 14))


def test_batch_tuner_picks_a_measured_layout():
    """The tuner times the basis's own layout against global and staged
    bucket tables and keeps the fastest; the choice and the times are
    reported per operator, and the products stay bit-identical."""
    sectors = _mixed_sectors()
    nrhs = [1] * len(sectors)
    ops, xs, ys, refs = _setup(sectors, nrhs)
    batch = ls.Batch(ops, nrhs)
    batch.matvec(xs, ys)
    torch.cuda.synchronize()
    for k, (op, x, y, (sec, b, _)) in enumerate(zip(ops, xs, ys, refs)):
        assert torch.equal(op.matvec(x), y), sec.name
        got = batch.search(k)
        print(f"[gpu] tuner {sec.name} dim {b.dim}: {got}", flush=True)
        assert got["mode"] in ("hash", "buckets", "staged", "rank")
        if got["mode"] != "rank" and b.dim >= 4096:
            assert got["own_ns"] > 0 and 0 < got["chosen_ns"] <= got["own_ns"]
