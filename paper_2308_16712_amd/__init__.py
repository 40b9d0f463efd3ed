"""Symmetry-adapted exact diagonalization on one MI355X.

Thin Python face of the C ABI in ``include/ls_ed.h`` (library
``libls_ed.so``, hand-written HIP for gfx950).  The functions below carry the
ABI's names and only marshal arguments; device buffers are torch tensors.

    basis = ls_basis_build(sector)            # representatives, search layout
    reps, chi, norm = ls_state_info(basis, states)
    idx = ls_index_lookup(basis, keys)
    op = ls_operator_create(basis, terms)
    y = ls_matvec(op, x)                      # y = H x, x: [dim] or [dim][nrhs]
    res = ls_lanczos(op, max_iter=100, tol=1e-10)
"""
from __future__ import annotations

from ._lib import (EXPORTS, LIB_PATH, LSError, Basis, Batch, Operator, Solver, load, sector_check,
                   sector_count)  # noqa: F401


def ls_batch_create(ops, nrhs, graph: bool = True, search=None) -> Batch:
    """Many products in one persistent launch per kernel variant; `search`
    fixes the search layout instead of tuning it (ls_batch_set_search)."""
    return Batch(ops, nrhs, graph, search)


def ls_batch_matvec(batch: Batch, xs, ys, stream=None):
    return batch.matvec(xs, ys, stream)


def ls_sector_check(sector) -> dict:
    """Validate a sector and compile its group on the host only."""
    g = sector.group
    return sector_check(sector.n_sites, sector.weight, g.perm, g.flip, g.chi)


def ls_sector_count(sector, rank_begin: int = 0, rank_end: int = 2**64 - 1, stream=None) -> tuple:
    """(members, candidates) of a sector over a candidate-rank range, without
    storing the representatives."""
    g = sector.group
    return sector_count(sector.n_sites, sector.weight, g.perm, g.flip, g.chi, rank_begin, rank_end, stream)


def ls_basis_build(sector, stream=None) -> Basis:
    """Build the basis of a sector (an object with n_sites, weight and a
    group holding perm/flip/chi arrays)."""
    return Basis.from_sector(sector, stream)


def ls_state_info(basis: Basis, states, stream=None):
    return basis.state_info(states, stream)


def ls_index_lookup(basis: Basis, keys, stream=None):
    return basis.index_lookup(keys, stream)


def ls_operator_create(basis: Basis, term_table) -> Operator:
    return Operator(basis, term_table)


def ls_operator_store(op: Operator, max_bytes: int = 2**64 - 1, stream=None) -> int:
    """Keep the operator's matrix elements in device memory; later products
    read them (bit-identical results).  Returns the bytes held."""
    return op.store(max_bytes, stream)


def ls_operator_count(op: Operator, stream=None) -> int:
    return op.count_elements(stream)


def ls_operator_search_kind(op: Operator):
    """The orbit search the products run and whether a compile-time torus
    shape is used: ("generic" | "ring32" | "torus" | "ring64", bool)."""
    return op.search_kind()


def ls_matvec(op: Operator, x, y=None, stream=None):
    return op.matvec(x, y, stream)


def ls_matvec_push(op: Operator, x, y=None, stream=None):
    """Push (transposed, atomic) form of the product, a comparison variant."""
    return op.matvec_push(x, y, stream)


def ls_lanczos(op: Operator, max_iter: int, tol: float = 0.0, seed: int = 1, v0=None, reorth=True,
               stream=None):
    return op.lanczos(max_iter, tol, seed, v0, reorth, stream)
