"""The C ABI on the CPU: the library loads, exports every function the
header declares, and rejects invalid sectors before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2308_16712_amd as ls
from paper_2308_16712_amd import _lib
from workloads import lattice

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(ls_\w+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_function():
    L = _lib.load()
    declared = _declared_functions()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(L, name), name
    assert set(_lib.EXPORTS) <= declared


def test_version_and_no_error_initially():
    L = _lib.load()
    assert b"gfx950" in L.ls_version()


def _desc(n, w, perm, flip, chi):
    perm = np.ascontiguousarray(perm, np.uint16)
    flip = np.ascontiguousarray(flip, np.uint8)
    chi = np.ascontiguousarray(chi, np.float64)
    d = _lib.SectorDesc(n, w, perm.shape[0], perm.ctypes.data, flip.ctypes.data, chi.ctypes.data)
    return d, (perm, flip, chi)


def _build_status(n, w, perm, flip, chi):
    L = _lib.load()
    d, keep = _desc(n, w, perm, flip, chi)
    h = ctypes.c_void_p()
    st = L.ls_basis_build(ctypes.byref(d), None, ctypes.byref(h))
    return st, L.ls_last_error().decode(), h


@pytest.mark.parametrize("case", [
    "not_bijective", "duplicate", "not_closed", "bad_character", "no_identity", "flip_weight",
    "n_too_large", "weight_too_large", "modulus",
])
def test_invalid_sector_is_rejected_before_device_work(case):
    n = 6
    g = lattice.ring_group(n, 1)
    perm, flip, chi = g.perm.copy(), g.flip.copy(), g.chi.copy()
    w = 3
    if case == "not_bijective":
        perm[2, 0] = perm[2, 1]
    elif case == "duplicate":
        perm = np.concatenate([perm, perm[1:2]])
        flip = np.concatenate([flip, flip[1:2]])
        chi = np.concatenate([chi, chi[1:2]])
    elif case == "not_closed":
        perm, flip, chi = perm[:3], flip[:3], chi[:3]
    elif case == "bad_character":
        chi[1] = [np.cos(0.3), np.sin(0.3)]
    elif case == "no_identity":
        perm, flip, chi = perm[1:], flip[1:], chi[1:]
    elif case == "flip_weight":
        g = lattice.ring_group(n, 0, 0, 1)
        perm, flip, chi = g.perm, g.flip, g.chi
        w = 2
    elif case == "n_too_large":
        n = 65
        perm = np.arange(65, dtype=np.uint16)[None]
        flip, chi = np.zeros(1), np.array([[1.0, 0.0]])
    elif case == "weight_too_large":
        w = 7
    elif case == "modulus":
        chi = chi * 1.5
    st, msg, h = _build_status(n, w, perm, flip, chi)
    assert st == _lib.LS_EINVAL, (case, st, msg)
    assert msg
    assert not h.value
    # the count-only enumeration runs the same checks first
    with pytest.raises(_lib.LSError) as e:
        _lib.sector_count(n, w, perm, flip, chi)
    assert e.value.status == _lib.LS_EINVAL


def test_null_arguments():
    L = _lib.load()
    h = ctypes.c_void_p()
    assert L.ls_basis_build(None, None, ctypes.byref(h)) == _lib.LS_EINVAL
    assert L.ls_matvec(None, 1, None, None, None) == _lib.LS_EINVAL
    assert L.ls_matvec_push(None, 1, None, None, None) == _lib.LS_EINVAL
    assert L.ls_state_info(None, 0, None, None, None, None, None) == _lib.LS_EINVAL
    assert L.ls_index_lookup(None, 0, None, None, None) == _lib.LS_EINVAL
    assert L.ls_lanczos(None, None, None, None, None, None) == _lib.LS_EINVAL
    m = ctypes.c_uint64()
    assert L.ls_sector_count(None, 0, 1, ctypes.byref(m), None, None) == _lib.LS_EINVAL
    assert L.ls_operator_store(None, 0, None, None) == _lib.LS_EINVAL
    assert L.ls_operator_search_kind(None, None, None) == _lib.LS_EINVAL
    g = lattice.ring_group(6, 0)
    with pytest.raises(_lib.LSError) as e:     # rank_begin > rank_end
        _lib.sector_count(6, 3, g.perm, g.flip, g.chi, 5, 4)
    assert e.value.status == _lib.LS_EINVAL
    L.ls_basis_destroy(None)
    L.ls_operator_destroy(None)


def test_binding_names_match_abi():
    for name in ("ls_basis_build", "ls_state_info", "ls_index_lookup", "ls_matvec", "ls_lanczos",
                 "ls_operator_create", "ls_operator_store", "ls_operator_count", "ls_operator_search_kind", "ls_matvec_push",
                 "ls_sector_count",
                 "ls_sector_check", "ls_batch_create", "ls_batch_matvec"):
        assert callable(getattr(ls, name))


def _groups_for_structure():
    from workloads import lattice as L
    perm = [5, 2, 9, 0, 11, 7, 1, 10, 3, 8, 6, 4]
    return [
        ("trivial16", 16, 8, L.trivial_group(16), (1, 1, 0)),
        ("ringT20", 20, 10, L.ring_group(20, 3), (20, 1, 0)),
        ("ringD32Z", 32, 16, L.ring_group(32, 0, 1, 1), (32, 1, 1)),
        ("ringD36Z", 36, 18, L.ring_group(36, 0, 1, 1), (36, 1, 1)),
        ("ring40D_w3", 40, 3, L.ring_group(40, 0, 1), (40, 1, 0)),
        ("torus6x6", 36, 18, L.torus_group(6, 6, 0, 0, "full", None, 1), (6, 6, 1)),
        ("torus4x6", 24, 12, L.torus_group(6, 4, 0, 0, "full", None, 1), (6, 4, 1)),
        ("torus4x4_k", 16, 8, L.torus_group(4, 4, 1, 2, "none"), (4, 4, 0)),
        ("scrambled12", 12, 6, L.relabel_group(L.ring_group(12, 2), perm), (1, 1, 0)),
        ("flip_only", 10, 5, L.close_group(10, [(list(range(10)), 1, -1.0)]), (1, 1, 1)),
    ]


@pytest.mark.parametrize("case", _groups_for_structure(), ids=lambda c: c[0])
def test_group_compiler_structure(case):
    """The host group compiler finds the translation layout and covers the
    group exactly with cosets (its Benes self-check runs on every wire)."""
    name, n, w, g, (lx, ly, pf) = case
    info = _lib.sector_check(n, w, g.perm, g.flip, g.chi)
    assert (info["lx"], info["ly"], info["pair_flip"]) == (lx, ly, pf)
    assert info["n_cosets"] * info["lx"] * info["ly"] * (2 if info["pair_flip"] else 1) == g.size


def test_group_compiler_random_relabelings():
    """Benes routing of many unstructured permutations (self-checked in the
    library on every wire) for 32- and 64-bit words."""
    from workloads import lattice as L
    from workloads import rng
    st = rng.Stream(123)
    for n in (7, 16, 31, 32, 33, 47, 64):
        perm = list(range(n))
        for i in range(n - 1, 0, -1):
            j = st.randint(0, i + 1)
            perm[i], perm[j] = perm[j], perm[i]
        g = L.relabel_group(L.ring_group(n, 0, 1), perm)
        info = _lib.sector_check(n, 2, g.perm, g.flip, g.chi)
        assert info["n_cosets"] * info["lx"] * info["ly"] == g.size


# ---------------------------------------------------------------- binding checks
#
# The binding refuses buffers the kernels would read or write past: wrong
# element type, wrong length, y unlike x, non-64-bit states.  The checks run
# before any library call, so they are exercised here on handle objects that
# hold no library handle.

def _fake_operator(dim, cplx):
    op = _lib.Operator.__new__(_lib.Operator)
    op._h = None
    op.dim = dim
    op.is_complex = cplx
    return op


def _fake_basis():
    b = _lib.Basis.__new__(_lib.Basis)
    b._h = None
    b.dim = 10
    return b


@pytest.mark.parametrize("cplx", [False, True])
def test_binding_rejects_mismatched_vectors(cplx):
    import torch
    op = _fake_operator(10, cplx)
    good = torch.complex128 if cplx else torch.float64
    bad = torch.float64 if cplx else torch.complex128
    with pytest.raises(TypeError):
        op.matvec(torch.zeros(10, dtype=torch.float32))
    with pytest.raises(TypeError):
        op.matvec(torch.zeros(10, dtype=bad))
    with pytest.raises(ValueError):
        op.matvec(torch.zeros(9, dtype=good))                   # short
    with pytest.raises(ValueError):
        op.matvec(torch.zeros(10, 65, dtype=good))              # nrhs above 64
    with pytest.raises(ValueError):
        op.matvec(torch.zeros(10, 2, 2, dtype=good))
    with pytest.raises(TypeError):
        op.matvec_push(torch.zeros(10, dtype=bad))
    with pytest.raises(ValueError):
        op.lanczos(5, v0=torch.zeros(9, dtype=good))
    with pytest.raises(TypeError):
        op.lanczos(5, v0=torch.zeros(10, dtype=bad))
    with pytest.raises(ValueError):
        op.lanczos(0)
    with pytest.raises(ValueError):
        _lib.Solver(op, 5, v0=torch.zeros(11, dtype=good))


def test_binding_rejects_y_unlike_x():
    import torch
    x = torch.zeros(10, dtype=torch.float64)
    for y in (torch.zeros(10, dtype=torch.float32), torch.zeros(9, dtype=torch.float64),
              torch.zeros(10, 1, dtype=torch.float64)):
        with pytest.raises(ValueError):
            _lib._same_as(y, x)
    with pytest.raises(TypeError):
        _lib._same_as(np.zeros(10), x)


def test_binding_rejects_non_64bit_states():
    import torch
    b = _fake_basis()
    for bad in (torch.zeros(4, dtype=torch.int32), torch.zeros(4, dtype=torch.float64)):
        with pytest.raises(TypeError):
            b.state_info(bad)
        with pytest.raises(TypeError):
            b.index_lookup(bad)
    with pytest.raises(ValueError):
        b.index_lookup(torch.zeros(2, 2, dtype=torch.int64))


def test_binding_rejects_host_buffers():
    """Correct dtype and shape, but host memory: refused before the call."""
    import torch
    op = _fake_operator(10, False)
    with pytest.raises(ValueError, match="GPU"):
        op.matvec(torch.zeros(10, dtype=torch.float64))


def test_batch_binding_checks_every_vector():
    import torch
    B = _lib.Batch.__new__(_lib.Batch)
    B._h = None
    B.ops = [_fake_operator(10, False), _fake_operator(6, True)]
    B.nrhs = [2, 1]
    c6 = torch.zeros(6, dtype=torch.complex128)
    with pytest.raises(TypeError):       # element type of the operator
        B.matvec([torch.zeros(10, 2, dtype=torch.complex128), c6], [c6, c6])
    with pytest.raises(ValueError):      # nrhs of the batch entry
        B.matvec([torch.zeros(10, 3, dtype=torch.float64), c6], [c6, c6])
    with pytest.raises(ValueError):      # length
        B.matvec([torch.zeros(11, 2, dtype=torch.float64), c6], [c6, c6])
    with pytest.raises(ValueError):
        B.matvec([c6], [c6])             # one x and one y per operator
