"""Oracle for the symmetry-adapted exact-diagonalization path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``smoke()`` and by the
CPU-baseline leg of ``bench.py``, never by the product package.  It shares
no code with the GPU library; the only module both use is ``workloads``
(seeded inputs).

Contents:
  * C core (``oracle.c``): brute-force orbit search, Gosper enumeration,
    hash-map index, column-by-column product, getRow.
  * Here: ctypes marshalling (optionally split over host threads), the
    sector Hamiltonian assembled from getRow as a SciPy sparse matrix, and
    the Lanczos recurrence in FP64 numpy with the tridiagonal eigenproblem
    solved by SciPy (library primitives).

Parity pins of every function live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Tuple

import numpy as np

from . import _build

_HERE = os.path.dirname(os.path.abspath(__file__))


class _Sector(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("weight", ctypes.c_int32),
                ("n_elements", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("perm", ctypes.c_void_p), ("flip", ctypes.c_void_p), ("chi", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.library_path()
        if not os.path.exists(path) or _build.stale():
            _build.build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32, u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
        L.orc_apply.argtypes = [P, ctypes.c_int, u64]
        L.orc_apply.restype = u64
        L.orc_state_info.argtypes = [P, i64, P, P, P, P]
        L.orc_state_info.restype = None
        L.orc_enumerate.argtypes = [P, P, P, i64]
        L.orc_enumerate.restype = i64
        L.orc_index_lookup.argtypes = [P, i64, i64, P, P]
        L.orc_index_lookup.restype = None
        L.orc_matvec_columns.argtypes = [P, P, P, i64, P, i32, i32, P, P, i64, i64]
        L.orc_matvec_columns.restype = i64
        L.orc_get_row.argtypes = [P, u64, P, i32, P, P, i32]
        L.orc_get_row.restype = i32
        _lib = L
    return _lib


class Problem:
    """A sector (group + characters + weight) and optionally a term table,
    held in the layouts the C core reads."""

    def __init__(self, sector):
        g = sector.group
        self.n_sites = int(sector.n_sites)
        self.weight = int(sector.weight)
        self.perm = np.ascontiguousarray(g.perm, dtype=np.uint16)
        self.flip = np.ascontiguousarray(g.flip, dtype=np.uint8)
        self.chi = np.ascontiguousarray(g.chi, dtype=np.float64)
        self.n_elements = int(self.perm.shape[0])
        self.terms = np.ascontiguousarray(sector.terms) if sector.terms is not None else None
        self._c = _Sector(self.n_sites, self.weight, self.n_elements, 0,
                          self.perm.ctypes.data, self.flip.ctypes.data, self.chi.ctypes.data)
        self.is_real = bool(np.all(self.chi[:, 1] == 0.0) and
                            (self.terms is None or np.all(self.terms["im"] == 0.0)))

    @property
    def ptr(self):
        return ctypes.addressof(self._c)


def apply(prob: Problem, g: int, s: int) -> int:
    return int(lib().orc_apply(prob.ptr, int(g), int(s)))


def enumerate_basis(prob: Problem) -> Tuple[np.ndarray, np.ndarray]:
    """Sorted representatives and their stabilizer sizes."""
    L = lib()
    d = int(L.orc_enumerate(prob.ptr, None, None, 0))
    reps = np.zeros(d, np.uint64)
    stab = np.zeros(d, np.uint16)
    d2 = int(L.orc_enumerate(prob.ptr, reps.ctypes.data, stab.ctypes.data, d))
    assert d2 == d
    return reps, stab


def count_basis(prob: Problem) -> int:
    return int(lib().orc_enumerate(prob.ptr, None, None, 0))


def _workers(workers) -> int:
    if workers is None or workers <= 0:
        return max(1, min(16, os.cpu_count() or 1))
    return int(workers)


def state_info(prob: Problem, states, workers: int = 1) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(representative, chi(g*), norm) per state.  With workers > 1 the
    states are split into contiguous chunks handled by host threads (the C
    core releases the interpreter lock); each state's result is the same."""
    s = np.ascontiguousarray(states, dtype=np.uint64)
    n = s.shape[0]
    reps = np.zeros(n, np.uint64)
    chi = np.zeros((n, 2), np.float64)
    norm = np.zeros(n, np.float64)
    nw = _workers(workers)

    def run(lo, hi):
        if hi > lo:
            lib().orc_state_info(prob.ptr, hi - lo, s[lo:].ctypes.data, reps[lo:].ctypes.data,
                                 chi[lo:].ctypes.data, norm[lo:].ctypes.data)

    if nw == 1 or n < 4096:
        run(0, n)
    else:
        from concurrent.futures import ThreadPoolExecutor
        step = max(4096, -(-n // (nw * 8)))
        with ThreadPoolExecutor(max_workers=nw) as ex:
            list(ex.map(lambda lo: run(lo, min(n, lo + step)), range(0, n, step)))
    return reps, chi[:, 0] + 1j * chi[:, 1], norm


def index_lookup(reps: np.ndarray, keys) -> np.ndarray:
    reps = np.ascontiguousarray(reps, dtype=np.uint64)
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros(k.shape[0], np.int64)
    lib().orc_index_lookup(reps.ctypes.data, reps.shape[0], k.shape[0], k.ctypes.data,
                           out.ctypes.data)
    return out


def matvec(prob: Problem, reps, stab, x, columns=None) -> np.ndarray:
    """y = H x in the symmetry-adapted basis, column by column.

    x: [d] or [d][nrhs], real or complex.  Returns complex unless the problem
    and x are real.  ``columns`` = (begin, end) restricts the scatter to a
    column range (for timing samples); the result then holds only those
    columns' contributions.
    """
    reps = np.ascontiguousarray(reps, dtype=np.uint64)
    stab = np.ascontiguousarray(stab, dtype=np.uint16)
    d = reps.shape[0]
    xa = np.asarray(x)
    squeeze = xa.ndim == 1
    if d == 0:
        return np.zeros_like(xa)
    xc = np.ascontiguousarray(xa.reshape(d, -1), dtype=np.complex128)
    nrhs = xc.shape[1]
    y = np.zeros((d, nrhs), np.complex128)
    b, e = (0, d) if columns is None else columns
    n = lib().orc_matvec_columns(prob.ptr, reps.ctypes.data, stab.ctypes.data, d,
                                 prob.terms.ctypes.data, len(prob.terms), nrhs,
                                 xc.ctypes.data, y.ctypes.data, int(b), int(e))
    if n < 0:
        raise RuntimeError("oracle: a neighbour representative in the sector is missing")
    matvec.last_applied = int(n)
    if prob.is_real and not np.iscomplexobj(xa):
        y = y.real.copy()
    return y[:, 0] if squeeze else y


matvec.last_applied = 0


def get_row(prob: Problem, r: int, cap: int = 4096):
    """(representatives, coefficients) of the non-zeros of row r (getRow)."""
    out_r = np.zeros(cap, np.uint64)
    out_c = np.zeros((cap, 2), np.float64)
    n = int(lib().orc_get_row(prob.ptr, int(r), prob.terms.ctypes.data, len(prob.terms),
                              out_r.ctypes.data, out_c.ctypes.data, cap))
    if n < 0:
        raise ValueError("not a representative in the sector")
    if n > cap:
        return get_row(prob, r, n)
    return out_r[:n].copy(), out_c[:n, 0] + 1j * out_c[:n, 1]


def dense(prob: Problem, reps, stab) -> np.ndarray:
    """The sector Hamiltonian as a dense matrix, one column per unit vector."""
    d = len(reps)
    return matvec(prob, reps, stab, np.eye(d, dtype=np.complex128))


def get_rows(prob: Problem, rs, workers: int = 1):
    """get_row for every representative in rs (host threads when workers > 1)."""
    rs = [int(r) for r in rs]
    nw = _workers(workers)
    if nw == 1 or len(rs) < 64:
        return [get_row(prob, r) for r in rs]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=nw) as ex:
        return list(ex.map(lambda r: get_row(prob, r), rs, chunksize=64))


def sparse_matrix(prob: Problem, reps, workers: int = 1):
    """The sector Hamiltonian as a SciPy CSR matrix assembled row by row from
    getRow (Section 5.3): row i holds <r~_i|H|r~_j> at the index j of each
    neighbour's representative (entries of one (i, j) summed).  Same elements
    as the column-by-column product, in a form a library sparse product can
    apply many times (Lanczos parity at sizes where the column loop is slow)."""
    import scipy.sparse as sp
    reps = np.ascontiguousarray(reps, dtype=np.uint64)
    d = reps.shape[0]
    rows = get_rows(prob, reps, workers)
    cnt = np.array([len(nb) for nb, _ in rows], dtype=np.int64)
    nb = np.concatenate([r[0] for r in rows]) if d else np.zeros(0, np.uint64)
    coef = np.concatenate([r[1] for r in rows]) if d else np.zeros(0, np.complex128)
    cols = index_lookup(reps, nb)
    if np.any(cols < 0):
        raise RuntimeError("oracle: a neighbour representative in the sector is missing")
    ri = np.repeat(np.arange(d, dtype=np.int64), cnt)
    if prob.is_real:
        coef = coef.real.copy()
    return sp.csr_matrix((coef, (ri, cols)), shape=(d, d))


def cgs_selective(Vm: np.ndarray, w: np.ndarray):
    """One classical Gram-Schmidt pass of w against the rows of Vm, and a
    second one only when the first removed more than half of ||w||^2 (the
    criterion of Daniel, Gragg, Kaufman and Stewart, Math. Comp. 30 (1976),
    with eta^2 = 1/2).  Returns (w, passes run)."""
    n0 = np.vdot(w, w).real
    w = w - Vm.T @ (Vm.conj() @ w)
    if np.vdot(w, w).real < 0.5 * n0:
        return w - Vm.T @ (Vm.conj() @ w), 2
    return w, 1


def lanczos(apply_h, v0: np.ndarray, m: int, reorth=True, tol: float = 0.0):
    """Lanczos three-term recurrence in FP64 with optional full CGS2
    reorthogonalization (reorth True), or a second Gram-Schmidt pass only when
    the first needs it (reorth "selective", cgs_selective); the tridiagonal
    eigenproblem by SciPy.

    Step k: w = H v_k; alpha_k = Re <v_k, w>; w -= alpha_k v_k + beta_k v_{k-1};
    (CGS2: twice w -= V (V^H w)); beta_{k+1} = ||w||; v_{k+1} = w / beta_{k+1}.
    alpha_k is taken before reorthogonalization.  With tol > 0 the loop stops
    once successive lowest Ritz values differ by less than tol*max(1,|E0|)
    and beta_{k+1} |s_k| < sqrt(tol)*max(1,|E0|).
    Returns dict(e0, alpha, beta, resid, iters, converged).
    """
    from scipy.linalg import eigh_tridiagonal

    v = np.asarray(v0)
    v = v / np.sqrt(np.vdot(v, v).real)
    V = [v]
    alpha, beta = [], []
    prev = None
    e0 = None
    resid = np.inf
    converged = False
    for k in range(m):
        w = apply_h(V[k])
        a = float(np.vdot(V[k], w).real)
        w = w - a * V[k]
        if k > 0:
            w = w - beta[k - 1] * V[k - 1]
        if reorth == "selective":
            w, _ = cgs_selective(np.stack(V, axis=0), w)
        elif reorth:
            Vm = np.stack(V, axis=0)
            for _ in range(2):
                h = Vm.conj() @ w
                w = w - Vm.T @ h
        b = float(np.sqrt(np.vdot(w, w).real))
        alpha.append(a)
        evals, evecs = eigh_tridiagonal(np.array(alpha), np.array(beta),
                                        select="i", select_range=(0, 0))
        e0 = float(evals[0])
        resid = b * abs(evecs[-1, 0])
        scale = max(1.0, abs(e0))
        if tol > 0 and prev is not None and abs(e0 - prev) < tol * scale and resid < np.sqrt(tol) * scale:
            converged = True
            break
        prev = e0
        if k + 1 < m:
            if b == 0.0:
                break
            beta.append(b)
            V.append(w / b)
    return dict(e0=e0, alpha=np.array(alpha), beta=np.array(beta), resid=resid,
                iters=len(alpha), converged=converged)
