"""ctypes binding of ``libls_ed.so`` (the C ABI declared in include/ls_ed.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device buffers are torch tensors on the current HIP device; the
stream is torch's current stream unless one is given.  The binding fails
loudly when the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libls_ed.so")

LS_OK, LS_WNOTCONV, LS_EINVAL, LS_ENOMEM, LS_EDEVICE, LS_EINTERNAL = 0, 1, -1, -2, -3, -4
_NAMES = {0: "LS_OK", 1: "LS_WNOTCONV", -1: "LS_EINVAL", -2: "LS_ENOMEM", -3: "LS_EDEVICE", -4: "LS_EINTERNAL"}

EXPORTS = ["ls_sector_check", "ls_sector_count", "ls_sector_count_noalloc", "ls_basis_build", "ls_basis_info", "ls_basis_copy", "ls_basis_destroy", "ls_state_info",
           "ls_index_lookup", "ls_operator_create", "ls_operator_destroy", "ls_operator_info",
           "ls_operator_count", "ls_operator_store", "ls_operator_search_kind", "ls_operator_check",
           "ls_basis_test_drop_key", "ls_matvec", "ls_matvec_push",
           "ls_batch_create", "ls_batch_matvec", "ls_batch_info", "ls_batch_search", "ls_batch_set_search",
           "ls_batch_set_graph",
           "ls_batch_destroy",
           "ls_lanczos", "ls_solver_footprint", "ls_solver_create", "ls_solver_step", "ls_solver_step_n",
           "ls_solver_result",
           "ls_solver_destroy", "ls_last_error", "ls_version"]


class LSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class SectorDesc(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_uint32), ("hamming_weight", ctypes.c_int32),
                ("n_elements", ctypes.c_uint32), ("perm", ctypes.c_void_p),
                ("flip", ctypes.c_void_p), ("chi", ctypes.c_void_p)]


class Term(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double), ("sel_mask", ctypes.c_uint64),
                ("sel_value", ctypes.c_uint64), ("flip", ctypes.c_uint64), ("sign_mask", ctypes.c_uint64)]


class LanczosOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_uint32), ("reorth", ctypes.c_uint32), ("tol", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("d_v0", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
                ("beta", ctypes.c_void_p)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (no build, no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
                          " (or python paper_2308_16712_amd/build.py)")
    L = ctypes.CDLL(path)
    P, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
    sig = {
        "ls_sector_check": ([P, P, P, P, P], i32),
        "ls_sector_count": ([P, u64, u64, P, P, P], i32),
        "ls_sector_count_noalloc": ([P, u64, u64, P, P, P], i32),
        "ls_basis_build": ([P, P, P], i32),
        "ls_operator_store": ([P, u64, P, P], i32),
        "ls_basis_info": ([P, P, P, P], i32),
        "ls_basis_copy": ([P, P, P, P], i32),
        "ls_basis_destroy": ([P], None),
        "ls_state_info": ([P, u64, P, P, P, P, P], i32),
        "ls_index_lookup": ([P, u64, P, P, P], i32),
        "ls_operator_create": ([P, u32, P, P], i32),
        "ls_operator_destroy": ([P], None),
        "ls_operator_info": ([P, P, P], i32),
        "ls_operator_count": ([P, P, P], i32),
        "ls_operator_search_kind": ([P, P, P], i32),
        "ls_operator_check": ([P, P], i32),
        "ls_basis_test_drop_key": ([P, u64, P], i32),
        "ls_matvec": ([P, u32, P, P, P], i32),
        "ls_matvec_push": ([P, u32, P, P, P], i32),
        "ls_batch_create": ([u32, P, P, P], i32),
        "ls_batch_matvec": ([P, P, P, P], i32),
        "ls_batch_info": ([P, P, P, P], i32),
        "ls_batch_search": ([P, ctypes.c_uint32, P, P, P, P, P], i32),
        "ls_batch_set_search": ([P, ctypes.c_int, ctypes.c_uint32], i32),
        "ls_batch_set_graph": ([P, ctypes.c_int], i32),
        "ls_batch_destroy": ([P], None),
        "ls_lanczos": ([P, P, P, P, P, P], i32),
        "ls_solver_footprint": ([P, u32, P], i32),
        "ls_solver_create": ([P, P, P, P], i32),
        "ls_solver_step": ([P, u32, P], i32),
        "ls_solver_step_n": ([P, u32, u32, P], i32),
        "ls_solver_result": ([P, P, P, P, P, P], i32),
        "ls_solver_destroy": ([P], None),
        "ls_last_error": ([], ctypes.c_char_p),
        "ls_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(status: int, ok=(LS_OK,)):
    if status not in ok:
        raise LSError(status, load().ls_last_error().decode())
    return status


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t) -> ctypes.c_void_p:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("device buffers are torch tensors")
    if t.device.type != "cuda":
        raise ValueError("device buffers must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _vector(t, dim: int, cplx: bool, name: str, max_rhs: int = 64) -> int:
    """Checks a device vector [dim] or [dim][nrhs] of the operator's element
    type before its pointer reaches the library (a wrong dtype or a short
    buffer would make the kernels read or write past the allocation).
    Returns nrhs."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    want = torch.complex128 if cplx else torch.float64
    if t.dtype != want:
        raise TypeError(f"{name} must be {want}, got {t.dtype}")
    if t.dim() not in (1, 2) or t.shape[0] != dim:
        raise ValueError(f"{name} must have shape [{dim}] or [{dim}][nrhs], got {tuple(t.shape)}")
    nrhs = 1 if t.dim() == 1 else int(t.shape[1])
    if not 1 <= nrhs <= max_rhs:
        raise ValueError(f"{name}: nrhs must be in 1..{max_rhs}")
    _dptr(t)   # on the GPU, contiguous
    return nrhs


def _same_as(y, x, name: str = "y"):
    import torch
    if not isinstance(y, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if y.dtype != x.dtype or tuple(y.shape) != tuple(x.shape) or y.device != x.device:
        raise ValueError(f"{name} must match x in dtype, shape and device "
                         f"({y.dtype}, {tuple(y.shape)}, {y.device} vs {x.dtype}, {tuple(x.shape)}, {x.device})")
    _dptr(y)


def _states(t, name: str):
    """A device array of basis states / keys: 1-D int64 (uint64 bit patterns)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype not in (torch.int64, getattr(torch, "uint64", torch.int64)):
        raise TypeError(f"{name} must hold 64-bit states (int64 or uint64), got {t.dtype}")
    if t.dim() != 1:
        raise ValueError(f"{name} must be one-dimensional")
    _dptr(t)


def sector_check(n_sites: int, hamming_weight: int, perm, flip, chi) -> dict:
    """Validate a sector and compile its group on the host (ls_sector_check)."""
    L = load()
    perm = np.ascontiguousarray(perm, dtype=np.uint16)
    flip = np.ascontiguousarray(flip, dtype=np.uint8)
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    desc = SectorDesc(n_sites, hamming_weight, perm.shape[0], perm.ctypes.data, flip.ctypes.data,
                      chi.ctypes.data)
    lx, ly, pf, nc = (ctypes.c_uint32() for _ in range(4))
    _check(L.ls_sector_check(ctypes.byref(desc), ctypes.byref(lx), ctypes.byref(ly), ctypes.byref(pf),
                             ctypes.byref(nc)))
    return dict(lx=lx.value, ly=ly.value, pair_flip=pf.value, n_cosets=nc.value)


def sector_count(n_sites: int, hamming_weight: int, perm, flip, chi, rank_begin: int = 0,
                 rank_end: int = 2**64 - 1, stream=None, noalloc: bool = False) -> tuple:
    """(members, candidates) among the candidates of rank [rank_begin,
    rank_end), counted on the GPU without storing them (ls_sector_count, or
    ls_sector_count_noalloc when noalloc: no device allocation)."""
    L = load()
    perm = np.ascontiguousarray(perm, dtype=np.uint16)
    flip = np.ascontiguousarray(flip, dtype=np.uint8)
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    desc = SectorDesc(n_sites, hamming_weight, perm.shape[0], perm.ctypes.data, flip.ctypes.data,
                      chi.ctypes.data)
    m, c = ctypes.c_uint64(), ctypes.c_uint64()
    # synchronous: without a stream the count runs on the null stream
    fn = L.ls_sector_count_noalloc if noalloc else L.ls_sector_count
    _check(fn(ctypes.byref(desc), rank_begin, rank_end, ctypes.byref(m), ctypes.byref(c),
              _stream_ptr(stream) if stream is not None else None))
    return m.value, c.value


class Basis:
    """Handle of a built basis (ls_basis_build)."""

    def __init__(self, n_sites: int, hamming_weight: int, perm, flip, chi, stream=None):
        L = load()
        self._perm = np.ascontiguousarray(perm, dtype=np.uint16)
        self._flip = np.ascontiguousarray(flip, dtype=np.uint8)
        self._chi = np.ascontiguousarray(chi, dtype=np.float64)
        if self._perm.ndim != 2 or self._perm.shape[1] != n_sites:
            raise ValueError("perm must be [n_elements][n_sites]")
        desc = SectorDesc(n_sites, hamming_weight, self._perm.shape[0], self._perm.ctypes.data,
                          self._flip.ctypes.data, self._chi.ctypes.data)
        h = ctypes.c_void_p()
        _check(L.ls_basis_build(ctypes.byref(desc), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.n_sites = n_sites
        self.weight = hamming_weight
        dim = ctypes.c_uint64()
        is_real = ctypes.c_int()
        _check(L.ls_basis_info(h, ctypes.byref(dim), ctypes.byref(is_real), None))
        self.dim = int(dim.value)
        self.is_real = bool(is_real.value)

    @classmethod
    def from_sector(cls, sector, stream=None) -> "Basis":
        g = sector.group
        return cls(sector.n_sites, sector.weight, g.perm, g.flip, g.chi, stream)

    @property
    def handle(self):
        return self._h

    def copy(self, stream=None):
        """(reps int64 view of uint64, stab int16 view of uint16) as new device tensors."""
        import torch
        reps = torch.empty(max(self.dim, 1), dtype=torch.int64, device="cuda")
        stab = torch.empty(max(self.dim, 1), dtype=torch.int16, device="cuda")
        _check(load().ls_basis_copy(self._h, _dptr(reps), _dptr(stab), _stream_ptr(stream)))
        return reps[: self.dim], stab[: self.dim]

    def state_info(self, states, stream=None):
        import torch
        _states(states, "states")
        n = states.numel()
        reps = torch.empty(n, dtype=torch.int64, device=states.device)
        chi = torch.empty((n, 2), dtype=torch.float64, device=states.device)
        norm = torch.empty(n, dtype=torch.float64, device=states.device)
        if n:
            _check(load().ls_state_info(self._h, n, _dptr(states), _dptr(reps), _dptr(chi), _dptr(norm),
                                        _stream_ptr(stream)))
        return reps, chi, norm

    def index_lookup(self, keys, stream=None):
        import torch
        _states(keys, "keys")
        n = keys.numel()
        out = torch.empty(n, dtype=torch.int64, device=keys.device)
        if n:
            _check(load().ls_index_lookup(self._h, n, _dptr(keys), _dptr(out), _stream_ptr(stream)))
        return out

    def test_drop_key(self, index: int, stream=None):
        """Fault injection for tests: take representative `index` out of the
        hash index so that products meeting it raise the lookup-miss flag
        (ls_basis_test_drop_key)."""
        _check(load().ls_basis_test_drop_key(self._h, int(index), _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None):
            load().ls_basis_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def terms_to_ctypes(term_table) -> ctypes.Array:
    n = len(term_table)
    arr = (Term * max(n, 1))()
    for k in range(n):
        t = term_table[k]
        arr[k] = Term(float(t["re"]), float(t["im"]), int(t["sel_mask"]), int(t["sel_value"]),
                      int(t["flip"]), int(t["sign_mask"]))
    return arr



REORTH_CODES = {"none": 0, "full": 1, "selective": 2}


def reorth_code(reorth) -> int:
    """ls_lanczos_opts.reorth from True/False, "none"/"full"/"selective" or 0/1/2:
    none, full CGS2 (two Gram-Schmidt passes every step), or a second pass only
    when the first removed more than half of ||w||^2."""
    if isinstance(reorth, str):
        return REORTH_CODES[reorth]
    if isinstance(reorth, bool):
        return 1 if reorth else 0
    code = int(reorth)
    if code not in (0, 1, 2):
        raise ValueError("reorth must be 0, 1 or 2")
    return code


class Operator:
    """Handle of a compiled Hamiltonian (ls_operator_create)."""

    def __init__(self, basis: Basis, term_table):
        L = load()
        self.basis = basis
        self._terms = terms_to_ctypes(term_table)
        h = ctypes.c_void_p()
        _check(L.ls_operator_create(basis.handle, len(term_table), self._terms, ctypes.byref(h)))
        self._h = h
        c = ctypes.c_int()
        _check(L.ls_operator_info(h, ctypes.byref(c), None))
        self.is_complex = bool(c.value)
        self.dim = basis.dim

    @property
    def handle(self):
        return self._h

    def count_elements(self, stream=None) -> int:
        """Off-diagonal element applications of one product (ls_operator_count)."""
        n = ctypes.c_uint64()
        _check(load().ls_operator_count(self._h, ctypes.byref(n), _stream_ptr(stream)))
        return int(n.value)

    SEARCH_KINDS = ("generic", "ring32", "torus", "ring64")

    def search_kind(self):
        """(orbit search of the products, compile-time torus shape) as
        ("generic" | "ring32" | "torus" | "ring64", bool) (ls_operator_search_kind)."""
        k = ctypes.c_uint32()
        f = ctypes.c_uint32()
        _check(load().ls_operator_search_kind(self._h, ctypes.byref(k), ctypes.byref(f)))
        return self.SEARCH_KINDS[k.value], bool(f.value)

    def check(self, stream=None):
        """Raise LSError(LS_EINTERNAL) when a product since the last check met a
        lookup miss of an in-sector representative (ls_operator_check)."""
        _check(load().ls_operator_check(self._h, _stream_ptr(stream)))

    def store(self, max_bytes: int = 2**64 - 1, stream=None) -> int:
        """Keep the matrix elements in device memory for later products
        (ls_operator_store); returns the bytes held."""
        b = ctypes.c_uint64()
        _check(load().ls_operator_store(self._h, int(max_bytes), _stream_ptr(stream), ctypes.byref(b)))
        return int(b.value)

    def matvec(self, x, y=None, stream=None):
        """y = H x for x of shape [dim] or [dim][nrhs] (float64 / complex128)."""
        import torch
        nrhs = _vector(x, self.dim, self.is_complex, "x")
        if y is None:
            y = torch.empty_like(x)
        _same_as(y, x)
        _check(load().ls_matvec(self._h, nrhs, _dptr(x), _dptr(y), _stream_ptr(stream)))
        return y

    def matvec_push(self, x, y=None, stream=None):
        """y = H x in the push (transposed, atomic) form (ls_matvec_push)."""
        import torch
        nrhs = _vector(x, self.dim, self.is_complex, "x")
        if y is None:
            y = torch.empty_like(x)
        _same_as(y, x)
        _check(load().ls_matvec_push(self._h, nrhs, _dptr(x), _dptr(y), _stream_ptr(stream)))
        return y

    def lanczos(self, max_iter: int, tol: float = 0.0, seed: int = 1, v0=None, reorth=True,
                stream=None):
        m = int(max_iter)
        if m < 1:
            raise ValueError("max_iter must be >= 1")
        if v0 is not None:
            _vector(v0, self.dim, self.is_complex, "v0", max_rhs=1)
        alpha = np.zeros(m)
        beta = np.zeros(m)
        opts = LanczosOpts(m, reorth_code(reorth), float(tol), int(seed),
                           _dptr(v0) if v0 is not None else None, alpha.ctypes.data, beta.ctypes.data)
        e0 = ctypes.c_double()
        it = ctypes.c_uint32()
        res = ctypes.c_double()
        st = _check(load().ls_lanczos(self._h, ctypes.byref(opts), _stream_ptr(stream), ctypes.byref(e0),
                                      ctypes.byref(it), ctypes.byref(res)), ok=(LS_OK, LS_WNOTCONV))
        k = int(it.value)
        return dict(e0=e0.value, iters=k, resid=res.value, alpha=alpha[:k].copy(),
                    beta=beta[: max(k - 1, 0)].copy(), converged=(st == LS_OK) and tol > 0)

    def close(self):
        if getattr(self, "_h", None):
            load().ls_operator_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """One Lanczos solve advanced step by step (ls_solver_create); many
    solvers advance together with Solver.step_all (one fused product)."""

    def __init__(self, op: "Operator", max_iter: int, tol: float = 0.0, seed: int = 1, v0=None,
                 reorth=True, stream=None):
        self.op = op
        if int(max_iter) < 1:
            raise ValueError("max_iter must be >= 1")
        if v0 is not None:
            _vector(v0, op.dim, op.is_complex, "v0", max_rhs=1)
        opts = LanczosOpts(int(max_iter), reorth_code(reorth), float(tol), int(seed),
                           _dptr(v0) if v0 is not None else None, None, None)
        h = ctypes.c_void_p()
        _check(load().ls_solver_create(op.handle, ctypes.byref(opts), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def footprint(op: "Operator", max_iter: int) -> int:
        b = ctypes.c_uint64()
        _check(load().ls_solver_footprint(op.handle, int(max_iter), ctypes.byref(b)))
        return int(b.value)

    @staticmethod
    def step_all(solvers, stream=None, steps: int = 1):
        """One iteration of every solver (ls_solver_step), or up to `steps`
        with one synchronisation (ls_solver_step_n)."""
        n = len(solvers)
        if n == 0:
            return
        arr = (ctypes.c_void_p * n)(*[s._h.value for s in solvers])
        if steps == 1:
            _check(load().ls_solver_step(arr, n, _stream_ptr(stream)))
        else:
            _check(load().ls_solver_step_n(arr, n, int(steps), _stream_ptr(stream)))

    def result(self) -> dict:
        e0, res = ctypes.c_double(), ctypes.c_double()
        it = ctypes.c_uint32()
        done, conv = ctypes.c_int(), ctypes.c_int()
        _check(load().ls_solver_result(self._h, ctypes.byref(e0), ctypes.byref(it), ctypes.byref(res),
                                       ctypes.byref(done), ctypes.byref(conv)))
        return dict(e0=e0.value, iters=it.value, resid=res.value, done=bool(done.value),
                    converged=bool(conv.value))

    def close(self):
        if getattr(self, "_h", None):
            load().ls_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Handle of a batched product (ls_batch_create): many operators, each
    with its own number of right-hand sides, in one persistent launch per
    kernel variant, replayed from a HIP graph."""

    def __init__(self, ops, nrhs, graph: bool = True, search=None):
        L = load()
        self.ops = list(ops)
        self.nrhs = [int(v) for v in nrhs]
        if len(self.ops) != len(self.nrhs) or not self.ops:
            raise ValueError("ops and nrhs must be non-empty and of equal length")
        n = len(self.ops)
        self._handles = (ctypes.c_void_p * n)(*[op.handle.value for op in self.ops])
        self._nrhs = (ctypes.c_uint32 * n)(*self.nrhs)
        h = ctypes.c_void_p()
        _check(L.ls_batch_create(n, self._handles, self._nrhs, ctypes.byref(h)))
        self._h = h
        if not graph:
            _check(L.ls_batch_set_graph(h, 0))
        if search is not None:
            # ("buckets", bits), ("staged", bits) or "own": ls_batch_set_search
            mode, bits = (search, 0) if isinstance(search, str) else search
            code = {"buckets": 0, "own": 3, "staged": 4}[mode]
            _check(L.ls_batch_set_search(h, code, int(bits)))

    def matvec(self, xs, ys, stream=None):
        """ys[k] = H_k xs[k] for every k (torch tensors [dim_k][nrhs_k])."""
        n = len(self.ops)
        if len(xs) != n or len(ys) != n:
            raise ValueError("one x and one y per operator")
        for k, (op, x, y, r) in enumerate(zip(self.ops, xs, ys, self.nrhs)):
            if _vector(x, op.dim, op.is_complex, f"xs[{k}]") != r:
                raise ValueError(f"xs[{k}] does not have nrhs = {r} columns")
            _same_as(y, x, f"ys[{k}]")
        px = (ctypes.c_void_p * n)(*[_dptr(x).value for x in xs])
        py = (ctypes.c_void_p * n)(*[_dptr(y).value for y in ys])
        _check(load().ls_batch_matvec(self._h, px, py, _stream_ptr(stream)))
        return ys

    def info(self) -> dict:
        a, b, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(load().ls_batch_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return dict(launches=a.value, tiles=b.value, graph=bool(c.value))

    SEARCH_MODES = {0: "buckets", 1: "rank", 2: "identity", 3: "hash", 4: "staged"}

    def search(self, item: int) -> dict:
        """Search layout used for operator `item` and the lookup sweep times
        behind the choice (ls_batch_search)."""
        m, b = ctypes.c_uint32(), ctypes.c_uint32()
        o, c, s = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(load().ls_batch_search(self._h, int(item), ctypes.byref(m), ctypes.byref(b), ctypes.byref(o),
                                      ctypes.byref(c), ctypes.byref(s)))
        return dict(mode=self.SEARCH_MODES.get(m.value, str(m.value)), bits=b.value, own_ns=o.value,
                    chosen_ns=c.value, staged_ns=s.value)

    def close(self):
        if getattr(self, "_h", None):
            load().ls_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
