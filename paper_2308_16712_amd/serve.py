"""Serving loop: Lanczos ground-state requests with continuous batching.

Requests (a sector and its Hamiltonian) arrive over time.  The server
admits a queued request when its HBM footprint fits the budget, builds its
basis and operator, and creates a Lanczos solver whose Krylov vectors stay
resident.  Every iteration of the loop advances *all* admitted solves by one
Lanczos step with one fused product launch (ls_solver_step); a solve leaves
as soon as it converges and its memory returns to the budget, so requests
that arrive while others run join the next step.

The baseline serves the same trace one request at a time with ls_lanczos.

The footprint is known before anything is allocated: the sector dimension
follows from the character formula dim = (1/|G|) sum_g conj(chi(g)) fix_w(g),
where fix_w(g) counts the weight-w states that g fixes (a product over the
cycles of the permutation).
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from ._lib import LS_EINTERNAL, Basis, LSError, Operator, Solver


def _cycles(perm) -> List[int]:
    n = len(perm)
    seen = [False] * n
    out = []
    for i in range(n):
        if seen[i]:
            continue
        L, j = 0, i
        while not seen[j]:
            seen[j] = True
            j = int(perm[j])
            L += 1
        out.append(L)
    return out


def _fixed(perm, flip, n, w) -> int:
    cyc = _cycles(perm)
    if flip:
        if any(L % 2 for L in cyc) or (w >= 0 and 2 * w != n):
            return 0
        return 2 ** len(cyc)
    if w < 0:
        return 2 ** len(cyc)
    poly = [1]
    for L in cyc:
        nxt = [0] * (len(poly) + L)
        for k, c in enumerate(poly):
            nxt[k] += c
            nxt[k + L] += c
        poly = nxt
    return poly[w] if w < len(poly) else 0


def sector_dimension(sector) -> int:
    g = sector.group
    chi = g.chi[:, 0] - 1j * g.chi[:, 1]          # conj(chi)
    tot = 0j
    for e in range(g.size):
        tot += chi[e] * _fixed(g.perm[e], g.flip[e], sector.n_sites, sector.weight)
    return int(round((tot / g.size).real))


def _search_bytes(dim: int) -> int:
    """Hash index of the basis build: 16-byte slots, a power of two with load
    factor at most 1/8 while the table fits 8 GiB, else 1/4 within 64 GiB,
    else 1/2 or 3/4 within 128 GiB (the library's hash_capacity); above that
    the bucket table (at most 2^22 + 1 four-byte offsets)."""
    for num, den, limit in ((8, 1, 8 << 30), (4, 1, 64 << 30), (2, 1, 128 << 30), (4, 3, 128 << 30)):
        cap = 1024
        while cap * den < num * dim:
            cap *= 2
        if cap * 16 <= limit:
            return cap * 16
    return ((1 << 22) + 1) * 4


def footprint_bytes(sector, max_iter: int) -> int:
    """Device bytes a request holds while admitted: representatives and
    stabilizers, search layout, Krylov space, and the build's mark words."""
    from math import comb
    dim = sector_dimension(sector)
    complex_ = not (np.all(sector.group.chi[:, 1] == 0) and np.all(sector.terms["im"] == 0))
    es = 16 if complex_ else 8
    m = min(max_iter, max(dim, 1))
    cand = comb(sector.n_sites, sector.weight) if sector.weight >= 0 else 2 ** sector.n_sites
    return dim * 10 + _search_bytes(dim) + (m + 1) * dim * es + 2048 * m * 16 + cand // 8 + (64 << 20)


@dataclass
class Record:
    rid: int
    name: str
    dim: int
    arrival: float
    admitted: float = 0.0
    done: float = 0.0
    e0: float = float("nan")
    iters: int = 0
    converged: bool = False
    status: str = "ok"        # ok | rejected | failed | cancelled
    error: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Live:
    rec: Record
    basis: Basis
    op: Operator
    solver: Solver
    bytes: int


@dataclass
class ServeStats:
    records: List[Record] = field(default_factory=list)
    makespan: float = 0.0
    steps: int = 0
    max_active: int = 0
    peak_bytes: int = 0
    build_s: float = 0.0      # basis + operator (+ element store) set-up
    stored_bytes: int = 0     # matrix elements stored over the run
    step_s: float = 0.0       # Lanczos steps (or whole solves, one at a time)

    def summary(self) -> dict:
        ok = [r for r in self.records if r.status == "ok"]
        lat = np.array([r.latency for r in ok] or [0.0]) * 1e3
        by = {k: sum(r.status == k for r in self.records) for k in ("ok", "rejected", "failed", "cancelled")}
        return dict(requests=len(self.records), completed=len(ok), makespan_s=self.makespan,
                    throughput_rps=len(ok) / self.makespan if self.makespan > 0 else 0.0,
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    mean_ms=float(lat.mean()), steps=self.steps, max_active=self.max_active,
                    peak_bytes=self.peak_bytes, build_s=self.build_s, step_s=self.step_s,
                    stored_bytes=self.stored_bytes, status=by,
                    converged=int(sum(r.converged for r in ok)))


def _wait_until(t0: float, t: float):
    d = t - (time.perf_counter() - t0)
    if d > 0:
        time.sleep(d)


SMALL_DIM = 1 << 20   # below this a single product cannot fill the GPU
# Steps of a lone small solve per synchronisation (ls_solver_step_n): a step
# of a small solve costs about as much as a synchronisation, and ls_lanczos
# runs the same chunks, so a lone small solve is served at the one-at-a-time
# pace; an arrival waits at most one chunk to join.
SMALL_CHUNK = 8


def _steps_per_sync(step) -> int:
    """Iterations per synchronisation for the solves advanced together: a
    lone small solve takes SMALL_CHUNK; a fused step of a few small solves
    takes fewer, since every solve that converges inside a chunk has the
    rest of the chunk computed and discarded; many solves, or a large one,
    take single steps (their step already outweighs the synchronisation)."""
    if any(lv.rec.dim >= SMALL_DIM for lv in step):
        return 1
    if len(step) == 1:
        return SMALL_CHUNK
    return 4 if len(step) <= 3 else 1


def _pick(live, policy: str):
    """Solves advanced in this iteration.

    "sjf" (default): while any small solve is admitted (its product alone
    cannot fill the GPU), the iteration advances all small solves together
    in one fused step and nothing else; otherwise the large solve with the
    smallest dimension advances (ties: oldest first).  Large solves saturate
    the device on their own, so running them one at a time, shortest first
    and preemptively (a paused solve keeps its Krylov space resident), loses
    no throughput and minimises the mean latency.
    "fifo": as "sjf", but the oldest large solve advances.
    "all": every admitted solve in one fused step (plain lock-step)."""
    if policy == "all":
        return list(live)
    small = [lv for lv in live if lv.rec.dim < SMALL_DIM]
    if small:
        return small
    if policy == "fifo":
        return [min(live, key=lambda lv: (lv.rec.arrival, lv.rec.rid))]
    return [min(live, key=lambda lv: (lv.rec.dim, lv.rec.arrival, lv.rec.rid))]


def serve(trace, hbm_budget: int, max_iter: int = 150, tol: float = 1e-10, log=None,
          policy: str = "sjf", store_elements: bool = False, cancel: Optional[Dict[int, float]] = None,
          on_built: Optional[Callable] = None) -> ServeStats:
    """Continuous batching: admit by footprint, advance the admitted solves
    with fused steps (see _pick), retire converged ones.  Arrivals are
    replayed in real time.

    Bases and operators of admitted requests are built by a worker thread on
    a stream of their own while the loop keeps stepping the live solves on
    another (the library releases the interpreter lock in every call); a
    request joins the steps once its build has finished.

    With store_elements, the builder also stores the operator's matrix
    elements (ls_operator_store) when they fit the budget left at that
    moment; the solve then steps with stored products (results identical bit
    for bit) and the stored bytes count against the budget until it retires.

    One request cannot take the others down: a request whose footprint
    exceeds the whole budget is rejected on arrival; a failed build, a
    failed solver creation or a solve stopped by the library (LS_EINTERNAL,
    a lookup miss in its product) fails that request only, and its memory
    returns to the budget.  cancel maps a request id to a time (seconds
    since the start) at which it is withdrawn, wherever it then is: queued,
    building or stepping.  Every request ends with a record whose status is
    ok, rejected, failed or cancelled.  on_built(request, basis, operator),
    if given, is called after each build (a test hook)."""
    import torch
    from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait

    pending = sorted(trace, key=lambda r: r.arrival)
    queue: List = []
    live: List[_Live] = []
    building = []           # (request, bytes, record, future)
    needs = {}              # request id -> footprint bytes
    cancel = dict(cancel or {})
    stats = ServeStats()
    step_stream = torch.cuda.Stream()
    build_stream = torch.cuda.Stream()

    lock = threading.Lock()
    budget = {"used": 0}
    t0 = time.perf_counter()

    def now():
        return time.perf_counter() - t0

    def finish(rec, status, error=""):
        rec.status, rec.error = status, error
        rec.done = now()
        stats.records.append(rec)
        if log and status != "ok":
            log(f"[serve] t={rec.done:.3f}s {status} {rec.rid} {rec.name}: {error}")

    def release(nbytes):
        with lock:
            budget["used"] -= nbytes

    def build(req):
        t = time.perf_counter()
        b = Basis.from_sector(req.sector, build_stream)
        try:
            op = Operator(b, req.sector.terms)
        except Exception:
            b.close()
            raise
        stored = 0
        if store_elements:
            with lock:      # reserve what is left of the budget for the store
                room = max(hbm_budget - budget["used"], 0)
                budget["used"] += room
            try:
                stored = op.store(room, build_stream)
            except LSError:
                stored = 0
            with lock:      # keep what the store holds, return the rest
                budget["used"] -= room - stored
        if on_built is not None:
            on_built(req, b, op)
        return b, op, stored, time.perf_counter() - t

    def retire(lv, status, error=""):
        lv.solver.close()
        lv.op.close()
        lv.basis.close()
        release(lv.bytes)
        finish(lv.rec, status, error)

    pool = ThreadPoolExecutor(max_workers=1)
    i = 0
    try:
        with torch.cuda.stream(step_stream):
            while i < len(pending) or queue or live or building:
                while i < len(pending) and pending[i].arrival <= now():
                    queue.append(pending[i])
                    i += 1
                # withdrawn requests: queued ones leave at once, live ones now,
                # building ones when their build returns
                due = {rid for rid, tc in cancel.items() if tc <= now()}
                for req in [q for q in queue if q.rid in due]:
                    queue.remove(req)
                    cancel.pop(req.rid)
                    finish(Record(req.rid, req.sector.name, 0, req.arrival), "cancelled", "withdrawn while queued")
                for lv in [lv for lv in live if lv.rec.rid in due]:
                    live.remove(lv)
                    cancel.pop(lv.rec.rid)
                    retire(lv, "cancelled", f"withdrawn after {lv.solver.result()['iters']} steps")
                # first-fit admission in arrival order; the build starts now
                for req in list(queue):
                    if req.rid not in needs:     # the character formula runs once per request
                        needs[req.rid] = footprint_bytes(req.sector, max_iter)
                    need = needs[req.rid]
                    if need > hbm_budget:
                        queue.remove(req)
                        finish(Record(req.rid, req.sector.name, 0, req.arrival), "rejected",
                               f"needs {need} bytes, more than the whole budget of {hbm_budget}")
                        continue
                    with lock:
                        if budget["used"] + need > hbm_budget:
                            continue
                        budget["used"] += need
                        stats.peak_bytes = max(stats.peak_bytes, budget["used"])
                    queue.remove(req)
                    rec = Record(req.rid, req.sector.name, 0, req.arrival, admitted=now())
                    building.append((req, need, rec, pool.submit(build, req)))
                # finished builds join the live set
                for item in list(building):
                    req, need, rec, fut = item
                    if not fut.done():
                        continue
                    building.remove(item)
                    try:
                        b, op, stored, dt = fut.result()
                    except Exception as e:   # this request only
                        release(need)
                        finish(rec, "failed", f"build: {e}")
                        continue
                    stats.build_s += dt
                    stats.stored_bytes += stored
                    with lock:
                        stats.peak_bytes = max(stats.peak_bytes, budget["used"])
                    rec.dim = b.dim
                    if req.rid in cancel and cancel[req.rid] <= now():
                        cancel.pop(req.rid)
                        op.close()
                        b.close()
                        release(need + stored)
                        finish(rec, "cancelled", "withdrawn while building")
                        continue
                    try:
                        s = Solver(op, max_iter, tol=tol, seed=req.sector.seed)
                    except LSError as e:
                        op.close()
                        b.close()
                        release(need + stored)
                        finish(rec, "failed", f"solver: {e}")
                        continue
                    live.append(_Live(rec, b, op, s, need + stored))
                    if log:
                        log(f"[serve] t={now():.3f}s start {req.rid} {req.sector.name} "
                            f"dim={b.dim} active={len(live)}")
                if live:
                    stats.max_active = max(stats.max_active, len(live))
                    step = _pick(live, policy)
                    ts = time.perf_counter()
                    try:
                        Solver.step_all([lv.solver for lv in step], steps=_steps_per_sync(step))
                    except LSError as e:
                        # the stopped solves report LS_EINTERNAL in their result;
                        # anything else is not a per-request condition
                        if e.status != LS_EINTERNAL:
                            raise
                    stats.step_s += time.perf_counter() - ts
                    stats.steps += 1
                    keep = []
                    stepped = {id(lv) for lv in step}
                    for lv in live:
                        if id(lv) not in stepped:
                            keep.append(lv)
                            continue
                        try:
                            r = lv.solver.result()
                        except LSError as e:
                            if e.status != LS_EINTERNAL:
                                raise
                            retire(lv, "failed", str(e))
                            continue
                        if r["done"]:
                            lv.rec.e0, lv.rec.iters, lv.rec.converged = r["e0"], r["iters"], r["converged"]
                            retire(lv, "ok")
                        else:
                            keep.append(lv)
                    live = keep
                elif building:
                    wait([item[3] for item in building], return_when=FIRST_COMPLETED, timeout=0.05)
                elif i < len(pending) and not queue:
                    later = [tc for tc in cancel.values() if tc > now()]
                    _wait_until(t0, min([pending[i].arrival] + later))
    finally:
        pool.shutdown(wait=True)
    step_stream.synchronize()
    stats.makespan = now()
    stats.records.sort(key=lambda r: r.rid)
    return stats


def serve_one_at_a_time(trace, max_iter: int = 150, tol: float = 1e-10, store_elements: bool = False,
                        hbm_budget: Optional[int] = None) -> ServeStats:
    """Baseline: each request in arrival order, alone, with ls_lanczos.  With
    store_elements each operator's elements are stored first (when they fit
    hbm_budget less the request's footprint), as the server does."""
    pending = sorted(trace, key=lambda r: r.arrival)
    stats = ServeStats()
    t0 = time.perf_counter()
    for req in pending:
        _wait_until(t0, req.arrival)
        tb = time.perf_counter()
        rec = Record(req.rid, req.sector.name, 0, req.arrival, admitted=tb - t0)
        need = footprint_bytes(req.sector, max_iter)
        if hbm_budget is not None and need > hbm_budget:
            rec.status, rec.error = "rejected", "footprint above the budget"
            rec.done = time.perf_counter() - t0
            stats.records.append(rec)
            continue
        b = Basis.from_sector(req.sector)
        op = Operator(b, req.sector.terms)
        if store_elements:
            room = (hbm_budget if hbm_budget is not None else 1 << 62) - need
            try:
                stats.stored_bytes += op.store(max(room, 0))
            except LSError:
                pass
        ts = time.perf_counter()
        stats.build_s += ts - tb
        r = op.lanczos(max_iter, tol=tol, seed=req.sector.seed)
        stats.step_s += time.perf_counter() - ts
        rec.dim = b.dim
        rec.done = time.perf_counter() - t0
        rec.e0, rec.iters, rec.converged = r["e0"], r["iters"], r["converged"]
        stats.records.append(rec)
        stats.steps += r["iters"]
        op.close()
        b.close()
    stats.makespan = time.perf_counter() - t0
    stats.max_active = 1
    stats.records.sort(key=lambda r: r.rid)
    return stats
