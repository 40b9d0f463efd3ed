"""Benchmark: H matrix elements applied per second on one MI355X.

Workload (default): square-lattice J1-J2 Heisenberg model on a 6x6 torus,
J1 = 1, J2 = 0.5, Sz = 0, k = (0,0), full C4v x translations x spin
inversion (576 elements), 15,804,956 representatives, FP64 vectors.

A step is one on-the-fly product y = H x over the whole sector (getRow,
orbit minimum, stateToIndex and accumulation for every row); the basis is
built once before timing (its build time is reported beside the metric).
Element applications per step = (off-diagonal terms acting on each row,
summed over rows) + one diagonal element per row.

Prints one JSON line.  ``--gpus`` > 1 is not supported (one GPU only).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12            # B/s, MI355X HBM3E
# Integer/logic VALU lane-operations per second: 256 CUs x 4 SIMDs x 16
# lanes per clock x 2.4 GHz (one 32-bit op per lane per clock).
PEAK_VALU = 256 * 64 * 2.4e9
# Algorithmic HBM bytes of the on-the-fly product: per row the
# representative, x_i and y_i (8 B each); per off-diagonal element the
# gathered x_j and the matched key of stateToIndex (8 B each).
ALG_ROW_BYTES = 24
ALG_ELEMENT_BYTES = 16


def workload(name: str):
    from workloads import configs
    if name == "square6x6":
        return configs.square_j1j2(), "square-lattice J1-J2 6x6 torus (J2=0.5), Sz=0, k=0, C4v x T x Z2 (576)"
    if name == "ring32":
        return configs.ring32_symmetric(), "Heisenberg ring N=32, Sz=0, k=0, R=+1, Z=+1 (128)"
    if name == "ring16":
        return configs.ring16_u1(), "Heisenberg ring N=16, Sz=0, no lattice symmetry"
    if name == "chain40":
        return configs.ring_symmetric(40, 0, 1, 1), "Heisenberg chain N=40 (Table 2), Sz=0, k=0, R=+1, Z=+1 (160)"
    raise SystemExit(f"unknown workload {name}")


def count_elements(reps, term_table):
    """(off-diagonal element applications, rows) of one product."""
    import numpy as np
    off = term_table[term_table["flip"] != 0]
    n_off = 0
    for lo in range(0, len(reps), 1 << 22):
        r = reps[lo: lo + (1 << 22)]
        for t in off:
            n_off += int(np.count_nonzero((r & np.uint64(t["sel_mask"])) == np.uint64(t["sel_value"])))
    return n_off, len(reps)


def host_cores() -> int:
    """Host threads for the oracle: the GPU's share of the host (at most 16)."""
    return max(1, min(16, os.cpu_count() or 1))


def cpu_baseline(sector, budget_s: float):
    """The oracle's getRow timed on the host cores, as it stands: rows drawn
    by the oracle itself (seeded random states of the sector's weight ->
    their representatives in the sector), first on one thread, then split
    over all host cores (rows in parallel), each until its share of the time
    budget is spent."""
    import numpy as np
    import oracle
    from workloads import rng
    P = oracle.Problem(sector)
    n = sector.n_sites
    w = sector.weight
    # seeded random weight-w states: the w sites with the smallest counter
    # values of each row of an m x n draw
    m = 65536
    keys = rng.counter_u64(2024, np.arange(m * n, dtype=np.uint64)).reshape(m, n)
    sites = np.argsort(keys, axis=1, kind="stable")[:, :w].astype(np.uint64)
    states = np.bitwise_or.reduce(np.left_shift(np.uint64(1), sites), axis=1)
    reps, chi, norm = oracle.state_info(P, states, workers=host_cores())
    rows = np.unique(reps[norm > 0])
    off = sector.terms[sector.terms["flip"] != 0]
    acting = [int(np.count_nonzero((np.uint64(r) & off["sel_mask"]) == off["sel_value"])) + 1 for r in rows]

    # one thread
    t0 = time.perf_counter()
    e1 = d1 = 0
    for r, a in zip(rows, acting):
        oracle.get_row(P, int(r))
        e1 += a
        d1 += 1
        if time.perf_counter() - t0 > budget_s / 3:
            break
    dt1 = time.perf_counter() - t0
    # all host cores: the rows not used above, in chunks, until the budget is spent
    cores = host_cores()
    t0 = time.perf_counter()
    ea = da = 0
    k = d1
    while k < len(rows) and time.perf_counter() - t0 < budget_s * 2 / 3:
        chunk = rows[k:k + 64 * cores]
        oracle.get_rows(P, chunk, workers=cores)
        ea += sum(acting[k:k + len(chunk)])
        da += len(chunk)
        k += len(chunk)
    dta = time.perf_counter() - t0
    return {"value": ea / dta, "unit": "elements/s", "cores": cores, "kind": "oracle",
            "sample": f"getRow of {da} representatives ({ea} element applications) in {dta:.1f} s on {cores} "
                      f"host threads; rows drawn by the oracle from seeded random weight-{w} states",
            "single_thread": {"value": e1 / dt1, "unit": "elements/s", "cores": 1,
                              "sample": f"getRow of {d1} representatives, {e1} element applications in {dt1:.1f} s"},
            "host_cpu_count": os.cpu_count()}


def copy_peak(mib: int = 4096, reps: int = 5):
    """A plain device-to-device copy (the HBM rate a streaming kernel can
    reach on this GPU): bytes read + written per second, best of reps."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    stream = torch.cuda.current_stream()
    best = 1e30
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        b.copy_(a)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return {"bytes": 2 * n * 8, "ms": best, "gbps": 2 * n * 8 / (best * 1e-3) / 1e9,
            "frac_of_spec": 2 * n * 8 / (best * 1e-3) / PEAK_HBM}


def small_configs(steps: int):
    """The product alone on the N=16 ring (no lattice symmetry) and the
    N=32 symmetric ring: elements applied per second and the algorithmic HBM
    rate, per product on the launch stream."""
    import torch
    import paper_2308_16712_amd as ls
    from workloads import configs, rng

    out = {}
    for key, sec, desc in (("ring16", configs.ring16_u1(), "Heisenberg ring N=16, Sz=0, no lattice symmetry"),
                           ("ring32", configs.ring32_symmetric(),
                            "Heisenberg ring N=32, Sz=0, k=0, R=+1, Z=+1 (128)")):
        b = ls.ls_basis_build(sec)
        op = ls.ls_operator_create(b, sec.terms)
        n_off = op.count_elements()
        x = torch.from_numpy(rng.vector(sec.seed, b.dim)).cuda()
        y = torch.empty_like(x)
        ls.ls_matvec(op, x, y)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = max(steps, 50 if b.dim < 1 << 20 else steps)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            ls.ls_matvec(op, x, y)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        op.check()
        elements = n_off + b.dim
        alg = b.dim * ALG_ROW_BYTES + n_off * ALG_ELEMENT_BYTES
        out[key] = {"workload": desc, "dim": b.dim, "elements_per_product": elements, "ms_per_product": ms,
                    "elements_per_s": elements / (ms * 1e-3), "hbm_algorithmic_gbps": alg / (ms * 1e-3) / 1e9,
                    "orbit_search": op.search_kind()[0]}
        op.close()
        b.close()
    return out


def batched_vs_plain(count: int, nrhs: int, reps_timed: int = 3):
    """64 independent ring sectors (N uniform in {20..32}, J2 ~ U[0,0.6],
    random k, translations only, complex), nrhs right-hand sides each:
    one batched call (persistent launch, graph replay) vs count*nrhs plain
    single-RHS ls_matvec calls on the same data."""
    import numpy as np
    import torch
    import paper_2308_16712_amd as ls
    from workloads import configs, rng

    secs = configs.batched_rings(count)
    ops, xs, ys, xp, yp = [], [], [], [], []
    elements = 0
    t0 = time.perf_counter()
    for k, sec in enumerate(secs):
        b = ls.ls_basis_build(sec)
        op = ls.ls_operator_create(b, sec.terms)
        elements += (op.count_elements() + b.dim) * nrhs
        x = torch.from_numpy(rng.vector(sec.seed, b.dim, nrhs, complex_=op.is_complex)).cuda()
        ops.append(op)
        xs.append(x)
        ys.append(torch.empty_like(x))
        xp.append([x[:, q].contiguous() for q in range(nrhs)])
        yp.append([torch.empty_like(xp[-1][q]) for q in range(nrhs)])
    build_s = time.perf_counter() - t0
    batch = ls.Batch(ops, [nrhs] * count)
    batch.matvec(xs, ys)          # tunes and captures
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def timed(fn):
        best = 1e30
        for _ in range(reps_timed):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    def plain():
        for op, xl, yl in zip(ops, xp, yp):
            for q in range(nrhs):
                ls.ls_matvec(op, xl[q], yl[q])

    ym = [torch.empty_like(x) for x in xs]

    def plain_multi():
        for op, x, y in zip(ops, xs, ym):
            ls.ls_matvec(op, x, y)

    t_batch = timed(lambda: batch.matvec(xs, ys))
    t_plain = timed(plain)
    t_multi = timed(plain_multi)
    # the same batch with every search layout fixed to the largest bucket
    # table staged in LDS (2^13 buckets), for comparison with the tuned choice
    staged = ls.Batch(ops, [nrhs] * count, search=("staged", 13))
    ys_st = [torch.empty_like(x) for x in xs]
    staged.matvec(xs, ys_st)
    t_staged = timed(lambda: staged.matvec(xs, ys_st))
    for op in ops:
        op.check()
    # same results (the row arithmetic is shared)
    same = all(torch.equal(ys[k][:, q], yp[k][q]) for k in range(count) for q in range(nrhs))
    same = same and all(torch.equal(ys[k], ym[k]) and torch.equal(ys[k], ys_st[k]) for k in range(count))
    dims = [op.dim for op in ops]
    layouts = [batch.search(k) for k in range(count)]
    chosen = {}
    for lay in layouts:
        chosen[lay["mode"]] = chosen.get(lay["mode"], 0) + 1
    med = lambda v: float(np.median(v)) if v else None
    search = {"chosen": chosen,
              "median_ns_per_lookup": {"own": med([l["own_ns"] for l in layouts if l["own_ns"] > 0]),
                                       "chosen": med([l["chosen_ns"] for l in layouts if l["chosen_ns"] > 0]),
                                       "best_staged": med([l["staged_ns"] for l in layouts if l["staged_ns"] > 0])},
              "all_staged_13_bits_ms": t_staged,
              "note": "per basis the tuner times lookup sweeps of its own layout (hash index), bucket tables "
                      "in global memory and bucket tables staged in LDS, and keeps the fastest"}
    staged.close()
    return {"sectors": count, "nrhs": nrhs, "dtype": "c128", "dim_min": min(dims), "dim_max": max(dims),
            "dim_total": int(sum(dims)), "element_applications": elements,
            "batched_ms": t_batch, "plain_ms": t_plain, "speedup": t_plain / t_batch,
            "plain_multi_rhs_ms": t_multi, "speedup_vs_plain_multi_rhs": t_multi / t_batch,
            "batched_elements_per_s": elements / (t_batch * 1e-3),
            "plain_elements_per_s": elements / (t_plain * 1e-3),
            "identical_results": bool(same), "launches_batched": batch.info()["launches"],
            "search_layout": search,
            "launches_plain": count * nrhs, "launches_plain_multi_rhs": count, "basis_build_s": build_s,
            "note": "plain: one single-column ls_matvec per sector and column; plain_multi_rhs: one "
                    f"{nrhs}-column ls_matvec per sector (the columns share each orbit search, as in the batch)"}


def _serve_compare(trace, budget: int, max_iter: int, tol: float, log):
    """One trace served with continuous batching and one request at a time,
    each with generated and with stored elements; energies compared."""
    from paper_2308_16712_amd import serve as sv

    # first use of the kernels and tables each path needs, untimed, so that
    # neither side pays it inside the comparison
    warm = [type(r)(r.rid, 0.0, r.sector) for r in trace[:4]]
    sv.serve(warm, budget, max_iter=max_iter, tol=tol)
    sv.serve_one_at_a_time(warm, max_iter=max_iter, tol=tol)
    served = sv.serve(trace, budget, max_iter=max_iter, tol=tol, log=log)
    alone = sv.serve_one_at_a_time(trace, max_iter=max_iter, tol=tol)
    served_st = sv.serve(trace, budget, max_iter=max_iter, tol=tol, log=log, store_elements=True)
    alone_st = sv.serve_one_at_a_time(trace, max_iter=max_iter, tol=tol, store_elements=True, hbm_budget=budget)
    s, b, ss, bs = served.summary(), alone.summary(), served_st.summary(), alone_st.summary()

    def de(x, y):
        return max(abs(a.e0 - c.e0) / max(1.0, abs(c.e0)) for a, c in zip(x.records, y.records)
                   if a.status == c.status == "ok")

    # one-at-a-time service time per request (build + solve, no queueing):
    # the rate a one-at-a-time server sustains
    service = (b["build_s"] + b["step_s"]) / max(1, b["completed"])
    return {"requests": len(trace), "dims": sorted({r.dim for r in served.records}),
            "served": s, "one_at_a_time": b,
            "speedup_throughput": s["throughput_rps"] / b["throughput_rps"],
            "p50_ratio": b["p50_ms"] / s["p50_ms"], "p99_ratio": b["p99_ms"] / s["p99_ms"],
            "max_rel_e0_diff_served_vs_alone": de(served, alone),
            "stored": {"served": ss, "one_at_a_time": bs,
                       "speedup_throughput": ss["throughput_rps"] / bs["throughput_rps"],
                       "p50_ratio": bs["p50_ms"] / ss["p50_ms"], "p99_ratio": bs["p99_ms"] / ss["p99_ms"],
                       "max_rel_e0_diff_vs_generated": de(served_st, alone)},
            "one_at_a_time_service_s_per_request": service,
            "one_at_a_time_capacity_rps": 1.0 / service if service > 0 else None}


def serving(count: int, rate: float, budget_gb: float, max_iter: int, tol: float, full_count: int):
    """Poisson streams of ground-state requests on fully symmetric sectors,
    served with continuous batching and one request at a time on the same
    trace: (1) `count` requests over the smaller sectors of the serving mix
    (rings N = 24, 26, 28 and the 4x6 J1-J2 torus); (2) `full_count`
    requests over the whole mix (rings N = 24..36, 4x6 and 6x6)."""
    from workloads import configs

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    budget = int(budget_gb * 2 ** 30)
    out = {"arrival_rate_per_s": rate, "tol": tol, "max_iter": max_iter, "hbm_budget_gb": budget_gb,
           "policy": "sjf (small solves fused first, then the shortest large one; builds overlapped with steps)"}
    small = configs.serving_trace(count=count, rate=rate, ring_sizes=(24, 26, 28), squares=((4, 6),))
    out["small_mix"] = _serve_compare(small, budget, max_iter, tol, log)
    # the same mix offered ten times faster: above one-at-a-time capacity, so
    # requests overlap and steps carry many solves
    fast = configs.serving_trace(count=count, rate=10 * rate, ring_sizes=(24, 26, 28), squares=((4, 6),))
    out["small_mix_saturated"] = _serve_compare(fast, budget, max_iter, tol, log)
    out["small_mix_saturated"]["arrival_rate_per_s"] = 10 * rate
    full = configs.serving_trace(count=full_count, rate=rate)
    out["full_mix"] = _serve_compare(full, budget, max_iter, tol, log)
    for key, r in (("small_mix", rate), ("small_mix_saturated", 10 * rate), ("full_mix", rate)):
        cap = out[key]["one_at_a_time_capacity_rps"]
        out[key]["offered_load"] = r / cap if cap else None
        out[key]["offered_load_note"] = (f"arrivals at {r:g}/s against a one-at-a-time capacity of "
                                         f"{cap:.2f}/s (load {r / cap:.2f}); latency includes queueing"
                                         if cap else "")
    return out


def lookups(basis, sector, n_states: int = 1 << 22, reps_timed: int = 3):
    """ls_state_info on seeded random states of the sector's weight (orbit
    minimum, character and norm of each) and ls_index_lookup of every
    representative (stateToIndex), timed on the launch stream."""
    import torch
    import paper_2308_16712_amd as ls

    n = sector.n_sites
    w = max(sector.weight, 0)
    g = torch.Generator(device="cuda")
    g.manual_seed(17)
    # a random weight-w state: the sites of the w smallest of n uniform draws
    pos = torch.rand(n_states, n, device="cuda", generator=g).argsort(dim=1)[:, :w]
    states = (torch.ones_like(pos) << pos).sum(dim=1)
    del pos
    reps, _ = basis.copy()
    stream = torch.cuda.current_stream()

    def timed(fn):
        best = 1e30
        for _ in range(reps_timed):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    ls.ls_state_info(basis, states)
    ms_si = timed(lambda: ls.ls_state_info(basis, states))
    idx = ls.ls_index_lookup(basis, reps)
    ok = bool(torch.equal(idx, torch.arange(basis.dim, device="cuda")))
    ms_lu = timed(lambda: ls.ls_index_lookup(basis, reps))
    return {"state_info": {"states": n_states, "ms": ms_si, "states_per_s": n_states / (ms_si * 1e-3),
                           "what": "orbit minimum, character of the element reaching it and norm, per state"},
            "index_lookup": {"keys": basis.dim, "ms": ms_lu, "keys_per_s": basis.dim / (ms_lu * 1e-3),
                             "every_representative_found_at_its_index": ok}}


def push_product(op, x, pull_ms: float, elements: int, steps: int):
    """The push (transposed, atomic-add) form of the same product on the same
    input: time per product on the launch stream, and its distance from the
    pull result."""
    import torch
    import paper_2308_16712_amd as ls

    y_pull = ls.ls_matvec(op, x)
    y = ls.ls_matvec_push(op, x)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        ls.ls_matvec_push(op, x, y)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    rel = float(torch.linalg.norm(y - y_pull) / torch.linalg.norm(y_pull))
    del y, y_pull
    return {"ms_per_product": ms, "elements_per_s": elements / (ms * 1e-3), "pull_over_push_time": ms / pull_ms,
            "rel_l2_vs_pull": rel, "form": "transposed: y_j += conj(H_ij) x_i with FP64 atomic adds"}


def lanczos_leg(steps: int = 100):
    """Heisenberg ring N=32 (Sz=0, k=0, R=+1, Z=+1; 4,707,969 states): a
    100-step Lanczos solve (full CGS2, tol 0), with generated and with stored
    elements; time per step and the share spent in the products; and the
    same solves with the second Gram-Schmidt pass only where needed."""
    import torch
    import paper_2308_16712_amd as ls
    from workloads import configs

    sec = configs.ring32_symmetric()
    b = ls.ls_basis_build(sec)
    out = {"workload": "Heisenberg ring N=32, Sz=0, k=0, R=+1, Z=+1 (128)", "dim": b.dim, "steps": steps}
    for form in ("generated", "stored"):
        op = ls.ls_operator_create(b, sec.terms)
        if form == "stored":
            op.store()
        x = torch.empty(b.dim, dtype=torch.float64, device="cuda").uniform_(-1, 1)
        y = torch.empty_like(x)
        ls.ls_matvec(op, x, y)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(10):
            ls.ls_matvec(op, x, y)
        e1.record(stream)
        torch.cuda.synchronize()
        product_ms = e0.elapsed_time(e1) / 10
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = op.lanczos(steps, tol=0.0, seed=1)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[form] = {"e0": r["e0"], "iters": r["iters"], "s": wall, "ms_per_step": wall * 1e3 / r["iters"],
                     "product_ms": product_ms, "product_share": product_ms * r["iters"] / (wall * 1e3)}
        print(f"[bench] lanczos ring32 {form}: {wall:.2f}s, e0={r['e0']:.12f}", file=sys.stderr, flush=True)
        # the same solve with the second Gram-Schmidt pass only where needed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = op.lanczos(steps, tol=0.0, seed=1, reorth="selective")
        torch.cuda.synchronize()
        wall_s = time.perf_counter() - t0
        out[form]["selective_reorth"] = {"e0": rs["e0"], "ms_per_step": wall_s * 1e3 / rs["iters"],
                                         "e0_diff_vs_full": abs(rs["e0"] - r["e0"])}
        print(f"[bench] lanczos ring32 {form} selective: {wall_s:.2f}s, e0={rs['e0']:.12f}", file=sys.stderr,
              flush=True)
        op.close()
        del x, y
    out["e0_identical"] = out["generated"]["e0"] == out["stored"]["e0"]
    b.close()
    torch.cuda.empty_cache()
    return out


def stored_product(basis, sector, x, y, fly_ms: float, elements: int, n_off: int, steps: int, workload: str):
    """The same product from stored elements (ls_operator_store): store time
    and size, product time on the launch stream, bit-identity with the
    on-the-fly result, and the HBM roofline of the stored product
    (algorithmic bytes: the stored form read once, one x_j gather per
    off-diagonal element, x_i and y_i per row)."""
    import torch
    import paper_2308_16712_amd as ls

    op = ls.ls_operator_create(basis, sector.terms)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nbytes = op.store()
    torch.cuda.synchronize()
    store_s = time.perf_counter() - t0
    y2 = torch.empty_like(y)
    ls.ls_matvec(op, x, y2)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        ls.ls_matvec(op, x, y2)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    fly = ls.ls_operator_create(basis, sector.terms)
    ls.ls_matvec(fly, x, y)
    torch.cuda.synchronize()
    same = bool(torch.equal(y, y2))
    op.check()
    op.close()
    fly.close()
    del y2
    torch.cuda.empty_cache()
    rows = basis.dim
    alg = nbytes + n_off * 8 + rows * 16
    # one 4-byte column per slot plus a 1-byte value code (at most 256
    # distinct values) or, failing that, the value itself
    coded = nbytes < n_off * 8
    layout = ("sliced ELLPACK, 64-row slices; per slot a uint32 column and "
              + ("a 1-byte code into a per-operator table of distinct values" if coded else "an FP64 value"))
    roof = {"bound": "hbm", "kernel": "k_spmv", "kernel_ms": ms, "achieved": alg / (ms * 1e-3) / 1e9,
            "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": alg / (ms * 1e-3) / PEAK_HBM,
            "algorithmic_bytes_per_launch": alg,
            "algorithmic_model": "stored form read once + 8 B x_j gather per off-diagonal element + "
                                 "x_i and y_i per row"}
    roof.update(counter_fields(counter_record("k_spmv", workload), ms, elements, alg))
    return {"bytes": nbytes, "store_s": store_s, "ms_per_product": ms, "elements_per_s": elements / (ms * 1e-3),
            "speedup_vs_on_the_fly": fly_ms / ms, "identical_to_on_the_fly": same, "roofline": roof,
            "layout": layout}


def chain_products(ns, steps: int = 3):
    """The paper's own workload: closed Heisenberg chains (J = 1, nearest
    neighbours), Sz = 0, fully symmetric sector of D_N x Z2 (Table 2's
    sectors), one product on the fly per step.  x is drawn on the device
    (its values do not change the work)."""
    import torch
    import paper_2308_16712_amd as ls
    from workloads import configs

    out = {}
    for n in ns:
        sec = configs.ring_symmetric(n, 0, 1, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = ls.ls_basis_build(sec)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        op = ls.ls_operator_create(b, sec.terms)
        elements = op.count_elements() + b.dim
        g = torch.Generator(device="cuda")
        g.manual_seed(n)
        x = torch.rand(b.dim, dtype=torch.float64, device="cuda", generator=g) * 2 - 1
        y = torch.empty_like(x)
        ls.ls_matvec(op, x, y)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            ls.ls_matvec(op, x, y)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[f"chain_N{n}"] = {"dim": b.dim, "elements_per_product": elements, "basis_build_s": build_s,
                              "ms_per_product": ms, "elements_per_s": elements / (ms * 1e-3)}
        print(f"[bench] chain N={n}: {ms:.1f} ms per product", file=sys.stderr, flush=True)
        del x, y
        op.close()
        b.close()
        torch.cuda.empty_cache()
    out["paper_context"] = ("40 spins: one product takes at least 40 s on 4 nodes of 2x64-core AMD Rome; "
                            "42 spins: 424 s per core of element generation on one 128-core node")
    return out


def table2_dims():
    """Closed-chain sector dimensions printed in the paper (Section 6, Table 2)."""
    out = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "table2_chain_dims.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            n, d = line.split()
            out[int(n)] = int(d)
    return out


def enumeration(count_ns, build_n):
    """Count-only enumeration (ls_sector_count) of the fully symmetric
    closed-chain sectors of Table 2, split into rank slices that print
    progress, and one stored basis build; candidates filtered per second."""
    from math import comb
    import torch
    import paper_2308_16712_amd as ls
    from workloads import configs

    want = table2_dims()
    out = {}
    for n in count_ns:
        sec = configs.ring_symmetric(n, 0, 1, 1)
        total = comb(n, n // 2)
        slices = max(1, min(64, total >> 40))
        got = 0
        t0 = time.perf_counter()
        for k in range(slices):
            m, _ = ls.ls_sector_count(sec, total * k // slices, total * (k + 1) // slices)
            got += m
            if slices > 1:
                print(f"[bench] N={n} slice {k + 1}/{slices} t={time.perf_counter() - t0:.1f}s", file=sys.stderr,
                      flush=True)
        dt = time.perf_counter() - t0
        out[f"count_N{n}"] = {"dim": got, "table2": want.get(n), "matches_table2": got == want.get(n),
                              "candidates": total, "s": dt, "candidates_per_s": total / dt}
        print(f"[bench] count N={n}: {got} in {dt:.2f}s", file=sys.stderr, flush=True)
    if build_n:
        sec = configs.ring_symmetric(build_n, 0, 1, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = ls.ls_basis_build(sec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"build_N{build_n}"] = {"dim": b.dim, "table2": want.get(build_n),
                                    "matches_table2": b.dim == want.get(build_n), "s": dt,
                                    "candidates_per_s": comb(build_n, build_n // 2) / dt,
                                    "reps_gb": b.dim * 8 / 1e9}
        b.close()
        torch.cuda.empty_cache()
    return out


# the sources of each profiled kernel: a counter record taken on other
# sources no longer describes it
KERNEL_SOURCES = {
    "k_matvec": ("matvec.hip", "matvec_impl.hpp", "dispatch.hpp", "orbit.hpp"),
    "k_spmv": ("stored.hip", "matvec_impl.hpp"),
}


def sources_sha256(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2308_16712_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def counter_record(kernel: str, name: str):
    """The committed rocprofv3 counter record of a kernel on a workload
    (HBM bytes per launch from FETCH_SIZE / WRITE_SIZE, VALU and LDS
    counters per launch), if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"counters_{kernel}_{name}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != sources_sha256(kernel):
        return None
    return rec


def counter_fields(rec, kernel_ms: float, elements: int, alg_bytes: float) -> dict:
    """Executed work of a launch from its counter record, over the live
    kernel time."""
    if rec is None:
        return {"traffic": None, "counters": "no record taken on the current kernel sources"}
    t = kernel_ms * 1e-3
    tb = rec["bytes_per_launch"]
    out = {"traffic": tb, "traffic_gbps": tb / t / 1e9, "traffic_frac_of_hbm_peak": tb / t / PEAK_HBM,
           "traffic_over_algorithmic": tb / alg_bytes}
    c = rec.get("counters_per_launch", {})
    if "SQ_INSTS_VALU" in c:
        out["valu_executed_frac"] = c["SQ_INSTS_VALU"] * 64 / t / PEAK_VALU
        out["valu_lane_instructions_per_element"] = c["SQ_INSTS_VALU"] * 64 / elements
    if "SQ_INSTS_LDS" in c and c["SQ_INSTS_LDS"] > 0 and "SQ_LDS_BANK_CONFLICT" in c:
        out["lds_bank_conflict_cycles_per_lds_instruction"] = c["SQ_LDS_BANK_CONFLICT"] / c["SQ_INSTS_LDS"]
    out["counter_record"] = rec.get("file")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="square6x6")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--batched-count", type=int, default=64)
    ap.add_argument("--batched-nrhs", type=int, default=4)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving comparison")
    ap.add_argument("--serve-count", type=int, default=120, help="requests of the small-sector trace")
    ap.add_argument("--serve-full-count", type=int, default=12, help="requests of the whole-mix trace")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-max-iter", type=int, default=150)
    ap.add_argument("--no-enumeration", action="store_true", help="skip the Table 2 enumeration leg")
    ap.add_argument("--no-stored", action="store_true", help="skip the stored-elements product")
    ap.add_argument("--no-push", action="store_true", help="skip the push (atomic) product")
    ap.add_argument("--no-lanczos", action="store_true", help="skip the 100-step Lanczos leg (ring N=32)")
    ap.add_argument("--no-small", action="store_true", help="skip the N=16 and N=32 ring products")
    ap.add_argument("--chains", default="40,42", help="paper-workload chain sizes to time (empty: none)")
    ap.add_argument("--enum-counts", default="40,42,44,46,48", help="chain sizes counted without storage")
    ap.add_argument("--enum-build", type=int, default=40, help="chain size built and stored (0: none)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="run only a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus must be 1 (the multi-GPU design is described "
              "but not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2308_16712_amd as ls
    from workloads import rng

    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 3}))
        return

    sector, desc = workload(args.workload)
    print(f"[bench] building basis {args.workload}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    basis = ls.ls_basis_build(sector)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    op = ls.ls_operator_create(basis, sector.terms)
    n_off, rows = op.count_elements(), basis.dim
    elements = n_off + rows
    if basis.dim <= 1 << 27:
        x = torch.from_numpy(rng.vector(sector.seed, basis.dim, complex_=op.is_complex)).cuda()
    else:   # paper-size sectors: drawn on the device (the values do not change the work)
        g = torch.Generator(device="cuda")
        g.manual_seed(sector.seed)
        x = torch.rand(basis.dim, dtype=torch.float64, device="cuda", generator=g) * 2 - 1
    y = torch.empty_like(x)
    print(f"[bench] dim={basis.dim} elements/step={elements} build={build_s:.3f}s", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        ls.ls_matvec(op, x, y)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        ls.ls_matvec(op, x, y)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    ms_per_step = wall * 1e3 / args.steps
    value = elements * args.steps / wall

    alg_bytes = rows * ALG_ROW_BYTES + n_off * ALG_ELEMENT_BYTES
    achieved = alg_bytes / (kernel_ms * 1e-3)
    roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": achieved / PEAK_HBM, "kernel": "k_matvec", "kernel_ms": kernel_ms,
            "algorithmic_bytes_per_launch": alg_bytes,
            "algorithmic_model": f"{ALG_ROW_BYTES} B per row (representative, x_i, y_i) + {ALG_ELEMENT_BYTES} B "
                                 "per off-diagonal element (x_j, matched key)"}
    roof.update(counter_fields(counter_record("k_matvec", args.workload), kernel_ms, elements, alg_bytes))
    # the exhaustive-search model, kept under its own name: one
    # compare-select per group image and 32-bit word for every element
    words = (sector.n_sites + 31) // 32
    dense_ops = float(n_off) * sector.group.size * words
    roof["dense_equivalent_ops_frac"] = dense_ops / (kernel_ms * 1e-3) / PEAK_VALU
    cp = copy_peak()
    roof["measured_copy_gbps"] = cp["gbps"]
    roof["frac_of_measured_copy"] = achieved / (cp["gbps"] * 1e9)
    out = {
        "metric": "H matrix elements/s", "value": value, "unit": "elements/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "dim": basis.dim, "elements_per_step": elements,
                   "group_order": sector.group.size, "nrhs": 1},
        "roofline": roof,
        "basis_build_s": build_s,
        "orbit_search": dict(zip(("kind", "compile_time_shape"), op.search_kind())),
        "copy_peak": cp,
    }
    op.check()
    out["state_info_and_lookup"] = lookups(basis, sector)
    if not args.no_push:
        print("[bench] push form", file=sys.stderr, flush=True)
        out["push"] = push_product(op, x, kernel_ms, elements, args.steps)
    if not args.no_stored:
        print("[bench] stored elements", file=sys.stderr, flush=True)
        out["stored"] = stored_product(basis, sector, x, y, kernel_ms, elements, n_off, args.steps, args.workload)
    del x, y, op, basis
    torch.cuda.empty_cache()
    if not args.no_small:
        print("[bench] ring16 and ring32 products", file=sys.stderr, flush=True)
        out["small_configs"] = small_configs(args.steps)
    if not args.no_batched:
        print("[bench] batched vs plain", file=sys.stderr, flush=True)
        out["batched"] = batched_vs_plain(args.batched_count, args.batched_nrhs)
        torch.cuda.empty_cache()
    if not args.no_lanczos:
        print("[bench] lanczos", file=sys.stderr, flush=True)
        out["lanczos"] = lanczos_leg()
    chain_ns = [int(v) for v in args.chains.split(",") if v]
    if chain_ns:
        print("[bench] paper-workload chains", file=sys.stderr, flush=True)
        out["paper_chains"] = chain_products(chain_ns)
    if not args.no_enumeration:
        print("[bench] enumeration", file=sys.stderr, flush=True)
        ns = [int(v) for v in args.enum_counts.split(",") if v]
        out["enumeration"] = enumeration(ns, args.enum_build)
    if not args.no_serving:
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serving"] = serving(args.serve_count, args.serve_rate, args.serve_budget_gb, args.serve_max_iter,
                                 1e-10, args.serve_full_count)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sector, args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
