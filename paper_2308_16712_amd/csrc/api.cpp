// The C ABI: argument checks, exception-to-status translation, handles.

#include <cstring>
#include <new>

#include "ls_internal.hpp"

namespace ls {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error() { return g_last_error.c_str(); }

void *dev_alloc(size_t bytes, hipStream_t stream) {
    void *p = nullptr;
    if (hipMallocAsync(&p, bytes > 0 ? bytes : 1, stream) != hipSuccess || p == nullptr)
        throw Error{LS_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    return p;
}

void dev_free(void *p, hipStream_t stream) {
    if (p) (void)hipFreeAsync(p, stream);
}

namespace {
thread_local std::vector<std::pair<StreamSet *, hipStream_t>> t_pending;   // marks of the current call
}

void StreamSet::add(hipStream_t st) {
    for (const auto &p : t_pending)
        if (p.first == this && p.second == st) return;
    t_pending.push_back({this, st});
}

void StreamSet::mark(hipStream_t st) {
    std::lock_guard<std::mutex> lk(mu);
    hipEvent_t ev = nullptr;
    for (const auto &m : marks)
        if (m.first == st) ev = m.second;
    if (!ev) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamSynchronize(st);   // no event: wait for the stream now
            return;
        }
        marks.push_back({st, ev});
    }
    if (hipEventRecord(ev, st) != hipSuccess) (void)hipStreamSynchronize(st);
}

void flush_marks() {
    std::vector<std::pair<StreamSet *, hipStream_t>> p;
    p.swap(t_pending);
    for (const auto &m : p) m.first->mark(m.second);
}

void StreamSet::drain() {
    std::vector<std::pair<StreamSet *, hipStream_t>> keep;
    for (const auto &p : t_pending) {
        if (p.first == this) mark(p.second);
        else keep.push_back(p);
    }
    t_pending.swap(keep);
    std::lock_guard<std::mutex> lk(mu);
    for (const auto &m : marks) {
        (void)hipEventSynchronize(m.second);
        (void)hipEventDestroy(m.second);
    }
    marks.clear();
}

void touch(const ls_operator *op, hipStream_t st) {
    op->used.add(st);
    op->basis->used.add(st);
}

}  // namespace ls

namespace {

// Runs an entry point's body: exceptions become statuses, and the handles'
// use marks noted during the call are recorded once its work is enqueued.
template <typename F>
ls_status guarded(F &&f) {
    struct Flush {
        ~Flush() { ls::flush_marks(); }
    } flush;
    try {
        return f();
    } catch (const ls::Error &e) {
        ls::set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        ls::set_error("host allocation failed");
        return LS_ENOMEM;
    } catch (const std::exception &e) {
        ls::set_error(e.what());
        return LS_EINTERNAL;
    }
}

void free_basis(ls_basis *b) {
    if (!b) return;
    b->used.drain();
    ls::dev_free(b->d_reps);
    ls::dev_free(b->d_stab);
    ls::dev_free(b->d_buckets);
    ls::dev_free(b->d_table);
    ls::dev_free(b->d_binom);
    ls::dev_free(b->d_cosets);
    ls::dev_free(b->d_chi);
    ls::dev_free(b->d_chi_one);
    ls::dev_free(b->d_pair_lut);
    ls::dev_free(b->d_stab_tab);
    delete b;
}

void free_operator(ls_operator *op) {
    if (!op) return;
    op->used.drain();
    ls::dev_free(op->d_terms);
    ls::dev_free(op->d_cflip);
    ls::dev_free(op->d_err);
    ls::dev_free(op->d_st_off);
    ls::dev_free(op->d_st_width);
    ls::dev_free(op->d_st_cols);
    ls::dev_free(op->d_st_vals);
    ls::dev_free(op->d_st_codes);
    ls::dev_free(op->d_st_vtab);
    ls::dev_free(op->d_st_diag);
    delete op;
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

const char *ls_last_error(void) { return ls::last_error(); }

const char *ls_version(void) { return "ls_ed 0.1 (gfx950)"; }

ls_status ls_basis_build(const ls_sector_desc *desc, void *stream, ls_basis **out) {
    ls_basis *b = nullptr;
    ls_status st = guarded([&] {
        LS_REQUIRE(desc != nullptr && out != nullptr, "desc and out must not be NULL");
        ls::GroupPlan plan = ls::compile_group(*desc);
        b = new ls_basis();
        b->plan = std::move(plan);
        b->weight = desc->hamming_weight;
        b->perm_copy.assign(desc->perm, desc->perm + static_cast<size_t>(desc->n_elements) * desc->n_sites);
        b->flip_copy.assign(desc->flip, desc->flip + desc->n_elements);
        LS_HIP_CHECK(hipGetDevice(&b->device));
        b->used.add(as_stream(stream));
        ls::build_basis(b, as_stream(stream));
        *out = b;
        return LS_OK;
    });
    if (st != LS_OK) free_basis(b);
    return st;
}

ls_status ls_sector_count(const ls_sector_desc *desc, uint64_t rank_begin, uint64_t rank_end, uint64_t *n_members,
                          uint64_t *n_candidates, void *stream) {
    ls_basis *b = nullptr;
    ls_status st = guarded([&] {
        LS_REQUIRE(desc != nullptr && n_members != nullptr, "desc and n_members must not be NULL");
        LS_REQUIRE(rank_begin <= rank_end, "rank_begin must not exceed rank_end");
        ls::GroupPlan plan = ls::compile_group(*desc);
        b = new ls_basis();
        b->plan = std::move(plan);
        b->weight = desc->hamming_weight;
        LS_HIP_CHECK(hipGetDevice(&b->device));
        b->used.add(as_stream(stream));
        ls::upload_plan(b, as_stream(stream));
        *n_members = ls::count_members(b, rank_begin, rank_end, as_stream(stream));
        if (n_candidates) *n_candidates = ls::candidate_count(b);
        return LS_OK;
    });
    free_basis(b);
    return st;
}

ls_status ls_sector_count_noalloc(const ls_sector_desc *desc, uint64_t rank_begin, uint64_t rank_end,
                                  uint64_t *n_members, uint64_t *n_candidates, void *stream) {
    return guarded([&] {
        LS_REQUIRE(desc != nullptr && n_members != nullptr, "desc and n_members must not be NULL");
        LS_REQUIRE(rank_begin <= rank_end, "rank_begin must not exceed rank_end");
        const ls::GroupPlan plan = ls::compile_group(*desc);
        uint64_t cand = 0;
        *n_members = ls::count_members_noalloc(plan, desc->hamming_weight, rank_begin, rank_end,
                                               as_stream(stream), &cand);
        if (n_candidates) *n_candidates = cand;
        return LS_OK;
    });
}

ls_status ls_sector_check(const ls_sector_desc *desc, uint32_t *lx, uint32_t *ly, uint32_t *pair_flip,
                          uint32_t *n_cosets) {
    return guarded([&] {
        LS_REQUIRE(desc != nullptr, "desc must not be NULL");
        const ls::GroupPlan plan = ls::compile_group(*desc);
        if (lx) *lx = plan.lx;
        if (ly) *ly = plan.ly;
        if (pair_flip) *pair_flip = plan.pair_flip;
        if (n_cosets) *n_cosets = static_cast<uint32_t>(plan.cosets.size());
        return LS_OK;
    });
}

ls_status ls_basis_info(const ls_basis *b, uint64_t *dim, int *is_real, const uint64_t **d_reps) {
    return guarded([&] {
        LS_REQUIRE(b != nullptr, "basis must not be NULL");
        if (dim) *dim = b->dim;
        if (is_real) *is_real = b->plan.chi_mode != ls::kChiComplex;
        if (d_reps) *d_reps = b->d_reps;
        return LS_OK;
    });
}

ls_status ls_basis_copy(const ls_basis *b, uint64_t *d_reps_out, uint16_t *d_stab_out, void *stream) {
    return guarded([&] {
        LS_REQUIRE(b != nullptr, "basis must not be NULL");
        if (b->dim == 0) return LS_OK;
        b->used.add(as_stream(stream));
        if (d_reps_out)
            LS_HIP_CHECK(hipMemcpyAsync(d_reps_out, b->d_reps, b->dim * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                                        as_stream(stream)));
        if (d_stab_out)
            LS_HIP_CHECK(hipMemcpyAsync(d_stab_out, b->d_stab, b->dim * sizeof(uint16_t), hipMemcpyDeviceToDevice,
                                        as_stream(stream)));
        return LS_OK;
    });
}

void ls_basis_destroy(ls_basis *b) { free_basis(b); }

ls_status ls_state_info(const ls_basis *b, uint64_t n, const uint64_t *d_states, uint64_t *d_reps, double *d_chi,
                        double *d_norm, void *stream) {
    return guarded([&] {
        LS_REQUIRE(b != nullptr, "basis must not be NULL");
        if (n == 0) return LS_OK;
        LS_REQUIRE(d_states && d_reps && d_chi && d_norm, "device pointers must not be NULL");
        b->used.add(as_stream(stream));
        ls::launch_state_info(b, n, d_states, d_reps, d_chi, d_norm, as_stream(stream));
        return LS_OK;
    });
}

ls_status ls_index_lookup(const ls_basis *b, uint64_t n, const uint64_t *d_keys, int64_t *d_index, void *stream) {
    return guarded([&] {
        LS_REQUIRE(b != nullptr, "basis must not be NULL");
        if (n == 0) return LS_OK;
        LS_REQUIRE(d_keys && d_index, "device pointers must not be NULL");
        b->used.add(as_stream(stream));
        ls::launch_index_lookup(b, n, d_keys, d_index, as_stream(stream));
        return LS_OK;
    });
}

ls_status ls_operator_create(const ls_basis *b, uint32_t n_terms, const ls_term *terms, ls_operator **out) {
    ls_operator *op = nullptr;
    ls_status st = guarded([&] {
        LS_REQUIRE(b != nullptr && out != nullptr, "basis and out must not be NULL");
        op = new ls_operator();
        op->basis = b;
        ls::compile_terms(b, n_terms, terms, op);
        // created without a stream: the default stream, waited for here
        hipStream_t st0 = nullptr;
        op->used.add(st0);
        const size_t bytes = std::max<size_t>(op->host_terms.size(), 1) * sizeof(ls_term_dev);
        op->d_terms = ls::dev_alloc_n<ls_term_dev>(std::max<size_t>(op->host_terms.size(), 1), st0);
        if (!op->host_terms.empty())
            LS_HIP_CHECK(hipMemcpyAsync(op->d_terms, op->host_terms.data(), bytes, hipMemcpyHostToDevice, st0));
        if (!op->host_cflip.empty()) {
            op->d_cflip = ls::dev_alloc_n<uint64_t>(op->host_cflip.size(), st0);
            LS_HIP_CHECK(hipMemcpyAsync(op->d_cflip, op->host_cflip.data(), op->host_cflip.size() * sizeof(uint64_t),
                                        hipMemcpyHostToDevice, st0));
        }
        op->d_err = ls::dev_alloc_n<uint32_t>(1, st0);
        const uint32_t zero = 0;
        LS_HIP_CHECK(hipMemcpyAsync(op->d_err, &zero, sizeof(uint32_t), hipMemcpyHostToDevice, st0));
        LS_HIP_CHECK(hipStreamSynchronize(st0));
        *out = op;
        return LS_OK;
    });
    if (st != LS_OK && op) free_operator(op);
    return st;
}

void ls_operator_destroy(ls_operator *op) { free_operator(op); }

ls_status ls_operator_store(ls_operator *op, uint64_t max_bytes, void *stream, uint64_t *bytes) {
    return guarded([&] {
        LS_REQUIRE(op != nullptr, "operator must not be NULL");
        ls::touch(op, as_stream(stream));
        const uint64_t b = ls::store_elements(op, max_bytes, as_stream(stream));
        if (bytes) *bytes = b;
        return LS_OK;
    });
}

ls_status ls_operator_info(const ls_operator *op, int *is_complex, uint64_t *dim) {
    return guarded([&] {
        LS_REQUIRE(op != nullptr, "operator must not be NULL");
        if (is_complex) *is_complex = op->is_complex ? 1 : 0;
        if (dim) *dim = op->basis->dim;
        return LS_OK;
    });
}

ls_status ls_operator_count(const ls_operator *op, uint64_t *n_offdiag, void *stream) {
    return guarded([&] {
        LS_REQUIRE(op != nullptr && n_offdiag != nullptr, "operator and output must not be NULL");
        ls::touch(op, as_stream(stream));
        *n_offdiag = ls::count_elements(op, as_stream(stream));
        return LS_OK;
    });
}

ls_status ls_operator_check(const ls_operator *op, void *stream) {
    return guarded([&] {
        LS_REQUIRE(op != nullptr, "operator must not be NULL");
        ls::touch(op, as_stream(stream));
        ls::check_operator(op, as_stream(stream));
        return LS_OK;
    });
}

ls_status ls_basis_test_drop_key(ls_basis *b, uint64_t index, void *stream) {
    return guarded([&] {
        LS_REQUIRE(b != nullptr, "basis must not be NULL");
        LS_REQUIRE(index < b->dim, "index must be below the dimension");
        b->used.add(as_stream(stream));
        ls::drop_key(b, index, as_stream(stream));
        return LS_OK;
    });
}

ls_status ls_operator_search_kind(const ls_operator *op, uint32_t *kind, uint32_t *fixed_shape) {
    return guarded([&] {
        LS_REQUIRE(op != nullptr, "operator must not be NULL");
        uint32_t k = 0, f = 0;
        ls::search_kind(op, &k, &f);
        if (kind) *kind = k;
        if (fixed_shape) *fixed_shape = f;
        return LS_OK;
    });
}

ls_status ls_matvec(const ls_operator *op, uint32_t nrhs, const void *d_x, void *d_y, void *stream) {
    return guarded([&] {
        LS_REQUIRE(op != nullptr, "operator must not be NULL");
        LS_REQUIRE(nrhs >= 1 && nrhs <= 64, "nrhs must be in 1..64");
        if (op->basis->dim == 0) return LS_OK;
        LS_REQUIRE(d_x != nullptr && d_y != nullptr, "x and y must not be NULL");
        const size_t bytes = op->basis->dim * nrhs * (op->is_complex ? 16u : 8u);
        const char *xb = static_cast<const char *>(d_x);
        const char *yb = static_cast<const char *>(d_y);
        LS_REQUIRE(xb + bytes <= yb || yb + bytes <= xb, "x and y must not overlap");
        ls::touch(op, as_stream(stream));
        ls::launch_matvec(op, nrhs, d_x, d_y, as_stream(stream));
        return LS_OK;
    });
}

ls_status ls_matvec_push(const ls_operator *op, uint32_t nrhs, const void *d_x, void *d_y, void *stream) {
    return guarded([&] {
        LS_REQUIRE(op != nullptr, "operator must not be NULL");
        LS_REQUIRE(nrhs >= 1 && nrhs <= 64, "nrhs must be in 1..64");
        if (op->basis->dim == 0) return LS_OK;
        LS_REQUIRE(d_x != nullptr && d_y != nullptr, "x and y must not be NULL");
        const size_t bytes = op->basis->dim * nrhs * (op->is_complex ? 16u : 8u);
        const char *xb = static_cast<const char *>(d_x);
        const char *yb = static_cast<const char *>(d_y);
        LS_REQUIRE(xb + bytes <= yb || yb + bytes <= xb, "x and y must not overlap");
        ls::touch(op, as_stream(stream));
        ls::launch_matvec_push(op, nrhs, d_x, d_y, as_stream(stream));
        return LS_OK;
    });
}

ls_status ls_batch_create(uint32_t n, const ls_operator *const *ops, const uint32_t *nrhs, ls_batch **out) {
    return guarded([&] {
        ls::batch_create(n, ops, nrhs, out);
        return LS_OK;
    });
}

ls_status ls_batch_matvec(ls_batch *batch, const void *const *d_x, void *const *d_y, void *stream) {
    return guarded([&] {
        LS_REQUIRE(batch != nullptr, "batch must not be NULL");
        ls::batch_matvec(batch, d_x, d_y, as_stream(stream));
        return LS_OK;
    });
}

ls_status ls_batch_info(const ls_batch *batch, uint32_t *n_launches, uint32_t *n_tiles, uint32_t *graph) {
    return guarded([&] {
        LS_REQUIRE(batch != nullptr, "batch must not be NULL");
        ls::batch_info(batch, n_launches, n_tiles, graph);
        return LS_OK;
    });
}

ls_status ls_batch_search(const ls_batch *batch, uint32_t item, uint32_t *mode, uint32_t *bits, double *own_ns,
                          double *chosen_ns, double *staged_ns) {
    return guarded([&] {
        LS_REQUIRE(batch != nullptr, "batch must not be NULL");
        ls::batch_search(batch, item, mode, bits, own_ns, chosen_ns, staged_ns);
        return LS_OK;
    });
}

ls_status ls_batch_set_search(ls_batch *batch, int mode, uint32_t bits) {
    return guarded([&] {
        LS_REQUIRE(batch != nullptr, "batch must not be NULL");
        ls::batch_set_search(batch, mode, bits);
        return LS_OK;
    });
}

ls_status ls_batch_set_graph(ls_batch *batch, int enabled) {
    return guarded([&] {
        LS_REQUIRE(batch != nullptr, "batch must not be NULL");
        ls::batch_set_graph(batch, enabled != 0);
        return LS_OK;
    });
}

void ls_batch_destroy(ls_batch *batch) {
    if (batch) ls::batch_destroy(batch);
}

ls_status ls_solver_footprint(const ls_operator *op, uint32_t max_iter, uint64_t *bytes) {
    return guarded([&] {
        LS_REQUIRE(op != nullptr && bytes != nullptr, "operator and output must not be NULL");
        *bytes = ls::solver_footprint(op, max_iter);
        return LS_OK;
    });
}

ls_status ls_solver_create(const ls_operator *op, const ls_lanczos_opts *opts, void *stream, ls_solver **out) {
    return guarded([&] {
        LS_REQUIRE(op != nullptr && opts != nullptr && out != nullptr, "operator, opts and out must not be NULL");
        LS_REQUIRE(opts->max_iter >= 1, "max_iter must be >= 1");
        LS_REQUIRE(opts->reorth <= 2, "reorth must be 0, 1 or 2");
        LS_REQUIRE(std::isfinite(opts->tol) && opts->tol >= 0, "tol must be >= 0");
        LS_REQUIRE(op->basis->dim > 0, "the basis is empty");
        ls::touch(op, as_stream(stream));
        *out = ls::solver_create(op, opts, as_stream(stream));
        return LS_OK;
    });
}

ls_status ls_solver_step(ls_solver *const *solvers, uint32_t n, void *stream) {
    return guarded([&] {
        LS_REQUIRE(n == 0 || solvers != nullptr, "solvers must not be NULL");
        ls::solver_step(solvers, n, 1, as_stream(stream));
        return LS_OK;
    });
}

ls_status ls_solver_step_n(ls_solver *const *solvers, uint32_t n, uint32_t steps, void *stream) {
    return guarded([&] {
        LS_REQUIRE(n == 0 || solvers != nullptr, "solvers must not be NULL");
        LS_REQUIRE(steps >= 1 && steps <= 1024, "steps must be in 1..1024");
        ls::solver_step(solvers, n, steps, as_stream(stream));
        return LS_OK;
    });
}

ls_status ls_solver_result(const ls_solver *solver, double *e0, uint32_t *iters, double *resid_bound, int *done,
                           int *converged) {
    return guarded([&] {
        LS_REQUIRE(solver != nullptr, "solver must not be NULL");
        ls::solver_result(solver, e0, iters, resid_bound, done, converged);
        if (ls::solver_failed(solver))
            throw ls::Error{LS_EINTERNAL, "the solve was stopped: its product met a neighbour whose "
                                          "representative lies in the sector but is missing from the basis"};
        return LS_OK;
    });
}

void ls_solver_destroy(ls_solver *solver) {
    if (solver) ls::solver_destroy(solver);
}

ls_status ls_lanczos(const ls_operator *op, const ls_lanczos_opts *opts, void *stream, double *e0, uint32_t *iters,
                     double *resid_bound) {
    return guarded([&] {
        LS_REQUIRE(op != nullptr && opts != nullptr, "operator and opts must not be NULL");
        LS_REQUIRE(opts->max_iter >= 1, "max_iter must be >= 1");
        LS_REQUIRE(opts->reorth <= 2, "reorth must be 0, 1 or 2");
        LS_REQUIRE(std::isfinite(opts->tol) && opts->tol >= 0, "tol must be >= 0");
        LS_REQUIRE(op->basis->dim > 0, "the basis is empty");
        ls::touch(op, as_stream(stream));
        return ls::run_lanczos(op, opts, as_stream(stream), e0, iters, resid_bound);
    });
}

}  // extern "C"
