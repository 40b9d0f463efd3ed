// y = H x on the fly, row by row (Section 5.3, first listing, "pull" form):
// one launch per product (or per column slice of a multi-RHS product).
// The device work is in matvec_impl.hpp; variant selection in dispatch.hpp.

#include <algorithm>

#include "dispatch.hpp"

namespace ls {

namespace {

// Waves per SIMD the register allocator must allow.  The real single-RHS
// torus search with a compile-time shape fits 64 VGPRs without spilling:
// 8 waves per SIMD, so two 1024-thread workgroups share a CU and twice the
// waves are in flight to cover the latency of the random gathers (measured
// 12% faster on the 6x6 product than the compiler's 71-register choice).
// The 33..63-site ring search with trivial characters (the paper's chains)
// fits as well for one or two columns.  Other variants would spill at 64
// registers (with non-trivial characters the stabilizer walk of a lookup
// miss is compiled into the element loop) and keep the launch bound.
constexpr int waves_per_simd(int kind, int chi, bool cplx, int nr, uint32_t lx) {
    return ((kind == kOrbitTorus && !cplx && nr == 1 && lx != 0) ||
            (kind == kOrbitRing64 && chi == kChiTrivial && nr <= 2))
               ? 8
               : 1;
}

// The first rows_per_wg threads of a workgroup take rows (lane = workgroup
// * rows_per_wg + thread, then strides of n_lanes); the others only help to
// stage the LDS tables.  A sector with fewer rows than the lanes that fill
// the GPU runs with fewer rows per workgroup, so that its rows spread over
// every CU instead of a few full workgroups.  A row's elements are summed by
// one lane in term order whatever the mapping, so the results do not depend
// on it.
template <typename W, int KIND, int CHI, bool CPLX, int NR, uint32_t LX, uint32_t LY, uint32_t NZ>
__global__ void __launch_bounds__(block_of(KIND)) __attribute__((amdgpu_waves_per_eu(waves_per_simd(KIND, CHI, CPLX, NR, LX))))
k_matvec(MatvecJob a, uint64_t n_lanes, uint32_t rows_per_lane, uint32_t rows_per_wg) {
    constexpr int BLOCK = block_of(KIND);
    extern __shared__ __align__(16) unsigned char smem[];
    const LdsTables L = lds_tables<KIND, LX, BLOCK>(a, smem);
    stage_tables<KIND, LX, BLOCK>(a, L);
    __syncthreads();
    if (threadIdx.x >= rows_per_wg) return;
    const uint64_t lane = static_cast<uint64_t>(blockIdx.x) * rows_per_wg + threadIdx.x;
    run_rows<W, KIND, CHI, CPLX, NR, LX, LY, NZ>(a, L, lane, n_lanes, rows_per_lane);
}

// Small sectors, single column: kGroupLanes lanes per row (run_rows_group),
// 256-thread workgroups; the tables are staged per workgroup as in k_matvec.
constexpr int kGroupBlock = 256;
template <typename W, int KIND, int CHI, bool CPLX, uint32_t LX, uint32_t LY, uint32_t NZ>
__global__ void __launch_bounds__(kGroupBlock) k_matvec_group(MatvecJob a, uint64_t n_groups) {
    extern __shared__ __align__(16) unsigned char smem[];
    const LdsTables L = lds_tables<KIND, LX, kGroupBlock>(a, smem);
    stage_tables<KIND, LX, kGroupBlock>(a, L);
    __syncthreads();
    const uint64_t group = (static_cast<uint64_t>(blockIdx.x) * kGroupBlock + threadIdx.x) / kGroupLanes;
    run_rows_group<W, KIND, CHI, CPLX, LX, LY, NZ>(a, L, group, n_groups);
}

// Push form (comparison variant): same launch shape as k_matvec.
template <typename W, int KIND, int CHI, bool CPLX, int NR, uint32_t LX, uint32_t LY, uint32_t NZ>
__global__ void __launch_bounds__(block_of(KIND))
    k_matvec_push(MatvecJob a, uint64_t n_lanes, uint32_t rows_per_lane, uint32_t rows_per_wg) {
    constexpr int BLOCK = block_of(KIND);
    extern __shared__ __align__(16) unsigned char smem[];
    const LdsTables L = lds_tables<KIND, LX, BLOCK>(a, smem);
    stage_tables<KIND, LX, BLOCK>(a, L);
    __syncthreads();
    if (threadIdx.x >= rows_per_wg) return;
    const uint64_t lane = static_cast<uint64_t>(blockIdx.x) * rows_per_wg + threadIdx.x;
    push_rows<W, KIND, CHI, CPLX, NR, LX, LY, NZ>(a, L, lane, n_lanes, rows_per_lane);
}

__global__ void k_clear_flag(uint32_t *f) { *f = 0u; }

// y = 0 for the push form (a fill kernel, so the sequence may be captured)
__global__ void __launch_bounds__(256) k_zero(double *y, uint64_t n) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) y[i] = 0.0;
}

// Single-column products of sectors below this many rows take the row-group
// form (several lanes per row).
constexpr uint64_t group_rows_below(int kind) { return kind == kOrbitTorus ? 256ull * 1024 : 65536ull; }

struct SingleLaunch {
    MatvecJob job;
    hipStream_t st;
    bool push = false;
    template <typename W, int KIND, int CHI, bool CPLX, int NR, uint32_t LX, uint32_t LY, uint32_t NZ>
    void run() {
        constexpr int BLOCK = block_of(KIND);
        constexpr uint64_t kCUs = 256;
        const uint64_t fill = kCUs * 4 * 8 * 64;   // 256 CUs x 4 SIMDs x 8 waves
        const uint32_t rpl =
            static_cast<uint32_t>(std::min<uint64_t>(16, std::max<uint64_t>(1, job.dim / fill)));
        // rows per workgroup: whole workgroups, unless the rows are too few
        // to give every CU one (then whole waves, spread over the CUs)
        uint64_t wg_rows = BLOCK;
        if (job.dim < kCUs * BLOCK) {
            const uint64_t per_cu = (job.dim + kCUs - 1) / kCUs;
            wg_rows = std::min<uint64_t>(BLOCK, std::max<uint64_t>(64, (per_cu + 63) / 64 * 64));
        }
        uint64_t lanes = (job.dim + rpl - 1) / rpl;
        lanes = (lanes + wg_rows - 1) / wg_rows * wg_rows;
        const dim3 grid(static_cast<uint32_t>(lanes / wg_rows));
        const uint32_t rows_per_wg = static_cast<uint32_t>(wg_rows);
        const size_t lds = lds_bytes(KIND, job.n_terms, job.n_terms - job.n_diag, job.plan.lx);
        // a single column of a sector with fewer rows than the GPU has lanes:
        // several lanes per row (run_rows_group), so that each lane's chain
        // of searches and lookups is short.  The ring searches are cheap next
        // to the exchanges, so rings take it only below 2^16 rows (4x6 torus,
        // 15,578 rows: 645 -> 200 us; 26-site ring, 101,340 rows: slower).
        if constexpr (NR == 1) {
            if (!push && job.ld == 1 && job.dim < group_rows_below(KIND)) {
                const uint64_t groups_per_wg = kGroupBlock / kGroupLanes;
                const uint64_t wgs = (job.dim + groups_per_wg - 1) / groups_per_wg;
                hipLaunchKernelGGL((k_matvec_group<W, KIND, CHI, CPLX, LX, LY, NZ>),
                                   dim3(static_cast<uint32_t>(wgs)), dim3(kGroupBlock), lds, st, job,
                                   wgs * groups_per_wg);
                return;
            }
        }
        if (push) {
            // the push form runs one column per launch
            if constexpr (NR == 1)
                hipLaunchKernelGGL((k_matvec_push<W, KIND, CHI, CPLX, 1, LX, LY, NZ>), grid, dim3(BLOCK), lds, st,
                                   job, lanes, rpl, rows_per_wg);
            else
                throw Error{LS_EINTERNAL, "push products run one column per launch"};
        } else
            hipLaunchKernelGGL((k_matvec<W, KIND, CHI, CPLX, NR, LX, LY, NZ>), grid, dim3(BLOCK), lds, st, job, lanes,
                               rpl, rows_per_wg);
    }
};

// Off-diagonal element applications: per row, the acting off-diagonal terms.
__global__ void __launch_bounds__(256) k_count_elements(const uint64_t *reps, uint64_t dim,
                                                        const ls_term_dev *terms, uint32_t n_diag, uint32_t n_terms,
                                                        unsigned long long *total) {
    __shared__ unsigned long long sh[256];
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x;
    unsigned long long c = 0;
    if (i < dim) {
        const uint64_t r = reps[i];
        for (uint32_t t = n_diag; t < n_terms; ++t) c += (r & terms[t].sel) == terms[t].val ? 1ull : 0ull;
    }
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(total, sh[0]);
}

}  // namespace

uint64_t count_elements(const ls_operator *op, hipStream_t st) {
    const ls_basis *b = op->basis;
    if (b->dim == 0) return 0;
    unsigned long long *d = dev_alloc_n<unsigned long long>(1, st);
    unsigned long long h = 0;
    hipError_t e = hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_count_elements, dim3(static_cast<uint32_t>((b->dim + 255) / 256)), dim3(256), 0, st,
                           b->d_reps, b->dim, op->d_terms, op->n_diag, op->n_diag + op->n_off, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dev_free(d, st);
    LS_HIP_CHECK(e);
    return h;
}

uint32_t matvec_max_terms() { return kMaxLdsTerms; }

void enqueue_flag_read(const ls_operator *op, uint32_t *dst, hipStream_t st) {
    LS_HIP_CHECK(hipMemcpyAsync(dst, op->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, st, op->d_err);
    LS_HIP_CHECK(hipGetLastError());
}

void check_operator(const ls_operator *op, hipStream_t st) {
    uint32_t flag = 0;
    enqueue_flag_read(op, &flag, st);
    LS_HIP_CHECK(hipStreamSynchronize(st));
    if (flag)
        throw Error{LS_EINTERNAL,
                    "a product met a neighbour whose representative lies in the sector but is missing from the "
                    "basis (inconsistent basis or search layout)"};
}

void search_kind(const ls_operator *op, uint32_t *kind, uint32_t *fixed_shape) {
    const Variant v = variant_of(op);
    *kind = static_cast<uint32_t>(v.kind);
    *fixed_shape = v.lx != 0 ? 1u : 0u;
}

MatvecJob job_of(const ls_operator *op, const void *x, void *y, uint32_t ld, uint32_t col) {
    const ls_basis *b = op->basis;
    MatvecJob a{};
    a.plan = b->plan_dev;
    a.search = b->search_dev;
    a.stab = b->d_stab;
    a.terms = op->d_terms;
    a.cflip = op->d_cflip;
    a.n_diag = op->n_diag;
    a.n_terms = op->n_diag + op->n_off;
    a.dim = b->dim;
    a.ld = ld;
    a.col = col;
    a.x = x;
    a.y = y;
    a.err = op->d_err;
    return a;
}

Variant variant_of(const ls_operator *op) {
    const GroupPlan &gp = op->basis->plan;
    Variant v{};
    v.word64 = gp.n_sites > 32 ? 1 : 0;
    v.cplx = op->is_complex;
    v.chi = op->is_complex ? kChiComplex : gp.chi_mode;
    const bool torus = gp.torus && op->d_cflip != nullptr &&
                       lds_bytes(kOrbitTorus, op->n_diag + op->n_off, op->n_off, gp.lx) + kPairTableBytes <= kMaxLds;
    if (!v.word64 && gp.ly == 1 && gp.lx == gp.n_sites) {
        v.kind = kOrbitRing32;
    } else if (v.word64 && gp.ly == 1 && gp.lx == gp.n_sites && gp.n_sites < 64) {
        v.kind = kOrbitRing64;
    } else if (torus) {
        v.kind = kOrbitTorus;
        const uint32_t nz = gp.pair_flip ? 2 : 1;
        // compile-time shapes: square tori with the full point group (eight
        // coset representatives) and spin inversion
        if (gp.cosets.size() == kTorusCosetSlots && nz == 2 &&
            ((gp.lx == 6 && gp.ly == 6) || (gp.lx == 4 && gp.ly == 4))) {
            v.lx = gp.lx;
            v.ly = gp.ly;
            v.nz = nz;
        }
    } else {
        v.kind = kOrbitGeneric;
    }
    return v;
}

int nr_chunk(uint32_t left) { return left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1; }

void launch_matvec(const ls_operator *op, uint32_t nrhs, const void *x, void *y, hipStream_t st) {
    if (op->basis->dim == 0) return;
    if (op->stored) {
        launch_stored(op, nrhs, x, y, st);
        return;
    }
    const Variant v = variant_of(op);
    uint32_t col = 0;
    while (col < nrhs) {
        const int nr = nr_chunk(nrhs - col);
        SingleLaunch L{job_of(op, x, y, nrhs, col), st};
        dispatch(v, nr, L);
        LS_HIP_CHECK(hipGetLastError());
        col += static_cast<uint32_t>(nr);
    }
}

bool grouped_product(const ls_operator *op) {
    return !op->stored && op->basis->dim > 0 && op->basis->dim < group_rows_below(variant_of(op).kind);
}

void launch_matvec_push(const ls_operator *op, uint32_t nrhs, const void *x, void *y, hipStream_t st) {
    const uint64_t dim = op->basis->dim;
    if (dim == 0) return;
    const uint64_t nd = dim * nrhs * (op->is_complex ? 2 : 1);
    hipLaunchKernelGGL(k_zero, dim3(static_cast<uint32_t>((nd + 255) / 256)), dim3(256), 0, st, static_cast<double *>(y),
                       nd);
    LS_HIP_CHECK(hipGetLastError());
    const Variant v = variant_of(op);
    for (uint32_t col = 0; col < nrhs; ++col) {
        SingleLaunch L{job_of(op, x, y, nrhs, col), st, true};
        dispatch(v, 1, L);
        LS_HIP_CHECK(hipGetLastError());
    }
}

}  // namespace ls
