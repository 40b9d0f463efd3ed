// Stored matrix elements: the products of an operator taken from memory
// instead of being regenerated.
//
// The paper generates elements on the fly because a stored Hamiltonian does
// not fit the memory of its machines (Section 2.2); one GPU with 288 GB of
// HBM holds the elements of sectors with up to a few billion of them (the
// 6x6 J1-J2 sector: 1.19e9 elements), and a product then reads them at HBM
// speed instead of redoing the orbit searches.
//
// Layout (sliced ELLPACK, slice = 64 consecutive rows = one wavefront): for
// slice g of width w_g (the most off-diagonal terms acting on one of its
// rows), element k of row i sits at off[g] + 64 k + (i mod 64), so the 64
// lanes of a wavefront read 64 consecutive slots.  Element k of a row is the
// row's k-th acting term in term order; a term whose neighbour is not in the
// basis, and padding, hold column kNoCol.  The diagonal sum of each row is
// stored separately.
//
// Values.  A real operator has few distinct element values (a coupling
// times a sign times sqrt(stab_j / stab_i), times a real character), so a
// slot holds a one-byte code into a table of at most 256 values (the table
// is filled during the store by an open-addressing set of the values' bit
// patterns, and staged in LDS by the product): 5 bytes per slot instead of
// 12.  When a sector has more than 256 distinct values, or the operator is
// complex, the slots hold the values themselves.
//
// The store runs the same row code as the on-the-fly product (diag_sum,
// neighbour_rep, lookup, element_value) and the stored product accumulates
// in the same order with the same operations on the same value bits, so
// both give the same results bit for bit.

#include <algorithm>
#include <vector>

#include "dispatch.hpp"

namespace ls {

namespace {

constexpr uint32_t kSlice = 64;
constexpr uint32_t kNoCol = 0xFFFFFFFFu;
constexpr uint32_t kCodes = 256;                       // values of the coded form
constexpr uint64_t kNoValue = 0xFFFFFFFFFFFFFFFFull;   // free entry (a NaN pattern no element takes)

// Width of every slice: the most acting off-diagonal terms over its rows.
__global__ void __launch_bounds__(256) k_slice_width(const uint64_t *reps, uint64_t dim, const ls_term_dev *terms,
                                                     uint32_t n_diag, uint32_t n_terms, uint32_t *width) {
    const uint64_t row = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x;
    uint32_t c = 0;
    if (row < dim) {
        const uint64_t r = reps[row];
        for (uint32_t t = n_diag; t < n_terms; ++t) c += (r & terms[t].sel) == terms[t].val ? 1u : 0u;
    }
    // a wavefront is one slice: maximum over its 64 lanes
    for (int o = 32; o > 0; o >>= 1) c = max(c, static_cast<uint32_t>(__shfl_xor(static_cast<int>(c), o, 64)));
    if ((row & (kSlice - 1)) == 0 && row < dim) width[row / kSlice] = c;
}

struct StoreArgs {
    MatvecJob job;
    const uint64_t *off;     // [slices]
    uint32_t *cols;          // [slots]
    void *vals;              // [slots] double or double2 (full values), or null
    uint8_t *codes;          // [slots] value codes (coded form), or null
    uint64_t *vtab;          // [kCodes] value bit patterns of the coded form
    uint32_t *overflow;      // set when the coded form needs more than kCodes values
    void *diag;              // [dim] double (dre) or double2 (dre, dim)
};

// Code of a value in the coded form's table: linear probing over the
// table from a hash of the value's bits; a free entry is claimed with a
// compare-and-swap (entries only ever go from free to a value, so a stale
// read of a free entry is settled by the swap's result).  All kCodes
// entries taken by other values: the overflow flag is raised.
__device__ __forceinline__ uint32_t value_code(double v, uint64_t *vtab, uint32_t *overflow) {
    const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(v));
    uint32_t h = static_cast<uint32_t>((bits * 0x9E3779B97F4A7C15ull) >> 56);
    for (uint32_t n = 0; n < kCodes; ++n) {
        const uint64_t k = __hip_atomic_load(&vtab[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == bits) return h;
        if (k == kNoValue) {
            const unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long *>(&vtab[h]),
                                                      static_cast<unsigned long long>(kNoValue),
                                                      static_cast<unsigned long long>(bits));
            if (prev == kNoValue || prev == bits) return h;
        }
        h = (h + 1) & (kCodes - 1);
    }
    atomicOr(overflow, 1u);
    return 0;
}

template <typename W, int KIND, int CHI, bool CPLX, uint32_t LX, uint32_t LY, uint32_t NZ>
__global__ void __launch_bounds__(block_of(KIND)) k_store(StoreArgs s) {
    constexpr int BLOCK = block_of(KIND);
    constexpr bool TRACK = CHI != kChiTrivial;
    using T = typename Val<CPLX>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const MatvecJob &a = s.job;
    const LdsTables L = lds_tables<KIND, LX, BLOCK>(a, smem);
    stage_tables<KIND, LX, BLOCK>(a, L);
    __syncthreads();
    const uint64_t row = static_cast<uint64_t>(blockIdx.x) * BLOCK + threadIdx.x;
    if (row >= a.dim) return;
    const uint64_t r = a.search.reps[row];
    const auto rs = row_stab<uses_ratio_table(KIND, false)>(a.plan, L, a.stab[row]);
    double dre, dim_;
    diag_sum<CPLX>(L.terms, a.n_diag, r, dre, dim_);
    if constexpr (CPLX) static_cast<double2 *>(s.diag)[row] = make_double2(dre, dim_);
    else static_cast<double *>(s.diag)[row] = dre;
    W pr[kTorusCosetSlots] = {};
    if constexpr (KIND == kOrbitTorus) row_images<W>(a.plan, r, pr);
    const uint64_t base = s.off[row / kSlice] + (row & (kSlice - 1));
    uint32_t k = 0;
    for (uint32_t t = a.n_diag; t < a.n_terms; ++t) {
        const ls_term_dev &Tm = L.terms[t];
        if ((r & Tm.sel) != Tm.val) continue;
        uint32_t code;
        const W rep = neighbour_rep<W, KIND, TRACK, LX, LY, NZ>(a, L, r, pr, t, code);
        uint32_t st_j = 0;
        const int64_t j = lookup_index_stab(a.search, static_cast<uint64_t>(rep), a.stab, st_j);
        const uint64_t slot = base + static_cast<uint64_t>(k) * kSlice;
        ++k;
        if (j < 0) {           // the slot keeps kNoCol
            lookup_miss<W, KIND, CHI>(a, rep);
            continue;
        }
        s.cols[slot] = static_cast<uint32_t>(j);
        const T v = element_value<CHI, CPLX>(Tm, r, stab_factor(a.plan, L, rs, st_j), a.plan, code);
        if constexpr (CPLX) {
            static_cast<T *>(s.vals)[slot] = v;
        } else {
            if (s.codes) s.codes[slot] = static_cast<uint8_t>(value_code(v, s.vtab, s.overflow));
            else static_cast<T *>(s.vals)[slot] = v;
        }
    }
}

struct StoreLaunch {
    StoreArgs args;
    hipStream_t st;
    template <typename W, int KIND, int CHI, bool CPLX, int NR, uint32_t LX, uint32_t LY, uint32_t NZ>
    void run() {
        if constexpr (NR != 1) {
            throw Error{LS_EINTERNAL, "the element store runs with one right-hand side"};
        } else {
            constexpr int BLOCK = block_of(KIND);
            const MatvecJob &j = args.job;
            const size_t lds = lds_bytes(KIND, j.n_terms, j.n_terms - j.n_diag, j.plan.lx);
            const uint64_t blocks = (j.dim + BLOCK - 1) / BLOCK;
            hipLaunchKernelGGL((k_store<W, KIND, CHI, CPLX, LX, LY, NZ>), dim3(static_cast<uint32_t>(blocks)),
                               dim3(BLOCK), lds, st, args);
        }
    }
};

// y = H x from the stored elements; one lane per row, NR columns.  CODED:
// values through the code table (staged in LDS), else read per slot.
template <bool CPLX, int NR, bool CODED>
__global__ void __launch_bounds__(256) k_spmv(const uint64_t *off, const uint32_t *width, const uint32_t *cols,
                                              const void *vals_, const uint8_t *codes, const uint64_t *vtab_g,
                                              const void *diag_, uint64_t dim, uint32_t ld, uint32_t col0,
                                              const void *x_, void *y_) {
    using T = typename Val<CPLX>::T;
    __shared__ double vtab[CODED ? kCodes : 1];
    if constexpr (CODED) {
        for (uint32_t q = threadIdx.x; q < kCodes; q += 256) vtab[q] = __longlong_as_double(static_cast<long long>(vtab_g[q]));
        __syncthreads();
    }
    const uint64_t row = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (row >= dim) return;
    const T *x = static_cast<const T *>(x_);
    const T *vals = static_cast<const T *>(vals_);
    T *y = static_cast<T *>(y_);
    double dre, dim_ = 0.0;
    if constexpr (CPLX) {
        const double2 d = static_cast<const double2 *>(diag_)[row];
        dre = d.x;
        dim_ = d.y;
    } else {
        dre = static_cast<const double *>(diag_)[row];
    }
    T acc[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] = diag_times<CPLX>(dre, dim_, x[row * ld + col0 + q]);
    const uint64_t g = row / kSlice;
    const uint32_t w = width[g];      // the same for the whole wavefront
    const uint64_t base = off[g] + (row & (kSlice - 1));
    auto value = [&](uint64_t slot) -> T {
        if constexpr (CODED) return vtab[__builtin_nontemporal_load(&codes[slot])];
        else return vals[slot];
    };
    // U elements per step: their columns, values and x gathers are all issued
    // before the first add, so U gathers per lane are in flight at once; the
    // adds keep the element order (same bits as the one-by-one loop).  The
    // stored form is read once, with non-temporal loads, so that it displaces
    // less of x from the caches.  (A masked last step in place of the
    // one-by-one tail measured 11.3 ms against 7.4 ms on the 6x6 sector.)
    constexpr int U = NR == 1 ? (CPLX ? 16 : 32) : NR == 2 ? 4 : 1;
    uint32_t k = 0;
    for (; k + U <= w; k += U) {
        uint32_t j[U];
        T v[U], xv[U][NR];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t slot = base + static_cast<uint64_t>(k + u) * kSlice;
            j[u] = __builtin_nontemporal_load(&cols[slot]);
            v[u] = value(slot);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j[u] != kNoCol) {
#pragma unroll
                for (int q = 0; q < NR; ++q) xv[u][q] = x[static_cast<uint64_t>(j[u]) * ld + col0 + q];
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j[u] != kNoCol) {
#pragma unroll
                for (int q = 0; q < NR; ++q) accumulate(acc[q], v[u], xv[u][q]);
            }
    }
    for (; k < w; ++k) {
        const uint64_t slot = base + static_cast<uint64_t>(k) * kSlice;
        const uint32_t j = __builtin_nontemporal_load(&cols[slot]);
        if (j == kNoCol) continue;
        const T v = value(slot);
#pragma unroll
        for (int q = 0; q < NR; ++q) accumulate(acc[q], v, x[static_cast<uint64_t>(j) * ld + col0 + q]);
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) y[row * ld + col0 + q] = acc[q];
}

template <bool CPLX, bool CODED>
void launch_spmv_nr(const ls_operator *op, int nr, uint32_t nrhs, uint32_t col, const void *x, void *y,
                    hipStream_t st) {
    const uint64_t dim = op->basis->dim;
    const dim3 grid(static_cast<uint32_t>((dim + 255) / 256));
#define LS_SPMV(NRV)                                                                                                \
    hipLaunchKernelGGL((k_spmv<CPLX, NRV, CODED>), grid, dim3(256), 0, st, op->d_st_off, op->d_st_width,          \
                       op->d_st_cols, op->d_st_vals, op->d_st_codes, op->d_st_vtab, op->d_st_diag, dim, nrhs, col, \
                       x, y)
    switch (nr) {
        case 8: LS_SPMV(8); break;
        case 4: LS_SPMV(4); break;
        case 2: LS_SPMV(2); break;
        default: LS_SPMV(1); break;
    }
#undef LS_SPMV
}

// Device buffers of a store attempt, released in stream order on the
// store's stream unless handed to the operator.
struct StoreBufs {
    hipStream_t st;
    uint32_t *width = nullptr, *cols = nullptr, *overflow = nullptr;
    uint64_t *off = nullptr, *vtab = nullptr;
    void *vals = nullptr, *diag = nullptr;
    uint8_t *codes = nullptr;
    explicit StoreBufs(hipStream_t s) : st(s) {}
    ~StoreBufs() {
        dev_free(width, st);
        dev_free(off, st);
        dev_free(cols, st);
        dev_free(vals, st);
        dev_free(codes, st);
        dev_free(vtab, st);
        dev_free(overflow, st);
        dev_free(diag, st);
    }
};

}  // namespace

uint64_t store_elements(ls_operator *op, uint64_t max_bytes, hipStream_t st) {
    if (op->stored) return op->st_bytes;
    const ls_basis *b = op->basis;
    const uint64_t dim = b->dim;
    const uint64_t slices = (dim + kSlice - 1) / kSlice;
    const size_t es = op->is_complex ? sizeof(double2) : sizeof(double);
    StoreBufs B(st);
    std::vector<uint32_t> width(slices, 0);
    std::vector<uint64_t> off(slices, 0);
    if (slices > 0) {
        B.width = dev_alloc_n<uint32_t>(slices, st);
        hipLaunchKernelGGL(k_slice_width, dim3(static_cast<uint32_t>((dim + 255) / 256)), dim3(256), 0, st, b->d_reps,
                           dim, op->d_terms, op->n_diag, op->n_diag + op->n_off, B.width);
        LS_HIP_CHECK(hipGetLastError());
        LS_HIP_CHECK(hipMemcpyAsync(width.data(), B.width, slices * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        LS_HIP_CHECK(hipStreamSynchronize(st));
    }
    uint64_t slots = 0;
    for (uint64_t g = 0; g < slices; ++g) {
        off[g] = slots;
        slots += static_cast<uint64_t>(width[g]) * kSlice;
    }
    const uint64_t fixed = slices * (sizeof(uint64_t) + sizeof(uint32_t)) + dim * es;
    const uint64_t full_bytes = slots * (sizeof(uint32_t) + es) + fixed;
    const uint64_t coded_bytes = slots * (sizeof(uint32_t) + 1) + kCodes * sizeof(uint64_t) + fixed;
    bool coded = !op->is_complex;
    uint64_t bytes = coded ? coded_bytes : full_bytes;
    if (bytes > max_bytes) throw Error{LS_ENOMEM, "the stored elements would exceed max_bytes"};
    auto alloc = [&](void **p, uint64_t n) { *p = dev_alloc(n, st); };
    alloc(reinterpret_cast<void **>(&B.off), slices * sizeof(uint64_t));
    alloc(reinterpret_cast<void **>(&B.cols), slots * sizeof(uint32_t));
    alloc(&B.diag, dim * es);
    if (slices > 0)
        LS_HIP_CHECK(hipMemcpyAsync(B.off, off.data(), slices * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    // one pass in the coded form; a second in the full form when the values
    // do not fit the code table
    for (int attempt = 0; attempt < 2; ++attempt) {
        if (coded) {
            alloc(reinterpret_cast<void **>(&B.codes), slots);
            alloc(reinterpret_cast<void **>(&B.vtab), kCodes * sizeof(uint64_t));
            alloc(reinterpret_cast<void **>(&B.overflow), sizeof(uint32_t));
            LS_HIP_CHECK(hipMemsetAsync(B.vtab, 0xFF, kCodes * sizeof(uint64_t), st));
            LS_HIP_CHECK(hipMemsetAsync(B.overflow, 0, sizeof(uint32_t), st));
        } else {
            alloc(&B.vals, slots * es);
        }
        if (slots > 0) LS_HIP_CHECK(hipMemsetAsync(B.cols, 0xFF, slots * sizeof(uint32_t), st));
        if (dim > 0) {
            StoreLaunch L{StoreArgs{job_of(op, nullptr, nullptr, 1, 0), B.off, B.cols, B.vals, B.codes, B.vtab,
                                    B.overflow, B.diag},
                          st};
            dispatch(variant_of(op), 1, L);
            LS_HIP_CHECK(hipGetLastError());
        }
        // a lookup miss of an in-sector representative fails the store
        check_operator(op, st);
        if (!coded) break;
        uint32_t over = 0;
        LS_HIP_CHECK(hipMemcpyAsync(&over, B.overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        LS_HIP_CHECK(hipStreamSynchronize(st));
        if (!over) break;
        dev_free(B.codes, st);
        dev_free(B.vtab, st);
        dev_free(B.overflow, st);
        B.codes = nullptr;
        B.vtab = nullptr;
        B.overflow = nullptr;
        coded = false;
        bytes = full_bytes;
        if (bytes > max_bytes) throw Error{LS_ENOMEM, "the stored elements would exceed max_bytes"};
    }
    op->d_st_width = B.width;
    op->d_st_off = B.off;
    op->d_st_cols = B.cols;
    op->d_st_vals = B.vals;
    op->d_st_codes = B.codes;
    op->d_st_vtab = B.vtab;
    op->d_st_diag = B.diag;
    B.width = B.cols = nullptr;
    B.off = B.vtab = nullptr;
    B.vals = B.diag = nullptr;
    B.codes = nullptr;
    op->st_slots = slots;
    op->st_bytes = bytes;
    op->stored = true;
    return bytes;
}

void launch_stored(const ls_operator *op, uint32_t nrhs, const void *x, void *y, hipStream_t st) {
    if (op->basis->dim == 0) return;
    uint32_t col = 0;
    while (col < nrhs) {
        const int nr = nr_chunk(nrhs - col);
        if (op->is_complex) launch_spmv_nr<true, false>(op, nr, nrhs, col, x, y, st);
        else if (op->d_st_codes) launch_spmv_nr<false, true>(op, nr, nrhs, col, x, y, st);
        else launch_spmv_nr<false, false>(op, nr, nrhs, col, x, y, st);
        LS_HIP_CHECK(hipGetLastError());
        col += static_cast<uint32_t>(nr);
    }
}

}  // namespace ls
