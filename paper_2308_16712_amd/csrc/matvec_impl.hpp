// Device implementation of the on-the-fly product, shared by the single
// launch (matvec.hip) and the persistent batched launch (batch.hip).
//
// Row i of the sector Hamiltonian is generated from its representative r:
//   acc = (sum of diagonal terms acting on r) * x_i
//   for each off-diagonal term t acting on r (r & sel == val):
//       s    = r ^ flip_t,  a = conj(c_t) (-1)^popcount(r & sign_t)
//       rep  = orbit minimum of s, g* an element reaching it   (getRow)
//       j    = stateToIndex(rep), with stab_j                   (lookup)
//       acc += a * chi(g*) * sqrt(stab_j / stab_i) * x_j
//   y_i = acc                                     (one store, no atomics)
// This is <r~_i|H|r~_j> written with P|s> = conj(chi(g*)) P|rep> and the
// Hermiticity of H; a neighbour whose orbit the projector annihilates is
// absent from the basis and contributes nothing.  Any other miss means the
// basis or its search layout is inconsistent (stateToIndex of Section 5.3
// presumes the state is present): it raises the operator's error flag,
// which the host reports as LS_EINTERNAL.
//
// Work layout.  Each off-diagonal term acts on only part of the rows (a
// Heisenberg exchange term on about a quarter of them), so a loop over the
// terms that is uniform across a wavefront would run the orbit search for
// every term with most lanes idle.  Instead every lane walks its own list:
// one loop iteration = one element (the lane's next acting term of its
// current row); when a lane's row is exhausted it stores y_i and moves to
// its next row.  A lane owns several rows strided by a fixed step, so
// per-row differences in the number of acting terms average out.  The term
// table is staged in LDS once per workgroup (per item in a batch).
//
// Tori (pruned search): permutations act linearly on bits, so for a coset
// representative p, p(r ^ f) = p(r) ^ pi_p(f).  A lane computes p(r) once per
// row and each neighbour's images with one XOR per coset, reading pi_p(f)
// from a per-operator table staged in LDS.  Workgroups of 1024 threads share
// the LDS tables among 16 wavefronts.
//
// Right-hand sides: x and y are [dim][ld] row-major; a job handles NR
// consecutive columns starting at `col`, so the orbit search is shared by
// NR vectors.
#pragma once

#include "orbit.hpp"

namespace ls {

constexpr int kMaxLdsTerms = 1024;
constexpr size_t kMaxLds = 64 * 1024;

// One product (or a column slice of one): everything a workgroup needs.
struct MatvecJob {
    PlanDev plan;
    SearchDev search;
    const uint16_t *stab;
    const ls_term_dev *terms;
    const uint64_t *cflip;  // [n_off][kTorusCosetSlots] (torus search only)
    uint32_t n_diag, n_terms;
    uint64_t dim;
    uint32_t ld;           // row stride of x and y in elements
    uint32_t col;          // first column handled
    const void *x;
    void *y;
    uint32_t *err;         // operator's error flag (lookup miss of an in-sector orbit)
};

__device__ __forceinline__ double sign_of(uint64_t v) {
    return (__builtin_popcountll(v) & 1) ? -1.0 : 1.0;
}

template <bool CPLX>
struct Val;
template <>
struct Val<false> {
    using T = double;
};
template <>
struct Val<true> {
    using T = double2;
};

// Shared arithmetic of a row: the on-the-fly product, the element store and
// the stored product all go through these, so they round identically.

// acc = diagonal sum (dre + i dim) times x_i
template <bool CPLX>
__device__ __forceinline__ typename Val<CPLX>::T diag_times(double dre, double dim_, typename Val<CPLX>::T v) {
    if constexpr (CPLX) return make_double2(dre * v.x - dim_ * v.y, dre * v.y + dim_ * v.x);
    else return dre * v;
}

// Element value conj(c_t) (-1)^popcount(r & sign_t) chi(g*) sqrt(stab_j / stab_i)
// (the term table already holds conj(c_t)); fs = sqrt(stab_j / stab_i).
template <int CHI, bool CPLX>
__device__ __forceinline__ typename Val<CPLX>::T element_value(const ls_term_dev &Tm, uint64_t r, double fs,
                                                               const PlanDev &P, uint32_t code) {
    const double f = sign_of(r & Tm.sign) * fs;
    if constexpr (!CPLX) {
        double coef = f * Tm.re;
        if constexpr (CHI == kChiReal) coef *= P.chi[code].x;
        return coef;
    } else {
        double cre = f * Tm.re, cim = f * Tm.im;
        if constexpr (CHI != kChiTrivial) {
            const double2 c = P.chi[code];
            const double tre = cre * c.x - cim * c.y;
            cim = cre * c.y + cim * c.x;
            cre = tre;
        }
        return make_double2(cre, cim);
    }
}

// acc += value * x_j
__device__ __forceinline__ void accumulate(double &acc, double c, double v) { acc = fma(c, v, acc); }
__device__ __forceinline__ void accumulate(double2 &acc, double2 c, double2 v) {
    acc.x = fma(c.x, v.x, fma(-c.y, v.y, acc.x));
    acc.y = fma(c.x, v.y, fma(c.y, v.x, acc.y));
}

constexpr int block_of(int kind) { return kind == kOrbitTorus ? 1024 : 256; }

__host__ __device__ constexpr size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

// LDS: the torus search's pair table is a static array (its address is then
// a compile-time constant that folds into the lookups); the dynamic part is
// col_ge | flip images (torus only) | terms.
constexpr uint32_t kPairTableEntries = 1u << 12;   // 4^lx for lx <= 6

// Dynamic LDS bytes of a launch (a staged bucket table goes after them).
__host__ __device__ inline size_t lds_bytes(int kind, uint32_t n_terms, uint32_t n_off, uint32_t lx) {
    (void)lx;
    size_t b = align16((n_terms > 0 ? n_terms : 1) * sizeof(ls_term_dev));
    if (kind == kOrbitTorus) b += 64 + static_cast<size_t>(n_off) * kTorusCosetSlots * sizeof(uint64_t);
    return b;
}

// Static LDS of the torus kernels.
constexpr size_t kPairTableBytes = kPairTableEntries * sizeof(uint32_t);

// Kernels that read the element normalisation from the stabilizer-ratio
// table (5.6 KB of static LDS): the single launches of the ring and generic
// searches, whose LDS is otherwise idle (N=32 ring product 2.04 -> 1.92 ms).
// The others divide and take the square root per element: in the torus
// kernels the table gains 0.5% (6x6 product) for LDS a staged bucket table
// could use, and it costs the persistent batched launch an occupancy step
// (complex ring columns 94 -> 99 VGPRs, 5 -> 4 waves per SIMD).
constexpr bool uses_ratio_table(int kind, bool batched) { return kind != kOrbitTorus && !batched; }

struct LdsTables {
    ls_term_dev *terms;
    uint32_t *lut;
    uint64_t *col;
    uint64_t *cflip;   // [slot][n_off]
    uint32_t *bkt;     // staged bucket table (kLookupStaged)
    uint8_t *scls;     // class of every stabilizer size
    double *sratio;    // sqrt(d_b / d_a) by classes
};

template <int KIND, uint32_t LX, int BLOCK, bool TAB = uses_ratio_table(KIND, false)>
__device__ __forceinline__ LdsTables lds_tables(const MatvecJob &a, unsigned char *smem) {
    LdsTables L;
    if constexpr (TAB) {
        __shared__ __align__(8) double stab_ratio[kStabClsMax * kStabClsMax];
        __shared__ __align__(8) uint8_t stab_cls[kStabMapBytes];
        L.scls = stab_cls;
        L.sratio = stab_ratio;
    } else {
        L.scls = nullptr;
        L.sratio = nullptr;
    }
    if constexpr (KIND == kOrbitTorus) {
        __shared__ uint32_t pair_table[kPairTableEntries];
        L.lut = pair_table;
        L.col = reinterpret_cast<uint64_t *>(smem);
        L.cflip = L.col + 8;
        L.terms = reinterpret_cast<ls_term_dev *>(
            smem + 64 + static_cast<size_t>(a.n_terms - a.n_diag) * kTorusCosetSlots * sizeof(uint64_t));
    } else {
        L.lut = nullptr;
        L.col = nullptr;
        L.cflip = nullptr;
        L.terms = reinterpret_cast<ls_term_dev *>(smem);
    }
    L.bkt = reinterpret_cast<uint32_t *>(smem + lds_bytes(KIND, a.n_terms, a.n_terms - a.n_diag, LX));
    return L;
}

// All threads of the workgroup stage the job's tables; caller syncs.
template <int KIND, uint32_t LX, int BLOCK, bool TAB = uses_ratio_table(KIND, false)>
__device__ __forceinline__ void stage_tables(const MatvecJob &a, const LdsTables &L) {
    for (uint32_t t = threadIdx.x; t < a.n_terms; t += BLOCK) L.terms[t] = a.terms[t];
    if constexpr (KIND == kOrbitTorus) {
        const uint32_t n_off = a.n_terms - a.n_diag;
        const uint32_t lut_n = 1u << (2 * (LX ? LX : a.plan.lx));
        for (uint32_t q = threadIdx.x; q < lut_n; q += BLOCK) L.lut[q] = a.plan.pair_lut[q];
        if (threadIdx.x < 8) L.col[threadIdx.x] = a.plan.col_ge[threadIdx.x];
        for (uint32_t q = threadIdx.x; q < n_off * kTorusCosetSlots; q += BLOCK) {
            const uint32_t k = q / kTorusCosetSlots, p = q % kTorusCosetSlots;
            L.cflip[p * n_off + k] = a.cflip[q];   // transposed: lanes spread over banks
        }
    }
    if (a.search.mode == kLookupStaged)
        for (uint32_t q = threadIdx.x; q < a.search.n_bkt; q += BLOCK) L.bkt[q] = a.search.buckets[q];
    if (TAB && a.plan.n_stab_cls) {
        const uint32_t *cw = reinterpret_cast<const uint32_t *>(a.plan.stab_cls);
        uint32_t *lw = reinterpret_cast<uint32_t *>(L.scls);
        for (uint32_t q = threadIdx.x; q < kStabMapBytes / 4; q += BLOCK) lw[q] = cw[q];
        for (uint32_t q = threadIdx.x; q < a.plan.n_stab_cls * a.plan.n_stab_cls; q += BLOCK)
            L.sratio[q] = a.plan.stab_ratio[q];
    }
}

// The row's part of the element normalisation: its stabilizer size, and the
// offset of its class's row of the ratio table (kernels without the table:
// the size).
template <bool TAB>
struct RowStab {
    uint32_t st;
    uint32_t base;
};
template <>
struct RowStab<false> {
    double st;
};

template <bool TAB>
__device__ __forceinline__ RowStab<TAB> row_stab(const PlanDev &P, const LdsTables &L, uint32_t st) {
    if constexpr (!TAB) {
        return RowStab<TAB>{static_cast<double>(st)};
    } else {
        return RowStab<TAB>{st, P.n_stab_cls ? static_cast<uint32_t>(L.scls[st]) * P.n_stab_cls : 0u};
    }
}

// sqrt(stab_j / stab_i), correctly rounded: read from the ratio table when
// the kernel and the group have one, else divided and rooted (the same bits).
template <bool TAB>
__device__ __forceinline__ double stab_factor(const PlanDev &P, const LdsTables &L, const RowStab<TAB> &R,
                                              uint32_t st_j) {
    if constexpr (!TAB) {
        return __dsqrt_rn(__ddiv_rn(static_cast<double>(st_j), R.st));
    } else {
        if (P.n_stab_cls) return L.sratio[R.base + L.scls[st_j]];
        return __dsqrt_rn(__ddiv_rn(static_cast<double>(st_j), static_cast<double>(R.st)));
    }
}

// Sum of the diagonal terms acting on r: dre + i dim_.
template <bool CPLX>
__device__ __forceinline__ void diag_sum(const ls_term_dev *sterm, uint32_t n_diag, uint64_t r, double &dre,
                                         double &dim_) {
    dre = 0.0;
    dim_ = 0.0;
    for (uint32_t q = 0; q < n_diag; ++q) {
        const ls_term_dev &D = sterm[q];
        if ((r & D.sel) != D.val) continue;
        const double sg = sign_of(r & D.sign);
        dre += sg * D.re;
        if constexpr (CPLX) dim_ += sg * D.im;
    }
}

// Torus search: p(r) for every coset representative p of the row.
template <typename W>
__device__ __forceinline__ void row_images(const PlanDev &P, uint64_t r, W *pr) {
#pragma unroll
    for (uint32_t p = 0; p < kTorusCosetSlots; ++p)
        if (p < P.n_cosets) pr[p] = apply_coset<W>(P.cosets[p], static_cast<W>(r), P);
}

// Orbit minimum of the neighbour r ^ flip_t of off-diagonal term t, and the
// code of an element reaching it (tori: from the row's coset images).
template <typename W, int KIND, bool TRACK, uint32_t LX, uint32_t LY, uint32_t NZ>
__device__ __forceinline__ W neighbour_rep(const MatvecJob &a, const LdsTables &L, uint64_t r, const W *pr,
                                           uint32_t t, uint32_t &code) {
    if constexpr (KIND == kOrbitTorus) {
        const uint32_t n_off = a.n_terms - a.n_diag;
        const uint32_t ko = t - a.n_diag;
        return torus_orbit_min<W, TRACK, LX, LY, NZ>(a.plan, pr, L.cflip + ko, n_off, L.lut, L.col, code);
    } else {
        (void)pr;
        return orbit_min<W, KIND, TRACK>(a.plan, static_cast<W>(r ^ L.terms[t].flip), code);
    }
}

// A neighbour's representative rep was not found by stateToIndex.  That is
// correct when the projector annihilates its orbit, i.e. some element that
// fixes rep has a character other than 1 -- never with trivial characters,
// where every orbit lies in the sector.  Otherwise the error flag is raised.
// The stabilizer walk runs on misses only.
template <typename W, int KIND, int CHI>
__device__ __forceinline__ void lookup_miss(const MatvecJob &a, W rep) {
    if constexpr (CHI != kChiTrivial) {
        constexpr int WALK = KIND == kOrbitRing32 ? kOrbitRing32 : kOrbitGeneric;
        bool annihilated = false;
        for_each_image<W, WALK>(a.plan, rep, [&](W v, uint32_t code) {
            if (v == rep && !chi_is_one(a.plan, code)) {
                annihilated = true;
                return false;
            }
            return true;
        });
        if (annihilated) return;
    }
    atomicOr(a.err, 1u);
}

// stateToIndex of a neighbour with its stabilizer size, in the job's layout.
template <bool STAGED>
__device__ __forceinline__ int64_t lookup_stab(const MatvecJob &a, const LdsTables &L, uint64_t key, uint32_t &st) {
    if constexpr (STAGED) {
        if (a.search.mode == kLookupStaged) {
            const int64_t j = lookup_staged(a.search, L.bkt, key);
            if (j >= 0) st = a.stab[j];
            return j;
        }
    }
    return lookup_index_stab(a.search, key, a.stab, st);
}

// Rows as run_rows, for the searches that are cheap next to the memory
// latency of the lookup (rings and the generic walk): the element loop is
// software-pipelined one element deep.  An iteration searches element e+1 and
// issues the load of its home hash slot, then finishes element e, whose slot
// load was issued one search earlier.  Elements are still accumulated one by
// one in term order, so the sums (and their bits) are those of run_rows.
template <typename W, int KIND, int CHI, bool CPLX, int NR, uint32_t LX, uint32_t LY, uint32_t NZ, bool STAGED>
__device__ __forceinline__ void run_rows_ahead(const MatvecJob &a, const LdsTables &L, uint64_t row0,
                                               uint64_t step, uint32_t count) {
    constexpr bool TRACK = CHI != kChiTrivial;
    using T = typename Val<CPLX>::T;
    const T *x = static_cast<const T *>(a.x);
    T *y = static_cast<T *>(a.y);
    const ls_term_dev *sterm = L.terms;
    const SearchDev &S = a.search;
    const bool hash = S.mode == kLookupHash;

    uint64_t row = row0;
    uint32_t k = 0;
    if (count == 0 || row >= a.dim) return;

    uint64_t r = 0;
    RowStab<uses_ratio_table(KIND, STAGED)> rs{};
    T acc[NR];
    uint32_t t = a.n_diag;
    W pr[kTorusCosetSlots] = {};   // unused by these searches

    auto begin_row = [&]() {
        r = a.search.reps[row];
        rs = row_stab<uses_ratio_table(KIND, STAGED)>(a.plan, L, a.stab[row]);
        double dre, dim_;
        diag_sum<CPLX>(sterm, a.n_diag, r, dre, dim_);
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[q] = diag_times<CPLX>(dre, dim_, x[row * a.ld + a.col + q]);
        t = a.n_diag;
    };
    begin_row();

    // the element whose home-slot load is in flight
    bool pend = false;
    uint64_t p_rep = 0, p_slot = 0;
    uint32_t p_code = 0, p_t = 0;
    uint4 p_e = make_uint4(0u, 0u, 0u, 0u);

    for (;;) {
        while (t < a.n_terms && (r & sterm[t].sel) != sterm[t].val) ++t;
        const bool more = t < a.n_terms;
        // stage 1: search the next element, issue its home-slot load
        uint64_t n_rep = 0, n_slot = 0;
        uint32_t n_code = 0;
        uint4 n_e = make_uint4(0u, 0u, 0u, 0u);
        bool n_live = false;
        if (more) {
            n_rep = static_cast<uint64_t>(neighbour_rep<W, KIND, TRACK, LX, LY, NZ>(a, L, r, pr, t, n_code));
            if (hash) {
                n_live = n_rep >= S.kmin && n_rep <= S.kmax;   // outside: not in the basis
                if (n_live) {
                    n_slot = slot_of(n_rep, S.hash_shift);
                    n_e = *reinterpret_cast<const uint4 *>(S.table + n_slot);
                } else {
                    lookup_miss<W, KIND, CHI>(a, static_cast<W>(n_rep));
                }
            } else {
                n_live = true;
            }
        }
        // stage 2: finish the pending element of this row
        if (pend) {
            int64_t j;
            uint32_t st_j = 0;
            if (hash) {
                uint64_t sl = p_slot;
                uint4 e = p_e;
                for (;;) {
                    const uint64_t key = static_cast<uint64_t>(e.x) | (static_cast<uint64_t>(e.y) << 32);
                    if (key == p_rep) {
                        j = static_cast<int64_t>(e.z);
                        st_j = e.w;
                        break;
                    }
                    if (key == kEmptyKey) {
                        j = -1;
                        break;
                    }
                    sl = (sl + 1) & S.hash_mask;
                    e = *reinterpret_cast<const uint4 *>(S.table + sl);
                }
            } else {
                j = lookup_stab<STAGED>(a, L, p_rep, st_j);
            }
            if (j >= 0) {
                const T c = element_value<CHI, CPLX>(sterm[p_t], r, stab_factor(a.plan, L, rs, st_j), a.plan, p_code);
#pragma unroll
                for (int q = 0; q < NR; ++q) accumulate(acc[q], c, x[j * a.ld + a.col + q]);
            } else {
                lookup_miss<W, KIND, CHI>(a, static_cast<W>(p_rep));
            }
        }
        if (!more) {
#pragma unroll
            for (int q = 0; q < NR; ++q) y[row * a.ld + a.col + q] = acc[q];
            ++k;
            row += step;
            if (k >= count || row >= a.dim) break;
            begin_row();
            pend = false;
            continue;
        }
        pend = n_live;
        p_rep = n_rep;
        p_slot = n_slot;
        p_code = n_code;
        p_t = t;
        p_e = n_e;
        ++t;
    }
}

// Rows row0, row0 + step, ... (count of them, below dim) of one job.
// STAGED: the batched launch, whose job's search layout may be a bucket table
// staged in LDS; the other launches never meet one.
template <typename W, int KIND, int CHI, bool CPLX, int NR, uint32_t LX, uint32_t LY, uint32_t NZ,
          bool STAGED = false>
__device__ __forceinline__ void run_rows(const MatvecJob &a, const LdsTables &L, uint64_t row0, uint64_t step,
                                         uint32_t count) {
    // the pipelined loop pays off where up to four columns leave registers
    // for the element in flight (64 ring sectors x 4 columns: 271 -> 259 ms
    // as separate products, 267 -> 261 ms batched); wider products keep the
    // plain loop
    if constexpr (KIND != kOrbitTorus && NR <= 4) {
        run_rows_ahead<W, KIND, CHI, CPLX, NR, LX, LY, NZ, STAGED>(a, L, row0, step, count);
        return;
    }
    constexpr bool TRACK = CHI != kChiTrivial;
    using T = typename Val<CPLX>::T;
    const T *x = static_cast<const T *>(a.x);
    T *y = static_cast<T *>(a.y);
    const ls_term_dev *sterm = L.terms;

    uint64_t row = row0;
    uint32_t k = 0;
    if (count == 0 || row >= a.dim) return;

    uint64_t r = 0;
    RowStab<uses_ratio_table(KIND, STAGED)> rs{};
    T acc[NR];
    uint32_t t = a.n_diag;
    W pr[kTorusCosetSlots] = {};   // p(r) for every coset (torus search)

    auto begin_row = [&]() {
        r = a.search.reps[row];
        rs = row_stab<uses_ratio_table(KIND, STAGED)>(a.plan, L, a.stab[row]);
        double dre, dim_;
        diag_sum<CPLX>(sterm, a.n_diag, r, dre, dim_);
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[q] = diag_times<CPLX>(dre, dim_, x[row * a.ld + a.col + q]);
        if constexpr (KIND == kOrbitTorus) row_images<W>(a.plan, r, pr);
        t = a.n_diag;
    };
    begin_row();

    for (;;) {
        while (t < a.n_terms && (r & sterm[t].sel) != sterm[t].val) ++t;
        if (t >= a.n_terms) {
#pragma unroll
            for (int q = 0; q < NR; ++q) y[row * a.ld + a.col + q] = acc[q];
            ++k;
            row += step;
            if (k >= count || row >= a.dim) break;
            begin_row();
            continue;
        }
        const ls_term_dev &Tm = sterm[t];
        uint32_t code;
        const W rep = neighbour_rep<W, KIND, TRACK, LX, LY, NZ>(a, L, r, pr, t, code);
        ++t;
        uint32_t st_j = 0;
        const int64_t j = lookup_stab<STAGED>(a, L, static_cast<uint64_t>(rep), st_j);
        if (j < 0) {
            lookup_miss<W, KIND, CHI>(a, rep);
            continue;
        }
        const T c = element_value<CHI, CPLX>(Tm, r, stab_factor(a.plan, L, rs, st_j), a.plan, code);
#pragma unroll
        for (int q = 0; q < NR; ++q) accumulate(acc[q], c, x[j * a.ld + a.col + q]);
    }
}

// Lanes per row of the row-group form.
constexpr int kGroupLanes = 16;

// One value from lane `src` of the wavefront (all lanes must be active).
__device__ __forceinline__ double lane_value(double v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ double2 lane_value(double2 v, int src) {
    return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

// Rows of a small sector, kGroupLanes lanes per row (a group of consecutive
// lanes of a wavefront).  A row's acting terms are dealt out in term order:
// lane q of the group generates the row's acting terms number q, q + T,
// q + 2T, ... (T = kGroupLanes).  After each round of T elements every lane
// of the group adds the round's elements to the row's sum in term order,
// reading them from the group's lanes, so the sum is the chain of run_rows
// (diagonal first, then one fma per element in term order) bit for bit,
// while each lane's chain of searches and dependent loads is T times
// shorter.  Groups take rows group, group + n_groups, ...  Single column.
// Every lane of a wavefront stays active through the exchanges: the loops
// run until no lane of the wavefront has work left.
template <typename W, int KIND, int CHI, bool CPLX, uint32_t LX, uint32_t LY, uint32_t NZ>
__device__ __forceinline__ void run_rows_group(const MatvecJob &a, const LdsTables &L, uint64_t group,
                                               uint64_t n_groups) {
    constexpr bool TRACK = CHI != kChiTrivial;
    constexpr uint32_t T = kGroupLanes;
    using V = typename Val<CPLX>::T;
    const V *x = static_cast<const V *>(a.x);
    V *y = static_cast<V *>(a.y);
    const ls_term_dev *sterm = L.terms;
    const uint32_t q = threadIdx.x % T;
    const int lane0 = static_cast<int>((threadIdx.x & 63u) - q);   // the group's first lane in the wavefront
    for (uint64_t row = group;; row += n_groups) {
        const bool live = row < a.dim;
        if (!__any(live)) break;
        uint64_t r = 0;
        RowStab<uses_ratio_table(KIND, false)> rs{};
        V acc{};
        W pr[kTorusCosetSlots] = {};
        if (live) {
            r = a.search.reps[row];
            rs = row_stab<uses_ratio_table(KIND, false)>(a.plan, L, a.stab[row]);
            double dre, dim_;
            diag_sum<CPLX>(sterm, a.n_diag, r, dre, dim_);
            acc = diag_times<CPLX>(dre, dim_, x[row * a.ld + a.col]);
            if constexpr (KIND == kOrbitTorus) row_images<W>(a.plan, r, pr);
        }
        uint32_t t = a.n_diag;   // scan position
        uint32_t seen = 0;       // acting terms passed
        for (uint32_t round = 0;; ++round) {
            // this lane's acting term of the round: number round * T + q
            const uint32_t want = round * T + q;
            bool have = false;
            if (live) {
                while (t < a.n_terms) {
                    if ((r & sterm[t].sel) == sterm[t].val) {
                        if (seen == want) break;
                        ++seen;
                    }
                    ++t;
                }
                have = t < a.n_terms;
            }
            if (!__any(have)) break;
            bool present = false;
            V c{}, xv{};
            if (have) {
                uint32_t code;
                const W rep = neighbour_rep<W, KIND, TRACK, LX, LY, NZ>(a, L, r, pr, t, code);
                uint32_t st_j = 0;
                const int64_t j = lookup_index_stab(a.search, static_cast<uint64_t>(rep), a.stab, st_j);
                if (j >= 0) {
                    c = element_value<CHI, CPLX>(sterm[t], r, stab_factor(a.plan, L, rs, st_j), a.plan, code);
                    xv = x[static_cast<uint64_t>(j) * a.ld + a.col];
                    present = true;
                } else {
                    lookup_miss<W, KIND, CHI>(a, rep);
                }
                ++seen;
                ++t;
            }
            // the round's elements in term order: lanes q = 0 .. T-1 of the group
#pragma unroll
            for (uint32_t s = 0; s < T; ++s) {
                const int src = lane0 + static_cast<int>(s);
                const bool ps = __shfl(present ? 1 : 0, src, 64) != 0;
                const V cs = lane_value(c, src);
                const V xs = lane_value(xv, src);
                if (ps) accumulate(acc, cs, xs);
            }
        }
        if (live && q == 0) y[row * a.ld + a.col] = acc;
    }
}

// y_j += conj(v) x_i with device-scope atomic adds (push form)
__device__ __forceinline__ void scatter_add(double *y, double v, double xi) { unsafeAtomicAdd(y, v * xi); }
__device__ __forceinline__ void scatter_add(double2 *y, double2 v, double2 xi) {
    // conj(v) * xi
    unsafeAtomicAdd(&y->x, v.x * xi.x + v.y * xi.y);
    unsafeAtomicAdd(&y->y, v.x * xi.y - v.y * xi.x);
}

// Push (transposed) form of the product, the second listing of Section 5.3:
// row i's elements H_ij are generated as in the pull form, and H_ji x_i =
// conj(H_ij) x_i is added into y_j (y_i gets the diagonal) with atomic adds,
// so y must start at zero.  The order of the adds into one y_j varies from
// run to run.  Rows row0, row0 + step, ... (count of them).
template <typename W, int KIND, int CHI, bool CPLX, int NR, uint32_t LX, uint32_t LY, uint32_t NZ>
__device__ __forceinline__ void push_rows(const MatvecJob &a, const LdsTables &L, uint64_t row0, uint64_t step,
                                          uint32_t count) {
    constexpr bool TRACK = CHI != kChiTrivial;
    using T = typename Val<CPLX>::T;
    const T *x = static_cast<const T *>(a.x);
    T *y = static_cast<T *>(a.y);
    uint64_t row = row0;
    for (uint32_t k = 0; k < count && row < a.dim; ++k, row += step) {
        const uint64_t r = a.search.reps[row];
        const auto rs = row_stab<uses_ratio_table(KIND, false)>(a.plan, L, a.stab[row]);
        T xi[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) xi[q] = x[row * a.ld + a.col + q];
        double dre, dim_;
        diag_sum<CPLX>(L.terms, a.n_diag, r, dre, dim_);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const T d = diag_times<CPLX>(dre, dim_, xi[q]);
            if constexpr (CPLX) {
                unsafeAtomicAdd(&y[row * a.ld + a.col + q].x, d.x);
                unsafeAtomicAdd(&y[row * a.ld + a.col + q].y, d.y);
            } else {
                unsafeAtomicAdd(&y[row * a.ld + a.col + q], d);
            }
        }
        W pr[kTorusCosetSlots] = {};
        if constexpr (KIND == kOrbitTorus) row_images<W>(a.plan, r, pr);
        for (uint32_t t = a.n_diag; t < a.n_terms; ++t) {
            const ls_term_dev &Tm = L.terms[t];
            if ((r & Tm.sel) != Tm.val) continue;
            uint32_t code;
            const W rep = neighbour_rep<W, KIND, TRACK, LX, LY, NZ>(a, L, r, pr, t, code);
            uint32_t st_j = 0;
            const int64_t j = lookup_index_stab(a.search, static_cast<uint64_t>(rep), a.stab, st_j);
            if (j < 0) {
                lookup_miss<W, KIND, CHI>(a, rep);
                continue;
            }
            const T v = element_value<CHI, CPLX>(Tm, r, stab_factor(a.plan, L, rs, st_j), a.plan, code);
#pragma unroll
            for (int q = 0; q < NR; ++q) scatter_add(&y[static_cast<uint64_t>(j) * a.ld + a.col + q], v, xi[q]);
        }
    }
}

// Kernel variant of an operator: word size, orbit kind, torus shape.
struct Variant {
    int word64;      // 0: 32-bit states, 1: 64-bit
    int kind;        // OrbitKind
    uint32_t lx, ly, nz;   // compile-time torus shape (0 = runtime)
    int chi;         // ChiMode used by the kernel
    bool cplx;
    bool operator==(const Variant &o) const {
        return word64 == o.word64 && kind == o.kind && lx == o.lx && ly == o.ly && nz == o.nz && chi == o.chi &&
               cplx == o.cplx;
    }
};

}  // namespace ls
