// y = H x on the fly, row by row (Section 5.3, first listing, "pull" form).
//
// Row i of the sector Hamiltonian is generated from its representative r:
//   acc = (sum of diagonal terms acting on r) * x_i
//   for each off-diagonal term t acting on r (r & sel == val):
//       s    = r ^ flip_t,  a = conj(c_t) (-1)^popcount(r & sign_t)
//       rep  = orbit minimum of s, g* an element reaching it   (getRow)
//       j    = stateToIndex(rep)                                (lookup)
//       acc += a * chi(g*) * sqrt(stab_j / stab_i) * x_j
//   y_i = acc                                     (one store, no atomics)
// This is <r~_i|H|r~_j> written with P|s> = conj(chi(g*)) P|rep> and the
// Hermiticity of H; a neighbour whose orbit the projector annihilates is
// absent from the basis and contributes nothing.
//
// Work layout.  Each off-diagonal term acts on only part of the rows (a
// Heisenberg exchange term on about a quarter of them), so a loop over the
// terms that is uniform across a wavefront would run the orbit search for
// every term with most lanes idle.  Instead every lane walks its own list:
// one loop iteration = one element (the lane's next acting term of its
// current row); when a lane's row is exhausted it stores y_i and moves to
// its next row.  A lane owns `rows_per_lane` rows strided by the total lane
// count, so per-row differences in the number of acting terms average out.
// The term table is staged in LDS once per workgroup.
//
// Tori (pruned search): permutations act linearly on bits, so for a coset
// representative p, p(r ^ f) = p(r) ^ pi_p(f).  A lane computes p(r) once per
// row and each neighbour's images with one XOR per coset, reading pi_p(f)
// from a per-operator table staged in LDS.  Workgroups of 1024 threads share
// the LDS tables among 16 wavefronts.
//
// Right-hand sides: x and y are [dim][ld] row-major; a launch handles NR
// consecutive columns, so the orbit search is shared by NR vectors.

#include <algorithm>

#include "orbit.hpp"

namespace ls {

namespace {

constexpr int kMaxLdsTerms = 1024;
constexpr size_t kMaxLds = 64 * 1024;

struct MatvecArgs {
    PlanDev plan;
    SearchDev search;
    const uint16_t *stab;
    const ls_term_dev *terms;
    const uint64_t *cflip;  // [n_off][kTorusCosetSlots] (torus search only)
    uint32_t n_diag, n_terms;
    uint64_t dim;
    uint64_t n_lanes;      // total lanes of the launch
    uint32_t rows_per_lane;
    uint32_t ld;           // row stride of x and y in elements
    uint32_t col;          // first column handled by this launch
    const void *x;
    void *y;
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

constexpr int block_of(int kind) { return kind == kOrbitTorus ? 1024 : 256; }

__host__ __device__ constexpr size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

// LDS layout: terms | pair table | col_ge | flip images (torus only)
size_t lds_bytes(int kind, uint32_t n_terms, uint32_t n_off, uint32_t lx) {
    size_t b = align16(std::max<size_t>(n_terms, 1) * sizeof(ls_term_dev));
    if (kind == kOrbitTorus)
        b += align16((size_t(1) << (2 * lx)) * sizeof(uint32_t)) + 64 +
             static_cast<size_t>(n_off) * kTorusCosetSlots * sizeof(uint64_t);
    return b;
}

// CHI: character mode; CPLX: complex vectors and coefficients; LX, LY, NZ:
// torus layout known at compile time (0 = from the plan).
template <typename W, int KIND, int CHI, bool CPLX, int NR, uint32_t LX, uint32_t LY, uint32_t NZ>
__global__ void __launch_bounds__(block_of(KIND)) k_matvec(MatvecArgs a) {
    constexpr int BLOCK = block_of(KIND);
    constexpr bool TRACK = CHI != kChiTrivial;
    using T = typename Val<CPLX>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    ls_term_dev *sterm = reinterpret_cast<ls_term_dev *>(smem);
    for (uint32_t t = threadIdx.x; t < a.n_terms; t += BLOCK) sterm[t] = a.terms[t];
    const uint32_t n_off = a.n_terms - a.n_diag;
    const size_t terms_bytes = align16(static_cast<size_t>(a.n_terms > 0 ? a.n_terms : 1) * sizeof(ls_term_dev));
    uint32_t *slut = reinterpret_cast<uint32_t *>(smem + terms_bytes);
    const uint32_t lut_n = KIND == kOrbitTorus ? (1u << (2 * (LX ? LX : a.plan.lx))) : 0u;
    uint64_t *scol = reinterpret_cast<uint64_t *>(smem + terms_bytes + align16(lut_n * sizeof(uint32_t)));
    uint64_t *scf = scol + 8;   // [slot][n_off]: transposed so lanes spread over banks
    if constexpr (KIND == kOrbitTorus) {
        for (uint32_t q = threadIdx.x; q < lut_n; q += BLOCK) slut[q] = a.plan.pair_lut[q];
        if (threadIdx.x < 8) scol[threadIdx.x] = a.plan.col_ge[threadIdx.x];
        for (uint32_t q = threadIdx.x; q < n_off * kTorusCosetSlots; q += BLOCK) {
            const uint32_t k = q / kTorusCosetSlots, p = q % kTorusCosetSlots;
            scf[p * n_off + k] = a.cflip[q];
        }
    }
    __syncthreads();

    const T *x = static_cast<const T *>(a.x);
    T *y = static_cast<T *>(a.y);
    const uint64_t lane = static_cast<uint64_t>(blockIdx.x) * BLOCK + threadIdx.x;

    uint64_t row = lane;
    uint32_t k = 0;
    if (row >= a.dim) return;

    uint64_t r = 0;
    double st_i = 1.0;
    T acc[NR];
    uint32_t t = a.n_diag;
    W pr[kTorusCosetSlots] = {};   // p(r) for every coset (torus search)

    auto begin_row = [&]() {
        r = a.search.reps[row];
        st_i = static_cast<double>(a.stab[row]);
        double dre = 0.0, dim_ = 0.0;
        for (uint32_t q = 0; q < a.n_diag; ++q) {
            const ls_term_dev &D = sterm[q];
            if ((r & D.sel) != D.val) continue;
            const double sg = sign_of(r & D.sign);
            dre += sg * D.re;
            if constexpr (CPLX) dim_ += sg * D.im;
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const T v = x[row * a.ld + a.col + q];
            if constexpr (CPLX) acc[q] = make_double2(dre * v.x - dim_ * v.y, dre * v.y + dim_ * v.x);
            else acc[q] = dre * v;
        }
        if constexpr (KIND == kOrbitTorus) {
#pragma unroll
            for (uint32_t p = 0; p < kTorusCosetSlots; ++p)
                if (p < a.plan.n_cosets) pr[p] = apply_coset<W>(a.plan.cosets[p], static_cast<W>(r), a.plan);
        }
        t = a.n_diag;
    };
    begin_row();

    for (;;) {
        while (t < a.n_terms && (r & sterm[t].sel) != sterm[t].val) ++t;
        if (t >= a.n_terms) {
#pragma unroll
            for (int q = 0; q < NR; ++q) y[row * a.ld + a.col + q] = acc[q];
            ++k;
            row += a.n_lanes;
            if (k >= a.rows_per_lane || row >= a.dim) break;
            begin_row();
            continue;
        }
        const ls_term_dev &Tm = sterm[t];
        uint32_t code;
        W rep;
        if constexpr (KIND == kOrbitTorus) {
            const uint32_t ko = t - a.n_diag;
            W us[kTorusCosetSlots];
#pragma unroll
            for (uint32_t p = 0; p < kTorusCosetSlots; ++p)
                us[p] = p < a.plan.n_cosets ? (pr[p] ^ static_cast<W>(scf[p * n_off + ko])) : W(0);
            rep = torus_orbit_min<W, TRACK, LX, LY, NZ>(a.plan, us, slut, scol, code);
        } else {
            const W s = static_cast<W>(r ^ Tm.flip);
            rep = orbit_min<W, KIND, TRACK>(a.plan, s, code);
        }
        ++t;
        const int64_t j = lookup_index(a.search, static_cast<uint64_t>(rep));
        if (j < 0) continue;
        const double f = sign_of(r & Tm.sign) * __dsqrt_rn(__ddiv_rn(static_cast<double>(a.stab[j]), st_i));
        if constexpr (!CPLX) {
            double coef = f * Tm.re;
            if constexpr (CHI == kChiReal) coef *= a.plan.chi[code].x;
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[q] = fma(coef, x[j * a.ld + a.col + q], acc[q]);
        } else {
            double cre = f * Tm.re, cim = f * Tm.im;
            if constexpr (CHI != kChiTrivial) {
                const double2 c = a.plan.chi[code];
                const double tre = cre * c.x - cim * c.y;
                cim = cre * c.y + cim * c.x;
                cre = tre;
            }
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const double2 v = x[j * a.ld + a.col + q];
                acc[q].x = fma(cre, v.x, fma(-cim, v.y, acc[q].x));
                acc[q].y = fma(cre, v.y, fma(cim, v.x, acc[q].y));
            }
        }
    }
}

template <typename W, int KIND, int CHI, bool CPLX, uint32_t LX, uint32_t LY, uint32_t NZ>
void launch_nr(MatvecArgs a, int nr, hipStream_t st) {
    constexpr int BLOCK = block_of(KIND);
    const uint64_t fill = 256ull * 4 * 8 * 64;   // 256 CUs x 4 SIMDs x 8 waves
    const uint32_t rpl = static_cast<uint32_t>(std::min<uint64_t>(16, std::max<uint64_t>(1, a.dim / fill)));
    uint64_t lanes = (a.dim + rpl - 1) / rpl;
    lanes = (lanes + BLOCK - 1) / BLOCK * BLOCK;
    a.n_lanes = lanes;
    a.rows_per_lane = rpl;
    const dim3 grid(static_cast<uint32_t>(lanes / BLOCK));
    const size_t lds = lds_bytes(KIND, a.n_terms, a.n_terms - a.n_diag, a.plan.lx);
    switch (nr) {
        case 8: hipLaunchKernelGGL((k_matvec<W, KIND, CHI, CPLX, 8, LX, LY, NZ>), grid, dim3(BLOCK), lds, st, a); break;
        case 4: hipLaunchKernelGGL((k_matvec<W, KIND, CHI, CPLX, 4, LX, LY, NZ>), grid, dim3(BLOCK), lds, st, a); break;
        case 2: hipLaunchKernelGGL((k_matvec<W, KIND, CHI, CPLX, 2, LX, LY, NZ>), grid, dim3(BLOCK), lds, st, a); break;
        default: hipLaunchKernelGGL((k_matvec<W, KIND, CHI, CPLX, 1, LX, LY, NZ>), grid, dim3(BLOCK), lds, st, a); break;
    }
}

template <typename W, int KIND, uint32_t LX = 0, uint32_t LY = 0, uint32_t NZ = 0>
void launch_chi(const MatvecArgs &a, int chi, bool cplx, int nr, hipStream_t st) {
    if (cplx) launch_nr<W, KIND, kChiComplex, true, LX, LY, NZ>(a, nr, st);
    else if (chi == kChiReal) launch_nr<W, KIND, kChiReal, false, LX, LY, NZ>(a, nr, st);
    else launch_nr<W, KIND, kChiTrivial, false, LX, LY, NZ>(a, nr, st);
}

template <typename W>
void launch_torus(const MatvecArgs &a, const GroupPlan &gp, int chi, bool cplx, int nr, hipStream_t st) {
    const uint32_t nz = gp.pair_flip ? 2 : 1;
    if (gp.lx == 6 && gp.ly == 6 && nz == 2) launch_chi<W, kOrbitTorus, 6, 6, 2>(a, chi, cplx, nr, st);
    else if (gp.lx == 6 && gp.ly == 4 && nz == 2) launch_chi<W, kOrbitTorus, 6, 4, 2>(a, chi, cplx, nr, st);
    else if (gp.lx == 4 && gp.ly == 4 && nz == 2) launch_chi<W, kOrbitTorus, 4, 4, 2>(a, chi, cplx, nr, st);
    else launch_chi<W, kOrbitTorus>(a, chi, cplx, nr, st);
}

}  // namespace

uint32_t matvec_max_terms() { return kMaxLdsTerms; }

void launch_matvec(const ls_operator *op, uint32_t nrhs, const void *x, void *y, hipStream_t st) {
    const ls_basis *b = op->basis;
    if (b->dim == 0) return;
    MatvecArgs a{};
    a.plan = b->plan_dev;
    a.search = b->search_dev;
    a.stab = b->d_stab;
    a.terms = op->d_terms;
    a.cflip = op->d_cflip;
    a.n_diag = op->n_diag;
    a.n_terms = op->n_diag + op->n_off;
    a.dim = b->dim;
    a.ld = nrhs;
    a.x = x;
    a.y = y;
    const GroupPlan &gp = b->plan;
    const bool cplx = op->is_complex;
    const int chi = gp.chi_mode;
    const bool torus = gp.torus && op->d_cflip != nullptr &&
                       lds_bytes(kOrbitTorus, a.n_terms, op->n_off, gp.lx) <= kMaxLds;
    uint32_t col = 0;
    while (col < nrhs) {
        const uint32_t left = nrhs - col;
        const int nr = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
        a.col = col;
        if (gp.n_sites <= 32) {
            if (gp.ly == 1 && gp.lx == gp.n_sites) launch_chi<uint32_t, kOrbitRing32>(a, chi, cplx, nr, st);
            else if (torus) launch_torus<uint32_t>(a, gp, chi, cplx, nr, st);
            else launch_chi<uint32_t, kOrbitGeneric>(a, chi, cplx, nr, st);
        } else {
            if (torus) launch_torus<uint64_t>(a, gp, chi, cplx, nr, st);
            else launch_chi<uint64_t, kOrbitGeneric>(a, chi, cplx, nr, st);
        }
        LS_HIP_CHECK(hipGetLastError());
        col += static_cast<uint32_t>(nr);
    }
}

}  // namespace ls
