// y = H x on the fly, row by row (Section 5.3, first listing, "pull" form).
//
// One lane owns one row i of the sector Hamiltonian:
//   r = reps[i];  acc = (sum of diagonal terms acting on r) * x_i
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
// Right-hand sides: x and y are [dim][ld] row-major; a launch handles NR
// consecutive columns, so the orbit search is shared by NR vectors.

#include "orbit.hpp"

namespace ls {

namespace {

constexpr int kBlock = 256;

struct MatvecArgs {
    PlanDev plan;
    SearchDev search;
    const uint16_t *stab;
    const ls_term_dev *terms;
    uint32_t n_diag, n_terms;
    uint64_t dim;
    uint32_t ld;           // row stride of x and y in elements
    uint32_t col;          // first column handled by this launch
    const void *x;
    void *y;
};

__device__ __forceinline__ double sign_of(uint64_t v) {
    return (__builtin_popcountll(v) & 1) ? -1.0 : 1.0;
}

// CHI: character mode; CPLX: complex vectors and coefficients.
template <typename W, int KIND, int CHI, bool CPLX, int NR>
__global__ void __launch_bounds__(kBlock) k_matvec(MatvecArgs a) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= a.dim) return;
    const uint64_t r64 = a.search.reps[i];
    const double st_i = static_cast<double>(a.stab[i]);

    double dre = 0.0, dim_ = 0.0;
    for (uint32_t t = 0; t < a.n_diag; ++t) {
        const ls_term_dev T = a.terms[t];
        if ((r64 & T.sel) != T.val) continue;
        const double sg = sign_of(r64 & T.sign);
        dre += sg * T.re;
        if constexpr (CPLX) dim_ += sg * T.im;
    }

    if constexpr (!CPLX) {
        const double *x = static_cast<const double *>(a.x);
        double acc[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[q] = dre * x[i * a.ld + a.col + q];
        for (uint32_t t = a.n_diag; t < a.n_terms; ++t) {
            const ls_term_dev T = a.terms[t];
            if ((r64 & T.sel) != T.val) continue;
            const W s = static_cast<W>(r64 ^ T.flip);
            uint32_t code;
            const W rep = orbit_min<W, KIND, (CHI != kChiTrivial)>(a.plan, s, code);
            const int64_t j = lookup_index(a.search, static_cast<uint64_t>(rep));
            if (j < 0) continue;
            double coef = sign_of(r64 & T.sign) * T.re *
                          __dsqrt_rn(__ddiv_rn(static_cast<double>(a.stab[j]), st_i));
            if constexpr (CHI == kChiReal) coef *= a.plan.chi[code].x;
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[q] = fma(coef, x[j * a.ld + a.col + q], acc[q]);
        }
        double *y = static_cast<double *>(a.y);
#pragma unroll
        for (int q = 0; q < NR; ++q) y[i * a.ld + a.col + q] = acc[q];
    } else {
        const double2 *x = static_cast<const double2 *>(a.x);
        double2 acc[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const double2 v = x[i * a.ld + a.col + q];
            acc[q] = make_double2(dre * v.x - dim_ * v.y, dre * v.y + dim_ * v.x);
        }
        for (uint32_t t = a.n_diag; t < a.n_terms; ++t) {
            const ls_term_dev T = a.terms[t];
            if ((r64 & T.sel) != T.val) continue;
            const W s = static_cast<W>(r64 ^ T.flip);
            uint32_t code;
            const W rep = orbit_min<W, KIND, (CHI != kChiTrivial)>(a.plan, s, code);
            const int64_t j = lookup_index(a.search, static_cast<uint64_t>(rep));
            if (j < 0) continue;
            const double sg = sign_of(r64 & T.sign) * __dsqrt_rn(__ddiv_rn(static_cast<double>(a.stab[j]), st_i));
            double cre = sg * T.re, cim = sg * T.im;
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
        double2 *y = static_cast<double2 *>(a.y);
#pragma unroll
        for (int q = 0; q < NR; ++q) y[i * a.ld + a.col + q] = acc[q];
    }
}

template <typename W, int KIND, int CHI, bool CPLX>
void launch_nr(const MatvecArgs &a, int nr, hipStream_t st) {
    const dim3 grid(static_cast<uint32_t>((a.dim + kBlock - 1) / kBlock));
    switch (nr) {
        case 8: hipLaunchKernelGGL((k_matvec<W, KIND, CHI, CPLX, 8>), grid, dim3(kBlock), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_matvec<W, KIND, CHI, CPLX, 4>), grid, dim3(kBlock), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_matvec<W, KIND, CHI, CPLX, 2>), grid, dim3(kBlock), 0, st, a); break;
        default: hipLaunchKernelGGL((k_matvec<W, KIND, CHI, CPLX, 1>), grid, dim3(kBlock), 0, st, a); break;
    }
}

template <typename W, int KIND>
void launch_chi(const MatvecArgs &a, int chi, bool cplx, int nr, hipStream_t st) {
    if (cplx) launch_nr<W, KIND, kChiComplex, true>(a, nr, st);
    else if (chi == kChiReal) launch_nr<W, KIND, kChiReal, false>(a, nr, st);
    else launch_nr<W, KIND, kChiTrivial, false>(a, nr, st);
}

}  // namespace

void launch_matvec(const ls_operator *op, uint32_t nrhs, const void *x, void *y, hipStream_t st) {
    const ls_basis *b = op->basis;
    if (b->dim == 0) return;
    MatvecArgs a{};
    a.plan = b->plan_dev;
    a.search = b->search_dev;
    a.stab = b->d_stab;
    a.terms = op->d_terms;
    a.n_diag = op->n_diag;
    a.n_terms = op->n_diag + op->n_off;
    a.dim = b->dim;
    a.ld = nrhs;
    a.x = x;
    a.y = y;
    const GroupPlan &gp = b->plan;
    const bool cplx = op->is_complex;
    const int chi = gp.chi_mode;
    uint32_t col = 0;
    while (col < nrhs) {
        const uint32_t left = nrhs - col;
        const int nr = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
        a.col = col;
        if (gp.n_sites <= 32) {
            if (gp.ly == 1 && gp.lx == gp.n_sites) launch_chi<uint32_t, kOrbitRing32>(a, chi, cplx, nr, st);
            else launch_chi<uint32_t, kOrbitGeneric>(a, chi, cplx, nr, st);
        } else {
            launch_chi<uint64_t, kOrbitGeneric>(a, chi, cplx, nr, st);
        }
        LS_HIP_CHECK(hipGetLastError());
        col += static_cast<uint32_t>(nr);
    }
}

}  // namespace ls
