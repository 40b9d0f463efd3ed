// Host-side selection of the product kernel's template variant.
#pragma once

#include "matvec_impl.hpp"

namespace ls {

MatvecJob job_of(const ls_operator *op, const void *x, void *y, uint32_t ld, uint32_t col);
Variant variant_of(const ls_operator *op);
int nr_chunk(uint32_t left);   // right-hand sides per launch: 8, 4, 2 or 1

template <typename W, int KIND, int CHI, bool CPLX, uint32_t LX, uint32_t LY, uint32_t NZ, class F>
void dispatch_nr(int nr, F &f) {
    switch (nr) {
        case 8: f.template run<W, KIND, CHI, CPLX, 8, LX, LY, NZ>(); break;
        case 4: f.template run<W, KIND, CHI, CPLX, 4, LX, LY, NZ>(); break;
        case 2: f.template run<W, KIND, CHI, CPLX, 2, LX, LY, NZ>(); break;
        default: f.template run<W, KIND, CHI, CPLX, 1, LX, LY, NZ>(); break;
    }
}

template <typename W, int KIND, uint32_t LX, uint32_t LY, uint32_t NZ, class F>
void dispatch_chi(const Variant &v, int nr, F &f) {
    if (v.cplx) dispatch_nr<W, KIND, kChiComplex, true, LX, LY, NZ>(nr, f);
    else if (v.chi == kChiReal) dispatch_nr<W, KIND, kChiReal, false, LX, LY, NZ>(nr, f);
    else dispatch_nr<W, KIND, kChiTrivial, false, LX, LY, NZ>(nr, f);
}

template <typename W, class F>
void dispatch_kind(const Variant &v, int nr, F &f) {
    if (v.kind == kOrbitRing32) {
        if constexpr (sizeof(W) == 4) dispatch_chi<W, kOrbitRing32, 0, 0, 0>(v, nr, f);
    } else if (v.kind == kOrbitRing64) {
        if constexpr (sizeof(W) == 8) dispatch_chi<W, kOrbitRing64, 0, 0, 0>(v, nr, f);
    } else if (v.kind == kOrbitTorus) {
        if constexpr (sizeof(W) == 8) {
            if (v.lx == 6 && v.ly == 6 && v.nz == 2) return dispatch_chi<W, kOrbitTorus, 6, 6, 2>(v, nr, f);
        } else {
            if (v.lx == 4 && v.ly == 4 && v.nz == 2) return dispatch_chi<W, kOrbitTorus, 4, 4, 2>(v, nr, f);
        }
        dispatch_chi<W, kOrbitTorus, 0, 0, 0>(v, nr, f);
    } else {
        dispatch_chi<W, kOrbitGeneric, 0, 0, 0>(v, nr, f);
    }
}

template <class F>
void dispatch(const Variant &v, int nr, F &f) {
    if (v.word64) dispatch_kind<uint64_t>(v, nr, f);
    else dispatch_kind<uint32_t>(v, nr, f);
}

}  // namespace ls
