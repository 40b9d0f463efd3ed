// Term-table compiler: validation and device layout of the Hamiltonian.
//
// The paper compiles symbolic Hamiltonians to kernels in its front end
// (Section 4); here H arrives as elementary terms
//   c * sum_{s: s & sel == val} (-1)^popcount(s & sign) |s ^ flip><s|
// and is validated before use:
//   * Hermitian as a whole (required by the pull form of the product, which
//     reads row i of H from the terms acting on r_i);
//   * weight conserving when the sector fixes the Hamming weight;
//   * invariant under every group element, so H commutes with the
//     projector onto the sector.
// Terms are compared in a canonical form: sign bits inside sel are folded
// into the coefficient (those bits of s are fixed by val), equal
// (sel, val, flip, sign) merge by summing coefficients, zeros drop out.

#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <tuple>

#include "ls_internal.hpp"

namespace ls {

namespace {

using cplx = std::complex<double>;
using Key = std::tuple<uint64_t, uint64_t, uint64_t, uint64_t>;   // sel, val, flip, sign

struct Term {
    cplx c;
    uint64_t sel, val, flip, sign;
};

int parity(uint64_t v) { return __builtin_popcountll(v) & 1; }

std::map<Key, cplx> canonical(const std::vector<Term> &ts) {
    std::map<Key, cplx> m;
    for (const Term &t : ts) {
        cplx c = t.c;
        if (parity(t.val & t.sign & t.sel)) c = -c;
        const uint64_t sign = t.sign & ~t.sel;
        m[Key{t.sel, t.val, t.flip, sign}] += c;
    }
    return m;
}

bool same_operator(const std::map<Key, cplx> &a, const std::map<Key, cplx> &b, double tol) {
    auto it = a.begin();
    auto jt = b.begin();
    // walk both ordered maps, treating missing keys as zero
    while (it != a.end() || jt != b.end()) {
        if (jt == b.end() || (it != a.end() && it->first < jt->first)) {
            if (std::abs(it->second) > tol) return false;
            ++it;
        } else if (it == a.end() || jt->first < it->first) {
            if (std::abs(jt->second) > tol) return false;
            ++jt;
        } else {
            if (std::abs(it->second - jt->second) > tol) return false;
            ++it;
            ++jt;
        }
    }
    return true;
}

uint64_t permute_mask(uint64_t m, const uint16_t *perm, uint32_t n) {
    uint64_t out = 0;
    for (uint32_t i = 0; i < n; ++i)
        if ((m >> i) & 1ULL) out |= 1ULL << perm[i];
    return out;
}

}  // namespace

void compile_terms(const ls_basis *b, uint32_t n_terms, const ls_term *terms, ls_operator *op) {
    LS_REQUIRE(n_terms == 0 || terms != nullptr, "terms must not be NULL");
    LS_REQUIRE(n_terms <= matvec_max_terms(), "too many terms (the product stages at most 1024 in LDS)");
    const GroupPlan &gp = b->plan;
    const uint32_t n = gp.n_sites;
    const uint64_t full = gp.full;
    std::vector<Term> ts;
    ts.reserve(n_terms);
    double cmax = 0.0;
    bool complex_coef = false;
    for (uint32_t k = 0; k < n_terms; ++k) {
        const ls_term &t = terms[k];
        LS_REQUIRE(std::isfinite(t.re) && std::isfinite(t.im), "term coefficient is not finite");
        LS_REQUIRE(((t.sel_mask | t.sel_value | t.flip | t.sign_mask) & ~full) == 0,
                   "term masks use bits at or above n_sites");
        LS_REQUIRE((t.sel_value & ~t.sel_mask) == 0, "sel_value has bits outside sel_mask");
        if (b->weight >= 0 && t.flip != 0) {
            LS_REQUIRE((t.flip & ~t.sel_mask) == 0,
                       "with a fixed Hamming weight, flip must lie inside sel_mask");
            LS_REQUIRE(__builtin_popcountll(t.flip & t.sel_value) == __builtin_popcountll(t.flip & ~t.sel_value),
                       "term does not conserve the Hamming weight");
        }
        ts.push_back(Term{cplx(t.re, t.im), t.sel_mask, t.sel_value, t.flip, t.sign_mask});
        cmax = std::max(cmax, std::abs(ts.back().c));
        complex_coef = complex_coef || t.im != 0.0;
    }
    const double tol = 1e-12 * std::max(1.0, cmax);
    const auto canon = canonical(ts);

    // Hermiticity: the adjoint of every term, compared as an operator
    {
        std::vector<Term> adj;
        adj.reserve(ts.size());
        for (const Term &t : ts) {
            cplx c = std::conj(t.c);
            if (parity(t.flip & t.sign)) c = -c;
            adj.push_back(Term{c, t.sel, t.val ^ (t.flip & t.sel), t.flip, t.sign});
        }
        LS_REQUIRE(same_operator(canon, canonical(adj), tol), "the term list is not Hermitian");
    }
    // invariance under the group: U_g H U_g^dagger == H
    {
        const auto &perms = b->perm_copy;
        const auto &flips = b->flip_copy;
        std::vector<Term> tr;
        tr.reserve(ts.size());
        for (uint32_t g = 0; g < gp.n_elements; ++g) {
            const uint16_t *p = perms.data() + static_cast<size_t>(g) * n;
            tr.clear();
            for (const Term &t : ts) {
                Term u;
                u.sel = permute_mask(t.sel, p, n);
                u.val = permute_mask(t.val, p, n);
                u.flip = permute_mask(t.flip, p, n);
                u.sign = permute_mask(t.sign, p, n);
                u.c = t.c;
                if (flips[g]) {
                    u.val ^= u.sel;
                    if (parity(t.sign)) u.c = -u.c;
                }
                tr.push_back(u);
            }
            LS_REQUIRE(same_operator(canon, canonical(tr), tol),
                       "the term list does not commute with the symmetry group");
        }
    }

    op->is_complex = gp.chi_mode == kChiComplex || complex_coef;
    // device layout: diagonal terms first, coefficients conjugated for the
    // pull form (row i uses conj(a_t(r_i)))
    op->host_terms.clear();
    for (int pass = 0; pass < 2; ++pass)
        for (const Term &t : ts) {
            if ((t.flip == 0) != (pass == 0)) continue;
            ls_term_dev d{};
            d.re = t.c.real();
            d.im = -t.c.imag();
            d.sel = t.sel;
            d.val = t.val;
            d.flip = t.flip;
            d.sign = t.sign;
            op->host_terms.push_back(d);
        }
    op->n_diag = 0;
    for (const Term &t : ts) op->n_diag += t.flip == 0 ? 1u : 0u;
    op->n_off = static_cast<uint32_t>(ts.size()) - op->n_diag;

    // p(r ^ f) = p(r) ^ pi_p(f) for a coset representative p = (pi_p, flip):
    // the images of each flip mask let the kernel reuse p(r) for a whole row
    op->host_cflip.clear();
    if (gp.torus) {
        const int wires = n <= 32 ? 32 : 64;
        op->host_cflip.assign(static_cast<size_t>(op->n_off) * kTorusCosetSlots, 0);
        for (uint32_t k = 0; k < op->n_off; ++k) {
            const uint64_t f = op->host_terms[op->n_diag + k].flip;
            for (uint32_t p = 0; p < gp.cosets.size(); ++p) {
                const CosetRep &c = gp.cosets[p];
                uint64_t g = f;
                if (c.kind == kCosetReverse) {
                    g = 0;
                    for (uint32_t i = 0; i < n; ++i)
                        if ((f >> i) & 1ULL) g |= 1ULL << (n - 1 - i);
                } else if (c.kind == kCosetBenes) {
                    g = benes_apply_host(f, c.masks, static_cast<int>(gp.n_stages), wires);
                }
                op->host_cflip[static_cast<size_t>(k) * kTorusCosetSlots + p] = g;
            }
        }
    }
}

}  // namespace ls
