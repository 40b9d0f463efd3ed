// Host-side group compiler: validation of a symmetry sector, Benes routing
// of bit permutations, and the coset split used by the device orbit search.
//
// The paper builds symmetry groups in its Haskell front end and leaves the
// representative test to the literature (Section 4 "Multiple languages",
// Section 5.2).  Here a group arrives as explicit permutations with
// characters; it is checked to be a group with a one-dimensional
// representation and compiled for the GPU.
//
// Benes networks: a permutation of n = 2^k wires is realised by 2k-1 stages
// of conditional exchanges (Benes 1964); on a machine word every stage is a
// "delta swap" (exchange bit j with bit j+d wherever mask bit j is set),
// stage distances n/2, ..., 2, 1, 2, ..., n/2.  The masks are found with the
// classic looping algorithm: the two wires of every input pair must enter
// different half-size subnetworks, and so must the two sources of every
// output pair; following these constraints around each cycle 2-colours the
// wires, then each half is routed recursively.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "ls_internal.hpp"

namespace ls {

namespace {

struct Elem {
    std::vector<uint16_t> perm;
    uint8_t flip;
};

std::string key_of(const uint16_t *perm, uint32_t n, uint8_t flip) {
    std::string k(reinterpret_cast<const char *>(perm), n * sizeof(uint16_t));
    k.push_back(static_cast<char>(flip));
    return k;
}

// Recursive looping-algorithm router on block [off, off+m) at a given level.
void route_block(const std::vector<int> &pi, int off, int m, int level, int n_levels,
                 uint64_t *masks) {
    if (m == 2) {
        if (pi[0] == 1) masks[level] |= 1ULL << off;
        return;
    }
    const int h = m / 2;
    std::vector<int> inv(m), side(m, -1);
    for (int i = 0; i < m; ++i) inv[pi[i]] = i;
    for (int j = 0; j < h; ++j) {
        if (side[j] >= 0) continue;
        int i = j;
        int s = 0;
        while (side[i] < 0) {
            side[i] = s;
            // the other source of i's output pair goes to the other half
            int o2 = pi[i] ^ h;
            int i2 = inv[o2];
            if (side[i2] >= 0) break;
            side[i2] = 1 - s;
            // the input partner of i2 goes to the half opposite to i2
            i = i2 ^ h;
            s = s;  // i2's partner gets 1 - (1 - s) = s
        }
    }
    std::vector<int> sub0(h), sub1(h);
    const int first = level, last = 2 * (n_levels - 1) - level;
    for (int i = 0; i < m; ++i) {
        const int pos_in = i & (h - 1);
        const int pos_out = pi[i] & (h - 1);
        if (side[i] == 0) {
            sub0[pos_in] = pos_out;
            if (i >= h) masks[first] |= 1ULL << (off + pos_in);   // bottom input moved up
            if (pi[i] >= h) masks[last] |= 1ULL << (off + pos_out);
        } else {
            sub1[pos_in] = pos_out;
            if (i < h) masks[first] |= 1ULL << (off + pos_in);     // top input moved down
        }
    }
    route_block(sub0, off, h, level + 1, n_levels, masks);
    route_block(sub1, off + h, h, level + 1, n_levels, masks);
}

}  // namespace

int benes_route(const std::vector<int> &dest, int n, uint64_t *masks) {
    int k = 0;
    while ((1 << k) < n) ++k;
    const int n_stages = 2 * k - 1;
    for (int s = 0; s < kMaxStages; ++s) masks[s] = 0;
    route_block(dest, 0, n, 0, k, masks);
    return n_stages;
}

uint64_t benes_apply_host(uint64_t x, const uint64_t *masks, int n_stages, int n) {
    const int k = (n_stages + 1) / 2;
    for (int s = 0; s < n_stages; ++s) {
        const int lvl = s < k ? s : 2 * (k - 1) - s;
        const int d = n >> (lvl + 1);
        const uint64_t t = ((x >> d) ^ x) & masks[s];
        x ^= t ^ (t << d);
    }
    if (n < 64) x &= (1ULL << n) - 1ULL;
    return x;
}

GroupPlan compile_group(const ls_sector_desc &d) {
    const uint32_t n = d.n_sites;
    LS_REQUIRE(n >= 1 && n <= 64, "n_sites must be in 1..64");
    LS_REQUIRE(d.hamming_weight >= -1 && d.hamming_weight <= static_cast<int32_t>(n),
               "hamming_weight must be -1 or in 0..n_sites");
    LS_REQUIRE(d.hamming_weight >= 0 || n <= 36, "without U(1) the library enumerates 2^N states; N must be <= 36");
    LS_REQUIRE(d.n_elements >= 1 && d.n_elements <= 4096, "n_elements must be in 1..4096");
    LS_REQUIRE(d.perm && d.flip && d.chi, "perm, flip and chi must not be NULL");
    const uint32_t ng = d.n_elements;

    std::unordered_map<std::string, int> index;
    index.reserve(ng * 2);
    for (uint32_t g = 0; g < ng; ++g) {
        const uint16_t *p = d.perm + static_cast<size_t>(g) * n;
        std::vector<char> seen(n, 0);
        for (uint32_t i = 0; i < n; ++i) {
            LS_REQUIRE(p[i] < n, "perm entry out of range");
            LS_REQUIRE(!seen[p[i]], "perm is not a bijection");
            seen[p[i]] = 1;
        }
        LS_REQUIRE(d.flip[g] <= 1, "flip must be 0 or 1");
        if (d.flip[g]) LS_REQUIRE(d.hamming_weight < 0 || 2 * d.hamming_weight == static_cast<int32_t>(n),
                                  "spin inversion needs hamming_weight = n_sites / 2");
        const double re = d.chi[2 * g], im = d.chi[2 * g + 1];
        LS_REQUIRE(std::isfinite(re) && std::isfinite(im) && std::fabs(std::hypot(re, im) - 1.0) < 1e-9,
                   "characters must have modulus 1");
        auto ins = index.emplace(key_of(p, n, d.flip[g]), static_cast<int>(g));
        LS_REQUIRE(ins.second, "duplicate group element");
    }
    // identity present with character 1
    std::vector<uint16_t> ident(n);
    for (uint32_t i = 0; i < n; ++i) ident[i] = static_cast<uint16_t>(i);
    auto it_id = index.find(key_of(ident.data(), n, 0));
    LS_REQUIRE(it_id != index.end(), "the group must contain the identity");
    {
        const int g = it_id->second;
        LS_REQUIRE(std::fabs(d.chi[2 * g] - 1.0) < 1e-9 && std::fabs(d.chi[2 * g + 1]) < 1e-9,
                   "the identity must have character 1");
    }
    // closure and homomorphism: chi(g h) = chi(g) chi(h)
    std::vector<uint16_t> comp(n);
    for (uint32_t g = 0; g < ng; ++g) {
        const uint16_t *pg = d.perm + static_cast<size_t>(g) * n;
        for (uint32_t h = 0; h < ng; ++h) {
            const uint16_t *ph = d.perm + static_cast<size_t>(h) * n;
            for (uint32_t i = 0; i < n; ++i) comp[i] = pg[ph[i]];
            auto it = index.find(key_of(comp.data(), n, d.flip[g] ^ d.flip[h]));
            LS_REQUIRE(it != index.end(), "the elements are not closed under composition");
            const int gh = it->second;
            const double are = d.chi[2 * g], aim = d.chi[2 * g + 1];
            const double bre = d.chi[2 * h], bim = d.chi[2 * h + 1];
            const double pre = are * bre - aim * bim, pim = are * bim + aim * bre;
            LS_REQUIRE(std::fabs(pre - d.chi[2 * gh]) < 1e-9 && std::fabs(pim - d.chi[2 * gh + 1]) < 1e-9,
                       "chi is not a one-dimensional representation (chi(gh) != chi(g) chi(h))");
        }
    }

    GroupPlan P;
    P.n_sites = n;
    P.n_elements = ng;
    P.full = n == 64 ? ~0ULL : ((1ULL << n) - 1ULL);
    P.n_stages = n <= 32 ? 9 : 11;
    const int wires = n <= 32 ? 32 : 64;

    auto find_elem = [&](const std::vector<uint16_t> &perm, uint8_t flip) -> int {
        auto it = index.find(key_of(perm.data(), n, flip));
        return it == index.end() ? -1 : it->second;
    };

    // spin inversion pairing
    P.pair_flip = find_elem(ident, 1) >= 0 ? 1 : 0;

    // translation layout: lx * ly = n, every (x,y) -> (x+a, y+b) present
    auto trans_perm = [&](uint32_t lx, uint32_t ly, uint32_t a, uint32_t b) {
        std::vector<uint16_t> p(n);
        if (lx * ly != n) {   // no translation layout: T = {identity}
            for (uint32_t i = 0; i < n; ++i) p[i] = static_cast<uint16_t>(i);
            return p;
        }
        for (uint32_t y = 0; y < ly; ++y)
            for (uint32_t x = 0; x < lx; ++x)
                p[x + lx * y] = static_cast<uint16_t>(((x + a) % lx) + lx * ((y + b) % ly));
        return p;
    };
    std::vector<uint32_t> shapes;
    shapes.push_back(n);
    for (uint32_t lx = n - 1; lx >= 2; --lx)
        if (n % lx == 0) shapes.push_back(lx);
    P.lx = 1;
    P.ly = 1;
    if (ng > 1) {
        for (uint32_t lx : shapes) {
            const uint32_t ly = n / lx;
            if (lx == 1) continue;
            bool ok = true;
            for (uint32_t b = 0; b < ly && ok; ++b)
                for (uint32_t a = 0; a < lx && ok; ++a)
                    ok = find_elem(trans_perm(lx, ly, a, b), 0) >= 0;
            if (ok) { P.lx = lx; P.ly = ly; break; }
        }
    }
    for (uint32_t y = 0; y < P.ly; ++y) P.col0 |= 1ULL << (P.lx * y);
    const uint32_t nt = P.lx * P.ly;
    const uint32_t nz = P.pair_flip ? 2 : 1;

    // the elements of (Z x T) o g
    auto coset_of = [&](int g) {
        std::vector<int> out;
        const uint16_t *pg = d.perm + static_cast<size_t>(g) * n;
        for (uint32_t t = 0; t < nt; ++t) {
            auto tp = trans_perm(P.lx, P.ly, t % P.lx, t / P.lx);
            std::vector<uint16_t> c(n);
            for (uint32_t i = 0; i < n; ++i) c[i] = tp[pg[i]];
            for (uint32_t z = 0; z < nz; ++z) {
                int e = find_elem(c, static_cast<uint8_t>(d.flip[g] ^ z));
                if (e < 0) throw Error{LS_EINTERNAL, "coset element missing from a closed group"};
                out.push_back(e);
            }
        }
        return out;
    };
    std::vector<uint16_t> reverse(n);
    for (uint32_t i = 0; i < n; ++i) reverse[i] = static_cast<uint16_t>(n - 1 - i);
    const int rev_elem = find_elem(reverse, 0);

    std::vector<char> covered(ng, 0);
    std::vector<int> reps;
    auto take = [&](int g) {
        auto c = coset_of(g);
        int best = -1, rank = 4;
        for (int e : c) {
            int r;
            if (e == it_id->second) r = 0;
            else if (e == rev_elem) r = 1;
            else if (d.flip[e] == 0) r = 2;
            else r = 3;
            if (r < rank || (r == rank && e < best)) { rank = r; best = e; }
        }
        for (int e : c) {
            if (covered[e]) throw Error{LS_EINTERNAL, "cosets overlap"};
            covered[e] = 1;
        }
        reps.push_back(best);
    };
    take(it_id->second);
    for (uint32_t g = 0; g < ng; ++g)
        if (!covered[g]) take(static_cast<int>(g));

    // Benes networks for the coset representatives
    for (int e : reps) {
        CosetRep cr{};
        cr.flip = d.flip[e];
        const uint16_t *pe = d.perm + static_cast<size_t>(e) * n;
        bool is_id = true, is_rev = true;
        for (uint32_t i = 0; i < n; ++i) {
            is_id = is_id && pe[i] == i;
            is_rev = is_rev && pe[i] == n - 1 - i;
        }
        if (is_id) {
            cr.kind = kCosetIdentity;
        } else if (is_rev) {
            cr.kind = kCosetReverse;
        } else {
            cr.kind = kCosetBenes;
            std::vector<int> dest(wires);
            for (int i = 0; i < wires; ++i) dest[i] = i < static_cast<int>(n) ? pe[i] : i;
            const int st = benes_route(dest, wires, cr.masks);
            if (st != static_cast<int>(P.n_stages)) throw Error{LS_EINTERNAL, "Benes stage count"};
            for (int i = 0; i < wires; ++i) {
                const uint64_t got = benes_apply_host(1ULL << i, cr.masks, st, wires);
                if (got != (1ULL << dest[i])) throw Error{LS_EINTERNAL, "Benes routing self-check failed"};
            }
        }
        P.cosets.push_back(cr);
    }

    // character table by code ((p * nt) + t) * nz + f, element F^f o tau_t o p
    const uint32_t ncode = static_cast<uint32_t>(P.cosets.size()) * nt * nz;
    if (ncode != ng) throw Error{LS_EINTERNAL, "coset split does not cover the group"};
    P.chi.assign(2 * ng, 0.0);
    P.chi_one.assign((ng + 31) / 32, 0u);
    P.code_to_index.assign(ng, -1);
    std::vector<char> hit(ng, 0);
    bool trivial = true, real = true;
    for (uint32_t p = 0; p < P.cosets.size(); ++p) {
        const uint16_t *pp = d.perm + static_cast<size_t>(reps[p]) * n;
        for (uint32_t t = 0; t < nt; ++t) {
            auto tp = trans_perm(P.lx, P.ly, t % P.lx, t / P.lx);
            std::vector<uint16_t> c(n);
            for (uint32_t i = 0; i < n; ++i) c[i] = tp[pp[i]];
            for (uint32_t f = 0; f < nz; ++f) {
                const uint32_t code = (p * nt + t) * nz + f;
                const int e = find_elem(c, static_cast<uint8_t>(d.flip[reps[p]] ^ f));
                if (e < 0 || hit[e]) throw Error{LS_EINTERNAL, "code table is not a bijection"};
                hit[e] = 1;
                P.code_to_index[code] = e;
                double re = d.chi[2 * e], im = d.chi[2 * e + 1];
                const bool one = std::fabs(re - 1.0) < 1e-9 && std::fabs(im) < 1e-9;
                if (!one) trivial = false;
                if (std::fabs(im) >= 1e-9) real = false;
                P.chi[2 * code] = re;
                P.chi[2 * code + 1] = im;
                if (one) P.chi_one[code / 32] |= 1u << (code % 32);
            }
        }
    }
    P.chi_mode = trivial ? kChiTrivial : (real ? kChiReal : kChiComplex);

    // Pruning table for tori: the top two rows of an image decide the order
    // unless they tie, and for each pair of rows the x-rotation that makes
    // the pair smallest is fixed by the pair alone.
    if (P.lx >= 2 && P.lx <= 6 && P.ly >= 2 && P.cosets.size() <= 8 && P.cosets.size() * P.ly * nz <= 128) {
        P.torus = true;
        const uint32_t L = P.lx, rm = (1u << L) - 1u;
        auto rot = [&](uint32_t v, uint32_t a) { return a == 0 ? v : (((v << a) | (v >> (L - a))) & rm); };
        const uint32_t nq = 1u << (2 * L);
        std::vector<uint32_t> single(nq);
        for (uint32_t q = 0; q < nq; ++q) {
            const uint32_t top = q >> L, second = q & rm;
            uint32_t best = ~0u, arg = 0, ties = 0;
            for (uint32_t a = 0; a < L; ++a) {
                const uint32_t v = (rot(top, a) << L) | rot(second, a);
                if (v < best) { best = v; arg = a; ties = 1; }
                else if (v == best) ++ties;
            }
            single[q] = (best << 4) | ((ties > 1 ? 1u : 0u) << 3) | arg;
        }
        // each entry also carries the entry of the spin-flipped pair
        P.pair_lut.resize(nq);
        for (uint32_t q = 0; q < nq; ++q) P.pair_lut[q] = single[q] | (single[q ^ (nq - 1)] << 16);
        for (uint32_t a = 0; a < L; ++a) {
            const uint64_t rowpat = static_cast<uint64_t>(rm & ~((1u << a) - 1u));
            uint64_t m = 0;
            for (uint32_t y = 0; y < P.ly; ++y) m |= rowpat << (L * y);
            P.col_ge[a] = m;
        }
    }
    if (P.chi_mode != kChiComplex) {
        // characters within 1e-9 of +-1 are used as exactly +-1
        for (uint32_t c = 0; c < ng; ++c) {
            P.chi[2 * c] = P.chi[2 * c] > 0 ? 1.0 : -1.0;
            P.chi[2 * c + 1] = 0.0;
        }
    }
    return P;
}

}  // namespace ls
