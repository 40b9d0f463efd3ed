// Device helpers: group action, orbit search and stateToIndex.
//
// Every lane owns one basis state and walks the whole group in registers:
// for each coset representative p (identity, full bit reversal or a Benes
// network of delta swaps), the translated images tau_t(p(s)) are produced
// by shifts (x-rotation of every row, rotation of the word by one row), and
// with spin inversion in the group each image v is paired with v ^ full.
// The representative is the minimum image (the orbit minimum).
#pragma once

#include "ls_internal.hpp"

namespace ls {

// Structure kinds the kernels are specialised for.
enum OrbitKind : int {
    kOrbitGeneric = 0,   // runtime lx, ly (ring, torus, or no translations)
    kOrbitRing32 = 1,    // N <= 32 ring: all rotations from one funnel shift each
    kOrbitTorus = 2,     // lx <= 6, ly >= 2 torus: pruned by the pair table
    kOrbitRing64 = 3,    // 32 < N < 64 ring: rotations pruned by the longest zero run
};

// A value that is the same in every active lane, moved to a scalar register.
// Loop counters of the group walk are uniform, but the walk runs inside
// each lane's own element loop, where the compiler cannot prove it; scalar
// counters keep coset masks in scalar loads and index arithmetic off the
// vector ALU.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

template <typename W>
__device__ __forceinline__ W benes_apply(W x, const uint64_t *m) {
    if constexpr (sizeof(W) == 4) {
        constexpr int dl[9] = {16, 8, 4, 2, 1, 2, 4, 8, 16};
#pragma unroll
        for (int s = 0; s < 9; ++s) {
            const W t = ((x >> dl[s]) ^ x) & static_cast<W>(m[s]);
            x ^= t ^ (t << dl[s]);
        }
    } else {
        constexpr int dl[11] = {32, 16, 8, 4, 2, 1, 2, 4, 8, 16, 32};
#pragma unroll
        for (int s = 0; s < 11; ++s) {
            const W t = ((x >> dl[s]) ^ x) & static_cast<W>(m[s]);
            x ^= t ^ (t << dl[s]);
        }
    }
    return x;
}

template <typename W>
__device__ __forceinline__ W bit_reverse(W x, uint32_t n) {
    if constexpr (sizeof(W) == 4)
        return static_cast<W>(__builtin_bitreverse32(static_cast<uint32_t>(x)) >> (32u - n));
    else
        return static_cast<W>(__builtin_bitreverse64(static_cast<uint64_t>(x)) >> (64u - n));
}

template <typename W>
__device__ __forceinline__ W apply_coset(const CosetRep &c, W s, const PlanDev &P) {
    W u;
    if (c.kind == kCosetIdentity)
        u = s;
    else if (c.kind == kCosetReverse)
        u = bit_reverse<W>(s, P.n_sites);
    else
        u = benes_apply<W>(s, c.masks);
    if (c.flip) u ^= static_cast<W>(P.full);
    return u;
}

// (x, y) -> (x + 1, y) for every row of an lx-wide layout
template <typename W>
__device__ __forceinline__ W xrot(W v, const PlanDev &P) {
    const W c0 = static_cast<W>(P.col0), full = static_cast<W>(P.full);
    return ((v << 1) & ~c0 & full) | ((v >> (P.lx - 1)) & c0);
}

// (x, y) -> (x, y + 1): rotate the N-bit word by one row
template <typename W>
__device__ __forceinline__ W yrot(W v, const PlanDev &P) {
    return ((v << P.lx) | (v >> (P.n_sites - P.lx))) & static_cast<W>(P.full);
}

__device__ __forceinline__ bool chi_is_one(const PlanDev &P, uint32_t code) {
    return (P.chi_one[code >> 5] >> (code & 31)) & 1u;
}

// Visit every group image of s: f(v, code).  Returning false from f stops.
template <typename W, int KIND, typename F>
__device__ __forceinline__ void for_each_image(const PlanDev &P, W s, F &&f) {
    const uint32_t nz = P.pair_flip ? 2u : 1u;
    const W full = static_cast<W>(P.full);
    for (uint32_t p0 = 0; p0 < P.n_cosets; ++p0) {
        const uint32_t p = uni(p0);
        const CosetRep c = P.cosets[p];
        W u = apply_coset<W>(c, s, P);
        if constexpr (KIND == kOrbitRing32) {
            // u doubled into 64 bits: rotating right by t is one funnel shift
            const uint32_t n = P.n_sites;
            const uint64_t uu = static_cast<uint64_t>(u) | (static_cast<uint64_t>(u) << n);
            const uint32_t lo = static_cast<uint32_t>(uu), hi = static_cast<uint32_t>(uu >> 32);
            for (uint32_t t0 = 0; t0 < n; ++t0) {
                const uint32_t t = uni(t0);
                const W v = static_cast<W>(__builtin_amdgcn_alignbit(hi, lo, t)) & full;
                // right rotation by t is the translation a = (n - t) mod n
                const uint32_t a = t == 0 ? 0u : n - t;
                const uint32_t base = uni((p * n + a) * nz);
                if (!f(v, base)) return;
                if (P.pair_flip && !f(static_cast<W>(v ^ full), base + 1)) return;
            }
        } else {
            for (uint32_t b = 0; b < P.ly; ++b) {
                W v = u;
                for (uint32_t a = 0; a < P.lx; ++a) {
                    const uint32_t base = uni((p * P.n_trans + a + P.lx * b) * nz);
                    if (!f(v, base)) return;
                    if (P.pair_flip && !f(static_cast<W>(v ^ full), base + 1)) return;
                    if (a + 1 < P.lx) v = xrot<W>(v, P);
                }
                if (b + 1 < P.ly) u = yrot<W>(u, P);
            }
        }
    }
}

// Rotations of the low n bits of a 64-bit word (0 <= k < n < 64).
__device__ __forceinline__ uint64_t rotl_n(uint64_t w, uint32_t k, uint32_t n, uint64_t full) {
    return ((w << k) | (w >> (n - k))) & full;
}
__device__ __forceinline__ uint64_t rotr_n(uint64_t w, uint32_t k, uint32_t n, uint64_t full) {
    return ((w >> k) | (w << (n - k))) & full;
}

// Longest cyclic run of zeros of the n-bit ring word w (32 < n < 64): its
// length L and the mask of the bits where such a run starts (runs go upward,
// wrapping from bit n-1 to bit 0).  Doubling masks R_k (bit i set when zeros
// occupy i .. i+k-1) and binary lifting of the length.  L = 0 when w has no
// zero; L = n and start mask 1 when w is zero.
__device__ __forceinline__ uint64_t ring64_runs(uint64_t w, uint32_t n, uint64_t full, uint32_t &L) {
    const uint64_t z = ~w & full;
    if (z == 0) {
        L = 0;
        return 0;
    }
    if (z == full) {
        L = n;
        return 1;
    }
    uint64_t R[6];               // runs of 1, 2, 4, 8, 16, 32 zeros (32 < n)
    R[0] = z;
#pragma unroll
    for (uint32_t l = 1; l < 6; ++l) R[l] = R[l - 1] & rotr_n(R[l - 1], 1u << (l - 1), n, full);
    uint64_t cur = z;
    uint32_t len = 1;
#pragma unroll
    for (int l = 5; l >= 0; --l) {
        const uint32_t k = 1u << l;
        if (len + k < n) {
            const uint64_t c = cur & rotr_n(R[l], len, n, full);
            if (c) {
                cur = c;
                len += k;
            }
        }
    }
    L = len;
    return cur;
}

// The smallest rotation of w puts one of its longest zero runs on top (a
// smaller word has more leading zeros): compare the rotations that lift each
// run start in `starts` (runs of length L) to bit n-1, folding into (best,
// arg).  Rotating left by k is the translation with code code0 + k * nz.
template <bool TRACK>
__device__ __forceinline__ void ring64_eval(uint64_t w, uint64_t starts, uint32_t L, uint32_t n, uint64_t full,
                                            uint32_t code0, uint32_t nz, uint64_t &best, uint32_t &arg) {
    if (L == 0 || L >= n) {      // all ones / all zeros: every rotation is w
        if (w < best) {
            best = w;
            if constexpr (TRACK) arg = code0;
        }
        return;
    }
    while (starts) {
        const uint32_t i = static_cast<uint32_t>(__builtin_ctzll(starts));
        starts &= starts - 1;
        uint32_t top = i + L - 1;             // the run's highest bit
        if (top >= n) top -= n;
        const uint32_t k = n - 1 - top;       // rotate it to bit n-1
        const uint64_t v = rotl_n(w, k, n, full);
        if (v < best) {
            best = v;
            if constexpr (TRACK) arg = code0 + k * nz;
        }
    }
}

// Run starts of the reversed word: a run of L zeros starting at i in w
// starts at n - L - i (mod n) in the bit reversal of w.
__device__ __forceinline__ uint64_t ring64_mirror(uint64_t starts, uint32_t L, uint32_t n, uint64_t full) {
    if (L == 0 || L >= n) return starts;
    const uint64_t r = __builtin_bitreverse64(starts) >> (64u - n);   // i -> n-1-i
    return rotr_n(r, L - 1, n, full);
}

// Orbit minimum; with TRACK also the code of the first element reaching it.
template <typename W, int KIND, bool TRACK>
__device__ __forceinline__ W orbit_min(const PlanDev &P, W s, uint32_t &code) {
    W best = s;
    uint32_t arg = 0;
    if constexpr (KIND == kOrbitRing64) {
        const uint64_t full = P.full;
        const uint32_t n = P.n_sites;
        const uint32_t nz = P.pair_flip ? 2u : 1u;
        const uint64_t w = static_cast<uint64_t>(s);
        uint64_t b64 = w;        // s itself is the identity image (code 0)
        if (P.n_cosets == 2 && P.cosets[1].kind == kCosetReverse && P.cosets[1].flip == 0) {
            // dihedral group (x spin flip): the reversed word's runs mirror
            // w's, and with the flip only the longer of the zero and one runs
            // can put the minimum's leading zeros on top
            uint32_t Lz, Lo = 0;
            const uint64_t sz = ring64_runs(w, n, full, Lz);
            uint64_t so = 0;
            if (P.pair_flip) so = ring64_runs(w ^ full, n, full, Lo);
            const uint64_t rw = __builtin_bitreverse64(w) >> (64u - n);
            if (Lz >= Lo) {
                ring64_eval<TRACK>(w, sz, Lz, n, full, 0, nz, b64, arg);
                ring64_eval<TRACK>(rw, ring64_mirror(sz, Lz, n, full), Lz, n, full, n * nz, nz, b64, arg);
            }
            if (P.pair_flip && Lo >= Lz) {
                ring64_eval<TRACK>(w ^ full, so, Lo, n, full, 1, nz, b64, arg);
                ring64_eval<TRACK>(rw ^ full, ring64_mirror(so, Lo, n, full), Lo, n, full, n * nz + 1, nz, b64,
                                   arg);
            }
        } else {
            for (uint32_t p0 = 0; p0 < P.n_cosets; ++p0) {
                const uint32_t p = uni(p0);
                const uint64_t u = static_cast<uint64_t>(apply_coset<W>(P.cosets[p], s, P));
                uint32_t L;
                uint64_t st = ring64_runs(u, n, full, L);
                ring64_eval<TRACK>(u, st, L, n, full, p * n * nz, nz, b64, arg);
                if (P.pair_flip) {
                    st = ring64_runs(u ^ full, n, full, L);
                    ring64_eval<TRACK>(u ^ full, st, L, n, full, p * n * nz + 1, nz, b64, arg);
                }
            }
        }
        best = static_cast<W>(b64);
    } else if constexpr (!TRACK && KIND == kOrbitRing32) {
        // plain min, two images per rotation with spin inversion
        const W full = static_cast<W>(P.full);
        const uint32_t n = P.n_sites;
        for (uint32_t p0 = 0; p0 < P.n_cosets; ++p0) {
            const CosetRep c = P.cosets[uni(p0)];
            const W u = apply_coset<W>(c, s, P);
            const uint64_t uu = static_cast<uint64_t>(u) | (static_cast<uint64_t>(u) << n);
            const uint32_t lo = static_cast<uint32_t>(uu), hi = static_cast<uint32_t>(uu >> 32);
            if (P.pair_flip) {
                for (uint32_t t = 0; t < n; ++t) {
                    const W v = static_cast<W>(__builtin_amdgcn_alignbit(hi, lo, t)) & full;
                    best = min(best, min(v, static_cast<W>(v ^ full)));
                }
            } else {
                for (uint32_t t = 0; t < n; ++t) {
                    const W v = static_cast<W>(__builtin_amdgcn_alignbit(hi, lo, t)) & full;
                    best = min(best, v);
                }
            }
        }
    } else {
        for_each_image<W, KIND>(P, s, [&](W v, uint32_t c) {
            if constexpr (TRACK) {
                if (v < best) { best = v; arg = c; }
            } else {
                best = v < best ? v : best;
            }
            return true;
        });
    }
    code = arg;
    return best;
}

// Pruned orbit minimum on an lx-by-ly torus (lx <= 6, ly >= 2).
//
// The images p(s) = p(r) ^ pi_p(f) of the coset representatives are formed
// from the row's images p(r) (pr[]) and the flip images pi_p(f) (cf[p * cstride]).
// Pass 1a walks every coset p and y-shift b: the top two rows of
// tau_{0,b}(p(s)) index the pair table, whose entry holds, for the pair and
// for its spin-flipped partner, the smallest value the two rows take over
// all x-shifts (the key) and the x-shift reaching it.  The minimum image has
// the smallest key, so pass 1b marks the (p, b, f) that reach the smallest
// key in a 128-bit mask, and pass 2 evaluates only those candidates in full
// at the x-shift the table names (at every x-shift when several shifts tie
// on the two rows).  LX, LY, NZ are the layout and |Z| when known at compile
// time (0: read from the plan).
//   lut   packed pair table in LDS: entry(q) | entry(q ^ all-ones) << 16,
//         entry = key << 4 | ambiguous << 3 | argmin_a;
//   lcol  col_ge masks in LDS.
constexpr uint32_t kTorusMaxCosets = kTorusCosetSlots;

template <typename W, bool TRACK, uint32_t LX, uint32_t LY, uint32_t NZ>
__device__ __forceinline__ W torus_orbit_min(const PlanDev &P, const W *pr, const uint64_t *cf, uint32_t cstride,
                                             const uint32_t *lut, const uint64_t *lcol, uint32_t &code) {
    const uint32_t L = LX ? LX : P.lx, Ly = LY ? LY : P.ly;
    const uint32_t nz = NZ ? NZ : (P.pair_flip ? 2u : 1u);
    const uint32_t rm = (1u << L) - 1u, m2 = (1u << (2 * L)) - 1u;
    // the compile-time shapes are built for the full point group only
    const uint32_t ncos = LX ? kTorusMaxCosets : P.n_cosets;
    const W full = static_cast<W>(P.full);
    // bits [sh, sh + 32) of u shifted up by 2: an index times 4 is the byte
    // offset of its 4-byte entry
    auto x4 = [&](W u, uint32_t sh) -> uint32_t {
        return sh >= 2 ? static_cast<uint32_t>(u >> (sh - 2)) : static_cast<uint32_t>(u) << (2 - sh);
    };
    // byte offset of the entry of the top two rows of tau_{0,b}(u): rows
    // ly-1-b and ly-2-b (mod ly)
    auto pair_of = [&](W u, uint32_t b) -> uint32_t {
        const uint32_t ty = Ly - 1 - b;
        if (ty >= 1) return x4(u, L * (ty - 1)) & (m2 << 2);
        return ((static_cast<uint32_t>(u) & rm) << (L + 2)) | (x4(u, L * (Ly - 1)) & (rm << 2));
    };
    auto entry = [&](uint32_t off) -> uint32_t {
        return *reinterpret_cast<const uint32_t *>(reinterpret_cast<const unsigned char *>(lut) + off);
    };
    // image p(s) = p(r) ^ pi_p(f) of coset p: fixed p (unrolled loops), or a
    // p that differs between lanes
#define LS_IMG(p) (pr[p] ^ static_cast<W>(cf[(p) * cstride]))
    using u16x2 = unsigned short __attribute__((ext_vector_type(2)));
    W rmin = static_cast<W>(~static_cast<W>(0));
    uint32_t arg = 0;
    // pass 1a: the smallest entry of every coset (both flip entries of a
    // table word folded with one packed minimum), then the smallest key
    uint32_t cmin[kTorusMaxCosets];
    uint32_t ball = 0xFFFFu;
    uint64_t cf_next = cf[0];
#pragma unroll
    for (uint32_t p = 0; p < kTorusMaxCosets; ++p) {
        cmin[p] = 0xFFFFu;
        if (p >= ncos) continue;
        u16x2 m = {0xFFFFu, 0xFFFFu};
        if constexpr (LY != 0) {
            // the next coset's flip image and all of this coset's table
            // reads in flight before the first minimum
            const W u = pr[p] ^ static_cast<W>(cf_next);
            if (p + 1 < kTorusMaxCosets) cf_next = cf[(p + 1) * cstride];
            uint32_t e[LY];
#pragma unroll
            for (uint32_t b = 0; b < LY; ++b) e[b] = entry(pair_of(u, b));
#pragma unroll
            for (uint32_t b = 0; b < LY; ++b) m = __builtin_elementwise_min(m, __builtin_bit_cast(u16x2, e[b]));
        } else {
            for (uint32_t b1 = 0; b1 < Ly; ++b1)
                m = __builtin_elementwise_min(m, __builtin_bit_cast(u16x2, entry(pair_of(LS_IMG(p), uni(b1)))));
        }
        cmin[p] = nz == 2 ? min(static_cast<uint32_t>(m.x), static_cast<uint32_t>(m.y))
                          : static_cast<uint32_t>(m.x);
        ball = min(ball, cmin[p]);
    }
    const uint32_t best = ball >> 4;
    // the cosets that reach the smallest key
    uint32_t cm = 0;
#pragma unroll
    for (uint32_t p = 0; p < kTorusMaxCosets; ++p) cm |= ((cmin[p] >> 4) == best ? 1u : 0u) << p;
    if constexpr (!TRACK) {
        // one mask bit per (coset, y-shift), and only the cosets that reach
        // the smallest key are scanned twice; the kernels that also track g*
        // do not have the registers for it and keep one bit per (coset,
        // y-shift, flip)
        // pass 1b and 2: in those cosets only (a loop per lane), the y-shifts
        // that reach it with either entry (the key fields of both entries are
        // compared at once against the pattern), and a full evaluation of the
        // images they give, with the coset image already at hand
        const uint32_t pat = (best << 4) | (best << 20);
        const uint32_t keys = nz == 2 ? 0xFFF0FFF0u : 0x0000FFF0u;
        while (cm) {
            const uint32_t p = static_cast<uint32_t>(__builtin_ctz(cm));
            cm &= cm - 1;
            W u = pr[0];
#pragma unroll
            for (uint32_t q = 1; q < kTorusMaxCosets; ++q) u = (q < ncos && p == q) ? pr[q] : u;
            u ^= static_cast<W>(cf[p * cstride]);
            uint64_t mb = 0;
            if constexpr (LY != 0) {
                uint32_t e[LY];
#pragma unroll
                for (uint32_t b = 0; b < LY; ++b) e[b] = entry(pair_of(u, b));
#pragma unroll
                for (uint32_t b = 0; b < LY; ++b) {
                    const uint32_t d = (e[b] ^ pat) & keys;
                    mb |= ((d & 0xFFFFu) == 0 || (nz == 2 && (d >> 16) == 0)) ? (1ull << b) : 0ull;
                }
            } else {
                for (uint32_t b1 = 0; b1 < Ly; ++b1) {
                    const uint32_t b = uni(b1);
                    const uint32_t d = (entry(pair_of(u, b)) ^ pat) & keys;
                    mb |= ((d & 0xFFFFu) == 0 || (nz == 2 && (d >> 16) == 0)) ? (1ull << b) : 0ull;
                }
            }
            while (mb) {
                const uint32_t b = static_cast<uint32_t>(__builtin_ctzll(mb));
                mb &= mb - 1;
                W v0 = u;
                if (b) v0 = ((v0 << (L * b)) | (v0 >> (P.n_sites - L * b))) & full;
                // low entry: v0's top two rows; high entry: those of v0 ^ full
                const uint32_t e2 = entry(x4(v0, L * (Ly - 2)) & (m2 << 2));
#pragma unroll
                for (uint32_t f = 0; f < 2; ++f) {
                    if (f >= nz) break;
                    const uint32_t e = f ? (e2 >> 16) : (e2 & 0xFFFFu);
                    if ((e >> 4) != best) continue;
                    W v = f ? static_cast<W>(v0 ^ full) : v0;
                    const uint32_t base = (p * P.n_trans + L * b) * nz + f;
                    if (e & 8u) {
                        for (uint32_t a = 0; a < L; ++a) {
                            if (v < rmin) { rmin = v; arg = base + a * nz; }
                            if (a + 1 < L) v = xrot<W>(v, P);
                        }
                    } else {
                        const uint32_t a = e & 7u;
                        W c = v;
                        if (a) {
                            const W ma = static_cast<W>(lcol[a]);
                            c = ((v << a) & ma) | ((v >> (L - a)) & ~ma & full);
                        }
                        if (c < rmin) { rmin = c; arg = base + a * nz; }
                    }
                }
            }
        }
    } else {
        // pass 1b: in those cosets only, which (p, b, f) reach it
        // (bit (p*ly + b)*nz + f)
        uint64_t M0 = 0, M1 = 0;
        while (cm) {
            const uint32_t p = static_cast<uint32_t>(__builtin_ctz(cm));
            cm &= cm - 1;
            W u = pr[0];
#pragma unroll
            for (uint32_t q = 1; q < kTorusMaxCosets; ++q) u = (q < ncos && p == q) ? pr[q] : u;
            u ^= static_cast<W>(cf[p * cstride]);
#pragma unroll
            for (uint32_t b0 = 0; b0 < (LY ? LY : 1u); ++b0) {
                for (uint32_t b1 = 0; b1 < (LY ? 1u : Ly); ++b1) {
                    const uint32_t b = LY ? b0 : uni(b1);
                    const uint32_t e = entry(pair_of(u, b));
                    const uint32_t idx = (p * Ly + b) * nz;
                    const uint64_t hit = (((e >> 4) & 0xFFFu) == best ? 1ull : 0ull) |
                                         ((nz == 2 && (e >> 20) == best) ? 2ull : 0ull);
                    if (idx < 63) M0 |= hit << idx;
                    else if (idx == 63) { M0 |= hit << 63; M1 |= hit >> 1; }
                    else M1 |= hit << (idx - 64);
                }
            }
        }
        while (M0 | M1) {
            uint32_t idx;
            if (M0) {
                idx = static_cast<uint32_t>(__builtin_ctzll(M0));
                M0 &= M0 - 1;
            } else {
                idx = 64u + static_cast<uint32_t>(__builtin_ctzll(M1));
                M1 &= M1 - 1;
            }
            const uint32_t f = idx % nz, pb = idx / nz;
            const uint32_t b = pb % Ly, p = pb / Ly;
            W v = pr[0];
#pragma unroll
            for (uint32_t q = 1; q < kTorusMaxCosets; ++q) v = (q < ncos && p == q) ? pr[q] : v;
            v ^= static_cast<W>(cf[p * cstride]);
            if (b) v = ((v << (L * b)) | (v >> (P.n_sites - L * b))) & full;
            if (f) v ^= full;
            const uint32_t e = entry(x4(v, L * (Ly - 2)) & (m2 << 2)) & 0xFFFFu;
            const uint32_t base = (p * P.n_trans + L * b) * nz + f;
            if (e & 8u) {
                for (uint32_t a = 0; a < L; ++a) {
                    if (v < rmin) { rmin = v; arg = base + a * nz; }
                    if (a + 1 < L) v = xrot<W>(v, P);
                }
            } else {
                const uint32_t a = e & 7u;
                W c = v;
                if (a) {
                    const W ma = static_cast<W>(lcol[a]);
                    c = ((v << a) & ma) | ((v >> (L - a)) & ~ma & full);
                }
                if (c < rmin) { rmin = c; arg = base + a * nz; }
            }
        }
    }
    if constexpr (TRACK) code = arg;
    else code = 0;
    return rmin;
#undef LS_IMG
}

// Binomial coefficient table [65][65] in device memory.
__device__ __forceinline__ uint64_t binom(const uint64_t *t, uint32_t n, uint32_t k) {
    return t[n * 65u + k];
}

// Position of s among the weight-w bitstrings in increasing order.
__device__ __forceinline__ uint64_t colex_rank(uint64_t s, const uint64_t *tab) {
    uint64_t r = 0;
    uint32_t k = 1;
    while (s) {
        const uint32_t p = static_cast<uint32_t>(__builtin_ctzll(s));
        r += binom(tab, p, k);
        ++k;
        s &= s - 1;
    }
    return r;
}

// Home slot of a key in a hash index of 2^(64 - shift) slots: Fibonacci
// hashing (the top bits of key * 2^64/phi), so every key bit moves the slot.
__host__ __device__ __forceinline__ uint64_t slot_of(uint64_t key, uint32_t shift) {
    return (key * 0x9E3779B97F4A7C15ULL) >> shift;
}

// Hash index: linear probing from the key's slot; the table always has free
// slots, so every probe sequence ends.  One 16-byte load per probe.
__device__ __forceinline__ int64_t lookup_hash(const SearchDev &S, uint64_t key, uint32_t &stab) {
    uint64_t s = slot_of(key, S.hash_shift);
    for (;;) {
        const uint4 e = *reinterpret_cast<const uint4 *>(S.table + s);
        const uint64_t k = static_cast<uint64_t>(e.x) | (static_cast<uint64_t>(e.y) << 32);
        if (k == key) {
            stab = e.w;
            return static_cast<int64_t>(e.z);
        }
        if (k == kEmptyKey) return -1;
        s = (s + 1) & S.hash_mask;
    }
}

// Binary search for key among reps[lo, end) (one bucket of the sorted array).
__device__ __forceinline__ int64_t search_bucket(const uint64_t *reps, uint32_t lo, uint32_t end, uint64_t key) {
    uint32_t hi = end;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (reps[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < end && reps[lo] == key) ? static_cast<int64_t>(lo) : -1;
}

// stateToIndex: hash index, or bucket of the key's high bits then binary
// search, or the colex rank (U(1) without lattice symmetry).
__device__ __forceinline__ int64_t lookup_index(const SearchDev &S, uint64_t key) {
    if (S.mode == kLookupHash) {
        if (key < S.kmin || key > S.kmax) return -1;
        uint32_t st;
        return lookup_hash(S, key, st);
    }
    if (S.mode == kLookupIdentity)
        return (S.n_sites == 64 || (key >> S.n_sites) == 0) ? static_cast<int64_t>(key) : -1;
    if (S.mode == kLookupRank) {
        if ((S.n_sites < 64 && (key >> S.n_sites) != 0) || __builtin_popcountll(key) != S.weight) return -1;
        return static_cast<int64_t>(colex_rank(key, S.binom));
    }
    if (key < S.kmin || key > S.kmax) return -1;
    const uint64_t b = (key - S.kmin) >> S.shift;
    return search_bucket(S.reps, S.buckets[b], S.buckets[b + 1], key);
}

// The bucket search with the bucket table staged in LDS (lb, S.n_bkt
// entries): the bucket's bounds are LDS reads, only the search inside the
// bucket reads reps.
__device__ __forceinline__ int64_t lookup_staged(const SearchDev &S, const uint32_t *lb, uint64_t key) {
    if (key < S.kmin || key > S.kmax) return -1;
    const uint32_t b = static_cast<uint32_t>((key - S.kmin) >> S.shift);
    return search_bucket(S.reps, lb[b], lb[b + 1], key);
}

// Index and stabilizer size of a key (the hash index holds both in one slot).
__device__ __forceinline__ int64_t lookup_index_stab(const SearchDev &S, uint64_t key, const uint16_t *stab_arr,
                                                     uint32_t &stab) {
    if (S.mode == kLookupHash) {
        if (key < S.kmin || key > S.kmax) return -1;
        return lookup_hash(S, key, stab);
    }
    const int64_t j = lookup_index(S, key);
    if (j >= 0) stab = stab_arr[j];
    return j;
}

}  // namespace ls
