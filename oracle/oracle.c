/*
 * Oracle for the symmetry-adapted exact-diagonalization path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * Plain, slow and deliberately literal:
 *   - a group element is applied by a loop over the N bits;
 *   - the representative of a state is the minimum over its whole orbit,
 *     found by trying every group element (brute-force orbit search; the
 *     paper defers the "condition" of Section 5.2 to the literature, and
 *     the reading adopted is "keep s iff s is the minimum of its orbit and
 *     the sector's projector does not annihilate it");
 *   - the basis is every weight-w bitstring in increasing order (Gosper's
 *     next-combination step), filtered by that condition (Section 5.2);
 *   - stateToIndex (Section 5.3) is a hash map from representative to
 *     position, on purpose unlike a sorted search;
 *   - the product is the transposed, column-by-column form of Section 5.3
 *     (y = 0, then for each column scatter H_ij x_j into y), run serially;
 *   - getRow of Section 5.3 is also provided, for checks of single rows.
 *
 * Matrix elements in the symmetry-adapted basis |r~> = P|r>/||P|r>||,
 * P = (1/|G|) sum_g conj(chi(g)) U_g (the paper's Section 2.1 shows the
 * reduction; the formulas are derived from the projector):
 *   column form: H|r_j~> has component on |r_i~>
 *       sum_t a_t(r_j) conj(chi(g*_s)) sqrt(stab(r_i)/stab(r_j)),
 *   row form:    <r_i~|H|r_j~> = sum_t conj(a_t(r_i)) chi(g*_s)
 *                                  sqrt(stab(r_j)/stab(r_i)),
 * with s = r ^ flip_t, a_t(r) = c_t (-1)^popcount(r & sign_t), g* the
 * lowest-index element with g*(s) = rep(s).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n_sites;
    int32_t weight;       /* -1: no fixed Hamming weight */
    int32_t n_elements;
    int32_t pad_;
    const uint16_t *perm; /* [nG][N] */
    const uint8_t *flip;  /* [nG] */
    const double *chi;    /* [nG][2] */
} orc_sector;

typedef struct {
    double re, im;
    uint64_t sel, val, flip, sign;
} orc_term;

static uint64_t full_mask(int n) { return n >= 64 ? ~0ULL : ((1ULL << n) - 1ULL); }

static int popcount64(uint64_t v) {
    int c = 0;
    while (v) { c += (int)(v & 1ULL); v >>= 1; }
    return c;
}

/* g.s: bit i of s moves to bit perm[g][i]; then all N bits inverted if flip[g]. */
uint64_t orc_apply(const orc_sector *S, int g, uint64_t s) {
    const int n = S->n_sites;
    uint64_t out = 0;
    for (int i = 0; i < n; ++i)
        if ((s >> i) & 1ULL) out |= 1ULL << S->perm[(size_t)g * n + i];
    if (S->flip[g]) out ^= full_mask(n);
    return out;
}

/* Orbit minimum; *gstar = lowest index g with g.s equal to it. */
static uint64_t orbit_min(const orc_sector *S, uint64_t s, int *gstar) {
    uint64_t best = 0;
    int arg = -1;
    for (int g = 0; g < S->n_elements; ++g) {
        uint64_t v = orc_apply(S, g, s);
        if (arg < 0 || v < best) { best = v; arg = g; }
    }
    if (gstar) *gstar = arg;
    return best;
}

/* Stabilizer size of r and whether P|r> != 0: Re sum_{g.r=r} conj(chi(g)) > 1/2. */
static int sector_test(const orc_sector *S, uint64_t r, int *stab) {
    double re = 0.0;
    int cnt = 0;
    for (int g = 0; g < S->n_elements; ++g) {
        if (orc_apply(S, g, r) == r) {
            ++cnt;
            re += S->chi[2 * g];  /* Re conj(chi) = Re chi */
        }
    }
    if (stab) *stab = cnt;
    return re > 0.5;
}

static int weight_ok(const orc_sector *S, uint64_t s) {
    if (S->n_sites < 64 && (s >> S->n_sites) != 0) return 0;
    return S->weight < 0 || popcount64(s) == S->weight;
}

/* Per state: representative, character of g* (0 if not in the sector),
 * norm sqrt(stab/|G|) (0 if not in the sector or of the wrong weight).
 * A state with bits at or above N is returned unchanged with chi = norm = 0. */
void orc_state_info(const orc_sector *S, int64_t n, const uint64_t *states,
                    uint64_t *reps, double *chi, double *norm) {
    for (int64_t k = 0; k < n; ++k) {
        uint64_t s = states[k];
        if (S->n_sites < 64 && (s >> S->n_sites) != 0) {
            reps[k] = s; chi[2 * k] = 0.0; chi[2 * k + 1] = 0.0; norm[k] = 0.0;
            continue;
        }
        int gs;
        uint64_t r = orbit_min(S, s, &gs);
        int stab = 0;
        int in = weight_ok(S, s) && sector_test(S, r, &stab);
        reps[k] = r;
        if (in) {
            chi[2 * k] = S->chi[2 * gs];
            chi[2 * k + 1] = S->chi[2 * gs + 1];
            norm[k] = sqrt((double)stab / (double)S->n_elements);
        } else {
            chi[2 * k] = 0.0; chi[2 * k + 1] = 0.0; norm[k] = 0.0;
        }
    }
}

/* Gosper's step: the next larger integer with the same number of set bits. */
static uint64_t next_combination(uint64_t x) {
    uint64_t c = x & (~x + 1ULL);
    uint64_t r = x + c;
    return (((r ^ x) >> 2) / c) | r;
}

static int is_member(const orc_sector *S, uint64_t s, int *stab) {
    for (int g = 0; g < S->n_elements; ++g)
        if (orc_apply(S, g, s) < s) return 0;   /* not the orbit minimum */
    return sector_test(S, s, stab);
}

/* Enumerate the basis in increasing order.  Writes at most cap entries
 * (reps/stab may be NULL for counting) and returns the full count. */
int64_t orc_enumerate(const orc_sector *S, uint64_t *reps, uint16_t *stab, int64_t cap) {
    const int n = S->n_sites;
    int64_t count = 0;
    if (S->weight >= 0) {
        if (S->weight > n) return 0;
        uint64_t s = S->weight == 0 ? 0ULL : full_mask(S->weight);
        uint64_t last = S->weight == 0 ? 0ULL : (full_mask(S->weight) << (n - S->weight));
        for (;;) {
            int st;
            if (is_member(S, s, &st)) {
                if (count < cap) {
                    if (reps) reps[count] = s;
                    if (stab) stab[count] = (uint16_t)st;
                }
                ++count;
            }
            if (s == last) break;
            s = next_combination(s);
        }
    } else {
        const uint64_t end = full_mask(n);
        for (uint64_t s = 0;; ++s) {
            int st;
            if (is_member(S, s, &st)) {
                if (count < cap) {
                    if (reps) reps[count] = s;
                    if (stab) stab[count] = (uint16_t)st;
                }
                ++count;
            }
            if (s == end) break;
        }
    }
    return count;
}

/* ---- stateToIndex as an open-addressing hash map -------------------------------- */

typedef struct {
    uint64_t cap_mask;
    uint64_t *keys;
    int64_t *vals;   /* -1 = empty */
} orc_index;

static uint64_t mix64(uint64_t x) {
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
    return x ^ (x >> 31);
}

void *orc_index_new(const uint64_t *reps, int64_t d) {
    orc_index *h = (orc_index *)calloc(1, sizeof(orc_index));
    uint64_t cap = 16;
    while (cap < (uint64_t)(2 * d + 1)) cap <<= 1;
    h->cap_mask = cap - 1;
    h->keys = (uint64_t *)calloc(cap, sizeof(uint64_t));
    h->vals = (int64_t *)malloc(cap * sizeof(int64_t));
    for (uint64_t i = 0; i < cap; ++i) h->vals[i] = -1;
    for (int64_t i = 0; i < d; ++i) {
        uint64_t p = mix64(reps[i]) & h->cap_mask;
        while (h->vals[p] >= 0) p = (p + 1) & h->cap_mask;
        h->keys[p] = reps[i];
        h->vals[p] = i;
    }
    return h;
}

int64_t orc_index_get(const void *hp, uint64_t key) {
    const orc_index *h = (const orc_index *)hp;
    uint64_t p = mix64(key) & h->cap_mask;
    while (h->vals[p] >= 0) {
        if (h->keys[p] == key) return h->vals[p];
        p = (p + 1) & h->cap_mask;
    }
    return -1;
}

void orc_index_free(void *hp) {
    orc_index *h = (orc_index *)hp;
    if (!h) return;
    free(h->keys); free(h->vals); free(h);
}

void orc_index_lookup(const uint64_t *reps, int64_t d, int64_t n, const uint64_t *keys, int64_t *out) {
    void *h = orc_index_new(reps, d);
    for (int64_t k = 0; k < n; ++k) out[k] = orc_index_get(h, keys[k]);
    orc_index_free(h);
}

/* ---- the product ---------------------------------------------------------------- */

/* Transposed (column-by-column) product, serial.  x, y: complex [d][nrhs][2].
 * Columns are processed for j in [j_begin, j_end); y is not cleared here
 * (the caller zeroes it), so a column sample accumulates partial results.
 * Returns the number of element applications (diagonal and off-diagonal
 * terms that act on a column), or -1 if a neighbour's representative is in
 * the sector but missing from the index (an inconsistent basis). */
int64_t orc_matvec_columns(const orc_sector *S, const uint64_t *reps, const uint16_t *stab, int64_t d,
                           const orc_term *terms, int32_t n_terms, int32_t nrhs,
                           const double *x, double *y, int64_t j_begin, int64_t j_end) {
    void *h = orc_index_new(reps, d);
    int64_t applied = 0;
    if (j_end > d) j_end = d;
    for (int64_t j = j_begin; j < j_end; ++j) {
        const uint64_t rj = reps[j];
        for (int t = 0; t < n_terms; ++t) {
            const orc_term *T = &terms[t];
            if ((rj & T->sel) != T->val) continue;
            ++applied;
            const uint64_t s = rj ^ T->flip;
            const double sg = (popcount64(rj & T->sign) & 1) ? -1.0 : 1.0;
            const double a_re = T->re * sg, a_im = T->im * sg;
            int gs;
            const uint64_t r = orbit_min(S, s, &gs);
            const int64_t i = orc_index_get(h, r);
            if (i < 0) {
                if (sector_test(S, r, NULL)) { orc_index_free(h); return -1; }
                continue;   /* the projector annihilates this orbit */
            }
            /* a * conj(chi(g*)) * sqrt(stab_i / stab_j) */
            const double c_re = S->chi[2 * gs], c_im = -S->chi[2 * gs + 1];
            const double ratio = sqrt((double)stab[i] / (double)stab[j]);
            const double f_re = (a_re * c_re - a_im * c_im) * ratio;
            const double f_im = (a_re * c_im + a_im * c_re) * ratio;
            for (int q = 0; q < nrhs; ++q) {
                const double xr = x[2 * (j * nrhs + q)], xi = x[2 * (j * nrhs + q) + 1];
                y[2 * (i * nrhs + q)] += f_re * xr - f_im * xi;
                y[2 * (i * nrhs + q) + 1] += f_re * xi + f_im * xr;
            }
        }
    }
    orc_index_free(h);
    return applied;
}

/* getRow: the non-zero elements <r~|H|rep_k~> of the row of representative r
 * (one entry per acting term, not merged).  r must be in the sector.
 * Returns the number of entries written (at most cap), or -1 if r is not a
 * representative in the sector. */
int32_t orc_get_row(const orc_sector *S, uint64_t r, const orc_term *terms, int32_t n_terms,
                    uint64_t *out_reps, double *out_coef, int32_t cap) {
    int gr, stab_r;
    if (orbit_min(S, r, &gr) != r || !weight_ok(S, r) || !sector_test(S, r, &stab_r)) return -1;
    int32_t cnt = 0;
    for (int t = 0; t < n_terms; ++t) {
        const orc_term *T = &terms[t];
        if ((r & T->sel) != T->val) continue;
        const uint64_t s = r ^ T->flip;
        const double sg = (popcount64(r & T->sign) & 1) ? -1.0 : 1.0;
        const double a_re = T->re * sg, a_im = -T->im * sg;   /* conj(a) */
        int gs, stab_s;
        const uint64_t rs = orbit_min(S, s, &gs);
        if (!sector_test(S, rs, &stab_s)) continue;
        const double c_re = S->chi[2 * gs], c_im = S->chi[2 * gs + 1];  /* chi(g*) */
        const double ratio = sqrt((double)stab_s / (double)stab_r);
        if (cnt < cap) {
            out_reps[cnt] = rs;
            out_coef[2 * cnt] = (a_re * c_re - a_im * c_im) * ratio;
            out_coef[2 * cnt + 1] = (a_re * c_im + a_im * c_re) * ratio;
        }
        ++cnt;
    }
    return cnt;
}
