// Basis construction (Section 5.2), state_info and stateToIndex kernels.
//
// Enumeration: the candidates are all weight-w bitstrings in increasing
// order (colex rank 0 .. C(N,w)-1), or 0 .. 2^N-1 without U(1).  The paper
// splits this range into chunks, filters each chunk and then places the
// survivors with a histogram -> cumulative sum -> offsets scheme (Section
// 5.1 "Block to hashed", Section 5.2).  On one GPU the same scheme becomes
// an order-preserving stream compaction:
//   pass 1  every lane filters 64 consecutive candidates (Gosper's
//           next-combination step between them) and keeps a 64-bit mark
//           word; a workgroup reduction gives per-chunk counts;
//   scan    an exclusive scan of the chunk counts gives chunk offsets;
//   pass 2  a workgroup scan of the lanes' mark popcounts gives each lane's
//           offset; the lane regenerates its candidates and writes the
//           marked ones.  No atomics; the output is sorted by construction.
// The "condition" kept by the filter: s is the minimum of its orbit, and P
// does not annihilate it (every stabilizer element has character 1).

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <string>

#include "orbit.hpp"

namespace ls {

namespace {

constexpr int kBlock = 256;
constexpr int kCandPerLane = 64;

__device__ uint64_t unrank_colex(uint64_t rank, uint32_t n, int32_t w, const uint64_t *tab) {
    uint64_t s = 0;
    uint32_t k = static_cast<uint32_t>(w);
    for (int p = static_cast<int>(n) - 1; p >= 0 && k > 0; --p) {
        const uint64_t c = binom(tab, static_cast<uint32_t>(p), k);
        if (c <= rank) {
            s |= 1ULL << p;
            rank -= c;
            --k;
        }
    }
    return s;
}

template <typename W>
__device__ __forceinline__ W next_combination(W x) {
    const W c = x & (~x + 1);
    const W r = x + c;
    const int z = sizeof(W) == 4 ? __builtin_ctz(static_cast<uint32_t>(x))
                                 : __builtin_ctzll(static_cast<uint64_t>(x));
    return (((r ^ x) >> 2) >> z) | r;
}

// Membership of cnt consecutive candidates s, next(s), ...: s is kept iff no
// group image is smaller and every image equal to s has chi == 1.  hit(q)
// is called for every kept candidate q.
//
// Most candidates are rejected after one or two images, while a member (about
// one candidate in |G|) needs every image.  A loop over candidates with the
// group walk inside would run each wave at the pace of its slowest lane for
// every candidate; here one iteration checks one image (with its spin-flipped
// partner) of the lane's current candidate, and a lane moves on to its next
// candidate as soon as the current one is decided, so a wave's time is the
// largest per-lane total over the run rather than the sum of per-candidate
// maxima.  Group order as in for_each_image: coset p, y-shift b, x-shift a.
template <typename W, int KIND, typename Hit>
__device__ __forceinline__ void walk_members(const PlanDev &P, W s, uint32_t cnt, bool gosper, Hit &&hit) {
    const W full = static_cast<W>(P.full);
    const bool pf = P.pair_flip != 0;
    const uint32_t nz = pf ? 2u : 1u;
    const uint32_t n = P.n_sites, lx = P.lx, ly = P.ly, nc = P.n_cosets, nt = P.n_trans;
    uint32_t q = 0, a = 0, b = 0, p = 0;
    // cosets[0] is the identity: the walk of every candidate starts at s
    W ub = s, v = s;
    uint32_t lo = 0, hi = 0;   // ring32: the coset image doubled into 64 bits
    if constexpr (KIND == kOrbitRing32) {
        const uint64_t uu = static_cast<uint64_t>(s) | (static_cast<uint64_t>(s) << n);
        lo = static_cast<uint32_t>(uu);
        hi = static_cast<uint32_t>(uu >> 32);
    }
    for (;;) {
        const W vf = static_cast<W>(v ^ full);
        bool out = v < s || (pf && vf < s);
        if (!out && (v == s || (pf && vf == s))) {
            uint32_t code;
            if constexpr (KIND == kOrbitRing32) code = (p * n + (a == 0 ? 0u : n - a)) * nz;
            else code = (p * nt + a + lx * b) * nz;
            if (v == s && !chi_is_one(P, code)) out = true;
            if (pf && vf == s && !chi_is_one(P, code + 1)) out = true;
        }
        bool end = false;
        if constexpr (KIND == kOrbitRing32) {
            // a counts right rotations here
            if (++a < n) {
                v = static_cast<W>(__builtin_amdgcn_alignbit(hi, lo, a)) & full;
            } else {
                a = 0;
                if (++p < nc) {
                    const W u = apply_coset<W>(P.cosets[p], s, P);
                    const uint64_t uu = static_cast<uint64_t>(u) | (static_cast<uint64_t>(u) << n);
                    lo = static_cast<uint32_t>(uu);
                    hi = static_cast<uint32_t>(uu >> 32);
                    v = u;
                } else {
                    end = true;
                }
            }
        } else {
            if (++a < lx) {
                v = xrot<W>(v, P);
            } else {
                a = 0;
                if (++b < ly) {
                    ub = yrot<W>(ub, P);
                    v = ub;
                } else {
                    b = 0;
                    if (++p < nc) {
                        ub = apply_coset<W>(P.cosets[p], s, P);
                        v = ub;
                    } else {
                        end = true;
                    }
                }
            }
        }
        if (out || end) {
            if (!out) hit(q);
            if (++q >= cnt) break;
            if (gosper) s = next_combination<W>(s);
            else s = static_cast<W>(s + 1);
            a = b = p = 0;
            ub = v = s;
            if constexpr (KIND == kOrbitRing32) {
                const uint64_t uu = static_cast<uint64_t>(s) | (static_cast<uint64_t>(s) << n);
                lo = static_cast<uint32_t>(uu);
                hi = static_cast<uint32_t>(uu >> 32);
            }
        }
    }
}

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const uint32_t r = sh[0];
    __syncthreads();
    return r;
}

// exclusive scan over the block
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const uint32_t add = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const uint32_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

struct EnumArgs {
    PlanDev plan;
    const uint64_t *binom;
    uint64_t total;        // candidates
    uint32_t n_sites;
    int32_t weight;
    uint64_t *marks;       // [lanes]
    uint32_t *counts;      // [blocks]
    const uint64_t *offsets;  // [blocks], pass 2
    uint64_t *reps;        // pass 2
};

template <typename W>
__device__ __forceinline__ W first_candidate(const EnumArgs &a, uint64_t start) {
    return a.weight >= 0 ? static_cast<W>(unrank_colex(start, a.n_sites, a.weight, a.binom))
                         : static_cast<W>(start);
}

template <typename W>
__device__ __forceinline__ W next_candidate(const EnumArgs &a, W s) {
    return a.weight >= 0 ? next_combination<W>(s) : static_cast<W>(s + 1);
}

template <typename W, int KIND>
__global__ void __launch_bounds__(kBlock) k_enum_mark(EnumArgs a) {
    __shared__ uint32_t sh[kBlock];
    const uint64_t lane = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const uint64_t start = lane * kCandPerLane;
    uint64_t mask = 0;
    if (start < a.total) {
        const uint32_t cnt = static_cast<uint32_t>(min<uint64_t>(kCandPerLane, a.total - start));
        walk_members<W, KIND>(a.plan, first_candidate<W>(a, start), cnt, a.weight >= 0,
                              [&](uint32_t q) { mask |= 1ULL << q; });
        a.marks[lane] = mask;
    }
    const uint32_t c = block_sum(static_cast<uint32_t>(__builtin_popcountll(mask)), sh);
    if (threadIdx.x == 0) a.counts[blockIdx.x] = c;
}

// Count-only pass over candidates [begin, end): each lane takes per_lane
// consecutive candidates; block totals are added into *acc (integer atomic
// adds: the total does not depend on their order), so launches on one stream
// over consecutive ranges accumulate.
template <typename W, int KIND>
__global__ void __launch_bounds__(kBlock) k_enum_count(EnumArgs a, uint64_t begin, uint64_t end, uint32_t per_lane,
                                                       unsigned long long *acc) {
    __shared__ uint32_t sh[kBlock];
    const uint64_t lane = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const uint64_t start = begin + lane * per_lane;
    uint32_t c = 0;
    if (start < end) {
        const uint32_t cnt = static_cast<uint32_t>(min<uint64_t>(per_lane, end - start));
        walk_members<W, KIND>(a.plan, first_candidate<W>(a, start), cnt, a.weight >= 0, [&](uint32_t) { ++c; });
    }
    const uint32_t t = block_sum(c, sh);
    if (threadIdx.x == 0 && t != 0) atomicAdd(acc, static_cast<unsigned long long>(t));
}

template <typename W>
__global__ void __launch_bounds__(kBlock) k_enum_write(EnumArgs a) {
    __shared__ uint32_t sh[kBlock];
    const uint64_t lane = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const uint64_t start = lane * kCandPerLane;
    uint64_t mask = start < a.total ? a.marks[lane] : 0ULL;
    const uint32_t local = block_exclusive_scan(static_cast<uint32_t>(__builtin_popcountll(mask)), sh);
    if (mask == 0) return;
    uint64_t pos = a.offsets[blockIdx.x] + local;
    const uint32_t cnt = static_cast<uint32_t>(min<uint64_t>(kCandPerLane, a.total - start));
    W s = first_candidate<W>(a, start);
    for (uint32_t q = 0; q < cnt; ++q) {
        if ((mask >> q) & 1ULL) a.reps[pos++] = static_cast<uint64_t>(s);
        if (q + 1 < cnt) s = next_candidate<W>(a, s);
    }
}

// Single-workgroup exclusive scan of n counts (n up to a few million).
__global__ void __launch_bounds__(1024) k_scan_counts(const uint32_t *counts, uint64_t n, uint64_t *offsets,
                                                      uint64_t *total) {
    __shared__ uint64_t sh[1024];
    const int t = threadIdx.x;
    const uint64_t per = (n + 1023) / 1024;
    const uint64_t b = min<uint64_t>(n, per * t), e = min<uint64_t>(n, b + per);
    uint64_t s = 0;
    for (uint64_t i = b; i < e; ++i) s += counts[i];
    sh[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t add = t >= off ? sh[t - off] : 0ull;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    uint64_t run = sh[t] - s;
    for (uint64_t i = b; i < e; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
    if (t == 1023) *total = sh[1023];
}

template <typename W, int KIND>
__global__ void __launch_bounds__(kBlock) k_stab(PlanDev P, const uint64_t *reps, uint64_t d, uint16_t *stab) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= d) return;
    const W r = static_cast<W>(reps[i]);
    uint32_t cnt = 0;
    for_each_image<W, KIND>(P, r, [&](W v, uint32_t) {
        cnt += v == r ? 1u : 0u;
        return true;
    });
    stab[i] = static_cast<uint16_t>(cnt);
}

// buckets[k] = first index whose key reaches bucket k (k = 0 .. nb; entry
// nb is d): one binary search per bucket, so empty stretches of the key
// range cost no more than full ones.
__global__ void __launch_bounds__(kBlock) k_buckets(const uint64_t *reps, uint64_t d, uint64_t kmin, uint32_t shift,
                                                    uint64_t nb, uint32_t *buckets) {
    const uint64_t k = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k > nb) return;
    uint64_t lo = 0, hi = d;
    if (k < nb) {
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (((reps[mid] - kmin) >> shift) < k) lo = mid + 1; else hi = mid;
        }
    } else {
        lo = d;
    }
    buckets[k] = static_cast<uint32_t>(lo);
}

// Hash index insert: keys are distinct, so each claims the first free slot
// of its probe sequence with a compare-and-swap; the table has more slots
// than keys, so every sequence ends.
__global__ void __launch_bounds__(kBlock) k_hash_insert(const uint64_t *reps, const uint16_t *stab, uint64_t d,
                                                        HashSlot *table, uint64_t mask, uint32_t shift) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= d) return;
    const uint64_t key = reps[i];
    uint64_t s = slot_of(key, shift);
    for (;;) {
        const unsigned long long prev =
            atomicCAS(reinterpret_cast<unsigned long long *>(&table[s].key), static_cast<unsigned long long>(kEmptyKey),
                      static_cast<unsigned long long>(key));
        if (prev == kEmptyKey) {
            table[s].idx = static_cast<uint32_t>(i);
            table[s].stab = stab[i];
            return;
        }
        s = (s + 1) & mask;
    }
}

// Test hook: the slot holding `key` gets `repl`, a key above every
// representative (lookups above kmax stop before probing), so the slot stays
// occupied, the probe sequences through it still end, and `key` misses.
// One thread; the walk is bounded by the table size.
__global__ void k_drop_key(HashSlot *table, uint64_t mask, uint32_t shift, uint64_t key, uint64_t repl) {
    uint64_t s = slot_of(key, shift);
    for (uint64_t n = 0; n <= mask; ++n) {
        const uint64_t k = table[s].key;
        if (k == key) {
            table[s].key = repl;
            return;
        }
        if (k == kEmptyKey) return;
        s = (s + 1) & mask;
    }
}

template <typename W, int KIND>
__global__ void __launch_bounds__(kBlock) k_state_info(PlanDev P, int32_t weight, uint64_t n, const uint64_t *states,
                                                       uint64_t *reps, double *chi, double *norm) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint64_t s64 = states[i];
    if (P.n_sites < 64 && (s64 >> P.n_sites) != 0) {
        reps[i] = s64;
        chi[2 * i] = 0.0;
        chi[2 * i + 1] = 0.0;
        norm[i] = 0.0;
        return;
    }
    const W s = static_cast<W>(s64);
    W best = s;
    uint32_t arg = 0, stab = 0;
    bool bad = false;
    for_each_image<W, KIND>(P, s, [&](W v, uint32_t code) {
        if (v < best) { best = v; arg = code; }
        if (v == s) {
            ++stab;
            bad = bad || !chi_is_one(P, code);
        }
        return true;
    });
    const bool in = !bad && (weight < 0 || __builtin_popcountll(s64) == weight);
    reps[i] = static_cast<uint64_t>(best);
    if (in) {
        const double2 c = P.chi[arg];
        chi[2 * i] = c.x;
        chi[2 * i + 1] = c.y;
        norm[i] = __dsqrt_rn(__ddiv_rn(static_cast<double>(stab), static_cast<double>(P.n_elements)));
    } else {
        chi[2 * i] = 0.0;
        chi[2 * i + 1] = 0.0;
        norm[i] = 0.0;
    }
}

__global__ void __launch_bounds__(kBlock) k_index_lookup(SearchDev S, uint64_t n, const uint64_t *keys, int64_t *out) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    out[i] = lookup_index(S, keys[i]);
}

template <typename W>
int orbit_kind(const GroupPlan &p) {
    return (sizeof(W) == 4 && p.ly == 1 && p.lx == p.n_sites && p.n_sites <= 32) ? kOrbitRing32 : kOrbitGeneric;
}

uint64_t grid_for(uint64_t n) { return (n + kBlock - 1) / kBlock; }

// Device scratch of a build, allocated and released in order on the build's
// stream: unlike hipFree, hipFreeAsync does not wait for the whole device,
// so a build beside running products (the serving loop) is not held up by
// them.
struct StreamBuf {
    void *p = nullptr;
    hipStream_t st;
    StreamBuf(size_t bytes, hipStream_t s) : st(s) { LS_HIP_CHECK(hipMallocAsync(&p, bytes, s)); }
    ~StreamBuf() {
        if (p) (void)hipFreeAsync(p, st);
    }
    StreamBuf(const StreamBuf &) = delete;
    StreamBuf &operator=(const StreamBuf &) = delete;
    template <class T>
    T *as() const {
        return static_cast<T *>(p);
    }
};

template <typename W>
void enumerate_impl(ls_basis *b, hipStream_t st, uint64_t total, uint64_t **out_reps, uint64_t *out_dim) {
    const GroupPlan &gp = b->plan;
    const uint64_t lanes = (total + kCandPerLane - 1) / kCandPerLane;
    const uint64_t blocks = grid_for(lanes);
    StreamBuf marks_b(std::max<uint64_t>(lanes, 1) * sizeof(uint64_t), st);
    StreamBuf counts_b(std::max<uint64_t>(blocks, 1) * sizeof(uint32_t), st);
    StreamBuf offsets_b(std::max<uint64_t>(blocks, 1) * sizeof(uint64_t), st);
    StreamBuf total_b(sizeof(uint64_t), st);
    uint64_t *marks = marks_b.as<uint64_t>(), *offsets = offsets_b.as<uint64_t>(), *d_total = total_b.as<uint64_t>();
    uint32_t *counts = counts_b.as<uint32_t>();
    EnumArgs a{};
    a.plan = b->plan_dev;
    a.binom = b->d_binom;
    a.total = total;
    a.n_sites = gp.n_sites;
    a.weight = b->weight;
    a.marks = marks;
    a.counts = counts;
    a.offsets = offsets;
    const int kind = orbit_kind<W>(gp);
    if (blocks > 0) {
        if (kind == kOrbitRing32)
            hipLaunchKernelGGL((k_enum_mark<W, kOrbitRing32>), dim3(blocks), dim3(kBlock), 0, st, a);
        else
            hipLaunchKernelGGL((k_enum_mark<W, kOrbitGeneric>), dim3(blocks), dim3(kBlock), 0, st, a);
        LS_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, counts, blocks, offsets, d_total);
        LS_HIP_CHECK(hipGetLastError());
    }
    uint64_t dim = 0;
    if (blocks > 0) {
        LS_HIP_CHECK(hipMemcpyAsync(&dim, d_total, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        LS_HIP_CHECK(hipStreamSynchronize(st));
    }
    uint64_t *reps = dev_alloc_n<uint64_t>(std::max<uint64_t>(dim, 1), st);
    a.reps = reps;
    hipError_t e = hipSuccess;
    if (dim > 0) {
        hipLaunchKernelGGL((k_enum_write<W>), dim3(blocks), dim3(kBlock), 0, st, a);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        dev_free(reps, st);
        LS_HIP_CHECK(e);
    }
    *out_reps = reps;
    *out_dim = dim;
}

template <typename W>
void stab_impl(ls_basis *b, hipStream_t st) {
    if (b->dim == 0) return;
    if (orbit_kind<W>(b->plan) == kOrbitRing32)
        hipLaunchKernelGGL((k_stab<W, kOrbitRing32>), dim3(grid_for(b->dim)), dim3(kBlock), 0, st, b->plan_dev,
                           b->d_reps, b->dim, b->d_stab);
    else
        hipLaunchKernelGGL((k_stab<W, kOrbitGeneric>), dim3(grid_for(b->dim)), dim3(kBlock), 0, st, b->plan_dev,
                           b->d_reps, b->dim, b->d_stab);
    LS_HIP_CHECK(hipGetLastError());
}

uint64_t host_binom(uint32_t n, uint32_t k) {
    if (k > n) return 0;
    uint64_t r = 1;
    for (uint32_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;   // exact: r*(n-k+i) divisible by i
    return r;
}

}  // namespace

// Binomial table and the compiled group in device memory (PlanDev).
// Slots of the hash index, a power of two: load factor at most 1/8 while the
// table fits 8 GiB, else 1/4 within 64 GiB, else 1/2 or 3/4 within 128 GiB;
// 0 above that.  A sparse table makes a second probe (a second dependent
// memory round trip) rare: load 1/2 -> 1/8 took the 6x6 product from 40.0 to
// 36.7 ms, load 0.4 -> 0.2 the 40-spin chain product from 442 to 421 ms, and
// load 0.75 -> 0.37 (a 128 GiB table) the 42-spin chain product from 2425
// to 1756 ms.
uint64_t hash_capacity(uint64_t dim) {
    struct Tier {
        uint64_t num, den, limit;   // slots >= dim * num / den while slots * 16 <= limit
    };
    const Tier tiers[] = {{8, 1, 8ULL << 30}, {4, 1, 64ULL << 30}, {2, 1, 128ULL << 30}, {4, 3, 128ULL << 30}};
    for (const Tier &t : tiers) {
        uint64_t cap = 1024;
        while (cap * t.den < t.num * dim) cap <<= 1;
        if (cap * sizeof(HashSlot) <= t.limit) return cap;
    }
    return 0;
}

namespace {

// Host images of the device tables of a compiled group, shared by
// upload_plan (device allocations) and the allocation-free count (static
// scratch): binomial table [65][65], coset representatives, characters by
// code, chi == 1 bitset, pair table (tori).
struct PlanTables {
    std::vector<uint64_t> binom;
};

PlanTables plan_tables() {
    PlanTables t;
    t.binom.assign(65 * 65, 0);
    for (uint32_t i = 0; i <= 64; ++i)
        for (uint32_t k = 0; k <= i; ++k) t.binom[i * 65 + k] = host_binom(i, k);
    return t;
}

// PlanDev fields that do not point into device memory.
void fill_plan_dev(const GroupPlan &gp, PlanDev &pd) {
    pd.n_sites = gp.n_sites;
    pd.lx = gp.lx;
    pd.ly = gp.ly;
    pd.n_trans = gp.lx * gp.ly;
    pd.n_cosets = static_cast<uint32_t>(gp.cosets.size());
    pd.pair_flip = gp.pair_flip;
    pd.n_stages = gp.n_stages;
    pd.n_elements = gp.n_elements;
    pd.full = gp.full;
    pd.col0 = gp.col0;
    pd.pair_lut = nullptr;
    for (int a = 0; a < 8; ++a) pd.col_ge[a] = gp.col_ge[a];
    pd.n_stab_cls = 0;
    pd.stab_cls = nullptr;
    pd.stab_ratio = nullptr;
}

// Stabilizer-ratio table of a group: the class of every divisor of |G|
// (0xFF for the other sizes) followed, at offset kStabMapBytes, by the
// correctly rounded sqrt(d_b / d_a) over pairs of divisors (IEEE division
// and square root, the bits the kernels' own division and square root give).
// Empty when |G| or its number of divisors is above the table's limits.
std::vector<unsigned char> stab_table(uint32_t ng, uint32_t &n_cls) {
    n_cls = 0;
    if (ng > kStabMapMax) return {};
    std::vector<uint32_t> div;
    for (uint32_t d = 1; d <= ng; ++d)
        if (ng % d == 0) div.push_back(d);
    if (div.size() > kStabClsMax) return {};
    const uint32_t nd = static_cast<uint32_t>(div.size());
    std::vector<unsigned char> t(kStabMapBytes + static_cast<size_t>(nd) * nd * sizeof(double), 0xFF);
    for (uint32_t c = 0; c < nd; ++c) t[div[c]] = static_cast<unsigned char>(c);
    double *r = reinterpret_cast<double *>(t.data() + kStabMapBytes);
    for (uint32_t a = 0; a < nd; ++a)
        for (uint32_t c = 0; c < nd; ++c)
            r[a * nd + c] = std::sqrt(static_cast<double>(div[c]) / static_cast<double>(div[a]));
    n_cls = nd;
    return t;
}

}  // namespace

void upload_plan(ls_basis *b, hipStream_t st) {
    const GroupPlan &gp = b->plan;
    const PlanTables t = plan_tables();
    b->d_binom = dev_alloc_n<uint64_t>(t.binom.size(), st);
    LS_HIP_CHECK(hipMemcpyAsync(b->d_binom, t.binom.data(), t.binom.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    const size_t ncos = gp.cosets.size();
    b->d_cosets = dev_alloc_n<CosetRep>(ncos, st);
    LS_HIP_CHECK(hipMemcpyAsync(b->d_cosets, gp.cosets.data(), ncos * sizeof(CosetRep), hipMemcpyHostToDevice, st));
    b->d_chi = dev_alloc_n<double2>(gp.n_elements, st);
    LS_HIP_CHECK(hipMemcpyAsync(b->d_chi, gp.chi.data(), gp.n_elements * sizeof(double2), hipMemcpyHostToDevice, st));
    b->d_chi_one = dev_alloc_n<uint32_t>(gp.chi_one.size(), st);
    LS_HIP_CHECK(hipMemcpyAsync(b->d_chi_one, gp.chi_one.data(), gp.chi_one.size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice, st));
    PlanDev &pd = b->plan_dev;
    fill_plan_dev(gp, pd);
    pd.cosets = b->d_cosets;
    pd.chi = b->d_chi;
    pd.chi_one = b->d_chi_one;
    if (gp.torus) {
        b->d_pair_lut = dev_alloc_n<uint32_t>(gp.pair_lut.size(), st);
        LS_HIP_CHECK(hipMemcpyAsync(b->d_pair_lut, gp.pair_lut.data(), gp.pair_lut.size() * sizeof(uint32_t),
                                    hipMemcpyHostToDevice, st));
        pd.pair_lut = b->d_pair_lut;
    }
    uint32_t n_cls = 0;
    const std::vector<unsigned char> stab = stab_table(gp.n_elements, n_cls);
    if (n_cls) {
        unsigned char *d = dev_alloc_n<unsigned char>(stab.size(), st);
        b->d_stab_tab = d;
        LS_HIP_CHECK(hipMemcpyAsync(d, stab.data(), stab.size(), hipMemcpyHostToDevice, st));
        pd.n_stab_cls = n_cls;
        pd.stab_cls = d;
        pd.stab_ratio = reinterpret_cast<const double *>(d + kStabMapBytes);
    }
    // the host tables are released on return: the copies complete first
    LS_HIP_CHECK(hipStreamSynchronize(st));
}

uint64_t candidate_count(const ls_basis *b) {
    const uint32_t n = b->plan.n_sites;
    if (b->weight >= 0) return host_binom(n, static_cast<uint32_t>(b->weight));
    return n == 64 ? ~0ULL : (1ULL << n);
}

namespace {

__global__ void k_clear_u64(unsigned long long *p) { *p = 0ull; }

// Members among the candidates of rank [begin, end) (end within range),
// accumulated into *acc (device, 8 bytes; cleared here by a fill kernel);
// the plan's tables must be on the device.
template <typename W>
uint64_t count_impl(const GroupPlan &gp, const PlanDev &pd, const uint64_t *binom, int32_t weight, uint64_t begin,
                    uint64_t end, unsigned long long *acc, hipStream_t st) {
    // 64 candidates per lane as in the mark pass; a launch covers up to 2^20
    // workgroups (1.7e10 candidates, a fraction of a second)
    constexpr uint32_t kPerLane = kCandPerLane;
    constexpr uint64_t kSpan = (1ull << 20) * kBlock * kPerLane;
    unsigned long long total = 0;
    hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(1), 0, st, acc);
    LS_HIP_CHECK(hipGetLastError());
    EnumArgs a{};
    a.plan = pd;
    a.binom = binom;
    a.total = end;
    a.n_sites = gp.n_sites;
    a.weight = weight;
    const int kind = orbit_kind<W>(gp);
    for (uint64_t lo = begin; lo < end;) {
        const uint64_t hi = end - lo > kSpan ? lo + kSpan : end;
        const uint64_t lanes = (hi - lo + kPerLane - 1) / kPerLane;
        const uint32_t blocks = static_cast<uint32_t>((lanes + kBlock - 1) / kBlock);
        if (kind == kOrbitRing32)
            hipLaunchKernelGGL((k_enum_count<W, kOrbitRing32>), dim3(blocks), dim3(kBlock), 0, st, a, lo, hi,
                               kPerLane, acc);
        else
            hipLaunchKernelGGL((k_enum_count<W, kOrbitGeneric>), dim3(blocks), dim3(kBlock), 0, st, a, lo, hi,
                               kPerLane, acc);
        LS_HIP_CHECK(hipGetLastError());
        lo = hi;
    }
    LS_HIP_CHECK(hipMemcpyAsync(&total, acc, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    LS_HIP_CHECK(hipStreamSynchronize(st));
    return static_cast<uint64_t>(total);
}

uint64_t candidates_of(const GroupPlan &gp, int32_t weight) {
    const uint32_t n = gp.n_sites;
    if (weight >= 0) return host_binom(n, static_cast<uint32_t>(weight));
    return n == 64 ? ~0ULL : (1ULL << n);
}

}  // namespace

uint64_t count_members(ls_basis *b, uint64_t begin, uint64_t end, hipStream_t st) {
    const uint64_t total = candidate_count(b);
    end = std::min(end, total);
    if (begin >= end) return 0;
    StreamBuf acc_b(sizeof(unsigned long long), st);
    unsigned long long *acc = acc_b.as<unsigned long long>();
    const GroupPlan &gp = b->plan;
    return gp.n_sites <= 32 ? count_impl<uint32_t>(gp, b->plan_dev, b->d_binom, b->weight, begin, end, acc, st)
                            : count_impl<uint64_t>(gp, b->plan_dev, b->d_binom, b->weight, begin, end, acc, st);
}

// ---- the allocation-free count --------------------------------------------
//
// The same count for callers that cannot allocate device memory: the
// compiled group's tables and the accumulator live in `scratch`, a
// file-scope device array of kCountScratchBytes that each GPU holds for the
// life of the process.  Host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in symbol): the device
// address of each GPU's copy is taken once with hipGetSymbolAddress, with
// that GPU current, and used everywhere.  Calls are serialised by a
// process-wide lock, since every call on a GPU shares its array; calls from
// several processes on one GPU use separate arrays.

constexpr size_t kCountScratchBytes = 256 * 1024;
static __device__ __align__(256) unsigned char scratch[kCountScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[256] = {};   // per device ordinal

void *scratch_address(int dev) {
    if (dev < 0 || dev >= 256) throw Error{LS_EDEVICE, "device ordinal out of range"};
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            throw Error{LS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

uint64_t count_members_noalloc(const GroupPlan &gp, int32_t weight, uint64_t begin, uint64_t end, hipStream_t st,
                               uint64_t *n_candidates) {
    const uint64_t total = candidates_of(gp, weight);
    if (n_candidates) *n_candidates = total;
    end = std::min(end, total);
    // layout: accumulator | binomials | cosets | characters | chi == 1 bits | pair table
    const PlanTables t = plan_tables();
    const size_t o_binom = 256;
    const size_t o_cos = align_up(o_binom + t.binom.size() * sizeof(uint64_t), 256);
    const size_t o_chi = align_up(o_cos + gp.cosets.size() * sizeof(CosetRep), 256);
    const size_t o_one = align_up(o_chi + gp.chi.size() / 2 * sizeof(double2), 256);
    const size_t o_lut = align_up(o_one + gp.chi_one.size() * sizeof(uint32_t), 256);
    const size_t need = o_lut + (gp.torus ? gp.pair_lut.size() * sizeof(uint32_t) : 0);
    if (need > kCountScratchBytes)
        throw Error{LS_EINVAL, "the compiled group needs " + std::to_string(need) + " bytes of device tables, above the " +
                                   std::to_string(kCountScratchBytes) +
                                   "-byte scratch of the allocation-free count (use ls_sector_count)"};
    if (begin >= end) return 0;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    int dev = 0;
    LS_HIP_CHECK(hipGetDevice(&dev));
    unsigned char *base = static_cast<unsigned char *>(scratch_address(dev));
    auto put = [&](size_t off, const void *src, size_t bytes) {
        if (bytes) LS_HIP_CHECK(hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, st));
    };
    put(o_binom, t.binom.data(), t.binom.size() * sizeof(uint64_t));
    put(o_cos, gp.cosets.data(), gp.cosets.size() * sizeof(CosetRep));
    put(o_chi, gp.chi.data(), gp.chi.size() * sizeof(double));
    put(o_one, gp.chi_one.data(), gp.chi_one.size() * sizeof(uint32_t));
    PlanDev pd{};
    fill_plan_dev(gp, pd);
    pd.cosets = reinterpret_cast<const CosetRep *>(base + o_cos);
    pd.chi = reinterpret_cast<const double2 *>(base + o_chi);
    pd.chi_one = reinterpret_cast<const uint32_t *>(base + o_one);
    if (gp.torus) {
        put(o_lut, gp.pair_lut.data(), gp.pair_lut.size() * sizeof(uint32_t));
        pd.pair_lut = reinterpret_cast<const uint32_t *>(base + o_lut);
    }
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(base);
    const uint64_t *binom = reinterpret_cast<const uint64_t *>(base + o_binom);
    return gp.n_sites <= 32 ? count_impl<uint32_t>(gp, pd, binom, weight, begin, end, acc, st)
                            : count_impl<uint64_t>(gp, pd, binom, weight, begin, end, acc, st);
}

void build_basis(ls_basis *b, hipStream_t st) {
    const GroupPlan &gp = b->plan;
    const uint32_t n = gp.n_sites;
    upload_plan(b, st);

    // candidates
    const uint64_t total = candidate_count(b);
    if (n <= 32) enumerate_impl<uint32_t>(b, st, total, &b->d_reps, &b->dim);
    else enumerate_impl<uint64_t>(b, st, total, &b->d_reps, &b->dim);
    if (b->dim >= 0xFFFFFFFFull) throw Error{LS_EINVAL, "basis dimension must be below 2^32 - 1"};

    b->d_stab = dev_alloc_n<uint16_t>(std::max<uint64_t>(b->dim, 1), st);
    if (n <= 32) stab_impl<uint32_t>(b, st);
    else stab_impl<uint64_t>(b, st);

    // search layout
    SearchDev &S = b->search_dev;
    S.n_sites = n;
    S.weight = b->weight;
    S.dim = b->dim;
    S.reps = b->d_reps;
    S.binom = b->d_binom;
    if (gp.n_elements == 1 && b->weight < 0) {
        S.mode = kLookupIdentity;
    } else if (gp.n_elements == 1) {
        S.mode = kLookupRank;
    } else {
        uint64_t kmin = 0, kmax = 0;
        if (b->dim > 0) {
            LS_HIP_CHECK(hipMemcpyAsync(&kmin, b->d_reps, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
            LS_HIP_CHECK(hipMemcpyAsync(&kmax, b->d_reps + (b->dim - 1), sizeof(uint64_t), hipMemcpyDeviceToHost, st));
            LS_HIP_CHECK(hipStreamSynchronize(st));
        }
        S.kmin = kmin;
        S.kmax = kmax;
        // Hash index (hash_capacity); when it would pass 128 GiB, or when asked
        // for, the bucket search.
        const char *env = std::getenv("LS_ED_SEARCH");
        const bool want_buckets = env != nullptr && std::string(env) == "buckets";
        const uint64_t cap = hash_capacity(b->dim);
        if (!want_buckets && cap != 0 && kmax != kEmptyKey) {
            S.mode = kLookupHash;
            S.hash_mask = cap - 1;
            S.hash_shift = 64;
            for (uint64_t c = cap; c > 1; c >>= 1) --S.hash_shift;
            b->d_table = dev_alloc_n<HashSlot>(cap, st);
            LS_HIP_CHECK(hipMemsetAsync(b->d_table, 0xFF, cap * sizeof(HashSlot), st));
            if (b->dim > 0)
                hipLaunchKernelGGL(k_hash_insert, dim3(grid_for(b->dim)), dim3(kBlock), 0, st, b->d_reps, b->d_stab,
                                   b->dim, b->d_table, S.hash_mask, S.hash_shift);
            LS_HIP_CHECK(hipGetLastError());
            S.table = b->d_table;
            LS_HIP_CHECK(hipStreamSynchronize(st));
            return;
        }
        S.mode = kLookupSearch;
        // about 4 keys per bucket, 2^8 .. 2^22 buckets
        uint32_t bits = 8;
        while (bits < 22 && (1ULL << bits) * 4 < b->dim) ++bits;
        const uint64_t range = kmax - kmin;
        uint32_t len = 0;
        while (len < 64 && (range >> len) != 0) ++len;
        S.bits = bits;
        S.shift = len > bits ? len - bits : 0;
        const uint64_t nb = (range >> S.shift) + 1;   // buckets 0 .. nb-1
        b->d_buckets = dev_alloc_n<uint32_t>(nb + 1, st);
        hipLaunchKernelGGL(k_buckets, dim3(grid_for(nb + 1)), dim3(kBlock), 0, st, b->d_reps, b->dim, kmin, S.shift,
                           nb, b->d_buckets);
        LS_HIP_CHECK(hipGetLastError());
        S.buckets = b->d_buckets;
    }
    LS_HIP_CHECK(hipStreamSynchronize(st));
}

void drop_key(ls_basis *b, uint64_t index, hipStream_t st) {
    const SearchDev &S = b->search_dev;
    LS_REQUIRE(S.mode == kLookupHash, "only a hash search layout can drop a key");
    LS_REQUIRE(S.kmax + 1 != kEmptyKey, "no free key value above the representatives");
    uint64_t key = 0;
    LS_HIP_CHECK(hipMemcpyAsync(&key, b->d_reps + index, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    LS_HIP_CHECK(hipStreamSynchronize(st));
    hipLaunchKernelGGL(k_drop_key, dim3(1), dim3(1), 0, st, b->d_table, S.hash_mask, S.hash_shift, key, S.kmax + 1);
    LS_HIP_CHECK(hipGetLastError());
    LS_HIP_CHECK(hipStreamSynchronize(st));
}

void launch_state_info(const ls_basis *b, uint64_t n, const uint64_t *states, uint64_t *reps, double *chi,
                       double *norm, hipStream_t st) {
    if (n == 0) return;
    const GroupPlan &gp = b->plan;
    if (gp.n_sites <= 32) {
        if (orbit_kind<uint32_t>(gp) == kOrbitRing32)
            hipLaunchKernelGGL((k_state_info<uint32_t, kOrbitRing32>), dim3(grid_for(n)), dim3(kBlock), 0, st,
                               b->plan_dev, b->weight, n, states, reps, chi, norm);
        else
            hipLaunchKernelGGL((k_state_info<uint32_t, kOrbitGeneric>), dim3(grid_for(n)), dim3(kBlock), 0, st,
                               b->plan_dev, b->weight, n, states, reps, chi, norm);
    } else {
        hipLaunchKernelGGL((k_state_info<uint64_t, kOrbitGeneric>), dim3(grid_for(n)), dim3(kBlock), 0, st,
                           b->plan_dev, b->weight, n, states, reps, chi, norm);
    }
    LS_HIP_CHECK(hipGetLastError());
}

void launch_index_lookup(const ls_basis *b, uint64_t n, const uint64_t *keys, int64_t *index, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_index_lookup, dim3(grid_for(n)), dim3(kBlock), 0, st, b->search_dev, n, keys, index);
    LS_HIP_CHECK(hipGetLastError());
}

}  // namespace ls
