// Batched products: many operators (sectors, couplings, dimensions) and
// right-hand sides in one persistent launch per kernel variant.
//
// Work is cut into tiles of (job, first row); a job is one operator and a
// slice of its right-hand-side columns.  A fixed grid of workgroups pulls
// tiles from a counter in device memory (reset by a one-thread kernel, so
// the sequence can be captured in a HIP graph and replayed); when the job
// changes, the workgroup restages the job's LDS tables.  Tiles are ordered
// by decreasing job cost, so the tail of the queue is made of small tiles.
//
// An autotuner picks, per variant group, the rows per lane of a tile and the
// number of resident workgroups by timing the candidates on first use, and,
// per basis that uses the bucket search layout (hash layouts are used as
// built), the number of bucket bits by timing a lookup sweep (the batch owns
// these tables; the basis is not modified).
// Results are cached per process.

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "dispatch.hpp"

namespace ls {

namespace {

struct Tile {
    uint32_t job;
    uint32_t pad_;
    uint64_t row0;
};

// Workgroup size of the persistent kernel: the complex torus search holds
// more live state than 128 VGPRs (the most a 1024-thread workgroup allows)
// around the tile loop, so it runs in 512-thread workgroups.
constexpr int batch_block(int kind, bool cplx) { return (kind == kOrbitTorus && cplx) ? 512 : block_of(kind); }

template <typename W, int KIND, int CHI, bool CPLX, int NR, uint32_t LX, uint32_t LY, uint32_t NZ>
__global__ void __launch_bounds__(batch_block(KIND, CPLX))
    k_matvec_batch(const MatvecJob *jobs, const Tile *tiles, uint32_t n_tiles, uint32_t *counter, uint32_t rpl,
                   uint32_t tile_rows) {
    constexpr int BLOCK = batch_block(KIND, CPLX);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_tile;
    uint32_t cur = 0xFFFFFFFFu;
    LdsTables L{};
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t tile = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (tile >= n_tiles) break;
        const Tile T = tiles[tile];
        const uint32_t jid = __builtin_amdgcn_readfirstlane(T.job);
        const MatvecJob &a = jobs[jid];
        if (jid != cur) {
            L = lds_tables<KIND, LX, BLOCK, false>(a, smem);
            stage_tables<KIND, LX, BLOCK, false>(a, L);
            __syncthreads();
            cur = jid;
        }
        // a tile is rows row0 + t + k * tile_rows (t < tile_rows, k < rpl);
        // tile_rows < BLOCK spreads small jobs over more workgroups
        if (threadIdx.x < tile_rows)
            run_rows<W, KIND, CHI, CPLX, NR, LX, LY, NZ, true>(a, L, T.row0 + threadIdx.x, tile_rows, rpl);
    }
}

__global__ void k_reset_counter(uint32_t *c) { *c = 0u; }

// Bucket table for a candidate number of bits (same rule as the basis build).
__global__ void k_buckets_tuned(const uint64_t *reps, uint64_t d, uint64_t kmin, uint32_t shift, uint64_t nb,
                                uint32_t *buckets) {
    const uint64_t k = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x;
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

// Right-hand sides per job of the persistent kernel.  Its tile loop holds
// more live state than the single launch, and with 1024-thread workgroups
// (128 VGPRs at most) the wider torus variants would spill to scratch; the
// cap keeps every instantiated variant in registers.  Columns are computed
// independently, so the cap changes no result bit.
constexpr int nr_cap(bool word64, int kind) { return kind != kOrbitTorus ? 8 : word64 ? 1 : 2; }
int batch_nr_cap(const Variant &v) { return nr_cap(v.word64 != 0, v.kind); }

// Lookup sweep used to time a search layout, in the shape of the batched
// launch (a persistent grid of 1024-thread workgroups, each staging a staged
// layout's bucket table once): keys are representatives taken in a scattered
// order, and every lookup also yields the stabilizer size, as in a product.
constexpr int kSweepBlock = 1024;
__global__ void __launch_bounds__(kSweepBlock)
    k_lookup_sweep(SearchDev S, const uint16_t *stab, uint64_t n, uint64_t magic, uint64_t *sink) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *lb = reinterpret_cast<uint32_t *>(smem);
    if (S.mode == kLookupStaged) {
        for (uint32_t q = threadIdx.x; q < S.n_bkt; q += kSweepBlock) lb[q] = S.buckets[q];
        __syncthreads();
    }
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kSweepBlock;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kSweepBlock + threadIdx.x; i < n; i += stride) {
        const uint64_t j = __umul64hi(i * 0x9E3779B97F4A7C15ULL, S.dim);
        const uint64_t key = S.reps[j];
        uint32_t st = 0;
        int64_t idx;
        if (S.mode == kLookupStaged) {
            idx = lookup_staged(S, lb, key);
            if (idx >= 0) st = stab[idx];
        } else {
            idx = lookup_index_stab(S, key, stab, st);
        }
        // magic is a value no sum takes; the store keeps the lookup live
        if (static_cast<uint64_t>(idx) + st == magic) *sink = j;
    }
}

struct Group {
    Variant v;
    int nr = 1;
    std::vector<MatvecJob> jobs;
    std::vector<std::pair<uint32_t, uint32_t>> item_col;   // (item, first column) per job
    std::vector<double> cost;
    MatvecJob *d_jobs = nullptr;
    Tile *d_tiles = nullptr;
    uint32_t *d_counter = nullptr;
    uint32_t n_tiles = 0;
    uint32_t rpl = 4;
    uint32_t tile_rows = 0;   // rows per tile step (0: the workgroup size)
    uint32_t grid = 0;
    size_t lds = 0;
    bool tuned = false;
    size_t cap_jobs = 0, cap_tiles = 0;   // device table capacities (fused path)
};

struct BatchLaunch {
    Group *g;
    hipStream_t st;
    template <typename W, int KIND, int CHI, bool CPLX, int NR, uint32_t LX, uint32_t LY, uint32_t NZ>
    void run() {
        // variants above the cap are never grouped (batch_nr_cap) and never built
        if constexpr (NR > nr_cap(sizeof(W) == 8, KIND)) {
            throw Error{LS_EINTERNAL, "batched job wider than its variant's cap"};
        } else {
            constexpr int BLOCK = batch_block(KIND, CPLX);
            hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, g->d_counter);
            hipLaunchKernelGGL((k_matvec_batch<W, KIND, CHI, CPLX, NR, LX, LY, NZ>), dim3(g->grid), dim3(BLOCK),
                               g->lds, st, g->d_jobs, g->d_tiles, g->n_tiles, g->d_counter, g->rpl,
                               g->tile_rows ? g->tile_rows : static_cast<uint32_t>(BLOCK));
        }
    }
};

int block_for(const Variant &v) { return batch_block(v.kind, v.cplx); }

// Tiles for the current rows-per-lane, ordered by decreasing job cost.
void build_tiles(Group &g, hipStream_t st) {
    const uint64_t rows_per_tile = static_cast<uint64_t>(g.tile_rows ? g.tile_rows : block_for(g.v)) * g.rpl;
    std::vector<uint32_t> order(g.jobs.size());
    for (uint32_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return g.cost[a] > g.cost[b]; });
    std::vector<Tile> tiles;
    for (uint32_t j : order)
        for (uint64_t r = 0; r < g.jobs[j].dim; r += rows_per_tile) tiles.push_back(Tile{j, 0, r});
    dev_free(g.d_tiles, st);
    g.d_tiles = dev_alloc_n<Tile>(std::max<size_t>(tiles.size(), 1), st);
    if (!tiles.empty())
        LS_HIP_CHECK(hipMemcpyAsync(g.d_tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, st));
    LS_HIP_CHECK(hipStreamSynchronize(st));
    g.n_tiles = static_cast<uint32_t>(tiles.size());
}

void upload_jobs(Group &g, hipStream_t st) {
    LS_HIP_CHECK(hipMemcpyAsync(g.d_jobs, g.jobs.data(), g.jobs.size() * sizeof(MatvecJob), hipMemcpyHostToDevice,
                                st));
}

using TuneKey = std::tuple<int, int, int, uint32_t, uint32_t, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<uint32_t, uint32_t>> g_tune_cache;   // -> (rpl, workgroups per CU)
// (dim, kmin, kmax, LDS free) -> (mode, bits, own, chosen, best staged ns per lookup)
std::map<std::tuple<uint64_t, uint64_t, uint64_t, uint64_t>, std::tuple<uint32_t, uint32_t, double, double, double>>
    g_search_cache;

TuneKey tune_key(const Group &g) {
    uint64_t rows = 0;
    for (const auto &j : g.jobs) rows += j.dim;
    int lg = 0;
    while ((1ull << lg) < rows) ++lg;
    int lj = 0;
    while ((1u << lj) < g.jobs.size()) ++lj;
    return TuneKey{g.v.word64, g.v.kind, g.v.chi, g.v.lx, g.v.ly, g.v.cplx ? 1 : 0, g.nr, lg, lj};
}

float time_group(Group &g, hipStream_t st) {
    hipEvent_t e0, e1;
    LS_HIP_CHECK(hipEventCreate(&e0));
    LS_HIP_CHECK(hipEventCreate(&e1));
    BatchLaunch L{&g, st};
    dispatch(g.v, g.nr, L);   // warm
    LS_HIP_CHECK(hipEventRecord(e0, st));
    dispatch(g.v, g.nr, L);
    LS_HIP_CHECK(hipEventRecord(e1, st));
    LS_HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    LS_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    LS_HIP_CHECK(hipGetLastError());
    return ms;
}

void tune_group(Group &g, hipStream_t st, int n_cu) {
    const int block = block_for(g.v);
    const int max_wg_per_cu = std::max(1, 2048 / block);   // 32 waves per CU
    const TuneKey key = tune_key(g);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            g.rpl = it->second.first;
            g.grid = static_cast<uint32_t>(n_cu * it->second.second);
            build_tiles(g, st);
            g.tuned = true;
            return;
        }
    }
    float best = 1e30f;
    uint32_t best_rpl = 4, best_wpc = static_cast<uint32_t>(max_wg_per_cu);
    for (uint32_t rpl : {1u, 2u, 4u, 8u}) {
        g.rpl = rpl;
        build_tiles(g, st);
        for (int wpc = 1; wpc <= max_wg_per_cu; wpc *= 2) {
            g.grid = static_cast<uint32_t>(std::min<uint64_t>(static_cast<uint64_t>(n_cu) * wpc,
                                                              std::max<uint32_t>(g.n_tiles, 1)));
            const float ms = time_group(g, st);
            if (ms < best) {
                best = ms;
                best_rpl = rpl;
                best_wpc = static_cast<uint32_t>(wpc);
            }
        }
    }
    g.rpl = best_rpl;
    g.grid = static_cast<uint32_t>(n_cu * best_wpc);
    build_tiles(g, st);
    g.tuned = true;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {best_rpl, best_wpc};
}

}  // namespace

}  // namespace ls

namespace ls {
// A batch's search layout for one basis and the lookup sweep times behind
// the choice (ns per lookup; 0 when no sweep ran).
struct SearchChoice {
    SearchDev S;
    double own_ns = 0.0, chosen_ns = 0.0, staged_ns = 0.0;
};
}  // namespace ls

struct ls_batch {
    std::vector<const ls_operator *> ops;
    std::vector<uint32_t> nrhs;
    std::vector<ls::Group> groups;
    std::vector<const void *> cur_x;
    std::vector<void *> cur_y;
    std::vector<uint32_t *> own_buckets;     // tuned search layouts (one per basis)
    std::vector<ls::SearchChoice> search;    // per item
    hipStream_t cap = nullptr;               // stream used for graph capture
    ls::StreamSet used;                      // streams of its products
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int force_mode = -1;                     // ls_batch_set_search (-1: tune)
    uint32_t force_bits = 0;
    bool use_graph = true;
    bool ready = false;
    int n_cu = 256;
};

namespace ls {

namespace {

// A bucket table of 2^nbits buckets over the keys' range of basis b (the
// build's bucket rule), in a batch-owned allocation *out.
SearchDev bucket_layout(const ls_basis *b, uint32_t mode, uint32_t nbits, uint32_t **out, hipStream_t st) {
    SearchDev T = b->search_dev;
    const uint64_t range = T.kmax - T.kmin;
    uint32_t len = 0;
    while (len < 64 && (range >> len) != 0) ++len;
    T.mode = mode;
    T.bits = nbits;
    T.shift = len > nbits ? len - nbits : 0;
    const uint64_t nb = (range >> T.shift) + 1;
    *out = dev_alloc_n<uint32_t>(nb + 1, st);
    hipLaunchKernelGGL(k_buckets_tuned, dim3(static_cast<uint32_t>((nb + 1 + 255) / 256)), dim3(256), 0, st,
                       b->d_reps, b->dim, T.kmin, T.shift, nb, *out);
    LS_HIP_CHECK(hipGetLastError());
    T.buckets = *out;
    T.n_bkt = static_cast<uint32_t>(nb + 1);
    return T;
}

bool staged_fits(uint32_t nbits, size_t lds_free) {
    return nbits <= kMaxStagedBits && ((1ULL << nbits) + 2) * sizeof(uint32_t) <= lds_free;
}

// Search layout of one basis for the batch: the fastest, by a timed lookup
// sweep, of the basis's own layout (hash index or bucket search, as built),
// bucket tables of several sizes read from global memory, and bucket tables
// staged in LDS (when they fit beside the jobs' own LDS tables: lds_free
// bytes); or the layout ls_batch_set_search forced.  The batch owns the
// tables it builds; the basis is not modified.  Tuning results are cached
// per process by (dim, kmin, kmax, lds_free).
SearchChoice tuned_search(ls_batch *B, const ls_basis *b, size_t lds_free, hipStream_t st) {
    SearchChoice C;
    C.S = b->search_dev;
    const SearchDev &own = b->search_dev;
    if (own.mode != kLookupSearch && own.mode != kLookupHash) return C;
    if (B->force_mode >= 0) {
        if (B->force_mode == static_cast<int>(kLookupHash)) return C;   // the basis's own
        const uint32_t mode = static_cast<uint32_t>(B->force_mode);
        if (mode == kLookupStaged && !staged_fits(B->force_bits, lds_free))
            throw Error{LS_EINVAL, "the forced staged bucket table does not fit in LDS beside the jobs' tables"};
        uint32_t *tab = nullptr;
        C.S = bucket_layout(b, mode, B->force_bits, &tab, st);
        B->own_buckets.push_back(tab);
        return C;
    }
    if (b->dim < 4096) return C;
    const auto key = std::make_tuple(b->dim, own.kmin, own.kmax, static_cast<uint64_t>(lds_free));
    auto table = [&](uint32_t mode, uint32_t nbits, uint32_t **out) { return bucket_layout(b, mode, nbits, out, st); };
    std::tuple<uint32_t, uint32_t, double, double, double> pick;   // mode, bits, own, chosen, staged (ns/key)
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_search_cache.find(key);
        if (it != g_search_cache.end()) {
            pick = it->second;
            cached = true;
        }
    }
    if (!cached) {
        // candidates: the basis's own layout, then (mode, bits) tables around
        // the build rule of about 4 keys per bucket
        uint32_t b0 = 8;
        while (b0 < 22 && (1ULL << b0) * 4 < b->dim) ++b0;
        std::vector<std::pair<uint32_t, uint32_t>> cands = {{own.mode, own.mode == kLookupSearch ? own.bits : 0u}};
        for (int d : {-2, 0, 2}) {
            const int nb = static_cast<int>(b0) + d;
            if (nb >= 8 && nb <= 24 && !(own.mode == kLookupSearch && static_cast<uint32_t>(nb) == own.bits))
                cands.push_back({kLookupSearch, static_cast<uint32_t>(nb)});
        }
        const uint32_t sb = std::min(b0, kMaxStagedBits);
        for (uint32_t nb : {sb, sb - 2})
            if (nb >= 8 && staged_fits(nb, lds_free)) cands.push_back({kLookupStaged, nb});
        uint64_t *sink = dev_alloc_n<uint64_t>(1, st);
        hipEvent_t e0, e1;
        LS_HIP_CHECK(hipEventCreate(&e0));
        LS_HIP_CHECK(hipEventCreate(&e1));
        const uint64_t n = std::min<uint64_t>(b->dim, 1u << 22);
        const uint32_t grid = static_cast<uint32_t>(std::min<uint64_t>(
            static_cast<uint64_t>(B->n_cu) * 2, (n + kSweepBlock - 1) / kSweepBlock));
        double best = 1e30, own_ns = 0.0, staged_ns = 0.0;
        uint32_t best_mode = own.mode, best_bits = cands[0].second;
        for (size_t c = 0; c < cands.size(); ++c) {
            uint32_t *tab = nullptr;
            const SearchDev T = c == 0 ? own : table(cands[c].first, cands[c].second, &tab);
            const size_t lds = T.mode == kLookupStaged ? static_cast<size_t>(T.n_bkt) * sizeof(uint32_t) : 0;
            for (int rep = 0; rep < 2; ++rep) {   // warm, then timed
                if (rep == 1) LS_HIP_CHECK(hipEventRecord(e0, st));
                hipLaunchKernelGGL(k_lookup_sweep, dim3(grid), dim3(kSweepBlock), lds, st, T, b->d_stab, n,
                                   ~0ULL - 1, sink);
            }
            LS_HIP_CHECK(hipEventRecord(e1, st));
            LS_HIP_CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            LS_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
            if (tab) dev_free(tab, st);
            const double ns = static_cast<double>(ms) * 1e6 / static_cast<double>(n);
            if (c == 0) own_ns = ns;
            if (cands[c].first == kLookupStaged && (staged_ns == 0.0 || ns < staged_ns)) staged_ns = ns;
            if (ns < best) {
                best = ns;
                best_mode = cands[c].first;
                best_bits = cands[c].second;
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        dev_free(sink, st);
        pick = std::make_tuple(best_mode, best_bits, own_ns, best, staged_ns);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_search_cache[key] = pick;
    }
    C.own_ns = std::get<2>(pick);
    C.chosen_ns = std::get<3>(pick);
    C.staged_ns = std::get<4>(pick);
    const uint32_t mode = std::get<0>(pick), nbits = std::get<1>(pick);
    if (mode == own.mode && (mode == kLookupHash || nbits == own.bits)) return C;   // the basis's own
    uint32_t *tab = nullptr;
    C.S = table(mode, nbits, &tab);
    B->own_buckets.push_back(tab);
    return C;
}

void free_batch(ls_batch *B) {
    if (!B) return;
    B->used.drain();
    for (auto &g : B->groups) {
        dev_free(g.d_jobs);
        dev_free(g.d_tiles);
        dev_free(g.d_counter);
    }
    for (auto *p : B->own_buckets) dev_free(p);
    if (B->exec) hipGraphExecDestroy(B->exec);
    if (B->graph) hipGraphDestroy(B->graph);
    if (B->cap) hipStreamDestroy(B->cap);
    delete B;
}

}  // namespace

void batch_create(uint32_t n, const ls_operator *const *ops, const uint32_t *nrhs, ls_batch **out) {
    LS_REQUIRE(n >= 1 && ops != nullptr && nrhs != nullptr && out != nullptr, "invalid batch arguments");
    ls_batch *B = new ls_batch();
    try {
        for (uint32_t i = 0; i < n; ++i) {
            LS_REQUIRE(ops[i] != nullptr, "operator must not be NULL");
            LS_REQUIRE(nrhs[i] >= 1 && nrhs[i] <= 64, "nrhs must be in 1..64");
            B->ops.push_back(ops[i]);
            B->nrhs.push_back(nrhs[i]);
        }
        B->cur_x.assign(n, nullptr);
        B->cur_y.assign(n, nullptr);
        int dev = 0;
        LS_HIP_CHECK(hipGetDevice(&dev));
        LS_HIP_CHECK(hipDeviceGetAttribute(&B->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        LS_HIP_CHECK(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    } catch (...) {
        free_batch(B);
        throw;
    }
    *out = B;
}

void batch_destroy(ls_batch *B) { free_batch(B); }

// First call: search layouts, grouping, tiles, tuning; later calls reuse them.
static void batch_prepare(ls_batch *B, hipStream_t st) {
    const uint32_t n = static_cast<uint32_t>(B->ops.size());
    // one tuned search layout per distinct basis; a staged bucket table must
    // fit beside the LDS tables of every job on that basis
    std::map<const ls_basis *, size_t> lds_free;
    for (uint32_t i = 0; i < n; ++i) {
        const ls_operator *op = B->ops[i];
        const int kind = variant_of(op).kind;
        const size_t own = lds_bytes(kind, op->n_diag + op->n_off, op->n_off, op->basis->plan.lx) +
                           (kind == kOrbitTorus ? kPairTableBytes : 0);
        const size_t fr = own + 16 <= kMaxLds ? kMaxLds - own - 16 : 0;
        auto it = lds_free.find(op->basis);
        if (it == lds_free.end()) lds_free.emplace(op->basis, fr);
        else it->second = std::min(it->second, fr);
    }
    std::map<const ls_basis *, SearchChoice> by_basis;
    B->search.resize(n);
    for (uint32_t i = 0; i < n; ++i) {
        const ls_basis *b = B->ops[i]->basis;
        auto it = by_basis.find(b);
        if (it == by_basis.end()) it = by_basis.emplace(b, tuned_search(B, b, lds_free[b], st)).first;
        B->search[i] = it->second;
    }
    for (uint32_t i = 0; i < n; ++i) {
        const ls_operator *op = B->ops[i];
        if (op->basis->dim == 0) continue;
        const Variant v = variant_of(op);
        uint32_t col = 0;
        while (col < B->nrhs[i]) {
            const int nr = std::min(nr_chunk(B->nrhs[i] - col), batch_nr_cap(v));
            Group *g = nullptr;
            for (auto &gg : B->groups)
                if (gg.v == v && gg.nr == nr) g = &gg;
            if (!g) {
                B->groups.emplace_back();
                g = &B->groups.back();
                g->v = v;
                g->nr = nr;
            }
            MatvecJob j = job_of(op, B->cur_x[i], B->cur_y[i], B->nrhs[i], col);
            j.search = B->search[i].S;
            g->jobs.push_back(j);
            g->item_col.push_back({i, col});
            const double nterm = static_cast<double>(op->n_off) + 1.0;
            g->cost.push_back(static_cast<double>(op->basis->dim) * nterm * op->basis->plan.n_elements);
            size_t lds = lds_bytes(v.kind, op->n_diag + op->n_off, op->n_off, op->basis->plan.lx);
            if (j.search.mode == kLookupStaged) lds += static_cast<size_t>(j.search.n_bkt) * sizeof(uint32_t);
            g->lds = std::max(g->lds, lds);
            col += static_cast<uint32_t>(nr);
        }
    }
    for (auto &g : B->groups) {
        g.d_jobs = dev_alloc_n<MatvecJob>(g.jobs.size(), st);
        g.d_counter = dev_alloc_n<uint32_t>(1, st);
        upload_jobs(g, st);
        tune_group(g, st, B->n_cu);
    }
    B->ready = true;
}

void batch_matvec(ls_batch *B, const void *const *xs, void *const *ys, hipStream_t st) {
    const uint32_t n = static_cast<uint32_t>(B->ops.size());
    LS_REQUIRE(xs != nullptr && ys != nullptr, "x and y arrays must not be NULL");
    B->used.add(st);
    for (const ls_operator *op : B->ops) touch(op, st);
    bool changed = false;
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t dim = B->ops[i]->basis->dim;
        if (dim == 0) continue;
        LS_REQUIRE(xs[i] != nullptr && ys[i] != nullptr, "x and y must not be NULL");
        const size_t bytes = dim * B->nrhs[i] * (B->ops[i]->is_complex ? 16u : 8u);
        const char *xb = static_cast<const char *>(xs[i]);
        const char *yb = static_cast<const char *>(ys[i]);
        LS_REQUIRE(xb + bytes <= yb || yb + bytes <= xb, "x and y must not overlap");
        if (xs[i] != B->cur_x[i] || ys[i] != B->cur_y[i]) changed = true;
        B->cur_x[i] = xs[i];
        B->cur_y[i] = ys[i];
    }
    if (changed && B->ready) {
        for (auto &g : B->groups) {
            for (size_t k = 0; k < g.jobs.size(); ++k) {
                const uint32_t item = g.item_col[k].first;
                g.jobs[k].x = B->cur_x[item];
                g.jobs[k].y = B->cur_y[item];
            }
            upload_jobs(g, st);
        }
    }
    if (!B->ready) batch_prepare(B, st);
    if (B->groups.empty()) return;
    if (!B->use_graph) {
        for (auto &g : B->groups) {
            BatchLaunch L{&g, st};
            dispatch(g.v, g.nr, L);
            LS_HIP_CHECK(hipGetLastError());
        }
        return;
    }
    if (!B->exec) {
        // capture on the library's own stream; the graph reads job tables by
        // pointer, so later pointer changes only rewrite those tables
        LS_HIP_CHECK(hipStreamSynchronize(st));
        LS_HIP_CHECK(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
        for (auto &g : B->groups) {
            BatchLaunch L{&g, B->cap};
            dispatch(g.v, g.nr, L);
        }
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(B->cap, &graph);
        LS_HIP_CHECK(e);
        B->graph = graph;
        LS_HIP_CHECK(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    }
    LS_HIP_CHECK(hipGraphLaunch(B->exec, st));
}

void batch_info(const ls_batch *B, uint32_t *n_launches, uint32_t *n_tiles, uint32_t *graph) {
    if (n_launches) *n_launches = static_cast<uint32_t>(B->groups.size());
    if (n_tiles) {
        uint32_t t = 0;
        for (const auto &g : B->groups) t += g.n_tiles;
        *n_tiles = t;
    }
    if (graph) *graph = B->exec != nullptr ? 1u : 0u;
}

void batch_set_graph(ls_batch *B, bool on) { B->use_graph = on; }

void batch_set_search(ls_batch *B, int mode, uint32_t bits) {
    LS_REQUIRE(!B->ready, "the search layout is fixed by the first ls_batch_matvec");
    LS_REQUIRE(mode == -1 || mode == static_cast<int>(kLookupSearch) || mode == static_cast<int>(kLookupHash) ||
                   mode == static_cast<int>(kLookupStaged),
               "mode must be -1 (tune), 0 (buckets), 3 (the basis's own) or 4 (staged)");
    if (mode == static_cast<int>(kLookupSearch) || mode == static_cast<int>(kLookupStaged))
        LS_REQUIRE(bits >= 1 && bits <= (mode == static_cast<int>(kLookupStaged) ? kMaxStagedBits : 30u),
                   "bucket bits out of range (1..30, staged 1..13)");
    B->force_mode = mode;
    B->force_bits = bits;
}

void batch_search(const ls_batch *B, uint32_t item, uint32_t *mode, uint32_t *bits, double *own_ns, double *chosen_ns,
                  double *staged_ns) {
    LS_REQUIRE(item < B->ops.size(), "item must be below the number of operators");
    SearchChoice C;
    if (item < B->search.size()) C = B->search[item];
    else C.S = B->ops[item]->basis->search_dev;
    if (mode) *mode = C.S.mode;
    if (bits) *bits = (C.S.mode == kLookupSearch || C.S.mode == kLookupStaged) ? C.S.bits : 0u;
    if (own_ns) *own_ns = C.own_ns;
    if (chosen_ns) *chosen_ns = C.chosen_ns;
    if (staged_ns) *staged_ns = C.staged_ns;
}

// ---- fused products for the Lanczos stepper --------------------------------
//
// The set of products changes from call to call (solves join and leave), so
// there is no graph and no tuning here: tiles use the tuned parameters of a
// matching batch when the cache has them, else 4 rows per lane and as many
// workgroups per CU as occupancy allows; a group with few rows in all takes
// one row per lane in tiles of whole waves, spread over every workgroup.  Device tables grow by doubling and
// are reused; the state lives until the process ends (the stepper holds
// one, under its lock).

struct FusedState {
    std::vector<Group> groups;
    std::vector<std::vector<Tile>> host_tiles;
    int n_cu = 256;
};

FusedState *fused_create() {
    FusedState *f = new FusedState();
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        hipDeviceGetAttribute(&f->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    return f;
}

namespace {
template <typename T>
void ensure_capacity(T **p, size_t *cap, size_t need) {
    if (need <= *cap) return;
    size_t c = std::max<size_t>(need, *cap * 2 + 16);
    if (*p) LS_HIP_CHECK(hipFree(*p));
    *p = nullptr;
    LS_HIP_CHECK(hipMalloc(p, c * sizeof(T)));
    *cap = c;
}
}  // namespace

void fused_matvec(FusedState *f, uint32_t n, const ls_operator *const *ops, const void *const *xs, void *const *ys,
                  hipStream_t st, HostKeep *keep) {
    for (auto &g : f->groups) {
        g.jobs.clear();
        g.cost.clear();
        g.lds = 0;
    }
    for (uint32_t i = 0; i < n; ++i) {
        const ls_operator *op = ops[i];
        if (op->basis->dim == 0) continue;
        const Variant v = variant_of(op);
        Group *g = nullptr;
        for (auto &gg : f->groups)
            if (gg.v == v) g = &gg;
        if (!g) {
            f->groups.emplace_back();
            g = &f->groups.back();
            g->v = v;
            g->nr = 1;
            LS_HIP_CHECK(hipMalloc(&g->d_counter, sizeof(uint32_t)));
        }
        g->jobs.push_back(job_of(op, xs[i], ys[i], 1, 0));
        g->cost.push_back(static_cast<double>(op->basis->dim) * (op->n_off + 1.0) * op->basis->plan.n_elements);
        g->lds = std::max(g->lds, lds_bytes(v.kind, op->n_diag + op->n_off, op->n_off, op->basis->plan.lx));
    }
    f->host_tiles.resize(f->groups.size());
    for (size_t gi = 0; gi < f->groups.size(); ++gi) {
        Group &g = f->groups[gi];
        if (g.jobs.empty()) continue;
        g.rpl = 4;
        uint32_t wpc = static_cast<uint32_t>(std::max(1, 2048 / block_for(g.v)));   // full occupancy
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(tune_key(g));
            if (it != g_tune_cache.end()) {
                g.rpl = it->second.first;
                wpc = it->second.second;
            }
        }
        // few rows in all (small solves): one row per lane and tiles of whole
        // waves, so that the rows spread over every resident workgroup
        uint64_t total = 0;
        for (const auto &j : g.jobs) total += j.dim;
        const uint64_t block = static_cast<uint64_t>(block_for(g.v));
        const uint64_t slots = static_cast<uint64_t>(f->n_cu) * wpc;
        g.tile_rows = 0;
        if (total < slots * block) {
            g.rpl = 1;
            const uint64_t per = (total + slots - 1) / slots;
            g.tile_rows = static_cast<uint32_t>(std::min<uint64_t>(block, std::max<uint64_t>(64, (per + 63) / 64 * 64)));
        } else {
            // at least one tile per resident workgroup
            g.rpl = static_cast<uint32_t>(std::min<uint64_t>(g.rpl, std::max<uint64_t>(1, total / (slots * block))));
        }
        const uint64_t rows_per_tile = static_cast<uint64_t>(g.tile_rows ? g.tile_rows : block) * g.rpl;
        std::vector<uint32_t> order(g.jobs.size());
        for (uint32_t j = 0; j < order.size(); ++j) order[j] = j;
        std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return g.cost[a] > g.cost[b]; });
        auto &tiles = f->host_tiles[gi];
        tiles.clear();
        for (uint32_t j : order)
            for (uint64_t r = 0; r < g.jobs[j].dim; r += rows_per_tile) tiles.push_back(Tile{j, 0, r});
        ensure_capacity(&g.d_jobs, &g.cap_jobs, g.jobs.size());
        ensure_capacity(&g.d_tiles, &g.cap_tiles, tiles.size());
        // with `keep`, the tables are uploaded from copies that outlive this
        // call (the caller enqueues more work before synchronising)
        const MatvecJob *src_jobs = keep ? keep_copy(*keep, g.jobs.data(), g.jobs.size()) : g.jobs.data();
        const Tile *src_tiles = keep ? keep_copy(*keep, tiles.data(), tiles.size()) : tiles.data();
        LS_HIP_CHECK(hipMemcpyAsync(g.d_jobs, src_jobs, g.jobs.size() * sizeof(MatvecJob), hipMemcpyHostToDevice,
                                    st));
        LS_HIP_CHECK(hipMemcpyAsync(g.d_tiles, src_tiles, tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, st));
        g.n_tiles = static_cast<uint32_t>(tiles.size());
        g.grid = static_cast<uint32_t>(std::min<uint64_t>(static_cast<uint64_t>(f->n_cu) * wpc, g.n_tiles));
        BatchLaunch L{&g, st};
        dispatch(g.v, 1, L);
        LS_HIP_CHECK(hipGetLastError());
    }
}

}  // namespace ls
