// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "ls_ed.h"

namespace ls {

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);
const char *last_error();

struct Error {
    ls_status status;
    std::string msg;
};

#define LS_HIP_CHECK(expr)                                                            \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw ::ls::Error{e_ == hipErrorOutOfMemory ? LS_ENOMEM : LS_EDEVICE,      \
                              std::string(#expr) + ": " + hipGetErrorString(e_)};     \
    } while (0)

#define LS_REQUIRE(cond, msg)                                                         \
    do {                                                                              \
        if (!(cond)) throw ::ls::Error{LS_EINVAL, (msg)};                             \
    } while (0)

// ---------------------------------------------------------------- handle memory
//
// Device memory of library handles is allocated in stream order
// (hipMallocAsync) on the stream of the call that creates it, and released
// with hipFreeAsync on the null stream once every stream the handle was used
// on has drained.  hipFree would wait for the whole device: a handle retired
// beside work on other streams (a build, another solve) would wait for it.

// Allocates `bytes` (at least 1) on `stream`; throws LS_ENOMEM.
void *dev_alloc(size_t bytes, hipStream_t stream);
template <class T>
T *dev_alloc_n(size_t count, hipStream_t stream) {
    return static_cast<T *>(dev_alloc(count * sizeof(T), stream));
}
// Stream-ordered release on `stream` (the null stream once the handle's
// streams have drained); null pointers are ignored.
void dev_free(void *p, hipStream_t stream = nullptr);

// Where a handle's device work ends on each stream it was used on: one
// event per stream, recorded after the last call's work on it.  add() notes
// the stream during a call; the event is recorded when the library call
// returns (flush_marks, after all of the call's work is enqueued), so a
// destroy waits for the handle's own work only, not for what other handles
// enqueue on the same streams later.
struct StreamSet {
    std::mutex mu;
    std::vector<std::pair<hipStream_t, hipEvent_t>> marks;
    void add(hipStream_t s);          // during a call: mark s when it returns
    void mark(hipStream_t s);         // record s's event now
    // Records this thread's pending marks of the set, then waits for every
    // event and releases them.
    void drain();
};
// Records the marks noted by add() during the calling thread's library call.
void flush_marks();

// ---------------------------------------------------------------- group plan
//
// The group is split as G = union over p in P of (Z x T) o p, where
//   T = all translations of an lx-by-ly block layout of the sites
//       (site = x + lx*y; a ring is lx = N, ly = 1; no structure: 1 x 1),
//   Z = {identity, global spin flip F} when F is in G, else {identity},
//   P = one representative per right coset.
// An element is addressed by the code ((p * |T|) + t) * |Z| + f, with
// t = a + lx*b for the translation (x, y) -> (x+a, y+b).  On the device a
// coset representative is applied once (identity, full bit reversal, or a
// Benes network), the translations are then walked with shifts, and the
// flip partner of every image is v ^ full.

constexpr int kMaxStages = 11;

enum CosetKind : uint32_t { kCosetIdentity = 0, kCosetReverse = 1, kCosetBenes = 2 };

struct CosetRep {
    uint32_t kind;      // CosetKind
    uint32_t flip;      // 1: invert all spins after the permutation
    uint64_t masks[kMaxStages];
};

enum ChiMode : int { kChiTrivial = 0, kChiReal = 1, kChiComplex = 2 };

constexpr uint32_t kTorusCosetSlots = 8;   // coset representatives kept per lane

struct GroupPlan {
    uint32_t n_sites = 0;
    uint32_t n_elements = 0;
    uint32_t lx = 1, ly = 1;        // translation layout (1 x 1 = none)
    uint32_t pair_flip = 0;         // Z contains F
    uint32_t n_stages = 0;          // 9 for N <= 32, else 11
    uint64_t full = 0;              // low N bits set
    uint64_t col0 = 0;              // bits of column x = 0 of every row
    int chi_mode = kChiTrivial;
    std::vector<CosetRep> cosets;   // P
    std::vector<double> chi;        // [n_elements][2] by code
    std::vector<uint32_t> chi_one;  // bitset by code: chi == 1
    std::vector<int32_t> code_to_index;  // code -> index in the user's list
    // Pruned torus search (lx <= 6, ly >= 2): for every pair of rows
    // q = (top << lx | second) the smallest x-rotation of the pair, as
    // entry = key << 4 | ambiguous << 3 | argmin_a, stored as
    // entry(q) | entry(q with all bits flipped) << 16.
    bool torus = false;
    std::vector<uint32_t> pair_lut;
    uint64_t col_ge[8] = {};        // bits with x >= a in every row
};

// Validates the descriptor and compiles the plan.  Throws Error.
GroupPlan compile_group(const ls_sector_desc &d);

// Route a bit permutation (bit i -> bit dest[i]) on n = 32 or 64 wires into
// Benes delta-swap masks; returns the number of stages (2 log2 n - 1).
int benes_route(const std::vector<int> &dest, int n, uint64_t *masks);

// Host reference application of a routed network (used for self-checks).
uint64_t benes_apply_host(uint64_t x, const uint64_t *masks, int n_stages, int n);

// ---------------------------------------------------------------- device views

struct PlanDev {
    uint32_t n_sites, lx, ly, n_trans;
    uint32_t n_cosets, pair_flip, n_stages, n_elements;
    uint64_t full, col0;
    const CosetRep *cosets;     // device
    const double2 *chi;         // device, by code
    const uint32_t *chi_one;    // device bitset, by code
    const uint32_t *pair_lut;   // device, torus pruning table (or null)
    uint64_t col_ge[8];
    // Stabilizer-ratio table (0 classes = none): stab_cls[s] is the class of
    // the divisor s of |G|, stab_ratio[a * n_stab_cls + b] the correctly
    // rounded sqrt(d_b / d_a) of classes a and b.
    uint32_t n_stab_cls, pad_;
    const uint8_t *stab_cls;    // device [kStabMapBytes]
    const double *stab_ratio;   // device [n_stab_cls][n_stab_cls]
};

// Stabilizer sizes divide |G|, so the normalisation sqrt(stab_j / stab_i) of
// an element takes one of a few values: groups of at most kStabMapMax
// elements with at most kStabClsMax divisors get the table above, which the
// kernels that use it stage in LDS.
constexpr uint32_t kStabClsMax = 24;
constexpr uint32_t kStabMapMax = 1024;
constexpr size_t kStabMapBytes = kStabMapMax + 8;

// kLookupStaged: the bucket search with its bucket table staged in LDS by
// every workgroup (a layout the batched launch may pick; never built by a
// basis itself).
enum LookupMode : uint32_t {
    kLookupSearch = 0,
    kLookupRank = 1,
    kLookupIdentity = 2,
    kLookupHash = 3,
    kLookupStaged = 4
};
constexpr uint32_t kMaxStagedBits = 13;   // staged tables: at most 2^13 + 1 entries (32 KiB)

// One slot of the hash index: a representative, its position in the sorted
// array and its stabilizer size, read with one 16-byte load.
struct alignas(16) HashSlot {
    uint64_t key;       // kEmptyKey when free
    uint32_t idx;
    uint32_t stab;
};
constexpr uint64_t kEmptyKey = ~0ULL;

struct SearchDev {
    uint32_t mode;      // LookupMode
    uint32_t bits;      // bucket bits
    uint32_t shift;     // bucket = (key - kmin) >> shift
    int32_t weight;     // for rank / identity validation
    uint32_t n_sites;
    uint32_t hash_shift;        // slot = (key * golden) >> hash_shift (hash mode)
    uint32_t n_bkt;             // entries of the bucket table (staged mode)
    uint64_t dim;
    uint64_t kmin, kmax;
    const uint64_t *reps;       // device [dim]
    const uint32_t *buckets;    // device [2^bits + 1]
    const uint64_t *binom;      // device [65][65]
    const HashSlot *table;      // device [hash_mask + 1] (hash mode)
    uint64_t hash_mask;
};

}  // namespace ls

// ---------------------------------------------------------------- handles

struct ls_basis {
    ls::GroupPlan plan;
    mutable ls::StreamSet used;        // streams of the calls that read it
    std::vector<uint16_t> perm_copy;   // the descriptor's group, [nG][N]
    std::vector<uint8_t> flip_copy;    // [nG]
    int32_t weight = -1;
    uint64_t dim = 0;
    int device = 0;
    // device memory
    uint64_t *d_reps = nullptr;
    uint16_t *d_stab = nullptr;
    uint32_t *d_buckets = nullptr;
    ls::HashSlot *d_table = nullptr;
    uint64_t *d_binom = nullptr;
    ls::CosetRep *d_cosets = nullptr;
    double2 *d_chi = nullptr;
    uint32_t *d_chi_one = nullptr;
    uint32_t *d_pair_lut = nullptr;
    void *d_stab_tab = nullptr;
    ls::PlanDev plan_dev{};
    ls::SearchDev search_dev{};
};

struct ls_term_dev {
    double re, im;          // coefficient, already conjugated for the pull form
    uint64_t sel, val, flip, sign;
};

struct ls_operator {
    const ls_basis *basis = nullptr;
    mutable ls::StreamSet used;        // streams of the calls that ran its products
    bool is_complex = false;
    uint32_t n_diag = 0, n_off = 0;
    ls_term_dev *d_terms = nullptr;     // diagonal terms first, then off-diagonal
    std::vector<ls_term_dev> host_terms;
    // torus search: the permutation part of every coset representative
    // applied to every off-diagonal flip mask, [n_off][kTorusCosetSlots]
    std::vector<uint64_t> host_cflip;
    uint64_t *d_cflip = nullptr;
    // error flag: a product met a neighbour whose in-sector representative
    // stateToIndex did not find (set by the kernels, read by ls_operator_check,
    // ls_lanczos, ls_solver_step and ls_operator_store)
    uint32_t *d_err = nullptr;
    // stored elements (ls_operator_store), sliced ELLPACK over 64-row slices
    bool stored = false;
    uint64_t st_slots = 0, st_bytes = 0;
    uint64_t *d_st_off = nullptr;       // [slices] first slot of each slice
    uint32_t *d_st_width = nullptr;     // [slices] elements per row in the slice
    uint32_t *d_st_cols = nullptr;      // [slots] column, or ~0 for none
    void *d_st_vals = nullptr;          // [slots] double or double2 (full values)
    uint8_t *d_st_codes = nullptr;      // [slots] value codes (coded form, real operators)
    uint64_t *d_st_vtab = nullptr;      // [256] the coded form's values (double bit patterns)
    void *d_st_diag = nullptr;          // [dim] diagonal sum, double or double2
};

namespace ls {

// basis.hip
void upload_plan(ls_basis *b, hipStream_t stream);
// Test hook: the representative at `index` is taken out of the hash index
// (its slot keeps a key no lookup asks for), so lookups of it miss.
void drop_key(ls_basis *b, uint64_t index, hipStream_t stream);
// C(N, w) with U(1), else 2^N
uint64_t candidate_count(const ls_basis *b);
void build_basis(ls_basis *b, hipStream_t stream);
// Members among the candidates of colex rank [begin, end) (end clamped to
// the number of candidates); the plan must be uploaded.
uint64_t count_members(ls_basis *b, uint64_t begin, uint64_t end, hipStream_t stream);
// The same count with the compiled group and the accumulator in a static
// device array (no device allocation); *n_candidates = C(N, w) or 2^N.
uint64_t count_members_noalloc(const GroupPlan &gp, int32_t weight, uint64_t begin, uint64_t end,
                               hipStream_t stream, uint64_t *n_candidates);
void launch_state_info(const ls_basis *b, uint64_t n, const uint64_t *states, uint64_t *reps,
                       double *chi, double *norm, hipStream_t stream);
void launch_index_lookup(const ls_basis *b, uint64_t n, const uint64_t *keys, int64_t *index,
                         hipStream_t stream);

// terms.cpp
void compile_terms(const ls_basis *b, uint32_t n_terms, const ls_term *terms, ls_operator *op);

// Records `stream` as used by op and its basis.
void touch(const ls_operator *op, hipStream_t stream);

// matvec.hip
uint32_t matvec_max_terms();   // the term table is staged in LDS
// Waits for `stream`; throws LS_EINTERNAL (clearing the flag) when a product
// of op met a lookup miss of an in-sector representative.
void check_operator(const ls_operator *op, hipStream_t stream);
// Enqueues a copy of op's flag into host memory *dst, then a clear of the
// flag, on `stream` (the caller synchronises before reading *dst).
void enqueue_flag_read(const ls_operator *op, uint32_t *dst, hipStream_t stream);
uint64_t count_elements(const ls_operator *op, hipStream_t stream);
// Orbit search the products of op use (OrbitKind) and whether a torus
// search runs with a compile-time shape.
void search_kind(const ls_operator *op, uint32_t *kind, uint32_t *fixed_shape);
void launch_matvec(const ls_operator *op, uint32_t nrhs, const void *x, void *y, hipStream_t stream);
// Whether a single-column product of op runs in the row-group form (a small
// sector: several lanes per row); such products are not fused.
bool grouped_product(const ls_operator *op);
// Push (transposed, atomic) form of the product; y is zeroed first.
void launch_matvec_push(const ls_operator *op, uint32_t nrhs, const void *x, void *y, hipStream_t stream);
// Stores the operator's elements (at most max_bytes); returns the bytes held.
uint64_t store_elements(ls_operator *op, uint64_t max_bytes, hipStream_t stream);
void launch_stored(const ls_operator *op, uint32_t nrhs, const void *x, void *y, hipStream_t stream);

// batch.hip
void batch_create(uint32_t n, const ls_operator *const *ops, const uint32_t *nrhs, ls_batch **out);
void batch_destroy(ls_batch *b);
void batch_matvec(ls_batch *b, const void *const *xs, void *const *ys, hipStream_t stream);
void batch_info(const ls_batch *b, uint32_t *n_launches, uint32_t *n_tiles, uint32_t *graph);
void batch_set_graph(ls_batch *b, bool on);
void batch_set_search(ls_batch *b, int mode, uint32_t bits);
void batch_search(const ls_batch *b, uint32_t item, uint32_t *mode, uint32_t *bits, double *own_ns, double *chosen_ns,
                  double *staged_ns);

// fused products over a changing set of operators (batch.hip)
struct FusedState;
FusedState *fused_create();
// Host bytes of uploads enqueued before a synchronisation, kept alive (and
// unchanged) until it: the copies read them in stream order.
using HostKeep = std::vector<std::vector<unsigned char>>;
template <class T>
const T *keep_copy(HostKeep &keep, const T *data, size_t count) {
    const unsigned char *b = reinterpret_cast<const unsigned char *>(data);
    keep.emplace_back(b, b + count * sizeof(T));
    return reinterpret_cast<const T *>(keep.back().data());
}
void fused_matvec(FusedState *f, uint32_t n, const ls_operator *const *ops, const void *const *xs,
                  void *const *ys, hipStream_t stream, HostKeep *keep = nullptr);

// Lanczos stepper (lanczos.hip)
uint64_t solver_footprint(const ls_operator *op, uint32_t max_iter);
ls_solver *solver_create(const ls_operator *op, const ls_lanczos_opts *o, hipStream_t stream);
void solver_destroy(ls_solver *s);
void solver_step(ls_solver *const *solvers, uint32_t n, uint32_t steps, hipStream_t stream);
void solver_result(const ls_solver *s, double *e0, uint32_t *iters, double *resid, int *done, int *converged);
bool solver_failed(const ls_solver *s);   // stopped by a lookup miss in its product

// lanczos.hip
ls_status run_lanczos(const ls_operator *op, const ls_lanczos_opts *o, hipStream_t stream,
                      double *e0, uint32_t *iters, double *resid);

}  // namespace ls
