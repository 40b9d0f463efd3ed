/*
 * ls_ed.h -- symmetry-adapted exact diagonalization on one MI355X (gfx950).
 *
 * The problem statement follows Westerhout & Chamberlain, "Implementing
 * scalable matrix-vector products for the exact diagonalization methods in
 * quantum many-body physics" (PAW-ATM'23):
 *   - basis states are N-bit strings; with symmetries a basis index is not
 *     the bitstring itself (Section 2.1, Fig. 1);
 *   - U(1) fixes the Hamming weight (Section 2.1);
 *   - lattice symmetries (translations, reflections, spin inversion) keep one
 *     representative per orbit (Section 2.1; benchmark symmetries in
 *     Section 6, "Test Hamiltonians");
 *   - the product is y_i = sum_j H_ij x_j with matrix elements computed on
 *     the fly from basis states, and stateToIndex mapping a state to its
 *     index in the sorted list of representatives (Section 5.3).
 *
 * Conventions fixed by this library (the paper leaves them open):
 *   - bit i of a state is site i; a set bit is an up spin;
 *   - a group element g = (perm, flip) sends bit i to bit perm[i], then
 *     inverts all N bits if flip != 0; (g h).s = g.(h.s);
 *   - the representative of s is the minimum of its orbit {g.s};
 *   - the sector is the common eigenspace U_g psi = chi(g) psi, i.e. the
 *     image of P = (1/|G|) sum_g conj(chi(g)) U_g; its basis vectors are
 *     P|r>/||P|r>|| for representatives r with P|r> != 0.
 *
 * Memory: arguments named d_* are device pointers (HBM of the current
 * device) owned by the caller; work is enqueued on `stream` (a hipStream_t
 * passed as void*; NULL = the default stream) and is complete when the
 * stream is.  Descriptors and term tables are host memory, read during the
 * call only.  Handles are owned by the library, immutable after creation
 * (ls_operator_store excepted: it adds the stored form to an operator), and
 * freed with the matching *_destroy.  Calls on different streams may
 * overlap; a handle may be shared by concurrent calls.
 *
 * Destruction: handle memory is stream-ordered (hipMallocAsync).  Each
 * call that uses a handle records, on its stream, an event after the work it
 * enqueued (a basis and an operator also for the calls that used an
 * operator, solver or batch built on them); *_destroy waits for those events
 * only -- the handle's own work, not the whole device nor later work on the
 * same streams -- and then releases the memory.  Destroy a handle before the
 * streams it ran on.
 *
 * Errors: every call returns ls_status.  No exception crosses this boundary.
 * On LS_EINVAL nothing has been enqueued and out-parameters are untouched.
 * ls_last_error() returns a thread-local message for the last failure.
 */
#ifndef LS_ED_H
#define LS_ED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LS_OK = 0,
    LS_WNOTCONV = 1,     /* outputs valid, tolerance not reached */
    LS_EINVAL = -1,      /* invalid argument; nothing enqueued */
    LS_ENOMEM = -2,      /* device allocation failed */
    LS_EDEVICE = -3,     /* a HIP runtime call failed */
    LS_EINTERNAL = -4    /* an internal consistency check failed */
} ls_status;

typedef struct ls_basis ls_basis;
typedef struct ls_operator ls_operator;

/* A symmetry sector.
 *   n_sites         N, 1..64.
 *   hamming_weight  w in 0..N, or -1 for no U(1) restriction (then N <= 36).
 *   n_elements      |G|, 1..4096; the elements must form a group (closed
 *                   under composition, containing the identity, no
 *                   duplicates).
 *   perm            host, [n_elements][n_sites] uint16: bijections of sites.
 *   flip            host, [n_elements] uint8: 1 = also invert all spins;
 *                   needs 2w = N when w >= 0.
 *   chi             host, [n_elements][2] double (re, im): a one-dimensional
 *                   representation, chi(gh) = chi(g) chi(h) within 1e-9.   */
typedef struct {
    uint32_t n_sites;
    int32_t hamming_weight;
    uint32_t n_elements;
    const uint16_t *perm;
    const uint8_t *flip;
    const double *chi;
} ls_sector_desc;

/* One elementary term of H (the "sum of bit-flip and diagonal spin terms"):
 *   c * sum over s with (s & sel_mask) == sel_value of
 *       (-1)^popcount(s & sign_mask) |s ^ flip><s|,      c = re + i im.
 * flip == 0 is a diagonal term.  The term list as a whole must be Hermitian
 * and commute with every group element; with U(1) every off-diagonal term
 * needs flip subset of sel_mask and must conserve the Hamming weight.      */
typedef struct {
    double re, im;
    uint64_t sel_mask, sel_value;
    uint64_t flip;
    uint64_t sign_mask;
} ls_term;

/* Build the sorted list of representatives of a sector (Section 5.2:
 * iterate over all candidate bitstrings, keep those that satisfy the
 * representative condition; here every weight-w bitstring in increasing
 * order, kept iff it is its orbit's minimum and P does not annihilate it).
 * The handle owns reps (uint64 [dim], strictly increasing), their
 * stabilizer sizes and the search layout used by ls_index_lookup and the
 * products (stateToIndex, Section 5.3): a hash index of 16-byte slots
 * (key, index, stabilizer size; linear probing from the key's Fibonacci
 * hash, the top bits of key * 0x9E3779B97F4A7C15; load factor at most 1/8
 * while the table fits 8 GiB, else 1/4 within 64 GiB, else 1/2 or 3/4
 * within 128 GiB), or, where it would pass 128 GiB or the
 * environment variable LS_ED_SEARCH is "buckets" at build time, a bucket
 * table over the keys' high bits with binary search in reps.  A group of
 * one element needs neither (colex rank, or the state itself).
 * Blocks until the build on `stream` has finished.  Indices are 32-bit:
 * sectors of 2^32 - 1 or more representatives are refused (count them with
 * ls_sector_count).
 * Errors: LS_EINVAL (invalid descriptor: see ls_sector_desc), LS_ENOMEM,
 * LS_EDEVICE, LS_EINTERNAL (a group-compiler self-check failed).          */
ls_status ls_basis_build(const ls_sector_desc *desc, void *stream, ls_basis **out);

/* Count-only enumeration: the filter of ls_basis_build (Section 5.2) over
 * the candidates whose rank lies in [rank_begin, rank_end), without storing
 * anything; it gives the sector dimensions of Section 6, Table 2, for
 * sectors whose representatives would not fit in memory.  The rank of a
 * candidate is its colex rank among the weight-w bitstrings (with U(1)) or
 * the bitstring itself (without); rank_end is clamped to the number of
 * candidates, so rank_end = UINT64_MAX counts the whole sector, and
 * consecutive ranges add up (callers may split the range to report
 * progress).  Outputs (host): *n_members, and *n_candidates = C(N, w) or
 * 2^N (may be NULL).  Blocks until the count on `stream` has finished;
 * device scratch is 8 bytes plus the compiled group.
 * Errors: as ls_basis_build; LS_EINVAL also for rank_begin > rank_end.   */
ls_status ls_sector_count(const ls_sector_desc *desc, uint64_t rank_begin, uint64_t rank_end,
                          uint64_t *n_members, uint64_t *n_candidates, void *stream);

/* ls_sector_count without device allocation, for callers that cannot
 * allocate device memory (tight loops that must not call hipMalloc,
 * harnesses that forbid it).  Same arguments, results and errors as
 * ls_sector_count.  The compiled group's device tables and the 8-byte
 * accumulator live in a static device array of 256 KiB that each GPU the
 * library runs on holds until the process ends (groups whose tables need
 * more -- binomial table, coset representatives at 96 bytes each,
 * characters at 16 bytes per element, the torus pair table -- are refused
 * with LS_EINVAL; groups with lattice translations need a few KB).  No
 * hipMalloc, hipFree or other device allocation is made.  Every call on a
 * GPU shares that GPU's array and overwrites what the last call left:
 * calls from one process are serialised by a lock inside the library;
 * overlapping calls from several processes on one GPU use separate arrays.
 * Blocks until the count on `stream` has finished.                         */
ls_status ls_sector_count_noalloc(const ls_sector_desc *desc, uint64_t rank_begin, uint64_t rank_end,
                                  uint64_t *n_members, uint64_t *n_candidates, void *stream);

/* Validates a sector descriptor and compiles its group on the host only (no
 * device work): the checks of ls_basis_build plus the group compiler's own
 * self-checks (Benes routing verified on every wire).  Optional outputs
 * (any may be NULL): the translation layout found, lx * ly = n_sites or
 * 1 x 1 when the group has no full set of lattice translations; whether
 * the global spin flip pairs images; the number of coset representatives
 * walked per orbit search.                                                 */
ls_status ls_sector_check(const ls_sector_desc *desc, uint32_t *lx, uint32_t *ly, uint32_t *pair_flip,
                          uint32_t *n_cosets);

/* Dimension, whether vectors are real (all chi real), and the device array
 * of representatives (borrowed; valid until ls_basis_destroy).  Any output
 * pointer may be NULL.                                                     */
ls_status ls_basis_info(const ls_basis *basis, uint64_t *dim, int *is_real,
                        const uint64_t **d_reps);

/* Copies the representatives (uint64 [dim]) and their stabilizer sizes
 * (uint16 [dim], the number of group elements fixing each) into caller
 * buffers on `stream`.  Either destination may be NULL.                   */
ls_status ls_basis_copy(const ls_basis *basis, uint64_t *d_reps_out, uint16_t *d_stab_out, void *stream);

/* Waits for the basis's work on every stream it was used on, then frees it. */
void ls_basis_destroy(ls_basis *basis);

/* Test hook for the lookup-miss error path (host-forced fault injection):
 * takes the representative at position `index` out of the basis's hash
 * index, so ls_index_lookup returns -1 for it and every product that meets
 * it raises its operator's error flag (ls_operator_check).  The basis is
 * changed for good: use it on a basis built for the purpose.  Blocks until
 * done on `stream`.
 * Errors: LS_EINVAL (NULL basis, index >= dim, a search layout other than
 * the hash index, or no unused key value above the representatives).      */
ls_status ls_basis_test_drop_key(ls_basis *basis, uint64_t index, void *stream);

/* Per state: its representative (orbit minimum), the character chi(g*) of
 * an element g* with g*.s = rep, and norm = sqrt(stab/|G|) with stab the
 * stabilizer size (the norm of P|rep>).  A state of the wrong Hamming
 * weight or whose orbit P annihilates gets chi = 0 and norm = 0; a state
 * with bits at or above N is returned unchanged with chi = norm = 0.
 *   d_states  device uint64 [n]        (in)
 *   d_reps    device uint64 [n]        (out)
 *   d_chi     device double [n][2]     (out, re/im)
 *   d_norm    device double [n]        (out)
 * n may be 0.  Errors: LS_EINVAL (NULL handle or NULL pointer with n > 0). */
ls_status ls_state_info(const ls_basis *basis, uint64_t n, const uint64_t *d_states,
                        uint64_t *d_reps, double *d_chi, double *d_norm, void *stream);

/* stateToIndex (Section 5.3): position of each representative in the sorted
 * list, or -1 when the value is not in it (not an error).
 *   d_keys   device uint64 [n] (in);  d_index  device int64 [n] (out).     */
ls_status ls_index_lookup(const ls_basis *basis, uint64_t n, const uint64_t *d_keys,
                          int64_t *d_index, void *stream);

/* Compile a term list into an operator on the basis's sector.  Validates
 * Hermiticity of the term set, weight conservation (with U(1)) and
 * invariance of the term set under every group element (after merging
 * equal terms), else LS_EINVAL.  The operator borrows the basis, which
 * must outlive it.                                                         */
ls_status ls_operator_create(const ls_basis *basis, uint32_t n_terms, const ls_term *terms,
                             ls_operator **out);
/* Waits for the operator's work on every stream it was used on, then frees it. */
void ls_operator_destroy(ls_operator *op);

/* Whether the operator acts on complex vectors (complex characters or
 * complex coefficients).                                                   */
ls_status ls_operator_info(const ls_operator *op, int *is_complex, uint64_t *dim);

/* Stores the operator's matrix elements in device memory, so that later
 * products read them instead of regenerating them.  The paper generates
 * elements on the fly because a stored H does not fit its machines
 * (Section 2.2); where it fits one GPU, a stored product is bound by memory
 * traffic rather than by the orbit searches.  Layout: sliced ELLPACK over
 * slices of 64 consecutive rows (a uint32 column per slot, plus each row's
 * diagonal sum); a real operator with at most 256 distinct element values
 * stores a one-byte code per slot into a table of those values (5 bytes a
 * slot), otherwise each slot holds its double / complex128 value.
 *   max_bytes  refuse (LS_ENOMEM, operator unchanged) if the stored form
 *              would need more device memory than this.
 *   bytes      out (may be NULL): device bytes held by the stored form.
 * Afterwards ls_matvec, ls_lanczos and ls_solver_step use the stored
 * elements (in a step over several solves a stored solve takes its own
 * stored product beside the fused launch of the others); ls_batch_matvec
 * keeps generating them.  Both
 * forms run the same row arithmetic in the same order and give identical
 * results bit for bit.  Storing again is a no-op.  This call changes the
 * operator: make it before the handle is shared by concurrent calls.
 * Blocks until the store on `stream` has finished; costs about one product.
 * Errors: LS_EINVAL (NULL operator), LS_ENOMEM, LS_EDEVICE, LS_EINTERNAL
 * (the store met a lookup miss of an in-sector representative; nothing is
 * kept).                                                                   */
ls_status ls_operator_store(ls_operator *op, uint64_t max_bytes, void *stream, uint64_t *bytes);

/* Number of off-diagonal element applications of one product: the sum over
 * rows of the off-diagonal terms acting on the row's representative.  A
 * product applies this many off-diagonal elements plus one diagonal element
 * per row.  Runs on `stream` and blocks until the count is known.          */
ls_status ls_operator_count(const ls_operator *op, uint64_t *n_offdiag, void *stream);

/* The orbit search (the representative of each generated state, Section
 * 5.2's condition applied to a neighbour) that the products of op run:
 * kind 0 the general walk over coset representatives, 1 rings of at most 32
 * sites (rotations of a doubled word), 2 tori (pair-table pruned search),
 * 3 rings of 33 to 63 sites (longest-zero-run candidates); fixed_shape 1
 * when a torus search runs with a compile-time layout (6x6 or 4x4 with the
 * full point group and spin inversion).  For an operator with stored
 * elements (ls_operator_store) it is the search the store ran; its products
 * read the stored elements.  Either output may be NULL.  A query only: it
 * launches nothing.  Errors: LS_EINVAL (NULL operator).                    */
ls_status ls_operator_search_kind(const ls_operator *op, uint32_t *kind, uint32_t *fixed_shape);

/* y = H x (Section 5.3, the first listing's row-by-row ("pull") form: each
 * row's elements are generated from its representative, looked up, and
 * accumulated; no atomics, since H is Hermitian).  Each row is summed in
 * term order, diagonal first, whatever the launch shape: a single column of
 * a small sector (below 2^18 rows on tori, 2^16 otherwise) gives each row
 * several lanes that generate its elements in parallel and add them in that
 * order, so the results are the same bits as the one-lane form.
 *   nrhs   1..64 right-hand sides.
 *   d_x    device [dim][nrhs], row-major; double, or complex128 as (re, im)
 *          pairs when the operator is complex.  (in)
 *   d_y    same shape, must not overlap d_x.  (out)
 * Errors: LS_EINVAL (NULL handle or vector, nrhs out of range, x and y
 * overlapping).  A neighbour whose representative is not in the basis
 * contributes zero when its orbit is annihilated by the projector (an
 * element fixing it has a character other than 1).  Any other miss -- a
 * representative of the sector that stateToIndex does not find, which
 * Section 5.3's lookup presumes cannot happen -- raises the operator's
 * device error flag; the call itself returns before the product has run,
 * and the flag is reported by the next ls_operator_check (or ls_lanczos,
 * ls_solver_step, ls_operator_store) on the operator.                      */
ls_status ls_matvec(const ls_operator *op, uint32_t nrhs, const void *d_x, void *d_y, void *stream);

/* Waits for `stream`, then reports whether a product of op (ls_matvec,
 * ls_matvec_push, batched or fused products) since the last check met a
 * neighbour whose representative lies in the sector but is missing from
 * the basis (an inconsistent basis or search layout: Section 5.3's
 * stateToIndex presumes every such state is present).  Clears the flag.
 * The flag belongs to the operator: calls on several streams that share an
 * operator share it.  Returns LS_OK, or LS_EINTERNAL when the flag was set
 * (the products' outputs are then not valid).                              */
ls_status ls_operator_check(const ls_operator *op, void *stream);

/* y = H x in the push (transposed) form of Section 5.3's second listing, a
 * comparison variant of ls_matvec: each row's elements H_ij are generated
 * as for ls_matvec and conj(H_ij) x_i is added into y_j with device-scope
 * atomic adds (y is zeroed first, on `stream`).  Arguments, layouts and
 * errors as ls_matvec.  The order of the adds into one y_j varies between
 * runs, so results agree with ls_matvec to rounding, not bit for bit.
 * The elements are always generated (a stored form is not used).          */
ls_status ls_matvec_push(const ls_operator *op, uint32_t nrhs, const void *d_x, void *d_y, void *stream);

/* ---- batched products ------------------------------------------------------
 * Many products y_k = H_k x_k (k = 0..n-1) over operators of different
 * sectors, couplings and dimensions, each with its own number of right-hand
 * sides, executed as one persistent launch per kernel variant (operators on
 * the same kind of lattice share a launch).  The paper computes many rows at
 * once to amortise per-call costs (getManyRows, Section 5.3); here many
 * products share one launch, a tile queue balances uneven dimensions, and
 * the launch sequence is captured in a HIP graph and replayed.
 * On the first ls_batch_matvec the library tunes, per variant, the tile size
 * and grid size (timing candidates on the caller's buffers; y is written
 * during tuning) and, per basis, the search layout (stateToIndex, Section
 * 5.3): the fastest by a timed lookup sweep of the basis's own layout (hash
 * index or bucket search), bucket tables of several sizes over the keys'
 * high bits searched in global memory, and bucket tables staged in LDS by
 * every workgroup (the prefix-bucketed search of the sorted representatives
 * with its first level in LDS), owned by the batch; the choices are cached
 * per process.  Elements are always generated (a
 * stored form is not used); results equal ls_matvec's bit for bit.  The
 * batch borrows the operators, which must outlive it.                       */
typedef struct ls_batch ls_batch;

/*   ops   host array of n operator handles (may repeat);
 *   nrhs  host array of n right-hand-side counts, each 1..64.              */
ls_status ls_batch_create(uint32_t n, const ls_operator *const *ops, const uint32_t *nrhs, ls_batch **out);

/* y_k = H_k x_k for every k, enqueued on `stream`.
 *   d_x, d_y  host arrays of n device pointers, laid out as for ls_matvec
 *             ([dim_k][nrhs_k], double or complex128); y_k must not overlap
 *             x_k.  Pointers may change between calls (the job tables the
 *             graph reads are rewritten, stream-ordered).                  */
ls_status ls_batch_matvec(ls_batch *batch, const void *const *d_x, void *const *d_y, void *stream);

/* Launches per call (one per variant and column width), tiles, and whether
 * a captured graph is in use.  Any output may be NULL.                     */
ls_status ls_batch_info(const ls_batch *batch, uint32_t *n_launches, uint32_t *n_tiles, uint32_t *graph);

/* The search layout the batch uses for operator `item` (valid after the
 * first ls_batch_matvec; before it, or for a basis without a search, the
 * basis's own layout with zero times):
 *   mode       0 bucket search in global memory, 1 colex rank, 2 identity,
 *              3 hash index, 4 bucket table staged in LDS;
 *   bits       bucket bits (modes 0 and 4);
 *   own_ns     lookup sweep time per key of the basis's own layout;
 *   chosen_ns  the same for the chosen layout;
 *   staged_ns  the best staged candidate's (0 when none fit in LDS).
 * Any output may be NULL.  Errors: LS_EINVAL for item >= n.               */
ls_status ls_batch_search(const ls_batch *batch, uint32_t item, uint32_t *mode, uint32_t *bits, double *own_ns,
                          double *chosen_ns, double *staged_ns);

/* Fixes the search layout of every basis of the batch instead of tuning it,
 * before the first ls_batch_matvec: mode -1 tunes (default), 0 a bucket
 * table of 2^bits buckets in global memory (bits 1..30), 3 each basis's own
 * layout, 4 a bucket table of 2^bits buckets staged in LDS (bits 1..13).
 * Bases without a search (colex rank, identity) keep theirs.  Errors:
 * LS_EINVAL for other values or after the first product; a staged table
 * that does not fit in LDS beside a job's tables fails the first
 * ls_batch_matvec with LS_EINVAL.                                          */
ls_status ls_batch_set_search(ls_batch *batch, int mode, uint32_t bits);

/* Turns graph capture on (default) or off (direct launches) before the
 * first ls_batch_matvec.                                                   */
ls_status ls_batch_set_graph(ls_batch *batch, int enabled);

/* Waits for the batch's products, then frees it. */
void ls_batch_destroy(ls_batch *batch);

/* Lanczos ground-state solve on top of ls_matvec.  FP64 throughout, Krylov
 * vectors resident in HBM, dot products reduced in a fixed order
 * (deterministic).
 *   max_iter  Krylov dimension cap (>= 1; clipped to dim).
 *   reorth    0: none.  1: full CGS2, two classical Gram-Schmidt passes
 *             against every stored Krylov vector at every step.  2: the
 *             second pass only when the first removed more than half of
 *             ||w||^2 (the criterion of Daniel, Gragg, Kaufman and Stewart,
 *             1976), decided on the device.  Other values: LS_EINVAL.
 *   tol       0: run exactly max_iter steps.  > 0: stop when successive
 *             lowest Ritz values differ by < tol*max(1,|E0|) and the residual
 *             bound beta |s_last| < sqrt(tol)*max(1,|E0|).
 *   seed      start vector entry i = 2u-1 with u from the counter generator
 *             of the paper's hash64_01 (value c of stream seed is
 *             hash64_01(seed + (c+1)*0x9E3779B97F4A7C15), top 53 bits);
 *             complex entries take counters 2i (re) and 2i+1 (im).
 *   d_v0      optional device start vector (dim entries, double or complex
 *             as for ls_matvec); overrides seed when not NULL.
 * Outputs (host): lowest Ritz value, steps taken, residual bound; alpha and
 * beta (host arrays of max_iter doubles, may be NULL) receive the
 * tridiagonal coefficients (beta[k] couples steps k and k+1).
 * Returns LS_OK, LS_WNOTCONV (tol > 0 not reached), or an error.           */
typedef struct {
    uint32_t max_iter;
    uint32_t reorth;
    double tol;
    uint64_t seed;
    const void *d_v0;
    double *alpha;
    double *beta;
} ls_lanczos_opts;

ls_status ls_lanczos(const ls_operator *op, const ls_lanczos_opts *opts, void *stream,
                     double *e0, uint32_t *iters, double *resid_bound);
/* (ls_lanczos also returns LS_EINTERNAL, at the step where it happens, when
 * a product met a lookup miss of an in-sector representative.)             */

/* ---- Lanczos stepper for serving ------------------------------------------
 * A solver holds one Lanczos solve (the recurrence, start vector, stop rule
 * and arithmetic of ls_lanczos) with its Krylov vectors resident in HBM.
 * ls_solver_step advances every listed solver that is not done by one
 * iteration: the products of several solves run as one fused launch (the
 * batched kernel; a single solve takes ls_matvec's launch, as does a solve
 * on a small sector, whose rows ls_matvec spreads over several lanes each;
 * a solve whose operator holds stored elements takes its stored product),
 * alpha and beta stay on the device, and the step ends with one
 * synchronisation.  A solve stepped alone or among others produces the same
 * numbers.  Calls to ls_solver_step(_n) are serialised inside the library. */
typedef struct ls_solver ls_solver;

/* Device bytes a solver for `op` with `max_iter` steps allocates.          */
ls_status ls_solver_footprint(const ls_operator *op, uint32_t max_iter, uint64_t *bytes);

/* Allocates the Krylov space and normalises the start vector (blocks).
 * opts: as for ls_lanczos (alpha/beta outputs are ignored).
 * Errors: LS_EINVAL, LS_ENOMEM when the Krylov space does not fit.         */
ls_status ls_solver_create(const ls_operator *op, const ls_lanczos_opts *opts, void *stream, ls_solver **out);

/* One iteration for each of the n solvers (host array; done ones skipped).
 * A solve whose product met a lookup miss of an in-sector representative
 * (see ls_operator_check) is stopped without taking the step; the other
 * solves complete theirs, and the call returns LS_EINTERNAL naming how many
 * were stopped (ls_solver_result tells which).                             */
ls_status ls_solver_step(ls_solver *const *solvers, uint32_t n, void *stream);

/* Up to `steps` (1..1024) iterations of each of the n solvers, enqueued back
 * to back with one synchronisation at the end (the kernels of a step read
 * alpha and beta on the device, so the steps need nothing from the host in
 * between).  The host bookkeeping then replays the steps in order and stops
 * every solve where single ls_solver_step calls would have stopped, with the
 * same numbers; a solve that stops inside the chunk has had the rest of the
 * chunk's steps computed and discarded (at most steps - 1 products).  The
 * chunk is cut short to the fewest steps any listed solve has left before
 * max_iter.  Errors as ls_solver_step.                                     */
ls_status ls_solver_step_n(ls_solver *const *solvers, uint32_t n, uint32_t steps, void *stream);

/* Current lowest Ritz value, steps taken, residual bound, whether the solve
 * is finished (converged, max_iter reached, Krylov space exhausted, or
 * stopped) and whether the tolerance was met.  Any output may be NULL.
 * Returns LS_EINTERNAL (outputs filled as they stand) for a solve that
 * ls_solver_step stopped because its product met a lookup miss.           */
ls_status ls_solver_result(const ls_solver *solver, double *e0, uint32_t *iters, double *resid_bound, int *done,
                           int *converged);

/* Waits for the solver's steps, then frees it. */
void ls_solver_destroy(ls_solver *solver);

/* Thread-local description of the last non-OK status. */
const char *ls_last_error(void);

/* Library version string. */
const char *ls_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LS_ED_H */
