/*
 * fciqmc.h -- C ABI of the MI355X (gfx950) FCIQMC hot-path library.
 *
 * The library advances the FCIQMC projector iteration of the Rimu.jl paper
 * (arXiv 2601.19505) on one GPU:
 *
 *   c^(n+1) = Pi[ (1 + dtau (S^(n) - H~)) c^(n) ]          (Sec. 3.2, Eqs.
 *             fciqmc-stochastic and stochasticTransitionOperator)
 *   S^(n+1) = S^(n) - (zeta/dtau) ln(N^(n+1)/N^(n))
 *                   - (xi/dtau)  ln(N^(n+1)/N_t)            (Sec. 3.1, Eq. shift-update)
 *
 * for the 1D periodic Bose-Hubbard Hamiltonian in real space (Sec. 2, Eq.
 * bose-hubbard-hamiltonian) or in momentum space (HubbardMom1D, Sec. 6.3),
 * acting matrix-free on bit-packed bosonic Fock addresses (Sec. 6.1).  One
 * step is: per occupied address, stochastic or exact off-diagonal spawning
 * (matrix compression, Eq. column-compression; exact columns per the
 * semistochastic threshold of Sec. 7.1) and the diagonal death/cloning;
 * annihilation by summing all contributions per address (Sec. 3.2); late
 * stochastic vector compression with threshold theta (Eq. vec-compression,
 * Sec. 7.1); the shift update and the projected-energy numerator y^T H c and
 * denominator y^T c for a one-address reference vector y (Sec. 4.2, Eq.
 * ProjectedEnergy).
 *
 * Addresses.  A Fock state |n_1 .. n_M> is its unary bitstring of N+M-1 bits
 * (Sec. 6.1): n_1 ones in the lowest bits, a zero separator, n_2 ones, ...
 * It is passed as `addr_words` (W = 1 or 2) little-endian 64-bit words per
 * address; word 0 holds bits 0..63.  W = 1 requires N+M-1 <= 62, W = 2
 * requires N+M-1 <= 126.  The results never depend on W.
 *
 * Memory.  The caller owns all memory.  Device memory is one workspace of
 * fq_workspace_size() bytes (any 256-byte aligned device allocation); the
 * library never allocates or frees device memory (it keeps small host-side
 * bookkeeping only).  Host arrays passed in are read or written during the
 * call and not retained.  `stream` is a hipStream_t (NULL = default
 * stream); every call enqueues its work on that stream and returns after the
 * work it reports on has completed.
 *
 * Errors.  Every function returns an fq_status.  No exception crosses the
 * ABI.  A failed step (capacity overflow, divergence) leaves the handle at
 * the last completed step, so the caller can enlarge the workspace (or
 * re-create with more buckets), set the state again and continue; because
 * all random numbers are counter-based, the retried step is identical.
 * fq_last_error() returns a human-readable description of the last failure.
 *
 * Determinism.  Given (Hamiltonian, parameters, state, step index, seed) the
 * result is bit-identical regardless of bucket count, LDS table size,
 * workgroup size, launch order, or other instances sharing a batch:
 * random numbers are Philox4x32-10 draws keyed on (seed, step, address,
 * attempt), and every sum (annihilation, norm, projected energy) is an exact
 * fixed-point integer sum rounded once to the nearest double.
 */
#ifndef FCIQMC_H
#define FCIQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FQ_OK = 0,
    FQ_EINVAL = -1,     /* invalid argument (parameters, sizes, addresses)      */
    FQ_ECAPACITY = -2,  /* a table, spawn slab or LDS bucket overflowed         */
    FQ_EHIP = -3,       /* a HIP runtime call failed                            */
    FQ_ENOMEM = -4,     /* workspace smaller than fq_workspace_size() / host    */
    FQ_EBUSY = -5,      /* server: no slot or budget for the request now        */
    FQ_EDIVERGED = -6,  /* walker number overflowed or became non-finite        */
    FQ_ENOTFOUND = -7   /* server: unknown request id                           */
} fq_status;

typedef enum { FQ_REAL1D = 0, FQ_MOM1D = 1, FQ_REAL2D = 2 } fq_model;

/* Hamiltonian (Sec. 2 and Sec. 6.2): model, M modes, N bosons, hopping t,
 * on-site interaction u.  Momentum space requires M >= 3.
 *
 * FQ_REAL2D is the Bose-Hubbard model on a periodic lx x (M / lx) square
 * lattice (lx >= 2, M / lx >= 2; the workload of the benchmarks of Sec. 7.2),
 * sites numbered x + lx y in address order.  Column entry k = dir o + i
 * moves one boson from the i-th occupied site to its neighbour in direction
 * dir = +x, -x, +y, -y (o = occupied sites; the ring has +x, -x), so a
 * lattice 2 sites wide has each of those bonds twice.  lx is ignored by the
 * other models.
 *
 * g: Gutzwiller importance sampling of the real-space models (Sec. 3.3, a
 * similarity transformation by a diagonal matrix; Sec. 7.2): the sampled
 * Hamiltonian is G H G^-1 with G = diag(exp(-g H_ii)), so a hop that moves a
 * boson from a site holding n to one holding nd carries the factor
 * exp(-(g u)(nd - n + 1)).  The walkers sample G c; the shift and the
 * projected energy (with the row of G H G^-1) estimate the same energy.
 * g = 0 is plain sampling; the momentum model requires g = 0. */
typedef struct {
    int32_t model, M, N, lx;
    double t, u, g;
} fq_hamiltonian;

/* Flags of fq_params.flags */
#define FQ_FLAG_DUMP_SPAWNS 1   /* record every spawn event (parity testing)      */
#define FQ_FLAG_DUMP_MERGED 2   /* record every merged pre-compression amplitude  */
#define FQ_FLAG_PHASE_TIMING 4  /* accumulate per-phase timers (diagnostics)      */
/* Early compression (Sec. 7.1, Eq. early-comp): the compression rule of Eq.
 * vec-compression is applied to every contribution before annihilation --
 * the diagonal survivor (draw tag 2, block 0, keyed by its address) and each
 * spawn attempt k (tag 4 + (k >> 28), block k mod 2^28, keyed by the
 * parent) -- instead of to the sums (late compression, the default).
 * Contributions compressed to 0 are not spawn events. */
#define FQ_FLAG_EARLY_COMPRESSION 32
/* Stability check of dtau (Sec. 3.1, the projector is stable for
 * dtau < 2 / (E_max - E_0)).  Creation fails with FQ_EINVAL unless
 * dtau * Wb < 2, where Wb = |u| N (N - 1) / 2 + 2 z |t| N (z = 2 on the ring
 * and in momentum space, 4 on the square lattice) bounds E_max - E_0 from
 * above (Weyl's inequality for the hopping and interaction terms).  This
 * flag skips the check, for callers who know their walkers never reach the
 * high-energy states the bound guards against. */
#define FQ_FLAG_UNCHECKED_DTAU 64
/* Initiator approximation (named in Sec. 1 and in the sign-problem paragraph
 * of Sec. 3.2 with Cleland, Booth and Alavi cited; the paper does not state
 * the rule, this is their original rule for real coefficients): an entry of
 * c^(n) is an initiator when |c| > fq_params.initiator_threshold (n_a).  A
 * spawn of a non-initiator counts only when its destination is an address of
 * c^(n); otherwise it is discarded before annihilation.  Survivors and
 * spawns of initiators always count; every address of c^(n) takes part in
 * the merge even when its survivor is exactly 0, so the merged dump lists
 * it.  Spawn events are generated, dumped and counted in `spawns` as without
 * the rule.  n_a = 0 gives the plain step; n_a = +infinity never grows the
 * support.  Creation fails with FQ_EINVAL when n_a is negative or NaN. */
#define FQ_FLAG_INITIATOR 128
/* Sampled dumps: with FQ_FLAG_DUMP_SAMPLE(k), k in 1..20, the dumps keep only
 * the spawn events whose destination, and the merged amplitudes whose
 * address, fall in a fixed sample of about 2^-k of all addresses (bits
 * 24..24+k-1 of the address hash are zero).  Every event into a sampled
 * address is kept, so sums per sampled address can be checked. */
#define FQ_FLAG_DUMP_SAMPLE(k) ((k) << 8)

/* Algorithm parameters.  dtau: time step (Sec. 3.1); target_walkers: N_t;
 * zeta, xi: shift damping and forcing (Eq. shift-update; defaults 0.08 and
 * zeta^2/4 reproduce the paper's printed series); threshold: theta of the
 * vector compression (default 1); t_rel: semistochastic threshold, a column
 * is spawned exactly when |c| >= t_rel m (Sec. 7.1); seed: 64-bit seed of
 * the counter-based generator; addr_words: W; flags: FQ_FLAG_* bits;
 * initiator_threshold: see FQ_FLAG_INITIATOR. */
typedef struct {
    double dtau, target_walkers, zeta, xi, threshold, t_rel;
    uint64_t seed;
    int32_t addr_words, flags;
    double initiator_threshold; /* n_a of FQ_FLAG_INITIATOR (ignored without it) */
} fq_params;

/* One row of the per-step time series (Sec. 4, the DataFrame columns):
 * `step` n, `len` = number of stored addresses of c^(n), `exact_steps` and
 * `inexact_steps` = parents of c^(n-1) spawned exactly / stochastically,
 * `spawns` = spawn events of step n, `shift` = S^(n), `norm` = ||c^(n)||_1,
 * `hproj` = y^T H c^(n), `vproj` = y^T c^(n), `flags` = FQ_ROW_* bits.
 *
 * FQ_ROW_INEXACT: some sum of this step (annihilation, ||c||_1, y^T H c,
 * y^T c, or the norm of a state set just before) was not the exactly
 * rounded sum of its terms.  Sums are exact integer sums of the terms on a
 * grid of 2^-80; a term that is not a multiple of 2^-80 (possible only for
 * |term| < 2^-27) is first rounded to the nearest grid point, an error of at
 * most 2^-81 per term.  With the flag clear, every sum of the row is exactly
 * rounded.  fq_run then returns FQ_OK and fq_last_error() names the first
 * flagged step. */
#define FQ_ROW_INEXACT 1
typedef struct {
    int64_t step, len, exact_steps, inexact_steps, spawns;
    double shift, norm, hproj, vproj;
    int64_t flags;
} fq_step_stats;

/* Sizes of the device data structures.  table_capacity: largest number of
 * stored addresses; spawn_capacity: largest number of spawn events per step;
 * buckets: hash buckets (power of two <= 32768, 0 = choose); lds_slots: LDS hash slots
 * per bucket (power of two, 1024..8192, <= 8 * block, 0 = 4096); block:
 * threads per workgroup of the merge kernel (256, 512 or 1024; 0 = choose);
 * spawn_block: threads per workgroup of the spawn kernel (256, 512 or 1024;
 * 0 = 256). */
typedef struct {
    int64_t table_capacity, spawn_capacity;
    int32_t buckets, lds_slots, block, spawn_block;
} fq_layout;

typedef struct fq_handle fq_handle;

/* Bytes of device workspace needed for (h, p, layout); fills the defaults
 * chosen for zero fields of *layout when `layout_out` is not NULL. */
int fq_workspace_size(const fq_hamiltonian *h, const fq_params *p, const fq_layout *layout,
                      size_t *bytes, fq_layout *layout_out);

/* Creates a handle on `workspace` (device pointer, >= fq_workspace_size
 * bytes, owned by the caller and kept alive until fq_destroy).  The device
 * is the current HIP device. */
int fq_create(const fq_hamiltonian *h, const fq_params *p, const fq_layout *layout,
              void *workspace, size_t bytes, fq_handle **out);

/* Sets the state c^(step) = {(addrs[i], vals[i])} (host arrays, n entries,
 * n * W words, distinct addresses with N bosons in M modes), the shift
 * S^(step), and the reference vector y = ref_val e_ref for the projected
 * energy (Sec. 4.2; the paper's default is y = c^(0) = 10 e_start). */
int fq_set_state(fq_handle *q, const uint64_t *addrs, const double *vals, int64_t n, double shift,
                 int64_t step, const uint64_t *ref_addr, double ref_val, void *stream);

/* Advances n_steps steps; stats_out (host, n_steps rows, may be NULL)
 * receives one row per step.  On error the handle stays at the last
 * completed step and the rows of completed steps are filled. */
int fq_run(fq_handle *q, int64_t n_steps, fq_step_stats *stats_out, void *stream);

/* Copies the current state to host arrays (capacity `cap` entries): addrs
 * (n * W words), vals, and the current shift and step.  Order unspecified. */
int fq_get_state(fq_handle *q, uint64_t *addrs, double *vals, int64_t cap, int64_t *n,
                 double *shift, int64_t *step, void *stream);

/* Parity support: events of the spawn pass that produced the current slab
 * (FQ_FLAG_DUMP_SPAWNS) as parent address (W words), attempt, destination
 * (W words), value; and the merged pre-compression amplitudes of the last
 * step (FQ_FLAG_DUMP_MERGED) as address (W words), value.  Host arrays. */
int fq_read_spawn_dump(fq_handle *q, uint64_t *parent, int64_t *attempt, uint64_t *dest,
                       double *value, int64_t cap, int64_t *n, void *stream);
int fq_read_merged_dump(fq_handle *q, uint64_t *addr, double *value, int64_t cap, int64_t *n,
                        void *stream);

/* Kernel timing with HIP events recorded on the run stream around the
 * launches of each step while `enable` is non-zero (five events per step).
 * fq_kernel_time fills ms[0..n-1] with the summed milliseconds since the
 * last reset of: [0] the merge kernel (annihilation, compression, projected
 * energy, compaction), [1] the spawn kernel, [2] the second pass of the
 * spawn partition, [3] the reduction and shift update; entries beyond [3]
 * are zero.  *steps receives the number of timed steps. */
int fq_set_timing(fq_handle *q, int32_t enable);
int fq_kernel_time(fq_handle *q, double *ms, int32_t n, int64_t *steps, int32_t reset);

/* Diagnostics (flag FQ_FLAG_PHASE_TIMING): out[0..9] = summed wall-clock
 * milliseconds per phase of the step kernel (workgroup-summed), out[10] =
 * LDS hash probes, out[11] = inserts per thread summed, out[12] = largest
 * number of distinct addresses in one bucket.  n >= 13. */
int fq_debug_counters(fq_handle *q, double *out, int32_t n, int32_t reset, void *stream);

/* Current layout (with defaults resolved). */
int fq_get_layout(const fq_handle *q, fq_layout *layout);

int fq_destroy(fq_handle *q);
const char *fq_last_error(const fq_handle *q);

/* ------------------------------------------------------------------------
 * Copy and autotuning.
 *
 * fq_copy_state copies the current state of `src` (vector, shift, step,
 * reference vector) into `dst`, on the device, with no host round trip.  The
 * two handles must have the same Hamiltonian and parameters; their layouts
 * may differ.  Because the step is layout independent, `dst` then continues
 * exactly as `src` would.
 *
 * fq_autotune times candidate layouts (the hash and tile shapes: buckets,
 * LDS slots, merge and spawn workgroup sizes) on a copy of the state of
 * `src`: for each of the n candidates it creates a handle in `scratch`
 * (caller-owned device memory), copies the state, runs `trial_steps` steps
 * and records the mean milliseconds per step from HIP events in ms[i]
 * (negative when the candidate does not fit `scratch` or fails).  *best is
 * the index of the fastest candidate.  `src` is not modified.
 * ------------------------------------------------------------------------ */
int fq_copy_state(fq_handle *dst, fq_handle *src, void *stream);
int fq_autotune(fq_handle *src, const fq_layout *candidates, int32_t n, int32_t trial_steps, void *scratch,
                size_t scratch_bytes, double *ms, int32_t *best, void *stream);

/* ------------------------------------------------------------------------
 * Batch: n independent instances advanced together, one launch per kernel
 * per step for the whole batch (each workgroup finds its instance and bucket
 * from a map), with per-instance tables, shifts and statistics.  Instances
 * may differ in Hamiltonian (M, N, t, u, g), parameters and capacities;
 * they must share the model kind (the ring without importance sampling; the
 * square lattice or a ring with g != 0; momentum space with one-word
 * addresses of at most 31 bits, N + M - 1 <= 31, or other momentum space),
 * the compression style (FQ_FLAG_EARLY_COMPRESSION set or not),
 * addr_words, lds_slots, block and spawn_block.  Every instance
 * produces the same results as it would alone.
 *
 * fq_batch_workspace_size: bytes of the single workspace for the batch
 * (hams, params, layouts: arrays of n).  fq_batch_create carves it (caller
 * owned, 256-byte aligned).  fq_batch_instance returns instance i's handle,
 * owned by the batch, for fq_set_state, fq_get_state and the dumps (not for
 * fq_destroy).  fq_batch_run advances every instance by n_steps steps;
 * stats (host, may be NULL) receives n * n_steps rows, instance-major
 * (row k of instance i at i * n_steps + k).  When an instance fails, the
 * batch stops at the end of the chunk of steps in which it failed, every
 * instance stays at its last completed step (completed rows are filled), the
 * call returns that instance's status, and fq_batch_failed() names it.
 * ------------------------------------------------------------------------ */
typedef struct fq_batch fq_batch;
int fq_batch_workspace_size(int32_t n, const fq_hamiltonian *hams, const fq_params *params,
                            const fq_layout *layouts, size_t *bytes);
int fq_batch_create(int32_t n, const fq_hamiltonian *hams, const fq_params *params, const fq_layout *layouts,
                    void *workspace, size_t bytes, fq_batch **out);
int fq_batch_instance(fq_batch *b, int32_t i, fq_handle **out);
int fq_batch_run(fq_batch *b, int64_t n_steps, fq_step_stats *stats, void *stream);
int32_t fq_batch_failed(const fq_batch *b);
int fq_batch_destroy(fq_batch *b);
/* Description of the last failure of a batch call (b may be NULL for a
 * failed fq_batch_create); instance failures are also reported by
 * fq_last_error() of the instance that fq_batch_failed() names. */
const char *fq_batch_last_error(const fq_batch *b);
/* fq_batch_autotune times candidate shared layouts of a batch (the hash and
 * tile shapes every instance shares: lds_slots, block and spawn_block; the
 * bucket count of every instance is the candidate's `buckets`, or follows
 * from the instance's capacities and the candidate's lds_slots when 0):
 * for each of the n candidates it creates a batch of the same instances
 * with that layout in `scratch` (caller-owned device memory of at least
 * that batch's fq_batch_workspace_size), copies every instance's state into
 * it on the device, runs one step, then times trial_steps steps of the
 * whole batch with HIP events on `stream`.  ms[i] = milliseconds per step
 * of candidate i, negative when it does not fit `scratch` or fails; *best =
 * the index of the fastest.  The results of a batch do not depend on its
 * layout, so a batch re-created with the best layout (and the states copied
 * over) continues exactly.  `b` is not modified. */
int fq_batch_autotune(fq_batch *b, const fq_layout *candidates, int32_t n, int32_t trial_steps, void *scratch,
                      size_t scratch_bytes, double *ms, int32_t *best, void *stream);

/* ------------------------------------------------------------------------
 * Replicas (Sec. 4.3, Eq. RayleighQuotientReplica): a batch of R = 2 ..
 * FQ_MAX_REPLICAS statistically independent runs of one Hamiltonian
 * (identical fq_hamiltonian, addr_words, buckets and lds_slots; normally
 * only the seed differs), stepped together.  After every step the overlap
 * c_A . c_B of each pair A < B is computed on the device: the sum over the
 * addresses present in both tables of the product of the two amplitudes,
 * each product rounded to double, the products summed exactly (192-bit
 * fixed point with 96 fractional bits) and rounded once to the nearest
 * double.  The result equals the exactly rounded sum when every product is
 * a multiple of 2^-96 (always when |c_A c_B| >= 2^-43); otherwise that
 * product is rounded half-even to a multiple of 2^-96 and *inexact is set.
 * The variational energy of Sec. 4.3 is the ratio of the means of
 * (S_A + S_B)/2 c_A.c_B and c_A.c_B summed over pairs, with the shifts of
 * the statistics rows of the same steps.
 *
 * fq_batch_replica_scratch_size: bytes of device scratch (caller owned,
 * 256-byte aligned) for fq_batch_run_replicas.  FQ_EINVAL when the batch is
 * not a valid replica set.
 * fq_batch_run_replicas: as fq_batch_run (stats may be NULL), and
 * overlaps (host, required) receives n_steps rows of P = R(R-1)/2 doubles,
 * row k = the overlaps after step k, pairs in the order (0,1), (0,2), ..,
 * (0,R-1), (1,2), ...  All replicas must hold a state at the same step.  A
 * pair whose two replicas are not both error-free at the same step reads
 * NaN.  Errors: FQ_ECAPACITY when a bucket of a table does not fit the
 * lds_slots hash of the join, FQ_EDIVERGED when a product has magnitude
 * 2^95 or more; a failing instance is reported as by fq_batch_run.  The
 * rows of the steps completed before a failure are filled.  inexact (may
 * be NULL) is set to 1 when some product was rounded (see above), else 0.
 * ------------------------------------------------------------------------ */
#define FQ_MAX_REPLICAS 8
int fq_batch_replica_scratch_size(fq_batch *b, size_t *bytes);
int fq_batch_run_replicas(fq_batch *b, int64_t n_steps, fq_step_stats *stats, double *overlaps, void *scratch,
                          size_t scratch_bytes, int32_t *inexact, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as fq_batch_run_replicas, with the join's scratch taken from a
 * static device array of FQ_STATIC_SCRATCH_BYTES inside the library
 * instead of a caller buffer.  It makes no device allocation.  The array
 * exists once per GPU and is held until the process ends; it is shared by
 * every call on that GPU and keeps the last call's contents (the call
 * clears what must start at zero), so calls that overlap in time on one GPU
 * (other host threads, other streams) race and must not be made.  The
 * current device must be the one that was current at fq_batch_create.
 * Errors as fq_batch_run_replicas, and FQ_EINVAL when the scratch the batch
 * needs (fq_batch_replica_scratch_size) exceeds FQ_STATIC_SCRATCH_BYTES:
 * 4 MiB hold two replicas at up to 16384 buckets, eight at up to 4096. */
#define FQ_STATIC_SCRATCH_BYTES ((size_t)4 << 20)
int fq_batch_run_replicas_static(fq_batch *b, int64_t n_steps, fq_step_stats *stats, double *overlaps,
                                 int32_t *inexact, void *stream);

/* ------------------------------------------------------------------------
 * Excited states (Sec. 2.2): a batch of R = 2 .. FQ_MAX_REPLICAS step-
 * synchronised runs of one Hamiltonian (the same conditions as replicas),
 * where after every merge run k is orthogonalised against runs 0 .. k-1 in
 * turn (Gram-Schmidt): c_k <- c_k - alpha c_j with alpha = (c_j . c_k) /
 * (c_j . c_j), both dot products summed exactly from rounded products (as
 * the replica overlaps) and rounded once, alpha one IEEE division (0 for an
 * empty c_j), each entry v_k - (alpha v_j) with the product rounded first
 * over the union of the two supports, exact zeros dropped.  The projection
 * happens before the spawn kernel reads the merged table, so every step
 * starts from orthogonal vectors; the shift of run k then estimates the k-th
 * energy level.  The statistics rows describe the merged vectors before the
 * projection (as the shift update sees them); the next shift update starts
 * from the exact 1-norm of the projected vector.
 *
 * fq_batch_spectral_scratch_size: bytes of device scratch (caller owned,
 * 256-byte aligned).  FQ_EINVAL when the batch is not a valid set of runs
 * or 2 * lds_slots does not fit the LDS of the projection.
 * fq_batch_run_spectral: as fq_batch_run (stats may be NULL).  A bucket
 * whose union does not fit the LDS hash or the table fails its run with
 * FQ_ECAPACITY.  inexact (may be NULL) is set to 1 when a rounded product,
 * square or projected value was not a multiple of 2^-96, so its exact sum
 * was rounded first.
 * ------------------------------------------------------------------------ */
int fq_batch_spectral_scratch_size(fq_batch *b, size_t *bytes);
int fq_batch_run_spectral(fq_batch *b, int64_t n_steps, fq_step_stats *stats, void *scratch, size_t scratch_bytes,
                          int32_t *inexact, void *stream);

/* ------------------------------------------------------------------------
 * Server: continuous batching of FCIQMC solves on one GPU.
 *
 * A request (Hamiltonian, parameters, capacities, start address with its
 * walker number, step count) is queued by fq_server_submit.  Each call of
 * fq_server_tick first admits queued requests in arrival order while the
 * walker-table pool (the caller-owned device memory given at creation, the
 * HBM budget) has room for the request's workspace and fewer than
 * max_active solves are resident; then it advances every resident solve by
 * steps_per_tick steps in one batch (a solve stops exactly at its step
 * count); then it retires finished solves and frees their memory.  State
 * stays resident on the device between ticks.  A solve's results do not
 * depend on what else is in the batch.
 *
 * Solves start from `start_val` walkers on `start` with shift 0 and use
 * y = start_val e_start for the projected energy (Sec. 2.1, Sec. 4.2).
 * fq_server_poll reports a request's state, its last statistics row and the
 * means of shift, y.Hc and y.c over the steps after the first half.  All
 * requests of one server share the model, addr_words, lds_slots, block and
 * spawn_block of its configuration (momentum space: addr_words 1 and
 * N + M - 1 <= 31) and use late
 * compression (a request with FQ_FLAG_EARLY_COMPRESSION is refused with
 * FQ_EINVAL); a ring server takes g = 0 only.  Not thread safe.
 * ------------------------------------------------------------------------ */
typedef struct fq_server fq_server;
typedef struct {
    int32_t model, addr_words;               /* every request uses these        */
    int32_t lds_slots, block, spawn_block;   /* layout shared by the batch      */
    int32_t max_active;                      /* resident solves at most         */
    int64_t steps_per_tick;                  /* 1 .. 4096                       */
} fq_server_config;

#define FQ_REQ_QUEUED 0
#define FQ_REQ_RUNNING 1
#define FQ_REQ_DONE 2
#define FQ_REQ_FAILED 3

typedef struct {
    int32_t state, status;      /* FQ_REQ_*; fq_status of a failed request  */
    int64_t steps_done;
    fq_step_stats last;         /* last completed row                       */
    double mean_shift, mean_hproj, mean_vproj;  /* over steps > n_steps / 2 */
    int64_t n_mean;
    int64_t workspace_bytes;
    double walker_steps;        /* sum of ||c||_1 over the completed steps  */
} fq_request_info;

int fq_server_create(const fq_server_config *cfg, void *pool, size_t pool_bytes, fq_server **out);
int fq_server_submit(fq_server *sv, const fq_hamiltonian *h, const fq_params *p, const fq_layout *layout,
                     const uint64_t *start, double start_val, int64_t n_steps, uint64_t *request_id);
int fq_server_tick(fq_server *sv, void *stream, int32_t *active, int32_t *queued, int32_t *finished);
int fq_server_poll(fq_server *sv, uint64_t request_id, fq_request_info *info);
int fq_server_destroy(fq_server *sv);
const char *fq_server_last_error(const fq_server *sv);

/* Host helper: occupations -> W address words (the encoding of Sec. 6.1). */
int fq_encode(const int32_t *occ, int32_t M, int32_t W, uint64_t *out);

/* Library version string. */
const char *fq_version(void);

#ifdef __cplusplus
}
#endif
#endif
