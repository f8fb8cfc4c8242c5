/*
 * qram.h -- C ABI of the MI355X trajectory simulator for amplitude-damped
 * bucket-brigade QRAM queries (qubit and qutrit encodings).
 *
 * A query of an (n,k)-QRAM maps sum_i c_i |i>|0>_bus to sum_i c_i |i>|d_i>
 * (Eq. nk-qram).  Each time slice of the T = 6n+2k slice schedule applies its
 * gates and then one joint amplitude-damping layer over the M = 2(2^n - 1)
 * tree sites (Sec. II B, Eq. kraus / kraus-tri, Eq. layerkraus).  One
 * trajectory samples the candidate history in advance, resolves every layer
 * with one auxiliary draw (Theorem 4), measures the tree at the end and
 * returns the fidelity of the normalised post-measurement state with the ideal
 * output, whose tree is in the ground state (App. C).  The "pruned" mode
 * evolves only the bad branches plus one reference branch and predicts the
 * others in closed form (Alg. 1, Proposition 1, Theorems 2-3); the "full"
 * mode evolves every branch.  Both give the same fidelity up to rounding.
 *
 * Input class: the data-loading input with uniform address amplitudes
 * c_i = 2^{-n/2} and bus word 0 (Sec. VI, App. D).
 *
 * Random numbers (fixed contract, identical for every mode and launch shape):
 * Philox4x32-10 keyed by the 64-bit seed.  Candidate history: the tree site q
 * of slice s is linear index L = (s-1) M + q, candidates are i.i.d.
 * Bernoulli(gamma) drawn by a geometric walk in 64-site blocks with counters
 * (block, draw, trajectory, 1); the auxiliary uniform of slice s uses
 * (s, 0, trajectory, 2); the final tree measurement (0, 0, trajectory, 3).
 * Trajectory indices are global within a seed: a run over [traj0, traj0+a+b)
 * equals the runs over [traj0, traj0+a) and [traj0+a, traj0+a+b) entry by
 * entry.  traj0 + ntraj must not exceed 2^32.
 *
 * Ownership: the caller owns every buffer it passes; the library never frees
 * caller memory.  A context owns the device memory it allocates (tables and
 * work buffers) until qram_destroy.  A context is not thread-safe; use one
 * context per host thread or lock around calls.
 *
 * Errors: every call returns a qram_status.  Nothing throws across the ABI.
 * After an error the context stays usable and qram_last_error describes it.
 */
#ifndef QRAM_H
#define QRAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qram_ctx qram_ctx;

typedef enum { QRAM_QUTRIT = 0, QRAM_QUBIT = 1 } qram_encoding;

typedef enum {
  QRAM_OK = 0,
  QRAM_E_INVAL = -1,    /* null pointer, gamma outside [0,1), bad enum/mode */
  QRAM_E_NOMEM = -2,    /* device or host allocation failed */
  QRAM_E_DEVICE = -3,   /* a HIP call failed */
  QRAM_E_RANGE = -4,    /* n or k outside the supported range */
  QRAM_E_CAPACITY = -5  /* an output or work buffer is too small */
} qram_status;

/* FULL: every branch explicit in the trajectory kernel, which carries a
 * component untouched by any jump implicitly (its sites follow from the
 * schedule) and decides the slices before a trajectory's first jump and the
 * final sums of a jump-free trajectory in closed form.  PRUNED: Alg. 1, the
 * bad branches plus the reference explicit, the good branches predicted.
 * PLAIN: the plain full evolution of App. D / Table 2 ("full: D explicit
 * branches"): every component of every branch carries its own site list and
 * complex amplitude through every slice, nothing predicted or implicit. */
typedef enum { QRAM_MODE_FULL = 0, QRAM_MODE_PRUNED = 1, QRAM_MODE_PLAIN = 2 } qram_mode;

/* Per-trajectory statistics (32 bytes, naturally aligned). */
typedef struct {
  uint32_t n_cand;           /* candidates drawn over slices 1..T-1 */
  uint32_t n_bad;            /* bad addresses under the marking rule */
  uint32_t ref_addr;         /* reference address (smallest good), UINT32_MAX if none */
  uint32_t n_explicit;       /* components evolved explicitly */
  uint16_t n_jumps;          /* damping layers whose joint outcome J was nonempty */
  uint16_t first_jump_slice; /* slice of the first nonempty J, 0 if none */
  uint8_t ref_survived;      /* 1 if the reference branch was never annihilated */
  uint8_t q_ground;          /* 1 if the tree measurement gave the ground state */
  uint8_t flags;             /* bit 0: candidate buffer overflow, bit 1: list overflow */
  uint8_t pad;
  double fid_pre;            /* |<psi_id|psi>|^2 / <psi|psi> before the tree measurement */
} qram_traj_stats;

/*
 * Create a context for an (n,k)-QRAM in the given encoding with damping
 * strength gamma (Sec. II B; Theorem 4 needs gamma < 1).
 *   n_addr      1..15 (qubit), 1..14 (qutrit); k_data 1..8 with k <= n; the
 *               qubit encoding also needs n + k <= 16 (at most 65536
 *               components per trajectory).  Qubit k_data 7 and 8 run on the
 *               plain engine (see qram_create_ex).
 *   memory_bits host array of 2^n words; bit b of word i is d_i^(b); only the
 *               low k bits are used.  Copied: the caller may free it after the
 *               call returns.
 *   out         receives the context.
 * The current HIP device at the time of the call is used for every later call.
 * Returns QRAM_E_RANGE when gamma is so large that the damping weights of the
 * deepest orbit underflow double precision.
 */
qram_status qram_create(int n_addr, int k_data, qram_encoding enc, double gamma,
                        const uint32_t *memory_bits, qram_ctx **out);

/*
 * Context with depolarizing noise and a general input (Sec. II B, Sec. IV D,
 * App. C).  gamma, enc, n_addr, k_data and memory_bits as in qram_create.
 *   eps          depolarizing strength in [0, 1).  In slice s every site of
 *                the layers above the leaf layer whose router holds its
 *                address bit both before and after the gates of s (stored at
 *                slice 3t+2, unstored at T-3t-2) suffers a fault with
 *                probability eps: X, Z or ZX (= iY) with equal probability
 *                on a qubit site (and the qutrit data slot), one of the eight
 *                nontrivial Weyl operators on a qutrit router.  Faults act
 *                after the slice's gates and before its damping layer, are
 *                drawn in advance (Philox counters (block, draw, trajectory,
 *                4), a geometric walk over the active positions, the type
 *                from the draw's third word) and mark their bad range by the
 *                encoding's rule, whatever their type (Alg. 1).
 *   input_amp    [2 * 2^n] amplitude (re, im) of each address, normalised by
 *                the library; NULL = uniform.  Addresses with amplitude 0 are
 *                absent (no branch).
 *   input_bus    [2^n] bus word of each address (one column per address);
 *                NULL = 0.  The ideal output is sum_i c_i |i>|j_i xor d_i>.
 *   input_ab     [2 * 2^n * 2^k] amplitude (re, im) of every (address i,
 *                bus word j) pair, address-major (index i * 2^k + j),
 *                normalised by the library; NULL = none.  Excludes
 *                input_amp and input_bus.  The ideal output is
 *                sum_ij c_ij |i>|j xor d_i> (the random branch sets of
 *                Sec. VI draw such pairs).  The qutrit encoding then carries
 *                one component per pair.  The reference (Alg. 1) is the
 *                smallest good address holding exactly one bus word; good
 *                addresses holding several are predicted bus word by bus
 *                word from it (Theorem 3: O(k 2^k) each, Table 2).
 *   truncate     nonzero: Hamming truncation at w_max (Sec. V): the output
 *                words of every good address but the reference that lie
 *                more than w_max bit flips from its ideal word are dropped
 *                before the tree measurement (qubit encoding; no effect on
 *                the qutrit, whose good branches end in the ideal word).
 *                Every mode computes the same truncated quantity.  Needs
 *                one bus word per address (else QRAM_E_INVAL) and
 *                0 <= w_max <= k.
 * The qubit encoding accepts k_data up to 8 here (n + k <= 16).  Contexts
 * with eps > 0, a general input, truncation, or qubit k > 6 run every mode
 * on the plain engine: QRAM_MODE_FULL as QRAM_MODE_PLAIN, QRAM_MODE_PRUNED as Alg. 1 on
 * explicit site lists (bad branches plus the reference explicit, the good
 * branches carried by the reference's weights and final state).  One
 * exception: with eps > 0 on the data-loading input (qubit k <= 6), a
 * pruned run hands every trajectory that drew no depolarizing fault to the
 * trajectory kernel of the damping-only contexts (such a trajectory is a
 * damping-only one: same candidates, bad set, draws and result), and only
 * the others to the plain engine.  qram_export_state and qram_run_forced
 * keep such contexts on the plain engine.
 */
typedef struct {
  int n_addr, k_data;
  qram_encoding enc;
  double gamma;
  double eps;
  const uint32_t *memory_bits;  /* host, 2^n words; copied */
  const double *input_amp;      /* host, 2 * 2^n doubles, or NULL; copied */
  const uint32_t *input_bus;    /* host, 2^n words, or NULL; copied */
  const double *input_ab;       /* host, 2 * 2^n * 2^k doubles, or NULL; copied */
  int truncate, w_max;          /* Hamming truncation (truncate = 0: none) */
} qram_params;

qram_status qram_create_ex(const qram_params *params, qram_ctx **out);

/* Release a context and all device memory it owns.  NULL is allowed. */
void qram_destroy(qram_ctx *ctx);

/* Message for the last failing call on ctx (or for qram_create when ctx is
 * NULL); valid until the next call on the same context. */
const char *qram_last_error(const qram_ctx *ctx);

/*
 * Candidate histories and branch classification (Alg. 1 steps 1-2) of
 * trajectories traj0 .. traj0+ntraj-1, synchronously, into host buffers.
 *   n_cand      [ntraj] number of candidates of each trajectory.
 *   cand_digest [ntraj] FNV-1a 64 of the ascending candidate indices L, each
 *               folded as 4 little-endian bytes (offset basis
 *               0xcbf29ce484222325, prime 0x100000001b3).  May be NULL.
 *   n_bad       [ntraj] number of bad addresses.  May be NULL.
 *   bad_bits    [ntraj * ceil(2^n / 64)] bitmap of bad addresses (bit i%64 of
 *               word i/64).  May be NULL.
 *   cand_L      optional dump of all candidate lists, concatenated in
 *               trajectory order; cand_cap entries available.  If the total
 *               exceeds cand_cap the dump is skipped and QRAM_E_CAPACITY is
 *               returned after every other output has been written.
 */
qram_status qram_sample_faults(qram_ctx *ctx, uint64_t seed, uint64_t traj0,
                               uint32_t ntraj, uint32_t *n_cand,
                               uint64_t *cand_digest, uint32_t *n_bad,
                               uint64_t *bad_bits, uint32_t *cand_L,
                               uint64_t cand_cap);

/*
 * Depolarizing faults of trajectories traj0 .. traj0+ntraj-1 (contexts with
 * eps > 0; otherwise every count is 0): n_dep [ntraj] counts; dep (optional)
 * all lists concatenated in trajectory order, each entry site | slice << 16
 * | type << 24 with type a | b << 2 for the operator Z^b X^a, ascending
 * (slice, site); cap entries available, else the dump is skipped and
 * QRAM_E_CAPACITY returned after the counts are written.
 */
qram_status qram_sample_depol(qram_ctx *ctx, uint64_t seed, uint64_t traj0, uint32_t ntraj,
                              uint32_t *n_dep, uint32_t *dep, uint64_t cap);

/*
 * Full evolution of every branch (the comparator mode), synchronously.
 *   fid [ntraj] post-measurement fidelity of each trajectory.
 *   st  [ntraj] statistics, or NULL.
 */
qram_status qram_run_full(qram_ctx *ctx, uint64_t seed, uint64_t traj0,
                          uint32_t ntraj, double *fid, qram_traj_stats *st);

/*
 * Pruned evolution (Alg. 1): bad branches plus one reference branch evolve
 * explicitly; good branches are predicted (Proposition 1 for the qutrit
 * encoding, Theorem 3 and the XOR mirror for the qubit encoding) and enter
 * every joint damping draw through their closed-form weights (Eq. maskweight).
 * Same arguments as qram_run_full; same results up to rounding.
 */
qram_status qram_run_pruned(qram_ctx *ctx, uint64_t seed, uint64_t traj0,
                            uint32_t ntraj, double *fid, qram_traj_stats *st);

/*
 * Plain full evolution (QRAM_MODE_PLAIN), the comparator of App. D: all D
 * branches evolved explicitly, every component slice by slice with its own
 * site list and complex FP64 amplitude (the damping factors and phases of
 * the slices without a jump counted beside it and multiplied in where an
 * amplitude is needed); one workgroup per trajectory.  Same arguments as
 * qram_run_full; same results up to rounding.
 */
qram_status qram_run_plain(qram_ctx *ctx, uint64_t seed, uint64_t traj0,
                           uint32_t ntraj, double *fid, qram_traj_stats *st);

/*
 * Device-buffer variants: d_fid [ntraj] and d_st [ntraj] (or NULL) are device
 * pointers; the work is enqueued on stream (a hipStream_t, NULL = the null
 * stream) and the call returns without waiting.  The outputs are valid once
 * the stream has reached this point.  Work buffers stay owned by the context;
 * a later call on the same context may reuse them only after this one is
 * ordered before it on the stream (same stream, or caller-side sync).
 */
qram_status qram_run_full_async(qram_ctx *ctx, uint64_t seed, uint64_t traj0,
                                uint32_t ntraj, double *d_fid,
                                qram_traj_stats *d_st, void *stream);
qram_status qram_run_pruned_async(qram_ctx *ctx, uint64_t seed, uint64_t traj0,
                                  uint32_t ntraj, double *d_fid,
                                  qram_traj_stats *d_st, void *stream);
qram_status qram_run_plain_async(qram_ctx *ctx, uint64_t seed, uint64_t traj0,
                                 uint32_t ntraj, double *d_fid,
                                 qram_traj_stats *d_st, void *stream);

/* Mean and standard error of the mean of fid[0..ntraj-1] (host arrays). */
qram_status qram_fidelity(const double *fid, uint32_t ntraj, double *mean,
                          double *sem);

/*
 * Launch shape of a mode.  Trajectories are grouped by their number of
 * explicitly evolved components; each group runs as its own launch whose
 * workgroups hold about slots_per_thread components per thread (4, 8, 16, 32
 * or 64; 0 restores the automatic choice).  schedule bit 0: 0 hands
 * trajectories to workgroups round robin, 1 takes them from a device queue,
 * longest first; bit 1: keep the component state words in device memory
 * instead of workgroup shared memory (smaller workgroups per compute unit
 * footprint, more trajectories in flight).  Modes that run on the plain
 * engine (QRAM_MODE_PLAIN, and every mode of a context with depolarizing
 * noise, a general input, truncation or qubit k > 6): slots_per_thread is the
 * number of workgroups per compute unit (1..32, capped by what fits; 0 =
 * automatic: all that fit; the kernel has builds for three register budgets,
 * and a launch takes the largest budget that still fits the number asked
 * for) and schedule the threads per workgroup (64, 128,
 * 256, 512 or 1024; 0 = automatic: 256, or 64 (pruned) / 128 (full) when a
 * trajectory holds at most 256 components and the run is not split, or 1024
 * for the plain share of a split run whose batch expects at most ten
 * faulted trajectories per compute unit, a trajectory holding at least 2048
 * components; qram_get_launch reports the last run's choice), plus 1 to work on
 * each component record in device memory instead of staging it in shared
 * memory while a thread applies a slice's gates to it.  The launch stays
 * within 16 GiB of per-trajectory state, and the plain share of a split
 * pruned run takes at most 1.5 times its expected number of trajectories in
 * workgroups.  qram_get_launch returns the shape in use.  The shape changes
 * only the speed:
 * results are identical across shapes up to the rounding of the per-slice
 * weight sums.
 */
qram_status qram_set_launch(qram_ctx *ctx, qram_mode mode, int slots_per_thread,
                            int schedule);
qram_status qram_get_launch(const qram_ctx *ctx, qram_mode mode,
                            int *slots_per_thread, int *schedule);

/*
 * Options (value 0/1; all default to 0).
 *   QRAM_OPT_TIER2_GLOBAL: keep every explicit site list of a component whose
 *     routing a jump changed in global memory instead of registers, one list
 *     per component (the qubit encoding otherwise shares one list among the
 *     bus words of an address); on the plain engine, work on each component
 *     record in device memory instead of staging it in shared memory.  Same
 *     results; for testing the list paths against each other.
 *   QRAM_OPT_GRAPH: run each batch (sampling, classification, bucketing and
 *     every bucket's persistent evolution launch) as one HIP graph.  The
 *     graph is captured on the context's stream, instantiated once and then
 *     updated in place for the next batch, and launched on the caller's
 *     stream.  Results are identical to the eager path.  Stage timing then
 *     reports the whole batch as the evolution stage.
 *   QRAM_OPT_SUBTREE_MARKING: qubit encoding only (a no-op for the qutrit
 *     encoding).  Mark each damping candidate's own subtree (Eq. subtree)
 *     instead of the family-divergence range of Eq. badrange.  Sec. III B
 *     and Sec. VI B: a damping jump needs an excitation and an idle qubit has
 *     none, so damping creates no strays and its damage stays inside the
 *     candidate's subtree; the uniform rule of Alg. 1 marks a superset.
 *     Every path here simulates damping only, so the tighter set is exact:
 *     fidelities equal the full evolution's, and fewer addresses are evolved
 *     explicitly.  Changes n_bad, ref_addr, n_explicit and the bad bitmap of
 *     the qubit encoding (sampling, candidate lists and jump statistics are
 *     unchanged).
 */
enum { QRAM_OPT_TIER2_GLOBAL = 1, QRAM_OPT_GRAPH = 2, QRAM_OPT_SUBTREE_MARKING = 3 };
qram_status qram_set_option(qram_ctx *ctx, int option, int value);

/*
 * Measure every launch shape of a mode on trajectories [traj0, traj0+ntraj)
 * of seed and keep the fastest (the autotuner).  Each shape times the whole
 * evolution of the sample (every work bucket's launch).  A shape with the
 * component state in device memory must be 3% faster than the best with
 * the state in shared memory to be kept: within that margin it only adds
 * HBM traffic.  On the plain engine it tries 64, 128 and 256 threads per
 * workgroup, each with all, half and a quarter of the workgroups that fit a
 * compute unit, with the records staged in shared memory and in device
 * memory, on the first 16384 trajectories of the sample, best of two (a
 * split pruned run is timed whole: ordering, the trajectory kernel's buckets
 * and the plain share).  best_ms receives the kept shape's time.
 */
qram_status qram_autotune(qram_ctx *ctx, qram_mode mode, uint64_t seed,
                          uint64_t traj0, uint32_t ntraj, double *best_ms);

/*
 * Device time of the last synchronous run's kernels (milliseconds): sampling,
 * classification and evolution, measured with HIP events on the context's
 * stream.  times[3].
 */
qram_status qram_last_kernel_ms(const qram_ctx *ctx, double *times);

/*
 * Stage timing of the device-buffer variants.  With timing on, every batch a
 * *_async call enqueues records HIP events on the caller's stream around
 * sampling, classification (with ordering) and evolution.  qram_stage_times
 * waits for the recorded events, returns the summed milliseconds of the three
 * stages since timing was switched on or last read (ms[3]) and the number of
 * batches (nbatches, may be NULL), and starts a new accumulation.
 */
qram_status qram_set_timing(qram_ctx *ctx, int on);
qram_status qram_stage_times(qram_ctx *ctx, double *ms, uint32_t *nbatches);
/* Evolution kernel launches (one per work bucket and batch) inside the
 * batches the current accumulation timed; read it before qram_stage_times,
 * which starts a new accumulation. */
qram_status qram_stage_launches(const qram_ctx *ctx, uint32_t *evolve_launches);
/* Per-bucket evolution timing of the same accumulation (read it before
 * qram_stage_times): arrays of 6 entries, one per work bucket (trajectories
 * grouped by explicit-component count, largest last).  ms[i]: summed
 * milliseconds of bucket i's evolution launches (HIP events around each
 * launch on the caller's stream); launches[i]: their number; ntraj_last[i]:
 * trajectories bucket i held in the last timed batch; emax[i]: the bucket's
 * bound on explicit components; *nbuckets: buckets in use.  The plain mode
 * has no buckets (*nbuckets = 0). */
qram_status qram_stage_buckets(qram_ctx *ctx, double *ms, uint32_t *launches, uint32_t *ntraj_last,
                               uint32_t *emax, int *nbuckets);

/*
 * Test entry: one trajectory under a forced history instead of the random
 * draws.  cand_L [ncand] ascending linear indices; u_aux [T] auxiliary
 * uniforms indexed by slice (entry 0 unused); u_fin the final uniform.
 * Runs the given mode; returns the fidelity and statistics.  In a context
 * with eps > 0 the depolarizing faults are still drawn, for seed 0 and
 * trajectory 0.
 */
qram_status qram_run_forced(qram_ctx *ctx, qram_mode mode,
                            const uint32_t *cand_L, uint32_t ncand,
                            const double *u_aux, double u_fin, double *fid,
                            qram_traj_stats *st);

/*
 * Dense whole-register cross-check for tiny trees (App. C): the complete
 * loading circuit of the context (same schedule, memory, input, gamma and
 * eps) on an ordinary register whose basis labels hold every digit:
 * address bit t (t = 0 the root's bit) most significant, then bus bit b,
 * then tree site q (router 2v, data slot 2v+1); a qutrit router has three
 * levels (W, L, R = 0, 1, 2), every other digit two; the last digit varies
 * fastest.  No sampling, no branch bookkeeping.
 *
 * qram_dense_dim: the number N of basis labels.
 *
 * qram_dense_density: the density matrix of the query under explicit
 * channels, slice by slice: the gates, the depolarizing channel of strength
 * eps on the active positions, amplitude damping on every tree site
 * (Eq. kraus, Eq. kraus-tri), then two channels the outlook of Sec. VII
 * names (each with a diagonal no-jump operator, applied to every tree
 * site): dephasing of strength `dephase` ((1-p) rho + p Z rho Z+ on a qubit
 * site; (1-p) rho + (p/2) sum_{m=1,2} Z^m rho Z^m+ on a qutrit router) and
 * heating of strength `heat` (level 0 rises with probability p: to 1 on a
 * qubit site, to L or R with p/2 each on a qutrit router; no-jump operator
 * diag(sqrt(1-p), 1, 1)).  Hadamard walls on the bus for the qubit
 * encoding.  Outputs F_rho = <psi_id| rho |psi_id> against the ideal output
 * sum_ij c_ij |i>|j xor d_i>|ground>, and the trace.  N <= 4096 (n <= 2),
 * else QRAM_E_RANGE.  Device memory: two N x N complex buffers, allocated
 * and freed by the call.
 *
 * qram_dense_forced: the state vector before the second wall under a given
 * history: jumps [njumps] in the jump-log format of qram_export_state (site
 * | level << 16 | slice << 24, slices ascending; every other damping layer
 * applies K_empty) and depolarizing faults [nfaults] in the format of
 * qram_sample_depol (site | slice << 16 | type << 24, slices ascending),
 * each fault after its slice's gates and before its damping layer.  psi
 * [2 * cap] host doubles receive (re, im) of every basis label; cap >= N
 * (else QRAM_E_CAPACITY).  n <= 3 and N <= 2^25, else QRAM_E_RANGE.
 */
qram_status qram_dense_dim(const qram_ctx *ctx, uint64_t *N);
qram_status qram_dense_density(qram_ctx *ctx, double dephase, double heat, double *F_rho, double *trace);
qram_status qram_dense_forced(qram_ctx *ctx, const uint32_t *jumps, uint32_t njumps, const uint32_t *faults,
                              uint32_t nfaults, double *psi, uint64_t cap);

/*
 * Test entry: the final pre-measurement state of one trajectory, component by
 * component, and its jump log.  The paper validates its pruned evolution by
 * matching complete complex amplitudes, the residual tree configuration and
 * the input-branch label of every component, and the jump decisions, between
 * pruned and full runs driven from the same history (Sec. VI A, App. D).
 *   history   sampled from (seed, traj) when u_aux is NULL; otherwise forced
 *             as in qram_run_forced (cand_L [ncand] ascending, u_aux [T],
 *             u_fin), and seed/traj only draw the depolarizing faults of a
 *             context with eps > 0.
 *   comp      [comp_cap * (3 + lmax)] uint32 words, lmax = 2n + k (qubit) or
 *             4n + k (qutrit); comp_cap >= 2^n * 2^k (qubit) or 2^n
 *             (qutrit), else QRAM_E_CAPACITY.  Record x = address * 2^k + bus
 *             word (qubit) or address (qutrit) of the initial label:
 *               [0] final address | final bus word << 16 | sign << 24 |
 *                   1 << 25 (bit 25 clear: the component was annihilated);
 *               [1] exposure e;
 *               [2] number m of excited tree sites after the last slice;
 *               [3 .. 3+m) site | level << 16 (1: excited qubit, qutrit L or
 *                   data qubit; 2: qutrit R).
 *             The state before the second Hadamard wall and the tree
 *             measurement is sum_x A_x |label, bus, tree> with
 *             A_x = c_i 2^(-k/2) (-1)^sign gamma^(J/2) a^e (qubit; the qutrit
 *             has no 2^(-k/2)), c_i = 2^(-n/2), a = sqrt(1-gamma) and J the
 *             total number of jump-log entries.  Pruned runs export the
 *             explicit components and the predicted good branches (Theorem 3,
 *             Proposition 1); a predicted branch is present only while the
 *             reference survives.  The plain engine (QRAM_MODE_PLAIN, and
 *             every mode of a context made by qram_create_ex with eps > 0,
 *             a general input or qubit k > 6) carries amplitudes as
 *             numbers: its records hold sign 0 and exposure 0; its pruned
 *             mode exports the explicit components only, and
 *   amp       [comp_cap * 2] (plain engine, required there; else may be
 *             NULL and is not written) receives each record's complex
 *             amplitude (real, imaginary), the factor gamma^(J/2) and the
 *             input amplitude c_i included.
 *             A component holding more than lmax excited sites (depolarizing
 *             strays on the plain engine) makes the call return
 *             QRAM_E_CAPACITY after writing the first lmax.
 *   jlog      [jcap] jump-log entries in order of slice: site | level << 16 |
 *             slice << 24 (levels as above); *njl receives the number of
 *             entries, which may exceed jcap (the rest are not written).
 *   fid, st   as in qram_run_forced.
 */
qram_status qram_export_state(qram_ctx *ctx, qram_mode mode, uint64_t seed, uint32_t traj,
                              const uint32_t *cand_L, uint32_t ncand, const double *u_aux,
                              double u_fin, uint32_t *comp, uint32_t comp_cap, double *amp,
                              uint32_t *jlog, uint32_t jcap, uint32_t *njl, double *fid,
                              qram_traj_stats *st);

/*
 * Test entry: qram_run_full / qram_run_pruned (mode) with the jump log of
 * every trajectory (the jump decisions of Sec. VI A): jlog [ntraj * jcap]
 * entries as in qram_export_state, trajectory t's at jlog + t * jcap;
 * njl [ntraj] the number of entries of each (may exceed jcap).
 */
qram_status qram_run_jumplog(qram_ctx *ctx, qram_mode mode, uint64_t seed, uint64_t traj0,
                             uint32_t ntraj, double *fid, qram_traj_stats *st, uint32_t *jlog,
                             uint32_t jcap, uint32_t *njl);

/*
 * Device memory.  qram_footprint: bytes of device memory the context holds
 * for runs of `mode` with up to ntraj trajectories per call (its tables plus
 * the work buffers of one batch; the caller's output arrays not included).
 * Allocates nothing.  qram_reserve: allocate those buffers now, so that such
 * runs allocate nothing later.  qram_errors: after the caller has waited for
 * its stream, report (QRAM_E_CAPACITY) and clear a capacity overflow that a
 * *_async run flagged on the device.
 */
qram_status qram_footprint(qram_ctx *ctx, qram_mode mode, uint32_t ntraj,
                           uint64_t *bytes);
qram_status qram_reserve(qram_ctx *ctx, qram_mode mode, uint32_t ntraj);
qram_status qram_errors(qram_ctx *ctx);

/*
 * qram_run_pruned_async with no device allocation, for callers that cannot
 * allocate: work enqueued under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, outputs and results as
 * qram_run_pruned_async (d_fid [ntraj] and d_st [ntraj] or NULL are the
 * caller's device buffers; the work is enqueued on `stream` and the call
 * returns without waiting).  The work buffers (candidate lists, bad
 * bitmaps, explicit lists, queues, tier-2 pools) live in one static device
 * array of 64 MiB per device, held until the process ends; the call itself
 * allocates nothing (no hipMalloc, no events, no graphs), and the context
 * must already exist.  Trajectories run in batches that fit the array, and
 * the evolution launches use at most as many workgroups as the array's
 * per-workgroup pools allow, so large configurations run with fewer
 * workgroups in flight than qram_run_pruned_async.  Returns
 * QRAM_E_CAPACITY when a single workgroup's buffers do not fit the array
 * (no supported configuration reaches this), QRAM_E_DEVICE when the array
 * has no address on the context's device, QRAM_E_INVAL for a context that
 * runs on the plain engine (qram_create_ex with eps > 0, a general or pair
 * input, truncation, or qubit k > 6).  Every call on one device
 * shares that device's array and its contents persist between calls:
 * calls that overlap on one device (other streams, other host threads,
 * other contexts) race and must be ordered by the caller.  The array's
 * error word is cleared at the start of each call; qram_errors reports a
 * capacity overflow of the last call once its stream has been waited for.
 */
qram_status qram_run_pruned_async_noalloc(qram_ctx *ctx, uint64_t seed, uint64_t traj0,
                                          uint32_t ntraj, double *d_fid,
                                          qram_traj_stats *d_st, void *stream);

/*
 * Request server: continuous batching of simulation requests on the current
 * device.  A host thread owns one context per admitted request.  Requests
 * are admitted in arrival order as soon as an execution slot is free
 * (max_active slots, one HIP stream each) and their footprint fits the
 * budget: qram_footprint for chunks of `chunk` trajectories plus 8 bytes per
 * shot for the device-resident results.  An admitted request runs `chunk`
 * trajectories per launch on its slot's stream, so chunks of different
 * requests overlap on the device.  A request's results are those of
 * qram_run_{full,pruned}(seed, traj0, shots) on its own context, whatever
 * else is in flight.  The server copies memory_bits at submission and owns
 * all memory it allocates; a request larger than the budget fails with
 * QRAM_E_CAPACITY.  The functions are thread-safe.
 */
typedef struct qram_server qram_server;

typedef struct {
  int n_addr, k_data;
  qram_encoding enc;
  double gamma;
  const uint32_t *memory_bits; /* host, 2^n words; copied */
  uint64_t seed, traj0;
  uint32_t shots;              /* trajectories */
  qram_mode mode;
} qram_request;

typedef struct {
  uint64_t ticket;
  int state;                /* 0 waiting, 1 running, 2 done, 3 failed */
  qram_status status;       /* failure reason when state is 3 */
  double mean, sem;         /* fidelity estimate when state is 2 */
  uint32_t shots;
  uint64_t footprint_bytes; /* admission footprint */
  double queue_ms;          /* submission to admission */
  double latency_ms;        /* submission to results on the host */
} qram_result;

qram_status qram_server_create(uint64_t hbm_budget_bytes, int max_active,
                               uint32_t chunk, qram_server **out);
qram_status qram_server_submit(qram_server *srv, const qram_request *req,
                               uint64_t *ticket);
/* Current state of a request (does not wait). */
qram_status qram_server_poll(qram_server *srv, uint64_t ticket,
                             qram_result *res);
/* Wait until the request is done or failed, or timeout_ms (<0: no limit). */
qram_status qram_server_wait(qram_server *srv, uint64_t ticket,
                             double timeout_ms, qram_result *res);
/* Per-trajectory fidelities of a finished request (fid[n], n >= shots). */
qram_status qram_server_fidelities(qram_server *srv, uint64_t ticket,
                                   double *fid, uint32_t n);
/* Forget a finished request. */
qram_status qram_server_release(qram_server *srv, uint64_t ticket);
/* Finish every submitted request, then stop the thread and free all. */
void qram_server_destroy(qram_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* QRAM_H */
