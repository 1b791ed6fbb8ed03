/*
 * sqa.h - C ABI of the MI355X (gfx950) simulated-quantum-annealing and
 * parallel-tempering library for embedded all-to-all Ising problems.
 *
 * Method: T. Albash, W. Vinci, D. A. Lidar, "Simulated Quantum Annealing
 * Comparison between All-to-All Connectivity Schemes", arXiv:1603.03755.
 *   - logical problem: Eq. (1), Sec. II
 *   - annealing Hamiltonian H(t) = A(t) H_X + B(t) H_P: Eq. (2), Sec. II
 *   - minor embedding with ferromagnetic chains: Sec. II A
 *   - LHZ parity embedding with 3- and 4-body constraints: Eq. (3), Sec. II B
 *   - majority-vote decoding: Eq. (4) (ME, Sec. II D), Eq. (5) (LHZ, Sec. II E,
 *     Appendix A, Eqs. (A1)-(A2))
 *   - minimum-weight decoding: Sec. IV A, Eqs. (6)-(10)
 *   - SQA and PT: Sec. III and Appendix B, Eqs. (B1)-(B2)
 *
 * Conventions shared by every call
 *   - Spins are int8_t with values +1 / -1.
 *   - J is int32_t n*n row-major; only the upper triangle (i < j) is read.
 *     J_ij < 0 is ferromagnetic.  h is int32_t[n] or NULL (all zero).
 *   - Penalties are signed Hamiltonian coefficients: the ME chain coupling
 *     J_F and the LHZ constraint coefficient C multiply s s' (ME) or the
 *     product of the constraint's spins (LHZ); the paper's penalty strength
 *     lambda corresponds to C = -lambda, so -2 is a penalty of strength 2.
 *   - Physical site numbering.  ME: chain i, slot r -> i*(n-1)+r; J_ij (i<j)
 *     couples slot j-1 of chain i with slot i of chain j; h_i sits on slot 0.
 *     LHZ: pair (i,j), i<j -> i*(2n-i-1)/2 + (j-i-1).
 *     ME on Chimera (Sec. II A, chains of ceil(n/4)+1 on the Chimera graph
 *     C_m, m = ceil(n/4)): chain i (block b = i/4, k = i%4), slot t ->
 *     i*(m+1)+t; slot t is the horizontal qubit (row b, column t, k) for
 *     t <= b and the vertical qubit (row t-1, column b, k) for t > b; J_ij
 *     (i<j) couples slot j/4+1 of chain i with slot i/4 of chain j (the
 *     vertical and horizontal qubits of cell (j/4, i/4)); h_i on slot 0.
 *   - SQA state layout in host and device memory: [replica][slice][site]
 *     (slice-major), int8.  Energies: [replica][slice], int32.
 *   - All device work is asynchronous on the HIP stream passed as `stream`
 *     (a hipStream_t; NULL = the default stream).  Reading calls synchronise
 *     with the handle's last stream themselves.
 *   - Every call returns sqa_status; nothing throws across the ABI.  On
 *     failure sqa_last_error() returns a thread-local message.
 *   - The library deep-copies every input at create/submit time.  Caller
 *     buffers passed to read calls must hold at least `len` elements; a
 *     shorter `len` than required returns SQA_ERR_INVALID.
 *   - Results depend only on (problem, embedding, schedule, seed): never on
 *     batch composition, launch shape or how the sweeps are split into calls.
 */
#ifndef SQA_MI355X_H
#define SQA_MI355X_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define SQA_API __attribute__((visibility("default")))
#else
#define SQA_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SQA_OK = 0,
  SQA_ERR_INVALID = -1,     /* bad argument, short buffer, wrong state */
  SQA_ERR_OOM = -2,         /* device or host allocation failed */
  SQA_ERR_DEVICE = -3,      /* a HIP call failed; the handle is poisoned */
  SQA_ERR_UNSUPPORTED = -4, /* valid for the method, outside this library's limits */
  SQA_ERR_BUSY = -5,        /* server: no slot / memory right now */
  SQA_ERR_NOT_READY = -6,   /* server: result not finished yet */
  SQA_ERR_CANCELLED = -7    /* server: the job was cancelled before it finished */
} sqa_status;

typedef enum { SQA_EMB_ME = 0, SQA_EMB_LHZ = 1, SQA_EMB_ME_CHIMERA = 2 } sqa_emb_kind;

/* Eq. (1): H_P = sum_i h_i s_i + sum_{i<j} J_ij s_i s_j. */
typedef struct {
  int32_t n;          /* logical spins; ME: 2..256, LHZ: 3..256 */
  const int32_t *J;   /* n*n, row-major, i<j read */
  const int32_t *h;   /* n or NULL; must be NULL/zero for LHZ (ancilla not supported) */
} sqa_problem;

typedef struct {
  int32_t kind;       /* sqa_emb_kind */
  int32_t penalty;    /* ME: J_F; LHZ: C (signed coefficient, e.g. -2) */
} sqa_embedding;

/* SQA update move (Sec. III).
 *   SQA_MOVE_METROPOLIS  single-site Metropolis on the space-time lattice; a
 *                        sweep visits every (site, slice) once, by slice
 *                        parity, colour class, slice, site.
 *   SQA_MOVE_WOLFF       the paper's move: for every site, one Wolff cluster
 *                        along imaginary time.  Aligned ring bonds join with
 *                        probability 1 - tanh(beta Gamma / L), the cluster is
 *                        the run of joined bonds through a uniform seed slice,
 *                        and it flips with min(1, exp(2 beta B / L sum s f)).
 *                        A sweep visits the sites by colour class, then index.
 * Random words: Philox4x32-10 keyed by the seed, stream SQA (2) for
 * Metropolis and WOLFF (7) for Wolff moves; both moves start from the same
 * INIT-stream lattice. */
typedef enum { SQA_MOVE_METROPOLIS = 0, SQA_MOVE_WOLFF = 1 } sqa_move;

/* Annealing schedule (Eq. (2)): sweep m uses Gamma_m (transverse field A) and
 * B_m.  Gamma_m = gamma_start (1 - t) + gamma_end t, t = m / (sweeps - 1),
 * unless `gamma` supplies all `sweeps` values; B_m = 1 unless `bscale` does.
 * Trotter slices L: 1 (classical) or even, at most 64. */
typedef struct {
  double beta;        /* inverse temperature, > 0 */
  int32_t slices;     /* L */
  int32_t sweeps;     /* M >= 1 */
  int32_t replicas;   /* independent Markov chains, 1..65536 */
  double gamma_start;
  double gamma_end;
  const double *gamma;   /* [sweeps] or NULL */
  const double *bscale;  /* [sweeps] or NULL */
  uint64_t seed;         /* Philox key */
  int32_t move;          /* sqa_move; 0 = SQA_MOVE_METROPOLIS */
} sqa_schedule;

/* Device-memory provider.  alloc(bytes, ctx) returns device memory of at least
 * `bytes` bytes on the current device, aligned to 256 bytes, or NULL when it has
 * none; free(ptr, ctx) gives it back.  A handle takes all of its device buffers
 * from it (site records, tables, lattice, energies, logical problem, decoder
 * scratch) and frees them in sqa_destroy, after its queued work has finished;
 * the server also takes its launch scratch from it.  The callbacks may be called
 * from the server's worker thread.  The struct is copied; `ctx` must stay valid
 * while anything created with it lives.  NULL = hipMalloc / hipFree. */
typedef struct {
  void *(*alloc)(size_t bytes, void *ctx);
  void (*free)(void *ptr, void *ctx);
  void *ctx;
} sqa_allocator;

typedef struct sqa_handle sqa_handle;
typedef struct sqa_batch sqa_batch;
typedef struct pt_handle pt_handle;
typedef struct sqa_server sqa_server;

/* Launch shape of the persistent sweep kernel.  Every field 0 = choose
 * automatically (the autotuner's cached choice for this device and shape).
 * Chosen automatically, a set of Metropolis handles holding at most 1024
 * replicas in all runs in team mode instead: each workgroup anneals a single
 * replica with up to 8 waves that share its colour classes (lower latency when
 * few replicas are resident; results are identical).  A nonzero
 * waves_per_group keeps one wave per replica. */
typedef struct {
  int32_t waves_per_group;    /* replicas processed together by one workgroup: 1..8 */
  int32_t groups_per_cu;      /* resident workgroups per compute unit targeted by the grid */
} sqa_launch_config;

/* ---------------------------------------------------------------- SQA */

/* Builds the embedding (Sec. II A / II B), its four-colour update classes,
 * the per-sweep acceptance-threshold table and the device buffers, which come
 * from `allocator` (NULL = hipMalloc): one block for the handle, and a second
 * one later for the scratch of the LHZ decoders.  No device work is queued;
 * the lattice is initialised by the first anneal.
 * Errors: SQA_ERR_INVALID (null pointers, n out of range, slices odd > 1,
 * sweeps < 1, replicas out of range, beta <= 0, negative Gamma, an allocator
 * without both callbacks), SQA_ERR_UNSUPPORTED (LHZ with h != 0, slices > 64,
 * a site whose |h| + sum of |incident coefficients| exceeds 255),
 * SQA_ERR_OOM (the allocator returned NULL or hipMalloc failed: nothing is
 * left allocated and *out is NULL), SQA_ERR_DEVICE. */
SQA_API sqa_status sqa_create(const sqa_problem *problem, const sqa_embedding *embedding,
                      const sqa_schedule *schedule, const sqa_allocator *allocator, sqa_handle **out);

/* Runs sweeps 0..M-1 from the seeded initial state (Philox INIT stream) and
 * computes per-slice energies.  Asynchronous on `stream`. */
SQA_API sqa_status sqa_anneal(sqa_handle *h, void *stream);

/* Runs sweeps m0..m1-1 (0 <= m0 < m1 <= M) on the current device state
 * (initialising it first if no sweep has run), then recomputes energies.
 * Splitting 0..M into ranges gives bit-identical results (checkpoint/resume). */
SQA_API sqa_status sqa_anneal_range(sqa_handle *h, int32_t m0, int32_t m1, void *stream);

/* Resets the device state to the seeded initial lattice. */
SQA_API sqa_status sqa_reset(sqa_handle *h, void *stream);

/* Waits for the handle's queued work.  SQA_ERR_DEVICE if it failed. */
SQA_API sqa_status sqa_sync(sqa_handle *h);

/* Copies the spins [replica][slice][site] (len >= replicas*slices*sites) or
 * the energies [replica][slice] to host memory, after waiting for the handle. */
SQA_API sqa_status sqa_read_spins(sqa_handle *h, int8_t *out, size_t len);
SQA_API sqa_status sqa_read_energies(sqa_handle *h, int32_t *out, size_t len);

/* Replaces the device state (checkpoint restore); values must be +1/-1. */
SQA_API sqa_status sqa_write_spins(sqa_handle *h, const int8_t *in, size_t len);

/* Device addresses of the spin and energy buffers (for zero-copy use from
 * frameworks that wrap device pointers).  Owned by the handle. */
SQA_API void *sqa_device_spins(sqa_handle *h);
SQA_API void *sqa_device_energies(sqa_handle *h);

/* Decoders, on slice `readout_slice` of every replica; all run on the device.
 *   SQA_DEC_ME_MAJORITY  Eq. (4): qbar_i = sign(sum of chain i), tie -> +1.
 *   SQA_DEC_LHZ_TREES    Eq. (5): majority over n_trees spanning trees given
 *                        as parent arrays tree_parents[n_trees][n] rooted at
 *                        logical spin 0 (parent -1), qbar_0 = +1, tie -> +1.
 *                        n <= 256.
 *   SQA_DEC_LHZ_MWD      Sec. IV A: the constraint-satisfying state nearest in
 *                        Hamming distance; exhaustive search over the 2^(n-1)
 *                        logical states with qbar_0 = +1, ties -> the candidate
 *                        whose bit pattern (bit b set <=> qbar_{b+1} = -1) is
 *                        smallest.  n <= 32.
 *   SQA_DEC_LHZ_MLD      Sec. IV B, Eq. (11): qbar_i = sign <qbar_0 qbar_i> of the
 *                        thermal average at the Nishimori inverse temperature
 *                        beta_N = ln((1-p)/p)/2 of P(sigma) ~ exp(beta_N sum
 *                        s_ij sigma_i sigma_j), exact over the 2^(n-1) states;
 *                        Boltzmann weights relative to the best state are
 *                        quantised to 2^-36 and summed in 64-bit integers.
 *                        tie -> +1.  n <= 24.  p = error_rate.
 *   SQA_DEC_LHZ_BP       Sec. IV D: pair values x = s updated `iterations`
 *                        times, all pairs together, by the weighted vote
 *                        x_ij <- sign(w0 s_ij + w1 sum_{l != i,j} x_il x_lj),
 *                        w0 = ln((1-p)/p), w1 = ln((1-p2)/p2), p2 = 2p(1-p),
 *                        a tie keeps s_ij; then the trees decode x as for
 *                        SQA_DEC_LHZ_TREES (the paper reads out with one random
 *                        tree).  n <= 32.
 * Outputs: logical[replica][n] (+1/-1) and logical energy[replica] (Eq. (1) of
 * the decoded state).
 * Errors: SQA_ERR_INVALID on a decoder/embedding mismatch, bad slice, bad
 * trees, error rate outside (0, 1/2) or negative iterations;
 * SQA_ERR_UNSUPPORTED above the size limits. */
typedef enum {
  SQA_DEC_ME_MAJORITY = 0,
  SQA_DEC_LHZ_TREES = 1,
  SQA_DEC_LHZ_MWD = 2,
  SQA_DEC_LHZ_MLD = 3,
  SQA_DEC_LHZ_BP = 4
} sqa_decoder;

typedef struct {
  int32_t decoder;               /* sqa_decoder */
  int32_t readout_slice;         /* 0..slices-1 */
  const int32_t *tree_parents;   /* [n_trees][n], for SQA_DEC_LHZ_TREES and SQA_DEC_LHZ_BP */
  int32_t n_trees;
  double error_rate;             /* p of SQA_DEC_LHZ_MLD and SQA_DEC_LHZ_BP */
  int32_t iterations;            /* rounds of SQA_DEC_LHZ_BP (0 = trees on the raw readout) */
} sqa_decode_params;

/* Queues the decoder on `stream` after the handle's previous work.  With both
 * outputs NULL the call returns at once and the results stay in device memory
 * (sqa_device_logical / sqa_device_logical_energies); otherwise it waits and
 * copies them to logical_out (len replicas*n) and logical_energy_out (len
 * replicas).  Decoders that take host tables (trees, MLD, BP) first wait for
 * the handle's earlier work. */
SQA_API sqa_status sqa_decode_ex(sqa_handle *h, const sqa_decode_params *params, int8_t *logical_out,
                         int32_t *logical_energy_out, void *stream);

/* Blocking form on the default stream, with error_rate = 0.2 and 10 iterations
 * (the paper's BP settings, Sec. IV E). */
SQA_API sqa_status sqa_decode(sqa_handle *h, int32_t decoder, int32_t readout_slice,
                      const int32_t *tree_parents, int32_t n_trees,
                      int8_t *logical_out, int32_t *logical_energy_out);

/* Device buffers holding the last decode's logical states [replica][n] (int8)
 * and logical energies [replica] (int32).  Owned by the handle. */
SQA_API void *sqa_device_logical(sqa_handle *h);
SQA_API void *sqa_device_logical_energies(sqa_handle *h);

/* Waits for the handle and copies the last decode's logical states (len >=
 * replicas*n) and logical energies (elen >= replicas); either may be NULL. */
SQA_API sqa_status sqa_read_logical(sqa_handle *h, int8_t *logical_out, size_t len, int32_t *energy_out,
                            size_t elen);

/* Exact ground state of the logical problem (Eq. (1)) by exhaustive search on
 * the device over the 2^(n-1) states with s_0 = +1 and their global flips:
 * the ground energy and one ground state (the first in the order: candidate
 * index m, bit b set <=> s_{b+1} = -s_0, then unflipped before flipped).
 * Used to score decoded anneals (success probability).  Blocking.
 * Errors: SQA_ERR_INVALID (null, n < 2); SQA_ERR_UNSUPPORTED (n > 32,
 * |J| or |h| >= 2^15).  Either output may be NULL. */
SQA_API sqa_status sqa_ground_state(const sqa_problem *problem, int32_t *energy_out, int8_t *state_out);

/* Uniform random labelled spanning trees of K_n (Pruefer sequences drawn from
 * the Philox TREE stream keyed by `seed`), as parent arrays rooted at 0:
 * parents_out[n_trees][n]. */
SQA_API sqa_status sqa_random_trees(uint64_t seed, int32_t n, int32_t n_trees, int32_t *parents_out);

/* Exports the handle's acceptance-threshold table T[m][a+F][(b+2)/2]
 * (uint32, M*(2F+1)*3 entries) and F, for parity checks.  Metropolis
 * handles only (SQA_ERR_INVALID for a Wolff handle). */
SQA_API sqa_status sqa_export_table(sqa_handle *h, uint32_t *out, size_t len, int32_t *F_out);

/* Exports a Wolff handle's tables: join thresholds padd[M] (accept a bond iff
 * word < threshold, or always for 0xFFFFFFFF) and acceptance thresholds
 * acc[rows][2 L F + 1] indexed by A + L F (rows = M when the schedule has
 * bscale, else 1).  Either output may be NULL; rows_out / width_out report the
 * shape.  SQA_ERR_INVALID for a Metropolis handle or a short buffer. */
SQA_API sqa_status sqa_export_wolff_tables(sqa_handle *h, uint32_t *padd_out, size_t padd_len, uint32_t *acc_out,
                                   size_t acc_len, int32_t *rows_out, int32_t *width_out);

/* Device bytes the handle holds through its allocator: its own block plus the
 * decoder scratch allocated so far. */
SQA_API sqa_status sqa_handle_device_bytes(sqa_handle *h, size_t *bytes_out);

/* Shape queries. */
SQA_API int64_t sqa_physical_sites(int32_t kind, int32_t n);
SQA_API sqa_status sqa_handle_info(sqa_handle *h, int32_t *sites, int32_t *slices, int32_t *replicas,
                           int32_t *sweeps, int32_t *fmax);

SQA_API void sqa_destroy(sqa_handle *h);

/* ------------------------------------------------------- batched SQA */

/* A batch runs every handle's full anneal (init, sweeps 0..M-1, energies) in
 * ONE persistent launch: work items (handle, group of replicas) are sorted
 * by cost (longest first) and pulled from a device work counter.  The launch
 * sequence is captured once in a HIP graph and replayed by sqa_batch_run.
 * `config` NULL or zero fields = autotuned.  The handles must outlive the
 * batch and must not be used concurrently with it. */
SQA_API sqa_status sqa_batch_create(sqa_handle *const *handles, int32_t count,
                            const sqa_launch_config *config, sqa_batch **out);
/* sqa_batch_create with a decoder per handle, captured in a second graph that
 * sqa_batch_run replays right after the anneal's on the same stream: every run
 * does init -> sweeps -> energies -> decoding (Eq. (4), Eq. (5), Sec. IV A-D)
 * and leaves each handle's logical states and their energies in its device
 * buffers (sqa_read_logical, sqa_device_logical).
 * decoders[count], one per handle; an entry whose decoder is -1 decodes
 * nothing.  The decoders' host tables (tree orders, MLD weights, BP votes) are
 * copied at creation into scratch the batch owns; tree parents are copied.
 * Errors: those of sqa_batch_create and of sqa_decode_ex's checks. */
SQA_API sqa_status sqa_batch_create_decoded(sqa_handle *const *handles, int32_t count,
                                    const sqa_launch_config *config, const sqa_decode_params *decoders,
                                    sqa_batch **out);
SQA_API sqa_status sqa_batch_run(sqa_batch *b, void *stream);
/* Durations of the last sqa_batch_run, from HIP events recorded on its stream
 * before the anneal graph, between it and the decoder graph, and after both:
 * the anneal's and the decoders' (0 without decoders).  Waits for the run.
 * SQA_ERR_INVALID before any run. */
SQA_API sqa_status sqa_batch_timing(sqa_batch *b, float *anneal_ms, float *decode_ms);
SQA_API sqa_status sqa_batch_config(sqa_batch *b, sqa_launch_config *out);
SQA_API void sqa_batch_destroy(sqa_batch *b);

/* One-shot convenience: create, run on `stream`, destroy (no graph reuse). */
SQA_API sqa_status sqa_anneal_batch(sqa_handle *const *handles, int32_t count, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): sqa_anneal_batch with
 * the same results, whose launch scratch (handle descriptors, work items, work
 * counters) is a file-scope device array of the library, 4 MiB per GPU, held by
 * every GPU the library runs on until the process ends, instead of a fresh
 * allocation.  It calls no allocating routine and captures no graph; it returns
 * after the launch on `stream` has finished.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (from several host threads) race.
 * SQA_ERR_UNSUPPORTED when the batch's scratch (descriptors of `count` handles
 * plus at most one work item per replica) exceeds the array. */
SQA_API sqa_status sqa_anneal_batch_noalloc(sqa_handle *const *handles, int32_t count, void *stream);

/* Autotuner: times candidate launch shapes on the given handles (short
 * sweep ranges, device state restored afterwards) and stores the best per
 * (device architecture, shape class) in the JSON cache at `cache_path`
 * (NULL = $SQA_AUTOTUNE_CACHE or no file).  Returns the choice in *best. */
SQA_API sqa_status sqa_autotune(sqa_handle *const *handles, int32_t count, const char *cache_path,
                        sqa_launch_config *best);

/* ------------------------------------------------------ parallel tempering */

/* Appendix B: `temps` replicas of the classical embedded Hamiltonian at
 * beta_r = beta_max (beta_min/beta_max)^(r/(temps-1)) (slot 0 coldest),
 * single-spin Metropolis sweeps, and after every sweeps_per_swap sweeps one
 * swap phase (even slot pairs, then odd pairs) with Eq. (B1)'s probability.
 * temps: 1..64. */
typedef struct {
  double beta_min;
  double beta_max;
  int32_t temps;
  int32_t sweeps;
  int32_t sweeps_per_swap;
  uint64_t seed;
} pt_params;

SQA_API sqa_status pt_create(const sqa_problem *problem, const sqa_embedding *embedding,
                     const pt_params *params, pt_handle **out);
/* Runs the whole PT schedule from the seeded initial state on `stream` and
 * waits for it (blocking). */
SQA_API sqa_status pt_run_handle(pt_handle *h, void *stream);
/* All handles in one launch (one workgroup per ladder); blocking. */
SQA_API sqa_status pt_run_batch(pt_handle *const *handles, int32_t count, void *stream);
/* Results after a run, blocking.  spins_out[temp][site] and energies_out[temp]
 * are ordered BY SLOT (temperature), slot_to_replica_out[temp] gives the
 * replica in each slot, swap_accepts_out[temps-1] counts accepted swaps per
 * slot pair.  Any output may be NULL. */
SQA_API sqa_status pt_read(pt_handle *h, int8_t *spins_out, size_t spins_len, int32_t *energies_out,
                   int32_t *slot_to_replica_out, uint64_t *swap_accepts_out);
SQA_API void pt_destroy(pt_handle *h);

/* One-shot: create, run, read, destroy. */
SQA_API sqa_status pt_run(const sqa_problem *problem, const sqa_embedding *embedding,
                  const pt_params *params, void *stream, int8_t *spins_out, size_t spins_len,
                  int32_t *energies_out, int32_t *slot_to_replica_out,
                  uint64_t *swap_accepts_out);

/* ------------------------------------------------------------- serving */

/* Continuous batching.  Jobs wait in FIFO order and are admitted while their
 * device bytes fit in `hbm_budget_bytes` and fewer than `max_slots` are
 * resident; admitted jobs advance together, `chunk_sweeps` sweeps per
 * persistent launch, and a job that finishes is decoded on the device, copied
 * to the host, and frees its slot and memory for the next waiting job at the
 * following launch boundary.  Results are bit-identical to running the job
 * alone.  Device memory (job handles, decoder scratch, the shared launch
 * scratch) comes from `allocator` (NULL = hipMalloc).  Admission counts it
 * exactly: a job is charged its handle's block, its decoder's scratch and its
 * entries in the launch scratch, each rounded up to 4 KiB
 * (sqa_server_job_bytes), and the launch scratch's fixed part (4 KiB) is
 * charged once; the sum of what the allocator holds never exceeds the budget.
 * A server thread owns the device work. */
SQA_API sqa_status sqa_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t chunk_sweeps,
                             const sqa_allocator *allocator, sqa_server **out);
/* Queues a job (inputs deep-copied; the embedding, layout and tables are built
 * here, on the caller's thread).  `decode` picks the decoder run on the device
 * when the job finishes (Eq. (4), Eq. (5), Sec. IV A-D; tree parents are
 * copied); NULL = majority vote of the chains (ME, ME on Chimera) or
 * minimum-weight decoding (LHZ, n <= 32; chain-tree decoding, Eq. (A1), above),
 * on slice 0.  SQA_ERR_INVALID for a bad job or decoder, SQA_ERR_BUSY if the
 * job alone exceeds the budget. */
SQA_API sqa_status sqa_server_submit(sqa_server *s, const sqa_problem *problem,
                             const sqa_embedding *embedding, const sqa_schedule *schedule,
                             const sqa_decode_params *decode, uint64_t *ticket);
/* Device bytes admission charges for a queued or running job. */
SQA_API sqa_status sqa_server_job_bytes(sqa_server *s, uint64_t ticket, size_t *bytes_out);
/* Cancels a job: a waiting job is dropped at once, a running one at the next
 * launch boundary (its device memory is then freed).  Its wait and result then
 * return SQA_ERR_CANCELLED (result releases the ticket).  SQA_ERR_INVALID for an
 * unknown ticket or a job that has already finished. */
SQA_API sqa_status sqa_server_cancel(sqa_server *s, uint64_t ticket);
/* *done = 1 once the job has finished (or been cancelled, or failed). */
SQA_API sqa_status sqa_server_poll(sqa_server *s, uint64_t ticket, int32_t *done);
/* Blocks until done (timeout_ms < 0: forever); SQA_ERR_NOT_READY on timeout,
 * else the job's status. */
SQA_API sqa_status sqa_server_wait(sqa_server *s, uint64_t ticket, int32_t timeout_ms);
/* Copies a finished job's spins [replica][slice][site], energies
 * [replica][slice], decoded logical states [replica][n] and their energies
 * under Eq. (1) [replica]; any output may be NULL.  Latency in seconds from
 * submit to result-on-host goes to *latency_s (may be NULL).  The ticket is
 * released. */
SQA_API sqa_status sqa_server_result(sqa_server *s, uint64_t ticket, int8_t *spins, size_t spins_len,
                             int32_t *energies, size_t energies_len, int8_t *logical, size_t logical_len,
                             int32_t *logical_energies, size_t logical_energies_len, double *latency_s);
/* Counters: completed jobs, device launches, peak resident bytes. */
SQA_API sqa_status sqa_server_stats(sqa_server *s, uint64_t *completed, uint64_t *launches,
                            uint64_t *peak_bytes);
SQA_API void sqa_server_destroy(sqa_server *s);

/* ------------------------------------------------------------- misc */
SQA_API const char *sqa_last_error(void);
SQA_API const char *sqa_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SQA_MI355X_H */
