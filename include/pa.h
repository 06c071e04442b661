/*
 * pa.h -- C ABI of the MI355X (gfx950) pilot-assignment library.
 *
 * The library runs the K-means-seeded elitist two-dimensional genetic
 * algorithm of Alqudah & Khokhar, "Efficient Parallel Implementation of the
 * Pilot Assignment Problem in Massive MIMO Systems":
 *   - a chromosome is an L x K matrix of pilot indices, row j being the
 *     pilots of the K users of cell j, a permutation of the tau = K pilots
 *     (Sec. 4.1, chromosome encoding; Sec. 3.3, pilots unique inside a cell
 *     and reused across cells);
 *   - its fitness is the uplink sum spectral efficiency (Sec. 3.2, Eq. 5-6),
 *     the objective of Eq. 7, optionally scaled by the share 1 - tau/T of the
 *     coherence interval left after uplink training (Sec. 3);
 *   - the population is seeded by K-means clustering of the users
 *     (Sec. 1 contribution 2, Sec. 4.1, Alg. 1) and evolved with elitism
 *     (Sec. 1 contribution 1), selection, crossover and mutation (Alg. 1).
 *
 * Conventions
 *   - Status: every call returns pa_status; 0 is success, negative is an
 *     error.  pa_last_error() returns a thread-local message for the last
 *     error raised on the calling thread.  No C++ exception crosses the ABI.
 *   - Memory: "HOST" pointers are ordinary host memory, "DEVICE" pointers are
 *     device memory of the context's GPU (e.g. a torch tensor's data_ptr()).
 *     The caller owns every buffer it passes; objects created by the library
 *     own only their internal copies and are released by their destroy call.
 *   - Streams: `stream` is a hipStream_t of the context's device (NULL = the
 *     null stream).  Calls marked "async" only enqueue work; their outputs are
 *     valid once the stream has been synchronised.  Calls marked "blocking"
 *     return after their host outputs are written.
 *   - Layouts are dense, row-major, with the index names of the paper:
 *       beta[(l*L + j)*K + k]  large-scale fading of user k of cell j at the
 *                              BS of cell l (Sec. 3.1, Eq. 1-2), FP64;
 *       pop[(n*L + j)*K + k]   pilot (0..K-1) of user k of cell j in
 *                              chromosome n, uint8;
 *       fit[n]                 FP32 sum SE of chromosome n (pre-log applied).
 *   - Random numbers: every random decision is a pure function of
 *     (seed, instance_id, generation, slot), drawn from Philox4x32-10, so
 *     results do not depend on launch shapes, batching or timing.
 *   - Thread safety: a context and its instances must not be used from two
 *     threads at once.  The server's submit and poll calls are thread-safe.
 */
#ifndef PA_H
#define PA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pa_status;
enum {
  PA_OK = 0,
  PA_EINVAL = -1,      /* an argument is out of its documented range */
  PA_ENOMEM = -2,      /* device or host allocation failed */
  PA_EDEVICE = -3,     /* a HIP runtime call or kernel launch failed */
  PA_EAGAIN = -4,      /* not finished yet (server poll) or queue full */
  PA_ECANCELED = -5,   /* request cancelled */
  PA_EINTERNAL = -6,   /* library bug: please report */
  PA_EUNSUPPORTED = -7 /* valid request the library cannot serve (e.g. not a gfx950 device) */
};

/* Fitness modes.
 * PA_SE_ASYMPTOTIC: Eq. 5, the M -> infinity uplink SE
 *   SE_ik = log2(1 + beta_iik^2 / sum_{j != i} beta_ijk'^2), where k' is the
 *   user of cell j that reuses user (i,k)'s pilot.  M and rho are ignored.
 * PA_SE_FINITE_M: the finite-antenna uplink bound whose limit is Eq. 5 (the
 *   paper's Eq. 3 is garbled): maximum-ratio combining, MMSE estimates from
 *   tau-symbol orthogonal pilots, pilot and data SNR rho:
 *   SINR = M tau rho^2 b^2 / ((1 + rho B_i)(1 + tau rho S) + M tau rho^2 I),
 *   b = beta_iik, S = sum_j beta_ijk' (own user included),
 *   I = sum_{j != i} beta_ijk'^2, B_i = sum over all users of beta_i..   */
enum { PA_SE_ASYMPTOTIC = 0, PA_SE_FINITE_M = 1 };

/* Objectives (the GA maximises the fitness).
 * PA_OBJ_SUM_SE: Eq. 7, the sum over all users of their SE, x pre-log.
 * PA_OBJ_MIN_SINR: the smallest SINR of any user (SIR in asymptotic mode):
 *   the max-min SIR criterion the paper names beside the sum (Sec. 2).  SE is
 *   monotone in SINR, so this is also the max-min SE assignment; the SINR
 *   keeps FP32 precision where log2(1 + SINR) of a weak user would not.
 * PA_OBJ_INTERCLUSTER: minus the inter-cluster interference of Eq. 8
 *   (Sec. 4.2), read with tau = K as clusters of one user per (cell, pilot):
 *   -sum over users (i, k) of sum_{j != i} beta_ijk' / beta_iik, first powers
 *   of beta, k' the user of cell j on the pilot of (i, k); no pre-log;
 *   asymptotic mode only (PA_EINVAL with PA_SE_FINITE_M). */
enum { PA_OBJ_SUM_SE = 0, PA_OBJ_MIN_SINR = 1, PA_OBJ_INTERCLUSTER = 2 };

typedef struct pa_context pa_context;
typedef struct pa_instance pa_instance;
typedef struct pa_server pa_server;

/* One pilot-assignment problem (the inputs of Alg. 1/Alg. 2: cells L,
 * pilots K, the fading table beta; plus the coherence length T).
 *   L        cells, 1..64 (2..64 in asymptotic mode: one cell has no
 *            interference and an unbounded SINR)
 *   K        users per cell, 1..64
 *   tau      pilots; must equal K (pilots are a permutation inside a cell)
 *   T        coherence length in symbols; 0 = no pre-log, else T > tau
 *   M        BS antennas (finite-M mode), >= 1
 *   rho      transmit SNR (finite-M mode), > 0
 *   se_mode  PA_SE_ASYMPTOTIC or PA_SE_FINITE_M
 *   objective  PA_OBJ_SUM_SE (0), PA_OBJ_MIN_SINR (1) or PA_OBJ_INTERCLUSTER (2)
 *   beta     HOST [L][L][K] FP64, finite; > 0 in asymptotic mode, >= 0 in
 *            finite-M mode; per BS l the ratio max/min over the nonzero
 *            entries must not exceed 2^60 (FP32 range after normalisation)
 *   user_xy  HOST [L][K][2] metres, or NULL (then only kmeans_frac == 0)
 *   bs_xy    HOST [L][2] metres, or NULL (same)
 *            user offsets from their own BS must be below 8388 m.        */
typedef struct pa_problem {
  int32_t L, K, tau, T, M;
  double rho;
  int32_t se_mode;
  const double *beta;
  const double *user_xy;
  const double *bs_xy;
  int32_t objective;
} pa_problem;

/* GA parameters.
 *   pop          population size N, 2..65536
 *   gens         generations G >= 0 (a fixed number reads "termination")
 *   elite        E in [0, N]: slots 0..E-1 receive the E best, in order
 *   p_cross      probability of single-point crossover on the cell axis
 *   p_mut        per-gene probability of a swap mutation
 *   kmeans_frac  share of the initial population derived from the K-means
 *                seed (0 = random initialisation, the conventional GA)
 *   p_init       per-gene swap probability used to perturb the seed
 *   seed         64-bit Philox key
 *   instance_id  distinguishes instances sharing a seed (Philox counter)   */
typedef struct pa_ga_params {
  int32_t pop, gens, elite;
  double p_cross, p_mut, kmeans_frac, p_init;
  uint64_t seed;
  uint32_t instance_id;
} pa_ga_params;

/* Result of a solve.
 *   best        HOST, caller-allocated, L*K bytes: best chromosome of the
 *               last population
 *   best_fit    its FP32 fitness
 *   best_index  its slot in the last population
 *   trace       HOST [gens+1] or NULL: best fitness of each generation
 *   device_ms   device time of the solve (events on the solve's stream)  */
typedef struct pa_result {
  uint8_t *best;
  float best_fit;
  int32_t best_index;
  float *trace;
  double device_ms;
} pa_result;

/* ---- validation (host only, no device needed) ------------------------ */

/* Checks a problem against the ranges documented at pa_problem.  Returns
 * PA_OK or PA_EINVAL (message in pa_last_error()). */
pa_status pa_problem_check(const pa_problem *prob);
/* Checks GA parameters against the ranges documented at pa_ga_params, for
 * the given (valid) problem (kmeans_frac > 0 needs positions). */
pa_status pa_params_check(const pa_problem *prob, const pa_ga_params *params);

/* ---- context and instances ------------------------------------------- */

/* Creates a context on HIP device `device`.  Blocking. */
pa_status pa_context_create(int32_t device, pa_context **out);
void pa_context_destroy(pa_context *ctx);

/* Validates a problem (see pa_problem), copies beta and the positions to the
 * device and builds the device-side tables: per BS l, beta is scaled by a
 * power of two 2^-e_l so its largest entry lies in [0.5, 1) (this leaves
 * Eq. 5 unchanged and keeps squares inside FP32 range) and the squares are
 * rounded to FP32.  Blocking.  PA_EINVAL on invalid input. */
pa_status pa_instance_create(pa_context *ctx, const pa_problem *prob, pa_instance **out);
void pa_instance_destroy(pa_instance *inst);

/* ---- the per-generation hot path ------------------------------------- */

/* K-means seeding and the initial population (Sec. 4.1; the population
 * initialisation of Alg. 1): clusters the users' offsets from their own BS
 * (integer millimetres) into K groups (farthest-point start, integer Lloyd
 * iterations, at most 100), matches each cell's users to the clusters
 * greedily (cluster index = pilot) to form the seed chromosome, then fills
 * d_pop [N][L][K] (DEVICE): slot 0 the seed, slots 1..n_km-1 the seed
 * swap-mutated at rate p_init, the rest uniformly random permutations, with
 * n_km = max(1, floor(kmeans_frac*N + 1/2)) (0 when kmeans_frac == 0).
 * Async. */
pa_status pa_kmeans_init(pa_instance *inst, const pa_ga_params *params, uint8_t *d_pop,
                         void *stream);

/* Fitness (Eq. 5-7) of n chromosomes: d_pop [n][L][K] (DEVICE) ->
 * d_fit [n] (DEVICE, FP32).  Rows must be permutations (not checked).
 * The FP32 result is within 1e-5 relative of the FP64 definition and is
 * bit-identical for a chromosome whatever n, the batch or the launch shape.
 * Async.  n == 0 is a no-op. */
pa_status pa_fitness(pa_instance *inst, const uint8_t *d_pop, int32_t n, float *d_fit,
                     void *stream);

/* One generation (Alg. 1 loop body): from d_pop_in [N][L][K] and its
 * fitness d_fit_in [N] (both DEVICE) writes d_pop_out [N][L][K] (DEVICE):
 * slots 0..E-1 = the E best (fitness descending, lower slot first on ties,
 * NaN last), then children in pairs (a, a+1): two binary tournaments choose
 * the parents, single-point crossover on the cell axis with p_cross, swap
 * mutation per gene with p_mut.  d_pop_in and d_pop_out must not overlap.
 * Async. */
pa_status pa_ga_step(pa_instance *inst, const pa_ga_params *params, int32_t gen,
                     const uint8_t *d_pop_in, const float *d_fit_in, uint8_t *d_pop_out,
                     void *stream);

/* A whole solve: seeding, then `gens` generations of select / evolve /
 * evaluate with the population resident on the device, then the best
 * chromosome of the last population (Alg. 1, which returns the best
 * assignment).  Children are built, written and evaluated in LDS by one
 * fused generation kernel.  The first call with given parameters builds a
 * plan: when every task of a generation fits on the device at once (small
 * instances) all generations run in one launch, either separated by grid
 * barriers (persistent form) or, when the population and the table fit one
 * CU's LDS, in one workgroup that keeps them there (one-workgroup form), the
 * form and the tasks' size autotuned on the instance itself; otherwise the
 * whole solve (one launch per generation) is captured into a hipGraph.
 * Later calls with the same parameters replay the plan.  The form and the
 * shape never change a result bit.  The environment variable
 * PA_PERSIST_BLOCK=256 or 512, read when a plan is built, restricts the
 * autotuner to that workgroup size (for reproducible profiles; unset, both
 * are tried); PA_SMALL_FORM=persistent or workgroup keeps only that form.
 * PA_EINTERNAL if a grid barrier wait times out (the results are then
 * invalid).  Blocking. */
pa_status pa_solve(pa_instance *inst, const pa_ga_params *params, pa_result *out, void *stream);

/* Many independent solves in one: n instances of the same context, each with
 * its own parameters (sizes may differ), run generation by generation, each
 * generation one launch per class of (L, padded K, SE mode) covering every
 * instance of the class; the whole batch is captured once into a hipGraph
 * and replayed while (instances, params) stay the same.  results[i] is filled
 * as pa_solve would fill it and is bit-identical to a pa_solve of instance i
 * alone; device_ms is the time of the whole batch.  An instance may appear
 * only once.  Blocking. */
pa_status pa_solve_batch(pa_context *ctx, int32_t n, pa_instance *const *insts,
                         const pa_ga_params *params, pa_result *results, void *stream);

/* Stepwise solve, for callers that decide themselves when to stop (Alg. 1
 * loops until an unspecified termination condition holds); same kernels and
 * bits as pa_solve.
 *   pa_solve_begin  seeding, initial population and its fitness.  Async.
 *   pa_solve_next   ngens more generations (one launch in the persistent
 *                   and one-workgroup forms, else one fused launch each); at most
 *                   params->gens in total since the last begin.  Async.
 *   pa_solve_state  best chromosome and fitness of the current population,
 *                   trace[0..gens_done]; *gens_done = generations run so far.
 *                   device_ms covers only this call.  Blocking. */
pa_status pa_solve_begin(pa_instance *inst, const pa_ga_params *params, void *stream);
pa_status pa_solve_next(pa_instance *inst, int32_t ngens, void *stream);
pa_status pa_solve_state(pa_instance *inst, pa_result *out, int32_t *gens_done, void *stream);

/* Stepwise form of pa_solve_batch (same plan, kernels and bits): begin
 * seeds every instance and evaluates its initial population, next runs
 * ngens more generations of every instance (one fused launch per class and
 * generation, or one persistent launch), state copies the best chromosome,
 * fitness and trace of each instance's current population into results[i]
 * (results[i].best and .trace as in pa_solve_batch) and *gens_done.  An
 * instance whose own gens is below the generations run stays at its last
 * generation.  begin and next: async; state: blocking. */
pa_status pa_solve_batch_begin(pa_context *ctx, int32_t n, pa_instance *const *insts,
                               const pa_ga_params *params, void *stream);
pa_status pa_solve_batch_next(pa_context *ctx, int32_t ngens, void *stream);
pa_status pa_solve_batch_state(pa_context *ctx, pa_result *results, int32_t *gens_done,
                               void *stream);

/* The current population of one instance of a solve plan (Alg. 1's
 * population P after the generations run so far): inst != NULL selects the
 * plan of pa_solve / pa_solve_begin on inst (index 0), inst == NULL the
 * context's batch plan (index = the instance's position in the batch call).
 * pop: HOST [N][L][K] bytes, fit: HOST [N] FP32 (either may be NULL); *gen
 * (may be NULL) = the generation that population belongs to.  PA_EINVAL
 * when there is no plan or it has not run, or index is out of range.
 * Blocking (orders after the work enqueued on `stream`). */
pa_status pa_solve_population(pa_context *ctx, pa_instance *inst, int32_t index, uint8_t *pop,
                              float *fit, int32_t *gen, void *stream);

/* Resume of a stepwise solve from a saved state (Alg. 1: the loop state is
 * the population P of generation gen and its fitness; every random word of a
 * generation is keyed by (seed, instance_id, generation, slot), so the
 * generations after gen depend on nothing else).  Loads into inst's solve
 * plan (built for params as pa_solve_begin builds it, without seeding):
 *   pop    HOST [N][L][K] bytes, N = params->pop: the population of
 *          generation gen, as pa_solve_population returns it; every row must
 *          be a permutation of 0..K-1 (checked: PA_EINVAL otherwise)
 *   fit    HOST [N] FP32, its fitness as this library computed it, or NULL
 *          to recompute it on the device (the same bits)
 *   trace  HOST [gen] FP32, the best fitness of generations 0..gen-1 (as
 *          pa_solve_state returned them), or NULL: those entries read NaN
 * The caller keeps ownership of the three buffers; they are copied before
 * the call returns.  Then pa_solve_next(inst, k) runs generations gen ..
 * gen + k - 1 (gen + k <= params->gens) and pa_solve_state reports as in an
 * uninterrupted solve: the same populations, best and trace entries from gen
 * on, bit for bit.  PA_EINVAL for invalid parameters, gen outside
 * [0, params->gens] or a NULL pop.  Blocking. */
pa_status pa_solve_resume(pa_instance *inst, const pa_ga_params *params, int32_t gen,
                          const uint8_t *pop, const float *fit, const float *trace,
                          void *stream);

/* The same solve as one launch per step (seeding, fitness, then per
 * generation a pa_ga_step launch and a pa_fitness launch), no fusion and no
 * graph: the plain comparator.  Bit-identical results to pa_solve. */
pa_status pa_solve_plain(pa_instance *inst, const pa_ga_params *params, pa_result *out,
                         void *stream);

/* pa_solve for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve and the same result bits as pa_solve, but no allocation of
 * any kind.  The descriptor, task lists and double-buffered populations and
 * fitness live in a fixed scratch array of the library, one per device, of
 * PA_NOALLOC_SCRATCH_BYTES (8 MiB; the solve needs about 2 N L K + 8 N
 * bytes plus 16 bytes per task of block / K chromosomes).  Outputs go to
 * caller-owned DEVICE memory:
 *   d_best      DEVICE L*K bytes: best chromosome of the last population
 *   d_best_fit  DEVICE 1 float: its fitness
 *   d_trace     DEVICE gens+1 floats (best fitness per generation), or NULL
 * It also leaves the instance's K-means state as pa_kmeans_init does.
 * Async on `stream`: outputs are valid once the stream has been
 * synchronised.  PA_EINVAL for invalid parameters or a solve larger than the
 * scratch; PA_EDEVICE when the scratch could not be located on the device.
 * Every call on a device uses that device's one scratch array: calls that
 * overlap on one device (other streams or threads) race, and a call must
 * not start before the previous one on its device has finished unless both
 * are on the same stream. */
#define PA_NOALLOC_SCRATCH_BYTES (8u << 20)
pa_status pa_solve_noalloc(pa_instance *inst, const pa_ga_params *params, uint8_t *d_best,
                           float *d_best_fit, float *d_trace, void *stream);

/* pa_fitness with an explicit launch shape, for tuning and tests:
 *   block     threads per workgroup (64..1024, multiple of 64, >= K; 0 = default)
 *   grid_cap  maximum workgroups (0 = enough to fill the GPU)
 *   generic   1 forces the runtime-L kernel instead of the unrolled one
 * Results are bit-identical to pa_fitness for every shape.  Async. */
pa_status pa_fitness_shaped(pa_instance *inst, const uint8_t *d_pop, int32_t n, float *d_fit,
                            int32_t block, int32_t grid_cap, int32_t generic, void *stream);

/* Execution form of the current solve plan of `inst` (inst != NULL, after
 * pa_solve or pa_solve_begin) or of the context's batch plan (inst == NULL,
 * after pa_solve_batch): *persistent = 1 for the persistent form (one launch,
 * grid barriers), 2 for the one-workgroup form (one workgroup per instance,
 * population in LDS), 0 for the captured graph; threads per workgroup,
 * children per task (of the first class, for its first instance's K; all
 * children in the one-workgroup form) and workgroups per launch.  Any output
 * pointer may be NULL.  PA_EINVAL when there is no plan. */
pa_status pa_solve_shape(pa_context *ctx, pa_instance *inst, int32_t *persistent, int32_t *block,
                         int32_t *children_per_task, int32_t *workgroups);

/* ---- the parallel K-means GA (islands) ------------------------------- */

/* K-means of a population into `clusters` islands (the "apply K-means" step
 * of Alg. 2, PK-means GA, Sec. 4.3): each chromosome is the point of Z^{LK}
 * formed by its pilot indices (squared Euclidean distance, exact integers);
 * farthest-point start from the best-ranked chromosome of d_fit (fitness
 * descending, lower index first; ties of distance to the lowest index), then
 * at most kmeans_iters Lloyd iterations (nearest centroid, ties to the lowest
 * cluster; centroid = per-gene rounded mean floor((2 s + n) / (2 n)); an empty
 * cluster keeps its centroid) until no label changes.
 *   d_pop [n][L][K], d_fit [n] (DEVICE): the population and its fitness
 *   d_labels [n] (DEVICE, out): island of each chromosome, 0..clusters-1
 * 1 <= clusters <= 16, clusters <= n <= 4096.  Async. */
pa_status pa_population_kmeans(pa_instance *inst, int32_t clusters, int32_t kmeans_iters,
                               const uint8_t *d_pop, const float *d_fit, int32_t n,
                               int32_t *d_labels, void *stream);

/* One generation of every island (Alg. 2 loop body: selection, crossover and
 * mutation inside each cluster), island c being the positions labelled c in
 * d_labels [N] (DEVICE): its first E_c positions receive its E_c best (in
 * rank order; E_c = 0 if E = 0, else min(n_c, max(1, floor(E n_c / N + 1/2)))),
 * its other positions children in pairs of consecutive island positions,
 * from binary tournaments among its members, cell-axis crossover and swap
 * mutation as in pa_ga_step.  The random streams are pa_ga_step's with the
 * island index in bits 16..23 of the block counter: with every label 0 the
 * result is pa_ga_step's, bit for bit.  A position whose label lies outside
 * [0, clusters) is copied unchanged.  pop <= 4096, 1 <= clusters <= 16.
 * Async (device scratch of 16 pop bytes, stream-ordered). */
pa_status pa_island_step(pa_instance *inst, const pa_ga_params *params, int32_t clusters,
                         int32_t gen, const int32_t *d_labels, const uint8_t *d_pop_in,
                         const float *d_fit_in, uint8_t *d_pop_out, void *stream);

/* The whole PK-means GA (Alg. 2): seeding and initial population as in
 * pa_solve, then per generation: K-means of the population into `clusters`
 * islands at generation 0 and every recluster_every generations (0: only at
 * 0; Sec. 6.1 uses 3), one island step, the fitness of the new population.
 * Fills out as pa_solve does; labels (HOST [pop] or NULL) receives the last
 * partition.  clusters = 1 gives pa_solve's result.  Blocking. */
pa_status pa_island_solve(pa_instance *inst, const pa_ga_params *params, int32_t clusters,
                          int32_t recluster_every, int32_t kmeans_iters, pa_result *out,
                          int32_t *labels, void *stream);

/* ---- exhaustive search ------------------------------------------------ */

/* Exhaustive search (the EX-PA reference, Sec. 3.3 and Sec. 6): every
 * assignment with cell 0's pilots fixed to the identity (the sum SE is
 * invariant under a global relabelling of pilots, so each class of K!
 * equivalent assignments is visited once), i.e. K!^(L-1) chromosomes in
 * odometer order (cell L-1 fastest, each cell's permutations in
 * lexicographic order), scored by the pa_fitness kernel.  Fills out->best
 * (HOST, L*K bytes, may be NULL), out->best_fit (FP32; ties to the lowest
 * rank), out->device_ms; out->best_index = -1 and out->trace is untouched;
 * *best_rank = the enumeration rank of the best, *count = K!^(L-1) (either
 * may be NULL).  PA_EINVAL when K > 12 or K!^(L-1) > max_count (0 = 2^32).
 * Blocking. */
pa_status pa_exhaustive(pa_instance *inst, int64_t max_count, pa_result *out, int64_t *best_rank,
                        int64_t *count, void *stream);

/* ---- continuous-batching server -------------------------------------- */

/* Many independent solves arriving over time (not in the paper; the serving
 * form of the batched solve).  A server owns a worker thread, a HIP stream, a
 * table of max_slots slots for resident requests and one device arena of the
 * HBM budget.  Each tick the worker retires requests cancelled while
 * resident, admits queued requests in arrival order while a slot is free and
 * the arena holds the head request's own bytes (its tables, double-buffered
 * populations and result, about 12 L^2 K + 2 N L K + 8 N bytes: a request
 * takes what its sizes need, not what the largest would), runs ONE
 * generation of every resident request (each at its own generation; one
 * launch per class of (L, padded K, SE mode)), and returns the requests that
 * reached their last generation.  A request's result is bit-identical to
 * pa_solve of the same problem and parameters.  If a tick fails on the
 * device, the requests resident at that moment fail with PA_EDEVICE and the
 * worker goes on with the queue while the device still answers (otherwise
 * every request fails and submit returns PA_EDEVICE).
 *   max_slots   resident requests at most (0 = 512)
 *   max_queue   waiting requests at most; beyond, submit returns PA_EAGAIN
 *               (0 = 1048576)
 *   max_L, max_K, max_pop, max_gens   largest accepted request
 *               (0 = 37, 32, 1024, 1000)
 *   hbm_budget  bytes of device memory for the arena (0 = 80% of free); the
 *               arena is the smaller of this and max_slots largest requests
 * Test hook: the environment variable PA_SERVER_FAULT_TICK=n, read at
 * creation, makes the n-th tick report a device error after its work has
 * completed (the recovery path runs, the device is not disturbed). */
typedef struct pa_server_cfg {
  int32_t max_slots, max_queue;
  int32_t max_L, max_K, max_pop, max_gens;
  double hbm_budget;
} pa_server_cfg;

/* Server counters: slots, resident and queued requests, requests submitted
 * and completed, ticks run, arena bytes of the largest accepted request, the
 * most generation tasks one workgroup ran in a single launch, the most
 * requests resident at once, requests cancelled and failed, the arena's size
 * and its peak use in bytes. */
typedef struct pa_server_counters {
  int32_t slots, resident, queued;
  uint64_t submitted, completed, ticks;
  double slot_bytes;
  int32_t max_tasks_per_workgroup;
  int32_t max_resident;
  uint64_t cancelled, failed;
  double arena_bytes, arena_peak_bytes;
} pa_server_counters;

/* Creates a server on the context's device (cfg may be NULL for defaults).
 * PA_ENOMEM when the budget holds no request.  Blocking. */
pa_status pa_server_create(pa_context *ctx, const pa_server_cfg *cfg, pa_server **out);
/* Queues a request: the problem's host arrays are copied, so the caller may
 * reuse them at once.  *ticket identifies it.  PA_EINVAL for an invalid
 * problem or parameters or one above the server's maxima, PA_ENOMEM for one
 * whose bytes exceed the whole arena, PA_EAGAIN when the queue is full.
 * Thread-safe. */
pa_status pa_server_submit(pa_server *srv, const pa_problem *prob, const pa_ga_params *params,
                           uint64_t *ticket);
/* Result of a request: fills out as pa_solve would (best and trace are
 * HOST, caller-allocated, L*K bytes and gens+1 floats, either may be NULL);
 * device_ms = time from submit to the result being on the host, in ms.
 * block = 0: PA_EAGAIN while the request runs; block != 0: waits.  A ticket
 * can be polled successfully once.  Thread-safe. */
pa_status pa_server_poll(pa_server *srv, uint64_t ticket, pa_result *out, int32_t block);
/* Cancels a request: a queued one ends at once, a resident one before the
 * worker's next tick (its arena block and slot are freed); polling it then
 * returns PA_ECANCELED.  PA_EINVAL for an unknown ticket or one that has
 * already finished.  Thread-safe. */
pa_status pa_server_cancel(pa_server *srv, uint64_t ticket);
/* Counters of the server.  Thread-safe. */
pa_status pa_server_stats(pa_server *srv, pa_server_counters *out);
/* Stops the worker after its current tick and frees the server; requests
 * not yet polled are dropped.  No other call on srv may run concurrently with
 * or after it. */
void pa_server_destroy(pa_server *srv);

/* ---- diagnostics ------------------------------------------------------ */

/* After pa_kmeans_init with kmeans_frac > 0: copies the K-means state to
 * HOST buffers (any may be NULL): seed [L][K], centroids [K][2] (int32 mm),
 * labels [L*K], iterations.  Blocking. */
pa_status pa_instance_kmeans_state(pa_instance *inst, uint8_t *seed, int32_t *centroids,
                                   int32_t *labels, int32_t *iters);

/* Peak rates of the context's device, measured by probe kernels (the
 * denominators of the LDS-gather rooflines; not part of the method):
 *   lds_b32    bytes per clock per CU of conflict-free ds_read_b32 gathers
 *              (each half-wave reads 32 words in 32 distinct banks)
 *   lds_b128   bytes per clock per CU of ds_read_b128 (consecutive words)
 *   valu_f32   wave64 v_add_f32 instructions per clock per CU
 *   clock_mhz  the shader clock during the probes (cycles over event time)
 *   cus        compute units.
 * Blocking; allocates and frees a few KiB of device memory. */
typedef struct pa_peak_rates {
  double lds_b32, lds_b128, valu_f32, clock_mhz;
  int32_t cus;
} pa_peak_rates;
pa_status pa_device_peaks(pa_context *ctx, pa_peak_rates *out);

const char *pa_status_string(pa_status s);
const char *pa_last_error(void);
/* Library version string. */
const char *pa_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PA_H */
