/*
 * nbody.h -- C-ABI of the MI355X (gfx950) block-step Hermite N-body hot path.
 *
 * The method (paper: Abstract; Sec. "Codes description"): direct summation of
 * softened Newtonian gravity between all particles, integrated with a
 * 4th-, 6th- or 8th-order Hermite predictor-corrector scheme and individual
 * hierarchical (power-of-two) block time steps, with the force evaluated in
 * mixed FP32/FP64 precision (paper: Fig. 1 and Fig. 5 captions).  The paper
 * names the scheme without formulas; the library follows the standard
 * published ones: the force-derivative recursion, corrector and generalised
 * time-step criterion of Nitadori & Makino (2008), and Aarseth's criterion
 * for order 4.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers owned by the caller, unless the
 *    comment says "host".  The library never allocates device memory: the
 *    caller passes one workspace at create time.
 *  - 3-vector arrays are component-major [3][len]: the x components of all
 *    elements, then the y components, then the z components.
 *  - Time is an integer tick count of 2^-40 time units (int64: times up to
 *    2^23 units).  A particle on level k (k_min <= k <= k_max <= 40) has
 *    dt = 2^-k = 2^(40-k) ticks; its time is always a multiple of its dt.
 *  - Work is enqueued on the HIP stream given to nbody_create.  Entry points
 *    that return host values (n_act, t_next, energies) synchronise that
 *    stream; the others are asynchronous.
 *  - Errors come back as a negative nbody_status; nbody_last_error() gives a
 *    message (thread-local).  Nothing aborts or throws across the ABI.
 *  - Calls on one context are not thread-safe; use one context per thread.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NBODY_OK = 0,
    NBODY_E_INVALID = -1,     /* bad argument: null / misaligned pointer, bad size or option */
    NBODY_E_HIP = -2,         /* a HIP runtime call failed */
    NBODY_E_WORKSPACE = -3,   /* workspace missing, too small or not 256-byte aligned */
    NBODY_E_STATE = -4,       /* call out of order (e.g. force before any predict) */
    NBODY_E_UNSUPPORTED = -5, /* option not supported on this device / build */
    NBODY_E_NONFINITE = -6    /* a corrected value was NaN or infinite */
} nbody_status;

/* Arithmetic of the pairwise force (the corrector, time step, predictor and
 * energy are FP64 in every mode). */
typedef enum {
    NBODY_FP64 = 0,  /* all FP64 */
    NBODY_MIXED = 1, /* double-single (hi + lo float) position and velocity
                        differences, FP32 rsqrt and pairwise arithmetic, FP32
                        partial sums over j-chunks of 128 terms added into FP64
                        accumulators */
    NBODY_DS = 2     /* FP32-only hardware: double-single (hi + lo float)
                        positions and velocities, FP32 arithmetic, compensated
                        (two-sum) double-single accumulation of every term */
} nbody_precision;

typedef struct {
    int32_t order;      /* Hermite order: 4, 6 or 8 */
    int32_t precision;  /* nbody_precision */
    int64_t n;          /* number of particles, 2 <= n <= 2^26 */
    int64_t n_hard;     /* pairs with BOTH indices < n_hard are unsoftened (eps = 0); 0 <= n_hard <= n */
    double eps2;        /* softening length squared for all other pairs, >= 0;
                           eps2 == 0 makes every pair unsoftened */
    double eta;         /* time-step accuracy parameter (inside the square root for order 4,
                           outside the power for orders 6 and 8) */
    double eta_start;   /* initial step: dt0 = eta_start |a| / |jerk| */
    int32_t k_min;      /* largest step 2^-k_min */
    int32_t k_max;      /* smallest step 2^-k_max, k_min <= k_max <= 40 */
    int32_t dt_rule;    /* time-step criterion at orders 6 and 8 (order 4 always uses Aarseth's):
                           1 = generalised Aarseth criterion of the scheme's order,
                           dt = eta (A_1 / A_(p-2))^(1/(p-3)), A_k = sqrt(|a^(k-1)||a^(k+1)|) + |a^(k)|;
                           2 = its order-4 form dt = eta A_1 / A_2 (reads a .. a^(3) only);
                           0 = 2 for MIXED / DS or order 8, else 1.  The full-order form
                           reads derivatives interpolated with weights ~ h^-(p-1); their
                           rounding noise (FP32 force terms, or FP64 at order 8) makes dt_crit
                           collapse to 2^-k_max at short steps. */
    double c_light;     /* speed of light in the model's units (G = 1); > 0 with pn_terms != 0
                           adds post-Newtonian terms between the hard particles (the paper's
                           relativistic corrections for black-hole binaries, Introduction): for
                           every pair of particles with indices < n_hard, the 1PN, 2PN and / or
                           2.5PN two-body relative acceleration in harmonic coordinates,
                           -(M/r^2)[A n + B v] with the A, B terms of Blanchet's review
                           (Living Rev. Relativ. 17, 2), body 1 taking m2/M of it and body 2
                           -m1/M, and its jerk, snap and crackle along the pair's Newtonian
                           two-body motion (as many as the order uses); added by nbody_init,
                           nbody_step and nbody_run to the forces of active hard particles,
                           from their positions and velocities predicted in FP64.
                           n_hard <= 1024 (the pairs cost n_hard^2); not in the batched form
                           (NBODY_E_UNSUPPORTED).  0 = off. */
    int32_t pn_terms;   /* a sum of 1 = 1PN, 2 = 2PN, 4 = 2.5PN (radiation reaction); 0 = off */
} nbody_config;

/* Particle state, DEVICE pointers, caller-owned, 8-byte aligned.
 * m[n]; x, v [3][n]; d[k] = k-th derivative of the acceleration a^(k), [3][n],
 * for k = 0 .. order-3 (a, jerk; + snap, crackle for order >= 6; + a^(4), a^(5)
 * for order 8), unused entries NULL; t_tick[n] particle times; level[n]. */
typedef struct {
    double *m;
    double *x;
    double *v;
    double *d[6];
    int64_t *t_tick;
    int32_t *level;
} nbody_state;

/* Counters kept by a context since creation (host copy). */
typedef struct {
    int64_t steps;          /* block steps taken by nbody_step */
    int64_t sum_n_act;      /* sum of n_act over those steps */
    double interactions;    /* sum of n_act * n over force evaluations */
    int64_t dt_underflow;   /* corrected particles whose dt_crit was below 2^-k_max */
    int64_t nonfinite;      /* corrected particles with a non-finite value */
} nbody_stats;

typedef struct nbody_ctx nbody_ctx;

/* Bytes of device workspace a context for this configuration needs. */
nbody_status nbody_workspace_size(const nbody_config *cfg, size_t *bytes /* host */);

/* Create a context.  workspace: DEVICE memory of at least
 * nbody_workspace_size() bytes, 256-byte aligned, owned by the caller and kept
 * alive until nbody_destroy.  stream: a hipStream_t (NULL = default stream).
 * *out (host) receives the context.  The context allocates no device memory;
 * it takes 64 bytes of pinned host memory (hipHostMalloc, coherent), into
 * which the block-step scheduler writes its result so that nbody_step and
 * nbody_run wait for it by polling (if that allocation fails they copy the
 * result and synchronise the stream instead).  nbody_destroy synchronises
 * the stream and frees it. */
nbody_status nbody_create(const nbody_config *cfg, void *workspace, size_t bytes, void *stream,
                          nbody_ctx **out);
nbody_status nbody_destroy(nbody_ctx *ctx);

/* Initial forces and steps at t = 0 (all particles): acceleration and jerk
 * from (x, v); snap and crackle from a second FP64 pass that uses them; for
 * order 8, a^(4) = a^(5) = 0.  Sets t_tick = 0 and each level from
 * dt0 = eta_start |a|/|jerk| (largest 2^-k <= dt0, clamped to [k_min, k_max]).
 * Reads m, x, v; writes d[], t_tick, level. */
nbody_status nbody_init(nbody_ctx *ctx, nbody_state *state);

/* Predict every particle to time t_tick (Taylor series of its stored
 * derivatives about its own time: x to dt^(p-1), v to dt^(p-2), a to dt^(p-3),
 * jerk to dt^(p-4)) into the context's j-particle records, which
 * nbody_force_block reads.  t_tick must be >= every particle's time. */
nbody_status nbody_predict(nbody_ctx *ctx, const nbody_state *state, int64_t t_tick);

/* Force and derivatives on the active particles act_idx[0 .. n_act) from
 * the predicted records of the last nbody_predict: for each active i, the sum
 * over all j != i of the softened pairwise acceleration, jerk, snap (order
 * >= 6), crackle (order 8) and potential -m_j / sqrt(r^2 + eps_ij^2).
 * act_idx: int32 indices in [0, n), no duplicates (order free).
 * Outputs [3][n_act] (pot: [n_act]) FP64, row q belongs to act_idx[q].
 * snp / crk may be NULL when the order does not define them; pot may be
 * NULL.  The j-sum order is fixed, so reruns are bitwise identical.
 * Newtonian force only: the post-Newtonian terms of a context with c_light
 * set are added by nbody_init, nbody_step and nbody_run, not here. */
nbody_status nbody_force_block(nbody_ctx *ctx, int64_t n_act, const int32_t *act_idx, double *acc,
                               double *jrk, double *snp, double *crk, double *pot);

/* nbody_predict followed by nbody_force_block on act_idx, with the same
 * arguments, outputs and results bit for bit.  When the launch shape for n_act
 * is the wave j-split kernel (jpath 3; see nbody_set_launch) and fusion is on
 * (nbody_set_fusion; the default), one kernel does both: each workgroup
 * predicts the j-particles of its split as it walks them (the paper's block
 * step predicts every particle to the block time before the force, Sec.
 * "Codes description"), so the stored state is read once and no record is
 * written.  The records are then stale: nbody_force_block, nbody_get_predicted
 * and nbody_autotune need a new nbody_predict.  nbody_step and nbody_run take
 * the same route. */
nbody_status nbody_predict_force(nbody_ctx *ctx, const nbody_state *state, int64_t t_tick, int64_t n_act,
                                 const int32_t *act_idx, double *acc, double *jrk, double *snp, double *crk,
                                 double *pot);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the work of
 * nbody_predict_force with fusion on and the wave j-split kernel (jpath 3,
 * default split), without a context or workspace.  cfg: as for
 * nbody_create (host); state (host struct of DEVICE pointers): m, x, v, d[],
 * t_tick are read, level is not; t_tick: the time every particle is
 * predicted to (>= each particle's time); act_idx, outputs, results: as
 * nbody_predict_force, bit for bit equal to it when that call runs the same
 * kernel and split (a context set to nbody_set_launch(ctx, 1, 64, 0, 3)).
 * stream: a hipStream_t of the current device (NULL = default stream); the
 * call is asynchronous on it.  1 <= n_act <= 1024 (0 does nothing), else
 * NBODY_E_INVALID: the j-split partial sums live in a static device array of
 * 65536 rows x 13 doubles (6.8 MB per GPU, held until the process ends),
 * whose device address is looked up once per device.  The call allocates
 * nothing.  Every call on one GPU shares that array: calls that overlap on
 * one GPU (other streams, other host threads) race.  Each call writes every
 * partial sum it reads, so nothing needs clearing between calls. */
nbody_status nbody_predict_force_noalloc(const nbody_config *cfg, const nbody_state *state, int64_t t_tick,
                                         int64_t n_act, const int32_t *act_idx, double *acc, double *jrk,
                                         double *snp, double *crk, double *pot, void *stream);

/* enable = 1 (default): nbody_predict_force, nbody_step and nbody_run fold
 * the predictor into the wave j-split force kernel; 0: they always run the
 * predictor kernel and then the force kernel.  Results are the same. */
nbody_status nbody_set_fusion(nbody_ctx *ctx, int32_t enable);

/* Force on the active particles split by neighbour spheres, with the
 * neighbour lists: the regular/irregular split of the Ahmad & Cohen (1973)
 * scheme used by the paper's second code, NBODY6++GPU (Sec. "Results", the
 * laohu tests), whose GPU part is exactly this: the force from the distant
 * particles and the neighbour lists.  Order-4 contexts in FP64 or MIXED
 * precision; reads the predicted records of the last nbody_predict.
 * For active row q (particle i = act_idx[q]) with neighbour radius squared
 * h2[q] (host-side meaning: h_i^2; NaN or <= 0 gives no neighbours), particle
 * j != i is a neighbour when its unsoftened squared distance |x_j - x_i|^2,
 * evaluated in the kernel's precision (FP64, or FP32 from the double-single
 * differences in MIXED), is below h2[q].  The softened acceleration and jerk
 * of every pair (as in nbody_force_block) are summed over the other particles
 * into acc_reg, jrk_reg and over the neighbours into acc_irr, jrk_irr.
 * Outputs (DEVICE): acc_*, jrk_* [3][n_act] FP64; nb_count[n_act] int32 =
 * number of neighbours; nb_list[n_act][max_nb] int32 = the first
 * min(nb_count[q], max_nb) neighbours in increasing index order (entries past
 * them are not written).  The irregular part is summed over the list, so a
 * row whose list was cut (nb_count[q] > max_nb) gets NaN in acc_irr and
 * jrk_irr; its regular part is complete.  h2 (DEVICE) [n_act] FP64.  max_nb
 * in [0, 4096]; nb_list may be NULL when max_nb is 0 (regular part and counts
 * only).  Uses the context's force scratch of R = max(2^21, min(16 n, 2^26))
 * rows: n_act * (13 + max_nb) must stay below 26 R, else NBODY_E_INVALID
 * (call in pieces).
 * The sum orders are fixed, so reruns are bitwise identical. */
nbody_status nbody_force_block_nb(nbody_ctx *ctx, int64_t n_act, const int32_t *act_idx, const double *h2,
                                  int32_t max_nb, double *acc_irr, double *jrk_irr, double *acc_reg,
                                  double *jrk_reg, int32_t *nb_count, int32_t *nb_list);

/* Hermite corrector, interpolated higher derivatives and new time step for
 * the active particles, whose next time must be t_tick: x, v and d[] are
 * overwritten with their values at t_tick, t_tick[i] = t_tick, level[i] the
 * new level.  acc .. crk are the force outputs at t_tick ([3][n_act] as from
 * nbody_force_block; only the first order/2 are read). */
nbody_status nbody_correct(nbody_ctx *ctx, nbody_state *state, int64_t n_act, const int32_t *act_idx,
                           int64_t t_tick, const double *acc, const double *jrk, const double *snp,
                           const double *crk);

/* Block-step selection: t_next = min_i (t_i + dt_i); act_idx_out (DEVICE,
 * room for n) receives the active set {i : t_i + dt_i == t_next} in
 * increasing order.  *t_next_out, *n_act_out (host) receive the results. */
nbody_status nbody_schedule(nbody_ctx *ctx, const nbody_state *state, int32_t *act_idx_out,
                            int64_t *t_next_out, int64_t *n_act_out);

/* One whole block step: schedule, predict all, force on the active set,
 * correct.  *t_tick_out / *n_act_out (host, may be NULL) receive the new time
 * and the number of particles advanced.  Returns NBODY_E_NONFINITE when a
 * corrected value became NaN or infinite. */
nbody_status nbody_step(nbody_ctx *ctx, nbody_state *state, int64_t *t_tick_out, int64_t *n_act_out);

/* Block steps (as nbody_step) until the next block time would exceed
 * t_end_tick, or max_steps steps: *steps_out (host) = steps taken,
 * *t_tick_out (host) = time of the last step (0 if none); both may be NULL.
 * The corrector's counters are read with the next step's scheduler result,
 * so a run costs one host round trip per step.  Returns NBODY_E_NONFINITE
 * (after the step that produced it, or the one after) when a corrected value
 * became NaN or infinite. */
nbody_status nbody_run(nbody_ctx *ctx, nbody_state *state, int64_t t_end_tick, int64_t max_steps,
                       int64_t *steps_out, int64_t *t_tick_out);

/* FP64 energy of the state (meaningful when all particles share one time):
 * *ekin = sum m v^2 / 2, *epot = - sum_{i<j} m_i m_j / sqrt(r^2 + eps_ij^2).
 * Host outputs; fixed summation order. */
nbody_status nbody_energy(nbody_ctx *ctx, const nbody_state *state, double *ekin, double *epot);

/* Copy the predicted records of the last nbody_predict out as FP64 arrays
 * [3][n] (DEVICE pointers): position, velocity, and for order >= 6 the
 * acceleration, order 8 the jerk (ap / jp may be NULL).  In MIXED and DS mode
 * these are the values the force kernel sees (FP32 acceleration / jerk,
 * double-single hi + lo sums). */
nbody_status nbody_get_predicted(nbody_ctx *ctx, double *xp, double *vp, double *ap, double *jp);

/* Counters since creation (host output). */
nbody_status nbody_get_stats(nbody_ctx *ctx, nbody_stats *out);

/* Launch shape of the force kernel: ni = active particles per lane (1 or 2),
 * block = threads per workgroup (64, 128 or 256), n_split = j-range splits
 * (0 = chosen per call from n_act), jpath = how j records reach the lanes
 * (0 = default for the precision, 1 = wave-uniform scalar loads, 2 = LDS
 * tiles, 3 = wave j-split for small active sets: 1, 4 or 16 active rows per
 * 64-lane workgroup, each row's j range spread over 64, 16 or 4 lanes and
 * folded across them; ni and block are ignored).  A shape set here is used
 * for every later force call (it replaces an autotuned table).  Without
 * either, a call uses the wave j-split kernel for n_act <= 32, else ni = 1,
 * the narrowest workgroup of 64, 128 or 256 lanes that holds n_act, and the
 * default split.  A call lowers n_split where it exceeds what the partial-sum
 * scratch holds (n_act * n_split <= max(2^21, min(16 n, 2^26))) or gives
 * splits shorter than 128 j; nbody_get_last_launch tells the shape used.
 * Results do not depend on ni, block or jpath; they depend on n_split only
 * through the FP64 summation order (and, in MIXED mode, where the FP32 chunks
 * start). */
nbody_status nbody_set_launch(nbody_ctx *ctx, int32_t ni, int32_t block, int32_t n_split, int32_t jpath);

/* Autotuner of the force launch (i-tile, j-tile path and j-split per active
 * size): for n_act = 1, 2, 4, ... up to min(max_n_act, n) (at most 31 sizes,
 * and min(max_n_act, n) itself), times `reps` launches of every shape
 * ni in {1, 2} x block in {64, 128, 256} x jpath in {1, 2} (and jpath 3 for
 * n_act <= 64) x n_split in {s/2, s, 2s} (s = the default split) with HIP
 * events, on the records of the
 * last nbody_predict and the first n_act particles, and keeps the fastest.
 * Later force calls use the row of the smallest tuned n_act >= their n_act
 * (the largest row above the table).  Overwrites the context's force scratch;
 * leaves the state and the counters alone.  Needs a prior nbody_predict. */
nbody_status nbody_autotune(nbody_ctx *ctx, int64_t max_n_act, int32_t reps);

/* The tuned table (HOST arrays of max_rows): n_act[k], shape[4k .. 4k+3] =
 * ni, block, n_split, jpath, ms[k] = time per launch; each may be NULL.
 * *rows = rows in the table (0 when not tuned). */
nbody_status nbody_get_tuning(nbody_ctx *ctx, int32_t max_rows, int64_t *n_act, int32_t *shape, double *ms,
                              int32_t *rows);

/* The launch shape of the last force kernel this context ran (any entry
 * point that computes forces; HOST out[4]): ni, block, n_split (as launched,
 * after the bounds of nbody_set_launch), jpath (1, 2 or 3).  Zeros before the
 * first force call. */
nbody_status nbody_get_last_launch(nbody_ctx *ctx, int32_t out[4]);

/* Phase timers of nbody_step, measured with HIP events on the context's
 * stream.  nbody_set_timing(ctx, 1) creates the events and starts
 * accumulating; 0 stops.  nbody_get_timers writes, in milliseconds summed over
 * the timed steps: [0] scheduler, [1] host round trip between scheduling and
 * prediction, [2] predictor, [3] force (pairwise kernel and split reduction;
 * with the predictor inside, see nbody_predict_force, [2] is then empty),
 * [4] corrector + time step; *steps (host) = number of timed steps. */
nbody_status nbody_set_timing(nbody_ctx *ctx, int32_t enable);
nbody_status nbody_get_timers(nbody_ctx *ctx, double ms[5] /* host */, int64_t *steps /* host */);

/* ------------------------------------------------------------------------
 * Batched form: many independent clusters (separate N-body systems that share
 * one configuration) advanced together.  Particles of cluster c are
 * [off[c], off[c+1]) of one concatenated state (all arrays [3][n] with
 * n = off[n_clusters]); pairs never cross clusters; n_hard counts from the
 * first particle of each cluster.  Each batched step advances every cluster
 * by one block step of its own (its own t_next and active set), with the
 * same arithmetic as nbody_step.  The launch sequence of a step does not
 * depend on the data (fixed grids; a persistent force kernel takes
 * (cluster, i-tile, j-split) work items from per-XCD device queues, largest
 * clusters first), so it can be captured once in a HIP graph and replayed.
 * ------------------------------------------------------------------------ */
typedef struct nbody_batch nbody_batch;

/* Workspace bytes for a batch.  cfg->n = off[n_clusters]; off: HOST array of
 * n_clusters + 1 offsets, off[0] = 0, every cluster at least 2 particles,
 * 1 <= n_clusters <= 65535, cfg->n_hard <= the smallest cluster. */
nbody_status nbody_batch_workspace_size(const nbody_config *cfg, int32_t n_clusters, const int64_t *off /* host */,
                                        size_t *bytes /* host */);

/* Create a batch context (same workspace and stream rules as nbody_create;
 * graph capture needs a stream other than the default stream). */
nbody_status nbody_batch_create(const nbody_config *cfg, int32_t n_clusters, const int64_t *off /* host */,
                                void *workspace, size_t bytes, void *stream, nbody_batch **out);
nbody_status nbody_batch_destroy(nbody_batch *b);

/* nbody_init for every cluster (each at t = 0, forces from its own particles). */
nbody_status nbody_batch_init(nbody_batch *b, nbody_state *state);

/* Clusters whose next block time would exceed t_end_tick rest (take no step);
 * default: no limit. */
nbody_status nbody_batch_set_end(nbody_batch *b, int64_t t_end_tick);

/* Enqueue k batched steps directly (asynchronous; no host round trip). */
nbody_status nbody_batch_step(nbody_batch *b, nbody_state *state, int64_t k);

/* Capture one batched step on `state` (its pointers are baked in) into a HIP
 * graph; nbody_batch_replay launches it k times.  A new capture replaces the
 * old one. */
nbody_status nbody_batch_capture(nbody_batch *b, nbody_state *state);
nbody_status nbody_batch_replay(nbody_batch *b, int64_t k);

/* Synchronising poll: *n_live (host) = clusters that took a step in the last
 * batched step (0 once every cluster rests); t_cur (host, n_clusters
 * entries, may be NULL) = each cluster's time (its last completed step). */
nbody_status nbody_batch_poll(nbody_batch *b, int64_t *n_live, int64_t *t_cur);

/* The last batched step's work (synchronising): aoff (HOST, n_clusters + 1) =
 * offsets of the clusters' active lists in the concatenated list; act (DEVICE,
 * room for n, may be NULL) = the list, increasing within each cluster;
 * forces (DEVICE, may be NULL) = [order/2][3][n_act] FP64 force derivatives
 * (acc, jerk, snap, crackle) at the step's end, row q for act[q]. */
nbody_status nbody_batch_last_step(nbody_batch *b, int64_t *aoff, int32_t *act, double *forces);

/* Per-cluster FP64 energies (HOST arrays of n_clusters), as nbody_energy. */
nbody_status nbody_batch_energy(nbody_batch *b, const nbody_state *state, double *ekin, double *epot);

/* Counters over all clusters since creation (steps = batched steps). */
nbody_status nbody_batch_get_stats(nbody_batch *b, nbody_stats *out);

/* Persistent force launch: force_grid workgroups (0 = as many as fit on the
 * device at once), items_per_wg work items aimed for per workgroup (1..32,
 * 0 = 8: each step's padded work is cut into about force_grid * items_per_wg
 * items of equal cost, at most 2^22 / i_tile, by splitting each cluster's
 * j-range into pieces of at least 128) and i_tile active rows per work item
 * (64, 128 or 256, 0 = 64).  Applies to later steps and captures (a captured graph keeps
 * the shape it was captured with).  Results depend on the shape only through
 * the FP64 summation order of the split partials (and, in MIXED mode, where
 * the FP32 chunks start). */
nbody_status nbody_batch_set_launch(nbody_batch *b, int32_t force_grid, int32_t items_per_wg, int32_t i_tile);

/* The shape in use (HOST out[3]): force_grid, items_per_wg, i_tile. */
nbody_status nbody_batch_get_launch(nbody_batch *b, int32_t out[3]);

/* Autotuner over `steps` batched steps: before each step, for every i_tile
 * in {64, 128, 256} and items_per_wg in {2, 4, 8, 16, 32}, plans that step
 * for the shape and times its force phase (persistent force kernel and split
 * reduction) once after one untimed pass, with HIP events; then takes the
 * step (real: the clusters advance by `steps` batched steps, with the shape
 * in use before the call).  Every shape is timed on the same steps; keeps the
 * shape with the least total time.  Drops a captured graph (capture again). */
nbody_status nbody_batch_autotune(nbody_batch *b, nbody_state *state, int32_t steps);

/* Message for the last non-OK status returned on this thread. */
const char *nbody_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
