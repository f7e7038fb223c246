// internal.h -- shared definitions of the gfx950 N-body library (not part of
// the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "nbody.h"

namespace nb {

// Record an error message (thread-local, returned by nbody_last_error) and
// return s.
nbody_status fail(nbody_status s, const char *fmt, ...);
const char *last_error();
// Validate a configuration (records the message on failure).
nbody_status check_config_checked(const nbody_config *c);

#define NB_HIP(call)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return nb::fail(NBODY_E_HIP, "%s: %s", #call, hipGetErrorString(e_));  \
    } while (0)

constexpr int kLevelMax = 40;               // time tick = 2^-40 time units; levels k <= 40
constexpr int64_t kTicksPerUnit = int64_t(1) << kLevelMax;
constexpr int kSchedBlock = 256;            // threads per scheduler block
constexpr int kSchedPerThread = 4;          // particles per scheduler thread
constexpr int kSchedChunk = kSchedBlock * kSchedPerThread;
constexpr int kMixedChunk = 128;            // FP32 partial-sum length in MIXED mode
constexpr int64_t kPartEntries = int64_t(1) << 21;  // j-split partial rows (n_act * n_split), at least
// Rows of j-split partial sums a context keeps (n_act * n_split <= rows): 16 per
// particle, so that an all-active force call can still take 16 splits, at
// least kPartEntries and at most 2^26 (7 GB of doubles).
inline int64_t part_rows_for(int64_t n)
{
    const int64_t r = 16 * n;
    return r < kPartEntries ? kPartEntries : (r > (int64_t(1) << 26) ? (int64_t(1) << 26) : r);
}
constexpr int kMaxComp = 13;                // acc3 + jerk3 + snap3 + crackle3 + pot
constexpr int kMaxNeighbours = 4096;        // neighbour-list capacity per row, at most

// Time-step rule in use (orders 6, 8): 1 = generalised criterion of the
// scheme's order, 2 = its order-4 form.  dt_rule 0 picks the order-4 form
// where the interpolated derivatives of the full-order criterion are
// dominated by rounding noise at short steps: a force with single-precision
// arithmetic, or order 8.
inline int dt_rule_of(const nbody_config &c)
{
    if (c.dt_rule != 0) return c.dt_rule;
    return (c.precision != NBODY_FP64 || c.order == 8) ? 2 : 1;
}

// Post-Newtonian terms between hard particles switched on.
inline bool pn_on(const nbody_config &c) { return c.c_light > 0.0 && c.pn_terms != 0 && c.n_hard >= 2; }

// Components of a force result for a Hermite order: 3 per derivative + pot.
inline int n_comp(int order) { return 3 * (order / 2) + 1; }

// Bytes of one predicted j-particle record.
int record_bytes(int order, int precision);

// Offsets of the sub-buffers inside the caller's workspace (bytes).
struct Layout {
    size_t rec;        // predicted records, n * record_bytes
    size_t part;       // j-split partial sums, part_rows_for(n) * kMaxComp doubles
    size_t force;      // step force outputs, kMaxComp-1 rows of n doubles ([12][n])
    size_t act;        // active indices, n int32
    size_t sched;      // scheduler per-block scratch (min ticks, counts, offsets)
    size_t scal;       // device scalars: t_next, n_act, counters
    size_t energy;     // energy partials
    size_t init;       // init scratch: 4 x [3][n] doubles (a, j, s, c of the two passes)
    size_t irec;       // init records (FP64 order-8 layout), n * 112
    size_t total;
};
Layout make_layout(const nbody_config &c);

// Device scalars at Layout::scal.
struct DevScalars {
    int64_t t_next;
    int64_t n_act;
    unsigned long long underflow;
    unsigned long long nonfinite;
    int64_t pad[4];
};

// Force launch request.
struct ForceArgs {
    const void *rec;        // predicted records
    int64_t n;
    const int32_t *act;
    int64_t n_act;
    double eps2;
    int64_t n_hard;         // already n when eps2 == 0
    double *out[5];         // acc, jrk, snp, crk, pot ([3][n_act] / [n_act]); may be null
    double *part;           // partial-sum scratch
    int64_t part_rows;      // its capacity in rows of kMaxComp doubles (n_act * n_split <= part_rows)
    int ni, block, n_split; // launch shape (n_split 0 = auto)
    int jpath;              // 0 auto, 1 scalar loads, 2 LDS tiles
};

// The launch shape a force call ran with (n_split after the scratch bound).
struct UsedShape {
    int ni, block, n_split, jpath;
};

hipError_t launch_force(int order, int precision, const ForceArgs &a, hipStream_t s, UsedShape *used);

// j-splits and split length (a multiple of the MIXED chunk) of a force launch:
// n_split_req > 0 is taken as given, bounded by the partial-sum scratch
// (n_act * n_split <= part_rows) and by the split length (at least one MIXED
// chunk); 0 chooses from n_act and the shape.
void split_shape(int64_t n, int64_t n_act, int n_split_req, int ni, int block, int jpath, int64_t part_rows,
                 int *n_split, int64_t *j_chunk);

// Fixed-order sum of n_split partial results in a.part into a.out.
// the split reduction for partial sums in part[component][row][split] (wave j-split kernels)
hipError_t launch_split_reduce_sf(int order, const ForceArgs &a, int n_split, hipStream_t s);

// The stored state the predictor reads, and the time it predicts to.
struct PredIn {
    const double *m, *x, *v;
    const double *d[6];      // stored derivatives a^(0..p-3), [3][n] each
    const int64_t *t_tick;
    int64_t t;
};

// The wave j-split force (ForceArgs.jpath 3) with the predictor in its j
// loads: a.rec is not read; the j-particles and the active i-particles are
// predicted from `in` to in.t, exactly as the predictor kernel writes them.
hipError_t launch_force_pred(int order, int precision, const ForceArgs &a, const PredIn &in, hipStream_t s,
                             UsedShape *used);

// Force split by neighbour spheres (order-4 terms) with the neighbour lists.
struct NbArgs {
    const void *rec;        // predicted records (order 4)
    int64_t n;
    const int32_t *act;
    int64_t n_act;
    const double *h2;       // neighbour radius squared per active row
    double eps2;
    int64_t n_hard;         // already n when eps2 == 0
    int max_nb;             // list capacity per row
    double *scratch;        // partial sums and per-split lists
    double *acc_irr, *jrk_irr, *acc_reg, *jrk_reg;   // [3][n_act]
    int32_t *nb_count;      // [n_act]
    int32_t *nb_list;       // [n_act][max_nb] (may be null when max_nb == 0)
};
// Scratch bytes per (split, row); the split count for a scratch of the given
// size (0 when it cannot hold one split); the launch (FP64 or MIXED).
int64_t nb_scratch_per_row(int max_nb);
int nb_split(int64_t n, int64_t n_act, int max_nb, int64_t scratch_bytes, int n_split_req);
hipError_t launch_force_nb(int precision, const NbArgs &a, int n_split, hipStream_t s, int *used_split);

// j-splits that give about 8 waves per SIMD for n_act rows in workgroups of
// `block` lanes with ni rows per lane (the default when n_split is 0).
int auto_split(int64_t n, int64_t n_act, int ni, int block, int64_t part_rows);
// The default split of a j path (jpath 3, the wave j-split kernel, sizes its
// own workgroups: 1, 4 or 16 active rows in 64 lanes).
int auto_split_path(int64_t n, int64_t n_act, int ni, int block, int jpath, int64_t part_rows);

// One row of the force-launch table filled by nbody_autotune.
struct TuneRow {
    int64_t n_act;
    int ni, block, n_split, jpath;
    double ms;
};
constexpr int kTuneRows = 32;

// Pack FP64 order-8 records {x, m, v, a, j} from state arrays (a, j may be null = 0).
hipError_t launch_pack_f64(int64_t n, const double *m, const double *x, const double *v, const double *a,
                           const double *j, void *rec, hipStream_t s);

hipError_t launch_predict(int order, int precision, int64_t n, const nbody_state &st, int64_t t_tick,
                          void *rec, hipStream_t s);

// Corrector for act[0..n_act); when src is non-null the count and the end
// time are read from it on the device (n_act is then an upper bound).
hipError_t launch_correct(const nbody_config &c, const nbody_state &st, int64_t n_act, const int32_t *act,
                          const DevScalars *src, int64_t t_tick_host, const double *const f[4],
                          DevScalars *sc, hipStream_t s);

hipError_t launch_iota(int64_t n, int32_t *a, hipStream_t s);

// Adds the post-Newtonian terms of the hard pairs to acc, jrk and, when not
// null, snp and crk ([3][n_act]) for the rows of act (increasing indices; the hard particles,
// indices below n_hard, come first) predicted to t_tick (t_tick_of null: the
// state as it is).
hipError_t launch_pn(const nbody_config &c, const nbody_state &st, const int64_t *t_tick_of, int64_t t_tick,
                     const int32_t *act, int64_t n_act, double *acc, double *jrk, double *snp, double *crk,
                     hipStream_t s);

hipError_t launch_unpack(int order, int precision, int64_t n, const void *rec, double *xp, double *vp, double *ap,
                         double *jp, hipStream_t s);

// The scheduler's result for the host: written by the scheduler into
// pinned, coherent host memory, the sequence number last, so that the host
// can wait for it by polling instead of a copy and a stream synchronisation.
struct HostScalars {
    int64_t t_next;
    int64_t n_act;
    unsigned long long underflow;
    unsigned long long nonfinite;
    int64_t seq;
    int64_t pad[3];
};

// pub (device address of a HostScalars, may be null) receives the result
// with sequence number seq.
hipError_t launch_schedule(int64_t n, const int64_t *t_tick, const int32_t *level, void *sched_scratch,
                           int32_t *act_out, DevScalars *sc, HostScalars *pub, int64_t seq, hipStream_t s);

hipError_t launch_init_levels(const nbody_config &c, const nbody_state &st, const double *a, const double *j,
                              hipStream_t s);

// Energy partials of n particles whose [3][.] arrays have row stride `stride`.
hipError_t launch_energy(int64_t n, int64_t stride, int64_t n_hard, double eps2, const double *m, const double *x,
                         const double *v, double *partials, int *n_partials, hipStream_t s);

}  // namespace nb

struct nbody_ctx {
    nbody_config cfg;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    nb::Layout lay;
    int device;
    nb::HostScalars *pub_host;        // pinned host copy of the scheduler result (null: copy path)
    nb::HostScalars *pub_dev;         // its device address
    int64_t pub_seq;
    bool predicted;
    bool fuse;                        // predictor folded into the wave j-split force (nbody_set_fusion)
    int ni, block, n_split, jpath;   // launch shape fixed by nbody_set_launch (when manual)
    nb::UsedShape last_shape;         // shape of the last force launch (nbody_get_last_launch)
    bool manual;
    bool tuned;                       // tune[] filled by nbody_autotune
    int n_tune;
    nb::TuneRow tune[nb::kTuneRows];
    nbody_stats stats;
    bool timing;              // record phase events in nbody_step
    hipEvent_t ev[6];         // phase boundaries (created on first enable)
    bool ev_made;
    double phase_ms[5];
    int64_t timed_steps;
};
