// api.cpp -- the C-ABI of the library: argument checks, workspace layout,
// and the order of kernel launches for each entry point.  All device memory
// comes from the caller (one workspace per context); the library never
// allocates on the device.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

namespace {

using nb::fail;

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

nbody_status check_config(const nbody_config *c)
{
    if (!c) return fail(NBODY_E_INVALID, "config is NULL");
    if (c->order != 4 && c->order != 6 && c->order != 8)
        return fail(NBODY_E_INVALID, "order must be 4, 6 or 8 (got %d)", c->order);
    if (c->precision < NBODY_FP64 || c->precision > NBODY_DS)
        return fail(NBODY_E_INVALID, "precision must be 0 (FP64), 1 (MIXED) or 2 (DS) (got %d)", c->precision);
    if (c->n < 2 || c->n > (int64_t(1) << 26)) return fail(NBODY_E_INVALID, "n must be in [2, 2^26] (got %lld)", (long long)c->n);
    if (c->n_hard < 0 || c->n_hard > c->n) return fail(NBODY_E_INVALID, "n_hard must be in [0, n]");
    if (!(c->eps2 >= 0.0) || !std::isfinite(c->eps2)) return fail(NBODY_E_INVALID, "eps2 must be finite and >= 0");
    if (!(c->eta > 0.0) || !std::isfinite(c->eta)) return fail(NBODY_E_INVALID, "eta must be > 0");
    if (!(c->eta_start > 0.0) || !std::isfinite(c->eta_start)) return fail(NBODY_E_INVALID, "eta_start must be > 0");
    if (c->dt_rule < 0 || c->dt_rule > 2) return fail(NBODY_E_INVALID, "dt_rule must be 0, 1 or 2 (got %d)", c->dt_rule);
    if (c->k_min < 0 || c->k_min > c->k_max || c->k_max > nb::kLevelMax)
        return fail(NBODY_E_INVALID, "need 0 <= k_min <= k_max <= %d (got %d, %d)", nb::kLevelMax, c->k_min, c->k_max);
    if (!(c->c_light >= 0.0) || !std::isfinite(c->c_light)) return fail(NBODY_E_INVALID, "c_light must be finite and >= 0");
    if (c->pn_terms < 0 || c->pn_terms > 7)
        return fail(NBODY_E_INVALID, "pn_terms must be a sum of 1 (1PN), 2 (2PN) and 4 (2.5PN) (got %d)",
                    c->pn_terms);
    if (nb::pn_on(*c) && c->n_hard > 1024)
        return fail(NBODY_E_INVALID, "post-Newtonian terms take at most 1024 hard particles (got %lld)",
                    (long long)c->n_hard);
    return NBODY_OK;
}

nbody_status check_state(const nbody_ctx *ctx, const nbody_state *st)
{
    if (!st) return fail(NBODY_E_INVALID, "state is NULL");
    const void *ptrs[] = {st->m, st->x, st->v, st->t_tick, st->level};
    for (const void *p : ptrs)
        if (!p || !aligned8(p)) return fail(NBODY_E_INVALID, "state pointers must be non-NULL and 8-byte aligned");
    for (int k = 0; k <= ctx->cfg.order - 3; ++k)
        if (!st->d[k] || !aligned8(st->d[k]))
            return fail(NBODY_E_INVALID, "state d[%d] must be non-NULL and 8-byte aligned for order %d", k, ctx->cfg.order);
    return NBODY_OK;
}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

template <class T> T *ws_at(nbody_ctx *ctx, size_t off) { return reinterpret_cast<T *>(ctx->ws + off); }

nb::DevScalars *scalars(nbody_ctx *ctx) { return ws_at<nb::DevScalars>(ctx, ctx->lay.scal); }

int64_t hard_count(const nbody_config &c) { return c.eps2 == 0.0 ? c.n : c.n_hard; }

// Force arguments and the launch shape for n_act active particles: the shape
// set by nbody_set_launch, else the tuned table's, else the default.
nb::ForceArgs force_args(nbody_ctx *ctx, const void *rec, int64_t n_act, const int32_t *act, double *acc,
                         double *jrk, double *snp, double *crk, double *pot)
{
    nb::ForceArgs a{};
    a.rec = rec;
    a.n = ctx->cfg.n;
    a.act = act;
    a.n_act = n_act;
    a.eps2 = ctx->cfg.eps2;
    a.n_hard = hard_count(ctx->cfg);
    a.out[0] = acc;
    a.out[1] = jrk;
    a.out[2] = snp;
    a.out[3] = crk;
    a.out[4] = pot;
    a.part = ws_at<double>(ctx, ctx->lay.part);
    a.part_rows = nb::part_rows_for(ctx->cfg.n);
    if (ctx->manual) {
        a.ni = ctx->ni;
        a.block = ctx->block;
        a.n_split = ctx->n_split;
        a.jpath = ctx->jpath;
    } else if (ctx->tuned) {
        // the smallest tuned bucket that holds n_act (else the largest)
        int r = 0;
        while (r + 1 < ctx->n_tune && ctx->tune[r].n_act < n_act) ++r;
        a.ni = ctx->tune[r].ni;
        a.block = ctx->tune[r].block;
        a.n_split = ctx->tune[r].n_split;
        a.jpath = ctx->tune[r].jpath;
    } else {
        // untuned default: the wave j-split kernel for active sets of up to 32
        // (the autotuner's choice there on MI355X in every precision), else
        // workgroups no wider than the active set needs
        a.ni = 1;
        a.block = n_act <= 64 ? 64 : (n_act <= 128 ? 128 : 256);
        a.n_split = 0;
        a.jpath = n_act <= 32 ? 3 : 0;
    }
    return a;
}

nbody_status run_force(nbody_ctx *ctx, int order, int precision, const void *rec, int64_t n_act,
                       const int32_t *act, double *acc, double *jrk, double *snp, double *crk, double *pot)
{
    const nb::ForceArgs a = force_args(ctx, rec, n_act, act, acc, jrk, snp, crk, pot);
    NB_HIP(nb::launch_force(order, precision, a, ctx->stream, &ctx->last_shape));
    ctx->stats.interactions += double(n_act) * double(ctx->cfg.n);
    return NBODY_OK;
}

// Prediction of every particle to t followed by the force on the active set.
// When the launch shape is the wave j-split kernel and fusion is on, one
// kernel does both (the records are then not written); otherwise the
// predictor kernel writes the records and the force kernel reads them.
// *fused (may be null) tells which.
nbody_status run_predict_force(nbody_ctx *ctx, const nbody_state *st, int64_t t, int64_t n_act, const int32_t *act,
                               double *acc, double *jrk, double *snp, double *crk, double *pot, bool *fused)
{
    const nbody_config &c = ctx->cfg;
    const nb::ForceArgs a = force_args(ctx, ctx->ws + ctx->lay.rec, n_act, act, acc, jrk, snp, crk, pot);
    const bool f = ctx->fuse && a.jpath == 3;
    if (fused) *fused = f;
    if (f) {
        nb::PredIn in{};
        in.m = st->m;
        in.x = st->x;
        in.v = st->v;
        for (int k = 0; k < 6; ++k) in.d[k] = k <= c.order - 3 ? st->d[k] : nullptr;
        in.t_tick = st->t_tick;
        in.t = t;
        ctx->predicted = false;   // the records are stale from here on
        NB_HIP(nb::launch_force_pred(c.order, c.precision, a, in, ctx->stream, &ctx->last_shape));
    } else {
        NB_HIP(nb::launch_predict(c.order, c.precision, c.n, *st, t, ctx->ws + ctx->lay.rec, ctx->stream));
        ctx->predicted = true;
        NB_HIP(nb::launch_force(c.order, c.precision, a, ctx->stream, &ctx->last_shape));
    }
    ctx->stats.interactions += double(n_act) * double(c.n);
    return NBODY_OK;
}

nbody_status read_scalars(nbody_ctx *ctx, nb::DevScalars *h)
{
    NB_HIP(hipMemcpyAsync(h, scalars(ctx), sizeof(*h), hipMemcpyDeviceToHost, ctx->stream));
    NB_HIP(hipStreamSynchronize(ctx->stream));
    return NBODY_OK;
}

// The scheduler result with sequence number seq, read from the pinned host
// copy as soon as the scheduler has written it (the later kernels of the
// step may still run).  The wait polls host memory and, every few thousand
// polls, the stream: a stream error is returned, and a stream that finished
// without the result (which should not happen) falls back to the copy.
nbody_status read_published(nbody_ctx *ctx, int64_t seq, nb::DevScalars *h)
{
    if (!ctx->pub_host) return read_scalars(ctx, h);
    const nb::HostScalars *p = ctx->pub_host;
    unsigned spins = 0;
    while (__atomic_load_n(&p->seq, __ATOMIC_ACQUIRE) != seq) {
        if ((++spins & 4095u) == 0) {
            const hipError_t e = hipStreamQuery(ctx->stream);
            if (e == hipSuccess) {
                if (__atomic_load_n(&p->seq, __ATOMIC_ACQUIRE) == seq) break;
                return read_scalars(ctx, h);
            }
            if (e != hipErrorNotReady) return fail(NBODY_E_HIP, "scheduler: %s", hipGetErrorString(e));
        }
    }
    h->t_next = p->t_next;
    h->n_act = p->n_act;
    h->underflow = p->underflow;
    h->nonfinite = p->nonfinite;
    return NBODY_OK;
}

}  // namespace

namespace nb {

nbody_status check_config_checked(const nbody_config *c) { return ::check_config(c); }

namespace {
thread_local char g_err[512] = "";
}

nbody_status fail(nbody_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

const char *last_error() { return g_err; }

Layout make_layout(const nbody_config &c)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += up256(bytes);
        return at;
    };
    const size_t n = size_t(c.n);
    const size_t nb = (n + kSchedChunk - 1) / kSchedChunk;
    L.rec = take(n * size_t(record_bytes(c.order, c.precision)));
    L.part = take(size_t(part_rows_for(c.n)) * kMaxComp * sizeof(double));
    L.force = take(12 * n * sizeof(double));
    L.act = take(n * sizeof(int32_t));
    L.sched = take(nb * (2 * sizeof(int64_t) + sizeof(int32_t)));
    L.scal = take(sizeof(DevScalars));
    L.energy = take(2 * ((n + 255) / 256) * sizeof(double));
    L.init = 0;
    L.irec = take(n * 112);
    L.total = off;
    return L;
}

}  // namespace nb

extern "C" {

const char *nbody_last_error(void) { return nb::last_error(); }

nbody_status nbody_workspace_size(const nbody_config *cfg, size_t *bytes)
{
    nbody_status s = check_config(cfg);
    if (s != NBODY_OK) return s;
    if (!bytes) return fail(NBODY_E_INVALID, "bytes is NULL");
    *bytes = nb::make_layout(*cfg).total;
    return NBODY_OK;
}

nbody_status nbody_create(const nbody_config *cfg, void *workspace, size_t bytes, void *stream, nbody_ctx **out)
{
    nbody_status s = check_config(cfg);
    if (s != NBODY_OK) return s;
    if (!out) return fail(NBODY_E_INVALID, "out is NULL");
    const nb::Layout L = nb::make_layout(*cfg);
    if (!workspace) return fail(NBODY_E_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) & 255u) return fail(NBODY_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < L.total) return fail(NBODY_E_WORKSPACE, "workspace too small: %zu < %zu bytes", bytes, L.total);
    nbody_ctx *ctx = new (std::nothrow) nbody_ctx();
    if (!ctx) return fail(NBODY_E_INVALID, "out of host memory");
    ctx->cfg = *cfg;
    ctx->stream = static_cast<hipStream_t>(stream);
    ctx->ws = static_cast<char *>(workspace);
    ctx->ws_bytes = bytes;
    ctx->lay = L;
    ctx->predicted = false;
    ctx->fuse = true;
    ctx->ni = 1;
    ctx->block = 256;
    ctx->n_split = 0;
    ctx->jpath = 0;
    ctx->manual = false;
    ctx->tuned = false;
    ctx->n_tune = 0;
    ctx->last_shape = nb::UsedShape{0, 0, 0, 0};
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    hipError_t e = hipGetDevice(&ctx->device);
    if (e == hipSuccess) e = hipMemsetAsync(scalars(ctx), 0, sizeof(nb::DevScalars), ctx->stream);
    // 64 bytes of pinned, coherent host memory for the scheduler result
    // (without it the steps copy the result and synchronise instead)
    if (e == hipSuccess &&
        hipHostMalloc(reinterpret_cast<void **>(&ctx->pub_host), sizeof(nb::HostScalars), hipHostMallocCoherent) ==
            hipSuccess) {
        ctx->pub_host->seq = 0;
        if (hipHostGetDevicePointer(reinterpret_cast<void **>(&ctx->pub_dev), ctx->pub_host, 0) != hipSuccess) {
            (void)hipHostFree(ctx->pub_host);
            ctx->pub_host = nullptr;
            ctx->pub_dev = nullptr;
        }
    } else {
        ctx->pub_host = nullptr;
        (void)hipGetLastError();
    }
    ctx->pub_seq = 0;
    if (e != hipSuccess) {
        delete ctx;
        return fail(NBODY_E_HIP, "nbody_create: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return NBODY_OK;
}

nbody_status nbody_destroy(nbody_ctx *ctx)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    if (ctx->ev_made)
        for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
    if (ctx->pub_host) {
        (void)hipStreamSynchronize(ctx->stream);   // no scheduler kernel may still write it
        (void)hipHostFree(ctx->pub_host);
    }
    delete ctx;
    return NBODY_OK;
}

nbody_status nbody_set_timing(nbody_ctx *ctx, int32_t enable)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    if (enable && !ctx->ev_made) {
        for (hipEvent_t &e : ctx->ev) NB_HIP(hipEventCreate(&e));
        ctx->ev_made = true;
    }
    ctx->timing = enable != 0;
    return NBODY_OK;
}

nbody_status nbody_get_timers(nbody_ctx *ctx, double ms[5], int64_t *steps)
{
    if (!ctx || !ms) return fail(NBODY_E_INVALID, "ctx and ms are required");
    for (int k = 0; k < 5; ++k) ms[k] = ctx->phase_ms[k];
    if (steps) *steps = ctx->timed_steps;
    return NBODY_OK;
}

nbody_status nbody_set_launch(nbody_ctx *ctx, int32_t ni, int32_t block, int32_t n_split, int32_t jpath)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    if (jpath < 0 || jpath > 3)
        return fail(NBODY_E_INVALID, "jpath must be 0 (auto), 1 (scalar), 2 (LDS) or 3 (wave j-split)");
    if (ni != 1 && ni != 2) return fail(NBODY_E_INVALID, "ni must be 1 or 2");
    if (block != 64 && block != 128 && block != 256) return fail(NBODY_E_INVALID, "block must be 64, 128 or 256");
    if (n_split < 0 || n_split > 65535) return fail(NBODY_E_INVALID, "n_split must be in [0, 65535]");
    ctx->ni = ni;
    ctx->block = block;
    ctx->n_split = n_split;
    ctx->jpath = jpath;
    ctx->manual = true;
    return NBODY_OK;
}

nbody_status nbody_autotune(nbody_ctx *ctx, int64_t max_n_act, int32_t reps)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    if (!ctx->predicted) return fail(NBODY_E_STATE, "nbody_autotune before nbody_predict");
    if (max_n_act < 1) return fail(NBODY_E_INVALID, "max_n_act must be >= 1");
    if (reps < 1 || reps > 1000) return fail(NBODY_E_INVALID, "reps must be in [1, 1000]");
    const nbody_config &c = ctx->cfg;
    const int64_t top = max_n_act < c.n ? max_n_act : c.n;
    std::vector<int64_t> sizes;
    for (int64_t k = 1; k <= top && int(sizes.size()) < nb::kTuneRows - 1; k *= 2) sizes.push_back(k);
    if (sizes.back() != top) sizes.push_back(top);
    int32_t *all = ws_at<int32_t>(ctx, ctx->lay.act);
    NB_HIP(nb::launch_iota(c.n, all, ctx->stream));
    double *F = ws_at<double>(ctx, ctx->lay.force);
    const int64_t n = c.n;
    hipEvent_t e0, e1;
    NB_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(NBODY_E_HIP, "hipEventCreate failed");
    }
    nbody_status st = NBODY_OK;
    int rows = 0;
    for (int64_t na : sizes) {
        nb::TuneRow best{na, 1, 256, 0, 0, 1e300};
        for (int ni : {1, 2})
            for (int block : {64, 128, 256})
                for (int jpath : {1, 2, 3}) {
                    // the wave j-split kernel ignores ni and block, and serves small active sets
                    if (jpath == 3 && (ni != 1 || block != 64 || na > 64)) continue;
                    const int64_t prow = nb::part_rows_for(n);
                    const int base = nb::auto_split_path(n, na, ni, block, jpath, prow);
                    int prev = -1;
                    for (int mult : {1, 2, 4}) {   // splits base / 2, base, base * 2
                        int sp = mult == 1 ? base / 2 : (mult == 2 ? base : base * 2);
                        sp = sp < 1 ? 1 : (sp > 65535 ? 65535 : sp);
                        if (int64_t(sp) * na > prow) sp = int(prow / na);
                        if (sp == prev) continue;
                        prev = sp;
                        nb::ForceArgs a{};
                        a.rec = ctx->ws + ctx->lay.rec;
                        a.n = n;
                        a.act = all;
                        a.n_act = na;
                        a.eps2 = c.eps2;
                        a.n_hard = hard_count(c);
                        a.out[0] = F;
                        a.out[1] = F + 3 * n;
                        a.out[2] = c.order >= 6 ? F + 6 * n : nullptr;
                        a.out[3] = c.order >= 8 ? F + 9 * n : nullptr;
                        a.out[4] = nullptr;
                        a.part = ws_at<double>(ctx, ctx->lay.part);
                        a.part_rows = prow;
                        a.ni = ni;
                        a.block = block;
                        a.n_split = sp;
                        a.jpath = jpath;
                        hipError_t e = nb::launch_force(c.order, c.precision, a, ctx->stream, nullptr);
                        if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
                        for (int r = 0; e == hipSuccess && r < reps; ++r)
                            e = nb::launch_force(c.order, c.precision, a, ctx->stream, nullptr);
                        if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
                        if (e == hipSuccess) e = hipEventSynchronize(e1);
                        float ms = 0.0f;
                        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                        if (e != hipSuccess) {
                            st = fail(NBODY_E_HIP, "nbody_autotune: %s", hipGetErrorString(e));
                            break;
                        }
                        const double per = double(ms) / reps;
                        if (per < best.ms) best = nb::TuneRow{na, ni, block, sp, jpath, per};
                    }
                    if (st != NBODY_OK) break;
                }
        if (st != NBODY_OK) break;
        ctx->tune[rows++] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != NBODY_OK) return st;
    ctx->n_tune = rows;
    ctx->tuned = true;
    ctx->manual = false;
    return NBODY_OK;
}

nbody_status nbody_get_tuning(nbody_ctx *ctx, int32_t max_rows, int64_t *n_act, int32_t *shape, double *ms,
                              int32_t *rows)
{
    if (!ctx || !rows) return fail(NBODY_E_INVALID, "ctx and rows are required");
    if (max_rows < 0) return fail(NBODY_E_INVALID, "max_rows must be >= 0");
    const int r = ctx->tuned ? (ctx->n_tune < max_rows ? ctx->n_tune : max_rows) : 0;
    for (int k = 0; k < r; ++k) {
        if (n_act) n_act[k] = ctx->tune[k].n_act;
        if (shape) {
            shape[4 * k + 0] = ctx->tune[k].ni;
            shape[4 * k + 1] = ctx->tune[k].block;
            shape[4 * k + 2] = ctx->tune[k].n_split;
            shape[4 * k + 3] = ctx->tune[k].jpath;
        }
        if (ms) ms[k] = ctx->tune[k].ms;
    }
    *rows = ctx->tuned ? ctx->n_tune : 0;
    return NBODY_OK;
}

nbody_status nbody_get_last_launch(nbody_ctx *ctx, int32_t out[4])
{
    if (!ctx || !out) return fail(NBODY_E_INVALID, "ctx and out are required");
    out[0] = ctx->last_shape.ni;
    out[1] = ctx->last_shape.block;
    out[2] = ctx->last_shape.n_split;
    out[3] = ctx->last_shape.jpath;
    return NBODY_OK;
}

nbody_status nbody_init(nbody_ctx *ctx, nbody_state *st)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    nbody_status s = check_state(ctx, st);
    if (s != NBODY_OK) return s;
    const nbody_config &c = ctx->cfg;
    void *irec = ctx->ws + ctx->lay.irec;
    int32_t *all = ws_at<int32_t>(ctx, ctx->lay.act);
    NB_HIP(nb::launch_iota(c.n, all, ctx->stream));
    // pass 1: acceleration and jerk from positions and velocities
    NB_HIP(nb::launch_pack_f64(c.n, st->m, st->x, st->v, nullptr, nullptr, irec, ctx->stream));
    s = run_force(ctx, 8, NBODY_FP64, irec, c.n, all, st->d[0], st->d[1], nullptr, nullptr, nullptr);
    if (s != NBODY_OK) return s;
    if (c.order >= 6) {
        // pass 2: snap and crackle, using the pass-1 acceleration and jerk
        NB_HIP(nb::launch_pack_f64(c.n, st->m, st->x, st->v, st->d[0], st->d[1], irec, ctx->stream));
        s = run_force(ctx, 8, NBODY_FP64, irec, c.n, all, nullptr, nullptr, st->d[2], st->d[3], nullptr);
        if (s != NBODY_OK) return s;
    }
    if (nb::pn_on(c))   // hard pairs at t = 0, from the state itself, after pass 2 (Newtonian a, jerk)
        NB_HIP(nb::launch_pn(c, *st, nullptr, 0, all, c.n, st->d[0], st->d[1], c.order >= 6 ? st->d[2] : nullptr,
                             c.order >= 6 ? st->d[3] : nullptr, ctx->stream));
    NB_HIP(nb::launch_init_levels(c, *st, st->d[0], st->d[1], ctx->stream));
    ctx->predicted = false;
    return NBODY_OK;
}

nbody_status nbody_predict(nbody_ctx *ctx, const nbody_state *st, int64_t t_tick)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    nbody_status s = check_state(ctx, st);
    if (s != NBODY_OK) return s;
    if (t_tick < 0) return fail(NBODY_E_INVALID, "t_tick must be >= 0");
    NB_HIP(nb::launch_predict(ctx->cfg.order, ctx->cfg.precision, ctx->cfg.n, *st, t_tick, ctx->ws + ctx->lay.rec,
                              ctx->stream));
    ctx->predicted = true;
    return NBODY_OK;
}

nbody_status nbody_force_block(nbody_ctx *ctx, int64_t n_act, const int32_t *act_idx, double *acc, double *jrk,
                               double *snp, double *crk, double *pot)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    if (!ctx->predicted) return fail(NBODY_E_STATE, "nbody_force_block before nbody_predict");
    if (n_act < 0 || n_act > ctx->cfg.n) return fail(NBODY_E_INVALID, "n_act must be in [0, n]");
    if (n_act == 0) return NBODY_OK;
    if (!act_idx || (reinterpret_cast<uintptr_t>(act_idx) & 3u)) return fail(NBODY_E_INVALID, "act_idx must be non-NULL, 4-byte aligned");
    if (!acc || !jrk || !aligned8(acc) || !aligned8(jrk)) return fail(NBODY_E_INVALID, "acc and jrk must be non-NULL, 8-byte aligned");
    const double *opt[3] = {snp, crk, pot};
    for (const double *p : opt)
        if (p && !aligned8(p)) return fail(NBODY_E_INVALID, "outputs must be 8-byte aligned");
    if (ctx->cfg.order < 6) snp = nullptr;
    if (ctx->cfg.order < 8) crk = nullptr;
    return run_force(ctx, ctx->cfg.order, ctx->cfg.precision, ctx->ws + ctx->lay.rec, n_act, act_idx, acc, jrk, snp,
                     crk, pot);
}

nbody_status nbody_predict_force(nbody_ctx *ctx, const nbody_state *st, int64_t t_tick, int64_t n_act,
                                 const int32_t *act_idx, double *acc, double *jrk, double *snp, double *crk,
                                 double *pot)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    nbody_status s = check_state(ctx, st);
    if (s != NBODY_OK) return s;
    if (t_tick < 0) return fail(NBODY_E_INVALID, "t_tick must be >= 0");
    if (n_act < 0 || n_act > ctx->cfg.n) return fail(NBODY_E_INVALID, "n_act must be in [0, n]");
    if (n_act == 0) return nbody_predict(ctx, st, t_tick);
    if (!act_idx || (reinterpret_cast<uintptr_t>(act_idx) & 3u)) return fail(NBODY_E_INVALID, "act_idx must be non-NULL, 4-byte aligned");
    if (!acc || !jrk || !aligned8(acc) || !aligned8(jrk)) return fail(NBODY_E_INVALID, "acc and jrk must be non-NULL, 8-byte aligned");
    const double *opt[3] = {snp, crk, pot};
    for (const double *p : opt)
        if (p && !aligned8(p)) return fail(NBODY_E_INVALID, "outputs must be 8-byte aligned");
    if (ctx->cfg.order < 6) snp = nullptr;
    if (ctx->cfg.order < 8) crk = nullptr;
    return run_predict_force(ctx, st, t_tick, n_act, act_idx, acc, jrk, snp, crk, pot, nullptr);
}

nbody_status nbody_force_block_nb(nbody_ctx *ctx, int64_t n_act, const int32_t *act_idx, const double *h2,
                                  int32_t max_nb, double *acc_irr, double *jrk_irr, double *acc_reg,
                                  double *jrk_reg, int32_t *nb_count, int32_t *nb_list)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    const nbody_config &c = ctx->cfg;
    if (c.order != 4) return fail(NBODY_E_INVALID, "neighbour forces need an order-4 context (got %d)", c.order);
    if (c.precision != NBODY_FP64 && c.precision != NBODY_MIXED)
        return fail(NBODY_E_INVALID, "neighbour forces support FP64 and MIXED precision");
    if (!ctx->predicted) return fail(NBODY_E_STATE, "nbody_force_block_nb before nbody_predict");
    if (n_act < 0 || n_act > c.n) return fail(NBODY_E_INVALID, "n_act must be in [0, n]");
    if (max_nb < 0 || max_nb > nb::kMaxNeighbours)
        return fail(NBODY_E_INVALID, "max_nb must be in [0, %d] (got %d)", nb::kMaxNeighbours, max_nb);
    if (n_act == 0) return NBODY_OK;
    if (!act_idx || (reinterpret_cast<uintptr_t>(act_idx) & 3u)) return fail(NBODY_E_INVALID, "act_idx must be non-NULL, 4-byte aligned");
    if (!h2 || !aligned8(h2)) return fail(NBODY_E_INVALID, "h2 must be non-NULL, 8-byte aligned");
    const double *outs[4] = {acc_irr, jrk_irr, acc_reg, jrk_reg};
    for (const double *p : outs)
        if (!p || !aligned8(p)) return fail(NBODY_E_INVALID, "force outputs must be non-NULL, 8-byte aligned");
    if (!nb_count || (reinterpret_cast<uintptr_t>(nb_count) & 3u)) return fail(NBODY_E_INVALID, "nb_count must be non-NULL, 4-byte aligned");
    if (max_nb > 0 && (!nb_list || (reinterpret_cast<uintptr_t>(nb_list) & 3u)))
        return fail(NBODY_E_INVALID, "nb_list must be non-NULL, 4-byte aligned when max_nb > 0");
    const int64_t scratch = nb::part_rows_for(c.n) * nb::kMaxComp * int64_t(sizeof(double));
    const int sp = nb::nb_split(c.n, n_act, max_nb, scratch, 0);
    if (sp < 1)
        return fail(NBODY_E_INVALID, "n_act * (13 + max_nb) = %lld exceeds the scratch (%lld); call with fewer rows",
                    (long long)(n_act * (13 + int64_t(max_nb))), (long long)(scratch / 4));
    nb::NbArgs a{};
    a.rec = ctx->ws + ctx->lay.rec;
    a.n = c.n;
    a.act = act_idx;
    a.n_act = n_act;
    a.h2 = h2;
    a.eps2 = c.eps2;
    a.n_hard = hard_count(c);
    a.max_nb = max_nb;
    a.scratch = ws_at<double>(ctx, ctx->lay.part);
    a.acc_irr = acc_irr;
    a.jrk_irr = jrk_irr;
    a.acc_reg = acc_reg;
    a.jrk_reg = jrk_reg;
    a.nb_count = nb_count;
    a.nb_list = nb_list;
    int used = 0;
    NB_HIP(nb::launch_force_nb(c.precision, a, sp, ctx->stream, &used));
    ctx->stats.interactions += double(n_act) * double(c.n);
    return NBODY_OK;
}

nbody_status nbody_set_fusion(nbody_ctx *ctx, int32_t enable)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    if (enable != 0 && enable != 1) return fail(NBODY_E_INVALID, "enable must be 0 or 1 (got %d)", enable);
    ctx->fuse = enable == 1;
    return NBODY_OK;
}

nbody_status nbody_correct(nbody_ctx *ctx, nbody_state *st, int64_t n_act, const int32_t *act_idx, int64_t t_tick,
                           const double *acc, const double *jrk, const double *snp, const double *crk)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    nbody_status s = check_state(ctx, st);
    if (s != NBODY_OK) return s;
    if (n_act < 0 || n_act > ctx->cfg.n) return fail(NBODY_E_INVALID, "n_act must be in [0, n]");
    if (n_act == 0) return NBODY_OK;
    if (!act_idx) return fail(NBODY_E_INVALID, "act_idx is NULL");
    if (!acc || !jrk) return fail(NBODY_E_INVALID, "acc and jrk are required");
    if (ctx->cfg.order >= 6 && !snp) return fail(NBODY_E_INVALID, "snp is required for order >= 6");
    if (ctx->cfg.order >= 8 && !crk) return fail(NBODY_E_INVALID, "crk is required for order 8");
    const double *f[4] = {acc, jrk, snp, crk};
    NB_HIP(nb::launch_correct(ctx->cfg, *st, n_act, act_idx, nullptr, t_tick, f, scalars(ctx), ctx->stream));
    return NBODY_OK;
}

nbody_status nbody_schedule(nbody_ctx *ctx, const nbody_state *st, int32_t *act_idx_out, int64_t *t_next_out,
                            int64_t *n_act_out)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    nbody_status s = check_state(ctx, st);
    if (s != NBODY_OK) return s;
    if (!act_idx_out) return fail(NBODY_E_INVALID, "act_idx_out is NULL");
    NB_HIP(nb::launch_schedule(ctx->cfg.n, st->t_tick, st->level, ctx->ws + ctx->lay.sched, act_idx_out,
                               scalars(ctx), nullptr, 0, ctx->stream));
    nb::DevScalars h;
    s = read_scalars(ctx, &h);
    if (s != NBODY_OK) return s;
    if (t_next_out) *t_next_out = h.t_next;
    if (n_act_out) *n_act_out = h.n_act;
    return NBODY_OK;
}

}  // extern "C"

namespace {

// Record the device counters read in h; NBODY_E_NONFINITE when the number of
// non-finite corrected values grew since the last read.
nbody_status take_counters(nbody_ctx *ctx, const nb::DevScalars &h, int64_t t_tick)
{
    const int64_t nonfinite_before = ctx->stats.nonfinite;
    ctx->stats.dt_underflow = int64_t(h.underflow);
    ctx->stats.nonfinite = int64_t(h.nonfinite);
    if (ctx->stats.nonfinite > nonfinite_before)
        return fail(NBODY_E_NONFINITE, "%lld corrected particles became non-finite at tick %lld",
                    (long long)(ctx->stats.nonfinite - nonfinite_before), (long long)t_tick);
    return NBODY_OK;
}

// One block step unless its time would exceed t_limit (*stepped = false then,
// and nothing but the scheduler ran).  The scheduler's result is read back to
// size the force launch; with `check` the counters are read again after the
// corrector (else the next call's first read sees them).
nbody_status step_impl(nbody_ctx *ctx, nbody_state *st, int64_t t_limit, bool check, int64_t *t_out,
                       int64_t *n_act_out, bool *stepped, int64_t *t_prev)
{
    const nbody_config &c = ctx->cfg;
    int32_t *act = ws_at<int32_t>(ctx, ctx->lay.act);
    const bool tm = ctx->timing && ctx->ev_made;
    *stepped = false;
    if (tm) NB_HIP(hipEventRecord(ctx->ev[0], ctx->stream));
    const int64_t seq = ++ctx->pub_seq;
    NB_HIP(nb::launch_schedule(c.n, st->t_tick, st->level, ctx->ws + ctx->lay.sched, act, scalars(ctx),
                               ctx->pub_dev, seq, ctx->stream));
    if (tm) NB_HIP(hipEventRecord(ctx->ev[1], ctx->stream));
    nb::DevScalars h;
    nbody_status s = read_published(ctx, seq, &h);
    if (s != NBODY_OK) return s;
    s = take_counters(ctx, h, *t_prev);   // the previous corrector's counters
    if (s != NBODY_OK) return s;
    const int64_t t_next = h.t_next, n_act = h.n_act;
    if (n_act <= 0 || n_act > c.n) return fail(NBODY_E_STATE, "scheduler found %lld active particles", (long long)n_act);
    if (t_next > t_limit) return NBODY_OK;
    if (tm) NB_HIP(hipEventRecord(ctx->ev[2], ctx->stream));
    double *F = ws_at<double>(ctx, ctx->lay.force);
    double *acc = F, *jrk = F + 3 * n_act, *snp = F + 6 * n_act, *crk = F + 9 * n_act;
    const nb::ForceArgs shape = force_args(ctx, nullptr, n_act, act, acc, jrk, snp, crk, nullptr);
    if (ctx->fuse && shape.jpath == 3) {
        // predictor inside the force kernel: the predictor phase is empty
        if (tm) NB_HIP(hipEventRecord(ctx->ev[3], ctx->stream));
        s = run_predict_force(ctx, st, t_next, n_act, act, acc, jrk, c.order >= 6 ? snp : nullptr,
                              c.order >= 8 ? crk : nullptr, nullptr, nullptr);
        if (s != NBODY_OK) return s;
    } else {
        s = nbody_predict(ctx, st, t_next);
        if (s != NBODY_OK) return s;
        if (tm) NB_HIP(hipEventRecord(ctx->ev[3], ctx->stream));
        s = run_force(ctx, c.order, c.precision, ctx->ws + ctx->lay.rec, n_act, act, acc, jrk,
                      c.order >= 6 ? snp : nullptr, c.order >= 8 ? crk : nullptr, nullptr);
        if (s != NBODY_OK) return s;
    }
    if (nb::pn_on(c))   // active hard particles come first in the ordered active list
        NB_HIP(nb::launch_pn(c, *st, st->t_tick, t_next, act, n_act, acc, jrk, c.order >= 6 ? snp : nullptr,
                             c.order >= 8 ? crk : nullptr, ctx->stream));
    if (tm) NB_HIP(hipEventRecord(ctx->ev[4], ctx->stream));
    const double *f[4] = {acc, jrk, snp, crk};
    NB_HIP(nb::launch_correct(c, *st, n_act, act, nullptr, t_next, f, scalars(ctx), ctx->stream));
    if (tm) NB_HIP(hipEventRecord(ctx->ev[5], ctx->stream));
    ctx->stats.steps += 1;
    ctx->stats.sum_n_act += n_act;
    *stepped = true;
    *t_out = t_next;
    *n_act_out = n_act;
    *t_prev = t_next;
    if (tm) {
        NB_HIP(hipEventSynchronize(ctx->ev[5]));
        for (int k = 0; k < 5; ++k) {
            float ms = 0.0f;
            NB_HIP(hipEventElapsedTime(&ms, ctx->ev[k], ctx->ev[k + 1]));
            ctx->phase_ms[k] += ms;
        }
        ctx->timed_steps += 1;
    }
    if (check) {
        s = read_scalars(ctx, &h);
        if (s != NBODY_OK) return s;
        return take_counters(ctx, h, t_next);
    }
    return NBODY_OK;
}

}  // namespace

extern "C" {

nbody_status nbody_step(nbody_ctx *ctx, nbody_state *st, int64_t *t_tick_out, int64_t *n_act_out)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    nbody_status s = check_state(ctx, st);
    if (s != NBODY_OK) return s;
    int64_t t = 0, na = 0, prev = 0;
    bool stepped = false;
    s = step_impl(ctx, st, INT64_MAX, true, &t, &na, &stepped, &prev);
    if (s != NBODY_OK) return s;
    if (t_tick_out) *t_tick_out = t;
    if (n_act_out) *n_act_out = na;
    return NBODY_OK;
}

nbody_status nbody_run(nbody_ctx *ctx, nbody_state *st, int64_t t_end_tick, int64_t max_steps, int64_t *steps_out,
                       int64_t *t_tick_out)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    nbody_status s = check_state(ctx, st);
    if (s != NBODY_OK) return s;
    if (t_end_tick < 0 || max_steps < 0) return fail(NBODY_E_INVALID, "t_end_tick and max_steps must be >= 0");
    int64_t steps = 0, t = 0, na = 0, prev = 0;
    bool stepped = true;
    while (steps < max_steps) {
        s = step_impl(ctx, st, t_end_tick, false, &t, &na, &stepped, &prev);
        if (s != NBODY_OK || !stepped) break;
        ++steps;
    }
    if (s == NBODY_OK && stepped) {   // the last corrector's counters were not read yet
        nb::DevScalars h;
        s = read_scalars(ctx, &h);
        if (s == NBODY_OK) s = take_counters(ctx, h, prev);
    }
    if (steps_out) *steps_out = steps;
    if (t_tick_out) *t_tick_out = prev;
    return s;
}

nbody_status nbody_energy(nbody_ctx *ctx, const nbody_state *st, double *ekin, double *epot)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    nbody_status s = check_state(ctx, st);
    if (s != NBODY_OK) return s;
    if (!ekin || !epot) return fail(NBODY_E_INVALID, "ekin and epot are required");
    int np = 0;
    double *part = ws_at<double>(ctx, ctx->lay.energy);
    NB_HIP(nb::launch_energy(ctx->cfg.n, ctx->cfg.n, hard_count(ctx->cfg), ctx->cfg.eps2, st->m, st->x, st->v, part, &np,
                             ctx->stream));
    std::vector<double> h(2 * size_t(np));
    NB_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    NB_HIP(hipStreamSynchronize(ctx->stream));
    double T = 0.0, W = 0.0;
    for (int b = 0; b < np; ++b) {
        T += h[2 * b];
        W += h[2 * b + 1];
    }
    *ekin = T;
    *epot = W;
    return NBODY_OK;
}

nbody_status nbody_get_predicted(nbody_ctx *ctx, double *xp, double *vp, double *ap, double *jp)
{
    if (!ctx) return fail(NBODY_E_INVALID, "ctx is NULL");
    if (!ctx->predicted) return fail(NBODY_E_STATE, "nbody_get_predicted before nbody_predict");
    if (!xp || !vp || !aligned8(xp) || !aligned8(vp)) return fail(NBODY_E_INVALID, "xp and vp must be non-NULL, 8-byte aligned");
    if (ctx->cfg.order < 6) ap = nullptr;
    if (ctx->cfg.order < 8) jp = nullptr;
    NB_HIP(nb::launch_unpack(ctx->cfg.order, ctx->cfg.precision, ctx->cfg.n, ctx->ws + ctx->lay.rec, xp, vp, ap, jp,
                             ctx->stream));
    return NBODY_OK;
}

nbody_status nbody_get_stats(nbody_ctx *ctx, nbody_stats *out)
{
    if (!ctx || !out) return fail(NBODY_E_INVALID, "ctx and out are required");
    nb::DevScalars h;
    nbody_status s = read_scalars(ctx, &h);
    if (s != NBODY_OK) return s;
    ctx->stats.dt_underflow = int64_t(h.underflow);
    ctx->stats.nonfinite = int64_t(h.nonfinite);
    *out = ctx->stats;
    return NBODY_OK;
}

}  // extern "C"
