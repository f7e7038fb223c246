// batch_api.cpp -- C-ABI of the batched form: argument checks, the batch
// workspace layout, and the launch sequence of initialisation and of one
// batched step (also what a graph capture records).
#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "batch.h"

namespace {

using nb::fail;

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

struct BatchLayout {
    size_t off, ord, cid, tnext, bmin, bcnt, blk, plan, nact, aoff, ioff, poff, jchunk, split, tcur, rank, ctr, act,
        part, force, rec, energy, total;
};

int64_t max_cluster(const std::vector<int64_t> &off)
{
    int64_t m = 0;
    for (size_t c = 0; c + 1 < off.size(); ++c) m = std::max(m, off[c + 1] - off[c]);
    return m;
}

// Scheduling blocks of all clusters (each cluster in blocks of kBatchSchedBlock).
int64_t sched_blocks(const std::vector<int64_t> &off)
{
    int64_t s = 0;
    for (size_t c = 0; c + 1 < off.size(); ++c) s += (off[c + 1] - off[c] + nb::kBatchSchedBlock - 1) / nb::kBatchSchedBlock;
    return s;
}

int64_t sum_energy_blocks(const std::vector<int64_t> &off)
{
    int64_t s = 0;
    for (size_t c = 0; c + 1 < off.size(); ++c) s += (off[c + 1] - off[c] + 255) / 256;
    return s;
}

BatchLayout make_batch_layout(const nbody_config &c, const std::vector<int64_t> &off, int nb)
{
    BatchLayout L{};
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t r = at;
        at += up256(bytes);
        return r;
    };
    const size_t n = size_t(c.n), nc = off.size() - 1, cells = nc * size_t(nb);
    L.off = take((nc + 1) * sizeof(int64_t));
    L.ord = take(nc * sizeof(int32_t));
    L.cid = take(n * sizeof(int32_t));
    L.tnext = take(nc * sizeof(int64_t));
    L.bmin = take(cells * sizeof(int64_t));
    L.bcnt = take(cells * sizeof(int32_t));
    L.blk = take(2 * size_t(sched_blocks(off)) * sizeof(int32_t));
    L.plan = take(sizeof(nb::BatchPlan));
    L.nact = take(nc * sizeof(int64_t));
    L.aoff = take((nc + 1) * sizeof(int64_t));
    L.ioff = take((nc + 1) * sizeof(int64_t));
    L.poff = take((nc + 1) * sizeof(int64_t));
    L.jchunk = take(nc * sizeof(int64_t));
    L.split = take(nc * sizeof(int32_t));
    L.tcur = take(nc * sizeof(int64_t));
    L.rank = take(nc * sizeof(nb::BatchRank));
    L.ctr = take(sizeof(nb::BatchCounters));
    L.act = take(n * sizeof(int32_t));
    // split partials: the plan keeps sum_c splits_c * active_c <= i_tile *
    // items + n; 12 components (the order-8 initialisation passes)
    L.part = take(12 * (size_t(nb::kBatchMaxRows) + n) * sizeof(double));
    L.force = take(12 * n * sizeof(double));
    L.rec = take(n * size_t(std::max(nb::record_bytes(c.order, c.precision), nb::record_bytes(8, NBODY_FP64))));
    L.energy = take(2 * size_t(sum_energy_blocks(off)) * sizeof(double));
    L.total = at;
    return L;
}

nbody_status check_batch(const nbody_config *cfg, int32_t nc, const int64_t *off, std::vector<int64_t> *out,
                         int *nb_out)
{
    nbody_status s = nb::check_config_checked(cfg);
    if (s == NBODY_OK && nb::pn_on(*cfg))
        s = fail(NBODY_E_UNSUPPORTED, "post-Newtonian terms are not available in the batched form");
    if (s != NBODY_OK) return s;
    if (nc < 1 || nc > 65535) return fail(NBODY_E_INVALID, "n_clusters must be in [1, 65535] (got %d)", nc);
    if (!off) return fail(NBODY_E_INVALID, "off is NULL");
    if (off[0] != 0) return fail(NBODY_E_INVALID, "off[0] must be 0");
    int64_t smallest = INT64_MAX;
    for (int c = 0; c < nc; ++c) {
        const int64_t sz = off[c + 1] - off[c];
        if (sz < 2) return fail(NBODY_E_INVALID, "cluster %d has %lld particles (need >= 2)", c, (long long)sz);
        if (sz >= (int64_t(1) << 31))
            return fail(NBODY_E_UNSUPPORTED, "cluster %d has %lld particles (at most 2^31 - 1)", c, (long long)sz);
        smallest = std::min(smallest, sz);
    }
    if (off[nc] != cfg->n) return fail(NBODY_E_INVALID, "off[n_clusters] = %lld must equal n = %lld",
                                       (long long)off[nc], (long long)cfg->n);
    if (cfg->n_hard > smallest) return fail(NBODY_E_INVALID, "n_hard must not exceed the smallest cluster");
    out->assign(off, off + nc + 1);
    const int64_t nb = (max_cluster(*out) + nb::kBatchSchedBlock - 1) / nb::kBatchSchedBlock;
    if (nb * int64_t(nc) > (int64_t(1) << 22))
        return fail(NBODY_E_UNSUPPORTED, "clusters too many and too uneven: %lld scheduling blocks of %d per cluster",
                    (long long)nb, nb::kBatchSchedBlock);
    *nb_out = int(nb);
    return NBODY_OK;
}

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

}  // namespace

struct nbody_batch {
    nbody_config cfg;
    int nc;
    std::vector<int64_t> off;
    std::vector<int32_t> ord;
    std::vector<int32_t> blk;   // (cluster, block) of every scheduling block
    hipStream_t stream;
    char *ws;
    BatchLayout lay;
    nb::BatchLaunch L;
    int device;
    int force_grid_req;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

nbody_status check_bstate(const nbody_batch *b, const nbody_state *st)
{
    if (!st) return fail(NBODY_E_INVALID, "state is NULL");
    const void *ptrs[] = {st->m, st->x, st->v, st->t_tick, st->level};
    for (const void *p : ptrs)
        if (!p || !aligned8(p)) return fail(NBODY_E_INVALID, "state pointers must be non-NULL and 8-byte aligned");
    for (int k = 0; k <= b->cfg.order - 3; ++k)
        if (!st->d[k] || !aligned8(st->d[k]))
            return fail(NBODY_E_INVALID, "state d[%d] must be non-NULL and 8-byte aligned for order %d", k,
                        b->cfg.order);
    return NBODY_OK;
}

template <class T> T *at(nbody_batch *b, size_t off) { return reinterpret_cast<T *>(b->ws + off); }

nbody_status enqueue_step(nbody_batch *b, const nbody_state &st)
{
    const nbody_config &c = b->cfg;
    const nb::BatchLaunch &L = b->L;
    double *F = L.force;
    const int64_t n = c.n;
    void *rec = b->ws + b->lay.rec;
    NB_HIP(nb::batch_schedule(L, st, 0, c.order, b->stream));
    NB_HIP(nb::batch_predict(L, st, c.order, c.precision, rec, b->stream));
    NB_HIP(nb::batch_force(L, c.order, c.precision, rec, b->stream));
    NB_HIP(nb::batch_reduce(L, c.order, F, F + 3 * n, F + 6 * n, F + 9 * n, b->stream));
    NB_HIP(nb::batch_correct(L, c, st, b->stream));
    return NBODY_OK;
}

void drop_graph(nbody_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

nbody_status sync(nbody_batch *b)
{
    NB_HIP(hipStreamSynchronize(b->stream));
    return NBODY_OK;
}

}  // namespace

extern "C" {

nbody_status nbody_batch_workspace_size(const nbody_config *cfg, int32_t n_clusters, const int64_t *off,
                                        size_t *bytes)
{
    std::vector<int64_t> o;
    int nb = 0;
    nbody_status s = check_batch(cfg, n_clusters, off, &o, &nb);
    if (s != NBODY_OK) return s;
    if (!bytes) return fail(NBODY_E_INVALID, "bytes is NULL");
    *bytes = make_batch_layout(*cfg, o, nb).total;
    return NBODY_OK;
}

nbody_status nbody_batch_create(const nbody_config *cfg, int32_t n_clusters, const int64_t *off, void *workspace,
                                size_t bytes, void *stream, nbody_batch **out)
{
    std::vector<int64_t> o;
    int nb = 0;
    nbody_status s = check_batch(cfg, n_clusters, off, &o, &nb);
    if (s != NBODY_OK) return s;
    if (!out) return fail(NBODY_E_INVALID, "out is NULL");
    const BatchLayout lay = make_batch_layout(*cfg, o, nb);
    if (!workspace) return fail(NBODY_E_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) & 255u) return fail(NBODY_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < lay.total) return fail(NBODY_E_WORKSPACE, "workspace too small: %zu < %zu bytes", bytes, lay.total);
    nbody_batch *b = new (std::nothrow) nbody_batch();
    if (!b) return fail(NBODY_E_INVALID, "out of host memory");
    b->cfg = *cfg;
    b->nc = n_clusters;
    b->off = o;
    b->stream = static_cast<hipStream_t>(stream);
    b->ws = static_cast<char *>(workspace);
    b->lay = lay;
    b->graph = nullptr;
    b->exec = nullptr;
    // clusters by decreasing size (ties by index): the largest work items first
    b->ord.resize(size_t(n_clusters));
    std::iota(b->ord.begin(), b->ord.end(), 0);
    std::stable_sort(b->ord.begin(), b->ord.end(), [&](int32_t a, int32_t c) {
        return o[size_t(a) + 1] - o[size_t(a)] > o[size_t(c) + 1] - o[size_t(c)];
    });
    nb::BatchLaunch &L = b->L;
    L.nc = n_clusters;
    L.nb = nb;
    L.n = cfg->n;
    L.off = at<int64_t>(b, lay.off);
    L.ord = at<int32_t>(b, lay.ord);
    L.cid = at<int32_t>(b, lay.cid);
    L.tnext = at<int64_t>(b, lay.tnext);
    L.bmin = at<int64_t>(b, lay.bmin);
    L.bcnt = at<int32_t>(b, lay.bcnt);
    for (int c = 0; c < n_clusters; ++c) {
        const int64_t nbc = (o[size_t(c) + 1] - o[size_t(c)] + nb::kBatchSchedBlock - 1) / nb::kBatchSchedBlock;
        for (int64_t k = 0; k < nbc; ++k) {
            b->blk.push_back(c);
            b->blk.push_back(int32_t(k));
        }
    }
    L.nblk = int(b->blk.size() / 2);
    L.blk = at<int32_t>(b, lay.blk);
    L.plan = at<nb::BatchPlan>(b, lay.plan);
    L.ctr = at<nb::BatchCounters>(b, lay.ctr);
    L.act = at<int32_t>(b, lay.act);
    L.part = at<double>(b, lay.part);
    L.force = at<double>(b, lay.force);
    L.eps2 = cfg->eps2;
    L.n_hard = cfg->eps2 == 0.0 ? (int64_t(1) << 40) : cfg->n_hard;
    L.per_wg = 8;
    L.itile = 64;
    nb::BatchPlan hp{};
    hp.t_end = INT64_MAX;
    hp.n_live = 0;
    hp.nact = at<int64_t>(b, lay.nact);
    hp.aoff = at<int64_t>(b, lay.aoff);
    hp.ioff = at<int64_t>(b, lay.ioff);
    hp.poff = at<int64_t>(b, lay.poff);
    hp.jchunk = at<int64_t>(b, lay.jchunk);
    hp.split = at<int32_t>(b, lay.split);
    hp.tcur = at<int64_t>(b, lay.tcur);
    hp.rank = at<nb::BatchRank>(b, lay.rank);
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) {
        b->force_grid_req = 0;
        L.force_grid = nb::batch_force_resident(cfg->order, cfg->precision, L.itile, b->device);
        if (L.force_grid <= 0) e = hipErrorInvalidDeviceFunction;
        L.k_items = int(std::min<int64_t>(int64_t(L.force_grid) * L.per_wg, nb::kBatchMaxRows / L.itile));
    }
    if (e == hipSuccess) e = hipMemcpyAsync(L.plan, &hp, sizeof(hp), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(const_cast<int64_t *>(L.off), b->off.data(), b->off.size() * sizeof(int64_t),
                                            hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(const_cast<int32_t *>(L.ord), b->ord.data(), b->ord.size() * sizeof(int32_t),
                                            hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(const_cast<int32_t *>(L.blk), b->blk.data(), b->blk.size() * sizeof(int32_t),
                                            hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L.ctr, 0, sizeof(nb::BatchCounters), b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(hp.tcur, 0, size_t(n_clusters) * sizeof(int64_t), b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(hp.aoff, 0, size_t(n_clusters + 1) * sizeof(int64_t), b->stream);
    if (e == hipSuccess) e = nb::batch_cid(L, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        delete b;
        return fail(NBODY_E_HIP, "nbody_batch_create: %s", hipGetErrorString(e));
    }
    *out = b;
    return NBODY_OK;
}

nbody_status nbody_batch_destroy(nbody_batch *b)
{
    if (!b) return fail(NBODY_E_INVALID, "batch is NULL");
    drop_graph(b);
    delete b;
    return NBODY_OK;
}

nbody_status nbody_batch_init(nbody_batch *b, nbody_state *st)
{
    if (!b) return fail(NBODY_E_INVALID, "batch is NULL");
    nbody_status s = check_bstate(b, st);
    if (s != NBODY_OK) return s;
    const nbody_config &c = b->cfg;
    const nb::BatchLaunch &L = b->L;
    void *rec = b->ws + b->lay.rec;
    // every particle active at t = 0; FP64 order-8 pairwise terms
    NB_HIP(nb::batch_schedule(L, *st, 1, 8, b->stream));
    // pass 1: acceleration and jerk from positions and velocities
    NB_HIP(nb::launch_pack_f64(c.n, st->m, st->x, st->v, nullptr, nullptr, rec, b->stream));
    NB_HIP(nb::batch_force(L, 8, NBODY_FP64, rec, b->stream));
    NB_HIP(nb::batch_reduce(L, 8, st->d[0], st->d[1], nullptr, nullptr, b->stream));
    if (c.order >= 6) {
        // pass 2: snap and crackle, using the pass-1 acceleration and jerk
        NB_HIP(nb::batch_requeue(L, b->stream));
        NB_HIP(nb::launch_pack_f64(c.n, st->m, st->x, st->v, st->d[0], st->d[1], rec, b->stream));
        NB_HIP(nb::batch_force(L, 8, NBODY_FP64, rec, b->stream));
        NB_HIP(nb::batch_reduce(L, 8, nullptr, nullptr, st->d[2], st->d[3], b->stream));
    }
    NB_HIP(nb::launch_init_levels(c, *st, st->d[0], st->d[1], b->stream));
    NB_HIP(hipMemsetAsync(L.ctr, 0, sizeof(nb::BatchCounters), b->stream));
    return NBODY_OK;
}

nbody_status nbody_batch_set_end(nbody_batch *b, int64_t t_end_tick)
{
    if (!b) return fail(NBODY_E_INVALID, "batch is NULL");
    if (t_end_tick < 0) return fail(NBODY_E_INVALID, "t_end_tick must be >= 0");
    // the value must outlive the asynchronous copy: copy, then synchronise
    const int64_t v = t_end_tick;
    NB_HIP(hipMemcpyAsync(reinterpret_cast<char *>(b->L.plan) + offsetof(nb::BatchPlan, t_end), &v, sizeof(v),
                          hipMemcpyHostToDevice, b->stream));
    return sync(b);
}

nbody_status nbody_batch_step(nbody_batch *b, nbody_state *st, int64_t k)
{
    if (!b) return fail(NBODY_E_INVALID, "batch is NULL");
    nbody_status s = check_bstate(b, st);
    if (s != NBODY_OK) return s;
    if (k < 0) return fail(NBODY_E_INVALID, "k must be >= 0");
    for (int64_t r = 0; r < k; ++r) {
        s = enqueue_step(b, *st);
        if (s != NBODY_OK) return s;
    }
    return NBODY_OK;
}

nbody_status nbody_batch_capture(nbody_batch *b, nbody_state *st)
{
    if (!b) return fail(NBODY_E_INVALID, "batch is NULL");
    nbody_status s = check_bstate(b, st);
    if (s != NBODY_OK) return s;
    if (!b->stream) return fail(NBODY_E_UNSUPPORTED, "graph capture needs a stream other than the default stream");
    drop_graph(b);
    NB_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    s = enqueue_step(b, *st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (s != NBODY_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return s != NBODY_OK ? s : fail(NBODY_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    b->graph = g;
    const hipError_t e2 = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
        b->exec = nullptr;
        drop_graph(b);
        return fail(NBODY_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
    }
    return NBODY_OK;
}

nbody_status nbody_batch_replay(nbody_batch *b, int64_t k)
{
    if (!b) return fail(NBODY_E_INVALID, "batch is NULL");
    if (!b->exec) return fail(NBODY_E_STATE, "nbody_batch_replay before nbody_batch_capture");
    if (k < 0) return fail(NBODY_E_INVALID, "k must be >= 0");
    for (int64_t r = 0; r < k; ++r) NB_HIP(hipGraphLaunch(b->exec, b->stream));
    return NBODY_OK;
}

nbody_status nbody_batch_poll(nbody_batch *b, int64_t *n_live, int64_t *t_cur)
{
    if (!b || !n_live) return fail(NBODY_E_INVALID, "batch and n_live are required");
    nb::BatchPlan hp;
    NB_HIP(hipMemcpyAsync(&hp, b->L.plan, sizeof(hp), hipMemcpyDeviceToHost, b->stream));
    nbody_status s = sync(b);
    if (s != NBODY_OK) return s;
    *n_live = hp.n_live;
    if (t_cur) {
        NB_HIP(hipMemcpyAsync(t_cur, hp.tcur, size_t(b->nc) * sizeof(int64_t), hipMemcpyDeviceToHost, b->stream));
        return sync(b);
    }
    return NBODY_OK;
}

nbody_status nbody_batch_last_step(nbody_batch *b, int64_t *aoff, int32_t *act, double *forces)
{
    if (!b || !aoff) return fail(NBODY_E_INVALID, "batch and aoff are required");
    if (forces && !aligned8(forces)) return fail(NBODY_E_INVALID, "forces must be 8-byte aligned");
    nb::BatchPlan hp;
    NB_HIP(hipMemcpyAsync(&hp, b->L.plan, sizeof(hp), hipMemcpyDeviceToHost, b->stream));
    nbody_status s = sync(b);
    if (s != NBODY_OK) return s;
    NB_HIP(hipMemcpyAsync(aoff, hp.aoff, size_t(b->nc + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, b->stream));
    s = sync(b);
    if (s != NBODY_OK) return s;
    const int64_t na = aoff[b->nc];
    if (na > 0 && act)
        NB_HIP(hipMemcpyAsync(act, b->L.act, size_t(na) * sizeof(int32_t), hipMemcpyDeviceToDevice, b->stream));
    if (na > 0 && forces) {
        const size_t rows = size_t(3 * (b->cfg.order / 2));
        NB_HIP(hipMemcpy2DAsync(forces, size_t(na) * sizeof(double), b->L.force, size_t(b->cfg.n) * sizeof(double),
                                size_t(na) * sizeof(double), rows, hipMemcpyDeviceToDevice, b->stream));
    }
    return sync(b);
}

nbody_status nbody_batch_energy(nbody_batch *b, const nbody_state *st, double *ekin, double *epot)
{
    if (!b) return fail(NBODY_E_INVALID, "batch is NULL");
    nbody_status s = check_bstate(b, st);
    if (s != NBODY_OK) return s;
    if (!ekin || !epot) return fail(NBODY_E_INVALID, "ekin and epot are required");
    double *part = at<double>(b, b->lay.energy);
    std::vector<int> np(size_t(b->nc));
    std::vector<size_t> first(size_t(b->nc));
    size_t used = 0;
    for (int c = 0; c < b->nc; ++c) {
        const int64_t o = b->off[size_t(c)], nn = b->off[size_t(c) + 1] - o;
        const int64_t nh = b->cfg.eps2 == 0.0 ? nn : b->cfg.n_hard;
        first[size_t(c)] = used;
        NB_HIP(nb::launch_energy(nn, b->cfg.n, nh, b->cfg.eps2, st->m + o, st->x + o, st->v + o, part + used,
                                 &np[size_t(c)], b->stream));
        used += 2 * size_t(np[size_t(c)]);
    }
    std::vector<double> h(used);
    NB_HIP(hipMemcpyAsync(h.data(), part, used * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    s = sync(b);
    if (s != NBODY_OK) return s;
    for (int c = 0; c < b->nc; ++c) {
        double T = 0.0, W = 0.0;
        for (int k = 0; k < np[size_t(c)]; ++k) {
            T += h[first[size_t(c)] + 2 * size_t(k)];
            W += h[first[size_t(c)] + 2 * size_t(k) + 1];
        }
        ekin[c] = T;
        epot[c] = W;
    }
    return NBODY_OK;
}

nbody_status nbody_batch_get_stats(nbody_batch *b, nbody_stats *out)
{
    if (!b || !out) return fail(NBODY_E_INVALID, "batch and out are required");
    nb::BatchCounters h;
    NB_HIP(hipMemcpyAsync(&h, b->L.ctr, sizeof(h), hipMemcpyDeviceToHost, b->stream));
    nbody_status s = sync(b);
    if (s != NBODY_OK) return s;
    out->steps = h.steps;
    out->sum_n_act = h.sum_n_act;
    out->interactions = double(h.interactions);
    out->dt_underflow = int64_t(h.underflow);
    out->nonfinite = int64_t(h.nonfinite);
    return NBODY_OK;
}

nbody_status nbody_batch_set_launch(nbody_batch *b, int32_t force_grid, int32_t per_wg, int32_t i_tile)
{
    if (!b) return fail(NBODY_E_INVALID, "batch is NULL");
    if (force_grid < 0 || force_grid > (1 << 20)) return fail(NBODY_E_INVALID, "force_grid must be in [0, 2^20]");
    if (per_wg < 0 || per_wg > nb::kBatchMaxPerWG)
        return fail(NBODY_E_INVALID, "items_per_wg must be in [0, %d]", nb::kBatchMaxPerWG);
    if (i_tile != 0 && i_tile != 64 && i_tile != 128 && i_tile != 256)
        return fail(NBODY_E_INVALID, "i_tile must be 0, 64, 128 or 256");
    nb::BatchLaunch &L = b->L;
    L.itile = i_tile > 0 ? i_tile : 64;
    L.per_wg = per_wg > 0 ? per_wg : 8;
    b->force_grid_req = force_grid;
    L.force_grid = force_grid > 0 ? force_grid : nb::batch_force_resident(b->cfg.order, b->cfg.precision, L.itile, b->device);
    if (L.force_grid <= 0) return fail(NBODY_E_HIP, "occupancy query of the batched force kernel failed");
    L.k_items = int(std::min<int64_t>(int64_t(L.force_grid) * L.per_wg, nb::kBatchMaxRows / L.itile));
    return NBODY_OK;
}

nbody_status nbody_batch_get_launch(nbody_batch *b, int32_t out[3])
{
    if (!b || !out) return fail(NBODY_E_INVALID, "batch and out are required");
    out[0] = b->L.force_grid;
    out[1] = b->L.per_wg;
    out[2] = b->L.itile;
    return NBODY_OK;
}

nbody_status nbody_batch_autotune(nbody_batch *b, nbody_state *st, int32_t steps)
{
    if (!b) return fail(NBODY_E_INVALID, "batch is NULL");
    nbody_status s = check_bstate(b, st);
    if (s != NBODY_OK) return s;
    if (steps < 1 || steps > 100000) return fail(NBODY_E_INVALID, "steps must be in [1, 100000]");
    drop_graph(b);
    const nbody_config &c = b->cfg;
    nb::BatchLaunch &L = b->L;
    void *rec = b->ws + b->lay.rec;
    double *F = L.force;
    const int64_t n = c.n;
    const int keep_t = L.per_wg, keep_i = L.itile;
    const int itiles[3] = {64, 128, 256};
    const int targets[5] = {2, 4, 8, 16, 32};
    double total_ms[3][5] = {};
    // planning a step writes the counters, the clusters' times and the live
    // count: kept aside around each sweep and put back
    nb::BatchCounters ctr0;
    int64_t live0 = 0;
    std::vector<int64_t> tcur0(size_t(b->nc));
    int64_t *tcur = at<int64_t>(b, b->lay.tcur);
    char *live_dev = reinterpret_cast<char *>(L.plan) + offsetof(nb::BatchPlan, n_live);
    hipEvent_t e0, e1;
    NB_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(NBODY_E_HIP, "hipEventCreate failed");
    }
    for (int k = 0; s == NBODY_OK && k < steps; ++k) {
        if (hipMemcpyAsync(&ctr0, L.ctr, sizeof(ctr0), hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
            hipMemcpyAsync(&live0, live_dev, sizeof(live0), hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
            hipMemcpyAsync(tcur0.data(), tcur, tcur0.size() * sizeof(int64_t), hipMemcpyDeviceToHost, b->stream) !=
                hipSuccess)
            s = fail(NBODY_E_HIP, "counter copy failed");
        if (s == NBODY_OK) s = sync(b);
        bool predicted = false;
        for (int a = 0; s == NBODY_OK && a < 3; ++a)
            for (int t = 0; s == NBODY_OK && t < 5; ++t) {
                s = nbody_batch_set_launch(b, b->force_grid_req, targets[t], itiles[a]);
                // this step planned for the shape (the active sets and records
                // do not depend on it); one untimed and one timed force phase
                if (s == NBODY_OK && nb::batch_schedule(L, *st, 0, c.order, b->stream) != hipSuccess)
                    s = fail(NBODY_E_HIP, "schedule launch failed");
                if (s == NBODY_OK && !predicted) {
                    if (nb::batch_predict(L, *st, c.order, c.precision, rec, b->stream) != hipSuccess)
                        s = fail(NBODY_E_HIP, "predictor launch failed");
                    predicted = true;
                }
                for (int r = 0; s == NBODY_OK && r < 2; ++r) {
                    if (r == 1 && hipEventRecord(e0, b->stream) != hipSuccess) s = fail(NBODY_E_HIP, "event record failed");
                    if (s == NBODY_OK && (nb::batch_requeue(L, b->stream) != hipSuccess ||
                                          nb::batch_force(L, c.order, c.precision, rec, b->stream) != hipSuccess ||
                                          nb::batch_reduce(L, c.order, F, F + 3 * n, F + 6 * n, F + 9 * n, b->stream) !=
                                              hipSuccess))
                        s = fail(NBODY_E_HIP, "force launch failed");
                }
                if (s == NBODY_OK && hipEventRecord(e1, b->stream) != hipSuccess) s = fail(NBODY_E_HIP, "event record failed");
                if (s == NBODY_OK) s = sync(b);
                float ms = 0.0f;
                if (s == NBODY_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                    s = fail(NBODY_E_HIP, "event timing failed");
                total_ms[a][t] += double(ms);
            }
        if (s == NBODY_OK &&
            (hipMemcpyAsync(L.ctr, &ctr0, sizeof(ctr0), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
             hipMemcpyAsync(live_dev, &live0, sizeof(live0), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
             hipMemcpyAsync(tcur, tcur0.data(), tcur0.size() * sizeof(int64_t), hipMemcpyHostToDevice, b->stream) !=
                 hipSuccess))
            s = fail(NBODY_E_HIP, "restoring the counters failed");
        // then the step itself, with the shape in use before the call
        if (s == NBODY_OK) s = nbody_batch_set_launch(b, b->force_grid_req, keep_t, keep_i);
        if (s == NBODY_OK) s = enqueue_step(b, *st);
        if (s == NBODY_OK) s = sync(b);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != NBODY_OK) {
        (void)nbody_batch_set_launch(b, b->force_grid_req, keep_t, keep_i);
        return s;
    }
    int best_a = 0, best_t = 0;
    for (int a = 0; a < 3; ++a)
        for (int t = 0; t < 5; ++t)
            if (total_ms[a][t] < total_ms[best_a][best_t]) {
                best_a = a;
                best_t = t;
            }
    return nbody_batch_set_launch(b, b->force_grid_req, targets[best_t], itiles[best_a]);
}

}  // extern "C"
