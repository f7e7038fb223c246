// noalloc.hip -- nbody_predict_force_noalloc: the predictor folded into the
// wave j-split force kernel (the work of nbody_predict_force for a small
// active set) without a context or workspace, for callers that cannot
// allocate device memory.  The only scratch of that kernel pair, the j-split
// partial sums, lives in a static device array of fixed size.
#include <mutex>

#include "internal.h"

namespace {

using nb::fail;

// Partial-sum rows (active rows x j-splits) the static array holds, and the
// largest active set the entry point takes: with the default split of the
// wave j-split kernel, n_act <= 1024 needs at most about 34 000 rows.
constexpr int64_t kNoAllocRows = int64_t(1) << 16;
constexpr int64_t kNoAllocMaxAct = 1024;
constexpr int kMaxDevices = 64;

}  // namespace

// One copy per GPU (6.8 MB), held until the process ends.  In host code this
// name is not a device address: the address comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kNoAllocRows * nb::kMaxComp];

namespace {

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device
// (with that device current).
nbody_status scratch_address(double **out)
{
    int dev = -1;
    NB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(NBODY_E_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(NBODY_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<double *>(g_scratch_ptr[dev]);
    return NBODY_OK;
}

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

}  // namespace

extern "C" nbody_status nbody_predict_force_noalloc(const nbody_config *cfg, const nbody_state *st, int64_t t_tick,
                                                    int64_t n_act, const int32_t *act_idx, double *acc, double *jrk,
                                                    double *snp, double *crk, double *pot, void *stream)
{
    nbody_status s = nb::check_config_checked(cfg);
    if (s != NBODY_OK) return s;
    if (!st) return fail(NBODY_E_INVALID, "state is NULL");
    const void *ptrs[] = {st->m, st->x, st->v, st->t_tick};
    for (const void *p : ptrs)
        if (!p || !aligned(p, 8)) return fail(NBODY_E_INVALID, "state m, x, v, t_tick must be non-NULL, 8-byte aligned");
    for (int k = 0; k <= cfg->order - 3; ++k)
        if (!st->d[k] || !aligned(st->d[k], 8))
            return fail(NBODY_E_INVALID, "state d[%d] must be non-NULL and 8-byte aligned for order %d", k, cfg->order);
    if (t_tick < 0) return fail(NBODY_E_INVALID, "t_tick must be >= 0");
    if (n_act < 0 || n_act > cfg->n) return fail(NBODY_E_INVALID, "n_act must be in [0, n]");
    if (n_act > kNoAllocMaxAct)
        return fail(NBODY_E_INVALID, "nbody_predict_force_noalloc takes at most %lld active particles (got %lld): its "
                    "static scratch holds %lld partial-sum rows", (long long)kNoAllocMaxAct, (long long)n_act,
                    (long long)kNoAllocRows);
    if (n_act == 0) return NBODY_OK;
    if (!act_idx || !aligned(act_idx, 4)) return fail(NBODY_E_INVALID, "act_idx must be non-NULL, 4-byte aligned");
    if (!acc || !jrk || !aligned(acc, 8) || !aligned(jrk, 8))
        return fail(NBODY_E_INVALID, "acc and jrk must be non-NULL, 8-byte aligned");
    const double *opt[3] = {snp, crk, pot};
    for (const double *p : opt)
        if (p && !aligned(p, 8)) return fail(NBODY_E_INVALID, "outputs must be 8-byte aligned");
    if (cfg->order < 6) snp = nullptr;
    if (cfg->order < 8) crk = nullptr;
    double *part = nullptr;
    s = scratch_address(&part);
    if (s != NBODY_OK) return s;

    nb::ForceArgs a{};
    a.rec = nullptr;   // the fused kernel predicts from the state; no records
    a.n = cfg->n;
    a.act = act_idx;
    a.n_act = n_act;
    a.eps2 = cfg->eps2;
    a.n_hard = cfg->eps2 == 0.0 ? cfg->n : cfg->n_hard;
    a.out[0] = acc;
    a.out[1] = jrk;
    a.out[2] = snp;
    a.out[3] = crk;
    a.out[4] = pot;
    a.part = part;
    a.part_rows = kNoAllocRows;
    a.ni = 1;
    a.block = 64;
    a.n_split = 0;   // the default split of the wave j-split kernel, as nbody_predict_force
    a.jpath = 3;
    nb::PredIn in{};
    in.m = st->m;
    in.x = st->x;
    in.v = st->v;
    for (int k = 0; k < 6; ++k) in.d[k] = k <= cfg->order - 3 ? st->d[k] : nullptr;
    in.t_tick = st->t_tick;
    in.t = t_tick;
    NB_HIP(nb::launch_force_pred(cfg->order, cfg->precision, a, in, static_cast<hipStream_t>(stream), nullptr));
    return NBODY_OK;
}
