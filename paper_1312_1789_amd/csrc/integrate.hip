// integrate.hip -- the O(n) and O(n_act) kernels of a block step on gfx950:
// block-step scheduler, predictor, Hermite corrector with interpolation and
// time step, initial levels, and the FP64 energy diagnostic.
//
// Method (paper: Abstract; Sec. "Codes description"): Hermite integration of
// order 4, 6 or 8 with individual hierarchical block time steps.  Formulas:
// time-symmetric Hermite corrector (order 4: Hut & Makino; orders 6 and 8:
// Nitadori & Makino 2008), derivatives at the end of the step from the
// Hermite interpolant through both ends, Aarseth's step criterion (order 4)
// and its generalisation (orders 6 and 8, Nitadori & Makino 2008).
#include <climits>

#include "hermite.h"

namespace nb {
namespace {

template <int P, int PREC>
__global__ void __launch_bounds__(256)
k_predict(int64_t n, const double *__restrict__ m, const double *__restrict__ x, const double *__restrict__ v,
          const double *__restrict__ d0, const double *__restrict__ d1, const double *__restrict__ d2,
          const double *__restrict__ d3, const double *__restrict__ d4, const double *__restrict__ d5,
          const int64_t *__restrict__ t_tick, int64_t t, void *__restrict__ rec_out)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double dt = double(t - t_tick[i]) * (1.0 / double(kTicksPerUnit));
    const double *ds[6] = {d0, d1, d2, d3, d4, d5};
    predict_one<P, PREC>(n, i, dt, m, x, v, ds, rec_out);
}

// Predicted records back to FP64 arrays [3][n] (inspection and tests).
template <int P, int PREC>
__global__ void __launch_bounds__(256)
k_unpack(int64_t n, const void *__restrict__ rec, double *__restrict__ xp, double *__restrict__ vp,
         double *__restrict__ ap, double *__restrict__ jp)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double X[3], V[3], A[3] = {0, 0, 0}, J[3] = {0, 0, 0};
    if constexpr (PREC == NBODY_FP64) {
        const RecF64<P> r = static_cast<const RecF64<P> *>(rec)[i];
        X[0] = r.x; X[1] = r.y; X[2] = r.z; V[0] = r.vx; V[1] = r.vy; V[2] = r.vz;
        if constexpr (P >= 6) { A[0] = r.ax; A[1] = r.ay; A[2] = r.az; }
        if constexpr (P >= 8) { J[0] = r.jx; J[1] = r.jy; J[2] = r.jz; }
    } else {
        const RecDS<P> r = static_cast<const RecDS<P> *>(rec)[i];
        X[0] = double(r.xh) + double(r.xl); X[1] = double(r.yh) + double(r.yl); X[2] = double(r.zh) + double(r.zl);
        V[0] = double(r.vxh) + double(r.vxl); V[1] = double(r.vyh) + double(r.vyl); V[2] = double(r.vzh) + double(r.vzl);
        if constexpr (P >= 6) { A[0] = r.ax; A[1] = r.ay; A[2] = r.az; }
        if constexpr (P >= 8) { J[0] = r.jx; J[1] = r.jy; J[2] = r.jz; }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xp[c * n + i] = X[c];
        vp[c * n + i] = V[c];
        if (ap) ap[c * n + i] = A[c];
        if (jp) jp[c * n + i] = J[c];
    }
}

// FP64 order-8 records from plain arrays (initialisation passes).
__global__ void __launch_bounds__(256)
k_pack_f64(int64_t n, const double *__restrict__ m, const double *__restrict__ x, const double *__restrict__ v,
           const double *__restrict__ a, const double *__restrict__ j, RecF64<8> *__restrict__ rec)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    RecF64<8> r{};
    r.x = x[i]; r.y = x[n + i]; r.z = x[2 * n + i]; r.m = m[i];
    r.vx = v[i]; r.vy = v[n + i]; r.vz = v[2 * n + i];
    if (a) { r.ax = a[i]; r.ay = a[n + i]; r.az = a[2 * n + i]; }
    if (j) { r.jx = j[i]; r.jy = j[n + i]; r.jz = j[2 * n + i]; }
    rec[i] = r;
}

// Corrector + interpolation + new step for the active particles.
template <int P>
__global__ void __launch_bounds__(256)
k_correct(int64_t n, int64_t n_act_host, const int32_t *__restrict__ act, const DevScalars *src,
          int64_t t1_host, double *__restrict__ x, double *__restrict__ v, double *__restrict__ d0,
          double *__restrict__ d1, double *__restrict__ d2, double *__restrict__ d3, double *__restrict__ d4,
          double *__restrict__ d5, int64_t *__restrict__ t_tick, int32_t *__restrict__ level,
          const double *__restrict__ f0, const double *__restrict__ f1, const double *__restrict__ f2,
          const double *__restrict__ f3, double eta, int rule, int k_min, int k_max, DevScalars *sc)
{
    // active count and end time from the host, or from the device scheduler
    const int64_t qi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t na = src ? src->n_act : n_act_host;
    if (qi >= na) return;
    const int64_t t1 = src ? src->t_next : t1_host;
    const int64_t i = act[qi];
    if (i < 0 || i >= n) return;   // an index outside [0, n) is ignored
    double *dst[6] = {d0, d1, d2, d3, d4, d5};
    const double *fnew[4] = {f0, f1, f2, f3};
    const int fl = correct_one<P>(n, i, t1, fnew, na, qi, x, v, dst, t_tick, level, eta, rule, k_min, k_max);
    if (fl & 2) atomicAdd(&sc->underflow, 1ull);
    if (fl & 1) atomicAdd(&sc->nonfinite, 1ull);
}

// Initial levels from dt0 = eta_start |a| / |jerk|; times zero.
__global__ void __launch_bounds__(256)
k_init_levels(int64_t n, const double *__restrict__ a, const double *__restrict__ j, double eta_start, int k_min,
              int k_max, int64_t *__restrict__ t_tick, int32_t *__restrict__ level)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double am = norm3(a[i], a[n + i], a[2 * n + i]);
    const double jm = norm3(j[i], j[n + i], j[2 * n + i]);
    level[i] = level_for(eta_start * am / jm, k_min, k_max);
    t_tick[i] = 0;
}

// --------------------------------------------------------------------------
// Scheduler.  Pass 1: per block, the minimum of t_i + dt_i and how many of
// its particles reach it.  Pass 2 (one block): t_next = the least block
// minimum; exclusive scan of the counts of the blocks whose minimum is t_next
// (the others have no active particle), n_act.  Pass 3: each block writes its
// active indices in increasing order at its offset.
__device__ __forceinline__ int64_t next_time(const int64_t *t_tick, const int32_t *level, int64_t i)
{
    return t_tick[i] + (int64_t(1) << (kLevelMax - level[i]));
}

// (minimum, count at the minimum) of two partial results
__device__ __forceinline__ void min_count(int64_t &m, int &c, int64_t m2, int c2)
{
    if (m2 < m) {
        m = m2;
        c = c2;
    } else if (m2 == m) {
        c += c2;
    }
}

__global__ void __launch_bounds__(kSchedBlock)
k_sched_min(int64_t n, const int64_t *__restrict__ t_tick, const int32_t *__restrict__ level,
            int64_t *__restrict__ bmin, int32_t *__restrict__ bcnt)
{
    __shared__ int64_t sm[kSchedBlock];
    __shared__ int sc[kSchedBlock];
    const int64_t base = int64_t(blockIdx.x) * kSchedChunk;
    int64_t mn = INT64_MAX;
    int c = 0;
#pragma unroll
    for (int k = 0; k < kSchedPerThread; ++k) {
        const int64_t i = base + int64_t(k) * kSchedBlock + threadIdx.x;
        if (i < n) min_count(mn, c, next_time(t_tick, level, i), 1);
    }
    sm[threadIdx.x] = mn;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int s = kSchedBlock / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) {
            int64_t m = sm[threadIdx.x];
            int cc = sc[threadIdx.x];
            min_count(m, cc, sm[threadIdx.x + s], sc[threadIdx.x + s]);
            sm[threadIdx.x] = m;
            sc[threadIdx.x] = cc;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bmin[blockIdx.x] = sm[0];
        bcnt[blockIdx.x] = sc[0];
    }
}

__global__ void __launch_bounds__(kSchedBlock)
k_sched_scan(const int64_t *__restrict__ bmin, const int32_t *__restrict__ bcnt, int nb,
             int64_t *__restrict__ boff, DevScalars *__restrict__ sc, HostScalars *__restrict__ pub, int64_t seq)
{
    // one block: t_next from the block minima, then sequential chunks of
    // kSchedBlock counts scanned in LDS
    __shared__ int64_t s[kSchedBlock];
    int64_t mn = INT64_MAX;
    for (int b = threadIdx.x; b < nb; b += kSchedBlock) mn = bmin[b] < mn ? bmin[b] : mn;
    s[threadIdx.x] = mn;
    __syncthreads();
    for (int o = kSchedBlock / 2; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o) s[threadIdx.x] = s[threadIdx.x + o] < s[threadIdx.x] ? s[threadIdx.x + o] : s[threadIdx.x];
        __syncthreads();
    }
    const int64_t tn = s[0];
    __syncthreads();
    int64_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += kSchedBlock) {
        const int b = b0 + threadIdx.x;
        const int64_t v = (b < nb && bmin[b] == tn) ? bcnt[b] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kSchedBlock; o <<= 1) {
            const int64_t add = int(threadIdx.x) >= o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (b < nb) boff[b] = carry + s[threadIdx.x] - v;
        carry += s[kSchedBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sc->t_next = tn;
        sc->n_act = carry;
        if (pub) {
            // the fields first, then (after a system-scope fence) the
            // sequence number the host waits for
            pub->t_next = tn;
            pub->n_act = carry;
            pub->underflow = sc->underflow;
            pub->nonfinite = sc->nonfinite;
            __threadfence_system();
            __hip_atomic_store(&pub->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

__global__ void __launch_bounds__(kSchedBlock)
k_sched_compact(int64_t n, const int64_t *__restrict__ t_tick, const int32_t *__restrict__ level,
                const int64_t *__restrict__ boff, const DevScalars *__restrict__ sc, int32_t *__restrict__ act)
{
    __shared__ int s[kSchedBlock];
    const int64_t tn = sc->t_next;
    const int64_t base = int64_t(blockIdx.x) * kSchedChunk + int64_t(threadIdx.x) * kSchedPerThread;
    int flags[kSchedPerThread];
    int c = 0;
#pragma unroll
    for (int k = 0; k < kSchedPerThread; ++k) {
        const int64_t i = base + k;
        flags[k] = (i < n && next_time(t_tick, level, i) == tn) ? 1 : 0;
        c += flags[k];
    }
    s[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < kSchedBlock; o <<= 1) {
        const int add = int(threadIdx.x) >= o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t pos = boff[blockIdx.x] + s[threadIdx.x] - c;
#pragma unroll
    for (int k = 0; k < kSchedPerThread; ++k)
        if (flags[k]) act[pos++] = int32_t(base + k);
}

// --------------------------------------------------------------------------
// FP64 energy: per block, sum over its i of m_i v_i^2 and of
// m_i sum_{j != i} m_j / sqrt(r_ij^2 + eps_ij^2); fixed-order tree in LDS.
__global__ void __launch_bounds__(256)
k_energy(int64_t n, int64_t stride, int64_t n_hard, double eps2, const double *__restrict__ m, const double *__restrict__ x,
         const double *__restrict__ v, double *__restrict__ partial)
{
    __shared__ double sk[256], sw[256];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t ii = i < n ? i : n - 1;
    const double xi = x[ii], yi = x[stride + ii], zi = x[2 * stride + ii];
    double w = 0.0;
    const int64_t jh = n_hard < n ? n_hard : n;
    for (int64_t j = 0; j < jh; ++j) {
        const double dx = x[j] - xi, dy = x[stride + j] - yi, dz = x[2 * stride + j] - zi;
        const double e = ii < n_hard ? 0.0 : eps2;
        double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, e)));
        const bool ok = j != ii;
        r2 = ok ? r2 : 1.0;
        w += ok ? m[j] * rsqrt64(r2) : 0.0;
    }
    for (int64_t j = jh; j < n; ++j) {
        const double dx = x[j] - xi, dy = x[stride + j] - yi, dz = x[2 * stride + j] - zi;
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        w += m[j] * rsqrt64(r2);
    }
    if (ii >= jh) w -= m[ii] * rsqrt64(eps2);   // self pair of the softened loop
    const double vx = v[ii], vy = v[stride + ii], vz = v[2 * stride + ii];
    sk[threadIdx.x] = i < n ? m[ii] * __builtin_fma(vx, vx, __builtin_fma(vy, vy, vz * vz)) : 0.0;
    sw[threadIdx.x] = i < n ? m[ii] * w : 0.0;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) {
            sk[threadIdx.x] += sk[threadIdx.x + s];
            sw[threadIdx.x] += sw[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = 0.5 * sk[0];
        partial[2 * blockIdx.x + 1] = -0.5 * sw[0];
    }
}

__global__ void k_iota(int64_t n, int32_t *__restrict__ a)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) a[i] = int32_t(i);
}

__global__ void k_fill(int64_t n, double *__restrict__ a, double val)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) a[i] = val;
}

unsigned blocks_for(int64_t n, int b) { return unsigned((n + b - 1) / b); }

template <int P>
hipError_t predict_p(int precision, int64_t n, const nbody_state &st, int64_t t, void *rec, hipStream_t s)
{
    const unsigned g = blocks_for(n, 256);
#define NB_PRED(PREC)                                                                                           \
    hipLaunchKernelGGL((k_predict<P, PREC>), dim3(g), dim3(256), 0, s, n, st.m, st.x, st.v, st.d[0], st.d[1],  \
                       st.d[2], st.d[3], st.d[4], st.d[5], st.t_tick, t, rec)
    if (precision == NBODY_MIXED) NB_PRED(NBODY_MIXED);
    else if (precision == NBODY_DS) NB_PRED(NBODY_DS);
    else NB_PRED(NBODY_FP64);
#undef NB_PRED
    return hipGetLastError();
}

}  // namespace

hipError_t launch_predict(int order, int precision, int64_t n, const nbody_state &st, int64_t t_tick, void *rec,
                          hipStream_t s)
{
    if (order == 4) return predict_p<4>(precision, n, st, t_tick, rec, s);
    if (order == 6) return predict_p<6>(precision, n, st, t_tick, rec, s);
    return predict_p<8>(precision, n, st, t_tick, rec, s);
}

hipError_t launch_unpack(int order, int precision, int64_t n, const void *rec, double *xp, double *vp, double *ap,
                         double *jp, hipStream_t s)
{
    const unsigned g = blocks_for(n, 256);
#define NB_UNP(P, PREC) hipLaunchKernelGGL((k_unpack<P, PREC>), dim3(g), dim3(256), 0, s, n, rec, xp, vp, ap, jp)
#define NB_UNP_P(P)                                                   \
    if (precision == NBODY_MIXED) NB_UNP(P, NBODY_MIXED);             \
    else if (precision == NBODY_DS) NB_UNP(P, NBODY_DS);              \
    else NB_UNP(P, NBODY_FP64)
    if (order == 4) { NB_UNP_P(4); }
    else if (order == 6) { NB_UNP_P(6); }
    else { NB_UNP_P(8); }
#undef NB_UNP_P
#undef NB_UNP
    return hipGetLastError();
}

hipError_t launch_pack_f64(int64_t n, const double *m, const double *x, const double *v, const double *a,
                           const double *j, void *rec, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_f64, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, m, x, v, a, j,
                       static_cast<RecF64<8> *>(rec));
    return hipGetLastError();
}

hipError_t launch_correct(const nbody_config &c, const nbody_state &st, int64_t n_act, const int32_t *act,
                          const DevScalars *src, int64_t t_tick_host, const double *const f[4],
                          DevScalars *sc, hipStream_t s)
{
    const unsigned g = blocks_for(n_act, 256);   // n_act: exact, or an upper bound when src is set
    if (g == 0) return hipSuccess;
#define NB_CORR(P)                                                                                             \
    hipLaunchKernelGGL((k_correct<P>), dim3(g), dim3(256), 0, s, c.n, n_act, act, src, t_tick_host,            \
                       st.x, st.v, st.d[0], st.d[1], st.d[2], st.d[3], st.d[4], st.d[5], st.t_tick, st.level, \
                       f[0], f[1], f[2], f[3], c.eta, dt_rule_of(c), int(c.k_min), int(c.k_max), sc)
    if (c.order == 4) NB_CORR(4);
    else if (c.order == 6) NB_CORR(6);
    else NB_CORR(8);
#undef NB_CORR
    return hipGetLastError();
}

hipError_t launch_schedule(int64_t n, const int64_t *t_tick, const int32_t *level, void *scratch,
                           int32_t *act_out, DevScalars *sc, HostScalars *pub, int64_t seq, hipStream_t s)
{
    const int nb = int((n + kSchedChunk - 1) / kSchedChunk);
    int64_t *bmin = static_cast<int64_t *>(scratch);
    int64_t *boff = bmin + nb;
    int32_t *bcnt = reinterpret_cast<int32_t *>(boff + nb);
    hipLaunchKernelGGL(k_sched_min, dim3(nb), dim3(kSchedBlock), 0, s, n, t_tick, level, bmin, bcnt);
    hipLaunchKernelGGL(k_sched_scan, dim3(1), dim3(kSchedBlock), 0, s, bmin, bcnt, nb, boff, sc, pub, seq);
    hipLaunchKernelGGL(k_sched_compact, dim3(nb), dim3(kSchedBlock), 0, s, n, t_tick, level, boff, sc, act_out);
    return hipGetLastError();
}

hipError_t launch_init_levels(const nbody_config &c, const nbody_state &st, const double *a, const double *j,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_init_levels, dim3(blocks_for(c.n, 256)), dim3(256), 0, s, c.n, a, j, c.eta_start,
                       int(c.k_min), int(c.k_max), st.t_tick, st.level);
    if (c.order == 8) {
        hipLaunchKernelGGL(k_fill, dim3(blocks_for(3 * c.n, 256)), dim3(256), 0, s, 3 * c.n, st.d[4], 0.0);
        hipLaunchKernelGGL(k_fill, dim3(blocks_for(3 * c.n, 256)), dim3(256), 0, s, 3 * c.n, st.d[5], 0.0);
    }
    return hipGetLastError();
}

hipError_t launch_iota(int64_t n, int32_t *a, hipStream_t s)
{
    hipLaunchKernelGGL(k_iota, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, a);
    return hipGetLastError();
}

hipError_t launch_energy(int64_t n, int64_t stride, int64_t n_hard, double eps2, const double *m, const double *x,
                         const double *v, double *partials, int *n_partials, hipStream_t s)
{
    const unsigned g = blocks_for(n, 256);
    *n_partials = int(g);
    hipLaunchKernelGGL(k_energy, dim3(g), dim3(256), 0, s, n, stride, n_hard, eps2, m, x, v, partials);
    return hipGetLastError();
}

}  // namespace nb
