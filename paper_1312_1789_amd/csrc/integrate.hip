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
// Scheduler.  Pass 1: per block of kSchedChunk particles, the minimum of
// t_i + dt_i and how many of its particles reach it.  With at most
// kSchedOwnOffsets blocks, pass 2 is the compaction itself: every block takes
// t_next as the least block minimum and its output offset as the number of
// particles at t_next in the blocks before it (block 0 also publishes t_next
// and n_act), then writes its active indices in increasing order.  With more
// blocks a one-block kernel computes t_next and the offsets first.
constexpr int kSchedWaves = kSchedBlock / 64;
constexpr int kSchedOwnOffsets = 1024;   // blocks (n <= 2^20) for which each block finds its own offset

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

__device__ __forceinline__ int64_t wave_min(int64_t m)
{
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t t = __shfl_xor(m, o, 64);
        m = t < m ? t : m;
    }
    return m;
}

__device__ __forceinline__ int64_t wave_sum(int64_t v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive prefix of c over the block's threads in thread order (wave
// scans, then the wave totals through LDS).  Synchronises the block.
__device__ __forceinline__ int block_excl_scan(int c, int *wsum)
{
    const int lane = int(threadIdx.x) & 63, w = int(threadIdx.x) >> 6;
    int incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int before = 0;
    for (int k = 0; k < w; ++k) before += wsum[k];
    return before + incl - c;
}

// The step's t_next and n_act into the device scalars and, when given, the
// pinned host copy: the fields first, then (after a system-scope fence) the
// sequence number the host waits for.
__device__ __forceinline__ void publish(DevScalars *sc, HostScalars *pub, int64_t seq, int64_t tn, int64_t n_act)
{
    sc->t_next = tn;
    sc->n_act = n_act;
    if (pub) {
        pub->t_next = tn;
        pub->n_act = n_act;
        pub->underflow = sc->underflow;
        pub->nonfinite = sc->nonfinite;
        __threadfence_system();
        __hip_atomic_store(&pub->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__global__ void __launch_bounds__(kSchedBlock)
k_sched_min(int64_t n, const int64_t *__restrict__ t_tick, const int32_t *__restrict__ level,
            int64_t *__restrict__ bmin, int32_t *__restrict__ bcnt)
{
    __shared__ int64_t wm[kSchedWaves];
    __shared__ int wc[kSchedWaves];
    const int64_t base = int64_t(blockIdx.x) * kSchedChunk;
    int64_t mn = INT64_MAX;
    int c = 0;
#pragma unroll
    for (int k = 0; k < kSchedPerThread; ++k) {
        const int64_t i = base + int64_t(k) * kSchedBlock + threadIdx.x;
        if (i < n) min_count(mn, c, next_time(t_tick, level, i), 1);
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t m2 = __shfl_xor(mn, o, 64);
        const int c2 = __shfl_xor(c, o, 64);
        min_count(mn, c, m2, c2);
    }
    if ((threadIdx.x & 63) == 0) {
        wm[threadIdx.x >> 6] = mn;
        wc[threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kSchedWaves; ++k) min_count(mn, c, wm[k], wc[k]);
        bmin[blockIdx.x] = mn;
        bcnt[blockIdx.x] = c;
    }
}

// This block's particles at t_next written from act[off] on, in increasing
// index order (each thread takes kSchedPerThread consecutive particles).
__device__ __forceinline__ void compact_block(int64_t n, const int64_t *__restrict__ t_tick,
                                              const int32_t *__restrict__ level, int64_t tn, int64_t off,
                                              int *wsum, int32_t *__restrict__ act)
{
    const int64_t base = int64_t(blockIdx.x) * kSchedChunk + int64_t(threadIdx.x) * kSchedPerThread;
    int flags[kSchedPerThread];
    int c = 0;
#pragma unroll
    for (int k = 0; k < kSchedPerThread; ++k) {
        const int64_t i = base + k;
        flags[k] = (i < n && next_time(t_tick, level, i) == tn) ? 1 : 0;
        c += flags[k];
    }
    int64_t pos = off + block_excl_scan(c, wsum);
#pragma unroll
    for (int k = 0; k < kSchedPerThread; ++k)
        if (flags[k] && pos < n) act[pos++] = int32_t(base + k);
}

__global__ void __launch_bounds__(kSchedBlock)
k_sched_compact_own(int64_t n, const int64_t *__restrict__ t_tick, const int32_t *__restrict__ level,
                    const int64_t *__restrict__ bmin, const int32_t *__restrict__ bcnt, int nb,
                    DevScalars *__restrict__ sc, HostScalars *__restrict__ pub, int64_t seq,
                    int32_t *__restrict__ act)
{
    __shared__ int64_t wm[kSchedWaves], wo[kSchedWaves], wt[kSchedWaves];
    __shared__ int wsum[kSchedWaves];
    const int lane = int(threadIdx.x) & 63, w = int(threadIdx.x) >> 6;
    int64_t mn = INT64_MAX;
    for (int b = threadIdx.x; b < nb; b += kSchedBlock) mn = bmin[b] < mn ? bmin[b] : mn;
    mn = wave_min(mn);
    if (lane == 0) wm[w] = mn;
    __syncthreads();
    int64_t tn = wm[0];
    for (int k = 1; k < kSchedWaves; ++k) tn = wm[k] < tn ? wm[k] : tn;
    // particles at t_next in the blocks before this one, and in all blocks
    int64_t off = 0, tot = 0;
    for (int b = threadIdx.x; b < nb; b += kSchedBlock) {
        const int64_t v = bmin[b] == tn ? bcnt[b] : 0;
        tot += v;
        if (b < int(blockIdx.x)) off += v;
    }
    off = wave_sum(off);
    tot = wave_sum(tot);
    if (lane == 0) {
        wo[w] = off;
        wt[w] = tot;
    }
    __syncthreads();
    off = 0;
    tot = 0;
    for (int k = 0; k < kSchedWaves; ++k) {
        off += wo[k];
        tot += wt[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) publish(sc, pub, seq, tn, tot);
    compact_block(n, t_tick, level, tn, off, wsum, act);
}

__global__ void __launch_bounds__(kSchedBlock)
k_sched_scan(const int64_t *__restrict__ bmin, const int32_t *__restrict__ bcnt, int nb,
             int64_t *__restrict__ boff, DevScalars *__restrict__ sc, HostScalars *__restrict__ pub, int64_t seq)
{
    // one block: t_next from the block minima, then sequential chunks of
    // kSchedBlock counts scanned with wave scans
    __shared__ int64_t wm[kSchedWaves];
    __shared__ int wsum[kSchedWaves];
    const int lane = int(threadIdx.x) & 63, w = int(threadIdx.x) >> 6;
    int64_t mn = INT64_MAX;
    for (int b = threadIdx.x; b < nb; b += kSchedBlock) mn = bmin[b] < mn ? bmin[b] : mn;
    mn = wave_min(mn);
    if (lane == 0) wm[w] = mn;
    __syncthreads();
    int64_t tn = wm[0];
    for (int k = 1; k < kSchedWaves; ++k) tn = wm[k] < tn ? wm[k] : tn;
    int64_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += kSchedBlock) {
        const int b = b0 + threadIdx.x;
        const int v = (b < nb && bmin[b] == tn) ? bcnt[b] : 0;   // <= kSchedChunk
        const int ex = block_excl_scan(v, wsum);
        if (b < nb) boff[b] = carry + ex;
        int chunk = 0;
        for (int k = 0; k < kSchedWaves; ++k) chunk += wsum[k];
        carry += chunk;
        __syncthreads();   // wsum is rewritten by the next chunk
    }
    if (threadIdx.x == 0) publish(sc, pub, seq, tn, carry);
}

__global__ void __launch_bounds__(kSchedBlock)
k_sched_compact(int64_t n, const int64_t *__restrict__ t_tick, const int32_t *__restrict__ level,
                const int64_t *__restrict__ boff, const DevScalars *__restrict__ sc, int32_t *__restrict__ act)
{
    __shared__ int wsum[kSchedWaves];
    compact_block(n, t_tick, level, sc->t_next, boff[blockIdx.x], wsum, act);
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
    if (nb <= kSchedOwnOffsets) {
        hipLaunchKernelGGL(k_sched_compact_own, dim3(nb), dim3(kSchedBlock), 0, s, n, t_tick, level, bmin, bcnt, nb,
                           sc, pub, seq, act_out);
    } else {
        hipLaunchKernelGGL(k_sched_scan, dim3(1), dim3(kSchedBlock), 0, s, bmin, bcnt, nb, boff, sc, pub, seq);
        hipLaunchKernelGGL(k_sched_compact, dim3(nb), dim3(kSchedBlock), 0, s, n, t_tick, level, boff, sc,
                           act_out);
    }
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
