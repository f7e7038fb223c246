// force.hip -- the O(n_act * n) pairwise force kernels (acceleration, jerk,
// snap, crackle, potential) for gfx950, in FP64, MIXED and DS arithmetic.
//
// Direct summation of softened gravity over all j != i (paper: Abstract,
// where correlations between distant particles rule out approximations), with
// the time derivatives a Hermite scheme of order 4, 6 or 8 needs (paper:
// Sec. "Codes description").  Derivative recursion: Nitadori & Makino (2008).
//
// Launch shape: grid (i-tiles, j-splits).  A lane holds NI active particles
// in registers; the block's lanes walk the same j range, so every j record is
// read with a wave-uniform address into SGPRs and feeds the VALU directly
// (no LDS staging, no per-lane j traffic).  With one split the kernel writes
// the final FP64 sums; with several, each split writes its partial sums and a
// second kernel adds them in split order (deterministic).
#include "internal.h"
#include "records.h"

namespace nb {
namespace {

// --------------------------------------------------------------------------
// Accumulator layout: 0-2 acceleration, 3-5 jerk, 6-8 snap, 9-11 crackle,
// 12 sum of m_j / sqrt(f) (the potential is its negative).
constexpr int kPot = 12;

__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// One interaction, given the differences (j minus i) d = position, w =
// velocity, e = acceleration, f = jerk, mr = m_j / sqrt(r^2 + eps^2),
// rinv2 = 1 / (r^2 + eps^2).  With mu = m_j / (r^2+eps^2)^(3/2),
// alpha = d.w / f2, beta = (w.w + d.e) / f2 + alpha^2,
// gamma = (3 w.e + d.f) / f2 + alpha (3 beta - 4 alpha^2), the terms
//   A = mu d, J = mu w - 3 alpha A, S = mu e - 6 alpha J - 3 beta A,
//   C = mu f - 9 alpha S - 9 beta J - 3 gamma A
// are expanded into linear combinations of d, w, e, f and added with FMAs.
template <int P, class T>
__device__ __forceinline__ void core_fma(T dx, T dy, T dz, T wx, T wy, T wz, T ex, T ey, T ez, T fx, T fy, T fz,
                                         T mr, T rinv2, T *A)
{
    const T mu = mr * rinv2;
    A[kPot] += mr;
    A[0] = fmad(mu, dx, A[0]);
    A[1] = fmad(mu, dy, A[1]);
    A[2] = fmad(mu, dz, A[2]);
    const T al = fmad(dx, wx, fmad(dy, wy, dz * wz)) * rinv2;
    const T cj = T(-3) * al * mu;
    A[3] = fmad(mu, wx, fmad(cj, dx, A[3]));
    A[4] = fmad(mu, wy, fmad(cj, dy, A[4]));
    A[5] = fmad(mu, wz, fmad(cj, dz, A[5]));
    if constexpr (P >= 6) {
        const T s = fmad(wx, wx, fmad(wy, wy, fmad(wz, wz,
                    fmad(dx, ex, fmad(dy, ey, dz * ez)))));
        const T be = fmad(s, rinv2, al * al);
        const T cs1 = T(2) * cj;
        const T cs2 = fmad(T(18) * al, al, T(-3) * be) * mu;
        A[6] = fmad(mu, ex, fmad(cs1, wx, fmad(cs2, dx, A[6])));
        A[7] = fmad(mu, ey, fmad(cs1, wy, fmad(cs2, dy, A[7])));
        A[8] = fmad(mu, ez, fmad(cs1, wz, fmad(cs2, dz, A[8])));
        if constexpr (P >= 8) {
            const T t = fmad(T(3), fmad(wx, ex, fmad(wy, ey, wz * ez)),
                                      fmad(dx, fx, fmad(dy, fy, dz * fz)));
            const T ga = fmad(t, rinv2, al * fmad(T(3), be, T(-4) * al * al));
            const T c1 = T(-9) * al * mu;
            const T c2 = T(-9) * fmad(al, cs1, be * mu);
            const T c3 = fmad(T(-9), fmad(al, cs2, be * cj), T(-3) * ga * mu);
            A[9] = fmad(mu, fx, fmad(c1, ex, fmad(c2, wx, fmad(c3, dx, A[9]))));
            A[10] = fmad(mu, fy, fmad(c1, ey, fmad(c2, wy, fmad(c3, dy, A[10]))));
            A[11] = fmad(mu, fz, fmad(c1, ez, fmad(c2, wz, fmad(c3, dz, A[11]))));
        }
    }
    (void)ex; (void)ey; (void)ez; (void)fx; (void)fy; (void)fz;
}

// --------------------------------------------------------------------------
// FP64 policy.
template <int P> struct PolF64 {
    using Rec = RecF64<P>;
    using Part = double;                 // accumulate straight into FP64
    static constexpr int kChunk = 0;
    struct I { double x, y, z, vx, vy, vz, ax, ay, az, jx, jy, jz; };

    __device__ static I load(const Rec &r)
    {
        I i{};
        i.x = r.x; i.y = r.y; i.z = r.z; i.vx = r.vx; i.vy = r.vy; i.vz = r.vz;
        if constexpr (P >= 6) { i.ax = r.ax; i.ay = r.ay; i.az = r.az; }
        if constexpr (P >= 8) { i.jx = r.jx; i.jy = r.jy; i.jz = r.jz; }
        return i;
    }
    template <bool MASK>
    __device__ static void pair(const I &i, const Rec &j, double eps2, bool valid, double *A)
    {
        const double dx = j.x - i.x, dy = j.y - i.y, dz = j.z - i.z;
        const double wx = j.vx - i.vx, wy = j.vy - i.vy, wz = j.vz - i.vz;
        double ex = 0, ey = 0, ez = 0, fx = 0, fy = 0, fz = 0;
        if constexpr (P >= 6) { ex = j.ax - i.ax; ey = j.ay - i.ay; ez = j.az - i.az; }
        if constexpr (P >= 8) { fx = j.jx - i.jx; fy = j.jy - i.jy; fz = j.jz - i.jz; }
        double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
        if (MASK) r2 = valid ? r2 : 1.0;
        const double rinv = rsqrt64(r2);
        double mr = j.m * rinv;
        if (MASK) mr = valid ? mr : 0.0;
        core_fma<P, double>(dx, dy, dz, wx, wy, wz, ex, ey, ez, fx, fy, fz, mr, rinv * rinv, A);
    }
    __device__ static double self_pot(const Rec &r, double eps2) { return r.m * rsqrt64(eps2); }
};

// MIXED policy: FP64 differences of position and velocity rounded to FP32,
// FP32 acceleration / jerk differences, FP32 rsqrt and arithmetic, FP32
// partial sums over chunks of kMixedChunk j, added into FP64.
template <int P> struct PolMx {
    using Rec = RecMx<P>;
    using Part = float;
    static constexpr int kChunk = kMixedChunk;
    struct I { double x, y, z, vx, vy, vz; float ax, ay, az, jx, jy, jz; };

    __device__ static I load(const Rec &r)
    {
        I i{};
        i.x = r.x; i.y = r.y; i.z = r.z; i.vx = r.vx; i.vy = r.vy; i.vz = r.vz;
        if constexpr (P >= 6) { i.ax = r.ax; i.ay = r.ay; i.az = r.az; }
        if constexpr (P >= 8) { i.jx = r.jx; i.jy = r.jy; i.jz = r.jz; }
        return i;
    }
    template <bool MASK>
    __device__ static void pair(const I &i, const Rec &j, float eps2, bool valid, float *A)
    {
        const float dx = float(j.x - i.x), dy = float(j.y - i.y), dz = float(j.z - i.z);
        const float wx = float(j.vx - i.vx), wy = float(j.vy - i.vy), wz = float(j.vz - i.vz);
        float ex = 0, ey = 0, ez = 0, fx = 0, fy = 0, fz = 0;
        if constexpr (P >= 6) { ex = j.ax - i.ax; ey = j.ay - i.ay; ez = j.az - i.az; }
        if constexpr (P >= 8) { fx = j.jx - i.jx; fy = j.jy - i.jy; fz = j.jz - i.jz; }
        float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
        if (MASK) r2 = valid ? r2 : 1.0f;
        const float rinv = __builtin_amdgcn_rsqf(r2);
        float mr = j.m * rinv;
        if (MASK) mr = valid ? mr : 0.0f;
        core_fma<P, float>(dx, dy, dz, wx, wy, wz, ex, ey, ez, fx, fy, fz, mr, rinv * rinv, A);
    }
    __device__ static double self_pot(const Rec &r, double eps2)
    {
        const float e2 = float(eps2);
        return double(r.m * __builtin_amdgcn_rsqf(e2));
    }
};

// DS policy: no FP64 instruction in the j loop.  Differences of
// double-single values: (hi_j - hi_i) + (lo_j - lo_i), whose rounding error
// is relative to the difference itself; every term is added into a (hi, lo)
// pair with the error-free two-sum of Knuth.
struct DS { float hi, lo; };

__device__ __forceinline__ void two_sum_add(DS &s, float t)
{
    const float a = s.hi;
    const float sum = a + t;
    const float bv = sum - a;
    const float av = sum - bv;
    const float err = (a - av) + (t - bv);
    s.hi = sum;
    s.lo += err;
}

template <int P> struct PolDS {
    using Rec = RecDS<P>;
    using Part = DS;
    static constexpr int kChunk = 0;
    struct I { float xh, yh, zh, xl, yl, zl, vxh, vyh, vzh, vxl, vyl, vzl, ax, ay, az, jx, jy, jz; };

    __device__ static I load(const Rec &r)
    {
        I i{};
        i.xh = r.xh; i.yh = r.yh; i.zh = r.zh; i.xl = r.xl; i.yl = r.yl; i.zl = r.zl;
        i.vxh = r.vxh; i.vyh = r.vyh; i.vzh = r.vzh; i.vxl = r.vxl; i.vyl = r.vyl; i.vzl = r.vzl;
        if constexpr (P >= 6) { i.ax = r.ax; i.ay = r.ay; i.az = r.az; }
        if constexpr (P >= 8) { i.jx = r.jx; i.jy = r.jy; i.jz = r.jz; }
        return i;
    }
    template <bool MASK>
    __device__ static void pair(const I &i, const Rec &j, float eps2, bool valid, DS *A)
    {
        const float dx = (j.xh - i.xh) + (j.xl - i.xl);
        const float dy = (j.yh - i.yh) + (j.yl - i.yl);
        const float dz = (j.zh - i.zh) + (j.zl - i.zl);
        const float wx = (j.vxh - i.vxh) + (j.vxl - i.vxl);
        const float wy = (j.vyh - i.vyh) + (j.vyl - i.vyl);
        const float wz = (j.vzh - i.vzh) + (j.vzl - i.vzl);
        float ex = 0, ey = 0, ez = 0, fx = 0, fy = 0, fz = 0;
        if constexpr (P >= 6) { ex = j.ax - i.ax; ey = j.ay - i.ay; ez = j.az - i.az; }
        if constexpr (P >= 8) { fx = j.jx - i.jx; fy = j.jy - i.jy; fz = j.jz - i.jz; }
        float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
        if (MASK) r2 = valid ? r2 : 1.0f;
        const float rinv = __builtin_amdgcn_rsqf(r2);
        float mr = j.m * rinv;
        if (MASK) mr = valid ? mr : 0.0f;
        // explicit terms (FMA-fused accumulation would hide the rounding the
        // two-sum must capture)
        float T[13];
#pragma unroll
        for (int c = 0; c < 13; ++c) T[c] = 0.0f;
        core_fma<P, float>(dx, dy, dz, wx, wy, wz, ex, ey, ez, fx, fy, fz, mr, rinv * rinv, T);
        constexpr int nv = 3 * (P / 2);
#pragma unroll
        for (int c = 0; c < nv; ++c) two_sum_add(A[c], T[c]);
        two_sum_add(A[kPot], T[kPot]);
    }
    __device__ static double self_pot(const Rec &r, double eps2)
    {
        const float e2 = float(eps2);
        return double(r.m * __builtin_amdgcn_rsqf(e2));
    }
};

template <class Part> __device__ __forceinline__ void zero_part(Part &p) { p = Part(0); }
template <> __device__ __forceinline__ void zero_part<DS>(DS &p) { p.hi = 0.0f; p.lo = 0.0f; }
__device__ __forceinline__ double to_double(double v) { return v; }
__device__ __forceinline__ double to_double(float v) { return double(v); }
__device__ __forceinline__ double to_double(const DS &v) { return double(v.hi) + double(v.lo); }

template <class Pol> struct EpsT { using type = float; };
template <> struct EpsT<PolF64<4>> { using type = double; };
template <> struct EpsT<PolF64<6>> { using type = double; };
template <> struct EpsT<PolF64<8>> { using type = double; };

// --------------------------------------------------------------------------
// The force kernel.  blockIdx.x: i-tile of blockDim.x * NI active particles;
// blockIdx.y: j-split [split * j_chunk, min(n, (split+1) * j_chunk)).
// Pairs with both indices below n_hard are unsoftened and the self pair is
// masked there; above n_hard the self pair is evaluated with eps2 > 0 (its
// acceleration and derivatives are exactly zero, since every difference is)
// and its potential term is removed after the loop.
template <class Pol, int P, int NI>
__global__ void __launch_bounds__(256)
k_force(const typename Pol::Rec *__restrict__ rec, int64_t n, const int32_t *__restrict__ act, int64_t n_act,
        double eps2, int64_t n_hard, int64_t j_chunk, int n_split, double *__restrict__ o_acc,
        double *__restrict__ o_jrk, double *__restrict__ o_snp, double *__restrict__ o_crk,
        double *__restrict__ o_pot, double *__restrict__ part)
{
    using Rec = typename Pol::Rec;
    using Part = typename Pol::Part;
    using ET = typename EpsT<Pol>::type;
    constexpr int NV = 3 * (P / 2);
    const ET e2 = ET(eps2);

    const int64_t tile0 = int64_t(blockIdx.x) * blockDim.x * NI + threadIdx.x;
    const int split = blockIdx.y;
    const int64_t j0 = int64_t(split) * j_chunk;
    const int64_t j1 = (j0 + j_chunk < n) ? j0 + j_chunk : n;

    typename Pol::I ip[NI];
    int64_t iidx[NI];
    double acc[NI][13];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        int64_t q = tile0 + int64_t(k) * blockDim.x;
        if (q >= n_act) q = n_act - 1;  // padding lanes recompute the last row; never stored
        const int64_t ia = act[q];
        iidx[k] = (ia >= 0 && ia < n) ? ia : 0;   // an index outside [0, n) yields an undefined row, never a fault
        ip[k] = Pol::load(rec[iidx[k]]);
#pragma unroll
        for (int c = 0; c < 13; ++c) acc[k][c] = 0.0;
    }

    // unsoftened block: j < n_hard, per-lane softening and self mask
    const int64_t jh1 = (j1 < n_hard) ? j1 : n_hard;
    for (int64_t j = j0; j < jh1; ++j) {
        const Rec rj = rec[j];
        Part p[NI][13];
#pragma unroll
        for (int k = 0; k < NI; ++k) {
#pragma unroll
            for (int c = 0; c < 13; ++c) zero_part(p[k][c]);
            const ET el = (iidx[k] < n_hard) ? ET(0) : e2;
            Pol::template pair<true>(ip[k], rj, el, j != iidx[k], p[k]);
#pragma unroll
            for (int c = 0; c < 13; ++c) acc[k][c] += to_double(p[k][c]);
        }
    }

    // softened bulk
    const int64_t js0 = (j0 > n_hard) ? j0 : n_hard;
    if constexpr (Pol::kChunk == 0) {
        Part p[NI][13];
#pragma unroll
        for (int k = 0; k < NI; ++k)
#pragma unroll
            for (int c = 0; c < 13; ++c) zero_part(p[k][c]);
#pragma unroll 2
        for (int64_t j = js0; j < j1; ++j) {
            const Rec rj = rec[j];
#pragma unroll
            for (int k = 0; k < NI; ++k) Pol::template pair<false>(ip[k], rj, e2, true, p[k]);
        }
#pragma unroll
        for (int k = 0; k < NI; ++k)
#pragma unroll
            for (int c = 0; c < 13; ++c) acc[k][c] += to_double(p[k][c]);
    } else {
        for (int64_t jc = js0; jc < j1; jc += Pol::kChunk) {
            const int64_t je = (jc + Pol::kChunk < j1) ? jc + Pol::kChunk : j1;
            Part p[NI][13];
#pragma unroll
            for (int k = 0; k < NI; ++k)
#pragma unroll
                for (int c = 0; c < 13; ++c) zero_part(p[k][c]);
#pragma unroll 2
            for (int64_t j = jc; j < je; ++j) {
                const Rec rj = rec[j];
#pragma unroll
                for (int k = 0; k < NI; ++k) Pol::template pair<false>(ip[k], rj, e2, true, p[k]);
            }
#pragma unroll
            for (int k = 0; k < NI; ++k)
#pragma unroll
                for (int c = 0; c < 13; ++c) acc[k][c] += to_double(p[k][c]);
        }
    }

#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int64_t q = tile0 + int64_t(k) * blockDim.x;
        if (q >= n_act) continue;
        const int64_t i = iidx[k];
        double pot = acc[k][kPot];
        if (i >= js0 && i < j1) pot -= Pol::self_pot(rec[i], eps2);  // self pair was in the bulk loop
        if (n_split == 1) {
            double *outs[4] = {o_acc, o_jrk, o_snp, o_crk};
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                double *o = outs[c / 3];
                if (o) o[(c % 3) * n_act + q] = acc[k][c];
            }
            if (o_pot) o_pot[q] = -pot;
        } else {
            constexpr int NC = NV + 1;
            double *base = part + int64_t(split) * NC * n_act;
#pragma unroll
            for (int c = 0; c < NV; ++c) base[int64_t(c) * n_act + q] = acc[k][c];
            base[int64_t(NV) * n_act + q] = -pot;
        }
    }
}

// Sum of the j-split partial results in split order.
template <int P>
__global__ void __launch_bounds__(256)
k_reduce(const double *__restrict__ part, int64_t n_act, int n_split, double *__restrict__ o_acc,
         double *__restrict__ o_jrk, double *__restrict__ o_snp, double *__restrict__ o_crk,
         double *__restrict__ o_pot)
{
    constexpr int NV = 3 * (P / 2);
    constexpr int NC = NV + 1;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n_act * NC) return;
    const int c = int(t / n_act);
    const int64_t q = t - int64_t(c) * n_act;
    double s = 0.0;
    for (int sp = 0; sp < n_split; ++sp) s += part[(int64_t(sp) * NC + c) * n_act + q];
    if (c == NV) {
        if (o_pot) o_pot[q] = s;
        return;
    }
    double *outs[4] = {o_acc, o_jrk, o_snp, o_crk};
    double *o = outs[c / 3];
    if (o) o[(c % 3) * n_act + q] = s;
}

template <class Pol, int P, int NI>
hipError_t run(const ForceArgs &a, hipStream_t s, int block, int n_split, int64_t j_chunk)
{
    const int64_t per_block = int64_t(block) * NI;
    const int64_t tiles = (a.n_act + per_block - 1) / per_block;
    const dim3 grid{unsigned(tiles), unsigned(n_split), 1u};
    hipLaunchKernelGGL((k_force<Pol, P, NI>), grid, dim3(block), 0, s,
                       static_cast<const typename Pol::Rec *>(a.rec), a.n, a.act, a.n_act, a.eps2, a.n_hard,
                       j_chunk, n_split, a.out[0], a.out[1], a.out[2], a.out[3], a.out[4], a.part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_split == 1) return e;
    const int64_t work = a.n_act * (3 * (P / 2) + 1);
    hipLaunchKernelGGL((k_reduce<P>), dim3(unsigned((work + 255) / 256)), dim3(256), 0, s, a.part, a.n_act,
                       n_split, a.out[0], a.out[1], a.out[2], a.out[3], a.out[4]);
    return hipGetLastError();
}

template <class Pol, int P>
hipError_t run_ni(const ForceArgs &a, hipStream_t s, int ni, int block, int n_split, int64_t j_chunk)
{
    if (ni == 2) return run<Pol, P, 2>(a, s, block, n_split, j_chunk);
    return run<Pol, P, 1>(a, s, block, n_split, j_chunk);
}

template <int P>
hipError_t run_prec(int precision, const ForceArgs &a, hipStream_t s, int ni, int block, int n_split,
                    int64_t j_chunk)
{
    switch (precision) {
    case NBODY_MIXED: return run_ni<PolMx<P>, P>(a, s, ni, block, n_split, j_chunk);
    case NBODY_DS: return run_ni<PolDS<P>, P>(a, s, ni, block, n_split, j_chunk);
    default: return run_ni<PolF64<P>, P>(a, s, ni, block, n_split, j_chunk);
    }
}

}  // namespace

int record_bytes(int order, int precision)
{
    if (precision == NBODY_FP64) return order == 4 ? 64 : order == 6 ? 80 : 112;
    return order == 8 ? 80 : 64;
}

// Number of j-splits: enough waves to cover every SIMD several times when the
// active set is small, bounded by the partial-sum scratch and by keeping at
// least 256 j per split.
static int auto_split(int64_t n, int64_t n_act, int ni, int block)
{
    const int64_t per_block = int64_t(block) * ni;
    const int64_t tiles = (n_act + per_block - 1) / per_block;
    const int64_t waves = tiles * (block / 64);
    const int64_t target_waves = 256 * 4 * 4;   // CUs x SIMDs x waves per SIMD
    int64_t sp = (target_waves + waves - 1) / waves;
    const int64_t max_by_n = n / 256 > 0 ? n / 256 : 1;
    const int64_t max_by_part = kPartEntries / (n_act > 0 ? n_act : 1);
    if (sp > max_by_n) sp = max_by_n;
    if (sp > max_by_part) sp = max_by_part;
    if (sp > 65535) sp = 65535;
    return sp < 1 ? 1 : int(sp);
}

hipError_t launch_force(int order, int precision, const ForceArgs &a, hipStream_t s, int *used_split)
{
    const int ni = (a.ni == 2) ? 2 : 1;
    const int block = (a.block == 64 || a.block == 128) ? a.block : 256;
    int sp = a.n_split > 0 ? a.n_split : auto_split(a.n, a.n_act, ni, block);
    if (int64_t(sp) * a.n_act > kPartEntries) sp = int(kPartEntries / a.n_act);
    if (sp < 1) sp = 1;
    // split length: a multiple of the MIXED chunk so every chunk is full
    int64_t j_chunk = (a.n + sp - 1) / sp;
    j_chunk = (j_chunk + kMixedChunk - 1) / kMixedChunk * kMixedChunk;
    sp = int((a.n + j_chunk - 1) / j_chunk);
    if (used_split) *used_split = sp;
    switch (order) {
    case 4: return run_prec<4>(precision, a, s, ni, block, sp, j_chunk);
    case 6: return run_prec<6>(precision, a, s, ni, block, sp, j_chunk);
    default: return run_prec<8>(precision, a, s, ni, block, sp, j_chunk);
    }
}

}  // namespace nb
