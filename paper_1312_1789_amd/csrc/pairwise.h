// pairwise.h -- the pairwise interaction of softened gravity with its time
// derivatives (acceleration, jerk, snap, crackle, potential) in the three
// precision policies, shared by the single-system and batched force kernels.
//
// Direct summation of softened gravity (paper: Abstract; Sec. "Codes
// description"); derivative recursion of Nitadori & Makino (2008).
#pragma once

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
// are expanded into linear combinations of d, w, e, f and added with FMAs:
//   J = mu w + cj d,                     cj  = -3 alpha mu
//   S = mu e + cs1 w + cs2 d,            cs1 = 2 cj,
//                                        cs2 = (18 alpha^2 - 3 beta) mu = 3 mu (5 alpha^2 - (w.w + d.e)/f2)
//   C = mu f + c1 e + c2 w + c3 d,       c1 = 3 cj, c2 = -9 (alpha cs1 + beta mu),
//                                        c3 = -9 (alpha cs2 + beta cj) - 3 gamma mu
template <int P, bool POT, class T>
__device__ __forceinline__ void core_fma(T dx, T dy, T dz, T wx, T wy, T wz, T ex, T ey, T ez, T fx, T fy, T fz,
                                         T mr, T rinv2, T *A)
{
    const T mu = mr * rinv2;
    if constexpr (POT) A[kPot] += mr;
    A[0] = fmad(mu, dx, A[0]);
    A[1] = fmad(mu, dy, A[1]);
    A[2] = fmad(mu, dz, A[2]);
    const T al = fmad(dx, wx, fmad(dy, wy, dz * wz)) * rinv2;
    const T mu3 = T(3) * mu;
    const T cj = -(al * mu3);
    A[3] = fmad(mu, wx, fmad(cj, dx, A[3]));
    A[4] = fmad(mu, wy, fmad(cj, dy, A[4]));
    A[5] = fmad(mu, wz, fmad(cj, dz, A[5]));
    if constexpr (P >= 6) {
        const T s = fmad(wx, wx, fmad(wy, wy, fmad(wz, wz, fmad(dx, ex, fmad(dy, ey, dz * ez)))));
        const T sf = s * rinv2;
        const T al2 = al * al;
        const T cs1 = T(2) * cj;
        const T cs2 = fmad(T(5), al2, -sf) * mu3;
        A[6] = fmad(mu, ex, fmad(cs1, wx, fmad(cs2, dx, A[6])));
        A[7] = fmad(mu, ey, fmad(cs1, wy, fmad(cs2, dy, A[7])));
        A[8] = fmad(mu, ez, fmad(cs1, wz, fmad(cs2, dz, A[8])));
        if constexpr (P >= 8) {
            const T be = sf + al2;
            const T t = fmad(T(3), fmad(wx, ex, fmad(wy, ey, wz * ez)), fmad(dx, fx, fmad(dy, fy, dz * fz)));
            const T ga = fmad(t, rinv2, al * fmad(T(3), be, T(-4) * al2));
            const T c1 = T(3) * cj;
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
// FP64 policy.  POT: whether the potential is accumulated.
template <int P, bool POT> struct PolF64 {
    using Rec = RecF64<P>;
    using Part = double;                 // accumulate straight into FP64
    using ET = double;                   // softening type
    static constexpr int kChunk = 0;
    static constexpr bool kWithPot = POT;
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
        core_fma<P, POT, double>(dx, dy, dz, wx, wy, wz, ex, ey, ez, fx, fy, fz, mr, rinv * rinv, A);
    }
};

// Double-single inputs shared by the MIXED and DS policies: positions and
// velocities as hi + lo floats, FP32 mass, acceleration and jerk.  The
// difference (hi_j - hi_i) + (lo_j - lo_i) is accurate to FP32 rounding
// relative to the difference itself (the hi subtraction's error is relative
// to its own result), so close pairs keep their relative precision.
template <int P> struct DSIn {
    struct I { float xh, yh, zh, xl, yl, zl, vxh, vyh, vzh, vxl, vyl, vzl, ax, ay, az, jx, jy, jz; };

    __device__ static I load(const RecDS<P> &r)
    {
        I i{};
        i.xh = r.xh; i.yh = r.yh; i.zh = r.zh; i.xl = r.xl; i.yl = r.yl; i.zl = r.zl;
        i.vxh = r.vxh; i.vyh = r.vyh; i.vzh = r.vzh; i.vxl = r.vxl; i.vyl = r.vyl; i.vzl = r.vzl;
        if constexpr (P >= 6) { i.ax = r.ax; i.ay = r.ay; i.az = r.az; }
        if constexpr (P >= 8) { i.jx = r.jx; i.jy = r.jy; i.jz = r.jz; }
        return i;
    }
    // FP32 pair terms added into A (FMA-accumulated) -- the shared arithmetic.
    template <bool MASK, bool POT>
    __device__ static void terms(const I &i, const RecDS<P> &j, float eps2, bool valid, float *A)
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
        core_fma<P, POT, float>(dx, dy, dz, wx, wy, wz, ex, ey, ez, fx, fy, fz, mr, rinv * rinv, A);
    }
};

// MIXED policy: FP32 arithmetic on double-single differences, FP32 partial
// sums over chunks of kMixedChunk j (counted from the start of the j range,
// the same in every launch shape), each chunk added into FP64 accumulators.
template <int P, bool POT> struct PolMx {
    using Rec = RecDS<P>;
    using Part = float;
    using ET = float;
    using I = typename DSIn<P>::I;
    static constexpr int kChunk = kMixedChunk;
    static constexpr bool kWithPot = POT;
    __device__ static I load(const Rec &r) { return DSIn<P>::load(r); }
    template <bool MASK>
    __device__ static void pair(const I &i, const Rec &j, float eps2, bool valid, float *A)
    {
        DSIn<P>::template terms<MASK, POT>(i, j, eps2, valid, A);
    }
};

// DS policy: no FP64 instruction in the j loop; every term is added into a
// (hi, lo) pair with Knuth's error-free two-sum.
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

template <int P, bool POT> struct PolDS {
    using Rec = RecDS<P>;
    using Part = DS;
    using ET = float;
    using I = typename DSIn<P>::I;
    static constexpr int kChunk = 0;
    static constexpr bool kWithPot = POT;
    __device__ static I load(const Rec &r) { return DSIn<P>::load(r); }
    template <bool MASK>
    __device__ static void pair(const I &i, const Rec &j, float eps2, bool valid, DS *A)
    {
        // explicit terms (accumulating with FMAs would hide the rounding the
        // two-sum must capture)
        float T[13];
#pragma unroll
        for (int c = 0; c < 13; ++c) T[c] = 0.0f;
        DSIn<P>::template terms<MASK, POT>(i, j, eps2, valid, T);
        constexpr int nv = 3 * (P / 2);
#pragma unroll
        for (int c = 0; c < nv; ++c) two_sum_add(A[c], T[c]);
        if constexpr (POT) two_sum_add(A[kPot], T[kPot]);
    }
};

template <class Part> __device__ __forceinline__ void zero_part(Part &p) { p = Part(0); }
template <> __device__ __forceinline__ void zero_part<DS>(DS &p) { p.hi = 0.0f; p.lo = 0.0f; }
__device__ __forceinline__ double to_double(double v) { return v; }
__device__ __forceinline__ double to_double(float v) { return double(v); }
__device__ __forceinline__ double to_double(const DS &v) { return double(v.hi) + double(v.lo); }

// --------------------------------------------------------------------------
// Kernel-structure pieces shared by the force kernels.  A lane holds NI active
// rows: row0, row0 + blockDim.x, ...
template <class Pol, int NI>
__device__ __forceinline__ void load_rows(const typename Pol::Rec *__restrict__ rec, int64_t n,
                                          const int32_t *__restrict__ act, int64_t n_act, int64_t row0,
                                          typename Pol::I *ip, int64_t *iidx, double (*acc)[13])
{
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        int64_t q = row0 + int64_t(k) * blockDim.x;
        if (q >= n_act) q = n_act - 1;  // padding lanes recompute the last row; never stored
        const int64_t ia = act[q];
        iidx[k] = (ia >= 0 && ia < n) ? ia : 0;   // an index outside [0, n) yields an undefined row, never a fault
        ip[k] = Pol::load(rec[iidx[k]]);
#pragma unroll
        for (int c = 0; c < 13; ++c) acc[k][c] = 0.0;
    }
}

// Pairs among the first n_hard particles counted from base are unsoftened:
// j in [j0, jh1) (all below base + n_hard), per-lane softening, self pair
// masked by index.
template <class Pol, int NI, class ET>
__device__ __forceinline__ void hard_pairs(const typename Pol::Rec *__restrict__ rec, int64_t j0, int64_t jh1,
                                           int64_t base, int64_t n_hard, ET e2, const typename Pol::I *ip,
                                           const int64_t *iidx, double (*acc)[13])
{
    using Part = typename Pol::Part;
    for (int64_t j = j0; j < jh1; ++j) {
        const typename Pol::Rec rj = rec[j];
        Part p[NI][13];
#pragma unroll
        for (int k = 0; k < NI; ++k) {
#pragma unroll
            for (int c = 0; c < 13; ++c) zero_part(p[k][c]);
            const ET el = (iidx[k] - base < n_hard) ? ET(0) : e2;
            Pol::template pair<true>(ip[k], rj, el, j != iidx[k], p[k]);
#pragma unroll
            for (int c = 0; c < 13; ++c) acc[k][c] += to_double(p[k][c]);
        }
    }
}

template <class Part, int NI>
__device__ __forceinline__ void flush(Part (*p)[13], double (*acc)[13])
{
#pragma unroll
    for (int k = 0; k < NI; ++k)
#pragma unroll
        for (int c = 0; c < 13; ++c) {
            acc[k][c] += to_double(p[k][c]);
            zero_part(p[k][c]);
        }
}

// Records [js0, j1) through double-buffered LDS tiles of TILE records (the
// next tile's global loads in flight during the current tile's arithmetic),
// read with same-address (broadcast) LDS loads so that every VALU operand is
// a VGPR.  FP32 partial sums are added into acc every Pol::kChunk j counted
// from js0.  Every thread of the block must call it (it synchronises).
template <class Pol, int NI, int BLOCK, int UNROLL, int TILE>
__device__ __forceinline__ void lds_tiles(const typename Pol::Rec *__restrict__ rec, int64_t js0, int64_t j1,
                                          typename Pol::ET e2, const typename Pol::I *ip, const int64_t *iidx,
                                          typename Pol::Rec (*tile)[TILE], double (*acc)[13])
{
    using Rec = typename Pol::Rec;
    using Part = typename Pol::Part;
    constexpr int PIECES = int(sizeof(Rec) / 16);              // 16-byte pieces per record
    constexpr int PER_T = (TILE * PIECES + BLOCK - 1) / BLOCK;  // pieces each thread moves per tile
    typedef uint4 __attribute__((may_alias)) piece_t;           // raw 16-byte view of records
    constexpr int CH = Pol::kChunk > 0 ? Pol::kChunk : (1 << 30);
    Part p[NI][13];
#pragma unroll
    for (int k = 0; k < NI; ++k)
#pragma unroll
        for (int c = 0; c < 13; ++c) zero_part(p[k][c]);
    int since = 0;   // j since the last flush (uniform)
    // global -> registers for the tile starting at jt (coalesced 16-byte pieces)
    piece_t pre[PER_T];
#pragma unroll
    for (int k = 0; k < PER_T; ++k) pre[k] = piece_t{0u, 0u, 0u, 0u};
    if (js0 < j1) {
        const piece_t *src = reinterpret_cast<const piece_t *>(rec + js0);
        const int64_t avail = (j1 - js0) * PIECES;
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
            const int pc = int(threadIdx.x) + k * BLOCK;
            if (pc < TILE * PIECES && pc < avail) pre[k] = src[pc];
        }
    }
    int buf = 0;
    for (int64_t jt = js0; jt < j1; jt += TILE) {
        piece_t *dst = reinterpret_cast<piece_t *>(tile[buf]);
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
            const int pc = int(threadIdx.x) + k * BLOCK;
            if (pc < TILE * PIECES) dst[pc] = pre[k];
        }
        __syncthreads();   // tile ready; the other buffer is no longer read
        if (jt + TILE < j1) {
            const piece_t *src = reinterpret_cast<const piece_t *>(rec + jt + TILE);
            const int64_t avail = (j1 - jt - TILE) * PIECES;
#pragma unroll
            for (int k = 0; k < PER_T; ++k) {
                const int pc = int(threadIdx.x) + k * BLOCK;
                if (pc < TILE * PIECES && pc < avail) pre[k] = src[pc];
            }
        }
        const Rec *tr = tile[buf];
        const int cnt = (j1 - jt < TILE) ? int(j1 - jt) : TILE;
        // the next record is read from LDS while the current one is used
        Rec nxt = tr[0];
#pragma unroll UNROLL
        for (int u = 0; u < cnt; ++u) {
            const Rec rj = nxt;
            nxt = tr[(u + 1 < cnt) ? u + 1 : u];
            const int64_t j = jt + u;
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                // the self pair adds nothing to a, jerk, ...; only the
                // potential needs it masked
                if constexpr (Pol::kWithPot) Pol::template pair<true>(ip[k], rj, e2, j != iidx[k], p[k]);
                else Pol::template pair<false>(ip[k], rj, e2, true, p[k]);
            }
            if (++since == CH) {
                flush<Part, NI>(p, acc);
                since = 0;
            }
        }
        buf ^= 1;
    }
    flush<Part, NI>(p, acc);
}

}  // namespace
}  // namespace nb
