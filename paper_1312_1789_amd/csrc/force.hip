// force.hip -- the O(n_act * n) pairwise force kernels (acceleration, jerk,
// snap, crackle, potential) for gfx950, in FP64, MIXED and DS arithmetic.
//
// Direct summation of softened gravity over all j != i (paper: Abstract,
// where correlations between distant particles rule out approximations), with
// the time derivatives a Hermite scheme of order 4, 6 or 8 needs (paper:
// Sec. "Codes description").  Derivative recursion: Nitadori & Makino (2008).
//
// Launch shape: grid (i-tiles, j-splits).  A lane holds NI active particles
// in registers and the block walks its split's j range; the j records reach
// the lanes either through wave-uniform scalar loads (kernel A) or through
// LDS tiles (kernel B).  With one split the kernel writes the final FP64
// sums; with several, each split writes its partial sums and a second kernel
// adds them in split order (deterministic).
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
    __device__ static double self_pot(const Rec &r, double eps2) { return r.m * rsqrt64(eps2); }
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
    // the self pair's potential term, computed exactly as in the loop
    __device__ static double self_pot(const RecDS<P> &r, double eps2)
    {
        const float e2 = float(eps2);
        const float r2 = __builtin_fmaf(0.0f, 0.0f, __builtin_fmaf(0.0f, 0.0f, __builtin_fmaf(0.0f, 0.0f, e2)));
        return double(r.m * __builtin_amdgcn_rsqf(r2));
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
    __device__ static double self_pot(const Rec &r, double eps2) { return DSIn<P>::self_pot(r, eps2); }
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
    __device__ static double self_pot(const Rec &r, double eps2) { return DSIn<P>::self_pot(r, eps2); }
};

template <class Part> __device__ __forceinline__ void zero_part(Part &p) { p = Part(0); }
template <> __device__ __forceinline__ void zero_part<DS>(DS &p) { p.hi = 0.0f; p.lo = 0.0f; }
__device__ __forceinline__ double to_double(double v) { return v; }
__device__ __forceinline__ double to_double(float v) { return double(v); }
__device__ __forceinline__ double to_double(const DS &v) { return double(v.hi) + double(v.lo); }


// --------------------------------------------------------------------------
// Pieces shared by both force kernels.  blockIdx.x: i-tile of blockDim.x * NI
// active particles (lane t holds rows t, t + blockDim.x, ...); blockIdx.y:
// j-split [split * j_chunk, min(n, (split+1) * j_chunk)).  Pairs with both
// indices below n_hard are unsoftened and their self pair is masked; above
// n_hard the self pair is evaluated with eps2 > 0 (its acceleration and
// derivatives are exactly zero, every difference being zero) and its
// potential term is removed at the end.
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

template <class Pol, int NI, class ET>
__device__ __forceinline__ void hard_pairs(const typename Pol::Rec *__restrict__ rec, int64_t j0, int64_t jh1,
                                           int64_t n_hard, ET e2, const typename Pol::I *ip, const int64_t *iidx,
                                           double (*acc)[13])
{
    using Part = typename Pol::Part;
    for (int64_t j = j0; j < jh1; ++j) {
        const typename Pol::Rec rj = rec[j];
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

template <class Pol, int P, int NI>
__device__ __forceinline__ void store_rows(const typename Pol::Rec *__restrict__ rec, int64_t n_act, int64_t row0,
                                           int split, int n_split, int64_t js0, int64_t j1, double eps2,
                                           const int64_t *iidx, double (*acc)[13], double *__restrict__ o_acc,
                                           double *__restrict__ o_jrk, double *__restrict__ o_snp,
                                           double *__restrict__ o_crk, double *__restrict__ o_pot,
                                           double *__restrict__ part)
{
    constexpr int NV = 3 * (P / 2);
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int64_t q = row0 + int64_t(k) * blockDim.x;
        if (q >= n_act) continue;
        const int64_t i = iidx[k];
        double pot = acc[k][kPot];
        if (Pol::kWithPot && i >= js0 && i < j1) pot -= Pol::self_pot(rec[i], eps2);  // self pair was in the softened loop
        if (n_split == 1) {
            double *outs[4] = {o_acc, o_jrk, o_snp, o_crk};
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                double *o = outs[c / 3];
                if (o) o[(c % 3) * n_act + q] = acc[k][c];
            }
            if (Pol::kWithPot && o_pot) o_pot[q] = -pot;
        } else {
            constexpr int NC = NV + 1;
            double *base = part + int64_t(split) * NC * n_act;
#pragma unroll
            for (int c = 0; c < NV; ++c) base[int64_t(c) * n_act + q] = acc[k][c];
            if (Pol::kWithPot) base[int64_t(NV) * n_act + q] = -pot;
        }
    }
}

// Kernel A (scalar j path): every lane walks the same j range, so each j
// record is read with a wave-uniform address into SGPRs and feeds the VALU
// directly.  Suits FP64 arithmetic, which issues at one wave instruction per
// four cycles whatever the operand source.
template <class Pol, int P, int NI>
__global__ void __launch_bounds__(256)
k_force(const typename Pol::Rec *__restrict__ rec, int64_t n, const int32_t *__restrict__ act, int64_t n_act,
        double eps2, int64_t n_hard, int64_t j_chunk, int n_split, double *__restrict__ o_acc,
        double *__restrict__ o_jrk, double *__restrict__ o_snp, double *__restrict__ o_crk,
        double *__restrict__ o_pot, double *__restrict__ part)
{
    using Rec = typename Pol::Rec;
    using Part = typename Pol::Part;
    using ET = typename Pol::ET;
    const ET e2 = ET(eps2);
    const int64_t row0 = int64_t(blockIdx.x) * blockDim.x * NI + threadIdx.x;
    const int split = blockIdx.y;
    const int64_t j0 = int64_t(split) * j_chunk;
    const int64_t j1 = (j0 + j_chunk < n) ? j0 + j_chunk : n;

    typename Pol::I ip[NI];
    int64_t iidx[NI];
    double acc[NI][13];
    load_rows<Pol, NI>(rec, n, act, n_act, row0, ip, iidx, acc);
    hard_pairs<Pol, NI>(rec, j0, (j1 < n_hard) ? j1 : n_hard, n_hard, e2, ip, iidx, acc);

    const int64_t js0 = (j0 > n_hard) ? j0 : n_hard;
    constexpr int64_t CH = Pol::kChunk > 0 ? Pol::kChunk : (int64_t(1) << 40);
    Part p[NI][13];
#pragma unroll
    for (int k = 0; k < NI; ++k)
#pragma unroll
        for (int c = 0; c < 13; ++c) zero_part(p[k][c]);
    for (int64_t jc = js0; jc < j1; jc += CH) {
        const int64_t je = (jc + CH < j1) ? jc + CH : j1;
#pragma unroll 2
        for (int64_t j = jc; j < je; ++j) {
            const Rec rj = rec[j];
#pragma unroll
            for (int k = 0; k < NI; ++k) Pol::template pair<false>(ip[k], rj, e2, true, p[k]);
        }
        flush<Part, NI>(p, acc);
    }
    store_rows<Pol, P, NI>(rec, n_act, row0, split, n_split, js0, j1, eps2, iidx, acc, o_acc, o_jrk, o_snp, o_crk,
                           o_pot, part);
}

// Kernel B (LDS j path): the block stages BLOCK j records at a time in LDS
// (double-buffered, the next tile's global loads in flight during the
// current tile's arithmetic) and every lane reads them with same-address
// (broadcast) LDS loads into VGPRs.  All VALU operands are then VGPRs, which
// lets FP32 instructions of two waves on a SIMD issue together -- about twice
// the FP32 rate of SGPR-operand instructions on gfx950.  The FP32 chunk
// boundaries are those of kernel A, so both give identical bits.
template <class Pol, int P, int NI, int BLOCK, int UNROLL, int TILE>
__global__ void __launch_bounds__(BLOCK)
k_force_lds(const typename Pol::Rec *__restrict__ rec, int64_t n, const int32_t *__restrict__ act, int64_t n_act,
            double eps2, int64_t n_hard, int64_t j_chunk, int n_split, double *__restrict__ o_acc,
            double *__restrict__ o_jrk, double *__restrict__ o_snp, double *__restrict__ o_crk,
            double *__restrict__ o_pot, double *__restrict__ part)
{
    using Rec = typename Pol::Rec;
    using Part = typename Pol::Part;
    using ET = typename Pol::ET;
    constexpr int PIECES = int(sizeof(Rec) / 16);              // 16-byte pieces per record
    constexpr int PER_T = (TILE * PIECES + BLOCK - 1) / BLOCK;  // pieces each thread moves per tile
    typedef uint4 __attribute__((may_alias)) piece_t;           // raw 16-byte view of records
    __shared__ Rec tile[2][TILE];
    const ET e2 = ET(eps2);
    const int64_t row0 = int64_t(blockIdx.x) * BLOCK * NI + threadIdx.x;
    const int split = blockIdx.y;
    const int64_t j0 = int64_t(split) * j_chunk;
    const int64_t j1 = (j0 + j_chunk < n) ? j0 + j_chunk : n;

    typename Pol::I ip[NI];
    int64_t iidx[NI];
    double acc[NI][13];
    load_rows<Pol, NI>(rec, n, act, n_act, row0, ip, iidx, acc);
    hard_pairs<Pol, NI>(rec, j0, (j1 < n_hard) ? j1 : n_hard, n_hard, e2, ip, iidx, acc);

    const int64_t js0 = (j0 > n_hard) ? j0 : n_hard;
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
        int jj = 0;
        while (jj < cnt) {
            const int seg = (cnt - jj < CH - since) ? cnt - jj : CH - since;
#pragma unroll UNROLL
            for (int u = 0; u < seg; ++u) {
                const Rec rj = tr[jj + u];
#pragma unroll
                for (int k = 0; k < NI; ++k) Pol::template pair<false>(ip[k], rj, e2, true, p[k]);
            }
            jj += seg;
            since += seg;
            if (since == CH) {
                flush<Part, NI>(p, acc);
                since = 0;
            }
        }
        buf ^= 1;
    }
    flush<Part, NI>(p, acc);
    store_rows<Pol, P, NI>(rec, n_act, row0, split, n_split, js0, j1, eps2, iidx, acc, o_acc, o_jrk, o_snp, o_crk,
                           o_pot, part);
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

struct Shape {
    int ni, block, n_split, jpath;
    int64_t j_chunk;
};

template <class Pol, int P, int NI>
hipError_t run(const ForceArgs &a, hipStream_t s, const Shape &sh)
{
    const int64_t per_block = int64_t(sh.block) * NI;
    const int64_t tiles = (a.n_act + per_block - 1) / per_block;
    const dim3 grid{unsigned(tiles), unsigned(sh.n_split), 1u};
    const auto *rec = static_cast<const typename Pol::Rec *>(a.rec);
#define NB_FORCE_ARGS rec, a.n, a.act, a.n_act, a.eps2, a.n_hard, sh.j_chunk, sh.n_split, a.out[0], a.out[1], \
                      a.out[2], a.out[3], a.out[4], a.part
    if (sh.jpath == 1) {
        hipLaunchKernelGGL((k_force<Pol, P, NI>), grid, dim3(sh.block), 0, s, NB_FORCE_ARGS);
    } else if (sh.block == 64) {
        hipLaunchKernelGGL((k_force_lds<Pol, P, NI, 64, 2, 64>), grid, dim3(64), 0, s, NB_FORCE_ARGS);
    } else if (sh.block == 128) {
        hipLaunchKernelGGL((k_force_lds<Pol, P, NI, 128, 2, 128>), grid, dim3(128), 0, s, NB_FORCE_ARGS);
    } else {
        hipLaunchKernelGGL((k_force_lds<Pol, P, NI, 256, 2, 128>), grid, dim3(256), 0, s, NB_FORCE_ARGS);
    }
#undef NB_FORCE_ARGS
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || sh.n_split == 1) return e;
    const int64_t work = a.n_act * (3 * (P / 2) + 1);
    hipLaunchKernelGGL((k_reduce<P>), dim3(unsigned((work + 255) / 256)), dim3(256), 0, s, a.part, a.n_act,
                       sh.n_split, a.out[0], a.out[1], a.out[2], a.out[3], a.out[4]);
    return hipGetLastError();
}

template <class Pol, int P>
hipError_t run_ni(const ForceArgs &a, hipStream_t s, const Shape &sh)
{
    if (sh.ni == 2) return run<Pol, P, 2>(a, s, sh);
    return run<Pol, P, 1>(a, s, sh);
}

template <int P, bool POT>
hipError_t run_pot(int precision, const ForceArgs &a, hipStream_t s, const Shape &sh)
{
    switch (precision) {
    case NBODY_MIXED: return run_ni<PolMx<P, POT>, P>(a, s, sh);
    case NBODY_DS: return run_ni<PolDS<P, POT>, P>(a, s, sh);
    default: return run_ni<PolF64<P, POT>, P>(a, s, sh);
    }
}

// The potential is accumulated only when it is asked for.
template <int P>
hipError_t run_prec(int precision, const ForceArgs &a, hipStream_t s, const Shape &sh)
{
    return a.out[4] ? run_pot<P, true>(precision, a, s, sh) : run_pot<P, false>(precision, a, s, sh);
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
    const int64_t target_waves = 256 * 4 * 8;   // CUs x SIMDs x waves per SIMD
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
    Shape sh{};
    sh.ni = (a.ni == 2) ? 2 : 1;
    sh.block = (a.block == 64 || a.block == 128) ? a.block : 256;
    // j path: FP64 reads j records from SGPRs, the FP32 modes from LDS
    sh.jpath = a.jpath == 1 || a.jpath == 2 ? a.jpath : (precision == NBODY_FP64 ? 1 : 2);
    int sp = a.n_split > 0 ? a.n_split : auto_split(a.n, a.n_act, sh.ni, sh.block);
    if (int64_t(sp) * a.n_act > kPartEntries) sp = int(kPartEntries / a.n_act);
    if (sp < 1) sp = 1;
    // split length: a multiple of the MIXED chunk so chunks never straddle splits
    int64_t j_chunk = (a.n + sp - 1) / sp;
    j_chunk = (j_chunk + kMixedChunk - 1) / kMixedChunk * kMixedChunk;
    sh.j_chunk = j_chunk;
    sh.n_split = int((a.n + j_chunk - 1) / j_chunk);
    if (used_split) *used_split = sh.n_split;
    switch (order) {
    case 4: return run_prec<4>(precision, a, s, sh);
    case 6: return run_prec<6>(precision, a, s, sh);
    default: return run_prec<8>(precision, a, s, sh);
    }
}

}  // namespace nb
