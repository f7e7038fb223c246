// hermite.h -- per-particle device arithmetic of the Hermite block-step
// scheme, shared by the single-system and the batched kernels: Taylor
// predictor and record writer, time-symmetric corrector with Hermite
// interpolation of the higher derivatives, time-step criterion and block
// quantisation.
//
// Method (paper: Abstract; Sec. "Codes description"): Hermite integration of
// order 4, 6 or 8 with individual hierarchical block time steps.  Formulas:
// time-symmetric Hermite corrector (order 4: Hut & Makino; orders 6 and 8:
// Nitadori & Makino 2008), derivatives at the end of the step from the
// Hermite interpolant through both ends, Aarseth's step criterion (order 4)
// and its generalisation (orders 6 and 8, Nitadori & Makino 2008), of the
// scheme's order or of order 4.
#pragma once

#include "internal.h"
#include "records.h"

namespace nb {
namespace {

// --------------------------------------------------------------------------
// Predictor: Taylor series about each particle's own time to t, in Horner
// form.  D[0..p-1] = x, v, a, jerk, ...; returns sum_k D[k] dt^k / k!.
template <int N>
__device__ __forceinline__ double taylor(const double *D, double dt)
{
    double s = D[N - 1];
#pragma unroll
    for (int k = N - 1; k >= 1; --k) s = __builtin_fma(s, dt * (1.0 / double(k)), D[k - 1]);
    return s;
}

// The stored state of one particle that the predictor reads: mass and, per
// component, x, v and the stored derivatives a^(0..p-3).
template <int P> struct PState {
    double m;
    double D[3][P];
};

template <int P>
__device__ __forceinline__ PState<P> load_pstate(int64_t n, int64_t i, const double *__restrict__ m,
                                                 const double *__restrict__ x, const double *__restrict__ v,
                                                 const double *const *ds)
{
    PState<P> s;
    s.m = m[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        s.D[c][0] = x[c * n + i];
        s.D[c][1] = v[c * n + i];
#pragma unroll
        for (int k = 0; k < P - 2; ++k) s.D[c][k + 2] = ds[k][c * n + i];
    }
    return s;
}

// The j-particle record of a stored state predicted by dt: RecF64<P> (FP64)
// or RecDS<P> (double-single position and velocity, FP32 mass, acceleration
// and jerk) for PREC = NBODY_FP64 or otherwise.
template <int P, int PREC> struct PredRec { using type = RecDS<P>; };
template <int P> struct PredRec<P, NBODY_FP64> { using type = RecF64<P>; };

template <int P, int PREC>
__device__ __forceinline__ typename PredRec<P, PREC>::type predict_state(const PState<P> &s, double dt)
{
    double xp[3], vp[3], ap[3], jp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xp[c] = taylor<P>(s.D[c], dt);
        vp[c] = taylor<P - 1>(s.D[c] + 1, dt);
        if constexpr (P >= 6) ap[c] = taylor<P - 2>(s.D[c] + 2, dt);
        if constexpr (P >= 8) jp[c] = taylor<P - 3>(s.D[c] + 3, dt);
    }
    const double mi = s.m;
    if constexpr (PREC == NBODY_FP64) {
        RecF64<P> r{};
        r.x = xp[0]; r.y = xp[1]; r.z = xp[2]; r.m = mi;
        r.vx = vp[0]; r.vy = vp[1]; r.vz = vp[2];
        if constexpr (P >= 6) { r.ax = ap[0]; r.ay = ap[1]; r.az = ap[2]; }
        if constexpr (P >= 8) { r.jx = jp[0]; r.jy = jp[1]; r.jz = jp[2]; }
        return r;
    } else {
        RecDS<P> r{};
        float hx[3], lx[3], hv[3], lv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            hx[c] = float(xp[c]);
            lx[c] = float(xp[c] - double(hx[c]));
            hv[c] = float(vp[c]);
            lv[c] = float(vp[c] - double(hv[c]));
        }
        r.xh = hx[0]; r.yh = hx[1]; r.zh = hx[2]; r.m = float(mi);
        r.xl = lx[0]; r.yl = lx[1]; r.zl = lx[2];
        r.vxh = hv[0]; r.vyh = hv[1]; r.vzh = hv[2];
        r.vxl = lv[0]; r.vyl = lv[1]; r.vzl = lv[2];
        if constexpr (P >= 6) { r.ax = float(ap[0]); r.ay = float(ap[1]); r.az = float(ap[2]); }
        if constexpr (P >= 8) { r.jx = float(jp[0]); r.jy = float(jp[1]); r.jz = float(jp[2]); }
        return r;
    }
}

// Particle i (state arrays [3][n]) predicted by dt.
template <int P, int PREC>
__device__ __forceinline__ typename PredRec<P, PREC>::type predict_rec(int64_t n, int64_t i, double dt,
                                                                      const double *__restrict__ m,
                                                                      const double *__restrict__ x,
                                                                      const double *__restrict__ v,
                                                                      const double *const *ds)
{
    return predict_state<P, PREC>(load_pstate<P>(n, i, m, x, v, ds), dt);
}

// Predict particle i by dt and write its record.
template <int P, int PREC>
__device__ __forceinline__ void predict_one(int64_t n, int64_t i, double dt, const double *__restrict__ m,
                                            const double *__restrict__ x, const double *__restrict__ v,
                                            const double *const *ds, void *__restrict__ rec_out)
{
    using Rec = typename PredRec<P, PREC>::type;
    static_cast<Rec *>(rec_out)[i] = predict_rec<P, PREC>(n, i, dt, m, x, v, ds);
}

// --------------------------------------------------------------------------
// Time-step level.  Largest 2^-k <= dt, i.e. k = -floor(log2 dt), clamped to
// [k_min, k_max]; NaN or zero gives k_max.
__device__ __forceinline__ int level_for(double dt, int k_min, int k_max)
{
    if (!(dt > 0.0)) return k_max;
    if (dt >= ldexp(1.0, -k_min)) return k_min;
    int k = -ilogb(dt);
    if (k < k_min) k = k_min;
    if (k > k_max) k = k_max;
    return k;
}

__device__ __forceinline__ double norm3(double a, double b, double c)
{
    return __builtin_sqrt(__builtin_fma(a, a, __builtin_fma(b, b, c * c)));
}

// Integer coefficients of the Hermite interpolant's derivatives at the end of
// a step of length h, with scaled inputs P_k = a^(k)(t0) h^k and
// Q_k = a^(k)(t1) h^k (k < p/2):  a^(m)(t1) h^m = sum_k CP[m][k] P_k + CQ[m][k] Q_k.
// (Derived by solving the confluent interpolation conditions symbolically.)
template <int P>
__device__ __forceinline__ double interp(int m, const double *Ps, const double *Qs)
{
    constexpr int q = P / 2;
    constexpr double CP4[2][2] = {{6, 2}, {12, 6}};
    constexpr double CQ4[2][2] = {{-6, 4}, {-12, 6}};
    constexpr double CP6[3][3] = {{-60, -24, -3}, {-360, -168, -24}, {-720, -360, -60}};
    constexpr double CQ6[3][3] = {{60, -36, 9}, {360, -192, 36}, {720, -360, 60}};
    constexpr double CP8[4][4] = {{840, 360, 60, 4}, {10080, 4680, 840, 60}, {50400, 24480, 4680, 360},
                                  {100800, 50400, 10080, 840}};
    constexpr double CQ8[4][4] = {{-840, 480, -120, 16}, {-10080, 5400, -1200, 120},
                                  {-50400, 25920, -5400, 480}, {-100800, 50400, -10080, 840}};
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < q; ++k) {
        double cp, cq;
        if constexpr (P == 4) { cp = CP4[m][k]; cq = CQ4[m][k]; }
        else if constexpr (P == 6) { cp = CP6[m][k]; cq = CQ6[m][k]; }
        else { cp = CP8[m][k]; cq = CQ8[m][k]; }
        s = __builtin_fma(cp, Ps[k], __builtin_fma(cq, Qs[k], s));
    }
    return s;
}

// Corrector + interpolation + new step of particle i, whose step ends at t1.
// fnew[k][stride * c + row] are the force derivatives a^(k) at t1 (k < p/2).
// rule (orders 6, 8): 1 = generalised criterion of order P, 2 = its order-4
// form, which reads only a .. a^(3).  Returns flags: bit 0 = a corrected
// value is not finite, bit 1 = dt_crit fell below 2^-k_max.
template <int P>
__device__ __forceinline__ int correct_one(int64_t n, int64_t i, int64_t t1, const double *const *fnew,
                                           int64_t stride, int64_t row, double *__restrict__ x,
                                           double *__restrict__ v, double *const *dst,
                                           int64_t *__restrict__ t_tick, int32_t *__restrict__ level, double eta,
                                           int rule, int k_min, int k_max)
{
    constexpr int q = P / 2;
    const double h = double(t1 - t_tick[i]) * (1.0 / double(kTicksPerUnit));
    double all[P][3];   // a^(0..p-1) at t1
    double xn[3], vn[3];
    bool finite = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double A0[q], A1[q];
#pragma unroll
        for (int k = 0; k < q; ++k) {
            A0[k] = dst[k][c * n + i];
            A1[k] = fnew[k][c * stride + row];
        }
        const double x0 = x[c * n + i], v0 = v[c * n + i];
        // velocity: integral of the interpolant of a(t); position: the same
        // quadrature applied to v(t) with the corrected end velocity
        double v1, x1;
        if constexpr (P == 4) {
            v1 = v0 + h * __builtin_fma(h, (A0[1] - A1[1]) * (1.0 / 12.0), 0.5 * (A0[0] + A1[0]));
            x1 = x0 + h * __builtin_fma(h, (A0[0] - A1[0]) * (1.0 / 12.0), 0.5 * (v0 + v1));
        } else if constexpr (P == 6) {
            v1 = v0 + h * __builtin_fma(h, __builtin_fma(h, (A0[2] + A1[2]) * (1.0 / 120.0),
                                                          (A0[1] - A1[1]) * (1.0 / 10.0)),
                                        0.5 * (A0[0] + A1[0]));
            x1 = x0 + h * __builtin_fma(h, __builtin_fma(h, (A0[1] + A1[1]) * (1.0 / 120.0),
                                                          (A0[0] - A1[0]) * (1.0 / 10.0)),
                                        0.5 * (v0 + v1));
        } else {
            v1 = v0 + h * __builtin_fma(h, __builtin_fma(h, __builtin_fma(h, (A0[3] - A1[3]) * (1.0 / 1680.0),
                                                                          (A0[2] + A1[2]) * (1.0 / 84.0)),
                                                          (A0[1] - A1[1]) * (3.0 / 28.0)),
                                        0.5 * (A0[0] + A1[0]));
            x1 = x0 + h * __builtin_fma(h, __builtin_fma(h, __builtin_fma(h, (A0[2] - A1[2]) * (1.0 / 1680.0),
                                                                          (A0[1] + A1[1]) * (1.0 / 84.0)),
                                                          (A0[0] - A1[0]) * (3.0 / 28.0)),
                                        0.5 * (v0 + v1));
        }
        xn[c] = x1;
        vn[c] = v1;
        finite = finite && __builtin_isfinite(x1) && __builtin_isfinite(v1);
        // higher derivatives at t1 from the interpolant
        double Ps[q], Qs[q];
        double hk = 1.0;
#pragma unroll
        for (int k = 0; k < q; ++k) {
            Ps[k] = A0[k] * hk;
            Qs[k] = A1[k] * hk;
            all[k][c] = A1[k];
            hk *= h;
        }
#pragma unroll
        for (int m = 0; m < q; ++m) {
            all[q + m][c] = interp<P>(m, Ps, Qs) / hk;
            hk *= h;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c * n + i] = xn[c];
        v[c * n + i] = vn[c];
#pragma unroll
        for (int k = 0; k <= P - 3; ++k) dst[k][c * n + i] = all[k][c];
    }
    double F[P];
#pragma unroll
    for (int k = 0; k < P; ++k) F[k] = norm3(all[k][0], all[k][1], all[k][2]);
    double dtc;
    if constexpr (P == 4) {
        dtc = __builtin_sqrt(eta * __builtin_fma(F[0], F[2], F[1] * F[1]) / __builtin_fma(F[1], F[3], F[2] * F[2]));
    } else {
        // eta (A_1 / A_(q-2))^(1/(q-3)), A_k = sqrt(|a^(k-1)| |a^(k+1)|) + |a^(k)|, q = P or 4
        const double a1 = __builtin_sqrt(F[0] * F[2]) + F[1];
        if (rule == 2) {
            dtc = eta * (a1 / (__builtin_sqrt(F[1] * F[3]) + F[2]));
        } else {
            const double ak = __builtin_sqrt(F[P - 3] * F[P - 1]) + F[P - 2];
            dtc = (P == 6) ? eta * cbrt(a1 / ak) : eta * pow(a1 / ak, 0.2);
        }
    }
    const int old = level[i];
    int k = level_for(dtc, k_min, k_max);
    if (k < old) {
        const int kd = old - 1;
        const int64_t dt2 = int64_t(1) << (kLevelMax - kd);
        k = (kd >= k_min && (t1 % dt2) == 0) ? kd : old;
    }
    level[i] = k;
    t_tick[i] = t1;
    return (finite ? 0 : 1) | ((dtc >= ldexp(1.0, -k_max)) ? 0 : 2);
}

}  // namespace
}  // namespace nb
