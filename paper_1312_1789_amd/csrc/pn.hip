// pn.hip -- post-Newtonian terms between the hard particles (the paper's
// relativistic corrections for black-hole binaries, Introduction).
//
// For a pair with total mass M, symmetric mass ratio nu = m1 m2 / M^2,
// relative position x = x1 - x2 (r = |x|, n = x / r), relative velocity
// v = v1 - v2 and rdot = n.v, the post-Newtonian part of the relative
// acceleration in harmonic coordinates (G = 1, speed of light c) is
// -(M / r^2) [A n + B v] with (Blanchet, Living Rev. Relativ. 17, 2)
//   1PN:   A = (-3/2 nu rdot^2 + (1 + 3 nu) v^2 - 2 (2 + nu) M/r) / c^2,
//          B = -2 (2 - nu) rdot / c^2,
//   2PN:   A = (15/8 nu rdot^4 - 45/8 nu^2 rdot^4 - 9/2 nu rdot^2 v^2 + 6 nu^2 rdot^2 v^2
//               + 3 nu v^4 - 4 nu^2 v^4 + (M/r)(-2 rdot^2 - 25 nu rdot^2 - 2 nu^2 rdot^2
//               - 13/2 nu v^2 + 2 nu^2 v^2) + (M/r)^2 (9 + 87/4 nu)) / c^4,
//          B = (9/2 nu rdot^3 + 3 nu^2 rdot^3 - 15/2 nu rdot v^2 - 2 nu^2 rdot v^2
//               + (M/r)(2 + 41/2 nu + 4 nu^2) rdot) / c^4,
//   2.5PN: A = -8/5 nu (M/r) rdot (17/3 M/r + 3 v^2) / c^5,
//          B =  8/5 nu (M/r) (3 M/r + v^2) / c^5.
// Body 1 takes m2 / M of it, body 2 minus m1 / M.  Jerk, snap and crackle
// are its time derivatives along the pair's Newtonian two-body motion,
// carried through every operation as truncated Taylor series in t.
// Positions and velocities are predicted in FP64 from the stored state, so
// the terms do not depend on the force kernel's precision or records.
#include "hermite.h"

namespace nb {
namespace {

// Truncated Taylor series in t of degree 3: f_k = f^(k)(0) / k!.
struct TS {
    double c[4];
};
__device__ __forceinline__ TS tconst(double v) { return TS{{v, 0.0, 0.0, 0.0}}; }
__device__ __forceinline__ TS operator+(TS a, TS b)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) a.c[k] += b.c[k];
    return a;
}
__device__ __forceinline__ TS operator*(double s, TS a)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) a.c[k] *= s;
    return a;
}
__device__ __forceinline__ TS operator*(TS a, TS b)
{
    TS r;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i <= k; ++i) t += a.c[i] * b.c[k - i];
        r.c[k] = t;
    }
    return r;
}
__device__ __forceinline__ TS operator/(TS a, TS b)
{
    TS r;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double t = a.c[k];
#pragma unroll
        for (int i = 1; i <= k; ++i) t -= b.c[i] * r.c[k - i];
        r.c[k] = t / b.c[0];
    }
    return r;
}
__device__ __forceinline__ TS tsqrt(TS a)
{
    TS r;
    r.c[0] = sqrt(a.c[0]);
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        double t = a.c[k];
#pragma unroll
        for (int i = 1; i < k; ++i) t -= r.c[i] * r.c[k - i];
        r.c[k] = t / (2.0 * r.c[0]);
    }
    return r;
}
__device__ __forceinline__ TS tdot(const TS *a, const TS *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// The post-Newtonian part of the relative acceleration and its first three
// time derivatives (d[k][l], k = 0..3) along the two-body Newtonian motion
// from (x, v): the trajectory's series from x'' = -M x / |x|^3 coefficient
// by coefficient (the acceleration's coefficient k fixes x's coefficient
// k + 2), then the terms evaluated on the series.
__device__ void pn_relative(double M, double nu, double c, int terms, const double *x, const double *v,
                            double (*d)[3])
{
    TS X[3];
    double x4[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        X[l] = tconst(x[l]);
        X[l].c[1] = v[l];
        x4[l] = 0.0;
    }
#pragma unroll
    for (int k = 0; k <= 2; ++k) {
        const TS r2 = tdot(X, X);
        const TS r3 = r2 * tsqrt(r2);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const TS acc = ((-M) * X[l]) / r3;
            const double xk = acc.c[k] / ((k + 1.0) * (k + 2.0));
            if (k + 2 < 4) X[l].c[k + 2] = xk;
            else x4[l] = xk;
        }
    }
    TS V[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
#pragma unroll
        for (int k = 0; k < 3; ++k) V[l].c[k] = (k + 1.0) * X[l].c[k + 1];
        V[l].c[3] = 4.0 * x4[l];
    }
    const TS r2 = tdot(X, X);
    const TS r = tsqrt(r2);
    TS n[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) n[l] = X[l] / r;
    const TS rdot = tdot(n, V);
    const TS v2 = tdot(V, V);
    const TS Mr = tconst(M) / r;
    TS A = tconst(0.0), B = tconst(0.0);
    if (terms & 1) {
        const double ic2 = 1.0 / (c * c);
        A = A + ic2 * ((-1.5 * nu) * (rdot * rdot) + (1.0 + 3.0 * nu) * v2 + (-2.0 * (2.0 + nu)) * Mr);
        B = B + (-2.0 * (2.0 - nu) * ic2) * rdot;
    }
    if (terms & 2) {
        // grouped by powers of rdot and v^2; the same terms as the 2PN A, B
        const double ic4 = 1.0 / (c * c * c * c);
        const double nu2 = nu * nu;
        const TS rd2 = rdot * rdot;
        const TS rm = Mr * rdot;
        const TS a2 = rd2 * ((15.0 / 8.0 * nu - 45.0 / 8.0 * nu2) * rd2 + (6.0 * nu2 - 4.5 * nu) * v2) +
                      (3.0 * nu - 4.0 * nu2) * (v2 * v2) +
                      Mr * ((-2.0 - 25.0 * nu - 2.0 * nu2) * rd2 + (2.0 * nu2 - 6.5 * nu) * v2 +
                            (9.0 + 87.0 / 4.0 * nu) * Mr);
        const TS b2 = rdot * ((4.5 * nu + 3.0 * nu2) * rd2 + (-7.5 * nu - 2.0 * nu2) * v2) +
                      (2.0 + 20.5 * nu + 4.0 * nu2) * rm;
        A = A + ic4 * a2;
        B = B + ic4 * b2;
    }
    if (terms & 4) {
        const double ic5 = 1.0 / (c * c * c * c * c);
        A = A + (-1.6 * nu * ic5) * (Mr * rdot * ((17.0 / 3.0) * Mr + 3.0 * v2));
        B = B + (1.6 * nu * ic5) * (Mr * (3.0 * Mr + v2));
    }
    const TS pre = tconst(-M) / r2;
    const double fact[4] = {1.0, 1.0, 2.0, 6.0};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const TS t = pre * (A * n[l] + B * V[l]);
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k][l] = fact[k] * t.c[k];
    }
}

// One lane per leading row of the active list (the hard particles come
// first in an ordered list): for a hard particle i, the terms of every pair
// (i, k) with k < n_hard, k != i, added to its acceleration and jerk, and to
// its snap and crackle when those outputs are given (orders 6 and 8).
struct PnDs {
    const double *d[6];   // the stored derivatives a^(0..p-3) ([3][n] each), passed by value
};

template <int P>
__global__ void __launch_bounds__(64)
k_pn(int64_t n, int64_t n_hard, int rows, const double *__restrict__ m, const double *__restrict__ x,
     const double *__restrict__ v, PnDs ds, const int64_t *__restrict__ t_tick_of, int64_t t,
     double c, int terms, const int32_t *__restrict__ act, int64_t n_act, double *__restrict__ acc,
     double *__restrict__ jrk, double *__restrict__ snp, double *__restrict__ crk)
{
    const int q = int(blockIdx.x) * 64 + int(threadIdx.x);
    if (q >= rows) return;
    const int64_t i = act[q];
    if (i < 0 || i >= n_hard) return;
    constexpr double kInvTick = 1.0 / double(kTicksPerUnit);
    // predicted to t; without times (initialisation) the state itself, read
    // directly (the higher stored derivatives may not be set yet)
    const auto pred = [&](int64_t k) {
        if (!t_tick_of) {
            RecF64<P> r{};
            r.x = x[k]; r.y = x[n + k]; r.z = x[2 * n + k]; r.m = m[k];
            r.vx = v[k]; r.vy = v[n + k]; r.vz = v[2 * n + k];
            return r;
        }
        return predict_state<P, NBODY_FP64>(load_pstate<P>(n, k, m, x, v, ds.d), double(t - t_tick_of[k]) * kInvTick);
    };
    const RecF64<P> pi = pred(i);
    double s[4][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int64_t k = 0; k < n_hard; ++k) {
        if (k == i) continue;
        const RecF64<P> pk = pred(k);
        const double xr[3] = {pi.x - pk.x, pi.y - pk.y, pi.z - pk.z};
        const double vr[3] = {pi.vx - pk.vx, pi.vy - pk.vy, pi.vz - pk.vz};
        const double M = pi.m + pk.m, nu = pi.m * pk.m / (M * M), w = pk.m / M;
        double d[4][3];
        pn_relative(M, nu, c, terms, xr, vr, d);
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int l = 0; l < 3; ++l) s[o][l] += w * d[o][l];
    }
    double *outs[4] = {acc, jrk, snp, crk};
#pragma unroll
    for (int o = 0; o < 4; ++o)
        if (outs[o])
#pragma unroll
            for (int l = 0; l < 3; ++l) outs[o][l * n_act + q] += s[o][l];
}

}  // namespace

hipError_t launch_pn(const nbody_config &c, const nbody_state &st, const int64_t *t_tick_of, int64_t t_tick,
                     const int32_t *act, int64_t n_act, double *acc, double *jrk, double *snp, double *crk,
                     hipStream_t s)
{
    const int64_t nh = c.n_hard < c.n ? c.n_hard : c.n;
    const int rows = int(n_act < nh ? n_act : nh);
    if (rows <= 0) return hipSuccess;
    const dim3 g(unsigned((rows + 63) / 64));
    const PnDs ds{{st.d[0], st.d[1], st.d[2], st.d[3], st.d[4], st.d[5]}};
#define NB_PN(P)                                                                                              \
    hipLaunchKernelGGL((k_pn<P>), g, dim3(64), 0, s, c.n, nh, rows, st.m, st.x, st.v, ds, t_tick_of, t_tick, \
                       c.c_light, int(c.pn_terms), act, n_act, acc, jrk, snp, crk)
    if (c.order == 4) NB_PN(4);
    else if (c.order == 6) NB_PN(6);
    else NB_PN(8);
#undef NB_PN
    return hipGetLastError();
}

}  // namespace nb
