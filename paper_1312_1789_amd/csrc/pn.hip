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
//   2.5PN: A = -8/5 nu (M/r) rdot (17/3 M/r + 3 v^2) / c^5,
//          B =  8/5 nu (M/r) (3 M/r + v^2) / c^5.
// Body 1 takes m2 / M of it, body 2 minus m1 / M.  The jerk is its time
// derivative along dx/dt = v, dv/dt = -M x / r^3 (the pair's Newtonian
// motion), carried through every operation with (value, derivative) pairs.
// Positions and velocities are predicted in FP64 from the stored state, so
// the terms do not depend on the force kernel's precision or records.
#include "hermite.h"

namespace nb {
namespace {

struct Dual {
    double v, d;   // value, time derivative
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b)
{
    const double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual dsqrt(Dual a)
{
    const double r = sqrt(a.v);
    return {r, 0.5 * a.d / r};
}

__device__ void pn_relative(double M, double nu, double c, int terms, const double *x, const double *v, double *a,
                            double *j)
{
    const double r0 = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const double k0 = -M / (r0 * r0 * r0);
    Dual X[3], V[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        X[l] = {x[l], v[l]};
        V[l] = {v[l], k0 * x[l]};
    }
    const Dual r2 = X[0] * X[0] + X[1] * X[1] + X[2] * X[2];
    const Dual r = dsqrt(r2);
    Dual n[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) n[l] = X[l] / r;
    const Dual rdot = n[0] * V[0] + n[1] * V[1] + n[2] * V[2];
    const Dual v2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
    const Dual Mr = Dual{M, 0.0} / r;
    Dual A{0.0, 0.0}, B{0.0, 0.0};
    if (terms & 1) {
        const double ic2 = 1.0 / (c * c);
        A = A + ic2 * ((-1.5 * nu) * (rdot * rdot) + (1.0 + 3.0 * nu) * v2 + (-2.0 * (2.0 + nu)) * Mr);
        B = B + (-2.0 * (2.0 - nu) * ic2) * rdot;
    }
    if (terms & 4) {
        const double ic5 = 1.0 / (c * c * c * c * c);
        A = A + (-1.6 * nu * ic5) * (Mr * rdot * ((17.0 / 3.0) * Mr + 3.0 * v2));
        B = B + (1.6 * nu * ic5) * (Mr * (3.0 * Mr + v2));
    }
    const Dual pre = Dual{-M, 0.0} / r2;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const Dual t = pre * (A * n[l] + B * V[l]);
        a[l] = t.v;
        j[l] = t.d;
    }
}

// One lane per leading row of the active list (the hard particles come
// first in an ordered list): for a hard particle i, the terms of every pair
// (i, k) with k < n_hard, k != i, added to its acceleration and jerk.
__global__ void __launch_bounds__(64)
k_pn(int64_t n, int64_t n_hard, int rows, const double *__restrict__ m, const double *__restrict__ x,
     const double *__restrict__ v, const double *__restrict__ d0, const double *__restrict__ d1,
     const int64_t *__restrict__ t_tick_of, int64_t t, double c, int terms, const int32_t *__restrict__ act,
     int64_t n_act, double *__restrict__ acc, double *__restrict__ jrk)
{
    const int q = int(blockIdx.x) * 64 + int(threadIdx.x);
    if (q >= rows) return;
    const int64_t i = act[q];
    if (i < 0 || i >= n_hard) return;
    constexpr double kInvTick = 1.0 / double(kTicksPerUnit);
    const double *ds[2] = {d0, d1};
    const auto pred = [&](int64_t k) {
        const double dt = t_tick_of ? double(t - t_tick_of[k]) * kInvTick : 0.0;
        return predict_state<4, NBODY_FP64>(load_pstate<4>(n, k, m, x, v, ds), dt);
    };
    const RecF64<4> pi = pred(i);
    double sa[3] = {0.0, 0.0, 0.0}, sj[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < n_hard; ++k) {
        if (k == i) continue;
        const RecF64<4> pk = pred(k);
        const double xr[3] = {pi.x - pk.x, pi.y - pk.y, pi.z - pk.z};
        const double vr[3] = {pi.vx - pk.vx, pi.vy - pk.vy, pi.vz - pk.vz};
        const double M = pi.m + pk.m, nu = pi.m * pk.m / (M * M), w = pk.m / M;
        double a[3], j[3];
        pn_relative(M, nu, c, terms, xr, vr, a, j);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            sa[l] += w * a[l];
            sj[l] += w * j[l];
        }
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        acc[l * n_act + q] += sa[l];
        jrk[l * n_act + q] += sj[l];
    }
}

}  // namespace

hipError_t launch_pn(const nbody_config &c, const nbody_state &st, const int64_t *t_tick_of, int64_t t_tick,
                     const int32_t *act, int64_t n_act, double *acc, double *jrk, hipStream_t s)
{
    const int64_t nh = c.n_hard < c.n ? c.n_hard : c.n;
    const int rows = int(n_act < nh ? n_act : nh);
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pn, dim3(unsigned((rows + 63) / 64)), dim3(64), 0, s, c.n, nh, rows, st.m, st.x, st.v,
                       st.d[0], st.d[1], t_tick_of, t_tick, c.c_light, int(c.pn_terms), act, n_act, acc, jrk);
    return hipGetLastError();
}

}  // namespace nb
