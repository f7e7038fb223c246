/*
 * nbody_oracle.c -- plain, slow CPU FP64 oracle for the block-step Hermite
 * N-body hot path.  TEST INFRASTRUCTURE ONLY: it is called by the tests, by the
 * package's smoke check and by the CPU-baseline leg of the benchmark, never by
 * the product path.  It shares no code with the HIP library.
 *
 * What it computes (the paper, Abstract and Sec. "Codes description"): direct
 * summation of softened Newtonian gravity, integrated with a 4th-, 6th- or
 * 8th-order Hermite scheme and individual hierarchical block time steps.  The
 * paper names the method but gives no formulas, so every formula below is the
 * standard published one it refers to:
 *   - force and its time derivatives: the recursion of Nitadori & Makino (2008)
 *     (alpha, beta, gamma coefficients);
 *   - corrector: the time-symmetric Hermite corrector (Hut & Makino form for
 *     order 4, Nitadori & Makino 2008 for orders 6 and 8);
 *   - higher derivatives at the end of a step: the unique Hermite interpolant
 *     of degree p-1 through the derivatives known at both ends;
 *   - time step: Aarseth's criterion (order 4) and its generalisation by
 *     Nitadori & Makino (2008) (orders 6 and 8), either of the scheme's order
 *     or of order 4 (the form that reads only a .. a^(3), for forces that
 *     carry single-precision noise);
 *   - block time steps: power-of-two steps, t_i always a multiple of dt_i,
 *     a step may double only when commensurate;
 *   - neighbour-split force (Ahmad & Cohen 1973, the scheme of the paper's
 *     second code): acceleration and jerk summed separately over the
 *     particles inside a neighbour sphere and over the rest, with the
 *     neighbour list;
 *   - post-Newtonian corrections between black holes (the paper's relativistic
 *     corrections for its black-hole binaries, Introduction): the 1PN, 2PN
 *     and 2.5PN terms of the two-body relative acceleration in harmonic
 *     coordinates (Blanchet 2014, Living Rev. Relativ. 17, 2, the A and B
 *     coefficients), added pairwise to the hard particles.
 * Build: gcc -O2 -ffp-contract=off -fopenmp, so rounding follows the source.
 *
 * Layouts: every 3-vector array is component-major [3][n] (x[0..n) are the
 * x components, x[n..2n) the y components, ...).  Time is kept in integer
 * ticks of 2^-40 time units; a particle on level k (k <= 40) has
 * dt = 2^(40-k) ticks.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TICKS_PER_UNIT (1LL << 40)
#define LEVEL_MAX 40

typedef struct {
    int order;        /* 4, 6 or 8 */
    double eps2;      /* softening squared for every pair ... */
    int64_t n_hard;   /* ... except pairs with both indices below n_hard (eps2 = 0) */
    double eta;       /* accuracy parameter of the time-step criterion */
    double eta_start; /* initial step parameter */
    int k_min, k_max; /* levels allowed: dt in [2^-k_max, 2^-k_min] */
    int dt_rule;      /* orders 6, 8: 1 = generalised criterion of the scheme's order,
                         2 = its order-4 form (reads a .. a^(3) only) */
    double c_light;   /* speed of light in the model's units; > 0 turns the
                         post-Newtonian terms of hard pairs on */
    int pn_terms;     /* which, a sum of: 1 = 1PN, 2 = 2PN, 4 = 2.5PN (radiation reaction) */
} oracle_config;

/* Particle state.  d[k] is the k-th derivative of the acceleration a^(k)
 * (d[0] = a, d[1] = jerk, d[2] = snap, d[3] = crackle, d[4], d[5]); the state
 * keeps k = 0 .. order-3. */
typedef struct {
    int64_t n;
    double *m;
    double *x, *v;
    double *d[6];
    int64_t *t_tick;
    int32_t *level;
} oracle_state;

static double pair_eps2(const oracle_config *c, int64_t i, int64_t j)
{
    return (i < c->n_hard && j < c->n_hard) ? 0.0 : c->eps2;
}

static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static double norm3(const double *a)
{
    return sqrt(dot3(a, a));
}

/* ------------------------------------------------------------------------ */
/* Pairwise force and its derivatives (Nitadori & Makino 2008 recursion).
 *
 * For pair (i, j) with relative position r, velocity v, acceleration a and
 * jerk jk (all "j minus i") and f = r.r + eps_ij^2:
 *   alpha = r.v / f
 *   beta  = (v.v + r.a) / f + alpha^2
 *   gamma = (3 v.a + r.jk) / f + alpha (3 beta - 4 alpha^2)
 *   A = m_j r / f^(3/2)
 *   J = m_j v / f^(3/2) - 3 alpha A
 *   S = m_j a / f^(3/2) - 6 alpha J - 3 beta A
 *   C = m_j jk / f^(3/2) - 9 alpha S - 9 beta J - 3 gamma A
 *   pot_i += -m_j / sqrt(f)
 * These are the successive time derivatives of m_j r / f^(3/2) along the
 * particles' trajectories.  Sums run over j != i in index order; the
 * self-pair is excluded by index.
 *
 * Inputs are the (predicted) states of all n particles.  Outputs are [3][n_act]
 * for the active list act[]; jk may be NULL for order < 8 and a for order < 6.
 * snp / crk / pot may be NULL.
 */
int oracle_force(const oracle_config *c, int64_t n, const double *m, const double *x, const double *v,
                 const double *a, const double *jk, int64_t n_act, const int32_t *act,
                 double *acc, double *jrk, double *snp, double *crk, double *pot)
{
    const int order = c->order;
    int64_t q;
#pragma omp parallel for schedule(dynamic, 16)
    for (q = 0; q < n_act; ++q) {
        const int64_t i = act[q];
        double sa[3] = {0, 0, 0}, sj[3] = {0, 0, 0}, ss[3] = {0, 0, 0}, sc[3] = {0, 0, 0};
        double sp = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r[3], w[3], aa[3] = {0, 0, 0}, jj[3] = {0, 0, 0};
            for (int k = 0; k < 3; ++k) {
                r[k] = x[k * n + j] - x[k * n + i];
                w[k] = v[k * n + j] - v[k * n + i];
                if (order >= 6) aa[k] = a[k * n + j] - a[k * n + i];
                if (order >= 8) jj[k] = jk[k * n + j] - jk[k * n + i];
            }
            const double f = dot3(r, r) + pair_eps2(c, i, j);
            const double rinv = 1.0 / sqrt(f);
            const double mu = m[j] * rinv * rinv * rinv;
            const double alpha = dot3(r, w) / f;
            const double beta = (dot3(w, w) + dot3(r, aa)) / f + alpha * alpha;
            const double gamma = (3.0 * dot3(w, aa) + dot3(r, jj)) / f + alpha * (3.0 * beta - 4.0 * alpha * alpha);
            double A[3], J[3], S[3], C[3];
            for (int k = 0; k < 3; ++k) {
                A[k] = mu * r[k];
                J[k] = mu * w[k] - 3.0 * alpha * A[k];
                S[k] = mu * aa[k] - 6.0 * alpha * J[k] - 3.0 * beta * A[k];
                C[k] = mu * jj[k] - 9.0 * alpha * S[k] - 9.0 * beta * J[k] - 3.0 * gamma * A[k];
                sa[k] += A[k];
                sj[k] += J[k];
                ss[k] += S[k];
                sc[k] += C[k];
            }
            sp -= m[j] * rinv;
        }
        for (int k = 0; k < 3; ++k) {
            acc[k * n_act + q] = sa[k];
            jrk[k * n_act + q] = sj[k];
            if (snp) snp[k * n_act + q] = ss[k];
            if (crk) crk[k * n_act + q] = sc[k];
        }
        if (pot) pot[q] = sp;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Force split by a neighbour sphere (the Ahmad & Cohen 1973 scheme, which the
 * paper's second code, NBODY6++GPU, uses: Sec. "Results", the laohu tests).
 * For active particle i with neighbour radius squared h2[q], particle j != i
 * is a neighbour when its unsoftened squared distance |x_j - x_i|^2 is below
 * h2[q].  The acceleration and jerk terms of each pair (as in oracle_force,
 * softened by eps_ij) are summed separately over the neighbours (irregular
 * part) and over the other particles (regular part), each in index order.
 * nb_count[q] = number of neighbours; nb_list[q * max_nb + k] for
 * k < min(nb_count[q], max_nb) = their indices in increasing order.
 * Outputs [3][n_act] (acc_*, jrk_*), [n_act] (nb_count), [n_act][max_nb]. */
int oracle_force_nb(const oracle_config *c, int64_t n, const double *m, const double *x, const double *v,
                    int64_t n_act, const int32_t *act, const double *h2, int32_t max_nb, double *acc_irr,
                    double *jrk_irr, double *acc_reg, double *jrk_reg, int32_t *nb_count, int32_t *nb_list)
{
    int64_t q;
#pragma omp parallel for schedule(dynamic, 16)
    for (q = 0; q < n_act; ++q) {
        const int64_t i = act[q];
        double ai[3] = {0, 0, 0}, ji[3] = {0, 0, 0}, ar[3] = {0, 0, 0}, jr[3] = {0, 0, 0};
        int32_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r[3], w[3];
            for (int k = 0; k < 3; ++k) {
                r[k] = x[k * n + j] - x[k * n + i];
                w[k] = v[k * n + j] - v[k * n + i];
            }
            const int is_nb = dot3(r, r) < h2[q];
            const double f = dot3(r, r) + pair_eps2(c, i, j);
            const double rinv = 1.0 / sqrt(f);
            const double mu = m[j] * rinv * rinv * rinv;
            const double alpha = dot3(r, w) / f;
            double *sa = is_nb ? ai : ar, *sj = is_nb ? ji : jr;
            for (int k = 0; k < 3; ++k) {
                const double A = mu * r[k];
                sa[k] += A;
                sj[k] += mu * w[k] - 3.0 * alpha * A;
            }
            if (is_nb) {
                if (cnt < max_nb) nb_list[q * max_nb + cnt] = (int32_t)j;
                ++cnt;
            }
        }
        for (int k = 0; k < 3; ++k) {
            acc_irr[k * n_act + q] = ai[k];
            jrk_irr[k * n_act + q] = ji[k];
            acc_reg[k * n_act + q] = ar[k];
            jrk_reg[k * n_act + q] = jr[k];
        }
        nb_count[q] = cnt;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Post-Newtonian terms (G = 1, speed of light c).  For a pair with total mass
 * M, symmetric mass ratio nu = m1 m2 / M^2, relative position x = x1 - x2
 * (r = |x|, n = x / r), relative velocity v = v1 - v2 and rdot = n.v, the
 * relative acceleration is  -(M / r^2) [(1 + A) n + B v]  with
 *   A_1PN   = ( -3/2 nu rdot^2 + (1 + 3 nu) v^2 - 2 (2 + nu) M / r ) / c^2
 *   B_1PN   = ( -2 (2 - nu) rdot ) / c^2
 *   A_2PN   = ( 15/8 nu rdot^4 - 45/8 nu^2 rdot^4 - 9/2 nu rdot^2 v^2
 *               + 6 nu^2 rdot^2 v^2 + 3 nu v^4 - 4 nu^2 v^4
 *               + (M / r) (-2 rdot^2 - 25 nu rdot^2 - 2 nu^2 rdot^2
 *                          - 13/2 nu v^2 + 2 nu^2 v^2)
 *               + (M / r)^2 (9 + 87/4 nu) ) / c^4
 *   B_2PN   = ( 9/2 nu rdot^3 + 3 nu^2 rdot^3 - 15/2 nu rdot v^2
 *               - 2 nu^2 rdot v^2 + (M / r) (2 + 41/2 nu + 4 nu^2) rdot ) / c^4
 *   A_2.5PN = -8/5 nu (M / r) rdot ( 17/3 M / r + 3 v^2 ) / c^5
 *   B_2.5PN =  8/5 nu (M / r) ( 3 M / r + v^2 ) / c^5
 * (the Newtonian part is the pair term of the direct sum).  Body 1 takes
 * m2 / M of the correction, body 2 minus m1 / M of it.  Its time derivatives
 * (jerk, snap, crackle) are taken along the pair's Newtonian two-body motion:
 * every quantity is carried as a truncated Taylor series in t of degree 3
 * (coefficients f_k = f^(k)(0) / k!), the trajectory's series coming from
 * the two-body equation x'' = -M x / |x|^3 itself, coefficient by coefficient. */
#define TS_N 4
typedef struct { double c[TS_N]; } tser;

static tser ts_const(double v) { tser r = {{v, 0.0, 0.0, 0.0}}; return r; }
static tser ts_add(tser a, tser b) { for (int k = 0; k < TS_N; ++k) a.c[k] += b.c[k]; return a; }
static tser ts_scl(double s, tser a) { for (int k = 0; k < TS_N; ++k) a.c[k] *= s; return a; }
static tser ts_mul(tser a, tser b)
{
    tser r;
    for (int k = 0; k < TS_N; ++k) {
        double t = 0.0;
        for (int i = 0; i <= k; ++i) t += a.c[i] * b.c[k - i];
        r.c[k] = t;
    }
    return r;
}
static tser ts_div(tser a, tser b)
{
    tser r;
    for (int k = 0; k < TS_N; ++k) {
        double t = a.c[k];
        for (int i = 1; i <= k; ++i) t -= b.c[i] * r.c[k - i];
        r.c[k] = t / b.c[0];
    }
    return r;
}
static tser ts_sqrt(tser a)
{
    tser r;
    r.c[0] = sqrt(a.c[0]);
    for (int k = 1; k < TS_N; ++k) {
        double t = a.c[k];
        for (int i = 1; i < k; ++i) t -= r.c[i] * r.c[k - i];
        r.c[k] = t / (2.0 * r.c[0]);
    }
    return r;
}
static tser ts_dot(const tser *a, const tser *b)
{
    return ts_add(ts_add(ts_mul(a[0], b[0]), ts_mul(a[1], b[1])), ts_mul(a[2], b[2]));
}

/* Derivatives 0..3 of the post-Newtonian part of the relative acceleration
 * along the two-body motion from (x, v): out[k][0..2] = d^k a_PN / dt^k. */
void oracle_pn_rel_derivs(double M, double nu, double c, int terms, const double *x, const double *v,
                          double out[4][3])
{
    /* trajectory: x(t) series to degree 4 (x4 kept apart), v(t) = x'(t) */
    tser X[3];
    double x4[3] = {0.0, 0.0, 0.0};
    for (int l = 0; l < 3; ++l) {
        X[l] = ts_const(x[l]);
        X[l].c[1] = v[l];
    }
    for (int k = 0; k <= 2; ++k) {   /* the acceleration's coefficient k fixes x's coefficient k + 2 */
        const tser r2 = ts_dot(X, X);
        const tser r3 = ts_mul(r2, ts_sqrt(r2));
        for (int l = 0; l < 3; ++l) {
            const tser acc = ts_div(ts_scl(-M, X[l]), r3);
            const double xk = acc.c[k] / ((k + 1.0) * (k + 2.0));
            if (k + 2 < TS_N) X[l].c[k + 2] = xk;
            else x4[l] = xk;
        }
    }
    tser V[3];
    for (int l = 0; l < 3; ++l) {
        for (int k = 0; k < TS_N - 1; ++k) V[l].c[k] = (k + 1.0) * X[l].c[k + 1];
        V[l].c[TS_N - 1] = TS_N * x4[l];
    }
    const tser r2 = ts_dot(X, X);
    const tser r = ts_sqrt(r2);
    tser n[3];
    for (int l = 0; l < 3; ++l) n[l] = ts_div(X[l], r);
    const tser rdot = ts_dot(n, V);
    const tser v2 = ts_dot(V, V);
    const tser Mr = ts_div(ts_const(M), r);
    tser A = ts_const(0.0), B = ts_const(0.0);
    if (terms & 1) {
        const double c2 = c * c;
        const tser a1 = ts_add(ts_add(ts_scl(-1.5 * nu, ts_mul(rdot, rdot)), ts_scl(1.0 + 3.0 * nu, v2)),
                               ts_scl(-2.0 * (2.0 + nu), Mr));
        A = ts_add(A, ts_scl(1.0 / c2, a1));
        B = ts_add(B, ts_scl(-2.0 * (2.0 - nu) / c2, rdot));
    }
    if (terms & 2) {
        const double c4 = c * c * c * c;
        const double nu2 = nu * nu;
        const tser rd2 = ts_mul(rdot, rdot);
        const tser rd3 = ts_mul(rd2, rdot);
        const tser rd4 = ts_mul(rd2, rd2);
        const tser v4 = ts_mul(v2, v2);
        const tser rd2v2 = ts_mul(rd2, v2);
        const tser rdv2 = ts_mul(rdot, v2);
        tser a2 = ts_scl(15.0 / 8.0 * nu, rd4);
        a2 = ts_add(a2, ts_scl(-45.0 / 8.0 * nu2, rd4));
        a2 = ts_add(a2, ts_scl(-9.0 / 2.0 * nu, rd2v2));
        a2 = ts_add(a2, ts_scl(6.0 * nu2, rd2v2));
        a2 = ts_add(a2, ts_scl(3.0 * nu, v4));
        a2 = ts_add(a2, ts_scl(-4.0 * nu2, v4));
        tser a2m = ts_scl(-2.0, rd2);
        a2m = ts_add(a2m, ts_scl(-25.0 * nu, rd2));
        a2m = ts_add(a2m, ts_scl(-2.0 * nu2, rd2));
        a2m = ts_add(a2m, ts_scl(-13.0 / 2.0 * nu, v2));
        a2m = ts_add(a2m, ts_scl(2.0 * nu2, v2));
        a2 = ts_add(a2, ts_mul(Mr, a2m));
        a2 = ts_add(a2, ts_scl(9.0 + 87.0 / 4.0 * nu, ts_mul(Mr, Mr)));
        tser b2 = ts_scl(9.0 / 2.0 * nu, rd3);
        b2 = ts_add(b2, ts_scl(3.0 * nu2, rd3));
        b2 = ts_add(b2, ts_scl(-15.0 / 2.0 * nu, rdv2));
        b2 = ts_add(b2, ts_scl(-2.0 * nu2, rdv2));
        b2 = ts_add(b2, ts_scl(2.0 + 41.0 / 2.0 * nu + 4.0 * nu2, ts_mul(Mr, rdot)));
        A = ts_add(A, ts_scl(1.0 / c4, a2));
        B = ts_add(B, ts_scl(1.0 / c4, b2));
    }
    if (terms & 4) {
        const double c5 = c * c * c * c * c;
        const tser a25 = ts_mul(ts_mul(Mr, rdot), ts_add(ts_scl(17.0 / 3.0, Mr), ts_scl(3.0, v2)));
        const tser b25 = ts_mul(Mr, ts_add(ts_scl(3.0, Mr), v2));
        A = ts_add(A, ts_scl(-1.6 * nu / c5, a25));
        B = ts_add(B, ts_scl(1.6 * nu / c5, b25));
    }
    const tser pre = ts_div(ts_const(-M), r2);
    const double fact[4] = {1.0, 1.0, 2.0, 6.0};
    for (int l = 0; l < 3; ++l) {
        const tser t = ts_mul(pre, ts_add(ts_mul(A, n[l]), ts_mul(B, V[l])));
        for (int k = 0; k < TS_N; ++k) out[k][l] = fact[k] * t.c[k];
    }
}

void oracle_pn_rel(double M, double nu, double c, int terms, const double *x, const double *v, double *apn,
                   double *jpn)
{
    double out[4][3];
    oracle_pn_rel_derivs(M, nu, c, terms, x, v, out);
    for (int l = 0; l < 3; ++l) {
        apn[l] = out[0][l];
        jpn[l] = out[1][l];
    }
}

/* Adds the post-Newtonian terms to acc, jrk (and snp, crk when not NULL)
 * ([3][n_act]) of the active hard particles (index below n_hard), one pair at
 * a time with every other hard particle, from the (predicted) states x, v.
 * No-op unless c_light > 0. */
int oracle_pn(const oracle_config *c, int64_t n, const double *m, const double *x, const double *v, int64_t n_act,
              const int32_t *act, double *acc, double *jrk, double *snp, double *crk)
{
    if (!(c->c_light > 0.0) || c->pn_terms == 0) return 0;
    const int64_t nh = c->n_hard < n ? c->n_hard : n;
    double *outs[4] = {acc, jrk, snp, crk};
    for (int64_t q = 0; q < n_act; ++q) {
        const int64_t i = act[q];
        if (i >= nh) continue;
        for (int64_t k = 0; k < nh; ++k) {
            if (k == i) continue;
            const double M = m[i] + m[k], nu = m[i] * m[k] / (M * M);
            double xr[3], vr[3], d[4][3];
            for (int l = 0; l < 3; ++l) {
                xr[l] = x[l * n + i] - x[l * n + k];
                vr[l] = v[l * n + i] - v[l * n + k];
            }
            oracle_pn_rel_derivs(M, nu, c->c_light, c->pn_terms, xr, vr, d);
            for (int o = 0; o < 4; ++o)
                if (outs[o])
                    for (int l = 0; l < 3; ++l) outs[o][l * n_act + q] += m[k] / M * d[o][l];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Predictor: Taylor series of the particle's trajectory about its own time,
 * using every stored derivative.  With D[0] = x, D[1] = v, D[k+2] = a^(k)
 * (k = 0 .. p-3) and delta = t - t_i, the predicted q-th derivative is
 *   sum_{k=0}^{p-1-q} D[q+k] delta^k / k!
 * (x to delta^(p-1), v to delta^(p-2), a to delta^(p-3), jerk to delta^(p-4)),
 * evaluated in Horner form.  Outputs [3][n]; ap / jp only for order >= 6 / 8. */
static double taylor(const double *D, int top, int q, double delta)
{
    /* D[q..top] are the derivatives; returns sum_k D[q+k] delta^k / k! */
    double s = D[top];
    for (int k = top - 1; k >= q; --k) s = D[k] + s * delta / (double)(k + 1 - q);
    return s;
}

int oracle_predict(const oracle_config *c, const oracle_state *s, int64_t t_tick,
                   double *xp, double *vp, double *ap, double *jp)
{
    const int p = c->order;
    const int64_t n = s->n;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        const double delta = (double)(t_tick - s->t_tick[i]) / (double)TICKS_PER_UNIT;
        for (int k = 0; k < 3; ++k) {
            double D[8];
            D[0] = s->x[k * n + i];
            D[1] = s->v[k * n + i];
            for (int l = 0; l <= p - 3; ++l) D[l + 2] = s->d[l][k * n + i];
            xp[k * n + i] = taylor(D, p - 1, 0, delta);
            vp[k * n + i] = taylor(D, p - 1, 1, delta);
            if (p >= 6 && ap) ap[k * n + i] = taylor(D, p - 1, 2, delta);
            if (p >= 8 && jp) jp[k * n + i] = taylor(D, p - 1, 3, delta);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Hermite interpolation.  With q = p/2 derivatives a^(0..q-1) known at the start
 * (D0) and at the end (D1) of an interval of length h, the polynomial of degree
 * p-1 matching all 2q values is unique; its derivatives a^(q..p-1) at the end
 * point are the fixed linear combinations below.  (They follow from writing
 * the polynomial about the end point and solving the 2q x 2q confluent
 * Vandermonde system; the tests check exactness on random polynomials.)
 * H[k] receives a^(q+k)(t1), k = 0 .. q-1 (one component). */
static void hermite_high(int p, double h, const double *D0, const double *D1, double *H)
{
    const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h, h6 = h5 * h, h7 = h6 * h;
    if (p == 4) {
        H[0] = 2.0 * (3.0 * D0[0] + D0[1] * h - 3.0 * D1[0] + 2.0 * D1[1] * h) / h2;
        H[1] = 6.0 * (2.0 * D0[0] + D0[1] * h - 2.0 * D1[0] + D1[1] * h) / h3;
    } else if (p == 6) {
        H[0] = 3.0 * (-20.0 * D0[0] - 8.0 * D0[1] * h - D0[2] * h2
                      + 20.0 * D1[0] - 12.0 * D1[1] * h + 3.0 * D1[2] * h2) / h3;
        H[1] = 12.0 * (-30.0 * D0[0] - 14.0 * D0[1] * h - 2.0 * D0[2] * h2
                       + 30.0 * D1[0] - 16.0 * D1[1] * h + 3.0 * D1[2] * h2) / h4;
        H[2] = 60.0 * (-12.0 * D0[0] - 6.0 * D0[1] * h - D0[2] * h2
                       + 12.0 * D1[0] - 6.0 * D1[1] * h + D1[2] * h2) / h5;
    } else {
        H[0] = 4.0 * (210.0 * D0[0] + 90.0 * D0[1] * h + 15.0 * D0[2] * h2 + D0[3] * h3
                      - 210.0 * D1[0] + 120.0 * D1[1] * h - 30.0 * D1[2] * h2 + 4.0 * D1[3] * h3) / h4;
        H[1] = 60.0 * (168.0 * D0[0] + 78.0 * D0[1] * h + 14.0 * D0[2] * h2 + D0[3] * h3
                       - 168.0 * D1[0] + 90.0 * D1[1] * h - 20.0 * D1[2] * h2 + 2.0 * D1[3] * h3) / h5;
        H[2] = 120.0 * (420.0 * D0[0] + 204.0 * D0[1] * h + 39.0 * D0[2] * h2 + 3.0 * D0[3] * h3
                        - 420.0 * D1[0] + 216.0 * D1[1] * h - 45.0 * D1[2] * h2 + 4.0 * D1[3] * h3) / h6;
        H[3] = 840.0 * (120.0 * D0[0] + 60.0 * D0[1] * h + 12.0 * D0[2] * h2 + D0[3] * h3
                        - 120.0 * D1[0] + 60.0 * D1[1] * h - 12.0 * D1[2] * h2 + D1[3] * h3) / h7;
    }
}

/* Exposed for the interpolation-exactness tests: one component. */
void oracle_hermite_high(int p, double h, const double *D0, const double *D1, double *H)
{
    hermite_high(p, h, D0, D1, H);
}

/* Time-symmetric Hermite corrector (one component).  The velocity update is
 * the exact integral over the step of the degree-(p-1) interpolant of a(t);
 * the position update applies the same quadrature to v(t), using the
 * corrected end velocity:
 *   p=4: v1 = v0 + h/2(a0+a1) - h^2/12(j1-j0)
 *   p=6: v1 = v0 + h/2(a0+a1) - h^2/10(j1-j0) + h^3/120(s0+s1)
 *   p=8: v1 = v0 + h/2(a0+a1) - 3h^2/28(j1-j0) + h^3/84(s0+s1) - h^4/1680(c1-c0)
 * and x1 likewise with (x, v, a, j, s) in place of (v, a, j, s, c). */
static void hermite_correct(int p, double h, double x0, double v0, const double *D0, const double *D1,
                            double *x1, double *v1)
{
    const double h2 = h * h, h3 = h2 * h, h4 = h3 * h;
    if (p == 4) {
        *v1 = v0 + h / 2.0 * (D0[0] + D1[0]) - h2 / 12.0 * (D1[1] - D0[1]);
        *x1 = x0 + h / 2.0 * (v0 + *v1) - h2 / 12.0 * (D1[0] - D0[0]);
    } else if (p == 6) {
        *v1 = v0 + h / 2.0 * (D0[0] + D1[0]) - h2 / 10.0 * (D1[1] - D0[1]) + h3 / 120.0 * (D0[2] + D1[2]);
        *x1 = x0 + h / 2.0 * (v0 + *v1) - h2 / 10.0 * (D1[0] - D0[0]) + h3 / 120.0 * (D0[1] + D1[1]);
    } else {
        *v1 = v0 + h / 2.0 * (D0[0] + D1[0]) - 3.0 * h2 / 28.0 * (D1[1] - D0[1])
              + h3 / 84.0 * (D0[2] + D1[2]) - h4 / 1680.0 * (D1[3] - D0[3]);
        *x1 = x0 + h / 2.0 * (v0 + *v1) - 3.0 * h2 / 28.0 * (D1[0] - D0[0])
              + h3 / 84.0 * (D0[1] + D1[1]) - h4 / 1680.0 * (D1[2] - D0[2]);
    }
}

void oracle_hermite_correct(int p, double h, double x0, double v0, const double *D0, const double *D1,
                            double *x1, double *v1)
{
    hermite_correct(p, h, x0, v0, D0, D1, x1, v1);
}

/* ------------------------------------------------------------------------ */
/* Time-step criterion.  F[k] = |a^(k)| at the end of the step, k = 0 .. p-1.
 *   p = 4 (Aarseth):  dt = sqrt(eta (|a||a2| + |a1|^2) / (|a1||a3| + |a2|^2))
 *   p = 6, 8 (generalised Aarseth, Nitadori & Makino 2008):
 *       A_k = sqrt(|a^(k-1)| |a^(k+1)|) + |a^(k)|
 *       dt  = eta (A_1 / A_(p-2))^(1/(p-3))                                  */
double oracle_dt_crit(int p, double eta, const double *F, int rule)
{
    if (p == 4) return sqrt(eta * (F[0] * F[2] + F[1] * F[1]) / (F[1] * F[3] + F[2] * F[2]));
    /* generalised criterion of order q: dt = eta (A_1 / A_(q-2))^(1/(q-3)),
     * A_k = sqrt(|a^(k-1)| |a^(k+1)|) + |a^(k)| */
    const int q = (rule == 2) ? 4 : p;
    const double A1 = sqrt(F[0] * F[2]) + F[1];
    const double Ak = sqrt(F[q - 3] * F[q - 1]) + F[q - 2];
    return eta * pow(A1 / Ak, 1.0 / (double)(q - 3));
}

/* Block quantisation: the largest power of two 2^-k <= dt_crit with k clamped
 * to [k_min, k_max].  After a step ending at t1 the step may grow by at most a
 * factor two, and only when t1 is a multiple of the doubled step (so that
 * t_i stays a multiple of dt_i); it may shrink by any factor. */
static int level_of(double dt_crit, int k_min, int k_max)
{
    int k = k_min;
    while (k < k_max && !(ldexp(1.0, -k) <= dt_crit)) ++k; /* NaN -> k_max */
    return k;
}

int oracle_new_level(double dt_crit, int level_old, int64_t t1_tick, int k_min, int k_max)
{
    int k = level_of(dt_crit, k_min, k_max);
    if (k >= level_old) return k;                   /* same or smaller step */
    /* wants a larger step: at most one doubling, only if commensurate */
    const int kd = level_old - 1;
    if (kd < k_min) return level_old;
    const int64_t dt2 = (int64_t)1 << (LEVEL_MAX - kd);
    return (t1_tick % dt2 == 0) ? kd : level_old;
}

/* ------------------------------------------------------------------------ */
/* Initialisation at t = 0: pass 1 gives a, jerk from (x, v); pass 2 gives
 * snap, crackle with the a, jerk of pass 1 as inputs.  The state keeps
 * a^(0..p-3): order 4 keeps a, jerk; order 6 also snap and crackle; order 8
 * in addition a^(4), a^(5), started at zero.  The first step follows
 * dt0 = eta_start |a| / |jerk|, quantised without the doubling rule. */
int oracle_init(const oracle_config *c, oracle_state *s)
{
    const int64_t n = s->n;
    const int p = c->order;
    int32_t *all = (int32_t *)malloc(sizeof(int32_t) * n);
    double *a = (double *)malloc(sizeof(double) * 3 * n);
    double *j = (double *)malloc(sizeof(double) * 3 * n);
    double *a2 = (double *)malloc(sizeof(double) * 3 * n);
    double *j2 = (double *)malloc(sizeof(double) * 3 * n);
    double *sn = (double *)malloc(sizeof(double) * 3 * n);
    double *cr = (double *)malloc(sizeof(double) * 3 * n);
    double *zero = (double *)calloc(3 * n, sizeof(double));
    if (!all || !a || !j || !a2 || !j2 || !sn || !cr || !zero) return -1;
    for (int64_t i = 0; i < n; ++i) all[i] = (int32_t)i;
    oracle_config c8 = *c;
    c8.order = 8;
    oracle_force(&c8, n, s->m, s->x, s->v, zero, zero, n, all, a, j, NULL, NULL, NULL);
    oracle_force(&c8, n, s->m, s->x, s->v, a, j, n, all, a2, j2, sn, cr, NULL);
    /* hard pairs, when switched on (after pass 2, which used the Newtonian a, jerk) */
    oracle_pn(c, n, s->m, s->x, s->v, n, all, a, j, p >= 6 ? sn : NULL, p >= 6 ? cr : NULL);
    /* pass 2 recomputes a and jerk identically (they do not depend on a, jerk);
     * the pass-1 values are the ones kept */
    memcpy(s->d[0], a, sizeof(double) * 3 * n);
    memcpy(s->d[1], j, sizeof(double) * 3 * n);
    if (p >= 6) {
        memcpy(s->d[2], sn, sizeof(double) * 3 * n);
        memcpy(s->d[3], cr, sizeof(double) * 3 * n);
    }
    if (p >= 8) {
        memset(s->d[4], 0, sizeof(double) * 3 * n);
        memset(s->d[5], 0, sizeof(double) * 3 * n);
    }
    for (int64_t i = 0; i < n; ++i) {
        double av[3], jv[3];
        for (int k = 0; k < 3; ++k) {
            av[k] = a[k * n + i];
            jv[k] = j[k * n + i];
        }
        const double dt0 = c->eta_start * norm3(av) / norm3(jv);
        s->level[i] = level_of(dt0, c->k_min, c->k_max);
        s->t_tick[i] = 0;
    }
    free(all); free(a); free(j); free(a2); free(j2); free(sn); free(cr); free(zero);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One block step (the hot path, in plain form):
 *   1. t_next = min_i (t_i + dt_i); the active set is every i with
 *      t_i + dt_i == t_next, in increasing index order;
 *   2. predict all particles to t_next;
 *   3. force and derivatives on the active set from the predicted states;
 *   4. correct the active particles; interpolate the higher derivatives;
 *   5. new time step and level;  6. t_i <- t_next.
 * Returns n_act (or -1 on allocation failure); *t_next_out gets the new time.
 * stats (optional, length 2): [0] += number of particles whose level hit
 * k_max because dt_crit was below 2^-k_max, [1] += number of non-finite
 * corrected values. */
int64_t oracle_block_step(const oracle_config *c, oracle_state *s, int64_t *t_next_out, int64_t *stats)
{
    const int64_t n = s->n;
    const int p = c->order, q = p / 2;
    int64_t t_next = INT64_MAX;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t tn = s->t_tick[i] + ((int64_t)1 << (LEVEL_MAX - s->level[i]));
        if (tn < t_next) t_next = tn;
    }
    int32_t *act = (int32_t *)malloc(sizeof(int32_t) * n);
    double *xp = (double *)malloc(sizeof(double) * 3 * n);
    double *vp = (double *)malloc(sizeof(double) * 3 * n);
    double *ap = (double *)malloc(sizeof(double) * 3 * n);
    double *jp = (double *)malloc(sizeof(double) * 3 * n);
    if (!act || !xp || !vp || !ap || !jp) return -1;
    int64_t n_act = 0;
    for (int64_t i = 0; i < n; ++i)
        if (s->t_tick[i] + ((int64_t)1 << (LEVEL_MAX - s->level[i])) == t_next) act[n_act++] = (int32_t)i;

    oracle_predict(c, s, t_next, xp, vp, ap, jp);

    double *F = (double *)malloc(sizeof(double) * 3 * (size_t)n_act * 4);
    double *acc = F, *jrk = F + 3 * n_act, *snp = F + 6 * n_act, *crk = F + 9 * n_act;
    oracle_force(c, n, s->m, xp, vp, ap, jp, n_act, act, acc, jrk, snp, crk, NULL);
    oracle_pn(c, n, s->m, xp, vp, n_act, act, acc, jrk, p >= 6 ? snp : NULL, p >= 8 ? crk : NULL);

    int64_t under = 0, nonfinite = 0;
    int64_t qq;
#pragma omp parallel for schedule(static) reduction(+ : under, nonfinite)
    for (qq = 0; qq < n_act; ++qq) {
        const int64_t i = act[qq];
        const double h = (double)(t_next - s->t_tick[i]) / (double)TICKS_PER_UNIT;
        const double *newd[4] = {acc, jrk, snp, crk};
        double Dall[3][8]; /* a^(0..p-1) at t1 per component */
        for (int k = 0; k < 3; ++k) {
            double D0[4], D1[4], H[4], x1, v1;
            for (int l = 0; l < q; ++l) {
                D0[l] = s->d[l][k * n + i];
                D1[l] = newd[l][k * n_act + qq];
            }
            hermite_correct(p, h, s->x[k * n + i], s->v[k * n + i], D0, D1, &x1, &v1);
            hermite_high(p, h, D0, D1, H);
            s->x[k * n + i] = x1;
            s->v[k * n + i] = v1;
            for (int l = 0; l < q; ++l) Dall[k][l] = D1[l];
            for (int l = 0; l < q; ++l) Dall[k][q + l] = H[l];
            for (int l = 0; l <= p - 3; ++l) s->d[l][k * n + i] = Dall[k][l];
            if (!isfinite(x1) || !isfinite(v1)) ++nonfinite;
        }
        double Fn[8];
        for (int l = 0; l < p; ++l) {
            double w[3] = {Dall[0][l], Dall[1][l], Dall[2][l]};
            Fn[l] = norm3(w);
        }
        const double dtc = oracle_dt_crit(p, c->eta, Fn, c->dt_rule);
        if (!(dtc >= ldexp(1.0, -c->k_max))) ++under;
        s->level[i] = oracle_new_level(dtc, s->level[i], t_next, c->k_min, c->k_max);
        s->t_tick[i] = t_next;
    }
    if (stats) {
        stats[0] += under;
        stats[1] += nonfinite;
    }
    free(F); free(act); free(xp); free(vp); free(ap); free(jp);
    if (t_next_out) *t_next_out = t_next;
    return n_act;
}

/* Integrate with block steps until every particle reaches t_end_tick (a
 * multiple of the largest step) or max_steps block steps were taken.
 * out[0] = block steps taken, out[1] = sum of n_act, out[2] = interactions
 * (sum of n_act * n), out[3] = underflow count, out[4] = non-finite count.
 * nact_hist (optional, 21 entries): histogram of floor(log2(n_act)). */
int oracle_integrate(const oracle_config *c, oracle_state *s, int64_t t_end_tick, int64_t max_steps,
                     int64_t *out, int64_t *nact_hist)
{
    int64_t steps = 0, sum_act = 0, stats[2] = {0, 0};
    for (;;) {
        int64_t tmin = INT64_MAX;
        for (int64_t i = 0; i < s->n; ++i) {
            const int64_t tn = s->t_tick[i] + ((int64_t)1 << (LEVEL_MAX - s->level[i]));
            if (tn < tmin) tmin = tn;
        }
        if (tmin > t_end_tick || steps >= max_steps) break;
        int64_t t_next;
        const int64_t na = oracle_block_step(c, s, &t_next, stats);
        if (na < 0) return -1;
        ++steps;
        sum_act += na;
        if (nact_hist) {
            int b = 0;
            while ((2LL << b) <= na && b < 20) ++b;
            nact_hist[b] += 1;
        }
    }
    if (out) {
        out[0] = steps;
        out[1] = sum_act;
        out[2] = sum_act * s->n;
        out[3] = stats[0];
        out[4] = stats[1];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Energy: kinetic T = sum m v^2 / 2 and potential
 * W = - sum_{i<j} m_i m_j / sqrt(r_ij^2 + eps_ij^2). */
int oracle_energy(const oracle_config *c, int64_t n, const double *m, const double *x, const double *v,
                  double *ekin, double *epot)
{
    double T = 0.0, W = 0.0;
    int64_t i;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : T, W)
    for (i = 0; i < n; ++i) {
        double vi[3] = {v[i], v[n + i], v[2 * n + i]};
        T += 0.5 * m[i] * dot3(vi, vi);
        double wi = 0.0;
        for (int64_t j = i + 1; j < n; ++j) {
            double r[3] = {x[j] - x[i], x[n + j] - x[n + i], x[2 * n + j] - x[2 * n + i]};
            wi -= m[j] / sqrt(dot3(r, r) + pair_eps2(c, i, j));
        }
        W += m[i] * wi;
    }
    *ekin = T;
    *epot = W;
    return 0;
}

/* Number of OpenMP threads the oracle runs with (for reporting). */
int oracle_num_threads(void)
{
    int t = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
#endif
    return t;
}
