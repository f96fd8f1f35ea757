/*
 * CPU oracle for the hybrid symplectic N-body hot path of Mercury-Opal
 * (arXiv 2601.19654).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It is a plain, serial,
 * FP64 reference written from the paper and from the textbook definitions the
 * paper relies on; it shares no code, header, table or constant with the HIP
 * library.  Build flags: -O2 -fno-fast-math -ffp-contract=off.
 *
 * The paper prints no formula.  What it fixes, by section:
 *   Sec. 2.1.1  the integrator is Mercury's second-order mixed-variable
 *               symplectic (hybrid) scheme in democratic-heliocentric
 *               coordinates (heliocentric positions, barycentric velocities);
 *               the Hamiltonian splits into Kepler drift, interaction and
 *               stellar-motion parts; the critical radius is a multiple of the
 *               Hill radius, which is recomputed every step from the
 *               star-planet separation.
 *   Sec. 3.1    force block: per target body, a sum over all source bodies
 *               (skipping the star); Hamiltonian block: velocity update, then
 *               a sum over bodies, then positions; drift block: every body is
 *               propagated on its Kepler orbit about the star, with a
 *               per-body failure flag and a copy of positions and velocities
 *               taken first; encounter block: per body extremes over the
 *               step, widened by the critical radius, then every unordered
 *               pair (i<j) whose minimum separation over the step is at or
 *               below the critical distance is appended to a pair list and
 *               both bodies get flag value 2.
 * Where the paper is silent, the readings used are those listed with each
 * function below (units, changeover function, Hill radius, encounter
 * interpolant, drift formulation, energy, drag).
 *
 * Conventions: bodies are indexed 0..n-1 and exclude the star (the paper's
 * index 1 is the star); position/velocity/acceleration arrays are row-major
 * n x 3.  All pair and body sums are taken in index order with Neumaier
 * compensation, so the oracle's own summation error stays near one ulp.
 *
 * Parity-unpinned parts: gas drag (Sec. 2.1 names aerodynamic drag; the disk
 * model is in a companion paper that is not available).  Its tests pin only
 * limits and closed forms of the formula chosen here.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <float.h>
#include <stdlib.h>

/* ------------------------------------------------------------------ */
/* Compensated (Neumaier) accumulation                                 */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;

static void ns_add(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double ns_val(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Changeover function (Sec. 2.1.1: interaction part trusted only      */
/* outside the critical radius).  Reading: y = (r - f rc)/((1-f) rc),  */
/* K = 0 for y<=0, y^2/(2y^2-2y+1) for 0<y<1, 1 for y>=1, f = inner.   */
/* Returns K and dK/dr.                                                 */
/* ------------------------------------------------------------------ */
void orc_changeover(double r, double rc, double inner, double *K, double *dKdr)
{
    double ri = inner * rc;
    double width = (1.0 - inner) * rc;
    if (r >= rc) {
        *K = 1.0;
        *dKdr = 0.0;
    } else if (r <= ri) {
        *K = 0.0;
        *dKdr = 0.0;
    } else {
        double y = (r - ri) / width;
        double den = 2.0 * y * y - 2.0 * y + 1.0;
        *K = y * y / den;
        *dKdr = 2.0 * y * (1.0 - y) / (den * den * width);
    }
}

/* ------------------------------------------------------------------ */
/* Critical radius (Sec. 2.1.1 footnotes): a multiple n_hill of the     */
/* Hill radius, which depends on the star-planet separation:           */
/* rc_i = n_hill |Q_i| (m_i / (3 m0))^(1/3).                            */
/* ------------------------------------------------------------------ */
void orc_rcrit(int n, double m0, const double *m, const double *Q, double n_hill, double *rc)
{
    for (int i = 0; i < n; ++i) {
        double r = sqrt(Q[3 * i] * Q[3 * i] + Q[3 * i + 1] * Q[3 * i + 1] + Q[3 * i + 2] * Q[3 * i + 2]);
        rc[i] = n_hill * r * cbrt(m[i] / (3.0 * m0));
    }
}

/* ------------------------------------------------------------------ */
/* Interaction acceleration (Sec. 3.1, force block, loop 2).           */
/* a_i = sum_{j != i} G m_j w(r_ij) (Q_j - Q_i),                         */
/* w = K/r^3 - (dK/dr)/r^2 with rc_ij = max(rc_i, rc_j): the exact        */
/* gradient of the potential -G m_i m_j K(r)/r.  Coincident distinct     */
/* bodies (r = 0) contribute nothing; the self term is skipped by index.  */
/* ------------------------------------------------------------------ */
/* Big and small bodies (Sec. 2.1): only the first nbig bodies of a system are
 * gravity sources; the others are massless and feel the big ones only.
 * The acceleration of one target i: the sum over sources j < nbig, j != i,
 * in index order. */
static void force_target(int i, int nbig, double G, double inner, const double *m,
                         const double *Q, const double *rc, double *ai)
{
    nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0};
    for (int j = 0; j < nbig; ++j) {
        if (j == i)
            continue;
        double dx = Q[3 * j] - Q[3 * i];
        double dy = Q[3 * j + 1] - Q[3 * i + 1];
        double dz = Q[3 * j + 2] - Q[3 * i + 2];
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 == 0.0)
            continue;
        double r = sqrt(r2);
        double rcij = rc[i] > rc[j] ? rc[i] : rc[j];
        double K, dK;
        orc_changeover(r, rcij, inner, &K, &dK);
        double w = K / (r2 * r) - dK / r2;
        double f = G * m[j] * w;
        ns_add(&ax, f * dx);
        ns_add(&ay, f * dy);
        ns_add(&az, f * dz);
    }
    ai[0] = ns_val(&ax);
    ai[1] = ns_val(&ay);
    ai[2] = ns_val(&az);
}

/* Every target of the system.  Targets are independent, so the OpenMP build
 * (the threaded CPU baseline) splits them over threads with bit-identical
 * results. */
void orc_force_nb(int n, int nbig, double G, double inner, const double *m, const double *Q,
                  const double *rc, double *a)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int i = 0; i < n; ++i)
        force_target(i, nbig, G, inner, m, Q, rc, a + 3 * i);
}

void orc_force(int n, double G, double inner, const double *m, const double *Q,
               const double *rc, double *a)
{
    orc_force_nb(n, n, G, inner, m, Q, rc, a);
}

/* The same sum for selected targets only (large-N sampled checks): a[k] is
 * the acceleration of body idx[k]. */
void orc_force_subset(int n, int nbig, double G, double inner, const double *m, const double *Q,
                      const double *rc, int k, const int32_t *idx, double *a)
{
    (void)n;
    for (int t = 0; t < k; ++t)
        force_target(idx[t], nbig, G, inner, m, Q, rc, a + 3 * t);
}

/* Interaction kick (Sec. 3.1, Hamiltonian block loop 1): V += h a. */
void orc_kick(int n, double h, const double *a, double *V)
{
    for (int k = 0; k < 3 * n; ++k)
        V[k] += h * a[k];
}

/* Sum of m_i V_i over the system's bodies (Sec. 3.1, Hamiltonian block loop 2). */
void orc_momentum(int n, const double *m, const double *V, double *P)
{
    nsum px = {0, 0}, py = {0, 0}, pz = {0, 0};
    for (int i = 0; i < n; ++i) {
        ns_add(&px, m[i] * V[3 * i]);
        ns_add(&py, m[i] * V[3 * i + 1]);
        ns_add(&pz, m[i] * V[3 * i + 2]);
    }
    P[0] = ns_val(&px);
    P[1] = ns_val(&py);
    P[2] = ns_val(&pz);
}

/* Stellar-motion drift (Hamiltonian block loops 2-3): Q += h P / m0. */
void orc_sun_drift(int n, double h, double m0, const double *m, const double *V, double *Q)
{
    double P[3];
    orc_momentum(n, m, V, P);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k)
            Q[3 * i + k] += h * P[k] / m0;
}

/* Heliocentric -> democratic heliocentric (Sec. 2.1.1 footnote):
 * Q = x_h, V = v_h - sum_j m_j v_h,j / (m0 + sum_j m_j). */
void orc_helio_to_dh(int n, double m0, const double *m, const double *xh, const double *vh,
                     double *Q, double *V)
{
    nsum px = {0, 0}, py = {0, 0}, pz = {0, 0}, mt = {0, 0};
    for (int i = 0; i < n; ++i) {
        ns_add(&px, m[i] * vh[3 * i]);
        ns_add(&py, m[i] * vh[3 * i + 1]);
        ns_add(&pz, m[i] * vh[3 * i + 2]);
        ns_add(&mt, m[i]);
    }
    double M = m0 + ns_val(&mt);
    double c[3] = {ns_val(&px) / M, ns_val(&py) / M, ns_val(&pz) / M};
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            Q[3 * i + k] = xh[3 * i + k];
            V[3 * i + k] = vh[3 * i + k] - c[k];
        }
}

/* Democratic heliocentric -> heliocentric: v_h = V + sum_j m_j V_j / m0. */
void orc_dh_to_helio(int n, double m0, const double *m, const double *Q, const double *V,
                     double *xh, double *vh)
{
    double P[3];
    orc_momentum(n, m, V, P);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            xh[3 * i + k] = Q[3 * i + k];
            vh[3 * i + k] = V[3 * i + k] + P[k] / m0;
        }
}

/* ------------------------------------------------------------------ */
/* Kepler drift (Sec. 2.1 and 3.1: every body follows its Kepler orbit  */
/* about the star for the full step).  Reading: universal-variable      */
/* (Stumpff-function) formulation with mu = G m0.                        */
/* ------------------------------------------------------------------ */

/* Stumpff functions c_k(z) = sum_n (-z)^n / (2n+k)!, k = 0..3.
 * Power series for |z| <= 1, trigonometric / hyperbolic closed forms beyond. */
void orc_stumpff(double z, double c[4])
{
    if (fabs(z) <= 1.0) {
        /* c0 and c1 from their series; c2, c3 likewise (independent sums). */
        for (int k = 0; k < 4; ++k) {
            double term = 1.0;
            for (int j = 2; j <= k; ++j)
                term /= (double)j;               /* 1/k! */
            double s = term;
            for (int nn = 1; nn < 40; ++nn) {
                term *= -z / ((double)(2 * nn + k - 1) * (double)(2 * nn + k));
                double s2 = s + term;
                if (s2 == s)
                    break;
                s = s2;
            }
            c[k] = s;
        }
    } else if (z > 0.0) {
        double x = sqrt(z);
        c[0] = cos(x);
        c[1] = sin(x) / x;
        c[2] = (1.0 - c[0]) / z;
        c[3] = (1.0 - c[1]) / z;
    } else {
        double x = sqrt(-z);
        c[0] = cosh(x);
        c[1] = sinh(x) / x;
        c[2] = (1.0 - c[0]) / z;
        c[3] = (1.0 - c[1]) / z;
    }
}

/* G_k(s) = s^k c_k(beta s^2), k = 0..3 */
static void gfun(double beta, double s, double G[4])
{
    double c[4];
    orc_stumpff(beta * s * s, c);
    G[0] = c[0];
    G[1] = s * c[1];
    G[2] = s * s * c[2];
    G[3] = s * s * s * c[3];
}

/* Propagate one body on its Kepler orbit (mu = G m0) for time tau.
 * Solves F(s) = r0 s + eta0 G2(s) + zeta0 G3(s) - tau = 0 (F' = r > 0, so the
 * root is unique) by Newton's method kept inside a bracket, with bisection
 * whenever a Newton step leaves it; converged at |ds| <= 4u|s|; at most 100
 * iterations.  On failure the body is left unchanged and 1 is returned. */
int orc_kepler_drift(double mu, double tau, double *q, double *v)
{
    if (tau == 0.0)
        return 0;
    double r0 = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double eta0 = q[0] * v[0] + q[1] * v[1] + q[2] * v[2];
    double beta = 2.0 * mu / r0 - v2;
    double zeta0 = mu - beta * r0;
    if (!(r0 > 0.0) || !isfinite(r0) || !isfinite(v2))
        return 1;

    double G[4];
    /* bracket [lo, hi] with F(lo) <= 0 <= F(hi); F(0) = -tau */
    double lo, hi;
    double s = tau / r0;
    if (tau > 0.0) {
        lo = 0.0;
        hi = s;
        for (int k = 0; k < 200; ++k) {
            gfun(beta, hi, G);
            double F = r0 * hi + eta0 * G[2] + zeta0 * G[3] - tau;
            if (F >= 0.0 || !isfinite(F))
                break;
            lo = hi;
            hi *= 2.0;
        }
    } else {
        hi = 0.0;
        lo = s;
        for (int k = 0; k < 200; ++k) {
            gfun(beta, lo, G);
            double F = r0 * lo + eta0 * G[2] + zeta0 * G[3] - tau;
            if (F <= 0.0 || !isfinite(F))
                break;
            hi = lo;
            lo *= 2.0;
        }
    }
    if (!(s > lo && s < hi))
        s = 0.5 * (lo + hi);

    const double tol = 4.0 * (0.5 * DBL_EPSILON);   /* 4u */
    int ok = 0;
    for (int it = 0; it < 100; ++it) {
        gfun(beta, s, G);
        double F = r0 * s + eta0 * G[2] + zeta0 * G[3] - tau;
        double dF = r0 + eta0 * G[1] + zeta0 * G[2];   /* = r(s) */
        if (F == 0.0) {
            ok = 1;
            break;
        }
        if (F < 0.0)
            lo = s;
        else
            hi = s;
        double sn = (isfinite(F) && dF > 0.0) ? s - F / dF : 0.5 * (lo + hi);
        if (!(sn > lo && sn < hi))
            sn = 0.5 * (lo + hi);             /* bisection fallback */
        double ds = sn - s;
        s = sn;
        if (fabs(ds) <= tol * fabs(s) || (hi - lo) <= tol * fabs(s)) {
            ok = 1;
            break;
        }
    }
    if (!ok)
        return 1;

    gfun(beta, s, G);
    double r = r0 + eta0 * G[1] + zeta0 * G[2];
    double f = 1.0 - mu * G[2] / r0;
    double g = tau - mu * G[3];
    double fd = -mu * G[1] / (r * r0);
    double gd = 1.0 - mu * G[2] / r;
    double qn[3], vn[3];
    for (int k = 0; k < 3; ++k) {
        qn[k] = f * q[k] + g * v[k];
        vn[k] = fd * q[k] + gd * v[k];
    }
    if (!isfinite(qn[0] + qn[1] + qn[2] + vn[0] + vn[1] + vn[2]))
        return 1;
    memcpy(q, qn, sizeof qn);
    memcpy(v, vn, sizeof vn);
    return 0;
}

/* Drift every body of a system; returns the number of failures and sets
 * flag[i] = 1 for each (those bodies keep their pre-drift state). */
int orc_drift(int n, double mu, double tau, double *Q, double *V, int32_t *flag)
{
    int nfail = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nfail)
#endif
    for (int i = 0; i < n; ++i) {
        int f = orc_kepler_drift(mu, tau, Q + 3 * i, V + 3 * i);
        if (flag)
            flag[i] = f;
        nfail += f;
    }
    return nfail;
}

/* ------------------------------------------------------------------ */
/* Close-encounter predicate (Sec. 3.1, encounter block).  Reading: the  */
/* squared separation d2(s), s in [0,1] over the step, is the cubic       */
/* Hermite interpolant through f0 = |dQ0|^2, f1 = |dQ1|^2 with slopes      */
/* g0 = 2 tau dQ0.dV0, g1 = 2 tau dQ1.dV1 (d = body j minus body i); its   */
/* minimum over [0,1], clamped at 0, is the pair's minimum separation      */
/* squared.  A pair i<j is flagged iff that minimum <= rc_ij^2 with        */
/* rc_ij = max(rc_i, rc_j).                                                 */
/* ------------------------------------------------------------------ */
double orc_pair_min_d2(double tau, const double *q0i, const double *v0i, const double *q1i,
                       const double *v1i, const double *q0j, const double *v0j,
                       const double *q1j, const double *v1j)
{
    double d0[3], e0[3], d1[3], e1[3];
    for (int k = 0; k < 3; ++k) {
        d0[k] = q0j[k] - q0i[k];
        e0[k] = v0j[k] - v0i[k];
        d1[k] = q1j[k] - q1i[k];
        e1[k] = v1j[k] - v1i[k];
    }
    double f0 = d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2];
    double f1 = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
    double g0 = 2.0 * tau * (d0[0] * e0[0] + d0[1] * e0[1] + d0[2] * e0[2]);
    double g1 = 2.0 * tau * (d1[0] * e1[0] + d1[1] * e1[1] + d1[2] * e1[2]);
    /* power-basis coefficients of the Hermite cubic */
    double c0 = f0, c1 = g0;
    double c2 = -3.0 * f0 - 2.0 * g0 + 3.0 * f1 - g1;
    double c3 = 2.0 * f0 + g0 - 2.0 * f1 + g1;
    double fmin = f0 < f1 ? f0 : f1;
    /* stationary points: 3 c3 s^2 + 2 c2 s + c1 = 0 */
    double A = 3.0 * c3, B = 2.0 * c2, C = c1;
    double roots[2];
    int nr = 0;
    if (A == 0.0) {
        if (B != 0.0)
            roots[nr++] = -C / B;
    } else {
        double disc = B * B - 4.0 * A * C;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double qq = -0.5 * (B + (B >= 0.0 ? sq : -sq));
            if (qq != 0.0) {
                roots[nr++] = qq / A;
                roots[nr++] = C / qq;
            } else {
                roots[nr++] = 0.0;
            }
        }
    }
    for (int k = 0; k < nr; ++k) {
        double s = roots[k];
        if (s > 0.0 && s < 1.0) {
            double fs = c0 + s * (c1 + s * (c2 + s * c3));
            if (fs < fmin)
                fmin = fs;
        }
    }
    return fmin > 0.0 ? fmin : 0.0;
}

/* The pair (i, j), i < j: its minimum squared separation over the step and
 * the threshold rc_ij^2, rc_ij = max(rc_i, rc_j).  Flagged iff d2 <= thr. */
static void pair_test(int i, int j, double tau, const double *Q0, const double *V0,
                      const double *Q1, const double *V1, const double *rc, double *d2,
                      double *thr)
{
    *d2 = orc_pair_min_d2(tau, Q0 + 3 * i, V0 + 3 * i, Q1 + 3 * i, V1 + 3 * i, Q0 + 3 * j,
                          V0 + 3 * j, Q1 + 3 * j, V1 + 3 * j);
    double rcij = rc[i] > rc[j] ? rc[i] : rc[j];
    *thr = rcij * rcij;
}

/* All unordered pairs i<j of one system.  Flagged pairs go to (ice, jce) in
 * (i, j) lexicographic order (up to cap entries; the true count is returned
 * in *nce); ce[i] = ce[j] = 2 for flagged bodies, 0 otherwise.  Pairs whose
 * minimum lies within tie*rc_ij^2 of the threshold are reported in
 * (tie_i, tie_j) (up to tie_cap; true count in *ntie).
 * With nbig < n the bodies from nbig on are small: two small bodies do not
 * interact (Sec. 2.1), so only pairs with i < nbig are tested (i < j).
 * Rows i are independent: the OpenMP build tests them on several threads and
 * appends each row's hits in row order (an ordered section), so the list is
 * the same as the serial one. */
void orc_encounters_nb(int n, int nbig, double tau, const double *Q0, const double *V0,
                       const double *Q1, const double *V1, const double *rc, int cap,
                       int32_t *ice, int32_t *jce, int32_t *ce, int *nce, double tie,
                       int tie_cap, int32_t *tie_i, int32_t *tie_j, int *ntie)
{
    int cnt = 0, tcnt = 0;
    for (int i = 0; i < n; ++i)
        ce[i] = 0;
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        /* one row's hits (2 bits per source: flagged, in the tie band) */
        unsigned char *row = (unsigned char *)malloc(n > 0 ? (size_t)n : 1);
#ifdef _OPENMP
#pragma omp for ordered schedule(static, 1)
#endif
        for (int i = 0; i < nbig; ++i) {
            for (int j = i + 1; j < n; ++j) {
                double d2, thr;
                pair_test(i, j, tau, Q0, V0, Q1, V1, rc, &d2, &thr);
                row[j] = (unsigned char)((d2 <= thr ? 1 : 0) | (fabs(d2 - thr) <= tie * thr ? 2 : 0));
            }
#ifdef _OPENMP
#pragma omp ordered
#endif
            for (int j = i + 1; j < n; ++j) {
                if (row[j] & 1) {
                    if (cnt < cap) {
                        ice[cnt] = i;
                        jce[cnt] = j;
                    }
                    ++cnt;
                    ce[i] = 2;
                    ce[j] = 2;
                }
                if (row[j] & 2) {
                    if (tcnt < tie_cap) {
                        tie_i[tcnt] = i;
                        tie_j[tcnt] = j;
                    }
                    ++tcnt;
                }
            }
        }
        free(row);
    }
    *nce = cnt;
    *ntie = tcnt;
}

void orc_encounters(int n, double tau, const double *Q0, const double *V0, const double *Q1,
                    const double *V1, const double *rc, int cap, int32_t *ice, int32_t *jce,
                    int32_t *ce, int *nce, double tie, int tie_cap, int32_t *tie_i,
                    int32_t *tie_j, int *ntie)
{
    orc_encounters_nb(n, n, tau, Q0, V0, Q1, V1, rc, cap, ice, jce, ce, nce, tie, tie_cap, tie_i,
                      tie_j, ntie);
}

/* One body i against every other body j of the system (large-N sampled
 * checks): flag[j] = 1 if the pair (min(i,j), max(i,j)) is flagged by the same
 * predicate, tie[j] = 1 if its minimum lies in the tie band. */
void orc_pair_scan(int n, int nbig, double tau, const double *Q0, const double *V0,
                   const double *Q1, const double *V1, const double *rc, int i, double tie,
                   int32_t *flag, int32_t *tieflag)
{
    for (int j = 0; j < n; ++j) {
        flag[j] = 0;
        tieflag[j] = 0;
        if (j == i || (i >= nbig && j >= nbig))
            continue;
        double d2, thr;
        pair_test(i < j ? i : j, i < j ? j : i, tau, Q0, V0, Q1, V1, rc, &d2, &thr);
        flag[j] = d2 <= thr;
        tieflag[j] = fabs(d2 - thr) <= tie * thr;
    }
}

/* ------------------------------------------------------------------ */
/* Energy, angular momentum and stellar momentum (Sec. 2.1.1, energy    */
/* and momentum routine).  In DH variables:                              */
/*  E  = sum m|V|^2/2 + |P|^2/(2 m0) - sum G m0 m_i/|Q_i|                  */
/*       - sum_{i<j} G m_i m_j / r_ij                                      */
/*  EK = the same with each pair term weighted by K(r_ij; rc_ij)          */
/*  L  = sum m_i Q_i x V_i,   P = sum m_i V_i                              */
/* ------------------------------------------------------------------ */
void orc_energy(int n, double G, double m0, double inner, const double *m, const double *Q,
                const double *V, const double *rc, double *E, double *EK, double *L, double *P)
{
    nsum kin = {0, 0}, star = {0, 0}, pair = {0, 0}, pairk = {0, 0};
    nsum lx = {0, 0}, ly = {0, 0}, lz = {0, 0};
    orc_momentum(n, m, V, P);
    for (int i = 0; i < n; ++i) {
        const double *q = Q + 3 * i, *v = V + 3 * i;
        ns_add(&kin, 0.5 * m[i] * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
        double r = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        ns_add(&star, -G * m0 * m[i] / r);
        ns_add(&lx, m[i] * (q[1] * v[2] - q[2] * v[1]));
        ns_add(&ly, m[i] * (q[2] * v[0] - q[0] * v[2]));
        ns_add(&lz, m[i] * (q[0] * v[1] - q[1] * v[0]));
    }
    for (int i = 0; i < n; ++i) {
        for (int j = i + 1; j < n; ++j) {
            double dx = Q[3 * j] - Q[3 * i];
            double dy = Q[3 * j + 1] - Q[3 * i + 1];
            double dz = Q[3 * j + 2] - Q[3 * i + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r == 0.0)
                continue;
            double u = -G * m[i] * m[j] / r;
            double rcij = rc[i] > rc[j] ? rc[i] : rc[j];
            double K, dK;
            orc_changeover(r, rcij, inner, &K, &dK);
            ns_add(&pair, u);
            ns_add(&pairk, K * u);
        }
    }
    double sun = (P[0] * P[0] + P[1] * P[1] + P[2] * P[2]) / (2.0 * m0);
    nsum e = kin;
    ns_add(&e, star.s);
    ns_add(&e, star.c);
    ns_add(&e, sun);
    nsum ek = e;
    ns_add(&e, pair.s);
    ns_add(&e, pair.c);
    ns_add(&ek, pairk.s);
    ns_add(&ek, pairk.c);
    *E = ns_val(&e);
    *EK = ns_val(&ek);
    L[0] = ns_val(&lx);
    L[1] = ns_val(&ly);
    L[2] = ns_val(&lz);
}

/* ------------------------------------------------------------------ */
/* Aerodynamic gas drag (Sec. 2.1 names it; the disk model itself is    */
/* not in the paper).  PARITY UNPINNED BY THE PAPER.  Reading: quadratic */
/* drag a = -k |u| u with u = v_helio - v_gas, k = 3 C_D rho_g/(8 rho_p s),*/
/* s = (3 m/(4 pi rho_p))^(1/3); rho_g = Sigma(R)/(sqrt(2 pi) H)           */
/* exp(-z^2/(2H^2)), Sigma(R) = sigma0 (R/1)^-1, H = h R;                   */
/* v_gas = sqrt(1 - 3 h^2) sqrt(G m0/R) phi_hat (R cylindrical).            */
/* ------------------------------------------------------------------ */
void orc_drag_accel(int n, double G, double m0, const double *m, const double *Q,
                    const double *V, const double *P, double sigma0, double h, double cd,
                    double rho_p, double *ad)
{
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        const double *q = Q + 3 * i;
        double vh[3];
        for (int k = 0; k < 3; ++k)
            vh[k] = V[3 * i + k] + P[k] / m0;
        double R = sqrt(q[0] * q[0] + q[1] * q[1]);
        double H = h * R;
        double sig = sigma0 / R;
        double rho = sig / (sqrt(2.0 * pi) * H) * exp(-q[2] * q[2] / (2.0 * H * H));
        double vk = sqrt(G * m0 / R) * sqrt(1.0 - 3.0 * h * h);
        double vg[3] = {-vk * q[1] / R, vk * q[0] / R, 0.0};
        double u[3] = {vh[0] - vg[0], vh[1] - vg[1], vh[2] - vg[2]};
        double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double s = cbrt(3.0 * m[i] / (4.0 * pi * rho_p));
        double k = (m[i] > 0.0 && sigma0 > 0.0) ? 3.0 * cd * rho / (8.0 * rho_p * s) : 0.0;
        for (int c = 0; c < 3; ++c)
            ad[3 * i + c] = -k * um * u[c];
    }
}

/* Kick including drag evaluated with the current velocities. */
void orc_kick_drag(int n, double h, double G, double m0, const double *m, const double *Q,
                   const double *a, double *V, double sigma0, double hr, double cd, double rho_p,
                   double *scratch /* 3n */)
{
    double P[3];
    orc_momentum(n, m, V, P);
    orc_drag_accel(n, G, m0, m, Q, V, P, sigma0, hr, cd, rho_p, scratch);
    for (int k = 0; k < 3 * n; ++k)
        V[k] += h * (a[k] + scratch[k]);
}

/* ------------------------------------------------------------------ */
/* One hybrid step of one system in hot-path mode (no close-encounter    */
/* resolution): K(h) S(h) D(tau) C S(h) [rc, force] K(h), h = tau/2.     */
/* On entry a and rc hold the force and critical radii at the current Q   */
/* (first-same-as-last); on exit they hold those at the new Q.            */
/* Q0, V0 receive the pre-drift copies; the encounter outputs are those    */
/* of orc_encounters.  Returns the number of Kepler failures.              */
/* ------------------------------------------------------------------ */
int orc_step(int n, int nbig, double G, double m0, double n_hill, double inner, const double *m,
             double *Q, double *V, double *a, double *rc, double tau, int drag, double sigma0,
             double hr, double cd, double rho_p, double *Q0, double *V0, int32_t *kflag,
             double *scratch, int cap, int32_t *ice, int32_t *jce, int32_t *ce, int *nce)
{
    double h = 0.5 * tau;
    if (drag)
        orc_kick_drag(n, h, G, m0, m, Q, a, V, sigma0, hr, cd, rho_p, scratch);
    else
        orc_kick(n, h, a, V);
    orc_sun_drift(n, h, m0, m, V, Q);
    memcpy(Q0, Q, sizeof(double) * 3 * n);
    memcpy(V0, V, sizeof(double) * 3 * n);
    int nfail = orc_drift(n, G * m0, tau, Q, V, kflag);
    int ntie = 0;
    int32_t ti = 0, tj = 0;
    orc_encounters_nb(n, nbig, tau, Q0, V0, Q, V, rc, cap, ice, jce, ce, nce, 0.0, 0, &ti, &tj,
                      &ntie);
    orc_sun_drift(n, h, m0, m, V, Q);
    orc_rcrit(n, m0, m, Q, n_hill, rc);
    orc_force_nb(n, nbig, G, inner, m, Q, rc, a);
    if (drag)
        orc_kick_drag(n, h, G, m0, m, Q, a, V, sigma0, hr, cd, rho_p, scratch);
    else
        orc_kick(n, h, a, V);
    return nfail;
}

/* ------------------------------------------------------------------ */
/* Close-encounter resolution, the full hybrid method (Sec. 2.1.1,     */
/* footnote on the critical radius: inside it the interaction and the   */
/* Kepler parts of the bodies involved are advanced by Bulirsch-Stoer;  */
/* Sec. 3 and 3.2: that integration runs on the host after the bodies   */
/* are restored to their state before the drift).                       */
/*                                                                      */
/* Readings.  Flagged pairs join bodies into groups (connected          */
/* components of the pair graph; members in index order, groups ordered */
/* by their smallest member).  Each group restarts from (Q0, V0) and     */
/* follows, for the whole step tau, the flow of                          */
/*   H0 = sum_i [m_i |V_i|^2 / 2 - G m0 m_i / |Q_i|]                    */
/*        - sum_{i<j in the group} G m_i m_j (1 - K(r_ij)) / r_ij,       */
/* the part of the Hamiltonian the Kepler drift leaves out inside the    */
/* changeover zone:                                                      */
/*   dQ_i/dt = V_i,                                                      */
/*   dV_i/dt = -G m0 Q_i / |Q_i|^3                                       */
/*             + sum_j G m_j [(1 - K)/r^3 + (dK/dr)/r^2] (Q_j - Q_i),    */
/* with rc_ij = max(rc_i, rc_j) from the step's encounter check.         */
/* Integrator: Gragg's modified midpoint rule with polynomial            */
/* extrapolation in h^2 (Bulirsch-Stoer), substeps 2, 4, 6, ..., 16;     */
/* error of a column = largest per-body |dQ|/|Q| or |dV|/|V| between the  */
/* last two extrapolants; a step is taken when that error <= tol, and   */
/* the next step length scales by 0.94 (0.65 tol/err)^(1/(2k+1)),        */
/* clamped to [0.02, 4].                                                 */
/* ------------------------------------------------------------------ */
#define ORC_BS_COLS 8
#define ORC_BS_MAXSTEPS 100000

/* y holds, per member b, Q at y[6b..6b+2] and V at y[6b+3..6b+5]. */
static void h0_deriv(int k, double G, double m0, double inner, const double *m, const double *rc,
                     const double *y, double *dy)
{
    for (int b = 0; b < k; ++b) {
        const double *q = y + 6 * b;
        double r2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
        double r = sqrt(r2);
        double c = -G * m0 / (r2 * r);
        nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0};
        ns_add(&ax, c * q[0]);
        ns_add(&ay, c * q[1]);
        ns_add(&az, c * q[2]);
        for (int o = 0; o < k; ++o) {
            if (o == b)
                continue;
            const double *p = y + 6 * o;
            double dx = p[0] - q[0], dy_ = p[1] - q[1], dz = p[2] - q[2];
            double s2 = dx * dx + dy_ * dy_ + dz * dz;
            if (s2 == 0.0)
                continue;
            double s = sqrt(s2);
            double K, dK;
            orc_changeover(s, fmax(rc[b], rc[o]), inner, &K, &dK);
            double w = G * m[o] * ((1.0 - K) / (s2 * s) + dK / s2);
            ns_add(&ax, w * dx);
            ns_add(&ay, w * dy_);
            ns_add(&az, w * dz);
        }
        dy[6 * b] = y[6 * b + 3];
        dy[6 * b + 1] = y[6 * b + 4];
        dy[6 * b + 2] = y[6 * b + 5];
        dy[6 * b + 3] = ns_val(&ax);
        dy[6 * b + 4] = ns_val(&ay);
        dy[6 * b + 5] = ns_val(&az);
    }
}

/* Gragg's modified midpoint rule: nsub substeps of H from y0 into out.
 * z, zp, f are scratch of 6k doubles each. */
static void modified_midpoint(int k, double G, double m0, double inner, const double *m,
                              const double *rc, const double *y0, double H, int nsub, double *out,
                              double *zp, double *z, double *f)
{
    const int d = 6 * k;
    double h = H / nsub;
    h0_deriv(k, G, m0, inner, m, rc, y0, f);
    for (int c = 0; c < d; ++c) {
        zp[c] = y0[c];
        z[c] = y0[c] + h * f[c];
    }
    for (int s = 1; s < nsub; ++s) {
        h0_deriv(k, G, m0, inner, m, rc, z, f);
        for (int c = 0; c < d; ++c) {
            double zn = zp[c] + 2.0 * h * f[c];
            zp[c] = z[c];
            z[c] = zn;
        }
    }
    h0_deriv(k, G, m0, inner, m, rc, z, f);
    for (int c = 0; c < d; ++c)
        out[c] = 0.5 * (z[c] + zp[c] + h * f[c]);
}

/* Largest per-body relative difference of positions and velocities. */
static double bs_err(int k, const double *a, const double *b)
{
    double e = 0.0;
    for (int i = 0; i < k; ++i) {
        for (int part = 0; part < 2; ++part) {
            const double *x = a + 6 * i + 3 * part, *y = b + 6 * i + 3 * part;
            double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
            double nd = sqrt(dx * dx + dy * dy + dz * dz);
            double nx = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
            double q = nx > 0.0 ? nd / nx : nd;
            if (!(q <= e))
                e = q;            /* also takes a NaN */
        }
    }
    return e;
}

/* Advance one group (k members, state y in the layout above) by tau under
 * H0 with relative tolerance tol.  work holds orc_bs_work_doubles(k)
 * doubles.  Returns 0, or 1 when the step count limit or a non-finite
 * state ends the integration (y is then left unchanged). */
int orc_bs_work_doubles(int k) { return (2 * ORC_BS_COLS + 4) * 6 * k; }

int orc_bs_h0(int k, double G, double m0, double inner, const double *m, const double *rc,
              double tau, double tol, double *y, double *work, int *nsteps_out)
{
    const int d = 6 * k;
    /* extrapolation tableau, two rows: prev[j] = T(c-1, j), cur[j] = T(c, j) */
    double *prev = work, *cur = prev + ORC_BS_COLS * d;
    double *zp = cur + ORC_BS_COLS * d, *z = zp + d, *f = z + d, *yc = f + d;
    memcpy(yc, y, sizeof(double) * d);
    double t = 0.0, H = tau;
    int nsteps = 0;
    while (t != tau) {
        if (++nsteps > ORC_BS_MAXSTEPS)
            return 1;
        double rem = tau - t;
        int last = fabs(H) >= fabs(rem);
        if (last)
            H = rem;
        int accepted = 0;
        double fac = 0.25;
        for (int c = 0; c < ORC_BS_COLS; ++c) {
            const int nc = 2 * (c + 1);                  /* substeps of row c */
            modified_midpoint(k, G, m0, inner, m, rc, yc, H, nc, cur, zp, z, f);
            for (int j = 1; j <= c; ++j) {
                double ratio = (double)nc / (double)(2 * (c - j + 1));
                double den = ratio * ratio - 1.0;
                for (int e = 0; e < d; ++e)
                    cur[j * d + e] = cur[(j - 1) * d + e] +
                                     (cur[(j - 1) * d + e] - prev[(j - 1) * d + e]) / den;
            }
            if (c > 0) {
                double err = bs_err(k, cur + c * d, cur + (c - 1) * d) / tol;
                if (!isfinite(err))
                    break;
                double g = (err > 0.0) ? 0.94 * pow(0.65 / err, 1.0 / (2 * c + 1)) : 4.0;
                if (err <= 1.0) {
                    fac = fmin(4.0, fmax(0.02, g));
                    memcpy(yc, cur + c * d, sizeof(double) * d);
                    accepted = 1;
                    break;
                }
                fac = fmin(0.5, fmax(0.02, g));
            }
            double *sw = prev;
            prev = cur;
            cur = sw;
        }
        if (accepted)
            t = last ? tau : t + H;
        H *= fac;
        for (int e = 0; e < d; ++e)
            if (!isfinite(yc[e]))
                return 1;
    }
    memcpy(y, yc, sizeof(double) * d);
    if (nsteps_out)
        *nsteps_out = nsteps;
    return 0;
}

/* Connected components of the pair graph over n bodies: comp[i] is the
 * smallest member of body i's group, or -1 for a body in no pair. */
static int find_root(int32_t *parent, int i)
{
    while (parent[i] != i)
        i = parent[i];
    return i;
}

/* Resolve every group of one system: members restart from (Q0, V0) and are
 * advanced by tau under H0; the others keep (Q, V).  comp (n ints) receives
 * each body's group label (its smallest member) or -1.  work holds
 * orc_resolve_work_doubles(n) doubles.  Returns the number of groups whose
 * integration failed; their members keep the Kepler-drifted state. */
int orc_resolve_work_doubles(int n) { return orc_bs_work_doubles(n) + 6 * n + 2 * n; }

int orc_resolve(int n, double G, double m0, double inner, const double *m, const double *rc,
                double tau, double tol, const double *Q0, const double *V0, int nce,
                const int32_t *ice, const int32_t *jce, double *Q, double *V, int32_t *comp,
                double *work, int *ngroups_out, int *max_steps_out)
{
    for (int i = 0; i < n; ++i)
        comp[i] = i;
    int32_t *inpair = (int32_t *)(work + orc_bs_work_doubles(n) + 6 * n);
    for (int i = 0; i < n; ++i)
        inpair[i] = 0;
    for (int p = 0; p < nce; ++p) {
        int a = find_root(comp, ice[p]), b = find_root(comp, jce[p]);
        inpair[ice[p]] = inpair[jce[p]] = 1;
        if (a != b) {
            if (a < b)
                comp[b] = a;
            else
                comp[a] = b;
        }
    }
    for (int i = 0; i < n; ++i)
        comp[i] = inpair[i] ? find_root(comp, i) : -1;
    double *y = work + orc_bs_work_doubles(n);
    double *gm = (double *)malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
    int *mem = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int nfail = 0, ngroups = 0, maxst = 0;
    for (int root = 0; root < n; ++root) {
        if (comp[root] != root)
            continue;
        int k = 0;
        for (int i = root; i < n; ++i)
            if (comp[i] == root)
                mem[k++] = i;
        for (int b = 0; b < k; ++b) {
            int i = mem[b];
            memcpy(y + 6 * b, Q0 + 3 * i, 3 * sizeof(double));
            memcpy(y + 6 * b + 3, V0 + 3 * i, 3 * sizeof(double));
            gm[b] = m[i];
            gm[n + b] = rc[i];
        }
        int st = 0;
        int fail = orc_bs_h0(k, G, m0, inner, gm, gm + n, tau, tol, y, work, &st);
        ++ngroups;
        if (st > maxst)
            maxst = st;
        if (fail) {
            ++nfail;
            continue;
        }
        for (int b = 0; b < k; ++b) {
            int i = mem[b];
            memcpy(Q + 3 * i, y + 6 * b, 3 * sizeof(double));
            memcpy(V + 3 * i, y + 6 * b + 3, 3 * sizeof(double));
        }
    }
    free(gm);
    free(mem);
    if (ngroups_out)
        *ngroups_out = ngroups;
    if (max_steps_out)
        *max_steps_out = maxst;
    return nfail;
}

/* One step of the full hybrid method: the hot-path step with the flagged
 * groups resolved between the encounter check and the second stellar drift.
 * Returns Kepler failures + resolver failures (the latter also in *bsfail). */
int orc_step_full(int n, int nbig, double G, double m0, double n_hill, double inner, const double *m,
                  double *Q, double *V, double *a, double *rc, double tau, int drag, double sigma0,
                  double hr, double cd, double rho_p, double tol, double *Q0, double *V0,
                  int32_t *kflag, double *scratch, int cap, int32_t *ice, int32_t *jce, int32_t *ce,
                  int *nce, int32_t *comp, double *work, int *bsfail, int *ngroups)
{
    double h = 0.5 * tau;
    if (drag)
        orc_kick_drag(n, h, G, m0, m, Q, a, V, sigma0, hr, cd, rho_p, scratch);
    else
        orc_kick(n, h, a, V);
    orc_sun_drift(n, h, m0, m, V, Q);
    memcpy(Q0, Q, sizeof(double) * 3 * n);
    memcpy(V0, V, sizeof(double) * 3 * n);
    int nfail = orc_drift(n, G * m0, tau, Q, V, kflag);
    int ntie = 0;
    int32_t ti = 0, tj = 0;
    orc_encounters_nb(n, nbig, tau, Q0, V0, Q, V, rc, cap, ice, jce, ce, nce, 0.0, 0, &ti, &tj,
                      &ntie);
    int k = *nce < cap ? *nce : cap;
    *bsfail = orc_resolve(n, G, m0, inner, m, rc, tau, tol, Q0, V0, k, ice, jce, Q, V, comp, work,
                          ngroups, NULL);
    orc_sun_drift(n, h, m0, m, V, Q);
    orc_rcrit(n, m0, m, Q, n_hill, rc);
    orc_force_nb(n, nbig, G, inner, m, Q, rc, a);
    if (drag)
        orc_kick_drag(n, h, G, m0, m, Q, a, V, sigma0, hr, cd, rho_p, scratch);
    else
        orc_kick(n, h, a, V);
    return nfail + *bsfail;
}

/* ------------------------------------------------------------------ */
/* Collisions, star impacts, ejections and the removal of lost bodies    */
/* (Sec. 2.1.1: physical radii from mce_init, mxx_elim; Sec. 2.1.2:      */
/* mce_coll for planet-planet and planet-star collisions, ejections      */
/* checked every 200 yr for bodies beyond 400 AU).  The paper names the  */
/* events and their schedule, not their arithmetic; the readings used:    */
/*  - physical radius R = (3 m/(4 pi rho))^(1/3), one bulk density rho;    */
/*  - star impact: the body's Kepler arc of the step's drift comes within  */
/*    r_star of the star; the impactors' mass joins the star, whose        */
/*    centre moves to the centre of mass of star and impactors (so every   */
/*    other heliocentric position shifts by minus that displacement);      */
/*  - collision: a flagged pair of the step whose minimum separation over  */
/*    the step (the encounter predicate's Hermite minimum) is at most      */
/*    R_i + R_j; bodies joined by colliding pairs merge perfectly into the */
/*    smallest index: summed mass, mass-weighted position and velocity;    */
/*  - ejection: heliocentric distance beyond r_eject; the body leaves, and */
/*    the barycentric velocities of the rest follow the new barycentre.    */
/* ------------------------------------------------------------------ */
void orc_phys_radius(int n, const double *m, double rho, double *R)
{
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i)
        R[i] = cbrt(3.0 * m[i] / (4.0 * pi * rho));
}

/* Closest approach to the star along the Kepler arc of duration tau from
 * (q0, v0) to (q1, v1) (mu = G m0): the smaller end distance, or the
 * pericentre distance q = h^2 / (mu (1 + e)) when the arc passes a pericentre.
 * Bound orbits: the arc covers the mean anomalies from M0 to M0 + n tau, and a
 * pericentre lies at every multiple of 2 pi; unbound orbits have one
 * pericentre, where the radial velocity turns from inward to outward. */
double orc_star_min(double mu, double tau, const double *q0, const double *v0, const double *q1,
                    const double *v1)
{
    const double pi = 3.14159265358979323846;
    double r0 = sqrt(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2]);
    double r1 = sqrt(q1[0] * q1[0] + q1[1] * q1[1] + q1[2] * q1[2]);
    double rmin = r0 < r1 ? r0 : r1;
    double eta0 = q0[0] * v0[0] + q0[1] * v0[1] + q0[2] * v0[2];
    double eta1 = q1[0] * v1[0] + q1[1] * v1[1] + q1[2] * v1[2];
    double hx = q0[1] * v0[2] - q0[2] * v0[1];
    double hy = q0[2] * v0[0] - q0[0] * v0[2];
    double hz = q0[0] * v0[1] - q0[1] * v0[0];
    double h2 = hx * hx + hy * hy + hz * hz;
    double v2 = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
    double alpha = 2.0 / r0 - v2 / mu;                  /* 1/a */
    double ecosE = 1.0 - r0 * alpha;
    double e2 = 1.0 - h2 * alpha / mu;
    double e = sqrt(e2 > 0.0 ? e2 : 0.0);
    int passed;
    if (alpha > 0.0) {
        /* eccentric anomaly E0 and mean anomaly M0 = E0 - e sin E0 at the start */
        double esinE = eta0 * sqrt(alpha / mu);
        double E0 = atan2(esinE, ecosE);
        double M0 = E0 - esinE;
        double M1 = M0 + sqrt(mu * alpha * alpha * alpha) * tau;
        double lo = M0 < M1 ? M0 : M1, hi = M0 < M1 ? M1 : M0;
        /* a multiple of 2 pi in [lo, hi] */
        passed = floor(hi / (2.0 * pi)) * (2.0 * pi) >= lo;
    } else {
        passed = tau >= 0.0 ? (eta0 < 0.0 && eta1 >= 0.0) : (eta1 < 0.0 && eta0 >= 0.0);
    }
    if (passed) {
        double q = h2 / (mu * (1.0 + e));
        if (q < rmin)
            rmin = q;
    }
    return rmin;
}

/* The events of one step of one system, applied in this order: star impacts,
 * collisions (among the step's flagged pairs ice/jce, i < j, of bodies not
 * lost to the star), ejections (r_eject > 0).  (Q0,V0), (Q1,V1): the step's
 * drift arcs; Q, V: the state at the end of the step (changed in place), m and
 * *m0 likewise.  lost[i] = 0 kept, 1 star impact, 2 merged into another body,
 * 3 ejected; lost bodies get m = 0.  Counts in ev[4]: star impacts, colliding
 * pairs, bodies merged away, ejections. */
void orc_events(int n, double G, double *m0, double *m, double *Q, double *V, const double *Q0,
                const double *V0, const double *Q1, const double *V1, double tau, int nce,
                const int32_t *ice, const int32_t *jce, double rho, double r_star, double r_eject,
                int32_t *lost, int32_t *ev)
{
    for (int k = 0; k < 4; ++k)
        ev[k] = 0;
    for (int i = 0; i < n; ++i)
        lost[i] = 0;
    /* 1. star impacts: all of one step's impactors join the star together */
    nsum ms = {0, 0}, sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
    for (int i = 0; i < n; ++i) {
        if (orc_star_min(G * *m0, tau, Q0 + 3 * i, V0 + 3 * i, Q1 + 3 * i, V1 + 3 * i) <= r_star) {
            lost[i] = 1;
            ++ev[0];
            ns_add(&ms, m[i]);
            ns_add(&sx, m[i] * Q[3 * i]);
            ns_add(&sy, m[i] * Q[3 * i + 1]);
            ns_add(&sz, m[i] * Q[3 * i + 2]);
        }
    }
    if (ev[0] > 0) {
        double mnew = *m0 + ns_val(&ms);
        double s[3] = {ns_val(&sx) / mnew, ns_val(&sy) / mnew, ns_val(&sz) / mnew};
        for (int i = 0; i < n; ++i) {
            if (lost[i]) {
                m[i] = 0.0;
                continue;
            }
            for (int c = 0; c < 3; ++c)
                Q[3 * i + c] -= s[c];
        }
        *m0 = mnew;
    }
    /* 2. collisions: connected components of the colliding pairs merge into
     * their smallest member */
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    double *R = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    orc_phys_radius(n, m, rho, R);
    for (int i = 0; i < n; ++i)
        parent[i] = i;
    for (int p = 0; p < nce; ++p) {
        int i = ice[p], j = jce[p];
        if (lost[i] || lost[j])
            continue;
        double d2 = orc_pair_min_d2(tau, Q0 + 3 * i, V0 + 3 * i, Q1 + 3 * i, V1 + 3 * i,
                                    Q0 + 3 * j, V0 + 3 * j, Q1 + 3 * j, V1 + 3 * j);
        double rr = R[i] + R[j];
        if (d2 <= rr * rr) {
            ++ev[1];
            int a = find_root(parent, i), b = find_root(parent, j);
            if (a != b) {
                if (a < b)
                    parent[b] = a;
                else
                    parent[a] = b;
            }
        }
    }
    for (int root = 0; root < n; ++root) {
        if (lost[root] || find_root(parent, root) != root)
            continue;
        int members = 0;
        nsum mm = {0, 0}, px = {0, 0}, py = {0, 0}, pz = {0, 0}, vx = {0, 0}, vy = {0, 0},
             vz = {0, 0};
        for (int i = root; i < n; ++i) {
            if (lost[i] || find_root(parent, i) != root)
                continue;
            ++members;
            ns_add(&mm, m[i]);
            ns_add(&px, m[i] * Q[3 * i]);
            ns_add(&py, m[i] * Q[3 * i + 1]);
            ns_add(&pz, m[i] * Q[3 * i + 2]);
            ns_add(&vx, m[i] * V[3 * i]);
            ns_add(&vy, m[i] * V[3 * i + 1]);
            ns_add(&vz, m[i] * V[3 * i + 2]);
        }
        if (members < 2)
            continue;
        double M = ns_val(&mm);
        if (M > 0.0) {
            Q[3 * root] = ns_val(&px) / M;
            Q[3 * root + 1] = ns_val(&py) / M;
            Q[3 * root + 2] = ns_val(&pz) / M;
            V[3 * root] = ns_val(&vx) / M;
            V[3 * root + 1] = ns_val(&vy) / M;
            V[3 * root + 2] = ns_val(&vz) / M;
        }
        m[root] = M;
        for (int i = root + 1; i < n; ++i)
            if (!lost[i] && find_root(parent, i) == root) {
                lost[i] = 2;
                m[i] = 0.0;
                ++ev[2];
            }
    }
    free(parent);
    free(R);
    /* 3. ejections: the ejected bodies' momentum leaves with them */
    if (r_eject > 0.0) {
        nsum mt = {0, 0}, me = {0, 0}, ex = {0, 0}, ey = {0, 0}, ez = {0, 0};
        ns_add(&mt, *m0);
        for (int i = 0; i < n; ++i) {
            if (lost[i])
                continue;
            ns_add(&mt, m[i]);
            double r = sqrt(Q[3 * i] * Q[3 * i] + Q[3 * i + 1] * Q[3 * i + 1] +
                            Q[3 * i + 2] * Q[3 * i + 2]);
            if (r > r_eject) {
                lost[i] = 3;
                ++ev[3];
                ns_add(&me, m[i]);
                ns_add(&ex, m[i] * V[3 * i]);
                ns_add(&ey, m[i] * V[3 * i + 1]);
                ns_add(&ez, m[i] * V[3 * i + 2]);
            }
        }
        if (ev[3] > 0) {
            double rest = ns_val(&mt) - ns_val(&me);
            double dv[3] = {ns_val(&ex) / rest, ns_val(&ey) / rest, ns_val(&ez) / rest};
            for (int i = 0; i < n; ++i) {
                if (lost[i] == 3)
                    m[i] = 0.0;
                else if (!lost[i])
                    for (int c = 0; c < 3; ++c)
                        V[3 * i + c] += dv[c];
            }
        }
    }
}

/* Removal of lost bodies (mxx_elim): the kept bodies in their order; index[k]
 * is the old index of kept body k.  Returns the number kept. */
int orc_compact(int n, const int32_t *lost, const double *m, const double *Q, const double *V,
                double *m_out, double *Q_out, double *V_out, int32_t *index)
{
    int k = 0;
    for (int i = 0; i < n; ++i) {
        if (lost[i])
            continue;
        m_out[k] = m[i];
        memcpy(Q_out + 3 * k, Q + 3 * i, 3 * sizeof(double));
        memcpy(V_out + 3 * k, V + 3 * i, 3 * sizeof(double));
        index[k] = i;
        ++k;
    }
    return k;
}
