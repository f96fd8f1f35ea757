/* Exercise the CPU oracle's entry points under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by tests/test_sanitize.py).
 * Inputs: a few bodies on near-circular orbits from a fixed linear
 * congruential sequence, packed close enough that pairs are flagged and
 * grouped; list capacities both large and too small (the overflow path). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_rcrit(int n, double m0, const double *m, const double *Q, double n_hill, double *rc);
void orc_force_nb(int n, int nbig, double G, double inner, const double *m, const double *Q,
                  const double *rc, double *a);
void orc_force_subset(int n, int nbig, double G, double inner, const double *m, const double *Q,
                      const double *rc, int k, const int32_t *idx, double *a);
int orc_drift(int n, double mu, double tau, double *Q, double *V, int32_t *flag);
void orc_encounters_nb(int n, int nbig, double tau, const double *Q0, const double *V0,
                       const double *Q1, const double *V1, const double *rc, int cap,
                       int32_t *ice, int32_t *jce, int32_t *ce, int *nce, double tie,
                       int tie_cap, int32_t *tie_i, int32_t *tie_j, int *ntie);
void orc_pair_scan(int n, int nbig, double tau, const double *Q0, const double *V0,
                   const double *Q1, const double *V1, const double *rc, int i, double tie,
                   int32_t *flag, int32_t *tieflag);
void orc_energy(int n, double G, double m0, double inner, const double *m, const double *Q,
                const double *V, const double *rc, double *E, double *EK, double *L, double *P);
int orc_step(int n, int nbig, double G, double m0, double n_hill, double inner, const double *m,
             double *Q, double *V, double *a, double *rc, double tau, int drag, double sigma0,
             double hr, double cd, double rho_p, double *Q0, double *V0, int32_t *kflag,
             double *scratch, int cap, int32_t *ice, int32_t *jce, int32_t *ce, int *nce);
int orc_resolve_work_doubles(int n);
int orc_step_full(int n, int nbig, double G, double m0, double n_hill, double inner, const double *m,
                  double *Q, double *V, double *a, double *rc, double tau, int drag, double sigma0,
                  double hr, double cd, double rho_p, double tol, double *Q0, double *V0,
                  int32_t *kflag, double *scratch, int cap, int32_t *ice, int32_t *jce, int32_t *ce,
                  int *nce, int32_t *comp, double *work, int *bsfail, int *ngroups);

void orc_events(int n, double G, double *m0, double *m, double *Q, double *V, const double *Q0,
                const double *V0, const double *Q1, const double *V1, double tau, int nce,
                const int32_t *ice, const int32_t *jce, double rho, double r_star, double r_eject,
                int32_t *lost, int32_t *ev);
int orc_compact(int n, const int32_t *lost, const double *m, const double *Q, const double *V,
                double *m_out, double *Q_out, double *V_out, int32_t *index);

static uint64_t lcg = 12345;
static double unif(void)
{
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) * 0x1p-53;
}

static void setup(int n, double G, double *m, double *Q, double *V, double mass)
{
    for (int i = 0; i < n; ++i) {
        double r = 1.0 + 0.01 * unif(), th = 0.3 * unif();
        double v = sqrt(G / r);
        m[i] = mass * (0.5 + unif());
        Q[3 * i] = r * cos(th);
        Q[3 * i + 1] = r * sin(th);
        Q[3 * i + 2] = 1e-3 * (unif() - 0.5);
        V[3 * i] = -v * sin(th);
        V[3 * i + 1] = v * cos(th);
        V[3 * i + 2] = 1e-3 * (unif() - 0.5);
    }
}

static int run(int n, int nbig, int cap, int drag, int full)
{
    const double G = 39.476926421373, m0 = 1.0, tau = 0.02;
    double *m = malloc(sizeof(double) * n), *Q = malloc(sizeof(double) * 3 * n);
    double *V = malloc(sizeof(double) * 3 * n), *a = malloc(sizeof(double) * 3 * n);
    double *rc = malloc(sizeof(double) * n), *Q0 = malloc(sizeof(double) * 3 * n);
    double *V0 = malloc(sizeof(double) * 3 * n), *sc = malloc(sizeof(double) * 3 * n);
    int32_t *kf = malloc(sizeof(int32_t) * n), *ce = malloc(sizeof(int32_t) * n);
    int32_t *ice = malloc(sizeof(int32_t) * (cap > 0 ? cap : 1));
    int32_t *jce = malloc(sizeof(int32_t) * (cap > 0 ? cap : 1));
    int32_t *comp = malloc(sizeof(int32_t) * n), *fl = malloc(sizeof(int32_t) * n);
    int32_t *tf = malloc(sizeof(int32_t) * n), ti[4], tj[4];
    double *work = malloc(sizeof(double) * orc_resolve_work_doubles(n));
    setup(n, G, m, Q, V, 1e-6);
    for (int i = nbig; i < n; ++i)
        m[i] = 0.0;
    orc_rcrit(n, m0, m, Q, 3.0, rc);
    orc_force_nb(n, nbig, G, 0.1, m, Q, rc, a);
    int32_t idx[3] = {0, n / 2, n - 1};
    double as[9];
    orc_force_subset(n, nbig, G, 0.1, m, Q, rc, 3, idx, as);
    int total = 0;
    for (int s = 0; s < 5; ++s) {
        int nce = 0, bsf = 0, ng = 0;
        if (full)
            orc_step_full(n, nbig, G, m0, 3.0, 0.1, m, Q, V, a, rc, tau, drag, 1e-4, 0.05, 1.0,
                          3e7, 1e-12, Q0, V0, kf, sc, cap, ice, jce, ce, &nce, comp, work, &bsf,
                          &ng);
        else
            orc_step(n, nbig, G, m0, 3.0, 0.1, m, Q, V, a, rc, tau, drag, 1e-4, 0.05, 1.0, 3e7, Q0,
                     V0, kf, sc, cap, ice, jce, ce, &nce);
        total += nce;
    }
    double Q1[3 * 64], V1[3 * 64];
    int nn = n < 64 ? n : 64, nce = 0, ntie = 0;
    memcpy(Q1, Q0, sizeof(double) * 3 * nn);
    memcpy(V1, V0, sizeof(double) * 3 * nn);
    orc_drift(nn, G * m0, tau, Q1, V1, fl);
    orc_encounters_nb(nn, nbig < nn ? nbig : nn, tau, Q0, V0, Q1, V1, rc, cap, ice, jce, ce, &nce,
                      1e-6, 4, ti, tj, &ntie);
    orc_pair_scan(nn, nbig < nn ? nbig : nn, tau, Q0, V0, Q1, V1, rc, nn - 1, 1e-6, fl, tf);
    double E, EK, L[3], P[3];
    orc_energy(n, G, m0, 0.1, m, Q, V, rc, &E, &EK, L, P);
    /* collisions among the listed pairs (a low density: large bodies), star
     * impacts and ejections, then the compaction */
    {
        int32_t ev[4], *lost = malloc(sizeof(int32_t) * nn);
        double mm0 = m0, *mo = malloc(sizeof(double) * nn), *Qo = malloc(sizeof(double) * 3 * nn);
        double *Vo = malloc(sizeof(double) * 3 * nn);
        int32_t *io = malloc(sizeof(int32_t) * nn);
        int k = nce < cap ? nce : cap;
        orc_events(nn, G, &mm0, m, Q1, V1, Q0, V0, Q1, V1, tau, k, ice, jce, 0.1, 0.999, 1.005,
                   lost, ev);
        int kept = orc_compact(nn, lost, m, Q1, V1, mo, Qo, Vo, io);
        printf("events: star %d, colliding pairs %d, merged %d, ejected %d, kept %d\n", ev[0],
               ev[1], ev[2], ev[3], kept);
        free(lost); free(mo); free(Qo); free(Vo); free(io);
    }
    printf("n=%d nbig=%d cap=%d drag=%d full=%d: %d flagged, E=%.6e\n", n, nbig, cap, drag, full,
           total, E);
    free(m); free(Q); free(V); free(a); free(rc); free(Q0); free(V0); free(sc); free(kf);
    free(ce); free(ice); free(jce); free(comp); free(fl); free(tf); free(work);
    return total;
}

int main(void)
{
    int flagged = 0;
    flagged += run(40, 40, 1000, 0, 0);
    flagged += run(40, 40, 2, 0, 0);          /* list overflow */
    flagged += run(33, 33, 1000, 1, 0);       /* gas drag */
    flagged += run(50, 7, 1000, 0, 0);        /* big and small bodies */
    flagged += run(40, 40, 1000, 0, 1);       /* full method: groups by Bulirsch-Stoer */
    flagged += run(1, 1, 4, 0, 1);
    return flagged > 0 ? 0 : 2;
}
