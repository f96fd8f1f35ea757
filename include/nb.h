/*
 * nb.h -- C ABI of the MI355X hot path of a Mercury-style hybrid symplectic
 * N-body step (Mercury-Opal, arXiv 2601.19654).
 *
 * What one step computes, in democratic-heliocentric (DH) variables: heliocentric
 * positions Q and barycentric velocities V of the bodies; the star of each
 * system sits outside the body arrays with mass m0 (the paper's index 1, Sec. 3.1):
 *
 *   K(h)   V += h a                              interaction kick  (Sec. 3.1, Hamiltonian block, loop 1)
 *   S(h)   Q += h P/m0,  P = sum m V              stellar motion     (Hamiltonian block, loops 2-3)
 *   D(dt)  (Q0,V0) <- (Q,V); Kepler flow about    Kepler drift       (Sec. 2.1, Sec. 3.1 drift block)
 *          the star, mu = G m0, for time dt
 *   C      flag pairs i<j whose minimum           encounter check    (Sec. 3.1, encounter block)
 *          separation over the step <= rc_ij
 *   S(h)
 *   rc_i = n_hill |Q_i| (m_i/(3 m0))^(1/3)        critical radius    (Sec. 2.1.1, Hill radius footnotes)
 *   a_i  = sum_j G m_j w(r_ij)(Q_j - Q_i)          interaction force  (Sec. 3.1, force block, loop 2)
 *          w = K/r^3 - (dK/dr)/r^2, rc_ij = max(rc_i, rc_j), K the changeover function
 *   K(h)                                           h = dt/2
 *
 * With nb_params.resolve = 1 (the full hybrid method), after C every group of
 * bodies joined by flagged pairs restarts from (Q0,V0) and is advanced over dt
 * on the host by Bulirsch-Stoer under the Kepler part plus the (1 - K)-weighted
 * pair part (Sec. 2.1.1, critical-radius footnote; Sec. 3 and 3.2 keep this on
 * the host), before the second S(h).
 *
 * Conventions
 *  - Every call returns NB_OK (0) or a negative NB_E_* code; nothing throws or
 *    aborts across the ABI.  nb_strerror() names a code; nb_last_error() gives the
 *    context's last message.
 *  - Bodies of all systems are stored back to back: system s owns global indices
 *    off[s] .. off[s+1]-1.  Indices are 0-based.
 *  - Vector arrays at the boundary are plane-major (SoA): x[c*ntot + i] is
 *    component c (0,1,2 = x,y,z) of body i.
 *  - Calls enqueue work on the context's HIP stream and are asynchronous, except
 *    those that return host-visible values (counts, diagnostics, host copies),
 *    which synchronize that stream before returning.
 *  - One context is used by one host thread at a time.
 *  - The library never allocates device memory: the caller allocates the
 *    workspace (size from nb_workspace_size) and keeps it alive until nb_destroy.
 *    Host pointers passed in are read or written before the call returns.
 *  - Units are the caller's; G is a parameter.  The tests use AU, Msun, yr.
 */
#ifndef NB_H
#define NB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NB_VERSION_MAJOR 0
#define NB_VERSION_MINOR 3

/* status codes */
#define NB_OK            0
#define NB_E_INVALID    -1   /* bad argument, size or layout */
#define NB_E_NOT_READY  -2   /* no state uploaded yet, or no drift before nb_encounters */
#define NB_E_HIP        -3   /* HIP runtime error; nb_last_error() has its text */
#define NB_E_NONFINITE  -4   /* NaN/Inf (or a negative mass, a non-positive m0) in an upload */
#define NB_E_CAPACITY   -5   /* encounter list overflow: the true count is still reported */
#define NB_E_KEPLER     -6   /* >= 1 body failed to converge in the Kepler solve; those
                                bodies keep their pre-drift state, the rest are drifted */
#define NB_E_WORKSPACE  -7   /* workspace smaller than nb_workspace_size() or not 256-B aligned */

/* pair arithmetic of the force kernel */
#define NB_FP64   0   /* FP64 pair terms */
#define NB_FP32C  1   /* FP32 pair terms from hi/lo split positions with compensated
                         accumulation; pairs near the changeover zone in FP64 */

/* frames */
#define NB_HELIO  0   /* heliocentric positions and velocities */
#define NB_DH     1   /* heliocentric positions, barycentric velocities */

/* pointer kinds */
#define NB_HOST   0
#define NB_DEVICE 1

typedef struct nb_ctx nb_ctx;

typedef struct nb_params {
    double  G;            /* gravitational constant */
    double  n_hill;       /* critical radius in Hill radii (3) */
    double  chg_inner;    /* inner edge of the changeover zone as a fraction of rc (0.1) */
    int32_t mode;         /* NB_FP64 or NB_FP32C */
    int32_t drag;         /* 0: no gas drag; 1: quadratic gas drag in every kick */
    double  drag_sigma0;  /* gas surface density at R = 1 (mass / length^2) */
    double  drag_h;       /* disk aspect ratio H/R */
    double  drag_cd;      /* drag coefficient */
    double  drag_rho_p;   /* bulk density of the bodies (mass / length^3) */
    int32_t force_jchunk; /* sources per force work item (0: tuned default) */
    int32_t force_r;      /* targets per lane in the force kernel: 1, 2 or 4 (0: default) */
    int32_t enc_jchunk;   /* sources per encounter work item (0: default) */
    int32_t enc_algo;     /* encounter check: 0 automatic, 1 every pair through a per-pair
                             reach filter, 2 spatially sorted tiles with tile-pair culling,
                             3 every body against the big bodies of its system (at most 256
                             big bodies per system; automatic when some bodies are small),
                             4 in nb_step the check of 2 done inside the force pass, which
                             then runs over the sorted order (Sec. 3.1 force and encounter
                             blocks in one tile loop; FP32C, every body big, resolve 0 and
                             the symmetric force, else 2; nb_encounters and nb_force run as
                             with 2) */
    int32_t step_algo;    /* nb_step: 0 automatic (the tuning table's choice, else 1), 1 one
                             launch per phase over all systems (HIP graph), 2 one persistent
                             launch in which a workgroup owns a system for many steps (FP64
                             pair arithmetic; systems of at most NB_PERSISTENT_MAX_N bodies; not
                             with resolve; keeps no drift arcs for nb_encounters or nb_events) */
    int32_t resolve;      /* 0: flag close encounters only (hot-path mode); 1: the full
                             hybrid method, every flagged group resolved on the host by
                             Bulirsch-Stoer inside each nb_step (Sec. 2.1.1, Sec. 3.2) */
    int32_t resolve_threads; /* host threads of the resolver (0: up to 16, by the host) */
    int32_t force_algo;   /* force: 0 automatic, 1 every ordered pair (i, j) evaluated,
                             2 each unordered pair once and applied to both bodies (tile pairs;
                             every body big); automatic takes 2 where it applies;
                             4 (FP32C) as 2 over the bodies of every system in order of
                             distance from the star, the order set by nb_upload: tiles of 64
                             consecutive bodies are thin shells, and a pair of them whose
                             radial gap exceeds 2^21 times their low parts' norms and both
                             critical radii takes the FP32 high parts only (each pair's
                             difference within 2^-21 of its length, changeover weight K = 1,
                             Sec. 3.1 force block).
                             Results then depend on the order, so a run resumed by
                             nb_upload rounds as a fresh upload of that state.  In FP64
                             mode, and with enc_algo 4, it is 2. */
    double  bs_tol;       /* Bulirsch-Stoer relative tolerance (0: 1e-12) */
    const char *autotune_path; /* tuning table written by the autotuner (text; NULL: none).
                             When every tile and algorithm field (force_jchunk, force_r,
                             enc_jchunk, enc_algo, step_algo, force_algo, force_g) is 0,
                             nb_workspace_size and nb_create take them from the table's
                             entry for this GPU, mode and size class (largest system and
                             system count, and the largest big-body count when some
                             bodies are small, each rounded up to a power of two); a
                             class the table lacks keeps the defaults.  An unreadable
                             file is NB_E_INVALID.  Read during the call only. */
    int32_t force_g;      /* symmetric force: tiles of 64 force_r bodies per super-tile, 1, 2
                             or 4 (0: the tuning table's, else automatic: 4 when that gives at
                             least 8192 work items, else 2 when that does, else 1).  A body
                             receives one partial sum per super-tile of its system, so wider
                             super-tiles write fewer partials, at the cost of a barrier per
                             round in the force kernel. */
} nb_params;

/* largest system the persistent step launch accepts */
#define NB_PERSISTENT_MAX_N 8192

typedef struct nb_stats {
    int64_t total_nce;      /* flagged pairs summed over the steps */
    int32_t max_nce;        /* largest per-step count */
    int32_t overflow_steps; /* steps whose count exceeded the list capacity */
    int64_t kepler_fail;    /* failed Kepler solves summed over the steps */
    int64_t near_pairs;     /* pair evaluations inside the changeover zone (in FP64 for FP32C);
                               with symmetric tile pairs one evaluation serves both bodies */
    int64_t resolved_groups; /* resolve: groups integrated by Bulirsch-Stoer, summed */
    int64_t resolved_bodies; /* resolve: their members, summed */
    int32_t max_group;      /* resolve: largest group */
    int32_t bs_fail;        /* resolve: groups whose integration failed (members keep the
                               Kepler-drifted state) */
} nb_stats;

/* Library version. */
int nb_version(int *major, int *minor);

/* Static text for a status code. */
const char *nb_strerror(int code);

/* Fill p with the defaults used by the tests: G = (0.01720209895*365.25)^2
 * (AU, Msun, yr), n_hill = 3, chg_inner = 0.1, NB_FP64, no drag, drag constants for
 * Sigma(1 AU) = 1000 g/cm^2, h = 0.05, C_D = 1, rho_p = 2 g/cm^3 in those units. */
void nb_default_params(nb_params *p);

/* Bytes of device workspace a context needs for nsys systems with host offsets
 * off[0..nsys] (off[0] = 0, non-decreasing) and an encounter list of enc_cap pairs.
 * nbig (host, nsys entries, may be NULL = every body big): the first nbig[s]
 * bodies of system s are big, the rest small (Sec. 2.1: only big bodies are
 * gravity sources; small bodies are massless, feel the big ones, and two small
 * bodies never interact, so the force costs (N_s) x nbig[s] pairs and the
 * encounter check tests only pairs with a big member).  0 <= nbig[s] <= N_s.
 * Gas drag needs a mass for the body size, so drag with small bodies is
 * NB_E_INVALID. */
int nb_workspace_size(const nb_params *p, int nsys, const int32_t *off, const int32_t *nbig,
                      int enc_cap, size_t *bytes);

/* Create a context on the current device.  off and nbig as for nb_workspace_size.
 * workspace: device memory of at least nb_workspace_size() bytes, 256-byte
 * aligned, owned by the caller.  stream: a hipStream_t (NULL = the null stream;
 * nb_step then runs without a HIP graph).  nb_upload rejects a small body with a
 * nonzero mass (NB_E_INVALID). */
int nb_create(const nb_params *p, int nsys, const int32_t *off, const int32_t *nbig, int enc_cap,
              void *workspace, size_t bytes, void *stream, nb_ctx **out);

/* Last error message of the context (empty if none). */
const char *nb_last_error(const nb_ctx *ctx);

/* Upload a state: m0[nsys], m[ntot], x[3*ntot], v[3*ntot] (plane-major), in frame
 * NB_HELIO (converted to DH, Sec. 2.1.1 footnote) or NB_DH.  where: NB_HOST or
 * NB_DEVICE for all four pointers.  Validates (finite, m >= 0, m0 > 0), then
 * computes the critical radii and the force at the new state (first-same-as-last). */
int nb_upload(nb_ctx *ctx, const double *m0, const double *m, const double *x,
              const double *v, int frame, int where);

/* Copy the state out: x, v plane-major [3*ntot] in frame NB_HELIO or NB_DH (the
 * DH -> heliocentric change v = V + P/m0 of Sec. 2.1.1's coordinate footnote;
 * the paper copies x and v back to the host every step, Sec. 3.2). */
int nb_download(nb_ctx *ctx, double *x, double *v, int frame, int where);

/* Recompute critical radii (Sec. 2.1.1, Hill-radius footnotes) and the interaction
 * acceleration a at the current Q (Sec. 3.1, force block loop 2: the
 * changeover-weighted pair sum of the header's formula). */
int nb_force(nb_ctx *ctx);

/* Interaction kick with the current a: V += h a (Sec. 3.1, Hamiltonian block loop
 * 1), plus the gas drag of force block loop 5 if enabled. */
int nb_kick(nb_ctx *ctx, double h);

/* Stellar-motion drift: Q += h P / m0 per system, P = sum m V (Sec. 3.1,
 * Hamiltonian block loops 2-3). */
int nb_sun_drift(nb_ctx *ctx, double h);

/* Snapshot (Q0,V0) <- (Q,V), then Kepler-drift every body for dt (dt may be
 * negative: the integration direction).  *nfail (may be NULL) receives the number of
 * bodies whose solve failed; returns NB_E_KEPLER if any did. */
int nb_drift(nb_ctx *ctx, double dt, int *nfail);

/* Encounter check on the last drift: pairs i<j of one system whose minimum
 * separation between (Q0,V0) and (Q,V) is <= max(rc_i, rc_j).  Needs nb_drift
 * since the last call that changed the state (upload, force, kick, sun drift,
 * step), else NB_E_NOT_READY; after nb_step use nb_get_encounters.  Writes up to cap
 * pairs to ice/jce (global indices, sorted by (i,j)) and per-body flags ce[ntot]
 * (2 = in an encounter, else 0); *nce = the true count.  Any of ice/jce/ce may be
 * NULL.  Returns NB_E_CAPACITY if the count exceeds cap or the context's list. */
int nb_encounters(nb_ctx *ctx, int cap, int *nce, int32_t *ice, int32_t *jce, int32_t *ce,
                  int where);

/* Read the list of the last encounter check (by nb_encounters or the last step
 * of nb_step) without recomputing it; the same layout as nb_encounters (the
 * list is put in (i,j) order as it is read, the check itself appends in an
 * arbitrary order). */
int nb_get_encounters(nb_ctx *ctx, int cap, int *nce, int32_t *ice, int32_t *jce, int32_t *ce,
                      int where);

/* nsteps hybrid steps K S D C S F K of every system (graph-captured when the
 * stream is not NULL and resolve is 0).  With resolve = 1 each step
 * synchronizes the stream after C, copies the flagged groups' members to the
 * host, integrates them there and writes them back (only members cross PCIe).
 * st (may be NULL) receives the run's statistics.  Returns NB_E_KEPLER /
 * NB_E_CAPACITY if any step had such an event (with resolve, an overflowing
 * step resolves the pairs the list holds); the state is still advanced. */
int nb_step(nb_ctx *ctx, double dt, int nsteps, nb_stats *st);

/* Capture, ahead of time, the HIP graphs that nb_step(ctx, dt, nsteps) replays
 * (runs of 8 steps and one run of the remainder, kept per run length for one
 * dt; a new dt replaces them), so that the nb_step call itself only launches
 * them.  Runs no step and leaves the state alone.  Does nothing (NB_OK) without
 * a stream, with resolve = 1 or with the persistent step launch.  An
 * implementation aid for timing and for callers that must not capture inside
 * their loop; not a step of the method. */
int nb_prepare(nb_ctx *ctx, double dt, int nsteps);

typedef struct nb_resolve_info {
    int32_t groups;     /* groups integrated */
    int32_t bodies;     /* their members */
    int32_t max_group;  /* largest group */
    int32_t failed;     /* groups whose integration failed */
    int32_t max_steps;  /* most Bulirsch-Stoer step attempts of one group */
} nb_resolve_info;

/* Host close-encounter resolver on host arrays of one system (no GPU work;
 * the same code nb_step runs with resolve = 1).  Sec. 2.1.1 (critical-radius
 * footnote) and Sec. 3.2: bodies joined by the nce flagged pairs (ice[k],
 * jce[k]), 0-based local indices, are grouped (connected components); each group
 * restarts from (Q0,V0) and is advanced by tau under
 *   dQ/dt = V,  dV_i/dt = -G m0 Q_i/|Q_i|^3
 *                         + sum_j G m_j [(1-K)/r^3 + (dK/dr)/r^2] (Q_j - Q_i)
 * (j over the group, rc_ij = max(rc_i, rc_j), changeover inner edge chg_inner
 * rc_ij) by Bulirsch-Stoer with relative tolerance tol (0: 1e-12); its result
 * is written to Q, V.  Other bodies keep Q, V.  Arrays are row-major n x 3 (Q0,
 * V0, Q, V) and n (m, rc).  group[n] (may be NULL) receives each body's group
 * label (its smallest member) or -1.  nthreads: host threads (0: up to 16).
 * A failed group keeps Q, V and is counted in info->failed (info may be NULL).
 * Returns NB_E_INVALID for bad sizes or indices. */
int nb_resolve_host(int n, double G, double m0, double chg_inner, double tol, double tau,
                    const double *m, const double *rc, const double *Q0, const double *V0,
                    int nce, const int32_t *ice, const int32_t *jce, double *Q, double *V,
                    int32_t *group, int nthreads, nb_resolve_info *info);

/* Collisions, star impacts and ejections after a step (Sec. 2.1.1: physical
 * radii, removal of lost bodies; Sec. 2.1.2: planet-planet and planet-star
 * collisions, ejections of distant bodies, checked by the paper every 200 yr
 * beyond 400 AU).  The paper gives no arithmetic for them; the readings:
 *  - physical radius R = (3 m/(4 pi rho))^(1/3) from one bulk density rho;
 *  - star impact (r_star > 0): the Kepler arc of the last drift comes within
 *    r_star of the star (the nearer end, or the pericentre distance when the
 *    arc passes a pericentre); the impactors' mass joins m0 and the star moves
 *    to the centre of mass of star and impactors, so every other body's
 *    heliocentric position shifts by minus that displacement;
 *  - collision: a listed pair of the last encounter check, neither member lost
 *    to the star, whose minimum separation over the step (the encounter
 *    predicate's Hermite minimum) is at most R_i + R_j; bodies joined by
 *    colliding pairs merge into their smallest index: summed mass,
 *    mass-weighted position and velocity;
 *  - ejection (r_eject > 0): a body farther than r_eject from the star leaves
 *    with its momentum; the barycentric velocities of the rest change by
 *    sum m_e V_e / (m0 + sum m - sum m_e).
 * Applied in that order to the state after the last step (nb_step, or nb_drift
 * followed by nb_encounters); NB_E_NOT_READY otherwise (also after the
 * persistent step launch, which keeps no drift arcs).  Lost bodies keep their
 * slot with m = 0 until nb_compact; lost[ntot] (may be NULL; host or device per
 * `where`) receives 0 kept, 1 star impact, 2 merged away, 3 ejected.  When a
 * body was lost the critical radii and the force are computed again.
 * NB_E_CAPACITY if the list had overflowed (only the kept pairs are tested).
 * Collisions are tested by one workgroup, quadratic in the members of colliding
 * pairs: meant for a few per call. */
typedef struct nb_event_params {
    double rho;      /* bulk density of the bodies (mass / length^3), > 0 */
    double r_star;   /* star radius (0: no star impacts) */
    double r_eject;  /* ejection distance from the star (0: no ejections) */
} nb_event_params;

typedef struct nb_event_counts {
    int32_t star;     /* bodies that fell into their star */
    int32_t collide;  /* colliding pairs */
    int32_t merged;   /* bodies merged into another one */
    int32_t ejected;  /* bodies ejected */
} nb_event_counts;

int nb_events(nb_ctx *ctx, const nb_event_params *ep, nb_event_counts *counts, int32_t *lost,
              int where);

/* Remove the bodies nb_events marked lost (the paper's removal of lost bodies,
 * Sec. 2.1.1), keeping the order of the rest in every system, and continue with
 * the smaller arrays in the same workspace: the work tables are rebuilt for the
 * new offsets, the critical radii and the force computed again (a new upload of
 * the kept state).  The kept bodies among a system's first nbig stay its big
 * bodies.  Outputs (host or device per `where`, each may be NULL): off_out[nsys+1]
 * the new offsets, nbig_out[nsys] the new big-body counts, index[new ntot] the
 * old index of every kept body.  NB_E_NOT_READY without nb_events on the current
 * state; NB_E_WORKSPACE if the new layout needs more workspace than the context
 * has (possible only when an automatic algorithm choice changes with the sizes):
 * the context is then left as it was. */
int nb_compact(nb_ctx *ctx, int32_t *off_out, int32_t *nbig_out, int32_t *index, int where);

/* Per system s (host arrays): E[s] total energy, EK[s] the changeover-weighted
 * energy the hot path conserves, L[3s..3s+2] = sum m Q x V, P[3s..3s+2] = sum m V.
 * Any pointer may be NULL.  Returns NB_E_NONFINITE if a value is not finite. */
int nb_diagnostics(nb_ctx *ctx, double *E, double *EK, double *L, double *P);

/* Copy the last interaction acceleration a (G included, drag excluded), plane-major
 * (the force block's output, Sec. 3.1 loop 2). */
int nb_get_accel(nb_ctx *ctx, double *a, int where);

/* Copy the current critical radii rc[ntot]. */
int nb_get_rcrit(nb_ctx *ctx, double *rc, int where);

/* Kernels that nb_time_kernel can time. */
#define NB_K_FORCE      0   /* the pair force kernel (FP64 or FP32C per the mode) */
#define NB_K_ENCOUNTER  1   /* the encounter check (the list is sorted when read) */
#define NB_K_DRIFT      2   /* the Kepler drift */
#define NB_K_STEP       3   /* whole hybrid steps, enqueued the way nb_step runs them */
#define NB_K_FORCE_EVAL 4   /* one whole force evaluation: critical radii and source
                               records, the force kernel and the sum of its splits */
#define NB_K_FORCE_FUSED 5  /* enc_algo 4: the force pass with the encounter test in it,
                               on the sorted order of the last per-phase step (its list
                               is made again once after the timed launches) */

/* Measurement helper: enqueue kernel `which` alone `reps` times on the context's
 * stream between two HIP events (after one untimed launch) and return the mean
 * duration per launch in milliseconds.  The state is used as it is; NB_K_DRIFT
 * and NB_K_STEP advance it by dt per launch; NB_K_ENCOUNTER overwrites the last
 * encounter list (with the dt of the last drift or step). */
int nb_time_kernel(nb_ctx *ctx, int which, int reps, double dt, double *ms_per_launch);

/* The algorithms the context resolved its automatic choices to (any pointer may
 * be NULL): force 1 (ordered pairs), 2 (symmetric tile pairs), 3 (few-source
 * kernels) or 4 (symmetric tile pairs over the radial order); encounter check 1 (direct), 2 (sorted tiles), 3 (big bodies only as
 * partners) or 4 (sorted tiles inside the force pass); step launch 1
 * (per phase) or 2 (persistent). */
int nb_get_choices(const nb_ctx *ctx, int32_t *force_algo, int32_t *enc_algo, int32_t *step_algo);

/* The parameters the context runs with (tile and algorithm fields after the
 * tuning table and the automatic choices of nb_create; autotune_path NULL);
 * *tuned (may be NULL) = 1 if they came from the tuning table. */
int nb_get_params(const nb_ctx *ctx, nb_params *out, int32_t *tuned);

/* Force evaluation without a context, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  The same computation as nb_upload (frame NB_DH) followed
 * by nb_force and nb_get_accel on a context with the same parameters, for one
 * system: critical radii rc_i = n_hill |x_i| (m_i/(3 m0))^(1/3), then
 * a_i = G sum_j m_j w(r_ij; rc_ij) (x_j - x_i) by the symmetric force kernels
 * (every body big), equal bit for bit to that context's result.
 *   p: G, n_hill, chg_inner, mode, force_r (0, 1, 2, 4), force_g (0, 1, 2, 4) and
 *      force_algo (0 or 2) are used; the other fields are ignored.
 *   n: bodies, 0 <= n <= NB_NOALLOC_MAX_N.  m0: the star's mass (> 0).
 *   m[n], x[3n] (plane-major DH positions), a[3n] (output, plane-major, G
 *      included): device pointers owned by the caller; m and x are only read.
 *   stream: hipStream_t (NULL: the null stream); the call only enqueues work.
 * Nothing is allocated: the work tables, critical radii, source records and
 * partial sums live in a static device array of NB_NOALLOC_SCRATCH_MB MiB that
 * every GPU the library runs on holds until the process ends.  Every call on a
 * GPU uses that GPU's one array, so calls that overlap on one GPU (other streams,
 * other host threads) race; successive calls on one stream are ordered.  Inputs
 * are not checked for finite values.  Returns NB_E_WORKSPACE when n exceeds
 * NB_NOALLOC_MAX_N or the layout for the asked force_r / force_g does not fit the
 * array (the automatic widths fit up to NB_NOALLOC_MAX_N), NB_E_INVALID for other
 * bad arguments, NB_E_HIP if a launch fails. */
#define NB_NOALLOC_MAX_N 16384
#define NB_NOALLOC_SCRATCH_MB 32
int nb_force_noalloc(const nb_params *p, int n, double m0, const double *m, const double *x,
                     double *a, void *stream);

/* Release the context (not the workspace). */
int nb_destroy(nb_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* NB_H */
