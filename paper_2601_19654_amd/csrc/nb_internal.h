// Internal layout shared by the device kernels (nb_kernels.hip) and the host
// runtime (nb_runtime.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nb {

constexpr int kBlock = 256;      // threads of every O(N) kernel and of the pair kernels
constexpr int kScanChunkCells = 1024;   // cells per block of the counting sort's scan
// Sets of drift outputs (what the encounter check of a step reads): one per
// step of a captured run, so that the checks of a run, on a second queue, hold
// up no drift of the run (a run ends with one join).
constexpr int kSnapSets = 8;

// Work items the automatic super-tile width g (2 or 4) of the symmetric force
// needs (one workgroup of g waves per item).
constexpr long long kSymMinItems(int g) { return g >= 2 ? 8192 : 0; }

// A block of an O(N) kernel: bodies [start, end) of one system (end - start <= kBlock).
struct RBlk {
    int sys, start, end;
    int rt0;              // force over the radial order: the block's first tile of 64 positions
};

// A force work item: targets [i0, i0+ni), sources [j0, j0+nj) of one system;
// the partial sum goes to split slot `slot`.  Source tiles of kBlock bodies
// coincide with O(N) blocks; rb0 is the O(N) block index of the first one.
struct FWork {
    int i0, ni, j0, nj;
    int slot, sys, rb0, pad;
};

// An unordered-pair work item: targets [i0, i0+ni), sources [j0, j0+nj); only
// pairs with j > i are visited.
struct PWork {
    int i0, ni, j0, nj;
};

// A body's encounter record in spatially sorted order (sorted encounter check;
// the exact test reads the first 112 bytes, the filters read FP32 records).
struct SRec {
    double q0[3], v0[3], q1[3], v1[3];
    double rc;
    int body, big;        // global index; 1 for a big body (a gravity source)
    double M[3], c[3];    // chord midpoint and chord Q1 - Q0
    double e34, pad;      // 3/4 of the largest endpoint deviation (widened for rounding)
};

// A tile of up to 64 consecutive sorted bodies of one system; `last` is the
// index of the system's last tile.
struct Tile {
    int sys, start, count, last;
};

// Bounding data of a tile: centre and radius of the chord midpoints, of the
// chords and of the endpoint velocity deviations (dt V - chord), and the
// largest critical radius.
struct TileB {
    double cm[3], sm;
    double cc[3], sc;
    double ce[3], se;
    double rc;
    int big, all_big;     // the tile holds at least one big body / only big bodies
    double pad2[2];
};

// A system run by the persistent step launch (one workgroup each).
struct PSys {
    int sys, start, n, nbig;
};

// Device statistics block (one per context).
struct DevStats {
    long long total_nce;
    long long kepler_fail;
    long long near_pairs;
    int max_nce;
    int overflow_steps;
    int cur_nce;      // count of the current encounter check
    int cur_kfail;    // failures of the current drift
    int cur_tp;       // tile pairs surviving the cull (sorted encounter check)
    int pad;
};

// What a drift leaves for the encounter check (snapshots, copies, chord
// records); a context keeps two sets so that the check of one step can run
// beside the next step.
struct Snap {
    double *q0x, *q0y, *q0z, *v0x, *v0y, *v0z;
    double *q1x, *q1y, *q1z, *v1x, *v1y, *v1z, *rc1;
    double4 *mr, *cr;
    double *lnr_part;
};

// Device pointers of a context; every array lives in the caller's workspace.
struct Dev {
    int ntot, nsys;
    // state planes (FP64, ntot each)
    double *m, *qx, *qy, *qz, *vx, *vy, *vz;
    double *ax, *ay, *az, *rc;
    double *tile_rc2;     // per O(N) block: largest rc^2 of its bodies (set with rc)
    double *q0x, *q0y, *q0z, *v0x, *v0y, *v0z;
    // after a drift: copies of Q1, V1 and the critical radii for the encounter
    // check, so that it can run beside the next S(h), force and kick
    double *q1x, *q1y, *q1z, *v1x, *v1y, *v1z, *rc1;
    float4 *pk;           // FP32C source records: 2 per body {xhi,yhi,zhi,m},{xlo,ylo,zlo,rc2}
    double4 *mr;          // per body after a drift: chord midpoint (x,y,z) and encounter reach R
    double4 *cr;          // per body after a drift: chord Q1 - Q0 and 3/4 eps (widened)
    int *kflag, *ce, *sys_of;
    double *m0;           // nsys
    int *off;             // nsys+1
    int *nsplit;          // nsys: force splits per system
    int *rb_first, *rb_count;   // nsys: O(N) blocks of each system
    // tables
    RBlk *rblk;  int nrb;
    FWork *fwork; int nfw; int maxs;
    int ns_all;           // the split count of every system with bodies, if they all share it; else 0
    PWork *ework; int new_;
    PWork *dwork; int ndw;
    // scratch
    double *rpart;        // 3 x nrb x 4: per-block sums of m V.  First: after a kick (or
                          // from the momentum kernel); rpart_drift(): after a drift (and,
                          // with gas drag, before a kick); rpart_prev(): see below
    double *rpart_drift() const { return rpart + (size_t)nrb * 4; }
    // a copy of the last drift's sums taken by the second S(h): the momentum
    // before the next kicks, which leave it unchanged (the pair forces cancel)
    double *rpart_prev() const { return rpart + (size_t)nrb * 8; }
    double *ptot;         // nsys x 4: per-system sums of m V for the stellar drifts
    int sys_total;        // some system has more than 64 blocks: its momentum is summed once
                          // per stellar drift into ptot instead of by each of its blocks
    double *fpart;        // 3 x maxs x ntot force partials (FP64 pair arithmetic)
    float *fpart32;       // the same in FP32 (FP32C pair arithmetic; fpart is then null)
    double *dpart;        // ndw x 4 double-double pair sums (E pair, EK pair)
    double *bpart;        // nrb x 16 body partial sums for diagnostics
    double *diag;         // nsys x 8 results: E, EK, L3, P3
    unsigned long long *keys;  int keys_p2;   // encounter keys (i<<32 | j), pow2 capacity
    int enc_cap;
    int *ice, *jce;       // sorted list (enc_cap)
    DevStats *stats;
    // sorted encounter check
    int enc_sorted;
    int enc_few;          // few big bodies: each body against its system's big bodies
    double *lnr_part;     // nrb x 2: min, max of ln R (cylindrical) of chord midpoints
    int *cell_of, *slot_of;   // ntot
    int *cell_cnt, *cell_off; int ncell;
    int *sys_cell_base, *sys_cell_cnt;   // nsys
    int *ord;             // ntot: sorted position -> body
    SRec *srec;           // ntot
    int *scan_part;       // per chunk of kScanChunkCells cells: count sums (large grids)
    Tile *tiles; int ntile;
    TileB *tileb;         // ntile
    int2 *tpairs; int tp_cap;
    int2 *units; int nunit;   // culling units: tile A against tiles [b0, b0 + 64) (B >= A)
    int *tile_first;      // nsys: first tile of every system
    // force and encounter check in one pass over the sorted order (FP32C,
    // every body big)
    int enc_fused;
    // symmetric FP32C force over the radial order (bodies of each system by
    // distance from the star, set at upload): rord position -> body, tiles of
    // 64 positions from rtf[s] for system s, and their bounds written with the
    // FP32C records (least and greatest |xh|, greatest low-part norm, largest
    // widened rc^2)
    int force_rsort;
    int *rord;
    int nrtile;
    int *rtf;             // nsys
    float4 *rtb;          // nrtile
    // sorted check: per sorted position two FP32 records for the pair filter,
    // the chord midpoint with the widened bound of 3/4 eps + rc, and the chord
    // with rc rounded up (its sign bit set for a small body) ...
    float4 *em;
    // ... and one for the target's test against a tile's bounds: the mean
    // endpoint deviation with the deviation radius rounded up
    float4 *eg;
    // persistent step launch
    PSys *psys; int npsys; int pmax_n;
    int *step_nce; int step_chunk;   // flagged pairs per step of one launch
    int *flag;            // validation flags (4 ints)
    double *stage;        // 7 x ntot staging for host transfers, transforms and the compaction
    // collisions, star impacts, ejections and compaction
    int *lost;            // ntot: 0 kept, 1 star impact, 2 merged away, 3 ejected
    int *evroot;          // ntot: union-find parents of colliding bodies
    int *evflag;          // max(enc_cap, nrb): colliding-pair flags, then kept counts per block
    int *evmem;           // 2 enc_cap: members of colliding pairs
    int *evcnt;           // 4: star impacts, colliding pairs, bodies merged away, ejections
    int *cmp_pos;         // nrb + 1: first kept slot of every block, then the kept total
    int *evidx;           // ntot: old index of every kept body
    double *evpart;       // nrb x 8 per-block event sums
    double *evsys;        // nsys x 8 per-system shift (star impact) or dv (ejection), count
    // close-encounter resolver (resolve = 1): records of both ends of up to res_cap
    // listed pairs (20 doubles per pair) and result rows (7 doubles per member)
    double *res_buf; double *res_rows; int res_cap;
    int *nbig;            // per system: bodies [off[s], off[s] + nbig[s]) are big
    int force_few;        // every system has at most 256 big bodies and the targets are many:
                          // the few-source force kernels
    int force_sym;        // every body big: work items are unordered pairs of super-tiles
    int sym_g;            // tiles per super-tile (1, 2 or 4; the symmetric kernels' waves)
    Snap alt[kSnapSets - 1];   // sets 1 .. nsnap - 1 of drift outputs
    int nsnap;            // sets of drift outputs (2 .. kSnapSets)

    Snap snap() const
    {
        return Snap{q0x, q0y, q0z, v0x, v0y, v0z, q1x, q1y, q1z, v1x, v1y, v1z, rc1, mr, cr, lnr_part};
    }
    // this context with the drift outputs of set `set` (0: the first set)
    Dev with_snap(int set) const
    {
        Dev e = *this;
        if (set > 0) {
            const Snap a = alt[set - 1];
            e.q0x = a.q0x; e.q0y = a.q0y; e.q0z = a.q0z;
            e.v0x = a.v0x; e.v0y = a.v0y; e.v0z = a.v0z;
            e.q1x = a.q1x; e.q1y = a.q1y; e.q1z = a.q1z;
            e.v1x = a.v1x; e.v1y = a.v1y; e.v1z = a.v1z;
            e.rc1 = a.rc1; e.mr = a.mr; e.cr = a.cr; e.lnr_part = a.lnr_part;
        }
        return e;
    }
};

struct Params {
    double G, n_hill, inner;
    int mode, drag;
    double sigma0, h, cd, rho_p;
    int force_r, force_j, enc_j;
    int enc_algo;         // 1: all pairs with the reach prefilter, 2: sorted tiles,
                          // 3: each body against its system's big bodies (at most kBlock)
    int step_algo;        // 1: per-phase launches, 2: persistent per-system launch
    int force_algo;       // 0 automatic, 1 ordered pairs, 2 symmetric tile pairs, 4 symmetric
                          // over the radial order (FP32C; FP64: as 2)
    int force_g;          // symmetric force: tiles per super-tile (0 automatic, 1, 2, 4)
    int resolve;          // 1: resolve flagged groups on the host every step
    int resolve_threads;
    double bs_tol;
};

// ---- launchers (nb_kernels.hip) --------------------------------------------
hipError_t launch_fill_i32(int *p, int n, int value, hipStream_t s);
hipError_t launch_validate(const Dev &d, const double *m0, const double *m, const double *x,
                           const double *v, hipStream_t s);
hipError_t launch_to_dh(const Dev &d, const double *x, const double *v, int frame, hipStream_t s);
hipError_t launch_from_dh(const Dev &d, double *x, double *v, int frame, hipStream_t s);
// per-block sums of m V into part (rpart or rpart_drift())
hipError_t launch_momentum(const Dev &d, double *part, hipStream_t s);
hipError_t launch_kick(const Dev &d, const Params &p, double h, hipStream_t s);
// S(h) from the per-block sums of m V in `part`; rcrit: also the critical radii
// (and the FP32C records and per-block largest rc^2)
hipError_t launch_sun_drift(const Dev &d, double h, int rcrit, const Params &p, const double *part,
                            double *copy_to, hipStream_t s);
// the drift D(dt), preceded by S(sun_h) from the sums after the kick (sun_h = 0: no
// sun drift); writes the sums after the drift to rpart_drift()
hipError_t launch_drift(const Dev &d, const Params &p, double dt, double sun_h,
                        const double *part_in, hipStream_t s);
hipError_t launch_force(const Dev &d, const Params &p, hipStream_t s);
// tables of a single system of d.ntot bodies (O(N) blocks, m0, super-tile pairs of
// ST bodies, nt super-tiles) and a cleared statistics block, written on the device
hipError_t launch_single_tables(const Dev &d, int ST, int nt, double m0, hipStream_t s);
// a from the split partials; kick_h != 0: then `kicks` kicks V += kick_h a (and the
// sums of m V after them into rpart)
// ord: partials by sorted position (the fused pass); enc_count: also the
// statistics of the encounter list the fused pass wrote
hipError_t launch_force_finalize(const Dev &d, const Params &p, double kick_h, int kicks,
                                 hipStream_t s, const int *ord = nullptr, bool enc_count = false);
hipError_t launch_encounters(const Dev &d, double dt, hipStream_t s);
hipError_t launch_diagnostics(const Dev &d, const Params &p, hipStream_t s);
// star impacts, collisions among the listed pairs, ejections (r_eject > 0) of
// the last step (drift arcs of d.snap(), the sorted list), applied in place
hipError_t launch_events(const Dev &d, const Params &p, double tau, double rho, double r_star,
                         double r_eject, hipStream_t s);
// kept bodies (lost == 0) in order: out = 7 planes of ntot (m, Q, V), idx = old index
hipError_t launch_compact(const Dev &d, double *out, int *idx, hipStream_t s);
hipError_t launch_persistent_steps(const Dev &d, const Params &p, double dt, int nsteps,
                                   hipStream_t s);
hipError_t launch_step_stats(const Dev &d, int nsteps, hipStream_t s);
hipError_t launch_enc_sort(const Dev &d, int accumulate, hipStream_t s);
hipError_t launch_enc_gather(const Dev &d, double dt, hipStream_t s);
// fused mode, before the force: an empty list and no flags, the sorted order
// and records of the last drift, and the tile bounds
hipError_t launch_enc_prepare(const Dev &d, double dt, hipStream_t s);
// fused mode: the force and the encounter test in one pass, then (count != 0) the
// list's count
hipError_t launch_force_fused(const Dev &d, const Params &p, double dt, int count, hipStream_t s);
hipError_t launch_enc_test(const Dev &d, double dt, hipStream_t s);
// resolver transfers: both ends of listed pairs [k0, k0 + n) -> res_buf (per end
// m0, m, rc, Q0, V0, index); res_rows (index, Q, V; rows not finite skipped) -> state
hipError_t launch_gather_pairs(const Dev &d, int k0, int n, hipStream_t s);
hipError_t launch_scatter_members(const Dev &d, int k, hipStream_t s);

}  // namespace nb
