// Host runtime of the C ABI declared in include/nb.h: work-table construction,
// workspace carving, validation, state transfer, step sequencing and HIP-graph
// capture.  The library never allocates device memory; every array lives in
// the caller's workspace.
#include "nb.h"
#include "nb_internal.h"
#include "nb_resolve.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

using namespace nb;

struct nb_ctx {
    Params p;
    bool tuned = false;   // tile and algorithm fields taken from the tuning table
    int nsys = 0, ntot = 0, enc_cap = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    Dev d{};
    std::vector<int> off, nbig, rb_first;
    // the caller's workspace (the layout is carved again when bodies are removed)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool have_state = false, have_drift = false, have_enc = false;
    // nb_events ran on the current state: its lost flags are what nb_compact removes
    bool have_events = false;
    // the drift outputs of set `snap` hold the last drift or per-phase step
    // (the persistent step launch does not write them)
    bool snap_valid = false;
    double last_dt = 0.0;
    // captured runs of steps, one per length (1 .. kMaxGraphSteps) for one dt
    struct Graph {
        int steps;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    // second stream on which the sorted encounter test overlaps S(h) and the force
    hipStream_t side = nullptr;
    // one fork and one join event per set of drift outputs
    hipEvent_t ev_fork[kSnapSets] = {}, ev_join[kSnapSets] = {};
    int snap = 0;         // the set of drift outputs the latest drift wrote
    // rpart_prev() holds the momentum of the current V (kept by the steps)
    bool mom_valid = false;
    double graph_dt = 0.0;
    std::string err;
    // close-encounter resolver (resolve = 1): pinned staging of the step's count
    // and pair records (host reads), result rows (host writes; the next step's
    // synchronisation orders their reuse after the copy)
    std::unique_ptr<WorkerPool> pool;
    Groups groups;
    DevStats *h_stats = nullptr;
    double *h_pairs = nullptr, *h_rows = nullptr;
    int res_k = 256;                 // pairs copied with the count (adapts to the counts seen)
    std::vector<int32_t> h_ice, h_jce;
    std::vector<std::pair<int32_t, int32_t>> h_ends;   // (body, record) of every pair end
    std::vector<Member> h_in;
    std::vector<double> h_out;
    long long res_groups = 0, res_bodies = 0;
    int res_max_group = 0, res_fail = 0;
};

namespace {

constexpr size_t kAlign = 256;
constexpr int kDefaultForceJ = 1024;
constexpr int kDefaultForceR = 2;
constexpr int kDefaultEncJ = 1024;
constexpr int kMaxGraphSteps = 8;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int set_err(nb_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIP_OK(ctx, call)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_err((ctx), NB_E_HIP, "%s: %s", #call, hipGetErrorString(e_));        \
    } while (0)

Params to_internal(const nb_params &q)
{
    Params p;
    p.G = q.G;
    p.n_hill = q.n_hill;
    p.inner = q.chg_inner;
    p.mode = q.mode;
    p.drag = q.drag;
    p.sigma0 = q.drag_sigma0;
    p.h = q.drag_h;
    p.cd = q.drag_cd;
    p.rho_p = q.drag_rho_p;
    p.force_r = q.force_r > 0 ? q.force_r : kDefaultForceR;
    // source chunks are whole tiles of kBlock bodies
    p.force_j = q.force_jchunk > 0 ? (q.force_jchunk + kBlock - 1) / kBlock * kBlock : kDefaultForceJ;
    p.enc_j = q.enc_jchunk > 0 ? q.enc_jchunk : kDefaultEncJ;
    p.enc_algo = q.enc_algo;
    p.step_algo = q.step_algo;
    p.force_algo = q.force_algo;
    p.force_g = q.force_g;
    p.resolve = q.resolve;
    p.resolve_threads = q.resolve_threads;
    p.bs_tol = q.bs_tol > 0.0 ? q.bs_tol : 1e-12;
    return p;
}

int resolver_threads(int requested)
{
    if (requested > 0)
        return requested;
    const unsigned hw = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(hw, 16u));
}

int next_pow2(int n);

// Tuning table (written by the autotuner): one line per size class,
//   <arch>/<fp64|fp32c>/n<N>/s<S>[/b<B>] force_algo force_r force_jchunk enc_algo enc_jchunk step_algo [force_g]
// with N the largest system and S the number of systems rounded up to powers of
// two, and B (only when some bodies are small) the largest big-body count, also
// rounded up; '#' starts a comment.  When every tile and algorithm field of the
// parameters is 0 and the table has the context's class, its fields are used.
// Returns NB_E_INVALID if the file cannot be read, NB_OK otherwise (a class not
// in the table leaves the defaults).
int apply_tuning(const nb_params &u, int nsys, const int32_t *off, const int32_t *nbig, Params &q,
                 bool *tuned, std::string *why)
{
    *tuned = false;
    if (!u.autotune_path || u.force_r || u.force_jchunk || u.enc_jchunk || u.enc_algo ||
        u.step_algo || u.force_algo || u.force_g)
        return NB_OK;
    FILE *f = std::fopen(u.autotune_path, "r");
    if (!f) {
        if (why)
            *why = std::string("cannot read the tuning table ") + u.autotune_path;
        return NB_E_INVALID;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        arch = arch.substr(0, arch.find(':'));
    }
    int nmax = 0, bmax = 0;
    bool small = false;
    for (int s = 0; s < nsys; ++s) {
        const int n = off[s + 1] - off[s], b = nbig ? nbig[s] : n;
        nmax = std::max(nmax, n);
        bmax = std::max(bmax, b);
        small = small || b < n;
    }
    std::string key = arch + (q.mode == NB_FP32C ? "/fp32c" : "/fp64") + "/n" +
                      std::to_string(next_pow2(std::max(nmax, 1))) + "/s" +
                      std::to_string(next_pow2(nsys));
    if (small)
        key += "/b" + std::to_string(next_pow2(std::max(bmax, 1)));
    char line[512], k[256];
    int fa, fr, fj, ea, ej, sa, fg;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#')
            continue;
        // the super-tile width (eighth field) may be absent: automatic
        fg = 0;
        const int nf = std::sscanf(line, "%255s %d %d %d %d %d %d %d", k, &fa, &fr, &fj, &ea, &ej, &sa, &fg);
        if (nf < 7 || key != k)
            continue;
        if (fa < 0 || fa == 3 || fa > 4 || (fr != 1 && fr != 2 && fr != 4) || fj <= 0 || ea < 0 || ea > 4 ||
            ej <= 0 || sa < 0 || sa > 2 || (fg != 0 && fg != 1 && fg != 2 && fg != 4))
            break;     // a malformed entry is ignored
        q.force_algo = fa;
        q.force_g = fg;
        q.force_r = fr;
        q.force_j = (fj + kBlock - 1) / kBlock * kBlock;
        q.enc_algo = ea;
        q.enc_j = ej;
        // the persistent launch cannot hand groups to the host resolver
        q.step_algo = q.resolve ? 0 : sa;
        *tuned = true;
        break;
    }
    std::fclose(f);
    return NB_OK;
}

// Step launch: the persistent per-system launch when asked for (or chosen by
// the tuning table) and applicable, else one launch per phase.  It is not an
// automatic choice: it won only for a single system of about 100 bodies, and it
// keeps no drift arcs for nb_encounters / nb_events after a run.
int choose_step_algo(const Params &p, int nsys, const int32_t *off)
{
    int nmax = 0;
    for (int s = 0; s < nsys; ++s)
        nmax = std::max(nmax, off[s + 1] - off[s]);
    bool fits = nmax <= NB_PERSISTENT_MAX_N && p.mode == NB_FP64 && !p.resolve;
    return p.step_algo == 2 && fits ? 2 : 1;
}

// Encounter algorithm: explicit choice, else sorted tiles when bodies have
// many candidate partners on average (tested pairs per body >= 512); with few
// big bodies or small systems every pair through the filters is cheaper.
bool has_small(int nsys, const int32_t *off, const int32_t *nbig);

int max_big(int nsys, const int32_t *off, const int32_t *nbig)
{
    int mb = 0;
    for (int s = 0; s < nsys; ++s)
        mb = std::max(mb, nbig ? nbig[s] : off[s + 1] - off[s]);
    return mb;
}

int choose_enc_algo(const Params &p, int nsys, const int32_t *off, const int32_t *nbig);

// The force pass with the encounter test in it holds four targets per lane only
// by spilling registers: with enc_algo 4 it takes tiles of 128 (two per lane).
void fused_tiles(Params &p, int nsys, const int32_t *off, const int32_t *nbig)
{
    if (choose_enc_algo(p, nsys, off, nbig) == 4 && p.force_r == 4)
        p.force_r = 2;
}

int choose_enc_algo(const Params &p, int nsys, const int32_t *off, const int32_t *nbig)
{
    // 4: the sorted check fused into the symmetric force pass, where it applies
    // (FP32C, every body big, the hot-path mode); else the sorted check alone
    if (p.enc_algo == 4)
        return p.mode == NB_FP32C && !p.resolve && !has_small(nsys, off, nbig) ? 4 : 2;
    if (p.enc_algo >= 1 && p.enc_algo <= 3)
        return p.enc_algo;
    // small bodies and at most kBlock big bodies per system: every body against
    // the big bodies of its system
    if (has_small(nsys, off, nbig) && max_big(nsys, off, nbig) <= kBlock)
        return 3;
    long long pairs = 0;
    for (int s = 0; s < nsys; ++s) {
        const long long n = off[s + 1] - off[s], nb = nbig ? nbig[s] : n;
        pairs += nb * (n - 1) - nb * (nb - 1) / 2;
    }
    return pairs >= 512ll * std::max(off[nsys], 1) ? 2 : 1;
}

int check_params(const nb_params *p)
{
    if (!p)
        return NB_E_INVALID;
    if (!(p->G > 0.0) || !(p->n_hill >= 0.0) || !(p->chg_inner >= 0.0 && p->chg_inner < 1.0))
        return NB_E_INVALID;
    if (p->mode != NB_FP64 && p->mode != NB_FP32C)
        return NB_E_INVALID;
    if (p->drag != 0 && p->drag != 1)
        return NB_E_INVALID;
    if (p->force_r != 0 && p->force_r != 1 && p->force_r != 2 && p->force_r != 4)
        return NB_E_INVALID;
    if (p->force_jchunk < 0 || p->enc_jchunk < 0 || p->enc_algo < 0 || p->enc_algo > 4 ||
        p->step_algo < 0 || p->step_algo > 2)
        return NB_E_INVALID;
    if ((p->resolve != 0 && p->resolve != 1) || p->resolve_threads < 0 || p->force_algo < 0 ||
        (p->force_algo > 2 && p->force_algo != 4) ||
        !(p->bs_tol >= 0.0 && p->bs_tol < 1.0) || (p->resolve && p->step_algo == 2))
        return NB_E_INVALID;
    if (p->drag && !(p->drag_h > 0.0 && p->drag_h * p->drag_h * 3.0 < 1.0 && p->drag_rho_p > 0.0 &&
                     p->drag_sigma0 >= 0.0 && p->drag_cd >= 0.0))
        return NB_E_INVALID;
    return NB_OK;
}

int check_offsets(int nsys, const int32_t *off, const int32_t *nbig)
{
    if (nsys <= 0 || !off || off[0] != 0)
        return NB_E_INVALID;
    for (int s = 0; s < nsys; ++s)
        if (off[s + 1] < off[s] || (nbig && (nbig[s] < 0 || nbig[s] > off[s + 1] - off[s])))
            return NB_E_INVALID;
    if (off[nsys] <= 0)
        return NB_E_INVALID;
    return NB_OK;
}

bool has_small(int nsys, const int32_t *off, const int32_t *nbig)
{
    if (!nbig)
        return false;
    for (int s = 0; s < nsys; ++s)
        if (nbig[s] < off[s + 1] - off[s])
            return true;
    return false;
}

// Host-side tables of a context.
struct Tables {
    std::vector<RBlk> rblk;
    std::vector<int> rb_first, rb_count;
    std::vector<FWork> fwork;
    std::vector<int> nsplit;
    int maxs = 1;
    std::vector<PWork> ework, dwork;
    std::vector<int> dw_first, dw_count;
    std::vector<int> sys_of;
    // sorted encounter check
    std::vector<int> cell_base, cell_cnt;
    int ncell = 0;
    std::vector<Tile> tiles;
    long long tp_cap = 0;
    std::vector<int2> units;    // sorted check: (tile A, first of 64 tiles B >= A) culling units
    bool enc_sorted = false;
    bool enc_few = false;
    bool enc_fused = false;   // sorted check inside the symmetric force pass
    std::vector<int> tile_first;
    bool force_few = false;
    bool force_sym = false;
    int sym_g = 1;        // tiles per super-tile of the symmetric force
    // symmetric FP32C force over the radial order: tiles of 64 positions
    bool force_rsort = false;
    int nrtile = 0;
    std::vector<int> rtf;
    // persistent step launch: systems largest first
    std::vector<PSys> psys;
};

// Unordered pair items (i < j) of one system with i < nb (the big bodies: pairs
// of two small bodies do not interact): targets in tiles of kBlock, sources in
// chunks of J; an item exists when some source index exceeds some target index.
void pair_items(int a, int n, int nb, int J, std::vector<PWork> &out)
{
    for (int i0 = 0; i0 < nb; i0 += kBlock) {
        int ni = std::min(kBlock, nb - i0);
        for (int j0 = 0; j0 < n; j0 += J) {
            int nj = std::min(J, n - j0);
            if (j0 + nj - 1 > i0)
                out.push_back(PWork{a + i0, ni, a + j0, nj});
        }
    }
}

// Split partials of the symmetric force: 3 values per body and super-tile of
// TI bodies of its system (quadratic in the system size; doubles, or floats with
// FP32C pair arithmetic).
constexpr long long kSymPartialMax = 4ll << 30;

// Most source chunks per system of the ordered force (its partials: 3 doubles
// per body and chunk).
constexpr int kMaxOrderedSplits = 64;

long long sym_partial_bytes(const Params &p, int nsys, const int32_t *off, int TI)
{
    const long long per = p.mode == NB_FP32C ? 3 * sizeof(float) : 3 * sizeof(double);
    long long b = 0;
    for (int s = 0; s < nsys; ++s) {
        const long long n = off[s + 1] - off[s];
        b += per * n * ((n + TI - 1) / TI);
    }
    return b;
}

long long sym_items(int nsys, const int32_t *off, int TI)
{
    long long c = 0;
    for (int s = 0; s < nsys; ++s) {
        const long long nt = (off[s + 1] - off[s] + TI - 1) / TI;
        c += nt * (nt + 1) / 2;
    }
    return c;
}

// Tiles per super-tile of the symmetric force: the one asked for, else the
// widest whose work items (super-tile pairs, one workgroup each) reach
// kSymMinItems(g).  Measured on whole steps: wider super-tiles write fewer
// partials but cost the force kernel its rounds' barriers, which pays from
// about 32 workgroups per compute unit (256 systems of 200-4000 bodies: 2;
// 131072 bodies: 4), not at 16384 bodies (1).
int sym_width(const Params &p, int nsys, const int32_t *off)
{
    if (p.force_g == 1 || p.force_g == 2 || p.force_g == 4)
        return p.force_g;
    const int T = 64 * p.force_r;
    for (int g = 4; g > 1; g /= 2)
        if (sym_items(nsys, off, g * T) >= kSymMinItems(g))
            return g;
    return 1;
}

void build_tables(const Params &p, int nsys, const int32_t *off, const int32_t *nbig, Tables &t)
{
    const int ea = choose_enc_algo(p, nsys, off, nbig);
    t.enc_sorted = ea == 2 || ea == 4;
    t.enc_few = ea == 3;
    t.enc_fused = ea == 4;
    // symmetric tile pairs: every body big (asked for, or automatic while their
    // split partials, 3 values per body and tile of its system, stay within
    // kSymPartialMax; beyond that the ordered pairs' partials are bounded)
    t.sym_g = sym_width(p, nsys, off);
    t.force_sym = p.force_algo != 1 && !has_small(nsys, off, nbig) &&
                  (p.force_algo == 2 || p.force_algo == 4 ||
                   sym_partial_bytes(p, nsys, off, t.sym_g * 64 * p.force_r) <= kSymPartialMax);
    // the fused pass is the symmetric force's: without it, the sorted check alone
    t.enc_fused = t.enc_fused && t.force_sym;
    // 4: the symmetric FP32C force over the radial order (not with the fused
    // pass, which runs over the encounter check's order)
    t.force_rsort = p.force_algo == 4 && p.mode == NB_FP32C && t.force_sym && !t.enc_fused;
    t.rtf.assign(nsys, 0);
    t.nrtile = 0;
    if (t.force_rsort)
        for (int s = 0; s < nsys; ++s) {
            t.rtf[s] = t.nrtile;
            t.nrtile += (off[s + 1] - off[s] + 63) / 64;
        }
    t.rb_first.assign(nsys, 0);
    t.rb_count.assign(nsys, 0);
    t.nsplit.assign(nsys, 0);
    t.dw_first.assign(nsys, 0);
    t.dw_count.assign(nsys, 0);
    t.sys_of.assign(off[nsys], 0);
    const int TI = 64 * p.force_r;
    for (int s = 0; s < nsys; ++s) {
        int a = off[s], n = off[s + 1] - off[s];
        for (int i = a; i < a + n; ++i)
            t.sys_of[i] = s;
        t.rb_first[s] = (int)t.rblk.size();
        for (int b = 0; b < n; b += kBlock)
            t.rblk.push_back(RBlk{s, a + b, a + std::min(n, b + kBlock), t.rtf[s] + b / 64});
        t.rb_count[s] = (int)t.rblk.size() - t.rb_first[s];
        if (n == 0)
            continue;
        // sources are the big bodies [a, a + nb) only (Sec. 2.1)
        const int nb = nbig ? nbig[s] : n;
        if (t.force_sym) {
            // unordered pairs (I <= J) of super-tiles of ST bodies; super-tile I's
            // sums go to slot J, super-tile J's to slot I (the item's pad field)
            const int ST = t.sym_g * TI;
            const int nt = (n + ST - 1) / ST;
            t.nsplit[s] = nt;
            t.maxs = std::max(t.maxs, nt);
            for (int I = 0; I < nt; ++I)
                for (int J = I; J < nt; ++J)
                    t.fwork.push_back(FWork{a + I * ST, std::min(ST, n - I * ST), a + J * ST,
                                            std::min(ST, n - J * ST), J, s,
                                            t.rb_first[s] + (J * ST) / kBlock, I});
        } else {
            // source chunks of J bodies, widened (whole O(N) blocks) so that a
            // system has at most kMaxOrderedSplits of them
            int J = p.force_j;
            if ((nb + J - 1) / J > kMaxOrderedSplits)
                J = ((nb + kMaxOrderedSplits - 1) / kMaxOrderedSplits + kBlock - 1) / kBlock * kBlock;
            int S = (nb + J - 1) / J;
            t.nsplit[s] = S;
            t.maxs = std::max(t.maxs, S);
            for (int i0 = 0; i0 < n; i0 += TI)
                for (int k = 0; k < S; ++k) {
                    int j0 = k * J;
                    t.fwork.push_back(FWork{a + i0, std::min(TI, n - i0), a + j0,
                                            std::min(J, nb - j0), k, s,
                                            t.rb_first[s] + j0 / kBlock, 0});
                }
        }
        pair_items(a, n, nb, p.enc_j, t.ework);
        t.dw_first[s] = (int)t.dwork.size();
        pair_items(a, n, nb, p.enc_j, t.dwork);
        t.dw_count[s] = (int)t.dwork.size() - t.dw_first[s];
    }
    // few-source force kernels: every system's sources fit one LDS slice (and one
    // split), and there are enough target tiles (>= 1024) to fill the GPU by waves
    {
        int maxnb = 0;
        for (int s = 0; s < nsys; ++s)
            maxnb = std::max(maxnb, nbig ? nbig[s] : off[s + 1] - off[s]);
        t.force_few = !t.force_sym && maxnb <= 256 && maxnb <= p.force_j && t.fwork.size() >= 1024;
    }
    // sorted encounter check: about N_s/8 cells per system (a power of two) and
    // tiles of 64 consecutive sorted bodies
    t.cell_base.assign(nsys, 0);
    t.cell_cnt.assign(nsys, 0);
    for (int s = 0; s < nsys; ++s) {
        int n = off[s + 1] - off[s];
        int c = 1;
        while (c * 8 < n)
            c <<= 1;
        t.cell_base[s] = t.ncell;
        t.cell_cnt[s] = c;
        t.ncell += c;
        int first = (int)t.tiles.size();
        t.tile_first.push_back(first);
        int nt = (n + 63) / 64;
        for (int k = 0; k < nt; ++k)
            t.tiles.push_back(Tile{s, off[s] + 64 * k, std::min(64, n - 64 * k), first + nt - 1});
        t.tp_cap += (long long)nt * (nt + 1) / 2;
        for (int A = first; A < first + nt; ++A)
            for (int b0 = A; b0 < first + nt; b0 += 64)
                t.units.push_back(make_int2(A, b0));
    }
    for (int s = 0; s < nsys; ++s)
        if (off[s + 1] > off[s])
            t.psys.push_back(PSys{s, off[s], off[s + 1] - off[s],
                                  nbig ? nbig[s] : off[s + 1] - off[s]});
    std::stable_sort(t.psys.begin(), t.psys.end(),
                     [](const PSys &x, const PSys &y) { return x.n > y.n; });
    // longest work first, so the hardware dispatcher packs the tail; over the
    // radial order the super-tile pairs nearest the diagonal (neighbouring
    // shells: no far tile pairs, most changeover pairs) cost most
    const bool rs = t.force_rsort;
    std::stable_sort(t.fwork.begin(), t.fwork.end(), [rs](const FWork &x, const FWork &y) {
        const long long cx = (long long)x.ni * x.nj, cy = (long long)y.ni * y.nj;
        if (cx != cy || !rs)
            return cx > cy;
        return x.j0 - x.i0 < y.j0 - y.i0;
    });
    auto pairs = [](const PWork &w) {
        long long c = 0;
        for (int k = 0; k < w.ni; ++k) {
            int i = w.i0 + k;
            int lo = std::max(w.j0, i + 1);
            c += std::max(0, w.j0 + w.nj - lo);
        }
        return c;
    };
    std::vector<std::pair<long long, int>> cost;
    for (size_t k = 0; k < t.ework.size(); ++k)
        cost.push_back({pairs(t.ework[k]), (int)k});
    std::stable_sort(cost.begin(), cost.end(),
                     [](const std::pair<long long, int> &x, const std::pair<long long, int> &y) {
                         return x.first > y.first;
                     });
    std::vector<PWork> e2;
    for (auto &c : cost)
        e2.push_back(t.ework[c.second]);
    t.ework.swap(e2);
}

int next_pow2(int n)
{
    int p = 1;
    while (p < n)
        p <<= 1;
    return p;
}

// Carve the workspace (base == nullptr: sizes only).  Returns total bytes.
// Bytes of drift outputs the further sets may take.
constexpr long long kSnapSetBytes = 1ll << 30;

// Sets of drift outputs: kSnapSets when the check of a step may run on a second
// queue (per-phase steps, the check outside the force pass, no host resolver)
// and the further sets fit in kSnapSetBytes; else two.
int snap_sets(const Params &p, const Tables &t, int ntot)
{
    const long long per = (long long)ntot * (13 * sizeof(double) + 2 * sizeof(double4));
    if (p.resolve || p.step_algo == 2 || t.enc_fused || per * (kSnapSets - 1) > kSnapSetBytes)
        return 2;
    return kSnapSets;
}

size_t carve(const Params &p, int nsys, int ntot, int enc_cap, const Tables &t, char *base, Dev &d)
{
    size_t cur = 0;
    auto take = [&](size_t bytes) -> char * {
        size_t at = cur;
        cur = align_up(cur + bytes);
        return base ? base + at : nullptr;
    };
    const size_t nd = (size_t)ntot * sizeof(double);
    d.ntot = ntot;
    d.nsys = nsys;
    double **planes[] = {&d.m,   &d.qx,  &d.qy,  &d.qz,  &d.vx,  &d.vy,  &d.vz,  &d.ax,
                         &d.ay,  &d.az,  &d.rc,  &d.q0x, &d.q0y, &d.q0z, &d.v0x, &d.v0y,
                         &d.v0z, &d.q1x, &d.q1y, &d.q1z, &d.v1x, &d.v1y, &d.v1z, &d.rc1};
    for (double **pl : planes)
        *pl = (double *)take(nd);
    d.pk = (float4 *)take((size_t)ntot * 2 * sizeof(float4));
    d.mr = (double4 *)take((size_t)ntot * sizeof(double4));
    d.cr = (double4 *)take((size_t)ntot * sizeof(double4));
    // further sets of drift outputs: one per step of a captured run when the
    // check runs on a second queue and the sets stay within kSnapSetBytes, else two
    d.nsnap = snap_sets(p, t, ntot);
    for (int k = 0; k + 1 < d.nsnap; ++k) {
        Snap &a = d.alt[k];
        double **alt[] = {&a.q0x, &a.q0y, &a.q0z, &a.v0x, &a.v0y, &a.v0z, &a.q1x,
                          &a.q1y, &a.q1z, &a.v1x, &a.v1y, &a.v1z, &a.rc1};
        for (double **pl : alt)
            *pl = (double *)take(nd);
        a.mr = (double4 *)take((size_t)ntot * sizeof(double4));
        a.cr = (double4 *)take((size_t)ntot * sizeof(double4));
    }
    d.kflag = (int *)take((size_t)ntot * sizeof(int));
    d.ce = (int *)take((size_t)ntot * sizeof(int));
    d.sys_of = (int *)take((size_t)ntot * sizeof(int));
    d.nbig = (int *)take((size_t)nsys * sizeof(int));
    d.m0 = (double *)take((size_t)nsys * sizeof(double));
    d.off = (int *)take((size_t)(nsys + 1) * sizeof(int));
    // nsplit, then diagnostic item ranges (dw_first, dw_count) right after it
    d.nsplit = (int *)take((size_t)3 * nsys * sizeof(int));
    d.rb_first = (int *)take((size_t)nsys * sizeof(int));
    d.rb_count = (int *)take((size_t)nsys * sizeof(int));
    d.nrb = (int)t.rblk.size();
    d.rblk = (RBlk *)take(t.rblk.size() * sizeof(RBlk));
    d.nfw = (int)t.fwork.size();
    d.fwork = (FWork *)take(t.fwork.size() * sizeof(FWork));
    d.maxs = t.maxs;
    d.ns_all = t.maxs;
    for (int s = 0; s < nsys; ++s)
        if (t.rb_count[s] > 0 && t.nsplit[s] != t.maxs)
            d.ns_all = 0;
    d.new_ = (int)t.ework.size();
    d.ework = (PWork *)take(t.ework.size() * sizeof(PWork));
    d.ndw = (int)t.dwork.size();
    d.dwork = (PWork *)take(t.dwork.size() * sizeof(PWork));
    d.rpart = (double *)take((size_t)d.nrb * 12 * sizeof(double));
    d.tile_rc2 = (double *)take((size_t)std::max(d.nrb, 1) * sizeof(double));
    d.ptot = (double *)take((size_t)std::max(nsys, 1) * 4 * sizeof(double));
    d.sys_total = 0;
    for (int s = 0; s < nsys; ++s)
        if (t.rb_count[s] > 64)
            d.sys_total = 1;
    // split partials: FP32 with FP32C pair arithmetic (each rounding at most
    // 2^-24 of a partial, so of A_i over all of a body's partials), else FP64
    d.fpart = nullptr;
    d.fpart32 = nullptr;
    if (p.mode == NB_FP32C)
        d.fpart32 = (float *)take((size_t)3 * d.maxs * ntot * sizeof(float));
    else
        d.fpart = (double *)take((size_t)3 * d.maxs * ntot * sizeof(double));
    d.dpart = (double *)take((size_t)std::max(d.ndw, 1) * 4 * sizeof(double));
    d.bpart = (double *)take((size_t)std::max(d.nrb, 1) * 8 * sizeof(double));
    d.diag = (double *)take((size_t)nsys * 8 * sizeof(double));
    d.enc_cap = enc_cap;
    d.keys_p2 = next_pow2(std::max(enc_cap, 2));
    d.keys = (unsigned long long *)take((size_t)d.keys_p2 * sizeof(unsigned long long));
    d.ice = (int *)take((size_t)std::max(enc_cap, 1) * sizeof(int));
    d.jce = (int *)take((size_t)std::max(enc_cap, 1) * sizeof(int));
    d.stats = (DevStats *)take(sizeof(DevStats));
    d.step_chunk = 256;
    d.step_nce = (int *)take((size_t)d.step_chunk * sizeof(int));
    d.npsys = (int)t.psys.size();
    d.pmax_n = t.psys.empty() ? 0 : t.psys[0].n;
    d.psys = (PSys *)take(t.psys.size() * sizeof(PSys));
    d.enc_sorted = t.enc_sorted;
    d.enc_few = t.enc_few ? 1 : 0;
    d.force_few = t.force_few ? 1 : 0;
    d.force_sym = t.force_sym ? 1 : 0;
    d.sym_g = t.sym_g;
    d.force_rsort = t.force_rsort ? 1 : 0;
    d.nrtile = t.nrtile;
    d.rord = d.force_rsort ? (int *)take((size_t)ntot * sizeof(int)) : nullptr;
    d.rtf = d.force_rsort ? (int *)take((size_t)nsys * sizeof(int)) : nullptr;
    d.rtb = d.force_rsort ? (float4 *)take((size_t)t.nrtile * sizeof(float4)) : nullptr;
    if (d.enc_sorted) {
        d.lnr_part = (double *)take((size_t)std::max(d.nrb, 1) * 2 * sizeof(double));
        for (int k = 0; k + 1 < d.nsnap; ++k)
            d.alt[k].lnr_part = (double *)take((size_t)std::max(d.nrb, 1) * 2 * sizeof(double));
        d.cell_of = (int *)take((size_t)ntot * sizeof(int));
        d.slot_of = (int *)take((size_t)ntot * sizeof(int));
        d.ncell = t.ncell;
        d.cell_cnt = (int *)take((size_t)t.ncell * sizeof(int));
        d.cell_off = (int *)take((size_t)t.ncell * sizeof(int));
        d.scan_part = (int *)take((size_t)(t.ncell / kScanChunkCells + 1) * sizeof(int));
        d.sys_cell_base = (int *)take((size_t)nsys * sizeof(int));
        d.sys_cell_cnt = (int *)take((size_t)nsys * sizeof(int));
        d.ord = (int *)take((size_t)ntot * sizeof(int));
        d.srec = (SRec *)take((size_t)ntot * sizeof(SRec));
        d.ntile = (int)t.tiles.size();
        d.tiles = (Tile *)take(t.tiles.size() * sizeof(Tile));
        d.tileb = (TileB *)take(t.tiles.size() * sizeof(TileB));
        d.tp_cap = (int)std::min<long long>(t.tp_cap, 1ll << 30);
        d.tpairs = (int2 *)take((size_t)d.tp_cap * sizeof(int2));
        d.nunit = (int)t.units.size();
        d.units = (int2 *)take(t.units.size() * sizeof(int2));
        d.tile_first = (int *)take((size_t)nsys * sizeof(int));
    }
    d.enc_fused = t.enc_fused ? 1 : 0;
    d.em = t.enc_sorted ? (float4 *)take((size_t)ntot * 2 * sizeof(float4)) : nullptr;
    d.eg = t.enc_sorted ? (float4 *)take((size_t)ntot * sizeof(float4)) : nullptr;
    d.flag = (int *)take(4 * sizeof(int));
    d.stage = (double *)take((size_t)7 * nd);
    d.lost = (int *)take((size_t)ntot * sizeof(int));
    d.evroot = (int *)take((size_t)ntot * sizeof(int));
    d.evflag = (int *)take((size_t)std::max(std::max(enc_cap, d.nrb), 1) * sizeof(int));
    d.evmem = (int *)take((size_t)2 * std::max(enc_cap, 1) * sizeof(int));
    d.evcnt = (int *)take(4 * sizeof(int));
    d.cmp_pos = (int *)take((size_t)(d.nrb + 1) * sizeof(int));
    d.evidx = (int *)take((size_t)std::max(ntot, 1) * sizeof(int));
    d.evpart = (double *)take((size_t)std::max(d.nrb, 1) * 8 * sizeof(double));
    d.evsys = (double *)take((size_t)std::max(nsys, 1) * 8 * sizeof(double));
    if (p.resolve) {
        // every member of a resolved group is an end of a listed pair
        d.res_cap = std::max(enc_cap, 1);
        d.res_buf = (double *)take((size_t)d.res_cap * 20 * sizeof(double));
        d.res_rows = (double *)take((size_t)d.res_cap * 2 * 7 * sizeof(double));
    }
    return cur;
}

int sync(nb_ctx *c)
{
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return NB_OK;
}

int read_int(nb_ctx *c, const int *dev, int *host)
{
    HIP_OK(c, hipMemcpyAsync(host, dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

int copy(nb_ctx *c, void *dst, const void *src, size_t bytes)
{
    if (bytes == 0)
        return NB_OK;
    HIP_OK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, c->stream));
    return NB_OK;
}

int reset_stats(nb_ctx *c)
{
    HIP_OK(c, launch_fill_i32((int *)c->d.stats, (int)(sizeof(DevStats) / sizeof(int)), 0,
                              c->stream));
    return NB_OK;
}

// Critical radii (and FP32 source records), then the force at the current Q.
int enqueue_force(nb_ctx *c)
{
    HIP_OK(c, launch_sun_drift(c->d, 0.0, 1, c->p, c->d.rpart, nullptr, c->stream));
    HIP_OK(c, launch_force(c->d, c->p, c->stream));
    HIP_OK(c, launch_force_finalize(c->d, c->p, 0.0, 1, c->stream));
    return NB_OK;
}

// One hybrid step K(h) S(h) D(dt) C S(h) [rc, F] K(h).  In a run of steps the
// closing K(h) of one step and the opening K(h) of the next are one launch that
// kicks twice (rounded as two kicks): only the run's first step opens with a
// kick launch (`first`), only its last closes with a single kick (`last`).  The
// first S(h) takes P from the momentum before the kicks (rpart_prev(), kept by
// the previous second S(h), or summed at the start of a call): the kicks leave
// it unchanged, the pair forces cancelling in the sum.  Not with gas drag, whose
// kick depends on V and changes P: there each step kicks on its own and its
// S(h) takes P after the kick.
bool merged_kicks(const nb_ctx *c)
{
    return !c->p.drag;
}

// K(h) S(h) D(dt) C of a step (S(h) inside the drift launch), the drift's
// outputs in set 0.
int enqueue_step_head(nb_ctx *c, double dt, bool first)
{
    const double h = 0.5 * dt;
    const Dev &d = c->d;
    if (first)
        HIP_OK(c, launch_kick(d, c->p, h, c->stream));
    HIP_OK(c, launch_drift(d, c->p, dt, h, merged_kicks(c) ? d.rpart_prev() : d.rpart, c->stream));
    // fused: the sorted order and tile bounds now, the pair test inside the force pass
    if (d.enc_fused)
        HIP_OK(c, launch_enc_prepare(d, dt, c->stream));
    else
        HIP_OK(c, launch_encounters(d, dt, c->stream));
    c->snap = 0;
    return NB_OK;
}

// S(h), critical radii, F, K(h) of a step (and the next step's K(h) unless `last`).
int enqueue_step_tail(nb_ctx *c, double dt, bool last)
{
    const double h = 0.5 * dt;
    const Dev &d = c->d;
    HIP_OK(c, launch_sun_drift(d, h, 1, c->p, d.rpart_drift(),
                               merged_kicks(c) ? d.rpart_prev() : nullptr, c->stream));
    // fused: the force over the sorted order with the encounter test in it; its
    // partials are by sorted position, which the finalize maps back to bodies
    const bool fz = d.enc_fused;
    const int *ord = fz ? d.ord : nullptr;
    if (fz)
        HIP_OK(c, launch_force_fused(d, c->p, dt, 0, c->stream));
    else
        HIP_OK(c, launch_force(d, c->p, c->stream));
    if (c->p.drag) {
        HIP_OK(c, launch_force_finalize(d, c->p, 0.0, 1, c->stream, ord, fz));
        HIP_OK(c, launch_kick(d, c->p, h, c->stream));
    } else {
        HIP_OK(c, launch_force_finalize(d, c->p, h, last ? 1 : 2, c->stream, ord, fz));
    }
    return NB_OK;
}

// A run of `steps` steps (kicks merged between them).  On a context with a
// stream the encounter check of a step runs on a second stream (graph branches
// under capture) beside the rest of that step and the next ones: the drifts
// write the nsnap sets of drift outputs in turn, and a drift waits only for the
// check that read its set nsnap steps earlier (none in a captured run of at most
// nsnap steps); the run ends with a join.  The
// step's own chain is enqueued (recorded) before the branch, so that it keeps
// the stream's hardware queue and only the branch and the joins cross queues.
int enqueue_run(nb_ctx *c, double dt, int steps)
{
    const bool merge = merged_kicks(c);
    const double h = 0.5 * dt;
    for (int k = 0; k < steps; ++k) {
        const bool first = k == 0 || !merge, last = k == steps - 1 || !merge;
        int r;
        if (!c->side || c->d.enc_fused) {
            if ((r = enqueue_step_head(c, dt, first)) || (r = enqueue_step_tail(c, dt, last)))
                return r;
            continue;
        }
        const int par = k % c->d.nsnap;
        const Dev d = c->d.with_snap(par);
        if (k >= c->d.nsnap)
            HIP_OK(c, hipStreamWaitEvent(c->stream, c->ev_join[par], 0));
        if (first)
            HIP_OK(c, launch_kick(d, c->p, h, c->stream));
        HIP_OK(c, launch_drift(d, c->p, dt, h, merge ? d.rpart_prev() : d.rpart, c->stream));
        HIP_OK(c, hipEventRecord(c->ev_fork[par], c->stream));
        if ((r = enqueue_step_tail(c, dt, last)))
            return r;
        HIP_OK(c, hipStreamWaitEvent(c->side, c->ev_fork[par], 0));
        HIP_OK(c, launch_encounters(d, dt, c->side));
        HIP_OK(c, hipEventRecord(c->ev_join[par], c->side));
        c->snap = par;
    }
    if (c->side && !c->d.enc_fused && steps > 0)
        HIP_OK(c, hipStreamWaitEvent(c->stream, c->ev_join[(steps - 1) % c->d.nsnap], 0));
    return NB_OK;
}

// Between C and the second S(h) of the full method.  The device packs both ends
// of the step's listed pairs (the first res_k of them, more on a second pass);
// one synchronisation brings the count and those records to the host, which
// groups the pairs, integrates every group and sends (index, Q, V) rows back to
// a scatter kernel; the rest of the step is enqueued without waiting.
int resolve_step(nb_ctx *c, double dt)
{
    Dev &d = c->d;
    const int kcap = d.res_cap;
    if (!c->h_stats) {
        HIP_OK(c, hipHostMalloc((void **)&c->h_stats, sizeof(DevStats), hipHostMallocDefault));
        HIP_OK(c, hipHostMalloc((void **)&c->h_pairs, (size_t)kcap * 20 * sizeof(double),
                                hipHostMallocDefault));
        HIP_OK(c, hipHostMalloc((void **)&c->h_rows, (size_t)kcap * 2 * 7 * sizeof(double),
                                hipHostMallocDefault));
    }
    int K = std::min(c->res_k, kcap);
    // the list in (i, j) order, so that the groups do not depend on the append order
    HIP_OK(c, launch_enc_sort(d, 0, c->stream));
    HIP_OK(c, launch_gather_pairs(d.with_snap(c->snap), 0, K, c->stream));
    HIP_OK(c, hipMemcpyAsync(c->h_stats, d.stats, sizeof(DevStats), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipMemcpyAsync(c->h_pairs, d.res_buf, (size_t)K * 20 * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    int r = sync(c);
    if (r)
        return r;
    const int npairs = std::min(c->h_stats->cur_nce, d.enc_cap);
    if (npairs > K) {
        // more pairs than expected: gather and copy the rest
        HIP_OK(c, launch_gather_pairs(d.with_snap(c->snap), K, npairs - K, c->stream));
        HIP_OK(c, hipMemcpyAsync(c->h_pairs + (size_t)K * 20, d.res_buf,
                                 (size_t)(npairs - K) * 20 * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        if ((r = sync(c)))
            return r;
    }
    // next step's prefetch: twice this count, at least 256 pairs
    int nk = 256;
    while (nk < 2 * npairs && nk < kcap)
        nk <<= 1;
    c->res_k = nk;
    if (npairs <= 0)
        return NB_OK;
    c->h_ice.resize(npairs);
    c->h_jce.resize(npairs);
    c->h_ends.resize(2 * (size_t)npairs);
    for (int k = 0; k < npairs; ++k) {
        const double *rec = c->h_pairs + 20 * (size_t)k;
        const double bi = rec[9], bj = rec[19];
        if (!(bi >= 0.0 && bi < c->ntot && bj >= 0.0 && bj < c->ntot))
            return set_err(c, NB_E_HIP, "resolver: pair %d has an index out of range", k);
        c->h_ice[k] = (int32_t)bi;
        c->h_jce[k] = (int32_t)bj;
        c->h_ends[2 * (size_t)k] = {c->h_ice[k], 2 * k};
        c->h_ends[2 * (size_t)k + 1] = {c->h_jce[k], 2 * k + 1};
    }
    std::sort(c->h_ends.begin(), c->h_ends.end());
    build_groups(npairs, c->h_ice.data(), c->h_jce.data(), c->groups);
    const int k = (int)c->groups.body.size();
    c->h_in.resize(k);
    c->h_out.resize((size_t)6 * k);
    for (int e = 0; e < k; ++e) {
        const int32_t b = c->groups.body[e];
        auto it = std::lower_bound(c->h_ends.begin(), c->h_ends.end(), std::make_pair(b, (int32_t)-1));
        std::memcpy(&c->h_in[e], c->h_pairs + 10 * (size_t)it->second, sizeof(Member));
        c->h_in[e].pad = 0.0;
    }
    if (!c->pool && resolver_threads(c->p.resolve_threads) > 1)
        c->pool.reset(new WorkerPool(resolver_threads(c->p.resolve_threads)));
    ResolveTotals t = resolve_groups(c->groups, c->h_in.data(), c->h_out.data(), c->p.G,
                                     c->p.inner, dt, c->p.bs_tol, c->pool.get());
    c->res_groups += t.groups;
    c->res_bodies += t.bodies;
    c->res_max_group = std::max(c->res_max_group, t.max_group);
    c->res_fail += t.failed;
    for (int e = 0; e < k; ++e) {
        double *row = c->h_rows + 7 * (size_t)e;
        row[0] = (double)c->groups.body[e];
        std::memcpy(row + 1, c->h_out.data() + 6 * (size_t)e, 6 * sizeof(double));
    }
    HIP_OK(c, hipMemcpyAsync(d.res_rows, c->h_rows, (size_t)k * 7 * sizeof(double),
                             hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, launch_scatter_members(d, k, c->stream));
    // the second S(h) takes the momentum of the resolved velocities
    HIP_OK(c, launch_momentum(d, d.rpart_drift(), c->stream));
    return NB_OK;
}

void drop_graph(nb_ctx *c)
{
    for (auto &g : c->graphs)
        (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

// The captured run of `steps` steps for this dt: from the cache, else captured
// and instantiated now (a new dt drops the runs of the old one).
int graph_for(nb_ctx *c, double dt, int steps, hipGraphExec_t *out)
{
    if (!c->graphs.empty() && c->graph_dt != dt)
        drop_graph(c);
    for (auto &g : c->graphs)
        if (g.steps == steps) {
            *out = g.exec;
            return NB_OK;
        }
    hipGraph_t g = nullptr;
    // capturing runs nothing: the set of drift outputs of the last step run
    // stays what it was
    const int snap = c->snap;
    HIP_OK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_run(c, dt, steps);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->snap = snap;
    if (rc != NB_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess)
        return set_err(c, NB_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return set_err(c, NB_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    c->graph_dt = dt;
    c->graphs.push_back({steps, x});
    *out = x;
    return NB_OK;
}

// How nb_step splits nsteps steps into captured runs: full runs of
// kMaxGraphSteps, then one run of the remainder.
void graph_lengths(int nsteps, int *full, int *rest)
{
    *full = nsteps / kMaxGraphSteps;
    *rest = nsteps % kMaxGraphSteps;
}

// nsteps whole steps on the context's stream, by the context's step launch.
int enqueue_steps(nb_ctx *c, double dt, int nsteps)
{
    int r = NB_OK;
    int done = 0;
    if (c->p.step_algo != 2 && merged_kicks(c) && !c->mom_valid && nsteps > 0) {
        // the first S(h) takes P from the momentum before the kicks
        HIP_OK(c, launch_momentum(c->d, c->d.rpart_prev(), c->stream));
        c->mom_valid = true;
    }
    if (c->p.resolve) {
        // the host takes part in every step: direct launches, no graph
        for (; done < nsteps; ++done) {
            if ((r = enqueue_step_head(c, dt, true)) || (r = resolve_step(c, dt)) ||
                (r = enqueue_step_tail(c, dt, true)))
                return r;
            c->snap_valid = true;
        }
        return NB_OK;
    }
    if (c->p.step_algo == 2) {
        // persistent per-system launches of at most step_chunk steps each
        c->snap = 0;
        c->mom_valid = false;
        while (done < nsteps) {
            int k = std::min(nsteps - done, c->d.step_chunk);
            HIP_OK(c, launch_fill_i32(&c->d.stats->cur_nce, 1, 0, c->stream));
            HIP_OK(c, launch_persistent_steps(c->d, c->p, dt, k, c->stream));
            HIP_OK(c, launch_step_stats(c->d, k, c->stream));
            done += k;
        }
        if (nsteps > 0) {
            HIP_OK(c, launch_enc_sort(c->d, 0, c->stream));
            // the persistent launch keeps its drift outputs in registers and LDS
            c->snap_valid = false;
        }
        return NB_OK;
    }
    if (c->stream && nsteps > 0) {
        // captured runs: full runs of kMaxGraphSteps, then the remainder
        int full, rest;
        graph_lengths(nsteps, &full, &rest);
        hipGraphExec_t gx = nullptr;
        if (full > 0 && (r = graph_for(c, dt, kMaxGraphSteps, &gx)))
            return r;
        for (int k = 0; k < full; ++k)
            HIP_OK(c, hipGraphLaunch(gx, c->stream));
        if (rest > 0) {
            if ((r = graph_for(c, dt, rest, &gx)))
                return r;
            HIP_OK(c, hipGraphLaunch(gx, c->stream));
        }
        // a run's steps write the sets of drift outputs in turn, from set 0
        c->snap = ((rest > 0 ? rest : kMaxGraphSteps) - 1) % c->d.nsnap;
        c->snap_valid = true;
        return NB_OK;
    }
    // no stream (the null stream cannot be captured): direct launches in runs
    // of kMaxGraphSteps, then the remainder
    while (done < nsteps) {
        const int g = std::min(nsteps - done, kMaxGraphSteps);
        if ((r = enqueue_run(c, dt, g)))
            return r;
        done += g;
    }
    if (nsteps > 0)
        c->snap_valid = true;
    return NB_OK;
}

int copy_list(nb_ctx *c, int cap, int *nce, int32_t *ice, int32_t *jce, int32_t *ce, int where)
{
    // the latest check's list, put in (i, j) order as it is read
    HIP_OK(c, launch_enc_sort(c->d, 0, c->stream));
    DevStats st;
    HIP_OK(c, hipMemcpyAsync(&st, c->d.stats, sizeof st, hipMemcpyDeviceToHost, c->stream));
    int r = sync(c);
    if (r)
        return r;
    int count = st.cur_nce;
    if (nce)
        *nce = count;
    int n = std::min(count, std::min(cap, c->enc_cap));
    if (n < 0)
        n = 0;
    (void)where;   // hipMemcpyDefault resolves host or device pointers
    if (ice && (r = copy(c, ice, c->d.ice, (size_t)n * sizeof(int))))
        return r;
    if (jce && (r = copy(c, jce, c->d.jce, (size_t)n * sizeof(int))))
        return r;
    if (ce && (r = copy(c, ce, c->d.ce, (size_t)c->ntot * sizeof(int))))
        return r;
    if ((r = sync(c)))
        return r;
    if (count > cap || count > c->enc_cap)
        return set_err(c, NB_E_CAPACITY, "encounter count %d exceeds capacity %d", count,
                       std::min(cap, c->enc_cap));
    return NB_OK;
}

// Free what the context owns (graph, side stream, events) and the context.
void release(nb_ctx *c)
{
    drop_graph(c);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    for (int k = 0; k < kSnapSets; ++k) {
        if (c->ev_fork[k])
            (void)hipEventDestroy(c->ev_fork[k]);
        if (c->ev_join[k])
            (void)hipEventDestroy(c->ev_join[k]);
    }
    if (c->h_stats)
        (void)hipHostFree(c->h_stats);
    if (c->h_pairs)
        (void)hipHostFree(c->h_pairs);
    if (c->h_rows)
        (void)hipHostFree(c->h_rows);
    delete c;
}

// Work tables and workspace layout for systems with offsets off and big-body
// counts nbig (NULL: all big) in the context's workspace, and the device copies
// of the tables; the state itself is not set.  Used at creation and again when
// lost bodies are removed.
int setup_layout(nb_ctx *c, int nsys, const int32_t *off, const int32_t *nbig)
{
    Tables t;
    build_tables(c->p, nsys, off, nbig, t);
    Dev d{};
    const size_t need = carve(c->p, nsys, off[nsys], c->enc_cap, t, nullptr, d);
    if (c->ws_bytes < need)
        return set_err(c, NB_E_WORKSPACE, "workspace of %zu bytes, %zu needed", c->ws_bytes, need);
    drop_graph(c);
    c->nsys = nsys;
    c->ntot = off[nsys];
    c->off.assign(off, off + nsys + 1);
    c->nbig.resize(nsys);
    for (int s = 0; s < nsys; ++s)
        c->nbig[s] = nbig ? nbig[s] : off[s + 1] - off[s];
    c->rb_first = t.rb_first;
    c->d = Dev{};
    carve(c->p, nsys, c->ntot, c->enc_cap, t, (char *)c->ws, c->d);
    std::vector<int> ranges(3 * (size_t)nsys);
    for (int s = 0; s < nsys; ++s) {
        ranges[s] = t.nsplit[s];
        ranges[nsys + s] = t.dw_first[s];
        ranges[2 * nsys + s] = t.dw_count[s];
    }
    int r = NB_OK;
    auto up = [&](void *dst, const void *src, size_t n) {
        if (r == NB_OK && n)
            r = copy(c, dst, src, n);
    };
    up(c->d.off, off, (nsys + 1) * sizeof(int));
    up(c->d.nbig, c->nbig.data(), nsys * sizeof(int));
    up(c->d.nsplit, ranges.data(), ranges.size() * sizeof(int));
    up(c->d.rb_first, t.rb_first.data(), nsys * sizeof(int));
    up(c->d.rb_count, t.rb_count.data(), nsys * sizeof(int));
    up(c->d.sys_of, t.sys_of.data(), t.sys_of.size() * sizeof(int));
    up(c->d.rblk, t.rblk.data(), t.rblk.size() * sizeof(RBlk));
    up(c->d.fwork, t.fwork.data(), t.fwork.size() * sizeof(FWork));
    up(c->d.ework, t.ework.data(), t.ework.size() * sizeof(PWork));
    up(c->d.dwork, t.dwork.data(), t.dwork.size() * sizeof(PWork));
    up(c->d.psys, t.psys.data(), t.psys.size() * sizeof(PSys));
    c->p.step_algo = choose_step_algo(c->p, nsys, off);
    if (r == NB_OK && launch_fill_i32(c->d.step_nce, c->d.step_chunk, 0, c->stream) != hipSuccess)
        r = set_err(c, NB_E_HIP, "clearing the step counters failed");
    if (r == NB_OK && c->ntot > 0 && launch_fill_i32(c->d.lost, c->ntot, 0, c->stream) != hipSuccess)
        r = set_err(c, NB_E_HIP, "clearing the lost flags failed");
    // the radial order's tiles; until the first upload sets the order, every
    // body at its own position
    std::vector<int> ident;
    if (c->d.force_rsort) {
        up(c->d.rtf, t.rtf.data(), nsys * sizeof(int));
        ident.resize(c->ntot);
        for (int i = 0; i < c->ntot; ++i)
            ident[i] = i;
        up(c->d.rord, ident.data(), ident.size() * sizeof(int));
    }
    if (c->d.enc_sorted) {
        up(c->d.sys_cell_base, t.cell_base.data(), nsys * sizeof(int));
        up(c->d.sys_cell_cnt, t.cell_cnt.data(), nsys * sizeof(int));
        up(c->d.tiles, t.tiles.data(), t.tiles.size() * sizeof(Tile));
        up(c->d.units, t.units.data(), t.units.size() * sizeof(int2));
        up(c->d.tile_first, t.tile_first.data(), nsys * sizeof(int));
        if (r == NB_OK && launch_fill_i32(c->d.cell_cnt, c->d.ncell, 0, c->stream) != hipSuccess)
            r = set_err(c, NB_E_HIP, "clearing the cell counts failed");
    }
    if (r == NB_OK)
        r = reset_stats(c);
    if (r == NB_OK)
        r = sync(c);
    c->have_state = c->have_drift = c->have_enc = c->snap_valid = c->mom_valid = false;
    c->have_events = false;
    c->snap = 0;
    return r;
}

// The radial order of the symmetric FP32C force (force_algo 4): the bodies of
// every system by distance from the star, ties by index, from the DH positions
// on the device.  Any order gives the same pairs; this one makes tiles of 64
// consecutive positions thin shells, so that most tile pairs are provably far
// apart, and it stays so while orbits stay near-circular.
int radial_order(nb_ctx *c)
{
    if (!c->d.force_rsort || c->ntot == 0)
        return NB_OK;
    const size_t n = (size_t)c->ntot;
    std::vector<double> q(3 * n);
    int r;
    if ((r = copy(c, q.data(), c->d.qx, n * sizeof(double))) ||
        (r = copy(c, q.data() + n, c->d.qy, n * sizeof(double))) ||
        (r = copy(c, q.data() + 2 * n, c->d.qz, n * sizeof(double))) || (r = sync(c)))
        return r;
    std::vector<double> d2(n);
    for (size_t i = 0; i < n; ++i)
        d2[i] = q[i] * q[i] + q[n + i] * q[n + i] + q[2 * n + i] * q[2 * n + i];
    std::vector<int> ord(n);
    for (size_t i = 0; i < n; ++i)
        ord[i] = (int)i;
    for (int s = 0; s < c->nsys; ++s)
        std::sort(ord.begin() + c->off[s], ord.begin() + c->off[s + 1],
                  [&](int a, int b) { return d2[a] < d2[b] || (d2[a] == d2[b] && a < b); });
    if ((r = copy(c, c->d.rord, ord.data(), n * sizeof(int))))
        return r;
    return sync(c);
}

int enter(nb_ctx *c)
{
    if (!c)
        return NB_E_INVALID;
    c->err.clear();
    HIP_OK(c, hipSetDevice(c->device));
    return NB_OK;
}

}  // namespace

extern "C" {

int nb_version(int *major, int *minor)
{
    if (major)
        *major = NB_VERSION_MAJOR;
    if (minor)
        *minor = NB_VERSION_MINOR;
    return NB_OK;
}

const char *nb_strerror(int code)
{
    switch (code) {
    case NB_OK: return "ok";
    case NB_E_INVALID: return "invalid argument";
    case NB_E_NOT_READY: return "state not ready";
    case NB_E_HIP: return "HIP runtime error";
    case NB_E_NONFINITE: return "non-finite or invalid value";
    case NB_E_CAPACITY: return "encounter list capacity exceeded";
    case NB_E_KEPLER: return "Kepler solve failed for at least one body";
    case NB_E_WORKSPACE: return "workspace too small or misaligned";
    default: return "unknown status";
    }
}

void nb_default_params(nb_params *p)
{
    if (!p)
        return;
    std::memset(p, 0, sizeof *p);
    const double k = 0.01720209895 * 365.25;
    p->G = k * k;
    p->n_hill = 3.0;
    p->chg_inner = 0.1;
    p->mode = NB_FP64;
    p->drag = 0;
    const double au_cm = 1.495978707e13, msun_g = 1.98840987e33;
    p->drag_sigma0 = 1000.0 / (msun_g / (au_cm * au_cm));
    p->drag_h = 0.05;
    p->drag_cd = 1.0;
    p->drag_rho_p = 2.0 / (msun_g / (au_cm * au_cm * au_cm));
}

int nb_workspace_size(const nb_params *p, int nsys, const int32_t *off, const int32_t *nbig,
                      int enc_cap, size_t *bytes)
{
    if (!bytes || check_params(p) || check_offsets(nsys, off, nbig) || enc_cap < 0 ||
        (p->drag && has_small(nsys, off, nbig)) ||
        (p->enc_algo == 3 && max_big(nsys, off, nbig) > kBlock))
        return NB_E_INVALID;
    Params q = to_internal(*p);
    bool tuned = false;
    if (apply_tuning(*p, nsys, off, nbig, q, &tuned, nullptr))
        return NB_E_INVALID;
    if (q.enc_algo == 3 && max_big(nsys, off, nbig) > kBlock)
        q.enc_algo = 0;
    fused_tiles(q, nsys, off, nbig);
    Tables t;
    build_tables(q, nsys, off, nbig, t);
    Dev d{};
    *bytes = carve(q, nsys, off[nsys], enc_cap, t, nullptr, d);
    return NB_OK;
}

int nb_create(const nb_params *p, int nsys, const int32_t *off, const int32_t *nbig, int enc_cap,
              void *workspace, size_t bytes, void *stream, nb_ctx **out)
{
    if (!out)
        return NB_E_INVALID;
    *out = nullptr;
    if (check_params(p) || check_offsets(nsys, off, nbig) || enc_cap < 0 ||
        (p->drag && has_small(nsys, off, nbig)) ||
        (p->enc_algo == 3 && max_big(nsys, off, nbig) > kBlock))
        return NB_E_INVALID;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0)
        return NB_E_WORKSPACE;
    nb_ctx *c = new nb_ctx();
    c->p = to_internal(*p);
    {
        std::string why;
        if (apply_tuning(*p, nsys, off, nbig, c->p, &c->tuned, &why)) {
            delete c;
            return NB_E_INVALID;
        }
        if (c->p.enc_algo == 3 && max_big(nsys, off, nbig) > kBlock)
            c->p.enc_algo = 0;
        fused_tiles(c->p, nsys, off, nbig);
    }
    c->enc_cap = enc_cap;
    c->stream = (hipStream_t)stream;
    c->ws = workspace;
    c->ws_bytes = bytes;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return NB_E_HIP;
    }
    int r = setup_layout(c, nsys, off, nbig);
    if (r == NB_E_WORKSPACE) {
        delete c;
        return r;
    }
    if (r == NB_OK && c->stream) {
        // default priority, like every stream here
        if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess)
            r = set_err(c, NB_E_HIP, "nb_create: side stream");
        for (int k = 0; r == NB_OK && k < kSnapSets; ++k)
            if (hipEventCreateWithFlags(&c->ev_fork[k], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_join[k], hipEventDisableTiming) != hipSuccess)
                r = set_err(c, NB_E_HIP, "nb_create: side stream events");
    }
    if (r != NB_OK) {
        release(c);
        return r;
    }
    *out = c;
    return NB_OK;
}

const char *nb_last_error(const nb_ctx *c) { return c ? c->err.c_str() : ""; }

int nb_upload(nb_ctx *c, const double *m0, const double *m, const double *x, const double *v,
              int frame, int where)
{
    int r = enter(c);
    if (r)
        return r;
    if (!m0 || !m || !x || !v || (frame != NB_HELIO && frame != NB_DH) ||
        (where != NB_HOST && where != NB_DEVICE))
        return set_err(c, NB_E_INVALID, "nb_upload: bad argument");
    const size_t nd = (size_t)c->ntot * sizeof(double);
    drop_graph(c);
    const double *xs = x, *vs = v;
    if ((r = copy(c, c->d.m, m, nd)) || (r = copy(c, c->d.m0, m0, c->nsys * sizeof(double))))
        return r;
    if (where == NB_HOST) {
        if ((r = copy(c, c->d.stage, x, 3 * nd)) || (r = copy(c, c->d.stage + 3 * (size_t)c->ntot, v, 3 * nd)))
            return r;
        xs = c->d.stage;
        vs = c->d.stage + 3 * (size_t)c->ntot;
    }
    HIP_OK(c, launch_fill_i32(c->d.flag, 1, 0, c->stream));
    HIP_OK(c, launch_validate(c->d, c->d.m0, c->d.m, xs, vs, c->stream));
    int bad = 0;
    if ((r = read_int(c, c->d.flag, &bad)))
        return r;
    if (bad & 1) {
        c->have_state = false;
        return set_err(c, NB_E_NONFINITE, "nb_upload: non-finite value, negative mass or m0 <= 0");
    }
    if (bad & 2) {
        c->have_state = false;
        return set_err(c, NB_E_INVALID, "nb_upload: a small body has a nonzero mass");
    }
    HIP_OK(c, launch_to_dh(c->d, xs, vs, frame, c->stream));
    if ((r = radial_order(c)))
        return r;
    if ((r = enqueue_force(c)))
        return r;
    if ((r = sync(c)))
        return r;
    c->have_state = true;
    c->have_drift = false;
    c->snap_valid = false;
    c->mom_valid = false;
    c->have_enc = false;
    c->have_events = false;
    return NB_OK;
}

int nb_download(nb_ctx *c, double *x, double *v, int frame, int where)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_state)
        return set_err(c, NB_E_NOT_READY, "nb_download: no state");
    if (!x || !v || (frame != NB_HELIO && frame != NB_DH) || (where != NB_HOST && where != NB_DEVICE))
        return set_err(c, NB_E_INVALID, "nb_download: bad argument");
    const size_t n3 = 3 * (size_t)c->ntot;
    double *xd = where == NB_DEVICE ? x : c->d.stage;
    double *vd = where == NB_DEVICE ? v : c->d.stage + n3;
    HIP_OK(c, launch_from_dh(c->d, xd, vd, frame == NB_HELIO ? 0 : 1, c->stream));
    if (where == NB_HOST) {
        if ((r = copy(c, x, xd, n3 * sizeof(double))) || (r = copy(c, v, vd, n3 * sizeof(double))))
            return r;
    }
    return sync(c);
}

int nb_force(nb_ctx *c)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_state)
        return set_err(c, NB_E_NOT_READY, "nb_force: no state");
    c->have_drift = false;
    return enqueue_force(c);
}

int nb_kick(nb_ctx *c, double h)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_state)
        return set_err(c, NB_E_NOT_READY, "nb_kick: no state");
    if (!std::isfinite(h))
        return set_err(c, NB_E_INVALID, "nb_kick: h not finite");
    c->have_drift = false;
    c->mom_valid = false;
    HIP_OK(c, launch_kick(c->d, c->p, h, c->stream));
    return NB_OK;
}

int nb_sun_drift(nb_ctx *c, double h)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_state)
        return set_err(c, NB_E_NOT_READY, "nb_sun_drift: no state");
    if (!std::isfinite(h))
        return set_err(c, NB_E_INVALID, "nb_sun_drift: h not finite");
    c->have_drift = false;
    HIP_OK(c, launch_momentum(c->d, c->d.rpart, c->stream));
    HIP_OK(c, launch_sun_drift(c->d, h, 0, c->p, c->d.rpart, nullptr, c->stream));
    return NB_OK;
}

int nb_drift(nb_ctx *c, double dt, int *nfail)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_state)
        return set_err(c, NB_E_NOT_READY, "nb_drift: no state");
    if (!std::isfinite(dt))
        return set_err(c, NB_E_INVALID, "nb_drift: dt not finite");
    HIP_OK(c, launch_fill_i32(&c->d.stats->cur_kfail, 1, 0, c->stream));
    HIP_OK(c, launch_drift(c->d, c->p, dt, 0.0, c->d.rpart, c->stream));
    c->snap = 0;
    int nf = 0;
    if ((r = read_int(c, &c->d.stats->cur_kfail, &nf)))
        return r;
    if (nfail)
        *nfail = nf;
    c->have_drift = true;
    c->snap_valid = true;
    c->mom_valid = false;
    c->last_dt = dt;
    if (nf > 0)
        return set_err(c, NB_E_KEPLER, "nb_drift: %d bodies failed to converge", nf);
    return NB_OK;
}

int nb_encounters(nb_ctx *c, int cap, int *nce, int32_t *ice, int32_t *jce, int32_t *ce, int where)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_drift)
        return set_err(c, NB_E_NOT_READY, "nb_encounters: no drift since the last upload");
    if (cap < 0 || (where != NB_HOST && where != NB_DEVICE))
        return set_err(c, NB_E_INVALID, "nb_encounters: bad argument");
    HIP_OK(c, launch_fill_i32(c->d.ce, c->ntot, 0, c->stream));
    HIP_OK(c, launch_fill_i32(&c->d.stats->cur_nce, 1, 0, c->stream));
    HIP_OK(c, launch_encounters(c->d.with_snap(c->snap), c->last_dt, c->stream));
    c->have_enc = true;
    return copy_list(c, cap, nce, ice, jce, ce, where);
}

int nb_get_encounters(nb_ctx *c, int cap, int *nce, int32_t *ice, int32_t *jce, int32_t *ce,
                      int where)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_enc)
        return set_err(c, NB_E_NOT_READY, "nb_get_encounters: no encounter check yet");
    if (cap < 0 || (where != NB_HOST && where != NB_DEVICE))
        return set_err(c, NB_E_INVALID, "nb_get_encounters: bad argument");
    return copy_list(c, cap, nce, ice, jce, ce, where);
}

int nb_step(nb_ctx *c, double dt, int nsteps, nb_stats *st)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_state)
        return set_err(c, NB_E_NOT_READY, "nb_step: no state");
    if (!std::isfinite(dt) || nsteps < 0)
        return set_err(c, NB_E_INVALID, "nb_step: bad argument");
    if ((r = reset_stats(c)))
        return r;
    c->res_groups = c->res_bodies = 0;
    c->res_max_group = c->res_fail = 0;
    if ((r = enqueue_steps(c, dt, nsteps)))
        return r;
    DevStats ds;
    HIP_OK(c, hipMemcpyAsync(&ds, c->d.stats, sizeof ds, hipMemcpyDeviceToHost, c->stream));
    if ((r = sync(c)))
        return r;
    if (st) {
        st->total_nce = ds.total_nce;
        st->max_nce = ds.max_nce;
        st->overflow_steps = ds.overflow_steps;
        st->kepler_fail = ds.kepler_fail;
        st->near_pairs = ds.near_pairs;
        st->resolved_groups = c->res_groups;
        st->resolved_bodies = c->res_bodies;
        st->max_group = c->res_max_group;
        st->bs_fail = c->res_fail;
    }
    if (nsteps > 0) {
        // the snapshot and the state no longer form a drift pair
        c->have_drift = false;
        c->have_enc = true;
        c->last_dt = dt;
    }
    if (ds.kepler_fail > 0)
        return set_err(c, NB_E_KEPLER, "nb_step: %lld failed Kepler solves", ds.kepler_fail);
    if (ds.overflow_steps > 0)
        return set_err(c, NB_E_CAPACITY, "nb_step: %d steps overflowed the encounter list",
                       ds.overflow_steps);
    return NB_OK;
}

int nb_prepare(nb_ctx *c, double dt, int nsteps)
{
    int r = enter(c);
    if (r)
        return r;
    if (!std::isfinite(dt) || nsteps < 0)
        return set_err(c, NB_E_INVALID, "nb_prepare: bad argument");
    // only captured runs are prepared: not without a stream, with the host
    // resolver or with the persistent launch
    if (!c->stream || c->p.resolve || c->p.step_algo == 2 || nsteps == 0)
        return NB_OK;
    int full, rest;
    hipGraphExec_t gx;
    graph_lengths(nsteps, &full, &rest);
    if (full > 0 && (r = graph_for(c, dt, kMaxGraphSteps, &gx)))
        return r;
    if (rest > 0 && (r = graph_for(c, dt, rest, &gx)))
        return r;
    return NB_OK;
}

int nb_diagnostics(nb_ctx *c, double *E, double *EK, double *L, double *P)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_state)
        return set_err(c, NB_E_NOT_READY, "nb_diagnostics: no state");
    HIP_OK(c, launch_diagnostics(c->d, c->p, c->stream));
    std::vector<double> out((size_t)c->nsys * 8);
    HIP_OK(c, hipMemcpyAsync(out.data(), c->d.diag, out.size() * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    if ((r = sync(c)))
        return r;
    bool finite = true;
    for (int s = 0; s < c->nsys; ++s) {
        const double *o = &out[(size_t)s * 8];
        for (int k = 0; k < 8; ++k)
            finite &= std::isfinite(o[k]);
        if (E)
            E[s] = o[0];
        if (EK)
            EK[s] = o[1];
        for (int k = 0; k < 3; ++k) {
            if (L)
                L[3 * s + k] = o[2 + k];
            if (P)
                P[3 * s + k] = o[5 + k];
        }
    }
    if (!finite)
        return set_err(c, NB_E_NONFINITE, "nb_diagnostics: non-finite value");
    return NB_OK;
}

int nb_get_accel(nb_ctx *c, double *a, int where)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_state)
        return set_err(c, NB_E_NOT_READY, "nb_get_accel: no state");
    if (!a || (where != NB_HOST && where != NB_DEVICE))
        return set_err(c, NB_E_INVALID, "nb_get_accel: bad argument");
    const size_t nd = (size_t)c->ntot * sizeof(double);
    if ((r = copy(c, a, c->d.ax, nd)) || (r = copy(c, a + c->ntot, c->d.ay, nd)) ||
        (r = copy(c, a + 2 * (size_t)c->ntot, c->d.az, nd)))
        return r;
    return sync(c);
}

int nb_get_rcrit(nb_ctx *c, double *rc, int where)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_state)
        return set_err(c, NB_E_NOT_READY, "nb_get_rcrit: no state");
    if (!rc || (where != NB_HOST && where != NB_DEVICE))
        return set_err(c, NB_E_INVALID, "nb_get_rcrit: bad argument");
    if ((r = copy(c, rc, c->d.rc, (size_t)c->ntot * sizeof(double))))
        return r;
    return sync(c);
}

int nb_time_kernel(nb_ctx *c, int which, int reps, double dt, double *ms)
{
    int r = enter(c);
    if (r)
        return r;
    if (!c->have_state)
        return set_err(c, NB_E_NOT_READY, "nb_time_kernel: no state");
    if (!ms || reps <= 0 || which < NB_K_FORCE || which > NB_K_FORCE_FUSED || !std::isfinite(dt))
        return set_err(c, NB_E_INVALID, "nb_time_kernel: bad argument");
    if (which == NB_K_FORCE_FUSED && !(c->d.enc_fused && c->snap_valid && c->have_enc))
        return set_err(c, NB_E_NOT_READY,
                       "nb_time_kernel: the fused force pass needs enc_algo 4 and a per-phase "
                       "step before it");
    if (which == NB_K_ENCOUNTER && !c->snap_valid)
        return set_err(c, NB_E_NOT_READY,
                       "nb_time_kernel: no drift outputs for the encounter check (no drift or "
                       "per-phase step since the upload, or the last steps ran persistent)");
    auto once = [&]() -> int {
        switch (which) {
        case NB_K_FORCE:
            HIP_OK(c, launch_force(c->d, c->p, c->stream));
            return NB_OK;
        case NB_K_ENCOUNTER:
            // each check starts from an empty list, as after a drift
            HIP_OK(c, launch_fill_i32(&c->d.stats->cur_nce, 1, 0, c->stream));
            HIP_OK(c, launch_encounters(c->d.with_snap(c->snap), c->last_dt, c->stream));
            return NB_OK;
        case NB_K_DRIFT:
            HIP_OK(c, launch_drift(c->d, c->p, dt, 0.0, c->d.rpart, c->stream));
            c->snap = 0;
            c->snap_valid = true;
            return NB_OK;
        case NB_K_FORCE_EVAL:
            return enqueue_force(c);
        case NB_K_FORCE_FUSED:
            // the force pass alone (its appends run past the list's count)
            HIP_OK(c, launch_force_fused(c->d, c->p, c->last_dt, 0, c->stream));
            return NB_OK;
        default:
            // the runs the timed call replays, captured here, outside the timed
            // region (one untimed step)
            if (c->stream && !c->p.resolve && c->p.step_algo != 2) {
                int full, rest, r2;
                hipGraphExec_t gx;
                graph_lengths(reps, &full, &rest);
                if (full > 0 && (r2 = graph_for(c, dt, kMaxGraphSteps, &gx)))
                    return r2;
                if (rest > 0 && (r2 = graph_for(c, dt, rest, &gx)))
                    return r2;
            }
            return enqueue_steps(c, dt, 1);
        }
    };
    if ((r = once()))
        return r;
    hipEvent_t e0, e1;
    HIP_OK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_err(c, NB_E_HIP, "hipEventCreate failed");
    }
    hipError_t he = hipEventRecord(e0, c->stream);
    if (which == NB_K_STEP)
        r = enqueue_steps(c, dt, reps);     // the way nb_step runs them
    else
        for (int k = 0; k < reps && r == NB_OK && he == hipSuccess; ++k)
            r = once();
    if (he == hipSuccess)
        he = hipEventRecord(e1, c->stream);
    if (he == hipSuccess)
        he = hipEventSynchronize(e1);
    float t = 0.0f;
    if (he == hipSuccess)
        he = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r)
        return r;
    if (he != hipSuccess)
        return set_err(c, NB_E_HIP, "timing events: %s", hipGetErrorString(he));
    *ms = (double)t / reps;
    if (which == NB_K_FORCE_FUSED) {
        // the last step's list again, from an empty one
        HIP_OK(c, launch_enc_prepare(c->d, c->last_dt, c->stream));
        HIP_OK(c, launch_force_fused(c->d, c->p, c->last_dt, 1, c->stream));
        if ((r = sync(c)))
            return r;
    }
    if (which == NB_K_DRIFT) {
        c->mom_valid = false;
        c->have_drift = true;
        c->last_dt = dt;
    }
    if (which == NB_K_STEP) {
        // as after nb_step: the list of the last step can be read, and the
        // encounter check can be timed on its drift outputs (per-phase steps)
        c->have_drift = false;
        c->have_enc = true;
        c->last_dt = dt;
    }
    return NB_OK;
}

int nb_resolve_host(int n, double G, double m0, double chg_inner, double tol, double tau,
                    const double *m, const double *rc, const double *Q0, const double *V0,
                    int nce, const int32_t *ice, const int32_t *jce, double *Q, double *V,
                    int32_t *group, int nthreads, nb_resolve_info *info)
{
    if (n < 0 || nce < 0 || nthreads < 0 || !(G > 0.0) || !(m0 > 0.0) ||
        !(chg_inner >= 0.0 && chg_inner < 1.0) || !(tol >= 0.0 && tol < 1.0) ||
        !std::isfinite(tau))
        return NB_E_INVALID;
    if (n > 0 && (!m || !rc || !Q0 || !V0 || !Q || !V))
        return NB_E_INVALID;
    if (nce > 0 && (!ice || !jce))
        return NB_E_INVALID;
    for (int k = 0; k < nce; ++k)
        if (ice[k] < 0 || ice[k] >= n || jce[k] < 0 || jce[k] >= n || ice[k] == jce[k])
            return NB_E_INVALID;
    Groups g;
    build_groups(nce, ice, jce, g);
    const int k = (int)g.body.size();
    std::vector<Member> in(k);
    for (int e = 0; e < k; ++e) {
        const int i = g.body[e];
        Member &mb = in[e];
        mb.m0 = m0;
        mb.m = m[i];
        mb.rc = rc[i];
        for (int c = 0; c < 3; ++c) {
            mb.q[c] = Q0[3 * i + c];
            mb.v[c] = V0[3 * i + c];
        }
        mb.pad = 0.0;
    }
    std::vector<double> out((size_t)6 * k);
    std::unique_ptr<WorkerPool> pool;
    const int nt = resolver_threads(nthreads);
    if (nt > 1 && g.count() > 1)
        pool.reset(new WorkerPool(std::min(nt, g.count())));
    ResolveTotals t = resolve_groups(g, in.data(), out.data(), G, chg_inner, tau,
                                     tol > 0.0 ? tol : 1e-12, pool.get());
    for (int e = 0; e < k; ++e) {
        const double *o = out.data() + 6 * (size_t)e;
        bool ok = true;
        for (int c = 0; c < 6; ++c)
            ok = ok && std::isfinite(o[c]);
        if (!ok)
            continue;
        const int i = g.body[e];
        for (int c = 0; c < 3; ++c) {
            Q[3 * i + c] = o[c];
            V[3 * i + c] = o[3 + c];
        }
    }
    if (group) {
        for (int i = 0; i < n; ++i)
            group[i] = -1;
        for (int gi = 0; gi < g.count(); ++gi)
            for (int e = g.start[gi]; e < g.start[gi + 1]; ++e)
                group[g.body[e]] = g.body[g.start[gi]];
    }
    if (info) {
        info->groups = t.groups;
        info->bodies = t.bodies;
        info->max_group = t.max_group;
        info->failed = t.failed;
        info->max_steps = t.max_steps;
    }
    return NB_OK;
}

int nb_events(nb_ctx *c, const nb_event_params *ep, nb_event_counts *counts, int32_t *lost,
              int where)
{
    int r = enter(c);
    if (r)
        return r;
    if (!ep || !(ep->rho > 0.0) || !std::isfinite(ep->rho) || !(ep->r_star >= 0.0) ||
        !(ep->r_eject >= 0.0) || !std::isfinite(ep->r_star) || !std::isfinite(ep->r_eject) ||
        (where != NB_HOST && where != NB_DEVICE))
        return set_err(c, NB_E_INVALID, "nb_events: bad argument");
    if (!c->have_state || !c->snap_valid || !c->have_enc)
        return set_err(c, NB_E_NOT_READY,
                       "nb_events: needs the drift arcs and the encounter list of the last step");
    // the pairs in (i, j) order: the groups do not depend on the append order
    HIP_OK(c, launch_enc_sort(c->d, 0, c->stream));
    HIP_OK(c, launch_events(c->d.with_snap(c->snap), c->p, c->last_dt, ep->rho, ep->r_star,
                            ep->r_eject, c->stream));
    int cnt[4] = {0, 0, 0, 0};
    DevStats st;
    HIP_OK(c, hipMemcpyAsync(cnt, c->d.evcnt, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipMemcpyAsync(&st, c->d.stats, sizeof st, hipMemcpyDeviceToHost, c->stream));
    if (lost && (r = copy(c, lost, c->d.lost, (size_t)c->ntot * sizeof(int))))
        return r;
    if ((r = sync(c)))
        return r;
    if (counts) {
        counts->star = cnt[0];
        counts->collide = cnt[1];
        counts->merged = cnt[2];
        counts->ejected = cnt[3];
    }
    c->have_events = true;
    if (cnt[0] + cnt[2] + cnt[3] > 0) {
        // masses, star masses, positions or velocities changed: new critical
        // radii and force (first-same-as-last), momentum summed again
        if ((r = enqueue_force(c)) || (r = sync(c)))
            return r;
        c->have_drift = c->have_enc = c->snap_valid = c->mom_valid = false;
    }
    if (st.cur_nce > c->enc_cap)
        return set_err(c, NB_E_CAPACITY, "nb_events: %d listed pairs, only %d kept", st.cur_nce,
                       c->enc_cap);
    return NB_OK;
}

int nb_compact(nb_ctx *c, int32_t *off_out, int32_t *nbig_out, int32_t *index, int where)
{
    int r = enter(c);
    if (r)
        return r;
    if (where != NB_HOST && where != NB_DEVICE)
        return set_err(c, NB_E_INVALID, "nb_compact: bad argument");
    if (!c->have_state || !c->have_events)
        return set_err(c, NB_E_NOT_READY, "nb_compact: no nb_events on the current state");
    const int n = c->ntot, nsys = c->nsys;
    if ((r = sync(c)))
        return r;
    double *out = c->d.stage;
    HIP_OK(c, launch_compact(c->d, out, c->d.evidx, c->stream));
    std::vector<int> pos(c->d.nrb + 1, 0);
    if ((r = copy(c, pos.data(), c->d.cmp_pos, pos.size() * sizeof(int))))
        return r;
    if ((r = sync(c)))
        return r;
    const int kept = n > 0 ? pos[c->d.nrb] : 0;
    std::vector<int32_t> noff(nsys + 1, 0), nbig(nsys, 0), idx(kept);
    std::vector<double> st7((size_t)7 * kept), m0(nsys);
    // a system's first block (for a system without bodies: the next system's)
    for (int s = 0; s < nsys; ++s)
        noff[s] = n > 0 ? pos[c->rb_first[s]] : 0;
    noff[nsys] = kept;
    for (int k = 0; k < 7; ++k)
        if (kept && (r = copy(c, st7.data() + (size_t)k * kept, out + (size_t)k * n,
                              (size_t)kept * sizeof(double))))
            return r;
    if (kept && (r = copy(c, idx.data(), c->d.evidx, (size_t)kept * sizeof(int))))
        return r;
    if ((r = copy(c, m0.data(), c->d.m0, (size_t)nsys * sizeof(double))) || (r = sync(c)))
        return r;
    // big bodies stay first in every system: the kept ones among the first nbig
    for (int s = 0; s < nsys; ++s)
        for (int k = noff[s]; k < noff[s + 1]; ++k)
            nbig[s] += idx[k] < c->off[s] + c->nbig[s];
    if (kept < n) {
        if ((r = setup_layout(c, nsys, noff.data(), nbig.data())))
            return r;
        // the kept state again (DH), with new critical radii and force
        if ((r = nb_upload(c, m0.data(), st7.data(), st7.data() + (size_t)kept,
                           st7.data() + (size_t)4 * kept, NB_DH, NB_HOST)))
            return r;
    }
    c->have_events = false;
    if (off_out && (r = copy(c, off_out, noff.data(), (nsys + 1) * sizeof(int32_t))))
        return r;
    if (nbig_out && (r = copy(c, nbig_out, nbig.data(), nsys * sizeof(int32_t))))
        return r;
    if (index && (r = copy(c, index, idx.data(), (size_t)kept * sizeof(int32_t))))
        return r;
    return sync(c);
}

int nb_get_choices(const nb_ctx *c, int32_t *force_algo, int32_t *enc_algo, int32_t *step_algo)
{
    if (!c)
        return NB_E_INVALID;
    if (force_algo)
        *force_algo = c->d.force_rsort ? 4 : (c->d.force_sym ? 2 : (c->d.force_few ? 3 : 1));
    if (enc_algo)
        *enc_algo = c->d.enc_fused ? 4 : (c->d.enc_sorted ? 2 : (c->d.enc_few ? 3 : 1));
    if (step_algo)
        *step_algo = c->p.step_algo;
    return NB_OK;
}

int nb_get_params(const nb_ctx *c, nb_params *out, int32_t *tuned)
{
    if (!c || !out)
        return NB_E_INVALID;
    std::memset(out, 0, sizeof *out);
    const Params &p = c->p;
    out->G = p.G;
    out->n_hill = p.n_hill;
    out->chg_inner = p.inner;
    out->mode = p.mode;
    out->drag = p.drag;
    out->drag_sigma0 = p.sigma0;
    out->drag_h = p.h;
    out->drag_cd = p.cd;
    out->drag_rho_p = p.rho_p;
    out->force_jchunk = p.force_j;
    out->force_r = p.force_r;
    out->enc_jchunk = p.enc_j;
    out->enc_algo = p.enc_algo;
    out->step_algo = p.step_algo;
    out->resolve = p.resolve;
    out->resolve_threads = p.resolve_threads;
    out->force_algo = p.force_algo;
    out->force_g = c->d.force_sym ? c->d.sym_g : p.force_g;
    out->bs_tol = p.bs_tol;
    out->autotune_path = nullptr;
    if (tuned)
        *tuned = c->tuned ? 1 : 0;
    return NB_OK;
}

int nb_destroy(nb_ctx *c)
{
    if (!c)
        return NB_E_INVALID;
    (void)hipSetDevice(c->device);
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    else
        (void)hipDeviceSynchronize();
    release(c);
    return NB_OK;
}

}  // extern "C"
