// Host runtime of the C ABI declared in include/nb.h: work-table construction,
// workspace carving, validation, state transfer, step sequencing and HIP-graph
// capture.  The library never allocates device memory; every array lives in
// the caller's workspace.
#include "nb.h"
#include "nb_internal.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace nb;

struct nb_ctx {
    Params p;
    int nsys = 0, ntot = 0, enc_cap = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    Dev d{};
    std::vector<int> off;
    bool have_state = false, have_drift = false, have_enc = false;
    double last_dt = 0.0;
    hipGraphExec_t gexec = nullptr;
    double graph_dt = 0.0;
    int graph_steps = 0;
    std::string err;
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
    return p;
}

// Encounter algorithm: explicit choice, else sorted tiles for large totals.
int choose_enc_algo(const Params &p, int ntot)
{
    if (p.enc_algo == 1 || p.enc_algo == 2)
        return p.enc_algo;
    return ntot >= 8192 ? 2 : 1;
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
    if (p->force_jchunk < 0 || p->enc_jchunk < 0 || p->enc_algo < 0 || p->enc_algo > 2)
        return NB_E_INVALID;
    if (p->drag && !(p->drag_h > 0.0 && p->drag_h * p->drag_h * 3.0 < 1.0 && p->drag_rho_p > 0.0 &&
                     p->drag_sigma0 >= 0.0 && p->drag_cd >= 0.0))
        return NB_E_INVALID;
    return NB_OK;
}

int check_offsets(int nsys, const int32_t *off)
{
    if (nsys <= 0 || !off || off[0] != 0)
        return NB_E_INVALID;
    for (int s = 0; s < nsys; ++s)
        if (off[s + 1] < off[s])
            return NB_E_INVALID;
    if (off[nsys] <= 0)
        return NB_E_INVALID;
    return NB_OK;
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
};

// Unordered-pair items of one system: targets in tiles of kBlock, sources in
// chunks of J; an item exists when some source index exceeds some target index.
void pair_items(int a, int n, int J, std::vector<PWork> &out)
{
    for (int i0 = 0; i0 < n; i0 += kBlock) {
        int ni = std::min(kBlock, n - i0);
        for (int j0 = 0; j0 < n; j0 += J) {
            int nj = std::min(J, n - j0);
            if (j0 + nj - 1 > i0)
                out.push_back(PWork{a + i0, ni, a + j0, nj});
        }
    }
}

void build_tables(const Params &p, int nsys, const int32_t *off, Tables &t)
{
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
            t.rblk.push_back(RBlk{s, a + b, a + std::min(n, b + kBlock), 0});
        t.rb_count[s] = (int)t.rblk.size() - t.rb_first[s];
        if (n == 0)
            continue;
        int S = (n + p.force_j - 1) / p.force_j;
        t.nsplit[s] = S;
        t.maxs = std::max(t.maxs, S);
        for (int i0 = 0; i0 < n; i0 += TI)
            for (int k = 0; k < S; ++k) {
                int j0 = k * p.force_j;
                t.fwork.push_back(FWork{a + i0, std::min(TI, n - i0), a + j0,
                                        std::min(p.force_j, n - j0), k, s,
                                        t.rb_first[s] + j0 / kBlock, 0});
            }
        pair_items(a, n, p.enc_j, t.ework);
        t.dw_first[s] = (int)t.dwork.size();
        pair_items(a, n, p.enc_j, t.dwork);
        t.dw_count[s] = (int)t.dwork.size() - t.dw_first[s];
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
        int nt = (n + 63) / 64;
        for (int k = 0; k < nt; ++k)
            t.tiles.push_back(Tile{s, off[s] + 64 * k, std::min(64, n - 64 * k), first + nt - 1});
        t.tp_cap += (long long)nt * (nt + 1) / 2;
    }
    // longest work first, so the hardware dispatcher packs the tail
    std::stable_sort(t.fwork.begin(), t.fwork.end(), [](const FWork &x, const FWork &y) {
        return (long long)x.ni * x.nj > (long long)y.ni * y.nj;
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
    double **planes[] = {&d.m,  &d.qx, &d.qy, &d.qz, &d.vx,  &d.vy,  &d.vz,  &d.ax, &d.ay,
                         &d.az, &d.rc, &d.q0x, &d.q0y, &d.q0z, &d.v0x, &d.v0y, &d.v0z};
    for (double **pl : planes)
        *pl = (double *)take(nd);
    d.pk = (float4 *)take((size_t)ntot * 2 * sizeof(float4));
    d.mr = (double4 *)take((size_t)ntot * sizeof(double4));
    d.kflag = (int *)take((size_t)ntot * sizeof(int));
    d.ce = (int *)take((size_t)ntot * sizeof(int));
    d.sys_of = (int *)take((size_t)ntot * sizeof(int));
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
    d.new_ = (int)t.ework.size();
    d.ework = (PWork *)take(t.ework.size() * sizeof(PWork));
    d.ndw = (int)t.dwork.size();
    d.dwork = (PWork *)take(t.dwork.size() * sizeof(PWork));
    d.rpart = (double *)take((size_t)d.nrb * 8 * sizeof(double));
    d.tile_rc2 = (double *)take((size_t)std::max(d.nrb, 1) * sizeof(double));
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
    d.enc_sorted = choose_enc_algo(p, ntot) == 2;
    if (d.enc_sorted) {
        d.lnr_part = (double *)take((size_t)std::max(d.nrb, 1) * 2 * sizeof(double));
        d.cell_of = (int *)take((size_t)ntot * sizeof(int));
        d.slot_of = (int *)take((size_t)ntot * sizeof(int));
        d.ncell = t.ncell;
        d.cell_cnt = (int *)take((size_t)t.ncell * sizeof(int));
        d.cell_off = (int *)take((size_t)t.ncell * sizeof(int));
        d.sys_cell_base = (int *)take((size_t)nsys * sizeof(int));
        d.sys_cell_cnt = (int *)take((size_t)nsys * sizeof(int));
        d.ord = (int *)take((size_t)ntot * sizeof(int));
        d.srec = (SRec *)take((size_t)ntot * sizeof(SRec));
        d.ntile = (int)t.tiles.size();
        d.tiles = (Tile *)take(t.tiles.size() * sizeof(Tile));
        d.tileb = (TileB *)take(t.tiles.size() * sizeof(TileB));
        d.tp_cap = (int)std::min<long long>(t.tp_cap, 1ll << 30);
        d.tpairs = (int2 *)take((size_t)d.tp_cap * sizeof(int2));
    }
    d.flag = (int *)take(4 * sizeof(int));
    d.stage = (double *)take((size_t)6 * nd);
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
    HIP_OK(c, launch_sun_drift(c->d, 0.0, 1, c->p, c->stream));
    HIP_OK(c, launch_force(c->d, c->p, c->stream));
    HIP_OK(c, launch_force_finalize(c->d, c->p, 0.0, c->stream));
    return NB_OK;
}

// One hybrid step K(h) S(h) D(dt) C S(h) [rc, F] K(h).
int enqueue_step(nb_ctx *c, double dt)
{
    const double h = 0.5 * dt;
    const Dev &d = c->d;
    HIP_OK(c, launch_kick(d, c->p, h, c->stream));
    HIP_OK(c, launch_sun_drift(d, h, 0, c->p, c->stream));
    HIP_OK(c, launch_drift(d, c->p, dt, c->stream));
    HIP_OK(c, launch_encounters(d, dt, c->stream));
    HIP_OK(c, launch_sun_drift(d, h, 1, c->p, c->stream));
    HIP_OK(c, launch_force(d, c->p, c->stream));
    if (c->p.drag) {
        HIP_OK(c, launch_force_finalize(d, c->p, 0.0, c->stream));
        HIP_OK(c, launch_kick(d, c->p, h, c->stream));
    } else {
        HIP_OK(c, launch_force_finalize(d, c->p, h, c->stream));
    }
    return NB_OK;
}

void drop_graph(nb_ctx *c)
{
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    c->graph_steps = 0;
}

int build_graph(nb_ctx *c, double dt, int steps)
{
    drop_graph(c);
    hipGraph_t g = nullptr;
    HIP_OK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = NB_OK;
    for (int k = 0; k < steps && rc == NB_OK; ++k)
        rc = enqueue_step(c, dt);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc != NB_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess)
        return set_err(c, NB_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->gexec = nullptr;
        return set_err(c, NB_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    c->graph_dt = dt;
    c->graph_steps = steps;
    return NB_OK;
}

int copy_list(nb_ctx *c, int cap, int *nce, int32_t *ice, int32_t *jce, int32_t *ce, int where)
{
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

int nb_workspace_size(const nb_params *p, int nsys, const int32_t *off, int enc_cap, size_t *bytes)
{
    if (!bytes || check_params(p) || check_offsets(nsys, off) || enc_cap < 0)
        return NB_E_INVALID;
    Params q = to_internal(*p);
    Tables t;
    build_tables(q, nsys, off, t);
    Dev d{};
    *bytes = carve(q, nsys, off[nsys], enc_cap, t, nullptr, d);
    return NB_OK;
}

int nb_create(const nb_params *p, int nsys, const int32_t *off, int enc_cap, void *workspace,
              size_t bytes, void *stream, nb_ctx **out)
{
    if (!out)
        return NB_E_INVALID;
    *out = nullptr;
    if (check_params(p) || check_offsets(nsys, off) || enc_cap < 0)
        return NB_E_INVALID;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0)
        return NB_E_WORKSPACE;
    nb_ctx *c = new nb_ctx();
    c->p = to_internal(*p);
    c->nsys = nsys;
    c->ntot = off[nsys];
    c->enc_cap = enc_cap;
    c->off.assign(off, off + nsys + 1);
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return NB_E_HIP;
    }
    Tables t;
    build_tables(c->p, nsys, off, t);
    size_t need = carve(c->p, nsys, c->ntot, enc_cap, t, nullptr, c->d);
    if (bytes < need) {
        delete c;
        return NB_E_WORKSPACE;
    }
    carve(c->p, nsys, c->ntot, enc_cap, t, (char *)workspace, c->d);
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
    up(c->d.nsplit, ranges.data(), ranges.size() * sizeof(int));
    up(c->d.rb_first, t.rb_first.data(), nsys * sizeof(int));
    up(c->d.rb_count, t.rb_count.data(), nsys * sizeof(int));
    up(c->d.sys_of, t.sys_of.data(), t.sys_of.size() * sizeof(int));
    up(c->d.rblk, t.rblk.data(), t.rblk.size() * sizeof(RBlk));
    up(c->d.fwork, t.fwork.data(), t.fwork.size() * sizeof(FWork));
    up(c->d.ework, t.ework.data(), t.ework.size() * sizeof(PWork));
    up(c->d.dwork, t.dwork.data(), t.dwork.size() * sizeof(PWork));
    if (c->d.enc_sorted) {
        up(c->d.sys_cell_base, t.cell_base.data(), nsys * sizeof(int));
        up(c->d.sys_cell_cnt, t.cell_cnt.data(), nsys * sizeof(int));
        up(c->d.tiles, t.tiles.data(), t.tiles.size() * sizeof(Tile));
        if (r == NB_OK && launch_fill_i32(c->d.cell_cnt, c->d.ncell, 0, c->stream) != hipSuccess)
            r = set_err(c, NB_E_HIP, "nb_create: clearing the cell counts failed");
    }
    if (r == NB_OK)
        r = reset_stats(c);
    if (r == NB_OK)
        r = sync(c);
    if (r != NB_OK) {
        delete c;
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
    if (bad) {
        c->have_state = false;
        return set_err(c, NB_E_NONFINITE, "nb_upload: non-finite value, negative mass or m0 <= 0");
    }
    HIP_OK(c, launch_to_dh(c->d, xs, vs, frame, c->stream));
    if ((r = enqueue_force(c)))
        return r;
    if ((r = sync(c)))
        return r;
    c->have_state = true;
    c->have_drift = false;
    c->have_enc = false;
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
    HIP_OK(c, launch_momentum(c->d, c->stream));
    HIP_OK(c, launch_sun_drift(c->d, h, 0, c->p, c->stream));
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
    HIP_OK(c, launch_drift(c->d, c->p, dt, c->stream));
    int nf = 0;
    if ((r = read_int(c, &c->d.stats->cur_kfail, &nf)))
        return r;
    if (nfail)
        *nfail = nf;
    c->have_drift = true;
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
    HIP_OK(c, launch_encounters(c->d, c->last_dt, c->stream));
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
    int done = 0;
    if (c->stream && nsteps > 0) {
        int g = std::min(nsteps, kMaxGraphSteps);
        if (!c->gexec || c->graph_dt != dt || c->graph_steps != g)
            if ((r = build_graph(c, dt, g)))
                return r;
        while (nsteps - done >= c->graph_steps) {
            HIP_OK(c, hipGraphLaunch(c->gexec, c->stream));
            done += c->graph_steps;
        }
    }
    for (; done < nsteps; ++done)
        if ((r = enqueue_step(c, dt)))
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
    if (!ms || reps <= 0 || which < NB_K_FORCE || which > NB_K_STEP || !std::isfinite(dt))
        return set_err(c, NB_E_INVALID, "nb_time_kernel: bad argument");
    if (which == NB_K_ENCOUNTER && !c->have_drift && !c->have_enc)
        return set_err(c, NB_E_NOT_READY, "nb_time_kernel: no drift before the encounter check");
    auto once = [&]() -> int {
        switch (which) {
        case NB_K_FORCE:
            HIP_OK(c, launch_force(c->d, c->p, c->stream));
            return NB_OK;
        case NB_K_ENCOUNTER:
            HIP_OK(c, launch_encounters(c->d, c->last_dt, c->stream));
            return NB_OK;
        case NB_K_DRIFT:
            HIP_OK(c, launch_drift(c->d, c->p, dt, c->stream));
            return NB_OK;
        default:
            return enqueue_step(c, dt);
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
    if (which == NB_K_DRIFT || which == NB_K_STEP) {
        c->have_drift = true;
        c->last_dt = dt;
    }
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
    drop_graph(c);
    delete c;
    return NB_OK;
}

}  // extern "C"
