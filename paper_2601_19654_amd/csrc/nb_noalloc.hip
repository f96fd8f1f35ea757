// Force evaluation of one system without a context and without any device
// allocation: every table and partial sum the force kernels need lives in one
// file-scope device array of fixed size (each GPU the library runs on holds its
// own copy until the process ends).  For callers that cannot allocate device
// memory (HIP graph capture, tight serving loops).
#include "nb.h"
#include "nb_internal.h"

#include <cmath>
#include <cstdint>
#include <mutex>

using namespace nb;

namespace {

constexpr size_t kScratchBytes = (size_t)NB_NOALLOC_SCRATCH_MB << 20;
constexpr int kMaxDevices = 64;

// The scratch array.  In host code its name is only a stand-in for the symbol:
// the device address comes from hipGetSymbolAddress (scratch_of below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lock;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the scratch array (looked up once
// per device, with that device current).
hipError_t scratch_of(int dev, void **out)
{
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

size_t al(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

int nb_force_noalloc(const nb_params *p, int n, double m0, const double *m, const double *x,
                     double *a, void *stream)
{
    if (n > NB_NOALLOC_MAX_N)
        return NB_E_WORKSPACE;
    if (!p || n < 0 || !(std::isfinite(m0) && m0 > 0.0) ||
        (p->mode != NB_FP64 && p->mode != NB_FP32C) || (p->force_algo != 0 && p->force_algo != 2) ||
        (p->force_r != 0 && p->force_r != 1 && p->force_r != 2 && p->force_r != 4) ||
        (p->force_g != 0 && p->force_g != 1 && p->force_g != 2 && p->force_g != 4) ||
        !(std::isfinite(p->G) && std::isfinite(p->n_hill) && std::isfinite(p->chg_inner)))
        return NB_E_INVALID;
    if (n == 0)
        return NB_OK;
    if (!m || !x || !a)
        return NB_E_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return NB_E_HIP;
    void *base = nullptr;
    if (scratch_of(dev, &base) != hipSuccess || !base)
        return NB_E_HIP;

    Params q{};
    q.G = p->G;
    q.n_hill = p->n_hill;
    q.inner = p->chg_inner;
    q.mode = p->mode;
    q.force_r = p->force_r ? p->force_r : 2;
    q.force_algo = 2;
    // super-tile width: asked for, or chosen as nb_create chooses it
    const int T = 64 * q.force_r;
    int g = p->force_g;
    if (!g) {
        g = 1;
        for (int w = 4; w > 1 && g == 1; w /= 2) {
            const long long nt = (n + (long long)w * T - 1) / ((long long)w * T);
            if (nt * (nt + 1) / 2 >= kSymMinItems(w))
                g = w;
        }
    }
    const int ST = g * T;
    const int nt = (n + ST - 1) / ST;
    const int nrb = (n + kBlock - 1) / kBlock;
    const long long nitems = (long long)nt * (nt + 1) / 2;

    // layout of the scratch array
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t o = at;
        at = al(at + bytes);
        return o;
    };
    const size_t o_m0 = take(sizeof(double));
    const size_t o_rblk = take((size_t)nrb * sizeof(RBlk));
    const size_t o_trc = take((size_t)nrb * sizeof(double));
    const size_t o_rc = take((size_t)n * sizeof(double));
    const size_t o_pk = take(p->mode == NB_FP32C ? (size_t)n * 2 * sizeof(float4) : 0);
    const size_t o_fw = take((size_t)nitems * sizeof(FWork));
    const size_t o_st = take(sizeof(DevStats));
    const size_t o_fp = take((size_t)3 * nt * n * (p->mode == NB_FP32C ? sizeof(float) : sizeof(double)));
    if (at > kScratchBytes)
        return NB_E_WORKSPACE;

    char *b = (char *)base;
    Dev d{};
    d.ntot = n;
    d.nsys = 1;
    d.m = const_cast<double *>(m);
    d.qx = const_cast<double *>(x);
    d.qy = const_cast<double *>(x) + n;
    d.qz = const_cast<double *>(x) + 2 * (size_t)n;
    d.ax = a;
    d.ay = a + n;
    d.az = a + 2 * (size_t)n;
    d.m0 = (double *)(b + o_m0);
    d.rblk = (RBlk *)(b + o_rblk);
    d.nrb = nrb;
    d.tile_rc2 = (double *)(b + o_trc);
    d.rc = (double *)(b + o_rc);
    d.pk = p->mode == NB_FP32C ? (float4 *)(b + o_pk) : nullptr;
    d.fwork = (FWork *)(b + o_fw);
    d.nfw = (int)nitems;
    d.maxs = nt;
    d.ns_all = nt;
    d.stats = (DevStats *)(b + o_st);
    if (p->mode == NB_FP32C)
        d.fpart32 = (float *)(b + o_fp);
    else
        d.fpart = (double *)(b + o_fp);
    d.force_sym = 1;
    d.sym_g = g;

    hipStream_t s = (hipStream_t)stream;
    // tables, critical radii (and FP32C source records) at x, the force kernel,
    // the sum of its partials times G into a: the kernels of nb_force
    if (launch_single_tables(d, ST, nt, m0, s) != hipSuccess ||
        launch_sun_drift(d, 0.0, 1, q, nullptr, nullptr, s) != hipSuccess ||
        launch_force(d, q, s) != hipSuccess || launch_force_finalize(d, q, 0.0, 1, s) != hipSuccess)
        return NB_E_HIP;
    return NB_OK;
}
