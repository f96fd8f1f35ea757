// Device kernels of the hybrid symplectic hot path for gfx950 (MI355X).
//
// Paper: Mercury-Opal, arXiv 2601.19654.  Sec. 3.1 gives the five per-step
// blocks (force, Hamiltonian, drift, encounter check) and Sec. 3.2 the data
// kept on the device; Sec. 2.1.1 the coordinates (democratic heliocentric) and
// the Hill-radius based critical radius.  The kernels here are a new MI355X
// design, not a translation of the paper's OpenACC loops:
//   * state lives in HBM as FP64 structure-of-arrays planes for the whole run;
//   * pair kernels hold R targets per lane in VGPRs and stream sources through
//     LDS tiles read as wave-wide broadcasts; sources are split into chunks so a
//     single system fills all 256 CUs, and the chunk partials are summed in a
//     fixed order (bit-reproducible runs);
//   * O(N) phases run over blocks that never straddle two systems, with
//     per-system sums formed from per-block partials in a fixed order;
//   * no atomics touch floating-point data; the encounter list uses one
//     integer atomic per wave and is sorted afterwards.
#include "nb_internal.h"

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <float.h>
#include <math.h>
#include <type_traits>

namespace nb {

// ----------------------------------------------------------------------------
// small helpers
// ----------------------------------------------------------------------------

// Error-free sum (Knuth two-sum) accumulated into a (hi, lo) pair.
struct dd {
    double hi, lo;
};
__device__ __forceinline__ void dd_add(dd &a, double b)
{
    double s = a.hi + b;
    double bp = s - a.hi;
    double e = (a.hi - (s - bp)) + (b - bp);
    a.hi = s;
    a.lo += e;
}
__device__ __forceinline__ void dd_add(dd &a, const dd &b)
{
    dd_add(a, b.hi);
    a.lo += b.lo;
}

// 1/sqrt(x) in FP64 to the last bits (diagnostics): the hardware estimate
// refined through (1-e)^(-1/2) ~ 1 + e/2 + 3e^2/8, e = 1 - x y^2, then one
// Newton step.
__device__ __forceinline__ double rsqrt64_acc(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    double t = fma(0.375, e, 0.5);
    y = fma(y * e, t, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// Deterministic block-wide sum of W doubles per thread (kBlock threads, fixed
// order): each wave's 64 values by an xor-shuffle butterfly (both lanes of a
// pair add the same two values, so every lane ends with the same bits), then
// the wave sums in wave order.  Every thread returns the block's sums.
template <int W>
__device__ __forceinline__ void block_sum(double (&v)[W], double *sh)
{
    constexpr int NW = kBlock / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int w = 0; w < W; ++w)
        for (int o = 32; o > 0; o >>= 1)
            v[w] += __shfl_xor(v[w], o);
    if (lane == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w)
            sh[w * NW + wv] = v[w];
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < W; ++w) {
        double t = sh[w * NW];
        for (int q = 1; q < NW; ++q)
            t += sh[w * NW + q];
        v[w] = t;
    }
    __syncthreads();
}

// Sum of the first W columns of the per-block partials of one system, in block order.
template <int W>
__device__ __forceinline__ void system_sum(const double *__restrict__ part, int stride, int first,
                                           int count, double (&out)[W], double *sh)
{
#pragma unroll
    for (int w = 0; w < W; ++w)
        out[w] = 0.0;
    for (int b = threadIdx.x; b < count; b += kBlock)
#pragma unroll
        for (int w = 0; w < W; ++w)
            out[w] += part[(size_t)(first + b) * stride + w];
    block_sum<W>(out, sh);
}

// Changeover weight w = K/r^3 - (dK/dr)/r^2 for a pair at squared distance r2
// with pair critical radius rc (inner edge `inner` rc).  K = 0 below the inner
// edge, 1 beyond rc and y^2/(2y^2-2y+1) in between, y = (r - inner rc)/((1-inner) rc).
__device__ __forceinline__ double changeover_w_inl(double r2, double rc, double inner)
{
    if (!(r2 > 0.0))
        return 0.0;
    double r = sqrt(r2);
    if (r >= rc)
        return 1.0 / (r2 * r);
    double r_in = inner * rc;
    if (r <= r_in)
        return 0.0;
    double width = rc - r_in;
    double y = (r - r_in) / width;
    double q = 2.0 * y * (y - 1.0) + 1.0;
    double K = y * y / q;
    double dK = 2.0 * y * (1.0 - y) / (q * q * width);
    return (K / r - dK) / r2;
}

// Out of line: the pair loops call it only for the rare pairs inside rc.
__device__ __noinline__ double changeover_w(double r2, double rc, double inner)
{
    return changeover_w_inl(r2, rc, inner);
}

// K itself (diagnostics).
__device__ __forceinline__ double changeover_K(double r, double rc, double inner)
{
    if (r >= rc)
        return 1.0;
    double r_in = inner * rc;
    if (r <= r_in)
        return 0.0;
    double y = (r - r_in) / (rc - r_in);
    return y * y / (2.0 * y * (y - 1.0) + 1.0);
}

// ----------------------------------------------------------------------------
// fills, validation, transforms
// ----------------------------------------------------------------------------
__global__ void k_fill_i32(int *p, int n, int value)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = value;
}

// flag bit 1: a non-finite value, a negative mass or m0 <= 0; bit 2: a small
// body (index >= off[s] + nbig[s]) with a nonzero mass.
__global__ void k_validate(int ntot, int nsys, const double *__restrict__ m0,
                           const double *__restrict__ m, const double *__restrict__ x,
                           const double *__restrict__ v, const int *__restrict__ sys_of,
                           const int *__restrict__ off, const int *__restrict__ nbig, int *flag)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (i < ntot) {
        double mi = m[i];
        bad = (!isfinite(mi) || mi < 0.0) ? 1 : 0;
        for (int c = 0; c < 3; ++c)
            bad |= (!isfinite(x[(size_t)c * ntot + i]) || !isfinite(v[(size_t)c * ntot + i])) ? 1 : 0;
        const int s = sys_of[i];
        if (i - off[s] >= nbig[s] && mi != 0.0)
            bad |= 2;
    }
    if (i < nsys)
        bad |= (!(m0[i] > 0.0) || !isfinite(m0[i])) ? 1 : 0;
    if (bad)
        atomicOr(flag, bad);
}

// Per-block partial of sum m v (columns 0-2) and sum m (column 3).
__global__ void k_partial_mv(const RBlk *__restrict__ rblk, const double *__restrict__ m,
                             const double *__restrict__ vx, const double *__restrict__ vy,
                             const double *__restrict__ vz, double *__restrict__ part)
{
    __shared__ double sh[4 * kBlock];
    RBlk b = rblk[blockIdx.x];
    int i = b.start + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < b.end) {
        double mi = m[i];
        v[0] = mi * vx[i];
        v[1] = mi * vy[i];
        v[2] = mi * vz[i];
        v[3] = mi;
    }
    block_sum<4>(v, sh);
    if (threadIdx.x == 0)
        for (int w = 0; w < 4; ++w)
            part[(size_t)blockIdx.x * 4 + w] = v[w];
}

// Heliocentric -> DH: Q = x, V = v - sum m v / (m0 + sum m); or a plain copy.
__global__ void k_to_dh(const RBlk *__restrict__ rblk, const int *__restrict__ rb_first,
                        const int *__restrict__ rb_count, const double *__restrict__ m0,
                        const double *__restrict__ part, int ntot, const double *__restrict__ x,
                        const double *__restrict__ v, int helio, double *qx, double *qy,
                        double *qz, double *vx, double *vy, double *vz)
{
    __shared__ double sh[4 * kBlock];
    RBlk b = rblk[blockIdx.x];
    double c[3] = {0.0, 0.0, 0.0};
    if (helio) {
        double P[4];
        system_sum<4>(part, 4, rb_first[b.sys], rb_count[b.sys], P, sh);
        double M = m0[b.sys] + P[3];
        c[0] = P[0] / M;
        c[1] = P[1] / M;
        c[2] = P[2] / M;
    }
    int i = b.start + threadIdx.x;
    if (i < b.end) {
        qx[i] = x[i];
        qy[i] = x[(size_t)ntot + i];
        qz[i] = x[(size_t)2 * ntot + i];
        vx[i] = v[i] - c[0];
        vy[i] = v[(size_t)ntot + i] - c[1];
        vz[i] = v[(size_t)2 * ntot + i] - c[2];
    }
}

// DH -> heliocentric (v = V + P/m0) or DH copy, into plane-major x, v.
__global__ void k_from_dh(const RBlk *__restrict__ rblk, const int *__restrict__ rb_first,
                          const int *__restrict__ rb_count, const double *__restrict__ m0,
                          const double *__restrict__ part, int ntot, int helio,
                          const double *__restrict__ qx, const double *__restrict__ qy,
                          const double *__restrict__ qz, const double *__restrict__ vx,
                          const double *__restrict__ vy, const double *__restrict__ vz, double *x,
                          double *v)
{
    __shared__ double sh[4 * kBlock];
    RBlk b = rblk[blockIdx.x];
    double c[3] = {0.0, 0.0, 0.0};
    if (helio) {
        double P[3];
        system_sum<3>(part, 4, rb_first[b.sys], rb_count[b.sys], P, sh);
        double mm = m0[b.sys];
        c[0] = P[0] / mm;
        c[1] = P[1] / mm;
        c[2] = P[2] / mm;
    }
    int i = b.start + threadIdx.x;
    if (i < b.end) {
        x[i] = qx[i];
        x[(size_t)ntot + i] = qy[i];
        x[(size_t)2 * ntot + i] = qz[i];
        v[i] = vx[i] + c[0];
        v[(size_t)ntot + i] = vy[i] + c[1];
        v[(size_t)2 * ntot + i] = vz[i] + c[2];
    }
}

// ----------------------------------------------------------------------------
// Kick (Hamiltonian block loop 1), optionally with gas drag, and the partial
// sums of m V after it (the following stellar drift needs them).
// ----------------------------------------------------------------------------
struct DragP {
    double G, sigma0, h, cd, rho_p;
};

// Quadratic gas drag on one body (parity unpinned by the paper: Sec. 2.1 names
// aerodynamic drag, its disk model is elsewhere).  a = -k |u| u, u = v_helio -
// v_gas, k = 3 C_D rho_g / (8 rho_p s), s = (3 m/(4 pi rho_p))^(1/3),
// rho_g = Sigma0/R / (sqrt(2 pi) h R) exp(-z^2/(2 (h R)^2)),
// v_gas = sqrt(1 - 3 h^2) sqrt(G m0 / R) phi_hat, R cylindrical.
__device__ void drag_accel(const DragP &p, double m0, double mi, double x, double y, double z,
                           double ux, double uy, double uz, double &ax, double &ay, double &az)
{
    const double kPi = 3.141592653589793238462643;
    double R2 = x * x + y * y;
    double R = sqrt(R2);
    double H = p.h * R;
    double rho = p.sigma0 / R / (sqrt(2.0 * kPi) * H) * exp(-z * z / (2.0 * H * H));
    double vk = sqrt(p.G * m0 / R) * sqrt(1.0 - 3.0 * p.h * p.h);
    double gx = -vk * y / R, gy = vk * x / R;
    double wx = ux - gx, wy = uy - gy, wz = uz;
    double wm = sqrt(wx * wx + wy * wy + wz * wz);
    double s = cbrt(3.0 * mi / (4.0 * kPi * p.rho_p));
    double k = (mi > 0.0 && p.sigma0 > 0.0) ? 3.0 * p.cd * rho / (8.0 * p.rho_p * s) : 0.0;
    ax = -k * wm * wx;
    ay = -k * wm * wy;
    az = -k * wm * wz;
}

__global__ void k_kick(const RBlk *__restrict__ rblk, double h, const double *__restrict__ m,
                       const double *__restrict__ ax, const double *__restrict__ ay,
                       const double *__restrict__ az, double *vx, double *vy, double *vz,
                       double *__restrict__ part_out,
                       // drag (part_in == nullptr: no drag)
                       const double *__restrict__ part_in, const int *__restrict__ rb_first,
                       const int *__restrict__ rb_count, const double *__restrict__ m0,
                       const double *__restrict__ qx, const double *__restrict__ qy,
                       const double *__restrict__ qz, DragP dp)
{
    __shared__ double sh[4 * kBlock];
    RBlk b = rblk[blockIdx.x];
    double P[3] = {0.0, 0.0, 0.0};
    double mm = 1.0;
    if (part_in) {
        system_sum<3>(part_in, 4, rb_first[b.sys], rb_count[b.sys], P, sh);
        mm = m0[b.sys];
    }
    int i = b.start + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (i < b.end) {
        double mi = m[i];
        double a0 = ax[i], a1 = ay[i], a2 = az[i];
        double u0 = vx[i], u1 = vy[i], u2 = vz[i];
        if (part_in) {
            double d0, d1, d2;
            drag_accel(dp, mm, mi, qx[i], qy[i], qz[i], u0 + P[0] / mm, u1 + P[1] / mm,
                       u2 + P[2] / mm, d0, d1, d2);
            a0 += d0;
            a1 += d1;
            a2 += d2;
        }
        // fused multiply-add, as in k_force_finalize: two kicks there equal two here
        u0 = fma(h, a0, u0);
        u1 = fma(h, a1, u1);
        u2 = fma(h, a2, u2);
        vx[i] = u0;
        vy[i] = u1;
        vz[i] = u2;
        v[0] = mi * u0;
        v[1] = mi * u1;
        v[2] = mi * u2;
    }
    if (part_out) {
        block_sum<3>(v, sh);
        if (threadIdx.x == 0) {
            part_out[(size_t)blockIdx.x * 4 + 0] = v[0];
            part_out[(size_t)blockIdx.x * 4 + 1] = v[1];
            part_out[(size_t)blockIdx.x * 4 + 2] = v[2];
            part_out[(size_t)blockIdx.x * 4 + 3] = 0.0;
        }
    }
}

// ----------------------------------------------------------------------------
// Stellar drift Q += h P/m0 (Hamiltonian block loops 2-3), optionally followed
// by the critical radius rc = n_hill |Q| (m/(3 m0))^(1/3) (Sec. 2.1.1) and the
// FP32 hi/lo source records of the FP32C force.
// ----------------------------------------------------------------------------
// Per-system sums of the first three columns of the per-block partials (one
// workgroup per system, the same order as an inline system_sum), for systems with
// so many blocks that every block summing them again would read the partials
// quadratically often.
__global__ void k_sys_total(const int *__restrict__ rb_first, const int *__restrict__ rb_count,
                            const double *__restrict__ part, double *__restrict__ tot)
{
    __shared__ double sh[3 * kBlock];
    double P[3];
    system_sum<3>(part, 4, rb_first[blockIdx.x], rb_count[blockIdx.x], P, sh);
    if (threadIdx.x < 3)
        tot[(size_t)blockIdx.x * 4 + threadIdx.x] = P[threadIdx.x];
}

__global__ void k_sun_drift(const RBlk *__restrict__ rblk, const int *__restrict__ rb_first,
                            const int *__restrict__ rb_count, const double *__restrict__ m0,
                            const double *__restrict__ part, double h, double *qx, double *qy,
                            double *qz, int rcrit, const double *__restrict__ m, double n_hill,
                            double *__restrict__ rc, float4 *__restrict__ pk,
                            double *__restrict__ tile_rc2, double *__restrict__ copy_to,
                            const double *__restrict__ ptot, const int *__restrict__ rord,
                            float4 *__restrict__ rtb)
{
    // copy_to: this block's entry of `part` is copied there (nothing else reads
    // that array during the launch)
    if (copy_to && threadIdx.x < 4)
        copy_to[(size_t)blockIdx.x * 4 + threadIdx.x] = part[(size_t)blockIdx.x * 4 + threadIdx.x];
    __shared__ double sh[3 * kBlock];
    double rc2 = 0.0;
    RBlk b = rblk[blockIdx.x];
    // rord: the block's positions of the radial order (their bodies from
    // rord), each wave one tile of 64, whose bounds it writes to rtb
    const int pos = b.start + threadIdx.x;
    const bool on = pos < b.end;
    const int i = rord && on ? rord[pos] : pos;
    float tr = INFINITY, tR = 0.0f, tl = 0.0f, tc = 0.0f;
    // the body's position, loaded while the system's momentum is summed
    const double x0 = on ? qx[i] : 0.0, y0 = on ? qy[i] : 0.0, z0 = on ? qz[i] : 0.0;
    const double mi = on && rcrit ? m[i] : 0.0;
    double c[3] = {0.0, 0.0, 0.0};
    double mm = m0[b.sys];
    if (h != 0.0) {
        // the system's momentum: precomputed per system (ptot) or summed here
        double P[3];
        if (ptot) {
            P[0] = ptot[(size_t)b.sys * 4];
            P[1] = ptot[(size_t)b.sys * 4 + 1];
            P[2] = ptot[(size_t)b.sys * 4 + 2];
        } else {
            system_sum<3>(part, 4, rb_first[b.sys], rb_count[b.sys], P, sh);
        }
        c[0] = h * P[0] / mm;
        c[1] = h * P[1] / mm;
        c[2] = h * P[2] / mm;
    }
    if (on) {
        double x = x0 + c[0], y = y0 + c[1], z = z0 + c[2];
        // with h = 0 (critical radii only) Q is left as it is: the positions
        // may then be a caller's read-only input
        if (h != 0.0) {
            qx[i] = x;
            qy[i] = y;
            qz[i] = z;
        }
        if (rcrit) {
            double r = sqrt(x * x + y * y + z * z);
            double rci = n_hill * r * cbrt(mi / (3.0 * mm));
            rc[i] = rci;
            rc2 = rci * rci;
            if (pk) {
                float hx = (float)x, hy = (float)y, hz = (float)z;
                float lx = (float)(x - (double)hx), ly = (float)(y - (double)hy),
                      lz = (float)(z - (double)hz);
                // squared radius widened by 2^-9 so the FP32 zone test is a superset of
                // the FP64 one; never below 2^-80, so that pairs closer than 2^-40 (where
                // the FP32 weight r^-3 would overflow: massless bodies have rc = 0, and
                // 0 * inf is NaN) and coincident bodies take the FP64 path
                float r2 = (float)(rci * rci * (1.0 + 0x1p-9));
                r2 = fmaxf(r2, 0x1p-80f);
                pk[2 * (size_t)i] = make_float4(hx, hy, hz, (float)mi);
                pk[2 * (size_t)i + 1] = make_float4(lx, ly, lz, r2);
                if (rtb) {
                    // |xh| and |xl| in FP64 (products of floats are exact),
                    // widened by 2^-22 before rounding to nearest so that the
                    // floats bound them from the safe side
                    const double rh = sqrt((double)hx * hx + (double)hy * hy + (double)hz * hz);
                    const double rl = sqrt((double)lx * lx + (double)ly * ly + (double)lz * lz);
                    tr = (float)(rh * (1.0 - 0x1p-22));
                    tR = (float)(rh * (1.0 + 0x1p-22));
                    tl = (float)(rl * (1.0 + 0x1p-22));
                    tc = r2;
                }
            }
        }
    }
    if (rtb) {
        for (int o = 32; o > 0; o >>= 1) {
            tr = fminf(tr, __shfl_xor(tr, o));
            tR = fmaxf(tR, __shfl_xor(tR, o));
            tl = fmaxf(tl, __shfl_xor(tl, o));
            tc = fmaxf(tc, __shfl_xor(tc, o));
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0 && b.start + 64 * w < b.end)
            rtb[b.rt0 + w] = make_float4(tr, tR, tl, tc);
    }
    if (rcrit) {
        // largest rc^2 of this block's bodies: the zone threshold of the ordered and
        // few-source force kernels (over the radial order, which only the symmetric
        // kernel uses, the bodies of the block's positions)
        for (int o = 32; o > 0; o >>= 1)
            rc2 = fmax(rc2, __shfl_xor(rc2, o));
        if ((threadIdx.x & 63) == 0)
            sh[threadIdx.x >> 6] = rc2;
        __syncthreads();
        if (threadIdx.x == 0) {
            double r = sh[0];
            for (int w = 1; w < kBlock / 64; ++w)
                r = fmax(r, sh[w]);
            tile_rc2[blockIdx.x] = r;
        }
    }
}

// ----------------------------------------------------------------------------
// Kepler drift (Sec. 2.1: WHFAST-derived drift; Sec. 3.1: one body per thread
// with a failure flag, positions and velocities copied first).  Universal
// variables: s solves r0 s + eta0 G2(s) + zeta0 G3(s) = dt with
// G_k(s) = s^k c_k(beta s^2), beta = 2 mu/r0 - v^2, zeta0 = mu - beta r0.
// ----------------------------------------------------------------------------
__host__ __device__ constexpr double inv_fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i)
        f *= (double)i;
    return 1.0 / f;
}

// c_k(z) = sum_n (-z)^n/(2n+k)! by a fixed-length Horner polynomial (|z| <= 1).
template <int K>
__device__ __forceinline__ double stumpff_series(double mz)
{
    double p = inv_fact(2 * 11 + K);
#pragma unroll
    for (int n = 10; n >= 0; --n)
        p = fma(p, mz, inv_fact(2 * n + K));
    return p;
}

__device__ __forceinline__ void gfuncs(double beta, double s, double &G1, double &G2, double &G3)
{
    double z = beta * s * s;
    double c1, c2, c3;
    if (fabs(z) <= 1.0) {
        c1 = stumpff_series<1>(-z);
        c2 = stumpff_series<2>(-z);
        c3 = stumpff_series<3>(-z);
    } else if (z > 0.0) {
        double x = sqrt(z), sx, cx;
        sincos(x, &sx, &cx);
        c1 = sx / x;
        c2 = (1.0 - cx) / z;
        c3 = (1.0 - c1) / z;
    } else {
        double x = sqrt(-z);
        c1 = sinh(x) / x;
        c2 = (1.0 - cosh(x)) / z;
        c3 = (1.0 - c1) / z;
    }
    G1 = s * c1;
    G2 = s * s * c2;
    G3 = s * s * s * c3;
}

// Returns 0 on success; on failure the body is left unchanged.
__device__ int kepler_drift(double mu, double dt, double &x, double &y, double &z, double &u,
                            double &v, double &w)
{
    if (dt == 0.0)
        return 0;
    double r0 = sqrt(x * x + y * y + z * z);
    double v2 = u * u + v * v + w * w;
    double eta0 = x * u + y * v + z * w;
    double beta = 2.0 * mu / r0 - v2;
    double zeta0 = mu - beta * r0;
    if (!(r0 > 0.0) || !isfinite(r0 + v2))
        return 1;

    const double tol = 2.0 * DBL_EPSILON;   // 4 u
    // second-order starting value of s
    double s = dt / r0;
    double corr = 1.0 - 0.5 * eta0 * dt / (r0 * r0);
    if (corr > 0.5 && corr < 2.0)
        s *= corr;
    double lo = dt > 0.0 ? 0.0 : -INFINITY;
    double hi = dt > 0.0 ? INFINITY : 0.0;
    double G1, G2, G3;
    bool ok = false;
    for (int it = 0; it < 100; ++it) {
        gfuncs(beta, s, G1, G2, G3);
        double F = r0 * s + eta0 * G2 + zeta0 * G3 - dt;
        double dF = r0 + eta0 * G1 + zeta0 * G2;
        if (F == 0.0) {
            ok = true;
            break;
        }
        if (F < 0.0)
            lo = s;
        else
            hi = s;
        double sn = s - F / dF;
        if (!(sn > lo && sn < hi)) {
            if (isfinite(lo) && isfinite(hi))
                sn = 0.5 * (lo + hi);
            else if (isfinite(lo))
                sn = lo > 0.0 ? 2.0 * lo : fabs(dt / r0);
            else
                sn = hi < 0.0 ? 2.0 * hi : -fabs(dt / r0);
        }
        double ds = sn - s;
        s = sn;
        if (fabs(ds) <= tol * fabs(s) || (hi - lo) <= tol * fabs(s)) {
            ok = true;
            break;
        }
    }
    if (!ok)
        return 1;
    gfuncs(beta, s, G1, G2, G3);
    double r = r0 + eta0 * G1 + zeta0 * G2;
    double fm1 = -mu * G2 / r0;
    double g = dt - mu * G3;
    double fd = -mu * G1 / (r * r0);
    double gdm1 = -mu * G2 / r;
    double nx = x + (fm1 * x + g * u), ny = y + (fm1 * y + g * v), nz = z + (fm1 * z + g * w);
    double nu = u + (fd * x + gdm1 * u), nv = v + (fd * y + gdm1 * v), nw = w + (fd * z + gdm1 * w);
    if (!isfinite(nx + ny + nz + nu + nv + nw))
        return 1;
    x = nx;
    y = ny;
    z = nz;
    u = nu;
    v = nv;
    w = nw;
    return 0;
}

// Snapshot, drift, failure flags and counters, the encounter check's records,
// and the partial sums of m V after the drift (for the second stellar drift).
// The check clears its own list and flags, since it may run beside the next drift.
__global__ void k_drift(const RBlk *__restrict__ rblk, const double *__restrict__ m0, double G,
                        double dt, const double *__restrict__ m, double *qx, double *qy,
                        double *qz, double *vx, double *vy, double *vz, double *__restrict__ q0x,
                        double *__restrict__ q0y, double *__restrict__ q0z,
                        double *__restrict__ v0x, double *__restrict__ v0y,
                        double *__restrict__ v0z, int *__restrict__ kflag,
                        DevStats *stats, double *__restrict__ part_out,
                        const double *__restrict__ rc, double4 *__restrict__ mr,
                        double4 *__restrict__ cr, double *__restrict__ lnr_part,
                        double *__restrict__ q1x, double *__restrict__ q1y,
                        double *__restrict__ q1z, double *__restrict__ v1x,
                        double *__restrict__ v1y, double *__restrict__ v1z,
                        double *__restrict__ rc1, const double *__restrict__ part_in,
                        double sun_h, const int *__restrict__ rb_first,
                        const int *__restrict__ rb_count, const double *__restrict__ ptot)
{
    __shared__ double sh[3 * kBlock];
    double lnr_lo = INFINITY, lnr_hi = -INFINITY;
    RBlk b = rblk[blockIdx.x];
    int i = b.start + threadIdx.x;
    const bool on = i < b.end;
    // the body's state, loaded while the system's momentum is summed
    const double xs = on ? qx[i] : 0.0, ys = on ? qy[i] : 0.0, zs = on ? qz[i] : 0.0;
    const double us = on ? vx[i] : 0.0, vs = on ? vy[i] : 0.0, ws = on ? vz[i] : 0.0;
    const double rci = on ? rc[i] : 0.0, mi = on ? m[i] : 0.0;
    double mu = G * m0[b.sys];
    bool fail = false;
    double pv[3] = {0.0, 0.0, 0.0};
    // the sun drift S(sun_h) that precedes the drift, from the per-block sums of
    // m V in part_in (same arithmetic as k_sun_drift)
    double sd[3] = {0.0, 0.0, 0.0};
    if (sun_h != 0.0) {
        // the system's momentum: precomputed per system (ptot) or summed here
        double P[3];
        if (ptot) {
            P[0] = ptot[(size_t)b.sys * 4];
            P[1] = ptot[(size_t)b.sys * 4 + 1];
            P[2] = ptot[(size_t)b.sys * 4 + 2];
        } else {
            system_sum<3>(part_in, 4, rb_first[b.sys], rb_count[b.sys], P, sh);
        }
        const double mm = m0[b.sys];
        sd[0] = sun_h * P[0] / mm;
        sd[1] = sun_h * P[1] / mm;
        sd[2] = sun_h * P[2] / mm;
    }
    if (on) {
        double x = xs + sd[0], y = ys + sd[1], z = zs + sd[2];
        double u = us, v = vs, w = ws;
        const double sx = x, sy = y, sz = z;
        q0x[i] = x;
        q0y[i] = y;
        q0z[i] = z;
        v0x[i] = u;
        v0y[i] = v;
        v0z[i] = w;
        fail = kepler_drift(mu, dt, x, y, z, u, v, w) != 0;
        // Encounter reach of this body over the step: chord c = Q1 - Q0 with
        // half-length rho, endpoint velocity deviations e = dt V - c with
        // largest norm eps; R = 2 rho + 3 eps/4 + rc (widened by 2^-20 for
        // rounding).  Pairs whose chord midpoints are farther apart than
        // R_i + R_j cannot be flagged (see k_encounter).
        {
            double cx = x - sx, cy = y - sy, cz = z - sz;
            double rho = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
            double ax0 = dt * us - cx, ay0 = dt * vs - cy, az0 = dt * ws - cz;
            double ax1 = dt * u - cx, ay1 = dt * v - cy, az1 = dt * w - cz;
            double eps = sqrt(fmax(ax0 * ax0 + ay0 * ay0 + az0 * az0, ax1 * ax1 + ay1 * ay1 + az1 * az1));
            double R = (2.0 * rho + 0.75 * eps + rci) * (1.0 + 0x1p-20);
            double mx = sx + 0.5 * cx, my = sy + 0.5 * cy, mz = sz + 0.5 * cz;
            mr[i] = make_double4(mx, my, mz, R);
            // relative pair filter data: the chord and 3/4 eps, widened by 2^-20
            // and by 2^-45 (|M| + |c|) to cover the rounding of midpoint and chord
            // differences (see k_encounter)
            double e34 = 0.75 * eps * (1.0 + 0x1p-20) +
                         0x1p-45 * (sqrt(mx * mx + my * my + mz * mz) + 2.0 * rho);
            cr[i] = make_double4(cx, cy, cz, e34);
            double lnr = log(fmax(sqrt(mx * mx + my * my), 1e-300));
            lnr_lo = lnr;
            lnr_hi = lnr;
        }
        qx[i] = x;
        qy[i] = y;
        qz[i] = z;
        vx[i] = u;
        vy[i] = v;
        vz[i] = w;
        q1x[i] = x;
        q1y[i] = y;
        q1z[i] = z;
        v1x[i] = u;
        v1y[i] = v;
        v1z[i] = w;
        rc1[i] = rci;
        kflag[i] = fail ? 1 : 0;
        pv[0] = mi * u;
        pv[1] = mi * v;
        pv[2] = mi * w;
    }
    unsigned long long mask = __ballot(fail);
    if (mask && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)mask) - 1)) {
        atomicAdd((unsigned long long *)&stats->kepler_fail, (unsigned long long)__popcll(mask));
        atomicAdd(&stats->cur_kfail, (int)__popcll(mask));
    }
    if (lnr_part) {
        // range of ln R over the block (the sorted encounter check bins by it)
        for (int o = 32; o > 0; o >>= 1) {
            lnr_lo = fmin(lnr_lo, __shfl_xor(lnr_lo, o));
            lnr_hi = fmax(lnr_hi, __shfl_xor(lnr_hi, o));
        }
        if ((threadIdx.x & 63) == 0) {
            sh[threadIdx.x >> 6] = lnr_lo;
            sh[kBlock / 64 + (threadIdx.x >> 6)] = lnr_hi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double lo = sh[0], hi = sh[kBlock / 64];
            for (int w = 1; w < kBlock / 64; ++w) {
                lo = fmin(lo, sh[w]);
                hi = fmax(hi, sh[kBlock / 64 + w]);
            }
            lnr_part[2 * (size_t)blockIdx.x] = lo;
            lnr_part[2 * (size_t)blockIdx.x + 1] = hi;
        }
        __syncthreads();
    }
    block_sum<3>(pv, sh);
    if (threadIdx.x == 0) {
        part_out[(size_t)blockIdx.x * 4 + 0] = pv[0];
        part_out[(size_t)blockIdx.x * 4 + 1] = pv[1];
        part_out[(size_t)blockIdx.x * 4 + 2] = pv[2];
        part_out[(size_t)blockIdx.x * 4 + 3] = 0.0;
    }
}

// ----------------------------------------------------------------------------
// Interaction force (Sec. 3.1 force block, loop 2): per target i the sum over
// sources j != i of m_j w(r_ij) (Q_j - Q_i); G is applied in the finalize pass.
// Pairs at or beyond rc_ij take the Newtonian term; pairs inside rc_ij take
// the exact changeover weight in a divergent branch.  The branch test is one
// compare per pair against a per-lane, per-tile threshold max(rc_i^2, max_j
// rc_j^2); the branch itself applies the exact pair test.
// ----------------------------------------------------------------------------

// m y^3 with y = 1/sqrt(r2): the hardware estimate y0 (worst relative error
// 2^-24.2 on gfx950) corrected through (1 - e)^(-3/2) = 1 + 3e/2 + O(e^2),
// e = 1 - r2 y0^2; the dropped 15e^2/8 term is below 2.1e-14.  m15 = 1.5 m.
__device__ __forceinline__ double m_rinv3(double m, double m15, double r2)
{
    double y0 = __builtin_amdgcn_rsq(r2);
    double y2 = y0 * y0;
    double e = fma(-r2, y2, 1.0);
    return (y0 * y2) * fma(m15, e, m);
}

// Work item layout shared by both force kernels: the block's 64*R targets are
// the same for its kBlock/64 waves; each source tile of kBlock bodies is staged
// in LDS and wave w takes its sources [64w, 64w+64).  The waves' sums are added
// in wave order through LDS at the end, so results do not depend on timing.
constexpr int kWaves = kBlock / 64;

template <int R>
__global__ __launch_bounds__(kBlock) void k_force64(const FWork *__restrict__ work,
                                                    const double *__restrict__ qx,
                                                    const double *__restrict__ qy,
                                                    const double *__restrict__ qz,
                                                    const double *__restrict__ m,
                                                    const double *__restrict__ rc,
                                                    const double *__restrict__ tile_rc2,
                                                    double *__restrict__ fpart, int ntot, int maxs,
                                                    double inner, DevStats *stats)
{
    __shared__ double4 sj[kBlock];
    __shared__ double2 sx[kBlock];                 // {1.5 m, rc}
    __shared__ double red[kWaves - 1][3 * R][64];
    const FWork wk = work[blockIdx.x];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    double xi[R], yi[R], zi[R], rci[R], r2i[R], ax[R], ay[R], az[R];
    int near = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        int li = lane + 64 * k;
        int i = wk.i0 + (li < wk.ni ? li : 0);
        xi[k] = qx[i];
        yi[k] = qy[i];
        zi[k] = qz[i];
        rci[k] = rc[i];
        r2i[k] = fmax(rci[k] * rci[k], DBL_MIN);
        ax[k] = ay[k] = az[k] = 0.0;
    }
    const int jend = wk.j0 + wk.nj;
    int tile = wk.rb0;
    for (int jt = wk.j0; jt < jend; jt += kBlock, ++tile) {
        const int cnt = min(kBlock, jend - jt);
        __syncthreads();
        if (t < cnt) {
            int j = jt + t;
            double mj = m[j];
            sj[t] = make_double4(qx[j], qy[j], qz[j], mj);
            sx[t] = make_double2(1.5 * mj, rc[j]);
        }
        const double tmax = tile_rc2[tile];
        double thr[R];
#pragma unroll
        for (int k = 0; k < R; ++k)
            thr[k] = fmax(r2i[k], tmax);
        __syncthreads();
        // the waves take the tile's sources in turn (wave w: w, w + 4, ...), so a
        // short or ragged source range still splits evenly over the 4 waves
#pragma unroll 2
        for (int jj = wv; jj < cnt; jj += kWaves) {
            const double4 J = sj[jj];
            const double m15 = sx[jj].x;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                double dx = J.x - xi[k], dy = J.y - yi[k], dz = J.z - zi[k];
                double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                double s = m_rinv3(J.w, m15, r2);
                if (r2 < thr[k]) {
                    double rcj = sx[jj].y;
                    if (r2 < fmax(r2i[k], fmax(rcj * rcj, DBL_MIN))) {
                        s = J.w * changeover_w(r2, fmax(rci[k], rcj), inner);
                        ++near;
                    }
                }
                ax[k] = fma(s, dx, ax[k]);
                ay[k] = fma(s, dy, ay[k]);
                az[k] = fma(s, dz, az[k]);
            }
        }
    }
    if (wv > 0) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            red[wv - 1][3 * k + 0][lane] = ax[k];
            red[wv - 1][3 * k + 1][lane] = ay[k];
            red[wv - 1][3 * k + 2][lane] = az[k];
        }
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            for (int w = 0; w < kWaves - 1; ++w) {
                ax[k] += red[w][3 * k + 0][lane];
                ay[k] += red[w][3 * k + 1][lane];
                az[k] += red[w][3 * k + 2][lane];
            }
            int li = lane + 64 * k;
            if (li < wk.ni) {
                int i = wk.i0 + li;
                fpart[((size_t)0 * maxs + wk.slot) * ntot + i] = ax[k];
                fpart[((size_t)1 * maxs + wk.slot) * ntot + i] = ay[k];
                fpart[((size_t)2 * maxs + wk.slot) * ntot + i] = az[k];
            }
        }
    }
    // pairs evaluated in the changeover zone (self pairs included), one atomic per wave
    for (int o = 32; o > 0; o >>= 1)
        near += __shfl_xor(near, o);
    if (lane == 0 && near)
        atomicAdd((unsigned long long *)&stats->near_pairs, (unsigned long long)near);
}

// FP32C: pair terms in FP32 from hi/lo split positions (the difference of two
// hi parts is exact for nearby bodies, the lo parts restore the rest), summed
// in FP32 over runs of kMerge sources and merged by two-sum into a per-target
// (hi, lo) accumulator.  Pairs whose FP32 distance falls inside a widened
// critical radius are evaluated in FP64 from the FP64 state instead.
constexpr int kMerge = 32;

__device__ __forceinline__ void two_sum_f(float &hi, float &lo, float t)
{
    float s = hi + t;
    float bp = s - hi;
    float e = (hi - (s - bp)) + (t - bp);
    hi = s;
    lo += e;
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_force32c(const FWork *__restrict__ work,
                                                     const float4 *__restrict__ pk,
                                                     const double *__restrict__ qx,
                                                     const double *__restrict__ qy,
                                                     const double *__restrict__ qz,
                                                     const double *__restrict__ m,
                                                     const double *__restrict__ rc,
                                                     const double *__restrict__ tile_rc2,
                                                     float *__restrict__ fpart, int ntot,
                                                     int maxs, double inner, DevStats *stats)
{
    __shared__ float4 sa[kBlock];
    __shared__ float4 sb[kBlock];
    __shared__ double red[kWaves - 1][3 * R][64];
    const FWork wk = work[blockIdx.x];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    float xh[R], yh[R], zh[R], xl[R], yl[R], zl[R], r2i[R];
    float hx[R], hy[R], hz[R], lx[R], ly[R], lz[R], tx[R], ty[R], tz[R];
    double nx[R], ny[R], nz[R];
    int ii[R];
    int near = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        int li = lane + 64 * k;
        int i = wk.i0 + (li < wk.ni ? li : 0);
        ii[k] = i;
        float4 A = pk[2 * (size_t)i], B = pk[2 * (size_t)i + 1];
        xh[k] = A.x; yh[k] = A.y; zh[k] = A.z;
        xl[k] = B.x; yl[k] = B.y; zl[k] = B.z;
        r2i[k] = B.w;
        hx[k] = hy[k] = hz[k] = lx[k] = ly[k] = lz[k] = tx[k] = ty[k] = tz[k] = 0.0f;
        nx[k] = ny[k] = nz[k] = 0.0;
    }
    const int jend = wk.j0 + wk.nj;
    int tile = wk.rb0;
    for (int jt = wk.j0; jt < jend; jt += kBlock, ++tile) {
        const int cnt = min(kBlock, jend - jt);
        __syncthreads();
        if (t < cnt) {
            sa[t] = pk[2 * (size_t)(jt + t)];
            sb[t] = pk[2 * (size_t)(jt + t) + 1];
        }
        // widened like the per-body FP32 radii so the FP32 test stays a superset
        const float tmax = (float)(tile_rc2[tile] * (1.0 + 0x1p-9));
        float thr[R];
#pragma unroll
        for (int k = 0; k < R; ++k)
            thr[k] = fmaxf(r2i[k], tmax);
        __syncthreads();
        // the waves take the tile's sources in turn (wave w: w, w + 4, ...); each
        // run of kMerge of a wave's sources is summed in FP32, then merged
        for (int jb = wv; jb < cnt; jb += kWaves * kMerge) {
            const int jm = min(cnt, jb + kWaves * kMerge);
#pragma unroll 2
            for (int jj = jb; jj < jm; jj += kWaves) {
                const float4 A = sa[jj];
                const float4 B = sb[jj];
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    float dx = (A.x - xh[k]) + (B.x - xl[k]);
                    float dy = (A.y - yh[k]) + (B.y - yl[k]);
                    float dz = (A.z - zh[k]) + (B.z - zl[k]);
                    float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    float y = __builtin_amdgcn_rsqf(r2);
                    float s = (A.w * y) * (y * y);
                    if (r2 < thr[k]) {
                        if (r2 < fmaxf(r2i[k], B.w)) {
                            // FP64 changeover pair from the FP64 state
                            int i = ii[k], j = jt + jj;
                            double ex = qx[j] - qx[i], ey = qy[j] - qy[i], ez = qz[j] - qz[i];
                            double d2 = fma(ez, ez, fma(ey, ey, ex * ex));
                            double wgt = m[j] * changeover_w(d2, fmax(rc[i], rc[j]), inner);
                            nx[k] = fma(wgt, ex, nx[k]);
                            ny[k] = fma(wgt, ey, ny[k]);
                            nz[k] = fma(wgt, ez, nz[k]);
                            s = 0.0f;
                            ++near;
                        }
                    }
                    tx[k] = fmaf(s, dx, tx[k]);
                    ty[k] = fmaf(s, dy, ty[k]);
                    tz[k] = fmaf(s, dz, tz[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < R; ++k) {
                two_sum_f(hx[k], lx[k], tx[k]);
                two_sum_f(hy[k], ly[k], ty[k]);
                two_sum_f(hz[k], lz[k], tz[k]);
                tx[k] = ty[k] = tz[k] = 0.0f;
            }
        }
    }
    double sx_[R], sy_[R], sz_[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        sx_[k] = ((double)hx[k] + (double)lx[k]) + nx[k];
        sy_[k] = ((double)hy[k] + (double)ly[k]) + ny[k];
        sz_[k] = ((double)hz[k] + (double)lz[k]) + nz[k];
    }
    if (wv > 0) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            red[wv - 1][3 * k + 0][lane] = sx_[k];
            red[wv - 1][3 * k + 1][lane] = sy_[k];
            red[wv - 1][3 * k + 2][lane] = sz_[k];
        }
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            for (int w = 0; w < kWaves - 1; ++w) {
                sx_[k] += red[w][3 * k + 0][lane];
                sy_[k] += red[w][3 * k + 1][lane];
                sz_[k] += red[w][3 * k + 2][lane];
            }
            int li = lane + 64 * k;
            if (li < wk.ni) {
                int i = wk.i0 + li;
                fpart[((size_t)0 * maxs + wk.slot) * ntot + i] = (float)sx_[k];
                fpart[((size_t)1 * maxs + wk.slot) * ntot + i] = (float)sy_[k];
                fpart[((size_t)2 * maxs + wk.slot) * ntot + i] = (float)sz_[k];
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1)
        near += __shfl_xor(near, o);
    if (lane == 0 && near)
        atomicAdd((unsigned long long *)&stats->near_pairs, (unsigned long long)near);
}

// Few sources (every system has at most kFewMax big bodies, one split): each
// wave owns the 64 R targets of a work item and sums over all of the system's
// sources, held in the wave's own LDS slice; waves stride over the items and
// restage the sources only when the system changes.  Same pair arithmetic and
// per-target source order as the kernels above, no cross-wave reduction.
constexpr int kFewMax = 256;

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_force64_few(const FWork *__restrict__ work, int nfw,
                                                        const double *__restrict__ qx,
                                                        const double *__restrict__ qy,
                                                        const double *__restrict__ qz,
                                                        const double *__restrict__ m,
                                                        const double *__restrict__ rc,
                                                        const double *__restrict__ tile_rc2,
                                                        double *__restrict__ fpart, int ntot, int maxs,
                                                        double inner, DevStats *stats)
{
    __shared__ double4 sj[kWaves][kFewMax];
    __shared__ double2 sx[kWaves][kFewMax];     // {1.5 m, rc}
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int cached = -1, near = 0;
    for (int it = blockIdx.x * kWaves + wv; it < nfw; it += gridDim.x * kWaves) {
        const FWork wk = work[it];
        if (wk.j0 != cached) {
            for (int k = lane; k < wk.nj; k += 64) {
                const int j = wk.j0 + k;
                const double mj = m[j];
                sj[wv][k] = make_double4(qx[j], qy[j], qz[j], mj);
                sx[wv][k] = make_double2(1.5 * mj, rc[j]);
            }
            cached = wk.j0;
            wave_lds_sync();
        }
        double xi[R], yi[R], zi[R], rci[R], r2i[R], thr[R], ax[R], ay[R], az[R];
        const double tmax = tile_rc2[wk.rb0];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int li = lane + 64 * k;
            const int i = wk.i0 + (li < wk.ni ? li : 0);
            xi[k] = qx[i];
            yi[k] = qy[i];
            zi[k] = qz[i];
            rci[k] = rc[i];
            r2i[k] = fmax(rci[k] * rci[k], DBL_MIN);
            thr[k] = fmax(r2i[k], tmax);
            ax[k] = ay[k] = az[k] = 0.0;
        }
#pragma unroll 2
        for (int jj = 0; jj < wk.nj; ++jj) {
            const double4 J = sj[wv][jj];
            const double m15 = sx[wv][jj].x;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                double dx = J.x - xi[k], dy = J.y - yi[k], dz = J.z - zi[k];
                double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                double s = m_rinv3(J.w, m15, r2);
                if (r2 < thr[k]) {
                    double rcj = sx[wv][jj].y;
                    if (r2 < fmax(r2i[k], fmax(rcj * rcj, DBL_MIN))) {
                        s = J.w * changeover_w(r2, fmax(rci[k], rcj), inner);
                        ++near;
                    }
                }
                ax[k] = fma(s, dx, ax[k]);
                ay[k] = fma(s, dy, ay[k]);
                az[k] = fma(s, dz, az[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int li = lane + 64 * k;
            if (li < wk.ni) {
                const int i = wk.i0 + li;
                fpart[((size_t)0 * maxs + wk.slot) * ntot + i] = ax[k];
                fpart[((size_t)1 * maxs + wk.slot) * ntot + i] = ay[k];
                fpart[((size_t)2 * maxs + wk.slot) * ntot + i] = az[k];
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1)
        near += __shfl_xor(near, o);
    if (lane == 0 && near)
        atomicAdd((unsigned long long *)&stats->near_pairs, (unsigned long long)near);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_force32c_few(const FWork *__restrict__ work, int nfw,
                                                         const float4 *__restrict__ pk,
                                                         const double *__restrict__ qx,
                                                         const double *__restrict__ qy,
                                                         const double *__restrict__ qz,
                                                         const double *__restrict__ m,
                                                         const double *__restrict__ rc,
                                                         const double *__restrict__ tile_rc2,
                                                         float *__restrict__ fpart, int ntot,
                                                         int maxs, double inner, DevStats *stats)
{
    __shared__ float4 sa[kWaves][kFewMax];
    __shared__ float4 sb[kWaves][kFewMax];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int cached = -1, near = 0;
    for (int it = blockIdx.x * kWaves + wv; it < nfw; it += gridDim.x * kWaves) {
        const FWork wk = work[it];
        if (wk.j0 != cached) {
            for (int k = lane; k < wk.nj; k += 64) {
                sa[wv][k] = pk[2 * (size_t)(wk.j0 + k)];
                sb[wv][k] = pk[2 * (size_t)(wk.j0 + k) + 1];
            }
            cached = wk.j0;
            wave_lds_sync();
        }
        float xh[R], yh[R], zh[R], xl[R], yl[R], zl[R], r2i[R], thr[R];
        float hx[R], hy[R], hz[R], lx[R], ly[R], lz[R], tx[R], ty[R], tz[R];
        double nx[R], ny[R], nz[R];
        int ii[R];
        const float tmax = (float)(tile_rc2[wk.rb0] * (1.0 + 0x1p-9));
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int li = lane + 64 * k;
            const int i = wk.i0 + (li < wk.ni ? li : 0);
            ii[k] = i;
            const float4 A = pk[2 * (size_t)i], B = pk[2 * (size_t)i + 1];
            xh[k] = A.x; yh[k] = A.y; zh[k] = A.z;
            xl[k] = B.x; yl[k] = B.y; zl[k] = B.z;
            r2i[k] = B.w;
            thr[k] = fmaxf(r2i[k], tmax);
            hx[k] = hy[k] = hz[k] = lx[k] = ly[k] = lz[k] = tx[k] = ty[k] = tz[k] = 0.0f;
            nx[k] = ny[k] = nz[k] = 0.0;
        }
        for (int jb = 0; jb < wk.nj; jb += kMerge) {
            const int jm = min(wk.nj, jb + kMerge);
#pragma unroll 2
            for (int jj = jb; jj < jm; ++jj) {
                const float4 A = sa[wv][jj];
                const float4 B = sb[wv][jj];
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    float dx = (A.x - xh[k]) + (B.x - xl[k]);
                    float dy = (A.y - yh[k]) + (B.y - yl[k]);
                    float dz = (A.z - zh[k]) + (B.z - zl[k]);
                    float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    float y = __builtin_amdgcn_rsqf(r2);
                    float s = (A.w * y) * (y * y);
                    if (r2 < thr[k]) {
                        if (r2 < fmaxf(r2i[k], B.w)) {
                            int i = ii[k], j = wk.j0 + jj;
                            double ex = qx[j] - qx[i], ey = qy[j] - qy[i], ez = qz[j] - qz[i];
                            double d2 = fma(ez, ez, fma(ey, ey, ex * ex));
                            double wgt = m[j] * changeover_w(d2, fmax(rc[i], rc[j]), inner);
                            nx[k] = fma(wgt, ex, nx[k]);
                            ny[k] = fma(wgt, ey, ny[k]);
                            nz[k] = fma(wgt, ez, nz[k]);
                            s = 0.0f;
                            ++near;
                        }
                    }
                    tx[k] = fmaf(s, dx, tx[k]);
                    ty[k] = fmaf(s, dy, ty[k]);
                    tz[k] = fmaf(s, dz, tz[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < R; ++k) {
                two_sum_f(hx[k], lx[k], tx[k]);
                two_sum_f(hy[k], ly[k], ty[k]);
                two_sum_f(hz[k], lz[k], tz[k]);
                tx[k] = ty[k] = tz[k] = 0.0f;
            }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int li = lane + 64 * k;
            if (li < wk.ni) {
                const int i = wk.i0 + li;
                fpart[((size_t)0 * maxs + wk.slot) * ntot + i] = (float)(((double)hx[k] + (double)lx[k]) + nx[k]);
                fpart[((size_t)1 * maxs + wk.slot) * ntot + i] = (float)(((double)hy[k] + (double)ly[k]) + ny[k]);
                fpart[((size_t)2 * maxs + wk.slot) * ntot + i] = (float)(((double)hz[k] + (double)lz[k]) + nz[k]);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1)
        near += __shfl_xor(near, o);
    if (lane == 0 && near)
        atomicAdd((unsigned long long *)&stats->near_pairs, (unsigned long long)near);
}

// Symmetric pairs (every body big): each unordered pair is evaluated once and
// applied to both bodies, a_i += m_j q d and a_j -= m_i q d with the mass-free
// weight q = K/r^3 - K'/r^2 (Newtonian q = 1/r^3 refined from the hardware
// estimate as in m_rinv3).  Bodies of a system form tiles of T = 64 R and
// super-tiles of G tiles.  A work item is a pair of super-tiles (I <= J),
// owned by a workgroup of G waves: wave w holds the R targets per lane of tile
// w of I in registers, the G tiles of J sit in LDS together with their
// accumulators, and in round k wave w meets tile (w + k) mod G of J, so that no
// two waves update one source tile at once.  Within a tile pair, at step k of
// sub-tile t, lane L pairs with source 64 t + (L xor k), so the 64 lanes touch
// 64 different sources and update their accumulators without atomics.  Item
// (I, J) writes super-tile I's sums to split slot J and super-tile J's sums to
// slot I (both to slot I on the diagonal, where each pair is met once), so
// every body receives exactly one partial per super-tile of its system, summed
// in slot order by the finalize pass: G times fewer partials than tiles, in a
// fixed order whatever the schedule.  The register budget keeps three waves
// per SIMD (two at R = 4), as with one wave per work item.
__device__ __forceinline__ double rinv3(double r2)
{
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double y2 = y0 * y0;
    const double e = fma(-r2, y2, 1.0);
    return (y0 * y2) * fma(1.5, e, 1.0);
}

// Largest value over the wave, returned in a scalar register (every lane active).
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o));
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// max of two non-negative finite floats through their bit patterns (one
// integer instruction, no NaN handling needed)
__device__ __forceinline__ float max_nonneg(float a, float b)
{
    return __int_as_float(max(__float_as_int(a), __float_as_int(b)));
}

__device__ __forceinline__ float wave_max_nonneg(float v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = max_nonneg(v, __shfl_xor(v, o));
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// LDS addresses as 32-bit integers, for the rotating source index of the
// symmetric kernels: with a tile array aligned to 64 elements, the address of
// element 64 t + (lane xor k) is that of element 64 t + lane with k times the
// element size xored in.
typedef float lds_v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) lds_v4f lds_float4;
typedef __attribute__((address_space(3))) double lds_double;

__device__ __forceinline__ uint32_t lds_addr(float4 *p)
{
    return (uint32_t)(uintptr_t)(lds_float4 *)p;
}

__device__ __forceinline__ uint32_t lds_addr(double *p)
{
    return (uint32_t)(uintptr_t)(lds_double *)p;
}

__device__ __forceinline__ float4 lds_ld4(uint32_t a)
{
    const lds_v4f v = *(const lds_float4 *)(uintptr_t)a;
    return make_float4(v.x, v.y, v.z, v.w);
}

// x, y, z of a 16-byte record (the fourth word is neither read nor written)
typedef float lds_v3f __attribute__((ext_vector_type(3)));
typedef __attribute__((address_space(3))) lds_v3f lds_float3;

__device__ __forceinline__ lds_v3f lds_ld3(uint32_t a)
{
    return *(const lds_float3 *)(uintptr_t)a;
}

__device__ __forceinline__ void lds_st3(uint32_t a, float x, float y, float z)
{
    *(lds_float3 *)(uintptr_t)a = lds_v3f{x, y, z};
}

__device__ __forceinline__ double lds_ld8(uint32_t a)
{
    return *(const lds_double *)(uintptr_t)a;
}

__device__ __forceinline__ void lds_st8(uint32_t a, double v)
{
    *(lds_double *)(uintptr_t)a = v;
}

// Tile J of one wave in LDS, one array per component (consecutive lanes touch
// consecutive 8-byte words: no bank conflicts for the rotating accesses).
template <int T>
struct alignas(512) SymTile64 {
    double x[T], y[T], z[T], m[T];
    double r2[T];                      // max(rc^2, DBL_MIN)
    double rc[T];
    double ax[T], ay[T], az[T];        // tile J's sums
};
static_assert(offsetof(SymTile64<64>, m) == 8 * 3 * 64 && offsetof(SymTile64<64>, r2) == 8 * 4 * 64 &&
                  offsetof(SymTile64<64>, rc) == 8 * 5 * 64 && offsetof(SymTile64<64>, ax) == 8 * 6 * 64,
              "SymTile64 layout");

template <int R, bool DIAG, int T>
__device__ __forceinline__ void sym_tile64(SymTile64<T> &L, int lane, int i0, int ni, double inner,
                                           const double *__restrict__ rc, const double (&xi)[R],
                                           const double (&yi)[R], const double (&zi)[R],
                                           const double (&mi)[R], double tmi, double (&ax)[R],
                                           double (&ay)[R], double (&az)[R], int &near)
{
#pragma unroll 1
    for (int t = 0; t < R; ++t) {
        // Step k: lane L pairs its targets with source L xor k of sub-tile t,
        // so the lanes of a step touch distinct sources and each lane meets
        // every source once in 64 steps.  The sums a step reads were written by
        // another lane one step earlier: LDS operations of a wave complete in
        // issue order, and the compiler barrier keeps the read after that
        // write.  Sources are read-only and read one step ahead.
        // the largest rc^2 of the wave's targets and of the sub-tile's sources:
        // one compare per pair outside the rare branch
        const double thr = fmax(tmi, wave_max(L.r2[64 * t + lane]));
        // LDS address of x[64 t + lane]; the other arrays at fixed offsets
        const uint32_t self = lds_addr(&L.x[64 * t + lane]);
        uint32_t ac = self;
        double jxs = lds_ld8(ac), jys = lds_ld8(ac + 8 * T), jzs = lds_ld8(ac + 16 * T),
               jms = lds_ld8(ac + 24 * T);
#pragma unroll 2
        for (int k = 0; k < 64; ++k) {
            const uint32_t an = self ^ (uint32_t)(((k + 1) & 63) << 3);
            const double xn = lds_ld8(an), yn = lds_ld8(an + 8 * T), zn = lds_ld8(an + 16 * T),
                         mn = lds_ld8(an + 24 * T);
            double jx = lds_ld8(ac + 48 * T), jy = lds_ld8(ac + 56 * T), jz = lds_ld8(ac + 64 * T);
            // the R pairs' geometry first, then one branch for the rare ones,
            // so that the R chains share one basic block
            double dxr[R], dyr[R], dzr[R], r2r[R], qr[R];
            bool cand = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                dxr[r] = jxs - xi[r];
                dyr[r] = jys - yi[r];
                dzr[r] = jzs - zi[r];
                r2r[r] = fma(dzr[r], dzr[r], fma(dyr[r], dyr[r], dxr[r] * dxr[r]));
                qr[r] = rinv3(r2r[r]);
                const bool on = !DIAG || (64 * r + lane < 64 * t + (lane ^ k));
                cand |= r2r[r] < thr && on;
                if (DIAG)
                    qr[r] = on ? qr[r] : 0.0;
            }
            if (cand) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const bool on = !DIAG || (64 * r + lane < 64 * t + (lane ^ k));
                    if (r2r[r] < thr && on) {
                        // rare: the target's rc from memory (a padded target is a copy
                        // of body i0), the source's rc^2 and rc from its LDS record
                        const int li = 64 * r + lane;
                        const double rci = rc[i0 + (li < ni ? li : 0)];
                        if (r2r[r] < fmax(fmax(rci * rci, DBL_MIN), lds_ld8(ac + 32 * T))) {
                            qr[r] = changeover_w(r2r[r], fmax(rci, lds_ld8(ac + 40 * T)), inner);
                            ++near;
                        }
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double dx = dxr[r], dy = dyr[r], dz = dzr[r], q = qr[r];
                const double wi = jms * q, wj = mi[r] * q;
                ax[r] = fma(wi, dx, ax[r]);
                ay[r] = fma(wi, dy, ay[r]);
                az[r] = fma(wi, dz, az[r]);
                jx = fma(-wj, dx, jx);
                jy = fma(-wj, dy, jy);
                jz = fma(-wj, dz, jz);
            }
            lds_st8(ac + 48 * T, jx);
            lds_st8(ac + 56 * T, jy);
            lds_st8(ac + 64 * T, jz);
            __asm__ __volatile__("" ::: "memory");
            ac = an;
            jxs = xn;
            jys = yn;
            jzs = zn;
            jms = mn;
        }
    }
}

// A double moved one lane down the wave: lane L gets lane (L + 1) mod 64's
// value (DPP wave rotate, one VALU per 32-bit half).
__device__ __forceinline__ double wave_rotl1(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, 0x134, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x134, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Tile J of one wave for the FP64 loop with source sums in registers (R <= 2).
// Each sub-tile's source records are stored twice over (entry 64 + j repeats
// j), so that lane L reads source (L + k) mod 64 at entry L + k: a fixed
// offset from the lane's own entry, no wrap.  Only the FP64 totals of the
// sources' sums live here.
template <int R>
struct alignas(512) SymTile64R {
    struct Sub {
        double x[128], y[128], z[128], m[128];
    } s[R];
    double r2[64 * R];                 // max(rc^2, DBL_MIN)
    double rc[64 * R];
    double ax[64 * R], ay[64 * R], az[64 * R];   // tile J's FP64 totals
};

template <int R>
__device__ __forceinline__ void put_src64(SymTile64R<R> &S, int e, double x, double y, double z,
                                          double m, double rcj)
{
    typename SymTile64R<R>::Sub &U = S.s[e / 64];
    const int j = e % 64;
    U.x[j] = U.x[j + 64] = x;
    U.y[j] = U.y[j + 64] = y;
    U.z[j] = U.z[j + 64] = z;
    U.m[j] = U.m[j + 64] = m;
    S.rc[e] = rcj;
    S.r2[e] = fmax(rcj * rcj, DBL_MIN);
    S.ax[e] = S.ay[e] = S.az[e] = 0.0;
}

template <int T>
__device__ __forceinline__ void put_src64(SymTile64<T> &S, int e, double x, double y, double z,
                                          double m, double rcj)
{
    S.x[e] = x;
    S.y[e] = y;
    S.z[e] = z;
    S.m[e] = m;
    S.rc[e] = rcj;
    S.r2[e] = fmax(rcj * rcj, DBL_MIN);
    S.ax[e] = S.ay[e] = S.az[e] = 0.0;
}

// The tile pair of sym_tile64 with the sources' running sums in registers:
// in step k lane L pairs its targets with source (L + k) mod 64 of sub-tile t
// and holds that source's sums; after the step the sums move one lane down
// (wave_rotl1), where that source is met next.  After 64 steps every lane
// holds its own source's sums again and adds them to the FP64 totals.  The LDS
// then carries only the source records (32 B per lane and step instead of 80
// with the sums' read-modify-write), which keeps the FP64 loop off the LDS
// bandwidth limit; the moves cost 6 VALU per step.
template <int R, bool DIAG>
__device__ __forceinline__ void sym_tile64_rot(SymTile64R<R> &L, int lane, int i0, int ni,
                                               double inner, const double *__restrict__ rc,
                                               const double (&xi)[R], const double (&yi)[R],
                                               const double (&zi)[R], const double (&mi)[R],
                                               double tmi, double (&ax)[R], double (&ay)[R],
                                               double (&az)[R], int &near)
{
#pragma unroll 1
    for (int t = 0; t < R; ++t) {
        const double thr = fmax(tmi, wave_max(L.r2[64 * t + lane]));
        // LDS address of x[lane] of sub-tile t; y, z, m at fixed offsets
        constexpr uint32_t kY = 8 * 128, kZ = 16 * 128, kM = 24 * 128;
        uint32_t ac = lds_addr(&L.s[t].x[lane]);
        double jxs = lds_ld8(ac), jys = lds_ld8(ac + kY), jzs = lds_ld8(ac + kZ), jms = lds_ld8(ac + kM);
        double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll 2
        for (int k = 0; k < 64; ++k) {
            const uint32_t an = ac + 8;
            const double xn = lds_ld8(an), yn = lds_ld8(an + kY), zn = lds_ld8(an + kZ),
                         mn = lds_ld8(an + kM);
            double dxr[R], dyr[R], dzr[R], r2r[R], qr[R];
            bool cand = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                dxr[r] = jxs - xi[r];
                dyr[r] = jys - yi[r];
                dzr[r] = jzs - zi[r];
                r2r[r] = fma(dzr[r], dzr[r], fma(dyr[r], dyr[r], dxr[r] * dxr[r]));
                qr[r] = rinv3(r2r[r]);
                const bool on = !DIAG || (64 * r + lane < 64 * t + ((lane + k) & 63));
                cand |= r2r[r] < thr && on;
                if (DIAG)
                    qr[r] = on ? qr[r] : 0.0;
            }
            if (cand) {
                const int sj = 64 * t + ((lane + k) & 63);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const bool on = !DIAG || (64 * r + lane < sj);
                    if (r2r[r] < thr && on) {
                        const int li = 64 * r + lane;
                        const double rci = rc[i0 + (li < ni ? li : 0)];
                        if (r2r[r] < fmax(fmax(rci * rci, DBL_MIN), L.r2[sj])) {
                            qr[r] = changeover_w(r2r[r], fmax(rci, L.rc[sj]), inner);
                            ++near;
                        }
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double dx = dxr[r], dy = dyr[r], dz = dzr[r], q = qr[r];
                const double wi = jms * q, wj = mi[r] * q;
                ax[r] = fma(wi, dx, ax[r]);
                ay[r] = fma(wi, dy, ay[r]);
                az[r] = fma(wi, dz, az[r]);
                jx = fma(-wj, dx, jx);
                jy = fma(-wj, dy, jy);
                jz = fma(-wj, dz, jz);
            }
            jx = wave_rotl1(jx);
            jy = wave_rotl1(jy);
            jz = wave_rotl1(jz);
            ac = an;
            jxs = xn;
            jys = yn;
            jzs = zn;
            jms = mn;
        }
        L.ax[64 * t + lane] += jx;
        L.ay[64 * t + lane] += jy;
        L.az[64 * t + lane] += jz;
    }
}

template <int R, bool DIAG, int T>
__device__ __forceinline__ void sym_round64(SymTile64R<R> &L, int lane, int i0, int ni, double inner,
                                            const double *__restrict__ rc, const double (&xi)[R],
                                            const double (&yi)[R], const double (&zi)[R],
                                            const double (&mi)[R], double tmi, double (&ax)[R],
                                            double (&ay)[R], double (&az)[R], int &near)
{
    sym_tile64_rot<R, DIAG>(L, lane, i0, ni, inner, rc, xi, yi, zi, mi, tmi, ax, ay, az, near);
}

template <int R, bool DIAG, int T>
__device__ __forceinline__ void sym_round64(SymTile64<T> &L, int lane, int i0, int ni, double inner,
                                            const double *__restrict__ rc, const double (&xi)[R],
                                            const double (&yi)[R], const double (&zi)[R],
                                            const double (&mi)[R], double tmi, double (&ax)[R],
                                            double (&ay)[R], double (&az)[R], int &near)
{
    sym_tile64<R, DIAG, T>(L, lane, i0, ni, inner, rc, xi, yi, zi, mi, tmi, ax, ay, az, near);
}

template <int R, int G>
__global__ __launch_bounds__(64 * G, R == 4 ? 2 : 3) void k_force64_sym(const FWork *__restrict__ work, int nitems,
                                                        const double *__restrict__ qx,
                                                        const double *__restrict__ qy,
                                                        const double *__restrict__ qz,
                                                        const double *__restrict__ m,
                                                        const double *__restrict__ rc,
                                                        double *__restrict__ fpart, int ntot, int maxs,
                                                        double inner, DevStats *stats)
{
    constexpr int T = 64 * R;
    // R <= 2: the sources' sums in registers, moved between lanes (LDS holds
    // the records only); R = 4 amortises the sums' LDS traffic over four
    // targets per lane and keeps them in LDS, within its LDS budget
    using Tile = typename std::conditional<(R <= 2), SymTile64R<R>, SymTile64<T>>::type;
    __shared__ Tile tl[G];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int near = 0;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const FWork wk = work[it];
        const bool diag = wk.i0 == wk.j0;
        // the G source tiles of super-tile J (nj real records from j0)
        for (int k = threadIdx.x; k < G * T; k += 64 * G) {
            // sources past the end: massless and far away (r^2 ~ 1e300, so
            // their weight underflows to 0 instead of meeting a target at r = 0)
            const bool ok = k < wk.nj;
            const int j = wk.j0 + (ok ? k : 0);
            put_src64(tl[k / T], k % T, ok ? qx[j] : 1e150, ok ? qy[j] : 1e150, ok ? qz[j] : 1e150,
                      ok ? m[j] : 0.0, ok ? rc[j] : 0.0);
        }
        __syncthreads();
        // this wave's target tile: tni bodies from ti0 (none when tni <= 0)
        const int ti0 = wk.i0 + wv * T;
        const int tni = min(T, wk.ni - wv * T);
        double xi[R], yi[R], zi[R], mi[R], ax[R], ay[R], az[R];
        double tmi = DBL_MIN;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int li = 64 * r + lane;
            const bool ok = li < tni;
            const int i = ok ? ti0 + li : wk.i0;
            xi[r] = qx[i];
            yi[r] = qy[i];
            zi[r] = qz[i];
            // targets past the tile end are massless: they add nothing to the sources
            mi[r] = ok ? m[i] : 0.0;
            tmi = fmax(tmi, rc[i] * rc[i]);
            ax[r] = ay[r] = az[r] = 0.0;
        }
        tmi = wave_max(tmi);
        // rounds as in the FP32C kernel: wave w meets source tile (w + k) mod G
        const int nr = diag ? G / 2 + 1 : G;
        for (int k = 0; k < nr; ++k) {
            const int s = (wv + k) % G;
            const bool go = tni > 0 && s * T < wk.nj && !(diag && 2 * k == G && wv >= G / 2);
            if (go) {
                if (diag && k == 0)
                    sym_round64<R, true, T>(tl[s], lane, ti0, tni, inner, rc, xi, yi, zi, mi, tmi,
                                            ax, ay, az, near);
                else
                    sym_round64<R, false, T>(tl[s], lane, ti0, tni, inner, rc, xi, yi, zi, mi, tmi,
                                             ax, ay, az, near);
            }
            __syncthreads();
        }
        // super-tile I's sums to slot J (on the diagonal together with the same
        // bodies' sums as sources)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int li = 64 * r + lane;
            if (li < tni) {
                double sx_ = ax[r], sy_ = ay[r], sz_ = az[r];
                if (diag) {
                    sx_ += tl[wv].ax[li];
                    sy_ += tl[wv].ay[li];
                    sz_ += tl[wv].az[li];
                }
                const int i = ti0 + li;
                fpart[((size_t)0 * maxs + wk.slot) * ntot + i] = sx_;
                fpart[((size_t)1 * maxs + wk.slot) * ntot + i] = sy_;
                fpart[((size_t)2 * maxs + wk.slot) * ntot + i] = sz_;
            }
        }
        if (!diag) {
            // super-tile J's sums to slot I
            for (int k = threadIdx.x; k < wk.nj; k += 64 * G) {
                const Tile &S = tl[k / T];
                const int e = k % T, j = wk.j0 + k;
                fpart[((size_t)0 * maxs + wk.pad) * ntot + j] = S.ax[e];
                fpart[((size_t)1 * maxs + wk.pad) * ntot + j] = S.ay[e];
                fpart[((size_t)2 * maxs + wk.pad) * ntot + j] = S.az[e];
            }
        }
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1)
        near += __shfl_xor(near, o);
    if (lane == 0 && near)
        atomicAdd((unsigned long long *)&stats->near_pairs, (unsigned long long)near);
}

// FP32C form of the symmetric tile pairs.  Pair terms in FP32 from the hi/lo
// records.  Tile I's sums: FP32 runs of half a sub-tile round (32 steps)
// merged by two-sum into a (hi, lo) pair per target.  Tile J's sums: an FP32
// run sum per source in LDS over the same 32 steps, added to the source's FP64
// total when the run ends.  Changeover pairs in FP64 from the FP64 state: the
// target's part into its (hi, lo) pair, the source's part to its FP64 total.
// Each split partial is stored rounded to FP32: a rounding of at most 2^-24 of
// the partial, which is at most the sum of its terms' magnitudes, so all of a
// body's partials together add at most 2^-24 A_i (A_i the sum of the magnitudes
// of its pair terms), below the FP32 pair terms' own error.
// Aligned to 1024 bytes, so that the LDS address of a[64 t + (lane xor k)]
// is that of a[64 t + lane] with 16 k xored in (k < 64): one VALU per step
// addresses a[], b[] and run[] (fixed offsets 16 T and 32 T from a[]).
template <int T>
struct alignas(1024) SymTile32 {
    float4 a[T];                    // hi parts and mass
    float4 b[T];                    // lo parts and widened rc^2
    float4 run[T];                  // current FP32 run sums of tile J (x, y, z, -)
    double ax[T], ay[T], az[T];     // FP64 totals of tile J (consecutive planes)
};
static_assert(offsetof(SymTile32<64>, b) == 16 * 64 && offsetof(SymTile32<64>, run) == 32 * 64,
              "SymTile32 layout");
static_assert(offsetof(SymTile32<128>, b) == 16 * 128 && offsetof(SymTile32<128>, run) == 32 * 128,
              "SymTile32 layout");

// The target's FP64 part of a changeover pair (hit: the pair was one).
struct ChgPart {
    double x, y, z;
    int hit;
};

// The rare branch of the FP32C pair loop, out of line so that it adds nothing
// to the loop: target li of the item (position i0 + li, or a padded copy of
// position i0 when li >= ni) against source jj (position j0 + jj, found from the
// LDS addresses of its record, ja, and of the tile's first record, a0) at FP32
// squared distance r2.  Positions are body indices, or with a sorted order
// (ord != nullptr) the bodies ord[position].
// Unless r2 is inside the pair's widened critical radius it returns hit = 0.
// Otherwise the pair is evaluated in FP64 from the FP64 state: -m_i w (Q_j - Q_i)
// goes to source jj's FP64 totals tot[jj], tot[T + jj], tot[2 T + jj], and the
// target's part m_j w (Q_j - Q_i) is returned (zero for a padded target).
__device__ __noinline__ ChgPart changeover_pair32(float r2, float r2j, const float4 *__restrict__ pk,
                                                  int i0, int li, int ni, int j0, uint32_t ja,
                                                  uint32_t a0, int T, double *tot,
                                                  const double *__restrict__ qx,
                                                  const double *__restrict__ qy,
                                                  const double *__restrict__ qz,
                                                  const double *__restrict__ m,
                                                  const double *__restrict__ rc, double inner,
                                                  const int *__restrict__ ord)
{
    ChgPart out{0.0, 0.0, 0.0, 0};
    const bool ok = li < ni;
    const int i = i0 + (ok ? li : 0);
    const int bi = ord ? ord[i] : i;
    if (!(r2 < max_nonneg(pk[2 * (size_t)bi + 1].w, r2j)))
        return out;
    out.hit = 1;
    const int jj = (int)((ja - a0) >> 4);
    const int bj = ord ? ord[j0 + jj] : j0 + jj;
    const double gx = qx[bj] - qx[bi], gy = qy[bj] - qy[bi], gz = qz[bj] - qz[bi];
    const double d2 = fma(gz, gz, fma(gy, gy, gx * gx));
    const double w = changeover_w_inl(d2, fmax(rc[bi], rc[bj]), inner);
    if (ok) {
        const double wi = m[bj] * w;
        out.x = wi * gx;
        out.y = wi * gy;
        out.z = wi * gz;
        const double wj = m[bi] * w;
        tot[jj] = fma(-wj, gx, tot[jj]);
        tot[T + jj] = fma(-wj, gy, tot[T + jj]);
        tot[2 * T + jj] = fma(-wj, gz, tot[2 * T + jj]);
    }
    return out;
}

// An FP64 term into a (hi, lo) FP32 accumulator: its leading float by two-sum,
// the float of the remainder into lo.
__device__ __forceinline__ void add_f64_to_pair(float &hi, float &lo, double v)
{
    const float vh = (float)v;
    two_sum_f(hi, lo, vh);
    lo += (float)(v - (double)vh);
}

// What the FP32C pair loop needs for the encounter test fused into it (sorted
// order): the sorted records, the step, and the list and flags to append to.
struct EncCtx {
    const SRec *srec;
    double dt;
    unsigned long long *keys;
    int cap;
    int *ce;
    DevStats *stats;
};

// Exact encounter test of two sorted positions, with the append of a flagged
// pair (defined with the encounter check).
__device__ __noinline__ void enc_candidate(const SRec *__restrict__ srec, double dt,
                                           unsigned long long *keys, int cap, int *ce,
                                           DevStats *stats, int pi, int pj);

// The tile of 64 R sources with, after the FP32C fields, each source's
// encounter records in FP32: chord midpoint M with the widened bound b' of
// 3/4 eps + rc (em), and chord c (ec).  The FP32C tile is a member, not a base:
// a base's tail padding may hold the derived members, while a member object
// keeps its whole size, so em[] starts exactly sizeof(SymTile32<T>) bytes after
// the tile's first record and ec[] 16 T bytes after that.
template <int T>
struct alignas(1024) SymTile32E {
    SymTile32<T> t;
    float4 em[T];
    float4 ec[T];
};
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winvalid-offsetof"
static_assert(offsetof(SymTile32E<64>, em) == sizeof(SymTile32<64>) &&
                  offsetof(SymTile32E<128>, em) == sizeof(SymTile32<128>) &&
                  offsetof(SymTile32E<256>, em) == sizeof(SymTile32<256>) &&
                  offsetof(SymTile32E<64>, ec) == sizeof(SymTile32<64>) + 16 * 64 &&
                  offsetof(SymTile32E<128>, ec) == sizeof(SymTile32<128>) + 16 * 128 &&
                  offsetof(SymTile32E<256>, ec) == sizeof(SymTile32<256>) + 16 * 256,
              "SymTile32E: em[] and ec[] right after the FP32C tile");
#pragma clang diagnostic pop

// ENC: the encounter test fused in (sorted order).  Target r of sub-tile t is
// tested against the sources when bit t R + r of `live` is set (the tile pair
// survived the culling): the relative-chord filter in FP32 (midpoints emi[r],
// chords eci[r] and the source's em, ec records), and the pairs that pass go to
// the exact test.  The source records are read from the LDS tile at fixed
// offsets past the FP32C fields (em, ec of SymTile32E).
// FAR: bit t of `far` set means every target of the wave lies apart from every
// source of sub-tile t by more than 2^21 times their low parts' norms and
// outside their critical radii (the radial tile bounds prove it): those pairs
// take the differences of the high parts alone, with no changeover test.
template <int R, bool DIAG, int T, bool ENC = false, bool FAR = false>
__device__ __forceinline__ void sym_tile32c(SymTile32<T> &L, int lane, int i0, int ni, int j0,
                                            double inner, const float4 *__restrict__ pk,
                                            const double *__restrict__ qx,
                                            const double *__restrict__ qy,
                                            const double *__restrict__ qz,
                                            const double *__restrict__ m,
                                            const double *__restrict__ rc, const float (&xh)[R],
                                            const float (&yh)[R], const float (&zh)[R],
                                            const float (&xl)[R], const float (&yl)[R],
                                            const float (&zl)[R], const float (&mi)[R], float tmi,
                                            float (&hx)[R], float (&hy)[R], float (&hz)[R],
                                            float (&lx)[R], float (&ly)[R], float (&lz)[R],
                                            int &near, const int *__restrict__ ord,
                                            const EncCtx &ec, const float4 (&emi)[R],
                                            const float4 (&eci)[R], unsigned live,
                                            unsigned far = 0u)
{
#pragma unroll 1
    for (int t = 0; t < R; ++t) {
        const bool fart = FAR && !DIAG && ((far >> t) & 1u);
        // the largest widened rc^2 of the wave's targets and of the sub-tile's
        // sources: one compare per pair outside the rare branch
        const float thr = max_nonneg(tmi, wave_max_nonneg(L.b[64 * t + lane].w));
        // targets of this wave that meet sub-tile t in a tile pair the culling kept
        const unsigned livet = ENC ? (live >> (t * R)) & ((1u << R) - 1u) : 0u;
#pragma unroll 1
        for (int half = 0; half < 2; ++half) {
            float tx[R], ty[R], tz[R];
#pragma unroll
            for (int r = 0; r < R; ++r)
                tx[r] = ty[r] = tz[r] = 0.0f;
            // Step k: lane L pairs its targets with source L xor k of sub-tile t,
            // so the lanes of a step touch distinct sources and each lane meets
            // every source once in 64 steps.  The run sum a step reads was
            // written by another lane one step earlier: LDS operations of a
            // wave complete in issue order, and the compiler barrier keeps the
            // read after that write.  Source records are read-only and fetched
            // one step ahead.
            const int k0 = 32 * half;
            const uint32_t a0 = lds_addr(&L.a[0]);
            const uint32_t self = lds_addr(&L.a[64 * t + lane]);
            uint32_t ac = self ^ (uint32_t)(k0 << 4);
            if (fart) {
                // far sub-tile: high parts only, no changeover test, no low
                // records read
                float4 A = lds_ld4(ac);
#pragma unroll 2
                for (int kk = 0; kk < 32; ++kk) {
                    const uint32_t an = self ^ (uint32_t)(((k0 + kk + 1) & 63) << 4);
                    const float4 An = lds_ld4(an);
                    const lds_v3f S = lds_ld3(ac + 32 * T);
                    float jx = S.x, jy = S.y, jz = S.z;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const float dx = A.x - xh[r], dy = A.y - yh[r], dz = A.z - zh[r];
                        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                        const float y = __builtin_amdgcn_rsqf(r2);
                        const float q = y * (y * y);
                        const float wi = A.w * q, wj = mi[r] * q;
                        tx[r] = fmaf(wi, dx, tx[r]);
                        ty[r] = fmaf(wi, dy, ty[r]);
                        tz[r] = fmaf(wi, dz, tz[r]);
                        jx = fmaf(-wj, dx, jx);
                        jy = fmaf(-wj, dy, jy);
                        jz = fmaf(-wj, dz, jz);
                    }
                    lds_st3(ac + 32 * T, jx, jy, jz);
                    __asm__ __volatile__("" ::: "memory");
                    ac = an;
                    A = An;
                }
            } else {
            float4 A = lds_ld4(ac), B = lds_ld4(ac + 16 * T);
#pragma unroll 2
            for (int kk = 0; kk < 32; ++kk) {
                const uint32_t an = self ^ (uint32_t)(((k0 + kk + 1) & 63) << 4);
                const float4 An = lds_ld4(an), Bn = lds_ld4(an + 16 * T);
                const lds_v3f S = lds_ld3(ac + 32 * T);
                float jx = S.x, jy = S.y, jz = S.z;
                // the R pairs' geometry first, then one branch for the rare
                // ones, so that the R chains share one basic block
                float dxr[R], dyr[R], dzr[R], r2r[R], qr[R];
                bool cand = false;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    dxr[r] = (A.x - xh[r]) + (B.x - xl[r]);
                    dyr[r] = (A.y - yh[r]) + (B.y - yl[r]);
                    dzr[r] = (A.z - zh[r]) + (B.z - zl[r]);
                    r2r[r] = fmaf(dzr[r], dzr[r], fmaf(dyr[r], dyr[r], dxr[r] * dxr[r]));
                    const float y = __builtin_amdgcn_rsqf(r2r[r]);
                    qr[r] = y * (y * y);
                    const bool on = !DIAG || (64 * r + lane < 64 * t + (lane ^ (k0 + kk)));
                    cand |= r2r[r] < thr && on;
                    if (DIAG)
                        qr[r] = on ? qr[r] : 0.0f;
                }
                // fused encounter test: the relative-chord filter in FP32,
                // |dM|^2 <= 2 (|dc|^2 + (b'_i + b'_j + max(rc_i, rc_j))^2) with
                // the bounds b' widened for the FP32 rounding (padded targets
                // and sources carry NaN midpoints and never pass; every body is
                // big on this path, so no b' carries the small-body sign)
                bool encr[R] = {};
                bool ecand = false;
                if (ENC && livet) {
                    const float4 E = lds_ld4(ac + (uint32_t)sizeof(SymTile32<T>));
                    const float4 F = lds_ld4(ac + (uint32_t)(sizeof(SymTile32<T>) + 16 * T));
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const float ex = E.x - emi[r].x, ey = E.y - emi[r].y, ez = E.z - emi[r].z;
                        const float cx = F.x - eci[r].x, cy = F.y - eci[r].y, cz = F.z - eci[r].z;
                        const float D2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
                        const float C2 = fmaf(cz, cz, fmaf(cy, cy, cx * cx));
                        const float Sr = (E.w + emi[r].w) + fmaxf(F.w, eci[r].w);
                        const bool on = !DIAG || (64 * r + lane < 64 * t + (lane ^ (k0 + kk)));
                        encr[r] = ((livet >> r) & 1u) && on &&
                                  D2 <= fmaf(Sr, Sr, C2) * (2.0f * (1.0f + 0x1p-18f));
                        ecand |= encr[r];
                    }
                }
                if (cand || ecand) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const bool on = !DIAG || (64 * r + lane < 64 * t + (lane ^ (k0 + kk)));
                        if (r2r[r] < thr && on) {
                            const ChgPart c = changeover_pair32(r2r[r], B.w, pk, i0, 64 * r + lane,
                                                                ni, j0, ac, a0, T, L.ax, qx, qy,
                                                                qz, m, rc, inner, ord);
                            if (c.hit) {
                                add_f64_to_pair(hx[r], lx[r], c.x);
                                add_f64_to_pair(hy[r], ly[r], c.y);
                                add_f64_to_pair(hz[r], lz[r], c.z);
                                qr[r] = 0.0f;
                                ++near;
                            }
                        }
                        if (ENC && encr[r])
                            enc_candidate(ec.srec, ec.dt, ec.keys, ec.cap, ec.ce, ec.stats,
                                          i0 + 64 * r + lane, j0 + (int)((ac - a0) >> 4));
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float dx = dxr[r], dy = dyr[r], dz = dzr[r], q = qr[r];
                    const float wi = A.w * q, wj = mi[r] * q;
                    tx[r] = fmaf(wi, dx, tx[r]);
                    ty[r] = fmaf(wi, dy, ty[r]);
                    tz[r] = fmaf(wi, dz, tz[r]);
                    jx = fmaf(-wj, dx, jx);
                    jy = fmaf(-wj, dy, jy);
                    jz = fmaf(-wj, dz, jz);
                }
                lds_st3(ac + 32 * T, jx, jy, jz);
                __asm__ __volatile__("" ::: "memory");
                ac = an;
                A = An;
                B = Bn;
            }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                two_sum_f(hx[r], lx[r], tx[r]);
                two_sum_f(hy[r], ly[r], ty[r]);
                two_sum_f(hz[r], lz[r], tz[r]);
            }
            // end of the run: every source of sub-tile t had its 32 steps; lane
            // L moves source 64 t + L's run sum into its FP64 total
            const int js = 64 * t + lane;
            const float4 S = L.run[js];
            L.ax[js] += (double)S.x;
            L.ay[js] += (double)S.y;
            L.az[js] += (double)S.z;
            L.run[js] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            __asm__ __volatile__("" ::: "memory");
        }
    }
}

// Two 64-body tiles of the radial order are far apart for the FP32C pair loop
// when the gap between their shells, |xh_i| in [rmin, rmax] (records written
// by k_sun_drift with the FP32C records), exceeds 2^21 times the sum of their low parts' largest norms
// and its square exceeds both largest widened rc^2.  Then for i in one and j in
// the other |xh_j - xh_i| >= gap: dropping the low parts moves the pair's
// difference by at most 2^-21 of its length, and the pair lies outside the
// changeover zone (weight 1, no rare branch).  Margins of 2^-20 and 2^-18 cover
// the FP32 rounding of the test itself.
__device__ __forceinline__ bool far_tiles(float4 a, float4 b)
{
    const float gap = fmaxf(b.x - a.y, a.x - b.y) * (1.0f - 0x1p-20f);
    return gap >= 0x1p21f * (a.z + b.z) * (1.0f + 0x1p-20f) &&
           gap * gap >= fmaxf(a.w, b.w) * (1.0f + 0x1p-18f);
}

// SORT: the positions of the work items are positions of the radial order
// (ord: position -> body), whose tile bounds rtb (system s's tiles from
// rtf[s], 64 positions each from off[s]) mark the far sub-tile pairs.
template <int R, int G, bool SORT = false>
__global__ __launch_bounds__(64 * G, R == 4 ? 2 : 3) void k_force32c_sym(const FWork *__restrict__ work, int nitems,
                                                         const float4 *__restrict__ pk,
                                                         const double *__restrict__ qx,
                                                         const double *__restrict__ qy,
                                                         const double *__restrict__ qz,
                                                         const double *__restrict__ m,
                                                         const double *__restrict__ rc,
                                                         float *__restrict__ fpart, int ntot,
                                                         int maxs, double inner, DevStats *stats,
                                                         const int *__restrict__ ord = nullptr,
                                                         const float4 *__restrict__ rtb = nullptr,
                                                         const int *__restrict__ rtf = nullptr,
                                                         const int *__restrict__ off = nullptr)
{
    constexpr int T = 64 * R;
    __shared__ SymTile32<T> tl[G];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const size_t plane = (size_t)maxs * ntot;
    int near = 0;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const FWork wk = work[it];
        const bool diag = wk.i0 == wk.j0;
        // the G source tiles of super-tile J (nj real records from j0)
        for (int k = threadIdx.x; k < G * T; k += 64 * G) {
            SymTile32<T> &S = tl[k / T];
            const int e = k % T;
            // sources past the end: massless and far away (r^2 ~ 1e36, so the
            // weight underflows to 0 instead of meeting a target at r = 0)
            if (k < wk.nj) {
                const int b = SORT ? ord[wk.j0 + k] : wk.j0 + k;
                S.a[e] = pk[2 * (size_t)b];
                S.b[e] = pk[2 * (size_t)b + 1];
            } else {
                S.a[e] = make_float4(1e18f, 1e18f, 1e18f, 0.0f);
                S.b[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
            S.run[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            S.ax[e] = S.ay[e] = S.az[e] = 0.0;
        }
        __syncthreads();
        // this wave's target tile: tni bodies from ti0 (none when tni <= 0)
        const int ti0 = wk.i0 + wv * T;
        const int tni = min(T, wk.ni - wv * T);
        float xh[R], yh[R], zh[R], xl[R], yl[R], zl[R], mi[R];
        float hx[R], hy[R], hz[R], lx[R], ly[R], lz[R];
        float tmi = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int li = 64 * r + lane;
            const bool ok = li < tni;
            const int i = SORT ? ord[ok ? ti0 + li : wk.i0] : (ok ? ti0 + li : wk.i0);
            const float4 A = pk[2 * (size_t)i], B = pk[2 * (size_t)i + 1];
            xh[r] = A.x; yh[r] = A.y; zh[r] = A.z;
            xl[r] = B.x; yl[r] = B.y; zl[r] = B.z;
            // targets past the tile end are massless: they add nothing to the sources
            mi[r] = ok ? A.w : 0.0f;
            tmi = max_nonneg(tmi, B.w);
            hx[r] = hy[r] = hz[r] = lx[r] = ly[r] = lz[r] = 0.0f;
        }
        tmi = wave_max_nonneg(tmi);
        const EncCtx noenc{};
        float4 noem[R];
        // Round k: wave w pairs its target tile with source tile (w + k) mod G, so
        // that the waves of a round update distinct source tiles.  Off the
        // diagonal G rounds cover the G x G tile pairs.  On the diagonal (I = J)
        // round 0 takes the pairs inside each tile, rounds 1 .. G/2 - 1 every
        // other tile pair once, and round G/2 (even G) only its first G/2 waves,
        // whose partners the other half would meet again.
        const int nr = diag ? G / 2 + 1 : G;
        for (int k = 0; k < nr; ++k) {
            const int s = (wv + k) % G;
            const bool go = tni > 0 && s * T < wk.nj && !(diag && 2 * k == G && wv >= G / 2);
            if (go) {
                if (diag && k == 0) {
                    sym_tile32c<R, true, T>(tl[s], lane, ti0, tni, wk.j0 + s * T, inner, pk, qx,
                                            qy, qz, m, rc, xh, yh, zh, xl, yl, zl, mi, tmi, hx, hy,
                                            hz, lx, ly, lz, near, SORT ? ord : nullptr, noenc, noem,
                                            noem, 0u);
                } else {
                    // far source sub-tiles (radial order, no padded targets)
                    unsigned far = 0u;
                    if (SORT && tni == T) {
                        const int tb0 = rtf[wk.sys], o = off[wk.sys], sj0 = wk.j0 + s * T;
#pragma unroll
                        for (int t = 0; t < R; ++t) {
                            if (s * T + 64 * t >= wk.nj)
                                continue;
                            const float4 Bt = rtb[tb0 + (sj0 + 64 * t - o) / 64];
                            bool f = true;
#pragma unroll
                            for (int r = 0; r < R; ++r)
                                f = f && far_tiles(rtb[tb0 + (ti0 + 64 * r - o) / 64], Bt);
                            far |= f ? 1u << t : 0u;
                        }
                    }
                    sym_tile32c<R, false, T, false, SORT>(tl[s], lane, ti0, tni, wk.j0 + s * T,
                                                          inner, pk, qx, qy, qz, m, rc, xh, yh, zh,
                                                          xl, yl, zl, mi, tmi, hx, hy, hz, lx, ly,
                                                          lz, near, SORT ? ord : nullptr, noenc,
                                                          noem, noem, 0u, far);
                }
            }
            __syncthreads();
        }
        // super-tile I's sums to slot J (on the diagonal together with the same
        // bodies' sums as sources)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int li = 64 * r + lane;
            if (li < tni) {
                const int i = ti0 + li;
                double sx_ = (double)hx[r] + (double)lx[r];
                double sy_ = (double)hy[r] + (double)ly[r];
                double sz_ = (double)hz[r] + (double)lz[r];
                if (diag) {
                    sx_ += tl[wv].ax[li];
                    sy_ += tl[wv].ay[li];
                    sz_ += tl[wv].az[li];
                }
                fpart[(size_t)wk.slot * ntot + i] = (float)sx_;
                fpart[plane + (size_t)wk.slot * ntot + i] = (float)sy_;
                fpart[2 * plane + (size_t)wk.slot * ntot + i] = (float)sz_;
            }
        }
        if (!diag) {
            // super-tile J's sums to slot I
            for (int k = threadIdx.x; k < wk.nj; k += 64 * G) {
                const SymTile32<T> &S = tl[k / T];
                const int e = k % T, j = wk.j0 + k;
                fpart[((size_t)0 * maxs + wk.pad) * ntot + j] = (float)S.ax[e];
                fpart[((size_t)1 * maxs + wk.pad) * ntot + j] = (float)S.ay[e];
                fpart[((size_t)2 * maxs + wk.pad) * ntot + j] = (float)S.az[e];
            }
        }
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1)
        near += __shfl_xor(near, o);
    if (lane == 0 && near)
        atomicAdd((unsigned long long *)&stats->near_pairs, (unsigned long long)near);
}

// a = G * sum over the body's split partials (fixed order); optionally `kicks`
// (1 or 2) kicks V += h a, rounded as that many k_kick launches.  A workgroup of
// kFinThreads threads takes B = kFinThreads / nsl bodies: thread group g (B
// threads) reads slice g of every body's partials (slots [g ns / nsl, (g + 1) ns
// / nsl) in order, eight loads in flight per lane), and the slice sums are added
// in slice order.  nsl (a power of two, at most 16) follows the largest split
// count, so that few-split systems do not leave most threads idle.  The sums of
// m V are not needed after it: the next S(h) takes the momentum from before the
// kicks.
constexpr int kFinThreads = 1024;

template <typename P>
__global__ __launch_bounds__(kFinThreads) void k_force_finalize(
    const int *__restrict__ sys_of, const int *__restrict__ nsplit, const P *__restrict__ fpart,
    int ntot, int maxs, int ns_all, int nsl, double G, double *__restrict__ ax,
    double *__restrict__ ay, double *__restrict__ az, double h, int kicks, double *vx, double *vy,
    double *vz, const int *__restrict__ ord, int count_cap, DevStats *stats)
{
    __shared__ double gs[3 * kFinThreads];
    // count_cap >= 0: also the encounter list's statistics (as k_enc_count), for
    // the check that ran inside the force pass before this launch
    if (count_cap >= 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        const int count = stats->cur_nce;
        stats->total_nce += count;
        if (count > stats->max_nce)
            stats->max_nce = count;
        if (count > count_cap)
            stats->overflow_steps += 1;
    }
    const int B = kFinThreads / nsl;
    const int t = threadIdx.x % B, g = threadIdx.x / B;
    // i: the partials' position; bi: the body (the sorted order maps them)
    const int i = blockIdx.x * B + t;
    const int bi = ord && i < ntot ? ord[i] : i;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    // the velocities to kick, fetched while the partials load
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    if (g == 0 && i < ntot && h != 0.0) {
        v0 = vx[bi];
        v1 = vy[bi];
        v2 = vz[bi];
    }
    if (i < ntot) {
        // ns_all != 0: every system has that split count
        const int ns = ns_all ? ns_all : nsplit[sys_of[i]];
        const int k0 = g * ns / nsl, k1 = (g + 1) * ns / nsl;
        const P *px = fpart + i, *py = px + (size_t)maxs * ntot, *pz = py + (size_t)maxs * ntot;
        int k = k0;
        for (; k + 8 <= k1; k += 8) {
            P ux[8], uy[8], uz[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                ux[u] = px[(size_t)(k + u) * ntot];
                uy[u] = py[(size_t)(k + u) * ntot];
                uz[u] = pz[(size_t)(k + u) * ntot];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                s0 += (double)ux[u];
                s1 += (double)uy[u];
                s2 += (double)uz[u];
            }
        }
        for (; k < k1; ++k) {
            s0 += (double)px[(size_t)k * ntot];
            s1 += (double)py[(size_t)k * ntot];
            s2 += (double)pz[(size_t)k * ntot];
        }
    }
    if (g > 0) {
        double *o = gs + (size_t)(g - 1) * 3 * B;
        o[t] = s0;
        o[B + t] = s1;
        o[2 * B + t] = s2;
    }
    __syncthreads();
    if (g == 0 && i < ntot) {
        for (int q = 0; q < nsl - 1; ++q) {
            const double *o = gs + (size_t)q * 3 * B;
            s0 += o[t];
            s1 += o[B + t];
            s2 += o[2 * B + t];
        }
        s0 *= G;
        s1 *= G;
        s2 *= G;
        ax[bi] = s0;
        ay[bi] = s1;
        az[bi] = s2;
        if (h != 0.0) {
            double u0 = fma(h, s0, v0), u1 = fma(h, s1, v1), u2 = fma(h, s2, v2);
            if (kicks == 2) {
                u0 = fma(h, s0, u0);
                u1 = fma(h, s1, u1);
                u2 = fma(h, s2, u2);
            }
            vx[bi] = u0;
            vy[bi] = u1;
            vz[bi] = u2;
        }
    }
}

// ----------------------------------------------------------------------------
// Encounter check (Sec. 3.1, encounter block): every pair i<j of a system
// whose minimum separation over the step is <= rc_ij = max(rc_i, rc_j).  The
// squared separation over s in [0,1] is taken as the cubic Hermite through
// f0 = |dQ0|^2, f1 = |dQ1|^2 with slopes g0 = 2 dt dQ0.dV0, g1 = 2 dt dQ1.dV1.
// Its minimum is bounded below by min(f0,f1) - 4/27 (max(0,-g0) + max(0,g1)),
// which serves as a cheap conservative filter before the exact minimum.
// ----------------------------------------------------------------------------
__device__ double hermite_min(double f0, double f1, double g0, double g1)
{
    double b = 3.0 * (f1 - f0) - 2.0 * g0 - g1;   // s^2 coefficient
    double c = 2.0 * (f0 - f1) + g0 + g1;         // s^3 coefficient
    double best = fmin(f0, f1);
    // f'(s) = g0 + 2 b s + 3 c s^2
    double A = 3.0 * c, B = 2.0 * b, C = g0;
    double s1 = -1.0, s2 = -1.0;
    if (A != 0.0) {
        double disc = B * B - 4.0 * A * C;
        if (disc >= 0.0) {
            double q = -0.5 * (B + copysign(sqrt(disc), B));
            if (q != 0.0) {
                s1 = q / A;
                s2 = C / q;
            }
        }
    } else if (B != 0.0) {
        s1 = -C / B;
    }
    if (s1 > 0.0 && s1 < 1.0)
        best = fmin(best, f0 + s1 * (g0 + s1 * (b + s1 * c)));
    if (s2 > 0.0 && s2 < 1.0)
        best = fmin(best, f0 + s2 * (g0 + s2 * (b + s2 * c)));
    return fmax(best, 0.0);
}

struct EncRec {
    double q0[3], v0[3], q1[3], v1[3];
    double rc, pad;
};

// Two-stage pair test, one target per lane, sources broadcast from LDS.
// Stage 1 (every pair): chord midpoints M and reaches R (from the drift).  The
// Hermite data split into the straight-chord part |dQ0 + s dc|^2 (which the
// cubic reproduces exactly and which is >= (D - rho_i - rho_j)^2, D = |dM|)
// and the endpoint velocity deviations e = dt V - c, weighted by h10(s) and
// h11(s) with |h10| + |h11| = s(1-s) <= 1/4.  So
// f(s) >= (D-P)^2 - (1/2)(D+P)E with P = rho_i + rho_j, E = eps_i + eps_j,
// which exceeds (rc_i + rc_j)^2 >= rc_ij^2 whenever D > R_i + R_j with
// R = 2 rho + 3 eps/4 + rc.  So only pairs with |dM|^2 <= (R_i + R_j)^2 go on.
// Stage 1b (relative chords): the same split around the relative chord dc =
// c_j - c_i gives f(s) >= (D - a)^2 - (1/2)(D + a)E with a = |dc|/2, which
// exceeds rc_ij^2 whenever D > |dc| + 3E/4 + rc_ij; as (x + y)^2 <= 2x^2 + 2y^2,
// pairs with D^2 > 2|dc|^2 + 2(3E/4 + rc_ij)^2 are dropped.  Bodies moving
// together (neighbours on similar orbits) have short relative chords, so this
// keeps far fewer pairs than stage 1 when steps are long.  The 3/4 eps term
// stored per body is widened by 2^-20 and by 2^-45 (|M| + |c|) for the rounding
// of the differences.
// Stage 2 (candidates): the 4/27 lower bound on the full Hermite data, then
// the exact minimum.
__global__ __launch_bounds__(kBlock) void k_encounter(const PWork *__restrict__ work, double dt,
                                                      const double4 *__restrict__ mr,
                                                      const double4 *__restrict__ cr,
                                                      const double *__restrict__ q0x,
                                                      const double *__restrict__ q0y,
                                                      const double *__restrict__ q0z,
                                                      const double *__restrict__ v0x,
                                                      const double *__restrict__ v0y,
                                                      const double *__restrict__ v0z,
                                                      const double *__restrict__ qx,
                                                      const double *__restrict__ qy,
                                                      const double *__restrict__ qz,
                                                      const double *__restrict__ vx,
                                                      const double *__restrict__ vy,
                                                      const double *__restrict__ vz,
                                                      const double *__restrict__ rc,
                                                      unsigned long long *__restrict__ keys,
                                                      int cap, int *__restrict__ ce,
                                                      DevStats *stats)
{
    __shared__ double4 smr[kBlock];
    __shared__ double4 scr[kBlock];
    __shared__ EncRec sj[kBlock];
    const PWork wk = work[blockIdx.x];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const double t2 = 2.0 * dt;
    const double k427 = 4.0 / 27.0;
    const bool has_i = t < wk.ni;
    const int i = wk.i0 + (has_i ? t : 0);
    const double4 Mi = mr[i];
    const double4 Ci = cr[i];
    const double a0[3] = {q0x[i], q0y[i], q0z[i]}, b0[3] = {v0x[i], v0y[i], v0z[i]};
    const double a1[3] = {qx[i], qy[i], qz[i]}, b1[3] = {vx[i], vy[i], vz[i]};
    const double rci = rc[i];
    const int jend = wk.j0 + wk.nj;
    for (int jt = wk.j0; jt < jend; jt += kBlock) {
        const int cnt = min(kBlock, jend - jt);
        __syncthreads();
        if (t < cnt) {
            int j = jt + t;
            smr[t] = mr[j];
            scr[t] = cr[j];
            EncRec r;
            r.q0[0] = q0x[j]; r.q0[1] = q0y[j]; r.q0[2] = q0z[j];
            r.v0[0] = v0x[j]; r.v0[1] = v0y[j]; r.v0[2] = v0z[j];
            r.q1[0] = qx[j];  r.q1[1] = qy[j];  r.q1[2] = qz[j];
            r.v1[0] = vx[j];  r.v1[1] = vy[j];  r.v1[2] = vz[j];
            r.rc = rc[j];
            r.pad = 0.0;
            sj[t] = r;
        }
        __syncthreads();
        // only tiles that reach past the target index hold pairs j > i
        const bool diag = jt < wk.i0 + wk.ni;
        for (int jj = 0; jj < cnt; ++jj) {
            const int j = jt + jj;
            const double4 Mj = smr[jj];
            double dx = Mj.x - Mi.x, dy = Mj.y - Mi.y, dz = Mj.z - Mi.z;
            double D2 = fma(dz, dz, fma(dy, dy, dx * dx));
            double S = Mi.w + Mj.w;
            bool cand = has_i && D2 <= S * S && (!diag || j > i);
            if (!__any(cand))
                continue;
            {
                // relative chord filter
                const double4 Cj = scr[jj];
                double cx = Cj.x - Ci.x, cy = Cj.y - Ci.y, cz = Cj.z - Ci.z;
                double C2 = fma(cz, cz, fma(cy, cy, cx * cx));
                double bb = Ci.w + Cj.w + fmax(rci, sj[jj].rc);
                cand = cand && D2 <= fma(2.0, C2, 2.0 * bb * bb) * (1.0 + 0x1p-20);
            }
            if (!__any(cand))
                continue;
            bool hit = false;
            if (cand) {
                const EncRec &J = sj[jj];
                double d0x = J.q0[0] - a0[0], d0y = J.q0[1] - a0[1], d0z = J.q0[2] - a0[2];
                double d1x = J.q1[0] - a1[0], d1y = J.q1[1] - a1[1], d1z = J.q1[2] - a1[2];
                double e0x = J.v0[0] - b0[0], e0y = J.v0[1] - b0[1], e0z = J.v0[2] - b0[2];
                double e1x = J.v1[0] - b1[0], e1y = J.v1[1] - b1[1], e1z = J.v1[2] - b1[2];
                double f0 = fma(d0z, d0z, fma(d0y, d0y, d0x * d0x));
                double f1 = fma(d1z, d1z, fma(d1y, d1y, d1x * d1x));
                double g0 = t2 * fma(d0z, e0z, fma(d0y, e0y, d0x * e0x));
                double g1 = t2 * fma(d1z, e1z, fma(d1y, e1y, d1x * e1x));
                double lower = fmin(f0, f1) - k427 * (fmax(0.0, -g0) + fmax(0.0, g1));
                double rcij = fmax(rci, J.rc);
                double thr = rcij * rcij;
                if (lower <= thr * (1.0 + 1e-6) + 1e-15 * (f0 + f1 + fabs(g0) + fabs(g1)))
                    hit = hermite_min(f0, f1, g0, g1) <= thr;
            }
            unsigned long long mask = __ballot(hit);
            if (mask) {
                int leader = __ffsll((long long)mask) - 1;
                int base = 0;
                if (lane == leader)
                    base = atomicAdd(&stats->cur_nce, (int)__popcll(mask));
                base = __shfl(base, leader);
                if (hit) {
                    unsigned long long below = mask & ((1ull << lane) - 1ull);
                    int pos = base + (int)__popcll(below);
                    if (pos < cap)
                        keys[pos] = ((unsigned long long)(unsigned)i << 32) | (unsigned)j;
                    __hip_atomic_store(&ce[i], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&ce[j], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
}

// Few big bodies (every system has at most kBlock big bodies; small bodies are
// massless and never meet each other): one lane per body j of an O(N) block,
// tested against the big bodies i < j of its system, which the block stages in
// LDS once.  Same two-stage pair test as k_encounter, so the same pairs are
// flagged.
__global__ __launch_bounds__(kBlock) void k_encounter_few(const RBlk *__restrict__ rblk,
                                                          const int *__restrict__ off,
                                                          const int *__restrict__ nbig, double dt,
                                                          const double4 *__restrict__ mr,
                                                          const double4 *__restrict__ cr,
                                                          const double *__restrict__ q0x,
                                                          const double *__restrict__ q0y,
                                                          const double *__restrict__ q0z,
                                                          const double *__restrict__ v0x,
                                                          const double *__restrict__ v0y,
                                                          const double *__restrict__ v0z,
                                                          const double *__restrict__ qx,
                                                          const double *__restrict__ qy,
                                                          const double *__restrict__ qz,
                                                          const double *__restrict__ vx,
                                                          const double *__restrict__ vy,
                                                          const double *__restrict__ vz,
                                                          const double *__restrict__ rc,
                                                          unsigned long long *__restrict__ keys,
                                                          int cap, int *__restrict__ ce,
                                                          DevStats *stats)
{
    __shared__ double4 smr[kBlock];
    __shared__ double4 scr[kBlock];
    __shared__ EncRec si[kBlock];
    const RBlk b = rblk[blockIdx.x];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int a = off[b.sys], nb = min(nbig[b.sys], kBlock);
    const double t2 = 2.0 * dt;
    const double k427 = 4.0 / 27.0;
    // the system's big bodies
    if (t < nb) {
        const int i = a + t;
        smr[t] = mr[i];
        scr[t] = cr[i];
        EncRec r;
        r.q0[0] = q0x[i]; r.q0[1] = q0y[i]; r.q0[2] = q0z[i];
        r.v0[0] = v0x[i]; r.v0[1] = v0y[i]; r.v0[2] = v0z[i];
        r.q1[0] = qx[i];  r.q1[1] = qy[i];  r.q1[2] = qz[i];
        r.v1[0] = vx[i];  r.v1[1] = vy[i];  r.v1[2] = vz[i];
        r.rc = rc[i];
        r.pad = 0.0;
        si[t] = r;
    }
    __syncthreads();
    const bool has_j = b.start + t < b.end;
    const int j = b.start + (has_j ? t : 0);
    const int ni = has_j ? min(nb, j - a) : 0;     // big bodies i < j
    const double4 Mj = mr[j];
    const double4 Cj = cr[j];
    const double a0[3] = {q0x[j], q0y[j], q0z[j]}, b0[3] = {v0x[j], v0y[j], v0z[j]};
    const double a1[3] = {qx[j], qy[j], qz[j]}, b1[3] = {vx[j], vy[j], vz[j]};
    const double rcj = rc[j];
    for (int ii = 0; ii < nb; ++ii) {
        const double4 Mi = smr[ii];
        const double dx = Mj.x - Mi.x, dy = Mj.y - Mi.y, dz = Mj.z - Mi.z;
        const double D2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const double S = Mi.w + Mj.w;
        bool cand = ii < ni && D2 <= S * S;
        if (!__any(cand))
            continue;
        {
            // relative chord filter
            const double4 Ci = scr[ii];
            const double cx = Cj.x - Ci.x, cy = Cj.y - Ci.y, cz = Cj.z - Ci.z;
            const double C2 = fma(cz, cz, fma(cy, cy, cx * cx));
            const double bb = Ci.w + Cj.w + fmax(si[ii].rc, rcj);
            cand = cand && D2 <= fma(2.0, C2, 2.0 * bb * bb) * (1.0 + 0x1p-20);
        }
        if (!__any(cand))
            continue;
        bool hit = false;
        if (cand) {
            const EncRec &I = si[ii];
            const double d0x = a0[0] - I.q0[0], d0y = a0[1] - I.q0[1], d0z = a0[2] - I.q0[2];
            const double d1x = a1[0] - I.q1[0], d1y = a1[1] - I.q1[1], d1z = a1[2] - I.q1[2];
            const double e0x = b0[0] - I.v0[0], e0y = b0[1] - I.v0[1], e0z = b0[2] - I.v0[2];
            const double e1x = b1[0] - I.v1[0], e1y = b1[1] - I.v1[1], e1z = b1[2] - I.v1[2];
            const double f0 = fma(d0z, d0z, fma(d0y, d0y, d0x * d0x));
            const double f1 = fma(d1z, d1z, fma(d1y, d1y, d1x * d1x));
            const double g0 = t2 * fma(d0z, e0z, fma(d0y, e0y, d0x * e0x));
            const double g1 = t2 * fma(d1z, e1z, fma(d1y, e1y, d1x * e1x));
            const double lower = fmin(f0, f1) - k427 * (fmax(0.0, -g0) + fmax(0.0, g1));
            const double rcij = fmax(I.rc, rcj);
            const double thr = rcij * rcij;
            if (lower <= thr * (1.0 + 1e-6) + 1e-15 * (f0 + f1 + fabs(g0) + fabs(g1)))
                hit = hermite_min(f0, f1, g0, g1) <= thr;
        }
        const unsigned long long mask = __ballot(hit);
        if (mask) {
            const int leader = __ffsll((long long)mask) - 1;
            int base = 0;
            if (lane == leader)
                base = atomicAdd(&stats->cur_nce, (int)__popcll(mask));
            base = __shfl(base, leader);
            if (hit) {
                const int i = a + ii;
                const int pos = base + (int)__popcll(mask & ((1ull << lane) - 1ull));
                if (pos < cap)
                    keys[pos] = ((unsigned long long)(unsigned)i << 32) | (unsigned)j;
                __hip_atomic_store(&ce[i], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ce[j], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Spatially sorted encounter check.  Each step the bodies of every system are
// binned by the chord midpoint's cylindrical (ln R, phi) into a power-of-two
// grid of about N_s/8 cells traversed in Morton order, counting-sorted, and
// cut into tiles of 64 consecutive bodies.  A tile carries the centre and
// radius of its chord midpoints M, chords c and endpoint velocity deviations
// e = dt V - c.  For i in tile A and j in tile B the Hermite data split into
// the chord quadratic |dM + (s - 1/2) dc|^2 and the deviations weighted by
// |h10| + |h11| = s(1-s) <= 1/4 give f(s) >= Lmin^2 - Qmax Em / 2 with
//   Lmin = D - sm_A - sm_B - Cm/2,  Qmax = D + sm_A + sm_B + Cm/2,
//   D = |cm_B - cm_A|, Cm = |cc_B - cc_A| + sc_A + sc_B, Em = |ce_B - ce_A| + se_A + se_B,
// so a tile pair whose bound exceeds max rc^2 holds no flagged pair.  Surviving
// tile pairs are tested pair by pair exactly as in k_encounter.  The bodies of
// a cell are put in index order after the binning, so the sorted order does
// not depend on the timing of its atomics; the output list is sorted.
// ----------------------------------------------------------------------------
__device__ __forceinline__ unsigned morton2(unsigned band, int nb, unsigned pb, int np)
{
    unsigned code = 0;
    int k = 0, bit = 0;
    for (; k < nb || k < np; ++k) {
        if (k < np)
            code |= ((pb >> k) & 1u) << bit++;
        if (k < nb)
            code |= ((band >> k) & 1u) << bit++;
    }
    return code;
}

__global__ void k_cells(const RBlk *__restrict__ rblk, const int *__restrict__ rb_first,
                        const int *__restrict__ rb_count, const double *__restrict__ lnr_part,
                        const int *__restrict__ sys_cell_base, const int *__restrict__ sys_cell_cnt,
                        const double4 *__restrict__ mr, int *__restrict__ cell_cnt,
                        int *__restrict__ cell_of, int *__restrict__ slot_of, int *__restrict__ ce)
{
    __shared__ double sh[2 * kBlock];
    const RBlk b = rblk[blockIdx.x];
    // ln R range of the whole system, from its blocks' partials
    double lo = INFINITY, hi = -INFINITY;
    for (int k = threadIdx.x; k < rb_count[b.sys]; k += kBlock) {
        lo = fmin(lo, lnr_part[2 * (size_t)(rb_first[b.sys] + k)]);
        hi = fmax(hi, lnr_part[2 * (size_t)(rb_first[b.sys] + k) + 1]);
    }
    sh[threadIdx.x] = lo;
    sh[kBlock + threadIdx.x] = hi;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + st]);
            sh[kBlock + threadIdx.x] = fmax(sh[kBlock + threadIdx.x], sh[kBlock + threadIdx.x + st]);
        }
        __syncthreads();
    }
    lo = sh[0];
    hi = sh[kBlock];
    const int C = sys_cell_cnt[b.sys];          // power of two
    int lc = 31 - __clz(C);
    // bands B x phi bins P = C with square cells in (ln R, phi): B ~ sqrt(C span / 2 pi)
    const double span = fmax(hi - lo, 0.0);
    int lb = 0;
    double bstar = sqrt((double)C * span / 6.283185307179586);
    if (bstar > 1.0)
        lb = min(lc, (int)floor(log2(bstar) + 0.5));
    const int lp = lc - lb;
    const int i = b.start + threadIdx.x;
    if (i < b.end) {
        double4 M = mr[i];
        double R = sqrt(M.x * M.x + M.y * M.y);
        double lnr = log(fmax(R, 1e-300));
        unsigned band = 0, pb = 0;
        if (span > 0.0)
            band = (unsigned)min((1 << lb) - 1, max(0, (int)((lnr - lo) / span * (double)(1 << lb))));
        double phi = atan2(M.y, M.x);
        pb = (unsigned)min((1 << lp) - 1, max(0, (int)((phi + 3.141592653589793) *
                                                      (0.15915494309189535 * (double)(1 << lp)))));
        int cell = sys_cell_base[b.sys] + (int)morton2(band, lb, pb, lp);
        cell_of[i] = cell;
        slot_of[i] = atomicAdd(&cell_cnt[cell], 1);
        // no encounter flag yet (the check of this drift sets them)
        ce[i] = 0;
    }
}

// Exclusive scan of the cell counts (one workgroup), zeroing them for the next
// step, and reset of the surviving-tile-pair counter.
// 256 threads (one wave per SIMD): blocks this small still find room on a CU
// beside the force pass's waves, so the encounter check's scan need not wait
// for the force pass to drain a whole CU.
constexpr int kScanThreads = 256;
constexpr int kScanChunk = kScanChunkCells;    // cells per block pass, 4 per thread
static_assert(kScanChunk == 4 * kScanThreads, "four cells per scan thread");

// Exclusive scan over the kScanThreads threads of a block; *total gets the sum.
__device__ __forceinline__ int block_exscan(int v, int *sh, int &total)
{
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o)
            x += y;
    }
    if (lane == 63)
        sh[wv] = x;
    __syncthreads();
    if (t < 64) {
        int w = t < kScanThreads / 64 ? sh[t] : 0;
        for (int o = 1; o < 64; o <<= 1) {
            int y = __shfl_up(w, o);
            if (lane >= o)
                w += y;
        }
        if (t < kScanThreads / 64)
            sh[32 + t] = w;               // inclusive wave totals
    }
    __syncthreads();
    total = sh[32 + kScanThreads / 64 - 1];
    const int before = wv > 0 ? sh[32 + wv - 1] : 0;
    __syncthreads();                      // sh is reused by the next call
    return before + x - v;
}

// Four consecutive cells of chunk `base` per thread, guarded at ncell.
__device__ __forceinline__ void load4(const int *__restrict__ cnt, int base, int ncell, int (&c)[4])
{
    const int k0 = base + 4 * (int)threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        c[q] = k0 + q < ncell ? cnt[k0 + q] : 0;
}

// Exclusive scan of one chunk with a carried offset: cell_off, counts cleared.
__device__ __forceinline__ int scan_chunk(int *__restrict__ cell_cnt, int *__restrict__ cell_off,
                                          int base, int ncell, int carry, int *sh)
{
    int c[4];
    load4(cell_cnt, base, ncell, c);
    int tot;
    int run = carry + block_exscan(c[0] + c[1] + c[2] + c[3], sh, tot);
    const int k0 = base + 4 * (int)threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (k0 + q < ncell) {
            cell_off[k0 + q] = run;
            cell_cnt[k0 + q] = 0;
        }
        run += c[q];
    }
    return tot;
}

// Counting-sort offsets: cell_off = exclusive scan of cell_cnt (all systems'
// cells back to back), counts cleared for the next step.  One block walks
// the cells in chunks (up to kScanSerialChunks chunks); larger grids use
// k_scan_sums + k_scan_apply.
constexpr int kScanSerialChunks = 16;
__global__ __launch_bounds__(kScanThreads) void k_cell_scan(int *__restrict__ cell_cnt,
                                                            int *__restrict__ cell_off, int ncell,
                                                            DevStats *stats)
{
    __shared__ int sh[64];
    int carry = 0;
    for (int base = 0; base < ncell; base += kScanChunk)
        carry += scan_chunk(cell_cnt, cell_off, base, ncell, carry, sh);
    if (threadIdx.x == 0) {
        stats->cur_tp = 0;
        stats->cur_nce = 0;
    }
}

// Block b: sum of the counts of chunk b.
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(const int *__restrict__ cell_cnt,
                                                            int ncell, int *__restrict__ part)
{
    __shared__ int sh[64];
    int c[4];
    load4(cell_cnt, blockIdx.x * kScanChunk, ncell, c);
    int tot;
    (void)block_exscan(c[0] + c[1] + c[2] + c[3], sh, tot);
    if (threadIdx.x == 0)
        part[blockIdx.x] = tot;
}

// Block b: exclusive offset of chunk b from the chunk sums (in order), then the
// chunk's own scan.  Block 0 also resets the tile-pair count.
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int *__restrict__ cell_cnt,
                                                             int *__restrict__ cell_off, int ncell,
                                                             const int *__restrict__ part,
                                                             DevStats *stats)
{
    __shared__ int sh[64];
    int pre = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += kScanThreads)
        pre += part[k];
    int tot;
    (void)block_exscan(pre, sh, tot);
    (void)scan_chunk(cell_cnt, cell_off, blockIdx.x * kScanChunk, ncell, tot, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        stats->cur_tp = 0;
        stats->cur_nce = 0;
    }
}

// Sorted position of every body: its cell's offset plus the slot the binning
// took (the order inside a cell follows the atomics' timing until
// k_cell_order puts it in index order).  slot_of[i] becomes the position.
__global__ void k_scatter(const RBlk *__restrict__ rblk, const int *__restrict__ cell_of,
                          int *__restrict__ slot_of, const int *__restrict__ cell_off,
                          int *__restrict__ ord)
{
    const RBlk b = rblk[blockIdx.x];
    const int i = b.start + threadIdx.x;
    if (i >= b.end)
        return;
    const int pos = cell_off[cell_of[i]] + slot_of[i];
    ord[pos] = i;
    slot_of[i] = pos;
}

// The bodies of every cell in index order, so that the sorted order, its tiles
// and the tile pairs are the same from run to run.  One wave per cell: a body's
// new slot is the number of smaller indices in its cell.  A cell of more than
// kCellSortMax bodies keeps the binning's order (its set is still right).
constexpr int kCellSortMax = 512;

__global__ __launch_bounds__(kBlock) void k_cell_order(const int *__restrict__ cell_off, int ncell,
                                                       int ntot, int *__restrict__ ord,
                                                       int *__restrict__ pos_of)
{
    __shared__ int sb[kBlock / 64][kCellSortMax];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = blockIdx.x * (kBlock / 64) + wv;
    int start = 0, k = 0;
    if (c < ncell) {
        start = cell_off[c];
        k = (c + 1 < ncell ? cell_off[c + 1] : ntot) - start;
    }
    const bool go = k > 1 && k <= kCellSortMax;
    if (go)
        for (int e = lane; e < k; e += 64)
            sb[wv][e] = ord[start + e];
    __syncthreads();
    if (go)
        for (int e = lane; e < k; e += 64) {
            const int me = sb[wv][e];
            int rank = 0;
            for (int q = 0; q < k; ++q)
                rank += sb[wv][q] < me;
            ord[start + rank] = me;
            pos_of[me] = start + rank;
        }
}

// The sorted records from the drift outputs, body by body (coalesced reads),
// each written to the body's sorted position.
__global__ void k_srec(int ntot, const int *__restrict__ pos_of, const int *__restrict__ sys_of,
                       const double *__restrict__ q0x, const double *__restrict__ q0y,
                       const double *__restrict__ q0z, const double *__restrict__ v0x,
                       const double *__restrict__ v0y, const double *__restrict__ v0z,
                       const double *__restrict__ qx, const double *__restrict__ qy,
                       const double *__restrict__ qz, const double *__restrict__ vx,
                       const double *__restrict__ vy, const double *__restrict__ vz,
                       const double *__restrict__ rc, const double4 *__restrict__ mr,
                       const double4 *__restrict__ cr, const int *__restrict__ off,
                       const int *__restrict__ nbig, SRec *__restrict__ srec,
                       float4 *__restrict__ em, float4 *__restrict__ eg, double dt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot)
        return;
    const int pos = pos_of[i];
    const int sy = sys_of[i];
    SRec r;
    r.q0[0] = q0x[i]; r.q0[1] = q0y[i]; r.q0[2] = q0z[i];
    r.v0[0] = v0x[i]; r.v0[1] = v0y[i]; r.v0[2] = v0z[i];
    r.q1[0] = qx[i];  r.q1[1] = qy[i];  r.q1[2] = qz[i];
    r.v1[0] = vx[i];  r.v1[1] = vy[i];  r.v1[2] = vz[i];
    r.rc = rc[i];
    r.body = i;
    r.big = (i - off[sy]) < nbig[sy] ? 1 : 0;
    const double4 M = mr[i], C = cr[i];
    r.M[0] = M.x; r.M[1] = M.y; r.M[2] = M.z;
    r.c[0] = C.x; r.c[1] = C.y; r.c[2] = C.z;
    r.e34 = C.w;
    r.pad = 0.0;
    srec[pos] = r;
    if (em) {
        // FP32 records of the pair filter: midpoint M and chord c, and the
        // bound b' of 3/4 eps widened by 2^-21 (|M|_1 + |c|_1) for the FP32
        // rounding of M, c and their differences, and by 2^-18 relative for the
        // rounding of the bound itself, negated (sign bit set) for a small body;
        // the chord's fourth word is rc rounded up.  A pair's bound is
        // |b'_i| + |b'_j| + max(rc_i, rc_j).
        const double w = (C.w + 0x1p-21 * (fabs(M.x) + fabs(M.y) + fabs(M.z) + fabs(C.x) +
                                           fabs(C.y) + fabs(C.z))) * (1.0 + 0x1p-18);
        const float rcu = (float)(rc[i] * (1.0 + 0x1p-20));
        em[2 * (size_t)pos] = make_float4((float)M.x, (float)M.y, (float)M.z, r.big ? (float)w : -(float)w);
        em[2 * (size_t)pos + 1] = make_float4((float)C.x, (float)C.y, (float)C.z, rcu);
        // the endpoint deviations of the step (as the tile bounds take them):
        // their mean eb and half their difference's norm se, rounded up
        double s2 = 0.0, eb[3];
        for (int k = 0; k < 3; ++k) {
            const double e0 = dt * r.v0[k] - (r.q1[k] - r.q0[k]), e1 = dt * r.v1[k] - (r.q1[k] - r.q0[k]);
            eb[k] = 0.5 * (e0 + e1);
            s2 += (e0 - e1) * (e0 - e1);
        }
        eg[pos] = make_float4((float)eb[0], (float)eb[1], (float)eb[2],
                              (float)(0.5 * sqrt(s2) * (1.0 + 0x1p-20)));
    }
}

// Chord midpoint M, chord c, mean deviation eb and deviation radius se of one record.
__device__ __forceinline__ void rec_geometry(const SRec &r, double dt, double M[3], double c[3],
                                             double eb[3], double &se)
{
    double s2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        c[k] = r.q1[k] - r.q0[k];
        M[k] = r.q0[k] + 0.5 * c[k];
        double e0 = dt * r.v0[k] - c[k], e1 = dt * r.v1[k] - c[k];
        eb[k] = 0.5 * (e0 + e1);
        s2 += (e0 - e1) * (e0 - e1);
    }
    se = 0.5 * sqrt(s2);
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_maxd(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double norm3(double x, double y, double z)
{
    return sqrt(x * x + y * y + z * z);
}

// One wave per tile: centres (means) and radii (maxima) of its bodies' geometry.
__global__ __launch_bounds__(kBlock) void k_tile_bounds(const Tile *__restrict__ tiles, int ntile,
                                                        const SRec *__restrict__ srec, double dt,
                                                        TileB *__restrict__ tileb)
{
    const int tw = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (tw >= ntile)
        return;
    const Tile T = tiles[tw];
    const bool on = lane < T.count;
    double M[3] = {0, 0, 0}, c[3] = {0, 0, 0}, eb[3] = {0, 0, 0}, se = 0.0, rc = 0.0;
    bool big = false;
    if (on) {
        const SRec r = srec[T.start + lane];
        rec_geometry(r, dt, M, c, eb, se);
        rc = r.rc;
        big = r.big != 0;
    }
    const bool any_big = __any(big), all_big = __all(!on || big);
    const double inv = 1.0 / (double)T.count;
    double cm[3], cc[3], ce[3];
    for (int k = 0; k < 3; ++k) {
        cm[k] = wave_sum(M[k]) * inv;
        cc[k] = wave_sum(c[k]) * inv;
        ce[k] = wave_sum(eb[k]) * inv;
    }
    double dm = 0.0, dc = 0.0, de = 0.0;
    if (on) {
        dm = norm3(M[0] - cm[0], M[1] - cm[1], M[2] - cm[2]);
        dc = norm3(c[0] - cc[0], c[1] - cc[1], c[2] - cc[2]);
        de = norm3(eb[0] - ce[0], eb[1] - ce[1], eb[2] - ce[2]) + se;
    }
    // radii widened by 2^-20 to cover the rounding of the centres and norms
    const double wf = 1.0 + 0x1p-20;
    const double sm = wave_maxd(dm) * wf, sc = wave_maxd(dc) * wf, sde = wave_maxd(de) * wf;
    const double rcm = wave_maxd(rc);
    if (lane == 0) {
        TileB B;
        for (int k = 0; k < 3; ++k) {
            B.cm[k] = cm[k];
            B.cc[k] = cc[k];
            B.ce[k] = ce[k];
        }
        B.sm = sm;
        B.sc = sc;
        B.se = sde;
        B.rc = rcm;
        B.big = any_big ? 1 : 0;
        B.all_big = all_big ? 1 : 0;
        B.pad2[0] = B.pad2[1] = 0.0;
        tileb[tw] = B;
    }
}

// True when a pair between the two bounded sets may be flagged.  The rounding
// margin is relative to the squared scales involved.
__device__ __forceinline__ bool may_meet(const double cmA[3], double smA, const double ccA[3],
                                         double scA, const double ceA[3], double seA, double rcA,
                                         const TileB &B)
{
    double D = norm3(B.cm[0] - cmA[0], B.cm[1] - cmA[1], B.cm[2] - cmA[2]);
    double Cm = norm3(B.cc[0] - ccA[0], B.cc[1] - ccA[1], B.cc[2] - ccA[2]) + scA + B.sc;
    double Em = norm3(B.ce[0] - ceA[0], B.ce[1] - ceA[1], B.ce[2] - ceA[2]) + seA + B.se;
    double Lmin = D - smA - B.sm - 0.5 * Cm;
    double Qmax = D + smA + B.sm + 0.5 * Cm;
    double RC = fmax(rcA, B.rc);
    if (!(Lmin > 0.0))
        return true;
    double lhs = Lmin * Lmin - 0.5 * Qmax * Em;
    return !(lhs > RC * RC * (1.0 + 1e-6) + 1e-12 * Qmax * Qmax);
}

// One wave per culling unit (tile A against tiles [b0, b0 + 64) of the same
// system with B >= A; kTpWaves units per workgroup): its lanes test one tile B
// each and the pairs that may meet are appended.  The survivors are counted
// first and the workgroup reserves its whole range with one atomic (a counter
// that every wave of the grid hits is a serial point), then the test is
// repeated to write the pairs.
constexpr int kTpWaves = 4;

__device__ __forceinline__ bool tile_pair_kept(const Tile &TA, const TileB &BA,
                                               const TileB *__restrict__ tileb, int B)
{
    // two small bodies never interact: a pair of tiles without a big body is skipped
    return B <= TA.last && (BA.big || tileb[B].big) &&
           may_meet(BA.cm, BA.sm, BA.cc, BA.sc, BA.ce, BA.se, BA.rc, tileb[B]);
}

__global__ __launch_bounds__(64 * kTpWaves) void k_tile_pairs(const Tile *__restrict__ tiles,
                                                             const int2 *__restrict__ units,
                                                             int nunit,
                                                             const TileB *__restrict__ tileb,
                                                             int2 *__restrict__ tpairs, int tp_cap,
                                                             DevStats *stats)
{
    __shared__ int wcount[kTpWaves];
    __shared__ int wbase[kTpWaves];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int u = blockIdx.x * kTpWaves + wv;
    const bool has = u < nunit;
    int A = 0, B = 0;
    bool ok = false;
    if (has) {
        const int2 U = units[u];
        A = U.x;
        B = U.y + lane;
        const Tile TA = tiles[A];
        const TileB BA = tileb[A];
        ok = tile_pair_kept(TA, BA, tileb, B);
    }
    const unsigned long long mask = __ballot(ok);
    if (lane == 0)
        wcount[wv] = (int)__popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < kTpWaves; ++w) {
            wbase[w] = tot;
            tot += wcount[w];
        }
        const int base = tot ? atomicAdd(&stats->cur_tp, tot) : 0;
        for (int w = 0; w < kTpWaves; ++w)
            wbase[w] += base;
    }
    __syncthreads();
    if (ok) {
        const int p = wbase[wv] + (int)__popcll(mask & ((1ull << lane) - 1ull));
        if (p < tp_cap)
            tpairs[p] = make_int2(A, B);
    }
}

// The exact test's fields of one sorted record.
struct HRec {
    double q0[3], v0[3], q1[3], v1[3];
    double rc;
    int body;
};

// Exact encounter test of a pair (the Hermite bound, then the minimum over the
// step) and the append of a flagged pair.
__device__ __forceinline__ void enc_exact(const HRec &I, const SRec &J, double dt,
                                          unsigned long long *keys, int cap, int *ce,
                                          DevStats *stats)
{
    const double t2 = 2.0 * dt, k427 = 4.0 / 27.0;
    const double d0x = J.q0[0] - I.q0[0], d0y = J.q0[1] - I.q0[1], d0z = J.q0[2] - I.q0[2];
    const double d1x = J.q1[0] - I.q1[0], d1y = J.q1[1] - I.q1[1], d1z = J.q1[2] - I.q1[2];
    const double e0x = J.v0[0] - I.v0[0], e0y = J.v0[1] - I.v0[1], e0z = J.v0[2] - I.v0[2];
    const double e1x = J.v1[0] - I.v1[0], e1y = J.v1[1] - I.v1[1], e1z = J.v1[2] - I.v1[2];
    const double f0 = fma(d0z, d0z, fma(d0y, d0y, d0x * d0x));
    const double f1 = fma(d1z, d1z, fma(d1y, d1y, d1x * d1x));
    const double g0 = t2 * fma(d0z, e0z, fma(d0y, e0y, d0x * e0x));
    const double g1 = t2 * fma(d1z, e1z, fma(d1y, e1y, d1x * e1x));
    const double lower = fmin(f0, f1) - k427 * (fmax(0.0, -g0) + fmax(0.0, g1));
    const double rcij = fmax(I.rc, J.rc);
    const double thr = rcij * rcij;
    if (!(lower <= thr * (1.0 + 1e-6) + 1e-15 * (f0 + f1 + fabs(g0) + fabs(g1))))
        return;
    if (!(hermite_min(f0, f1, g0, g1) <= thr))
        return;
    const int pos = atomicAdd(&stats->cur_nce, 1);
    const int bi = I.body, bj = J.body;
    const unsigned lo = (unsigned)min(bi, bj), hi = (unsigned)max(bi, bj);
    if (pos < cap)
        keys[pos] = ((unsigned long long)lo << 32) | hi;
    __hip_atomic_store(&ce[bi], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ce[bj], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The same for two sorted positions, every field of both records read at once.
__device__ __noinline__ void enc_candidate(const SRec *__restrict__ srec, double dt,
                                           unsigned long long *keys, int cap, int *ce,
                                           DevStats *stats, int pi, int pj)
{
    const SRec &R = srec[pi];
    HRec I;
    for (int k = 0; k < 3; ++k) {
        I.q0[k] = R.q0[k];
        I.v0[k] = R.v0[k];
        I.q1[k] = R.q1[k];
        I.v1[k] = R.v1[k];
    }
    I.rc = R.rc;
    I.body = R.body;
    enc_exact(I, srec[pj], dt, keys, cap, ce, stats);
}

// One wave per kept tile pair (A, B), the waves striding over the count: lane
// L holds the FP32 filter records of body L of tile A (midpoint with widened
// bound, chord with big flag: 32 B), tile B's sit in the wave's LDS slice, and
// every lane meets the 64 sources in turn with the relative-chord filter in
// FP32, a superset of the pairs that can be flagged (the widening covers the
// rounding).  A lane first meets tile B's bounds with the tile-pair test, as a
// tile of one body whose FP32 records stand for small balls around its FP64
// values (third record: the mean endpoint deviation and its radius).  The
// pairs the filter keeps are queued in the wave's LDS and take the exact test
// from the sorted FP64 records in memory 64 at a time, one per lane (with long
// steps most pairs of a dense ring pass the filter, and a test per pass would
// run on a few lanes); a tile pair reads 5 KB of filter records instead of the
// 176-byte records of both tiles.
__global__ __launch_bounds__(kBlock) void k_enc_pairs(const Tile *__restrict__ tiles,
                                                      const TileB *__restrict__ tileb,
                                                      const int2 *__restrict__ tpairs, int tp_cap,
                                                      const SRec *__restrict__ srec,
                                                      const float4 *__restrict__ em,
                                                      const float4 *__restrict__ eg, double dt,
                                                      unsigned long long *__restrict__ keys,
                                                      int cap, int *__restrict__ ce,
                                                      DevStats *stats)
{
    __shared__ float4 sm_[kBlock / 64][64], sc_[kBlock / 64][64];
    // per wave: queued pairs (lane | source << 8), fewer than 64 between drains
    __shared__ int qe[kBlock / 64][128];
    // per wave: tile A's exact-test fields (q0, v0, q1, v1, rc by plane; body
    // index), staged at the tile pair's first full drain: a drain's 64 pairs
    // hold many targets and few sources
    __shared__ double ha[kBlock / 64][13][64];
    __shared__ int hb[kBlock / 64][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int npair = min(stats->cur_tp, tp_cap);
    const float qnan = __int_as_float(0x7fc00000);
    for (int p = blockIdx.x * (kBlock / 64) + wv; p < npair; p += gridDim.x * (kBlock / 64)) {
        const int2 AB = tpairs[p];
        Tile TA = tiles[AB.x], TB = tiles[AB.y];
        // uniform over the wave (one tile pair a wave): kept in scalar registers
        TA.start = __builtin_amdgcn_readfirstlane(TA.start);
        TA.count = __builtin_amdgcn_readfirstlane(TA.count);
        TB.start = __builtin_amdgcn_readfirstlane(TB.start);
        TB.count = __builtin_amdgcn_readfirstlane(TB.count);
        // tile B's FP32 filter records in the wave's LDS slice (padding: NaN
        // midpoints, which no test passes)
        if (lane < TB.count) {
            sm_[wv][lane] = em[2 * (size_t)(TB.start + lane)];
            sc_[wv][lane] = em[2 * (size_t)(TB.start + lane) + 1];
        } else {
            sm_[wv][lane] = make_float4(qnan, qnan, qnan, 0.0f);
            sc_[wv][lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        wave_lds_sync();
        const bool on = lane < TA.count;
        const float4 Mi = on ? em[2 * (size_t)(TA.start + lane)] : make_float4(qnan, qnan, qnan, 0.0f);
        const float4 Ci = on ? em[2 * (size_t)(TA.start + lane) + 1] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        // the lane against tile B's bounds with the tile-pair test, the lane a
        // tile of one body whose FP32 records stand for balls around them: 2^-23
        // of each vector's norm covers its rounding, se and rc are rounded up
        bool lane_ok = false;
        if (on) {
            const float4 Gi = eg[TA.start + lane];
            const double Mv[3] = {Mi.x, Mi.y, Mi.z}, cv[3] = {Ci.x, Ci.y, Ci.z},
                         ev[3] = {Gi.x, Gi.y, Gi.z};
            const double sM = 0x1p-23 * norm3(Mv[0], Mv[1], Mv[2]);
            const double sC = 0x1p-23 * norm3(cv[0], cv[1], cv[2]);
            const double sE = (double)Gi.w + 0x1p-23 * norm3(ev[0], ev[1], ev[2]);
            const TileB &BB = tileb[AB.y];
            lane_ok = (__float_as_int(Mi.w) >= 0 || BB.big) &&
                      may_meet(Mv, sM, cv, sC, ev, sE, (double)Ci.w, BB);
        }
        const bool diag = AB.x == AB.y;
        const int nj = __builtin_amdgcn_ballot_w64(lane_ok) ? TB.count : 0;
        const float wi = fabsf(Mi.w);
        int qn = 0;
        bool staged = false;
        // the exact test of queue entry e (this lane's): target from the staged
        // fields, source record from memory
        auto test_entry = [&](int e) {
            const int li = e & 255;
            HRec I;
            for (int k = 0; k < 3; ++k) {
                I.q0[k] = ha[wv][k][li];
                I.v0[k] = ha[wv][3 + k][li];
                I.q1[k] = ha[wv][6 + k][li];
                I.v1[k] = ha[wv][9 + k][li];
            }
            I.rc = ha[wv][12][li];
            I.body = hb[wv][li];
            enc_exact(I, srec[TB.start + (e >> 8)], dt, keys, cap, ce, stats);
        };
        auto stage = [&]() {
            if (!staged) {
                if (on) {
                    const SRec &R = srec[TA.start + lane];
                    for (int k = 0; k < 3; ++k) {
                        ha[wv][k][lane] = R.q0[k];
                        ha[wv][3 + k][lane] = R.v0[k];
                        ha[wv][6 + k][lane] = R.q1[k];
                        ha[wv][9 + k][lane] = R.v1[k];
                    }
                    ha[wv][12][lane] = R.rc;
                    hb[wv][lane] = R.body;
                }
                staged = true;
            }
        };
        // the pair loop, with the diagonal's order test and the small-small
        // test only where the tile pair needs them
        auto pair_loop = [&](auto diag_c, auto small_c) {
        constexpr bool DG = decltype(diag_c)::value, SM = decltype(small_c)::value;
        for (int jj = 0; jj < nj; ++jj) {
            // source jj's FP32 filter records (one broadcast read each)
            const float4 E = sm_[wv][jj], F = sc_[wv][jj];
            // relative chord filter in FP32 (the bound's widening covers the
            // rounding), every lane without a branch
            const float ex = E.x - Mi.x, ey = E.y - Mi.y, ez = E.z - Mi.z;
            const float cx = F.x - Ci.x, cy = F.y - Ci.y, cz = F.z - Ci.z;
            const float D2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
            const float C2 = fmaf(cz, cz, fmaf(cy, cy, cx * cx));
            const float Sr = (fabsf(E.w) + wi) + max_nonneg(F.w, Ci.w);
            bool cand = lane_ok & (D2 <= fmaf(Sr, Sr, C2) * (2.0f * (1.0f + 0x1p-18f)));
            if (DG)
                cand &= jj > lane;
            if (SM)
                cand &= (__float_as_int(E.w) & __float_as_int(Mi.w)) >= 0;
            // the pairs the filter keeps join the wave's queue; 64 of them at a
            // time take the exact test, one per lane
            const unsigned long long mk = __builtin_amdgcn_ballot_w64(cand);
            if (mk) {
                if ((mk >> lane) & 1ull)
                    qe[wv][qn + __popcll(mk & ((1ull << lane) - 1ull))] = lane | (jj << 8);
                qn += __popcll(mk);
                if (qn >= 64) {
                    stage();
                    wave_lds_sync();
                    test_entry(qe[wv][lane]);
                    const int rest = qn - 64;
                    const int v = lane < rest ? qe[wv][64 + lane] : 0;
                    wave_lds_sync();
                    if (lane < rest)
                        qe[wv][lane] = v;
                    wave_lds_sync();
                    qn = rest;
                }
            }
        }
        };
        // a small body in tile A (the sign of a lane's bound) or in tile B
        const bool small = __builtin_amdgcn_ballot_w64(on && __float_as_int(Mi.w) < 0) != 0 ||
                           !tileb[AB.y].all_big;
        if (diag) {
            if (small)
                pair_loop(std::true_type{}, std::true_type{});
            else
                pair_loop(std::true_type{}, std::false_type{});
        } else {
            if (small)
                pair_loop(std::false_type{}, std::true_type{});
            else
                pair_loop(std::false_type{}, std::false_type{});
        }
        if (qn > 0) {
            // the rest: from the staged fields if a full drain staged them, else
            // both records from memory (a tile pair with few pairs to test)
            wave_lds_sync();
            if (lane < qn) {
                const int e = qe[wv][lane];
                if (staged)
                    test_entry(e);
                else
                    enc_candidate(srec, dt, keys, cap, ce, stats, TA.start + (e & 255),
                                  TB.start + (e >> 8));
            }
        }
        // the slices, the queue and the staged fields are refilled for the
        // next pair only after every lane's reads
        wave_lds_sync();
    }
}

// ----------------------------------------------------------------------------
// Force and encounter check in one pass over spatially sorted tiles (FP32C,
// every body big).  The symmetric force runs over super-tile pairs of sorted
// positions (sources and targets gathered through the sorted order, split
// partials by position, mapped back to bodies by the finalize).  In every
// round the wave bounds the tile pairs of its target sub-tiles and the source
// sub-tiles with the culling lemma of the sorted check (may_meet on the tiles
// of 64); where a tile pair may hold a flagged pair, each pair of it also gets
// the FP32 relative-chord filter, and the pairs it passes the exact Hermite
// test in FP64 from the sorted records.  Each unordered pair is met once, so
// each flagged pair is appended once.
// ----------------------------------------------------------------------------
// Tile of 64 sorted positions holding position p of system sy.
__device__ __forceinline__ int tile_of(const int *__restrict__ tile_first, const int *__restrict__ off,
                                       int sy, int p)
{
    return tile_first[sy] + (p - off[sy]) / 64;
}

template <int R, int G>
__global__ __launch_bounds__(64 * G, R == 4 ? 1 : 2) void k_force32c_fused(
    const FWork *__restrict__ work, int nitems, const int *__restrict__ ord,
    const float4 *__restrict__ pk, const float4 *__restrict__ em, const TileB *__restrict__ tileb,
    const int *__restrict__ tile_first, const int *__restrict__ off, const double *__restrict__ qx,
    const double *__restrict__ qy, const double *__restrict__ qz, const double *__restrict__ m,
    const double *__restrict__ rc, float *__restrict__ fpart, int ntot, int maxs, double inner,
    EncCtx ec)
{
    constexpr int T = 64 * R;
    __shared__ SymTile32E<T> tl[G];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const size_t plane = (size_t)maxs * ntot;
    const float qnan = __int_as_float(0x7fc00000);
    int near = 0;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const FWork wk = work[it];
        const bool diag = wk.i0 == wk.j0;
        // the G source tiles of super-tile J, gathered through the sorted order
        for (int k = threadIdx.x; k < G * T; k += 64 * G) {
            SymTile32<T> &S = tl[k / T].t;
            const int e = k % T;
            if (k < wk.nj) {
                const int b = ord[wk.j0 + k];
                S.a[e] = pk[2 * (size_t)b];
                S.b[e] = pk[2 * (size_t)b + 1];
                tl[k / T].em[e] = em[2 * (size_t)(wk.j0 + k)];
                tl[k / T].ec[e] = em[2 * (size_t)(wk.j0 + k) + 1];
            } else {
                S.a[e] = make_float4(1e18f, 1e18f, 1e18f, 0.0f);
                S.b[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                tl[k / T].em[e] = make_float4(qnan, qnan, qnan, 0.0f);
                tl[k / T].ec[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
            S.run[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            S.ax[e] = S.ay[e] = S.az[e] = 0.0;
        }
        __syncthreads();
        const int ti0 = wk.i0 + wv * T;
        const int tni = min(T, wk.ni - wv * T);
        float xh[R], yh[R], zh[R], xl[R], yl[R], zl[R], mi[R];
        float hx[R], hy[R], hz[R], lx[R], ly[R], lz[R];
        float4 emi[R], eci[R];
        float tmi = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int li = 64 * r + lane;
            const bool ok = li < tni;
            const int b = ord[ok ? ti0 + li : wk.i0];
            const float4 A = pk[2 * (size_t)b], B = pk[2 * (size_t)b + 1];
            xh[r] = A.x; yh[r] = A.y; zh[r] = A.z;
            xl[r] = B.x; yl[r] = B.y; zl[r] = B.z;
            mi[r] = ok ? A.w : 0.0f;
            tmi = max_nonneg(tmi, B.w);
            emi[r] = ok ? em[2 * (size_t)(ti0 + li)] : make_float4(qnan, qnan, qnan, 0.0f);
            eci[r] = ok ? em[2 * (size_t)(ti0 + li) + 1] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            hx[r] = hy[r] = hz[r] = lx[r] = ly[r] = lz[r] = 0.0f;
        }
        tmi = wave_max_nonneg(tmi);
        const int nr = diag ? G / 2 + 1 : G;
        // The tile pairs that may hold a flagged pair, for every round at once:
        // lane (k R + t) R + r bounds target sub-tile r against sub-tile t of
        // round k's source tile (G R^2 <= 64 lanes), so the bounds' loads and
        // square roots are in flight together, once per item.
        unsigned long long livemask;
        {
            constexpr int RR = R * R;
            const int k = lane / RR, t = (lane % RR) / R, r = lane % R;
            const int s = (wv + k) % G;
            bool lv = false;
            if (k < nr && 64 * r < tni && s * T + 64 * t < wk.nj) {
                const TileB &A = tileb[tile_of(tile_first, off, wk.sys, ti0 + 64 * r)];
                lv = may_meet(A.cm, A.sm, A.cc, A.sc, A.ce, A.se, A.rc,
                              tileb[tile_of(tile_first, off, wk.sys, wk.j0 + s * T + 64 * t)]);
            }
            livemask = __ballot(lv);
        }
        for (int k = 0; k < nr; ++k) {
            const int s = (wv + k) % G;
            const bool go = tni > 0 && s * T < wk.nj && !(diag && 2 * k == G && wv >= G / 2);
            if (go) {
                // this round's bits: t R + r
                const int sj0 = wk.j0 + s * T;
                const unsigned live =
                    (unsigned)(livemask >> (k * R * R)) & (unsigned)((1ull << (R * R)) - 1ull);
                if (diag && k == 0)
                    sym_tile32c<R, true, T, true>(tl[s].t, lane, ti0, tni, sj0, inner, pk, qx, qy,
                                                  qz, m, rc, xh, yh, zh, xl, yl, zl, mi, tmi, hx,
                                                  hy, hz, lx, ly, lz, near, ord, ec, emi, eci,
                                                  live);
                else
                    sym_tile32c<R, false, T, true>(tl[s].t, lane, ti0, tni, sj0, inner, pk, qx, qy,
                                                   qz, m, rc, xh, yh, zh, xl, yl, zl, mi, tmi, hx,
                                                   hy, hz, lx, ly, lz, near, ord, ec, emi, eci,
                                                   live);
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int li = 64 * r + lane;
            if (li < tni) {
                const int i = ti0 + li;
                double sx_ = (double)hx[r] + (double)lx[r];
                double sy_ = (double)hy[r] + (double)ly[r];
                double sz_ = (double)hz[r] + (double)lz[r];
                if (diag) {
                    sx_ += tl[wv].t.ax[li];
                    sy_ += tl[wv].t.ay[li];
                    sz_ += tl[wv].t.az[li];
                }
                fpart[(size_t)wk.slot * ntot + i] = (float)sx_;
                fpart[plane + (size_t)wk.slot * ntot + i] = (float)sy_;
                fpart[2 * plane + (size_t)wk.slot * ntot + i] = (float)sz_;
            }
        }
        if (!diag) {
            for (int k = threadIdx.x; k < wk.nj; k += 64 * G) {
                const SymTile32<T> &S = tl[k / T].t;
                const int e = k % T, j = wk.j0 + k;
                fpart[((size_t)0 * maxs + wk.pad) * ntot + j] = (float)S.ax[e];
                fpart[((size_t)1 * maxs + wk.pad) * ntot + j] = (float)S.ay[e];
                fpart[((size_t)2 * maxs + wk.pad) * ntot + j] = (float)S.az[e];
            }
        }
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1)
        near += __shfl_xor(near, o);
    if (lane == 0 && near)
        atomicAdd((unsigned long long *)&ec.stats->near_pairs, (unsigned long long)near);
}

// ----------------------------------------------------------------------------
// Persistent step launch: one workgroup owns one system and runs `nsteps`
// whole hybrid steps K S D C S F K without leaving the kernel (all phases at
// workgroup scope, separated by workgroup barriers).  Systems are handed out
// largest first.  FP64 pair arithmetic; every sum has a fixed order, so runs
// are bit-reproducible (the order differs from the per-phase launches, so the
// two paths agree to rounding, not bit for bit).
// ----------------------------------------------------------------------------
constexpr int kPJ = 256;    // sources staged in LDS per tile

template <int NT, int W>
__device__ __forceinline__ void pblock_sum(double (&v)[W], double *sh)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int w = 0; w < W; ++w)
        sh[w * NT + t] = v[w];
    __syncthreads();
    for (int st = NT / 2; st > 0; st >>= 1) {
        if (t < st) {
#pragma unroll
            for (int w = 0; w < W; ++w)
                sh[w * NT + t] += sh[w * NT + t + st];
        }
        __syncthreads();
    }
#pragma unroll
    for (int w = 0; w < W; ++w)
        v[w] = sh[w * NT];
    __syncthreads();
}

// Sum of m V over the workgroup's system (each thread walks its own bodies).
template <int NT>
__device__ __forceinline__ void psys_momentum(int a, int n, const double *__restrict__ m,
                                              const double *vx, const double *vy,
                                              const double *vz, double (&P)[3], double *sh)
{
    P[0] = P[1] = P[2] = 0.0;
    for (int i = a + (int)threadIdx.x; i < a + n; i += NT) {
        double mi = m[i];
        P[0] += mi * vx[i];
        P[1] += mi * vy[i];
        P[2] += mi * vz[i];
    }
    pblock_sum<NT, 3>(P, sh);
}

template <int NT>
__device__ __forceinline__ void pkick(int a, int n, double h, double mm, const double (&P)[3],
                                      int drag, const DragP &dp, const double *__restrict__ m,
                                      const double *qx, const double *qy, const double *qz,
                                      const double *ax, const double *ay, const double *az,
                                      double *vx, double *vy, double *vz)
{
    for (int i = a + (int)threadIdx.x; i < a + n; i += NT) {
        double a0 = ax[i], a1 = ay[i], a2 = az[i];
        double u0 = vx[i], u1 = vy[i], u2 = vz[i];
        if (drag) {
            double d0, d1, d2;
            drag_accel(dp, mm, m[i], qx[i], qy[i], qz[i], u0 + P[0] / mm, u1 + P[1] / mm,
                       u2 + P[2] / mm, d0, d1, d2);
            a0 += d0;
            a1 += d1;
            a2 += d2;
        }
        vx[i] = u0 + h * a0;
        vy[i] = u1 + h * a1;
        vz[i] = u2 + h * a2;
    }
}

// Encounter record staged in LDS by the persistent launch.
struct PRec {
    double4 M;              // chord midpoint and reach
    double q0[3], v0[3], q1[3], v1[3];
    double rc, pad;
};
static_assert(sizeof(PRec) % sizeof(double) == 0, "PRec must be a whole number of doubles");

template <int NT>
__global__ __launch_bounds__(NT) void k_steps_persistent(
    const PSys *__restrict__ psys, int nsteps, double dt, double G, double n_hill, double inner,
    int drag, DragP dp, const double *__restrict__ m0, const double *__restrict__ m, double *qx,
    double *qy, double *qz, double *vx, double *vy, double *vz, double *ax, double *ay,
    double *az, double *rc, double *q0x, double *q0y, double *q0z, double *v0x, double *v0y,
    double *v0z, int *kflag, int *ce, double4 *mr, unsigned long long *keys, int cap,
    DevStats *stats, int *step_nce)
{
    // one LDS buffer, viewed per phase: block sums, encounter tile, force tile
    constexpr int kRecWords = (int)(sizeof(PRec) / sizeof(double));
    constexpr int kWords = (3 * NT > kPJ * kRecWords ? 3 * NT : kPJ * kRecWords);
    static_assert(kWords >= 2 * 4 * kPJ, "force tile must fit the buffer");
    __shared__ double lds[kWords];
    double *sh = lds;
    PRec *se = reinterpret_cast<PRec *>(lds);
    double4 *sj = reinterpret_cast<double4 *>(lds);
    double4 *sx = reinterpret_cast<double4 *>(lds) + kPJ;
    const PSys S = psys[blockIdx.x];
    const int a = S.start, n = S.n, nb = S.nbig, t = threadIdx.x, lane = t & 63;
    const int wave0 = t & ~63;             // first thread index of this wave
    const double mm = m0[S.sys], mu = G * mm, h = 0.5 * dt;
    const double t2 = 2.0 * dt, k427 = 4.0 / 27.0;
    for (int step = 0; step < nsteps; ++step) {
        const bool last = step == nsteps - 1;
        double P[3] = {0.0, 0.0, 0.0};
        // K(h); with drag the heliocentric velocity needs the current sum m V
        if (drag)
            psys_momentum<NT>(a, n, m, vx, vy, vz, P, sh);
        pkick<NT>(a, n, h, mm, P, drag, dp, m, qx, qy, qz, ax, ay, az, vx, vy, vz);
        // S(h)
        psys_momentum<NT>(a, n, m, vx, vy, vz, P, sh);
        for (int i = a + t; i < a + n; i += NT) {
            qx[i] += h * P[0] / mm;
            qy[i] += h * P[1] / mm;
            qz[i] += h * P[2] / mm;
        }
        // D(dt): snapshot, drift, failure flags, encounter reach, cleared flags
        int nf = 0;
        for (int i = a + t; i < a + n; i += NT) {
            double x = qx[i], y = qy[i], z = qz[i], u = vx[i], v = vy[i], w = vz[i];
            q0x[i] = x; q0y[i] = y; q0z[i] = z;
            v0x[i] = u; v0y[i] = v; v0z[i] = w;
            const double x0 = x, y0 = y, z0 = z, u0 = u, v0 = v, w0 = w;
            const bool fail = kepler_drift(mu, dt, x, y, z, u, v, w) != 0;
            nf += fail;
            qx[i] = x; qy[i] = y; qz[i] = z;
            vx[i] = u; vy[i] = v; vz[i] = w;
            kflag[i] = fail ? 1 : 0;
            ce[i] = 0;
            double cx = x - x0, cy = y - y0, cz = z - z0;
            double rho = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
            double ex0 = dt * u0 - cx, ey0 = dt * v0 - cy, ez0 = dt * w0 - cz;
            double ex1 = dt * u - cx, ey1 = dt * v - cy, ez1 = dt * w - cz;
            double eps = sqrt(fmax(ex0 * ex0 + ey0 * ey0 + ez0 * ez0, ex1 * ex1 + ey1 * ey1 + ez1 * ez1));
            double R = (2.0 * rho + 0.75 * eps + rc[i]) * (1.0 + 0x1p-20);
            mr[i] = make_double4(x0 + 0.5 * cx, y0 + 0.5 * cy, z0 + 0.5 * cz, R);
        }
        for (int o = 32; o > 0; o >>= 1)
            nf += __shfl_xor(nf, o);
        if (lane == 0 && nf)
            atomicAdd((unsigned long long *)&stats->kepler_fail, (unsigned long long)nf);
        double P2[3];
        psys_momentum<NT>(a, n, m, vx, vy, vz, P2, sh);   // also orders the drift's writes
        // C: ordered pairs (i, j) with i < j tested when i + j is even, i > j when
        // odd, so each unordered pair is tested once and every thread sees all j.
        for (int i0 = 0; i0 < n; i0 += NT) {
            const bool vi = i0 + t < n;
            const bool wave_on = i0 + wave0 < n;
            const int i = a + (vi ? i0 + t : 0);
            const double4 Mi = mr[i];
            const double a0[3] = {q0x[i], q0y[i], q0z[i]}, b0[3] = {v0x[i], v0y[i], v0z[i]};
            const double a1[3] = {qx[i], qy[i], qz[i]}, b1[3] = {vx[i], vy[i], vz[i]};
            const double rci = rc[i];
            for (int j0 = 0; j0 < n; j0 += kPJ) {
                const int cnt = min(kPJ, n - j0);
                __syncthreads();
                for (int k = t; k < cnt; k += NT) {
                    const int j = a + j0 + k;
                    PRec r;
                    r.M = mr[j];
                    r.q0[0] = q0x[j]; r.q0[1] = q0y[j]; r.q0[2] = q0z[j];
                    r.v0[0] = v0x[j]; r.v0[1] = v0y[j]; r.v0[2] = v0z[j];
                    r.q1[0] = qx[j];  r.q1[1] = qy[j];  r.q1[2] = qz[j];
                    r.v1[0] = vx[j];  r.v1[1] = vy[j];  r.v1[2] = vz[j];
                    r.rc = rc[j];
                    r.pad = 0.0;
                    se[k] = r;
                }
                __syncthreads();
                if (!wave_on)
                    continue;
                for (int jj = 0; jj < cnt; ++jj) {
                    const int j = a + j0 + jj;
                    const PRec &J = se[jj];
                    double dx = J.M.x - Mi.x, dy = J.M.y - Mi.y, dz = J.M.z - Mi.z;
                    double D2 = fma(dz, dz, fma(dy, dy, dx * dx));
                    double Sr = Mi.w + J.M.w;
                    // two small bodies (both at or past a + nb) never interact
                    bool mine = vi && j != i && ((i < j) == (((i + j) & 1) == 0)) &&
                                min(i, j) < a + nb;
                    bool cand = mine && D2 <= Sr * Sr;
                    if (!__any(cand))
                        continue;
                    bool hit = false;
                    if (cand) {
                        double d0x = J.q0[0] - a0[0], d0y = J.q0[1] - a0[1], d0z = J.q0[2] - a0[2];
                        double d1x = J.q1[0] - a1[0], d1y = J.q1[1] - a1[1], d1z = J.q1[2] - a1[2];
                        double e0x = J.v0[0] - b0[0], e0y = J.v0[1] - b0[1], e0z = J.v0[2] - b0[2];
                        double e1x = J.v1[0] - b1[0], e1y = J.v1[1] - b1[1], e1z = J.v1[2] - b1[2];
                        double f0 = fma(d0z, d0z, fma(d0y, d0y, d0x * d0x));
                        double f1 = fma(d1z, d1z, fma(d1y, d1y, d1x * d1x));
                        double g0 = t2 * fma(d0z, e0z, fma(d0y, e0y, d0x * e0x));
                        double g1 = t2 * fma(d1z, e1z, fma(d1y, e1y, d1x * e1x));
                        double lower = fmin(f0, f1) - k427 * (fmax(0.0, -g0) + fmax(0.0, g1));
                        double rcij = fmax(rci, J.rc);
                        double thr = rcij * rcij;
                        if (lower <= thr * (1.0 + 1e-6) + 1e-15 * (f0 + f1 + fabs(g0) + fabs(g1)))
                            hit = hermite_min(f0, f1, g0, g1) <= thr;
                    }
                    const unsigned long long mask = __ballot(hit);
                    if (mask) {
                        const int leader = __ffsll((long long)mask) - 1;
                        if (lane == leader)
                            atomicAdd(&step_nce[step], (int)__popcll(mask));
                        if (last) {
                            int base = 0;
                            if (lane == leader)
                                base = atomicAdd(&stats->cur_nce, (int)__popcll(mask));
                            base = __shfl(base, leader);
                            if (hit) {
                                const int pos = base + (int)__popcll(mask & ((1ull << lane) - 1ull));
                                const unsigned lo = (unsigned)min(i, j), hi = (unsigned)max(i, j);
                                if (pos < cap)
                                    keys[pos] = ((unsigned long long)lo << 32) | hi;
                            }
                        }
                        if (hit) {
                            __hip_atomic_store(&ce[i], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            __hip_atomic_store(&ce[j], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                }
            }
        }
        __syncthreads();
        // S(h) and the critical radii at the new positions
        for (int i = a + t; i < a + n; i += NT) {
            double x = qx[i] + h * P2[0] / mm, y = qy[i] + h * P2[1] / mm, z = qz[i] + h * P2[2] / mm;
            qx[i] = x;
            qy[i] = y;
            qz[i] = z;
            rc[i] = n_hill * sqrt(x * x + y * y + z * z) * cbrt(m[i] / (3.0 * mm));
        }
        __syncthreads();
        // F: each thread sums its targets over every big source, tile by tile in order
        for (int i0 = 0; i0 < n; i0 += NT) {
            const bool vi = i0 + t < n;
            const bool wave_on = i0 + wave0 < n;
            const int i = a + (vi ? i0 + t : 0);
            const double xi = qx[i], yi = qy[i], zi = qz[i], rci = rc[i];
            const double r2i = fmax(rci * rci, DBL_MIN);
            double sx0 = 0.0, sy0 = 0.0, sz0 = 0.0;
            for (int j0 = 0; j0 < nb; j0 += kPJ) {
                const int cnt = min(kPJ, nb - j0);
                __syncthreads();
                for (int k = t; k < cnt; k += NT) {
                    const int j = a + j0 + k;
                    const double mj = m[j], rj = rc[j];
                    sj[k] = make_double4(qx[j], qy[j], qz[j], mj);
                    sx[k] = make_double4(1.5 * mj, rj, fmax(rj * rj, DBL_MIN), 0.0);
                }
                __syncthreads();
                if (!wave_on)
                    continue;
#pragma unroll 2
                for (int jj = 0; jj < cnt; ++jj) {
                    const double4 J = sj[jj];
                    const double4 X = sx[jj];
                    double dx = J.x - xi, dy = J.y - yi, dz = J.z - zi;
                    double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                    double w = m_rinv3(J.w, X.x, r2);
                    if (r2 < fmax(r2i, X.z))
                        w = J.w * changeover_w(r2, fmax(rci, X.y), inner);
                    sx0 = fma(w, dx, sx0);
                    sy0 = fma(w, dy, sy0);
                    sz0 = fma(w, dz, sz0);
                }
            }
            if (vi) {
                ax[i] = G * sx0;
                ay[i] = G * sy0;
                az[i] = G * sz0;
            }
        }
        __syncthreads();
        // K(h)
        if (drag)
            psys_momentum<NT>(a, n, m, vx, vy, vz, P, sh);
        pkick<NT>(a, n, h, mm, P, drag, dp, m, qx, qy, qz, ax, ay, az, vx, vy, vz);
        __syncthreads();
    }
}

// Per-step counts of one persistent launch into the run statistics (one workgroup).
__global__ __launch_bounds__(kBlock) void k_step_stats(int *__restrict__ step_nce, int nsteps,
                                                       int cap, DevStats *stats)
{
    __shared__ long long st[kBlock];
    __shared__ int mx[kBlock], ov[kBlock];
    long long tot = 0;
    int mxv = 0, ovc = 0;
    for (int k = threadIdx.x; k < nsteps; k += kBlock) {
        int c = step_nce[k];
        tot += c;
        mxv = max(mxv, c);
        ovc += c > cap;
        step_nce[k] = 0;
    }
    st[threadIdx.x] = tot;
    mx[threadIdx.x] = mxv;
    ov[threadIdx.x] = ovc;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            st[threadIdx.x] += st[threadIdx.x + o];
            mx[threadIdx.x] = max(mx[threadIdx.x], mx[threadIdx.x + o]);
            ov[threadIdx.x] += ov[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stats->total_nce += st[0];
        stats->max_nce = max(stats->max_nce, mx[0]);
        stats->overflow_steps += ov[0];
    }
}

// Sort the encounter keys (one workgroup, bitonic) and split them into (ice,
// jce); `accumulate`: also fold the count into the run statistics.
constexpr int kSortThreads = 1024;
constexpr int kSortLds = 16384;  // 128 KiB of keys in LDS

// The check's totals: count, largest count and overflowing checks.  The list
// itself stays in append order until it is read (k_enc_sort).
__global__ void k_enc_count(int cap, DevStats *stats)
{
    if (threadIdx.x == 0) {
        const int count = stats->cur_nce;
        stats->total_nce += count;
        if (count > stats->max_nce)
            stats->max_nce = count;
        if (count > cap)
            stats->overflow_steps += 1;
    }
}

__global__ __launch_bounds__(kSortThreads) void k_enc_sort(unsigned long long *keys, int keys_p2,
                                                           int cap, int *__restrict__ ice,
                                                           int *__restrict__ jce, DevStats *stats,
                                                           int accumulate)
{
    __shared__ unsigned long long sk[kSortLds];
    const int t = threadIdx.x;
    const int count = stats->cur_nce;
    const int n = min(count, cap);
    if (t == 0 && accumulate) {
        stats->total_nce += count;
        if (count > stats->max_nce)
            stats->max_nce = count;
        if (count > cap)
            stats->overflow_steps += 1;
    }
    if (n <= 1) {
        if (n == 1 && t == 0) {
            ice[0] = (int)(keys[0] >> 32);
            jce[0] = (int)(keys[0] & 0xffffffffull);
        }
        return;
    }
    int P = 1;
    while (P < n)
        P <<= 1;
    const unsigned long long kMax = ~0ull;
    if (P <= kSortLds) {
        for (int k = t; k < P; k += kSortThreads)
            sk[k] = k < n ? keys[k] : kMax;
        __syncthreads();
        for (int size = 2; size <= P; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int k = t; k < P; k += kSortThreads) {
                    int l = k ^ stride;
                    if (l > k) {
                        bool up = (k & size) == 0;
                        unsigned long long a = sk[k], b = sk[l];
                        if ((a > b) == up) {
                            sk[k] = b;
                            sk[l] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int k = t; k < n; k += kSortThreads) {
            ice[k] = (int)(sk[k] >> 32);
            jce[k] = (int)(sk[k] & 0xffffffffull);
        }
    } else {
        // P <= keys_p2 by construction of the key buffer
        for (int k = n + t; k < P; k += kSortThreads)
            keys[k] = kMax;
        __syncthreads();
        for (int size = 2; size <= P; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int k = t; k < P; k += kSortThreads) {
                    int l = k ^ stride;
                    if (l > k) {
                        bool up = (k & size) == 0;
                        unsigned long long a = keys[k], b = keys[l];
                        if ((a > b) == up) {
                            keys[k] = b;
                            keys[l] = a;
                        }
                    }
                }
                __threadfence_block();
                __syncthreads();
            }
        }
        for (int k = t; k < n; k += kSortThreads) {
            ice[k] = (int)(keys[k] >> 32);
            jce[k] = (int)(keys[k] & 0xffffffffull);
        }
    }
}

// ----------------------------------------------------------------------------
// Diagnostics (Sec. 2.1.1 energy and momentum routine), FP64 with error-free
// accumulation: per pair work item the double-double sums of m_i m_j / r and of
// K m_i m_j / r; per body block kinetic, stellar potential, L and P; then one
// thread per system combines them in a fixed order.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_diag_pairs(const PWork *__restrict__ work,
                                                       const double *__restrict__ qx,
                                                       const double *__restrict__ qy,
                                                       const double *__restrict__ qz,
                                                       const double *__restrict__ m,
                                                       const double *__restrict__ rc, double inner,
                                                       double *__restrict__ dpart)
{
    __shared__ double4 sj[kBlock];
    __shared__ double sh[4 * kBlock];
    const PWork wk = work[blockIdx.x];
    const int t = threadIdx.x;
    const bool has_i = t < wk.ni;
    const int i = wk.i0 + (has_i ? t : 0);
    const double xi = qx[i], yi = qy[i], zi = qz[i], rci = rc[i];
    dd acc = {0.0, 0.0}, acck = {0.0, 0.0};
    const int jend = wk.j0 + wk.nj;
    __shared__ double srj[kBlock];
    for (int jt = wk.j0; jt < jend; jt += kBlock) {
        const int cnt = min(kBlock, jend - jt);
        __syncthreads();
        if (t < cnt) {
            int j = jt + t;
            sj[t] = make_double4(qx[j], qy[j], qz[j], m[j]);
            srj[t] = rc[j];
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; ++jj) {
            const int j = jt + jj;
            if (!has_i || j <= i)
                continue;
            double4 J = sj[jj];
            double dx = J.x - xi, dy = J.y - yi, dz = J.z - zi;
            double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            if (!(r2 > 0.0))
                continue;
            double y = rsqrt64_acc(r2);
            double u = J.w * y;
            dd_add(acc, u);
            double rcij = fmax(rci, srj[jj]);
            if (r2 < rcij * rcij) {
                double r = r2 * y;
                u *= changeover_K(r, rcij, inner);
            }
            dd_add(acck, u);
        }
    }
    double mi = has_i ? m[i] : 0.0;
    // m_i times the per-target sums, then a fixed-tree sum of the (hi, lo) parts
    double v[4] = {mi * acc.hi, mi * acc.lo, mi * acck.hi, mi * acck.lo};
    block_sum<4>(v, sh);
    if (t == 0)
        for (int w = 0; w < 4; ++w)
            dpart[(size_t)blockIdx.x * 4 + w] = v[w];
}

__global__ void k_diag_bodies(const RBlk *__restrict__ rblk, const double *__restrict__ m0,
                              const double *__restrict__ m, const double *__restrict__ qx,
                              const double *__restrict__ qy, const double *__restrict__ qz,
                              const double *__restrict__ vx, const double *__restrict__ vy,
                              const double *__restrict__ vz, double *__restrict__ bpart)
{
    __shared__ double sh[8 * kBlock];
    RBlk b = rblk[blockIdx.x];
    int i = b.start + threadIdx.x;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i < b.end) {
        double mi = m[i];
        double x = qx[i], y = qy[i], z = qz[i], u = vx[i], w = vy[i], s = vz[i];
        v[0] = 0.5 * mi * (u * u + w * w + s * s);
        v[1] = -m0[b.sys] * mi / sqrt(x * x + y * y + z * z);   // G applied later
        v[2] = mi * (y * s - z * w);
        v[3] = mi * (z * u - x * s);
        v[4] = mi * (x * w - y * u);
        v[5] = mi * u;
        v[6] = mi * w;
        v[7] = mi * s;
    }
    block_sum<8>(v, sh);
    if (threadIdx.x == 0)
        for (int w = 0; w < 8; ++w)
            bpart[(size_t)blockIdx.x * 8 + w] = v[w];
}

__global__ void k_diag_final(int nsys, const int *__restrict__ rb_first,
                             const int *__restrict__ rb_count, const int *__restrict__ dw_first,
                             const int *__restrict__ dw_count, const double *__restrict__ bpart,
                             const double *__restrict__ dpart, const double *__restrict__ m0,
                             double G, double *__restrict__ out)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys)
        return;
    dd q[8];
    for (int w = 0; w < 8; ++w)
        q[w] = {0.0, 0.0};
    for (int b = rb_first[s], e = b + rb_count[s]; b < e; ++b)
        for (int w = 0; w < 8; ++w)
            dd_add(q[w], bpart[(size_t)b * 8 + w]);
    dd pe = {0.0, 0.0}, pk = {0.0, 0.0};
    for (int k = dw_first[s], e = k + dw_count[s]; k < e; ++k) {
        dd_add(pe, dd{dpart[(size_t)k * 4 + 0], dpart[(size_t)k * 4 + 1]});
        dd_add(pk, dd{dpart[(size_t)k * 4 + 2], dpart[(size_t)k * 4 + 3]});
    }
    double P0 = q[5].hi + q[5].lo, P1 = q[6].hi + q[6].lo, P2 = q[7].hi + q[7].lo;
    dd base = q[0];
    dd_add(base, G * q[1].hi);
    dd_add(base, G * q[1].lo);
    dd_add(base, (P0 * P0 + P1 * P1 + P2 * P2) / (2.0 * m0[s]));
    dd e1 = base, e2 = base;
    dd_add(e1, -G * pe.hi);
    dd_add(e1, -G * pe.lo);
    dd_add(e2, -G * pk.hi);
    dd_add(e2, -G * pk.lo);
    double *o = out + (size_t)s * 8;
    o[0] = e1.hi + e1.lo;
    o[1] = e2.hi + e2.lo;
    o[2] = q[2].hi + q[2].lo;
    o[3] = q[3].hi + q[3].lo;
    o[4] = q[4].hi + q[4].lo;
    o[5] = P0;
    o[6] = P1;
    o[7] = P2;
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Resolver transfers.  k_gather_pairs packs both ends of listed pairs
// [k0, k0 + n) (n capped by the step's count and the list): per pair two
// records of 10 doubles (m0, m, rc, Q0, V0, body index); k_scatter_members
// writes rows of 7 doubles (body index, Q, V) back, skipping rows that are not
// finite (a failed group keeps its drifted state).
__global__ __launch_bounds__(kBlock) void k_gather_pairs(
    const int *__restrict__ ice, const int *__restrict__ jce, int k0, int n, int cap,
    const DevStats *__restrict__ stats, const int *__restrict__ sys_of,
    const double *__restrict__ m0, const double *__restrict__ m, const double *__restrict__ rc,
    const double *__restrict__ q0x, const double *__restrict__ q0y, const double *__restrict__ q0z,
    const double *__restrict__ v0x, const double *__restrict__ v0y, const double *__restrict__ v0z,
    double *__restrict__ out)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int k = k0 + t;
    if (t >= n || k >= min(stats->cur_nce, cap))
        return;
    const int body[2] = {ice[k], jce[k]};
    for (int e = 0; e < 2; ++e) {
        const int i = body[e];
        double *o = out + 20 * (size_t)t + 10 * e;
        o[0] = m0[sys_of[i]];
        o[1] = m[i];
        o[2] = rc[i];
        o[3] = q0x[i];
        o[4] = q0y[i];
        o[5] = q0z[i];
        o[6] = v0x[i];
        o[7] = v0y[i];
        o[8] = v0z[i];
        o[9] = (double)i;
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter_members(const double *__restrict__ rows, int k,
                                                            int ntot, double *qx, double *qy,
                                                            double *qz, double *vx, double *vy,
                                                            double *vz)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= k)
        return;
    const double *r = rows + 7 * (size_t)t;
    const double a = r[1], b = r[2], c = r[3], u = r[4], v = r[5], w = r[6];
    const int i = (int)r[0];
    if (!isfinite(a + b + c + u + v + w) || i < 0 || i >= ntot)
        return;
    qx[i] = a;
    qy[i] = b;
    qz[i] = c;
    vx[i] = u;
    vy[i] = v;
    vz[i] = w;
}

hipError_t launch_gather_pairs(const Dev &d, int k0, int n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    if (n > d.res_cap)
        return hipErrorInvalidValue;
    k_gather_pairs<<<cdiv(n, kBlock), kBlock, 0, s>>>(d.ice, d.jce, k0, n, d.enc_cap, d.stats, d.sys_of,
                                                       d.m0, d.m, d.rc, d.q0x, d.q0y, d.q0z, d.v0x,
                                                       d.v0y, d.v0z, d.res_buf);
    return hipGetLastError();
}

hipError_t launch_scatter_members(const Dev &d, int k, hipStream_t s)
{
    if (k <= 0)
        return hipSuccess;
    if (k > 2 * d.res_cap)
        return hipErrorInvalidValue;
    k_scatter_members<<<cdiv(k, kBlock), kBlock, 0, s>>>(d.res_rows, k, d.ntot, d.qx, d.qy, d.qz,
                                                          d.vx, d.vy, d.vz);
    return hipGetLastError();
}

// Tables of one system of n bodies for a force evaluation without a context:
// the O(N) blocks, the star's mass and the symmetric force's super-tile pairs
// (I <= J of nt super-tiles of ST bodies, row I's items from I nt - I (I - 1) / 2,
// in the layout the context's tables use; the order of the items does not
// change the sums, which the finalize takes in slot order).  Also clears the
// statistics block.
__global__ void k_single_tables(int n, int ST, int nt, double m0v, RBlk *__restrict__ rblk, int nrb,
                                double *__restrict__ m0, FWork *__restrict__ fw,
                                DevStats *__restrict__ stats)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nrb)
        rblk[t] = RBlk{0, t * kBlock, min(n, (t + 1) * kBlock), 0};
    if (t == 0) {
        m0[0] = m0v;
        *stats = DevStats{};
    }
    if (t < nt * nt) {
        const int I = t / nt, J = t % nt;
        if (J >= I) {
            const int at = I * nt - I * (I - 1) / 2 + (J - I);
            fw[at] = FWork{I * ST, min(ST, n - I * ST), J * ST, min(ST, n - J * ST), J, 0,
                           (J * ST) / kBlock, I};
        }
    }
}

hipError_t launch_single_tables(const Dev &d, int ST, int nt, double m0v, hipStream_t s)
{
    const int total = std::max(d.nrb, nt * nt);
    if (total <= 0)
        return hipSuccess;
    k_single_tables<<<cdiv(total, kBlock), kBlock, 0, s>>>(d.ntot, ST, nt, m0v, d.rblk, d.nrb, d.m0,
                                                           d.fwork, d.stats);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int n, int value, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    k_fill_i32<<<cdiv(n, kBlock), kBlock, 0, s>>>(p, n, value);
    return hipGetLastError();
}

hipError_t launch_validate(const Dev &d, const double *m0, const double *m, const double *x,
                           const double *v, hipStream_t s)
{
    int n = d.ntot > d.nsys ? d.ntot : d.nsys;
    k_validate<<<cdiv(n, kBlock), kBlock, 0, s>>>(d.ntot, d.nsys, m0, m, x, v, d.sys_of, d.off,
                                                   d.nbig, d.flag);
    return hipGetLastError();
}

hipError_t launch_to_dh(const Dev &d, const double *x, const double *v, int frame, hipStream_t s)
{
    if (d.nrb == 0)
        return hipSuccess;
    int helio = frame == 0;
    if (helio)
        k_partial_mv<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.m, v, v + d.ntot, v + 2 * (size_t)d.ntot,
                                               d.rpart);
    k_to_dh<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.rb_first, d.rb_count, d.m0, d.rpart, d.ntot, x, v,
                                      helio, d.qx, d.qy, d.qz, d.vx, d.vy, d.vz);
    return hipGetLastError();
}

hipError_t launch_from_dh(const Dev &d, double *x, double *v, int frame, hipStream_t s)
{
    if (d.nrb == 0)
        return hipSuccess;
    int helio = frame == 0;
    if (helio)
        k_partial_mv<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.m, d.vx, d.vy, d.vz, d.rpart);
    k_from_dh<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.rb_first, d.rb_count, d.m0, d.rpart, d.ntot,
                                        helio, d.qx, d.qy, d.qz, d.vx, d.vy, d.vz, x, v);
    return hipGetLastError();
}

hipError_t launch_momentum(const Dev &d, double *part, hipStream_t s)
{
    if (d.nrb == 0)
        return hipSuccess;
    k_partial_mv<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.m, d.vx, d.vy, d.vz, part);
    return hipGetLastError();
}

static DragP drag_params(const Params &p)
{
    DragP dp;
    dp.G = p.G;
    dp.sigma0 = p.sigma0;
    dp.h = p.h;
    dp.cd = p.cd;
    dp.rho_p = p.rho_p;
    return dp;
}

hipError_t launch_kick(const Dev &d, const Params &p, double h, hipStream_t s)
{
    if (d.nrb == 0)
        return hipSuccess;
    double *part_b = d.rpart_drift();
    if (p.drag) {
        // partial sums of m V before the kick, for the heliocentric velocity
        k_partial_mv<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.m, d.vx, d.vy, d.vz, part_b);
        k_kick<<<d.nrb, kBlock, 0, s>>>(d.rblk, h, d.m, d.ax, d.ay, d.az, d.vx, d.vy, d.vz, d.rpart,
                                         part_b, d.rb_first, d.rb_count, d.m0, d.qx, d.qy, d.qz,
                                         drag_params(p));
    } else {
        k_kick<<<d.nrb, kBlock, 0, s>>>(d.rblk, h, d.m, d.ax, d.ay, d.az, d.vx, d.vy, d.vz, d.rpart,
                                         nullptr, d.rb_first, d.rb_count, d.m0, d.qx, d.qy, d.qz,
                                         drag_params(p));
    }
    return hipGetLastError();
}

hipError_t launch_sun_drift(const Dev &d, double h, int rcrit, const Params &p, const double *part,
                            double *copy_to, hipStream_t s)
{
    if (d.nrb == 0)
        return hipSuccess;
    const bool pre = h != 0.0 && d.sys_total;
    if (pre)
        k_sys_total<<<d.nsys, kBlock, 0, s>>>(d.rb_first, d.rb_count, part, d.ptot);
    // the FP32C records over the radial order, with its tile bounds
    const bool rs = p.mode == 1 && rcrit && d.force_rsort;
    k_sun_drift<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.rb_first, d.rb_count, d.m0, part, h, d.qx,
                                          d.qy, d.qz, rcrit, d.m, p.n_hill, d.rc,
                                          p.mode == 1 ? d.pk : nullptr, d.tile_rc2, copy_to,
                                          pre ? d.ptot : nullptr, rs ? d.rord : nullptr,
                                          rs ? d.rtb : nullptr);
    return hipGetLastError();
}

hipError_t launch_drift(const Dev &d, const Params &p, double dt, double sun_h,
                        const double *part_in, hipStream_t s)
{
    if (d.nrb == 0)
        return hipSuccess;
    const bool pre = sun_h != 0.0 && d.sys_total;
    if (pre)
        k_sys_total<<<d.nsys, kBlock, 0, s>>>(d.rb_first, d.rb_count, part_in, d.ptot);
    k_drift<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.m0, p.G, dt, d.m, d.qx, d.qy, d.qz, d.vx, d.vy,
                                      d.vz, d.q0x, d.q0y, d.q0z, d.v0x, d.v0y, d.v0z, d.kflag,
                                      d.stats, d.rpart_drift(), d.rc, d.mr, d.cr,
                                      d.enc_sorted ? d.lnr_part : nullptr, d.q1x, d.q1y, d.q1z,
                                      d.v1x, d.v1y, d.v1z, d.rc1, part_in, sun_h, d.rb_first,
                                      d.rb_count, pre ? d.ptot : nullptr);
    return hipGetLastError();
}

hipError_t launch_force(const Dev &d, const Params &p, hipStream_t s)
{
    if (d.nfw == 0)
        return hipSuccess;
    if (d.force_sym) {
        // one workgroup of G waves per super-tile pair
        const int grid = std::min(d.nfw, 1 << 22);
#define NB_SYM_ARGS d.fwork, d.nfw, d.qx, d.qy, d.qz, d.m, d.rc, d.fpart, d.ntot, d.maxs, \
                    p.inner, d.stats
#define NB_SYM32_ARGS d.fwork, d.nfw, d.pk, d.qx, d.qy, d.qz, d.m, d.rc, d.fpart32, d.ntot, \
                      d.maxs, p.inner, d.stats
#define NB_RSYM32_ARGS NB_SYM32_ARGS, d.rord, d.rtb, d.rtf, d.off
#define NB_SYM_G(R_)                                                                          \
    do {                                                                                      \
        if (p.mode == 1 && d.force_rsort) {                                                   \
            if (d.sym_g == 4)                                                                 \
                k_force32c_sym<R_, 4, true><<<grid, 256, 0, s>>>(NB_RSYM32_ARGS);             \
            else if (d.sym_g == 2)                                                            \
                k_force32c_sym<R_, 2, true><<<grid, 128, 0, s>>>(NB_RSYM32_ARGS);             \
            else                                                                              \
                k_force32c_sym<R_, 1, true><<<grid, 64, 0, s>>>(NB_RSYM32_ARGS);              \
        } else if (p.mode == 1) {                                                             \
            if (d.sym_g == 4)                                                                 \
                k_force32c_sym<R_, 4><<<grid, 256, 0, s>>>(NB_SYM32_ARGS);                    \
            else if (d.sym_g == 2)                                                            \
                k_force32c_sym<R_, 2><<<grid, 128, 0, s>>>(NB_SYM32_ARGS);                    \
            else                                                                              \
                k_force32c_sym<R_, 1><<<grid, 64, 0, s>>>(NB_SYM32_ARGS);                     \
        } else {                                                                              \
            if (d.sym_g == 4)                                                                 \
                k_force64_sym<R_, 4><<<grid, 256, 0, s>>>(NB_SYM_ARGS);                       \
            else if (d.sym_g == 2)                                                            \
                k_force64_sym<R_, 2><<<grid, 128, 0, s>>>(NB_SYM_ARGS);                       \
            else                                                                              \
                k_force64_sym<R_, 1><<<grid, 64, 0, s>>>(NB_SYM_ARGS);                        \
        }                                                                                     \
    } while (0)
        if (p.force_r == 1)
            NB_SYM_G(1);
        else if (p.force_r == 4)
            NB_SYM_G(4);
        else
            NB_SYM_G(2);
#undef NB_SYM_G
#undef NB_SYM_ARGS
#undef NB_RSYM32_ARGS
#undef NB_SYM32_ARGS
        return hipGetLastError();
    }
    if (d.force_few) {
        // waves stride over the items; about 8 workgroups per CU
        const int grid = std::min(cdiv(d.nfw, kWaves), 2048);
#define NB_FEW_ARGS d.fwork, d.nfw, d.qx, d.qy, d.qz, d.m, d.rc, d.tile_rc2, d.fpart, d.ntot, d.maxs, \
                    p.inner, d.stats
#define NB_FEW32_ARGS d.fwork, d.nfw, d.pk, d.qx, d.qy, d.qz, d.m, d.rc, d.tile_rc2, d.fpart32, d.ntot, \
                      d.maxs, p.inner, d.stats
        if (p.mode == 1) {
            if (p.force_r == 1)
                k_force32c_few<1><<<grid, kBlock, 0, s>>>(NB_FEW32_ARGS);
            else if (p.force_r == 4)
                k_force32c_few<4><<<grid, kBlock, 0, s>>>(NB_FEW32_ARGS);
            else
                k_force32c_few<2><<<grid, kBlock, 0, s>>>(NB_FEW32_ARGS);
        } else {
            if (p.force_r == 1)
                k_force64_few<1><<<grid, kBlock, 0, s>>>(NB_FEW_ARGS);
            else if (p.force_r == 4)
                k_force64_few<4><<<grid, kBlock, 0, s>>>(NB_FEW_ARGS);
            else
                k_force64_few<2><<<grid, kBlock, 0, s>>>(NB_FEW_ARGS);
        }
#undef NB_FEW_ARGS
#undef NB_FEW32_ARGS
        return hipGetLastError();
    }
    if (p.mode == 1) {
        switch (p.force_r) {
        case 1:
            k_force32c<1><<<d.nfw, kBlock, 0, s>>>(d.fwork, d.pk, d.qx, d.qy, d.qz, d.m, d.rc,
                                                    d.tile_rc2, d.fpart32, d.ntot, d.maxs, p.inner, d.stats);
            break;
        case 4:
            k_force32c<4><<<d.nfw, kBlock, 0, s>>>(d.fwork, d.pk, d.qx, d.qy, d.qz, d.m, d.rc,
                                                    d.tile_rc2, d.fpart32, d.ntot, d.maxs, p.inner, d.stats);
            break;
        default:
            k_force32c<2><<<d.nfw, kBlock, 0, s>>>(d.fwork, d.pk, d.qx, d.qy, d.qz, d.m, d.rc,
                                                    d.tile_rc2, d.fpart32, d.ntot, d.maxs, p.inner, d.stats);
        }
    } else {
        switch (p.force_r) {
        case 1:
            k_force64<1><<<d.nfw, kBlock, 0, s>>>(d.fwork, d.qx, d.qy, d.qz, d.m, d.rc,
                                                   d.tile_rc2, d.fpart,
                                                   d.ntot, d.maxs, p.inner, d.stats);
            break;
        case 4:
            k_force64<4><<<d.nfw, kBlock, 0, s>>>(d.fwork, d.qx, d.qy, d.qz, d.m, d.rc,
                                                   d.tile_rc2, d.fpart,
                                                   d.ntot, d.maxs, p.inner, d.stats);
            break;
        default:
            k_force64<2><<<d.nfw, kBlock, 0, s>>>(d.fwork, d.qx, d.qy, d.qz, d.m, d.rc,
                                                   d.tile_rc2, d.fpart,
                                                   d.ntot, d.maxs, p.inner, d.stats);
        }
    }
    return hipGetLastError();
}

hipError_t launch_force_finalize(const Dev &d, const Params &p, double kick_h, int kicks,
                                 hipStream_t s, const int *ord, bool enc_count)
{
    if (d.ntot == 0)
        return hipSuccess;
    // eight slots per slice at the largest split count
    int nsl = 1;
    while (nsl < 16 && nsl * 8 < d.maxs)
        nsl *= 2;
    const int grid = cdiv(d.ntot, kFinThreads / nsl), cc = enc_count ? d.enc_cap : -1;
    // the radial order's partials are by position too
    if (!ord && d.force_rsort)
        ord = d.rord;
    if (d.fpart32)
        k_force_finalize<float><<<grid, kFinThreads, 0, s>>>(
            d.sys_of, d.nsplit, d.fpart32, d.ntot, d.maxs, d.ns_all, nsl, p.G, d.ax, d.ay, d.az,
            kick_h, kicks, d.vx, d.vy, d.vz, ord, cc, d.stats);
    else
        k_force_finalize<double><<<grid, kFinThreads, 0, s>>>(
            d.sys_of, d.nsplit, d.fpart, d.ntot, d.maxs, d.ns_all, nsl, p.G, d.ax, d.ay, d.az,
            kick_h, kicks, d.vx, d.vy, d.vz, ord, cc, d.stats);
    return hipGetLastError();
}

// Encounter check in two parts: the gather part bins the drift records and
// copies them into the sorted record array (sorted algorithm only), the test
// part tests pairs.  Both read only what the drift wrote (Q0, V0, the Q1, V1
// and rc copies, the midpoint and chord records), so the whole check may run
// beside the next S(h), force and kick.
hipError_t launch_enc_gather(const Dev &d, double dt, hipStream_t s)
{
    if (d.enc_sorted && d.nrb > 0) {
        k_cells<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.rb_first, d.rb_count, d.lnr_part,
                                          d.sys_cell_base, d.sys_cell_cnt, d.mr, d.cell_cnt,
                                          d.cell_of, d.slot_of, d.ce);
        const int nchunk = cdiv(d.ncell, kScanChunk);
        if (nchunk <= kScanSerialChunks) {
            k_cell_scan<<<1, kScanThreads, 0, s>>>(d.cell_cnt, d.cell_off, d.ncell, d.stats);
        } else {
            k_scan_sums<<<nchunk, kScanThreads, 0, s>>>(d.cell_cnt, d.ncell, d.scan_part);
            k_scan_apply<<<nchunk, kScanThreads, 0, s>>>(d.cell_cnt, d.cell_off, d.ncell,
                                                         d.scan_part, d.stats);
        }
        k_scatter<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.cell_of, d.slot_of, d.cell_off, d.ord);
        k_cell_order<<<cdiv(d.ncell, kBlock / 64), kBlock, 0, s>>>(d.cell_off, d.ncell, d.ntot, d.ord,
                                                                    d.slot_of);
        k_srec<<<cdiv(d.ntot, kBlock), kBlock, 0, s>>>(d.ntot, d.slot_of, d.sys_of, d.q0x, d.q0y, d.q0z,
                                                       d.v0x, d.v0y, d.v0z, d.q1x, d.q1y, d.q1z,
                                                       d.v1x, d.v1y, d.v1z, d.rc1, d.mr, d.cr, d.off,
                                                       d.nbig, d.srec, d.em, d.eg, dt);
    }
    return hipGetLastError();
}

hipError_t launch_enc_test(const Dev &d, double dt, hipStream_t s)
{
    if (d.enc_sorted) {
        if (d.ntile > 0) {
            k_tile_bounds<<<cdiv(d.ntile, kBlock / 64), kBlock, 0, s>>>(d.tiles, d.ntile, d.srec, dt,
                                                                         d.tileb);
            k_tile_pairs<<<cdiv(d.nunit, kTpWaves), 64 * kTpWaves, 0, s>>>(
                d.tiles, d.units, d.nunit, d.tileb, d.tpairs, d.tp_cap, d.stats);
            // one wave per kept tile pair
            int grid = std::min(std::max(1, cdiv(d.tp_cap, kBlock / 64)), 8192);
            k_enc_pairs<<<grid, kBlock, 0, s>>>(d.tiles, d.tileb, d.tpairs, d.tp_cap, d.srec, d.em, d.eg, dt,
                                                 d.keys, d.enc_cap, d.ce, d.stats);
        }
    } else if (d.enc_few) {
        if (d.nrb > 0)
            k_encounter_few<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.off, d.nbig, dt, d.mr, d.cr, d.q0x,
                                                      d.q0y, d.q0z, d.v0x, d.v0y, d.v0z, d.q1x,
                                                      d.q1y, d.q1z, d.v1x, d.v1y, d.v1z, d.rc1,
                                                      d.keys, d.enc_cap, d.ce, d.stats);
    } else if (d.new_ > 0) {
        k_encounter<<<d.new_, kBlock, 0, s>>>(d.ework, dt, d.mr, d.cr, d.q0x, d.q0y, d.q0z, d.v0x,
                                               d.v0y, d.v0z, d.q1x, d.q1y, d.q1z, d.v1x, d.v1y,
                                               d.v1z, d.rc1, d.keys, d.enc_cap, d.ce, d.stats);
    }
    k_enc_count<<<1, 64, 0, s>>>(d.enc_cap, d.stats);
    return hipGetLastError();
}

hipError_t launch_enc_prepare(const Dev &d, double dt, hipStream_t s)
{
    // the binning clears the flags, the cell scan the list count
    hipError_t e = launch_enc_gather(d, dt, s);
    if (e == hipSuccess && d.ntile > 0)
        k_tile_bounds<<<cdiv(d.ntile, kBlock / 64), kBlock, 0, s>>>(d.tiles, d.ntile, d.srec, dt,
                                                                     d.tileb);
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_force_fused(const Dev &d, const Params &p, double dt, int count, hipStream_t s)
{
    if (d.nfw > 0) {
        const int grid = std::min(d.nfw, 1 << 22);
        const EncCtx ec{d.srec, dt, d.keys, d.enc_cap, d.ce, d.stats};
#define NB_FUSED_ARGS d.fwork, d.nfw, d.ord, d.pk, d.em, d.tileb, d.tile_first, d.off, d.qx, d.qy, \
                      d.qz, d.m, d.rc, d.fpart32, d.ntot, d.maxs, p.inner, ec
#define NB_FUSED_G(R_)                                                                        \
    do {                                                                                      \
        if (d.sym_g == 4)                                                                     \
            k_force32c_fused<R_, 4><<<grid, 256, 0, s>>>(NB_FUSED_ARGS);                      \
        else if (d.sym_g == 2)                                                                \
            k_force32c_fused<R_, 2><<<grid, 128, 0, s>>>(NB_FUSED_ARGS);                      \
        else                                                                                  \
            k_force32c_fused<R_, 1><<<grid, 64, 0, s>>>(NB_FUSED_ARGS);                       \
    } while (0)
        if (p.force_r == 1)
            NB_FUSED_G(1);
        else if (p.force_r == 4)
            NB_FUSED_G(4);
        else
            NB_FUSED_G(2);
#undef NB_FUSED_G
#undef NB_FUSED_ARGS
    }
    if (count)
        k_enc_count<<<1, 64, 0, s>>>(d.enc_cap, d.stats);
    return hipGetLastError();
}

hipError_t launch_encounters(const Dev &d, double dt, hipStream_t s)
{
    // an empty list and no flags (the check may run beside the next drift, so
    // the drift does not clear them); the sorted check's binning clears the
    // flags and its scan the count
    hipError_t e = hipSuccess;
    if (!(d.enc_sorted && d.nrb > 0)) {
        e = launch_fill_i32(&d.stats->cur_nce, 1, 0, s);
        if (e == hipSuccess)
            e = launch_fill_i32(d.ce, d.ntot, 0, s);
    }
    if (e == hipSuccess)
        e = launch_enc_gather(d, dt, s);
    return e != hipSuccess ? e : launch_enc_test(d, dt, s);
}

hipError_t launch_enc_sort(const Dev &d, int accumulate, hipStream_t s)
{
    k_enc_sort<<<1, kSortThreads, 0, s>>>(d.keys, d.keys_p2, d.enc_cap, d.ice, d.jce, d.stats,
                                          accumulate);
    return hipGetLastError();
}

hipError_t launch_persistent_steps(const Dev &d, const Params &p, double dt, int nsteps,
                                   hipStream_t s)
{
    if (d.npsys == 0 || nsteps <= 0)
        return hipSuccess;
    // workgroup size from the largest system (psys[0] after the largest-first order)
#define NB_PERSIST_ARGS                                                                         \
    d.psys, nsteps, dt, p.G, p.n_hill, p.inner, p.drag, drag_params(p), d.m0, d.m, d.qx, d.qy, \
        d.qz, d.vx, d.vy, d.vz, d.ax, d.ay, d.az, d.rc, d.q0x, d.q0y, d.q0z, d.v0x, d.v0y,     \
        d.v0z, d.kflag, d.ce, d.mr, d.keys, d.enc_cap, d.stats, d.step_nce
    // (512 threads at most: 8 waves keep the full register budget without spills)
    if (d.pmax_n <= 128)
        k_steps_persistent<128><<<d.npsys, 128, 0, s>>>(NB_PERSIST_ARGS);
    else if (d.pmax_n <= 256)
        k_steps_persistent<256><<<d.npsys, 256, 0, s>>>(NB_PERSIST_ARGS);
    else
        k_steps_persistent<512><<<d.npsys, 512, 0, s>>>(NB_PERSIST_ARGS);
#undef NB_PERSIST_ARGS
    return hipGetLastError();
}

hipError_t launch_step_stats(const Dev &d, int nsteps, hipStream_t s)
{
    k_step_stats<<<1, kBlock, 0, s>>>(d.step_nce, nsteps, d.enc_cap, d.stats);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Collisions, star impacts, ejections and the removal of lost bodies (Sec.
// 2.1.1: physical radii, removal of lost bodies from the arrays; Sec. 2.1.2:
// planet-planet and planet-star collisions, ejections of bodies far from the
// star).  The paper gives the events and their schedule, not their arithmetic;
// the readings: physical radius R = (3 m/(4 pi rho))^(1/3); a star impact when
// the step's Kepler arc comes within r_star of the star (its mass joins the
// star, whose centre moves to the centre of mass of star and impactors); a
// collision when a flagged pair's minimum separation over the step (the
// encounter predicate's Hermite minimum) is at most R_i + R_j, bodies joined
// by colliding pairs merging perfectly into the smallest index; an ejection
// beyond r_eject, the body leaving with its momentum.  Applied in that order,
// on the state at the end of the step.  Lost bodies keep their slot with
// m = 0 and a nonzero flag until the compaction.
// ----------------------------------------------------------------------------
// Closest approach to the star along the Kepler arc of duration tau from
// (q0, v0) to (q1, v1), mu = G m0: the nearer end, or the pericentre distance
// h^2/(mu (1 + e)) when the arc passes a pericentre (bound orbits: a multiple
// of 2 pi between the mean anomalies at the ends; unbound orbits: the radial
// velocity changes sign from inward to outward along the direction of time).
__device__ double star_min_dist(double mu, double tau, const double (&q0)[3], const double (&v0)[3],
                                const double (&q1)[3], const double (&v1)[3])
{
    const double r0 = sqrt(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2]);
    const double r1 = sqrt(q1[0] * q1[0] + q1[1] * q1[1] + q1[2] * q1[2]);
    double rmin = fmin(r0, r1);
    const double eta0 = q0[0] * v0[0] + q0[1] * v0[1] + q0[2] * v0[2];
    const double eta1 = q1[0] * v1[0] + q1[1] * v1[1] + q1[2] * v1[2];
    const double hx = q0[1] * v0[2] - q0[2] * v0[1];
    const double hy = q0[2] * v0[0] - q0[0] * v0[2];
    const double hz = q0[0] * v0[1] - q0[1] * v0[0];
    const double h2 = hx * hx + hy * hy + hz * hz;
    const double vv = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
    const double alpha = 2.0 / r0 - vv / mu;        // 1/a
    const double e2 = 1.0 - h2 * alpha / mu;
    const double e = sqrt(fmax(e2, 0.0));
    bool passed;
    if (alpha > 0.0) {
        const double twopi = 6.283185307179586;
        const double esinE = eta0 * sqrt(alpha / mu), ecosE = 1.0 - r0 * alpha;
        const double M0 = atan2(esinE, ecosE) - esinE;
        const double M1 = M0 + sqrt(mu * alpha * alpha * alpha) * tau;
        const double lo = fmin(M0, M1), hi = fmax(M0, M1);
        passed = floor(hi / twopi) * twopi >= lo;
    } else {
        passed = tau >= 0.0 ? (eta0 < 0.0 && eta1 >= 0.0) : (eta1 < 0.0 && eta0 >= 0.0);
    }
    if (passed)
        rmin = fmin(rmin, h2 / (mu * (1.0 + e)));
    return rmin;
}

// Star impacts, per body: lost = 1 when the arc reaches r_star (r_star > 0);
// every flag cleared otherwise and every union-find parent set to the body.
// Per-block sums of the impactors' m, m Q and count into part (8 per block).
__global__ void k_ev_star(const RBlk *__restrict__ rblk, const double *__restrict__ m0, double G,
                          double tau, Snap a, const double *__restrict__ m,
                          const double *__restrict__ qx, const double *__restrict__ qy,
                          const double *__restrict__ qz, double r_star, int *__restrict__ lost,
                          int *__restrict__ root, double *__restrict__ part)
{
    __shared__ double sh[8 * kBlock / 64];
    const RBlk b = rblk[blockIdx.x];
    const int i = b.start + threadIdx.x;
    double w[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < b.end) {
        int flag = 0;
        if (r_star > 0.0) {
            const double q0[3] = {a.q0x[i], a.q0y[i], a.q0z[i]}, v0[3] = {a.v0x[i], a.v0y[i], a.v0z[i]};
            const double q1[3] = {a.q1x[i], a.q1y[i], a.q1z[i]}, v1[3] = {a.v1x[i], a.v1y[i], a.v1z[i]};
            flag = star_min_dist(G * m0[b.sys], tau, q0, v0, q1, v1) <= r_star;
        }
        lost[i] = flag;
        root[i] = i;
        if (flag) {
            const double mi = m[i];
            w[0] = mi;
            w[1] = mi * qx[i];
            w[2] = mi * qy[i];
            w[3] = mi * qz[i];
            w[4] = 1.0;
        }
    }
    block_sum<5>(w, sh);
    if (threadIdx.x < 5)
        part[(size_t)blockIdx.x * 8 + threadIdx.x] = w[threadIdx.x];
}

// One workgroup per system: the impactors join the star (m0 += their mass) and
// the star's centre moves to the centre of mass of star and impactors; the
// shift is kept in sys[8 s .. 8 s + 2] for the bodies.  cnt[0] += impacts.
__global__ void k_ev_star_sys(const int *__restrict__ rb_first, const int *__restrict__ rb_count,
                              const double *__restrict__ part, double *__restrict__ m0,
                              double *__restrict__ sys, int *__restrict__ cnt)
{
    __shared__ double sh[8 * kBlock / 64];
    double t[5];
    system_sum<5>(part + 0, 8, rb_first[blockIdx.x], rb_count[blockIdx.x], t, sh);
    if (threadIdx.x == 0) {
        double *o = sys + (size_t)blockIdx.x * 8;
        o[0] = o[1] = o[2] = 0.0;
        const int k = (int)t[4];
        if (k > 0) {
            const double mnew = m0[blockIdx.x] + t[0];
            o[0] = t[1] / mnew;
            o[1] = t[2] / mnew;
            o[2] = t[3] / mnew;
            m0[blockIdx.x] = mnew;
            atomicAdd(&cnt[0], k);
        }
        o[3] = (double)k;
    }
}

// Impactors lose their mass; every other body of a system with impacts moves
// by minus the star's shift (its heliocentric position is relative to the star).
__global__ void k_ev_star_apply(const RBlk *__restrict__ rblk, const double *__restrict__ sys,
                                const int *__restrict__ lost, double *__restrict__ m,
                                double *__restrict__ qx, double *__restrict__ qy,
                                double *__restrict__ qz)
{
    const RBlk b = rblk[blockIdx.x];
    const int i = b.start + threadIdx.x;
    if (i >= b.end)
        return;
    const double *o = sys + (size_t)b.sys * 8;
    if (o[3] == 0.0)
        return;
    if (lost[i]) {
        m[i] = 0.0;
    } else {
        qx[i] -= o[0];
        qy[i] -= o[1];
        qz[i] -= o[2];
    }
}

__device__ int uf_find(int *root, int i)
{
    while (root[i] != i)
        i = root[i];
    return i;
}

// Collisions among the step's listed pairs (sorted by (i, j); pairs with a
// lost member are skipped).  Every thread tests pairs: the Hermite minimum of
// the step's arcs against (R_i + R_j)^2.  Then thread 0 joins colliding pairs
// (union-find, the smaller root wins), lists the members in index order and
// merges every group into its smallest member: summed mass, mass-weighted
// position and velocity (compensated sums in index order); the others get
// lost = 2 and m = 0.  One workgroup; collisions are rare, and the member
// list is ordered by insertion (quadratic in the members of colliding pairs).
__global__ __launch_bounds__(kBlock) void k_ev_collide(
    const DevStats *__restrict__ stats, int cap, const int *__restrict__ ice,
    const int *__restrict__ jce, double tau, Snap a, double rho, int *__restrict__ lost,
    int *__restrict__ root, int *__restrict__ pflag, int *__restrict__ mem, double *m, double *qx,
    double *qy, double *qz, double *vx, double *vy, double *vz, int *__restrict__ cnt)
{
    const int nce = min(stats->cur_nce, cap);
    const double k3 = 3.0 / (4.0 * 3.141592653589793 * rho);
    const double t2 = 2.0 * tau;
    for (int p = threadIdx.x; p < nce; p += blockDim.x) {
        const int i = ice[p], j = jce[p];
        int hit = 0;
        if (!lost[i] && !lost[j]) {
            const double d0x = a.q0x[j] - a.q0x[i], d0y = a.q0y[j] - a.q0y[i], d0z = a.q0z[j] - a.q0z[i];
            const double d1x = a.q1x[j] - a.q1x[i], d1y = a.q1y[j] - a.q1y[i], d1z = a.q1z[j] - a.q1z[i];
            const double e0x = a.v0x[j] - a.v0x[i], e0y = a.v0y[j] - a.v0y[i], e0z = a.v0z[j] - a.v0z[i];
            const double e1x = a.v1x[j] - a.v1x[i], e1y = a.v1y[j] - a.v1y[i], e1z = a.v1z[j] - a.v1z[i];
            const double f0 = d0x * d0x + d0y * d0y + d0z * d0z;
            const double f1 = d1x * d1x + d1y * d1y + d1z * d1z;
            const double g0 = t2 * (d0x * e0x + d0y * e0y + d0z * e0z);
            const double g1 = t2 * (d1x * e1x + d1y * e1y + d1z * e1z);
            const double rr = cbrt(k3 * m[i]) + cbrt(k3 * m[j]);
            hit = hermite_min(f0, f1, g0, g1) <= rr * rr;
        }
        pflag[p] = hit;
    }
    __syncthreads();
    if (threadIdx.x != 0)
        return;
    int ncoll = 0, nm = 0;
    for (int p = 0; p < nce; ++p) {
        if (!pflag[p])
            continue;
        ++ncoll;
        const int i = ice[p], j = jce[p];
        const int ra = uf_find(root, i), rb = uf_find(root, j);
        if (ra != rb) {
            if (ra < rb)
                root[rb] = ra;
            else
                root[ra] = rb;
        }
        // members in increasing index order, each once
        for (int e = 0; e < 2; ++e) {
            const int b = e ? j : i;
            int k = nm;
            while (k > 0 && mem[k - 1] > b)
                --k;
            if (k > 0 && mem[k - 1] == b)
                continue;
            for (int q = nm; q > k; --q)
                mem[q] = mem[q - 1];
            mem[k] = b;
            ++nm;
        }
    }
    int merged = 0;
    for (int e = 0; e < nm; ++e) {
        const int r = mem[e];
        if (uf_find(root, r) != r)
            continue;
        dd sm{0, 0}, px{0, 0}, py{0, 0}, pz{0, 0}, ux{0, 0}, uy{0, 0}, uz{0, 0};
        for (int f = e; f < nm; ++f) {
            const int b = mem[f];
            if (uf_find(root, b) != r)
                continue;
            const double mb = m[b];
            dd_add(sm, mb);
            dd_add(px, mb * qx[b]);
            dd_add(py, mb * qy[b]);
            dd_add(pz, mb * qz[b]);
            dd_add(ux, mb * vx[b]);
            dd_add(uy, mb * vy[b]);
            dd_add(uz, mb * vz[b]);
        }
        const double M = sm.hi + sm.lo;
        if (M > 0.0) {
            qx[r] = (px.hi + px.lo) / M;
            qy[r] = (py.hi + py.lo) / M;
            qz[r] = (pz.hi + pz.lo) / M;
            vx[r] = (ux.hi + ux.lo) / M;
            vy[r] = (uy.hi + uy.lo) / M;
            vz[r] = (uz.hi + uz.lo) / M;
        }
        m[r] = M;
        for (int f = e + 1; f < nm; ++f) {
            const int b = mem[f];
            if (uf_find(root, b) == r) {
                lost[b] = 2;
                m[b] = 0.0;
                ++merged;
            }
        }
    }
    cnt[1] += ncoll;
    cnt[2] += merged;
}

// Ejections, per body not lost: lost = 3 beyond r_eject.  Per-block sums of
// the mass of the bodies not lost before this check, of the ejected mass, of
// the ejected momentum and of the count.
__global__ void k_ev_eject(const RBlk *__restrict__ rblk, double r_eject, int *__restrict__ lost,
                           const double *__restrict__ m, const double *__restrict__ qx,
                           const double *__restrict__ qy, const double *__restrict__ qz,
                           const double *__restrict__ vx, const double *__restrict__ vy,
                           const double *__restrict__ vz, double *__restrict__ part)
{
    __shared__ double sh[8 * kBlock / 64];
    const RBlk b = rblk[blockIdx.x];
    const int i = b.start + threadIdx.x;
    double w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < b.end && !lost[i]) {
        const double mi = m[i];
        w[0] = mi;
        const double r = sqrt(qx[i] * qx[i] + qy[i] * qy[i] + qz[i] * qz[i]);
        if (r > r_eject) {
            lost[i] = 3;
            w[1] = mi;
            w[2] = mi * vx[i];
            w[3] = mi * vy[i];
            w[4] = mi * vz[i];
            w[5] = 1.0;
        }
    }
    block_sum<6>(w, sh);
    if (threadIdx.x < 6)
        part[(size_t)blockIdx.x * 8 + threadIdx.x] = w[threadIdx.x];
}

// One workgroup per system: the ejected momentum leaves, so the barycentric
// velocities of the rest change by dv = sum m_e V_e / (m0 + sum m - sum m_e).
__global__ void k_ev_eject_sys(const int *__restrict__ rb_first, const int *__restrict__ rb_count,
                               const double *__restrict__ part, const double *__restrict__ m0,
                               double *__restrict__ sys, int *__restrict__ cnt)
{
    __shared__ double sh[8 * kBlock / 64];
    double t[6];
    system_sum<6>(part, 8, rb_first[blockIdx.x], rb_count[blockIdx.x], t, sh);
    if (threadIdx.x == 0) {
        double *o = sys + (size_t)blockIdx.x * 8;
        const int k = (int)t[5];
        o[0] = o[1] = o[2] = 0.0;
        if (k > 0) {
            const double rest = (m0[blockIdx.x] + t[0]) - t[1];
            o[0] = t[2] / rest;
            o[1] = t[3] / rest;
            o[2] = t[4] / rest;
            atomicAdd(&cnt[3], k);
        }
        o[3] = (double)k;
    }
}

__global__ void k_ev_eject_apply(const RBlk *__restrict__ rblk, const double *__restrict__ sys,
                                 const int *__restrict__ lost, double *__restrict__ m,
                                 double *__restrict__ vx, double *__restrict__ vy,
                                 double *__restrict__ vz)
{
    const RBlk b = rblk[blockIdx.x];
    const int i = b.start + threadIdx.x;
    if (i >= b.end)
        return;
    const double *o = sys + (size_t)b.sys * 8;
    if (o[3] == 0.0)
        return;
    const int f = lost[i];
    if (f == 3) {
        m[i] = 0.0;
    } else if (f == 0) {
        vx[i] += o[0];
        vy[i] += o[1];
        vz[i] += o[2];
    }
}

// Order-preserving compaction of the bodies with lost == 0: per-block kept
// counts, their exclusive scan over all blocks (systems are contiguous, so
// the scan is also each system's), then every kept body to its place.
__global__ void k_cmp_count(const RBlk *__restrict__ rblk, const int *__restrict__ lost,
                            int *__restrict__ kept)
{
    __shared__ int sh[kBlock / 64];
    const RBlk b = rblk[blockIdx.x];
    const int i = b.start + threadIdx.x;
    const int k = __popcll(__ballot(i < b.end && lost[i] == 0));
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = k;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kBlock / 64; ++w)
            t += sh[w];
        kept[blockIdx.x] = t;
    }
}

// pos[b] = kept[0] + ... + kept[b-1], pos[n] = the total (one workgroup).
__global__ void k_cmp_scan(int n, const int *__restrict__ kept, int *__restrict__ pos)
{
    __shared__ int sh[kBlock];
    int carry = 0;
    for (int b0 = 0; b0 < n; b0 += kBlock) {
        const int b = b0 + threadIdx.x;
        const int v = b < n ? kept[b] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        // inclusive Hillis-Steele scan of the chunk
        for (int o = 1; o < kBlock; o <<= 1) {
            const int t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (b < n)
            pos[b] = carry + sh[threadIdx.x] - v;
        carry += sh[kBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        pos[n] = carry;
}

// out: 7 planes of ntot (m, Q, V); idx[k] = the old index of kept body k.
__global__ void k_cmp_scatter(const RBlk *__restrict__ rblk, const int *__restrict__ lost,
                              const int *__restrict__ pos, int ntot, const double *__restrict__ m,
                              const double *__restrict__ qx, const double *__restrict__ qy,
                              const double *__restrict__ qz, const double *__restrict__ vx,
                              const double *__restrict__ vy, const double *__restrict__ vz,
                              double *__restrict__ out, int *__restrict__ idx)
{
    __shared__ int sh[kBlock / 64];
    const RBlk b = rblk[blockIdx.x];
    const int i = b.start + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool keep = i < b.end && lost[i] == 0;
    const unsigned long long mask = __ballot(keep);
    if (lane == 0)
        sh[wv] = __popcll(mask);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wv; ++w)
        before += sh[w];
    if (!keep)
        return;
    const int o = pos[blockIdx.x] + before + (int)__popcll(mask & ((1ull << lane) - 1ull));
    const size_t n = (size_t)ntot;
    out[o] = m[i];
    out[n + o] = qx[i];
    out[2 * n + o] = qy[i];
    out[3 * n + o] = qz[i];
    out[4 * n + o] = vx[i];
    out[5 * n + o] = vy[i];
    out[6 * n + o] = vz[i];
    idx[o] = i;
}

hipError_t launch_events(const Dev &d, const Params &p, double tau, double rho, double r_star,
                         double r_eject, hipStream_t s)
{
    if (d.nrb == 0)
        return hipSuccess;
    const Snap a = d.snap();
    k_fill_i32<<<1, 64, 0, s>>>(d.evcnt, 4, 0);
    k_ev_star<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.m0, p.G, tau, a, d.m, d.qx, d.qy, d.qz, r_star,
                                        d.lost, d.evroot, d.evpart);
    k_ev_star_sys<<<d.nsys, kBlock, 0, s>>>(d.rb_first, d.rb_count, d.evpart, d.m0, d.evsys,
                                             d.evcnt);
    k_ev_star_apply<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.evsys, d.lost, d.m, d.qx, d.qy, d.qz);
    k_ev_collide<<<1, kBlock, 0, s>>>(d.stats, d.enc_cap, d.ice, d.jce, tau, a, rho, d.lost,
                                       d.evroot, d.evflag, d.evmem, d.m, d.qx, d.qy, d.qz, d.vx,
                                       d.vy, d.vz, d.evcnt);
    if (r_eject > 0.0) {
        k_ev_eject<<<d.nrb, kBlock, 0, s>>>(d.rblk, r_eject, d.lost, d.m, d.qx, d.qy, d.qz, d.vx,
                                             d.vy, d.vz, d.evpart);
        k_ev_eject_sys<<<d.nsys, kBlock, 0, s>>>(d.rb_first, d.rb_count, d.evpart, d.m0, d.evsys,
                                                  d.evcnt);
        k_ev_eject_apply<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.evsys, d.lost, d.m, d.vx, d.vy, d.vz);
    }
    return hipGetLastError();
}

hipError_t launch_compact(const Dev &d, double *out, int *idx, hipStream_t s)
{
    if (d.nrb == 0)
        return hipSuccess;
    k_cmp_count<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.lost, d.evflag);
    k_cmp_scan<<<1, kBlock, 0, s>>>(d.nrb, d.evflag, d.cmp_pos);
    k_cmp_scatter<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.lost, d.cmp_pos, d.ntot, d.m, d.qx, d.qy,
                                            d.qz, d.vx, d.vy, d.vz, out, idx);
    return hipGetLastError();
}

hipError_t launch_diagnostics(const Dev &d, const Params &p, hipStream_t s)
{
    if (d.ndw > 0)
        k_diag_pairs<<<d.ndw, kBlock, 0, s>>>(d.dwork, d.qx, d.qy, d.qz, d.m, d.rc, p.inner,
                                               d.dpart);
    if (d.nrb > 0)
        k_diag_bodies<<<d.nrb, kBlock, 0, s>>>(d.rblk, d.m0, d.m, d.qx, d.qy, d.qz, d.vx, d.vy,
                                                d.vz, d.bpart);
    const int *dw_first = d.nsplit + d.nsys;      // laid out after nsplit by the runtime
    const int *dw_count = dw_first + d.nsys;
    k_diag_final<<<cdiv(d.nsys, 64), 64, 0, s>>>(d.nsys, d.rb_first, d.rb_count, dw_first,
                                                  dw_count, d.bpart, d.dpart, d.m0, p.G, d.diag);
    return hipGetLastError();
}

}  // namespace nb
