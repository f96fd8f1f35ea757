// Host close-encounter resolver: grouping, worker pool, Bulirsch-Stoer on H0.
//
// H0 of a group (Sec. 2.1.1: inside the critical radius the interaction and
// Kepler parts of the bodies concerned are advanced by Bulirsch-Stoer):
//   H0 = sum_i [m_i |V_i|^2 / 2 - G m0 m_i / |Q_i|]
//        - sum_{i<j} G m_i m_j (1 - K(r_ij)) / r_ij,
// so dQ_i/dt = V_i and
//   dV_i/dt = -G m0 Q_i/|Q_i|^3 + sum_j G m_j [(1 - K)/r^3 + K'(r)/r^2] (Q_j - Q_i),
// K the changeover function with rc_ij = max(rc_i, rc_j) and inner edge
// `inner` rc_ij.  Integrator: Gragg's modified midpoint rule, substeps
// 2, 4, ..., 16, with polynomial extrapolation in h^2; a column's error is the
// largest per-body |dQ|/|Q| or |dV|/|V| between its two best extrapolants; a
// step is accepted at the first column with error <= tol and the next step is
// scaled by 0.94 (0.65 tol / err)^(1/(2c+1)) within [0.02, 4] (within
// [0.02, 0.5] after a rejection).
#include "nb_resolve.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>

namespace nb {

namespace {

constexpr int kCols = 8;            // extrapolation rows: 2, 4, ..., 16 substeps
constexpr int kMaxSteps = 100000;   // attempts per group before giving up

int uf_find(std::vector<int32_t> &p, int x)
{
    while (p[x] != x) {
        p[x] = p[p[x]];             // path halving
        x = p[x];
    }
    return x;
}

// Changeover K(r) and dK/dr on [inner rc, rc] (rational smooth step).
inline void changeover(double r, double rc, double inner, double &K, double &dK)
{
    const double lo = inner * rc, w = rc - lo;
    if (r >= rc) {
        K = 1.0;
        dK = 0.0;
        return;
    }
    if (r <= lo) {
        K = 0.0;
        dK = 0.0;
        return;
    }
    const double y = (r - lo) / w;
    const double q = 2.0 * y * (y - 1.0) + 1.0;
    K = y * y / q;
    dK = 2.0 * y * (1.0 - y) / (q * q * w);
}

// One group's state and scratch; layout per body b: q at 6b, v at 6b+3.
class GroupBS {
public:
    GroupBS(const Member *mem, int k, double G, double inner)
        : k_(k), n_(6 * k), G_(G), inner_(inner), m_(k), rc_(k), gm0_(k)
    {
        for (int b = 0; b < k; ++b) {
            m_[b] = mem[b].m;
            rc_[b] = mem[b].rc;
            gm0_[b] = G * mem[b].m0;
        }
        y_.resize(n_);
        for (int b = 0; b < k; ++b)
            for (int c = 0; c < 3; ++c) {
                y_[6 * b + c] = mem[b].q[c];
                y_[6 * b + 3 + c] = mem[b].v[c];
            }
        tab_.resize((size_t)kCols * n_);
        z0_.resize(n_);
        z1_.resize(n_);
        f_.resize(n_);
    }

    // Advance by tau; false when the attempt limit or a non-finite state ends it.
    bool advance(double tau, double tol, int &attempts)
    {
        double t = 0.0, H = tau;
        attempts = 0;
        while (t != tau) {
            if (++attempts > kMaxSteps)
                return false;
            const double rem = tau - t;
            const bool last = std::fabs(H) >= std::fabs(rem);
            if (last)
                H = rem;
            double fac = 0.25;
            bool ok = false;
            // In-place Aitken-Neville: before column c, row l holds T(c-1, c-1-l);
            // the midpoint result enters row c, and the sweep l = c..1 turns
            // row l-1 into T(c, c-l+1), so row 0 ends as T(c, c), row 1 as T(c, c-1).
            for (int c = 0; c < kCols; ++c) {
                const int nc = 2 * (c + 1);
                midpoint(H, nc, tab_.data() + (size_t)c * n_);
                for (int l = c; l >= 1; --l) {
                    const double r = (double)nc / (double)(2 * l);      // n_c / n_{l-1}
                    const double inv = 1.0 / (r * r - 1.0);
                    const double *hi = tab_.data() + (size_t)l * n_;
                    double *lo = tab_.data() + (size_t)(l - 1) * n_;
                    for (int e = 0; e < n_; ++e)
                        lo[e] = hi[e] + (hi[e] - lo[e]) * inv;
                }
                if (c == 0)
                    continue;
                const double err = rel_diff(tab_.data(), tab_.data() + n_) / tol;
                if (!std::isfinite(err))
                    break;
                const double g = err > 0.0 ? 0.94 * std::pow(0.65 / err, 1.0 / (2 * c + 1)) : 4.0;
                if (err <= 1.0) {
                    std::memcpy(y_.data(), tab_.data(), sizeof(double) * n_);
                    fac = std::min(4.0, std::max(0.02, g));
                    ok = true;
                    break;
                }
                fac = std::min(0.5, std::max(0.02, g));
            }
            if (ok)
                t = last ? tau : t + H;
            H *= fac;
            for (double x : y_)
                if (!std::isfinite(x))
                    return false;
        }
        return true;
    }

    const double *state() const { return y_.data(); }

private:
    // Largest per-body relative difference of positions and velocities.
    double rel_diff(const double *a, const double *b) const
    {
        double e = 0.0;
        for (int s = 0; s < 2 * k_; ++s) {
            const double *x = a + 3 * s, *y = b + 3 * s;
            const double d = std::sqrt((x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]) +
                                       (x[2] - y[2]) * (x[2] - y[2]));
            const double nx = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
            const double q = nx > 0.0 ? d / nx : d;
            if (!(q <= e))
                e = q;
        }
        return e;
    }

    // Time derivative of the state; each pair evaluated once for both bodies.
    void deriv(const double *y, double *dy) const
    {
        for (int b = 0; b < k_; ++b) {
            const double *q = y + 6 * b;
            const double r2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
            const double c = -gm0_[b] / (r2 * std::sqrt(r2));
            dy[6 * b + 0] = q[3];
            dy[6 * b + 1] = q[4];
            dy[6 * b + 2] = q[5];
            dy[6 * b + 3] = c * q[0];
            dy[6 * b + 4] = c * q[1];
            dy[6 * b + 5] = c * q[2];
        }
        for (int b = 0; b < k_; ++b) {
            const double *qb = y + 6 * b;
            for (int o = b + 1; o < k_; ++o) {
                const double *qo = y + 6 * o;
                const double dx = qo[0] - qb[0], dyy = qo[1] - qb[1], dz = qo[2] - qb[2];
                const double s2 = dx * dx + dyy * dyy + dz * dz;
                if (s2 == 0.0)
                    continue;
                const double s = std::sqrt(s2);
                double K, dK;
                changeover(s, std::max(rc_[b], rc_[o]), inner_, K, dK);
                const double w = G_ * ((1.0 - K) / (s2 * s) + dK / s2);
                const double wb = w * m_[o], wo = w * m_[b];
                dy[6 * b + 3] += wb * dx;
                dy[6 * b + 4] += wb * dyy;
                dy[6 * b + 5] += wb * dz;
                dy[6 * o + 3] -= wo * dx;
                dy[6 * o + 4] -= wo * dyy;
                dy[6 * o + 5] -= wo * dz;
            }
        }
    }

    // Gragg's modified midpoint rule over H with ns substeps, from y_ into out.
    void midpoint(double H, int ns, double *out)
    {
        const double h = H / ns, h2 = 2.0 * h;
        double *zp = z0_.data(), *z = z1_.data(), *f = f_.data();
        deriv(y_.data(), f);
        for (int e = 0; e < n_; ++e) {
            zp[e] = y_[e];
            z[e] = y_[e] + h * f[e];
        }
        for (int s = 1; s < ns; ++s) {
            deriv(z, f);
            for (int e = 0; e < n_; ++e) {
                const double zn = zp[e] + h2 * f[e];
                zp[e] = z[e];
                z[e] = zn;
            }
        }
        deriv(z, f);
        for (int e = 0; e < n_; ++e)
            out[e] = 0.5 * (z[e] + zp[e] + h * f[e]);
    }

    int k_, n_;
    double G_, inner_;
    std::vector<double> m_, rc_, gm0_, y_, tab_, z0_, z1_, f_;
};

}  // namespace

void build_groups(int npairs, const int32_t *ice, const int32_t *jce, Groups &g)
{
    g.body.clear();
    g.start.clear();
    if (npairs <= 0)
        return;
    std::vector<int32_t> nodes;
    nodes.reserve(2 * (size_t)npairs);
    for (int p = 0; p < npairs; ++p) {
        nodes.push_back(ice[p]);
        nodes.push_back(jce[p]);
    }
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    const int nn = (int)nodes.size();
    auto slot = [&](int32_t b) {
        return (int)(std::lower_bound(nodes.begin(), nodes.end(), b) - nodes.begin());
    };
    std::vector<int32_t> parent(nn);
    std::iota(parent.begin(), parent.end(), 0);
    for (int p = 0; p < npairs; ++p) {
        int a = uf_find(parent, slot(ice[p])), b = uf_find(parent, slot(jce[p]));
        if (a != b)
            parent[std::max(a, b)] = std::min(a, b);   // the smaller slot stays the root
    }
    // label = root slot (= smallest member, since slots follow body order)
    std::vector<int32_t> label(nn), count(nn, 0);
    for (int s = 0; s < nn; ++s) {
        label[s] = uf_find(parent, s);
        ++count[label[s]];
    }
    std::vector<int32_t> first(nn, -1);
    int ng = 0, pos = 0;
    for (int s = 0; s < nn; ++s)
        if (label[s] == s) {
            first[s] = pos;
            pos += count[s];
            ++ng;
        }
    g.body.resize(nn);
    g.start.resize(ng + 1);
    std::vector<int32_t> fill(first);
    for (int s = 0; s < nn; ++s)
        g.body[fill[label[s]]++] = nodes[s];
    int gi = 0;
    for (int s = 0; s < nn; ++s)
        if (label[s] == s)
            g.start[gi++] = first[s];
    g.start[ng] = nn;
}

ResolveTotals resolve_groups(const Groups &g, const Member *in, double *out, double G,
                             double inner, double tau, double tol, WorkerPool *pool)
{
    ResolveTotals tot;
    const int ng = g.count();
    tot.groups = ng;
    tot.bodies = (int)g.body.size();
    if (ng == 0)
        return tot;
    // longest first: order by size (cost ~ k^2 per substep), ties by position
    std::vector<int> order(ng);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return g.start[a + 1] - g.start[a] > g.start[b + 1] - g.start[b];
    });
    std::vector<int> steps(ng, 0);
    std::vector<char> fail(ng, 0);
    auto job = [&](int t) {
        const int gi = order[t];
        const int a = g.start[gi], k = g.start[gi + 1] - a;
        GroupBS bs(in + a, k, G, inner);
        int st = 0;
        const bool ok = bs.advance(tau, tol, st);
        steps[gi] = st;
        if (ok) {
            std::memcpy(out + 6 * (size_t)a, bs.state(), sizeof(double) * 6 * k);
        } else {
            fail[gi] = 1;
            std::fill(out + 6 * (size_t)a, out + 6 * (size_t)(a + k),
                      std::numeric_limits<double>::quiet_NaN());
        }
    };
    if (pool && ng > 1)
        pool->run(ng, job);
    else
        for (int t = 0; t < ng; ++t)
            job(t);
    for (int gi = 0; gi < ng; ++gi) {
        tot.max_group = std::max(tot.max_group, g.start[gi + 1] - g.start[gi]);
        tot.max_steps = std::max(tot.max_steps, steps[gi]);
        tot.failed += fail[gi];
    }
    return tot;
}

WorkerPool::WorkerPool(int nthreads)
{
    for (int t = 1; t < nthreads; ++t)
        threads_.emplace_back([this] { loop(); });
}

WorkerPool::~WorkerPool()
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    wake_.notify_all();
    for (auto &t : threads_)
        t.join();
}

void WorkerPool::drain()
{
    for (;;) {
        const int t = next_.fetch_add(1);
        if (t >= njobs_)
            return;
        (*job_)(t);
    }
}

void WorkerPool::loop()
{
    uint64_t seen = 0;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu_);
            wake_.wait(lk, [&] { return stop_ || epoch_ != seen; });
            if (stop_)
                return;
            seen = epoch_;
            ++busy_;
        }
        drain();
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (--busy_ == 0)
                done_.notify_all();
        }
    }
}

void WorkerPool::run(int njobs, const std::function<void(int)> &job)
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        job_ = &job;
        njobs_ = njobs;
        next_.store(0);
        ++epoch_;
    }
    wake_.notify_all();
    drain();
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return busy_ == 0; });
    job_ = nullptr;
}

}  // namespace nb
