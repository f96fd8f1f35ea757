// Exercise the host close-encounter resolver of the library (grouping, the
// Bulirsch-Stoer integration of every group, the worker pool) under the
// sanitizers (built and run by tests/test_sanitize.py).  Members are bodies on
// near-circular orbits paired into chains and cliques by a fixed pair list.
#include "nb_resolve.h"

#include <cmath>
#include <cstdio>
#include <vector>

int main()
{
    const double G = 39.476926421373, tau = 0.02;
    const int n = 24;
    std::vector<int32_t> ice, jce;
    // a chain 0-1-2-3, a clique {10, 11, 12}, a pair (20, 23), a repeated pair
    int pairs[][2] = {{0, 1}, {1, 2}, {2, 3}, {10, 11}, {10, 12}, {11, 12}, {20, 23}, {0, 1}};
    for (auto &p : pairs) {
        ice.push_back(p[0]);
        jce.push_back(p[1]);
    }
    nb::Groups g;
    nb::build_groups((int)ice.size(), ice.data(), jce.data(), g);
    std::vector<nb::Member> in(g.body.size());
    for (size_t e = 0; e < g.body.size(); ++e) {
        const int i = g.body[e];
        const double r = 1.0 + 1e-3 * i, th = 1e-3 * i, v = std::sqrt(G / r);
        in[e] = nb::Member{1.0, 1e-6, 5e-3, {r * std::cos(th), r * std::sin(th), 0.0},
                           {-v * std::sin(th), v * std::cos(th), 1e-4 * i}, 0.0};
    }
    std::vector<double> out(6 * in.size()), out2(6 * in.size());
    nb::ResolveTotals t1 = nb::resolve_groups(g, in.data(), out.data(), G, 0.1, tau, 1e-12, nullptr);
    nb::WorkerPool pool(4);
    nb::ResolveTotals t2 = nb::resolve_groups(g, in.data(), out2.data(), G, 0.1, tau, 1e-12, &pool);
    for (int rep = 0; rep < 3; ++rep)
        nb::resolve_groups(g, in.data(), out2.data(), G, 0.1, tau, 1e-12, &pool);
    bool same = out == out2;
    std::printf("%d groups, %d bodies, largest %d, failed %d; pool result %s\n", t1.groups,
                t1.bodies, t1.max_group, t1.failed, same ? "identical" : "DIFFERENT");
    return (t1.groups == 3 && t2.groups == 3 && t1.bodies == 9 && t1.failed == 0 && same) ? 0 : 2;
}
