// Host close-encounter resolver (full hybrid method).
//
// Bodies flagged by the encounter check are joined into groups (connected
// components of the pair graph).  Each group restarts from its pre-drift state
// and is advanced over the whole step by Bulirsch-Stoer under the Kepler part
// plus the (1 - K)-weighted pair part of the Hamiltonian (Sec. 2.1.1, footnote
// on the critical radius; Sec. 3 and 3.2 keep this integration on the host).
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace nb {

// One member of a group as the device hands it over: the system's star mass,
// the body's mass and critical radius, its pre-drift position and velocity.
struct Member {
    double m0, m, rc, q[3], v[3], pad;
};
static_assert(sizeof(Member) == 10 * sizeof(double), "Member is 10 doubles");

// Groups as ranges of a member array: group g owns [start[g], start[g+1]).
struct Groups {
    std::vector<int32_t> body;    // global body index of each member, grouped
    std::vector<int32_t> start;   // ngroups + 1 offsets
    int count() const { return start.empty() ? 0 : (int)start.size() - 1; }
};

// Group the bodies of a pair list (global indices; pairs never span systems).
// Members of a group are in ascending index order, groups by smallest member.
void build_groups(int npairs, const int32_t *ice, const int32_t *jce, Groups &g);

struct ResolveTotals {
    int groups = 0, bodies = 0, max_group = 0, failed = 0, max_steps = 0;
};

// Fixed pool of worker threads; run() blocks until every job index is done
// and the calling thread takes part.
class WorkerPool {
public:
    explicit WorkerPool(int nthreads);
    ~WorkerPool();
    WorkerPool(const WorkerPool &) = delete;
    WorkerPool &operator=(const WorkerPool &) = delete;
    int size() const { return (int)threads_.size() + 1; }
    void run(int njobs, const std::function<void(int)> &job);

private:
    void loop();
    void drain();
    std::vector<std::thread> threads_;
    std::mutex mu_;
    std::condition_variable wake_, done_;
    const std::function<void(int)> *job_ = nullptr;
    std::atomic<int> next_{0};
    int njobs_ = 0, busy_ = 0;
    uint64_t epoch_ = 0;
    bool stop_ = false;
};

// Advance every group by tau.  in: one Member per entry of g.body; out: the
// new position and velocity (6 doubles) per member.  A group whose
// integration fails gets its members' out rows set to NaN and is counted.
ResolveTotals resolve_groups(const Groups &g, const Member *in, double *out, double G,
                             double inner, double tau, double tol, WorkerPool *pool);

}  // namespace nb
