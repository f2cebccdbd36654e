// Host-side check of the request loop's admission state machine (paper_2212_09807_amd/csrc/admission.hpp) under fake
// device-memory budgets: built and run by tests/test_admission_cpu.py.  A simulated lane repeatedly takes the queue's
// head events (batch limit 16), "sizes" a tentative batch with a fake need model (fixed pool + bytes per event) and
// runs it through the same decision, shrink and requeue code the library's lanes use.  Prints one line per scenario:
// name, then the batches run (event ids) and the rejected events, for the Python test to check.
#include <algorithm>
#include <cstdio>
#include <deque>
#include <string>
#include <vector>

#include "admission.hpp"

using namespace ltsim;

struct Scenario {
    std::string name;
    std::vector<long long> ev_bytes;   // device bytes each event needs
    long long fixed;                   // bytes of the pool independent of the events
    long long share, free_bytes, reserve;
};

static void run(const Scenario &sc) {
    std::deque<int> q;
    for (int i = 0; i < (int)sc.ev_bytes.size(); ++i) q.push_back(i);
    std::printf("%s", sc.name.c_str());
    int guard = 0;
    while (!q.empty() && ++guard < 1000) {
        std::vector<int> batch;
        while (!q.empty() && batch.size() < 16) {
            batch.push_back(q.front());
            q.pop_front();
        }
        long long ran_total = -1;
        const int ran = admission_loop((int32_t)batch.size(), [&](int32_t k) {
            long long total = sc.fixed;
            for (int e = 0; e < k; ++e) total += sc.ev_bytes[batch[e]];
            const Admit a = admit_decision(k, total, total, sc.share, sc.free_bytes, sc.reserve);
            if (a == Admit::Run) ran_total = total;
            return a;
        });
        if (ran == 0) {                                   // head rejected: it leaves, the rest go back
            std::printf(" reject:%d", batch[0]);
            requeue_tail(q, batch, 1);
            continue;
        }
        requeue_tail(q, batch, (size_t)ran);
        std::printf(" run:");
        for (size_t e = 0; e < batch.size(); ++e) std::printf("%s%d", e ? "," : "", batch[e]);
        std::printf("@%lld", ran_total);
    }
    std::printf("\n");
}

// Two kinds of buffer (e.g. charge cells and summed columns): an event needs (a, b) bytes of them, the lane's pool
// keeps each kind at the largest size a batch needed, and a batch's footprint is fixed + max(pool_a, sum a) +
// max(pool_b, sum b).  release() empties the pool.  Prints the batches run (event ids) and rejected events.
static void run_pool(const char *name, const std::vector<std::pair<long long, long long>> &ev, long long fixed,
                     long long share) {
    std::deque<int> q;
    for (int i = 0; i < (int)ev.size(); ++i) q.push_back(i);
    long long pool_a = 0, pool_b = 0;
    int releases = 0;
    std::printf("%s", name);
    while (!q.empty()) {
        std::vector<int> batch;
        while (!q.empty() && batch.size() < 16) {
            batch.push_back(q.front());
            q.pop_front();
        }
        const int ran = admission_loop(
            (int32_t)batch.size(),
            [&](int32_t k) {
                long long a = 0, b = 0;
                for (int e = 0; e < k; ++e) {
                    a += ev[batch[e]].first;
                    b += ev[batch[e]].second;
                }
                const long long na = std::max(pool_a, a), nb = std::max(pool_b, b);
                const Admit d = admit_decision(k, fixed + na + nb, 0, share, 1ll << 50, 0);
                if (d == Admit::Run) {
                    pool_a = na;
                    pool_b = nb;
                }
                return d;
            },
            [&] {
                if (pool_a == 0 && pool_b == 0) return false;
                pool_a = pool_b = 0;
                ++releases;
                return true;
            });
        if (ran == 0) {
            std::printf(" reject:%d", batch[0]);
            requeue_tail(q, batch, 1);
            continue;
        }
        requeue_tail(q, batch, (size_t)ran);
        std::printf(" run:");
        for (size_t e = 0; e < batch.size(); ++e) std::printf("%s%d", e ? "," : "", batch[e]);
        std::printf("@%lld", fixed + pool_a + pool_b);
    }
    std::printf(" released:%d\n", releases);
}

int main() {
    const long long MB = 1 << 20;
    std::vector<long long> uniform(20, 100 * MB);
    run({"all_fit", uniform, 50 * MB, 4000 * MB, 64000 * MB, 1000 * MB});
    run({"budget_5", uniform, 50 * MB, 560 * MB, 64000 * MB, 1000 * MB});
    run({"free_memory_3", uniform, 50 * MB, 4000 * MB, 1360 * MB, 1000 * MB});
    std::vector<long long> big_head = uniform;
    big_head[0] = 5000 * MB;
    big_head[7] = 5000 * MB;
    run({"big_events", big_head, 50 * MB, 4000 * MB, 64000 * MB, 1000 * MB});
    std::vector<long long> mixed = {10 * MB, 900 * MB, 20 * MB, 30 * MB, 700 * MB, 5 * MB, 5 * MB, 1500 * MB,
                                    60 * MB, 400 * MB, 2 * MB, 800 * MB};
    run({"mixed", mixed, 50 * MB, 1000 * MB, 64000 * MB, 1000 * MB});
    run({"nothing_fits", uniform, 50 * MB, 100 * MB, 64000 * MB, 1000 * MB});
    // 16 events heavy in kind a grow the pool to 3200 MB of it; the next event needs 2000 MB of kind b and fits the
    // 4000 MB share only once the pool is released; the last one needs 5000 MB and is rejected after the release
    std::vector<std::pair<long long, long long>> two;
    for (int i = 0; i < 16; ++i) two.push_back({200 * MB, 0});
    two.push_back({0, 2000 * MB});
    two.push_back({0, 5000 * MB});
    run_pool("pool_release", two, 50 * MB, 4000 * MB);
    return 0;
}
