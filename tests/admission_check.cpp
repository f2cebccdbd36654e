// Host-side check of the request loop's admission state machine (paper_2212_09807_amd/csrc/admission.hpp) under fake
// device-memory budgets: built and run by tests/test_admission_cpu.py.  A simulated lane repeatedly takes the queue's
// head events (batch limit 16), "sizes" a tentative batch with a fake need model (fixed pool + bytes per event) and
// runs it through the same decision, shrink and requeue code the library's lanes use.  Prints one line per scenario:
// name, then the batches run (event ids) and the rejected events, for the Python test to check.
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
    return 0;
}
