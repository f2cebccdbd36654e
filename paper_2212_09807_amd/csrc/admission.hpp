// admission.hpp -- memory-based admission of the request loop's batches (host logic only, no device calls, so the
// state machine can be exercised on a CPU with fake budgets).
//
// A lane owns a share of the server's device-memory budget (mem_budget / n_lanes).  It takes the queue's head events
// (up to the batch limits) as a tentative batch and sizes it on the device; the sizing gives the exact bytes every
// buffer of the call needs.  The batch runs if the lane's footprint after growing to those sizes stays within its
// share and the growth fits in the device's free memory less a reserve; otherwise the batch is halved (the events
// cut off go back to the queue front, in order) and sized again.  A single event that does not fit is sized once
// more after the lane releases its pooled scratch (buffers earlier, larger batches grew), and fails with
// LTS_ERR_OOM only if it still does not fit.  The summed induction learns the size of its piece lists only half-way through a call, so a call may
// be sized (and refused) a second time there.
#pragma once

#include <algorithm>
#include <cstdint>

namespace ltsim {

enum class Admit { Run, Shrink, Reject };

// `total`: the lane's device footprint (scratch pool + outputs) if the call runs; `growth`: the part of it not yet
// allocated; `free_bytes`: device memory not allocated by anyone.
inline Admit admit_decision(int32_t k, int64_t total, int64_t growth, int64_t share, int64_t free_bytes,
                            int64_t reserve) {
    if (total <= share && growth <= std::max<int64_t>(free_bytes - reserve, 0)) return Admit::Run;
    return k > 1 ? Admit::Shrink : Admit::Reject;
}

// Batch size after a refusal: half, rounded down, at least one event.
inline int32_t admit_shrink(int32_t k) { return std::max(1, k / 2); }

// Admission of one tentative batch of k0 queued events: attempt(k) sizes the first k events as one call and returns
// the decision for it (running the call when it is Run).  When a single event is refused, release() frees the lane's
// pooled scratch and returns whether that happened (then the event is sized once more).  Returns the number of
// events that ran, or 0 if the first event alone was rejected.
template <class Attempt, class Release>
int32_t admission_loop(int32_t k0, Attempt attempt, Release release) {
    int32_t k = std::max(k0, 1);
    bool released = false;
    for (;;) {
        const Admit a = attempt(k);
        if (a == Admit::Run) return k;
        if (a == Admit::Reject || k == 1) {
            if (!released && release()) {
                released = true;
                k = 1;
                continue;
            }
            return 0;
        }
        k = admit_shrink(k);
    }
}
template <class Attempt>
int32_t admission_loop(int32_t k0, Attempt attempt) {
    return admission_loop(k0, attempt, [] { return false; });
}

// Puts batch[keep ..] back at the front of the queue, in their order, and cuts the batch to `keep` events.
template <class Queue, class Vec>
void requeue_tail(Queue &q, Vec &batch, size_t keep) {
    for (size_t e = batch.size(); e-- > keep;) q.push_front(batch[e]);
    batch.resize(keep);
}

}  // namespace ltsim
