// xdrop_admission.h -- which slot a batch is admitted to (host code, no HIP).
//
// A context runs each admitted batch in a slot: device buffers sized for a
// record capacity, a stream and a worker.  Admission is by HBM footprint:
// the bytes of all slots' buffers stay within the context's budget.  The
// decision is a pure function of the slots' state so that it can be tested
// on its own; the runtime applies it under the context lock.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace xd {

struct SlotView {
    bool busy;       // a batch is running in the slot
    uint32_t cap;    // record capacity of its buffers (0: empty)
    size_t bytes;    // bytes its buffers hold
};

struct AdmitPlan {
    enum Kind { kNone, kReuse, kNew, kResize };
    Kind kind = kNone;
    int slot = -1;              // kReuse, kResize: the slot that takes the batch
    std::vector<int> release;   // kResize: idle slots emptied, in order (the target among them)
};

// Admission of a batch of n records whose slot would have capacity cap and
// footprint need (bytes), with `used` bytes held by the slots now:
//   kReuse   the smallest idle slot whose capacity holds n;
//   kNew     a new slot, when the slot count and the budget allow it;
//   kResize  idle slots are emptied, largest first, until the new buffers fit
//            the budget, and the largest is re-sized for the batch (it is
//            emptied too if room was made without it).  Nothing is released
//            unless that makes room: when even emptying every idle slot
//            leaves too little, the plan is kNone and the caller waits for a
//            busy slot to finish.
// With no slot busy, a batch with need <= budget is always admitted.
inline AdmitPlan plan_admission(const std::vector<SlotView> &slots, uint32_t n, size_t need, size_t used,
                                size_t budget, size_t max_slots)
{
    AdmitPlan p;
    for (int k = 0; k < (int)slots.size(); ++k) {
        const SlotView &s = slots[k];
        if (!s.busy && s.cap >= n && (p.slot < 0 || s.cap < slots[p.slot].cap)) p.slot = k;
    }
    if (p.slot >= 0) {
        p.kind = AdmitPlan::kReuse;
        return p;
    }
    if (slots.size() < max_slots && used + need <= budget) {
        p.kind = AdmitPlan::kNew;
        return p;
    }
    std::vector<int> idle;
    size_t idle_bytes = 0;
    for (int k = 0; k < (int)slots.size(); ++k)
        if (!slots[k].busy) {
            idle.push_back(k);
            idle_bytes += slots[k].bytes;
        }
    if (idle.empty() || used - idle_bytes + need > budget) return p;
    std::stable_sort(idle.begin(), idle.end(), [&](int a, int b) { return slots[a].bytes > slots[b].bytes; });
    p.kind = AdmitPlan::kResize;
    p.slot = idle[0];
    size_t u = used;
    for (int k : idle) {
        if (u + need <= budget) break;
        u -= slots[k].bytes;
        p.release.push_back(k);
    }
    if (p.release.empty() || p.release[0] != p.slot) p.release.push_back(p.slot);
    return p;
}

}  // namespace xd
