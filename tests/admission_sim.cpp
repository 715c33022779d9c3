// Host-side checks of the admission policy (paper_2309_07270_amd/csrc/
// xdrop_admission.h) with a model of the runtime's slots: footprint grows
// with the record capacity, capacities are powers of two from 1024.
//
//   1. an idle-slot layout that the first policy left waiting for ever: two
//      idle 32k slots, a budget of 2.5 of them, a 40k batch;
//   2. random sequences of submits and completions under tight budgets, with
//      the invariants checked after every step;
//   3. producer threads that wait for admission under one lock and a
//      condition variable, as the runtime's submit does, and run their batch
//      outside it; every batch must be admitted and complete.
//
// Built and run by tests/test_host_admission.py, plain and under
// AddressSanitizer / ThreadSanitizer (g++, no GPU).  Exit status 0 = pass.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../paper_2309_07270_amd/csrc/xdrop_admission.h"

using xd::AdmitPlan;
using xd::SlotView;

static std::atomic<int> failures{0};
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);             \
            std::fprintf(stderr, "\n");                    \
            ++failures;                                    \
        }                                                  \
    } while (0)

static uint32_t round_cap(size_t n)
{
    uint32_t c = 1024;
    while (c < n) c <<= 1;
    return c;
}

// bytes of a slot of `cap` records: per-record buffers plus a fixed part
static size_t footprint(uint32_t cap) { return (size_t)cap * 300 + ((size_t)4 << 20); }

struct Model {
    std::vector<SlotView> slots;
    size_t used = 0, budget = 0, max_slots = 8;

    // the runtime's try_admit: returns the slot index, or -1
    int admit(uint32_t n, AdmitPlan *out = nullptr)
    {
        const uint32_t cap = round_cap(n);
        const size_t need = footprint(cap);
        const AdmitPlan p = xd::plan_admission(slots, n, need, used, budget, max_slots);
        if (out) *out = p;
        switch (p.kind) {
        case AdmitPlan::kReuse:
            return p.slot;
        case AdmitPlan::kNew:
            slots.push_back(SlotView{false, cap, need});
            used += need;
            return (int)slots.size() - 1;
        case AdmitPlan::kResize:
            for (int k : p.release) {
                used -= slots[k].bytes;
                slots[k].cap = 0;
                slots[k].bytes = 0;
            }
            slots[p.slot].cap = cap;
            slots[p.slot].bytes = need;
            used += need;
            return p.slot;
        case AdmitPlan::kNone:
            break;
        }
        return -1;
    }

    bool any_busy() const
    {
        for (auto &s : slots)
            if (s.busy) return true;
        return false;
    }

    void check(const char *where) const
    {
        size_t sum = 0;
        for (auto &s : slots) sum += s.bytes;
        CHECK(sum == used, "%s: used %zu != sum of slot bytes %zu", where, used, sum);
        CHECK(used <= budget, "%s: used %zu > budget %zu", where, used, budget);
        CHECK(slots.size() <= max_slots, "%s: %zu slots", where, slots.size());
    }
};

static void layout_that_used_to_wait()
{
    Model m;
    const size_t f32 = footprint(32768);
    m.budget = f32 * 5 / 2;
    m.slots = {SlotView{false, 32768, f32}, SlotView{false, 32768, f32}};
    m.used = 2 * f32;
    m.max_slots = 8;
    CHECK(footprint(round_cap(40000)) <= m.budget, "the 40k batch must fit alone");
    AdmitPlan p;
    const int k = m.admit(40000, &p);
    CHECK(k >= 0, "a 40k batch with every slot idle must be admitted");
    CHECK(p.kind == AdmitPlan::kResize && p.release.size() == 2, "both idle slots are emptied (kind %d, %zu)",
          (int)p.kind, p.release.size());
    m.check("layout");
    CHECK(k >= 0 && m.slots[k].cap >= 40000, "re-sized slot holds the batch");
}

static void random_sequences()
{
    std::mt19937_64 rng(2309);
    for (int trial = 0; trial < 400; ++trial) {
        Model m;
        const size_t fmax = footprint(65536);
        m.budget = fmax + (size_t)(rng() % (3 * fmax));   // room for one to four large slots
        m.max_slots = 1 + rng() % 8;
        std::vector<int> busy;
        for (int step = 0; step < 300; ++step) {
            if (!busy.empty() && (rng() % 3 == 0)) {
                const size_t i = rng() % busy.size();
                m.slots[busy[i]].busy = false;
                busy.erase(busy.begin() + i);
                m.check("complete");
                continue;
            }
            const uint32_t n = 1 + (uint32_t)(rng() % 60000);
            const size_t need = footprint(round_cap(n));
            if (need > m.budget) continue;   // refused up front by the runtime (does not fit alone)
            const size_t used0 = m.used;
            const std::vector<SlotView> slots0 = m.slots;
            AdmitPlan p;
            const int k = m.admit(n, &p);
            m.check("admit");
            if (k < 0) {
                CHECK(m.any_busy(), "trial %d step %d: refused with no slot busy (n %u)", trial, step, n);
                CHECK(m.used == used0, "a refused batch releases nothing");
                continue;
            }
            CHECK(!m.slots[k].busy, "admitted to a busy slot");
            CHECK(m.slots[k].cap >= n, "slot capacity %u < %u", m.slots[k].cap, n);
            if (p.kind == AdmitPlan::kResize) {
                for (int r : p.release) CHECK(!slots0[r].busy, "released a busy slot");
                // with two or more released, each was needed: before the last
                // one was emptied the new buffers did not fit yet
                if (p.release.size() >= 2) {
                    size_t before_last = used0;
                    for (size_t q = 0; q + 1 < p.release.size(); ++q) before_last -= slots0[p.release[q]].bytes;
                    CHECK(before_last + need > m.budget, "trial %d step %d: an idle slot released without need",
                          trial, step);
                }
            }
            m.slots[k].busy = true;
            busy.push_back(k);
        }
    }
}

static void producer_threads()
{
    struct Shared {
        std::mutex mu;
        std::condition_variable cv;
        Model m;
        long done = 0;
    } sh;
    sh.m.budget = footprint(65536) * 3;
    sh.m.max_slots = 8;
    const int P = 12, per = 150;
    std::atomic<bool> stop{false};
    std::vector<std::thread> th;
    for (int p = 0; p < P; ++p) {
        th.emplace_back([&, p] {
            std::mt19937_64 rng(100 + p);
            for (int b = 0; b < per && !stop; ++b) {
                const uint32_t n = 1000 + (uint32_t)(rng() % 49001);
                int k;
                {
                    std::unique_lock<std::mutex> lk(sh.mu);
                    for (;;) {
                        k = sh.m.admit(n);
                        sh.m.check("threads");
                        if (k >= 0) break;
                        sh.cv.wait(lk);
                    }
                    sh.m.slots[k].busy = true;
                }
                std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));   // the batch runs
                {
                    std::lock_guard<std::mutex> lk(sh.mu);
                    sh.m.slots[k].busy = false;
                    ++sh.done;
                }
                sh.cv.notify_all();
            }
        });
    }
    // watchdog: every batch completes well within this bound unless admission deadlocks
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(sh.mu);
            if (sh.done == (long)P * per) break;
        }
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60)) {
            stop = true;
            CHECK(false, "admission stalled: %ld of %d batches done", sh.done, P * per);
            std::_Exit(2);   // threads may be blocked for ever; no join
        }
        std::this_thread::sleep_for(std::chrono::milliseconds(10));
    }
    for (auto &t : th) t.join();
    sh.m.check("threads end");
}

int main()
{
    layout_that_used_to_wait();
    random_sequences();
    producer_threads();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures.load());
        return 1;
    }
    std::printf("admission: all checks passed\n");
    return 0;
}
