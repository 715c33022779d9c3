// xdrop_capi.cpp -- host runtime of libxdrop.so: read store, validation,
// admission, per-slot batch pipelines, hipGraph capture, C ABI.
//
// One context owns a device-resident 2-bit read store and a pool of "slots".
// A slot is the set of device and pinned host buffers of one in-flight batch
// together with its own HIP stream and worker thread.  A submitted batch is
// admitted when a slot is free and its device footprint fits the HBM budget
// (growing or re-sizing slots as needed); the slot's worker runs the batch
// (copy-in, kernels, copy-out) and completes the ticket.  Several slots run at
// once, so batches that arrive while others are on the GPU overlap on the
// device: this is the continuous-batching serving loop that replaces the
// paper's MPI ranks taking turns on the GPU ("Method": One-to-all and
// One-to-one schedulers).
//
// Execution forms ("Method", Baseline: batches of 10,000 pairs fed one at a
// time):
//   XDROP_MODE_PLAIN       one launch sequence per 10,000-record chunk, one
//                          wavefront per extension, no reordering;
//   XDROP_MODE_PERSISTENT  the whole batch in one captured hipGraph: records
//                          are classed by drop, bucketed longest-first, and
//                          persistent work-stealing kernels drain each class.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "xdrop_admission.h"
#include "xdrop_internal.h"


using namespace xd;

namespace {

constexpr uint32_t kPlainChunk = 10000;
// admission budget when the caller gives none: room for a 4M-record batch
// (about 9.5 GB with its 8 GiB carry pool) and slots of the serving loop
// beside it, a ninth of one MI355X's 288 GB
constexpr uint64_t kDefaultBudget = 32ull << 30;
constexpr uint64_t kGuardBases = 8192 + 64;   // unused bases before and after the store (kernel loads reach 8192 bases past a read)

using clk = std::chrono::steady_clock;

double now_ms()
{
    return std::chrono::duration<double, std::milli>(clk::now().time_since_epoch()).count();
}

std::mutex g_err_mu;
std::string g_err_text;

void set_global_error(const std::string &s)
{
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_err_text = s;
}

int8_t base_code(char c)
{
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
    }
}

struct Slot;

struct Ticket {
    uint64_t id = 0;
    size_t n = 0;
    bool device = false;
    const xdrop_record *d_in = nullptr;   // device path input
    xdrop_result *out = nullptr;          // host or device output
    uint64_t *cells = nullptr;
    hipStream_t ustream = nullptr;
    Slot *slot = nullptr;
    bool done = false;
    xdrop_status status = XDROP_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    float dev_ms = 0.f;
    uint64_t total_cells = 0;
    double stage_ms[XDROP_NUM_STAGES] = {};
    uint64_t stage_cells[XDROP_NUM_STAGES] = {};
    uint64_t stage_tasks[XDROP_NUM_STAGES] = {};
    uint64_t stage_slots[XDROP_NUM_STAGES] = {};
};

struct Slot {
    uint32_t cap = 0;
    size_t bytes = 0;                 // device footprint
    void *dblock = nullptr;
    int32_t *scratch = nullptr;       // generic-kernel diagonals
    uint64_t scratch_stride = 0;
    uint32_t generic_blocks = 0;      // workgroups of the unbounded kernel
    BatchDev dev{};
    uint32_t *d_n = nullptr;          // batch size word read by the reset kernel
    xdrop_record *h_recs = nullptr;   // pinned staging
    xdrop_result *h_res = nullptr;
    uint64_t *h_cells = nullptr;
    uint32_t *h_misc = nullptr;       // [0] = n, [1] = error count
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
    std::vector<hipEvent_t> sev;      // stage boundary events, 9 per chunk (profiling)
    unsigned long long *h_stage = nullptr;   // pinned copy of the per-stage sums
    hipGraphExec_t graph[2] = {nullptr, nullptr};   // [count_cells]
    bool busy = false;
    std::shared_ptr<Ticket> job;
    std::thread worker;
    std::condition_variable cv;
};

}  // namespace

struct xdrop_ctx {
    int device = 0;
    uint32_t mode = XDROP_MODE_PERSISTENT;
    uint32_t max_inflight = 4;
    uint64_t budget = kDefaultBudget;
    uint64_t used = 0;
    int cus = 256;
    bool profile = false;

    // store
    uint32_t *d_words = nullptr;
    ReadInfo *d_reads = nullptr;
    std::vector<uint32_t> h_len;
    StoreDev st{};
    uint64_t store_bytes = 0;

    Tuning tune{};
    std::string tuning_path;

    mutable std::mutex mu;
    std::condition_variable cv;
    std::vector<std::unique_ptr<Slot>> slots;
    std::unordered_map<uint64_t, std::shared_ptr<Ticket>> tickets;
    uint64_t next_id = 1;
    bool stop = false;
    bool poisoned = false;

    // last error text: its own lock, since fail() is called both with and
    // without mu held (slot workers, submit, find_seeds)
    mutable std::mutex err_mu;
    std::string err;

    void fail(const std::string &s)
    {
        {
            std::lock_guard<std::mutex> lk(err_mu);
            err = s;
        }
        set_global_error(s);
    }
};

namespace {

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            throw std::runtime_error(std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                                 \
    } while (0)

Tuning default_tuning()
{
    Tuning t{};
    t.grow_margin = 8;
    t.shrink_margin = 6;
    t.waves_per_cu = 32;
    t.buckets = 1;
    // 256 extensions of unbounded band at once (one workgroup per CU: each
    // holds a 96 KB LDS ring); fewer when their scratch would pass 256 MiB
    t.generic_waves = 256 * kGenericBlockWaves;
    t.narrow_x = 20;
    // a smaller batch holds too few narrow extensions to hide the narrow
    // stage's tail (its longest extension), which then adds to the adaptive
    // stage's own: one wavefront per extension finishes such a batch sooner
    t.narrow_min = 100000;
    // 2048-slot class: two wavefronts share a window of 2 x 1024 slots (three
    // such wavefronts per SIMD) instead of one wavefront of 32 cells per lane
    // (one per SIMD)
    t.wide_waves = 2;
    return t;
}

bool load_tuning(const std::string &path, Tuning &t)
{
    std::ifstream f(path);
    if (!f) return false;
    std::string key;
    while (f >> key) {
        if (key == "grow_margin") {
            f >> t.grow_margin;
        } else if (key == "shrink_margin") {
            f >> t.shrink_margin;
        } else if (key == "waves_per_cu") {
            f >> t.waves_per_cu;
        } else if (key == "buckets") {
            f >> t.buckets;
        } else if (key == "generic_waves") {
            f >> t.generic_waves;
        } else if (key == "narrow_x") {
            f >> t.narrow_x;
        } else if (key == "narrow_min_records") {
            f >> t.narrow_min;
        } else if (key == "wide_waves") {
            f >> t.wide_waves;
        } else {
            std::string rest;
            std::getline(f, rest);
        }
    }
    return true;
}

bool validate_host(const xdrop_ctx *c, const xdrop_record &R, std::string &why)
{
    const uint32_t nr = (uint32_t)c->h_len.size();
    if (R.read_a >= nr || R.read_b >= nr) { why = "read id out of range"; return false; }
    const uint64_t la = c->h_len[R.read_a], lb = c->h_len[R.read_b];
    if (R.k < 1) { why = "k = 0"; return false; }
    if ((uint64_t)R.pos_a + R.k > la || (uint64_t)R.pos_b + R.k > lb) { why = "seed outside a read"; return false; }
    if (R.strand > 1) { why = "strand must be 0 or 1"; return false; }
    if (R.x < 0 || R.x > XDROP_MAX_X) { why = "x out of range"; return false; }
    if (R.match < 1 || R.match > 1024 || R.mismatch >= R.match || R.mismatch < -1024 || R.gap > -1 ||
        R.gap < -1024) {
        why = "bad weights";
        return false;
    }
    const int64_t w = (int64_t)R.match - R.mismatch - R.gap;
    if (w * (int64_t)(la + lb) > (1ll << 29)) { why = "weights too large for these read lengths"; return false; }
    return true;
}

// carry pool of a slot: 1024 words per record of capacity, at most 2 Gi
// words (8 GiB).  The c4 stress mix hands about 0.9 extensions per record
// from the adaptive to the first wide class (528 words each: a 256-slot
// window) and 0.04 from the first wide class on (2,576 words each), about
// 570 words per record; a full pool only makes the remaining hand-overs
// restart from the seed, which repeats an extension's start in a window far
// wider than its early band
uint32_t carry_words_for(uint32_t cap)
{
    return (uint32_t)std::min<uint64_t>((uint64_t)cap * 1024u, 1ull << 31);
}

size_t slot_bytes(uint32_t cap)
{
    const size_t n = cap;
    size_t b = 0;
    auto add = [&](size_t x) { b += (x + 255) & ~size_t(255); };
    add(n * sizeof(xdrop_record));
    add(n * sizeof(xdrop_result));
    add(n * sizeof(uint64_t));
    add(n * sizeof(int32_t));
    add(n);
    add(2 * n * sizeof(TaskOut));
    add((size_t)kNumClasses * 2 * n * sizeof(uint32_t));   // qbuf
    add((size_t)kNumClasses * 2 * n * sizeof(uint32_t));   // qkey
    add((size_t)kNumClasses * 2 * n * sizeof(uint32_t));   // qstate
    add((size_t)carry_words_for(cap) * sizeof(int32_t));   // carry pool
    add(CtrLayout::kWords * sizeof(uint32_t) + 64);
    add((size_t)kNumClasses * kNumBuckets * sizeof(uint32_t));
    add(kStageSumWords * sizeof(unsigned long long));
    return b;
}

// Releases every buffer of a slot and leaves it empty (cap 0, no pointers):
// an empty slot is never picked for a batch.
void free_slot_buffers(Slot &s)
{
    for (auto &g : s.graph)
        if (g) { hipGraphExecDestroy(g); g = nullptr; }
    if (s.dblock) hipFree(s.dblock);
    if (s.scratch) hipFree(s.scratch);
    if (s.h_recs) hipHostFree(s.h_recs);
    if (s.h_res) hipHostFree(s.h_res);
    if (s.h_cells) hipHostFree(s.h_cells);
    if (s.h_misc) hipHostFree(s.h_misc);
    if (s.h_stage) hipHostFree(s.h_stage);
    for (auto e : s.sev) hipEventDestroy(e);
    s.sev.clear();
    s.h_stage = nullptr;
    s.dblock = nullptr; s.scratch = nullptr; s.h_recs = nullptr; s.h_res = nullptr; s.h_cells = nullptr;
    s.h_misc = nullptr;
    s.dev = BatchDev{};
    s.d_n = nullptr;
    s.scratch_stride = 0;
    s.generic_blocks = 0;
    s.cap = 0;
    s.bytes = 0;
}

// Unbounded-kernel workgroups of a slot: the tuned count, fewer when the
// reads are so long that their scratch (three anti-diagonals of the longest
// read per workgroup, used only by bands wider than the LDS ring) would pass
// 256 MiB
uint64_t scratch_stride_of(const xdrop_ctx *c) { return ((uint64_t)c->st.max_len + 2 + 63) & ~uint64_t(63); }

uint32_t slot_generic_blocks(const xdrop_ctx *c)
{
    const uint64_t per_block = 3 * scratch_stride_of(c) * sizeof(int32_t);
    const uint64_t fit = std::max<uint64_t>(1, (256ull << 20) / per_block);
    return (uint32_t)std::min<uint64_t>(generic_blocks(c->tune.generic_waves), fit);
}

// Allocates the buffers of an empty slot for `cap` records.  All or nothing:
// on failure everything allocated here is released, the slot stays empty
// (cap 0) and the error is rethrown.
void alloc_slot_buffers_impl(xdrop_ctx *c, Slot &s, uint32_t cap);

void alloc_slot_buffers(xdrop_ctx *c, Slot &s, uint32_t cap)
{
    try {
        alloc_slot_buffers_impl(c, s, cap);
    } catch (...) {
        (void)hipGetLastError();   // an allocation failure must not linger as the stream's error
        free_slot_buffers(s);
        throw;
    }
}

void alloc_slot_buffers_impl(xdrop_ctx *c, Slot &s, uint32_t cap)
{
    // pointers are committed to the slot as they are allocated (so that a
    // failure can release them); cap and bytes only once everything exists
    s.cap = 0;
    s.bytes = 0;
    const size_t dbytes = slot_bytes(cap);
    HIP_TRY(hipMalloc(&s.dblock, dbytes));
    char *p = (char *)s.dblock;
    auto take = [&](size_t x) {
        char *q = p;
        p += (x + 255) & ~size_t(255);
        return (void *)q;
    };
    const size_t n = cap;
    s.dev.recs = (const xdrop_record *)take(n * sizeof(xdrop_record));
    s.dev.res = (xdrop_result *)take(n * sizeof(xdrop_result));
    s.dev.cells = (uint64_t *)take(n * sizeof(uint64_t));
    s.dev.seed = (int32_t *)take(n * sizeof(int32_t));
    s.dev.valid = (uint8_t *)take(n);
    s.dev.tout = (TaskOut *)take(2 * n * sizeof(TaskOut));
    s.dev.qbuf = (uint32_t *)take((size_t)kNumClasses * 2 * n * sizeof(uint32_t));
    s.dev.qkey = (uint32_t *)take((size_t)kNumClasses * 2 * n * sizeof(uint32_t));
    s.dev.qstate = (uint32_t *)take((size_t)kNumClasses * 2 * n * sizeof(uint32_t));
    s.dev.carry_words = carry_words_for(cap);
    s.dev.carry = (int32_t *)take((size_t)s.dev.carry_words * sizeof(int32_t));
    s.dev.ctr = (uint32_t *)take(CtrLayout::kWords * sizeof(uint32_t) + 64);
    s.d_n = s.dev.ctr + CtrLayout::kWords;
    s.dev.bucket_hist = (uint32_t *)take((size_t)kNumClasses * kNumBuckets * sizeof(uint32_t));
    s.dev.stage_sum = (unsigned long long *)take(kStageSumWords * sizeof(unsigned long long));
    s.dev.cap = cap;
    // unbounded-kernel scratch: three anti-diagonals per workgroup
    s.generic_blocks = slot_generic_blocks(c);
    s.scratch_stride = scratch_stride_of(c);
    const size_t sbytes = (size_t)s.generic_blocks * 3 * s.scratch_stride * sizeof(int32_t);
    HIP_TRY(hipMalloc(&s.scratch, sbytes));
    HIP_TRY(hipHostMalloc((void **)&s.h_recs, n * sizeof(xdrop_record), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&s.h_res, n * sizeof(xdrop_result), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&s.h_cells, n * sizeof(uint64_t), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&s.h_misc, 64, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&s.h_stage, kStageSumWords * sizeof(unsigned long long), hipHostMallocDefault));
    if (c->profile) {
        // plain form: one event set per chunk; persistent form: one set
        const size_t sets = c->mode == XDROP_MODE_PLAIN ? (cap + kPlainChunk - 1) / kPlainChunk : 1;
        s.sev.resize((kNumStages + 1) * sets, nullptr);
        for (auto &e : s.sev) HIP_TRY(hipEventCreate(&e));
    }
    s.cap = cap;
    s.bytes = dbytes + sbytes;
}

size_t slot_footprint(const xdrop_ctx *c, uint32_t cap)
{
    return slot_bytes(cap) + (size_t)slot_generic_blocks(c) * 3 * scratch_stride_of(c) * sizeof(int32_t);
}

uint32_t round_cap(size_t n)
{
    uint32_t c = 1024;
    while (c < n) c <<= 1;
    return c;
}

// Scratch of the unbounded-band kernel: `blocks` workgroups, three
// anti-diagonals of `stride` ints each.
struct GenericScratch {
    int32_t *base;
    uint64_t stride;
    uint32_t blocks;
};

// Kernel sequence of one batch (or chunk) on `s`.  `b` may be a view into the
// slot buffers (plain chunks); n_src non-null means "read n from device".
void enqueue_kernels(xdrop_ctx *c, const Tuning &tu, const GenericScratch &gs, const BatchDev &b, uint32_t n,
                     const uint32_t *n_src, bool persistent, bool count, hipStream_t s, hipEvent_t *ev)
{
    // ev (nullable): kNumStages + 1 stage-boundary events recorded between the
    // launches; ev[1 + k] after class k
    if (ev) HIP_TRY(hipEventRecord(ev[0], s));
    launch_reset_n(b, n_src, n, s);
    const bool stage = persistent && tu.buckets > 0;
    // the plain form runs one wavefront per extension: no narrow class
    Tuning tp = tu;
    if (!persistent) tp.narrow_x = -1;
    launch_prep(b, c->st, tp, n, stage, s);
    if (stage) launch_bucket(b, c->st, n, s);
    if (ev) HIP_TRY(hipEventRecord(ev[1], s));
    const uint32_t resident = (uint32_t)c->cus * (uint32_t)std::max(1, tu.waves_per_cu);
    if (tp.narrow_x >= 0) launch_narrow(b, c->st, tu, resident, count, s);
    if (ev) HIP_TRY(hipEventRecord(ev[2 + kNarrowClass], s));
    // plain form: one wavefront per extension
    launch_adaptive(b, c->st, tu, persistent ? resident : std::max<uint32_t>(2 * n, 4), count, s);
    if (ev) HIP_TRY(hipEventRecord(ev[2 + kAdaptiveClass], s));
    for (int w = 0; w < kWideClasses; ++w) {
        launch_wide(w, b, c->st, (uint32_t)c->cus, tu.wide_waves, count, s);
        if (ev) HIP_TRY(hipEventRecord(ev[2 + kAdaptiveClass + 1 + w], s));
    }
    launch_generic(b, c->st, gs.base, gs.stride, gs.blocks, count, s);
    if (ev) HIP_TRY(hipEventRecord(ev[2 + kGenericClass], s));
    launch_finalize(b, c->st, n, count, s);
    if (ev) HIP_TRY(hipEventRecord(ev[kNumStages], s));
}

GenericScratch slot_scratch(const Slot &sl) { return GenericScratch{sl.scratch, sl.scratch_stride, sl.generic_blocks}; }

// The persistent form's kernel sequence captured once per slot (and per cell
// counting flag); kernels read the batch size from device memory, so one
// graph serves every batch up to the slot capacity.  With profiling on, the
// stage events are captured as event-record nodes; if the runtime refuses
// that, profiling falls back to direct launches of the same kernels.
hipGraphExec_t get_graph(xdrop_ctx *c, Slot &sl, bool count)
{
    hipGraphExec_t &g = sl.graph[count ? 1 : 0];
    if (g) return g;
    hipGraph_t graph = nullptr;
    (void)hipGetLastError();   // start the capture with no stale error
    HIP_TRY(hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_kernels(c, c->tune, slot_scratch(sl), sl.dev, sl.cap, sl.d_n, true, count, sl.stream, nullptr);
    } catch (...) {
        hipStreamEndCapture(sl.stream, &graph);
        if (graph) hipGraphDestroy(graph);
        hipGetLastError();
        throw;
    }
    HIP_TRY(hipStreamEndCapture(sl.stream, &graph));
    const hipError_t e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
        g = nullptr;
        throw std::runtime_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    return g;
}

void run_batch(xdrop_ctx *c, Slot &sl, Ticket &t)
{
    const uint32_t n = (uint32_t)t.n;
    hipStream_t s = (t.device && t.ustream) ? t.ustream : sl.stream;
    const bool count = t.cells != nullptr;
    HIP_TRY(hipSetDevice(c->device));
    if (t.device)
        HIP_TRY(hipMemcpyAsync((void *)sl.dev.recs, t.d_in, (size_t)n * sizeof(xdrop_record), hipMemcpyDeviceToDevice, s));
    else
        HIP_TRY(hipMemcpyAsync((void *)sl.dev.recs, sl.h_recs, (size_t)n * sizeof(xdrop_record), hipMemcpyHostToDevice, s));
    sl.h_misc[0] = n;
    HIP_TRY(hipMemcpyAsync(sl.d_n, sl.h_misc, sizeof(uint32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(sl.ev0, s));
    if (c->mode == XDROP_MODE_PERSISTENT) {
        // Profiling times each stage with HIP events between launches on this
        // stream, so it launches the graph's kernel sequence directly (same
        // kernels, grids and order); otherwise the captured graph runs.
        if (!c->profile)
            HIP_TRY(hipGraphLaunch(get_graph(c, sl, count), s));
        else
            enqueue_kernels(c, c->tune, slot_scratch(sl), sl.dev, n, nullptr, true, count, s, sl.sev.data());
    } else {
        HIP_TRY(hipMemsetAsync(sl.d_n + 1, 0, sizeof(uint32_t), s));
        for (uint32_t off = 0; off < n; off += kPlainChunk) {
            const uint32_t m = std::min(kPlainChunk, n - off);
            BatchDev v = sl.dev;
            v.recs += off; v.res += off; v.cells += off; v.seed += off; v.valid += off; v.tout += 2 * (size_t)off;
            enqueue_kernels(c, c->tune, slot_scratch(sl), v, m, nullptr, false, count, s,
                            c->profile ? sl.sev.data() + (kNumStages + 1) * (size_t)(off / kPlainChunk) : nullptr);
            // chunk errors accumulate in the slot's error word
            launch_accum_errors(v, sl.d_n + 1, s);
        }
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(sl.ev1, s));
    if (t.device) {
        HIP_TRY(hipMemcpyAsync(t.out, sl.dev.res, (size_t)n * sizeof(xdrop_result), hipMemcpyDeviceToDevice, s));
        if (count) HIP_TRY(hipMemcpyAsync(t.cells, sl.dev.cells, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
    } else {
        HIP_TRY(hipMemcpyAsync(sl.h_res, sl.dev.res, (size_t)n * sizeof(xdrop_result), hipMemcpyDeviceToHost, s));
        if (count) HIP_TRY(hipMemcpyAsync(sl.h_cells, sl.dev.cells, (size_t)n * 8, hipMemcpyDeviceToHost, s));
    }
    const uint32_t *err_src = c->mode == XDROP_MODE_PERSISTENT ? sl.dev.ctr + CtrLayout::kErrors : sl.d_n + 1;
    HIP_TRY(hipMemcpyAsync(sl.h_misc + 1, err_src, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    if (count && c->mode == XDROP_MODE_PERSISTENT)
        HIP_TRY(hipMemcpyAsync(sl.h_stage, sl.dev.stage_sum, kStageSumWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(sl.ev2, s));
    HIP_TRY(hipEventSynchronize(sl.ev2));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, sl.ev0, sl.ev1));
    t.dev_ms = ms;
    if (c->profile) {
        const bool plain = c->mode == XDROP_MODE_PLAIN;
        const size_t chunks = plain ? (n + kPlainChunk - 1) / kPlainChunk : 1;
        for (size_t ch = 0; ch < chunks; ++ch) {
            hipEvent_t *e = sl.sev.data() + (kNumStages + 1) * (plain ? ch : 0);
            for (int k = 0; k < kNumStages; ++k) {
                float a = 0.f;
                HIP_TRY(hipEventElapsedTime(&a, e[k], e[k + 1]));
                t.stage_ms[k] += a;
            }
        }
    }
    if (count && c->mode == XDROP_MODE_PERSISTENT) {
        for (int k = 0; k < XDROP_NUM_STAGES; ++k) {
            t.stage_cells[k] = sl.h_stage[k];
            t.stage_tasks[k] = sl.h_stage[8 + k];
            t.stage_slots[k] = sl.h_stage[16 + k];
        }
    }
    const uint32_t errors = sl.h_misc[1];
    if (!t.device) {
        std::memcpy(t.out, sl.h_res, (size_t)n * sizeof(xdrop_result));
        if (count) std::memcpy(t.cells, sl.h_cells, (size_t)n * 8);
    }
    if (count) {
        uint64_t tot = 0;
        if (t.device) {
            // per-record counts stay on the device; stats carry no total
        } else {
            for (uint32_t i = 0; i < n; ++i) tot += t.cells[i];
        }
        t.total_cells = tot;
    }
    t.status = errors ? XDROP_E_INVALID : XDROP_OK;
}

void slot_worker(xdrop_ctx *c, Slot *sl)
{
    hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(c->mu);
    for (;;) {
        sl->cv.wait(lk, [&] { return c->stop || sl->job != nullptr; });
        if (sl->job == nullptr && c->stop) break;
        std::shared_ptr<Ticket> t = sl->job;
        lk.unlock();
        xdrop_status st = XDROP_OK;
        std::string msg;
        if (t->n > 0) {
            try {
                run_batch(c, *sl, *t);
                st = t->status;
            } catch (const std::exception &e) {
                st = XDROP_E_DEVICE;
                msg = e.what();
            }
        }
        lk.lock();
        if (st == XDROP_E_DEVICE) {
            c->poisoned = true;
            c->fail(msg);
            for (auto &kv : c->tickets)
                if (!kv.second->done) kv.second->status = XDROP_E_DEVICE;
        }
        t->status = c->poisoned ? XDROP_E_DEVICE : st;
        t->t_done = now_ms();
        t->done = true;
        sl->job = nullptr;
        sl->busy = false;
        c->cv.notify_all();
    }
}

Slot *new_slot(xdrop_ctx *c)
{
    auto s = std::make_unique<Slot>();
    HIP_TRY(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreate(&s->ev0));
    HIP_TRY(hipEventCreate(&s->ev1));
    HIP_TRY(hipEventCreateWithFlags(&s->ev2, hipEventBlockingSync));
    Slot *raw = s.get();
    raw->worker = std::thread(slot_worker, c, raw);
    c->slots.push_back(std::move(s));
    return raw;
}

// Admission (called with c->mu held): a free slot with enough capacity, or a
// new / re-sized slot when the HBM budget allows.  Returns nullptr if none;
// then at least one slot is busy (a batch that fits the budget alone always
// fits once every idle slot has been emptied), and its completion wakes the
// waiters.  Throws when an allocation fails (the slot involved is left empty).
Slot *try_admit(xdrop_ctx *c, size_t n)
{
    std::vector<SlotView> view;
    for (auto &s : c->slots) view.push_back(SlotView{s->busy, s->cap, s->bytes});
    const uint32_t cap = round_cap(n);
    const size_t need = slot_footprint(c, cap);
    const AdmitPlan p = plan_admission(view, (uint32_t)n, need, c->used, c->budget, c->max_inflight);
    switch (p.kind) {
    case AdmitPlan::kReuse:
        return c->slots[p.slot].get();
    case AdmitPlan::kNew: {
        Slot *s = new_slot(c);
        alloc_slot_buffers(c, *s, cap);
        c->used += s->bytes;
        return s;
    }
    case AdmitPlan::kResize: {
        for (int k : p.release) {
            c->used -= c->slots[k]->bytes;
            free_slot_buffers(*c->slots[k]);
        }
        Slot *target = c->slots[p.slot].get();
        alloc_slot_buffers(c, *target, cap);
        c->used += target->bytes;
        return target;
    }
    case AdmitPlan::kNone:
        break;
    }
    return nullptr;
}

xdrop_status submit_common(xdrop_ctx *c, std::shared_ptr<Ticket> t, const xdrop_record *host_recs,
                           int64_t admit_timeout_us, xdrop_ticket *ticket)
{
    t->t_submit = now_ms();
    std::unique_lock<std::mutex> lk(c->mu);
    if (c->poisoned) return XDROP_E_DEVICE;
    t->id = c->next_id++;
    if (t->n == 0) {
        t->done = true;
        t->t_admit = t->t_done = now_ms();
        c->tickets[t->id] = t;
        *ticket = t->id;
        return XDROP_OK;
    }
    if (slot_footprint(c, round_cap(t->n)) > c->budget) {
        c->fail("batch does not fit the HBM budget even alone");
        return XDROP_E_NOMEM;
    }
    const auto deadline = clk::now() + std::chrono::microseconds(admit_timeout_us > 0 ? admit_timeout_us : 0);
    Slot *sl = nullptr;
    for (;;) {
        if (c->poisoned) return XDROP_E_DEVICE;
        try {
            sl = try_admit(c, t->n);
        } catch (const std::exception &e) {
            c->fail(e.what());
            return XDROP_E_NOMEM;
        }
        if (sl) break;
        if (admit_timeout_us == 0) return XDROP_E_BUSY;
        if (admit_timeout_us < 0) {
            c->cv.wait(lk);
        } else if (c->cv.wait_until(lk, deadline) == std::cv_status::timeout) {
            try {
                sl = try_admit(c, t->n);
            } catch (const std::exception &e) {
                c->fail(e.what());
                return XDROP_E_NOMEM;
            }
            if (!sl) return XDROP_E_BUSY;
            break;
        }
    }
    sl->busy = true;
    t->slot = sl;
    t->t_admit = now_ms();
    c->tickets[t->id] = t;
    *ticket = t->id;
    if (host_recs) {
        lk.unlock();
        std::memcpy(sl->h_recs, host_recs, t->n * sizeof(xdrop_record));
        lk.lock();
    }
    sl->job = t;
    sl->cv.notify_one();
    return XDROP_OK;
}

bool ctx_idle(xdrop_ctx *c)
{
    for (auto &sl : c->slots)
        if (sl->busy) return false;
    return true;
}

void clamp_tuning(Tuning &t)
{
    t.grow_margin = std::min(std::max(t.grow_margin, 2), 64);
    t.shrink_margin = std::min(std::max(t.shrink_margin, 2), 64);
    t.waves_per_cu = std::min(std::max(t.waves_per_cu, 1), 64);
    t.buckets = t.buckets ? 1 : 0;
    t.generic_waves = (std::min(std::max(t.generic_waves, kGenericBlockWaves), 4096) + kGenericBlockWaves - 1) /
                      kGenericBlockWaves * kGenericBlockWaves;
    t.narrow_x = std::min(std::max(t.narrow_x, -1), kNarrowMaxX);
    t.narrow_min = std::max(t.narrow_min, 0);
    t.wide_waves = t.wide_waves >= 4 ? 4 : t.wide_waves >= 2 ? 2 : 1;
}

// new launch parameters: captured graphs hold the old ones; the unbounded
// kernel's scratch is sized by its workgroup count (called with c->mu held, idle)
void apply_tuning(xdrop_ctx *c, const Tuning &t)
{
    const bool rescratch = generic_blocks(t.generic_waves) != generic_blocks(c->tune.generic_waves);
    c->tune = t;
    for (auto &sl : c->slots) {
        for (auto &g : sl->graph)
            if (g) { hipGraphExecDestroy(g); g = nullptr; }
        if (rescratch && sl->cap) {
            const uint32_t cap = sl->cap;
            c->used -= sl->bytes;
            free_slot_buffers(*sl);
            alloc_slot_buffers(c, *sl, cap);
            c->used += sl->bytes;
        }
    }
}

// ---------------------------------------------------------------------------
// Batch buffers without allocation (xdrop_batch_run_noalloc).  Every buffer a
// batch needs beyond its records and results -- seed scores, validity flags,
// task results, class queues, counters, bucket histograms, the carry pool and
// the unbounded kernel's scratch -- is carved, per call, out of one array in
// device memory that the code object holds for the life of the process (one
// copy per GPU).  Host code never uses the array's name as an address: its
// device address is looked up once per device with hipGetSymbolAddress at
// context creation and kept in noalloc_base.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = XDROP_NOALLOC_BYTES;
constexpr size_t kNoAllocGenericBytes = 24ull << 20;   // unbounded-kernel scratch share
constexpr int kNoAllocMaxDevices = 64;
static_assert(kNoAllocBytes % 256 == 0, "array size");

std::mutex g_noalloc_mu;
void *g_noalloc_base[kNoAllocMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocBytes];

namespace {

// Device address of this device's copy of noalloc_scratch (the device must be
// current); looked up once per device.
bool noalloc_resolve(int device, std::string &why)
{
    if (device < 0 || device >= kNoAllocMaxDevices) {
        why = "device ordinal beyond the no-alloc table";
        return false;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_base[device]) return true;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        why = std::string("hipGetSymbolAddress(noalloc_scratch): ") + hipGetErrorString(e);
        return false;
    }
    g_noalloc_base[device] = p;
    return true;
}

void *noalloc_base(int device)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    return device >= 0 && device < kNoAllocMaxDevices ? g_noalloc_base[device] : nullptr;
}

// The buffers of one no-alloc batch of n records (records, results and cell
// counts are the caller's), laid out from `base`: the per-record arrays as in
// a slot of capacity n, then counters, histograms and stage sums, then the
// unbounded kernel's scratch (as many workgroups as fit its share, at most
// the tuned count), then the carry pool in what is left (at most 256 words
// per record; a smaller pool only makes more handed-over tasks restart).
// Returns false with `why` set when the batch does not fit the array.
bool noalloc_layout(const xdrop_ctx *c, const Tuning &tu, char *base, uint32_t n, BatchDev &b, GenericScratch &gs,
                    std::string &why)
{
    if (n > XDROP_NOALLOC_MAX_RECORDS) {
        why = "batch of " + std::to_string(n) + " records exceeds the no-alloc limit of " +
              std::to_string(XDROP_NOALLOC_MAX_RECORDS);
        return false;
    }
    size_t off = 0;
    auto take = [&](size_t x) {
        char *q = base + off;
        off += (x + 255) & ~size_t(255);
        return (void *)q;
    };
    const size_t cap = n;
    b = BatchDev{};
    b.seed = (int32_t *)take(cap * sizeof(int32_t));
    b.valid = (uint8_t *)take(cap);
    b.tout = (TaskOut *)take(2 * cap * sizeof(TaskOut));
    b.qbuf = (uint32_t *)take((size_t)kNumClasses * 2 * cap * sizeof(uint32_t));
    b.qkey = (uint32_t *)take((size_t)kNumClasses * 2 * cap * sizeof(uint32_t));
    b.qstate = (uint32_t *)take((size_t)kNumClasses * 2 * cap * sizeof(uint32_t));
    b.ctr = (uint32_t *)take(CtrLayout::kWords * sizeof(uint32_t) + 64);
    b.bucket_hist = (uint32_t *)take((size_t)kNumClasses * kNumBuckets * sizeof(uint32_t));
    b.stage_sum = (unsigned long long *)take(kStageSumWords * sizeof(unsigned long long));
    b.cap = n;
    const uint64_t stride = scratch_stride_of(c);
    const uint64_t per_block = 3 * stride * sizeof(int32_t);
    const uint64_t fit = kNoAllocGenericBytes / per_block;
    if (fit == 0) {
        why = "reads too long for the no-alloc buffer: the unbounded kernel needs " + std::to_string(per_block) +
              " bytes per workgroup, its share is " + std::to_string(kNoAllocGenericBytes);
        return false;
    }
    gs.blocks = (uint32_t)std::min<uint64_t>(generic_blocks(tu.generic_waves), fit);
    gs.stride = stride;
    gs.base = (int32_t *)take((size_t)gs.blocks * per_block);
    if (off > kNoAllocBytes) {   // cannot happen within the record limit; checked all the same
        why = "no-alloc layout exceeds the array";
        return false;
    }
    const uint64_t left_words = (kNoAllocBytes - off) / sizeof(int32_t);
    b.carry_words = (uint32_t)std::min<uint64_t>({left_words, (uint64_t)n * 256u, 64ull << 20});
    b.carry = (int32_t *)(base + off);
    return true;
}

bool write_tuning(const std::string &path, const Tuning &t)
{
    std::ofstream f(path);
    if (!f) return false;
    f << "grow_margin " << t.grow_margin << "\n"
      << "shrink_margin " << t.shrink_margin << "\n"
      << "waves_per_cu " << t.waves_per_cu << "\n"
      << "buckets " << t.buckets << "\n"
      << "generic_waves " << t.generic_waves << "\n"
      << "narrow_x " << t.narrow_x << "\n"
      << "narrow_min_records " << t.narrow_min << "\n"
      << "wide_waves " << t.wide_waves << "\n";
    return (bool)f;
}

}  // namespace

extern "C" {

const char *xdrop_status_string(xdrop_status s)
{
    switch (s) {
    case XDROP_OK: return "ok";
    case XDROP_E_INVALID: return "invalid argument or record";
    case XDROP_E_NOMEM: return "out of memory";
    case XDROP_E_DEVICE: return "device error";
    case XDROP_E_TIMEOUT: return "timed out";
    case XDROP_E_BUSY: return "admission refused (busy)";
    case XDROP_E_STATE: return "bad ticket or context state";
    default: return "unknown status";
    }
}

const char *xdrop_last_error(const xdrop_ctx *c)
{
    // a copy per calling thread: valid until that thread's next call
    thread_local std::string copy;
    if (c) {
        std::lock_guard<std::mutex> lk(c->err_mu);
        copy = c->err;
    } else {
        std::lock_guard<std::mutex> lk(g_err_mu);
        copy = g_err_text;
    }
    return copy.c_str();
}

xdrop_status xdrop_batch_create(const xdrop_config *cfg, xdrop_ctx **out)
{
    if (!cfg || !out) return XDROP_E_INVALID;
    if (cfg->n_reads == 0 || !cfg->reads || !cfg->lengths) {
        set_global_error("empty read store");
        return XDROP_E_INVALID;
    }
    if (cfg->mode > XDROP_MODE_PLAIN) {
        set_global_error("unknown mode");
        return XDROP_E_INVALID;
    }
    std::unique_ptr<xdrop_ctx> c(new xdrop_ctx);
    c->device = cfg->device;
    c->mode = cfg->mode;
    c->max_inflight = cfg->max_inflight ? cfg->max_inflight : 4;
    c->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : kDefaultBudget;
    c->profile = (cfg->flags & XDROP_FLAG_PROFILE) != 0;
    c->tune = default_tuning();
    if (cfg->tuning_cache) {
        c->tuning_path = cfg->tuning_cache;
        load_tuning(c->tuning_path, c->tune);
    }
    clamp_tuning(c->tune);
    // pack the store: fwd and reverse complement of every read, each starting
    // on a word boundary, 2 bits per base
    const uint32_t nr = cfg->n_reads;
    c->h_len.assign(cfg->lengths, cfg->lengths + nr);
    std::vector<ReadInfo> info(nr);
    uint64_t pos = kGuardBases;
    uint32_t max_len = 0;
    for (uint32_t r = 0; r < nr; ++r) {
        const uint32_t L = cfg->lengths[r];
        if (L == 0 || L > XDROP_MAX_READ_LEN || !cfg->reads[r]) {
            set_global_error("read " + std::to_string(r) + ": empty or too long");
            return XDROP_E_INVALID;
        }
        max_len = std::max(max_len, L);
        info[r].len = L;
        info[r].fwd = pos;
        pos += ((uint64_t)L + 15) & ~uint64_t(15);
        info[r].rc = pos;
        pos += ((uint64_t)L + 15) & ~uint64_t(15);
    }
    const uint64_t total_bases = pos + kGuardBases;
    const uint64_t nwords = (total_bases + 15) / 16 + 16;
    std::vector<uint32_t> words(nwords, 0u);
    std::atomic<int64_t> bad{-1};
    {
        const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (unsigned w = 0; w < nt; ++w) {
            th.emplace_back([&, w] {
                for (uint32_t r = w; r < nr; r += nt) {
                    const char *s = cfg->reads[r];
                    const uint32_t L = info[r].len;
                    for (uint32_t p = 0; p < L; ++p) {
                        const int8_t v = base_code(s[p]);
                        if (v < 0) {
                            bad = r;
                            return;
                        }
                        const uint64_t f = info[r].fwd + p;
                        const uint64_t q = info[r].rc + (L - 1 - p);
                        words[f >> 4] |= (uint32_t)v << ((f & 15) * 2);
                        words[q >> 4] |= (uint32_t)(3 - v) << ((q & 15) * 2);
                    }
                }
            });
        }
        for (auto &t : th) t.join();
    }
    if (bad >= 0) {
        set_global_error("read " + std::to_string((long long)bad) + ": non-ACGT base");
        return XDROP_E_INVALID;
    }
    try {
        HIP_TRY(hipSetDevice(c->device));
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, c->device));
        c->cus = prop.multiProcessorCount;
        // device address of this GPU's no-alloc buffer, looked up once per
        // device with it current; a failure is reported by the no-alloc entry
        // point (which tries again) and does not affect the other calls
        std::string why;
        if (!noalloc_resolve(c->device, why)) set_global_error(why);
        HIP_TRY(hipMalloc(&c->d_words, nwords * sizeof(uint32_t)));
        HIP_TRY(hipMalloc(&c->d_reads, (size_t)nr * sizeof(ReadInfo)));
        HIP_TRY(hipMemcpy(c->d_words, words.data(), nwords * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->d_reads, info.data(), (size_t)nr * sizeof(ReadInfo), hipMemcpyHostToDevice));
    } catch (const std::exception &e) {
        set_global_error(e.what());
        if (c->d_words) hipFree(c->d_words);
        if (c->d_reads) hipFree(c->d_reads);
        return XDROP_E_DEVICE;
    }
    c->store_bytes = nwords * 4 + (uint64_t)nr * sizeof(ReadInfo);
    c->st.words = c->d_words;
    c->st.reads = c->d_reads;
    c->st.n_reads = nr;
    c->st.max_len = max_len;
    *out = c.release();
    return XDROP_OK;
}

xdrop_status xdrop_batch_submit(xdrop_ctx *c, const xdrop_record *recs, size_t n, xdrop_result *out,
                                uint64_t *cells, int64_t admit_timeout_us, xdrop_ticket *ticket)
{
    if (!c || !ticket || (n && (!recs || !out))) return XDROP_E_INVALID;
    if (n > 0x7fffffffu) {
        c->fail("batch too large");
        return XDROP_E_INVALID;
    }
    std::string why;
    for (size_t i = 0; i < n; ++i) {
        if (!validate_host(c, recs[i], why)) {
            std::lock_guard<std::mutex> lk(c->mu);
            c->fail("record " + std::to_string(i) + ": " + why);
            return XDROP_E_INVALID;
        }
    }
    auto t = std::make_shared<Ticket>();
    t->n = n;
    t->out = out;
    t->cells = cells;
    return submit_common(c, t, recs, admit_timeout_us, ticket);
}

xdrop_status xdrop_batch_submit_device(xdrop_ctx *c, const xdrop_record *d_recs, size_t n, xdrop_result *d_out,
                                       uint64_t *d_cells, void *stream, xdrop_ticket *ticket)
{
    if (!c || !ticket || (n && (!d_recs || !d_out))) return XDROP_E_INVALID;
    if (n > 0x7fffffffu) return XDROP_E_INVALID;
    auto t = std::make_shared<Ticket>();
    t->n = n;
    t->device = true;
    t->d_in = d_recs;
    t->out = d_out;
    t->cells = d_cells;
    t->ustream = (hipStream_t)stream;
    return submit_common(c, t, nullptr, -1, ticket);
}

xdrop_status xdrop_batch_wait(xdrop_ctx *c, xdrop_ticket id, int64_t timeout_us, xdrop_batch_stats *stats)
{
    if (!c) return XDROP_E_INVALID;
    std::unique_lock<std::mutex> lk(c->mu);
    auto it = c->tickets.find(id);
    if (it == c->tickets.end()) return XDROP_E_STATE;
    std::shared_ptr<Ticket> t = it->second;
    if (!t->done) {
        if (timeout_us == 0) return XDROP_E_TIMEOUT;
        if (timeout_us < 0) {
            c->cv.wait(lk, [&] { return t->done; });
        } else if (!c->cv.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return t->done; })) {
            return XDROP_E_TIMEOUT;
        }
    }
    c->tickets.erase(id);
    if (stats) {
        stats->records = t->n;
        stats->cells = t->total_cells;
        stats->queue_ms = t->t_admit - t->t_submit;
        stats->device_ms = t->dev_ms;
        stats->total_ms = t->t_done - t->t_submit;
        for (int k = 0; k < XDROP_NUM_STAGES; ++k) {
            stats->stage_ms[k] = t->stage_ms[k];
            stats->stage_cells[k] = t->stage_cells[k];
            stats->stage_tasks[k] = t->stage_tasks[k];
            stats->stage_slots[k] = t->stage_slots[k];
        }
    }
    return t->status;
}

xdrop_status xdrop_get_tuning(const xdrop_ctx *c, xdrop_tuning *out)
{
    if (!c || !out) return XDROP_E_INVALID;
    std::lock_guard<std::mutex> lk(c->mu);   // set_tuning / autotune write under the same lock
    out->grow_margin = c->tune.grow_margin;
    out->shrink_margin = c->tune.shrink_margin;
    out->waves_per_cu = c->tune.waves_per_cu;
    out->buckets = c->tune.buckets;
    out->generic_waves = c->tune.generic_waves;
    out->narrow_x = c->tune.narrow_x;
    out->narrow_min_records = c->tune.narrow_min;
    out->wide_waves = c->tune.wide_waves;
    return XDROP_OK;
}

xdrop_status xdrop_set_tuning(xdrop_ctx *c, const xdrop_tuning *in)
{
    if (!c || !in) return XDROP_E_INVALID;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!ctx_idle(c)) return XDROP_E_BUSY;
    Tuning t = c->tune;
    t.grow_margin = in->grow_margin;
    t.shrink_margin = in->shrink_margin;
    t.waves_per_cu = in->waves_per_cu;
    t.buckets = in->buckets;
    t.generic_waves = in->generic_waves;
    t.narrow_x = in->narrow_x;
    t.narrow_min = in->narrow_min_records;
    t.wide_waves = in->wide_waves;
    clamp_tuning(t);
    try {
        apply_tuning(c, t);
    } catch (const std::exception &e) {
        c->fail(e.what());
        return XDROP_E_NOMEM;
    }
    return XDROP_OK;
}

xdrop_status xdrop_autotune(xdrop_ctx *c, const xdrop_record *recs, size_t n, const char *cache_path,
                            double *best_ms)
{
    if (!c || !recs || n == 0) return XDROP_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        if (!ctx_idle(c)) return XDROP_E_BUSY;
    }
    std::vector<xdrop_result> out(n);
    auto time_once = [&](double &ms) -> xdrop_status {
        xdrop_ticket tk;
        xdrop_status st = xdrop_batch_submit(c, recs, n, out.data(), nullptr, -1, &tk);
        if (st != XDROP_OK) return st;
        xdrop_batch_stats s{};
        st = xdrop_batch_wait(c, tk, -1, &s);
        ms = s.device_ms;
        return st;
    };
    // Coordinate descent: each knob in turn is swept over its values with the
    // others held at the best setting so far; two rounds.  A setting is timed
    // by the better of two runs after a warm-up run (graph capture).
    auto measure = [&](const Tuning &cand, double &ms) -> xdrop_status {
        {
            std::lock_guard<std::mutex> lk(c->mu);
            try {
                apply_tuning(c, cand);
            } catch (const std::exception &e) {
                c->fail(e.what());
                return XDROP_E_NOMEM;
            }
        }
        double ms0 = 0, ms1 = 0, ms2 = 0;
        xdrop_status st = time_once(ms0);
        if (st == XDROP_OK) st = time_once(ms1);
        if (st == XDROP_OK) st = time_once(ms2);
        ms = std::min(ms1, ms2);
        return st;
    };
    struct Knob {
        std::vector<std::pair<int, int>> values;   // (first, second) field values
        void (*set)(Tuning &, std::pair<int, int>);
    };
    const std::vector<Knob> knobs = {
        {{{8, 0}, {16, 0}, {24, 0}, {32, 0}, {40, 0}}, [](Tuning &t, std::pair<int, int> v) { t.waves_per_cu = v.first; }},
        {{{0, 0}, {1, 0}}, [](Tuning &t, std::pair<int, int> v) { t.buckets = v.first; }},
        {{{2, 2}, {4, 2}, {6, 3}, {8, 4}, {8, 6}, {12, 8}, {16, 12}},
         [](Tuning &t, std::pair<int, int> v) { t.grow_margin = v.first; t.shrink_margin = v.second; }},
        {{{256, 0}, {1024, 0}, {4096, 0}},
         [](Tuning &t, std::pair<int, int> v) { t.generic_waves = v.first; }},
        // two extensions per wavefront for drops up to: off, 15, 20, 30, 40
        {{{-1, 0}, {15, 0}, {20, 0}, {30, 0}, {40, 0}},
         [](Tuning &t, std::pair<int, int> v) { t.narrow_x = v.first; }},
        // wavefronts per extension of bands of 1281-2048 cells: 1, 2 or 4
        {{{1, 0}, {2, 0}, {4, 0}}, [](Tuning &t, std::pair<int, int> v) { t.wide_waves = v.first; }},
    };
    const Tuning start = c->tune;
    Tuning best = start;
    double best_t = 1e300;
    {
        const xdrop_status st = measure(best, best_t);
        if (st != XDROP_OK) return st;
    }
    for (int round = 0; round < 2; ++round) {
        for (const Knob &k : knobs) {
            for (const auto &v : k.values) {
                Tuning cand = best;
                k.set(cand, v);
                clamp_tuning(cand);
                if (std::memcmp(&cand, &best, sizeof(Tuning)) == 0) continue;
                double ms = 0;
                const xdrop_status st = measure(cand, ms);
                if (st != XDROP_OK) return st;
                if (ms < best_t) {
                    best_t = ms;
                    best = cand;
                }
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(c->mu);
        try {
            apply_tuning(c, best);
        } catch (const std::exception &e) {
            c->fail(e.what());
            return XDROP_E_NOMEM;
        }
        if (cache_path && !write_tuning(cache_path, best)) {
            c->fail(std::string("cannot write tuning cache ") + cache_path);
            return XDROP_E_INVALID;
        }
    }
    if (best_ms) *best_ms = best_t;
    return XDROP_OK;
}

xdrop_status xdrop_batch_run_noalloc(xdrop_ctx *c, const xdrop_record *d_recs, size_t n, xdrop_result *d_out,
                                     uint64_t *d_cells, uint32_t *d_invalid, void *stream)
{
    if (!c || (n && (!d_recs || !d_out))) return XDROP_E_INVALID;
    Tuning tu;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        if (c->poisoned) return XDROP_E_DEVICE;
        tu = c->tune;
    }
    if (n > XDROP_NOALLOC_MAX_RECORDS) {
        c->fail("xdrop_batch_run_noalloc: batch of " + std::to_string(n) + " records exceeds the limit of " +
                std::to_string(XDROP_NOALLOC_MAX_RECORDS));
        return XDROP_E_INVALID;
    }
    std::string why;
    if (hipSetDevice(c->device) != hipSuccess) {
        (void)hipGetLastError();
        c->fail("xdrop_batch_run_noalloc: hipSetDevice failed");
        return XDROP_E_DEVICE;
    }
    if (!noalloc_resolve(c->device, why)) {
        c->fail("xdrop_batch_run_noalloc: " + why);
        return XDROP_E_DEVICE;
    }
    hipStream_t s = (hipStream_t)stream;
    BatchDev b{};
    GenericScratch gs{};
    if (!noalloc_layout(c, tu, (char *)noalloc_base(c->device), (uint32_t)n, b, gs, why)) {
        c->fail("xdrop_batch_run_noalloc: " + why);
        return XDROP_E_INVALID;
    }
    b.recs = d_recs;
    b.res = d_out;
    b.cells = d_cells;
    try {
        // the persistent form's kernel sequence, launched directly on the
        // caller's stream (no graph, no events); the batch size is immediate.
        // An empty batch only clears the counters (the invalid count is 0).
        if (n == 0)
            launch_reset_n(b, nullptr, 0u, s);
        else
            enqueue_kernels(c, tu, gs, b, (uint32_t)n, nullptr, true, d_cells != nullptr, s, nullptr);
        if (d_invalid)
            HIP_TRY(hipMemcpyAsync(d_invalid, b.ctr + CtrLayout::kErrors, sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipGetLastError());
    } catch (const std::exception &e) {
        c->fail(std::string("xdrop_batch_run_noalloc: ") + e.what());
        return XDROP_E_DEVICE;
    }
    return XDROP_OK;
}

uint64_t xdrop_batch_footprint(const xdrop_ctx *c, size_t n)
{
    if (!c) return 0;
    return (uint64_t)slot_footprint(c, round_cap(n));
}

xdrop_status xdrop_batch_destroy(xdrop_ctx *c)
{
    if (!c) return XDROP_OK;
    {
        std::unique_lock<std::mutex> lk(c->mu);
        c->cv.wait(lk, [&] {
            for (auto &s : c->slots)
                if (s->busy) return false;
            return true;
        });
        c->stop = true;
        for (auto &s : c->slots) s->cv.notify_all();
    }
    for (auto &s : c->slots)
        if (s->worker.joinable()) s->worker.join();
    hipSetDevice(c->device);
    for (auto &s : c->slots) {
        free_slot_buffers(*s);
        if (s->ev0) hipEventDestroy(s->ev0);
        if (s->ev1) hipEventDestroy(s->ev1);
        if (s->ev2) hipEventDestroy(s->ev2);
        if (s->stream) hipStreamDestroy(s->stream);
    }
    if (c->d_words) hipFree(c->d_words);
    if (c->d_reads) hipFree(c->d_reads);
    delete c;
    return XDROP_OK;
}

xdrop_status xdrop_find_seeds(xdrop_ctx *c, const xdrop_seed_params *p, xdrop_record *out, size_t max_records,
                              int out_on_device, size_t *n_found, xdrop_seed_stats *stats)
{
    if (!c || !p || !n_found || (max_records && !out)) return XDROP_E_INVALID;
    if (p->k < 1 || p->k > 31 || p->stride < 1 || p->lo < 1 || p->lo > p->hi || p->hi > 4096 || p->x < 0 ||
        p->x > XDROP_MAX_X || p->match < 1 || p->match > 1024 || p->mismatch >= p->match || p->mismatch < -1024 ||
        p->gap > -1 || p->gap < -1024 || max_records > 0xffffffffu) {
        c->fail("xdrop_find_seeds: bad parameters");
        return XDROP_E_INVALID;
    }
    {
        std::lock_guard<std::mutex> lk(c->mu);
        if (c->poisoned) return XDROP_E_DEVICE;
    }
    uint64_t kmers = 0;
    for (uint32_t len : c->h_len)
        if (len >= p->k) kmers += (len - p->k) / p->stride + 1;
    auto pow2 = [](uint64_t v) { uint64_t r = 1024; while (r < v) r <<= 1; return r; };
    SeedDev sd{};
    sd.k = (int)p->k; sd.stride = (int)p->stride; sd.lo = (int)p->lo; sd.hi = (int)p->hi;
    sd.cap = pow2(2 * kmers);                       // load factor <= 1/2
    sd.max_reliable = (uint32_t)std::min<uint64_t>(kmers / p->lo + 1, 0xffffffffu);
    sd.pcap = pow2(2 * (uint64_t)max_records);
    std::vector<void *> bufs;
    hipStream_t s = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto release = [&]() {
        if (s) hipStreamSynchronize(s);
        for (void *b : bufs) hipFree(b);
        for (auto e : ev) if (e) hipEventDestroy(e);
        if (s) hipStreamDestroy(s);
    };
    try {
        HIP_TRY(hipSetDevice(c->device));
        auto dalloc = [&](size_t bytes) {
            void *ptr = nullptr;
            if (hipMalloc(&ptr, std::max<size_t>(bytes, 256)) != hipSuccess) {
                (void)hipGetLastError();
                throw std::bad_alloc();
            }
            bufs.push_back(ptr);
            return ptr;
        };
        sd.keys = (uint64_t *)dalloc(sd.cap * 8);
        sd.counts = (uint32_t *)dalloc(sd.cap * 4);
        sd.rid = (int32_t *)dalloc(sd.cap * 4);
        sd.fill = (uint32_t *)dalloc((size_t)sd.max_reliable * 4);
        sd.occ = (uint64_t *)dalloc((size_t)sd.max_reliable * p->hi * 8);
        sd.pkeys = (uint64_t *)dalloc(sd.pcap * 8);
        sd.pvals = (uint64_t *)dalloc(sd.pcap * 8);
        sd.ctr = (uint32_t *)dalloc(kSeedCounters * 4);
        sd.n_chunks = (uint32_t)c->cus * 8u * 4u;                 // wavefronts of the reliable passes
        sd.chunk = ((sd.cap + sd.n_chunks - 1) / sd.n_chunks + 63) / 64 * 64;
        sd.wcount = (uint32_t *)dalloc((size_t)sd.n_chunks * 4);
        xdrop_record *d_out = out_on_device ? out : (xdrop_record *)dalloc(max_records * sizeof(xdrop_record));
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        HIP_TRY(hipEventCreate(&ev[0]));
        HIP_TRY(hipEventCreate(&ev[1]));
        launch_seeds(sd, c->st, d_out, (uint32_t)max_records, p->x, p->match, p->mismatch, p->gap, c->cus, s, ev);
        HIP_TRY(hipGetLastError());
        uint32_t ctr[kSeedCounters] = {};
        HIP_TRY(hipMemcpyAsync(ctr, sd.ctr, sizeof(ctr), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const size_t written = std::min<size_t>(ctr[kSeedPairs], max_records);
        if (!out_on_device && written)
            HIP_TRY(hipMemcpy(out, d_out, written * sizeof(xdrop_record), hipMemcpyDeviceToHost));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
        *n_found = ctr[kSeedPairs];
        if (stats) {
            stats->kmers = kmers;
            stats->distinct = ctr[kSeedDistinct];
            stats->reliable = ctr[kSeedReliable];
            stats->pairs = ctr[kSeedPairs];
            stats->device_ms = ms;
        }
        release();
        if (ctr[kSeedOverflow] || ctr[kSeedPairs] > max_records) {
            c->fail("xdrop_find_seeds: more read pairs than max_records");
            return XDROP_E_NOMEM;
        }
        return XDROP_OK;
    } catch (const std::bad_alloc &) {
        release();
        c->fail("xdrop_find_seeds: device memory");
        return XDROP_E_NOMEM;
    } catch (const std::exception &e) {
        release();
        c->fail(e.what());
        return XDROP_E_DEVICE;
    }
}

}  // extern "C"
