// xdrop_internal.h -- structures shared by the HIP kernels and the host runtime
// of libxdrop.so.  Not part of the public ABI (include/xdrop.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/xdrop.h"

namespace xd {

// One read of the device store.  Both orientations are packed 2 bits per base,
// 16 bases per uint32 (base p of the store sits in word p >> 4, bits
// 2*(p & 15)); fwd/rc are global base indices of the first base.
struct ReadInfo {
    uint64_t fwd;
    uint64_t rc;
    uint32_t len;
    uint32_t pad;
};

// Result of one extension (task).  Task t belongs to record t >> 1; t & 1 is
// the side (0 = left, 1 = right).
struct TaskOut {
    int32_t score;
    int32_t i, j;
    uint32_t status;   // class that completed the task (stage index - 1)
    uint64_t cells;    // candidate cells (cell counting only)
    uint64_t slots;    // window lanes stepped over: slot-steps of the window (cell counting only)
};

// Extension kernels ("classes"), tried in order; a task whose live band
// outgrows a class moves to the next one (a wide class hands over its state
// when the carry pool has room; otherwise the task restarts there):
//   0  narrow bands (small drops): two extensions per wavefront, each in a
//      window of 32 or 64 slots over one half of the lanes;
//   1  adaptive register window, 1..4 cells per lane (64..256 slots), the
//      width following the band;
//   2  register window of 8, 12, 16 or 20 cells per lane (512..1280 slots),
//      the width following the band;
//   3  register window of 2048 slots: one wavefront of 24 or 32 cells per
//      lane (1536..2048 slots), or 2 or 4 wavefronts of a workgroup sharing
//      the window (tuning knob wide_waves);
//   4  unbounded band: one workgroup per extension, anti-diagonals in an LDS
//      ring (global memory beyond 8192 cells).
constexpr int kNarrowClass = 0;
constexpr int kAdaptiveClass = 1;
constexpr int kWideClasses = 2;
constexpr int kWideC[kWideClasses] = {20, 32};   // widest window of each wide class, cells per lane
constexpr int kGenericClass = kAdaptiveClass + 1 + kWideClasses;
constexpr int kNumClasses = kGenericClass + 1;
constexpr int kNumStages = kNumClasses + 2;   // ingest, classes..., finalize
static_assert(kNumStages == XDROP_NUM_STAGES, "stages of the public statistics");
constexpr int kNumBuckets = 64;
// narrow class: drops up to this bound by default, when the weights allow
// (match 1, gap -1, mismatch 0, -1 or -2); larger values of the tuning knob
// are clamped to it
constexpr int kNarrowMaxX = 64;

// Device buffers of one batch (all device pointers).
constexpr int kStageSumWords = 24;

struct BatchDev {
    const xdrop_record *recs;
    xdrop_result *res;
    uint64_t *cells;          // nullable, per record
    int32_t *seed;            // per record
    uint8_t *valid;           // per record
    TaskOut *tout;            // 2 per record
    uint32_t *qbuf;           // kNumClasses queues of capacity 2*cap (task ids)
    uint32_t *qkey;           // unsorted queue staging: (task id) per class, capacity 2*cap
    uint32_t *qstate;         // per queue entry of classes >= 1: word offset of its carried state, or kNoCarry
    int32_t *carry;           // carried states of extensions handed to a wider class (CarryLayout)
    uint32_t carry_words;     // capacity of carry, in words
    uint32_t *ctr;            // counters, see CtrLayout
    uint32_t *bucket_hist;    // kNumClasses * kNumBuckets
    unsigned long long *stage_sum;  // kStageSumWords: [0..7] cells, [8..15] tasks completed, [16..23] slot-steps
                                    // per stage (1 + class); cells and slot-steps count the work each stage did
    uint32_t cap;             // record capacity of the buffers
};

// Counter block layout (uint32 words).
struct CtrLayout {
    static constexpr int kCount = 0;                       // per class: queue length
    static constexpr int kHead = kNumClasses;              // per class: next task to fetch
    static constexpr int kStage = 2 * kNumClasses;         // per class: staging length (bucketing)
    static constexpr int kErrors = 3 * kNumClasses;        // invalid records
    static constexpr int kN = 3 * kNumClasses + 1;         // record count of the batch
    static constexpr int kCarry = 3 * kNumClasses + 2;     // words of the carry pool handed out
    static constexpr int kWords = 3 * kNumClasses + 3;
};

// State of an extension handed from a wide class to the next one: a header,
// then the live window of anti-diagonals d-1 and d-2, win slots each, in
// the window's units (Z = S + |gap| * anti-diagonal; dead = below -2^29).
// Slot k of anti-diagonal e holds cell i = base + floor(e / 2) + k.
constexpr uint32_t kNoCarry = 0xffffffffu;
struct CarryLayout {
    static constexpr int kD = 0;       // next anti-diagonal
    static constexpr int kBase = 1;
    static constexpr int kT = 2;       // best score so far and its cell
    static constexpr int kBi = 3;
    static constexpr int kBj = 4;
    static constexpr int kMn = 5;      // live slots over both anti-diagonals
    static constexpr int kMx = 6;
    static constexpr int kWin = 7;     // window slots
    static constexpr int kCells = 8;   // two words each (cell counting)
    static constexpr int kSlots = 10;
    static constexpr int kHeader = 16;
};

struct StoreDev {
    const uint32_t *words;    // packed store, with guard words at both ends
    const ReadInfo *reads;
    uint32_t n_reads;
    uint32_t max_len;
};

// Tunable launch parameters (the autotuner picks them).
struct Tuning {
    int32_t grow_margin;                    // adaptive: free slots per side after widening
    int32_t shrink_margin;                  // adaptive: narrow when the band fits C-1 with this slack
    int32_t waves_per_cu;                   // persistent grid size per class kernel
    int32_t buckets;                        // 0: no length bucketing
    int32_t generic_waves;                  // grid of the unbounded kernel
    int32_t narrow_x;                       // narrow class for drops <= narrow_x (-1: off)
    int32_t narrow_min;                     // ... and only in batches of at least this many records
    int32_t wide_waves;                     // wavefronts per extension in the 2048-slot class: 1, 2 or 4
};

// Kernel launchers (xdrop_kernels.hip).  All are asynchronous on `s`.
// Zero the batch counters; n comes from *n_src (device) when non-null, else n_imm.
void launch_reset_n(const BatchDev &b, const uint32_t *n_src, uint32_t n_imm, hipStream_t s);
void launch_accum_errors(const BatchDev &b, uint32_t *acc, hipStream_t s);
void launch_prep(const BatchDev &b, const StoreDev &st, const Tuning &tu, uint32_t n,
                 bool stage, hipStream_t s);
void launch_bucket(const BatchDev &b, const StoreDev &st, uint32_t n, hipStream_t s);
void launch_narrow(const BatchDev &b, const StoreDev &st, const Tuning &tu, uint32_t grid_waves, bool count_cells,
                   hipStream_t s);
void launch_adaptive(const BatchDev &b, const StoreDev &st, const Tuning &tu, uint32_t grid_waves,
                     bool count_cells, hipStream_t s);
void launch_wide(int which, const BatchDev &b, const StoreDev &st, uint32_t cus, int ext_waves, bool count_cells,
                 hipStream_t s);
// Unbounded kernel: one workgroup of kGenericBlockWaves wavefronts per
// extension; `blocks` workgroups, each with three anti-diagonals of
// scratch_stride ints in `scratch` (used only by bands wider than its LDS ring).
constexpr int kGenericBlockWaves = 16;
inline uint32_t generic_blocks(int32_t generic_waves)
{
    return generic_waves >= kGenericBlockWaves ? (uint32_t)generic_waves / kGenericBlockWaves : 1u;
}
void launch_generic(const BatchDev &b, const StoreDev &st, int32_t *scratch, uint64_t scratch_stride,
                    uint32_t blocks, bool count_cells, hipStream_t s);
void launch_finalize(const BatchDev &b, const StoreDev &st, uint32_t n, bool stage_sums, hipStream_t s);

// Seed discovery: device tables of one call (see seed_kernels.hip).
enum : int { kSeedOverflow = 0, kSeedDistinct = 1, kSeedReliable = 2, kSeedPairs = 3, kSeedCounters = 4 };
struct SeedDev {
    uint64_t *keys;           // k-mer table: canonical code, ~0 = empty
    uint32_t *counts;         //   occurrences of the entry
    int32_t *rid;             //   index among the reliable k-mers, -1 if not reliable
    uint64_t cap;             //   slots (power of two)
    uint32_t *fill;           // per reliable k-mer: occurrences stored
    uint64_t *occ;            // per reliable k-mer: hi slots of (read << 32 | pos << 1 | reverse)
    uint32_t max_reliable;    // reliable k-mers the buffers hold
    uint64_t *pkeys;          // pair table: read_a << 32 | read_b, ~0 = empty
    uint64_t *pvals;          //   smallest pos_a << 32 | pos_b << 1 | strand
    uint64_t pcap;            //   slots (power of two)
    uint32_t *ctr;            // kSeedCounters counters
    uint32_t *wcount;         // per table chunk: reliable entries, then their first index
    uint64_t chunk;           // table slots per chunk (a multiple of 64)
    uint32_t n_chunks;        // chunks = wavefronts of the reliable passes
    int k, stride, lo, hi;
};

// init, count, reliable (count, scan, assign), occurrences, pairs, emit;
// sd.n_chunks must equal the wavefronts of cus * 8 blocks of 256 threads and
// sd.chunk * n_chunks >= sd.cap; ev[0] / ev[1] (nullable)
// are recorded after init and after emit
void launch_seeds(const SeedDev &sd, const StoreDev &st, xdrop_record *d_out, uint32_t max_out, int x, int ma,
                  int mi, int gap, int cus, hipStream_t s, hipEvent_t *ev);

}  // namespace xd
