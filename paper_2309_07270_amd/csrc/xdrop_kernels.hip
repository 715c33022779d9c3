// xdrop_kernels.hip -- gfx950 kernels of batched X-drop seed-and-extend.
//
// Method (paper, "Related works": BELLA's seed-and-extend scored with an
// X-drop; LOGAN computes the X-drop table anti-diagonal by anti-diagonal
// because the cells of one anti-diagonal are independent; "Results": the
// aligner is Needleman-Wunsch / Smith-Waterman with an X-drop).  The exact
// rules (live predecessors, strict drop test against the best score of the
// previous anti-diagonals, two dead anti-diagonals to stop, first-reached end
// cell) are stated in include/xdrop.h.
//
// Layout on the device:
//   * reads: 2 bits per base, both orientations, in one word array;
//   * in the window kernels one wavefront runs one extension (task); all
//     control is wave-uniform and lives in SGPRs.  The narrow class (small
//     drops) runs two extensions per wavefront, one per half of the lanes,
//     with the per-half control in pairs of SGPRs and per-lane thresholds;
//     the 2048-slot class can share one window among the wavefronts of a
//     workgroup (one segment each, an LDS exchange per anti-diagonal);
//   * window kernels: the live band of anti-diagonals d-1 and d-2 is held in
//     VGPRs, 64 lanes x C cells, indexed by slot s = C*lane + r with
//     i = o_d + s and o_d = base + floor(d/2).  With that origin the diagonal
//     predecessor of a cell sits in the same slot two anti-diagonals back and
//     the two gap predecessors are slots (s-1, s) on odd d and (s, s+1) on
//     even d, so one DPP wave rotate per anti-diagonal feeds the recurrence;
//   * values are stored as Z = S + |gap| * d, which removes the gap add from
//     the recurrence; the drop and improvement thresholds move by |gap| per
//     anti-diagonal in SGPRs;
//   * work proceeds in blocks of up to 32 (odd, even) anti-diagonal pairs per
//     load of codes, run as halves of 16.  A block starts with the band away
//     from the window edges (re-centred through LDS if needed) and ends when
//     the even anti-diagonal of a pair has a live cell in an edge slot, which
//     keeps every candidate inside the window.  At one cell per lane a half
//     runs unrolled without tests and is rerun with them if an edge slot went
//     live.  A band that outgrows the window moves to a wider window through
//     LDS, or to the next class, which resumes from its carried state;
//   * unbounded kernel: one workgroup per extension, first in a 4096-slot
//     window shared by its wavefronts, then with the last three
//     anti-diagonals in an LDS ring indexed by i (global memory for bands
//     wider than the ring), any band width.
#include <hip/hip_runtime.h>

#include "xdrop_internal.h"

namespace xd {

namespace {

constexpr int NEG = -(1 << 30) - (1 << 20);   // dead / outside the table
constexpr int NEG_HALF = -(1 << 29);          // anything below is "no live predecessor"
constexpr int UMAX = 16;                      // anti-diagonal pairs per half block
constexpr int kRecentre = 4;                  // a block starting nearer an edge re-centres the band

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Wave-uniform fetch-and-add of `v` (the value of lane 0).  Every lane takes
// part (the others add 0) so that no lane-dependent branch surrounds the
// atomic: lane-divergent control flow next to cross-lane operations lets the
// compiler split a loop so that some lanes re-enter it without the others.
__device__ __forceinline__ uint32_t wave_fetch_add(uint32_t *p, uint32_t v)
{
    const uint32_t old = atomicAdd(p, (threadIdx.x & 63) == 0 ? v : 0u);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)old);
}

// bases p .. p+15 as 2-bit fields (base p in bits 0-1); reads one word past
// the base p+15 at most, which the store's guard words cover
__device__ __forceinline__ uint32_t codes16_at(const uint32_t *__restrict__ W, uint64_t p)
{
    const uint32_t *w = W + (p >> 4);
    return __builtin_amdgcn_alignbit(w[1], w[0], (uint32_t)(p & 15) * 2u);
}

// Guard of the store: reads keep at least kGuardWords words (8192 bases) before
// their first and after their last base.  A window always holds its live
// band, so a lane's code window reaches at most one window width (4096 slots
// at most) plus one block of codes past either end of its sequence and never
// leaves the store.
constexpr int kGuardWords = 512;

// 16*NW codes starting at code p of a sequence whose first base sits at bit
// 2*ph of word 0 of `seq` (seq = &store[first base / 16], ph = first base % 16):
// code t at bits 2*(t & 15) of out[t >> 4].  Reads NW+1 words through a
// wave-uniform base pointer and a 32-bit lane offset.
template <int NW>
__device__ __forceinline__ void load_codes(const uint32_t *__restrict__ seq, int ph, int p, uint32_t (&out)[NW])
{
    const int q = p + ph + 16 * kGuardWords;           // >= 0 for every window position
    const uint32_t *w = seq - kGuardWords + (q >> 4);
    const uint32_t sh = (uint32_t)(q & 15) * 2u;
    uint32_t raw[NW + 1];
#pragma unroll
    for (int i = 0; i <= NW; ++i) raw[i] = w[i];
#pragma unroll
    for (int i = 0; i < NW; ++i) out[i] = __builtin_amdgcn_alignbit(raw[i + 1], raw[i], sh);
}

// 16 codes starting at code f (compile-time) of a loaded window
template <int NW>
__device__ __forceinline__ uint32_t codes16(const uint32_t (&w)[NW], int f)
{
    const int q = f >> 4, r = f & 15;
    return r == 0 ? w[q] : __builtin_amdgcn_alignbit(w[q + 1], w[q], 2u * (uint32_t)r);
}

struct Geo {
    uint64_t abase, bbase;
    int32_t m, n;
};

// Orientation of one extension.  Both sequences are read forwards from the
// store: the right extension reads A and B' after the seed; the left
// extension reads the reverse complements of A and B' from the mirrored seed
// start.  Complementing both sides keeps every match/mismatch decision.
__device__ __forceinline__ Geo task_geo(const xdrop_record &R, const ReadInfo *__restrict__ ri, int side)
{
    const ReadInfo A = ri[R.read_a], B = ri[R.read_b];
    const uint32_t k = R.k;
    const uint32_t pb = R.strand ? B.len - R.pos_b - k : R.pos_b;
    Geo g;
    if (side) {
        g.m = (int32_t)(A.len - R.pos_a - k);
        g.n = (int32_t)(B.len - pb - k);
        g.abase = A.fwd + R.pos_a + k;
        g.bbase = (R.strand ? B.rc : B.fwd) + pb + k;
    } else {
        g.m = (int32_t)R.pos_a;
        g.n = (int32_t)pb;
        g.abase = A.rc + (A.len - R.pos_a);
        g.bbase = (R.strand ? B.fwd : B.rc) + (B.len - pb);
    }
    return g;
}

__device__ __forceinline__ uint64_t uni64(uint64_t x)
{
    return ((uint64_t)(uint32_t)uni((int)(x >> 32)) << 32) | (uint32_t)uni((int)(uint32_t)x);
}

// A task as wave-uniform scalars: the record and the geometry of one side.
struct Task {
    Geo g;
    int x, ma, mi, gap;
};

__device__ __forceinline__ Task load_task(const xdrop_record *__restrict__ recs, const ReadInfo *__restrict__ ri,
                                          uint32_t t)
{
    const xdrop_record R = recs[t >> 1];
    Geo g = task_geo(R, ri, (int)(t & 1));
    Task k;
    k.g.abase = uni64(g.abase);
    k.g.bbase = uni64(g.bbase);
    k.g.m = uni(g.m);
    k.g.n = uni(g.n);
    k.x = uni(R.x);
    k.ma = uni(R.match);
    k.mi = uni(R.mismatch);
    k.gap = uni(R.gap);
    return k;
}

__device__ __forceinline__ bool record_ok(const xdrop_record &R, const StoreDev &st)
{
    if (R.read_a >= st.n_reads || R.read_b >= st.n_reads) return false;
    const uint32_t la = st.reads[R.read_a].len, lb = st.reads[R.read_b].len;
    if (R.k < 1 || (uint64_t)R.pos_a + R.k > la || (uint64_t)R.pos_b + R.k > lb) return false;
    if (R.strand > 1 || R.x < 0 || R.x > XDROP_MAX_X) return false;
    if (R.match < 1 || R.match > 1024 || R.mismatch >= R.match || R.mismatch < -1024 ||
        R.gap > -1 || R.gap < -1024)
        return false;
    const int64_t w = (int64_t)R.match - R.mismatch - R.gap;
    if (w * ((int64_t)la + lb) > (1ll << 29)) return false;
    return true;
}

__device__ __forceinline__ int wave_max(int v)
{
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ int bucket_of(uint32_t key)
{
    // quarter-octave buckets of the expected extension length, longest first
    const uint32_t k = key + 1;
    const int lg = 31 - __clz(k);
    const int frac = lg >= 2 ? (int)((k >> (lg - 2)) & 3u) : 0;
    int b = lg * 4 + frac;
    b = b > kNumBuckets - 1 ? kNumBuckets - 1 : b;
    return kNumBuckets - 1 - b;
}

}  // namespace

// ---------------------------------------------------------------------------
// Counters reset (a kernel, so that it can sit inside a captured graph).
// ---------------------------------------------------------------------------
__global__ void reset_kernel(uint32_t *ctr, uint32_t *hist, unsigned long long *stage_sum, const uint32_t *n_src,
                             uint32_t n_imm)
{
    const int t = threadIdx.x;
    static_assert(CtrLayout::kWords <= 256, "one thread per counter word");
    if (t < CtrLayout::kWords && t != CtrLayout::kN) ctr[t] = 0;
    if (t == 0) ctr[CtrLayout::kN] = n_src ? *n_src : n_imm;
    if (t < kStageSumWords) stage_sum[t] = 0ull;
    for (int i = t; i < kNumClasses * kNumBuckets; i += blockDim.x) hist[i] = 0;
}

__global__ void accum_errors_kernel(const uint32_t *ctr, uint32_t *acc)
{
    if (threadIdx.x == 0) acc[0] += ctr[CtrLayout::kErrors];
}

// ---------------------------------------------------------------------------
// Record ingest: validation, seed score, class of both extensions.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) prep_kernel(BatchDev b, StoreDev st, Tuning tu, int stage)
{
    // per-block histogram of bucket keys, flushed with one global atomic per bin
    __shared__ uint32_t hist[kNumClasses * kNumBuckets];
    if (stage) {
        for (int i = threadIdx.x; i < kNumClasses * kNumBuckets; i += blockDim.x) hist[i] = 0;
        __syncthreads();
    }
    const uint32_t n = b.ctr[CtrLayout::kN];
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = r < n;
    xdrop_record R{};
    bool ok = false;
    if (in) {
        R = b.recs[r];
        ok = record_ok(R, st);
        b.valid[r] = ok ? 1 : 0;
        if (!ok) atomicAdd(&b.ctr[CtrLayout::kErrors], 1u);
    }
    int cls = -1;
    uint32_t key0 = 0, key1 = 0;
    if (ok) {
        const ReadInfo A = st.reads[R.read_a], B = st.reads[R.read_b];
        const uint32_t pb = R.strand ? B.len - R.pos_b - R.k : R.pos_b;
        const uint64_t aseed = A.fwd + R.pos_a;
        const uint64_t bseed = R.strand ? B.rc + pb : B.fwd + pb;
        // seed score: mismatches of 16 bases at a time (xor of 2-bit codes)
        uint32_t mism = 0;
        for (uint32_t t = 0; t < R.k; t += 16) {
            uint32_t x = codes16_at(st.words, aseed + t) ^ codes16_at(st.words, bseed + t);
            x = (x | (x >> 1)) & 0x55555555u;
            const uint32_t left = R.k - t;
            if (left < 16) x &= (1u << (2u * left)) - 1u;
            mism += (uint32_t)__builtin_popcount(x);
        }
        b.seed[r] = (int)(R.k - mism) * R.match + (int)mism * R.mismatch;
        // small drops with match 1, gap -1 and mismatch 0 / -1 / -2 in a
        // large batch: two extensions per wavefront (narrow class)
        const bool narrow = n >= (uint32_t)tu.narrow_min && R.x <= tu.narrow_x && R.match == 1 && R.gap == -1 &&
                            R.mismatch >= -2;
        cls = narrow ? kNarrowClass : kAdaptiveClass;
        key0 = min(R.pos_a, pb);
        key1 = min(A.len - R.pos_a - R.k, B.len - pb - R.k);
    }
    // wave-aggregated queue appends (two tasks per record, same class)
    uint32_t *dst = stage ? b.qkey : b.qbuf;
    const uint32_t qcap = 2u * b.cap;
    for (int q = 0; q < kNumClasses; ++q) {
        const uint64_t mask = ballot(cls == q);
        if (!mask) continue;
        const int lane = lane_id();
        const uint32_t cnt = 2u * (uint32_t)__builtin_popcountll(mask);
        const uint32_t base = wave_fetch_add(&b.ctr[(stage ? CtrLayout::kStage : CtrLayout::kCount) + q], cnt);
        if (cls == q) {
            const uint32_t before = 2u * (uint32_t)__builtin_popcountll(mask & ((1ull << lane) - 1ull));
            dst[q * qcap + base + before] = 2u * r;
            dst[q * qcap + base + before + 1] = 2u * r + 1u;
            if (stage) {
                atomicAdd(&hist[q * kNumBuckets + bucket_of(key0)], 1u);
                atomicAdd(&hist[q * kNumBuckets + bucket_of(key1)], 1u);
            }
        }
    }
    if (stage) {
        __syncthreads();
        for (int i = threadIdx.x; i < kNumClasses * kNumBuckets; i += blockDim.x)
            if (hist[i]) atomicAdd(&b.bucket_hist[i], hist[i]);
    }
}

// ---------------------------------------------------------------------------
// Length bucketing: counting sort of each class queue by quarter-octave
// buckets of min(remaining A, remaining B), longest first.
// ---------------------------------------------------------------------------
__global__ void bucket_scan_kernel(BatchDev b)
{
    // one thread per class: exclusive scan of its histogram, counts copied
    const int q = threadIdx.x;
    if (q >= kNumClasses) return;
    uint32_t acc = 0;
    for (int k = 0; k < kNumBuckets; ++k) {
        const uint32_t c = b.bucket_hist[q * kNumBuckets + k];
        b.bucket_hist[q * kNumBuckets + k] = acc;
        acc += c;
    }
    b.ctr[CtrLayout::kCount + q] = acc;
}

__global__ void __launch_bounds__(256) bucket_scatter_kernel(BatchDev b, StoreDev st)
{
    // ranks within the block come from LDS atomics; one global atomic per
    // (block, bucket) reserves the block's range (order inside a bucket is free)
    __shared__ uint32_t cnt_l[kNumBuckets], base_l[kNumBuckets];
    const uint32_t qcap = 2u * b.cap;
    const uint32_t first = blockIdx.x * blockDim.x;
    const uint32_t idx = first + threadIdx.x;
    for (int q = 0; q < kNumClasses; ++q) {
        const uint32_t cnt = b.ctr[CtrLayout::kStage + q];
        if (first >= cnt) continue;                  // uniform over the block
        for (int i = threadIdx.x; i < kNumBuckets; i += blockDim.x) cnt_l[i] = 0;
        __syncthreads();
        int bk = -1;
        uint32_t t = 0, rank = 0;
        if (idx < cnt) {
            t = b.qkey[q * qcap + idx];
            const xdrop_record R = b.recs[t >> 1];
            const ReadInfo A = st.reads[R.read_a], B = st.reads[R.read_b];
            const uint32_t pb = R.strand ? B.len - R.pos_b - R.k : R.pos_b;
            const uint32_t key = (t & 1) ? min(A.len - R.pos_a - R.k, B.len - pb - R.k) : min(R.pos_a, pb);
            bk = bucket_of(key);
            rank = atomicAdd(&cnt_l[bk], 1u);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kNumBuckets; i += blockDim.x)
            base_l[i] = cnt_l[i] ? atomicAdd(&b.bucket_hist[q * kNumBuckets + i], cnt_l[i]) : 0u;
        __syncthreads();
        if (bk >= 0) b.qbuf[q * qcap + base_l[bk] + rank] = t;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Register-window X-drop extension.
// ---------------------------------------------------------------------------

// Wave-uniform state of one extension; it survives changes of window width.
struct XState {
    int d;          // next anti-diagonal to compute
    int base;       // o_d = base + floor(d/2): i of slot 0 on anti-diagonal d
    int T, bi, bj;  // best score so far and its cell
    uint64_t cells;
    uint64_t slots; // slot-steps of the windows that ran the extension (cell counting)
    int mn, mx;     // live slots over the last two anti-diagonals (on kGrow / kShrink)
};

constexpr int WMAX = 256;   // widest window of the adaptive kernel (C = 4): LDS slots per array
enum : uint32_t { kDone = 0, kGrow = 1, kShrink = 2 };

// Per-anti-diagonal sigma term.  SIGF: sigma - 2*gap of a match and of a
// mismatch both lie in [0, 3]; each pair's value then sits in a 2-bit field
// of a per-block word (one bfe + one add per cell).  Otherwise the diagonal
// term is sm + bit * nd from the mismatch bit (bfe, mad, add).
template <int C, bool COUNT, bool MA1, bool SIGF, int STRIDE = WMAX>
struct Window {
    static constexpr int WIN = 64 * C;
    // pairs per block: two halves of UMAX pairs (one code load) for the
    // adaptive widths, one half for the wide windows (register budget)
    static constexpr int NH = C <= 4 ? 2 : 1;
    static constexpr int PB = NH * UMAX;
    static constexpr int NWC = (C + PB + 16) / 16;   // words of codes per lane and block
    static_assert(STRIDE >= WIN, "LDS stride must hold the window");

    int Z1[C];                // anti-diagonal d-1 (Z units: S + |gap| * d; NEG = dead)
    int Z2[C];                // anti-diagonal d-2
    uint32_t mmo[C], mme[C];  // per pair u: mismatch bit (bit 2u) or, SIGF, sigma field (bits 2u..2u+1)
    uint32_t mmo2[C], mme2[C];  // the same for pairs UMAX .. 2*UMAX-1 (NH = 2)

    // deferred end cell (MA1, C > 1): last improving anti-diagonal since the
    // last resolve(), its improvement mask over lanes and, per lane, the
    // first improving slot r
    int last_d;
    uint64_t last_imp;
    int last_r;
    // C = 1: the same per parity of d (odd / even step of a pair), as the
    // pair offset 2u of the step within its half (-1: none since resolve())
    int lu_o, lu_e;
    uint64_t li_o, li_e;

    // fresh extension: only (0,0) live, in the middle slot
    __device__ __forceinline__ void init(XState &s)
    {
        const int lane = lane_id();
        const int s0 = WIN / 2 - 1;
        s.base = -s0;
        s.d = 1;
        s.T = 0; s.bi = 0; s.bj = 0; s.cells = 0; s.slots = 0;
        s.mn = s.mx = s0;
#pragma unroll
        for (int r = 0; r < C; ++r) {
            Z1[r] = (C * lane + r == s0) ? 0 : NEG;
            Z2[r] = NEG;
        }
    }

    // window contents -> LDS, by slot
    __device__ __forceinline__ void save(int *lds) const
    {
        const int lane = lane_id();
#pragma unroll
        for (int r = 0; r < C; ++r) {
            lds[C * lane + r] = Z1[r];
            lds[STRIDE + C * lane + r] = Z2[r];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // take over a window of from_win slots saved in LDS: new slot s holds old slot s + delta
    __device__ __forceinline__ void load(const int *lds, int from_win, int delta)
    {
        const int lane = lane_id();
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const int s = C * lane + r + delta;
            const bool ok = s >= 0 && s < from_win;
            const int sc = ok ? s : 0;
            const int a = lds[sc], b2 = lds[STRIDE + sc];
            Z1[r] = ok ? a : NEG;
            Z2[r] = ok ? b2 : NEG;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // One anti-diagonal d (ODD = d & 1) at pair offset ub = 2u of the block.
    // tp / ti: drop and improvement thresholds of d in Z units (T_{d-1} - X
    // and T_{d-1}, plus |gap| * d); on return they hold those of d+1.  Returns
    // the live cells of d in the two edge slots on either side of the window
    // (bit per lane).
    template <bool ODD, bool BOUNDS, int KU = -1>
    __device__ __forceinline__ uint64_t step(XState &s, int d, uint32_t ub_rt, int &tp, int &ti, int sm, int nd,
                                             int G, int X, int lo_s = 0, int hi_s = 0)
    {
        // KU >= 0: the pair offset is the compile-time constant KU (unrolled loop)
        const uint32_t ub = KU >= 0 ? (uint32_t)KU : ub_rt;
        const int lane = lane_id();
        int t[C];
        // Gap predecessors come from the neighbouring slot of d-1, one lane
        // over at the lane boundary.  A wave rotate (no invalid lanes) feeds
        // it: the value wrapped into slot 0 / WIN-1 is that of the opposite
        // edge slot, which run() keeps dead.
        if (ODD) {
            // slots s-1 and s (wave_ror: lane l reads lane l-1, lane 0 reads lane 63)
            t[0] = max(__builtin_amdgcn_mov_dpp(Z1[C - 1], 0x13C, 0xf, 0xf, true), Z1[0]);
#pragma unroll
            for (int r = 1; r < C; ++r) t[r] = max(Z1[r - 1], Z1[r]);
        } else {
            // slots s and s+1 (wave_rol: lane l reads lane l+1, lane 63 reads lane 0)
#pragma unroll
            for (int r = 0; r < C - 1; ++r) t[r] = max(Z1[r], Z1[r + 1]);
            t[C - 1] = max(__builtin_amdgcn_mov_dpp(Z1[0], 0x134, 0xf, 0xf, true), Z1[C - 1]);
        }
        // BOUNDS: candidates only in slots lo_s .. hi_s (j <= n, i <= m)
        uint64_t imp = 0, lm[C];
        int v[C];
        // Without clipping and with several cells per lane, the improvement
        // test compares the lane's largest value once (a max3 tree, about C/2
        // vector ops) instead of every cell, whose C masks would also cost
        // C-1 scalar ORs per anti-diagonal.
        constexpr bool LANE_MAX = !BOUNDS && C > 1;
        int vm = NEG;
        if (COUNT) s.slots += (uint64_t)WIN;
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const uint32_t w = ODD ? mmo[r] : mme[r];
            int sig;
            if (SIGF) {
                sig = (int)__builtin_amdgcn_ubfe(w, ub, 2u);
            } else {
                const int bit = (int)__builtin_amdgcn_ubfe(w, ub, 1u);
                sig = __mul24(bit, nd) + sm;          // sigma - 2*gap
            }
            v[r] = max(t[r], Z2[r] + sig);
            // lane masks from single compares (a ballot of a compound
            // condition costs two extra vector ops)
            const int sl = C * lane + r;
            const uint64_t inbm = BOUNDS ? ballot(sl >= lo_s) & ballot(sl <= hi_s) : ~0ull;
            if (LANE_MAX)
                vm = max(vm, v[r]);
            else
                imp |= ballot(v[r] > ti) & inbm;
            if (COUNT) s.cells += (uint64_t)__builtin_popcountll(ballot(v[r] > NEG_HALF) & inbm);
            lm[r] = ballot(v[r] >= tp) & inbm;
            const bool keep = BOUNDS ? (sl >= lo_s && sl <= hi_s && v[r] >= tp) : v[r] >= tp;
            t[r] = keep ? v[r] : NEG;
        }
        if (LANE_MAX) imp = ballot(vm > ti);
        if (MA1 && C == 1) {
            // match weight 1: an improving cell holds exactly T_{d-1} + 1.
            // Keep the last improvement mask and pair offset of this parity,
            // then ti += G + (imp != 0) and tp = ti - X, all on the scalar
            // unit without a branch.
            uint64_t &li = ODD ? li_o : li_e;
            int &lu = ODD ? lu_o : lu_e;
            if (KU >= 0) {
                asm volatile("s_cmp_lg_u64 %[imp], 0\n\t"
                             "s_cselect_b64 %[li], %[imp], %[li]\n\t"
                             "s_cselect_b32 %[lu], %[ub], %[lu]\n\t"
                             "s_addc_u32 %[ti], %[ti], %[g]\n\t"
                             "s_sub_i32 %[tp], %[ti], %[x]"
                             : [li] "+s"(li), [lu] "+s"(lu), [ti] "+s"(ti), [tp] "=s"(tp)
                             : [imp] "s"(imp), [ub] "i"(KU < 0 ? 0 : KU), [g] "s"(G), [x] "s"(X)
                             : "scc");
            } else {
                asm volatile("s_cmp_lg_u64 %[imp], 0\n\t"
                             "s_cselect_b64 %[li], %[imp], %[li]\n\t"
                             "s_cselect_b32 %[lu], %[ub], %[lu]\n\t"
                             "s_addc_u32 %[ti], %[ti], %[g]\n\t"
                             "s_sub_i32 %[tp], %[ti], %[x]"
                             : [li] "+s"(li), [lu] "+s"(lu), [ti] "+s"(ti), [tp] "=s"(tp)
                             : [imp] "s"(imp), [ub] "s"(ub), [g] "s"(G), [x] "s"(X)
                             : "scc");
            }
        } else if (MA1) {
            if (imp) {
                last_d = d;
                last_imp = imp;
                int rl = C - 1;
#pragma unroll
                for (int r = C - 1; r >= 0; --r) {
                    const int sl = C * lane + r;
                    const bool inb = !BOUNDS || (sl >= lo_s && sl <= hi_s);
                    if (inb && v[r] > ti) rl = r;
                }
                last_r = rl;
                ++tp;
                ++ti;
            }
            tp += G;
            ti += G;
        } else {
            if (imp) {
                int lm_ = vm;
                if (!LANE_MAX) {
#pragma unroll
                    for (int r = 0; r < C; ++r) {
                        const int sl = C * lane + r;
                        const bool inb = !BOUNDS || (sl >= lo_s && sl <= hi_s);
                        lm_ = max(lm_, inb ? v[r] : NEG);
                    }
                }
                const int vmax = uni(wave_max(lm_));
                // first slot (smallest lane, then smallest r) holding vmax
                int rl = C;
#pragma unroll
                for (int r = C - 1; r >= 0; --r) {
                    const int sl = C * lane + r;
                    const bool inb = !BOUNDS || (sl >= lo_s && sl <= hi_s);
                    if (inb && v[r] == vmax) rl = r;
                }
                const uint64_t any = ballot(rl < C);
                const int l = __builtin_ctzll(any);
                const int rr = __builtin_amdgcn_readlane(rl, l);
                s.bi = s.base + (d >> 1) + C * l + rr;
                s.bj = d - s.bi;
                tp += vmax - ti;
                ti = vmax;
            }
            tp += G;
            ti += G;
        }
#pragma unroll
        for (int r = 0; r < C; ++r) {
            Z2[r] = Z1[r];
            Z1[r] = t[r];
        }
        // slots 0, 1 (lane 0 unless C = 1) and WIN-2, WIN-1 (lane 63 unless C = 1)
        if (C == 1) return lm[0];   // next_pair masks lanes 0, 1, 62, 63
        return ((lm[0] | lm[1]) & 1ull) | ((lm[C - 2] | lm[C - 1]) & (1ull << 63));
    }

    // end cell of the last improvement recorded in the half that began at d0
    // (MA1): at C = 1 the later of the last odd and the last even improving step
    __device__ __forceinline__ void resolve(XState &s, int d0)
    {
        if (!MA1) return;
        if (C == 1) {
            if ((lu_o & lu_e) < 0) return;                 // both -1: none
            const bool ev = lu_e >= lu_o;
            const uint64_t im = ev ? li_e : li_o;
            const int dd = d0 + (ev ? lu_e + 1 : lu_o);
            s.bi = s.base + (dd >> 1) + __builtin_ctzll(im);
            s.bj = dd - s.bi;
            lu_o = lu_e = -1;
            return;
        }
        if (last_d < 0) return;
        const int l = __builtin_ctzll(last_imp);
        const int rr = __builtin_amdgcn_readlane(last_r, l);
        s.bi = s.base + (last_d >> 1) + C * l + rr;
        s.bj = last_d - s.bi;
        last_d = -1;
    }

    // ub + 2, plus 64 when e has a live edge cell: s_and_b64 sets SCC, a
    // select and one add (a second loop exit would cost a chain of selects)
    __device__ __forceinline__ static uint32_t next_pair(uint32_t ub, uint64_t e)
    {
        const uint64_t edge = C == 1 ? 0xC000000000000003ull : ~0ull;
        uint64_t tmp;
        uint32_t inc;
        asm volatile("s_and_b64 %[tmp], %[e], %[edge]\n\t"
                     "s_cselect_b32 %[inc], 66, 2\n\t"
                     "s_add_u32 %[ub], %[ub], %[inc]"
                     : [tmp] "=&s"(tmp), [inc] "=&s"(inc), [ub] "+s"(ub)
                     : [e] "s"(e), [edge] "s"(edge)
                     : "scc");
        return ub;
    }

    // Up to np <= UMAX pairs from odd anti-diagonal d0 on the current sigma
    // words.  Under the invariant (band of d-1 inside [2, WIN-3], of d-2 inside
    // [1, WIN-2]) the odd step's live cells stay in [1, WIN-2] and the even
    // step's in [0, WIN-2]; only the even step needs the edge check.  The loop
    // counts in ub = 2u (the bit offset of pair u in the code words); a live
    // edge cell adds 64 on top, which ends the loop (2 * UMAX < 64) and
    // leaves the pair count in the low bits.  Returns ub.
    // UMAX pairs without clipping, unrolled and without a test between them:
    // bit offsets and recorded pair offsets are immediates and the live masks
    // of the even steps are OR-ed into acc.  Exact if acc ends with no edge
    // lane set (then the invariant held before every pair); otherwise the
    // caller restores the state and reruns the half with pairs<false>.
    template <int K = 0>
    __device__ __forceinline__ uint64_t pairs_spec(XState &s, int d0, int &tp, int &ti, int sm, int nd, int G,
                                                   int X, int m, int n, uint64_t acc)
    {
        if constexpr (K == UMAX) {
            return acc;
        } else {
            step<true, false, 2 * K>(s, d0 + 2 * K, 0u, tp, ti, sm, nd, G, X);
            acc |= step<false, false, 2 * K>(s, d0 + 2 * K + 1, 0u, tp, ti, sm, nd, G, X);
            return pairs_spec<K + 1>(s, d0, tp, ti, sm, nd, G, X, m, n, acc);
        }
    }

    // one half of UMAX pairs at C = 1 without clipping: speculative run,
    // rolled back and rerun with per-pair checks if an edge lane went live
    __device__ __forceinline__ uint32_t half_c1(XState &s, int d0, int &tp, int &ti, int sm, int nd, int G, int X,
                                                int m, int n)
    {
        const int z1 = Z1[0], z2 = Z2[0], tp0 = tp, ti0 = ti, luo = lu_o, lue = lu_e;
        const uint64_t lio = li_o, lie = li_e, cells0 = s.cells, slots0 = s.slots;
        const uint64_t acc = pairs_spec(s, d0, tp, ti, sm, nd, G, X, m, n, 0ull);
        if (!(acc & 0xC000000000000003ull)) return 2u * UMAX;   // lanes 0, 1, 62, 63
        Z1[0] = z1; Z2[0] = z2; tp = tp0; ti = ti0;
        lu_o = luo; lu_e = lue; li_o = lio; li_e = lie; s.cells = cells0; s.slots = slots0;
        return pairs<false>(s, d0, UMAX, tp, ti, sm, nd, G, X, m, n);
    }

    template <bool BOUNDS>
    __device__ __forceinline__ uint32_t pairs(XState &s, int d0, int np, int &tp, int &ti, int sm, int nd, int G,
                                              int X, int m, int n)
    {
        // clipping (BOUNDS): only j <= n and i <= m can fail, since a cell
        // with i < 0 or j < 0 has no live predecessor (moves never decrease
        // i or j from (0, 0)).  With o = base + floor(d/2) the lowest slot
        // with j <= n, d - n - o, rises by one per pair at the odd step; the
        // highest slot with i <= m, m - o, falls by one at the even step.
        const int o0 = s.base + (d0 >> 1);
        int lo_s = d0 - n - o0, hi_s = m - o0;
        const uint32_t ube = 2u * (uint32_t)np;
        uint32_t ub = 0;
        do {
            step<true, BOUNDS>(s, d0 + (int)ub, ub, tp, ti, sm, nd, G, X, lo_s, hi_s);
            const uint64_t e =
                step<false, BOUNDS>(s, d0 + (int)ub + 1, ub, tp, ti, sm, nd, G, X, lo_s, hi_s - 1);
            ++lo_s;
            --hi_s;
            ub = next_pair(ub, e);
        } while (ub < ube);
        return ub;
    }

    // some live slot on the last two anti-diagonals
    __device__ __forceinline__ bool alive() const
    {
        int z = NEG;
#pragma unroll
        for (int r = 0; r < C; ++r) z = max(z, max(Z1[r], Z2[r]));
        return ballot(z > NEG_HALF) != 0;
    }

    // live slots over the last two anti-diagonals; false when both are dead
    __device__ __forceinline__ bool band(int &mn, int &mx) const
    {
        mn = 1 << 30;
        mx = -1;
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const uint64_t u = ballot(max(Z1[r], Z2[r]) > NEG_HALF);
            if (u) {
                mn = min(mn, C * __builtin_ctzll(u) + r);
                mx = max(mx, C * (63 - __builtin_clzll(u)) + r);
            }
        }
        return mx >= 0;
    }

    // Advance the extension block by block.  Returns kDone, or kGrow / kShrink
    // with the window saved to LDS and s.mn / s.mx set (shrink_width < 0: never).
    //
    // A block covers up to PB anti-diagonal pairs (odd d, even d+1) with one
    // load of codes.  The odd step of a pair can add a candidate one slot to
    // the right of the band, the even step one slot to the left.  A block
    // starts with the live band of the last two anti-diagonals inside
    // [2, WIN-3] and ends after the first pair whose even anti-diagonal has a
    // live cell in slot 0, 1, WIN-2 or WIN-1.  Before every pair the even
    // anti-diagonal is then live inside [2, WIN-3] and the odd one inside
    // [1, WIN-2]: every candidate lies in the window and the value a rotate
    // wraps around from the far edge slot is dead.
    __device__ uint32_t run(const uint32_t *__restrict__ W, const Geo &g, int X, int ma, int mi,
                            int gap, int *lds, XState &s, int shrink_width)
    {
        const int lane = lane_id();
        const int m = g.m, n = g.n;
        const int G = -gap;
        const int sm = ma + 2 * G;          // sigma(match) - 2*gap
        const int sx = mi + 2 * G;          // sigma(mismatch) - 2*gap
        const int nd = mi - ma;             // mismatch - match
        const int dend = m + n;
        const uint32_t *aseq = W + (g.abase >> 4), *bseq = W + (g.bbase >> 4);
        const int aph = (int)(g.abase & 15), bph = (int)(g.bbase & 15);
        last_d = -1;
        lu_o = lu_e = -1;
        li_o = li_e = 0;
        // improvement threshold of s.d in Z units, carried from block to block
        int ti = s.T + G * s.d;
        while (s.d <= dend) {
            int mn, mx;
            if (!band(mn, mx)) break;                 // two dead anti-diagonals
            const int width = mx - mn + 1;
            if (width + 4 > WIN || width <= shrink_width) {
                save(lds);
                s.mn = mn;
                s.mx = mx;
                s.T = ti - G * s.d;
                return width + 4 > WIN ? kGrow : kShrink;
            }
            // re-centre the band when it starts closer than kRecentre slots to an edge
            if (min(mn, WIN - 1 - mx) < kRecentre) {
                const int delta = mn - (WIN - width) / 2;
                save(lds);
                load(lds, WIN, delta);
                s.base += delta;
            }
            const int d = s.d;
            const int P = min(PB, (dend - d + 2) >> 1);      // pairs up to the far corner
            // codes for this block: slot r of this lane meets a[A0 + C*lane + r + u
            // (+1 on even d)] and b[B0 - C*lane - r + u] at pair u
            const int e0 = (d - 1) >> 1;
            const int A0 = s.base + e0 - 1;
            const int B0 = e0 - s.base;
            uint32_t aw[NWC], bw[NWC];
            load_codes<NWC>(aseq, aph, A0 + C * lane, aw);
            load_codes<NWC>(bseq, bph, B0 - C * lane - (C - 1), bw);
#pragma unroll
            for (int h = 0; h < NH; ++h) {
#pragma unroll
                for (int r = 0; r < C; ++r) {
                    const uint32_t bb = codes16<NWC>(bw, C - 1 - r + 16 * h);
                    const uint32_t xo = codes16<NWC>(aw, r + 16 * h) ^ bb;
                    const uint32_t xe = codes16<NWC>(aw, r + 1 + 16 * h) ^ bb;
                    const uint32_t mo = (xo | (xo >> 1)) & 0x55555555u;   // 1 = mismatch, at bit 2u
                    const uint32_t me = (xe | (xe >> 1)) & 0x55555555u;
                    uint32_t fo = mo, fe = me;
                    if (SIGF) {
                        // field u = sigma'' of pair u: sm ^ (mismatch ? sm ^ sx : 0)
                        const uint32_t base_f = (uint32_t)sm * 0x55555555u;
                        const uint32_t k = (uint32_t)(sm ^ sx);
                        fo = base_f ^ ((k & 1u) ? mo : 0u) ^ ((k & 2u) ? (mo << 1) : 0u);
                        fe = base_f ^ ((k & 1u) ? me : 0u) ^ ((k & 2u) ? (me << 1) : 0u);
                    }
                    if (h == 0) { mmo[r] = fo; mme[r] = fe; }
                    else { mmo2[r] = fo; mme2[r] = fe; }
                }
            }
            int tp = ti - X;
            const int dlast = d + 2 * P - 1;
            // no clipping needed when every slot that can hold a candidate
            // (0 .. WIN-2) of every anti-diagonal of the block has i <= m and
            // j <= n; i >= 0 and j >= 0 hold for every candidate
            const int o_last = s.base + (dlast >> 1);
            const bool fast = o_last + WIN - 2 <= m && o_last >= dlast - n;
            const int p0 = min(P, UMAX);
            uint32_t ub;
            if (C == 1 && MA1 && fast && p0 == UMAX)
                ub = half_c1(s, d, tp, ti, sm, nd, G, X, m, n);
            else if (fast)
                ub = pairs<false>(s, d, p0, tp, ti, sm, nd, G, X, m, n);
            else
                ub = pairs<true>(s, d, p0, tp, ti, sm, nd, G, X, m, n);
            int u = (int)(ub & 63u) >> 1;
            if (NH == 2 && ub < 64u && P > UMAX && alive()) {
                // second half: end cell of the first, then its sigma words
                resolve(s, d);
                const int d1 = d + 2 * UMAX;
#pragma unroll
                for (int r = 0; r < C; ++r) {
                    mmo[r] = mmo2[r];
                    mme[r] = mme2[r];
                }
                if (C == 1 && MA1 && fast && P == PB)
                    ub = half_c1(s, d1, tp, ti, sm, nd, G, X, m, n);
                else if (fast)
                    ub = pairs<false>(s, d1, P - UMAX, tp, ti, sm, nd, G, X, m, n);
                else
                    ub = pairs<true>(s, d1, P - UMAX, tp, ti, sm, nd, G, X, m, n);
                u = UMAX + ((int)(ub & 63u) >> 1);
                resolve(s, d1);
            } else {
                resolve(s, d);
            }
            s.d = d + 2 * u;
        }
        s.T = ti - G * s.d;
        return kDone;
    }
};


// sigma - 2*gap of a match and of a mismatch both in [0, 3]
__device__ __forceinline__ bool sigma_fits_2bits(const Task &k)
{
    const int sm = k.ma - 2 * k.gap, sx = k.mi - 2 * k.gap;
    return sm >= 0 && sm <= 3 && sx >= 0 && sx <= 3;
}

// Smallest adaptive width (cells per lane) whose window holds `width` live
// slots with `margin` slots of slack on each side; 0 if none does.
__device__ __forceinline__ int fit_c(int width, int margin)
{
#pragma unroll
    for (int c = 1; c <= 4; ++c)
        if (width + 2 * margin <= 64 * c) return c;
    return 0;
}
// (a window must hold the band plus one block pair and one edge slot per side)

// One extension with a window that widens and narrows with its band:
// C = 1..4 cells per lane, the live band handed over through LDS.  Returns
// false if the band outgrew the widest window; the window is then saved in
// LDS (win_out slots per anti-diagonal) for the hand-over to the next class.
template <bool COUNT, bool MA1, bool SIGF>
__device__ bool run_adaptive(const uint32_t *__restrict__ W, const Task &k, int *lds, XState &s,
                             int grow_margin, int shrink_margin, int &win_out)
{
    // margins >= 2: a band that was just narrowed fits its new window with
    // two free slots per side (an edge slot plus one pair), so it cannot be
    // widened again before a block runs
    grow_margin = max(grow_margin, 2);
    shrink_margin = max(shrink_margin, 2);
    int C = 1, from_win = 0, delta = 0;
    bool fresh = true;
    for (;;) {
        // narrow back once the band fits the next smaller window with shrink_margin to spare
        const int shrink_width = C > 1 ? 64 * (C - 1) - 2 * shrink_margin : -1;
        uint32_t st;
        switch (C) {
        case 1: {
            Window<1, COUNT, MA1, SIGF> w;
            if (fresh) w.init(s); else w.load(lds, from_win, delta);
            st = w.run(W, k.g, k.x, k.ma, k.mi, k.gap, lds, s, shrink_width);
        } break;
        case 2: {
            Window<2, COUNT, MA1, SIGF> w;
            if (fresh) w.init(s); else w.load(lds, from_win, delta);
            st = w.run(W, k.g, k.x, k.ma, k.mi, k.gap, lds, s, shrink_width);
        } break;
        case 3: {
            Window<3, COUNT, MA1, SIGF> w;
            if (fresh) w.init(s); else w.load(lds, from_win, delta);
            st = w.run(W, k.g, k.x, k.ma, k.mi, k.gap, lds, s, shrink_width);
        } break;
        default: {
            Window<4, COUNT, MA1, SIGF> w;
            if (fresh) w.init(s); else w.load(lds, from_win, delta);
            st = w.run(W, k.g, k.x, k.ma, k.mi, k.gap, lds, s, shrink_width);
        } break;
        }
        if (st == kDone) return true;
        fresh = false;
        const int width = s.mx - s.mn + 1;
        int nc;
        if (st == kGrow) {
            nc = fit_c(width, grow_margin);
            if (nc == 0) nc = fit_c(width, 2);
            if (nc == 0) {
                win_out = 64 * C;   // the window run() saved to LDS
                return false;
            }
        } else {
            nc = C - 1;
        }
        from_win = 64 * C;
        delta = s.mn - (64 * nc - width) / 2;
        s.base += delta;
        C = nc;
    }
}

// ---------------------------------------------------------------------------
// Narrow class: two extensions per wavefront.
//
// Small drops keep small bands: at X = 20 and 15 % error an extension holds
// about 20 live cells, a third of a 64-lane window.  Here each half of the
// wavefront (a "group" of 32 lanes) runs its own extension in a window of
// 32*C slots, C = 1 or 2 cells per lane (the same for both groups): slot
// s = C*(lane & 31) + r of the group, cell i = o_d + s as in Window.  The
// groups step together, one anti-diagonal of each per step and both at the
// same parity, so one step is the instruction sequence of one window: one
// 64-lane DPP rotate feeds the gap predecessors of both groups (the value it
// moves across the middle comes from an edge slot, which band control keeps
// dead as at the wave's ends).  What differs per group lives per lane
// (thresholds, drop, clipping bounds, sigma fields) or in a pair of SGPRs
// (band control, end cell, sequences).
//
// Only weights with match 1 and gap -1 (mismatch 0, -1 or -2) come here: an
// improving cell then holds exactly T + 1, so each group's threshold rises
// by 1 + (improvement) per anti-diagonal -- one v_addc per step for both
// groups, fed by a per-group "improved" mask built on the scalar unit.  A
// group whose extension ends takes the next task at the start of the next
// block (blocks start at odd anti-diagonals, as every extension does); a
// band wider than a 64-slot window sends its task to the adaptive class,
// where it restarts.
// ---------------------------------------------------------------------------
constexpr uint32_t kNoTask = 0xffffffffu;

// Wave-uniform state of the extension of one group.
struct GroupX {
    uint32_t t;          // task, kNoTask when the group is empty
    int d, base;         // next anti-diagonal; slot 0 of anti-diagonal d holds i = base + floor(d/2)
    int bi, bj;          // best cell so far (the best score is the group's threshold minus d)
    int m, n, x, sx;     // lengths, drop, sigma - 2*gap of a mismatch (a match: 3)
    uint64_t abase, bbase;
    uint64_t cells, slots;
    uint32_t li;         // group lanes that improved at the group's last improving step of the half
    int lu;              // that step's offset in the half (-1: none)
    int mn, mx;          // live slots over the last two anti-diagonals (set at block starts)
};

constexpr int kNarrowSm = 3;   // sigma - 2*gap of a match (match 1, gap -1)

template <int C, bool COUNT>
struct PairWin {
    static constexpr int WIN = 32 * C;                 // slots per group
    static constexpr int PB = 2 * UMAX;                // pairs per block: two halves per load of codes
    static constexpr int NWC = (C + PB + 16) / 16;     // words of codes per lane and block
    static constexpr int STRIDE = 128;                 // LDS slots per anti-diagonal (two groups of <= 64)
    // edge slots 0, 1, WIN-2, WIN-1 of both groups
    static constexpr uint64_t EDGE = C == 1 ? 0xC0000003C0000003ull : 0x8000000180000001ull;

    int Z1[C], Z2[C];               // anti-diagonals d-1 and d-2 in Z units (S + d); NEG = dead
    uint32_t mmo[C], mme[C];        // sigma'' fields of the pairs of the current half
    uint32_t mmo2[C], mme2[C];      // the same for the second half
    int rs;                         // C = 2: first improving r of this lane at its group's last improving step

    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int r = 0; r < C; ++r) { Z1[r] = NEG; Z2[r] = NEG; }
        rs = 0;
    }

    // lanes of group g: a fresh extension (only (0,0) live, in the middle
    // slot) or, fresh = false, all dead
    __device__ __forceinline__ void set_group(int g, bool fresh)
    {
        const int lane = lane_id();
        const bool mine = (lane >> 5) == g;
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const int s = C * (lane & 31) + r;
            Z1[r] = mine ? ((fresh && s == WIN / 2 - 1) ? 0 : NEG) : Z1[r];
            Z2[r] = mine ? NEG : Z2[r];
        }
    }

    __device__ __forceinline__ void save(int *lds) const
    {
        const int lane = lane_id();
#pragma unroll
        for (int r = 0; r < C; ++r) {
            lds[C * lane + r] = Z1[r];
            lds[STRIDE + C * lane + r] = Z2[r];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // take over windows of from_win slots per group saved in LDS: new slot s
    // of a group holds its old slot s + dl (dl: this lane's group's shift)
    __device__ __forceinline__ void load(const int *lds, int from_win, int dl)
    {
        const int lane = lane_id(), g = lane >> 5;
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const int s = C * (lane & 31) + r + dl;
            const bool ok = s >= 0 && s < from_win;
            const int idx = g * from_win + (ok ? s : 0);
            const int a = lds[idx], b2 = lds[STRIDE + idx];
            Z1[r] = ok ? a : NEG;
            Z2[r] = ok ? b2 : NEG;
        }
        rs = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // live slots of each group over the last two anti-diagonals
    __device__ __forceinline__ void bands(GroupX &g0, GroupX &g1) const
    {
        g0.mn = g1.mn = 1 << 30;
        g0.mx = g1.mx = -1;
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const uint64_t u = ballot(max(Z1[r], Z2[r]) > NEG_HALF);
            const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
            if (lo) {
                g0.mn = min(g0.mn, C * __builtin_ctz(lo) + r);
                g0.mx = max(g0.mx, C * (31 - __builtin_clz(lo)) + r);
            }
            if (hi) {
                g1.mn = min(g1.mn, C * __builtin_ctz(hi) + r);
                g1.mx = max(g1.mx, C * (31 - __builtin_clz(hi)) + r);
            }
        }
    }

    __device__ __forceinline__ bool alive() const
    {
        int z = NEG;
#pragma unroll
        for (int r = 0; r < C; ++r) z = max(z, max(Z1[r], Z2[r]));
        return ballot(z > NEG_HALF) != 0;
    }

    // Per group: keep the improvement mask and step offset `so` of this step
    // when the group improved; returns the lanes of the groups that improved.
    template <int SO>
    __device__ __forceinline__ static uint64_t record(GroupX &g0, GroupX &g1, uint64_t imp, uint32_t so_rt)
    {
        const uint32_t ilo = (uint32_t)imp, ihi = (uint32_t)(imp >> 32);
        uint32_t mlo, mhi;
        if (SO >= 0) {
            asm volatile("s_cmp_lg_u32 %[ilo], 0\n\t"
                         "s_cselect_b32 %[li0], %[ilo], %[li0]\n\t"
                         "s_cselect_b32 %[lu0], %[so], %[lu0]\n\t"
                         "s_cselect_b32 %[mlo], -1, 0\n\t"
                         "s_cmp_lg_u32 %[ihi], 0\n\t"
                         "s_cselect_b32 %[li1], %[ihi], %[li1]\n\t"
                         "s_cselect_b32 %[lu1], %[so], %[lu1]\n\t"
                         "s_cselect_b32 %[mhi], -1, 0"
                         : [li0] "+s"(g0.li), [lu0] "+s"(g0.lu), [li1] "+s"(g1.li), [lu1] "+s"(g1.lu),
                           [mlo] "=&s"(mlo), [mhi] "=&s"(mhi)
                         : [ilo] "s"(ilo), [ihi] "s"(ihi), [so] "i"(SO < 0 ? 0 : SO)
                         : "scc");
        } else {
            asm volatile("s_cmp_lg_u32 %[ilo], 0\n\t"
                         "s_cselect_b32 %[li0], %[ilo], %[li0]\n\t"
                         "s_cselect_b32 %[lu0], %[so], %[lu0]\n\t"
                         "s_cselect_b32 %[mlo], -1, 0\n\t"
                         "s_cmp_lg_u32 %[ihi], 0\n\t"
                         "s_cselect_b32 %[li1], %[ihi], %[li1]\n\t"
                         "s_cselect_b32 %[lu1], %[so], %[lu1]\n\t"
                         "s_cselect_b32 %[mhi], -1, 0"
                         : [li0] "+s"(g0.li), [lu0] "+s"(g0.lu), [li1] "+s"(g1.li), [lu1] "+s"(g1.lu),
                           [mlo] "=&s"(mlo), [mhi] "=&s"(mhi)
                         : [ilo] "s"(ilo), [ihi] "s"(ihi), [so] "s"(so_rt)
                         : "scc");
        }
        return ((uint64_t)mhi << 32) | mlo;
    }

    // One anti-diagonal of both groups.  ub: bit offset 2u of the pair in the
    // sigma words (KU >= 0: the constant KU); ti / tp: this lane's group's
    // improvement and drop thresholds in Z units, on return those of the next
    // anti-diagonal; lo_s / hi_s (BOUNDS): this lane's group's candidate
    // slots.  Returns the live-cell mask of the step (edge lanes tested by
    // the caller).
    template <bool ODD, bool BOUNDS, int KU = -1>
    __device__ __forceinline__ uint64_t step(GroupX &g0, GroupX &g1, uint32_t ub_rt, int &ti, int &tp, int xv,
                                             int lo_s, int hi_s, uint32_t sinc0, uint32_t sinc1)
    {
        const uint32_t ub = KU >= 0 ? (uint32_t)KU : ub_rt;
        const int lane = lane_id();
        int t[C];
        if (ODD) {
            t[0] = max(__builtin_amdgcn_mov_dpp(Z1[C - 1], 0x13C, 0xf, 0xf, true), Z1[0]);   // wave_ror:1
#pragma unroll
            for (int r = 1; r < C; ++r) t[r] = max(Z1[r - 1], Z1[r]);
        } else {
#pragma unroll
            for (int r = 0; r < C - 1; ++r) t[r] = max(Z1[r], Z1[r + 1]);
            t[C - 1] = max(__builtin_amdgcn_mov_dpp(Z1[0], 0x134, 0xf, 0xf, true), Z1[C - 1]);   // wave_rol:1
        }
        uint64_t imp = 0, imp0 = 0, lm = 0;
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const uint32_t w = ODD ? mmo[r] : mme[r];
            const int v = max(t[r], Z2[r] + (int)__builtin_amdgcn_ubfe(w, ub, 2u));
            const int sl = C * (lane & 31) + r;
            const uint64_t inbm = BOUNDS ? ballot(sl >= lo_s) & ballot(sl <= hi_s) : ~0ull;
            const uint64_t ir = ballot(v > ti) & inbm;
            if (r == 0) imp0 = ir;
            imp |= ir;
            if (COUNT) {
                const uint64_t cm = ballot(v > NEG_HALF) & inbm;
                g0.cells += (uint64_t)__builtin_popcount((uint32_t)cm);
                g1.cells += (uint64_t)__builtin_popcount((uint32_t)(cm >> 32));
            }
            lm |= ballot(v >= tp) & inbm;
            const bool keep = BOUNDS ? (sl >= lo_s && sl <= hi_s && v >= tp) : v >= tp;
            t[r] = keep ? v : NEG;
        }
        if (COUNT) {
            g0.slots += sinc0;
            g1.slots += sinc1;
        }
        // step offset in the half: 2u on the odd step, 2u + 1 on the even one
        uint64_t mg;
        if (KU >= 0)
            mg = record<KU < 0 ? 0 : (ODD ? KU : KU + 1)>(g0, g1, imp, 0u);
        else
            mg = record<-1>(g0, g1, imp, ODD ? ub : ub + 1u);
        // ti += 1 + (this lane's group improved), tp = ti - x
        uint64_t co;
        asm("v_addc_co_u32_e64 %0, %1, %2, 1, %3" : "=v"(ti), "=s"(co) : "v"(ti), "s"(mg));
        tp = ti - xv;
        if (C > 1) {
            const int rcur = ((imp0 >> lane) & 1ull) ? 0 : 1;
            rs = ((mg >> lane) & 1ull) ? rcur : rs;
        }
#pragma unroll
        for (int r = 0; r < C; ++r) {
            Z2[r] = Z1[r];
            Z1[r] = t[r];
        }
        return lm;
    }

    // ub + 2, plus 64 when e has a live cell in an edge slot of either group
    __device__ __forceinline__ static uint32_t next_pair(uint32_t ub, uint64_t e)
    {
        const uint64_t edge = EDGE;
        uint64_t tmp;
        uint32_t inc;
        asm volatile("s_and_b64 %[tmp], %[e], %[edge]\n\t"
                     "s_cselect_b32 %[inc], 66, 2\n\t"
                     "s_add_u32 %[ub], %[ub], %[inc]"
                     : [tmp] "=&s"(tmp), [inc] "=&s"(inc), [ub] "+s"(ub)
                     : [e] "s"(e), [edge] "s"(edge)
                     : "scc");
        return ub;
    }

    // this lane's group's candidate slots on the first anti-diagonal of the
    // half starting dh anti-diagonals after the block start (j <= n: slot >=
    // d - n - o; i <= m: slot <= m - o); none for an empty group
    __device__ __forceinline__ static void bounds_at(const GroupX &g0, const GroupX &g1, int dh, int &lo_s,
                                                     int &hi_s)
    {
        const int o0 = g0.base + ((g0.d + dh) >> 1), o1 = g1.base + ((g1.d + dh) >> 1);
        const int lo0 = g0.t != kNoTask ? g0.d + dh - g0.n - o0 : (1 << 30);
        const int hi0 = g0.t != kNoTask ? g0.m - o0 : -(1 << 30);
        const int lo1 = g1.t != kNoTask ? g1.d + dh - g1.n - o1 : (1 << 30);
        const int hi1 = g1.t != kNoTask ? g1.m - o1 : -(1 << 30);
        const bool hi = lane_id() >= 32;
        lo_s = hi ? lo1 : lo0;
        hi_s = hi ? hi1 : hi0;
    }

    // Up to np pairs (odd, even anti-diagonal) from dh anti-diagonals after
    // the block start, ending after the first pair whose even step leaves a
    // live cell in an edge slot (then ub has 64 added).  Returns ub.
    template <bool BOUNDS>
    __device__ __forceinline__ uint32_t pairs(GroupX &g0, GroupX &g1, int dh, int np, int &ti, int &tp, int xv,
                                              uint32_t sinc0, uint32_t sinc1)
    {
        int lo_s = 0, hi_s = 0;
        if (BOUNDS) bounds_at(g0, g1, dh, lo_s, hi_s);
        const uint32_t ube = 2u * (uint32_t)np;
        uint32_t ub = 0;
        do {
            step<true, BOUNDS>(g0, g1, ub, ti, tp, xv, lo_s, hi_s, sinc0, sinc1);
            const uint64_t e = step<false, BOUNDS>(g0, g1, ub, ti, tp, xv, lo_s, hi_s - 1, sinc0, sinc1);
            if (BOUNDS) {
                ++lo_s;
                --hi_s;
            }
            ub = next_pair(ub, e);
        } while (ub < ube);
        return ub;
    }

    template <int K = 0>
    __device__ __forceinline__ uint64_t pairs_spec(GroupX &g0, GroupX &g1, int &ti, int &tp, int xv, uint32_t sinc0,
                                                   uint32_t sinc1, uint64_t acc)
    {
        if constexpr (K == UMAX) {
            return acc;
        } else {
            step<true, false, 2 * K>(g0, g1, 0u, ti, tp, xv, 0, 0, sinc0, sinc1);
            acc |= step<false, false, 2 * K>(g0, g1, 0u, ti, tp, xv, 0, 0, sinc0, sinc1);
            return pairs_spec<K + 1>(g0, g1, ti, tp, xv, sinc0, sinc1, acc);
        }
    }

    // one half of UMAX pairs at C = 1 without clipping: unrolled with no test
    // between the pairs, rolled back and rerun with per-pair checks if an
    // edge slot went live
    __device__ __forceinline__ uint32_t half_c1(GroupX &g0, GroupX &g1, int dh, int &ti, int &tp, int xv,
                                                uint32_t sinc0, uint32_t sinc1)
    {
        const int z1 = Z1[0], z2 = Z2[0], ti0 = ti, tp0 = tp;
        const uint32_t li0 = g0.li, li1 = g1.li;
        const int lu0 = g0.lu, lu1 = g1.lu;
        const uint64_t c0 = g0.cells, c1 = g1.cells, s0 = g0.slots, s1 = g1.slots;
        const uint64_t acc = pairs_spec(g0, g1, ti, tp, xv, sinc0, sinc1, 0ull);
        if (!(acc & EDGE)) return 2u * UMAX;
        Z1[0] = z1; Z2[0] = z2; ti = ti0; tp = tp0;
        g0.li = li0; g1.li = li1; g0.lu = lu0; g1.lu = lu1;
        g0.cells = c0; g1.cells = c1; g0.slots = s0; g1.slots = s1;
        return pairs<false>(g0, g1, dh, UMAX, ti, tp, xv, sinc0, sinc1);
    }

    // end cell of group g's last improvement in the half that began at its
    // anti-diagonal d0
    __device__ __forceinline__ void resolve(GroupX &g, int gi, int d0) const
    {
        if (g.lu < 0) return;
        const int dd = d0 + g.lu;
        const int l = __builtin_ctz(g.li);
        int slot = C * l;
        if (C > 1) slot += __builtin_amdgcn_readlane(rs, 32 * gi + l);
        g.bi = g.base + (dd >> 1) + slot;
        g.bj = dd - g.bi;
        g.lu = -1;
    }
};

// Queue of the narrow class, as seen by one wavefront.
struct NarrowQueue {
    uint32_t cnt;     // tasks in the queue
    bool drained;     // a fetch came back empty
};

// Ends group g's extension: result written, lanes dead, threshold reset
// (so that its drop threshold stays far above the dead value)
template <int C, bool COUNT>
__device__ __forceinline__ void narrow_end(const BatchDev &b, PairWin<C, COUNT> &w, GroupX &g, int gi, int &ti)
{
    const int T = __builtin_amdgcn_readlane(ti, 32 * gi) - g.d;
    TaskOut o;
    o.score = T; o.i = g.bi; o.j = g.bj; o.status = (uint32_t)kNarrowClass; o.cells = g.cells; o.slots = g.slots;
    b.tout[g.t] = o;
    g.t = kNoTask;
    w.set_group(gi, false);
    ti = ((lane_id() >> 5) == gi) ? 0 : ti;
}

// Starts task t in group g: fresh window lanes, threshold of anti-diagonal 1
template <int C, bool COUNT>
__device__ __forceinline__ void narrow_start(const BatchDev &b, const StoreDev &st, PairWin<C, COUNT> &w, GroupX &g,
                                             int gi, uint32_t t, int &ti)
{
    const Task k = load_task(b.recs, st.reads, t);
    g.t = t;
    g.d = 1;
    g.base = -(PairWin<C, COUNT>::WIN / 2 - 1);
    g.bi = 0; g.bj = 0;
    g.m = k.g.m; g.n = k.g.n; g.x = k.x;
    g.sx = k.mi + 2;
    g.abase = k.g.abase; g.bbase = k.g.bbase;
    g.cells = 0; g.slots = 0;
    g.li = 0; g.lu = -1;
    g.mn = g.mx = PairWin<C, COUNT>::WIN / 2 - 1;
    w.set_group(gi, true);
    ti = ((lane_id() >> 5) == gi) ? 1 : ti;   // T = 0, plus d = 1 (Z units, gap 1)
}

// Runs blocks until both groups are empty and the queue is drained (kDone),
// or until the window must change width (kGrow / kShrink, the window saved
// to LDS and each group's mn / mx set).  shrink_width < 0: never narrow.
template <int C, bool COUNT>
__device__ uint32_t narrow_run(const BatchDev &b, const StoreDev &st, PairWin<C, COUNT> &w, GroupX &g0, GroupX &g1,
                               int &ti, int *lds, NarrowQueue &q, int shrink_width)
{
    using PW = PairWin<C, COUNT>;
    constexpr int WIN = PW::WIN;
    const uint32_t *__restrict__ W = st.words;
    const uint32_t qcap = 2u * b.cap;
    const int lane = lane_id();
    const bool hi = lane >= 32;
    const int gl = lane & 31;
    for (;;) {
        w.bands(g0, g1);
        // extensions that ended: two dead anti-diagonals, or past the far corner
        if (g0.t != kNoTask && (g0.mx < 0 || g0.d > g0.m + g0.n)) narrow_end(b, w, g0, 0, ti);
        if (g1.t != kNoTask && (g1.mx < 0 || g1.d > g1.m + g1.n)) narrow_end(b, w, g1, 1, ti);
        // empty groups take the next tasks
        if (!q.drained && (g0.t == kNoTask || g1.t == kNoTask)) {
            const uint32_t k = (g0.t == kNoTask ? 1u : 0u) + (g1.t == kNoTask ? 1u : 0u);
            uint32_t idx = wave_fetch_add(&b.ctr[CtrLayout::kHead + kNarrowClass], k);
            if (g0.t == kNoTask) {
                if (idx < q.cnt) narrow_start(b, st, w, g0, 0, (uint32_t)uni((int)b.qbuf[kNarrowClass * qcap + idx]), ti);
                ++idx;
            }
            if (g1.t == kNoTask && idx < q.cnt)
                narrow_start(b, st, w, g1, 1, (uint32_t)uni((int)b.qbuf[kNarrowClass * qcap + idx]), ti);
            if (idx >= q.cnt) q.drained = true;
        }
        const bool e0 = g0.t == kNoTask, e1 = g1.t == kNoTask;
        if (e0 && e1) return kDone;
        const int w0 = e0 ? 0 : g0.mx - g0.mn + 1;
        const int w1 = e1 ? 0 : g1.mx - g1.mn + 1;
        if (w0 + 4 > WIN || w1 + 4 > WIN) {
            if (C == 1) {
                w.save(lds);
                return kGrow;
            }
            // wider than the widest window: the task restarts in the adaptive class
            for (int gi = 0; gi < 2; ++gi) {
                GroupX &g = gi ? g1 : g0;
                if ((gi ? w1 : w0) + 4 <= WIN) continue;
                const uint32_t pos = wave_fetch_add(&b.ctr[CtrLayout::kCount + kAdaptiveClass], 1u);
                b.qbuf[kAdaptiveClass * qcap + pos] = g.t;
                g.t = kNoTask;
                w.set_group(gi, false);
                ti = ((lane >> 5) == gi) ? 0 : ti;
            }
            continue;
        }
        if (w0 <= shrink_width && w1 <= shrink_width) {
            w.save(lds);
            return kShrink;
        }
        // re-centre a band that starts closer than kRecentre slots to an edge
        const int dl0 = (!e0 && min(g0.mn, WIN - 1 - g0.mx) < kRecentre) ? g0.mn - (WIN - w0) / 2 : 0;
        const int dl1 = (!e1 && min(g1.mn, WIN - 1 - g1.mx) < kRecentre) ? g1.mn - (WIN - w1) / 2 : 0;
        if (dl0 | dl1) {
            w.save(lds);
            w.load(lds, WIN, hi ? dl1 : dl0);
            g0.base += dl0;
            g1.base += dl1;
        }
        // pairs up to each group's far corner; the block runs the longer and
        // clips the other
        const int P0 = e0 ? 0 : min(PW::PB, (g0.m + g0.n - g0.d + 2) >> 1);
        const int P1 = e1 ? 0 : min(PW::PB, (g1.m + g1.n - g1.d + 2) >> 1);
        const int P = max(P0, P1);
        // no clipping when every slot that can hold a candidate (0 .. WIN-2)
        // of every anti-diagonal of the block lies inside the group's table
        auto clear_of_ends = [&](const GroupX &g, bool e) {
            if (e) return true;
            const int dlast = g.d + 2 * P - 1;
            const int o_last = g.base + (dlast >> 1);
            return o_last + WIN - 2 <= g.m && o_last >= dlast - g.n;
        };
        const bool fast = clear_of_ends(g0, e0) && clear_of_ends(g1, e1);
        // codes of this lane's group (an empty group reads the other's, which
        // keeps its loads inside the store; its cells are dead)
        const GroupX &ga = e0 ? g1 : g0;
        const GroupX &gb = e1 ? g0 : g1;
        const uint64_t abase = hi ? gb.abase : ga.abase, bbase = hi ? gb.bbase : ga.bbase;
        const int dsel = hi ? gb.d : ga.d, bsel = hi ? gb.base : ga.base;
        const int sx = hi ? gb.sx : ga.sx;
        const int xv = hi ? g1.x : g0.x;
        {
            const uint32_t *aseq = W + (abase >> 4), *bseq = W + (bbase >> 4);
            const int aph = (int)(abase & 15), bph = (int)(bbase & 15);
            const int e0d = (dsel - 1) >> 1;
            const int A0 = bsel + e0d - 1, B0 = e0d - bsel;
            uint32_t aw[PW::NWC], bw[PW::NWC];
            load_codes<PW::NWC>(aseq, aph, A0 + C * gl, aw);
            load_codes<PW::NWC>(bseq, bph, B0 - C * gl - (C - 1), bw);
            const uint32_t base_f = (uint32_t)kNarrowSm * 0x55555555u;
            const uint32_t kx = (uint32_t)(kNarrowSm ^ sx);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int r = 0; r < C; ++r) {
                    const uint32_t bb = codes16<PW::NWC>(bw, C - 1 - r + 16 * h);
                    const uint32_t xo = codes16<PW::NWC>(aw, r + 16 * h) ^ bb;
                    const uint32_t xe = codes16<PW::NWC>(aw, r + 1 + 16 * h) ^ bb;
                    const uint32_t mo = (xo | (xo >> 1)) & 0x55555555u;   // 1 = mismatch, at bit 2u
                    const uint32_t me = (xe | (xe >> 1)) & 0x55555555u;
                    // field u = sigma'' of pair u: sm ^ (mismatch ? sm ^ sx : 0)
                    const uint32_t fo = base_f ^ ((kx & 1u) ? mo : 0u) ^ ((kx & 2u) ? (mo << 1) : 0u);
                    const uint32_t fe = base_f ^ ((kx & 1u) ? me : 0u) ^ ((kx & 2u) ? (me << 1) : 0u);
                    if (h == 0) { w.mmo[r] = fo; w.mme[r] = fe; }
                    else { w.mmo2[r] = fo; w.mme2[r] = fe; }
                }
            }
        }
        // slot-steps charged to each group (an empty group's lanes to the other)
        const uint32_t sinc0 = e0 ? 0u : (e1 ? 2u * WIN : (uint32_t)WIN);
        const uint32_t sinc1 = e1 ? 0u : (e0 ? 2u * WIN : (uint32_t)WIN);
        int tp = ti - xv;
        const int p0 = min(P, UMAX);
        uint32_t ub;
        if (C == 1 && fast && p0 == UMAX)
            ub = w.half_c1(g0, g1, 0, ti, tp, xv, sinc0, sinc1);
        else if (fast)
            ub = w.template pairs<false>(g0, g1, 0, p0, ti, tp, xv, sinc0, sinc1);
        else
            ub = w.template pairs<true>(g0, g1, 0, p0, ti, tp, xv, sinc0, sinc1);
        int u = (int)(ub & 63u) >> 1;
        if (ub < 64u && P > UMAX && w.alive()) {
            w.resolve(g0, 0, g0.d);
            w.resolve(g1, 1, g1.d);
#pragma unroll
            for (int r = 0; r < C; ++r) {
                w.mmo[r] = w.mmo2[r];
                w.mme[r] = w.mme2[r];
            }
            if (C == 1 && fast && P == PW::PB)
                ub = w.half_c1(g0, g1, 2 * UMAX, ti, tp, xv, sinc0, sinc1);
            else if (fast)
                ub = w.template pairs<false>(g0, g1, 2 * UMAX, P - UMAX, ti, tp, xv, sinc0, sinc1);
            else
                ub = w.template pairs<true>(g0, g1, 2 * UMAX, P - UMAX, ti, tp, xv, sinc0, sinc1);
            u = UMAX + ((int)(ub & 63u) >> 1);
            w.resolve(g0, 0, g0.d + 2 * UMAX);
            w.resolve(g1, 1, g1.d + 2 * UMAX);
        } else {
            w.resolve(g0, 0, g0.d);
            w.resolve(g1, 1, g1.d);
        }
        if (!e0) g0.d += 2 * u;
        if (!e1) g1.d += 2 * u;
    }
}

// Class 0: narrow bands, two extensions per wavefront (weights match 1, gap
// -1, mismatch 0 / -1 / -2 and drops up to the narrow_x knob; the ingest
// kernel queues only those).  Each wavefront drains the queue two tasks at a
// time until it is empty; a band wider than 64 slots sends its task to the
// adaptive class.
template <bool COUNT>
__global__ void __launch_bounds__(256) narrow_kernel(BatchDev b, StoreDev st, int shrink_margin)
{
    __shared__ int lds_all[4][2 * PairWin<2, COUNT>::STRIDE];
    int *lds = lds_all[threadIdx.x >> 6];
    NarrowQueue q;
    q.cnt = b.ctr[CtrLayout::kCount + kNarrowClass];
    q.drained = false;
    GroupX g0{}, g1{};
    g0.t = g1.t = kNoTask;
    g0.lu = g1.lu = -1;
    int ti = 0;
    // back to 32 slots once every band fits them with shrink_margin to spare
    const int shrink2 = 32 - 2 * max(shrink_margin, 2);
    int C = 1, from_win = 0, dl = 0;
    bool fresh = true;
    for (;;) {
        uint32_t r;
        if (C == 1) {
            PairWin<1, COUNT> w;
            if (fresh) w.clear(); else w.load(lds, from_win, dl);
            r = narrow_run(b, st, w, g0, g1, ti, lds, q, -1);
        } else {
            PairWin<2, COUNT> w;
            w.load(lds, from_win, dl);
            r = narrow_run(b, st, w, g0, g1, ti, lds, q, shrink2);
        }
        if (r == kDone) break;
        fresh = false;
        const int nc = r == kGrow ? 2 : 1;
        from_win = 32 * C;
        int dl0 = 0, dl1 = 0;
        if (g0.t != kNoTask) {
            dl0 = g0.mn - (32 * nc - (g0.mx - g0.mn + 1)) / 2;
            g0.base += dl0;
        }
        if (g1.t != kNoTask) {
            dl1 = g1.mn - (32 * nc - (g1.mx - g1.mn + 1)) / 2;
            g1.base += dl1;
        }
        dl = lane_id() >= 32 ? dl1 : dl0;
        C = nc;
    }
}

// ---------------------------------------------------------------------------
// Hand-over between classes.  A wide window that overflows stores its state
// in the carry pool, and the next class resumes from it instead of
// recomputing the anti-diagonals done so far.
// ---------------------------------------------------------------------------

// `need` words of the carry pool (wave-uniform offset), or kNoCarry when full
__device__ __forceinline__ uint32_t carry_alloc(const BatchDev &b, uint32_t need)
{
    // a stale read of the counter only costs an add that then fails the bound
    if ((uint32_t)uni((int)b.ctr[CtrLayout::kCarry]) >= b.carry_words) return kNoCarry;
    const uint32_t off = wave_fetch_add(&b.ctr[CtrLayout::kCarry], need);
    return (uint64_t)off + need <= (uint64_t)b.carry_words ? off : kNoCarry;
}

// the window a wide run saved to LDS (anti-diagonal d-1 at lds[0, win), d-2
// at lds[stride, stride + win)) and its state, into the record at `off`
__device__ void carry_store(const BatchDev &b, uint32_t off, const XState &s, const int *lds, int win, int stride)
{
    int32_t *rec = b.carry + off;
    const int lane = lane_id();
    for (int k = lane; k < win; k += 64) {
        rec[CarryLayout::kHeader + k] = lds[k];
        rec[CarryLayout::kHeader + win + k] = lds[stride + k];
    }
    if (lane == 0) {
        rec[CarryLayout::kD] = s.d;
        rec[CarryLayout::kBase] = s.base;
        rec[CarryLayout::kT] = s.T;
        rec[CarryLayout::kBi] = s.bi;
        rec[CarryLayout::kBj] = s.bj;
        rec[CarryLayout::kMn] = s.mn;
        rec[CarryLayout::kMx] = s.mx;
        rec[CarryLayout::kWin] = win;
        rec[CarryLayout::kCells] = (int32_t)(uint32_t)s.cells;
        rec[CarryLayout::kCells + 1] = (int32_t)(uint32_t)(s.cells >> 32);
        rec[CarryLayout::kSlots] = (int32_t)(uint32_t)s.slots;
        rec[CarryLayout::kSlots + 1] = (int32_t)(uint32_t)(s.slots >> 32);
    }
}

// wave-uniform header word of a carried state
__device__ __forceinline__ int carry_word(const int32_t *rec, int k) { return uni(rec[k]); }

__device__ __forceinline__ void carry_state(const int32_t *rec, XState &s)
{
    s.d = carry_word(rec, CarryLayout::kD);
    s.base = carry_word(rec, CarryLayout::kBase);
    s.T = carry_word(rec, CarryLayout::kT);
    s.bi = carry_word(rec, CarryLayout::kBi);
    s.bj = carry_word(rec, CarryLayout::kBj);
    s.mn = carry_word(rec, CarryLayout::kMn);
    s.mx = carry_word(rec, CarryLayout::kMx);
    s.cells = (uint64_t)(uint32_t)carry_word(rec, CarryLayout::kCells) |
              ((uint64_t)(uint32_t)carry_word(rec, CarryLayout::kCells + 1) << 32);
    s.slots = (uint64_t)(uint32_t)carry_word(rec, CarryLayout::kSlots) |
              ((uint64_t)(uint32_t)carry_word(rec, CarryLayout::kSlots + 1) << 32);
}

// Task t moves from class cls to the next one's queue, with the carried
// state at `off` (kNoCarry: none, it restarts there from the seed).
template <bool COUNT>
__device__ void hand_over(const BatchDev &b, uint32_t t, int cls, const XState &s, uint32_t off)
{
    const uint32_t qcap = 2u * b.cap;
    const uint32_t pos = wave_fetch_add(&b.ctr[CtrLayout::kCount + cls + 1], 1u);
    b.qbuf[(cls + 1) * qcap + pos] = t;
    b.qstate[(cls + 1) * qcap + pos] = off;
    if (COUNT && off != kNoCarry && lane_id() == 0) {
        // the carried state keeps the task's running cell and slot-step
        // totals, which the class that completes it reports: credit this
        // class with what it computed so far and debit the next one the same
        // (modulo 2^64), so that each stage's sums hold only its own work
        const int stg = 1 + cls;
        atomicAdd(&b.stage_sum[stg], (unsigned long long)s.cells);
        atomicAdd(&b.stage_sum[stg + 1], 0ull - (unsigned long long)s.cells);
        atomicAdd(&b.stage_sum[16 + stg], (unsigned long long)s.slots);
        atomicAdd(&b.stage_sum[16 + stg + 1], 0ull - (unsigned long long)s.slots);
    }
}

// A task whose band outgrew class cls: its window (saved in LDS, win slots
// per anti-diagonal at the given stride) and state go to the carry pool when
// it has room, and the task to the next class.
template <bool COUNT>
__device__ void carry_out(const BatchDev &b, uint32_t t, int cls, const XState &s, const int *lds, int win,
                          int stride)
{
    const uint32_t off = carry_alloc(b, CarryLayout::kHeader + 2 * (uint32_t)win);
    if (off != kNoCarry) carry_store(b, off, s, lds, win, stride);
    hand_over<COUNT>(b, t, cls, s, off);
}

// Class 1: adaptive windows.  A task whose band outgrows 256 cells hands its
// window and state to the first wide class, which resumes it.  Registers
// capped for 6 wavefronts per SIMD (the compiler's own choice allows 5).
template <bool COUNT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) adaptive_kernel(BatchDev b, StoreDev st, int grow_margin, int shrink_margin)
{
    __shared__ int lds_all[4][2 * WMAX];
    int *lds = lds_all[threadIdx.x >> 6];
    const int cls = kAdaptiveClass;
    const uint32_t qcap = 2u * b.cap;
    const uint32_t cnt = b.ctr[CtrLayout::kCount + cls];
    for (;;) {
        const uint32_t idx = wave_fetch_add(&b.ctr[CtrLayout::kHead + cls], 1u);
        if (idx >= cnt) break;
        const uint32_t t = (uint32_t)uni((int)b.qbuf[cls * qcap + idx]);
        const Task k = load_task(b.recs, st.reads, t);
        XState s;
        bool ok;
        int win = 0;
        if (k.ma != 1)
            ok = run_adaptive<COUNT, false, false>(st.words, k, lds, s, grow_margin, shrink_margin, win);
        else if (sigma_fits_2bits(k))
            ok = run_adaptive<COUNT, true, true>(st.words, k, lds, s, grow_margin, shrink_margin, win);
        else
            ok = run_adaptive<COUNT, true, false>(st.words, k, lds, s, grow_margin, shrink_margin, win);
        if (ok) {
            TaskOut o;   // every lane stores the same (wave-uniform) values
            o.score = s.T; o.i = s.bi; o.j = s.bj; o.status = (uint32_t)cls; o.cells = s.cells; o.slots = s.slots;
            b.tout[t] = o;
        } else {
            carry_out<COUNT>(b, t, cls, s, lds, win, WMAX);
        }
    }
}

// Window widths (cells per lane) of the two wide classes.  Each class widens
// and narrows its window along its ladder as the band changes, handing the
// band over through LDS as the adaptive kernel does; its widest window is
// the class limit (kWideC).
template <int L> struct WideLadder;
template <> struct WideLadder<0> {
    static constexpr int N = 5;   // C = 8, 10, 12, 16, 20: 512..1280 slots
    static constexpr __host__ __device__ int c(int ci) { return ci < 3 ? 8 + 2 * ci : 16 + 4 * (ci - 3); }
};
template <> struct WideLadder<1> {
    static constexpr int N = 2;   // C = 24, 32: 1536, 2048 slots
    static constexpr __host__ __device__ int c(int ci) { return ci == 0 ? 24 : 32; }
};
static_assert(WideLadder<0>::c(WideLadder<0>::N - 1) == kWideC[0] &&
              WideLadder<1>::c(WideLadder<1>::N - 1) == kWideC[1], "class limits");
constexpr int kWideGrowMargin = 32;     // free slots per side after widening
constexpr int kWideShrinkMargin = 64;   // narrow once the band fits the next smaller window with this slack

template <int L>
__device__ __forceinline__ int ladder_c(int ci)
{
    return WideLadder<L>::c(ci);
}

// smallest rung whose window holds `width` slots with `margin` free on each side; -1 if none
template <int L>
__device__ __forceinline__ int ladder_fit(int width, int margin)
{
    for (int ci = 0; ci < WideLadder<L>::N; ++ci)
        if (width + 2 * margin <= 64 * ladder_c<L>(ci)) return ci;
    return -1;
}

// The run of rung ci of class L's ladder (rungs I and up; a chain of tests
// that the compiler unrolls): a fresh window (only at rung 0) or one loaded
// from the window saved in LDS.
template <int L, int I, bool COUNT, bool MA1, bool SIGF>
__device__ __forceinline__ uint32_t run_rung(int ci, bool fresh, const StoreDev &st, const Task &k, int *lds,
                                             XState &s, int from_win, int delta, int shrink_width)
{
    if constexpr (I >= WideLadder<L>::N) {
        return kDone;   // not reached: ci < N
    } else {
        if (ci == I) {
            Window<WideLadder<L>::c(I), COUNT, MA1, SIGF, 64 * kWideC[L]> w;
            if (I == 0 && fresh) w.init(s); else w.load(lds, from_win, delta);
            return w.run(st.words, k.g, k.x, k.ma, k.mi, k.gap, lds, s, shrink_width);
        }
        return run_rung<L, I + 1, COUNT, MA1, SIGF>(ci, fresh, st, k, lds, s, from_win, delta, shrink_width);
    }
}

// One extension in wide class L: fresh, or resumed from the state a
// narrower class carried over (its band re-centred in the rung that fits).
// When the band outgrows the widest rung the state goes to the carry pool;
// returns kDone or kGrow and sets `out_off` to the record (kNoCarry: none,
// the task restarts in the next class).
template <int L, bool COUNT, bool MA1, bool SIGF>
__device__ uint32_t run_ladder(const BatchDev &b, const StoreDev &st, const Task &k, int *lds, XState &s,
                               uint32_t coff, uint32_t &out_off)
{
    using LD = WideLadder<L>;
    constexpr int STRIDE = 64 * kWideC[L];
    out_off = kNoCarry;
    int ci = 0, from_win = 0, delta = 0;
    bool fresh = true;
    // a carried window is narrower than the widest rung, so some rung holds it
    if (coff != kNoCarry) {
        const int32_t *rec = b.carry + coff;
        carry_state(rec, s);
        from_win = carry_word(rec, CarryLayout::kWin);   // a narrower class's window: fits this stride
        for (int q = lane_id(); q < from_win; q += 64) {
            lds[q] = rec[CarryLayout::kHeader + q];
            lds[STRIDE + q] = rec[CarryLayout::kHeader + from_win + q];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int width = s.mx - s.mn + 1;
        ci = ladder_fit<L>(width, kWideGrowMargin);
        if (ci < 0) ci = LD::N - 1;   // width <= from_win < the widest rung - 4
        delta = s.mn - (64 * ladder_c<L>(ci) - width) / 2;
        s.base += delta;
        fresh = false;
    }
    for (;;) {
        const int shrink_width = ci > 0 ? 64 * ladder_c<L>(ci - 1) - 2 * kWideShrinkMargin : -1;
        const uint32_t stt = run_rung<L, 0, COUNT, MA1, SIGF>(ci, fresh, st, k, lds, s, from_win, delta, shrink_width);
        if (stt == kDone) return kDone;
        fresh = false;
        const int width = s.mx - s.mn + 1;
        const int cur = 64 * ladder_c<L>(ci);
        int nci = ci - 1;   // kShrink
        if (stt == kGrow) {
            // width + 4 > cur, so any fitting rung is wider than this one
            nci = ladder_fit<L>(width, kWideGrowMargin);
            if (nci < 0) nci = ladder_fit<L>(width, 2);
            if (nci < 0) {
                // the window (saved in LDS by run) goes to the next class
                out_off = carry_alloc(b, CarryLayout::kHeader + 2 * cur);
                if (out_off != kNoCarry) carry_store(b, out_off, s, lds, cur, STRIDE);
                return kGrow;
            }
        }
        from_win = cur;
        delta = s.mn - (64 * ladder_c<L>(nci) - width) / 2;
        s.base += delta;
        ci = nci;
    }
}

// Wide class L for bands the adaptive kernel cannot hold.  The first class
// (up to 1280 slots) runs 2 wavefronts per SIMD (256 VGPRs, a few spills at
// task entry); the second, in this one-wavefront form (up to 2048 slots),
// needs the whole register file and runs 1 per SIMD, so bands up to 1276
// cells stay in the first.
template <int L, bool COUNT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(L == 0 ? 2 : 1)))
wide_kernel(BatchDev b, StoreDev st, int cls)
{
    constexpr int STRIDE = 64 * kWideC[L];
    extern __shared__ int lds_wide[];
    int *lds = lds_wide + (threadIdx.x >> 6) * (2 * STRIDE);
    const uint32_t qcap = 2u * b.cap;
    const uint32_t cnt = b.ctr[CtrLayout::kCount + cls];
    for (;;) {
        const uint32_t idx = wave_fetch_add(&b.ctr[CtrLayout::kHead + cls], 1u);
        if (idx >= cnt) break;
        const uint32_t t = (uint32_t)uni((int)b.qbuf[cls * qcap + idx]);
        const uint32_t coff = (uint32_t)uni((int)b.qstate[cls * qcap + idx]);
        const Task k = load_task(b.recs, st.reads, t);
        XState s;
        uint32_t status, out_off;
        if (k.ma != 1)
            status = run_ladder<L, COUNT, false, false>(b, st, k, lds, s, coff, out_off);
        else if (sigma_fits_2bits(k))
            status = run_ladder<L, COUNT, true, true>(b, st, k, lds, s, coff, out_off);
        else
            status = run_ladder<L, COUNT, true, false>(b, st, k, lds, s, coff, out_off);
        if (status == kDone) {
            TaskOut o;
            o.score = s.T; o.i = s.bi; o.j = s.bj; o.status = (uint32_t)cls; o.cells = s.cells; o.slots = s.slots;
            b.tout[t] = o;
        } else {
            hand_over<COUNT>(b, t, cls, s, out_off);
        }
    }
}

// ---------------------------------------------------------------------------
// Second wide class with several wavefronts per extension (tuning knob
// wide_waves = W of 2 or 4; 1 runs wide_kernel<1> above).  The class's
// 2048-slot window is split into W segments of 64*C slots, one per
// wavefront of a workgroup: global slot S = 64*C*w + C*lane + r, cell
// i = o_d + S as in Window.  Every anti-diagonal ends with an exchange
// through LDS and one barrier: each wavefront publishes whether one of its
// cells beat the improvement threshold, the edge cell its neighbour reads as
// a gap predecessor on the next anti-diagonal (the rotate brings it in from
// the wrong wavefront), and, on even anti-diagonals, whether a window edge
// slot went live.  With match 1 an improving cell holds exactly T + 1, so
// the flags decide the threshold; other weights take a second exchange of
// the wavefronts' largest values on improving anti-diagonals.  Block control
// (band, re-centring, end cell, two dead anti-diagonals, hand-over) uses
// group-wide reductions, so every wavefront takes every branch and every
// barrier together.  The window moves between two widths (group_run); a band
// that outgrows the wider one goes to the unbounded kernel with its state.
// ---------------------------------------------------------------------------
constexpr int kGroupWin = 64 * kWideC[1];   // slots of the window (the class limit)

template <int W, int WSLOTS>
struct GroupShared {
    int win[2 * WSLOTS];      // anti-diagonals d-1, d-2 of the window (re-centring, resume, hand-over)
    int xch[2][W][2];         // per parity of d and wavefront: flags, edge cell
    int vmx[W];               // largest values on an improving anti-diagonal (weights other than match 1)
    int red[W][4];            // block-level reductions
    uint32_t task;            // queue index taken by wavefront 0
};

template <int C, int W, bool COUNT, bool MA1, bool SIGF, int WSLOTS = W * 64 * C>
struct GroupWindow {
    static constexpr int SEG = 64 * C;   // slots per wavefront
    static constexpr int WIN = W * SEG;
    static constexpr int STRIDE = WSLOTS;   // shared LDS copy: sized for the widest window of the class
    static constexpr int NWC = (C + UMAX + 16) / 16;   // words of codes per lane and block
    static_assert(WIN <= WSLOTS && WSLOTS <= 4096, "a lane's code window stays within the store's guard");
    using Shared = GroupShared<W, WSLOTS>;

    int Z1[C], Z2[C];
    uint32_t mmo[C], mme[C];
    int wv;                  // this wavefront's segment (wave-uniform)
    int s0;                  // its first slot, SEG * wv
    int nb;                  // neighbour's edge cell for the next anti-diagonal (same in every lane)
    // end cell: last anti-diagonal with an improving cell in this segment
    // since the last resolve(); MA1: its improvement mask over lanes and,
    // per lane, the first improving r; other weights: the cell's slot
    int last_d, last_r, last_s;
    uint64_t last_imp;
    Shared *sh;

    // group-wide reduction of up to four values per wavefront: every
    // wavefront sees all of them (q = 0 .. W-1) after the call
    __device__ __forceinline__ void publish(int a, int b2 = 0, int c = 0, int e = 0)
    {
        if (lane_id() == 0) {
            sh->red[wv][0] = a; sh->red[wv][1] = b2; sh->red[wv][2] = c; sh->red[wv][3] = e;
        }
        __syncthreads();
    }
    __device__ __forceinline__ int got(int q, int k) const { return uni(sh->red[q][k]); }
    __device__ __forceinline__ void done_reading() const { __syncthreads(); }

    __device__ __forceinline__ void init(XState &s)
    {
        const int lane = lane_id();
        const int c0 = WIN / 2 - 1;
        s.base = -c0;
        s.d = 1;
        s.T = 0; s.bi = 0; s.bj = 0; s.cells = 0; s.slots = 0;
        s.mn = s.mx = c0;
#pragma unroll
        for (int r = 0; r < C; ++r) {
            Z1[r] = (s0 + C * lane + r == c0) ? 0 : NEG;
            Z2[r] = NEG;
        }
    }

    // segment -> the shared window buffer, by global slot
    __device__ __forceinline__ void save()
    {
        const int lane = lane_id();
#pragma unroll
        for (int r = 0; r < C; ++r) {
            sh->win[s0 + C * lane + r] = Z1[r];
            sh->win[STRIDE + s0 + C * lane + r] = Z2[r];
        }
        __syncthreads();
    }

    // take over a window of from_win slots in the shared buffer: new slot S
    // holds old slot S + delta
    __device__ __forceinline__ void load(int from_win, int delta)
    {
        const int lane = lane_id();
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const int q = s0 + C * lane + r + delta;
            const bool ok = q >= 0 && q < from_win;
            const int qc = ok ? q : 0;
            const int a = sh->win[qc], b2 = sh->win[STRIDE + qc];
            Z1[r] = ok ? a : NEG;
            Z2[r] = ok ? b2 : NEG;
        }
        __syncthreads();   // read by every wavefront before the buffer is written again
    }

    // live slots over the last two anti-diagonals, group-wide; false when both are dead
    __device__ bool band(int &mn, int &mx)
    {
        int lmn = 1 << 30, lmx = -1;
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const uint64_t u = ballot(max(Z1[r], Z2[r]) > NEG_HALF);
            if (u) {
                lmn = min(lmn, s0 + C * __builtin_ctzll(u) + r);
                lmx = max(lmx, s0 + C * (63 - __builtin_clzll(u)) + r);
            }
        }
        publish(lmn, lmx);
        mn = 1 << 30;
        mx = -1;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            mn = min(mn, got(q, 0));
            mx = max(mx, got(q, 1));
        }
        done_reading();
        return mx >= 0;
    }

    // before the first (odd) anti-diagonal of a block: lane 0 of each
    // segment needs the last slot of the previous segment's d-1
    __device__ __forceinline__ void prime()
    {
        publish(__builtin_amdgcn_readlane(Z1[C - 1], 63));
        nb = wv > 0 ? got(wv - 1, 0) : NEG;
        done_reading();
    }

    // One anti-diagonal d.  Returns whether a window edge slot (0, 1, WIN-2,
    // WIN-1) holds a live cell of d (even d; false for odd d).
    template <bool ODD, bool BOUNDS>
    __device__ __forceinline__ bool step(XState &s, int d, uint32_t ub, int &tp, int &ti, int sm, int nd, int G,
                                         int X, int lo_s = 0, int hi_s = 0)
    {
        const int lane = lane_id();
        int t[C];
        if (ODD) {
            // slots S-1 and S: lane 0 takes the previous segment's last slot
            int x = __builtin_amdgcn_mov_dpp(Z1[C - 1], 0x13C, 0xf, 0xf, true);   // wave_ror:1
            x = lane == 0 ? nb : x;
            t[0] = max(x, Z1[0]);
#pragma unroll
            for (int r = 1; r < C; ++r) t[r] = max(Z1[r - 1], Z1[r]);
        } else {
            // slots S and S+1: lane 63 takes the next segment's first slot
#pragma unroll
            for (int r = 0; r < C - 1; ++r) t[r] = max(Z1[r], Z1[r + 1]);
            int x = __builtin_amdgcn_mov_dpp(Z1[0], 0x134, 0xf, 0xf, true);       // wave_rol:1
            x = lane == 63 ? nb : x;
            t[C - 1] = max(x, Z1[C - 1]);
        }
        int v[C];
        int vm = NEG;
        uint64_t le = 0, re = 0;   // live masks of the window's edge slots (even d)
        if (COUNT) s.slots += (uint64_t)SEG;
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const uint32_t w = ODD ? mmo[r] : mme[r];
            int sig;
            if (SIGF) {
                sig = (int)__builtin_amdgcn_ubfe(w, ub, 2u);
            } else {
                const int bit = (int)__builtin_amdgcn_ubfe(w, ub, 1u);
                sig = __mul24(bit, nd) + sm;          // sigma - 2*gap
            }
            v[r] = max(t[r], Z2[r] + sig);
            const int sl = s0 + C * lane + r;
            const bool inb = !BOUNDS || (sl >= lo_s && sl <= hi_s);
            vm = max(vm, inb ? v[r] : NEG);
            if (COUNT) s.cells += (uint64_t)__builtin_popcountll(ballot(inb && v[r] > NEG_HALF));
            const bool keep = inb && v[r] >= tp;
            if (!ODD && (r == 0 || r == 1)) le |= ballot(keep);
            if (!ODD && (r == C - 2 || r == C - 1)) re |= ballot(keep);
            t[r] = keep ? v[r] : NEG;
        }
        const uint64_t imp = ballot(vm > ti);
        int fl = imp ? 1 : 0;
        if (!ODD && ((wv == 0 && (le & 1ull)) || (wv == W - 1 && (re >> 63)))) fl |= 2;
        // the edge cell the neighbour needs next: after an odd d the first
        // slot (for the previous segment), after an even d the last slot
        const int edge = ODD ? __builtin_amdgcn_readlane(t[0], 0) : __builtin_amdgcn_readlane(t[C - 1], 63);
        int *x = sh->xch[ODD ? 1 : 0][wv];
        if (lane == 0) {
            x[0] = fl;
            x[1] = edge;
        }
        __syncthreads();
        // lane q reads wavefront q's flags
        const int fq = sh->xch[ODD ? 1 : 0][lane < W ? lane : 0][0];
        const int f = (ballot(lane < W && (fq & 1)) ? 1 : 0) | (ballot(lane < W && (fq & 2)) ? 2 : 0);
        if (ODD) nb = wv < W - 1 ? uni(sh->xch[1][wv + 1][1]) : NEG;
        else nb = wv > 0 ? uni(sh->xch[0][wv - 1][1]) : NEG;
        if (MA1) {
            if (imp) {
                // first improving slot of this segment: smallest lane, then smallest r
                last_d = d;
                last_imp = imp;
                int rl = C - 1;
#pragma unroll
                for (int r = C - 1; r >= 0; --r) {
                    const int sl = s0 + C * lane + r;
                    const bool inb = !BOUNDS || (sl >= lo_s && sl <= hi_s);
                    if (inb && v[r] > ti) rl = r;
                }
                last_r = rl;
            }
            const int inc = f & 1;
            tp += G + inc;
            ti += G + inc;
        } else {
            if (f & 1) {
                // the group's largest value of d is the new threshold
                const int wmax = uni(wave_max(vm));
                if (lane == 0) sh->vmx[wv] = wmax;
                __syncthreads();
                int gmax = NEG;
#pragma unroll
                for (int q = 0; q < W; ++q) gmax = max(gmax, uni(sh->vmx[q]));
                if (wmax == gmax) {
                    // first slot of this segment holding it
                    int rl = C;
#pragma unroll
                    for (int r = C - 1; r >= 0; --r) {
                        const int sl = s0 + C * lane + r;
                        const bool inb = !BOUNDS || (sl >= lo_s && sl <= hi_s);
                        if (inb && v[r] == gmax) rl = r;
                    }
                    const uint64_t any = ballot(rl < C);
                    const int l = __builtin_ctzll(any);
                    last_d = d;
                    last_s = s0 + C * l + __builtin_amdgcn_readlane(rl, l);
                }
                tp += gmax - ti;
                ti = gmax;
            }
            tp += G;
            ti += G;
        }
#pragma unroll
        for (int r = 0; r < C; ++r) {
            Z2[r] = Z1[r];
            Z1[r] = t[r];
        }
        return (f & 2) != 0;
    }

    // end cell of the last improvement since the previous call: the last
    // anti-diagonal any segment improved on, then its smallest slot
    __device__ void resolve(XState &s)
    {
        int ld = -1, ls = 0;
        if (last_d >= 0) {
            ld = last_d;
            if (MA1) {
                const int l = __builtin_ctzll(last_imp);
                ls = s0 + C * l + __builtin_amdgcn_readlane(last_r, l);
            } else {
                ls = last_s;
            }
        }
        publish(ld, ls);
        int gd = -1, gs = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int qd = got(q, 0), qs = got(q, 1);
            if (qd > gd) { gd = qd; gs = qs; }   // segments in slot order: the first wins a tie
        }
        done_reading();
        if (gd >= 0) {
            s.bi = s.base + (gd >> 1) + gs;
            s.bj = gd - s.bi;
        }
        last_d = -1;
    }

    template <bool BOUNDS>
    __device__ __forceinline__ uint32_t pairs(XState &s, int d0, int np, int &tp, int &ti, int sm, int nd, int G,
                                              int X, int m, int n)
    {
        // clipping bounds in global slots, as in Window::pairs
        const int o0 = s.base + (d0 >> 1);
        int lo_s = d0 - n - o0, hi_s = m - o0;
        const uint32_t ube = 2u * (uint32_t)np;
        uint32_t ub = 0;
        do {
            step<true, BOUNDS>(s, d0 + (int)ub, ub, tp, ti, sm, nd, G, X, lo_s, hi_s);
            const bool e = step<false, BOUNDS>(s, d0 + (int)ub + 1, ub, tp, ti, sm, nd, G, X, lo_s, hi_s - 1);
            ++lo_s;
            --hi_s;
            ub += e ? 66u : 2u;   // a live edge slot ends the block (2 * UMAX < 64)
        } while (ub < ube);
        return ub;
    }

    // Advance the extension block by block (Window::run with group-wide
    // control).  Returns kDone, or kGrow with the window saved to the shared
    // buffer and s.mn / s.mx set.
    __device__ uint32_t run(const uint32_t *__restrict__ Wd, const Geo &g, int X, int ma, int mi, int gap,
                            XState &s, int shrink_width = -1)
    {
        const int lane = lane_id();
        const int m = g.m, n = g.n;
        const int G = -gap;
        const int sm = ma + 2 * G;
        const int sx = mi + 2 * G;
        const int nd = mi - ma;
        const int dend = m + n;
        const uint32_t *aseq = Wd + (g.abase >> 4), *bseq = Wd + (g.bbase >> 4);
        const int aph = (int)(g.abase & 15), bph = (int)(g.bbase & 15);
        last_d = -1;
        int ti = s.T + G * s.d;
        while (s.d <= dend) {
            int mn, mx;
            if (!band(mn, mx)) break;                 // two dead anti-diagonals
            const int width = mx - mn + 1;
            if (width + 4 > WIN || width <= shrink_width) {
                save();
                s.mn = mn;
                s.mx = mx;
                s.T = ti - G * s.d;
                return width + 4 > WIN ? kGrow : kShrink;
            }
            if (min(mn, WIN - 1 - mx) < kRecentre) {
                const int delta = mn - (WIN - width) / 2;
                save();
                load(WIN, delta);
                s.base += delta;
            }
            const int d = s.d;
            const int P = min(UMAX, (dend - d + 2) >> 1);
            const int e0 = (d - 1) >> 1;
            const int A0 = s.base + e0 - 1;
            const int B0 = e0 - s.base;
            uint32_t aw[NWC], bw[NWC];
            load_codes<NWC>(aseq, aph, A0 + s0 + C * lane, aw);
            load_codes<NWC>(bseq, bph, B0 - s0 - C * lane - (C - 1), bw);
#pragma unroll
            for (int r = 0; r < C; ++r) {
                const uint32_t bb = codes16<NWC>(bw, C - 1 - r);
                const uint32_t xo = codes16<NWC>(aw, r) ^ bb;
                const uint32_t xe = codes16<NWC>(aw, r + 1) ^ bb;
                const uint32_t mo = (xo | (xo >> 1)) & 0x55555555u;
                const uint32_t me = (xe | (xe >> 1)) & 0x55555555u;
                uint32_t fo = mo, fe = me;
                if (SIGF) {
                    const uint32_t base_f = (uint32_t)sm * 0x55555555u;
                    const uint32_t k = (uint32_t)(sm ^ sx);
                    fo = base_f ^ ((k & 1u) ? mo : 0u) ^ ((k & 2u) ? (mo << 1) : 0u);
                    fe = base_f ^ ((k & 1u) ? me : 0u) ^ ((k & 2u) ? (me << 1) : 0u);
                }
                mmo[r] = fo;
                mme[r] = fe;
            }
            int tp = ti - X;
            const int dlast = d + 2 * P - 1;
            const int o_last = s.base + (dlast >> 1);
            const bool fast = o_last + WIN - 2 <= m && o_last >= dlast - n;
            prime();
            const uint32_t ub = fast ? pairs<false>(s, d, P, tp, ti, sm, nd, G, X, m, n)
                                     : pairs<true>(s, d, P, tp, ti, sm, nd, G, X, m, n);
            resolve(s);
            s.d = d + 2 * ((int)(ub & 63u) >> 1);
        }
        s.T = ti - G * s.d;
        return kDone;
    }
};

// One extension in a window shared by a workgroup: fresh, or resumed from
// the state a narrower class carried over.  The window moves between two
// widths, W x 64 x CLO and W x 64 x CHI slots, through the shared LDS copy
// (CLO == CHI: one width): it widens when the band outgrows the narrower one
// and narrows once the band fits it with 64 slots to spare per side.  Cell
// and slot-step counts are summed over the wavefronts into every
// wavefront's state.
template <int CLO, int CHI, int W, bool COUNT, bool MA1, bool SIGF>
__device__ uint32_t group_run(const BatchDev &b, const StoreDev &st, const Task &k,
                              GroupShared<W, W * 64 * CHI> &sh, int wv, XState &s, uint32_t coff)
{
    constexpr int WHI = W * 64 * CHI, WLO = W * 64 * CLO;
    using Lo = GroupWindow<CLO, W, COUNT, MA1, SIGF, WHI>;
    using Hi = GroupWindow<CHI, W, COUNT, MA1, SIGF, WHI>;
    bool hi = CLO == CHI, fresh = true;
    int from_win = 0, delta = 0;
    if (coff != kNoCarry) {
        const int32_t *rec = b.carry + coff;
        carry_state(rec, s);
        from_win = carry_word(rec, CarryLayout::kWin);   // a narrower class's window
        for (int q = (int)threadIdx.x; q < from_win; q += 64 * W) {
            sh.win[q] = rec[CarryLayout::kHeader + q];
            sh.win[WHI + q] = rec[CarryLayout::kHeader + from_win + q];
        }
        __syncthreads();
        const int width = s.mx - s.mn + 1;
        hi = hi || width + 2 * kWideGrowMargin > WLO;
        delta = s.mn - ((hi ? WHI : WLO) - width) / 2;
        s.base += delta;
        fresh = false;
        if (COUNT && wv != 0) { s.cells = 0; s.slots = 0; }   // wavefront 0 holds the carried totals
    }
    uint32_t stt;
    for (;;) {
        if (hi) {
            Hi w;
            w.sh = &sh; w.wv = wv; w.s0 = w.SEG * wv;
            if (fresh) w.init(s); else w.load(from_win, delta);
            stt = w.run(st.words, k.g, k.x, k.ma, k.mi, k.gap, s, CLO == CHI ? -1 : WLO - 2 * kWideShrinkMargin);
        } else {
            Lo w;
            w.sh = &sh; w.wv = wv; w.s0 = w.SEG * wv;
            if (fresh) w.init(s); else w.load(from_win, delta);
            stt = w.run(st.words, k.g, k.x, k.ma, k.mi, k.gap, s);
        }
        if (stt == kDone || (stt == kGrow && hi)) break;   // done, or out of the class (window saved)
        // the other width: the band was saved to the shared copy by run()
        fresh = false;
        const int width = s.mx - s.mn + 1;
        from_win = hi ? WHI : WLO;
        hi = stt == kGrow;
        delta = s.mn - ((hi ? WHI : WLO) - width) / 2;
        s.base += delta;
    }
    if (COUNT) {
        Hi w;
        w.sh = &sh; w.wv = wv;
        w.publish((int)(uint32_t)s.cells, (int)(uint32_t)(s.cells >> 32), (int)(uint32_t)s.slots,
                  (int)(uint32_t)(s.slots >> 32));
        uint64_t c = 0, sl = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            c += (uint64_t)(uint32_t)w.got(q, 0) | ((uint64_t)(uint32_t)w.got(q, 1) << 32);
            sl += (uint64_t)(uint32_t)w.got(q, 2) | ((uint64_t)(uint32_t)w.got(q, 3) << 32);
        }
        w.done_reading();
        s.cells = c;
        s.slots = sl;
    }
    return stt;
}

// The second wide class with W wavefronts per extension, one workgroup per
// extension; wavefront 0 takes the tasks and writes results and hand-overs.
template <int CLO, int CHI, int W, bool COUNT>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(W == 2 ? 3 : 4)))
group_kernel(BatchDev b, StoreDev st, int cls)
{
    __shared__ GroupShared<W, kGroupWin> sh;
    static_assert(64 * CHI * W == kGroupWin, "the widest window is the class limit");
    const int wv = uni((int)(threadIdx.x >> 6));
    const uint32_t qcap = 2u * b.cap;
    const uint32_t cnt = b.ctr[CtrLayout::kCount + cls];
    for (;;) {
        if (wv == 0) {
            const uint32_t idx = wave_fetch_add(&b.ctr[CtrLayout::kHead + cls], 1u);
            if (lane_id() == 0) sh.task = idx;
        }
        __syncthreads();
        const uint32_t idx = (uint32_t)uni((int)sh.task);
        __syncthreads();         // read by every wavefront before wavefront 0 writes it again
        if (idx >= cnt) break;   // uniform over the workgroup
        const uint32_t t = (uint32_t)uni((int)b.qbuf[cls * qcap + idx]);
        const uint32_t coff = (uint32_t)uni((int)b.qstate[cls * qcap + idx]);
        const Task k = load_task(b.recs, st.reads, t);
        XState s;
        uint32_t status;
        if (k.ma != 1)
            status = group_run<CLO, CHI, W, COUNT, false, false>(b, st, k, sh, wv, s, coff);
        else if (sigma_fits_2bits(k))
            status = group_run<CLO, CHI, W, COUNT, true, true>(b, st, k, sh, wv, s, coff);
        else
            status = group_run<CLO, CHI, W, COUNT, true, false>(b, st, k, sh, wv, s, coff);
        if (wv == 0) {
            if (status == kDone) {
                TaskOut o;
                o.score = s.T; o.i = s.bi; o.j = s.bj; o.status = (uint32_t)cls; o.cells = s.cells; o.slots = s.slots;
                b.tout[t] = o;
            } else {
                // the window (saved by run) goes to the unbounded kernel
                carry_out<COUNT>(b, t, cls, s, sh.win, kGroupWin, kGroupWin);
            }
        }
        __syncthreads();   // the shared window is read by wavefront 0 before the next task writes it
    }
}

// ---------------------------------------------------------------------------
// Unbounded X-drop extension.  One workgroup of 1024 threads runs one
// extension: its threads sweep the candidate range of an anti-diagonal
// together, and one block reduction per anti-diagonal gives the live range,
// the best value (smallest i on ties) and the cell count.  The last three
// anti-diagonals sit in an LDS ring indexed by i mod kRing while every
// candidate range fits it, then in global memory indexed by i.  Used only
// for bands wider than the widest register window.
// ---------------------------------------------------------------------------
constexpr int kGenericWaves = kGenericBlockWaves;
constexpr int kGenericThreads = 64 * kGenericWaves;
constexpr int kRing = 8192;   // LDS ring slots per anti-diagonal (power of two)

struct GState {
    int d;                 // next anti-diagonal
    int lo1, hi1;          // live range of d-1 (lo > hi: none)
    int lo2, hi2;          // live range of d-2
    int T, bi, bj;         // best so far and its cell
    uint64_t cells, slots;
    bool prev_dead;        // d-1 had no live cell
};

// per-wavefront partial of one anti-diagonal
struct GPart {
    int lo, hi, v, i;
    uint32_t cells, pad[3];
};

// the identity of each operation is passed as the DPP "old" value, so that
// lanes without a source keep their value and mov_dpp + op fuse into one
// DPP-modified instruction
struct OpMin {
    static constexpr int kIdent = 0x7fffffff;
    __device__ int operator()(int a, int b) const { return min(a, b); }
};
struct OpMax {
    static constexpr int kIdent = -0x7fffffff - 1;
    __device__ int operator()(int a, int b) const { return max(a, b); }
};
struct OpAdd {
    static constexpr int kIdent = 0;
    __device__ int operator()(int a, int b) const { return a + b; }
};

// Whole-wavefront reduction with DPP (quad permutes, row mirrors, then the
// row broadcasts of lanes 15 and 31); the result is read from lane 63.
template <typename Op>
__device__ __forceinline__ int wave_reduce(int v, Op op)
{
    constexpr int ident = Op::kIdent;
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0xB1, 0xf, 0xf, false));    // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x4E, 0xf, 0xf, false));    // quad_perm [2,3,0,1]
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x141, 0xf, 0xf, false));   // row_half_mirror
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x140, 0xf, 0xf, false));   // row_mirror
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x142, 0xa, 0xf, false));   // row_bcast:15 -> rows 1, 3
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x143, 0xc, 0xf, false));   // row_bcast:31 -> rows 2, 3
    return __builtin_amdgcn_readlane(v, 63);
}

// The same over each row of 16 lanes (every lane of a row ends with its row's
// result), read from lane 0.
template <typename Op>
__device__ __forceinline__ int row_reduce(int v, Op op)
{
    constexpr int ident = Op::kIdent;
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0xB1, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x4E, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x141, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x140, 0xf, 0xf, false));
    return __builtin_amdgcn_readfirstlane(v);
}

// Anti-diagonals s.d, s.d+1, ... with the previous two in P1 and P2 (RING:
// LDS slots i mod kRing; else global arrays indexed by i).  Returns true when
// the extension has ended; false (RING only) before an anti-diagonal whose
// candidate range does not fit the ring, with the state of the last one done
// and P1 / P2 pointing at the arrays of s.d-1 / s.d-2.
template <bool COUNT, bool RING>
__device__ bool generic_diags(const uint32_t *__restrict__ W, const Geo &g, int X, int ma, int mi, int gap,
                              int *&P2, int *&P1, int *&P0, GState &s, GPart (*part)[kGenericWaves])
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr uint32_t MASK = RING ? (uint32_t)kRing - 1u : 0xffffffffu;
    const int m = g.m, n = g.n;
    const uint32_t *aseq = W + (g.abase >> 4), *bseq = W + (g.bbase >> 4);
    const int aph = (int)(g.abase & 15) - 1, bph = (int)(g.bbase & 15) - 1;   // a_i = code aph + i
    for (; s.d <= m + n; ++s.d) {
        const int d = s.d;
        // candidates: successors of live cells on d-1 (i, i+1) and on d-2 (i+1), inside the table
        int slo = 1 << 30, shi = -(1 << 30);
        if (s.lo1 <= s.hi1) { slo = min(slo, s.lo1); shi = max(shi, s.hi1 + 1); }
        if (s.lo2 <= s.hi2) { slo = min(slo, s.lo2 + 1); shi = max(shi, s.hi2 + 1); }
        slo = max(slo, max(0, d - n));
        shi = min(shi, min(m, d));
        if (RING && shi - slo + 1 > kRing) return false;   // uniform over the block
        const int thr = s.T - X;
        // wave-uniform live range and candidate count from ballots (the
        // lanes of a wavefront hold consecutive i in every pass of the loop);
        // per lane the best value and its first i
        int wlo = 0x7fffffff, whi = -1, bv = NEG, bidx = 0x7fffffff;
        uint32_t wcand = 0;
        for (int i = slo + tid; i <= shi; i += kGenericThreads) {
            // a live range lies inside the table of its anti-diagonal, so a
            // predecessor inside it has i >= 0 and j >= 0
            const bool hd = i - 1 >= s.lo2 && i - 1 <= s.hi2;
            const bool hu = i - 1 >= s.lo1 && i - 1 <= s.hi1;
            const bool hl = i >= s.lo1 && i <= s.hi1;
            // codes of a_i and b_j (i, j >= 0: at worst one base before the
            // sequence, inside the store's guard words), loaded before the
            // predecessors so that both latencies overlap
            const int pa = aph + i, pb = bph + (d - i);
            const uint32_t wa = aseq[pa >> 4], wb = bseq[pb >> 4];
            int pd, pu, pl;
            if (RING) {
                // every ring slot is inside the array: load, then select
                pd = P2[(uint32_t)(i - 1) & MASK];
                pu = P1[(uint32_t)(i - 1) & MASK];
                pl = P1[(uint32_t)i & MASK];
                pd = hd ? pd : NEG;
                pu = hu ? pu : NEG;
                pl = hl ? pl : NEG;
            } else {
                pd = hd ? P2[i - 1] : NEG;
                pu = hu ? P1[i - 1] : NEG;
                pl = hl ? P1[i] : NEG;
            }
            // keeps the code loads above this point (the compiler would sink
            // them into the diagonal-move branch, after the predecessor loads)
            asm volatile("" ::"v"(wa), "v"(wb));
            const bool okd = pd > NEG_HALF, oku = pu > NEG_HALF, okl = pl > NEG_HALF;
            const uint32_t ca = __builtin_amdgcn_ubfe(wa, (uint32_t)(pa & 15) * 2u, 2u);
            const uint32_t cb = __builtin_amdgcn_ubfe(wb, (uint32_t)(pb & 15) * 2u, 2u);
            int v = okd ? pd + (ca == cb ? ma : mi) : NEG;
            v = oku ? max(v, pu + gap) : v;
            v = okl ? max(v, pl + gap) : v;
            const bool cand = okd || oku || okl;
            const bool lv = cand && v >= thr;
            P0[(uint32_t)i & MASK] = lv ? v : NEG;
            if (COUNT) wcand += (uint32_t)__builtin_popcountll(ballot(cand));
            const uint64_t lm = ballot(lv);
            if (lm) {
                const int i0 = uni(i - lane);   // i of lane 0 in this pass
                wlo = min(wlo, i0 + (int)__builtin_ctzll(lm));
                whi = max(whi, i0 + 63 - (int)__builtin_clzll(lm));
            }
            const bool up = lv && v > bv;   // i rises along the loop: first i kept on ties
            bidx = up ? i : bidx;
            bv = up ? v : bv;
        }
        // wavefront partials, then every thread reduces the partials of all wavefronts
        GPart *pp = part[d & 1];
        {
            const int wv = wave_reduce(bv, OpMax());
            // smallest i holding the maximum: the lowest such lane unless
            // several passes of the loop hold it
            const uint64_t at = ballot(bv == wv);
            int wi = __builtin_amdgcn_readlane(bidx, (int)__builtin_ctzll(at | (1ull << 63)));
            if (shi - slo >= kGenericThreads && __builtin_popcountll(at) > 1)
                wi = wave_reduce(bv == wv ? bidx : 0x7fffffff, OpMin());
            if (lane == 0) {
                GPart q;
                q.lo = wlo; q.hi = whi; q.v = wv; q.i = wi; q.cells = wcand;
                q.pad[0] = q.pad[1] = q.pad[2] = 0;
                pp[wid] = q;
            }
        }
        // One barrier per anti-diagonal: it orders this anti-diagonal's
        // stores before the next one's loads.  The partials alternate
        // between two buffers and the three anti-diagonal arrays rotate, so a
        // location is written again only after every thread has passed the
        // barrier that follows its last read.
        __syncthreads();
        // lane l of every row of 16 reads the partial of wavefront l
        static_assert(kGenericWaves == 16, "one partial per lane of a DPP row");
        const GPart q = pp[lane & 15];
        const int nlo = row_reduce(q.lo, OpMin());
        const int nhi = row_reduce(q.hi, OpMax());
        const int vmax = row_reduce(q.v, OpMax());
        const int imin = row_reduce(q.v == vmax ? q.i : 0x7fffffff, OpMin());
        const uint32_t ctot = COUNT ? (uint32_t)row_reduce((int)q.cells, OpAdd()) : 0u;
        if (COUNT) {
            s.cells += ctot;
            if (shi >= slo) s.slots += (uint64_t)((shi - slo + 64) / 64) * 64;
        }
        const bool live = nhi >= 0;
        if (live && vmax > s.T) { s.T = vmax; s.bi = imin; s.bj = d - imin; }
        int *tp = P2; P2 = P1; P1 = P0; P0 = tp;
        s.lo2 = s.lo1; s.hi2 = s.hi1;
        s.lo1 = live ? nlo : 1; s.hi1 = live ? nhi : 0;
        if (!live && s.prev_dead) return true;
        s.prev_dead = !live;
    }
    return true;
}

// Ring state of an unbounded extension resumed from a window of `win` slots
// in window units (anti-diagonal d-1 at z1[0, win), d-2 at z2[0, win), slot
// q of anti-diagonal e holding cell i = base + floor(e / 2) + q, Z = S +
// |gap| * e); s.d, T, the best cell and the counts are set.  The live cells
// go into the rings by i, as scores.
__device__ void generic_resume(const int *z1src, const int *z2src, int win, int base, int gap, int *P1, int *P2,
                               GState &s)
{
    __shared__ int s_rng[4];
    const int tid = threadIdx.x;
    s.prev_dead = false;
    if (tid == 0) { s_rng[0] = 0x7fffffff; s_rng[1] = -1; s_rng[2] = 0x7fffffff; s_rng[3] = -1; }
    // Every slot of the two rings starts dead: the anti-diagonals read any
    // slot between the live ends, and a carried band has dead cells inside
    // it, which would otherwise keep what an earlier task left in the ring.
    for (int q = tid; q < kRing; q += kGenericThreads) {
        P1[q] = NEG;
        P2[q] = NEG;
    }
    __syncthreads();
    const int G = -gap, d1 = s.d - 1, d2 = s.d - 2;
    const int o1 = base + (d1 >> 1), o2 = base + (d2 >> 1);   // i of slot 0 (d2 >= 0: a window ran)
    for (int q = tid; q < win; q += kGenericThreads) {
        const int z1 = z1src[q], z2 = z2src[q];
        if (z1 > NEG_HALF) {
            const int i = o1 + q;   // live cells lie inside the table: i >= 0
            P1[(uint32_t)i & (kRing - 1)] = z1 - G * d1;
            atomicMin(&s_rng[0], i);
            atomicMax(&s_rng[1], i);
        }
        if (z2 > NEG_HALF) {
            const int i = o2 + q;
            P2[(uint32_t)i & (kRing - 1)] = z2 - G * d2;
            atomicMin(&s_rng[2], i);
            atomicMax(&s_rng[3], i);
        }
    }
    __syncthreads();
    s.lo1 = s_rng[0]; s.hi1 = s_rng[1];
    s.lo2 = s_rng[2]; s.hi2 = s_rng[3];
    if (s.lo1 > s.hi1) { s.lo1 = 1; s.hi1 = 0; s.prev_dead = true; }
    if (s.lo2 > s.hi2) { s.lo2 = 1; s.hi2 = 0; }
    __syncthreads();   // s_rng read by every thread before another task resets it
}

// The ring phase of an unbounded extension, from the register window the
// task's band outgrew (its state in xs, its anti-diagonals in z1 / z2).
template <bool COUNT>
__device__ void generic_run(const uint32_t *__restrict__ W, const Geo &g, int X, int ma, int mi, int gap,
                            const XState &xs, const int *z1, const int *z2, int win, int *ring, int *G2, int *G1,
                            int *G0, GPart (*part)[kGenericWaves], TaskOut &o)
{
    const int tid = threadIdx.x;
    GState s;
    int *P0 = ring, *P1 = ring + kRing, *P2 = ring + 2 * kRing;
    s.d = xs.d; s.T = xs.T; s.bi = xs.bi; s.bj = xs.bj; s.cells = xs.cells; s.slots = xs.slots;
    generic_resume(z1, z2, win, xs.base, gap, P1, P2, s);
    if (!generic_diags<COUNT, true>(W, g, X, ma, mi, gap, P2, P1, P0, s, part)) {
        // the band outgrew the ring: the live cells of the last two
        // anti-diagonals move to global memory
        for (int i = s.lo1 + tid; i <= s.hi1; i += kGenericThreads) G1[i] = P1[(uint32_t)i & (kRing - 1)];
        for (int i = s.lo2 + tid; i <= s.hi2; i += kGenericThreads) G2[i] = P2[(uint32_t)i & (kRing - 1)];
        __threadfence_block();
        __syncthreads();
        generic_diags<COUNT, false>(W, g, X, ma, mi, gap, G2, G1, G0, s, part);
    }
    o.score = s.T; o.i = s.bi; o.j = s.bj; o.status = (uint32_t)kGenericClass; o.cells = s.cells; o.slots = s.slots;
}

// Unbounded class.  Each extension first runs in a register window of
// kGenericWin slots shared by the workgroup's 16 wavefronts (4 cells per
// lane), resumed from the 2048-slot class's carried state; a band that
// outgrows it continues in the LDS ring (and in global memory beyond it).
constexpr int kGenericWin = 4096;
constexpr int kGenericC = kGenericWin / (64 * kGenericWaves);

template <bool COUNT>
__global__ void __launch_bounds__(kGenericThreads) generic_kernel(BatchDev b, StoreDev st, int32_t *scratch,
                                                                  uint64_t stride)
{
    __shared__ int ring[3 * kRing];
    __shared__ GPart part[2][kGenericWaves];
    __shared__ GroupShared<kGenericWaves, kGenericWin> gsh;
    __shared__ uint32_t s_task;
    const uint32_t qcap = 2u * b.cap;
    const int cls = kGenericClass;
    const uint32_t cnt = b.ctr[CtrLayout::kCount + cls];
    const int wv = uni((int)(threadIdx.x >> 6));
    int *base = scratch + (uint64_t)blockIdx.x * 3 * stride;
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(&b.ctr[CtrLayout::kHead + cls], 1u);
        __syncthreads();
        const uint32_t idx = s_task;
        __syncthreads();         // read by every thread before thread 0 writes it again
        if (idx >= cnt) break;   // uniform over the block
        const uint32_t t = (uint32_t)uni((int)b.qbuf[cls * qcap + idx]);
        const uint32_t coff = (uint32_t)uni((int)b.qstate[cls * qcap + idx]);
        const Task k = load_task(b.recs, st.reads, t);
        XState xs;
        uint32_t stt;
        if (k.ma != 1)
            stt = group_run<kGenericC, kGenericC, kGenericWaves, COUNT, false, false>(b, st, k, gsh, wv, xs, coff);
        else if (sigma_fits_2bits(k))
            stt = group_run<kGenericC, kGenericC, kGenericWaves, COUNT, true, true>(b, st, k, gsh, wv, xs, coff);
        else
            stt = group_run<kGenericC, kGenericC, kGenericWaves, COUNT, true, false>(b, st, k, gsh, wv, xs, coff);
        TaskOut o;
        if (stt == kDone) {
            o.score = xs.T; o.i = xs.bi; o.j = xs.bj; o.status = (uint32_t)cls; o.cells = xs.cells;
            o.slots = xs.slots;
        } else {
            generic_run<COUNT>(st.words, k.g, k.x, k.ma, k.mi, k.gap, xs, gsh.win, gsh.win + kGenericWin,
                               kGenericWin, ring, base, base + stride, base + 2 * stride, part, o);
        }
        if (threadIdx.x == 0) b.tout[t] = o;
        __syncthreads();         // ring, window and scratch of this task no longer read before the next one starts
    }
}

// ---------------------------------------------------------------------------
// Result write-back.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) finalize_kernel(BatchDev b, StoreDev st, int stage_sums)
{
    // per-stage totals (cells, extensions and slot-steps of each class) are
    // summed in LDS, then added with one global atomic per counter and block
    __shared__ unsigned long long acc[kStageSumWords];
    if (stage_sums) {
        if (threadIdx.x < kStageSumWords) acc[threadIdx.x] = 0ull;
        __syncthreads();
    }
    const uint32_t n = b.ctr[CtrLayout::kN];
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = r < n && b.valid[r];
    if (stage_sums && ok) {
        for (int s = 0; s < 2; ++s) {
            const TaskOut o = b.tout[2 * r + s];
            const int stg = 1 + (int)o.status;
            atomicAdd(&acc[stg], (unsigned long long)o.cells);
            atomicAdd(&acc[8 + stg], 1ull);
            atomicAdd(&acc[16 + stg], (unsigned long long)o.slots);
        }
    }
    if (r < n) {
        xdrop_result out{};
        uint64_t c = 0;
        if (ok) {
            const xdrop_record R = b.recs[r];
            const ReadInfo B = st.reads[R.read_b];
            const uint32_t pb = R.strand ? B.len - R.pos_b - R.k : R.pos_b;
            const TaskOut L = b.tout[2 * r], Rt = b.tout[2 * r + 1];
            const int s = b.seed[r];
            out.left_score = L.score;
            out.right_score = Rt.score;
            out.seed_score = s;
            out.score = L.score + s + Rt.score;
            out.a_begin = R.pos_a - (uint32_t)L.i;
            out.a_end = R.pos_a + R.k + (uint32_t)Rt.i;
            out.b_begin = pb - (uint32_t)L.j;
            out.b_end = pb + R.k + (uint32_t)Rt.j;
            c = L.cells + Rt.cells;
        }
        b.res[r] = out;
        if (b.cells) b.cells[r] = c;
    }
    if (stage_sums) {
        __syncthreads();
        if (threadIdx.x < kStageSumWords && acc[threadIdx.x]) atomicAdd(&b.stage_sum[threadIdx.x], acc[threadIdx.x]);
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_reset_n(const BatchDev &b, const uint32_t *n_src, uint32_t n_imm, hipStream_t s)
{
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(256), 0, s, b.ctr, b.bucket_hist, b.stage_sum, n_src, n_imm);
}

void launch_accum_errors(const BatchDev &b, uint32_t *acc, hipStream_t s)
{
    hipLaunchKernelGGL(accum_errors_kernel, dim3(1), dim3(64), 0, s, (const uint32_t *)b.ctr, acc);
}

void launch_prep(const BatchDev &b, const StoreDev &st, const Tuning &tu, uint32_t n, bool stage, hipStream_t s)
{
    const uint32_t blocks = (n + 255) / 256;
    if (blocks) hipLaunchKernelGGL(prep_kernel, dim3(blocks), dim3(256), 0, s, b, st, tu, stage ? 1 : 0);
}

void launch_bucket(const BatchDev &b, const StoreDev &st, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(bucket_scan_kernel, dim3(1), dim3(64), 0, s, b);
    const uint32_t blocks = (2 * n + 255) / 256;
    if (blocks) hipLaunchKernelGGL(bucket_scatter_kernel, dim3(blocks), dim3(256), 0, s, b, st);
}

void launch_narrow(const BatchDev &b, const StoreDev &st, const Tuning &tu, uint32_t grid_waves, bool count_cells,
                   hipStream_t s)
{
    const uint32_t blocks = (grid_waves + 3) / 4;
    if (count_cells)
        hipLaunchKernelGGL(narrow_kernel<true>, dim3(blocks), dim3(256), 0, s, b, st, tu.shrink_margin);
    else
        hipLaunchKernelGGL(narrow_kernel<false>, dim3(blocks), dim3(256), 0, s, b, st, tu.shrink_margin);
}

void launch_adaptive(const BatchDev &b, const StoreDev &st, const Tuning &tu, uint32_t grid_waves, bool count_cells,
                     hipStream_t s)
{
    const uint32_t blocks = (grid_waves + 3) / 4;
    if (count_cells)
        hipLaunchKernelGGL(adaptive_kernel<true>, dim3(blocks), dim3(256), 0, s, b, st, tu.grow_margin, tu.shrink_margin);
    else
        hipLaunchKernelGGL(adaptive_kernel<false>, dim3(blocks), dim3(256), 0, s, b, st, tu.grow_margin, tu.shrink_margin);
}

template <int L>
static void launch_wide_c(const BatchDev &b, const StoreDev &st, int cls, uint32_t grid_waves, bool count,
                          hipStream_t s)
{
    const uint32_t blocks = (grid_waves + 3) / 4;
    const size_t lds = 4 * 2 * 64 * kWideC[L] * sizeof(int);
    if (count)
        hipLaunchKernelGGL((wide_kernel<L, true>), dim3(blocks), dim3(256), lds, s, b, st, cls);
    else
        hipLaunchKernelGGL((wide_kernel<L, false>), dim3(blocks), dim3(256), lds, s, b, st, cls);
}

template <int CLO, int CHI, int W>
static void launch_group_c(const BatchDev &b, const StoreDev &st, int cls, uint32_t grid_waves, bool count,
                           hipStream_t s)
{
    const uint32_t blocks = (grid_waves + W - 1) / W;
    if (count)
        hipLaunchKernelGGL((group_kernel<CLO, CHI, W, true>), dim3(blocks), dim3(64 * W), 0, s, b, st, cls);
    else
        hipLaunchKernelGGL((group_kernel<CLO, CHI, W, false>), dim3(blocks), dim3(64 * W), 0, s, b, st, cls);
}

void launch_wide(int which, const BatchDev &b, const StoreDev &st, uint32_t cus, int ext_waves, bool count_cells,
                 hipStream_t s)
{
    static_assert(kWideClasses == 2, "wide classes");
    const int cls = kAdaptiveClass + 1 + which;
    if (which == 0) launch_wide_c<0>(b, st, cls, cus * 8u, count_cells, s);
    else if (ext_waves == 2) launch_group_c<12, 16, 2>(b, st, cls, cus * 12u, count_cells, s);
    else if (ext_waves == 4) launch_group_c<6, 8, 4>(b, st, cls, cus * 16u, count_cells, s);
    else launch_wide_c<1>(b, st, cls, cus * 8u, count_cells, s);
}

void launch_generic(const BatchDev &b, const StoreDev &st, int32_t *scratch, uint64_t stride, uint32_t blocks,
                    bool count_cells, hipStream_t s)
{
    // one task per workgroup of kGenericThreads; workgroup k owns
    // scratch[3 * stride * k, 3 * stride * (k + 1))
    blocks = max(1u, blocks);
    if (count_cells)
        hipLaunchKernelGGL(generic_kernel<true>, dim3(blocks), dim3(kGenericThreads), 0, s, b, st, scratch, stride);
    else
        hipLaunchKernelGGL(generic_kernel<false>, dim3(blocks), dim3(kGenericThreads), 0, s, b, st, scratch, stride);
}

void launch_finalize(const BatchDev &b, const StoreDev &st, uint32_t n, bool stage_sums, hipStream_t s)
{
    const uint32_t blocks = (n + 255) / 256;
    if (blocks) hipLaunchKernelGGL(finalize_kernel, dim3(blocks), dim3(256), 0, s, b, st, stage_sums ? 1 : 0);
}

}  // namespace xd
