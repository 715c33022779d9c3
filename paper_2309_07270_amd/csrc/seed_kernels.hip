// seed_kernels.hip -- gfx950 kernels of seed discovery: read pairs that share
// a reliable k-mer, one seed per pair (paper, "Related works": BELLA finds
// overlaps from shared k-mers, filters unreliable ones and extends the seeds
// with an X-drop; "Method": k-mers of length 31 at stride 1 whose frequency
// lies in a window, [20, 30] for the 29x set and [20, 50] for the 100x set).
//
// Definitions (stated in include/xdrop.h): canonical k-mer = the smaller,
// as a base-4 number with the first base most significant, of a k-mer and
// its reverse complement; frequency = occurrences over all reads and
// positions; a pair's seed = the smallest (pos_a, pos_b, strand) over the
// occurrences of its shared reliable k-mers.
//
// Pipeline, with no sort:
//   1. count: every k-mer of every read into an open-addressing table
//      (64-bit compare-and-swap on the key, linear probing);
//   2. reliable: each entry with lo <= count <= hi gets a dense index
//      (per-wavefront counts over table chunks, a scan, an assignment);
//   3. occurrences: each occurrence of a reliable k-mer is appended to the
//      k-mer's list (hi slots per reliable k-mer);
//   4. pairs: every two occurrences of one list from different reads give a
//      candidate seed, kept per read pair by a 64-bit atomic minimum in a
//      second table;
//   5. emit: one record per table entry (order unspecified).
// One wavefront walks the positions of one read, 64 at a time, so the code
// windows of neighbouring lanes share words.
#include <hip/hip_runtime.h>

#include "xdrop_internal.h"

namespace xd {

namespace {

constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    // finaliser of splitmix64 (Steele, Lea, Flood, "Fast splittable
    // pseudorandom number generators", 2014)
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

// k-mer at base index b of the store: canonical code and orientation
// (true when the store holds the reverse complement of the canonical string)
__device__ __forceinline__ uint64_t canonical_at(const uint32_t *__restrict__ W, uint64_t b, int k, bool &rev)
{
    const uint32_t *w = W + (b >> 4);
    const uint32_t sh = (uint32_t)(b & 15) * 2u;
    const uint32_t lo = __builtin_amdgcn_alignbit(w[1], w[0], sh);
    const uint32_t hi = __builtin_amdgcn_alignbit(w[2], w[1], sh);
    const uint64_t mask = (k == 32) ? ~0ull : ((1ull << (2 * k)) - 1ull);
    const uint64_t lsb = (((uint64_t)hi << 32) | lo) & mask;   // base i at bits 2i, 2i+1
    // first base most significant: reverse the 2-bit groups
    uint64_t y = __builtin_bitreverse64(lsb);
    y = ((y >> 1) & 0x5555555555555555ull) | ((y & 0x5555555555555555ull) << 1);
    const uint64_t fwd = y >> (64 - 2 * k);
    // reverse complement, first base most significant: base k-1-i of the
    // reverse complement is 3 - base i, at group i -- the complement of lsb
    const uint64_t rc = ~lsb & mask;
    rev = rc < fwd;
    return rev ? rc : fwd;
}

// table slot holding `key`, inserting it if absent (insert) or -1 if absent
// (lookup); -1 if the table is full.  A key already present is found by a
// plain load; the compare-and-swap is only tried on an empty slot.
__device__ __forceinline__ int64_t slot_of(uint64_t *keys, uint64_t cap, uint64_t key, bool insert)
{
    uint64_t h = mix64(key) & (cap - 1);
    for (uint64_t probe = 0; probe < cap; ++probe) {
        uint64_t cur = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
        if (cur == kEmpty) {
            if (!insert) return -1;
            cur = atomicCAS((unsigned long long *)&keys[h], (unsigned long long)kEmpty, (unsigned long long)key);
            if (cur == kEmpty) return (int64_t)h;
        }
        if (cur == key) return (int64_t)h;
        h = (h + 1) & (cap - 1);
    }
    return -1;
}

// Wave-uniform fetch-and-add of `v` (the value of lane 0); every lane takes
// part so that no lane-dependent branch surrounds the atomic.
__device__ __forceinline__ uint32_t wave_fetch_add(uint32_t *p, uint32_t v)
{
    const uint32_t old = atomicAdd(p, (threadIdx.x & 63) == 0 ? v : 0u);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)old);
}

// positions of read r that start a k-mer: 0, s, 2s, ...
__device__ __forceinline__ uint32_t n_positions(uint32_t len, int k, int s)
{
    return len >= (uint32_t)k ? (len - (uint32_t)k) / (uint32_t)s + 1u : 0u;
}

__global__ void __launch_bounds__(256) kmer_count_kernel(SeedDev sd, StoreDev st)
{
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t waves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    for (uint32_t r = wave; r < st.n_reads; r += waves) {
        const ReadInfo R = st.reads[r];
        const uint32_t np = n_positions(R.len, sd.k, sd.stride);
        for (uint32_t q = lane; q < np; q += 64) {
            bool rev;
            const uint64_t key = canonical_at(st.words, R.fwd + (uint64_t)q * sd.stride, sd.k, rev);
            const int64_t h = slot_of(sd.keys, sd.cap, key, true);
            if (h >= 0) atomicAdd(&sd.counts[h], 1u);
            else atomicOr(&sd.ctr[kSeedOverflow], 1u);
        }
    }
}

// Reliable k-mers get dense indices in two passes over contiguous chunks of
// the table, one chunk per wavefront: count, exclusive scan over the chunks,
// assign.  One global atomic per wavefront in all (a counter per entry would
// serialise on one address).
__device__ __forceinline__ void chunk_of(const SeedDev &sd, uint32_t wave, uint64_t &h0, uint64_t &h1)
{
    h0 = min((uint64_t)wave * sd.chunk, sd.cap);
    h1 = min(h0 + sd.chunk, sd.cap);
}

__device__ __forceinline__ bool reliable_at(const SeedDev &sd, uint64_t h, bool &used)
{
    used = sd.keys[h] != kEmpty;
    const uint32_t c = used ? sd.counts[h] : 0u;
    return used && c >= (uint32_t)sd.lo && c <= (uint32_t)sd.hi;
}

__global__ void __launch_bounds__(256) kmer_reliable_count_kernel(SeedDev sd)
{
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    uint64_t h0, h1;
    chunk_of(sd, wave, h0, h1);
    uint32_t n_used = 0, n_rel = 0;
    for (uint64_t h = h0 + lane; h < h1; h += 64) {       // chunk: a multiple of 64 slots
        bool used;
        const bool rel = reliable_at(sd, h, used);
        n_used += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(used));
        n_rel += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(rel));
    }
    wave_fetch_add(&sd.ctr[kSeedDistinct], n_used);
    sd.wcount[wave] = n_rel;   // every lane stores the same (wave-uniform) value
}

// exclusive scan of n values in one block of 1024 threads; the total goes
// to *total
__global__ void __launch_bounds__(1024) scan_kernel(uint32_t *v, uint32_t n, uint32_t *total)
{
    __shared__ uint32_t part[1024];
    const uint32_t t = threadIdx.x;
    const uint32_t per = (n + 1023) / 1024;
    const uint32_t b = t * per, e = min(b + per, n);
    uint32_t sum = 0;
    for (uint32_t i = b; i < e; ++i) sum += v[i];
    part[t] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {      // inclusive Hillis-Steele scan
        const uint32_t x = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (uint32_t i = b; i < e; ++i) {
        const uint32_t x = v[i];
        v[i] = run;
        run += x;
    }
    if (t == 1023) *total = part[1023];
}

__global__ void __launch_bounds__(256) kmer_reliable_assign_kernel(SeedDev sd)
{
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    uint64_t h0, h1;
    chunk_of(sd, wave, h0, h1);
    uint32_t next = h0 < h1 ? sd.wcount[wave] : 0u;
    for (uint64_t h = h0 + lane; h < h1; h += 64) {
        bool used;
        const bool rel = reliable_at(sd, h, used);
        const uint64_t rm = __builtin_amdgcn_ballot_w64(rel);
        const uint32_t id = next + (uint32_t)__builtin_popcountll(rm & ((1ull << lane) - 1ull));
        next += (uint32_t)__builtin_popcountll(rm);
        sd.rid[h] = (rel && id < sd.max_reliable) ? (int32_t)id : -1;
    }
}

__global__ void __launch_bounds__(256) kmer_occurrence_kernel(SeedDev sd, StoreDev st)
{
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t waves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    for (uint32_t r = wave; r < st.n_reads; r += waves) {
        const ReadInfo R = st.reads[r];
        const uint32_t np = n_positions(R.len, sd.k, sd.stride);
        for (uint32_t q = lane; q < np; q += 64) {
            bool rev;
            const uint32_t p = q * (uint32_t)sd.stride;
            const uint64_t key = canonical_at(st.words, R.fwd + p, sd.k, rev);
            const int64_t h = slot_of(sd.keys, sd.cap, key, false);
            if (h < 0) continue;
            const int32_t id = sd.rid[h];
            if (id < 0) continue;
            const uint32_t at = atomicAdd(&sd.fill[id], 1u);
            if (at < (uint32_t)sd.hi)
                sd.occ[(uint64_t)id * sd.hi + at] = ((uint64_t)r << 32) | ((uint64_t)p << 1) | (rev ? 1u : 0u);
        }
    }
}

// one thread per (reliable k-mer, first occurrence i): pairs (i, j > i)
__global__ void __launch_bounds__(256) seed_pair_kernel(SeedDev sd)
{
    const uint32_t n_rel = min(sd.ctr[kSeedReliable], sd.max_reliable);
    const uint64_t total = (uint64_t)n_rel * sd.hi;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total; t += stride) {
        const uint32_t id = (uint32_t)(t / sd.hi), i = (uint32_t)(t % sd.hi);
        const uint32_t n = min(sd.fill[id], (uint32_t)sd.hi);
        if (i >= n) continue;
        const uint64_t *L = sd.occ + (uint64_t)id * sd.hi;
        const uint64_t x = L[i];
        for (uint32_t j = i + 1; j < n; ++j) {
            const uint64_t y = L[j];
            const uint32_t rx = (uint32_t)(x >> 32), ry = (uint32_t)(y >> 32);
            if (rx == ry) continue;
            const uint64_t a = rx < ry ? x : y, b = rx < ry ? y : x;
            const uint64_t pa = (a >> 1) & 0x7fffffffull, pb = (b >> 1) & 0x7fffffffull;
            const uint64_t strand = (a ^ b) & 1ull;
            // (pos_a, pos_b, strand) ordered as one number
            const uint64_t cand = (pa << 32) | (pb << 1) | strand;
            const uint64_t pkey = ((a >> 32) << 32) | (b >> 32);
            const int64_t h = slot_of(sd.pkeys, sd.pcap, pkey, true);
            if (h < 0) {
                atomicOr(&sd.ctr[kSeedOverflow], 4u);
                continue;
            }
            // stored values only decrease: a candidate not below a (possibly
            // stale) stored value cannot be the minimum
            if (cand < __atomic_load_n(&sd.pvals[h], __ATOMIC_RELAXED))
                atomicMin((unsigned long long *)&sd.pvals[h], (unsigned long long)cand);
        }
    }
}

__global__ void __launch_bounds__(256) seed_emit_kernel(SeedDev sd, xdrop_record *out, uint32_t max_out, int x,
                                                       int ma, int mi, int gap)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t h = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; h < sd.pcap; h += stride) {
        const uint64_t key = sd.pkeys[h];
        if (key == kEmpty) continue;
        const uint32_t at = atomicAdd(&sd.ctr[kSeedPairs], 1u);
        if (at >= max_out) continue;
        const uint64_t v = sd.pvals[h];
        xdrop_record R{};
        R.read_a = (uint32_t)(key >> 32);
        R.read_b = (uint32_t)key;
        R.pos_a = (uint32_t)(v >> 32);
        R.pos_b = (uint32_t)((v >> 1) & 0x7fffffffull);
        R.strand = (uint8_t)(v & 1ull);
        R.k = (uint16_t)sd.k;
        R.x = x;
        R.match = (int16_t)ma;
        R.mismatch = (int16_t)mi;
        R.gap = (int16_t)gap;
        out[at] = R;
    }
}

__global__ void seed_init_kernel(SeedDev sd)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    for (uint64_t h = t0; h < sd.cap; h += stride) {
        sd.keys[h] = kEmpty;
        sd.counts[h] = 0u;
    }
    for (uint64_t h = t0; h < sd.pcap; h += stride) {
        sd.pkeys[h] = kEmpty;
        sd.pvals[h] = ~0ull;
    }
    for (uint64_t i = t0; i < sd.max_reliable; i += stride) sd.fill[i] = 0u;
    if (t0 < kSeedCounters) sd.ctr[t0] = 0u;
}

}  // namespace

void launch_seeds(const SeedDev &sd, const StoreDev &st, xdrop_record *d_out, uint32_t max_out, int x, int ma,
                  int mi, int gap, int cus, hipStream_t s, hipEvent_t *ev)
{
    const int blocks = cus * 8;
    hipLaunchKernelGGL(seed_init_kernel, dim3(blocks), dim3(256), 0, s, sd);
    if (ev) hipEventRecord(ev[0], s);
    hipLaunchKernelGGL(kmer_count_kernel, dim3(blocks), dim3(256), 0, s, sd, st);
    hipLaunchKernelGGL(kmer_reliable_count_kernel, dim3(blocks), dim3(256), 0, s, sd);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, sd.wcount, sd.n_chunks, sd.ctr + kSeedReliable);
    hipLaunchKernelGGL(kmer_reliable_assign_kernel, dim3(blocks), dim3(256), 0, s, sd);
    hipLaunchKernelGGL(kmer_occurrence_kernel, dim3(blocks), dim3(256), 0, s, sd, st);
    hipLaunchKernelGGL(seed_pair_kernel, dim3(blocks), dim3(256), 0, s, sd);
    hipLaunchKernelGGL(seed_emit_kernel, dim3(blocks), dim3(256), 0, s, sd, d_out, max_out, x, ma, mi, gap);
    if (ev) hipEventRecord(ev[1], s);
}

}  // namespace xd
