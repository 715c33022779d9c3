/*
 * xdrop.h -- C ABI of libxdrop.so: batched X-drop seed-and-extend of long-read
 * pairs on one AMD Instinct MI355X (gfx950).
 *
 * What is computed (paper, "Related works": BELLA's seed-and-extend with an
 * X-drop; LOGAN's GPU X-drop over anti-diagonals; "Results": the aligner is a
 * Needleman-Wunsch / Smith-Waterman recurrence with an X-drop):
 *
 *   For each record, read B is oriented (B' = B, or its reverse complement
 *   when strand = 1), the seed A[pos_a, pos_a+k) vs B'[pos_b', pos_b'+k) is
 *   scored base by base, and the alignment is extended to the left and to the
 *   right with an X-drop dynamic programme over anti-diagonals:
 *     - cell (i,j) of an extension lies on anti-diagonal d = i+j; S(0,0) = 0;
 *     - a cell is evaluated when one of (i-1,j-1), (i-1,j), (i,j-1) is live;
 *       its value is the best of S(i-1,j-1)+sigma, S(i-1,j)+gap, S(i,j-1)+gap
 *       over live predecessors (linear gap, no zero floor);
 *     - it dies when its value is strictly below T_{d-1} - X, T_{d-1} being
 *       the best live value on anti-diagonals 0..d-1;
 *     - the extension stops after two consecutive anti-diagonals without a
 *       live cell (or at the far corner); its result is the best value T and
 *       the first cell reaching it (smallest d, then smallest i).
 *   Batches follow the paper's baseline scheduler ("Method", Baseline): the
 *   caller hands over one batch of records per call.
 *
 * Conventions: every call returns xdrop_status (0 = OK, < 0 = error).  Scores
 * are exact int32; nothing is approximated.  Reads are ASCII A/C/G/T (either
 * case).  Coordinates are 0-based, spans half-open.
 *
 * Threading: xdrop_batch_submit*, xdrop_batch_wait may be called concurrently
 * from many threads on one context (producers).
 * xdrop_batch_destroy must not race any other call on the same context.
 */
#ifndef XDROP_H
#define XDROP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    XDROP_OK = 0,
    XDROP_E_INVALID = -1,  /* bad argument or record (nothing was submitted)     */
    XDROP_E_NOMEM = -2,    /* host or device allocation failed                   */
    XDROP_E_DEVICE = -3,   /* HIP runtime or kernel error; context is poisoned   */
    XDROP_E_TIMEOUT = -4,  /* wait timed out; the batch is still running         */
    XDROP_E_BUSY = -5,     /* admission refused with timeout 0 (back-pressure)   */
    XDROP_E_STATE = -6     /* unknown or already-consumed ticket, bad ctx state  */
} xdrop_status;

enum {
    XDROP_MODE_PERSISTENT = 0, /* whole batch in one graph: bucketed longest-first
                                  tasks, persistent work-stealing kernels        */
    XDROP_MODE_PLAIN = 1       /* one launch sequence per 10,000-record chunk, one
                                  wavefront per extension, no reordering          */
};

typedef struct xdrop_ctx xdrop_ctx;   /* opaque */
typedef uint64_t xdrop_ticket;

typedef struct {
    /* read store, copied and packed at create (caller may free afterwards) */
    const char *const *reads;     /* n_reads pointers to ASCII bases        */
    const uint32_t *lengths;      /* n_reads lengths (each <= XDROP_MAX_READ_LEN) */
    uint32_t n_reads;
    int32_t device;               /* HIP device ordinal                     */
    uint32_t mode;                /* XDROP_MODE_*                           */
    uint32_t max_inflight;        /* batches admitted at once; 0 -> 4       */
    uint64_t hbm_budget_bytes;    /* device bytes for in-flight batches; 0 -> 32 GiB */
    const char *tuning_cache;     /* path of the autotuner cache, or NULL   */
    uint32_t flags;               /* XDROP_FLAG_*                           */
} xdrop_config;

enum {
    XDROP_FLAG_PROFILE = 1        /* time every kernel stage with HIP events
                                     (stats.stage_ms); adds ~1 us per stage  */
};

/* Kernel stages reported in xdrop_batch_stats.stage_ms / stage_cells.  An
 * extension with a small drop (x <= the narrow_x tuning knob, persistent
 * form, batches of at least narrow_min_records records) and weights match 1,
 * gap -1, mismatch 0, -1 or -2 runs in the narrow kernel first; every other
 * one in the adaptive kernel.  It moves to the next stage only when its live
 * band outgrows the current one: out of the narrow kernel it restarts from
 * the seed; from the adaptive kernel on it carries its state over
 * (restarting only when the batch's carry pool is full). */
enum {
    XDROP_STAGE_INGEST = 0,       /* counter reset, validation, seed, bucketing  */
    XDROP_STAGE_NARROW = 1,       /* two extensions per wavefront, windows of
                                     32 or 64 slots over half the lanes     */
    XDROP_STAGE_ADAPTIVE = 2,     /* register window of 64..256 slots that
                                     follows the band width                 */
    XDROP_STAGE_WIDE1280 = 3,     /* register window of 512..1280 slots that
                                     follows the band width                 */
    XDROP_STAGE_WIDE2048 = 4,     /* register window of 2048 slots, shared by
                                     the wide_waves wavefronts of a workgroup
                                     (one wavefront: 1536..2048 slots)      */
    XDROP_STAGE_GENERIC = 5,      /* unbounded band: one 16-wavefront
                                     workgroup per extension, a shared
                                     4096-slot register window, then an LDS
                                     ring (global memory for bands over 8192
                                     cells)                                 */
    XDROP_STAGE_FINALIZE = 6,     /* result write-back                      */
    XDROP_NUM_STAGES = 7
};

#define XDROP_MAX_READ_LEN (1u << 24)
#define XDROP_MAX_X (1 << 30)

typedef struct {                  /* 32 bytes, little-endian, packed naturally */
    uint32_t read_a, read_b;      /* read ids in the store                  */
    uint32_t pos_a, pos_b;        /* seed start; pos_b in B's own (stored) coordinates */
    uint16_t k;                   /* seed length, >= 1                      */
    uint8_t strand;               /* 0: B as stored, 1: B reverse-complemented */
    uint8_t pad;
    int32_t x;                    /* drop, 0 <= x <= XDROP_MAX_X            */
    int16_t match, mismatch, gap; /* match >= 1, mismatch < match, gap <= -1;
                                     |weights| <= 1024 and
                                     (match - mismatch - gap) * (|A| + |B|) <= 2^29,
                                     which keeps every score inside int32 */
    int16_t pad2;
} xdrop_record;

typedef struct {                  /* 32 bytes */
    int32_t score;                /* left_score + seed_score + right_score  */
    int32_t left_score, right_score, seed_score;
    uint32_t a_begin, a_end;      /* aligned span [a_begin, a_end) of A     */
    uint32_t b_begin, b_end;      /* span of B' (the reverse-complement frame
                                     when strand = 1); in B's own frame it is
                                     [|B| - b_end, |B| - b_begin)            */
} xdrop_result;

typedef struct {
    uint64_t records;
    uint64_t cells;               /* candidate cells evaluated (left + right);
                                     only filled when cell counting was asked */
    double queue_ms;              /* submit entry -> admitted               */
    double device_ms;             /* first kernel start -> last kernel end  */
    double total_ms;              /* submit entry -> completion             */
    double stage_ms[XDROP_NUM_STAGES];      /* XDROP_FLAG_PROFILE only; summed over
                                               chunks in the plain form    */
    uint64_t stage_cells[XDROP_NUM_STAGES]; /* cells each stage computed for the
                                               extensions it completed or handed
                                               over with their state (cell counting,
                                               persistent form only); work lost to a
                                               restart is not counted      */
    uint64_t stage_tasks[XDROP_NUM_STAGES]; /* extensions each stage completed (idem) */
    uint64_t stage_slots[XDROP_NUM_STAGES]; /* window lane-steps of the same work
                                               (idem); stage_cells / stage_slots is
                                               the lane occupancy of the stage     */
} xdrop_batch_stats;

/* Create a context on cfg->device: packs the reads to 2 bits per base (both
 * orientations) and uploads them.  Returns XDROP_E_INVALID for a non-ACGT base,
 * an empty/oversized read or a bad field; *out is set only on XDROP_OK. */
xdrop_status xdrop_batch_create(const xdrop_config *cfg, xdrop_ctx **out);

/* Submit n host records.  The whole batch is validated first (bad read id,
 * seed outside a read, k = 0, x out of range, bad weights -> XDROP_E_INVALID,
 * nothing submitted).  recs is copied before return.  out (n results) and
 * cells (n uint64, nullable: per-record left+right cell counts) are written
 * when the batch completes and must stay valid until xdrop_batch_wait returns
 * XDROP_OK for the ticket.  admit_timeout_us: 0 -> XDROP_E_BUSY when no slot or
 * HBM budget is free; < 0 -> block until admitted; > 0 -> wait at most that
 * long, then XDROP_E_BUSY.  n = 0 is allowed (completes immediately). */
xdrop_status xdrop_batch_submit(xdrop_ctx *c, const xdrop_record *recs, size_t n,
                                xdrop_result *out, uint64_t *cells,
                                int64_t admit_timeout_us, xdrop_ticket *ticket);

/* Submit n records that already live in device memory of the context's GPU;
 * results (and cells, nullable) are written to device memory.  The work is
 * ordered on `stream` (a hipStream_t; NULL = the context's own stream).
 * Records are validated on the device: an invalid record makes the ticket's
 * wait return XDROP_E_INVALID and its result row is zero-filled.  Buffers
 * must stay valid until wait returns. */
xdrop_status xdrop_batch_submit_device(xdrop_ctx *c, const xdrop_record *d_recs, size_t n,
                                       xdrop_result *d_out, uint64_t *d_cells,
                                       void *stream, xdrop_ticket *ticket);

/* Wait for a ticket.  timeout_us < 0 waits forever, 0 polls.  On XDROP_OK the
 * ticket is consumed and stats (nullable) is filled.  XDROP_E_TIMEOUT leaves
 * the ticket outstanding. */
xdrop_status xdrop_batch_wait(xdrop_ctx *c, xdrop_ticket t, int64_t timeout_us,
                              xdrop_batch_stats *stats);

/* Drain outstanding batches, then free everything.  NULL is a no-op. */
xdrop_status xdrop_batch_destroy(xdrop_ctx *c);

typedef struct {
    int32_t grow_margin;          /* adaptive window: free slots per side after widening (>= 2) */
    int32_t shrink_margin;        /* adaptive window: narrow when the band fits C-1 cells
                                     per lane with this many free slots per side (>= 2) */
    int32_t waves_per_cu;         /* persistent grid: wavefronts per compute unit           */
    int32_t buckets;              /* 1: order extensions longest-first; 0: arrival order   */
    int32_t generic_waves;        /* grid of the unbounded-band kernel, in wavefronts: one
                                     workgroup of 16 per extension (multiple of 16)          */
    int32_t narrow_x;             /* persistent form: records with x <= narrow_x and weights
                                     match 1, gap -1, mismatch 0 / -1 / -2 run two extensions
                                     per wavefront (narrow stage); -1: off; at most 64        */
    int32_t narrow_min_records;   /* ... only in batches of at least this many records (>= 0):
                                     a smaller batch has too few such extensions to hide the
                                     narrow stage's tail                                      */
    int32_t wide_waves;           /* wavefronts per extension for bands of 1281-2048 cells: 1
                                     (32 cells per lane), 2 or 4 (a workgroup shares the
                                     window; other values are rounded down to these)          */
} xdrop_tuning;

/* Current launch parameters of a context. */
xdrop_status xdrop_get_tuning(const xdrop_ctx *c, xdrop_tuning *out);

/* Replace the launch parameters; only while no batch is in flight
 * (XDROP_E_BUSY otherwise).  Values are clamped to their valid ranges. */
xdrop_status xdrop_set_tuning(xdrop_ctx *c, const xdrop_tuning *t);

/* Autotuner: run the n host records (a representative sample, e.g. 10k-200k
 * records) under launch parameters chosen by coordinate descent -- each knob
 * (persistent grid size, length bucketing, adaptive window margins, grid of
 * the unbounded-band kernel, drop bound of the two-extensions-per-wavefront
 * narrow stage, wavefronts per extension of the 2048-slot stage) swept in
 * turn with the others at the best so far, two rounds, each setting timed by
 * the better of two runs after a warm-up -- keep the fastest by device time
 * and make it the context's tuning.  narrow_min_records is not swept (a
 * sample is one batch size).  Every setting gives the same results.  When
 * cache_path is non-NULL the choice is
 * written there (text, one "key value" per line) and later contexts created
 * with cfg->tuning_cache = cache_path start from it.  *best_ms (nullable)
 * gets the best device time.  Only while no batch is in flight. */
xdrop_status xdrop_autotune(xdrop_ctx *c, const xdrop_record *recs, size_t n, const char *cache_path,
                            double *best_ms);

/* Device bytes that admitting a batch of n records takes from the context's
 * HBM budget (buffers sized for the next power of two >= max(n, 1024),
 * including the unbounded kernel's scratch).  0 for a NULL context. */
uint64_t xdrop_batch_footprint(const xdrop_ctx *c, size_t n);

/* ---- Batches without allocation -----------------------------------------
 * For callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The same computation as
 * xdrop_batch_submit_device in the persistent form (same kernels and
 * results), but no call of the library allocates anything on its behalf:
 * every buffer a batch needs besides its records and results lives in one
 * array of XDROP_NOALLOC_BYTES of device memory that the library holds on
 * each GPU it is loaded on until the process ends.
 *   d_recs:    n records in device memory of the context's GPU (read only);
 *   d_out:     n results, device memory (written);
 *   d_cells:   nullable, n uint64 per-record cell counts (device memory);
 *   d_invalid: nullable, one uint32 in device memory: the number of invalid
 *              records (their result rows are zero-filled, as in
 *              xdrop_batch_submit_device);
 *   stream:    hipStream_t of the context's GPU the kernels are launched on
 *              (NULL: the null stream).
 * The call only enqueues work and returns: nothing is ready until the stream
 * reaches it, and there is no ticket or wait (no stats).  Every argument
 * buffer, and the context (its read store), must stay valid until then.
 * Errors: XDROP_E_INVALID for n > XDROP_NOALLOC_MAX_RECORDS, for reads so
 * long that one workgroup's scratch of the unbounded-band kernel does not
 * fit the array's share for it (reads over about 2 million bases), or a NULL
 * buffer with n > 0; XDROP_E_DEVICE when the array's device address cannot
 * be found or a launch fails.  All calls on one GPU share its array, and it
 * keeps the last call's contents: calls whose work overlaps on one GPU
 * (different streams, threads or contexts) race and give wrong results, so
 * order them on one stream or synchronize between them. */
#define XDROP_NOALLOC_BYTES (128ull << 20)
#define XDROP_NOALLOC_MAX_RECORDS (1u << 19)
xdrop_status xdrop_batch_run_noalloc(xdrop_ctx *c, const xdrop_record *d_recs, size_t n, xdrop_result *d_out,
                                     uint64_t *d_cells, uint32_t *d_invalid, void *stream);

/* ---- Seed discovery (the step before the batches) ------------------------
 * Records for the read pairs of the context's store that share a reliable
 * k-mer (paper, "Related works": BELLA detects overlaps from shared k-mers
 * after filtering unreliable ones, then extends the seeds with an X-drop;
 * "Method": k-mer length 31, stride 1, frequency window [20, 30] for the 29x
 * data set and [20, 50] for the 100x one):
 *   - each read contributes the k-mers starting at positions 0, s, 2s, ...;
 *   - a k-mer and its reverse complement are one k-mer, represented by the
 *     lexicographically smaller string (A < C < G < T);
 *   - its frequency is its number of occurrences over all reads and
 *     positions; it is reliable when lo <= frequency <= hi;
 *   - two different reads a < b sharing a reliable k-mer give one record:
 *     every pair of occurrences is a candidate seed (pos_a, pos_b, strand)
 *     with strand 1 when the two occurrences have opposite orientations, and
 *     the record takes the smallest candidate in (pos_a, pos_b, strand)
 *     order; positions are in the reads' stored coordinates, as everywhere
 *     in xdrop_record, so the seed is exact in A against B'.
 * k, x and the weights are copied into every record.  */
typedef struct {
    uint32_t k;                   /* 1..31                                    */
    uint32_t stride;              /* >= 1                                     */
    uint32_t lo, hi;              /* frequency window, 1 <= lo <= hi <= 4096  */
    int32_t x;                    /* X-drop of the records (0..2^30)          */
    int16_t match, mismatch, gap; /* weights of the records (record rules)    */
    int16_t pad;
} xdrop_seed_params;

typedef struct {
    uint64_t kmers;               /* k-mer occurrences counted                */
    uint64_t distinct;            /* distinct canonical k-mers                */
    uint64_t reliable;            /* canonical k-mers inside [lo, hi]         */
    uint64_t pairs;               /* read pairs found                         */
    double device_ms;             /* kernels, first to last                   */
} xdrop_seed_stats;

/* Find the seed records of the whole store.  out receives min(pairs,
 * max_records) records in unspecified order; it is host memory, or device
 * memory of the context's GPU when out_on_device != 0 (out may be NULL when
 * max_records = 0).  *n_found gets the number of pairs.  Returns
 * XDROP_E_INVALID for bad parameters, XDROP_E_NOMEM when out is too small
 * (*n_found then says how many records are needed; the records written are
 * a subset) or device memory runs out.  Scratch (about 16 B per k-mer plus
 * 8 B per occurrence slot of the reliable k-mers) is allocated per call,
 * outside the HBM budget of the batches, and freed before returning.  May
 * run concurrently with batches on the same context. */
xdrop_status xdrop_find_seeds(xdrop_ctx *c, const xdrop_seed_params *p, xdrop_record *out, size_t max_records,
                              int out_on_device, size_t *n_found, xdrop_seed_stats *stats);

/* Human-readable text of a status code (static storage). */
const char *xdrop_status_string(xdrop_status s);

/* Last error message recorded on the context (or globally when c is NULL).
 * The text is a copy owned by the calling thread, valid until that thread
 * calls xdrop_last_error again; safe while other threads record errors. */
const char *xdrop_last_error(const xdrop_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* XDROP_H */
