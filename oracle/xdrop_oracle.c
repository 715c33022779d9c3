/*
 * xdrop_oracle.c -- CPU oracle for batched X-drop seed-and-extend.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file: only tests/, the smoke check in __graft_entry__.py and the
 * cpu_baseline leg of bench.py use it.  It shares no code, header, table or
 * constant with the HIP path.
 *
 * What it computes (paper: "Related works", the BELLA and LOGAN paragraphs;
 * "Results", comparison of small and large data sets, where the aligner is
 * described as Needleman-Wunsch / Smith-Waterman with an X-drop):
 *
 *   A record is a pair of reads (A, B) with a shared seed of length k at
 *   A[pos_a..) and B'[pos_b'..), where B' is B or its reverse complement.
 *   The seed is scored position by position and extended to the left and to
 *   the right by an X-drop dynamic programme.  The paper fixes none of the
 *   details of the X-drop; the reading implemented here is:
 *
 *   Extension of a[1..m] against b[1..n] with weights match ma > 0,
 *   mismatch mi < ma, linear gap g < 0 and drop X >= 0.  Cell (i,j) sits on
 *   anti-diagonal d = i + j.
 *     - S(0,0) = 0 and it is live; T_0 = 0; best = (0,0).
 *     - For d = 1, 2, ..., m+n: a cell on d is a candidate when at least one
 *       of its predecessors (i-1,j-1) on d-2, (i-1,j) or (i,j-1) on d-1 is
 *       live.  Its value is the maximum over the live predecessors of
 *       S(i-1,j-1)+sigma(a_i,b_j), S(i-1,j)+g, S(i,j-1)+g (no zero floor).
 *       The candidate dies when its value is strictly below T_{d-1} - X,
 *       otherwise it is live.
 *     - T_d = max(T_{d-1}, largest live value on d).  When that strictly
 *       exceeds T_{d-1}, best becomes the live cell of d with the largest
 *       value and, among those, the smallest i.
 *     - Stop after two consecutive anti-diagonals without a live cell, or
 *       after d = m+n.
 *     - The result is (T, i*, j*, cells), cells being the number of
 *       candidate cells evaluated, live or dead.
 *
 * Every function is a plain, sequential transcription of that definition.
 * Integer arithmetic is done in int64_t; the library's int32 bounds are far
 * away.
 *
 * Build (done by the repository's build step):
 *   gcc -O2 -shared -fPIC -pthread oracle/xdrop_oracle.c -o oracle/liboracle.so
 *
 * OX_MUTATION (compile-time, default 0) plants a known mistake; it exists
 * only so that the test-suite can show that its pins catch such mistakes.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef OX_MUTATION
#define OX_MUTATION 0
#endif

#define OX_NEG (INT64_MIN / 4)

typedef struct {
    int64_t score;   /* T at the end of the extension            */
    int64_t i, j;    /* end cell (number of bases used of a, b)  */
    uint64_t cells;  /* candidate cells evaluated (live or dead) */
} ox_ext_t;

typedef struct {
    int64_t score, left, right, seed;
    int64_t a_begin, a_end, b_begin, b_end;  /* b span in the oriented frame B' */
    uint64_t cells_left, cells_right;
} ox_rec_t;

static int64_t ox_max(int64_t x, int64_t y) { return x > y ? x : y; }
static int64_t ox_min(int64_t x, int64_t y) { return x < y ? x : y; }

static int64_t ox_sigma(uint8_t x, uint8_t y, int64_t ma, int64_t mi)
{
#if OX_MUTATION == 6
    (void)x; (void)y;
    return ma; /* planted: every pair scored as a match */
#else
    return x == y ? ma : mi;
#endif
}

/* ------------------------------------------------------------------------ */
/* X-drop extension, live-range form.  Three anti-diagonals are kept, indexed */
/* by i; for each one the range [lo, hi] of its live cells is remembered and  */
/* any lookup outside that range reads as "not live".  Only cells that can   */
/* have a live predecessor are visited.                                      */
/* ------------------------------------------------------------------------ */
/* max_width (nullable): the widest live range hi - lo + 1 over all
   anti-diagonals, written when non-NULL (an observation of the run; it
   changes nothing in it). */
static int ox_extend_core(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                          int64_t ma, int64_t mi, int64_t g, int64_t X, ox_ext_t *out,
                          int64_t *max_width)
{
    if (max_width) *max_width = 1;   /* anti-diagonal 0: (0,0) */
    int64_t *buf[3];
    for (int t = 0; t < 3; ++t) {
        buf[t] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 2));
        if (!buf[t]) {
            for (int u = 0; u < t; ++u) free(buf[u]);
            return -1;
        }
    }
    int64_t *P2 = buf[0], *P1 = buf[1], *P0 = buf[2];
    int64_t lo2 = 1, hi2 = 0;   /* diagonal -1: empty           */
    int64_t lo1 = 0, hi1 = 0;   /* diagonal 0: only (0,0), live */
    P1[0] = 0;
    int64_t T = 0, bi = 0, bj = 0;
    uint64_t cells = 0;
    int prev_dead = 0;

    for (int64_t d = 1; d <= m + n; ++d) {
        const int64_t ilo = ox_max(0, d - n), ihi = ox_min(m, d);
        int64_t slo = INT64_MAX, shi = INT64_MIN;
        if (lo1 <= hi1) { slo = ox_min(slo, lo1); shi = ox_max(shi, hi1 + 1); }
#if OX_MUTATION != 1
        if (lo2 <= hi2) { slo = ox_min(slo, lo2 + 1); shi = ox_max(shi, hi2 + 1); }
#endif
        slo = ox_max(slo, ilo);
        shi = ox_min(shi, ihi);

        int64_t nlo = 1, nhi = 0, dmax = OX_NEG, dmi = -1;
        for (int64_t i = slo; i <= shi; ++i) {
            const int64_t j = d - i;
            int cand = 0;
            int64_t v = OX_NEG;
            if (i >= 1 && j >= 1 && i - 1 >= lo2 && i - 1 <= hi2 && P2[i - 1] != OX_NEG) {
                v = ox_max(v, P2[i - 1] + ox_sigma(a[i - 1], b[j - 1], ma, mi));
                cand = 1;
            }
            if (i >= 1 && i - 1 >= lo1 && i - 1 <= hi1 && P1[i - 1] != OX_NEG) {
                v = ox_max(v, P1[i - 1] + g);          /* from (i-1, j) */
                cand = 1;
            }
            if (j >= 1 && i >= lo1 && i <= hi1 && P1[i] != OX_NEG) {
                v = ox_max(v, P1[i] + g);              /* from (i, j-1) */
                cand = 1;
            }
            if (!cand) { P0[i] = OX_NEG; continue; }
            ++cells;
#if OX_MUTATION == 2
            if (v <= T - X) { P0[i] = OX_NEG; continue; }   /* planted: non-strict drop test */
#elif OX_MUTATION == 4
            if (v < ox_max(T, dmax) - X) { P0[i] = OX_NEG; continue; } /* planted: threshold updated inside d */
#else
            if (v < T - X) { P0[i] = OX_NEG; continue; }
#endif
            P0[i] = v;
            if (nlo > nhi) nlo = i;
            nhi = i;
#if OX_MUTATION == 5
            if (v >= dmax) { dmax = v; dmi = i; }    /* planted: largest i wins ties */
#else
            if (v > dmax) { dmax = v; dmi = i; }
#endif
        }
        const int live = nlo <= nhi;
        if (max_width && live && nhi - nlo + 1 > *max_width) *max_width = nhi - nlo + 1;
#if OX_MUTATION == 7
        if (live && dmax >= T) { T = dmax; bi = dmi; bj = d - dmi; } /* planted: later diagonal wins ties */
#else
        if (live && dmax > T) { T = dmax; bi = dmi; bj = d - dmi; }
#endif
        int64_t *t = P2; P2 = P1; P1 = P0; P0 = t;
        lo2 = lo1; hi2 = hi1; lo1 = nlo; hi1 = nhi;
#if OX_MUTATION == 3
        if (!live) break;                               /* planted: stop at first dead diagonal */
#else
        if (!live && prev_dead) break;
#endif
        prev_dead = !live;
    }
    out->score = T; out->i = bi; out->j = bj; out->cells = cells;
    for (int u = 0; u < 3; ++u) free(buf[u]);
    return 0;
}

int ox_extend(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
              int64_t ma, int64_t mi, int64_t g, int64_t X, ox_ext_t *out)
{
    return ox_extend_core(a, m, b, n, ma, mi, g, X, out, NULL);
}

/* The same extension, also reporting the widest live range of an
   anti-diagonal (used by tests to predict which band widths a run meets). */
int ox_extend_band(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                   int64_t ma, int64_t mi, int64_t g, int64_t X, ox_ext_t *out,
                   int64_t *max_width)
{
    return ox_extend_core(a, m, b, n, ma, mi, g, X, out, max_width);
}

/* ------------------------------------------------------------------------ */
/* The same definition over the whole (m+1) x (n+1) table: every cell of    */
/* every anti-diagonal is visited and its predecessors are looked up in the */
/* table; there is no range bookkeeping at all.  O(mn) time and memory, for  */
/* small inputs only.                                                        */
/* ------------------------------------------------------------------------ */
int ox_extend_dense(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                    int64_t ma, int64_t mi, int64_t g, int64_t X, ox_ext_t *out)
{
    const int64_t W = n + 1;
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)((m + 1) * W));
    uint8_t *L = (uint8_t *)calloc((size_t)((m + 1) * W), 1);
    if (!S || !L) { free(S); free(L); return -1; }
    S[0] = 0; L[0] = 1;
    int64_t T = 0, bi = 0, bj = 0;
    uint64_t cells = 0;
    int prev_dead = 0;
    for (int64_t d = 1; d <= m + n; ++d) {
        int any = 0;
        int64_t dmax = OX_NEG, dmi = -1;
        for (int64_t i = ox_max(0, d - n); i <= ox_min(m, d); ++i) {
            const int64_t j = d - i;
            int cand = 0;
            int64_t v = OX_NEG;
            if (i >= 1 && j >= 1 && L[(i - 1) * W + (j - 1)]) {
                v = ox_max(v, S[(i - 1) * W + (j - 1)] + (a[i - 1] == b[j - 1] ? ma : mi));
                cand = 1;
            }
            if (i >= 1 && L[(i - 1) * W + j]) { v = ox_max(v, S[(i - 1) * W + j] + g); cand = 1; }
            if (j >= 1 && L[i * W + (j - 1)]) { v = ox_max(v, S[i * W + (j - 1)] + g); cand = 1; }
            if (!cand) continue;
            ++cells;
            if (v < T - X) continue;
            S[i * W + j] = v;
            L[i * W + j] = 1;
            any = 1;
            if (v > dmax) { dmax = v; dmi = i; }
        }
        if (any && dmax > T) { T = dmax; bi = dmi; bj = d - dmi; }
        if (!any && prev_dead) break;
        prev_dead = !any;
    }
    out->score = T; out->i = bi; out->j = bj; out->cells = cells;
    free(S); free(L);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Full Needleman-Wunsch prefix table with no drop at all, filled row by    */
/* row: H(i,j) is the best score of an alignment of a[1..i] with b[1..j].    */
/* Returns the maximum over the table, ties broken by the smallest i+j and  */
/* then the smallest i.  This is the result an X-drop extension must reach  */
/* when X is so large that nothing is ever dropped.                         */
/* ------------------------------------------------------------------------ */
int ox_nw_best(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
               int64_t ma, int64_t mi, int64_t g, ox_ext_t *out)
{
    const int64_t W = n + 1;
    int64_t *H = (int64_t *)malloc(sizeof(int64_t) * (size_t)((m + 1) * W));
    if (!H) return -1;
    int64_t best = 0, bi = 0, bj = 0;
    for (int64_t i = 0; i <= m; ++i) {
        for (int64_t j = 0; j <= n; ++j) {
            int64_t h;
            if (i == 0 && j == 0) h = 0;
            else if (i == 0) h = H[j - 1] + g;
            else if (j == 0) h = H[(i - 1) * W] + g;
            else {
                const int64_t s = a[i - 1] == b[j - 1] ? ma : mi;
                h = H[(i - 1) * W + (j - 1)] + s;
                h = ox_max(h, H[(i - 1) * W + j] + g);
                h = ox_max(h, H[i * W + (j - 1)] + g);
            }
            H[i * W + j] = h;
            if (h > best || (h == best && (i + j < bi + bj || (i + j == bi + bj && i < bi)))) {
                best = h; bi = i; bj = j;
            }
        }
    }
    out->score = best; out->i = bi; out->j = bj;
    out->cells = (uint64_t)((m + 1) * (n + 1) - 1);
    free(H);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Record level: orientation, seed score, left and right extension.          */
/* Bases are codes A=0, C=1, G=2, T=3; the complement of x is 3-x.            */
/* ------------------------------------------------------------------------ */
int ox_record(const uint8_t *A, int64_t la, const uint8_t *B, int64_t lb,
              int64_t pos_a, int64_t pos_b, int64_t k, int strand,
              int64_t X, int64_t ma, int64_t mi, int64_t g, ox_rec_t *out)
{
    if (k < 1 || pos_a < 0 || pos_b < 0 || pos_a + k > la || pos_b + k > lb) return -2;
    /* B' = B for strand '+', reverse complement of B for strand '-';
       pos_b is given in B's own coordinates. */
    uint8_t *Bp = (uint8_t *)malloc((size_t)lb + 1);
    uint8_t *ra = (uint8_t *)malloc((size_t)la + 1);
    uint8_t *rb = (uint8_t *)malloc((size_t)lb + 1);
    if (!Bp || !ra || !rb) { free(Bp); free(ra); free(rb); return -1; }
    int64_t pb;
    if (strand) {
        for (int64_t t = 0; t < lb; ++t) Bp[t] = (uint8_t)(3 - B[lb - 1 - t]);
        pb = lb - pos_b - k;
    } else {
        memcpy(Bp, B, (size_t)lb);
        pb = pos_b;
    }
    int64_t seed = 0;
    for (int64_t t = 0; t < k; ++t) seed += ox_sigma(A[pos_a + t], Bp[pb + t], ma, mi);

    /* left: both prefixes read backwards from the seed */
    for (int64_t t = 0; t < pos_a; ++t) ra[t] = A[pos_a - 1 - t];
    for (int64_t t = 0; t < pb; ++t) rb[t] = Bp[pb - 1 - t];
    ox_ext_t L, R;
    int rc = ox_extend(ra, pos_a, rb, pb, ma, mi, g, X, &L);
    if (rc == 0)
        rc = ox_extend(A + pos_a + k, la - pos_a - k, Bp + pb + k, lb - pb - k, ma, mi, g, X, &R);
    if (rc == 0) {
        out->left = L.score; out->right = R.score; out->seed = seed;
        out->score = L.score + seed + R.score;
        out->a_begin = pos_a - L.i; out->a_end = pos_a + k + R.i;
        out->b_begin = pb - L.j;    out->b_end = pb + k + R.j;
        out->cells_left = L.cells; out->cells_right = R.cells;
    }
    free(Bp); free(ra); free(rb);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Many records over a pool of threads; each record is computed by one      */
/* thread with ox_record.  Reads are given as one concatenated code buffer    */
/* with per-read offsets and lengths; records as separate field arrays.      */
/* ------------------------------------------------------------------------ */
typedef struct {
    const uint8_t *codes; const int64_t *roff; const int64_t *rlen;
    const int64_t *ra, *rb, *pa, *pbv, *kk, *st, *xx, *wma, *wmi, *wg;
    int64_t n;
    ox_rec_t *out;
    int *status;
    int64_t next;
    pthread_mutex_t mu;
} ox_batch_job;

static void *ox_batch_worker(void *arg)
{
    ox_batch_job *J = (ox_batch_job *)arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        const int64_t s = J->next;
        J->next += 16;
        pthread_mutex_unlock(&J->mu);
        if (s >= J->n) break;
        const int64_t e = ox_min(J->n, s + 16);
        for (int64_t r = s; r < e; ++r) {
            const int64_t a = J->ra[r], b = J->rb[r];
            J->status[r] = ox_record(J->codes + J->roff[a], J->rlen[a], J->codes + J->roff[b], J->rlen[b],
                                     J->pa[r], J->pbv[r], J->kk[r], (int)J->st[r], J->xx[r],
                                     J->wma[r], J->wmi[r], J->wg[r], &J->out[r]);
        }
    }
    return NULL;
}

int ox_batch(const uint8_t *codes, const int64_t *roff, const int64_t *rlen,
             const int64_t *read_a, const int64_t *read_b, const int64_t *pos_a,
             const int64_t *pos_b, const int64_t *k, const int64_t *strand,
             const int64_t *x, const int64_t *ma, const int64_t *mi, const int64_t *g,
             int64_t n, int nthreads, ox_rec_t *out, int *status)
{
    ox_batch_job J = {codes, roff, rlen, read_a, read_b, pos_a, pos_b, k, strand, x, ma, mi, g,
                      n, out, status, 0, PTHREAD_MUTEX_INITIALIZER};
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    if (!th) return -1;
    int started = 0;
    for (int t = 0; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, ox_batch_worker, &J) == 0) ++started;
    if (started == 0) ox_batch_worker(&J);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    free(th);
    return started == 0 ? 1 : started;
}

int ox_mutation(void) { return OX_MUTATION; }
