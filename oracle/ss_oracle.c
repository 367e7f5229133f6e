/*
 * SneakySnake CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the slow, obviously-correct reference against which the GPU
 * filter is checked.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  The GPU library never links, loads or
 * calls anything here, and nothing here is shared with the GPU path.
 *
 * What it computes (Alser et al., "SneakySnake: a fast and accurate universal
 * genome pre-alignment filter for CPUs, GPUs and FPGAs"):
 *   - the chip maze Z of Section 2.3, one cell at a time, exactly as the four
 *     cases of Equation 1 (rows i = 1..2E+1, columns j = 1..m, 1-based);
 *   - the greedy SneakySnake walk of Section 2.4, steps (1)-(5), evaluating the
 *     maze implicitly: a row is examined from the checkpoint only up to its
 *     first obstacle (the "implicit chip maze" paragraph of Section 2.4);
 *   - Snake-on-Chip's decomposition (Section 2.5): the same walk run on
 *     non-overlapping sub-mazes of t columns, the counts summed;
 *   - pairs of unequal length (the note of Section 2.4 between steps 4 and 5):
 *     the maze over the longer length, the walk, and the deduction of the
 *     leading and trailing obstacles caused by the fourth case of Equation 1
 *     (the reading is stated at ss_oracle_pair_uneq);
 *   - two checkers used to pin the walk:
 *       * the minimum number of obstacles over every legal signal net, by an
 *         exhaustive dynamic programme over checkpoints (the quantity that
 *         Theorem 2 says the greedy walk reaches);
 *       * the Levenshtein edit distance by the textbook full DP (Section 1
 *         defines the filter as a lower bound on it, Section 2.1).
 *
 * Sequence roles: R is the reference (its positions index the maze columns),
 * Q is the query (read).  Bytes are case-folded; the oracle compares bytes and
 * does not validate the alphabet.
 *
 * Readings taken where the paper is silent:
 *   - a cell whose Q index falls outside 1..m is an obstacle (Eq. 1 "otherwise");
 *   - a row that reaches column m without an obstacle ends the walk without
 *     counting; an obstacle exactly at column m is counted;
 *   - when every row starts with an obstacle the escape segment is that single
 *     obstacle (Section 2.4, step 2);
 *   - the walk stops as soon as the count exceeds E, so a rejected pair reports
 *     E+1 (step 4); accept iff count <= E (steps 4-5).
 *
 * Built with plain gcc -O2; no intrinsics, no bit tricks.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <time.h>

typedef struct {
    int64_t checkpoints;   /* iterations of steps 2-3 */
    int64_t c_last;        /* last column reached by the walk, clipped to m */
    int64_t cells;         /* maze cells evaluated by the implicit walk */
} ss_oracle_stats;

static uint8_t fold(uint8_t c) { return (c >= 'a' && c <= 'z') ? (uint8_t)(c - 'a' + 'A') : c; }

/* Equation 1 (Section 2.3).  i in 1..2E+1, j in 1..m, both 1-based.
 *   i = E+1      : compare R[j] with Q[j]              (matches / substitutions)
 *   1 <= i <= E  : compare R[j] with Q[j-i]            (deletions in Q)
 *   i > E+1      : compare R[j] with Q[j+i-E-1]        (insertions in Q)
 *   otherwise    : 1 (obstacle), which includes a Q index outside 1..m.
 * Returns 0 for a match (free path) and 1 for an obstacle. */
int ss_oracle_cell(const uint8_t* R, const uint8_t* Q, int m, int E, int i, int j)
{
    int q;
    if (j < 1 || j > m || i < 1 || i > 2 * E + 1) return 1;
    if (i == E + 1)      q = j;
    else if (i <= E)     q = j - i;
    else                 q = j + i - E - 1;
    if (q < 1 || q > m) return 1;
    return fold(Q[q - 1]) == fold(R[j - 1]) ? 0 : 1;
}

/* Length of the run of zeros of row i starting at column c (1-based): the
 * number of consecutive free cells from the checkpoint up to, not including,
 * the first obstacle or the end of the row.  Cells are computed one by one. */
static int run_from(const uint8_t* R, const uint8_t* Q, int m, int E, int i, int c, int64_t* cells)
{
    int L = 0;
    while (c + L <= m) {
        if (cells) (*cells)++;
        if (ss_oracle_cell(R, Q, m, E, i, c + L) != 0) break;
        L++;
    }
    return L;
}

/* The greedy walk of Section 2.4.  Returns 1 (accept: alignment needed) or 0
 * (reject: edit distance guaranteed > E).  *edits receives the number of
 * obstacles on the net found; with stop_early the walk halts as soon as that
 * number exceeds E (step 4), so rejected pairs report E+1.  With stop_early=0
 * the walk runs to the last column and reports the full count.
 * seg_rows/seg_ends (optional, capacity cap) record each escape segment's row
 * (lowest row index among equally long runs) and end column, for inspection. */
int ss_oracle_pair_ex(const uint8_t* R, const uint8_t* Q, int m, int E, int stop_early,
                      int32_t* edits, ss_oracle_stats* st,
                      int32_t* seg_rows, int32_t* seg_ends, int cap, int32_t* nseg)
{
    int c = 1;               /* step 1: the first column is the first checkpoint */
    int n = 0;
    int64_t cps = 0, cells = 0;
    int segs = 0;
    while (c <= m) {                                   /* until the destination ... */
        int best = -1, best_row = 0;
        for (int i = 1; i <= 2 * E + 1; i++) {         /* step 2: longest run over all rows */
            int L = run_from(R, Q, m, E, i, c, &cells);
            if (L > best) { best = L; best_row = i; }
        }
        cps++;
        /* the escape segment is that run plus its first following obstacle;
         * a run that reaches the end of the row has no obstacle to count */
        int end = c + best;
        if (end <= m) n++;
        if (seg_rows && segs < cap) { seg_rows[segs] = best_row; seg_ends[segs] = end <= m ? end : m; }
        segs++;
        c = end + 1;                                   /* step 3: new checkpoint */
        if (stop_early && n > E) break;                /* ... or the delay exceeds E obstacles */
    }
    if (edits) *edits = n;
    if (nseg) *nseg = segs;
    if (st) {
        st->checkpoints = cps;
        st->c_last = (c - 1 < m) ? (c - 1) : m;
        st->cells = cells;
    }
    return n <= E ? 1 : 0;                             /* step 5 */
}

int ss_oracle_pair(const uint8_t* R, const uint8_t* Q, int m, int E, int32_t* edits, ss_oracle_stats* st)
{
    return ss_oracle_pair_ex(R, Q, m, E, 1, edits, st, NULL, NULL, 0, NULL);
}

/* Snake-on-Chip's decomposition (Section 2.5): the maze is cut into
 * non-overlapping sub-mazes of t consecutive columns (the last one may be
 * narrower) and 2E+1 rows; each is solved on its own by the greedy walk of
 * Section 2.4, whose first checkpoint is the sub-maze's first column and whose
 * destination is its last column (a run reaching it counts no obstacle).
 * Cells keep their Equation 1 values at their global positions.  The count is
 * the sum over the sub-mazes; with stop_early the walk stops once the sum
 * exceeds E (rejected pairs report E+1).  The paper's per-module limit (y
 * instances per sub-maze) is a hardware parameter described in its missing
 * supplement and is not modelled: every sub-maze is solved completely.
 * Returns 1 for accept (sum <= E). */
static int run_within(const uint8_t* R, const uint8_t* Q, int m, int E, int i, int c, int last)
{
    int L = 0;
    while (c + L <= last && ss_oracle_cell(R, Q, m, E, i, c + L) == 0) L++;
    return L;
}

int ss_oracle_submaze(const uint8_t* R, const uint8_t* Q, int m, int E, int t, int stop_early, int32_t* edits)
{
    int sum = 0;                                           /* obstacles over all sub-mazes */
    if (t < 1) t = 1;
    for (int first = 1; first <= m && !(stop_early && sum > E); first += t) {
        const int last = first + t - 1 < m ? first + t - 1 : m;
        int c = first;                                     /* the sub-maze's first checkpoint */
        while (c <= last) {
            int best = -1;
            for (int i = 1; i <= 2 * E + 1; i++) {
                int L = run_within(R, Q, m, E, i, c, last);
                if (L > best) best = L;
            }
            int end = c + best;
            if (end <= last) sum++;                        /* the segment's obstacle */
            c = end + 1;
            if (stop_early && E < sum) break;             /* the sum exceeds E */
        }
    }
    if (edits) *edits = sum;
    return sum <= E;
}

/* ss_oracle_submaze over a batch (pair i: reads/refs at offsets[i], lengths[i]). */
void ss_oracle_submaze_batch(const uint8_t* reads, const uint8_t* refs, const int64_t* offsets, const int32_t* lengths,
                             int64_t n, int E, int t, uint8_t* accept, int32_t* edits)
{
    for (int64_t i = 0; i < n; i++)
        accept[i] = (uint8_t)ss_oracle_submaze(refs + offsets[i], reads + offsets[i], lengths[i], E, t, 1, &edits[i]);
}

/* Minimum number of obstacles over all legal signal nets (Section 2.2 rules on
 * the maze of Section 2.3), by exhaustive search over checkpoints; this is the
 * optimum that Theorem 2 claims the greedy walk attains.  A net is a sequence
 * of escape segments: from a checkpoint c a segment follows one row through its
 * free cells up to that row's first obstacle, passes it (cost 1) and the next
 * segment starts at the following column, on any row; a segment whose row is
 * free up to column m reaches the destination at no cost.
 * best[c] = fewest obstacles paid to stand at checkpoint c (1-based). */
int ss_oracle_min_obstacles(const uint8_t* R, const uint8_t* Q, int m, int E)
{
    if (m <= 0) return 0;
    int* best = (int*)malloc(sizeof(int) * (size_t)(m + 2));
    const int INF = 1 << 29;
    for (int c = 0; c <= m + 1; c++) best[c] = INF;
    best[1] = 0;
    int answer = INF;
    for (int c = 1; c <= m; c++) {
        if (best[c] >= INF) continue;
        for (int i = 1; i <= 2 * E + 1; i++) {
            int L = run_from(R, Q, m, E, i, c, NULL);
            int end = c + L;
            if (end > m) {                      /* free to the destination */
                if (best[c] < answer) answer = best[c];
            } else {
                int nxt = end + 1;              /* pass the obstacle at column end */
                int cost = best[c] + 1;
                if (nxt > m) { if (cost < answer) answer = cost; }
                else if (cost < best[nxt]) best[nxt] = cost;
            }
        }
    }
    free(best);
    return answer;
}

/* Levenshtein distance (unit-cost substitution, insertion, deletion) by the
 * textbook O(la*lb) dynamic programme over prefixes. */
int ss_oracle_levenshtein(const uint8_t* a, int la, const uint8_t* b, int lb)
{
    int* prev = (int*)malloc(sizeof(int) * (size_t)(lb + 1));
    int* cur = (int*)malloc(sizeof(int) * (size_t)(lb + 1));
    for (int y = 0; y <= lb; y++) prev[y] = y;
    for (int x = 1; x <= la; x++) {
        cur[0] = x;
        for (int y = 1; y <= lb; y++) {
            int sub = prev[y - 1] + (fold(a[x - 1]) == fold(b[y - 1]) ? 0 : 1);
            int del = prev[y] + 1;
            int ins = cur[y - 1] + 1;
            int v = sub < del ? sub : del;
            cur[y] = v < ins ? v : ins;
        }
        int* t = prev; prev = cur; cur = t;
    }
    int d = prev[lb];
    free(prev); free(cur);
    return d;
}

/* ---- pairs of unequal length (Section 2.4, the note between steps 4 and 5) ----
 *
 * Reading taken here (the paper gives the rule in one sentence and no
 * example):
 *   - R has m characters, Q has n.  The maze has 2E+1 rows and as many columns
 *     as the longer sequence, W = max(m, n); columns index R as in Equation 1.
 *     A cell whose comparison needs a character that does not exist (a column
 *     past the end of R, or a Q index outside 1..n) is an obstacle: the fourth
 *     case of Equation 1.  For m = n this is exactly the maze of ss_oracle_cell.
 *   - The walk of steps 1-4 runs over the W columns unchanged, to the
 *     destination (the deduction needs the whole net).
 *   - The obstacles "caused by the fourth case" are those lying in a column
 *     that holds no comparison between two existing characters: every one of
 *     its 2E+1 cells is a fourth-case cell, so the column carries no evidence of
 *     a difference.  The leading ones (a run of such obstacles at the start of
 *     the net) and the trailing ones (a run at its end) are deducted from the
 *     count before the decision, which is then taken as in step 5.
 *   - The count bounds the (global) edit distance between R and Q, the
 *     distance Section 1 defines.  Columns with a real comparison are
 *     1..min(m, n + E) when n >= 1 and none when n = 0, so for m = n nothing is
 *     deducted.
 * Returns 1 for accept; *edits = min(count after the deduction, E+1); *full
 * and *net_out (optional) = the count before and after the deduction. */
static int cell_uneq(const uint8_t* R, int m, const uint8_t* Q, int n, int E, int i, int j)
{
    if (i < 1 || i > 2 * E + 1) return 1;  /* no such row */
    if (j < 1 || j > m) return 1;          /* R has no j-th character */
    /* the Q index row i compares with R[j]: rows 1..E look back, row E+1 on the
     * diagonal, rows E+2..2E+1 ahead (Equation 1) */
    const int q = (i <= E) ? j - i : ((i == E + 1) ? j : j + i - (E + 1));
    if (q < 1 || q > n) return 1;          /* Q has no q-th character */
    return fold(R[j - 1]) != fold(Q[q - 1]);
}

/* 1 when some row of column j compares two existing characters */
static int real_column(int m, int n, int E, int j)
{
    for (int i = 1; i <= 2 * E + 1; i++) {
        int q = (i == E + 1) ? j : (i <= E ? j - i : j + i - E - 1);
        if (j >= 1 && j <= m && q >= 1 && q <= n) return 1;
    }
    return 0;
}

int ss_oracle_pair_uneq(const uint8_t* R, int m, const uint8_t* Q, int n, int E, int32_t* edits, int32_t* full,
                        int32_t* net_out)
{
    const int W = m > n ? m : n;
    int* obst = (int*)malloc(sizeof(int) * (size_t)(W + 1));
    int cnt = 0;
    int c = 1;                                         /* step 1 */
    while (c <= W) {                                   /* until the destination */
        int best = -1;
        for (int i = 1; i <= 2 * E + 1; i++) {         /* step 2: longest run over all rows */
            int L = 0;
            while (c + L <= W && cell_uneq(R, m, Q, n, E, i, c + L) == 0) L++;
            if (L > best) best = L;
        }
        int end = c + best;
        if (end <= W) obst[cnt++] = end;               /* the segment's obstacle */
        c = end + 1;                /* step 3: the next checkpoint */
    }
    int lead = 0;
    while (lead < cnt && !real_column(m, n, E, obst[lead])) lead++;
    int trail = 0;
    while (trail < cnt - lead && !real_column(m, n, E, obst[cnt - 1 - trail])) trail++;
    free(obst);
    const int net = cnt - lead - trail;
    if (full) *full = cnt;
    if (net_out) *net_out = net;
    if (edits) *edits = net <= E ? net : E + 1;
    return net <= E ? 1 : 0;                           /* step 5 */
}

/* The fewest obstacles outside fourth-case-only columns over every legal
 * signal net of the W-column maze above (exhaustive search over checkpoints,
 * as ss_oracle_min_obstacles; an obstacle in a column without a real
 * comparison costs nothing). */
int ss_oracle_min_obstacles_uneq(const uint8_t* R, int m, const uint8_t* Q, int n, int E)
{
    const int W = m > n ? m : n;
    if (W <= 0) return 0;
    int* best = (int*)malloc(sizeof(int) * (size_t)(W + 2));
    const int INF = 1 << 29;
    for (int c = 0; c <= W + 1; c++) best[c] = INF;
    best[1] = 0;
    int answer = INF;
    for (int c = 1; c <= W; c++) {
        if (best[c] >= INF) continue;
        for (int i = 1; i <= 2 * E + 1; i++) {
            int L = 0;
            while (c + L <= W && cell_uneq(R, m, Q, n, E, i, c + L) == 0) L++;
            int end = c + L;
            if (end > W) {
                if (best[c] < answer) answer = best[c];
            } else {
                int cost = best[c] + real_column(m, n, E, end);
                int nxt = end + 1;
                if (nxt > W) { if (cost < answer) answer = cost; }
                else if (cost < best[nxt]) best[nxt] = cost;
            }
        }
    }
    free(best);
    return answer;
}

/* Unequal-length batch: query p at reads[read_off[p] .. + read_len[p]),
 * reference p at refs[ref_off[p] .. + ref_len[p]).  Single thread per slice. */
typedef struct {
    const uint8_t* reads; const int64_t* read_off; const int32_t* read_len;
    const uint8_t* refs; const int64_t* ref_off; const int32_t* ref_len;
    const int32_t* E_per_pair; int32_t E; int64_t lo, hi;
    uint8_t* accept; int32_t* edits;
} uneq_job;

static void* uneq_worker(void* arg)
{
    uneq_job* J = (uneq_job*)arg;
    for (int64_t p = J->lo; p < J->hi; p++) {
        int E = J->E_per_pair ? J->E_per_pair[p] : J->E;
        int32_t e = 0;
        int acc = ss_oracle_pair_uneq(J->refs + J->ref_off[p], J->ref_len[p], J->reads + J->read_off[p],
                                      J->read_len[p], E, &e, NULL, NULL);
        J->accept[p] = (uint8_t)acc;
        J->edits[p] = e;
    }
    return NULL;
}

double ss_oracle_batch_uneq(const uint8_t* reads, const int64_t* read_off, const int32_t* read_len,
                            const uint8_t* refs, const int64_t* ref_off, const int32_t* ref_len, int64_t n,
                            const int32_t* E_per_pair, int32_t E, int threads, uint8_t* accept, int32_t* edits)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if ((int64_t)threads > n) threads = n > 0 ? (int)n : 1;
    uneq_job jobs[256];
    pthread_t tid[256];
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int t = 0; t < threads; t++) {
        uneq_job* J = &jobs[t];
        J->reads = reads; J->read_off = read_off; J->read_len = read_len;
        J->refs = refs; J->ref_off = ref_off; J->ref_len = ref_len;
        J->E_per_pair = E_per_pair; J->E = E;
        J->lo = n * t / threads; J->hi = n * (t + 1) / threads;
        J->accept = accept; J->edits = edits;
    }
    if (threads == 1) uneq_worker(&jobs[0]);
    else {
        for (int t = 0; t < threads; t++) pthread_create(&tid[t], NULL, uneq_worker, &jobs[t]);
        for (int t = 0; t < threads; t++) pthread_join(tid[t], NULL);
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    return (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
}

/* ---- batch drivers (contiguous slices, one plain thread each) ---------- */

typedef struct {
    const uint8_t* reads; const uint8_t* refs;
    const int64_t* offsets; const int32_t* lengths;
    const int32_t* E_per_pair; int32_t E;
    int64_t lo, hi;
    uint8_t* accept; int32_t* edits; int64_t* stats;   /* stats: 3 per pair, may be NULL */
    int stop_early;
} batch_job;

static void* batch_worker(void* arg)
{
    batch_job* J = (batch_job*)arg;
    for (int64_t p = J->lo; p < J->hi; p++) {
        int m = J->lengths[p];
        int E = J->E_per_pair ? J->E_per_pair[p] : J->E;
        const uint8_t* Q = J->reads + J->offsets[p];
        const uint8_t* R = J->refs + J->offsets[p];
        int32_t e = 0;
        ss_oracle_stats st;
        int acc = ss_oracle_pair_ex(R, Q, m, E, J->stop_early, &e, &st, NULL, NULL, 0, NULL);
        if (J->accept) J->accept[p] = (uint8_t)acc;
        if (J->edits) J->edits[p] = e;
        if (J->stats) {
            J->stats[3 * p + 0] = st.checkpoints;
            J->stats[3 * p + 1] = st.c_last;
            J->stats[3 * p + 2] = st.cells;
        }
    }
    return NULL;
}

/* reads (queries) and refs are concatenated; pair p occupies
 * [offsets[p], offsets[p]+lengths[p]) in both.  E_per_pair may be NULL, in
 * which case E applies to every pair.  Returns the wall time in seconds of
 * the filtering loop only. */
double ss_oracle_batch(const uint8_t* reads, const uint8_t* refs, const int64_t* offsets,
                       const int32_t* lengths, int64_t n, const int32_t* E_per_pair, int32_t E,
                       int threads, int stop_early, uint8_t* accept, int32_t* edits, int64_t* stats)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if ((int64_t)threads > n) threads = n > 0 ? (int)n : 1;
    batch_job jobs[256];
    pthread_t tid[256];
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int t = 0; t < threads; t++) {
        batch_job* J = &jobs[t];
        J->reads = reads; J->refs = refs; J->offsets = offsets; J->lengths = lengths;
        J->E_per_pair = E_per_pair; J->E = E;
        J->lo = n * t / threads; J->hi = n * (t + 1) / threads;
        J->accept = accept; J->edits = edits; J->stats = stats; J->stop_early = stop_early;
    }
    if (threads == 1) batch_worker(&jobs[0]);
    else {
        for (int t = 0; t < threads; t++) pthread_create(&tid[t], NULL, batch_worker, &jobs[t]);
        for (int t = 0; t < threads; t++) pthread_join(tid[t], NULL);
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    return (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
}

/* Batch versions of the two checkers, same pair layout, single thread. */
void ss_oracle_min_obstacles_batch(const uint8_t* reads, const uint8_t* refs, const int64_t* offsets,
                                   const int32_t* lengths, int64_t n, const int32_t* E_per_pair,
                                   int32_t E, int32_t* out)
{
    for (int64_t p = 0; p < n; p++) {
        int e = E_per_pair ? E_per_pair[p] : E;
        out[p] = ss_oracle_min_obstacles(refs + offsets[p], reads + offsets[p], lengths[p], e);
    }
}

void ss_oracle_levenshtein_batch(const uint8_t* reads, const uint8_t* refs, const int64_t* offsets,
                                 const int32_t* lengths, int64_t n, int32_t* out)
{
    for (int64_t p = 0; p < n; p++)
        out[p] = ss_oracle_levenshtein(refs + offsets[p], lengths[p], reads + offsets[p], lengths[p]);
}

/* Checkers over an unequal-length batch (layout as ss_oracle_batch_uneq), one
 * thread: the count after the deduction without the stop at E+1, the
 * exhaustive minimum of ss_oracle_min_obstacles_uneq, and the Levenshtein
 * distance (any of the outputs may be NULL). */
void ss_oracle_uneq_checks(const uint8_t* reads, const int64_t* read_off, const int32_t* read_len,
                           const uint8_t* refs, const int64_t* ref_off, const int32_t* ref_len, int64_t n, int32_t E,
                           int32_t* net, int32_t* minobs, int32_t* ed)
{
    for (int64_t p = 0; p < n; p++) {
        const uint8_t* R = refs + ref_off[p];
        const uint8_t* Q = reads + read_off[p];
        if (net) ss_oracle_pair_uneq(R, ref_len[p], Q, read_len[p], E, NULL, NULL, &net[p]);
        if (minobs) minobs[p] = ss_oracle_min_obstacles_uneq(R, ref_len[p], Q, read_len[p], E);
        if (ed) ed[p] = ss_oracle_levenshtein(R, ref_len[p], Q, read_len[p]);
    }
}
