/*
 * ss.h -- C ABI of the MI355X SneakySnake pre-alignment filter (libss.so).
 *
 * The filter follows the problem statement of Alser et al., "SneakySnake: a
 * fast and accurate universal genome pre-alignment filter for CPUs, GPUs and
 * FPGAs": given a reference R[1..m], a query Q[1..m] and an edit threshold E
 * (a number of tolerated character differences, Section 2.3), build the
 * (2E+1) x m chip maze of Equation 1 and walk it greedily (Section 2.4,
 * steps 1-5).  The number of obstacles on the net found is a lower bound on
 * the edit distance for every pair whose edit distance is <= E (Section 2.1,
 * Theorem 2); the pair is accepted (alignment needed) when that number is
 * <= E and rejected otherwise.  The walk stops as soon as the count exceeds
 * E, so a rejected pair reports E+1.
 *
 * Conventions for every entry point:
 *  - "reads" are the queries Q, "refs" the references R.  Maze columns index
 *    R; the count is not symmetric in R and Q, and the library never swaps
 *    them.
 *  - Pairs are concatenated: pair i occupies [offsets[i], offsets[i] +
 *    lengths[i]) in both reads and refs (equal lengths).  Bytes must be one of
 *    A C G T a c g t; anything else is SS_EBASE.
 *  - Every function returns an ss_status.  No C++ exception crosses the ABI.
 *  - Validation (null pointers, counts, lengths, thresholds, alphabet) runs
 *    before any output is written: on a validation error the outputs are left
 *    untouched.  After SS_EDEVICE the outputs are unspecified.
 *  - n_pairs == 0 is valid and returns SS_OK without touching the device.
 *  - Host pointers are owned by the caller and are not retained after the
 *    call returns.  Device pointers passed to the asynchronous *_async entry
 *    points must stay valid until the work enqueued on the given stream has
 *    completed; the caller synchronises.
 *  - A context is not thread-safe; use one per host thread.
 *  - There is no CPU fallback: without a usable gfx950 device every entry
 *    point that needs one returns SS_EDEVICE.
 */
#ifndef SS_H
#define SS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SS_OK = 0,
    SS_EINVAL = -1,       /* null pointer, negative count, bad flag or threshold */
    SS_EBASE = -2,        /* a byte outside ACGTacgt in reads or refs */
    SS_ELEN = -3,         /* a length or threshold beyond what the kernel supports */
    SS_ENOMEM = -4,       /* device or pinned allocation failed */
    SS_EBUDGET = -5,      /* a serving request alone exceeds the HBM budget */
    SS_EDEVICE = -6,      /* HIP runtime error or no usable device */
    SS_EAGAIN = -7,       /* serving: result not ready yet / queue full */
    SS_ETIMEOUT = -8      /* serving: wait deadline passed */
} ss_status;

/* Human-readable name of a status code (static string). */
const char* ss_status_str(int status);

/* Library limits. */
#define SS_MAX_E_SLICED   32      /* lane-sliced kernel: 0 <= E <= 32 */
#define SS_MAX_E_PLAIN    31      /* one-pair-per-lane kernel: 0 <= E <= 31 */
#define SS_MAX_E          16383   /* any path: counts must fit 14 bits */
#define SS_MAX_E_PLANNED  8191    /* batched launch and serving: 2E+1 rows in 64 lanes x 8 slices */
#define SS_MAX_LEN        (1 << 24)
#define SS_MAX_LEN_FUSED  2048    /* fused encode-and-filter kernel: m <= 2048 */
#define SS_MAX_LEN_VERIFY 65536   /* verification: m <= 65536 (one pair per lane up to 256) */
#define SS_MAX_E_VERIFY_BANDED 16351  /* banded verification: 2 E + 65 <= 16 x 2048 window positions */
/* wavefront, batched and serving paths: a bit stream of at most this many
 * bases (each plane under 4 GiB: its words are read with 32-bit offsets) */
#define SS_MAX_STREAM_BASES (32LL * ((1LL << 30) - 64))

/* Device result word, one per pair: bit 15 = accept, bits 0..14 = obstacle
 * count reported by the walk (min(count, E+1)). */
#define SS_RESULT_ACCEPT  0x8000u
#define SS_RESULT_COUNT   0x7FFFu

/* ------------------------------------------------------------------------
 * ss_filter_batch -- the one-call host API.
 * Synchronous; host pointers in and out; uses HIP device 0 of the process
 * (or the device made current with hipSetDevice before the first call).
 *   reads, refs : n_pairs concatenated sequences (see conventions), host.
 *   lengths     : n_pairs lengths, 0 <= lengths[i] <= SS_MAX_LEN, host.
 *   E           : threshold for every pair, 0 <= E <= SS_MAX_E.
 *   accept_out  : n_pairs bytes, 1 = accept (alignment needed), 0 = reject.
 *   edits_out   : n_pairs obstacle counts, min(count, E+1).
 * Internally: copy to HBM, encode (2-bit planes), filter, copy back.
 * The one-call host entry points (ss_filter_batch, ss_filter_batch_var,
 * ss_filter_batch_pairs) share one context per device; concurrent calls from
 * several host threads are safe and run one at a time.
 * ---------------------------------------------------------------------- */
int ss_filter_batch(const uint8_t* reads, const uint8_t* refs, const int32_t* lengths,
                    int64_t n_pairs, int32_t E, uint8_t* accept_out, int32_t* edits_out);

/* Same, with a threshold per pair (E_per_pair[i] in [0, SS_MAX_E]). */
int ss_filter_batch_var(const uint8_t* reads, const uint8_t* refs, const int32_t* lengths,
                        const int32_t* E_per_pair, int64_t n_pairs,
                        uint8_t* accept_out, int32_t* edits_out);

/* Pairs of unequal length, host pointers (the note of Section 2.4 between steps
 * 4 and 5).  Read (query) i has read_lengths[i] bases, reference i has
 * ref_lengths[i] (any lengths >= 0, <= SS_MAX_LEN); reads and refs are each the
 * concatenation of their sequences.  The maze spans the longer of the two;
 * a comparison with a character that does not exist is the fourth case of
 * Equation 1, and the obstacles the walk meets in leading or trailing columns
 * that hold no comparison of two existing characters are deducted before the
 * decision.  The reported count is min(count after the deduction, E+1); it
 * never exceeds the edit distance of the pair when that is <= E (Section 2.1),
 * and for equal lengths the result is ss_filter_batch's.  E_per_pair (host,
 * may be NULL) overrides E pair by pair.  Synchronous; alphabet errors return
 * SS_EBASE with the outputs untouched. */
int ss_filter_batch_pairs(const uint8_t* reads, const int32_t* read_lengths, const uint8_t* refs,
                          const int32_t* ref_lengths, int64_t n_pairs, const int32_t* E_per_pair, int32_t E,
                          uint8_t* accept_out, int32_t* edits_out);

/* ------------------------------------------------------------------------
 * Context: owns device scratch, the plan/work-queue buffers of the batched
 * path and the tuning table.  Bound to one HIP device.
 * ---------------------------------------------------------------------- */
typedef struct ss_ctx ss_ctx;
int ss_create(ss_ctx** out, int hip_device);
int ss_destroy(ss_ctx* ctx);

/* ------------------------------------------------------------------------
 * Lane-sliced layout (equal-length pairs).
 *
 * n_pairs pairs of common length m are encoded with base code A=0 C=1 G=2
 * T=3 split into a low-bit plane and a high-bit plane, transposed so that
 * bit s of a 32-bit word belongs to pair 32*g + s ("group" g).  Planes are
 * ordered Q0, Q1, R0, R1; positions are grouped in chunks of four.  Groups
 * come in blocks of 64, and a block's words are contiguous: with
 * G = ceil(n_pairs/32), nc = ceil(m/4), b = g / 64 and Gb = min(64, G - 64 b)
 * (the groups of block b), the word for (plane p, position j, group g) sits at
 * index
 *     (256 nc b + (p * nc + j/4) * Gb + g % 64) * 4 + j%4,
 * so that the 64 lanes of a wavefront, one group each, read 1 KiB contiguous
 * per chunk and one contiguous stretch over the whole sweep.  Slots of the
 * last group beyond n_pairs are encoded as all-'A' pairs.
 * ---------------------------------------------------------------------- */

/* Bytes of a lane-sliced buffer for n_pairs pairs of length m. */
int64_t ss_sliced_bytes(int64_t n_pairs, int32_t m);

/* Encode into the lane-sliced layout.  All pointers are device pointers.
 *   reads, refs : ASCII, pair i at offsets[i] (or at i*m when offsets is
 *                 NULL); every selected pair must have length m.
 *   index       : optional n_pairs pair indices (slot s encodes pair
 *                 index[s]); NULL selects pairs 0..n_pairs-1.
 *   packed      : ss_sliced_bytes(n_pairs, m) bytes, written in full.
 *   err         : one device uint32; bit 0 is OR-ed in when a byte outside
 *                 ACGTacgt is seen (the caller zeroes it beforehand).
 * Asynchronous on stream. */
int ss_pack_sliced_async(ss_ctx* ctx, const uint8_t* reads, const uint8_t* refs,
                         const int64_t* offsets, const int64_t* index, int64_t n_pairs, int32_t m,
                         uint32_t* packed, uint32_t* err, void* stream);

/* Filter a lane-sliced buffer with threshold E (0 <= E <= SS_MAX_E_SLICED);
 * writes n_pairs result words (see SS_RESULT_*) to out (device), in slot
 * order.  Asynchronous on stream.  This is the column-sweep kernel: every
 * lane advances 32 pairs by one maze column per step (Equation 1 cells for
 * all 2E+1 rows, the longest-run test of Section 2.4 as "no row still free
 * since the checkpoint"). */
int ss_filter_sliced_async(ss_ctx* ctx, const uint32_t* packed, int64_t n_pairs, int32_t m,
                           int32_t E, uint16_t* out, void* stream);

/* Filter a lane-sliced buffer at every threshold E_lo..E_hi (0 <= E_lo <=
 * E_hi <= SS_MAX_E_SLICED; a threshold sweep as in the paper's evaluation):
 * the result words of threshold E go to out + (E - E_lo) * out_stride
 * (device; n_pairs words each, in slot order), each equal to
 * ss_filter_sliced_async's at that threshold (Equation 1 rows, Section 2.4
 * walk).  Runs of thresholds that fit one kernel's registers (0..4 and
 * 5..7) share one pass over the buffer, every threshold keeping its own row
 * states and count over the same loaded words; the others take a pass each.
 *   out        : 16-byte aligned; out_stride >= n_pairs, a multiple of 8
 *   SS_EINVAL for a bad argument or alignment, SS_ELEN for E_hi or m past
 *   the limits.  Asynchronous on stream. */
int ss_filter_sliced_range_async(ss_ctx* ctx, const uint32_t* packed, int64_t n_pairs, int32_t m, int32_t E_lo,
                                 int32_t E_hi, uint16_t* out, int64_t out_stride, void* stream);

/* Snake-on-Chip's decomposition (Section 2.5) over a lane-sliced buffer: the
 * maze is cut into non-overlapping sub-mazes of sub_width columns (>= 1; the
 * last may be narrower) solved independently by the same walk, each starting
 * at its own first column, and the obstacle counts are summed.  The sum never
 * exceeds the whole-maze count (it underestimates; sub_width >= m gives
 * ss_filter_sliced_async's result).  Result words as ss_filter_sliced_async
 * (count saturated at E+1, accept iff sum <= E).  The paper's per-module
 * limit of its FPGA design (y instances per sub-maze) is not modelled: every
 * sub-maze is solved completely.  Asynchronous on stream. */
int ss_filter_submaze_async(ss_ctx* ctx, const uint32_t* packed, int64_t n_pairs, int32_t m, int32_t E,
                            int32_t sub_width, uint16_t* out, void* stream);

/* Encode and filter in one call, for pairs of one length m stored back to
 * back (pair i at byte i*m of reads and of refs; device pointers).  The
 * results are identical to ss_pack_sliced_async followed by
 * ss_filter_sliced_async (Equation 1 operands, Section 2.4 walk); the schedule
 * depends on E:
 *   E <= 10: one fused kernel.  Three wavefronts of each workgroup encode
 *            tiles of tile_groups groups of 32 pairs into one of two on-chip
 *            buffers while the fourth sweeps the previous tile from the other
 *            (for 16-byte aligned reads and refs and m <= 224 each encoding
 *            wavefront works alone and they meet the sweeping one through
 *            counters in on-chip memory; otherwise the four share the block's
 *            barriers), so the packed encoding never reaches device memory.
 *            With tile_groups = 0 and 16-byte aligned reads and refs the
 *            fused kernel runs only in the first form (m <= 224); longer
 *            aligned pairs take the two kernels below, which are faster there.
 *   E > 10 (and the longer aligned pairs above): the two kernels over
 *            chunks of packed data (192 MB up to E = 8, 400 MB above), kept
 *            in a buffer owned by ctx (allocated on first use, grown when a
 *            longer m needs it): calls that take this schedule on one context
 *            must be ordered (one stream), or use one context per stream.
 *   n_pairs >= 0; 0 <= m <= SS_MAX_LEN_FUSED; 0 <= E <= SS_MAX_E_SLICED
 *   tile_groups : groups per tile of the fused kernel, 1..256, or 0 for the
 *                 automatic choice (the largest tile whose two buffers keep
 *                 two workgroups per CU: 16 at 100 bp); SS_EINVAL when two
 *                 tiles and the staging do not fit on-chip memory (at
 *                 100 bp, 40 groups fit and 64 do not)
 *   out         : n_pairs result words (see SS_RESULT_*), 16-byte aligned
 *   err         : one device uint32; bit 0 is OR-ed in when a byte outside
 *                 ACGTacgt is seen (the caller zeroes it beforehand); the
 *                 results are then unspecified.  Bit 1 is OR-ed in if a wait
 *                 between the fused kernel's wavefronts gave up after its
 *                 bound (~0.1 s; not expected), with results unspecified.
 * Asynchronous on stream; the caller keeps every buffer alive until the
 * stream has passed this call. */
int ss_filter_ascii_async(ss_ctx* ctx, const uint8_t* reads, const uint8_t* refs, int64_t n_pairs, int32_t m,
                          int32_t E, int32_t tile_groups, uint16_t* out, uint32_t* err, void* stream);

/* ------------------------------------------------------------------------
 * Without allocation: for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it).
 *
 * ss_filter_ascii_noalloc is ss_filter_ascii_async with the automatic tile
 * (same arguments, same results, same limits: m <= SS_MAX_LEN_FUSED and
 * E <= SS_MAX_E_SLICED, else SS_ELEN) that calls no hipMalloc, hipFree or
 * allocating routine.  Where ss_filter_ascii_async would encode a chunk into a
 * buffer the context allocates, this one uses a scratch array of
 * SS_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends (looked up by ss_create), processing the batch in
 * chunks that fit it; the fused schedule needs no scratch.  Every call on one
 * GPU shares that array, so calls that overlap on one GPU (several streams,
 * several threads) race and must be ordered by the caller.  The context gives
 * the device; no buffer of the context is used.  Asynchronous on stream. */
#define SS_NOALLOC_SCRATCH_BYTES (32LL << 20)
int ss_filter_ascii_noalloc(ss_ctx* ctx, const uint8_t* reads, const uint8_t* refs, int64_t n_pairs, int32_t m,
                            int32_t E, uint16_t* out, uint32_t* err, void* stream);

/* ------------------------------------------------------------------------
 * Bit-stream layout (any lengths).
 *
 * Four planes (Q0, Q1, R0, R1), each a little-endian stream of total_bases
 * bits: base b of the concatenation is bit b%32 of word b/32.  Each plane
 * occupies ss_stream_words(total_bases) 32-bit words (two guard words
 * included); plane p starts at word p * ss_stream_words(total_bases).
 * ---------------------------------------------------------------------- */
int64_t ss_stream_words(int64_t total_bases);

/* Encode the concatenated ASCII reads/refs (device) into bit streams
 * (device, 4 * ss_stream_words(total_bases) words).  err as above. */
int ss_pack_stream_async(ss_ctx* ctx, const uint8_t* reads, const uint8_t* refs,
                         int64_t total_bases, uint32_t* packed, uint32_t* err, void* stream);

/* One pair per lane (the granularity of the paper's GPU design, Section
 * 2.6): each lane builds its pair's 2E+1 rows one 32-column word at a time
 * (Equation 1 as XOR/OR masks) and runs the greedy walk of Section 2.4 on
 * them.  0 <= E <= SS_MAX_E_PLAIN.  offsets/lengths are device arrays.
 * E_per_pair (device, may be NULL) overrides E pair by pair; then every
 * E_per_pair[i] must be <= E, which bounds the rows built. */
int ss_filter_plain_async(ss_ctx* ctx, const uint32_t* packed, int64_t total_bases,
                          const int64_t* offsets, const int32_t* lengths,
                          const int32_t* E_per_pair, int64_t n_pairs, int32_t E,
                          uint16_t* out, void* stream);

/* Wavefront-cooperative filter: one or more pairs per 64-lane wavefront,
 * the 2E+1 rows spread over lanes as 32-row bit slices; every column is
 * one step of the sweep and an OR over the pair's lanes decides whether any
 * row is still free since the checkpoint.  Any E up to SS_MAX_E.  Arguments
 * as ss_filter_plain_async (E is the per-launch maximum when E_per_pair is
 * given); SS_ELEN for total_bases above SS_MAX_STREAM_BASES. */
int ss_filter_wave_async(ss_ctx* ctx, const uint32_t* packed, int64_t total_bases,
                         const int64_t* offsets, const int32_t* lengths,
                         const int32_t* E_per_pair, int64_t n_pairs, int32_t E,
                         uint16_t* out, void* stream);

/* ------------------------------------------------------------------------
 * One entry point for any batch: the batch descriptor.
 *
 * The problem of Section 2.1 and 2.3 for a batch: n_pairs (reference, query)
 * pairs, a threshold per pair, one accept/count result per pair (Section 2.4,
 * step 5).  The inputs are device buffers in one of three forms, and the
 * kernel is chosen by the caller or, with SS_KERNEL_AUTO, from the pairs'
 * shape:
 *   - a lane-sliced buffer (SS_INPUT_PACKED_SLICED)      -> the column sweep;
 *   - a plan given                                      -> its persistent launch;
 *   - ASCII, one length, one threshold <= SS_MAX_E_SLICED -> the one-call path
 *     (fused encode + sweep) when the pairs lie back to back (offsets NULL) and
 *     m <= SS_MAX_LEN_FUSED, else encode to the lane-sliced layout + sweep;
 *   - anything else (several lengths, unequal lengths, thresholds per pair,
 *     larger thresholds, bit streams) -> the wavefront kernel.
 * Forcing a kernel whose conditions the batch does not meet returns SS_EINVAL
 * (or SS_ELEN for a length or threshold beyond its limit).
 * ---------------------------------------------------------------------- */
#define SS_INPUT_ASCII          0x0u   /* reads / refs: ASCII bases (device) */
#define SS_INPUT_PACKED         0x1u   /* reads / refs: each side packed apart by ss_pack */
#define SS_INPUT_PACKED_SLICED  0x2u   /* reads: ss_pack_sliced_async's buffer (both sides); refs unused */
#define SS_INPUT_MASK           0x0Fu
#define SS_KERNEL_AUTO          0x00u
#define SS_KERNEL_FUSED         0x10u  /* ASCII back to back, one length <= SS_MAX_LEN_FUSED, E <= SS_MAX_E_SLICED */
#define SS_KERNEL_SLICED        0x20u  /* one length, one threshold <= SS_MAX_E_SLICED (ASCII or lane-sliced input) */
#define SS_KERNEL_PLAIN         0x30u  /* one pair per lane, equal lengths, E <= SS_MAX_E_PLAIN (ASCII or ss_pack input) */
#define SS_KERNEL_WAVE          0x40u  /* wavefront-cooperative sweep: any lengths, E <= SS_MAX_E */
#define SS_KERNEL_PERSISTENT    0x50u  /* the persistent launch of desc->plan (equal lengths, E_per_pair required) */
#define SS_KERNEL_MASK          0xF0u

typedef struct ss_plan ss_plan;

typedef struct ss_batch_desc {
    const void* reads;            /* device: queries in the input form of flags */
    const void* refs;             /* device: references (NULL for SS_INPUT_PACKED_SLICED) */
    const int64_t* offsets;       /* device, n_pairs: first base of query i in reads (bit for ss_pack input),
                                     and of reference i when ref_offsets is NULL; NULL: i * length */
    const int32_t* lengths;       /* device, n_pairs: query lengths (and reference lengths when ref_lengths is
                                     NULL); NULL: every pair has `length` bases */
    const int64_t* ref_offsets;   /* device, may be NULL: references at offsets[] */
    const int32_t* ref_lengths;   /* device, may be NULL: references as long as their queries; given together
                                     with ref_offsets, for pairs of unequal length (ss_filter_batch_pairs) */
    const int32_t* E_per_pair;    /* device, may be NULL: threshold of each pair, each <= E */
    const ss_plan* plan;          /* for SS_KERNEL_PERSISTENT: a plan of these pairs' host lengths and
                                     thresholds (ss_plan_create) on this context's device */
    int64_t n_pairs;
    int64_t read_bases;           /* bases in reads (the concatenation; ASCII and ss_pack input) */
    int64_t ref_bases;            /* bases in refs */
    int32_t length;               /* >= 0: every pair (both sides) has this many bases; -1: see lengths */
    int32_t E;                    /* the threshold, or the largest of E_per_pair */
    uint32_t flags;               /* SS_INPUT_* | SS_KERNEL_* */
    uint32_t reserved;            /* 0 */
    uint16_t* out;                /* device, n_pairs result words (SS_RESULT_*), 16-byte aligned */
    uint32_t* err;                /* device word (required for ASCII input; the caller zeroes it): bit 0 a byte
                                     outside ACGTacgt, bit 1 a wait in the fused kernel that gave up; the results
                                     are then unspecified */
} ss_batch_desc;

/* Words ss_pack writes for `bases` bases: two planes (low and high bit of the
 * code A=0 C=1 G=2 T=3) of the bit-stream layout above, each
 * ss_stream_words(bases) words; -1 for a negative count. */
int64_t ss_pack_words(int64_t bases);

/* Encode one side (reads or refs, ASCII in device memory) into the 2-bit
 * planes of ss_pack_words(bases) words at packed (device).  err as for
 * ss_pack_stream_async.  SS_ELEN above SS_MAX_STREAM_BASES.  Asynchronous on
 * stream. */
int ss_pack(ss_ctx* ctx, const uint8_t* ascii, int64_t bases, uint32_t* packed, uint32_t* err, void* stream);

/* Filter the batch a descriptor describes (rows a1-a5: encode when the input
 * is ASCII, build the Equation 1 rows, walk, decide and write), enqueued on
 * stream; the caller synchronises.  Device arrays (offsets, lengths, thresholds)
 * cannot be checked on the host: the caller guarantees that every pair lies
 * inside its buffers and that each E_per_pair[i] <= E.  Without offsets (pairs
 * back to back at i * length) the bit-stream kernels (plain, wavefront,
 * persistent) need n_pairs * length <= read_bases (and <= ref_bases when the
 * references follow the queries' offsets): SS_EINVAL otherwise.  Buffers the context
 * owns (encodings of ASCII input) are reused by the next call on the context:
 * calls on one context must be ordered (one stream). */
int ss_filter_batch_ex(ss_ctx* ctx, const ss_batch_desc* desc, void* stream);

/* ------------------------------------------------------------------------
 * Verification (not part of SneakySnake): the step a pre-alignment filter
 * exists to shorten (Section 1: only accepted pairs go on to alignment;
 * Section 3 measures the filter's false accept rate against the exact edit
 * distance).  These compute the exact edit distance (unit-cost Levenshtein
 * distance) of the pairs a filter accepted, on the GPU, so that a batch can
 * be filtered and verified without leaving the device.
 * ---------------------------------------------------------------------- */

/* Exact edit distance of n pairs in the bit-stream layout (device arrays as
 * for ss_filter_wave_async).  index: optional n pair indices (entry k
 * verifies pair index[k]; NULL: pairs 0..n-1).  max_len >= every listed
 * pair's length, <= SS_MAX_LEN_VERIFY (SS_ELEN beyond).  ed_out[k] (device,
 * int32) = edit distance of the k-th listed pair (-1 for a pair longer than
 * max_len).  Myers' bit-vector algorithm (J. ACM 1999) in its
 * global-distance form: one pair per lane for max_len <= 256, else one pair
 * per wavefront (each lane a 32 W-position stretch of the query, W the
 * smallest power of two with 2048 W >= max_len; the addition's carries cross
 * lanes by one carry-lookahead step per column), so a batch of short and
 * long pairs is best verified in two calls, each over its own index list.
 * Asynchronous on stream. */
int ss_verify_async(ss_ctx* ctx, const uint32_t* packed, int64_t total_bases, const int64_t* offsets,
                    const int32_t* lengths, const int64_t* index, int64_t n, int32_t max_len, int32_t* ed_out,
                    void* stream);

/* Banded verification, any length (up to SS_MAX_LEN): ed_out[k] = the edit
 * distance of the k-th listed pair when it is at most that pair's threshold
 * (E_per_pair[p], or E for every pair when E_per_pair is NULL), else the
 * threshold + 1.  E must be >= every listed threshold (it sizes the window;
 * a pair whose threshold needs a wider window than E's gets -1),
 * <= SS_MAX_E_VERIFY_BANDED (SS_ELEN beyond).  Pairs of equal length in the
 * bit-stream layout, index as for ss_verify_async.  One pair per wavefront:
 * Myers' bit-vector algorithm over a window of the query that follows the
 * diagonal band |i - j| <= threshold (Ukkonen's observation that a path of
 * cost <= k never leaves it), in 32-row words that leave the window at the
 * bottom and enter it at the top as the band moves; rows outside the window
 * are taken at values never below their true ones, so the distance is exact
 * whenever it is within the threshold.  Time ~ m * threshold / 2048 per pair
 * instead of m * m.  Asynchronous on stream. */
int ss_verify_banded_async(ss_ctx* ctx, const uint32_t* packed, int64_t total_bases, const int64_t* offsets,
                           const int32_t* lengths, const int32_t* E_per_pair, int32_t E, const int64_t* index,
                           int64_t n, int32_t* ed_out, void* stream);

/* Indices of the accepted pairs of n result words (bit 15 set), written to
 * index_out (device, room for n entries) in no particular order; their number
 * to *count_out (device int64, cleared by this call with a kernel, not a
 * memset).  Asynchronous on stream. */
int ss_select_accepted_async(ss_ctx* ctx, const uint16_t* results, int64_t n, int64_t* index_out,
                             int64_t* count_out, void* stream);

/* ------------------------------------------------------------------------
 * Batched launch: pairs of uneven lengths with a threshold per pair, all in
 * one persistent kernel.  Not part of the paper (its GPU design launches one
 * thread per pair, Section 2.6); it runs the wavefront sweep above on work
 * items popped from a device queue.
 *
 * A plan is built on the host from the pairs' lengths and thresholds (host
 * arrays, copied; the plan keeps no pointer to them): each pair gets a shape
 * (lanes per pair, 32-row slices per lane, at most slices_per_lane = 1, 2, 4
 * or 8: fewer slices per lane spread a pair over more lanes, for lower
 * latency per pair at some cost in total work)
 * from its threshold; pairs are sorted by shape and length, cut into work
 * items of one 256-thread block round, and the items ordered largest
 * estimated cost first (by input position among items of about the same
 * cost).  The plan owns its device buffers (permutation, item
 * table, queue counter) and is bound to the device current at creation.
 * A pair's 2E+1 rows must fit one wavefront (64 lanes x slices_per_lane x 32
 * rows): slices_per_lane is raised to the smallest width that holds the
 * largest threshold (ss_plan_info reports the width used), and thresholds
 * above SS_MAX_E_PLANNED return SS_ELEN (the standalone wavefront kernel,
 * ss_filter_wave_async, covers them up to SS_MAX_E).
 * ---------------------------------------------------------------------- */
int ss_plan_create(ss_ctx* ctx, const int32_t* lengths, const int32_t* E_per_pair, int64_t n_pairs,
                   int32_t slices_per_lane, ss_plan** out);
int ss_plan_destroy(ss_plan* plan);
/* Host only (no device work; for inspection and tests): the work items a plan
 * for these pairs holds, in queue order.  *n_items receives their number;
 * when items is non-null, up to max_items of them as five int64 each (first
 * slot in the permutation, pairs, lanes per pair, slices per lane, largest
 * threshold); when perm is non-null, the n_pairs-entry permutation (pair
 * index per slot).  Errors as ss_plan_create. */
int ss_plan_items_host(const int32_t* lengths, const int32_t* E_per_pair, int64_t n_pairs, int32_t slices_per_lane,
                       int64_t* n_items, int64_t* items, int64_t max_items, int64_t* perm);
/* Items in the queue, shape classes, persistent grid size, slices per lane. */
int ss_plan_info(const ss_plan* plan, int64_t* n_items, int32_t* n_classes, int32_t* grid,
                 int32_t* slices_per_lane);

/* Run a plan on bit-stream encoded pairs (device arrays as for
 * ss_filter_wave_async; E_per_pair is required; SS_ELEN for total_bases
 * above SS_MAX_STREAM_BASES, here and in the capture and autotuner calls).
 * Enqueues a counter reset and the persistent kernel on stream.  One call at
 * a time per plan (the queue counter is part of the plan). */
int ss_filter_planned_async(ss_ctx* ctx, const ss_plan* plan, const uint32_t* packed, int64_t total_bases,
                            const int64_t* offsets, const int32_t* lengths, const int32_t* E_per_pair,
                            uint16_t* out, void* stream);

/* Capture the planned launch for these device buffers into a HIP graph held
 * by the plan (replacing any earlier capture); ss_plan_launch replays it on
 * stream.  The buffers must outlive every replay. */
int ss_plan_capture(ss_ctx* ctx, ss_plan* plan, const uint32_t* packed, int64_t total_bases,
                    const int64_t* offsets, const int32_t* lengths, const int32_t* E_per_pair, uint16_t* out);
int ss_plan_launch(ss_plan* plan, void* stream);

/* Autotuned plan: times the candidate shapes (1, 2, 4, 8 slices per lane),
 * each with the persistent grid at as many resident blocks per CU as fit and
 * at two, on this batch with the given device buffers (out_dev is
 * overwritten), keeps the fastest and records it in the JSON file cache_path
 * (may be NULL; value = slices + 100 x blocks per CU, 0 meaning as many as
 * fit) under a key made of the device architecture and a coarse signature of
 * the batch; a later call with a matching key skips the timing.
 * *chosen_slices (may be NULL) receives the slice width; ss_plan_info reports
 * the grid.  Synchronous. */
int ss_plan_create_tuned(ss_ctx* ctx, const int32_t* lengths, const int32_t* E_per_pair, int64_t n_pairs,
                         const uint32_t* packed, int64_t total_bases, const int64_t* offsets_dev,
                         const int32_t* lengths_dev, const int32_t* E_dev, uint16_t* out_dev,
                         const char* cache_path, ss_plan** out, int32_t* chosen_slices);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of filter requests on one device (not part of
 * the paper).  The server owns n_slots slots (a stream each); inputs are
 * staged in pooled pinned host blocks at submission, device memory comes from
 * the stream-ordered pool and is kept resident between requests.  Admission is
 * by HBM budget: the device footprints (ss_server_footprint) of the requests
 * in flight never total more than hbm_budget_bytes; requests that do not fit
 * wait in FIFO order until slots and memory free up.  Each admitted request is
 * encoded, planned (batched launch above) and filtered on its slot's stream,
 * so requests in different slots overlap on the device.  Threads: a
 * dispatcher and a completion thread per server; submit / poll / wait are
 * thread-safe.  The server uses the device current at creation.
 * ---------------------------------------------------------------------- */
typedef struct ss_server ss_server;
typedef uint64_t ss_ticket;
int ss_server_create(ss_ctx* ctx, size_t hbm_budget_bytes, int32_t n_slots, ss_server** out);
/* Device bytes a request of n_pairs pairs and total_bases bases needs (its
 * share of the budget); -1 for negative arguments. */
int64_t ss_server_footprint(int64_t n_pairs, int64_t total_bases);

/* The same server with a device-resident request loop (not part of the
 * paper): one persistent kernel serves every request.  An admitted request is
 * handed over by writing its descriptor into one of n_slots (at most 64)
 * slots of a control block in coherent pinned host memory; no HIP call is
 * made per request.  The kernel's scheduling wavefront activates published
 * requests; its other blocks encode each request's ASCII straight from its
 * staging block (coherent pinned host memory) into bit planes and sweep the
 * request's plan (the batched launch's items), oldest admission first, writing
 * the result words into the staging block; the block that finishes a
 * request's last item marks the slot done, and the completion thread polls
 * those marks.  The kernel ends after 200 ms with nothing to do and is launched
 * again when a request arrives.  While it runs it holds one block on every CU,
 * so other kernels on the device wait until it has been idle for 200 ms: one
 * loop server per device at a time (a second creation on the same device
 * returns SS_EAGAIN until the first is destroyed), and other GPU work of the
 * process is best kept off the device while requests flow.
 * Device memory: hbm_budget_bytes are reserved at creation as one arena; a
 * request takes the room of its four bit planes, 16 * (ceil(total_bases / 32)
 * + 2) bytes rounded up to 256, from it, and admission waits while the arena
 * has no such room.  slices_per_lane (1, 2, 4 or 8) is fixed: a request with
 * a threshold that needs wider slices is refused (SS_ELEN), as is one whose
 * plan has more than 2^24 - 1 items or encoding units.  Every other call
 * below works on either kind of server, except ss_server_set_slices
 * (SS_EINVAL here); ss_server_stages reports no enqueue stream events here:
 * h2d_ns is the device time from activation to the end of encoding (reading
 * the ASCII over the host link), compute_ns the rest up to the last item,
 * d2h_ns 0 (results are written in place).  If the kernel cannot be launched
 * or reports that no unit finished for 2 s with requests active, requests in
 * flight fail with SS_EDEVICE and later submissions are refused with
 * SS_EDEVICE. */
int ss_server_create_loop(ss_ctx* ctx, size_t hbm_budget_bytes, int32_t n_slots, int32_t slices_per_lane,
                          ss_server** out);
/* Device-resident loop only: how long (microseconds, 1 .. 60 s; 200 ms by
 * default) the loop kernel stays resident with nothing to do before it ends
 * and frees the CUs; a request that arrives after that pays a kernel launch.
 * Takes effect at the next launch of the loop.  SS_EINVAL for a server of the
 * other kind. */
int ss_server_set_loop_idle(ss_server* server, int64_t idle_us);

/* Submit one request (host arrays, copied before returning; E_per_pair is
 * required).  accept_out / edits_out (host, n_pairs entries) are written by
 * the server before the ticket reports done, and must stay valid until then.
 * SS_EBUDGET if the request alone needs more than the budget; SS_ELEN for a
 * threshold above SS_MAX_E_PLANNED or more than SS_MAX_STREAM_BASES bases.
 * Validation of lengths and thresholds
 * happens here; the alphabet is checked on the device and reported by
 * ss_server_wait (outputs then untouched). */
int ss_server_submit(ss_server* server, const uint8_t* reads, const uint8_t* refs, const int32_t* lengths,
                     const int32_t* E_per_pair, int64_t n_pairs, uint8_t* accept_out, int32_t* edits_out,
                     ss_ticket* ticket);
/* Submission without the copy of the bases (either kind of server).
 * ss_server_stage_alloc returns a block of `bytes` bytes of pinned host memory
 * from the server's staging (mapped to the device on a device-resident loop
 * server, whose kernel reads it there; copied from by DMA on the other kind),
 * or NULL when bytes is 0 or the staging is full.  The caller writes a request's bases into it (the reads
 * concatenated from its start, the references concatenated from refs_offset,
 * a multiple of 16 recommended) and hands it to ss_server_submit_staged, which
 * checks and plans the request as ss_server_submit does but reads the bases
 * from the block on the device instead of copying them: the block then
 * belongs to the request and returns to the staging when the request is done
 * or cancelled (the caller must not touch it again).  On any status other
 * than SS_OK the block stays the caller's; ss_server_stage_free returns a
 * block that was never submitted (SS_EINVAL for any other pointer).  SS_EINVAL
 * too when the two sides do not fit the block apart (refs_offset < the total
 * of lengths, or past the block's end).  Blocks still held at
 * ss_server_destroy are freed with the server. */
void* ss_server_stage_alloc(ss_server* server, size_t bytes);
int ss_server_stage_free(ss_server* server, void* block);
int ss_server_submit_staged(ss_server* server, void* block, size_t refs_offset, const int32_t* lengths,
                            const int32_t* E_per_pair, int64_t n_pairs, uint8_t* accept_out, int32_t* edits_out,
                            ss_ticket* ticket);
/* *done = 1 once the request has finished (or was cancelled). */
int ss_server_poll(ss_server* server, ss_ticket ticket, int* done);
/* Wait up to timeout_us (negative: no limit).  Returns the request's status
 * (SS_OK, SS_EBASE, SS_EDEVICE, ...), SS_ETIMEOUT if still running, or
 * SS_EAGAIN if it was cancelled.  The request keeps running after a timeout. */
int ss_server_wait(ss_server* server, ss_ticket ticket, int64_t timeout_us);
/* Steady-clock nanoseconds of submission, admission and completion (0 = not yet). */
int ss_server_times(ss_server* server, ss_ticket ticket, int64_t* submit_ns, int64_t* admit_ns, int64_t* done_ns);
/* Where a finished request's time went (nanoseconds, 0 until it is done): the
 * host's time to enqueue its work on its slot's stream after admission, and,
 * from timing events on that stream, the copy of its inputs to the device,
 * the encoding and filter kernels, and the copy of its results back. */
int ss_server_stages(ss_server* server, ss_ticket ticket, int64_t* enqueue_ns, int64_t* h2d_ns, int64_t* compute_ns,
                     int64_t* d2h_ns);
/* Cancel a request that is still queued (SS_EAGAIN once admitted). */
int ss_server_cancel(ss_server* server, ss_ticket ticket);
/* Forget a finished ticket (SS_EAGAIN while queued or running). */
int ss_server_release(ss_server* server, ss_ticket ticket);
/* Pause (hold != 0) or resume dispatching; paused requests stay queued.  For
 * tests of the timeout and queueing paths. */
int ss_server_set_hold(ss_server* server, int hold);
/* Slice width (1, 2, 4 or 8 32-row slices per lane, default 1) used to plan
 * requests submitted from now on: fewer slices spread each pair over more
 * lanes and shorten the longest pair's sweep, which bounds a request's
 * latency.  A request whose largest threshold needs a wider slice gets it. */
int ss_server_set_slices(ss_server* server, int32_t slices_per_lane);
int ss_server_stats(ss_server* server, int64_t* admitted, int64_t* deferred, int64_t* completed,
                    int64_t* peak_bytes, int64_t* peak_in_flight);
/* Cancels queued requests, waits for running ones, frees everything. */
int ss_server_destroy(ss_server* server);

/* Expand device result words into accept bytes and int32 counts (device). */
int ss_unpack_results_async(ss_ctx* ctx, const uint16_t* results, int64_t n_pairs,
                            uint8_t* accept_out, int32_t* edits_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SS_H */
