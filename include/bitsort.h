/*
 * bitsort.h -- C ABI of the MI355X (gfx950) bitmap sort library, libbitsort.so.
 *
 * The operation (Yordzhev, "The bitwise operations related to a fast sorting
 * algorithm", arXiv:1312.0138): sort an integer array ascending (Section IV,
 * Section V, Theorem 1), here for distinct unsigned keys bounded by
 * R = 2^range_bits.  Each key is marked as one bit of a bit-vector (shift and
 * OR: Section II Table I, Section III Examples 2 and 3); the words are then
 * scanned in order, set bits counted (Example 6), and the positions of the
 * set bits written out (Example 1; bit 0 is the rightmost, Section II).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Key and output pointers are DEVICE pointers (hipMalloc'ed or a torch
 *   tensor's data pointer).  The caller owns them; the library never frees
 *   them.  Unless stated otherwise, offsets / range_bits arrays are device
 *   pointers too.
 * - `stream` is a hipStream_t passed as an opaque pointer; NULL means the
 *   default stream.  Every call only enqueues work on `stream` and returns;
 *   nothing is synchronised except where a function says so.
 * - Return value: BITSORT_OK or a BITSORT_ERR_* code, decided on the host
 *   before anything is enqueued (argument checks) or from a failed HIP call.
 * - Data errors found on the device (a key >= R, a duplicate key) are not
 *   return codes: they set BITSORT_STATUS_* flags that bitsort_get_status()
 *   reads after the work has finished.  No such key causes a write outside
 *   the output array.
 * - A key >= R is dropped.  With duplicates each distinct key is written
 *   once.  In both cases out[0 .. d) holds the d distinct in-range keys in
 *   ascending order, and d is reported as bitsort_status_t.count.  Slots
 *   out[d .. n) are left untouched when only out-of-range keys occurred; after
 *   a duplicate their content is unspecified.
 * - Thread safety: calls on different streams may run concurrently; calls on
 *   one stream are ordered by that stream.
 */
#ifndef BITSORT_H
#define BITSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *bitsort_stream_t; /* a hipStream_t */

/* Return codes. */
#define BITSORT_OK 0
#define BITSORT_ERR_INVALID_ARG 1 /* null pointer with n > 0, range_bits > 32, partial overlap, ... */
#define BITSORT_ERR_TOO_LARGE 2   /* n > 2^range_bits, n >= 2^32, or beyond a stated limit */
#define BITSORT_ERR_NO_MEMORY 3   /* workspace allocation failed, or a caller workspace is too small */
#define BITSORT_ERR_HIP 4         /* a HIP runtime call or kernel launch failed */

/* Device status flags (bitsort_status_t.flags). */
#define BITSORT_STATUS_OUT_OF_RANGE 1u /* some key was >= 2^range_bits and was dropped */
#define BITSORT_STATUS_DUPLICATE 2u    /* some key occurred more than once */
#define BITSORT_STATUS_TIMEOUT 32u     /* a bounded wait between workgroups gave up: the output is invalid */
#define BITSORT_STATUS_BAD_STATE 64u   /* bitsort_u32_atomic found its bit-vector not all zero: nothing written */

typedef struct bitsort_status {
    uint32_t flags;  /* BITSORT_STATUS_* bits */
    uint32_t _pad;
    uint64_t count;  /* d: number of keys written (distinct, in range) */
} bitsort_status_t;

/* Library version, e.g. 10000 for 1.0.0. */
int bitsort_version(void);

/* Human-readable text for a return code (static storage). */
const char *bitsort_error_string(int code);

/*
 * Sort n distinct uint32 keys, each < 2^range_bits, ascending into out.
 *   keys        device, n elements, read only.
 *   n           number of keys, n < 2^32 and n <= 2^range_bits.
 *   range_bits  0..32; the key range is [0, 2^range_bits).
 *   out         device, n elements.  out == keys (exact alias, in-place
 *               sort) is allowed; any other overlap is BITSORT_ERR_INVALID_ARG.
 *   stream      see above.
 * Uses a workspace the library allocates on first use per (device, stream)
 * and keeps, growing it when a larger problem comes (about 4n bytes plus a
 * small table).  n = 0 enqueues nothing.
 * Method: Sections II-III (mark with shift/OR), Example 6 (count), Example 1
 * (emit), Theorem 1 (ascending result).
 */
int bitsort_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits, uint32_t *out,
                bitsort_stream_t stream);

/*
 * The same sort as bitsort_u32, done the direct way: every key ORs its bit
 * into a bit-vector kept in HBM with an atomic OR (Table I: OR-ing a 1 sets a
 * bit, in any order and any number of times; the word index by a right shift,
 * Example 3; the mask by a left shift, Example 2), lanes of a wave holding
 * keys of the same word first combining their masks so that one atomic per
 * word and wave is issued; then the ones of every 1024-word chunk are counted
 * (Example 6), a device-wide exclusive prefix of the counts taken, and the set
 * bits written out lowest first (Example 1) into out.  Arguments, errors and
 * result as bitsort_u32 (repeated keys collapse into one; the status, read
 * with bitsort_get_status on the same stream, flags them).  Its bit-vector
 * (2^range_bits / 8 bytes, at least 4 KiB) is allocated per (device, stream),
 * zeroed once, and left zero by every call: the emission clears the words it
 * reads.  Four launches: mark, chunk counts, prefix, emission.
 */
int bitsort_u32_atomic(const uint32_t *keys, uint64_t n, uint32_t range_bits, uint32_t *out,
                       bitsort_stream_t stream);

/*
 * The bitmap sort for 64-bit keys (Algorithm 1 of Section V is written for
 * any integer type T; the result is again the ascending arrangement of
 * Theorem 1): n distinct uint64 keys, each < 2^range_bits, range_bits 0..36,
 * ascending into out.  The range is cut into 2^(range_bits - 32) groups of
 * 2^32 keys by the bits above bit 31 (one group when range_bits <= 32); the
 * keys' low 32 bits are gathered group by group, each group is sorted by the
 * plain path's kernels (all groups in one pointer-array launch: mark into LDS
 * slices by shift and OR, Table I and Examples 2-3; count, Example 6; emit,
 * Example 1), and the groups are written back as 64-bit keys in order.
 *   keys, out   device, n uint64 each; out == keys allowed, any other overlap
 *               is rejected.
 *   n           n < 2^32 and n <= 2^range_bits.
 * Status with bitsort_get_status on the same stream: count = distinct keys
 * written, OUT_OF_RANGE / DUPLICATE as for bitsort_u32; out[0 .. count) holds
 * them ascending.  The call waits on the host once, after the grouping, for
 * the groups' sizes (they plan the pointer-array launch).  Workspace: the
 * stream's (about 4n bytes plus small tables) and its batch workspace.
 * Errors: BITSORT_ERR_INVALID_ARG (range_bits > 36, null pointers, partial
 * overlap), BITSORT_ERR_TOO_LARGE, BITSORT_ERR_NO_MEMORY, BITSORT_ERR_HIP.
 */
int bitsort_u64(const uint64_t *keys, uint64_t n, uint32_t range_bits, uint64_t *out, bitsort_stream_t stream);

/*
 * The same bitmap sort for signed keys (the paper sorts any integer type,
 * negative keys included: Section V's BitwiseSort puts the negative keys
 * first).  Keys are distinct int32 in [-2^(range_bits-1), 2^(range_bits-1))
 * (range_bits 1..32; 0 allows only the key 0).  Each key is shifted by
 * 2^(range_bits-1) on load, which maps that range onto [0, 2^range_bits) in
 * order, and shifted back on output, inside the same kernels: no extra pass.
 * Arguments, errors, status and workspace as bitsort_u32; a key outside the
 * signed range is dropped and raises BITSORT_STATUS_OUT_OF_RANGE.
 */
int bitsort_i32(const int32_t *keys, uint64_t n, uint32_t range_bits, int32_t *out, bitsort_stream_t stream);

/* Bytes of caller workspace bitsort_u32_ws needs for (n, range_bits); 0 on
 * invalid arguments. */
size_t bitsort_workspace_bytes(uint64_t n, uint32_t range_bits);

/*
 * bitsort_u32 with a caller-provided device workspace of at least
 * bitsort_workspace_bytes(n, range_bits) bytes, 256-byte aligned.  Its first
 * sizeof(bitsort_status_t) bytes receive the status of this call; read them
 * with bitsort_workspace_status().  Errors: as bitsort_u32, plus
 * BITSORT_ERR_NO_MEMORY when ws_bytes is too small and BITSORT_ERR_INVALID_ARG
 * when the workspace is misaligned.
 */
int bitsort_u32_ws(const uint32_t *keys, uint64_t n, uint32_t range_bits, uint32_t *out,
                   void *workspace, size_t ws_bytes, bitsort_stream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sort of
 * bitsort_u32, with the same arguments, result and errors, that allocates
 * nothing.  Its workspace is one fixed device array of
 * BITSORT_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs
 * on until the process ends.
 *   status  device pointer to one bitsort_status_t (8-byte aligned, not
 *           overlapping keys or out) that receives this call's status when
 *           the work has run; NULL to discard it.  n = 0 writes a zero status.
 * Returns BITSORT_ERR_TOO_LARGE, before touching the device, when the
 * problem's workspace would exceed the array: bitsort_workspace_bytes(n,
 * range_bits) <= BITSORT_NOALLOC_SCRATCH_BYTES is the limit (10^6 keys over
 * 2^24 need about 4.3 MB; 2^22 keys over 2^24 about 18.4 MB).  Every call on
 * one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (different streams, or different host threads) race and give undefined
 * results.  The first call on a device looks up the array's address there.
 */
#define BITSORT_NOALLOC_SCRATCH_BYTES (32u << 20)
int bitsort_u32_noalloc(const uint32_t *keys, uint64_t n, uint32_t range_bits, uint32_t *out,
                        bitsort_status_t *status, bitsort_stream_t stream);

/* Synchronise `stream`, then copy the status of the last call made on it
 * (library workspace) into *status.  A two-kernel plain sort leaves its totals
 * (flags, count, and after a repeated key the compaction of out[0 .. d)) to
 * this read, which runs them on `stream` before it copies: read the status
 * before using out when the input may hold a repeated key.  The same holds
 * for bitsort_workspace_status and bitsort_graph_status. */
int bitsort_get_status(bitsort_stream_t stream, bitsort_status_t *status);

/*
 * Give the library a workspace for the calls on `stream` (bitsort_u32,
 * bitsort_i32, bitsort_pairs_u32, bitsort_count_u32 and the radix sorts),
 * instead of the memory
 * it would allocate and keep for that stream.
 *   workspace  device pointer, 256-byte aligned, or NULL: the library
 *              allocates its own again on the next call that needs it.
 *   bytes      its size (at least 256); a later call whose workspace
 *              (bitsort_workspace_bytes, bitsort_radix_workspace_bytes;
 *              for bitsort_pairs_u32 the first rounded up to 256 plus
 *              4 * 2^range_bits) is larger returns BITSORT_ERR_NO_MEMORY
 *              and allocates nothing.
 * The caller owns the memory, keeps it alive and leaves it alone while work
 * enqueued on `stream` may still use it; the library never frees it.  A
 * workspace the library had allocated for the stream is freed here (after
 * synchronising `stream`).  The status of calls made before this one can no
 * longer be read.
 */
int bitsort_set_workspace(void *workspace, size_t bytes, bitsort_stream_t stream);

/* Synchronise `stream`, then copy the status held in a caller workspace. */
int bitsort_workspace_status(const void *workspace, bitsort_stream_t stream,
                             bitsort_status_t *status);

/*
 * Segmented sort: num_segments independent arrays sorted by one persistent
 * launch (each segment is the problem of bitsort_u32 with its own range: the
 * ascending arrangement of Section IV and Theorem 1, by the marking of Table I
 * and Examples 2-3, the counting of Example 6 and the bit test of Example 1).
 *   keys          device uint32, offsets[num_segments] elements in all.
 *   offsets       device uint64[num_segments + 1]; offsets[0] = 0 and
 *                 non-decreasing; segment s is keys[offsets[s] .. offsets[s+1]).
 *   num_segments  1 .. BITSORT_BATCH_MAX_SEGMENTS.
 *   range_bits    device uint8[num_segments], each 0..BITSORT_BATCH_MAX_RANGE_BITS.
 *   out           device uint32, same length as keys; must not overlap keys.
 *   max_keys      host: the number of elements allocated for keys and for
 *                 out.  A segment reaching past it is skipped and flagged
 *                 BITSORT_STATUS_BAD_SEGMENT; also used for the overlap check.
 * Segment s's sorted keys land in out[offsets[s] .. offsets[s] + d_s).  The
 * segment sizes are read on the device, so the host never waits.  Per-segment
 * statuses: bitsort_batch_status().  A segment with a decreasing offset or a
 * range_bits above the limit is skipped and flagged BITSORT_STATUS_BAD_SEGMENT.
 * With a duplicate key, the segment's output slots are unspecified (writes
 * stay inside the segment) and BITSORT_STATUS_DUPLICATE is set.
 */
#define BITSORT_BATCH_MAX_RANGE_BITS 24
#define BITSORT_BATCH_MAX_SEGMENTS (1u << 24)
#define BITSORT_STATUS_BAD_SEGMENT 4u
int bitsort_batch_u32(const uint32_t *keys, const uint64_t *offsets, uint32_t num_segments,
                      const uint8_t *range_bits, uint32_t *out, uint64_t max_keys,
                      bitsort_stream_t stream);

/* Synchronise `stream`, then copy per-segment statuses of the last
 * bitsort_batch_u32 on it into host status[0 .. num_segments). */
int bitsort_batch_status(bitsort_stream_t stream, bitsort_status_t *status, uint32_t num_segments);

/*
 * The segmented sort in two steps, for callers that capture the sort into
 * their own HIP graph or must not allocate while it runs.  The problem is
 * bitsort_batch_u32's (Section IV, Theorem 1, per segment).
 *
 * bitsort_batch_plan checks the segments on the host and sets up the work:
 *   offsets     HOST uint64[num_segments + 1], offsets[0] = 0, non-decreasing.
 *   range_bits  HOST uint8[num_segments], each 0..BITSORT_BATCH_MAX_RANGE_BITS,
 *               with offsets[s+1] - offsets[s] <= 2^range_bits[s].
 *   plan        receives the plan; it owns a device workspace (allocated here,
 *               on the current device, freed by bitsort_batch_plan_destroy).
 * Errors: BITSORT_ERR_INVALID_ARG (null pointers, num_segments out of
 * 1..BITSORT_BATCH_MAX_SEGMENTS, offsets[0] != 0, a decreasing offset, a
 * width above the limit), BITSORT_ERR_TOO_LARGE (a segment longer than its
 * range, 2^40 keys or more in all), BITSORT_ERR_NO_MEMORY.
 *
 * bitsort_batch_run enqueues the sort: keys/out as bitsort_batch_u32 (the
 * plan's offsets[num_segments] elements each, no overlap), offsets and
 * range_bits the DEVICE copies of the arrays given to the plan.  It allocates
 * nothing and makes no memset or host synchronisation, so it can be stream-
 * captured; runs of one plan share its workspace and must not overlap in
 * time.  Call on the plan's device.  bitsort_batch_plan_status synchronises
 * `stream` and copies the per-segment statuses of the plan's last run (count
 * <= num_segments).
 */
typedef struct bitsort_batch_plan bitsort_batch_plan_t;
int bitsort_batch_plan(const uint64_t *offsets, const uint8_t *range_bits, uint32_t num_segments,
                       bitsort_batch_plan_t **plan);
int bitsort_batch_run(const bitsort_batch_plan_t *plan, const uint32_t *keys, const uint64_t *offsets,
                      const uint8_t *range_bits, uint32_t *out, bitsort_stream_t stream);
int bitsort_batch_plan_status(const bitsort_batch_plan_t *plan, bitsort_stream_t stream, bitsort_status_t *status,
                              uint32_t count);
int bitsort_batch_plan_destroy(bitsort_batch_plan_t *plan);

/*
 * Pointer-array batch: count independent arrays, each sorted by the plain
 * path's method (partition into LDS slices, mark by shift and OR -- Table I,
 * Examples 2-3 --, count ones -- Example 6 --, emit set bits -- Example 1),
 * each array's result its ascending arrangement (Theorem 1), all arrays in
 * one launch of each kernel -- any range_bits up to 32 per array, and every
 * key read once by the partition (the segmented launch above reads a segment
 * once per 2^20-bit slice of its range).  An array emits from LDS, or, when
 * range_bits >= 21 and its bit-vector is at most twice its keys' bytes
 * (2^range_bits / 8 <= 2 n), through a bit-vector in the workspace and one
 * more launch that emits every such array's words.
 *
 *   keys, out    host arrays of count device pointers; array a is keys[a][0 ..
 *                n[a]) and its result goes to out[a][0 .. n[a]).  out[a] ==
 *                keys[a] is allowed; any other overlap between an array's
 *                input and output is rejected; different arrays must not share
 *                memory.
 *   n            host array of count sizes, n[a] <= 2^range_bits[a], < 2^32.
 *   range_bits   host array of count widths, 0..32.
 *   count        1 .. BITSORT_BATCH_MAX_SEGMENTS.
 *   stream       HIP stream; the call enqueues work (the host arrays may be
 *                reused as soon as it returns).
 *
 * Per-array status (flags and keys written) with bitsort_batch_status on the
 * same stream, as for bitsort_batch_u32.  Errors as bitsort_u32, checked per
 * array on the host.
 */
int bitsort_batch_ptr_u32(const uint32_t *const *keys, const uint64_t *n, const uint8_t *range_bits,
                          uint32_t *const *out, uint32_t count, bitsort_stream_t stream);

/*
 * LSD radix sort of arbitrary uint32 keys, duplicates kept: the paper's own
 * sort (Algorithm 1, Section V; correctness by Theorem 1), a stable partition
 * by each key bit from bit 0 up, run here as ceil(key_bits / 8) stable passes
 * over 8-bit digits (eight consecutive one-bit stable partitions order the
 * keys exactly as one stable pass over their 8-bit digit).
 *
 *   keys      device pointer to n uint32 keys (any values; read only).
 *   n         number of keys, n < 2^30.
 *   key_bits  0..32: the keys are ordered by their low key_bits bits, stably
 *             (the order Algorithm 1 gives after key_bits passes).  A key
 *             with a bit set at or above key_bits raises
 *             BITSORT_STATUS_OUT_OF_RANGE; it is still written, placed by its
 *             low bits.  Use 32 for arbitrary keys.
 *   out       device pointer to n uint32 (written): the keys in that order.
 *             out == keys is allowed; any other overlap is rejected.
 *   stream    HIP stream; the call only enqueues work.
 *
 * Status (bitsort_get_status on the same stream): count = n, flags as above;
 * BITSORT_STATUS_TIMEOUT if a workgroup's wait for an earlier one gave up.
 * Errors: BITSORT_ERR_INVALID_ARG (key_bits > 32, null pointers with n > 0,
 * partial overlap), BITSORT_ERR_TOO_LARGE (n >= 2^30), BITSORT_ERR_NO_MEMORY.
 * Workspace: grown per stream like bitsort_u32's (4n bytes plus n/8 bytes of
 * look-back state per pass); the _ws form takes the caller's (256-byte
 * aligned, bitsort_radix_workspace_bytes(n, key_bits) bytes, status readable
 * with bitsort_workspace_status).
 */
int bitsort_radix_u32(const uint32_t *keys, uint64_t n, uint32_t key_bits, uint32_t *out, bitsort_stream_t stream);
size_t bitsort_radix_workspace_bytes(uint64_t n, uint32_t key_bits);
int bitsort_radix_u32_ws(const uint32_t *keys, uint64_t n, uint32_t key_bits, uint32_t *out, void *workspace,
                         size_t ws_bytes, bitsort_stream_t stream);

/*
 * Multiset sort by counting: keys in [0, 2^range_bits) that may repeat,
 * written out ascending with every repeat kept (counting sort, which the
 * paper sets beside its own method; the result equals Algorithm 1's for
 * in-range keys).  The bitmap path's partition routes keys to slices of
 * 2^sb keys; each slice keeps one 32-bit counter per key in LDS instead of
 * one bit, and writes each key as many times as it was counted.
 *
 *   keys        device pointer to n uint32 keys (read only).
 *   n           number of keys, n < 2^32.
 *   range_bits  0..27 (at most 2^12 slices of 2^15 counters).
 *   out         device pointer to n uint32: out[0..count) receives the kept
 *               keys ascending with repeats; out == keys is allowed, any other
 *               overlap is rejected.
 *   stream      HIP stream; the call only enqueues work.
 *
 * Keys >= 2^range_bits are dropped and raise BITSORT_STATUS_OUT_OF_RANGE
 * (out[count..n) is then left unspecified); count = number of kept keys.
 * Status with bitsort_get_status on the same stream.  Errors:
 * BITSORT_ERR_INVALID_ARG (range_bits > 27, null pointers with n > 0, partial
 * overlap), BITSORT_ERR_TOO_LARGE (n >= 2^32), BITSORT_ERR_NO_MEMORY.
 */
int bitsort_count_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits, uint32_t *out, bitsort_stream_t stream);

/*
 * LSD radix sort of arbitrary int32 keys, duplicates kept: the order of the
 * paper's BitwiseSort (Section V: negative keys first, each sign group sorted
 * by BitwiseSort1 over its low 31 bits), which is the order of the keys with
 * their sign bit flipped read as unsigned.  The digits are taken from
 * key ^ 2^31; the keys themselves move unchanged.  Four passes; arguments,
 * errors, status and workspace as bitsort_radix_u32 with key_bits = 32.
 */
int bitsort_radix_i32(const int32_t *keys, uint64_t n, int32_t *out, bitsort_stream_t stream);

/*
 * The radix sort for T = uint64 (Algorithm 1 is written for any integer type
 * T with 8 * sizeof(T) bit passes): keys ordered by their low key_bits bits
 * (0..64), ceil(key_bits / 8) passes, duplicates kept.  keys/out are device
 * pointers to n uint64; everything else as bitsort_radix_u32 (status on the
 * stream, out == keys allowed, n < 2^30).
 */
int bitsort_radix_u64(const uint64_t *keys, uint64_t n, uint32_t key_bits, uint64_t *out, bitsort_stream_t stream);

/*
 * Key-value radix sort: records (keys[i], values[i]) ordered by the low
 * key_bits bits of the key, stably -- the partition of Algorithm 1 moves the
 * whole record, so each value travels with its key and records with equal
 * keys keep their input order.  All four arrays are device pointers to n
 * uint32.  out_keys == keys and out_values == values are allowed; any other
 * overlap among the outputs and between an output and an input is rejected.
 * Otherwise as bitsort_radix_u32.
 */
int bitsort_radix_pairs_u32(const uint32_t *keys, const uint32_t *values, uint64_t n, uint32_t key_bits,
                            uint32_t *out_keys, uint32_t *out_values, bitsort_stream_t stream);

/*
 * Bitmap sort of (key, value) records: Section V's element type T taken as a
 * record ordered by its key, sorted by the marking, counting and emission of
 * bitsort_u32 (Table I, Examples 2-3, 6 and 1; Theorem 1: with distinct keys
 * the ascending arrangement, values included, is unique).
 *   keys, values      device arrays of n uint32 each, record i = (keys[i],
 *                     values[i]); keys below 2^range_bits;
 *   out_keys          as bitsort_u32 writes them;
 *   out_values[j]     the value that came with out_keys[j].
 * A record goes to its key's rank among the distinct keys.  Inputs of more
 * than 8192 keys at a density above 1/256 stage the records by slice and
 * place each value at its key's rank in LDS (workspace about 8n bytes);
 * smaller or sparser ones carry the values on a table of one word per
 * possible key (the plain workspace plus 4 * 2^range_bits bytes, touched
 * only where keys fall), where bitsort_radix_pairs_u32 can be faster.  range_bits <= 30
 * (BITSORT_ERR_INVALID_ARG otherwise).  Status (bitsort_get_status) as for
 * bitsort_u32; a repeated key keeps one of its values (which one is
 * unspecified); entries past the status count are unspecified, as for the
 * keys.  out_keys may equal keys and out_values may equal values; any other
 * overlap among the four arrays, or a null array with n > 0, is
 * BITSORT_ERR_INVALID_ARG.  Stream-ordered, allocation only when the
 * workspace grows: once a call has grown the stream's workspace, later calls
 * of that size on the stream can be captured into a HIP graph.
 */
int bitsort_pairs_u32(const uint32_t *keys, const uint32_t *values, uint64_t n, uint32_t range_bits,
                      uint32_t *out_keys, uint32_t *out_values, bitsort_stream_t stream);

/*
 * Device-side input generator (the synthetic workloads): out[i] = pi(first + i)
 * for i < count, where pi is the seeded keyed permutation of [0, 2^range_bits)
 * (4-round alternating Feistel network over halves of ceil(range_bits/2) and
 * floor(range_bits/2) bits; round keys from SplitMix64).
 * Gives distinct keys in pseudo-random order.  first + count <= 2^range_bits.
 */
int bitsort_generate_u32(uint32_t *out, uint64_t first, uint64_t count, uint32_t range_bits,
                         uint64_t seed, bitsort_stream_t stream);

/*
 * Diagnostics that run the same device code as bitsort_u32 and stop at an
 * intermediate step, for tests:
 * - bitsort_debug_bitmap_u32: the mark step; writes the whole bit-vector,
 *   max(1, 2^range_bits / 32) uint32 words, to device `bitmap` (word w bit b
 *   set iff key 32w + b occurred).
 * - bitsort_debug_prefix_u32: the scan step; writes, for every word w, the
 *   number of set bits in words 0 .. w-1 to device uint64 `prefix` (one entry
 *   per word).
 * Both need range_bits <= 30 (the dump must fit in memory comfortably).
 */
int bitsort_debug_bitmap_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits,
                             uint32_t *bitmap, bitsort_stream_t stream);
int bitsort_debug_prefix_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits,
                             uint64_t *prefix, bitsort_stream_t stream);
/*
 * - bitsort_debug_split_u32: after bitsort_u32_ws(keys, n, range_bits, ...,
 *   workspace, ..., stream), synchronises `stream` and writes to host
 *   *published how many slices that sort found heavy and published for
 *   sharing among workgroups (bit-vector route; the first 64 are shared, the
 *   rest stay whole); 0 when the plan for (n, range_bits) does not share
 *   slices.  Reads 4 bytes of the workspace; changes nothing.
 */
int bitsort_debug_split_u32(const void *workspace, uint64_t n, uint32_t range_bits, uint32_t *published,
                            bitsort_stream_t stream);

/*
 * Tuning knobs for the plain path (0 = library default).
 *   slice_bits  bits of key range per LDS slice (10..20);
 *   tile_log2   keys per partition tile as a power of two (12..15);
 *   emit_path   1: emit each slice from LDS (k_slice), scanning every word;
 *               2: write the bit-vector to HBM and emit from it at full
 *               occupancy (k_slice + k_emit, needs slice_bits >= 15);
 *               3: emit from LDS through a summary bit per word, reading only
 *               nonzero words (needs slice_bits = 20);
 *               4: path 2, and a slice holding more than four times the mean
 *               keys (at least 2^16) is cut into up to 4 chunks of tiles that
 *               workgroups done with their own slices mark into partial
 *               slices and OR together; for skewed keys.  The workspace
 *               grows by 256 partial slices (2^(slice_bits-3) bytes each:
 *               32 MiB at 2^20-bit slices), which bitsort_workspace_bytes
 *               includes;
 *               0: choose by size (the HBM bit-vector when R/8 <= 2n, the
 *               summary when n <= R/32 and the slice has 2^20 bits).
 * Affects calls made afterwards in this process.
 */
int bitsort_set_tuning(uint32_t slice_bits, uint32_t tile_log2, uint32_t emit_path);

/* The slice_bits, tile_log2 (0 for the single-workgroup path), number of
 * slices and emit path (0 single workgroup, 1 LDS, 2 HBM bit-vector, 3 LDS
 * through the word summary, 4 HBM bit-vector with heavy slices shared) that
 * the plain path would use for (n, range_bits). */
int bitsort_plan_info(uint64_t n, uint32_t range_bits, uint32_t *slice_bits, uint32_t *tile_log2,
                      uint32_t *buckets, uint32_t *emit_path);

/*
 * HIP graphs: the launches of one sort (plain or batch) captured once and
 * replayed on any stream with bitsort_graph_launch().  Each replay computes
 * what bitsort_u32 or bitsort_batch_u32 computes (Section IV, Theorem 1: the
 * ascending arrangement; marking by Table I and Examples 2-3, counting by
 * Example 6, emission by Example 1).  The device buffers are
 * fixed at creation; their contents may change between replays (a batch is
 * re-planned on the device at every replay).  A graph owns its workspace, so
 * replays allocate nothing.  Replays of one graph must not overlap in time.
 *   bitsort_graph_status  synchronises `stream`, then copies the status of the
 *                         last replay: one entry for a plain graph, up to
 *                         num_segments for a batch graph.
 */
typedef struct bitsort_graph bitsort_graph_t;
int bitsort_graph_create_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits, uint32_t *out,
                             bitsort_graph_t **graph);
int bitsort_graph_create_batch_u32(const uint32_t *keys, const uint64_t *offsets, uint32_t num_segments,
                                   const uint8_t *range_bits, uint32_t *out, uint64_t max_keys,
                                   bitsort_graph_t **graph);
int bitsort_graph_launch(bitsort_graph_t *graph, bitsort_stream_t stream);
int bitsort_graph_status(bitsort_graph_t *graph, bitsort_stream_t stream, bitsort_status_t *status,
                         uint32_t count);
int bitsort_graph_destroy(bitsort_graph_t *graph);

/*
 * Autotuning.  bitsort_autotune_u32 times every valid (slice_bits,
 * tile_log2, emit_path) on a generated input of n keys in [0, 2^range_bits)
 * (reps timed runs each, HIP events on `stream`; it allocates and frees its
 * own buffers) and makes the fastest the default for inputs with the same
 * range_bits and ceil(log2 n).  bitsort_autotune_batch_u32 times the batch
 * kernel's workgroup size (256/512/1024) and LDS slice bits (16..20) on the
 * caller's batch (out is overwritten) and makes the fastest the default.
 * Explicit bitsort_set_tuning values still take precedence.
 * bitsort_tuning_save/load write and read the chosen settings as JSON lines
 * keyed by GPU architecture and CU count (entries for another device are
 * ignored on load); bitsort_tuning_clear forgets them.
 */
typedef struct bitsort_tuning {
    uint32_t slice_bits;  /* plain and batch */
    uint32_t tile_log2;   /* plain */
    uint32_t emit_path;   /* plain: 1 LDS, 2 HBM bit-vector, 3 LDS with word summary */
    uint32_t batch_block; /* batch: workgroup size */
    float ms;             /* measured time per call */
} bitsort_tuning_t;

int bitsort_autotune_u32(uint64_t n, uint32_t range_bits, int reps, bitsort_stream_t stream,
                         bitsort_tuning_t *best);
int bitsort_autotune_batch_u32(const uint32_t *keys, const uint64_t *offsets, uint32_t num_segments,
                               const uint8_t *range_bits, uint32_t *out, uint64_t max_keys, int reps,
                               bitsort_stream_t stream, bitsort_tuning_t *best);
int bitsort_tuning_save(const char *path);
int bitsort_tuning_load(const char *path, int *entries);
int bitsort_tuning_clear(void);

/*
 * Serving loop: continuous batching of sort requests under a device-memory
 * budget.  Request i names a synthetic input -- n keys pi(0 .. n-1) of the
 * seeded keyed permutation of [0, 2^range_bits), the bitsort_generate_u32
 * generator -- and an arrival time.  The loop admits requests in arrival
 * order as launch slots and memory free up, materialises their keys on the
 * device, and sorts them: consecutive requests with range_bits <=
 * plain_range_bits together in one segmented launch (bitsort_batch_u32's
 * kernels), consecutive wider requests of fewer than 2^23 keys together in
 * one pointer-array launch (bitsort_batch_ptr_u32's kernels: the partition
 * reads every key once however wide the range), and a wider request of 2^23
 * keys or more alone through the plain path -- a launch takes at most
 * max_batch_requests requests and, unless one request alone exceeds it,
 * max_batch_keys keys; up to
 * `streams` launches are in flight at once, each on its own stream.  The
 * memory of a launch (keys, output, workspace) is one region of an arena of
 * budget_bytes, held until the launch finishes.  The arena is the caller's
 * device memory at `arena` (256-byte aligned, not touched by anything else
 * during the call) or, when that is NULL, allocated and freed by the call.  Requests that arrive while
 * others run are admitted as soon as a slot and memory are free.  A request
 * that cannot fit the budget on its own is rejected.  The call blocks until
 * every request is done (real time: arrivals are released at arrival_s
 * seconds after the start; simulate = 1 runs the same scheduler on a virtual
 * clock with no GPU, the device serving launches one after another in
 * sim_overhead_s + keys / sim_keys_per_s).  With verify = 1 each request's
 * result carries the digest of its sorted output (see bitsort_digest_u32), so
 * it can be compared with the same request sorted alone.  Times are seconds
 * from the start of the call; GPU-side times come from HIP events.
 */
#define BITSORT_REQ_REJECTED 8u  /* result flag: larger than the whole budget */
#define BITSORT_REQ_INVALID 16u  /* result flag: range_bits > 32 or n > 2^range_bits */

typedef struct bitsort_request {
    uint64_t n;
    uint32_t range_bits;
    uint32_t _pad;
    uint64_t seed;
    double arrival_s;
} bitsort_request_t;

typedef struct bitsort_request_result {
    double launch_s;  /* left the queue: memory reserved and its launch enqueued */
    double ready_s;   /* its keys were materialised on the GPU (the sort starts after this) */
    double done_s;    /* its launch finished on the GPU */
    uint64_t digest;  /* digest of its sorted output (verify = 1), else 0 */
    uint64_t count;   /* keys written */
    uint32_t flags;   /* BITSORT_STATUS_* | BITSORT_REQ_* */
    uint32_t batch;   /* index of the launch that carried it */
} bitsort_request_result_t;

typedef struct bitsort_serve_config {
    void *arena;                 /* device memory of budget_bytes for the arena, or NULL: allocated per call */
    uint64_t budget_bytes;
    uint32_t streams;            /* 1 .. 16 */
    uint32_t max_batch_requests; /* >= 1 */
    uint64_t max_batch_keys;     /* >= 1 */
    uint32_t plain_range_bits;   /* narrower requests share segmented launches; 0: 20, at most 24 */
    uint32_t verify;
    uint32_t simulate;
    uint32_t _pad;
    double sim_overhead_s;
    double sim_keys_per_s;
    uint32_t *const *outputs;    /* NULL, or a host array of `count` device pointers: request i's sorted keys
                                    (results[i].count of them) are copied to outputs[i] (NULL: not copied)
                                    on its launch's stream before the launch counts as done */
} bitsort_serve_config_t;

typedef struct bitsort_serve_stats {
    double makespan_s;              /* first arrival to last completion */
    uint64_t keys;                  /* keys written in all */
    uint32_t launches;
    uint32_t max_inflight_requests;
    uint64_t peak_bytes;            /* most arena bytes held at once */
} bitsort_serve_stats_t;

int bitsort_serve_run(const bitsort_request_t *requests, uint32_t count, const bitsort_serve_config_t *config,
                      bitsort_request_result_t *results, bitsort_serve_stats_t *stats);

/* Order-dependent digest of n uint32 values on the device:
 * sum over i of SplitMix64_finalizer((i << 32) ^ data[i] + 0x9E3779B97F4A7C15)
 * modulo 2^64.  Synchronises `stream`; *digest is a host pointer. */
int bitsort_digest_u32(const uint32_t *data, uint64_t n, uint64_t *digest, bitsort_stream_t stream);

/*
 * Kernel timing for benchmarks.  While enabled, every kernel the library
 * launches is bracketed by two HIP events recorded on the launch's own
 * stream.  bitsort_profile_read() waits for those events and returns, per
 * kernel name, the number of launches and their summed duration since the
 * last reset (at most max_entries entries; *n_entries receives the count).
 * Enabling costs two event records per kernel launch.
 */
typedef struct bitsort_profile_entry {
    char kernel[32];      /* k_partition, k_slice, k_emit, k_finish, k_direct, k_batch_plan, k_batch_run,
                             k_radix_hist, k_radix_scan, k_radix_pass, k_count_slice,
                             k_partition_multi, k_slice_multi, k_finish_multi */
    uint64_t launches;
    double total_ms;
} bitsort_profile_entry_t;

int bitsort_profile_enable(int on);
int bitsort_profile_reset(void);
int bitsort_profile_read(bitsort_profile_entry_t *entries, int max_entries, int *n_entries);

#ifdef __cplusplus
}
#endif

#endif /* BITSORT_H */
