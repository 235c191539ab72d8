/*
 * bitsort_oracle.c -- CPU oracle for the bitmap sort and for the paper's own
 * "Bitwise sorting" (Algorithm 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, single-threaded, deliberately unoptimised
 * C99.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with the
 * HIP library, and the library never calls it.
 *
 * Source: K. Yordzhev, "The bitwise operations related to a fast sorting
 * algorithm", arXiv:1312.0138.  Facts used, by section:
 *   S2  bits are numbered right to left; the rightmost bit is bit 0.
 *   S2, Table I   truth table of &, |, ^, ~ : OR-ing a 1 sets a bit, and
 *                 1 | 1 = 1, so marking twice is the same as marking once.
 *   S2  x << k multiplies by 2^k; shifts should be done on unsigned values.
 *   S3, Example 1 value of bit i of x: (x & 1<<i) != 0.
 *   S3, Example 2 2^n computed as 1 << n.
 *   S3, Example 3 division by 2^n with a right shift.
 *   S3, Example 4 the bits of a 16-bit two's-complement number, MSB first
 *                 (Table II lists fifteen of them).
 *   S3, Example 6 number of ones in a word.
 *   S4  the problem: sort an integer array ascending; counting sort needs
 *       extra memory proportional to the key range.
 *   S5, Algorithm 1 BitwiseSort1: one stable partition per bit k, elements
 *       with bit k = 0 first; BitwiseSort: split by sign, sort each part,
 *       negatives first.
 *   S6, Theorem 1 the output is sorted.
 *
 * Readings taken where the paper is silent, ambiguous or wrong:
 *   O1 keys are unsigned 32-bit; 0 <= range_bits <= 32; R = 2^range_bits is
 *      held in 64 bits (2^32 does not fit in 32).
 *   O2 masks use an unsigned one (1u << b); Example 2's signed 1 << 31 is
 *      undefined in C.
 *   O3 Example 3 is read as division: word index = key >> 5, bit = key & 31.
 *   O4 ones are counted over all 32 bits of a word (Example 6 stops at bit 30).
 *   O5 on unsigned keys BitwiseSort1 runs all 32 bit passes; the listing's
 *      k < t-1 is right only inside one sign group (BitwiseSort).
 *   O6 duplicate keys: the bitmap keeps one copy.  out[0..d) holds the d
 *      distinct in-range keys ascending, ORACLE_FLAG_DUPLICATE is raised.
 *   O7 a key >= R is dropped and ORACLE_FLAG_OUT_OF_RANGE is raised.
 *   O8 a bitmap for range_bits < 5 is one partly used 32-bit word.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_NOMEM (-2)

#define ORACLE_FLAG_OUT_OF_RANGE 1u
#define ORACLE_FLAG_DUPLICATE 2u

/* ---- S3: elementary bit helpers ------------------------------------------ */

/* Example 1: the value (0 or 1) of bit i of x; bit 0 is the rightmost (S2). */
uint32_t oracle_bit_value(uint32_t x, uint32_t i)
{
    return ((x & (1u << i)) == 0) ? 0u : 1u;
}

/* Example 2: 2^n by a left shift, with an unsigned one (reading O2). */
uint32_t oracle_power2(uint32_t n)
{
    return 1u << n;
}

/* Example 6: number of ones in x, over all 32 bits (reading O4). */
uint32_t oracle_count_ones(uint32_t x)
{
    uint32_t c = 0;
    for (uint32_t i = 0; i < 32; i++)
        if (oracle_bit_value(x, i))
            c++;
    return c;
}

/* Example 4: the 16 bits of a short as text, most significant bit first. */
void oracle_bin_repl_i16(int16_t v, char out[17])
{
    uint32_t u = (uint32_t)(uint16_t)v;
    for (int d = 15; d >= 0; d--)
        out[15 - d] = oracle_bit_value(u, (uint32_t)d) ? '1' : '0';
    out[16] = '\0';
}

/* ---- the bitmap: one bit per possible key --------------------------------- */

/* Number of 32-bit words holding R = 2^range_bits bits (reading O8); 0 when
 * range_bits > 32. */
uint64_t oracle_bitmap_words(uint32_t range_bits)
{
    if (range_bits > 32)
        return 0;
    uint64_t r = (uint64_t)1 << range_bits;
    return r < 32 ? 1 : r / 32;
}

/* Mark step: bit (key & 31) of word (key >> 5) is OR-ed to one for every key
 * (Examples 2 and 3, Table I).  The bitmap must hold oracle_bitmap_words()
 * words; it is OR-ed into, not cleared.  *flags collects O6/O7. */
int oracle_bitmap_mark_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits,
                           uint32_t *bitmap, uint32_t *flags)
{
    if (range_bits > 32 || (n > 0 && (keys == NULL || bitmap == NULL)) || flags == NULL)
        return ORACLE_ERR_ARG;
    uint64_t r = (uint64_t)1 << range_bits;
    for (uint64_t i = 0; i < n; i++) {
        uint32_t k = keys[i];
        if ((uint64_t)k >= r) {
            *flags |= ORACLE_FLAG_OUT_OF_RANGE;
            continue;
        }
        uint64_t w = (uint64_t)(k >> 5);
        uint32_t m = oracle_power2(k & 31u);
        if (bitmap[w] & m)
            *flags |= ORACLE_FLAG_DUPLICATE;
        bitmap[w] = bitmap[w] | m;
    }
    return ORACLE_OK;
}

/* Scan step: prefix[w] = number of set bits in words 0..w-1, for
 * w = 0..words (so prefix[words] is the total); Example 6 per word. */
int oracle_bitmap_scan_u32(const uint32_t *bitmap, uint64_t words, uint64_t *prefix)
{
    if (prefix == NULL || (words > 0 && bitmap == NULL))
        return ORACLE_ERR_ARG;
    prefix[0] = 0;
    for (uint64_t w = 0; w < words; w++)
        prefix[w + 1] = prefix[w] + oracle_count_ones(bitmap[w]);
    return ORACLE_OK;
}

/* Emit step: for words in ascending order and bits 0..31 in ascending order
 * (S2 numbering), every set bit b of word w gives the key 32*w + b
 * (Example 1 tests the bit).  Returns the number of keys written. */
uint64_t oracle_bitmap_emit_u32(const uint32_t *bitmap, uint64_t words, uint32_t *out)
{
    uint64_t j = 0;
    for (uint64_t w = 0; w < words; w++) {
        if (bitmap[w] == 0)
            continue; /* no set bit: nothing to emit */
        for (uint32_t b = 0; b < 32; b++)
            if (oracle_bit_value(bitmap[w], b))
                out[j++] = (uint32_t)(w * 32u + b);
    }
    return j;
}

/* The whole bitmap sort of distinct keys in [0, 2^range_bits): mark, then
 * emit.  out must hold n elements and may be the same array as keys.
 * *n_out receives d, the number of keys written; *flags the O6/O7 flags.
 * out[d..n) is left as it was. */
int oracle_bitmap_sort_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits,
                           uint32_t *out, uint64_t *n_out, uint32_t *flags)
{
    if (range_bits > 32 || n_out == NULL || flags == NULL ||
        (n > 0 && (keys == NULL || out == NULL)))
        return ORACLE_ERR_ARG;
    *flags = 0;
    *n_out = 0;
    uint64_t words = oracle_bitmap_words(range_bits);
    uint32_t *bitmap = (uint32_t *)calloc((size_t)words, sizeof(uint32_t));
    if (bitmap == NULL)
        return ORACLE_ERR_NOMEM;
    int rc = oracle_bitmap_mark_u32(keys, n, range_bits, bitmap, flags);
    if (rc == ORACLE_OK)
        *n_out = oracle_bitmap_emit_u32(bitmap, words, out);
    free(bitmap);
    return rc;
}

/* Mark only, into a freshly zeroed bitmap: the state the mark step must
 * reach (used to pin the GPU's mark stage). */
int oracle_bitmap_build_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits,
                            uint32_t *bitmap, uint32_t *flags)
{
    if (range_bits > 32 || bitmap == NULL || flags == NULL)
        return ORACLE_ERR_ARG;
    *flags = 0;
    memset(bitmap, 0, (size_t)oracle_bitmap_words(range_bits) * sizeof(uint32_t));
    return oracle_bitmap_mark_u32(keys, n, range_bits, bitmap, flags);
}

/* Same sort with 64-bit words (key >> 6, key & 63).  The word width is the
 * paper's generic w of S2; the result must not depend on it. */
int oracle_bitmap_sort_u32_w64(const uint32_t *keys, uint64_t n, uint32_t range_bits,
                               uint32_t *out, uint64_t *n_out)
{
    if (range_bits > 32 || n_out == NULL || (n > 0 && (keys == NULL || out == NULL)))
        return ORACLE_ERR_ARG;
    uint64_t r = (uint64_t)1 << range_bits;
    uint64_t words = r < 64 ? 1 : r / 64;
    uint64_t *bitmap = (uint64_t *)calloc((size_t)words, sizeof(uint64_t));
    if (bitmap == NULL)
        return ORACLE_ERR_NOMEM;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t k = keys[i];
        if (k >= r)
            continue;
        bitmap[k >> 6] = bitmap[k >> 6] | ((uint64_t)1 << (k & 63));
    }
    uint64_t j = 0;
    for (uint64_t w = 0; w < words; w++) {
        if (bitmap[w] == 0)
            continue;
        for (uint64_t b = 0; b < 64; b++)
            if ((bitmap[w] & ((uint64_t)1 << b)) != 0)
                out[j++] = (uint32_t)(w * 64 + b);
    }
    *n_out = j;
    free(bitmap);
    return ORACLE_OK;
}

/* Same sort with 8-bit words (key >> 3, key & 7). */
int oracle_bitmap_sort_u32_w8(const uint32_t *keys, uint64_t n, uint32_t range_bits,
                              uint32_t *out, uint64_t *n_out)
{
    if (range_bits > 32 || n_out == NULL || (n > 0 && (keys == NULL || out == NULL)))
        return ORACLE_ERR_ARG;
    uint64_t r = (uint64_t)1 << range_bits;
    uint64_t words = r < 8 ? 1 : r / 8;
    uint8_t *bitmap = (uint8_t *)calloc((size_t)words, 1);
    if (bitmap == NULL)
        return ORACLE_ERR_NOMEM;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t k = keys[i];
        if (k >= r)
            continue;
        bitmap[k >> 3] = (uint8_t)(bitmap[k >> 3] | (1u << (k & 7)));
    }
    uint64_t j = 0;
    for (uint64_t w = 0; w < words; w++) {
        if (bitmap[w] == 0)
            continue;
        for (uint32_t b = 0; b < 8; b++)
            if ((bitmap[w] & (1u << b)) != 0)
                out[j++] = (uint32_t)(w * 8 + b);
    }
    *n_out = j;
    free(bitmap);
    return ORACLE_OK;
}

/* Segmented form: segment s holds keys[offsets[s] .. offsets[s+1]) with its own
 * range_bits[s]; each segment is sorted on its own into the same slots of out.
 * n_out[s] and flags[s] are per segment. */
int oracle_bitmap_sort_segments_u32(const uint32_t *keys, const uint64_t *offsets,
                                    uint32_t num_segments, const uint8_t *range_bits,
                                    uint32_t *out, uint64_t *n_out, uint32_t *flags)
{
    if (offsets == NULL || range_bits == NULL || n_out == NULL || flags == NULL)
        return ORACLE_ERR_ARG;
    for (uint32_t s = 0; s < num_segments; s++) {
        if (offsets[s + 1] < offsets[s])
            return ORACLE_ERR_ARG;
        int rc = oracle_bitmap_sort_u32(keys + offsets[s], offsets[s + 1] - offsets[s],
                                        range_bits[s], out + offsets[s], &n_out[s], &flags[s]);
        if (rc != ORACLE_OK)
            return rc;
    }
    return ORACLE_OK;
}

/* ---- the paper's Algorithm 1 ---------------------------------------------- */

/* One pass of Algorithm 1 (S5), written from its definition rather than from
 * the printed listing: a stable partition of src[0..n) by one bit into dst.
 * Elements whose bit `bit` equals `front` go first and the others after them,
 * each group in the order it had in src.  The size of the first group is
 * counted beforehand, so both groups are placed in a single sweep; it is
 * returned. */
static uint64_t split_by_bit_u32(const uint32_t *src, uint32_t *dst, uint64_t n, uint32_t bit, uint32_t front)
{
    uint64_t first = 0;
    for (uint64_t i = 0; i < n; i++)
        first += (oracle_bit_value(src[i], bit) == front);
    uint64_t at_front = 0, at_back = first;
    for (uint64_t i = 0; i < n; i++) {
        if (oracle_bit_value(src[i], bit) == front)
            dst[at_front++] = src[i];
        else
            dst[at_back++] = src[i];
    }
    return first;
}

/* BitwiseSort1 on unsigned 32-bit keys: for k = 0 .. passes-1, the stable
 * partition by bit k with the zeros first.  The passes alternate between A and
 * one scratch array.  passes = 32 sorts every uint32 array (reading O5);
 * fewer passes leave A ordered by its low `passes` bits (Theorem 1). */
int oracle_bitwise_sort1_u32(uint32_t *A, uint64_t n, uint32_t passes)
{
    if (passes > 32 || (n > 0 && A == NULL))
        return ORACLE_ERR_ARG;
    if (n == 0)
        return ORACLE_OK;
    uint32_t *scratch = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    if (scratch == NULL)
        return ORACLE_ERR_NOMEM;
    uint32_t *from = A, *to = scratch;
    for (uint32_t k = 0; k < passes; k++) {
        split_by_bit_u32(from, to, n, k, 0u);
        uint32_t *t = from;
        from = to;
        to = t;
    }
    if (from != A)
        memcpy(A, from, (size_t)n * sizeof(uint32_t));
    free(scratch);
    return ORACLE_OK;
}

/* The same pass for T = uint64: bit k of a 64-bit element, k < 64. */
static void split_by_bit_u64(const uint64_t *src, uint64_t *dst, uint64_t n, uint32_t k)
{
    const uint64_t mask = (uint64_t)1 << k;
    uint64_t zeros = 0;
    for (uint64_t i = 0; i < n; i++)
        zeros += ((src[i] & mask) == 0);
    uint64_t z = 0, o = zeros;
    for (uint64_t i = 0; i < n; i++) {
        if ((src[i] & mask) == 0)
            dst[z++] = src[i];
        else
            dst[o++] = src[i];
    }
}

/* BitwiseSort1 for T = uint64 (t = 64 bits): the stable partition by bit k,
 * zeros first, for k = 0 .. passes-1, passes <= 64. */
int oracle_bitwise_sort1_u64(uint64_t *A, uint64_t n, uint32_t passes)
{
    if (passes > 64 || (n > 0 && A == NULL))
        return ORACLE_ERR_ARG;
    if (n == 0)
        return ORACLE_OK;
    uint64_t *scratch = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    if (scratch == NULL)
        return ORACLE_ERR_NOMEM;
    uint64_t *from = A, *to = scratch;
    for (uint32_t k = 0; k < passes; k++) {
        split_by_bit_u64(from, to, n, k);
        uint64_t *t = from;
        from = to;
        to = t;
    }
    if (from != A)
        memcpy(A, from, (size_t)n * sizeof(uint64_t));
    free(scratch);
    return ORACLE_OK;
}

/* The pass on records (key, value): the bit test reads the key and the whole
 * record moves, so each value stays with its key. */
static void split_records_by_bit(const uint32_t *sk, const uint32_t *sv, uint32_t *dk, uint32_t *dv, uint64_t n,
                                 uint32_t k)
{
    uint64_t zeros = 0;
    for (uint64_t i = 0; i < n; i++)
        zeros += (oracle_bit_value(sk[i], k) == 0u);
    uint64_t lo = 0, hi = zeros;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t *slot = (oracle_bit_value(sk[i], k) == 0u) ? &lo : &hi;
        dk[*slot] = sk[i];
        dv[*slot] = sv[i];
        (*slot)++;
    }
}

/* BitwiseSort1 on records (K[i], V[i]): records with equal keys keep their
 * input order, since every pass is stable. */
int oracle_bitwise_sort1_pairs_u32(uint32_t *K, uint32_t *V, uint64_t n, uint32_t passes)
{
    if (passes > 32 || (n > 0 && (K == NULL || V == NULL)))
        return ORACLE_ERR_ARG;
    if (n == 0)
        return ORACLE_OK;
    uint32_t *sk = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    uint32_t *sv = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    if (sk == NULL || sv == NULL) {
        free(sk);
        free(sv);
        return ORACLE_ERR_NOMEM;
    }
    uint32_t *fk = K, *fv = V, *tk = sk, *tv = sv;
    for (uint32_t k = 0; k < passes; k++) {
        split_records_by_bit(fk, fv, tk, tv, n, k);
        uint32_t *t = fk;
        fk = tk;
        tk = t;
        t = fv;
        fv = tv;
        tv = t;
    }
    if (fk != K) {
        memcpy(K, fk, (size_t)n * sizeof(uint32_t));
        memcpy(V, fv, (size_t)n * sizeof(uint32_t));
    }
    free(sk);
    free(sv);
    return ORACLE_OK;
}

/* BitwiseSort on signed 32-bit keys (S5): first the sign split -- the
 * negatives, whose sign bit is 1, in front of the rest, each group in input
 * order -- then each group sorted by BitwiseSort1 over the t-1 = 31 bits below
 * the sign bit, which every element of a group shares. */
int oracle_bitwise_sort_i32(int32_t *A, uint64_t n)
{
    if (n > 0 && A == NULL)
        return ORACLE_ERR_ARG;
    if (n == 0)
        return ORACLE_OK;
    uint32_t *bits = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    uint32_t *grouped = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    if (bits == NULL || grouped == NULL) {
        free(bits);
        free(grouped);
        return ORACLE_ERR_NOMEM;
    }
    for (uint64_t i = 0; i < n; i++)
        bits[i] = (uint32_t)A[i];
    const uint64_t negatives = split_by_bit_u32(bits, grouped, n, 31u, 1u);
    int rc = oracle_bitwise_sort1_u32(grouped, negatives, 31);
    if (rc == ORACLE_OK)
        rc = oracle_bitwise_sort1_u32(grouped + negatives, n - negatives, 31);
    if (rc == ORACLE_OK)
        for (uint64_t i = 0; i < n; i++)
            A[i] = (int32_t)grouped[i];
    free(bits);
    free(grouped);
    return rc;
}

/* ---- counting sort (S4): keeps duplicates ---------------------------------- */

/* Counting sort of keys in [0, 2^range_bits) with range_bits <= 30: count
 * every key value, then write each value as many times as it was counted, in
 * ascending order.  Keys >= R are dropped and flagged.  *n_out receives the
 * number written. */
int oracle_counting_sort_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits,
                             uint32_t *out, uint64_t *n_out, uint32_t *flags)
{
    if (range_bits > 30 || n_out == NULL || flags == NULL ||
        (n > 0 && (keys == NULL || out == NULL)))
        return ORACLE_ERR_ARG;
    uint64_t r = (uint64_t)1 << range_bits;
    uint64_t *count = (uint64_t *)calloc((size_t)r, sizeof(uint64_t));
    if (count == NULL)
        return ORACLE_ERR_NOMEM;
    *flags = 0;
    for (uint64_t i = 0; i < n; i++) {
        if ((uint64_t)keys[i] >= r) {
            *flags |= ORACLE_FLAG_OUT_OF_RANGE;
            continue;
        }
        count[keys[i]]++;
    }
    uint64_t j = 0;
    for (uint64_t v = 0; v < r; v++)
        for (uint64_t c = 0; c < count[v]; c++)
            out[j++] = (uint32_t)v;
    *n_out = j;
    free(count);
    return ORACLE_OK;
}

/* ---- 64-bit keys ------------------------------------------------------------ */

/* Bitmap sort of distinct uint64 keys in [0, 2^range_bits), range_bits <= 36,
 * with 64-bit words.  Same conventions as oracle_bitmap_sort_u32. */
int oracle_bitmap_sort_u64(const uint64_t *keys, uint64_t n, uint32_t range_bits,
                           uint64_t *out, uint64_t *n_out, uint32_t *flags)
{
    if (range_bits > 36 || n_out == NULL || flags == NULL ||
        (n > 0 && (keys == NULL || out == NULL)))
        return ORACLE_ERR_ARG;
    uint64_t r = (uint64_t)1 << range_bits;
    uint64_t words = r < 64 ? 1 : r / 64;
    uint64_t *bitmap = (uint64_t *)calloc((size_t)words, sizeof(uint64_t));
    if (bitmap == NULL)
        return ORACLE_ERR_NOMEM;
    *flags = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t k = keys[i];
        if (k >= r) {
            *flags |= ORACLE_FLAG_OUT_OF_RANGE;
            continue;
        }
        uint64_t m = (uint64_t)1 << (k & 63);
        if (bitmap[k >> 6] & m)
            *flags |= ORACLE_FLAG_DUPLICATE;
        bitmap[k >> 6] = bitmap[k >> 6] | m;
    }
    uint64_t j = 0;
    for (uint64_t w = 0; w < words; w++) {
        if (bitmap[w] == 0)
            continue;
        for (uint64_t b = 0; b < 64; b++)
            if ((bitmap[w] & ((uint64_t)1 << b)) != 0)
                out[j++] = w * 64 + b;
    }
    *n_out = j;
    free(bitmap);
    return ORACLE_OK;
}
