/*
 * Drives every entry point of the CPU oracle on seeded inputs (including the
 * edge sizes: empty input, range_bits 0, 31 and 32 bit keys, repeats, keys past
 * the range) so that an AddressSanitizer / UndefinedBehaviorSanitizer build of
 * the oracle reports any out-of-bounds access, leak, overflow or undefined
 * shift.  Test infrastructure only; checks the obvious output properties too.
 * Exit status 0 = every check held.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint32_t oracle_bit_value(uint32_t x, uint32_t i);
uint32_t oracle_power2(uint32_t n);
uint32_t oracle_count_ones(uint32_t x);
void oracle_bin_repl_i16(int16_t v, char out[17]);
uint64_t oracle_bitmap_words(uint32_t range_bits);
int oracle_bitmap_scan_u32(const uint32_t *bitmap, uint64_t words, uint64_t *prefix);
int oracle_bitmap_sort_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits, uint32_t *out,
                           uint64_t *n_out, uint32_t *flags);
int oracle_bitmap_build_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits, uint32_t *bitmap,
                            uint32_t *flags);
int oracle_bitmap_sort_u32_w64(const uint32_t *keys, uint64_t n, uint32_t range_bits, uint32_t *out,
                               uint64_t *n_out);
int oracle_bitmap_sort_u32_w8(const uint32_t *keys, uint64_t n, uint32_t range_bits, uint32_t *out,
                              uint64_t *n_out);
int oracle_bitmap_sort_segments_u32(const uint32_t *keys, const uint64_t *offsets, uint32_t num_segments,
                                    const uint8_t *range_bits, uint32_t *out, uint64_t *n_out, uint32_t *flags);
int oracle_bitwise_sort1_u32(uint32_t *A, uint64_t n, uint32_t passes);
int oracle_bitwise_sort1_u64(uint64_t *A, uint64_t n, uint32_t passes);
int oracle_bitwise_sort1_pairs_u32(uint32_t *K, uint32_t *V, uint64_t n, uint32_t passes);
int oracle_bitwise_sort_i32(int32_t *A, uint64_t n);
int oracle_counting_sort_u32(const uint32_t *keys, uint64_t n, uint32_t range_bits, uint32_t *out,
                             uint64_t *n_out, uint32_t *flags);
int oracle_bitmap_sort_u64(const uint64_t *keys, uint64_t n, uint32_t range_bits, uint64_t *out,
                           uint64_t *n_out, uint32_t *flags);

static uint64_t state = 0x13120138u;
static uint64_t next64(void)
{
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            failures++;                                                   \
        }                                                                 \
    } while (0)

static void run_bitmap(uint64_t n, uint32_t rb, int repeats, int full)
{
    uint32_t *keys = malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *out = malloc((n ? n : 1) * sizeof(uint32_t));
    const uint64_t r = (uint64_t)1 << rb;
    for (uint64_t i = 0; i < n; i++)
        keys[i] = (uint32_t)(next64() % r);
    if (repeats && n > 2)
        keys[n - 1] = keys[0];
    uint64_t d = 0;
    uint32_t flags = 0;
    CHECK(oracle_bitmap_sort_u32(keys, n, rb, out, &d, &flags) == 0);
    CHECK(d <= n);
    for (uint64_t i = 1; i < d; i++)
        CHECK(out[i - 1] < out[i]);
    if (!full) {  /* the widest ranges: only the sort itself (its bit-vector is 512 MiB) */
        free(keys), free(out);
        return;
    }
    uint64_t d64 = 0, d8 = 0;
    uint32_t *o64 = malloc((n ? n : 1) * sizeof(uint32_t)), *o8 = malloc((n ? n : 1) * sizeof(uint32_t));
    CHECK(oracle_bitmap_sort_u32_w64(keys, n, rb, o64, &d64) == 0 && d64 == d);
    CHECK(oracle_bitmap_sort_u32_w8(keys, n, rb, o8, &d8) == 0 && d8 == d);
    CHECK(memcmp(out, o64, d * 4) == 0 && memcmp(out, o8, d * 4) == 0);
    const uint64_t words = oracle_bitmap_words(rb);
    uint32_t *bm = malloc(words * sizeof(uint32_t));
    uint64_t *pre = malloc((words + 1) * sizeof(uint64_t));
    CHECK(oracle_bitmap_build_u32(keys, n, rb, bm, &flags) == 0);
    CHECK(oracle_bitmap_scan_u32(bm, words, pre) == 0 && pre[words] == d);
    uint32_t *a = malloc((n ? n : 1) * sizeof(uint32_t));
    memcpy(a, keys, n * 4);
    CHECK(oracle_bitwise_sort1_u32(a, n, 32) == 0);
    for (uint64_t i = 1; i < n; i++)
        CHECK(a[i - 1] <= a[i]);
    if (rb <= 24) {
        uint64_t c = 0;
        CHECK(oracle_counting_sort_u32(keys, n, rb, a, &c, &flags) == 0 && c == n);
    }
    free(keys), free(out), free(o64), free(o8), free(bm), free(pre), free(a);
}

int main(void)
{
    char txt[17];
    for (uint32_t i = 0; i < 32; i++)
        CHECK(oracle_bit_value(oracle_power2(i), i) == 1 && oracle_count_ones(oracle_power2(i)) == 1);
    CHECK(oracle_count_ones(0xFFFFFFFFu) == 32);
    oracle_bin_repl_i16(-32768, txt);
    CHECK(txt[0] == '1' && txt[16] == '\0');
    oracle_bin_repl_i16(32767, txt);
    CHECK(txt[0] == '0');
    const uint32_t widths[] = {0, 1, 4, 5, 6, 16, 20};
    for (unsigned w = 0; w < sizeof widths / sizeof widths[0]; w++) {
        const uint32_t rb = widths[w];
        const uint64_t cap = rb >= 12 ? 3000 : ((uint64_t)1 << rb);
        run_bitmap(0, rb, 0, 1);
        run_bitmap(cap, rb, 0, 1);
        run_bitmap(cap, rb, 1, 1);
    }
    run_bitmap(3000, 32, 1, 0);
    /* keys past the range are dropped and flagged */
    {
        uint32_t keys[5] = {1, 9, 3, 200, 7}, out[5];
        uint64_t d = 0;
        uint32_t f = 0;
        CHECK(oracle_bitmap_sort_u32(keys, 5, 4, out, &d, &f) == 0 && d == 4 && (f & 1u));
    }
    /* segments, one empty */
    {
        uint32_t keys[10] = {5, 1, 3, 9, 2, 0, 7, 4, 6, 8}, out[10];
        uint64_t offs[4] = {0, 4, 4, 10}, nout[3];
        uint8_t rbits[3] = {4, 3, 4};
        uint32_t flags[3];
        CHECK(oracle_bitmap_sort_segments_u32(keys, offs, 3, rbits, out, nout, flags) == 0);
        CHECK(nout[0] == 4 && nout[1] == 0 && nout[2] == 6);
    }
    /* Algorithm 1 on 64-bit keys, records and signed keys */
    {
        const uint64_t n = 2000;
        uint64_t *a = malloc(n * 8);
        uint32_t *k = malloc(n * 4), *v = malloc(n * 4);
        int32_t *s = malloc(n * 4);
        for (uint64_t i = 0; i < n; i++) {
            a[i] = next64();
            k[i] = (uint32_t)(next64() & 0xFFu);
            v[i] = (uint32_t)i;
            s[i] = (int32_t)(uint32_t)next64();
        }
        s[0] = INT32_MIN;
        s[1] = INT32_MAX;
        s[2] = 0;
        s[3] = -1;
        CHECK(oracle_bitwise_sort1_u64(a, n, 64) == 0);
        CHECK(oracle_bitwise_sort1_pairs_u32(k, v, n, 32) == 0);
        CHECK(oracle_bitwise_sort_i32(s, n) == 0);
        for (uint64_t i = 1; i < n; i++) {
            CHECK(a[i - 1] <= a[i]);
            CHECK(k[i - 1] < k[i] || (k[i - 1] == k[i] && v[i - 1] < v[i]));
            CHECK(s[i - 1] <= s[i]);
        }
        CHECK(oracle_bitwise_sort1_u64(a, 0, 64) == 0 && oracle_bitwise_sort_i32(s, 0) == 0);
        free(a), free(k), free(v), free(s);
    }
    /* 64-bit bitmap sort over 36 bits */
    {
        uint64_t keys[4] = {((uint64_t)1 << 36) - 1, 5, (uint64_t)1 << 35, (uint64_t)1 << 36}, out[4], d = 0;
        uint32_t f = 0;
        CHECK(oracle_bitmap_sort_u64(keys, 4, 36, out, &d, &f) == 0 && d == 3 && (f & 1u));
        CHECK(out[0] == 5 && out[2] == ((uint64_t)1 << 36) - 1);
    }
    if (failures)
        fprintf(stderr, "%d check(s) failed\n", failures);
    return failures ? 1 : 0;
}
