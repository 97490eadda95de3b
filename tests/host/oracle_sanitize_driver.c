/* Drives every entry point of the CPU oracle over many shapes and operation
 * sequences so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (host code only) checks its memory accesses and arithmetic.  The two internal
 * forms (lists, buckets) are cross-checked after every operation with orc_check.
 * Prints "ok <operations>" on success; a sanitizer report or a failed check
 * ends the program with a non-zero status. */
#include "../../oracle/ggoracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t rnd(void)
{
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return rng_state >> 11;
}

#define CHECK(cond)                                                         \
    do {                                                                    \
        if (!(cond)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                       \
        }                                                                   \
    } while (0)

int main(void)
{
    static const uint32_t elems[] = {4, 8};
    static const uint32_t vs[] = {1, 3, 64};
    static const uint64_t fs[] = {1, 2, 1024};
    uint64_t thr[16];
    for (int k = 0; k < 16; k++)
        thr[k] = (uint64_t)(k + 1) << 59 | (uint64_t)k;
    uint64_t ops = 0;
    for (int ie = 0; ie < 2; ie++)
        for (int iv = 0; iv < 3; iv++)
            for (int jf = 0; jf < 3; jf++) {
                const uint32_t eb = elems[ie], V = vs[iv];
                orc_array *a = orc_create(eb, V, fs[jf], ORC_FORM_LIST | ORC_FORM_BUCKETS);
                CHECK(a != NULL);
                for (int step = 0; step < 24; step++, ops++) {
                    const uint64_t n = rnd() % 3000;
                    const int kind = (int)(rnd() % 8);
                    if (kind == 0) {
                        uint64_t *vals = (uint64_t *)malloc(8 * (n + 1));
                        uint8_t *flags = (uint8_t *)malloc(n + 1);
                        for (uint64_t i = 0; i < n; i++) {
                            vals[i] = rnd();
                            flags[i] = (uint8_t)(rnd() & 1);
                        }
                        CHECK(orc_insert(a, vals, (rnd() & 1) ? flags : NULL, n) == ORC_OK);
                        free(vals);
                        free(flags);
                    } else if (kind == 1) {
                        const uint32_t mx = 1 + (uint32_t)(rnd() % 16);
                        uint64_t *vals = (uint64_t *)malloc(8 * (n * mx + 1));
                        uint8_t *counts = (uint8_t *)malloc(n + 1);
                        for (uint64_t i = 0; i < n * mx; i++)
                            vals[i] = rnd();
                        for (uint64_t i = 0; i < n; i++)
                            counts[i] = (uint8_t)(rnd() % 20);
                        CHECK(orc_insert_counts(a, vals, counts, mx, n) == ORC_OK);
                        /* the same counts (up to 19) against the packed layout: enough
                         * values, then one value short of them */
                        uint64_t need = 0;
                        for (uint64_t i = 0; i < n; i++)
                            need += counts[i];
                        uint64_t *pk = (uint64_t *)malloc(8 * (need + 1));
                        for (uint64_t i = 0; i < need; i++)
                            pk[i] = rnd();
                        CHECK(orc_insert_packed(a, pk, need, counts, n) == ORC_OK);
                        if (need)
                            CHECK(orc_insert_packed(a, pk, need - 1, counts, n) == ORC_ERANGE);
                        free(pk);
                        free(vals);
                        free(counts);
                    } else if (kind == 2) {
                        const uint32_t g = 1 + (uint32_t)(rnd() % 4);
                        const uint32_t shift = g == ORC_GEN_KEYED ? 32 : 20;
                        CHECK(orc_insert_gen(a, g, rnd() % 256, (uint32_t)(rnd() % 8), shift, 16, thr, n,
                                             rnd() % 64) == ORC_OK);
                    } else if (kind == 3) {
                        const uint32_t den = 1 + (uint32_t)(rnd() % 7);
                        CHECK(orc_shrink(a, (uint32_t)(rnd() % (den + 1)), den) == ORC_OK);
                    } else if (kind == 4) {
                        CHECK(orc_rw(a, (uint32_t)(rnd() % 3)) == ORC_OK);
                    } else if (kind == 5) {
                        const uint64_t s = orc_size(a);
                        uint8_t *out = (uint8_t *)malloc(eb * (s + 1));
                        CHECK(orc_flatten(a, out, s) == ORC_OK);
                        if (s)
                            CHECK(orc_flatten(a, out, s - 1) == ORC_ERANGE);
                        free(out);
                    } else if (kind == 6) {
                        const uint64_t s = orc_size(a), m = 1 + rnd() % 100;
                        uint64_t *idx = (uint64_t *)malloc(8 * m);
                        uint8_t *out = (uint8_t *)malloc(eb * m);
                        for (uint64_t i = 0; i < m; i++)
                            idx[i] = rnd() % (s + 5);
                        (void)orc_gather(a, idx, m, out);
                        uint64_t x;
                        for (uint64_t i = 0; i < m; i++)
                            (void)orc_at(a, idx[i], &x);
                        free(idx);
                        free(out);
                    } else {
                        uint64_t *sz = (uint64_t *)malloc(8 * V);
                        uint64_t *pre = (uint64_t *)malloc(8 * (V + 1));
                        uint32_t *nb = (uint32_t *)malloc(4 * V);
                        orc_vector_sizes(a, sz);
                        orc_prefix(a, pre);
                        orc_vector_nbuckets(a, nb);
                        CHECK(pre[V] == orc_size(a));
                        (void)orc_capacity(a);
                        free(sz);
                        free(pre);
                        free(nb);
                    }
                    CHECK(orc_check(a) == 0);
                }
                orc_destroy(a);
            }
    uint32_t b;
    uint64_t off;
    for (uint64_t i = 0; i < 100000; i++, ops++)
        orc_walk(1ull << (rnd() % 15), rnd() % (1ull << 40), &b, &off);
    printf("ok %llu\n", (unsigned long long)ops);
    return 0;
}
