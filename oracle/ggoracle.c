/*
 * CPU oracle for the GGArray hot path.
 *
 * Paper: E. Meneses, C. A. Navarro, H. Ferrada, "GGArray: A Dynamically Growable
 * GPU Array" (arXiv 2209.00103).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It includes nothing from the
 * HIP library and the HIP library includes nothing from it; the two share no code.
 *
 * What is computed.  A GGArray is an array of V LFVectors, one per thread block
 * (Sec. IV, Fig. 1-2).  As a data structure it returns exactly what a plain
 * growable array per LFVector would return, so the result of every operation has
 * a plain definition, which this file writes out twice:
 *
 *   form LIST    - one contiguous, realloc-grown array per LFVector (the plain
 *                  definition of the observable state);
 *   form BUCKETS - the LFVector of Alg. 1 / Alg. 2 taken literally: a table of
 *                  buckets, bucket b holding first_bucket * 2^b elements (the size
 *                  law of Alg. 2), allocated on first touch; an element index is
 *                  located by walking the bucket starts one by one (brute force,
 *                  no closed form).
 *
 * Readings of points the paper leaves open (each also listed in the design notes):
 *   - logical thread gid feeds LFVector floor(gid / ceil(n_threads / V))
 *     (contiguous chunks; the paper fixes one LFVector per block, Sec. IV, and
 *     allows thread coarsening, but gives no mapping);
 *   - inside a round, elements are appended in gid order, a thread's own elements
 *     contiguous and in their own order (the scan of Sec. III-B gives each
 *     inserting thread a unique index; the order itself is not stated);
 *   - the bucket size is first_bucket * 2^b with log base 2 and first_bucket a
 *     power of two (Alg. 2);
 *   - buckets are allocated lazily, so an empty LFVector owns no bucket (Alg. 1);
 *   - shrink removes floor(s * num / den) trailing elements of every LFVector and
 *     frees every bucket that starts at or past the new size (shrinking is not
 *     studied by the paper, which names it only as a generic vector feature,
 *     Sec. I);
 *   - flatten copies the LFVectors, in index order, into a contiguous buffer and
 *     leaves the GGArray unchanged (Sec. VI-C, last paragraphs; abstract);
 *   - element arithmetic wraps modulo 2^(8 * elem_bytes).
 *
 * Parity pins live in the test suite: the closed-form index mapping against the
 * brute-force walk, stream compaction, closed-form sizes and capacities, affine
 * closed forms of the r/w operations, and the published SplitMix64 vectors.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ERANGE (-3)

#define ORC_FORM_LIST 1
#define ORC_FORM_BUCKETS 2

#define ORC_MAX_BUCKETS 64

/* r/w operations of Sec. VI-C; the paper's own operation adds 1, thirty times. */
#define ORC_OP_ADD1 0
#define ORC_OP_MUL3ADD1 1
#define ORC_OP_ADD1_X30 2

/* Workload generators (payload producers of the benchmark configurations). */
#define ORC_GEN_BERNOULLI 1
#define ORC_GEN_ROUND_TAG 2
#define ORC_GEN_POISSON 3
#define ORC_GEN_KEYED 4

typedef struct {
    uint64_t len, cap;
    uint64_t *data;
} orc_list;

typedef struct {
    uint64_t size;
    uint64_t *bucket[ORC_MAX_BUCKETS];
} orc_lfvector;

typedef struct orc_array {
    uint32_t elem_bytes;
    uint32_t n_vectors;
    uint64_t first_bucket;
    uint64_t mask;
    int forms;
    orc_list *lists;
    orc_lfvector *vecs;
    uint64_t n_allocs; /* buckets allocated so far (Alg. 2 winners) */
    uint64_t n_frees;  /* buckets released by shrink */
} orc_array;

/* ------------------------------------------------------------------------- */
/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the output produced when the  */
/* generator state is x, i.e. add the golden-ratio increment, then mix.        */
/* ------------------------------------------------------------------------- */
uint64_t orc_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* K(seed, a, b) = splitmix64((seed << 56) ^ (a << 8) ^ b). */
uint64_t orc_K(uint64_t seed, uint64_t a, uint64_t b)
{
    return orc_splitmix64((seed << 56) ^ (a << 8) ^ b);
}

/* ------------------------------------------------------------------------- */
/* Bucket law (Alg. 2): bucket b holds first_bucket * 2^b elements and the     */
/* buckets of an LFVector are laid end to end in index space.  Locate index    */
/* idx by walking bucket starts; no closed form is used here.                  */
/* ------------------------------------------------------------------------- */
void orc_walk(uint64_t F, uint64_t idx, uint32_t *b_out, uint64_t *off_out)
{
    uint64_t start = 0;
    uint32_t b = 0;
    while (idx >= start + (F << b)) {
        start += F << b;
        b++;
    }
    *b_out = b;
    *off_out = idx - start;
}

/* orc_walk over an array of indices (saves one foreign call per index). */
void orc_walk_many(uint64_t F, const uint64_t *idx, uint64_t n, uint32_t *b_out, uint64_t *off_out)
{
    for (uint64_t i = 0; i < n; i++)
        orc_walk(F, idx[i], &b_out[i], &off_out[i]);
}

/* First index held by bucket b: the sum of the sizes of buckets 0..b-1. */
uint64_t orc_bucket_start(uint64_t F, uint32_t b)
{
    uint64_t start = 0;
    for (uint32_t k = 0; k < b; k++)
        start += F << k;
    return start;
}

/* Number of buckets an LFVector of s elements holds when buckets are only
 * allocated on first touch: the buckets that contain indices 0..s-1. */
uint32_t orc_nbuckets_for(uint64_t F, uint64_t s)
{
    uint32_t nb = 0;
    uint64_t covered = 0;
    while (covered < s) {
        covered += F << nb;
        nb++;
    }
    return nb;
}

static int is_pow2(uint64_t x) { return x != 0 && (x & (x - 1)) == 0; }

/* ------------------------------------------------------------------------- */
/* Lifetime                                                                    */
/* ------------------------------------------------------------------------- */
orc_array *orc_create(uint32_t elem_bytes, uint32_t n_vectors, uint64_t first_bucket, int forms)
{
    if ((elem_bytes != 4 && elem_bytes != 8) || n_vectors == 0 || !is_pow2(first_bucket) ||
        (forms & (ORC_FORM_LIST | ORC_FORM_BUCKETS)) == 0)
        return NULL;
    orc_array *a = (orc_array *)calloc(1, sizeof(orc_array));
    if (!a)
        return NULL;
    a->elem_bytes = elem_bytes;
    a->n_vectors = n_vectors;
    a->first_bucket = first_bucket;
    a->mask = elem_bytes == 4 ? 0xFFFFFFFFull : ~0ull;
    a->forms = forms;
    if (forms & ORC_FORM_LIST)
        a->lists = (orc_list *)calloc(n_vectors, sizeof(orc_list));
    if (forms & ORC_FORM_BUCKETS)
        a->vecs = (orc_lfvector *)calloc(n_vectors, sizeof(orc_lfvector));
    if (((forms & ORC_FORM_LIST) && !a->lists) || ((forms & ORC_FORM_BUCKETS) && !a->vecs)) {
        free(a->lists);
        free(a->vecs);
        free(a);
        return NULL;
    }
    return a;
}

void orc_destroy(orc_array *a)
{
    if (!a)
        return;
    if (a->lists)
        for (uint32_t v = 0; v < a->n_vectors; v++)
            free(a->lists[v].data);
    if (a->vecs)
        for (uint32_t v = 0; v < a->n_vectors; v++)
            for (int b = 0; b < ORC_MAX_BUCKETS; b++)
                free(a->vecs[v].bucket[b]);
    free(a->lists);
    free(a->vecs);
    free(a);
}

/* ------------------------------------------------------------------------- */
/* push_back on one LFVector                                                   */
/* ------------------------------------------------------------------------- */
static int list_push(orc_list *l, uint64_t e)
{
    if (l->len == l->cap) {
        uint64_t ncap = l->cap ? 2 * l->cap : 16;
        uint64_t *nd = (uint64_t *)realloc(l->data, ncap * sizeof(uint64_t));
        if (!nd)
            return ORC_ENOMEM;
        l->data = nd;
        l->cap = ncap;
    }
    l->data[l->len++] = e;
    return ORC_OK;
}

/* Alg. 1 with Alg. 2 inlined, executed by one thread at a time: the insertion
 * index is the current size, the bucket is found by walking, a missing bucket
 * of first_bucket * 2^b elements is allocated, then the element is stored. */
static int bucket_push(orc_array *a, orc_lfvector *vec, uint64_t e)
{
    uint64_t idx = vec->size;
    uint32_t b;
    uint64_t off;
    orc_walk(a->first_bucket, idx, &b, &off);
    if (b >= ORC_MAX_BUCKETS)
        return ORC_ENOMEM;
    if (vec->bucket[b] == NULL) {
        vec->bucket[b] = (uint64_t *)malloc((size_t)(a->first_bucket << b) * sizeof(uint64_t));
        if (!vec->bucket[b])
            return ORC_ENOMEM;
        a->n_allocs++;
    }
    vec->bucket[b][off] = e;
    vec->size = idx + 1;
    return ORC_OK;
}

static int push(orc_array *a, uint32_t v, uint64_t e)
{
    e &= a->mask;
    if (a->lists) {
        int st = list_push(&a->lists[v], e);
        if (st)
            return st;
    }
    if (a->vecs) {
        int st = bucket_push(a, &a->vecs[v], e);
        if (st)
            return st;
    }
    return ORC_OK;
}

static uint64_t load_elem(const void *values, uint32_t elem_bytes, uint64_t i)
{
    if (elem_bytes == 4)
        return ((const uint32_t *)values)[i];
    return ((const uint64_t *)values)[i];
}

/* Logical threads 0..n-1 are split into V contiguous chunks of ceil(n/V) threads;
 * chunk v feeds LFVector v.  Return the chunk length. */
static uint64_t chunk_len(uint64_t n_threads, uint32_t V)
{
    return (n_threads + V - 1) / V;
}

/* ------------------------------------------------------------------------- */
/* Insertion rounds.  LFVectors in index order, threads of a chunk in gid order,  */
/* a thread's own elements in their order.                                     */
/* ------------------------------------------------------------------------- */

/* Buffer mode: thread gid inserts values[gid] iff flags == NULL or flags[gid] != 0. */
int orc_insert(orc_array *a, const void *values, const uint8_t *flags, uint64_t n_threads)
{
    if (!a || (n_threads && !values))
        return ORC_EINVAL;
    if (n_threads == 0)
        return ORC_OK;
    uint64_t chunk = chunk_len(n_threads, a->n_vectors);
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        uint64_t g0 = (uint64_t)v * chunk;
        uint64_t g1 = g0 + chunk < n_threads ? g0 + chunk : n_threads;
        for (uint64_t gid = g0; gid < g1; gid++) {
            if (flags && !flags[gid])
                continue;
            int st = push(a, v, load_elem(values, a->elem_bytes, gid));
            if (st)
                return st;
        }
    }
    return ORC_OK;
}

/* Buffer mode with several elements per thread: thread gid inserts
 * values[gid * max_count + j] for j < min(counts[gid], max_count) (the library's
 * contract clamps larger counts). */
int orc_insert_counts(orc_array *a, const void *values, const uint8_t *counts, uint32_t max_count,
                      uint64_t n_threads)
{
    if (!a || (n_threads && (!values || !counts)) || max_count == 0)
        return ORC_EINVAL;
    if (n_threads == 0)
        return ORC_OK;
    uint64_t chunk = chunk_len(n_threads, a->n_vectors);
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        uint64_t g0 = (uint64_t)v * chunk;
        uint64_t g1 = g0 + chunk < n_threads ? g0 + chunk : n_threads;
        for (uint64_t gid = g0; gid < g1; gid++) {
            const uint32_t c = counts[gid] < max_count ? counts[gid] : max_count;
            for (uint32_t j = 0; j < c; j++) {
                int st = push(a, v, load_elem(values, a->elem_bytes, gid * max_count + j));
                if (st)
                    return st;
            }
        }
    }
    return ORC_OK;
}

/* Packed buffer mode: thread gid inserts counts[gid] elements, the next ones of
 * `values` in thread order (the values of all threads lie back to back, so thread
 * gid's are values[P .. P + counts[gid]) with P the sum of the counts before it).
 * The multi-element insertion of Sec. III-B with another input layout.  Counts
 * asking for more than n_values values: ORC_ERANGE, nothing inserted. */
int orc_insert_packed(orc_array *a, const void *values, uint64_t n_values, const uint8_t *counts,
                      uint64_t n_threads)
{
    if (!a || (n_threads && !counts) || (n_values && !values))
        return ORC_EINVAL;
    uint64_t total = 0;
    for (uint64_t gid = 0; gid < n_threads; gid++)
        total += counts[gid];
    if (total > n_values)
        return ORC_ERANGE;
    if (n_threads == 0)
        return ORC_OK;
    uint64_t chunk = chunk_len(n_threads, a->n_vectors);
    uint64_t next = 0; /* index of the next value to take */
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        uint64_t g0 = (uint64_t)v * chunk;
        uint64_t g1 = g0 + chunk < n_threads ? g0 + chunk : n_threads;
        for (uint64_t gid = g0; gid < g1; gid++) {
            for (uint32_t j = 0; j < counts[gid]; j++) {
                int st = push(a, v, load_elem(values, a->elem_bytes, next++));
                if (st)
                    return st;
            }
        }
    }
    return ORC_OK;
}

/* Segment append (restoring a flat snapshot): LFVector v appends
 * values[prefix[v] .. prefix[v + 1]).  An LFVector whose pair decreases, runs past
 * n_values or spans 2^32 elements or more keeps its contents and the call returns
 * ORC_ERANGE after the other LFVectors have appended theirs. */
int orc_insert_segments(orc_array *a, const void *values, const uint64_t *prefix, uint64_t n_values)
{
    if (!a || !prefix || (n_values && !values))
        return ORC_EINVAL;
    int rc = ORC_OK;
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        const uint64_t lo = prefix[v], hi = prefix[v + 1];
        if (hi < lo || hi > n_values || hi - lo >= (1ull << 32)) {
            rc = ORC_ERANGE;
            continue;
        }
        for (uint64_t i = lo; i < hi; i++) {
            int st = push(a, v, load_elem(values, a->elem_bytes, i));
            if (st)
                return st;
        }
    }
    return rc;
}

/* Generated payloads (the benchmark workloads):
 *   BERNOULLI: h = K(seed, gid, round); insert h iff its top bit is set;
 *   ROUND_TAG: insert (round << tag_shift) | gid;
 *   POISSON:   u = K(seed, gid, 0x80 | round); c = #{k < max_count : u >= thr[k]};
 *              insert K(seed, gid, 16 * round + j) for j < c;
 *   KEYED:     insert K(seed, (tag << tag_shift) | gid, round), with 1 <= tag_shift <= 47,
 *              gid < 2^tag_shift and tag < 2^(48 - tag_shift), so the key stays below 2^48.
 * Values are truncated to the element width. */
int orc_insert_gen(orc_array *a, uint32_t kind, uint64_t seed, uint32_t round, uint32_t tag_shift,
                   uint32_t max_count, const uint64_t *thresholds, uint64_t n_threads, uint64_t tag)
{
    if (!a || seed >= 256)
        return ORC_EINVAL;
    if (kind == ORC_GEN_POISSON && (!thresholds || max_count == 0 || max_count > 16 || round >= 8))
        return ORC_EINVAL;
    if (kind == ORC_GEN_ROUND_TAG && tag_shift >= 64)
        return ORC_EINVAL;
    if ((kind == ORC_GEN_BERNOULLI || kind == ORC_GEN_KEYED) && round >= 256)
        return ORC_EINVAL;
    if (kind == ORC_GEN_KEYED &&
        (tag_shift < 1 || tag_shift > 47 || (tag >> (48 - tag_shift)) != 0 || n_threads > (1ull << tag_shift)))
        return ORC_EINVAL;
    if (kind < ORC_GEN_BERNOULLI || kind > ORC_GEN_KEYED)
        return ORC_EINVAL;
    if (n_threads == 0)
        return ORC_OK;
    uint64_t chunk = chunk_len(n_threads, a->n_vectors);
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        uint64_t g0 = (uint64_t)v * chunk;
        uint64_t g1 = g0 + chunk < n_threads ? g0 + chunk : n_threads;
        for (uint64_t gid = g0; gid < g1; gid++) {
            int st = ORC_OK;
            if (kind == ORC_GEN_BERNOULLI) {
                uint64_t h = orc_K(seed, gid, round);
                if (h >> 63)
                    st = push(a, v, h);
            } else if (kind == ORC_GEN_ROUND_TAG) {
                st = push(a, v, ((uint64_t)round << tag_shift) | gid);
            } else if (kind == ORC_GEN_KEYED) {
                st = push(a, v, orc_K(seed, (tag << tag_shift) | gid, round));
            } else {
                uint64_t u = orc_K(seed, gid, 0x80u | round);
                uint32_t c = 0;
                for (uint32_t k = 0; k < max_count; k++)
                    if (u >= thresholds[k])
                        c++;
                for (uint32_t j = 0; j < c && st == ORC_OK; j++)
                    st = push(a, v, orc_K(seed, gid, 16u * round + j));
            }
            if (st)
                return st;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Shrink: every LFVector pops floor(s * num / den) elements; buckets that start */
/* at or past the new size are freed at once.                                  */
/* ------------------------------------------------------------------------- */
int orc_shrink(orc_array *a, uint32_t num, uint32_t den)
{
    if (!a || den == 0 || num > den)
        return ORC_EINVAL;
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        uint64_t s = a->lists ? a->lists[v].len : a->vecs[v].size;
        /* floor(s * num / den) without overflowing 64 bits */
        uint64_t k = (s / den) * num + ((s % den) * num) / den;
        uint64_t ns = s - k;
        if (a->lists)
            a->lists[v].len = ns;
        if (a->vecs) {
            orc_lfvector *vec = &a->vecs[v];
            vec->size = ns;
            for (uint32_t b = 0; b < ORC_MAX_BUCKETS; b++) {
                if (vec->bucket[b] && orc_bucket_start(a->first_bucket, b) >= ns) {
                    free(vec->bucket[b]);
                    vec->bucket[b] = NULL;
                    a->n_frees++;
                }
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Regular read/write over every live element (Sec. VI-B rw_b, Sec. VI-C).     */
/* ------------------------------------------------------------------------- */
static uint64_t apply_op(uint32_t op, uint64_t x, uint64_t mask)
{
    if (op == ORC_OP_ADD1)
        return (x + 1) & mask;
    if (op == ORC_OP_MUL3ADD1)
        return (x * 3 + 1) & mask;
    for (int i = 0; i < 30; i++) /* the paper's kernel adds 1, thirty times */
        x = (x + 1) & mask;
    return x;
}

int orc_rw(orc_array *a, uint32_t op)
{
    if (!a || op > ORC_OP_ADD1_X30)
        return ORC_EINVAL;
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        if (a->lists) {
            orc_list *l = &a->lists[v];
            for (uint64_t i = 0; i < l->len; i++)
                l->data[i] = apply_op(op, l->data[i], a->mask);
        }
        if (a->vecs) {
            orc_lfvector *vec = &a->vecs[v];
            for (uint64_t i = 0; i < vec->size; i++) {
                uint32_t b;
                uint64_t off;
                orc_walk(a->first_bucket, i, &b, &off);
                vec->bucket[b][off] = apply_op(op, vec->bucket[b][off], a->mask);
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Sizes, prefix, capacity                                                     */
/* ------------------------------------------------------------------------- */
static uint64_t vsize(const orc_array *a, uint32_t v)
{
    return a->lists ? a->lists[v].len : a->vecs[v].size;
}

/* Global size: the sum of the LFVector sizes (Sec. IV). */
uint64_t orc_size(const orc_array *a)
{
    uint64_t s = 0;
    for (uint32_t v = 0; v < a->n_vectors; v++)
        s += vsize(a, v);
    return s;
}

void orc_vector_sizes(const orc_array *a, uint64_t *out)
{
    for (uint32_t v = 0; v < a->n_vectors; v++)
        out[v] = vsize(a, v);
}

/* Exclusive prefix sum of the LFVector sizes: the first global index held by
 * each LFVector (Sec. IV); out has V + 1 entries, the last being the size. */
void orc_prefix(const orc_array *a, uint64_t *out)
{
    uint64_t run = 0;
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        out[v] = run;
        run += vsize(a, v);
    }
    out[a->n_vectors] = run;
}

/* Elements held by allocated buckets.  With the bucket form this counts the
 * buckets actually present; with the list form alone it is the count a lazily
 * grown LFVector of that size would hold. */
uint64_t orc_capacity(const orc_array *a)
{
    uint64_t c = 0;
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        if (a->vecs) {
            for (uint32_t b = 0; b < ORC_MAX_BUCKETS; b++)
                if (a->vecs[v].bucket[b])
                    c += a->first_bucket << b;
        } else {
            uint32_t nb = orc_nbuckets_for(a->first_bucket, vsize(a, v));
            for (uint32_t b = 0; b < nb; b++)
                c += a->first_bucket << b;
        }
    }
    return c;
}

/* Allocated buckets per LFVector (bucket form), else the lazily grown count. */
void orc_vector_nbuckets(const orc_array *a, uint32_t *out)
{
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        if (a->vecs) {
            uint32_t n = 0;
            for (uint32_t b = 0; b < ORC_MAX_BUCKETS; b++)
                n += a->vecs[v].bucket[b] != NULL;
            out[v] = n;
        } else {
            out[v] = orc_nbuckets_for(a->first_bucket, vsize(a, v));
        }
    }
}

uint64_t orc_alloc_count(const orc_array *a) { return a->n_allocs; }
uint64_t orc_free_count(const orc_array *a) { return a->n_frees; }

/* ------------------------------------------------------------------------- */
/* Flatten: LFVectors in index order into a contiguous buffer of out_cap        */
/* elements.  Writes nothing and returns ORC_ERANGE when it does not fit.       */
/* ------------------------------------------------------------------------- */
int orc_flatten(const orc_array *a, void *out, uint64_t out_cap)
{
    if (!a)
        return ORC_EINVAL;
    uint64_t total = orc_size(a);
    if (total > out_cap)
        return ORC_ERANGE;
    if (total && !out)
        return ORC_EINVAL;
    uint64_t pos = 0;
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        uint64_t s = vsize(a, v);
        for (uint64_t i = 0; i < s; i++) {
            uint64_t e;
            if (a->lists) {
                e = a->lists[v].data[i];
            } else {
                uint32_t b;
                uint64_t off;
                orc_walk(a->first_bucket, i, &b, &off);
                e = a->vecs[v].bucket[b][off];
            }
            if (a->elem_bytes == 4)
                ((uint32_t *)out)[pos] = (uint32_t)e;
            else
                ((uint64_t *)out)[pos] = e;
            pos++;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Access by global index (rw_g of Sec. VI-B): global index i is found by       */
/* walking the LFVectors in order and subtracting their sizes (no prefix, no    */
/* search), then the element by the bucket walk (or the list).                  */
/* ------------------------------------------------------------------------- */
int orc_at(const orc_array *a, uint64_t i, uint64_t *out)
{
    if (!a || !out)
        return ORC_EINVAL;
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        uint64_t s = vsize(a, v);
        if (i < s) {
            if (a->lists) {
                *out = a->lists[v].data[i];
            } else {
                uint32_t b;
                uint64_t off;
                orc_walk(a->first_bucket, i, &b, &off);
                *out = a->vecs[v].bucket[b][off];
            }
            return ORC_OK;
        }
        i -= s;
    }
    return ORC_ERANGE;
}

/* out[k] = element at global index idx[k]; an index past the end leaves out[k]
 * untouched and makes the call return ORC_ERANGE (the others are still read). */
int orc_gather(const orc_array *a, const uint64_t *idx, uint64_t n, void *out)
{
    int rc = ORC_OK;
    for (uint64_t k = 0; k < n; k++) {
        uint64_t e;
        if (orc_at(a, idx[k], &e) != ORC_OK) {
            rc = ORC_ERANGE;
            continue;
        }
        if (a->elem_bytes == 4)
            ((uint32_t *)out)[k] = (uint32_t)e;
        else
            ((uint64_t *)out)[k] = e;
    }
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Self-check: the two forms hold the same sizes and elements, and each bucketed */
/* LFVector holds exactly the buckets that cover its live indices.              */
/* Returns 0, or 1 + the first LFVector that disagrees.                         */
/* ------------------------------------------------------------------------- */
int64_t orc_check(const orc_array *a)
{
    if (!a->vecs)
        return 0;
    for (uint32_t v = 0; v < a->n_vectors; v++) {
        const orc_lfvector *vec = &a->vecs[v];
        uint32_t nb = orc_nbuckets_for(a->first_bucket, vec->size);
        for (uint32_t b = 0; b < ORC_MAX_BUCKETS; b++)
            if ((vec->bucket[b] != NULL) != (b < nb))
                return 1 + (int64_t)v;
        if (a->lists) {
            const orc_list *l = &a->lists[v];
            if (l->len != vec->size)
                return 1 + (int64_t)v;
            for (uint64_t i = 0; i < l->len; i++) {
                uint32_t b;
                uint64_t off;
                orc_walk(a->first_bucket, i, &b, &off);
                if (vec->bucket[b][off] != l->data[i])
                    return 1 + (int64_t)v;
            }
        }
    }
    return 0;
}
