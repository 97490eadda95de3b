/*
 * ggarray.h - C ABI of the GGArray library for AMD Instinct MI355X (gfx950).
 *
 * A GGArray (Meneses, Navarro, Ferrada, "GGArray: A Dynamically Growable GPU
 * Array", arXiv 2209.00103) is an array of V LFVectors.  Each LFVector is a table
 * of buckets: bucket b holds first_bucket * 2^b elements (Alg. 2), buckets are
 * allocated only when an insertion first reaches them (Alg. 1), and elements never
 * move once written.  Insertion is block-cooperative: a block of threads computes
 * the prefix sum of its insertion counts and claims one index range per round
 * (Sec. III-B, parallel prefix-sum insertion), growing the LFVector from the GPU
 * without a host round trip (Sec. IV).  The global size is the sum of the
 * LFVector sizes and the prefix sum of those sizes locates each LFVector's
 * elements (Sec. IV); flatten copies the elements into one contiguous buffer
 * (Sec. VI-C, two-phase use).
 *
 * Conventions shared by every entry point:
 *  - Return value: GGA_OK (0) or a negative GGA_E* status.  Nothing throws across
 *    the ABI.  Argument errors are detected on the host and returned at once,
 *    before any work is queued.
 *  - Device-side errors (bucket pool exhausted, flatten output too small) are
 *    sticky per array: the first one is kept and reported by the next call that
 *    synchronises (ggarray_last_error, ggarray_size, ggarray_capacity).
 *  - Streams: every call is ordered on the caller's stream `s` (a hipStream_t
 *    passed as void*; NULL is the default stream).  Only calls documented as
 *    synchronising block the host.  Handles are not thread-safe, and two streams
 *    must not work on one array at the same time.
 *  - Memory: pointers named dev_* / values / flags / counts / out are device
 *    pointers owned by the caller.  The bucket pool memory is owned by the
 *    caller; the library owns the buckets it carves from it and its own small
 *    metadata allocations.
 *  - Element types: 4-byte or 8-byte unsigned integers; element arithmetic wraps
 *    modulo 2^(8 * elem_bytes).
 *  - Thread -> LFVector mapping: an insertion round with n logical threads feeds
 *    LFVector v with threads [v*c, (v+1)*c) where c = ceil(n / V).  Inside a round
 *    the elements land in thread-rank order, a thread's own elements contiguous
 *    and in their order.  The result is therefore a pure function of the inputs,
 *    V and first_bucket; block size and launch shape never change it.
 *  - HIP graphs: the single-array calls may be captured on `s`.  During capture
 *    nothing is allocated: an insertion round needing more look-back words than
 *    an earlier eager round of the array left returns GGA_EINVAL (run the same
 *    round once eagerly first).  The size prefix and the tile table that r/w and
 *    flatten read are recomputed inside the graph (once per size change within
 *    one capture), so a replay sees the sizes of its own moment.  Once a
 *    captured call changes an array's sizes, every later eager r/w, flatten or
 *    prefix call on it recomputes them too, since replays change the sizes
 *    without the library seeing it.  Calls on one array must be
 *    ordered on one stream, in a graph as outside it.  Internal buffers an array
 *    outgrows are kept until ggarray_destroy, so a graph captured earlier stays
 *    valid.
 */
#ifndef GGARRAY_H
#define GGARRAY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status --- */
#define GGA_OK 0
#define GGA_EINVAL (-1) /* invalid argument */
#define GGA_ENOMEM (-2) /* bucket pool exhausted (device side, sticky) */
#define GGA_ERANGE (-3) /* output buffer or static capacity too small (sticky) */
#define GGA_EHIP (-4)   /* a HIP runtime call failed */
#define GGA_EBUSY (-5)  /* object still referenced (pool with live arrays) */

typedef void *gga_stream; /* hipStream_t */
typedef struct gga_pool gga_pool;
typedef struct ggarray ggarray;
typedef struct gga_static gga_static;
typedef struct gga_semistatic gga_semistatic;
typedef struct gga_mapped gga_mapped;
typedef struct gga_batch gga_batch;

/* r/w operations (Sec. VI-C times an operation over every element; the paper's
 * kernel adds 1 thirty times, GGA_ADD1_X30). */
#define GGA_ADD1 0     /* x = x + 1 */
#define GGA_MUL3ADD1 1 /* x = 3x + 1 */
#define GGA_ADD1_X30 2 /* x = x + 1, thirty times */

/* Generated payloads: the insertion workloads produced on the device, the way a
 * user kernel computes the element it pushes back.  K(seed, a, b) is
 * SplitMix64 (Steele, Lea, Flood 2014) applied to (seed << 56) ^ (a << 8) ^ b. */
#define GGA_GEN_BERNOULLI 1 /* h = K(seed, gid, round); insert h iff h >> 63 */
#define GGA_GEN_ROUND_TAG 2 /* insert (round << tag_shift) | gid */
#define GGA_GEN_POISSON 3   /* u = K(seed, gid, 0x80 | round);
                               c = #{k < max_count : u >= thresholds[k]};
                               insert K(seed, gid, 16 * round + j), j < c */
#define GGA_GEN_KEYED 4     /* insert K(seed, (tag << tag_shift) | gid, round); in a
                               batch the array's position is added to tag */
typedef struct {
    uint32_t kind;           /* GGA_GEN_* */
    uint32_t round;          /* BERNOULLI, KEYED: < 256; POISSON: < 8 */
    uint64_t seed;           /* < 256 */
    uint32_t tag_shift;      /* ROUND_TAG: < 64; KEYED: 1..47 */
    uint32_t max_count;      /* POISSON: 1..16 */
    uint64_t thresholds[16]; /* POISSON: host copy, the first max_count used */
    uint64_t tag;            /* KEYED: tag (+ batch position) < 2^(48 - tag_shift),
                                gid < 2^tag_shift (so the key stays below 2^48) */
} gga_gen;

/* The last HIP call that failed in this thread (name and HIP error), after a
 * GGA_EHIP; a static per-thread string. */
const char *gga_last_hip_error(void);

/* Human-readable name of a status code (static string). */
const char *gga_strerror(int status);

/* ------------------------------------------------------------ bucket pool --- */
/* Device sub-allocator that serves bucket allocations from inside the insertion
 * kernels (Alg. 2 allocates with device malloc; here a lock-free pool over
 * caller-owned HBM does, so growth needs no host round trip).
 *
 * gga_pool_create: dev_base is caller-owned device memory of `bytes` bytes,
 *   256-byte aligned, at least 3 MiB; it must outlive the pool.  The pool keeps
 *   a 2 MiB header (4096 free lists per size class) at the start and carves
 *   buckets (power-of-two sizes, >= 256 B) from the rest, through 256 arena
 *   shards that each sub-allocate chunks of about 1/1024 of the region
 *   (64 KiB .. 16 MiB), so up to 256 chunks may be partly used.  Synchronises
 *   s.  EINVAL on a NULL/unaligned/small buffer.
 * gga_pool_destroy: frees the host handle; EBUSY while arrays still use it.
 * gga_pool_stats: out[0..6] = bytes in use, bytes carved from the region so far
 *   (an upper bound of the peak in use), allocations, frees, the same carved
 *   bytes, region bytes, allocation attempts counted for fault injection.
 *   Synchronises s.
 * gga_pool_set_fault: the fault_at-th allocation attempt from now fails as if
 *   the pool were exhausted (0 disables).  For failure-handling tests. */
int gga_pool_create(gga_pool **out, void *dev_base, uint64_t bytes, gga_stream s);
int gga_pool_destroy(gga_pool *p);
int gga_pool_stats(gga_pool *p, uint64_t out[7], gga_stream s);
int gga_pool_set_fault(gga_pool *p, uint64_t fault_at, gga_stream s);

/* ---------------------------------------------------------------- GGArray --- */
/* ggarray_create: an empty GGArray of n_vectors LFVectors (Sec. IV, Fig. 1-2)
 *   whose first bucket holds first_bucket elements (Alg. 2).  elem_bytes is 4 or
 *   8; first_bucket is a power of two >= 1; n_vectors is 1..2^20.  No bucket is
 *   allocated (lazy growth, Alg. 1).  Metadata is device memory the library
 *   allocates here (about 350 bytes per LFVector).  Queued on s. */
int ggarray_create(ggarray **out, gga_pool *p, uint32_t elem_bytes, uint32_t n_vectors,
                   uint64_t first_bucket, gga_stream s);

/* ggarray_destroy: returns every bucket to the pool and frees the metadata.  The
 *   caller guarantees no work on the array is pending on other streams; the
 *   call synchronises s. */
int ggarray_destroy(ggarray *a, gga_stream s);

/* ggarray_insert: one insertion round, LFVector push_back (Alg. 1) with
 *   new_bucket (Alg. 2).  Logical thread gid (0 <= gid < n_threads) inserts
 *   values[gid] iff flags == NULL or flags[gid] != 0.  values: n_threads
 *   elements; flags: n_threads bytes or NULL; both device memory.  Missing buckets
 *   are allocated on the device.  Pool exhaustion leaves every affected LFVector
 *   exactly as it was before the round, freezes it for later insertions and sets
 *   the sticky GGA_ENOMEM.  With flags, a round that gives an LFVector more than
 *   one tile of 4096 threads runs as a few launches (flag masks and tile counts,
 *   their prefix, growth, copy) in a per-array buffer of about 0.13 bytes per
 *   thread, grown when needed (under graph capture, where it cannot grow, the
 *   round runs as one launch with a per-LFVector look-back instead).  Those
 *   launches read 16-byte payload vectors when values is 16-byte aligned, flags
 *   is aligned to E = 16 / element bytes, and n_threads and every LFVector's
 *   share ceil(n_threads / V) are multiples of E; any other input gives the same
 *   result through one-element loads. */
int ggarray_insert(ggarray *a, const void *values, const uint8_t *flags, uint64_t n_threads,
                   gga_stream s);

/* ggarray_insert_counts: as ggarray_insert, but thread gid inserts
 *   values[gid * max_count + j] for j < counts[gid]; 1 <= max_count <= 16 and
 *   counts[gid] <= max_count (larger counts are clamped to max_count). */
int ggarray_insert_counts(ggarray *a, const void *values, const uint8_t *counts,
                          uint32_t max_count, uint64_t n_threads, gga_stream s);

/* ggarray_insert_packed: one insertion round in which logical thread gid inserts
 *   counts[gid] elements (0..255; each thread's count enters the block prefix
 *   sum of Sec. III-B), taken in order from a packed buffer: thread gid's
 *   elements are values[P(gid) .. P(gid) + counts[gid]), P the exclusive prefix
 *   sum of the counts (values: n_values elements, counts: n_threads bytes, both
 *   device memory; for one round into an empty array the flatten equals the
 *   first sum-of-counts values).  Because a tile's values and its outputs are
 *   both contiguous, the round streams from the buffer into the buckets.  If the
 *   counts sum to more than n_values nothing is inserted and the sticky
 *   GGA_ERANGE is set.  The library keeps one offset word per 1024 logical
 *   threads (grown like the look-back words: not during graph capture).  The
 *   prefix sum is taken over the whole round first, so every LFVector's growth
 *   is known before any element is copied: one launch grows the LFVectors,
 *   the next copies, with no waits between blocks. */
int ggarray_insert_packed(ggarray *a, const void *values, uint64_t n_values, const uint8_t *counts,
                          uint64_t n_threads, gga_stream s);

/* ggarray_insert_packed_noalloc: for callers that cannot allocate device memory
 *   (code being captured into a HIP graph, tight serving loops, harnesses that
 *   forbid hipMalloc).  Same arguments and results as ggarray_insert_packed, but
 *   the call allocates nothing: the per-tile value offsets live in a static
 *   device array of the library (69664 words, about 545 KiB, one copy per GPU,
 *   held until the process ends).  Buckets still come from the array's pool on the
 *   device.  Limit: the round may span at most 65536 tiles, a tile being 1024
 *   logical threads of one LFVector (V * ceil(ceil(n_threads / V) / 1024) <=
 *   65536); a larger round returns GGA_ERANGE at once and queues nothing.
 *   Every call on one GPU shares that array: calls that overlap on one GPU
 *   (other streams, other host threads) race and must not be issued; calls
 *   ordered on one stream are safe, since each writes every word it reads. */
int ggarray_insert_packed_noalloc(ggarray *a, const void *values, uint64_t n_values, const uint8_t *counts,
                                  uint64_t n_threads, gga_stream s);

/* ggarray_insert_gen: one insertion round whose payloads are generated on the
 *   device by g (see GGA_GEN_*); `g` is a host pointer read before returning. */
int ggarray_insert_gen(ggarray *a, const gga_gen *g, uint64_t n_threads, gga_stream s);

/* ggarray_insert_segments: LFVector v appends values[prefix[v] .. prefix[v + 1])
 *   in order, for every v (values: n_values elements, prefix: V + 1 uint64, both
 *   device memory).  With ggarray_prefix and ggarray_flatten this restores an
 *   array from a flat snapshot: the flatten of the Sec. VI-C two-phase use, run
 *   backwards.  An LFVector whose pair decreases, runs past n_values or spans 2^32
 *   elements or more is left unchanged and the sticky GGA_ERANGE is set.  Buckets
 *   are allocated on the device as for ggarray_insert. */
int ggarray_insert_segments(ggarray *a, const void *values, const uint64_t *prefix, uint64_t n_values,
                            gga_stream s);

/* ggarray_shrink: every LFVector pops floor(s_v * num / den) trailing elements
 *   and returns each bucket that starts at or past its new size to the pool.
 *   0 <= num <= den, den > 0.  (The paper studies growth only; shrinking follows
 *   the generic vector interface it names in Sec. I.) */
int ggarray_shrink(ggarray *a, uint32_t num, uint32_t den, gga_stream s);

/* ggarray_insert_gen_shrink: ggarray_insert_gen(a, g, n_threads) followed by
 *   ggarray_shrink(a, num, den), with the same results (sizes, contents,
 *   capacity, pool counts, errors; an LFVector whose growth fails in the round is
 *   still shrunk).  A round of round-tag or keyed payloads that runs one wave per
 *   LFVector (at most 8 tiles of 4096 threads per LFVector, or 512 LFVectors or
 *   more) does both in one launch: the wave stores its elements, sets the size
 *   the shrink leaves and releases the buckets past it.  Other rounds take two
 *   launches.  den == 0 or num > den: GGA_EINVAL, nothing
 *   launched. */
int ggarray_insert_gen_shrink(ggarray *a, const gga_gen *g, uint64_t n_threads, uint32_t num, uint32_t den,
                              gga_stream s);

/* ggarray_insert_gen_rounds: with clear_first != 0, first ggarray_shrink(a, 1, 1);
 *   then n_rounds insertion rounds in order, round r of n_threads[r] logical
 *   threads with the payloads of gens[r] (as ggarray_insert_gen), each followed by
 *   ggarray_shrink(a, num, den) when num > 0 (the generic vector interface Sec. I
 *   names; a round is Alg. 1 with Alg. 2).  gens, n_threads: host arrays of
 *   n_rounds entries (at most GGA_MAX_ROUNDS), read before returning.  Sizes,
 *   contents, capacity and pool counts are those of the calls made one by one.
 *   One launch runs everything when the rounds are of round-tag or keyed payloads
 *   that differ only in round and thread count, each runs one wave per LFVector
 *   (at most 8 tiles of 4096 threads per LFVector, or 512 LFVectors or more), and
 *   there are two rounds or more or a clear: each LFVector's wave takes it through
 *   the clear and every round; the clear keeps each bucket in place for the round
 *   that reaches it again (counted as released and allocated) and returns the
 *   others at the end of the launch.  Any other list runs call by call.  In the one
 *   launch the LFVectors reach the pool in another order, so when it runs dry the
 *   LFVectors that freeze (GGA_ENOMEM), and the buckets they keep, can differ from
 *   those of the calls one by one.  den == 0, num > den, too many rounds or an
 *   invalid generator or round size in any round: GGA_EINVAL, nothing launched. */
#define GGA_MAX_ROUNDS 16
int ggarray_insert_gen_rounds(ggarray *a, const gga_gen *gens, const uint64_t *n_threads, uint32_t n_rounds,
                              uint32_t num, uint32_t den, uint32_t clear_first, gga_stream s);

/* ggarray_rw: x = op(x) for every live element, in place, LFVector by LFVector
 *   through the bucket tables (the per-block read/write rw_b of Sec. VI-B). */
int ggarray_rw(ggarray *a, uint32_t op, gga_stream s);

/* ggarray_rw_global: the same result as ggarray_rw, computed element by element
 *   from the global index (the rw_g variant of Sec. VI-B): global index i lies in
 *   the last LFVector v with P[v] <= i (P as for flatten, so empty LFVectors are
 *   skipped), at local index i - P[v], whose bucket and offset follow from the
 *   closed form of the bucket law (Alg. 2). */
int ggarray_rw_global(ggarray *a, uint32_t op, gga_stream s);

/* ggarray_gather: out[k] = element at global index idx[k] for k < n (idx and out
 *   device memory, out of n elements; the order of the global index is the
 *   flatten order).  An index at or past the size leaves out[k] unwritten and
 *   sets the sticky GGA_ERANGE; the other entries are still written. */
int ggarray_gather(ggarray *a, const uint64_t *idx, uint64_t n, void *out, gga_stream s);

/* ggarray_flatten: copies LFVector 0, then 1, ... into out (device memory of
 *   out_cap_elems elements), element i of LFVector v landing at P[v] + i where P
 *   is the exclusive prefix sum of the LFVector sizes (Sec. IV).  The GGArray is
 *   unchanged.  If out_cap_elems is smaller than the size, nothing is written and
 *   the sticky GGA_ERANGE is set. */
int ggarray_flatten(ggarray *a, void *out, uint64_t out_cap_elems, gga_stream s);

/* ggarray_size: global size = sum of the LFVector sizes (Sec. IV), into *out_host.
 *   Synchronises s.  Returns the sticky device error if one is set; *out_host is
 *   written in that case too (the size of the committed contents). */
int ggarray_size(ggarray *a, uint64_t *out_host, gga_stream s);

/* ggarray_capacity: elements held by the allocated buckets, into *out_host: the
 *   memory side of the structure, which the paper bounds at about twice the live
 *   data (abstract, Sec. V); exactly, each LFVector of s >= 1 elements holds
 *   first_bucket * (2^nb - 1) <= 2 s + first_bucket - 1 elements, where nb is the
 *   fewest buckets of Alg. 2 that reach s, and an empty LFVector holds none.
 *   Synchronises s. */
int ggarray_capacity(ggarray *a, uint64_t *out_host, gga_stream s);

/* ggarray_footprint: device bytes the array holds besides its buckets, from host
 *   state (no synchronisation): out[0] metadata (sizes, bucket tables, prefixes,
 *   tickets), out[1] look-back words, out[2] tile tables (current and outgrown
 *   ones kept for captured graphs).  Bucket bytes: ggarray_capacity x elem_bytes. */
int ggarray_footprint(ggarray *a, uint64_t out[3]);

/* ggarray_vector_sizes: copies the V LFVector sizes (uint64) to dev_out. Queued. */
int ggarray_vector_sizes(ggarray *a, uint64_t *dev_out, gga_stream s);

/* ggarray_prefix: writes the V + 1 entries of the exclusive prefix sum of the
 *   LFVector sizes (uint64; the last entry is the global size) to dev_out. Queued. */
int ggarray_prefix(ggarray *a, uint64_t *dev_out, gga_stream s);

/* ggarray_kernel_timing: a measurement aid.  With on != 0 the array's r/w and
 *   flatten kernels, and its insertion rounds that run as one launch (rounds of
 *   round-tag or keyed payloads, or of a buffer without flags, with one wave per
 *   LFVector), when not captured in a graph, are dispatched with a pair of HIP
 *   events that the dispatch itself records at the kernel's start and end (the
 *   library creates and owns them; on == 0 destroys them).
 * ggarray_kernel_ms: the duration in milliseconds of the array's last timed r/w
 *   (kind 0) or flatten (kind 1) kernel, or of its last insertion round (kind 2)
 *   if that round was timed; waits for it to end.  GGA_EINVAL when there is no
 *   such timed kernel. */
int ggarray_kernel_timing(ggarray *a, uint32_t on);
int ggarray_kernel_ms(ggarray *a, uint32_t kind, float *ms);

/* ggarray_last_error: the sticky device error of the array (GGA_OK if none).
 *   Synchronises s.  Does not clear it.  The paper's growth (Alg. 2) does not say
 *   what happens when an allocation fails; here a failed bucket allocation drops
 *   the round of the affected LFVector, freezes it and sets GGA_ENOMEM, a bounded
 *   wait that expires sets GGA_EHIP, and a flatten into a too-small buffer sets
 *   GGA_ERANGE; the first error is kept until the array is destroyed. */
int ggarray_last_error(ggarray *a, gga_stream s);

/* ggarray_set_spin_limit: a failure-handling aid.  Every wait of an insertion
 *   kernel on another workgroup (look-back, a bucket pointer, allocation counts)
 *   gives up after `polls` polls (0 restores the default, 2^22), freezes the
 *   LFVector it serves and sets the sticky GGA_EHIP; a tiny limit forces that
 *   path from the host while every kernel still ends normally.  Applies to later
 *   single-array calls on `a` (batches and servers copy the array's descriptor
 *   when they are created).  After such an expiry the frozen LFVectors' contents
 *   are unspecified; every other LFVector holds exactly its round. */
int ggarray_set_spin_limit(ggarray *a, uint32_t polls);

/* ------------------------------------------------------ device-side API --- */
/* For user kernels that push elements themselves with gga::block_push_back
 * (include/ggarray_device.h, the block-cooperative push_back of Alg. 1 used from
 * inside any kernel, as the paper intends the structure to be used).
 *
 * ggarray_device_ref: copies the array's device descriptor (a gga::ArrRef,
 *   `bytes` must equal its size) to the host memory at out; pass it to the user
 *   kernel by value.  It stays valid until the array is destroyed.
 * ggarray_device_done: declares that kernels queued on s may have changed the
 *   array's sizes, so the next operation rescans them (call it after queueing
 *   such kernels, before any other call on the array). */
int ggarray_device_ref(ggarray *a, void *out, uint64_t bytes);
int ggarray_device_done(ggarray *a, gga_stream s);

/* ---------------------------------------------------------------- batches --- */
/* A batch drives many GGArrays together: one launch inserts a round into every
 * array, one launch scans all their sizes, one launch does the r/w or the
 * flatten of all of them.  Each array keeps its own LFVectors, first bucket and
 * results: a batch call gives every array exactly the result the same call on
 * that array alone would give.  (The paper evaluates one array at a time; the
 * batch is the multi-array form of the same operations.)
 *
 * gga_batch_create: arrays[0..n) are distinct GGArrays with one element size,
 *   n >= 1; they must outlive the batch and not be used by other streams while
 *   batch calls are pending.  The batch copies their descriptors to the device.
 *   Synchronises s.
 * gga_batch_insert_gen: one round: array i runs g with n_threads[i] logical
 *   threads (host array of n entries; 0 skips the array).  Kinds ROUND_TAG,
 *   BERNOULLI and KEYED.  The first call with a new set of thread counts uploads
 *   a small table (and synchronises s); later calls with the same counts launch
 *   one kernel and nothing else, so they can be captured in a HIP graph.
 * gga_batch_shrink: ggarray_shrink(num, den) on every array, one launch.
 * gga_batch_rw: x = op(x) over every live element of every array.
 * gga_batch_flatten: array 0, then 1, ... into out (out_cap_elems elements);
 *   array i starts at offset[i], the exclusive prefix of the array sizes.  If the
 *   total exceeds out_cap_elems nothing is written and the batch's sticky
 *   GGA_ERANGE is set.
 * gga_batch_set_grid: workgroups that r/w and flatten launch (1..2^20; 0
 *   restores the defaults: one per tile of the batch's tile table, at most
 *   131072, or 8192 for r/w and 65536 for flatten when the batch streams
 *   without a table).  A launch-shape knob for tuning; results do not depend on it.
 * gga_batch_offsets: the n + 1 offsets (uint64, last = total) to dev_out.
 * gga_batch_last_error: the batch's sticky error.  Synchronises s. */
/* gga_batch_step: a whole step of every array in ONE persistent launch:
 *   `rounds` insertion rounds (round r runs gens[r] on array i with
 *   n_threads[r * n + i] logical threads; kinds ROUND_TAG, BERNOULLI and KEYED;
 *   at most 8 rounds), then x = op(x) over every live element (op GGA_RW_NONE:
 *   none), then, unless out is NULL, the flatten of every array into out as
 *   gga_batch_flatten writes it.  The result is that of gga_batch_insert_gen for
 *   each round, gga_batch_rw and gga_batch_flatten in that order.  LFVectors are
 *   independent (Sec. IV), so each workgroup takes its LFVectors through all
 *   rounds (Sec. III-B's prefix sum per tile of 1024 logical threads, buckets
 *   allocated on the device as in Alg. 1-2) and the r/w without waiting on
 *   another; two grid-wide barriers give the flatten its size prefix.  The grid
 *   is sized to be resident at once and launched cooperatively (not under graph
 *   capture, where it is recorded as a plain launch: run nothing beside a
 *   captured step).  Suited to many short LFVectors (each LFVector's rounds run
 *   in one workgroup); rounds that give an LFVector many tiles are faster with
 *   the per-round calls.  A new table of thread counts is uploaded (and s
 *   synchronised) the first time it is seen; capturing a step needs a table an
 *   eager step has used.  Pool exhaustion: the LFVector is frozen with the size
 *   it had before the round, as in the per-round calls (the buckets it holds may
 *   differ).  The flatten's GGA_ERANGE is the batch's sticky error. */
#define GGA_RW_NONE 0xFFFFFFFFu
int gga_batch_step(gga_batch *b, const gga_gen *gens, uint32_t rounds, const uint64_t *n_threads, uint32_t op,
                   void *out, uint64_t out_cap_elems, gga_stream s);

/* gga_batch_step_clear: gga_batch_shrink(b, 1, 1) followed by gga_batch_step
 *   with the same arguments, in that one launch.  The result (sizes, contents,
 *   the pool's allocation and release counts, out) is that of the two calls;
 *   a bucket an LFVector held before the clear and reaches again in the rounds
 *   stays in place rather than going through its free list (a push and a pop of
 *   the same block), and the held buckets the rounds do not reach go back to the
 *   pool at the end.  A frozen LFVector gives back every bucket and stays
 *   frozen, as after ggarray_shrink.  Same validation, graph capture and error
 *   behaviour as gga_batch_step. */
int gga_batch_step_clear(gga_batch *b, const gga_gen *gens, uint32_t rounds, const uint64_t *n_threads, uint32_t op,
                         void *out, uint64_t out_cap_elems, gga_stream s);

int gga_batch_create(gga_batch **out, ggarray *const *arrays, uint32_t n, gga_stream s);
int gga_batch_destroy(gga_batch *b, gga_stream s);
int gga_batch_insert_gen(gga_batch *b, const gga_gen *g, const uint64_t *n_threads, gga_stream s);
int gga_batch_shrink(gga_batch *b, uint32_t num, uint32_t den, gga_stream s);
int gga_batch_rw(gga_batch *b, uint32_t op, gga_stream s);
int gga_batch_flatten(gga_batch *b, void *out, uint64_t out_cap_elems, gga_stream s);
int gga_batch_set_grid(gga_batch *b, uint32_t stream_blocks);
int gga_batch_offsets(gga_batch *b, uint64_t *dev_out, gga_stream s);
int gga_batch_last_error(gga_batch *b, gga_stream s);

/* ----------------------------------------------------------------- serving --- */
/* A request loop over resident arrays (an extension of the paper's operations:
 * the paper runs one array at a time).  A request is one operation on one array:
 *   GGA_REQ_APPEND:  one insertion round of length[r] threads, thread j inserting
 *                    K(seed, (r << append_shift) | j, append_round) (as a KEYED
 *                    round with tag r), r the request's index in the trace;
 *   GGA_REQ_RW:      ggarray_rw(rw_op);
 *   GGA_REQ_FLATTEN: ggarray_flatten into the server's output arena.
 * Requests on one array run in arrival order, one at a time; requests on
 * different arrays run concurrently.  Every result therefore equals the result of
 * running that array's requests alone, in order, with the single-array calls.
 *
 * GGA_SERVE_BATCHED: continuous batching.  The host admits arrived requests into
 *   steps of at most max_step requests, at most one per array and none on an
 *   array whose previous request is still in flight, oldest first; a step is one
 *   table copy plus one insertion launch for its appends and one scan + one
 *   streaming launch for its r/w and flatten requests.  Up to `lanes` steps are
 *   in flight on their own streams, so new requests join as earlier ones finish.
 * GGA_SERVE_PER_REQUEST: the baseline: each request issued alone with the
 *   single-array calls, in arrival order, on one stream, at most `depth` in flight.
 *
 * Admission.  The server tracks each array's size on the host (initial size plus
 * admitted appends) and charges it elem_bytes * (2 size + V F) bytes, the bound on
 * an array's capacity (Sec. IV); a flatten also holds its output bytes in the
 * arena until it completes.  A request waits while the charges plus the arena
 * bytes in use would exceed cap_bytes (or the arena has no room), and is
 * rejected (status GGA_ENOMEM, nothing run) when it could not fit even with the
 * arena empty.
 *
 * gga_server_create: arrays[0..n) distinct GGArrays of one element size, which
 *   must outlive the server and not be used elsewhere during a run; arena is a
 *   caller-owned device buffer of arena_bytes bytes (flatten outputs, allocated
 *   as a ring, 256-byte aligned).  The server creates its own streams (default
 *   priority) and pinned staging.
 * gga_server_run: replays the n requests of the trace (host arrays; arrival_ns
 *   non-decreasing, relative to the start of the run) in real time and returns
 *   when all have completed.  It synchronises the device before starting.
 *   Per request (host arrays of n entries): t_issue_ns, t_done_ns (host clock,
 *   relative to the start; t_done is when the host saw the request's work
 *   finish), status (GGA_OK or GGA_ENOMEM), out_offset (flatten: byte offset of
 *   its output in the arena, else UINT64_MAX; the output stays valid until the
 *   ring reuses that space).  dev_out_len (device, n entries, may be NULL)
 *   receives each flatten's element count.  stats (host, 8 entries, may be NULL):
 *   steps, largest step, requests issued, rejected, waits for memory, peak
 *   charged bytes, elapsed ns, arena wraps.  Returns GGA_ERANGE if a flatten
 *   found its array larger than its reservation (then that output is not
 *   written), GGA_EHIP on a runtime error. */
#define GGA_REQ_APPEND 0
#define GGA_REQ_RW 1
#define GGA_REQ_FLATTEN 2
#define GGA_SERVE_BATCHED 0
#define GGA_SERVE_PER_REQUEST 1

typedef struct gga_server gga_server;
typedef struct gga_server_config {
    uint64_t cap_bytes;     /* admission budget, bytes */
    uint32_t mode;          /* GGA_SERVE_* */
    uint32_t lanes;         /* BATCHED: steps in flight, 1..8 */
    uint32_t max_step;      /* BATCHED: requests per step, 1..65536 */
    uint32_t depth;         /* PER_REQUEST: requests in flight, 1..65536 */
    uint64_t seed;          /* append payload key, < 256 */
    uint32_t append_round;  /* < 256 */
    uint32_t append_shift;  /* 1..47; appends need length <= 2^shift, r < 2^(48 - shift) */
    uint32_t rw_op;         /* GGA_ADD1 .. GGA_ADD1_X30 */
} gga_server_config;

typedef struct gga_trace {
    uint64_t n;
    const uint64_t *arrival_ns;
    const uint8_t *kind;     /* GGA_REQ_* */
    const uint32_t *target;  /* array index */
    const uint32_t *length;  /* APPEND: threads, >= 1 */
} gga_trace;

int gga_server_create(gga_server **out, ggarray *const *arrays, uint32_t n, void *arena,
                      uint64_t arena_bytes, const gga_server_config *cfg);
int gga_server_destroy(gga_server *sv);
int gga_server_run(gga_server *sv, const gga_trace *tr, uint64_t *t_issue_ns, uint64_t *t_done_ns,
                   int32_t *status, uint64_t *out_offset, uint64_t *dev_out_len, uint64_t *stats);

/* ------------------------------------------------- static array baseline --- */
/* The pre-allocated flat array of Sec. III-A1: caller-owned device buffer of
 * cap_elems elements; insertion uses the same block prefix sum and one global
 * atomic per block round (Sec. III-B2), so the order across blocks is not fixed.
 * Insertions past the capacity are dropped and set the sticky GGA_ERANGE. */
int gga_static_create(gga_static **out, void *dev_buf, uint64_t cap_elems, uint32_t elem_bytes,
                      gga_stream s);
int gga_static_destroy(gga_static *st, gga_stream s);
int gga_static_insert(gga_static *st, const void *values, const uint8_t *flags,
                      uint64_t n_threads, gga_stream s);
int gga_static_insert_gen(gga_static *st, const gga_gen *g, uint64_t n_threads, gga_stream s);
/* The per-element strategy the paper compares against the scan (Sec. VI-A):
 * every inserting thread takes its slot with its own atomic add on the size.
 * Kinds BERNOULLI, ROUND_TAG and KEYED.  Order across threads not fixed. */
int gga_static_insert_gen_atomic(gga_static *st, const gga_gen *g, uint64_t n_threads, gga_stream s);
int gga_static_rw(gga_static *st, uint32_t op, gga_stream s);
int gga_static_size(gga_static *st, uint64_t *out_host, gga_stream s); /* synchronises */
int gga_static_last_error(gga_static *st, gga_stream s);                /* synchronises */
/* Empties the array and clears its sticky error (the buffer is kept).  Queued. */
int gga_static_clear(gga_static *st, gga_stream s);
/* Sets the size to n <= capacity (the first n elements of the buffer become the
 *   live ones), e.g. after the buffer was filled by a GGArray flatten for a work
 *   phase (the two-phase use of Sec. VI-C, VI-D).  Queued.  EINVAL past the capacity. */
int gga_static_set_size(gga_static *st, uint64_t n, gga_stream s);

/* ----------------------------------------- semi-static array baseline ------ */
/* The host-resized array of Sec. III-A2: before each insertion round the host
 * reads the size, and if the worst case of the round does not fit it doubles
 * the capacity (new device allocation, device-to-device copy, free of the old
 * one, all on s).  Insertion and r/w then run as for the static array.  The
 * library allocates its buffer with the stream-ordered HIP allocator. */
int gga_semi_create(gga_semistatic **out, uint32_t elem_bytes, uint64_t initial_cap,
                    gga_stream s);
int gga_semi_destroy(gga_semistatic *ss, gga_stream s);
int gga_semi_insert(gga_semistatic *ss, const void *values, const uint8_t *flags,
                    uint64_t n_threads, gga_stream s);
int gga_semi_insert_gen(gga_semistatic *ss, const gga_gen *g, uint64_t n_threads, gga_stream s);
int gga_semi_rw(gga_semistatic *ss, uint32_t op, gga_stream s);
int gga_semi_size(gga_semistatic *ss, uint64_t *out_host, gga_stream s); /* synchronises */
/* Current device buffer and capacity (elements); valid until the next insert. */
int gga_semi_data(gga_semistatic *ss, void **dev_data, uint64_t *cap_elems);
/* Number of host-driven resizes so far. */
int gga_semi_resizes(gga_semistatic *ss, uint64_t *out_host);

/* ------------------------------------------- mapped (memMap) array baseline --- */
/* The host-grown array without copies that the paper measures beside the
 * semi-static one (Table II, memMap): a virtual range for max_elems elements is
 * reserved once; before each insertion round the host reads the size and, if
 * the round's worst case does not fit, maps more physical memory (whole
 * allocation-granularity chunks covering the shortfall) onto the end of the
 * mapped part, so growing never moves elements.  Insertion and r/w then run as
 * for the static array.  A round that could pass max_elems returns GGA_ERANGE
 * before anything runs.  GGA_EHIP if the device lacks virtual memory management.
 * Destroy synchronises s, unmaps and releases everything. */
int gga_mapped_create(gga_mapped **out, uint32_t elem_bytes, uint64_t max_elems, gga_stream s);
int gga_mapped_destroy(gga_mapped *m, gga_stream s);
int gga_mapped_insert(gga_mapped *m, const void *values, const uint8_t *flags, uint64_t n_threads,
                      gga_stream s);
int gga_mapped_insert_gen(gga_mapped *m, const gga_gen *g, uint64_t n_threads, gga_stream s);
int gga_mapped_rw(gga_mapped *m, uint32_t op, gga_stream s);
int gga_mapped_size(gga_mapped *m, uint64_t *out_host, gga_stream s); /* synchronises */
/* Base of the range and the elements mapped so far (the range never moves). */
int gga_mapped_data(gga_mapped *m, void **dev_data, uint64_t *mapped_elems);
/* Number of host-driven mappings so far. */
int gga_mapped_maps(gga_mapped *m, uint64_t *out_host);

#ifdef __cplusplus
}
#endif

#endif /* GGARRAY_H */
