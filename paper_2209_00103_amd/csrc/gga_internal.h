// Host-side objects and the launch functions shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>

#include "ggarray.h"
#include "ggarray_device.h"

struct gga_pool {
  gga::PoolRef ref;
  void* dev_base;
  uint64_t bytes;
  int n_arrays;
  uint32_t next_salt;  // salt of the next array: arrays take consecutive free-list shards
};

struct ggarray {
  gga_pool* pool;
  uint32_t elem_bytes;
  uint32_t elem_log2;
  uint32_t V;
  uint32_t log2F;
  void* meta;             // one device allocation holding the per-array metadata
  gga::ArrRef ref;
  uint64_t status_cap;    // look-back words available
  bool prefix_valid;      // prefix / tprefix match the current sizes
  uint64_t size_ub;       // host upper bound of the size (sets launch shapes only)
  uint64_t* tile_tab;     // device: per tile, its first element's address and its
                          // destination offset | element count << 48 (r/w, flatten)
  uint64_t tab_cap;       // tiles the table holds
  uint64_t sizes_gen;     // advanced whenever the LFVector sizes may change
  uint64_t tab_gen;       // sizes_gen the table was built for
  // Device buffers the array has outgrown (look-back words, tile tables): kept
  // until the array is destroyed, so that a HIP graph captured earlier never
  // reads freed memory.  Both grow at least twofold, so few are retired.
  void* retired[64];
  uint32_t n_retired;
  uint64_t* scan_tot;     // device: per 1024 LFVectors, their total size and tiles
  uint64_t last_rw_gen;   // sizes_gen + 1 when the last streaming call was an r/w (0: not)
  uint64_t scan_tag;      // capture tag (stream_capture_tag) the current prefix was built under
  uint64_t tab_tag;       // capture tag the current tile table was built under
  bool graph_sized;       // a captured call changes the sizes (replays do so unseen)
  hipEvent_t tev[3][2];   // kernel timing: start / end events of the last r/w (0), flatten (1), round (2)
  uint32_t tev_set;       // bit k: events of kind k were recorded by a dispatch
  uint64_t meta_bytes;    // size of the metadata allocation
  uint64_t retired_tab_bytes;  // outgrown tile tables kept until destroy
  uint64_t* pk_off;       // device: per-tile value offsets of packed rounds (+ total)
  uint64_t pk_cap;        // words pk_off holds
};

// Hands an outgrown device buffer to the array, to be freed with it.
inline int retire_buffer(ggarray* a, void* p, hipStream_t s) {
  if (!p) return GGA_OK;
  if (a->n_retired < sizeof(a->retired) / sizeof(a->retired[0])) {
    a->retired[a->n_retired++] = p;
    return GGA_OK;
  }
  return hipFreeAsync(p, s) == hipSuccess ? GGA_OK : GGA_EHIP;
}

// True while `s` records into a HIP graph (or when that cannot be told): then
// nothing may be allocated, and derived state is rebuilt inside the graph.
inline bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone;
}

// The LFVector sizes are about to change (insertion, shrink, device-side use) by
// work issued on `s`: the prefix and the tile table must be rebuilt before the
// next walk.  When that work goes into a graph, every replay changes the sizes
// without the host seeing it, so from then on eager calls rebuild them each time.
inline void sizes_changed(ggarray* a, hipStream_t s) {
  a->prefix_valid = false;
  ++a->sizes_gen;
  if (stream_capturing(s)) a->graph_sized = true;
}

// 0 when `s` is not capturing; otherwise 1 + the capture's id, or ~0 when the id
// cannot be told.  Derived state (prefix, tile table) recorded earlier in the same
// capture is reused by later calls of that capture, never by other graphs.
inline uint64_t stream_capture_tag(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  unsigned long long id = 0;
  if (hipStreamGetCaptureInfo(s, &st, &id) != hipSuccess) return ~0ull;
  if (st == hipStreamCaptureStatusNone) return 0;
  return st == hipStreamCaptureStatusActive ? (uint64_t)id + 1 : ~0ull;
}

// Whether derived state built under capture tag `built` may serve a call under
// capture tag `now` (the same sizes assumed): eagerly built state serves eager
// calls unless a graph changes the sizes, state recorded in a capture serves
// later calls of that capture.
inline bool capture_reuse(const ggarray* a, uint64_t built, uint64_t now) {
  return built == now && now != ~0ull && (now != 0 || !a->graph_sized);
}

struct gga_static {
  void* data;
  uint64_t cap;
  uint32_t elem_bytes;
  void* meta;          // device block: size counter, sticky error, round completion count
  uint64_t* d_size;
  uint32_t* d_err;
  uint32_t* d_done;
  bool rw_last;        // the last operation was an r/w (its loads then stream past the caches)
  uint64_t size_ub;    // host upper bound of the size (sizes the r/w grid)
};

namespace gga {
struct BatchArr;
}

// A set of arrays driven together (one launch per phase for all of them).
struct gga_batch {
  ggarray** arrays;
  uint32_t n;
  uint32_t elem_bytes;
  gga::BatchArr* d_arrays;   // device: the arrays' descriptors (rw, flatten, scans)
  uint64_t* d_tile_begin;    // device: n + 1 exclusive prefix of the arrays' tiles
  uint64_t* d_elem_begin;    // device: n + 1 exclusive prefix of the arrays' sizes
  uint32_t* d_err;           // device: sticky batch error (flatten output too small)
  uint64_t* d_vbegin;        // device: n + 1 exclusive prefix of the arrays' LFVector counts
  uint64_t total_vectors;
  uint32_t stream_blocks;    // workgroups of the r/w and flatten launches (0: default)
  uint64_t* h_pin;           // pinned host scratch
  // Round tables uploaded so far (descriptors + block offsets), reused when the
  // same round shape comes again, so a captured graph always reads a stable table.
  struct Table {
    uint64_t key;           // hash of the round's shape (look-back buffers excluded)
    uint64_t blocks;
    gga::BatchArr* items;   // device
    uint64_t* begins;       // device
    gga::BatchArr* host;    // host copy of items
  };
  Table* tables;
  uint32_t n_tables;
  uint32_t cap_tables;
  // Prefix scans and tile table of the batch, valid for the member arrays' size
  // generations they were built for (see batch_gen).
  bool scan_valid;
  uint64_t scan_gen;
  uint64_t scan_tag;       // capture tags the scans and the table were built under
  uint64_t tab_tag;
  uint64_t* tile_tab;      // device: two words per tile of the whole batch
  uint64_t tab_cap;
  bool tab_valid;
  uint64_t tab_gen;
  void* retired[64];       // outgrown tables, freed with the batch
  uint32_t n_retired;
  // Persistent step (gga_batch_step): the batch index of every LFVector, the
  // launch's barrier words (zero between launches) and chunk totals, and the
  // per-round thread-count tables uploaded so far (reused by shape, so that a
  // captured step uploads nothing).
  uint32_t* d_varr;
  uint32_t* d_step_sync;
  uint64_t* d_step_chunks;
  uint64_t* d_step_vsize;    // final size of every LFVector (the per-wave step's flatten prefix)
  struct StepCounts {
    uint64_t key;
    uint64_t* dev;
  };
  StepCounts* step_counts;
  uint32_t n_step_counts;
  uint32_t cap_step_counts;
};

struct gga_semistatic {
  gga_static st;      // current buffer, resized by the host
  uint64_t resizes;
};

struct gga_mapped {
  gga_static st;                    // data = start of the reserved range, cap = mapped elements
  uint64_t va_bytes;                // reserved range
  uint64_t mapped_bytes;
  uint64_t gran;                    // allocation granularity
  int device;
  uint64_t maps;
  uint64_t n_handles, cap_handles;
  hipMemGenericAllocationHandle_t* handles;
  uint64_t* handle_bytes;
};

namespace gga {

// One array of a batch as the batch kernels see it, with its share of the
// current insertion round.
struct BatchArr {
  ArrRef A;
  uint64_t n_threads;  // logical threads of this array in the round
  uint64_t chunk;      // ceil(n_threads / V)
  uint64_t tpv;        // tiles per LFVector
  uint64_t tag;        // key of this array's generated payloads (keyed rounds)
  uint32_t index;      // position in the batch
  uint32_t elem_log2;
};

// Largest i in [0, n) with begins[i] <= x, where begins is non-decreasing and
// begins[0] <= x: a 64-way search by one wave (each round one load per lane).
__device__ __forceinline__ uint32_t wave_search(const uint64_t* begins, uint32_t n, uint64_t x) {
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t step = (hi - lo + 63) / 64;
    const uint32_t idx = lo + lane * step;
    const bool ok = idx < hi && begins[idx] <= x;
    const uint64_t m = __ballot(ok);
    const uint32_t last = 63u - (uint32_t)__clzll(m);
    lo = lo + last * step;
    hi = lo + step < hi ? lo + step : hi;
  }
  return lo;
}

// One insertion round of a persistent step (gga_batch_step).
constexpr uint32_t kMaxStepRounds = 8;
struct StepRound {
  uint32_t kind;       // kModeBernoulli, kModeRoundTag or kModeKeyed
  uint32_t round;
  uint64_t seed;
  uint32_t tag_shift;
  uint32_t pad;
  uint64_t tag;        // keyed: the batch's tag; array i adds i
};
struct StepDesc {
  uint32_t n_rounds;
  uint32_t clear;  // shrink every LFVector 1/1 ahead of the rounds (buckets it uses again stay in place)
  StepRound r[kMaxStepRounds];
};
constexpr uint32_t kStepChunkMax = 1024;  // LFVector chunks of the step's size prefix
constexpr uint32_t kOpNone = 0xFFFFFFFEu; // a step without r/w

// One r/w or flatten request of a served step, on an array of its own.
constexpr uint32_t kOpFlatten = 0xFFFFFFFFu;
struct ServeItem {
  ArrRef A;
  void* out;          // flatten destination
  uint64_t cap;       // elements reserved at out
  uint64_t* len_out;  // device word that receives the flattened length (may be null)
  uint32_t op;        // r/w operation, or kOpFlatten
  uint32_t elem_log2;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The r/w operation on the elements of one 16-byte vector.
template <typename T>
__device__ __forceinline__ u32x4 op_vec(uint32_t op, u32x4 x) {
  if (sizeof(T) == 4) {
    x.x = apply_op<uint32_t>(op, x.x);
    x.y = apply_op<uint32_t>(op, x.y);
    x.z = apply_op<uint32_t>(op, x.z);
    x.w = apply_op<uint32_t>(op, x.w);
  } else {
    uint64_t lo = ((uint64_t)x.y << 32) | x.x, hi = ((uint64_t)x.w << 32) | x.z;
    lo = apply_op<uint64_t>(op, lo);
    hi = apply_op<uint64_t>(op, hi);
    x.x = (uint32_t)lo;
    x.y = (uint32_t)(lo >> 32);
    x.z = (uint32_t)hi;
    x.w = (uint32_t)(hi >> 32);
  }
  return x;
}

// A 16-byte store that streams past the caches (nt) with device-scope coherence
// (sc1).  Used by the insertion of generated payloads: on configuration 2 the r/w
// that follows the rounds reads such lines faster than after plain non-temporal
// stores (step 0.919 -> 0.907 ms, r/w 5.52 -> 5.61 TB/s, three runs each; sc1
// alone or no hint behave like plain write-back stores, whose dirty lines the
// r/w pays for).
// There is no builtin for the sc1 bit, hence the inline assembly.  The compiler
// does not count this store in its wait counters: a later wait that it places
// for a load also covers the store (the vector-memory counter completes in
// order), so the store only makes such waits longer, never too short.
__device__ __forceinline__ void store_nt_sc1(gptr<u32x4> p, u32x4 x) {
  asm volatile("global_store_dwordx4 %0, %1, off nt sc1" : : "v"(p), "v"(x) : "memory");
}

// Elements an LFVector of s elements keeps when a shrink pops floor(s num / den)
// of them (num <= den; the product is split so that it cannot overflow).
__host__ __device__ __forceinline__ uint64_t shrink_keep(uint64_t s, uint32_t num, uint32_t den) {
  return s - ((s / den) * num + ((s % den) * num) / den);
}

// Lane b of a wave releases bucket b of LFVector v when keep <= b < hi: a live
// bucket goes back to the pool and its slot is cleared (a failed-allocation
// marker is only cleared).  With `held` the caller passes the slot's value in
// `cur` (a bucket it allocated itself), otherwise it is read.
__device__ __forceinline__ void release_bucket(const ArrRef& A, uint32_t v, uint32_t b, uint32_t keep, uint32_t hi,
                                               bool held, uint64_t cur, uint32_t elem_log2) {
  if (b < keep || b >= hi) return;
  uint64_t* slot = A.bptr + (uint64_t)v * kMaxBuckets + b;
  const uint64_t p = held ? cur : *slot;
  if (p > kFailedPtr)
    pool_free(A.pool, reinterpret_cast<uint8_t*>(p), bucket_class(A.log2F, elem_log2, b), pool_shard(v, b, A.salt));
  if (p) *slot = 0;
}

// Shrink (pop floor(s num / den) per LFVector) and bucket release: one wave per
// LFVector, lane b looks after bucket b, so the releases of one LFVector run in
// parallel and go to different pool shards.
__device__ __forceinline__ void shrink_vector(const ArrRef& A, uint32_t v, uint32_t num, uint32_t den,
                                              uint32_t elem_log2) {
  const uint32_t b = threadIdx.x & 63u;
  const uint64_t s = A.size[v];
  const uint64_t ns = shrink_keep(s, num, den);
  uint32_t hi = A.dead[v] ? (uint32_t)kMaxBuckets : nbuckets_for(A.log2F, s);
  if (hi > (uint32_t)kMaxBuckets) hi = kMaxBuckets;
  release_bucket(A, v, b, nbuckets_for(A.log2F, ns), hi, false, 0, elem_log2);
  if (b == 0) A.size[v] = ns;  // every lane has read the old size: one wave, program order
}

// Tiles of an LFVector of s elements: every bucket below s contributes
// ceil(live elements of the bucket / te) tiles.  In closed form: the nb - 1 full
// buckets hold F 2^b elements, one tile each while F 2^b <= te and F 2^b / te
// tiles after that (a geometric sum), and the last bucket holds the rest.
__host__ __device__ __forceinline__ uint64_t tiles_for(uint32_t log2F, uint64_t s, uint32_t te_log2) {
  const uint32_t nb = nbuckets_for(log2F, s);
  if (nb == 0) return 0;
  const uint32_t full = nb - 1;
  const uint32_t small = te_log2 > log2F ? (te_log2 - log2F < full ? te_log2 - log2F : full) : 0u;
  uint64_t n = small;
  if (full > small) n += (1ull << (log2F + full - te_log2)) - (1ull << (log2F + small - te_log2));
  return n + ((s - bucket_start(log2F, full) + (1ull << te_log2) - 1) >> te_log2);
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t x) {
  const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  return x;
}

// Exclusive prefix sums of one array's LFVector sizes and tile counts (entry V
// holds the totals), by one wave: lane l takes a contiguous run of LFVectors.
__device__ __forceinline__ void scan_array_wave(const ArrRef& A, uint32_t te_log2) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t V = A.V;
  const uint32_t per = (V + 63) / 64;
  const uint32_t v0 = lane * per < V ? lane * per : V;
  const uint32_t v1 = v0 + per < V ? v0 + per : V;
  uint64_t e = 0, t = 0;
  for (uint32_t v = v0; v < v1; ++v) {
    const uint64_t s = A.size[v];
    e += s;
    t += tiles_for(A.log2F, s, te_log2);
  }
  const uint64_t ie = wave_incl_scan64(e), it = wave_incl_scan64(t);
  uint64_t re = ie - e, rt = it - t;
  for (uint32_t v = v0; v < v1; ++v) {
    const uint64_t s = A.size[v];
    A.prefix[v] = re;
    A.tprefix[v] = rt;
    re += s;
    rt += tiles_for(A.log2F, s, te_log2);
  }
  const uint64_t te = __shfl(ie, 63, 64), tt = __shfl(it, 63, 64);
  if (lane == 0) {
    A.prefix[V] = te;
    A.tprefix[V] = tt;
  }
}

// How an insertion round produces its candidates.
enum InsertMode : uint32_t {
  kModeBuffer = 0,   // values[gid], flags[gid]
  kModeCounts = 1,   // values[gid * max + j], j < counts[gid]
  kModeBernoulli = 2,
  kModeRoundTag = 3,
  kModePoisson = 4,
  kModeKeyed = 5,    // every thread inserts K(seed, (tag << tag_shift) | gid, round)
};

struct InsertDesc {
  uint32_t mode;
  const void* values;
  const uint8_t* flags;  // flags or counts
  uint32_t max_count;
  uint64_t n_threads;
  uint64_t seed;
  uint32_t round;
  uint32_t tag_shift;
  uint64_t thresholds[16];
  uint64_t tag;
};

// Insertion tile of the 0/1 producers: one wavefront, kInsertSlots candidate
// slots per lane, so kInsertTile logical threads per tile.
#ifndef GGA_INSERT_SLOTS
#define GGA_INSERT_SLOTS 64
#endif
constexpr uint32_t kInsertSlots = GGA_INSERT_SLOTS;
constexpr uint32_t kInsertTile = 64u * kInsertSlots;

// Tile geometry of the element-streaming kernels (rw, flatten): 16 KiB per tile.
constexpr uint32_t kRwThreads = 256;
__host__ __device__ constexpr uint32_t rw_tile_elems(uint32_t elem_log2) {
  return 16384u >> elem_log2;
}

// An insertion round, then (sh_den != 0) a shrink sh_num / sh_den fused into the
// same launch where the round runs one wave per LFVector, else launched after it.
int launch_insert(ggarray* a, const InsertDesc& d, hipStream_t s, uint32_t sh_num = 0, uint32_t sh_den = 0);
// Round numbers and thread counts of the rounds one launch runs.
constexpr uint32_t kMaxFusedRounds = GGA_MAX_ROUNDS;
struct RoundList {
  uint32_t n;
  uint32_t round[kMaxFusedRounds];
  uint64_t n_threads[kMaxFusedRounds];
};
int launch_insert_rounds(ggarray* a, const InsertDesc* ds, uint32_t n, hipStream_t s, uint32_t sh_num,
                         uint32_t sh_den, bool clear);
int launch_static_insert(gga_static* st, const InsertDesc& d, hipStream_t s);
int launch_static_insert_atomic(gga_static* st, const InsertDesc& d, hipStream_t s);
int launch_scan(ggarray* a, hipStream_t s, uint64_t* copy = nullptr);
int launch_insert_packed(ggarray* a, const void* values, const uint8_t* counts, uint64_t n_threads,
                         uint64_t n_values, hipStream_t s);
// The same round with its per-call buffers in the library's static scratch.
int launch_insert_packed_noalloc(ggarray* a, const void* values, const uint8_t* counts, uint64_t n_threads,
                                 uint64_t n_values, hipStream_t s);
int launch_insert_segments(ggarray* a, const void* values, const uint64_t* prefix, uint64_t n_values,
                           hipStream_t s);  // copy: also write the prefix there
int launch_shrink(ggarray* a, uint32_t num, uint32_t den, hipStream_t s);
int launch_rw(ggarray* a, uint32_t op, hipStream_t s);
int launch_flatten(ggarray* a, void* out, uint64_t cap, hipStream_t s);
int launch_rw_global(ggarray* a, uint32_t op, hipStream_t s);
int launch_gather(ggarray* a, const uint64_t* idx, uint64_t n, void* out, hipStream_t s);
int launch_capacity(ggarray* a, uint64_t* d_out, hipStream_t s);
int launch_free_all(ggarray* a, hipStream_t s);
int launch_static_rw(gga_static* st, uint32_t op, hipStream_t s);
int launch_batch_insert(gga_batch* b, const InsertDesc& d, const uint64_t* n_threads, hipStream_t s);
// A whole step of the batch in one persistent launch (d_counts: rounds x n
// thread counts on the device; out NULL: no flatten).
int launch_batch_step(gga_batch* b, const StepDesc& D, const uint64_t* d_counts, uint32_t op, void* out,
                      uint64_t out_cap, hipStream_t s);
int launch_batch_scan(gga_batch* b, hipStream_t s);
int launch_batch_shrink(gga_batch* b, uint32_t num, uint32_t den, hipStream_t s);
int launch_batch_stream(gga_batch* b, uint32_t op, void* out, uint64_t cap, bool flatten, hipStream_t s);

// Served steps.  prepare_round_item fills the descriptor of one insertion round of
// n threads on a (growing its look-back words on stream s when the round's kernel
// uses them) and returns its tiles.
int prepare_round_item(ggarray* a, uint64_t n, uint64_t tag, uint32_t index, BatchArr* item, uint64_t* ntiles,
                       hipStream_t s, bool lookback);
// launch_serve_front: the step's append rounds (keyed payloads) and the size
// scans of the n_s arrays in sitems, one launch.  launch_serve_stream: the r/w
// and flatten requests of sitems (scanned before), one streaming launch (plus one
// prefix launch when n_s exceeds kServeFusedItems).
constexpr uint32_t kServeFusedItems = 4096;
int launch_serve_front(const BatchArr* items, const uint64_t* begins, uint32_t n_a, uint64_t blocks,
                       const ServeItem* sitems, uint32_t n_s, uint32_t elem_bytes, uint64_t seed, uint32_t round,
                       uint32_t shift, hipStream_t s);
int launch_serve_stream(const ServeItem* items, uint32_t n, uint64_t* tile_begin, uint64_t* elem_begin,
                        uint32_t* err, uint32_t elem_bytes, uint32_t grid, hipStream_t s);

inline int hip_status(hipError_t e) { return e == hipSuccess ? GGA_OK : GGA_EHIP; }

// Host upper bound of an array's size: raised by the elements a round may add,
// dropped to zero by a full shrink, unknown (maximal) after user kernels.
// FNV-1a over n bytes (host): keys of the uploaded round and step tables.
inline uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
  const uint8_t* b = static_cast<const uint8_t*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 0x100000001B3ull;
  return h;
}

inline void grow_bound(ggarray* a, uint64_t n) {
  const uint64_t lim = ~0ull >> 2;
  a->size_ub = n > lim - a->size_ub ? lim : a->size_ub + n;
}

}  // namespace gga
