// Device-side layout and primitives of the GGArray library (gfx950), and the
// device API for user kernels: gga::block_push_back, the block-cooperative
// push_back of Alg. 1 callable from any HIP kernel (see the end of this file).
//
// Layout in HBM
//   pool:   [PoolHdr | pad to 2 MiB | bucket region ...]   (caller-owned memory)
//   array:  size[V] u64 | bptr[V][kMaxBuckets] u64 | dead[V] u32 |
//           alloc_done[V] u32 | prefix[V+1] u64 | tprefix[V+1] u64 |
//           vticket[V] u64 | rbase[V] u64 | err u32 | status[...] u64
//           (look-back words, grown on demand)
//
// Bucket law (Alg. 2): bucket b of an LFVector holds F * 2^b elements, F a power
// of two, so bucket b starts at local index F * (2^b - 1).  For local index i,
// p = i + F has its top set bit at h = floor(log2 p); then the bucket is
// b = h - log2 F and the offset inside it is p - 2^h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gga {

constexpr int kMaxBuckets = 40;     // F * (2^40 - 1) elements per LFVector
constexpr int kMinClassLog2 = 8;    // smallest pool block: 256 B
constexpr int kMaxClassLog2 = 40;   // largest pool block: 1 TiB
constexpr int kNumClasses = kMaxClassLog2 + 1;
constexpr int kFreeShards = 4096;   // pool free-list shards
constexpr int kArenaShards = 256;   // pool arena / statistics shards
constexpr uint64_t kFailedPtr = 1;  // bucket-table marker: allocation failed
constexpr uint64_t kIdxMask = (1ull << 40) - 1;

// Sticky device error codes (the host maps them to GGA_* statuses).
constexpr uint32_t kErrNoMem = 2;   // reported as GGA_ENOMEM
constexpr uint32_t kErrRange = 3;   // reported as GGA_ERANGE
constexpr uint32_t kErrStall = 4;   // a bounded wait expired; reported as GGA_EHIP

// Every cross-workgroup wait is bounded: after this many polls (seconds of
// waiting, far beyond any legitimate wait) it gives up and sets kErrStall, so a
// logic error surfaces as a status instead of a kernel that never ends.
constexpr uint32_t kSpinLimit = 1u << 22;

struct PoolShard {        // one 64-byte line per shard
  uint64_t arena;         // current chunk id (offset / 256 + 1) << 32 | used 256-byte units
  uint64_t in_use;        // bytes handed out and not returned (may wrap per shard)
  uint64_t n_alloc;
  uint64_t n_free;
  uint64_t pad[4];
};

struct PoolHdr {
  uint64_t bump;          // next unused byte of the region for chunks and large blocks
  uint64_t limit;         // bytes in the region
  uint64_t chunk_log2;    // arena chunk size
  uint64_t n_attempt;     // allocation attempts (fault injection counts these)
  uint64_t fault_at;      // attempt number that fails; 0 = never
  uint64_t pad[3];
  uint64_t nonempty[kNumClasses][kFreeShards / 64];  // bit s: free list s of the class may hold blocks
  uint64_t heads[kNumClasses * kFreeShards];         // tagged Treiber-stack heads
  PoolShard shard[kArenaShards];
};

constexpr uint64_t kPoolHdrBytes = 2ull << 20;
static_assert(sizeof(PoolHdr) <= kPoolHdrBytes, "pool header too large");

struct PoolRef {
  PoolHdr* hdr;
  uint8_t* base;  // start of the bucket region
};

// Everything a kernel needs to reach one array's device metadata.
struct ArrRef {
  uint64_t* size;
  uint64_t* bptr;
  uint32_t* dead;
  uint32_t* alloc_done;  // this round's bucket allocations: count | failures << 16
  uint64_t* prefix;
  uint64_t* tprefix;
  uint32_t* err;
  uint64_t* vticket;     // per-LFVector tile tickets of the insertion kernel
  uint64_t* rbase;       // per-LFVector size before the current dense round (grow -> store)
  uint64_t* status;
  PoolRef pool;
  uint32_t V;
  uint32_t log2F;
  uint32_t salt;         // spreads the pool shards of different arrays
  uint32_t spin;         // polls before a bounded wait gives up (kSpinLimit; a
                         // failure-handling test may lower it from the host)
};

// ------------------------------------------------------------------ atomics --
// Agent-scope atomics: the 8 XCDs of the MI355X each have their own L2, so
// words shared between workgroups go through agent-scope atomics, which the
// compiler lowers to the coherent forms of the gfx950 memory model.
__device__ __forceinline__ uint64_t ld_acq(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_rlx(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_acq32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_rlx32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t fetch_add(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t fetch_add32(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void set_error(uint32_t* err, uint32_t code) {
  uint32_t zero = 0;
  __hip_atomic_compare_exchange_strong(err, &zero, code, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void spin_pause() { __builtin_amdgcn_s_sleep(1); }

// --------------------------------------------------------------- bucket law --
__host__ __device__ __forceinline__ uint64_t bucket_start(uint32_t log2F, uint32_t b) {
  return ((1ull << b) - 1) << log2F;
}
__host__ __device__ __forceinline__ uint64_t bucket_len(uint32_t log2F, uint32_t b) {
  return 1ull << (b + log2F);
}
__device__ __forceinline__ uint32_t bucket_of(uint32_t log2F, uint64_t idx) {
  uint64_t p = idx + (1ull << log2F);
  return (63u - (uint32_t)__clzll(p)) - log2F;
}
__device__ __forceinline__ uint64_t offset_in(uint32_t log2F, uint64_t idx, uint32_t b) {
  return idx - bucket_start(log2F, b);
}
// Buckets held by an LFVector of s elements: the b with start_b < s.
__host__ __device__ __forceinline__ uint32_t nbuckets_for(uint32_t log2F, uint64_t s) {
  if (s == 0) return 0;
  uint64_t p = (s - 1) + (1ull << log2F);
#ifdef __HIP_DEVICE_COMPILE__
  uint32_t h = 63u - (uint32_t)__clzll(p);
#else
  uint32_t h = 63u - (uint32_t)__builtin_clzll(p);
#endif
  return h - log2F + 1;
}
// Pool size class (log2 bytes) of bucket b.
__device__ __forceinline__ uint32_t bucket_class(uint32_t log2F, uint32_t elem_log2, uint32_t b) {
  uint32_t c = log2F + b + elem_log2;
  return c < (uint32_t)kMinClassLog2 ? (uint32_t)kMinClassLog2 : c;
}

// ------------------------------------------------------------- device pool --
// Lock-free bucket pool over the caller's region, built so that thousands of
// LFVectors can grow in the same kernel without meeting on one address:
//
//  * Bucket b of LFVector v of an array with salt z belongs to free-list shard
//    f = (v + b + z) mod 4096 and to arena shard (f / 16) mod 256, so the
//    LFVectors of an array (up to 4096 of them) never share a free list for a
//    given bucket, and a bucket released by shrink is found again by the same
//    LFVector.  Sixteen consecutive LFVectors share an arena shard, so buckets
//    that grow in the same launch lie side by side in the order in which r/w
//    and flatten visit them (scattered 8-64 KiB buckets stream about 5% slower
//    than the same bytes in address order; configuration 3's r/w measured
//    4.79-4.93 -> 4.84-5.07 TB/s with this mapping, insertion unchanged).
//  * Freed blocks go to one tagged Treiber stack per (size class, free shard).
//    A head packs a 24-bit version tag above the 40-bit block index (offset /
//    256 + 1, 0 = empty); the tag changes on every update, so a stale head never
//    matches (ABA).  A free block keeps the index of the next one in its first
//    8 bytes.  A per-class bit mask hints which free lists may hold blocks.
//  * Fresh blocks up to a quarter of a chunk come from the arena shard: a chunk
//    carved from the global bump pointer, sub-allocated with one atomic add on
//    the shard's arena word (chunk id << 32 | used 256-byte units).  The add that
//    crosses the end of the chunk installs the next chunk; adds that land past
//    the end in the meantime take their block from the global bump pointer
//    instead of waiting.  Larger blocks always come from the global bump pointer.
//  * Only when the region is exhausted does an allocation look through the other
//    free lists (steal), guided by the hint masks.
//
// No operation uses release/acquire fences (on gfx950 those write back or
// invalidate the whole L2 of an XCD).  Ordering comes from completion: a push
// writes the link with an atomic exchange and waits for its return before the
// head CAS is issued; a pop reads the head, then the link at an address that
// depends on it, then CASes values that depend on both.  All are agent-scope
// atomics, performed at the coherence point in that order.
__device__ __forceinline__ uint32_t pool_shard(uint32_t v, uint32_t b, uint32_t salt) {
  return (v + b + salt) & (uint32_t)(kFreeShards - 1);
}
__device__ __forceinline__ uint32_t arena_shard(uint32_t f) { return (f >> 4) & (uint32_t)(kArenaShards - 1); }
// The statistics words a block is counted in: neighbouring free-list shards use
// different lines (16 LFVectors that share an arena shard would otherwise meet on
// one counter line in every allocation and release; a clear of configuration 4's
// 81224 LFVectors measured 136 against 95 us).  Only their sum is ever read.
__device__ __forceinline__ uint32_t stat_shard(uint32_t f) { return f & (uint32_t)(kArenaShards - 1); }

__device__ __forceinline__ bool cas_rlx(uint64_t* p, uint64_t& expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_nr(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void sub_nr(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint8_t* pool_pop(PoolRef P, uint32_t cls, uint32_t s) {
  PoolHdr* H = P.hdr;
  uint64_t* head = &H->heads[(uint64_t)cls * kFreeShards + s];
  uint64_t h = ld_rlx(head);
  while (h & kIdxMask) {
    const uint64_t off = ((h & kIdxMask) - 1) << kMinClassLog2;
    const uint64_t nxt = ld_rlx(reinterpret_cast<const uint64_t*>(P.base + off)) & kIdxMask;
    const uint64_t nh = (((h >> 40) + 1) << 40) | nxt;
    if (cas_rlx(head, h, nh)) return P.base + off;  // the shard's hint stays set (see pool_alloc)
  }
  return nullptr;
}

// One atomic add claims [old, old + bytes); a claim that runs past the limit
// fails and is never undone, so the pointer only grows and no two claims
// overlap (at most the tail that the first failing claim passed stays unused).
// (Undoing failed adds is not safe: a failed add undone after a smaller add has
// succeeded past it moves the pointer back over that block, which the next
// allocation then receives a second time.  A compare-and-swap loop is safe but
// serialises the thousands of waves that meet here when a fresh pool installs
// its first arena chunks.)
__device__ __forceinline__ uint8_t* global_bump(PoolRef P, uint64_t bytes) {
  PoolHdr* H = P.hdr;
  const uint64_t limit = H->limit;  // written by the host before any launch
  const uint64_t old = fetch_add(&H->bump, bytes);
  if (old + bytes > limit) return nullptr;
  return P.base + old;
}

__device__ __forceinline__ uint8_t* arena_alloc(PoolRef P, uint32_t s, uint64_t bytes, uint32_t clog) {
  PoolHdr* H = P.hdr;
  const uint64_t units = bytes >> kMinClassLog2;
  const uint64_t cap = 1ull << (clog - kMinClassLog2);
  uint64_t* word = &H->shard[s].arena;
  const uint64_t old = fetch_add(word, units);
  const uint64_t cid = old >> 32, used = old & 0xFFFFFFFFull;
  if (cid && used + units <= cap) return P.base + ((cid - 1) << kMinClassLog2) + (used << kMinClassLog2);
  const bool installer = cid ? (used <= cap && used + units > cap) : (used == 0);
  if (!installer) return nullptr;  // the caller takes the global bump pointer
  uint8_t* c = global_bump(P, 1ull << clog);
  if (!c) {
    __hip_atomic_exchange(word, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return nullptr;
  }
  const uint64_t ncid = ((uint64_t)(c - P.base) >> kMinClassLog2) + 1;
  __hip_atomic_exchange(word, (ncid << 32) | units, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return c;
}

__device__ __forceinline__ uint8_t* pool_alloc(PoolRef P, uint32_t cls, uint32_t fs) {
  PoolHdr* H = P.hdr;
  const uint64_t bytes = 1ull << cls;
  // fault_at and chunk_log2 only change between launches (host writes), so plain
  // loads see them and can issue together with the first atomic.
  const uint64_t fault_at = H->fault_at;
  const uint32_t clog = (uint32_t)H->chunk_log2;
  if (fault_at) {
    const uint64_t n = fetch_add(&H->n_attempt, 1) + 1;
    if (n == fault_at) return nullptr;
  }
  if (cls > (uint32_t)kMaxClassLog2) return nullptr;
  const uint32_t as = arena_shard(fs);
  uint8_t* q = pool_pop(P, cls, fs);
  if (!q && cls + 2 <= clog) q = arena_alloc(P, as, bytes, clog);
  if (!q) q = global_bump(P, bytes);
  // Region exhausted: steal from other shards.  A shard's hint bit is set by
  // every push and cleared only here, when a steal finds the shard empty, so a
  // pop costs no hint update and a set bit may be stale.
  for (uint32_t wi = 0; !q && wi < (uint32_t)kFreeShards / 64; ++wi) {
    uint64_t mask = ld_rlx(&H->nonempty[cls][wi]);
    while (!q && mask) {
      const uint32_t b = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
      const uint32_t s = wi * 64 + b;
      q = pool_pop(P, cls, s);
      if (!q) {
        uint64_t* m = &H->nonempty[cls][wi];
        __hip_atomic_fetch_and(m, ~(1ull << b), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ld_rlx(&H->heads[(uint64_t)cls * kFreeShards + s]) & kIdxMask)  // a push got in between
          __hip_atomic_fetch_or(m, 1ull << b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      mask &= mask - 1;
    }
  }
  if (!q) return nullptr;
  add_nr(&H->shard[stat_shard(fs)].in_use, bytes);
  add_nr(&H->shard[stat_shard(fs)].n_alloc, 1ull);
  return q;
}

__device__ __forceinline__ void pool_free(PoolRef P, uint8_t* ptr, uint32_t cls, uint32_t s) {
  PoolHdr* H = P.hdr;
  const uint64_t idx = ((uint64_t)(ptr - P.base) >> kMinClassLog2) + 1;
  uint64_t* head = &H->heads[(uint64_t)cls * kFreeShards + s];
  uint64_t h = ld_rlx(head);
  for (;;) {
    const uint64_t prev = __hip_atomic_exchange(reinterpret_cast<uint64_t*>(ptr), h & kIdxMask,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // Consuming the exchange's result makes the wave wait until the link has
    // landed before the CAS below can publish the block.
    asm volatile("" ::"v"((uint32_t)prev) : "memory");
    const uint64_t nh = (((h >> 40) + 1) << 40) | idx;
    if (cas_rlx(head, h, nh)) break;
  }
  if ((h & kIdxMask) == 0)
    __hip_atomic_fetch_or(&H->nonempty[cls][s >> 6], 1ull << (s & 63), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
  sub_nr(&H->shard[stat_shard(s)].in_use, 1ull << cls);
  add_nr(&H->shard[stat_shard(s)].n_free, 1ull);
}

// A block of class cls taken for free-list shard s and given back to it in the
// same launch with nothing written into it (a bucket that a round reaches and
// its fused shrink releases again).  When that list is not empty, its pop and
// push would leave it as it was (the top block back on top, with the same link),
// so the call only counts one allocation and one release; an empty list, or a
// pool with fault injection armed, takes the full path (arena or bump pointer,
// failure included, then the push).  Returns false where the allocation fails.
__device__ __forceinline__ bool pool_alloc_release(PoolRef P, uint32_t cls, uint32_t s) {
  PoolHdr* H = P.hdr;
  if (cls <= (uint32_t)kMaxClassLog2 && !H->fault_at &&
      (ld_rlx(&H->heads[(uint64_t)cls * kFreeShards + s]) & kIdxMask)) {
    add_nr(&H->shard[stat_shard(s)].n_alloc, 1ull);
    add_nr(&H->shard[stat_shard(s)].n_free, 1ull);
    return true;
  }
  uint8_t* p = pool_alloc(P, cls, s);
  if (!p) return false;
  pool_free(P, p, cls, s);
  return true;
}

// A block that a clear earlier in the same launch released to free-list shard s,
// taken again by the same LFVector with nothing written to it in between: a
// push followed by a pop of that list gives the block back and leaves the list
// as it was, so the call counts one release and one allocation and the block
// stays where it is.  With fault injection armed the allocation attempt counts
// too and may fail (false: the caller then releases the block for real, as the
// clear would have).
__device__ __forceinline__ bool pool_reuse(PoolRef P, uint32_t s) {
  PoolHdr* H = P.hdr;
  const uint64_t fault_at = H->fault_at;
  if (fault_at && fetch_add(&H->n_attempt, 1) + 1 == fault_at) return false;
  add_nr(&H->shard[stat_shard(s)].n_alloc, 1ull);
  add_nr(&H->shard[stat_shard(s)].n_free, 1ull);
  return true;
}

// -------------------------------------------------------- element pointers --
// Bucket pointers are kept as integers, so the compiler cannot tell that they
// address device memory and would access elements with flat instructions, whose
// completion the hardware counts together with LDS and scalar loads: a wait for
// an LDS read would then also wait for earlier element stores.  Element accesses
// go through this global-memory view instead.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gmem(T* p) {
  return (gptr<T>)p;
}

// ------------------------------------------------------------------ payloads --
// SplitMix64 output for generator state x (Steele, Lea, Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t K(uint64_t seed, uint64_t a, uint64_t b) {
  return splitmix64((seed << 56) ^ (a << 8) ^ b);
}

// r/w operations.
template <typename T>
__device__ __forceinline__ T apply_op(uint32_t op, T x) {
  if (op == 0) return x + (T)1;
  if (op == 1) return x * (T)3 + (T)1;
  return x + (T)30;  // thirty increments by one, folded
}

// ------------------------------------------------------- device-side API --
// Block-cooperative push_back (Alg. 1) for user kernels: the "fully in GPU" use
// the paper designs the structure for.  Obtain the array's ArrRef on the host
// with ggarray_device_ref, pass it to the kernel by value, and call
// ggarray_device_done after the kernel is queued (the next size, r/w or flatten
// then rescans the sizes).
//
// Every thread of the block must call block_push_back, the same number of times,
// with the same LFVector v (the paper assigns one LFVector per block); thread t
// inserts `value` iff keep.  The block's kept elements land at the end of
// LFVector v in thread order; blocks that push to one LFVector concurrently get
// disjoint ranges in the order of their single atomic add on its size, as in
// the paper.  The bucket whose first index falls in a block's range is
// allocated by that block (the Alg. 2 winner); blocks needing it wait for its
// pointer.  Returns the element's local index in v, or ~0 for a thread that
// does not insert.  If a bucket cannot be allocated the elements that would go
// there are dropped, the LFVector is frozen and the array's sticky GGA_ENOMEM
// is set (its contents past the failure are then unspecified).
template <typename T>
__device__ uint64_t block_push_back(const ArrRef& A, uint32_t v, bool keep, T value) {
  __shared__ uint32_t s_wave[16];  // kept elements per wave (up to 1024 threads)
  __shared__ uint64_t s_base;
  __shared__ uint64_t s_bp[64];
  __shared__ uint32_t s_blo;
  const uint32_t tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const uint32_t nthreads = blockDim.x * blockDim.y * blockDim.z;
  const uint32_t lane = tid & 63u, w = tid >> 6, nw = (nthreads + 63u) / 64u;
  const uint64_t m = __ballot(keep);
  const uint32_t rank_w = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  if (lane == 0) s_wave[w] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t before = 0, n = 0;
  for (uint32_t k = 0; k < nw; ++k) {
    if (k < w) before += s_wave[k];
    n += s_wave[k];
  }
  if (tid < 64) {  // wave 0: reserve the range, then allocate or wait for its buckets
    uint64_t base = ~0ull;
    if (tid == 0 && n && !ld_rlx32(&A.dead[v])) base = fetch_add(&A.size[v], n);
    base = __shfl(base, 0, 64);
    uint32_t b_lo = 0;
    if (base != ~0ull) {
      b_lo = bucket_of(A.log2F, base);
      const uint32_t b = b_lo + tid;
      uint64_t p = kFailedPtr;
      if (b <= bucket_of(A.log2F, base + n - 1)) {
        if (b < (uint32_t)kMaxBuckets) {
          uint64_t* slot = &A.bptr[(uint64_t)v * kMaxBuckets + b];
          if (bucket_start(A.log2F, b) >= base) {
            uint8_t* q = pool_alloc(A.pool, bucket_class(A.log2F, sizeof(T) == 4 ? 2u : 3u, b),
                                    pool_shard(v, b, A.salt));
            p = q ? (uint64_t)q : kFailedPtr;
            st_rlx(slot, p);
          } else {
            uint32_t spins = 0;
            while ((p = ld_rlx(slot)) == 0 && spins < A.spin) {
              ++spins;
              spin_pause();
            }
            if (p == 0) {
              p = kFailedPtr;
              set_error(A.err, kErrStall);
            }
          }
        }
        s_bp[tid] = p;
        if (p <= kFailedPtr) {
          set_error(A.err, kErrNoMem);
          st_rlx32(&A.dead[v], 1u);
        }
      }
    }
    if (tid == 0) {
      s_base = base;
      s_blo = b_lo;
    }
  }
  __syncthreads();
  const uint64_t base = s_base;
  if (!keep || base == ~0ull) return ~0ull;
  const uint64_t idx = base + before + rank_w;
  const uint32_t b = bucket_of(A.log2F, idx);
  const uint64_t p = s_bp[b - s_blo];
  if (p > kFailedPtr) gmem(reinterpret_cast<T*>(p))[offset_in(A.log2F, idx, b)] = value;
  return idx;
}

}  // namespace gga
