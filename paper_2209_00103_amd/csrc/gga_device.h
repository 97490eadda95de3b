// Device-side layout and primitives of the GGArray library (gfx950).
//
// Layout in HBM
//   pool:   [PoolHdr | pad to 4 KiB | bucket region ...]   (caller-owned memory)
//   array:  size[V] u64 | bptr[V][kMaxBuckets] u64 | dead[V] u32 |
//           alloc_done[V] u32 | prefix[V+1] u64 | tprefix[V+1] u64 | err u32 |
//           ticket u64 | status[...] u64 (look-back words, grown on demand)
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
constexpr int kShards = 8;          // free-list shards per size class
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

struct PoolHdr {
  uint64_t bump;        // next unused byte of the bucket region
  uint64_t limit;       // bytes in the bucket region
  uint64_t in_use;      // bytes handed out and not returned
  uint64_t high_water;  // max of in_use
  uint64_t n_alloc;
  uint64_t n_free;
  uint64_t n_attempt;   // allocation attempts (fault injection counts these)
  uint64_t fault_at;    // attempt number that fails; 0 = never
  uint64_t heads[kNumClasses * kShards];  // tagged Treiber-stack heads
};

constexpr uint64_t kPoolHdrBytes = 4096;
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
  uint64_t* ticket;
  uint64_t* status;
  PoolRef pool;
  uint32_t V;
  uint32_t log2F;
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
__device__ __forceinline__ void fetch_max(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas_acq_rel(uint64_t* p, uint64_t& expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_ACQ_REL,
                                              __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
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
// Lock-free pool: one tagged Treiber stack per (size class, shard) holds freed
// blocks, a bump pointer hands out fresh ones.  A stack head packs a 24-bit
// version tag above the 40-bit block index (offset / 256 + 1, 0 = empty); the
// tag changes on every successful update so a stale head never matches (ABA).
// A free block stores the index of the next free block in its first 8 bytes.
__device__ __forceinline__ uint8_t* pool_alloc(PoolRef P, uint32_t cls, uint32_t shard) {
  PoolHdr* H = P.hdr;
  const uint64_t bytes = 1ull << cls;
  const uint64_t fault_at = ld_rlx(&H->fault_at);
  if (fault_at) {
    uint64_t n = fetch_add(&H->n_attempt, 1) + 1;
    if (n == fault_at) return nullptr;
  }
  if (cls > (uint32_t)kMaxClassLog2) return nullptr;
  for (int k = 0; k < kShards; ++k) {
    uint64_t* head = &H->heads[cls * kShards + ((shard + k) & (kShards - 1))];
    if ((ld_rlx(head) & kIdxMask) == 0) continue;  // empty: skip the acquire
    uint64_t h = ld_acq(head);
    while (h & kIdxMask) {
      const uint64_t off = ((h & kIdxMask) - 1) << kMinClassLog2;
      const uint64_t nxt = ld_rlx(reinterpret_cast<const uint64_t*>(P.base + off)) & kIdxMask;
      const uint64_t nh = (((h >> 40) + 1) << 40) | nxt;
      if (cas_acq_rel(head, h, nh)) {
        uint64_t used = fetch_add(&H->in_use, bytes) + bytes;
        fetch_max(&H->high_water, used);
        fetch_add(&H->n_alloc, 1);
        return P.base + off;
      }
    }
  }
  const uint64_t old = fetch_add(&H->bump, bytes);
  if (old + bytes > ld_rlx(&H->limit)) {
    __hip_atomic_fetch_sub(&H->bump, bytes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return nullptr;
  }
  uint64_t used = fetch_add(&H->in_use, bytes) + bytes;
  fetch_max(&H->high_water, used);
  fetch_add(&H->n_alloc, 1);
  return P.base + old;
}

__device__ __forceinline__ void pool_free(PoolRef P, uint8_t* ptr, uint32_t cls, uint32_t shard) {
  PoolHdr* H = P.hdr;
  const uint64_t bytes = 1ull << cls;
  const uint64_t idx = ((uint64_t)(ptr - P.base) >> kMinClassLog2) + 1;
  uint64_t* head = &H->heads[cls * kShards + (shard & (kShards - 1))];
  uint64_t h = ld_rlx(head);
  for (;;) {
    st_rlx(reinterpret_cast<uint64_t*>(ptr), h & kIdxMask);
    const uint64_t nh = (((h >> 40) + 1) << 40) | idx;
    if (cas_acq_rel(head, h, nh)) break;
  }
  __hip_atomic_fetch_sub(&H->in_use, bytes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  fetch_add(&H->n_free, 1);
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

}  // namespace gga
