// Producers of insertion rounds: how logical thread gid decides whether it
// inserts and what (the synthetic workloads of the benchmark configurations and
// the buffer inputs of the C ABI).  Shared by the round kernels and the
// persistent step kernel, so every path produces the same elements.
#pragma once

#include "gga_internal.h"

namespace gga {

// Thread gid inserts values[gid] iff flags[gid] != 0.  Without flags (every
// thread inserts) only the dense kernels run, and they read values alone, so
// flag() reads flags unconditionally (a test per slot would keep each flag load
// under a branch, which costs a memory round trip per slot).
template <typename T>
struct ProdBuffer {
  static constexpr bool kMulti = false;
  static constexpr bool kDense = false;
  static constexpr bool kLoads = true;  // flags and payloads come from memory
  const T* values;
  const uint8_t* flags;
  __device__ __forceinline__ bool flag(uint64_t g) const { return flags[g] != 0; }
  __device__ __forceinline__ T value(uint64_t g) const { return values[g]; }
};
template <typename T>
struct ProdBernoulli {  // h = K(seed, gid, round); insert (T)h iff top bit
  static constexpr bool kMulti = false;
  static constexpr bool kDense = false;
  static constexpr bool kLoads = false;
  uint64_t seed;
  uint32_t round;
  __device__ __forceinline__ bool flag(uint64_t g) const { return (K(seed, g, round) >> 63) != 0; }
  __device__ __forceinline__ T value(uint64_t g) const { return (T)K(seed, g, round); }
  __device__ __forceinline__ bool take(uint64_t g, T& v) const {  // flag and value from one hash
    const uint64_t h = K(seed, g, round);
    v = (T)h;
    return (h >> 63) != 0;
  }
  __device__ __forceinline__ void bind(const BatchArr&) {}
};
template <typename T>
struct ProdRoundTag {  // insert (round << shift) | gid
  static constexpr bool kMulti = false;
  static constexpr bool kDense = true;  // every thread inserts
  static constexpr bool kLoads = false;
  uint32_t round;
  uint32_t shift;
  __device__ __forceinline__ bool flag(uint64_t) const { return true; }
  __device__ __forceinline__ T value(uint64_t g) const { return (T)(((uint64_t)round << shift) | g); }
  __device__ __forceinline__ bool take(uint64_t g, T& v) const {
    v = value(g);
    return true;
  }
  __device__ __forceinline__ void bind(const BatchArr&) {}
};
template <typename T>
struct ProdKeyed {  // every thread inserts K(seed, (tag << shift) | gid, round)
  static constexpr bool kMulti = false;
  static constexpr bool kDense = true;
  static constexpr bool kLoads = false;
  uint64_t seed;
  uint32_t round;
  uint32_t shift;
  uint64_t tag;
  __device__ __forceinline__ bool flag(uint64_t) const { return true; }
  __device__ __forceinline__ T value(uint64_t g) const { return (T)K(seed, (tag << shift) | g, round); }
  __device__ __forceinline__ bool take(uint64_t g, T& v) const {
    v = value(g);
    return true;
  }
  __device__ __forceinline__ void bind(const BatchArr& it) { tag = it.tag; }  // each array its own key
};
template <typename T>
struct ProdCounts {  // insert values[gid * max + j], j < counts[gid]
  static constexpr bool kMulti = true;
  const T* values;
  const uint8_t* counts;
  uint32_t max_count;
  __device__ __forceinline__ uint32_t count(uint64_t g) const {
    const uint32_t c = counts[g];
    return c < max_count ? c : max_count;
  }
  __device__ __forceinline__ T value(uint64_t g, uint32_t r) const {
    return values[g * max_count + r];
  }
};
template <typename T>
struct ProdPoisson {  // c = #{k : K(seed,gid,0x80|round) >= thr[k]}; insert K(seed,gid,16 round + j)
  static constexpr bool kMulti = true;
  uint64_t seed;
  uint32_t round;
  uint32_t max_count;
  uint64_t thr[16];
  __device__ __forceinline__ uint32_t count(uint64_t g) const {
    const uint64_t u = K(seed, g, 0x80u | round);
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) c += (k < (int)max_count && u >= thr[k]) ? 1u : 0u;
    return c;
  }
  __device__ __forceinline__ T value(uint64_t g, uint32_t r) const {
    return (T)K(seed, g, 16u * round + r);
  }
};

}  // namespace gga
