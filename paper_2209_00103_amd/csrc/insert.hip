// Insertion rounds: block-cooperative push_back (Alg. 1) with in-kernel bucket
// growth (Alg. 2), for the GGArray and for the static-array baseline.
//
// The logical threads of a round are cut into tiles, numbered in (LFVector,
// position) order.  For the 0/1 producers (at most one element per thread) one
// wavefront handles one tile of kInsertTile threads; the multi-element producers
// use 256-thread workgroups over 1024-thread tiles.  Per tile:
//   1. the producer's flags (or counts) are evaluated and counted: a wave ballot
//      per candidate slot (mbcnt gives each kept candidate its rank), or a scan
//      of the per-thread counts;
//   2. the tile's first index in its LFVector: the first tile of the LFVector
//      reads the LFVector size, later tiles use a decoupled look-back over the
//      tiles before them (each tile publishes its count, then its inclusive
//      prefix, in one tagged 64-bit word); tiles take per-LFVector tickets, so
//      every tile a tile waits for is held by a wave that is already running;
//   3. the tile allocates every bucket whose first index falls in its range
//      (exactly one tile holds each bucket start, which makes it the Alg. 2
//      winner without a CAS) and waits for the buckets a predecessor allocates;
//   4. the last tile of the LFVector commits the new size, or, if any bucket
//      allocation of the round failed, leaves the size as it was and freezes
//      the LFVector;
//   5. the elements are stored at their positions: with 16-byte non-temporal
//      stores when every thread of the tile inserts into one bucket, else one
//      element per lane and slot, located by the closed form.
// The static baseline replaces 2-4 by one global atomicAdd per tile.
#include <mutex>
#include <new>
#include <type_traits>

#include <hip/hip_ext.h>

#include "gga_internal.h"
#include "producers.h"

namespace gga {
namespace {

constexpr int kB = 256;                  // threads per insertion workgroup
constexpr int kW = kB / 64;              // waves per workgroup
constexpr int kFlagTile = (int)kInsertTile;  // logical threads per tile, 0/1 producers (one wave)
constexpr int kCountK = 4;               // candidates per thread, multi-element producers
constexpr int kCountTile = kB * kCountK; // 1024 logical threads per tile
constexpr uint32_t kOwnWindow = 8192;     // outputs per owner-map pass (16-bit entries, 16 KiB)

// Look-back status word: epoch (30 bits) | flag (2 bits) | value (32 bits).  The
// value is a count or an inclusive prefix relative to the LFVector's size at the
// start of the round (the host rejects rounds that could add 2^32 or more
// elements to one LFVector).  The epoch is the launch number carried by the
// LFVector's ticket word, so words left by earlier launches never match.
constexpr uint64_t kStA = 1;  // status flag: tile count published
constexpr uint64_t kStP = 2;  // status flag: inclusive prefix published
constexpr uint64_t kValMask = 0xFFFFFFFFull;
constexpr uint64_t kEpochMask = (1ull << 30) - 1;

struct TileArgs {
  uint64_t n_threads;
  uint64_t chunk;        // logical threads per LFVector, ceil(n / V)
  uint64_t tpv;          // tiles per LFVector
  uint32_t elem_log2;
  uint32_t sh_num = 0;   // a shrink num / den fused after the round (sh_den 0: none;
  uint32_t sh_den = 0;   // honoured by the one-wave-per-LFVector grow + store only)
  uint32_t reuse = 0;    // a clear came first in the same launch: buckets still in the table are taken again
};

struct StaticRef {
  void* data;
  uint64_t cap;
  uint64_t* size;
  uint32_t* err;
  uint32_t* done;  // waves of the current closed-form round that have finished
};

struct TileShared {
  uint64_t tile;
  uint64_t base;
  uint64_t bp[64];     // bucket pointers of buckets b_lo .. b_lo + nb - 1
  uint32_t b_lo;
  uint32_t nb;
  uint32_t n_tile;
  uint32_t writable;   // static baseline: elements that fit
  uint32_t frozen;     // the LFVector's frozen flag as the block read it
  uint32_t cnt[64];
};

__device__ __forceinline__ uint64_t pack_status(uint64_t epoch, uint64_t flag, uint64_t value) {
  return ((epoch & kEpochMask) << 34) | (flag << 32) | (value & kValMask);
}
__device__ __forceinline__ uint64_t status_flag(uint64_t w) { return (w >> 32) & 3u; }
__device__ __forceinline__ bool status_current(uint64_t w, uint64_t epoch) {
  return (w >> 34) == (epoch & kEpochMask) && status_flag(w) != 0;
}
__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  return x;
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// -------------------------------------------------------- look-back (wave 0) --
// Exclusive prefix of tile `tile`, which is tile t > 0 of its LFVector.  Lane l
// inspects predecessor tile - 1 - l (window of 64), waiting until it has
// published; the nearest predecessor with an inclusive prefix ends the search.
// Returns false if a bounded wait expired.
__device__ bool lookback(const uint64_t* status, uint64_t tile, uint64_t t, uint64_t epoch,
                         uint32_t limit, uint64_t& out) {
  const uint32_t lane = lane_id();
  const int64_t lo = (int64_t)(tile - t);
  int64_t hi = (int64_t)tile - 1;
  uint64_t sum = 0;
  for (;;) {
    const int64_t mine = hi - (int64_t)lane;
    const bool in = mine >= lo;
    uint64_t w = 0;
    bool ok = true;
    if (in) {
      for (uint32_t spins = 0;; ++spins) {
        w = ld_rlx(&status[mine]);
        if (status_current(w, epoch)) break;
        if (spins >= limit) {
          ok = false;
          break;
        }
        spin_pause();
      }
    }
    if (__ballot(!ok)) return false;
    const uint64_t pmask = __ballot(in && status_flag(w) == kStP);
    if (pmask) {
      const uint32_t first = (uint32_t)__ffsll((unsigned long long)pmask) - 1u;
      sum += wave_sum64((in && lane <= first) ? (w & kValMask) : 0ull);
      out = sum;
      return true;
    }
    sum += wave_sum64(in ? (w & kValMask) : 0ull);
    hi -= 64;
  }
}

// ------------------------------------------------ growth + commit (one wave) --
// What a tile needs to store its elements.  Wave-uniform except bp.
struct WaveRes {
  uint64_t base;   // index of the tile's first element in its LFVector
  uint64_t bp;     // lane i: pointer of bucket b_lo + i (kFailedPtr if none)
  uint32_t b_lo;
  uint32_t nb;
  uint32_t n_out;  // elements to store: the tile count, or 0 if the tile stalled
};

// Resolves the tile's first index, allocates or waits for its buckets, and lets
// the last tile of the LFVector commit the round.  Executed by one whole wave.
// size0 is the LFVector size the caller read when it started (used when t == 0;
// only the last tile of the LFVector writes the size, after every other tile of
// the round has published, so an early read is current).
__device__ WaveRes resolve_wave(const ArrRef& A, const TileArgs& I, uint32_t v, uint64_t t,
                                uint64_t tile, bool is_last, uint32_t n_t, uint64_t size0,
                                uint64_t epoch) {
  WaveRes r{0, kFailedPtr, 0, 0, 0};
  const uint32_t lane = lane_id();
  const uint32_t log2F = A.log2F;
  const uint64_t old_size = size0;
  uint64_t base = 0;
  bool stalled = false;
  if (t == 0) {
    if (lane == 0 && !is_last) st_rlx(&A.status[tile], pack_status(epoch, kStP, n_t));
    base = old_size;
  } else {
    uint64_t rel = 0;
    if (lane == 0 && !is_last) st_rlx(&A.status[tile], pack_status(epoch, kStA, n_t));
    stalled = !lookback(A.status, tile, t, epoch, A.spin, rel);
    if (lane == 0 && !is_last && !stalled)
      st_rlx(&A.status[tile], pack_status(epoch, kStP, rel + n_t));
    base = old_size + rel;
  }
  if (stalled) {
    // Predecessors never published: leave the LFVector as it was and freeze it.
    if (lane == 0) {
      set_error(A.err, kErrStall);
      st_rlx32(&A.dead[v], 1u);
    }
    return r;
  }

  uint32_t b_lo = 0, nb = 0, n_alloc = 0, n_fail = 0;
  if (n_t) {
    b_lo = bucket_of(log2F, base);
    nb = bucket_of(log2F, base + n_t - 1) - b_lo + 1;
    const uint32_t b = b_lo + lane;
    bool allocated = false, failed = false, late = false;
    if (lane < nb) {
      uint64_t p = kFailedPtr;
      const bool holds_start = bucket_start(log2F, b) >= base;
      if (b >= (uint32_t)kMaxBuckets) {
        allocated = failed = holds_start;
      } else {
        uint64_t* slot = &A.bptr[(uint64_t)v * kMaxBuckets + b];
        if (holds_start) {
          // This tile writes the bucket's first index: it is the one that allocates.
          uint8_t* q = pool_alloc(A.pool, bucket_class(log2F, I.elem_log2, b), pool_shard(v, b, A.salt));
          p = q ? (uint64_t)q : kFailedPtr;
          st_rlx(slot, p);
          allocated = true;
          failed = !q;
        } else {
          uint32_t spins = 0;
          while ((p = ld_rlx(slot)) == 0 && spins < A.spin) {
            ++spins;
            spin_pause();
          }
          if (p == 0) {
            p = kFailedPtr;
            late = true;
          }
        }
      }
      r.bp = p;
    }
    // One atomic reports an earlier tile's allocations to the last tile: the
    // count in the low half, the failures in the high half.  The last tile
    // counts its own allocations locally.
    n_alloc = (uint32_t)__popcll(__ballot(allocated));
    n_fail = (uint32_t)__popcll(__ballot(failed));
    if (lane == 0 && n_fail) set_error(A.err, kErrNoMem);
    if (lane == 0 && __ballot(late)) {  // elements of this tile stay unwritten: freeze
      set_error(A.err, kErrStall);
      st_rlx32(&A.dead[v], 1u);
    }
    if (lane == 0 && n_alloc && !is_last) fetch_add32(&A.alloc_done[v], n_alloc | (n_fail << 16));
  }

  if (is_last && lane == 0) {
    const uint64_t old = old_size;
    const uint64_t nsize = base + n_t;
    const uint32_t others = nbuckets_for(log2F, nsize) - nbuckets_for(log2F, old) - n_alloc;
    uint32_t failed = n_fail;
    if (others) {
      uint32_t done, spins = 0;
      while (((done = ld_rlx32(&A.alloc_done[v])) & 0xFFFFu) < others && spins < A.spin) {
        ++spins;
        spin_pause();
      }
      if ((done & 0xFFFFu) < others) {
        set_error(A.err, kErrStall);
        failed = 1;
      } else {
        failed += done >> 16;
        st_rlx32(&A.alloc_done[v], 0u);
      }
    }
    if (failed)
      st_rlx32(&A.dead[v], 1u);
    else
      st_rlx(&A.size[v], nsize);
  }
  r.base = base;
  r.b_lo = b_lo;
  r.nb = nb;
  r.n_out = n_t;
  return r;
}

// Block kernels: wave 0 resolves and leaves the result in LDS.
__device__ __forceinline__ void resolve_tile(const ArrRef& A, const TileArgs& I, uint32_t v, uint64_t t,
                                             uint64_t tile, bool is_last, uint32_t n_t, uint64_t epoch,
                                             TileShared& sh) {
  const uint32_t lane = lane_id();
  uint64_t size0 = 0;
  if (lane == 0) size0 = ld_rlx(&A.size[v]);
  const WaveRes r = resolve_wave(A, I, v, t, tile, is_last, n_t, __shfl(size0, 0, 64), epoch);
  if (lane < r.nb) sh.bp[lane] = r.bp;
  if (lane == 0) {
    sh.base = r.base;
    sh.b_lo = r.b_lo;
    sh.nb = r.nb;
    sh.n_tile = r.n_out;
  }
}

// Static baseline: one global atomic per tile claims the index range.
__device__ void resolve_static(const StaticRef& S, uint32_t n_t, TileShared& sh) {
  if (threadIdx.x == 0) {
    const uint64_t base = n_t ? fetch_add(S.size, n_t) : 0;
    uint64_t fit = 0;
    if (base < S.cap) fit = (S.cap - base) < n_t ? (S.cap - base) : n_t;
    if (fit < n_t) set_error(S.err, kErrRange);
    sh.base = base;
    sh.writable = (uint32_t)fit;
  }
}

// Takes this block's ticket of LFVector v (one lane; the result is waited for
// later).  The ticket word is epoch << 32 | count.  The LFVector's tpv blocks
// each take one; the last taker resets the count and advances the epoch, so the
// next launch's tiles tag their status words differently.  Every launch with
// several tiles per LFVector advances every LFVector's epoch once, so all
// LFVectors of an array share one epoch sequence.
__device__ __forceinline__ uint64_t take_ticket(const ArrRef& A, uint32_t v) {
  return fetch_add(&A.vticket[v], 1);
}
__device__ __forceinline__ void settle_ticket(const ArrRef& A, uint32_t v, uint64_t k, uint64_t tpv) {
  if ((k & 0xFFFFFFFFull) == tpv - 1) st_rlx(&A.vticket[v], ((k >> 32) + 1) << 32);
}

// Logical-thread range of tile t of LFVector v.
__device__ __forceinline__ void tile_range(const TileArgs& I, uint32_t v, uint64_t t, uint64_t tile_len,
                                           uint64_t& g0, uint64_t& gend) {
  const uint64_t c0 = (uint64_t)v * I.chunk;
  g0 = c0 + t * tile_len;
  gend = c0 + I.chunk < I.n_threads ? c0 + I.chunk : I.n_threads;
}

// ------------------------------------------------------ 0/1 producer kernel --
// One wavefront handles one tile of 4096 logical threads: slot j of lane l is
// logical thread g0 + 64 j + l, so every producer load is coalesced and the
// order (slot, lane) is the logical-thread order.  A first pass keeps only the
// insert flags, one bit per slot in a 64-bit mask, and counts them.  Once the
// tile's first index is known, a second pass re-derives every kept candidate's
// position from the slot ballots (running total + mbcnt) and stores the value,
// which the producer computes or loads again: a slot's stores by the wave cover
// one contiguous range.  Holding a mask instead of the values keeps the wave to
// a few registers and no LDS, so a CU keeps 32 tiles in flight.
//
// Static tiles never wait on one another, nor does the only tile of an
// LFVector, so their position is the block index.  Otherwise the wave takes the
// next ticket of its LFVector, so every tile it may wait for is held by a wave
// that is already running.  Blocks are normally dispatched in index order, so
// the first pass runs for the position the index suggests while the ticket is
// in flight, and is redone in the rare case the ticket differs.
constexpr int kWaveSlots = (int)kInsertSlots;
constexpr int kWaveTile = 64 * kWaveSlots;
constexpr int kMaskWords = kWaveSlots / 64;
static_assert(kWaveSlots % 64 == 0 && kMaskWords >= 1, "whole 64-bit slot masks");

struct SlotMask {  // bit j: slot j of this lane inserts
  uint64_t w[kMaskWords];
  __device__ __forceinline__ bool get(int j) const { return (w[j >> 6] >> (j & 63)) & 1u; }
  __device__ __forceinline__ uint32_t count() const {
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kMaskWords; ++k) c += (uint32_t)__popcll(w[k]);
    return c;
  }
};

// Flags read from memory: every lane reads the flag of every slot, at the last
// thread of the tile for slots past its end, and masks afterwards.  A flag read
// under a divergent branch costs a full memory round trip per slot (the
// compiler waits for each such load before the branch joins), while
// unconditional loads, 16 of them gathered before any result is used, are
// issued back to back (buffer-mode Bernoulli rounds: 1.76 -> 3.30 TB/s).
// Computed flags keep the plain loop (batching them only adds registers).
template <class Prod>
__device__ __forceinline__ SlotMask wave_flags(const Prod& prod, uint64_t g0, uint64_t gend) {
  const uint32_t lane = lane_id();
  SlotMask m;
#pragma unroll
  for (int k = 0; k < kMaskWords; ++k) m.w[k] = 0;
  if constexpr (!Prod::kLoads) {  // computed flags: no loads to batch
#pragma unroll 16
    for (int j = 0; j < kWaveSlots; ++j) {
      const uint64_t g = g0 + (uint64_t)j * 64 + lane;
      if (g < gend && prod.flag(g)) m.w[j >> 6] |= 1ull << (j & 63);
    }
    return m;
  }
  if (g0 >= gend) return m;
  const uint64_t last = gend - 1;
#pragma unroll 1
  for (int j0 = 0; j0 < kWaveSlots; j0 += 16) {  // 16 flags in flight before the first is used
    bool f[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint64_t g = g0 + (uint64_t)(j0 + k) * 64 + lane;
      f[k] = prod.flag(g < gend ? g : last);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int j = j0 + k;
      if (f[k] && g0 + (uint64_t)j * 64 + lane < gend) m.w[j >> 6] |= 1ull << (j & 63);
    }
  }
  return m;
}

// Computed 0/1 producers (take(): flag and payload from one hash): every slot's
// payload is kept in registers from the flag pass, so the store pass does not
// hash again (a hash under the flag branch costs the whole wave its issue slots
// whatever the flags; configuration-2 sparse rounds: 159 -> 193 Gelem/s, at 110
// VGPRs for 4-byte elements).
template <typename T, class Prod>
__device__ __forceinline__ SlotMask wave_take(const Prod& prod, uint64_t g0, uint64_t gend, T (&vals)[kWaveSlots]) {
  const uint32_t lane = lane_id();
  SlotMask m;
#pragma unroll
  for (int k = 0; k < kMaskWords; ++k) m.w[k] = 0;
#pragma unroll
  for (int j = 0; j < kWaveSlots; ++j) {
    const uint64_t g = g0 + (uint64_t)j * 64 + lane;
    T v = 0;
    const bool f = g < gend && prod.take(g, v);
    vals[j] = v;
    if (f) m.w[j >> 6] |= 1ull << (j & 63);
  }
  return m;
}

// The payloads of slots [j0, j0 + kValBatch) of this lane, loaded before any of
// them is stored (a store may alias the payload buffer, so the compiler cannot
// move later loads above it); slots past the tile read its last thread.
constexpr int kValBatch = 16;
static_assert(kWaveSlots % kValBatch == 0, "whole payload batches");
template <typename T, class Prod>
__device__ __forceinline__ void wave_values(const Prod& prod, uint64_t g0, uint64_t gend, int j0,
                                            T (&v)[kValBatch]) {
  const uint32_t lane = lane_id();
  const uint64_t last = gend - 1;
#pragma unroll
  for (int k = 0; k < kValBatch; ++k) {
    const uint64_t g = g0 + (uint64_t)(j0 + k) * 64 + lane;
    v[k] = prod.value(g < gend ? g : last);
  }
}

// Every thread of the tile inserts and the tile lies in one bucket: element i is
// thread g0 + i at dst + i.  The wave writes the run with 16-byte non-temporal
// stores, a quarter of the store instructions of one element per lane and slot,
// starting on a 128-byte boundary (element stores for the ragged head and tail),
// so that each store instruction of the wave covers whole 128-byte lines: with
// 16-byte alignment only, every instruction left two partial lines for its
// neighbour to complete (about 6% more HBM writes, measured).
template <typename T, class Prod>
__device__ __forceinline__ void dense_store(T* dst, const Prod& prod, uint64_t g0, uint32_t n) {
  constexpr uint32_t VPL = 16 / sizeof(T);
  const uint32_t lane = lane_id();
  constexpr uint32_t kLine = 128 / sizeof(T);
  const uint32_t mis = (uint32_t)((reinterpret_cast<uintptr_t>(dst) & 127u) / sizeof(T));
  uint32_t head = mis ? kLine - mis : 0u;
  if (head > n) head = n;
  const gptr<T> d = gmem(dst);
  if (lane < head) d[lane] = prod.value(g0 + lane);
  const uint32_t nv = (n - head) / VPL;
  if constexpr (Prod::kDense) {  // generated payloads: no loads in the loop
    for (uint32_t q = lane; q < nv; q += 64) {
      const uint32_t e = head + q * VPL;
      T tmp[VPL];
#pragma unroll
      for (uint32_t k = 0; k < VPL; ++k) tmp[k] = prod.value(g0 + e + k);
      u32x4 x;
      __builtin_memcpy(&x, tmp, 16);
      store_nt_sc1(reinterpret_cast<gptr<u32x4>>(d + e), x);
    }
  } else {
    // Payloads from memory: kU vectors per lane are loaded (clamped to the last
    // one) before any is stored, since a store may alias the payload buffer.
    constexpr uint32_t kU = 4;
    for (uint32_t q0 = 0; q0 < nv; q0 += 64 * kU) {
      u32x4 x[kU];
#pragma unroll
      for (uint32_t u = 0; u < kU; ++u) {
        const uint32_t q = q0 + u * 64 + lane;
        const uint32_t e = head + (q < nv ? q : nv - 1) * VPL;
        T tmp[VPL];
#pragma unroll
        for (uint32_t k = 0; k < VPL; ++k) tmp[k] = prod.value(g0 + e + k);
        __builtin_memcpy(&x[u], tmp, 16);
      }
#pragma unroll
      for (uint32_t u = 0; u < kU; ++u) {
        const uint32_t q = q0 + u * 64 + lane;
        if (q < nv) __builtin_nontemporal_store(x[u], reinterpret_cast<gptr<u32x4>>(d + head + q * VPL));
      }
    }
  }
  const uint32_t tail = head + nv * VPL + lane;
  if (tail < n) d[tail] = prod.value(g0 + tail);
}

// One wave, one tile; `block` is the wave's index among the launch's waves for
// this array (the block index, or its offset inside a batch launch).
template <typename T, class Prod, bool kStatic>
__device__ __forceinline__ void wave_tile(const ArrRef& A, const StaticRef& S, const TileArgs& I,
                                          const Prod& prod, uint64_t block) {
  const uint32_t lane = lane_id();
  const bool ticketed = !kStatic && I.tpv > 1;
  const uint32_t v = kStatic ? 0u : (uint32_t)(block / I.tpv);
  uint64_t t = kStatic ? block : block - (uint64_t)v * I.tpv;
  uint64_t k = 0, size0 = 0;
  if (ticketed && lane == 0) k = take_ticket(A, v);
  if (!kStatic && lane == 0) size0 = ld_rlx(&A.size[v]);  // needed if this is tile 0
  uint64_t g0, gend;
  if (kStatic) {
    g0 = t * kWaveTile;
    gend = I.n_threads;
  } else {
    tile_range(I, v, t, kWaveTile, g0, gend);
  }
  // The static array's rounds are bound by the atomic on its size, not by
  // hashing: they keep the smaller register footprint.
  constexpr bool kKeep = !Prod::kLoads && !Prod::kDense && !kStatic;
  T kept[kKeep ? kWaveSlots : 1];
  SlotMask bits;
  if constexpr (kKeep) bits = wave_take<T, Prod>(prod, g0, gend, kept);
  else bits = wave_flags<Prod>(prod, g0, gend);
  uint64_t epoch = 0;
  if (ticketed) {
    if (lane == 0) settle_ticket(A, v, k, I.tpv);
    k = __shfl(k, 0, 64);
    epoch = k >> 32;
    k &= 0xFFFFFFFFull;
    if (k != t) {  // dispatched out of order: redo the first pass for the ticket
      t = k;
      tile_range(I, v, t, kWaveTile, g0, gend);
      if constexpr (kKeep) bits = wave_take<T, Prod>(prod, g0, gend, kept);
      else bits = wave_flags<Prod>(prod, g0, gend);
    }
  }
  if (g0 >= gend) return;
  if (!kStatic && ld_rlx32(&A.dead[v])) return;
  const bool is_last = g0 + kWaveTile >= gend;
  const uint32_t n_t = (uint32_t)wave_sum64((uint64_t)bits.count());

  T* dst;
  uint64_t lim = n_t;
  const uint32_t log2F = A.log2F;
  WaveRes r{0, kFailedPtr, 0, 0, 0};
  if (kStatic) {
    uint64_t base = 0;
    if (lane == 0 && n_t) base = fetch_add(S.size, n_t);
    base = __shfl(base, 0, 64);
    lim = base < S.cap ? (S.cap - base < n_t ? S.cap - base : n_t) : 0;
    if (lane == 0 && lim < n_t) set_error(S.err, kErrRange);
    dst = reinterpret_cast<T*>(S.data) + base;
  } else {
    r = resolve_wave(A, I, v, t, (uint64_t)v * I.tpv + t, is_last, n_t, __shfl(size0, 0, 64), epoch);
    if (r.n_out == 0) return;
    const uint64_t p0 = __shfl(r.bp, 0, 64);
    dst = reinterpret_cast<T*>(p0) + (r.base - bucket_start(log2F, r.b_lo));
    if (r.nb == 1 && p0 <= kFailedPtr) return;
  }
  uint32_t run = 0;
  if ((kStatic || r.nb == 1) && n_t == gend - g0 && lim == n_t) {
    dense_store<T, Prod>(dst, prod, g0, n_t);
    return;
  }
  if constexpr (kKeep) {
    if (r.nb == 1) {
#pragma unroll
      for (int j = 0; j < kWaveSlots; ++j) {
        const bool f = bits.get(j);
        const uint64_t m = __ballot(f);
        const uint32_t q = run + mbcnt(m);
        if (f && q < lim) gmem(dst)[q] = kept[j];
        run += (uint32_t)__popcll(m);
      }
      return;
    }
#pragma unroll
    for (int j = 0; j < kWaveSlots; ++j) {
      const bool f = bits.get(j);
      const uint64_t m = __ballot(f);
      const uint64_t idx = r.base + run + mbcnt(m);
      const uint32_t b = f ? bucket_of(log2F, idx) : r.b_lo;
      const uint64_t p = __shfl(r.bp, (int)(b - r.b_lo), 64);
      if (f && p > kFailedPtr) gmem(reinterpret_cast<T*>(p))[offset_in(log2F, idx, b)] = kept[j];
      run += (uint32_t)__popcll(m);
    }
    return;
  }
  if ((kStatic || r.nb == 1) && !Prod::kLoads) {
#pragma unroll 16
    for (int j = 0; j < kWaveSlots; ++j) {
      const bool f = bits.get(j);
      const uint64_t m = __ballot(f);
      const uint32_t q = run + mbcnt(m);
      if (f && q < lim) gmem(dst)[q] = prod.value(g0 + (uint64_t)j * 64 + lane);
      run += (uint32_t)__popcll(m);
    }
    return;
  }
  if (kStatic || r.nb == 1) {
#pragma unroll 1  // one batch of payloads in registers at a time
    for (int j0 = 0; j0 < kWaveSlots; j0 += kValBatch) {
      T v[kValBatch];
      wave_values<T, Prod>(prod, g0, gend, j0, v);
#pragma unroll
      for (int k = 0; k < kValBatch; ++k) {
        const bool f = bits.get(j0 + k);
        const uint64_t m = __ballot(f);
        const uint32_t q = run + mbcnt(m);
        if (f && q < lim) gmem(dst)[q] = v[k];
        run += (uint32_t)__popcll(m);
      }
    }
    return;
  }
  // The tile spans several buckets: locate each element by the closed form.
  if constexpr (!Prod::kLoads) {
    for (int j = 0; j < kWaveSlots; ++j) {
      const bool f = bits.get(j);
      const uint64_t m = __ballot(f);
      const uint64_t idx = r.base + run + mbcnt(m);
      const uint32_t b = f ? bucket_of(log2F, idx) : r.b_lo;
      const uint64_t p = __shfl(r.bp, (int)(b - r.b_lo), 64);
      if (f && p > kFailedPtr)
        gmem(reinterpret_cast<T*>(p))[offset_in(log2F, idx, b)] = prod.value(g0 + (uint64_t)j * 64 + lane);
      run += (uint32_t)__popcll(m);
    }
    return;
  }
  for (int j0 = 0; j0 < kWaveSlots; j0 += kValBatch) {
    T v[kValBatch];
    wave_values<T, Prod>(prod, g0, gend, j0, v);
#pragma unroll
    for (int k = 0; k < kValBatch; ++k) {
      const bool f = bits.get(j0 + k);
      const uint64_t m = __ballot(f);
      const uint64_t idx = r.base + run + mbcnt(m);
      const uint32_t b = f ? bucket_of(log2F, idx) : r.b_lo;
      const uint64_t p = __shfl(r.bp, (int)(b - r.b_lo), 64);
      if (f && p > kFailedPtr) gmem(reinterpret_cast<T*>(p))[offset_in(log2F, idx, b)] = v[k];
      run += (uint32_t)__popcll(m);
    }
  }
}

template <typename T, class Prod, bool kStatic>
__global__ __launch_bounds__(64) void insert_wave_kernel(ArrRef A, StaticRef S, TileArgs I, Prod prod) {
  wave_tile<T, Prod, kStatic>(A, S, I, prod, blockIdx.x);
}

// Batch launch: one insertion round of many arrays.  The waves of array i are
// the blocks [begins[i], begins[i+1]); each wave finds its array with a 64-way
// search and then runs exactly as in a single-array launch.
template <typename T, class Prod>
__device__ __forceinline__ void batch_wave(const BatchArr* items, const uint64_t* begins, uint32_t n,
                                           const Prod& prod, uint64_t blk) {
  const uint32_t i = wave_search(begins, n, blk);
  const BatchArr it = items[i];
  TileArgs I;
  I.n_threads = it.n_threads;
  I.chunk = it.chunk;
  I.tpv = it.tpv;
  I.elem_log2 = it.elem_log2;
  Prod p = prod;
  p.bind(it);
  wave_tile<T, Prod, false>(it.A, StaticRef{}, I, p, blk - begins[i]);
}

template <typename T, class Prod>
__global__ __launch_bounds__(64) void batch_insert_kernel(const BatchArr* items, const uint64_t* begins,
                                                          uint32_t n, Prod prod) {
  batch_wave<T, Prod>(items, begins, n, prod, blockIdx.x);
}

// Front half of a served step in one launch: waves [0, blocks) run the step's
// append rounds exactly as batch_insert_kernel; the next waves, one per array,
// scan the sizes of the arrays that the step's r/w and flatten requests read.
template <typename T>
__global__ __launch_bounds__(64) void serve_front_kernel(const BatchArr* items, const uint64_t* begins, uint32_t n_a,
                                                         uint64_t blocks, const ServeItem* sitems, uint32_t te_log2,
                                                         ProdKeyed<T> prod) {
  const uint64_t blk = blockIdx.x;
  if (blk >= blocks) {
    scan_array_wave(sitems[blk - blocks].A, te_log2);
    return;
  }
  batch_wave<T, ProdKeyed<T>>(items, begins, n_a, prod, blk);
}

// ------------------------------------------ dense rounds: grow, then store --
// When every logical thread of a round inserts exactly one element, LFVector v
// receives exactly the threads of its chunk, so its growth is known before any
// element is produced.  Such a round runs as the two phases the paper times
// separately (Table II: grow, then insert): grow_kernel allocates every bucket
// the round reaches (one wave per LFVector, one lane per bucket) and moves the
// size, keeping the old one in rbase; dense_insert_kernel then has one wave per
// tile store its elements from rbase[v] + t * kInsertTile on.  No tile waits on
// another and no atomic is taken outside the pool.  An LFVector whose growth
// fails is frozen with its size unchanged (its round is dropped), as in the
// single-kernel path.
// LFVector v grows by cnt elements (one wave): every bucket the new elements
// reach is allocated, the size moves and the old one is kept in rbase[v].
__device__ __forceinline__ void grow_vector_by(const ArrRef& A, uint32_t elem_log2, uint32_t v, uint64_t cnt) {
  const uint32_t lane = lane_id();
  if (cnt == 0 || A.dead[v]) return;
  const uint64_t s0 = A.size[v];
  const uint32_t lo = nbuckets_for(A.log2F, s0), hi = nbuckets_for(A.log2F, s0 + cnt);
  const uint32_t b = lo + lane;
  bool failed = false;
  if (b < hi) {
    if (b >= (uint32_t)kMaxBuckets) {
      failed = true;
    } else {
      uint8_t* q = pool_alloc(A.pool, bucket_class(A.log2F, elem_log2, b), pool_shard(v, b, A.salt));
      A.bptr[(uint64_t)v * kMaxBuckets + b] = q ? (uint64_t)q : kFailedPtr;
      failed = !q;
    }
  }
  if (__ballot(failed)) {
    if (lane == 0) {
      set_error(A.err, kErrNoMem);
      A.dead[v] = 1u;
    }
  } else if (lane == 0) {
    A.rbase[v] = s0;
    A.size[v] = s0 + cnt;
  }
}

__device__ __forceinline__ void grow_vector(const ArrRef& A, const TileArgs& I, uint32_t v) {
  const uint64_t c0 = (uint64_t)v * I.chunk;
  const uint64_t cnt = c0 < I.n_threads ? (I.n_threads - c0 < I.chunk ? I.n_threads - c0 : I.chunk) : 0;
  grow_vector_by(A, I.elem_log2, v, cnt);
}

template <typename T, class Prod>
__device__ __forceinline__ void store_tile(const ArrRef& A, const TileArgs& I, const Prod& prod, uint64_t block) {
  const uint32_t v = (uint32_t)(block / I.tpv);
  const uint64_t t = block - (uint64_t)v * I.tpv;
  uint64_t g0, gend;
  tile_range(I, v, t, kWaveTile, g0, gend);
  if (g0 >= gend || A.dead[v]) return;
  const uint32_t n = gend - g0 < (uint64_t)kWaveTile ? (uint32_t)(gend - g0) : (uint32_t)kWaveTile;
  const uint32_t log2F = A.log2F;
  const uint64_t base = A.rbase[v] + t * (uint64_t)kWaveTile;
  for (uint32_t i = 0; i < n;) {  // one run per bucket the tile reaches
    const uint64_t idx = base + i;
    const uint32_t b = bucket_of(log2F, idx);
    const uint64_t bs = bucket_start(log2F, b);
    const uint64_t room = bs + bucket_len(log2F, b) - idx;
    const uint32_t run = (uint64_t)(n - i) < room ? n - i : (uint32_t)room;
    T* dst = reinterpret_cast<T*>(A.bptr[(uint64_t)v * kMaxBuckets + b]) + (idx - bs);
    dense_store<T, Prod>(dst, prod, g0 + i, run);
    i += run;
  }
}

// One wave per LFVector grows it and then stores its elements, in one launch.
// Used when that still fills the GPU: rounds of up to 8 tiles per LFVector, or
// arrays of 512 or more LFVectors (on configuration 2, 512 waves writing up to
// 1 MiB each reach 4.8 TB/s, against 4.5 for a grow launch plus a store launch
// of one wave per tile).  Fewer, longer LFVectors take the two-launch form.  The
// new bucket pointers stay in the lanes that allocated them; a bucket that
// existed before the round is read from the table, written by an earlier launch.
// LFVector v appends the elements the producer gives for g = c0 .. c0 + cnt - 1.
// With a fused shrink (I.sh_den != 0) the wave then leaves the size the shrink
// would leave and releases the buckets past it, exactly as a shrink launch after
// the round would (an LFVector that fails to grow is frozen, then still shrunk).
template <typename T, class Prod>
__device__ __forceinline__ void grow_store_range(const ArrRef& A, const TileArgs& I, const Prod& prod, uint32_t v,
                                                 uint64_t c0, uint64_t cnt) {
  const uint32_t lane = lane_id();
  if (cnt == 0 || A.dead[v]) {
    if (I.sh_den) shrink_vector(A, v, I.sh_num, I.sh_den, I.elem_log2);
    return;
  }
  const uint32_t log2F = A.log2F;
  const uint64_t s0 = A.size[v];
  const uint32_t lo = nbuckets_for(log2F, s0), hi = nbuckets_for(log2F, s0 + cnt);
  // With a fused shrink, the buckets from `keep` on go back to the pool at the end
  // of this launch; those the round itself reaches are allocated and released
  // with nothing stored in them (pool_alloc_release: counted, not moved).
  const uint64_t fin = I.sh_den ? shrink_keep(s0 + cnt, I.sh_num, I.sh_den) : s0 + cnt;
  const uint32_t keep = nbuckets_for(log2F, fin);
  const uint32_t b = lo + lane;
  uint64_t q = 0;
  bool failed = false;
  if (b < hi) {
    if (b >= (uint32_t)kMaxBuckets) {
      failed = true;
    } else {
      // After a clear in the same launch (I.reuse) a bucket may still be in the
      // table: the round takes it again, counted as the release the clear would
      // have made and the allocation the round makes (pool_reuse); one the round
      // reaches and its shrink releases goes back to the pool now.
      uint64_t* slot = A.bptr + (uint64_t)v * kMaxBuckets + b;
      const uint64_t kept = I.reuse ? *slot : 0;
      const uint32_t cls = bucket_class(log2F, I.elem_log2, b);
      if (I.sh_den && b >= keep) {
        if (kept) {
          pool_free(A.pool, reinterpret_cast<uint8_t*>(kept), cls, pool_shard(v, b, A.salt));
          *slot = 0;
        }
        failed = !pool_alloc_release(A.pool, cls, pool_shard(v, b, A.salt));
      } else if (kept) {
        q = kept;
        failed = !pool_reuse(A.pool, pool_shard(v, b, A.salt));
      } else {
        uint8_t* p = pool_alloc(A.pool, cls, pool_shard(v, b, A.salt));
        q = p ? (uint64_t)p : kFailedPtr;
        *slot = q;
        failed = !p;
      }
    }
  }
  // Bucket `lane`'s pointer when this round allocated it (lane lo + k holds bucket lo + k).
  const uint64_t mine = I.sh_den ? __shfl(q, (int)((lane - lo) & 63u), 64) : 0;
  const bool held = lane >= lo && lane < hi;
  if (__ballot(failed)) {
    if (lane == 0) {
      set_error(A.err, kErrNoMem);
      A.dead[v] = 1u;
    }
    if (I.sh_den) {  // the shrink of an LFVector that has just failed: it keeps shrink_keep(s0) and no bucket
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the slot stores above land before they are cleared
      release_bucket(A, v, lane, nbuckets_for(log2F, shrink_keep(s0, I.sh_num, I.sh_den)), kMaxBuckets, held, mine,
                     I.elem_log2);
      if (lane == 0) A.size[v] = shrink_keep(s0, I.sh_num, I.sh_den);
    }
    return;
  }
  if (lane == 0) A.size[v] = fin;
  // With a fused shrink, elements that would land in a bucket the shrink releases
  // are popped anyway: they are not stored, so no store of this wave can still be
  // in flight to a bucket when it goes back to the pool (whose link word the
  // release writes), and the release needs no fence.
  uint64_t upto = s0 + cnt;
  if (I.sh_den && bucket_start(log2F, keep) < upto) upto = bucket_start(log2F, keep) > s0 ? bucket_start(log2F, keep) : s0;
  const uint32_t n = (uint32_t)(upto - s0);
  for (uint32_t i = 0; i < n;) {
    const uint64_t idx = s0 + i;
    const uint32_t bk = bucket_of(log2F, idx);
    const uint64_t bs = bucket_start(log2F, bk);
    const uint64_t room = bs + bucket_len(log2F, bk) - idx;
    const uint32_t run = (uint64_t)(n - i) < room ? n - i : (uint32_t)room;
    const uint64_t p = bk >= lo ? __shfl(q, (int)(bk - lo), 64) : A.bptr[(uint64_t)v * kMaxBuckets + bk];
    dense_store<T, Prod>(reinterpret_cast<T*>(p) + (idx - bs), prod, c0 + i, run);
    i += run;
  }
  if (I.sh_den && keep < hi)  // the fused shrink: release the buckets past the kept elements
    release_bucket(A, v, lane, keep, hi, held, mine, I.elem_log2);
}

// The round's share of LFVector v: logical threads [v chunk, v chunk + chunk).
template <typename T, class Prod>
__device__ __forceinline__ void grow_store_vector(const ArrRef& A, const TileArgs& I, const Prod& prod, uint32_t v) {
  const uint64_t c0 = (uint64_t)v * I.chunk;
  const uint64_t cnt = c0 < I.n_threads ? (I.n_threads - c0 < I.chunk ? I.n_threads - c0 : I.chunk) : 0;
  grow_store_range<T, Prod>(A, I, prod, v, c0, cnt);
}

template <typename T, class Prod>
__global__ __launch_bounds__(256) void grow_store_kernel(ArrRef A, TileArgs I, Prod prod) {
  const uint32_t v = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (v < A.V) grow_store_vector<T, Prod>(A, I, prod, v);
}

// Several rounds of generated payloads, each followed by the same shrink, in one
// launch.  LFVectors never wait on one another, so the wave of LFVector v takes
// it through every round in order, each as grow_store_range does one (grow,
// store, shrink); a round's share of v is threads [v chunk_r, (v + 1) chunk_r)
// as in its own launch.  Between rounds the wave fences, so that its loads of
// the size, the frozen flag and the bucket table see what its own lanes stored
// the round before.  Workgroup scope is enough: every lane of the wave runs on
// one CU and reads through that CU's cache, which holds the wave's own stores
// once they are complete; a device-scope fence would also write back the XCD's
// L2 each round (configuration 2's twelve rounds: 337 us with it, 225 us with
// the workgroup fence, 309-317 us as twelve launches).
//
// With I.reuse the launch starts with a clear (every LFVector emptied, as a
// shrink of 1/1): a live LFVector only sets its size to 0 and keeps its buckets
// in the table for the rounds to take again (grow_store_range), and the ones no round
// took go back to the pool at the end; a frozen LFVector releases them at once,
// as the clear does.  Sizes, contents, capacity and pool counts are those of the
// clear and the rounds as calls of their own.
template <typename T, class Prod>
__global__ __launch_bounds__(256) void grow_store_rounds_kernel(ArrRef A, TileArgs I, Prod prod, RoundList R) {
  const uint32_t v = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (v >= A.V) return;
  const uint32_t lane = lane_id();
  if (I.reuse) {
    if (A.dead[v])
      shrink_vector(A, v, 1, 1, I.elem_log2);
    else if (lane == 0)
      A.size[v] = 0;
  }
#pragma unroll 1
  for (uint32_t r = 0; r < R.n; ++r) {
    if (r || I.reuse) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    I.n_threads = R.n_threads[r];
    I.chunk = (I.n_threads + A.V - 1) / A.V;
    prod.round = R.round[r];
    grow_store_vector<T, Prod>(A, I, prod, v);
  }
  if (I.reuse) {  // buckets kept through the clear that no round took
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    const uint64_t s = A.size[v];
    release_bucket(A, v, lane, nbuckets_for(A.log2F, s), kMaxBuckets, false, 0, I.elem_log2);
  }
}

// Segment append: LFVector v appends values[prefix[v] .. prefix[v + 1]).  A
// decreasing pair, a segment past n_values or one of 2^32 elements or more sets
// GGA_ERANGE and leaves the LFVector unchanged.
template <typename T>
__global__ __launch_bounds__(256) void segments_kernel(ArrRef A, TileArgs I, const T* values, const uint64_t* prefix,
                                                       uint64_t n_values) {
  const uint32_t v = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (v >= A.V) return;
  const uint64_t lo = prefix[v], hi = prefix[v + 1];
  if (hi < lo || hi > n_values || hi - lo >= (1ull << 32)) {
    if (lane_id() == 0) set_error(A.err, kErrRange);
    return;
  }
  grow_store_range<T, ProdBuffer<T>>(A, I, ProdBuffer<T>{values, nullptr}, v, lo, hi - lo);
}

__global__ __launch_bounds__(256) void grow_kernel(ArrRef A, TileArgs I) {
  const uint32_t v = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (v < A.V) grow_vector(A, I, v);
}

template <typename T, class Prod>
__global__ __launch_bounds__(64) void dense_insert_kernel(ArrRef A, TileArgs I, Prod prod) {
  store_tile<T, Prod>(A, I, prod, blockIdx.x);
}

// The same two phases for one round of many arrays: wave w of the grow launch is
// LFVector w - vbegin[i] of array i, wave w of the store launch is tile
// w - begins[i] of array i.
__device__ __forceinline__ TileArgs item_args(const BatchArr& it) {
  TileArgs I;
  I.n_threads = it.n_threads;
  I.chunk = it.chunk;
  I.tpv = it.tpv;
  I.elem_log2 = it.elem_log2;
  return I;
}

__global__ __launch_bounds__(256) void batch_grow_kernel(const BatchArr* items, const uint64_t* vbegin, uint32_t n) {
  const uint64_t w = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
  if (w >= vbegin[n]) return;
  const uint32_t i = wave_search(vbegin, n, w);
  const BatchArr it = items[i];
  if (it.n_threads) grow_vector(it.A, item_args(it), (uint32_t)(w - vbegin[i]));
}

// The one-launch form for a round of many arrays: wave w is LFVector
// w - vbegin[i] of array i.
template <typename T, class Prod>
__global__ __launch_bounds__(256) void batch_grow_store_kernel(const BatchArr* items, const uint64_t* vbegin,
                                                               uint32_t n, Prod prod) {
  const uint64_t w = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
  if (w >= vbegin[n]) return;
  const uint32_t i = wave_search(vbegin, n, w);
  const BatchArr it = items[i];
  if (!it.n_threads) return;
  Prod p = prod;
  p.bind(it);
  grow_store_vector<T, Prod>(it.A, item_args(it), p, (uint32_t)(w - vbegin[i]));
}

template <typename T, class Prod>
__global__ __launch_bounds__(64) void batch_dense_kernel(const BatchArr* items, const uint64_t* begins, uint32_t n,
                                                         Prod prod) {
  const uint64_t blk = blockIdx.x;
  const uint32_t i = wave_search(begins, n, blk);
  const BatchArr it = items[i];
  Prod p = prod;
  p.bind(it);
  store_tile<T, Prod>(it.A, item_args(it), p, blk - begins[i]);
}

// --------------------------------------- static array, closed-form rounds --
// A round in which every thread inserts has its positions in closed form on the
// static array too: thread g of the round lands at size + g.  One wave per tile of
// 4096 threads stores its run exactly as the GGArray's dense rounds do (16-byte
// non-temporal stores on whole 128-byte lines), so the two layouts are compared
// on the same algorithm.  Every wave reads the size before the round (nothing
// changes it during the launch); the last workgroup to finish moves it.  Elements past
// the capacity are dropped with the sticky GGA_ERANGE, and the size counts them,
// as in the atomic rounds.
constexpr uint32_t kDenseWaves = 16;  // tiles (waves) per workgroup of the static closed-form round
template <typename T, class Prod>
__global__ __launch_bounds__(64 * kDenseWaves) void static_dense_kernel(StaticRef S, uint64_t n, uint64_t nblocks,
                                                                        Prod prod) {
  const uint32_t lane = lane_id();
  // The size before the round.  Nothing writes it until every workgroup has
  // counted itself done below, so a plain load is current (and served by the
  // cache after the first: every wave reading it with device scope, and one
  // counter atomic per wave, measured slower than the stores themselves).
  const uint64_t base = *S.size;
  const uint64_t g0 = ((uint64_t)blockIdx.x * kDenseWaves + (threadIdx.x >> 6)) * kWaveTile;
  if (g0 < n) {
    const uint32_t cnt = n - g0 < (uint64_t)kWaveTile ? (uint32_t)(n - g0) : (uint32_t)kWaveTile;
    const uint64_t pos = base + g0;
    const uint32_t lim = pos < S.cap ? (S.cap - pos < cnt ? (uint32_t)(S.cap - pos) : cnt) : 0u;
    if (lim) dense_store<T, Prod>(reinterpret_cast<T*>(S.data) + pos, prod, g0, lim);
    if (lane == 0 && lim < cnt) set_error(S.err, kErrRange);
  }
  // Every wave of the workgroup has its size (the stores needed it) before the
  // workgroup counts itself; the last workgroup moves the size.
  __syncthreads();
  if (threadIdx.x == 0 && fetch_add32(S.done, 1u) == nblocks - 1) {
    st_rlx(S.size, base + n);
    st_rlx32(S.done, 0u);
  }
}

// ------------------------------------ static array, one atomic per element --
// The other insertion strategy the paper compares (Sec. VI-A): every inserting
// thread takes its own slot with an atomic add on the size, so the order across
// threads is not fixed.  (The compiler may combine the atomics of a wavefront
// that target one address into one; that is the strategy as the hardware runs
// it.)
template <typename T, class Prod>
__global__ __launch_bounds__(256) void static_atomic_kernel(StaticRef S, uint64_t n, Prod prod) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  bool over = false;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += stride) {
    if (!prod.flag(g)) continue;
    const uint64_t pos = fetch_add(S.size, 1);
    if (pos < S.cap) gmem(reinterpret_cast<T*>(S.data))[pos] = prod.value(g);
    else over = true;
  }
  if (over) set_error(S.err, kErrRange);
}

// --------------------------------------------- multi-element producer kernel --
// Thread tid owns logical threads g0 + 4 tid .. g0 + 4 tid + 3 (blocked), so a
// plain scan of per-thread counts orders the elements.  Once the tile's first
// index is known, each thread writes, for each of its outputs, who produces it
// into an LDS owner map of 16-bit entries (tid << 6 | j << 4 | r: element r of
// logical thread 4 tid + j).  The outputs are then produced in output order by
// consecutive lanes (no divergence from uneven counts), a segment per bucket run:
// element stores up to the first 128-byte line of the run, then 16-byte
// non-temporal stores of VPL consecutive outputs per lane that cover whole lines
// across the wave (partial lines left by element-wise stores cost about 5% extra
// HBM writes, measured), then the ragged tail.  Bucket and offset are computed
// once per run, not per element.  The map covers 8192 outputs at a time.
template <typename Prod>
__device__ __forceinline__ uint32_t produce_counts(const Prod& prod, uint64_t gt, uint64_t gend,
                                                   uint32_t* cnt) {
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < kCountK; ++j) {
    cnt[j] = (gt + j < gend) ? prod.count(gt + j) : 0u;
    c += cnt[j];
  }
  return c;
}

// Outputs own[0 .. n) of a run, stored at dst (element-aligned).
template <typename T, class Prod>
__device__ __forceinline__ void store_owned_run(T* dst_, const uint16_t* own, uint32_t n, const Prod& prod,
                                                uint64_t g0) {
  constexpr uint32_t VPL = 16 / sizeof(T), kLine = 128 / sizeof(T);
  const uint32_t tid = threadIdx.x;
  const gptr<T> dst = gmem(dst_);
  const uint32_t mis = (uint32_t)((reinterpret_cast<uintptr_t>(dst_) & 127u) / sizeof(T));
  uint32_t head = mis ? kLine - mis : 0u;
  if (head > n) head = n;
  if (tid < head) {
    const uint32_t o = own[tid];
    __builtin_nontemporal_store(prod.value(g0 + (o >> 4), o & 15u), dst + tid);
  }
  const uint32_t nv = (n - head) / VPL;
  for (uint32_t q = tid; q < nv; q += kB) {
    const uint32_t e = head + q * VPL;
    T tmp[VPL];
#pragma unroll
    for (uint32_t k = 0; k < VPL; ++k) {
      const uint32_t o = own[e + k];
      tmp[k] = prod.value(g0 + (o >> 4), o & 15u);
    }
    u32x4 x;
    __builtin_memcpy(&x, tmp, 16);
    __builtin_nontemporal_store(x, reinterpret_cast<gptr<u32x4>>(dst + e));
  }
  const uint32_t tail = head + nv * VPL + tid;
  if (tail < n) {
    const uint32_t o = own[tail];
    __builtin_nontemporal_store(prod.value(g0 + (o >> 4), o & 15u), dst + tail);
  }
}

template <typename T, class Prod, bool kStatic>
__global__ __launch_bounds__(kB) void insert_count_kernel(ArrRef A, StaticRef S, TileArgs I,
                                                          Prod prod) {
  __shared__ uint16_t s_own[kOwnWindow];  // output -> (thread, logical thread, element)
  __shared__ TileShared sh;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const bool ticketed = !kStatic && I.tpv > 1;
  const uint32_t v = kStatic ? 0u : (uint32_t)(blockIdx.x / I.tpv);
  uint64_t t = kStatic ? blockIdx.x : blockIdx.x - (uint64_t)v * I.tpv;
  uint64_t k = 0;
  if (ticketed && tid == 0) k = take_ticket(A, v);
  uint64_t g0, gend;
  if (kStatic) {
    g0 = t * kCountTile;
    gend = I.n_threads;
  } else {
    tile_range(I, v, t, kCountTile, g0, gend);
  }
  uint32_t cnt[kCountK];
  uint64_t gt = g0 + (uint64_t)tid * kCountK;
  uint32_t c = produce_counts<Prod>(prod, gt, gend, cnt);
  if (ticketed && tid == 0) {
    sh.tile = k;
    settle_ticket(A, v, k, I.tpv);
  }
  __syncthreads();
  const uint64_t epoch = ticketed ? sh.tile >> 32 : 0;
  if (ticketed && (sh.tile & 0xFFFFFFFFull) != t) {  // dispatched out of order: produce for the ticket
    t = sh.tile & 0xFFFFFFFFull;
    tile_range(I, v, t, kCountTile, g0, gend);
    gt = g0 + (uint64_t)tid * kCountK;
    c = produce_counts<Prod>(prod, gt, gend, cnt);
  }
  if (g0 >= gend) return;
  const bool is_last = g0 + kCountTile >= gend;

  const uint32_t incl = wave_incl_scan(c);
  if (lane == 63) sh.cnt[w] = incl;
  // One read of the frozen flag for the whole block: another tile of this
  // LFVector may set it during this launch (a stalled look-back), and waves that
  // read it at different moments would disagree on whether the tile runs.
  if (!kStatic && tid == 0) sh.frozen = ld_rlx32(&A.dead[v]);
  __syncthreads();
  if (!kStatic && sh.frozen) return;  // block-uniform
  uint32_t before = 0, n_t = 0;
#pragma unroll
  for (int q = 0; q < kW; ++q) {
    const uint32_t x = sh.cnt[q];
    before += (q < (int)w) ? x : 0u;
    n_t += x;
  }
  const uint32_t excl = before + incl - c;
  if (kStatic) {
    resolve_static(S, n_t, sh);
  } else if (w == 0) {
    resolve_tile(A, I, v, t, (uint64_t)v * I.tpv + t, is_last, n_t, epoch, sh);
  }
  __syncthreads();
  const uint32_t n_out = kStatic ? (sh.writable < n_t ? sh.writable : n_t) : sh.n_tile;  // 0 if stalled
  const uint32_t log2F = A.log2F;
  const uint64_t base = sh.base;
  for (uint32_t w0 = 0; w0 < n_out; w0 += kOwnWindow) {
    const uint32_t w1 = n_out - w0 < kOwnWindow ? n_out : w0 + kOwnWindow;
    if (w0) __syncthreads();  // the previous window has been read
    // Each thread names itself as the producer of its outputs in this window.
    uint32_t e = excl - w0;  // wraps for outputs before the window, which fail the test
#pragma unroll
    for (uint32_t j = 0; j < (uint32_t)kCountK; ++j) {
      const uint32_t ent = (tid << 6) | (j << 4);
      for (uint32_t r = 0; r < cnt[j]; ++r, ++e)
        if (e < kOwnWindow) s_own[e] = (uint16_t)(ent | r);
    }
    __syncthreads();
    if (kStatic) {
      store_owned_run<T, Prod>(reinterpret_cast<T*>(S.data) + base + w0, s_own, w1 - w0, prod, g0);
      continue;
    }
    for (uint32_t i = w0; i < w1;) {  // one run per bucket the window's outputs reach
      const uint64_t idx = base + i;
      const uint32_t b = bucket_of(log2F, idx);
      const uint64_t bs = bucket_start(log2F, b);
      const uint64_t room = bs + bucket_len(log2F, b) - idx;
      const uint32_t run = (uint64_t)(w1 - i) < room ? w1 - i : (uint32_t)room;
      const uint64_t p = sh.bp[b - sh.b_lo];
      if (p > kFailedPtr) store_owned_run<T, Prod>(reinterpret_cast<T*>(p) + (idx - bs), s_own + (i - w0), run, prod, g0);
      i += run;
    }
  }
}

// ------------------------------------------- packed multi-element producer --
// Thread gid inserts counts[gid] elements taken in order from a packed buffer:
// its elements are values[P(gid) .. P(gid) + counts[gid]), P the exclusive prefix
// of the counts over all threads.  Tiles are those of the multi-element kernel
// (1024 logical threads, numbered LFVector by LFVector), so a tile's values are
// contiguous in the buffer and its outputs contiguous in its LFVector.  Two
// pre-passes give every tile the offset of its first value (an exclusive scan of
// the tile totals over the whole round: Sec. III-B's prefix sum, taken once for
// all tiles instead of per block), so each LFVector's growth is known before any
// element moves.  The round then runs as the dense rounds do: one wave per
// LFVector allocates the buckets and moves the size (packed_grow_kernel), then
// one workgroup per tile copies its contiguous range of values into at most a
// few bucket runs (packed_copy_kernel), with no waits, no look-back and no
// per-element arithmetic.

// The offset buffer of a packed round: words [0, ntiles) hold each tile's value
// offset within its group of kPackGroup consecutive tiles, words [ntiles,
// ntiles + ngroups] the exclusive prefix of the group totals (the last one is
// the round's total).
constexpr uint32_t kPackGroup = 16;
__host__ __device__ __forceinline__ uint64_t packed_groups(uint64_t ntiles) {
  return (ntiles + kPackGroup - 1) / kPackGroup;
}
__device__ __forceinline__ uint64_t packed_offset(const uint64_t* off, uint64_t ntiles, uint64_t t) {
  const uint64_t* gpre = off + ntiles;
  return t < ntiles ? gpre[t / kPackGroup] + off[t] : gpre[packed_groups(ntiles)];
}

// Count total of one tile (logical threads [g0, gend), at most 1024), by one wave.
__device__ __forceinline__ uint32_t wave_count_sum(const uint8_t* counts, uint64_t g0, uint64_t gend) {
  const uint32_t lane = lane_id();
  uint32_t c = 0;
  if (gend - g0 == (uint64_t)kCountTile && (g0 & 15u) == 0) {  // whole aligned tile: 16 bytes per lane
    const u32x4 x = *reinterpret_cast<gptr<const u32x4>>(gmem(counts + g0 + 16u * lane));
    c = __builtin_amdgcn_sad_u8(x[0], 0u, c);  // sum of the four bytes
    c = __builtin_amdgcn_sad_u8(x[1], 0u, c);
    c = __builtin_amdgcn_sad_u8(x[2], 0u, c);
    c = __builtin_amdgcn_sad_u8(x[3], 0u, c);
  } else {
#pragma unroll
    for (uint32_t k = 0; k < (uint32_t)kCountTile / 64; ++k) {
      const uint64_t g = g0 + 64u * k + lane;
      if (g < gend) c += counts[g];
    }
  }
  return (uint32_t)wave_sum64(c);
}

// Pre-pass 1: one workgroup per group of kPackGroup tiles, one wave per tile at a
// time: tile totals, their exclusive prefix within the group (written to
// off[tile]) and the group total (written to the group's prefix slot, which the
// scan then turns into the prefix).
__global__ __launch_bounds__(kB) void packed_group_kernel(TileArgs I, const uint8_t* counts, uint64_t* off,
                                                          uint64_t ntiles) {
  __shared__ uint32_t s_sum[kPackGroup];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint64_t first = (uint64_t)blockIdx.x * kPackGroup;
  for (uint32_t j = w; j < kPackGroup; j += kW) {
    const uint64_t tile = first + j;
    uint32_t c = 0;
    if (tile < ntiles) {
      const uint32_t v = (uint32_t)(tile / I.tpv);
      uint64_t g0, gend;
      tile_range(I, v, tile - (uint64_t)v * I.tpv, kCountTile, g0, gend);
      if (g0 < gend) c = wave_count_sum(counts, g0, gend);
    }
    if (lane == 0) s_sum[j] = c;
  }
  __syncthreads();
  if (tid < kPackGroup) {
    uint64_t before = 0, all = 0;
    for (uint32_t q = 0; q < kPackGroup; ++q) {
      before += q < tid ? s_sum[q] : 0u;
      all += s_sum[q];
    }
    if (first + tid < ntiles) off[first + tid] = before;
    if (tid == 0) off[ntiles + blockIdx.x] = all;
  }
}

// Pre-pass 2: exclusive prefix of the group totals in place (one workgroup of
// 1024 threads, 8 consecutive groups per thread and pass); entry ntiles gets the
// total.
__global__ __launch_bounds__(1024) void packed_tile_scan_kernel(uint64_t* tile_off, uint64_t ntiles) {
  __shared__ uint64_t wtot[16];
  __shared__ uint64_t carry_s;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  uint64_t carry = 0;
  for (uint64_t base = 0; base < ntiles; base += 8192) {
    uint64_t x[8], sum = 0;
    const uint64_t i0 = base + (uint64_t)tid * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      x[k] = i0 + k < ntiles ? tile_off[i0 + k] : 0;
      sum += x[k];
    }
    const uint64_t incl = wave_incl_scan64(sum);
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    uint64_t before = carry, all = carry;
    for (uint32_t q = 0; q < 16; ++q) {
      before += q < w ? wtot[q] : 0;
      all += wtot[q];
    }
    uint64_t run = before + incl - sum;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (i0 + k < ntiles) tile_off[i0 + k] = run;
      run += x[k];
    }
    carry = all;
    __syncthreads();  // wtot is reused by the next pass
  }
  if (tid == 0) carry_s = carry;
  __syncthreads();
  if (tid == 0) tile_off[ntiles] = carry_s;
}

// Phase 1: LFVector v grows by the values of its tiles v tpv .. (v + 1) tpv - 1
// (one wave per LFVector).  Counts asking for more values than given insert
// nothing.
__global__ __launch_bounds__(256) void packed_grow_kernel(ArrRef A, TileArgs I, const uint64_t* off,
                                                          uint64_t ntiles, uint64_t n_values) {
  const uint32_t v = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (packed_offset(off, ntiles, ntiles) > n_values) {
    if (v == 0 && lane_id() == 0) set_error(A.err, kErrRange);
    return;
  }
  if (v >= A.V) return;
  const uint64_t t0 = (uint64_t)v * I.tpv;
  grow_vector_by(A, I.elem_log2, v, packed_offset(off, ntiles, t0 + I.tpv) - packed_offset(off, ntiles, t0));
}

// One run of a packed round: n elements from src to a bucket, from its element
// e0 on, copied by threads tid = 0 .. nthr - 1 of the workgroup.  Buckets are
// 256-byte aligned, so the split into a head up to the destination's first
// 128-byte line, whole-line 16-byte stores and a tail is known before the
// bucket's pointer: load() issues the first pass (up to kU vectors per thread,
// the head and tail elements) and store(bucket) writes it and copies the rest.
// The loads are unconditional, their indices clamped into the run (surplus
// lanes read what another lane stores): a load under a divergent branch makes
// the compiler wait for it before the branch joins, which would serialise the
// pass.  Only the stores are predicated.
template <typename T>
struct RunCopy {
  typedef u32x4 u32x4_a4 __attribute__((aligned(4)));
  static constexpr uint32_t VPL = 16 / sizeof(T), kLine = 128 / sizeof(T), kU = 8;
  gptr<const T> src;
  uint64_t e0;
  uint32_t n, head, nv, tid, nthr;
  u32x4 x[kU];
  T hv, tv;

  __device__ __forceinline__ void load(const T* src_, uint64_t e0_, uint32_t n_, uint32_t tid_, uint32_t nthr_) {
    src = gmem(src_);
    e0 = e0_;
    n = n_;
    tid = tid_;
    nthr = nthr_;
    const uint32_t mis = (uint32_t)(e0 & (kLine - 1));
    head = mis ? kLine - mis : 0u;
    if (head > n) head = n;
    nv = (n - head) / VPL;
    if (nv == 0) return;  // a short run is copied element by element in store()
    const gptr<const u32x4_a4> vsrc = reinterpret_cast<gptr<const u32x4_a4>>(src + head);
#pragma unroll
    for (uint32_t k = 0; k < kU; ++k) {
      const uint32_t q = k * nthr + tid;
      x[k] = __builtin_nontemporal_load(vsrc + (q < nv ? q : nv - 1));
    }
    const uint32_t tail = head + nv * VPL + tid;
    hv = __builtin_nontemporal_load(src + (tid < head ? tid : 0u));
    tv = __builtin_nontemporal_load(src + (tail < n ? tail : n - 1));
  }

  __device__ __forceinline__ void store(T* bucket) const {
    const gptr<T> dst = gmem(bucket + e0);
    if (nv == 0) {
      for (uint32_t i = tid; i < n; i += nthr) __builtin_nontemporal_store(src[i], dst + i);
      return;
    }
#pragma unroll
    for (uint32_t k = 0; k < kU; ++k) {
      const uint32_t q = k * nthr + tid;
      if (q < nv) __builtin_nontemporal_store(x[k], reinterpret_cast<gptr<u32x4>>(dst + head + q * VPL));
    }
    const uint32_t tail = head + nv * VPL + tid;
    if (tid < head) __builtin_nontemporal_store(hv, dst + tid);
    if (tail < n) __builtin_nontemporal_store(tv, dst + tail);
    const gptr<const u32x4_a4> vsrc = reinterpret_cast<gptr<const u32x4_a4>>(src + head);
    u32x4 y[kU];
    for (uint32_t q0 = kU * nthr; q0 < nv; q0 += kU * nthr) {  // runs longer than one pass
#pragma unroll
      for (uint32_t k = 0; k < kU; ++k) {
        const uint32_t q = q0 + k * nthr + tid;
        y[k] = __builtin_nontemporal_load(vsrc + (q < nv ? q : nv - 1));
      }
#pragma unroll
      for (uint32_t k = 0; k < kU; ++k) {
        const uint32_t q = q0 + k * nthr + tid;
        if (q < nv) __builtin_nontemporal_store(y[k], reinterpret_cast<gptr<u32x4>>(dst + head + q * VPL));
      }
    }
  }
};

// The run into the bucket whose pointer is at *slot (read once the loads are out).
template <typename T>
__device__ __forceinline__ void block_copy_slot(const uint64_t* slot, uint64_t e0, const T* src, uint32_t n,
                                                uint32_t tid, uint32_t nthr) {
  if (n == 0) return;
  RunCopy<T> rc;
  rc.load(src, e0, n, tid, nthr);
  rc.store(reinterpret_cast<T*>(*slot));
}

// Phase 2: tile t of LFVector v copies its values to rbase[v] + (its offset
// within the LFVector's share of the round).  The tile's offsets, rbase and the
// frozen flag are read together; the bucket runs follow from rbase alone.
template <typename T>
__global__ __launch_bounds__(kB) void packed_copy_kernel(ArrRef A, TileArgs I, const T* values,
                                                         const uint64_t* tile_off, uint64_t ntiles,
                                                         uint64_t n_values) {
  const uint64_t tile = blockIdx.x;
  const uint32_t v = (uint32_t)(tile / I.tpv);
  const uint64_t off = packed_offset(tile_off, ntiles, tile);
  const uint64_t end = packed_offset(tile_off, ntiles, tile + 1);
  const uint64_t first = packed_offset(tile_off, ntiles, (uint64_t)v * I.tpv);
  const uint64_t total = packed_offset(tile_off, ntiles, ntiles);
  const uint64_t rb = A.rbase[v];
  const uint32_t dead = A.dead[v];
  const uint32_t n = (uint32_t)(end - off);
  if (n == 0 || dead || total > n_values) return;  // frozen before or by this round; refused round
  const uint32_t log2F = A.log2F;
  const uint64_t base = rb + (off - first);
  const T* src = values + off;
  const uint64_t* row = A.bptr + (uint64_t)v * kMaxBuckets;
  const uint32_t b0 = bucket_of(log2F, base), b1 = bucket_of(log2F, base + n - 1);
  if (b1 == b0 + 1) {
    // Two runs (the tile crosses one bucket boundary): waves 0-1 copy the first,
    // waves 2-3 the second, so the loads of both are in flight together.
    const uint64_t split = bucket_start(log2F, b1);
    const uint32_t na = (uint32_t)(split - base);
    const uint32_t half = kB / 2, tid = threadIdx.x;
    if (tid < half)
      block_copy_slot<T>(row + b0, base - bucket_start(log2F, b0), src, na, tid, half);
    else
      block_copy_slot<T>(row + b1, 0, src + na, n - na, tid - half, half);
    return;
  }
  for (uint32_t i = 0; i < n;) {  // one run per bucket the tile's outputs reach
    const uint64_t idx = base + i;
    const uint32_t b = bucket_of(log2F, idx);
    const uint64_t bs = bucket_start(log2F, b);
    const uint64_t room = bs + bucket_len(log2F, b) - idx;
    const uint32_t run = (uint64_t)(n - i) < room ? n - i : (uint32_t)room;
    block_copy_slot<T>(row + b, idx - bs, src + i, run, threadIdx.x, kB);
    i += run;
  }
}

// One tile per LFVector (tpv == 1): the tile's workgroup grows its LFVector and
// copies in one pass.  The runs follow from the LFVector's size alone, so the
// value loads go out first; wave 0 allocates the buckets the round reaches
// while they are in flight (as grow_vector_by does: all or the LFVector is
// frozen with its size unchanged) and hands the pointers to the other waves
// through LDS; the stores follow.  The prefix is known, so counts asking for
// more values than given are refused before anything grows.
template <typename T>
__global__ __launch_bounds__(kB) void packed_grow_copy_kernel(ArrRef A, TileArgs I, const T* values,
                                                              const uint64_t* tile_off, uint64_t ntiles,
                                                              uint64_t n_values) {
  __shared__ uint64_t s_bp[kMaxBuckets];
  __shared__ uint32_t s_fail;
  const uint32_t v = blockIdx.x, tid = threadIdx.x, lane = tid & 63u;
  const uint64_t off = packed_offset(tile_off, ntiles, v);
  const uint64_t end = packed_offset(tile_off, ntiles, (uint64_t)v + 1);
  const uint64_t total = packed_offset(tile_off, ntiles, ntiles);
  const uint64_t s0 = A.size[v];
  const uint32_t dead = A.dead[v];
  if (total > n_values) {
    if (v == 0 && tid == 0) set_error(A.err, kErrRange);
    return;
  }
  const uint32_t n = (uint32_t)(end - off);
  if (n == 0 || dead) return;
  const uint32_t log2F = A.log2F;
  const T* src = values + off;
  const uint32_t b0 = bucket_of(log2F, s0), b1 = bucket_of(log2F, s0 + n - 1);
  // This thread's run (one run: all threads; two: waves 0-1 and 2-3).
  RunCopy<T> rc;
  uint32_t mine = b0;
  if (b1 == b0) {
    rc.load(src, s0 - bucket_start(log2F, b0), n, tid, kB);
  } else if (b1 == b0 + 1) {
    const uint32_t na = (uint32_t)(bucket_start(log2F, b1) - s0), half = kB / 2;
    if (tid < half) {
      rc.load(src, s0 - bucket_start(log2F, b0), na, tid, half);
    } else {
      rc.load(src + na, 0, n - na, tid - half, half);
      mine = b1;
    }
  }
  const uint32_t lo = nbuckets_for(log2F, s0), hi = nbuckets_for(log2F, s0 + n);
  if (tid < lo) s_bp[tid] = A.bptr[(uint64_t)v * kMaxBuckets + tid];  // buckets from earlier rounds
  if (tid < 64) {
    const uint32_t b = lo + lane;
    bool failed = false;
    if (b < hi) {
      if (b >= (uint32_t)kMaxBuckets) {
        failed = true;
      } else {
        uint8_t* q = pool_alloc(A.pool, bucket_class(log2F, I.elem_log2, b), pool_shard(v, b, A.salt));
        const uint64_t p = q ? (uint64_t)q : kFailedPtr;
        A.bptr[(uint64_t)v * kMaxBuckets + b] = p;
        s_bp[b] = p;
        failed = !q;
      }
    }
    const bool any = __ballot(failed) != 0;
    if (lane == 0) {
      s_fail = any ? 1u : 0u;
      if (any) {
        set_error(A.err, kErrNoMem);
        A.dead[v] = 1u;
      } else {
        A.size[v] = s0 + n;
      }
    }
  }
  __syncthreads();
  if (s_fail) return;
  if (b1 <= b0 + 1) {
    rc.store(reinterpret_cast<T*>(s_bp[mine]));
    return;
  }
  for (uint32_t i = 0; i < n;) {  // three runs or more (small first buckets)
    const uint64_t idx = s0 + i;
    const uint32_t b = bucket_of(log2F, idx);
    const uint64_t bs = bucket_start(log2F, b);
    const uint64_t room = bs + bucket_len(log2F, b) - idx;
    const uint32_t run = (uint64_t)(n - i) < room ? n - i : (uint32_t)room;
    RunCopy<T> r;
    r.load(src + i, idx - bs, run, tid, kB);
    r.store(reinterpret_cast<T*>(s_bp[b]));
    i += run;
  }
}

// ------------------------------------------- flagged rounds in two passes --
// The mask pass holds nothing but the flags, so all of a lane's flag bytes are
// loaded before the first is tested (64 loads in flight, against 16 in the
// one-launch kernel, whose payload registers leave no room for more): the
// configuration-2 mask pass drops from 71 to 56 us.
__device__ __forceinline__ SlotMask mask_pass_flags(const uint8_t* flags, uint64_t g0, uint64_t gend) {
  const uint32_t lane = lane_id();
  SlotMask m;
#pragma unroll
  for (int k = 0; k < kMaskWords; ++k) m.w[k] = 0;
  if (g0 >= gend) return m;
  const uint64_t last = gend - 1;
  uint8_t f[kWaveSlots];
#pragma unroll
  for (int j = 0; j < kWaveSlots; ++j) {
    const uint64_t g = g0 + (uint64_t)j * 64 + lane;
    f[j] = flags[g < gend ? g : last];  // clamped: slots past the tile read its last flag
  }
#pragma unroll
  for (int j = 0; j < kWaveSlots; ++j)
    if (f[j] && g0 + (uint64_t)j * 64 + lane < gend) m.w[j >> 6] |= 1ull << (j & 63);
  return m;
}

// Lane-blocked masks.  When every tile of a round starts and ends on a whole
// 16-byte payload vector (the LFVector chunk and the thread count multiples of
// E = 16 / sizeof(T), the payloads 16-byte aligned, the flags E-byte aligned),
// lane l of a tile owns threads g0 + 64 E c + E l + i (chunk c < 64 / E, i < E)
// as bit E c + i of its mask word: the mask pass reads E flag bytes per load and
// the copy pass one 16-byte payload vector per chunk, where the slot layout
// reads one byte and one element per lane and load.
template <uint32_t E>
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t x) {
  uint32_t b = 0;
#pragma unroll
  for (uint32_t i = 0; i < E; ++i) b |= (uint32_t)(((x >> (8 * i)) & 0xFFu) != 0u) << i;
  return b;
}

// One tile in lane-blocked masks, every flag word loaded before the first is
// tested (batching a wave's four tiles of the mask pass into one set of loads
// measured slower: 51 against 44 us).
template <uint32_t E>
__device__ __forceinline__ uint64_t mask_pass_blocked(const uint8_t* flags, uint64_t g0, uint64_t gend) {
  static_assert(E == 2 || E == 4, "16-byte vectors of 4- or 8-byte elements");
  typedef typename std::conditional<E == 4, uint32_t, uint16_t>::type W;
  constexpr uint32_t C = 64 / E;
  const uint32_t lane = lane_id();
  if (g0 >= gend) return 0;
  W f[C];
#pragma unroll
  for (uint32_t c = 0; c < C; ++c) {
    const uint64_t g = g0 + (uint64_t)c * 64 * E + lane * E;
    f[c] = *reinterpret_cast<const W*>(flags + (g < gend ? g : gend - E));  // clamped to the tile's last E flags
  }
  uint64_t m = 0;
#pragma unroll
  for (uint32_t c = 0; c < C; ++c)
    if (g0 + (uint64_t)c * 64 * E + lane * E < gend) m |= (uint64_t)nonzero_bytes<E>(f[c]) << (c * E);
  return m;
}

// A round from buffers with flags, whose LFVectors span several 4096-thread
// tiles, runs in the packed form instead of one launch with per-LFVector tickets
// and the decoupled look-back: flag_mask_kernel reads the flags once (one wave
// per tile, as the one-launch kernel does), keeps each lane's slot mask (512
// bytes per tile) and writes the tile's count in the packed offset layout; the
// group scan and the grow launch of the packed rounds follow; flag_copy_kernel
// then takes each tile's masks and payloads and stores the kept payloads at
// offsets known in advance, with no waits.  Element order, sizes and buckets are
// those of the one-launch kernel; the flags cost 1/8 byte per thread more (the
// masks written and read back).  E = 1: the slot layout; E = 2, 4: lane-blocked
// masks (configuration-2 sparse rounds, 2^27 threads at V = 512: mask pass 56 ->
// 44 us, copy pass 166 -> 161 us).
template <uint32_t E>
__global__ __launch_bounds__(kB) void flag_mask_kernel(TileArgs I, const uint8_t* flags, uint64_t* masks,
                                                       uint64_t* off, uint64_t ntiles) {
  __shared__ uint32_t s_sum[kPackGroup];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint64_t first = (uint64_t)blockIdx.x * kPackGroup;
  for (uint32_t j = w; j < kPackGroup; j += kW) {
    const uint64_t tile = first + j;
    uint32_t c = 0;
    if (tile < ntiles) {
      const uint32_t v = (uint32_t)(tile / I.tpv);
      uint64_t g0, gend;
      tile_range(I, v, tile - (uint64_t)v * I.tpv, kWaveTile, g0, gend);
      if constexpr (E == 1) {
        const SlotMask m = mask_pass_flags(flags, g0, gend);
#pragma unroll
        for (int k = 0; k < kMaskWords; ++k) masks[(tile * kMaskWords + k) * 64 + lane] = m.w[k];
        c = (uint32_t)wave_sum64((uint64_t)m.count());
      } else {
        const uint64_t m = mask_pass_blocked<E>(flags, g0, gend);
        masks[tile * 64 + lane] = m;
        c = (uint32_t)wave_sum64((uint64_t)__popcll(m));
      }
    }
    if (lane == 0) s_sum[j] = c;
  }
  __syncthreads();
  if (tid < kPackGroup) {
    uint64_t before = 0, all = 0;
    for (uint32_t q = 0; q < kPackGroup; ++q) {
      before += q < tid ? s_sum[q] : 0u;
      all += s_sum[q];
    }
    if (first + tid < ntiles) off[first + tid] = before;
    if (tid == 0) off[ntiles + blockIdx.x] = all;
  }
}

// One wave per tile: the tile's kept payloads go to the LFVector's elements
// rbase[v] + (tile offset within the LFVector) on, in slot order (the logical
// thread order), payloads loaded kValBatch slots ahead of their stores.  The
// buckets were allocated by the grow launch; lane k holds the pointer of the
// k-th bucket the tile reaches.
template <typename T>
__global__ __launch_bounds__(64) void flag_copy_kernel(ArrRef A, TileArgs I, const T* values,
                                                       const uint64_t* masks, const uint64_t* off,
                                                       uint64_t ntiles) {
  const uint64_t tile = blockIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t v = (uint32_t)(tile / I.tpv);
  uint64_t g0, gend;
  tile_range(I, v, tile - (uint64_t)v * I.tpv, kWaveTile, g0, gend);
  if (g0 >= gend || A.dead[v]) return;
  const uint64_t o0 = packed_offset(off, ntiles, tile);
  const uint32_t n_t = (uint32_t)(packed_offset(off, ntiles, tile + 1) - o0);
  if (n_t == 0) return;
  const uint64_t base = A.rbase[v] + (o0 - packed_offset(off, ntiles, (uint64_t)v * I.tpv));
  SlotMask bits;
#pragma unroll
  for (int k = 0; k < kMaskWords; ++k) bits.w[k] = masks[(tile * kMaskWords + k) * 64 + lane];
  const uint32_t log2F = A.log2F;
  const uint32_t b_lo = bucket_of(log2F, base), b_hi = bucket_of(log2F, base + n_t - 1);
  const uint64_t bp = b_lo + lane <= b_hi ? A.bptr[(uint64_t)v * kMaxBuckets + b_lo + lane] : 0;
  const ProdBuffer<T> prod{values, nullptr};
  uint32_t run = 0;
  if (b_lo == b_hi) {
    const gptr<T> dst = gmem(reinterpret_cast<T*>(__shfl(bp, 0, 64)) + offset_in(log2F, base, b_lo));
    for (int j0 = 0; j0 < kWaveSlots; j0 += kValBatch) {
      T val[kValBatch];
      wave_values<T, ProdBuffer<T>>(prod, g0, gend, j0, val);
#pragma unroll
      for (int k = 0; k < kValBatch; ++k) {
        const bool f = bits.get(j0 + k);
        const uint64_t m = __ballot(f);
        if (f) dst[run + mbcnt(m)] = val[k];
        run += (uint32_t)__popcll(m);
      }
    }
    return;
  }
  for (int j0 = 0; j0 < kWaveSlots; j0 += kValBatch) {
    T val[kValBatch];
    wave_values<T, ProdBuffer<T>>(prod, g0, gend, j0, val);
#pragma unroll
    for (int k = 0; k < kValBatch; ++k) {
      const bool f = bits.get(j0 + k);
      const uint64_t m = __ballot(f);
      const uint64_t idx = base + run + mbcnt(m);
      const uint32_t b = f ? bucket_of(log2F, idx) : b_lo;
      const uint64_t p = __shfl(bp, (int)(b - b_lo), 64);
      if (f) gmem(reinterpret_cast<T*>(p))[offset_in(log2F, idx, b)] = val[k];
      run += (uint32_t)__popcll(m);
    }
  }
}

// The copy pass over lane-blocked masks: chunk c of the tile is one 16-byte
// payload vector per lane (kChunkBatch chunks loaded ahead of their stores); the
// kept elements of a chunk take their places in thread order from E ballots
// (bit i of every lane's E bits) and the lane's own rank, are gathered in LDS,
// and leave it as contiguous runs (64 consecutive elements per store, as the
// slot layout's ballots give: stores scattered over a lane-blocked chunk
// measured 181 against 166 us).  kOne: the tile's elements all land in one
// bucket, at dst1 on.
constexpr uint32_t kChunkBatch = 8;
template <typename T, bool kOne>
__device__ __forceinline__ void copy_blocked(const T* values, uint64_t g0, uint64_t gend, uint64_t word,
                                             gptr<T> dst1, uint64_t base, uint32_t log2F, uint32_t b_lo,
                                             uint64_t bp, T* s_keep) {
  constexpr uint32_t E = 16 / sizeof(T), C = 64 / E;
  static_assert(kMaskWords == 1 && C % kChunkBatch == 0, "one 64-bit mask word per lane");
  const uint32_t lane = lane_id();
  const gptr<const T> src = gmem(values);
  uint32_t run = 0;
#pragma unroll 1
  for (uint32_t c0 = 0; c0 < C; c0 += kChunkBatch) {
    u32x4 x[kChunkBatch];
#pragma unroll
    for (uint32_t u = 0; u < kChunkBatch; ++u) {
      const uint64_t g = g0 + (uint64_t)(c0 + u) * 64 * E + lane * E;
      x[u] = *reinterpret_cast<gptr<const u32x4>>(src + (g < gend ? g : gend - E));  // clamped to the tile's last vector
    }
    const uint32_t first = run;  // the batch's first position in the tile
#pragma unroll
    for (uint32_t u = 0; u < kChunkBatch; ++u) {
      const uint32_t bits = (uint32_t)(word >> ((c0 + u) * E)) & ((1u << E) - 1u);
      uint32_t pos = run - first;
#pragma unroll
      for (uint32_t i = 0; i < E; ++i) {
        const uint64_t m = __ballot((bits >> i) & 1u);
        pos += mbcnt(m);
        run += (uint32_t)__popcll(m);
      }
      T el[E];
      __builtin_memcpy(el, &x[u], 16);
#pragma unroll
      for (uint32_t i = 0; i < E; ++i) {
        if ((bits >> i) & 1u) s_keep[pos++] = el[i];
      }
    }
    __syncthreads();  // one wave: its LDS writes before its reads
    const uint32_t cnt = run - first;
    for (uint32_t e0 = 0; e0 < cnt; e0 += 64) {  // uniform trip count: the shuffle below needs every lane
      const uint32_t e = e0 + lane;
      const bool f = e < cnt;
      const T val = s_keep[f ? e : 0];
      if constexpr (kOne) {
        if (f) dst1[first + e] = val;
      } else {
        const uint64_t idx = base + first + e;
        const uint32_t b = f ? bucket_of(log2F, idx) : b_lo;
        const uint64_t p = __shfl(bp, (int)(b - b_lo), 64);
        if (f) gmem(reinterpret_cast<T*>(p))[offset_in(log2F, idx, b)] = val;
      }
    }
    __syncthreads();  // the reads before the next batch's writes
  }
}

template <typename T>
__global__ __launch_bounds__(64) void flag_copy_blocked_kernel(ArrRef A, TileArgs I, const T* values,
                                                               const uint64_t* masks, const uint64_t* off,
                                                               uint64_t ntiles) {
  __shared__ T s_keep[kChunkBatch * 64 * (16 / sizeof(T))];
  const uint64_t tile = blockIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t v = (uint32_t)(tile / I.tpv);
  uint64_t g0, gend;
  tile_range(I, v, tile - (uint64_t)v * I.tpv, kWaveTile, g0, gend);
  if (g0 >= gend || A.dead[v]) return;
  const uint64_t o0 = packed_offset(off, ntiles, tile);
  const uint32_t n_t = (uint32_t)(packed_offset(off, ntiles, tile + 1) - o0);
  if (n_t == 0) return;
  const uint64_t base = A.rbase[v] + (o0 - packed_offset(off, ntiles, (uint64_t)v * I.tpv));
  const uint64_t word = masks[tile * 64 + lane];
  const uint32_t log2F = A.log2F;
  const uint32_t b_lo = bucket_of(log2F, base), b_hi = bucket_of(log2F, base + n_t - 1);
  const uint64_t bp = b_lo + lane <= b_hi ? A.bptr[(uint64_t)v * kMaxBuckets + b_lo + lane] : 0;
  if (b_lo == b_hi) {
    const gptr<T> dst1 = gmem(reinterpret_cast<T*>(__shfl(bp, 0, 64)) + offset_in(log2F, base, b_lo));
    copy_blocked<T, true>(values, g0, gend, word, dst1, base, log2F, b_lo, bp, s_keep);
  } else {
    copy_blocked<T, false>(values, g0, gend, word, gptr<T>{}, base, log2F, b_lo, bp, s_keep);
  }
}

// ---------------------------------------------------------------- dispatch --
template <typename T, bool kStatic>
int dispatch(const ArrRef& A, const StaticRef& S, const TileArgs& I, const InsertDesc& d,
             uint64_t ntiles, hipStream_t s) {
  const dim3 grid((uint32_t)ntiles), block(kB);
  switch (d.mode) {
    case kModeBuffer: {
      ProdBuffer<T> p{static_cast<const T*>(d.values), d.flags};
      hipLaunchKernelGGL((insert_wave_kernel<T, ProdBuffer<T>, kStatic>), grid, dim3(64), 0, s, A, S, I, p);
      break;
    }
    case kModeBernoulli: {
      ProdBernoulli<T> p{d.seed, d.round};
      hipLaunchKernelGGL((insert_wave_kernel<T, ProdBernoulli<T>, kStatic>), grid, dim3(64), 0, s, A, S, I, p);
      break;
    }
    case kModeRoundTag: {
      ProdRoundTag<T> p{d.round, d.tag_shift};
      hipLaunchKernelGGL((insert_wave_kernel<T, ProdRoundTag<T>, kStatic>), grid, dim3(64), 0, s, A, S, I, p);
      break;
    }
    case kModeKeyed: {
      ProdKeyed<T> p{d.seed, d.round, d.tag_shift, d.tag};
      hipLaunchKernelGGL((insert_wave_kernel<T, ProdKeyed<T>, kStatic>), grid, dim3(64), 0, s, A, S, I, p);
      break;
    }
    case kModeCounts: {
      ProdCounts<T> p{static_cast<const T*>(d.values), d.flags, d.max_count};
      hipLaunchKernelGGL((insert_count_kernel<T, ProdCounts<T>, kStatic>), grid, block, 0, s, A, S, I, p);
      break;
    }
    case kModePoisson: {
      ProdPoisson<T> p;
      p.seed = d.seed;
      p.round = d.round;
      p.max_count = d.max_count;
      for (int k = 0; k < 16; ++k) p.thr[k] = d.thresholds[k];
      hipLaunchKernelGGL((insert_count_kernel<T, ProdPoisson<T>, kStatic>), grid, block, 0, s, A, S, I, p);
      break;
    }
    default:
      return GGA_EINVAL;
  }
  return hip_status(hipGetLastError());
}

bool multi_mode(uint32_t mode) { return mode == kModeCounts || mode == kModePoisson; }

// Whether a dense round runs as one launch in which one wave per LFVector grows
// and stores it (else a grow launch, then one workgroup per tile).
inline bool wave_per_vector(const TileArgs& I, uint32_t V) { return I.tpv <= 8 || V >= 512; }

template <typename T>
int launch_dense(const ArrRef& A, const TileArgs& I, const InsertDesc& d, uint64_t ntiles, hipStream_t s,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  if (wave_per_vector(I, A.V)) {
    const dim3 grid((A.V + 3) / 4), block(256);
    switch (d.mode) {
      case kModeBuffer:
        hipExtLaunchKernelGGL(grow_store_kernel<T, ProdBuffer<T>>, grid, block, 0, s, e0, e1, 0, A, I,
                           ProdBuffer<T>{static_cast<const T*>(d.values), nullptr});
        break;
      case kModeRoundTag:
        hipExtLaunchKernelGGL(grow_store_kernel<T, ProdRoundTag<T>>, grid, block, 0, s, e0, e1, 0, A, I,
                           ProdRoundTag<T>{d.round, d.tag_shift});
        break;
      case kModeKeyed:
        hipExtLaunchKernelGGL(grow_store_kernel<T, ProdKeyed<T>>, grid, block, 0, s, e0, e1, 0, A, I,
                           ProdKeyed<T>{d.seed, d.round, d.tag_shift, d.tag});
        break;
      default:
        return GGA_EINVAL;
    }
    return hip_status(hipGetLastError());
  }
  hipLaunchKernelGGL(grow_kernel, dim3((A.V + 3) / 4), dim3(256), 0, s, A, I);
  const dim3 grid((uint32_t)ntiles), block(64);
  switch (d.mode) {
    case kModeBuffer:
      hipLaunchKernelGGL((dense_insert_kernel<T, ProdBuffer<T>>), grid, block, 0, s, A, I,
                         ProdBuffer<T>{static_cast<const T*>(d.values), nullptr});
      break;
    case kModeRoundTag:
      hipLaunchKernelGGL((dense_insert_kernel<T, ProdRoundTag<T>>), grid, block, 0, s, A, I,
                         ProdRoundTag<T>{d.round, d.tag_shift});
      break;
    case kModeKeyed:
      hipLaunchKernelGGL((dense_insert_kernel<T, ProdKeyed<T>>), grid, block, 0, s, A, I,
                         ProdKeyed<T>{d.seed, d.round, d.tag_shift, d.tag});
      break;
    default:
      return GGA_EINVAL;
  }
  return hip_status(hipGetLastError());
}

// Look-back words (needed only when an LFVector spans several tiles): grown on
// demand and zeroed when new (a zero word is never current).  Their epochs come
// from the ticket words, so launches need no host-side state and a captured
// graph can be replayed.  Nothing is allocated while the stream is capturing
// (run the same round eagerly first); an outgrown buffer is retired, not freed,
// so graphs that use it stay valid.
int ensure_status(ggarray* a, uint64_t ntiles, hipStream_t s) {
  if (ntiles <= a->status_cap) return GGA_OK;
  if (stream_capturing(s)) return GGA_EINVAL;  // nothing is allocated inside a graph
  uint64_t cap = a->status_cap ? a->status_cap : 4096;
  while (cap < ntiles) cap *= 2;
  if (retire_buffer(a, a->ref.status, s) != GGA_OK) return GGA_EHIP;
  a->ref.status = nullptr;
  a->status_cap = 0;
  void* p = nullptr;
  if (hipMallocAsync(&p, cap * sizeof(uint64_t), s) != hipSuccess) return GGA_EHIP;
  if (hipMemsetAsync(p, 0, cap * sizeof(uint64_t), s) != hipSuccess) return GGA_EHIP;
  a->ref.status = static_cast<uint64_t*>(p);
  a->status_cap = cap;
  return GGA_OK;
}


}  // namespace

static int queue_flag_rounds(ggarray* a, const InsertDesc& d, const TileArgs& I, uint64_t ntiles, hipStream_t s);
static bool flag_rounds_fit(const ggarray* a, uint64_t ntiles, hipStream_t s);

// Rounds ds[0..n) of one generated producer, each followed by the shrink
// sh_num / sh_den (0: none).  One launch when every round is dense (round-tag or
// keyed payloads) and runs one wave per LFVector, and only the round number and
// the thread count change between rounds; otherwise the rounds one by one.
// Every round is checked before anything is queued.
int launch_insert_rounds(ggarray* a, const InsertDesc* ds, uint32_t n, hipStream_t s, uint32_t sh_num,
                         uint32_t sh_den, bool clear) {
  if (sh_num == 0) sh_den = 0;
  bool fuse = (n >= 2 || (n == 1 && clear)) && n <= kMaxFusedRounds;
  for (uint32_t r = 0; r < n; ++r) {
    const InsertDesc& d = ds[r];
    const uint64_t chunk = (d.n_threads + a->V - 1) / a->V;
    const uint64_t tile = multi_mode(d.mode) ? kCountTile : kFlagTile;
    const uint64_t tpv = (chunk + tile - 1) / tile;
    if (tpv * a->V > 0x7FFFFFFFull || chunk * (multi_mode(d.mode) ? d.max_count : 1u) >= (1ull << 32))
      return GGA_EINVAL;
    TileArgs I{};
    I.tpv = tpv;
    fuse = fuse && (d.mode == kModeRoundTag || d.mode == kModeKeyed) && d.mode == ds[0].mode &&
           d.seed == ds[0].seed && d.tag_shift == ds[0].tag_shift && d.tag == ds[0].tag && wave_per_vector(I, a->V);
  }
  if (!fuse) {
    if (clear) {
      const int st = launch_shrink(a, 1, 1, s);
      if (st) return st;
    }
    for (uint32_t r = 0; r < n; ++r) {
      const int st = launch_insert(a, ds[r], s, sh_num, sh_den);
      if (st) return st;
    }
    return GGA_OK;
  }
  a->tev_set &= ~4u;  // not a timed round
  if (clear) a->size_ub = 0;
  RoundList R{};
  R.n = n;
  for (uint32_t r = 0; r < n; ++r) {
    R.round[r] = ds[r].round;
    R.n_threads[r] = ds[r].n_threads;
    grow_bound(a, ds[r].n_threads);
  }
  TileArgs I{};
  I.elem_log2 = a->elem_log2;
  I.sh_num = sh_num;
  I.sh_den = sh_den;
  I.reuse = clear ? 1u : 0u;
  const dim3 grid((a->V + 3) / 4), block(256);
  const InsertDesc& d = ds[0];
  if (d.mode == kModeRoundTag) {
    if (a->elem_bytes == 4)
      hipLaunchKernelGGL((grow_store_rounds_kernel<uint32_t, ProdRoundTag<uint32_t>>), grid, block, 0, s, a->ref, I,
                         ProdRoundTag<uint32_t>{0, d.tag_shift}, R);
    else
      hipLaunchKernelGGL((grow_store_rounds_kernel<uint64_t, ProdRoundTag<uint64_t>>), grid, block, 0, s, a->ref, I,
                         ProdRoundTag<uint64_t>{0, d.tag_shift}, R);
  } else {
    if (a->elem_bytes == 4)
      hipLaunchKernelGGL((grow_store_rounds_kernel<uint32_t, ProdKeyed<uint32_t>>), grid, block, 0, s, a->ref, I,
                         ProdKeyed<uint32_t>{d.seed, 0, d.tag_shift, d.tag}, R);
    else
      hipLaunchKernelGGL((grow_store_rounds_kernel<uint64_t, ProdKeyed<uint64_t>>), grid, block, 0, s, a->ref, I,
                         ProdKeyed<uint64_t>{d.seed, 0, d.tag_shift, d.tag}, R);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e);
  sizes_changed(a, s);
  if (sh_den && sh_num == sh_den) a->size_ub = 0;
  return GGA_OK;
}

int launch_insert(ggarray* a, const InsertDesc& d, hipStream_t s, uint32_t sh_num, uint32_t sh_den) {
  if (sh_num == 0) sh_den = 0;  // a shrink that pops nothing
  a->tev_set &= ~4u;            // set again below if this round is timed
  if (d.n_threads == 0) return sh_den ? launch_shrink(a, sh_num, sh_den, s) : GGA_OK;
  const uint64_t tile = multi_mode(d.mode) ? kCountTile : kFlagTile;
  const uint64_t chunk = (d.n_threads + a->V - 1) / a->V;
  const uint64_t tpv = (chunk + tile - 1) / tile;
  const uint64_t ntiles = tpv * a->V;
  if (ntiles > 0x7FFFFFFFull) return GGA_EINVAL;
  // One round may add fewer than 2^32 elements to an LFVector (status words hold
  // round-relative 32-bit values).
  if (chunk * (multi_mode(d.mode) ? d.max_count : 1u) >= (1ull << 32)) return GGA_EINVAL;

  TileArgs I;
  I.n_threads = d.n_threads;
  I.chunk = chunk;
  I.tpv = tpv;
  I.elem_log2 = a->elem_log2;
  grow_bound(a, d.n_threads * (multi_mode(d.mode) ? d.max_count : 1u));
  const bool dense = d.mode == kModeRoundTag || d.mode == kModeKeyed || (d.mode == kModeBuffer && !d.flags);
  if (dense) {
    const bool fused = sh_den && wave_per_vector(I, a->V);
    if (fused) {
      I.sh_num = sh_num;
      I.sh_den = sh_den;
    }
    // Kernel timing: a round that is one launch records the array's round events.
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (a->tev[2][0] && wave_per_vector(I, a->V) && !stream_capturing(s)) {
      e0 = a->tev[2][0];
      e1 = a->tev[2][1];
      a->tev_set |= 4u;
    }
    int st = a->elem_bytes == 4 ? launch_dense<uint32_t>(a->ref, I, d, ntiles, s, e0, e1)
                                : launch_dense<uint64_t>(a->ref, I, d, ntiles, s, e0, e1);
    if (st == GGA_OK) sizes_changed(a, s);
    if (fused && st == GGA_OK && sh_num == sh_den) a->size_ub = 0;
    if (!fused && sh_den && st == GGA_OK) st = launch_shrink(a, sh_num, sh_den, s);
    return st;
  }

  if (d.mode == kModeBuffer && d.flags && tpv > 1 && flag_rounds_fit(a, ntiles, s)) {
    int st = queue_flag_rounds(a, d, I, ntiles, s);
    if (sh_den && st == GGA_OK) st = launch_shrink(a, sh_num, sh_den, s);
    return st;
  }
  if (tpv > 1) {
    const int rc = ensure_status(a, ntiles, s);
    if (rc) return rc;
  }
  StaticRef S{};
  int st = a->elem_bytes == 4 ? dispatch<uint32_t, false>(a->ref, S, I, d, ntiles, s)
                              : dispatch<uint64_t, false>(a->ref, S, I, d, ntiles, s);
  if (st == GGA_OK) sizes_changed(a, s);
  if (sh_den && st == GGA_OK) st = launch_shrink(a, sh_num, sh_den, s);
  return st;
}

int launch_insert_segments(ggarray* a, const void* values, const uint64_t* prefix, uint64_t n_values,
                           hipStream_t s) {
  TileArgs I{};
  I.elem_log2 = a->elem_log2;
  a->tev_set &= ~4u;  // not a timed round
  grow_bound(a, n_values);
  const dim3 grid((a->V + 3) / 4), block(256);
  if (a->elem_bytes == 4)
    hipLaunchKernelGGL(segments_kernel<uint32_t>, grid, block, 0, s, a->ref, I, static_cast<const uint32_t*>(values),
                       prefix, n_values);
  else
    hipLaunchKernelGGL(segments_kernel<uint64_t>, grid, block, 0, s, a->ref, I, static_cast<const uint64_t*>(values),
                       prefix, n_values);
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) sizes_changed(a, s);
  return hip_status(e);
}

// Value offsets of a packed round (ntiles + ngroups + 1 words), grown like the
// look-back words (nothing is allocated while the stream is capturing).
static int ensure_packed_offsets(ggarray* a, uint64_t words, hipStream_t s) {
  if (words <= a->pk_cap) return GGA_OK;
  if (stream_capturing(s)) return GGA_EINVAL;
  uint64_t cap = a->pk_cap ? a->pk_cap : 4096;
  while (cap < words) cap *= 2;
  if (retire_buffer(a, a->pk_off, s) != GGA_OK) return GGA_EHIP;
  a->pk_off = nullptr;
  a->pk_cap = 0;
  void* p = nullptr;
  if (hipMallocAsync(&p, cap * sizeof(uint64_t), s) != hipSuccess) return GGA_EHIP;
  a->pk_off = static_cast<uint64_t*>(p);
  a->pk_cap = cap;
  return GGA_OK;
}

// The kernels of one packed round: tile totals and their prefix (off: ntiles +
// ngroups + 1 words), the growth of every LFVector, then the copy.
static int queue_packed(ggarray* a, uint64_t* off, const void* values, const uint8_t* counts, const TileArgs& I,
                        uint64_t ntiles, uint64_t n_values, hipStream_t s) {
  grow_bound(a, n_values);
  const uint64_t ngroups = packed_groups(ntiles);
  hipLaunchKernelGGL(packed_group_kernel, dim3((uint32_t)ngroups), dim3(kB), 0, s, I, counts, off, ntiles);
  hipLaunchKernelGGL(packed_tile_scan_kernel, dim3(1), dim3(1024), 0, s, off + ntiles, ngroups);
  const dim3 grid((uint32_t)ntiles), block(kB);
  const uint64_t* o = off;
  if (I.tpv == 1) {  // one tile per LFVector: grow and copy in one pass
    if (a->elem_bytes == 4)
      hipLaunchKernelGGL(packed_grow_copy_kernel<uint32_t>, grid, block, 0, s, a->ref, I,
                         static_cast<const uint32_t*>(values), o, ntiles, n_values);
    else
      hipLaunchKernelGGL(packed_grow_copy_kernel<uint64_t>, grid, block, 0, s, a->ref, I,
                         static_cast<const uint64_t*>(values), o, ntiles, n_values);
  } else {
    hipLaunchKernelGGL(packed_grow_kernel, dim3((a->V + 3) / 4), dim3(256), 0, s, a->ref, I, o, ntiles, n_values);
    if (a->elem_bytes == 4)
      hipLaunchKernelGGL(packed_copy_kernel<uint32_t>, grid, block, 0, s, a->ref, I,
                         static_cast<const uint32_t*>(values), o, ntiles, n_values);
    else
      hipLaunchKernelGGL(packed_copy_kernel<uint64_t>, grid, block, 0, s, a->ref, I,
                         static_cast<const uint64_t*>(values), o, ntiles, n_values);
  }
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) sizes_changed(a, s);
  return hip_status(e);
}

// Words of a flagged round in two passes: the slot masks, then the packed offsets.
static uint64_t flag_round_words(uint64_t ntiles) {
  return ntiles * kMaskWords * 64 + ntiles + packed_groups(ntiles) + 1;
}

// Whether the two-pass form can run: its buffer is large enough or can be grown
// (not while the stream is capturing; a captured round then takes the one-launch
// form).
static bool flag_rounds_fit(const ggarray* a, uint64_t ntiles, hipStream_t s) {
  return flag_round_words(ntiles) <= a->pk_cap || !stream_capturing(s);
}

// A buffer round with flags over LFVectors of several tiles: masks and tile
// counts, their prefix, the growth of every LFVector, then the copy.
static int queue_flag_rounds(ggarray* a, const InsertDesc& d, const TileArgs& I, uint64_t ntiles, hipStream_t s) {
  int rc = ensure_packed_offsets(a, flag_round_words(ntiles), s);
  if (rc) return rc;
  uint64_t* masks = a->pk_off;
  uint64_t* off = masks + ntiles * kMaskWords * 64;
  const uint64_t ngroups = packed_groups(ntiles);
  // Lane-blocked masks when every tile starts and ends on a whole 16-byte payload
  // vector and the buffers are aligned for the vector loads; else the slot layout.
  const uint32_t E = 16u / a->elem_bytes;
  const bool blocked = I.chunk % E == 0 && I.n_threads % E == 0 &&
                       (reinterpret_cast<uintptr_t>(d.values) & 15u) == 0 &&
                       (reinterpret_cast<uintptr_t>(d.flags) & (E - 1)) == 0;
  const dim3 mgrid((uint32_t)ngroups), mblock(kB), cgrid((uint32_t)ntiles), cblock(64);
  if (!blocked)
    hipLaunchKernelGGL(flag_mask_kernel<1>, mgrid, mblock, 0, s, I, d.flags, masks, off, ntiles);
  else if (E == 4)
    hipLaunchKernelGGL(flag_mask_kernel<4>, mgrid, mblock, 0, s, I, d.flags, masks, off, ntiles);
  else
    hipLaunchKernelGGL(flag_mask_kernel<2>, mgrid, mblock, 0, s, I, d.flags, masks, off, ntiles);
  hipLaunchKernelGGL(packed_tile_scan_kernel, dim3(1), dim3(1024), 0, s, off + ntiles, ngroups);
  hipLaunchKernelGGL(packed_grow_kernel, dim3((a->V + 3) / 4), dim3(256), 0, s, a->ref, I, off, ntiles, ~0ull);
  if (a->elem_bytes == 4) {
    const uint32_t* vals = static_cast<const uint32_t*>(d.values);
    if (blocked)
      hipLaunchKernelGGL(flag_copy_blocked_kernel<uint32_t>, cgrid, cblock, 0, s, a->ref, I, vals, masks, off, ntiles);
    else
      hipLaunchKernelGGL(flag_copy_kernel<uint32_t>, cgrid, cblock, 0, s, a->ref, I, vals, masks, off, ntiles);
  } else {
    const uint64_t* vals = static_cast<const uint64_t*>(d.values);
    if (blocked)
      hipLaunchKernelGGL(flag_copy_blocked_kernel<uint64_t>, cgrid, cblock, 0, s, a->ref, I, vals, masks, off, ntiles);
    else
      hipLaunchKernelGGL(flag_copy_kernel<uint64_t>, cgrid, cblock, 0, s, a->ref, I, vals, masks, off, ntiles);
  }
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) sizes_changed(a, s);
  return hip_status(e);
}

// Tile geometry of a packed round; GGA_EINVAL if the round is too large.
static int packed_geometry(const ggarray* a, uint64_t n_threads, TileArgs& I, uint64_t& ntiles) {
  const uint64_t chunk = (n_threads + a->V - 1) / a->V;
  const uint64_t tpv = (chunk + kCountTile - 1) / kCountTile;
  ntiles = tpv * a->V;
  if (ntiles > 0x7FFFFFFFull || chunk * 255u >= (1ull << 32)) return GGA_EINVAL;
  I = TileArgs{};
  I.n_threads = n_threads;
  I.chunk = chunk;
  I.tpv = tpv;
  I.elem_log2 = a->elem_log2;
  return GGA_OK;
}

int launch_insert_packed(ggarray* a, const void* values, const uint8_t* counts, uint64_t n_threads,
                         uint64_t n_values, hipStream_t s) {
  a->tev_set &= ~4u;  // not a timed round
  if (n_threads == 0) return GGA_OK;
  TileArgs I;
  uint64_t ntiles = 0;
  int rc = packed_geometry(a, n_threads, I, ntiles);
  if (rc) return rc;
  rc = ensure_packed_offsets(a, ntiles + packed_groups(ntiles) + 1, s);
  if (rc) return rc;
  return queue_packed(a, a->pk_off, values, counts, I, ntiles, n_values, s);
}

// ------------------------------------------- packed round without allocation --
// The tile offsets of ggarray_insert_packed_noalloc (ntiles + ngroups + 1 words)
// live in this file-scope array: each device holds its own copy for the life of
// the process.  Host code never passes the symbol itself to a kernel: its device
// address is looked up once per device and kept.
constexpr uint64_t kNoAllocTiles = 65536;
constexpr uint64_t kScratchWords = kNoAllocTiles + kNoAllocTiles / kPackGroup + 32;  // whole 256-byte lines
static __device__ __align__(256) uint64_t scratch[kScratchWords];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static uint64_t* g_scratch_ptr[kMaxScratchDevices] = {};

// The current device's copy of `scratch`, resolved on the first call on it.
static int scratch_base(uint64_t** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GGA_EHIP;
  if (dev < 0 || dev >= kMaxScratchDevices) return GGA_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return GGA_EHIP;
    }
    g_scratch_ptr[dev] = static_cast<uint64_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return GGA_OK;
}

int launch_insert_packed_noalloc(ggarray* a, const void* values, const uint8_t* counts, uint64_t n_threads,
                                 uint64_t n_values, hipStream_t s) {
  a->tev_set &= ~4u;
  if (n_threads == 0) return GGA_OK;
  TileArgs I;
  uint64_t ntiles = 0;
  int rc = packed_geometry(a, n_threads, I, ntiles);
  if (rc) return rc;
  if (ntiles > kNoAllocTiles) return GGA_ERANGE;  // beyond the scratch: nothing queued
  uint64_t* sc = nullptr;
  rc = scratch_base(&sc);
  if (rc) return rc;
  return queue_packed(a, sc, values, counts, I, ntiles, n_values, s);  // every word it reads is written first
}

// A round of n threads (each inserting at most `per`) raises the host's bound
// of the static array's size by at most n * per, never past the capacity.
static void static_grow_bound(gga_static* st, uint64_t n, uint64_t per) {
  const uint64_t room = st->cap - (st->size_ub < st->cap ? st->size_ub : st->cap);
  st->size_ub += (per && n > room / per) ? room : n * per;
}

int launch_static_insert_atomic(gga_static* st, const InsertDesc& d, hipStream_t s) {
  st->rw_last = false;
  if (d.n_threads == 0) return GGA_OK;
  static_grow_bound(st, d.n_threads, 1);
  StaticRef S{st->data, st->cap, st->d_size, st->d_err, st->d_done};
  uint64_t blocks = (d.n_threads + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  const dim3 grid((uint32_t)blocks), block(256);
  const bool u32 = st->elem_bytes == 4;
  switch (d.mode) {
    case kModeBernoulli:
      if (u32) hipLaunchKernelGGL((static_atomic_kernel<uint32_t, ProdBernoulli<uint32_t>>), grid, block, 0, s, S, d.n_threads, ProdBernoulli<uint32_t>{d.seed, d.round});
      else hipLaunchKernelGGL((static_atomic_kernel<uint64_t, ProdBernoulli<uint64_t>>), grid, block, 0, s, S, d.n_threads, ProdBernoulli<uint64_t>{d.seed, d.round});
      break;
    case kModeRoundTag:
      if (u32) hipLaunchKernelGGL((static_atomic_kernel<uint32_t, ProdRoundTag<uint32_t>>), grid, block, 0, s, S, d.n_threads, ProdRoundTag<uint32_t>{d.round, d.tag_shift});
      else hipLaunchKernelGGL((static_atomic_kernel<uint64_t, ProdRoundTag<uint64_t>>), grid, block, 0, s, S, d.n_threads, ProdRoundTag<uint64_t>{d.round, d.tag_shift});
      break;
    case kModeKeyed:
      if (u32) hipLaunchKernelGGL((static_atomic_kernel<uint32_t, ProdKeyed<uint32_t>>), grid, block, 0, s, S, d.n_threads, ProdKeyed<uint32_t>{d.seed, d.round, d.tag_shift, d.tag});
      else hipLaunchKernelGGL((static_atomic_kernel<uint64_t, ProdKeyed<uint64_t>>), grid, block, 0, s, S, d.n_threads, ProdKeyed<uint64_t>{d.seed, d.round, d.tag_shift, d.tag});
      break;
    default:
      return GGA_EINVAL;
  }
  return hip_status(hipGetLastError());
}

template <typename T>
int launch_static_dense(const StaticRef& S, const InsertDesc& d, uint64_t ntiles, hipStream_t s) {
  const uint64_t nblocks = (ntiles + kDenseWaves - 1) / kDenseWaves;
  const dim3 grid((uint32_t)nblocks), block(64 * kDenseWaves);
  switch (d.mode) {
    case kModeBuffer:
      hipLaunchKernelGGL((static_dense_kernel<T, ProdBuffer<T>>), grid, block, 0, s, S, d.n_threads, nblocks,
                         ProdBuffer<T>{static_cast<const T*>(d.values), nullptr});
      break;
    case kModeRoundTag:
      hipLaunchKernelGGL((static_dense_kernel<T, ProdRoundTag<T>>), grid, block, 0, s, S, d.n_threads, nblocks,
                         ProdRoundTag<T>{d.round, d.tag_shift});
      break;
    case kModeKeyed:
      hipLaunchKernelGGL((static_dense_kernel<T, ProdKeyed<T>>), grid, block, 0, s, S, d.n_threads, nblocks,
                         ProdKeyed<T>{d.seed, d.round, d.tag_shift, d.tag});
      break;
    default:
      return GGA_EINVAL;
  }
  return hip_status(hipGetLastError());
}

int launch_static_insert(gga_static* st, const InsertDesc& d, hipStream_t s) {
  st->rw_last = false;
  if (d.n_threads == 0) return GGA_OK;
  static_grow_bound(st, d.n_threads, multi_mode(d.mode) ? d.max_count : 1u);
  const uint64_t tile = multi_mode(d.mode) ? kCountTile : kFlagTile;
  const uint64_t ntiles = (d.n_threads + tile - 1) / tile;
  if (ntiles > 0x7FFFFFFFull) return GGA_EINVAL;
  const bool dense = d.mode == kModeRoundTag || d.mode == kModeKeyed || (d.mode == kModeBuffer && !d.flags);
  if (dense) {
    StaticRef S{st->data, st->cap, st->d_size, st->d_err, st->d_done};
    return st->elem_bytes == 4 ? launch_static_dense<uint32_t>(S, d, ntiles, s)
                               : launch_static_dense<uint64_t>(S, d, ntiles, s);
  }
  TileArgs I{};
  I.n_threads = d.n_threads;
  I.elem_log2 = st->elem_bytes == 4 ? 2u : 3u;
  StaticRef S{st->data, st->cap, st->d_size, st->d_err, st->d_done};
  ArrRef A{};
  const int rc = st->elem_bytes == 4 ? dispatch<uint32_t, true>(A, S, I, d, ntiles, s)
                                     : dispatch<uint64_t, true>(A, S, I, d, ntiles, s);
  return rc;
}


namespace {
}  // namespace

int prepare_round_item(ggarray* a, uint64_t n, uint64_t tag, uint32_t index, BatchArr* item, uint64_t* ntiles,
                       hipStream_t s, bool lookback) {
  const uint64_t chunk = n ? (n + a->V - 1) / a->V : 0;
  const uint64_t tpv = n ? (chunk + kFlagTile - 1) / kFlagTile : 0;
  *ntiles = tpv * a->V;
  if (chunk >= (1ull << 32)) return GGA_EINVAL;
  if (lookback && tpv > 1) {
    const int rc = ensure_status(a, *ntiles, s);
    if (rc) return rc;
  }
  *item = BatchArr{a->ref, n, chunk, tpv, tag, index, a->elem_log2};
  return GGA_OK;
}

int launch_serve_front(const BatchArr* items, const uint64_t* begins, uint32_t n_a, uint64_t blocks,
                       const ServeItem* sitems, uint32_t n_s, uint32_t elem_bytes, uint64_t seed, uint32_t round,
                       uint32_t shift, hipStream_t s) {
  const uint64_t waves = blocks + n_s;
  if (!waves) return GGA_OK;
  if (waves > 0x7FFFFFFFull) return GGA_EINVAL;
  const uint32_t te_log2 = elem_bytes == 4 ? 12u : 11u;
  const dim3 grid((uint32_t)waves), block(64);
  if (elem_bytes == 4)
    hipLaunchKernelGGL(serve_front_kernel<uint32_t>, grid, block, 0, s, items, begins, n_a, blocks, sitems, te_log2,
                       ProdKeyed<uint32_t>{seed, round, shift, 0});
  else
    hipLaunchKernelGGL(serve_front_kernel<uint64_t>, grid, block, 0, s, items, begins, n_a, blocks, sitems, te_log2,
                       ProdKeyed<uint64_t>{seed, round, shift, 0});
  return hip_status(hipGetLastError());
}

int launch_batch_insert(gga_batch* b, const InsertDesc& d, const uint64_t* n_threads, hipStream_t s) {
  if (d.mode != kModeRoundTag && d.mode != kModeBernoulli && d.mode != kModeKeyed) return GGA_EINVAL;
  const bool dense = d.mode != kModeBernoulli;  // every thread inserts: grow, then store
  BatchArr* items = new (std::nothrow) BatchArr[b->n];
  uint64_t* begins = new (std::nothrow) uint64_t[b->n + 1];
  if (!items || !begins) {
    delete[] items;
    delete[] begins;
    return GGA_EHIP;
  }
  int rc = GGA_OK;
  uint64_t blocks = 0;
  uint64_t max_tpv = 0;
  bool grew = false;
  for (uint32_t i = 0; i < b->n && rc == GGA_OK; ++i) {
    uint64_t ntiles = 0;
    const uint64_t* before = b->arrays[i]->ref.status;
    rc = prepare_round_item(b->arrays[i], n_threads[i], d.tag + i, i, &items[i], &ntiles, s, !dense);
    if (rc == GGA_OK && n_threads[i] && items[i].tpv > max_tpv) max_tpv = items[i].tpv;
    grow_bound(b->arrays[i], n_threads[i]);
    grew = grew || b->arrays[i]->ref.status != before;
    if (rc == GGA_OK && blocks + ntiles > 0x7FFFFFFFull) rc = GGA_EINVAL;
    begins[i] = blocks;
    blocks += ntiles;
  }
  begins[b->n] = blocks;
  // A table is keyed by the round's shape, without the look-back buffers; when an
  // array's buffer moves (it grew), every cached table is patched and uploaded
  // again now, so that a later capture of a known shape uploads nothing.
  for (uint32_t k = 0; grew && rc == GGA_OK && k < b->n_tables; ++k) {
    gga_batch::Table& t = b->tables[k];
    for (uint32_t i = 0; i < b->n; ++i) t.host[i].A.status = b->arrays[i]->ref.status;
    if (hipMemcpyAsync(t.items, t.host, sizeof(BatchArr) * b->n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = GGA_EHIP;
  }
  gga_batch::Table* tab = nullptr;
  if (rc == GGA_OK && blocks) {
    uint64_t key = 0xCBF29CE484222325ull;
    for (uint32_t i = 0; i < b->n; ++i) {
      BatchArr shape = items[i];
      shape.A.status = nullptr;
      key = fnv1a(&shape, sizeof(BatchArr), key);
    }
    key = fnv1a(begins, sizeof(uint64_t) * (b->n + 1), key);
    for (uint32_t k = 0; k < b->n_tables; ++k)
      if (b->tables[k].key == key) tab = &b->tables[k];
    if (!tab) {  // first time this round shape is seen: upload its table
      if (b->n_tables == b->cap_tables) {
        const uint32_t ncap = b->cap_tables ? 2 * b->cap_tables : 8;
        gga_batch::Table* nt = new (std::nothrow) gga_batch::Table[ncap];
        if (!nt) rc = GGA_EHIP;
        else {
          for (uint32_t k = 0; k < b->n_tables; ++k) nt[k] = b->tables[k];
          delete[] b->tables;
          b->tables = nt;
          b->cap_tables = ncap;
        }
      }
      if (rc == GGA_OK) {
        gga_batch::Table t{key, blocks, nullptr, nullptr, new (std::nothrow) BatchArr[b->n]};
        if (!t.host || hipMalloc(&t.items, sizeof(BatchArr) * b->n) != hipSuccess ||
            hipMalloc(&t.begins, sizeof(uint64_t) * (b->n + 1)) != hipSuccess ||
            hipMemcpyAsync(t.items, items, sizeof(BatchArr) * b->n, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(t.begins, begins, sizeof(uint64_t) * (b->n + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
          if (t.items) (void)hipFree(t.items);
          if (t.begins) (void)hipFree(t.begins);
          delete[] t.host;
          rc = GGA_EHIP;
        } else {
          for (uint32_t i = 0; i < b->n; ++i) t.host[i] = items[i];
          b->tables[b->n_tables++] = t;
          tab = &b->tables[b->n_tables - 1];
        }
      }
    }
  }
  delete[] items;
  delete[] begins;
  if (rc != GGA_OK || !blocks) return rc;
  const dim3 grid((uint32_t)blocks), block(64);
  const bool u32 = b->elem_bytes == 4;
  if (dense && (max_tpv <= 8 || b->total_vectors >= 512)) {  // one wave per LFVector, as for one array
    const dim3 vgrid((uint32_t)((b->total_vectors + 3) / 4)), vblock(256);
    if (d.mode == kModeRoundTag) {
      if (u32) hipLaunchKernelGGL((batch_grow_store_kernel<uint32_t, ProdRoundTag<uint32_t>>), vgrid, vblock, 0, s, tab->items, b->d_vbegin, b->n, ProdRoundTag<uint32_t>{d.round, d.tag_shift});
      else hipLaunchKernelGGL((batch_grow_store_kernel<uint64_t, ProdRoundTag<uint64_t>>), vgrid, vblock, 0, s, tab->items, b->d_vbegin, b->n, ProdRoundTag<uint64_t>{d.round, d.tag_shift});
    } else {
      if (u32) hipLaunchKernelGGL((batch_grow_store_kernel<uint32_t, ProdKeyed<uint32_t>>), vgrid, vblock, 0, s, tab->items, b->d_vbegin, b->n, ProdKeyed<uint32_t>{d.seed, d.round, d.tag_shift, 0});
      else hipLaunchKernelGGL((batch_grow_store_kernel<uint64_t, ProdKeyed<uint64_t>>), vgrid, vblock, 0, s, tab->items, b->d_vbegin, b->n, ProdKeyed<uint64_t>{d.seed, d.round, d.tag_shift, 0});
    }
  } else if (dense) {
    hipLaunchKernelGGL(batch_grow_kernel, dim3((uint32_t)((b->total_vectors + 3) / 4)), dim3(256), 0, s, tab->items,
                       b->d_vbegin, b->n);
    if (d.mode == kModeRoundTag) {
      if (u32) hipLaunchKernelGGL((batch_dense_kernel<uint32_t, ProdRoundTag<uint32_t>>), grid, block, 0, s, tab->items, tab->begins, b->n, ProdRoundTag<uint32_t>{d.round, d.tag_shift});
      else hipLaunchKernelGGL((batch_dense_kernel<uint64_t, ProdRoundTag<uint64_t>>), grid, block, 0, s, tab->items, tab->begins, b->n, ProdRoundTag<uint64_t>{d.round, d.tag_shift});
    } else {
      if (u32) hipLaunchKernelGGL((batch_dense_kernel<uint32_t, ProdKeyed<uint32_t>>), grid, block, 0, s, tab->items, tab->begins, b->n, ProdKeyed<uint32_t>{d.seed, d.round, d.tag_shift, 0});
      else hipLaunchKernelGGL((batch_dense_kernel<uint64_t, ProdKeyed<uint64_t>>), grid, block, 0, s, tab->items, tab->begins, b->n, ProdKeyed<uint64_t>{d.seed, d.round, d.tag_shift, 0});
    }
  } else if (d.mode == kModeRoundTag) {
    if (u32) hipLaunchKernelGGL((batch_insert_kernel<uint32_t, ProdRoundTag<uint32_t>>), grid, block, 0, s, tab->items, tab->begins, b->n, ProdRoundTag<uint32_t>{d.round, d.tag_shift});
    else hipLaunchKernelGGL((batch_insert_kernel<uint64_t, ProdRoundTag<uint64_t>>), grid, block, 0, s, tab->items, tab->begins, b->n, ProdRoundTag<uint64_t>{d.round, d.tag_shift});
  } else if (d.mode == kModeBernoulli) {
    if (u32) hipLaunchKernelGGL((batch_insert_kernel<uint32_t, ProdBernoulli<uint32_t>>), grid, block, 0, s, tab->items, tab->begins, b->n, ProdBernoulli<uint32_t>{d.seed, d.round});
    else hipLaunchKernelGGL((batch_insert_kernel<uint64_t, ProdBernoulli<uint64_t>>), grid, block, 0, s, tab->items, tab->begins, b->n, ProdBernoulli<uint64_t>{d.seed, d.round});
  } else {
    if (u32) hipLaunchKernelGGL((batch_insert_kernel<uint32_t, ProdKeyed<uint32_t>>), grid, block, 0, s, tab->items, tab->begins, b->n, ProdKeyed<uint32_t>{d.seed, d.round, d.tag_shift, 0});
    else hipLaunchKernelGGL((batch_insert_kernel<uint64_t, ProdKeyed<uint64_t>>), grid, block, 0, s, tab->items, tab->begins, b->n, ProdKeyed<uint64_t>{d.seed, d.round, d.tag_shift, 0});
  }
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    for (uint32_t i = 0; i < b->n; ++i) sizes_changed(b->arrays[i], s);
  return hip_status(e);
}

}  // namespace gga
