// A whole step of a batch in one persistent launch: insertion rounds, r/w and
// flatten of every array.
//
// LFVectors are independent (Sec. IV: each is grown by its own block, and no
// operation but the size prefix looks across them), so one workgroup can take an
// LFVector through all of its insertion rounds and its r/w without waiting for
// anyone: it reads the LFVector's size and bucket table once, runs each round's
// tiles of 1024 candidates in order (Sec. III-B's block prefix sum over the
// tile, one index range claimed per tile, buckets allocated by the workgroup
// itself as Alg. 1 and 2 do), and applies the r/w to the elements it has just
// written, which are still in the cache.  Workgroup w takes LFVectors w, w + G,
// ... of the batch (arrays in order, each array's LFVectors in order).
//
// The flatten needs the exclusive prefix of every LFVector's size (each final
// size is also written to a flat per-LFVector array), so grid-wide barriers
// follow: after the first, chunks of consecutive LFVectors are summed; after the
// second, each workgroup scans the chunk totals and copies its own LFVectors to
// their places.  With at most 1024 LFVectors a chunk is one LFVector and the
// second barrier is not needed.  A workgroup copies the LFVectors it
// wrote itself, so element data never crosses workgroups; the sizes and the
// chunk totals do, through device-scope atomic loads and stores.  The grid is no
// larger than what the device holds at once (an occupancy query), and the
// launch is cooperative, so every workgroup reaches the barriers; every wait is
// still bounded.
#include <hip/hip_cooperative_groups.h>

#include "gga_internal.h"
#include "producers.h"

namespace gga {
namespace {

constexpr uint32_t kSB = 256;            // threads per workgroup
constexpr uint32_t kSW = kSB / 64;       // waves per workgroup
constexpr uint32_t kSSlots = 4;          // candidates per thread and tile
constexpr uint32_t kSTile = kSB * kSSlots;

__device__ __forceinline__ uint32_t s_lane() { return threadIdx.x & 63u; }
__device__ __forceinline__ uint32_t s_mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

struct StepShared {
  uint64_t bp[kMaxBuckets];   // the LFVector's bucket pointers
  uint64_t reused;            // buckets below keep_hi that the rounds have taken again
  uint32_t keep_hi;           // with a clear: buckets [0, keep_hi) held from before it
  uint64_t size;
  uint32_t cnt[kSSlots * kSW];
  uint32_t fail;
  uint32_t dead;
  uint64_t red[kSW];
};

// One round on LFVector v: logical threads c0 .. c0 + cnt - 1 of the round, in
// tiles of 1024 (slot j of thread t is logical thread t0 + 256 j + t, so the
// order (slot, wave, lane) is the logical order).  Returns false if a bucket
// could not be allocated; the caller then restores the size the round started
// from and freezes the LFVector.
// Wave 0 allocates the buckets whose first index lies in [s, s + n) (one per
// lane) into the LFVector's table and sh.bp; sh.fail says whether any failed.
// After a clear in the same launch, a bucket the LFVector held before it is taken
// again in place (pool_reuse) instead of from the pool.
__device__ void step_alloc(const ArrRef& A, uint32_t v, uint32_t elem_log2, uint64_t s, uint64_t n,
                           StepShared& sh) {
  const uint32_t lane = s_lane();
  if (threadIdx.x >= 64) return;
  const uint32_t log2F = A.log2F;
  const uint32_t lo = nbuckets_for(log2F, s), hi = nbuckets_for(log2F, s + n);
  const uint32_t b = lo + lane;
  bool failed = false, reuse = false;
  if (b < hi) {
    if (b >= (uint32_t)kMaxBuckets) {
      failed = true;
    } else if (b < sh.keep_hi) {
      reuse = pool_reuse(A.pool, pool_shard(v, b, A.salt));
      failed = !reuse;
    } else {
      uint8_t* q = pool_alloc(A.pool, bucket_class(log2F, elem_log2, b), pool_shard(v, b, A.salt));
      const uint64_t p = q ? (uint64_t)q : kFailedPtr;
      A.bptr[(uint64_t)v * kMaxBuckets + b] = p;
      sh.bp[b] = p;
      failed = !q;
    }
  }
  // Both ballots are taken by the whole wave (a ballot under `lane == 0` would see
  // lane 0 alone); bit l of the reuse ballot is bucket lo + l.
  const uint64_t rm = __ballot(reuse);
  const uint64_t fm = __ballot(failed);
  if (lane == 0) {
    sh.fail = fm ? 1u : 0u;
    sh.reused |= rm << lo;
  }
}

// The clear ahead of a step's rounds, for one LFVector: a frozen LFVector gives
// back every bucket it holds (as shrink does), any other keeps its buckets
// [0, keep_hi) for the rounds to take again.  `lane` is the caller's lane in the
// wave that does it.
__device__ __forceinline__ uint32_t step_clear(const ArrRef& A, uint32_t v, uint32_t elem_log2, uint32_t lane,
                                               uint64_t size, bool dead) {
  if (dead) {
    release_bucket(A, v, lane, 0, kMaxBuckets, false, 0, elem_log2);
    return 0;
  }
  return nbuckets_for(A.log2F, size);
}

// After the rounds: the clear's release of the held buckets [0, keep_hi) the
// rounds did not take again (nothing of this launch was written to them, so no
// fence is needed before they go back).
__device__ __forceinline__ void step_release_unused(const ArrRef& A, uint32_t v, uint32_t elem_log2, uint32_t lane,
                                                    uint32_t keep_hi, uint64_t reused, uint64_t& bp) {
  if (lane < keep_hi && !((reused >> lane) & 1u)) {
    if (bp > kFailedPtr)
      pool_free(A.pool, reinterpret_cast<uint8_t*>(bp), bucket_class(A.log2F, elem_log2, lane),
                pool_shard(v, lane, A.salt));
    A.bptr[(uint64_t)v * kMaxBuckets + lane] = 0;
    bp = 0;
  }
}

// A round in which every logical thread inserts (round-tag, keyed): element i
// of the round lands at s + i, so the round's buckets are allocated at once and
// each bucket run is written with whole 16-byte vectors, no scan needed.
template <typename T, class Prod>
__device__ bool step_round_dense(const ArrRef& A, uint32_t v, uint32_t elem_log2, uint64_t c0, uint64_t cnt,
                                 const Prod& prod, StepShared& sh) {
  constexpr uint32_t VPL = 16 / sizeof(T);
  const uint32_t tid = threadIdx.x;
  const uint32_t log2F = A.log2F;
  const uint64_t s = sh.size;
  step_alloc(A, v, elem_log2, s, cnt, sh);
  __syncthreads();
  if (sh.fail) return false;
  for (uint64_t i = 0; i < cnt;) {  // one run per bucket
    const uint64_t idx = s + i;
    const uint32_t b = bucket_of(log2F, idx);
    const uint64_t bs = bucket_start(log2F, b);
    const uint64_t room = bs + bucket_len(log2F, b) - idx;
    const uint64_t run = cnt - i < room ? cnt - i : room;
    const gptr<T> dst = gmem(reinterpret_cast<T*>(sh.bp[b]) + (idx - bs));
    // head up to a 16-byte boundary (buckets are 256-byte aligned), vectors, tail
    const uint32_t mis = (uint32_t)((idx - bs) & (VPL - 1));
    uint32_t head = mis ? VPL - mis : 0u;
    if (head > run) head = (uint32_t)run;
    if (tid < head) dst[tid] = prod.value(c0 + i + tid);
    const uint64_t nv = (run - head) / VPL;
    for (uint64_t q = tid; q < nv; q += kSB) {
      T t[VPL];
#pragma unroll
      for (uint32_t k = 0; k < VPL; ++k) t[k] = prod.value(c0 + i + head + q * VPL + k);
      u32x4 x;
      __builtin_memcpy(&x, t, 16);
      *reinterpret_cast<gptr<u32x4>>(dst + head + q * VPL) = x;
    }
    const uint64_t tail = head + nv * VPL + tid;
    if (tail < run) dst[tail] = prod.value(c0 + i + tail);
    i += run;
  }
  __syncthreads();  // every thread has read sh.size
  if (tid == 0) sh.size = s + cnt;
  __syncthreads();
  return true;
}

template <typename T, class Prod>
__device__ bool step_round(const ArrRef& A, uint32_t v, uint32_t elem_log2, uint64_t c0, uint64_t cnt,
                           const Prod& prod, StepShared& sh) {
  if constexpr (Prod::kDense) return step_round_dense<T>(A, v, elem_log2, c0, cnt, prod, sh);
  const uint32_t tid = threadIdx.x, lane = s_lane(), w = tid >> 6;
  const uint32_t log2F = A.log2F;
  uint64_t s = sh.size;
  for (uint64_t t0 = 0; t0 < cnt; t0 += kSTile) {
    T val[kSSlots];
    uint32_t rank[kSSlots];
    uint32_t fl = 0;
#pragma unroll
    for (uint32_t j = 0; j < kSSlots; ++j) {
      const uint64_t local = t0 + (uint64_t)j * kSB + tid;
      val[j] = 0;
      if (local < cnt && prod.take(c0 + local, val[j])) fl |= 1u << j;
      const uint64_t m = __ballot((fl >> j) & 1u);
      rank[j] = s_mbcnt(m);
      if (lane == 0) sh.cnt[j * kSW + w] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    uint32_t total = 0;
    uint32_t before[kSSlots];
#pragma unroll
    for (uint32_t j = 0; j < kSSlots; ++j) {
      before[j] = total;
      for (uint32_t q = 0; q < kSW; ++q) {
        const uint32_t c = sh.cnt[j * kSW + q];
        before[j] += q < w ? c : 0u;
        total += c;
      }
    }
    // Buckets whose first index this tile writes: allocated by wave 0, one per lane.
    step_alloc(A, v, elem_log2, s, total, sh);
    __syncthreads();
    if (sh.fail) return false;
#pragma unroll
    for (uint32_t j = 0; j < kSSlots; ++j) {
      if ((fl >> j) & 1u) {
        const uint64_t idx = s + before[j] + rank[j];
        const uint32_t b = bucket_of(log2F, idx);
        gmem(reinterpret_cast<T*>(sh.bp[b]))[offset_in(log2F, idx, b)] = val[j];
      }
    }
    s += total;
    __syncthreads();  // sh.cnt is rewritten by the next tile
  }
  sh.size = s;
  return true;
}

// x = op(x) over the live elements of LFVector v (sh.bp, sh.size current).
template <typename T>
__device__ void step_rw(uint32_t log2F, uint32_t op, const StepShared& sh) {
  constexpr uint32_t VPL = 16 / sizeof(T);
  const uint64_t s = sh.size;
  for (uint32_t b = 0; b < (uint32_t)kMaxBuckets && bucket_start(log2F, b) < s; ++b) {
    const uint64_t st = bucket_start(log2F, b);
    const uint64_t len = bucket_len(log2F, b);
    const uint32_t live = (uint32_t)(s - st < len ? s - st : len);
    const gptr<T> p = gmem(reinterpret_cast<T*>(sh.bp[b]));  // 256-byte aligned
    const uint32_t nv = live / VPL;
    for (uint32_t q = threadIdx.x; q < nv; q += kSB) {
      const gptr<u32x4> a = reinterpret_cast<gptr<u32x4>>(p + (uint64_t)q * VPL);
      *a = op_vec<T>(op, *a);
    }
    const uint32_t e = nv * VPL + threadIdx.x;
    if (e < live) p[e] = apply_op<T>(op, p[e]);
  }
}

// n elements from src to dst by the workgroup: stores aligned to dst's 128-byte
// lines, loads taking src's alignment.
template <typename T>
__device__ void step_copy(T* dst_, const T* src_, uint32_t n) {
  typedef u32x4 u32x4_a4 __attribute__((aligned(4)));
  constexpr uint32_t VPL = 16 / sizeof(T), kLine = 128 / sizeof(T);
  const uint32_t tid = threadIdx.x;
  const gptr<T> dst = gmem(dst_);
  const gptr<const T> src = gmem(src_);
  const uint32_t mis = (uint32_t)((reinterpret_cast<uintptr_t>(dst_) & 127u) / sizeof(T));
  uint32_t head = mis ? kLine - mis : 0u;
  if (head > n) head = n;
  if (tid < head) __builtin_nontemporal_store(src[tid], dst + tid);
  const uint32_t nv = (n - head) / VPL;
  for (uint32_t q = tid; q < nv; q += kSB) {
    const u32x4 x = *reinterpret_cast<gptr<const u32x4_a4>>(src + head + q * VPL);
    __builtin_nontemporal_store(x, reinterpret_cast<gptr<u32x4>>(dst + head + q * VPL));
  }
  const uint32_t tail = head + nv * VPL + tid;
  if (tail < n) __builtin_nontemporal_store(src[tail], dst + tail);
}

// Grid-wide barrier: arrival after every earlier store of the workgroup has
// completed (the workgroup barrier waits for them, and the stores that other
// workgroups read are device-scope), then a bounded wait for all G arrivals.
__device__ void step_barrier(uint32_t* ctr, uint32_t G, uint32_t spin, uint32_t* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // waits for the wave's stores to complete
    fetch_add32(ctr, 1u);
    for (uint32_t n = 0; ld_rlx32(ctr) < G; ++n) {
      if (n >= spin) {
        set_error(err, kErrStall);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
}

// Block-wide sum of one value per thread.
__device__ uint64_t step_block_sum(uint64_t x, StepShared& sh) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  __syncthreads();
  if (s_lane() == 0) sh.red[threadIdx.x >> 6] = x;
  __syncthreads();
  uint64_t t = 0;
  for (uint32_t q = 0; q < kSW; ++q) t += sh.red[q];
  return t;
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kSB) void step_kernel(const BatchArr* arrs, const uint32_t* varr, const uint64_t* vbegin,
                                                   uint64_t total_v, StepDesc D, const uint64_t* counts, uint32_t n_arr,
                                                   uint32_t op, T* out, uint64_t out_cap, uint32_t* sync,
                                                   uint64_t* chunk_sum, uint64_t chunk_len, uint32_t* berr,
                                                   uint32_t spin, uint64_t* vsize) {
  __shared__ StepShared sh;
  __shared__ uint64_t cpre[kStepChunkMax];
  const uint32_t tid = threadIdx.x;
  const uint32_t G = gridDim.x;

  // Phase A: rounds and r/w, LFVector by LFVector.
  for (uint64_t wv = blockIdx.x; wv < total_v; wv += G) {
    const uint32_t i = varr[wv];
    const ArrRef A = arrs[i].A;
    const uint32_t elem_log2 = arrs[i].elem_log2;
    const uint32_t v = (uint32_t)(wv - vbegin[i]);
    if (tid < (uint32_t)kMaxBuckets) sh.bp[tid] = A.bptr[(uint64_t)v * kMaxBuckets + tid];
    if (tid == 0) {
      sh.size = A.size[v];
      sh.dead = A.dead[v];
      sh.keep_hi = 0;
      sh.reused = 0;
    }
    __syncthreads();
    bool changed = false;
    if (D.clear) {
      const uint64_t s_old = sh.size;
      const bool was_dead = sh.dead != 0;
      __syncthreads();  // every thread has read the old size
      if (tid < 64) {
        const uint32_t kh = step_clear(A, v, elem_log2, tid, s_old, was_dead);
        if (tid == 0) {
          sh.keep_hi = kh;
          sh.size = 0;
        }
      }
      __syncthreads();
      changed = true;
    }
    for (uint32_t r = 0; r < D.n_rounds && !sh.dead; ++r) {
      const uint64_t nthr = counts[(uint64_t)r * n_arr + i];
      const uint64_t chunk = (nthr + A.V - 1) / A.V;
      const uint64_t c0 = (uint64_t)v * chunk;
      const uint64_t cnt = c0 < nthr ? (nthr - c0 < chunk ? nthr - c0 : chunk) : 0;
      if (cnt == 0) continue;
      const StepRound& R = D.r[r];
      const uint64_t s_round = sh.size;
      bool ok;
      if (R.kind == kModeBernoulli)
        ok = step_round<T>(A, v, elem_log2, c0, cnt, ProdBernoulli<T>{R.seed, R.round}, sh);
      else if (R.kind == kModeRoundTag)
        ok = step_round<T>(A, v, elem_log2, c0, cnt, ProdRoundTag<T>{R.round, R.tag_shift}, sh);
      else
        ok = step_round<T>(A, v, elem_log2, c0, cnt, ProdKeyed<T>{R.seed, R.round, R.tag_shift, R.tag + i}, sh);
      changed = true;
      if (!ok) {  // the round is dropped and the LFVector frozen, as in the per-round calls
        if (tid == 0) {
          sh.size = s_round;
          sh.dead = 1;
          A.dead[v] = 1u;
          set_error(A.err, kErrNoMem);
        }
        __syncthreads();
      }
    }
    if (D.clear) {
      __syncthreads();  // the rounds' bucket bookkeeping is complete
      if (tid < 64) {
        uint64_t bp = tid < (uint32_t)kMaxBuckets ? sh.bp[tid] : 0;
        step_release_unused(A, v, elem_log2, tid, sh.keep_hi, sh.reused, bp);
        if (tid < (uint32_t)kMaxBuckets) sh.bp[tid] = bp;
      }
      __syncthreads();
    }
    if (changed && tid == 0) st_rlx(&A.size[v], sh.size);
    if (tid == 0) st_rlx(&vsize[wv], sh.size);
    if (op != kOpNone) step_rw<T>(A.log2F, op, sh);
    __syncthreads();  // sh is reloaded for the next LFVector
  }

  if (out) {
    // Phase B: totals of chunks of chunk_len consecutive LFVectors (with at most
    // kStepChunkMax LFVectors a chunk is one LFVector: its size is the total).
    step_barrier(&sync[0], G, spin, berr);
    const uint64_t nchunks = (total_v + chunk_len - 1) / chunk_len;
    const uint64_t* ctot = chunk_len == 1 ? vsize : chunk_sum;
    if (chunk_len > 1) {
      for (uint64_t c = blockIdx.x; c < nchunks; c += G) {
        uint64_t x = 0;
        for (uint64_t wv = c * chunk_len + tid; wv < total_v && wv < (c + 1) * chunk_len; wv += kSB)
          x += ld_rlx(&vsize[wv]);
        x = step_block_sum(x, sh);
        if (tid == 0) st_rlx(&chunk_sum[c], x);
      }
      step_barrier(&sync[1], G, spin, berr);
    }

    // Phase C: every workgroup scans the chunk totals (nchunks <= kStepChunkMax:
    // four per thread), then copies its own LFVectors to their places.
    constexpr uint32_t kPer = kStepChunkMax / kSB;
    uint64_t x[kPer], sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
      const uint64_t c = (uint64_t)tid * kPer + k;
      x[k] = c < nchunks ? ld_rlx(&ctot[c]) : 0;
      sum += x[k];
    }
    uint64_t incl = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(incl, d, 64);
      if (s_lane() >= (uint32_t)d) incl += y;
    }
    if (s_lane() == 63) sh.red[tid >> 6] = incl;
    __syncthreads();
    uint64_t run = incl - sum, total = 0;
    for (uint32_t q = 0; q < kSW; ++q) {
      run += q < (tid >> 6) ? sh.red[q] : 0;
      total += sh.red[q];
    }
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
      cpre[tid * kPer + k] = run;
      run += x[k];
    }
    __syncthreads();
    if (total > out_cap) {
      if (blockIdx.x == 0 && tid == 0) set_error(berr, kErrRange);
    } else {
      for (uint64_t wv = blockIdx.x; wv < total_v; wv += G) {
        const uint32_t i = varr[wv];
        const ArrRef& A = arrs[i].A;
        const uint32_t v = (uint32_t)(wv - vbegin[i]);
        // the chunk's prefix plus the LFVectors of the chunk before this one
        const uint64_t c = wv / chunk_len;
        uint64_t y = 0;
        for (uint64_t u = c * chunk_len + tid; u < wv; u += kSB) y += ld_rlx(&vsize[u]);
        const uint64_t off = cpre[c] + (chunk_len > 1 ? step_block_sum(y, sh) : 0);
        const uint64_t sz = ld_rlx(&vsize[wv]);
        T* dst = out + off;
        for (uint32_t b = 0; b < (uint32_t)kMaxBuckets && bucket_start(A.log2F, b) < sz; ++b) {
          const uint64_t st = bucket_start(A.log2F, b);
          const uint64_t len = bucket_len(A.log2F, b);
          const uint32_t live = (uint32_t)(sz - st < len ? sz - st : len);
          step_copy<T>(dst + st, reinterpret_cast<const T*>(A.bptr[(uint64_t)v * kMaxBuckets + b]), live);
        }
      }
    }
  }

  // The last workgroup out clears the barrier words for the next launch.
  __syncthreads();
  if (tid == 0 && fetch_add32(&sync[2], 1u) == G - 1) {
    st_rlx32(&sync[0], 0u);
    st_rlx32(&sync[1], 0u);
    st_rlx32(&sync[2], 0u);
  }
}

// ------------------------------------------------- one wave per LFVector --
// For batches of many LFVectors each wave takes its own LFVectors (wave gw takes
// gw, gw + W, ..., W the grid's waves) through the rounds, the r/w and the
// flatten, wave-synchronously: four LFVectors per workgroup are in flight at
// once, so the allocation and pointer latencies of one are hidden by the others.
// Lane b holds bucket b's pointer.  Final sizes also go to a flat array (vsize),
// so the flatten's prefix reads contiguous words.
namespace {

// Wave 0 .. 63: allocate buckets [nbuckets(s), nbuckets(s + n)) (lane b: bucket
// b), keeping the pointer in the lane; a bucket below keep_hi (held from before
// the step's clear) is taken again in place.  False if any allocation failed.
__device__ bool wave_alloc(const ArrRef& A, uint32_t v, uint32_t elem_log2, uint64_t s, uint64_t n, uint64_t& bp,
                           uint32_t keep_hi, uint64_t& reused) {
  const uint32_t lane = s_lane(), log2F = A.log2F;
  const uint32_t lo = nbuckets_for(log2F, s), hi = nbuckets_for(log2F, s + n);
  bool failed = false, reuse = false;
  if (lane >= lo && lane < hi) {
    if (lane >= (uint32_t)kMaxBuckets) {
      failed = true;
    } else if (lane < keep_hi) {
      reuse = pool_reuse(A.pool, pool_shard(v, lane, A.salt));
      failed = !reuse;
    } else {
      uint8_t* q = pool_alloc(A.pool, bucket_class(log2F, elem_log2, lane), pool_shard(v, lane, A.salt));
      bp = q ? (uint64_t)q : kFailedPtr;
      A.bptr[(uint64_t)v * kMaxBuckets + lane] = bp;
      failed = !q;
    }
  }
  reused |= __ballot(reuse);
  return __ballot(failed) == 0;
}

// A round of LFVector v by one wave.  Dense producers (every thread inserts):
// buckets for the whole round at once, then 16-byte vector stores per bucket
// run.  Others: 1024 candidates at a time (16 per lane, slot j of lane l is
// candidate t0 + 64 j + l), positions from the slot ballots.
template <typename T, class Prod>
__device__ bool wave_round(const ArrRef& A, uint32_t v, uint32_t elem_log2, uint64_t c0, uint64_t cnt,
                           const Prod& prod, uint64_t& bp, uint64_t& s, uint32_t keep_hi, uint64_t& reused) {
  constexpr uint32_t VPL = 16 / sizeof(T);
  const uint32_t lane = s_lane(), log2F = A.log2F;
  if constexpr (Prod::kDense) {
    if (!wave_alloc(A, v, elem_log2, s, cnt, bp, keep_hi, reused)) return false;
    for (uint64_t i = 0; i < cnt;) {
      const uint64_t idx = s + i;
      const uint32_t b = bucket_of(log2F, idx);
      const uint64_t bs = bucket_start(log2F, b);
      const uint64_t room = bs + bucket_len(log2F, b) - idx;
      const uint64_t run = cnt - i < room ? cnt - i : room;
      const gptr<T> dst = gmem(reinterpret_cast<T*>(__shfl(bp, (int)b, 64)) + (idx - bs));
      const uint32_t mis = (uint32_t)((idx - bs) & (VPL - 1));
      uint32_t head = mis ? VPL - mis : 0u;
      if (head > run) head = (uint32_t)run;
      if (lane < head) dst[lane] = prod.value(c0 + i + lane);
      const uint64_t nv = (run - head) / VPL;
      for (uint64_t q = lane; q < nv; q += 64) {
        T t[VPL];
#pragma unroll
        for (uint32_t k = 0; k < VPL; ++k) t[k] = prod.value(c0 + i + head + q * VPL + k);
        u32x4 x;
        __builtin_memcpy(&x, t, 16);
        *reinterpret_cast<gptr<u32x4>>(dst + head + q * VPL) = x;
      }
      const uint64_t tail = head + nv * VPL + lane;
      if (tail < run) dst[tail] = prod.value(c0 + i + tail);
      i += run;
    }
    s += cnt;
    return true;
  } else {
    constexpr uint32_t kSlots = 16;
    for (uint64_t t0 = 0; t0 < cnt; t0 += 64 * kSlots) {
      T val[kSlots];
      uint64_t m[kSlots];
      uint32_t total = 0;
#pragma unroll
      for (uint32_t j = 0; j < kSlots; ++j) {
        const uint64_t local = t0 + 64u * j + lane;
        val[j] = 0;
        const bool f = local < cnt && prod.take(c0 + local, val[j]);
        m[j] = __ballot(f);
        total += (uint32_t)__popcll(m[j]);
      }
      if (!wave_alloc(A, v, elem_log2, s, total, bp, keep_hi, reused)) return false;
      uint64_t run = s;
#pragma unroll
      for (uint32_t j = 0; j < kSlots; ++j) {
        const bool f = (m[j] >> lane) & 1u;
        const uint64_t idx = run + s_mbcnt(m[j]);
        const uint32_t b = f ? bucket_of(log2F, idx) : 0u;
        const uint64_t p = __shfl(bp, (int)b, 64);
        if (f) gmem(reinterpret_cast<T*>(p))[offset_in(log2F, idx, b)] = val[j];
        run += (uint32_t)__popcll(m[j]);
      }
      s += total;
    }
    return true;
  }
}

// x = op(x) over the s live elements (lane b: bucket b's pointer), eight
// vectors per lane in flight (unconditional loads, clamped indices; only the
// lane that owns a vector stores it).
template <typename T>
__device__ void wave_rw(uint32_t log2F, uint32_t op, uint64_t bp, uint64_t s) {
  constexpr uint32_t VPL = 16 / sizeof(T), kU = 8;
  const uint32_t lane = s_lane();
  for (uint32_t b = 0; b < (uint32_t)kMaxBuckets && bucket_start(log2F, b) < s; ++b) {
    const uint64_t st = bucket_start(log2F, b), len = bucket_len(log2F, b);
    const uint64_t live = s - st < len ? s - st : len;
    const gptr<T> p = gmem(reinterpret_cast<T*>(__shfl(bp, (int)b, 64)));
    const gptr<u32x4> vp = reinterpret_cast<gptr<u32x4>>(p);
    const uint64_t nv = live / VPL;
    for (uint64_t q0 = 0; q0 < nv; q0 += kU * 64) {
      u32x4 x[kU];
#pragma unroll
      for (uint32_t k = 0; k < kU; ++k) {
        const uint64_t q = q0 + 64u * k + lane;
        x[k] = vp[q < nv ? q : nv - 1];
      }
#pragma unroll
      for (uint32_t k = 0; k < kU; ++k) {
        const uint64_t q = q0 + 64u * k + lane;
        if (q < nv) vp[q] = op_vec<T>(op, x[k]);
      }
    }
    const uint64_t e = nv * VPL + lane;
    if (e < live) p[e] = apply_op<T>(op, p[e]);
  }
}

// n elements from src (a bucket, 256-byte aligned) to dst by one wave: stores
// aligned to dst's 128-byte lines, loads taking src's alignment, eight vectors
// per lane in flight (unconditional loads, clamped indices).
template <typename T>
__device__ void wave_copy(T* dst_, const T* src_, uint64_t n) {
  typedef u32x4 u32x4_a4 __attribute__((aligned(4)));
  constexpr uint32_t VPL = 16 / sizeof(T), kLine = 128 / sizeof(T), kU = 8;
  const uint32_t lane = s_lane();
  if (n == 0) return;
  const gptr<T> dst = gmem(dst_);
  const gptr<const T> src = gmem(src_);
  const uint32_t mis = (uint32_t)((reinterpret_cast<uintptr_t>(dst_) & 127u) / sizeof(T));
  uint64_t head = mis ? kLine - mis : 0u;
  if (head > n) head = n;
  if (lane < head) __builtin_nontemporal_store(src[lane], dst + lane);
  const uint64_t nv = (n - head) / VPL;
  if (nv) {
    const gptr<const u32x4_a4> vs = reinterpret_cast<gptr<const u32x4_a4>>(src + head);
    const gptr<u32x4> vd = reinterpret_cast<gptr<u32x4>>(dst + head);
    for (uint64_t q0 = 0; q0 < nv; q0 += kU * 64) {
      u32x4 x[kU];
#pragma unroll
      for (uint32_t k = 0; k < kU; ++k) {
        const uint64_t q = q0 + 64u * k + lane;
        x[k] = vs[q < nv ? q : nv - 1];
      }
#pragma unroll
      for (uint32_t k = 0; k < kU; ++k) {
        const uint64_t q = q0 + 64u * k + lane;
        if (q < nv) __builtin_nontemporal_store(x[k], vd + q);
      }
    }
  }
  const uint64_t tail = head + nv * VPL + lane;
  if (tail < n) __builtin_nontemporal_store(src[tail], dst + tail);
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kSB) void step_wave_kernel(const BatchArr* arrs, const uint32_t* varr,
                                                        const uint64_t* vbegin, uint64_t total_v, StepDesc D,
                                                        const uint64_t* counts, uint32_t n_arr, uint32_t op, T* out,
                                                        uint64_t out_cap, uint32_t* sync, uint64_t* chunk_sum,
                                                        uint64_t chunk_len, uint32_t* berr, uint32_t spin,
                                                        uint64_t* vsize) {
  __shared__ StepShared sh;
  __shared__ uint64_t cpre[kStepChunkMax];
  const uint32_t tid = threadIdx.x, lane = s_lane();
  const uint32_t G = gridDim.x;
  const uint64_t gw = (uint64_t)blockIdx.x * kSW + (tid >> 6), GW = (uint64_t)G * kSW;

  // Phase A: rounds and r/w, one LFVector per wave at a time.
  for (uint64_t wv = gw; wv < total_v; wv += GW) {
    const uint32_t i = varr[wv];
    const ArrRef A = arrs[i].A;
    const uint32_t elem_log2 = arrs[i].elem_log2;
    const uint32_t v = (uint32_t)(wv - vbegin[i]);
    uint64_t bp = lane < (uint32_t)kMaxBuckets ? A.bptr[(uint64_t)v * kMaxBuckets + lane] : 0;
    uint64_t s = A.size[v];
    bool dead = A.dead[v] != 0;
    bool changed = false;
    uint32_t keep_hi = 0;
    uint64_t reused = 0;
    if (D.clear) {
      keep_hi = step_clear(A, v, elem_log2, lane, s, dead);
      if (dead) bp = 0;
      s = 0;
      changed = true;
    }
    for (uint32_t r = 0; r < D.n_rounds && !dead; ++r) {
      const uint64_t nthr = counts[(uint64_t)r * n_arr + i];
      const uint64_t chunk = (nthr + A.V - 1) / A.V;
      const uint64_t c0 = (uint64_t)v * chunk;
      const uint64_t cnt = c0 < nthr ? (nthr - c0 < chunk ? nthr - c0 : chunk) : 0;
      if (cnt == 0) continue;
      const StepRound& R = D.r[r];
      const uint64_t s_round = s;
      bool ok;
      if (R.kind == kModeBernoulli)
        ok = wave_round<T>(A, v, elem_log2, c0, cnt, ProdBernoulli<T>{R.seed, R.round}, bp, s, keep_hi, reused);
      else if (R.kind == kModeRoundTag)
        ok = wave_round<T>(A, v, elem_log2, c0, cnt, ProdRoundTag<T>{R.round, R.tag_shift}, bp, s, keep_hi, reused);
      else
        ok = wave_round<T>(A, v, elem_log2, c0, cnt, ProdKeyed<T>{R.seed, R.round, R.tag_shift, R.tag + i}, bp, s,
                           keep_hi, reused);
      changed = true;
      if (!ok) {  // the round is dropped and the LFVector frozen, as in the per-round calls
        s = s_round;
        dead = true;
        if (lane == 0) {
          A.dead[v] = 1u;
          set_error(A.err, kErrNoMem);
        }
      }
    }
    if (D.clear) step_release_unused(A, v, elem_log2, lane, keep_hi, reused, bp);
    if (changed && lane == 0) st_rlx(&A.size[v], s);
    if (lane == 0) st_rlx(&vsize[wv], s);
    if (op != kOpNone) wave_rw<T>(A.log2F, op, bp, s);
  }

  if (out) {
    // Phase B: totals of chunks of chunk_len consecutive LFVectors.
    step_barrier(&sync[0], G, spin, berr);
    const uint64_t nchunks = (total_v + chunk_len - 1) / chunk_len;
    const uint64_t* ctot = chunk_len == 1 ? vsize : chunk_sum;
    if (chunk_len > 1) {
      for (uint64_t c = blockIdx.x; c < nchunks; c += G) {
        uint64_t x = 0;
        for (uint64_t wv = c * chunk_len + tid; wv < total_v && wv < (c + 1) * chunk_len; wv += kSB)
          x += ld_rlx(&vsize[wv]);
        x = step_block_sum(x, sh);
        if (tid == 0) st_rlx(&chunk_sum[c], x);
      }
      step_barrier(&sync[1], G, spin, berr);
    }

    // Phase C: every workgroup scans the chunk totals; each wave copies its
    // LFVectors to their places.
    constexpr uint32_t kPer = kStepChunkMax / kSB;
    uint64_t x[kPer], sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
      const uint64_t c = (uint64_t)tid * kPer + k;
      x[k] = c < nchunks ? ld_rlx(&ctot[c]) : 0;
      sum += x[k];
    }
    uint64_t incl = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(incl, d, 64);
      if (lane >= (uint32_t)d) incl += y;
    }
    if (lane == 63) sh.red[tid >> 6] = incl;
    __syncthreads();
    uint64_t run = incl - sum, total = 0;
    for (uint32_t q = 0; q < kSW; ++q) {
      run += q < (tid >> 6) ? sh.red[q] : 0;
      total += sh.red[q];
    }
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
      cpre[tid * kPer + k] = run;
      run += x[k];
    }
    __syncthreads();
    if (total > out_cap) {
      if (blockIdx.x == 0 && tid == 0) set_error(berr, kErrRange);
    } else {
      for (uint64_t wv = gw; wv < total_v; wv += GW) {
        const uint32_t i = varr[wv];
        const ArrRef& A = arrs[i].A;
        const uint32_t v = (uint32_t)(wv - vbegin[i]);
        const uint64_t c = wv / chunk_len;
        uint64_t y = 0;
        for (uint64_t u = c * chunk_len + lane; u < wv; u += 64) y += ld_rlx(&vsize[u]);
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) y += __shfl_xor(y, d, 64);
        const uint64_t off = cpre[c] + y;
        const uint64_t sz = ld_rlx(&vsize[wv]);
        const uint64_t bp = lane < (uint32_t)kMaxBuckets ? A.bptr[(uint64_t)v * kMaxBuckets + lane] : 0;
        for (uint32_t b = 0; b < (uint32_t)kMaxBuckets && bucket_start(A.log2F, b) < sz; ++b) {
          const uint64_t st = bucket_start(A.log2F, b), len = bucket_len(A.log2F, b);
          const uint64_t live = sz - st < len ? sz - st : len;
          wave_copy<T>(out + off + st, reinterpret_cast<const T*>(__shfl(bp, (int)b, 64)), live);
        }
      }
    }
  }

  __syncthreads();
  if (tid == 0 && fetch_add32(&sync[2], 1u) == G - 1) {
    st_rlx32(&sync[0], 0u);
    st_rlx32(&sync[1], 0u);
    st_rlx32(&sync[2], 0u);
  }
}

// ------------------------------------------------------------------- host --
namespace {

template <typename T>
int queue_step(gga_batch* b, const StepDesc& D, const uint64_t* d_counts, uint32_t op, void* out, uint64_t out_cap,
               hipStream_t s) {
  // One workgroup per LFVector while the LFVectors are fewer than the device's
  // wave slots could take one at a time (configuration 1: 256 LFVectors of
  // 1024-candidate rounds spread over 4 waves each), else one wave per LFVector.
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return GGA_EHIP;
  const bool per_wave = b->total_vectors > (uint64_t)cus * 16;
  const void* fn = per_wave ? reinterpret_cast<const void*>(&step_wave_kernel<T>)
                            : reinterpret_cast<const void*>(&step_kernel<T>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kSB, 0) != hipSuccess) return GGA_EHIP;
  uint64_t G = (uint64_t)cus * (uint64_t)(per_cu > 0 ? per_cu : 1);
  const uint64_t need = per_wave ? (b->total_vectors + kSW - 1) / kSW : b->total_vectors;
  if (G > need) G = need;
  if (G < 1) G = 1;
  const uint64_t chunk_len = (b->total_vectors + kStepChunkMax - 1) / kStepChunkMax;
  const BatchArr* arrs = b->d_arrays;
  const uint32_t* varr = b->d_varr;
  const uint64_t* vbegin = b->d_vbegin;
  uint64_t total_v = b->total_vectors;
  uint32_t n_arr = b->n;
  T* o = static_cast<T*>(out);
  uint32_t* sync = b->d_step_sync;
  uint64_t* chunk_sum = b->d_step_chunks;
  uint32_t* berr = b->d_err;
  uint32_t spin = kSpinLimit;
  StepDesc desc = D;
  uint64_t clen = chunk_len;
  uint64_t* vsize = b->d_step_vsize;
  void* args[] = {&arrs, &varr, &vbegin, &total_v, &desc, &d_counts, &n_arr, &op, &o, &out_cap,
                  &sync, &chunk_sum, &clen, &berr, &spin, &vsize};
  hipError_t e;
  if (stream_capturing(s))  // recorded as a plain launch; the grid still fits the device at once
    e = hipLaunchKernel(fn, dim3((uint32_t)G), dim3(kSB), args, 0, s);
  else
    e = hipLaunchCooperativeKernel(fn, dim3((uint32_t)G), dim3(kSB), args, 0, s);
  return hip_status(e);
}

}  // namespace

int launch_batch_step(gga_batch* b, const StepDesc& D, const uint64_t* d_counts, uint32_t op, void* out,
                      uint64_t out_cap, hipStream_t s) {
  const int rc = b->elem_bytes == 4 ? queue_step<uint32_t>(b, D, d_counts, op, out, out_cap, s)
                                    : queue_step<uint64_t>(b, D, d_counts, op, out, out_cap, s);
  if (rc == GGA_OK)
    for (uint32_t i = 0; i < b->n; ++i) sizes_changed(b->arrays[i], s);
  return rc;
}

}  // namespace gga
