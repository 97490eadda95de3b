// Size/prefix scan, shrink, regular read/write, flatten and bucket release.
//
// Regular access walks the LFVectors bucket by bucket (the per-block access rw_b
// of Sec. VI-B), but the work is cut into bucket-aligned tiles of at most 16 KiB,
// so the number of LFVectors and their uneven sizes do not set the parallelism.
// A tile lies inside one bucket and streams 16-byte vectors.  For an array (or a
// batch) of at least 2048 tiles the tiles are listed once per state of the sizes
// in a tile table and workgroups take table entries; smaller arrays and served
// steps spread the tiles over a persistent grid that locates its share by a
// search of the tile prefix.
#include <hip/hip_ext.h>

#include "gga_internal.h"

namespace gga {
namespace {

constexpr uint32_t kScanThreads = 1024;
// Persistent grids of the batched and served streaming kernels (256-thread
// workgroups; 256 CUs).  Measured on configuration 2 with the search-located
// shares: r/w peaks at 4096-8192 workgroups, flatten keeps gaining up to 65536
// (4.47 TB/s at 2048, 4.70 at 16384, 5.13 at 32768, 5.27 at 65536).
constexpr uint32_t kRwBlocks = 8192;
constexpr uint32_t kFlattenBlocks = 65536;
// Table-driven r/w and flatten of one array: one workgroup per tile, up to this
// many workgroups, looping beyond (configuration 2: flatten 5.33 -> 5.7 TB/s
// against the search-located persistent grid).
constexpr uint32_t kTableBlocks = 131072;
// Largest tile table kept per array (128 MiB, arrays up to 128 GiB of elements);
// a larger array walks its buckets instead.  Arrays the host knows to hold fewer
// than kTableMinTiles tiles (32 MiB of elements) walk their buckets too: for them
// the table's extra launch costs more than it saves.
constexpr uint64_t kTableMaxTiles = 1ull << 23;
constexpr uint64_t kTableMinTiles = 2048;

// Workgroups are dispatched round robin over the 8 XCDs, each with its own L2
// and address-translation caches.  A streaming grid is therefore a multiple of
// 8, and the workgroups of XCD x (those with b % 8 == x) take the x-th
// contiguous eighth of the tiles, striding by the number of workgroups per XCD:
// each XCD's caches then see one region of the tile table and of the buckets it
// lists (measured: configuration 2's r/w 5.72 -> 6.00 TB/s after a flatten and
// 5.58 -> 5.72 after an r/w; configuration 3's 1-2% faster).
inline uint32_t xcd_grid(uint64_t g) {
  g = (g + 7) & ~7ull;
  return (uint32_t)(g < 8 ? 8 : g);
}

struct TileSpan {
  uint64_t t, end, step;
};

__device__ __forceinline__ TileSpan xcd_span(uint64_t total) {
  const uint64_t G = gridDim.x;
  if (G & 7u) return {blockIdx.x, total, G};
  const uint64_t part = (total + 7) >> 3, x = blockIdx.x & 7u;
  const uint64_t end = (x + 1) * part < total ? (x + 1) * part : total;
  return {x * part + (blockIdx.x >> 3), end, G >> 3};
}

// Workgroups for one array's r/w or flatten: enough for the tiles the array can
// hold (the host's upper bound of its size), at most `cap`, so a small array
// does not pay for dispatching a grid sized for the largest ones.
inline uint32_t stream_grid(const ggarray* a, uint32_t cap) {
  const uint32_t te_log2 = 14u - a->elem_log2;
  const uint64_t g = (a->size_ub >> te_log2) + 2ull * a->V;
  return xcd_grid(g > cap ? cap : g);
}

typedef u32x4 u32x4_a4 __attribute__((aligned(4)));

// Exclusive prefix sums of the LFVector sizes (element offsets, Sec. IV) and of
// their tile counts, by one workgroup of kScanThreads; entry V holds the totals.
__device__ __forceinline__ void scan_array(const ArrRef& A, uint32_t te_log2, uint64_t* copy = nullptr) {
  __shared__ uint64_t wsum_e[kScanThreads / 64], wsum_t[kScanThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint32_t V = A.V;
  const uint32_t per = (V + kScanThreads - 1) / kScanThreads;
  const uint32_t v0 = tid * per < V ? tid * per : V;
  const uint32_t v1 = v0 + per < V ? v0 + per : V;
  uint64_t e = 0, t = 0;
  for (uint32_t v = v0; v < v1; ++v) {
    const uint64_t s = A.size[v];
    e += s;
    t += tiles_for(A.log2F, s, te_log2);
  }
  const uint64_t ie = wave_incl_scan64(e), it = wave_incl_scan64(t);
  if (lane == 63) {
    wsum_e[w] = ie;
    wsum_t[w] = it;
  }
  __syncthreads();
  uint64_t be = 0, bt = 0, te = 0, tt = 0;
  for (uint32_t k = 0; k < kScanThreads / 64; ++k) {
    if (k < w) {
      be += wsum_e[k];
      bt += wsum_t[k];
    }
    te += wsum_e[k];
    tt += wsum_t[k];
  }
  uint64_t re = be + ie - e, rt = bt + it - t;
  for (uint32_t v = v0; v < v1; ++v) {
    const uint64_t s = A.size[v];
    A.prefix[v] = re;
    if (copy) copy[v] = re;
    A.tprefix[v] = rt;
    re += s;
    rt += tiles_for(A.log2F, s, te_log2);
  }
  if (tid == 0) {
    A.prefix[V] = te;
    if (copy) copy[V] = te;
    A.tprefix[V] = tt;
  }
}

// `copy`, if not null, receives the V + 1 prefix entries too (ggarray_prefix).
__global__ __launch_bounds__(kScanThreads) void scan_kernel(ArrRef A, uint32_t te_log2, uint64_t* copy) {
  scan_array(A, te_log2, copy);
}

// The same prefix sums for many LFVectors, over many workgroups in two passes.
// Pass 1: workgroup c scans LFVectors [1024 c, 1024 c + 1024) (one per thread,
// coalesced), writes their prefixes within the chunk and the chunk's totals.
__global__ __launch_bounds__(kScanThreads) void scan_chunks_kernel(ArrRef A, uint64_t* tot, uint32_t te_log2) {
  __shared__ uint64_t wsum_e[kScanThreads / 64], wsum_t[kScanThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint32_t v = blockIdx.x * kScanThreads + tid;
  const uint64_t e = v < A.V ? A.size[v] : 0;
  const uint64_t t = tiles_for(A.log2F, e, te_log2);
  const uint64_t ie = wave_incl_scan64(e), it = wave_incl_scan64(t);
  if (lane == 63) {
    wsum_e[w] = ie;
    wsum_t[w] = it;
  }
  __syncthreads();
  uint64_t be = 0, bt = 0, ce = 0, ct = 0;
  for (uint32_t k = 0; k < kScanThreads / 64; ++k) {
    if (k < w) {
      be += wsum_e[k];
      bt += wsum_t[k];
    }
    ce += wsum_e[k];
    ct += wsum_t[k];
  }
  if (v < A.V) {
    A.prefix[v] = be + ie - e;
    A.tprefix[v] = bt + it - t;
  }
  if (tid == 0) {
    tot[2 * blockIdx.x] = ce;
    tot[2 * blockIdx.x + 1] = ct;
  }
}

// Pass 2: workgroup c adds the totals of the chunks before it; the last chunk's
// workgroup writes entry V.
__global__ __launch_bounds__(kScanThreads) void scan_fix_kernel(ArrRef A, const uint64_t* tot, uint32_t nchunks,
                                                             uint64_t* copy) {
  __shared__ uint64_t red_e[kScanThreads / 64], red_t[kScanThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  uint64_t e = 0, t = 0;
  for (uint32_t c = tid; c < blockIdx.x; c += kScanThreads) {
    e += tot[2 * c];
    t += tot[2 * c + 1];
  }
  e = wave_incl_scan64(e);
  t = wave_incl_scan64(t);
  if (lane == 63) {
    red_e[w] = e;
    red_t[w] = t;
  }
  __syncthreads();
  uint64_t oe = 0, ot = 0;
  for (uint32_t k = 0; k < kScanThreads / 64; ++k) {
    oe += red_e[k];
    ot += red_t[k];
  }
  const uint32_t v = blockIdx.x * kScanThreads + tid;
  if (v < A.V) {
    A.prefix[v] += oe;
    if (copy) copy[v] = A.prefix[v];
    A.tprefix[v] += ot;
  }
  if (blockIdx.x == nchunks - 1 && tid == 0) {
    A.prefix[A.V] = oe + tot[2 * blockIdx.x];
    if (copy) copy[A.V] = oe + tot[2 * blockIdx.x];
    A.tprefix[A.V] = ot + tot[2 * blockIdx.x + 1];
  }
}

constexpr uint32_t kVecPerBlock = 4;  // shrink: 256 threads = 4 waves = 4 LFVectors

__global__ __launch_bounds__(256) void shrink_kernel(ArrRef A, uint32_t num, uint32_t den,
                                                     uint32_t elem_log2) {
  const uint32_t v = blockIdx.x * kVecPerBlock + (threadIdx.x >> 6);
  if (v < A.V) shrink_vector(A, v, num, den, elem_log2);
}

// Returns every bucket of the array to the pool (destroy).
__global__ __launch_bounds__(256) void free_all_kernel(ArrRef A, uint32_t elem_log2) {
  const uint32_t v = blockIdx.x * kVecPerBlock + (threadIdx.x >> 6);
  const uint32_t b = threadIdx.x & 63u;
  if (v >= A.V || b >= (uint32_t)kMaxBuckets) return;
  uint64_t* slot = A.bptr + (uint64_t)v * kMaxBuckets + b;
  const uint64_t p = *slot;
  if (p > kFailedPtr)
    pool_free(A.pool, reinterpret_cast<uint8_t*>(p), bucket_class(A.log2F, elem_log2, b), pool_shard(v, b, A.salt));
  *slot = 0;
}

// Elements held by allocated buckets.
__global__ void capacity_kernel(ArrRef A, uint64_t* out) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= A.V) return;
  const uint64_t* row = A.bptr + (uint64_t)v * kMaxBuckets;
  uint64_t c = 0;
  for (uint32_t b = 0; b < (uint32_t)kMaxBuckets; ++b)
    if (row[b] > kFailedPtr) c += bucket_len(A.log2F, b);
  if (c) fetch_add(out, c);
}

// One tile: cnt (<= te) elements at src (16-byte aligned); rw in place, or copy
// to dst (element aligned) for flatten.  Lane i of slot k handles the 16 bytes
// at element k * (256 * VPL) + i * VPL.  Every byte is touched once, so stores
// are non-temporal; so are flatten's loads, while r/w loads through the cache,
// which lets its non-temporal stores find the lines they overwrite (measured:
// r/w 4.80 -> 5.31 TB/s, flatten slower with cached loads).  Neither carries the
// device-scope bit that the insertion's stores do: with it r/w measured 5.0
// TB/s, and flatten gained 1.5% on configuration 2 but slowed the batched step
// that follows it by 3%.
template <typename T, bool kFlatten, bool kNtLoad = kFlatten>
__device__ __forceinline__ void stream_tile(T* src_, T* dst_, uint32_t cnt, uint32_t op) {
  const gptr<T> src = gmem(src_), dst = gmem(dst_);
  constexpr uint32_t VPL = 16 / sizeof(T);
  constexpr uint32_t kSlots = 4;
  constexpr uint32_t kSpan = kRwThreads * VPL;
  const uint32_t tid = threadIdx.x;
  if (kFlatten) {
    // A destination that is not 128-byte aligned: stage the tile in LDS (aligned
    // loads), then write the destination in whole 128-byte lines, each store
    // instruction of a wave covering complete lines (flatten 4.51 -> 4.70 TB/s;
    // taking the misalignment on the global loads instead was slower).
    __shared__ u32x4 stage[kSlots * kRwThreads];
    const uint32_t mis = (uint32_t)((reinterpret_cast<uintptr_t>(dst_) & 127u) / sizeof(T));
    if (mis) {
      const uint32_t nsrc = (cnt + VPL - 1) / VPL;
      for (uint32_t k = 0; k < kSlots; ++k) {
        const uint32_t q = k * kRwThreads + tid;
        if (q < nsrc) {
          if ((q + 1) * VPL <= cnt)
            stage[q] = __builtin_nontemporal_load(reinterpret_cast<gptr<const u32x4>>(src + q * VPL));
          else {
            T tmp[VPL] = {};
            for (uint32_t e = 0; e < VPL && q * VPL + e < cnt; ++e) tmp[e] = src[q * VPL + e];
            u32x4 x;
            __builtin_memcpy(&x, tmp, 16);
            stage[q] = x;
          }
        }
      }
      __syncthreads();
      const T* st = reinterpret_cast<const T*>(stage);
      const gptr<T> dal = dst - mis;
      const uint32_t nvec = (cnt + mis + VPL - 1) / VPL;
      for (uint32_t j = tid; j < nvec; j += kRwThreads) {
        const int64_t e0 = (int64_t)j * VPL - (int64_t)mis;
        if (e0 >= 0 && e0 + (int64_t)VPL <= (int64_t)cnt) {
          T tmp[VPL];
          for (uint32_t e = 0; e < VPL; ++e) tmp[e] = st[e0 + e];
          u32x4 x;
          __builtin_memcpy(&x, tmp, 16);
          __builtin_nontemporal_store(x, reinterpret_cast<gptr<u32x4>>(dal + (uint64_t)j * VPL));
        } else {
          for (uint32_t e = 0; e < VPL; ++e) {
            const int64_t i = e0 + e;
            if (i >= 0 && i < (int64_t)cnt) dst[i] = st[i];
          }
        }
      }
      __syncthreads();
      return;
    }
  }
  if (cnt == kSlots * kSpan) {
    u32x4 r[kSlots];
#pragma unroll
    for (uint32_t k = 0; k < kSlots; ++k)
      r[k] = kNtLoad ? __builtin_nontemporal_load(reinterpret_cast<gptr<const u32x4>>(src + k * kSpan + tid * VPL))
                      : *reinterpret_cast<gptr<const u32x4>>(src + k * kSpan + tid * VPL);
#pragma unroll
    for (uint32_t k = 0; k < kSlots; ++k) {
      if (kFlatten)
        __builtin_nontemporal_store(r[k], reinterpret_cast<gptr<u32x4_a4>>(dst + k * kSpan + tid * VPL));
      else
        __builtin_nontemporal_store(op_vec<T>(op, r[k]), reinterpret_cast<gptr<u32x4>>(src + k * kSpan + tid * VPL));
    }
    return;
  }
  for (uint32_t k = 0; k < kSlots; ++k) {
    const uint32_t e = k * kSpan + tid * VPL;
    if (e + VPL <= cnt) {
      const u32x4 x = kNtLoad ? __builtin_nontemporal_load(reinterpret_cast<gptr<const u32x4>>(src + e))
                               : *reinterpret_cast<gptr<const u32x4>>(src + e);
      if (kFlatten)
        __builtin_nontemporal_store(x, reinterpret_cast<gptr<u32x4_a4>>(dst + e));
      else
        __builtin_nontemporal_store(op_vec<T>(op, x), reinterpret_cast<gptr<u32x4>>(src + e));
    } else {
      for (uint32_t q = e; q < cnt && q < e + VPL; ++q) {
        if (kFlatten)
          dst[q] = src[q];
        else
          src[q] = apply_op<T>(op, src[q]);
      }
    }
  }
}

// Walk over the bucket-aligned tiles [t0, t1) of one array: find the first
// LFVector by binary search over the tile prefix, then walk forward; the bucket
// pointer and the destination offset are reloaded only when the walk enters a
// new bucket.
template <typename T, bool kFlatten>
__device__ __forceinline__ void stream_range(const ArrRef& A, uint64_t t0, uint64_t t1, uint32_t op,
                                             T* out, uint32_t te_log2) {
  const uint32_t V = A.V;
  if (t0 >= t1) return;
  uint32_t lo = 0, hi = V;  // tprefix[lo] <= t0 < tprefix[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (A.tprefix[mid] <= t0) lo = mid; else hi = mid;
  }
  uint32_t v = lo;
  uint64_t s = A.size[v];
  uint64_t k = t0 - A.tprefix[v];
  const uint32_t log2F = A.log2F;
  const uint64_t te = 1ull << te_log2;
  uint32_t b = 0;
  uint64_t live, nt;
  for (;;) {
    live = bucket_len(log2F, b);
    const uint64_t st = bucket_start(log2F, b);
    if (s - st < live) live = s - st;
    nt = (live + te - 1) >> te_log2;
    if (k < nt) break;
    k -= nt;
    ++b;
  }
  T* bucket = reinterpret_cast<T*>(A.bptr[(uint64_t)v * kMaxBuckets + b]);
  T* dbase = kFlatten ? out + A.prefix[v] + bucket_start(log2F, b) : nullptr;
  for (uint64_t t = t0;;) {
    const uint64_t e0 = k << te_log2;
    const uint64_t rem = live - e0;
    const uint32_t cnt = (uint32_t)(rem < te ? rem : te);
    stream_tile<T, kFlatten>(bucket + e0, kFlatten ? dbase + e0 : nullptr, cnt, op);
    if (++t >= t1) break;
    if (++k == nt) {
      k = 0;
      ++b;
      if (bucket_start(log2F, b) >= s) {
        b = 0;
        do {
          ++v;
          s = A.size[v];
        } while (s == 0);
      }
      live = bucket_len(log2F, b);
      const uint64_t st = bucket_start(log2F, b);
      if (s - st < live) live = s - st;
      nt = (live + te - 1) >> te_log2;
      bucket = reinterpret_cast<T*>(A.bptr[(uint64_t)v * kMaxBuckets + b]);
      if (kFlatten) dbase = out + A.prefix[v] + st;
    }
  }
}

// Tile table of one array, built once per state of the sizes (after the prefix
// scan): tile t, in the order of the tile prefix, gets the address of its first
// element and its destination offset in a flatten, with its element count in the
// top 16 bits.  One wave per LFVector, lanes over the tiles of each bucket.
// Entries from `cap` on are not written; the streaming kernels then walk the
// buckets instead.
__device__ __forceinline__ void table_vector(const ArrRef& A, uint32_t v, uint64_t* tab, uint64_t cap,
                                             uint32_t te_log2, uint32_t elem_log2, uint64_t t_base,
                                             uint64_t e_base) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t s = A.size[v];
  uint64_t t = t_base + A.tprefix[v];
  const uint64_t pv = e_base + A.prefix[v];
  const uint32_t log2F = A.log2F;
  const uint64_t te = 1ull << te_log2;
  typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
  for (uint32_t b = 0; b < (uint32_t)kMaxBuckets; ++b) {
    const uint64_t st = bucket_start(log2F, b);
    if (st >= s) break;
    uint64_t live = bucket_len(log2F, b);
    if (s - st < live) live = s - st;
    const uint64_t nt = (live + te - 1) >> te_log2;
    const uint64_t base = A.bptr[(uint64_t)v * kMaxBuckets + b];
    for (uint64_t i = lane; i < nt; i += 64) {
      const uint64_t e0 = i << te_log2;
      const uint64_t cnt = live - e0 < te ? live - e0 : te;
      if (t + i < cap) {
        const u64x2 d = {base + (e0 << elem_log2), (pv + st + e0) | (cnt << 48)};
        gmem(reinterpret_cast<u64x2*>(tab))[t + i] = d;
      }
    }
    t += nt;
  }
}

__global__ __launch_bounds__(256) void tile_table_kernel(ArrRef A, uint64_t* tab, uint64_t cap, uint32_t te_log2,
                                                         uint32_t elem_log2) {
  const uint32_t v = blockIdx.x * kVecPerBlock + (threadIdx.x >> 6);
  if (v < A.V) table_vector(A, v, tab, cap, te_log2, elem_log2, 0, 0);
}

// The tile table of a batch: the tiles of array i follow those of arrays before
// it (tile_begin), and destination offsets are positions in the batch flatten
// (elem_begin).  Wave w is LFVector w - vbegin[i] of array i.
__global__ __launch_bounds__(256) void batch_table_kernel(const BatchArr* items, const uint64_t* vbegin,
                                                          const uint64_t* tile_begin, const uint64_t* elem_begin,
                                                          uint32_t n, uint64_t* tab, uint64_t cap,
                                                          uint32_t te_log2) {
  const uint64_t w = (uint64_t)blockIdx.x * kVecPerBlock + (threadIdx.x >> 6);
  if (w >= vbegin[n]) return;
  const uint32_t i = wave_search(vbegin, n, w);
  table_vector(items[i].A, (uint32_t)(w - vbegin[i]), tab, cap, te_log2, items[i].elem_log2, tile_begin[i],
               elem_begin[i]);
}

// Load policy of r/w.  Non-temporal loads (kNtLoad) serve an r/w that directly
// follows another r/w of the array (configuration 2: 5.3 against 4.9 TB/s) and
// every r/w of at least kNtLoadBytes of elements; a smaller array read after an
// insertion or a flatten loads through the cache.  Measured on single arrays
// (u32, V = 512, r/w after an insertion), cached against non-temporal loads:
// 6.07 against 5.27 TB/s at 0.54 GB, 5.74 against 5.59 at 1.07 GB, 5.68 against
// 5.78 at 2.15 GB and 5.41 against 5.56 at 4.29 GB; configuration 4's batch
// (3.84 GB of buckets of at most 64 KiB) 4.40 against 4.70 TB/s.
constexpr uint64_t kNtLoadBytes = 5ull << 28;  // 1.25 GiB

// Tiles [sp.t, sp.end) of a tile table, stride sp.step.
template <typename T, bool kFlatten, bool kNtLoad>
__device__ __forceinline__ void table_tiles(const uint64_t* __restrict__ tab, const TileSpan& sp, uint32_t op,
                                            T* out) {
  for (uint64_t t = sp.t; t < sp.end; t += sp.step) {
    const uint64_t src = tab[2 * t], w = tab[2 * t + 1];
    stream_tile<T, kFlatten, kNtLoad>(reinterpret_cast<T*>(src), kFlatten ? out + (w & 0xFFFFFFFFFFFFull) : nullptr,
                                      (uint32_t)(w >> 48), op);
  }
}

// r/w or flatten of one array through its tile table: each XCD's workgroups
// stride over their eighth of the tiles (one tile each when the grid covers the
// array).  Without a table for the current state (more tiles than it holds) the
// grid walks the buckets.
template <typename T, bool kFlatten, bool kNtLoad = kFlatten>
__global__ __launch_bounds__(kRwThreads) void stream_table_kernel(ArrRef A, const uint64_t* __restrict__ tab,
                                                                 uint64_t cap, uint32_t op, T* out,
                                                                 uint64_t out_cap, uint32_t te_log2) {
  const uint64_t total = A.tprefix[A.V];
  if (kFlatten && A.prefix[A.V] > out_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_error(A.err, kErrRange);
    return;
  }
  const uint64_t G = gridDim.x;
  if (total > cap) {
    stream_range<T, kFlatten>(A, total * blockIdx.x / G, total * (blockIdx.x + 1) / G, op, out, te_log2);
    return;
  }
  const TileSpan sp = xcd_span(total);
  if (!kFlatten && !kNtLoad && A.prefix[A.V] * sizeof(T) >= kNtLoadBytes)
    table_tiles<T, false, true>(tab, sp, op, out);
  else
    table_tiles<T, kFlatten, kNtLoad>(tab, sp, op, out);
}

// Static / semi-static array r/w: the flat array cut into 16 KiB tiles, workgroup
// w streaming tiles w, w + G, ... (the GGArray's tile size and load policy
// without the bucket indirection).  A contiguous array streams faster in this
// plain order than with the GGArray's split of the tiles over the XCDs
// (configuration 2's static r/w 6.35 against 6.07 TB/s), so it keeps it.
template <typename T, bool kNtLoad>
__global__ __launch_bounds__(kRwThreads) void static_rw_kernel(T* data, const uint64_t* size,
                                                              uint64_t cap, uint32_t op, uint32_t te_log2) {
  uint64_t n = *size;
  if (n > cap) n = cap;
  const uint64_t te = 1ull << te_log2;
  const uint64_t total = (n + te - 1) >> te_log2;
  const TileSpan sp{blockIdx.x, total, gridDim.x};
  if (!kNtLoad && n * sizeof(T) >= kNtLoadBytes) {
    for (uint64_t t = sp.t; t < sp.end; t += sp.step) {
      const uint64_t e0 = t << te_log2;
      const uint64_t rem = n - e0;
      stream_tile<T, false, true>(data + e0, nullptr, (uint32_t)(rem < te ? rem : te), op);
    }
    return;
  }
  for (uint64_t t = sp.t; t < sp.end; t += sp.step) {
    const uint64_t e0 = t << te_log2;
    const uint64_t rem = n - e0;
    stream_tile<T, false, kNtLoad>(data + e0, nullptr, (uint32_t)(rem < te ? rem : te), op);
  }
}


// ----------------------------------------------------------------- batches --
// One workgroup per array of the batch: its own prefix sums.
__global__ __launch_bounds__(kScanThreads) void batch_scan_kernel(const BatchArr* items, uint32_t te_log2) {
  scan_array(items[blockIdx.x].A, te_log2);
}

// Exclusive prefix over the arrays of their tile counts and sizes (entry n holds
// the totals), by one workgroup.
template <class Item>
__global__ __launch_bounds__(kScanThreads) void batch_top_kernel(const Item* items, uint32_t n,
                                                                uint64_t* tile_begin, uint64_t* elem_begin) {
  __shared__ uint64_t wsum_e[kScanThreads / 64], wsum_t[kScanThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint32_t per = (n + kScanThreads - 1) / kScanThreads;
  const uint32_t i0 = tid * per < n ? tid * per : n;
  const uint32_t i1 = i0 + per < n ? i0 + per : n;
  uint64_t e = 0, t = 0;
  for (uint32_t i = i0; i < i1; ++i) {
    e += items[i].A.prefix[items[i].A.V];
    t += items[i].A.tprefix[items[i].A.V];
  }
  const uint64_t ie = wave_incl_scan64(e), it = wave_incl_scan64(t);
  if (lane == 63) {
    wsum_e[w] = ie;
    wsum_t[w] = it;
  }
  __syncthreads();
  uint64_t be = 0, bt = 0, te = 0, tt = 0;
  for (uint32_t k = 0; k < kScanThreads / 64; ++k) {
    if (k < w) {
      be += wsum_e[k];
      bt += wsum_t[k];
    }
    te += wsum_e[k];
    tt += wsum_t[k];
  }
  uint64_t re = be + ie - e, rt = bt + it - t;
  for (uint32_t i = i0; i < i1; ++i) {
    elem_begin[i] = re;
    tile_begin[i] = rt;
    re += items[i].A.prefix[items[i].A.V];
    rt += items[i].A.tprefix[items[i].A.V];
  }
  if (tid == 0) {
    elem_begin[n] = te;
    tile_begin[n] = tt;
  }
}

// Shrink of every array of the batch: one wave per LFVector; the waves of array
// i are [vbegin[i], vbegin[i+1]).
__global__ __launch_bounds__(256) void batch_shrink_kernel(const BatchArr* items, const uint64_t* vbegin,
                                                           uint32_t n, uint32_t num, uint32_t den) {
  const uint64_t w = (uint64_t)blockIdx.x * kVecPerBlock + (threadIdx.x >> 6);
  if (w >= vbegin[n]) return;
  const uint32_t i = wave_search(vbegin, n, w);
  shrink_vector(items[i].A, (uint32_t)(w - vbegin[i]), num, den, items[i].elem_log2);
}

// r/w or flatten of every array of the batch.  With a tile table covering the
// batch, each XCD's workgroups stride over their eighth of it (r/w with
// non-temporal loads from kNtLoadBytes of elements on); otherwise a persistent
// grid: workgroup w takes the w-th contiguous share of the tiles and walks it
// array by array.  Flatten writes array i at out + elem_begin[i].
template <typename T, bool kFlatten>
__global__ __launch_bounds__(kRwThreads) void batch_stream_kernel(const BatchArr* items, const uint64_t* tile_begin,
                                                                 const uint64_t* elem_begin, uint32_t n,
                                                                 const uint64_t* __restrict__ tab, uint64_t tcap,
                                                                 uint32_t op, T* out, uint64_t cap,
                                                                 uint32_t* err, uint32_t te_log2) {
  const uint64_t total = tile_begin[n];
  if (kFlatten && elem_begin[n] > cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_error(err, kErrRange);
    return;
  }
  const uint64_t G = gridDim.x;
  if (total <= tcap) {
    const TileSpan sp = xcd_span(total);
    if (!kFlatten && elem_begin[n] * sizeof(T) >= kNtLoadBytes)
      table_tiles<T, false, true>(tab, sp, op, out);
    else
      table_tiles<T, kFlatten, kFlatten>(tab, sp, op, out);
    return;
  }
  uint64_t g0 = total * blockIdx.x / G;
  const uint64_t g1 = total * (blockIdx.x + 1) / G;
  if (g0 >= g1) return;
  uint32_t i = wave_search(tile_begin, n, g0);
  while (g0 < g1 && i < n) {
    const uint64_t b0 = tile_begin[i], b1 = tile_begin[i + 1];
    const uint64_t hi = b1 < g1 ? b1 : g1;
    if (hi > g0)
      stream_range<T, kFlatten>(items[i].A, g0 - b0, hi - b0, op, kFlatten ? out + elem_begin[i] : nullptr, te_log2);
    if (hi > g0) g0 = hi;
    ++i;
  }
}

// ---------------------------------------------------------- served steps --
// Tile offsets of the step's items (exclusive prefix of their tile totals, entry
// n the sum) into tb, by one workgroup.
__device__ __forceinline__ void block_tile_offsets(const ServeItem* items, uint32_t n, uint64_t* tb) {
  __shared__ uint64_t wsum[kRwThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint32_t per = (n + kRwThreads - 1) / kRwThreads;
  const uint32_t i0 = tid * per < n ? tid * per : n;
  const uint32_t i1 = i0 + per < n ? i0 + per : n;
  uint64_t t = 0;
  for (uint32_t i = i0; i < i1; ++i) t += items[i].A.tprefix[items[i].A.V];
  const uint64_t it = wave_incl_scan64(t);
  if (lane == 63) wsum[w] = it;
  __syncthreads();
  uint64_t r = it - t, total = 0;
  for (uint32_t k = 0; k < kRwThreads / 64; ++k) {
    if (k < w) r += wsum[k];
    total += wsum[k];
  }
  for (uint32_t i = i0; i < i1; ++i) {
    tb[i] = r;
    r += items[i].A.tprefix[items[i].A.V];
  }
  if (tid == 0) tb[n] = total;
  __syncthreads();
}

// The r/w and flatten requests of one served step in one persistent grid: item i
// is r/w'd in place, or flattened to its own destination (written only if its
// reservation holds it).  The step's front launch scanned the arrays.  With
// kFused every workgroup forms the items' tile offsets in LDS itself; otherwise
// they come from tile_begin (batch_top_kernel).  Workgroup 0 also reports each
// flatten's length.
template <typename T, bool kFused>
__global__ __launch_bounds__(kRwThreads) void serve_stream_kernel(const ServeItem* items, const uint64_t* tile_begin,
                                                                 uint32_t n, uint32_t* err, uint32_t te_log2) {
  extern __shared__ uint64_t lds_tb[];
  if (blockIdx.x == 0)
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
      if (items[i].len_out) items[i].len_out[0] = items[i].A.prefix[items[i].A.V];
  const uint64_t* tb = tile_begin;
  if (kFused) {
    block_tile_offsets(items, n, lds_tb);
    tb = lds_tb;
  }
  const uint64_t total = tb[n];
  const uint64_t G = gridDim.x;
  uint64_t g0 = total * blockIdx.x / G;
  const uint64_t g1 = total * (blockIdx.x + 1) / G;
  if (g0 >= g1) return;
  uint32_t i = wave_search(tb, n, g0);
  while (g0 < g1 && i < n) {
    const uint64_t b0 = tb[i], b1 = tb[i + 1];
    const uint64_t hi = b1 < g1 ? b1 : g1;
    if (hi > g0) {
      const ServeItem& it = items[i];
      if (it.op != kOpFlatten)
        stream_range<T, false>(it.A, g0 - b0, hi - b0, it.op, nullptr, te_log2);
      else if (it.A.prefix[it.A.V] <= it.cap)
        stream_range<T, true>(it.A, g0 - b0, hi - b0, 0u, static_cast<T*>(it.out), te_log2);
      else if (threadIdx.x == 0)
        set_error(err, kErrRange);
      g0 = hi;
    }
    ++i;
  }
}

}  // namespace

int launch_serve_stream(const ServeItem* items, uint32_t n, uint64_t* tile_begin, uint64_t* elem_begin,
                        uint32_t* err, uint32_t elem_bytes, uint32_t grid, hipStream_t s) {
  if (n == 0) return GGA_OK;
  const uint32_t te_log2 = elem_bytes == 4 ? 12u : 11u;
  if (grid < 1) grid = 1;
  if (grid > kRwBlocks) grid = kRwBlocks;
  const bool fused = n <= kServeFusedItems;
  const size_t lds = fused ? (n + 1) * sizeof(uint64_t) : 0;
  if (!fused)
    hipLaunchKernelGGL(batch_top_kernel<ServeItem>, dim3(1), dim3(kScanThreads), 0, s, items, n, tile_begin,
                       elem_begin);
  if (elem_bytes == 4) {
    if (fused)
      hipLaunchKernelGGL((serve_stream_kernel<uint32_t, true>), dim3(grid), dim3(kRwThreads), lds, s, items,
                         tile_begin, n, err, te_log2);
    else
      hipLaunchKernelGGL((serve_stream_kernel<uint32_t, false>), dim3(grid), dim3(kRwThreads), 0, s, items,
                         tile_begin, n, err, te_log2);
  } else {
    if (fused)
      hipLaunchKernelGGL((serve_stream_kernel<uint64_t, true>), dim3(grid), dim3(kRwThreads), lds, s, items,
                         tile_begin, n, err, te_log2);
    else
      hipLaunchKernelGGL((serve_stream_kernel<uint64_t, false>), dim3(grid), dim3(kRwThreads), 0, s, items,
                         tile_begin, n, err, te_log2);
  }
  return hip_status(hipGetLastError());
}

int launch_scan(ggarray* a, hipStream_t s, uint64_t* copy) {
  const uint32_t te_log2 = 14u - a->elem_log2;
  if (a->V <= 4 * kScanThreads) {  // one workgroup, a few LFVectors per thread
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, s, a->ref, te_log2, copy);
  } else {  // one workgroup per 1024 LFVectors, two passes
    const uint32_t chunks = (a->V + kScanThreads - 1) / kScanThreads;
    hipLaunchKernelGGL(scan_chunks_kernel, dim3(chunks), dim3(kScanThreads), 0, s, a->ref, a->scan_tot, te_log2);
    hipLaunchKernelGGL(scan_fix_kernel, dim3(chunks), dim3(kScanThreads), 0, s, a->ref, a->scan_tot, chunks, copy);
  }
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    a->prefix_valid = true;
    a->scan_tag = stream_capture_tag(s);
  }
  return hip_status(e);
}

int launch_shrink(ggarray* a, uint32_t num, uint32_t den, hipStream_t s) {
  if (num == den) a->size_ub = 0;
  const uint32_t blocks = (a->V + kVecPerBlock - 1) / kVecPerBlock;
  hipLaunchKernelGGL(shrink_kernel, dim3(blocks), dim3(256), 0, s, a->ref, num, den, a->elem_log2);
  sizes_changed(a, s);
  return hip_status(hipGetLastError());
}

int launch_free_all(ggarray* a, hipStream_t s) {
  const uint32_t blocks = (a->V + kVecPerBlock - 1) / kVecPerBlock;
  hipLaunchKernelGGL(free_all_kernel, dim3(blocks), dim3(256), 0, s, a->ref, a->elem_log2);
  return hip_status(hipGetLastError());
}

int launch_capacity(ggarray* a, uint64_t* d_out, hipStream_t s) {
  if (hipMemsetAsync(d_out, 0, sizeof(uint64_t), s) != hipSuccess) return GGA_EHIP;
  const uint32_t blocks = (a->V + 255) / 256;
  hipLaunchKernelGGL(capacity_kernel, dim3(blocks), dim3(256), 0, s, a->ref, d_out);
  return hip_status(hipGetLastError());
}

// Builds the tile table for the current sizes (the prefix must be current).
// Under graph capture it is always rebuilt, inside the graph, and never grown.
static int ensure_table(ggarray* a, hipStream_t s) {
  const uint64_t tag = stream_capture_tag(s);
  const bool cap_mode = tag != 0;
  if (a->tab_gen == a->sizes_gen && capture_reuse(a, a->tab_tag, tag)) return GGA_OK;
  const uint32_t te_log2 = 14u - a->elem_log2;
  const uint64_t ub = a->size_ub;
  // Tiles of an LFVector of s elements: at most s / te + one partial tile per bucket.
  // With the sizes unknown to the host (after device-side pushes) the table is not grown.
  uint64_t need = a->tab_cap;
  if (ub < (1ull << 40)) {
    need = (ub >> te_log2) + (uint64_t)a->V * (nbuckets_for(a->log2F, ub) + 1);
    if (need > kTableMaxTiles) need = kTableMaxTiles;
  }
  if (need > a->tab_cap && !cap_mode) {
    uint64_t ncap = a->tab_cap * 2 > need ? a->tab_cap * 2 : need;
    if (ncap > kTableMaxTiles) ncap = kTableMaxTiles;
    void* p = nullptr;
    if (hipMallocAsync(&p, 16 * ncap, s) == hipSuccess) {
      if (retire_buffer(a, a->tile_tab, s) != GGA_OK) return GGA_EHIP;
      a->retired_tab_bytes += 16 * a->tab_cap;
      a->tile_tab = static_cast<uint64_t*>(p);
      a->tab_cap = ncap;
    } else {
      (void)hipGetLastError();  // keep the smaller table; a larger array walks its buckets
    }
  }
  if (a->tab_cap) {
    hipLaunchKernelGGL(tile_table_kernel, dim3((a->V + kVecPerBlock - 1) / kVecPerBlock), dim3(256), 0, s, a->ref,
                       a->tile_tab, a->tab_cap, te_log2, a->elem_log2);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_status(e);
  }
  a->tab_gen = a->sizes_gen;
  a->tab_tag = tag;
  return GGA_OK;
}

// The table to stream through (its capacity 0: walk the buckets), built if needed.
static int stream_source(ggarray* a, hipStream_t s, const uint64_t** tab, uint64_t* cap) {
  *tab = nullptr;
  *cap = 0;
  if ((a->size_ub >> (14u - a->elem_log2)) < kTableMinTiles) return GGA_OK;
  const int rc = ensure_table(a, s);
  if (rc) return rc;
  *tab = a->tile_tab;
  *cap = a->tab_cap;
  return GGA_OK;
}

// Launches an r/w (kind 0) or flatten (kind 1) kernel.  With kernel timing on and
// the stream not capturing, the dispatch itself records the array's start and end
// events of that kind, so they bracket the kernel alone.
template <typename... Args, typename F>
static void launch_streaming(ggarray* a, uint32_t kind, F kernel, dim3 grid, dim3 block, hipStream_t s,
                             Args... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (a->tev[kind][0] && !stream_capturing(s)) {
    e0 = a->tev[kind][0];
    e1 = a->tev[kind][1];
    a->tev_set |= 1u << kind;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, args...);
}

int launch_rw(ggarray* a, uint32_t op, hipStream_t s) {
  const uint64_t* tab;
  uint64_t tcap;
  const int rc = stream_source(a, s, &tab, &tcap);
  if (rc) return rc;
  const uint32_t te_log2 = 14u - a->elem_log2;
  const dim3 grid(stream_grid(a, tcap ? kTableBlocks : kRwBlocks)), block(kRwThreads);
  const bool nt = a->last_rw_gen == a->sizes_gen + 1;  // the array's previous streaming call was an r/w
  if (a->elem_bytes == 4) {
    if (nt)
      launch_streaming(a, 0, stream_table_kernel<uint32_t, false, true>, grid, block, s, a->ref, tab, tcap, op,
                       (uint32_t*)nullptr, (uint64_t)0, te_log2);
    else
      launch_streaming(a, 0, stream_table_kernel<uint32_t, false>, grid, block, s, a->ref, tab, tcap, op,
                       (uint32_t*)nullptr, (uint64_t)0, te_log2);
  } else {
    if (nt)
      launch_streaming(a, 0, stream_table_kernel<uint64_t, false, true>, grid, block, s, a->ref, tab, tcap, op,
                       (uint64_t*)nullptr, (uint64_t)0, te_log2);
    else
      launch_streaming(a, 0, stream_table_kernel<uint64_t, false>, grid, block, s, a->ref, tab, tcap, op,
                       (uint64_t*)nullptr, (uint64_t)0, te_log2);
  }
  a->last_rw_gen = a->sizes_gen + 1;
  return hip_status(hipGetLastError());
}

int launch_flatten(ggarray* a, void* out, uint64_t cap, hipStream_t s) {
  const uint64_t* tab;
  uint64_t tcap;
  const int rc = stream_source(a, s, &tab, &tcap);
  if (rc) return rc;
  a->last_rw_gen = 0;
  const uint32_t te_log2 = 14u - a->elem_log2;
  const dim3 grid(stream_grid(a, tcap ? kTableBlocks : kFlattenBlocks)), block(kRwThreads);
  if (a->elem_bytes == 4)
    launch_streaming(a, 1, stream_table_kernel<uint32_t, true>, grid, block, s, a->ref, tab, tcap, 0u,
                     static_cast<uint32_t*>(out), cap, te_log2);
  else
    launch_streaming(a, 1, stream_table_kernel<uint64_t, true>, grid, block, s, a->ref, tab, tcap, 0u,
                     static_cast<uint64_t*>(out), cap, te_log2);
  return hip_status(hipGetLastError());
}

// The static array's r/w in the GGArray's launch shape: one workgroup per 16 KiB
// tile of the host's bound of its size (up to kTableBlocks, looping beyond) and
// the same load policy, so that only the layout differs.  (A grid sized for the
// capacity dispatches a workgroup per empty tile: 2^30-element capacity holding
// 6.25e7 elements streamed at 5.0 TB/s against 6.35 for the same bytes sized to
// fit.)
int launch_static_rw(gga_static* st, uint32_t op, hipStream_t s) {
  const uint32_t te_log2 = st->elem_bytes == 4 ? 12u : 11u;
  const uint64_t ub = st->size_ub < st->cap ? st->size_ub : st->cap;
  const uint64_t tiles = (ub + (1ull << te_log2) - 1) >> te_log2;
  const dim3 grid(xcd_grid(tiles > kTableBlocks ? kTableBlocks : tiles)), block(kRwThreads);
  const bool nt = st->rw_last;
  if (st->elem_bytes == 4) {
    if (nt)
      hipLaunchKernelGGL((static_rw_kernel<uint32_t, true>), grid, block, 0, s, static_cast<uint32_t*>(st->data),
                         st->d_size, st->cap, op, te_log2);
    else
      hipLaunchKernelGGL((static_rw_kernel<uint32_t, false>), grid, block, 0, s, static_cast<uint32_t*>(st->data),
                         st->d_size, st->cap, op, te_log2);
  } else {
    if (nt)
      hipLaunchKernelGGL((static_rw_kernel<uint64_t, true>), grid, block, 0, s, static_cast<uint64_t*>(st->data),
                         st->d_size, st->cap, op, te_log2);
    else
      hipLaunchKernelGGL((static_rw_kernel<uint64_t, false>), grid, block, 0, s, static_cast<uint64_t*>(st->data),
                         st->d_size, st->cap, op, te_log2);
  }
  st->rw_last = true;
  return hip_status(hipGetLastError());
}


// Sum of the member arrays' size generations: unchanged exactly when no member's
// sizes can have changed since it was last taken.
static uint64_t batch_gen(const gga_batch* b) {
  uint64_t g = 0;
  for (uint32_t i = 0; i < b->n; ++i) g += b->arrays[i]->sizes_gen;
  return g;
}

// capture_reuse for a batch: eager reuse also needs that no graph changes the
// sizes of any member.
static bool batch_reuse(const gga_batch* b, uint64_t built, uint64_t now) {
  if (built != now || now == ~0ull) return false;
  if (now == 0)
    for (uint32_t i = 0; i < b->n; ++i)
      if (b->arrays[i]->graph_sized) return false;
  return true;
}

int launch_batch_scan(gga_batch* b, hipStream_t s) {
  const uint64_t gen = batch_gen(b);
  const uint64_t tag = stream_capture_tag(s);
  if (b->scan_valid && b->scan_gen == gen && batch_reuse(b, b->scan_tag, tag)) return GGA_OK;
  const uint32_t te_log2 = b->elem_bytes == 4 ? 12u : 11u;
  hipLaunchKernelGGL(batch_scan_kernel, dim3(b->n), dim3(kScanThreads), 0, s, b->d_arrays, te_log2);
  hipLaunchKernelGGL(batch_top_kernel<BatchArr>, dim3(1), dim3(kScanThreads), 0, s, b->d_arrays, b->n,
                     b->d_tile_begin, b->d_elem_begin);
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    for (uint32_t i = 0; i < b->n; ++i) {
      b->arrays[i]->prefix_valid = true;
      b->arrays[i]->scan_tag = tag;
    }
    b->scan_valid = true;
    b->scan_gen = gen;
    b->scan_tag = tag;
  }
  return hip_status(e);
}

// The batch's tile table for the current sizes (after launch_batch_scan); like
// the single-array table it is grown only outside graph capture, retired rather
// than freed, and always rebuilt under capture.  *tab / *tcap: what to stream
// through (capacity 0: the persistent walk).
static int ensure_batch_table(gga_batch* b, hipStream_t s, const uint64_t** tab, uint64_t* tcap, uint64_t* bound) {
  const uint32_t te_log2 = b->elem_bytes == 4 ? 12u : 11u;
  uint64_t need = 0;
  bool known = true;
  for (uint32_t i = 0; i < b->n; ++i) {
    const ggarray* a = b->arrays[i];
    if (a->size_ub >= (1ull << 40)) known = false;
    else need += (a->size_ub >> te_log2) + (uint64_t)a->V * (nbuckets_for(a->log2F, a->size_ub) + 1);
  }
  *bound = known ? need : kTableMaxTiles;
  *tab = nullptr;
  *tcap = 0;
  if (known && need < kTableMinTiles) return GGA_OK;
  if (!known) need = b->tab_cap;
  if (need > kTableMaxTiles) need = kTableMaxTiles;
  const uint64_t tag = stream_capture_tag(s);
  const bool cap_mode = tag != 0;
  const uint64_t gen = batch_gen(b);
  if (!(b->tab_valid && b->tab_gen == gen && batch_reuse(b, b->tab_tag, tag))) {
    if (need > b->tab_cap && !cap_mode) {
      uint64_t ncap = b->tab_cap * 2 > need ? b->tab_cap * 2 : need;
      if (ncap > kTableMaxTiles) ncap = kTableMaxTiles;
      void* p = nullptr;
      if (hipMalloc(&p, 16 * ncap) == hipSuccess) {  // freed with hipFree when the batch is destroyed
        if (b->tile_tab) {
          if (b->n_retired < sizeof(b->retired) / sizeof(b->retired[0])) b->retired[b->n_retired++] = b->tile_tab;
          else if (hipFree(b->tile_tab) != hipSuccess) return GGA_EHIP;  // waits for the device
        }
        b->tile_tab = static_cast<uint64_t*>(p);
        b->tab_cap = ncap;
      } else {
        (void)hipGetLastError();
      }
    }
    if (b->tab_cap) {
      hipLaunchKernelGGL(batch_table_kernel, dim3((uint32_t)((b->total_vectors + kVecPerBlock - 1) / kVecPerBlock)),
                         dim3(256), 0, s, b->d_arrays, b->d_vbegin, b->d_tile_begin, b->d_elem_begin, b->n,
                         b->tile_tab, b->tab_cap, te_log2);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_status(e);
    }
    b->tab_valid = true;
    b->tab_gen = gen;
    b->tab_tag = tag;
  }
  *tab = b->tile_tab;
  *tcap = b->tab_cap;
  return GGA_OK;
}

int launch_batch_shrink(gga_batch* b, uint32_t num, uint32_t den, hipStream_t s) {
  if (num == den)
    for (uint32_t i = 0; i < b->n; ++i) b->arrays[i]->size_ub = 0;
  const uint64_t blocks = (b->total_vectors + kVecPerBlock - 1) / kVecPerBlock;
  hipLaunchKernelGGL(batch_shrink_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, b->d_arrays, b->d_vbegin,
                     b->n, num, den);
  for (uint32_t i = 0; i < b->n; ++i) sizes_changed(b->arrays[i], s);
  return hip_status(hipGetLastError());
}

int launch_batch_stream(gga_batch* b, uint32_t op, void* out, uint64_t cap, bool flatten, hipStream_t s) {
  const uint32_t te_log2 = b->elem_bytes == 4 ? 12u : 11u;
  const uint64_t* tab;
  uint64_t tcap, bound;
  const int rc = ensure_batch_table(b, s, &tab, &tcap, &bound);
  if (rc) return rc;
  uint64_t g = b->stream_blocks;
  if (!g) g = tcap ? (bound < kTableBlocks ? bound : kTableBlocks) : (flatten ? kFlattenBlocks : kRwBlocks);
  const dim3 grid(tcap ? xcd_grid(g) : (uint32_t)g), block(kRwThreads);
  if (b->elem_bytes == 4) {
    if (flatten)
      hipLaunchKernelGGL((batch_stream_kernel<uint32_t, true>), grid, block, 0, s, b->d_arrays, b->d_tile_begin,
                         b->d_elem_begin, b->n, tab, tcap, 0u, static_cast<uint32_t*>(out), cap, b->d_err, te_log2);
    else
      hipLaunchKernelGGL((batch_stream_kernel<uint32_t, false>), grid, block, 0, s, b->d_arrays, b->d_tile_begin,
                         b->d_elem_begin, b->n, tab, tcap, op, (uint32_t*)nullptr, (uint64_t)0, b->d_err, te_log2);
  } else {
    if (flatten)
      hipLaunchKernelGGL((batch_stream_kernel<uint64_t, true>), grid, block, 0, s, b->d_arrays, b->d_tile_begin,
                         b->d_elem_begin, b->n, tab, tcap, 0u, static_cast<uint64_t*>(out), cap, b->d_err, te_log2);
    else
      hipLaunchKernelGGL((batch_stream_kernel<uint64_t, false>), grid, block, 0, s, b->d_arrays, b->d_tile_begin,
                         b->d_elem_begin, b->n, tab, tcap, op, (uint64_t*)nullptr, (uint64_t)0, b->d_err, te_log2);
  }
  return hip_status(hipGetLastError());
}

}  // namespace gga
