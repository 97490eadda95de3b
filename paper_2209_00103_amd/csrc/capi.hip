// C ABI of the GGArray library: argument validation, object lifetimes, error
// reporting, and the host-driven resize of the semi-static baseline.
#include <cstddef>
#include <new>

#include <cstdio>
#include <cstring>

#include "gga_internal.h"

using namespace gga;

namespace {

hipStream_t S(gga_stream s) { return static_cast<hipStream_t>(s); }
bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }
uint32_t ilog2(uint64_t x) { return 63u - (uint32_t)__builtin_clzll(x); }

int map_device_error(uint32_t e) {
  if (e == 0) return GGA_OK;
  if (e == kErrNoMem) return GGA_ENOMEM;
  if (e == kErrRange) return GGA_ERANGE;
  return GGA_EHIP;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) & ~(a - 1); }

// The last failing HIP call of this thread, for gga_last_hip_error.
thread_local char g_hip_error[192] = "";
int hip_fail(hipError_t e, const char* what) {
  std::snprintf(g_hip_error, sizeof(g_hip_error), "%s: %s (%d)", what, hipGetErrorName(e), (int)e);
  (void)hipGetLastError();  // clear it, so that a later launch check does not report it again
  return GGA_EHIP;
}

// Per-array host scratch for synchronising reads (pinned, so copies are async).
struct Pinned {
  uint64_t* p = nullptr;
  int init() { return hipHostMalloc(reinterpret_cast<void**>(&p), 64, hipHostMallocDefault) == hipSuccess ? GGA_OK : GGA_EHIP; }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
  }
};

struct ArrayExtra {
  Pinned pin;
  uint64_t* d_scratch;
};

int check_gen(const gga_gen* g, uint64_t n_threads, uint32_t* mode, uint32_t* maxc) {
  if (!g || g->seed >= 256) return GGA_EINVAL;
  switch (g->kind) {
    case GGA_GEN_BERNOULLI:
      if (g->round >= 256) return GGA_EINVAL;
      *mode = kModeBernoulli;
      *maxc = 1;
      return GGA_OK;
    case GGA_GEN_ROUND_TAG:
      if (g->tag_shift >= 64) return GGA_EINVAL;
      *mode = kModeRoundTag;
      *maxc = 1;
      return GGA_OK;
    case GGA_GEN_POISSON:
      if (g->round >= 8 || g->max_count == 0 || g->max_count > 16) return GGA_EINVAL;
      *mode = kModePoisson;
      *maxc = g->max_count;
      return GGA_OK;
    case GGA_GEN_KEYED:
      if (g->round >= 256 || g->tag_shift < 1 || g->tag_shift > 47 || (g->tag >> (48 - g->tag_shift)) != 0 ||
          n_threads > (1ull << g->tag_shift))
        return GGA_EINVAL;
      *mode = kModeKeyed;
      *maxc = 1;
      return GGA_OK;
    default:
      return GGA_EINVAL;
  }
}

InsertDesc gen_desc(const gga_gen* g, uint32_t mode, uint64_t n) {
  InsertDesc d{};
  d.mode = mode;
  d.n_threads = n;
  d.seed = g->seed;
  d.round = g->round;
  d.tag_shift = g->tag_shift;
  d.max_count = g->max_count;
  for (int k = 0; k < 16; ++k) d.thresholds[k] = g->thresholds[k];
  d.tag = g->tag;
  return d;
}

}  // namespace

// The host part of an array keeps a pointer to its extra host state right after
// the public struct.
struct ggarray_full {
  ggarray a;
  ArrayExtra x;
};

extern "C" {

const char* gga_last_hip_error(void) { return g_hip_error; }

const char* gga_strerror(int status) {
  switch (status) {
    case GGA_OK: return "ok";
    case GGA_EINVAL: return "invalid argument";
    case GGA_ENOMEM: return "bucket pool exhausted";
    case GGA_ERANGE: return "output or capacity too small";
    case GGA_EHIP: return "HIP runtime error";
    case GGA_EBUSY: return "object still in use";
    default: return "unknown status";
  }
}

// ---------------------------------------------------------------------- pool --
int gga_pool_create(gga_pool** out, void* dev_base, uint64_t bytes, gga_stream s) {
  if (!out || !dev_base || (reinterpret_cast<uintptr_t>(dev_base) & 255u) || bytes < kPoolHdrBytes + (1u << 20))
    return GGA_EINVAL;
  *out = nullptr;
  gga_pool* p = new (std::nothrow) gga_pool();
  if (!p) return GGA_EHIP;
  p->dev_base = dev_base;
  p->bytes = bytes;
  p->ref.hdr = static_cast<PoolHdr*>(dev_base);
  p->ref.base = static_cast<uint8_t*>(dev_base) + kPoolHdrBytes;
  PoolHdr* h = new (std::nothrow) PoolHdr();
  if (!h) {
    delete p;
    return GGA_EHIP;
  }
  h->limit = (bytes - kPoolHdrBytes) & ~255ull;
  // Arena chunks: about 1/1024 of the region, between 64 KiB and 16 MiB.
  uint64_t clog = 16;
  while (clog < 24 && (2ull << clog) <= h->limit / 1024) ++clog;
  h->chunk_log2 = clog;
  const bool ok = hipMemcpyAsync(p->ref.hdr, h, sizeof(PoolHdr), hipMemcpyHostToDevice, S(s)) == hipSuccess &&
                  hipStreamSynchronize(S(s)) == hipSuccess;
  delete h;
  if (!ok) {
    delete p;
    return GGA_EHIP;
  }
  *out = p;
  return GGA_OK;
}

int gga_pool_destroy(gga_pool* p) {
  if (!p) return GGA_EINVAL;
  if (p->n_arrays) return GGA_EBUSY;
  delete p;
  return GGA_OK;
}

int gga_pool_stats(gga_pool* p, uint64_t out[7], gga_stream s) {
  if (!p || !out) return GGA_EINVAL;
  PoolHdr* h = new (std::nothrow) PoolHdr();
  if (!h) return GGA_EHIP;
  if (hipMemcpyAsync(h, p->ref.hdr, sizeof(PoolHdr), hipMemcpyDeviceToHost, S(s)) != hipSuccess ||
      hipStreamSynchronize(S(s)) != hipSuccess) {
    delete h;
    return GGA_EHIP;
  }
  uint64_t in_use = 0, n_alloc = 0, n_free = 0;
  for (int k = 0; k < kArenaShards; ++k) {  // per-shard counters wrap individually; the sums do not
    in_use += h->shard[k].in_use;
    n_alloc += h->shard[k].n_alloc;
    n_free += h->shard[k].n_free;
  }
  // Failed claims leave the bump pointer past the limit: carved bytes stop there.
  const uint64_t carved = h->bump < h->limit ? h->bump : h->limit;
  out[0] = in_use;
  out[1] = carved;
  out[2] = n_alloc;
  out[3] = n_free;
  out[4] = carved;
  out[5] = h->limit;
  out[6] = h->n_attempt;
  delete h;
  return GGA_OK;
}

int gga_pool_set_fault(gga_pool* p, uint64_t fault_at, gga_stream s) {
  if (!p) return GGA_EINVAL;
  uint64_t v[2] = {0, fault_at};  // n_attempt, fault_at are adjacent
  static_assert(offsetof(PoolHdr, fault_at) == offsetof(PoolHdr, n_attempt) + 8, "layout");
  if (hipMemcpyAsync(&p->ref.hdr->n_attempt, v, sizeof(v), hipMemcpyHostToDevice, S(s)) != hipSuccess ||
      hipStreamSynchronize(S(s)) != hipSuccess)
    return GGA_EHIP;
  return GGA_OK;
}

int ggarray_set_spin_limit(ggarray* a, uint32_t polls) {
  if (!a) return GGA_EINVAL;
  a->ref.spin = polls ? polls : gga::kSpinLimit;
  return GGA_OK;
}

// ------------------------------------------------------------------- GGArray --
int ggarray_create(ggarray** out, gga_pool* p, uint32_t elem_bytes, uint32_t n_vectors,
                   uint64_t first_bucket, gga_stream s) {
  if (!out) return GGA_EINVAL;
  *out = nullptr;
  if (!p || (elem_bytes != 4 && elem_bytes != 8) || n_vectors == 0 || n_vectors > (1u << 20) ||
      !is_pow2(first_bucket) || first_bucket > (1ull << 32))
    return GGA_EINVAL;
  ggarray_full* f = new (std::nothrow) ggarray_full();
  if (!f) return GGA_EHIP;
  ggarray* a = &f->a;
  a->pool = p;
  a->elem_bytes = elem_bytes;
  a->elem_log2 = elem_bytes == 4 ? 2 : 3;
  a->V = n_vectors;
  a->log2F = ilog2(first_bucket);
  const uint64_t V = n_vectors;
  size_t off = 0;
  const size_t o_size = off;       off = align_up(off + 8 * V, 256);
  const size_t o_bptr = off;       off = align_up(off + 8 * V * kMaxBuckets, 256);
  const size_t o_dead = off;       off = align_up(off + 4 * V, 256);
  const size_t o_done = off;       off = align_up(off + 4 * V, 256);
  const size_t o_prefix = off;     off = align_up(off + 8 * (V + 1), 256);
  const size_t o_tprefix = off;    off = align_up(off + 8 * (V + 1), 256);
  const size_t o_vticket = off;    off = align_up(off + 8 * V, 256);
  const size_t o_rbase = off;      off = align_up(off + 8 * V, 256);
  const size_t o_misc = off;       off = align_up(off + 64, 256);  // err, scratch
  const size_t o_stot = off;       off = align_up(off + 16 * ((V + 1023) / 1024), 256);  // scan chunk totals
  if (hipMalloc(&a->meta, off) != hipSuccess) {
    delete f;
    return GGA_EHIP;
  }
  if (hipMemsetAsync(a->meta, 0, off, S(s)) != hipSuccess || f->x.pin.init() != GGA_OK) {
    (void)hipFree(a->meta);
    f->x.pin.release();
    delete f;
    return GGA_EHIP;
  }
  uint8_t* m = static_cast<uint8_t*>(a->meta);
  ArrRef& R = a->ref;
  R.size = reinterpret_cast<uint64_t*>(m + o_size);
  R.bptr = reinterpret_cast<uint64_t*>(m + o_bptr);
  R.dead = reinterpret_cast<uint32_t*>(m + o_dead);
  R.alloc_done = reinterpret_cast<uint32_t*>(m + o_done);
  R.prefix = reinterpret_cast<uint64_t*>(m + o_prefix);
  R.tprefix = reinterpret_cast<uint64_t*>(m + o_tprefix);
  R.err = reinterpret_cast<uint32_t*>(m + o_misc);
  R.vticket = reinterpret_cast<uint64_t*>(m + o_vticket);
  R.rbase = reinterpret_cast<uint64_t*>(m + o_rbase);
  f->x.d_scratch = reinterpret_cast<uint64_t*>(m + o_misc + 16);
  a->scan_tot = reinterpret_cast<uint64_t*>(m + o_stot);
  R.status = nullptr;
  R.pool = p->ref;
  R.V = n_vectors;
  R.log2F = a->log2F;
  R.salt = p->next_salt & (kFreeShards - 1);  // arrays created in a row: consecutive shards
  p->next_salt += n_vectors;
  R.spin = kSpinLimit;
  a->status_cap = 0;
  a->prefix_valid = true;  // all sizes zero and prefix arrays zeroed
  a->size_ub = 0;
  a->tile_tab = nullptr;
  a->tab_cap = 0;
  a->sizes_gen = 0;
  a->tab_gen = ~0ull;
  a->n_retired = 0;
  a->last_rw_gen = 0;
  a->scan_tag = 0;
  a->tab_tag = 0;
  a->graph_sized = false;
  for (auto& k : a->tev) k[0] = k[1] = nullptr;
  a->tev_set = 0;
  a->meta_bytes = off;
  a->retired_tab_bytes = 0;
  a->pk_off = nullptr;
  a->pk_cap = 0;
  p->n_arrays += 1;
  *out = a;
  return GGA_OK;
}

int ggarray_destroy(ggarray* a, gga_stream s) {
  if (!a) return GGA_EINVAL;
  ggarray_full* f = reinterpret_cast<ggarray_full*>(a);
  int rc = launch_free_all(a, S(s));
  if (a->ref.status && hipFreeAsync(a->ref.status, S(s)) != hipSuccess) rc = GGA_EHIP;
  if (a->tile_tab && hipFreeAsync(a->tile_tab, S(s)) != hipSuccess) rc = GGA_EHIP;
  if (a->pk_off && hipFreeAsync(a->pk_off, S(s)) != hipSuccess) rc = GGA_EHIP;
  for (uint32_t i = 0; i < a->n_retired; ++i)
    if (hipFreeAsync(a->retired[i], S(s)) != hipSuccess) rc = GGA_EHIP;
  if (hipStreamSynchronize(S(s)) != hipSuccess) rc = GGA_EHIP;
  if (hipFree(a->meta) != hipSuccess) rc = GGA_EHIP;
  for (auto& k : a->tev)
    for (hipEvent_t& e : k)
      if (e && hipEventDestroy(e) != hipSuccess) rc = GGA_EHIP;
  f->x.pin.release();
  a->pool->n_arrays -= 1;
  delete f;
  return rc;
}

int ggarray_insert(ggarray* a, const void* values, const uint8_t* flags, uint64_t n_threads,
                   gga_stream s) {
  if (!a || (n_threads && !values)) return GGA_EINVAL;
  InsertDesc d{};
  d.mode = kModeBuffer;
  d.values = values;
  d.flags = flags;
  d.max_count = 1;
  d.n_threads = n_threads;
  return launch_insert(a, d, S(s));
}

int ggarray_insert_counts(ggarray* a, const void* values, const uint8_t* counts, uint32_t max_count,
                          uint64_t n_threads, gga_stream s) {
  if (!a || max_count == 0 || max_count > 16 || (n_threads && (!values || !counts)))
    return GGA_EINVAL;
  InsertDesc d{};
  d.mode = kModeCounts;
  d.values = values;
  d.flags = counts;
  d.max_count = max_count;
  d.n_threads = n_threads;
  return launch_insert(a, d, S(s));
}

int ggarray_insert_packed(ggarray* a, const void* values, uint64_t n_values, const uint8_t* counts,
                          uint64_t n_threads, gga_stream s) {
  if (!a || (n_threads && !counts) || (n_values && !values)) return GGA_EINVAL;
  return launch_insert_packed(a, values, counts, n_threads, n_values, S(s));
}

int ggarray_insert_packed_noalloc(ggarray* a, const void* values, uint64_t n_values, const uint8_t* counts,
                                  uint64_t n_threads, gga_stream s) {
  if (!a || (n_threads && !counts) || (n_values && !values)) return GGA_EINVAL;
  return launch_insert_packed_noalloc(a, values, counts, n_threads, n_values, S(s));
}

int ggarray_insert_gen(ggarray* a, const gga_gen* g, uint64_t n_threads, gga_stream s) {
  uint32_t mode = 0, maxc = 0;
  if (!a) return GGA_EINVAL;
  const int rc = check_gen(g, n_threads, &mode, &maxc);
  if (rc) return rc;
  const InsertDesc d = gen_desc(g, mode, n_threads);
  return launch_insert(a, d, S(s));
}

int ggarray_kernel_timing(ggarray* a, uint32_t on) {
  if (!a) return GGA_EINVAL;
  if (!on) {
    for (auto& k : a->tev)
      for (hipEvent_t& e : k) {
        if (e && hipEventDestroy(e) != hipSuccess) return GGA_EHIP;
        e = nullptr;
      }
    a->tev_set = 0;
    return GGA_OK;
  }
  for (auto& k : a->tev)
    for (hipEvent_t& e : k)
      if (!e && hipEventCreate(&e) != hipSuccess) return GGA_EHIP;
  return GGA_OK;
}

int ggarray_kernel_ms(ggarray* a, uint32_t kind, float* ms) {
  if (!a || kind > 2 || !ms || !(a->tev_set >> kind & 1u)) return GGA_EINVAL;
  if (hipEventSynchronize(a->tev[kind][1]) != hipSuccess) return GGA_EHIP;
  return hip_status(hipEventElapsedTime(ms, a->tev[kind][0], a->tev[kind][1]));
}

int ggarray_insert_gen_shrink(ggarray* a, const gga_gen* g, uint64_t n_threads, uint32_t num, uint32_t den,
                              gga_stream s) {
  uint32_t mode = 0, maxc = 0;
  if (!a || den == 0 || num > den) return GGA_EINVAL;
  const int rc = check_gen(g, n_threads, &mode, &maxc);
  if (rc) return rc;
  const InsertDesc d = gen_desc(g, mode, n_threads);
  return launch_insert(a, d, S(s), num, den);
}

int ggarray_insert_gen_rounds(ggarray* a, const gga_gen* gens, const uint64_t* n_threads, uint32_t n_rounds,
                              uint32_t num, uint32_t den, uint32_t clear_first, gga_stream s) {
  if (!a || den == 0 || num > den || n_rounds > GGA_MAX_ROUNDS || (n_rounds && (!gens || !n_threads)))
    return GGA_EINVAL;
  InsertDesc ds[GGA_MAX_ROUNDS];
  for (uint32_t r = 0; r < n_rounds; ++r) {
    uint32_t mode = 0, maxc = 0;
    const int rc = check_gen(&gens[r], n_threads[r], &mode, &maxc);
    if (rc) return rc;
    ds[r] = gen_desc(&gens[r], mode, n_threads[r]);
  }
  return launch_insert_rounds(a, ds, n_rounds, S(s), num, den, clear_first != 0);
}

int ggarray_insert_segments(ggarray* a, const void* values, const uint64_t* prefix, uint64_t n_values,
                            gga_stream s) {
  if (!a || !prefix || (n_values && !values)) return GGA_EINVAL;
  return launch_insert_segments(a, values, prefix, n_values, S(s));
}

int ggarray_shrink(ggarray* a, uint32_t num, uint32_t den, gga_stream s) {
  if (!a || den == 0 || num > den) return GGA_EINVAL;
  if (num == 0) return GGA_OK;
  return launch_shrink(a, num, den, S(s));
}

// A prefix is reused only where it was built: eagerly for eager calls, in the
// same capture for captured calls, so that a replay never reads a prefix left
// over from before its capture.
static int ensure_prefix(ggarray* a, hipStream_t s) {
  return a->prefix_valid && capture_reuse(a, a->scan_tag, stream_capture_tag(s)) ? GGA_OK : launch_scan(a, s);
}

int ggarray_rw(ggarray* a, uint32_t op, gga_stream s) {
  if (!a || op > GGA_ADD1_X30) return GGA_EINVAL;
  int rc = ensure_prefix(a, S(s));
  return rc ? rc : launch_rw(a, op, S(s));
}

int ggarray_rw_global(ggarray* a, uint32_t op, gga_stream s) {
  if (!a || op > GGA_ADD1_X30) return GGA_EINVAL;
  int rc = ensure_prefix(a, S(s));
  return rc ? rc : launch_rw_global(a, op, S(s));
}

int ggarray_gather(ggarray* a, const uint64_t* idx, uint64_t n, void* out, gga_stream s) {
  if (!a || (n && (!idx || !out))) return GGA_EINVAL;
  int rc = ensure_prefix(a, S(s));
  return rc ? rc : launch_gather(a, idx, n, out, S(s));
}

int ggarray_flatten(ggarray* a, void* out, uint64_t out_cap_elems, gga_stream s) {
  if (!a || (!out && out_cap_elems)) return GGA_EINVAL;
  int rc = ensure_prefix(a, S(s));
  return rc ? rc : launch_flatten(a, out, out_cap_elems, S(s));
}

static int read_back(ggarray* a, const uint64_t* dev_word, uint64_t* out_host, hipStream_t s) {
  ggarray_full* f = reinterpret_cast<ggarray_full*>(a);
  uint64_t* h = f->x.pin.p;
  if (dev_word && hipMemcpyAsync(h, dev_word, 8, hipMemcpyDeviceToHost, s) != hipSuccess) return GGA_EHIP;
  if (hipMemcpyAsync(h + 1, a->ref.err, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return GGA_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return GGA_EHIP;
  if (out_host && dev_word) *out_host = h[0];
  return map_device_error((uint32_t)h[1]);
}

int ggarray_size(ggarray* a, uint64_t* out_host, gga_stream s) {
  if (!a || !out_host) return GGA_EINVAL;
  int rc = ensure_prefix(a, S(s));
  return rc ? rc : read_back(a, a->ref.prefix + a->V, out_host, S(s));
}

int ggarray_capacity(ggarray* a, uint64_t* out_host, gga_stream s) {
  if (!a || !out_host) return GGA_EINVAL;
  ggarray_full* f = reinterpret_cast<ggarray_full*>(a);
  int rc = launch_capacity(a, f->x.d_scratch, S(s));
  return rc ? rc : read_back(a, f->x.d_scratch, out_host, S(s));
}

int ggarray_footprint(ggarray* a, uint64_t out[3]) {
  if (!a || !out) return GGA_EINVAL;
  out[0] = a->meta_bytes;
  out[1] = (a->status_cap + a->pk_cap) * sizeof(uint64_t);
  out[2] = 16 * a->tab_cap + a->retired_tab_bytes;
  return GGA_OK;
}

int ggarray_vector_sizes(ggarray* a, uint64_t* dev_out, gga_stream s) {
  if (!a || !dev_out) return GGA_EINVAL;
  return hip_status(hipMemcpyAsync(dev_out, a->ref.size, 8ull * a->V, hipMemcpyDeviceToDevice, S(s)));
}

int ggarray_prefix(ggarray* a, uint64_t* dev_out, gga_stream s) {
  if (!a || !dev_out) return GGA_EINVAL;
  if (!a->prefix_valid || !capture_reuse(a, a->scan_tag, stream_capture_tag(S(s))))
    return launch_scan(a, S(s), dev_out);  // the scan writes both
  return hip_status(hipMemcpyAsync(dev_out, a->ref.prefix, 8ull * (a->V + 1), hipMemcpyDeviceToDevice, S(s)));
}

int ggarray_last_error(ggarray* a, gga_stream s) {
  if (!a) return GGA_EINVAL;
  return read_back(a, nullptr, nullptr, S(s));
}

// ------------------------------------------------------------ device API --
int ggarray_device_ref(ggarray* a, void* out, uint64_t bytes) {
  if (!a || !out || bytes != sizeof(ArrRef)) return GGA_EINVAL;
  std::memcpy(out, &a->ref, sizeof(ArrRef));
  return GGA_OK;
}

int ggarray_device_done(ggarray* a, gga_stream s) {
  if (!a) return GGA_EINVAL;
  sizes_changed(a, S(s));
  a->size_ub = ~0ull >> 2;  // sizes unknown to the host now
  return GGA_OK;
}

// ------------------------------------------------------------------- batches --
static void batch_free(gga_batch* b) {
  if (b->d_arrays) (void)hipFree(b->d_arrays);
  if (b->d_tile_begin) (void)hipFree(b->d_tile_begin);
  if (b->h_pin) (void)hipHostFree(b->h_pin);
  for (uint32_t k = 0; k < b->n_tables; ++k) {
    (void)hipFree(b->tables[k].items);
    (void)hipFree(b->tables[k].begins);
    delete[] b->tables[k].host;
  }
  delete[] b->tables;
  if (b->tile_tab) (void)hipFree(b->tile_tab);  // hipFree waits for the device
  for (uint32_t k = 0; k < b->n_retired; ++k) (void)hipFree(b->retired[k]);
  if (b->d_varr) (void)hipFree(b->d_varr);
  if (b->d_step_sync) (void)hipFree(b->d_step_sync);
  for (uint32_t k = 0; k < b->n_step_counts; ++k) (void)hipFree(b->step_counts[k].dev);
  delete[] b->step_counts;
  delete[] b->arrays;
  delete b;
}

int gga_batch_create(gga_batch** out, ggarray* const* arrays, uint32_t n, gga_stream s) {
  if (!out) return GGA_EINVAL;
  *out = nullptr;
  if (!arrays || n == 0) return GGA_EINVAL;
  for (uint32_t i = 0; i < n; ++i) {
    if (!arrays[i] || arrays[i]->elem_bytes != arrays[0]->elem_bytes) return GGA_EINVAL;
    for (uint32_t j = 0; j < i; ++j)
      if (arrays[j] == arrays[i]) return GGA_EINVAL;
  }
  gga_batch* b = new (std::nothrow) gga_batch();
  if (!b) return GGA_EHIP;
  b->n = n;
  b->elem_bytes = arrays[0]->elem_bytes;
  b->arrays = new (std::nothrow) ggarray*[n];
  BatchArr* h = new (std::nothrow) BatchArr[n];
  if (!b->arrays || !h) {
    delete[] h;
    batch_free(b);
    return GGA_EHIP;
  }
  for (uint32_t i = 0; i < n; ++i) {
    b->arrays[i] = arrays[i];
    h[i] = BatchArr{arrays[i]->ref, 0, 0, 0, 0, i, arrays[i]->elem_log2};
  }
  const size_t words = 3 * (size_t)(n + 1) + 1;  // tile_begin, elem_begin, vbegin, error word
  bool ok = hipMalloc(&b->d_arrays, sizeof(BatchArr) * n) == hipSuccess &&
            hipMalloc(&b->d_tile_begin, sizeof(uint64_t) * words) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&b->h_pin), 64, hipHostMallocDefault) == hipSuccess;
  if (ok) {
    b->d_elem_begin = b->d_tile_begin + (n + 1);
    b->d_vbegin = b->d_elem_begin + (n + 1);
    b->d_err = reinterpret_cast<uint32_t*>(b->d_vbegin + (n + 1));
    uint64_t* vb = new (std::nothrow) uint64_t[n + 1];
    ok = vb != nullptr;
    uint32_t* varr = nullptr;
    if (ok) {
      vb[0] = 0;
      for (uint32_t i = 0; i < n; ++i) vb[i + 1] = vb[i] + arrays[i]->V;
      b->total_vectors = vb[n];
      // the batch index of every LFVector, for the persistent step
      varr = new (std::nothrow) uint32_t[vb[n]];
      ok = varr != nullptr;
      for (uint32_t i = 0; ok && i < n; ++i)
        for (uint64_t w = vb[i]; w < vb[i + 1]; ++w) varr[w] = i;
    }
    // barrier words, chunk totals, per-LFVector sizes
    const size_t step_bytes = 256 + sizeof(uint64_t) * kStepChunkMax + sizeof(uint64_t) * (ok ? vb[n] : 0);
    ok = ok && hipMalloc(&b->d_varr, sizeof(uint32_t) * vb[n]) == hipSuccess &&
         hipMalloc(&b->d_step_sync, step_bytes) == hipSuccess;
    if (ok) {
      b->d_step_chunks = reinterpret_cast<uint64_t*>(reinterpret_cast<uint8_t*>(b->d_step_sync) + 256);
      b->d_step_vsize = b->d_step_chunks + kStepChunkMax;
      ok = hipMemcpyAsync(b->d_arrays, h, sizeof(BatchArr) * n, hipMemcpyHostToDevice, S(s)) == hipSuccess &&
           hipMemsetAsync(b->d_tile_begin, 0, sizeof(uint64_t) * words, S(s)) == hipSuccess &&
           hipMemcpyAsync(b->d_vbegin, vb, sizeof(uint64_t) * (n + 1), hipMemcpyHostToDevice, S(s)) == hipSuccess &&
           hipMemcpyAsync(b->d_varr, varr, sizeof(uint32_t) * vb[n], hipMemcpyHostToDevice, S(s)) == hipSuccess &&
           hipMemsetAsync(b->d_step_sync, 0, step_bytes, S(s)) == hipSuccess &&
           hipStreamSynchronize(S(s)) == hipSuccess;
    }
    delete[] vb;
    delete[] varr;
  }
  delete[] h;
  if (!ok) {
    batch_free(b);
    return GGA_EHIP;
  }
  *out = b;
  return GGA_OK;
}

int gga_batch_destroy(gga_batch* b, gga_stream s) {
  if (!b) return GGA_EINVAL;
  const int rc = hip_status(hipStreamSynchronize(S(s)));
  batch_free(b);
  return rc;
}

int gga_batch_insert_gen(gga_batch* b, const gga_gen* g, const uint64_t* n_threads, gga_stream s) {
  uint32_t mode = 0, maxc = 0;
  if (!b || !n_threads) return GGA_EINVAL;
  const int rc = check_gen(g, 0, &mode, &maxc);
  if (rc) return rc;
  if (g->kind == GGA_GEN_KEYED) {
    if (((g->tag + b->n - 1) >> (48 - g->tag_shift)) != 0) return GGA_EINVAL;
    for (uint32_t i = 0; i < b->n; ++i)
      if (n_threads[i] > (1ull << g->tag_shift)) return GGA_EINVAL;
  }
  return launch_batch_insert(b, gen_desc(g, mode, 0), n_threads, S(s));
}

static int batch_step(gga_batch* b, const gga_gen* gens, uint32_t rounds, const uint64_t* n_threads, uint32_t op,
                      void* out, uint64_t out_cap_elems, gga_stream s, bool clear) {
  if (!b || rounds > kMaxStepRounds || (rounds && (!gens || !n_threads)) || (op > GGA_ADD1_X30 && op != GGA_RW_NONE))
    return GGA_EINVAL;
  StepDesc D{};
  D.n_rounds = rounds;
  D.clear = clear ? 1u : 0u;
  for (uint32_t r = 0; r < rounds; ++r) {
    const gga_gen* g = &gens[r];
    uint32_t mode = 0, maxc = 0;
    if (g->kind != GGA_GEN_BERNOULLI && g->kind != GGA_GEN_ROUND_TAG && g->kind != GGA_GEN_KEYED) return GGA_EINVAL;
    const int rc = check_gen(g, 0, &mode, &maxc);
    if (rc) return rc;
    if (g->kind == GGA_GEN_KEYED) {
      if (((g->tag + b->n - 1) >> (48 - g->tag_shift)) != 0) return GGA_EINVAL;
      for (uint32_t i = 0; i < b->n; ++i)
        if (n_threads[(uint64_t)r * b->n + i] > (1ull << g->tag_shift)) return GGA_EINVAL;
    }
    D.r[r] = StepRound{mode, g->round, g->seed, g->tag_shift, 0, g->tag};
  }
  // The thread counts go to the device once per distinct table; a step recorded
  // into a graph must use a table an eager step has uploaded.
  const uint64_t words = (uint64_t)rounds * b->n;
  uint64_t key = fnv1a(&rounds, sizeof(rounds), 0xCBF29CE484222325ull);
  if (words) key = fnv1a(n_threads, sizeof(uint64_t) * words, key);
  uint64_t* dev = nullptr;
  for (uint32_t k = 0; k < b->n_step_counts; ++k)
    if (b->step_counts[k].key == key) dev = b->step_counts[k].dev;
  if (!dev) {
    if (stream_capturing(S(s))) return GGA_EINVAL;
    if (b->n_step_counts == b->cap_step_counts) {
      const uint32_t ncap = b->cap_step_counts ? 2 * b->cap_step_counts : 4;
      gga_batch::StepCounts* nt = new (std::nothrow) gga_batch::StepCounts[ncap];
      if (!nt) return GGA_EHIP;
      for (uint32_t k = 0; k < b->n_step_counts; ++k) nt[k] = b->step_counts[k];
      delete[] b->step_counts;
      b->step_counts = nt;
      b->cap_step_counts = ncap;
    }
    if (hipMalloc(&dev, sizeof(uint64_t) * (words ? words : 1)) != hipSuccess) return GGA_EHIP;
    if ((words && hipMemcpyAsync(dev, n_threads, sizeof(uint64_t) * words, hipMemcpyHostToDevice, S(s)) != hipSuccess) ||
        hipStreamSynchronize(S(s)) != hipSuccess) {
      (void)hipFree(dev);
      return GGA_EHIP;
    }
    b->step_counts[b->n_step_counts++] = gga_batch::StepCounts{key, dev};
  }
  for (uint32_t i = 0; i < b->n; ++i) {
    uint64_t add = 0;
    for (uint32_t r = 0; r < rounds; ++r) add += n_threads[(uint64_t)r * b->n + i];
    if (clear) b->arrays[i]->size_ub = 0;
    grow_bound(b->arrays[i], add);
  }
  return launch_batch_step(b, D, dev, op == GGA_RW_NONE ? kOpNone : op, out, out_cap_elems, S(s));
}

int gga_batch_step(gga_batch* b, const gga_gen* gens, uint32_t rounds, const uint64_t* n_threads, uint32_t op,
                   void* out, uint64_t out_cap_elems, gga_stream s) {
  return batch_step(b, gens, rounds, n_threads, op, out, out_cap_elems, s, false);
}

int gga_batch_step_clear(gga_batch* b, const gga_gen* gens, uint32_t rounds, const uint64_t* n_threads, uint32_t op,
                         void* out, uint64_t out_cap_elems, gga_stream s) {
  return batch_step(b, gens, rounds, n_threads, op, out, out_cap_elems, s, true);
}

int gga_batch_shrink(gga_batch* b, uint32_t num, uint32_t den, gga_stream s) {
  if (!b || den == 0 || num > den) return GGA_EINVAL;
  if (num == 0) return GGA_OK;
  return launch_batch_shrink(b, num, den, S(s));
}

int gga_batch_rw(gga_batch* b, uint32_t op, gga_stream s) {
  if (!b || op > GGA_ADD1_X30) return GGA_EINVAL;
  int rc = launch_batch_scan(b, S(s));
  return rc ? rc : launch_batch_stream(b, op, nullptr, 0, false, S(s));
}

int gga_batch_flatten(gga_batch* b, void* out, uint64_t out_cap_elems, gga_stream s) {
  if (!b || (!out && out_cap_elems)) return GGA_EINVAL;
  int rc = launch_batch_scan(b, S(s));
  return rc ? rc : launch_batch_stream(b, 0, out, out_cap_elems, true, S(s));
}

int gga_batch_set_grid(gga_batch* b, uint32_t stream_blocks) {
  if (!b || stream_blocks > (1u << 20)) return GGA_EINVAL;
  b->stream_blocks = stream_blocks;
  return GGA_OK;
}

int gga_batch_offsets(gga_batch* b, uint64_t* dev_out, gga_stream s) {
  if (!b || !dev_out) return GGA_EINVAL;
  int rc = launch_batch_scan(b, S(s));
  if (rc) return rc;
  return hip_status(hipMemcpyAsync(dev_out, b->d_elem_begin, sizeof(uint64_t) * (b->n + 1),
                                   hipMemcpyDeviceToDevice, S(s)));
}

int gga_batch_last_error(gga_batch* b, gga_stream s) {
  if (!b) return GGA_EINVAL;
  if (hipMemcpyAsync(b->h_pin, b->d_err, 4, hipMemcpyDeviceToHost, S(s)) != hipSuccess ||
      hipStreamSynchronize(S(s)) != hipSuccess)
    return GGA_EHIP;
  return map_device_error((uint32_t)b->h_pin[0]);
}

// -------------------------------------------------------------- static array --
static int static_init(gga_static* st, void* buf, uint64_t cap, uint32_t elem_bytes, hipStream_t s) {
  st->data = buf;
  st->cap = cap;
  st->elem_bytes = elem_bytes;
  if (hipMalloc(&st->meta, 256) != hipSuccess) return GGA_EHIP;
  if (hipMemsetAsync(st->meta, 0, 256, s) != hipSuccess) {
    (void)hipFree(st->meta);
    return GGA_EHIP;
  }
  uint8_t* m = static_cast<uint8_t*>(st->meta);
  st->d_size = reinterpret_cast<uint64_t*>(m);
  st->d_err = reinterpret_cast<uint32_t*>(m + 16);
  st->d_done = reinterpret_cast<uint32_t*>(m + 128);  // its own cache line: the size's is read by every wave
  st->rw_last = false;
  st->size_ub = 0;
  return GGA_OK;
}

static int static_read(gga_static* st, uint64_t* size_out, hipStream_t s) {
  uint64_t h[2] = {0, 0};
  if (hipMemcpyAsync(&h[0], st->d_size, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&h[1], st->d_err, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GGA_EHIP;
  if (size_out) {
    *size_out = h[0] < st->cap ? h[0] : st->cap;
    st->size_ub = *size_out;
  }
  return map_device_error((uint32_t)h[1]);
}

int gga_static_create(gga_static** out, void* dev_buf, uint64_t cap_elems, uint32_t elem_bytes,
                      gga_stream s) {
  if (!out) return GGA_EINVAL;
  *out = nullptr;
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) & 15u) || (elem_bytes != 4 && elem_bytes != 8))
    return GGA_EINVAL;
  gga_static* st = new (std::nothrow) gga_static();
  if (!st) return GGA_EHIP;
  const int rc = static_init(st, dev_buf, cap_elems, elem_bytes, S(s));
  if (rc) {
    delete st;
    return rc;
  }
  *out = st;
  return GGA_OK;
}

int gga_static_destroy(gga_static* st, gga_stream s) {
  if (!st) return GGA_EINVAL;
  int rc = hip_status(hipStreamSynchronize(S(s)));
  if (hipFree(st->meta) != hipSuccess) rc = GGA_EHIP;
  delete st;
  return rc;
}

int gga_static_insert(gga_static* st, const void* values, const uint8_t* flags, uint64_t n_threads,
                      gga_stream s) {
  if (!st || (n_threads && !values)) return GGA_EINVAL;
  InsertDesc d{};
  d.mode = kModeBuffer;
  d.values = values;
  d.flags = flags;
  d.max_count = 1;
  d.n_threads = n_threads;
  return launch_static_insert(st, d, S(s));
}

int gga_static_insert_gen(gga_static* st, const gga_gen* g, uint64_t n_threads, gga_stream s) {
  uint32_t mode = 0, maxc = 0;
  if (!st) return GGA_EINVAL;
  const int rc = check_gen(g, n_threads, &mode, &maxc);
  if (rc) return rc;
  return launch_static_insert(st, gen_desc(g, mode, n_threads), S(s));
}

int gga_static_insert_gen_atomic(gga_static* st, const gga_gen* g, uint64_t n_threads, gga_stream s) {
  uint32_t mode = 0, maxc = 0;
  if (!st) return GGA_EINVAL;
  const int rc = check_gen(g, n_threads, &mode, &maxc);
  if (rc) return rc;
  if (maxc != 1) return GGA_EINVAL;  // 0/1 producers only
  return launch_static_insert_atomic(st, gen_desc(g, mode, n_threads), S(s));
}

int gga_static_rw(gga_static* st, uint32_t op, gga_stream s) {
  if (!st || op > GGA_ADD1_X30) return GGA_EINVAL;
  return launch_static_rw(st, op, S(s));
}

int gga_static_size(gga_static* st, uint64_t* out_host, gga_stream s) {
  if (!st || !out_host) return GGA_EINVAL;
  return static_read(st, out_host, S(s));
}

int gga_static_last_error(gga_static* st, gga_stream s) {
  if (!st) return GGA_EINVAL;
  return static_read(st, nullptr, S(s));
}

int gga_static_clear(gga_static* st, gga_stream s) {
  if (!st) return GGA_EINVAL;
  if (hipMemsetAsync(st->d_size, 0, 8, S(s)) != hipSuccess ||
      hipMemsetAsync(st->d_err, 0, 4, S(s)) != hipSuccess)
    return GGA_EHIP;
  st->rw_last = false;
  st->size_ub = 0;
  return GGA_OK;
}

int gga_static_set_size(gga_static* st, uint64_t n, gga_stream s) {
  if (!st || n > st->cap) return GGA_EINVAL;
  if (hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(st->d_size), (int)(uint32_t)n, 1, S(s)) != hipSuccess ||
      hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(reinterpret_cast<uint32_t*>(st->d_size) + 1),
                        (int)(uint32_t)(n >> 32), 1, S(s)) != hipSuccess)
    return GGA_EHIP;
  st->rw_last = false;
  st->size_ub = n;
  return GGA_OK;
}

// --------------------------------------------------------- semi-static array --
int gga_semi_create(gga_semistatic** out, uint32_t elem_bytes, uint64_t initial_cap, gga_stream s) {
  if (!out) return GGA_EINVAL;
  *out = nullptr;
  if ((elem_bytes != 4 && elem_bytes != 8) || initial_cap == 0) return GGA_EINVAL;
  gga_semistatic* ss = new (std::nothrow) gga_semistatic();
  if (!ss) return GGA_EHIP;
  void* buf = nullptr;
  if (hipMallocAsync(&buf, initial_cap * elem_bytes, S(s)) != hipSuccess) {
    delete ss;
    return GGA_EHIP;
  }
  const int rc = static_init(&ss->st, buf, initial_cap, elem_bytes, S(s));
  if (rc) {
    (void)hipFreeAsync(buf, S(s));
    delete ss;
    return rc;
  }
  *out = ss;
  return GGA_OK;
}

int gga_semi_destroy(gga_semistatic* ss, gga_stream s) {
  if (!ss) return GGA_EINVAL;
  int rc = hip_status(hipFreeAsync(ss->st.data, S(s)));
  if (hipStreamSynchronize(S(s)) != hipSuccess) rc = GGA_EHIP;
  if (hipFree(ss->st.meta) != hipSuccess) rc = GGA_EHIP;
  delete ss;
  return rc;
}

// Host-driven resize (Sec. III-A2): read the size, double until the round's
// worst case fits, reallocate and copy.
static int semi_reserve(gga_semistatic* ss, uint64_t worst, hipStream_t s) {
  uint64_t size = 0;
  int rc = static_read(&ss->st, &size, s);
  if (rc) return rc;
  if (size + worst <= ss->st.cap) return GGA_OK;
  uint64_t cap = ss->st.cap;
  while (cap < size + worst) cap *= 2;
  void* nb = nullptr;
  if (hipMallocAsync(&nb, cap * ss->st.elem_bytes, s) != hipSuccess) return GGA_EHIP;
  if (size && hipMemcpyAsync(nb, ss->st.data, size * ss->st.elem_bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return GGA_EHIP;
  if (hipFreeAsync(ss->st.data, s) != hipSuccess) return GGA_EHIP;
  ss->st.data = nb;
  ss->st.cap = cap;
  ss->resizes += 1;
  return GGA_OK;
}

int gga_semi_insert(gga_semistatic* ss, const void* values, const uint8_t* flags, uint64_t n_threads,
                    gga_stream s) {
  if (!ss || (n_threads && !values)) return GGA_EINVAL;
  int rc = semi_reserve(ss, n_threads, S(s));
  return rc ? rc : gga_static_insert(&ss->st, values, flags, n_threads, s);
}

int gga_semi_insert_gen(gga_semistatic* ss, const gga_gen* g, uint64_t n_threads, gga_stream s) {
  uint32_t mode = 0, maxc = 0;
  if (!ss) return GGA_EINVAL;
  int rc = check_gen(g, n_threads, &mode, &maxc);
  if (rc) return rc;
  rc = semi_reserve(ss, n_threads * maxc, S(s));
  return rc ? rc : launch_static_insert(&ss->st, gen_desc(g, mode, n_threads), S(s));
}

int gga_semi_rw(gga_semistatic* ss, uint32_t op, gga_stream s) {
  if (!ss) return GGA_EINVAL;
  return gga_static_rw(&ss->st, op, s);
}

int gga_semi_size(gga_semistatic* ss, uint64_t* out_host, gga_stream s) {
  if (!ss || !out_host) return GGA_EINVAL;
  return static_read(&ss->st, out_host, S(s));
}

int gga_semi_data(gga_semistatic* ss, void** dev_data, uint64_t* cap_elems) {
  if (!ss || !dev_data || !cap_elems) return GGA_EINVAL;
  *dev_data = ss->st.data;
  *cap_elems = ss->st.cap;
  return GGA_OK;
}

int gga_semi_resizes(gga_semistatic* ss, uint64_t* out_host) {
  if (!ss || !out_host) return GGA_EINVAL;
  *out_host = ss->resizes;
  return GGA_OK;
}

// ----------------------------------------------------- mapped (memMap) array --
static hipMemAllocationProp mapped_prop(int device) {
  hipMemAllocationProp prop{};
  prop.type = hipMemAllocationTypePinned;
  prop.location.type = hipMemLocationTypeDevice;
  prop.location.id = device;
  return prop;
}

static void mapped_release(gga_mapped* m) {
  uint64_t off = 0;
  for (uint64_t k = 0; k < m->n_handles; ++k) {
    (void)hipMemUnmap(static_cast<uint8_t*>(m->st.data) + off, m->handle_bytes[k]);
    (void)hipMemRelease(m->handles[k]);
    off += m->handle_bytes[k];
  }
  if (m->st.data) (void)hipMemAddressFree(m->st.data, m->va_bytes);
  if (m->st.meta) (void)hipFree(m->st.meta);
  delete[] m->handles;
  delete[] m->handle_bytes;
  delete m;
}

int gga_mapped_create(gga_mapped** out, uint32_t elem_bytes, uint64_t max_elems, gga_stream s) {
  if (!out) return GGA_EINVAL;
  *out = nullptr;
  if ((elem_bytes != 4 && elem_bytes != 8) || max_elems == 0 || max_elems > (1ull << 40)) return GGA_EINVAL;
  int dev = 0, vmm = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipDeviceGetAttribute(&vmm, hipDeviceAttributeVirtualMemoryManagementSupported, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  if (!vmm) return hip_fail(hipErrorNotSupported, "virtual memory management");
  gga_mapped* m = new (std::nothrow) gga_mapped();
  if (!m) return GGA_EHIP;
  m->device = dev;
  const hipMemAllocationProp prop = mapped_prop(dev);
  size_t gran = 0;
  e = hipMemGetAllocationGranularity(&gran, &prop, hipMemAllocationGranularityRecommended);
  if (e != hipSuccess || !gran) {
    delete m;
    return hip_fail(e, "hipMemGetAllocationGranularity");
  }
  m->gran = gran;
  m->va_bytes = align_up(max_elems * elem_bytes, gran);
  void* va = nullptr;
  e = hipMemAddressReserve(&va, m->va_bytes, gran, nullptr, 0);
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "hipMemAddressReserve");
  }
  const int rc = static_init(&m->st, va, 0, elem_bytes, S(s));
  if (rc) {
    m->st.meta = nullptr;
    mapped_release(m);
    return rc;
  }
  *out = m;
  return GGA_OK;
}

int gga_mapped_destroy(gga_mapped* m, gga_stream s) {
  if (!m) return GGA_EINVAL;
  const int rc = hip_status(hipStreamSynchronize(S(s)));
  mapped_release(m);
  return rc;
}

// Maps chunks onto the end of the mapped part until `worst` more elements fit.
static int mapped_reserve(gga_mapped* m, uint64_t worst, hipStream_t s) {
  uint64_t size = 0;
  int rc = static_read(&m->st, &size, s);
  if (rc) return rc;
  const uint64_t need = (size + worst) * m->st.elem_bytes;
  if (need <= m->mapped_bytes) return GGA_OK;
  if (need > m->va_bytes) return GGA_ERANGE;
  const uint64_t bytes = align_up(need - m->mapped_bytes, m->gran);
  if (m->n_handles == m->cap_handles) {
    const uint64_t nc = m->cap_handles ? 2 * m->cap_handles : 16;
    auto* nh = new (std::nothrow) hipMemGenericAllocationHandle_t[nc];
    auto* nb = new (std::nothrow) uint64_t[nc];
    if (!nh || !nb) {
      delete[] nh;
      delete[] nb;
      return GGA_EHIP;
    }
    for (uint64_t k = 0; k < m->n_handles; ++k) {
      nh[k] = m->handles[k];
      nb[k] = m->handle_bytes[k];
    }
    delete[] m->handles;
    delete[] m->handle_bytes;
    m->handles = nh;
    m->handle_bytes = nb;
    m->cap_handles = nc;
  }
  const hipMemAllocationProp prop = mapped_prop(m->device);
  hipMemGenericAllocationHandle_t h;
  hipError_t e = hipMemCreate(&h, bytes, &prop, 0);
  if (e != hipSuccess) return hip_fail(e, "hipMemCreate");
  uint8_t* at = static_cast<uint8_t*>(m->st.data) + m->mapped_bytes;
  e = hipMemMap(at, bytes, 0, h, 0);
  if (e != hipSuccess) {
    (void)hipMemRelease(h);
    return hip_fail(e, "hipMemMap");
  }
  hipMemAccessDesc desc{};
  desc.location = prop.location;
  desc.flags = hipMemAccessFlagsProtReadWrite;
  // Access is granted over the whole mapped prefix of the range: on this runtime
  // a multi-granule chunk mapped past the start of a reservation rejects an
  // access call that covers only itself, while one from the start succeeds.
  e = hipMemSetAccess(m->st.data, m->mapped_bytes + bytes, &desc, 1);
  if (e != hipSuccess) {
    (void)hipMemUnmap(at, bytes);
    (void)hipMemRelease(h);
    return hip_fail(e, "hipMemSetAccess");
  }
  m->handles[m->n_handles] = h;
  m->handle_bytes[m->n_handles] = bytes;
  m->n_handles += 1;
  m->mapped_bytes += bytes;
  m->st.cap = m->mapped_bytes / m->st.elem_bytes;
  m->maps += 1;
  return GGA_OK;
}

int gga_mapped_insert(gga_mapped* m, const void* values, const uint8_t* flags, uint64_t n_threads, gga_stream s) {
  if (!m || (n_threads && !values)) return GGA_EINVAL;
  int rc = mapped_reserve(m, n_threads, S(s));
  return rc ? rc : gga_static_insert(&m->st, values, flags, n_threads, s);
}

int gga_mapped_insert_gen(gga_mapped* m, const gga_gen* g, uint64_t n_threads, gga_stream s) {
  uint32_t mode = 0, maxc = 0;
  if (!m) return GGA_EINVAL;
  int rc = check_gen(g, n_threads, &mode, &maxc);
  if (rc) return rc;
  rc = mapped_reserve(m, n_threads * maxc, S(s));
  return rc ? rc : launch_static_insert(&m->st, gen_desc(g, mode, n_threads), S(s));
}

int gga_mapped_rw(gga_mapped* m, uint32_t op, gga_stream s) {
  if (!m) return GGA_EINVAL;
  return gga_static_rw(&m->st, op, s);
}

int gga_mapped_size(gga_mapped* m, uint64_t* out_host, gga_stream s) {
  if (!m || !out_host) return GGA_EINVAL;
  return static_read(&m->st, out_host, S(s));
}

int gga_mapped_data(gga_mapped* m, void** dev_data, uint64_t* mapped_elems) {
  if (!m || !dev_data || !mapped_elems) return GGA_EINVAL;
  *dev_data = m->st.data;
  *mapped_elems = m->st.cap;
  return GGA_OK;
}

int gga_mapped_maps(gga_mapped* m, uint64_t* out_host) {
  if (!m || !out_host) return GGA_EINVAL;
  *out_host = m->maps;
  return GGA_OK;
}

}  // extern "C"
