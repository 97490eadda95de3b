// Host-side objects and the launch functions shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>

#include "ggarray.h"
#include "gga_device.h"

struct gga_pool {
  gga::PoolRef ref;
  void* dev_base;
  uint64_t bytes;
  int n_arrays;
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
  uint64_t epoch;         // look-back epoch of the last insertion launch
  bool prefix_valid;      // prefix / tprefix match the current sizes
};

struct gga_static {
  void* data;
  uint64_t cap;
  uint32_t elem_bytes;
  void* meta;          // device block: size counter, sticky error
  uint64_t* d_size;
  uint32_t* d_err;
};

struct gga_semistatic {
  gga_static st;      // current buffer, resized by the host
  uint64_t resizes;
};

namespace gga {

// How an insertion round produces its candidates.
enum InsertMode : uint32_t {
  kModeBuffer = 0,   // values[gid], flags[gid]
  kModeCounts = 1,   // values[gid * max + j], j < counts[gid]
  kModeBernoulli = 2,
  kModeRoundTag = 3,
  kModePoisson = 4,
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
};

// Tile geometry of the element-streaming kernels (rw, flatten): 16 KiB per tile.
constexpr uint32_t kRwThreads = 256;
__host__ __device__ constexpr uint32_t rw_tile_elems(uint32_t elem_log2) {
  return 16384u >> elem_log2;
}

int launch_insert(ggarray* a, const InsertDesc& d, hipStream_t s);
int launch_static_insert(gga_static* st, const InsertDesc& d, hipStream_t s);
int launch_scan(ggarray* a, hipStream_t s);
int launch_shrink(ggarray* a, uint32_t num, uint32_t den, hipStream_t s);
int launch_rw(ggarray* a, uint32_t op, hipStream_t s);
int launch_flatten(ggarray* a, void* out, uint64_t cap, hipStream_t s);
int launch_capacity(ggarray* a, uint64_t* d_out, hipStream_t s);
int launch_free_all(ggarray* a, hipStream_t s);
int launch_static_rw(gga_static* st, uint32_t op, hipStream_t s);

inline int hip_status(hipError_t e) { return e == hipSuccess ? GGA_OK : GGA_EHIP; }

}  // namespace gga
