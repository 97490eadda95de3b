// Test kernels for the device-side API (gga::block_push_back): user kernels that
// grow a GGArray from inside, one call per block and round.  Built next to the
// tests by __graft_entry__.build(); loaded only by tests/test_gpu_device_api.py.
#include <hip/hip_runtime.h>

#include <cstring>

#include "ggarray_device.h"

namespace {

// Block b pushes into LFVector b % V.  In round r thread t keeps
// K(seed, gid, r) (gid = b * blockDim.x + t) iff its top bit is set.
template <typename T>
__global__ void bernoulli_push(gga::ArrRef A, uint64_t seed, uint32_t round0, uint32_t rounds) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t v = blockIdx.x % A.V;
  for (uint32_t r = round0; r < round0 + rounds; ++r) {
    const uint64_t h = gga::K(seed, gid, r);
    gga::block_push_back<T>(A, v, (h >> 63) != 0, (T)h);
  }
}

}  // namespace

extern "C" int ggt_bernoulli_push(const void* ref, uint64_t ref_bytes, uint32_t elem_bytes, uint32_t blocks,
                                  uint32_t threads, uint64_t seed, uint32_t round0, uint32_t rounds,
                                  void* stream) {
  if (!ref || ref_bytes != sizeof(gga::ArrRef) || blocks == 0 || threads == 0 || threads > 1024 ||
      (elem_bytes != 4 && elem_bytes != 8) || seed >= 256 || round0 + rounds > 256)
    return -1;
  gga::ArrRef A;
  std::memcpy(&A, ref, sizeof(A));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (elem_bytes == 4)
    hipLaunchKernelGGL(bernoulli_push<uint32_t>, dim3(blocks), dim3(threads), 0, s, A, seed, round0, rounds);
  else
    hipLaunchKernelGGL(bernoulli_push<uint64_t>, dim3(blocks), dim3(threads), 0, s, A, seed, round0, rounds);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

extern "C" uint64_t ggt_ref_bytes() { return sizeof(gga::ArrRef); }

// ---------------------------------------------------------------- pool stress --
// Thread t owns slots t * k .. t * k + k - 1 of ptr[] / cls[].  Phase 0 allocates
// every slot, phase 1 frees the odd slots, phase 2 allocates them again, phase 3
// checks the signature words of every slot, phase 4 frees every slot.  A block of
// class c (2^c bytes, c >= 8) carries the slot number in its first and its last
// 8 bytes while it is live.  Class and free-list shard of a slot come from
// K(seed, slot, phase); classes span 2^8 .. 2^(8 + nclass - 1) bytes.
namespace {

__global__ void pool_stress(gga::PoolRef P, uint32_t threads, uint32_t k, uint32_t phase, uint64_t seed,
                            uint32_t nclass, uint64_t* ptr, uint32_t* cls, uint32_t* err) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= threads) return;
  for (uint32_t j = 0; j < k; ++j) {
    const uint64_t slot = (uint64_t)t * k + j;
    const bool odd = (j & 1u) != 0;
    if (phase == 0 || (phase == 2 && odd)) {
      const uint64_t h = gga::K(seed, slot, phase);
      const uint32_t c = 8u + (uint32_t)(h % nclass);
      uint8_t* p = gga::pool_alloc(P, c, (uint32_t)(h >> 32) & (uint32_t)(gga::kFreeShards - 1));
      ptr[slot] = (uint64_t)p;
      cls[slot] = c;
      if (!p) {
        atomicAdd(err, 1u);
        continue;
      }
      reinterpret_cast<uint64_t*>(p)[0] = slot;
      reinterpret_cast<uint64_t*>(p + (1ull << c) - 8)[0] = slot;
    } else if ((phase == 1 && odd) || phase == 4) {
      uint8_t* p = reinterpret_cast<uint8_t*>(ptr[slot]);
      if (p) gga::pool_free(P, p, cls[slot], (uint32_t)(gga::K(seed, slot, 99) & (gga::kFreeShards - 1)));
      ptr[slot] = 0;
    } else if (phase == 3) {
      const uint8_t* p = reinterpret_cast<const uint8_t*>(ptr[slot]);
      if (p && (reinterpret_cast<const uint64_t*>(p)[0] != slot ||
                reinterpret_cast<const uint64_t*>(p + (1ull << cls[slot]) - 8)[0] != slot))
        atomicAdd(err, 1u << 16);
    }
  }
}

}  // namespace

extern "C" int ggt_pool_stress(const void* ref, uint64_t ref_bytes, uint32_t threads, uint32_t k, uint32_t phase,
                               uint64_t seed, uint32_t nclass, uint64_t* ptr, uint32_t* cls, uint32_t* err,
                               void* stream) {
  if (!ref || ref_bytes != sizeof(gga::ArrRef) || threads == 0 || k == 0 || phase > 4 || nclass == 0 ||
      nclass > 12 || !ptr || !cls || !err)
    return -1;
  gga::ArrRef A;
  std::memcpy(&A, ref, sizeof(A));
  hipLaunchKernelGGL(pool_stress, dim3((threads + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     A.pool, threads, k, phase, seed, nclass, ptr, cls, err);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
