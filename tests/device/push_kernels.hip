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
