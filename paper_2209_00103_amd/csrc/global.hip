// Access by global index (the rw_g variant of Sec. VI-B).  Global element i is
// element i - P[v] of LFVector v, where P is the exclusive prefix of the
// LFVector sizes (Sec. IV) and v the last LFVector with P[v] <= i; an empty
// LFVector shares its offset with the next one, so this choice skips it.  Inside
// the LFVector the closed form gives bucket and offset.  One thread per element:
// a binary search over P, a bucket-pointer load, then the element itself.
#include "gga_internal.h"

namespace gga {
namespace {

constexpr uint32_t kGlobalThreads = 256;
constexpr uint32_t kGlobalBlocks = 8192;  // 32 workgroups per CU, grid-stride

// Largest v < V with prefix[v] <= i, given i < prefix[V].
__device__ __forceinline__ uint32_t vector_of(const uint64_t* prefix, uint32_t V, uint64_t i) {
  uint32_t lo = 0, hi = V;  // prefix[lo] <= i < prefix[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (prefix[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ gptr<T> element_at(const ArrRef& A, uint64_t i) {
  const uint32_t v = vector_of(A.prefix, A.V, i);
  const uint64_t j = i - A.prefix[v];
  const uint32_t b = bucket_of(A.log2F, j);
  return gmem(reinterpret_cast<T*>(A.bptr[(uint64_t)v * kMaxBuckets + b])) + offset_in(A.log2F, j, b);
}

template <typename T>
__global__ __launch_bounds__(kGlobalThreads) void rw_global_kernel(ArrRef A, uint32_t op) {
  const uint64_t n = A.prefix[A.V];
  const uint64_t stride = (uint64_t)gridDim.x * kGlobalThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kGlobalThreads + threadIdx.x; i < n; i += stride) {
    const gptr<T> p = element_at<T>(A, i);
    *p = apply_op<T>(op, *p);
  }
}

template <typename T>
__global__ __launch_bounds__(kGlobalThreads) void gather_kernel(ArrRef A, const uint64_t* idx, uint64_t n,
                                                               T* out) {
  const uint64_t size = A.prefix[A.V];
  const uint64_t stride = (uint64_t)gridDim.x * kGlobalThreads;
  bool bad = false;
  for (uint64_t k = (uint64_t)blockIdx.x * kGlobalThreads + threadIdx.x; k < n; k += stride) {
    const uint64_t i = idx[k];
    if (i < size) out[k] = *element_at<T>(A, i);
    else bad = true;
  }
  if (bad) set_error(A.err, kErrRange);
}

}  // namespace

int launch_rw_global(ggarray* a, uint32_t op, hipStream_t s) {
  if (a->elem_bytes == 4)
    hipLaunchKernelGGL(rw_global_kernel<uint32_t>, dim3(kGlobalBlocks), dim3(kGlobalThreads), 0, s, a->ref, op);
  else
    hipLaunchKernelGGL(rw_global_kernel<uint64_t>, dim3(kGlobalBlocks), dim3(kGlobalThreads), 0, s, a->ref, op);
  return hip_status(hipGetLastError());
}

int launch_gather(ggarray* a, const uint64_t* idx, uint64_t n, void* out, hipStream_t s) {
  if (n == 0) return GGA_OK;
  uint64_t blocks = (n + kGlobalThreads - 1) / kGlobalThreads;
  if (blocks > kGlobalBlocks) blocks = kGlobalBlocks;
  if (a->elem_bytes == 4)
    hipLaunchKernelGGL(gather_kernel<uint32_t>, dim3((uint32_t)blocks), dim3(kGlobalThreads), 0, s, a->ref, idx, n,
                       static_cast<uint32_t*>(out));
  else
    hipLaunchKernelGGL(gather_kernel<uint64_t>, dim3((uint32_t)blocks), dim3(kGlobalThreads), 0, s, a->ref, idx, n,
                       static_cast<uint64_t*>(out));
  return hip_status(hipGetLastError());
}

}  // namespace gga
