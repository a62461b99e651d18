// Bandwidth reference of the device: a plain copy that reads and writes the
// same number of bytes, as the step does, one 16-byte vector per thread with a
// non-temporal store, on a flat grid (one thread per vector).  Among the
// variants measured on MI355X (4 GiB each way) this was the fastest:
// 6.30 TB/s, against 6.19 with regular stores, 5.69 with four consecutive
// vectors per thread and 4.4-4.7 on a persistent grid-stride loop with four
// loads in flight (1024-4096 blocks); torch's FP64 negation 6.18.  Its rate is
// the practical ceiling of a kernel whose traffic is half reads and half
// writes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gplbm {

typedef unsigned int StreamVec __attribute__((ext_vector_type(4)));
constexpr int kStreamThreads = 256;

__global__ void __launch_bounds__(kStreamThreads)
    k_stream_copy(const StreamVec* __restrict__ src, StreamVec* __restrict__ dst, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(src[i], &dst[i]);
}

}  // namespace gplbm
