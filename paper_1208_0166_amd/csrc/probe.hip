// probe.hip -- streaming bandwidth of the device, measured with plain
// grid-stride kernels of 16-byte loads and stores: the achievable rates the
// benchmarks' roofline fractions are read against (a read-only stream of a
// buffer larger or smaller than the Infinity Cache, and a copy).  Not part of
// the method.
#include "engine.h"

namespace {

__global__ __launch_bounds__(256) void stream_read_kernel(const float4* __restrict__ a, size_t n,
                                                          float* __restrict__ sink) {
  float s = 0.f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float4 v = a[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  // the buffer holds zeros: the store never happens, but the loads cannot be dropped
  if (s != 0.f) sink[0] = s;
}

__global__ __launch_bounds__(256) void stream_copy_kernel(const float4* __restrict__ a, float4* __restrict__ b,
                                                          size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void zero_f4_kernel(float4* __restrict__ a, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    a[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace

namespace u1ml {

hipError_t launch_stream_probe(int kind, const void* a, void* b, size_t n_bytes, float* sink, int blocks,
                               hipStream_t st) {
  const size_t n = n_bytes / 16;
  if (kind == 0)
    hipLaunchKernelGGL(stream_read_kernel, dim3(blocks), dim3(256), 0, st, (const float4*)a, n, sink);
  else if (kind == 1)
    hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks), dim3(256), 0, st, (const float4*)a, (float4*)b, n);
  else
    hipLaunchKernelGGL(zero_f4_kernel, dim3(blocks), dim3(256), 0, st, (float4*)b, n);
  return hipGetLastError();
}

}  // namespace u1ml
