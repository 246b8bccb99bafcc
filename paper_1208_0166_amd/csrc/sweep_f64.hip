// sweep_f64.hip -- FP64 link updates with deterministic elementary functions.
// Built with -ffp-contract=off: every floating-point step is one IEEE-754
// operation in source order, so the update sequence is reproducible.
#include "engine.h"
#include "sweep_impl.h"

namespace u1ml {

hipError_t launch_init_f64(double* links, const LatDesc* lats, BlockTable bt, int hot, hipStream_t st) {
  if (bt.n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(init_links_kernel<Det64>, dim3(bt.n_blocks), dim3(bt.block), 0, st, links, lats, bt.dev, hot);
  return hipGetLastError();
}

hipError_t launch_class_pass_f64(int kind, double* links, const LatDesc& d, int block, int xcd_map, int mu, int parity,
                                 int th_frozen, int n_hits, uint64_t* pass_ids, uint8_t* log, int bump_n,
                                 hipStream_t st) {
  if (kind == kMetropolis)
    return launch_pass_single<Det64, 0>(links, d, block, xcd_map, mu, parity, th_frozen, n_hits, pass_ids, log, 0, st);
  return launch_pass_single<Det64, 1>(links, d, block, xcd_map, mu, parity, th_frozen, n_hits, pass_ids, log, bump_n, st);
}

hipError_t launch_class_pass_batch_f64(int kind, double* links, const LatDesc* lats, const int4* blocks,
                                       int n_blocks, int block, int xcd_map, int mu, int parity, int n_hits,
                                       uint64_t* pass_ids, int bump_n, hipStream_t st) {
  if (kind == kMetropolis)
    return launch_pass_batch<Det64, 0>(links, lats, blocks, n_blocks, block, xcd_map, mu, parity, n_hits, pass_ids, 0, st);
  return launch_pass_batch<Det64, 1>(links, lats, blocks, n_blocks, block, xcd_map, mu, parity, n_hits, pass_ids, bump_n,
                                     st);
}

__global__ void bump_pass_ids_kernel(uint64_t* pass_ids, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pass_ids[i] += 1;
}

__global__ void fill_u8_kernel(uint8_t* p, size_t n, uint8_t v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_bump_pass_ids(uint64_t* pass_ids, int n, hipStream_t st) {
  hipLaunchKernelGGL(bump_pass_ids_kernel, dim3((n + 63) / 64), dim3(64), 0, st, pass_ids, n);
  return hipGetLastError();
}

}  // namespace u1ml
