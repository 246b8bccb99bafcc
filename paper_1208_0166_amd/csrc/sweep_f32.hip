// sweep_f32.hip -- FP32 link updates with hardware transcendentals.
#include "engine.h"
#include "sweep_impl.h"

namespace u1ml {

hipError_t launch_init_f32(float* links, const LatDesc* lats, BlockTable bt, int hot, hipStream_t st) {
  if (bt.n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(init_links_kernel<Fast32>, dim3(bt.n_blocks), dim3(bt.block), 0, st, links, lats, bt.dev,
                     hot);
  return hipGetLastError();
}

hipError_t launch_class_pass_f32(int kind, float* links, const LatDesc& d, int block, int xcd_map, int mu, int parity,
                                 int th_frozen, int n_hits, uint64_t* pass_ids, uint8_t* log, int bump_n,
                                 hipStream_t st) {
  if (kind == kMetropolis)
    return launch_pass_single<Fast32, 0>(links, d, block, xcd_map, mu, parity, th_frozen, n_hits, pass_ids, log, 0, st);
  return launch_pass_single<Fast32, 1>(links, d, block, xcd_map, mu, parity, th_frozen, n_hits, pass_ids, log, bump_n, st);
}

hipError_t launch_class_pass_batch_f32(int kind, float* links, const LatDesc* lats, const int4* blocks,
                                       int n_blocks, int block, int xcd_map, int mu, int parity, int n_hits,
                                       uint64_t* pass_ids, int bump_n, hipStream_t st) {
  if (kind == kMetropolis)
    return launch_pass_batch<Fast32, 0>(links, lats, blocks, n_blocks, block, xcd_map, mu, parity, n_hits, pass_ids, 0, st);
  return launch_pass_batch<Fast32, 1>(links, lats, blocks, n_blocks, block, xcd_map, mu, parity, n_hits, pass_ids, bump_n,
                                     st);
}

}  // namespace u1ml
