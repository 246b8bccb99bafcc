// sweep_impl.h -- checkerboard link-update kernels (Metropolis and
// overrelaxation) for compact U(1) with the Wilson action, Eq. (3).
//
// One launch updates one class (mu, parity): links of one class never share
// a plaquette, so the class is updated in parallel with no ordering
// constraint.  Kernels are specialised per direction mu so that the staple's
// six plaquettes unroll with compile-time directions, and neighbour sites are
// found as n +- stride (32-bit, periodic corrections precomputed per site).
// With frozen slabs (multilevel) threads are mapped onto the free links only.
//
// The arithmetic policy P fixes the number type and elementary functions:
//   Det64  - FP64 angles, deterministic sin/cos/atan2 (translation unit built
//            with -ffp-contract=off): the reproducible update path;
//   Fast32 - FP32 angles, hardware sin/cos/exp and a short atan2 series: the
//            fast update path.
#pragma once

#include "device_common.h"

namespace u1ml {

struct Det64 {
  using real = double;
  static __device__ __forceinline__ void sincos(double x, double& s, double& c) { det_sincos(x, s, c); }
  static __device__ __forceinline__ double atan2(double y, double x) { return det_atan2(y, x); }
  static __device__ __forceinline__ double expo(double x) { return ::exp(x); }
  static __device__ __forceinline__ double wrap(double a) { return wrap_f64(a); }
  // Metropolis uniforms (u1, u2): Philox4x64-10, counter (n, 2<<32 | hit<<8 | mu, pass_id, 0),
  // key (seed, 0); u = (w >> 11) 2^-53 from words 0 and 1
  static __device__ __forceinline__ void metro_uniforms(uint32_t n, int hit, int mu, uint64_t pass_id,
                                                        uint64_t seed, double& u1, double& u2) {
    const U64x4 w = philox4x64_10(n, kPurposeMetro | ((uint64_t)hit << 8) | (uint64_t)mu, pass_id, 0, seed, 0);
    u1 = u01_f64(w.v[0]);
    u2 = u01_f64(w.v[1]);
  }
  static __device__ __forceinline__ double from_f64(double v) { return v; }
};

struct Fast32 {
  using real = float;
  static constexpr float kPiF = 3.14159265358979f;
  static constexpr float kTwoPiF = 6.28318530717959f;
  static __device__ __forceinline__ void sincos(float x, float& s, float& c) { __sincosf(x, &s, &c); }
  // atan2 to ~1e-7 rad: fold to t in [0, 1], t -> (t-1)/(t+1) above tan(pi/8),
  // then the Gregory series through u^17 (|u| <= 0.4143).
  static __device__ __forceinline__ float atan2(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const bool swap = ay > ax;
    const float num = swap ? ax : ay, den = swap ? ay : ax;
    const float t = den > 0.f ? num * __builtin_amdgcn_rcpf(den) : 0.f;
    const bool red = t > 0.41421356f;
    const float u = red ? (t - 1.f) * __builtin_amdgcn_rcpf(t + 1.f) : t;
    const float z = u * u;
    float p = 1.f / 17.f;
    p = p * z - 1.f / 15.f;
    p = p * z + 1.f / 13.f;
    p = p * z - 1.f / 11.f;
    p = p * z + 1.f / 9.f;
    p = p * z - 1.f / 7.f;
    p = p * z + 1.f / 5.f;
    p = p * z - 1.f / 3.f;
    float a = u + (u * z) * p;
    a += red ? 0.78539816f : 0.f;
    a = swap ? 1.57079633f - a : a;
    a = x < 0.f ? 3.14159265f - a : a;
    return y < 0.f ? -a : a;
  }
  static __device__ __forceinline__ float expo(float x) { return __expf(x); }
  // fold into [-pi, pi] by whole periods (branch-free)
  static __device__ __forceinline__ float wrap(float a) { return a - kTwoPiF * rintf(a * (1.f / kTwoPiF)); }
  // Metropolis uniforms (u1, u2): Philox4x32-10, counter
  // (n, 2<<16 | hit<<8 | mu, pass_id low, pass_id high), key (seed low, seed high);
  // u = (w >> 8) 2^-24 from words 0 and 1
  static __device__ __forceinline__ void metro_uniforms(uint32_t n, int hit, int mu, uint64_t pass_id,
                                                        uint64_t seed, float& u1, float& u2) {
    const U32x4 w = philox4x32_10(n, (2u << 16) | ((uint32_t)hit << 8) | (uint32_t)mu, (uint32_t)pass_id,
                                  (uint32_t)(pass_id >> 32), (uint32_t)seed, (uint32_t)(seed >> 32));
    u1 = u01_f32_w32(w.v[0]);
    u2 = u01_f32_w32(w.v[1]);
  }
  static __device__ __forceinline__ float from_f64(double v) { return wrap((float)v); }
};

// Hot start theta = pi (2u - 1), u from counter (n, 1<<32 | mu, 0, 0); cold start 0.
// One thread per link: index i over [0, 4 V) = [0, 8 V/2) in the layout order of one lattice.
template <class P>
__global__ void init_links_kernel(typename P::real* __restrict__ links, const LatDesc* __restrict__ lats,
                                  const int2* __restrict__ blocks, int hot) {
  const int2 bk = blocks[blockIdx.x];
  const LatDesc d = lats[bk.x];
  const uint32_t i = (uint32_t)bk.y + threadIdx.x;
  if (i >= 8u * (uint32_t)d.V2) return;
  const int mu = (int)(i / (2u * (uint32_t)d.V2));
  const uint32_t rem = i - (uint32_t)mu * 2u * (uint32_t)d.V2;
  const int parity = rem >= (uint32_t)d.V2;
  const uint32_t h = rem - (parity ? (uint32_t)d.V2 : 0u);
  double th = 0.0;
  if (hot) {
    const Site s = site_of(d, h, parity);
    const uint32_t n = natural_index(d, s.t, s.x, s.y, s.z);
    const U64x4 w = philox4x64_10(n, kPurposeInit | (uint64_t)mu, 0, 0, d.seed, 0);
    th = kPi * (2.0 * u01_f64(w.v[0]) - 1.0);
  }
  links[d.off + i] = P::from_f64(th);
}

// The per-link update of the link of class (MU, parity) at time slice t and
// offset off = (z L + y) L/2 + x/2 within the slice.  Neighbour half-indices
// are h plus per-direction half-displacements: the strides along t, y, z are
// even, and along x the displacement depends on the parity of x; periodic
// wrap-around is folded into the displacements.
template <class P, int MU, int KIND>
__device__ __forceinline__ void update_link(typename P::real* __restrict__ base, const LatDesc& d, int t,
                                            uint32_t off, int parity, int n_hits, uint64_t pass_id,
                                            uint8_t* __restrict__ log) {
  using R = typename P::real;
  const int L = d.L, Lh = L >> 1;
  const int per_slice = d.L3 >> 1;
  const uint32_t h = (uint32_t)t * (uint32_t)per_slice + off;
  const uint32_t qy = fdiv(off, d.div_Lh);
  const int xh = (int)(off - qy * (uint32_t)Lh);
  const uint32_t qz = fdiv(qy, d.div_L);
  const int y = (int)(qy - qz * (uint32_t)L);
  const int z = (int)qz;
  const int xb = (parity ^ (t + z + y)) & 1;
  const int x = 2 * xh + xb;
  // half-displacements, directions (t, x, y, z)
  int hp[4], hm[4];
  hp[0] = t == d.T - 1 ? -(d.T - 1) * per_slice : per_slice;
  hm[0] = t == 0 ? (d.T - 1) * per_slice : -per_slice;
  hp[1] = x == L - 1 ? 1 - Lh : xb;
  hm[1] = x == 0 ? Lh - 1 : xb - 1;
  hp[2] = y == L - 1 ? -(L - 1) * Lh : Lh;
  hm[2] = y == 0 ? (L - 1) * Lh : -Lh;
  hp[3] = z == L - 1 ? -(L - 1) * Lh * L : Lh * L;
  hm[3] = z == 0 ? (L - 1) * Lh * L : -Lh * L;
  const uint32_t V2 = (uint32_t)d.V2;
  const int q = parity ^ 1;
  const int hh = (int)h;
  // scalar base of each (direction, parity) array + a 32-bit vector byte
  // offset per neighbour half-index (shared by the arrays that use it)
  const char* cbase = (const char*)base;
  auto ld = [&](int dir, int par, int hi) -> R {
    const char* arr = cbase + (size_t)((uint32_t)(2 * dir + par) * V2) * sizeof(R);
    return *(const R*)(arr + (uint32_t)hi * (uint32_t)sizeof(R));
  };
  R sr = (R)0, si = (R)0;
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == MU) continue;
    const int h_xpmu = hh + hp[MU];
    const int h_xpnu = hh + hp[nu];
    const int h_xmnu = hh + hm[nu];
    const int h_xpmu_mnu = h_xpmu + hm[nu];
    const R a_nu_xpmu = ld(nu, q, h_xpmu);
    const R a_mu_xpnu = ld(MU, q, h_xpnu);
    const R a_nu_x = ld(nu, parity, hh);
    const R a_mu_xmnu = ld(MU, q, h_xmnu);
    const R a_nu_xpmumnu = ld(nu, parity, h_xpmu_mnu);
    const R a_nu_xmnu = ld(nu, q, h_xmnu);
    const R ap = (a_nu_xpmu - a_mu_xpnu) - a_nu_x;
    const R am = -((a_mu_xmnu + a_nu_xpmumnu) - a_nu_xmnu);
    R sn, cs;
    P::sincos(ap, sn, cs);
    sr += cs;
    si += sn;
    P::sincos(am, sn, cs);
    sr += cs;
    si += sn;
  }
  R* self = (R*)((char*)base + ((uint32_t)(2 * MU + parity) * V2 + h) * (uint32_t)sizeof(R));
  R th0 = *self;
  if (KIND == 0) {
    const uint32_t n = 2u * h + (uint32_t)xb;  // natural site index
    const R beta = (R)d.beta, eps = (R)d.eps;
    for (int k = 0; k < n_hits; ++k) {
      R u1, u2;
      P::metro_uniforms(n, k, MU, pass_id, d.seed, u1, u2);
      const R thn = P::wrap(th0 + eps * ((R)2 * u1 - (R)1));
      R s0, c0, s1, c1;
      P::sincos(th0, s0, c0);
      P::sincos(thn, s1, c1);
      const R dS = beta * ((c0 * sr - s0 * si) - (c1 * sr - s1 * si));
      const bool acc = (dS <= (R)0) || (u2 < P::expo(-dS));
      if (acc) th0 = thn;
      if (log != nullptr) log[(size_t)h * n_hits + k] = acc ? 1 : 0;
    }
  } else {
    if (sr == (R)0 && si == (R)0) return;
    const R alpha = P::atan2(si, sr);
    th0 = P::wrap(-th0 - (R)2 * alpha);
  }
  *self = th0;
}

// Single lattice: geometry in the kernel arguments; grid (blocks per slice,
// updated slices), walked in XCD-contiguous order (xcd_map != 0) or in the
// hardware's round-robin order.
template <class P, int MU, int KIND>
__global__ void class_pass_kernel(typename P::real* __restrict__ links, LatDesc d, int parity, int th_frozen,
                                  int n_hits, uint64_t* __restrict__ pass_ids, uint8_t* __restrict__ log,
                                  int bump_n, int xcd_map) {
  if (KIND == 1 && bump_n > 0 && blockIdx.x == 0 && blockIdx.y == 0)
    for (int i = threadIdx.x; i < bump_n; i += blockDim.x) pass_ids[i] += 1;
  const uint32_t lin = blockIdx.y * gridDim.x + blockIdx.x;
  const uint32_t lb = xcd_map ? xcd_block(lin, gridDim.x * gridDim.y) : lin;
  const uint32_t by = lb / gridDim.x, bx = lb - by * gridDim.x;
  const uint32_t off = bx * blockDim.x + threadIdx.x;
  if (off >= ((uint32_t)d.L3 >> 1)) return;
  const int t = class_slice((int)by, MU, th_frozen);
  update_link<P, MU, KIND>(links + d.off, d, t, off, parity, n_hits, KIND == 0 ? pass_ids[0] : 0, log);
}

// Batch: blocks[b] = {lattice, time slice, first offset in the slice, 0},
// walked in XCD-contiguous order (xcd_map != 0) or in table order.
template <class P, int MU, int KIND>
__global__ void class_pass_batch_kernel(typename P::real* __restrict__ links, const LatDesc* __restrict__ lats,
                                        const int4* __restrict__ blocks, int parity, int n_hits,
                                        uint64_t* __restrict__ pass_ids, int bump_n, int xcd_map) {
  if (KIND == 1 && bump_n > 0 && blockIdx.x == 0)
    for (int i = threadIdx.x; i < bump_n; i += blockDim.x) pass_ids[i] += 1;
  const int4 bk = blocks[xcd_map ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x];
  const LatDesc d = lats[bk.x];
  const uint32_t off = (uint32_t)bk.z + threadIdx.x;
  if (off >= ((uint32_t)d.L3 >> 1)) return;
  update_link<P, MU, KIND>(links + d.off, d, bk.y, off, parity, n_hits, KIND == 0 ? pass_ids[bk.x] : 0, nullptr);
}

hipError_t launch_bump_pass_ids(uint64_t* pass_ids, int n, hipStream_t st);

// Launch helpers shared by the FP64 and FP32 translation units.
template <class P, int KIND>
hipError_t launch_pass_single(typename P::real* links, const LatDesc& d, int block, int xcd_map, int mu, int parity,
                              int th, int n_hits, uint64_t* pass_ids, uint8_t* log, int bump_n, hipStream_t st) {
  const int slices = class_slices(d.T, mu, th);
  if (slices == 0) return bump_n > 0 ? launch_bump_pass_ids(pass_ids, bump_n, st) : hipSuccess;
  const dim3 grid((d.L3 / 2 + block - 1) / block, slices);
  switch (mu) {
    case 0:
      hipLaunchKernelGGL((class_pass_kernel<P, 0, KIND>), grid, dim3(block), 0, st, links, d, parity, th, n_hits,
                         pass_ids, log, bump_n, xcd_map);
      break;
    case 1:
      hipLaunchKernelGGL((class_pass_kernel<P, 1, KIND>), grid, dim3(block), 0, st, links, d, parity, th, n_hits,
                         pass_ids, log, bump_n, xcd_map);
      break;
    case 2:
      hipLaunchKernelGGL((class_pass_kernel<P, 2, KIND>), grid, dim3(block), 0, st, links, d, parity, th, n_hits,
                         pass_ids, log, bump_n, xcd_map);
      break;
    default:
      hipLaunchKernelGGL((class_pass_kernel<P, 3, KIND>), grid, dim3(block), 0, st, links, d, parity, th, n_hits,
                         pass_ids, log, bump_n, xcd_map);
      break;
  }
  return hipGetLastError();
}

template <class P, int KIND>
hipError_t launch_pass_batch(typename P::real* links, const LatDesc* lats, const int4* blocks, int n_blocks,
                             int block, int xcd_map, int mu, int parity, int n_hits, uint64_t* pass_ids, int bump_n,
                             hipStream_t st) {
  if (n_blocks == 0) return bump_n > 0 ? launch_bump_pass_ids(pass_ids, bump_n, st) : hipSuccess;
  switch (mu) {
    case 0:
      hipLaunchKernelGGL((class_pass_batch_kernel<P, 0, KIND>), dim3(n_blocks), dim3(block), 0, st, links, lats,
                         blocks, parity, n_hits, pass_ids, bump_n, xcd_map);
      break;
    case 1:
      hipLaunchKernelGGL((class_pass_batch_kernel<P, 1, KIND>), dim3(n_blocks), dim3(block), 0, st, links, lats,
                         blocks, parity, n_hits, pass_ids, bump_n, xcd_map);
      break;
    case 2:
      hipLaunchKernelGGL((class_pass_batch_kernel<P, 2, KIND>), dim3(n_blocks), dim3(block), 0, st, links, lats,
                         blocks, parity, n_hits, pass_ids, bump_n, xcd_map);
      break;
    default:
      hipLaunchKernelGGL((class_pass_batch_kernel<P, 3, KIND>), dim3(n_blocks), dim3(block), 0, st, links, lats,
                         blocks, parity, n_hits, pass_ids, bump_n, xcd_map);
      break;
  }
  return hipGetLastError();
}

}  // namespace u1ml
