// measure_common.h -- device helpers shared by the measurement and field
// contraction translation units (internal linkage in each).
#pragma once

#include "engine.h"

namespace u1ml {
namespace {

constexpr int kRedBlock = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum v over the block (blockDim.x a multiple of 64, at most 1024); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) r += sh[w];
  }
  __syncthreads();
  return r;
}

template <typename R>
__device__ __forceinline__ double ld(const R* links, uint64_t i) {
  return (double)links[i];
}

struct Coords {
  int t, x, y, z;
};

__device__ __forceinline__ Coords coords_natural(const LatDesc& d, uint32_t n) {
  Coords c;
  const uint32_t q = fdiv(n, d.div_L);
  c.x = (int)(n - q * (uint32_t)d.L);
  const uint32_t q2 = fdiv(q, d.div_L);
  c.y = (int)(q - q2 * (uint32_t)d.L);
  const uint32_t q3 = fdiv(q2, d.div_L);
  c.z = (int)(q2 - q3 * (uint32_t)d.L);
  c.t = (int)q3;
  return c;
}

__device__ __forceinline__ Site as_site(Coords c) {
  Site s;
  s.t = c.t; s.x = c.x; s.y = c.y; s.z = c.z;
  return s;
}

// plaquette angle theta_mu(x) + theta_nu(x+mu) - theta_mu(x+nu) - theta_nu(x)
template <typename R>
__device__ __forceinline__ double plaq_angle(const R* links, const LatDesc& d, Site s, int mu, int nu) {
  const double a = ld(links, link_at(d, mu, s));
  const double b = ld(links, link_at(d, nu, shift2(d, s, mu, 1, nu, 0)));
  const double c = ld(links, link_at(d, mu, shift2(d, s, nu, 1, mu, 0)));
  const double e = ld(links, link_at(d, nu, s));
  return ((a + b) - c) - e;
}

// Insertion operator of one plaquette angle: sqrt(beta) Im P (Eq. (5)), or
// with SQ the squared component beta (1 - Re P) = 2 beta sin^2(theta / 2)
// (Eq. (6)); the prefactor is applied by the caller.  FP32 links (the fast
// path) in FP32 arithmetic with the hardware sine, returned as FP64 for the
// FP64 sums.
template <bool SQ>
__device__ __forceinline__ double plaq_op(const double* links, const LatDesc& d, Site s, int mu, int nu) {
  const double a = plaq_angle(links, d, s, mu, nu);
  if (SQ) {
    const double h = sin(0.5 * a);
    return 2.0 * (h * h);
  }
  return sin(a);
}
template <bool SQ>
__device__ __forceinline__ double plaq_op(const float* links, const LatDesc& d, Site s, int mu, int nu) {
  const float a = links[link_at(d, mu, s)];
  const float b = links[link_at(d, nu, shift2(d, s, mu, 1, nu, 0))];
  const float c = links[link_at(d, mu, shift2(d, s, nu, 1, mu, 0))];
  const float e = links[link_at(d, nu, s)];
  const float th = ((a + b) - c) - e;
  if (SQ) {
    const float h = __sinf(0.5f * th);
    return (double)(2.0f * (h * h));
  }
  return (double)__sinf(th);
}

// o[c] += the six insertion operators at site st, before the prefactor:
// E_x, E_y, E_z, B_x, B_y, B_z from P_01, P_02, P_03, P_23, P_31 = conj(P_13),
// P_12 (the squared components do not depend on the orientation)
template <bool SQ, typename R>
__device__ __forceinline__ void add_field_ops(const R* links, const LatDesc& d, Site st, double o[6]) {
  o[0] += plaq_op<SQ>(links, d, st, 0, 1);
  o[1] += plaq_op<SQ>(links, d, st, 0, 2);
  o[2] += plaq_op<SQ>(links, d, st, 0, 3);
  o[3] += plaq_op<SQ>(links, d, st, 2, 3);
  if (SQ)
    o[4] += plaq_op<SQ>(links, d, st, 1, 3);
  else
    o[4] -= plaq_op<SQ>(links, d, st, 1, 3);
  o[5] += plaq_op<SQ>(links, d, st, 1, 2);
}

// The links the six plaquettes at one site read, each loaded once: the four
// links theta_mu(s) of the site and the twelve links theta_a(s + b) (a != b)
// of its four forward neighbours.  Site indices come from one natural index
// and the periodic forward displacements (not recomputed per plaquette).
template <typename R>
struct SiteLinks {
  R at[4];      // at[mu] = theta_mu(s)
  R fwd[4][4];  // fwd[b][a] = theta_a(s + b), a != b
};

template <typename R>
__device__ __forceinline__ void load_site_links(const R* links, const LatDesc& d, int t, int x, int y, int z,
                                                SiteLinks<R>& sl) {
  const uint32_t L = (uint32_t)d.L, L2 = L * L, L3 = (uint32_t)d.L3;
  const uint32_t n = (((uint32_t)t * L + (uint32_t)z) * L + (uint32_t)y) * L + (uint32_t)x;
  const int p = (t + x + y + z) & 1;
  const uint64_t V2 = (uint64_t)d.V2;
  const R* base = links + d.off;
  // natural index of the forward neighbour along b (t, x, y, z), periodic
  const uint32_t nb[4] = {t == d.T - 1 ? n - (uint32_t)(d.T - 1) * L3 : n + L3,
                          x == d.L - 1 ? n - (L - 1) : n + 1,
                          y == d.L - 1 ? n - (L - 1) * L : n + L,
                          z == d.L - 1 ? n - (L - 1) * L2 : n + L2};
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) sl.at[mu] = base[(uint64_t)(2 * mu + p) * V2 + (n >> 1)];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (a != b) sl.fwd[b][a] = base[(uint64_t)(2 * a + (p ^ 1)) * V2 + (nb[b] >> 1)];
  }
}

// insertion operator of the plaquette (mu, nu) from the loaded links, in the
// arithmetic of plaq_op (FP64 with the library sine; FP32 with the hardware
// sine, returned as FP64), before the prefactor
template <bool SQ>
__device__ __forceinline__ double plaq_op_loaded(const SiteLinks<double>& sl, int mu, int nu) {
  const double a = ((sl.at[mu] + sl.fwd[mu][nu]) - sl.fwd[nu][mu]) - sl.at[nu];
  if (SQ) {
    const double h = sin(0.5 * a);
    return 2.0 * (h * h);
  }
  return sin(a);
}
template <bool SQ>
__device__ __forceinline__ double plaq_op_loaded(const SiteLinks<float>& sl, int mu, int nu) {
  const float th = ((sl.at[mu] + sl.fwd[mu][nu]) - sl.fwd[nu][mu]) - sl.at[nu];
  if (SQ) {
    const float h = __sinf(0.5f * th);
    return (double)(2.0f * (h * h));
  }
  return (double)__sinf(th);
}

// add_field_ops from the loaded links (same components, order and signs)
template <bool SQ, typename R>
__device__ __forceinline__ void add_field_ops_loaded(const SiteLinks<R>& sl, double o[6]) {
  o[0] += plaq_op_loaded<SQ>(sl, 0, 1);
  o[1] += plaq_op_loaded<SQ>(sl, 0, 2);
  o[2] += plaq_op_loaded<SQ>(sl, 0, 3);
  o[3] += plaq_op_loaded<SQ>(sl, 2, 3);
  if (SQ)
    o[4] += plaq_op_loaded<SQ>(sl, 1, 3);
  else
    o[4] -= plaq_op_loaded<SQ>(sl, 1, 3);
  o[5] += plaq_op_loaded<SQ>(sl, 1, 2);
}

// sum_t theta_0 over [t0, t0 + nt) at spatial site x3
template <typename R>
__device__ __forceinline__ double time_line(const R* links, const LatDesc& d, int x3, int t0, int nt) {
  Site s;
  s.x = x3 % d.L;
  s.y = (x3 / d.L) % d.L;
  s.z = x3 / (d.L * d.L);
  double a = 0.0;
  for (int t = t0; t < t0 + nt; ++t) {
    s.t = t;
    a += ld(links, link_at(d, 0, s));
  }
  return a;
}

__device__ __forceinline__ int shift_x(const LatDesc& d, int x3, int r) {
  const int x = x3 % d.L;
  int xr = x + r;
  xr -= (xr >= d.L) ? d.L : 0;
  return x3 - x + xr;
}

// x3 + r e_axis (periodic) for an encoded separation v = r | axis << 16,
// axis 0, 1, 2 = x, y, z; x3 = (z L + y) L + x
__device__ __forceinline__ int shift_axis(const LatDesc& d, int x3, int v) {
  const int r = v & 0xffff, axis = v >> 16;
  const int stride = axis == 0 ? 1 : (axis == 1 ? d.L : d.L * d.L);
  const int c = (x3 / stride) % d.L;
  int cr = c + r;
  cr -= (cr >= d.L) ? d.L : 0;
  return x3 + (cr - c) * stride;
}

// Stores of per-sample data that is read back only at the end of an outer
// iteration or of the run: marked non-temporal so that they do not displace
// the lattices from the caches.
__device__ __forceinline__ void store_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(float* p, double v) { __builtin_nontemporal_store((float)v, p); }
__device__ __forceinline__ void store_stream(double2* p, double2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

// Complex arithmetic of the level averages and their products, written as
// explicit fused multiply-adds with contraction off around them: every
// kernel that forms the same average, product or sum (the row-staged and the
// per-site fold, the field weights) rounds it the same way, whatever the
// code around it.
// a b
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
#pragma clang fp contract(off)
  return make_double2(__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x));
}
// acc + conj(a) b
__device__ __forceinline__ double2 cmac_conj(double2 acc, double2 a, double2 b) {
#pragma clang fp contract(off)
  return make_double2(__builtin_fma(a.x, b.x, __builtin_fma(a.y, b.y, acc.x)),
                      __builtin_fma(a.x, b.y, __builtin_fma(-a.y, b.x, acc.y)));
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
#pragma clang fp contract(off)
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) {
#pragma clang fp contract(off)
  return make_double2(a.x * s, a.y * s);
}

__device__ __forceinline__ double2 cexpi(double phi) {
  double s, c;
  sincos(phi, &s, &c);
  return make_double2(c, s);
}

// average over the stored samples of T(x0, r) = conj(e(x0)) e(x0 + r) of inner slab cs
__device__ __forceinline__ double2 inner_avg(const double2* ell, int n_samples, int ns, int L3, int cs, int x0,
                                             int x0r) {
  double2 a = make_double2(0.0, 0.0);
  for (int i = 0; i < n_samples; ++i) {
    const double2* e = ell + ((size_t)i * ns + cs) * L3;
    a = cmac_conj(a, e[x0], e[x0r]);
  }
  return cscale(a, 1.0 / (double)n_samples);
}

__global__ void zero_kernel(double2* __restrict__ p, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(0.0, 0.0);
}

inline int blocks_for(uint64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace
}  // namespace u1ml
