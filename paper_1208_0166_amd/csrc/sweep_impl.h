// sweep_impl.h -- checkerboard link-update kernels (Metropolis and
// overrelaxation) for compact U(1) with the Wilson action, Eq. (3).
//
// One launch updates one class (mu, parity) on every lattice of a batch.
// Links of one class never share a plaquette, so the class is updated in
// parallel with no ordering constraint.  The arithmetic policy P fixes the
// number type and the elementary functions:
//   Det64  - FP64 angles, deterministic sin/cos/atan2 (translation unit built
//            with -ffp-contract=off): the reproducible update path;
//   Fast32 - FP32 angles, hardware transcendentals: the fast update path.
#pragma once

#include "device_common.h"

namespace u1ml {

struct Det64 {
  using real = double;
  static __device__ __forceinline__ void sincos(double x, double& s, double& c) { det_sincos(x, s, c); }
  static __device__ __forceinline__ double atan2(double y, double x) { return det_atan2(y, x); }
  static __device__ __forceinline__ double expo(double x) { return ::exp(x); }
  static __device__ __forceinline__ double wrap(double a) { return wrap_f64(a); }
  static __device__ __forceinline__ double uni(uint64_t w) { return u01_f64(w); }
  static __device__ __forceinline__ double from_f64(double v) { return v; }
};

struct Fast32 {
  using real = float;
  static constexpr float kPiF = 3.14159265358979f;
  static constexpr float kTwoPiF = 6.28318530717959f;
  static __device__ __forceinline__ void sincos(float x, float& s, float& c) { __sincosf(x, &s, &c); }
  static __device__ __forceinline__ float atan2(float y, float x) { return ::atan2f(y, x); }
  static __device__ __forceinline__ float expo(float x) { return __expf(x); }
  static __device__ __forceinline__ float wrap(float a) {
    while (a >= kPiF) a -= kTwoPiF;
    while (a < -kPiF) a += kTwoPiF;
    return a;
  }
  static __device__ __forceinline__ float uni(uint64_t w) { return u01_f32(w); }
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

// Staple sum S of link (s, mu) so that the six plaquettes containing it add up
// to Re(exp(i theta) S): for each nu != mu (ascending) the forward plaquette
// phase  th_nu(x+mu) - th_mu(x+nu) - th_nu(x)  then the backward one
// -(th_mu(x-nu) + th_nu(x+mu-nu) - th_nu(x-nu)).
template <class P>
__device__ __forceinline__ void staple(const typename P::real* __restrict__ links, const LatDesc& d, Site s,
                                       int mu, typename P::real& sr, typename P::real& si) {
  using R = typename P::real;
  R accr = (R)0, acci = (R)0;
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    const Site xpmu = shift2(d, s, mu, 1, nu, 0);
    const Site xpnu = shift2(d, s, nu, 1, mu, 0);
    const Site xmnu = shift2(d, s, nu, -1, mu, 0);
    const Site xpmu_mnu = shift2(d, s, mu, 1, nu, -1);
    const R a_nu_xpmu = links[link_at(d, nu, xpmu)];
    const R a_mu_xpnu = links[link_at(d, mu, xpnu)];
    const R a_nu_x = links[link_at(d, nu, s)];
    const R a_mu_xmnu = links[link_at(d, mu, xmnu)];
    const R a_nu_xpmumnu = links[link_at(d, nu, xpmu_mnu)];
    const R a_nu_xmnu = links[link_at(d, nu, xmnu)];
    const R ap = (a_nu_xpmu - a_mu_xpnu) - a_nu_x;
    const R am = -((a_mu_xmnu + a_nu_xpmumnu) - a_nu_xmnu);
    R sn, cs;
    P::sincos(ap, sn, cs);
    accr += cs;
    acci += sn;
    P::sincos(am, sn, cs);
    accr += cs;
    acci += sn;
  }
  sr = accr;
  si = acci;
}

// Re(exp(i phi) S)
template <class P>
__device__ __forceinline__ typename P::real re_phase(typename P::real phi, typename P::real sr,
                                                     typename P::real si) {
  typename P::real sn, cs;
  P::sincos(phi, sn, cs);
  return cs * sr - sn * si;
}

// kind 0: Metropolis with n_hits hits per link, proposal theta + eps (2u1 - 1),
//         accepted iff u2 < exp(-dS), u1/u2 from counter
//         (n, 2<<32 | hit<<8 | mu, pass_id, 0) under key (seed, 0);
// kind 1: overrelaxation theta -> -theta - 2 arg S (identity when S = 0).
// Frozen links (spatial links on time slices t = 0 mod th_frozen) are skipped.
// log (optional, single lattice): one byte per (half-site, hit): 1 accepted,
// 0 rejected, 2 frozen.
template <class P, int kKind>
__global__ void class_pass_kernel(typename P::real* __restrict__ links, const LatDesc* __restrict__ lats,
                                  const int2* __restrict__ blocks, int mu, int parity, int th_frozen,
                                  int n_hits, const uint64_t* __restrict__ pass_ids,
                                  uint8_t* __restrict__ log) {
  using R = typename P::real;
  const int2 bk = blocks[blockIdx.x];
  const LatDesc d = lats[bk.x];
  const uint32_t h = (uint32_t)bk.y + threadIdx.x;
  if (h >= (uint32_t)d.V2) return;
  const Site s = site_of(d, h, parity);
  if (th_frozen > 0 && mu > 0 && (s.t % th_frozen) == 0) {
    if (kKind == 0 && log != nullptr)
      for (int k = 0; k < n_hits; ++k) log[(size_t)h * n_hits + k] = 2;
    return;
  }
  const uint64_t self = link_slot(d, mu, parity, h);
  R sr, si;
  staple<P>(links, d, s, mu, sr, si);
  R th = links[self];
  if (kKind == 0) {
    const uint32_t n = natural_index(d, s.t, s.x, s.y, s.z);
    const uint64_t pid = pass_ids[bk.x];
    const R beta = (R)d.beta, eps = (R)d.eps;
    for (int k = 0; k < n_hits; ++k) {
      const U64x4 w = philox4x64_10(n, kPurposeMetro | ((uint64_t)k << 8) | (uint64_t)mu, pid, 0, d.seed, 0);
      const R u1 = P::uni(w.v[0]), u2 = P::uni(w.v[1]);
      const R thn = P::wrap(th + eps * ((R)2 * u1 - (R)1));
      const R dS = beta * (re_phase<P>(th, sr, si) - re_phase<P>(thn, sr, si));
      const bool acc = (dS <= (R)0) || (u2 < P::expo(-dS));
      if (acc) th = thn;
      if (log != nullptr) log[(size_t)h * n_hits + k] = acc ? 1 : 0;
    }
  } else {
    if (sr == (R)0 && si == (R)0) return;
    const R alpha = P::atan2(si, sr);
    th = P::wrap(-th - (R)2 * alpha);
  }
  links[self] = th;
}

}  // namespace u1ml
