// device_common.h -- device-side building blocks of the u1ml kernels (gfx950).
//
//  * Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11),
//    with the multipliers and Weyl increments published there.
//  * Deterministic FP64 sin/cos/atan2 for the FP64 update path.  They use only
//    IEEE-754 +,-,*,/ in a fixed order (the translation units that include
//    them for FP64 updates are compiled with -ffp-contract=off), so a link
//    update is a fixed function of its inputs: Cody & Waite reduction by pi/2
//    with a three-part pi/2, Taylor series of sin (to r^19) and cos (to r^18)
//    in Horner form; atan via t -> (t-1)/(t+1) above tan(pi/8) and the
//    Gregory series to u^39.
//  * Parity-split link layout: links[mu][parity][h], h = n >> 1 where
//    n = ((t*L + z)*L + y)*L + x is the natural site index (mu = 0 is time).
//    Time is the slowest coordinate, so a time slab is a contiguous range of h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace u1ml {

// ---------------------------------------------------------------------------
// Philox4x64-10
// ---------------------------------------------------------------------------
struct U64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U64x4 r;
  r.v[0] = c0; r.v[1] = c1; r.v[2] = c2; r.v[3] = c3;
  return r;
}

// Philox4x32-10 (same publication; 32-bit multipliers and Weyl increments).
struct U32x4 {
  uint32_t v[4];
};

__device__ __forceinline__ U32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                               uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    // one 32 x 32 -> 64-bit multiply per product (v_mad_u64_u32) gives both halves
    const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U32x4 r;
  r.v[0] = c0; r.v[1] = c1; r.v[2] = c2; r.v[3] = c3;
  return r;
}

// FP32 uniform in [0, 1) from the top 24 bits of a 32-bit word
__device__ __forceinline__ float u01_f32_w32(uint32_t w) { return (float)(w >> 8) * 0x1.0p-24f; }

// counter word 1: purpose << 32 | hit << 8 | mu
constexpr uint64_t kPurposeInit = 1ULL << 32;
constexpr uint64_t kPurposeMetro = 2ULL << 32;

__device__ __forceinline__ double u01_f64(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }
__device__ __forceinline__ float u01_f32(uint64_t w) { return (float)(uint32_t)(w >> 40) * 0x1.0p-24f; }

// ---------------------------------------------------------------------------
// Deterministic FP64 elementary functions
// ---------------------------------------------------------------------------
constexpr double kPi = 0x1.921fb54442d18p+1;  // double nearest pi
constexpr double kTwoPi = 2.0 * kPi;
// pi/2 = P1 + P2 + P3, P1 and P2 with 32 significant bits (k*P exact for |k| < 2^20)
constexpr double kPio2_1 = 0x1.921fb544p+0;
constexpr double kPio2_2 = 0x1.0b4611a6p-34;
constexpr double kPio2_3 = 0x1.3198a2e037073p-69;
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
constexpr double kTanPi8 = 0x1.a827999fcef32p-2;  // sqrt(2) - 1, correctly rounded

__device__ __forceinline__ void det_sincos(double x, double& s, double& c) {
  const double q = x * kTwoOverPi;
  const int k = (int)(q >= 0.0 ? q + 0.5 : q - 0.5);
  const double kd = (double)k;
  const double r = ((x - kd * kPio2_1) - kd * kPio2_2) - kd * kPio2_3;
  const double z = r * r;
  double ps = -1.0 / 121645100408832000.0;
  ps = ps * z + 1.0 / 355687428096000.0;
  ps = ps * z - 1.0 / 1307674368000.0;
  ps = ps * z + 1.0 / 6227020800.0;
  ps = ps * z - 1.0 / 39916800.0;
  ps = ps * z + 1.0 / 362880.0;
  ps = ps * z - 1.0 / 5040.0;
  ps = ps * z + 1.0 / 120.0;
  ps = ps * z - 1.0 / 6.0;
  const double sn = r + (r * z) * ps;
  double pc = 1.0 / 6402373705728000.0;
  pc = pc * z - 1.0 / 20922789888000.0;
  pc = pc * z + 1.0 / 87178291200.0;
  pc = pc * z - 1.0 / 479001600.0;
  pc = pc * z + 1.0 / 3628800.0;
  pc = pc * z - 1.0 / 40320.0;
  pc = pc * z + 1.0 / 720.0;
  pc = pc * z - 1.0 / 24.0;
  pc = pc * z + 1.0 / 2.0;
  const double cs = 1.0 - z * pc;
  switch (k & 3) {
    case 0: s = sn; c = cs; break;
    case 1: s = cs; c = -sn; break;
    case 2: s = -sn; c = -cs; break;
    default: s = -cs; c = sn; break;
  }
}

__device__ __forceinline__ double det_atan2(double y, double x) {
  const double ax = fabs(x), ay = fabs(y);
  if (ax == 0.0 && ay == 0.0) return 0.0;
  const bool swap = ay > ax;
  const double t = swap ? ax / ay : ay / ax;
  double base = 0.0, u = t;
  if (t > kTanPi8) {
    u = (t - 1.0) / (t + 1.0);
    base = kPi / 4.0;
  }
  const double z = u * u;
  double p = -1.0 / 39.0;
  p = p * z + 1.0 / 37.0;
  p = p * z - 1.0 / 35.0;
  p = p * z + 1.0 / 33.0;
  p = p * z - 1.0 / 31.0;
  p = p * z + 1.0 / 29.0;
  p = p * z - 1.0 / 27.0;
  p = p * z + 1.0 / 25.0;
  p = p * z - 1.0 / 23.0;
  p = p * z + 1.0 / 21.0;
  p = p * z - 1.0 / 19.0;
  p = p * z + 1.0 / 17.0;
  p = p * z - 1.0 / 15.0;
  p = p * z + 1.0 / 13.0;
  p = p * z - 1.0 / 11.0;
  p = p * z + 1.0 / 9.0;
  p = p * z - 1.0 / 7.0;
  p = p * z + 1.0 / 5.0;
  p = p * z - 1.0 / 3.0;
  double a = base + (u + (u * z) * p);
  if (swap) a = kPi / 2.0 - a;
  if (x < 0.0) a = kPi - a;
  if (y < 0.0) a = -a;
  return a;
}

__device__ __forceinline__ double wrap_f64(double a) {
  while (a >= kPi) a -= kTwoPi;
  while (a < -kPi) a += kTwoPi;
  return a;
}

// ---------------------------------------------------------------------------
// Lattice geometry
// ---------------------------------------------------------------------------
// Exact unsigned division n / d by multiply-high, valid for n * d < 2^32:
// q = mulhi(n, ceil(2^32 / d)); d = 1 is carried by the mask (m = 0, q = n).
struct FastDiv {
  uint32_t d, m, one;
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.m = d == 1 ? 0u : (uint32_t)(0xFFFFFFFFULL / d + 1ULL);
  f.one = d == 1 ? 0xFFFFFFFFu : 0u;
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) { return __umulhi(n, f.m) + (n & f.one); }

// One lattice of a batch.  Every launch covers all lattices of its batch; the
// block table maps each block to (lattice, first half-site).
struct LatDesc {
  int L, T;
  int V2;        // L^3 T / 2
  int L3;        // L^3
  FastDiv div_Lh, div_L, div_slice;  // by L/2, L, L^3/2
  double beta, eps, sqrt_beta;
  uint64_t seed;
  uint64_t off;  // offset of links[0][0][0] in the batch link buffer (elements)
};

// Time slice of the j-th updated slice of class mu: every slice, or with
// frozen slabs (spatial mu, th > 0) the slices t = 1..th-1 (mod th).
__host__ __device__ inline int class_slice(int j, int mu, int th) {
  if (mu == 0 || th <= 0) return j;
  return (j / (th - 1)) * th + (j % (th - 1)) + 1;
}
__host__ __device__ inline int class_slices(int T, int mu, int th) {
  if (mu == 0 || th <= 0) return T;
  return (T / th) * (th - 1);
}

// Workgroups go to the 8 XCDs round-robin by linear id, and every XCD has an
// L2 of its own.  xcd_block maps the linear id b of nb workgroups to a logical
// block such that XCD k runs one contiguous range of logical blocks, so that
// neighbouring sites (which read each other's links) share an L2.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t xcd = b % kXcds, local = b / kXcds;
  const uint32_t q = nb / kXcds, r = nb % kXcds;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

struct Site {
  int t, x, y, z;
};

// coordinates of the site with half-index h and the given parity
__device__ __forceinline__ Site site_of(const LatDesc& d, uint32_t h, int parity) {
  const uint32_t Lh = (uint32_t)(d.L >> 1);
  const uint32_t q = fdiv(h, d.div_Lh);
  const uint32_t xh = h - q * Lh;
  const uint32_t q2 = fdiv(q, d.div_L);
  Site s;
  s.y = (int)(q - q2 * (uint32_t)d.L);
  const uint32_t q3 = fdiv(q2, d.div_L);
  s.z = (int)(q2 - q3 * (uint32_t)d.L);
  s.t = (int)q3;
  const int b = (parity ^ (s.t + s.z + s.y)) & 1;
  s.x = 2 * (int)xh + b;
  return s;
}

__device__ __forceinline__ uint32_t natural_index(const LatDesc& d, int t, int x, int y, int z) {
  return (((uint32_t)t * d.L + z) * d.L + y) * d.L + x;
}

__device__ __forceinline__ uint32_t half_of(const LatDesc& d, int t, int x, int y, int z) {
  return natural_index(d, t, x, y, z) >> 1;
}

__device__ __forceinline__ int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// coordinates displaced by a*e_mu + b*e_nu (|a|,|b| <= 1), periodic
__device__ __forceinline__ Site shift2(const LatDesc& d, Site s, int mu, int a, int nu, int b) {
  int c[4] = {s.t, s.x, s.y, s.z};
  c[mu] += a;
  c[nu] += b;
  Site r;
  r.t = wrapc(c[0], d.T);
  r.x = wrapc(c[1], d.L);
  r.y = wrapc(c[2], d.L);
  r.z = wrapc(c[3], d.L);
  return r;
}

__device__ __forceinline__ uint64_t link_slot(const LatDesc& d, int mu, int parity, uint32_t h) {
  return d.off + ((uint64_t)(mu * 2 + parity) * (uint64_t)d.V2 + h);
}

__device__ __forceinline__ uint64_t link_at(const LatDesc& d, int mu, Site s) {
  const int p = (s.t + s.x + s.y + s.z) & 1;
  return link_slot(d, mu, p, half_of(d, s.t, s.x, s.y, s.z));
}

}  // namespace u1ml
