// field.hip -- contraction of the stored field insertions (Eq. (9)) into the
// E/B profiles over the mediator plane.
//
// Every inner sample keeps its slab time-line phases (ell) and the slab sums
// of the field operators (oall).  After the run the weights are known, and
//   F(dy, dz) = sum_{samples, slabs, x0} W(x0) O(x0 + m e_x + dy e_y + dz e_z)
// is a cyclic correlation over the (y, z) plane for every x, evaluated with
// 2D discrete Fourier transforms: G(p, q) = sum What(-p, -q) Ohat(p, q), and
// F is L^-2 times the inverse transform of G.  All sums are FP64 in a fixed
// order.
#include <algorithm>

#include "fft_reg.h"
#include "measure_common.h"

namespace u1ml {

namespace {

// tavg[((m * n_rf + f) * ns + s) * L3 + x0] = average over the n_inner samples
// of stored outer iteration m of T(x0, rf[f]) in inner slab s
__global__ void field_tavg_kernel(const LatDesc* __restrict__ lat, const MLDesc* __restrict__ mlp,
                                  const FieldLat* __restrict__ flp, FieldParams fp,
                                  const double2* __restrict__ mlbuf, double* __restrict__ fbuf) {
  const LatDesc d = *lat;
  const MLDesc ml = *mlp;
  const FieldLat fl = *flp;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= fp.n_stored * fl.ns * d.L3 * fp.n_rf) return;
  const int x0 = item % d.L3;
  const int s = (item / d.L3) % fl.ns;
  const int f = (item / (d.L3 * fl.ns)) % fp.n_rf;
  const int m = item / (d.L3 * fl.ns * fp.n_rf);
  // the slabs without the insertion take the correlator's lines: multihit
  // means for r >= 2 when enabled
  const uint64_t base = ml.multihit && fp.rf[f] >= 2 ? ml.ell_mh : ml.ell;
  const double2* ell = mlbuf + base + (size_t)m * fp.n_inner * fl.ns * d.L3;
  ((double2*)(fbuf + fl.tavg))[item] = inner_avg(ell, fp.n_inner, fl.ns, d.L3, s, x0, shift_x(d, x0, fp.rf[f]));
}

// ptop[(k * n_rf + f) * L3 + x0] = prod_{j != k} A_j(x0, rf[f]) / n_0^(n_top - 1)
// over the other top-level slabs j (two levels; the final averages A_j are
// the level-0 sums over the n_0 outer iterations); 1 for one level
__global__ void field_ptop_kernel(const LatDesc* __restrict__ lat, const MLDesc* __restrict__ mlp,
                                  const FieldLat* __restrict__ flp, FieldParams fp,
                                  const double2* __restrict__ accbuf, double* __restrict__ fbuf) {
  const LatDesc d = *lat;
  const MLDesc ml = *mlp;
  const FieldLat fl = *flp;
  const int ntop = fl.n_top;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= ntop * d.L3) return;
  // site-major: the n_top threads of one site read the same accumulator
  // lines, which the caches then serve
  const int k = item % ntop, x0 = item / ntop;
  const double inv = 1.0 / (double)fp.n_outer;
  double2* out = (double2*)(fbuf + fl.ptop);
  for (int f = 0; f < fp.n_rf; ++f) {
    double2 p = make_double2(1.0, 0.0);
    for (int j = 0; j < ntop && fp.n_levels == 2; ++j) {
      if (j == k) continue;
      const double2 a = accbuf[ml.acc[0] + ((size_t)j * d.L3 + x0) * ml.nR + fp.rf_k[f]];
      p = cmul(p, make_double2(a.x * inv, a.y * inv));
    }
    out[((size_t)k * fp.n_rf + f) * d.L3 + x0] = p;
  }
}

// w[((m * n_rf + f) * ns + s) * L3 + x0] = weight of an insertion in inner
// slab s during outer iteration m:
//   one level:  prod_{s' != s} [T]_{s'} / (n V)
//   two levels: prod_{j != k} A_j * prod_{s' in k, s' != s} [T]_{s',m} / (n_0 n_1 V)
// with k the top slab holding s and A_j the top-level averages (ptop).
__global__ void field_weights_kernel(const LatDesc* __restrict__ lat, const FieldLat* __restrict__ flp,
                                     FieldParams fp, double* __restrict__ fbuf) {
  const LatDesc d = *lat;
  const FieldLat fl = *flp;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= fp.n_stored * fp.n_rf * fl.ns * d.L3) return;
  const int x0 = item % d.L3;
  const int s = (item / d.L3) % fl.ns;
  const int f = (item / (d.L3 * fl.ns)) % fp.n_rf;
  const int m = item / (d.L3 * fl.ns * fp.n_rf);
  const int children = fl.ns / fl.n_top;
  const int k = s / children;
  const double2* tavg = (const double2*)(fbuf + fl.tavg) + (size_t)m * fp.n_rf * fl.ns * d.L3;
  double2 p = ((const double2*)(fbuf + fl.ptop))[((size_t)k * fp.n_rf + f) * d.L3 + x0];
  const int first = (s / children) * children;
  for (int j = 0; j < children; ++j) {
    const int sp = first + j;
    if (sp == s) continue;
    p = cmul(p, tavg[((size_t)f * fl.ns + sp) * d.L3 + x0]);
  }
  double norm = (double)fp.n_inner * (double)d.V2 * 2.0;
  if (fp.n_levels == 2) norm *= (double)fp.n_outer;
  ((double2*)(fbuf + fl.w))[item] = make_double2(p.x / norm, p.y / norm);
}

// 2D DFT over (y, z) of one x-plane per block, in place in LDS:
//   out[b][p][q] = sum_{y,z} v(x, y, z) exp(-2 pi i (p y + q z) / L)
// KIND 0: v = the stored field slab sums O_c of sample k (real);
// KIND 1: v = W_f(x0) = w[m][s][x0][f] T_k(x0, s; rf[f]) built on the fly,
//         transformed with exp(+2 pi i ...) so that out[b][p][q] = What(-p, -q).
// Block b enumerates (k, a, s, x) with x fastest; a = c (KIND 0) or f (KIND 1).
constexpr int kDftThreads = 256;
constexpr int kDftMaxPer = 16;  // ceil(62^2 / 256)

template <int KIND, typename O>
__global__ __launch_bounds__(kDftThreads) void field_dft_kernel(const LatDesc* __restrict__ lat,
                                                                const MLDesc* __restrict__ mlp,
                                                                const FieldLat* __restrict__ flp, FieldParams fp,
                                                                int sample0, const double2* __restrict__ mlbuf,
                                                                const double* __restrict__ fbuf,
                                                                double2* __restrict__ out) {
  extern __shared__ double2 sm[];
  const LatDesc d = *lat;
  const FieldLat fl = *flp;
  const int L = d.L, L2 = L * L, ns = fl.ns;
  const int A = KIND == 0 ? 6 : fp.n_rf;
  double2* tw = sm;       // exp(-2 pi i k / L)
  double2* buf = sm + L;  // plane [y][z] -> [y][q] -> [p][q]
  const int b = blockIdx.x;
  const int x = b % L, s = (b / L) % ns, a = (b / (L * ns)) % A, k = b / (L * ns * A);
  const int sample = sample0 + k;
  for (int i = threadIdx.x; i < L; i += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)i / (double)L, &sn, &cs);
    tw[i] = make_double2(cs, KIND == 0 ? -sn : sn);
  }
  if (KIND == 0) {
    const O* src = (const O*)(fbuf + fl.oall) + (((size_t)sample * 6 + a) * ns + s) * d.L3;
    for (int i = threadIdx.x; i < L2; i += blockDim.x) {
      const int y = i / L, z = i - y * L;
      buf[i] = make_double2((double)src[(size_t)(z * L + y) * L + x], 0.0);
    }
  } else {
    const MLDesc ml = *mlp;
    const int m = sample / fp.n_inner;
    const double2* e = mlbuf + ml.ell + ((size_t)sample * ns + s) * d.L3;
    const double2* w = (const double2*)(fbuf + fl.w);
    for (int i = threadIdx.x; i < L2; i += blockDim.x) {
      const int y = i / L, z = i - y * L;
      const int x0 = (z * L + y) * L + x;
      const double2 u = e[x0], v = e[shift_x(d, x0, fp.rf[a])];
      const double2 t = make_double2(u.x * v.x + u.y * v.y, u.x * v.y - u.y * v.x);
      buf[i] = cmul(w[(((size_t)m * fp.n_rf + a) * ns + s) * d.L3 + x0], t);
    }
  }
  __syncthreads();
  double2 r[kDftMaxPer];
  // along z: buf[y][z] -> [y][q]
#pragma unroll
  for (int j = 0; j < kDftMaxPer; ++j) {
    const int i = threadIdx.x + j * kDftThreads;
    if (i < L2) {
      const int y = i / L, q = i - y * L;
      double re = 0.0, im = 0.0;
      int kk = 0;
      for (int z = 0; z < L; ++z) {
        const double2 v = buf[y * L + z], t = tw[kk];
        re += v.x * t.x - v.y * t.y;
        im += v.x * t.y + v.y * t.x;
        kk += q;
        kk -= (kk >= L) ? L : 0;
      }
      r[j] = make_double2(re, im);
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kDftMaxPer; ++j) {
    const int i = threadIdx.x + j * kDftThreads;
    if (i < L2) buf[i] = r[j];
  }
  __syncthreads();
  // along y: [y][q] -> [p][q]
  double2* dst = out + (size_t)b * L2;
#pragma unroll
  for (int j = 0; j < kDftMaxPer; ++j) {
    const int i = threadIdx.x + j * kDftThreads;
    if (i < L2) {
      const int p = i / L, q = i - p * L;
      double re = 0.0, im = 0.0;
      int kk = 0;
      for (int y = 0; y < L; ++y) {
        const double2 v = buf[y * L + q], t = tw[kk];
        re += v.x * t.x - v.y * t.y;
        im += v.x * t.y + v.y * t.x;
        kk += p;
        kk -= (kk >= L) ? L : 0;
      }
      dst[i] = make_double2(re, im);
    }
  }
}

// part[((((k * n_rf + f) * ns + s) * 2 + plane) * 6 + c) * L2 + pq] =
//   sum_x What[k][f][s][x](-pq) * Ohat[k][c][s][x + m_plane](pq),  m_0 = (r-1)/2, m_1 = r/2.
// Block (pq tile, s, k); threads (pq in tile, f, plane).  The W tile of all x
// and the O tile of one component at a time are staged in LDS, so every
// transformed value is read from memory once.
__global__ void field_gacc_kernel(FieldParams fp, int L, int ns, int pt, const double2* __restrict__ what,
                                  const double2* __restrict__ ohat, double2* __restrict__ part) {
  extern __shared__ double2 sm[];
  const int L2 = L * L;
  const int s = blockIdx.y, k = blockIdx.z;
  const int pq0 = blockIdx.x * pt;
  const int npq = min(pt, L2 - pq0);
  double2* wt = sm;                      // [f][x][pt]
  double2* ot = sm + fp.n_rf * L * pt;  // [x][pt]
  const int tid = threadIdx.x;
  const int j = tid % pt, fpl = tid / pt;  // fpl = f * 2 + plane
  const bool active = fpl < 2 * fp.n_rf && j < npq;
  const int f = fpl >> 1, plane = fpl & 1;
  int m = 0;
  if (fpl < 2 * fp.n_rf) {
    const int r = fp.rf[f];
    m = plane == 0 ? (r - 1) / 2 : r / 2;
  }
  for (int i = tid; i < fp.n_rf * L * pt; i += blockDim.x) {
    const int jj = i % pt, x = (i / pt) % L, ff = i / (pt * L);
    wt[i] = jj < npq ? what[((((size_t)k * fp.n_rf + ff) * ns + s) * L + x) * L2 + pq0 + jj] : make_double2(0.0, 0.0);
  }
  double2 acc[6];
  for (int c = 0; c < 6; ++c) {
    __syncthreads();
    for (int i = tid; i < L * pt; i += blockDim.x) {
      const int jj = i % pt, x = i / pt;
      ot[i] = jj < npq ? ohat[((((size_t)k * 6 + c) * ns + s) * L + x) * L2 + pq0 + jj] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double re = 0.0, im = 0.0;
    if (active) {
      const double2* wr = wt + (size_t)f * L * pt + j;
      int xx = m;
      for (int x = 0; x < L; ++x) {
        const double2 w = wr[x * pt], o = ot[xx * pt + j];
        re += w.x * o.x - w.y * o.y;
        im += w.x * o.y + w.y * o.x;
        ++xx;
        xx -= (xx >= L) ? L : 0;
      }
    }
    acc[c] = make_double2(re, im);
  }
  if (active)
    for (int c = 0; c < 6; ++c)
      part[(((((size_t)k * fp.n_rf + f) * ns + s) * 2 + plane) * 6 + c) * L2 + pq0 + j] = acc[c];
}

// G[((f * 2 + plane) * 6 + c) * L2 + pq] += sum_k sum_s part[...] (fixed order)
__global__ void field_gred_kernel(FieldParams fp, int L, int ns, int nk, const double2* __restrict__ part,
                                  double2* __restrict__ G) {
  const int L2 = L * L;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= fp.n_rf * 12 * L2) return;
  const int pq = item % L2;
  const int pc = (item / L2) % 12;  // plane * 6 + c
  const int f = item / (12 * L2);
  double re = 0.0, im = 0.0;
  for (int k = 0; k < nk; ++k)
    for (int s = 0; s < ns; ++s) {
      const double2 v = part[((((size_t)k * fp.n_rf + f) * ns + s) * 12 + pc) * L2 + pq];
      re += v.x;
      im += v.y;
    }
  G[item].x += re;
  G[item].y += im;
}

// F[((f * 2 + plane) * 6 + c) * L2 + (dy, dz)] = L^-2 sum_{p,q} G(p, q) exp(+2 pi i (p dy + q dz) / L)
__global__ void field_final_kernel(FieldParams fp, int L, const double2* __restrict__ G, double2* __restrict__ F) {
  const int L2 = L * L;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= fp.n_rf * 12 * L2) return;
  const int dd = item % L2;
  const int dy = dd / L, dz = dd - dy * L;
  const double2* g = G + (size_t)(item / L2) * L2;
  double re = 0.0, im = 0.0;
  for (int p = 0; p < L; ++p)
    for (int q = 0; q < L; ++q) {
      const int k = (p * dy + q * dz) % L;
      double sn, cs;
      sincospi(2.0 * (double)k / (double)L, &sn, &cs);
      const double2 v = g[p * L + q];
      re += v.x * cs - v.y * sn;
      im += v.x * sn + v.y * cs;
    }
  const double inv = 1.0 / (double)L2;
  F[item] = make_double2(re * inv, im * inv);
}

// ---------------------------------------------------------------------------
// Fast path (L with factors 2, 3, 5 only, L <= kFxMaxL).  Each 1D transform is
// split over a lane pair: half-length FFTs in registers (fft_reg.h) and one
// radix-2 step through LDS, rows from memory into registers and columns from
// the LDS plane out to memory.  The O planes are real: two neighbouring x
// planes are transformed together as one complex plane Z = O_a + i O_b
// (field_ohat_kernel) and separated in Fourier space by the contraction
// (field_zcon_kernel),
//   Ohat_a(k) = (Z(k) + conj Z(-k)) / 2,   Ohat_b(k) = (Z(k) - conj Z(-k)) / 2i.
// ---------------------------------------------------------------------------
constexpr int kFxMaxL = 48;
constexpr size_t kFxLds = 64512;  // most LDS per block of the transform kernels (bytes)

// Storage of the per-sample transforms between the fast-path kernels: FP64
// (double2), or FP32 (float2) for FP32 lattices, whose field operators carry
// FP32 sine errors of order 1e-6 already.  The transforms themselves and
// every sum are FP64 either way.
__device__ __forceinline__ void put(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void put(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ double2 get(const double2* p) { return *p; }
template <typename S>
struct ScalarOf {
  using type = double;
};
template <>
struct ScalarOf<float2> {
  using type = float;
};
__device__ __forceinline__ double2 get(const float2* p) {
  const float2 v = *p;
  return make_double2((double)v.x, (double)v.y);
}

// In-place FFT of the N values v[i * stride] (LDS, N even) by the two lanes
// h = 0, 1 of a lane pair
// (adjacent lanes of one wavefront): lane h transforms the samples n = 2 m + h
// in registers (N / 2 points), lane 1 applies exp(SIGN 2 pi i k / N), and one
// radix-2 step through LDS combines the halves:
//   X(k) = U_0(k) + w^k U_1(k),  X(k + N/2) = U_0(k) - w^k U_1(k).
// A wavefront performs its LDS operations in issue order; the fence keeps
// the compiler from moving the partner reads above the half write-back, and
// each output depends on the partner value read at its position, so that
// read always precedes the write.
template <int N, int SIGN>
__device__ __forceinline__ void fft_line_pair(double2* v, int stride, int h) {
  constexpr int M = N / 2;
  double2 y[M];
#pragma unroll
  for (int m = 0; m < M; ++m) y[fftreg::kPos<M>.v[m]] = v[(2 * m + h) * stride];
  fftreg::run<M, SIGN>(y);
  if (h) {
#pragma unroll
    for (int k = 1; k < M; ++k) y[k] = fftreg::cmulc(y[k], fftreg::kTw<N>.c[k], (double)SIGN * fftreg::kTw<N>.s[k]);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // both lanes' reads above are done
#pragma unroll
  for (int k = 0; k < M; ++k) v[(h * M + k) * stride] = y[k];
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // the halves are in LDS
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const double2 p = v[((1 - h) * M + k) * stride];
    v[(h * M + k) * stride] = h ? fftreg::csub(p, y[k]) : fftreg::cadd(y[k], p);
  }
}

// The combining step of fft_line_pair with the lane's half transform in
// registers: lane h holds in y[k] the transform U_h(k) of its samples
// n = 2 m + h; the pair exchanges the twiddled halves through the LDS line v
// (N values at the given stride, free for the pair to overwrite) and lane h
// ends with X(k + h N / 2) in y[k].
template <int N, int SIGN>
__device__ __forceinline__ void pair_exchange(double2 (&y)[N / 2], double2* v, int stride, int h) {
  constexpr int M = N / 2;
  if (h) {
#pragma unroll
    for (int k = 1; k < M; ++k) y[k] = fftreg::cmulc(y[k], fftreg::kTw<N>.c[k], (double)SIGN * fftreg::kTw<N>.s[k]);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // earlier reads of the line are done
#pragma unroll
  for (int k = 0; k < M; ++k) v[(h * M + k) * stride] = y[k];
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // the halves are in LDS
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const double2 p = v[((1 - h) * M + k) * stride];
    y[k] = h ? fftreg::csub(p, y[k]) : fftreg::cadd(y[k], p);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // the partner halves are read
}

// What[((k * n_rf + f) * ns + s) * L + x][p * L + q] = sum_{y,z} W(x, y, z) exp(+2 pi i (p y + q z) / L),
// i.e. the transform of W at (-p, -q).  Block: (s, k, f, group of npb x
// planes), a lane pair per row (x, y) and then per column (x, q).  Each row
// pair loads its samples of W from memory into registers and transforms them
// along z (the exchange and the result go to the row in LDS); each column
// pair transforms along y from LDS and stores its outputs, so that LDS
// carries only the exchanges and the transposition.
template <int L, typename S>
__global__ __launch_bounds__(512) void field_what_kernel(const LatDesc* __restrict__ lat,
                                                         const MLDesc* __restrict__ mlp,
                                                         const FieldLat* __restrict__ flp, FieldParams fp,
                                                         int sample0, int npb, const double2* __restrict__ mlbuf,
                                                         const double* __restrict__ fbuf, S* __restrict__ what) {
  extern __shared__ double2 pl[];  // [nx][L (y)][L + 1]
  constexpr int L1 = L + 1, M = L / 2;
  const LatDesc d = *lat;
  const FieldLat fl = *flp;
  const int ns = fl.ns;
  const int ngroups = (L + npb - 1) / npb;
  // logical block order [s][k][f][group], consecutive logical blocks on one
  // XCD: the blocks of one (k, s) read the same time lines, and consecutive
  // samples of one outer iteration the same weights of (m, f, s), which an
  // XCD's L2 then keeps (samples outermost, every sample would fetch all the
  // weights of its outer iteration again)
  const int b = (int)xcd_block(blockIdx.x, gridDim.x);
  const int nk = (int)gridDim.x / (ngroups * fp.n_rf * ns);
  const int grp = b % ngroups, f = (b / ngroups) % fp.n_rf, k = (b / (ngroups * fp.n_rf)) % nk;
  const int s = b / (ngroups * fp.n_rf * nk);
  const int x0 = grp * npb, nx = min(npb, L - x0);
  const int sample = sample0 + k, m = sample / fp.n_inner;
  const MLDesc ml = *mlp;
  const double2* e = mlbuf + ml.ell + ((size_t)sample * ns + s) * d.L3;
  const double2* w = (const double2*)(fbuf + fl.w) + (((size_t)m * fp.n_rf + f) * ns + s) * d.L3;
  const int r = fp.rf[f];
  const int tid = threadIdx.x, h = tid & 1, pair = tid >> 1;
  const bool active = pair < nx * L;
  // rows: pair = (x, y), x fastest so that neighbouring pairs read
  // neighbouring x; W(x, y, z) = w(x0) conj(e(x0)) e(x0 + r), x0 = (z L + y) L + x
  if (active) {
    const int xc = pair % nx, y = pair / nx, x = x0 + xc;
    int xr = x + r;
    xr -= xr >= L ? L : 0;
    double2 v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int row = ((2 * j + h) * L + y) * L;
      const double2 u = e[row + x], t = e[row + xr];
      v[fftreg::kPos<M>.v[j]] = cmul(w[row + x], make_double2(u.x * t.x + u.y * t.y, u.x * t.y - u.y * t.x));
    }
    fftreg::run<M, 1>(v);
    double2* line = pl + (xc * L + y) * L1;
    pair_exchange<L, 1>(v, line, 1, h);
#pragma unroll
    for (int j = 0; j < M; ++j) line[h * M + j] = v[j];
  }
  __syncthreads();
  // columns: pair = (x, q); outputs p = h M + j
  if (active) {
    const int xc = pair / L, q = pair % L;
    double2* col = pl + xc * L * L1 + q;
    double2 v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[fftreg::kPos<M>.v[j]] = col[(2 * j + h) * L1];
    fftreg::run<M, 1>(v);
    pair_exchange<L, 1>(v, col, L1, h);
    S* dst = what + ((((size_t)k * fp.n_rf + f) * ns + s) * L + x0 + xc) * L * L + q;
#pragma unroll
    for (int j = 0; j < M; ++j) put(dst + (size_t)(h * M + j) * L, v[j]);
  }
}

// Zhat[((k * ns + s) * 6 + c) * (L / 2) + j][p * L + q] (complex): the
// transform over (y, z) of Z = O_c(2 j) + i O_c(2 j + 1) for sample
// sample0 + k, inner slab s, from the stored slab sums O_c.  Block: (k, s, c,
// group of np pairs); as field_what_kernel, a lane pair per row (pair plane,
// y) loads its samples from memory and transforms them along z, and a lane
// pair per column (pair plane, q) transforms along y and stores.
template <int L, typename S>
__global__ __launch_bounds__(512) void field_ohat_kernel(const LatDesc* __restrict__ lat,
                                                         const FieldLat* __restrict__ flp, int sample0, int np,
                                                         const double* __restrict__ fbuf, S* __restrict__ zhat) {
  extern __shared__ double2 zp[];  // [np][L (y)][L + 1]
  constexpr int L1 = L + 1, L2 = L * L, NP = L / 2, M = L / 2;
  const LatDesc d = *lat;
  const FieldLat fl = *flp;
  const int ns = fl.ns, ngroups = (NP + np - 1) / np;
  const int b = (int)xcd_block(blockIdx.x, gridDim.x);  // the groups of one plane share cache lines
  const int grp = b % ngroups, c = (b / ngroups) % 6, s = (b / (ngroups * 6)) % ns, k = b / (ngroups * 6 * ns);
  const int j0 = grp * np, n = min(np, NP - j0);
  // the stored sums are in the storage precision (FP32 for FP32 links)
  using O = typename ScalarOf<S>::type;
  const O* o = (const O*)(fbuf + fl.oall) + (((size_t)(sample0 + k) * 6 + c) * ns + s) * d.L3;
  const int tid = threadIdx.x, h = tid & 1, pair = tid >> 1;
  const bool active = pair < n * L;
  // rows: pair = (pair plane, y), pair planes fastest
  if (active) {
    const int pr = pair % n, y = pair / n;
    double2 v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const O* a = o + (size_t)((2 * j + h) * L + y) * L + 2 * (j0 + pr);
      v[fftreg::kPos<M>.v[j]] = make_double2((double)a[0], (double)a[1]);
    }
    fftreg::run<M, -1>(v);
    double2* line = zp + (pr * L + y) * L1;
    pair_exchange<L, -1>(v, line, 1, h);
#pragma unroll
    for (int j = 0; j < M; ++j) line[h * M + j] = v[j];
  }
  __syncthreads();
  // columns: pair = (pair plane, q); outputs p = h M + j
  if (active) {
    const int pr = pair / L, q = pair % L;
    double2* col = zp + pr * L * L1 + q;
    double2 v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[fftreg::kPos<M>.v[j]] = col[(2 * j + h) * L1];
    fftreg::run<M, -1>(v);
    pair_exchange<L, -1>(v, col, L1, h);
    S* dst = zhat + ((((size_t)k * ns + s) * 6 + c) * NP + j0 + pr) * L2 + q;
#pragma unroll
    for (int j = 0; j < M; ++j) put(dst + (size_t)(h * M + j) * L, v[j]);
  }
}

// part[((k * nsg + sg) * 6 + c) * 2 n_rf L^2 + (2 f + plane) L^2 + p L + q]:
//   sum over the slabs s of group sg (s = sg sps .. sg sps + sps - 1) and over x
//   of What[k][f][s][x - m](p, q) * Ohat_c[k][s][x](p, q),  m_0 = (r - 1) / 2, m_1 = r / 2.
// Thread = (sample k, slab group sg, frequency (p, q), component half h, chunk
// of up to kZcF separations): the 3 components c = 3 h .. 3 h + 2 of every
// separation of the chunk and both planes in registers, so that each W value
// read serves three components and each Ohat value three separations.  Ohat
// comes from the pair transforms.  With m_1 = m_0 (odd r) or m_0 + 1 (even
// r), plane 1 at x uses the W plane that plane 0 used at x (odd) or x - 1
// (even), so every W value is read once per thread: w1 carries W(x - 1 - m_0)
// from pair to pair.  The values of the next x pair are loaded before the
// sums of the current one.  Summing the slabs of a group in registers
// divides the partial sums written, and read back by field_gsum_kernel, by
// sps.
constexpr int kZcF = 3;
constexpr int kZcSlabs = 3;  // slabs per contraction thread
template <int L, typename S>
__global__ __launch_bounds__(256) void field_zcon_kernel(const FieldLat* __restrict__ flp, FieldParams fp,
                                                         int nblk_e, int sps, const S* __restrict__ zhat,
                                                         const S* __restrict__ what, double2* __restrict__ part) {
  constexpr int L2 = L * L, NP = L / 2;
  const FieldLat fl = *flp;
  const int ns = fl.ns, nsg = (ns + sps - 1) / sps;
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x);  // the blocks of one (k, sg) share an L2
  const int eb = lb % nblk_e, sg = (lb / nblk_e) % nsg, k = lb / (nblk_e * nsg);
  const int n_fc = (fp.n_rf + kZcF - 1) / kZcF;
  const int e = eb * (int)blockDim.x + (int)threadIdx.x;
  if (e >= n_fc * 2 * L2) return;
  const int pq = e % L2, h = (e / L2) % 2, f0 = (e / (2 * L2)) * kZcF;
  const int nf = min(kZcF, fp.n_rf - f0);
  const int p = pq / L, q = pq - p * L;
  const int ib = (p == 0 ? 0 : L - p) * L + (q == 0 ? 0 : L - q);  // (-p, -q)
  // separations past the last of the chunk repeat the last one (loaded and
  // summed like the others, never stored), so that no branch separates the
  // loads of one x pair
  double2 g0[kZcF][3], g1[kZcF][3];
  int m0[kZcF], fj[kZcF];
  bool even[kZcF];
#pragma unroll
  for (int j = 0; j < kZcF; ++j) {
#pragma unroll
    for (int c = 0; c < 3; ++c) g0[j][c] = g1[j][c] = make_double2(0.0, 0.0);
    fj[j] = min(f0 + j, fp.n_rf - 1);
    const int r = fp.rf[fj[j]];
    m0[j] = (r - 1) / 2;
    even[j] = (r & 1) == 0;
  }
  const int s_end = min(ns, (sg + 1) * sps);
  for (int s = sg * sps; s < s_end; ++s) {
    const S* z = zhat + (((size_t)k * ns + s) * 6 + 3 * h) * NP * L2;
    const S* wk = what + ((size_t)k * fp.n_rf * ns + s) * L * L2 + pq;  // + (f ns L + x) L2
    const S* wfj[kZcF];
    int xa0[kZcF];  // W plane of plane 0 at x = 0
    double2 w1[kZcF];
#pragma unroll
    for (int j = 0; j < kZcF; ++j) {
      wfj[j] = wk + (size_t)fj[j] * ns * L * L2;
      xa0[j] = m0[j] == 0 ? 0 : L - m0[j];
      w1[j] = get(wfj[j] + (size_t)(L - 1 - m0[j]) * L2);  // W(-1 - m_0)
    }
    // offset of the W plane that plane 0 uses at x (0 <= x < L)
    auto wplane = [&](int j, int x) {
      const int a = xa0[j] + x;
      return (size_t)(a >= L ? a - L : a) * L2;
    };
    // the stored values of x pair jp (cz, cm: Zhat at (p, q) and (-p, -q);
    // ca, cb: W of plane 0 at x = 2 jp, 2 jp + 1); those of pair jp + 1 are
    // loaded before the sums of pair jp, and the last pair loads itself again
    // (unused)
    S cz[3], cm[3], ca[kZcF], cb[kZcF];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cz[c] = z[(size_t)c * NP * L2 + pq];
      cm[c] = z[(size_t)c * NP * L2 + ib];
    }
#pragma unroll
    for (int j = 0; j < kZcF; ++j) {
      ca[j] = wfj[j][wplane(j, 0)];
      cb[j] = wfj[j][wplane(j, 1)];
    }
    for (int jp = 0; jp < NP; ++jp) {
      const int jn = jp + 1 < NP ? jp + 1 : jp;
      S nz[3], nm[3], na[kZcF], nb[kZcF];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        nz[c] = z[((size_t)c * NP + jn) * L2 + pq];
        nm[c] = z[((size_t)c * NP + jn) * L2 + ib];
      }
#pragma unroll
      for (int j = 0; j < kZcF; ++j) {
        na[j] = wfj[j][wplane(j, 2 * jn)];
        nb[j] = wfj[j][wplane(j, 2 * jn + 1)];
      }
      double2 oa[3], ob[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double2 za = get(&cz[c]), zm = get(&cm[c]);
        oa[c] = make_double2(0.5 * (za.x + zm.x), 0.5 * (za.y - zm.y));   // Ohat of x = 2 jp
        ob[c] = make_double2(0.5 * (za.y + zm.y), -0.5 * (za.x - zm.x));  // Ohat of x = 2 jp + 1
      }
#pragma unroll
      for (int j = 0; j < kZcF; ++j) {
        const double2 wa = get(&ca[j]), wb = get(&cb[j]);
        const double2 ha = even[j] ? w1[j] : wa, hb = even[j] ? wa : wb;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          g0[j][c].x += (wa.x * oa[c].x - wa.y * oa[c].y) + (wb.x * ob[c].x - wb.y * ob[c].y);
          g0[j][c].y += (wa.x * oa[c].y + wa.y * oa[c].x) + (wb.x * ob[c].y + wb.y * ob[c].x);
          g1[j][c].x += (ha.x * oa[c].x - ha.y * oa[c].y) + (hb.x * ob[c].x - hb.y * ob[c].y);
          g1[j][c].y += (ha.x * oa[c].y + ha.y * oa[c].x) + (hb.x * ob[c].y + hb.y * ob[c].x);
        }
        w1[j] = wb;
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cz[c] = nz[c];
        cm[c] = nm[c];
      }
#pragma unroll
      for (int j = 0; j < kZcF; ++j) {
        ca[j] = na[j];
        cb[j] = nb[j];
      }
    }
  }
  const int n_ent = 2 * fp.n_rf * L2;
  double2* out = part + ((size_t)(k * nsg + sg) * 6 + 3 * h) * n_ent + pq;
#pragma unroll
  for (int j = 0; j < kZcF; ++j) {
    if (j < nf) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        out[(size_t)c * n_ent + (2 * (f0 + j)) * L2] = g0[j][c];
        out[(size_t)c * n_ent + (2 * (f0 + j) + 1) * L2] = g1[j][c];
      }
    }
  }
}

// F = L^-2 sum_{p,q} G(p, q) exp(+2 pi i (p dy + q dz) / L) for every
// (r_f, plane, c) plane of G (the field_final_kernel sum by row and column
// FFTs): block per plane, a lane pair per row, then per column.
template <int L>
__global__ __launch_bounds__(128) void field_final_fft_kernel(const double2* __restrict__ G, double2* __restrict__ F) {
  __shared__ double2 pl[L * (L + 1)];
  constexpr int L1 = L + 1, L2 = L * L;
  const double2* g = G + (size_t)blockIdx.x * L2;
  const int tid = threadIdx.x;
  for (int i = tid; i < L2; i += blockDim.x) pl[(i / L) * L1 + i % L] = g[i];
  __syncthreads();
  const bool active = tid < 2 * L;
  const int t = tid >> 1, h = tid & 1;
  if (active) fft_line_pair<L, 1>(pl + t * L1, 1, h);  // along q
  __syncthreads();
  if (active) fft_line_pair<L, 1>(pl + t, L1, h);  // along p
  __syncthreads();
  const double inv = 1.0 / (double)L2;
  double2* out = F + (size_t)blockIdx.x * L2;
  for (int i = tid; i < L2; i += blockDim.x) {
    const double2 v = pl[(i / L) * L1 + i % L];
    out[i] = make_double2(v.x * inv, v.y * inv);
  }
}

// G[((f * 2 + plane) * 6 + c) * L2 + pq] += sum over the n_terms (k, g) of
// part.  Block: kGsEnt entries x kGsSeg segments; segment j sums the terms
// j, j + kGsSeg, j + 2 kGsSeg, ... in two interleaved partial sums, and the
// segment sums are added in segment order (a fixed order throughout).
constexpr int kGsEnt = 32, kGsSeg = 8;
__global__ __launch_bounds__(kGsEnt * kGsSeg) void field_gsum_kernel(FieldParams fp, int L, int n_terms,
                                                                     const double2* __restrict__ part,
                                                                     double2* __restrict__ G) {
  __shared__ double2 seg[kGsSeg][kGsEnt];
  const int L2 = L * L, n_ent = 2 * fp.n_rf * L2;
  const int le = (int)threadIdx.x % kGsEnt, sj = (int)threadIdx.x / kGsEnt;
  const int item = (int)blockIdx.x * kGsEnt + le;
  double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
  if (item < 6 * n_ent) {
    const int pq = item % L2, c = (item / L2) % 6, fpl = item / (6 * L2);
    const double2* src = part + (size_t)c * n_ent + fpl * L2 + pq;
    const size_t stride = (size_t)6 * n_ent;  // one term (k, g)
    int j = sj;
    for (; j + kGsSeg < n_terms; j += 2 * kGsSeg) {
      const double2 u = src[(size_t)j * stride], v = src[(size_t)(j + kGsSeg) * stride];
      a.x += u.x;
      a.y += u.y;
      b.x += v.x;
      b.y += v.y;
    }
    if (j < n_terms) {
      const double2 u = src[(size_t)j * stride];
      a.x += u.x;
      a.y += u.y;
    }
  }
  seg[sj][le] = make_double2(a.x + b.x, a.y + b.y);
  __syncthreads();
  if (sj == 0 && item < 6 * n_ent) {
    double2 t = seg[0][le];
#pragma unroll
    for (int u = 1; u < kGsSeg; ++u) {
      t.x += seg[u][le].x;
      t.y += seg[u][le].y;
    }
    G[item].x += t.x;
    G[item].y += t.y;
  }
}

// planes per block of the transform kernels (field_what_kernel,
// field_ohat_kernel) over n_planes planes: the count that keeps the most
// planes resident per compute unit (kCuLds bytes of LDS, blocks of at most
// kFxLds), with idle lanes of a partial wavefront and idle planes of a
// partial last group counted as lost
constexpr size_t kCuLds = 160 * 1024;
constexpr int kCuThreads = 2048;
int transform_planes(int L, int n_planes) {
  const size_t pb = (size_t)L * (L + 1) * sizeof(double2);
  int best = 1;
  double best_score = -1.0;
  for (int np = 1; np <= n_planes && (size_t)np * pb <= kFxLds; ++np) {
    const int thr = (2 * np * L + 63) / 64 * 64;
    const int bpc = std::min<int>((int)(kCuLds / ((size_t)np * pb)), kCuThreads / thr);
    const int groups = (n_planes + np - 1) / np;
    const double score =
        (double)bpc * np * (2.0 * np * L / thr) * ((double)n_planes / ((double)groups * np));
    if (score > best_score + 1e-9) {
      best = np;
      best_score = score;
    }
  }
  return best;
}

// threads per block of field_zcon_kernel for n items per (k, g): the
// multiple of 64 up to 256 that leaves the fewest idle lanes (the largest
// among equals)
int zcon_threads(int n) {
  int best = 256;
  for (int t = 256; t >= 64; t -= 64)
    if ((n + t - 1) / t * t - n < (n + best - 1) / best * best - n) best = t;
  return best;
}

// the most planes per block a transform block can hold: LDS (kFxLds) and
// 512 threads (a lane pair per row of every plane)
int max_transform_planes(int L, int n_planes) {
  const size_t pb = (size_t)L * (L + 1) * sizeof(double2);
  return std::max(1, std::min<int>({n_planes, (int)(kFxLds / pb), 512 / (2 * L)}));
}

template <int L, typename S>
hipError_t launch_fast_contract(const LatDesc* lat, const MLDesc* ml, const FieldLat* fl, int ns, FieldParams fp,
                                const double2* mlbuf, const double* fbuf, double2* scratch, size_t scratch_elems,
                                double2* G, double2* F, bool finalize, FieldTuning tune, hipStream_t st) {
  const uint64_t L3 = (uint64_t)L * L * L, L2 = (uint64_t)L * L;
  const size_t plane_bytes = (size_t)L * (L + 1) * sizeof(double2);  // LDS rows padded to L + 1
  const int npb_w = tune.w_planes > 0 ? std::min(tune.w_planes, max_transform_planes(L, L)) : transform_planes(L, L);
  // pair planes per transform block
  const int np_o =
      tune.o_planes > 0 ? std::min(tune.o_planes, max_transform_planes(L, L / 2)) : transform_planes(L, L / 2);
  const int n_ent = 2 * fp.n_rf * (int)L2;
  const int thr_w = (2 * npb_w * L + 63) / 64 * 64;  // lane pairs per row
  const int thr_o = (2 * np_o * L + 63) / 64 * 64;
  const int ngroups_w = (L + npb_w - 1) / npb_w;
  const int ngroups_o = (L / 2 + np_o - 1) / np_o;
  const int sps = std::min(ns, kZcSlabs), nsg = (ns + sps - 1) / sps;
  const int n_zc = ((fp.n_rf + kZcF - 1) / kZcF) * 2 * (int)L2;  // contraction threads per (k, g)
  const int thr_z = tune.zcon_threads > 0 ? std::min(256, (tune.zcon_threads + 63) / 64 * 64) : zcon_threads(n_zc);
  const int nblk_e = (n_zc + thr_z - 1) / thr_z;
  // scratch bytes per sample: What [n_rf][ns][L3] and Zhat [ns][6][L3 / 2]
  // (storage type S), part [nsg][6][n_ent] (double2)
  const uint64_t per_sample = ((uint64_t)fp.n_rf * ns * L3 + (uint64_t)ns * 3 * L3) * sizeof(S) +
                              (uint64_t)nsg * 6 * n_ent * sizeof(double2);
  const int chunk =
      (int)std::max<uint64_t>(1, std::min<uint64_t>(64, scratch_elems * sizeof(double2) / per_sample));
  const int n_samples = fp.n_stored * fp.n_inner;
  for (int s0 = 0; s0 < n_samples; s0 += chunk) {
    const int nk = std::min(chunk, n_samples - s0);
    S* what = (S*)scratch;
    S* zhat = what + (uint64_t)nk * fp.n_rf * ns * L3;
    const uint64_t s_elems = (uint64_t)nk * (fp.n_rf * ns * L3 + ns * 3 * L3);
    double2* part = scratch + (s_elems * sizeof(S) + sizeof(double2) - 1) / sizeof(double2);
    hipLaunchKernelGGL((field_what_kernel<L, S>), dim3((unsigned)((uint64_t)nk * fp.n_rf * ns * ngroups_w)), dim3(thr_w),
                       npb_w * plane_bytes, st, lat, ml, fl, fp, s0, npb_w, mlbuf, fbuf, what);
    hipLaunchKernelGGL((field_ohat_kernel<L, S>), dim3((unsigned)((uint64_t)nk * ns * 6 * ngroups_o)), dim3(thr_o),
                       np_o * plane_bytes, st, lat, fl, s0, np_o, fbuf, zhat);
    hipLaunchKernelGGL((field_zcon_kernel<L, S>), dim3((unsigned)((uint64_t)nk * nsg * nblk_e)), dim3(thr_z), 0, st,
                       fl, fp, nblk_e, sps, zhat, what, part);
    hipLaunchKernelGGL(field_gsum_kernel, dim3((unsigned)((6 * (uint64_t)n_ent + kGsEnt - 1) / kGsEnt)),
                       dim3(kGsEnt * kGsSeg), 0, st, fp, L, nk * nsg, part, G);
  }
  if (finalize)
    hipLaunchKernelGGL(field_final_fft_kernel<L>, dim3(fp.n_rf * 12), dim3((2 * L + 63) / 64 * 64), 0, st, G, F);
  return hipGetLastError();
}

// the fast path for lattice size L: one of the instantiated lengths
typedef hipError_t (*FastContract)(const LatDesc*, const MLDesc*, const FieldLat*, int, FieldParams, const double2*,
                                   const double*, double2*, size_t, double2*, double2*, bool, FieldTuning,
                                   hipStream_t);
FastContract fast_contract_for(int L, bool fp32_store) {
  if (L > kFxMaxL) return nullptr;
  switch (L) {
#define U1ML_FAST_L(n) \
  case n:              \
    return fp32_store ? launch_fast_contract<n, float2> : launch_fast_contract<n, double2>;
    U1ML_FAST_L(2)
    U1ML_FAST_L(4)
    U1ML_FAST_L(6)
    U1ML_FAST_L(8)
    U1ML_FAST_L(10)
    U1ML_FAST_L(12)
    U1ML_FAST_L(16)
    U1ML_FAST_L(18)
    U1ML_FAST_L(20)
    U1ML_FAST_L(24)
    U1ML_FAST_L(30)
    U1ML_FAST_L(32)
    U1ML_FAST_L(36)
    U1ML_FAST_L(40)
    U1ML_FAST_L(48)
#undef U1ML_FAST_L
    default:
      return nullptr;
  }
}

}  // namespace

hipError_t launch_field_contract(const LatDesc* lat, const MLDesc* ml, const FieldLat* fl, const FieldLat& hfl,
                                 FieldParams fp, int L, const double2* mlbuf, const double2* accbuf, double* fbuf,
                                 double2* scratch, size_t scratch_elems, double2* F, bool general, bool fp32_store,
                                 bool zero_g, bool finalize, bool tavg_ready, FieldTuning tune, hipStream_t st) {
  const uint64_t L3 = (uint64_t)L * L * L, L2 = (uint64_t)L * L;
  const int ns = hfl.ns;
  const uint64_t nt = (uint64_t)fp.n_stored * ns * L3 * fp.n_rf;
  if (!tavg_ready)
    hipLaunchKernelGGL(field_tavg_kernel, dim3(blocks_for(nt, 256)), dim3(256), 0, st, lat, ml, fl, fp, mlbuf, fbuf);
  hipLaunchKernelGGL(field_ptop_kernel, dim3(blocks_for((uint64_t)hfl.n_top * L3, 256)), dim3(256), 0, st, lat, ml,
                     fl, fp, accbuf, fbuf);
  hipLaunchKernelGGL(field_weights_kernel, dim3(blocks_for(nt, 256)), dim3(256), 0, st, lat, fl, fp, fbuf);
  double2* G = (double2*)(fbuf + hfl.g);
  const uint64_t ng = (uint64_t)fp.n_rf * 12 * L2;
  if (zero_g) hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(ng, 256)), dim3(256), 0, st, G, ng);
  if (FastContract fc = general ? nullptr : fast_contract_for(L, fp32_store)) {
    return fc(lat, ml, fl, ns, fp, mlbuf, fbuf, scratch, scratch_elems, G, F, finalize, tune, st);
  }
  // general path: both transforms stored, contraction by pq tiles
  // scratch per chunk: What [nk][n_rf][ns][L3], Ohat [nk][6][ns][L3], part [nk][n_rf][ns][12][L2]
  const uint64_t per_sample = (uint64_t)(fp.n_rf + 6) * ns * L3 + (uint64_t)fp.n_rf * ns * 12 * L2;
  const int chunk = (int)std::max<uint64_t>(1, std::min<uint64_t>(64, scratch_elems / per_sample));
  const int n_samples = fp.n_stored * fp.n_inner;
  const size_t shm = (size_t)(L + L2) * sizeof(double2);
  // pq tile of the accumulation: LDS holds (n_rf + 1) L pt complex values
  int pt = 64;
  while (pt > 1 && (size_t)(fp.n_rf + 1) * L * pt * sizeof(double2) > 60000) pt >>= 1;
  const size_t gshm = (size_t)(fp.n_rf + 1) * L * pt * sizeof(double2);
  const int gthreads = ((2 * fp.n_rf * pt + 63) / 64) * 64;
  for (int s0 = 0; s0 < n_samples; s0 += chunk) {
    const int nk = std::min(chunk, n_samples - s0);
    double2* what = scratch;
    double2* ohat = what + (uint64_t)nk * fp.n_rf * ns * L3;
    double2* part = ohat + (uint64_t)nk * 6 * ns * L3;
    hipLaunchKernelGGL((field_dft_kernel<1, double>), dim3((unsigned)((uint64_t)nk * fp.n_rf * ns * L)), dim3(kDftThreads), shm,
                       st, lat, ml, fl, fp, s0, mlbuf, fbuf, what);
    if (fp32_store)
      hipLaunchKernelGGL((field_dft_kernel<0, float>), dim3((unsigned)((uint64_t)nk * 6 * ns * L)), dim3(kDftThreads),
                         shm, st, lat, ml, fl, fp, s0, mlbuf, fbuf, ohat);
    else
      hipLaunchKernelGGL((field_dft_kernel<0, double>), dim3((unsigned)((uint64_t)nk * 6 * ns * L)),
                         dim3(kDftThreads), shm, st, lat, ml, fl, fp, s0, mlbuf, fbuf, ohat);
    hipLaunchKernelGGL(field_gacc_kernel, dim3((unsigned)((L2 + pt - 1) / pt), ns, nk), dim3(gthreads), gshm, st, fp, L,
                       ns, pt, what, ohat, part);
    hipLaunchKernelGGL(field_gred_kernel, dim3(blocks_for(ng, 64)), dim3(64), 0, st, fp, L, ns, nk, part, G);
  }
  if (finalize) hipLaunchKernelGGL(field_final_kernel, dim3(blocks_for(ng, 64)), dim3(64), 0, st, fp, L, G, F);
  return hipGetLastError();
}

int field_max_planes(int L, bool pairs) {
  if (!fast_contract_for(L, false)) return 0;
  return max_transform_planes(L, pairs ? L / 2 : L);
}

}  // namespace u1ml
