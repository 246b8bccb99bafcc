// measure.hip -- observables and multilevel estimators, FP64 accumulation.
//
//  * plaquette (Eq. (3) normalised per plaquette) and the six field operators
//    a^2 F_munu = sqrt(beta) Im P_munu (Eq. (5)): E_i from P_0i, B_i from P_jk;
//  * Polyakov loop P(x) = exp(i sum_t theta_0(x, t)) and the plain correlator
//    C(r) = L^-3 sum_x P*(x) P(x + r e_x);
//  * multilevel (Sec. 2.2): time-line angle sums of the innermost slabs per
//    sample, slab averages of the two-link products T(x0, r) of Eq. (8) and
//    their nested products, and the field insertion of Eq. (9): every inner
//    sample's time lines and field slab sums stay in HBM and are contracted
//    with the final weights after the run, by 2D DFTs over the mediator plane.
// All sums are FP64 with a fixed reduction order (results do not depend on
// timing).  Links are read as FP64 or FP32 angles.
#include <algorithm>

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

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cexpi(double phi) {
  double s, c;
  sincos(phi, &s, &c);
  return make_double2(c, s);
}

// ---------------------------------------------------------------------------
// plain observables
// ---------------------------------------------------------------------------
template <typename R>
__global__ void plaq_field_kernel(const R* __restrict__ links, const LatDesc* __restrict__ lats,
                                  const int2* __restrict__ blocks, double* __restrict__ partial) {
  __shared__ double sh[16];
  const int2 bk = blocks[blockIdx.x];
  const LatDesc d = lats[bk.x];
  const uint32_t n = (uint32_t)bk.y + threadIdx.x;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  if (n < 2u * (uint32_t)d.V2) {
    const Site s = as_site(coords_natural(d, n));
    const double p01 = plaq_angle(links, d, s, 0, 1), p02 = plaq_angle(links, d, s, 0, 2);
    const double p03 = plaq_angle(links, d, s, 0, 3), p12 = plaq_angle(links, d, s, 1, 2);
    const double p13 = plaq_angle(links, d, s, 1, 3), p23 = plaq_angle(links, d, s, 2, 3);
    v[0] = ((((cos(p01) + cos(p02)) + cos(p03)) + cos(p12)) + cos(p13)) + cos(p23);
    const double sb = d.sqrt_beta;
    v[1] = sb * sin(p01);
    v[2] = sb * sin(p02);
    v[3] = sb * sin(p03);
    v[4] = sb * sin(p23);
    v[5] = -sb * sin(p13);
    v[6] = sb * sin(p12);
  }
  for (int j = 0; j < 7; ++j) {
    const double r = block_sum(v[j], sh);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * 7 + j] = r;
  }
}

// out[lat * width + col] = sum of partial[row * width + col] over the rows of lat
__global__ void reduce_rows_kernel(const double* __restrict__ partial, int width, const int* __restrict__ row_begin,
                                   double* __restrict__ out) {
  __shared__ double sh[16];
  const int lat = blockIdx.x, col = blockIdx.y;
  const int b = row_begin[lat], e = row_begin[lat + 1];
  double acc = 0.0;
  for (int r = b + (int)threadIdx.x; r < e; r += blockDim.x) acc += partial[(size_t)r * width + col];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[(size_t)lat * width + col] = s;
}

template <typename R>
__global__ void poly_lines_kernel(const R* __restrict__ links, const LatDesc* __restrict__ lats,
                                  const int2* __restrict__ blocks, const uint64_t* __restrict__ poly_off,
                                  double* __restrict__ poly) {
  const int2 bk = blocks[blockIdx.x];
  const LatDesc d = lats[bk.x];
  const int x3 = bk.y + (int)threadIdx.x;
  if (x3 >= d.L3) return;
  poly[poly_off[bk.x] + x3] = time_line(links, d, x3, 0, d.T);
}

// one row per spatial site: {cos P, sin P, then (Re, Im) of P*(x)P(x+r) per r}
__global__ void poly_corr_kernel(const LatDesc* __restrict__ lats, const int2* __restrict__ blocks,
                                 const uint64_t* __restrict__ poly_off, const double* __restrict__ poly,
                                 const int* __restrict__ rvals, int nR, const int* __restrict__ row_begin,
                                 double* __restrict__ rows) {
  const int2 bk = blocks[blockIdx.x];
  const LatDesc d = lats[bk.x];
  const int x3 = bk.y + (int)threadIdx.x;
  if (x3 >= d.L3) return;
  const double* pl = poly + poly_off[bk.x];
  const double phi = pl[x3];
  const int width = 2 + 2 * nR;
  double* row = rows + (size_t)(row_begin[bk.x] + x3) * width;
  double s, c;
  sincos(phi, &s, &c);
  row[0] = c;
  row[1] = s;
  for (int k = 0; k < nR; ++k) {
    const double dphi = pl[shift_x(d, x3, rvals[k])] - phi;
    sincos(dphi, &s, &c);
    row[2 + 2 * k] = c;
    row[3 + 2 * k] = s;
  }
}

// ---------------------------------------------------------------------------
// multilevel
// ---------------------------------------------------------------------------
template <typename R>
__global__ void ml_lines_kernel(const R* __restrict__ links, const LatDesc* __restrict__ lats,
                                const MLDesc* __restrict__ mls, const int2* __restrict__ blocks, int inner_th,
                                int sample, double2* __restrict__ mlbuf) {
  const int2 bk = blocks[blockIdx.x];
  const LatDesc d = lats[bk.x];
  const int ns = d.T / inner_th;
  const int item = bk.y + (int)threadIdx.x;
  if (item >= ns * d.L3) return;
  const int s = item / d.L3, x3 = item - s * d.L3;
  // exp(i l), l = sum of theta_0 over the slab's times: the slab product of U_0
  mlbuf[mls[bk.x].ell + ((size_t)sample * ns + s) * d.L3 + x3] = cexpi(time_line(links, d, x3, s * inner_th, inner_th));
}

// average over the stored samples of T(x0, r) = conj(e(x0)) e(x0 + r) of inner slab cs
__device__ __forceinline__ double2 inner_avg(const double2* ell, int n_samples, int ns, int L3, int cs, int x0,
                                             int x0r) {
  double2 a = make_double2(0.0, 0.0);
  for (int i = 0; i < n_samples; ++i) {
    const double2* e = ell + ((size_t)i * ns + cs) * L3;
    const double2 u = e[x0], v = e[x0r];
    a.x += u.x * v.x + u.y * v.y;
    a.y += u.x * v.y - u.y * v.x;
  }
  const double inv = 1.0 / (double)n_samples;
  return make_double2(a.x * inv, a.y * inv);
}

// acc_parent[S][x0][k] += prod over the children of S of the child averages.
// parent_level == n_levels denotes the top (one slab spanning all of T).
// One thread per (S, x0, block of up to kFoldR separations).
constexpr int kFoldR = 8;
__global__ void ml_fold_kernel(const LatDesc* __restrict__ lats, const MLDesc* __restrict__ mls,
                               const int2* __restrict__ blocks, int child_level, int parent_level, int n_levels,
                               int child_is_inner, int n_child, int sample_base, const int* __restrict__ rvals,
                               const double2* __restrict__ mlbuf, double2* __restrict__ accbuf) {
  const int2 bk = blocks[blockIdx.x];
  const LatDesc d = lats[bk.x];
  const MLDesc m = mls[bk.x];
  const int ns_child = m.ns[child_level];
  const int ns_parent = parent_level == n_levels ? 1 : m.ns[parent_level];
  const int children = ns_child / ns_parent;
  const int nchunk = (m.nR + kFoldR - 1) / kFoldR;
  const int item = bk.y + (int)threadIdx.x;
  if (item >= ns_parent * d.L3 * nchunk) return;
  const int chunk = item % nchunk;
  const int x0 = (item / nchunk) % d.L3;
  const int S = item / (nchunk * d.L3);
  const int k0 = chunk * kFoldR;
  const int kn = min(kFoldR, m.nR - k0);
  int xr[kFoldR];
  double2 prod[kFoldR];
#pragma unroll
  for (int j = 0; j < kFoldR; ++j) {
    xr[j] = j < kn ? shift_x(d, x0, rvals[m.r_off + k0 + j]) : x0;
    prod[j] = make_double2(1.0, 0.0);
  }
  const double inv = 1.0 / (double)n_child;
  for (int c = 0; c < children; ++c) {
    const int cs = S * children + c;
    double2 avg[kFoldR];
#pragma unroll
    for (int j = 0; j < kFoldR; ++j) avg[j] = make_double2(0.0, 0.0);
    if (child_is_inner) {
      const double2* ell = mlbuf + m.ell + ((size_t)sample_base * ns_child + cs) * d.L3;
      for (int i = 0; i < n_child; ++i) {
        const double2* e = ell + (size_t)i * ns_child * d.L3;
        const double2 u = e[x0];
#pragma unroll
        for (int j = 0; j < kFoldR; ++j) {
          if (j < kn) {
            const double2 v = e[xr[j]];
            avg[j].x += u.x * v.x + u.y * v.y;
            avg[j].y += u.x * v.y - u.y * v.x;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < kFoldR; ++j) avg[j] = make_double2(avg[j].x * inv, avg[j].y * inv);
    } else {
      double2* cp = accbuf + m.acc[child_level] + ((size_t)cs * d.L3 + x0) * m.nR + k0;
#pragma unroll
      for (int j = 0; j < kFoldR; ++j) {
        if (j < kn) {
          avg[j] = make_double2(cp[j].x * inv, cp[j].y * inv);
          cp[j] = make_double2(0.0, 0.0);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kFoldR; ++j) prod[j] = cmul(prod[j], avg[j]);
  }
  double2* pp = accbuf + m.acc[parent_level] + ((size_t)S * d.L3 + x0) * m.nR + k0;
#pragma unroll
  for (int j = 0; j < kFoldR; ++j) {
    if (j < kn) {
      pp[j].x += prod[j].x;
      pp[j].y += prod[j].y;
    }
  }
}

// The same fold for innermost children, one block per (parent slab S, x-row
// (y, z)): the rows of the stored samples are staged in LDS, so every time
// line is read from memory once instead of once per separation.  Threads own
// up to kFoldItems items (x0, k) with x0 fastest; the sample and child order of
// the sums is that of ml_fold_kernel, so both give the same bits.
constexpr int kFoldItems = 4;
constexpr int kFoldStage = 8;  // samples per LDS round
__global__ void ml_fold_rows_kernel(const LatDesc* __restrict__ lats, const MLDesc* __restrict__ mls,
                                    const int2* __restrict__ blocks, int child_level, int parent_level, int n_levels,
                                    int n_child, int sample_base, const int* __restrict__ rvals,
                                    const double2* __restrict__ mlbuf, double2* __restrict__ accbuf) {
  extern __shared__ double2 rowbuf[];  // [kFoldStage][L]
  const int2 bk = blocks[blockIdx.x];
  const LatDesc d = lats[bk.x];
  const MLDesc m = mls[bk.x];
  const int L = d.L, L2 = L * L;
  const int ns_child = m.ns[child_level];
  const int ns_parent = parent_level == n_levels ? 1 : m.ns[parent_level];
  const int children = ns_child / ns_parent;
  const int S = bk.y / L2, row = bk.y - S * L2;
  const int nitems = L * m.nR;
  int x0[kFoldItems], xr[kFoldItems];
  double2 prod[kFoldItems];
#pragma unroll
  for (int j = 0; j < kFoldItems; ++j) {
    const int item = (int)threadIdx.x + j * (int)blockDim.x;
    const int k = item / L;
    x0[j] = item - k * L;
    int x = item < nitems ? x0[j] + rvals[m.r_off + k] : x0[j];
    x -= x >= L ? L : 0;
    xr[j] = x;
    prod[j] = make_double2(1.0, 0.0);
  }
  const double inv = 1.0 / (double)n_child;
  for (int c = 0; c < children; ++c) {
    const int cs = S * children + c;
    double2 avg[kFoldItems];
#pragma unroll
    for (int j = 0; j < kFoldItems; ++j) avg[j] = make_double2(0.0, 0.0);
    for (int i0 = 0; i0 < n_child; i0 += kFoldStage) {
      const int nst = min(kFoldStage, n_child - i0);
      __syncthreads();
      for (int e = threadIdx.x; e < nst * L; e += blockDim.x) {
        const int i = e / L, x = e - i * L;
        rowbuf[e] = mlbuf[m.ell + ((size_t)(sample_base + i0 + i) * ns_child + cs) * d.L3 + (size_t)row * L + x];
      }
      __syncthreads();
      for (int i = 0; i < nst; ++i) {
        const double2* e = rowbuf + i * L;
#pragma unroll
        for (int j = 0; j < kFoldItems; ++j) {
          if ((int)threadIdx.x + j * (int)blockDim.x < nitems) {
            const double2 u = e[x0[j]], v = e[xr[j]];
            avg[j].x += u.x * v.x + u.y * v.y;
            avg[j].y += u.x * v.y - u.y * v.x;
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kFoldItems; ++j) prod[j] = cmul(prod[j], make_double2(avg[j].x * inv, avg[j].y * inv));
  }
#pragma unroll
  for (int j = 0; j < kFoldItems; ++j) {
    const int item = (int)threadIdx.x + j * (int)blockDim.x;
    if (item < nitems) {
      const int k = item / L;
      double2* pp = accbuf + m.acc[parent_level] + ((size_t)S * d.L3 + (size_t)row * L + x0[j]) * m.nR + k;
      pp->x += prod[j].x;
      pp->y += prod[j].y;
    }
  }
}

__global__ void zero_kernel(double2* __restrict__ p, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(0.0, 0.0);
}

// out[(lat * max_r + k) * 2 + {0,1}] = L^-3 sum_x0 acc_top[x0][k]
__global__ void ml_final_kernel(const LatDesc* __restrict__ lats, const MLDesc* __restrict__ mls, int max_r,
                                int top_level, const double2* __restrict__ accbuf, double* __restrict__ out) {
  __shared__ double sh[16];
  const int lat = blockIdx.x, k = blockIdx.y;
  const LatDesc d = lats[lat];
  const MLDesc m = mls[lat];
  if (k >= m.nR) return;  // uniform per block
  double re = 0.0, im = 0.0;
  const double2* a = accbuf + m.acc[top_level];
  for (int x0 = threadIdx.x; x0 < d.L3; x0 += blockDim.x) {
    const double2 v = a[(size_t)x0 * m.nR + k];
    re += v.x;
    im += v.y;
  }
  re = block_sum(re, sh);
  im = block_sum(im, sh);
  if (threadIdx.x == 0) {
    out[((size_t)lat * max_r + k) * 2] = re / (double)d.L3;
    out[((size_t)lat * max_r + k) * 2 + 1] = im / (double)d.L3;
  }
}

// ---------------------------------------------------------------------------
// field insertion: every inner sample keeps its time-line sums (ell) and its
// slab sums of the field operators; after the run they are contracted with
// the final weights, as a correlation over the mediator plane evaluated by 2D
// discrete Fourier transforms in (y, z).
// ---------------------------------------------------------------------------
// sin of the plaquette angle: FP64 links in FP64; FP32 links (the fast path)
// in FP32 arithmetic with the hardware sine, summed by the caller in FP64
__device__ __forceinline__ double plaq_sin(const double* links, const LatDesc& d, Site s, int mu, int nu) {
  return sin(plaq_angle(links, d, s, mu, nu));
}
__device__ __forceinline__ double plaq_sin(const float* links, const LatDesc& d, Site s, int mu, int nu) {
  const float a = links[link_at(d, mu, s)];
  const float b = links[link_at(d, nu, shift2(d, s, mu, 1, nu, 0))];
  const float c = links[link_at(d, mu, shift2(d, s, nu, 1, mu, 0))];
  const float e = links[link_at(d, nu, s)];
  return (double)__sinf(((a + b) - c) - e);
}

// oall[((sample * 6 + c) * ns + s) * L3 + y] = sum over the times t of inner
// slab s of O_c(y, t), O_c = sqrt(beta) Im P_munu (Eq. (5)).
template <typename R>
__global__ void field_o_kernel(const R* __restrict__ links, const LatDesc* __restrict__ lats,
                               const FieldLat* __restrict__ fls, const int2* __restrict__ blocks, int th_inner,
                               int sample, double* __restrict__ fbuf) {
  const int2 bk = blocks[blockIdx.x];
  const LatDesc d = lats[bk.x];
  const FieldLat fl = fls[bk.x];
  const int item = bk.y + (int)threadIdx.x;
  if (item >= fl.ns * d.L3) return;
  const int s = item / d.L3, y3 = item - s * d.L3;
  Site st;
  st.x = y3 % d.L;
  st.y = (y3 / d.L) % d.L;
  st.z = y3 / (d.L * d.L);
  double o[6] = {0, 0, 0, 0, 0, 0};
  for (int t = s * th_inner; t < (s + 1) * th_inner; ++t) {
    st.t = t;
    o[0] += plaq_sin(links, d, st, 0, 1);
    o[1] += plaq_sin(links, d, st, 0, 2);
    o[2] += plaq_sin(links, d, st, 0, 3);
    o[3] += plaq_sin(links, d, st, 2, 3);
    o[4] -= plaq_sin(links, d, st, 1, 3);
    o[5] += plaq_sin(links, d, st, 1, 2);
  }
  double* out = fbuf + fl.oall + (size_t)sample * 6 * fl.ns * d.L3;
  for (int c = 0; c < 6; ++c) out[((size_t)c * fl.ns + s) * d.L3 + y3] = d.sqrt_beta * o[c];
}

// tavg[((m * ns + s) * L3 + x0) * n_rf + f] = average over the n_inner samples
// of outer iteration m of T(x0, rf[f]) in inner slab s
__global__ void field_tavg_kernel(const LatDesc* __restrict__ lat, const MLDesc* __restrict__ mlp,
                                  const FieldLat* __restrict__ flp, FieldParams fp,
                                  const double2* __restrict__ mlbuf, double* __restrict__ fbuf) {
  const LatDesc d = *lat;
  const MLDesc ml = *mlp;
  const FieldLat fl = *flp;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= fp.n_outer * fl.ns * d.L3 * fp.n_rf) return;
  const int f = item % fp.n_rf;
  const int x0 = (item / fp.n_rf) % d.L3;
  const int s = (item / (fp.n_rf * d.L3)) % fl.ns;
  const int m = item / (fp.n_rf * d.L3 * fl.ns);
  const double2* ell = mlbuf + ml.ell + (size_t)m * fp.n_inner * fl.ns * d.L3;
  ((double2*)(fbuf + fl.tavg))[item] = inner_avg(ell, fp.n_inner, fl.ns, d.L3, s, x0, shift_x(d, x0, fp.rf[f]));
}

// weight of an insertion in inner slab s during outer iteration m:
//   one level:  prod_{s' != s} [T]_{s'} / (n V)
//   two levels: prod_{j != k} A_j * prod_{s' in k, s' != s} [T]_{s',m} / (n_0 n_1 V)
// with k the top slab holding s and A_j the top-level averages.
__global__ void field_weights_kernel(const LatDesc* __restrict__ lat, const MLDesc* __restrict__ mlp,
                                     const FieldLat* __restrict__ flp, FieldParams fp,
                                     const double2* __restrict__ accbuf, double* __restrict__ fbuf) {
  const LatDesc d = *lat;
  const MLDesc ml = *mlp;
  const FieldLat fl = *flp;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= fp.n_outer * fl.ns * d.L3 * fp.n_rf) return;
  const int f = item % fp.n_rf;
  const int x0 = (item / fp.n_rf) % d.L3;
  const int s = (item / (fp.n_rf * d.L3)) % fl.ns;
  const int m = item / (fp.n_rf * d.L3 * fl.ns);
  const int children = fp.n_levels == 2 ? fl.ns / ml.ns[0] : fl.ns;
  const int k = s / children;
  const double2* tavg = (const double2*)(fbuf + fl.tavg);
  double2 p = make_double2(1.0, 0.0);
  for (int j = 0; j < children; ++j) {
    const int sp = k * children + j;
    if (sp == s) continue;
    p = cmul(p, tavg[(((size_t)m * fl.ns + sp) * d.L3 + x0) * fp.n_rf + f]);
  }
  double norm = (double)fp.n_inner * (double)d.V2 * 2.0;
  if (fp.n_levels == 2) {
    const int ntop = ml.ns[0];
    const double inv = 1.0 / (double)fp.n_outer;
    for (int j = 0; j < ntop; ++j) {
      if (j == k) continue;
      const double2 a = accbuf[ml.acc[0] + ((size_t)j * d.L3 + x0) * ml.nR + fp.rf_k[f]];
      p = cmul(p, make_double2(a.x * inv, a.y * inv));
    }
    norm *= (double)fp.n_outer;
  }
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

template <int KIND>
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
    const double* src = fbuf + fl.oall + (((size_t)sample * 6 + a) * ns + s) * d.L3;
    for (int i = threadIdx.x; i < L2; i += blockDim.x) {
      const int y = i / L, z = i - y * L;
      buf[i] = make_double2(src[(size_t)(z * L + y) * L + x], 0.0);
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
      buf[i] = cmul(w[(((size_t)m * ns + s) * d.L3 + x0) * fp.n_rf + a], t);
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

inline int blocks_for(uint64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_plaq_field(int prec, const void* links, const LatDesc* lats, BlockTable bt, double* partial,
                             hipStream_t st) {
  if (prec == kFP64)
    hipLaunchKernelGGL(plaq_field_kernel<double>, dim3(bt.n_blocks), dim3(bt.block), 0, st,
                       (const double*)links, lats, bt.dev, partial);
  else
    hipLaunchKernelGGL(plaq_field_kernel<float>, dim3(bt.n_blocks), dim3(bt.block), 0, st, (const float*)links,
                       lats, bt.dev, partial);
  return hipGetLastError();
}

hipError_t launch_reduce_rows(const double* partial, int width, const int* lat_row_begin, int n_lats, double* out,
                              hipStream_t st) {
  hipLaunchKernelGGL(reduce_rows_kernel, dim3(n_lats, width), dim3(kRedBlock), 0, st, partial, width,
                     lat_row_begin, out);
  return hipGetLastError();
}

hipError_t launch_poly_lines(int prec, const void* links, const LatDesc* lats, BlockTable bt,
                             const uint64_t* poly_off, double* poly, hipStream_t st) {
  if (prec == kFP64)
    hipLaunchKernelGGL(poly_lines_kernel<double>, dim3(bt.n_blocks), dim3(bt.block), 0, st,
                       (const double*)links, lats, bt.dev, poly_off, poly);
  else
    hipLaunchKernelGGL(poly_lines_kernel<float>, dim3(bt.n_blocks), dim3(bt.block), 0, st, (const float*)links,
                       lats, bt.dev, poly_off, poly);
  return hipGetLastError();
}

hipError_t launch_poly_corr(const LatDesc* lats, BlockTable bt, const uint64_t* poly_off, const double* poly,
                            const int* rvals, int nR, const int* row_begin, double* rows, hipStream_t st) {
  hipLaunchKernelGGL(poly_corr_kernel, dim3(bt.n_blocks), dim3(bt.block), 0, st, lats, bt.dev, poly_off, poly,
                     rvals, nR, row_begin, rows);
  return hipGetLastError();
}

hipError_t launch_ml_lines(int prec, const void* links, const LatDesc* lats, const MLDesc* mls, BlockTable bt,
                           int inner_th, int sample, double2* mlbuf, hipStream_t st) {
  if (prec == kFP64)
    hipLaunchKernelGGL(ml_lines_kernel<double>, dim3(bt.n_blocks), dim3(bt.block), 0, st, (const double*)links,
                       lats, mls, bt.dev, inner_th, sample, mlbuf);
  else
    hipLaunchKernelGGL(ml_lines_kernel<float>, dim3(bt.n_blocks), dim3(bt.block), 0, st, (const float*)links,
                       lats, mls, bt.dev, inner_th, sample, mlbuf);
  return hipGetLastError();
}

hipError_t launch_ml_fold(const LatDesc* lats, const MLDesc* mls, BlockTable bt, int child_level, int parent_level,
                          int n_levels, int child_is_inner, int n_child, int sample_base, const int* rvals,
                          const double2* mlbuf, double2* accbuf, hipStream_t st) {
  hipLaunchKernelGGL(ml_fold_kernel, dim3(bt.n_blocks), dim3(bt.block), 0, st, lats, mls, bt.dev, child_level,
                     parent_level, n_levels, child_is_inner, n_child, sample_base, rvals, mlbuf, accbuf);
  return hipGetLastError();
}

hipError_t launch_ml_fold_rows(const LatDesc* lats, const MLDesc* mls, BlockTable bt, int threads, int max_L,
                               int child_level, int parent_level, int n_levels, int n_child, int sample_base,
                               const int* rvals, const double2* mlbuf, double2* accbuf, hipStream_t st) {
  if (bt.n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(ml_fold_rows_kernel, dim3(bt.n_blocks), dim3(threads),
                     (size_t)kFoldStage * max_L * sizeof(double2), st, lats, mls, bt.dev, child_level, parent_level,
                     n_levels, n_child, sample_base, rvals, mlbuf, accbuf);
  return hipGetLastError();
}

int ml_fold_rows_max_items() { return kFoldItems * 1024; }

hipError_t launch_ml_zero(double2* accbuf, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, accbuf, n);
  return hipGetLastError();
}

hipError_t launch_ml_final(const LatDesc* lats, const MLDesc* mls, int n_lats, int max_r, int top_level,
                           const double2* accbuf, double* out, hipStream_t st) {
  hipLaunchKernelGGL(ml_final_kernel, dim3(n_lats, max_r), dim3(kRedBlock), 0, st, lats, mls, max_r, top_level,
                     accbuf, out);
  return hipGetLastError();
}

hipError_t launch_field_o(int prec, const void* links, const LatDesc* lats, const FieldLat* fls, BlockTable bt,
                          int th_inner, int sample, double* fbuf, hipStream_t st) {
  if (bt.n_blocks == 0) return hipSuccess;
  if (prec == kFP64)
    hipLaunchKernelGGL(field_o_kernel<double>, dim3(bt.n_blocks), dim3(bt.block), 0, st, (const double*)links, lats,
                       fls, bt.dev, th_inner, sample, fbuf);
  else
    hipLaunchKernelGGL(field_o_kernel<float>, dim3(bt.n_blocks), dim3(bt.block), 0, st, (const float*)links, lats,
                       fls, bt.dev, th_inner, sample, fbuf);
  return hipGetLastError();
}

hipError_t launch_field_contract(const LatDesc* lat, const MLDesc* ml, const FieldLat* fl, const FieldLat& hfl,
                                 FieldParams fp, int L, const double2* mlbuf, const double2* accbuf, double* fbuf,
                                 double2* scratch, size_t scratch_elems, double2* F, hipStream_t st) {
  const uint64_t L3 = (uint64_t)L * L * L, L2 = (uint64_t)L * L;
  const int ns = hfl.ns;
  const uint64_t nt = (uint64_t)fp.n_outer * ns * L3 * fp.n_rf;
  hipLaunchKernelGGL(field_tavg_kernel, dim3(blocks_for(nt, 256)), dim3(256), 0, st, lat, ml, fl, fp, mlbuf, fbuf);
  hipLaunchKernelGGL(field_weights_kernel, dim3(blocks_for(nt, 256)), dim3(256), 0, st, lat, ml, fl, fp, accbuf,
                     fbuf);
  double2* G = (double2*)(fbuf + hfl.g);
  const uint64_t ng = (uint64_t)fp.n_rf * 12 * L2;
  hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(ng, 256)), dim3(256), 0, st, G, ng);
  // scratch per chunk: What [nk][n_rf][ns][L3], Ohat [nk][6][ns][L3], part [nk][n_rf][ns][12][L2]
  const uint64_t per_sample = (uint64_t)(fp.n_rf + 6) * ns * L3 + (uint64_t)fp.n_rf * ns * 12 * L2;
  const int chunk = (int)std::max<uint64_t>(1, std::min<uint64_t>(64, scratch_elems / per_sample));
  const int n_samples = fp.n_outer * fp.n_inner;
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
    hipLaunchKernelGGL(field_dft_kernel<1>, dim3((unsigned)((uint64_t)nk * fp.n_rf * ns * L)), dim3(kDftThreads), shm,
                       st, lat, ml, fl, fp, s0, mlbuf, fbuf, what);
    hipLaunchKernelGGL(field_dft_kernel<0>, dim3((unsigned)((uint64_t)nk * 6 * ns * L)), dim3(kDftThreads), shm, st,
                       lat, ml, fl, fp, s0, mlbuf, fbuf, ohat);
    hipLaunchKernelGGL(field_gacc_kernel, dim3((unsigned)((L2 + pt - 1) / pt), ns, nk), dim3(gthreads), gshm, st, fp, L,
                       ns, pt, what, ohat, part);
    hipLaunchKernelGGL(field_gred_kernel, dim3(blocks_for(ng, 64)), dim3(64), 0, st, fp, L, ns, nk, part, G);
  }
  hipLaunchKernelGGL(field_final_kernel, dim3(blocks_for(ng, 64)), dim3(64), 0, st, fp, L, G, F);
  return hipGetLastError();
}

}  // namespace u1ml
