// measure.hip -- observables and multilevel estimators, FP64 accumulation.
//
//  * plaquette (Eq. (3) normalised per plaquette) and the six field operators
//    a^2 F_munu = sqrt(beta) Im P_munu (Eq. (5)): E_i from P_0i, B_i from P_jk;
//  * Polyakov loop P(x) = exp(i sum_t theta_0(x, t)) and the plain correlator
//    C(r) = L^-3 sum_x P*(x) P(x + r e_x);
//  * multilevel (Sec. 2.2): time-line angle sums of the innermost slabs per
//    sample, slab averages of the two-link products T(x0, r) of Eq. (8) and
//    their nested products, and the field insertion of Eq. (9) evaluated by
//    replaying the update sequence with precomputed weights.
// All sums are FP64 with a fixed reduction order (results do not depend on
// timing).  Links are read as FP64 or FP32 angles.
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
                                int sample, double* __restrict__ mlbuf) {
  const int2 bk = blocks[blockIdx.x];
  const LatDesc d = lats[bk.x];
  const int ns = d.T / inner_th;
  const int item = bk.y + (int)threadIdx.x;
  if (item >= ns * d.L3) return;
  const int s = item / d.L3, x3 = item - s * d.L3;
  mlbuf[mls[bk.x].ell + ((size_t)sample * ns + s) * d.L3 + x3] = time_line(links, d, x3, s * inner_th, inner_th);
}

// average over the stored samples of T(x0, r) = exp(i (l(x0 + r) - l(x0))) of inner slab cs
__device__ __forceinline__ double2 inner_avg(const double* ell, int n_samples, int ns, int L3, int cs, int x0,
                                             int x0r) {
  double2 a = make_double2(0.0, 0.0);
  for (int i = 0; i < n_samples; ++i) {
    const double* e = ell + ((size_t)i * ns + cs) * L3;
    const double2 t = cexpi(e[x0r] - e[x0]);
    a.x += t.x;
    a.y += t.y;
  }
  const double inv = 1.0 / (double)n_samples;
  return make_double2(a.x * inv, a.y * inv);
}

// acc_parent[S][x0][k] += prod over the children of S of the child averages.
// parent_level == n_levels denotes the top (one slab spanning all of T).
__global__ void ml_fold_kernel(const LatDesc* __restrict__ lats, const MLDesc* __restrict__ mls,
                               const int2* __restrict__ blocks, int child_level, int parent_level, int n_levels,
                               int child_is_inner, int n_child, const int* __restrict__ rvals,
                               const double* __restrict__ mlbuf, double2* __restrict__ accbuf) {
  const int2 bk = blocks[blockIdx.x];
  const LatDesc d = lats[bk.x];
  const MLDesc m = mls[bk.x];
  const int ns_child = m.ns[child_level];
  const int ns_parent = parent_level == n_levels ? 1 : m.ns[parent_level];
  const int children = ns_child / ns_parent;
  const int item = bk.y + (int)threadIdx.x;
  if (item >= ns_parent * d.L3 * m.nR) return;
  const int k = item % m.nR;
  const int x0 = (item / m.nR) % d.L3;
  const int S = item / (m.nR * d.L3);
  const int x0r = shift_x(d, x0, rvals[m.r_off + k]);
  double2 prod = make_double2(1.0, 0.0);
  const double inv = 1.0 / (double)n_child;
  for (int j = 0; j < children; ++j) {
    const int cs = S * children + j;
    double2 avg;
    if (child_is_inner) {
      avg = inner_avg(mlbuf + m.ell, n_child, ns_child, d.L3, cs, x0, x0r);
    } else {
      double2* c = accbuf + m.acc[child_level] + ((size_t)cs * d.L3 + x0) * m.nR + k;
      avg = make_double2(c->x * inv, c->y * inv);
      *c = make_double2(0.0, 0.0);
    }
    prod = cmul(prod, avg);
  }
  double2* p = accbuf + m.acc[parent_level] + ((size_t)S * d.L3 + x0) * m.nR + k;
  p->x += prod.x;
  p->y += prod.y;
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
// field insertion (single lattice)
// ---------------------------------------------------------------------------
// tavg[((m * ns + s) * L3 + x0) * n_rf + f] = inner average of T at separation rf[f]
__global__ void field_store_tavg_kernel(const LatDesc* __restrict__ lat, const MLDesc* __restrict__ mlp,
                                        FieldDesc fd, int m, const double* __restrict__ mlbuf,
                                        double2* __restrict__ tavg) {
  const LatDesc d = *lat;
  const MLDesc ml = *mlp;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= fd.ns_inner * d.L3 * fd.n_rf) return;
  const int f = item % fd.n_rf;
  const int x0 = (item / fd.n_rf) % d.L3;
  const int s = item / (fd.n_rf * d.L3);
  const int x0r = shift_x(d, x0, fd.rf[f]);
  tavg[(((size_t)m * fd.ns_inner + s) * d.L3 + x0) * fd.n_rf + f] =
      inner_avg(mlbuf + ml.ell, fd.n_inner, fd.ns_inner, d.L3, s, x0, x0r);
}

// weight of an insertion in inner slab s during outer iteration m:
//   one level:  prod_{s' != s} [T]_{s'} / (n V)
//   two levels: prod_{j != k} A_j * prod_{s' in k, s' != s} [T]_{s',m} / (n_0 n_1 V)
// with k the top slab holding s and A_j the top-level averages.
__global__ void field_weights_kernel(const LatDesc* __restrict__ lat, const MLDesc* __restrict__ mlp, FieldDesc fd,
                                     const double2* __restrict__ tavg, const double2* __restrict__ accbuf,
                                     double2* __restrict__ w) {
  const LatDesc d = *lat;
  const MLDesc ml = *mlp;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= fd.n_outer * fd.ns_inner * d.L3 * fd.n_rf) return;
  const int f = item % fd.n_rf;
  const int x0 = (item / fd.n_rf) % d.L3;
  const int s = (item / (fd.n_rf * d.L3)) % fd.ns_inner;
  const int m = item / (fd.n_rf * d.L3 * fd.ns_inner);
  const int k = s / fd.children;
  double2 p = make_double2(1.0, 0.0);
  for (int j = 0; j < fd.children; ++j) {
    const int sp = k * fd.children + j;
    if (sp == s) continue;
    p = cmul(p, tavg[(((size_t)m * fd.ns_inner + sp) * d.L3 + x0) * fd.n_rf + f]);
  }
  double norm = (double)fd.n_inner * (double)d.V2 * 2.0;
  if (fd.n_levels == 2) {
    const int ntop = ml.ns[0];
    const double inv = 1.0 / (double)fd.n_outer;
    for (int j = 0; j < ntop; ++j) {
      if (j == k) continue;
      const double2 a = accbuf[ml.acc[0] + ((size_t)j * d.L3 + x0) * ml.nR + fd.rf_k[f]];
      p = cmul(p, make_double2(a.x * inv, a.y * inv));
    }
    norm *= (double)fd.n_outer;
  }
  w[(((size_t)m * fd.ns_inner + s) * d.L3 + x0) * fd.n_rf + f] = make_double2(p.x / norm, p.y / norm);
}

// oslab[(c * ns + s) * L3 + y] = sum over the times t of inner slab s of O_c(y, t)
template <typename R>
__global__ void field_oslab_kernel(const R* __restrict__ links, const LatDesc* __restrict__ lat, FieldDesc fd,
                                   double* __restrict__ oslab) {
  const LatDesc d = *lat;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= fd.ns_inner * d.L3) return;
  const int s = item / d.L3, y3 = item - s * d.L3;
  Site st;
  st.x = y3 % d.L;
  st.y = (y3 / d.L) % d.L;
  st.z = y3 / (d.L * d.L);
  double o[6] = {0, 0, 0, 0, 0, 0};
  for (int t = s * fd.th_inner; t < (s + 1) * fd.th_inner; ++t) {
    st.t = t;
    o[0] += sin(plaq_angle(links, d, st, 0, 1));
    o[1] += sin(plaq_angle(links, d, st, 0, 2));
    o[2] += sin(plaq_angle(links, d, st, 0, 3));
    o[3] += sin(plaq_angle(links, d, st, 2, 3));
    o[4] -= sin(plaq_angle(links, d, st, 1, 3));
    o[5] += sin(plaq_angle(links, d, st, 1, 2));
  }
  for (int c = 0; c < 6; ++c) oslab[((size_t)c * fd.ns_inner + s) * d.L3 + y3] = d.sqrt_beta * o[c];
}

// wslab[(f * ns + s) * L3 + x0] = w[m][s][x0][f] * T_i(x0, s; rf[f]) for the current sample
__global__ void field_wslab_kernel(const LatDesc* __restrict__ lat, const MLDesc* __restrict__ mlp, FieldDesc fd,
                                   int m, int sample, const double* __restrict__ mlbuf,
                                   const double2* __restrict__ w, double2* __restrict__ wslab) {
  const LatDesc d = *lat;
  const MLDesc ml = *mlp;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= fd.n_rf * fd.ns_inner * d.L3) return;
  const int x0 = item % d.L3;
  const int s = (item / d.L3) % fd.ns_inner;
  const int f = item / (d.L3 * fd.ns_inner);
  const double* e = mlbuf + ml.ell + ((size_t)sample * fd.ns_inner + s) * d.L3;
  const double2 t = cexpi(e[shift_x(d, x0, fd.rf[f])] - e[x0]);
  const double2 ww = w[(((size_t)m * fd.ns_inner + s) * d.L3 + x0) * fd.n_rf + f];
  wslab[item] = cmul(ww, t);
}

// fout[(((f * 2 + plane) * 6 + c) * L + dy) * L + dz] +=
//   sum_s sum_x0 wslab[f][s][x0] * oslab[c][s][x0 + (m_plane, dy, dz)]
__global__ void field_contract_kernel(const LatDesc* __restrict__ lat, FieldDesc fd,
                                      const double* __restrict__ oslab, const double2* __restrict__ wslab,
                                      double2* __restrict__ fout) {
  const LatDesc d = *lat;
  const int L = d.L, L2 = L * L;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= fd.n_rf * 2 * 6 * L2) return;
  const int dz = item % L, dy = (item / L) % L;
  const int c = (item / L2) % 6;
  const int plane = (item / (6 * L2)) % 2;
  const int f = item / (12 * L2);
  const int r = fd.rf[f];
  const int mx = plane == 0 ? (r - 1) / 2 : r / 2;
  double re = 0.0, im = 0.0;
  for (int s = 0; s < fd.ns_inner; ++s) {
    const double2* W = wslab + ((size_t)f * fd.ns_inner + s) * d.L3;
    const double* O = oslab + ((size_t)c * fd.ns_inner + s) * d.L3;
    for (int z = 0; z < L; ++z) {
      const int zz = (z + dz) % L;
      for (int y = 0; y < L; ++y) {
        const int yy = (y + dy) % L;
        const double2* Wr = W + (z * L + y) * L;
        const double* Or = O + (zz * L + yy) * L;
        for (int x = 0; x < L; ++x) {
          const int xx = (x + mx) % L;
          const double o = Or[xx];
          re += Wr[x].x * o;
          im += Wr[x].y * o;
        }
      }
    }
  }
  fout[item].x += re;
  fout[item].y += im;
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
                           int inner_th, int sample, double* mlbuf, hipStream_t st) {
  if (prec == kFP64)
    hipLaunchKernelGGL(ml_lines_kernel<double>, dim3(bt.n_blocks), dim3(bt.block), 0, st, (const double*)links,
                       lats, mls, bt.dev, inner_th, sample, mlbuf);
  else
    hipLaunchKernelGGL(ml_lines_kernel<float>, dim3(bt.n_blocks), dim3(bt.block), 0, st, (const float*)links,
                       lats, mls, bt.dev, inner_th, sample, mlbuf);
  return hipGetLastError();
}

hipError_t launch_ml_fold(const LatDesc* lats, const MLDesc* mls, BlockTable bt, int child_level, int parent_level,
                          int n_levels, int child_is_inner, int n_child, const int* rvals, const double* mlbuf,
                          double2* accbuf, hipStream_t st) {
  hipLaunchKernelGGL(ml_fold_kernel, dim3(bt.n_blocks), dim3(bt.block), 0, st, lats, mls, bt.dev, child_level,
                     parent_level, n_levels, child_is_inner, n_child, rvals, mlbuf, accbuf);
  return hipGetLastError();
}

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

hipError_t launch_field_store_tavg(const LatDesc* lat, const MLDesc* ml, FieldDesc fd, int L3, int m,
                                   const double* mlbuf, double2* tavg, hipStream_t st) {
  const uint64_t n = (uint64_t)fd.ns_inner * L3 * fd.n_rf;
  hipLaunchKernelGGL(field_store_tavg_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, lat, ml, fd, m, mlbuf,
                     tavg);
  return hipGetLastError();
}

hipError_t launch_field_weights(const LatDesc* lat, const MLDesc* ml, FieldDesc fd, int L3, const double2* tavg,
                                const double2* accbuf, double2* w, hipStream_t st) {
  const uint64_t n = (uint64_t)fd.n_outer * fd.ns_inner * L3 * fd.n_rf;
  hipLaunchKernelGGL(field_weights_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, lat, ml, fd, tavg, accbuf,
                     w);
  return hipGetLastError();
}

hipError_t launch_field_sample(int prec, const void* links, const LatDesc* lat, const MLDesc* ml, FieldDesc fd,
                               int L, int m, int sample, const double* mlbuf, const double2* w, double* oslab,
                               double2* wslab, double2* fout, hipStream_t st) {
  const uint64_t L3 = (uint64_t)L * L * L;
  const uint64_t no = (uint64_t)fd.ns_inner * L3;
  if (prec == kFP64)
    hipLaunchKernelGGL(field_oslab_kernel<double>, dim3(blocks_for(no, 256)), dim3(256), 0, st,
                       (const double*)links, lat, fd, oslab);
  else
    hipLaunchKernelGGL(field_oslab_kernel<float>, dim3(blocks_for(no, 256)), dim3(256), 0, st,
                       (const float*)links, lat, fd, oslab);
  const uint64_t nw = (uint64_t)fd.n_rf * no;
  hipLaunchKernelGGL(field_wslab_kernel, dim3(blocks_for(nw, 256)), dim3(256), 0, st, lat, ml, fd, m, sample,
                     mlbuf, w, wslab);
  const uint64_t nf = (uint64_t)fd.n_rf * 12 * L * L;
  hipLaunchKernelGGL(field_contract_kernel, dim3(blocks_for(nf, 64)), dim3(64), 0, st, lat, fd, oslab, wslab,
                     fout);
  return hipGetLastError();
}

}  // namespace u1ml
