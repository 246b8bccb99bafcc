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

#include "measure_common.h"

namespace u1ml {

namespace {

// ---------------------------------------------------------------------------
// plain observables
// ---------------------------------------------------------------------------
// Per block: the plaquette sum, the six field operators of Eq. (5) and the
// six squared components of Eq. (6), summed over the block's sites.
template <typename R>
__global__ __launch_bounds__(256) void plaq_field_kernel(const R* __restrict__ links, const LatDesc* __restrict__ lats,
                                  const int2* __restrict__ blocks, double* __restrict__ partial) {
  __shared__ double sh[16];
  // neighbouring sites (which read each other's links) on one XCD; the
  // partial row is that of the logical block
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int2 bk = blocks[lb];
  const LatDesc d = lats[bk.x];
  const uint32_t n = (uint32_t)bk.y + threadIdx.x;
  double v[kPlaqFieldWidth];
  for (int j = 0; j < kPlaqFieldWidth; ++j) v[j] = 0.0;
  if (n < 2u * (uint32_t)d.V2) {
    const Site s = as_site(coords_natural(d, n));
    // component order E_x, E_y, E_z, B_x, B_y, B_z from P_01, P_02, P_03,
    // P_23, P_31 = conj(P_13), P_12
    const double p[6] = {plaq_angle(links, d, s, 0, 1), plaq_angle(links, d, s, 0, 2),
                         plaq_angle(links, d, s, 0, 3), plaq_angle(links, d, s, 2, 3),
                         -plaq_angle(links, d, s, 1, 3), plaq_angle(links, d, s, 1, 2)};
    v[0] = ((((cos(p[0]) + cos(p[1])) + cos(p[2])) + cos(p[5])) + cos(p[4])) + cos(p[3]);
    const double sb = d.sqrt_beta;
    for (int c = 0; c < 6; ++c) {
      v[1 + c] = sb * sin(p[c]);
      const double h = sin(0.5 * p[c]);
      v[7 + c] = 2.0 * d.beta * (h * h);
    }
  }
  for (int j = 0; j < kPlaqFieldWidth; ++j) {
    const double r = block_sum(v[j], sh);
    if (threadIdx.x == 0) partial[(size_t)lb * kPlaqFieldWidth + j] = r;
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
// I_1(x) / I_0(x), x >= 0: power series of both functions with the common
// terms a_k = (x^2/4)^k / (k!)^2 (I_0 = sum a_k, I_1 = x/2 sum a_k / (k + 1));
// beyond x = 600 the large-x expansion to order x^-4.  The factors 1/k^2 and
// 1/(k+1) of the first kBesselTab terms come from a table (no division).
constexpr int kBesselTab = 64;
struct BesselTab {
  double inv_k2[kBesselTab], inv_k1[kBesselTab];
  constexpr BesselTab() : inv_k2(), inv_k1() {
    for (int k = 1; k < kBesselTab; ++k) {
      inv_k2[k] = 1.0 / ((double)k * (double)k);
      inv_k1[k] = 1.0 / (double)(k + 1);
    }
  }
};
__device__ constexpr BesselTab kBessel{};

__device__ __forceinline__ double bessel_i1_over_i0(double x) {
  if (x <= 0.0) return 0.0;
  if (x > 600.0) {
    const double u = 1.0 / x;
    return 1.0 - u * (0.5 + u * (0.125 + u * (0.125 + u * (25.0 / 128.0))));
  }
  const double q = 0.25 * x * x;
  double a = 1.0, s0 = 1.0, s1 = 1.0;
  int k = 1;
  for (; k < kBesselTab; ++k) {
    a *= q * kBessel.inv_k2[k];
    s0 += a;
    s1 += a * kBessel.inv_k1[k];
    if (a < 1e-18 * s0) return 0.5 * x * s1 / s0;
  }
  for (; k < 2000; ++k) {
    a *= q / ((double)k * (double)k);
    s0 += a;
    s1 += a / (double)(k + 1);
    if (a < 1e-18 * s0) break;
  }
  return 0.5 * x * s1 / s0;
}

// staple of the temporal link at s (Eq. (3)): S = sum over nu = 1..3 of the
// forward phase theta_nu(x + 0) - theta_0(x + nu) - theta_nu(x) and the
// backward phase -(theta_0(x - nu) + theta_nu(x + 0 - nu) - theta_nu(x - nu)),
// in the arithmetic of the links (FP64 with library sincos; FP32 with the
// hardware sine and cosine, the staple arithmetic of the FP32 path)
template <typename R>
__device__ __forceinline__ void temporal_staple(const R* links, const LatDesc& d, Site s, double& sr_out,
                                                double& si_out) {
  R sr = (R)0, si = (R)0;
  for (int nu = 1; nu < 4; ++nu) {
    const Site b = shift2(d, s, nu, -1, 0, 0);
    const R ap = (links[link_at(d, nu, shift2(d, s, 0, 1, nu, 0))] - links[link_at(d, 0, shift2(d, s, nu, 1, 0, 0))]) -
                 links[link_at(d, nu, s)];
    const R am = -((links[link_at(d, 0, b)] + links[link_at(d, nu, shift2(d, s, 0, 1, nu, -1))]) -
                   links[link_at(d, nu, b)]);
    R sn, cs;
    if constexpr (sizeof(R) == 4) {
      __sincosf(ap, &sn, &cs);
      sr += cs;
      si += sn;
      __sincosf(am, &sn, &cs);
    } else {
      sincos(ap, &sn, &cs);
      sr += cs;
      si += sn;
      sincos(am, &sn, &cs);
    }
    sr += cs;
    si += sn;
  }
  sr_out = (double)sr;
  si_out = (double)si;
}

// multihit mean of the temporal link at s: with the staple S the link's
// conditional density is exp(beta |S| cos(theta + arg S)) / norm, and the mean
// of exp(i theta) is conj(S) / |S| * I_1(beta |S|) / I_0(beta |S|)
template <typename R>
__device__ __forceinline__ double2 multihit_mean(const R* links, const LatDesc& d, Site s) {
  double sr, si;
  temporal_staple(links, d, s, sr, si);
  const double a = hypot(sr, si);
  if (a == 0.0) return make_double2(0.0, 0.0);
  const double q = bessel_i1_over_i0(d.beta * a) / a;
  return make_double2(q * sr, -q * si);
}

// One inner sample of every lattice, a thread per (inner slab s, spatial
// site x3): the slab's time line exp(i sum_t theta_0) (Eq. (8)), with
// multihit also the product of the temporal links' multihit means, and with
// FIELD the slab sums over t of the insertion operators O_c(x3, t) (Eq. (5),
// or Eq. (6) with SQ), stored in the link precision (FP32 lattices' sums
// carry FP32 sine errors):
//   oall[((sample * 6 + c) * ns + s) * L3 + x3].
// With the field inserted every inner sample is kept; after the run the
// samples are contracted with the final weights as a correlation over the
// mediator plane (field.hip).
template <typename R, bool FIELD, bool SQ>
__global__ void ml_sample_kernel(const R* __restrict__ links, const LatDesc* __restrict__ lats,
                                 const MLDesc* __restrict__ mls, const FieldLat* __restrict__ fls,
                                 const int2* __restrict__ blocks, int inner_th, int sample,
                                 double2* __restrict__ mlbuf, double* __restrict__ fbuf) {
  // neighbouring sites (which read each other's links) on one XCD
  const int2 bk = blocks[xcd_block(blockIdx.x, gridDim.x)];
  const LatDesc d = lats[bk.x];
  const int ns = d.T / inner_th;
  const int item = bk.y + (int)threadIdx.x;
  if (item >= ns * d.L3) return;
  const int s = item / d.L3, x3 = item - s * d.L3;
  const MLDesc* m = mls + bk.x;
  const size_t at = ((size_t)sample * ns + s) * d.L3 + x3;
  Site st;
  st.x = x3 % d.L;
  st.y = (x3 / d.L) % d.L;
  st.z = x3 / (d.L * d.L);
  // exp(i l), l = sum of theta_0 over the slab's times: the slab product of U_0
  double l = 0.0;
  double o[6] = {0, 0, 0, 0, 0, 0};
  if (FIELD) {
    // the slab's six plaquettes per time from sixteen loads per site
    for (int t = s * inner_th; t < (s + 1) * inner_th; ++t) {
      SiteLinks<R> sl;
      load_site_links(links, d, t, st.x, st.y, st.z, sl);
      l += (double)sl.at[0];
      add_field_ops_loaded<SQ>(sl, o);
    }
  } else {
    l = time_line(links, d, x3, s * inner_th, inner_th);
  }
  store_stream(mlbuf + m->ell + at, cexpi(l));
  if (m->multihit) {
    double2 p = make_double2(1.0, 0.0);
    for (int t = s * inner_th; t < (s + 1) * inner_th; ++t) {
      st.t = t;
      p = cmul(p, multihit_mean(links, d, st));
    }
    store_stream(mlbuf + m->ell_mh + at, p);
  }
  if (FIELD) {
    const FieldLat fl = fls[bk.x];
    const double pre = SQ ? d.beta : d.sqrt_beta;
    R* out = (R*)(fbuf + fl.oall) + (size_t)sample * 6 * ns * d.L3;
    for (int c = 0; c < 6; ++c) store_stream(out + ((size_t)c * ns + s) * d.L3 + x3, pre * o[c]);
  }
}

// acc_parent[S][x0][k] += prod over the children of S of the child averages.
// parent_level == n_levels denotes the top (one slab spanning all of T).
// One thread per (S, x0, block of up to kFoldR separations).
constexpr int kFoldR = 8;
__global__ __launch_bounds__(256) void ml_fold_kernel(const LatDesc* __restrict__ lats, const MLDesc* __restrict__ mls,
                               const int2* __restrict__ blocks, int child_level, int parent_level, int n_levels,
                               int child_is_inner, int n_child, int sample_base, const int* __restrict__ rvals,
                               const double2* __restrict__ mlbuf, double2* __restrict__ accbuf) {
  const int2 bk = blocks[xcd_block(blockIdx.x, gridDim.x)];  // neighbouring sites on one XCD
  const LatDesc d = lats[bk.x];
  const MLDesc& m = mls[bk.x];  // through the pointer (run-time level indices)
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
    xr[j] = j < kn ? shift_axis(d, x0, rvals[m.r_off + k0 + j]) : x0;
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
      const double2* emh = mlbuf + m.ell_mh + ((size_t)sample_base * ns_child + cs) * d.L3;
      for (int i = 0; i < n_child; ++i) {
        const double2* e = ell + (size_t)i * ns_child * d.L3;
        const double2* eh = emh + (size_t)i * ns_child * d.L3;
        const double2 u = e[x0];
        const double2 uh = m.multihit ? eh[x0] : u;
#pragma unroll
        for (int j = 0; j < kFoldR; ++j) {
          if (j < kn) {
            // multihit lines for r >= 2 (the two lines share no plaquette)
            const bool mh = m.multihit && (rvals[m.r_off + k0 + j] & 0xffff) >= 2;
            avg[j] = cmac_conj(avg[j], mh ? uh : u, mh ? eh[xr[j]] : e[xr[j]]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < kFoldR; ++j) avg[j] = cscale(avg[j], inv);
    } else {
      double2* cp = accbuf + m.acc[child_level] + ((size_t)cs * d.L3 + x0) * m.nR + k0;
#pragma unroll
      for (int j = 0; j < kFoldR; ++j) {
        if (j < kn) {
          avg[j] = cscale(cp[j], inv);
          cp[j] = make_double2(0.0, 0.0);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kFoldR; ++j) prod[j] = cmul(prod[j], avg[j]);
  }
  double2* pp = accbuf + m.acc[parent_level] + ((size_t)S * d.L3 + x0) * m.nR + k0;
#pragma unroll
  for (int j = 0; j < kFoldR; ++j)
    if (j < kn) pp[j] = cadd(pp[j], prod[j]);
}

// The same fold for innermost children, one block per (parent slab S, axis a,
// row along a), with the rows of the stored samples staged in LDS, so that
// every time line is read from memory once instead of once per separation.  A
// thread owns one position j along the row and K separations of the axis (K =
// 4, 6 or 8, chosen per launch so that the groups of K cover the separations
// with the fewest unused slots), so the line at j is read once per sample for
// all of them; the sample and child order of every sum is that of
// ml_fold_kernel and every step is one of the explicitly rounded complex
// helpers, so both (and both stagings) give the same bits.  MH: the run uses the multihit
// lines (known per launch, so that the plain run reads each line once).  Rows
// along x are contiguous; rows along y and z are strided by L and L^2.
// Staging: all children of S at once (PC false: children * n_child * L
// values, twice with multihit, one __syncthreads), or one child at a time (PC
// true: n_child * L values, two __syncthreads per child, every (j, group)
// item held by its own thread, blockDim >= L * groups), which keeps the LDS
// of a block small where S has many children (a single level: T / t_h).
constexpr size_t kFoldLds = 49152;  // bytes of staged rows per block
// values per thread that the pipelined one-child staging holds in registers
constexpr int fold_prefetch(bool mh) { return mh ? 8 : 4; }
// With tavg_m >= 0 (two-level runs with the field inserted) the x rows also
// store the inner averages of the field separations, tavg[((tavg_m n_rf + f)
// ns + s) L3 + x0] (the inputs of the field weights), so that the field
// contraction need not average the stored samples again.

// One position along the row and its group of K separations.
template <int K, bool MH>
struct FoldItem {
  int x0, k0, kn;
  int xr[K];      // position of x0 + r (periodic)
  bool mh[K];     // read the multihit lines (r >= 2)
  int fslot[K];   // field separation index, or -1
  double2 prod[K];
};

template <int K, bool MH>
__device__ __forceinline__ void fold_item_init(FoldItem<K, MH>& it, int item, int ngroups, int L, int axis, int n_r,
                                               int r_off, const int* __restrict__ rvals, bool tavg_on,
                                               const FieldParams& fp) {
  it.x0 = item / ngroups;
  it.k0 = (item - it.x0 * ngroups) * K;
  it.kn = min(K, n_r - it.k0);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    // separations past the group's last are read clamped and never used
    const int rv = rvals[r_off + axis * n_r + min(it.k0 + j, n_r - 1)];
    const int r = j < it.kn ? rv & 0xffff : 0;
    const int t = it.x0 + r;
    it.xr[j] = t >= L ? t - L : t;
    // multihit lines for r >= 2 (the two lines share no plaquette)
    it.mh[j] = MH && r >= 2;
    it.prod[j] = make_double2(1.0, 0.0);
    it.fslot[j] = -1;
  }
  if (tavg_on) {
    for (int f = 0; f < fp.n_rf; ++f) {
#pragma unroll
      for (int j = 0; j < K; ++j)
        if (j < it.kn && fp.rf_k[f] == it.k0 + j) it.fslot[j] = f;
    }
  }
}

// Average over the n_child samples of one child (rows ep[i * L + x], the
// multihit rows at ep[mh_off + i * L + x]), multiplied into the products;
// tavg_c: where the field inner averages of this child go, or nullptr.
template <int K, bool MH>
__device__ __forceinline__ void fold_item_child(FoldItem<K, MH>& it, const double2* ep, int mh_off, int n_child,
                                                int L, double inv, double2* tavg_c, size_t tavg_stride) {
  double2 avg[K];
#pragma unroll
  for (int j = 0; j < K; ++j) avg[j] = make_double2(0.0, 0.0);
  // every lane sums all K slots (those past the group's last take r = 0 and
  // are never stored), so that no branch splits the wavefront
#pragma unroll 2
  for (int i = 0; i < n_child; ++i) {
    const double2 u = ep[i * L + it.x0];
    double2 uh = u;
    if (MH) uh = ep[mh_off + i * L + it.x0];
#pragma unroll
    for (int j = 0; j < K; ++j)
      avg[j] = cmac_conj(avg[j], it.mh[j] ? uh : u, ep[(it.mh[j] ? mh_off : 0) + i * L + it.xr[j]]);
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    avg[j] = cscale(avg[j], inv);
    it.prod[j] = cmul(it.prod[j], avg[j]);
  }
  if (tavg_c) {
    // streamed: read back only by the field weights after the run
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (it.fslot[j] >= 0) store_stream(tavg_c + (size_t)it.fslot[j] * tavg_stride + it.x0, avg[j]);
  }
}

// acc[k0 + j] += prod[j] for the group's separations
template <int K, bool MH>
__device__ __forceinline__ void fold_item_store(const FoldItem<K, MH>& it, double2* pp) {
  // the accumulators are read together (clamped) before the updates
  double2 old[K];
#pragma unroll
  for (int j = 0; j < K; ++j) old[j] = pp[min(j, it.kn - 1)];
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (j < it.kn) pp[j] = cadd(old[j], it.prod[j]);
}

// rowbuf[e] = mlbuf[src(e)] for e < n.  The NLD loads of a thread are issued
// together, unconditionally (the index is clamped: past the end, the last
// value is loaded and stored again in its own place), so that no branch or
// wait separates them.
template <int NLD, typename Src>
__device__ __forceinline__ void fold_stage(double2* rowbuf, int n, const double2* __restrict__ mlbuf, Src src) {
  for (int e0 = threadIdx.x; e0 < n; e0 += NLD * (int)blockDim.x) {
    double2 v[NLD];
#pragma unroll
    for (int j = 0; j < NLD; ++j) v[j] = mlbuf[src(min(e0 + j * (int)blockDim.x, n - 1))];
#pragma unroll
    for (int j = 0; j < NLD; ++j) rowbuf[min(e0 + j * (int)blockDim.x, n - 1)] = v[j];
  }
}

template <int K, bool MH, bool PC>
__global__ __launch_bounds__(256) void ml_fold_rows_kernel(const LatDesc* __restrict__ lats, const MLDesc* __restrict__ mls,
                                    const int2* __restrict__ blocks, int child_level, int parent_level, int n_levels,
                                    int n_child, int sample_base, const int* __restrict__ rvals,
                                    const double2* __restrict__ mlbuf, double2* __restrict__ accbuf,
                                    const FieldLat* __restrict__ fls, FieldParams fp, int tavg_m,
                                    double* __restrict__ fbuf, int lds_vals) {
  // PC false: [children][n_child][L], then the multihit rows likewise;
  // PC true: [n_child][L] of one child, then its multihit rows (twice, for
  // the pipelined staging, where lds_vals, the double2 capacity, allows)
  extern __shared__ double2 rowbuf[];
  // neighbouring rows (adjacent in memory) on one XCD, so that its L2 and
  // memory requests see contiguous stretches of the time lines
  const int2 bk = blocks[xcd_block(blockIdx.x, gridDim.x)];
  const LatDesc d = lats[bk.x];
  // fields read through the pointer: a local copy indexed by a run-time level
  // would live in scratch memory
  const MLDesc* mp = mls + bk.x;
  const int L = d.L, L2 = L * L;
  const int ns_child = mp->ns[child_level];
  const int ns_parent = parent_level == n_levels ? 1 : mp->ns[parent_level];
  const int nR = mp->nR, n_r = mp->n_r, n_axes = mp->n_axes, r_off = mp->r_off;
  const uint64_t ell = mp->ell, ell_mh = mp->ell_mh, acc_parent = mp->acc[parent_level];
  const int children = ns_child / ns_parent;
  const int S = bk.y / (n_axes * L2), rem = bk.y - S * n_axes * L2;
  const int axis = rem / L2, row = rem - axis * L2;
  // row (a, b) across the axis: x-rows (y, z), y-rows (x, z), z-rows (x, y)
  const int ra = row % L, rb = row / L;
  const int stride = axis == 0 ? 1 : (axis == 1 ? L : L2);
  const int base = axis == 0 ? row * L : (axis == 1 ? rb * L2 + ra : rb * L + ra);
  const int ngroups = (n_r + K - 1) / K;
  const int per_child = n_child * L;
  // field separations stored by the x rows (uniform per block)
  const bool tavg_on = tavg_m >= 0 && axis == 0;
  double2* tv = tavg_on ? (double2*)(fbuf + fls[bk.x].tavg) + (size_t)tavg_m * fp.n_rf * ns_child * d.L3 : nullptr;
  const size_t tavg_stride = (size_t)ns_child * d.L3;
  const double inv = 1.0 / (double)n_child;
  // element (h, c, i, x) of the staged rows: line h (plain, multihit) of
  // sample i of child c at position x along the row
  auto line = [&](int h, int c, int i, int x) -> size_t {
    return (h ? ell_mh : ell) + ((size_t)(sample_base + i) * ns_child + S * children + c) * d.L3 + (size_t)base +
           (size_t)x * stride;
  };
  auto acc = [&](const FoldItem<K, MH>& it) {
    return accbuf + acc_parent + ((size_t)S * d.L3 + (size_t)base + (size_t)it.x0 * stride) * nR + axis * n_r + it.k0;
  };
  if constexpr (!PC) {
    const int staged = children * per_child;
    fold_stage<16>(rowbuf, (MH ? 2 : 1) * staged, mlbuf, [&](int e) {
      const int rw = e / L, x = e - rw * L;
      const int i = rw % n_child, hc = rw / n_child, c = hc % children, h = hc / children;
      return line(h, c, i, x);
    });
    __syncthreads();
    for (int item = threadIdx.x; item < L * ngroups; item += blockDim.x) {
      FoldItem<K, MH> it;
      fold_item_init(it, item, ngroups, L, axis, n_r, r_off, rvals, tavg_on, fp);
      for (int c = 0; c < children; ++c)
        fold_item_child(it, rowbuf + c * per_child, staged, n_child, L, inv,
                        tv ? tv + (size_t)(S * children + c) * d.L3 + base : nullptr, tavg_stride);
      fold_item_store(it, acc(it));
    }
  } else {
    const int items = L * ngroups;
    const bool active = (int)threadIdx.x < items;
    FoldItem<K, MH> it;
    fold_item_init(it, min((int)threadIdx.x, items - 1), ngroups, L, axis, n_r, r_off, rvals, tavg_on, fp);
    const int n_c = (MH ? 2 : 1) * per_child;  // staged values of one child
    auto src = [&](int c, int e) {
      const int rw = e / L, x = e - rw * L;
      return line(rw / n_child, c, rw % n_child, x);
    };
    auto fold_child = [&](int c, const double2* rows) {
      if (active)
        fold_item_child(it, rows, per_child, n_child, L, inv,
                        tv ? tv + (size_t)(S * children + c) * d.L3 + base : nullptr, tavg_stride);
    };
    constexpr int NP = fold_prefetch(MH);
    if (n_c <= NP * (int)blockDim.x && 2 * n_c <= lds_vals) {
      // software pipeline: the rows of child c + 1 are loaded into registers
      // while child c is folded from one of two LDS buffers, then stored to
      // the other.  One barrier per child: buffer (c + 1) & 1 was last read
      // while folding child c - 1, before the barrier that ended that step.
      // The loads and stores are clamped: past the end, the last value is
      // loaded and stored again in its own place.
      fold_stage<NP>(rowbuf, n_c, mlbuf, [&](int e) { return src(0, e); });
      __syncthreads();
      for (int c = 0; c < children; ++c) {
        const bool next = c + 1 < children;
        // plain doubles: an array of double2 here is kept in scratch memory
        double vx[NP], vy[NP];
        if (next) {
#pragma unroll
          for (int j = 0; j < NP; ++j) {
            const double2 t = mlbuf[src(c + 1, min((int)threadIdx.x + j * (int)blockDim.x, n_c - 1))];
            vx[j] = t.x;
            vy[j] = t.y;
          }
        }
        fold_child(c, rowbuf + (c & 1) * n_c);
        if (next) {
          double2* buf = rowbuf + ((c + 1) & 1) * n_c;
#pragma unroll
          for (int j = 0; j < NP; ++j)
            buf[min((int)threadIdx.x + j * (int)blockDim.x, n_c - 1)] = make_double2(vx[j], vy[j]);
        }
        __syncthreads();
      }
    } else {
      for (int c = 0; c < children; ++c) {
        if (c) __syncthreads();  // the previous child's rows are no longer read
        fold_stage<4>(rowbuf, n_c, mlbuf, [&](int e) { return src(c, e); });
        __syncthreads();
        fold_child(c, rowbuf);
      }
    }
    if (active) fold_item_store(it, acc(it));
  }
}

// out[(lat * max_r + k) * 2 + {0,1}] = L^-3 sum_x0 acc_top[x0][k]; with three
// axes the mean over the axes of the real part: the separation -r e
// estimates the complex conjugate of +r e exactly (every factor is), so the
// real part is the mean of both orientations.
__global__ __launch_bounds__(kRedBlock) void ml_final_kernel(const LatDesc* __restrict__ lats, const MLDesc* __restrict__ mls, int max_r,
                                int top_level, const double2* __restrict__ accbuf, double* __restrict__ out) {
  __shared__ double sh[16];
  const int lat = blockIdx.x, k = blockIdx.y;
  const LatDesc d = lats[lat];
  // read through the pointer: a local copy indexed by the run-time level
  // would live in scratch memory
  const MLDesc& m = mls[lat];
  if (k >= m.n_r) return;  // uniform per block
  double re = 0.0, im = 0.0;
  const double2* a = accbuf + m.acc[top_level];
  for (int ax = 0; ax < m.n_axes; ++ax) {
    double sr = 0.0, si = 0.0;
    for (int x0 = threadIdx.x; x0 < d.L3; x0 += blockDim.x) {
      const double2 v = a[(size_t)x0 * m.nR + ax * m.n_r + k];
      sr += v.x;
      si += v.y;
    }
    re += block_sum(sr, sh) / (double)d.L3;
    im += block_sum(si, sh) / (double)d.L3;
  }
  if (threadIdx.x == 0) {
    out[((size_t)lat * max_r + k) * 2] = re / (double)m.n_axes;
    out[((size_t)lat * max_r + k) * 2 + 1] = m.n_axes == 1 ? im : 0.0;
  }
}

// ---------------------------------------------------------------------------
// ensemble of multilevel runs and the connected profile of Eq. (7)
// ---------------------------------------------------------------------------
// acc[i] += src[i]
__global__ void ens_add_kernel(double* __restrict__ acc, const double* __restrict__ src, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) acc[i] += src[i];
}

// acc[lat][c] += red[lat][col0 + c] / V: the lattice averages of one set of
// six field operators from the reduced plain-observable rows
__global__ void ens_omean_kernel(const LatDesc* __restrict__ lats, const double* __restrict__ red, int width,
                                 int col0, int n_lats, double* __restrict__ acc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 6 * n_lats) return;
  const int lat = i / 6, c = i - lat * 6;
  acc[i] += red[(size_t)lat * width + col0 + c] / (2.0 * (double)lats[lat].V2);
}

// conn[e] = <P* P O_c>(r_f, d) / <P* P>(r_f) - <O_c> with ensemble means:
// fsum, csum and osum are sums over the same n runs, so the ratio takes the
// sums and only the subtracted mean divides by n.  e = ((f * 2 + plane) * 6
// + c) * L^2 + pq; cidx[f] is the index of r_f in the correlator.
__global__ void ens_connected_kernel(const double2* __restrict__ fsum, const double2* __restrict__ csum,
                                     const double* __restrict__ osum, FieldParams fp, int L, double inv_n,
                                     double2* __restrict__ conn) {
  const int L2 = L * L;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= fp.n_rf * 12 * L2) return;
  const int c = (e / L2) % 6, f = e / (12 * L2);
  const double2 a = fsum[e], b = csum[fp.rf_k[f]];
  const double den = b.x * b.x + b.y * b.y;
  conn[e] = make_double2((a.x * b.x + a.y * b.y) / den - osum[c] * inv_n, (a.y * b.x - a.x * b.y) / den);
}

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

namespace {
template <typename R, bool FIELD, bool SQ>
void launch_sample_t(const void* links, const LatDesc* lats, const MLDesc* mls, const FieldLat* fls, BlockTable bt,
                     int inner_th, int sample, double2* mlbuf, double* fbuf, hipStream_t st) {
  hipLaunchKernelGGL((ml_sample_kernel<R, FIELD, SQ>), dim3(bt.n_blocks), dim3(bt.block), 0, st, (const R*)links,
                     lats, mls, fls, bt.dev, inner_th, sample, mlbuf, fbuf);
}
template <typename R>
void launch_sample_r(const void* links, const LatDesc* lats, const MLDesc* mls, const FieldLat* fls, BlockTable bt,
                     int inner_th, int sample, bool field, bool squared, double2* mlbuf, double* fbuf, hipStream_t st) {
  if (!field)
    launch_sample_t<R, false, false>(links, lats, mls, fls, bt, inner_th, sample, mlbuf, fbuf, st);
  else if (squared)
    launch_sample_t<R, true, true>(links, lats, mls, fls, bt, inner_th, sample, mlbuf, fbuf, st);
  else
    launch_sample_t<R, true, false>(links, lats, mls, fls, bt, inner_th, sample, mlbuf, fbuf, st);
}
}  // namespace

hipError_t launch_ml_sample(int prec, const void* links, const LatDesc* lats, const MLDesc* mls, const FieldLat* fls,
                            BlockTable bt, int inner_th, int sample, bool field, bool squared, double2* mlbuf,
                            double* fbuf, hipStream_t st) {
  if (bt.n_blocks == 0) return hipSuccess;
  if (prec == kFP64)
    launch_sample_r<double>(links, lats, mls, fls, bt, inner_th, sample, field, squared, mlbuf, fbuf, st);
  else
    launch_sample_r<float>(links, lats, mls, fls, bt, inner_th, sample, field, squared, mlbuf, fbuf, st);
  return hipGetLastError();
}

hipError_t launch_ml_fold(const LatDesc* lats, const MLDesc* mls, BlockTable bt, int child_level, int parent_level,
                          int n_levels, int child_is_inner, int n_child, int sample_base, const int* rvals,
                          const double2* mlbuf, double2* accbuf, hipStream_t st) {
  hipLaunchKernelGGL(ml_fold_kernel, dim3(bt.n_blocks), dim3(bt.block), 0, st, lats, mls, bt.dev, child_level,
                     parent_level, n_levels, child_is_inner, n_child, sample_base, rvals, mlbuf, accbuf);
  return hipGetLastError();
}

template <int K, bool MH>
void launch_fold_rows_km(bool per_child, BlockTable bt, int threads, size_t lds, const LatDesc* lats,
                         const MLDesc* mls, int child_level, int parent_level, int n_levels, int n_child,
                         int sample_base, const int* rvals, const double2* mlbuf, double2* accbuf,
                         const FieldLat* fls, const FieldParams& fp, int tavg_m, double* fbuf, hipStream_t st) {
  if (per_child)
    hipLaunchKernelGGL((ml_fold_rows_kernel<K, MH, true>), dim3(bt.n_blocks), dim3(threads), lds, st, lats, mls,
                       bt.dev, child_level, parent_level, n_levels, n_child, sample_base, rvals, mlbuf, accbuf, fls,
                       fp, tavg_m, fbuf, (int)(lds / sizeof(double2)));
  else
    hipLaunchKernelGGL((ml_fold_rows_kernel<K, MH, false>), dim3(bt.n_blocks), dim3(threads), lds, st, lats, mls,
                       bt.dev, child_level, parent_level, n_levels, n_child, sample_base, rvals, mlbuf, accbuf, fls,
                       fp, tavg_m, fbuf, (int)(lds / sizeof(double2)));
}

template <int K>
void launch_fold_rows_k(bool multihit, bool per_child, BlockTable bt, int threads, size_t lds, const LatDesc* lats,
                        const MLDesc* mls, int child_level, int parent_level, int n_levels, int n_child,
                        int sample_base, const int* rvals, const double2* mlbuf, double2* accbuf,
                        const FieldLat* fls, const FieldParams& fp, int tavg_m, double* fbuf, hipStream_t st) {
  if (multihit)
    launch_fold_rows_km<K, true>(per_child, bt, threads, lds, lats, mls, child_level, parent_level, n_levels, n_child,
                                 sample_base, rvals, mlbuf, accbuf, fls, fp, tavg_m, fbuf, st);
  else
    launch_fold_rows_km<K, false>(per_child, bt, threads, lds, lats, mls, child_level, parent_level, n_levels,
                                  n_child, sample_base, rvals, mlbuf, accbuf, fls, fp, tavg_m, fbuf, st);
}

hipError_t launch_ml_fold_rows(const LatDesc* lats, const MLDesc* mls, BlockTable bt, int threads, size_t lds,
                               int k_slots, bool multihit, bool per_child, int child_level, int parent_level,
                               int n_levels, int n_child, int sample_base, const int* rvals, const double2* mlbuf,
                               double2* accbuf, const FieldLat* fls, const FieldParams& fp, int tavg_m, double* fbuf,
                               hipStream_t st) {
  if (bt.n_blocks == 0) return hipSuccess;
  if (k_slots == 4)
    launch_fold_rows_k<4>(multihit, per_child, bt, threads, lds, lats, mls, child_level, parent_level, n_levels,
                          n_child, sample_base, rvals, mlbuf, accbuf, fls, fp, tavg_m, fbuf, st);
  else if (k_slots == 6)
    launch_fold_rows_k<6>(multihit, per_child, bt, threads, lds, lats, mls, child_level, parent_level, n_levels,
                          n_child, sample_base, rvals, mlbuf, accbuf, fls, fp, tavg_m, fbuf, st);
  else if (k_slots == 8)
    launch_fold_rows_k<8>(multihit, per_child, bt, threads, lds, lats, mls, child_level, parent_level, n_levels,
                          n_child, sample_base, rvals, mlbuf, accbuf, fls, fp, tavg_m, fbuf, st);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int ml_fold_rows_k(int max_n_r) {
  // the fewest groups of at most 8, then the smallest K of 4, 6, 8 that
  // covers the separations in that many groups
  const int groups = (std::max(max_n_r, 1) + 7) / 8;
  const int per = (std::max(max_n_r, 1) + groups - 1) / groups;
  return per <= 4 ? 4 : (per <= 6 ? 6 : 8);
}

int ml_fold_rows_threads(int L, int n_r, int k_slots) {
  const int items = L * ((n_r + k_slots - 1) / k_slots);
  return std::min(256, (items + 63) / 64 * 64);
}
size_t ml_fold_rows_max_lds() { return kFoldLds; }
int ml_fold_rows_prefetch(bool multihit) { return fold_prefetch(multihit); }

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

hipError_t launch_ens_add(double* acc, const double* src, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(ens_add_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, acc, src, n);
  return hipGetLastError();
}

hipError_t launch_ens_omean(const LatDesc* lats, const double* red, int width, int col0, int n_lats, double* acc,
                            hipStream_t st) {
  hipLaunchKernelGGL(ens_omean_kernel, dim3(blocks_for(6 * (uint64_t)n_lats, 64)), dim3(64), 0, st, lats, red, width,
                     col0, n_lats, acc);
  return hipGetLastError();
}

hipError_t launch_ens_connected(const double2* fsum, const double2* csum, const double* osum, FieldParams fp, int L,
                                double inv_n, double2* conn, hipStream_t st) {
  const uint64_t n = (uint64_t)fp.n_rf * 12 * L * L;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(ens_connected_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, fsum, csum, osum, fp, L,
                     inv_n, conn);
  return hipGetLastError();
}

}  // namespace u1ml
