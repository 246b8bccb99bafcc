// engine.h -- host-side interface between the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace u1ml {

enum Precision { kFP64 = 0, kFP32 = 1 };
enum UpdateKind { kMetropolis = 0, kOverrelax = 1 };

// Blocks of a batched launch: blocks[b] = {lattice, first item of the block}.
struct BlockTable {
  const int2* dev = nullptr;
  int n_blocks = 0;
  int block = 0;
};

// --- link updates (sweep_f64.hip, sweep_f32.hip) ---
hipError_t launch_init_f64(double* links, const LatDesc* lats, BlockTable bt, int hot, hipStream_t st);
hipError_t launch_init_f32(float* links, const LatDesc* lats, BlockTable bt, int hot, hipStream_t st);
// one class pass of a single lattice (geometry by value); log as in u1ml_set_debug.
// bump_n > 0 (overrelaxation passes only, which do not read the pass ids):
// the pass also adds 1 to pass_ids[0 .. bump_n), once all its blocks are done
// reading nothing from them; used on the last pass of a compound sweep.
// xcd_map != 0: blocks in XCD-contiguous order (xcd_block), else hardware order
hipError_t launch_class_pass_f64(int kind, double* links, const LatDesc& d, int block, int xcd_map, int mu, int parity,
                                 int th_frozen, int n_hits, uint64_t* pass_ids, uint8_t* log, int bump_n,
                                 hipStream_t st);
hipError_t launch_class_pass_f32(int kind, float* links, const LatDesc& d, int block, int xcd_map, int mu, int parity,
                                 int th_frozen, int n_hits, uint64_t* pass_ids, uint8_t* log, int bump_n,
                                 hipStream_t st);
// one class pass of every lattice of a batch; blocks[b] = {lattice, time slice,
// first offset within the slice, 0}, one block per (updated slice, chunk)
hipError_t launch_class_pass_batch_f64(int kind, double* links, const LatDesc* lats, const int4* blocks,
                                       int n_blocks, int block, int xcd_map, int mu, int parity, int n_hits,
                                       uint64_t* pass_ids, int bump_n, hipStream_t st);
hipError_t launch_class_pass_batch_f32(int kind, float* links, const LatDesc* lats, const int4* blocks,
                                       int n_blocks, int block, int xcd_map, int mu, int parity, int n_hits,
                                       uint64_t* pass_ids, int bump_n, hipStream_t st);
hipError_t launch_bump_pass_ids(uint64_t* pass_ids, int n, hipStream_t st);
// fill n bytes with v (graph-safe replacement of a memset)
hipError_t launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t st);

// --- measurements (measure.hip); prec selects the link element type ---
// Per-lattice multilevel workspace layout (offsets in elements of the
// corresponding buffer).
constexpr int kMaxLevels = 3;
struct MLDesc {
  uint64_t ell;                  // double2: [samples][ns_inner][L3] exp(i * slab time-line angle sum)
  uint64_t ell_mh;               // double2: the same layout, products of multihit means (multihit only)
  uint64_t acc[kMaxLevels + 1];  // double2: level l < inner: [ns_l][L3][nR]; index n_levels = top [L3][nR]
  int ns[kMaxLevels];            // slabs per level
  int nR;                        // stored separations: n_axes * n_r, axis slowest
  int n_r;                       // separations of the r list
  int n_axes;                    // 1: along x; 3: along x, y, z (symmetric correlator)
  int r_off;                     // separations at rvals[r_off ...], encoded r | axis << 16
  int multihit;                  // correlator lines at r >= 2 from ell_mh
};
constexpr int kRAxisShift = 16;  // rvals entry = r | axis << kRAxisShift

// plaquette sum, the six field sums and the six squared-component sums:
// partial[blk][kPlaqFieldWidth], reduced to one such row per lattice
constexpr int kPlaqFieldWidth = 13;
hipError_t launch_plaq_field(int prec, const void* links, const LatDesc* lats, BlockTable bt, double* partial,
                             hipStream_t st);
// reduce per-lattice ranges of 'width'-wide partial rows: out[lat][width]
hipError_t launch_reduce_rows(const double* partial, int width, const int* lat_row_begin, int n_lats,
                              double* out, hipStream_t st);
// Polyakov loop angles poly[lat_off + x3] = sum_t theta_0(x3, t)
hipError_t launch_poly_lines(int prec, const void* links, const LatDesc* lats, BlockTable bt,
                             const uint64_t* poly_off, double* poly, hipStream_t st);
// per-block partials of P (re, im) and of P*(x)P(x + r e_x) for the r list
// one row per spatial site: {cos P, sin P, (Re, Im) of P*(x)P(x + r e_x) per r}
hipError_t launch_poly_corr(const LatDesc* lats, BlockTable bt, const uint64_t* poly_off, const double* poly,
                            const int* rvals, int nR, const int* row_begin, double* rows, hipStream_t st);

// multilevel
struct FieldLat;
// one inner sample: time lines (and multihit means), and with field the slab
// sums of the insertion operators (squared: Eq. (6) instead of Eq. (5))
hipError_t launch_ml_sample(int prec, const void* links, const LatDesc* lats, const MLDesc* mls, const FieldLat* fls,
                            BlockTable bt, int inner_th, int sample, bool field, bool squared, double2* mlbuf,
                            double* fbuf, hipStream_t st);
// sample_base: first stored inner sample of the current inner run (field runs keep them all)
hipError_t launch_ml_fold(const LatDesc* lats, const MLDesc* mls, BlockTable bt, int child_level, int parent_level,
                          int n_levels, int child_is_inner, int n_child, int sample_base, const int* rvals,
                          const double2* mlbuf, double2* accbuf, hipStream_t st);
// the innermost fold by rows: bt has one block per (parent slab, axis, row)
// of every lattice; k_slots = ml_fold_rows_k(largest n_r) separations per
// thread; threads = ml_fold_rows_threads(L, n_r, k_slots) for the largest
// lattice; multihit: the run's estimator (the same for every lattice of a
// run).  per_child false: all children of a parent slab staged at once, lds =
// children * n_child * max L complex values; per_child true: one child at a
// time, lds = n_child * max L complex values, and threads >= L * groups of
// every lattice (one item per thread); with twice that lds and threads *
// ml_fold_rows_prefetch(multihit) >= those values, the rows of the next
// child are loaded while the current one is folded.  Values count twice
// with multihit; lds is at most ml_fold_rows_max_lds() bytes.
// tavg_m >= 0: also store the inner averages of the field separations of
// outer iteration tavg_m into the field buffer (FieldLat::tavg)
struct FieldParams;
hipError_t launch_ml_fold_rows(const LatDesc* lats, const MLDesc* mls, BlockTable bt, int threads, size_t lds,
                               int k_slots, bool multihit, bool per_child, int child_level, int parent_level,
                               int n_levels, int n_child, int sample_base, const int* rvals, const double2* mlbuf,
                               double2* accbuf, const FieldLat* fls, const FieldParams& fp, int tavg_m, double* fbuf,
                               hipStream_t st);
int ml_fold_rows_k(int max_n_r);
int ml_fold_rows_threads(int L, int n_r, int k_slots);
size_t ml_fold_rows_max_lds();
int ml_fold_rows_prefetch(bool multihit);
hipError_t launch_ml_zero(double2* accbuf, uint64_t n, hipStream_t st);
hipError_t launch_ml_final(const LatDesc* lats, const MLDesc* mls, int n_lats, int max_r, int top_level,
                           const double2* accbuf, double* out, hipStream_t st);

// field insertion: per-lattice layout of the field buffer (offsets in doubles)
struct FieldLat {
  int ns;         // inner slabs
  int n_top;      // top-level slabs (two levels), else 1
  uint64_t oall;  // [n_samples][6][ns][L3] slab sums of the field operators, in the
                  // link precision (FP32 values packed two per double for FP32 links)
  uint64_t tavg;  // double2 [n_stored][n_rf][ns][L3]
  uint64_t w;     // double2 [n_stored][n_rf][ns][L3]
  uint64_t g;     // double2 [n_rf][2][6][L2] Fourier-space accumulator
  uint64_t ptop;  // double2 [n_top][n_rf][L3] products of the other top slabs' averages
};
struct FieldParams {
  int n_rf;
  int rf[32];    // field separations (U1ML_MAX_FIELD_R)
  int rf_k[32];  // index of each rf in the lattice's r list
  int n_levels;  // 1 or 2
  int n_outer;   // n_0 for two levels, 1 for one level
  int n_stored;  // outer iterations whose samples are stored: n_outer, or 1 when
                 // every outer iteration is contracted as it completes (replay)
  int n_inner;   // samples per inner run
};
// ensemble sums of multilevel runs (Eq. (7)): acc[i] += src[i]; the field
// means of one operator set (columns col0 .. col0 + 5 of the reduced rows,
// divided by V) into acc[lat][6]; the connected profile of one lattice
hipError_t launch_ens_add(double* acc, const double* src, uint64_t n, hipStream_t st);
hipError_t launch_ens_omean(const LatDesc* lats, const double* red, int width, int col0, int n_lats, double* acc,
                            hipStream_t st);
hipError_t launch_ens_connected(const double2* fsum, const double2* csum, const double* osum, FieldParams fp, int L,
                                double inv_n, double2* conn, hipStream_t st);
// launch shapes of the fast field path (0 = the default of the kernel): x
// planes per block of the W transform, plane pairs per block of the O
// transform, threads per block of the contraction; every choice gives the
// same bits
struct FieldTuning {
  int w_planes = 0;
  int o_planes = 0;
  int zcon_threads = 0;
};
// contraction of all stored samples of one lattice into the Fourier-space
// accumulator (cleared first if zero_g) and, if finalize, into F
// (tavg_ready: the inner averages of the field separations are in place
// already, written by the row fold)
// [n_rf][2][6][L][L] (complex); general = true takes the stored-transform path
// for any geometry; fp32_store keeps the fast path's per-sample transforms
// in FP32 between its kernels (FP32 lattices)
hipError_t launch_field_contract(const LatDesc* lat, const MLDesc* ml, const FieldLat* fl, const FieldLat& hfl,
                                 FieldParams fp, int L, const double2* mlbuf, const double2* accbuf, double* fbuf,
                                 double2* scratch, size_t scratch_elems, double2* F, bool general, bool fp32_store,
                                 bool zero_g, bool finalize, bool tavg_ready, FieldTuning tune, hipStream_t st);
// the largest x planes per block the W (pairs = false) or O (pairs = true)
// transform accepts at lattice size L (LDS and block-size limits); 0 when L
// has no fast path
int field_max_planes(int L, bool pairs);

// streaming probe (probe.hip): kind 0 reads n_bytes of a (16-byte loads),
// kind 1 copies a to b, kind 2 zeroes b; grid-stride over `blocks` blocks of 256
hipError_t launch_stream_probe(int kind, const void* a, void* b, size_t n_bytes, float* sink, int blocks,
                               hipStream_t st);

}  // namespace u1ml
