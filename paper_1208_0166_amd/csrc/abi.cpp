// abi.cpp -- the u1ml C ABI: lattice and batch handles, the update schedule
// (compound sweeps, multilevel nesting, field insertion), measurements,
// checkpoints, HIP-graph replay and the block-size autotuner.  Host code
// only; all lattice arithmetic runs in the kernels of sweep_f64.hip,
// sweep_f32.hip and measure.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/u1ml.h"
#include "engine.h"

using namespace u1ml;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define U1_HIP(expr)                                                                                      \
  do {                                                                                                    \
    hipError_t e_ = (expr);                                                                               \
    if (e_ != hipSuccess) return fail(U1ML_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define U1_TRY(expr)     \
  do {                   \
    int rc_ = (expr);    \
    if (rc_) return rc_; \
  } while (0)

// largest |theta| accepted from the host; the updates fold angles back into
// [-pi, pi) by whole periods, which needs them to be of moderate size
constexpr double kMaxAngle = 64.0;
// largest Metropolis width: theta + eps (2u - 1) with eps <= 2 pi already
// reaches every angle, and a bounded proposal keeps the fold into [-pi, pi)
// to a few periods
constexpr double kMaxEps = 2.0 * 3.14159265358979323846;
// scratch for the field contraction, per engine
constexpr size_t kFieldScratchBytes = 512u << 20;
// A two-level run with field insertion keeps every inner sample's time lines
// and field slab sums until the end.  When that storage would take more than
// this fraction of the device memory available to the run, the run is
// replayed instead: a first pass computes the top-level averages, a second
// pass repeats the identical update sequence (counter-based random numbers,
// restored links and pass ids) and contracts each outer iteration's samples
// as soon as that iteration completes, so only one outer iteration's samples
// are stored.
constexpr double kFieldStoreFraction = 0.6;
constexpr size_t kMaxGraphs = 16;
// multilevel runs of more sublattice updates than this launch kernel by
// kernel: capturing millions of launches costs more host time and memory
// than the graph saves
constexpr long long kMaxCapturedUpdates = 1 << 14;
// the mediator-plane transform keeps (L + L^2) complex values in 64 KiB of LDS
constexpr int kMaxFieldL = 62;

// device buffer that only grows
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = true;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p && owned) (void)hipFree(p);
  }
  int ensure(size_t want) {
    if (want <= bytes) return U1ML_OK;
    if (!owned) return fail(U1ML_ESTATE, "caller-owned buffer too small");
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (want == 0) return U1ML_OK;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      return fail(U1ML_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    bytes = want;
    return U1ML_OK;
  }
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};

struct Table {
  DevBuf buf;
  int n_blocks = 0;
  int block = 0;
  std::vector<int> lat_block_begin;  // n_lats + 1
};

// Bump allocator over a fixed device range (the allocation-free entry point
// places its whole workspace in the library's static device array).
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  // view of the next `bytes` (256-byte aligned) as a buffer the arena keeps
  int carve(DevBuf& b, size_t bytes) {
    const size_t at = (used + 255) & ~(size_t)255;
    if (at > cap || bytes > cap - at)
      return fail(U1ML_EINVAL, "the run's workspace (more than " + std::to_string(at + bytes) +
                                   " bytes) exceeds the static device array of " + std::to_string(cap) + " bytes");
    b.p = base + at;
    b.bytes = bytes;
    b.owned = false;
    used = at + bytes;
    return U1ML_OK;
  }
};

struct PassTable {
  DevBuf buf;
  int n_blocks = 0;
};

struct MLState {
  bool valid = false;        // a multilevel has completed
  bool field_valid = false;  // ... with the field insertion
  std::vector<long long> key;
  int n_levels = 0;
  int th[U1ML_MAX_LEVELS] = {0, 0, 0};
  int n[U1ML_MAX_LEVELS] = {0, 0, 0};
  int n_metro = 1, n_or = 0;
  int max_r = 0;
  std::vector<int> nR;        // per lattice
  std::vector<MLDesc> h_mls;  // per lattice
  DevBuf mls, rvals, mlbuf, accbuf, corr;
  uint64_t acc_elems = 0;
  // field insertion
  bool field = false;
  FieldParams fp{};
  std::vector<FieldLat> h_fls;
  std::vector<uint64_t> fout_off;  // per lattice, double2 elements
  DevBuf fls, fbuf, fout, scratch;
  size_t scratch_elems = 0;
  bool replay = false;        // two-pass run, one outer iteration stored
  bool tavg_from_fold = false;  // every inner fold of the run stored the field inner averages
  bool store_field = true;    // ml_sample stores the field slab sums
  DevBuf links_backup, pass_backup;
  // shape of the last completed run (r lists, field separations, operator set)
  std::vector<long long> shape;
  unsigned run_flags = 0;  // estimator flags of that run
};

// Sums over multilevel runs of the correlator, the field profile and the
// lattice means of the inserted operators (Eq. (7)).
struct Ensemble {
  std::vector<long long> shape;  // MLState::shape of the runs
  long long n = 0;
  unsigned flags = 0;
  int max_r = 0;
  std::vector<int> nR;
  bool field = false;
  FieldParams fp{};
  std::vector<uint64_t> fout_off;
  uint64_t fout_elems = 0;
  DevBuf corr, fsum, omean, partial, red, row_begin, conn;
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  int metro_passes = 0;
};

}  // namespace

struct Engine {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool use_graphs = true;
  int prec = U1ML_FP64;
  int block = 256;         // class-pass threads per block
  int xcd_map = 1;         // class-pass blocks in XCD-contiguous order
  int sample_block = 256;  // threads per block of the per-sample kernel
  int fold_threads = 0;    // threads per block of the row fold; 0 = by L and n_r
  int fold_stage = 0;      // row fold staging: 1 all children, 2 one child at a time, 0 by size
  FieldTuning ftune;       // launch shapes of the fast field path
  int n_lats = 0;
  std::vector<LatDesc> h_lats;
  DevBuf lats;
  DevBuf links;
  size_t link_elems = 0;
  DevBuf pass_ids;
  std::vector<uint64_t> h_pass_ids;
  std::map<std::pair<std::vector<int>, int>, std::unique_ptr<Table>> tables;
  std::map<std::pair<int, int>, std::unique_ptr<PassTable>> pass_tables;
  // debug log (single lattice)
  DevBuf log;
  size_t log_cap = 0, log_used = 0;
  bool debug = false;
  bool field_general = false;  // u1ml_set_debug flags & 2
  bool fold_general = false;   // u1ml_set_debug flags & 4
  bool force_replay = false;   // u1ml_set_debug flags & 8
  bool log_off = false;        // no accept-log recording (replayed updates)
  unsigned estimator = 0;      // u1ml_set_estimator flags
  // measurement scratch
  DevBuf partial, rows, poly, poly_off, row_begin, red_out, rvals_tmp;
  MLState ml;
  // the multilevel state the ML methods work on: ml, or during an
  // allocation-free run a state whose buffers are views into the arena
  MLState* mlp = &ml;
  // non-null during an allocation-free run: workspace and block tables are
  // carved from it instead of allocated (tables are then rebuilt per call)
  Arena* arena = nullptr;
  std::vector<std::unique_ptr<Table>> arena_tables;
  Ensemble ens;
  // plain observables of every lattice, valid while the links are unchanged:
  // epoch advances with every launch sequence that may write links
  uint64_t epoch = 0, obs_epoch = ~0ull;
  std::vector<u1ml_observables> obs_cache;
  // captured launch sequences
  std::map<std::vector<long long>, GraphEntry> graphs;
  bool capturing = false;
  // optional per-kernel timing (u1ml_profile_sweeps)
  std::vector<std::pair<hipEvent_t, hipEvent_t>>* prof[2] = {nullptr, nullptr};
  // optional timing of one measurement kernel family (autotuner): events
  // around every launch of family fam_id
  enum Family { kFamSample = 0, kFamFold = 1, kFamField = 2 };
  std::vector<std::pair<hipEvent_t, hipEvent_t>>* fam_prof = nullptr;
  int fam_id = -1;

  ~Engine() {
    if (stream) (void)hipStreamSynchronize(stream);
    drop_graphs();
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second.exec);
    graphs.clear();
  }

  size_t elem_size() const { return prec == U1ML_FP64 ? 8 : 4; }

  int set_device() {
    U1_HIP(hipSetDevice(device));
    return U1ML_OK;
  }

  // Host <-> device copy in this handle's stream order, complete on return.
  // Never through the legacy default stream: that would tie the handle to
  // the streams of other handles (and fail while one of them is being
  // captured into a graph by another thread).
  int copy(void* dst, const void* src, size_t n, hipMemcpyKind kind) {
    if (n == 0) return U1ML_OK;
    U1_HIP(hipMemcpyAsync(dst, src, n, kind, stream));
    U1_HIP(hipStreamSynchronize(stream));
    return U1ML_OK;
  }

  // block table for per-lattice item counts (built once, reused)
  int table(const std::vector<int>& items, int blk, Table** out) {
    if (arena) return arena_table(items, blk, out);
    auto key = std::make_pair(items, blk);
    auto it = tables.find(key);
    if (it != tables.end()) {
      *out = it->second.get();
      return U1ML_OK;
    }
    if (capturing) return fail(U1ML_ESTATE, "internal: block table built during graph capture");
    std::unique_ptr<Table> t(new Table());
    std::vector<int2> h;
    t->lat_block_begin.push_back(0);
    for (int i = 0; i < (int)items.size(); ++i) {
      for (int b = 0; b < items[i]; b += blk) h.push_back(make_int2(i, b));
      t->lat_block_begin.push_back((int)h.size());
    }
    t->n_blocks = (int)h.size();
    t->block = blk;
    if (!h.empty()) {
      U1_TRY(t->buf.ensure(h.size() * sizeof(int2)));
      U1_TRY(copy(t->buf.p, h.data(), h.size() * sizeof(int2), hipMemcpyHostToDevice));
    }
    *out = t.get();
    tables[key] = std::move(t);
    return U1ML_OK;
  }

  // the same table carved from the arena (not cached: the arena's contents
  // belong to the current call only)
  int arena_table(const std::vector<int>& items, int blk, Table** out) {
    std::unique_ptr<Table> t(new Table());
    std::vector<int2> h;
    t->lat_block_begin.push_back(0);
    for (int i = 0; i < (int)items.size(); ++i) {
      for (int b = 0; b < items[i]; b += blk) h.push_back(make_int2(i, b));
      t->lat_block_begin.push_back((int)h.size());
    }
    t->n_blocks = (int)h.size();
    t->block = blk;
    U1_TRY(arena->carve(t->buf, h.size() * sizeof(int2)));
    U1_TRY(copy(t->buf.p, h.data(), h.size() * sizeof(int2), hipMemcpyHostToDevice));
    *out = t.get();
    arena_tables.push_back(std::move(t));
    return U1ML_OK;
  }

  // a multilevel workspace buffer: allocated (grows, kept for later runs) or
  // carved from the arena
  int reserve(DevBuf& b, size_t bytes) { return arena ? arena->carve(b, bytes) : b.ensure(bytes); }

  // class-pass blocks of a batch: {lattice, slice, first offset, 0} for every
  // updated time slice (th = 0: all; else t != 0 mod th) of every lattice
  int pass_table(int th, PassTable** out) {
    auto key = std::make_pair(th, block);
    auto it = pass_tables.find(key);
    if (it != pass_tables.end()) {
      *out = it->second.get();
      return U1ML_OK;
    }
    if (capturing) return fail(U1ML_ESTATE, "internal: block table built during graph capture");
    std::unique_ptr<PassTable> t(new PassTable());
    std::vector<int4> h;
    for (int i = 0; i < n_lats; ++i) {
      const LatDesc& d = h_lats[i];
      const int slices = class_slices(d.T, th > 0 ? 1 : 0, th);
      for (int j = 0; j < slices; ++j)
        for (int o = 0; o < d.L3 / 2; o += block) h.push_back(make_int4(i, class_slice(j, th > 0 ? 1 : 0, th), o, 0));
    }
    t->n_blocks = (int)h.size();
    if (!h.empty()) {
      U1_TRY(t->buf.ensure(h.size() * sizeof(int4)));
      U1_TRY(copy(t->buf.p, h.data(), h.size() * sizeof(int4), hipMemcpyHostToDevice));
    }
    *out = t.get();
    pass_tables[key] = std::move(t);
    return U1ML_OK;
  }

  BlockTable bt(Table* t) const {
    BlockTable b;
    b.dev = t->buf.as<int2>();
    b.n_blocks = t->n_blocks;
    b.block = t->block;
    return b;
  }

  // --- updates ---
  int class_pass(int kind, int mu, int parity, int th_frozen, int n_hits, uint8_t* logp, int bump_n = 0) {
    ++epoch;
    hipError_t e;
    if (n_lats == 1) {
      if (prec == U1ML_FP64)
        e = launch_class_pass_f64(kind, links.as<double>(), h_lats[0], block, xcd_map, mu, parity, th_frozen,
                                  n_hits,
                                  pass_ids.as<uint64_t>(), logp, bump_n, stream);
      else
        e = launch_class_pass_f32(kind, links.as<float>(), h_lats[0], block, xcd_map, mu, parity, th_frozen,
                                  n_hits,
                                  pass_ids.as<uint64_t>(), logp, bump_n, stream);
    } else {
      PassTable* t;
      U1_TRY(pass_table(mu > 0 && th_frozen > 0 ? th_frozen : 0, &t));
      if (prec == U1ML_FP64)
        e = launch_class_pass_batch_f64(kind, links.as<double>(), lats.as<LatDesc>(), t->buf.as<int4>(),
                                        t->n_blocks, block, xcd_map, mu, parity, n_hits, pass_ids.as<uint64_t>(),
                                        bump_n, stream);
      else
        e = launch_class_pass_batch_f32(kind, links.as<float>(), lats.as<LatDesc>(), t->buf.as<int4>(),
                                        t->n_blocks, block, xcd_map, mu, parity, n_hits, pass_ids.as<uint64_t>(),
                                        bump_n, stream);
    }
    U1_HIP(e);
    return U1ML_OK;
  }

  int timed_class_pass(int kind, int mu, int parity, int th_frozen, int n_hits, uint8_t* logp, int bump_n = 0) {
    if (!prof[kind]) return class_pass(kind, mu, parity, th_frozen, n_hits, logp, bump_n);
    hipEvent_t a, z;
    U1_HIP(hipEventCreate(&a));
    U1_HIP(hipEventCreate(&z));
    prof[kind]->push_back(std::make_pair(a, z));
    U1_HIP(hipEventRecord(a, stream));
    int rc = class_pass(kind, mu, parity, th_frozen, n_hits, logp, bump_n);
    U1_HIP(hipEventRecord(z, stream));
    return rc;
  }

  // Compound sweep (Sec. 2.1): Metropolis pass then n_or OR passes, classes
  // mu = 0..3 outer, parity inner.
  int sweep(int n_metro, int n_or, int th_frozen) {
    if (n_metro > 0) {
      for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p) {
          uint8_t* lp = nullptr;
          if (debug && n_lats == 1 && !log_off) {
            size_t want = (size_t)h_lats[0].V2 * n_metro;
            if (log_used + want <= log_cap) {
              lp = log.as<uint8_t>() + log_used;
              log_used += want;
            }
          }
          U1_TRY(timed_class_pass(kMetropolis, mu, p, th_frozen, n_metro, lp));
        }
      // the pass ids advance once per sweep with Metropolis hits: by the last
      // OR pass (which reads none of them), else by a kernel of its own
      if (n_or == 0) U1_HIP(launch_bump_pass_ids(pass_ids.as<uint64_t>(), n_lats, stream));
      for (auto& v : h_pass_ids) v += 1;
    }
    for (int k = 0; k < n_or; ++k)
      for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p) {
          const bool last = n_metro > 0 && k == n_or - 1 && mu == 3 && p == 1;
          U1_TRY(timed_class_pass(kOverrelax, mu, p, th_frozen, 0, nullptr, last ? n_lats : 0));
        }
    return U1ML_OK;
  }

  // Run fn, or replay the graph captured for key.  The first call runs fn
  // eagerly (allocating whatever it needs) and then captures a second copy
  // of the same launch sequence for later calls.
  template <class Fn>
  int run_captured(const std::vector<long long>& key, Fn fn, bool capture = true) {
    const bool can = capture && use_graphs && !debug && !prof[0] && !prof[1] && !fam_prof;
    ++epoch;
    if (can) {
      auto it = graphs.find(key);
      if (it != graphs.end()) {
        U1_HIP(hipGraphLaunch(it->second.exec, stream));
        for (auto& v : h_pass_ids) v += it->second.metro_passes;
        return U1ML_OK;
      }
    }
    U1_TRY(fn());
    if (!can) return U1ML_OK;
    if (graphs.size() >= kMaxGraphs) drop_graphs();
    const std::vector<uint64_t> ids = h_pass_ids;
    hipGraph_t g;
    U1_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    capturing = true;
    int rc = fn();
    capturing = false;
    hipError_t ce = hipStreamEndCapture(stream, &g);
    const int passes = (int)(h_pass_ids[0] - ids[0]);
    h_pass_ids = ids;  // capturing ran nothing
    if (rc) {
      if (ce == hipSuccess) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ce != hipSuccess) return fail(U1ML_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
    GraphEntry ge;
    hipError_t ie = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(U1ML_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
    ge.metro_passes = passes;
    graphs[key] = ge;
    return U1ML_OK;
  }

  int init_links(int hot) {
    ++epoch;
    std::vector<int> items;
    for (auto& d : h_lats) items.push_back(8 * d.V2);
    Table* t;
    U1_TRY(table(items, 256, &t));
    hipError_t e = prec == U1ML_FP64 ? launch_init_f64(links.as<double>(), lats.as<LatDesc>(), bt(t), hot, stream)
                                     : launch_init_f32(links.as<float>(), lats.as<LatDesc>(), bt(t), hot, stream);
    U1_HIP(e);
    return U1ML_OK;
  }

  int upload_pass_ids() {
    U1_TRY(copy(pass_ids.p, h_pass_ids.data(), n_lats * sizeof(uint64_t), hipMemcpyHostToDevice));
    return U1ML_OK;
  }

  int upload_lats() {
    ++epoch;  // beta enters the field observables
    U1_TRY(copy(lats.p, h_lats.data(), n_lats * sizeof(LatDesc), hipMemcpyHostToDevice));
    drop_graphs();  // single-lattice kernels take the descriptor by value
    return U1ML_OK;
  }

  // --- host <-> device link transfer (natural order theta[t][z][y][x][mu]) ---
  static size_t natural_of(const LatDesc& d, int p, uint32_t h) {
    const int Lh = d.L / 2;
    uint32_t q = h / Lh, xh = h % Lh;
    int y = q % d.L;
    q /= d.L;
    int z = q % d.L;
    int t = q / d.L;
    int b = (p ^ (t + z + y)) & 1;
    int x = 2 * xh + b;
    return (((size_t)t * d.L + z) * d.L + y) * d.L + x;
  }

  int get_links(int i, double* host) {
    const LatDesc& d = h_lats[i];
    const size_t n = 8ull * d.V2;
    std::vector<char> raw(n * elem_size());
    U1_TRY(copy(raw.data(), links.as<char>() + d.off * elem_size(), raw.size(), hipMemcpyDeviceToHost));
    for (int mu = 0; mu < 4; ++mu)
      for (int p = 0; p < 2; ++p)
        for (uint32_t h = 0; h < (uint32_t)d.V2; ++h) {
          size_t src = ((size_t)(mu * 2 + p)) * d.V2 + h;
          double v = prec == U1ML_FP64 ? ((double*)raw.data())[src] : (double)((float*)raw.data())[src];
          host[natural_of(d, p, h) * 4 + mu] = v;
        }
    return U1ML_OK;
  }

  int set_links(int i, const double* host) {
    ++epoch;
    const LatDesc& d = h_lats[i];
    const size_t n = 8ull * d.V2;
    for (size_t k = 0; k < n; ++k)
      if (!(std::fabs(host[k]) <= kMaxAngle))
        return fail(U1ML_EINVAL, "set_links: angles must be finite, |theta| <= 64");
    std::vector<char> raw(n * elem_size());
    for (int mu = 0; mu < 4; ++mu)
      for (int p = 0; p < 2; ++p)
        for (uint32_t h = 0; h < (uint32_t)d.V2; ++h) {
          size_t dst = ((size_t)(mu * 2 + p)) * d.V2 + h;
          double v = host[natural_of(d, p, h) * 4 + mu];
          if (prec == U1ML_FP64)
            ((double*)raw.data())[dst] = v;
          else
            ((float*)raw.data())[dst] = (float)v;
        }
    U1_TRY(copy(links.as<char>() + d.off * elem_size(), raw.data(), raw.size(), hipMemcpyHostToDevice));
    return U1ML_OK;
  }

  // --- plain observables of every lattice ---
  int observables(std::vector<u1ml_observables>& res) {
    if (obs_epoch == epoch) {
      res = obs_cache;
      return U1ML_OK;
    }
    std::vector<int> items;
    for (auto& d : h_lats) items.push_back(2 * d.V2);
    Table* t;
    U1_TRY(table(items, 256, &t));
    const int W = kPlaqFieldWidth;
    U1_TRY(partial.ensure((size_t)t->n_blocks * W * sizeof(double)));
    U1_TRY(row_begin.ensure((n_lats + 1) * sizeof(int)));
    U1_TRY(red_out.ensure((size_t)n_lats * W * sizeof(double)));
    U1_TRY(copy(row_begin.p, t->lat_block_begin.data(), (n_lats + 1) * sizeof(int), hipMemcpyHostToDevice));
    U1_HIP(launch_plaq_field(prec, links.p, lats.as<LatDesc>(), bt(t), partial.as<double>(), stream));
    U1_HIP(launch_reduce_rows(partial.as<double>(), W, row_begin.as<int>(), n_lats, red_out.as<double>(), stream));
    std::vector<double> pf((size_t)n_lats * W);
    U1_TRY(copy(pf.data(), red_out.p, pf.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<std::vector<double>> pc;
    U1_TRY(poly_corr(std::vector<int>(), pc));
    res.resize(n_lats);
    for (int i = 0; i < n_lats; ++i) {
      const double V = 2.0 * h_lats[i].V2;
      res[i].plaquette = pf[i * W] / (6.0 * V);
      for (int c = 0; c < 6; ++c) {
        res[i].field_mean[c] = pf[i * W + 1 + c] / V;
        res[i].field2_mean[c] = pf[i * W + 7 + c] / V;
      }
      res[i].poly_re = pc[i][0];
      res[i].poly_im = pc[i][1];
      res[i].poly_abs = std::hypot(pc[i][0], pc[i][1]);
    }
    obs_cache = res;
    obs_epoch = epoch;
    return U1ML_OK;
  }

  // Polyakov loop average and plain correlator of every lattice (same r list):
  // out[lat] = {Re P, Im P, Re C(r_0), Im C(r_0), ...}
  int poly_corr(const std::vector<int>& r_list, std::vector<std::vector<double>>& out) {
    std::vector<int> items, rb{0};
    std::vector<uint64_t> offs;
    uint64_t o = 0;
    for (auto& d : h_lats) {
      items.push_back(d.L3);
      offs.push_back(o);
      o += d.L3;
      rb.push_back(rb.back() + d.L3);
    }
    Table* t;
    U1_TRY(table(items, 256, &t));
    const int nR = (int)r_list.size();
    const int width = 2 + 2 * nR;
    U1_TRY(poly.ensure(o * sizeof(double)));
    U1_TRY(poly_off.ensure(offs.size() * sizeof(uint64_t)));
    U1_TRY(rows.ensure(o * width * sizeof(double)));
    U1_TRY(row_begin.ensure(rb.size() * sizeof(int)));
    U1_TRY(rvals_tmp.ensure(std::max(nR, 1) * sizeof(int)));
    U1_TRY(red_out.ensure((size_t)n_lats * width * sizeof(double)));
    U1_TRY(copy(poly_off.p, offs.data(), offs.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
    U1_TRY(copy(row_begin.p, rb.data(), rb.size() * sizeof(int), hipMemcpyHostToDevice));
    if (nR) U1_TRY(copy(rvals_tmp.p, r_list.data(), nR * sizeof(int), hipMemcpyHostToDevice));
    U1_HIP(launch_poly_lines(prec, links.p, lats.as<LatDesc>(), bt(t), poly_off.as<uint64_t>(), poly.as<double>(),
                             stream));
    U1_HIP(launch_poly_corr(lats.as<LatDesc>(), bt(t), poly_off.as<uint64_t>(), poly.as<double>(),
                            rvals_tmp.as<int>(), nR, row_begin.as<int>(), rows.as<double>(), stream));
    U1_HIP(launch_reduce_rows(rows.as<double>(), width, row_begin.as<int>(), n_lats, red_out.as<double>(), stream));
    std::vector<double> h((size_t)n_lats * width);
    U1_TRY(copy(h.data(), red_out.p, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    out.assign(n_lats, std::vector<double>(width));
    for (int i = 0; i < n_lats; ++i)
      for (int c = 0; c < width; ++c) out[i][c] = h[(size_t)i * width + c] / (double)h_lats[i].L3;
    return U1ML_OK;
  }

  // --- multilevel (Sec. 2.2) ---
  // Allocate and describe the workspace; rl[i] = r list of lattice i; rf =
  // field separations (shared; each in every r list).
  int ml_setup(int n_levels, const int* th, const int* n_sub, int n_metro, int n_or,
               const std::vector<std::vector<int>>& rl, const std::vector<int>& rf) {
    MLState& m = *mlp;
    U1_HIP(hipStreamSynchronize(stream));  // buffers below may still be in use
    if (!arena) drop_graphs();             // captured sequences hold the old buffer addresses
    m.key.clear();
    m.valid = m.field_valid = false;
    m.n_levels = n_levels;
    for (int l = 0; l < n_levels; ++l) {
      m.th[l] = th[l];
      m.n[l] = n_sub[l];
    }
    m.n_metro = n_metro;
    m.n_or = n_or;
    m.field = !rf.empty();
    const int inner = n_levels - 1;
    const int n_outer = n_levels == 2 ? n_sub[0] : 1;
    // bytes of stored samples if every outer iteration is kept
    size_t store_all = 0;
    if (m.field && n_levels == 2)
      for (auto& d : h_lats) {
        const size_t ns_in = d.T / th[inner];
        const size_t lines = (estimator & U1ML_MULTIHIT) ? 2 : 1;
        store_all += (size_t)n_outer * n_sub[inner] * ns_in * d.L3 * (6 * elem_size() + lines * sizeof(double2));
      }
    bool too_big = false;
    if (store_all > 0) {
      size_t free_b = 0, total_b = 0;
      U1_HIP(hipMemGetInfo(&free_b, &total_b));
      // buffers of the previous layout are reused or freed by this one
      const size_t avail = free_b + m.fbuf.bytes + m.mlbuf.bytes;
      too_big = (double)store_all > kFieldStoreFraction * (double)avail;
    }
    m.replay = m.field && n_levels == 2 && (force_replay || too_big);
    const int n_stored = m.replay ? 1 : n_outer;
    const int n_samples_kept = m.field ? n_stored * n_sub[inner] : n_sub[inner];
    m.h_mls.assign(n_lats, MLDesc{});
    m.nR.assign(n_lats, 0);
    std::vector<int> rv;
    uint64_t ell = 0, acc = 0;
    m.max_r = 0;
    for (int i = 0; i < n_lats; ++i) {
      const LatDesc& d = h_lats[i];
      MLDesc& md = m.h_mls[i];
      md.n_r = (int)rl[i].size();
      md.n_axes = (estimator & U1ML_SYMMETRIC) ? 3 : 1;
      md.nR = md.n_axes * md.n_r;
      md.r_off = (int)rv.size();
      for (int a = 0; a < md.n_axes; ++a)
        for (int r : rl[i]) rv.push_back(r | a << kRAxisShift);
      m.nR[i] = md.n_r;
      m.max_r = std::max(m.max_r, md.n_r);
      for (int l = 0; l < n_levels; ++l) md.ns[l] = d.T / th[l];
      md.ell = ell;
      ell += (uint64_t)n_samples_kept * md.ns[inner] * d.L3;
      md.multihit = (estimator & U1ML_MULTIHIT) ? 1 : 0;
      md.ell_mh = md.ell;
      if (md.multihit) {
        md.ell_mh = ell;
        ell += (uint64_t)n_samples_kept * md.ns[inner] * d.L3;
      }
      for (int l = 0; l < n_levels; ++l) {
        md.acc[l] = acc;
        if (l < inner) acc += (uint64_t)md.ns[l] * d.L3 * md.nR;
      }
      md.acc[n_levels] = acc;
      acc += (uint64_t)d.L3 * md.nR;
    }
    m.acc_elems = acc;
    if (n_lats > 1) {
      PassTable* pt;
      U1_TRY(pass_table(0, &pt));
      for (int l = 0; l < n_levels; ++l) U1_TRY(pass_table(th[l], &pt));
    }
    U1_TRY(reserve(m.mls, n_lats * sizeof(MLDesc)));
    U1_TRY(reserve(m.rvals, rv.size() * sizeof(int)));
    U1_TRY(reserve(m.mlbuf, ell * sizeof(double2)));
    U1_TRY(reserve(m.accbuf, acc * sizeof(double2)));
    U1_TRY(reserve(m.corr, (size_t)n_lats * m.max_r * 2 * sizeof(double)));
    U1_TRY(copy(m.mls.p, m.h_mls.data(), n_lats * sizeof(MLDesc), hipMemcpyHostToDevice));
    U1_TRY(copy(m.rvals.p, rv.data(), rv.size() * sizeof(int), hipMemcpyHostToDevice));
    if (m.field) {
      FieldParams& fp = m.fp;
      fp = FieldParams{};
      fp.n_rf = (int)rf.size();
      for (int f = 0; f < fp.n_rf; ++f) {
        fp.rf[f] = rf[f];
        fp.rf_k[f] = (int)(std::find(rl[0].begin(), rl[0].end(), rf[f]) - rl[0].begin());
      }
      fp.n_levels = n_levels;
      fp.n_outer = n_outer;
      fp.n_stored = n_stored;
      fp.n_inner = n_sub[inner];
      m.h_fls.assign(n_lats, FieldLat{});
      m.fout_off.assign(n_lats, 0);
      uint64_t fb = 0, fo = 0;
      size_t per_sample_max = 0;
      for (int i = 0; i < n_lats; ++i) {
        const LatDesc& d = h_lats[i];
        FieldLat& fl = m.h_fls[i];
        fl.ns = m.h_mls[i].ns[inner];
        const uint64_t L3 = d.L3, L2 = (uint64_t)d.L * d.L;
        fl.oall = fb;
        fb += ((uint64_t)n_samples_kept * 6 * fl.ns * L3 * elem_size() + sizeof(double) - 1) / sizeof(double);
        fl.tavg = fb;
        fb += 2ull * n_stored * fl.ns * L3 * fp.n_rf;
        fl.w = fb;
        fb += 2ull * n_stored * fl.ns * L3 * fp.n_rf;
        fl.g = fb;
        fb += 2ull * fp.n_rf * 12 * L2;
        fl.n_top = n_levels == 2 ? m.h_mls[i].ns[0] : 1;
        fl.ptop = fb;
        fb += 2ull * fl.n_top * fp.n_rf * L3;
        m.fout_off[i] = fo;
        fo += (uint64_t)fp.n_rf * 12 * L2;
        // contraction scratch: one sample's transformed planes plus the per-slab partial sums
        per_sample_max = std::max<size_t>(per_sample_max, (size_t)(fp.n_rf + 6) * fl.ns * L3 +
                                                              (size_t)fp.n_rf * fl.ns * 12 * L2);
      }
      m.scratch_elems = std::max(per_sample_max, kFieldScratchBytes / sizeof(double2));
      U1_TRY(reserve(m.fls, n_lats * sizeof(FieldLat)));
      U1_TRY(reserve(m.fbuf, fb * sizeof(double)));
      U1_TRY(reserve(m.fout, fo * sizeof(double2)));
      U1_TRY(reserve(m.scratch, m.scratch_elems * sizeof(double2)));
      U1_TRY(copy(m.fls.p, m.h_fls.data(), n_lats * sizeof(FieldLat), hipMemcpyHostToDevice));
    }
    return U1ML_OK;
  }

  int ml_fold(int child, int parent, int sample_base) {
    MLState& m = *mlp;
    const int inner = m.n_levels - 1;
    if (child == inner && !fold_general) {
      int threads = 64, max_nr = 1;
      const bool multihit = m.h_mls[0].multihit != 0;
      for (int i = 0; i < n_lats; ++i) {
        max_nr = std::max(max_nr, m.h_mls[i].n_r);
        if ((m.h_mls[i].multihit != 0) != multihit) return fail(U1ML_EINVAL, "mixed estimators in one run");
      }
      const int k_slots = ml_fold_rows_k(max_nr);
      size_t all_lds = 0, child_lds = 0;
      int items = 0;
      for (int i = 0; i < n_lats; ++i) {
        const int nsp = parent == m.n_levels ? 1 : m.h_mls[i].ns[parent];
        const int children = m.h_mls[i].ns[child] / nsp;
        threads = std::max(threads, fold_threads > 0 ? fold_threads
                                                     : ml_fold_rows_threads(h_lats[i].L, m.h_mls[i].n_r, k_slots));
        const size_t rows = (size_t)(multihit ? 2 : 1) * m.n[child] * h_lats[i].L * sizeof(double2);
        child_lds = std::max(child_lds, rows);
        all_lds = std::max(all_lds, children * rows);
        items = std::max(items, h_lats[i].L * ((m.h_mls[i].n_r + k_slots - 1) / k_slots));
      }
      // one child at a time where asked (or, by default, where all children
      // would take more than 16 KB of LDS per block and so limit the blocks
      // per CU) and one thread per item fits a block; all at once where the
      // other does not apply
      const size_t max_lds_ok = ml_fold_rows_max_lds();
      const int pc_threads = (items + 63) / 64 * 64;
      const bool pc_fits = pc_threads <= 256 && child_lds <= max_lds_ok;
      const bool want_pc = fold_stage == 2 || (fold_stage == 0 && all_lds > 16384);
      const bool per_child = pc_fits && (want_pc || all_lds > max_lds_ok);
      size_t max_lds = per_child ? child_lds : all_lds;
      if (per_child) {
        threads = std::max(threads, pc_threads);
        // two buffers and enough threads to hold one child's rows in
        // registers: the next child's rows load while one is folded
        const int np = ml_fold_rows_prefetch(multihit);
        const int vals = (int)(child_lds / sizeof(double2));
        const int pipe_threads = ((vals + np - 1) / np + 63) / 64 * 64;
        if (pipe_threads <= 256 && 2 * child_lds <= max_lds_ok) {
          threads = std::max(threads, pipe_threads);
          max_lds = 2 * child_lds;
        }
      }
      if (max_lds <= max_lds_ok) {
        std::vector<int> rows;
        for (int i = 0; i < n_lats; ++i) {
          const int nsp = parent == m.n_levels ? 1 : m.h_mls[i].ns[parent];
          rows.push_back(nsp * m.h_mls[i].n_axes * h_lats[i].L * h_lats[i].L);
        }
        Table* t;
        U1_TRY(table(rows, 1, &t));
        // two levels with the field stored: the fold also writes the inner
        // averages of the field separations of this outer iteration
        const int tavg_m = (m.field && m.store_field && !m.replay && m.n_levels == 2 && parent == 0)
                               ? sample_base / m.n[child]
                               : -1;
        U1_TRY(fam_begin(kFamFold));
        U1_HIP(launch_ml_fold_rows(lats.as<LatDesc>(), m.mls.as<MLDesc>(), bt(t), threads, max_lds, k_slots,
                                   multihit, per_child, child, parent, m.n_levels, m.n[child], sample_base, m.rvals.as<int>(), m.mlbuf.as<double2>(),
                                   m.accbuf.as<double2>(), m.fls.as<FieldLat>(), m.fp, tavg_m, m.fbuf.as<double>(),
                                   stream));
        return fam_end(kFamFold);
      }
    }
    if (child == inner) m.tavg_from_fold = false;
    std::vector<int> it;
    for (int i = 0; i < n_lats; ++i) {
      int nsp = parent == m.n_levels ? 1 : m.h_mls[i].ns[parent];
      it.push_back(nsp * h_lats[i].L3 * ((m.h_mls[i].nR + 7) / 8));  // blocks of 8 separations
    }
    Table* t;
    U1_TRY(table(it, 256, &t));
    U1_HIP(launch_ml_fold(lats.as<LatDesc>(), m.mls.as<MLDesc>(), bt(t), child, parent, m.n_levels, child == inner,
                          m.n[child], sample_base, m.rvals.as<int>(), m.mlbuf.as<double2>(), m.accbuf.as<double2>(),
                          stream));
    return U1ML_OK;
  }

  int ml_sample(int sample) {
    MLState& m = *mlp;
    const int inner = m.n_levels - 1;
    std::vector<int> it;
    for (int i = 0; i < n_lats; ++i) it.push_back(m.h_mls[i].ns[inner] * h_lats[i].L3);
    Table* t;
    U1_TRY(table(it, sample_block, &t));
    U1_TRY(fam_begin(kFamSample));
    U1_HIP(launch_ml_sample(prec, links.p, lats.as<LatDesc>(), m.mls.as<MLDesc>(), m.fls.as<FieldLat>(), bt(t),
                            m.th[inner], sample, m.field && m.store_field, (estimator & U1ML_FIELD_SQUARED) != 0,
                            m.mlbuf.as<double2>(), m.fbuf.as<double>(), stream));
    return fam_end(kFamSample);
  }

  // n[l] iterations of: update with level l frozen, then measure (innermost)
  // or recurse and fold the inner averages into level l.
  int ml_level(int l, int outer_it) {
    MLState& m = *mlp;
    const int inner = m.n_levels - 1;
    for (int it = 0; it < m.n[l]; ++it) {
      U1_TRY(sweep(m.n_metro, m.n_or, m.th[l]));
      const int mo = l == 0 ? it : outer_it;
      // samples of every outer iteration are kept for the field contraction,
      // unless the run is replayed
      const bool keep = m.field && !m.replay;
      if (l == inner) {
        const int base = (keep && m.n_levels == 2) ? outer_it * m.n[inner] : 0;
        U1_TRY(ml_sample(base + it));
      } else {
        U1_TRY(ml_level(l + 1, mo));
        const int base = (keep && l + 1 == inner) ? mo * m.n[inner] : 0;
        U1_TRY(ml_fold(l + 1, l, base));
      }
    }
    return U1ML_OK;
  }

  int field_contract(bool zero_g, bool finalize) {
    MLState& m = *mlp;
    U1_TRY(fam_begin(kFamField));
    for (int i = 0; i < n_lats; ++i)
      U1_HIP(launch_field_contract(lats.as<LatDesc>() + i, m.mls.as<MLDesc>() + i, m.fls.as<FieldLat>() + i,
                                   m.h_fls[i], m.fp, h_lats[i].L, m.mlbuf.as<double2>(), m.accbuf.as<double2>(),
                                   m.fbuf.as<double>(), m.scratch.as<double2>(), m.scratch_elems,
                                   m.fout.as<double2>() + m.fout_off[i], field_general, prec == U1ML_FP32, zero_g,
                                   finalize, m.tavg_from_fold, ftune, stream));
    return fam_end(kFamField);
  }

  // event pair around the launches of one kernel family (autotuner timing)
  int fam_begin(int fam) {
    if (!fam_prof || fam != fam_id) return U1ML_OK;
    hipEvent_t a, z;
    U1_HIP(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&z);
    if (e != hipSuccess) {
      (void)hipEventDestroy(a);
      U1_HIP(e);
    }
    fam_prof->push_back(std::make_pair(a, z));
    U1_HIP(hipEventRecord(a, stream));
    return U1ML_OK;
  }
  int fam_end(int fam) {
    if (!fam_prof || fam != fam_id) return U1ML_OK;
    U1_HIP(hipEventRecord(fam_prof->back().second, stream));
    return U1ML_OK;
  }

  // Two-level run with field insertion in two passes over the same update
  // sequence: the first folds the correlator averages (the weights of every
  // insertion need the final top-level averages), the second, from the
  // restored links and pass ids, contracts each outer iteration's samples
  // with those weights as soon as the iteration completes.
  int ml_run_replay() {
    MLState& m = *mlp;
    const size_t lb = link_elems * elem_size(), pb = n_lats * sizeof(uint64_t);
    U1_TRY(m.links_backup.ensure(lb));
    U1_TRY(m.pass_backup.ensure(pb));
    U1_HIP(hipMemcpyAsync(m.links_backup.p, links.p, lb, hipMemcpyDeviceToDevice, stream));
    U1_HIP(hipMemcpyAsync(m.pass_backup.p, pass_ids.p, pb, hipMemcpyDeviceToDevice, stream));
    const std::vector<uint64_t> ids = h_pass_ids;
    m.store_field = false;
    const int rc = ml_level(0, 0);
    m.store_field = true;
    U1_TRY(rc);
    U1_HIP(hipMemcpyAsync(links.p, m.links_backup.p, lb, hipMemcpyDeviceToDevice, stream));
    U1_HIP(hipMemcpyAsync(pass_ids.p, m.pass_backup.p, pb, hipMemcpyDeviceToDevice, stream));
    h_pass_ids = ids;
    log_off = true;  // the accept log holds the first pass
    for (int it = 0; it < m.n[0] && !rc; ++it) {
      int r2 = sweep(m.n_metro, m.n_or, m.th[0]);
      for (int i = 0; i < m.n[1] && !r2; ++i) {
        r2 = sweep(m.n_metro, m.n_or, m.th[1]);
        if (!r2) r2 = ml_sample(i);
      }
      if (!r2) r2 = field_contract(it == 0, it == m.n[0] - 1);
      if (r2) {
        log_off = false;
        return r2;
      }
    }
    log_off = false;
    return U1ML_OK;
  }

  // full multilevel run, results in ml.corr (and ml.fout)
  int ml_run() {
    MLState& m = *mlp;
    // the inner folds of a stored two-level field run write the field inner
    // averages, unless one of them takes the per-site fold (which clears this)
    m.tavg_from_fold = m.field && !m.replay && m.n_levels == 2;
    U1_HIP(launch_ml_zero(m.accbuf.as<double2>(), m.acc_elems, stream));
    if (m.replay) {
      U1_TRY(ml_run_replay());
    } else {
      U1_TRY(ml_level(0, 0));
      // the weights need the top-level averages: contract before the top fold
      if (m.field) U1_TRY(field_contract(true, true));
    }
    U1_TRY(ml_fold(0, m.n_levels, 0));
    U1_HIP(launch_ml_final(lats.as<LatDesc>(), m.mls.as<MLDesc>(), n_lats, m.max_r, m.n_levels,
                           m.accbuf.as<double2>(), m.corr.as<double>(), stream));
    return U1ML_OK;
  }

  // --- ensemble of multilevel runs (Eq. (7)) ---
  void ensemble_reset() {
    ens.n = 0;
    ens.shape.clear();
  }

  // adds the last run's correlator and field profile and the current links'
  // means of the inserted operator set; asynchronous after the first call
  int ensemble_add() {
    if (!ml.valid) return fail(U1ML_ESTATE, "no multilevel result to add");
    if (ens.n > 0 && ens.shape != ml.shape)
      return fail(U1ML_EINVAL, "the ensemble holds runs of another shape; reset it first");
    const int W = kPlaqFieldWidth;
    std::vector<int> items;
    for (auto& d : h_lats) items.push_back(2 * d.V2);
    Table* t;
    U1_TRY(table(items, 256, &t));
    if (ens.n == 0) {
      ens.shape = ml.shape;
      ens.flags = ml.run_flags;
      ens.max_r = ml.max_r;
      ens.nR = ml.nR;
      ens.field = ml.field_valid;
      ens.fp = ml.fp;
      ens.fout_off = ml.fout_off;
      ens.fout_elems = 0;
      size_t conn_elems = 0;
      if (ens.field)
        for (int i = 0; i < n_lats; ++i) {
          const uint64_t n = (uint64_t)ens.fp.n_rf * 12 * h_lats[i].L * h_lats[i].L;
          ens.fout_elems = std::max<uint64_t>(ens.fout_elems, ens.fout_off[i] + n);
          conn_elems = std::max<size_t>(conn_elems, n);
        }
      U1_TRY(ens.corr.ensure((size_t)n_lats * ens.max_r * sizeof(double2)));
      U1_TRY(ens.fsum.ensure(ens.fout_elems * sizeof(double2)));
      U1_TRY(ens.conn.ensure(conn_elems * sizeof(double2)));
      U1_TRY(ens.omean.ensure((size_t)n_lats * 6 * sizeof(double)));
      U1_TRY(ens.partial.ensure((size_t)t->n_blocks * W * sizeof(double)));
      U1_TRY(ens.red.ensure((size_t)n_lats * W * sizeof(double)));
      U1_TRY(ens.row_begin.ensure((n_lats + 1) * sizeof(int)));
      U1_TRY(copy(ens.row_begin.p, t->lat_block_begin.data(), (n_lats + 1) * sizeof(int), hipMemcpyHostToDevice));
      // cleared by kernels, not memset nodes, in case the caller captures the stream
      U1_HIP(launch_ml_zero(ens.corr.as<double2>(), (uint64_t)n_lats * ens.max_r, stream));
      U1_HIP(launch_ml_zero(ens.fsum.as<double2>(), ens.fout_elems, stream));
      U1_HIP(launch_ml_zero(ens.omean.as<double2>(), (uint64_t)n_lats * 3, stream));
    }
    U1_HIP(launch_ens_add(ens.corr.as<double>(), ml.corr.as<double>(), (uint64_t)n_lats * ens.max_r * 2, stream));
    if (ens.field)
      U1_HIP(launch_ens_add(ens.fsum.as<double>(), ml.fout.as<double>(), ens.fout_elems * 2, stream));
    U1_HIP(launch_plaq_field(prec, links.p, lats.as<LatDesc>(), bt(t), ens.partial.as<double>(), stream));
    U1_HIP(launch_reduce_rows(ens.partial.as<double>(), W, ens.row_begin.as<int>(), n_lats, ens.red.as<double>(),
                              stream));
    U1_HIP(launch_ens_omean(lats.as<LatDesc>(), ens.red.as<double>(), W, (ens.flags & U1ML_FIELD_SQUARED) ? 7 : 1,
                            n_lats, ens.omean.as<double>(), stream));
    ++ens.n;
    return U1ML_OK;
  }

  int ensemble_read(int i, double* correlator, double* field_profile, double* connected) {
    if (ens.n == 0) return fail(U1ML_ESTATE, "the ensemble is empty");
    if ((field_profile || connected) && !ens.field) return fail(U1ML_ESTATE, "the ensemble's runs had no field");
    const double inv = 1.0 / (double)ens.n;
    const int L = h_lats[i].L;
    const size_t nf = (size_t)ens.fp.n_rf * 12 * L * L;
    if (connected)
      U1_HIP(launch_ens_connected(ens.fsum.as<double2>() + ens.fout_off[i], ens.corr.as<double2>() + (size_t)i * ens.max_r,
                                  ens.omean.as<double>() + 6 * i, ens.fp, L, inv, ens.conn.as<double2>(), stream));
    U1_HIP(hipStreamSynchronize(stream));
    if (correlator) {
      U1_TRY(copy(correlator, ens.corr.as<double2>() + (size_t)i * ens.max_r, ens.nR[i] * sizeof(double2),
                  hipMemcpyDeviceToHost));
      for (int k = 0; k < 2 * ens.nR[i]; ++k) correlator[k] *= inv;
    }
    if (field_profile) {
      U1_TRY(copy(field_profile, ens.fsum.as<double2>() + ens.fout_off[i], nf * sizeof(double2),
                  hipMemcpyDeviceToHost));
      for (size_t k = 0; k < 2 * nf; ++k) field_profile[k] *= inv;
    }
    if (connected)
      U1_TRY(copy(connected, ens.conn.p, nf * sizeof(double2), hipMemcpyDeviceToHost));
    return U1ML_OK;
  }

  // n_sweeps_before unfrozen compound sweeps, then a multilevel run
  int multilevel(int n_levels, const int* th, const int* n_sub, int n_metro, int n_or,
                 const std::vector<std::vector<int>>& rl, const std::vector<int>& rf, int n_sweeps_before) {
    std::vector<long long> key{1, n_levels, n_metro, n_or, n_sweeps_before, (long long)rf.size(), (long long)estimator};
    for (int l = 0; l < n_levels; ++l) {
      key.push_back(th[l]);
      key.push_back(n_sub[l]);
    }
    for (auto& v : rl) {
      key.push_back(-(long long)v.size());
      for (int r : v) key.push_back(r);
    }
    for (int r : rf) key.push_back(r);
    if (ml.key != key) {
      U1_TRY(ml_setup(n_levels, th, n_sub, n_metro, n_or, rl, rf));
      ml.key = key;
    }
    ml.valid = ml.field_valid = false;
    // compound sweeps of the run: sum over levels of the product of n_sub
    long long n_updates = n_sweeps_before, prod = 1;
    for (int l = 0; l < n_levels; ++l) {
      prod *= n_sub[l];
      n_updates += prod;
    }
    U1_TRY(run_captured(
        key,
        [&]() -> int {
          for (int s = 0; s < n_sweeps_before; ++s) U1_TRY(sweep(n_metro, n_or, 0));
          return ml_run();
        },
        n_updates <= kMaxCapturedUpdates));
    ml.valid = true;
    ml.field_valid = ml.field;
    ml.shape.assign(1, ml.field ? 1 : 0);
    ml.shape.push_back((estimator & U1ML_FIELD_SQUARED) ? 1 : 0);
    ml.shape.push_back((estimator & U1ML_SYMMETRIC) ? 1 : 0);
    for (auto& v : rl) {
      ml.shape.push_back(-(long long)v.size());
      for (int r : v) ml.shape.push_back(r);
    }
    for (int r : rf) ml.shape.push_back(r);
    ml.run_flags = estimator;
    return U1ML_OK;
  }

  // The multilevel run of multilevel() (no field, no preceding sweeps) with
  // its whole workspace carved from the device range [base, base + cap) and
  // the correlator written to the caller's device buffer out [n_r][2];
  // kernel by kernel, nothing allocated on the device and no graph made.
  // ml (the results kept for u1ml_measure) and the captured graphs are left
  // as they are.
  int multilevel_in_place(int n_levels, const int* th, const int* n_sub, int n_metro, int n_or,
                          const std::vector<int>& rl, void* base, size_t cap, double* out) {
    Arena ar;
    ar.base = (char*)base;
    ar.cap = cap;
    MLState st;
    arena = &ar;
    mlp = &st;
    int rc = ml_setup(n_levels, th, n_sub, n_metro, n_or, std::vector<std::vector<int>>(1, rl), {});
    if (!rc) {
      // the final kernel writes C(r) straight into the caller's buffer
      st.corr.p = out;
      st.corr.bytes = rl.size() * 2 * sizeof(double);
      ++epoch;
      rc = ml_run();
    }
    if (!rc) {
      hipError_t e = hipStreamSynchronize(stream);  // the arena tables are freed on the host below
      if (e != hipSuccess) rc = fail(U1ML_EDEVICE, std::string("multilevel_noalloc: ") + hipGetErrorString(e));
    }
    arena = nullptr;
    mlp = &ml;
    arena_tables.clear();
    return rc;
  }
};

struct u1ml_lattice {
  Engine e;
};
struct u1ml_batch {
  Engine e;
};

namespace {

// ---------------------------------------------------------------------------
// Static workspace of u1ml_multilevel_noalloc: one fixed array per GPU, held
// by every device the library runs on until the process ends.  Host code
// never passes the array's name to a kernel: the name is a host-side stand-in
// in host code, so the device address of each GPU's copy is looked up once
// per device (with that device current) and kept.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = (size_t)U1ML_NOALLOC_BYTES;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// once per device, with that device current (called from engine_create)
int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(U1ML_EDEVICE, "device index beyond the static workspace table");
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (g_scratch_ptr[device]) return U1ML_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(U1ML_EDEVICE, std::string("static workspace address: ") + hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return U1ML_OK;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  return g_scratch_ptr[device];
}

// block sizes found by u1ml_autotune, shared by every handle created later
// in the process: (L, T, precision) -> block
std::mutex g_tuned_mutex;
std::map<std::tuple<int, int, int>, int> g_tuned_block;

int tuned_block(int L, int T, int prec, int fallback) {
  std::lock_guard<std::mutex> lk(g_tuned_mutex);
  auto it = g_tuned_block.find(std::make_tuple(L, T, prec));
  return it != g_tuned_block.end() ? it->second : fallback;
}

void set_tuned_block(int L, int T, int prec, int block) {
  std::lock_guard<std::mutex> lk(g_tuned_mutex);
  g_tuned_block[std::make_tuple(L, T, prec)] = block;
}

// Metropolis hits per link of one pass: the hit index is a byte of the
// random-number counter
int check_hits(int n_metro, int n_or) {
  if (n_metro < 0 || n_metro > U1ML_MAX_HITS || n_or < 0)
    return fail(U1ML_EINVAL, "need 0 <= n_metro <= 255 and n_or >= 0");
  return U1ML_OK;
}

int validate_size(int L, int T) {
  if (L < 2 || T < 2 || (L & 1) || (T & 1) || L > 256 || T > 256)
    return fail(U1ML_EINVAL, "L and T must be even and in [2, 256]");
  const uint64_t V = (uint64_t)L * L * L * T;
  // 32-bit site arithmetic: the quotient tricks need V L < 2^32
  if (V * (uint64_t)L >= (1ull << 32) || 4 * V >= (1ull << 31)) return fail(U1ML_EINVAL, "lattice too large");
  return U1ML_OK;
}

LatDesc make_desc(int L, int T, double beta, double eps, uint64_t seed, uint64_t off) {
  LatDesc d{};
  d.L = L;
  d.T = T;
  d.V2 = L * L * L * T / 2;
  d.L3 = L * L * L;
  d.div_Lh = make_fastdiv((uint32_t)(L / 2));
  d.div_L = make_fastdiv((uint32_t)L);
  d.div_slice = make_fastdiv((uint32_t)(L * L * L / 2));
  d.beta = beta;
  d.eps = eps;
  d.sqrt_beta = std::sqrt(beta);
  d.seed = seed;
  d.off = off;
  return d;
}

int engine_create(Engine& e, const std::vector<int>& L, const std::vector<int>& T, const std::vector<double>& beta,
                  const std::vector<uint64_t>& seed, const u1ml_options* opt, bool allow_dev_buf) {
  u1ml_options o;
  u1ml_default_options(&o);
  if (opt) o = *opt;
  if (o.precision != U1ML_FP64 && o.precision != U1ML_FP32) return fail(U1ML_EINVAL, "precision");
  if (o.start != U1ML_COLD && o.start != U1ML_HOT) return fail(U1ML_EINVAL, "start");
  if (!(o.eps >= 0 && o.eps <= kMaxEps)) return fail(U1ML_EINVAL, "eps must be in [0, 2 pi]");
  if (o.block != 0 && (o.block < 64 || o.block > 1024 || (o.block % 64)))
    return fail(U1ML_EINVAL, "block must be a multiple of 64 in [64, 1024]");
  const int n = (int)L.size();
  uint64_t off = 0;
  for (int i = 0; i < n; ++i) {
    U1_TRY(validate_size(L[i], T[i]));
    if (!std::isfinite(beta[i]) || beta[i] < 0) return fail(U1ML_EINVAL, "beta must be finite and >= 0");
    e.h_lats.push_back(make_desc(L[i], T[i], beta[i], o.eps, seed[i], off));
    off += 4ull * L[i] * L[i] * L[i] * T[i];
  }
  U1_HIP(hipGetDevice(&e.device));
  U1_TRY(scratch_setup(e.device));
  e.stream = (hipStream_t)o.stream;
  if (!e.stream) {
    // a stream of our own (default priority) so that graph capture is possible
    U1_HIP(hipStreamCreateWithFlags(&e.stream, hipStreamNonBlocking));
    e.own_stream = true;
  }
  e.use_graphs = o.no_graphs == 0;
  e.prec = o.precision;
  e.n_lats = n;
  e.link_elems = off;
  e.block = o.block ? o.block : tuned_block(L[0], T[0], o.precision, 256);
  if (allow_dev_buf && o.dev_buf) {
    if (o.dev_bytes < off * e.elem_size()) return fail(U1ML_EINVAL, "dev_buf smaller than u1ml_link_bytes");
    e.links.p = o.dev_buf;
    e.links.bytes = o.dev_bytes;
    e.links.owned = false;
  } else {
    U1_TRY(e.links.ensure(off * e.elem_size()));
  }
  U1_TRY(e.lats.ensure(n * sizeof(LatDesc)));
  U1_TRY(e.upload_lats());
  U1_TRY(e.pass_ids.ensure(n * sizeof(uint64_t)));
  e.h_pass_ids.assign(n, 0);
  U1_TRY(e.upload_pass_ids());
  U1_TRY(e.init_links(o.start == U1ML_HOT));
  U1_HIP(hipStreamSynchronize(e.stream));
  return U1ML_OK;
}

int check_ml_args(const Engine& e, int n_levels, const int* th, const int* n_sub, int n_metro, int n_or) {
  if (n_levels < 1 || n_levels > U1ML_MAX_LEVELS || !th || !n_sub) return fail(U1ML_EINVAL, "multilevel arguments");
  U1_TRY(check_hits(n_metro, n_or));
  for (int l = 0; l < n_levels; ++l) {
    if (th[l] < 1 || n_sub[l] < 1) return fail(U1ML_EINVAL, "slab sizes and n_sub must be >= 1");
    if (l > 0 && th[l - 1] % th[l]) return fail(U1ML_EINVAL, "each slab size must divide the previous one");
    for (auto& d : e.h_lats)
      if (d.T % th[l]) return fail(U1ML_EINVAL, "slab sizes must divide T");
  }
  return U1ML_OK;
}

// shared argument checks of u1ml_multilevel / u1ml_batch_multilevel
int ml_entry(Engine& e, int n_levels, const int* th, const int* n_sub, int n_metro, int n_or, int n_r,
             const int* r_list, int n_rf, const int* rf_list) {
  U1_TRY(check_ml_args(e, n_levels, th, n_sub, n_metro, n_or));
  if (n_r < 1 || !r_list) return fail(U1ML_EINVAL, "need at least one r");
  if (n_rf < 0 || n_rf > U1ML_MAX_FIELD_R || (n_rf > 0 && !rf_list)) return fail(U1ML_EINVAL, "field r list");
  if (n_rf > 0 && n_levels > 2) return fail(U1ML_EINVAL, "field insertion supports one or two levels");
  for (auto& d : e.h_lats)
    if (n_rf > 0 && d.L > kMaxFieldL) return fail(U1ML_EINVAL, "field insertion supports L <= 62");
  std::vector<int> rl(r_list, r_list + n_r), rf;
  for (int r : rl)
    for (auto& d : e.h_lats)
      if (r < 1 || r >= d.L) return fail(U1ML_EINVAL, "r must be in [1, L)");
  for (int f = 0; f < n_rf; ++f) {
    if (std::find(rl.begin(), rl.end(), rf_list[f]) == rl.end())
      return fail(U1ML_EINVAL, "every field r must appear in r_list");
    rf.push_back(rf_list[f]);
  }
  U1_TRY(e.set_device());
  return e.multilevel(n_levels, th, n_sub, n_metro, n_or, std::vector<std::vector<int>>(e.n_lats, rl), rf, 0);
}

int read_results(Engine& e, int i, u1ml_observables* obs, double* correlator, double* field_profile) {
  U1_TRY(e.set_device());
  if ((correlator && !e.ml.valid) || (field_profile && !e.ml.field_valid))
    return fail(U1ML_ESTATE, "no multilevel result of that kind yet");
  if (obs) {
    std::vector<u1ml_observables> res;
    U1_TRY(e.observables(res));
    *obs = res[i];
  }
  U1_HIP(hipStreamSynchronize(e.stream));
  if (correlator)
    U1_TRY(e.copy(correlator, e.ml.corr.as<double>() + (size_t)i * e.ml.max_r * 2, e.ml.nR[i] * 2 * sizeof(double),
                  hipMemcpyDeviceToHost));
  if (field_profile) {
    const int L = e.h_lats[i].L;
    U1_TRY(e.copy(field_profile, e.ml.fout.as<double2>() + e.ml.fout_off[i],
                  (size_t)e.ml.fp.n_rf * 12 * L * L * sizeof(double2), hipMemcpyDeviceToHost));
  }
  return U1ML_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void u1ml_default_options(u1ml_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->start = U1ML_HOT;
  opt->precision = U1ML_FP64;
  opt->eps = 1.0;
}

size_t u1ml_link_bytes(int L, int T, int precision) {
  if (L < 2 || T < 2 || (L & 1) || (T & 1) || (precision != U1ML_FP64 && precision != U1ML_FP32)) return 0;
  return (size_t)4 * L * L * L * T * (precision == U1ML_FP64 ? 8 : 4);
}

size_t u1ml_workspace_bytes(int L, int T, int precision, int n_levels, const int* slab_sizes, const int* n_sub,
                            int n_r, int n_rf, unsigned estimator) {
  if (L < 2 || T < 2 || (L & 1) || (T & 1) || (precision != U1ML_FP64 && precision != U1ML_FP32) || n_levels < 1 ||
      n_levels > U1ML_MAX_LEVELS || !slab_sizes ||
      !n_sub || n_r < 1 || n_rf < 0 || n_rf > U1ML_MAX_FIELD_R || (n_rf > 0 && n_levels > 2))
    return 0;
  for (int l = 0; l < n_levels; ++l)
    if (slab_sizes[l] < 1 || T % slab_sizes[l] || n_sub[l] < 1 || (l > 0 && slab_sizes[l - 1] % slab_sizes[l]))
      return 0;
  // the layout of the multilevel workspace (every inner sample kept when
  // the field is inserted), as the multilevel set-up allocates it
  const int inner = n_levels - 1;
  const int n_outer = n_levels == 2 ? n_sub[0] : 1;
  const uint64_t kept = n_rf > 0 ? (uint64_t)n_outer * n_sub[inner] : (uint64_t)n_sub[inner];
  const uint64_t L3 = (uint64_t)L * L * L, L2 = (uint64_t)L * L, ns_in = (uint64_t)(T / slab_sizes[inner]);
  const uint64_t nR = (uint64_t)((estimator & U1ML_SYMMETRIC) ? 3 : 1) * n_r;
  const uint64_t ell = kept * ns_in * L3 * ((estimator & U1ML_MULTIHIT) ? 2 : 1);
  uint64_t acc = L3 * nR;
  for (int l = 0; l < inner; ++l) acc += (uint64_t)(T / slab_sizes[l]) * L3 * nR;
  size_t bytes = (ell + acc) * sizeof(double2) + (size_t)n_r * 2 * sizeof(double);
  if (n_rf > 0) {
    const uint64_t n_top = n_levels == 2 ? (uint64_t)(T / slab_sizes[0]) : 1;
    const uint64_t esz = precision == U1ML_FP64 ? 8 : 4;  // stored field sums in the link precision
    const uint64_t fb = (kept * 6 * ns_in * L3 * esz + 7) / 8 + 4ull * n_outer * ns_in * L3 * n_rf +
                        2ull * n_rf * 12 * L2 + 2ull * n_top * n_rf * L3;
    const uint64_t per_sample = (uint64_t)(n_rf + 6) * ns_in * L3 + (uint64_t)n_rf * ns_in * 12 * L2;
    const uint64_t scratch = std::max<uint64_t>(per_sample, kFieldScratchBytes / sizeof(double2));
    bytes += fb * sizeof(double) + ((uint64_t)n_rf * 12 * L2 + scratch) * sizeof(double2);
  }
  return bytes;
}

size_t u1ml_device_bytes(const u1ml_lattice* lat) {
  if (!lat) return 0;
  const MLState& m = lat->e.ml;
  return m.mlbuf.bytes + m.accbuf.bytes + m.corr.bytes + m.fbuf.bytes + m.fout.bytes + m.scratch.bytes;
}

int u1ml_init_lattice(int L, int T, double beta, uint64_t seed, const u1ml_options* opt, u1ml_lattice** out) {
  if (!out) return fail(U1ML_EINVAL, "out is NULL");
  *out = nullptr;
  std::unique_ptr<u1ml_lattice> lat(new (std::nothrow) u1ml_lattice());
  if (!lat) return fail(U1ML_ENOMEM, "host allocation");
  U1_TRY(engine_create(lat->e, {L}, {T}, {beta}, {seed}, opt, true));
  *out = lat.release();
  return U1ML_OK;
}

int u1ml_sweep(u1ml_lattice* lat, int n_metro, int n_or) {
  U1_TRY(check_hits(n_metro, n_or));
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  Engine& e = lat->e;
  U1_TRY(e.set_device());
  return e.run_captured({0, n_metro, n_or}, [&]() { return e.sweep(n_metro, n_or, 0); });
}

int u1ml_multilevel(u1ml_lattice* lat, int n_levels, const int* slab_sizes, const int* n_sub, int n_metro, int n_or,
                    int n_r, const int* r_list, int n_rf, const int* rf_list) {
  U1_TRY(check_hits(n_metro, n_or));
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  return ml_entry(lat->e, n_levels, slab_sizes, n_sub, n_metro, n_or, n_r, r_list, n_rf, rf_list);
}

int u1ml_measure(u1ml_lattice* lat, u1ml_observables* obs, double* correlator, double* field_profile) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  return read_results(lat->e, 0, obs, correlator, field_profile);
}

int u1ml_multilevel_noalloc(u1ml_lattice* lat, int n_levels, const int* slab_sizes, const int* n_sub, int n_metro,
                            int n_or, int n_r, const int* r_list, double* dev_correlator) {
  U1_TRY(check_hits(n_metro, n_or));
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  if (!dev_correlator) return fail(U1ML_EINVAL, "dev_correlator is NULL");
  Engine& e = lat->e;
  U1_TRY(check_ml_args(e, n_levels, slab_sizes, n_sub, n_metro, n_or));
  if (n_r < 1 || !r_list) return fail(U1ML_EINVAL, "need at least one r");
  std::vector<int> rl(r_list, r_list + n_r);
  for (int r : rl)
    if (r < 1 || r >= e.h_lats[0].L) return fail(U1ML_EINVAL, "r must be in [1, L)");
  U1_TRY(e.set_device());
  void* base = scratch_of(e.device);
  if (!base) return fail(U1ML_ESTATE, "no static workspace on this device");
  return e.multilevel_in_place(n_levels, slab_sizes, n_sub, n_metro, n_or, rl, base, kNoAllocBytes, dev_correlator);
}

static int ensemble_info(Engine& e, int i, int* n_runs, int* n_r, int* n_rf) {
  const Ensemble& en = e.ens;
  if (n_runs) *n_runs = (int)en.n;
  if (n_r) *n_r = en.n ? en.nR[i] : 0;
  if (n_rf) *n_rf = (en.n && en.field) ? en.fp.n_rf : 0;
  return U1ML_OK;
}

int u1ml_ensemble_reset(u1ml_lattice* lat) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  lat->e.ensemble_reset();
  return U1ML_OK;
}

int u1ml_ensemble_add(u1ml_lattice* lat) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  U1_TRY(lat->e.set_device());
  return lat->e.ensemble_add();
}

int u1ml_ensemble_info(u1ml_lattice* lat, int* n_runs, int* n_r, int* n_rf) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  return ensemble_info(lat->e, 0, n_runs, n_r, n_rf);
}

int u1ml_ensemble_read(u1ml_lattice* lat, double* correlator, double* field_profile, double* connected) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  U1_TRY(lat->e.set_device());
  return lat->e.ensemble_read(0, correlator, field_profile, connected);
}

int u1ml_plain_correlator(u1ml_lattice* lat, int n_r, const int* r_list, double* out) {
  if (!lat || n_r < 1 || !r_list || !out) return fail(U1ML_EINVAL, "plain_correlator arguments");
  Engine& e = lat->e;
  std::vector<int> rl(r_list, r_list + n_r);
  for (int r : rl)
    if (r < 0 || r >= e.h_lats[0].L) return fail(U1ML_EINVAL, "r must be in [0, L)");
  U1_TRY(e.set_device());
  std::vector<std::vector<double>> pc;
  U1_TRY(e.poly_corr(rl, pc));
  for (int k = 0; k < n_r; ++k) {
    out[2 * k] = pc[0][2 + 2 * k];
    out[2 * k + 1] = pc[0][3 + 2 * k];
  }
  return U1ML_OK;
}

int u1ml_get_links(u1ml_lattice* lat, double* host) {
  if (!lat || !host) return fail(U1ML_EINVAL, "get_links arguments");
  U1_TRY(lat->e.set_device());
  return lat->e.get_links(0, host);
}

int u1ml_set_links(u1ml_lattice* lat, const double* host) {
  if (!lat || !host) return fail(U1ML_EINVAL, "set_links arguments");
  U1_TRY(lat->e.set_device());
  return lat->e.set_links(0, host);
}

int u1ml_get_pass_id(u1ml_lattice* lat, uint64_t* pass_id) {
  if (!lat || !pass_id) return fail(U1ML_EINVAL, "get_pass_id arguments");
  *pass_id = lat->e.h_pass_ids[0];
  return U1ML_OK;
}

int u1ml_set_pass_id(u1ml_lattice* lat, uint64_t pass_id) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  U1_TRY(lat->e.set_device());
  lat->e.h_pass_ids[0] = pass_id;
  return lat->e.upload_pass_ids();
}

static int set_estimator(Engine& e, unsigned flags) {
  if (flags & ~(U1ML_MULTIHIT | U1ML_FIELD_SQUARED | U1ML_SYMMETRIC)) return fail(U1ML_EINVAL, "unknown estimator flags");
  U1_TRY(e.set_device());
  if (e.estimator != flags) {
    U1_HIP(hipStreamSynchronize(e.stream));
    e.estimator = flags;
    e.ml.key.clear();  // the next multilevel run lays out its workspace again
    e.drop_graphs();
  }
  return U1ML_OK;
}

int u1ml_set_estimator(u1ml_lattice* lat, unsigned flags) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  return set_estimator(lat->e, flags);
}

int u1ml_batch_set_estimator(u1ml_batch* b, unsigned flags) {
  if (!b) return fail(U1ML_EINVAL, "batch is NULL");
  return set_estimator(b->e, flags);
}

int u1ml_set_debug(u1ml_lattice* lat, unsigned flags, size_t capacity) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  Engine& e = lat->e;
  U1_TRY(e.set_device());
  U1_HIP(hipStreamSynchronize(e.stream));
  if (e.field_general != ((flags & 2u) != 0) || e.fold_general != ((flags & 4u) != 0) ||
      e.force_replay != ((flags & 8u) != 0)) {
    e.drop_graphs();  // captured schedules hold the other kernels
    e.field_general = (flags & 2u) != 0;
    e.fold_general = (flags & 4u) != 0;
    e.force_replay = (flags & 8u) != 0;
    e.ml.key.clear();  // the multilevel workspace depends on the replay choice
  }
  if (flags & 1u) {
    U1_TRY(e.log.ensure(capacity));
    // frozen links get no thread; their entries keep this marker
    U1_HIP(launch_fill_u8(e.log.as<uint8_t>(), capacity, 2, e.stream));
    e.debug = true;
    e.log_cap = capacity;
  } else {
    e.debug = false;
    e.log_cap = 0;
  }
  e.log_used = 0;
  return U1ML_OK;
}

int u1ml_get_accept_log(u1ml_lattice* lat, uint8_t* out, size_t cap, size_t* n_bytes) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  Engine& e = lat->e;
  U1_TRY(e.set_device());
  U1_HIP(hipStreamSynchronize(e.stream));
  if (n_bytes) *n_bytes = e.log_used;
  size_t n = std::min(cap, e.log_used);
  if (out && n) U1_TRY(e.copy(out, e.log.p, n, hipMemcpyDeviceToHost));
  return U1ML_OK;
}

}  // extern "C"

namespace {

// One lattice's checkpoint record: a text header line (format, L, T, beta,
// eps, seed, pass id, precision), then its FP64 links in the host order.
struct Record {
  double beta = 0.0, eps = 0.0;
  unsigned long long seed = 0, pass_id = 0;
  std::vector<double> links;
};

int write_record(Engine& e, int i, FILE* f) {
  const LatDesc& d = e.h_lats[i];
  std::vector<double> h(8ull * d.V2);
  U1_TRY(e.get_links(i, h.data()));
  if (std::fprintf(f, "u1ml-checkpoint-1 L=%d T=%d beta=%.17g eps=%.17g seed=%llu pass_id=%llu precision=%d\n",
                   d.L, d.T, d.beta, d.eps, (unsigned long long)d.seed, (unsigned long long)e.h_pass_ids[i],
                   e.prec) < 0 ||
      std::fwrite(h.data(), sizeof(double), h.size(), f) != h.size())
    return fail(U1ML_EIO, "short write");
  return U1ML_OK;
}

// reads the record of lattice i and checks it against that lattice; changes nothing
int read_record(const Engine& e, int i, FILE* f, Record* r) {
  char line[512];
  if (!std::fgets(line, sizeof line, f)) return fail(U1ML_EIO, "missing header");
  int L = 0, T = 0, prec = -1;
  if (std::sscanf(line, "u1ml-checkpoint-1 L=%d T=%d beta=%lg eps=%lg seed=%llu pass_id=%llu precision=%d", &L, &T,
                  &r->beta, &r->eps, &r->seed, &r->pass_id, &prec) != 7)
    return fail(U1ML_EIO, "bad header");
  const LatDesc& d = e.h_lats[i];
  if (L != d.L || T != d.T || prec != e.prec)
    return fail(U1ML_EINVAL, "checkpoint shape or precision differs from the lattice");
  if (!std::isfinite(r->beta) || r->beta < 0 || !(r->eps >= 0 && r->eps <= kMaxEps))
    return fail(U1ML_EINVAL, "checkpoint beta or eps out of range");
  r->links.resize(8ull * d.V2);
  if (std::fread(r->links.data(), sizeof(double), r->links.size(), f) != r->links.size())
    return fail(U1ML_EIO, "short read");
  return U1ML_OK;
}

// installs checked records for lattices 0..n-1 of the engine
int apply_records(Engine& e, const std::vector<Record>& rs) {
  U1_TRY(e.set_device());
  for (size_t i = 0; i < rs.size(); ++i) {
    LatDesc& d = e.h_lats[i];
    d.beta = rs[i].beta;
    d.eps = rs[i].eps;
    d.sqrt_beta = std::sqrt(rs[i].beta);
    d.seed = rs[i].seed;
    e.h_pass_ids[i] = rs[i].pass_id;
  }
  U1_TRY(e.upload_lats());
  U1_TRY(e.upload_pass_ids());
  for (size_t i = 0; i < rs.size(); ++i) U1_TRY(e.set_links((int)i, rs[i].links.data()));
  return U1ML_OK;
}

int save_engine(Engine& e, const char* path, bool batch) {
  U1_TRY(e.set_device());
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(U1ML_EIO, std::string("cannot open ") + path);
  int rc = U1ML_OK;
  if (batch && std::fprintf(f, "u1ml-batch-checkpoint-1 n=%d\n", e.n_lats) < 0) rc = fail(U1ML_EIO, "short write");
  for (int i = 0; i < e.n_lats && !rc; ++i) rc = write_record(e, i, f);
  if (std::fclose(f) != 0 && !rc) rc = fail(U1ML_EIO, "short write");
  return rc;
}

int load_engine(Engine& e, const char* path, bool batch) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(U1ML_EIO, std::string("cannot open ") + path);
  int rc = U1ML_OK;
  if (batch) {
    char line[128];
    int n = -1;
    if (!std::fgets(line, sizeof line, f) || std::sscanf(line, "u1ml-batch-checkpoint-1 n=%d", &n) != 1)
      rc = fail(U1ML_EIO, "bad batch header");
    else if (n != e.n_lats)
      rc = fail(U1ML_EINVAL, "checkpoint holds another number of lattices");
  }
  // every record is read and checked before any lattice changes
  std::vector<Record> rs(e.n_lats);
  for (int i = 0; i < e.n_lats && !rc; ++i) rc = read_record(e, i, f, &rs[i]);
  std::fclose(f);
  if (rc) return rc;
  return apply_records(e, rs);
}

}  // namespace

extern "C" {

int u1ml_save(u1ml_lattice* lat, const char* path) {
  if (!lat || !path) return fail(U1ML_EINVAL, "save arguments");
  return save_engine(lat->e, path, false);
}

int u1ml_load(u1ml_lattice* lat, const char* path) {
  if (!lat || !path) return fail(U1ML_EINVAL, "load arguments");
  return load_engine(lat->e, path, false);
}

int u1ml_synchronize(u1ml_lattice* lat) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  U1_TRY(lat->e.set_device());
  U1_HIP(hipStreamSynchronize(lat->e.stream));
  return U1ML_OK;
}

void u1ml_destroy(u1ml_lattice* lat) {
  if (!lat) return;
  (void)hipSetDevice(lat->e.device);
  delete lat;
}

// --- batches ---
int u1ml_batch_create(int n, const int* L, const int* T, const double* beta, const uint64_t* seed,
                      const u1ml_options* opt, u1ml_batch** out) {
  if (!out || n < 1 || !L || !T || !beta || !seed) return fail(U1ML_EINVAL, "batch_create arguments");
  *out = nullptr;
  std::unique_ptr<u1ml_batch> b(new (std::nothrow) u1ml_batch());
  if (!b) return fail(U1ML_ENOMEM, "host allocation");
  U1_TRY(engine_create(b->e, std::vector<int>(L, L + n), std::vector<int>(T, T + n),
                       std::vector<double>(beta, beta + n), std::vector<uint64_t>(seed, seed + n), opt, false));
  *out = b.release();
  return U1ML_OK;
}

int u1ml_batch_sweep(u1ml_batch* b, int n_metro, int n_or) {
  U1_TRY(check_hits(n_metro, n_or));
  if (!b) return fail(U1ML_EINVAL, "batch is NULL");
  Engine& e = b->e;
  U1_TRY(e.set_device());
  return e.run_captured({0, n_metro, n_or}, [&]() { return e.sweep(n_metro, n_or, 0); });
}

int u1ml_batch_multilevel(u1ml_batch* b, int n_levels, const int* slab_sizes, const int* n_sub, int n_metro,
                          int n_or, int n_r, const int* r_list, int n_rf, const int* rf_list) {
  U1_TRY(check_hits(n_metro, n_or));
  if (!b) return fail(U1ML_EINVAL, "batch is NULL");
  return ml_entry(b->e, n_levels, slab_sizes, n_sub, n_metro, n_or, n_r, r_list, n_rf, rf_list);
}

int u1ml_batch_cycle(u1ml_batch* b, int n_sweeps, int n_metro, int n_or, int th, int n_sub, int use_graph) {
  U1_TRY(check_hits(n_metro, n_or));
  if (!b || n_sweeps < 0) return fail(U1ML_EINVAL, "batch_cycle arguments");
  Engine& e = b->e;
  U1_TRY(check_ml_args(e, 1, &th, &n_sub, n_metro, n_or));
  U1_TRY(e.set_device());
  std::vector<std::vector<int>> rl(e.n_lats);
  for (int i = 0; i < e.n_lats; ++i)
    for (int r = 1; r <= e.h_lats[i].T / 2 && r < e.h_lats[i].L; ++r) rl[i].push_back(r);
  const bool keep = e.use_graphs;
  e.use_graphs = keep && use_graph != 0;
  int rc = e.multilevel(1, &th, &n_sub, n_metro, n_or, rl, {}, n_sweeps);
  e.use_graphs = keep;
  return rc;
}

int u1ml_batch_measure(u1ml_batch* b, int i, u1ml_observables* obs, double* correlator, double* field_profile) {
  if (!b || i < 0 || i >= b->e.n_lats) return fail(U1ML_EINVAL, "batch_measure arguments");
  return read_results(b->e, i, obs, correlator, field_profile);
}

int u1ml_batch_ensemble_reset(u1ml_batch* b) {
  if (!b) return fail(U1ML_EINVAL, "batch is NULL");
  b->e.ensemble_reset();
  return U1ML_OK;
}

int u1ml_batch_ensemble_add(u1ml_batch* b) {
  if (!b) return fail(U1ML_EINVAL, "batch is NULL");
  U1_TRY(b->e.set_device());
  return b->e.ensemble_add();
}

int u1ml_batch_ensemble_info(u1ml_batch* b, int i, int* n_runs, int* n_r, int* n_rf) {
  if (!b || i < 0 || i >= b->e.n_lats) return fail(U1ML_EINVAL, "batch_ensemble_info arguments");
  return ensemble_info(b->e, i, n_runs, n_r, n_rf);
}

int u1ml_batch_ensemble_read(u1ml_batch* b, int i, double* correlator, double* field_profile, double* connected) {
  if (!b || i < 0 || i >= b->e.n_lats) return fail(U1ML_EINVAL, "batch_ensemble_read arguments");
  U1_TRY(b->e.set_device());
  return b->e.ensemble_read(i, correlator, field_profile, connected);
}

int u1ml_batch_get_links(u1ml_batch* b, int i, double* host) {
  if (!b || i < 0 || i >= b->e.n_lats || !host) return fail(U1ML_EINVAL, "batch_get_links arguments");
  U1_TRY(b->e.set_device());
  return b->e.get_links(i, host);
}

int u1ml_batch_set_links(u1ml_batch* b, int i, const double* host) {
  if (!b || i < 0 || i >= b->e.n_lats || !host) return fail(U1ML_EINVAL, "batch_set_links arguments");
  U1_TRY(b->e.set_device());
  return b->e.set_links(i, host);
}

int u1ml_batch_get_pass_id(u1ml_batch* b, int i, uint64_t* pass_id) {
  if (!b || i < 0 || i >= b->e.n_lats || !pass_id) return fail(U1ML_EINVAL, "batch_get_pass_id arguments");
  *pass_id = b->e.h_pass_ids[i];
  return U1ML_OK;
}

int u1ml_batch_set_pass_id(u1ml_batch* b, int i, uint64_t pass_id) {
  if (!b || i < 0 || i >= b->e.n_lats) return fail(U1ML_EINVAL, "batch_set_pass_id arguments");
  U1_TRY(b->e.set_device());
  b->e.h_pass_ids[i] = pass_id;
  return b->e.upload_pass_ids();
}

int u1ml_batch_save(u1ml_batch* b, const char* path) {
  if (!b || !path) return fail(U1ML_EINVAL, "batch_save arguments");
  return save_engine(b->e, path, true);
}

int u1ml_batch_load(u1ml_batch* b, const char* path) {
  if (!b || !path) return fail(U1ML_EINVAL, "batch_load arguments");
  return load_engine(b->e, path, true);
}

int u1ml_batch_synchronize(u1ml_batch* b) {
  if (!b) return fail(U1ML_EINVAL, "batch is NULL");
  U1_TRY(b->e.set_device());
  U1_HIP(hipStreamSynchronize(b->e.stream));
  return U1ML_OK;
}

void u1ml_batch_destroy(u1ml_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->e.device);
  delete b;
}

int u1ml_autotune(u1ml_lattice* lat, int* best_block) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  Engine& e = lat->e;
  U1_TRY(e.set_device());
  if (e.debug) return fail(U1ML_ESTATE, "autotune with the debug log enabled");
  DevBuf save;
  U1_TRY(save.ensure(e.link_elems * e.elem_size()));
  U1_HIP(hipMemcpyAsync(save.p, e.links.p, e.link_elems * e.elem_size(), hipMemcpyDeviceToDevice, e.stream));
  const std::vector<uint64_t> ids = e.h_pass_ids;
  hipEvent_t a, z;
  U1_HIP(hipEventCreate(&a));
  U1_HIP(hipEventCreate(&z));
  const int cand[] = {64, 128, 256, 512, 1024};
  float best_ms = 1e30f;
  int best = e.block, rc = U1ML_OK;
  for (int blk : cand) {
    e.block = blk;
    if ((rc = e.sweep(1, 1, 0))) break;  // warm-up
    (void)hipEventRecord(a, e.stream);
    for (int k = 0; k < 3 && !rc; ++k) rc = e.sweep(1, 3, 0);
    (void)hipEventRecord(z, e.stream);
    (void)hipEventSynchronize(z);
    if (rc) break;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, z);
    if (ms < best_ms) {
      best_ms = ms;
      best = blk;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(z);
  e.block = best;
  e.drop_graphs();  // captured launches carry the old block size
  U1_HIP(hipMemcpyAsync(e.links.p, save.p, e.link_elems * e.elem_size(), hipMemcpyDeviceToDevice, e.stream));
  ++e.epoch;
  e.h_pass_ids = ids;
  int rc2 = e.upload_pass_ids();
  if (rc) return rc;
  if (rc2) return rc2;
  set_tuned_block(e.h_lats[0].L, e.h_lats[0].T, e.prec, best);
  if (best_block) *best_block = best;
  return U1ML_OK;
}

// --- launch-shape tuning ---
static void get_tuning(const Engine& e, u1ml_tuning* t) {
  t->pass_block = e.block;
  t->pass_xcd_map = e.xcd_map;
  t->sample_block = e.sample_block;
  t->fold_threads = e.fold_threads;
  t->field_w_planes = e.ftune.w_planes;
  t->field_o_planes = e.ftune.o_planes;
  t->field_zcon_threads = e.ftune.zcon_threads;
  t->fold_stage = e.fold_stage;
}

static int set_tuning(Engine& e, const u1ml_tuning& t) {
  auto mult64 = [](int v, int lo, int hi) { return v >= lo && v <= hi && v % 64 == 0; };
  if (!mult64(t.pass_block, 64, 1024) || (t.pass_xcd_map != 0 && t.pass_xcd_map != 1) ||
      !mult64(t.sample_block, 64, 1024) || (t.fold_threads != 0 && !mult64(t.fold_threads, 64, 256)) ||
      t.field_w_planes < 0 || t.field_w_planes > 64 || t.field_o_planes < 0 || t.field_o_planes > 64 ||
      (t.field_zcon_threads != 0 && !mult64(t.field_zcon_threads, 64, 256)) || t.fold_stage < 0 ||
      t.fold_stage > 2)
    return fail(U1ML_EINVAL, "tuning values out of range");
  U1_TRY(e.set_device());
  U1_HIP(hipStreamSynchronize(e.stream));
  e.block = t.pass_block;
  e.xcd_map = t.pass_xcd_map;
  e.sample_block = t.sample_block;
  e.fold_threads = t.fold_threads;
  e.ftune.w_planes = t.field_w_planes;
  e.ftune.o_planes = t.field_o_planes;
  e.ftune.zcon_threads = t.field_zcon_threads;
  e.fold_stage = t.fold_stage;
  e.drop_graphs();  // captured launches carry the old shapes
  return U1ML_OK;
}

// average of the recorded event intervals (ms); destroys the events
static int events_avg(Engine& e, std::vector<std::pair<hipEvent_t, hipEvent_t>>& ev, double* avg_ms) {
  hipError_t se = hipStreamSynchronize(e.stream);
  double tot = 0.0;
  for (auto& pr : ev) {
    float ms = 0.f;
    if (se == hipSuccess) (void)hipEventElapsedTime(&ms, pr.first, pr.second);
    tot += ms;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  *avg_ms = ev.empty() ? 0.0 : tot / (double)ev.size();
  ev.clear();
  U1_HIP(se);
  return U1ML_OK;
}

// Coordinate search over the launch shapes, one kernel family at a time (the
// others at their current best): class-pass block size and XCD order timed
// over compound sweeps; then with multilevel runs of the given shape (best of
// two per candidate) the per-sample kernel's block size, the row fold's
// threads, and with field separations the planes per block of both field
// transforms and the contraction's threads, each timed over its own launches
// only.  Every choice gives the same bits, and the links and pass ids are
// restored.
static int autotune_engine(Engine& e, int n_levels, const int* th, const int* n_sub,
                           const std::vector<std::vector<int>>& rl, const std::vector<int>& rf, u1ml_tuning* best) {
  if (e.debug) return fail(U1ML_ESTATE, "autotune with the debug log enabled");
  U1_TRY(e.set_device());
  DevBuf save, save_ids;
  const size_t lb = e.link_elems * e.elem_size(), ib = e.n_lats * sizeof(uint64_t);
  U1_TRY(save.ensure(lb));
  U1_TRY(save_ids.ensure(ib));
  U1_HIP(hipMemcpyAsync(save.p, e.links.p, lb, hipMemcpyDeviceToDevice, e.stream));
  U1_HIP(hipMemcpyAsync(save_ids.p, e.pass_ids.p, ib, hipMemcpyDeviceToDevice, e.stream));
  const std::vector<uint64_t> ids = e.h_pass_ids;
  e.drop_graphs();
  int rc = U1ML_OK;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  // 1. class passes: block size x block order, the best of two timings of 3 compound sweeps
  {
    double best_ms = 1e300;
    int bb = e.block, bx = e.xcd_map;
    for (int xcd = 1; xcd >= 0 && !rc; --xcd)
      for (int blk = 64; blk <= 1024 && !rc; blk *= 2) {
        e.block = blk;
        e.xcd_map = xcd;
        if ((rc = e.sweep(1, 1, 0))) break;  // warm-up (block tables of this size)
        double t_min = 1e300;
        for (int rep = 0; rep < 2 && !rc; ++rep) {
          e.prof[0] = e.prof[1] = &ev;
          for (int k = 0; k < 3 && !rc; ++k) rc = e.sweep(1, 3, 0);
          e.prof[0] = e.prof[1] = nullptr;
          double ms = 0;
          if (!rc) rc = events_avg(e, ev, &ms);
          t_min = std::min(t_min, ms);
        }
        if (!rc && t_min < best_ms) {
          best_ms = t_min;
          bb = blk;
          bx = xcd;
        }
      }
    e.block = bb;
    e.xcd_map = bx;
  }
  // 2. measurement kernels, each timed over a multilevel run of the given shape
  auto time_family = [&](int fam, double* ms) -> int {
    e.fam_prof = &ev;
    e.fam_id = fam;
    int r = e.multilevel(n_levels, th, n_sub, 1, 3, rl, rf, 0);
    e.fam_prof = nullptr;
    e.fam_id = -1;
    if (r) {
      for (auto& pr : ev) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
      }
      ev.clear();
      return r;
    }
    return events_avg(e, ev, ms);
  };
  // the better of two timings per candidate
  auto search = [&](int fam, int* knob, const std::vector<int>& cand) -> int {
    double best_ms = 1e300;
    int keep = *knob;
    for (int v : cand) {
      *knob = v;
      double ms = 1e300;
      for (int rep = 0; rep < 2; ++rep) {
        double t = 0.0;
        U1_TRY(time_family(fam, &t));
        ms = std::min(ms, t);
      }
      if (ms < best_ms) {
        best_ms = ms;
        keep = v;
      }
    }
    *knob = keep;
    return U1ML_OK;
  };
  if (!rc && n_levels > 0) {
    // the first run sets up the workspace and loads the kernels
    double ms = 0;
    rc = time_family(-1, &ms);
    if (!rc) rc = search(Engine::kFamSample, &e.sample_block, {64, 128, 256, 512, 1024});
    if (!rc) rc = search(Engine::kFamFold, &e.fold_threads, {64, 128, 192, 256});
    int max_w = 64, max_o = 64;
    for (auto& d : e.h_lats) {
      max_w = std::min(max_w, field_max_planes(d.L, false));
      max_o = std::min(max_o, field_max_planes(d.L, true));
    }
    if (!rc && !rf.empty() && !e.field_general && max_w > 0 && max_o > 0) {
      std::vector<int> cw, co;
      for (int v = 1; v <= max_w; ++v) cw.push_back(v);
      for (int v = 1; v <= max_o; ++v) co.push_back(v);
      rc = search(Engine::kFamField, &e.ftune.w_planes, cw);
      if (!rc) rc = search(Engine::kFamField, &e.ftune.o_planes, co);
      if (!rc) rc = search(Engine::kFamField, &e.ftune.zcon_threads, {64, 128, 192, 256});
    }
  }
  // restore the chain; the tuning runs' results are not kept
  e.drop_graphs();
  U1_HIP(hipMemcpyAsync(e.links.p, save.p, lb, hipMemcpyDeviceToDevice, e.stream));
  U1_HIP(hipMemcpyAsync(e.pass_ids.p, save_ids.p, ib, hipMemcpyDeviceToDevice, e.stream));
  U1_HIP(hipStreamSynchronize(e.stream));
  e.h_pass_ids = ids;
  ++e.epoch;
  e.ml.valid = e.ml.field_valid = false;
  if (rc) return rc;
  if (best) get_tuning(e, best);
  return U1ML_OK;
}

static int profile_sweeps(Engine& e, int n_sweeps, int n_metro, int n_or, double* avg_us) {
  if (!avg_us || n_sweeps < 0) return fail(U1ML_EINVAL, "profile arguments");
  U1_TRY(check_hits(n_metro, n_or));
  U1_TRY(e.set_device());
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[2];
  e.prof[0] = &ev[0];
  e.prof[1] = &ev[1];
  int rc = U1ML_OK;
  for (int s = 0; s < n_sweeps && !rc; ++s) rc = e.sweep(n_metro, n_or, 0);
  e.prof[0] = e.prof[1] = nullptr;
  hipError_t se = hipStreamSynchronize(e.stream);
  for (int k = 0; k < 2; ++k) {
    double tot = 0.0;
    for (auto& pr : ev[k]) {
      float ms = 0.f;
      if (se == hipSuccess && !rc) (void)hipEventElapsedTime(&ms, pr.first, pr.second);
      tot += ms;
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    avg_us[k] = ev[k].empty() ? 0.0 : 1e3 * tot / (double)ev[k].size();
  }
  if (rc) return rc;
  U1_HIP(se);
  return U1ML_OK;
}

int u1ml_get_tuning(u1ml_lattice* lat, u1ml_tuning* t) {
  if (!lat || !t) return fail(U1ML_EINVAL, "get_tuning arguments");
  get_tuning(lat->e, t);
  return U1ML_OK;
}

int u1ml_set_tuning(u1ml_lattice* lat, const u1ml_tuning* t) {
  if (!lat || !t) return fail(U1ML_EINVAL, "set_tuning arguments");
  return set_tuning(lat->e, *t);
}

int u1ml_batch_get_tuning(u1ml_batch* b, u1ml_tuning* t) {
  if (!b || !t) return fail(U1ML_EINVAL, "batch_get_tuning arguments");
  get_tuning(b->e, t);
  return U1ML_OK;
}

int u1ml_batch_set_tuning(u1ml_batch* b, const u1ml_tuning* t) {
  if (!b || !t) return fail(U1ML_EINVAL, "batch_set_tuning arguments");
  return set_tuning(b->e, *t);
}

int u1ml_batch_autotune(u1ml_batch* b, int n_levels, const int* slab_sizes, const int* n_sub, int n_r,
                        const int* r_list, int n_rf, const int* rf_list, u1ml_tuning* best) {
  if (!b) return fail(U1ML_EINVAL, "batch is NULL");
  Engine& e = b->e;
  std::vector<std::vector<int>> rl(e.n_lats);
  std::vector<int> rf;
  if (n_levels > 0) {
    U1_TRY(check_ml_args(e, n_levels, slab_sizes, n_sub, 1, 3));
    if (n_r < 1 || !r_list) return fail(U1ML_EINVAL, "need at least one r");
    if (n_rf < 0 || n_rf > U1ML_MAX_FIELD_R || (n_rf > 0 && (!rf_list || n_levels > 2)))
      return fail(U1ML_EINVAL, "field r list");
    for (auto& d : e.h_lats)
      for (int k = 0; k < n_r; ++k)
        if (r_list[k] < 1 || r_list[k] >= d.L || (n_rf > 0 && d.L > kMaxFieldL))
          return fail(U1ML_EINVAL, "r must be in [1, L) (field: L <= 62)");
    for (int f = 0; f < n_rf; ++f) {
      if (std::find(r_list, r_list + n_r, rf_list[f]) == r_list + n_r)
        return fail(U1ML_EINVAL, "every field r must appear in r_list");
      rf.push_back(rf_list[f]);
    }
    for (auto& v : rl) v.assign(r_list, r_list + n_r);
  } else if (n_levels < 0) {
    return fail(U1ML_EINVAL, "n_levels must be >= 0");
  }
  return autotune_engine(e, n_levels, slab_sizes, n_sub, rl, rf, best);
}

int u1ml_profile_sweeps(u1ml_lattice* lat, int n_sweeps, int n_metro, int n_or, double* avg_us) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  return profile_sweeps(lat->e, n_sweeps, n_metro, n_or, avg_us);
}

int u1ml_batch_profile_sweeps(u1ml_batch* b, int n_sweeps, int n_metro, int n_or, double* avg_us) {
  if (!b) return fail(U1ML_EINVAL, "batch is NULL");
  return profile_sweeps(b->e, n_sweeps, n_metro, n_or, avg_us);
}

int u1ml_stream_bandwidth(int kind, size_t n_bytes, int reps, double* gb_per_s) {
  if ((kind != 0 && kind != 1) || n_bytes < (1u << 20) || n_bytes % 16 || reps < 1 || !gb_per_s)
    return fail(U1ML_EINVAL, "stream_bandwidth: kind 0 or 1, n_bytes >= 1 MiB and a multiple of 16, reps >= 1");
  *gb_per_s = 0.0;
  // 8 blocks of 256 threads per compute unit in grid-stride loops
  constexpr int kBlocks = 2048;
  DevBuf a, b, sink;
  U1_TRY(a.ensure(n_bytes));
  if (kind == 1) U1_TRY(b.ensure(n_bytes));
  U1_TRY(sink.ensure(sizeof(float)));
  hipStream_t st;
  U1_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // zeros in the source: the read kernel's guarded store never happens
  if (e == hipSuccess) e = launch_stream_probe(2, nullptr, a.p, n_bytes, nullptr, kBlocks, st);
  if (e == hipSuccess) e = launch_stream_probe(kind, a.p, b.p, n_bytes, sink.as<float>(), kBlocks, st);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int k = 0; k < reps && e == hipSuccess; ++k)
    e = launch_stream_probe(kind, a.p, b.p, n_bytes, sink.as<float>(), kBlocks, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
  U1_HIP(e);
  if (!(ms > 0.f)) return fail(U1ML_EDEVICE, "stream_bandwidth: no elapsed time");
  *gb_per_s = (double)reps * (double)n_bytes * (kind == 1 ? 2.0 : 1.0) / (ms * 1e-3) / 1e9;
  return U1ML_OK;
}

const char* u1ml_strerror(int code) {
  switch (code) {
    case U1ML_OK: return "success";
    case U1ML_EINVAL: return "invalid argument";
    case U1ML_ENOMEM: return "out of memory";
    case U1ML_EDEVICE: return "HIP device error";
    case U1ML_ESTATE: return "invalid state for this call";
    case U1ML_EIO: return "checkpoint file error";
    default: return "unknown error";
  }
}

const char* u1ml_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
