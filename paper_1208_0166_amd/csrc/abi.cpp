// abi.cpp -- the u1ml C ABI: lattice and batch handles, the update schedule
// (compound sweeps, multilevel nesting, field replay), measurements,
// checkpoints and the block-size autotuner.  Host code only; all lattice
// arithmetic runs in the kernels of sweep_f64.hip, sweep_f32.hip and
// measure.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
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

#define U1_HIP(expr)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return fail(U1ML_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// device buffer that only grows
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = true;
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

// largest |theta| accepted from the host; the updates fold angles back into
// [-pi, pi) by whole periods, which needs them to be of moderate size
constexpr double kMaxAngle = 64.0;

struct Table {
  DevBuf buf;
  int n_blocks = 0;
  int block = 0;
  std::vector<int> lat_block_begin;  // n_lats + 1
};

struct MLState {
  bool valid = false;  // a multilevel has completed
  int n_levels = 0;
  int th[U1ML_MAX_LEVELS] = {0, 0, 0};
  int n[U1ML_MAX_LEVELS] = {0, 0, 0};
  int n_metro = 1, n_or = 0;
  int max_r = 0;
  std::vector<int> nR;        // per lattice
  std::vector<MLDesc> h_mls;  // per lattice
  DevBuf mls, rvals, mlbuf, accbuf, corr;
  uint64_t acc_elems = 0;
  // field insertion (single lattice)
  bool field = false;
  bool field_valid = false;
  FieldDesc fd{};
  DevBuf tavg, w, oslab, wslab, fout, snap_links, fd_dev;
  int replay = 0;  // 1 while replaying
};

}  // namespace

struct Engine {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int prec = U1ML_FP64;
  int start = U1ML_HOT;
  int block = 256;
  int n_lats = 0;
  std::vector<LatDesc> h_lats;
  DevBuf lats;
  DevBuf links;
  size_t link_elems = 0;
  DevBuf pass_ids;
  std::vector<uint64_t> h_pass_ids;
  std::map<std::pair<std::vector<int>, int>, std::unique_ptr<Table>> tables;
  // debug log (single lattice)
  DevBuf log;
  size_t log_cap = 0, log_used = 0;
  bool debug = false;
  // measurement scratch
  DevBuf partial, rows, poly, poly_off, row_begin, red_out, rvals_tmp;
  MLState ml;
  // batch cycle graph
  hipGraphExec_t graph_exec = nullptr;
  std::vector<int> graph_key;
  int graph_metro_passes = 0;

  ~Engine() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (own_stream && stream) {
      (void)hipStreamSynchronize(stream);
      (void)hipStreamDestroy(stream);
    }
  }

  size_t elem_size() const { return prec == U1ML_FP64 ? 8 : 4; }

  int set_device() {
    U1_HIP(hipSetDevice(device));
    return U1ML_OK;
  }

  // block table for per-lattice item counts
  int table(const std::vector<int>& items, int blk, Table** out) {
    auto key = std::make_pair(items, blk);
    auto it = tables.find(key);
    if (it != tables.end()) {
      *out = it->second.get();
      return U1ML_OK;
    }
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
      int rc = t->buf.ensure(h.size() * sizeof(int2));
      if (rc) return rc;
      U1_HIP(hipMemcpy(t->buf.p, h.data(), h.size() * sizeof(int2), hipMemcpyHostToDevice));
    }
    *out = t.get();
    tables[key] = std::move(t);
    return U1ML_OK;
  }

  BlockTable bt(Table* t) const {
    BlockTable b;
    b.dev = t->buf.as<int2>();
    b.n_blocks = t->n_blocks;
    b.block = t->block;
    return b;
  }

  std::vector<int> items_half() const {
    std::vector<int> v;
    for (auto& d : h_lats) v.push_back(d.V2);
    return v;
  }

  // --- updates ---
  int class_pass(int kind, int mu, int parity, int th_frozen, int n_hits, uint8_t* logp) {
    Table* t;
    int rc = table(items_half(), block, &t);
    if (rc) return rc;
    hipError_t e;
    if (prec == U1ML_FP64)
      e = launch_class_pass_f64(kind, links.as<double>(), lats.as<LatDesc>(), bt(t), mu, parity, th_frozen, n_hits,
                                pass_ids.as<uint64_t>(), logp, stream);
    else
      e = launch_class_pass_f32(kind, links.as<float>(), lats.as<LatDesc>(), bt(t), mu, parity, th_frozen, n_hits,
                                pass_ids.as<uint64_t>(), logp, stream);
    U1_HIP(e);
    return U1ML_OK;
  }

  int sweep(int n_metro, int n_or, int th_frozen) {
    if (n_metro > 0) {
      for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p) {
          uint8_t* lp = nullptr;
          if (debug && n_lats == 1) {
            size_t want = (size_t)h_lats[0].V2 * n_metro;
            if (log_used + want <= log_cap) {
              lp = log.as<uint8_t>() + log_used;
              log_used += want;
            }
          }
          int rc = class_pass(kMetropolis, mu, p, th_frozen, n_metro, lp);
          if (rc) return rc;
        }
      U1_HIP(launch_bump_pass_ids(pass_ids.as<uint64_t>(), n_lats, stream));
      for (auto& v : h_pass_ids) v += 1;
    }
    for (int k = 0; k < n_or; ++k)
      for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p) {
          int rc = class_pass(kOverrelax, mu, p, th_frozen, 0, nullptr);
          if (rc) return rc;
        }
    return U1ML_OK;
  }

  int init_links(int hot) {
    std::vector<int> items;
    for (auto& d : h_lats) items.push_back(8 * d.V2);
    Table* t;
    int rc = table(items, 256, &t);
    if (rc) return rc;
    hipError_t e = prec == U1ML_FP64 ? launch_init_f64(links.as<double>(), lats.as<LatDesc>(), bt(t), hot, stream)
                                     : launch_init_f32(links.as<float>(), lats.as<LatDesc>(), bt(t), hot, stream);
    U1_HIP(e);
    return U1ML_OK;
  }

  int upload_pass_ids() {
    U1_HIP(hipMemcpyAsync(pass_ids.p, h_pass_ids.data(), n_lats * sizeof(uint64_t), hipMemcpyHostToDevice, stream));
    U1_HIP(hipStreamSynchronize(stream));
    return U1ML_OK;
  }

  // --- host <-> device link transfer (natural order theta[t][z][y][x][mu]) ---
  int get_links(int i, double* host) {
    const LatDesc& d = h_lats[i];
    const size_t n = 8ull * d.V2;
    std::vector<char> raw(n * elem_size());
    U1_HIP(hipStreamSynchronize(stream));
    U1_HIP(hipMemcpy(raw.data(), links.as<char>() + d.off * elem_size(), raw.size(), hipMemcpyDeviceToHost));
    for (int mu = 0; mu < 4; ++mu)
      for (int p = 0; p < 2; ++p)
        for (uint32_t h = 0; h < (uint32_t)d.V2; ++h) {
          size_t src = ((size_t)(mu * 2 + p)) * d.V2 + h;
          size_t nat = natural_of(d, p, h);
          double v = prec == U1ML_FP64 ? ((double*)raw.data())[src] : (double)((float*)raw.data())[src];
          host[nat * 4 + mu] = v;
        }
    return U1ML_OK;
  }

  int set_links(int i, const double* host) {
    const LatDesc& d = h_lats[i];
    const size_t n = 8ull * d.V2;
    for (size_t k = 0; k < n; ++k)
      if (!(std::fabs(host[k]) <= kMaxAngle)) return fail(U1ML_EINVAL, "set_links: angles must be finite, |theta| <= 64");
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
    U1_HIP(hipStreamSynchronize(stream));
    U1_HIP(hipMemcpy(links.as<char>() + d.off * elem_size(), raw.data(), raw.size(), hipMemcpyHostToDevice));
    return U1ML_OK;
  }

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

  // --- plain observables for every lattice: out[lat][7] and poly rows ---
  int observables(std::vector<u1ml_observables>& res) {
    std::vector<int> items;
    for (auto& d : h_lats) items.push_back(2 * d.V2);
    Table* t;
    int rc = table(items, 256, &t);
    if (rc) return rc;
    if ((rc = partial.ensure((size_t)t->n_blocks * 7 * sizeof(double)))) return rc;
    U1_HIP(launch_plaq_field(prec, links.p, lats.as<LatDesc>(), bt(t), partial.as<double>(), stream));
    if ((rc = row_begin.ensure((n_lats + 1) * sizeof(int)))) return rc;
    U1_HIP(hipMemcpyAsync(row_begin.p, t->lat_block_begin.data(), (n_lats + 1) * sizeof(int), hipMemcpyHostToDevice,
                          stream));
    if ((rc = red_out.ensure((size_t)n_lats * 7 * sizeof(double)))) return rc;
    U1_HIP(launch_reduce_rows(partial.as<double>(), 7, row_begin.as<int>(), n_lats, red_out.as<double>(), stream));
    std::vector<double> pf((size_t)n_lats * 7);
    U1_HIP(hipMemcpyAsync(pf.data(), red_out.p, pf.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    U1_HIP(hipStreamSynchronize(stream));
    std::vector<std::vector<double>> pc;
    rc = poly_corr(std::vector<int>(), pc);
    if (rc) return rc;
    res.resize(n_lats);
    for (int i = 0; i < n_lats; ++i) {
      const double V = 2.0 * h_lats[i].V2;
      res[i].plaquette = pf[i * 7] / (6.0 * V);
      for (int c = 0; c < 6; ++c) res[i].field_mean[c] = pf[i * 7 + 1 + c] / V;
      res[i].poly_re = pc[i][0];
      res[i].poly_im = pc[i][1];
      res[i].poly_abs = std::hypot(pc[i][0], pc[i][1]);
    }
    return U1ML_OK;
  }

  // Polyakov loop average and plain correlator of every lattice (same r list):
  // out[lat] = {Re P, Im P, Re C(r_0), Im C(r_0), ...}
  int poly_corr(const std::vector<int>& r_list, std::vector<std::vector<double>>& out) {
    std::vector<int> items;
    std::vector<uint64_t> offs;
    std::vector<int> rb{0};
    uint64_t o = 0;
    for (auto& d : h_lats) {
      items.push_back(d.L3);
      offs.push_back(o);
      o += d.L3;
      rb.push_back(rb.back() + d.L3);
    }
    Table* t;
    int rc = table(items, 256, &t);
    if (rc) return rc;
    const int nR = (int)r_list.size();
    const int width = 2 + 2 * nR;
    if ((rc = poly.ensure(o * sizeof(double)))) return rc;
    if ((rc = poly_off.ensure(offs.size() * sizeof(uint64_t)))) return rc;
    if ((rc = rows.ensure(o * width * sizeof(double)))) return rc;
    if ((rc = row_begin.ensure(rb.size() * sizeof(int)))) return rc;
    if ((rc = rvals_tmp.ensure(std::max(nR, 1) * sizeof(int)))) return rc;
    if ((rc = red_out.ensure((size_t)n_lats * width * sizeof(double)))) return rc;
    U1_HIP(hipMemcpyAsync(poly_off.p, offs.data(), offs.size() * sizeof(uint64_t), hipMemcpyHostToDevice, stream));
    U1_HIP(hipMemcpyAsync(row_begin.p, rb.data(), rb.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    if (nR) U1_HIP(hipMemcpyAsync(rvals_tmp.p, r_list.data(), nR * sizeof(int), hipMemcpyHostToDevice, stream));
    U1_HIP(launch_poly_lines(prec, links.p, lats.as<LatDesc>(), bt(t), poly_off.as<uint64_t>(), poly.as<double>(),
                             stream));
    U1_HIP(launch_poly_corr(lats.as<LatDesc>(), bt(t), poly_off.as<uint64_t>(), poly.as<double>(),
                            rvals_tmp.as<int>(), nR, row_begin.as<int>(), rows.as<double>(), stream));
    U1_HIP(launch_reduce_rows(rows.as<double>(), width, row_begin.as<int>(), n_lats, red_out.as<double>(), stream));
    std::vector<double> h((size_t)n_lats * width);
    U1_HIP(hipMemcpyAsync(h.data(), red_out.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    U1_HIP(hipStreamSynchronize(stream));
    out.assign(n_lats, std::vector<double>(width));
    for (int i = 0; i < n_lats; ++i)
      for (int c = 0; c < width; ++c) out[i][c] = h[(size_t)i * width + c] / (double)h_lats[i].L3;
    return U1ML_OK;
  }

  // --- multilevel ---
  // r lists: per lattice (rl[i]); field only for a single lattice.
  int ml_setup(int n_levels, const int* th, const int* n_sub, int n_metro, int n_or,
               const std::vector<std::vector<int>>& rl, const std::vector<int>& rf) {
    MLState& m = ml;
    // buffers below may still be read by queued work of an earlier run
    U1_HIP(hipStreamSynchronize(stream));
    m.valid = false;
    m.field_valid = false;
    m.n_levels = n_levels;
    for (int l = 0; l < n_levels; ++l) {
      m.th[l] = th[l];
      m.n[l] = n_sub[l];
    }
    m.n_metro = n_metro;
    m.n_or = n_or;
    m.h_mls.assign(n_lats, MLDesc{});
    m.nR.assign(n_lats, 0);
    std::vector<int> rv;
    uint64_t ell = 0, acc = 0;
    m.max_r = 0;
    const int inner = n_levels - 1;
    for (int i = 0; i < n_lats; ++i) {
      const LatDesc& d = h_lats[i];
      MLDesc& md = m.h_mls[i];
      md.nR = (int)rl[i].size();
      md.r_off = (int)rv.size();
      for (int r : rl[i]) rv.push_back(r);
      m.nR[i] = md.nR;
      m.max_r = std::max(m.max_r, md.nR);
      for (int l = 0; l < n_levels; ++l) md.ns[l] = d.T / th[l];
      md.ell = ell;
      ell += (uint64_t)n_sub[inner] * md.ns[inner] * d.L3;
      for (int l = 0; l < n_levels; ++l) {
        md.acc[l] = acc;
        if (l < inner) acc += (uint64_t)md.ns[l] * d.L3 * md.nR;
      }
      md.acc[n_levels] = acc;
      acc += (uint64_t)d.L3 * md.nR;
    }
    m.acc_elems = acc;
    int rc;
    if ((rc = m.mls.ensure(n_lats * sizeof(MLDesc)))) return rc;
    if ((rc = m.rvals.ensure(rv.size() * sizeof(int)))) return rc;
    if ((rc = m.mlbuf.ensure(ell * sizeof(double)))) return rc;
    if ((rc = m.accbuf.ensure(acc * sizeof(double2)))) return rc;
    if ((rc = m.corr.ensure((size_t)n_lats * m.max_r * 2 * sizeof(double)))) return rc;
    U1_HIP(hipMemcpy(m.mls.p, m.h_mls.data(), n_lats * sizeof(MLDesc), hipMemcpyHostToDevice));
    U1_HIP(hipMemcpy(m.rvals.p, rv.data(), rv.size() * sizeof(int), hipMemcpyHostToDevice));
    // prepare block tables used by the run so that no allocation happens later
    Table* t;
    std::vector<int> it_lines, it_top;
    for (int i = 0; i < n_lats; ++i) {
      it_lines.push_back(m.h_mls[i].ns[inner] * h_lats[i].L3);
      it_top.push_back(h_lats[i].L3 * m.h_mls[i].nR);
    }
    if ((rc = table(it_lines, 256, &t))) return rc;
    if ((rc = table(it_top, 256, &t))) return rc;
    for (int l = 0; l < inner; ++l) {
      std::vector<int> it;
      for (int i = 0; i < n_lats; ++i) it.push_back(m.h_mls[i].ns[l] * h_lats[i].L3 * m.h_mls[i].nR);
      if ((rc = table(it, 256, &t))) return rc;
    }
    if ((rc = table(items_half(), block, &t))) return rc;
    // field insertion workspace
    m.field = !rf.empty();
    if (m.field) {
      const LatDesc& d = h_lats[0];
      FieldDesc& fd = m.fd;
      fd = FieldDesc{};
      fd.n_rf = (int)rf.size();
      for (int f = 0; f < fd.n_rf; ++f) {
        fd.rf[f] = rf[f];
        fd.rf_k[f] = (int)(std::find(rl[0].begin(), rl[0].end(), rf[f]) - rl[0].begin());
      }
      fd.n_levels = n_levels;
      fd.n_outer = n_levels == 2 ? n_sub[0] : 1;
      fd.n_inner = n_sub[inner];
      fd.ns_inner = m.h_mls[0].ns[inner];
      fd.children = n_levels == 2 ? th[0] / th[1] : fd.ns_inner;
      fd.th_inner = th[inner];
      const uint64_t tw = (uint64_t)fd.n_outer * fd.ns_inner * d.L3 * fd.n_rf;
      if ((rc = m.tavg.ensure(tw * sizeof(double2)))) return rc;
      if ((rc = m.w.ensure(tw * sizeof(double2)))) return rc;
      if ((rc = m.oslab.ensure((uint64_t)6 * fd.ns_inner * d.L3 * sizeof(double)))) return rc;
      if ((rc = m.wslab.ensure((uint64_t)fd.n_rf * fd.ns_inner * d.L3 * sizeof(double2)))) return rc;
      if ((rc = m.fout.ensure((uint64_t)fd.n_rf * 12 * d.L * d.L * sizeof(double2)))) return rc;
      if ((rc = m.snap_links.ensure(link_elems * elem_size()))) return rc;
    }
    return U1ML_OK;
  }

  int ml_fold(int child, int parent) {
    MLState& m = ml;
    const int inner = m.n_levels - 1;
    std::vector<int> it;
    for (int i = 0; i < n_lats; ++i) {
      int nsp = parent == m.n_levels ? 1 : m.h_mls[i].ns[parent];
      it.push_back(nsp * h_lats[i].L3 * m.h_mls[i].nR);
    }
    Table* t;
    int rc = table(it, 256, &t);
    if (rc) return rc;
    U1_HIP(launch_ml_fold(lats.as<LatDesc>(), m.mls.as<MLDesc>(), bt(t), child, parent, m.n_levels, child == inner,
                          m.n[child], m.rvals.as<int>(), m.mlbuf.as<double>(), m.accbuf.as<double2>(), stream));
    return U1ML_OK;
  }

  int ml_lines(int sample) {
    MLState& m = ml;
    const int inner = m.n_levels - 1;
    std::vector<int> it;
    for (int i = 0; i < n_lats; ++i) it.push_back(m.h_mls[i].ns[inner] * h_lats[i].L3);
    Table* t;
    int rc = table(it, 256, &t);
    if (rc) return rc;
    U1_HIP(launch_ml_lines(prec, links.p, lats.as<LatDesc>(), m.mls.as<MLDesc>(), bt(t), m.th[inner], sample,
                           m.mlbuf.as<double>(), stream));
    return U1ML_OK;
  }

  int ml_level(int l, int outer_it) {
    MLState& m = ml;
    const int inner = m.n_levels - 1;
    for (int it = 0; it < m.n[l]; ++it) {
      int rc = sweep(m.n_metro, m.n_or, m.th[l]);
      if (rc) return rc;
      const int mo = l == 0 ? it : outer_it;
      if (l == inner) {
        if ((rc = ml_lines(it))) return rc;
        if (m.replay) {
          U1_HIP(launch_field_sample(prec, links.p, lats.as<LatDesc>(), m.mls.as<MLDesc>(), m.fd, h_lats[0].L,
                                     m.n_levels == 2 ? outer_it : 0, it, m.mlbuf.as<double>(), m.w.as<double2>(),
                                     m.oslab.as<double>(), m.wslab.as<double2>(), m.fout.as<double2>(), stream));
        }
      } else {
        if ((rc = ml_level(l + 1, mo))) return rc;
        if (!m.replay) {
          if (m.field && l == 0)
            U1_HIP(launch_field_store_tavg(lats.as<LatDesc>(), m.mls.as<MLDesc>(), m.fd, h_lats[0].L3, it,
                                           m.mlbuf.as<double>(), m.tavg.as<double2>(), stream));
          if ((rc = ml_fold(l + 1, l))) return rc;
        }
      }
    }
    return U1ML_OK;
  }

  // full multilevel run, results to ml.corr (and ml.fout)
  int ml_run() {
    MLState& m = ml;
    int rc;
    U1_HIP(launch_ml_zero(m.accbuf.as<double2>(), m.acc_elems, stream));
    std::vector<uint64_t> snap_ids = h_pass_ids;
    if (m.field) U1_HIP(hipMemcpyAsync(m.snap_links.p, links.p, link_elems * elem_size(), hipMemcpyDeviceToDevice,
                                       stream));
    m.replay = 0;
    if ((rc = ml_level(0, 0))) return rc;
    if (m.field) {
      if (m.n_levels == 1)
        U1_HIP(launch_field_store_tavg(lats.as<LatDesc>(), m.mls.as<MLDesc>(), m.fd, h_lats[0].L3, 0,
                                       m.mlbuf.as<double>(), m.tavg.as<double2>(), stream));
      U1_HIP(launch_field_weights(lats.as<LatDesc>(), m.mls.as<MLDesc>(), m.fd, h_lats[0].L3, m.tavg.as<double2>(),
                                  m.accbuf.as<double2>(), m.w.as<double2>(), stream));
    }
    if ((rc = ml_fold(0, m.n_levels))) return rc;
    U1_HIP(launch_ml_final(lats.as<LatDesc>(), m.mls.as<MLDesc>(), n_lats, m.max_r, m.n_levels,
                           m.accbuf.as<double2>(), m.corr.as<double>(), stream));
    if (m.field) {
      // replay the identical update sequence, contracting the field insertion
      U1_HIP(launch_ml_zero(m.fout.as<double2>(), (uint64_t)m.fd.n_rf * 12 * h_lats[0].L * h_lats[0].L, stream));
      U1_HIP(hipMemcpyAsync(links.p, m.snap_links.p, link_elems * elem_size(), hipMemcpyDeviceToDevice, stream));
      h_pass_ids = snap_ids;
      if ((rc = upload_pass_ids())) return rc;
      m.replay = 1;
      size_t log_mark = log_used;
      bool dbg = debug;
      debug = false;  // the replay repeats decisions already recorded
      rc = ml_level(0, 0);
      debug = dbg;
      log_used = log_mark;
      m.replay = 0;
      if (rc) return rc;
      m.field_valid = true;
    }
    m.valid = true;
    return U1ML_OK;
  }
};

struct u1ml_lattice {
  Engine e;
};
struct u1ml_batch {
  Engine e;
};

namespace {

std::map<std::tuple<int, int, int>, int> g_tuned_block;  // (L, T, precision) -> block

int validate_size(int L, int T) {
  if (L < 2 || T < 2 || (L & 1) || (T & 1) || L > 256 || T > 256)
    return fail(U1ML_EINVAL, "L and T must be even and in [2, 256]");
  const uint64_t V2 = (uint64_t)L * L * L * T / 2;
  if (V2 * (uint64_t)L >= (1ull << 32) || 8 * V2 >= (1ull << 31)) return fail(U1ML_EINVAL, "lattice too large");
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
  if (!std::isfinite(o.eps) || o.eps < 0) return fail(U1ML_EINVAL, "eps must be finite and >= 0");
  if (o.block != 0 && (o.block < 64 || o.block > 1024 || (o.block % 64)))
    return fail(U1ML_EINVAL, "block must be a multiple of 64 in [64, 1024]");
  const int n = (int)L.size();
  uint64_t off = 0;
  for (int i = 0; i < n; ++i) {
    int rc = validate_size(L[i], T[i]);
    if (rc) return rc;
    if (!std::isfinite(beta[i]) || beta[i] < 0) return fail(U1ML_EINVAL, "beta must be finite and >= 0");
    e.h_lats.push_back(make_desc(L[i], T[i], beta[i], o.eps, seed[i], off));
    off += 4ull * L[i] * L[i] * L[i] * T[i];
  }
  U1_HIP(hipGetDevice(&e.device));
  e.stream = (hipStream_t)o.stream;
  if (!e.stream) {
    // a stream of our own (default priority) so that graph capture is possible
    U1_HIP(hipStreamCreateWithFlags(&e.stream, hipStreamNonBlocking));
    e.own_stream = true;
  }
  e.prec = o.precision;
  e.start = o.start;
  e.n_lats = n;
  e.link_elems = off;
  if (o.block)
    e.block = o.block;
  else {
    auto it = g_tuned_block.find(std::make_tuple(L[0], T[0], o.precision));
    e.block = it != g_tuned_block.end() ? it->second : 256;
  }
  int rc;
  if (allow_dev_buf && o.dev_buf) {
    if (o.dev_bytes < off * e.elem_size()) return fail(U1ML_EINVAL, "dev_buf smaller than u1ml_link_bytes");
    e.links.p = o.dev_buf;
    e.links.bytes = o.dev_bytes;
    e.links.owned = false;
  } else if ((rc = e.links.ensure(off * e.elem_size()))) {
    return rc;
  }
  if ((rc = e.lats.ensure(n * sizeof(LatDesc)))) return rc;
  U1_HIP(hipMemcpy(e.lats.p, e.h_lats.data(), n * sizeof(LatDesc), hipMemcpyHostToDevice));
  if ((rc = e.pass_ids.ensure(n * sizeof(uint64_t)))) return rc;
  e.h_pass_ids.assign(n, 0);
  if ((rc = e.upload_pass_ids())) return rc;
  if ((rc = e.init_links(o.start == U1ML_HOT))) return rc;
  U1_HIP(hipStreamSynchronize(e.stream));
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

int u1ml_init_lattice(int L, int T, double beta, uint64_t seed, const u1ml_options* opt, u1ml_lattice** out) {
  if (!out) return fail(U1ML_EINVAL, "out is NULL");
  *out = nullptr;
  std::unique_ptr<u1ml_lattice> lat(new (std::nothrow) u1ml_lattice());
  if (!lat) return fail(U1ML_ENOMEM, "host allocation");
  int rc = engine_create(lat->e, {L}, {T}, {beta}, {seed}, opt, true);
  if (rc) return rc;
  *out = lat.release();
  return U1ML_OK;
}

int u1ml_sweep(u1ml_lattice* lat, int n_metro, int n_or) {
  if (!lat || n_metro < 0 || n_or < 0) return fail(U1ML_EINVAL, "sweep arguments");
  int rc = lat->e.set_device();
  if (rc) return rc;
  return lat->e.sweep(n_metro, n_or, 0);
}

static int check_ml_args(const Engine& e, int n_levels, const int* th, const int* n_sub, int n_metro, int n_or) {
  if (n_levels < 1 || n_levels > U1ML_MAX_LEVELS || !th || !n_sub || n_metro < 0 || n_or < 0)
    return fail(U1ML_EINVAL, "multilevel arguments");
  for (int l = 0; l < n_levels; ++l) {
    if (th[l] < 1 || n_sub[l] < 1) return fail(U1ML_EINVAL, "slab sizes and n_sub must be >= 1");
    if (l > 0 && th[l - 1] % th[l]) return fail(U1ML_EINVAL, "each slab size must divide the previous one");
    for (auto& d : e.h_lats)
      if (d.T % th[l]) return fail(U1ML_EINVAL, "slab sizes must divide T");
  }
  return U1ML_OK;
}

int u1ml_multilevel(u1ml_lattice* lat, int n_levels, const int* slab_sizes, const int* n_sub, int n_metro, int n_or,
                    int n_r, const int* r_list, int n_rf, const int* rf_list) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  Engine& e = lat->e;
  int rc = check_ml_args(e, n_levels, slab_sizes, n_sub, n_metro, n_or);
  if (rc) return rc;
  if (n_r < 1 || !r_list) return fail(U1ML_EINVAL, "need at least one r");
  if (n_rf < 0 || n_rf > U1ML_MAX_FIELD_R || (n_rf > 0 && !rf_list)) return fail(U1ML_EINVAL, "field r list");
  if (n_rf > 0 && n_levels > 2) return fail(U1ML_EINVAL, "field insertion supports one or two levels");
  std::vector<int> rl(r_list, r_list + n_r), rf;
  for (int r : rl)
    if (r < 1 || r >= e.h_lats[0].L) return fail(U1ML_EINVAL, "r must be in [1, L)");
  for (int f = 0; f < n_rf; ++f) {
    if (std::find(rl.begin(), rl.end(), rf_list[f]) == rl.end())
      return fail(U1ML_EINVAL, "every field r must appear in r_list");
    rf.push_back(rf_list[f]);
  }
  if ((rc = e.set_device())) return rc;
  if ((rc = e.ml_setup(n_levels, slab_sizes, n_sub, n_metro, n_or, {rl}, rf))) return rc;
  return e.ml_run();
}

int u1ml_measure(u1ml_lattice* lat, u1ml_observables* obs, double* correlator, double* field_profile) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  Engine& e = lat->e;
  int rc = e.set_device();
  if (rc) return rc;
  if ((correlator && !e.ml.valid) || (field_profile && !e.ml.field_valid))
    return fail(U1ML_ESTATE, "no multilevel result of that kind yet");
  if (obs) {
    std::vector<u1ml_observables> res;
    if ((rc = e.observables(res))) return rc;
    *obs = res[0];
  }
  U1_HIP(hipStreamSynchronize(e.stream));
  if (correlator)
    U1_HIP(hipMemcpy(correlator, e.ml.corr.p, e.ml.nR[0] * 2 * sizeof(double), hipMemcpyDeviceToHost));
  if (field_profile) {
    const int L = e.h_lats[0].L;
    U1_HIP(hipMemcpy(field_profile, e.ml.fout.p, (size_t)e.ml.fd.n_rf * 12 * L * L * 2 * sizeof(double),
                     hipMemcpyDeviceToHost));
  }
  return U1ML_OK;
}

int u1ml_plain_correlator(u1ml_lattice* lat, int n_r, const int* r_list, double* out) {
  if (!lat || n_r < 1 || !r_list || !out) return fail(U1ML_EINVAL, "plain_correlator arguments");
  Engine& e = lat->e;
  std::vector<int> rl(r_list, r_list + n_r);
  for (int r : rl)
    if (r < 0 || r >= e.h_lats[0].L) return fail(U1ML_EINVAL, "r must be in [0, L)");
  int rc = e.set_device();
  if (rc) return rc;
  std::vector<std::vector<double>> pc;
  if ((rc = e.poly_corr(rl, pc))) return rc;
  for (int k = 0; k < n_r; ++k) {
    out[2 * k] = pc[0][2 + 2 * k];
    out[2 * k + 1] = pc[0][3 + 2 * k];
  }
  return U1ML_OK;
}

int u1ml_get_links(u1ml_lattice* lat, double* host) {
  if (!lat || !host) return fail(U1ML_EINVAL, "get_links arguments");
  int rc = lat->e.set_device();
  return rc ? rc : lat->e.get_links(0, host);
}

int u1ml_set_links(u1ml_lattice* lat, const double* host) {
  if (!lat || !host) return fail(U1ML_EINVAL, "set_links arguments");
  int rc = lat->e.set_device();
  return rc ? rc : lat->e.set_links(0, host);
}

int u1ml_get_pass_id(u1ml_lattice* lat, uint64_t* pass_id) {
  if (!lat || !pass_id) return fail(U1ML_EINVAL, "get_pass_id arguments");
  *pass_id = lat->e.h_pass_ids[0];
  return U1ML_OK;
}

int u1ml_set_pass_id(u1ml_lattice* lat, uint64_t pass_id) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  int rc = lat->e.set_device();
  if (rc) return rc;
  lat->e.h_pass_ids[0] = pass_id;
  return lat->e.upload_pass_ids();
}

int u1ml_set_debug(u1ml_lattice* lat, unsigned flags, size_t capacity) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  Engine& e = lat->e;
  int rc = e.set_device();
  if (rc) return rc;
  U1_HIP(hipStreamSynchronize(e.stream));
  if (flags & 1u) {
    if ((rc = e.log.ensure(capacity))) return rc;
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
  int rc = e.set_device();
  if (rc) return rc;
  U1_HIP(hipStreamSynchronize(e.stream));
  if (n_bytes) *n_bytes = e.log_used;
  size_t n = std::min(cap, e.log_used);
  if (out && n) U1_HIP(hipMemcpy(out, e.log.p, n, hipMemcpyDeviceToHost));
  return U1ML_OK;
}

int u1ml_save(u1ml_lattice* lat, const char* path) {
  if (!lat || !path) return fail(U1ML_EINVAL, "save arguments");
  Engine& e = lat->e;
  const LatDesc& d = e.h_lats[0];
  std::vector<double> h(8ull * d.V2);
  int rc = e.set_device();
  if (rc || (rc = e.get_links(0, h.data()))) return rc;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(U1ML_EIO, std::string("cannot open ") + path);
  std::fprintf(f, "u1ml-checkpoint-1 L=%d T=%d beta=%.17g eps=%.17g seed=%llu pass_id=%llu precision=%d\n", d.L, d.T,
               d.beta, d.eps, (unsigned long long)d.seed, (unsigned long long)e.h_pass_ids[0], e.prec);
  size_t w = std::fwrite(h.data(), sizeof(double), h.size(), f);
  int cl = std::fclose(f);
  if (w != h.size() || cl != 0) return fail(U1ML_EIO, "short write");
  return U1ML_OK;
}

int u1ml_load(u1ml_lattice* lat, const char* path) {
  if (!lat || !path) return fail(U1ML_EINVAL, "load arguments");
  Engine& e = lat->e;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(U1ML_EIO, std::string("cannot open ") + path);
  char line[512];
  if (!std::fgets(line, sizeof line, f)) {
    std::fclose(f);
    return fail(U1ML_EIO, "missing header");
  }
  int L = 0, T = 0, prec = -1;
  double beta = 0, eps = 0;
  unsigned long long seed = 0, pid = 0;
  if (std::sscanf(line, "u1ml-checkpoint-1 L=%d T=%d beta=%lg eps=%lg seed=%llu pass_id=%llu precision=%d", &L, &T,
                  &beta, &eps, &seed, &pid, &prec) != 7) {
    std::fclose(f);
    return fail(U1ML_EIO, "bad header");
  }
  LatDesc& d = e.h_lats[0];
  if (L != d.L || T != d.T || prec != e.prec) {
    std::fclose(f);
    return fail(U1ML_EINVAL, "checkpoint shape or precision differs from the lattice");
  }
  std::vector<double> h(8ull * d.V2);
  size_t r = std::fread(h.data(), sizeof(double), h.size(), f);
  std::fclose(f);
  if (r != h.size()) return fail(U1ML_EIO, "short read");
  int rc = e.set_device();
  if (rc) return rc;
  d.beta = beta;
  d.eps = eps;
  d.sqrt_beta = std::sqrt(beta);
  d.seed = seed;
  U1_HIP(hipMemcpy(e.lats.p, e.h_lats.data(), sizeof(LatDesc), hipMemcpyHostToDevice));
  e.h_pass_ids[0] = pid;
  if ((rc = e.upload_pass_ids())) return rc;
  return e.set_links(0, h.data());
}

int u1ml_synchronize(u1ml_lattice* lat) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  int rc = lat->e.set_device();
  if (rc) return rc;
  U1_HIP(hipStreamSynchronize(lat->e.stream));
  return U1ML_OK;
}

void u1ml_destroy(u1ml_lattice* lat) {
  if (!lat) return;
  (void)hipSetDevice(lat->e.device);
  (void)hipStreamSynchronize(lat->e.stream);
  delete lat;
}

// --- batches ---
int u1ml_batch_create(int n, const int* L, const int* T, const double* beta, const uint64_t* seed,
                      const u1ml_options* opt, u1ml_batch** out) {
  if (!out || n < 1 || !L || !T || !beta || !seed) return fail(U1ML_EINVAL, "batch_create arguments");
  *out = nullptr;
  std::unique_ptr<u1ml_batch> b(new (std::nothrow) u1ml_batch());
  if (!b) return fail(U1ML_ENOMEM, "host allocation");
  int rc = engine_create(b->e, std::vector<int>(L, L + n), std::vector<int>(T, T + n),
                         std::vector<double>(beta, beta + n), std::vector<uint64_t>(seed, seed + n), opt, false);
  if (rc) return rc;
  *out = b.release();
  return U1ML_OK;
}

int u1ml_batch_sweep(u1ml_batch* b, int n_metro, int n_or) {
  if (!b || n_metro < 0 || n_or < 0) return fail(U1ML_EINVAL, "batch_sweep arguments");
  int rc = b->e.set_device();
  return rc ? rc : b->e.sweep(n_metro, n_or, 0);
}

static int batch_cycle_eager(Engine& e, int n_sweeps, int n_metro, int n_or) {
  int rc;
  for (int s = 0; s < n_sweeps; ++s)
    if ((rc = e.sweep(n_metro, n_or, 0))) return rc;
  return e.ml_run();
}

int u1ml_batch_cycle(u1ml_batch* b, int n_sweeps, int n_metro, int n_or, int th, int n_sub, int use_graph) {
  if (!b || n_sweeps < 0) return fail(U1ML_EINVAL, "batch_cycle arguments");
  Engine& e = b->e;
  int rc = check_ml_args(e, 1, &th, &n_sub, n_metro, n_or);
  if (rc) return rc;
  if ((rc = e.set_device())) return rc;
  std::vector<int> key{n_sweeps, n_metro, n_or, th, n_sub};
  const bool have_graph = e.graph_exec && e.graph_key == key && !e.debug;
  if (!have_graph) {
    std::vector<std::vector<int>> rl(e.n_lats);
    for (int i = 0; i < e.n_lats; ++i)
      for (int r = 1; r <= e.h_lats[i].T / 2 && r < e.h_lats[i].L; ++r) rl[i].push_back(r);
    if ((rc = e.ml_setup(1, &th, &n_sub, n_metro, n_or, rl, {}))) return rc;
    if ((rc = batch_cycle_eager(e, n_sweeps, n_metro, n_or))) return rc;
    if (use_graph && !e.debug) {
      // capture the same cycle for later calls; all buffers and tables exist now
      if (e.graph_exec) {
        (void)hipGraphExecDestroy(e.graph_exec);
        e.graph_exec = nullptr;
      }
      std::vector<uint64_t> ids = e.h_pass_ids;
      hipGraph_t g;
      U1_HIP(hipStreamBeginCapture(e.stream, hipStreamCaptureModeThreadLocal));
      rc = batch_cycle_eager(e, n_sweeps, n_metro, n_or);
      hipError_t ce = hipStreamEndCapture(e.stream, &g);
      if (rc) return rc;
      if (ce != hipSuccess) return fail(U1ML_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
      e.graph_metro_passes = (int)(e.h_pass_ids[0] - ids[0]);
      e.h_pass_ids = ids;  // capture did not run anything
      hipError_t ie = hipGraphInstantiate(&e.graph_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        e.graph_exec = nullptr;
        return fail(U1ML_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
      }
      e.graph_key = key;
    }
    return U1ML_OK;
  }
  U1_HIP(hipGraphLaunch(e.graph_exec, e.stream));
  for (auto& v : e.h_pass_ids) v += e.graph_metro_passes;
  e.ml.valid = true;
  return U1ML_OK;
}

int u1ml_batch_measure(u1ml_batch* b, int i, u1ml_observables* obs, double* correlator) {
  if (!b || i < 0 || i >= b->e.n_lats) return fail(U1ML_EINVAL, "batch_measure arguments");
  Engine& e = b->e;
  int rc = e.set_device();
  if (rc) return rc;
  if (correlator && !e.ml.valid) return fail(U1ML_ESTATE, "no cycle has run yet");
  if (obs) {
    std::vector<u1ml_observables> res;
    if ((rc = e.observables(res))) return rc;
    *obs = res[i];
  }
  U1_HIP(hipStreamSynchronize(e.stream));
  if (correlator)
    U1_HIP(hipMemcpy(correlator, e.ml.corr.as<double>() + (size_t)i * e.ml.max_r * 2, e.ml.nR[i] * 2 * sizeof(double),
                     hipMemcpyDeviceToHost));
  return U1ML_OK;
}

int u1ml_batch_get_links(u1ml_batch* b, int i, double* host) {
  if (!b || i < 0 || i >= b->e.n_lats || !host) return fail(U1ML_EINVAL, "batch_get_links arguments");
  int rc = b->e.set_device();
  return rc ? rc : b->e.get_links(i, host);
}

int u1ml_batch_set_links(u1ml_batch* b, int i, const double* host) {
  if (!b || i < 0 || i >= b->e.n_lats || !host) return fail(U1ML_EINVAL, "batch_set_links arguments");
  int rc = b->e.set_device();
  return rc ? rc : b->e.set_links(i, host);
}

int u1ml_batch_synchronize(u1ml_batch* b) {
  if (!b) return fail(U1ML_EINVAL, "batch is NULL");
  int rc = b->e.set_device();
  if (rc) return rc;
  U1_HIP(hipStreamSynchronize(b->e.stream));
  return U1ML_OK;
}

void u1ml_batch_destroy(u1ml_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->e.device);
  (void)hipStreamSynchronize(b->e.stream);
  delete b;
}

int u1ml_autotune(u1ml_lattice* lat, int* best_block) {
  if (!lat) return fail(U1ML_EINVAL, "lattice is NULL");
  Engine& e = lat->e;
  int rc = e.set_device();
  if (rc) return rc;
  if (e.debug) return fail(U1ML_ESTATE, "autotune with the debug log enabled");
  DevBuf save;
  if ((rc = save.ensure(e.link_elems * e.elem_size()))) return rc;
  U1_HIP(hipMemcpyAsync(save.p, e.links.p, e.link_elems * e.elem_size(), hipMemcpyDeviceToDevice, e.stream));
  const std::vector<uint64_t> ids = e.h_pass_ids;
  hipEvent_t a, z;
  U1_HIP(hipEventCreate(&a));
  U1_HIP(hipEventCreate(&z));
  const int cand[] = {64, 128, 256, 512, 1024};
  float best_ms = 1e30f;
  int best = e.block;
  for (int blk : cand) {
    e.block = blk;
    if ((rc = e.sweep(1, 1, 0))) break;  // warm-up (builds the table)
    (void)hipEventRecord(a, e.stream);
    for (int k = 0; k < 3; ++k)
      if ((rc = e.sweep(1, 3, 0))) break;
    (void)hipEventRecord(z, e.stream);
    (void)hipEventSynchronize(z);
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
  U1_HIP(hipMemcpyAsync(e.links.p, save.p, e.link_elems * e.elem_size(), hipMemcpyDeviceToDevice, e.stream));
  e.h_pass_ids = ids;
  int rc2 = e.upload_pass_ids();
  if (rc) return rc;
  if (rc2) return rc2;
  g_tuned_block[std::make_tuple(e.h_lats[0].L, e.h_lats[0].T, e.prec)] = best;
  if (best_block) *best_block = best;
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
