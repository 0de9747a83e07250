// Host runtime of the GCP-CROWN library: argument validation, packing of
// networks / cuts / splits into device layouts, workspace management, and
// the launch schedules of the bound pass (Theorem 3.1), its adjoint and the
// projected Adam loop (Appendix C.1).  Everything below the C ABI runs on
// the caller's stream; no host synchronisation inside gcp_bound/gcp_optimize
// unless GCP_FLAG_VALIDATE is set.
#include "../../include/gcp.h"
#include "gcp_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

using namespace gcp;

namespace {

thread_local std::string g_err;
// Set while this thread runs an entry point that must not allocate: no
// autotuning trials (they need scratch outputs and a host wait) and no
// profiler events.
thread_local bool g_no_alloc = false;
struct NoAllocScope {
  NoAllocScope() { g_no_alloc = true; }
  ~NoAllocScope() { g_no_alloc = false; }
};

struct Err {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& m) { throw Err{code, m}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? GCP_ENOMEM : GCP_EDEVICE,
                            std::string(what) + ": " + hipGetErrorString(e));
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Workspace generations are unique across nets, so a cached launch table or
// graph keyed by (handle address, generation) never matches a new net that
// reuses a freed address.
uint64_t next_generation() {
  static std::atomic<uint64_t> g{1};
  return g.fetch_add(1);
}

// ------------------------------------------------------------------ profiler
// Process-wide record of kernel launches bracketed by HIP events (only while
// enabled).  Aggregation happens at read time.
struct Profiler {
  std::mutex mu;
  bool on = false;
  struct Rec { int cls; hipEvent_t e0, e1; double bytes, alg, flops; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  std::vector<std::string> names;
  std::map<std::string, int> ids;
  struct Agg { int64_t n = 0; double ms = 0, bytes = 0, alg = 0, flops = 0; };
  std::vector<Agg> agg;
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    return e;
  }
  void flush() {   // fold recorded events into the aggregates
    for (auto& r : recs) {
      hip_check(hipEventSynchronize(r.e1), "hipEventSynchronize");
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, r.e0, r.e1), "hipEventElapsedTime");
      if ((int)agg.size() <= r.cls) agg.resize(r.cls + 1);
      agg[r.cls].n++; agg[r.cls].ms += ms; agg[r.cls].bytes += r.bytes; agg[r.cls].alg += r.alg;
      agg[r.cls].flops += r.flops;
      pool.push_back(r.e0); pool.push_back(r.e1);
    }
    recs.clear();
  }
};
Profiler& prof() { static Profiler p; return p; }

// HBM bytes of one launch under two models: `all` = every operand read once
// and every result written once (what a launch must move when nothing stays
// on chip between launches); `alg` = the optimiser-state traffic the method
// itself needs (alpha / rho read in the bound pass, alpha / rho and their Adam
// moments read and written in the adjoint, multipliers and their moments in
// the multiplier update, the split mask), 0 for launches that carry none.
struct Bytes { double all, alg; };

// Launch `f` on `st`; while profiling, bracket it with events under `name`.
template <class F>
hipError_t timed(hipStream_t st, const std::string& name, Bytes bytes, double flops, F f) {
  Profiler& P = prof();
  if (!P.on || g_no_alloc) return f();
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(st, &cs);
  if (cs != hipStreamCaptureStatusNone) return f();   // graph replays are not timed per kernel
  std::lock_guard<std::mutex> lk(P.mu);
  hipEvent_t e0 = P.get(), e1 = P.get();
  hip_check(hipEventRecord(e0, st), "hipEventRecord");
  hipError_t err = f();
  hip_check(hipEventRecord(e1, st), "hipEventRecord");
  auto it = P.ids.find(name);
  int cls;
  if (it == P.ids.end()) { cls = (int)P.names.size(); P.ids[name] = cls; P.names.push_back(name); }
  else cls = it->second;
  P.recs.push_back(Profiler::Rec{cls, e0, e1, bytes.all, bytes.alg, flops});
  return err;
}

std::string cls_name(const char* kind, int bf16, int sign, int cfg) {
  int bm = 0, bn = 0;
  if (cfg >= 0) gemm_config_tile(cfg, &bm, &bn);
  std::string n = std::string(kind) + (bf16 ? ".bf16" : ".fp32") + (sign ? ".sign" : "");
  if (cfg >= 0) n += ".t" + std::to_string(bm) + "x" + std::to_string(bn);
  return n;
}

// Tile configuration an explicit-pi bound/adjoint GEMM runs with (the
// launcher instantiates those epilogues for the small tiles only).
int pi_cfg(int cfg) { return (cfg == 6 || cfg == 7) ? cfg : 5; }

// Owned device allocation (zero-filled at allocation), or a borrowed view of
// memory owned elsewhere (never freed here).  The fill and uploads run on the
// null stream and are waited for before returning: callers' streams may be
// non-blocking (no implicit order with the null stream), and their work on a
// new buffer must not race its clear.  A free first waits for the device, as
// work in flight on any stream may still use the buffer.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = true;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned) { o.p = nullptr; o.bytes = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; owned = o.owned;
      o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p && owned) {
      (void)hipDeviceSynchronize();
      (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
    owned = true;
  }
  void borrow(void* q, size_t n) {
    release();
    p = q;
    bytes = n;
    owned = false;
  }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    hip_check(hipMalloc(&p, n), "hipMalloc");
    bytes = n;
    hip_check(hipMemset(p, 0, n), "hipMemset");
    hip_check(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
  }
  void ensure(size_t n) {
    if (n > bytes) alloc(n);
  }
  template <class T> void upload(const std::vector<T>& v) {
    alloc(v.size() * sizeof(T));
    if (v.empty()) return;
    hip_check(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
    hip_check(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
  }
  template <class T> T* as() const { return (T*)p; }
};

// A recorded iteration schedule laid out for the persistent dataflow kernel
// (tables in one device buffer) and its synchronisation words.
struct PersistPlan {
  std::vector<uintptr_t> key;
  DBuf buf;          // steps, per-queue first items, GEMM arguments, epilogue blobs, elementwise and gamma jobs
  DBuf sync;         // claim heads, abort flag, panel counters (zeroed before every launch)
  size_t n_sync = 0;
  DBuf latch;        // set by a launch that aborted (zeroed once per call)
  PersistArgs args{};
  int grid = 0;
  int max_items = 0;   // most items one queue has in one iteration
  double bytes = 0.0, alg = 0.0, flops = 0.0;   // per iteration, both byte models and the GEMM FLOPs
};

struct EdgeH {
  int src, dst, kind;
  int kh = 0, kw = 0, stride = 1, pad = 0;
  int d_src = 0, d_dst = 0;
  ConvGeom cg{};
  DBuf W32;      // adjoint Bt: dense [d_dst][ld_src]; conv [co][ldk_f]
  DBuf W16;
  DBuf WT32;     // bound Bt: dense [d_src][ld_dst]; conv [ci][ldk_t]
  DBuf WT16;
  DBuf WT16f;    // conv: WT16's values as fp32 (read by the direct transposed conv in bf16 mode)
  DBuf Wraw;     // dense [d_dst][d_src] unpadded fp32 (for c-hat and W x0); conv: [co][ci][kh][kw]
  int ldk_f = 0, ldk_t = 0;   // conv: padded K of W32/W16 (adjoint) and WT32/WT16 (bound)
};

struct NodeH {
  int c, h, w, size, ld;
  bool relu;
  std::vector<int> in_edges;      // edges whose dst is this node
  std::vector<int> consumers;     // edges whose src is this node
  DBuf bias, rec, kind;
  std::vector<int32_t> rank_h;    // host copy of rank
  std::vector<double> l_h, u_h;   // host copies of the root bounds (as given)
  // outward rounding: Z = max(|l|, |u|) and Y = the largest |x_hat| the
  // relaxation faces (0 inactive, u active, max(-l, u) unstable), both from
  // the fp32 bounds the device holds
  std::vector<double> z_h, y_h;
  DBuf slack_w;                   // fp64 [5][ld]: the node's outward-rounding weights
  int n_unst = 0, rank0 = 0;
  NodeDev dev() const { return NodeDev{size, ld, rec.as<float4>(), kind.as<int32_t>()}; }
};

}  // namespace

struct gcp_net {
  ~gcp_net() {
    if (ws.gexec) (void)hipGraphExecDestroy(ws.gexec);
    if (ws.gstream) (void)hipStreamDestroy(ws.gstream);
  }
  int device = 0;
  int in_c, in_h, in_w, in_size, in_ld;
  std::vector<NodeH> nodes;
  std::vector<std::unique_ptr<EdgeH>> edges;
  int64_t n_relu = 0;
  int n_I = 0;
  int out = 0;
  // input consumers (edges with src = -1)
  std::vector<int> in_consumers;
  // the output's Lambda (= C) is materialised and pushed like any node's,
  // instead of the c-hat shortcut (C W precomputed, fused relaxation of the
  // nodes feeding the output): needed for conv edges into the output, an
  // output fed by the input, or a node feeding the output that has other
  // consumers
  bool out_general = false;
  // ---- workspace (grown on demand)
  struct WS {
    int M = 0, S = 0, nnz = 0, N = 0;
    std::vector<std::unique_ptr<DBuf>> lam, ahat, dahat, acc, addv;
    DBuf sign, partial, contrib, chat, cb, consts, step, flags, acc_in, gammaT;
    DBuf adam_tab;   // Adam constants of every iteration of a gcp_optimize call, [iters][4]
    DBuf chain_tab;  // per-node tables of the fused chain launch (ChainNode [L])
    std::vector<ChainNode> chain_host;
    DBuf tune_store, tune_alpha, tune_beta;   // autotuner trial outputs (lazy)
    DBuf ahat_tmp;      // a_hat of the node being differentiated, when recomputed
    DBuf slackw;        // outward rounding: combined weights of every node, then X_in
    // captured Adam iteration of gcp_optimize (valid for one argument set)
    hipStream_t gstream = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<uintptr_t> gkey;
    // persistent dataflow launch of gcp_optimize's iterations (one argument set)
    std::unique_ptr<PersistPlan> pplan;
    uint64_t gen = 0;   // new process-unique value whenever a workspace buffer is reallocated
    std::vector<int> chat_off;   // offset (floats) of each node's c-hat block
    int n_slots = 0;
  } ws;
};

struct gcp_cuts {
  // process-unique: cached launch tables and graphs key on it, so a handle
  // created at the address of a destroyed one never matches their entries
  uint64_t id = next_generation();
  int N = 0;
  int nnz_e = 0;
  DBuf row_ptr;     // [N + 1] over merged entries in cut-major order
  DBuf d;           // fp64 [N]
  struct Col {
    DBuf rng, ent, pos;
    bool any = false;
    CutCol dev() const {
      if (!any) return CutCol{nullptr, nullptr, nullptr};
      return CutCol{rng.as<int2>(), ent.as<float4>(), pos.as<int32_t>()};
    }
  };
  std::vector<Col> cols;   // per node; index n_nodes is the network input
  std::vector<int> nnz_node;   // merged entries per node (same indexing)
  // outward rounding: fp64 [3][N] = sum |coef| range over a cut's node
  // entries (range Z for H and G, 2 for Q), sum |coef| over its input
  // entries (times X_in per call), |d|; and the most entries of one column
  DBuf kap;
  int col_max = 0;
  const gcp_net* net = nullptr;
};

struct gcp_splits {
  uint64_t id = next_generation();   // process-unique (see gcp_cuts::id)
  int B = 0, K = 0;
  DBuf mask;        // int8 [B][n_I]
  DBuf zsplit;      // fp64 [B][K]: max(|l|, |u|) of slot k's neuron (0: unused slot), for outward rounding
  // host staging of splits_assign (kept until the handle is refilled again)
  std::vector<int8_t> mask_h;
  std::vector<double> zs_h;
  const gcp_net* net = nullptr;
};

namespace {

// ------------------------------------------------------------------ helpers

float round_down_f(double x) {
  float f = (float)x;
  if ((double)f > x) f = std::nextafter(f, -INFINITY);
  return f;
}
float round_up_f(double x) {
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, INFINITY);
  return f;
}

void check_finite(const float* p, size_t n, const char* what) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) fail(GCP_ENONFINITE, std::string(what) + " has a non-finite value");
}

std::vector<uint16_t> to_bf16(const std::vector<float>& v) {
  // round to nearest even
  std::vector<uint16_t> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    uint32_t b;
    std::memcpy(&b, &v[i], 4);
    uint32_t lsb = (b >> 16) & 1u;
    b += 0x7fffu + lsb;
    o[i] = (uint16_t)(b >> 16);
  }
  return o;
}

std::vector<float> bf16_as_f32(const std::vector<uint16_t>& v) {
  std::vector<float> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    const uint32_t b = (uint32_t)v[i] << 16;
    std::memcpy(&o[i], &b, 4);
  }
  return o;
}

int node_size_of(const gcp_net* net, int src) { return src < 0 ? net->in_size : net->nodes[src].size; }
int node_ld_of(const gcp_net* net, int src) { return src < 0 ? net->in_ld : net->nodes[src].ld; }

// ------------------------------------------------------------------ net create

// Accumulation bound of a K-term fp32 sum, K u / (1 - K u), with u = 2^-23:
// twice the unit roundoff of round-to-nearest, so that the bound also holds
// if the matrix cores round their internal steps another way.
double acc_bound(double K) {
  const double u = 0x1p-23;
  return K * u / (1.0 - K * u);
}

// The five outward-rounding weight vectors of every node (w0..w4 of
// SlackArgs).  Column j of a source p collects the terms of all of p's
// consumer edges, plus one addition per edge and the cut and relaxation
// terms: K_p = sum of the edges' terms + edges + 4.
void build_slack_weights(gcp_net* net, const std::vector<std::vector<double>>& e_wy,
                         const std::vector<double>& e_terms) {
  const int nn = (int)net->nodes.size();
  std::vector<double> kp(nn + 1, 4.0);   // index nn: the input
  for (size_t e = 0; e < net->edges.size(); ++e) {
    const int p = net->edges[e]->src;
    kp[p < 0 ? nn : p] += e_terms[e] + 1.0;
  }
  const double margin = 1.0 + 0x1p-30;   // covers the rounding of these host sums
  for (int i = 0; i < nn; ++i) {
    NodeH& n = net->nodes[i];
    std::vector<double> w((size_t)5 * n.ld, 0.0);
    for (int eid : n.in_edges) {
      const int p = net->edges[eid]->src;
      const double g = acc_bound(kp[p < 0 ? nn : p]);
      const std::vector<double>& wy = e_wy[eid];
      for (int k = 0; k < n.size; ++k) {
        if (p >= 0) {
          w[k] += g * wy[k];
          w[(size_t)n.ld + k] += wy[k];
        } else {
          w[(size_t)3 * n.ld + k] += g * wy[k];
          w[(size_t)4 * n.ld + k] += wy[k];
        }
      }
    }
    std::vector<float> b(n.size);
    hip_check(hipMemcpy(b.data(), n.bias.p, (size_t)n.size * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    for (int k = 0; k < n.size; ++k) w[(size_t)2 * n.ld + k] = (n.relu ? n.z_h[k] : 0.0) + std::fabs((double)b[k]);
    for (double& v : w) v *= margin;
    n.slack_w.upload(w);
  }
}

void build_net(const gcp_net_desc* d, gcp_net* net) {
  if (!d || !d->nodes) fail(GCP_EINVAL, "null network description");
  if (d->n_nodes < 1) fail(GCP_EINVAL, "a network needs an output node");
  if (d->in_c <= 0 || d->in_h <= 0 || d->in_w <= 0) fail(GCP_EINVAL, "bad input shape");
  hip_check(hipGetDevice(&net->device), "hipGetDevice");
  net->in_c = d->in_c; net->in_h = d->in_h; net->in_w = d->in_w;
  net->in_size = d->in_c * d->in_h * d->in_w;
  net->in_ld = round_up(net->in_size, 16);
  net->nodes.resize(d->n_nodes);
  net->out = d->n_nodes - 1;
  int rank0 = 0;
  // outward rounding, per edge: |W| Y_src (|W| 1 from the input) and the
  // number of terms one source column accumulates through the edge
  std::vector<std::vector<double>> e_wy;
  std::vector<double> e_terms;
  for (int i = 0; i < d->n_nodes; ++i) {
    const gcp_node_desc& nd = d->nodes[i];
    NodeH& n = net->nodes[i];
    if (nd.c <= 0 || nd.h <= 0 || nd.w <= 0) fail(GCP_EINVAL, "bad node shape at node " + std::to_string(i));
    n.c = nd.c; n.h = nd.h; n.w = nd.w;
    n.size = nd.c * nd.h * nd.w;
    n.ld = round_up(n.size, 16);
    n.relu = (i != net->out);
    if (!nd.bias) fail(GCP_EINVAL, "null bias at node " + std::to_string(i));
    check_finite(nd.bias, n.size, "bias");
    std::vector<float> b(nd.bias, nd.bias + n.size);
    n.bias.upload(b);
    std::vector<float4> rec(n.size);
    std::vector<int32_t> kind(n.size, 0);
    for (int j = 0; j < n.size; ++j) rec[j] = make_float4(0.f, 0.f, 0.f, b[j]);
    if (nd.n_edges <= 0 || !nd.edges) fail(GCP_EINVAL, "node " + std::to_string(i) + " has no input edge");
    if (n.relu) {
      if (!nd.lower || !nd.upper) fail(GCP_EINVAL, "missing root bounds at node " + std::to_string(i));
      std::vector<float> l(n.size), u(n.size), iul(n.size, 0.f);
      std::vector<int8_t> cls(n.size);
      std::vector<int32_t> rank(n.size, -1);
      n.rank0 = rank0;
      for (int j = 0; j < n.size; ++j) {
        double lo = nd.lower[j], hi = nd.upper[j];
        if (!std::isfinite(lo) || !std::isfinite(hi)) fail(GCP_ENONFINITE, "non-finite root bound");
        if (lo > hi) fail(GCP_EINVAL, "root bound l > u at node " + std::to_string(i));
        l[j] = round_down_f(lo);
        u[j] = round_up_f(hi);
        if (lo >= 0) cls[j] = ACTIVE;
        else if (hi <= 0) cls[j] = INACTIVE;
        else {
          cls[j] = UNSTABLE;
          rank[j] = rank0++;
          iul[j] = (float)(1.0 / ((double)u[j] - (double)l[j]));
        }
      }
      n.n_unst = rank0 - n.rank0;
      for (int j = 0; j < n.size; ++j) {
        rec[j] = make_float4(l[j], u[j], iul[j], b[j]);
        kind[j] = (rank[j] + 1) * 4 + cls[j];
      }
      n.rank_h = rank;
      n.l_h.assign(nd.lower, nd.lower + n.size);
      n.u_h.assign(nd.upper, nd.upper + n.size);
      n.z_h.resize(n.size);
      n.y_h.resize(n.size);
      for (int j = 0; j < n.size; ++j) {
        const double lo = l[j], hi = u[j];
        n.z_h[j] = std::max(std::fabs(lo), std::fabs(hi));
        n.y_h[j] = cls[j] == INACTIVE ? 0.0 : (cls[j] == ACTIVE ? hi : std::max(-lo, hi));
      }
      net->n_relu += n.size;
    }
    n.rec.upload(rec);
    n.kind.upload(kind);
    for (int e = 0; e < nd.n_edges; ++e) {
      const gcp_edge_desc& ed = nd.edges[e];
      if (ed.src < -1 || ed.src >= i) fail(GCP_EINVAL, "edge source must be an earlier node or the input");
      if (ed.src >= 0 && !net->nodes[ed.src].relu) fail(GCP_EINVAL, "edge from the output node");
      auto E = std::make_unique<EdgeH>();
      E->src = ed.src; E->dst = i; E->kind = ed.kind;
      E->d_src = node_size_of(net, ed.src);
      E->d_dst = n.size;
      int ld_src = node_ld_of(net, ed.src);
      if (ed.kind == GCP_EDGE_DENSE) {
        if (!ed.W) fail(GCP_EINVAL, "null dense weight");
        size_t cnt = (size_t)E->d_dst * E->d_src;
        check_finite(ed.W, cnt, "weight");
        std::vector<float> raw(ed.W, ed.W + cnt);
        std::vector<float> fw((size_t)E->d_dst * ld_src, 0.f), ft((size_t)E->d_src * n.ld, 0.f);
        for (int o = 0; o < E->d_dst; ++o)
          for (int k = 0; k < E->d_src; ++k) {
            float w = raw[(size_t)o * E->d_src + k];
            fw[(size_t)o * ld_src + k] = w;
            ft[(size_t)k * n.ld + o] = w;
          }
        E->Wraw.upload(raw);
        E->W32.upload(fw); E->W16.upload(to_bf16(fw));
        E->WT32.upload(ft); E->WT16.upload(to_bf16(ft));
        std::vector<double> wy(E->d_dst, 0.0);
        for (int o = 0; o < E->d_dst; ++o)
          for (int k = 0; k < E->d_src; ++k)
            wy[o] += std::fabs((double)raw[(size_t)o * E->d_src + k]) * (ed.src < 0 ? 1.0 : net->nodes[ed.src].y_h[k]);
        e_wy.push_back(std::move(wy));
        e_terms.push_back(E->d_dst);
      } else if (ed.kind == GCP_EDGE_CONV) {
        if (!ed.W) fail(GCP_EINVAL, "null conv weight");
        int ci, hi, wi;
        if (ed.src < 0) { ci = net->in_c; hi = net->in_h; wi = net->in_w; }
        else { ci = net->nodes[ed.src].c; hi = net->nodes[ed.src].h; wi = net->nodes[ed.src].w; }
        if (ed.kh <= 0 || ed.kw <= 0 || ed.stride <= 0 || ed.pad < 0) fail(GCP_EINVAL, "bad conv geometry");
        int ho = (hi + 2 * ed.pad - ed.kh) / ed.stride + 1;
        int wo = (wi + 2 * ed.pad - ed.kw) / ed.stride + 1;
        if (ho != n.h || wo != n.w) fail(GCP_EINVAL, "conv output shape does not match node " + std::to_string(i));
        E->kh = ed.kh; E->kw = ed.kw; E->stride = ed.stride; E->pad = ed.pad;
        E->cg = ConvGeom{ci, hi, wi, n.c, ho, wo, ed.kh, ed.kw, ed.stride, ed.pad};
        size_t cnt = (size_t)n.c * ci * ed.kh * ed.kw;
        check_finite(ed.W, cnt, "conv weight");
        std::vector<float> raw(ed.W, ed.W + cnt);
        E->Wraw.upload(raw);
        // kernel layouts: adjoint [co][ldk_f], bound [phase][ci][ldk_t]
        const int kf = conv_ldb(E->cg, 0), kt = conv_ldb(E->cg, 1);
        const int nph = ed.stride * ed.stride;
        std::vector<float> fw((size_t)n.c * kf), ft((size_t)nph * ci * kt);
        conv_pack_weights(E->cg, 0, raw.data(), fw.data());
        conv_pack_weights(E->cg, 1, raw.data(), ft.data());
        const ConvPlan pf = conv_plan(E->cg, 0), pt = conv_plan(E->cg, 1);
        if (pf.rows_max * pf.Wp * pf.Kch * 4 > 48 * 1024 || pt.rows_max * pt.Wp * pt.Kch * 4 > 48 * 1024)
          fail(GCP_EUNSUPPORTED, "conv rows too wide for an LDS slab");
        E->ldk_f = kf;
        E->ldk_t = kt;
        E->W32.upload(fw); E->W16.upload(to_bf16(fw));
        E->WT32.upload(ft); E->WT16.upload(to_bf16(ft));
        E->WT16f.upload(bf16_as_f32(to_bf16(ft)));
        std::vector<double> wy(E->d_dst, 0.0);
        for (int o = 0; o < n.c; ++o)
          for (int y = 0; y < ho; ++y)
            for (int x = 0; x < wo; ++x) {
              double t = 0.0;
              for (int cc = 0; cc < ci; ++cc)
                for (int ky = 0; ky < ed.kh; ++ky)
                  for (int kx = 0; kx < ed.kw; ++kx) {
                    const int iy = y * ed.stride - ed.pad + ky, ix = x * ed.stride - ed.pad + kx;
                    if (iy < 0 || iy >= hi || ix < 0 || ix >= wi) continue;
                    const size_t src_j = ((size_t)cc * hi + iy) * wi + ix;
                    t += std::fabs((double)raw[(((size_t)o * ci + cc) * ed.kh + ky) * ed.kw + kx]) *
                         (ed.src < 0 ? 1.0 : net->nodes[ed.src].y_h[src_j]);
                  }
              wy[((size_t)o * ho + y) * wo + x] = t;
            }
        e_wy.push_back(std::move(wy));
        e_terms.push_back((double)n.c * ed.kh * ed.kw);
      } else if (ed.kind == GCP_EDGE_IDENTITY) {
        if (E->d_src != E->d_dst) fail(GCP_EINVAL, "identity edge between different sizes");
        if (ed.src < 0) e_wy.emplace_back(E->d_dst, 1.0);
        else e_wy.push_back(net->nodes[ed.src].y_h);
        e_terms.push_back(1.0);
      } else {
        fail(GCP_EINVAL, "unknown edge kind");
      }
      int eid = (int)net->edges.size();
      n.in_edges.push_back(eid);
      if (ed.src >= 0) net->nodes[ed.src].consumers.push_back(eid);
      else net->in_consumers.push_back(eid);
      net->edges.push_back(std::move(E));
    }
  }
  net->n_I = rank0;
  for (int i = 0; i < net->out; ++i)
    if (net->nodes[i].consumers.empty()) fail(GCP_EUNSUPPORTED, "ReLU node without consumers");
  build_slack_weights(net, e_wy, e_terms);
  if (net->in_consumers.empty()) fail(GCP_EINVAL, "network input is unused");
  // the concretisation takes one pushed Lambda, through a dense or conv edge
  if (net->in_consumers.size() > 1) fail(GCP_EUNSUPPORTED, "several consumers of the network input");
  if (net->edges[net->in_consumers[0]]->kind == GCP_EDGE_IDENTITY)
    fail(GCP_EUNSUPPORTED, "identity edge from the network input");
  const char* og = std::getenv("GCP_OUT_GENERAL");
  net->out_general = og && *og && std::atoi(og) != 0;
  for (int eid : net->nodes[net->out].in_edges) {
    const EdgeH& E = *net->edges[eid];
    if (E.kind == GCP_EDGE_CONV || E.src < 0) net->out_general = true;
  }
  for (int i = 0; i < net->out; ++i) {
    const NodeH& n = net->nodes[i];
    int outs = 0;
    for (int eid : n.consumers) outs += (net->edges[eid]->dst == net->out);
    if (outs && n.consumers.size() > 1) net->out_general = true;
  }
}

// ------------------------------------------------------------------ tile choice
// Tile shapes come from a small autotuner: the first time a GEMM shape is
// launched on a net, every candidate tile runs a few times as an idempotent
// trial (same inputs, outputs that the real launch overwrites, or scratch)
// timed with HIP events, and the fastest is cached per (kind, precision,
// sign input, M, N, K).  GCP_AUTOTUNE=0 selects a fixed heuristic instead.
const int kTileCandidates[] = {0, 1, 2, 4, 5, 6, 7};   // 128x128 spills with the fused epilogues

bool autotune_enabled() {
  const char* e = std::getenv("GCP_AUTOTUNE");
  return !(e && e[0] == '0');
}

int heuristic_cfg(int M, int N) {
  static const int order[] = {1, 2, 0, 4, 5, 6, 7};
  for (int c : order) {
    int bm, bn;
    gemm_config_tile(c, &bm, &bn);
    long tiles = (long)((M + bm - 1) / bm) * ((N + bn - 1) / bn);
    if (tiles >= 1024) return c;
  }
  return 7;
}

// Process-wide tile cache.  With GCP_TILE_CACHE=<file> decisions are read
// from the file at first use (and again whenever the variable names another
// file) and every new decision is appended, so a later process (for example
// a profiler run) launches exactly the same tiles.
struct TileCache {
  std::mutex mu;
  bool loaded = false;
  std::string loaded_path;    // the file the decisions came from ("" = none)
  std::map<std::string, int> m;
  const char* path() { return std::getenv("GCP_TILE_CACHE"); }
  // (re)load when first used or when GCP_TILE_CACHE names another file
  void load() {
    const char* p = path();
    const std::string ps = p ? p : "";
    if (loaded && ps == loaded_path) return;
    loaded = true;
    loaded_path = ps;
    m.clear();
    if (!p) return;
    FILE* f = std::fopen(p, "r");
    if (!f) return;
    char key[160];
    int cfg;
    while (std::fscanf(f, "%159s %d", key, &cfg) == 2)
      if (cfg >= 0 && cfg < 16) m[key] = cfg;
    std::fclose(f);
  }
  void store(const std::string& key, int cfg) {
    m[key] = cfg;
    const char* p = path();
    if (!p) return;
    FILE* f = std::fopen(p, "a");
    if (!f) return;
    std::fprintf(f, "%s %d\n", key.c_str(), cfg);
    std::fclose(f);
  }
};
TileCache& tile_cache() { static TileCache t; return t; }

// Candidate list and fallback of one launch family.
struct Cands {
  std::vector<int> list;
  int fallback;
};
Cands dense_cands(int M, int N) {
  return Cands{std::vector<int>(std::begin(kTileCandidates), std::end(kTileCandidates)), heuristic_cfg(M, N)};
}
Cands conv_cands() {
  Cands c{{}, 0};
  for (int i = 0; i < conv_num_configs(); ++i) c.list.push_back(i);
  return c;
}
// The concretisation over the input: the direct transposed conv joins the
// candidates where it applies, and is the fallback there (GCP_CONV_DIRECT=0
// leaves it out).
bool conv_direct_enabled() {
  const char* e = std::getenv("GCP_CONV_DIRECT");
  return !(e && e[0] == '0');
}
Cands conc_conv_cands(const ConvGeom& g) {
  Cands c = conv_cands();
  if (conv_direct_enabled() && conv_direct_ok(g, EPI_CONC)) {
    c.list.push_back(kConvDirectCfg);
    c.fallback = kConvDirectCfg;
  }
  return c;
}
// Explicit-pi launches: the shapes their epilogues are instantiated for, and
// tile-cache keys of their own (epilogue kind + kPiKey).
constexpr int kPiKey = 16;
Cands pi_dense_cands(int M, int N) { return Cands{{5, 6, 7}, pi_cfg(heuristic_cfg(M, N))}; }
Cands pi_conv_cands() { return Cands{{0, 2}, 2}; }

template <class Trial>
int choose_cfg(const char* fam, int kind, int bf16, int sign, int M, int N, int K, hipStream_t st,
               const Cands& cands, Trial trial) {
  char kb[160];
  std::snprintf(kb, sizeof kb, "%s.k%d.b%d.s%d.M%d.N%d.K%d", fam, kind, bf16, sign, M, N, K);
  const std::string key(kb);
  TileCache& TC = tile_cache();
  {
    std::lock_guard<std::mutex> lk(TC.mu);
    TC.load();
    auto it = TC.m.find(key);
    if (it != TC.m.end()) return it->second;
  }
  int best = cands.fallback;
  if (g_no_alloc) return best;   // no trials, nothing recorded
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(st, &cs);
  if (autotune_enabled() && cs == hipStreamCaptureStatusNone && cands.list.size() > 1) {
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    float best_ms = 1e30f;
    for (int c : cands.list) {
      hip_check(trial(c), "autotune trial");
      hip_check(hipEventRecord(e0, st), "hipEventRecord");
      for (int rep = 0; rep < 3; ++rep) hip_check(trial(c), "autotune trial");
      hip_check(hipEventRecord(e1, st), "hipEventRecord");
      hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      if (ms < best_ms) { best_ms = ms; best = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  std::lock_guard<std::mutex> lk(TC.mu);
  TC.store(key, best);
  return best;
}

int slots_for_gemm(int N) { return (N + 31) / 32; }
int slots_for_elementwise(int N) { return (N + 255) / 256; }

}  // namespace

// ====================================================================== ABI

#define GCP_TRY try {
#define GCP_CATCH                                          \
  }                                                        \
  catch (const Err& e) {                                   \
    g_err = e.msg;                                         \
    return e.code;                                         \
  }                                                        \
  catch (const std::bad_alloc&) {                          \
    g_err = "host allocation failed";                      \
    return GCP_ENOMEM;                                     \
  }                                                        \
  catch (...) {                                            \
    g_err = "unexpected internal error";                   \
    return GCP_EDEVICE;                                    \
  }

extern "C" const char* gcp_last_error(void) { return g_err.c_str(); }
extern "C" const char* gcp_version(void) { return "gcp-mi355x 0.1 (gfx950)"; }

extern "C" int gcp_net_create(const gcp_net_desc* desc, gcp_net** out) {
  GCP_TRY
  if (!out) fail(GCP_EINVAL, "null output handle");
  auto net = std::make_unique<gcp_net>();
  build_net(desc, net.get());
  *out = net.release();
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}

extern "C" int gcp_net_destroy(gcp_net* net) {
  delete net;
  return GCP_OK;
}

extern "C" int gcp_net_get_info(const gcp_net* net, gcp_net_info* info) {
  if (!net || !info) { g_err = "null argument"; return GCP_EINVAL; }
  info->n_nodes = (int32_t)net->nodes.size();
  info->in_size = net->in_size;
  info->out_size = net->nodes[net->out].size;
  info->n_relu = net->n_relu;
  info->n_unstable = net->n_I;
  return GCP_OK;
}

extern "C" int gcp_net_get_unstable(const gcp_net* net, int32_t* node, int32_t* neuron, double* lower,
                                    double* upper) {
  GCP_TRY
  if (!net) fail(GCP_EINVAL, "null net");
  for (int i = 0; i < net->out; ++i) {
    const NodeH& n = net->nodes[i];
    for (int j = 0; j < n.size; ++j) {
      const int r = n.rank_h[j];
      if (r < 0) continue;
      if (node) node[r] = i;
      if (neuron) neuron[r] = j;
      if (lower) lower[r] = n.l_h[j];
      if (upper) upper[r] = n.u_h[j];
    }
  }
  return GCP_OK;
  GCP_CATCH
}

extern "C" int gcp_cuts_create(const gcp_net* net, int32_t n_cuts, int64_t nnz, const int32_t* cut,
                               const int32_t* node, const int32_t* neuron, const int8_t* kind,
                               const double* coef, const double* d, gcp_cuts** out) {
  GCP_TRY
  if (!net || !out) fail(GCP_EINVAL, "null argument");
  if (n_cuts < 0 || nnz < 0) fail(GCP_EINVAL, "negative size");
  if (nnz > 0 && (!cut || !node || !neuron || !kind || !coef)) fail(GCP_EINVAL, "null cut entry array");
  if (n_cuts > 0 && !d) fail(GCP_EINVAL, "null cut offsets");
  const int n_nodes = (int)net->nodes.size();
  // merge (cut, node, neuron) -> (H, G, Q)
  std::map<std::tuple<int, int, int>, std::array<double, 3>> m;
  for (int64_t e = 0; e < nnz; ++e) {
    int k = cut[e], nd = node[e], j = neuron[e], kd = kind[e];
    if (k < 0 || k >= n_cuts) fail(GCP_EINVAL, "cut index out of range");
    if (nd < -1 || nd >= n_nodes || (nd >= 0 && !net->nodes[nd].relu))
      fail(GCP_EINVAL, "cut entry on a node that is not a ReLU node or the input");
    if (kd < 0 || kd > 2) fail(GCP_EINVAL, "bad cut coefficient kind");
    if (nd < 0 && kd != GCP_CUT_G) fail(GCP_EINVAL, "input-variable cut entries must be of kind G");
    int sz = nd < 0 ? net->in_size : net->nodes[nd].size;
    if (j < 0 || j >= sz) fail(GCP_EINVAL, "cut neuron index out of range");
    if (!std::isfinite(coef[e])) fail(GCP_ENONFINITE, "non-finite cut coefficient");
    auto& a = m[std::make_tuple(k, nd, j)];
    a[kd] += coef[e];
  }
  for (int k = 0; k < n_cuts; ++k)
    if (!std::isfinite(d[k])) fail(GCP_ENONFINITE, "non-finite cut offset");
  // Coefficients are stored in fp32.  Where rounding changes one, the cut the
  // kernels see is  sum c' var <= d'  with d' = d + sum |c' - c| max|var|,
  // which every point satisfying the given cut satisfies too (var ranges:
  // x in [l, u] and x_hat in [0, max(u, 0)] from the root bounds, z in
  // [0, 1]), so the bound stays sound.  Input-variable coefficients have no
  // range before the call (x0, eps) and must be fp32 values.
  std::vector<double> slack(n_cuts, 0.0);
  for (auto& kv : m) {
    const int k = std::get<0>(kv.first), nd = std::get<1>(kv.first), j = std::get<2>(kv.first);
    for (int kd = 0; kd < 3; ++kd) {
      const double c = kv.second[kd];
      const double err = std::fabs((double)(float)c - c);
      if (err == 0.0) continue;
      if (nd < 0) fail(GCP_EINVAL, "input-variable cut coefficients must be fp32 values");
      const NodeH& n = net->nodes[nd];
      const double range = kd == GCP_CUT_H ? std::max(std::fabs(n.l_h[j]), std::fabs(n.u_h[j]))
                         : kd == GCP_CUT_G ? std::max(n.u_h[j], 0.0) : 1.0;
      slack[k] += err * range;
    }
  }
  auto C = std::make_unique<gcp_cuts>();
  C->N = n_cuts;
  C->net = net;
  C->nnz_e = (int)m.size();
  std::vector<int32_t> row_ptr(n_cuts + 1, 0);
  struct Ent { int k, nd, j, pos; float h, g, q; };
  std::vector<Ent> ents;
  ents.reserve(m.size());
  std::vector<double> kap((size_t)3 * n_cuts, 0.0);
  for (auto& kv : m) {
    const int k = std::get<0>(kv.first), nd = std::get<1>(kv.first), j = std::get<2>(kv.first);
    const double h = std::fabs((double)(float)kv.second[0]), g = std::fabs((double)(float)kv.second[1]),
                 q = std::fabs((double)(float)kv.second[2]);
    if (nd < 0) kap[(size_t)n_cuts + k] += g;
    else kap[k] += (h + g) * net->nodes[nd].z_h[j] + 2.0 * q;
  }
  int pos = 0;
  for (auto& kv : m) {   // std::map order = (cut, node, neuron): cut-major
    int k = std::get<0>(kv.first);
    row_ptr[k + 1]++;
    ents.push_back(Ent{k, std::get<1>(kv.first), std::get<2>(kv.first), pos++, (float)kv.second[0],
                       (float)kv.second[1], (float)kv.second[2]});
  }
  for (int k = 0; k < n_cuts; ++k) row_ptr[k + 1] += row_ptr[k];
  C->row_ptr.upload(row_ptr);
  std::vector<double> dv(d ? d : (const double*)nullptr, d ? d + n_cuts : (const double*)nullptr);
  for (int k = 0; k < n_cuts; ++k)
    if (slack[k] > 0.0) dv[k] = std::nextafter(dv[k] + slack[k], INFINITY);
  C->d.upload(dv);
  for (int k = 0; k < n_cuts; ++k) kap[(size_t)2 * n_cuts + k] = std::fabs(dv[k]);
  for (double& v : kap) v *= 1.0 + 0x1p-30;
  if (n_cuts > 0) C->kap.upload(kap);
  C->cols.resize(n_nodes + 1);
  C->nnz_node.assign(n_nodes + 1, 0);
  for (auto& e : ents) C->nnz_node[e.nd < 0 ? n_nodes : e.nd]++;
  for (int nd = -1; nd < n_nodes; ++nd) {
    if (nd >= 0 && !net->nodes[nd].relu) continue;
    int sz = nd < 0 ? net->in_size : net->nodes[nd].size;
    std::vector<Ent> mine;
    for (auto& e : ents)
      if (e.nd == nd) mine.push_back(e);
    auto& col = C->cols[nd < 0 ? n_nodes : nd];
    if (mine.empty()) continue;
    std::stable_sort(mine.begin(), mine.end(), [](const Ent& a, const Ent& b) { return a.j < b.j; });
    std::vector<int32_t> cp(sz + 1, 0), cpos;
    std::vector<float4> en;
    for (auto& e : mine) {
      cp[e.j + 1]++;
      cpos.push_back(e.pos);
      float kb;
      std::memcpy(&kb, &e.k, 4);
      en.push_back(make_float4(e.h, e.g, e.q, kb));
    }
    for (int j = 0; j < sz; ++j) C->col_max = std::max(C->col_max, cp[j + 1]);
    for (int j = 0; j < sz; ++j) cp[j + 1] += cp[j];
    std::vector<int2> rg(sz);
    for (int j = 0; j < sz; ++j) rg[j] = make_int2(cp[j], cp[j + 1]);
    col.rng.upload(rg); col.ent.upload(en); col.pos.upload(cpos);
    col.any = true;
  }
  *out = C.release();
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}

extern "C" int gcp_cuts_info(const gcp_cuts* cuts, int32_t* n_cuts) {
  GCP_TRY
  if (!cuts || !n_cuts) fail(GCP_EINVAL, "null argument");
  *n_cuts = cuts->N;
  return GCP_OK;
  GCP_CATCH
}

extern "C" int gcp_cuts_destroy(gcp_cuts* c) {
  delete c;
  return GCP_OK;
}

namespace {
// The device form of B domains' splits: mask [B][n_I] (0, +(slot+1) for
// x >= 0, -(slot+1) for x <= 0) and zsplit [B][K]; validates as
// gcp_splits_create documents.
void split_arrays(const gcp_net* net, int32_t B, int32_t K, const int32_t* node, const int32_t* neuron,
                  const int8_t* sign, std::vector<int8_t>& mask, std::vector<double>& zs) {
  if (B <= 0 || K < 0 || K > 127) fail(GCP_EINVAL, "need B >= 1 and 0 <= K <= 127");
  if (K > 0 && (!node || !neuron || !sign)) fail(GCP_EINVAL, "null split array");
  mask.assign((size_t)B * net->n_I, 0);
  zs.assign((size_t)B * K, 0.0);
  for (int b = 0; b < B; ++b)
    for (int k = 0; k < K; ++k) {
      size_t i = (size_t)b * K + k;
      int nd = node[i];
      if (nd < 0) continue;
      if (nd >= (int)net->nodes.size() || !net->nodes[nd].relu) fail(GCP_EINVAL, "split on a non-ReLU node");
      const NodeH& n = net->nodes[nd];
      int j = neuron[i];
      if (j < 0 || j >= n.size) fail(GCP_EINVAL, "split neuron out of range");
      if (sign[i] != 1 && sign[i] != -1) fail(GCP_EINVAL, "split sign must be +1 or -1");
      const int rk = n.rank_h[j];
      if (rk < 0) fail(GCP_EINVAL, "split neuron is not root-unstable");
      int8_t& mm = mask[(size_t)b * net->n_I + rk];
      if (mm != 0) fail(GCP_EINVAL, "neuron split twice in one domain");
      mm = (int8_t)(sign[i] > 0 ? (k + 1) : -(k + 1));
      zs[i] = n.z_h[j];
    }
}
}  // namespace

extern "C" int gcp_splits_create(const gcp_net* net, int32_t B, int32_t K, const int32_t* node,
                                 const int32_t* neuron, const int8_t* sign, gcp_splits** out) {
  GCP_TRY
  if (!net || !out) fail(GCP_EINVAL, "null argument");
  std::vector<int8_t> mask;
  std::vector<double> zs;
  split_arrays(net, B, K, node, neuron, sign, mask, zs);
  auto S = std::make_unique<gcp_splits>();
  S->B = B; S->K = K; S->net = net;
  S->mask.upload(mask);
  if (K > 0) S->zsplit.upload(zs);
  *out = S.release();
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}

namespace gcp {
int splits_assign(const gcp_net* net, gcp_splits** s, int32_t B, int32_t K, const int32_t* node,
                  const int32_t* neuron, const int8_t* sign, hipStream_t st) {
  GCP_TRY
  if (!net || !s) fail(GCP_EINVAL, "null argument");
  gcp_splits* h = *s;
  if (h && h->net != net) fail(GCP_EINVAL, "splits were created for another net");
  if (!h || h->mask.bytes < (size_t)B * net->n_I || h->zsplit.bytes < (size_t)B * K * 8) {
    if (h) gcp_splits_destroy(h);
    *s = nullptr;
    return gcp_splits_create(net, B, K, node, neuron, sign, s);
  }
  split_arrays(net, B, K, node, neuron, sign, h->mask_h, h->zs_h);
  if (!h->mask_h.empty())
    hip_check(hipMemcpyAsync(h->mask.p, h->mask_h.data(), h->mask_h.size(), hipMemcpyHostToDevice, st),
              "hipMemcpyAsync");
  if (!h->zs_h.empty())
    hip_check(hipMemcpyAsync(h->zsplit.p, h->zs_h.data(), h->zs_h.size() * 8, hipMemcpyHostToDevice, st),
              "hipMemcpyAsync");
  h->B = B; h->K = K;
  h->id = next_generation();   // new contents: cached plans keyed on the handle do not match it
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}
}  // namespace gcp

extern "C" int gcp_splits_destroy(gcp_splits* s) {
  delete s;
  return GCP_OK;
}

// ====================================================================== passes

namespace {

// One recorded launch of an iteration (batched optimisation): a dense GEMM
// with its epilogue arguments, or an elementwise relaxation.
struct Rec {
  int type;            // 0 GEMM, 1 elementwise bound
  int bf16, cfg, kind, sign;
  GemmArgs g;
  alignas(16) unsigned char epi[sizeof(AdjEpiArgs) > sizeof(BoundEpiArgs) ? sizeof(AdjEpiArgs) : sizeof(BoundEpiArgs)];
  ElemBoundJob ej;
  int tiles;           // workgroups of this problem
  double bytes, alg, flops; // HBM bytes (both models, see Bytes) and FLOPs of this launch
};
static_assert(sizeof(ConcEpiArgs) <= sizeof(Rec::epi) && sizeof(StoreEpiArgs) <= sizeof(Rec::epi), "epi blob");
struct Recorder {
  std::vector<Rec> bound, adj;   // in launch order
  bool in_adj = false;
  void push(const Rec& r) { (in_adj ? adj : bound).push_back(r); }
};

// ---------------------------------------------------------------- persistent dataflow plans
// How the persistent launches order their workgroups: with one claim queue
// per XCD (the probe found the XCDs), a producer's stores need only reach
// the L2 its consumers share; otherwise agent-scope release fences write
// the L2 back.  GCP_PERSIST_SYNC=agent forces the latter.
int persist_xcd_sync(int queues) {
  const char* e = std::getenv("GCP_PERSIST_SYNC");
  if (e && std::strcmp(e, "agent") == 0) return 0;
  return queues > 1 ? 1 : 0;
}

// Claim queues of the current device: the number of XCDs its workgroups
// report (the hardware XCC_ID register of a probe launch), when the ids are
// exactly 0 .. n-1 with n <= 8; else 1 (one queue, no XCD locality).
int persist_queues() {
  static std::mutex mu;
  static std::map<int, int> by_dev;
  int dev;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(mu);
  auto it = by_dev.find(dev);
  if (it != by_dev.end()) return it->second;
  int cus = 0;
  hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
  const int n = std::max(64, cus * 4);
  DBuf out;
  out.alloc((size_t)n * sizeof(int));
  hip_check(launch_xcc_probe(out.as<int>(), n, nullptr), "xcc probe");
  std::vector<int> ids(n);
  hip_check(hipMemcpy(ids.data(), out.p, (size_t)n * sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy");
  std::set<int> seen(ids.begin(), ids.end());
  int q = (int)seen.size();
  if (q > 8 || *seen.begin() != 0 || *seen.rbegin() != q - 1) q = 1;
  by_dev[dev] = q;
  return q;
}

// One instance's recorded iteration: its bound-pass and adjoint launches in
// order, and its multiplier update.
struct PersistInst {
  const Recorder* rec;
  bool has_gamma;
  GammaJob gj;
  int M;
};

// Lays the instances' schedules out as persistent steps: the w-th bound
// launch of every instance, then the w-th adjoint launch of every instance,
// then every multiplier update (dependent steps of one instance as far apart
// in the queue as the schedule allows).  Returns false when the schedule
// does not fit the kernel's step table.
bool build_persist(PersistPlan& plan, const std::vector<PersistInst>& in, int bf16) {
  const int n = (int)in.size();
  const int Q = persist_queues();
  const int xcd = persist_xcd_sync(Q);
  struct Ord { int inst; const Rec* r; };
  std::vector<Ord> order;
  size_t maxb = 0, maxa = 0;
  for (const auto& x : in) { maxb = std::max(maxb, x.rec->bound.size()); maxa = std::max(maxa, x.rec->adj.size()); }
  for (size_t w = 0; w < maxb; ++w)
    for (int i = 0; i < n; ++i) if (w < in[i].rec->bound.size()) order.push_back({i, &in[i].rec->bound[w]});
  for (size_t w = 0; w < maxa; ++w)
    for (int i = 0; i < n; ++i) if (w < in[i].rec->adj.size()) order.push_back({i, &in[i].rec->adj[w]});
  for (int i = 0; i < n; ++i) if (in[i].has_gamma) order.push_back({i, nullptr});
  const int ns = (int)order.size();
  if (ns == 0 || ns > kPersistMaxSteps) return false;
  std::vector<int> panels(n), base(n), acc(n, 0);
  int tot = 0;
  for (int i = 0; i < n; ++i) {
    panels[i] = (in[i].M + kPersistRows - 1) / kPersistRows;
    base[i] = tot;
    tot += panels[i];
  }
  std::vector<PersistStep> steps;
  std::vector<int> step_inst;
  std::vector<GemmArgs> gemm;
  std::vector<unsigned char> epi;
  std::vector<ElemBoundJob> elem;
  std::vector<GammaJob> gam;
  plan.bytes = plan.alg = plan.flops = 0.0;
  for (const Ord& o : order) {
    PersistStep st{};
    st.cnt0 = base[o.inst];
    st.panels = panels[o.inst];
    st.base = base[o.inst];
    if (!o.r) {
      const GammaJob& gj = in[o.inst].gj;
      st.kind = PK_GAMMA;
      st.job = (int)gam.size();
      gam.push_back(gj);
      st.ipp = (gj.N + 31) / 32;
      plan.bytes += (double)gj.M * (gj.N * 24.0);
      plan.alg += (double)gj.M * gj.N * 28.0;
    } else if (o.r->type == 1) {
      st.kind = PK_ELEM;
      st.job = (int)elem.size();
      elem.push_back(o.r->ej);
      st.ipp = (o.r->ej.a.nd.size + 255) / 256 * (kPersistRows / kElemRows);   // one item per kElemRows rows
      plan.bytes += o.r->bytes;
      plan.alg += o.r->alg;
    } else {
      if (o.r->kind == EPI_AHAT) return false;
      st.kind = o.r->kind;
      st.sign = o.r->sign;
      st.job = (int)gemm.size();
      gemm.push_back(o.r->g);
      const size_t off = epi.size();
      epi.resize(off + kEpiBlob, 0);
      std::memcpy(epi.data() + off, o.r->epi, sizeof(o.r->epi));
      st.ipp = (o.r->g.N + 31) / 32;
      plan.bytes += o.r->bytes;
      plan.alg += o.r->alg;
      plan.flops += o.r->flops;
    }
    if (st.ipp <= 0) continue;
    st.wait = acc[o.inst];
    acc[o.inst] += st.ipp;
    steps.push_back(st);
    step_inst.push_back(o.inst);
  }
  for (size_t k = 0; k < steps.size(); ++k) steps[k].per_iter = acc[step_inst[k]];
  const int nst = (int)steps.size();
  // per queue: first item of every step within an iteration
  std::vector<int> qfirst((size_t)Q * (nst + 1));
  for (int q = 0; q < Q; ++q) {
    int a = 0;
    for (int k = 0; k < nst; ++k) {
      qfirst[(size_t)q * (nst + 1) + k] = a;
      const PersistStep& st = steps[k];
      const int r = ((q - st.base) % Q + Q) % Q;
      const int owned = r < st.panels ? (st.panels - 1 - r) / Q + 1 : 0;
      a += owned * st.ipp;
    }
    qfirst[(size_t)q * (nst + 1) + nst] = a;
    plan.max_items = std::max(plan.max_items, a);
  }
  // one device buffer: [steps][qfirst][gemm][epi][elem][gam], 256-byte aligned parts
  std::vector<unsigned char> host;
  auto put = [&](const void* src, size_t bytes) {
    const size_t off = (host.size() + 255) / 256 * 256;
    host.resize(off + std::max<size_t>(bytes, 1), 0);
    if (bytes) std::memcpy(host.data() + off, src, bytes);
    return off;
  };
  const size_t o_steps = put(steps.data(), steps.size() * sizeof(PersistStep));
  const size_t o_q = put(qfirst.data(), qfirst.size() * sizeof(int));
  const size_t o_g = put(gemm.data(), gemm.size() * sizeof(GemmArgs));
  const size_t o_e = put(epi.data(), epi.size());
  const size_t o_el = put(elem.data(), elem.size() * sizeof(ElemBoundJob));
  const size_t o_gm = put(gam.data(), gam.size() * sizeof(GammaJob));
  plan.buf.upload(host);
  unsigned char* b = (unsigned char*)plan.buf.p;
  plan.n_sync = (size_t)Q + 1 + tot;
  plan.sync.alloc(plan.n_sync * sizeof(int));
  plan.latch.alloc(16);
  PersistArgs& a = plan.args;
  a = PersistArgs{};
  a.steps = (const PersistStep*)(b + o_steps);
  a.n_steps = nst;
  a.qfirst = (const int*)(b + o_q);
  a.Q = Q;
  a.gemm = (const GemmArgs*)(b + o_g);
  a.epi = b + o_e;
  a.elem = (const ElemBoundJob*)(b + o_el);
  a.gam = (const GammaJob*)(b + o_gm);
  a.sync = plan.sync.as<int>();
  a.xcd_sync = xcd;
  a.latch = plan.latch.as<int>();
  plan.grid = persist_grid(bf16, xcd);
  if (plan.grid <= 0) fail(GCP_EDEVICE, "persistent launch: occupancy query failed");
  return true;
}

// `iters` iterations of the plan in one launch, iteration t with the Adam
// constants of iteration iter0 + t from the table `tab`.
// The longest wait of a persistent launch before it aborts, in ticks of
// the 100 MHz wall clock: 1 s, or GCP_PERSIST_SPIN_TICKS (tests force the
// abort path with a tiny value).
unsigned long long persist_spin_ticks() {
  const char* e = std::getenv("GCP_PERSIST_SPIN_TICKS");
  return e && *e ? std::strtoull(e, nullptr, 10) : 100000000ull;
}

void run_persist(PersistPlan& plan, int bf16, int iters, int iter0, const AdamArgs& adam_tab, hipStream_t st) {
  // iterations per launch: a queue's items stay below the abort offset
  const int per_launch = std::max(1, (kPersistAbort / 2) / std::max(plan.max_items, 1));
  hip_check(launch_fill_f32((float*)plan.latch.p, 1, 0.f, st), "persist latch reset");
  for (int done = 0; done < iters; done += per_launch) {
    const int n = std::min(per_launch, iters - done);
    hip_check(launch_fill_f32((float*)plan.sync.p, (int64_t)plan.n_sync, 0.f, st), "persist sync reset");
    PersistArgs a = plan.args;
    a.iters = n;
    a.iter0 = iter0 + done;
    a.adam = adam_tab;
    a.spin_ticks = persist_spin_ticks();
    hip_check(timed(st, bf16 ? "persist.bf16" : "persist.fp32",
                    Bytes{plan.bytes * n, plan.alg * n}, plan.flops * n,
                    [&] { return launch_persist(bf16, a, plan.grid, st); }),
              "persistent launch");
  }
}

struct Call {
  Recorder* rec = nullptr;
  gcp_net* net;
  gcp_net::WS* ws = nullptr;   // the workspace of this call: the net's own, or a view of the static scratch
  bool no_alloc = false;       // no device allocation, autotuning trial or profiler event in this call
  const gcp_cuts* cuts;
  const gcp_splits* splits;
  const double* x0;
  double eps;
  const double* C;
  int S, M, B;
  RowParams rp;
  hipStream_t st;
  int nnz;
  int N;
  std::vector<uint8_t> recompute;   // per node: a_hat recomputed in the adjoint instead of stored
  // the spec-row constants (C b_out, c-hat = C W_out or the materialised
  // output Lambda) are already in the workspace for this C: later bound
  // passes of one optimisation skip them
  bool consts_done = false;
  // the bound pass subtracts its rounding slack (GCP_FLAG_OUTWARD)
  bool outward = false;
};

void ensure_ws(Call& c) {
  gcp_net* net = c.net;
  auto& ws = net->ws;
  const int nn = (int)net->nodes.size();
  bool grow = c.M > ws.M || c.nnz > ws.nnz || c.S > ws.S || c.N > ws.N || ws.lam.empty();
  if (!grow) return;
  int M = std::max(c.M, ws.M), S = std::max(c.S, ws.S), nnz = std::max(c.nnz, ws.nnz), Nc = std::max(c.N, ws.N);
  ws.lam.clear(); ws.ahat.clear(); ws.dahat.clear(); ws.acc.clear(); ws.addv.clear();
  for (int i = 0; i < nn; ++i) {
    const NodeH& n = net->nodes[i];
    size_t elems = (n.relu || (i == net->out && net->out_general)) ? (size_t)M * n.ld : 0;
    auto mk = [&](size_t bytes) { auto b = std::make_unique<DBuf>(); b->alloc(bytes); return b; };
    ws.lam.push_back(mk(elems * 4));
    ws.ahat.push_back(mk(0));         // sized by plan_ahat: stored only where not recomputed
    ws.dahat.push_back(mk(elems * 4));
    bool ident = false;
    for (int eid : n.in_edges) ident |= net->edges[eid]->kind == GCP_EDGE_IDENTITY;
    for (int eid : n.consumers) ident |= net->edges[eid]->kind == GCP_EDGE_IDENTITY;
    bool multi = n.relu && (n.consumers.size() > 1 || n.in_edges.size() > 1 || ident);
    ws.acc.push_back(mk(multi ? elems * 4 : 0));
    ws.addv.push_back(mk(n.relu ? (size_t)n.ld * 4 : 0));
  }
  ws.sign.alloc((size_t)M * net->in_ld);
  const int mp = round_up(M, 16);
  ws.contrib.alloc((size_t)mp * std::max(nnz, 1) * 4);
  ws.gammaT.alloc((size_t)mp * std::max(Nc, 1) * 4);
  ws.chat_off.assign(nn, -1);
  size_t chat_floats = 0;
  if (!net->out_general)
    for (int eid : net->nodes[net->out].in_edges) {
      int p = net->edges[eid]->src;
      ws.chat_off[p] = (int)chat_floats;
      chat_floats += (size_t)S * net->nodes[p].ld;
    }
  ws.chat.alloc(std::max<size_t>(chat_floats, 1) * 4);
  ws.cb.alloc((size_t)S * 8);
  ws.consts.alloc(16);
  ws.step.alloc(16);
  ws.flags.alloc(16);
  ws.acc_in.alloc((size_t)M * net->in_ld * 4);
  ws.M = M; ws.S = S; ws.nnz = nnz; ws.N = Nc;
  ws.gen = next_generation();
  ws.n_slots = 0;
  ws.partial.release();
}

CutCol cut_col(const Call& c, int node) {
  if (!c.cuts) return CutCol{nullptr, nullptr, nullptr};
  int idx = node < 0 ? (int)c.net->nodes.size() : node;
  return c.cuts->cols[idx].dev();
}

double nnz_of(const Call& c, int node) {
  if (!c.cuts) return 0.0;
  return (double)c.cuts->nnz_node[node < 0 ? (int)c.net->nodes.size() : node];
}
double unst_of(const Call& c, int node) { return node < 0 ? 0.0 : (double)c.net->nodes[node].n_unst; }
// optimiser-state bytes (Bytes::alg) of a bound-pass and of an adjoint launch on node p
double alg_bound(const Call& c, int p) {
  const double nu = unst_of(c, p);
  return (double)c.M * nu * (c.rp.rho ? 8.0 : 4.0) + (double)c.B * nu;
}
// multipliers: gamma read once by the bound pass, gamma and beta with their
// Adam moments read and written by the update (counted with the gamma update)
double alg_mult(const Call& c) { return (double)c.M * (c.N + c.rp.K) * 28.0; }
double alg_adj(const Call& c, int p, bool adam) {
  const double nu = unst_of(c, p);
  return (double)c.M * nu * (adam ? 24.0 : 8.0) * (c.rp.rho ? 2.0 : 1.0) + (double)c.B * nu;
}

float* tune_store(Call& c) {
  auto& ws = *c.ws;
  size_t need = 0;
  for (auto& n : c.net->nodes) need = std::max(need, (size_t)c.M * n.ld * 4);
  if (ws.tune_store.bytes < need) ws.tune_store.alloc(need);
  return ws.tune_store.as<float>();
}
float* tune_alpha(Call& c) {
  auto& ws = *c.ws;
  size_t need = (size_t)c.M * std::max(c.rp.n_I, 1) * 4;
  if (ws.tune_alpha.bytes < need) ws.tune_alpha.alloc(need);
  return ws.tune_alpha.as<float>();
}
float* tune_beta(Call& c) {
  auto& ws = *c.ws;
  size_t need = (size_t)c.M * std::max(c.rp.K, 1) * 4;
  if (ws.tune_beta.bytes < need) ws.tune_beta.alloc(need);
  return ws.tune_beta.as<float>();
}

// In recording mode a GEMM launch is stored instead of issued.
template <class A>
bool record_gemm(Call& c, int bf16, int cfg, EpiKind kind, const GemmArgs& g, const A& a, Bytes bytes) {
  if (!c.rec) return false;
  if constexpr (std::is_same_v<A, BoundEpiArgs> || std::is_same_v<A, AdjEpiArgs>)
    if (a.rp.rho) fail(GCP_EUNSUPPORTED, "batched optimisation takes Lemma A.1's pi* only");
  Rec r{};
  r.type = 0; r.bf16 = bf16; r.cfg = cfg; r.kind = kind; r.sign = g.a_is_sign;
  r.g = g;
  r.bytes = bytes.all;
  r.alg = bytes.alg;
  r.flops = 2.0 * g.M * g.N * g.K;
  std::memcpy(r.epi, &a, sizeof(A));
  int bm, bn;
  gemm_config_tile(cfg, &bm, &bn);
  r.tiles = ((g.N + bn - 1) / bn) * ((g.M + bm - 1) / bm);
  c.rec->push(r);
  return true;
}
void no_record(const Call& c, const char* what) {
  if (c.rec) fail(GCP_EUNSUPPORTED, std::string("batched optimisation supports dense edges only (") + what + ")");
}

const void* wt_bound(const EdgeH& E, int bf16) { return bf16 ? E.WT16.p : E.WT32.p; }
const void* w_adj(const EdgeH& E, int bf16) { return bf16 ? E.W16.p : E.W32.p; }

// ---------------------------------------------------------------- bound pass
// Processes nodes from the output backwards.  For each target p the pushes
// from its consumers are accumulated into acc[p] except the last one, which
// runs fused with p's relaxation (or the concretisation for the input).
struct BoundPass {
  Call& c;
  int bf16;
  bool keep_ahat;     // adjoint will follow
  bool want_contrib;  // gradient pieces for input cuts
  bool dry;           // count partial slots only
  int slot = 0;
  std::vector<int> pushes_left;   // per node (index n_nodes: input)
  // Per node: the fp32 Lambda that stands in for its accumulation buffer when
  // an identity edge is the first of exactly two pushes (the copy into the
  // buffer would be exact), or null.
  std::vector<const float*> acc_alias;

  BoundPass(Call& cc, int b, bool k, bool wc, bool d) : c(cc), bf16(b), keep_ahat(k), want_contrib(wc), dry(d) {}

  int esz() const { return bf16 ? 2 : 4; }

  BoundEpiArgs bound_args(int p, bool has_acc) {
    auto& ws = *c.ws;
    BoundEpiArgs a{};
    a.nd = c.net->nodes[p].dev();
    a.cc = cut_col(c, p);
    a.rp = c.rp;
    a.acc_in = has_acc ? (acc_alias[p] ? acc_alias[p] : ws.acc[p]->as<float>()) : nullptr;
    a.lam_out = ws.lam[p]->p;
    const bool rec = !c.recompute.empty() && c.recompute[p];
    a.ahat_out = (keep_ahat && !rec) ? ws.ahat[p]->p : nullptr;
    return a;
  }

  void check(hipError_t e) { hip_check(e, "kernel launch (bound pass)"); }

  void run() {
    gcp_net* net = c.net;
    const int nn = (int)net->nodes.size();
    auto& ws = *c.ws;
    pushes_left.assign(nn + 1, 0);
    acc_alias.assign(nn + 1, nullptr);
    for (int i = 0; i < nn; ++i) pushes_left[i] = (int)net->nodes[i].consumers.size();
    pushes_left[nn] = (int)net->in_consumers.size();
    // output node: c-hat = C W (per spec row), constant C b_out
    const NodeH& on = net->nodes[net->out];
    if (net->out_general) {
      // Lambda^(out) = C on every row, pushed through the output's edges
      if (c.rec) fail(GCP_EUNSUPPORTED, "grouped launches need the c-hat form of the output");
      if (!dry && !c.consts_done) {
        check(launch_out_const(c.C, c.S, on.size, on.bias.as<float>(), ws.cb.as<double>(), c.st));
        check(launch_spec_rows(bf16, c.C, c.S, on.size, c.M, ws.lam[net->out]->p, on.ld, c.st));
      }
      for (int eid : on.in_edges)
        if (net->edges[eid]->kind == GCP_EDGE_IDENTITY) push(eid);
      for (int eid : on.in_edges)
        if (net->edges[eid]->kind != GCP_EDGE_IDENTITY) push(eid);
    }
    if (!net->out_general && !dry && !c.rec && !c.consts_done) {
      check(launch_out_const(c.C, c.S, on.size, on.bias.as<float>(), ws.cb.as<double>(), c.st));
      for (int eid : on.in_edges) {
        const EdgeH& E = *net->edges[eid];
        float* ch = ws.chat.as<float>() + ws.chat_off[E.src];
        check(launch_chat(c.C, c.S, on.size, E.Wraw.as<float>(), E.d_src,
                          E.kind == GCP_EDGE_IDENTITY ? 2 : 0, ch, net->nodes[E.src].ld, c.st));
      }
    }
    for (int eid : net->out_general ? std::vector<int>{} : on.in_edges) {
      const EdgeH& E = *net->edges[eid];
      int p = E.src;
      // the output is p's only consumer (checked at creation): fused relaxation
      pushes_left[p]--;
      BoundEpiArgs a = bound_args(p, false);
      int nslot = slots_for_elementwise(net->nodes[p].size);
      const double M = c.M, d = net->nodes[p].size, esz = bf16 ? 2 : 4;
      const double bytes = c.S * d * 4 + M * d * esz + (keep_ahat ? M * d * esz : 0) + M * unst_of(c, p) * 4 +
                           (double)c.B * unst_of(c, p) + M * nnz_of(c, p) * 4 + M * nslot * 8;
      if (!dry && c.rec) {
        Rec r{};
        r.type = 1; r.bf16 = bf16; r.cfg = -1; r.kind = EPI_BOUND; r.sign = 0;
        r.ej = ElemBoundJob{ws.chat.as<float>() + ws.chat_off[p], nullptr, a, ws.partial.as<double>(), slot};
        r.tiles = ((c.M + kElemRows - 1) / kElemRows) * ((net->nodes[p].size + 255) / 256);
        r.bytes = bytes;
        r.alg = alg_bound(c, p);
        c.rec->push(r);
      } else if (!dry) {
        check(timed(c.st, cls_name("bound_elem", bf16, 0, -1), Bytes{bytes, alg_bound(c, p)}, 0.0, [&] {
          return launch_bound_elementwise(bf16, ws.chat.as<float>() + ws.chat_off[p], nullptr, a, ws.partial.as<double>(),
                                          slot, c.st);
        }));
      }
      slot += nslot;
    }
    for (int i = net->out - 1; i >= 0; --i) {
      const NodeH& n = net->nodes[i];
      // edges ordered: identity first (they can only store), then the rest
      std::vector<int> order;
      for (int eid : n.in_edges)
        if (net->edges[eid]->kind == GCP_EDGE_IDENTITY) order.push_back(eid);
      for (int eid : n.in_edges)
        if (net->edges[eid]->kind != GCP_EDGE_IDENTITY) order.push_back(eid);
      for (int eid : order) push(eid);
    }
  }

  // Lambda^(dst) pushed through edge E into target src.
  void push(int eid) {
    gcp_net* net = c.net;
    auto& ws = *c.ws;
    const EdgeH& E = *net->edges[eid];
    const int nn = (int)net->nodes.size();
    const int p = E.src;
    const int pidx = p < 0 ? nn : p;
    const bool last = (--pushes_left[pidx] == 0);
    const int total = p < 0 ? (int)net->in_consumers.size() : (int)net->nodes[p].consumers.size();
    const bool has_acc = total > 1;        // earlier pushes went to acc[p]
    const bool first = !has_acc || (pushes_left[pidx] == total - 1);
    const NodeH& dn = net->nodes[E.dst];
    const int d_src = E.d_src;
    const int ld_src = node_ld_of(net, p);
    float* accbuf = p < 0 ? ws.acc_in.as<float>() : ws.acc[p]->as<float>();
    const bool pi = c.rp.rho != nullptr;   // explicit pi: the pi-switched epilogues

    if (E.kind == GCP_EDGE_DENSE) {
      GemmArgs g{};
      g.M = c.M; g.N = d_src; g.K = dn.size;
      g.A = ws.lam[E.dst]->p; g.lda = dn.ld;
      g.Bt = wt_bound(E, bf16); g.ldb = dn.ld;
      g.a_is_sign = 0;
      g.mp = c.rp.mp;
      if (!last) {
        StoreEpiArgs s{d_src, ld_src, 1.f, first ? nullptr : accbuf, accbuf};
        g.partial = nullptr;
        if (!dry) {
          int cfg = choose_cfg("gemm", EPI_STORE, bf16, 0, g.M, g.N, g.K, c.st, dense_cands(g.M, g.N), [&](int cf) {
            StoreEpiArgs t = s;
            t.acc_in = nullptr;
            t.out = tune_store(c);
            return launch_gemm(bf16, cf, EPI_STORE, g, &t, c.st);
          });
          const double esz = bf16 ? 2 : 4;
          const double bytes = (double)g.M * g.K * esz + (double)g.N * g.K * esz + (double)g.M * g.N * 4 * (first ? 1 : 2);
          if (!record_gemm(c, bf16, cfg, EPI_STORE, g, s, Bytes{bytes, 0.0}))
            check(timed(c.st, cls_name("store", bf16, 0, cfg), Bytes{bytes, 0.0}, 2.0 * g.M * g.N * g.K,
                        [&] { return launch_gemm(bf16, cfg, EPI_STORE, g, &s, c.st); }));
        }
        return;
      }
      int nslot = slots_for_gemm(d_src);
      if (p >= 0) {
        BoundEpiArgs a = bound_args(p, has_acc);
        if (!dry) {
          GemmArgs gt = g;
          gt.partial = nullptr;
          int cfg = choose_cfg("gemm", pi ? EPI_BOUND + kPiKey : EPI_BOUND, bf16, 0, g.M, g.N, g.K, c.st,
                               pi ? pi_dense_cands(g.M, g.N) : dense_cands(g.M, g.N),
                               [&](int cf) { return launch_gemm(bf16, cf, EPI_BOUND, gt, &a, c.st); });
          g.partial = ws.partial.as<double>(); g.slot0 = slot;
          const double M = g.M, esz = bf16 ? 2 : 4, dp = g.N;
          const double bytes = M * g.K * esz + (double)g.N * g.K * esz + M * dp * esz + (keep_ahat ? M * dp * esz : 0) +
                               M * unst_of(c, p) * (pi ? 8 : 4) + (double)c.B * unst_of(c, p) + M * nnz_of(c, p) * 4 +
                               (has_acc ? M * dp * 4 : 0) + M * nslot * 8;
          if (!record_gemm(c, bf16, cfg, EPI_BOUND, g, a, Bytes{bytes, alg_bound(c, p)}))
            check(timed(c.st, pi ? cls_name("bound_pi", bf16, 0, pi_cfg(cfg)) : cls_name("bound", bf16, 0, cfg),
                        Bytes{bytes, alg_bound(c, p)},
                        2.0 * g.M * g.N * g.K, [&] { return launch_gemm(bf16, cfg, EPI_BOUND, g, &a, c.st); }));
        }
      } else {
        if (has_acc) fail(GCP_EUNSUPPORTED, "several consumers of the input");
        ConcEpiArgs a{};
        a.size = net->in_size; a.ld = net->in_ld; a.x0 = c.x0; a.eps = c.eps;
        a.cc = cut_col(c, -1); a.rp = c.rp;
        a.sign_out = keep_ahat ? ws.sign.as<int8_t>() : nullptr;
        a.contrib = want_contrib ? ws.contrib.as<float>() : nullptr;
        a.nnz_e = c.nnz;
        if (!dry) {
          GemmArgs gt = g;
          gt.partial = nullptr;
          int cfg = choose_cfg("gemm", EPI_CONC, bf16, 0, g.M, g.N, g.K, c.st, dense_cands(g.M, g.N),
                               [&](int cf) { return launch_gemm(bf16, cf, EPI_CONC, gt, &a, c.st); });
          g.partial = ws.partial.as<double>(); g.slot0 = slot;
          const double M = g.M, esz = bf16 ? 2 : 4;
          const double bytes = M * g.K * esz + (double)g.N * g.K * esz + (keep_ahat ? M * g.N : 0) +
                               M * nnz_of(c, -1) * 4 * (want_contrib ? 2 : 1) + M * nslot * 8;
          if (!record_gemm(c, bf16, cfg, EPI_CONC, g, a, Bytes{bytes, 0.0}))
            check(timed(c.st, cls_name("conc", bf16, 0, cfg), Bytes{bytes, 0.0}, 2.0 * g.M * g.N * g.K,
                        [&] { return launch_gemm(bf16, cfg, EPI_CONC, g, &a, c.st); }));
        }
      }
      slot += nslot;
      return;
    }
    if (E.kind == GCP_EDGE_CONV) {
      no_record(c, "conv");
      const ConvGeom& cg = E.cg;
      ConvArgs ca{};
      ca.M = c.M; ca.cg = cg; ca.trans = 1;
      ca.X = ws.lam[E.dst]->p; ca.ldx = dn.ld; ca.x_is_sign = 0;
      ca.Bt = bf16 ? E.WT16.p : E.WT32.p; ca.ldb = E.ldk_t;
      ca.Btf = (const float*)(bf16 ? E.WT16f.p : E.WT32.p);
      ca.mp = c.rp.mp; ca.partial = nullptr;
      const double M = c.M, esz = bf16 ? 2 : 4;
      // every multiply-add of the forward conv appears once in its transpose
      const double flops = 2.0 * M * cg.ho * cg.wo * cg.ci * cg.co * cg.kh * cg.kw;
      const double wbytes = (double)cg.stride * cg.stride * cg.ci * E.ldk_t * esz;
      if (!last) {
        StoreEpiArgs s{d_src, ld_src, 1.f, first ? nullptr : accbuf, accbuf};
        if (!dry) {
          int cfg = choose_cfg("convT", EPI_STORE, bf16, 0, c.M, d_src, dn.size, c.st, conv_cands(), [&](int cf) {
            StoreEpiArgs t = s;
            t.acc_in = nullptr;
            t.out = tune_store(c);
            return launch_conv(bf16, cf, EPI_STORE, ca, &t, c.st);
          });
          const double bytes = M * dn.size * esz + wbytes + M * d_src * 4 * (first ? 1 : 2);
          check(timed(c.st, cls_name("convT_store", bf16, 0, -1), Bytes{bytes, 0.0}, flops,
                      [&] { return launch_conv(bf16, cfg, EPI_STORE, ca, &s, c.st); }));
        }
        return;
      }
      const int nslot = conv_slots(cg, 1);
      if (p >= 0) {
        BoundEpiArgs a = bound_args(p, has_acc);
        if (!dry) {
          int cfg = choose_cfg("convT", pi ? EPI_BOUND + kPiKey : EPI_BOUND, bf16, 0, c.M, d_src, dn.size, c.st,
                               pi ? pi_conv_cands() : conv_cands(),
                               [&](int cf) { return launch_conv(bf16, cf, EPI_BOUND, ca, &a, c.st); });
          ConvArgs cr = ca;
          cr.partial = ws.partial.as<double>(); cr.slot0 = slot;
          const double bytes = M * dn.size * esz + wbytes + M * d_src * esz + (keep_ahat ? M * d_src * esz : 0) +
                               M * unst_of(c, p) * (pi ? 8 : 4) + (double)c.B * unst_of(c, p) + M * nnz_of(c, p) * 4 +
                               (has_acc ? M * d_src * 4 : 0) + M * nslot * 8;
          check(timed(c.st, cls_name(pi ? "convT_bound_pi" : "convT_bound", bf16, 0, -1), Bytes{bytes, alg_bound(c, p)},
                      flops,
                      [&] { return launch_conv(bf16, cfg, EPI_BOUND, cr, &a, c.st); }));
        }
      } else {
        if (has_acc) fail(GCP_EUNSUPPORTED, "several consumers of the input");
        ConcEpiArgs a{};
        a.size = net->in_size; a.ld = net->in_ld; a.x0 = c.x0; a.eps = c.eps;
        a.cc = cut_col(c, -1); a.rp = c.rp;
        a.sign_out = keep_ahat ? ws.sign.as<int8_t>() : nullptr;
        a.contrib = want_contrib ? ws.contrib.as<float>() : nullptr;
        a.nnz_e = c.nnz;
        if (!dry) {
          int cfg = choose_cfg("convT", EPI_CONC, bf16, 0, c.M, d_src, dn.size, c.st, conc_conv_cands(cg),
                               [&](int cf) { return launch_conv(bf16, cf, EPI_CONC, ca, &a, c.st); });
          ConvArgs cr = ca;
          cr.partial = ws.partial.as<double>(); cr.slot0 = slot;
          const double bytes = M * dn.size * esz + wbytes + (keep_ahat ? M * d_src : 0) +
                               M * nnz_of(c, -1) * 4 * (want_contrib ? 2 : 1) + M * nslot * 8;
          check(timed(c.st, cls_name("convT_conc", bf16, 0, -1) + (cfg == kConvDirectCfg ? ".direct" : ""),
                      Bytes{bytes, 0.0}, flops,
                      [&] { return launch_conv(bf16, cfg, EPI_CONC, cr, &a, c.st); }));
        }
      }
      slot += nslot;
      return;
    }
    if (E.kind == GCP_EDGE_IDENTITY) {
      no_record(c, "identity");
      if (p < 0) fail(GCP_EUNSUPPORTED, "identity edge from the network input");
      if (!last) {
        if (!bf16 && first && total == 2 && dn.ld == ld_src) {
          acc_alias[p] = ws.lam[E.dst]->as<float>();   // the last push reads it in place of the buffer
          return;
        }
        if (!dry)
          check(launch_identity_acc(bf16, c.M, d_src, ws.lam[E.dst]->p, dn.ld, 0, 1.f, first ? nullptr : accbuf,
                                    accbuf, ld_src, c.st));
        return;
      }
      BoundEpiArgs a = bound_args(p, has_acc);
      const int nslot = slots_for_elementwise(d_src);
      if (!dry)
        check(timed(c.st, cls_name("bound_elem", bf16, 0, -1), Bytes{(double)c.M * d_src * 16, alg_bound(c, p)}, 0.0, [&] {
          return launch_bound_elementwise(bf16, nullptr, ws.lam[E.dst]->p, a, ws.partial.as<double>(), slot, c.st);
        }));
      slot += nslot;
      return;
    }
    fail(GCP_EUNSUPPORTED, "unknown edge kind in the bound pass");
  }
};

// ---------------------------------------------------------------- adjoint
// What the adjoint adds to d Lambda^(i) (the derivative of the Lambda.b and
// input terms): the bias, plus W x0 for a node fed by the network input (made
// per call by AdjPass::prepare into the workspace).
const float* add_vec_of(const Call& c, int i) {
  const NodeH& n = c.net->nodes[i];
  for (int eid : n.in_edges)
    if (c.net->edges[eid]->src < 0) return c.ws->addv[i]->as<float>();
  return n.bias.as<float>();
}

struct AdjPass {
  Call& c;
  int bf16;
  AdamArgs adam;
  float* d_alpha; float* d_beta;
  float* alpha_rw; float* beta_rw;
  float *ma, *va, *mb, *vb;
  float* d_rho = nullptr; float* rho_rw = nullptr;   // explicit pi (c.rp.rho set)
  float* mr = nullptr; float* vr = nullptr;

  void check(hipError_t e) { hip_check(e, "kernel launch (adjoint)"); }

  // add vectors of the nodes fed by the input: bias + A x0, once per call
  // (the other nodes add their bias, read in place: add_vec_of)
  void prepare() {
    gcp_net* net = c.net;
    auto& ws = *c.ws;
    for (int i = 0; i < net->out; ++i) {
      const NodeH& n = net->nodes[i];
      bool seeded = false;
      for (int eid : n.in_edges) {
        const EdgeH& E = *net->edges[eid];
        if (E.src >= 0) continue;
        int kind = E.kind == GCP_EDGE_DENSE ? 0 : (E.kind == GCP_EDGE_CONV ? 1 : 2);
        check(launch_wx0(&E.cg, kind, E.Wraw.as<float>(), n.size, net->in_size, c.x0,
                         seeded ? nullptr : n.bias.as<float>(), ws.addv[i]->as<float>(), c.st));
        seeded = true;
      }
    }
  }

  void run() {
    for (int i = 0; i < c.net->out; ++i) node(i);
  }

  // a_hat of node i again from its consumer's Lambda: the bound pass's GEMM
  // (same operands, same tile configuration) with only the a_hat epilogue
  void recompute_ahat(int i) {
    gcp_net* net = c.net;
    auto& ws = *c.ws;
    if (c.rec) fail(GCP_EUNSUPPORTED, "a_hat recomputation in grouped launches");
    const NodeH& n = net->nodes[i];
    const EdgeH& E = *net->edges[n.consumers[0]];
    const NodeH& dn = net->nodes[E.dst];
    BoundEpiArgs a{};
    a.nd = n.dev();
    a.cc = cut_col(c, i);
    a.rp = c.rp;
    a.ahat_out = ws.ahat_tmp.p;
    const double M = c.M, esz = bf16 ? 2 : 4;
    if (E.kind == GCP_EDGE_DENSE) {
      GemmArgs g{};
      g.M = c.M; g.N = E.d_src; g.K = dn.size;
      g.A = ws.lam[E.dst]->p; g.lda = dn.ld;
      g.Bt = wt_bound(E, bf16); g.ldb = dn.ld;
      g.mp = c.rp.mp;
      const int cfg = choose_cfg("gemm", EPI_BOUND, bf16, 0, g.M, g.N, g.K, c.st, dense_cands(g.M, g.N),
                                 [&](int cf) { return launch_gemm(bf16, cf, EPI_AHAT, g, &a, c.st); });
      const double bytes = M * g.K * esz + (double)g.N * g.K * esz + M * g.N * esz + M * nnz_of(c, i) * 4;
      check(timed(c.st, cls_name("ahat", bf16, 0, cfg), Bytes{bytes, 0.0}, 2.0 * g.M * g.N * g.K,
                  [&] { return launch_gemm(bf16, cfg, EPI_AHAT, g, &a, c.st); }));
    } else {
      ConvArgs ca{};
      ca.M = c.M; ca.cg = E.cg; ca.trans = 1;
      ca.X = ws.lam[E.dst]->p; ca.ldx = dn.ld; ca.x_is_sign = 0;
      ca.Bt = bf16 ? E.WT16.p : E.WT32.p; ca.ldb = E.ldk_t;
      ca.Btf = (const float*)(bf16 ? E.WT16f.p : E.WT32.p);
      ca.mp = c.rp.mp; ca.partial = nullptr;
      const ConvGeom& cg = E.cg;
      const int cfg = choose_cfg("convT", EPI_BOUND, bf16, 0, c.M, E.d_src, dn.size, c.st, conv_cands(),
                                 [&](int cf) { return launch_conv(bf16, cf, EPI_AHAT, ca, &a, c.st); });
      const double bytes = M * dn.size * esz + (double)cg.stride * cg.stride * cg.ci * E.ldk_t * esz +
                           M * E.d_src * esz + M * nnz_of(c, i) * 4;
      check(timed(c.st, cls_name("convT_ahat", bf16, 0, -1), Bytes{bytes, 0.0},
                  2.0 * M * cg.ho * cg.wo * cg.ci * cg.co * cg.kh * cg.kw,
                  [&] { return launch_conv(bf16, cfg, EPI_AHAT, ca, &a, c.st); }));
    }
  }

  void node(int i) {
    gcp_net* net = c.net;
    auto& ws = *c.ws;
    const NodeH& n = net->nodes[i];
    if (!c.recompute.empty() && c.recompute[i]) recompute_ahat(i);
    std::vector<int> order;   // identity edges first: they can only accumulate
    for (int eid : n.in_edges)
      if (net->edges[eid]->kind == GCP_EDGE_IDENTITY) order.push_back(eid);
    for (int eid : n.in_edges)
      if (net->edges[eid]->kind != GCP_EDGE_IDENTITY) order.push_back(eid);
    float* accbuf = ws.acc[i]->p ? ws.acc[i]->as<float>() : nullptr;
    // what the fused epilogue reads as the accumulated dLambda: the buffer, or,
    // when an identity edge from an fp32 d a_hat is the first of exactly two
    // edges and the other is a GEMM edge (its copy into the buffer would be
    // exact), that d a_hat itself
    const float* acc_rd = accbuf;
    // the node's adjoint epilogue runs fused with its last GEMM, or
    // elementwise after all edges when the last edge is an identity
    const bool pi = c.rp.rho != nullptr;
    const bool fused_last = net->edges[order.back()]->kind != GCP_EDGE_IDENTITY;
    const bool use_acc = order.size() > 1 || !fused_last;
    const double M = c.M, esz = bf16 ? 2 : 4, di = n.size;
    auto adj_bytes = [&](double a_bytes, double w_bytes) {
      return a_bytes + w_bytes + M * di * esz + M * unst_of(c, i) * (adam.enabled ? 24 : 8) * (pi ? 2 : 1) +
             (double)c.B * unst_of(c, i) + M * nnz_of(c, i) * 8 + M * di * esz + (use_acc ? M * di * 4 : 0);
    };
    for (size_t q = 0; q < order.size(); ++q) {
      const EdgeH& E = *net->edges[order[q]];
      const bool last = q + 1 == order.size();
      const bool first = q == 0;
      const int p = E.src;
      const bool sign = p < 0;
      const float scale = sign ? (float)(-c.eps) : 1.f;
      const void* A = sign ? ws.sign.p : ws.dahat[p]->p;
      const int lda = sign ? net->in_ld : net->nodes[p].ld;
      const double a_bytes = M * E.d_src * (sign ? 1 : esz);
      if (E.kind == GCP_EDGE_DENSE) {
        GemmArgs g{};
        g.M = c.M; g.N = n.size; g.K = E.d_src;
        g.A = A; g.lda = lda;
        g.Bt = w_adj(E, bf16); g.ldb = lda;
        g.a_is_sign = sign;
        g.mp = c.rp.mp;
        if (!last || !fused_last) {
          StoreEpiArgs s{n.size, n.ld, scale, first ? nullptr : accbuf, accbuf};
          int cfg = choose_cfg("gemm", EPI_STORE, bf16, sign, g.M, g.N, g.K, c.st, dense_cands(g.M, g.N), [&](int cf) {
            StoreEpiArgs t = s;
            t.acc_in = nullptr;
            t.out = tune_store(c);
            return launch_gemm(bf16, cf, EPI_STORE, g, &t, c.st);
          });
          const double bytes = a_bytes + (double)g.N * g.K * esz + M * di * 4 * (first ? 1 : 2);
          if (!record_gemm(c, bf16, cfg, EPI_STORE, g, s, Bytes{bytes, 0.0}))
            check(timed(c.st, cls_name("store", bf16, sign, cfg), Bytes{bytes, 0.0}, 2.0 * g.M * g.N * g.K,
                        [&] { return launch_gemm(bf16, cfg, EPI_STORE, g, &s, c.st); }));
        } else {
          AdjEpiArgs a = epi(i, use_acc ? acc_rd : nullptr, scale);
          int cfg = choose_cfg("gemm", pi ? EPI_ADJ + kPiKey : EPI_ADJ, bf16, sign, g.M, g.N, g.K, c.st,
                               pi ? pi_dense_cands(g.M, g.N) : dense_cands(g.M, g.N), [&](int cf) {
            AdjEpiArgs t = a;     // gradient-only trial into scratch: no parameter moves
            t.adam.enabled = 0;
            t.d_alpha = tune_alpha(c);
            t.d_beta = tune_beta(c);
            if (pi) t.d_rho = t.d_alpha;   // same [M][n_I] shape, each element written by one thread
            return launch_gemm(bf16, cf, EPI_ADJ, g, &t, c.st);
          });
          const double bytes = adj_bytes(a_bytes, (double)g.N * g.K * esz);
          if (!record_gemm(c, bf16, cfg, EPI_ADJ, g, a, Bytes{bytes, alg_adj(c, i, adam.enabled)}))
            check(timed(c.st, pi ? cls_name("adj_pi", bf16, sign, pi_cfg(cfg)) : cls_name("adj", bf16, sign, cfg),
                        Bytes{bytes, alg_adj(c, i, adam.enabled)},
                        2.0 * g.M * g.N * g.K, [&] { return launch_gemm(bf16, cfg, EPI_ADJ, g, &a, c.st); }));
        }
      } else if (E.kind == GCP_EDGE_CONV) {
        no_record(c, "conv");
        ConvArgs ca{};
        ca.M = c.M; ca.cg = E.cg; ca.trans = 0;
        ca.X = A; ca.ldx = lda; ca.x_is_sign = sign;
        ca.Bt = bf16 ? E.W16.p : E.W32.p; ca.ldb = E.ldk_f;
        ca.mp = c.rp.mp; ca.partial = nullptr;
        const int HW = E.cg.ho * E.cg.wo;
        const double flops = 2.0 * M * HW * E.cg.co * E.cg.ci * E.cg.kh * E.cg.kw;
        const double wbytes = (double)E.cg.co * E.ldk_f * esz;
        if (!last || !fused_last) {
          StoreEpiArgs s{n.size, n.ld, scale, first ? nullptr : accbuf, accbuf};
          int cfg = choose_cfg("conv", EPI_STORE, bf16, sign, c.M, n.size, E.d_src, c.st, conv_cands(), [&](int cf) {
            StoreEpiArgs t = s;
            t.acc_in = nullptr;
            t.out = tune_store(c);
            return launch_conv(bf16, cf, EPI_STORE, ca, &t, c.st);
          });
          check(timed(c.st, cls_name("conv_store", bf16, sign, -1), Bytes{a_bytes + wbytes + M * di * 4 * (first ? 1 : 2), 0.0},
                      flops, [&] { return launch_conv(bf16, cfg, EPI_STORE, ca, &s, c.st); }));
        } else {
          AdjEpiArgs a = epi(i, use_acc ? acc_rd : nullptr, scale);
          int cfg = choose_cfg("conv", pi ? EPI_ADJ + kPiKey : EPI_ADJ, bf16, sign, c.M, n.size, E.d_src, c.st,
                               pi ? pi_conv_cands() : conv_cands(), [&](int cf) {
            AdjEpiArgs t = a;
            t.adam.enabled = 0;
            t.d_alpha = tune_alpha(c);
            t.d_beta = tune_beta(c);
            if (pi) t.d_rho = t.d_alpha;   // same [M][n_I] shape, each element written by one thread
            return launch_conv(bf16, cf, EPI_ADJ, ca, &t, c.st);
          });
          check(timed(c.st, cls_name(pi ? "conv_adj_pi" : "conv_adj", bf16, sign, -1),
                      Bytes{adj_bytes(a_bytes, wbytes), alg_adj(c, i, adam.enabled)}, flops,
                      [&] { return launch_conv(bf16, cfg, EPI_ADJ, ca, &a, c.st); }));
        }
      } else {   // identity: accumulate; the node's relaxation runs after the last edge
        no_record(c, "identity");
        if (!bf16 && !sign && first && !last && fused_last && order.size() == 2 && lda == n.ld) {
          acc_rd = (const float*)A;
          continue;
        }
        check(launch_identity_acc(bf16, c.M, n.size, A, lda, sign, scale, first ? nullptr : accbuf, accbuf, n.ld,
                                  c.st));
      }
    }
    if (!fused_last) {
      AdjEpiArgs a = epi(i, accbuf, 0.f);
      check(timed(c.st, cls_name("adj_elem", bf16, 0, -1), Bytes{adj_bytes(0, 0), alg_adj(c, i, adam.enabled)}, 0.0,
                  [&] { return launch_adj_elementwise(bf16, a, c.st); }));
    }
  }

  AdjEpiArgs epi(int i, const float* acc_in, float scale) {
    gcp_net* net = c.net;
    auto& ws = *c.ws;
    const NodeH& n = net->nodes[i];
    AdjEpiArgs a{};
    a.nd = n.dev();
    a.cc = cut_col(c, i);
    a.rp = c.rp;
    a.acc_in = acc_in;
    a.gemm_scale = scale;
    a.add_vec = add_vec_of(c, i);
    a.ahat = c.recompute.empty() || !c.recompute[i] ? ws.ahat[i]->p : ws.ahat_tmp.p;
    a.dahat_out = ws.dahat[i]->p;
    a.contrib = c.nnz ? ws.contrib.as<float>() : nullptr;
    a.nnz_e = c.nnz;
    a.d_alpha = d_alpha; a.d_beta = d_beta;
    a.m_alpha = ma; a.v_alpha = va; a.m_beta = mb; a.v_beta = vb;
    a.alpha_rw = alpha_rw; a.beta_rw = beta_rw;
    a.adam = adam;
    a.d_rho = d_rho; a.rho_rw = rho_rw; a.m_rho = mr; a.v_rho = vr;
    return a;
  }
};

void prepare_call(Call& c, gcp_net* net, const double* x0, double eps, const double* C, int32_t S,
                  const gcp_splits* splits, const gcp_cuts* cuts, const float* alpha, const float* beta,
                  const float* gamma, void* stream) {
  if (!net) fail(GCP_EINVAL, "null net");
  if (!splits) fail(GCP_EINVAL, "null splits (use a handle with K = 0 for no splits)");
  if (splits->net != net) fail(GCP_EINVAL, "splits were created for another net");
  if (cuts && cuts->net != net) fail(GCP_EINVAL, "cuts were created for another net");
  if (!x0 || !C) fail(GCP_EINVAL, "null x0 or C");
  if (!(eps >= 0.0) || !std::isfinite(eps)) fail(GCP_ERANGE, "eps must be finite and >= 0");
  if (S <= 0) fail(GCP_EINVAL, "S must be >= 1");
  int N = cuts ? cuts->N : 0;
  if (net->n_I > 0 && !alpha) fail(GCP_EINVAL, "null alpha");
  if (splits->K > 0 && !beta) fail(GCP_EINVAL, "null beta");
  if (N > 0 && !gamma) fail(GCP_EINVAL, "null gamma");
  int dev;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (dev != net->device) fail(GCP_EINVAL, "current device differs from the net's device");
  c.net = net; c.cuts = (cuts && cuts->N > 0) ? cuts : nullptr; c.splits = splits;
  c.x0 = x0; c.eps = eps; c.C = C; c.S = S; c.B = splits->B;
  long long M = (long long)splits->B * S;
  if (M > (1LL << 30)) fail(GCP_EINVAL, "too many rows");
  c.M = (int)M;
  c.nnz = c.cuts ? c.cuts->nnz_e : 0;
  c.st = (hipStream_t)stream;
  c.N = N;
  if (!c.no_alloc) {
    ensure_ws(c);
    c.ws = &net->ws;
  }
  c.rp = RowParams{c.M, S, round_up(c.M, 16), alpha, net->n_I, beta, splits->K,
                   c.ws ? c.ws->gammaT.as<float>() : nullptr, N,
                   splits->K > 0 ? splits->mask.as<int8_t>() : nullptr, 1.0 / S,
                   nullptr /* rho: set by the explicit-pi entry points */};
}

// Which nodes recompute a_hat in the adjoint (Theorem 3.1 needs a_hat of
// every ReLU layer there): a node whose a_hat comes from a single dense or
// conv consumer can rebuild it from that consumer's stored Lambda with one
// more GEMM, so only one layer's a_hat is live at a time instead of all of
// them.  GCP_FLAG_RECOMPUTE forces it, GCP_FLAG_STORE_AHAT disables it;
// otherwise it is used when the stored a_hat of all layers would exceed
// GCP_AHAT_BUDGET_MB, by default half of the device memory that is free
// or already held by a_hat buffers when the call is planned (storing is
// the faster form wherever it fits).  Sizes the buffers either way.
bool ahat_recomputable(const gcp_net* net, int i) {
  const NodeH& n = net->nodes[i];
  if (!n.relu || n.consumers.size() != 1) return false;
  const EdgeH& E = *net->edges[n.consumers[0]];
  return (E.kind == GCP_EDGE_DENSE || E.kind == GCP_EDGE_CONV) && E.dst != net->out;
}
void plan_ahat(Call& c, int32_t mode) {
  gcp_net* net = c.net;
  auto& ws = *c.ws;
  const int nn = (int)net->nodes.size();
  size_t stored = 0;
  for (int i = 0; i < nn; ++i)
    if (net->nodes[i].relu) stored += (size_t)c.M * net->nodes[i].ld * 4;
  const char* e = std::getenv("GCP_AHAT_BUDGET_MB");
  double budget = 8192.0 * 1048576.0;
  if (e && *e) {
    budget = std::atof(e) * 1048576.0;
  } else {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
      size_t held = ws.ahat_tmp.bytes;
      for (int i = 0; i < nn; ++i) held += ws.ahat[i]->bytes;
      budget = 0.5 * (double)(fr + held);
    }
  }
  const bool want = (mode & GCP_FLAG_RECOMPUTE) || (!(mode & GCP_FLAG_STORE_AHAT) && (double)stored > budget);
  c.recompute.assign(nn, 0);
  size_t tmp = 0;
  for (int i = 0; i < nn; ++i) {
    const NodeH& n = net->nodes[i];
    if (!n.relu) continue;
    const size_t bytes = (size_t)c.M * n.ld * 4;
    if (want && ahat_recomputable(net, i)) {
      c.recompute[i] = 1;
      tmp = std::max(tmp, bytes);
    } else if (ws.ahat[i]->bytes < bytes) {
      ws.ahat[i]->alloc(bytes);
      ws.gen = next_generation();
    }
  }
  if (ws.ahat_tmp.bytes < tmp) {
    ws.ahat_tmp.alloc(tmp);
    ws.gen = next_generation();
  }
}

void size_partials(Call& c, int bf16, bool keep, bool contrib) {
  BoundPass dry(c, bf16, keep, contrib, true);
  dry.run();
  auto& ws = *c.ws;
  const size_t need = (size_t)round_up(ws.M, 16) * (dry.slot + 1) * 8;   // + the outward-rounding slot
  if (need > ws.partial.bytes) {
    ws.partial.alloc(need);
    ws.gen = next_generation();
  }
  ws.n_slots = dry.slot;
}

void validate_params(Call& c, const float* alpha, const float* beta, const float* gamma) {
  auto& ws = *c.ws;
  hip_check(hipMemsetAsync(ws.flags.p, 0, 16, c.st), "hipMemsetAsync");
  int* f = ws.flags.as<int>();
  hip_check(launch_validate(alpha, (int64_t)c.M * c.rp.n_I, 0.f, 1.f, f, c.st), "validate");
  if (c.rp.rho) hip_check(launch_validate(c.rp.rho, (int64_t)c.M * c.rp.n_I, 0.f, 1.f, f, c.st), "validate");
  hip_check(launch_validate(beta, (int64_t)c.M * c.rp.K, 0.f, INFINITY, f, c.st), "validate");
  hip_check(launch_validate(gamma, (int64_t)c.M * c.N, 0.f, INFINITY, f, c.st), "validate");
  int h = 0;
  hip_check(hipMemcpyAsync(&h, f, 4, hipMemcpyDeviceToHost, c.st), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(c.st), "hipStreamSynchronize");
  if (h & 1) fail(GCP_ENONFINITE, "non-finite alpha, beta or gamma");
  if (h & 2) fail(GCP_ERANGE, "alpha or rho outside [0,1] or a negative multiplier");
}

// fp64 words of the combined outward-rounding weights (every node's ld, then X_in)
size_t slack_words(const gcp_net* net) {
  size_t w = 1;
  for (const NodeH& n : net->nodes) w += n.ld;
  return w;
}

// GCP_FLAG_OUTWARD: minus each row's rounding slack into partial slot `slot`
// (bounds and the derivation at SlackArgs; the constants below follow it).
void launch_outward(Call& c, int bf16, int slot) {
  gcp_net* net = c.net;
  auto& ws = *c.ws;
  const int nn = (int)net->nodes.size();
  if (nn > kSlackMaxNodes) fail(GCP_EUNSUPPORTED, "outward rounding handles nets of at most 64 nodes");
  SlackArgs a{};
  a.n_nodes = nn;
  int off = 0;
  for (int i = 0; i < nn; ++i) {
    const NodeH& n = net->nodes[i];
    const bool has_lam = n.relu || net->out_general;
    a.nodes[i] = SlackNode{n.slack_w.as<double>(), n.ld, n.size, off, has_lam ? ws.lam[i]->p : nullptr};
    off += n.ld;
  }
  const size_t words = slack_words(net);
  if (!c.no_alloc && ws.slackw.bytes < words * 8) ws.slackw.alloc(words * 8);
  if (ws.slackw.bytes < words * 8) fail(GCP_ENOMEM, "no room for the outward-rounding weights");
  a.total = off;
  a.wcomb = ws.slackw.as<double>();
  a.M = c.M; a.S = c.S; a.mp = c.rp.mp; a.bf16 = bf16;
  // u_op: operand rounding (bf16 weights and stored Lambda), e_r: the few
  // fp32 operations of a relaxation, e_st: Lambda stored vs the value its
  // row constant used, e64: the fp64 sums of a row
  const double u_op = bf16 ? 0x1p-8 : 0.0, e_r = 0x1p-20, e_st = bf16 ? 0x1p-8 : 0x1p-22;
  const double n64 = (double)net->n_relu + net->nodes[net->out].size + net->in_size + c.rp.N + slot + 64;
  const double e64 = n64 * 0x1p-52;
  a.c_sum = u_op + e_r + e64;
  a.c_zb = e_st + e64;
  a.c_in = u_op + e64;
  a.x0 = c.x0; a.d_in = net->in_size; a.eps = c.eps;
  a.C = c.C; a.d_out = net->nodes[net->out].size;
  a.out_off = off - net->nodes[net->out].ld;
  a.out_chat = net->out_general ? 0 : 1;
  a.beta = c.rp.beta; a.K = c.rp.K;
  a.zsplit = c.rp.K > 0 ? c.splits->zsplit.as<double>() : nullptr;
  a.c_beta = e_r + e_st + e64;
  a.gammaT = c.rp.gammaT; a.N = c.rp.N;
  a.kap = c.rp.N > 0 ? c.cuts->kap.as<double>() : nullptr;
  a.c_cut = acc_bound((c.cuts ? c.cuts->col_max : 0) + 4.0) + e_r + e_st + e64;
  a.c_d = e64;
  a.out = ws.partial.as<double>() + (size_t)slot * c.rp.mp;
  hip_check(timed(c.st, "outward_slack", Bytes{(double)c.M * (off * (bf16 ? 2.0 : 4.0) + 8.0), 0.0}, 0.0,
                  [&] { return launch_slack(a, c.st); }),
            "outward slack");
}

void bound_pass(Call& c, int bf16, bool keep_ahat, bool contrib, double* bound, uint8_t* verified) {
  size_partials(c, bf16, keep_ahat, contrib);
  BoundPass bp(c, bf16, keep_ahat, contrib, false);
  bp.run();
  auto& ws = *c.ws;
  const int n_slots = ws.n_slots + (c.outward ? 1 : 0);
  if (c.outward) launch_outward(c, bf16, ws.n_slots);
  const double rb = (double)c.M * (n_slots * 8.0 + c.rp.N * 4.0 + 8.0 + (verified ? 1 : 0));
  hip_check(timed(c.st, "reduce_rows", Bytes{rb, 0.0}, 0.0, [&] {
              return launch_reduce_rows(c.M, c.rp.mp, c.S, ws.partial.as<double>(), n_slots, ws.cb.as<double>(),
                                        c.rp.gammaT, c.rp.N, c.cuts ? c.cuts->d.as<double>() : nullptr, bound,
                                        verified, c.st);
            }),
            "reduce");
}

// The workspace of a bound call (with gradients when `grads`) laid out in the
// static scratch region instead of the net's own buffers: every buffer the
// call reads it also writes first, so nothing needs clearing; a_hat of every
// layer is stored (no recomputation).  Fails with ENOMEM when the call needs
// more than the region holds.
void carve_static(Call& c, gcp_net::WS& sws, int bf16, bool grads) {
  gcp_net* net = c.net;
  const int nn = (int)net->nodes.size();
  for (int i = 0; i < nn; ++i) {
    sws.lam.push_back(std::make_unique<DBuf>());
    sws.ahat.push_back(std::make_unique<DBuf>());
    sws.dahat.push_back(std::make_unique<DBuf>());
    sws.acc.push_back(std::make_unique<DBuf>());
    sws.addv.push_back(std::make_unique<DBuf>());
  }
  sws.chat_off.assign(nn, -1);
  size_t chat_floats = 0;
  if (!net->out_general)
    for (int eid : net->nodes[net->out].in_edges) {
      const int p = net->edges[eid]->src;
      sws.chat_off[p] = (int)chat_floats;
      chat_floats += (size_t)c.S * net->nodes[p].ld;
    }
  c.ws = &sws;
  c.recompute.assign(nn, 0);
  BoundPass dry(c, bf16, grads, grads && c.nnz > 0, true);
  dry.run();
  void* base = nullptr;
  size_t cap = 0;
  hip_check(scratch_region(&base, &cap), "static workspace");
  const size_t M = c.M, mp = c.rp.mp;
  size_t off = 0;
  auto take = [&](DBuf& b, size_t n) {
    off = (off + 255) / 256 * 256;
    b.borrow(n && off + n <= cap ? (char*)base + off : nullptr, n);
    off += n;
  };
  for (int i = 0; i < nn; ++i) {
    const NodeH& n = net->nodes[i];
    const size_t elems = (n.relu || (i == net->out && net->out_general)) ? M * n.ld : 0;
    bool ident = false;
    for (int eid : n.in_edges) ident |= net->edges[eid]->kind == GCP_EDGE_IDENTITY;
    for (int eid : n.consumers) ident |= net->edges[eid]->kind == GCP_EDGE_IDENTITY;
    const bool multi = n.relu && (n.consumers.size() > 1 || n.in_edges.size() > 1 || ident);
    take(*sws.lam[i], elems * 4);
    take(*sws.acc[i], multi ? elems * 4 : 0);
    if (grads) {
      take(*sws.ahat[i], n.relu ? elems * 4 : 0);
      take(*sws.dahat[i], elems * 4);
      take(*sws.addv[i], n.relu ? (size_t)n.ld * 4 : 0);
    }
  }
  if (grads) take(sws.sign, M * net->in_ld);
  if (grads && c.nnz) take(sws.contrib, mp * c.nnz * 4);
  if (c.N) take(sws.gammaT, mp * c.N * 4);
  take(sws.chat, std::max<size_t>(chat_floats, 1) * 4);
  take(sws.cb, (size_t)c.S * 8);
  take(sws.consts, 16);
  take(sws.step, 16);
  take(sws.flags, 16);
  take(sws.partial, mp * (dry.slot + 1) * 8);   // + the outward-rounding slot
  if (c.outward) take(sws.slackw, slack_words(net) * 8);
  if (off > cap) {
    char m[200];
    std::snprintf(m, sizeof m, "the call needs %.1f MiB of workspace; the static workspace holds %.0f MiB",
                  off / 1048576.0, cap / 1048576.0);
    fail(GCP_ENOMEM, m);
  }
  sws.M = c.M; sws.S = c.S; sws.nnz = c.nnz; sws.N = c.N;
  sws.n_slots = 0;
  c.rp.gammaT = sws.gammaT.as<float>();
}

// gcp_bound and gcp_bound_pi (rho non-null: explicit pi); no_alloc: the
// workspace is the static scratch region (gcp_bound_noalloc)
void bound_impl(const gcp_net* net_c, const double* x0, double eps, const double* C, int32_t S,
                const gcp_splits* splits, const gcp_cuts* cuts, const float* alpha, const float* beta,
                const float* gamma, const float* rho, int32_t mode, double* bound, uint8_t* verified, float* d_alpha,
                float* d_beta, float* d_gamma, float* d_rho, void* stream, bool no_alloc = false) {
  gcp_net* net = const_cast<gcp_net*>(net_c);
  Call c{};
  c.no_alloc = no_alloc;
  gcp_net::WS sws;
  prepare_call(c, net, x0, eps, C, S, splits, cuts, alpha, beta, gamma, stream);
  c.rp.rho = rho;
  const int bf16 = (mode & 0xff) == GCP_MODE_BF16;
  if ((mode & 0xff) != GCP_MODE_FP32 && !bf16) fail(GCP_EINVAL, "unknown mode");
  if (!bound) fail(GCP_EINVAL, "null bound output");
  const bool grads = d_alpha || d_beta || d_gamma;
  c.outward = (mode & GCP_FLAG_OUTWARD) != 0;
  if (grads) {
    if ((net->n_I > 0 && !d_alpha) || (splits->K > 0 && !d_beta) || (c.rp.N > 0 && !d_gamma) ||
        (rho && net->n_I > 0 && !d_rho))
      fail(GCP_EINVAL, "pass all gradient outputs or none");
  }
  if (no_alloc) {
    if (mode & GCP_FLAG_VALIDATE) fail(GCP_EINVAL, "GCP_FLAG_VALIDATE waits for the device; not available here");
    carve_static(c, sws, bf16, grads);
  }
  if (mode & GCP_FLAG_VALIDATE) validate_params(c, alpha, beta, gamma);
  if (c.N > 0) hip_check(launch_transpose(gamma, c.M, c.N, c.N, c.ws->gammaT.as<float>(), c.rp.mp, c.st), "transpose");
  if (grads && !no_alloc) plan_ahat(c, mode);
  bound_pass(c, bf16, grads, grads && c.nnz > 0, bound, verified);
  if (grads) {
    if (splits->K > 0) hip_check(launch_fill_f32(d_beta, (int64_t)c.M * splits->K, 0.f, c.st), "fill");
    AdjPass ap{c, bf16, AdamArgs{0, 0.f, 0.f, 0.f, nullptr}, d_alpha, d_beta, nullptr, nullptr,
               nullptr, nullptr, nullptr, nullptr, rho ? d_rho : nullptr};
    ap.prepare();
    ap.run();
    if (c.rp.N > 0)
      hip_check(timed(c.st, "gamma_grad", Bytes{(double)c.M * (c.nnz * 4.0 + c.rp.N * 4.0), (double)c.M * c.rp.N * 8.0},
                      0.0, [&] {
                  return launch_gamma_update(c.M, c.rp.mp, c.rp.N, c.cuts->row_ptr.as<int32_t>(),
                                             c.ws->contrib.as<float>(), c.cuts->d.as<double>(), nullptr, d_gamma,
                                             nullptr, nullptr, AdamArgs{0, 0.f, 0.f, 0.f, nullptr}, c.st);
                }),
                "gamma gradient");
  }
}

// ---------------------------------------------------------------- fused dense chains
// Whether the whole optimisation can run in the fused chain kernel: ReLU
// nodes 0..L-1 each fed by one dense edge from the node before (node 0 by
// the input), each feeding only the next, the output fed by node L-1 through
// the c-hat form, Lemma A.1's pi*, a_hat stored, and the workgroup's LDS
// (two activation buffers of kChainRows rows plus the signs of v) within
// 160 KB.  Opt-in (GCP_FUSED=1): on MI355X it measured slower than the
// per-layer launches (one workgroup per 16 rows walks the layers in order, so
// far fewer tiles are in flight per layer, and the weights it streams are
// spread over all layers at once instead of one layer's at a time).
struct ChainPlan {
  bool ok = false;
  int P = 0, sign_ld = 0;
  size_t lds = 0;
};
ChainPlan chain_plan(const Call& c, int bf16) {
  ChainPlan pl;
  const char* e = std::getenv("GCP_FUSED");
  if (!e || e[0] != '1') return pl;
  const gcp_net* net = c.net;
  if (net->out_general || c.rp.rho || c.rec || c.M <= 0) return pl;
  const int out = net->out;
  if (out < 1 || net->in_consumers.size() != 1) return pl;
  int ldmax = 0;
  for (int i = 0; i <= out; ++i) {
    const NodeH& n = net->nodes[i];
    if (n.in_edges.size() != 1) return pl;
    const EdgeH& E = *net->edges[n.in_edges[0]];
    if (E.kind != GCP_EDGE_DENSE || E.src != i - 1) return pl;
    if (i < out && (n.consumers.size() != 1 || !n.relu)) return pl;
    if (i < out) ldmax = std::max(ldmax, n.ld);
  }
  if (!c.recompute.empty())
    for (uint8_t rc : c.recompute)
      if (rc) return pl;
  const int esz = bf16 ? 2 : 4;
  pl.P = ldmax + 16 / esz;                               // row pitch: an odd number of 16-byte units apart
  pl.sign_ld = (net->in_ld + 255) / 256 * 256 + 16;      // signs: rows 16 bytes apart modulo 256
  const size_t buf = (size_t)kChainRows * pl.P * esz;
  pl.lds = 2 * buf + (size_t)kChainRows * pl.sign_ld;
  pl.ok = pl.lds <= 160 * 1024;
  return pl;
}

// All `iters` Adam iterations of an eligible chain in one launch.
void run_chain(Call& c, int bf16, const ChainPlan& pl, float* alpha, float* beta, float* ma, float* va, float* mb,
               float* vb, float* mg, float* vg, const gcp_opt* opt) {
  gcp_net* net = c.net;
  auto& ws = *c.ws;
  const int L = net->out;
  if (!c.consts_done) {
    const NodeH& on = net->nodes[net->out];
    hip_check(launch_out_const(c.C, c.S, on.size, on.bias.as<float>(), ws.cb.as<double>(), c.st), "out const");
    const EdgeH& E = *net->edges[on.in_edges[0]];
    hip_check(launch_chat(c.C, c.S, on.size, E.Wraw.as<float>(), E.d_src, 0, ws.chat.as<float>() + ws.chat_off[E.src],
                          net->nodes[E.src].ld, c.st),
              "c-hat");
    c.consts_done = true;
  }
  ws.chain_host.resize(L);
  double flops = 0.0, elems = 0.0;
  for (int i = 0; i < L; ++i) {
    const NodeH& n = net->nodes[i];
    const EdgeH& E = *net->edges[n.in_edges[0]];
    ChainNode& cn = ws.chain_host[i];
    cn.nd = n.dev();
    cn.cc = cut_col(c, i);
    cn.WT = wt_bound(E, bf16);
    cn.ldWT = n.ld;
    cn.W = w_adj(E, bf16);
    cn.ldW = node_ld_of(net, i - 1);
    cn.addv = add_vec_of(c, i);
    cn.ahat = ws.ahat[i]->p;
    cn.dahat = ws.dahat[i]->p;
    flops += 4.0 * c.M * E.d_src * E.d_dst;   // the bound-pass and adjoint GEMM of the in-edge
    elems += n.size;
  }
  ws.chain_tab.ensure(sizeof(ChainNode) * L);
  hip_check(hipMemcpyAsync(ws.chain_tab.p, ws.chain_host.data(), sizeof(ChainNode) * L, hipMemcpyHostToDevice, c.st),
            "hipMemcpyAsync");
  ChainArgs a{};
  a.L = L;
  a.nodes = ws.chain_tab.as<ChainNode>();
  a.in_size = net->in_size;
  a.in_ld = net->in_ld;
  a.x0 = c.x0;
  a.eps = c.eps;
  a.cc_in = cut_col(c, -1);
  a.sign = ws.sign.as<int8_t>();
  a.chat = ws.chat.as<float>() + ws.chat_off[L - 1];
  a.chat_ld = net->nodes[L - 1].ld;
  a.rp = c.rp;
  a.gammaT = ws.gammaT.as<float>();
  a.contrib = ws.contrib.as<float>();
  a.nnz_e = c.nnz;
  a.row_ptr = c.cuts ? c.cuts->row_ptr.as<int32_t>() : nullptr;
  a.cut_d = c.cuts ? c.cuts->d.as<double>() : nullptr;
  a.m_alpha = ma; a.v_alpha = va; a.m_beta = mb; a.v_beta = vb; a.m_gamma = mg; a.v_gamma = vg;
  a.alpha_rw = alpha; a.beta_rw = beta;
  a.adam = AdamArgs{1, opt->adam_b1, opt->adam_b2, opt->adam_eps, ws.adam_tab.as<float>()};
  a.iters = opt->iters;
  a.P = pl.P;
  const int esz = bf16 ? 2 : 4;
  a.off_buf0 = 0;
  a.off_buf1 = kChainRows * pl.P * esz;
  a.off_sign = 2 * kChainRows * pl.P * esz;
  a.sign_ld = pl.sign_ld;
  const double M = c.M, it = opt->iters, nI = c.rp.n_I, N = c.rp.N, K = c.rp.K, nnz = c.nnz;
  const double alg = it * (28.0 * M * (nI + N + K) + 2.0 * c.B * nI);
  const double all = it * (M * (nI * 28.0 + elems * 2.0 * esz + nnz * 12.0 + N * 24.0 + K * 28.0) + 2.0 * c.B * nI);
  const int tiles = (c.M + kChainRows - 1) / kChainRows;
  hip_check(timed(c.st, std::string("chain.") + (bf16 ? "bf16" : "fp32"), Bytes{all, alg}, it * flops,
                  [&] { return launch_chain_opt(bf16, a, tiles, pl.lds, c.st); }),
            "fused chain");
}

// constants of the output layer for one call (c-hat = C W, C b_out)
void launch_constants(Call& c) {
  gcp_net* net = c.net;
  auto& ws = *c.ws;
  if (net->out_general) fail(GCP_EUNSUPPORTED, "grouped launches need the c-hat form of the output");
  const NodeH& on = net->nodes[net->out];
  hip_check(launch_out_const(c.C, c.S, on.size, on.bias.as<float>(), ws.cb.as<double>(), c.st), "out const");
  for (int eid : on.in_edges) {
    const EdgeH& E = *net->edges[eid];
    hip_check(launch_chat(c.C, c.S, on.size, E.Wraw.as<float>(), E.d_src, E.kind == GCP_EDGE_IDENTITY ? 2 : 0,
                          ws.chat.as<float>() + ws.chat_off[E.src], net->nodes[E.src].ld, c.st),
              "c-hat");
  }
}

// Whether a call's iterations can run as one persistent launch: every edge
// dense (the recorded schedule is GEMM, elementwise and multiplier steps over
// rows), the output in the c-hat form, Lemma A.1's pi*, a_hat stored.
bool persist_eligible(const Call& c) {
  if (c.net->out_general || c.rp.rho || c.M <= 0) return false;
  for (const auto& e : c.net->edges)
    if (e->kind != GCP_EDGE_DENSE) return false;
  for (uint8_t r : c.recompute)
    if (r) return false;
  return true;
}

// gcp_optimize and gcp_optimize_pi (rho non-null: explicit pi, its Adam
// moments after gamma's in adam_state)
void optimize_impl(const gcp_net* net_c, const double* x0, double eps, const double* C, int32_t S,
                   const gcp_splits* splits, const gcp_cuts* cuts, float* alpha, float* beta, float* gamma,
                   float* rho, float* adam_state, const gcp_opt* opt, int32_t mode, double* bound,
                   uint8_t* verified, void* stream) {
  gcp_net* net = const_cast<gcp_net*>(net_c);
  Call c{};
  prepare_call(c, net, x0, eps, C, S, splits, cuts, alpha, beta, gamma, stream);
  c.rp.rho = rho;
  const int bf16 = (mode & 0xff) == GCP_MODE_BF16;
  if ((mode & 0xff) != GCP_MODE_FP32 && !bf16) fail(GCP_EINVAL, "unknown mode");
  if (!opt || opt->iters < 0) fail(GCP_EINVAL, "bad optimiser settings");
  if (!adam_state) fail(GCP_EINVAL, "null adam_state");
  if (!bound) fail(GCP_EINVAL, "null bound output");
  if (mode & GCP_FLAG_VALIDATE) validate_params(c, alpha, beta, gamma);
  plan_ahat(c, mode);
  const ChainPlan chain = chain_plan(c, bf16);
  auto& ws = *c.ws;
  const size_t M = c.M, nI = c.rp.n_I, K = c.rp.K, N = c.rp.N;
  float* ma = adam_state;
  float* va = ma + M * nI;
  float* mb = va + M * nI;
  float* vb = mb + M * K;
  float* mg = vb + M * K;
  float* vg = mg + M * N;
  float* mr = rho ? vg + M * N : nullptr;
  float* vr = rho ? mr + M * nI : nullptr;
  AdamArgs adam{1, opt->adam_b1, opt->adam_b2, opt->adam_eps, ws.consts.as<float>()};
  // eager iterations read their constants from a table made once per call;
  // replayed graph iterations make them from the step counter (same bits)
  ws.adam_tab.ensure((size_t)std::max(opt->iters, 1) * 16);
  hip_check(launch_adam_table(ws.adam_tab.as<float>(), opt->iters, opt->lr_alpha, opt->lr_mult, opt->decay,
                              opt->adam_b1, opt->adam_b2, c.st),
            "adam table");
  if (N > 0) hip_check(launch_transpose(gamma, c.M, (int)N, (int)N, ws.gammaT.as<float>(), c.rp.mp, c.st), "transpose");
  size_partials(c, bf16, true, c.nnz > 0);
  {
    AdjPass prep{c, bf16, adam, nullptr, nullptr, alpha, beta, ma, va, mb, vb, nullptr, rho, mr, vr};
    prep.prepare();
  }
  auto iteration = [&](Call& cc, int t) {   // t < 0: the step counter gives t (graph replay)
    AdamArgs ad = adam;
    if (t < 0)
      hip_check(launch_adam_prepare(ws.step.as<int>(), 0, opt->lr_alpha, opt->lr_mult, opt->decay, opt->adam_b1,
                                    opt->adam_b2, ws.consts.as<float>(), cc.st),
                "adam prepare");
    else
      ad.consts = ws.adam_tab.as<float>() + 4 * t;
    BoundPass bp(cc, bf16, true, cc.nnz > 0, false);
    bp.run();
    AdjPass ap{cc, bf16, ad, nullptr, nullptr, alpha, beta, ma, va, mb, vb, nullptr, rho, mr, vr};
    ap.run();
    if (N > 0)
      hip_check(timed(cc.st, "gamma_adam", Bytes{(double)cc.M * (cc.nnz * 4.0 + N * 24.0), alg_mult(cc)}, 0.0, [&] {
                  return launch_gamma_update(cc.M, cc.rp.mp, (int)N, cc.cuts->row_ptr.as<int32_t>(),
                                             ws.contrib.as<float>(), cc.cuts->d.as<double>(), ws.gammaT.as<float>(),
                                             nullptr, mg, vg, ad, cc.st);
                }),
                "gamma update");
  };
  // the argument set a captured graph or a persistent plan was made for
  auto plan_key = [&]() {
    std::vector<uintptr_t> key = {(uintptr_t)x0, (uintptr_t)C, (uintptr_t)splits->id, (uintptr_t)(c.cuts ? c.cuts->id : 0),
                                  (uintptr_t)alpha, (uintptr_t)beta, (uintptr_t)gamma, (uintptr_t)rho,
                                  (uintptr_t)adam_state,
                                  (uintptr_t)S, (uintptr_t)bf16, (uintptr_t)c.M,
                                  (uintptr_t)std::hash<double>()(eps), (uintptr_t)ws.gen};
    for (uint8_t r : c.recompute) key.push_back(r);
    for (float v : {opt->lr_alpha, opt->lr_mult, opt->decay, opt->adam_b1, opt->adam_b2, opt->adam_eps}) {
      uint32_t b;
      std::memcpy(&b, &v, 4);
      key.push_back(b);
    }
    return key;
  };
  int done = 0;
  const int* persist_latch = nullptr;   // set when the iterations ran as persistent launches
  if (chain.ok && opt->iters > 0) {   // every iteration in one launch
    run_chain(c, bf16, chain, alpha, beta, ma, va, mb, vb, mg, vg, opt);
    done = opt->iters;
  }
  // GCP_FLAG_PERSIST: the iterations as one persistent dataflow launch over
  // the recorded schedule of one iteration (dense networks in the c-hat
  // form, Lemma A.1's pi*, a_hat stored); bit-identical to the eager loop
  if (done == 0 && opt->iters > 0 && (mode & GCP_FLAG_PERSIST) && persist_eligible(c)) {
    const AdamArgs tab{1, opt->adam_b1, opt->adam_b2, opt->adam_eps, ws.adam_tab.as<float>()};
    std::vector<uintptr_t> key = plan_key();
    key.push_back((uintptr_t)persist_xcd_sync(persist_queues()));
    if (ws.pplan && ws.pplan->key == key) {
      launch_constants(c);
      run_persist(*ws.pplan, bf16, opt->iters, 0, tab, c.st);
      done = opt->iters;
      persist_latch = ws.pplan->latch.as<int>();
    } else {
      iteration(c, 0);   // tunes the per-layer tiles the schedule records, sizes buffers
      done = 1;
      c.consts_done = true;
      key = plan_key();
      key.push_back((uintptr_t)persist_xcd_sync(persist_queues()));
      Recorder rec;
      Call cr = c;
      cr.rec = &rec;
      BoundPass bp(cr, bf16, true, cr.nnz > 0, false);
      bp.run();
      rec.in_adj = true;
      AdjPass ap{cr, bf16, adam, nullptr, nullptr, alpha, beta, ma, va, mb, vb};
      ap.run();
      std::vector<PersistInst> in{PersistInst{&rec, N > 0,
                                              GammaJob{c.M, c.rp.mp, (int)N, N > 0 ? c.cuts->row_ptr.as<int32_t>() : nullptr,
                                                       ws.contrib.as<float>(), N > 0 ? c.cuts->d.as<double>() : nullptr,
                                                       ws.gammaT.as<float>(), mg, vg},
                                              c.M}};
      auto plan = std::make_unique<PersistPlan>();
      plan->key = key;
      if (build_persist(*plan, in, bf16)) {
        ws.pplan = std::move(plan);
        run_persist(*ws.pplan, bf16, opt->iters - done, done, tab, c.st);
        done = opt->iters;
        persist_latch = ws.pplan->latch.as<int>();
      }
    }
  }
  if (done == 0 && opt->iters > 0) {   // the first iteration runs eagerly (tunes tiles, sizes buffers)
    iteration(c, 0);
    done = 1;
    c.consts_done = !net->out_general || !bf16;
  }
  if (opt->use_graph && opt->iters > 1 && done < opt->iters) {
    std::vector<uintptr_t> key = plan_key();
    if (!ws.gstream) hip_check(hipStreamCreateWithFlags(&ws.gstream, hipStreamNonBlocking), "hipStreamCreate");
    // the replays continue the count from the eager iterations done so far
    hip_check(launch_adam_prepare(ws.step.as<int>(), done + 1, 0, 0, 0, 0, 0, nullptr, c.st), "adam step");
    hipEvent_t ev;
    hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
    hip_check(hipEventRecord(ev, c.st), "hipEventRecord");
    hip_check(hipStreamWaitEvent(ws.gstream, ev, 0), "hipStreamWaitEvent");
    if (!ws.gexec || ws.gkey != key) {
      if (ws.gexec) { (void)hipGraphExecDestroy(ws.gexec); ws.gexec = nullptr; }
      Call cg = c;
      cg.st = ws.gstream;
      hipGraph_t graph;
      hip_check(hipStreamBeginCapture(ws.gstream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      try {
        iteration(cg, -1);
      } catch (...) {
        hipGraph_t g2;
        (void)hipStreamEndCapture(ws.gstream, &g2);
        throw;
      }
      hip_check(hipStreamEndCapture(ws.gstream, &graph), "hipStreamEndCapture");
      hipError_t ie = hipGraphInstantiate(&ws.gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      hip_check(ie, "hipGraphInstantiate");
      ws.gkey = key;
    }
    for (; done < opt->iters; ++done) hip_check(hipGraphLaunch(ws.gexec, ws.gstream), "hipGraphLaunch");
    hip_check(hipEventRecord(ev, ws.gstream), "hipEventRecord");
    hip_check(hipStreamWaitEvent(c.st, ev, 0), "hipStreamWaitEvent");
    (void)hipEventDestroy(ev);
  }
  for (; done < opt->iters; ++done) iteration(c, done);
  if (N > 0) hip_check(launch_transpose(ws.gammaT.as<float>(), (int)N, c.M, c.rp.mp, gamma, (int)N, c.st), "transpose");
  // certifying pass: fp32 GEMMs, fp64 reductions, margin check
  c.outward = (mode & GCP_FLAG_OUTWARD) != 0;
  bound_pass(c, 0, false, false, bound, verified);
  if (persist_latch)   // a persistent launch that aborted leaves -inf bounds
    hip_check(launch_persist_guard(persist_latch, bound, verified, c.M, c.st), "persist guard");
}

}  // namespace

extern "C" int gcp_bound(const gcp_net* net, const double* x0, double eps, const double* C, int32_t S,
                         const gcp_splits* splits, const gcp_cuts* cuts, const float* alpha, const float* beta,
                         const float* gamma, int32_t mode, double* bound, uint8_t* verified, float* d_alpha,
                         float* d_beta, float* d_gamma, void* stream) {
  GCP_TRY
  bound_impl(net, x0, eps, C, S, splits, cuts, alpha, beta, gamma, nullptr, mode, bound, verified, d_alpha, d_beta,
             d_gamma, nullptr, stream);
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}

extern "C" int gcp_bound_noalloc(const gcp_net* net, const double* x0, double eps, const double* C, int32_t S,
                                 const gcp_splits* splits, const gcp_cuts* cuts, const float* alpha, const float* beta,
                                 const float* gamma, int32_t mode, double* bound, uint8_t* verified, float* d_alpha,
                                 float* d_beta, float* d_gamma, void* stream) {
  GCP_TRY
  NoAllocScope scope;
  bound_impl(net, x0, eps, C, S, splits, cuts, alpha, beta, gamma, nullptr, mode, bound, verified, d_alpha, d_beta,
             d_gamma, nullptr, stream, true);
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}

extern "C" int gcp_bound_pi(const gcp_net* net, const double* x0, double eps, const double* C, int32_t S,
                            const gcp_splits* splits, const gcp_cuts* cuts, const float* alpha, const float* beta,
                            const float* gamma, const float* rho, int32_t mode, double* bound, uint8_t* verified,
                            float* d_alpha, float* d_beta, float* d_gamma, float* d_rho, void* stream) {
  GCP_TRY
  if (net && net->n_I > 0 && !rho) fail(GCP_EINVAL, "null rho");
  bound_impl(net, x0, eps, C, S, splits, cuts, alpha, beta, gamma, rho, mode, bound, verified, d_alpha, d_beta,
             d_gamma, d_rho, stream);
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}

extern "C" int gcp_optimize(const gcp_net* net, const double* x0, double eps, const double* C, int32_t S,
                            const gcp_splits* splits, const gcp_cuts* cuts, float* alpha, float* beta,
                            float* gamma, float* adam_state, const gcp_opt* opt, int32_t mode, double* bound,
                            uint8_t* verified, void* stream) {
  GCP_TRY
  optimize_impl(net, x0, eps, C, S, splits, cuts, alpha, beta, gamma, nullptr, adam_state, opt, mode, bound,
                verified, stream);
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}

extern "C" int gcp_optimize_pi(const gcp_net* net, const double* x0, double eps, const double* C, int32_t S,
                               const gcp_splits* splits, const gcp_cuts* cuts, float* alpha, float* beta,
                               float* gamma, float* rho, float* adam_state, const gcp_opt* opt, int32_t mode,
                               double* bound, uint8_t* verified, void* stream) {
  GCP_TRY
  if (net && net->n_I > 0 && !rho) fail(GCP_EINVAL, "null rho");
  optimize_impl(net, x0, eps, C, S, splits, cuts, alpha, beta, gamma, rho, adam_state, opt, mode, bound, verified,
                stream);
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}

// gcp_prepare: one gradient bound pass in `mode`, one fp32 bound pass and
// an optimisation of `iters` iterations on zero inputs of the given shapes
// size every workspace buffer and tune every tile shape the calls of these
// shapes launch; the scratch inputs are freed at the end.
extern "C" int gcp_prepare(const gcp_net* net, int32_t S, const gcp_splits* splits, const gcp_cuts* cuts,
                           int32_t iters, int32_t mode, void* stream) {
  GCP_TRY
  if (!net || !splits) fail(GCP_EINVAL, "null net or splits");
  if (S <= 0 || iters < 0) fail(GCP_EINVAL, "need S >= 1 and iters >= 0");
  if (mode & GCP_FLAG_VALIDATE) fail(GCP_EINVAL, "GCP_FLAG_VALIDATE is a per-call check");
  const int bf16 = (mode & 0xff) == GCP_MODE_BF16;
  if ((mode & 0xff) != GCP_MODE_FP32 && !bf16) fail(GCP_EINVAL, "unknown mode");
  hipStream_t st = (hipStream_t)stream;
  const size_t M = (size_t)splits->B * S, nI = net->n_I, K = splits->K, N = cuts ? cuts->N : 0;
  DBuf x0, C, a, b, g, da, db, dg, state, bound, ver;
  x0.alloc((size_t)std::max(net->in_size, 1) * 8);
  C.alloc((size_t)S * net->nodes[net->out].size * 8);
  a.alloc(std::max<size_t>(M * nI, 1) * 4);
  b.alloc(std::max<size_t>(M * K, 1) * 4);
  g.alloc(std::max<size_t>(M * N, 1) * 4);
  da.alloc(std::max<size_t>(M * nI, 1) * 4);
  db.alloc(std::max<size_t>(M * K, 1) * 4);
  dg.alloc(std::max<size_t>(M * N, 1) * 4);
  state.alloc(std::max<size_t>(2 * M * (nI + K + N), 1) * 4);
  bound.alloc(M * 8);
  ver.alloc(M);
  float* pa = a.as<float>(); float* pb = K ? b.as<float>() : nullptr; float* pg = N ? g.as<float>() : nullptr;
  bound_impl(net, x0.as<double>(), 0.0, C.as<double>(), S, splits, cuts, pa, pb, pg, nullptr, mode, bound.as<double>(),
             ver.as<uint8_t>(), da.as<float>(), K ? db.as<float>() : nullptr, N ? dg.as<float>() : nullptr, nullptr, st);
  bound_impl(net, x0.as<double>(), 0.0, C.as<double>(), S, splits, cuts, pa, pb, pg, nullptr,
             GCP_MODE_FP32 | GCP_FLAG_OUTWARD, bound.as<double>(), ver.as<uint8_t>(), nullptr, nullptr, nullptr, nullptr,
             st);   // sizes the outward-rounding weights too
  gcp_opt o{std::max(iters, 1), 0.1f, 0.02f, 0.9f, 0.9f, 0.999f, 1e-8f, 0};
  optimize_impl(net, x0.as<double>(), 0.0, C.as<double>(), S, splits, cuts, pa, pb, pg, nullptr, state.as<float>(), &o,
                mode, bound.as<double>(), ver.as<uint8_t>(), st);
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}

extern "C" int gcp_profile_enable(int32_t on) {
  GCP_TRY
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  if (on) {
    P.flush();
    P.agg.clear();
  }
  P.on = on != 0;
  return GCP_OK;
  GCP_CATCH
}

extern "C" int gcp_profile_read(int32_t idx, char* name, int32_t name_len, int64_t* launches, double* total_ms,
                                double* bytes, double* alg_bytes, double* flops) {
  GCP_TRY
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  P.flush();
  if (idx < 0 || idx >= (int)P.names.size()) fail(GCP_EINVAL, "no such profile class");
  Profiler::Agg a = idx < (int)P.agg.size() ? P.agg[idx] : Profiler::Agg{};
  if (name && name_len > 0) {
    std::snprintf(name, name_len, "%s", P.names[idx].c_str());
  }
  if (launches) *launches = a.n;
  if (total_ms) *total_ms = a.ms;
  if (bytes) *bytes = a.bytes;
  if (alg_bytes) *alg_bytes = a.alg;
  if (flops) *flops = a.flops;
  return GCP_OK;
  GCP_CATCH
}

// ====================================================================== batch

namespace {


// Grouped launches of one iteration, tables in one device buffer.
struct Group {
  int type, bf16, cfg, kind, sign;
  int np, total;
  double bytes, alg, flops;               // summed over the group's problems
  size_t off_args, off_epi, off_prefix;   // byte offsets into the plan buffer
};
struct BatchPlan {
  std::vector<uintptr_t> key;
  DBuf buf;
  std::vector<Group> groups;              // in launch order
  size_t off_gjobs = 0, off_gprefix = 0;
  int g_np = 0, g_total = 0;
  double g_bytes = 0.0, g_alg = 0.0;      // bytes (both models) of the grouped gamma update
  hipGraphExec_t gexec = nullptr;
  hipStream_t gstream = nullptr;
  // GCP_FLAG_PERSIST: every instance's iterations in one persistent launch
  std::unique_ptr<PersistPlan> persist;
  DBuf adam_tab;                          // Adam constants of every iteration, [iters][4]
  hipGraphExec_t pexec = nullptr;         // the captured persistent launch (use_graph)
  int pexec_iters = -1;
  ~BatchPlan() {
    if (pexec) (void)hipGraphExecDestroy(pexec);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (gstream) (void)hipStreamDestroy(gstream);
  }
};
std::mutex g_batch_mu;
// One cached plan (the last argument set).  Deliberately never destroyed at
// process exit: its graph and buffers must not be released after the HIP
// runtime has shut down; a new argument set replaces it.
BatchPlan* g_batch = nullptr;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

void build_plan(BatchPlan& plan, std::vector<Recorder>& recs, std::vector<GammaJob>& gj) {
  // waves: the w-th recorded launch of every instance, bound part then adjoint
  // part; within a wave, one group per kernel instantiation
  std::vector<std::vector<const Rec*>> waves;
  size_t maxb = 0, maxa = 0;
  for (auto& r : recs) { maxb = std::max(maxb, r.bound.size()); maxa = std::max(maxa, r.adj.size()); }
  for (size_t w = 0; w < maxb; ++w) {
    waves.emplace_back();
    for (auto& r : recs) if (w < r.bound.size()) waves.back().push_back(&r.bound[w]);
  }
  for (size_t w = 0; w < maxa; ++w) {
    waves.emplace_back();
    for (auto& r : recs) if (w < r.adj.size()) waves.back().push_back(&r.adj[w]);
  }
  std::vector<unsigned char> host;
  auto put = [&](const void* p, size_t n) {
    size_t off = align_up(host.size(), 16);
    host.resize(off + n);
    std::memcpy(host.data() + off, p, n);
    return off;
  };
  for (auto& wave : waves) {
    std::map<std::tuple<int, int, int, int, int>, std::vector<const Rec*>> by;
    for (const Rec* r : wave) by[std::make_tuple(r->type, r->bf16, r->cfg, r->kind, r->sign)].push_back(r);
    for (auto& kv : by) {
      const auto& v = kv.second;
      Group G{};
      G.type = v[0]->type; G.bf16 = v[0]->bf16; G.cfg = v[0]->cfg; G.kind = v[0]->kind; G.sign = v[0]->sign;
      G.np = (int)v.size();
      std::vector<int> prefix(1, 0);
      for (const Rec* r : v) {
        prefix.push_back(prefix.back() + r->tiles);
        G.bytes += r->bytes;
        G.alg += r->alg;
        G.flops += r->flops;
      }
      G.total = prefix.back();
      if (G.type == 0) {
        std::vector<GemmArgs> ga;
        for (const Rec* r : v) ga.push_back(r->g);
        G.off_args = put(ga.data(), ga.size() * sizeof(GemmArgs));
        size_t esz = G.kind == EPI_BOUND ? sizeof(BoundEpiArgs)
                   : G.kind == EPI_CONC ? sizeof(ConcEpiArgs)
                   : G.kind == EPI_ADJ ? sizeof(AdjEpiArgs) : sizeof(StoreEpiArgs);
        std::vector<unsigned char> eb(esz * v.size());
        for (size_t i = 0; i < v.size(); ++i) std::memcpy(eb.data() + i * esz, v[i]->epi, esz);
        G.off_epi = put(eb.data(), eb.size());
      } else {
        std::vector<ElemBoundJob> jb;
        for (const Rec* r : v) jb.push_back(r->ej);
        G.off_args = put(jb.data(), jb.size() * sizeof(ElemBoundJob));
      }
      G.off_prefix = put(prefix.data(), prefix.size() * sizeof(int));
      plan.groups.push_back(G);
    }
  }
  if (!gj.empty()) {
    std::vector<int> prefix(1, 0);
    for (auto& j : gj) prefix.push_back(prefix.back() + j.N * ((j.M + 255) / 256));
    plan.off_gjobs = put(gj.data(), gj.size() * sizeof(GammaJob));
    plan.off_gprefix = put(prefix.data(), prefix.size() * sizeof(int));
    plan.g_np = (int)gj.size();
    plan.g_total = prefix.back();
  }
  plan.buf.alloc(std::max<size_t>(host.size(), 16));
  hip_check(hipMemcpy(plan.buf.p, host.data(), host.size(), hipMemcpyHostToDevice), "hipMemcpy");
  hip_check(hipStreamSynchronize(nullptr), "hipStreamSynchronize");   // ordered before any stream's launches
}

void run_grouped_iteration(BatchPlan& plan, int* step, float* consts, const gcp_opt* opt, AdamArgs adam,
                           hipStream_t st) {
  unsigned char* b = (unsigned char*)plan.buf.p;
  hip_check(launch_adam_prepare(step, 0, opt->lr_alpha, opt->lr_mult, opt->decay, opt->adam_b1, opt->adam_b2, consts,
                                st),
            "adam prepare");
  static const char* grp_names[] = {"store_grp", "bound_grp", "conc_grp", "adj_grp"};   // by EpiKind
  for (const Group& G : plan.groups) {
    if (G.type == 0)
      hip_check(timed(st, cls_name(grp_names[G.kind], G.bf16, G.sign, G.cfg), Bytes{G.bytes, G.alg}, G.flops, [&] {
                  return launch_gemm_grouped(G.bf16, G.cfg, (EpiKind)G.kind, G.sign,
                                             (const GemmArgs*)(b + G.off_args), b + G.off_epi,
                                             (const int*)(b + G.off_prefix), G.np, G.total, st);
                }),
                "grouped gemm");
    else
      hip_check(timed(st, cls_name("bound_elem_grp", G.bf16, 0, -1), Bytes{G.bytes, G.alg}, 0.0, [&] {
                  return launch_bound_elementwise_grouped(G.bf16, (const ElemBoundJob*)(b + G.off_args),
                                                          (const int*)(b + G.off_prefix), G.np, G.total, st);
                }),
                "grouped elementwise");
  }
  if (plan.g_np)
    hip_check(timed(st, "gamma_adam_grp", Bytes{plan.g_bytes, plan.g_alg}, 0.0, [&] {
                return launch_gamma_grouped((const GammaJob*)(b + plan.off_gjobs), (const int*)(b + plan.off_gprefix),
                                            plan.g_np, plan.g_total, adam, st);
              }),
              "grouped gamma");
}

}  // namespace

namespace {
// An instance whose widest layer holds at least this many (row, neuron)
// elements fills the chip with its own launches (about four 32x32 tiles per
// compute unit); grouping it with others only mixes more weights in the L2.
// GCP_BATCH_ALONE_WORK overrides the threshold.
long batch_alone_work() {
  const char* e = std::getenv("GCP_BATCH_ALONE_WORK");
  return e && *e ? std::atol(e) : (1L << 20);
}
// Internal streams (default priority, one set per device, kept for the life
// of the process) on which the large instances of a batch run concurrently,
// joined to the caller's stream by events.  GCP_BATCH_STREAMS sets how many
// (default 2; 1 runs them one after the other on the caller's stream).
std::mutex g_side_mu;
std::map<int, std::vector<hipStream_t>>* g_side = nullptr;
std::vector<hipStream_t> side_streams(int n) {
  int dev;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_side_mu);
  if (!g_side) g_side = new std::map<int, std::vector<hipStream_t>>();
  auto& v = (*g_side)[dev];
  while ((int)v.size() < n) {
    hipStream_t s;
    hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
    v.push_back(s);
  }
  return std::vector<hipStream_t>(v.begin(), v.begin() + n);
}
int batch_streams() {
  const char* e = std::getenv("GCP_BATCH_STREAMS");
  const int n = e && *e ? std::atoi(e) : 2;
  return std::max(1, std::min(n, 8));
}
long instance_work(const gcp_batch_item& it) {
  if (!it.net || !it.splits) return 0;
  int width = 0;
  for (const NodeH& nd : it.net->nodes) width = std::max(width, nd.ld);
  return (long)it.splits->B * it.S * width;
}
// Grouped launches replay a recorded schedule of dense GEMMs with fused
// epilogues: conv and identity edges and a materialised output Lambda have no
// recorded form.  Returns what stands in the way, or null.
const char* grouped_unsupported(const gcp_net* net) {
  for (const auto& e : net->edges) {
    if (e->kind == GCP_EDGE_CONV) return "conv";
    if (e->kind == GCP_EDGE_IDENTITY) return "identity";
  }
  return net->out_general ? "output Lambda not in the c-hat form" : nullptr;
}
}  // namespace

extern "C" int gcp_optimize_batch(int32_t n_all, const gcp_batch_item* items_all, const gcp_opt* opt, int32_t mode,
                                  void* stream) {
  GCP_TRY
  if (n_all <= 0 || !items_all) fail(GCP_EINVAL, "empty batch");
  if (!opt || opt->iters < 0) fail(GCP_EINVAL, "bad optimiser settings");
  const int bf16 = (mode & 0xff) == GCP_MODE_BF16;
  if ((mode & 0xff) != GCP_MODE_FP32 && !bf16) fail(GCP_EINVAL, "unknown mode");
  hipStream_t st = (hipStream_t)stream;
  for (int i = 0; i < n_all; ++i) {
    if (!items_all[i].net || !items_all[i].splits) fail(GCP_EINVAL, "null net or splits handle in a batch item");
    if (!items_all[i].adam_state || !items_all[i].bound) fail(GCP_EINVAL, "null adam_state or bound");
    for (int k = 0; k < i; ++k)
      if (items_all[k].net == items_all[i].net) fail(GCP_EINVAL, "each batch item needs its own net handle (workspace)");
  }
  // large instances: their own launches (the same kernels and tiles as
  // gcp_optimize), spread over a few streams by longest-first assignment
  // with GCP_FLAG_PERSIST every instance shares the one persistent launch
  // (measured: keeping the large instances on their own launches beside it
  // is slower still, since the persistent grid holds every compute unit
  // until its queues drain)
  const long alone = (mode & GCP_FLAG_PERSIST) ? std::numeric_limits<long>::max() : batch_alone_work();
  std::vector<gcp_batch_item> grouped;
  std::vector<std::pair<long, int>> big;
  for (int i = 0; i < n_all; ++i) {
    const long w = instance_work(items_all[i]);
    if (w < alone) grouped.push_back(items_all[i]);
    else big.push_back({w, i});
  }
  // every item's arguments are checked (and its workspace sized) before
  // anything is launched
  for (const gcp_batch_item& it : grouped) {
    if (const char* why = grouped_unsupported(it.net))
      fail(GCP_EUNSUPPORTED, std::string("batched optimisation supports dense edges only (") + why + ")");
  }
  for (const auto& b : big) {
    const gcp_batch_item& it = items_all[b.second];
    Call chk{};
    prepare_call(chk, const_cast<gcp_net*>(it.net), it.x0, it.eps, it.C, it.S, it.splits, it.cuts, it.alpha,
                 it.beta, it.gamma, stream);
  }
  const int n = (int)grouped.size();
  const gcp_batch_item* items = grouped.data();
  std::vector<Call> calls(n);
  for (int i = 0; i < n; ++i) {
    const gcp_batch_item& it = items[i];
    prepare_call(calls[i], const_cast<gcp_net*>(it.net), it.x0, it.eps, it.C, it.S, it.splits, it.cuts, it.alpha,
                 it.beta, it.gamma, stream);
    if (mode & GCP_FLAG_VALIDATE) validate_params(calls[i], it.alpha, it.beta, it.gamma);
    plan_ahat(calls[i], GCP_FLAG_STORE_AHAT);   // grouped launches replay a stored schedule
  }
  if (!big.empty()) {
    const int ns = std::min<int>(batch_streams(), (int)big.size());
    std::vector<hipStream_t> ss = ns > 1 ? side_streams(ns) : std::vector<hipStream_t>{st};
    std::sort(big.begin(), big.end(), [](const std::pair<long, int>& a, const std::pair<long, int>& b) {
      return a.first > b.first || (a.first == b.first && a.second < b.second);
    });
    std::vector<double> load(ns, 0.0);
    hipEvent_t start = nullptr;
    if (ns > 1) {
      hip_check(hipEventCreateWithFlags(&start, hipEventDisableTiming), "hipEventCreate");
      hip_check(hipEventRecord(start, st), "hipEventRecord");
      for (hipStream_t s : ss) hip_check(hipStreamWaitEvent(s, start, 0), "hipStreamWaitEvent");
    }
    int rc = GCP_OK;
    for (const auto& b : big) {
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[k] += (double)b.first;
      const gcp_batch_item& it = items_all[b.second];
      rc = gcp_optimize(it.net, it.x0, it.eps, it.C, it.S, it.splits, it.cuts, it.alpha, it.beta, it.gamma,
                        it.adam_state, opt, mode, it.bound, it.verified, ss[k]);
      if (rc != GCP_OK) break;
    }
    if (ns > 1) {   // the caller's stream waits for every side stream
      for (hipStream_t s : ss) {
        hipEvent_t done;
        hip_check(hipEventCreateWithFlags(&done, hipEventDisableTiming), "hipEventCreate");
        hip_check(hipEventRecord(done, s), "hipEventRecord");
        hip_check(hipStreamWaitEvent(st, done, 0), "hipStreamWaitEvent");
        (void)hipEventDestroy(done);
      }
      (void)hipEventDestroy(start);
    }
    if (rc != GCP_OK) return rc;
  }
  if (grouped.empty()) {
    g_err.clear();
    return GCP_OK;
  }
  std::lock_guard<std::mutex> lk(g_batch_mu);
  // shared Adam counter and constants: the first instance's workspace
  auto& ws0 = calls[0].net->ws;
  AdamArgs adam{1, opt->adam_b1, opt->adam_b2, opt->adam_eps, ws0.consts.as<float>()};
  struct Moments { float *ma, *va, *mb, *vb, *mg, *vg; };
  std::vector<Moments> mom(n);
  const bool persist = (mode & GCP_FLAG_PERSIST) != 0;
  std::vector<uintptr_t> key = {(uintptr_t)n, (uintptr_t)bf16, (uintptr_t)persist};
  // the captured graph and the recorded epilogue arguments hold these
  for (float v : {opt->lr_alpha, opt->lr_mult, opt->decay, opt->adam_b1, opt->adam_b2, opt->adam_eps}) {
    uint32_t b;
    std::memcpy(&b, &v, 4);
    key.push_back(b);
  }
  for (int i = 0; i < n; ++i) {
    Call& c = calls[i];
    const gcp_batch_item& it = items[i];
    const size_t M = c.M, nI = c.rp.n_I, K = c.rp.K, N = c.rp.N;
    Moments& m = mom[i];
    m.ma = it.adam_state; m.va = m.ma + M * nI; m.mb = m.va + M * nI; m.vb = m.mb + M * K;
    m.mg = m.vb + M * K; m.vg = m.mg + M * N;
    if (N > 0) hip_check(launch_transpose(it.gamma, c.M, (int)N, (int)N, c.net->ws.gammaT.as<float>(), c.rp.mp, st),
                         "transpose");
    size_partials(c, bf16, true, c.nnz > 0);
    launch_constants(c);
    AdjPass prep{c, bf16, adam, nullptr, nullptr, it.alpha, it.beta, m.ma, m.va, m.mb, m.vb};
    prep.prepare();
    for (uintptr_t v : {(uintptr_t)it.net, (uintptr_t)it.x0, (uintptr_t)it.C, (uintptr_t)it.S,
                        (uintptr_t)it.splits->id, (uintptr_t)(c.cuts ? c.cuts->id : 0), (uintptr_t)it.alpha,
                        (uintptr_t)it.beta,
                        (uintptr_t)it.gamma, (uintptr_t)it.adam_state, (uintptr_t)std::hash<double>()(it.eps),
                        (uintptr_t)c.net->ws.gen})
      key.push_back(v);
  }
  hip_check(launch_adam_prepare(ws0.step.as<int>(), 1, 0, 0, 0, 0, 0, nullptr, st), "adam reset");
  auto eager_iteration = [&]() {
    hip_check(launch_adam_prepare(ws0.step.as<int>(), 0, opt->lr_alpha, opt->lr_mult, opt->decay, opt->adam_b1,
                                  opt->adam_b2, ws0.consts.as<float>(), st),
              "adam prepare");
    for (int i = 0; i < n; ++i) {
      Call& c = calls[i];
      BoundPass bp(c, bf16, true, c.nnz > 0, false);
      bp.run();
      AdjPass ap{c, bf16, adam, nullptr, nullptr, items[i].alpha, items[i].beta, mom[i].ma, mom[i].va, mom[i].mb,
                 mom[i].vb};
      ap.run();
      if (c.rp.N > 0)
        hip_check(launch_gamma_update(c.M, c.rp.mp, c.rp.N, c.cuts->row_ptr.as<int32_t>(),
                                      c.net->ws.contrib.as<float>(), c.cuts->d.as<double>(),
                                      c.net->ws.gammaT.as<float>(), nullptr, mom[i].mg, mom[i].vg, adam, st),
                  "gamma update");
    }
  };
  int done = 0;
  const bool cached = g_batch && g_batch->key == key;
  if (!cached && opt->iters > 0) {
    eager_iteration();      // tunes tiles and sizes buffers of every instance
    done = 1;
    auto plan = std::make_unique<BatchPlan>();
    plan->key = key;
    std::vector<Recorder> recs(n);
    std::vector<GammaJob> gj;
    std::vector<PersistInst> pin;
    for (int i = 0; i < n; ++i) {
      Call c = calls[i];
      c.rec = &recs[i];
      BoundPass bp(c, bf16, true, c.nnz > 0, false);
      bp.run();
      recs[i].in_adj = true;
      AdjPass ap{c, bf16, adam, nullptr, nullptr, items[i].alpha, items[i].beta, mom[i].ma, mom[i].va, mom[i].mb,
                 mom[i].vb};
      ap.run();
      GammaJob g1{c.M, c.rp.mp, c.rp.N, c.rp.N > 0 ? c.cuts->row_ptr.as<int32_t>() : nullptr,
                  c.net->ws.contrib.as<float>(), c.rp.N > 0 ? c.cuts->d.as<double>() : nullptr,
                  c.net->ws.gammaT.as<float>(), mom[i].mg, mom[i].vg};
      if (c.rp.N > 0) {
        plan->g_bytes += (double)c.M * (c.nnz * 4.0 + c.rp.N * 24.0);
        plan->g_alg += alg_mult(c);
        gj.push_back(g1);
      }
      pin.push_back(PersistInst{&recs[i], c.rp.N > 0, g1, c.M});
    }
    build_plan(*plan, recs, gj);
    if (persist) {
      auto pp = std::make_unique<PersistPlan>();
      if (build_persist(*pp, pin, bf16)) plan->persist = std::move(pp);
    }
    delete g_batch;
    g_batch = plan.release();
  }
  BatchPlan& plan = *g_batch;
  const bool ran_persist = plan.persist && done < opt->iters;
  if (ran_persist) {
    // the remaining iterations of every instance in one persistent launch
    // (with use_graph: captured once per iteration count, replayed)
    plan.adam_tab.ensure((size_t)std::max(opt->iters, 1) * 16);
    const AdamArgs tab{1, opt->adam_b1, opt->adam_b2, opt->adam_eps, plan.adam_tab.as<float>()};
    const int todo = opt->iters - done, first = done;
    if (opt->use_graph) {
      if (!plan.gstream) hip_check(hipStreamCreateWithFlags(&plan.gstream, hipStreamNonBlocking), "hipStreamCreate");
      if (!plan.pexec || plan.pexec_iters != opt->iters * 1000 + first) {
        if (plan.pexec) { (void)hipGraphExecDestroy(plan.pexec); plan.pexec = nullptr; }
        hipGraph_t graph;
        hip_check(hipStreamBeginCapture(plan.gstream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        try {
          hip_check(launch_adam_table(plan.adam_tab.as<float>(), opt->iters, opt->lr_alpha, opt->lr_mult, opt->decay,
                                      opt->adam_b1, opt->adam_b2, plan.gstream),
                    "adam table");
          run_persist(*plan.persist, bf16, todo, first, tab, plan.gstream);
        } catch (...) {
          hipGraph_t g2;
          (void)hipStreamEndCapture(plan.gstream, &g2);
          throw;
        }
        hip_check(hipStreamEndCapture(plan.gstream, &graph), "hipStreamEndCapture");
        hipError_t ie = hipGraphInstantiate(&plan.pexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        hip_check(ie, "hipGraphInstantiate");
        plan.pexec_iters = opt->iters * 1000 + first;
      }
      hipEvent_t ev;
      hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
      hip_check(hipEventRecord(ev, st), "hipEventRecord");
      hip_check(hipStreamWaitEvent(plan.gstream, ev, 0), "hipStreamWaitEvent");
      hip_check(hipGraphLaunch(plan.pexec, plan.gstream), "hipGraphLaunch");
      hip_check(hipEventRecord(ev, plan.gstream), "hipEventRecord");
      hip_check(hipStreamWaitEvent(st, ev, 0), "hipStreamWaitEvent");
      (void)hipEventDestroy(ev);
    } else {
      hip_check(launch_adam_table(plan.adam_tab.as<float>(), opt->iters, opt->lr_alpha, opt->lr_mult, opt->decay,
                                  opt->adam_b1, opt->adam_b2, st),
                "adam table");
      run_persist(*plan.persist, bf16, todo, first, tab, st);
    }
    done = opt->iters;
  }
  if (opt->use_graph && opt->iters > 1 && done < opt->iters) {
    if (!plan.gstream) hip_check(hipStreamCreateWithFlags(&plan.gstream, hipStreamNonBlocking), "hipStreamCreate");
    hipEvent_t ev;
    hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
    hip_check(hipEventRecord(ev, st), "hipEventRecord");
    hip_check(hipStreamWaitEvent(plan.gstream, ev, 0), "hipStreamWaitEvent");
    if (!plan.gexec) {
      hipGraph_t graph;
      hip_check(hipStreamBeginCapture(plan.gstream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      try {
        run_grouped_iteration(plan, ws0.step.as<int>(), ws0.consts.as<float>(), opt, adam, plan.gstream);
      } catch (...) {
        hipGraph_t g2;
        (void)hipStreamEndCapture(plan.gstream, &g2);
        throw;
      }
      hip_check(hipStreamEndCapture(plan.gstream, &graph), "hipStreamEndCapture");
      hipError_t ie = hipGraphInstantiate(&plan.gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      hip_check(ie, "hipGraphInstantiate");
    }
    for (; done < opt->iters; ++done) hip_check(hipGraphLaunch(plan.gexec, plan.gstream), "hipGraphLaunch");
    hip_check(hipEventRecord(ev, plan.gstream), "hipEventRecord");
    hip_check(hipStreamWaitEvent(st, ev, 0), "hipStreamWaitEvent");
    (void)hipEventDestroy(ev);
  }
  for (; done < opt->iters; ++done)
    run_grouped_iteration(plan, ws0.step.as<int>(), ws0.consts.as<float>(), opt, adam, st);
  // certifying pass per instance, then gamma back to the caller's layout
  for (int i = 0; i < n; ++i) {
    Call& c = calls[i];
    c.outward = (mode & GCP_FLAG_OUTWARD) != 0;
    bound_pass(c, 0, false, false, items[i].bound, items[i].verified);
    if (ran_persist)   // a persistent launch that aborted leaves -inf bounds
      hip_check(launch_persist_guard(plan.persist->latch.as<int>(), items[i].bound, items[i].verified, c.M, st),
                "persist guard");
    if (c.rp.N > 0)
      hip_check(launch_transpose(c.net->ws.gammaT.as<float>(), c.rp.N, c.M, c.rp.mp, items[i].gamma, c.rp.N, st),
                "transpose");
  }
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}

// ====================================================================== intermediate bounds

namespace {
// Owning wrappers for the handles used by gcp_crown_bounds.
struct NetGuard { gcp_net* p = nullptr; ~NetGuard() { if (p) gcp_net_destroy(p); } };
struct SplitsGuard { gcp_splits* p = nullptr; ~SplitsGuard() { if (p) gcp_splits_destroy(p); } };
}  // namespace

extern "C" int gcp_crown_bounds(const gcp_net_desc* desc, const double* x0, double eps, double* const* lower,
                                double* const* upper, int32_t mode, void* stream) {
  return gcp_crown_bounds_domain(desc, x0, eps, 0, nullptr, nullptr, nullptr, lower, upper, mode, stream);
}

extern "C" int gcp_crown_bounds_domain(const gcp_net_desc* desc, const double* x0, double eps, int32_t n_split,
                                       const int32_t* split_node, const int32_t* split_neuron,
                                       const int8_t* split_sign, double* const* lower, double* const* upper,
                                       int32_t mode, void* stream) {
  GCP_TRY
  if (!desc || !desc->nodes || desc->n_nodes < 2) fail(GCP_EINVAL, "bad network description");
  if (!x0) fail(GCP_EINVAL, "null x0");
  if (!lower || !upper) fail(GCP_EINVAL, "null bound outputs");
  if ((mode & 0xff) != GCP_MODE_FP32 && (mode & 0xff) != GCP_MODE_BF16) fail(GCP_EINVAL, "unknown mode");
  const int out = desc->n_nodes - 1;
  hipStream_t st = (hipStream_t)stream;
  // the domain's splits, checked: node of a ReLU layer, neuron in range, sign
  // +-1, no neuron twice
  if (n_split < 0 || n_split > 127) fail(GCP_EINVAL, "need 0 <= n_split <= 127");
  if (n_split > 0 && (!split_node || !split_neuron || !split_sign)) fail(GCP_EINVAL, "null split arrays");
  std::set<std::pair<int, int>> seen;
  for (int s = 0; s < n_split; ++s) {
    const int k = split_node[s];
    if (k < 0 || k >= out) fail(GCP_EINVAL, "split on a node that is not a ReLU layer");
    const gcp_node_desc& nk = desc->nodes[k];
    if (split_neuron[s] < 0 || split_neuron[s] >= nk.c * nk.h * nk.w) fail(GCP_EINVAL, "split neuron out of range");
    if (split_sign[s] != 1 && split_sign[s] != -1) fail(GCP_EINVAL, "split sign must be +1 or -1");
    if (!seen.insert({k, split_neuron[s]}).second) fail(GCP_EINVAL, "neuron split twice");
  }
  std::vector<std::vector<double>> L(out), U(out);
  std::vector<gcp_node_desc> nodes(desc->nodes, desc->nodes + desc->n_nodes);
  constexpr int kRowsPerCall = 4096;
  for (int k = 0; k < out; ++k) {
    const gcp_node_desc& nk = desc->nodes[k];
    const int d = nk.c * nk.h * nk.w;
    if (d <= 0) fail(GCP_EINVAL, "bad node shape");
    if (!lower[k] || !upper[k]) fail(GCP_EINVAL, "null bound output of node " + std::to_string(k));
    // the prefix network: nodes 0..k with node k as its output (the
    // pre-activation), earlier nodes carrying the bounds found so far
    gcp_net_desc sub{desc->in_c, desc->in_h, desc->in_w, k + 1, nodes.data()};
    for (int i = 0; i < k; ++i) {
      nodes[i].lower = L[i].data();
      nodes[i].upper = U[i].data();
    }
    nodes[k] = nk;
    nodes[k].lower = nodes[k].upper = nullptr;
    NetGuard net;
    {
      const int rc = gcp_net_create(&sub, &net.p);
      if (rc != GCP_OK) return rc;
    }
    // CROWN-adaptive lower slopes of the prefix's unstable neurons (in alpha
    // row order: node by node, ascending neuron index)
    std::vector<float> arow;
    for (int i = 0; i < k; ++i)
      for (size_t j = 0; j < L[i].size(); ++j)
        if (L[i][j] < 0.0 && U[i][j] > 0.0) arow.push_back(U[i][j] >= -L[i][j] ? 1.f : 0.f);
    const size_t nI = arow.size();
    // splits of earlier nodes whose neuron is unstable under the bounds found
    // so far (a stable one already takes the piece its bounds allow)
    std::vector<int32_t> sn, sj;
    std::vector<int8_t> ss;
    for (int s = 0; s < n_split; ++s) {
      const int i = split_node[s], j = split_neuron[s];
      if (i < k && L[i][j] < 0.0 && U[i][j] > 0.0) {
        sn.push_back(i);
        sj.push_back(j);
        ss.push_back(split_sign[s]);
      }
    }
    const int K = (int)sn.size();
    SplitsGuard spl;
    {
      const int rc = gcp_splits_create(net.p, 1, K, sn.data(), sj.data(), ss.data(), &spl.p);
      if (rc != GCP_OK) return rc;
    }
    // spec rows: +e_j (lower bound of x_j) then -e_j (minus the upper bound)
    const int S_all = 2 * d;
    const int rows = std::min(kRowsPerCall, S_all);
    DBuf Cd, Ad, Bd, Zd;   // Zd: the split multipliers, all 0
    Cd.alloc((size_t)rows * d * 8);
    if (K) Zd.alloc((size_t)rows * K * 4);
    Ad.alloc(std::max<size_t>((size_t)rows * nI * 4, 4));
    Bd.alloc((size_t)rows * 8);
    std::vector<float> arows((size_t)rows * nI);
    for (int r = 0; r < rows; ++r) std::copy(arow.begin(), arow.end(), arows.begin() + (size_t)r * nI);
    if (nI) hip_check(hipMemcpyAsync(Ad.p, arows.data(), arows.size() * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    std::vector<double> Ch((size_t)rows * d), bh(rows);
    std::vector<double> lo(d), hi(d);
    for (int s0 = 0; s0 < S_all; s0 += rows) {
      const int S = std::min(rows, S_all - s0);
      std::fill(Ch.begin(), Ch.end(), 0.0);
      for (int r = 0; r < S; ++r) {
        const int g = s0 + r;
        Ch[(size_t)r * d + (g < d ? g : g - d)] = g < d ? 1.0 : -1.0;
      }
      hip_check(hipMemcpyAsync(Cd.p, Ch.data(), (size_t)S * d * 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
      const int rc = gcp_bound(net.p, x0, eps, Cd.as<double>(), S, spl.p, nullptr, nI ? Ad.as<float>() : nullptr,
                               K ? Zd.as<float>() : nullptr, nullptr, mode & (0xff | GCP_FLAG_OUTWARD),
                               Bd.as<double>(), nullptr, nullptr,
                               nullptr, nullptr, stream);
      if (rc != GCP_OK) return rc;
      hip_check(hipMemcpyAsync(bh.data(), Bd.p, (size_t)S * 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
      for (int r = 0; r < S; ++r) {
        const int g = s0 + r;
        if (g < d) lo[g] = bh[r];
        else hi[g - d] = -bh[r];
      }
    }
    for (int j = 0; j < d; ++j) {
      if (!std::isfinite(lo[j]) || !std::isfinite(hi[j]))
        fail(GCP_ENONFINITE, "non-finite intermediate bound at node " + std::to_string(k));
      // an exactly determined pre-activation (l = u in exact arithmetic) can
      // come out a rounding error apart in the two directions
      if (lo[j] > hi[j]) std::swap(lo[j], hi[j]);
    }
    // a split neuron of this node: its bounds over the domain are clamped at
    // 0; a split that contradicts them (empty domain, up to rounding) leaves
    // the neuron at exactly 0
    for (int s = 0; s < n_split; ++s) {
      if (split_node[s] != k) continue;
      const int j = split_neuron[s];
      if (split_sign[s] > 0) {
        lo[j] = std::max(lo[j], 0.0);
        hi[j] = std::max(hi[j], lo[j]);
      } else {
        hi[j] = std::min(hi[j], 0.0);
        lo[j] = std::min(lo[j], hi[j]);
      }
    }
    L[k] = std::move(lo);
    U[k] = std::move(hi);
    std::copy(L[k].begin(), L[k].end(), lower[k]);
    std::copy(U[k].begin(), U[k].end(), upper[k]);
  }
  g_err.clear();
  return GCP_OK;
  GCP_CATCH
}

namespace gcp {
// error text for gcp_last_error from the other host sources of the library
void set_last_error(const char* m) { g_err = m ? m : ""; }
}  // namespace gcp
