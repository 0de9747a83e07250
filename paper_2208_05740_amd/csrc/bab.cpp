// Branch and bound around the GCP-CROWN bounding step (the BaB procedure
// described in Appendix B, with the easiest-first order of Sec. 3.3).
//
// A domain is a set of ReLU splits (x_j >= 0 or x_j <= 0) on root-unstable
// neurons.  Each round bounds up to `batch` open domains with gcp_optimize
// (one call, all domains as rows of one batch), drops those whose bound is
// >= 0 (verified), and splits each remaining one on its highest-scoring
// unsplit unstable neuron into two children.  When more domains are open
// than fit in a batch, the ones with the largest parent bound go first.
// The branching score is static: the height u*(-l)/(u-l) of the triangle
// relaxation at the root bounds (the largest gap the relaxation leaves).
// Children start from their parent's optimised alpha, beta (the new split's
// multiplier at 0) and gamma, so a deep domain has accumulated the Adam
// steps of all its ancestors; a domain that cannot be split further is
// bounded again from its own optimum up to `retries` times before it counts
// as unresolved.
//
// The open domains' parameters stay on the device: a pool of rows (alpha,
// beta, gamma of each open domain) from which a round gathers its batch and
// into which it scatters the children's warm starts (the new split's beta
// column zeroed) after the bounding call, so a round moves only row indices
// to the device and the bounds back.  Built on the library's public calls
// plus the row-copy kernel and the in-place split-handle refill.
#include "../../include/gcp.h"
#include "gcp_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

namespace gcp {
void set_last_error(const char* m);
}

namespace {

struct BabErr {
  int code;
  std::string msg;
};

struct Domain {
  std::vector<int32_t> split;    // indices into the unstable list
  std::vector<int8_t> sign;      // +1: x >= 0, -1: x <= 0
  double parent;                 // bound of the parent domain (-inf at the root)
  int slot = 0;                  // pool row of the warm start (row 0: alpha CROWN-adaptive, beta = gamma = 0)
  int retry = 0;
};

struct DevMem {
  void* p = nullptr;
  size_t n = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  void need(size_t bytes) {
    if (bytes <= n) return;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    if (hipMalloc(&p, bytes) != hipSuccess) throw BabErr{GCP_ENOMEM, "device allocation failed"};
    n = bytes;
  }
};

void check(int rc) {
  if (rc != GCP_OK) throw rc;
}
void hcheck(hipError_t e, const char* what) {
  if (e != hipSuccess) throw BabErr{GCP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

struct SplitsHandle {
  gcp_splits* p = nullptr;
  ~SplitsHandle() {
    if (p) gcp_splits_destroy(p);
  }
};

// Rows of the parameter pool (alpha [nI], beta [K], gamma [N] per row); row 0
// is the root start and never freed.  Grows by doubling (device copy of the
// rows in use).
struct Pool {
  int nI, K, N;
  int cap = 0;
  DevMem a, b, g;
  std::vector<int> free_rows;
  void grow(int want, hipStream_t st) {
    int nc = std::max(cap * 2, want);
    DevMem na, nb, ng;
    na.need(std::max<size_t>((size_t)nc * nI * 4, 4));
    nb.need(std::max<size_t>((size_t)nc * K * 4, 4));
    ng.need(std::max<size_t>((size_t)nc * N * 4, 4));
    if (cap > 0) {
      if (nI) hcheck(hipMemcpyAsync(na.p, a.p, (size_t)cap * nI * 4, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
      if (K) hcheck(hipMemcpyAsync(nb.p, b.p, (size_t)cap * K * 4, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
      if (N) hcheck(hipMemcpyAsync(ng.p, g.p, (size_t)cap * N * 4, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
      hcheck(hipStreamSynchronize(st), "hipStreamSynchronize");
    }
    std::swap(a.p, na.p); std::swap(a.n, na.n);
    std::swap(b.p, nb.p); std::swap(b.n, nb.n);
    std::swap(g.p, ng.p); std::swap(g.n, ng.n);
    for (int r = nc - 1; r >= std::max(cap, 1); --r) free_rows.push_back(r);
    cap = nc;
  }
  int take(hipStream_t st) {
    if (free_rows.empty()) grow(cap + 1, st);
    const int r = free_rows.back();
    free_rows.pop_back();
    return r;
  }
  void release(int r) {
    if (r > 0) free_rows.push_back(r);
  }
};

// dst[dst_row[i]] = src[src_row[i]] for the index lists on the device, in
// launches of at most 65535 rows
void copy_rows(float* dst, int64_t ld_dst, const int32_t* dst_row, const float* src, int64_t ld_src,
               const int32_t* src_row, int n, int L, const int32_t* zero_col, hipStream_t st) {
  for (int i0 = 0; i0 < n; i0 += 65535) {
    const int c = std::min(65535, n - i0);
    hcheck(gcp::launch_copy_rows(dst, ld_dst, dst_row + i0, src, ld_src, src_row + i0, c, L,
                                 zero_col ? zero_col + i0 : nullptr, st),
           "row copy");
  }
}

}  // namespace

extern "C" int gcp_bab(const gcp_net* net, const double* x0, double eps, const double* c, const gcp_cuts* cuts,
                       const gcp_bab_opt* o, gcp_bab_result* res, void* stream) {
  try {
    if (!net || !x0 || !c || !o || !res) throw BabErr{GCP_EINVAL, "null argument"};
    if (o->batch < 1 || o->max_depth < 0 || o->max_domains < 1 || o->max_pool < 1 || o->retries < 0)
      throw BabErr{GCP_EINVAL, "bad branch-and-bound settings"};
    hipStream_t st = (hipStream_t)stream;
    gcp_net_info info{};
    check(gcp_net_get_info(net, &info));
    const int nI = (int)info.n_unstable;
    int32_t N = 0;
    if (cuts) check(gcp_cuts_info(cuts, &N));
    std::vector<int32_t> unode(nI), uneuron(nI);
    std::vector<double> ul(nI), uu(nI);
    if (nI > 0) check(gcp_net_get_unstable(net, unode.data(), uneuron.data(), ul.data(), uu.data()));
    const int K = std::min<int>(o->max_depth, nI);
    // static branching order and the CROWN-adaptive starting slopes
    std::vector<int32_t> order(nI);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> score(nI);
    std::vector<float> arow(nI);
    for (int r = 0; r < nI; ++r) {
      score[r] = uu[r] * (-ul[r]) / (uu[r] - ul[r]);
      arow[r] = uu[r] >= -ul[r] ? 1.f : 0.f;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return score[a] > score[b]; });

    std::vector<Domain> pool(1);
    pool[0].parent = -std::numeric_limits<double>::infinity();
    gcp_bab_result R{};
    R.status = GCP_BAB_UNKNOWN;
    double min_leaf = std::numeric_limits<double>::infinity();     // smallest verified leaf bound
    double min_open = std::numeric_limits<double>::infinity();     // smallest bound left unresolved
    const int Kc = std::max(K, 1);
    Pool P{nI, K, (int)N};
    P.grow(std::max(2, std::min<int>(4 * o->batch + 1, 1 << 16)), st);
    // row 0: the root start (alpha CROWN-adaptive, beta = gamma = 0; the
    // pool's fresh memory is zero)
    if (nI) hcheck(hipMemcpyAsync(P.a.p, arow.data(), (size_t)nI * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    if (K) hcheck(hipMemsetAsync(P.b.p, 0, (size_t)K * 4, st), "hipMemsetAsync");
    if (N) hcheck(hipMemsetAsync(P.g.p, 0, (size_t)N * 4, st), "hipMemsetAsync");
    DevMem alpha, beta, gamma, state, bound, verified, idx;
    SplitsHandle sp;
    std::vector<double> hb;
    // row-index lists of a round, staged on the host until the round's sync:
    // [0, Bp) gather rows, then (dst, src, zero column) of the scatter
    std::vector<int32_t> hidx;
    while (true) {
      // the previous round's scatter is done before its host lists and
      // device buffers are reused or regrown
      hcheck(hipStreamSynchronize(st), "hipStreamSynchronize");
      if (pool.empty()) {
        if (R.unresolved == 0) R.status = GCP_BAB_VERIFIED;
        break;
      }
      if (R.bounded >= o->max_domains || (int64_t)pool.size() > o->max_pool) break;
      // easiest first: the open domains with the largest parent bound
      const int take = (int)std::min<size_t>(pool.size(), (size_t)o->batch);
      if ((int)pool.size() > take)
        std::nth_element(pool.begin(), pool.begin() + take, pool.end(),
                         [](const Domain& a, const Domain& b) { return a.parent > b.parent; });
      std::vector<Domain> sel(std::make_move_iterator(pool.begin()), std::make_move_iterator(pool.begin() + take));
      pool.erase(pool.begin(), pool.begin() + take);
      // batch rows padded to a power of two (repeating the first domain) so
      // few distinct shapes are tuned
      int Bp = 1;
      while (Bp < take) Bp *= 2;
      Bp = std::min(Bp, std::max(o->batch, take));
      std::vector<int32_t> snode((size_t)Bp * Kc, -1), sneur((size_t)Bp * Kc, 0);
      std::vector<int8_t> ssign((size_t)Bp * Kc, 1);
      for (int b = 0; b < Bp; ++b) {
        const Domain& d = sel[b < take ? b : 0];
        for (size_t k = 0; k < d.split.size(); ++k) {
          snode[(size_t)b * Kc + k] = unode[d.split[k]];
          sneur[(size_t)b * Kc + k] = uneuron[d.split[k]];
          ssign[(size_t)b * Kc + k] = d.sign[k];
        }
      }
      check(gcp::splits_assign(net, &sp.p, Bp, K, K ? snode.data() : nullptr, K ? sneur.data() : nullptr,
                               K ? ssign.data() : nullptr, st));
      const size_t M = (size_t)Bp;     // one spec row per domain
      alpha.need(std::max<size_t>(M * nI * 4, 4));
      beta.need(std::max<size_t>(M * K * 4, 4));
      gamma.need(std::max<size_t>(M * N * 4, 4));
      state.need(std::max<size_t>(2 * M * (nI + K + N) * 4, 4));
      bound.need(M * 8);
      verified.need(M);
      // index lists: batch rows 0..Bp-1, their pool rows, then the scatter
      // lists (destination pool row, source batch row, zeroed beta column;
      // at most two entries per selected domain)
      const size_t n_sc = 2 * (size_t)take;
      hidx.assign(2 * M + 3 * n_sc, 0);
      for (size_t m = 0; m < M; ++m) {
        hidx[m] = (int32_t)m;
        hidx[M + m] = sel[m < (size_t)take ? m : 0].slot;
      }
      idx.need(hidx.size() * 4);
      const int32_t* d_rows = (const int32_t*)idx.p;
      const int32_t* d_slots = d_rows + M;
      hcheck(hipMemcpyAsync(idx.p, hidx.data(), 2 * M * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
      copy_rows((float*)alpha.p, nI, d_rows, (const float*)P.a.p, nI, d_slots, (int)M, nI, nullptr, st);
      copy_rows((float*)beta.p, K, d_rows, (const float*)P.b.p, K, d_slots, (int)M, K, nullptr, st);
      copy_rows((float*)gamma.p, N, d_rows, (const float*)P.g.p, N, d_slots, (int)M, N, nullptr, st);
      for (Domain& d : sel) {     // their rows are read before any later write on this stream
        P.release(d.slot);
        d.slot = 0;
      }
      hcheck(hipMemsetAsync(state.p, 0, 2 * M * (nI + K + N) * 4, st), "hipMemsetAsync");
      check(gcp_optimize(net, x0, eps, c, 1, sp.p, cuts, nI ? (float*)alpha.p : nullptr, K ? (float*)beta.p : nullptr,
                         N ? (float*)gamma.p : nullptr, (float*)state.p, &o->opt, o->mode, (double*)bound.p,
                         (uint8_t*)verified.p, stream));
      hb.resize(M);
      hcheck(hipMemcpyAsync(hb.data(), bound.p, M * 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      hcheck(hipStreamSynchronize(st), "hipStreamSynchronize");
      R.bounded += take;
      R.rounds += 1;
      // children (and retried domains) take pool rows holding this round's
      // optimum of their parent (the new split's beta column zeroed)
      int32_t* dst = hidx.data() + 2 * M;
      int32_t* src = dst + n_sc;
      int32_t* zc = src + n_sc;
      int n_copy = 0;
      auto keep = [&](int b, int zero_col) {
        const int r = P.take(st);
        dst[n_copy] = r; src[n_copy] = b; zc[n_copy] = zero_col;
        ++n_copy;
        return r;
      };
      for (int b = 0; b < take; ++b) {
        Domain& d = sel[b];
        const double g = hb[b];
        if (!std::isfinite(g)) throw BabErr{GCP_ENONFINITE, "non-finite bound"};
        if (g >= 0.0) {                      // verified: pruned
          min_leaf = std::min(min_leaf, g);
          continue;
        }
        int next = -1;
        if ((int)d.split.size() < K)
          for (int r : order)
            if (std::find(d.split.begin(), d.split.end(), r) == d.split.end()) {
              next = r;
              break;
            }
        if (next < 0) {                      // nothing left to split within the depth
          if (d.retry < o->retries) {
            d.retry += 1;
            d.parent = g;
            d.slot = keep(b, -1);
            pool.push_back(std::move(d));
            continue;
          }
          R.unresolved += 1;
          min_open = std::min(min_open, g);
          continue;
        }
        for (int8_t sg : {(int8_t)1, (int8_t)-1}) {
          Domain ch;
          ch.split = d.split;
          ch.sign = d.sign;
          ch.parent = g;
          ch.slot = keep(b, (int)d.split.size());
          ch.split.push_back(next);
          ch.sign.push_back(sg);
          pool.push_back(std::move(ch));
        }
      }
      if (n_copy > 0) {
        int32_t* d_dst = (int32_t*)idx.p + 2 * M;
        int32_t* d_src = d_dst + n_sc;
        int32_t* d_zc = d_src + n_sc;
        hcheck(hipMemcpyAsync(d_dst, dst, 3 * n_sc * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        copy_rows((float*)P.a.p, nI, d_dst, (const float*)alpha.p, nI, d_src, n_copy, nI, nullptr, st);
        copy_rows((float*)P.b.p, K, d_dst, (const float*)beta.p, K, d_src, n_copy, K, d_zc, st);
        copy_rows((float*)P.g.p, N, d_dst, (const float*)gamma.p, N, d_src, n_copy, N, nullptr, st);
      }
      R.max_open = std::max<int64_t>(R.max_open, (int64_t)pool.size());
    }
    for (const Domain& d : pool) min_open = std::min(min_open, d.parent);
    R.lower = R.status == GCP_BAB_VERIFIED ? min_leaf : min_open;
    R.open = (int64_t)pool.size();
    *res = R;
    gcp::set_last_error("");
    return GCP_OK;
  } catch (const BabErr& e) {
    gcp::set_last_error(e.msg.c_str());
    return e.code;
  } catch (int rc) {
    return rc;   // the failing library call has set the error text
  } catch (const std::bad_alloc&) {
    gcp::set_last_error("host allocation failed");
    return GCP_ENOMEM;
  } catch (...) {
    gcp::set_last_error("unexpected internal error");
    return GCP_EDEVICE;
  }
}
