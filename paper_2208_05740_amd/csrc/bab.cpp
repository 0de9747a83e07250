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
// as unresolved.  Built only on the library's public calls.
#include "../../include/gcp.h"

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
  std::vector<float> a, b, g;    // warm start (empty: alpha CROWN-adaptive, beta = gamma = 0)
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
    DevMem alpha, beta, gamma, state, bound, verified;
    std::vector<double> hb;
    while (true) {
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
      std::vector<Domain> sel(pool.begin(), pool.begin() + take);
      pool.erase(pool.begin(), pool.begin() + take);
      // batch rows padded to a power of two (repeating the first domain) so
      // few distinct shapes are tuned
      int Bp = 1;
      while (Bp < take) Bp *= 2;
      Bp = std::min(Bp, std::max(o->batch, take));
      const int Kc = std::max(K, 1);
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
      SplitsHandle sp;
      check(gcp_splits_create(net, Bp, K, K ? snode.data() : nullptr, K ? sneur.data() : nullptr,
                              K ? ssign.data() : nullptr, &sp.p));
      const size_t M = (size_t)Bp;     // one spec row per domain
      alpha.need(std::max<size_t>(M * nI * 4, 4));
      beta.need(std::max<size_t>(M * K * 4, 4));
      gamma.need(std::max<size_t>(M * N * 4, 4));
      state.need(std::max<size_t>(2 * M * (nI + K + N) * 4, 4));
      bound.need(M * 8);
      verified.need(M);
      std::vector<float> ha(M * nI), hbeta(M * K, 0.f), hg(M * N, 0.f);
      for (size_t m = 0; m < M; ++m) {
        const Domain& d = sel[m < (size_t)take ? m : 0];
        std::copy(d.a.empty() ? arow.begin() : d.a.begin(), d.a.empty() ? arow.end() : d.a.end(), ha.begin() + m * nI);
        std::copy(d.b.begin(), d.b.end(), hbeta.begin() + m * K);
        if (!d.g.empty()) std::copy(d.g.begin(), d.g.end(), hg.begin() + m * N);
      }
      if (nI) hcheck(hipMemcpyAsync(alpha.p, ha.data(), ha.size() * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
      if (K) hcheck(hipMemcpyAsync(beta.p, hbeta.data(), hbeta.size() * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
      if (N) hcheck(hipMemcpyAsync(gamma.p, hg.data(), hg.size() * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
      hcheck(hipMemsetAsync(state.p, 0, 2 * M * (nI + K + N) * 4, st), "hipMemsetAsync");
      check(gcp_optimize(net, x0, eps, c, 1, sp.p, cuts, nI ? (float*)alpha.p : nullptr, K ? (float*)beta.p : nullptr,
                         N ? (float*)gamma.p : nullptr, (float*)state.p, &o->opt, o->mode, (double*)bound.p,
                         (uint8_t*)verified.p, stream));
      hb.resize(M);
      hcheck(hipMemcpyAsync(hb.data(), bound.p, M * 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      if (nI) hcheck(hipMemcpyAsync(ha.data(), alpha.p, (size_t)take * nI * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      if (K) hcheck(hipMemcpyAsync(hbeta.data(), beta.p, (size_t)take * K * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      if (N) hcheck(hipMemcpyAsync(hg.data(), gamma.p, (size_t)take * N * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      hcheck(hipStreamSynchronize(st), "hipStreamSynchronize");
      R.bounded += take;
      R.rounds += 1;
      for (int b = 0; b < take; ++b) {
        Domain& d = sel[b];
        const double g = hb[b];
        if (!std::isfinite(g)) throw BabErr{GCP_ENONFINITE, "non-finite bound"};
        if (g >= 0.0) {                      // verified: pruned
          min_leaf = std::min(min_leaf, g);
          continue;
        }
        // optimised parameters of this domain: its children's start
        d.a.assign(ha.begin() + (size_t)b * nI, ha.begin() + (size_t)(b + 1) * nI);
        d.b.assign(hbeta.begin() + (size_t)b * K, hbeta.begin() + (size_t)b * K + d.split.size());
        d.g.assign(hg.begin() + (size_t)b * N, hg.begin() + (size_t)(b + 1) * N);
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
          ch.a = d.a;
          ch.b = d.b;
          ch.g = d.g;
          ch.split.push_back(next);
          ch.sign.push_back(sg);
          ch.b.push_back(0.f);
          pool.push_back(std::move(ch));
        }
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
