// gcp_bound_mlp: the Theorem 3.1 bound of a dense ReLU network through the
// C ABI alone (no Python, no torch): reads a problem from a text file,
// uploads the inputs with the HIP runtime, calls gcp_bound and prints one
// bound per (domain, spec row).
//
// File format (whitespace-separated numbers):
//   L  d_0 .. d_L                         layer widths (L layers after the input)
//   for i = 1..L:  W_i [d_i][d_{i-1}]  b_i [d_i]
//   for i = 1..L-1: l_i [d_i]  u_i [d_i] root pre-activation bounds
//   x0 [d_0]  eps
//   S  C [S][d_L]
//   B K  node [B][K]  neuron [B][K]  sign [B][K]     (node = -1: unused slot)
//   N nnz  (cut node neuron kind coef) x nnz  d [N]   (node = -1: the input)
//   n_I  alpha [B*S][n_I]  beta [B*S][K]  gamma [B*S][N]
// Usage: gcp_bound_mlp <problem file> [fp32|bf16]
#include "../../include/gcp.h"

#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <string_view>
#include <vector>

namespace {

FILE* g_in = nullptr;

double num() {
  double v;
  if (std::fscanf(g_in, "%lf", &v) != 1) {
    std::fprintf(stderr, "gcp_bound_mlp: malformed problem file\n");
    std::exit(2);
  }
  return v;
}
template <class T> std::vector<T> vec(size_t n) {
  std::vector<T> v(n);
  for (auto& x : v) x = (T)num();
  return v;
}
void check(int rc, const char* what) {
  if (rc != GCP_OK) {
    std::fprintf(stderr, "gcp_bound_mlp: %s failed (%d): %s\n", what, rc, gcp_last_error());
    std::exit(1);
  }
}
void hcheck(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    std::fprintf(stderr, "gcp_bound_mlp: %s: %s\n", what, hipGetErrorString(e));
    std::exit(1);
  }
}
template <class T> void* upload(const std::vector<T>& v) {
  if (v.empty()) return nullptr;
  void* p = nullptr;
  hcheck(hipMalloc(&p, v.size() * sizeof(T)), "hipMalloc");
  hcheck(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
  return p;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s <problem file> [fp32|bf16]\n", argv[0]);
    return 2;
  }
  g_in = std::fopen(argv[1], "r");
  if (!g_in) {
    std::perror(argv[1]);
    return 2;
  }
  const int mode = (argc > 2 && std::string_view(argv[2]) == "bf16") ? GCP_MODE_BF16 : GCP_MODE_FP32;

  const int L = (int)num();
  std::vector<int> d(L + 1);
  for (auto& x : d) x = (int)num();
  std::vector<std::vector<float>> W(L), b(L);
  for (int i = 0; i < L; ++i) {
    W[i] = vec<float>((size_t)d[i + 1] * d[i]);
    b[i] = vec<float>(d[i + 1]);
  }
  std::vector<std::vector<double>> lo(L), hi(L);
  for (int i = 0; i + 1 < L; ++i) {
    lo[i] = vec<double>(d[i + 1]);
    hi[i] = vec<double>(d[i + 1]);
  }
  const std::vector<double> x0 = vec<double>(d[0]);
  const double eps = num();
  const int S = (int)num();
  const std::vector<double> C = vec<double>((size_t)S * d[L]);
  const int B = (int)num(), K = (int)num();
  const std::vector<int32_t> snode = vec<int32_t>((size_t)B * K), sneuron = vec<int32_t>((size_t)B * K);
  const std::vector<int8_t> ssign = vec<int8_t>((size_t)B * K);
  const int N = (int)num();
  const int64_t nnz = (int64_t)num();
  std::vector<int32_t> ccut(nnz), cnode(nnz), cneuron(nnz);
  std::vector<int8_t> ckind(nnz);
  std::vector<double> ccoef(nnz);
  for (int64_t e = 0; e < nnz; ++e) {
    ccut[e] = (int32_t)num(); cnode[e] = (int32_t)num(); cneuron[e] = (int32_t)num();
    ckind[e] = (int8_t)num(); ccoef[e] = num();
  }
  const std::vector<double> cd = vec<double>(N);
  const int nI = (int)num();
  const int M = B * S;
  const std::vector<float> alpha = vec<float>((size_t)M * nI), beta = vec<float>((size_t)M * K),
                           gamma = vec<float>((size_t)M * N);
  std::fclose(g_in);

  // the network: node i (0-based) = layer i+1, one dense edge from node i-1
  std::vector<gcp_edge_desc> edges(L);
  std::vector<gcp_node_desc> nodes(L);
  for (int i = 0; i < L; ++i) {
    edges[i] = gcp_edge_desc{i - 1, GCP_EDGE_DENSE, W[i].data(), 0, 0, 0, 0};
    nodes[i] = gcp_node_desc{d[i + 1], 1, 1, b[i].data(), i + 1 < L ? lo[i].data() : nullptr,
                             i + 1 < L ? hi[i].data() : nullptr, 1, &edges[i]};
  }
  const gcp_net_desc desc{d[0], 1, 1, L, nodes.data()};
  gcp_net* net = nullptr;
  check(gcp_net_create(&desc, &net), "gcp_net_create");
  gcp_net_info info;
  check(gcp_net_get_info(net, &info), "gcp_net_get_info");
  if (info.n_unstable != nI) {
    std::fprintf(stderr, "gcp_bound_mlp: alpha rows have %d entries, the net has %lld unstable neurons\n", nI,
                 (long long)info.n_unstable);
    return 1;
  }
  gcp_splits* splits = nullptr;
  check(gcp_splits_create(net, B, K, snode.data(), sneuron.data(), ssign.data(), &splits), "gcp_splits_create");
  gcp_cuts* cuts = nullptr;
  if (N > 0)
    check(gcp_cuts_create(net, N, nnz, ccut.data(), cnode.data(), cneuron.data(), ckind.data(), ccoef.data(),
                          cd.data(), &cuts),
          "gcp_cuts_create");

  void* dx0 = upload(x0);
  void* dC = upload(C);
  void* da = upload(alpha);
  void* db = upload(beta);
  void* dg = upload(gamma);
  double* dbound = nullptr;
  hcheck(hipMalloc((void**)&dbound, (size_t)M * sizeof(double)), "hipMalloc");
  check(gcp_bound(net, (const double*)dx0, eps, (const double*)dC, S, splits, cuts, (const float*)da,
                  (const float*)db, (const float*)dg, mode, dbound, nullptr, nullptr, nullptr, nullptr, nullptr),
        "gcp_bound");
  std::vector<double> bound(M);
  hcheck(hipMemcpy(bound.data(), dbound, (size_t)M * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
  for (int r = 0; r < M; ++r) std::printf("%.17g\n", bound[r]);

  for (void* p : {dx0, dC, da, db, dg, (void*)dbound})
    if (p) (void)hipFree(p);
  if (cuts) gcp_cuts_destroy(cuts);
  gcp_splits_destroy(splits);
  gcp_net_destroy(net);
  return 0;
}
