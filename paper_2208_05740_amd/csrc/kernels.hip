// gfx950 kernels of the GCP-CROWN bound pass, its adjoint and the projected
// Adam step (arXiv 2208.05740, Theorem 3.1 / Lemma A.1; optimiser of
// Appendix C.1).  One row = one (domain, spec row) scalar problem.
//
// Layout: per-row activation buffers are row-major [M][ld] with ld a
// multiple of 16 elements and zero padding columns; weights are stored as
// "Bt" = [N][K] (K contiguous) so both MFMA operands stream along K:
//   bound direction  a_hat^(p) = Lambda^(i) W      uses Bt = W^T  [d_p][d_i]
//   adjoint          dLambda^(i) = da_hat^(p) W^T  uses Bt = W    [d_i][d_p]
#include "gcp_internal.h"
#include "epilogues.h"
#include "tiles.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace gcp {

template <typename T, int BM, int BN, int WM, int WN, int BK, bool SIGN, class Epi>
__global__ void __launch_bounds__(WM * WN * 64) gemm_epi_kernel(GemmArgs g, Epi epi) {
  const int total = ((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM);
  gemm_tile<T, BM, BN, WM, WN, BK, SIGN, Epi>(g, epi, xcd_tile(blockIdx.x, total));
}

// Several independent GEMM problems of one kernel instantiation in one
// launch: tiles of problem p occupy [prefix[p], prefix[p+1]) of the linear
// tile space; each workgroup finds its problem by binary search.
template <typename T, int BM, int BN, int WM, int WN, int BK, bool SIGN, class Epi>
__global__ void __launch_bounds__(WM * WN * 64)
gemm_epi_grouped(const GemmArgs* __restrict__ gs, const Epi* __restrict__ es, const int* __restrict__ prefix, int np) {
  const int t = xcd_tile(blockIdx.x, prefix[np]);
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const GemmArgs g = gs[lo];
  const Epi e = es[lo];
  gemm_tile<T, BM, BN, WM, WN, BK, SIGN, Epi>(g, e, t - prefix[lo]);
}

// Tile configurations available to the autotuner: (BM, BN, WM, WN).
struct TileCfg { int bm, bn; };
static const TileCfg kCfgs[] = {{64, 64}, {128, 64}, {64, 128}, {128, 128}, {32, 64}, {32, 32}, {16, 64}, {16, 32}};
static_assert(sizeof(kCfgs) / sizeof(kCfgs[0]) == 8, "tile table");
int gemm_num_configs() { return (int)(sizeof(kCfgs) / sizeof(kCfgs[0])); }
void gemm_config_tile(int cfg, int* bm, int* bn) { *bm = kCfgs[cfg].bm; *bn = kCfgs[cfg].bn; }

// Launch target: a single problem (GemmArgs by value) or a group (device
// tables of arguments and tile prefix sums).
struct GemmLaunch {
  const GemmArgs* g;          // single: host pointer to the arguments
  const void* epi;            // single: host pointer to the epilogue arguments
  const GemmArgs* d_gs;       // grouped: device tables
  const void* d_es;
  const int* d_prefix;
  int np, total_tiles;
};

template <typename T, int BM, int BN, int WM, int WN, bool SIGN, class Epi, class Args>
static hipError_t launch_cfg(const GemmLaunch& L, hipStream_t st) {
  constexpr int BK = (sizeof(T) == 4) ? 64 : 128;
  if (L.d_gs) {
    if (L.total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((gemm_epi_grouped<T, BM, BN, WM, WN, BK, SIGN, Epi>), dim3((unsigned)L.total_tiles),
                       dim3(WM * WN * 64), 0, st, L.d_gs, (const Epi*)L.d_es, L.d_prefix, L.np);
    return hipGetLastError();
  }
  const GemmArgs& g = *L.g;
  const long tiles = (long)((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM);
  hipLaunchKernelGGL((gemm_epi_kernel<T, BM, BN, WM, WN, BK, SIGN, Epi>), dim3((unsigned)tiles),
                     dim3(WM * WN * 64), 0, st, g, Epi{*(const Args*)L.epi});
  return hipGetLastError();
}

template <typename T, bool SIGN, class Epi, class Args>
static hipError_t launch_any(int cfg, const GemmLaunch& L, hipStream_t st) {
  switch (cfg) {
    case 0: return launch_cfg<T, 64, 64, 2, 2, SIGN, Epi, Args>(L, st);
    case 1: return launch_cfg<T, 128, 64, 2, 2, SIGN, Epi, Args>(L, st);
    case 2: return launch_cfg<T, 64, 128, 2, 2, SIGN, Epi, Args>(L, st);
    case 3: return launch_cfg<T, 128, 128, 2, 2, SIGN, Epi, Args>(L, st);
    case 4: return launch_cfg<T, 32, 64, 2, 2, SIGN, Epi, Args>(L, st);
    case 5: return launch_cfg<T, 32, 32, 2, 2, SIGN, Epi, Args>(L, st);
    case 6: return launch_cfg<T, 16, 64, 1, 4, SIGN, Epi, Args>(L, st);
    case 7: return launch_cfg<T, 16, 32, 1, 2, SIGN, Epi, Args>(L, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_typed(int cfg, EpiKind kind, int sign, const GemmLaunch& L, hipStream_t st) {
  switch (kind) {
    case EPI_BOUND: return launch_any<T, false, BoundEpi<T>, BoundEpiArgs>(cfg, L, st);
    case EPI_AHAT: return launch_any<T, false, AhatEpi<T>, BoundEpiArgs>(cfg, L, st);
    case EPI_CONC: return launch_any<T, false, ConcEpi, ConcEpiArgs>(cfg, L, st);
    case EPI_STORE:
      if (sign) return launch_any<T, true, StoreEpi, StoreEpiArgs>(cfg, L, st);
      return launch_any<T, false, StoreEpi, StoreEpiArgs>(cfg, L, st);
    case EPI_ADJ:
      if (sign) return launch_any<T, true, AdjEpi<T>, AdjEpiArgs>(cfg, L, st);
      return launch_any<T, false, AdjEpi<T>, AdjEpiArgs>(cfg, L, st);
  }
  return hipErrorInvalidValue;
}

// Explicit-pi epilogues (rho set): instantiated for the small tiles only
// (their fragments carry rho and its moments); a large-tile choice runs as
// 32x32.
template <typename T, bool SIGN, class Epi, class Args>
static hipError_t launch_small(int cfg, const GemmLaunch& L, hipStream_t st) {
  switch (cfg) {
    case 6: return launch_cfg<T, 16, 64, 1, 4, SIGN, Epi, Args>(L, st);
    case 7: return launch_cfg<T, 16, 32, 1, 2, SIGN, Epi, Args>(L, st);
    default: return launch_cfg<T, 32, 32, 2, 2, SIGN, Epi, Args>(L, st);
  }
}

template <typename T>
static hipError_t launch_pi(int cfg, EpiKind kind, int sign, const GemmLaunch& L, hipStream_t st) {
  if (kind == EPI_BOUND) return launch_small<T, false, BoundEpi<T, true>, BoundEpiArgs>(cfg, L, st);
  if (kind != EPI_ADJ) return hipErrorInvalidValue;
  if (sign) return launch_small<T, true, AdjEpi<T, true>, AdjEpiArgs>(cfg, L, st);
  return launch_small<T, false, AdjEpi<T, true>, AdjEpiArgs>(cfg, L, st);
}

hipError_t launch_gemm(int bf16_mode, int cfg, EpiKind kind, const GemmArgs& g, const void* epi,
                       hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (cfg < 0 || cfg >= gemm_num_configs()) return hipErrorInvalidValue;
  GemmLaunch L{&g, epi, nullptr, nullptr, nullptr, 0, 0};
  if (fused_explicit_pi(kind, epi))
    return bf16_mode ? launch_pi<bf16>(cfg, kind, g.a_is_sign, L, st) : launch_pi<float>(cfg, kind, g.a_is_sign, L, st);
  return bf16_mode ? launch_typed<bf16>(cfg, kind, g.a_is_sign, L, st)
                   : launch_typed<float>(cfg, kind, g.a_is_sign, L, st);
}

// Grouped problems carry Lemma A.1's pi* epilogues only (no rho).
hipError_t launch_gemm_grouped(int bf16_mode, int cfg, EpiKind kind, int sign, const GemmArgs* d_gs,
                               const void* d_epis, const int* d_prefix, int np, int total_tiles, hipStream_t st) {
  GemmLaunch L{nullptr, nullptr, d_gs, d_epis, d_prefix, np, total_tiles};
  return bf16_mode ? launch_typed<bf16>(cfg, kind, sign, L, st) : launch_typed<float>(cfg, kind, sign, L, st);
}

// ------------------------------------------------------------------ elementwise
template <typename T, bool PI>
__global__ void __launch_bounds__(256) bound_elem_kernel(const float* bcast, const void* src, BoundEpiArgs a,
                                                         double* partial, int slot0) {
  bound_elem_rows<T, PI>(bcast, src, a, partial, slot0, kElemRows * blockIdx.x, blockIdx.y);
}

hipError_t launch_bound_elementwise(int bf16_mode, const float* bcast, const void* src, const BoundEpiArgs& a,
                                    double* partial, int slot0, hipStream_t st) {
  if (a.rp.M <= 0) return hipSuccess;
  dim3 grid((a.rp.M + kElemRows - 1) / kElemRows, (a.nd.size + 255) / 256);
  const bool pi = a.rp.rho != nullptr;
  if (bf16_mode && pi)
    hipLaunchKernelGGL((bound_elem_kernel<bf16, true>), grid, dim3(256), 0, st, bcast, src, a, partial, slot0);
  else if (bf16_mode)
    hipLaunchKernelGGL((bound_elem_kernel<bf16, false>), grid, dim3(256), 0, st, bcast, src, a, partial, slot0);
  else if (pi)
    hipLaunchKernelGGL((bound_elem_kernel<float, true>), grid, dim3(256), 0, st, bcast, src, a, partial, slot0);
  else
    hipLaunchKernelGGL((bound_elem_kernel<float, false>), grid, dim3(256), 0, st, bcast, src, a, partial, slot0);
  return hipGetLastError();
}

// Grouped elementwise relaxation: block b of job p covers rows
// kElemRows * (b / nb) .. and columns 256 * (b % nb) .. of that job,
// nb = ceil(size / 256).
template <typename T>
__global__ void __launch_bounds__(256) bound_elem_grouped(const ElemBoundJob* __restrict__ jobs,
                                                          const int* __restrict__ prefix, int np) {
  const int t = blockIdx.x;
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const ElemBoundJob& jb = jobs[lo];
  const int nb = (jb.a.nd.size + 255) / 256;
  const int b = t - prefix[lo];
  bound_elem_rows<T, false>(jb.bcast, jb.src, jb.a, jb.partial, jb.slot0, kElemRows * (b / nb), b % nb);
}

hipError_t launch_bound_elementwise_grouped(int bf16_mode, const ElemBoundJob* d_jobs, const int* d_prefix, int np,
                                            int total_blocks, hipStream_t st) {
  if (total_blocks <= 0) return hipSuccess;
  if (bf16_mode)
    hipLaunchKernelGGL(bound_elem_grouped<bf16>, dim3(total_blocks), dim3(256), 0, st, d_jobs, d_prefix, np);
  else
    hipLaunchKernelGGL(bound_elem_grouped<float>, dim3(total_blocks), dim3(256), 0, st, d_jobs, d_prefix, np);
  return hipGetLastError();
}

template <typename T, bool PI>
__global__ void __launch_bounds__(256) adj_elem_kernel(AdjEpiArgs a) {
  const int r = blockIdx.x;
  const int j = blockIdx.y * 256 + threadIdx.x;
  AdjEpi<T, PI> epi{a};
  LaneCoords<1, 1, false> lc;
  lc.r[0] = r;
  lc.j[0][0] = j;
  float val[1][1] = {{0.f}};
  double rs[1] = {0.0};
  typename AdjEpi<T, PI>::template Frag<1, 1, false> fr;
  epi.template load<1, 1, false>(fr, lc, a.rp.M, a.nd.size);
  epi.template apply<1, 1, false>(fr, lc, val, rs, a.rp.M, a.nd.size);
}

hipError_t launch_adj_elementwise(int bf16_mode, const AdjEpiArgs& a, hipStream_t st) {
  dim3 grid(a.rp.M, (a.nd.size + 255) / 256);
  const bool pi = a.rp.rho != nullptr;
  if (bf16_mode && pi)
    hipLaunchKernelGGL((adj_elem_kernel<bf16, true>), grid, dim3(256), 0, st, a);
  else if (bf16_mode)
    hipLaunchKernelGGL((adj_elem_kernel<bf16, false>), grid, dim3(256), 0, st, a);
  else if (pi)
    hipLaunchKernelGGL((adj_elem_kernel<float, true>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((adj_elem_kernel<float, false>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// out[r][j] = (acc_in ? acc_in[r][j] : 0) + scale * src[r][j]  (identity edge);
// src is the operand type, or int8 signs when is_sign.
template <typename T>
__global__ void __launch_bounds__(256) identity_acc_kernel(int M, int size, const void* src, int ld_src, int is_sign,
                                                           float scale, const float* acc_in, float* out, int ld_out) {
  const int r = blockIdx.x;
  const int j = blockIdx.y * 256 + threadIdx.x;
  if (j >= size) return;
  const float x = is_sign ? (float)((const int8_t*)src)[(size_t)r * ld_src + j]
                          : from_t<T>(((const T*)src)[(size_t)r * ld_src + j]);
  out[(size_t)r * ld_out + j] = (acc_in ? acc_in[(size_t)r * ld_out + j] : 0.f) + scale * x;
}

hipError_t launch_identity_acc(int bf16_mode, int M, int size, const void* src, int ld_src, int is_sign, float scale,
                               const float* acc_in, float* out, int ld_out, hipStream_t st) {
  if (M == 0 || size == 0) return hipSuccess;
  dim3 grid(M, (size + 255) / 256);
  if (bf16_mode)
    hipLaunchKernelGGL(identity_acc_kernel<bf16>, grid, dim3(256), 0, st, M, size, src, ld_src, is_sign, scale,
                       acc_in, out, ld_out);
  else
    hipLaunchKernelGGL(identity_acc_kernel<float>, grid, dim3(256), 0, st, M, size, src, ld_src, is_sign, scale,
                       acc_in, out, ld_out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ small kernels
// chat[s][j] = sum_o C[s][o] * W[o][j]  (dense output edge), or C[s][j]
// (identity), accumulated in fp64.
__global__ void chat_kernel(const double* C, int S, int d_out, const float* W, int d_in, int kind,
                            float* chat, int ld) {
  int s = blockIdx.y;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d_in) return;
  double acc = 0.0;
  if (kind == 2) {
    acc = C[(size_t)s * d_out + j];
  } else {
    for (int o = 0; o < d_out; ++o) acc += C[(size_t)s * d_out + o] * (double)W[(size_t)o * d_in + j];
  }
  chat[(size_t)s * ld + j] = (float)acc;
}

hipError_t launch_chat(const double* C, int S, int d_out, const float* W, int d_in, int kind, float* chat,
                       int ld, hipStream_t st) {
  dim3 grid((d_in + 255) / 256, S);
  hipLaunchKernelGGL(chat_kernel, grid, dim3(256), 0, st, C, S, d_out, W, d_in, kind, chat, ld);
  return hipGetLastError();
}

__global__ void out_const_kernel(const double* C, int S, int d_out, const float* bias, double* cb) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double acc = 0.0;
  for (int o = 0; o < d_out; ++o) acc += C[(size_t)s * d_out + o] * (double)bias[o];
  cb[s] = acc;
}

// Lambda of the output node materialised: row r = C[r mod S] in the operand
// type (for outputs whose in-edges the c-hat shortcut cannot take).
template <typename T>
__global__ void __launch_bounds__(256) spec_rows_kernel(const double* C, int S, int d, int M, int nblk, T* out,
                                                        int ld) {
  const long b = blockIdx.x;
  const int r = (int)(b / nblk);
  const int j = (int)(b % nblk) * 256 + threadIdx.x;
  if (r < M && j < d) out[(size_t)r * ld + j] = to_t<T>((float)C[(size_t)(r % S) * d + j]);
}

hipError_t launch_spec_rows(int bf16_mode, const double* C, int S, int d, int M, void* out, int ld, hipStream_t st) {
  if (M <= 0 || d <= 0) return hipSuccess;
  const int nblk = (d + 255) / 256;
  const long blocks = (long)M * nblk;
  if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
  if (bf16_mode)
    hipLaunchKernelGGL(spec_rows_kernel<bf16>, dim3((unsigned)blocks), dim3(256), 0, st, C, S, d, M, nblk, (bf16*)out, ld);
  else
    hipLaunchKernelGGL(spec_rows_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, C, S, d, M, nblk, (float*)out,
                       ld);
  return hipGetLastError();
}

hipError_t launch_out_const(const double* C, int S, int d_out, const float* bias, double* cb, hipStream_t st) {
  hipLaunchKernelGGL(out_const_kernel, dim3((S + 63) / 64), dim3(64), 0, st, C, S, d_out, bias, cb);
  return hipGetLastError();
}

// out[j] = (bias ? bias[j] : out[j]) + (A x0)_j for an edge from the network
// input, fp64 sums; one wave per output, lanes stride over the inputs.
__global__ void __launch_bounds__(256) wx0_kernel(ConvGeom cg, int kind, const float* W, int d_out, int d_in,
                                                  const double* x0, const float* bias, float* out) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= d_out) return;
  double acc = 0.0;
  if (kind == 0) {
    for (int k = lane; k < d_in; k += 64) acc += (double)W[(size_t)j * d_in + k] * x0[k];
  } else if (kind == 1) {
    const int o = j / (cg.ho * cg.wo), y = (j / cg.wo) % cg.ho, x = j % cg.wo;
    const int taps = cg.ci * cg.kh * cg.kw;
    for (int t = lane; t < taps; t += 64) {
      const int c = t / (cg.kh * cg.kw), ky = (t / cg.kw) % cg.kh, kx = t % cg.kw;
      const int iy = y * cg.stride - cg.pad + ky, ix = x * cg.stride - cg.pad + kx;
      if (iy < 0 || iy >= cg.hi || ix < 0 || ix >= cg.wi) continue;
      acc += (double)W[((size_t)(o * cg.ci + c) * cg.kh + ky) * cg.kw + kx] * x0[(c * cg.hi + iy) * cg.wi + ix];
    }
  } else if (lane == 0) {
    acc = x0[j];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) out[j] = (float)((bias ? (double)bias[j] : (double)out[j]) + acc);
}

hipError_t launch_wx0(const ConvGeom* cg, int kind, const float* W, int d_out, int d_in, const double* x0,
                      const float* bias, float* out, hipStream_t st) {
  ConvGeom g = cg ? *cg : ConvGeom{};
  hipLaunchKernelGGL(wx0_kernel, dim3((d_out + 3) / 4), dim3(256), 0, st, g, kind, W, d_out, d_in, x0, bias, out);
  return hipGetLastError();
}

// bound[r] = sum_slots partial[slot][r] + c_s.b_out - gamma_r.d.  A block
// takes kRedRows rows; each row's slots and cuts are split over kRedParts
// threads (every kRedParts-th one, coalesced over rows) whose sums are
// combined in a fixed order, so the result is deterministic.
constexpr int kRedRows = 32, kRedParts = 8;
__global__ void __launch_bounds__(256) reduce_rows_kernel(int M, int mp, int S, const double* partial, int n_slots,
                                                          const double* cb, const float* gammaT, int N,
                                                          const double* d, double* bound, uint8_t* verified) {
  __shared__ double sh[kRedParts][kRedRows];
  const int rl = threadIdx.x % kRedRows, part = threadIdx.x / kRedRows;
  const int r = blockIdx.x * kRedRows + rl;
  double s = 0.0;
  if (r < M) {
    for (int k = part; k < n_slots; k += kRedParts) s += partial[(size_t)k * mp + r];
    for (int k = part; k < N; k += kRedParts) s -= (double)gammaT[(size_t)k * mp + r] * d[k];
  }
  sh[part][rl] = s;
  __syncthreads();
  if (part == 0 && r < M) {
    double t = 0.0;
#pragma unroll
    for (int p = 0; p < kRedParts; ++p) t += sh[p][rl];
    const double b = t + cb[r % S];
    bound[r] = b;
    if (verified) verified[r] = (b >= 0.0) ? 1 : 0;
  }
}

hipError_t launch_reduce_rows(int M, int mp, int S, const double* partial, int n_slots, const double* cb,
                              const float* gammaT, int N, const double* d, double* bound, uint8_t* verified,
                              hipStream_t st) {
  static_assert(kRedRows * kRedParts == 256, "one 256-thread block");
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_rows_kernel, dim3((M + kRedRows - 1) / kRedRows), dim3(256), 0, st, M, mp, S, partial,
                     n_slots, cb, gammaT, N, d, bound, verified);
  return hipGetLastError();
}

// ------------------------------------------------------------------ outward rounding
// X_in = max_j |x0_j| + eps, by one block (fixed reduction order).
__device__ inline double block_xin(const double* x0, int d_in, double eps, double* sh) {
  double m = 0.0;
  for (int j = threadIdx.x; j < d_in; j += blockDim.x) m = fmax(m, fabs(x0[j]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = fmax(t, sh[w]);
  __syncthreads();
  return t + eps;
}

// wcomb[off + k] = w0 + c_sum w1 + c_zb w2 + X_in (w3 + c_in w4) for the
// node blockIdx.y (0 beyond its size), wcomb[total] = X_in.
__global__ void __launch_bounds__(256) slack_weights_kernel(SlackArgs a) {
  __shared__ double sh[4];
  const double xin = block_xin(a.x0, a.d_in, a.eps, sh);
  const SlackNode& n = a.nodes[blockIdx.y];
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) a.wcomb[a.total] = xin;
  if (k >= n.ld) return;
  double w = 0.0;
  if (k < n.size) {
    const double* v = n.w;
    w = v[k] + a.c_sum * v[n.ld + k] + a.c_zb * v[2 * n.ld + k] + xin * (v[3 * n.ld + k] + a.c_in * v[4 * n.ld + k]);
  }
  a.wcomb[n.off + k] = w;
}

template <typename T>
__device__ inline double abs_dot(const T* lam, const double* w, int size, int lane) {
  double s = 0.0;
  for (int k = lane; k < size; k += 64) s += fabs((double)from_t<T>(lam[k])) * w[k];
  return s;
}

// One wave per row: the row's slack (sum |Lambda| w over its nodes, the
// spec-row term, |beta| and |gamma| terms), written negated into its
// partial slot.  Lanes stride over the neurons; the wave's sum is combined
// in a fixed order.
__global__ void __launch_bounds__(256) slack_rows_kernel(SlackArgs a) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= a.M) return;
  const double xin = a.wcomb[a.total];
  const int s = r % a.S, b = r / a.S;
  double acc = 0.0;
  for (int i = 0; i < a.n_nodes; ++i) {
    const SlackNode& n = a.nodes[i];
    if (!n.lam) continue;
    const double* w = a.wcomb + n.off;
    if (a.bf16) acc += abs_dot((const bf16*)n.lam + (size_t)r * n.ld, w, n.size, lane);
    else acc += abs_dot((const float*)n.lam + (size_t)r * n.ld, w, n.size, lane);
  }
  const double* Cs = a.C + (size_t)s * a.d_out;
  bool bad = false;
  for (int k = lane; k < a.d_out; k += 64) {
    const double c = Cs[k];
    if (a.out_chat) acc += fabs(c) * a.wcomb[a.out_off + k];
    else {   // the materialised output Lambda must be C itself
      const double held = a.bf16 ? (double)(float)to_t<bf16>((float)c) : (double)(float)c;
      bad |= held != c;
    }
  }
  for (int k = lane; k < a.K; k += 64)
    acc += a.c_beta * fabs((double)a.beta[(size_t)r * a.K + k]) * a.zsplit[(size_t)b * a.K + k];
  for (int c = lane; c < a.N; c += 64) {
    const double g = fabs((double)a.gammaT[(size_t)c * a.mp + r]);
    acc += g * (a.c_cut * (a.kap[c] + xin * a.kap[a.N + c]) + a.c_d * a.kap[2 * a.N + c]);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  bad = __any(bad);
  if (lane == 0) a.out[r] = bad ? -INFINITY : -(acc * (1.0 + 0x1p-40));
}

hipError_t launch_slack(const SlackArgs& a, hipStream_t st) {
  if (a.M <= 0) return hipSuccess;
  if (a.n_nodes <= 0 || a.n_nodes > kSlackMaxNodes) return hipErrorInvalidValue;
  int ldmax = 1;
  for (int i = 0; i < a.n_nodes; ++i) ldmax = ldmax > a.nodes[i].ld ? ldmax : a.nodes[i].ld;
  hipLaunchKernelGGL(slack_weights_kernel, dim3((ldmax + 255) / 256, a.n_nodes), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(slack_rows_kernel, dim3((a.M + 3) / 4), dim3(256), 0, st, a);
  return hipGetLastError();
}

// d bound / d gamma[r][k] = -d_k + sum of the cut's entry pieces (entries of
// cut k are contiguous in the cut-major order); then the Adam ascent step on
// gammaT (gamma >= 0, moments [N][M]) or the raw gradient into d_gamma[M][N].
// Thread per (k, r), rows fastest.
__global__ void __launch_bounds__(256) gamma_kernel(int M, int mp, int N, const int32_t* row_ptr,
                                                    const float* contrib, const double* d, float* gammaT,
                                                    float* d_gamma, float* m, float* v, AdamArgs adam) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= M) return;
  gamma_one(k, r, M, mp, N, row_ptr, contrib, d, gammaT, d_gamma, m, v, adam);
}

// Grouped gamma update: block b of job p covers rows 256 * (b % nr) .. of cut
// b / nr, nr = ceil(M / 256); same arithmetic as gamma_kernel.
__global__ void __launch_bounds__(256) gamma_grouped(const GammaJob* __restrict__ jobs, const int* __restrict__ prefix,
                                                     int np, AdamArgs adam) {
  const int t = blockIdx.x;
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const GammaJob jb = jobs[lo];
  const int nr = (jb.M + 255) / 256;
  const int b = t - prefix[lo];
  const int k = b / nr;
  const int r = (b % nr) * 256 + threadIdx.x;
  if (r >= jb.M) return;
  gamma_one(k, r, jb.M, jb.mp, jb.N, jb.row_ptr, jb.contrib, jb.d, jb.gammaT, nullptr, jb.m, jb.v, adam);
}

hipError_t launch_gamma_grouped(const GammaJob* d_jobs, const int* d_prefix, int np, int total_blocks, AdamArgs adam,
                                hipStream_t st) {
  if (total_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(gamma_grouped, dim3(total_blocks), dim3(256), 0, st, d_jobs, d_prefix, np, adam);
  return hipGetLastError();
}

hipError_t launch_gamma_update(int M, int mp, int N, const int32_t* row_ptr, const float* contrib, const double* d,
                               float* gammaT, float* d_gamma, float* m, float* v, AdamArgs adam, hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  dim3 grid((M + 255) / 256, N);
  hipLaunchKernelGGL(gamma_kernel, grid, dim3(256), 0, st, M, mp, N, row_ptr, contrib, d, gammaT, d_gamma, m, v,
                     adam);
  return hipGetLastError();
}

// [rows][cols] (pitch ld_in) -> [cols][ld_out], 32x32 tiles through LDS
__global__ void __launch_bounds__(256) transpose_kernel(const float* in, int rows, int cols, int ld_in, float* out,
                                                        int ld_out) {
  __shared__ float t[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int r = r0 + y, c = c0 + tx;
    t[y][tx] = (r < rows && c < cols) ? in[(size_t)r * ld_in + c] : 0.f;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int c = c0 + y, r = r0 + tx;
    if (c < cols && r < rows) out[(size_t)c * ld_out + r] = t[tx][y];
  }
}

hipError_t launch_transpose(const float* in, int rows, int cols, int ld_in, float* out, int ld_out, hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  dim3 grid((cols + 31) / 32, (rows + 31) / 32);
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, st, in, rows, cols, ld_in, out, ld_out);
  return hipGetLastError();
}

// Per-iteration Adam constants from the device step counter t, then t += 1;
// with reset the counter is only set to 0.  consts = {lr_a decay^t, lr_m decay^t, 1-b1^(t+1), 1-b2^(t+1)}.
// Adam constants of iteration t: learning rates lr * decay^t and the
// reciprocal bias corrections 1/(1 - b^(t+1)).  One function for the
// per-call table and the per-iteration kernel, so both give the same bits.
__device__ inline void adam_consts(int t, float lr_alpha, float lr_mult, float decay, float b1, float b2,
                                   float* out) {
  double dec = pow((double)decay, (double)t);
  out[0] = (float)(lr_alpha * dec);
  out[1] = (float)(lr_mult * dec);
  out[2] = (float)(1.0 / (1.0 - pow((double)b1, (double)(t + 1))));
  out[3] = (float)(1.0 / (1.0 - pow((double)b2, (double)(t + 1))));
}
__global__ void adam_prepare_kernel(int* step, int reset, float lr_alpha, float lr_mult, float decay, float b1,
                                    float b2, float* consts) {
  if (threadIdx.x != 0) return;
  if (reset) {            // set the step counter to reset - 1, no constants written
    *step = reset - 1;
    return;
  }
  int t = *step;
  adam_consts(t, lr_alpha, lr_mult, decay, b1, b2, consts);
  *step = t + 1;
}
__global__ void adam_table_kernel(float* tab, int iters, float lr_alpha, float lr_mult, float decay, float b1,
                                  float b2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < iters) adam_consts(t, lr_alpha, lr_mult, decay, b1, b2, tab + 4 * t);
}
hipError_t launch_adam_table(float* tab, int iters, float lr_alpha, float lr_mult, float decay, float b1, float b2,
                             hipStream_t st) {
  if (iters <= 0) return hipSuccess;
  hipLaunchKernelGGL(adam_table_kernel, dim3((iters + 63) / 64), dim3(64), 0, st, tab, iters, lr_alpha, lr_mult,
                     decay, b1, b2);
  return hipGetLastError();
}
hipError_t launch_adam_prepare(int* step, int reset, float lr_alpha, float lr_mult, float decay, float b1,
                               float b2, float* consts, hipStream_t st) {
  if (step == nullptr || (!reset && consts == nullptr)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(adam_prepare_kernel, dim3(1), dim3(64), 0, st, step, reset, lr_alpha, lr_mult, decay, b1,
                     b2, consts);
  return hipGetLastError();
}

__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// dst[dst_row[i]][j] = src[src_row[i]][j] (0 where j == zero_col[i]), j < L
__global__ void __launch_bounds__(256) copy_rows_kernel(float* dst, int64_t ld_dst, const int32_t* dst_row,
                                                        const float* src, int64_t ld_src, const int32_t* src_row,
                                                        int L, const int32_t* zero_col) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= L) return;
  const float v = src[(int64_t)src_row[i] * ld_src + j];
  dst[(int64_t)dst_row[i] * ld_dst + j] = (zero_col && zero_col[i] == j) ? 0.f : v;
}
hipError_t launch_copy_rows(float* dst, int64_t ld_dst, const int32_t* dst_row, const float* src, int64_t ld_src,
                            const int32_t* src_row, int n, int L, const int32_t* zero_col, hipStream_t st) {
  if (n <= 0 || L <= 0) return hipSuccess;
  if (n > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_rows_kernel, dim3((L + 255) / 256, n), dim3(256), 0, st, dst, ld_dst, dst_row, src, ld_src,
                     src_row, L, zero_col);
  return hipGetLastError();
}

// flags[0] |= 1 if any value is not finite, |= 2 if outside [lo, hi]
__global__ void validate_kernel(const float* p, int64_t n, float lo, float hi, int* flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int f = 0;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float x = p[i];
    if (!isfinite(x)) f |= 1;
    else if (x < lo || x > hi) f |= 2;
  }
  if (f) atomicOr(flags, f);
}
hipError_t launch_validate(const float* p, int64_t n, float lo, float hi, int* flags, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(validate_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, lo, hi, flags);
  return hipGetLastError();
}

__global__ void f32_to_bf16_kernel(const float* src, bf16* dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (bf16)src[i];
}
hipError_t launch_fill_bf16_from_f32(const float* src, bf16* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace gcp
