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

#include <hip/hip_runtime.h>
#include <math.h>

namespace gcp {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ MFMA
template <typename T> struct Op;
template <> struct Op<float> {
  static constexpr int VEC = 4;    // elements per 16-byte fragment
  static constexpr int KC = 16;    // K covered by one fragment per 4 lane groups
  __device__ static inline void mma(const uint4& a, const uint4& b, f4& c) {
    // Lane (row i = lane%16, group g = lane/16) holds A[i][4g..4g+3]; step t
    // feeds element t, so the four steps cover k = 4g + t for all g, t.
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
  }
};
template <> struct Op<bf16> {
  static constexpr int VEC = 8;
  static constexpr int KC = 32;
  __device__ static inline void mma(const uint4& a, const uint4& b, f4& c) {
    bf16x8 av = __builtin_bit_cast(bf16x8, a);
    bf16x8 bv = __builtin_bit_cast(bf16x8, b);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
};

template <typename T> __device__ inline T to_t(float x);
template <> __device__ inline float to_t<float>(float x) { return x; }
template <> __device__ inline bf16 to_t<bf16>(float x) { return (bf16)x; }

// ------------------------------------------------------------------ helpers
__device__ inline double wave_sum16(double v) {
  // sum over the 16 lanes that share lane/16 (lane bits 0..3)
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 8, 64);
  return v;
}

struct AdamStep {
  float lr_a, lr_m, b1, b2, eps, bc1, bc2;
  // consts = {lr_alpha * decay^t, lr_mult * decay^t, 1 - b1^(t+1), 1 - b2^(t+1)},
  // prepared on the device once per iteration (adam_prepare_kernel).
  __device__ AdamStep(const AdamArgs& a) {
    lr_a = a.consts[0]; lr_m = a.consts[1]; bc1 = a.consts[2]; bc2 = a.consts[3];
    b1 = a.b1; b2 = a.b2; eps = a.eps;
  }
  // Ascent step on x with gradient g, then projection onto [lo, hi].
  __device__ inline void update(float* x, float* m, float* v, float g, float lr, float lo,
                                float hi) const {
    float mm = b1 * (*m) + (1.0f - b1) * g;
    float vv = b2 * (*v) + (1.0f - b2) * g * g;
    *m = mm;
    *v = vv;
    float step = lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    *x = fminf(fmaxf(*x + step, lo), hi);
  }
};

// Split override of one (row, neuron): returns the effective class and the
// split slot (or -1).
__device__ inline int split_of(const RowParams& rp, int r, int rank, int cls, int* slot) {
  *slot = -1;
  if (rank < 0 || rp.mask == nullptr) return cls;
  int m = rp.mask[(size_t)(r / rp.S) * rp.n_I + rank];
  if (m > 0) { *slot = m - 1; return ACTIVE; }
  if (m < 0) { *slot = -m - 1; return INACTIVE; }
  return cls;
}

// ------------------------------------------------------------------ epilogues
// Each returns the element's contribution to its row's constant (fp64).

template <typename T>
struct BoundEpi {
  BoundEpiArgs a;
  __device__ inline double operator()(int r, int j, float acc) const {
    const NodeDev& nd = a.nd;
    const RowParams& rp = a.rp;
    size_t ij = (size_t)r * nd.ld + j;
    float ah = acc;
    if (a.acc_in) ah += a.acc_in[ij];
    float sG = 0.f, sH = 0.f, sQ = 0.f;
    if (a.cc.col_ptr) {
      int e0 = a.cc.col_ptr[j], e1 = a.cc.col_ptr[j + 1];
      const float* gr = rp.gamma + (size_t)r * rp.N;
      for (int e = e0; e < e1; ++e) {
        float g = gr[a.cc.cut[e]];
        sG += g * a.cc.cG[e];
        sH += g * a.cc.cH[e];
        sQ += g * a.cc.cQ[e];
      }
    }
    ah += sG;                      // a_hat = Lambda^(i+1) W + gamma^T G
    int rank = nd.rank[j];
    int slot;
    int c = split_of(rp, r, rank, nd.cls[j], &slot);
    float bterm = 0.f;
    if (slot >= 0) {
      float bv = rp.beta[(size_t)r * rp.K + slot];
      bterm = (c == ACTIVE) ? -bv : bv;
    }
    float lam, konst;
    if (c == ACTIVE) {             // x_hat = x, z = 1
      lam = ah + sH + bterm;
      konst = sQ;
    } else if (c == INACTIVE) {    // x_hat = 0, z = 0
      lam = sH + bterm;
      konst = 0.f;
    } else {                       // Lemma A.1 with C = [-a_hat]_+, q = -s
      float n = fmaxf(-ah, 0.f), p = fmaxf(ah, 0.f);
      float uu = nd.u[j], ll = nd.l[j];
      float pi, h;
      if (sQ >= uu * n) { pi = 0.f; h = 0.f; }
      else if (sQ <= ll * n) { pi = n; h = sQ; }
      else { pi = (uu * n - sQ) * nd.inv_ul[j]; h = ll * pi; }
      lam = rp.alpha[(size_t)r * rp.n_I + rank] * p - pi + sH;
      konst = h;
    }
    ((T*)a.lam_out)[ij] = to_t<T>(lam);
    if (a.ahat_out) a.ahat_out[ij] = ah;
    return (double)lam * (double)nd.bias[j] + (double)konst;
  }
};

struct ConcEpi {
  ConcEpiArgs a;
  __device__ inline double operator()(int r, int j, float acc) const {
    float v = acc;
    if (a.cc.col_ptr) {
      const float* gr = a.rp.gamma + (size_t)a.rp.N * r;
      for (int e = a.cc.col_ptr[j]; e < a.cc.col_ptr[j + 1]; ++e) v += gr[a.cc.cut[e]] * a.cc.cG[e];
    }
    float sg = (v > 0.f) ? 1.f : ((v < 0.f) ? -1.f : 0.f);
    if (a.sign_out) a.sign_out[(size_t)r * a.ld + j] = (int8_t)sg;
    if (a.contrib && a.cc.col_ptr) {
      float dv = (float)(a.x0[j] - a.eps * (double)sg);
      for (int e = a.cc.col_ptr[j]; e < a.cc.col_ptr[j + 1]; ++e)
        a.contrib[(size_t)r * a.nnz_e + a.cc.pos[e]] = a.cc.cG[e] * dv;
    }
    double vd = (double)v;
    return a.x0[j] * vd - a.eps * fabs(vd);
  }
};

template <typename T>
struct AdjEpi {
  AdjEpiArgs a;
  __device__ inline double operator()(int r, int j, float acc) const {
    const NodeDev& nd = a.nd;
    const RowParams& rp = a.rp;
    size_t ij = (size_t)r * nd.ld + j;
    float dL = a.gemm_scale * acc + a.add_vec[j];
    if (a.acc_in) dL += a.acc_in[ij];
    float ah = a.ahat[ij];
    float sQ = 0.f;
    const float* gr = rp.gamma + (size_t)r * rp.N;
    int e0 = 0, e1 = 0;
    if (a.cc.col_ptr) {
      e0 = a.cc.col_ptr[j];
      e1 = a.cc.col_ptr[j + 1];
      for (int e = e0; e < e1; ++e) sQ += gr[a.cc.cut[e]] * a.cc.cQ[e];
    }
    int rank = nd.rank[j];
    int slot;
    int c = split_of(rp, r, rank, nd.cls[j], &slot);
    float dA, dS, gA = 0.f;
    if (c == ACTIVE) {
      dA = dL; dS = 1.f;
    } else if (c == INACTIVE) {
      dA = 0.f; dS = 0.f;
    } else {
      float n = fmaxf(-ah, 0.f), p = fmaxf(ah, 0.f);
      float pos = ah > 0.f ? 1.f : 0.f, neg = ah < 0.f ? 1.f : 0.f;
      float uu = nd.u[j], ll = nd.l[j], iul = nd.inv_ul[j];
      float al = rp.alpha[(size_t)r * rp.n_I + rank];
      float dLda, dhda, dLds, dhds;
      if (sQ >= uu * n) { dLda = al * pos; dhda = 0.f; dLds = 0.f; dhds = 0.f; }
      else if (sQ <= ll * n) { dLda = al * pos + neg; dhda = 0.f; dLds = 0.f; dhds = 1.f; }
      else {
        dLda = al * pos + uu * iul * neg;
        dhda = -ll * uu * iul * neg;
        dLds = iul;
        dhds = -ll * iul;
      }
      dA = dL * dLda + dhda;
      dS = dL * dLds + dhds;
      gA = dL * p;
    }
    if (a.dahat_out) ((T*)a.dahat_out)[ij] = to_t<T>(dA);
    if (a.contrib) {
      for (int e = e0; e < e1; ++e)
        a.contrib[(size_t)r * a.nnz_e + a.cc.pos[e]] = a.cc.cG[e] * dA + a.cc.cH[e] * dL + a.cc.cQ[e] * dS;
    }
    if (rank >= 0) {
      size_t ia = (size_t)r * rp.n_I + rank;
      if (a.adam.enabled) {
        AdamStep st(a.adam);
        st.update(a.alpha_rw + ia, a.m_alpha + ia, a.v_alpha + ia, gA, st.lr_a, 0.f, 1.f);
      } else {
        a.d_alpha[ia] = gA;
      }
    }
    if (slot >= 0) {
      size_t ib = (size_t)r * rp.K + slot;
      float gB = (c == ACTIVE) ? -dL : dL;
      if (a.adam.enabled) {
        AdamStep st(a.adam);
        st.update(a.beta_rw + ib, a.m_beta + ib, a.v_beta + ib, gB, st.lr_m, 0.f, INFINITY);
      } else {
        a.d_beta[ib] = gB;
      }
    }
    return 0.0;
  }
};

struct StoreEpi {
  StoreEpiArgs a;
  __device__ inline double operator()(int r, int j, float acc) const {
    size_t ij = (size_t)r * a.ld + j;
    float v = a.scale * acc;
    if (a.acc_in) v += a.acc_in[ij];
    a.out[ij] = v;
    return 0.0;
  }
};

// ------------------------------------------------------------------ tile GEMM
// C[M][N] = A[M][K] * Bt[N][K]^T on MFMA, epilogue per element, row partial
// sums reduced deterministically (lanes, then waves through LDS) into
// partial[r][slot0 + blockIdx.x].
template <typename T, int BM, int BN, int WM, int WN, int BK, bool SIGN, class Epi>
__global__ void __launch_bounds__(WM * WN * 64)
gemm_epi_kernel(GemmArgs g, Epi epi) {
  constexpr int NT = WM * WN * 64;
  constexpr int VEC = Op<T>::VEC;
  constexpr int KC = Op<T>::KC;
  constexpr int LDS_LD = BK + VEC;          // 16-byte row padding
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int AV = BM * BK / VEC;         // 16-byte vectors per A stage
  constexpr int BV = BN * BK / VEC;
  constexpr int AIT = (AV + NT - 1) / NT;
  constexpr int BIT = (BV + NT - 1) / NT;
  static_assert(BK % KC == 0, "BK must be a multiple of the fragment K");

  __shared__ __attribute__((aligned(16))) T As[BM * LDS_LD];
  __shared__ __attribute__((aligned(16))) T Bs[BN * LDS_LD];
  __shared__ double red[WN][BM];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int k = 0; k < TN; ++k) acc[i][k] = f4{0.f, 0.f, 0.f, 0.f};

  uint4 ra[AIT], rb[BIT];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      int v = tid + it * NT;
      uint4 val = {0u, 0u, 0u, 0u};
      if (v < AV) {
        int row = v / (BK / VEC), kk = (v % (BK / VEC)) * VEC;
        int gr = m0 + row, gk = k0 + kk;
        if (gr < g.M && gk < g.lda) {
          if constexpr (SIGN) {
            const int8_t* src = (const int8_t*)g.A + (size_t)gr * g.lda + gk;
            T tmp[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) tmp[q] = to_t<T>((float)src[q]);
            val = *(const uint4*)tmp;
          } else {
            val = *(const uint4*)((const T*)g.A + (size_t)gr * g.lda + gk);
          }
        }
      }
      ra[it] = val;
    }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      int v = tid + it * NT;
      uint4 val = {0u, 0u, 0u, 0u};
      if (v < BV) {
        int row = v / (BK / VEC), kk = (v % (BK / VEC)) * VEC;
        int gn = n0 + row, gk = k0 + kk;
        if (gn < g.N && gk < g.ldb) val = *(const uint4*)((const T*)g.Bt + (size_t)gn * g.ldb + gk);
      }
      rb[it] = val;
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      int v = tid + it * NT;
      if (v < AV) {
        int row = v / (BK / VEC), kk = (v % (BK / VEC)) * VEC;
        *(uint4*)(As + row * LDS_LD + kk) = ra[it];
      }
    }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      int v = tid + it * NT;
      if (v < BV) {
        int row = v / (BK / VEC), kk = (v % (BK / VEC)) * VEC;
        *(uint4*)(Bs + row * LDS_LD + kk) = rb[it];
      }
    }
  };

  const int arow = wm * (BM / WM) + (lane & 15);
  const int bcol = wn * (BN / WN) + (lane & 15);
  const int kq = (lane >> 4) * VEC;

  if (g.K > 0) load_stage(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    __syncthreads();
    store_stage();
    __syncthreads();
    if (k0 + BK < g.K) load_stage(k0 + BK);
#pragma unroll
    for (int kc = 0; kc < BK; kc += KC) {
      uint4 fa[TM], fb[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) fa[i] = *(const uint4*)(As + (arow + i * 16) * LDS_LD + kc + kq);
#pragma unroll
      for (int k = 0; k < TN; ++k) fb[k] = *(const uint4*)(Bs + (bcol + k * 16) * LDS_LD + kc + kq);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int k = 0; k < TN; ++k) Op<T>::mma(fa[i], fb[k], acc[i][k]);
    }
  }

  // Epilogue: lane holds rows 4*(lane/16)+v, column lane%16 of each 16x16 tile.
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int rl = wm * (BM / WM) + i * 16 + (lane >> 4) * 4 + v;
      int r = m0 + rl;
      double rs = 0.0;
#pragma unroll
      for (int k = 0; k < TN; ++k) {
        int j = n0 + wn * (BN / WN) + k * 16 + (lane & 15);
        if (r < g.M && j < g.N) rs += epi(r, j, acc[i][k][v]);
      }
      rs = wave_sum16(rs);
      if ((lane & 15) == 0) red[wn][rl] = rs;
    }
  }
  if (g.partial) {
    __syncthreads();
    for (int rl = tid; rl < BM; rl += NT) {
      int r = m0 + rl;
      if (r < g.M) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WN; ++w) s += red[w][rl];
        g.partial[(size_t)r * g.n_slots + g.slot0 + blockIdx.x] = s;
      }
    }
  }
}

// Tile configurations available to the autotuner: (BM, BN, WM, WN).
struct TileCfg { int bm, bn; };
static const TileCfg kCfgs[] = {{64, 64}, {128, 64}, {64, 128}, {128, 128}, {32, 64}};
int gemm_num_configs() { return (int)(sizeof(kCfgs) / sizeof(kCfgs[0])); }
void gemm_config_tile(int cfg, int* bm, int* bn) { *bm = kCfgs[cfg].bm; *bn = kCfgs[cfg].bn; }

template <typename T, int BM, int BN, int WM, int WN, bool SIGN, class Epi>
static hipError_t launch_cfg(const GemmArgs& g, const Epi& epi, hipStream_t st) {
  constexpr int BK = (sizeof(T) == 4) ? 32 : 64;
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM);
  hipLaunchKernelGGL((gemm_epi_kernel<T, BM, BN, WM, WN, BK, SIGN, Epi>), grid, dim3(WM * WN * 64), 0, st,
                     g, epi);
  return hipGetLastError();
}

template <typename T, bool SIGN, class Epi>
static hipError_t launch_any(int cfg, const GemmArgs& g, const Epi& epi, hipStream_t st) {
  switch (cfg) {
    case 0: return launch_cfg<T, 64, 64, 2, 2, SIGN>(g, epi, st);
    case 1: return launch_cfg<T, 128, 64, 2, 2, SIGN>(g, epi, st);
    case 2: return launch_cfg<T, 64, 128, 2, 2, SIGN>(g, epi, st);
    case 3: return launch_cfg<T, 128, 128, 2, 2, SIGN>(g, epi, st);
    case 4: return launch_cfg<T, 32, 64, 1, 2, SIGN>(g, epi, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_typed(int cfg, EpiKind kind, const GemmArgs& g, const void* epi, hipStream_t st) {
  switch (kind) {
    case EPI_BOUND: return launch_any<T, false>(cfg, g, BoundEpi<T>{*(const BoundEpiArgs*)epi}, st);
    case EPI_CONC: return launch_any<T, false>(cfg, g, ConcEpi{*(const ConcEpiArgs*)epi}, st);
    case EPI_STORE:
      if (g.a_is_sign) return launch_any<T, true>(cfg, g, StoreEpi{*(const StoreEpiArgs*)epi}, st);
      return launch_any<T, false>(cfg, g, StoreEpi{*(const StoreEpiArgs*)epi}, st);
    case EPI_ADJ:
      if (g.a_is_sign) return launch_any<T, true>(cfg, g, AdjEpi<T>{*(const AdjEpiArgs*)epi}, st);
      return launch_any<T, false>(cfg, g, AdjEpi<T>{*(const AdjEpiArgs*)epi}, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm(int bf16_mode, int cfg, EpiKind kind, const GemmArgs& g, const void* epi,
                       hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  return bf16_mode ? launch_typed<bf16>(cfg, kind, g, epi, st) : launch_typed<float>(cfg, kind, g, epi, st);
}

// ------------------------------------------------------------------ elementwise
// One block = one row x 256 columns; row partial per column block.
template <typename T>
__global__ void __launch_bounds__(256) bound_elem_kernel(const float* bcast, BoundEpiArgs a, double* partial,
                                                         int n_slots, int slot0) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  const int j = blockIdx.y * 256 + threadIdx.x;
  BoundEpi<T> epi{a};
  double rs = 0.0;
  if (j < a.nd.size) {
    float pre = bcast ? bcast[(size_t)(r % a.rp.S) * a.nd.ld + j] : 0.f;
    rs = epi(r, j, pre);
  }
  for (int o = 32; o > 0; o >>= 1) rs += __shfl_xor(rs, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rs;
  __syncthreads();
  if (threadIdx.x == 0 && partial)
    partial[(size_t)r * n_slots + slot0 + blockIdx.y] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_bound_elementwise(int bf16_mode, const float* bcast, const BoundEpiArgs& a,
                                          double* partial, int n_slots, int slot0, hipStream_t st) {
  dim3 grid(a.rp.M, (a.nd.size + 255) / 256);
  if (bf16_mode)
    hipLaunchKernelGGL(bound_elem_kernel<bf16>, grid, dim3(256), 0, st, bcast, a, partial, n_slots, slot0);
  else
    hipLaunchKernelGGL(bound_elem_kernel<float>, grid, dim3(256), 0, st, bcast, a, partial, n_slots, slot0);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) adj_elem_kernel(AdjEpiArgs a) {
  const int r = blockIdx.x;
  const int j = blockIdx.y * 256 + threadIdx.x;
  AdjEpi<T> epi{a};
  if (j < a.nd.size) epi(r, j, 0.f);
}

hipError_t launch_adj_elementwise(int bf16_mode, const AdjEpiArgs& a, hipStream_t st) {
  dim3 grid(a.rp.M, (a.nd.size + 255) / 256);
  if (bf16_mode)
    hipLaunchKernelGGL(adj_elem_kernel<bf16>, grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(adj_elem_kernel<float>, grid, dim3(256), 0, st, a);
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

hipError_t launch_out_const(const double* C, int S, int d_out, const float* bias, double* cb, hipStream_t st) {
  hipLaunchKernelGGL(out_const_kernel, dim3((S + 63) / 64), dim3(64), 0, st, C, S, d_out, bias, cb);
  return hipGetLastError();
}

// out[j] = bias[j] + (A x0)_j for an edge from the network input (fp64 sums).
__global__ void wx0_kernel(ConvGeom cg, int kind, const float* W, int d_out, int d_in, const double* x0,
                           const float* bias, float* out) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d_out) return;
  double acc = bias ? (double)bias[j] : 0.0;
  if (kind == 0) {
    for (int k = 0; k < d_in; ++k) acc += (double)W[(size_t)j * d_in + k] * x0[k];
  } else if (kind == 1) {
    int o = j / (cg.ho * cg.wo), y = (j / cg.wo) % cg.ho, x = j % cg.wo;
    for (int c = 0; c < cg.ci; ++c)
      for (int ky = 0; ky < cg.kh; ++ky) {
        int iy = y * cg.stride - cg.pad + ky;
        if (iy < 0 || iy >= cg.hi) continue;
        for (int kx = 0; kx < cg.kw; ++kx) {
          int ix = x * cg.stride - cg.pad + kx;
          if (ix < 0 || ix >= cg.wi) continue;
          acc += (double)W[((size_t)(o * cg.ci + c) * cg.kh + ky) * cg.kw + kx] * x0[(c * cg.hi + iy) * cg.wi + ix];
        }
      }
  } else {
    acc += x0[j];
  }
  out[j] = (float)acc;
}

hipError_t launch_wx0(const ConvGeom* cg, int kind, const float* W, int d_out, int d_in, const double* x0,
                      const float* bias, float* out, hipStream_t st) {
  ConvGeom g = cg ? *cg : ConvGeom{};
  hipLaunchKernelGGL(wx0_kernel, dim3((d_out + 255) / 256), dim3(256), 0, st, g, kind, W, d_out, d_in, x0, bias,
                     out);
  return hipGetLastError();
}

// bound[r] = sum_slots partial[r][.] + c_s.b_out - gamma_r.d   (one wave per row)
__global__ void __launch_bounds__(256) reduce_rows_kernel(int M, int S, const double* partial, int n_slots,
                                                          const double* cb, const float* gamma, int N,
                                                          const double* d, double* bound, uint8_t* verified) {
  int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (r >= M) return;
  double s = 0.0;
  for (int k = lane; k < n_slots; k += 64) s += partial[(size_t)r * n_slots + k];
  for (int k = lane; k < N; k += 64) s -= (double)gamma[(size_t)r * N + k] * d[k];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) {
    double b = s + cb[r % S];
    bound[r] = b;
    if (verified) verified[r] = (b >= 0.0) ? 1 : 0;
  }
}

hipError_t launch_reduce_rows(int M, int S, const double* partial, int n_slots, const double* cb,
                              const float* gamma, int N, const double* d, double* bound, uint8_t* verified,
                              hipStream_t st) {
  hipLaunchKernelGGL(reduce_rows_kernel, dim3((M + 3) / 4), dim3(256), 0, st, M, S, partial, n_slots, cb, gamma,
                     N, d, bound, verified);
  return hipGetLastError();
}

// d bound / d gamma[r][k] = -d_k + sum of the cut's entry contributions;
// then the Adam ascent step (gamma >= 0) or the raw gradient.
__global__ void __launch_bounds__(256) gamma_kernel(int M, int N, const int32_t* row_ptr, const float* contrib,
                                                    int nnz_e, const double* d, float* gamma, float* d_gamma,
                                                    float* m, float* v, AdamArgs adam) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)M * N) return;
  int r = (int)(idx / N), k = (int)(idx % N);
  double g = -d[k];
  const float* cr = contrib + (size_t)r * nnz_e;
  for (int e = row_ptr[k]; e < row_ptr[k + 1]; ++e) g += (double)cr[e];
  if (adam.enabled) {
    AdamStep st(adam);
    st.update(gamma + idx, m + idx, v + idx, (float)g, st.lr_m, 0.f, INFINITY);
  } else {
    d_gamma[idx] = (float)g;
  }
}

hipError_t launch_gamma_update(int M, int N, const int32_t* row_ptr, const float* contrib, int nnz_e,
                               const double* d, float* gamma, float* d_gamma, float* m, float* v, AdamArgs adam,
                               hipStream_t st) {
  size_t n = (size_t)M * N;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(gamma_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M, N, row_ptr, contrib,
                     nnz_e, d, gamma, d_gamma, m, v, adam);
  return hipGetLastError();
}

// Per-iteration Adam constants from the device step counter t, then t += 1;
// with reset the counter is only set to 0.  consts = {lr_a decay^t, lr_m decay^t, 1-b1^(t+1), 1-b2^(t+1)}.
__global__ void adam_prepare_kernel(int* step, int reset, float lr_alpha, float lr_mult, float decay, float b1,
                                    float b2, float* consts) {
  if (threadIdx.x != 0) return;
  if (reset) {            // start of an optimisation: t = 0, no constants written
    *step = 0;
    return;
  }
  int t = *step;
  double dec = pow((double)decay, (double)t);
  consts[0] = (float)(lr_alpha * dec);
  consts[1] = (float)(lr_mult * dec);
  consts[2] = (float)(1.0 - pow((double)b1, (double)(t + 1)));
  consts[3] = (float)(1.0 - pow((double)b2, (double)(t + 1)));
  *step = t + 1;
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
