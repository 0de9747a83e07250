// Fused optimisation of dense ReLU chains (arXiv 2208.05740: Theorem 3.1's
// bound with Lemma A.1, its adjoint, and the projected Adam ascent of
// Appendix C.1), all iterations in one launch.
//
// Rows are independent scalar problems, so a workgroup owns kChainRows rows
// for the whole optimisation: every iteration it walks the chain down (the
// output's c-hat relaxation, then one MFMA GEMM + relaxation per layer, then
// the concretisation), back up (one GEMM + relaxation adjoint + Adam step per
// layer) and finishes with the multiplier update of its rows.  The A operand
// of every GEMM (Lambda, sign(v), d a_hat of the 16 rows) lives in LDS and
// the weights stream from L2, so per iteration only the optimiser state (alpha
// and its moments, multipliers, split mask), a_hat (stored for the adjoint)
// and the cut-gradient pieces touch memory.  The per-element arithmetic is the
// per-layer kernels' own (the same epilogue code, and each GEMM accumulates
// over K in the same order with the same MFMA instructions), so the result is
// bit for bit that of the per-layer launches.
#include "gcp_internal.h"
#include "epilogues.h"

#include <hip/hip_runtime.h>

#include <cstdlib>

namespace gcp {

// acc[k] += A x Bt^T for the lane's fragment: A = 16 rows in LDS (operand type
// at byte offset a_off with pitch a_ld elements, or int8 signs with pitch
// a_ld bytes when SIGN), Bt rows n0 + 16 k + lane % 16 in global memory.  K
// advances in the per-layer GEMM's order (Op<T>::KC per step, lane group g
// holding k = step + VEC g ..), with the B fragments of step s + D loaded
// while step s computes.
template <typename T, int TN, bool SIGN, int D>
__device__ inline void chain_mma(f4 (&acc)[TN], int a_off, int a_ld, const T* __restrict__ Bt, int ldb, int n0, int N,
                                 int K, int lane) {
  constexpr int VEC = Op<T>::VEC;
  constexpr int KC = Op<T>::KC;
  const int row = lane & 15;
  const int kq = (lane >> 4) * VEC;
  const T* bp[TN];
  bool bv[TN];
#pragma unroll
  for (int k = 0; k < TN; ++k) {
    const int col = n0 + 16 * k + row;
    bv[k] = col < N;
    bp[k] = Bt + (size_t)(bv[k] ? col : 0) * ldb + kq;
  }
  auto load_b = [&](uint4 (&b)[TN], int kc) {
    const int kk = kc + kq;
#pragma unroll
    for (int k = 0; k < TN; ++k) {
      uint4 v = {0u, 0u, 0u, 0u};
      if (bv[k] && kk < K) {
        v = *(const uint4*)(bp[k] + kc);
        if (kk + VEC > K) v = mask_tail<T>(v, K - kk);
      }
      b[k] = v;
    }
  };
  auto load_a = [&](int kc) {
    const int kk = kc + kq;
    uint4 v = {0u, 0u, 0u, 0u};
    if (kk < K) {
      if constexpr (SIGN) {
        const int8_t* src = (const int8_t*)(gcp_smem + a_off) + row * a_ld + kk;
        int8_t e[VEC];
        if constexpr (VEC == 8) *(uint2*)e = *(const uint2*)src;
        else *(uint32_t*)e = *(const uint32_t*)src;
        T tmp[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) tmp[q] = to_t<T>((float)e[q]);
        v = *(const uint4*)tmp;
      } else {
        v = *(const uint4*)(gcp_smem + a_off + (row * a_ld + kk) * (int)sizeof(T));
      }
      if (kk + VEC > K) v = mask_tail<T>(v, K - kk);
    }
    return v;
  };
  uint4 ring[D][TN];
#pragma unroll
  for (int d = 0; d < D; ++d) load_b(ring[d], d * KC);
  for (int kc = 0; kc < K; kc += D * KC) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int k0 = kc + d * KC;
      if (k0 < K) {
        const uint4 fa = load_a(k0);
#pragma unroll
        for (int k = 0; k < TN; ++k) Op<T>::mma(fa, ring[d][k], acc[k]);
        if (k0 + D * KC < K) load_b(ring[d], k0 + D * KC);
      }
    }
  }
}

// One GEMM layer of the chain for the workgroup's rows m0 .. m0 + 15: each
// wave takes TN column tiles of 16 at a time, accumulates over K and runs the
// epilogue on its fragment (the per-layer kernel's lane layout: rows
// 4 (lane / 16) + v, column lane % 16 of every tile), handing the produced
// activation to `sink`.
template <typename T, int NW, int TN, bool SIGN, int D, class Epi, class Sink>
__device__ inline void chain_layer(const Epi& epi, const Sink& sink, int m0, int M, int N, int K, int a_off, int a_ld,
                                   const T* Bt, int ldb) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int c0 = wave * TN * 16; c0 < N; c0 += NW * TN * 16) {
    LaneCoords<4, TN, false> lc;
    int mr = m0;
    asm volatile("" : "+s"(mr));   // row-derived addresses are formed per column chunk, not kept live across them
#pragma unroll
    for (int v = 0; v < 4; ++v) lc.r[v] = mr + 4 * (lane >> 4) + v;
#pragma unroll
    for (int k = 0; k < TN; ++k) lc.j[k][0] = c0 + 16 * k + (lane & 15);
    // the column's kind word and cut range go out before the K loop (the
    // loads the epilogue's rank- and cut-addressed loads wait on)
    ColPre<TN> pre;
    if constexpr (Epi::kColPre) {
      int col[TN];
#pragma unroll
      for (int k = 0; k < TN; ++k) col[k] = lc.j[k][0];
      col_prefetch<TN>(pre, epi.col_node(), epi.col_cuts(), col, N);
    }
    typename Epi::template Frag<4, TN, false> fr;
    if constexpr (Epi::kColPre) epi.template load<4, TN, false>(fr, lc, M, N, &pre);
    else epi.template load<4, TN, false>(fr, lc, M, N);
    f4 acc[TN];
#pragma unroll
    for (int k = 0; k < TN; ++k) acc[k] = f4{0.f, 0.f, 0.f, 0.f};
    chain_mma<T, TN, SIGN, D>(acc, a_off, a_ld, Bt, ldb, c0, N, K, lane);
    float val[TN][4];
#pragma unroll
    for (int k = 0; k < TN; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) val[k][v] = acc[k][v];
    double rs[4] = {0.0, 0.0, 0.0, 0.0};
    epi.template apply_to<4, TN, false>(fr, lc, val, rs, M, N, sink);
  }
}

// The output's in-edge folded into c-hat = C W_out per spec row: the last
// ReLU node's relaxation over a_hat = c-hat[r mod S] (+ cuts), elementwise,
// one column of four consecutive rows per item (the per-layer elementwise
// kernel's layout and sums).
template <typename T>
__device__ inline void chain_top(const BoundEpi<T>& epi, const LdsSink<T>& sink, const float* chat, int chat_ld, int S,
                                 int m0, int M, int n) {
  for (int it = threadIdx.x; it < 4 * n; it += blockDim.x) {
    const int g = it / n, j = it % n;
    LaneCoords<4, 1, false> lc;
#pragma unroll
    for (int v = 0; v < 4; ++v) lc.r[v] = m0 + 4 * g + v;
    lc.j[0][0] = j;
    float val[1][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = lc.r[v];
      float pre = 0.f;
      if (r < M) pre += chat[(size_t)(r % S) * chat_ld + j];
      val[0][v] = pre;
    }
    typename BoundEpi<T>::template Frag<4, 1, false> fr;
    epi.template load<4, 1, false>(fr, lc, M, n);
    double rs[4] = {0.0, 0.0, 0.0, 0.0};
    epi.template apply_to<4, 1, false>(fr, lc, val, rs, M, n, sink);
  }
}

template <typename T, int NW, int TN, int D>
__global__ void __launch_bounds__(NW * 64) chain_opt_kernel(ChainArgs a) {
  const int m0 = blockIdx.x * kChainRows;
  const int M = a.rp.M;
  const int L = a.L;
  const int off[2] = {a.off_buf0, a.off_buf1};
  for (int t = 0; t < a.iters; ++t) {
    AdamArgs ad = a.adam;
    ad.consts = a.adam.consts + 4 * t;
    // ---- bound pass: Lambda of node L-1 from c-hat, then down the chain
    int cur = 0;
    {
      const ChainNode& n = a.nodes[L - 1];
      BoundEpi<T> epi{BoundEpiArgs{n.nd, n.cc, a.rp, nullptr, nullptr, n.ahat}};
      chain_top<T>(epi, LdsSink<T>{off[cur], m0, a.P}, a.chat, a.chat_ld, a.rp.S, m0, M, n.nd.size);
    }
    __syncthreads();
    for (int i = L - 2; i >= 0; --i) {
      const ChainNode& up = a.nodes[i + 1];   // Lambda^(i+1) in LDS, pushed through node i+1's in-edge
      const ChainNode& n = a.nodes[i];
      BoundEpi<T> epi{BoundEpiArgs{n.nd, n.cc, a.rp, nullptr, nullptr, n.ahat}};
      chain_layer<T, NW, TN, false, D>(epi, LdsSink<T>{off[cur ^ 1], m0, a.P}, m0, M, n.nd.size, up.nd.size, off[cur],
                                       a.P, (const T*)up.WT, up.ldWT);
      __syncthreads();
      cur ^= 1;
    }
    {   // concretisation over the input box: sign(v) into LDS, input-cut pieces
      const ChainNode& n0 = a.nodes[0];
      ConcEpiArgs ca{a.in_size, a.in_ld, a.x0, a.eps, a.cc_in, a.rp, a.sign, a.nnz_e ? a.contrib : nullptr, a.nnz_e};
      ConcEpi epi{ca};
      chain_layer<T, NW, TN, false, D>(epi, LdsSink<int8_t>{a.off_sign, m0, a.sign_ld}, m0, M, a.in_size,
                                       n0.nd.size, off[cur], a.P, (const T*)n0.WT, n0.ldWT);
    }
    __syncthreads();
    // ---- adjoint, up the chain, with the Adam step of alpha and beta
    cur = 0;
    for (int i = 0; i < L; ++i) {
      const ChainNode& n = a.nodes[i];
      AdjEpiArgs aa{};
      aa.nd = n.nd; aa.cc = n.cc; aa.rp = a.rp;
      aa.acc_in = nullptr;
      aa.gemm_scale = i == 0 ? (float)(-a.eps) : 1.f;
      aa.add_vec = n.addv;
      aa.ahat = n.ahat;
      aa.dahat_out = n.dahat;
      aa.contrib = a.nnz_e ? a.contrib : nullptr;
      aa.nnz_e = a.nnz_e;
      aa.m_alpha = a.m_alpha; aa.v_alpha = a.v_alpha; aa.m_beta = a.m_beta; aa.v_beta = a.v_beta;
      aa.alpha_rw = a.alpha_rw; aa.beta_rw = a.beta_rw;
      aa.adam = ad;
      AdjEpi<T> epi{aa};
      if (i == 0) {
        chain_layer<T, NW, TN, true, D>(epi, LdsSink<T>{off[0], m0, a.P}, m0, M, n.nd.size, a.in_size, a.off_sign,
                                        a.sign_ld, (const T*)n.W, n.ldW);
        cur = 0;
      } else {
        chain_layer<T, NW, TN, false, D>(epi, LdsSink<T>{off[cur ^ 1], m0, a.P}, m0, M, n.nd.size,
                                         a.nodes[i - 1].nd.size, off[cur], a.P, (const T*)n.W, n.ldW);
        cur ^= 1;
      }
      __syncthreads();
    }
    // ---- multipliers of the workgroup's rows: d bound / d gamma from the
    // pieces just written (this workgroup's rows only), Adam on gamma
    for (int idx = threadIdx.x; idx < a.rp.N * kChainRows; idx += NW * 64) {
      const int k = idx / kChainRows, r = m0 + idx % kChainRows;
      if (r < M) gamma_one(k, r, M, a.rp.mp, a.rp.N, a.row_ptr, a.contrib, a.cut_d, a.gammaT, nullptr, a.m_gamma,
                           a.v_gamma, ad);
    }
    __syncthreads();
  }
}

template <typename T, int NW, int TN, int D>
static hipError_t launch_chain_t(const ChainArgs& a, int n_tiles, size_t lds, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)chain_opt_kernel<T, NW, TN, D>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((chain_opt_kernel<T, NW, TN, D>), dim3((unsigned)n_tiles), dim3(NW * 64), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_chain_opt(int bf16_mode, const ChainArgs& a, int n_tiles, size_t lds_bytes, hipStream_t st) {
  if (n_tiles <= 0 || a.iters <= 0) return hipSuccess;
  if (lds_bytes > 160 * 1024) return hipErrorInvalidValue;
  // waves per workgroup (GCP_CHAIN_WAVES = 4, 8 or 16; 4 measured fastest:
  // three workgroups fit on a compute unit)
  static const int waves = [] {
    const char* e = std::getenv("GCP_CHAIN_WAVES");
    return e ? std::atoi(e) : 4;
  }();
  if (waves == 16) {
    if (bf16_mode) return launch_chain_t<bf16, 16, 1, 4>(a, n_tiles, lds_bytes, st);
    return launch_chain_t<float, 16, 1, 4>(a, n_tiles, lds_bytes, st);
  }
  if (bf16_mode) return launch_chain_t<bf16, 4, 1, 4>(a, n_tiles, lds_bytes, st);
  return launch_chain_t<float, 4, 1, 4>(a, n_tiles, lds_bytes, st);
}

}  // namespace gcp
