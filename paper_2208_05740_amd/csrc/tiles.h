// Tile-level device code shared by the per-layer kernels (kernels.hip) and
// the persistent dataflow kernel (persist_kernels.hip): the tile GEMM with a
// fused epilogue on gfx950 MFMA, and the elementwise relaxation of a block
// of rows.
#pragma once
#include "gcp_internal.h"
#include "epilogues.h"

#include <hip/hip_runtime.h>

namespace gcp {

// ------------------------------------------------------------------ tile GEMM
// C[M][N] = A[M][K] * Bt[N][K]^T on MFMA, epilogue per element, row partial
// sums reduced deterministically (lanes, then waves through LDS) into
// partial[r][slot0 + blockIdx.x].
// XCD-aware tile order: workgroups are dispatched round-robin over the 8
// XCDs by linear id, so the ids an XCD receives map onto a contiguous run of
// tiles (row panel major) and all column tiles of a row panel share that
// XCD's L2 instead of fetching the A panel once per XCD.
__device__ inline int xcd_tile(int id, int total) {
  const int xcd = id % 8, kx = id / 8;
  const int per = total / 8, rem = total % 8;
  return xcd * per + (xcd < rem ? xcd : rem) + kx;
}

// LDS of one tile: the A and B stages (16-byte row padding) and the per-wave
// row partials.
template <typename T, int BM, int BN, int WN, int BK>
struct TileLds {
  static constexpr int LD = BK + Op<T>::VEC;
  __attribute__((aligned(16))) T As[BM * LD];
  __attribute__((aligned(16))) T Bs[BN * LD];
  double red[WN][BM];
};

// One output tile (linear index vt, row panel major) of one GEMM problem,
// staged through the LDS block `sm`.
// OPAQUE: the thread id is made opaque to the optimiser, so that inside a
// persistent loop the values derived from it are recomputed per tile instead
// of held live across all of them (it costs the single-tile kernels
// registers, so they keep the plain id).
template <typename T, int BM, int BN, int WM, int WN, int BK, bool SIGN, class Epi, bool OPAQUE = false>
__device__ inline void gemm_tile_lds(const GemmArgs& g, const Epi& epi, int vt, TileLds<T, BM, BN, WN, BK>& sm) {
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

  T* As = sm.As;
  T* Bs = sm.Bs;
  auto& red = sm.red;

  int tid = threadIdx.x;
  if constexpr (OPAQUE) asm volatile("" : "+v"(tid));
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int n_col = (g.N + BN - 1) / BN;
  const int bx = vt % n_col, by = vt / n_col;
  const int m0 = by * BM, n0 = bx * BN;

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
            // VEC int8 signs in one load (the row pitch and gk are multiples of VEC)
            const int8_t* src = (const int8_t*)g.A + (size_t)gr * g.lda + gk;
            int8_t e[VEC];
            if constexpr (VEC == 8) *(uint2*)e = *(const uint2*)src;
            else *(uint32_t*)e = *(const uint32_t*)src;
            T tmp[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) tmp[q] = to_t<T>((float)e[q]);
            val = *(const uint4*)tmp;
          } else {
            val = *(const uint4*)((const T*)g.A + (size_t)gr * g.lda + gk);
          }
          if (gk + VEC > g.K) val = mask_tail<T>(val, g.K - gk);
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
        if (gn < g.N && gk < g.ldb) {
          val = *(const uint4*)((const T*)g.Bt + (size_t)gn * g.ldb + gk);
          if (gk + VEC > g.K) val = mask_tail<T>(val, g.K - gk);
        }
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

  // output coordinates of this lane
  constexpr int R = TM * 4;
  LaneCoords<R, TN, false> lc;
  {
    const int row0 = m0 + wm * (BM / WM) + (lane >> 4) * 4;
    const int col0 = n0 + wn * (BN / WN) + (lane & 15);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) lc.r[i * 4 + v] = row0 + i * 16 + v;
#pragma unroll
    for (int k = 0; k < TN; ++k) lc.j[k][0] = col0 + k * 16;
  }
  ColPre<TN> pre;
  if constexpr (Epi::kColPre) {
    int col[TN];
#pragma unroll
    for (int k = 0; k < TN; ++k) col[k] = lc.j[k][0];
    col_prefetch<TN>(pre, epi.col_node(), epi.col_cuts(), col, g.N);
  }
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
  // Its operands are fetched after the K loop: the K loops of these layers
  // are a few steps long, so prefetching them before the loop hid little
  // latency while keeping them live across it cost registers, and the
  // occupancy that buys back was worth more (measured: the adjoint kernel of
  // the 784-256x6 MLP at 1024 domains went from 41 to 36 us).
  typename Epi::template Frag<R, TN, false> fr;
  if constexpr (Epi::kColPre) epi.template load<R, TN, false>(fr, lc, g.M, g.N, &pre);
  else epi.template load<R, TN, false>(fr, lc, g.M, g.N);
  {
    double rs[R];
#pragma unroll
    for (int q = 0; q < R; ++q) rs[q] = 0.0;
    float val[TN][R];
#pragma unroll
    for (int k = 0; k < TN; ++k)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) val[k][i * 4 + v] = acc[i][k][v];
    epi.template apply<R, TN, false>(fr, lc, val, rs, g.M, g.N);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double t = wave_sum16(rs[q]);
      if ((lane & 15) == 0) red[wn][lc.r[q] - m0] = t;
    }
  }
  if (g.partial) {
    // row partials: one slot per 32 output columns, independent of the tile;
    // this block's sum goes to its first slot, zeros to the others it covers
    __syncthreads();
    const int nsl = (g.N + 31) / 32;
    const int s0 = bx * (BN / 32);
    for (int rl = tid; rl < BM; rl += NT) {
      int r = m0 + rl;
      if (r < g.M) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WN; ++w) s += red[w][rl];
#pragma unroll
        for (int t = 0; t < BN / 32; ++t)
          if (s0 + t < nsl) g.partial[(size_t)(g.slot0 + s0 + t) * g.mp + r] = t == 0 ? s : 0.0;
      }
    }
  }
}

// The same tile with its LDS block of its own.
template <typename T, int BM, int BN, int WM, int WN, int BK, bool SIGN, class Epi>
__device__ inline void gemm_tile(const GemmArgs& g, const Epi& epi, int vt) {
  __shared__ TileLds<T, BM, BN, WN, BK> sm;
  gemm_tile_lds<T, BM, BN, WM, WN, BK, SIGN, Epi>(g, epi, vt, sm);
}

// Elementwise relaxation (no GEMM: a_hat = bcast row + src): one block =
// kElemRows consecutive rows x 256 columns, each thread one column of those
// rows, so a neuron's data is read once for them and their loads are in
// flight together; one row partial per (row, column block), summed over the
// block in a fixed order.  PI selects the explicit-pi relaxation (a.rp.rho
// set).
template <typename T, bool PI, bool OPAQUE = false>
__device__ __forceinline__ void bound_elem_rows(const float* bcast, const void* src, const BoundEpiArgs& a, double* partial,
                                       int slot0, int r0, int cb) {
  constexpr int R = kElemRows;
  __shared__ double red[R][4];
  int tx = threadIdx.x;
  if constexpr (OPAQUE) asm volatile("" : "+v"(tx));   // as in gemm_tile_lds
  const int j = cb * 256 + tx;
  const int M = a.rp.M;
  BoundEpi<T, PI> epi{a};
  LaneCoords<R, 1, false> lc;
#pragma unroll
  for (int q = 0; q < R; ++q) lc.r[q] = r0 + q;
  lc.j[0][0] = j;
  float val[1][R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = r0 + q;
    float pre = 0.f;
    if (j < a.nd.size && r < M) {
      if (bcast) pre += bcast[(size_t)(r % a.rp.S) * a.nd.ld + j];
      if (src) pre += from_t<T>(((const T*)src)[(size_t)r * a.nd.ld + j]);
    }
    val[0][q] = pre;
  }
  double rs[R];
#pragma unroll
  for (int q = 0; q < R; ++q) rs[q] = 0.0;
  typename BoundEpi<T, PI>::template Frag<R, 1, false> fr;
  epi.template load<R, 1, false>(fr, lc, M, a.nd.size);
  epi.template apply<R, 1, false>(fr, lc, val, rs, M, a.nd.size);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    double t = rs[q];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((tx & 63) == 0) red[q][tx >> 6] = t;
  }
  __syncthreads();
  if (tx < R && partial) {
    const int q = tx, r = r0 + q;
    if (r < M) partial[(size_t)(slot0 + cb) * a.rp.mp + r] = (red[q][0] + red[q][1]) + (red[q][2] + red[q][3]);
  }
}

}  // namespace gcp
