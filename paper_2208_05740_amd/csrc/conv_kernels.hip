// Convolution edges of the GCP-CROWN passes as implicit GEMMs on MFMA.
//
// Bound direction (a_hat^(src) = Lambda^(node) A, A the conv's matrix): a
// transposed convolution.  GEMM rows = (batch row r, source position y, x),
// columns = source channel c, K = (node channel o, ky, kx):
//   A[(r,y,x)][(o,ky,kx)] = Lambda[r][o][(y+p-ky)/s][(x+p-kx)/s]  when the
//   division is exact and inside the node's spatial range, else 0;
//   B[(o,ky,kx)][c] = W[o][c][ky][kx].
// Adjoint direction (dLambda^(node) = A da_hat^(src)): a convolution.  GEMM
// rows = (r, oy, ox), columns = node channel o, K = (c, ky, kx):
//   A[(r,oy,ox)][(c,ky,kx)] = X[r][c][oy*s-p+ky][ox*s-p+kx] (0 outside),
//   B[(c,ky,kx)][o] = W[o][c][ky][kx].
// A tiles are gathered element-wise into the same LDS layout the dense
// kernel uses; B (weights, K contiguous) streams with 16-byte loads.  The
// spatial size of the epilogue side is a multiple of the tile height, so a
// tile never straddles two batch rows and its row constant goes to one
// partial slot: slot0 + (spatial_tile16) * ceil(C/16) + channel_tile16.
#include "gcp_internal.h"
#include "epilogues.h"

#include <hip/hip_runtime.h>

namespace gcp {

template <typename T, int BM, int BN, int WM, int WN, int BK, bool TRANS, bool SIGN, class Epi>
__global__ void __launch_bounds__(WM * WN * 64) conv_epi_kernel(ConvArgs c, Epi epi) {
  constexpr int NT = WM * WN * 64;
  constexpr int VEC = Op<T>::VEC;
  constexpr int KC = Op<T>::KC;
  constexpr int LDS_LD = BK + VEC;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int AV = BM * BK / VEC;
  constexpr int BV = BN * BK / VEC;
  constexpr int AIT = (AV + NT - 1) / NT;
  constexpr int BIT = (BV + NT - 1) / NT;
  static_assert(BK % KC == 0, "BK must be a multiple of the fragment K");
  static_assert(BM % 16 == 0 && BN % 16 == 0, "tile");

  __shared__ __attribute__((aligned(16))) T As[BM * LDS_LD];
  __shared__ __attribute__((aligned(16))) T Bs[BN * LDS_LD];
  __shared__ double red[NT / 64];

  const ConvGeom& g = c.cg;
  const int HW = TRANS ? g.hi * g.wi : g.ho * g.wo;     // positions on the epilogue side
  const int Wd = TRANS ? g.wi : g.wo;
  const int Nch = TRANS ? g.ci : g.co;                   // GEMM columns
  const int Kch = TRANS ? g.co : g.ci;                   // channels summed over
  const int KK = Kch * g.kh * g.kw;
  const int Mg = c.M * HW;
  const int node_size = Nch * HW;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int n_col = (Nch + BN - 1) / BN;
  const int total = n_col * ((Mg + BM - 1) / BM);
  const int xcd = blockIdx.x % 8, kx8 = blockIdx.x / 8;
  const int per = total / 8, rem = total % 8;
  const int vt = xcd * per + (xcd < rem ? xcd : rem) + kx8;
  const int bx = vt % n_col, by = vt / n_col;
  const int m0 = by * BM, n0 = bx * BN;

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int k = 0; k < TN; ++k) acc[i][k] = f4{0.f, 0.f, 0.f, 0.f};

  // epilogue coordinates: row m -> (r, position), column n -> neuron n*HW + position
  constexpr int R = TM * 4;
  LaneCoords<R, TN, true> lc;
  {
    const int row0 = m0 + wm * (BM / WM) + (lane >> 4) * 4;
    const int col0 = n0 + wn * (BN / WN) + (lane & 15);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int q = i * 4 + v, m = row0 + i * 16 + v;
        const int sp = m % HW;
        lc.r[q] = m < Mg ? m / HW : c.M;
#pragma unroll
        for (int k = 0; k < TN; ++k) {
          const int n = col0 + k * 16;
          lc.j[k][q] = n < Nch ? n * HW + sp : node_size;
        }
      }
  }
  typename Epi::template Frag<R, TN, true> fr;
  epi.template load<R, TN, true>(fr, lc, c.M, node_size);

  uint4 ra[AIT], rb[BIT];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      const int v = tid + it * NT;
      T tmp[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) tmp[q] = to_t<T>(0.f);
      if (v < AV) {
        const int row = v / (BK / VEC), kk = (v % (BK / VEC)) * VEC;
        const int m = m0 + row;
        if (m < Mg) {
          const int r = m / HW, sp = m % HW, y = sp / Wd, x = sp % Wd;
          int k = k0 + kk;
          int ch = k / (g.kh * g.kw), ky = (k / g.kw) % g.kh, kx = k % g.kw;
#pragma unroll
          for (int q = 0; q < VEC; ++q) {
            if (k < KK) {
              int sy, sx, ok;
              if constexpr (TRANS) {
                const int ty = y + g.pad - ky, tx = x + g.pad - kx;
                sy = ty / g.stride; sx = tx / g.stride;
                ok = ty >= 0 && tx >= 0 && ty % g.stride == 0 && tx % g.stride == 0 && sy < g.ho && sx < g.wo;
              } else {
                sy = y * g.stride - g.pad + ky; sx = x * g.stride - g.pad + kx;
                ok = sy >= 0 && sx >= 0 && sy < g.hi && sx < g.wi;
              }
              if (ok) {
                const int hs = TRANS ? g.ho : g.hi, ws = TRANS ? g.wo : g.wi;
                const size_t off = (size_t)r * c.ldx + (size_t)(ch * hs + sy) * ws + sx;
                if constexpr (SIGN) tmp[q] = to_t<T>((float)((const int8_t*)c.X)[off]);
                else tmp[q] = ((const T*)c.X)[off];
              }
            }
            ++k;
            if (++kx == g.kw) { kx = 0; if (++ky == g.kh) { ky = 0; ++ch; } }
          }
        }
      }
      ra[it] = *(const uint4*)tmp;
    }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int v = tid + it * NT;
      uint4 val = {0u, 0u, 0u, 0u};
      if (v < BV) {
        const int row = v / (BK / VEC), kk = (v % (BK / VEC)) * VEC;
        const int gn = n0 + row, gk = k0 + kk;
        if (gn < Nch && gk < c.ldb) val = *(const uint4*)((const T*)c.Bt + (size_t)gn * c.ldb + gk);
      }
      rb[it] = val;
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      const int v = tid + it * NT;
      if (v < AV) *(uint4*)(As + (v / (BK / VEC)) * LDS_LD + (v % (BK / VEC)) * VEC) = ra[it];
    }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int v = tid + it * NT;
      if (v < BV) *(uint4*)(Bs + (v / (BK / VEC)) * LDS_LD + (v % (BK / VEC)) * VEC) = rb[it];
    }
  };

  const int arow = wm * (BM / WM) + (lane & 15);
  const int bcol = wn * (BN / WN) + (lane & 15);
  const int kq = (lane >> 4) * VEC;
  if (KK > 0) load_stage(0);
  for (int k0 = 0; k0 < KK; k0 += BK) {
    __syncthreads();
    store_stage();
    __syncthreads();
    if (k0 + BK < KK) load_stage(k0 + BK);
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

  double rs[R];
#pragma unroll
  for (int q = 0; q < R; ++q) rs[q] = 0.0;
  {
    float val[TN][R];
#pragma unroll
    for (int k = 0; k < TN; ++k)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) val[k][i * 4 + v] = acc[i][k][v];
    epi.template apply<R, TN, true>(fr, lc, val, rs, c.M, node_size);
  }
  if (c.partial) {
    // the whole tile belongs to batch row m0 / HW: sum lane, wave, block
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) t += rs[q];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) red[wave] = t;
    __syncthreads();
    if (tid == 0 && m0 < Mg) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += red[w];
      const int r = m0 / HW;
      const int ncol16 = (Nch + 15) / 16;
      const int srow = (m0 % HW) / 16, scol = n0 / 16;
      for (int a = 0; a < BM / 16; ++a)
        for (int b = 0; b < BN / 16; ++b)
          if (scol + b < ncol16)
            c.partial[(size_t)(c.slot0 + (srow + a) * ncol16 + scol + b) * c.mp + r] = (a == 0 && b == 0) ? s : 0.0;
    }
  }
}

struct CTile { int bm, bn; };
static const CTile kConv[] = {{64, 16}, {64, 32}, {64, 64}, {32, 32}, {32, 16}, {16, 16}, {16, 32}};
int conv_num_configs() { return (int)(sizeof(kConv) / sizeof(kConv[0])); }
void conv_config_tile(int cfg, int* bm, int* bn) { *bm = kConv[cfg].bm; *bn = kConv[cfg].bn; }

template <typename T, int BM, int BN, int WM, int WN, bool TRANS, bool SIGN, class Epi>
static hipError_t conv_cfg(const ConvArgs& c, const Epi& epi, hipStream_t st) {
  constexpr int BK = (sizeof(T) == 4) ? 64 : 128;
  const ConvGeom& g = c.cg;
  const int HW = TRANS ? g.hi * g.wi : g.ho * g.wo;
  const int Nch = TRANS ? g.ci : g.co;
  if (HW % BM != 0) return hipErrorInvalidValue;   // a tile must not straddle batch rows
  const long tiles = (long)((Nch + BN - 1) / BN) * (((long)c.M * HW + BM - 1) / BM);
  hipLaunchKernelGGL((conv_epi_kernel<T, BM, BN, WM, WN, BK, TRANS, SIGN, Epi>), dim3((unsigned)tiles),
                     dim3(WM * WN * 64), 0, st, c, epi);
  return hipGetLastError();
}

template <typename T, bool TRANS, bool SIGN, class Epi>
static hipError_t conv_any(int cfg, const ConvArgs& c, const Epi& epi, hipStream_t st) {
  switch (cfg) {
    case 0: return conv_cfg<T, 64, 16, 4, 1, TRANS, SIGN>(c, epi, st);
    case 1: return conv_cfg<T, 64, 32, 2, 2, TRANS, SIGN>(c, epi, st);
    case 2: return conv_cfg<T, 64, 64, 2, 2, TRANS, SIGN>(c, epi, st);
    case 3: return conv_cfg<T, 32, 32, 2, 2, TRANS, SIGN>(c, epi, st);
    case 4: return conv_cfg<T, 32, 16, 2, 1, TRANS, SIGN>(c, epi, st);
    case 5: return conv_cfg<T, 16, 16, 1, 1, TRANS, SIGN>(c, epi, st);
    case 6: return conv_cfg<T, 16, 32, 1, 2, TRANS, SIGN>(c, epi, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t conv_typed(int cfg, EpiKind kind, const ConvArgs& c, const void* epi, hipStream_t st) {
  if (c.trans) {
    switch (kind) {
      case EPI_BOUND: return conv_any<T, true, false>(cfg, c, BoundEpi<T>{*(const BoundEpiArgs*)epi}, st);
      case EPI_CONC: return conv_any<T, true, false>(cfg, c, ConcEpi{*(const ConcEpiArgs*)epi}, st);
      case EPI_STORE: return conv_any<T, true, false>(cfg, c, StoreEpi{*(const StoreEpiArgs*)epi}, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (kind) {
    case EPI_ADJ:
      if (c.x_is_sign) return conv_any<T, false, true>(cfg, c, AdjEpi<T>{*(const AdjEpiArgs*)epi}, st);
      return conv_any<T, false, false>(cfg, c, AdjEpi<T>{*(const AdjEpiArgs*)epi}, st);
    case EPI_STORE:
      if (c.x_is_sign) return conv_any<T, false, true>(cfg, c, StoreEpi{*(const StoreEpiArgs*)epi}, st);
      return conv_any<T, false, false>(cfg, c, StoreEpi{*(const StoreEpiArgs*)epi}, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_conv(int bf16_mode, int cfg, EpiKind kind, const ConvArgs& c, const void* epi, hipStream_t st) {
  if (c.M <= 0) return hipSuccess;
  return bf16_mode ? conv_typed<bf16>(cfg, kind, c, epi, st) : conv_typed<float>(cfg, kind, c, epi, st);
}

}  // namespace gcp
