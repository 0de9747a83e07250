// Convolution edges of the GCP-CROWN passes as implicit GEMMs on MFMA.
//
// Bound direction (a_hat^(src) = Lambda^(node) A, A the conv's matrix): a
// transposed convolution.  Output position (y, x) of the source grid meets
// the node grid only through taps with ky = (y + pad) mod s (+ s a) and
// likewise for kx, so the positions split into s^2 phases; within a phase
// every tap is real and
//   a_hat[c][y][x] = sum_(o,a,b) Lambda[o][Yb - a][Xb - b] Wph[c][(o,a,b)],
//   Yb = (y + pad - ry) / s,  Xb = (x + pad - rx) / s.
// Adjoint direction (dLambda^(node) = A da_hat^(src)): a convolution,
//   out[o][y][x] = sum_(c,ky,kx) X[c][y s - pad + ky][x s - pad + kx] W[o][(c,ky,kx)].
// Both are "slab GEMMs": one workgroup takes four consecutive batch rows and
// one band of output rows.  For each batch row in turn it copies the source
// rows the band reads into LDS (zero halo, so the inner loop has no bounds
// checks), forms MFMA A fragments by gathering from the slab at
// base(position) + koff(k), with koff precomputed per K index, and writes
// the band's results to that row's LDS result buffer.  B fragments (weights,
// K contiguous) are read from global memory, where the few KB of weights
// stay cached.  The fused epilogue then walks the band's neurons in memory
// order (a band of rows is a contiguous run of each channel plane), each
// lane one neuron of the four batch rows -- the layout of the dense GEMM
// epilogues, so a neuron's constants are read once for four rows and the
// row-minor buffers are 16-byte accesses.  The row constant of a band goes
// to one partial slot per batch row: slot0 + band.
#include "gcp_internal.h"
#include "epilogues.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace gcp {

namespace {
constexpr int kSlabBudget = 48 * 1024;   // bytes of fp32 slab + result bands a workgroup may use
constexpr int kRows = 4;                 // batch rows per workgroup
constexpr int kEpiN = 1;                 // neurons per lane in one epilogue step
constexpr int kLdsLimit = 64 * 1024;
constexpr int kDirNW = 8;               // waves per workgroup of the direct transposed conv
constexpr int kDirPF = 4;               // its staging vectors per thread held across a row's taps
constexpr int kDirCh = 2;               // its 64-position chunks per wave
__host__ __device__ inline int align16(int b) { return (b + 15) & ~15; }
}  // namespace

// Rows of phase ph inside band [yb0, yb1): source-side positions
// (yf + st*iy, xf + st*ix), iy < ny, ix < nx, st = s for the transposed
// direction (one phase per residue of y + pad and x + pad mod s), else 1.
__host__ __device__ inline void phase_rows(const ConvPlan& P, int ph, int yb0, int yb1, bool trans, int* yf, int* ny,
                                           int* xf, int* nx) {
  if (trans) {
    const int s = P.s, p = P.p, ry = ph / s, rx = ph % s;
    *yf = yb0 + (((ry - (yb0 + p)) % s) + s) % s;
    *ny = *yf < yb1 ? (yb1 - 1 - *yf) / s + 1 : 0;
    *xf = (((rx - p) % s) + s) % s;
    *nx = *xf < P.We ? (P.We - 1 - *xf) / s + 1 : 0;
  } else {
    *yf = yb0; *ny = yb1 - yb0; *xf = 0; *nx = P.We;
  }
}

ConvPlan conv_plan(const ConvGeom& g, int trans) {
  ConvPlan P{};
  const int s = g.stride;
  P.s = s;
  P.p = g.pad;
  if (trans) {
    P.He = g.hi; P.We = g.wi; P.Nch = g.ci; P.Kch = g.co; P.hs = g.ho; P.ws = g.wo;
    P.A = (g.kh + s - 1) / s;
    P.Bn = (g.kw + s - 1) / s;
    P.n_phase = s * s;
    P.Kreal = g.co * P.A * P.Bn;
    P.xl = P.Bn - 1;
    const int xmax = (g.wi - 1 + g.pad) / s;           // largest Xb
    P.Wp = P.xl + std::max(xmax + 1, g.wo);
  } else {
    P.He = g.ho; P.We = g.wo; P.Nch = g.co; P.Kch = g.ci; P.hs = g.hi; P.ws = g.wi;
    P.A = g.kh;
    P.Bn = g.kw;
    P.n_phase = 1;
    P.Kreal = g.ci * g.kh * g.kw;
    P.xl = g.pad;
    P.Wp = P.xl + std::max(g.wi, (g.wo - 1) * s - g.pad + g.kw);
  }
  P.KP = (P.Kreal + 31) / 32 * 32;
  auto rows_for = [&](int bh) { return trans ? (bh - 1) / s + 1 + P.A : (bh - 1) * s + g.kh; };
  auto bytes_for = [&](int bh) {
    return ((long)P.Kch * rows_for(bh) * P.Wp + (long)kRows * P.Nch * (bh * P.We + 1)) * 4;
  };
  int bh = P.He;
  while (bh > 1 && bytes_for(bh) > kSlabBudget) --bh;
  P.n_bands = (P.He + bh - 1) / bh;
  P.BH = (P.He + P.n_bands - 1) / P.n_bands;           // balance the bands
  P.rows_max = rows_for(P.BH);
  P.CHS = P.rows_max * P.Wp;
  P.OS = P.BH * P.We + 1;                              // odd: channel planes on different banks
  P.MT = 0;
  for (int b = 0; b < P.n_bands; ++b) {
    const int yb0 = b * P.BH, yb1 = std::min(P.He, yb0 + P.BH);
    int nt = 0;
    for (int ph = 0; ph < P.n_phase; ++ph) {
      int yf, ny, xf, nx;
      phase_rows(P, ph, yb0, yb1, trans != 0, &yf, &ny, &xf, &nx);
      nt += (ny * nx + 15) / 16;
    }
    P.MT = std::max(P.MT, nt);
  }
  return P;
}

int conv_ldb(const ConvGeom& g, int trans) { return conv_plan(g, trans).KP; }

void conv_pack_weights(const ConvGeom& g, int trans, const float* raw, float* out) {
  const ConvPlan P = conv_plan(g, trans);
  const int ldb = P.KP, s = g.stride;
  auto w = [&](int o, int c, int ky, int kx) { return raw[(((size_t)o * g.ci + c) * g.kh + ky) * g.kw + kx]; };
  if (!trans) {
    for (int o = 0; o < g.co; ++o)
      for (int k = 0; k < ldb; ++k) {
        float v = 0.f;
        if (k < P.Kreal) {
          const int c = k / (g.kh * g.kw), ky = (k / g.kw) % g.kh, kx = k % g.kw;
          v = w(o, c, ky, kx);
        }
        out[(size_t)o * ldb + k] = v;
      }
    return;
  }
  for (int ph = 0; ph < P.n_phase; ++ph) {
    const int ry = ph / s, rx = ph % s;
    for (int c = 0; c < g.ci; ++c)
      for (int k = 0; k < ldb; ++k) {
        float v = 0.f;
        if (k < P.Kreal) {
          const int o = k / (P.A * P.Bn), a = (k / P.Bn) % P.A, b = k % P.Bn;
          const int ky = ry + s * a, kx = rx + s * b;
          if (ky < g.kh && kx < g.kw) v = w(o, c, ky, kx);
        }
        out[((size_t)ph * g.ci + c) * ldb + k] = v;
      }
  }
}

static int conv_lds_bytes(const ConvPlan& P, int esz, int nw) {
  return align16(P.KP * 4) + align16(nw * 8 * kRows) + align16(P.MT * 4) + P.MT * 16 * 8 +
         align16(P.Kch * P.CHS * esz) + kRows * align16(P.Nch * P.OS * 4);
}

// direct transposed-conv kernel: reduction slots, fp32 slab, four result bands
static int conv_direct_lds_bytes(const ConvPlan& P) {
  return align16(kDirNW * 8 * kRows) + align16(P.Kch * P.CHS * 4) + kRows * align16(P.Nch * P.OS * 4);
}

// ---------------------------------------------------------------- slab fill
template <typename T, bool SIGN> struct SlabLoad;
template <> struct SlabLoad<bf16, false> {
  __device__ static inline void vec(const void* X, size_t off, bf16* d) {
    const uint4 v = *(const uint4*)((const bf16*)X + off);
    const bf16x8 e = __builtin_bit_cast(bf16x8, v);
#pragma unroll
    for (int q = 0; q < 8; ++q) d[q] = e[q];
  }
  __device__ static inline bf16 one(const void* X, size_t off) { return ((const bf16*)X)[off]; }
};
template <> struct SlabLoad<float, false> {
  __device__ static inline void vec(const void* X, size_t off, float* d) {
    const float4 v = *(const float4*)((const float*)X + off);
    d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
  }
  __device__ static inline float one(const void* X, size_t off) { return ((const float*)X)[off]; }
};
template <> struct SlabLoad<bf16, true> {
  __device__ static inline void vec(const void* X, size_t off, bf16* d) {
    const uint2 v = *(const uint2*)((const int8_t*)X + off);
    const int8_t* e = (const int8_t*)&v;
#pragma unroll
    for (int q = 0; q < 8; ++q) d[q] = (bf16)(float)e[q];
  }
  __device__ static inline bf16 one(const void* X, size_t off) { return (bf16)(float)((const int8_t*)X)[off]; }
};
template <> struct SlabLoad<float, true> {
  __device__ static inline void vec(const void* X, size_t off, float* d) {
    const uint32_t v = *(const uint32_t*)((const int8_t*)X + off);
    const int8_t* e = (const int8_t*)&v;
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = (float)e[q];
  }
  __device__ static inline float one(const void* X, size_t off) { return (float)((const int8_t*)X)[off]; }
};

// A fragment of one lane: VEC consecutive K indices of its GEMM row, gathered
// from the slab (uint4 in the MFMA operand layout).
template <typename T> struct Gather;
template <> struct Gather<bf16> {
  __device__ static inline uint4 get(const bf16* slab, int base, const int* ko) {
    const unsigned short* S = (const unsigned short*)slab;
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      w[q] = (uint32_t)S[base + ko[2 * q]] | ((uint32_t)S[base + ko[2 * q + 1]] << 16);
    return uint4{w[0], w[1], w[2], w[3]};
  }
};
template <> struct Gather<float> {
  __device__ static inline uint4 get(const float* slab, int base, const int* ko) {
    const uint32_t* S = (const uint32_t*)slab;
    return uint4{S[base + ko[0]], S[base + ko[1]], S[base + ko[2]], S[base + ko[3]]};
  }
};

// Fused epilogue of one workgroup's band, over the results of its kRows batch
// rows in LDS (row q at outs + q * OQ, channel n at n * OS, position
// (y - yb0) * We + x): walk the band's neurons in memory order, then sum the
// row constant of each batch row into its partial slot slot0 + band.
template <int NW, class Epi>
__device__ __forceinline__ void band_epilogue(const ConvArgs& c, const ConvPlan& P, const Epi& epi, const float* outs,
                                              int OQ, double* red, int r0, int band, int yb0, int yb1) {
  constexpr int NT = NW * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int HWe = P.He * P.We;
  const int node_size = P.Nch * HWe;
  // fused epilogue over the band's neurons in memory order: per step a lane
  // takes kEpiN neurons (NT apart) of the four batch rows, so that the
  // dependent load chains of several neurons are in flight together
  double rs[kRows];
#pragma unroll
  for (int q = 0; q < kRows; ++q) rs[q] = 0.0;
  {
    const int per_ch = (yb1 - yb0) * P.We;
    const int nel = P.Nch * per_ch;
    const int j0 = yb0 * P.We;
    const float inv_pc = 1.f / (float)per_ch;
    LaneCoords<kRows, kEpiN, false> lc;
#pragma unroll
    for (int q = 0; q < kRows; ++q) lc.r[q] = r0 + q;
    for (int e0 = tid; e0 < nel; e0 += kEpiN * NT) {
      float val[kEpiN][kRows];
#pragma unroll
      for (int k = 0; k < kEpiN; ++k) {
        const int e = e0 + k * NT;
        // e = n * per_ch + off; the float quotient is within one of n
        int n = (int)((float)e * inv_pc), off = e - n * per_ch;
        if (off < 0) { --n; off += per_ch; } else if (off >= per_ch) { ++n; off -= per_ch; }
        const bool ok = e < nel;
        lc.j[k][0] = ok ? n * HWe + j0 + off : node_size;   // node_size marks no neuron
#pragma unroll
        for (int q = 0; q < kRows; ++q) val[k][q] = ok && r0 + q < c.M ? outs[q * OQ + n * P.OS + off] : 0.f;
      }
      typename Epi::template Frag<kRows, kEpiN, false> fr;
      epi.template load<kRows, kEpiN, false>(fr, lc, c.M, node_size);
      epi.template apply<kRows, kEpiN, false>(fr, lc, val, rs, c.M, node_size);
    }
  }

  if (c.partial) {
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      double tsum = rs[q];
      for (int o = 32; o > 0; o >>= 1) tsum += __shfl_xor(tsum, o, 64);
      if (lane == 0) red[wave * kRows + q] = tsum;
    }
    __syncthreads();
    if (tid < kRows && r0 + tid < c.M) {
      double sum = 0.0;
      for (int w = 0; w < NW; ++w) sum += red[w * kRows + tid];
      c.partial[(size_t)(c.slot0 + band) * c.mp + r0 + tid] = sum;
    }
  }
}

template <typename T, int NW, int TN, bool TRANS, bool SIGN, class Epi>
__global__ void __launch_bounds__(NW * 64) conv_slab_kernel(ConvArgs c, ConvPlan P, Epi epi) {
  constexpr int NT = NW * 64;
  constexpr int VEC = Op<T>::VEC;
  constexpr int KC = Op<T>::KC;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  unsigned char* sp = smem;
  int* koff = (int*)sp;        sp += align16(P.KP * 4);
  double* red = (double*)sp;   sp += align16(NW * 8 * kRows);
  int* tph = (int*)sp;         sp += align16(P.MT * 4);        // phase of each 16-row tile
  int2* desc = (int2*)sp;      sp += P.MT * 16 * 8;            // per GEMM row: {slab base, result offset or -1}
  T* slab = (T*)sp;            sp += align16(P.Kch * P.CHS * (int)sizeof(T));
  float* outs = (float*)sp;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = (blockIdx.x / P.n_bands) * kRows, band = blockIdx.x % P.n_bands;
  const int OQ = align16(P.Nch * P.OS * 4) / 4;                    // floats between the rows' result buffers
  const int s = P.s, p = P.p;
  const int yb0 = band * P.BH, yb1 = min(P.He, yb0 + P.BH);
  const int sy0 = TRANS ? (yb0 + p) / s - (P.A - 1) : yb0 * s - p;   // source row of slab row 0
  const int HWe = P.He * P.We;
  const int node_size = P.Nch * HWe;
  const int safe_base = TRANS ? (P.A - 1) * P.Wp + P.Bn - 1 : 0;    // in-slab for every koff

  // K index -> slab offset relative to a row's base
  for (int k = tid; k < P.KP; k += NT) {
    int o = 0;
    if (k < P.Kreal) {
      const int ch = k / (P.A * P.Bn), a = (k / P.Bn) % P.A, b = k % P.Bn;
      o = TRANS ? ch * P.CHS - a * P.Wp - b : ch * P.CHS + a * P.Wp + b;
    }
    koff[k] = o;
  }
  // GEMM rows of the band, phase by phase, each phase padded to whole tiles
  int ntile = 0;
  for (int ph = 0; ph < P.n_phase; ++ph) {
    int yf, ny, xf, nx;
    phase_rows(P, ph, yb0, yb1, TRANS, &yf, &ny, &xf, &nx);
    const int npos = ny * nx, nt = (npos + 15) / 16;
    int base0, rstep, cstep;
    if constexpr (TRANS) {
      const int ry = ph / s, rx = ph % s;
      base0 = ((yf + p - ry) / s - sy0) * P.Wp + (xf + p - rx) / s + P.xl;
      rstep = P.Wp; cstep = 1;
    } else {
      base0 = (yf * s - p - sy0) * P.Wp + xf * s - p + P.xl;
      rstep = s * P.Wp; cstep = s;
    }
    const int st = TRANS ? s : 1;
    const int out0 = (yf - yb0) * P.We + xf;
    for (int i = tid; i < nt * 16; i += NT) {
      int2 d = make_int2(safe_base, -1);
      if (i < npos) {
        const int iy = i / nx, ix = i - iy * nx;
        d = make_int2(base0 + iy * rstep + ix * cstep, out0 + iy * st * P.We + ix * st);
      }
      desc[ntile * 16 + i] = d;
    }
    for (int i = tid; i < nt; i += NT) tph[ntile + i] = ph;
    ntile += nt;
  }
  {   // the halo stays zero for every row: only interior cells are rewritten
    uint4* z = (uint4*)slab;
    const int n16 = align16(P.Kch * P.CHS * (int)sizeof(T)) / 16;
    for (int v = tid; v < n16; v += NT) z[v] = uint4{0u, 0u, 0u, 0u};
  }
  const int nck = (P.Nch + 16 * TN - 1) / (16 * TN);
  const int g = lane >> 4;
  for (int q = 0; q < kRows && r0 + q < c.M; ++q) {
    const int r = r0 + q;
    float* outq = outs + q * OQ;
    __syncthreads();      // tables and zeros written; the previous row's MFMAs done with the slab
    {
      const size_t xrow = (size_t)r * c.ldx;
      const bool vec = P.ws % VEC == 0;
      const int cw = vec ? VEC : 1;
      const int nchunk = P.ws / cw;
      const int total = P.Kch * P.rows_max * nchunk;
      for (int v = tid; v < total; v += NT) {
        const int xc = v % nchunk, rest = v / nchunk;
        const int rho = rest % P.rows_max, ch = rest / P.rows_max;
        const int sy = sy0 + rho;
        if (sy < 0 || sy >= P.hs) continue;
        const size_t src = xrow + ((size_t)ch * P.hs + sy) * P.ws + (size_t)xc * cw;
        T* dst = slab + ch * P.CHS + rho * P.Wp + P.xl + xc * cw;
        if (vec) {
          T tmp[VEC];
          SlabLoad<T, SIGN>::vec(c.X, src, tmp);
#pragma unroll
          for (int e = 0; e < VEC; ++e) dst[e] = tmp[e];
        } else {
          dst[0] = SlabLoad<T, SIGN>::one(c.X, src);
        }
      }
    }
    __syncthreads();

    // MFMA tiles: (16-row tile, column chunk of 16*TN channels) -> this row's result band
    for (int t = wave; t < ntile * nck; t += NW) {
      const int tt = nck == 1 ? t : t / nck, ck = nck == 1 ? 0 : t - tt * nck;
      const int ph = __builtin_amdgcn_readfirstlane(tph[tt]);
      const int base = desc[tt * 16 + (lane & 15)].x;
      f4 acc[TN];
#pragma unroll
      for (int k = 0; k < TN; ++k) acc[k] = f4{0.f, 0.f, 0.f, 0.f};
      const T* Bp = (const T*)c.Bt + (size_t)ph * P.Nch * c.ldb;
      int nb[TN];
#pragma unroll
      for (int k = 0; k < TN; ++k) nb[k] = ck * 16 * TN + k * 16 + (lane & 15);
      for (int k0 = 0; k0 < P.KP; k0 += KC) {
        int ko[VEC];
        const int4* kp = (const int4*)(koff + k0 + VEC * g);
#pragma unroll
        for (int e = 0; e < VEC / 4; ++e) {
          const int4 t4 = kp[e];
          ko[4 * e] = t4.x; ko[4 * e + 1] = t4.y; ko[4 * e + 2] = t4.z; ko[4 * e + 3] = t4.w;
        }
        const uint4 fa = Gather<T>::get(slab, base, ko);
#pragma unroll
        for (int k = 0; k < TN; ++k) {
          uint4 fb = {0u, 0u, 0u, 0u};
          if (nb[k] < P.Nch) fb = *(const uint4*)(Bp + (size_t)nb[k] * c.ldb + k0 + VEC * g);
          Op<T>::mma(fa, fb, acc[k]);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = desc[tt * 16 + g * 4 + v].y;
        if (o < 0) continue;
#pragma unroll
        for (int k = 0; k < TN; ++k)
          if (nb[k] < P.Nch) outq[nb[k] * P.OS + o] = acc[k][v];
      }
    }
  }
  __syncthreads();

  band_epilogue<NW>(c, P, epi, outs, OQ, red, r0, band, yb0, yb1);
}

// One 16-byte vector of a slab row as fp32 values.
template <typename T> struct SlabCvt;
template <> struct SlabCvt<float> {
  __device__ static inline void get(const uint4& v, float* f) {
    f[0] = __uint_as_float(v.x); f[1] = __uint_as_float(v.y); f[2] = __uint_as_float(v.z); f[3] = __uint_as_float(v.w);
  }
};
template <> struct SlabCvt<bf16> {
  __device__ static inline void get(const uint4& v, float* f) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      f[2 * q] = __uint_as_float(w[q] << 16);
      f[2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);
    }
  }
};

// Transposed convolution into a source of at most four channels (the
// network's input image) on the vector ALUs.  An MFMA tile's 16 columns
// would carry NC real channels and padding, so here each lane computes all NC
// channels of one source position: per tap, one LDS read of Lambda feeds NC
// FMAs.  A wave takes 64 positions of one stride phase at a time, so the
// phase's weights (taps TA x TB per phase, fp32 in the operand precision) are
// wave-uniform scalar loads; the stride ST is a template parameter.  Band split, slab layout, per-row result buffers,
// fused epilogue and partial slots are those of conv_slab_kernel; the slab is
// held in fp32 for either operand type.  What does not depend on the batch
// row -- each wave's (at most kDirCh) position chunks with their phase, slab
// base and result offset, and each thread's (at most kDirPF) staging vectors
// with their source and slab offsets -- is worked out once per workgroup and
// kept in registers; the next row's staging loads are issued before this
// row's taps, so their latency is hidden behind the FMAs.
template <typename T, int NC, int TA, int TB, int ST, class Epi>
__global__ void __launch_bounds__(kDirNW * 64) convT_direct_kernel(ConvArgs c, ConvPlan Pr, Epi epi) {
  ConvPlan P = Pr;
  P.s = ST;              // the stride as a constant: phase arithmetic without divisions
  constexpr int NT = kDirNW * 64;
  constexpr int VEC = Op<T>::VEC;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  unsigned char* sp = smem;
  double* red = (double*)sp;  sp += align16(kDirNW * 8 * kRows);
  float* slab = (float*)sp;   sp += align16(P.Kch * P.CHS * 4);
  float* outs = (float*)sp;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = (blockIdx.x / P.n_bands) * kRows, band = blockIdx.x % P.n_bands;
  const int OQ = align16(P.Nch * P.OS * 4) / 4;
  const int s = P.s, p = P.p;
  const int yb0 = band * P.BH, yb1 = min(P.He, yb0 + P.BH);
  const int sy0 = (yb0 + p) / s - (TA - 1);
  {
    float4* z = (float4*)slab;
    const int n16 = align16(P.Kch * P.CHS * 4) / 16;
    for (int v = tid; v < n16; v += NT) z[v] = float4{0.f, 0.f, 0.f, 0.f};
  }
  // position chunks of this wave: chunk t = wave + k kDirNW of the band's
  // 64-position chunks, phase by phase
  int cph[kDirCh], cbase[kDirCh], coff[kDirCh];
  bool clive[kDirCh];
#pragma unroll
  for (int k = 0; k < kDirCh; ++k) {
    int tl = wave + k * kDirNW, ph = 0, yf = 0, ny = 0, xf = 0, nx = 0;
    for (; ph < P.n_phase; ++ph) {
      phase_rows(P, ph, yb0, yb1, true, &yf, &ny, &xf, &nx);
      const int nt = (ny * nx + 63) / 64;
      if (tl < nt) break;
      tl -= nt;
    }
    cph[k] = __builtin_amdgcn_readfirstlane(ph);      // n_phase: no chunk
    const int i = tl * 64 + lane;
    clive[k] = ph < P.n_phase && i < ny * nx;
    const int iy = clive[k] ? i / nx : 0, ix = clive[k] ? i - iy * nx : 0;
    const int ry = ph / s, rx = ph % s;
    cbase[k] = clive[k] ? ((yf + p - ry) / s - sy0 + iy) * P.Wp + (xf + p - rx) / s + ix + P.xl
                        : (TA - 1) * P.Wp + TB - 1;     // in-slab for every tap
    coff[k] = (yf - yb0 + iy * s) * P.We + xf + ix * s;
  }
  // staging: item v of a batch row is VEC consecutive source elements (one
  // where the rows are not whole vectors) of slab row rho, channel ch
  const bool vec = P.ws % VEC == 0;
  const int cw = vec ? VEC : 1;
  const int nck = P.ws / cw;
  const int total = P.Kch * P.rows_max * nck;
  auto item = [&](int v, int* src, int* dst) -> bool {
    const int xc = v % nck, rest = v / nck;
    const int rho = rest % P.rows_max, ch = rest / P.rows_max;
    const int sy = sy0 + rho;
    if (v >= total || sy < 0 || sy >= P.hs) return false;
    *src = (ch * P.hs + sy) * P.ws + xc * cw;
    *dst = ch * P.CHS + rho * P.Wp + P.xl + xc * cw;
    return true;
  };
  const bool pf = vec && total <= kDirPF * NT;
  int ssrc[kDirPF], sdst[kDirPF];                     // sdst < 0: nothing to stage
  uint4 nxt[kDirPF];
  if (pf) {
#pragma unroll
    for (int u = 0; u < kDirPF; ++u)
      if (!item(tid + u * NT, &ssrc[u], &sdst[u])) sdst[u] = -1;
  }
  auto fetch = [&](int r) {
    const T* xr = (const T*)c.X + (size_t)r * c.ldx;
#pragma unroll
    for (int u = 0; u < kDirPF; ++u)
      if (sdst[u] >= 0) nxt[u] = *(const uint4*)(xr + ssrc[u]);
  };
  if (pf) fetch(r0);
  for (int q = 0; q < kRows && r0 + q < c.M; ++q) {
    float* outq = outs + q * OQ;
    __syncthreads();      // zeros written; the previous row's taps read
    if (pf) {
#pragma unroll
      for (int u = 0; u < kDirPF; ++u) {
        if (sdst[u] < 0) continue;
        float f[VEC];
        SlabCvt<T>::get(nxt[u], f);
#pragma unroll
        for (int e = 0; e < VEC; ++e) slab[sdst[u] + e] = f[e];
      }
    } else {
      const size_t xrow = (size_t)(r0 + q) * c.ldx;
      for (int v = tid; v < total; v += NT) {
        int src, dst;
        if (!item(v, &src, &dst)) continue;
        if (vec) {
          T tmp[VEC];
          SlabLoad<T, false>::vec(c.X, xrow + src, tmp);
#pragma unroll
          for (int e = 0; e < VEC; ++e) slab[dst + e] = (float)tmp[e];
        } else {
          slab[dst] = (float)SlabLoad<T, false>::one(c.X, xrow + src);
        }
      }
    }
    __syncthreads();
    if (pf && q + 1 < kRows && r0 + q + 1 < c.M) fetch(r0 + q + 1);
#pragma unroll
    for (int k = 0; k < kDirCh; ++k) {
      if (cph[k] >= P.n_phase) continue;
      const GCP_CONSTANT_AS float* W = cst(c.Btf) + (size_t)cph[k] * P.Nch * c.ldb;
      float acc[NC];
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) acc[ch] = 0.f;
#pragma unroll 2
      for (int o = 0; o < P.Kch; ++o) {
        const float* so = slab + o * P.CHS + cbase[k];
        float v[TA][TB];
#pragma unroll
        for (int a = 0; a < TA; ++a)
#pragma unroll
          for (int b = 0; b < TB; ++b) v[a][b] = so[-a * P.Wp - b];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) {
          const GCP_CONSTANT_AS float* w = W + (size_t)ch * c.ldb + o * (TA * TB);
#pragma unroll
          for (int a = 0; a < TA; ++a)
#pragma unroll
            for (int b = 0; b < TB; ++b) acc[ch] = fmaf(v[a][b], w[a * TB + b], acc[ch]);
        }
      }
      if (clive[k]) {
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) outq[ch * P.OS + coff[k]] = acc[ch];
      }
    }
  }
  __syncthreads();
  band_epilogue<kDirNW>(c, P, epi, outs, OQ, red, r0, band, yb0, yb1);
}

// launch configurations: waves per workgroup x column tiles per wave
struct CCfg { int nw, tn; };
static const CCfg kConv[] = {{4, 1}, {4, 2}, {8, 1}, {8, 2}, {4, 4}, {2, 1}};
int conv_num_configs() { return (int)(sizeof(kConv) / sizeof(kConv[0])); }

template <typename T, int NW, int TN, bool TRANS, bool SIGN, class Epi>
static hipError_t conv_go(const ConvArgs& c, const ConvPlan& P, const Epi& epi, hipStream_t st) {
  const int lds = conv_lds_bytes(P, (int)sizeof(T), NW);
  if (lds > kLdsLimit) return hipErrorInvalidValue;
  const long grid = (long)((c.M + kRows - 1) / kRows) * P.n_bands;
  if (grid <= 0 || grid > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((conv_slab_kernel<T, NW, TN, TRANS, SIGN, Epi>), dim3((unsigned)grid), dim3(NW * 64),
                     (unsigned)lds, st, c, P, epi);
  return hipGetLastError();
}

template <typename T, bool TRANS, bool SIGN, class Epi>
static hipError_t conv_any(int cfg, const ConvArgs& c, const Epi& epi, hipStream_t st) {
  const ConvPlan P = conv_plan(c.cg, TRANS ? 1 : 0);
  if (c.ldb < P.KP || c.ldb % 32 != 0) return hipErrorInvalidValue;
  switch (cfg) {
    case 0: return conv_go<T, 4, 1, TRANS, SIGN>(c, P, epi, st);
    case 1: return conv_go<T, 4, 2, TRANS, SIGN>(c, P, epi, st);
    case 2: return conv_go<T, 8, 1, TRANS, SIGN>(c, P, epi, st);
    case 3: return conv_go<T, 8, 2, TRANS, SIGN>(c, P, epi, st);
    case 4: return conv_go<T, 4, 4, TRANS, SIGN>(c, P, epi, st);
    case 5: return conv_go<T, 2, 1, TRANS, SIGN>(c, P, epi, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t conv_typed(int cfg, EpiKind kind, const ConvArgs& c, const void* epi, hipStream_t st) {
  if (c.trans) {
    switch (kind) {
      case EPI_BOUND: return conv_any<T, true, false>(cfg, c, BoundEpi<T>{*(const BoundEpiArgs*)epi}, st);
      case EPI_AHAT: return conv_any<T, true, false>(cfg, c, AhatEpi<T>{*(const BoundEpiArgs*)epi}, st);
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

// Explicit-pi epilogues (rho set): instantiated for one column tile per
// wave only, 4 or 8 waves; the other shapes run as 8 waves.
template <typename T, bool TRANS, bool SIGN, class Epi>
static hipError_t conv_pi_any(int cfg, const ConvArgs& c, const Epi& epi, hipStream_t st) {
  const ConvPlan P = conv_plan(c.cg, TRANS ? 1 : 0);
  if (c.ldb < P.KP || c.ldb % 32 != 0) return hipErrorInvalidValue;
  if (cfg == 0) return conv_go<T, 4, 1, TRANS, SIGN>(c, P, epi, st);
  return conv_go<T, 8, 1, TRANS, SIGN>(c, P, epi, st);
}

template <typename T>
static hipError_t conv_typed_pi(int cfg, EpiKind kind, const ConvArgs& c, const void* epi, hipStream_t st) {
  if (c.trans)
    return kind == EPI_BOUND ? conv_pi_any<T, true, false>(cfg, c, BoundEpi<T, true>{*(const BoundEpiArgs*)epi}, st)
                             : hipErrorInvalidValue;
  if (kind != EPI_ADJ) return hipErrorInvalidValue;
  if (c.x_is_sign) return conv_pi_any<T, false, true>(cfg, c, AdjEpi<T, true>{*(const AdjEpiArgs*)epi}, st);
  return conv_pi_any<T, false, false>(cfg, c, AdjEpi<T, true>{*(const AdjEpiArgs*)epi}, st);
}

bool conv_direct_ok(const ConvGeom& g, EpiKind kind) {
  if (kind != EPI_CONC || g.ci < 1 || g.ci > 4) return false;
  const ConvPlan P = conv_plan(g, 1);
  if (!((P.A == 2 && P.Bn == 2 && P.s == 2) || (P.A == 3 && P.Bn == 3 && P.s == 1))) return false;
  for (int b = 0; b < P.n_bands; ++b) {      // every band's positions in kDirCh chunks per wave
    const int yb0 = b * P.BH, yb1 = std::min(P.He, yb0 + P.BH);
    int nchunk = 0;
    for (int ph = 0; ph < P.n_phase; ++ph) {
      int yf, ny, xf, nx;
      phase_rows(P, ph, yb0, yb1, true, &yf, &ny, &xf, &nx);
      nchunk += (ny * nx + 63) / 64;
    }
    if (nchunk > kDirNW * kDirCh) return false;
  }
  return conv_direct_lds_bytes(P) <= kLdsLimit;
}

template <typename T, int NC, int TA, int TB, int ST, class Epi>
static hipError_t direct_go(const ConvArgs& c, const ConvPlan& P, const Epi& epi, hipStream_t st) {
  const long grid = (long)((c.M + kRows - 1) / kRows) * P.n_bands;
  if (grid <= 0 || grid > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((convT_direct_kernel<T, NC, TA, TB, ST, Epi>), dim3((unsigned)grid), dim3(kDirNW * 64),
                     (unsigned)conv_direct_lds_bytes(P), st, c, P, epi);
  return hipGetLastError();
}

template <typename T, int NC, class Epi>
static hipError_t direct_taps(const ConvArgs& c, const ConvPlan& P, const Epi& epi, hipStream_t st) {
  if (P.A == 2 && P.Bn == 2 && P.s == 2) return direct_go<T, NC, 2, 2, 2>(c, P, epi, st);
  if (P.A == 3 && P.Bn == 3 && P.s == 1) return direct_go<T, NC, 3, 3, 1>(c, P, epi, st);
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t conv_direct(const ConvArgs& c, const ConcEpi& epi, hipStream_t st) {
  const ConvPlan P = conv_plan(c.cg, 1);
  if (!c.Btf || c.ldb < P.KP || c.ldb % 32 != 0 || conv_direct_lds_bytes(P) > kLdsLimit) return hipErrorInvalidValue;
  switch (P.Nch) {
    case 1: return direct_taps<T, 1>(c, P, epi, st);
    case 2: return direct_taps<T, 2>(c, P, epi, st);
    case 3: return direct_taps<T, 3>(c, P, epi, st);
    case 4: return direct_taps<T, 4>(c, P, epi, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_conv(int bf16_mode, int cfg, EpiKind kind, const ConvArgs& c, const void* epi, hipStream_t st) {
  if (c.M <= 0) return hipSuccess;
  if (cfg == kConvDirectCfg) {
    if (!c.trans || !conv_direct_ok(c.cg, kind)) return hipErrorInvalidValue;
    const ConcEpi e{*(const ConcEpiArgs*)epi};
    return bf16_mode ? conv_direct<bf16>(c, e, st) : conv_direct<float>(c, e, st);
  }
  if (cfg < 0 || cfg >= conv_num_configs()) return hipErrorInvalidValue;
  if (fused_explicit_pi(kind, epi))
    return bf16_mode ? conv_typed_pi<bf16>(cfg, kind, c, epi, st) : conv_typed_pi<float>(cfg, kind, c, epi, st);
  return bf16_mode ? conv_typed<bf16>(cfg, kind, c, epi, st) : conv_typed<float>(cfg, kind, c, epi, st);
}

}  // namespace gcp
