// Device-side building blocks shared by the dense and convolution kernels:
// MFMA operand types and the fused epilogues of the GCP-CROWN passes
// (arXiv 2208.05740, Theorem 3.1 with Lemma A.1; Adam of Appendix C.1).
//
// An epilogue sees the elements one lane holds after the MFMA K loop:
// R GEMM rows x TN GEMM columns.  LaneCoords maps them to (batch row r,
// neuron j of the node).  For dense layers (PE = false) the neuron depends
// on the column only and the R rows come in aligned groups of 4 consecutive
// batch rows; for convolutions (PE = true) every element has its own neuron
// (channel x spatial position) and all R rows belong to one batch row.
//
// Each epilogue is split in two: load() fetches everything that does not
// depend on the GEMM result (neuron data, cut gathers, stored a_hat, alpha
// and its moments, split overrides); apply() combines it with the
// accumulator and stores.  Frag holds the per-lane state between the two.
#pragma once
#include "gcp_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace gcp {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Memory that no thread writes while a kernel runs, read through the
// constant address space: a wave-uniform address then becomes a scalar load,
// and pointers read from it are known to address global memory.
// (The host pass only type-checks this code and has no address spaces.)
#if defined(__HIP_DEVICE_COMPILE__)
#define GCP_CONSTANT_AS __attribute__((address_space(4)))
#else
#define GCP_CONSTANT_AS
#endif
template <typename T>
__device__ inline const GCP_CONSTANT_AS T* cst(const T* p) {
  return (const GCP_CONSTANT_AS T*)p;
}

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
template <typename T> __device__ inline float from_t(T x);
template <> __device__ inline float from_t<float>(float x) { return x; }
template <> __device__ inline float from_t<bf16>(bf16 x) { return (float)x; }

// Keep the first `keep` elements of a 16-byte operand vector, zero the rest:
// columns >= K of a row are padding whose bytes may hold data of the other
// operand precision (buffers are shared by the bf16 and fp32 passes), so the
// K tail is masked explicitly instead of relying on zero padding.
template <typename T>
__device__ inline uint4 mask_tail(uint4 v, int keep) {
  T e[16 / sizeof(T)];
  *(uint4*)e = v;
#pragma unroll
  for (int q = 0; q < (int)(16 / sizeof(T)); ++q)
    if (q >= keep) e[q] = to_t<T>(0.f);
  return *(const uint4*)e;
}

// ------------------------------------------------------------------ output sinks
// Where an epilogue puts the per-row activation it produces (Lambda in the
// bound pass, d a_hat in the adjoint, sign(v) in the concretisation): the
// [M][ld] global buffer of a per-layer launch, or a row-major buffer in the
// workgroup's dynamic LDS (rows row0 .. of the tile, pitch ld elements,
// starting `off` bytes in) in the fused chain kernel.
extern __shared__ __attribute__((aligned(16))) unsigned char gcp_smem[];
template <typename T>
struct GlobalSink {
  T* base;
  __device__ inline void operator()(size_t ij, int, int, T v) const { base[ij] = v; }
};
template <typename T>
struct LdsSink {
  int off, row0, ld;
  __device__ inline void operator()(size_t, int row, int j, T v) const {
    *(T*)(gcp_smem + off + ((row - row0) * ld + j) * (int)sizeof(T)) = v;
  }
};

// ------------------------------------------------------------------ helpers
__device__ inline double wave_sum16(double v) {
  // sum over the 16 lanes that share lane/16 (lane bits 0..3)
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 8, 64);
  return v;
}

template <int R, int TN, bool PE>
struct LaneCoords {
  int r[R];        // batch row of GEMM row q (may be >= M in a ragged tile)
  int j[TN][R];    // neuron of element (k, q); for PE == false only j[k][0] is used
};

#define GCP_QC(q) (PE ? (q) : 0)

// Per-column words of a dense lane fetched before the GEMM's K loop (the
// neuron's kind word and its cut-entry range): the loads that the rank- and
// cut-dependent loads of the epilogue wait on, issued early so their
// latency hides under the K loop.  Columns >= N hold kind 0 and an empty
// range.
template <int TN>
struct ColPre {
  int kind[TN];
  int2 rng[TN];
};
template <int TN>
__device__ inline void col_prefetch(ColPre<TN>& p, const NodeDev& nd, const CutCol& cc, const int (&col)[TN], int N) {
#pragma unroll
  for (int k = 0; k < TN; ++k) {
    const bool v = col[k] < N;
    p.kind[k] = v ? nd.kind[col[k]] : 0;
    p.rng[k] = (v && cc.rng) ? cc.rng[col[k]] : make_int2(0, 0);
  }
}

// Row indices of a lane: rv = element row is real (< M); rc = row clamped
// below M, for row-major [M][.] buffers; rr = row for the row-minor [.][mp]
// buffers.  Dense lanes keep groups of 4 consecutive rows whole so 16-byte
// accesses stay aligned -- a group starting below mp lies entirely below mp
// (mp is a multiple of 16), else it is moved to rows 0..3.
template <int R, bool PE>
__device__ inline void lane_rows(const int (&rows)[R], int M, int mp, int (&rr)[R], int (&rc)[R], bool (&rv)[R]) {
#pragma unroll
  for (int q = 0; q < R; ++q) {
    rv[q] = rows[q] < M;
    rc[q] = rv[q] ? rows[q] : 0;
    if constexpr (!PE && R % 4 == 0) rr[q] = rows[q - q % 4] < mp ? rows[q] : q % 4;
    else rr[q] = rc[q];
  }
}

// gamma^T X (X in {G, H, Q}) at the lane's elements of column slot k; gamma
// is read from its transposed copy [N][mp].  Dense: one cut-entry list per
// column, four consecutive rows per 16-byte load.  PE: per element.
template <int R, bool PE>
__device__ inline void gather_cuts(const CutCol& cc, const float* __restrict__ gammaT, int mp, const int (&jq)[R],
                                   const bool (&jv)[R], const int (&rr)[R], float (&sG)[R], float (&sH)[R],
                                   float (&sQ)[R], const int2* rg_pre = nullptr) {
#pragma unroll
  for (int q = 0; q < R; ++q) sG[q] = sH[q] = sQ[q] = 0.f;
  if (!cc.rng) return;
  if constexpr (!PE) {
    if (!jv[0]) return;
    const int2 rg = rg_pre ? *rg_pre : cc.rng[jq[0]];
    // kCutStep entries per step: their entry loads, then their gamma loads,
    // are issued together (a neuron's list is walked in order, so the sums
    // are the same as one entry at a time; a missing entry adds 0)
    constexpr int kCutStep = 2;
    for (int e0 = rg.x; e0 < rg.y; e0 += kCutStep) {
      float4 en[kCutStep];
#pragma unroll
      for (int t = 0; t < kCutStep; ++t) en[t] = cc.ent[e0 + t < rg.y ? e0 + t : e0];
      float g[kCutStep][R];
#pragma unroll
      for (int t = 0; t < kCutStep; ++t) {
        const float* gk = gammaT + (size_t)__float_as_int(en[t].w) * mp;
        if constexpr (R % 4 == 0) {
#pragma unroll
          for (int q = 0; q < R; q += 4) {
            const float4 v = *(const float4*)(gk + rr[q]);
            g[t][q] = v.x; g[t][q + 1] = v.y; g[t][q + 2] = v.z; g[t][q + 3] = v.w;
          }
        } else {
#pragma unroll
          for (int q = 0; q < R; ++q) g[t][q] = gk[rr[q]];
        }
      }
#pragma unroll
      for (int t = 0; t < kCutStep; ++t) {
        const bool live = e0 + t < rg.y;
        const float ch = live ? en[t].x : 0.f, cg = live ? en[t].y : 0.f, cq = live ? en[t].z : 0.f;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          sG[q] += g[t][q] * cg;
          sH[q] += g[t][q] * ch;
          sQ[q] += g[t][q] * cq;
        }
      }
    }
  } else {
    int2 rg[R];
#pragma unroll
    for (int q = 0; q < R; ++q) rg[q] = jv[q] ? cc.rng[jq[q]] : make_int2(0, 0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      for (int e = rg[q].x; e < rg[q].y; ++e) {
        const float4 en = cc.ent[e];
        const float g = gammaT[(size_t)__float_as_int(en.w) * mp + rr[q]];
        sG[q] += g * en.y;
        sH[q] += g * en.x;
        sQ[q] += g * en.z;
      }
    }
  }
}

// floor(r / S) for 0 <= r < 2^31 through a double reciprocal, exact after a
// one-step correction (cheaper than an integer division)
__device__ inline int div_rows(int r, int S, double inv_S) {
  int q = (int)((double)r * inv_S);
  const int rem = r - q * S;
  return q + (rem >= S ? 1 : (rem < 0 ? -1 : 0));
}

// Adam step lr * m_hat / (sqrt(v_hat) + eps): the bias corrections come as
// reciprocals and the last quotient uses the hardware reciprocal (~1 ulp).
// The step only moves the iterate; its bound is computed exactly later.
__device__ inline float adam_step(float lr, float mm, float vv, float ibc1, float ibc2, float eps) {
  return lr * (mm * ibc1) * __builtin_amdgcn_rcpf(sqrtf(vv * ibc2) + eps);
}

// effective class and split slot of each element (row, neuron)
template <int R>
__device__ inline void split_class(const RowParams& rp, int rank, int cls, int rc, int* c, int* slot) {
  int m = 0;
  if (rank >= 0 && rp.mask) m = rp.mask[(size_t)div_rows(rc, rp.S, rp.inv_S) * rp.n_I + rank];
  *slot = m > 0 ? m - 1 : (m < 0 ? -m - 1 : -1);
  *c = m > 0 ? (int)ACTIVE : (m < 0 ? (int)INACTIVE : cls);
}

// ------------------------------------------------------------------ bound
// Theorem 3.1 relaxation of one ReLU node: a_hat = GEMM + acc_in + gamma^T G,
// Lambda and the row constant (bias, h, z-fixed Q terms).  PI: pi of an
// unstable neuron is rho * [-a_hat]_+ with rho = rp.rho (Appendix A: any pi
// in [0, [-a_hat]_+] is a feasible dual point) instead of Lemma A.1's pi*.
template <typename T, bool PI = false>
struct BoundEpi {
  BoundEpiArgs a;
  template <int R, int TN, bool PE> struct Frag {
    int rc[R];
    bool ev[TN][R];                       // element valid
    float bj[TN][PE ? R : 1], lj[TN][PE ? R : 1], uj[TN][PE ? R : 1], iul[TN][PE ? R : 1];
    float aoff[TN][R];   // acc_in + gamma^T G: added to the GEMM value -> a_hat
    float tadd[TN][R];   // gamma^T H and the split term: added to Lambda
    float sQ[TN][R];     // gamma^T Q
    float al[TN][R];     // alpha (unstable) or 0
    float rh[TN][PI ? R : 1];   // rho (PI only)
    int8_t c[TN][R];     // effective class
  };
  static constexpr bool kColPre = true;
  __device__ inline const NodeDev& col_node() const { return a.nd; }
  __device__ inline const CutCol& col_cuts() const { return a.cc; }
  template <int R, int TN, bool PE>
  __device__ inline void load(Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc, int M, int N,
                              const ColPre<TN>* pre = nullptr) const {
    const NodeDev& nd = a.nd;
    const RowParams& rp = a.rp;
    int rr[R];
    bool rv[R];
    lane_rows<R, PE>(lc.r, M, rp.mp, rr, f.rc, rv);
    // issue order: loads that need no other load first, then those addressed
    // by the neuron's rank or split slot, then the cut gathers
    int jq[TN][R], kv[TN][PE ? R : 1];
    bool jv[TN][R];
#pragma unroll
    for (int k = 0; k < TN; ++k) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        jv[k][q] = lc.j[k][GCP_QC(q)] < N;
        jq[k][q] = jv[k][q] ? lc.j[k][GCP_QC(q)] : 0;
        f.ev[k][q] = jv[k][q] && rv[q];
      }
#pragma unroll
      for (int q = 0; q < (PE ? R : 1); ++q) {
        const int j = jq[k][q];
        const float4 nr = nd.rec[j];
        f.lj[k][q] = nr.x; f.uj[k][q] = nr.y; f.iul[k][q] = nr.z; f.bj[k][q] = nr.w;
        kv[k][q] = (!PE && pre) ? pre->kind[k] : nd.kind[j];
      }
#pragma unroll
      for (int q = 0; q < R; ++q)
        f.aoff[k][q] = a.acc_in ? a.acc_in[(size_t)f.rc[q] * nd.ld + jq[k][GCP_QC(q)]] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < TN; ++k)
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int rk = kind_rank(kv[k][GCP_QC(q)]);
        int c, slot;
        split_class<R>(rp, rk, kind_cls(kv[k][GCP_QC(q)]), f.rc[q], &c, &slot);
        f.al[k][q] = rk >= 0 ? rp.alpha[(size_t)f.rc[q] * rp.n_I + rk] : 0.f;
        if constexpr (PI) f.rh[k][q] = rk >= 0 ? rp.rho[(size_t)f.rc[q] * rp.n_I + rk] : 0.f;
        const float bv = slot >= 0 ? rp.beta[(size_t)f.rc[q] * rp.K + slot] : 0.f;
        f.tadd[k][q] = c == ACTIVE ? -bv : (c == INACTIVE ? bv : 0.f);   // split term
        f.c[k][q] = (int8_t)c;
      }
#pragma unroll
    for (int k = 0; k < TN; ++k) {
      float sG[R], sH[R];
      gather_cuts<R, PE>(a.cc, rp.gammaT, rp.mp, jq[k], jv[k], rr, sG, sH, f.sQ[k], pre ? &pre->rng[k] : nullptr);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        f.aoff[k][q] = f.aoff[k][q] + sG[q];     // acc_in + gamma^T G
        f.tadd[k][q] = sH[q] + f.tadd[k][q];     // gamma^T H + split term
      }
    }
  }
  template <int R, int TN, bool PE>
  __device__ inline void apply(const Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc,
                               const float (&val)[TN][R], double (&rs)[R], int M, int N) const {
    apply_to<R, TN, PE>(f, lc, val, rs, M, N, GlobalSink<T>{(T*)a.lam_out});
  }
  // Lambda goes to `lam`; a_hat (if kept) to a.ahat_out
  template <int R, int TN, bool PE, class Sink>
  __device__ inline void apply_to(const Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc,
                                  const float (&val)[TN][R], double (&rs)[R], int M, int N, const Sink& lam_sink) const {
    const NodeDev& nd = a.nd;
#pragma unroll
    for (int k = 0; k < TN; ++k) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int qc = GCP_QC(q);
        const float ah = val[k][q] + f.aoff[k][q];   // a_hat = Lambda^(i+1) W + gamma^T G
        float lam, konst;
        if (f.c[k][q] == ACTIVE) {                   // x_hat = x, z = 1
          lam = ah + f.tadd[k][q];
          konst = f.sQ[k][q];
        } else if (f.c[k][q] == INACTIVE) {          // x_hat = 0, z = 0
          lam = f.tadd[k][q];
          konst = 0.f;
        } else {                                     // Lemma A.1, C = [-a_hat]_+, q = -s
          const float n = fmaxf(-ah, 0.f), p = fmaxf(ah, 0.f), sq = f.sQ[k][q];
          float pi, h;
          if constexpr (PI) {                        // h(pi) = l pi - [u (n - pi) + l pi - s]_+
            const float uj = f.uj[k][qc], lj = f.lj[k][qc];
            pi = f.rh[k][q] * n;
            h = lj * pi - fmaxf(uj * n - (uj - lj) * pi - sq, 0.f);
          } else if (sq >= f.uj[k][qc] * n) { pi = 0.f; h = 0.f; }
          else if (sq <= f.lj[k][qc] * n) { pi = n; h = sq; }
          else { pi = (f.uj[k][qc] * n - sq) * f.iul[k][qc]; h = f.lj[k][qc] * pi; }
          lam = f.al[k][q] * p - pi + f.tadd[k][q];
          konst = h;
        }
        if (f.ev[k][q]) {
          const size_t ij = (size_t)f.rc[q] * nd.ld + lc.j[k][qc];
          lam_sink(ij, f.rc[q], lc.j[k][qc], to_t<T>(lam));
          if (a.ahat_out) ((T*)a.ahat_out)[ij] = to_t<T>(ah);
          rs[q] += (double)lam * (double)f.bj[k][qc] + (double)konst;
        }
      }
    }
  }
};

// ------------------------------------------------------------------ a_hat only
// a_hat = GEMM + acc_in + gamma^T G recomputed for the adjoint instead of
// stored by the bound pass: the same sum as BoundEpi forms, written to
// a.ahat_out (operand type T); nothing else is read or written.
template <typename T>
struct AhatEpi {
  BoundEpiArgs a;
  static constexpr bool kColPre = false;
  template <int R, int TN, bool PE> struct Frag {
    int rc[R];
    bool ev[TN][R];
    float aoff[TN][R];
  };
  template <int R, int TN, bool PE>
  __device__ inline void load(Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc, int M, int N) const {
    const RowParams& rp = a.rp;
    int rr[R];
    bool rv[R];
    lane_rows<R, PE>(lc.r, M, rp.mp, rr, f.rc, rv);
#pragma unroll
    for (int k = 0; k < TN; ++k) {
      int jq[R];
      bool jv[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        jv[q] = lc.j[k][GCP_QC(q)] < N;
        jq[q] = jv[q] ? lc.j[k][GCP_QC(q)] : 0;
        f.ev[k][q] = jv[q] && rv[q];
      }
      float sG[R], sH[R], sQ[R];
      gather_cuts<R, PE>(a.cc, rp.gammaT, rp.mp, jq, jv, rr, sG, sH, sQ);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const float pre = a.acc_in ? a.acc_in[(size_t)f.rc[q] * a.nd.ld + jq[GCP_QC(q)]] : 0.f;
        f.aoff[k][q] = pre + sG[q];
      }
    }
  }
  template <int R, int TN, bool PE>
  __device__ inline void apply(const Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc,
                               const float (&val)[TN][R], double (&rs)[R], int M, int N) const {
#pragma unroll
    for (int k = 0; k < TN; ++k)
#pragma unroll
      for (int q = 0; q < R; ++q)
        if (f.ev[k][q])
          ((T*)a.ahat_out)[(size_t)f.rc[q] * a.nd.ld + lc.j[k][GCP_QC(q)]] = to_t<T>(val[k][q] + f.aoff[k][q]);
  }
};

// ------------------------------------------------------------------ concretisation
// v = GEMM + gamma^T G0 over the input box: x0.v - eps*|v|_1 into the row
// constant, sign(v) for the adjoint, input-cut gradient pieces.
struct ConcEpi {
  ConcEpiArgs a;
  static constexpr bool kColPre = false;
  template <int R, int TN, bool PE> struct Frag {
    int rr[R], rc[R];
    bool ev[TN][R];
    float sG[TN][R];
    double xj[TN][PE ? R : 1];   // x0 of the element's input coordinate
  };
  template <int R, int TN, bool PE>
  __device__ inline void load(Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc, int M, int N) const {
    bool rv[R];
    lane_rows<R, PE>(lc.r, M, a.rp.mp, f.rr, f.rc, rv);
#pragma unroll
    for (int k = 0; k < TN; ++k) {
      int jq[R];
      bool jv[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        jv[q] = lc.j[k][GCP_QC(q)] < N;
        jq[q] = jv[q] ? lc.j[k][GCP_QC(q)] : 0;
        f.ev[k][q] = jv[q] && rv[q];
      }
      // x0 is read here, not next to the stores of apply: int8 stores may
      // alias it, which would force one reload per element after each store
#pragma unroll
      for (int q = 0; q < (PE ? R : 1); ++q) f.xj[k][q] = a.x0[jq[q]];
      float sH[R], sQ[R];
      gather_cuts<R, PE>(a.cc, a.rp.gammaT, a.rp.mp, jq, jv, f.rr, f.sG[k], sH, sQ);
    }
  }
  template <int R, int TN, bool PE>
  __device__ inline void apply(const Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc,
                               const float (&val)[TN][R], double (&rs)[R], int M, int N) const {
    apply_to<R, TN, PE>(f, lc, val, rs, M, N, GlobalSink<int8_t>{a.sign_out});
  }
  // sign(v) goes to `sign_sink` (when a.sign_out is set)
  template <int R, int TN, bool PE, class Sink>
  __device__ inline void apply_to(const Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc,
                                  const float (&val)[TN][R], double (&rs)[R], int M, int N, const Sink& sign_sink) const {
#pragma unroll
    for (int k = 0; k < TN; ++k) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        if (!f.ev[k][q]) continue;
        const int j = lc.j[k][GCP_QC(q)];
        const double xj = f.xj[k][GCP_QC(q)];
        const float v = val[k][q] + f.sG[k][q];
        const float sg = (v > 0.f) ? 1.f : ((v < 0.f) ? -1.f : 0.f);
        if (a.sign_out) sign_sink((size_t)f.rc[q] * a.ld + j, f.rc[q], j, (int8_t)sg);
        if (a.contrib && a.cc.rng) {
          const float dv = (float)(xj - a.eps * (double)sg);
          const int2 rg = a.cc.rng[j];
          for (int e = rg.x; e < rg.y; ++e)
            a.contrib[(size_t)a.cc.pos[e] * a.rp.mp + f.rr[q]] = a.cc.ent[e].y * dv;
        }
        const double vd = (double)v;
        rs[q] += xj * vd - a.eps * fabs(vd);
      }
    }
  }
};

// ------------------------------------------------------------------ adjoint
// d bound / d Lambda arrives as the GEMM value; the relaxation's derivative
// gives d bound / d a_hat (operand of the next adjoint GEMM), the gradient
// pieces of the cuts, and d/d alpha, d/d beta -- applied by projected Adam in
// place or written out.  PI: the explicit-pi relaxation of BoundEpi<T,
// true>, with d/d rho applied to rho like alpha's.
template <typename T, bool PI = false>
struct AdjEpi {
  AdjEpiArgs a;
  template <int R, int TN, bool PE> struct Frag {
    int rr[R], rc[R];
    bool ev[TN][R];
    float lj[TN][PE ? R : 1], uj[TN][PE ? R : 1], iul[TN][PE ? R : 1], addj[TN][PE ? R : 1];
    int rk[TN][R];
    float ah[TN][R];     // stored a_hat
    float pre[TN][R];    // acc_in
    float sQ[TN][R];
    float al[TN][R], ma[TN][R], va[TN][R];
    float rh[TN][PI ? R : 1], mr[TN][PI ? R : 1], vr[TN][PI ? R : 1];
    int2 rgc[TN];        // prefetched cut-entry range of the column (GEMM lanes)
    bool has_rgc;        // rgc set; a compile-time constant after inlining
    int8_t c[TN][R], slot[TN][R];
  };
  static constexpr bool kColPre = true;
  __device__ inline const NodeDev& col_node() const { return a.nd; }
  __device__ inline const CutCol& col_cuts() const { return a.cc; }
  template <int R, int TN, bool PE>
  __device__ inline void load(Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc, int M, int N,
                              const ColPre<TN>* pre = nullptr) const {
    const NodeDev& nd = a.nd;
    const RowParams& rp = a.rp;
    bool rv[R];
    lane_rows<R, PE>(lc.r, M, rp.mp, f.rr, f.rc, rv);
    const bool adam = a.adam.enabled;
    // issue order: loads that need no other load first, then those addressed
    // by the neuron's rank, then the cut gathers
    int jq[TN][R], kv[TN][PE ? R : 1];
    bool jv[TN][R];
#pragma unroll
    for (int k = 0; k < TN; ++k) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        jv[k][q] = lc.j[k][GCP_QC(q)] < N;
        jq[k][q] = jv[k][q] ? lc.j[k][GCP_QC(q)] : 0;
        f.ev[k][q] = jv[k][q] && rv[q];
      }
#pragma unroll
      for (int q = 0; q < (PE ? R : 1); ++q) {
        const int j = jq[k][q];
        const float4 nr = nd.rec[j];
        f.lj[k][q] = nr.x; f.uj[k][q] = nr.y; f.iul[k][q] = nr.z; f.addj[k][q] = a.add_vec[j];
        kv[k][q] = (!PE && pre) ? pre->kind[k] : nd.kind[j];
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int j = jq[k][GCP_QC(q)];
        f.ah[k][q] = from_t<T>(((const T*)a.ahat)[(size_t)f.rc[q] * nd.ld + j]);
        f.pre[k][q] = a.acc_in ? a.acc_in[(size_t)f.rc[q] * nd.ld + j] : 0.f;
      }
    }
#pragma unroll
    for (int k = 0; k < TN; ++k)
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int rk = kind_rank(kv[k][GCP_QC(q)]);
        int c, slot;
        split_class<R>(rp, rk, kind_cls(kv[k][GCP_QC(q)]), f.rc[q], &c, &slot);
        f.rk[k][q] = rk;
        const size_t ia = (size_t)f.rc[q] * rp.n_I + (rk >= 0 ? rk : 0);
        f.al[k][q] = rk >= 0 ? rp.alpha[ia] : 0.f;
        f.ma[k][q] = (rk >= 0 && adam) ? a.m_alpha[ia] : 0.f;
        f.va[k][q] = (rk >= 0 && adam) ? a.v_alpha[ia] : 0.f;
        if constexpr (PI) {
          f.rh[k][q] = rk >= 0 ? rp.rho[ia] : 0.f;
          f.mr[k][q] = (rk >= 0 && adam) ? a.m_rho[ia] : 0.f;
          f.vr[k][q] = (rk >= 0 && adam) ? a.v_rho[ia] : 0.f;
        }
        f.c[k][q] = (int8_t)c;
        f.slot[k][q] = (int8_t)slot;
      }
#pragma unroll
    for (int k = 0; k < TN; ++k) {
      float sG[R], sH[R];
      f.has_rgc = !PE && pre != nullptr;
      if (f.has_rgc) f.rgc[k] = pre->rng[k];
      gather_cuts<R, PE>(a.cc, rp.gammaT, rp.mp, jq[k], jv[k], f.rr, sG, sH, f.sQ[k],
                         f.has_rgc ? &f.rgc[k] : nullptr);
    }
  }
  template <int R, int TN, bool PE>
  __device__ inline void apply(const Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc,
                               const float (&val)[TN][R], double (&rs)[R], int M, int N) const {
    apply_to<R, TN, PE>(f, lc, val, rs, M, N, GlobalSink<T>{(T*)a.dahat_out});
  }
  // d a_hat goes to `da_sink` (when a.dahat_out is set)
  template <int R, int TN, bool PE, class Sink>
  __device__ inline void apply_to(const Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc,
                                  const float (&val)[TN][R], double (&rs)[R], int M, int N, const Sink& da_sink) const {
    const NodeDev& nd = a.nd;
    const RowParams& rp = a.rp;
    float lr_a = 0.f, lr_m = 0.f, ibc1 = 1.f, ibc2 = 1.f;
    if (a.adam.enabled) {
      lr_a = a.adam.consts[0]; lr_m = a.adam.consts[1]; ibc1 = a.adam.consts[2]; ibc2 = a.adam.consts[3];
    }
    const float b1 = a.adam.b1, b2 = a.adam.b2, aeps = a.adam.eps;
    // dense lanes hold four consecutive rows per group: their cut-gradient
    // pieces go out as one 16-byte store per entry after the row loop
    constexpr bool kVecContrib = !PE && R % 4 == 0;
#pragma unroll
    for (int k = 0; k < TN; ++k) {
      float cA[R], cL[R], cS[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int qc = GCP_QC(q);
        const float dL = a.gemm_scale * val[k][q] + f.addj[k][qc] + f.pre[k][q];
        float dA, dS, gA = 0.f, gR = 0.f;
        const int c = f.c[k][q];
        if (c == ACTIVE) {
          dA = dL; dS = 1.f;
        } else if (c == INACTIVE) {
          dA = 0.f; dS = 0.f;
        } else {
          const float x = f.ah[k][q], n = fmaxf(-x, 0.f), p = fmaxf(x, 0.f), sq = f.sQ[k][q];
          const float pos = x > 0.f ? 1.f : 0.f, neg = x < 0.f ? 1.f : 0.f;
          const float uj = f.uj[k][qc], lj = f.lj[k][qc], iul = f.iul[k][qc], al = f.al[k][q];
          float dLda, dhda, dLds, dhds;
          if constexpr (PI) {
            // Lambda = alpha p - rho n + t,  h = l rho n - [w n - s]_+,  w = u - (u - l) rho
            const float rho = f.rh[k][q], w = uj - (uj - lj) * rho;
            const float ind = w * n - sq > 0.f ? 1.f : 0.f;
            dLda = al * pos + rho * neg;
            dhda = neg * (ind * w - lj * rho);
            dLds = 0.f;
            dhds = ind;
            gR = n * (lj + ind * (uj - lj) - dL);
          } else if (sq >= uj * n) { dLda = al * pos; dhda = 0.f; dLds = 0.f; dhds = 0.f; }
          else if (sq <= lj * n) { dLda = al * pos + neg; dhda = 0.f; dLds = 0.f; dhds = 1.f; }
          else {
            dLda = al * pos + uj * iul * neg;
            dhda = -lj * uj * iul * neg;
            dLds = iul;
            dhds = -lj * iul;
          }
          dA = dL * dLda + dhda;
          dS = dL * dLds + dhds;
          gA = dL * p;
        }
        cA[q] = dA; cL[q] = dL; cS[q] = dS;
        if (!f.ev[k][q]) continue;
        const int j = lc.j[k][qc];
        const size_t ij = (size_t)f.rc[q] * nd.ld + j;
        if (a.dahat_out) da_sink(ij, f.rc[q], j, to_t<T>(dA));
        if (!kVecContrib && a.contrib && a.cc.rng) {
          const int2 rg = a.cc.rng[j];
          for (int e = rg.x; e < rg.y; ++e) {
            const float4 en = a.cc.ent[e];
            a.contrib[(size_t)a.cc.pos[e] * rp.mp + f.rr[q]] = en.y * dA + en.x * dL + en.z * dS;
          }
        }
        const int rk = f.rk[k][q];
        if (rk >= 0) {
          const size_t ia = (size_t)f.rc[q] * rp.n_I + rk;
          if (a.adam.enabled) {
            const float mm = b1 * f.ma[k][q] + (1.f - b1) * gA;
            const float vv = b2 * f.va[k][q] + (1.f - b2) * gA * gA;
            a.m_alpha[ia] = mm;
            a.v_alpha[ia] = vv;
            const float stp = adam_step(lr_a, mm, vv, ibc1, ibc2, aeps);
            a.alpha_rw[ia] = fminf(fmaxf(f.al[k][q] + stp, 0.f), 1.f);
            if constexpr (PI) {
              const float mr = b1 * f.mr[k][q] + (1.f - b1) * gR;
              const float vr = b2 * f.vr[k][q] + (1.f - b2) * gR * gR;
              a.m_rho[ia] = mr;
              a.v_rho[ia] = vr;
              a.rho_rw[ia] = fminf(fmaxf(f.rh[k][q] + adam_step(lr_a, mr, vr, ibc1, ibc2, aeps), 0.f), 1.f);
            }
          } else {
            a.d_alpha[ia] = gA;
            if constexpr (PI) a.d_rho[ia] = gR;
          }
        }
        const int sl = f.slot[k][q];
        if (sl >= 0) {
          const size_t ib = (size_t)f.rc[q] * rp.K + sl;
          const float gB = (c == ACTIVE) ? -dL : dL;
          if (a.adam.enabled) {
            const float mm = b1 * a.m_beta[ib] + (1.f - b1) * gB;
            const float vv = b2 * a.v_beta[ib] + (1.f - b2) * gB * gB;
            a.m_beta[ib] = mm;
            a.v_beta[ib] = vv;
            const float stp = adam_step(lr_m, mm, vv, ibc1, ibc2, aeps);
            a.beta_rw[ib] = fmaxf(a.beta_rw[ib] + stp, 0.f);
          } else {
            a.d_beta[ib] = gB;
          }
        }
      }
      if constexpr (kVecContrib) {
        // rows of a group are consecutive and the group lies below mp; rows
        // in [M, mp) are padding of the contribution buffer, never read
        const int j = lc.j[k][0];
        if (a.contrib && a.cc.rng && j < N) {
          const int2 rg = f.has_rgc ? f.rgc[k] : a.cc.rng[j];
          for (int e = rg.x; e < rg.y; ++e) {
            const float4 en = a.cc.ent[e];
            float* dst = a.contrib + (size_t)a.cc.pos[e] * rp.mp;
#pragma unroll
            for (int q = 0; q < R; q += 4) {
              if (lc.r[q] >= M) continue;
              float4 v;
              v.x = en.y * cA[q] + en.x * cL[q] + en.z * cS[q];
              v.y = en.y * cA[q + 1] + en.x * cL[q + 1] + en.z * cS[q + 1];
              v.z = en.y * cA[q + 2] + en.x * cL[q + 2] + en.z * cS[q + 2];
              v.w = en.y * cA[q + 3] + en.x * cL[q + 3] + en.z * cS[q + 3];
              *(float4*)(dst + lc.r[q]) = v;
            }
          }
        }
      }
    }
  }
};

// ------------------------------------------------------------------ store
// out = scale * GEMM (+ acc_in): partial sums of a node with several edges
struct StoreEpi {
  StoreEpiArgs a;
  static constexpr bool kColPre = false;
  template <int R, int TN, bool PE> struct Frag {
    int rc[R];
    bool ev[TN][R];
    float pre[TN][R];
  };
  template <int R, int TN, bool PE>
  __device__ inline void load(Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc, int M, int N) const {
#pragma unroll
    for (int k = 0; k < TN; ++k)
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int j = lc.j[k][GCP_QC(q)];
        f.ev[k][q] = lc.r[q] < M && j < N;
        f.rc[q] = lc.r[q] < M ? lc.r[q] : 0;
        f.pre[k][q] = (a.acc_in && f.ev[k][q]) ? a.acc_in[(size_t)f.rc[q] * a.ld + j] : 0.f;
      }
  }
  template <int R, int TN, bool PE>
  __device__ inline void apply(const Frag<R, TN, PE>& f, const LaneCoords<R, TN, PE>& lc,
                               const float (&val)[TN][R], double (&rs)[R], int M, int N) const {
#pragma unroll
    for (int k = 0; k < TN; ++k)
#pragma unroll
      for (int q = 0; q < R; ++q)
        if (f.ev[k][q]) a.out[(size_t)f.rc[q] * a.ld + lc.j[k][GCP_QC(q)]] = a.scale * val[k][q] + f.pre[k][q];
  }
};

// ------------------------------------------------------------------ multipliers
// One (cut k, row r) of the gamma update.  The Adam state is read before the
// sum and the cut's entry pieces four at a time, so the loads are in flight
// together; the pieces are still added one by one in entry order.
__device__ inline void gamma_one(int k, int r, int M, int mp, int N, const int32_t* row_ptr, const float* contrib,
                                 const double* d, float* gammaT, float* d_gamma, float* m, float* v,
                                 const AdamArgs& adam) {
  const int e0 = row_ptr[k], e1 = row_ptr[k + 1];
  const size_t im = (size_t)k * M + r;
  float m0 = 0.f, v0 = 0.f, x0 = 0.f;
  float* gp = adam.enabled ? gammaT + (size_t)k * mp + r : nullptr;
  if (adam.enabled) {
    m0 = m[im];
    v0 = v[im];
    x0 = *gp;
  }
  double g = -d[k];
  for (int e = e0; e < e1; e += 4) {
    float c[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) c[t] = e + t < e1 ? contrib[(size_t)(e + t) * mp + r] : 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (e + t < e1) g += (double)c[t];
  }
  if (adam.enabled) {
    const float lr = adam.consts[1], ibc1 = adam.consts[2], ibc2 = adam.consts[3];
    const float gf = (float)g;
    const float mm = adam.b1 * m0 + (1.f - adam.b1) * gf;
    const float vv = adam.b2 * v0 + (1.f - adam.b2) * gf * gf;
    m[im] = mm;
    v[im] = vv;
    *gp = fmaxf(x0 + adam_step(lr, mm, vv, ibc1, ibc2, adam.eps), 0.f);
  } else {
    d_gamma[(size_t)r * N + k] = (float)g;
  }
}

}  // namespace gcp
