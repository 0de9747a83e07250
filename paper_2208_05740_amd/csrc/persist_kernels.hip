// Persistent dataflow execution of recorded optimisation iterations
// (arXiv 2208.05740: the bound of Theorem 3.1 with Lemma A.1, its adjoint
// and the projected Adam ascent of Appendix C.1).
//
// Every (domain, spec row) is an independent problem, so within one
// iteration a launch over a panel of rows depends only on the earlier
// launches over the same rows; the layer-by-layer launch sequence of the
// per-layer path orders whole layers instead.  Here one launch runs every
// tile of every step of several iterations: workgroups claim items from a
// queue in schedule order (iteration, step, column tile, panel), wait until
// the item's panel has completed all tiles of the earlier steps (one
// monotone counter per panel), run the item with the per-layer kernels' own
// tile code and epilogues, and count it complete.  Layers, instances and
// iterations overlap wherever their rows allow it, with no launch
// boundaries.
//
// Forward progress: an item waits only for items that precede it in its
// queue, and a workgroup claims a few consecutive items at a time and runs
// them in order, so the earliest unfinished item of a queue always has its
// dependencies met and its workgroup resident.  Every wait is bounded
// (spin_ticks of the 100 MHz wall clock, 1 s by default); a wait that runs
// out raises an abort flag, and the first workgroup to raise it latches it
// for the host side and moves every claim head past the end (once, so the
// heads stay within the int range), at which every workgroup stops: a
// stalled launch ends instead of hanging (and the call's bounds become -inf).
//
// Ordering between workgroups: the producer of an item makes its stores
// complete, then bumps the panel counter; the consumer reads the counter,
// then invalidates what it might hold stale (an agent-scope acquire).  With
// xcd_sync == 0 the producer's side is an agent-scope release (its L2 is
// written back: valid whatever XCD either side runs on).  With xcd_sync == 1
// the queues are per XCD -- a workgroup serves the queue of the XCD it runs
// on (hardware register XCC_ID) and every panel belongs to one queue -- so
// producer and consumer share one L2 and the producer only waits for its
// stores to reach it (vmcnt 0).  Results are bit-identical to the per-layer
// launches: the same epilogue code runs on the same accumulators, which
// every tile shape sums over K in the same order.
#include "gcp_internal.h"
#include "epilogues.h"
#include "tiles.h"

#include <hip/hip_runtime.h>

#include <cstdlib>

namespace gcp {

namespace {

constexpr int kPersistClaim = 4;                // consecutive items per claim

template <typename T>
struct PersistCfg {
  static constexpr int BK = sizeof(T) == 4 ? 64 : 128;
  using Lds = TileLds<T, kPersistRows, 32, 2, BK>;
};

// s_waitcnt vmcnt(0): this wave's vector memory operations, stores included,
// have completed (gfx9 encoding: expcnt 7, lgkmcnt 15 left unconstrained).
__device__ inline void wait_vm_zero() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ inline int xcc_id() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return (int)(v & 0xf);
}

// The job tables are read-only while the kernel runs, so they are read
// through the constant address space: the compiler then knows that the
// pointers inside them address global memory and accesses through them are
// global instructions (read as generic pointers they would be flat ones,
// which also count against the LDS counter, so every LDS wait of the tile
// loop would wait for them too).
// (cst() in epilogues.h.)

template <typename T, class Epi>
__device__ inline void run_gemm(const GemmArgs& g, const Epi& e, int vt, bool sign, typename PersistCfg<T>::Lds& sm) {
  constexpr int BK = PersistCfg<T>::BK;
  if (sign) gemm_tile_lds<T, kPersistRows, 32, 2, 2, BK, true, Epi, true>(g, e, vt, sm);
  else gemm_tile_lds<T, kPersistRows, 32, 2, 2, BK, false, Epi, true>(g, e, vt, sm);
}

}  // namespace

// WPE: waves per SIMD the register allocation targets.  The tables are
// separate __restrict__ arguments: their fields can be reloaded instead of
// held in registers, and the pointers read from them are known to address
// global memory (plain loads and stores rather than flat ones).
template <typename T, bool XCD, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
persist_kernel(PersistArgs a, const PersistStep* __restrict__ steps, const int* __restrict__ qfirst,
               const GemmArgs* __restrict__ gemm_tab, const unsigned char* __restrict__ epi_tab,
               const ElemBoundJob* __restrict__ elem_tab, const GammaJob* __restrict__ gam_tab) {
  __shared__ typename PersistCfg<T>::Lds sm;
  __shared__ int s_first[kPersistMaxSteps + 1];
  __shared__ int s_claim, s_bad;
  const int tid = threadIdx.x;
  // Control flow of the item loop is uniform per wave (conditions read with
  // readfirstlane, the claim / wait / completion done by all of wave 0 with
  // one lane contributing): a lane-divergent branch around the loop's
  // barriers lets the compiler send part of a wave back to the barrier
  // before the claiming lane has run.
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int one = (tid & 63) == 0 ? 1 : 0;
  const int q = a.Q > 1 ? xcc_id() % a.Q : 0;
  const int ns = a.n_steps;
  for (int i = tid; i <= ns; i += 256) s_first[i] = qfirst[(size_t)q * (ns + 1) + i];
  __syncthreads();
  const int per_iter = __builtin_amdgcn_readfirstlane(s_first[ns]);
  const int total = per_iter * a.iters;
  int* head = a.sync + q;
  int* abort_flag = a.sync + a.Q;
  int* counters = a.sync + a.Q + 1;
  int c = 0, c_end = 0;              // claimed items [c, c_end) of this queue
  const int* seen_ctr = nullptr;     // wave 0: the last counter read, and its value
  int seen_val = 0;
  for (;;) {
    if (c == c_end) {
      // kPersistClaim consecutive items per claim (an abort adds
      // kPersistAbort to every head, so later claims fall past the end)
      if (wave == 0) {
        s_claim = __builtin_amdgcn_readfirstlane(
            __hip_atomic_fetch_add(head, one * kPersistClaim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        s_bad = 0;
      }
      __syncthreads();
      c = __builtin_amdgcn_readfirstlane(s_claim);
      if (c >= total || c < 0) break;
      c_end = min(c + kPersistClaim, total);
    }
    // wave-uniform values in scalar registers, so the step's tables are read
    // with scalar loads
    const int t = c / per_iter;
    const int li = c - t * per_iter;
    // the step: the last s with s_first[s] <= li (steps this queue has no
    // items of share their successor's first index)
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (__builtin_amdgcn_readfirstlane(s_first[mid]) <= li) lo = mid; else hi = mid - 1;
    }
    const PersistStep st = cst(steps)[lo];
    const int local = li - __builtin_amdgcn_readfirstlane(s_first[lo]);
    // items of a step run panel-minor: the column tiles of one panel are
    // n_own items apart, so consecutive claims take different panels and
    // a panel's tiles run side by side
    const int base = __builtin_amdgcn_readfirstlane(st.base);
    const int panels = __builtin_amdgcn_readfirstlane(st.panels);
    const int r = ((q - base) % a.Q + a.Q) % a.Q;   // first panel of this instance owned by queue q
    const int n_own = (panels - 1 - r) / a.Q + 1;   // panels of the instance owned by queue q (> 0 here)
    const int loc = local / n_own;
    const int j = local - loc * n_own;
    const int p = r + a.Q * j;
    int* ctr = counters + __builtin_amdgcn_readfirstlane(st.cnt0) + p;
    const int target = __builtin_amdgcn_readfirstlane(t * st.per_iter + st.wait);
    // wait until the panel has completed `target` items; an earlier read of
    // the same counter that already showed them needs no new read (the
    // acquire after that read covers them)
    if (wave == 0 && target > 0 && !(ctr == seen_ctr && seen_val >= target)) {
      const uint64_t t0 = wall_clock64();
      int bad = 0;
      int v = __builtin_amdgcn_readfirstlane(__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      while (v < target) {
        if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
          bad = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        if (wall_clock64() - t0 > a.spin_ticks) {
          // only the first workgroup to abort moves the heads (once per
          // launch, so they stay far below the int range)
          const int was = __builtin_amdgcn_readfirstlane(
              __hip_atomic_fetch_add(abort_flag, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
          if (was == 0) {
            __hip_atomic_store(a.latch, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int k = 0; k < a.Q; ++k)
              __hip_atomic_fetch_add(a.sync + k, one * kPersistAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          bad = 1;
          break;
        }
        v = __builtin_amdgcn_readfirstlane(__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      }
      seen_ctr = ctr;
      seen_val = v;
      s_bad = bad;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_bad)) break;
    const int iter = a.iter0 + t;
    const int kind = __builtin_amdgcn_readfirstlane(st.kind);
    const int job = __builtin_amdgcn_readfirstlane(st.job);
    const bool sign = __builtin_amdgcn_readfirstlane(st.sign) != 0;
    if (kind == PK_ELEM) {
      const ElemBoundJob jb = cst(elem_tab)[job];
      // item loc: rows kElemRows * (loc / ncb) .. of the panel, column block loc % ncb
      const int M = __builtin_amdgcn_readfirstlane(jb.a.rp.M);
      const int ncb = (__builtin_amdgcn_readfirstlane(jb.a.nd.size) + 255) / 256;
      const int r0 = p * kPersistRows + (loc / ncb) * kElemRows;
      if (r0 < M) bound_elem_rows<T, false, true>(jb.bcast, jb.src, jb.a, jb.partial, jb.slot0, r0, loc % ncb);
    } else if (kind == PK_GAMMA) {
      const GammaJob jb = cst(gam_tab)[job];
      AdamArgs ad = a.adam;
      ad.consts = a.adam.consts + 4 * iter;
      const int row = p * kPersistRows + (tid & (kPersistRows - 1));
      constexpr int lanes = 256 / kPersistRows;
      if (row < jb.M)
        for (int k = loc * 32 + tid / kPersistRows; k < min(loc * 32 + 32, jb.N); k += lanes)
          gamma_one(k, row, jb.M, jb.mp, jb.N, jb.row_ptr, jb.contrib, jb.d, jb.gammaT, nullptr, jb.m, jb.v, ad);
    } else {
      const GemmArgs g = cst(gemm_tab)[job];
      const unsigned char* blob = epi_tab + (size_t)job * kEpiBlob;
      const int vt = p * __builtin_amdgcn_readfirstlane(st.ipp) + loc;
      switch (kind) {
        case PK_BOUND: {
          const BoundEpiArgs ea = *cst((const BoundEpiArgs*)blob);
          run_gemm<T>(g, BoundEpi<T>{ea}, vt, false, sm);
          break;
        }
        case PK_CONC: {
          const ConcEpiArgs ea = *cst((const ConcEpiArgs*)blob);
          run_gemm<T>(g, ConcEpi{ea}, vt, false, sm);
          break;
        }
        case PK_STORE: {
          const StoreEpiArgs ea = *cst((const StoreEpiArgs*)blob);
          run_gemm<T>(g, StoreEpi{ea}, vt, sign, sm);
          break;
        }
        case PK_ADJ: {
          AdjEpiArgs ea = *cst((const AdjEpiArgs*)blob);
          ea.adam.consts = a.adam.consts + 4 * iter;
          run_gemm<T>(g, AdjEpi<T>{ea}, vt, sign, sm);
          break;
        }
        default: break;
      }
    }
    // completion: this workgroup's stores reach the level its consumers read
    // from, then the panel's counter moves (by one: one lane of wave 0 adds)
    if constexpr (XCD) wait_vm_zero();
    else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (wave == 0) __hip_atomic_fetch_add(ctr, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ++c;
  }
}

namespace {
// GCP_PERSIST_WPE = 4 (default) or 5: the register budget of the kernel
int persist_wpe() {
  const char* e = std::getenv("GCP_PERSIST_WPE");
  return (e && std::atoi(e) == 5) ? 5 : 4;
}
template <typename T, bool XCD>
const void* persist_fn(int wpe) {
  return wpe == 5 ? (const void*)persist_kernel<T, XCD, 5> : (const void*)persist_kernel<T, XCD, 4>;
}
const void* persist_fn(int bf16_mode, int xcd_sync, int wpe) {
  if (bf16_mode) return xcd_sync ? persist_fn<bf16, true>(wpe) : persist_fn<bf16, false>(wpe);
  return xcd_sync ? persist_fn<float, true>(wpe) : persist_fn<float, false>(wpe);
}
}  // namespace

__global__ void __launch_bounds__(256) persist_guard_kernel(const int* latch, double* bound, uint8_t* verified, int M) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r < M && *latch != 0) {
    bound[r] = -__builtin_inf();
    if (verified) verified[r] = 0;
  }
}
hipError_t launch_persist_guard(const int* latch, double* bound, uint8_t* verified, int M, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(persist_guard_kernel, dim3((M + 255) / 256), dim3(256), 0, st, latch, bound, verified, M);
  return hipGetLastError();
}

// The XCD each of n workgroups ran on (plan set-up: how many claim queues
// the launches can use).
__global__ void xcc_probe_kernel(int* out) {
  if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}
hipError_t launch_xcc_probe(int* out, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(xcc_probe_kernel, dim3(n), dim3(64), 0, st, out);
  return hipGetLastError();
}

int persist_grid(int bf16_mode, int xcd_sync) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, persist_fn(bf16_mode, xcd_sync, persist_wpe()), 256, 0) !=
      hipSuccess)
    return 0;
  return cus * per;
}

hipError_t launch_persist(int bf16_mode, const PersistArgs& a, int grid, hipStream_t st) {
  if (a.iters <= 0 || a.n_steps <= 0) return hipSuccess;
  if (a.n_steps > kPersistMaxSteps || a.Q < 1 || grid <= 0) return hipErrorInvalidValue;
  void* args[] = {(void*)&a, (void*)&a.steps, (void*)&a.qfirst, (void*)&a.gemm, (void*)&a.epi, (void*)&a.elem,
                  (void*)&a.gam};
  return hipLaunchKernel(persist_fn(bf16_mode, a.xcd_sync, persist_wpe()), dim3(grid), dim3(256), args, 0, st);
}

}  // namespace gcp
