// Internal declarations shared by the host runtime (gcp_api.cpp) and the
// gfx950 kernels (kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gcp {

typedef __bf16 bf16;

enum Cls : int8_t { INACTIVE = 0, ACTIVE = 1, UNSTABLE = 2 };

// Per-node constant data on the device.
struct NodeDev {
  int size;          // neurons
  int ld;            // row pitch of per-row activation buffers (multiple of 16)
  // per neuron {l, u, 1/(u-l), bias}: root bounds (fp32, outward rounded),
  // the reciprocal width for unstable neurons (else 0), the layer bias
  const float4* rec;
  const int32_t* kind;   // (rank + 1) * 4 + root class; rank = column in an alpha row, or -1
};
__host__ __device__ inline int kind_rank(int v) { return (v >> 2) - 1; }
__host__ __device__ inline int kind_cls(int v) { return v & 3; }

// Cut entries of one node in column (neuron) order: entries
// rng[j].x .. rng[j].y-1 touch neuron j.  Each merged entry carries the
// three coefficients of one (cut, node, neuron) and the cut index,
// {cH, cG, cQ, cut as int bits}, and its position in the cut-major order
// used by the gamma gradient.
struct CutCol {
  const int2* rng;         // [size], null if the node has no entries
  const float4* ent;
  const int32_t* pos;
};

// Per-row parameters of one call.  Row-indexed internal buffers use the
// "row-minor" layout [x][mp] (mp = M rounded up to 16) so that the rows a
// lane owns (4 consecutive per MFMA fragment) are one 16-byte access.
struct RowParams {
  int M, S, mp;
  const float* alpha; int n_I;      // [M][n_I]   (caller layout)
  const float* beta;  int K;        // [M][K]     (caller layout)
  const float* gammaT; int N;       // [N][mp]    (internal transposed copy)
  const int8_t* mask;               // [B][n_I]: 0, +(slot+1) x>=0, -(slot+1) x<=0
  double inv_S;                     // 1 / S (domain of a row without an integer division)
  const float* rho;                 // [M][n_I] explicit pi / [-a_hat]_+, or null for Lemma A.1's pi*
                                    // (read only by the elementwise relaxation kernels)
};

struct AdamArgs {
  int enabled;           // 0: write raw gradients instead of updating
  float b1, b2, eps;
  const float* consts;   // device: {lr_alpha decay^t, lr_mult decay^t, 1/(1-b1^(t+1)), 1/(1-b2^(t+1))}
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return hipSuccess or the launch error.

// Epilogue selection for the tile GEMM.
enum EpiKind { EPI_STORE = 0, EPI_BOUND = 1, EPI_CONC = 2, EPI_ADJ = 3, EPI_AHAT = 4 };

struct BoundEpiArgs {       // Theorem 3.1 relaxation of one ReLU node
  NodeDev nd; CutCol cc; RowParams rp;
  const float* acc_in;      // optional extra pre-activation [M][ld] (fp32)
  void* lam_out;            // [M][ld] in the GEMM operand type
  void* ahat_out;           // optional [M][ld] in the GEMM operand type (kept for the adjoint)
};
// EPI_AHAT (recomputing a_hat for the adjoint) takes BoundEpiArgs and writes
// only ahat_out.
struct ConcEpiArgs {        // concretisation over the input box
  int size, ld;
  const double* x0; double eps;
  CutCol cc; RowParams rp;  // input-variable cuts (G on x)
  int8_t* sign_out;         // optional [M][ld] sign of v
  float* contrib;           // optional [nnz_e][mp] gamma-gradient pieces
  int nnz_e;
};
struct AdjEpiArgs {         // adjoint of one ReLU node's relaxation
  NodeDev nd; CutCol cc; RowParams rp;
  const float* acc_in;      // optional extra dLambda [M][ld]
  float gemm_scale;         // multiplies the GEMM result (-eps for the input edge)
  const float* add_vec;     // [size] added to dLambda (bias, or W x0 + b)
  const void* ahat;         // [M][ld] stored pre-activation coefficients (operand type)
  void* dahat_out;          // [M][ld] operand type, null if no consumer needs it
  float* contrib; int nnz_e;           // [nnz_e][mp]
  float* d_alpha; float* d_beta;      // raw gradient outputs (adam disabled)
  float* m_alpha; float* v_alpha;     // Adam moments (adam enabled)
  float* m_beta;  float* v_beta;
  float* alpha_rw; float* beta_rw;    // parameters updated in place
  AdamArgs adam;
  float* d_rho; float* m_rho; float* v_rho; float* rho_rw;   // explicit pi (rp.rho set)
};
// Explicit pi (rp.rho set) in a bound or adjoint epilogue: the GEMM and conv
// launchers run the pi-switched epilogue instantiations.
inline bool fused_explicit_pi(EpiKind kind, const void* epi) {
  if (kind == EPI_BOUND) return ((const BoundEpiArgs*)epi)->rp.rho != nullptr;
  if (kind == EPI_ADJ) return ((const AdjEpiArgs*)epi)->rp.rho != nullptr;
  return false;
}
struct StoreEpiArgs {       // raw accumulate into an fp32 buffer
  int size, ld;
  float scale;
  const float* acc_in;
  float* out;
};

struct GemmArgs {
  int M, N, K;
  const void* A; int lda;   // [M][lda] (operand type, or int8 sign if a_is_sign)
  const void* Bt; int ldb;  // [N][ldb] operand type
  int a_is_sign;
  double* partial; int mp; int slot0;   // row partial sums [slot][mp] (may be null);
                                        // a launch owns slots slot0 .. slot0 + ceil(N/32) - 1
};

hipError_t launch_gemm(int bf16, int cfg, EpiKind kind, const GemmArgs& g, const void* epi,
                       hipStream_t st);
int gemm_num_configs();
void gemm_config_tile(int cfg, int* bm, int* bn);
// Several GEMM problems of one instantiation (cfg, kind, sign, precision) in
// one launch: device tables d_gs[np], d_epis[np] (the kind's *EpiArgs) and
// d_prefix[np + 1] of cumulative tile counts (total_tiles = d_prefix[np]).
hipError_t launch_gemm_grouped(int bf16, int cfg, EpiKind kind, int sign, const GemmArgs* d_gs, const void* d_epis,
                               const int* d_prefix, int np, int total_tiles, hipStream_t st);

// Elementwise epilogues (no GEMM): the pre-activation comes from a per-spec
// broadcast [S][ld] (fp32) plus the optional acc_in of the epilogue args.
// rows per block of the elementwise relaxation kernels (one column of them
// per thread; 8 was measured slower than 4 on the 784-256x6 MLP: 26 vs 20 us)
constexpr int kElemRows = 4;
hipError_t launch_bound_elementwise(int bf16, const float* bcast, const void* src, const BoundEpiArgs& a,
                                    double* partial, int slot0, hipStream_t st);
// Grouped elementwise relaxation: job p has M rows x ceil(size/256) blocks.
struct ElemBoundJob {
  const float* bcast; const void* src;
  BoundEpiArgs a;
  double* partial; int slot0;
};
hipError_t launch_bound_elementwise_grouped(int bf16, const ElemBoundJob* d_jobs, const int* d_prefix, int np,
                                            int total_blocks, hipStream_t st);
// Grouped gamma Adam update: job p has N x ceil(M/256) blocks.
struct GammaJob {
  int M, mp, N;
  const int32_t* row_ptr; const float* contrib; const double* d;
  float* gammaT; float* m; float* v;
};
hipError_t launch_gamma_grouped(const GammaJob* d_jobs, const int* d_prefix, int np, int total_blocks, AdamArgs adam,
                                hipStream_t st);
// Identity edge: out = (acc_in ? acc_in : 0) + scale * src (src operand type or int8 sign)
hipError_t launch_identity_acc(int bf16, int M, int size, const void* src, int ld_src, int is_sign, float scale,
                               const float* acc_in, float* out, int ld_out, hipStream_t st);
hipError_t launch_adj_elementwise(int bf16, const AdjEpiArgs& a, hipStream_t st);

// Convolution edges as implicit GEMMs on MFMA (conv_kernels.hip).
struct ConvGeom { int ci, hi, wi, co, ho, wo, kh, kw, stride, pad; };
// Bound direction (transposed conv): Lambda over the node's (co, ho, wo) ->
// epilogue over the source's (ci, hi, wi).  The source positions split into
// stride^2 phases by (y + pad) mod stride; in phase (ry, rx) only the taps
// ky = ry + stride*a, kx = rx + stride*b meet the node grid, so
// Bt = [phase][ci][ldb], entry (o, a, b) = W[o][c][ry + s a][rx + s b]
// (0 past the kernel), K = co * ceil(kh/s) * ceil(kw/s) padded to ldb.
// Adjoint direction (conv): rows over the source's (ci, hi, wi) (operand
// type, or int8 signs) -> epilogue over the node's (co, ho, wo);
// Bt = W [co][ldb], entry (c, ky, kx), K = ci*kh*kw padded to ldb.
// ldb is a multiple of 32 in both.
struct ConvArgs {
  int M;                  // batch rows
  ConvGeom cg;
  int trans;              // 1: transposed (bound direction)
  const void* X; int ldx; int x_is_sign;
  const void* Bt; int ldb;
  const float* Btf;       // transposed direction: Bt's values as fp32 (bf16-rounded in bf16 mode), for the direct kernel
  double* partial; int mp; int slot0;
};
// Work split of one conv launch: the epilogue-side rows form bands of BH
// rows; one workgroup stages the source rows a band reads (with a zero halo)
// in LDS for one batch row, produces every output of that band into a second
// LDS buffer and runs the epilogue over it.
struct ConvPlan {
  int He, We, Nch, Kch, hs, ws;   // epilogue side (He x We, Nch channels), source side (Kch x hs x ws)
  int s, p, A, Bn;                // stride, pad; taps per phase and dimension
  int n_phase, Kreal, KP;         // phases; GEMM K per phase, padded
  int BH, n_bands;
  int rows_max, xl, Wp, CHS;      // LDS slab: rows per channel, left halo, pitch, channel stride
  int OS;                         // LDS result band: channel stride
  int MT;                         // most 16-row GEMM tiles in one band (phases padded to 16 rows)
};
ConvPlan conv_plan(const ConvGeom& g, int trans);
// conv weights laid out as the kernels read them (Bt above); raw is [co][ci][kh][kw]
int conv_ldb(const ConvGeom& g, int trans);
void conv_pack_weights(const ConvGeom& g, int trans, const float* raw, float* out);
hipError_t launch_conv(int bf16, int cfg, EpiKind kind, const ConvArgs& c, const void* epi, hipStream_t st);
int conv_num_configs();
// launch_conv's cfg for the direct (VALU) transposed convolution, and whether
// it applies: concretisation over a source of at most four channels, taps
// per phase 2x2 at stride 2 or 3x3 at stride 1
constexpr int kConvDirectCfg = 6;
bool conv_direct_ok(const ConvGeom& g, EpiKind kind);
// row-partial slots a conv launch owns: one per band
inline int conv_slots(const ConvGeom& g, int trans) { return conv_plan(g, trans).n_bands; }

hipError_t launch_chat(const double* C, int S, int d_out, const float* W, int d_in,
                       int kind, float* chat, int ld, hipStream_t st);
hipError_t launch_out_const(const double* C, int S, int d_out, const float* bias,
                            double* cb, hipStream_t st);
// out[r][j] = C[r mod S][j] in the operand type, r < M, j < d
hipError_t launch_spec_rows(int bf16, const double* C, int S, int d, int M, void* out, int ld, hipStream_t st);
hipError_t launch_wx0(const ConvGeom* cg, int kind, const float* W, int d_out, int d_in,
                      const double* x0, const float* bias, float* out, hipStream_t st);
hipError_t launch_reduce_rows(int M, int mp, int S, const double* partial, int n_slots,
                              const double* cb, const float* gammaT, int N, const double* d,
                              double* bound, uint8_t* verified, hipStream_t st);
// ---------------------------------------------------------------- outward rounding
// Rounding slack of the bound pass (GCP_FLAG_OUTWARD).  Every multiplier the
// pass stores (Lambda of each node, the spec rows, beta, gamma) is one valid
// dual point; the slack bounds how far the pass's floating-point value can
// exceed the exact value of the bound at that point.  Per node the host holds
// five weight vectors [5][ld] (fp64) that depend only on the net:
//   w0 = sum over in-edges from nodes p: g(K_p) |W_e| Y_p,  w1 = sum |W_e| Y_p,
//   w2 = Z + |b|,  w3 = g(K_in) |W_e| 1 (in-edges from the input),  w4 = |W_e| 1
// (Y: the largest |x_hat| a neuron's relaxation can face, Z = max(|l|, |u|),
// g(K): the accumulation bound of a K-term fp32 sum).  A call combines them
// into one weight per neuron, w = w0 + c_sum w1 + c_zb w2 + X_in (w3 + c_in w4)
// (X_in = max |x0| + eps), and a row's slack is sum |Lambda| w over its nodes
// plus the beta, gamma and spec-row terms.
constexpr int kSlackMaxNodes = 64;
struct SlackNode {
  const double* w;     // [5][ld]
  int ld, size, off;   // off: position of this node's weights in the combined vector
  const void* lam;     // [M][ld] in the operand type; null: the output in c-hat form
};
struct SlackArgs {
  int n_nodes;
  SlackNode nodes[kSlackMaxNodes];
  int M, S, mp, bf16;
  double c_sum, c_zb, c_in;          // per-call constants of the combined weights
  const double* x0; int d_in; double eps;
  double* wcomb;                     // [total + 1]: combined weights, then X_in
  int total;
  const double* C; int d_out;        // spec rows; out_off: the output's weights in wcomb
  int out_off, out_chat;             // out_chat: output in c-hat form (C W precomputed)
  const float* beta; int K; const double* zsplit; double c_beta;    // zsplit [B][K]
  const float* gammaT; int N; const double* kap; double c_cut, c_d;  // kap [3][N]: kappa, kappa_in, |d|
  double* out;                       // partial slot [mp]: minus the slack of each row
};
hipError_t launch_slack(const SlackArgs& a, hipStream_t st);

// d bound/d gamma from the entry pieces; Adam on gammaT (moments m, v are
// [N][M]) or the raw gradient into d_gamma [M][N].
hipError_t launch_gamma_update(int M, int mp, int N, const int32_t* row_ptr, const float* contrib,
                               const double* d, float* gammaT, float* d_gamma,
                               float* m, float* v, AdamArgs adam, hipStream_t st);
// [rows][cols] (pitch ld_in) -> [cols][ld_out]
hipError_t launch_transpose(const float* in, int rows, int cols, int ld_in, float* out, int ld_out,
                            hipStream_t st);
// reset = 0: write the constants of iteration *step to consts and advance
// *step; reset > 0: set *step = reset - 1 only
hipError_t launch_adam_prepare(int* step, int reset, float lr_alpha, float lr_mult, float decay, float b1,
                               float b2, float* consts, hipStream_t st);
// the constants of iterations 0 .. iters-1 into tab[4 * t ..] (same values
// as launch_adam_prepare at step t)
hipError_t launch_adam_table(float* tab, int iters, float lr_alpha, float lr_mult, float decay, float b1, float b2,
                             hipStream_t st);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st);
// dst[dst_row[i]][j] = src[src_row[i]][j] for i < n (n <= 65535), j < L; where
// zero_col is given, column zero_col[i] of row i is written as 0 instead.
// Row indices are device arrays.
hipError_t launch_copy_rows(float* dst, int64_t ld_dst, const int32_t* dst_row, const float* src, int64_t ld_src,
                            const int32_t* src_row, int n, int L, const int32_t* zero_col, hipStream_t st);
hipError_t launch_validate(const float* p, int64_t n, float lo, float hi, int* flags,
                           hipStream_t st);
hipError_t launch_fill_bf16_from_f32(const float* src, bf16* dst, int64_t n, hipStream_t st);

// ---------------------------------------------------------------- persistent dataflow
// A recorded iteration schedule (the launches of one bound pass, adjoint and
// multiplier update of one or more instances) executed for several
// iterations in one launch (persist_kernels.hip).  Rows are independent
// problems, so a step over a panel of kPersistRows rows depends only on the
// earlier steps over the same panel (its GEMM operand spans the previous
// layer's columns of those rows).  Items are (iteration, step, column tile,
// panel); every GEMM tile is kPersistRows x 32, so each step has the same
// number of items (`ipp`) on every panel of its instance.  Panels are dealt
// to Q claim queues (panel p of an instance whose first global panel is
// `base` belongs to queue (base + p) mod Q); a workgroup serves the queue of
// the XCD it runs on, so all items of a panel meet in one L2.
constexpr int kPersistRows = 32;
constexpr int kPersistMaxSteps = 2048;   // steps of one iteration (all instances)
constexpr int kPersistAbort = 1 << 29;   // added to every claim head when a wait runs out; items per queue stay below
enum PersistKind { PK_STORE = EPI_STORE, PK_BOUND = EPI_BOUND, PK_CONC = EPI_CONC, PK_ADJ = EPI_ADJ, PK_ELEM = 5,
                   PK_GAMMA = 6 };
struct PersistStep {
  int kind, sign, job;     // PersistKind; GEMM A operand is int8 signs; index into the kind's job table
  int cnt0, panels, base;  // the instance's first completion counter (one per panel), panel count, first global panel
  int ipp;                 // items per panel (column tiles / column blocks / cut groups)
  int wait;                // items per panel in the instance's earlier steps of an iteration
  int per_iter;            // items per panel in a whole iteration of the instance
};
constexpr size_t kEpiBlob = 16 * ((sizeof(AdjEpiArgs) > sizeof(BoundEpiArgs) ? sizeof(AdjEpiArgs) : sizeof(BoundEpiArgs)) / 16 + 1);
struct PersistArgs {
  const PersistStep* steps; int n_steps;
  const int* qfirst;       // [Q][n_steps + 1]: first item of each step within an iteration, per queue
  int Q, iters, iter0;     // iteration t of the launch uses the Adam constants of iteration iter0 + t
  const GemmArgs* gemm; const unsigned char* epi;   // GEMM jobs: arguments, epilogue blobs of kEpiBlob bytes
  const ElemBoundJob* elem; const GammaJob* gam;
  AdamArgs adam;           // consts: table of every iteration's constants, [4 * t ..]
  int* sync;               // [Q] claim heads, [Q] abort flag, [Q + 1 ..] panel completion counters (zeroed per launch)
  int xcd_sync;            // 1: every queue is served by one XCD, so a producer's stores need only reach its L2
  unsigned long long spin_ticks;   // longest wait (100 MHz wall clock) before the launch aborts
  int* latch;              // set to 1 when the launch aborts (kept across the launches of one call)
};
// Workgroups one launch runs (as many as are resident at once).
int persist_grid(int bf16, int xcd_sync);
// out[b] = the XCC_ID hardware register of workgroup b < n
hipError_t launch_xcc_probe(int* out, int n, hipStream_t st);
hipError_t launch_persist(int bf16, const PersistArgs& a, int grid, hipStream_t st);
// After the certifying pass of a call that ran persistent launches: if one
// of them aborted (*latch set), every row's bound becomes -inf (a valid lower
// bound) and no row counts as verified.
hipError_t launch_persist_guard(const int* latch, double* bound, uint8_t* verified, int M, hipStream_t st);

// ---------------------------------------------------------------- fused dense chains
// A network whose ReLU nodes 0..L-1 form a chain of dense layers (node i's
// only input is node i-1, node 0's the network input; the output's only
// input is node L-1) runs its whole projected-Adam optimisation in one
// launch (chain_kernels.hip): one workgroup per kChainRows rows performs
// every iteration's bound pass, concretisation, adjoint and multiplier
// update for its rows, holding Lambda / d a_hat in LDS between layers.
constexpr int kChainRows = 16;
struct ChainNode {            // ReLU node i with its in-edge from node i-1 (the input for i = 0)
  NodeDev nd; CutCol cc;
  const void* WT; int ldWT;   // in-edge, bound direction Bt [n_{i-1}][ldWT] (operand type)
  const void* W; int ldW;     // in-edge, adjoint direction Bt [n_i][ldW]
  const float* addv;          // added to d Lambda^(i): b_i (node 0: b_0 + W_0 x0)
  void* ahat;                 // [M][ld_i] a_hat^(i), operand type (bound pass -> adjoint)
  void* dahat;                // [M][ld_i] (the per-layer path's buffer; unused by the fused kernel)
};
struct ChainArgs {
  int L;                      // ReLU nodes
  const ChainNode* nodes;     // device [L]
  int in_size, in_ld;
  const double* x0; double eps;
  CutCol cc_in;               // input-variable cuts
  int8_t* sign;               // [M][in_ld] (the per-layer path's buffer; unused by the fused kernel)
  const float* chat; int chat_ld;     // [S][chat_ld]: C W_out per spec row (fp32)
  RowParams rp;
  float* gammaT;              // writable view of rp.gammaT
  float* contrib; int nnz_e;  // [nnz_e][mp] gamma-gradient pieces
  const int32_t* row_ptr; const double* cut_d;
  float *m_alpha, *v_alpha, *m_beta, *v_beta, *m_gamma, *v_gamma;
  float *alpha_rw, *beta_rw;
  AdamArgs adam;              // consts: table of every iteration, [iters][4]
  int iters;
  int P;                      // LDS pitch (elements) of the two activation buffers
  int off_buf0, off_buf1, off_sign, sign_ld;   // byte offsets into the dynamic LDS; sign pitch (bytes)
};
// lds_bytes: 2 kChainRows P esz + kChainRows sign_ld
hipError_t launch_chain_opt(int bf16, const ChainArgs& a, int n_tiles, size_t lds_bytes, hipStream_t st);

}  // namespace gcp
struct gcp_net;
struct gcp_splits;
namespace gcp {
// A split handle of `net` holding B domains of K slots (host arrays as
// gcp_splits_create takes them): *s is refilled in place, asynchronously on
// st, when its buffers are large enough (the host arrays are staged in the
// handle, which must not be refilled again before the copies are done),
// else replaced by a new handle.  Returns a GCP_* code.
int splits_assign(const gcp_net* net, gcp_splits** s, int32_t B, int32_t K, const int32_t* node,
                  const int32_t* neuron, const int8_t* sign, hipStream_t st);

// Static workspace (scratch.hip): the device address and size of the calling
// thread's current device's copy, looked up on its first use on that device.
constexpr size_t kScratchBytes = size_t(64) << 20;
hipError_t scratch_region(void** ptr, size_t* bytes);

}  // namespace gcp
