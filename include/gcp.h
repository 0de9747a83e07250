/*
 * gcp.h -- C ABI of the MI355X (gfx950) GCP-CROWN bound-propagation library.
 *
 * GCP-CROWN (arXiv 2208.05740) lower-bounds  min_{x in C} c^T f(x)  for a
 * ReLU network f over the L-inf box C = {x : |x - x0|_inf <= eps}
 * (Sec. 2, eq. verification_definition), given root pre-activation bounds
 * l <= x^(i) <= u (Sec. 2, neuron classes), BaB split constraints
 * (Sec. 3.1, "Connection to CROWN-like methods"; Appendix B) and general
 * cutting planes  sum_i H^(i) x^(i) + G^(i) x_hat^(i) + Q^(i) z^(i) <= d
 * (Sec. 3.1, eq. cuts).  The bound is the closed-form dual objective of
 * Theorem 3.1 (proof in Appendix A, Lemma A.1), with optimisable
 *   alpha  in [0,1]  -- lower-relaxation slope of each root-unstable neuron,
 *   beta   >= 0      -- multiplier of each split constraint,
 *   gamma  >= 0      -- multiplier of each cut row
 * (the paper names both multipliers beta).  Every (domain, spec row) pair is
 * an independent scalar problem; the library evaluates M = B*S of them in
 * one call, their gradients by a hand-written adjoint, and a projected Adam
 * ascent (Appendix C.1: 20 iterations, lr 0.1 for alpha, 0.02 for the
 * multipliers, decay 0.9 per iteration).
 *
 * Conventions for every entry point
 *  - Return 0 (GCP_OK) or a negative GCP_E* code; gcp_last_error() returns a
 *    thread-local message for the last failure.  No C++ exception crosses
 *    the ABI.  Inputs are not modified on error.
 *  - "host" pointers are read during the call only; "device" pointers are
 *    caller-owned HIP device memory on the device current at the call and
 *    must stay valid until the stream work completes.  Handles own their
 *    device copies and are released by the matching *_destroy.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t, NULL = the
 *    default stream); results are ready when the stream is synchronised.
 *    `stream` may be a non-blocking stream: device memory the library
 *    allocates (handles, workspace growth on a first call) is cleared and
 *    filled on the null stream and waited for before the call goes on, and
 *    a buffer is freed only after the device is idle.
 *  - Calls that share a gcp_net use its workspace: do not run two calls on
 *    the same net concurrently on different streams.
 *  - Row r of every per-row array is domain b = r / S, spec row s = r % S.
 */
#ifndef GCP_H
#define GCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define GCP_OK            0
#define GCP_EINVAL      (-1)   /* null pointer, bad shape or index           */
#define GCP_ERANGE      (-2)   /* alpha outside [0,1], multiplier < 0, eps<0 */
#define GCP_ENONFINITE  (-3)   /* NaN or Inf in an input                     */
#define GCP_ENOMEM      (-4)   /* device allocation failed                   */
#define GCP_EDEVICE     (-5)   /* HIP runtime error                          */
#define GCP_EUNSUPPORTED (-6)  /* valid input the library does not handle    */

/* ------------------------------------------------------------ network */
#define GCP_EDGE_DENSE    0    /* W host fp32 [out][in], row-major           */
#define GCP_EDGE_CONV     1    /* W host fp32 [c_out][c_in][kh][kw]          */
#define GCP_EDGE_IDENTITY 2    /* W unused; source and node shapes equal     */

/* One linear input of a node:  x_node += op(x_hat_src)  (Sec. 2, eq.
 * mip_layer; residual sums for DAG networks).  src = -1 is the input x. */
typedef struct {
  int32_t src;
  int32_t kind;
  const float* W;
  int32_t kh, kw, stride, pad;   /* conv only: square stride, symmetric pad */
} gcp_edge_desc;

/* A node  x = sum_e op_e(x_hat_src(e)) + bias,  shape (c, h, w) flattened in
 * C order (dense nodes: c = size, h = w = 1).  Every node but the last is
 * followed by a ReLU; the last node is the network output f(x).  lower/upper
 * are the root pre-activation bounds l, u of a ReLU node (host fp64, l <= u;
 * ignored for the output).  Neuron classes follow l, u: active if l >= 0,
 * else inactive if u <= 0, else unstable (l < 0 < u). */
typedef struct {
  int32_t c, h, w;
  const float* bias;
  const double* lower;
  const double* upper;
  int32_t n_edges;
  const gcp_edge_desc* edges;
} gcp_node_desc;

typedef struct {
  int32_t in_c, in_h, in_w;
  int32_t n_nodes;               /* >= 1: ReLU nodes, then the output        */
  const gcp_node_desc* nodes;    /* topological order: edges point backward */
} gcp_net_desc;

typedef struct gcp_net gcp_net;

/* Copies weights, biases and root bounds to the current device (fp32 and
 * bf16 copies of every weight).  Errors: EINVAL (shapes, edge sources not
 * earlier, conv geometry, an unused input), EUNSUPPORTED (a ReLU node without
 * consumers; the input feeding more than one edge, or an identity edge),
 * ENONFINITE (weights/bounds), ENOMEM, EDEVICE. */
int gcp_net_create(const gcp_net_desc* desc, gcp_net** out);
int gcp_net_destroy(gcp_net* net);

typedef struct {
  int32_t n_nodes;
  int32_t in_size;               /* d_0                                     */
  int32_t out_size;              /* d_L                                     */
  int64_t n_relu;                /* sum of ReLU node sizes                  */
  int64_t n_unstable;            /* n_I: length of an alpha row             */
} gcp_net_info;

/* Sizes of the network.  alpha rows list the root-unstable neurons node by
 * node (topological order), ascending neuron index within a node. */
int gcp_net_get_info(const gcp_net* net, gcp_net_info* info);

/* The root-unstable neurons in alpha row order: node[r], neuron[r] and the
 * root bounds lower[r], upper[r] as given to gcp_net_create, r < n_unstable
 * (host arrays; any may be NULL). */
int gcp_net_get_unstable(const gcp_net* net, int32_t* node, int32_t* neuron, double* lower, double* upper);

/* ------------------------------------------------------------ cuts */
#define GCP_CUT_H 0   /* coefficient on the pre-activation x_j   */
#define GCP_CUT_G 1   /* coefficient on the post-activation x_hat_j (node -1: input x_j) */
#define GCP_CUT_Q 2   /* coefficient on the ReLU indicator z_j    */

typedef struct gcp_cuts gcp_cuts;

/* N cut rows in coordinate form (host arrays of length nnz): entry e adds
 * coef[e] * var(kind[e]) of neuron `neuron[e]` of node `node[e]` to the
 * left side of cut `cut[e]`; d (host fp64 [N]) are the right sides
 * (eq. cuts).  node = -1 (input) allows only GCP_CUT_G.  Repeated
 * (cut, node, neuron, kind) entries are summed.  A Q term on a neuron that
 * is active in a domain uses z = 1 there, on an inactive one z = 0.
 * Coefficients are stored in fp32, d in fp64; where rounding a merged
 * coefficient c to fp32 changes it, d is widened by |fp32(c) - c| times the
 * largest magnitude the variable takes under the root bounds (|x| <=
 * max(|l|, |u|), 0 <= x_hat <= max(u, 0), 0 <= z <= 1), so the stored cut
 * still holds wherever the given one does.  Input-variable (node -1)
 * coefficients must be fp32 values (EINVAL otherwise).  n_cuts = 0 is allowed
 * (gamma rows then have length 0 and the bound is beta-CROWN's).
 * Errors: EINVAL (index out of range, bad kind), ENONFINITE. */
int gcp_cuts_create(const gcp_net* net, int32_t n_cuts, int64_t nnz,
                    const int32_t* cut, const int32_t* node, const int32_t* neuron,
                    const int8_t* kind, const double* coef, const double* d,
                    gcp_cuts** out);
int gcp_cuts_destroy(gcp_cuts* cuts);
/* Number of cut rows N (the length of a gamma row). */
int gcp_cuts_info(const gcp_cuts* cuts, int32_t* n_cuts);

/* ------------------------------------------------------------ splits */
typedef struct gcp_splits gcp_splits;

/* B BaB domains with up to K split slots each (host [B][K] arrays):
 * node[b][k] = -1 marks an unused slot; otherwise neuron `neuron[b][k]` of
 * ReLU node `node[b][k]` is split with sign[b][k] = +1 (x >= 0: the neuron
 * is treated as active and its multiplier enters as -beta) or -1 (x <= 0:
 * inactive, +beta).  Split neurons must be root-unstable and distinct
 * within a domain.  K = 0 (no splits) is allowed with B >= 1.
 * Errors: EINVAL (index, sign, stable or repeated neuron). */
int gcp_splits_create(const gcp_net* net, int32_t B, int32_t K,
                      const int32_t* node, const int32_t* neuron, const int8_t* sign,
                      gcp_splits** out);
int gcp_splits_destroy(gcp_splits* splits);

/* ------------------------------------------------------------ bounding */
#define GCP_MODE_FP32   0   /* GEMMs fp32 x fp32 -> fp32 on MFMA             */
#define GCP_MODE_BF16   1   /* GEMM operands bf16, fp32 accumulation          */
#define GCP_FLAG_VALIDATE 0x100  /* check alpha/beta/gamma ranges on device
                                    (synchronises the stream)               */
/* Pre-activation coefficients a_hat of every ReLU layer (Theorem 3.1) are
 * needed again by the adjoint.  By default they are stored by the bound pass
 * unless the stored copies of all layers would exceed half of the device
 * memory that is free (or already held by a_hat buffers) when the call is
 * planned, or GCP_AHAT_BUDGET_MB (environment, MiB) where that is set; then
 * a layer whose a_hat comes from a
 * single dense or conv consumer recomputes it in the adjoint from that
 * consumer's Lambda (one more GEMM, one layer's a_hat live at a time).
 * Results are identical either way.  The flags force one policy. */
#define GCP_FLAG_RECOMPUTE   0x200  /* recompute a_hat wherever possible      */
#define GCP_FLAG_STORE_AHAT  0x400  /* store a_hat of every layer             */
/* Outward rounding (the bound is sound in exact arithmetic, Theorem 3.1; its
 * floating-point value can exceed the exact one by rounding).  With
 * GCP_FLAG_OUTWARD the bound pass subtracts from every row a bound on that
 * excess, so the returned value is at most the exact Theorem 3.1 value of
 * the multipliers the pass used (each node's stored Lambda, beta, gamma and
 * the spec row: a valid dual point) and hence a lower bound on c.f(x) over
 * the box.  The slack is sum over nodes of |Lambda| w with per-neuron
 * weights w from |W| times the root-bound magnitudes and the accumulation
 * bound K u / (1 - K u) of each fp32 sum (u = 2^-23, twice the unit
 * roundoff, so that any rounding of the matrix cores' internal steps is
 * covered), plus the operand rounding of bf16 mode (2^-8 of |Lambda||W|),
 * the relaxation's fp32 operations, the |beta| and |gamma| terms and the
 * fp64 row sums.  It does not cover root bounds that are themselves wrong.
 * A net whose output Lambda is materialised (out_general) needs spec rows
 * exactly representable in the operand type, else the row's bound is -inf.
 * Applies to gcp_bound, gcp_bound_noalloc, gcp_bound_pi, the certifying
 * pass of gcp_optimize, gcp_optimize_pi and gcp_optimize_batch, and the
 * bounds of gcp_crown_bounds / gcp_crown_bounds_domain; gradients are those
 * of the bound without the slack.  Costs one extra read of every Lambda. */
#define GCP_FLAG_OUTWARD     0x800
/* Persistent dataflow iterations (gcp_optimize, gcp_optimize_batch): every
 * (domain, spec row) of Theorem 3.1 is an independent problem, so a layer's
 * step over a panel of rows needs only the earlier steps over the same rows.
 * With GCP_FLAG_PERSIST the Adam iterations run as one launch whose
 * workgroups claim (iteration, step, column tile, row panel) items in
 * schedule order and wait per panel for the steps before, instead of one
 * launch per layer (and, in gcp_optimize_batch, every instance shares that
 * one launch).  Results are bit-identical to the per-layer launches.  Used
 * for networks whose edges are all dense, whose output takes the c-hat form
 * and whose a_hat is stored (Lemma A.1's pi*); otherwise the flag is
 * ignored.  The first call of an argument set runs one iteration per layer
 * (tile tuning, buffer sizing) and records the schedule; later calls with
 * the same arguments run every iteration in the one launch. */
#define GCP_FLAG_PERSIST     0x1000
/* In every mode the row reductions (concretisation v.x0 - eps*|v|_1, bias,
 * h and cut-offset sums, gamma.d) accumulate in fp64; the bound is fp64. */

/* gcp_bound: the Theorem 3.1 bound for all M = B*S rows.
 *   x0     device fp64 [d_0]       centre of the box; eps >= 0
 *   C      device fp64 [S][d_L]    spec rows c_s (folded in as last layer)
 *   alpha  device fp32 [M][n_I]    in [0,1]
 *   beta   device fp32 [M][K]      >= 0 (K of `splits`)
 *   gamma  device fp32 [M][N]      >= 0 (N of `cuts`; NULL if N = 0)
 *   bound  device fp64 [M]         output
 *   verified device uint8 [M]      optional output: 1 where bound >= 0,
 *          i.e. the property is proven for that row (Sec. 2)
 *   d_alpha/d_beta/d_gamma device fp32, shapes as the inputs: optional
 *          outputs d bound_r / d param (row r's own parameters); pass all
 *          three or none.
 * The input term is v.x0 - eps*||v||_1 with v = Lambda^(1) W^(1). */
int gcp_bound(const gcp_net* net, const double* x0, double eps,
              const double* C, int32_t S,
              const gcp_splits* splits, const gcp_cuts* cuts,
              const float* alpha, const float* beta, const float* gamma,
              int32_t mode, double* bound, uint8_t* verified,
              float* d_alpha, float* d_beta, float* d_gamma, void* stream);

/* gcp_bound_noalloc: gcp_bound for callers that cannot allocate device
 * memory -- code being captured into a HIP graph, tight serving loops,
 * harnesses that forbid allocation.  Same arguments, results and errors as
 * gcp_bound, but the call allocates nothing: its workspace (Lambda, a_hat
 * and d a_hat of every layer, row partial sums, the transposed gamma, cut
 * gradient pieces) lies in a static device array of 64 MiB per device that
 * the library holds until the process ends, tile shapes come from the tile
 * cache (GCP_TILE_CACHE) or a fixed rule (no timing trials), and no profiler
 * events are recorded.  Limit: a call whose workspace exceeds 64 MiB fails
 * with GCP_ENOMEM (for the 784-256x6-10 MLP with 200 cuts, about 2500 rows
 * with gradients, 6500 without); GCP_FLAG_VALIDATE (which waits for the
 * device) is rejected with GCP_EINVAL.  Every call on one device shares that
 * device's array, so calls that overlap on one device -- on different streams
 * or from several threads -- race and must be serialised by the caller; the
 * array holds the last call's intermediate values, which no later call reads
 * before writing. */
int gcp_bound_noalloc(const gcp_net* net, const double* x0, double eps,
                      const double* C, int32_t S,
                      const gcp_splits* splits, const gcp_cuts* cuts,
                      const float* alpha, const float* beta, const float* gamma,
                      int32_t mode, double* bound, uint8_t* verified,
                      float* d_alpha, float* d_beta, float* d_gamma, void* stream);

/* Optimiser settings (Appendix C.1 defaults: iters 20, lr_alpha 0.1,
 * lr_mult 0.02, decay 0.9, Adam 0.9/0.999/1e-8). */
typedef struct {
  int32_t iters;
  float lr_alpha, lr_mult, decay;
  float adam_b1, adam_b2, adam_eps;
  int32_t use_graph;        /* capture one iteration in a hipGraph, replay */
} gcp_opt;

/* gcp_optimize: `iters` projected Adam ascent steps on sum_r bound_r, all on
 * the device: each iteration runs the bound pass (GEMMs in `mode`), the
 * adjoint, and the Adam update of alpha (clamped to [0,1]), beta and gamma
 * (clamped >= 0) with lr_t = lr * decay^t.  alpha, beta, gamma are updated
 * in place.  adam_state: device fp32, 2*M*(n_I + K + N) floats holding the
 * first and second moments, in this order: m_alpha [M][n_I], v_alpha
 * [M][n_I], m_beta [M][K], v_beta [M][K], m_gamma [N][M], v_gamma [N][M]
 * (caller-owned so optimisation can resume; zero for a fresh start).
 * Finally the bound at the final parameters is recomputed
 * with fp32 GEMMs and fp64 reductions (the certifying pass) into
 * bound/verified.  With the environment variable GCP_FUSED=1, a network whose
 * ReLU layers form a chain of dense layers runs all iterations in one launch
 * instead of one launch per layer (the same results bit for bit; slower on
 * MI355X at the sizes measured, kept for study). */
int gcp_optimize(const gcp_net* net, const double* x0, double eps,
                 const double* C, int32_t S,
                 const gcp_splits* splits, const gcp_cuts* cuts,
                 float* alpha, float* beta, float* gamma, float* adam_state,
                 const gcp_opt* opt, int32_t mode,
                 double* bound, uint8_t* verified, void* stream);

/* gcp_prepare: allocate and tune once, ahead of the bounding calls (the
 * problem statement's bound calls, Sec. 2, issued many times on one net).
 * Sizes the net's workspace for M = B*S rows (B of `splits`, the cut count
 * and entries of `cuts`, may be NULL) and runs the autotuner for every GEMM
 * and convolution shape that gcp_bound (with and without gradients, in `mode`
 * and in fp32) and gcp_optimize (in `mode`, with its fp32 certifying pass, up
 * to `iters` iterations) launch for these shapes; `mode` may carry
 * GCP_FLAG_RECOMPUTE / GCP_FLAG_STORE_AHAT.  Allocates device memory and
 * synchronises `stream`.  Afterwards, gcp_bound and gcp_optimize on this net
 * with the same S, number of domains, cuts and mode (and iters <= the
 * prepared count, use_graph = 0) allocate no device memory and never wait for
 * the device, so they can be issued inside a HIP stream capture.  Other
 * shapes tune (and may allocate) on first use as usual.  Errors: EINVAL,
 * ENOMEM, EDEVICE. */
int gcp_prepare(const gcp_net* net, int32_t S, const gcp_splits* splits, const gcp_cuts* cuts,
                int32_t iters, int32_t mode, void* stream);

/* ------------------------------------------------------------ explicit pi */
/* Variant of the unstable-neuron rule in which pi is a free variable
 * instead of Lemma A.1's maximiser.  In the proof of Theorem 3.1
 * (Appendix A) each unstable neuron's dual splits [-a_hat]_+ into pi and
 * the upper multiplier [-a_hat]_+ - pi; every split with both parts >= 0 is
 * a feasible dual point, and the closing remark of the proof notes that
 * optimising them (rather than taking the per-neuron optimum) can tighten
 * the bound.  Here pi = rho * [-a_hat]_+ with one rho in [0, 1] per
 * (row, root-unstable neuron), so that
 *   Lambda_j = alpha_j [a_hat]_+ - pi + t_j,
 *   h_j      = l pi - [u ([-a_hat]_+ - pi) + l pi - s_j]_+ .
 * rho = u / (u - l) gives Lemma A.1's pi* wherever s_j = 0.
 *
 * gcp_bound_pi: gcp_bound with rho (device fp32 [M][n_I], layout of
 * alpha, in [0,1]) and its gradient d_rho (optional like the others; pass
 * all four gradient outputs or none).  gcp_optimize_pi: gcp_optimize with
 * rho updated in place by projected Adam with alpha's learning rate and
 * clamp; adam_state holds 2*M*(n_I + K + N) + 2*M*n_I floats: the
 * gcp_optimize layout followed by m_rho [M][n_I], v_rho [M][n_I].  Dense
 * and conv edges run the relaxation fused in their epilogues; a node whose
 * last edge is an identity relaxes in an elementwise pass after its GEMMs,
 * and gcp_optimize_batch does not take this variant.  Errors: as gcp_bound / gcp_optimize;
 * EINVAL for a null rho when n_I > 0; ERANGE (with GCP_FLAG_VALIDATE) for
 * rho outside [0,1]. */
int gcp_bound_pi(const gcp_net* net, const double* x0, double eps,
                 const double* C, int32_t S,
                 const gcp_splits* splits, const gcp_cuts* cuts,
                 const float* alpha, const float* beta, const float* gamma, const float* rho,
                 int32_t mode, double* bound, uint8_t* verified,
                 float* d_alpha, float* d_beta, float* d_gamma, float* d_rho, void* stream);
int gcp_optimize_pi(const gcp_net* net, const double* x0, double eps,
                    const double* C, int32_t S,
                    const gcp_splits* splits, const gcp_cuts* cuts,
                    float* alpha, float* beta, float* gamma, float* rho, float* adam_state,
                    const gcp_opt* opt, int32_t mode,
                    double* bound, uint8_t* verified, void* stream);

/* ------------------------------------------------------------ intermediate bounds */
/* gcp_crown_bounds: pre-activation bounds l, u of every ReLU node of the
 * network `desc` (its lower/upper fields are ignored) over the L-inf box
 * ||x - x0|| <= eps, computed on the device layer by layer with CROWN
 * (Theorem 3.1 with beta = gamma = 0 and no splits): for node k the prefix
 * network ending at node k's pre-activation is bounded with spec rows +e_j
 * and -e_j by gcp_bound, the ReLU nodes before k using the bounds already
 * found and CROWN-adaptive lower slopes (alpha = 1 where u >= -l, else 0).
 * The first node's bounds are the exact concretisation of its affine map.
 * x0: device fp64 [d_0].  lower[k], upper[k]: host fp64 arrays of node k's
 * size for every ReLU node k (k < n_nodes - 1), written on success; their
 * values can be passed as the root bounds of gcp_net_create.  mode: the
 * GEMM precision (GCP_MODE_FP32 recommended: the bounds are then computed
 * like a certifying pass).  Synchronises `stream`.  Errors: as gcp_net_create
 * and gcp_bound. */
int gcp_crown_bounds(const gcp_net_desc* desc, const double* x0, double eps, double* const* lower,
                     double* const* upper, int32_t mode, void* stream);

/* gcp_crown_bounds_domain: the same bounds over one BaB domain, the box
 * restricted by n_split (<= 127) split constraints: neuron split_neuron[s]
 * of ReLU node split_node[s] with split_sign[s] = +1 (x >= 0) or -1
 * (x <= 0) (host arrays; each neuron at most once).  Layer by layer as in
 * gcp_crown_bounds, with two changes (Sec. 3.1 on splits, without split
 * multipliers): a split neuron of an earlier node that is unstable under
 * the bounds found so far takes its linear piece (x_hat = x for x >= 0,
 * x_hat = 0 for x <= 0) instead of its relaxation, and a split neuron's own
 * bounds are clamped at 0 (l = max(l, 0), resp. u = min(u, 0)).  A split
 * that contradicts its neuron's bounds (the domain is empty, up to
 * rounding) leaves that neuron at exactly [0, 0], so l <= u always holds
 * and the result can be passed to gcp_net_create as the domain's root
 * bounds.  n_split = 0 is gcp_crown_bounds.  Errors: as gcp_crown_bounds;
 * EINVAL for a bad split. */
int gcp_crown_bounds_domain(const gcp_net_desc* desc, const double* x0, double eps, int32_t n_split,
                            const int32_t* split_node, const int32_t* split_neuron, const int8_t* split_sign,
                            double* const* lower, double* const* upper, int32_t mode, void* stream);

/* ------------------------------------------------------------ branch and bound */
/* gcp_bab: branch and bound on one property c^T f(x) >= 0 over the box
 * (Appendix B's procedure, easiest domains first as in Sec. 3.3), with
 * gcp_optimize as the bounding step.  A domain is a set of splits
 * x_j >= 0 / x_j <= 0 of root-unstable neurons.  Each round bounds up to
 * `batch` open domains in one gcp_optimize call (the open domains with the
 * largest parent bound first when more are open), prunes those with a bound
 * >= 0, and splits each other one on its unsplit neuron of largest root
 * triangle height u(-l)/(u-l) into two children.  A domain that reaches
 * max_depth splits (or has no unstable neuron left) with a negative bound is
 * counted as unresolved after `retries` further rounds from its own
 * optimum.  The root starts from alpha = CROWN-adaptive (1 where u >= -l),
 * beta = gamma = 0; a child starts from its parent's optimised alpha, beta
 * (its new split's multiplier at 0) and gamma, with fresh Adam moments; cuts
 * apply to every domain.  c: device fp64 [d_out] (one spec row); x0 as gcp_bound.
 * The open domains' alpha, beta and gamma stay on the device (a pool of
 * rows); a round sends the device its split lists and row indices and reads
 * back the batch's bounds, synchronising `stream` twice. */
typedef struct {
  int32_t batch;           /* domains per bounding call, >= 1                */
  int32_t max_depth;       /* splits per domain at most (K slots)            */
  int64_t max_domains;     /* budget of bounded domains                      */
  int64_t max_pool;        /* open domains at most; more ends the search     */
  int32_t retries;         /* extra bounding rounds for a domain that cannot
                              be split further, each from its own optimum    */
  gcp_opt opt;             /* the bounding step's optimiser                  */
  int32_t mode;            /* GCP_MODE_* of the bounding step                */
} gcp_bab_opt;

#define GCP_BAB_VERIFIED 1  /* every leaf has a bound >= 0                  */
#define GCP_BAB_UNKNOWN  0  /* budget, pool or depth exhausted               */

typedef struct {
  int32_t status;          /* GCP_BAB_VERIFIED or GCP_BAB_UNKNOWN            */
  double lower;            /* verified: smallest leaf bound; otherwise the
                              smallest bound of an open or unresolved domain */
  int64_t bounded;         /* domains bounded                                */
  int64_t rounds;          /* bounding calls                                 */
  int64_t max_open;        /* largest number of open domains                 */
  int64_t open;            /* open domains left                              */
  int64_t unresolved;      /* domains at max_depth with a negative bound     */
} gcp_bab_result;

int gcp_bab(const gcp_net* net, const double* x0, double eps, const double* c, const gcp_cuts* cuts,
            const gcp_bab_opt* opt, gcp_bab_result* result, void* stream);

/* ------------------------------------------------------------ batching */
/* One verification instance of a batched optimisation: the arguments of
 * gcp_optimize for that instance. */
typedef struct {
  const gcp_net* net;
  const double* x0; double eps;
  const double* C; int32_t S;
  const gcp_splits* splits; const gcp_cuts* cuts;
  float* alpha; float* beta; float* gamma; float* adam_state;
  double* bound; uint8_t* verified;
} gcp_batch_item;

/* gcp_optimize_batch: gcp_optimize of every item with the same settings and mode.
 * Instances large enough to fill the device with their own launches (batch
 * rows x widest layer >= 2^20 elements; the environment variable
 * GCP_BATCH_ALONE_WORK overrides the threshold) run exactly as gcp_optimize,
 * concurrently on internal streams (GCP_BATCH_STREAMS, default 2) that are
 * joined to `stream` by events, longest instances first.
 * The others run each Adam iteration as a few grouped launches -- launches
 * of the same kernel at the same position of each instance's schedule become
 * one launch whose workgroups look up their instance in a device table --
 * instead of one launch per layer per instance.  The first call with an
 * argument set runs iteration 0 per instance (tuning tiles, recording the
 * schedule) and builds the tables; calls with the same argument set reuse
 * them.  With opt->use_graph the grouped iteration is captured once and
 * replayed.  Results equal per-instance gcp_optimize calls with the same
 * tiles.  Every item needs its own net handle; grouped instances must be
 * dense networks with the output in the c-hat form: a batch whose grouped
 * part holds conv or identity edges (or a materialised output Lambda) is
 * rejected with EUNSUPPORTED, and a batch with an item whose arguments
 * gcp_optimize would reject (null or foreign handles, null pointers, S, eps)
 * with that error, before anything is launched; only the value checks of
 * GCP_FLAG_VALIDATE on a large instance run with its own launches.  Calls
 * from several threads are serialised. */
int gcp_optimize_batch(int32_t n, const gcp_batch_item* items, const gcp_opt* opt, int32_t mode, void* stream);

/* ------------------------------------------------------------ profiling */
/* Kernel timing for roofline reports.  While enabled, every kernel the
 * library launches is bracketed by HIP events on the stream it runs on and
 * attributed to a class (one class per kernel instantiation: epilogue kind,
 * operand type, sign input, tile shape); each launch also records its FLOPs
 * and its HBM bytes under two models: `bytes` = every operand read once and
 * every result written once; `alg_bytes` = the optimiser-state traffic the
 * method needs (Appendix C.1's Adam on alpha, beta, gamma: 4 bytes of alpha
 * read per (row, unstable neuron) in the bound pass, 24 bytes of alpha and
 * its two moments read and written in the adjoint, 28 bytes per (row,
 * multiplier) counted with the multiplier update, 1 byte of split mask per
 * (domain, unstable neuron) and launch), 0 for launches without such state.
 * gcp_profile_enable(1) resets the records, (0) stops recording.
 * gcp_profile_read synchronises the recorded events and returns class idx
 * (0-based, GCP_EINVAL past the last class): its name (NUL-terminated,
 * truncated to name_len), launches, total milliseconds, both byte figures
 * and FLOPs (summed over the launches; any output may be NULL).
 * Autotuner trial launches are never recorded. */
int gcp_profile_enable(int32_t on);
int gcp_profile_read(int32_t idx, char* name, int32_t name_len, int64_t* launches,
                     double* total_ms, double* bytes, double* alg_bytes, double* flops);

/* Last error message of this thread ("" if none). */
const char* gcp_last_error(void);

/* Library version string. */
const char* gcp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GCP_H */
