/*
 * mf.h -- C ABI of the MI355X parallel mean-field library (libmf.so).
 *
 * The library runs the proximal-gradient parallel mean-field update of
 * Baque, Bagautdinov, Fleuret and Fua, "Principled Parallel Mean-Field
 * Inference for Discrete Random Fields":
 *
 *   m_i     = u_i + Theta S_i,      S_i = sum_{j in N(i)} w_ij q_j
 *   log q_i <- (1 - alpha) log q_i - alpha m_i, renormalised per node
 *
 * that is, the damped natural-parameter step of Eq. 15 (Sec. 3.1) with the
 * fixed step size alpha = eta = 1 / (1 + d) of Eq. 16 (Sec. 3.2), applied to
 * every node at once.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Energies.  Unaries u and compatibilities Theta are energies:
 *   P(x) is proportional to exp(-sum_i u_i(x_i) - sum_{(i,j)} w_ij Theta(x_i, x_j)),
 *   the pairwise model of Eq. 2 (Sec. 2.1) written with the sign of the
 *   natural parameters of Eq. 6.  Theta must be symmetric for the free
 *   energy and the convergence guarantee to hold.
 * - Layout.  Every per-node array is label-major and batch-outermost:
 *   element (b, l, n) of a [B][L][N] array is at ((b * L) + l) * N + n, with
 *   n = y * width + x on grids.  Theta is [L][L] row-major, Theta[l][k]
 *   being the energy of (x_i = l, x_j = k).
 * - Memory.  All array arguments are device pointers owned by the caller
 *   (HIP device memory, e.g. PyTorch tensors); they must stay valid until
 *   the work enqueued on them has completed and, for the pointers stored
 *   in an mf_desc, until mf_destroy.  The library never allocates device
 *   memory: scratch space is the caller's workspace buffer, sized by
 *   mf_workspace_size.  The library owns only the host-side handle.
 * - Streams.  Work is enqueued asynchronously on the caller's hipStream_t
 *   (desc.stream, NULL = the default stream).  Only mf_free_energy,
 *   mf_check and mf_lipschitz (whose results are host values) synchronise
 *   that stream.
 * - Errors.  Every entry point returns an mf_status; nothing throws or
 *   aborts across the ABI.  Arguments are validated on the host before any
 *   launch.  mf_last_error gives a message for the last failure.
 */
#ifndef MF_H_
#define MF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MF_ABI_VERSION 4
/* Largest label count: grids with the fixed-step rule take up to 128 labels
   (above 32 one step per launch, Theta S on the matrix cores); CSR and dense
   graphs, the other step rules, mf_step_many's shared launches, the adjoint
   and the power method take up to 32 (MF_EUNSUPPORTED above). */
#define MF_MAX_LABELS 128

/* Steps per launch of the persistent grid kernel (see mf_desc.steps_per_launch),
 * as mf_steps_per_launch reports it for a handle that runs that kernel. */
#define MF_PERSIST_STEPS_PER_LAUNCH 4096
/* n_labels * n_nodes of one problem must stay below this (2^30): the kernels
   address one problem's [L][N] planes with 32-bit byte offsets.  Larger
   problems are rejected with MF_EUNSUPPORTED.  General graphs (MF_CSR) also
   need n_nodes * LQ * 4 < 2^32, LQ = n_labels rounded up to 4 (L <= 12) or
   to 8: the node-major q rows they gather are addressed the same way. */
#define MF_MAX_LABEL_NODES ((size_t)1 << 30)

typedef enum {
  MF_OK = 0,
  MF_EINVAL = -1,         /* invalid argument; nothing was enqueued */
  MF_ENONFINITE = -2,     /* a non-finite unary or state was detected on the device */
  MF_EDEVICE = -3,        /* a HIP call or kernel launch failed */
  MF_EUNSUPPORTED = -4,   /* valid but not implemented (e.g. L > MF_MAX_LABELS) */
  MF_ENOWORKSPACE = -5    /* workspace missing or smaller than mf_workspace_size */
} mf_status;

/* Graph of the random field.  Grids have a free (non-periodic) boundary and
 * unit weights; 8-connectivity adds both diagonals.  CSR lists, for each
 * node i, the neighbours j and weights w_ij entering S_i.  DENSE is the fully
 * connected field with an explicit N x N kernel (Sec. 4.2, semantic
 * segmentation with a dense CRF). */
typedef enum { MF_GRID4 = 0, MF_GRID8 = 1, MF_CSR = 2, MF_DENSE = 3 } mf_graph;

/* GENERAL: the full L x L Theta.  POTTS: Theta = potts_w (1 1^T - I). */
typedef enum { MF_COMPAT_GENERAL = 0, MF_COMPAT_POTTS = 1 } mf_compat;

/* Precision of the neighbour messages.  The state log q, the step and the
 * log-sum-exp are FP32 in every mode; the *_MSG modes round q to BF16 or
 * FP16 where it is staged as the operand of the neighbour aggregation
 * (the dense product runs on MFMA in these modes) and accumulate in FP32. */
typedef enum { MF_P_F32 = 0, MF_P_BF16MSG = 1, MF_P_F16MSG = 2 } mf_precision;

/* Initial state.  The paper leaves q^0 open.  UNARY: q^0 = softmax(-u).
 * UNIFORM: q^0 = 1/L.  STATE: state buffer 0 already holds log q^0 written
 * by the caller (resume from a checkpoint). */
typedef enum { MF_INIT_UNARY = 0, MF_INIT_UNIFORM = 1, MF_INIT_STATE = 2 } mf_init_mode;

/* Step rule of mf_step / mf_solve.
 * FIXED    the parallel proximal step (Eq. 13-15, Sec. 3.1) with the fixed
 *          step alpha = 1 / (1 + d) of Eq. 16 (Sec. 3.2).
 * The others (grids with FP32 messages, one step per launch):
 * ADAPTIVE OURS-ADAPTIVE for binary variables (Eq. 19, Sec. 3.3): node i
 *          takes alpha_i = 1 / (1 + q_i0 q_i1 d) with d = 1 / alpha - 1.
 *          L = 2 only.
 * ADHOC    damping in mean parameters (Eq. 9, Sec. 2.2.2):
 *          q <- (1 - alpha) q + alpha softmax(-m).
 * MOMENTUM OURS-MOMENTUM (Eq. 20-21, Sec. 3.4): the message in the step is
 *          its exponential average mom <- g1 mom + (1 - g1) m (rule_gamma1 =
 *          g1), used right after the update; mom starts at m(q^0).
 * ADAM     OURS-ADAM (Eq. 22-23, Sec. 3.5), read as: the momentum average
 *          above (rule_gamma1); the per node-label second moment
 *          v <- g2 v + (1 - g2) g^2 of the natural gradient g = m + log q
 *          centred over labels (rule_gamma2, v^0 = rule_v0); the per
 *          node-label step d_t = max(sqrt(v) d + rule_eps - 1, 1e-6) with
 *          d = 1 / alpha - 1, alpha_t = 1 / (1 + d_t).
 * SWEEP    sequential mean field (Eq. 8, Sec. 2.2.1) as a chromatic
 *          Gauss-Seidel sweep: nodes are coloured so that neighbours differ
 *          (2 colours (x + y) mod 2 on 4-connected grids, 4 colours
 *          (x mod 2) + 2 (y mod 2) on 8-connected grids) and one step
 *          updates the colours in order, q_i <- softmax(-m_i) with the
 *          values of the colours already updated: exactly a sequential sweep
 *          in that node order.  alpha is not used. */
typedef enum {
  MF_RULE_FIXED = 0,
  MF_RULE_ADAPTIVE = 1,
  MF_RULE_ADHOC = 2,
  MF_RULE_MOMENTUM = 3,
  MF_RULE_ADAM = 4,
  MF_RULE_SWEEP = 5
} mf_rule;

typedef struct mf_desc {
  int32_t abi_version;     /* must be MF_ABI_VERSION */
  int32_t batch;           /* B >= 1 problems sharing graph, Theta and alpha */
  int32_t n_nodes;         /* N >= 1 */
  int32_t height, width;   /* grids: height * width == n_nodes; ignored otherwise */
  int32_t n_labels;        /* 1 <= L <= MF_MAX_LABELS (32 off grids, see MF_MAX_LABELS) */
  int32_t graph;           /* mf_graph */
  int32_t compat;          /* mf_compat */
  int32_t precision;       /* mf_precision */
  int32_t init;            /* mf_init_mode */
  double alpha;            /* step size eta = 1 / (1 + d), in (0, 1]; 1 = fully parallel */
  float potts_w;           /* POTTS weight (any finite value) */
  int32_t steps_per_launch; /* grids: proximal steps fused into one launch (temporal
                             * blocking); 0 = chosen by the library, 1 = one step per
                             * launch; clamped to what the tile fits in LDS.  With 0, a
                             * grid of at most 1024 nodes and 8 labels is held whole by
                             * one workgroup and takes up to 256 steps per launch; a
                             * grid with a general Theta, 8 < L <= 32 and at most 256
                             * tiles of 16 x 16 (B included) takes up to 4096 steps per
                             * launch in one resident workgroup per tile, the halo
                             * exchanged through the workspace after every step, when
                             * the device can hold all those workgroups at once.  Its
                             * tiles wait for each other: kernels on other streams
                             * that occupy compute units for more than 20 ms during
                             * such a launch make its waits give up (reported by
                             * mf_check); set steps_per_launch > 0 where that can
                             * happen */
  int32_t rule;            /* mf_rule (MF_RULE_FIXED = 0: the fixed-step proximal update) */
  float rule_gamma1;       /* MOMENTUM / ADAM: decay of the momentum average, in [0, 1) */
  float rule_gamma2;       /* ADAM: decay of the second moment, in [0, 1) */
  float rule_eps;          /* ADAM: epsilon >= 0 */
  float rule_v0;           /* ADAM: initial second moment >= 0 */
  /* CSR graph (graph == MF_CSR): row_ptr [N + 1] non-decreasing from 0,
   * col [nnz] in [0, N), weights [nnz] or NULL for unit weights.  The free
   * energy assumes the adjacency is symmetric. */
  const int32_t *csr_row_ptr;
  const int32_t *csr_col;
  const float *csr_w;
  int64_t csr_nnz;
  /* Dense graph (graph == MF_DENSE): K is N x N row-major bfloat16 bits
   * (uint16), symmetric with a zero diagonal; cooc is an optional [L][L]
   * symmetric co-occurrence energy applied to every pair with weight 1/N.
   * mf_init and mf_solve copy K into the workspace in the order the matrix
   * cores read it; the steps read that copy, so a change to K takes effect
   * at the next mf_init or mf_solve (mf_free_energy and mf_lipschitz read
   * dense_K itself). */
  const uint16_t *dense_K;
  const float *cooc;
  const float *unary;      /* [B][L][N] FP32, finite */
  const float *theta;      /* [L][L] FP32 (GENERAL); ignored for POTTS */
  float *state;            /* [2][B][L][N] FP32 log q, ping-pong */
  void *workspace;         /* device scratch of at least mf_workspace_size bytes */
  size_t workspace_bytes;
  void *stream;            /* hipStream_t */
  /* General graphs: lanes that gather one node's neighbour rows.  0 = the
   * library's choice (two for L > 12, one otherwise), 1 = one, 2 = two where
   * L > 12; any other value is MF_EINVAL.  One lane per node loads each row
   * whole in fewer, wider loads: faster where the node order keeps neighbours
   * close (the 2048 x 2048 grid as CSR, L = 21, FP32: 479 against 554 us
   * per step), slower on graphs without locality (a random graph of 2^20
   * nodes: 308 against 288 us) and with 16-bit messages.  Ignored for grids
   * and dense graphs. */
  int32_t csr_lanes;
} mf_desc;

typedef struct mf_handle mf_handle;

/* ABI version compiled into the library. */
int32_t mf_abi_version(void);

/* sizeof(mf_desc) as compiled into the library, for bindings that lay the
 * descriptor out themselves. */
size_t mf_desc_size(void);

/* Bytes of device workspace the problem needs (256-byte aligned start
 * required).  Returns 0 for an invalid descriptor. */
size_t mf_workspace_size(const mf_desc *d);

/* Host-side validation only: checks every rule that mf_init checks, makes
 * no HIP call.  MF_OK, MF_EINVAL, MF_EUNSUPPORTED or MF_ENOWORKSPACE. */
mf_status mf_validate(const mf_desc *d);

/* Validate, create a handle (*out), and enqueue the initialisation of
 * state buffer 0 according to d->init (Eq. 6: log q^0 = -u - lse(-u) for
 * MF_INIT_UNARY).  The descriptor is copied; its pointers are borrowed.
 * A non-finite unary is reported as MF_ENONFINITE by the next mf_check or
 * mf_free_energy.  On failure *out is NULL and nothing was enqueued. */
mf_status mf_init(const mf_desc *d, mf_handle **out);

/* Enqueue n_steps >= 0 parallel proximal steps (Eq. 15 with Eq. 16):
 * every node reads iteration t and writes t + 1 (Jacobi, double-buffered). */
mf_status mf_step(mf_handle *h, int32_t n_steps);

/* Re-initialise according to d->init, run iters steps, and if q_out is
 * not NULL write q = exp(log q) to q_out [B][L][N] (device).  With
 * MF_INIT_STATE the solve starts from whatever buffer 0 holds at the time
 * of the call (steps write buffers 1 and 0 in turn).  The fixed iteration
 * count is the stopping rule the paper uses in practice (Sec. 3.1). */
mf_status mf_solve(mf_handle *h, int32_t iters, float *q_out);

/* Free energy F(q) = E(q) - H(q) of Eq. 7 (Sec. 2.2.1) of the current
 * state, one FP64 value per batch item written to F_host[B] (host
 * memory), computed with FP64 arithmetic on the device.  F equals
 * KL(Q || P) - log Z (Eq. 5).  Synchronises the stream. */
mf_status mf_free_energy(mf_handle *h, double *F_host);

/* Enqueue q = exp(log q) of the current state into q_out [B][L][N]
 * (device): the mean parameters of Eq. 4 (Sec. 2.2).  Asynchronous. */
mf_status mf_marginals(mf_handle *h, float *q_out);

/* Synchronise the stream and report deferred device errors:
 * MF_ENONFINITE if a non-finite unary (or initial state) was seen, MF_EINVAL
 * for malformed CSR arrays, MF_EDEVICE on a HIP error or when a halo wait of
 * the persistent grid kernel gave up (its workgroups were not all resident;
 * the iterates of that launch are invalid; every wait is bounded, 20 ms or
 * the microseconds of the environment variable MF_PERSIST_WAIT_US, so the
 * launch still ends).  The conditions
 * accumulate over the initialisations since the handle was created or
 * since the last mf_check that reported one; reporting clears them. */
mf_status mf_check(mf_handle *h);

/* Device pointer to the current log q, [B][L][N] inside desc.state. */
const float *mf_current_state(const mf_handle *h);

/* Number of steps taken since the last (re)initialisation. */
int32_t mf_iteration(const mf_handle *h);

/* Proximal steps the handle fuses into one kernel launch (after the
 * library's choice and clamping), or -1 for a NULL handle. */
int32_t mf_steps_per_launch(const mf_handle *h);

/* Destroy the handle (host memory only).  Does not synchronise. */
void mf_destroy(mf_handle *h);

/* Message for the last failure on h, or of this thread when h is NULL.
 * Valid until the next call on the same handle / thread. */
const char *mf_last_error(const mf_handle *h);

/* Continuous batching (the parallel update of Eq. 15 applied to many
 * independent problems at once, Sec. 3.1): enqueue n_steps[i] >= 0
 * proximal steps for handle hs[i], i < count, in as few launches as
 * possible (grids with MF_RULE_FIXED only).
 *
 * hs:      host array of count handles; a handle may appear at most once.
 * n_steps: host array of count step counts (NULL is invalid when count > 0).
 * count:   >= 0; count == 0 enqueues nothing.
 *
 * The work runs in rounds: round r advances every handle with
 * n_steps[i] > r by one step, so problems move at their own pace inside
 * one call.  Within a round, handles with the same label count (at most 32),
 * connectivity, compatibility kind and precision share a launch; each keeps
 * its own sizes, alpha, arrays and iteration counter, with the same
 * per-tile arithmetic as mf_step at steps_per_launch = 1, so its iterates
 * are bitwise those of solving it alone that way.  A handle with more than
 * 32 labels is stepped on its own in its rounds (the kernel of mf_step at
 * one step per launch).  All handles must use the stream of hs[0]; work goes to
 * that stream.  Every argument is checked before anything is enqueued
 * (MF_EINVAL for a NULL array or handle, a negative count, a repeated
 * handle or a different stream; MF_EUNSUPPORTED for a non-grid graph or
 * another step rule). */
mf_status mf_step_many(mf_handle *const *hs, const int32_t *n_steps, int32_t count);

/* Reverse pass of T unrolled steps on a grid (hand-written adjoint of
 * Eq. 15 with Eq. 16, differentiated with respect to the unaries and every
 * entry of Theta as it appears in m = u + Theta S).
 *
 * ckpt_states: device [ceil(T / ckpt_every)][B][L][N], log q at t = 0,
 *   ckpt_every, 2 ckpt_every, ... as produced by the forward steps of h;
 *   the states between checkpoints are recomputed with one step per launch,
 *   so the forward must also have run one step per launch
 *   (steps_per_launch = 1) for the recomputation to reproduce it bitwise.
 * grad_logq_T: device [B][L][N], dLoss / d log q^T.
 * grad_unary:  device [B][L][N], overwritten with dLoss / du (including the
 *   path through log q^0 = -u - lse(-u) when h uses MF_INIT_UNARY).
 * grad_theta:  device [L][L], overwritten with dLoss / dTheta summed over
 *   the batch (for POTTS: the gradient with respect to the implied matrix).
 * work: device scratch of mf_backward_workspace_size bytes, 256-aligned.
 * Grids with MF_RULE_FIXED, FP32 messages (MF_P_F32) and at most 32 labels
 * only: MF_EUNSUPPORTED otherwise, and mf_backward_workspace_size returns 0.
 * Asynchronous on the stream of h; does not change the state of h. */
size_t mf_backward_workspace_size(const mf_handle *h, int32_t ckpt_every);
mf_status mf_backward(mf_handle *h, const float *ckpt_states, int32_t T, int32_t ckpt_every,
                      const float *grad_logq_T, float *grad_unary, float *grad_theta,
                      void *work, size_t work_bytes);

/* Lipschitz constant L-hat of the gradient of the expected energy on the
 * tangent space of the product of simplices: the largest eigenvalue of the
 * Hessian H of the pairwise (and co-occurrence) energy restricted to
 * label vectors that sum to zero at every node.  The step is admissible
 * for d > L-hat, i.e. alpha < 1 / (1 + L-hat) (Sec. 3.2; the paper
 * estimates L-hat by the power method, Sec. 3.2 and Fig. 2).  With P the
 * per-node centring, two runs of the power method:
 *   run 1 on P H P from P v0:  rho = |P H P v| / |v| at the last iteration
 *          (the spectral radius; |.| the Euclidean norm over all node-labels);
 *   run 2 on P H P + rho I from P v1 / |P v1|:  the Rayleigh quotient
 *          lambda_max + rho at the last iteration.
 * H does not depend on the unaries or the batch: item 0's graph is used.
 * v0, v1: device [L][N] FP32 start vectors (any values; centred inside).
 * iters >= 1: iterations of each run (a fixed count, as a solve's).
 * work: device scratch of mf_lipschitz_workspace_size bytes, 256-aligned.
 * lambda_max, rho: host.  FP32 Hessian-vector products, FP64 sums.
 * Synchronises the stream; does not change the state of h.  L = 1 gives
 * 0 and 0 (the tangent space is {0}); a run whose iterate vanishes stops
 * there (lambda_max = -rho when run 2 vanishes). */
/* The admissible fixed step of Sec. 3.2: alpha = 1 / (1 + d) with
 * d = margin * L-hat (d > L-hat needs margin > 1; a margin below 1 is taken
 * as 1).  L-hat <= 0 (or NaN) gives alpha = 1, the fully parallel update. */
double mf_admissible_alpha(double lipschitz, double margin);
size_t mf_lipschitz_workspace_size(const mf_handle *h);
mf_status mf_lipschitz(mf_handle *h, int32_t iters, const float *v0, const float *v1, void *work,
                       size_t work_bytes, double *lambda_max, double *rho);

/* Build the dense-CRF kernel K_ij = exp(-|f_i - f_j|^2 / 2), K_ii = 0
 * (the Gaussian kernel of the fully connected CRF, Sec. 4.2), rounded to
 * bfloat16 (round to nearest even) into K_bf16 [n][n] (device, uint16 bits).
 * features: device [n][dim] FP32, 1 <= dim <= 16.  Asynchronous. */
mf_status mf_dense_kernel(const float *features, int32_t n, int32_t dim, uint16_t *K_bf16,
                          void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mf_solve
 * without a handle and without a caller workspace.  The solve (the
 * initialisation of d->init, iters steps, q written to q_out when not NULL)
 * and, when F_out is not NULL, the FP64 free energy of the final state
 * (F_out[B], device) use the same kernels as mf_init + mf_solve +
 * mf_free_energy; their scratch (flags, FP64 partial sums, the CSR and
 * dense staging copies) is a static device array of MF_STATIC_SCRATCH_BYTES
 * that the library holds on each GPU it runs on until the process ends.
 *
 * d: as for mf_init; d->workspace and d->workspace_bytes are ignored.
 *    d->state [2][B][L][N], the unaries and every other array stay the
 *    caller's device memory.
 * flags_out: device int32 or NULL; receives the deferred-error bits of this
 *    call (bit 0: a non-finite unary or initial state, bit 1: malformed CSR
 *    arrays, bit 2: a halo wait of the persistent grid kernel gave up),
 *    which mf_check would report for a handle.
 * Returns MF_ENOWORKSPACE (before any HIP call) when the problem's
 * workspace (mf_workspace_size) exceeds MF_STATIC_SCRATCH_BYTES, and the
 * codes of mf_init otherwise.  Asynchronous on d->stream: nothing is
 * allocated, nothing synchronises.  Every call on one GPU shares that GPU's
 * scratch array and leaves its contents behind (the flags are cleared at
 * the start of each call): calls that overlap on one GPU, on different
 * streams or threads, race and give undefined results. */
#define MF_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
mf_status mf_solve_static(const mf_desc *d, int32_t iters, float *q_out, double *F_out, int32_t *flags_out);

#ifdef __cplusplus
}
#endif

#endif /* MF_H_ */
