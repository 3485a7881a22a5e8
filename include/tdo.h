/*
 * tdo.h - C-ABI of the MI355X (gfx950) hot path of the transformer
 * density-operator ansatz for steady states of dissipative spin chains
 * (arXiv 2502.20723).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Configurations of the doubled space are packed as uint64_t[2] per entry:
 *   word 0 = alpha, word 1 = beta (the row and column labels of
 *   rho(alpha, beta) in the vectorisation |rho>> = sum rho_ab |a>|b>, App. A).
 *   Bit i is site i; bit value 0 = spin up (sigma^z = +1), 1 = spin down.
 *   Bits at positions >= n are ignored: every result is that of the
 *   configuration with those bits cleared (connected configurations are
 *   written with them cleared; samples keep the bits of their inputs).
 * - Complex numbers are two consecutive floats (re, im) or doubles.
 * - Every pointer argument named as device memory must point to memory on the
 *   context's device; host pointers are marked "host".  The caller owns and
 *   allocates every input and output; the context owns its workspace.
 * - Calls are asynchronous on the given stream (NULL = the legacy default
 *   stream) unless stated otherwise; validation that needs only host data
 *   happens before any launch, and on error no kernel has been launched.
 * - Calls that take network parameters first check them for inf and nan
 *   (one read-only kernel on the stream, whose count the call waits for; the
 *   check is skipped while the stream is being captured into a graph) and
 *   return TDO_ENONFINITE with nothing else launched if any is found.
 * - Calls on one context share its workspace.  A call made on a different
 *   stream than the previous one waits (hipStreamWaitEvent, no host wait)
 *   for the end of that previous call before it touches the workspace, so a
 *   context may be used from several streams; its calls then run one after
 *   another.  Contexts are not thread-safe: one host thread at a time.
 * - Return value: TDO_OK (0) or a negative error code; the message of the
 *   last error of the calling thread is returned by tdo_last_error().
 *   Nothing aborts and no C++ exception crosses this interface.
 */
#ifndef TDO_H
#define TDO_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDO_OK 0
#define TDO_EINVAL (-1)       /* invalid argument (shape, model, pointer) */
#define TDO_ENOMEM (-2)       /* workspace budget too small or allocation failed */
#define TDO_EHIP (-3)         /* a HIP runtime call failed */
#define TDO_EUNSUPPORTED (-4) /* valid request outside what the library implements */
#define TDO_ENONFINITE (-5)   /* a network parameter is inf or nan; nothing computed */

/* Activation set of the network (tdo_arch_t.act).  TDO_ACT_RELU_FFN: exact GELU
 * u Phi(u) after each of the two embedding convolutions (Eq. circ-conv, the
 * second "in the same manner"), ReLU in the feed-forward sub-layer (the paper's
 * transformer block has none; it follows the position-wise feed-forward network
 * of the transformer it builds on).  The only set the kernels implement. */
#define TDO_ACT_RELU_FFN 0

/* Network shape.  d = width C2 of the site embeddings and attention
 * (main text, "Transformer density operator ansatz"; App. B), heads = number
 * of attention heads (d % heads == 0), layers = number of stacked
 * [attention + MLP] blocks, mlp = hidden width of the residual MLP.
 * c1 = number of filters of the first embedding convolution (App. B, C1);
 * 0 means c1 = d.  act = activation set (TDO_ACT_*).
 * Supported: d in {16, 32, 64}, d/heads in {8, 16}, mlp a multiple of 32 with
 * mlp <= 512, 1 <= layers <= 16, c1 in {0, d}, act = TDO_ACT_RELU_FFN; other
 * values return TDO_EUNSUPPORTED. */
typedef struct {
    int32_t d, heads, layers, mlp, c1, act;
} tdo_arch_t;

/* Dissipative spin chain with periodic bonds and jumps sqrt(gamma) sigma^-_i.
 * kind 0: Ising,  H = (V/4) sum sz_i sz_{i+1} + (g/2) sum sx_i  (Ising section)
 * kind 1: XYZ,    H = sum_i sum_k J_k sk_i sk_{i+1} + B_k sk_i   (Heisenberg section)
 * Fields Bx, By, Bz are used by kind 1 only; kind 0 ignores J*, B*.
 * rows: 0 or 1 for a chain.  rows = M > 1 (kind 0 only, n a multiple of M)
 * places the n sites on an M x (n/M) periodic square lattice, row-major
 * (site (r, c) is bit r (n/M) + c), and sums sz sz over its distinct
 * nearest-neighbour pairs (2D dissipative Ising paragraph of the results; a
 * ring of length 2 has one bond).  The network sees the sites in that order. */
typedef struct {
    int32_t kind, n;
    double V, g, Jx, Jy, Jz, Bx, By, Bz, gamma;
    int32_t rows;
} tdo_model_t;

typedef enum { TDO_FP32 = 0, TDO_BF16 = 1 } tdo_prec_t;

typedef struct tdo_ctx tdo_ctx_t;

/* Create a context on HIP device `device` with at most `workspace_bytes` of
 * device scratch (0 = a default of 8 GiB).  The workspace is allocated on
 * first use and reused; calls that need more than the budget process their
 * batch in chunks, and return TDO_ENOMEM only if a single chunk cannot fit. */
int32_t tdo_ctx_create(tdo_ctx_t **ctx, int32_t device, size_t workspace_bytes);
/* Synchronise the context's device and free everything it owns. */
int32_t tdo_ctx_destroy(tdo_ctx_t *ctx);

/* Number of real parameters of the ansatz (independent of n: the pooling of
 * App. B removes the chain length from the parameter shapes).  Flat layout,
 * row-major, x @ W convention, in this order:
 *   conv1_w[2 taps][2 channels][d], conv1_b[d], conv2_w[2 taps][d][d], conv2_b[d],
 *   per layer: Wq[d][d], Wk[d][d], Wv[d][d], Wo[d][d], W1[d][mlp], b1[mlp], W2[mlp][d], b2[d],
 *   head_w[d][2], head_b[2].
 * Tap 0 reads site i, tap 1 site i+1 (mod n); channel 0 = alpha, 1 = beta;
 * spins enter as s = 1 - 2*bit.  Returns -1 for an invalid arch. */
int64_t tdo_num_params(const tdo_arch_t *arch);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *tdo_last_error(void);

/* Per-kernel timing of the context's launches (measurement support, not part
 * of the method).  tdo_profile(ctx, 1) discards earlier records and starts
 * bracketing every launch of the kernel groups "fwd_layer" (one transformer
 * layer of the forward pass), "bwd_mlp" and "bwd_attn" (the backward of the
 * feed-forward and attention sub-layers) with HIP events recorded on the
 * launch stream; tdo_profile(ctx, 0) stops recording and discards the records.
 * tdo_profile_read waits for the recorded events of the named group and
 * returns the summed launch durations in milliseconds and the launch count
 * (both 0 if none).  Events are pooled by the context: no device memory is
 * allocated. */
int32_t tdo_profile(tdo_ctx_t *ctx, int32_t enable);
int32_t tdo_profile_read(tdo_ctx_t *ctx, const char *kernel, double *total_ms, int64_t *launches);

/* Nonzero entries of rows x_b = cfg[b] of the vectorised Lindbladian
 *   Lhat = -i(H (x) 1 - 1 (x) H^T) + sum_j gamma [L_j (x) L_j^* - 1/2 L_j^dag L_j (x) 1 - 1/2 1 (x) L_j^T L_j^*]
 * (Eq. VecLin; App. A), for the model.  For each row, in this slot order,
 * entries whose exact value is zero omitted:
 *   diagonal; moves on alpha (Ising: flip site i; XYZ: flip bond (i,i+1));
 *   moves on beta (same); XYZ with fields: single flips of alpha then beta;
 *   dissipator moves (flip site i of alpha and beta, present iff both bits are 1).
 * cfg: device uint64 [B][2]; conn: device uint64 [B][kmax][2]; mel: device
 * float [B][kmax][2] (complex Lhat(x; y)); n_conn: device int32 [B].  Slots
 * k >= n_conn[b] are not written.  kmax must be >= 3n+1 (5n+1 with fields).
 * Requires 3 <= n <= 64. */
int32_t tdo_connected(tdo_ctx_t *ctx, const tdo_model_t *model, const uint64_t *cfg, int64_t B,
                      int32_t kmax, uint64_t *conn, float *mel, int32_t *n_conn, hipStream_t stream);

/* Local Lindbladian estimator of App. C ("Optimization Procedure"):
 *   L(x_b) = sum_{k < n_conn[b]} mel[b][k] * exp(log_rho_conn[b][k] - log_rho_x[b]),
 * complex, in FP32.  A row with Re log_rho_x = -inf (rho(x) = 0) gives L = 0.
 * log_rho_x: device float [B][2]; mel, log_rho_conn: device float [B][kmax][2];
 * n_conn: device int32 [B]; lloc: device float [B][2]. */
int32_t tdo_local_lindbladian(tdo_ctx_t *ctx, int64_t B, const float *log_rho_x, const float *mel,
                              const int32_t *n_conn, int32_t kmax, const float *log_rho_conn,
                              float *lloc, hipStream_t stream);

/* log rho(alpha, beta) of the ansatz (Eq. log_sum_exp_conjugate on the network
 * of App. B) for B configurations of an n-site chain, 3 <= n <= 64.
 * params: device float [tdo_num_params]; cfg: device uint64 [B][2];
 * log_rho: device float [B][2] (re, im; im on the principal branch (-pi, pi]).
 * prec selects the GEMM precision (FP32 or BF16 operands, FP32 accumulation). */
int32_t tdo_log_rho(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params, int32_t n,
                    const uint64_t *cfg, int64_t B, tdo_prec_t prec, float *log_rho,
                    hipStream_t stream);

/* Vector-Jacobian product of log rho:
 *   grad = sum_b seed[b][0] * d Re log rho(x_b)/d theta + seed[b][1] * d Im log rho(x_b)/d theta.
 * seed: device float [B][2]; grad: device double [P], overwritten. */
int32_t tdo_log_rho_vjp(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params, int32_t n,
                        const uint64_t *cfg, int64_t B, tdo_prec_t prec, const float *seed,
                        double *grad, hipStream_t stream);

/* Cost and gradient at fixed samples (App. C, Eq. lossnetk):
 *   loss = sum_b w_b |L(x_b)|^2 / sum_b w_b,
 * with w_b = weights[b] (device double [B]) or 1 if weights is NULL.
 * grad_mode 0 ("B"): gradient of the self-normalised estimator
 *   F(theta) = sum r_b |L_b|^2 / sum r_b, r_b = w_b |rho_theta(x_b)|^2/|rho_theta0(x_b)|^2,
 *   at theta0, i.e.  2 Re sum w conj(L_b) sum_k c_k e^{lr(y_k)-lr(x_b)} O(y_k) - 2 loss sum w Re O(x_b)
 *   over sum w, O = d log rho/d theta; equal to d Cost/d theta when the
 *   weights are the exact |rho|^2 of all configurations.
 * grad_mode 1 ("A"): gradient of the weighted mean with w held fixed.
 * loss: device double [1]; grad: device double [P]; lloc_out: device float
 * [B][2] or NULL.  Reductions over samples are in FP64.
 * B >= 1 (a mean over no samples is rejected with TDO_EINVAL); the weights are
 * not inspected: their sum must be positive, as loss and gradient divide by it. */
int32_t tdo_loss_grad(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params,
                      const tdo_model_t *model, const uint64_t *cfg, int64_t B,
                      const double *weights, tdo_prec_t prec, int32_t grad_mode, double *loss,
                      double *grad, float *lloc_out, hipStream_t stream);

/* Cost and gradient (as tdo_loss_grad with lloc_out = NULL) of n_problems
 * independent problems sharing one architecture (App. C, Eq. lossnetk, for each
 * problem): problem p has the model models[p] (its own chain length and
 * couplings), parameters params[p] (device float [P]), samples cfg[p] (device
 * uint64 [B[p]][2]) and weights weights[p] (device double [B[p]], or NULL; the
 * array itself may be NULL), and writes loss[p] (device double [n_problems])
 * and grad[p] (device double [P]).  models, params, cfg, B, weights and grad are
 * host arrays of n_problems entries.  The problems run in order on the stream.
 * The first call with given arguments runs eagerly: it sizes the workspace for
 * the largest problem and autotunes the forward launch shape for every
 * distinct chain length.  The second identical call on a stream other than
 * the legacy default stream records the whole launch sequence into a HIP
 * graph, and every later identical call replays it (inputs are read when the
 * graph runs, so their contents may change between calls; their addresses may
 * not).  A call of any entry point that grows the context's workspace
 * invalidates the recording, which is then made again.  Every problem is
 * validated before anything is launched. */
int32_t tdo_loss_grad_batched(tdo_ctx_t *ctx, const tdo_arch_t *arch, int32_t n_problems,
                              const tdo_model_t *models, const float *const *params,
                              const uint64_t *const *cfg, const int64_t *B,
                              const double *const *weights, tdo_prec_t prec, int32_t grad_mode,
                              double *loss, double *const *grad, hipStream_t stream);

/* Tile shapes of the loss/gradient kernels for one problem's shape (chain length,
 * precision, width, head width, depth, MLP width), chosen by timing: the forward
 * layer kernel's waves per workgroup (8: two per SIMD sharing the LDS weights,
 * BF16 with n <= 32 only; or 4) and workgroups per CU (1 or 2), timed on the
 * forward over the samples; the BF16 feed-forward backward's waves per workgroup
 * at MLP width 256 (8 or 4), timed on whole loss/gradient evaluations, which
 * write loss and grad (device double [1] and [P]).  The choice is kept in the
 * context and used by every later call of that shape (tdo_loss_grad_batched
 * tunes its problems the same way on its first call); when the environment
 * variable TDO_AUTOTUNE_CACHE names a file when a context is created, tuned
 * shapes are read from that JSON file and written back to it.  The forward
 * shapes do not change results; the backward shape changes the order in which
 * weight gradients are summed, so results of one context are reproducible but
 * may differ by rounding from a context that tuned differently.  shapes: host
 * int32 [3] or NULL: forward waves, forward workgroups per CU, backward waves.
 * Waits on the host (event timing); not while the stream is captured. */
int32_t tdo_autotune(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params, const tdo_model_t *model,
                     const uint64_t *cfg, int64_t B, tdo_prec_t prec, int32_t grad_mode, double *loss,
                     double *grad, int32_t *shapes, hipStream_t stream);

/* Metropolis-Hastings on P ~ |rho|^2 (App. C, "Efficient Sampling Strategy"),
 * `chains` independent chains, `sweeps` sweeps of 2n proposals each.  Proposal
 * t of chain c draws Philox4x32-10 (Salmon et al., SC'11) with counter
 * (t mod 2^32, t >> 32, c, 0) and key (seed mod 2^32, seed >> 32), words r0..r2:
 *   pair move iff r0 < floor(p_pair 2^32), flipping alpha_i and beta_i at
 *   i = (r1 n) >> 32; otherwise flip bit j = (r1 2n) >> 32 of (alpha, beta);
 *   accept iff (r2 + 0.5) 2^-32 < exp(2 Re(log rho' - log rho)).
 * state: device uint64 [chains][2] in/out; state_log_rho: device float
 * [chains][2] in/out (log rho of the states, as returned by tdo_log_rho);
 * counter: host uint64, in/out, the proposal index t of the first proposal
 * (advanced by sweeps*2n); samples: device uint64 [sweeps][chains][2], the state
 * after each sweep.  0 <= p_pair <= 1. */
int32_t tdo_sample(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params, int32_t n,
                   int64_t chains, uint64_t *state, float *state_log_rho, uint64_t seed,
                   uint64_t *counter, int32_t sweeps, float p_pair, tdo_prec_t prec,
                   uint64_t *samples, hipStream_t stream);

/* Metropolis-Hastings on the diagonal, P(alpha) ~ |rho(alpha, alpha)|: the
 * distribution of the mixed-state observable estimators (supplementary section
 * on mixed-state observables; App. C, sampling strategy).  The ansatz's
 * diagonal is real but may be negative, so the chain targets its modulus and
 * the sign is applied as a weight by tdo_observables and tdo_purity.
 * `chains` independent chains, `sweeps` sweeps of n proposals each.  Proposal t
 * of chain c draws Philox4x32-10 with counter (t mod 2^32, t >> 32, c, 1) and
 * key (seed mod 2^32, seed >> 32), words r1, r2: flip site i = (r1 n) >> 32 of
 * alpha; accept iff (r2 + 0.5) 2^-32 < exp(Re log rho(alpha', alpha') -
 * Re log rho(alpha, alpha)).
 * state: device uint64 [chains] in/out (alpha); state_log_rho: device float
 * [chains][2] in/out, log rho(alpha, alpha) of the states (tdo_log_rho of the
 * rows (alpha, alpha)); counter: host uint64 in/out, the proposal index of the
 * first proposal (advanced by sweeps*n); samples: device uint64
 * [sweeps][chains], alpha after each sweep.  A chain whose state has
 * rho(alpha, alpha) = 0 accepts the first proposal with a nonzero diagonal. */
int32_t tdo_sample_diag(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params, int32_t n,
                        int64_t chains, uint64_t *state, float *state_log_rho, uint64_t seed,
                        uint64_t *counter, int32_t sweeps, tdo_prec_t prec, uint64_t *samples,
                        hipStream_t stream);

/* Local estimators of the magnetisation (supplementary section on mixed-state
 * observables; App. C, evaluation of local observables; Heisenberg section for
 * the site averages): for each sample alpha (device uint64 [B]),
 *   A~(alpha) = sum_beta rho(alpha, beta) / rho(alpha, alpha) <beta|A|alpha>
 * for A = (1/n) sum_i sigma^k_i, k = x, y, z, with bit 0 = spin up
 * (sigma^z = +1).  One sample costs n + 1 network evaluations, the rows
 * (alpha, alpha) and (alpha, alpha with site i flipped).
 * log_rho_diag: device float [B][2], log rho(alpha, alpha) (imaginary part pi
 * where the diagonal is negative, real part -inf where it vanishes);
 * local: device float [B][3][2], (re, im) of A~ for x, y, z; local_site:
 * device float [B][n][3][2] or NULL, the same for each single-site sigma^k_i
 * (local is their average over i).  Where
 * rho(alpha, alpha) = 0 the ratios are read as 0 (sigma^z keeps its diagonal
 * value).  mean: device double [7] or NULL: mean[0..5] = sum s A~ / sum s over
 * the B samples for x, y, z as (re, im), with s = sign of rho(alpha, alpha),
 * the estimate of <A> when the samples come from |rho(alpha, alpha)|
 * (tdo_sample_diag); mean[6] = sum s / B.  mean needs B >= 1; sum s = 0 gives
 * non-finite means.  Sums are FP64 in a fixed order. */
int32_t tdo_observables(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params, int32_t n,
                        const uint64_t *alpha, int64_t B, tdo_prec_t prec, float *log_rho_diag,
                        float *local, float *local_site, double *mean, hipStream_t stream);

/* Purity Tr(rho^2) / (Tr rho)^2 (Ising section) from P >= 1 pairs of
 * independent diagonal samples (alpha_p, beta_p) (device uint64 [P] each, e.g.
 * two different chains of tdo_sample_diag):
 *   out[0] = mean_p t_p / (mean s)^2,
 *   t_p = |rho(alpha, beta)|^2 / (|rho(alpha, alpha)| |rho(beta, beta)|),
 * with s the sign of the diagonal over all 2P samples; out[1] = mean s.
 * t_p = 0 when either diagonal vanishes.  Three network evaluations per pair.
 * out: device double [2].  Sums are FP64 in a fixed order. */
int32_t tdo_purity(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params, int32_t n,
                   const uint64_t *alpha, const uint64_t *beta, int64_t P, tdo_prec_t prec,
                   double *out, hipStream_t stream);

/* Learning rate of the training loop (App. C, learning-rate scheduling): eta0
 * for step < i_switch, then eta0 (1 + cos(pi x)) / 2 + alpha eta0 with
 * x = min(1, (step - i_switch) / i_decay) (the rate stays at alpha eta0 after
 * the decay period).  Host code: needs no device. */
double tdo_lr_schedule(int64_t step, double eta0, int64_t i_switch, int64_t i_decay, double alpha);

/* First-order update theta <- theta - lr grad (App. C, optimisation procedure,
 * SGD).  params: device float [P] in/out; grad: device double [P] (as written
 * by tdo_loss_grad).  Formed in FP64, rounded once to FP32.  P >= 0. */
int32_t tdo_sgd_step(int64_t P, float *params, const double *grad, double lr, hipStream_t stream);

/* Adam update (App. C, optimisation procedure; Kingma and Ba, ICLR 2015,
 * Algorithm 1) at step t >= 1: m <- beta1 m + (1 - beta1) g,
 * v <- beta2 v + (1 - beta2) g^2, theta <- theta - lr m_hat / (sqrt(v_hat) + eps)
 * with m_hat = m / (1 - beta1^t), v_hat = v / (1 - beta2^t).  params: device
 * float [P] in/out; grad: device double [P]; m, v: device double [P] in/out,
 * zero before step 1.  0 <= beta < 1, eps > 0.  Formed in FP64 without fused
 * multiply-adds, rounded once to FP32. */
int32_t tdo_adam_step(int64_t P, float *params, const double *grad, double *m, double *v, int64_t t,
                      double lr, double beta1, double beta2, double eps, hipStream_t stream);

/* Per-sample log-derivatives O_k(x_b) = d log rho(x_b) / d theta_k (App. C,
 * metric tensor of stochastic reconfiguration): jac, device double
 * [B][2][P], row (b, 0) the real and row (b, 1) the imaginary part.  Per
 * configuration one forward and one backward per row through the kernels of
 * tdo_log_rho_vjp, on weights packed once; configurations are spread over four
 * internal streams (default priority) that wait for `stream` and that `stream`
 * then waits for.  The call returns after the rows are written (it waits on
 * the host). */
int32_t tdo_log_rho_jacobian(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params, int32_t n,
                             const uint64_t *cfg, int64_t B, tdo_prec_t prec, double *jac,
                             hipStream_t stream);

/* Stochastic reconfiguration (App. C, metric tensor and hybrid update): x =
 * (S + lambda I)^-1 g with S = Re sum_b w_b conj(dO(x_b)) dO(x_b)^T,
 * dO = O - sum_b w_b O(x_b), weights normalised to sum 1 (weights: device
 * double [B], non-negative with a positive sum, or NULL for equal weights).  jac: device double [B][2][P] from
 * tdo_log_rho_jacobian, centred and scaled in place (rows sqrt(w_b) dO).
 * grad: device double [P]; x: device double [P], written.  Conjugate gradients
 * from x = 0 for exactly `iters` iterations (S is applied as J^T (J p), never
 * formed); info: device double [2] or NULL: the relative residual |r|/|g| of
 * the recurrence and |g|.  lambda > 0. */
int32_t tdo_sr_solve(tdo_ctx_t *ctx, double *jac, int64_t B, int64_t P, const double *weights,
                     const double *grad, double lambda, int32_t iters, double *x, double *info,
                     hipStream_t stream);

/* Jacobian-vector product of log rho (App. C, metric tensor of stochastic
 * reconfiguration: the products O(x_b) . p that apply S without forming it):
 *   jvp[b] = sum_k d log rho(x_b)/d theta_k tangent[k]   (complex: re, im),
 * by forward-mode differentiation of the network in FP32 (the tangent of every
 * stage evaluated with its value; not the fused MFMA kernels).  tangent: device
 * double [P]; jvp: device float [B][2].  3 <= n <= 64. */
int32_t tdo_log_rho_jvp(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params, int32_t n,
                        const uint64_t *cfg, int64_t B, const double *tangent, float *jvp,
                        hipStream_t stream);

/* Stochastic reconfiguration without the Jacobian (App. C, metric tensor and
 * hybrid update): the same solve as tdo_sr_solve, x = (S + lambda I)^-1 grad by
 * conjugate gradients from x = 0 for exactly `iters` iterations, with S applied
 * as S p = J^T (J p): per iteration one forward-mode pass over the samples
 * (tdo_log_rho_jvp, FP32) and one reverse-mode pass (tdo_log_rho_vjp in
 * precision prec) with the seeds w_b (t_b - sum_b' w_b' t_b'), t = J p, w the
 * weights normalised to sum 1.  Nothing of size B x P is stored, so B is bounded
 * only by the workspace chunking.  cfg: device uint64 [B][2]; weights: device
 * double [B] (non-negative, positive sum) or NULL; grad, x: device double [P];
 * info: device double [2] or NULL (relative residual of the recurrence, |g|). */
int32_t tdo_sr_solve_matfree(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params, int32_t n,
                             const uint64_t *cfg, int64_t B, const double *weights, tdo_prec_t prec,
                             const double *grad, double lambda, int32_t iters, double *x, double *info,
                             hipStream_t stream);

/* log rho exactly as tdo_log_rho computes it, without allocating device memory:
 * for callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The work memory is a fixed array of
 * TDO_NOALLOC_SCRATCH_BYTES in the library's device image, one per device, held
 * until the process ends; its device address is looked up when a context is
 * created on the device (tdo_ctx_create), so ctx must be a context of the device
 * that holds params, cfg and log_rho (its workspace is not used).  Batches of any
 * size run in chunks that fit the array; TDO_ENOMEM if the packed weights alone
 * do not (never for the supported architectures: at most 5.3 MB).  The call
 * launches kernels only: no allocation, no host wait, no parameter check (inf or
 * nan parameters give non-finite results).  Every call on one device uses the
 * same array: calls that overlap in time on one device (other streams, other
 * threads) race and give wrong results; calls ordered on one stream are safe. */
#define TDO_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int32_t tdo_log_rho_noalloc(tdo_ctx_t *ctx, const tdo_arch_t *arch, const float *params, int32_t n,
                            const uint64_t *cfg, int64_t B, tdo_prec_t prec, float *log_rho,
                            hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TDO_H */
