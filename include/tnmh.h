/*
 * tnmh.h -- C ABI of the MI355X (gfx950) tensor-network Metropolis-Hastings
 * library: boundary-MPS environments of the 2D Ising Boltzmann network, the
 * sequential sampler that draws whole configurations with their proposal
 * log-probability, the MH acceptance step and the derivative of ln Z~.
 *
 * Paper: "Collective Monte Carlo updates through tensor network
 * renormalization" (arXiv:2104.13264).
 *
 * Conventions shared by every call
 *   Lattice Ly x Lx, open boundaries; row r = 0..Ly-1, column c = 0..Lx-1,
 *   site i = r*Lx + c.  Spins are int8 +1/-1.
 *   Jh [Ly][Lx-1]  coupling of (r,c)-(r,c+1)          float64, row-major
 *   Jv [Ly-1][Lx]  coupling of (r,c)-(r+1,c)          float64, row-major
 *   h  [Ly][Lx]    site field, or NULL meaning 0      float64, row-major
 *   Energy H(s) = -sum h s - sum J s s'   (Sec. 2, Eq. ising).
 *   Pointers marked (dev) are device memory of the current HIP device owned
 *   by the caller; (host) are host memory owned by the caller.  Every call is
 *   asynchronous on the context's stream unless it returns a host value.
 *
 * Random numbers (the paper leaves them open): Philox4x32-10 with key = seed,
 *   spin draw of site i of proposal id at step t:
 *       counter (i/4, id, t, inst<<2 | 0), word i%4
 *   acceptance draw of chain j at step t:
 *       counter (0, j, t, inst<<2 | 1), word 0
 *   mapped to u = (x + 0.5) * 2^-32 in float64; spin +1 iff u < p+.
 *
 * Errors: every int-returning call returns TN_OK (0) or a negative code and
 *   leaves a message in tn_last_error(ctx).  No C++ exception crosses the ABI.
 */
#ifndef TNMH_H
#define TNMH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tn_ctx tn_ctx;

enum tn_status {
    TN_OK = 0,
    TN_EINVAL = -1,   /* bad argument (size, NULL pointer, non-finite beta) */
    TN_ENOMEM = -2,   /* device allocation failed */
    TN_EHIP = -3,     /* a HIP runtime call failed */
    TN_ENONPOS = -4,  /* Z~ <= 0 or not finite (App. A: positivity) */
    TN_ENOCONV = -5,  /* Jacobi SVD did not converge */
    TN_ESTATE = -6    /* call order: sampling before an environment exists */
};

/* Arithmetic of the sampler.  The environment build (QR/SVD truncation and
 * log-normalisers) is float64 in every case.
 *   TN_FP64       plain path: float64 vector arithmetic, one launch per row
 *   TN_FP32       batched path: float32 MFMA contractions (fp32 accumulate),
 *                 persistent kernel over all rows, p and ln q in float64
 *   TN_BF16       batched path with bf16 operands and fp32 accumulation
 *   TN_FP64_MFMA  batched path with float64 operands and vectors on the
 *                 fp64 matrix cores (D <= 32): the conditionals of the plain
 *                 path at batched cost, for low temperatures, where the small
 *                 conditional weights come out of cancelling inner products
 *                 that float32 cannot resolve.  Negative weights are clamped
 *                 to 0 as in TN_FP64.  Single instances only (the batched
 *                 uneven-instance and periodic calls take TN_FP64, TN_FP32 or
 *                 TN_BF16).                                                  */
enum tn_prec { TN_FP64 = 0, TN_FP32 = 1, TN_BF16 = 2, TN_FP64_MFMA = 3 };

/* Create a context bound to `hip_stream` (a hipStream_t, or NULL for the
 * null stream) on the current device.  *out receives the handle. */
int tn_create(tn_ctx **out, void *hip_stream);

/* Free the context, its environment stack and its scratch.  NULL is a no-op. */
int tn_destroy(tn_ctx *ctx);

/* Message of the last failed call on ctx (never NULL; "" after success). */
const char *tn_last_error(const tn_ctx *ctx);

/* Boundary-MPS environments (App. A, Eq. braket-top-tm-bot and the
 * MPO-MPS renormalisation figure), contracted bottom-up: env k (k=1..Ly-1)
 * approximates rows k..Ly-1 with their up legs open.  Each row MPO is applied
 * to env k+1 and the product is compressed to bond D by a left-to-right
 * Householder QR sweep and a right-to-left one-sided Jacobi SVD sweep keeping
 * the min(D, rows, cols) largest singular values ("successive SVD").
 *   Jh, Jv, h  (dev, fp64) couplings and field, layouts above (h may be NULL)
 *   beta       inverse temperature, finite
 *   D          bond dimension, 1 <= D <= 64
 *   prec       sampler arithmetic (enum tn_prec)
 *   logZ_out   (host, may be NULL) receives ln Z~ = sum_k ell_k + ln<top|env_1>
 * Replaces any previous environment.  Synchronises the stream when logZ_out
 * is not NULL.  TN_ENONPOS if <top|env_1> <= 0 or ln Z~ is not finite. */
int tn_build_env(tn_ctx *ctx, int Lx, int Ly, const double *Jh, const double *Jv,
                 const double *h, double beta, int D, int prec, double *logZ_out);

/* tn_build_env in three calls, for builds long enough to report progress:
 * begin records the instance (as tn_build_env) and prepares the build; each
 * tn_build_env_rows call builds the next `nrows` rows bottom-up and returns
 * when they are done (rows_left, host, may be NULL: rows still to build);
 * end builds what remains, the top overlap and the sampler operands and
 * gives ln Z~.  Other calls on the context fail with TN_ESTATE in between. */
int tn_build_env_begin(tn_ctx *ctx, int Lx, int Ly, const double *Jh, const double *Jv,
                       const double *h, double beta, int D, int prec);
int tn_build_env_rows(tn_ctx *ctx, int nrows, int *rows_left);
int tn_build_env_end(tn_ctx *ctx, double *logZ_out);

/* q-state Potts models: the method for a general local dimension d (App. A
 * writes any nearest-neighbour model whose variables take d values through
 * d x d bond matrices, Eq. pf_bond_description, split into site tensors,
 * Eq. tensor-general; Sec. 2 notes that the sampler carries over to the
 * Potts model).  Energy H(s) = - sum_<ij> J_ij delta(s_i, s_j)
 * - sum_i h_i(s_i), values s in 0..d-1 stored as int8.  The bond matrix
 * exp(beta J delta) is split through its eigenbasis (the uniform vector and
 * Helmert's orthonormal basis of its complement, lambda_0 = e^K - 1 + d,
 * lambda_mu = e^K - 1): P(s, mu) = e_mu(s) sqrt|lambda_mu|, Q(mu, s) =
 * sign(lambda_mu) sqrt|lambda_mu| e_mu(s).  The environments are built as
 * for Ising (bottom-up, QR sweep and successive SVD to D, fp64).
 *   d          number of values, 2..6
 *   Jh, Jv     (dev, fp64) couplings as in tn_build_env
 *   h          (dev, fp64 [Ly][Lx][d], or NULL for 0) field of every value
 *   D          bond dimension, 1..32
 *   logZ_out   (host, may be NULL) ln Z~
 * Afterwards the context is a Potts context until the next build: tn_sample,
 * tn_sample_noalloc, tn_sample_steps, tn_eval_logq, tn_mh_step, tn_mh_accept
 * and tn_mh_run work on value configurations (int8 [.][Ly][Lx], values
 * 0..d-1) with the plain fp64 sampler: snake order, each conditional the
 * categorical law of the d weights contracted from the same env, the draw
 * the smallest value k with u (w_0 + .. + w_{d-1}) < w_0 + .. + w_k (u as for
 * Ising); the Ising-only calls (tn_set_precision, tn_get_env, tn_grad,
 * tn_grad_two_sided, tn_logz_frozen, tn_metropolis_sweeps, tn_link_overlap,
 * tn_autotune) return TN_EINVAL.  Errors: TN_EINVAL for arguments out of
 * range, fitted compression (tn_set_compression > 0); TN_ENOCONV, TN_ENONPOS
 * as for tn_build_env.  Synchronises the stream. */
int tn_potts_build_env(tn_ctx *ctx, int Lx, int Ly, int d, const double *Jh, const double *Jv,
                       const double *h, double beta, int D, double *logZ_out);

/* Install an environment computed elsewhere (or saved by tn_get_env) instead
 * of building it.  Couplings as in tn_build_env (dev).  Host arrays:
 *   env   [(Ly-1)][Lx][D][2][D] fp64: env k=1..Ly-1, tensor E[a][u][b] of column
 *         c zero-padded to D x 2 x D (a: left bond, u: leg of the vertical
 *         bond above the env, b: right bond)
 *   dims  [(Ly-1)][Lx+1] int: bond dims of env k; dims[.][0] = dims[.][Lx] = 1
 *   ell   [Ly-1] fp64: log-normaliser of env k (informational)
 *   logZ  ln Z~ stored with the environment */
int tn_set_env(tn_ctx *ctx, int Lx, int Ly, const double *Jh, const double *Jv,
               const double *h, double beta, int D, int prec, const double *env,
               const int *dims, const double *ell, double logZ);

/* Copy the current environment to host arrays laid out as in tn_set_env
 * (any pointer may be NULL to skip it).  Synchronises the stream. */
int tn_get_env(tn_ctx *ctx, double *env, int *dims, double *ell, double *logZ);

/* Switch the sampler arithmetic of an existing environment (re-derives the
 * sampler operands from the fp64 environment; no rebuild). */
int tn_set_precision(tn_ctx *ctx, int prec);

/* Instance tag written into the Philox counter (inst << 2 | stream); 0..2^29-1. */
int tn_set_instance(tn_ctx *ctx, int inst);

/* Compression of the later builds on this context (tn_build_env, the
 * incremental build, tn_build_env_multi, tn_periodic_setup).  App. A names two
 * schemes: successive SVD (fit_sweeps = 0, the default) and two-site
 * variational compression, used there for the Gaussian-disorder runs.  With
 * fit_sweeps = n in 1..16 every row is first compressed by successive SVD,
 * then n sweeps (each a left-to-right and a right-to-left pass) of two-site
 * updates fit the bond-D MPS to the normalised MPO-MPS product: with the
 * blocks left and right of a bond orthonormal, the two-site tensor is the
 * product contracted with those blocks, split by an SVD truncated to D.  The
 * stored env is right-orthonormal with its centre at column 0 as before and
 * ell_k = ln of the product's norm removed by the QR sweep + ln |fit|.
 * Supported for D <= 32 (a build with larger D fails with TN_EINVAL).  The
 * frozen-truncation derivative tn_grad is defined for successive-SVD builds
 * only (TN_ESTATE after a fitted build); tn_grad_two_sided works with either.
 * Errors: TN_EINVAL for fit_sweeps outside 0..16. */
int tn_set_compression(tn_ctx *ctx, int fit_sweeps);

/* Draw `batch` independent proposals by the sequential Bayes chain rule
 * (Sec. 2, Eqs. bayes, pi-approx; App. A Eq. proba-ratio-apx), each
 * conditional normalised over s in {+1,-1} from the same stored environment.
 * Site order of the chain rule: snake order, row 0 first, even rows left to
 * right (c = 0..Lx-1), odd rows right to left (c = Lx-1..0); ln q is the sum
 * of the ln p of the conditionals taken in that order.  (The random word a
 * site draws is keyed by its row-major index i = r*Lx + c, whatever the
 * order.)  Proposal j uses id = first_id + j.
 *   spins  (dev, int8 [batch][Ly][Lx])  drawn configurations
 *   logq   (dev, fp64 [batch])          ln q(s) of the arithmetic that drew s
 *   energy (dev, fp64 [batch])          H(s)
 * Negative conditional weights are clamped to 0 by the FP64 path; the FP32
 * and BF16 paths raise every weight below 2^-24 of |w+| + |w-| to that floor,
 * so that each configuration keeps a positive proposal probability (either
 * way counted in tn_stats).  If both are <= 0 the draw uses p+ = 1/2.
 * TN_ESTATE before an environment. */
int tn_sample(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step, uint64_t first_id,
              int8_t *spins, double *logq, double *energy);

/* tn_sample for callers that cannot allocate device memory: code under HIP
 * graph capture of their own, tight serving loops, harnesses that forbid
 * hipMalloc.  Arguments, proposals (bitwise those of tn_sample with the same
 * arguments), errors and ownership as in tn_sample; the call allocates and
 * frees nothing (no hipMalloc, hipFree or allocating library routine).  The
 * sampler's scratch (the per-proposal right-environment tiles of the rows in
 * flight) comes from a fixed 64 MiB device array inside the library instead
 * of a context allocation; each GPU the library runs on holds its own copy
 * until the process ends.  Need: FP32/BF16 32 * Lx * Dp * (batch rounded up
 * to 128) bytes (Dp = D rounded up to 16), FP64 16 * Lx * D * batch bytes;
 * e.g. 4096 proposals of a 64-wide lattice at D = 32 in FP32.  A larger batch
 * fails with TN_EINVAL and a message giving both sizes.  Every call on a GPU
 * shares that GPU's array and leaves its contents there; nothing in it needs
 * to start at zero (a call reads only what it wrote).  Calls that overlap in
 * time on one GPU (on different streams, or from different contexts) race on
 * the array: the caller serialises them.  The context's device must be
 * current (TN_EINVAL otherwise); TN_EHIP if the array's address could not be
 * taken when the context was created. */
int tn_sample_noalloc(tn_ctx *ctx, int batch, uint64_t seed, uint64_t step, uint64_t first_id,
                      int8_t *spins, double *logq, double *energy);

/* ln q(s) and H(s) of given configurations by exactly the arithmetic of
 * tn_sample (the forced-spin mode of the same kernels).
 *   spins (dev, int8 [batch][Ly][Lx]), logq, energy (dev, fp64 [batch]) */
int tn_eval_logq(tn_ctx *ctx, int batch, const int8_t *spins, double *logq,
                 double *energy);

/* One step of Algorithm 1 for `chains` independent chains: chain j draws its
 * proposal with id = j at step `step`, accepts it with probability
 * min{1, q(w)/q(w') * exp(-beta (H(w') - H(w)))} (Eqs. mh-acc, tns-prior),
 * and on acceptance copies it into its state (in place).
 *   state_spins (dev, int8 [chains][Ly][Lx]); state_logq, state_energy (dev,
 *   fp64 [chains]) must hold ln q and H of the state (tn_eval_logq);
 *   accepted (dev, uint8 [chains]) receives 1/0.
 * Uses context-owned proposal buffers; launches only, so it can be captured
 * into a HIP graph after one warm-up call with the same chain count. */
int tn_mh_step(tn_ctx *ctx, int chains, uint64_t seed, uint64_t step,
               int8_t *state_spins, double *state_logq, double *state_energy,
               uint8_t *accepted);

/* The acceptance half of tn_mh_step for proposals the caller already drew
 * (tn_sample with first_id = 0 and the same step): chain j accepts proposal j
 * with the probability of Eqs. (mh-acc, tns-prior) and copies it into its
 * state on acceptance.
 *   prop_spins (dev, int8 [chains][Ly][Lx]), prop_logq, prop_energy (dev, fp64)
 *   state_* and accepted as in tn_mh_step. */
int tn_mh_accept(tn_ctx *ctx, int chains, uint64_t seed, uint64_t step,
                 const int8_t *prop_spins, const double *prop_logq,
                 const double *prop_energy, int8_t *state_spins, double *state_logq,
                 double *state_energy, uint8_t *accepted);

/* Proposals of `nsteps` consecutive MH steps in one call: the candidate of
 * Algorithm 1 is drawn from q alone, independently of the chain's state
 * (Sec. 2), so the proposals of several steps can be drawn together.
 * Proposal (t, j) has id first_id + j and step step0 + t and is bitwise the
 * one tn_sample(batch = chains, step = step0 + t, first_id) draws.
 *   spins (dev, int8 [nsteps][chains][Ly][Lx]), logq, energy (dev, fp64
 *   [nsteps][chains]).  TN_EINVAL for nsteps < 1 or chains < 0. */
int tn_sample_steps(tn_ctx *ctx, int chains, int nsteps, uint64_t seed, uint64_t step0,
                    uint64_t first_id, int8_t *spins, double *logq, double *energy);

/* `nsteps` steps of Algorithm 1 (steps step0 .. step0 + nsteps - 1) for
 * `chains` chains: the proposals of several steps are drawn per sampler
 * launch (tn_sample_steps, enough to fill the GPU), then accepted step by
 * step exactly as tn_mh_step would; the chains end bitwise where nsteps calls
 * of tn_mh_step leave them.
 *   state_* as in tn_mh_step; accepted (dev, uint8 [nsteps][chains]);
 *   energy_series (dev, fp64 [nsteps][chains], or NULL): the state energy
 *   after each step.  Context-owned proposal buffers hold up to the launch's
 *   steps. */
int tn_mh_run(tn_ctx *ctx, int chains, int nsteps, uint64_t seed, uint64_t step0,
              int8_t *state_spins, double *state_logq, double *state_energy,
              uint8_t *accepted, double *energy_series);

/* Single-spin-flip Metropolis sweeps of every chain's state, to interleave
 * with TNMH steps (Sec. 3 reports that spin-flip sweeps between TNMH moves
 * help chains the approximate prior alone leaves stuck).  A sweep updates all
 * sites with r + c even, then all with r + c odd (sites of one colour share no
 * bond); at site i with spin s and local field F = h_i + sum of J s over the
 * neighbours (left, right, up, down, in this order), the flip changes the
 * energy of Eq. (ising) by dE = 2 s F and is accepted iff u < exp(-beta dE).
 * u: word i % 4 of Philox4x32-10 at counter (sweep * 2^14 + i / 4, chain,
 * step, instance << 2 | 2) on key `seed`, mapped to (x + 1/2) 2^-32.
 * Afterwards ln q and E of the new states are evaluated by the arithmetic of
 * the proposals (as tn_eval_logq), so the next tn_mh_step weighs them alike.
 *   state_spins (dev, int8 [chains][Ly][Lx], updated in place), state_logq,
 *   state_energy (dev, fp64 [chains], overwritten).
 * Errors: TN_ESTATE without an environment; TN_EINVAL for chains or nsweeps
 * < 0, nsweeps >= 2^18, more than 65536 sites, NULL buffers.  Accepted flips
 * are counted in tn_stats. */
int tn_metropolis_sweeps(tn_ctx *ctx, int chains, int nsweeps, uint64_t seed, uint64_t step,
                         int8_t *state_spins, double *state_logq, double *state_energy);

/* Link overlap of configuration pairs: q[k] = sum over the bonds <ij> of
 * a_i a_j b_i b_j (k < n), the two-replica estimate of sum_<ij> <s_i s_j>^2 in
 * the equilibration test of Sec. 3, Eq. (Delta).
 *   a, b (dev, int8 [n][Ly][Lx]) on this context's lattice; q (dev, int32 [n]).
 * Errors: TN_ESTATE without an environment (the lattice size comes from it),
 * TN_EINVAL for n < 0 or NULL buffers. */
int tn_link_overlap(tn_ctx *ctx, int n, const int8_t *a, const int8_t *b, int32_t *q);

/* ---- Batched uneven instances -------------------------------------------
 * Many independent instances (lattice, couplings, beta, bond cap) sampled
 * together: their environment builds run side by side (one workgroup per
 * instance), and one MH step of all their chains is one sampler launch per
 * bond class (D rounded up to 16) and one acceptance launch.  Instance i draws
 * with Philox instance number i (counter word 3 = i << 2 | stream). */
typedef struct {
    int Lx, Ly, D;
    double beta;
    const double *Jh, *Jv, *h;   /* dev, fp64, as in tn_build_env (h may be NULL) */
    int chains;                  /* chains of this instance in tn_mh_step_multi */
} tn_instance;

/* Build the environments of n instances (the batched context's own ones,
 * replacing earlier ones); logZ_out (host, fp64 [n], may be NULL) receives
 * ln Z~ per instance.  prec as in tn_build_env for all instances.  Errors name
 * the first failing instance; synchronises. */
int tn_build_env_multi(tn_ctx *ctx, int n, const tn_instance *inst, int prec, double *logZ_out);

/* One MH step (Algorithm 1) of every chain of every instance: the arrays hold
 * n host pointers each, entry i pointing to instance i's device state
 * (spins int8 [chains_i][Ly_i][Lx_i], logq and energy fp64 [chains_i],
 * accepted uint8 [chains_i]).  Chains are bitwise those tn_mh_step gives a
 * single-instance context with the same instance number.  Errors: TN_EINVAL
 * if an instance was switched to TN_FP64_MFMA (tn_set_precision on
 * tn_multi_instance's context): batched steps take TN_FP64, TN_FP32 and
 * TN_BF16 instances. */
int tn_mh_step_multi(tn_ctx *ctx, uint64_t seed, uint64_t step, int8_t *const *state_spins,
                     double *const *state_logq, double *const *state_energy,
                     uint8_t *const *accepted);

/* Instance i of a batched context as a context of its own, borrowed (owned
 * and destroyed by ctx, valid until the next tn_build_env_multi): every
 * single-instance call applies to it (tn_eval_logq for initial states,
 * tn_sample, tn_mh_step, tn_stats, tn_grad).  NULL when i is out of range. */
tn_ctx *tn_multi_instance(tn_ctx *ctx, int i);

/* Capture the following tn_mh_step / tn_mh_step_multi calls of this context
 * (consecutive steps) into a HIP graph instead of running them.  The context
 * must have been created with a stream other than the legacy default one, and
 * every captured call must have been made once before (same chain counts and
 * state buffers: no allocation happens while capturing; a step that would
 * need a larger buffer fails with TN_ESTATE).  Between tn_graph_begin and
 * tn_graph_end_and_replay every other call on the context (tn_sample,
 * tn_sample_steps, tn_eval_logq, tn_mh_accept, tn_mh_run,
 * tn_metropolis_sweeps, tn_link_overlap, the builds, tn_get_env,
 * tn_set_precision, tn_grad, tn_stats, ...) returns TN_ESTATE: their random
 * streams would not follow the replays' step shift, or they synchronise. */
int tn_graph_begin(tn_ctx *ctx);

/* End the capture and replay the graph n_replays times: replay r runs the
 * captured steps shifted by r times their count, so the replays continue the
 * captured sequence step by step (bitwise the eager calls). */
int tn_graph_end_and_replay(tn_ctx *ctx, int n_replays);

/* Derivative of ln Z~, the logarithm of the approximate contraction (Sec. 4
 * compares energies taken from such derivatives with sampled ones, caption of
 * its TRG comparison figure), with the truncation isometries frozen: every
 * compression step of the environment build is replaced by the orthogonal
 * projector onto the span kept at its leftmost truncated bond (the identity
 * where nothing was truncated), which makes Z~ multilinear in the site
 * tensors; the adjoint sweeps the rows top-down with exact per-row
 * environments.  It is the exact derivative of that frozen contraction (equal
 * to Z~ at the build point), and of ln Z without truncation.  With
 * truncation it is not an estimate of the bond correlations: on a 128 x 128
 * fully frustrated lattice at D = 32 it gives 0.90 for a bulk bond whose
 * correlation is 0.46, and d ln Z~/d beta = 23882 against -<E> = 15070 (use
 * tn_grad_two_sided for those).
 *   dJh (dev, fp64 [Ly][Lx-1]), dJv (dev, fp64 [Ly-1][Lx]): d ln Z~ / dJ
 *   dbeta (host, may be NULL): d ln Z~ / d beta
 * Errors: TN_ESTATE without an environment, after a fitted build
 * (tn_set_compression) or while capturing; TN_EINVAL for NULL gradient
 * buffers or beta*J = 0 on a bond.  Synchronises the stream. */
int tn_grad(tn_ctx *ctx, double *dJh, double *dJv, double *dbeta);

/* The frozen contraction whose derivative tn_grad takes, evaluated at other
 * couplings, so that tn_grad can be checked by central finite differences
 * (Sec. 4 derives energies from derivatives of the approximate
 * contraction): ln Z~_frozen(J', h', beta') =
 * ln <top| P_1 TM_1 P_2 TM_2 ... P_{Ly-1} TM_{Ly-1} |.>, the transfer
 * matrices TM_k built from the given couplings and each P_k the orthogonal
 * projector onto the span the current build kept at its leftmost truncated
 * column (the identity where it truncated nothing).  At the build's own
 * couplings it equals ln Z~.  n coupling sets are evaluated as one batched
 * build (one workgroup per set and row), each an exact recompression of the
 * projected product (no further truncation).
 *   Jh, Jv, h: host arrays of n device pointers (fp64, layouts of
 *     tn_build_env on this context's lattice); h may be NULL, as may its
 *     entries (zero field)
 *   beta (host, fp64 [n]); logZ_out (host, fp64 [n]) receives the values
 * The context keeps one environment stack per set between calls (about
 * Ly * Lx * 2 D^2 doubles each).  Errors: TN_ESTATE without an environment
 * built by tn_build_env with successive SVD (tn_set_env and fitted builds
 * have no recorded cuts) or while capturing; TN_EINVAL for n < 1, NULL
 * arrays or a non-finite beta; TN_ENONPOS if a value is not positive.
 * Synchronises the stream. */
int tn_logz_frozen(tn_ctx *ctx, int n, const double *const *Jh, const double *const *Jv,
                   const double *const *h, const double *beta, double *logZ_out);

/* Two-sided estimate of d ln Z / dJ and d ln Z / d beta, i.e. of beta times
 * the bond correlations and of minus the mean energy (Sec. 4 compares energies
 * from derivatives of the approximate contraction with sampled ones).  Every
 * site's environment is the exact contraction of its row between the
 * top-down boundary MPS of the rows above and the stored bottom-up
 * environment of the rows below (App. A's recursion run from both sides),
 * divided by that row's value.  Exact without truncation; with truncation it
 * is not the derivative of ln Z~ (tn_grad is) but tracks the exact
 * derivative far more closely on frustrated lattices.  The top-down boundary
 * is the environment build of the upside-down lattice, made on the first call
 * after a tn_build_env / tn_set_env and kept with the context.
 *   dJh (dev, fp64 [Ly][Lx-1]), dJv (dev, fp64 [Ly-1][Lx]), dbeta (host, may
 *   be NULL), as in tn_grad.  Errors: TN_ESTATE without an environment or
 *   while capturing; TN_EINVAL for beta*J = 0.  Synchronises the stream. */
int tn_grad_two_sided(tn_ctx *ctx, double *dJh, double *dJv, double *dbeta);

/* ---- Launch-shape autotuning --------------------------------------------
 * The batched sampler has launch variants that draw bitwise the same
 * proposals and differ only in how they are packed onto the GPU (for D <= 32:
 * two or one sets of 16 proposals per wavefront, two or three wavefronts per
 * SIMD).  These calls time the candidates on the context's own instance with
 * HIP events and keep the fastest time per proposal (a candidate must beat an
 * earlier one by 1% to replace it).  Timing launches use internal buffers and
 * leave the caller's buffers, the counters of tn_stats and the random streams
 * as they were.
 * cache_path (host string, may be NULL): JSON file of earlier choices, one
 * member per line keyed by device architecture and problem; a key found there
 * is used without timing, a new choice is added and the file rewritten
 * through a temporary file renamed over it.  Both calls synchronise the
 * stream and are refused while capturing (TN_ESTATE). */

/* Tune this context's instance for tn_mh_run with `chains` chains and runs
 * of max_steps MH steps: every variant and every count m of MH steps per
 * sampler launch among 1, 2, 4, ..., max_steps (capped at 64 and by a
 * quarter of the free device memory), ranked by the time of max_steps steps
 * drawn in launches of m steps and one launch of the remainder (so a count
 * that leaves a small, poorly filled last launch can lose to one that does
 * not).  The
 * choice applies to tn_sample, tn_sample_steps, tn_eval_logq, tn_mh_step and
 * tn_mh_run while the lattice size, the bond dimension rounded up to 16 and
 * the precision stay those tuned (a new build with other couplings keeps it);
 * tn_mh_run then draws about the tuned number of proposals per launch.
 *   variant_out, steps_out (host, may be NULL): the chosen variant and steps
 *   per launch.  Errors: TN_ESTATE without an environment, TN_EINVAL for
 *   chains < 1 or max_steps < 1, TN_ENOMEM, TN_EHIP; the cache file cannot be
 *   written: TN_EINVAL.  An FP64 context tunes the steps per launch only. */
int tn_autotune(tn_ctx *ctx, int chains, int max_steps, const char *cache_path, int *variant_out,
                int *steps_out);

/* Tune the sampler launch of every group of tn_mh_step_multi (instances of
 * one bond class and precision share a launch) for the instances and chain
 * counts of the last tn_build_env_multi; later tn_mh_step_multi calls use the
 * choices.  variants_out (host, int [8], may be NULL): entry
 * 4 * bf16 + NT - 1 gets the variant of group (bf16, NT = D rounded up to 16,
 * divided by 16), -1 where there is no such group.  TN_ESTATE before
 * tn_build_env_multi; TN_EINVAL for a TN_FP64_MFMA instance, as in
 * tn_mh_step_multi. */
int tn_autotune_multi(tn_ctx *ctx, const char *cache_path, int *variants_out);

/* ---- Periodic boundaries by frozen lines ---------------------------------
 * Section "Arbitrary boundary conditions": a lattice whose opposite edges are
 * identified (a cylinder along x or y, or a torus) is sampled by keeping one
 * line of spins fixed during a TNMH step; the frozen spins act on their free
 * neighbours as fields and the free spins form an open lattice, sampled and
 * accepted as before.  Every chain gets its own open model (its frozen spins
 * differ), so a step builds one environment stack per chain, in one batched
 * build, and draws one proposal per chain.
 *
 * Geometry.  Ly x Lx sites, wrapped along x (wrap_x != 0) and/or y.  A wrapped
 * direction has at least 3 sites.  Jh[r][c] couples (r,c)-(r,(c+1) mod Lx):
 * [Ly][Lx] when wrapped along x, [Ly][Lx-1] otherwise; Jv[r][c] couples
 * (r,c)-((r+1) mod Ly,c): [Ly][Lx] when wrapped along y, [Ly-1][Lx] otherwise;
 * h [Ly][Lx] or NULL.  The energy is Eq. (ising) over every bond.
 *
 * Cut.  A step freezes column cut_col (if wrapped along x) and row cut_row (if
 * wrapped along y).  The open lattice is (Ly - wrap_y) x (Lx - wrap_x); its site
 * (r', c') is ((cut_row + 1 + r') mod Ly, (cut_col + 1 + c') mod Lx) in a
 * wrapped direction and (r', c') otherwise.  A free site next to the frozen
 * line gets the field J s_frozen of that bond, added to its own field in the
 * order left, right, up, down.  The acceptance of Eq. (mh-acc) uses the open
 * model's ln q and energies (they differ from the periodic energies by a term
 * of the frozen spins alone).  The caller chooses the cuts: any sequence
 * chosen independently of the states keeps the periodic Boltzmann law; on a
 * torus two fixed crosses leave the two sites where the row of one meets the
 * column of the other frozen for good, so cycle through three or more.
 *
 * Random numbers.  Chain j of instance m draws its proposal with id j and
 * instance m at step `step`, and its acceptance from counter
 * (0, j, step, m << 2 | 1), as chain j of instance m of tn_mh_step_multi. */
typedef struct {
    const double *Jh, *Jv, *h;   /* (dev, fp64) couplings and field (h may be NULL) */
    double beta;
    int chains;                  /* chains of this instance (>= 0) */
} tn_periodic_instance;

/* Set up n instances of one periodic lattice shape for tn_periodic_step.  The
 * couplings are copied; the context allocates the open models, environment
 * stacks and sampler buffers of every chain.  D (1..64) and prec (TN_FP64,
 * TN_FP32, TN_BF16) as in tn_build_env.  Errors: TN_EINVAL for bad shapes
 * (Lx, Ly >= 1, a wrapped direction >= 3 sites, open lattice at most 256
 * columns, at most 65536 sites, at least one chain), TN_ENOMEM.  Replaces an
 * earlier periodic set-up; independent of tn_build_env's instance.
 * Synchronises the stream. */
int tn_periodic_setup(tn_ctx *ctx, int Lx, int Ly, int wrap_x, int wrap_y, int D, int prec, int n,
                      const tn_periodic_instance *inst);

/* One TNMH step of every chain with the given cut.
 *   spins (dev, int8 [total chains][Ly][Lx], instance 0's chains first):
 *     updated in place (the frozen lines never change).
 *   energy (dev, fp64 [total chains]): periodic energies after the step.
 *   accepted (dev, uint8 [total chains]): 1 where the proposal was taken.
 *   cut_row, cut_col: in 0..Ly-1 / 0..Lx-1 for a wrapped direction, ignored
 *   otherwise.
 * Errors: TN_ESTATE before tn_periodic_setup or while capturing; TN_EINVAL
 * for NULL buffers or a cut out of range; TN_ENONPOS / TN_ENOCONV if a chain's
 * environment build fails (its step is not taken).  Synchronises the stream
 * (each step checks its builds). */
int tn_periodic_step(tn_ctx *ctx, uint64_t seed, uint64_t step, int cut_row, int cut_col, int8_t *spins,
                     double *energy, uint8_t *accepted);

/* nsweeps checkerboard single-spin-flip Metropolis sweeps of every chain on
 * the periodic lattice (Sec. 3 interleaves such sweeps with TNMH steps), in
 * place, then the periodic energies into energy (dev, fp64 [total chains]).
 * Site order r + c even first; local field h + left + right + up + down with
 * the wrapping neighbours, in that order; flip iff u < exp(-(beta 2 s F)),
 * u = word i % 4 of Philox4x32-10 at counter (sweep * 2^14 + i / 4, chain j,
 * step, instance m << 2 | 2).  Flips are counted in tn_stats.  Errors:
 * TN_ESTATE before tn_periodic_setup; TN_EINVAL for an odd length along a
 * wrapped direction (same-colour sites would share a bond) or nsweeps
 * outside 0..2^18-1. */
int tn_periodic_sweeps(tn_ctx *ctx, int nsweeps, uint64_t seed, uint64_t step, int8_t *spins, double *energy);

/* Periodic energies of given states (dev, int8 [total chains][Ly][Lx]) into
 * energy (dev, fp64 [total chains]).  TN_ESTATE before tn_periodic_setup. */
int tn_periodic_energy(tn_ctx *ctx, const int8_t *spins, double *energy);

/* Link overlap over every bond of the periodic lattice, sum of
 * a_i a_j b_i b_j, of n configuration pairs (dev, int8 [n][Ly][Lx]) into
 * q (dev, int32 [n]); the periodic counterpart of tn_link_overlap for
 * Eq. (Delta).  TN_ESTATE before tn_periodic_setup. */
int tn_periodic_link_overlap(tn_ctx *ctx, int n, const int8_t *a, const int8_t *b, int32_t *q);

typedef struct {
    uint64_t clamps;        /* conditional weights clamped (FP64: negative, to 0; FP32/BF16: below the floor) */
    uint64_t both_nonpos;   /* sites drawn with p+ = 1/2 */
    uint64_t near_threshold;/* draws with |u - p+| < 1e-6 */
    uint64_t accepted;      /* accepted MH moves since the last reset */
    uint64_t proposed;      /* MH proposals since the last reset */
    uint64_t degenerate_cuts;/* cuts (successive SVD and two-site fit) with s_chi-1 - s_chi < 1e-12 s_0 */
    double   logZ;          /* ln Z~ of the current environment */
    double   env_build_ms;  /* wall time of the last tn_build_env */
    uint64_t metropolis_flips; /* spins flipped by tn_metropolis_sweeps */
} tn_stats_t;

/* Counters of the sampler and the chains: how often the positivity of the
 * approximate weights failed (App. A remark that Z~ must stay positive for the
 * chain to be irreducible), the acceptance of Algorithm 1 (accepted /
 * proposed), the near-threshold draws and degenerate cuts that the parity
 * tests count.  One struct instead of one out-pointer per counter, so that
 * counters can be added without changing the signature; the three counters
 * asked of a minimal interface map as neg_weight_clamps = clamps,
 * both_nonpos = both_nonpos, accept_rate = accepted / proposed.
 * out (host) receives the values; reset != 0 clears the device counters.
 * Errors: TN_EINVAL for NULL arguments, TN_ESTATE while capturing.
 * Synchronises the stream. */
int tn_stats(tn_ctx *ctx, tn_stats_t *out, int reset);

/* Peak probes.  The rooflines of the kernels are quoted against MI355X's
 * published peaks; these probes measure what the chip attains for each unit
 * the kernels use, each unit alone at its highest rate, so that a kernel can
 * also be read against what is reachable (the attained rate includes the
 * clock the chip holds under that load).  Not part of the sampling path.
 *   TN_PEAK_MFMA_F32   v_mfma_f32_16x16x4_f32, eight independent chains per
 *                      wave, four waves per SIMD; amount = iterations
 *   TN_PEAK_MFMA_BF16  v_mfma_f32_16x16x32_bf16, as above
 *   TN_PEAK_MFMA_F64   v_mfma_f64_16x16x4_f64, four chains per wave
 *   TN_PEAK_FMA_F64    v_fma_f64 on every lane, sixteen chains; amount =
 *                      iterations
 *   TN_PEAK_HBM_READ   stream read of a buffer of `amount` bytes (16-byte
 *                      loads, eight in flight per lane)
 *   TN_PEAK_HBM_COPY   copy between two buffers of `amount` bytes each
 * One untimed launch, then one launch timed with HIP events on the null
 * stream of the current device.  Out (host): *seconds of the timed launch,
 * *work its flops (compute probes) or bytes moved, read plus written (memory
 * probes).  The buffers are allocated and freed by the call.  Errors:
 * TN_EINVAL for an unknown kind, amount < 1, compute amount above 2^30,
 * memory amount not a multiple of 16 or above 64 GiB, or NULL outputs;
 * TN_ENOMEM if the buffers cannot be allocated; TN_EHIP for a failed launch.
 * Synchronises the device. */
enum tn_peak_kind {
    TN_PEAK_MFMA_F32 = 0,
    TN_PEAK_MFMA_BF16 = 1,
    TN_PEAK_MFMA_F64 = 2,
    TN_PEAK_FMA_F64 = 3,
    TN_PEAK_HBM_READ = 4,
    TN_PEAK_HBM_COPY = 5
};
int tn_peak_probe(int kind, long long amount, double *seconds, double *work);

#ifdef __cplusplus
}
#endif

#endif /* TNMH_H */
