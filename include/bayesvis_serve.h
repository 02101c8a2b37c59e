/*
 * bayesvis_serve.h -- C ABI of the continuous-batching HMC server built on
 * the bayesvis evaluation path (include bayesvis.h first).
 */
#ifndef BAYESVIS_SERVE_H
#define BAYESVIS_SERVE_H

#include "bayesvis.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------ mass matrices --
 * Set-up of a chain's mass matrix (Sec. 4.2: the sampler is preconditioned
 * with an approximation of the Hessian of -log posterior; App. B: only the
 * Cholesky factor of a dense mass is needed).  The likelihood part is the
 * Gauss-Newton Hessian of U = chi^2 / 2, J^T J / sigma_n^2, with J the
 * Jacobian of the real and imaginary parts of the model visibilities of
 * vis_forward at (alm, gains, fwhm); the prior adds 1 / C for each sky
 * coefficient (alm_prior_var C, may be NULL for none), 2 / s_g^2 for each real
 * gain component (gain_prior_sigma s_g, 0 for none) and nothing for the flat F.
 * All pointers are device pointers in the layouts of bayesvis.h; `work` is
 * device scratch of at least hmc_mass_work_bytes(field) bytes owned by the
 * caller (not kept between calls).  The field's evaluation scratch is used,
 * so the calls are ordered with the field's other evaluations on `stream`.
 * Nothing is synchronised.  VIS_EINVAL: null pointers, sigma_n not positive
 * and finite, gain_prior_sigma negative; VIS_ENOMEM: work too small.       */
vis_status hmc_mass_work_bytes(const vis_field* field, size_t* bytes);

/* hmc_mass_diag: the diagonal h of the Gauss-Newton Hessian plus the prior
 * precision, and minv = 1 / h, both device float arrays in the server's
 * parameter layout (hmc_chain_init; padding entries get h = minv = 1); either
 * output may be NULL.  Sky coefficients and F take the Hutchinson estimate
 * mean_k (J^T z_k)^2 / sigma_n^2 over n_probes (1 .. 4096) complex probes
 * z_k with unit normal real and imaginary parts: probe k of visibility v
 * (row-major [n_time][n_freq][n_bl]) takes normals 2v, 2v + 1 of the Philox
 * stream with counter (v / 2, k, 0, 5) and key = seed (Box-Muller as for the
 * momenta); J^T z_k is the vis_adjoint pass with cotangent z_k.  The gains
 * take the exact diagonal: for both real components of g_a(nu),
 * sum over baselines (a, b) and times of |g_b|^2 |V_ab|^2 / sigma_n^2, V the
 * visibility without gains.  Accumulated in FP64.                          */
vis_status hmc_mass_diag(const vis_field* field, const float* alm, const vis_c64* gains,
                         const float* fwhm, float sigma_n, const float* alm_prior_var,
                         float gain_prior_sigma, int32_t n_probes, uint64_t seed, float* hdiag,
                         float* minv, void* work, size_t work_bytes, void* stream);

/* hmc_gain_mass_blocks: per channel nu the dense Gauss-Newton block of the
 * gains (components in layout order Re g_0, Im g_0, Re g_1, ...) plus
 * 2 / s_g^2 I, M_nu = H_nu + 2 / s_g^2 I, and its lower Cholesky factor
 * M_nu = L_nu L_nu^T, written to chol [n_freq][2 n_ant][2 n_ant] (float,
 * row-major, zero above the diagonal) as hmc_chain_init.gain_chol expects.
 * For baseline (i, j) and w = g_i g_j sum_t |V_ij|^2 / sigma_n^2:
 * H[Re g_i][Re g_j] = Re w, H[Im g_i][Im g_j] = -Re w,
 * H[Re g_i][Im g_j] = H[Im g_i][Re g_j] = Im w (symmetric), the diagonal as in
 * hmc_mass_diag.  Assembled and factored in FP64 on the device, one workgroup
 * per channel; a non-positive pivot (only with gain_prior_sigma = 0 and a
 * degenerate field, or non-finite inputs) leaves NaN in that channel's factor,
 * which hmc_chain_admit then refuses.  VIS_EINVAL also: 2 n_ant > 256.       */
vis_status hmc_gain_mass_blocks(const vis_field* field, const float* alm, const vis_c64* gains,
                                const float* fwhm, float sigma_n, float gain_prior_sigma,
                                float* chol, void* work, size_t work_bytes, void* stream);

/* ------------------------------------------------------------- serving --
 * Continuous-batching HMC server (Sec. 4.2, App. B with a diagonal mass
 * matrix, optionally with dense per-channel gain blocks; fixed-length
 * trajectories or the No-U-Turn sampler).  Each chain owns a field, data, a parameter vector q =
 * [a (n_freq*n_modes), gains as (Re, Im) pairs (n_freq*n_ant*2), F] and an
 * inverse mass diagonal of the same length, all resident in the server's
 * arena.  The potential is U = chi^2/2 + sum a^2 / (2 C) + sum |g - 1|^2 /
 * (2 s_g^2 / 2) (Gaussian priors; flat in F).  A trajectory draws
 * p = z / sqrt(minv), z from Philox-4x32-10 (key = seed, counter =
 * (block, trajectory, chain stream, 0)) with Box-Muller, takes n_leapfrog
 * steps and accepts with probability min(1, exp(H0 - H1)) (uniform from
 * counter (0xFFFFFFFF, trajectory, stream, 1)).  Each leapfrog step is one
 * chi^2 + gradient request; a worker thread batches the pending requests of
 * all chains into one sequence of batched kernel launches per tick (the
 * evaluations too, with batched = 1), and
 * admits new chains while others are in flight when the arena has room.
 * If adapt_step is set, after each trajectory eps <- eps / 1.2 when the
 * acceptance probability is below 0.2, else eps <- min(eps0, 1.2 eps)
 * (App. B, step-size adaptation).
 * Parameter layout (float): a at [0, n_freq*n_modes), zero padding up to
 * g_off = round_up(n_freq*n_modes, 64), gains as (Re, Im) pairs at
 * [g_off, g_off + 2*n_freq*n_ant), F last; length g_off + 2*n_freq*n_ant + 1.
 * The padding is ignored (its minv may be anything).  Each chain needs its
 * own field (the field holds the evaluation scratch).  A trajectory whose
 * final energy is non-finite (a divergence) is rejected like any other.  A
 * chain whose potential at its own position is non-finite reports
 * VIS_ENUMERIC once and stops; other chains are unaffected.  The server owns `stream` while it exists; it allocates only
 * host objects (a worker thread, events, pinned staging for tick tables).  */
typedef struct hmc_server hmc_server;

typedef struct {
  int32_t max_chains;          /* request-table capacity, >= 1 */
  int32_t max_batch;           /* requests per tick, >= 1 */
  int32_t batched;             /* 1: batched launches: every kernel of the evaluation
                                  sequence runs as one grid over all chains of the tick
                                  (chains with the same kernel sequence share each grid;
                                  such groups run concurrently on streams of their own);
                                  each chain's workgroups compute exactly what its own
                                  launch would;
                                  2: each chain's sequence is launched on its own, the
                                  chains spread over several streams;
                                  0: one chain after another on the server stream */
  int32_t inflight_ticks;       /* ticks queued on the device at once: 0 or 1 = one (the host
                                  builds the next tick after the current one completes),
                                  2 = two (the next tick is built and queued while the
                                  current one runs).  Two hide the host's tick work but
                                  double each request's latency and make NUTS chains run a
                                  no-op step after each trajectory; at ticks of milliseconds
                                  and more one is as fast. */
} hmc_server_config;

typedef struct {
  const vis_field* field;      /* must outlive the chain */
  const vis_c64* data;         /* device [n_time][n_freq][n_bl], read during the chain's life */
  float sigma_n;
  const float* q0;             /* device, initial position (copied into the arena) */
  const float* minv;           /* device, inverse mass diagonal (copied) */
  const float* alm_prior_var;  /* device [n_freq][n_modes] prior variance C (copied) */
  float gain_prior_sigma;      /* s_g: gains ~ 1 + s_g CN(0, 1) */
  float eps;                   /* leapfrog step size */
  int32_t n_leapfrog;          /* steps per trajectory, >= 1 */
  int32_t adapt_step;
  uint64_t seed;               /* Philox key */
  uint32_t stream_id;          /* Philox counter word 2 (distinct per chain) */
  /* Dense gain mass (App. B), or NULL for the diagonal minv everywhere.
   * Device [n_freq][2 n_ant][2 n_ant] float, row-major: for each channel f
   * the lower-triangular Cholesky factor L_f of the mass block M_f = L_f L_f^T
   * over that channel's gain components in layout order (Re g_0, Im g_0,
   * Re g_1, ...).  Only the lower triangle is read (copied into the arena at
   * admission); the diagonal must be positive and every entry finite, else
   * admission fails with VIS_EINVAL.  minv is then ignored on the gains; the
   * sky coefficients and F keep their diagonal masses.  With M_f dense the
   * server computes K = z^T z / 2 with L z = p (forward substitution), the
   * drift eps L^-T z (backward substitution) and momenta p = L z0, where z0
   * takes the normals a diagonal mass would use for the same elements; the
   * inverse of M_f is never formed.  2 n_ant <= 256.                       */
  const float* gain_chol;
  /* 0: fixed-length trajectories of n_leapfrog steps with a Metropolis test.
   * 1..10: the No-U-Turn sampler (Sec. 4.2; Hoffman & Gelman 2014) with at
   * most this many trajectory doublings (2^d - 1 leapfrog steps; n_leapfrog
   * is then ignored).  Doubling j grows 2^j steps in the direction given by
   * bit 0 of Philox counter (j, trajectory, stream, 2) (+1 if set); inside a
   * subtree the candidate is drawn multinomially (leaf replaces it with
   * probability w / sum w, w = exp(H0 - H), uniform from counter (s,
   * trajectory, stream, 3), s = the step index); a completed subtree's
   * candidate becomes the proposal with probability min(1, W_sub / W)
   * (biased progressive sampling, Betancourt 2017; counter (j, trajectory,
   * stream, 4)).  A span with end momenta p_a, p_b and momentum sum r turns
   * when (M^-1 p_a).(r - (p_a+p_b)/2) <= 0 or (M^-1 p_b).(...) <= 0; every
   * aligned power-of-two span inside a subtree and the whole trajectory after
   * each doubling are checked; a turn inside a subtree, or a leaf with
   * H - H0 > 1000 or non-finite, discards that subtree and ends the
   * trajectory.  The chain moves to the proposal (hmc_result.accepted = 1 if
   * it differs from the start).  Step-size adaptation uses the mean over the
   * leaves of min(1, exp(H0 - H)).  With gain_chol the velocities M^-1 p of
   * the checks come from the same triangular solves as the drift.          */
  int32_t nuts_max_depth;
} hmc_chain_init;

typedef struct {
  int32_t chain;
  int32_t trajectory;          /* 0-based trajectory index of this chain */
  int32_t accepted;
  int32_t status;              /* VIS_OK, VIS_ENUMERIC (non-finite H) or VIS_EDEVICE (a NUTS
                                  trajectory overran its step bound: an internal error) */
  double h0, h1;               /* Hamiltonian before / after (FP64) */
  double chi2;                 /* chi^2 at the chain's position after the transition */
  float eps;                   /* step size used */
  int32_t n_grad;              /* gradient evaluations in this trajectory */
  uint64_t t_submit_ns, t_done_ns;   /* host steady-clock timestamps */
  int32_t tree_depth;          /* NUTS: doublings begun (0 for fixed-length HMC) */
  float accept_stat;           /* Metropolis probability, or the NUTS mean of min(1, exp(H0 - H)) */
} hmc_result;

typedef struct {
  int64_t requests;            /* chi^2 + gradient requests completed */
  double p10_ms, p50_ms, p90_ms, p99_ms, max_ms; /* request latency: tick enqueue -> result
                                                   visible to the host; nearest-rank percentiles */
  int64_t arena_free_bytes;
  int32_t live_chains;
} hmc_stats;

/* Arena bytes one chain of this field occupies (its state vectors, prior
 * variances, reduction partials); admission succeeds when a free block of
 * this size exists.  The field workspace and the data are the caller's.    */
size_t hmc_chain_footprint_bytes(const vis_field* field);
/* The same for a chain admitted with gain_chol (adds two padded copies of the
 * factors: about 8 n_freq (2 n_ant)^2 bytes).                              */
size_t hmc_chain_footprint_dense_gain_bytes(const vis_field* field);
/* The same for a NUTS chain (adds the trajectory ends, candidate, proposal,
 * momentum sums and 20 checkpoint vectors: 32 vectors of the parameter length),
 * and for a NUTS chain with gain_chol (also 13 velocity vectors).          */
size_t hmc_chain_footprint_nuts_bytes(const vis_field* field);
size_t hmc_chain_footprint_nuts_dense_gain_bytes(const vis_field* field);
vis_status hmc_server_create(const hmc_server_config* cfg, void* arena_dev, size_t arena_bytes,
                             void* stream, hmc_server** out);
/* VIS_EAGAIN: the arena has no room for this chain now (retry after a release). */
vis_status hmc_chain_admit(hmc_server* s, const hmc_chain_init* init, int32_t* chain_id);
vis_status hmc_submit(hmc_server* s, int32_t chain_id, int32_t n_trajectories);
/* Copies up to max finished trajectories; waits up to timeout_ms (0 = no wait). */
vis_status hmc_poll(hmc_server* s, hmc_result* out, int32_t max, int32_t* n_out,
                    int32_t timeout_ms);
/* Copies the chain's current position (device pointer q_out, length of q).
 * VIS_EAGAIN while trajectories are queued or running; a tick that is still
 * in flight for the chain after its last result (a NUTS step scheduled before
 * the host saw the end of the trajectory) is waited for, up to 30 s.      */
vis_status hmc_chain_position(hmc_server* s, int32_t chain_id, float* q_out, void* stream);
vis_status hmc_chain_release(hmc_server* s, int32_t chain_id);
/* Request-latency percentiles since creation or the last reset.            */
vis_status hmc_server_stats(hmc_server* s, hmc_stats* out, int32_t reset);
/* Stops the worker after the ticks in flight complete; frees the handle.  */
vis_status hmc_server_destroy(hmc_server* s);

#ifdef __cplusplus
}
#endif
#endif /* BAYESVIS_SERVE_H */
