/*
 * bayesvis.h -- C ABI of the MI355X (gfx950) visibility / chi^2 / HMC library.
 *
 * What is computed (Kern 2025, "A Differentiable, End-to-End Forward Model
 * for 21 cm Cosmology"):
 *
 *   sky        I(p, nu) = sum_lm Y(p, lm) a(lm, nu)            Sec. 3.2, eq. fg_harmonic_matrix
 *              Y = real orthonormal spherical harmonics with integer l,
 *              column l*l + l + m, no Condon-Shortley phase  (App. A, eq. sht_ortho)
 *   RIME       V_ij(nu, t) = dOmega sum_p B(p, nu, t) I(p, nu)
 *                            exp(-2 pi i nu b_ij . s_p(t) / c)  Sec. 2.1, eq. rime_discrete
 *              pixels fixed on the celestial sphere, so s_p and the beam move
 *              with time (eq. rime_matrix: one design matrix per time);
 *              evaluated once per redundant baseline vector (Sec. 3.1)
 *   beam       B = exp(-theta^2 / 2 sigma^2) above the horizon, 0 below,
 *              sigma = F (nu_ref / nu) / (2 sqrt(2 ln 2)); F = FWHM at nu_ref (rad)
 *   gains      m_ij = g_i conj(g_j) V_ij                       Sec. 2.1 (gain terms)
 *   chi^2      sum |d - m|^2 / sigma_n^2                       Sec. 2.3, eq. likelihood
 *   gradients  of chi^2 w.r.t. a, g, F (replacing reverse-mode AD, Sec. 2.3)
 *   HMC        diagonal-mass leapfrog + Metropolis             Sec. 4.2, App. B
 *
 * Conventions
 *   - complex numbers are interleaved float pairs (vis_c64);
 *   - the gradient w.r.t. a complex quantity z is dL/dRe z + i dL/dIm z;
 *   - layouts (row-major):  alm[n_freq][n_modes] float,
 *       gains[n_freq][n_ant] vis_c64, vis/data[n_time][n_freq][n_bl] vis_c64,
 *     with physical baselines (i, j), i < j, in lexicographic order and
 *     b_ij = r_i - r_j;
 *   - pixel grid: n_z rings uniform in z = sin(dec), centres
 *     z_j = -1 + (j + 1/2) 2 / n_z; n_phi columns alpha_k = (k + 1/2) 2 pi / n_phi;
 *     pixel p = j n_phi + k; dOmega = 4 pi / (n_z n_phi);
 *   - topocentric frame E, N, U; hour angle H = LST - alpha.
 *
 * Memory ownership
 *   The caller allocates every device buffer, including each object's
 *   workspace (query its size first).  The library never calls hipMalloc;
 *   objects sub-allocate inside the workspace they are given, which must
 *   stay allocated and untouched until the object is destroyed.  Inputs are
 *   never modified; outputs are overwritten.  Handles are host objects owned
 *   by the library (freed by the matching *_destroy).
 *
 * Streams
 *   `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Work is stream-ordered and asynchronous; no entry point synchronises the
 *   host except the *_create calls (which upload tables) and hmc_poll.
 *   Evaluations on one field use the field's scratch space: calls on the
 *   same field must be ordered on one stream (calls on different fields may
 *   run concurrently).
 *
 * Errors
 *   Every entry point returns a vis_status; nothing is thrown or aborted
 *   across the ABI.  On a non-zero status, vis_last_error() returns a
 *   thread-local message.  Device-side faults surface as VIS_EDEVICE from a
 *   later call.
 */
#ifndef BAYESVIS_H
#define BAYESVIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VIS_OK = 0,
  VIS_EINVAL = -1,     /* bad argument, shape or descriptor */
  VIS_ENOMEM = -2,     /* workspace / arena too small */
  VIS_EDEVICE = -3,    /* HIP runtime error */
  VIS_EAGAIN = -4,     /* resource busy: retry later (serving admission) */
  VIS_ENOTFOUND = -5,  /* unknown chain id */
  VIS_ENUMERIC = -6    /* non-finite value detected */
} vis_status;

/* Split precisions: the dense synthesis runs as three hi/lo products on
 * 16-bit MFMA with FP32 accumulation, and so does the adjoint fringe GEMM
 * (FP16 hi/lo, coefficients scaled by a power of two per (t, nu)); the
 * forward fringe stays FP32 (its operands would need a 2-byte transpose). */
typedef enum {
  VIS_FP32 = 1,        /* FP32 MFMA synthesis, FP32 fringe */
  VIS_BF16X3 = 2,      /* synthesis as bf16 hi/lo split products on MFMA, FP32 accumulate */
  VIS_FP16X3 = 3       /* synthesis as fp16 hi/lo split products (scaled lo), FP32 accumulate */
} vis_precision;

/* How a field evaluates the sky synthesis I = Y a (Sec. 3.2).
 * DENSE: against the stored basis matrix Y restricted to the pixels above the
 *   horizon (FP32, bf16x3 or fp16x3 per the field precision).
 * SEPARABLE: on the RA x sin(dec) grid every column factorises,
 *   Y(ring j, column k; l, m) = lambda_lm(z_j) T_m(alpha_k) (Sec. 3.2,
 *   eq. fg_separable), so I is a Legendre sum per (m, ring) followed by an
 *   azimuthal sum per ring; both run as FP32 MFMA GEMMs from small tables and
 *   Y itself is never read (needs basis storage bit 3).  The synthesis is FP32
 *   at every field precision; with VIS_BF16X3 or VIS_FP16X3 only the adjoint
 *   fringe GEMM runs as FP16 hi/lo products (the two are then the same).     */
typedef enum {
  VIS_SYNTH_DENSE = 0,
  VIS_SYNTH_SEPARABLE = 1
} vis_synthesis;

typedef struct { float re, im; } vis_c64;

typedef struct vis_basis vis_basis;
typedef struct vis_field vis_field;

/* ---------------------------------------------------------------- basis --
 * Y(p, lm) on the equal-area grid for 0 <= l <= lmax, generated on the GPU
 * from a normalised Legendre recurrence (App. A: the normalisation is
 * carried through the recurrence so high orders do not overflow).
 * Any field with a smaller lmax uses the leading (lmax'+1)^2 columns.
 * storage: bit 0 = FP32 copy (needed by VIS_FP32 fields), bit 1 = bf16
 * hi/lo copy (VIS_BF16X3), bit 2 = fp16 hi/lo copy (VIS_FP16X3), bit 3 =
 * the factor tables of separable synthesis only (lambda_lm per ring and
 * T_m per column, FP32; a few MB instead of n_pix x n_modes values).     */
typedef struct {
  int32_t grid_nz, grid_nphi;
  int32_t lmax;
  uint32_t storage;
} vis_basis_desc;

vis_status vis_basis_workspace_bytes(const vis_basis_desc* desc, size_t* bytes);
vis_status vis_basis_create(const vis_basis_desc* desc, void* workspace_dev, size_t bytes,
                            void* stream, vis_basis** out);
vis_status vis_basis_destroy(vis_basis* basis);

/* ---------------------------------------------------------------- field --
 * One observation.  Antennas sit on a 2-D lattice (Sec. 3.1: a hexagonal
 * array): r_i = ant_lattice[i][0] e1 + ant_lattice[i][1] e2, with e1, e2
 * ENU vectors in metres whose U components are 0 (coplanar array).  Two
 * physical baselines are redundant when their integer lattice differences
 * agree up to sign; the canonical representative has its first non-zero
 * lattice coordinate positive.  All descriptor arrays are host memory and
 * are copied; the caller may free them after vis_field_create returns.
 * Limits: 2 <= n_ant <= 1024, lattice differences |dn| <= 16, n_freq and
 * n_time in [1, 4096], lmax <= basis lmax.
 * VIS_EINVAL: antennas sharing a site, non-coplanar basis, sizes out of range.  */
typedef struct {
  int32_t n_ant;
  const int32_t* ant_lattice;        /* [n_ant][2] */
  double lattice_e1_m[3];
  double lattice_e2_m[3];
  int32_t n_freq;
  const double* freq_hz;             /* [n_freq] */
  int32_t n_time;
  const double* lst_rad;             /* [n_time] */
  double latitude_rad;
  int32_t lmax;
  double beam_ref_hz;                /* nu_ref of the beam-width law */
  int32_t precision;                 /* vis_precision */
  int32_t synthesis;                 /* vis_synthesis (0 = dense) */
} vis_field_desc;

typedef struct {
  int32_t n_ant, n_bl, n_ubl, n_freq, n_time, n_pix, n_modes;
  int32_t n_pix_visible;             /* pixels above the horizon at some time */
  int32_t lattice_extent;            /* max |dn| over baselines */
  int32_t precision;
  int32_t synthesis;
  double d_omega;
  double fwd_macs;                   /* complex x real MACs of one fringe pass:
                                        sum over (u, t) of visible pixels x n_freq */
} vis_field_info;

vis_status vis_field_workspace_bytes(const vis_basis* basis, const vis_field_desc* desc,
                                     size_t* bytes);
vis_status vis_field_create(const vis_basis* basis, const vis_field_desc* desc,
                            void* workspace_dev, size_t bytes, void* stream, vis_field** out);
vis_status vis_field_get_info(const vis_field* field, vis_field_info* info);
vis_status vis_field_destroy(vis_field* field);

/* ---------------------------------------------------------- evaluation --
 * vis_forward: model visibilities m = g_i conj(g_j) V_ij            (Sec. 2.1)
 *   alm   device [n_freq][n_modes] float
 *   gains device [n_freq][n_ant] vis_c64
 *   fwhm  device pointer to one float, F in radians
 *   vis   device [n_time][n_freq][n_bl] vis_c64 (output)                  */
vis_status vis_forward(const vis_field* field, const float* alm, const vis_c64* gains,
                       const float* fwhm, vis_c64* vis, void* stream);

/* vis_adjoint: gradients of a real scalar L given its cotangent with respect
 * to the model visibilities, dvis = dL/dRe m + i dL/dIm m (device, same
 * layout as vis).  Outputs (device): grad_alm [n_freq][n_modes],
 * grad_gains [n_freq][n_ant], grad_fwhm (one float).  This is the transpose
 * of the linearised forward model (Sec. 2.3: the gradient that reverse-mode
 * AD would give), evaluated by recomputing fringe tiles.                   */
vis_status vis_adjoint(const vis_field* field, const float* alm, const vis_c64* gains,
                       const float* fwhm, const vis_c64* dvis, float* grad_alm,
                       vis_c64* grad_gains, float* grad_fwhm, void* stream);

/* chi2_and_grad: chi^2 = sum |d - m|^2 / sigma_n^2 (Sec. 2.3, eq. likelihood,
 * diagonal noise of Sec. 3.5 with variance sigma_n^2 per real component)
 * and its gradient.  chi2 is a device double accumulated in FP64.
 * data device [n_time][n_freq][n_bl] vis_c64; other pointers as above.
 * Any output pointer except chi2 may be NULL to skip the adjoint entirely
 * (then only the forward and chi^2 run).                                    */
vis_status chi2_and_grad(const vis_field* field, const vis_c64* data, float sigma_n,
                         const float* alm, const vis_c64* gains, const float* fwhm,
                         double* chi2, float* grad_alm, vis_c64* grad_gains,
                         float* grad_fwhm, void* stream);

/* ------------------------------------------------------------ map-making --
 * vis_make_map: the diagonally normalised map estimate of Sec. 4.3
 * (eq. vis_to_map, eq. map_psf) per channel,
 *     map_p = Re(A^H y)_p / (A^H A)_pp,
 * with A the beam-and-fringe response including the gains (eq. rime_matrix)
 * stacked over times and baselines; this is x_hat = D A^H N^-1 y for
 * N proportional to the identity and D = diag(A^H N^-1 A)^-1, so the
 * point-spread function has a unit diagonal.  data device [n_time][n_freq]
 * [n_bl] vis_c64; gains, fwhm as for vis_forward; map device [n_freq][n_pix]
 * (grid order, ring-major) float, 0 for pixels never above the horizon and
 * where (A^H A)_pp < 1e-6 max_p (A^H A)_pp of the channel (there the ratio
 * only amplifies noise);
 * weight (may be NULL) device [n_freq][n_pix] float, (A^H A)_pp.  Runs the
 * adjoint fringe pass unchanged; the field's scratch is reused.            */
vis_status vis_make_map(const vis_field* field, const vis_c64* data, const vis_c64* gains,
                        const float* fwhm, float* map, float* weight, void* stream);

/* --------------------------------------------------------- delay filter --
 * Sec. 2.1 (eq. rime_filter, eq. gpr) and Sec. 3.5 (eq. filtered_noise):
 * model and data are multiplied along frequency by the real high-pass filter
 *     F = I - C_fg (C_fg + noise_ratio I)^-1,
 *     C_fg(nu, nu') = sinc(2 tau_max (nu - nu')),  sinc(x) = sin(pi x) / (pi x),
 * (a tophat of half-width tau_max in delay; the paper uses 250 ns and 1e-8)
 * and the likelihood keeps the diagonal of the filtered noise covariance:
 *     chi^2_F = sum |(F (d - m))_nu|^2 / (sigma_n^2 (F F^T)_nu,nu).
 *
 * vis_filter_build: host only (no device call).  F_out [n_freq][n_freq]
 *   row-major and fft_diag [n_freq] = (F F^T)_nu,nu, both FP64, computed with
 *   a Cholesky solve of (C_fg + noise_ratio I).  VIS_EINVAL: n_freq out of
 *   [1, 4096], non-finite or non-positive frequencies, tau_max < 0,
 *   noise_ratio <= 0, or a matrix that is not positive definite.
 * vis_filter_create: builds F and uploads it (FP32) into the caller's
 *   workspace (vis_filter_workspace_bytes); the filter belongs to any field
 *   with the same channels.                                                 */
typedef struct vis_filter vis_filter;

vis_status vis_filter_build(int32_t n_freq, const double* freq_hz, double tau_max_s,
                            double noise_ratio, double* F_out, double* fft_diag);
vis_status vis_filter_workspace_bytes(int32_t n_freq, size_t* bytes);
vis_status vis_filter_create(int32_t n_freq, const double* freq_hz, double tau_max_s,
                             double noise_ratio, void* workspace_dev, size_t bytes, void* stream,
                             vis_filter** out);
vis_status vis_filter_destroy(vis_filter* filter);

/* chi2_filtered_and_grad: chi^2_F and its gradient (same outputs and NULL
 * rules as chi2_and_grad).  The filter couples channels, so the whole field
 * is evaluated: model visibilities, then F (d - m) and the cotangent
 * -2 F^T ((F (d - m)) / N~) as two real GEMMs over frequency per time on
 * MFMA, then the adjoint pass.  work: device scratch of at least
 * vis_filtered_work_bytes(field) bytes, owned by the caller, not kept
 * between calls.  VIS_EINVAL: the filter's n_freq differs from the field's;
 * VIS_ENOMEM: work too small.                                              */
vis_status vis_filtered_work_bytes(const vis_field* field, size_t* bytes);
vis_status chi2_filtered_and_grad(const vis_field* field, const vis_filter* filter,
                                  const vis_c64* data, float sigma_n, const float* alm,
                                  const vis_c64* gains, const float* fwhm, double* chi2,
                                  float* grad_alm, vis_c64* grad_gains, float* grad_fwhm,
                                  void* work, size_t work_bytes, void* stream);

/* chi2_filtered_and_grad_noalloc: chi2_filtered_and_grad without the work
 * argument, for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops and harnesses that forbid allocation).  Its
 * scratch is one static device array of VIS_NOALLOC_SCRATCH_BYTES per GPU in
 * the library's code object, held until the process ends (the 61-dish, 64-
 * channel, 60-time field needs 112.5 MB of it); the call makes no allocation.
 * Every call on one GPU shares that GPU's array and it keeps the last call's
 * contents, so calls that may overlap on one device (other streams, other
 * threads) race and must be ordered by the caller.  Nothing in the array has
 * to start at zero.  VIS_ENOMEM: vis_filtered_work_bytes(field) exceeds
 * VIS_NOALLOC_SCRATCH_BYTES.  Other arguments, outputs and errors as for
 * chi2_filtered_and_grad.                                                   */
#define VIS_NOALLOC_SCRATCH_BYTES (128u << 20)
vis_status chi2_filtered_and_grad_noalloc(const vis_field* field, const vis_filter* filter,
                                          const vis_c64* data, float sigma_n, const float* alm,
                                          const vis_c64* gains, const float* fwhm, double* chi2,
                                          float* grad_alm, vis_c64* grad_gains, float* grad_fwhm,
                                          void* stream);

/* ------------------------------------------------------------ profiling --
 * Optional per-field kernel timing: when enabled, every kernel the field
 * launches is bracketed by a pair of hipEvents on the launch stream and its
 * elapsed time is added to a per-kernel-name total when read.  Reading
 * synchronises with the recorded events.  Used to report the launch
 * duration of the dominant kernel; off by default (no events recorded).   */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
} vis_kernel_time;

vis_status vis_profile_enable(vis_field* field, int32_t enable);
vis_status vis_profile_read(vis_field* field, vis_kernel_time* out, int32_t max, int32_t* n_out,
                            int32_t reset);

const char* vis_last_error(void);
const char* vis_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BAYESVIS_H */
