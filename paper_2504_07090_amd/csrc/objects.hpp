// Internal layouts of the basis and field objects and the launchers that
// operate on them.  Not part of the C ABI.
#pragma once

#include <hip/hip_bf16.h>

#include <map>
#include <string>
#include <vector>

#include "common.hpp"

namespace bv {

// Per-field kernel timer: a pair of hipEvents around each launch while on.
struct Profiler {
  bool on = false;
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<long long, double>> totals;
  hipEvent_t get();
  void drain();   // waits for pending events and folds them into totals
  ~Profiler();
};

// Brackets one kernel launch when the field's profiler is on.
struct ProfScope {
  Profiler* p;
  const char* name;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(Profiler* p_, const char* n, hipStream_t s);
  ~ProfScope();
};

}  // namespace bv

struct vis_basis {
  int nz = 0, nphi = 0, lmax = 0;
  int n_pix = 0, n_modes = 0;
  int kpad = 0;                    // row stride of Y (modes rounded up to 64), zero-filled tail
  uint32_t storage = 0;
  float* y32 = nullptr;            // [n_pix][kpad] FP32
  __hip_bfloat16* ybh = nullptr;   // [n_pix][kpad] bf16 hi part
  __hip_bfloat16* ybl = nullptr;   // [n_pix][kpad] bf16 lo part (y - hi)
  _Float16* yhh = nullptr;         // [n_pix][kpad] fp16 hi part
  _Float16* yhl = nullptr;         // [n_pix][kpad] fp16 lo part, scaled by 2^11
  double* lam = nullptr;           // generator staging: normalised Legendre per ring
  double* trig = nullptr;          // generator staging: cos / sin (m alpha) per column
  // separable-synthesis factor tables (storage bit 3), FP32:
  //   sep_lam: per m >= 0 a block of nz rows of sep_lpad(m) = round_up(lmax - m + 1, 8)
  //   floats, row j holding lambda_lm(z_j) for l = m .. lmax then zeros; block m
  //   starts at sep_loff[m] (so both Legendre stages read consecutive l)
  //   sep_tt[c][k] = T_m(alpha_k) with c = m + lmax + kSepPad, zero for |m| > lmax; its
  //   rows hold nphi_b columns, zero beyond nphi
  int kaz_t = 0;                   // rows of sep_tt: round_up(2 lmax + 1 + 2 kSepPad, 4)
  int nphi_b = 0;                  // nphi rounded up to whole 32-column batches
  float* sep_lam = nullptr;
  int* sep_loff = nullptr;         // [lmax + 2] block offsets of sep_lam (floats)
  float* sep_tt = nullptr;
};

namespace bv {

// Per-evaluation scratch of one field (device).
struct FieldScratch {
  float* img = nullptr;            // [n_freq][nv_pad] sky at visible pixels
  float* apad = nullptr;           // [nf_pad][kpad] sky coefficients, zero-padded rows
  float* dimg = nullptr;           // [n_freq][nv_pad] dL/dI
  float* dsplit = nullptr;         // split fields: [nf_pad][nv_pad] floats holding the
                                   //   16-bit hi plane then the lo plane of dL/dI
  float* rscale = nullptr;         // split fields: [nf_pad] inverse row scales
  float* rmax = nullptr;           // split fields: [nf_pad][ceil(max(kpad, nv_pad) / 2048)]
  float* fscale = nullptr;         // split fields: [n_freq][kScaleParts] maxima of |I|, from
                                   //   which the forward fringe scales the weighted sky
  float* sep_g = nullptr;          // separable fields: [nz][kaz][n_freq] Legendre stage output
                                   //   (forward) or azimuthal stage output (adjoint)
  float* sep_dfull = nullptr;      // separable fields: [nz][n_freq][nphi_b] dL/dI on the full grid
                                   //   (zero at pixels never above the horizon and beyond nphi)
  float* sep_at = nullptr;         // separable fields: [n_modes][n_freq] sky coefficients transposed
  float2* vu = nullptr;            // [n_time][n_freq][n_ubl] gain-free unique visibilities
  float* gco = nullptr;            // [n_time][n_freq][gstride] adjoint coefficients, MFMA layout
  double* chi_part = nullptr;      // [n_time * n_freq]
  float2* g_part = nullptr;        // [n_time][n_freq][n_ant]
  float* f_part = nullptr;         // [n_freq * n_chunks]
  float* a_part = nullptr;         // split-K partials: [asplit][n_freq][kpad] of dL/da,
                                   // or [fsplit][n_freq][nv_pad] of the sky
};

// Immutable device tables of one field.
struct FieldTables {
  float* dnu = nullptr;            // [n_freq] nu_f - nu_c, Hz (nu_c: the field's reference frequency)
  float* sigr = nullptr;           // [n_freq] beam sigma per unit FWHM: (nu_ref / nu_f) / (2 sqrt(2 ln 2))
  int* vpix = nullptr;             // [nv_pad] pixel index of each visible slot
  int* vidx = nullptr;             // [n_pix] visible slot of each pixel or -1
  float2* q1 = nullptr;            // [n_time][nv_pad] (y, p) of lattice axis 1: p = (e1 . s) / c in
                                   //   seconds, y = nu_c p - rint(nu_c p) (cycles, formed in FP64)
  float2* q2 = nullptr;            // [n_time][nv_pad] the same for e2
  float* th2 = nullptr;            // [n_time][nv_pad] zenith angle^2, kBelowHorizon if U <= 0
  int2* chunk_t = nullptr;         // [n_chunks] first / last time the chunk is visible
  int* tchunk_off = nullptr;       // [n_time + 1] CSR of chunks active at each time
  int* tchunk = nullptr;           // [sum] chunk indices
  int2* bl_ant = nullptr;          // [n_bl] (i, j)
  int* bl_u = nullptr;             // [n_bl] unique index, negative-encoded sign: u or ~u
  int4* bl_pos = nullptr;          // [n_bl] position of baseline k in u_list, and of its
                                   //   (k, role 0) and (k, role 1) entries in a_list
  int* u_off = nullptr;            // [n_ubl + 1] CSR unique -> physical
  int* u_list = nullptr;           // [n_bl] (bl << 1) | (sign < 0)
  int* a_off = nullptr;            // [n_ant + 1] CSR antenna -> baselines
  int* a_list = nullptr;           // [2 n_bl] (bl << 1) | role (0: antenna is i, 1: is j)
  int2* ubl_nm = nullptr;          // [n_ubl] lattice (n1, n2), canonical
  int* ulut = nullptr;             // [(D+1) * (2D+1)] unique index of (n1, n2) or -1
  int4* cplan = nullptr;           // [gstride] source plan of each adjoint coefficient entry
  // separable fields: per ring j, the first columns of the 32-column batches
  // that hold a pixel above the horizon, sep_kb[sep_kb_off[j] .. sep_kb_off[j + 1])
  int* sep_kb_off = nullptr;       // [nz + 1]
  int* sep_kb = nullptr;           // [nz * ceil(nphi / 32)] at most
  int* sep_kb_ring = nullptr;      // the ring of each sep_kb entry
  int* sep_voff = nullptr;         // [nv_pad] offset of visible slot k's pixel in sep_dfull at
                                   //   channel 0: ring * n_freq * nphi_b + column
};

}  // namespace bv

struct vis_field {
  const vis_basis* basis = nullptr;
  int n_ant = 0, n_bl = 0, n_ubl = 0, n_freq = 0, n_time = 0;
  int n_modes = 0, lmax = 0;
  int nv = 0, nv_pad = 0, n_chunks = 0, n_tchunk = 0;
  int extent = 0;                  // D = max |n1|, |n2|
  int n_cu = 256;                  // compute units of the field's device
  int dtile = 0;                   // compile-time extent of the fringe kernels (>= extent)
  int gstride = 0;                 // floats per (t, nu) of the adjoint coefficient table
  int precision = VIS_FP32;
  int synthesis = VIS_SYNTH_DENSE;
  int kaz = 0;                     // separable: rows per ring of sep_g, round_up(2 lmax + 1, 4)
  int asplit = 1;                  // split-K factor of the adjoint synthesis
  int fsplit = 1;                  // split-K factor of the FP32 forward synthesis
  int sep_nkb = 0;                 // separable fields: entries of tab.sep_kb
  double d_omega = 0.0;
  double beam_ref_hz = 150e6;
  double fwd_macs = 0.0;
  bv::FieldTables tab;
  bv::FieldScratch scr;
  mutable bv::Profiler prof;
};

namespace bv {

// ---- launchers (stream-ordered, no host sync) ----------------------------
void launch_synth_fwd(const vis_field* f, const float* alm, float* img, hipStream_t st);
// Dense fields read dL/dI from dimg; separable fields take dimg == nullptr and
// read it from the full-grid scratch, where the adjoint fringe pass put it.
void launch_synth_adj(const vis_field* f, const float* dimg, float* grad_alm, hipStream_t st);
void launch_fringe_fwd(const vis_field* f, const float* img, const float* fwhm, float2* vu,
                       hipStream_t st);
// dL/dI goes to dimg ([n_freq][nv_pad]) or, for separable fields, with
// dimg == nullptr, to the full-grid scratch dfull ([n_pix][n_freq]).
void launch_fringe_adj(const vis_field* f, const float* img, const float* fwhm, const float* gco,
                       float* dimg, float* f_part, hipStream_t st, float* dfull = nullptr);

// Extent instantiated by the fringe kernels for a lattice extent D, and the
// layout of the adjoint coefficient table that the gains pass writes.
int fringe_tile_extent(int extent);
inline int fringe_tiles(int dtile) { return (2 * dtile + 15) / 16; }
// Channels that share one adjoint tile: for D = 4 two channels' coefficient
// matrices sit on the diagonal blocks of the 16 x 16 tile (the gains pass
// writes each channel's slice as usual; the kernel places them).
__host__ __device__ constexpr int adj_channels_per_tile(int D) { return D == 4 ? 2 : 1; }
// Extents whose 2 D coefficient rows leave a one-channel tile a free row
// (D = 2, 6, 12): the beta-axis coefficients omega(0, m) fill row 2 D, and the
// pixel operand's row 2 D of ones picks them up inside the tile product.
__host__ __device__ constexpr bool adj_axis_in_tile(int D) {
  return adj_channels_per_tile(D) == 1 && 2 * D < 16 * ((2 * D + 15) / 16);
}
// Split-precision fields run the fringe products as FP16 hi + lo pairs.
inline bool fringe_split(const vis_field* f) { return f->precision != VIS_FP32; }
inline int adj_coef_stride(int dtile, bool split) {
  const int rt = fringe_tiles(dtile);
  return static_cast<int>(round_up(rt * rt * (split ? 384 : 256) + 16 * rt + 4 * dtile + 1, 64));
}

// Delay-filtered likelihood: scratch carved from the caller's work buffer
// (model / cotangent visibilities, the weighted filtered residual, chi^2
// partials per wavefront), and the two GEMM passes over frequency.
struct FilteredWork {
  float2* m = nullptr;      // [n_time][n_freq][n_bl] model, then the cotangent
  float2* w = nullptr;      // [n_time][n_freq][n_bl] F (d - m) / N~
  double* part = nullptr;
  long nparts = 0;
  size_t bytes = 0;
};
FilteredWork carve_filtered_work(const vis_field* f, void* work, size_t bytes);
void launch_filter_chi2(const vis_field* f, const vis_filter* flt, const float2* data, float sigma_n,
                        const FilteredWork& w, double* chi2, hipStream_t st);
void launch_filter_cot(const vis_field* f, const vis_filter* flt, const FilteredWork& w, hipStream_t st);

// kGainMap: the adjoint pass's collapse of a given cotangent onto the unique
// baselines only (no gain gradient; the unique visibilities are not read).
enum GainMode { kGainFwd = 0, kGainChi2 = 1, kGainAdj = 2, kGainMap = 3 };
void launch_map_finish(const vis_field* f, const vis_c64* gains, const float* fwhm, float* map,
                       float* weight, hipStream_t st);
// Where each entry of a (t, nu) slice of adjoint coefficients comes from
// (the gains pass evaluates it from the slice's collapsed omega): see gains.hip.
std::vector<int4> coef_plan(const std::vector<int>& ulut, int extent, int dtile, bool split,
                            int gstride);
void launch_gains(const vis_field* f, GainMode mode, const float2* vu, const float2* gains,
                  const float2* data_or_dvis, float sigma_n, float2* vis_out, double* chi_part,
                  float* gco, float2* g_part, hipStream_t st);
void launch_reduce_grads(const vis_field* f, bool with_chi2, const double* chi_part,
                         double* chi2, const float2* g_part, float2* grad_gains,
                         const float* f_part, float* grad_fwhm, hipStream_t st);

// The evaluation sequences shared by the entry points: sky synthesis and the
// forward fringe pass into the field's scratch (img, vu); and, once the gains
// pass has written the adjoint coefficients and gain partials, the adjoint
// fringe pass, the gradient reductions and the adjoint synthesis.
void forward_core(const vis_field* f, const float* alm, const float* fwhm, hipStream_t s);
void adjoint_tail(const vis_field* f, const float* fwhm, float* grad_alm, float2* grad_gains,
                  float* grad_fwhm, bool with_chi2, double* chi2, hipStream_t s);

}  // namespace bv
