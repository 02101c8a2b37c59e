// Mass-matrix set-up for the HMC server: the Gauss-Newton diagonal of the
// potential and dense per-channel gain blocks with their Cholesky factors.
//
// Sec. 4.2: the sampler is preconditioned with a mass matrix that
// approximates the Hessian of -log posterior; App. B: only its Cholesky
// factor is needed.  Here the likelihood part of the Hessian is its
// Gauss-Newton form J^T J / sigma_n^2 (J the Jacobian of the real and
// imaginary parts of the model visibilities; U = chi^2 / 2 + prior), and the
// prior adds its own precision (1 / C on each sky coefficient, 2 / s_g^2 on
// each real gain component, nothing on the flat F).
//
// Diagonal.  Sky coefficients and F: the Hutchinson estimate
// mean_k (J^T z_k)^2, z_k complex probes with unit-variance real and
// imaginary parts (E[z z^T] = I), J^T z being the library's own adjoint pass
// with cotangent z.  Probe k of visibility v (row-major [t][nu][bl]) takes
// normals 2v and 2v + 1 of Philox counter (v / 2, k, 0, 5).  Gains: the exact
// diagonal, for either real component of g_a,
//     sum over baselines (a, b) and times of |g_b|^2 |V_ab|^2,
// V the visibility without gains (|V_ab| = |V_u| for its unique baseline u).
//
// Dense gain blocks.  For channel nu and baseline (i, j) with
// w = g_i g_j sum_t |V_ij|^2 / sigma_n^2 the Gauss-Newton block couples the
// components (x = Re g, y = Im g) as
//     H[x_i][x_j] = Re w,  H[y_i][y_j] = -Re w,  H[x_i][y_j] = H[y_i][x_j] = Im w,
// symmetric, with the diagonal above; the block plus 2 / s_g^2 I is positive
// definite and is factored in FP64 on the device (one workgroup per channel)
// and returned as FP32 lower-triangular factors.  Every sum runs in a fixed
// order, so the results do not depend on the launch.
#include <algorithm>

#include "../../include/bayesvis_serve.h"
#include "objects.hpp"
#include "philox.hpp"

namespace bv {

namespace {

constexpr int kMassThreads = 256;
constexpr int kMaxProbes = 4096;

// Complex probe of every visibility (see above).
__global__ void k_hutch_probe(float2* __restrict__ z, long nvis, uint64_t seed, uint32_t probe) {
  const long j = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (2 * j >= nvis) return;
  float n[4];
  philox_normals4(seed, static_cast<uint32_t>(j), probe, 0u, 5u, n);
  z[2 * j] = make_float2(n[0], n[1]);
  if (2 * j + 1 < nvis) z[2 * j + 1] = make_float2(n[2], n[3]);
}

// acc[i] = v_i^2 (first probe) or acc[i] + v_i^2, v = J^T z in the server's
// parameter layout [a | zero padding | gains (Re, Im) | F].
__global__ void k_hutch_acc(double* __restrict__ acc, const float* __restrict__ ga,
                            const float2* __restrict__ gg, const float* __restrict__ gf, int nalm,
                            int goff, int ngain, int len, int first) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float v = 0.f;
  if (i < nalm) {
    v = ga[i];
  } else if (i >= goff && i < goff + ngain) {
    const float2 g = gg[(i - goff) >> 1];
    v = ((i - goff) & 1) ? g.y : g.x;
  } else if (i == len - 1) {
    v = gf[0];
  }
  const double d = static_cast<double>(v) * v;
  acc[i] = first ? d : acc[i] + d;
}

// v2u[nu][u] = sum over times of |V_u(t, nu)|^2, times in order.
__global__ void k_vu_power(const float2* __restrict__ vu, int nt, int nf, int nubl,
                           double* __restrict__ v2u) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nf * nubl) return;
  double s = 0.0;
  for (int t = 0; t < nt; ++t) {
    const float2 v = vu[static_cast<size_t>(t) * nf * nubl + idx];
    s += static_cast<double>(v.x) * v.x + static_cast<double>(v.y) * v.y;
  }
  v2u[idx] = s;
}

// hg[nu][a] = sum over the baselines of antenna a (CSR order) of
// |g_other|^2 v2u[nu][u(bl)]  (no 1 / sigma_n^2 yet).
__global__ void k_gain_gn_diag(const double* __restrict__ v2u, const float2* __restrict__ gains,
                               const int* __restrict__ a_off, const int* __restrict__ a_list,
                               const int2* __restrict__ bl_ant, const int* __restrict__ bl_u,
                               int nf, int nant, int nubl, double* __restrict__ hg) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nf * nant) return;
  const int f = idx / nant, a = idx - f * nant;
  const float2* g = gains + static_cast<size_t>(f) * nant;
  double s = 0.0;
  for (int k = a_off[a]; k < a_off[a + 1]; ++k) {
    const int e = a_list[k];
    const int bl = e >> 1;
    const int2 ij = bl_ant[bl];
    const int other = (e & 1) ? ij.x : ij.y;
    const int u = bl_u[bl];
    const float2 go = g[other];
    const double g2 = static_cast<double>(go.x) * go.x + static_cast<double>(go.y) * go.y;
    s += g2 * v2u[static_cast<size_t>(f) * nubl + (u >= 0 ? u : ~u)];
  }
  hg[idx] = s;
}

// h = Gauss-Newton diagonal / sigma_n^2 + prior precision; minv = 1 / h.
// Padding entries get h = 1.
__global__ void k_mass_finalize(const double* __restrict__ acc, double inv_k, double inv_sig2,
                                const double* __restrict__ hg, const float* __restrict__ cvar,
                                double gprec, int nalm, int goff, int ngain, int len,
                                float* __restrict__ hdiag, float* __restrict__ minv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double h = 1.0;
  if (i < nalm) {
    h = acc[i] * inv_k * inv_sig2 + (cvar != nullptr ? 1.0 / static_cast<double>(cvar[i]) : 0.0);
  } else if (i >= goff && i < goff + ngain) {
    h = hg[(i - goff) >> 1] * inv_sig2 + gprec;
  } else if (i == len - 1) {
    h = acc[i] * inv_k * inv_sig2;
  }
  if (hdiag != nullptr) hdiag[i] = static_cast<float>(h);
  if (minv != nullptr) minv[i] = static_cast<float>(1.0 / h);
}

// Dense Gauss-Newton gain block of channel blockIdx.x into H [nb][nb] (FP64,
// row-major, nb = 2 n_ant), plus gprec on the diagonal.
__global__ void __launch_bounds__(kMassThreads)
k_gain_gn_assemble(const double* __restrict__ v2u, const double* __restrict__ hg,
                   const float2* __restrict__ gains, const int2* __restrict__ bl_ant,
                   const int* __restrict__ bl_u, int nant, int nbl, int nubl, double inv_sig2,
                   double gprec, double* __restrict__ H) {
  const int f = blockIdx.x;
  const int nb = 2 * nant;
  double* h = H + static_cast<size_t>(f) * nb * nb;
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) h[e] = 0.0;
  __syncthreads();
  const float2* g = gains + static_cast<size_t>(f) * nant;
  for (int a = threadIdx.x; a < nant; a += blockDim.x) {
    const double d = hg[static_cast<size_t>(f) * nant + a] * inv_sig2 + gprec;
    h[(2 * a) * nb + 2 * a] = d;
    h[(2 * a + 1) * nb + 2 * a + 1] = d;
  }
  // each baseline owns its eight entries (no two baselines share an antenna pair)
  for (int b = threadIdx.x; b < nbl; b += blockDim.x) {
    const int2 ij = bl_ant[b];
    const int u = bl_u[b];
    const double p = v2u[static_cast<size_t>(f) * nubl + (u >= 0 ? u : ~u)] * inv_sig2;
    const float2 gi = g[ij.x], gj = g[ij.y];
    const double wr = (static_cast<double>(gi.x) * gj.x - static_cast<double>(gi.y) * gj.y) * p;
    const double wi = (static_cast<double>(gi.x) * gj.y + static_cast<double>(gi.y) * gj.x) * p;
    const int xi = 2 * ij.x, yi = xi + 1, xj = 2 * ij.y, yj = xj + 1;
    h[xi * nb + xj] = wr;
    h[xj * nb + xi] = wr;
    h[yi * nb + yj] = -wr;
    h[yj * nb + yi] = -wr;
    h[xi * nb + yj] = wi;
    h[yj * nb + xi] = wi;
    h[yi * nb + xj] = wi;
    h[xj * nb + yi] = wi;
  }
}

// In-place Cholesky factor (lower) of channel blockIdx.x's block, right-looking
// by columns in FP64; thread c owns column c of the trailing update, which
// walks the rows below the pivot four at a time (each row coalesced across
// the workgroup).  A non-positive or non-finite pivot makes the factor NaN
// from there on (the server's admission check refuses such a factor).  Then
// the FP32 factor, zero above the diagonal, into L [nb][nb].
__global__ void __launch_bounds__(kMassThreads)
k_gain_chol(double* __restrict__ H, int nb, float* __restrict__ L) {
  __shared__ double col[kMassThreads];
  __shared__ double piv;
  const int f = blockIdx.x;
  const int c = threadIdx.x;
  double* h = H + static_cast<size_t>(f) * nb * nb;
  for (int j = 0; j < nb; ++j) {
    if (c == 0) {
      const double d = h[j * nb + j];
      piv = d > 0.0 ? sqrt(d) : __builtin_nan("");
    }
    __syncthreads();
    const double dj = piv;
    if (c == j) {
      h[j * nb + j] = dj;
      col[j] = dj;
    } else if (c > j && c < nb) {
      const double v = h[c * nb + j] / dj;
      h[c * nb + j] = v;
      col[c] = v;
    }
    __syncthreads();
    if (c > j && c < nb) {
      const double lc = col[c];
      int r = c;   // rows r >= c of column c change (row r's entries c <= r)
      for (; r + 3 < nb; r += 4) {
        double* p0 = h + static_cast<size_t>(r) * nb + c;
        const double a0 = p0[0], a1 = p0[nb], a2 = p0[2 * nb], a3 = p0[3 * nb];
        p0[0] = a0 - col[r] * lc;
        p0[nb] = a1 - col[r + 1] * lc;
        p0[2 * nb] = a2 - col[r + 2] * lc;
        p0[3 * nb] = a3 - col[r + 3] * lc;
      }
      for (; r < nb; ++r) h[static_cast<size_t>(r) * nb + c] -= col[r] * lc;
    }
    __syncthreads();
  }
  float* l = L + static_cast<size_t>(f) * nb * nb;
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int r = e / nb, cc = e - r * nb;
    l[e] = cc <= r ? static_cast<float>(h[e]) : 0.0f;
  }
}

struct MassWork {
  double* v2u = nullptr;   // [n_freq][n_ubl]
  double* hg = nullptr;    // [n_freq][n_ant]
  // diagonal
  float2* z = nullptr;     // [n_time][n_freq][n_bl]
  float* ga = nullptr;     // [n_freq][n_modes]
  float2* gg = nullptr;    // [n_freq][n_ant]
  float* gf = nullptr;     // [1]
  double* acc = nullptr;   // [len]
  // dense blocks
  double* H = nullptr;     // [n_freq][2 n_ant][2 n_ant]
  size_t bytes = 0;
};

long param_len(const vis_field* f, int* goff) {
  const long nalm = static_cast<long>(f->n_freq) * f->n_modes;
  *goff = static_cast<int>(round_up(nalm, 64));
  return *goff + 2L * f->n_freq * f->n_ant + 1;
}

MassWork carve_mass(const vis_field* f, void* work, size_t bytes) {
  Carver c{static_cast<char*>(work), bytes, 0};
  MassWork w;
  w.v2u = c.take<double>(static_cast<size_t>(f->n_freq) * f->n_ubl);
  w.hg = c.take<double>(static_cast<size_t>(f->n_freq) * f->n_ant);
  const size_t common = c.used;
  int goff;
  const long len = param_len(f, &goff);
  w.z = c.take<float2>(static_cast<size_t>(f->n_time) * f->n_freq * f->n_bl);
  w.ga = c.take<float>(static_cast<size_t>(f->n_freq) * f->n_modes);
  w.gg = c.take<float2>(static_cast<size_t>(f->n_freq) * f->n_ant);
  w.gf = c.take<float>(1);
  w.acc = c.take<double>(len);
  const size_t diag_end = c.used;
  c.used = common;
  const int nb = 2 * f->n_ant;
  w.H = c.take<double>(static_cast<size_t>(f->n_freq) * nb * nb);
  w.bytes = std::max(diag_end, c.used);
  return w;
}

void check_mass_args(const vis_field* f, const float* alm, const vis_c64* gains, const float* fwhm,
                     float sigma_n, float gain_prior_sigma) {
  BV_REQUIRE(f != nullptr, VIS_EINVAL, "null field");
  BV_REQUIRE(alm && gains && fwhm, VIS_EINVAL, "null device pointer");
  BV_REQUIRE(sigma_n > 0.f && sigma_n < 3.0e38f, VIS_EINVAL, "sigma_n must be positive and finite");
  BV_REQUIRE(gain_prior_sigma >= 0.f && gain_prior_sigma < 3.0e38f, VIS_EINVAL,
             "gain_prior_sigma must be >= 0 and finite");
}

void gain_power(const vis_field* f, const vis_c64* gains, const MassWork& w, hipStream_t s) {
  const auto& T = f->tab;
  const int n1 = f->n_freq * f->n_ubl, n2 = f->n_freq * f->n_ant;
  k_vu_power<<<ceil_div(n1, kMassThreads), kMassThreads, 0, s>>>(f->scr.vu, f->n_time, f->n_freq,
                                                                 f->n_ubl, w.v2u);
  check_launch("k_vu_power");
  k_gain_gn_diag<<<ceil_div(n2, kMassThreads), kMassThreads, 0, s>>>(
      w.v2u, reinterpret_cast<const float2*>(gains), T.a_off, T.a_list, T.bl_ant, T.bl_u,
      f->n_freq, f->n_ant, f->n_ubl, w.hg);
  check_launch("k_gain_gn_diag");
}

}  // namespace

}  // namespace bv

using namespace bv;

extern "C" {

vis_status hmc_mass_work_bytes(const vis_field* f, size_t* bytes) {
  return guarded([&] {
    BV_REQUIRE(f != nullptr && bytes != nullptr, VIS_EINVAL, "null argument");
    *bytes = carve_mass(f, nullptr, 0).bytes;
  });
}

vis_status hmc_mass_diag(const vis_field* f, const float* alm, const vis_c64* gains,
                         const float* fwhm, float sigma_n, const float* alm_prior_var,
                         float gain_prior_sigma, int32_t n_probes, uint64_t seed, float* hdiag,
                         float* minv, void* work, size_t work_bytes, void* stream) {
  return guarded([&] {
    check_mass_args(f, alm, gains, fwhm, sigma_n, gain_prior_sigma);
    BV_REQUIRE(n_probes >= 1 && n_probes <= kMaxProbes, VIS_EINVAL, "n_probes must be in [1, %d]",
               kMaxProbes);
    BV_REQUIRE(hdiag != nullptr || minv != nullptr, VIS_EINVAL, "no output");
    BV_REQUIRE(work != nullptr, VIS_EINVAL, "null work buffer");
    const MassWork w = carve_mass(f, work, work_bytes);
    BV_REQUIRE(work_bytes >= w.bytes, VIS_ENOMEM, "work buffer too small: need %zu bytes", w.bytes);
    hipStream_t s = as_stream(stream);
    int goff;
    const int len = static_cast<int>(param_len(f, &goff));
    const int nalm = f->n_freq * f->n_modes, ngain = 2 * f->n_freq * f->n_ant;
    const long nvis = static_cast<long>(f->n_time) * f->n_freq * f->n_bl;
    forward_core(f, alm, fwhm, s);
    for (int k = 0; k < n_probes; ++k) {
      k_hutch_probe<<<ceil_div((nvis + 1) / 2, kMassThreads), kMassThreads, 0, s>>>(
          w.z, nvis, seed, static_cast<uint32_t>(k));
      check_launch("k_hutch_probe");
      launch_gains(f, kGainAdj, f->scr.vu, reinterpret_cast<const float2*>(gains), w.z, 0.f, nullptr,
                   nullptr, f->scr.gco, f->scr.g_part, s);
      adjoint_tail(f, fwhm, w.ga, w.gg, w.gf, false, nullptr, s);
      k_hutch_acc<<<ceil_div(len, kMassThreads), kMassThreads, 0, s>>>(w.acc, w.ga, w.gg, w.gf, nalm,
                                                                      goff, ngain, len, k == 0);
      check_launch("k_hutch_acc");
    }
    gain_power(f, gains, w, s);
    const double gprec = gain_prior_sigma > 0.f
                             ? 2.0 / (static_cast<double>(gain_prior_sigma) * gain_prior_sigma)
                             : 0.0;
    k_mass_finalize<<<ceil_div(len, kMassThreads), kMassThreads, 0, s>>>(
        w.acc, 1.0 / n_probes, 1.0 / (static_cast<double>(sigma_n) * sigma_n), w.hg, alm_prior_var,
        gprec, nalm, goff, ngain, len, hdiag, minv);
    check_launch("k_mass_finalize");
  });
}

vis_status hmc_gain_mass_blocks(const vis_field* f, const float* alm, const vis_c64* gains,
                                const float* fwhm, float sigma_n, float gain_prior_sigma,
                                float* chol, void* work, size_t work_bytes, void* stream) {
  return guarded([&] {
    check_mass_args(f, alm, gains, fwhm, sigma_n, gain_prior_sigma);
    BV_REQUIRE(chol != nullptr, VIS_EINVAL, "null output");
    BV_REQUIRE(2 * f->n_ant <= kMassThreads, VIS_EINVAL, "dense gain blocks need 2 n_ant <= %d",
               kMassThreads);
    BV_REQUIRE(work != nullptr, VIS_EINVAL, "null work buffer");
    const MassWork w = carve_mass(f, work, work_bytes);
    BV_REQUIRE(work_bytes >= w.bytes, VIS_ENOMEM, "work buffer too small: need %zu bytes", w.bytes);
    hipStream_t s = as_stream(stream);
    const auto& T = f->tab;
    forward_core(f, alm, fwhm, s);
    gain_power(f, gains, w, s);
    const double gprec = gain_prior_sigma > 0.f
                             ? 2.0 / (static_cast<double>(gain_prior_sigma) * gain_prior_sigma)
                             : 0.0;
    k_gain_gn_assemble<<<f->n_freq, kMassThreads, 0, s>>>(
        w.v2u, w.hg, reinterpret_cast<const float2*>(gains), T.bl_ant, T.bl_u, f->n_ant, f->n_bl,
        f->n_ubl, 1.0 / (static_cast<double>(sigma_n) * sigma_n), gprec, w.H);
    check_launch("k_gain_gn_assemble");
    k_gain_chol<<<f->n_freq, kMassThreads, 0, s>>>(w.H, 2 * f->n_ant, chol);
    check_launch("k_gain_chol");
  });
}

}  // extern "C"
