// Delay (high-pass) filter along frequency and the filtered chi^2.
//
// Sec. 2.1, eq. rime_filter and eq. gpr: F = I - C_fg (C_fg + eps I)^-1 with
// C_fg(nu, nu') = sinc(2 tau_max (nu - nu')) (a tophat of half-width tau_max
// in delay) and eps the relative noise level.  Sec. 3.5, eq. filtered_noise:
// the filtered noise covariance N~ = F N F^T is used through its diagonal,
// sigma_n^2 (F F^T)_nu,nu.
//
// F is built once on the host in FP64 (Cholesky of C_fg + eps I) and kept on
// the device in FP32.  Per evaluation, with r = d - m laid out [t][nu][2 n_bl]
// (real and imaginary parts are independent columns, F being real):
//     Rf = F r                              (GEMM nu x nu' x 2 n_bl per time)
//     chi^2 = sum Rf^2 / N~_nu,             W = Rf / N~_nu
//     c = -2 F^T W                          (GEMM, the cotangent dL/dm)
// both GEMMs on v_mfma_f32_16x16x4_f32 with one 16 x 16 output tile per
// wavefront: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// D[i][j] in lane j + 16 (i / 4), register i % 4.  The chi^2 terms are summed
// per wavefront in FP64 and totalled in a fixed order.
#include <cmath>
#include <vector>

#include "objects.hpp"

struct vis_filter {
  int n = 0;
  float* F = nullptr;       // [n][n] row-major
  float* fft = nullptr;     // [n] (F F^T)_nu,nu
};

namespace bv {

typedef float f4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ host build --
static double sinc_pi(double x) {
  if (x == 0.0) return 1.0;
  const double y = kPi * x;
  return std::sin(y) / y;
}

static void build_filter(int n, const double* freq, double tau, double eps, std::vector<double>& F,
                         std::vector<double>& fft) {
  BV_REQUIRE(n >= 1 && n <= 4096, VIS_EINVAL, "n_freq %d out of range [1, 4096]", n);
  BV_REQUIRE(freq != nullptr, VIS_EINVAL, "null frequency list");
  BV_REQUIRE(std::isfinite(tau) && tau >= 0.0, VIS_EINVAL, "tau_max must be finite and >= 0");
  BV_REQUIRE(std::isfinite(eps) && eps > 0.0, VIS_EINVAL, "noise_ratio must be positive");
  for (int i = 0; i < n; ++i)
    BV_REQUIRE(std::isfinite(freq[i]) && freq[i] > 0.0, VIS_EINVAL, "frequency %d is not positive", i);
  const size_t N = static_cast<size_t>(n);
  std::vector<double> C(N * N), L(N * N, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C[i * N + j] = sinc_pi(2.0 * tau * (freq[i] - freq[j]));
  // Cholesky of K = C + eps I (lower triangle)
  for (int j = 0; j < n; ++j) {
    double d = C[j * N + j] + eps;
    for (int k = 0; k < j; ++k) d -= L[j * N + k] * L[j * N + k];
    BV_REQUIRE(d > 0.0, VIS_EINVAL, "filter covariance is not positive definite");
    const double ljj = std::sqrt(d);
    L[j * N + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double v = C[i * N + j];
      for (int k = 0; k < j; ++k) v -= L[i * N + k] * L[j * N + k];
      L[i * N + j] = v / ljj;
    }
  }
  // X = K^-1 C column by column; C symmetric, so C K^-1 = X^T and F = I - X^T
  F.assign(N * N, 0.0);
  std::vector<double> y(N);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {   // L y = C[:, c]
      double v = C[i * N + c];
      for (int k = 0; k < i; ++k) v -= L[i * N + k] * y[k];
      y[i] = v / L[i * N + i];
    }
    for (int i = n - 1; i >= 0; --i) {   // L^T x = y
      double v = y[i];
      for (int k = i + 1; k < n; ++k) v -= L[k * N + i] * y[k];
      y[i] = v / L[i * N + i];
    }
    for (int i = 0; i < n; ++i) F[c * N + i] = (c == i ? 1.0 : 0.0) - y[i];   // row c of X^T
  }
  fft.assign(N, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += F[i * N + j] * F[i * N + j];
    fft[i] = s;
  }
}

// --------------------------------------------------------------- kernels --
// Rf[t][nu][x] = sum_k F[nu][k] (d - m)[t][k][x];  W = Rf / N~;  part = per-wave chi^2.
// grid (ceil(nx / 16), ceil(nf / 16), nt), one wavefront per block.
__global__ void __launch_bounds__(64)
k_filter_resid(int nf, int nx, float inv_sig2, const float* __restrict__ F, const float* __restrict__ fft,
               const float* __restrict__ d, const float* __restrict__ m, float* __restrict__ W,
               double* __restrict__ part) {
  const int x0 = blockIdx.x * 16, n0 = blockIdx.y * 16, t = blockIdx.z;
  const int lane = threadIdx.x, i = lane & 15, kk = lane >> 4;
  const int row = min(n0 + i, nf - 1), col = min(x0 + i, nx - 1);
  const size_t tb = static_cast<size_t>(t) * nf * nx;
  f4 acc = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < nf; k0 += 16) {
    float a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 4 * q + kk;
      const bool ok = k < nf;
      const size_t o = tb + static_cast<size_t>(k) * nx + col;
      a[q] = ok ? F[static_cast<size_t>(row) * nf + k] : 0.f;
      b[q] = ok ? d[o] - m[o] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], b[q], acc, 0, 0, 0);
  }
  double chi = 0.0;
  const int xo = x0 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int nu = n0 + 4 * kk + r;
    if (nu < nf && xo < nx) {
      const float w = inv_sig2 / fft[nu];
      chi += static_cast<double>(acc[r]) * acc[r] * w;
      W[tb + static_cast<size_t>(nu) * nx + xo] = acc[r] * w;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) chi += __shfl_xor(chi, o);
  if (lane == 0) part[(static_cast<size_t>(t) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = chi;
}

// cot[t][nu'][x] = -2 sum_nu F[nu][nu'] W[t][nu][x];  grid as above.
__global__ void __launch_bounds__(64)
k_filter_cot(int nf, int nx, const float* __restrict__ F, const float* __restrict__ W,
             float* __restrict__ cot) {
  const int x0 = blockIdx.x * 16, n0 = blockIdx.y * 16, t = blockIdx.z;
  const int lane = threadIdx.x, i = lane & 15, kk = lane >> 4;
  const int row = min(n0 + i, nf - 1), col = min(x0 + i, nx - 1);
  const size_t tb = static_cast<size_t>(t) * nf * nx;
  f4 acc = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < nf; k0 += 16) {
    float a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 4 * q + kk;
      const bool ok = k < nf;
      a[q] = ok ? F[static_cast<size_t>(k) * nf + row] : 0.f;
      b[q] = ok ? W[tb + static_cast<size_t>(k) * nx + col] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], b[q], acc, 0, 0, 0);
  }
  const int xo = x0 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int nu = n0 + 4 * kk + r;
    if (nu < nf && xo < nx) cot[tb + static_cast<size_t>(nu) * nx + xo] = -2.0f * acc[r];
  }
}

// out = sum of part[0..n) in FP64, one 1024-thread block, fixed order.
__global__ void __launch_bounds__(1024) k_sum_f64(long n, const double* __restrict__ part, double* out) {
  __shared__ double red[16];
  const int tid = threadIdx.x;
  double p[4] = {0.0, 0.0, 0.0, 0.0};
  for (long i = tid; i < n; i += 1024) p[(i >> 10) & 3] += part[i];
  double acc = (p[0] + p[1]) + (p[2] + p[3]);
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += red[w];
    *out = s;
  }
}

// ------------------------------------------------------------ launchers --
FilteredWork carve_filtered_work(const vis_field* f, void* work, size_t bytes) {
  const size_t nvis = static_cast<size_t>(f->n_time) * f->n_freq * f->n_bl;
  FilteredWork w;
  w.nparts = static_cast<long>(f->n_time) * ceil_div(f->n_freq, 16) * ceil_div(2L * f->n_bl, 16);
  Carver cv{static_cast<char*>(work), bytes, 0};
  w.m = cv.take<float2>(nvis);
  w.w = cv.take<float2>(nvis);
  w.part = cv.take<double>(w.nparts);
  w.bytes = cv.used;
  return w;
}

static void check_filter(const vis_field* f, const vis_filter* flt) {
  BV_REQUIRE(flt != nullptr, VIS_EINVAL, "null filter");
  BV_REQUIRE(flt->n == f->n_freq, VIS_EINVAL, "filter has %d channels, the field %d", flt->n, f->n_freq);
}

void launch_filter_chi2(const vis_field* f, const vis_filter* flt, const float2* data, float sigma_n,
                        const FilteredWork& w, double* chi2, hipStream_t st) {
  check_filter(f, flt);
  const int nx = 2 * f->n_bl;
  dim3 grid(ceil_div(nx, 16), ceil_div(f->n_freq, 16), f->n_time);
  {
    ProfScope ps(&f->prof, "k_filter_resid", st);
    k_filter_resid<<<grid, 64, 0, st>>>(f->n_freq, nx, 1.0f / (sigma_n * sigma_n), flt->F, flt->fft,
                                        reinterpret_cast<const float*>(data),
                                        reinterpret_cast<const float*>(w.m),
                                        reinterpret_cast<float*>(w.w), w.part);
    check_launch("k_filter_resid");
  }
  ProfScope ps(&f->prof, "k_sum_f64", st);
  k_sum_f64<<<1, 1024, 0, st>>>(w.nparts, w.part, chi2);
  check_launch("k_sum_f64");
}

void launch_filter_cot(const vis_field* f, const vis_filter* flt, const FilteredWork& w, hipStream_t st) {
  check_filter(f, flt);
  const int nx = 2 * f->n_bl;
  dim3 grid(ceil_div(nx, 16), ceil_div(f->n_freq, 16), f->n_time);
  ProfScope ps(&f->prof, "k_filter_cot", st);
  k_filter_cot<<<grid, 64, 0, st>>>(f->n_freq, nx, flt->F, reinterpret_cast<const float*>(w.w),
                                    reinterpret_cast<float*>(w.m));
  check_launch("k_filter_cot");
}

}  // namespace bv

using namespace bv;

extern "C" {

vis_status vis_filter_build(int32_t n_freq, const double* freq_hz, double tau_max_s, double noise_ratio,
                            double* F_out, double* fft_diag) {
  return guarded([&] {
    BV_REQUIRE(F_out != nullptr && fft_diag != nullptr, VIS_EINVAL, "null output");
    std::vector<double> F, fft;
    build_filter(n_freq, freq_hz, tau_max_s, noise_ratio, F, fft);
    std::copy(F.begin(), F.end(), F_out);
    std::copy(fft.begin(), fft.end(), fft_diag);
  });
}

vis_status vis_filter_workspace_bytes(int32_t n_freq, size_t* bytes) {
  return guarded([&] {
    BV_REQUIRE(bytes != nullptr, VIS_EINVAL, "null output");
    BV_REQUIRE(n_freq >= 1 && n_freq <= 4096, VIS_EINVAL, "n_freq %d out of range [1, 4096]", n_freq);
    Carver cv;
    cv.take<float>(static_cast<size_t>(n_freq) * n_freq);
    cv.take<float>(n_freq);
    *bytes = cv.used;
  });
}

vis_status vis_filter_create(int32_t n_freq, const double* freq_hz, double tau_max_s, double noise_ratio,
                             void* ws, size_t bytes, void* stream, vis_filter** out) {
  vis_filter* flt = nullptr;
  vis_status st = guarded([&] {
    BV_REQUIRE(out != nullptr && ws != nullptr, VIS_EINVAL, "null workspace or output");
    std::vector<double> F, fft;
    build_filter(n_freq, freq_hz, tau_max_s, noise_ratio, F, fft);
    flt = new vis_filter();
    flt->n = n_freq;
    Carver cv{static_cast<char*>(ws), bytes, 0};
    flt->F = cv.take<float>(F.size());
    flt->fft = cv.take<float>(fft.size());
    std::vector<float> F32(F.begin(), F.end()), fft32(fft.begin(), fft.end());
    hipStream_t s = as_stream(stream);
    BV_HIP(hipMemcpyAsync(flt->F, F32.data(), F32.size() * sizeof(float), hipMemcpyHostToDevice, s));
    BV_HIP(hipMemcpyAsync(flt->fft, fft32.data(), fft32.size() * sizeof(float), hipMemcpyHostToDevice, s));
    BV_HIP(hipStreamSynchronize(s));
    *out = flt;
  });
  if (st != VIS_OK) delete flt;
  return st;
}

vis_status vis_filter_destroy(vis_filter* filter) {
  delete filter;
  return VIS_OK;
}

vis_status vis_filtered_work_bytes(const vis_field* field, size_t* bytes) {
  return guarded([&] {
    BV_REQUIRE(field != nullptr && bytes != nullptr, VIS_EINVAL, "null argument");
    *bytes = carve_filtered_work(field, nullptr, 0).bytes;
  });
}

}  // extern "C"
