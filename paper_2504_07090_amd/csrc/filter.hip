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
// both GEMMs on v_mfma_f32_16x16x4_f32 (A[i][k] in lane i + 16 k, B[k][j] in
// lane j + 16 k, D[i][j] in lane j + 16 (i / 4), register i % 4).  The chi^2
// terms are summed per wavefront in FP64 and totalled in a fixed order.
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
// Both GEMMs stream the visibility-sized operands once, so they are bound by
// HBM, not by the matrix cores: one wavefront per (time, 16 CT columns, 64
// rows) keeps a 64 x 16 CT output block in registers (4 x CT tiles of
// 16 x 16), reads each operand row segment once as 8-byte vectors, and loops
// over all nf rows of the contraction, 16 per step with all the step's loads
// in flight together.  In tile c, lane j holds column
// x0 + 32 (c >> 1) + 2 j + (c & 1), so one 8-byte load per lane feeds two
// tiles and every store is an 8-byte pair of adjacent columns.
//
// RESID: Rf = F (d - m);  W = Rf / N~;  part = chi^2 of the wave's block.
// COT:   cot = -2 F^T W.
constexpr int kFilterColTiles = 4;

template <bool RESID, int CT>
__global__ void __launch_bounds__(64)
k_filter_gemm(int nf, int nx, float inv_sig2, const float* __restrict__ F, const float* __restrict__ fft,
              const float* x_a, const float* x_b, float* __restrict__ out, double* __restrict__ part) {
  constexpr int NH = CT / 2;   // 8-byte loads per lane and contraction row
  const int x0 = blockIdx.x * 16 * CT, n0 = blockIdx.y * 64, t = blockIdx.z;
  const int lane = threadIdx.x, j = lane & 15, kk = lane >> 4;
  const size_t tb = static_cast<size_t>(t) * nf * nx;
  typedef float f2 __attribute__((ext_vector_type(2)));
  f4 acc[4][CT];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[r][c] = f4{0.f, 0.f, 0.f, 0.f};
  int arow[4];   // this lane's A row in each row tile (clamped: rows past nf are never stored)
#pragma unroll
  for (int r = 0; r < 4; ++r) arow[r] = min(n0 + 16 * r + j, nf - 1);
  bool colok[NH];
  int xc[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    xc[h] = x0 + 32 * h + 2 * j;   // even, and nx is even: the pair is whole or absent
    colok[h] = xc[h] < nx;
  }
  // operand rows k0 + 4 q + kk of one 16-row step and the filter entries
  // they meet, loaded unconditionally from clamped addresses so that all
  // loads of a step are in flight together (a load under a branch is waited
  // for before the branch ends); entries outside the matrix are zeroed when
  // the step uses them
  struct Rows { f2 a[4][NH], b[RESID ? 4 : 1][NH]; float f[4][4]; };
  auto load_b = [&](int k0, Rows& R) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = min(k0 + 4 * q + kk, nf - 1);
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const size_t o = tb + static_cast<size_t>(k) * nx + min(xc[h], nx - 2);
        R.a[q][h] = *reinterpret_cast<const f2*>(x_a + o);
        if (RESID) R.b[q][h] = *reinterpret_cast<const f2*>(x_b + o);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        R.f[q][r] = RESID ? F[static_cast<size_t>(arow[r]) * nf + k] : F[static_cast<size_t>(k) * nf + arow[r]];
    }
  };
  auto step = [&](int k0, const Rows& R) {
    f2 b[4][NH];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool kok = k0 + 4 * q + kk < nf;
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const f2 v = RESID ? R.a[q][h] - R.b[RESID ? q : 0][h] : R.a[q][h];
        b[q][h] = kok && colok[h] ? v : f2{0.f, 0.f};
      }
    }
    float a[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool kok = k0 + 4 * q + kk < nf;
#pragma unroll
      for (int r = 0; r < 4; ++r) a[q][r] = kok ? R.f[q][r] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q][r], b[q][c >> 1][c & 1], acc[r][c], 0, 0, 0);
  };
  for (int k0 = 0; k0 < nf; k0 += 16) {
    Rows R;
    load_b(k0, R);   // all loads of the step in flight at once
    step(k0, R);
  }
  double chi = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int nu = n0 + 16 * r + 4 * kk + q;
      if (nu >= nf) continue;
      const float w = RESID ? inv_sig2 / fft[nu] : -2.0f;
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        if (!colok[h]) continue;
        const float v0 = acc[r][2 * h][q], v1 = acc[r][2 * h + 1][q];
        if (RESID) chi += (static_cast<double>(v0) * v0 + static_cast<double>(v1) * v1) * w;
        *reinterpret_cast<f2*>(out + tb + static_cast<size_t>(nu) * nx + xc[h]) = f2{v0 * w, v1 * w};
      }
    }
  if (RESID) {
    for (int o = 32; o >= 1; o >>= 1) chi += __shfl_xor(chi, o);
    if (lane == 0) part[(static_cast<size_t>(t) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = chi;
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
  w.nparts = static_cast<long>(f->n_time) * ceil_div(f->n_freq, 64) *
             ceil_div(2L * f->n_bl, 16L * kFilterColTiles);
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
  dim3 grid(ceil_div(nx, 16 * kFilterColTiles), ceil_div(f->n_freq, 64), f->n_time);
  {
    ProfScope ps(&f->prof, "k_filter_resid", st);
    k_filter_gemm<true, kFilterColTiles><<<grid, 64, 0, st>>>(f->n_freq, nx, 1.0f / (sigma_n * sigma_n), flt->F, flt->fft,
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
  dim3 grid(ceil_div(nx, 16 * kFilterColTiles), ceil_div(f->n_freq, 64), f->n_time);
  ProfScope ps(&f->prof, "k_filter_cot", st);
  k_filter_gemm<false, kFilterColTiles><<<grid, 64, 0, st>>>(f->n_freq, nx, 0.f, flt->F, nullptr,
                                            reinterpret_cast<const float*>(w.w), nullptr,
                                            reinterpret_cast<float*>(w.m), nullptr);
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
