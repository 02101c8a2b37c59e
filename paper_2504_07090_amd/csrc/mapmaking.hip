// Map-making: x_hat = D A^H N^-1 y (Sec. 4.3, eq. vis_to_map, eq. map_psf).
//
// A is the beam-and-fringe response with gains (eq. rime_matrix), stacked
// over times and baselines.  Re(A^H y) at the pixels above the horizon is the
// adjoint fringe pass applied to the cotangent y (unique-baseline collapse in
// the gains kernel, then the adjoint fringe kernel, unchanged).  The diagonal
// normalisation D = diag(A^H A)^-1 makes the point-spread function unit on
// its diagonal (N is proportional to the identity, so the noise level
// cancels); the diagonal has the closed form
//     (A^H A)_pp = dOmega^2 sum_t B(p, t)^2 sum_{i<j} |g_i g_j|^2,
// evaluated here per (channel, visible pixel), and
//     sum_{i<j} |g_i g_j|^2 = ((sum |g|^2)^2 - sum |g|^4) / 2.
// Where the response is negligible the ratio only amplifies noise (it grows
// like 1 / B), so pixels whose weight is below kMapWeightFloor times the
// channel's largest weight map to 0, as do pixels never above the horizon.
#include "objects.hpp"

namespace bv {

constexpr float kMapWeightFloor = 1e-6f;

// w[f][k] = (A^H A)_pp for visible slot k; one wavefront per (64-pixel chunk,
// channel).  Also clears the channel maxima that k_map_wmax raises.
__global__ void __launch_bounds__(64)
k_map_weight(int nf, int nvp, int nant, double d_omega, const float* __restrict__ sigr,
             const float* __restrict__ TH2, const int2* __restrict__ chunk_t,
             const float2* __restrict__ gains, const float* __restrict__ fwhm, float* __restrict__ w,
             unsigned* __restrict__ wmax) {
  const int chunk = blockIdx.x, f = blockIdx.y, lane = threadIdx.x;
  if (chunk == 0 && lane == 0) wmax[f] = 0u;
  const float sig = fwhm[0] * sigr[f];
  const float kb = 1.0f / (2.0f * sig * sig * static_cast<float>(kLn2));
  double s2 = 0.0, s4 = 0.0;
  for (int a = lane; a < nant; a += 64) {
    const float2 g = gains[static_cast<size_t>(f) * nant + a];
    const double m2 = static_cast<double>(g.x) * g.x + static_cast<double>(g.y) * g.y;
    s2 += m2;
    s4 += m2 * m2;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    s2 += __shfl_xor(s2, o);
    s4 += __shfl_xor(s4, o);
  }
  const double sg = 0.5 * (s2 * s2 - s4);
  const int k = chunk * kChunk + lane;
  const int2 tr = chunk_t[chunk];
  // sum of B^2 = 2^(-2 theta^2 kb) over the visible times: four independent
  // partial sums so four loads are in flight; the hardware exponential
  // (a square below 2^-126 adds nothing to the weight)
  float sb[4] = {0.f, 0.f, 0.f, 0.f};
  int t = tr.x;
  for (; t + 3 <= tr.y; t += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      sb[q] += __builtin_amdgcn_exp2f(-2.0f * kb * TH2[static_cast<size_t>(t + q) * nvp + k]);
  }
  for (int q = 0; t <= tr.y; ++t, ++q)
    sb[q] += __builtin_amdgcn_exp2f(-2.0f * kb * TH2[static_cast<size_t>(t) * nvp + k]);
  const float sbt = (sb[0] + sb[1]) + (sb[2] + sb[3]);
  w[static_cast<size_t>(f) * nvp + k] = static_cast<float>(d_omega * d_omega * sg * sbt);
}

// wmax[f] = max_k w[f][k] as the bits of a non-negative float (whose order
// is that of the unsigned integers, so the atomic maximum of the slices is
// exact and independent of their order); one 256-thread block per (channel,
// slice of k).
__global__ void __launch_bounds__(256)
k_map_wmax(int nvp, int nsplit, const float* __restrict__ w, unsigned* __restrict__ wmax) {
  __shared__ float red[4];
  const int f = blockIdx.x, sl = blockIdx.y, tid = threadIdx.x;
  const int per = (nvp + nsplit - 1) / nsplit, k0 = sl * per, k1 = min(nvp, k0 + per);
  float m = 0.f;
  for (int k = k0 + tid; k < k1; k += 256) m = fmaxf(m, w[static_cast<size_t>(f) * nvp + k]);
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) atomicMax(wmax + f, __float_as_uint(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]))));
}

// map[f][p] = dimg[f][slot] / w[f][slot] where w >= floor * wmax[f], else 0.
__global__ void __launch_bounds__(256)
k_map_finish(int nf, int npix, int nvp, const int* __restrict__ vidx, const float* __restrict__ dimg,
             const float* __restrict__ w, const unsigned* __restrict__ wmax, float* __restrict__ map,
             float* __restrict__ weight) {
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<long>(nf) * npix) return;
  const int f = static_cast<int>(idx / npix), p = static_cast<int>(idx - static_cast<long>(f) * npix);
  const int slot = vidx[p];
  float x = 0.f, wt = 0.f;
  if (slot >= 0) {
    const float wm = __uint_as_float(wmax[f]);
    wt = w[static_cast<size_t>(f) * nvp + slot];
    if (wt > 0.f && wt >= kMapWeightFloor * wm) x = dimg[static_cast<size_t>(f) * nvp + slot] / wt;
  }
  map[idx] = x;
  if (weight != nullptr) weight[idx] = wt;
}

void launch_map_finish(const vis_field* f, const vis_c64* gains, const float* fwhm, float* map,
                       float* weight, hipStream_t st) {
  // the sky scratch is free after the adjoint fringe pass: it holds the
  // weights; the F-gradient partials (not needed here) the channel maxima
  float* w = f->scr.img;
  unsigned* wmax = reinterpret_cast<unsigned*>(f->scr.f_part);
  {
    ProfScope ps(&f->prof, "k_map_weight", st);
    k_map_weight<<<dim3(f->n_chunks, f->n_freq), 64, 0, st>>>(
        f->n_freq, f->nv_pad, f->n_ant, f->d_omega, f->tab.sigr, f->tab.th2,
        f->tab.chunk_t, reinterpret_cast<const float2*>(gains), fwhm, w, wmax);
    check_launch("k_map_weight");
  }
  const int nsplit = std::max(1, std::min(16, f->n_chunks));
  {
    ProfScope ps(&f->prof, "k_map_wmax", st);
    k_map_wmax<<<dim3(f->n_freq, nsplit), 256, 0, st>>>(f->nv_pad, nsplit, w, wmax);
    check_launch("k_map_wmax");
  }
  const long n = static_cast<long>(f->n_freq) * f->basis->n_pix;
  ProfScope ps(&f->prof, "k_map_finish", st);
  k_map_finish<<<ceil_div(n, 256), 256, 0, st>>>(f->n_freq, f->basis->n_pix, f->nv_pad, f->tab.vidx,
                                                  f->scr.dimg, w, wmax, map, weight);
  check_launch("k_map_finish");
}

}  // namespace bv
