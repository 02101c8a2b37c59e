// Sky synthesis I = Y a and its transpose dL/da = Y^T dL/dI on MFMA.
//
// Sec. 3.2 (eq. fg_harmonic_matrix): the sky at every pixel is a linear
// combination of the harmonic basis columns.  Only pixels that rise above the
// horizon at some time of the observation are synthesised (the beam is zero
// elsewhere, so those pixels never reach a visibility); their Y rows are
// gathered through the field's visible-pixel list.
//
// Shapes: M = n_freq (rows of a), N = visible pixels, K = n_modes.  Both
// operands are K-contiguous in the forward ("NT" product), so tiles stream
// straight from HBM into LDS.  The adjoint is M = n_freq, N = n_modes,
// K = visible pixels, split over K for occupancy and reduced in a fixed order.
//
// MFMA v_mfma_f32_16x16x4_f32 operand layout (wave64):
//   A[i][k]: lane i + 16 k;  B[k][j]: lane j + 16 k;  D[i][j]: lane j + 16 (i / 4), register i % 4.
#include "objects.hpp"

namespace bv {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// part[s][f][k] = sum_{c in split s, c < nm} alm[f][c] Y[vpix[k]][c]
// Block tile 64 (f) x 64 (k), K step 32, 4 waves as 2 x 2 sub-tiles of 32 x 32;
// the mode range is split over blockIdx.z so the grid fills the chip, and the
// splits are summed in a fixed order afterwards.
__global__ void __launch_bounds__(256)
k_synth_fwd_f32(int nf, int nm, int nvp, int kpad, int kps, const float* __restrict__ alm,
                const float* __restrict__ Y, const int* __restrict__ vpix, float* __restrict__ part) {
  __shared__ float As[2][64][33];
  __shared__ float Bs[2][64][33];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = blockIdx.x * 64, m0 = blockIdx.y * 64, split = blockIdx.z;
  const int kbeg = split * kps, kend = min(nm, kbeg + kps);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  const int arow = m0 + lr;
  const float* yrow = Y + static_cast<size_t>(vpix[n0 + lr]) * kpad;
  const float* arow_p = alm + static_cast<size_t>(arow) * nm;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  float ra[8];
  f4 rb0, rb1;
  const int ksteps = (kend - kbeg + 31) / 32;
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int c = k0 + lk + q;
      ra[q] = (arow < nf && c < kend) ? arow_p[c] : 0.f;
    }
    rb0 = *reinterpret_cast<const f4*>(yrow + k0 + lk);
    rb1 = *reinterpret_cast<const f4*>(yrow + k0 + lk + 4);
  };
  if (ksteps > 0) gload(kbeg);
  for (int s = 0; s < ksteps; ++s) {
    const int buf = s & 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      As[buf][lr][lk + q] = ra[q];
      As[buf][lr][lk + 4 + q] = ra[4 + q];
      Bs[buf][lr][lk + q] = rb0[q];
      Bs[buf][lr][lk + 4 + q] = rb1[q];
    }
    __syncthreads();
    if (s + 1 < ksteps) gload(kbeg + (s + 1) * 32);
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[buf][wm + 16 * i + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[buf][wn + 16 * j + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma4(a[i], b[j], acc[i][j]);
    }
  }
  float* out = part + static_cast<size_t>(split) * nf * nvp;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int k = n0 + wn + 16 * j + (lane & 15);
        if (f < nf) out[static_cast<size_t>(f) * nvp + k] = acc[i][j][r];
      }
}

// img[f][k] = sum_s part[s][f][k], fixed order over s.
__global__ void __launch_bounds__(256)
k_sum_fwd_splits(int nsplit, long n, const float* __restrict__ part, float* __restrict__ img) {
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  float s = 0.f;
  for (int q = 0; q < nsplit; ++q) s += part[q * n + idx];
  img[idx] = s;
}

// part[s][f][c] = sum_{k in split s} dimg[f][k] Y[vpix[k]][c]
// Block tile 64 (f) x 64 (c), K step 16 pixels.
__global__ void __launch_bounds__(256)
k_synth_adj_f32(int nf, int nvp, int kpad, int kps, const float* __restrict__ dimg,
                const float* __restrict__ Y, const int* __restrict__ vpix, float* __restrict__ part) {
  __shared__ float As[2][64][17];
  __shared__ float Bs[2][16][80];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = blockIdx.x * 64, m0 = blockIdx.y * 64, split = blockIdx.z;
  const int kbeg = split * kps, kend = min(nvp, kbeg + kps);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = tid >> 2, lk = (tid & 3) * 4;      // A loads: row f, 4 pixels
  const int br = tid >> 4, bc = (tid & 15) * 4;     // B loads: pixel row, 4 modes
  const int arow = m0 + lr;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  f4 ra, rb;
  const int ksteps = (kend - kbeg + 15) / 16;
  auto gload = [&](int k0) {
    const int ka = k0 + lk;
    ra = (arow < nf) ? *reinterpret_cast<const f4*>(dimg + static_cast<size_t>(arow) * nvp + ka)
                     : f4{0.f, 0.f, 0.f, 0.f};
    const int kb = k0 + br;
    rb = *reinterpret_cast<const f4*>(Y + static_cast<size_t>(vpix[kb]) * kpad + n0 + bc);
    // pixels past this split's end belong to the next split: zero their A values
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (ka + q >= kend) ra[q] = 0.f;
  };
  if (ksteps > 0) gload(kbeg);
  for (int s = 0; s < ksteps; ++s) {
    const int buf = s & 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) As[buf][lr][lk + q] = ra[q];
    *reinterpret_cast<f4*>(&Bs[buf][br][bc]) = rb;
    __syncthreads();
    if (s + 1 < ksteps) gload(kbeg + (s + 1) * 16);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[buf][wm + 16 * i + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[buf][4 * kk + (lane >> 4)][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma4(a[i], b[j], acc[i][j]);
    }
  }
  float* out = part + static_cast<size_t>(split) * nf * kpad;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int c = n0 + wn + 16 * j + (lane & 15);
        if (f < nf) out[static_cast<size_t>(f) * kpad + c] = acc[i][j][r];
      }
}

// grad[f][c] = sum_s part[s][f][c] for c < nm, fixed order over s.
__global__ void __launch_bounds__(256)
k_reduce_splits(int nsplit, int nf, int nm, int kpad, const float* __restrict__ part,
                float* __restrict__ grad) {
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<long>(nf) * nm) return;
  const int f = static_cast<int>(idx / nm), c = static_cast<int>(idx - static_cast<long>(f) * nm);
  float s = 0.f;
  for (int q = 0; q < nsplit; ++q) s += part[(static_cast<size_t>(q) * nf + f) * kpad + c];
  grad[idx] = s;
}

void launch_synth_fwd_bf16x3(const vis_field* f, const float* alm, float* img, hipStream_t st);
void launch_synth_adj_bf16x3(const vis_field* f, const float* dimg, int kps, hipStream_t st);

void launch_synth_fwd(const vis_field* f, const float* alm, float* img, hipStream_t st) {
  if (f->precision == VIS_BF16X3) {
    launch_synth_fwd_bf16x3(f, alm, img, st);
    return;
  }
  const vis_basis* b = f->basis;
  BV_REQUIRE(b->y32 != nullptr, VIS_EINVAL, "basis has no FP32 storage");
  const int nsplit = f->fsplit;
  const int kps = static_cast<int>(round_up(ceil_div(f->n_modes, nsplit), 32));
  dim3 grid(f->nv_pad / 64, ceil_div(f->n_freq, 64), nsplit);
  {
    ProfScope ps(&f->prof, "k_synth_fwd_f32", st);
    k_synth_fwd_f32<<<grid, 256, 0, st>>>(f->n_freq, f->n_modes, f->nv_pad, b->kpad, kps, alm,
                                           b->y32, f->tab.vpix, f->scr.a_part);
    check_launch("k_synth_fwd_f32");
  }
  const long n = static_cast<long>(f->n_freq) * f->nv_pad;
  ProfScope ps(&f->prof, "k_sum_fwd_splits", st);
  k_sum_fwd_splits<<<ceil_div(n, 256), 256, 0, st>>>(nsplit, n, f->scr.a_part, img);
  check_launch("k_sum_fwd_splits");
}

void launch_synth_adj(const vis_field* f, const float* dimg, float* grad_alm, hipStream_t st) {
  const vis_basis* b = f->basis;
  const int nsplit = f->asplit;
  if (f->precision == VIS_BF16X3) {
    const int kps = static_cast<int>(round_up(ceil_div(f->nv_pad, nsplit), 32));
    launch_synth_adj_bf16x3(f, dimg, kps, st);
  } else {
  BV_REQUIRE(b->y32 != nullptr, VIS_EINVAL, "basis has no FP32 storage");
  const int kps = static_cast<int>(round_up(ceil_div(f->nv_pad, nsplit), 16));
  const int ncol = static_cast<int>(round_up(f->n_modes, 64));
  dim3 grid(ncol / 64, ceil_div(f->n_freq, 64), nsplit);
  ProfScope ps(&f->prof, "k_synth_adj_f32", st);
  k_synth_adj_f32<<<grid, 256, 0, st>>>(f->n_freq, f->nv_pad, b->kpad, kps, dimg, b->y32,
                                         f->tab.vpix, f->scr.a_part);
  check_launch("k_synth_adj_f32");
  }
  const long n = static_cast<long>(f->n_freq) * f->n_modes;
  ProfScope ps(&f->prof, "k_reduce_splits", st);
  k_reduce_splits<<<ceil_div(n, 256), 256, 0, st>>>(nsplit, f->n_freq, f->n_modes, b->kpad,
                                                     f->scr.a_part, grad_alm);
  check_launch("k_reduce_splits");
}

}  // namespace bv
