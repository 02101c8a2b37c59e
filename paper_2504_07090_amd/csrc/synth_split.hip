// Sky synthesis on bf16 MFMA with hi/lo split operands ("bf16x3").
//
// Each FP32 operand x is carried as hi = bf16(x), lo = bf16(x - hi), so
// x = hi + lo to about 2^-16 relative.  A product is taken as
//     a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
// (the dropped a_lo b_lo term is ~2^-16 relative), three bf16 MFMAs
// accumulating in FP32.  Y is stored pre-split in HBM (2 + 2 bytes per
// element, the same bytes as FP32); the sky coefficients and dL/dI are split
// on the fly while staging tiles into LDS.
//
// v_mfma_f32_16x16x32_bf16: lane l holds A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j = 0..7; D as for the other 16x16 MFMAs.
#include "objects.hpp"

namespace bv {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4 mfma_bf(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Round-to-nearest-even FP32 -> bf16 bit pattern (finite inputs).
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  const unsigned u = __float_as_uint(x);
  const unsigned r = u + 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<unsigned short>(r >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short b) {
  return __uint_as_float(static_cast<unsigned>(b) << 16);
}
__device__ __forceinline__ void split2(float x, unsigned short& hi, unsigned short& lo) {
  hi = bf16_bits(x);
  lo = bf16_bits(x - bf16_val(hi));
}

constexpr int kBP = 40;  // LDS pitch (bf16 elements) of a 32-wide K tile: 80 bytes

__device__ __forceinline__ bf8 ld8(const unsigned short* p) {
  const us8 v = *reinterpret_cast<const us8*>(p);
  return __builtin_bit_cast(bf8, v);
}

// img[f][k] = sum_{c < nm} alm[f][c] Y[vpix[k]][c]; tile 64 (f) x 64 (k), K step 32.
__global__ void __launch_bounds__(256)
k_synth_fwd_bf16x3(int nf, int nm, int nvp, int kpad, const float* __restrict__ apad,
                   const unsigned short* __restrict__ Yh, const unsigned short* __restrict__ Yl,
                   const int* __restrict__ vpix, float* __restrict__ img) {
  __shared__ __attribute__((aligned(16))) unsigned short Ah[2][64 * kBP], Al[2][64 * kBP];
  __shared__ __attribute__((aligned(16))) unsigned short Bh[2][64 * kBP], Bl[2][64 * kBP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = blockIdx.x * 64, m0 = blockIdx.y * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  const int arow = m0 + lr;
  const float* ap = apad + static_cast<size_t>(arow) * kpad;   // zero-padded rows
  const size_t yoff = static_cast<size_t>(vpix[n0 + lr]) * kpad;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  float ra[8];
  us8 rbh, rbl;
  const int ksteps = (nm + 31) / 32;
  auto gload = [&](int k0) {
    const f4 u = *reinterpret_cast<const f4*>(ap + k0 + lk);
    const f4 v = *reinterpret_cast<const f4*>(ap + k0 + lk + 4);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ra[q] = u[q];
      ra[4 + q] = v[q];
    }
    rbh = *reinterpret_cast<const us8*>(Yh + yoff + k0 + lk);
    rbl = *reinterpret_cast<const us8*>(Yl + yoff + k0 + lk);
  };
  gload(0);
  for (int s = 0; s < ksteps; ++s) {
    const int buf = s & 1;
    us8 h, l;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      unsigned short a, b;
      split2(ra[q], a, b);
      h[q] = a;
      l[q] = b;
    }
    *reinterpret_cast<us8*>(&Ah[buf][lr * kBP + lk]) = h;
    *reinterpret_cast<us8*>(&Al[buf][lr * kBP + lk]) = l;
    *reinterpret_cast<us8*>(&Bh[buf][lr * kBP + lk]) = rbh;
    *reinterpret_cast<us8*>(&Bl[buf][lr * kBP + lk]) = rbl;
    __syncthreads();
    if (s + 1 < ksteps) gload((s + 1) * 32);
    bf8 ah[2], al[2], bh[2], bl[2];
    const int ko = 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ah[i] = ld8(&Ah[buf][(wm + 16 * i + (lane & 15)) * kBP + ko]);
      al[i] = ld8(&Al[buf][(wm + 16 * i + (lane & 15)) * kBP + ko]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      bh[j] = ld8(&Bh[buf][(wn + 16 * j + (lane & 15)) * kBP + ko]);
      bl[j] = ld8(&Bl[buf][(wn + 16 * j + (lane & 15)) * kBP + ko]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = mfma_bf(al[i], bh[j], acc[i][j]);
        acc[i][j] = mfma_bf(ah[i], bl[j], acc[i][j]);
        acc[i][j] = mfma_bf(ah[i], bh[j], acc[i][j]);
      }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int k = n0 + wn + 16 * j + (lane & 15);
        if (f < nf) img[static_cast<size_t>(f) * nvp + k] = acc[i][j][r];
      }
}

// part[s][f][c] = sum_{k in split s} dimg[f][k] Y[vpix[k]][c]; tile 64 (f) x 64 (c), K step 32.
__global__ void __launch_bounds__(256)
k_synth_adj_bf16x3(int nf, int nvp, int kpad, int kps, const float* __restrict__ dimg,
                   const unsigned short* __restrict__ Yh, const unsigned short* __restrict__ Yl,
                   const int* __restrict__ vpix, float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) unsigned short Ah[2][64 * kBP], Al[2][64 * kBP];
  __shared__ __attribute__((aligned(16))) unsigned short Bh[2][64 * kBP], Bl[2][64 * kBP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = blockIdx.x * 64, m0 = blockIdx.y * 64, split = blockIdx.z;
  const int kbeg = split * kps, kend = min(nvp, kbeg + kps);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = tid >> 2, lk = (tid & 3) * 8;      // A: row f, 8 pixels
  const int kr = tid >> 3, cg = (tid & 7) * 8;      // B: pixel row, 8 modes
  const int arow = m0 + lr;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  f4 ra0, ra1;
  us8 rbh, rbl;
  const int ksteps = (kend - kbeg + 31) / 32;
  auto gload = [&](int k0) {
    const int ka = k0 + lk;
    if (arow < nf) {
      const float* p = dimg + static_cast<size_t>(arow) * nvp + ka;
      ra0 = *reinterpret_cast<const f4*>(p);
      ra1 = *reinterpret_cast<const f4*>(p + 4);
    } else {
      ra0 = ra1 = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (ka + q >= kend) ra0[q] = 0.f;
      if (ka + 4 + q >= kend) ra1[q] = 0.f;
    }
    const int kb = min(k0 + kr, nvp - 1);
    const size_t yo = static_cast<size_t>(vpix[kb]) * kpad + n0 + cg;
    rbh = *reinterpret_cast<const us8*>(Yh + yo);
    rbl = *reinterpret_cast<const us8*>(Yl + yo);
  };
  if (ksteps > 0) gload(kbeg);
  for (int s = 0; s < ksteps; ++s) {
    const int buf = s & 1;
    us8 h, l;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      unsigned short a, b;
      split2(ra0[q], a, b);
      h[q] = a;
      l[q] = b;
      split2(ra1[q], a, b);
      h[4 + q] = a;
      l[4 + q] = b;
    }
    *reinterpret_cast<us8*>(&Ah[buf][lr * kBP + lk]) = h;
    *reinterpret_cast<us8*>(&Al[buf][lr * kBP + lk]) = l;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      Bh[buf][(cg + q) * kBP + kr] = rbh[q];
      Bl[buf][(cg + q) * kBP + kr] = rbl[q];
    }
    __syncthreads();
    if (s + 1 < ksteps) gload(kbeg + (s + 1) * 32);
    bf8 ah[2], al[2], bh[2], bl[2];
    const int ko = 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ah[i] = ld8(&Ah[buf][(wm + 16 * i + (lane & 15)) * kBP + ko]);
      al[i] = ld8(&Al[buf][(wm + 16 * i + (lane & 15)) * kBP + ko]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      bh[j] = ld8(&Bh[buf][(wn + 16 * j + (lane & 15)) * kBP + ko]);
      bl[j] = ld8(&Bl[buf][(wn + 16 * j + (lane & 15)) * kBP + ko]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = mfma_bf(al[i], bh[j], acc[i][j]);
        acc[i][j] = mfma_bf(ah[i], bl[j], acc[i][j]);
        acc[i][j] = mfma_bf(ah[i], bh[j], acc[i][j]);
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

void launch_synth_fwd_bf16x3(const vis_field* f, const float* apad, float* img, hipStream_t st) {
  const vis_basis* b = f->basis;
  BV_REQUIRE(b->ybh != nullptr, VIS_EINVAL, "basis has no bf16 split storage");
  dim3 grid(f->nv_pad / 64, ceil_div(f->n_freq, 64));
  ProfScope ps(&f->prof, "k_synth_fwd_bf16x3", st);
  k_synth_fwd_bf16x3<<<grid, 256, 0, st>>>(
      f->n_freq, f->n_modes, f->nv_pad, b->kpad, apad, reinterpret_cast<const unsigned short*>(b->ybh),
      reinterpret_cast<const unsigned short*>(b->ybl), f->tab.vpix, img);
  check_launch("k_synth_fwd_bf16x3");
}

void launch_synth_adj_bf16x3(const vis_field* f, const float* dimg, int kps, hipStream_t st) {
  const vis_basis* b = f->basis;
  BV_REQUIRE(b->ybh != nullptr, VIS_EINVAL, "basis has no bf16 split storage");
  const int ncol = static_cast<int>(round_up(f->n_modes, 64));
  dim3 grid(ncol / 64, ceil_div(f->n_freq, 64), f->asplit);
  ProfScope ps(&f->prof, "k_synth_adj_bf16x3", st);
  k_synth_adj_bf16x3<<<grid, 256, 0, st>>>(
      f->n_freq, f->nv_pad, b->kpad, kps, dimg, reinterpret_cast<const unsigned short*>(b->ybh),
      reinterpret_cast<const unsigned short*>(b->ybl), f->tab.vpix, f->scr.a_part);
  check_launch("k_synth_adj_bf16x3");
}

}  // namespace bv
