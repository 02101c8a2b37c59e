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
#include "batch.hpp"
#include "objects.hpp"

namespace bv {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// apad[f][c] = alm[f][c] for f < nf, c < nm, else 0 (rows of kpad floats,
// 64 rows per 64-row tile), so the GEMMs load aligned, unconditional vectors.
struct PadAlmArgs {
  int nf;
  int nm;
  int kpad;
  int nrows;
  const float* alm;
  float* apad;
};

struct KPadAlm {
  using Args = PadAlmArgs;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const PadAlmArgs& args_, const Blk& B_);
};

__device__ void KPadAlm::run(const PadAlmArgs& args_, const Blk& B_) {
  int nf = args_.nf;
  int nm = args_.nm;
  int kpad = args_.kpad;
  int nrows = args_.nrows;
  const float* __restrict__ alm = args_.alm;
  float* __restrict__ apad = args_.apad;

  const long idx = static_cast<long>(B_.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<long>(nrows) * kpad) return;
  const int f = static_cast<int>(idx / kpad), c = static_cast<int>(idx - static_cast<long>(f) * kpad);
  apad[idx] = (f < nf && c < nm) ? alm[static_cast<size_t>(f) * nm + c] : 0.f;
}

void pad_alm(const vis_field* f, const float* alm, hipStream_t st) {
  const int kpad = f->basis->kpad;
  const int nrows = static_cast<int>(round_up(f->n_freq, 64));
  const long n = static_cast<long>(nrows) * kpad;
  ProfScope ps(&f->prof, "k_pad_alm", st);
  launch_k<KPadAlm>(ceil_div(n, 256), 0, PadAlmArgs{f->n_freq, f->n_modes, kpad, nrows, alm, f->scr.apad}, st, "k_pad_alm");
}

// part[s][f][k] = sum_{c in split s, c < nm} alm[f][c] Y[vpix[k]][c]
// Block tile 64 (f) x 64 (k), K step 32, 4 waves as 2 x 2 sub-tiles of 32 x 32;
// the mode range is split over blockIdx.z and the splits are summed in a
// fixed order afterwards.  Three-stage pipeline: step t is computed from LDS
// buffer t % 3 while step t+1 is stored into the next buffer and step t+3 is
// being fetched into registers, so two compute phases cover each load.
struct SynthFwdF32Args {
  int nf;
  int nm;
  int nvp;
  int kpad;
  int kps;
  const float* apad;
  const float* Y;
  const int* vpix;
  float* part;
};

struct KSynthFwdF32 {
  using Args = SynthFwdF32Args;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const SynthFwdF32Args& args_, const Blk& B_);
};

__device__ void KSynthFwdF32::run(const SynthFwdF32Args& args_, const Blk& B_) {
  int nf = args_.nf;
  int nm = args_.nm;
  int nvp = args_.nvp;
  int kpad = args_.kpad;
  int kps = args_.kps;
  const float* __restrict__ apad = args_.apad;
  const float* __restrict__ Y = args_.Y;
  const int* __restrict__ vpix = args_.vpix;
  float* __restrict__ part = args_.part;

  // pitch 34: the operand reads (16 rows x 4 columns per instruction) land on
  // 2 row + column, distinct over each half-wavefront
  __shared__ __attribute__((aligned(16))) float As[3][64][34];
  __shared__ __attribute__((aligned(16))) float Bs[3][64][34];
  typedef float f2 __attribute__((ext_vector_type(2)));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = B_.x * 64, m0 = B_.y * 64, split = B_.z;
  const int kbeg = split * kps, kend = min(nm, kbeg + kps);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  const int arow = m0 + lr;
  const float* yrow = Y + static_cast<size_t>(vpix[n0 + lr]) * kpad;
  const float* arow_p = apad + static_cast<size_t>(arow) * kpad;   // padded rows: always in range
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  f4 ra[3][2];
  f4 rb[3][2];
  const int ksteps = (kend - kbeg + 31) / 32;
  // modes in [kend, next split) belong to the next split: zero them in A
  auto gload = [&](int t, f4 (&a)[2], f4 (&b)[2]) {
    const int kk = kbeg + 32 * min(t, ksteps - 1) + lk;
    a[0] = *reinterpret_cast<const f4*>(arow_p + kk);
    a[1] = *reinterpret_cast<const f4*>(arow_p + kk + 4);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[0][q] = kk + q < kend ? a[0][q] : 0.f;
      a[1][q] = kk + 4 + q < kend ? a[1][q] : 0.f;
    }
    b[0] = *reinterpret_cast<const f4*>(yrow + kk);
    b[1] = *reinterpret_cast<const f4*>(yrow + kk + 4);
  };
  auto store = [&](int buf, const f4 (&a)[2], const f4 (&b)[2]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f4& u = a[q >> 1];
      *reinterpret_cast<f2*>(&As[buf][lr][lk + 2 * q]) = f2{u[2 * (q & 1)], u[2 * (q & 1) + 1]};
      const f4& v = b[q >> 1];
      *reinterpret_cast<f2*>(&Bs[buf][lr][lk + 2 * q]) = f2{v[2 * (q & 1)], v[2 * (q & 1) + 1]};
    }
  };
  auto compute = [&](int buf) {
    float av[8][2], bv[8][2];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
#pragma unroll
      for (int i = 0; i < 2; ++i) av[kk][i] = As[buf][wm + 16 * i + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[kk][j] = Bs[buf][wn + 16 * j + (lane & 15)][4 * kk + (lane >> 4)];
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma4(av[kk][i], bv[kk][j], acc[i][j]);
  };
  // stage t: store step t+1 (fetched at stage t-2), sync, fetch step t+3, compute step t
  auto stage = [&](int t, int cur, int nxt) {
    if (t + 1 < ksteps) store(nxt, ra[nxt], rb[nxt]);
    __syncthreads();
    if (t + 3 < ksteps) gload(t + 3, ra[cur], rb[cur]);
    compute(cur);
  };
  if (ksteps > 0) {
    gload(0, ra[0], rb[0]);
    gload(1, ra[1], rb[1]);
    gload(2, ra[2], rb[2]);
    store(0, ra[0], rb[0]);
    for (int t = 0; t < ksteps; t += 3) {
      stage(t, 0, 1);
      if (t + 1 < ksteps) stage(t + 1, 1, 2);
      if (t + 2 < ksteps) stage(t + 2, 2, 0);
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
struct SumFwdSplitsArgs {
  int nsplit;
  long n;
  const float* part;
  float* img;
};

struct KSumFwdSplits {
  using Args = SumFwdSplitsArgs;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const SumFwdSplitsArgs& args_, const Blk& B_);
};

__device__ void KSumFwdSplits::run(const SumFwdSplitsArgs& args_, const Blk& B_) {
  int nsplit = args_.nsplit;
  long n = args_.n;
  const float* __restrict__ part = args_.part;
  float* __restrict__ img = args_.img;

  const long idx = static_cast<long>(B_.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  float s = 0.f;
  for (int q = 0; q < nsplit; ++q) s += part[q * n + idx];
  img[idx] = s;
}

// part[s][f][c] = sum_{k in split s} dimg[f][k] Y[vpix[k]][c]
// Block tile 64 (f) x 64 (c), K step 16 pixels, three-stage pipeline as in
// the forward.
struct SynthAdjF32Args {
  int nf;
  int nvp;
  int kpad;
  int kps;
  const float* dimg;
  const float* Y;
  const int* vpix;
  float* part;
};

struct KSynthAdjF32 {
  using Args = SynthAdjF32Args;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const SynthAdjF32Args& args_, const Blk& B_);
};

__device__ void KSynthAdjF32::run(const SynthAdjF32Args& args_, const Blk& B_) {
  int nf = args_.nf;
  int nvp = args_.nvp;
  int kpad = args_.kpad;
  int kps = args_.kps;
  const float* __restrict__ dimg = args_.dimg;
  const float* __restrict__ Y = args_.Y;
  const int* __restrict__ vpix = args_.vpix;
  float* __restrict__ part = args_.part;

  __shared__ __attribute__((aligned(16))) float As[3][64][18];
  __shared__ __attribute__((aligned(16))) float Bs[3][16][80];
  typedef float f2 __attribute__((ext_vector_type(2)));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = B_.x * 64, m0 = B_.y * 64, split = B_.z;
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
  f4 ra[3], rb[3];
  const int ksteps = (kend - kbeg + 15) / 16;
  auto gload = [&](int t, f4& a, f4& b) {
    const int k0 = kbeg + 16 * t;
    const int ka = k0 + lk;
    a = (t < ksteps && arow < nf)
            ? *reinterpret_cast<const f4*>(dimg + static_cast<size_t>(arow) * nvp + ka)
            : f4{0.f, 0.f, 0.f, 0.f};
    const int kb = t < ksteps ? k0 + br : kbeg + br;
    b = *reinterpret_cast<const f4*>(Y + static_cast<size_t>(vpix[kb]) * kpad + n0 + bc);
  };
  auto store = [&](int buf, const f4& a, const f4& b) {
    *reinterpret_cast<f2*>(&As[buf][lr][lk]) = f2{a[0], a[1]};
    *reinterpret_cast<f2*>(&As[buf][lr][lk + 2]) = f2{a[2], a[3]};
    *reinterpret_cast<f4*>(&Bs[buf][br][bc]) = b;
  };
  auto compute = [&](int buf) {
    float av[4][2], bv[4][2];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
#pragma unroll
      for (int i = 0; i < 2; ++i) av[kk][i] = As[buf][wm + 16 * i + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[kk][j] = Bs[buf][4 * kk + (lane >> 4)][wn + 16 * j + (lane & 15)];
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma4(av[kk][i], bv[kk][j], acc[i][j]);
  };
  auto stage = [&](int t, int cur, int nxt) {
    if (t + 1 < ksteps) store(nxt, ra[nxt], rb[nxt]);
    __syncthreads();
    if (t + 3 < ksteps) gload(t + 3, ra[cur], rb[cur]);
    compute(cur);
  };
  if (ksteps > 0) {
    gload(0, ra[0], rb[0]);
    gload(1, ra[1], rb[1]);
    gload(2, ra[2], rb[2]);
    store(0, ra[0], rb[0]);
    for (int t = 0; t < ksteps; t += 3) {
      stage(t, 0, 1);
      if (t + 1 < ksteps) stage(t + 1, 1, 2);
      if (t + 2 < ksteps) stage(t + 2, 2, 0);
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
struct ReduceSplitsArgs {
  int nsplit;
  int nf;
  int nm;
  int kpad;
  const float* part;
  float* grad;
};

struct KReduceSplits {
  using Args = ReduceSplitsArgs;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const ReduceSplitsArgs& args_, const Blk& B_);
};

__device__ void KReduceSplits::run(const ReduceSplitsArgs& args_, const Blk& B_) {
  int nsplit = args_.nsplit;
  int nf = args_.nf;
  int nm = args_.nm;
  int kpad = args_.kpad;
  const float* __restrict__ part = args_.part;
  float* __restrict__ grad = args_.grad;

  const long idx = static_cast<long>(B_.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<long>(nf) * nm) return;
  const int f = static_cast<int>(idx / nm), c = static_cast<int>(idx - static_cast<long>(f) * nm);
  float s = 0.f;
  for (int q = 0; q < nsplit; ++q) s += part[(static_cast<size_t>(q) * nf + f) * kpad + c];
  grad[idx] = s;
}

void launch_synth_fwd_split(const vis_field* f, const float* alm, float* dst, int nsplit, int kps,
                            hipStream_t st);
void launch_synth_adj_split(const vis_field* f, const float* dimg, int kps, hipStream_t st);
void launch_synth_fwd_sep(const vis_field* f, const float* alm, float* img, hipStream_t st);
void launch_synth_adj_sep(const vis_field* f, float* grad_alm, hipStream_t st);

void launch_synth_fwd(const vis_field* f, const float* alm, float* img, hipStream_t st) {
  if (f->synthesis == VIS_SYNTH_SEPARABLE) {
    launch_synth_fwd_sep(f, alm, img, st);
    return;
  }
  const vis_basis* b = f->basis;
  const int nsplit = f->fsplit;
  const int kps = static_cast<int>(round_up(ceil_div(f->n_modes, nsplit), 32));
  float* dst = nsplit > 1 ? f->scr.a_part : img;
  if (f->precision == VIS_FP32) {
    BV_REQUIRE(b->y32 != nullptr, VIS_EINVAL, "basis has no FP32 storage");
    pad_alm(f, alm, st);
    dim3 grid(f->nv_pad / 64, ceil_div(f->n_freq, 64), nsplit);
    ProfScope ps(&f->prof, "k_synth_fwd_f32", st);
    launch_k<KSynthFwdF32>(grid, 0, SynthFwdF32Args{f->n_freq, f->n_modes, f->nv_pad, b->kpad, kps,
                                           f->scr.apad, b->y32, f->tab.vpix, dst}, st, "k_synth_fwd_f32");
  } else {
    launch_synth_fwd_split(f, alm, dst, nsplit, kps, st);
  }
  if (nsplit > 1) {
    const long n = static_cast<long>(f->n_freq) * f->nv_pad;
    ProfScope ps(&f->prof, "k_sum_fwd_splits", st);
    launch_k<KSumFwdSplits>(ceil_div(n, 256), 0, SumFwdSplitsArgs{nsplit, n, f->scr.a_part, img}, st, "k_sum_fwd_splits");
  }
}

void launch_synth_adj(const vis_field* f, const float* dimg, float* grad_alm, hipStream_t st) {
  if (f->synthesis == VIS_SYNTH_SEPARABLE) {
    BV_REQUIRE(dimg == nullptr, VIS_EINVAL, "internal: separable synthesis adjoint reads the full-grid scratch");
    launch_synth_adj_sep(f, grad_alm, st);
    return;
  }
  BV_REQUIRE(dimg != nullptr, VIS_EINVAL, "internal: dense synthesis adjoint without dL/dI");
  const vis_basis* b = f->basis;
  const int nsplit = f->asplit;
  if (f->precision != VIS_FP32) {
    const int kps = static_cast<int>(round_up(ceil_div(f->nv_pad, nsplit), 32));
    launch_synth_adj_split(f, dimg, kps, st);
  } else {
    BV_REQUIRE(b->y32 != nullptr, VIS_EINVAL, "basis has no FP32 storage");
    const int kps = static_cast<int>(round_up(ceil_div(f->nv_pad, nsplit), 16));
    const int ncol = static_cast<int>(round_up(f->n_modes, 64));
    dim3 grid(ncol / 64, ceil_div(f->n_freq, 64), nsplit);
    ProfScope ps(&f->prof, "k_synth_adj_f32", st);
    launch_k<KSynthAdjF32>(grid, 0, SynthAdjF32Args{f->n_freq, f->nv_pad, b->kpad, kps, dimg, b->y32,
                                           f->tab.vpix, f->scr.a_part}, st, "k_synth_adj_f32");
  }
  const long n = static_cast<long>(f->n_freq) * f->n_modes;
  ProfScope ps(&f->prof, "k_reduce_splits", st);
  launch_k<KReduceSplits>(ceil_div(n, 256), 0, ReduceSplitsArgs{nsplit, f->n_freq, f->n_modes, b->kpad,
                                                     f->scr.a_part, grad_alm}, st, "k_reduce_splits");
}

}  // namespace bv
