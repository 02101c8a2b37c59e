// Sky synthesis on 16-bit MFMA with hi/lo split operands ("bf16x3", "fp16x3").
//
// Each FP32 operand x is carried as two 16-bit numbers,
//     bf16x3:  hi = bf16(x),      lo = bf16(x - hi)             (x = hi + lo),
//     fp16x3:  hi = fp16(x s),    lo = fp16((x s - hi) 2^11)    (x s = hi + lo 2^-11),
// where for fp16 (five exponent bits) every operand row is first multiplied
// by a power of two s that puts its largest magnitude in [2^13, 2^14); bf16
// has the FP32 exponent range and needs no scale (s = 1).  A product then
// takes three MFMAs accumulating in FP32,
//     x y s ~ hi_x hi_y + L (hi_x lo_y + lo_x hi_y),   L = 1 (bf16), 2^-11 (fp16),
// with the two groups in separate accumulators; the dropped lo_x lo_y term is
// ~2^-16 (bf16) or ~2^-22 (fp16) relative.  The row scale is removed exactly
// when the tile is written.  Y is stored split the same way by the basis
// generator (unscaled: its entries are bounded by ~3); the sky coefficients
// (forward) and dL/dI (adjoint) are split once per call into scratch rows, so
// the GEMM tiles stream 16-bit operands straight into LDS.
//
// v_mfma_f32_16x16x32_{bf16,f16}: lane l holds A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j = 0..7; D as for the other 16x16 MFMAs.
#include "batch.hpp"
#include "objects.hpp"

namespace bv {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

struct Bf16Split {
  static constexpr bool kScaled = false;
  static constexpr float kLo = 1.0f;       // lo carries the residual itself
  __device__ static f4 mma(us8 a, us8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                   __builtin_bit_cast(bf8, b), c, 0, 0, 0);
  }
  // round-to-nearest-even FP32 -> bf16 (finite inputs)
  __device__ static unsigned short bits(float x) {
    const unsigned u = __float_as_uint(x);
    return static_cast<unsigned short>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
  }
  __device__ static void split(float x, unsigned short& hi, unsigned short& lo) {
    hi = bits(x);
    lo = bits(x - __uint_as_float(static_cast<unsigned>(hi) << 16));
  }
};

struct F16Split {
  static constexpr bool kScaled = true;
  static constexpr float kLo = 2048.0f;    // lo carries 2^11 times the residual
  __device__ static f4 mma(us8 a, us8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a),
                                                  __builtin_bit_cast(h8, b), c, 0, 0, 0);
  }
  __device__ static void split(float x, unsigned short& hi, unsigned short& lo) {
    const _Float16 h = static_cast<_Float16>(x);
    const _Float16 l = static_cast<_Float16>((x - static_cast<float>(h)) * kLo);
    hi = __builtin_bit_cast(unsigned short, h);
    lo = __builtin_bit_cast(unsigned short, l);
  }
};

constexpr int kSplitCols = 2048;   // columns per block in the row-split kernels
constexpr int kHP = 40;            // LDS pitch (16-bit elements) of a 32-wide K tile

// pmax[r][ch] = max |src[r][c]| over the ch-th block of kSplitCols columns.
struct RowAbsmaxArgs {
  int ncols;
  int ld;
  const float* src;
  float* pmax;
};

struct KRowAbsmax {
  using Args = RowAbsmaxArgs;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const RowAbsmaxArgs& args_, const Blk& B_);
};

__device__ void KRowAbsmax::run(const RowAbsmaxArgs& args_, const Blk& B_) {
  int ncols = args_.ncols;
  int ld = args_.ld;
  const float* __restrict__ src = args_.src;
  float* __restrict__ pmax = args_.pmax;

  __shared__ float red[4];
  const int ch = B_.x, r = B_.y, tid = threadIdx.x;
  const float* row = src + static_cast<size_t>(r) * ld;
  float m = 0.f;
  for (int c = ch * kSplitCols + tid; c < min(ncols, (ch + 1) * kSplitCols); c += 256)
    m = fmaxf(m, fabsf(row[c]));
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0)
    pmax[static_cast<size_t>(r) * B_.nx + ch] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// Rows r < nrows of src (ncols valid columns) -> hi/lo rows of ld_dst
// columns, zero beyond ncols and for rows nrows..gridDim.y-1; rscale[r] = 1/s.
struct SplitRowsArgs {
  int nrows;
  int ncols;
  int ld_src;
  int ld_dst;
  const float* src;
  const float* pmax;
  int nch;
  unsigned short* hi;
  unsigned short* lo;
  float* rscale;
};

template <class Fmt>
struct KSplitRows {
  using Args = SplitRowsArgs;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const SplitRowsArgs& args_, const Blk& B_);
};

template <class Fmt>
__device__ void KSplitRows<Fmt>::run(const SplitRowsArgs& args_, const Blk& B_) {
  int nrows = args_.nrows;
  int ncols = args_.ncols;
  int ld_src = args_.ld_src;
  int ld_dst = args_.ld_dst;
  const float* __restrict__ src = args_.src;
  const float* __restrict__ pmax = args_.pmax;
  int nch = args_.nch;
  unsigned short* __restrict__ hi = args_.hi;
  unsigned short* __restrict__ lo = args_.lo;
  float* __restrict__ rscale = args_.rscale;

  const int ch = B_.x, r = B_.y, tid = threadIdx.x;
  float s = 1.0f;
  if (Fmt::kScaled && r < nrows) {
    float m = 0.f;
    for (int q = 0; q < nch; ++q) m = fmaxf(m, pmax[static_cast<size_t>(r) * nch + q]);
    if (m > 0.f && m < 3.0e38f) {
      int e = 0;
      frexpf(m, &e);                        // m < 2^e
      s = ldexpf(1.0f, min(100, 14 - e));   // m s in [2^13, 2^14)
    }
  }
  const float* row = src + static_cast<size_t>(r) * ld_src;
  unsigned short* h = hi + static_cast<size_t>(r) * ld_dst;
  unsigned short* l = lo + static_cast<size_t>(r) * ld_dst;
  for (int c = ch * kSplitCols + tid; c < min(ld_dst, (ch + 1) * kSplitCols); c += 256) {
    const float x = (r < nrows && c < ncols) ? row[c] * s : 0.f;
    Fmt::split(x, h[c], l[c]);
  }
  if (ch == 0 && tid == 0) rscale[r] = 1.0f / s;
}

// part[split][f][k] = sum_{c in split} a[f][c] Y[vpix[k]][c]; tile 64 (f) x 64 (k),
// K step 32.  A: split coefficient rows [nf_pad][kpad], zero beyond the modes.
struct SynthFwdSplitArgs {
  int nf;
  int nm;
  int nvp;
  int kpad;
  int kps;
  const unsigned short* Ahg;
  const unsigned short* Alg;
  const float* rscale;
  const unsigned short* Yh;
  const unsigned short* Yl;
  const int* vpix;
  float* part;
};

template <class Fmt>
struct KSynthFwdSplit {
  using Args = SynthFwdSplitArgs;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const SynthFwdSplitArgs& args_, const Blk& B_);
};

template <class Fmt>
__device__ void KSynthFwdSplit<Fmt>::run(const SynthFwdSplitArgs& args_, const Blk& B_) {
  int nf = args_.nf;
  int nm = args_.nm;
  int nvp = args_.nvp;
  int kpad = args_.kpad;
  int kps = args_.kps;
  const unsigned short* __restrict__ Ahg = args_.Ahg;
  const unsigned short* __restrict__ Alg = args_.Alg;
  const float* __restrict__ rscale = args_.rscale;
  const unsigned short* __restrict__ Yh = args_.Yh;
  const unsigned short* __restrict__ Yl = args_.Yl;
  const int* __restrict__ vpix = args_.vpix;
  float* __restrict__ part = args_.part;

  __shared__ __attribute__((aligned(16))) unsigned short Ah[2][64 * kHP], Al[2][64 * kHP];
  __shared__ __attribute__((aligned(16))) unsigned short Bh[2][64 * kHP], Bl[2][64 * kHP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = B_.x * 64, m0 = B_.y * 64, split = B_.z;
  const int kbeg = split * kps, kend = min(nm, kbeg + kps);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  const size_t aoff = static_cast<size_t>(m0 + lr) * kpad;   // padded rows: in range
  const size_t yoff = static_cast<size_t>(vpix[n0 + lr]) * kpad;
  f4 c1[2][2], c2[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) c1[i][j] = c2[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  us8 rah, ral, rbh, rbl;
  // kbeg and kps are multiples of 32, so a step never reaches into the next
  // split, and the coefficient rows are zero past the last mode
  const int ksteps = (kend - kbeg + 31) / 32;
  auto gload = [&](int k0) {
    rah = *reinterpret_cast<const us8*>(Ahg + aoff + k0 + lk);
    ral = *reinterpret_cast<const us8*>(Alg + aoff + k0 + lk);
    rbh = *reinterpret_cast<const us8*>(Yh + yoff + k0 + lk);
    rbl = *reinterpret_cast<const us8*>(Yl + yoff + k0 + lk);
  };
  if (ksteps > 0) gload(kbeg);
  for (int s = 0; s < ksteps; ++s) {
    const int buf = s & 1;   // two buffers: the one written here was last read two steps ago
    *reinterpret_cast<us8*>(&Ah[buf][lr * kHP + lk]) = rah;
    *reinterpret_cast<us8*>(&Al[buf][lr * kHP + lk]) = ral;
    *reinterpret_cast<us8*>(&Bh[buf][lr * kHP + lk]) = rbh;
    *reinterpret_cast<us8*>(&Bl[buf][lr * kHP + lk]) = rbl;
    __syncthreads();
    if (s + 1 < ksteps) gload(kbeg + (s + 1) * 32);
    us8 ah[2], al[2], bh[2], bl[2];
    const int ko = 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ah[i] = *reinterpret_cast<const us8*>(&Ah[buf][(wm + 16 * i + (lane & 15)) * kHP + ko]);
      al[i] = *reinterpret_cast<const us8*>(&Al[buf][(wm + 16 * i + (lane & 15)) * kHP + ko]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      bh[j] = *reinterpret_cast<const us8*>(&Bh[buf][(wn + 16 * j + (lane & 15)) * kHP + ko]);
      bl[j] = *reinterpret_cast<const us8*>(&Bl[buf][(wn + 16 * j + (lane & 15)) * kHP + ko]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        c2[i][j] = Fmt::mma(al[i], bh[j], c2[i][j]);
        c2[i][j] = Fmt::mma(ah[i], bl[j], c2[i][j]);
        c1[i][j] = Fmt::mma(ah[i], bh[j], c1[i][j]);
      }
  }
  float* out = part + static_cast<size_t>(split) * nf * nvp;
  constexpr float inv = 1.0f / Fmt::kLo;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int k = n0 + wn + 16 * j + (lane & 15);
        if (f < nf) out[static_cast<size_t>(f) * nvp + k] = (c1[i][j][r] + c2[i][j][r] * inv) * rscale[f];
      }
}

// part[split][f][c] = sum_{k in split} dimg[f][k] Y[vpix[k]][c]; tile 64 (f) x 64 (c),
// K step 32.  A: split dL/dI rows [nf_pad][nvp].
struct SynthAdjSplitArgs {
  int nf;
  int nvp;
  int kpad;
  int kps;
  const unsigned short* Dh;
  const unsigned short* Dl;
  const float* rscale;
  const unsigned short* Yh;
  const unsigned short* Yl;
  const int* vpix;
  float* part;
};

template <class Fmt>
struct KSynthAdjSplit {
  using Args = SynthAdjSplitArgs;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const SynthAdjSplitArgs& args_, const Blk& B_);
};

template <class Fmt>
__device__ void KSynthAdjSplit<Fmt>::run(const SynthAdjSplitArgs& args_, const Blk& B_) {
  int nf = args_.nf;
  int nvp = args_.nvp;
  int kpad = args_.kpad;
  int kps = args_.kps;
  const unsigned short* __restrict__ Dh = args_.Dh;
  const unsigned short* __restrict__ Dl = args_.Dl;
  const float* __restrict__ rscale = args_.rscale;
  const unsigned short* __restrict__ Yh = args_.Yh;
  const unsigned short* __restrict__ Yl = args_.Yl;
  const int* __restrict__ vpix = args_.vpix;
  float* __restrict__ part = args_.part;

  __shared__ __attribute__((aligned(16))) unsigned short Ah[2][64 * kHP], Al[2][64 * kHP];
  __shared__ __attribute__((aligned(16))) unsigned short Bh[2][64 * kHP], Bl[2][64 * kHP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = B_.x * 64, m0 = B_.y * 64, split = B_.z;
  const int kbeg = split * kps, kend = min(nvp, kbeg + kps);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = tid >> 2, lk = (tid & 3) * 8;      // A: row f, 8 pixels
  const int pq = (tid >> 5) * 4, cp = (tid & 31) * 2;   // B: 4 pixel rows, 2 modes
  const size_t aoff = static_cast<size_t>(m0 + lr) * nvp;   // padded rows: in range
  f4 c1[2][2], c2[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) c1[i][j] = c2[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  us8 rah, ral;
  unsigned rbh[4], rbl[4];   // modes (cp, cp + 1) of pixel rows pq .. pq + 3
  // kbeg and kps are multiples of 32 and nvp of 64: steps stay inside the split
  const int ksteps = (kend - kbeg + 31) / 32;
  auto gload = [&](int k0) {
    rah = *reinterpret_cast<const us8*>(Dh + aoff + k0 + lk);
    ral = *reinterpret_cast<const us8*>(Dl + aoff + k0 + lk);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const size_t yo = static_cast<size_t>(vpix[k0 + pq + r]) * kpad + n0 + cp;
      rbh[r] = *reinterpret_cast<const unsigned*>(Yh + yo);
      rbl[r] = *reinterpret_cast<const unsigned*>(Yl + yo);
    }
  };
  // B tile transposed into [mode][pixel]: four pixels of one mode per 64-bit store
  auto bstore = [&](unsigned short* B, const unsigned (&v)[4]) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const u2 even = u2{(v[0] & 0xFFFFu) | (v[1] << 16), (v[2] & 0xFFFFu) | (v[3] << 16)};
    const u2 odd = u2{(v[0] >> 16) | (v[1] & 0xFFFF0000u), (v[2] >> 16) | (v[3] & 0xFFFF0000u)};
    *reinterpret_cast<u2*>(&B[cp * kHP + pq]) = even;
    *reinterpret_cast<u2*>(&B[(cp + 1) * kHP + pq]) = odd;
  };
  if (ksteps > 0) gload(kbeg);
  for (int s = 0; s < ksteps; ++s) {
    const int buf = s & 1;
    *reinterpret_cast<us8*>(&Ah[buf][lr * kHP + lk]) = rah;
    *reinterpret_cast<us8*>(&Al[buf][lr * kHP + lk]) = ral;
    bstore(Bh[buf], rbh);
    bstore(Bl[buf], rbl);
    __syncthreads();
    if (s + 1 < ksteps) gload(kbeg + (s + 1) * 32);
    us8 ah[2], al[2], bh[2], bl[2];
    const int ko = 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ah[i] = *reinterpret_cast<const us8*>(&Ah[buf][(wm + 16 * i + (lane & 15)) * kHP + ko]);
      al[i] = *reinterpret_cast<const us8*>(&Al[buf][(wm + 16 * i + (lane & 15)) * kHP + ko]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      bh[j] = *reinterpret_cast<const us8*>(&Bh[buf][(wn + 16 * j + (lane & 15)) * kHP + ko]);
      bl[j] = *reinterpret_cast<const us8*>(&Bl[buf][(wn + 16 * j + (lane & 15)) * kHP + ko]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        c2[i][j] = Fmt::mma(al[i], bh[j], c2[i][j]);
        c2[i][j] = Fmt::mma(ah[i], bl[j], c2[i][j]);
        c1[i][j] = Fmt::mma(ah[i], bh[j], c1[i][j]);
      }
  }
  float* out = part + static_cast<size_t>(split) * nf * kpad;
  constexpr float inv = 1.0f / Fmt::kLo;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int c = n0 + wn + 16 * j + (lane & 15);
        if (f < nf) out[static_cast<size_t>(f) * kpad + c] = (c1[i][j][r] + c2[i][j][r] * inv) * rscale[f];
      }
}

// ------------------------------------------------------------ launchers --
namespace {

struct SplitY {
  const unsigned short* hi;
  const unsigned short* lo;
};

SplitY split_basis(const vis_field* f) {
  const vis_basis* b = f->basis;
  if (f->precision == VIS_BF16X3) {
    BV_REQUIRE(b->ybh != nullptr, VIS_EINVAL, "basis has no bf16 split storage");
    return {reinterpret_cast<const unsigned short*>(b->ybh), reinterpret_cast<const unsigned short*>(b->ybl)};
  }
  BV_REQUIRE(b->yhh != nullptr, VIS_EINVAL, "basis has no fp16 split storage");
  return {reinterpret_cast<const unsigned short*>(b->yhh), reinterpret_cast<const unsigned short*>(b->yhl)};
}

// rows [n_freq][ncols] (stride ld_src) -> hi/lo planes [nf_pad][ld_dst], row scales
template <class Fmt>
void split_rows(const vis_field* f, int ncols, int ld_src, int ld_dst, const float* src,
                unsigned short* hi, unsigned short* lo, hipStream_t st) {
  const int nrows = f->n_freq, nrows_pad = static_cast<int>(round_up(nrows, 64));
  const int nch_src = ceil_div(ncols, kSplitCols);
  if (Fmt::kScaled) {
    ProfScope ps(&f->prof, "k_row_absmax", st);
    launch_k<KRowAbsmax>(dim3(nch_src, nrows), 0, RowAbsmaxArgs{ncols, ld_src, src, f->scr.rmax}, st, "k_row_absmax");
  }
  ProfScope ps(&f->prof, "k_split_rows", st);
  launch_k<KSplitRows<Fmt>>(dim3(ceil_div(ld_dst, kSplitCols), nrows_pad), 0, SplitRowsArgs{
      nrows, ncols, ld_src, ld_dst, src, f->scr.rmax, nch_src, hi, lo, f->scr.rscale}, st, "k_split_rows");
}

template <class Fmt>
void fwd_split(const vis_field* f, const float* alm, float* dst, int nsplit, int kps, hipStream_t st) {
  const vis_basis* b = f->basis;
  const SplitY y = split_basis(f);
  const size_t plane = round_up(f->n_freq, 64) * static_cast<size_t>(b->kpad);
  unsigned short* ah = reinterpret_cast<unsigned short*>(f->scr.apad);   // nf_pad x kpad floats
  unsigned short* al = ah + plane;
  split_rows<Fmt>(f, f->n_modes, f->n_modes, b->kpad, alm, ah, al, st);
  dim3 grid(f->nv_pad / 64, ceil_div(f->n_freq, 64), nsplit);
  ProfScope ps(&f->prof, Fmt::kScaled ? "k_synth_fwd_fp16x3" : "k_synth_fwd_bf16x3", st);
  launch_k<KSynthFwdSplit<Fmt>>(grid, 0, SynthFwdSplitArgs{f->n_freq, f->n_modes, f->nv_pad, b->kpad, kps, ah, al,
                                               f->scr.rscale, y.hi, y.lo, f->tab.vpix, dst}, st, "k_synth_fwd_split");
}

template <class Fmt>
void adj_split(const vis_field* f, const float* dimg, int kps, hipStream_t st) {
  const vis_basis* b = f->basis;
  const SplitY y = split_basis(f);
  const size_t plane = round_up(f->n_freq, 64) * static_cast<size_t>(f->nv_pad);
  unsigned short* dh = reinterpret_cast<unsigned short*>(f->scr.dsplit);   // nf_pad x nv_pad floats
  unsigned short* dl = dh + plane;
  split_rows<Fmt>(f, f->nv_pad, f->nv_pad, f->nv_pad, dimg, dh, dl, st);
  const int ncol = static_cast<int>(round_up(f->n_modes, 64));
  dim3 grid(ncol / 64, ceil_div(f->n_freq, 64), f->asplit);
  ProfScope ps(&f->prof, Fmt::kScaled ? "k_synth_adj_fp16x3" : "k_synth_adj_bf16x3", st);
  launch_k<KSynthAdjSplit<Fmt>>(grid, 0, SynthAdjSplitArgs{f->n_freq, f->nv_pad, b->kpad, kps, dh, dl,
                                               f->scr.rscale, y.hi, y.lo, f->tab.vpix, f->scr.a_part}, st, "k_synth_adj_split");
}

}  // namespace

// Forward split synthesis into dst: nsplit partial planes [nsplit][n_freq][nv_pad]
// of kps modes each (kps a multiple of 32); with nsplit == 1, dst is the sky itself.
void launch_synth_fwd_split(const vis_field* f, const float* alm, float* dst, int nsplit, int kps,
                            hipStream_t st) {
  if (f->precision == VIS_BF16X3) fwd_split<Bf16Split>(f, alm, dst, nsplit, kps, st);
  else fwd_split<F16Split>(f, alm, dst, nsplit, kps, st);
}

// Adjoint split synthesis into the split-K partials a_part[asplit][n_freq][kpad]
// (kps pixels each, a multiple of 32).
void launch_synth_adj_split(const vis_field* f, const float* dimg, int kps, hipStream_t st) {
  if (f->precision == VIS_BF16X3) adj_split<Bf16Split>(f, dimg, kps, st);
  else adj_split<F16Split>(f, dimg, kps, st);
}

}  // namespace bv
