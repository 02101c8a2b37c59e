// Separable sky synthesis on the RA x sin(dec) grid (Sec. 3.2, eq. fg_separable).
//
// Every pixel sits on a ring j (z_j = sin dec) and a column k (alpha_k), and
// the real harmonic factorises as Y(j, k; l, m) = lambda_l|m|(z_j) T_m(alpha_k)
// with T_0 = 1, T_m = sqrt 2 cos(m alpha), T_-m = sqrt 2 sin(m alpha).  Hence
//     I(j, k, nu) = sum_m T_m(alpha_k) G_m(j, nu),
//     G_m(j, nu)  = sum_{l >= |m|} lambda_l|m|(z_j) a_lm(nu),
// a Legendre stage (one GEMM per m: rings x l x channels) and an azimuthal
// stage (one GEMM per ring: columns x m x channels).  The adjoint runs the
// transposes in reverse order:
//     H_m(j, nu)   = sum_k T_m(alpha_k) dL/dI(j, k, nu),
//     dL/da_lm(nu) = sum_j lambda_l|m|(z_j) H_m(j, nu).
// At lmax 100 on 128 x 384 pixels and 64 channels this is ~0.7e9 MACs per
// direction against 1.7e10 for the dense product with the visible rows of Y,
// and the factor tables take ~3 MB instead of 2 GB.  The Legendre stages run
// every ring; the azimuthal stages run only the 32-column batches of a ring
// that hold a pixel above the horizon at some time.  The forward writes the
// visible pixels into the sky scratch; the adjoint reads dL/dI on the full
// grid, where the adjoint fringe pass writes it (zero at the other pixels).
//
// Every GEMM is a grid of 16 x 16 output tiles, one wavefront each, on
// v_mfma_f32_16x16x4_f32: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// D[i][j] in lane j + 16 (i / 4), register i % 4.  Operands come straight
// from the small, cache-resident tables; K is unrolled so the loads of
// several MFMAs are in flight together.  The azimuthal stages, whose K runs
// over 2 lmax + 1 or nphi, also issue the next batch's loads into a second
// register set before the current batch's MFMAs (the loop is unrolled by two so
// the sets swap roles without copies, and a scheduling barrier keeps the
// batch's loads together); those loads use indices clamped into the tables and
// are always issued (a load under a divergent branch is waited for where the
// branch ends), and terms past the end of K are removed by zeroing one operand
// at the MFMA.
#include "batch.hpp"
#include "objects.hpp"

namespace bv {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 sep_mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Blocks are dealt round-robin over the 8 XCDs (block b to XCD b % 8).  The
// block's linear index is mapped to a logical one such that each XCD runs one
// contiguous range of logical blocks (the tail that does not fill all eight
// keeps its index): a bijection on [0, blocks).  Each stage decodes the
// logical index with the blocks that share operand rows adjacent, so those
// rows come from one XCD's L2 instead of being fetched once per XCD (the
// forward Legendre stage keeps the launch order).
__device__ __forceinline__ int sep_xcd_logical(const Blk& B) {
  const int total = B.nx * B.ny * B.nz;
  const int b = B.x + B.nx * (B.y + B.ny * B.z);
  const int per = total / 8;
  return b >= 8 * per ? b : (b % 8) * per + b / 8;
}

// (x, y, z) block coordinates of logical block L with y and z fastest (the
// Legendre stages: every block of one m shares that m's table rows).
__device__ __forceinline__ int3 sep_blocks_m_major(int L, const Blk& B) {
  const int nyz = B.ny * B.nz, yz = L % nyz;
  return make_int3(L / nyz, yz % B.ny, yz / B.ny);
}

// (x, y, z) of logical block L with x fastest (the azimuthal stages: the
// column or c tiles of one ring and channel tile share that ring's rows).
__device__ __forceinline__ int3 sep_blocks_x_fastest(int L, const Blk& B) {
  const int yz = L / B.nx;
  return make_int3(L % B.nx, yz % B.ny, yz / B.ny);
}

constexpr int kSepBatch = 8;              // MFMAs whose operand loads are issued together
static_assert(kSepStep == 4 * kSepBatch, "K covered per batch");

// at[mode][nu] = a[nu][mode]: the sky coefficients transposed through a
// 16-mode x 64-channel LDS tile (one block per 16 modes, so the grid fills the
// chip), so the Legendre stage reads 16 channels of one mode as one 64-byte
// segment.
constexpr int kTrModes = 16, kTrChans = 64;
struct AlmTransposeArgs {
  int nf;
  int nm;
  const float* a;
  float* at;
};

struct KAlmTranspose {
  using Args = AlmTransposeArgs;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const AlmTransposeArgs& args_, const Blk& B_);
};

__device__ void KAlmTranspose::run(const AlmTransposeArgs& args_, const Blk& B_) {
  int nf = args_.nf;
  int nm = args_.nm;
  const float* __restrict__ a = args_.a;
  float* __restrict__ at = args_.at;

  __shared__ float tile[kTrChans][kTrModes + 1];
  const int m0 = B_.x * kTrModes;
  const int t = threadIdx.x;
  for (int f0 = 0; f0 < nf; f0 += kTrChans) {
    // read: 16 consecutive modes of 16 channel rows per pass
    for (int e = t; e < kTrChans * kTrModes; e += 256) {
      const int r = e / kTrModes, c = e % kTrModes;
      const int f = f0 + r, m = m0 + c;
      tile[r][c] = (f < nf && m < nm) ? a[static_cast<size_t>(f) * nm + m] : 0.f;
    }
    __syncthreads();
    // write: 64 consecutive channels of 4 mode rows per pass
    for (int e = t; e < kTrChans * kTrModes; e += 256) {
      const int r = e / kTrChans, c = e % kTrChans;
      const int m = m0 + r, f = f0 + c;
      if (m < nm && f < nf) at[static_cast<size_t>(m) * nf + f] = tile[c][r];
    }
    __syncthreads();
  }
}

// G[j][c][nu] = sum_{l=|m|}^{lmax} lambda_l|m|(z_j) a[nu][l^2 + l + m],  c = m + lmax.
// grid (2 lmax + 1, ceil(nz / 16), ceil(nf / 16)); D rows = rings, columns = channels.
// In MFMA step q the lanes of group kk = lane / 16 take l = l0 + 8 kk + q, so
// every lane reads eight consecutive l of its ring's Legendre row (two
// 16-byte loads) and each group of 16 lanes one 64-byte segment of `at`.
struct SepLegFwdArgs {
  int nz;
  int nf;
  int lmax;
  int blmax;
  int kaz;
  const float* lam;
  const int* loff;
  const float* at;
  float* G;
};

struct KSepLegFwd {
  using Args = SepLegFwdArgs;
  static constexpr int kThreads = 64, kWaves = 1;
  static __device__ void run(const SepLegFwdArgs& args_, const Blk& B_);
};

__device__ void KSepLegFwd::run(const SepLegFwdArgs& args_, const Blk& B_) {
  int nz = args_.nz;
  int nf = args_.nf;
  int lmax = args_.lmax;
  int blmax = args_.blmax;
  int kaz = args_.kaz;
  const float* __restrict__ lam = args_.lam;
  const int* __restrict__ loff = args_.loff;
  const float* __restrict__ at = args_.at;
  float* __restrict__ G = args_.G;

  // blocks in launch order: grouping an m's blocks on one XCD, as the adjoint
  // does, measured slower here (the rows shorten with |m|, so contiguous m
  // ranges leave the XCDs unevenly loaded)
  const int m = static_cast<int>(B_.x) - lmax, am = m < 0 ? -m : m;
  const int j0 = B_.y * 16, f0 = B_.z * 16;
  const int lane = threadIdx.x, i = lane & 15, kk = lane >> 4;
  const int j = min(j0 + i, nz - 1), f = min(f0 + i, nf - 1);
  const int lp = sep_lpad(blmax, am);
  const float* lrow = lam + loff[am] + static_cast<size_t>(j) * lp;
  f4 acc = f4{0.f, 0.f, 0.f, 0.f};
  for (int l0 = am; l0 <= lmax; l0 += kSepStep) {
    const int lb = l0 + 8 * kk;          // this lane's l = lb .. lb + 7
    f4 a0 = f4{0.f, 0.f, 0.f, 0.f}, a1 = a0;
    if (lb - am < lp) {                  // lp is a multiple of 8: all eight in the row or none
      a0 = *reinterpret_cast<const f4*>(lrow + (lb - am));
      a1 = *reinterpret_cast<const f4*>(lrow + (lb - am) + 4);
    }
    float b[kSepBatch];
#pragma unroll
    for (int q = 0; q < kSepBatch; ++q) {
      const int l = lb + q;
      b[q] = l <= lmax ? at[static_cast<size_t>(l * l + l + m) * nf + f] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < kSepBatch; ++q) acc = sep_mfma(q < 4 ? a0[q] : a1[q - 4], b[q], acc);
  }
  const int c = m + lmax, fo = f0 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int jo = j0 + 4 * kk + r;
    if (jo < nz && fo < nf) G[(static_cast<size_t>(jo) * kaz + c) * nf + fo] = acc[r];
  }
}

// img[nu][slot(j, k)] = sum_{c < nc} G[j][c][nu] Tt[c + toff][k] for visible pixels
// (nc = 2 lmax + 1 rows of G per ring are used).
// grid (column batches that hold a pixel above the horizon at some time, 1,
// ceil(nf / 32)): block x takes batch kb[x] of ring kb_ring[x] (a ring's
// batches are consecutive); each wave computes a 2 x 2 block of 16 x 16 tiles
// (rows = channels, columns = pixels), so every operand load feeds two MFMAs.
struct SepAzFwdArgs {
  int nphi;
  int nf;
  int kaz;
  int nc;
  int toff;
  int tstride;        // row length of Tt (nphi rounded up to whole batches)
  const float* Tt;
  const float* G;
  const int* vidx;
  const int* kb;
  const int* kb_ring;
  int nvp;
  float* img;
};

struct KSepAzFwd {
  using Args = SepAzFwdArgs;
  static constexpr int kThreads = 64, kWaves = 1;
  static __device__ void run(const SepAzFwdArgs& args_, const Blk& B_);
};

__device__ void KSepAzFwd::run(const SepAzFwdArgs& args_, const Blk& B_) {
  int nphi = args_.nphi;
  int nf = args_.nf;
  int kaz = args_.kaz;
  int nc = args_.nc;
  int toff = args_.toff;
  const float* Tt = args_.Tt;
  const float* G = args_.G;
  const int* __restrict__ vidx = args_.vidx;
  int nvp = args_.nvp;
  float* __restrict__ img = args_.img;

  const int3 bk = sep_blocks_x_fastest(sep_xcd_logical(B_), B_);
  const int k0 = args_.kb[bk.x], j = args_.kb_ring[bk.x], f0 = bk.z * 32;
  const int lane = threadIdx.x, i = lane & 15, kk = lane >> 4;
  const float* grow[2];
  const float* tcol[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    grow[h] = G + static_cast<size_t>(j) * kaz * nf + min(f0 + 16 * h + i, nf - 1);
    tcol[h] = Tt + static_cast<size_t>(toff) * args_.tstride + min(k0 + 16 * h + i, nphi - 1);
  }
  f4 acc[2][2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int g = 0; g < 2; ++g) acc[h][g] = f4{0.f, 0.f, 0.f, 0.f};
  struct Batch {
    float a[kSepBatch][2], b[kSepBatch][2];
  };
  auto load = [&](int c0, Batch& B) {
#pragma unroll
    for (int q = 0; q < kSepBatch; ++q) {
      const int c = min(c0 + 4 * q + kk, nc - 1);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        B.a[q][h] = grow[h][static_cast<size_t>(c) * nf];
        B.b[q][h] = tcol[h][static_cast<size_t>(c) * args_.tstride];
      }
    }
  };
  auto mma = [&](int c0, const Batch& B) {
#pragma unroll
    for (int q = 0; q < kSepBatch; ++q) {
      const bool ok = c0 + 4 * q + kk < nc;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float av = ok ? B.a[q][h] : 0.f;
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[h][g] = sep_mfma(av, B.b[q][g], acc[h][g]);
      }
    }
  };
  Batch B0, B1;
  load(0, B0);
  for (int c0 = 0; c0 < nc; c0 += 2 * kSepStep) {
    load(c0 + kSepStep, B1);
    __builtin_amdgcn_sched_barrier(0);
    mma(c0, B0);
    if (c0 + kSepStep >= nc) break;
    load(c0 + 2 * kSepStep, B0);
    __builtin_amdgcn_sched_barrier(0);
    mma(c0 + kSepStep, B1);
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int ko = k0 + 16 * g + (lane & 15);
    if (ko >= nphi) continue;
    const int slot = vidx[j * nphi + ko];
    if (slot < 0) continue;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int fo = f0 + 16 * h + 4 * kk + r;
        if (fo < nf) img[static_cast<size_t>(fo) * nvp + slot] = acc[h][g][r];
      }
  }
}

// H[j][c][nu] = sum_k T[k][c + toff] dL/dI[j][nu][k] for c < nc = 2 lmax + 1,
// over the ring's column batches that hold a pixel above the horizon at some
// time (dL/dI is zero elsewhere).  grid (ceil(nc / 32), nz, ceil(nf / 32));
// each wave computes a 2 x 2 block of 16 x 16 tiles (rows = c, columns =
// channels).  In a group of four MFMA steps, lane group kk supplies columns
// k0 + 4 kk .. + 3 (one per step): the transposed table Tt[c][k] and the
// channel's dL/dI row are both contiguous in k, so each operand value of the
// four steps comes with one 16-byte load.  Rows are tstride (whole batches)
// long and zero beyond nphi in both, so no column needs masking.
struct SepAzAdjArgs {
  int nf;
  int kaz;
  int nc;
  int tstride;
  int toff;
  const float* Tt;
  const float* dfull;
  const int* kb_off;
  const int* kb;
  float* H;
};

struct KSepAzAdj {
  using Args = SepAzAdjArgs;
  static constexpr int kThreads = 64, kWaves = 1;
  static __device__ void run(const SepAzAdjArgs& args_, const Blk& B_);
};

__device__ void KSepAzAdj::run(const SepAzAdjArgs& args_, const Blk& B_) {
  const int nf = args_.nf, kaz = args_.kaz, nc = args_.nc, tstride = args_.tstride;
  float* __restrict__ H = args_.H;

  const int3 bk = sep_blocks_x_fastest(sep_xcd_logical(B_), B_);
  const int c0 = bk.x * 32, j = bk.y, f0 = bk.z * 32;
  const int lane = threadIdx.x, i = lane & 15, kk = lane >> 4;
  const float* trow[2];
  const float* drow[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    trow[h] = args_.Tt + static_cast<size_t>(min(c0 + 16 * h + i, nc - 1) + args_.toff) * tstride + 4 * kk;
    drow[h] = args_.dfull + (static_cast<size_t>(j) * nf + min(f0 + 16 * h + i, nf - 1)) * tstride + 4 * kk;
  }
  f4 acc[2][2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int g = 0; g < 2; ++g) acc[h][g] = f4{0.f, 0.f, 0.f, 0.f};
  // one batch: two groups of 16 columns, per group a 16-byte load of each row
  // (h) and each channel (g)
  struct Batch {
    f4 a[2][2], b[2][2];
  };
  auto load = [&](int k0, Batch& B) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        B.a[s][h] = *reinterpret_cast<const f4*>(trow[h] + k0 + 16 * s);
        B.b[s][h] = *reinterpret_cast<const f4*>(drow[h] + k0 + 16 * s);
      }
  };
  auto mma = [&](const Batch& B) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int g = 0; g < 2; ++g) acc[h][g] = sep_mfma(B.a[s][h][q], B.b[s][g][q], acc[h][g]);
  };
  const int* kb = args_.kb + args_.kb_off[j];
  const int nkb = args_.kb_off[j + 1] - args_.kb_off[j];
  if (nkb > 0) {
    // the batch after the last re-reads the last (always issued, never used)
    auto kb_at = [&](int q) { return kb[min(q, nkb - 1)]; };
    Batch B0, B1;
    load(kb[0], B0);
    for (int q = 0; q < nkb; q += 2) {
      load(kb_at(q + 1), B1);
      __builtin_amdgcn_sched_barrier(0);
      mma(B0);
      if (q + 1 >= nkb) break;
      load(kb_at(q + 2), B0);
      __builtin_amdgcn_sched_barrier(0);
      mma(B1);
    }
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int fo = f0 + 16 * g + (lane & 15);
    if (fo >= nf) continue;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = c0 + 16 * h + 4 * kk + r;
        if (co < nc) H[(static_cast<size_t>(j) * kaz + co) * nf + fo] = acc[h][g][r];
      }
  }
}

// grad[nu][l^2 + l + m] = sum_j lambda_l|m|(z_j) H[j][m + lmax][nu], l = |m| .. lmax;
// 16 lanes read 16 consecutive l of one ring row of the m-major Legendre table.
// grid (2 lmax + 1, ceil((lmax + 1) / 16), ceil(nf / 16)); D rows = l, columns = channels.
struct SepLegAdjArgs {
  int nz;
  int nf;
  int nm;
  int lmax;
  int blmax;
  int kaz;
  const float* lam;
  const int* loff;
  const float* H;
  float* grad;
};

struct KSepLegAdj {
  using Args = SepLegAdjArgs;
  static constexpr int kThreads = 64, kWaves = 1;
  static __device__ void run(const SepLegAdjArgs& args_, const Blk& B_);
};

__device__ void KSepLegAdj::run(const SepLegAdjArgs& args_, const Blk& B_) {
  int nz = args_.nz;
  int nf = args_.nf;
  int nm = args_.nm;
  int lmax = args_.lmax;
  int blmax = args_.blmax;
  int kaz = args_.kaz;
  const float* __restrict__ lam = args_.lam;
  const int* __restrict__ loff = args_.loff;
  const float* __restrict__ H = args_.H;
  float* __restrict__ grad = args_.grad;

  const int3 bk = sep_blocks_m_major(sep_xcd_logical(B_), B_);
  const int m = bk.x - lmax, am = m < 0 ? -m : m;
  const int l0 = am + 16 * bk.y, f0 = bk.z * 16;
  if (l0 > lmax) return;
  const int lane = threadIdx.x, i = lane & 15, kk = lane >> 4;
  const int l = min(l0 + i, lmax), f = min(f0 + i, nf - 1);
  const int c = m + lmax;
  const int lp = sep_lpad(blmax, am);
  const float* lcol = lam + loff[am] + (l - am);   // 16 lanes: 16 consecutive l of one ring
  const float* hcol = H + static_cast<size_t>(c) * nf + f;
  f4 acc = f4{0.f, 0.f, 0.f, 0.f};
  for (int jb = 0; jb < nz; jb += kSepStep) {
    float a[kSepBatch], b[kSepBatch];
#pragma unroll
    for (int q = 0; q < kSepBatch; ++q) {
      const int j = jb + 4 * q + kk;
      const bool ok = j < nz;
      a[q] = ok ? lcol[static_cast<size_t>(j) * lp] : 0.f;
      b[q] = ok ? hcol[static_cast<size_t>(j) * kaz * nf] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < kSepBatch; ++q) acc = sep_mfma(a[q], b[q], acc);
  }
  const int fo = f0 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int lo = l0 + 4 * kk + r;
    if (lo <= lmax && fo < nf) grad[static_cast<size_t>(fo) * nm + lo * lo + lo + m] = acc[r];
  }
}

void launch_synth_fwd_sep(const vis_field* f, const float* alm, float* img, hipStream_t st) {
  const vis_basis* b = f->basis;
  BV_REQUIRE(b->sep_lam != nullptr, VIS_EINVAL, "basis has no separable factor tables");
  const int L = f->lmax;
  const int toff = b->lmax + kSepPad - L;   // T column of c = 0 (m = -L)
  {
    ProfScope ps(&f->prof, "k_alm_transpose", st);
    launch_k<KAlmTranspose>(ceil_div(f->n_modes, kTrModes), 0, AlmTransposeArgs{f->n_freq, f->n_modes, alm,
                                                                     f->scr.sep_at}, st, "k_alm_transpose");
  }
  {
    ProfScope ps(&f->prof, "k_sep_leg_fwd", st);
    dim3 grid(2 * L + 1, ceil_div(b->nz, 16), ceil_div(f->n_freq, 16));
    launch_k<KSepLegFwd>(grid, 0, SepLegFwdArgs{b->nz, f->n_freq, L, b->lmax, f->kaz, b->sep_lam, b->sep_loff,
                                       f->scr.sep_at, f->scr.sep_g}, st, "k_sep_leg_fwd");
  }
  ProfScope ps(&f->prof, "k_sep_az_fwd", st);
  dim3 grid(f->sep_nkb, 1, ceil_div(f->n_freq, 32));
  launch_k<KSepAzFwd>(grid, 0, SepAzFwdArgs{b->nphi, f->n_freq, f->kaz, 2 * L + 1, toff, b->nphi_b, b->sep_tt, f->scr.sep_g,
                                    f->tab.vidx, f->tab.sep_kb, f->tab.sep_kb_ring, f->nv_pad, img},
                      st, "k_sep_az_fwd");
}

// dL/dI comes in the full-grid scratch sep_dfull, written there by the
// adjoint fringe pass (zero at pixels never above the horizon).
void launch_synth_adj_sep(const vis_field* f, float* grad_alm, hipStream_t st) {
  const vis_basis* b = f->basis;
  BV_REQUIRE(b->sep_lam != nullptr, VIS_EINVAL, "basis has no separable factor tables");
  const int L = f->lmax;
  const int toff = b->lmax + kSepPad - L;
  {
    ProfScope ps(&f->prof, "k_sep_az_adj", st);
    dim3 grid(ceil_div(2 * L + 1, 32), b->nz, ceil_div(f->n_freq, 32));
    launch_k<KSepAzAdj>(grid, 0, SepAzAdjArgs{f->n_freq, f->kaz, 2 * L + 1, b->nphi_b, toff, b->sep_tt,
                                      f->scr.sep_dfull, f->tab.sep_kb_off, f->tab.sep_kb, f->scr.sep_g},
                        st, "k_sep_az_adj");
  }
  ProfScope ps(&f->prof, "k_sep_leg_adj", st);
  dim3 grid(2 * L + 1, ceil_div(L + 1, 16), ceil_div(f->n_freq, 16));
  launch_k<KSepLegAdj>(grid, 0, SepLegAdjArgs{b->nz, f->n_freq, f->n_modes, L, b->lmax, f->kaz, b->sep_lam,
                                     b->sep_loff, f->scr.sep_g, grad_alm}, st, "k_sep_leg_adj");
}

}  // namespace bv
