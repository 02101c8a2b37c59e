// Forward and adjoint fringe contractions of the discrete RIME on MFMA.
//
// Sec. 2.1, eq. rime_discrete: V_u(nu, t) = sum_p S_p exp(-2 pi i nu b_u . s_p(t) / c)
// with S = dOmega B I, evaluated once per redundant baseline u (Sec. 3.1).
//
// Lattice factorisation.  Antennas sit on a lattice, so every unique baseline
// is b_u = n1 e1 + n2 e2 with integers 0 <= n1 <= D, |n2| <= D, and the fringe
// factorises exactly:
//     exp(-2 pi i nu b_u . s / c) = alpha^n1 beta^n2,
//     alpha = exp(-2 pi i x1), x1 = nu (e1 . s) / c,  beta likewise with e2.
// Writing beta^m S = c + i d and alpha^n = a_r + i a_i, the four real sums
//     P1 = sum a_r c,  P2 = sum a_i d,  P3 = sum a_r d,  P4 = sum a_i c
// give both signs of n2 at once:
//     V(n, +m) = (P1 - P2) + i (P3 + P4),   V(n, -m) = (P1 + P2) + i (P4 - P3).
// For each (nu, t) the P's for n, m in 1..D form one real GEMM
//     P[2D x 2D] = A[2D x pixels] Bm[pixels x 2D]
// (rows (n, Re/Im alpha^n), columns (m, Re/Im beta^m S)), run on MFMA with
// the pixels as the contraction dimension; the axis baselines n = 0 or m = 0
// are plain sums taken on the vector ALU.  The fringe x beam tiles exist only
// in registers and LDS; nothing of size pixels x baselines touches HBM.
//
// Phase accuracy: x = nu (e . s) / c is formed in FP64 and reduced to
// [-1/2, 1/2] before rounding to FP32, and the powers alpha^n, n <= D, are
// built by repeated complex multiplication, so the phase error of every term
// stays at the FP32 rounding level of a number below one cycle times D.
//
// The adjoint (transpose over the reals) of the same map, for coefficients
// omega_u = dL/dRe V_u - i dL/dIm V_u... (see the gains pass) is
//     Z_p = sum_u Re[omega_u alpha^n1 beta^n2]
//         = sum_{r,c} A[r][p] G[r][c] Bb[p][c] + axis terms,
// with G built from omega(n, +m), omega(n, -m); it runs as the GEMM
// T[r][p] = sum_c G[r][c] Bb[c][p] on MFMA followed by a per-pixel dot with A.
// dL/dI(p, nu) = dOmega sum_t B Z and dL/dF = dOmega sum (dB/dF) I Z follow.
#include "objects.hpp"

namespace bv {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sin and cos of 2 pi x for |x| <= 1/2
__device__ __forceinline__ void sincos_rev(float x, float& s, float& c) {
  sincospif(2.0f * x, &s, &c);
}

// Reduced phase of nu * p in cycles, in [-1/2, 1/2], formed in FP64.
__device__ __forceinline__ float reduced_cycles(double nu, double p) {
  const double x = nu * p;
  return static_cast<float>(x - rint(x));
}

// Block index -> logical index so that consecutive logical indices share an
// XCD (the dispatcher deals blocks round-robin over the 8 XCDs; consecutive
// logical work items reuse the same geometry rows from that XCD's L2).
__device__ __forceinline__ int xcd_logical(int bid, int nblocks) {
  const int per = (nblocks + 7) >> 3;
  return (bid & 7) * per + (bid >> 3);
}

template <int D>
struct Tile {
  static constexpr int RT = (2 * D + 15) / 16;  // 16-wide MFMA tiles per side
  static constexpr int W = 16 * RT;             // padded side
  static constexpr int PITCH = W + 17;          // odd-ish LDS pitch (floats)
};

// ------------------------------------------------------------------ forward --
// One wavefront per (t, nu); loops over the pixel chunks visible at t.
template <int D>
__global__ void __launch_bounds__(64)
k_fringe_fwd(int nf, int nt, int nvp, int nubl, int dr, float d_omega, double beam_ref,
             const double* __restrict__ freq, const double* __restrict__ P1,
             const double* __restrict__ P2, const float* __restrict__ TH2,
             const int* __restrict__ tchunk_off, const int* __restrict__ tchunk,
             const int2* __restrict__ ubl_nm, const float* __restrict__ img,
             const float* __restrict__ fwhm, float2* __restrict__ vu) {
  using T = Tile<D>;
  constexpr int RT = T::RT, W = T::W, PITCH = T::PITCH;
  __shared__ float As[64 * PITCH];
  __shared__ float Bs[64 * PITCH];
  const int lane = threadIdx.x;
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= nf * nt) return;
  const int t = L / nf, f = L - t * nf;
  const double nu = freq[f];
  const float sig = static_cast<float>(fwhm[0] * (beam_ref / nu) * kFwhmToSigma);
  const float kb = 1.0f / (2.0f * sig * sig * static_cast<float>(kLn2));

  f4 acc[RT][RT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < RT; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  float axr[D], axi[D], bxr[D], bxi[D];  // per-lane partial sums of alpha^n S and beta^m S
#pragma unroll
  for (int n = 0; n < D; ++n) axr[n] = axi[n] = bxr[n] = bxi[n] = 0.f;

  const int cbeg = tchunk_off[t], cend = tchunk_off[t + 1];
  float* arow = As + lane * PITCH;
  float* brow = Bs + lane * PITCH;
  for (int ci = cbeg; ci < cend; ++ci) {
    const int k = tchunk[ci] * kChunk + lane;
    const size_t g = static_cast<size_t>(t) * nvp + k;
    const float x1 = reduced_cycles(nu, P1[g]);
    const float x2 = reduced_cycles(nu, P2[g]);
    const float th2 = TH2[g];
    const float s = d_omega * exp2f(-th2 * kb) * img[static_cast<size_t>(f) * nvp + k];
    float s1, c1, s2, c2;
    sincos_rev(x1, s1, c1);
    sincos_rev(x2, s2, c2);
    // alpha^n and beta^m S, n, m = 1..D
    float ar = c1, ai = -s1;
    float br = c2 * s, bi = -s2 * s;
#pragma unroll
    for (int n = 0; n < D; ++n) {
      arow[2 * n] = ar;
      arow[2 * n + 1] = ai;
      brow[2 * n] = br;
      brow[2 * n + 1] = bi;
      axr[n] += ar * s;
      axi[n] += ai * s;
      bxr[n] += br;
      bxi[n] += bi;
      const float nar = ar * c1 + ai * s1;      // (ar + i ai)(c1 - i s1)
      const float nai = ai * c1 - ar * s1;
      const float nbr = br * c2 + bi * s2;
      const float nbi = bi * c2 - br * s2;
      ar = nar; ai = nai; br = nbr; bi = nbi;
    }
#pragma unroll
    for (int r = 2 * D; r < W; ++r) { arow[r] = 0.f; brow[r] = 0.f; }
    wave_sync();
#pragma unroll 4
    for (int q = 0; q < 16; ++q) {
      const int px = 4 * q + (lane >> 4);
      float a[RT], b[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) a[i] = As[px * PITCH + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < RT; ++j) b[j] = Bs[px * PITCH + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < RT; ++j) acc[i][j] = mfma4(a[i], b[j], acc[i][j]);
    }
    wave_sync();
  }
  // reduce the axis sums over the wavefront
#pragma unroll
  for (int n = 0; n < D; ++n) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      axr[n] += __shfl_xor(axr[n], o);
      axi[n] += __shfl_xor(axi[n], o);
      bxr[n] += __shfl_xor(bxr[n], o);
      bxi[n] += __shfl_xor(bxi[n], o);
    }
  }
  // P tile to LDS (reuse As as a W x W matrix), axis sums after it
  float* P = As;
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < RT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) P[(16 * i + 4 * (lane >> 4) + r) * W + 16 * j + (lane & 15)] = acc[i][j][r];
  float* AX = Bs;  // [D][4]: axr, axi, bxr, bxi
  if (lane == 0) {
#pragma unroll
    for (int n = 0; n < D; ++n) {
      AX[4 * n] = axr[n];
      AX[4 * n + 1] = axi[n];
      AX[4 * n + 2] = bxr[n];
      AX[4 * n + 3] = bxi[n];
    }
  }
  wave_sync();
  float2* out = vu + (static_cast<size_t>(t) * nf + f) * nubl;
  for (int u = lane; u < nubl; u += 64) {
    const int2 nm = ubl_nm[u];
    float2 v;
    if (nm.x == 0) {
      v = make_float2(AX[4 * (nm.y - 1) + 2], AX[4 * (nm.y - 1) + 3]);
    } else if (nm.y == 0) {
      v = make_float2(AX[4 * (nm.x - 1)], AX[4 * (nm.x - 1) + 1]);
    } else {
      const int m = nm.y > 0 ? nm.y : -nm.y;
      const int r0 = 2 * (nm.x - 1), c0 = 2 * (m - 1);
      const float p1 = P[r0 * W + c0], p3 = P[r0 * W + c0 + 1];
      const float p4 = P[(r0 + 1) * W + c0], p2 = P[(r0 + 1) * W + c0 + 1];
      v = nm.y > 0 ? make_float2(p1 - p2, p3 + p4) : make_float2(p1 + p2, p4 - p3);
    }
    out[u] = v;
  }
  (void)dr;
}

// ------------------------------------------------------------------ adjoint --
// One wavefront per (nu, chunk of 64 visible pixels); loops over the times at
// which the chunk is above the horizon.  w[t][nu][u] holds omega_u.
template <int D>
__global__ void __launch_bounds__(64)
k_fringe_adj(int nf, int nt, int nvp, int nchunks, int nubl, int dr, float d_omega,
             double beam_ref, const double* __restrict__ freq, const double* __restrict__ P1,
             const double* __restrict__ P2, const float* __restrict__ TH2,
             const int2* __restrict__ chunk_t, const int* __restrict__ ulut,
             const float* __restrict__ img, const float* __restrict__ fwhm,
             const float2* __restrict__ w, float* __restrict__ dimg, float* __restrict__ f_part) {
  using T = Tile<D>;
  constexpr int RT = T::RT, W = T::W, PITCH = T::PITCH;
  __shared__ float As[64 * PITCH];
  __shared__ float Bs[64 * PITCH];
  const int lane = threadIdx.x;
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= nf * nchunks) return;
  const int chunk = L / nf, f = L - chunk * nf;
  const double nu = freq[f];
  const float fw = fwhm[0];
  const float sig = static_cast<float>(fw * (beam_ref / nu) * kFwhmToSigma);
  const float kb = 1.0f / (2.0f * sig * sig * static_cast<float>(kLn2));
  const float kappa = 1.0f / (sig * sig * fw);   // dB/dF = B theta^2 kappa
  const int k = chunk * kChunk + lane;
  const float ival = img[static_cast<size_t>(f) * nvp + k];
  const int2 tr = chunk_t[chunk];
  const int lw = 2 * dr + 1;
  float acc_i = 0.f, acc_f = 0.f;
  float* arow = As + lane * PITCH;
  float* brow = Bs + lane * PITCH;

  for (int t = tr.x; t <= tr.y; ++t) {
    const float2* wt = w + (static_cast<size_t>(t) * nf + f) * nubl;
    const size_t g = static_cast<size_t>(t) * nvp + k;
    const float x1 = reduced_cycles(nu, P1[g]);
    const float x2 = reduced_cycles(nu, P2[g]);
    const float th2 = TH2[g];
    const float bm = exp2f(-th2 * kb);
    float s1, c1, s2, c2;
    sincos_rev(x1, s1, c1);
    sincos_rev(x2, s2, c2);
    float ar = c1, ai = -s1, br = c2, bi = -s2;
    float zax = 0.f;
#pragma unroll
    for (int n = 0; n < D; ++n) {
      arow[2 * n] = ar;
      arow[2 * n + 1] = ai;
      brow[2 * n] = br;
      brow[2 * n + 1] = bi;
      if (n < dr) {
        const int ua = ulut[(n + 1) * lw + dr];        // (n+1, 0)
        const int ub = ulut[0 * lw + (n + 1) + dr];    // (0, n+1)
        if (ua >= 0) { const float2 o = wt[ua]; zax += o.x * ar - o.y * ai; }
        if (ub >= 0) { const float2 o = wt[ub]; zax += o.x * br - o.y * bi; }
      }
      const float nar = ar * c1 + ai * s1;
      const float nai = ai * c1 - ar * s1;
      const float nbr = br * c2 + bi * s2;
      const float nbi = bi * c2 - br * s2;
      ar = nar; ai = nai; br = nbr; bi = nbi;
    }
#pragma unroll
    for (int r = 2 * D; r < W; ++r) { arow[r] = 0.f; brow[r] = 0.f; }
    // coefficient matrix in the MFMA A layout: G[r][c], r = 16 i + (lane & 15),
    // c = 16 kt + 4 s + (lane >> 4)
    float gco[RT][RT][4];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int kt = 0; kt < RT; ++kt)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int r = 16 * i + (lane & 15), c = 16 * kt + 4 * s + (lane >> 4);
          const int n = (r >> 1) + 1, m = (c >> 1) + 1;
          float v = 0.f;
          if (n <= dr && m <= dr) {
            const int up = ulut[n * lw + m + dr], um = ulut[n * lw - m + dr];
            const float2 op = up >= 0 ? wt[up] : make_float2(0.f, 0.f);
            const float2 om = um >= 0 ? wt[um] : make_float2(0.f, 0.f);
            const int pr = r & 1, pc = c & 1;
            if (pr == 0 && pc == 0) v = op.x + om.x;
            else if (pr == 1 && pc == 1) v = om.x - op.x;
            else if (pr == 0 && pc == 1) v = om.y - op.y;
            else v = -op.y - om.y;
          }
          gco[i][kt][s] = v;
        }
    wave_sync();
    float zcore = 0.f;
#pragma unroll
    for (int pg = 0; pg < 4; ++pg) {
      const int px = 16 * pg + (lane & 15);
      float zp = 0.f;
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        f4 tacc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < RT; ++kt)
#pragma unroll
          for (int s = 0; s < 4; ++s)
            tacc = mfma4(gco[i][kt][s], Bs[px * PITCH + 16 * kt + 4 * s + (lane >> 4)], tacc);
#pragma unroll
        for (int r = 0; r < 4; ++r) zp += As[px * PITCH + 16 * i + 4 * (lane >> 4) + r] * tacc[r];
      }
      zp += __shfl_xor(zp, 16);
      zp += __shfl_xor(zp, 32);
      if ((lane >> 4) == pg) zcore = zp;
    }
    wave_sync();
    const float z = zcore + zax;
    acc_i += bm * z;
    acc_f += bm * th2 * z;
  }
  dimg[static_cast<size_t>(f) * nvp + k] = d_omega * acc_i;
  float pf = acc_f * ival;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) pf += __shfl_xor(pf, o);
  if (lane == 0) f_part[static_cast<size_t>(f) * nchunks + chunk] = d_omega * kappa * pf;
}

// ------------------------------------------------------------ launchers --
template <int D>
static void fwd_d(const vis_field* f, const float* img, const float* fwhm, float2* vu, hipStream_t st) {
  const int nblk = static_cast<int>(round_up(static_cast<long>(f->n_freq) * f->n_time, 8));
  const auto& T = f->tab;
  ProfScope ps(&f->prof, "k_fringe_fwd", st);
  k_fringe_fwd<D><<<nblk, 64, 0, st>>>(f->n_freq, f->n_time, f->nv_pad, f->n_ubl, f->extent,
                                       static_cast<float>(f->d_omega), f->beam_ref_hz, T.freq, T.p1,
                                       T.p2, T.th2, T.tchunk_off, T.tchunk, T.ubl_nm, img, fwhm, vu);
  check_launch("k_fringe_fwd");
}

template <int D>
static void adj_d(const vis_field* f, const float* img, const float* fwhm, const float2* w,
                  float* dimg, float* f_part, hipStream_t st) {
  const int nblk = static_cast<int>(round_up(static_cast<long>(f->n_freq) * f->n_chunks, 8));
  const auto& T = f->tab;
  ProfScope ps(&f->prof, "k_fringe_adj", st);
  k_fringe_adj<D><<<nblk, 64, 0, st>>>(f->n_freq, f->n_time, f->nv_pad, f->n_chunks, f->n_ubl,
                                       f->extent, static_cast<float>(f->d_omega), f->beam_ref_hz,
                                       T.freq, T.p1, T.p2, T.th2, T.chunk_t, T.ulut, img, fwhm, w,
                                       dimg, f_part);
  check_launch("k_fringe_adj");
}

#define BV_DISPATCH_EXTENT(ext, CALL)          \
  do {                                         \
    const int e_ = (ext);                      \
    if (e_ <= 2) { CALL(2); }                  \
    else if (e_ <= 4) { CALL(4); }             \
    else if (e_ <= 6) { CALL(6); }             \
    else if (e_ <= 8) { CALL(8); }             \
    else if (e_ <= 12) { CALL(12); }           \
    else { CALL(16); }                         \
  } while (0)

void launch_fringe_fwd(const vis_field* f, const float* img, const float* fwhm, float2* vu,
                       hipStream_t st) {
#define BV_CALL_FWD(DD) fwd_d<DD>(f, img, fwhm, vu, st)
  BV_DISPATCH_EXTENT(f->extent, BV_CALL_FWD);
#undef BV_CALL_FWD
}

void launch_fringe_adj(const vis_field* f, const float* img, const float* fwhm, const float2* w,
                       float* dimg, float* f_part, hipStream_t st) {
#define BV_CALL_ADJ(DD) adj_d<DD>(f, img, fwhm, w, dimg, f_part, st)
  BV_DISPATCH_EXTENT(f->extent, BV_CALL_ADJ);
#undef BV_CALL_ADJ
}

}  // namespace bv
