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
// [-1/2, 1/2] before rounding to FP32, and the powers alpha^n, n <= D, come
// from the three-term recurrence u_{n+1} = 2 cos(theta) u_n - u_{n-1}.  A
// rounding error made at step k reaches step n multiplied by
// sin((n - k) theta) / sin(theta), at most n - k in size, so the error of
// alpha^n stays below about n^2 / 2 FP32 roundings (32 at n = 8).
//
// The adjoint (transpose over the reals) of the same map, for coefficients
// omega_u = dL/dRe V_u - i dL/dIm V_u (formed by the gains pass), is
//     Z_p = sum_u Re[omega_u alpha^n1 beta^n2]
//         = sum_{r,c} A[r][p] G[r][c] Bb[p][c] + axis terms,
// with G built from omega(n, +m), omega(n, -m); it runs as the GEMM
// T[r][p] = sum_c G[r][c] Bb[c][p] on MFMA followed by a per-pixel dot with A.
// dL/dI(p, nu) = dOmega sum_t B Z and dL/dF = dOmega sum (dB/dF) I Z follow.
#include "batch.hpp"
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

// sin and cos of 2 pi x for |x| <= 1/2.  The argument is already reduced to
// one turn in FP64, so the hardware transcendental units (which take their
// argument in turns) are used directly; BV_ACCURATE_TRIG selects the
// correctly-rounded library routine instead.
__device__ __forceinline__ void sincos_rev(float x, float& s, float& c) {
#ifdef BV_ACCURATE_TRIG
  sincospif(2.0f * x, &s, &c);
#else
  s = __builtin_amdgcn_sinf(x);
  c = __builtin_amdgcn_cosf(x);
#endif
}

// x[l] + x[l ^ 16] and x[l] + x[l ^ 32] with the gfx950 lane-swap instructions
// (vector ALU; a generic shuffle would go through the LDS crossbar).
__device__ __forceinline__ float sum_xor16(float x) {
  const unsigned u = __float_as_uint(x);
  const auto p = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
__device__ __forceinline__ float sum_xor32(float x) {
  const unsigned u = __float_as_uint(x);
  const auto p = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}

// 2^x on the hardware exponential unit (no denormal-range rescaling: the
// beam factors it forms are only ever weights, and one below 2^-126 adds
// nothing to a sum of beam-weighted terms).
__device__ __forceinline__ float beam_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Element k of a per-wave array through a 32-bit byte offset (the base is
// uniform over the wave, so the load takes the scalar-base form and no
// per-lane 64-bit address arithmetic is needed).
template <class V>
__device__ __forceinline__ V at_u32(const V* base, int k) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) +
                                     static_cast<uint32_t>(k) * static_cast<uint32_t>(sizeof(V)));
}

// Reduced phase of nu_f p in cycles, in [-1/2, 1/2], in FP32 from the
// table entry q = (y, p), y = nu_c p reduced modulo 1 on the host in FP64,
// and dnu = nu_f - nu_c: x = y + dnu p is at most a few cycles, so one fma
// and one round-to-integer keep the error near one FP32 rounding of x.
__device__ __forceinline__ float reduced_cycles(float dnu, float2 q) {
  const float x = __builtin_fmaf(dnu, q.y, q.x);
  return x - __builtin_rintf(x);
}

// Block index -> logical index so that consecutive logical indices share an
// XCD (the dispatcher deals blocks round-robin over the 8 XCDs; consecutive
// logical work items reuse the same geometry rows from that XCD's L2).
__device__ __forceinline__ int xcd_logical(int bid, int nblocks) {
  const int per = (nblocks + 7) >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// Logical index L -> (outer o, inner i) of an n_o x n_i grid, visited in
// tiles of to outers x ti inners (outer-major inside a tile), so that the
// blocks resident on one XCD at a time share few outer and few inner rows
// (geometry rows per outer, image or coefficient rows per inner) and both fit
// its L2.  A bijection for L < n_o n_i.
__device__ __forceinline__ void tile_map(int L, int n_o, int n_i, int to, int ti, int& o, int& i) {
  const int og = L / (to * n_i), o0 = og * to, tog = min(to, n_o - o0);
  int local = L - og * to * n_i;
  const int ig = local / (tog * ti), i0 = ig * ti, tig = min(ti, n_i - i0);
  local -= ig * tog * ti;
  o = o0 + local / tig;
  i = i0 + local % tig;
}

template <int D>
struct Tile {
  static constexpr int RT = (2 * D + 15) / 16;  // 16-wide MFMA tiles per side
  static constexpr int W = 16 * RT;             // padded side = LDS row length (floats)
};

// LDS layout of the per-pixel operand rows: row px holds W floats as W/4
// groups of 4; logical group g sits at physical group g ^ swz(px).  The
// swizzle makes a wavefront's 128-bit row writes hit every bank group evenly
// and keeps the MFMA operand reads (16 consecutive columns of one row per
// 16 lanes, the next row in the next 16 lanes) free of bank conflicts.
template <int W>
__device__ __forceinline__ int swz(int px) {
  return W == 16 ? ((px >> 1) & 3) : (((px & 1) << 2) | ((px >> 1) & 3));
}
template <int W>
__device__ __forceinline__ int lds_at(int px, int col) {
  return px * W + ((((col >> 2) ^ swz<W>(px))) << 2) + (col & 3);
}

// Powers alpha^n (n = 1..D) and beta^m w (m = 1..D) of one pixel into its LDS
// rows (row px of As / Bs, zero padding up to W); visit(n, alpha^n, beta^n w)
// sees every power while it is still in registers.  With alpha = exp(-i t),
// alpha^(n+1) = 2 cos(t) alpha^n - alpha^(n-1) (the three-term recurrence of
// cos(n t) and sin(n t)), one FMA per component; the same holds for beta^m w.
template <int D, class Visit>
__device__ __forceinline__ void powers_f32(float* av, float* bv, float c1, float s1, float c2,
                                           float s2, float w, Visit visit) {
  float ar0 = 1.f, ai0 = 0.f, ar = c1, ai = -s1;
  float br0 = w, bi0 = 0.f, br = c2 * w, bi = -s2 * w;
  const float t1 = 2.f * c1, t2 = 2.f * c2;
#pragma unroll
  for (int n = 0; n < D; ++n) {
    av[2 * n] = ar;
    av[2 * n + 1] = ai;
    bv[2 * n] = br;
    bv[2 * n + 1] = bi;
    visit(n, ar, ai, br, bi);
    const float nar = t1 * ar - ar0, nai = t1 * ai - ai0;
    const float nbr = t2 * br - br0, nbi = t2 * bi - bi0;
    ar0 = ar; ai0 = ai; br0 = br; bi0 = bi;
    ar = nar; ai = nai; br = nbr; bi = nbi;
  }
}
template <int W>
__device__ __forceinline__ void store_rows(float* As, float* Bs, int px, const float* av, const float* bv) {
#pragma unroll
  for (int g = 0; g < W / 4; ++g) {
    const int o = px * W + ((g ^ swz<W>(px)) << 2);
    *reinterpret_cast<f4*>(As + o) = f4{av[4 * g], av[4 * g + 1], av[4 * g + 2], av[4 * g + 3]};
    *reinterpret_cast<f4*>(Bs + o) = f4{bv[4 * g], bv[4 * g + 1], bv[4 * g + 2], bv[4 * g + 3]};
  }
}
template <int D, int W, class Visit>
__device__ __forceinline__ void write_powers(float* As, float* Bs, int px, float c1, float s1,
                                             float c2, float s2, float w, Visit visit) {
  float av[W], bv[W];
  powers_f32<D>(av, bv, c1, s1, c2, s2, w, visit);
#pragma unroll
  for (int r = 2 * D; r < W; ++r) av[r] = bv[r] = 0.f;
  store_rows<W>(As, Bs, px, av, bv);
}

// ------------------------------------------------- split-precision helpers --
// Split-precision fields run the fringe products on FP16 MFMA as hi + lo
// pairs (x ~ hi + lo, hi = fp16(x), lo = fp16(x - hi)), three products
// hi hi + hi lo + lo hi accumulated in FP32: about 22 significant bits per
// product instead of FP32's 24, at a sixth of the matrix-core time.
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma_h32(h8 a, h8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_h16(h4 a, h4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// hi halves of (x0, x1) packed into one register (round toward zero; the lo
// half carries the rest exactly enough either way)
__device__ __forceinline__ uint32_t split_hi2(float x0, float x1) {
  return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(x0, x1));
}
// lo halves fp16(x0 - hi0), fp16(x1 - hi1): one mixed-precision FMA each
// (hi read as FP16 from its half of `hi`, the difference rounded once to
// FP16 into the low or high half of the result)
__device__ __forceinline__ uint32_t split_lo2(float x0, float x1, uint32_t hi) {
  uint32_t r;
  asm("v_fma_mixlo_f16 %0, %2, -1.0, %1 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(x0), "v"(hi));
  asm("v_fma_mixhi_f16 %0, %2, -1.0, %1 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
      : "+v"(r) : "v"(x1), "v"(hi));
  return r;
}

// LDS layout of the split B operand of the adjoint (32-bit words).  The hi
// halves: rows of W halves padded to BH words, so that the 16-byte operand
// reads of consecutive pixel rows fall on distinct banks.  The lo halves: W/4
// planes of 64 rows x 8 bytes (plane q = halves 4q .. 4q + 3 of every row),
// planes BLP words apart; a K = 16 operand read takes one plane per 16 lanes
// (128 contiguous bytes), and BLP = 128 + 32 words puts the next plane on the
// other half of the banks.
template <int W> struct SplitRows {
  static constexpr int BH = W / 2 + 4;
  static constexpr int BLP = 64 * 2 + 32;
  static constexpr int BL_WORDS = (W / 4) * BLP;
};

// Powers of one pixel for the split adjoint: alpha^n in FP32 into its As row
// (as write_powers), beta^m as FP16 hi + lo pairs into its Bh / Bl rows.
template <int D, class Visit>
__device__ __forceinline__ void powers_split_adj(float* av, uint32_t* bh, uint32_t* bl, float c1,
                                                 float s1, float c2, float s2, Visit visit) {
  float ar0 = 1.f, ai0 = 0.f, ar = c1, ai = -s1;
  float br0 = 1.f, bi0 = 0.f, br = c2, bi = -s2;
  const float t1 = 2.f * c1, t2 = 2.f * c2;
#pragma unroll
  for (int n = 0; n < D; ++n) {
    av[2 * n] = ar;
    av[2 * n + 1] = ai;
    bh[n] = split_hi2(br, bi);
    bl[n] = split_lo2(br, bi, bh[n]);
    visit(n, ar, ai, br, bi);
    const float nar = t1 * ar - ar0, nai = t1 * ai - ai0;
    const float nbr = t2 * br - br0, nbi = t2 * bi - bi0;
    ar0 = ar; ai0 = ai; br0 = br; bi0 = bi;
    ar = nar; ai = nai; br = nbr; bi = nbi;
  }
}
template <int W>
__device__ __forceinline__ void store_rows_split_adj(float* As, uint32_t* Bh, uint32_t* Bl, int px,
                                                     const float* av, const uint32_t* bh,
                                                     const uint32_t* bl) {
  using R = SplitRows<W>;
#pragma unroll
  for (int g = 0; g < W / 4; ++g) {
    const int o = px * W + ((g ^ swz<W>(px)) << 2);
    *reinterpret_cast<f4*>(As + o) = f4{av[4 * g], av[4 * g + 1], av[4 * g + 2], av[4 * g + 3]};
  }
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  typedef uint32_t u2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int g = 0; g < W / 8; ++g)
    *reinterpret_cast<u4*>(Bh + px * R::BH + 4 * g) = u4{bh[4 * g], bh[4 * g + 1], bh[4 * g + 2], bh[4 * g + 3]};
#pragma unroll
  for (int g = 0; g < W / 4; ++g)
    *reinterpret_cast<u2*>(Bl + g * R::BLP + 2 * px) = u2{bl[2 * g], bl[2 * g + 1]};
}
template <int D, int W, class Visit>
__device__ __forceinline__ void write_powers_split(float* As, uint32_t* Bh, uint32_t* Bl, int px,
                                                   float c1, float s1, float c2, float s2,
                                                   Visit visit) {
  float av[W];
  uint32_t bh[W / 2], bl[W / 2];
  powers_split_adj<D>(av, bh, bl, c1, s1, c2, s2, visit);
#pragma unroll
  for (int r = 2 * D; r < W; ++r) av[r] = 0.f;
#pragma unroll
  for (int n = D; n < W / 2; ++n) bh[n] = bl[n] = 0u;
  store_rows_split_adj<W>(As, Bh, Bl, px, av, bh, bl);
}

// Forward split rows: each pixel row holds W halves (W / 2 words, pairs
// (Re, Im) of one power) in 16-byte groups, group g stored at g ^ swz_h(px)
// so that a wavefront's 16-byte row writes spread over the banks; four
// consecutive rows (4 aligned to 4) share the swizzle, which is what the
// transposing operand reads below assume.
template <int W>
__device__ __forceinline__ int swz_h(int px) {
  return W == 16 ? ((px >> 2) & 1) : ((px >> 2) & 3);
}
// Physical row of pixel row px.  A transposing operand read takes four whole
// consecutive rows per 16 lanes; with 32-byte rows (W = 16) the next 16 lanes'
// rows lie 256 bytes further, on the same banks.  Swapping the two halves of
// every odd 8-row block puts those rows on the other half of the banks (for
// W = 32 the swizzle above already separates them).  With it, the 16-byte
// row writes of rows px and px + 4 (and of a row and its swapped partner)
// land in different halves of their 32-byte rows through swz_h.
template <int W>
__device__ __forceinline__ int row_h(int px) {
  return W == 16 ? (px ^ (((px >> 3) & 1) << 2)) : px;
}

// Powers of one pixel for the split forward: alpha^n and beta^m w as FP16
// hi + lo pairs (one word per complex power) into ah, al (alpha) and bh, bl
// (beta); visit(n, ...) sees the FP32 values (beta^m w as generated, w
// already scaled).  store_rows_split writes a pixel's words to its rows of
// Ah, Al, Bh, Bl.
template <int D, class Visit>
__device__ __forceinline__ void powers_split_fwd(uint32_t* ah, uint32_t* al, uint32_t* bh, uint32_t* bl,
                                                 float c1, float s1, float c2, float s2, float w,
                                                 Visit visit) {
  float ar0 = 1.f, ai0 = 0.f, ar = c1, ai = -s1;
  float br0 = w, bi0 = 0.f, br = c2 * w, bi = -s2 * w;
  const float t1 = 2.f * c1, t2 = 2.f * c2;
#pragma unroll
  for (int n = 0; n < D; ++n) {
    ah[n] = split_hi2(ar, ai);
    al[n] = split_lo2(ar, ai, ah[n]);
    bh[n] = split_hi2(br, bi);
    bl[n] = split_lo2(br, bi, bh[n]);
    visit(n, ar, ai, br, bi);
    const float nar = t1 * ar - ar0, nai = t1 * ai - ai0;
    const float nbr = t2 * br - br0, nbi = t2 * bi - bi0;
    ar0 = ar; ai0 = ai; br0 = br; bi0 = bi;
    ar = nar; ai = nai; br = nbr; bi = nbi;
  }
}
template <int W>
__device__ __forceinline__ void store_rows_split(uint32_t* Ah, uint32_t* Al, uint32_t* Bh, uint32_t* Bl,
                                                 int px, const uint32_t* ah, const uint32_t* al,
                                                 const uint32_t* bh, const uint32_t* bl) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int g = 0; g < W / 8; ++g) {
    const int o = row_h<W>(px) * (W / 2) + ((g ^ swz_h<W>(px)) << 2);
    *reinterpret_cast<u4*>(Ah + o) = u4{ah[4 * g], ah[4 * g + 1], ah[4 * g + 2], ah[4 * g + 3]};
    *reinterpret_cast<u4*>(Al + o) = u4{al[4 * g], al[4 * g + 1], al[4 * g + 2], al[4 * g + 3]};
    *reinterpret_cast<u4*>(Bh + o) = u4{bh[4 * g], bh[4 * g + 1], bh[4 * g + 2], bh[4 * g + 3]};
    *reinterpret_cast<u4*>(Bl + o) = u4{bl[4 * g], bl[4 * g + 1], bl[4 * g + 2], bl[4 * g + 3]};
  }
}

// One K = 32 FP16 MFMA operand (eight consecutive pixels of one row or
// column per lane) of 16-column tile `tile` from rows stored pixel-major:
// lane l (index j = l & 15 in its group, group g = l >> 4) needs values
// [pix0 + 8 g .. + 7][16 tile + j].  ds_read_b64_tr_b16 gives lane j of a
// 16-lane group element (j & 3) of the 4-half chunk addressed by lane
// 4 k + (j >> 2), for k = 0..3; so lane j addresses row pix0 + 8 g + 4 h +
// (j >> 2), halves 16 tile + 4 (j & 3) .. + 3, and the two reads (h = 0, 1)
// give its eight pixels in order.
typedef short s4 __attribute__((ext_vector_type(4)));
template <int W>
__device__ __forceinline__ h8 tr_operand(const uint32_t* base, int pix0, int tile, int lane) {
  const int j = lane & 15, g = lane >> 4;
  const int row0 = pix0 + 8 * g + (j >> 2);
  const int col = 16 * tile + 4 * (j & 3);                 // halves
  const int grp = col >> 3, within = (col & 7) >> 1;       // 16-byte group, word in group
  s4 v[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int row = row0 + 4 * h;
    const uint32_t* a = base + row_h<W>(row) * (W / 2) + ((grp ^ swz_h<W>(row)) << 2) + within;
    v[h] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
        (__attribute__((address_space(3))) s4*)(reinterpret_cast<uintptr_t>(a)));
  }
  typedef short s8 __attribute__((ext_vector_type(8)));
  const s8 c = s8{v[0][0], v[0][1], v[0][2], v[0][3], v[1][0], v[1][1], v[1][2], v[1][3]};
  return __builtin_bit_cast(h8, c);
}

// Per-channel power-of-two scale of the split forward's beam-weighted sky.
// k_chan_scale writes the maximum |I| of each of kScaleParts segments of a
// channel's row; the forward kernel turns the channel's maxima into
// scale = 2^(13 - e) with dOmega max |I| < 2^e (B <= 1), so that every
// |dOmega B I scale| < 2^13 and its FP16 lo part stays a normal number.
struct ChanScaleArgs {
  int nvp;
  const float* img;
  float* part;   // [n_freq][kScaleParts]
};

struct KChanScale {
  using Args = ChanScaleArgs;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const ChanScaleArgs& a, const Blk& B) {
    __shared__ float red[4];
    const int seg = (a.nvp + kScaleParts - 1) / kScaleParts;
    const int k0 = B.y * seg, k1 = min(a.nvp, k0 + seg);
    const float* row = a.img + static_cast<size_t>(B.x) * a.nvp;
    float m = 0.f;
    for (int k = k0 + threadIdx.x; k < k1; k += 256) m = fmaxf(m, fabsf(row[k]));
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
      a.part[B.x * kScaleParts + B.y] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  }
};

__device__ __forceinline__ float chan_scale(const float* part, int f, float d_omega) {
  float mx = 0.f;
#pragma unroll
  for (int q = 0; q < kScaleParts; ++q) mx = fmaxf(mx, part[f * kScaleParts + q]);
  mx *= d_omega;
  float sc = 1.0f;
  if (mx > 0.f && isfinite(mx)) {
    int e;
    frexpf(mx, &e);   // mx < 2^e
    sc = ldexpf(1.0f, max(-100, min(100, 13 - e)));
  }
  return sc;
}

// ------------------------------------------------------------------ forward --
// One block of kFwdWaves wavefronts per (t, nu) (per (t, group of stacked
// channels) for D <= 4, see fwd_channels_per_tile); wave w takes every
// kFwdWaves-th pixel chunk visible at t, starting at chunk w, and the block
// adds the waves' partial tiles in a fixed order at the end.  Splitting a
// (t, nu) over the four SIMDs of a CU balances the SIMDs: with one wave per
// (t, nu), a 61-dish field's 3840 waves over 1024 SIMDs leave a quarter of
// the SIMDs with 4 waves and the rest with 3, and the kernel lasts as long
// as the busiest.  Software pipeline per chunk: the MFMA operands of chunk k
// are read from LDS into registers, then the 16 MFMAs of chunk k are
// interleaved with the vector-ALU generation of the wave's next chunk
// (written to LDS); geometry is loaded two of the wave's chunks ahead.  Four
// resident waves per SIMD (<= 128 VGPRs) for extents up to 8.
constexpr int kFwdWaves = 4;

struct FwdArgs {
  int nf, nt, nvp, nubl;
  float d_omega;
  const float* dnu;
  const float* sigr;
  const float2* Q1;
  const float2* Q2;
  const float* TH2;
  const int* tchunk_off;
  const int* tchunk;
  const int2* ubl_nm;
  const float* img;
  const float* fwhm;
  float2* vu;
  const float* cscale;   // SPLIT: [n_freq][kScaleParts] segment maxima of |I|
};

// Channels that share one 16 x 16 tile: a lattice extent D fills 2D of the
// tile's rows and columns, so for D <= 4 the rows and columns of 16 / (2D)
// channels are stacked and the tile's diagonal blocks are their P matrices
// (the off-diagonal blocks pair one channel's alpha with another's beta and
// are not read).  The MFMA work is shared; the generation is per channel.
__host__ __device__ constexpr int fwd_channels_per_tile(int D) { return 2 * D <= 8 ? 16 / (2 * D) : 1; }
// Extents whose 2 D operand rows leave a one-channel tile a free row and
// column (D = 6, 12): a row of ones in A and a column of the pixel weight w in
// B make the tile form the axis sums sum_p w beta^m (row 2 D) and
// sum_p w alpha^n (column 2 D) in the padding the MFMAs compute anyway.
__host__ __device__ constexpr bool fwd_axis_in_tile(int D) {
  return fwd_channels_per_tile(D) == 1 && 2 * D < 16 * ((2 * D + 15) / 16);
}

// SPLIT: the P tile runs on FP16 MFMA (K = 32) as three products of hi + lo
// pairs, A_hi B_hi + A_lo B_hi + A_hi B_lo, accumulated in FP32; the beam-
// weighted sky carries the channel's power-of-two scale, undone at the end.
template <int D, bool SPLIT = false>
struct KFringeFwd {
  using Args = FwdArgs;
  static constexpr int kThreads = 64 * kFwdWaves, kWaves = D <= 8 ? 4 : 2;
  static __device__ void run(const FwdArgs& args, const Blk& B);
};

template <int D, bool SPLIT>
__device__ void KFringeFwd<D, SPLIT>::run(const FwdArgs& args, const Blk& B) {
  const int nf = args.nf, nt = args.nt, nvp = args.nvp, nubl = args.nubl;
  const float d_omega = args.d_omega;
  const float2* Q1 = args.Q1;
  const float2* Q2 = args.Q2;
  const float* TH2 = args.TH2;
  const int* __restrict__ tchunk_off = args.tchunk_off;
  const int* __restrict__ tchunk = args.tchunk;
  const int2* __restrict__ ubl_nm = args.ubl_nm;
  const float* img = args.img;
  const float* __restrict__ fwhm = args.fwhm;
  float2* __restrict__ vu = args.vu;
  using T = Tile<D>;
  constexpr int RT = T::RT, W = T::W;
  __shared__ __attribute__((aligned(16))) float As_all[kFwdWaves][64 * W];
  __shared__ __attribute__((aligned(16))) float Bs_all[kFwdWaves][64 * W];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  float* As = As_all[wv];   // this wave's operand rows
  float* Bs = Bs_all[wv];
  // SPLIT: the same LDS as FP16 hi and lo row sets (64 rows of W halves each)
  uint32_t* Ah = reinterpret_cast<uint32_t*>(As);
  uint32_t* Al = Ah + 32 * W;
  uint32_t* Bh = reinterpret_cast<uint32_t*>(Bs);
  uint32_t* Bl = Bh + 32 * W;
  constexpr int NCH = fwd_channels_per_tile(D);
  static_assert(NCH == 1 || RT == 1, "stacked channels share one 16 x 16 tile");
  constexpr bool AXT = fwd_axis_in_tile(D);
  const int nfg = (nf + NCH - 1) / NCH;   // channel groups
  const int L = xcd_logical(B.x, B.nx);
  if (L >= nfg * nt) return;   // uniform over the block
  int t, fgrp;
  tile_map(L, nt, nfg, 4, 32, t, fgrp);   // 128 resident blocks per XCD: 4 times x 32 channel groups
  // channel c of the group: f = NCH fgrp + c; one past the band (an odd
  // channel count) runs with zero weight and is not written
  float dnu[NCH], csc[NCH], kb[NCH], chan_on[NCH];
  const float* imf[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int fc = NCH * fgrp + c, fl = min(fc, nf - 1);
    chan_on[c] = fc < nf ? 1.0f : 0.0f;
    dnu[c] = args.dnu[fl];
    csc[c] = SPLIT ? chan_scale(args.cscale, fl, d_omega) : 1.0f;   // power of two
    const float sig = fwhm[0] * args.sigr[fl];
    kb[c] = 1.0f / (2.0f * sig * sig * static_cast<float>(kLn2));
    imf[c] = img + static_cast<size_t>(fl) * nvp;
  }

  // NACC independent accumulator sets (consecutive MFMAs of a chunk go to
  // different sets); one set measured fastest at 61 dishes
  constexpr int NACC = 1;
  f4 acc[NACC][RT][RT];
#pragma unroll
  for (int h = 0; h < NACC; ++h)
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < RT; ++j) acc[h][i][j] = f4{0.f, 0.f, 0.f, 0.f};
  // per-lane partial sums of alpha^n S and beta^m S (the axis baselines;
  // unused where they ride in the tile)
  constexpr int DX = AXT ? 1 : D;
  float axr[NCH][DX], axi[NCH][DX], bxr[NCH][DX], bxi[NCH][DX];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int n = 0; n < DX; ++n) axr[c][n] = axi[c][n] = bxr[c][n] = bxi[c][n] = 0.f;

  const int cbeg = tchunk_off[t], cend = tchunk_off[t + 1];
  const float2* q1t = Q1 + static_cast<size_t>(t) * nvp;
  const float2* q2t = Q2 + static_cast<size_t>(t) * nvp;
  const float* tht = TH2 + static_cast<size_t>(t) * nvp;

  struct G { float2 q1, q2; float th, iv[NCH]; };
  auto load = [&](int ci) {
    const int k = tchunk[ci] * kChunk + lane;
    G g;
    g.q1 = at_u32(q1t, k);
    g.q2 = at_u32(q2t, k);
    g.th = at_u32(tht, k);
#pragma unroll
    for (int c = 0; c < NCH; ++c) g.iv[c] = at_u32(imf[c], k);
    return g;
  };
  // powers of one chunk into LDS, channel c in rows and columns 2D c ..;
  // `live` = 0 turns a padding pass into a no-op
  auto generate = [&](const G& g, float live) {
    float av[SPLIT ? 1 : W], bv[SPLIT ? 1 : W];
    uint32_t ah[SPLIT ? W / 2 : 1], al[SPLIT ? W / 2 : 1], bh[SPLIT ? W / 2 : 1], bl[SPLIT ? W / 2 : 1];
    float wlast = 0.f;   // the weight (times its scale) of the last channel
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const float x1 = reduced_cycles(dnu[c], g.q1);
      const float x2 = reduced_cycles(dnu[c], g.q2);
      const float s = live * chan_on[c] * d_omega * beam_exp2(-g.th * kb[c]) * g.iv[c];
      float s1, c1, s2, c2;
      sincos_rev(x1, s1, c1);
      sincos_rev(x2, s2, c2);
      auto visit = [&](int n, float ar, float ai, float br, float bi) {
        if constexpr (!AXT) {
          axr[c][n] += ar * s;
          axi[c][n] += ai * s;
          bxr[c][n] += br;   // SPLIT: scaled by csc, undone after the loop
          bxi[c][n] += bi;
        }
      };
      wlast = SPLIT ? s * csc[c] : s;
      if constexpr (SPLIT)
        powers_split_fwd<D>(ah + D * c, al + D * c, bh + D * c, bl + D * c, c1, s1, c2, s2,
                            wlast, visit);
      else
        powers_f32<D>(av + 2 * D * c, bv + 2 * D * c, c1, s1, c2, s2, s, visit);
    }
    if constexpr (SPLIT) {
#pragma unroll
      for (int n = NCH * D; n < W / 2; ++n) ah[n] = al[n] = bh[n] = bl[n] = 0u;
      if constexpr (AXT) {   // row 2 D: (1, 0); column 2 D: (w, 0), as hi + lo
        ah[D] = split_hi2(1.f, 0.f);
        bh[D] = split_hi2(wlast, 0.f);
        bl[D] = split_lo2(wlast, 0.f, bh[D]);
      }
      store_rows_split<W>(Ah, Al, Bh, Bl, lane, ah, al, bh, bl);
    } else {
#pragma unroll
      for (int r = 2 * NCH * D; r < W; ++r) av[r] = bv[r] = 0.f;
      if constexpr (AXT) {
        av[2 * D] = 1.f;
        bv[2 * D] = wlast;
      }
      store_rows<W>(As, Bs, lane, av, bv);
    }
  };
  float a[SPLIT ? 1 : 16][RT], b[SPLIT ? 1 : 16][RT];
  // SPLIT operands of the two K = 32 steps of a chunk: hi and lo of A and B
  h8 oah[SPLIT ? 2 : 1][RT], oal[SPLIT ? 2 : 1][RT], obh[SPLIT ? 2 : 1][RT], obl[SPLIT ? 2 : 1][RT];
  // MFMA step q reads row px = 4 q + (lane >> 4); the swizzle of row px
  // depends on q only through q & 1, so two per-lane offsets per column tile
  // plus a constant 8 W per step pair address every read (the constant goes
  // into the instruction's offset field instead of an address register)
  int ofs[2][RT];
#pragma unroll
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int i = 0; i < RT; ++i) ofs[e][i] = lds_at<W>(4 * e + (lane >> 4), 16 * i + (lane & 15));
  auto operands = [&]() {
    if constexpr (SPLIT) {
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          oah[ks][i] = tr_operand<W>(Ah, 32 * ks, i, lane);
          oal[ks][i] = tr_operand<W>(Al, 32 * ks, i, lane);
          obh[ks][i] = tr_operand<W>(Bh, 32 * ks, i, lane);
          obl[ks][i] = tr_operand<W>(Bl, 32 * ks, i, lane);
        }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          const int o = ofs[q & 1][i] + (q >> 1) * 8 * W;
          a[q][i] = As[o];
          b[q][i] = Bs[o];
        }
      }
    }
  };
  // one chunk: the MFMAs of chunk ci (register operands) interleaved with the
  // generation of chunk ci + 1 from `cur`, while chunk ci + 2's geometry loads
  // into `nxt`; the loop below is unrolled by two so the two geometry sets
  // swap roles without register copies
  constexpr int S = kFwdWaves;   // chunk stride of one wave
  auto chunk_step = [&](int ci, const G& cur, G& nxt) {
    nxt = load(min(ci + 2 * S, cend - 1));
    // keep the prefetch here: the sources are read-only, so the optimizer
    // would otherwise re-issue the loads right before their use
    asm volatile("" ::: "memory");
    if constexpr (SPLIT) {
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int j = 0; j < RT; ++j) {
            acc[0][i][j] = mfma_h32(oah[ks][i], obh[ks][j], acc[0][i][j]);
            acc[0][i][j] = mfma_h32(oal[ks][i], obh[ks][j], acc[0][i][j]);
            acc[0][i][j] = mfma_h32(oah[ks][i], obl[ks][j], acc[0][i][j]);
          }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q)
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int j = 0; j < RT; ++j)
            acc[q % NACC][i][j] = mfma4(a[q][i], b[q][j], acc[q % NACC][i][j]);
    }
    generate(cur, ci + S < cend ? 1.0f : 0.0f);
    if constexpr (SPLIT) {
#pragma unroll
      for (int q = 0; q < 6 * RT * RT; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 16 / (RT * RT), 0);  // vector ALU
        __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);   // one LDS write (128-bit)
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16 * RT * RT; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 8 / (RT * RT), 0);  // vector ALU
        __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);   // one LDS write (128-bit)
      }
    }
    wave_sync();
    operands();
    wave_sync();
  };
  const int c0 = cbeg + wv;
  if (c0 < cend) {   // uniform over the wave
    generate(load(c0), 1.0f);
    G ga = load(min(c0 + S, cend - 1)), gb;
    wave_sync();
    operands();
    wave_sync();
    for (int ci = c0; ci < cend; ci += 2 * S) {
      chunk_step(ci, ga, gb);
      if (ci + S >= cend) break;
      chunk_step(ci + S, gb, ga);
    }
  }
  // channel of each tile row / column block (its scale is undone on its block)
  float inv_csc[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    inv_csc[c] = 1.0f / csc[c];   // exact: a power of two
    if constexpr (!AXT) {
#pragma unroll
      for (int n = 0; n < D; ++n) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
          axr[c][n] += __shfl_xor(axr[c][n], o);
          axi[c][n] += __shfl_xor(axi[c][n], o);
          bxr[c][n] += __shfl_xor(bxr[c][n], o);
          bxi[c][n] += __shfl_xor(bxi[c][n], o);
        }
        if constexpr (SPLIT) {
          bxr[c][n] *= inv_csc[c];
          bxi[c][n] *= inv_csc[c];
        }
      }
    }
  }
  // this wave's P tile to its LDS rows (reused as a W x W matrix), its axis
  // sums to its Bs rows
  {
    float* Pw = As;
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < RT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float sum = acc[0][i][j][r];
#pragma unroll
          for (int h = 1; h < NACC; ++h) sum += acc[h][i][j][r];
          // column 16 j + (lane & 15) belongs to channel (lane & 15) / 2D
          if constexpr (SPLIT) {
            float isc = inv_csc[0];
#pragma unroll
            for (int c = 1; c < NCH; ++c)
              if ((lane & 15) >= 2 * D * c) isc = inv_csc[c];
            sum *= isc;
          }
          Pw[(16 * i + 4 * (lane >> 4) + r) * W + 16 * j + (lane & 15)] = sum;
        }
    float* AXw = Bs;  // [NCH][D][4]: axr, axi, bxr, bxi
    if (!AXT && lane == 0) {
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int n = 0; n < DX; ++n) {
          AXw[4 * (D * c + n)] = axr[c][n];
          AXw[4 * (D * c + n) + 1] = axi[c][n];
          AXw[4 * (D * c + n) + 2] = bxr[c][n];
          AXw[4 * (D * c + n) + 3] = bxi[c][n];
        }
    }
  }
  __syncthreads();
  // the block's totals, waves added in index order, into the last wave's
  // rows beyond the tiles (W x W + 4 D NCH floats fit in one wave's 64 W)
  constexpr int NAX = AXT ? 0 : 4 * D * NCH;
  float* P = Bs_all[kFwdWaves - 1] + NAX;
  float* AX = Bs_all[kFwdWaves - 1] + NAX + W * W;
  static_assert(2 * NAX + W * W <= 64 * W, "tile totals exceed one wave's rows");
  for (int e = threadIdx.x; e < W * W + NAX; e += 64 * kFwdWaves) {
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < kFwdWaves; ++w) sum += e < W * W ? As_all[w][e] : Bs_all[w][e - W * W];
    if (e < W * W) P[e] = sum; else AX[e - W * W] = sum;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int fc = NCH * fgrp + c;
    if (fc >= nf) break;   // uniform over the block
    float2* out = vu + (static_cast<size_t>(t) * nf + fc) * nubl;
    const float* AXc = AX + 4 * D * c;
    const int off = 2 * D * c;   // the channel's diagonal block
    for (int u = threadIdx.x; u < nubl; u += 64 * kFwdWaves) {
      const int2 nm = ubl_nm[u];
      float2 v;
      if (AXT && nm.x == 0) {   // row 2 D: sum_p of the B columns of beta^m w
        v = make_float2(P[2 * D * W + 2 * (nm.y - 1)], P[2 * D * W + 2 * (nm.y - 1) + 1]);
      } else if (AXT && nm.y == 0) {   // column 2 D: sum_p of alpha^n w
        v = make_float2(P[2 * (nm.x - 1) * W + 2 * D], P[(2 * (nm.x - 1) + 1) * W + 2 * D]);
      } else if (nm.x == 0) {
        v = make_float2(AXc[4 * (nm.y - 1) + 2], AXc[4 * (nm.y - 1) + 3]);
      } else if (nm.y == 0) {
        v = make_float2(AXc[4 * (nm.x - 1)], AXc[4 * (nm.x - 1) + 1]);
      } else {
        const int m = nm.y > 0 ? nm.y : -nm.y;
        const int r0 = off + 2 * (nm.x - 1), c0 = off + 2 * (m - 1);
        const float p1 = P[r0 * W + c0], p3 = P[r0 * W + c0 + 1];
        const float p4 = P[(r0 + 1) * W + c0], p2 = P[(r0 + 1) * W + c0 + 1];
        v = nm.y > 0 ? make_float2(p1 - p2, p3 + p4) : make_float2(p1 + p2, p4 - p3);
      }
      out[u] = v;
    }
  }
}

// ------------------------------------------------------------------ adjoint --
// One wavefront per (nu, chunk of 64 visible pixels) (per pair of channels
// for D = 4, see adj_channels_per_tile); loops over the times at which the
// chunk is above the horizon.  gco[t][nu] holds the coefficient
// matrix in MFMA A-operand order, then the alpha-axis accumulator inputs of
// every (row tile, lane group), then the axis coefficients (and, SPLIT, the
// inverse of the power-of-two scale of the FP16 coefficients).
//
// SPLIT: T = G Bb runs on FP16 MFMA, per 16 x 16 tile one K = 32 product
// [G_hi | G_lo] [B_hi; B_hi] and one K = 16 product G_hi B_lo; the coefficient
// operands come ready from the gains pass, only beta^m is split here.
template <int RT, bool SPLIT> struct AdjCoef { f4 gv[RT][RT]; };
template <int RT> struct AdjCoef<RT, true> { h8 ga[RT][RT]; h4 gb[RT][RT]; };

struct AdjArgs {
  int nf, nt, nvp, nchunks, gstride;
  float d_omega;
  const float* dnu;
  const float* sigr;
  const float2* Q1;
  const float2* Q2;
  const float* TH2;
  const int2* chunk_t;
  const float* img;
  const float* fwhm;
  const float* gco;
  const float* gco_lane;
  float* dimg;
  float* f_part;
  // non-null: dL/dI of visible slot k < nv goes to dfull[voff[k] + nu fstride]
  // (the full-grid rows of the separable adjoint synthesis), not dimg[nu][k]
  float* dfull;
  const int* voff;
  int nv, fstride;
};

template <int D, bool SPLIT>
struct KFringeAdj {
  using Args = AdjArgs;
  static constexpr int kThreads = 64, kWaves = 1;
  static __device__ void run(const AdjArgs& args, const Blk& B);
};

template <int D, bool SPLIT>
__device__ void KFringeAdj<D, SPLIT>::run(const AdjArgs& args, const Blk& B) {
  const int nf = args.nf, nvp = args.nvp, nchunks = args.nchunks, gstride = args.gstride;
  const float d_omega = args.d_omega;
  const float2* Q1 = args.Q1;
  const float2* Q2 = args.Q2;
  const float* TH2 = args.TH2;
  const int2* __restrict__ chunk_t = args.chunk_t;
  const float* __restrict__ img = args.img;
  const float* __restrict__ fwhm = args.fwhm;
  const float* __restrict__ gco = args.gco;
  const float* gco_lane = args.gco_lane;
  float* __restrict__ dimg = args.dimg;
  float* __restrict__ f_part = args.f_part;
  using T = Tile<D>;
  using R = SplitRows<T::W>;
  constexpr int RT = T::RT, W = T::W;
  constexpr int NMAT = RT * RT * (SPLIT ? 384 : 256);
  __shared__ __attribute__((aligned(16))) float As[64 * W];
  // FP32 B operand rows, or (SPLIT) the hi rows followed by the lo rows
  __shared__ __attribute__((aligned(16))) float Bs[SPLIT ? 64 * R::BH + R::BL_WORDS : 64 * W];
  uint32_t* Bh = reinterpret_cast<uint32_t*>(Bs);
  uint32_t* Bl = Bh + 64 * R::BH;
  const int lane = threadIdx.x;
  constexpr int NCH = adj_channels_per_tile(D);
  static_assert(NCH == 1 || (D == 4 && RT == 1), "two stacked channels: D = 4 only");
  // beta-axis terms in the tile's row 2 D (the gains pass put omega(0, m)
  // there) against a row of ones in the pixel operand
  constexpr bool AXT = adj_axis_in_tile(D);
  const int nfg = (nf + NCH - 1) / NCH;   // channel groups
  const int L = xcd_logical(B.x, B.nx);
  if (L >= nfg * nchunks) return;
  int chunk, fgrp;
  // 512 resident waves per XCD: 32 chunks x 16 channel groups (the field
  // set-up orders the chunks so that every 32-chunk tile holds about the
  // same number of (chunk, time) steps, so the XCDs' ranges balance)
  tile_map(L, nchunks, nfg, kAdjChunkTile, 16, chunk, fgrp);
  const int k = chunk * kChunk + lane;
  const float fw = fwhm[0];
  // channel c of the group: f = NCH fgrp + c (one past the band, for an odd
  // channel count, gets zero coefficients and is not written)
  int fch[NCH];
  float dnu[NCH], kb[NCH], kappa[NCH], ival[NCH], acc_i[NCH], acc_f[NCH], chan_on[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int fc = NCH * fgrp + c;
    fch[c] = min(fc, nf - 1);
    chan_on[c] = fc < nf ? 1.0f : 0.0f;
    dnu[c] = args.dnu[fch[c]];
    const float sig = fw * args.sigr[fch[c]];
    kb[c] = 1.0f / (2.0f * sig * sig * static_cast<float>(kLn2));
    kappa[c] = 1.0f / (sig * sig * fw);   // dB/dF = B theta^2 kappa
    ival[c] = img[static_cast<size_t>(fch[c]) * nvp + k];
    acc_i[c] = acc_f[c] = 0.f;
  }
  // NCH > 1: the tile's row block r / 2D and column block belong to one
  // channel each; a lane's coefficient operand is channel c's own operand of
  // lane `lane - src_shift c` on the diagonal blocks and zero elsewhere, and
  // its output rows 4 (lane >> 4) .. + 3 belong to channel (lane >> 4) / 2
  const int c_row = NCH > 1 ? (lane & 15) / (2 * D) : 0;
  const int c_out = NCH > 1 ? (lane >> 4) / (D / 2) : 0;
  const int2 tr = chunk_t[chunk];
  // Partial sums, over this lane's four rows of every row tile, of the core and
  // alpha-axis terms of the pixels of the four 16-pixel groups, weighted by B
  // and by B theta^2; reduced across the row groups once, after the time loop.
  float pz_i[4] = {0.f, 0.f, 0.f, 0.f}, pz_f[4] = {0.f, 0.f, 0.f, 0.f};
  __shared__ float2 BW[NCH][64];   // (B, B theta^2) of every pixel of the chunk at this t
  const size_t gst = static_cast<size_t>(nf) * gstride;
  // gco feeds the wave-uniform (scalar) loads of the axis coefficients;
  // gco_lane, the same table, the per-lane loads of the prefetch below: a
  // pointer not marked read-only-unaliased keeps the optimizer from moving
  // those loads to their use in the next step (as it does for Q1, Q2, TH2)
  auto gco_at = [&](int t, int c) { return gco + t * gst + static_cast<size_t>(fch[c]) * gstride; };
  // Software pipeline over t, unrolled by two so that the two register sets
  // swap roles without copies: the geometry and this lane's coefficients of
  // time t + 1 load while time t is processed.
  struct Step : AdjCoef<RT, SPLIT> {
    float2 q1, q2;
    float th2;
    // alpha-axis coefficients of this lane's rows 16 i + 4 (lane >> 4) + 0..3:
    // (Re, -Im) of omega(n, 0) for the two powers n of those rows, stored in
    // this order by the gains pass.  As the first MFMA's accumulator input
    // they put sum_n Re[omega(n, 0) alpha^n] into the per-pixel dot with A.
    f4 g1[RT];
  };
  // per-lane channel selection (NCH <= 2)
  auto chan_of = [&](const int* arr, int c) { return NCH == 1 || c == 0 ? arr[0] : arr[NCH - 1]; };
  auto load_step = [&](Step& S, int t) {
    const size_t row = static_cast<size_t>(t) * nvp;   // uniform over the wave
    S.q1 = at_u32(Q1 + row, k);
    S.q2 = at_u32(Q2 + row, k);
    S.th2 = at_u32(TH2 + row, k);
    const size_t tbase = static_cast<size_t>(t) * gst;
    // the coefficient operand: this lane's row channel's slice; zero off the
    // diagonal blocks and for a channel past the band
    const float* Gr = gco_lane + tbase + static_cast<size_t>(chan_of(fch, c_row)) * gstride;
    const float* Go = gco_lane + tbase + static_cast<size_t>(chan_of(fch, c_out)) * gstride;
    const bool row_on = NCH == 1 || (c_row == 0 ? chan_on[0] : chan_on[NCH - 1]) != 0.f;
    const bool on_blk = NCH == 1 || (row_on && c_row == c_out);
    const bool on_k32 = NCH == 1 || (row_on && c_row == ((lane >> 4) & 1));
    const int src = lane - 40 * c_row;          // FP32 and K = 16 operands
    const int src32 = lane - 24 * c_row;        // K = 32 operand
#pragma unroll
    for (int i = 0; i < RT; ++i) {
#pragma unroll
      for (int kt = 0; kt < RT; ++kt) {
        if constexpr (SPLIT) {
          const h8 va = *reinterpret_cast<const h8*>(Gr + ((i * RT + kt) * 64 + (on_k32 ? src32 : lane)) * 4);
          const h4 vb = *reinterpret_cast<const h4*>(Gr + RT * RT * 256 + ((i * RT + kt) * 64 + (on_blk ? src : lane)) * 2);
          S.ga[i][kt] = on_k32 ? va : h8{};
          S.gb[i][kt] = on_blk ? vb : h4{};
        } else {
          const f4 v = *reinterpret_cast<const f4*>(Gr + ((i * RT + kt) * 64 + (on_blk ? src : lane)) * 4);
          S.gv[i][kt] = on_blk ? v : f4{0.f, 0.f, 0.f, 0.f};
        }
      }
      S.g1[i] = *reinterpret_cast<const f4*>(Go + NMAT + 16 * i + 4 * ((lane >> 4) - (D / 2) * c_out));
    }
  };
  auto step = [&](int t, const Step& S, Step& next) {
    const float2 q1 = S.q1, q2 = S.q2;
    const float th2 = S.th2;
    // unconditional (the last step re-reads its own time) so that the waits
    // for this step's operands never cover the loads just issued
    load_step(next, min(t + 1, tr.y));
    float av[W], bv[SPLIT ? 1 : W];
    uint32_t bh[SPLIT ? W / 2 : 1], bl[SPLIT ? W / 2 : 1];
    float bm[NCH], zax[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const float* G = gco_at(t, c);
      bm[c] = beam_exp2(-th2 * kb[c]);
      const float x1 = reduced_cycles(dnu[c], q1);
      const float x2 = reduced_cycles(dnu[c], q2);
      float s1, c1, s2, c2;
      sincos_rev(x1, s1, c1);
      sincos_rev(x2, s2, c2);
      // beta-axis terms of this lane's pixel: sum_n Re[omega(0, n) beta^n]
      zax[c] = 0.f;
      auto visit = [&](int n, float ar, float ai, float br, float bi) {
        if constexpr (!AXT) {
          const f4 ax = *reinterpret_cast<const f4*>(G + NMAT + 16 * RT + 4 * n);
          zax[c] = __builtin_fmaf(ax[2], br, zax[c]);   // two FMAs, no separate add
          zax[c] = __builtin_fmaf(-ax[3], bi, zax[c]);
        }
      };
      if constexpr (SPLIT) {
        powers_split_adj<D>(av + 2 * D * c, bh + D * c, bl + D * c, c1, s1, c2, s2, visit);
        // T comes out scaled by the coefficients' power of two: the weights undo it
        const float isc = G[NMAT + 16 * RT + 4 * D];
        BW[c][lane] = make_float2(bm[c] * isc, bm[c] * th2 * isc);
      } else {
        powers_f32<D>(av + 2 * D * c, bv + 2 * D * c, c1, s1, c2, s2, 1.0f, visit);
        BW[c][lane] = make_float2(bm[c], bm[c] * th2);
      }
    }
    if constexpr (SPLIT) {
#pragma unroll
      for (int r = 2 * D * NCH; r < W; ++r) av[r] = 0.f;
#pragma unroll
      for (int n = D * NCH; n < W / 2; ++n) bh[n] = bl[n] = 0u;
      if constexpr (AXT) av[2 * D] = 1.f;
      store_rows_split_adj<W>(As, Bh, Bl, lane, av, bh, bl);
    } else {
#pragma unroll
      for (int r = 2 * D * NCH; r < W; ++r) av[r] = bv[r] = 0.f;
      if constexpr (AXT) av[2 * D] = 1.f;
      store_rows<W>(As, Bs, lane, av, bv);
    }
    wave_sync();
    float2 bw[4];
#pragma unroll
    for (int pg = 0; pg < 4; ++pg) bw[pg] = BW[NCH == 1 ? 0 : c_out][16 * pg + (lane & 15)];
    // T = G Bb + alpha-axis rows for the four 16-pixel groups: the four MFMA
    // chains are interleaved (pixel group innermost) so consecutive MFMAs are
    // independent
    // B operand: lane l supplies column 4 (l >> 4) + s of the 16-column block kt
    // in MFMA step s (the coefficient layout uses the same order), so its four
    // steps' values are one 16-byte read of group l >> 4 of its pixel's row
    // (conflict-free; four scalar reads of rows 16 apart would share banks)
    // SPLIT: lane l supplies, for pixel 16 pg + (l & 15), the hi halves of
    // columns 16 kt + 8 ((l >> 4) & 1) + 0..7 (K = 32 product: lane groups 0, 1
    // meet G_hi, groups 2, 3 meet G_lo) and the lo halves of columns
    // 16 kt + 4 (l >> 4) + 0..3 (K = 16 product)
    f4 bq[SPLIT ? 1 : RT][4];
    h8 bh8[SPLIT ? RT : 1][4];
    h4 bl4[SPLIT ? RT : 1][4];
#pragma unroll
    for (int kt = 0; kt < RT; ++kt)
#pragma unroll
      for (int pg = 0; pg < 4; ++pg) {
        const int px = 16 * pg + (lane & 15);
        if constexpr (SPLIT) {
          bh8[kt][pg] = *reinterpret_cast<const h8*>(Bh + px * R::BH + 8 * kt + 4 * ((lane >> 4) & 1));
          bl4[kt][pg] = *reinterpret_cast<const h4*>(Bl + (4 * kt + (lane >> 4)) * R::BLP + 2 * px);
        } else {
          bq[kt][pg] = *reinterpret_cast<const f4*>(Bs + lds_at<W>(px, 16 * kt + 4 * (lane >> 4)));
        }
      }
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      f4 tacc[4];
      if constexpr (SPLIT) {
#pragma unroll
        for (int kt = 0; kt < RT; ++kt) {
#pragma unroll
          for (int pg = 0; pg < 4; ++pg)
            tacc[pg] = mfma_h32(S.ga[i][kt], bh8[kt][pg], kt == 0 ? S.g1[i] : tacc[pg]);
#pragma unroll
          for (int pg = 0; pg < 4; ++pg) tacc[pg] = mfma_h16(S.gb[i][kt], bl4[kt][pg], tacc[pg]);
        }
      } else {
#pragma unroll
        for (int kt = 0; kt < RT; ++kt)
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int pg = 0; pg < 4; ++pg)
              tacc[pg] = mfma4(S.gv[i][kt][s], bq[kt][pg][s], (kt == 0 && s == 0) ? S.g1[i] : tacc[pg]);
      }
#pragma unroll
      for (int pg = 0; pg < 4; ++pg) {
        const int px = 16 * pg + (lane & 15);
        const f4 av = *reinterpret_cast<const f4*>(As + lds_at<W>(px, 16 * i + 4 * (lane >> 4)));
        float zp = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) zp += av[r] * tacc[pg][r];
        pz_i[pg] += bw[pg].x * zp;
        pz_f[pg] += bw[pg].y * zp;
      }
    }
    wave_sync();
    if constexpr (!AXT) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        acc_i[c] += bm[c] * zax[c];
        acc_f[c] += bm[c] * th2 * zax[c];
      }
    }
  };
  Step sa, sb;
  load_step(sa, tr.x);
  for (int t = tr.x; t <= tr.y; t += 2) {
    step(t, sa, sb);
    if (t + 1 > tr.y) break;
    step(t + 1, sb, sa);
  }
  const int own = lane >> 4;   // this lane's pixel is column lane & 15 of group lane >> 4
  if constexpr (NCH == 1) {
    // the four row groups of each pixel sit in lanes l, l ^ 16, l ^ 32, l ^ 48
#pragma unroll
    for (int pg = 0; pg < 4; ++pg) {
      pz_i[pg] = sum_xor32(sum_xor16(pz_i[pg]));
      pz_f[pg] = sum_xor32(sum_xor16(pz_f[pg]));
    }
    acc_i[0] += own == 0 ? pz_i[0] : own == 1 ? pz_i[1] : own == 2 ? pz_i[2] : pz_i[3];
    acc_f[0] += own == 0 ? pz_f[0] : own == 1 ? pz_f[1] : own == 2 ? pz_f[2] : pz_f[3];
  } else {
    // channel c's two row groups sit in lanes 32 c + (l & 15) + {0, 16}: add
    // them, then every lane fetches each channel's total for its own pixel
#pragma unroll
    for (int pg = 0; pg < 4; ++pg) {
      pz_i[pg] = sum_xor16(pz_i[pg]);
      pz_f[pg] = sum_xor16(pz_f[pg]);
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int from = 32 * c + (lane & 15);
#pragma unroll
      for (int pg = 0; pg < 4; ++pg) {
        const float vi = __shfl(pz_i[pg], from), vf = __shfl(pz_f[pg], from);
        if (pg == own) {
          acc_i[c] += vi;
          acc_f[c] += vf;
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    if (NCH * fgrp + c >= nf) break;   // uniform over the wave
    if (args.dfull != nullptr) {        // uniform over the wave
      if (k < args.nv)
        args.dfull[static_cast<size_t>(args.voff[k]) + static_cast<size_t>(fch[c]) * args.fstride] =
            d_omega * acc_i[c];
    } else {
      dimg[static_cast<size_t>(fch[c]) * nvp + k] = d_omega * acc_i[c];
    }
    float pf = acc_f[c] * ival[c];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) pf += __shfl_xor(pf, o);
    if (lane == 0) f_part[static_cast<size_t>(fch[c]) * nchunks + chunk] = d_omega * kappa[c] * pf;
  }
}

// ------------------------------------------------------------ launchers --
template <int D>
static void fwd_d(const vis_field* f, const float* img, const float* fwhm, float2* vu, hipStream_t st) {
  constexpr int nch = fwd_channels_per_tile(D);
  const int nblk = static_cast<int>(round_up(static_cast<long>((f->n_freq + nch - 1) / nch) * f->n_time, 8));
  const auto& T = f->tab;
  const bool split = fringe_split(f);
  if (split) {
    ProfScope ps(&f->prof, "k_chan_scale", st);
    launch_k<KChanScale>(dim3(f->n_freq, kScaleParts), 0,
                         ChanScaleArgs{f->nv_pad, img, f->scr.fscale}, st, "k_chan_scale");
  }
  ProfScope ps(&f->prof, "k_fringe_fwd", st);
  const FwdArgs a{f->n_freq, f->n_time, f->nv_pad, f->n_ubl, static_cast<float>(f->d_omega),
                  T.dnu, T.sigr, T.q1, T.q2, T.th2, T.tchunk_off, T.tchunk, T.ubl_nm,
                  img, fwhm, vu, split ? f->scr.fscale : nullptr};
  if (split)
    launch_k<KFringeFwd<D, true>>(dim3(nblk), 0, a, st, "k_fringe_fwd");
  else
    launch_k<KFringeFwd<D, false>>(dim3(nblk), 0, a, st, "k_fringe_fwd");
}

template <int D>
static void adj_d(const vis_field* f, const float* img, const float* fwhm, const float* gco,
                  float* dimg, float* dfull, float* f_part, hipStream_t st) {
  constexpr int nch = adj_channels_per_tile(D);
  const int nblk = static_cast<int>(round_up(static_cast<long>((f->n_freq + nch - 1) / nch) * f->n_chunks, 8));
  const auto& T = f->tab;
  ProfScope ps(&f->prof, "k_fringe_adj", st);
  BV_REQUIRE(f->dtile == D, VIS_EINVAL, "internal: adjoint tile mismatch");
  BV_REQUIRE((dimg == nullptr) != (dfull == nullptr), VIS_EINVAL, "internal: one adjoint output");
  const AdjArgs a{f->n_freq, f->n_time, f->nv_pad, f->n_chunks, f->gstride,
                  static_cast<float>(f->d_omega), T.dnu, T.sigr, T.q1, T.q2, T.th2,
                  T.chunk_t, img, fwhm, gco, gco, dimg, f_part, dfull, T.sep_voff, f->nv,
                  f->basis->nphi_b};
  if (fringe_split(f))
    launch_k<KFringeAdj<D, true>>(dim3(nblk), 0, a, st, "k_fringe_adj");
  else
    launch_k<KFringeAdj<D, false>>(dim3(nblk), 0, a, st, "k_fringe_adj");
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

int fringe_tile_extent(int e) {
  return e <= 2 ? 2 : e <= 4 ? 4 : e <= 6 ? 6 : e <= 8 ? 8 : e <= 12 ? 12 : 16;
}

void launch_fringe_adj(const vis_field* f, const float* img, const float* fwhm, const float* gco,
                       float* dimg, float* f_part, hipStream_t st, float* dfull) {
#define BV_CALL_ADJ(DD) adj_d<DD>(f, img, fwhm, gco, dimg, dfull, f_part, st)
  BV_DISPATCH_EXTENT(f->extent, BV_CALL_ADJ);
#undef BV_CALL_ADJ
}

}  // namespace bv
