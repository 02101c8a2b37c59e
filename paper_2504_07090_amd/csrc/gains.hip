// Per-antenna gains, residual, chi^2 and the gradient bookkeeping that links
// physical baselines to the unique-baseline fringe kernels.
//
// Sec. 2.1: m_ij = g_i conj(g_j) V_ij with V_ij = V_u (b_ij = b_u) or
// conj(V_u) (b_ij = -b_u) for a real sky and beam (Sec. 3.1: unique
// baselines are broadcast to the physical ones).
// Sec. 2.3, eq. likelihood: chi^2 = sum |d - m|^2 / sigma_n^2 (FP64 total).
// With the cotangent c = dL/dRe m + i dL/dIm m (c = -2 (d - m) / sigma_n^2 for
// chi^2):
//   omega_u = sum_{ij -> +u} conj(c_ij) G_ij + sum_{ij -> -u} c_ij conj(G_ij)
//     (G_ij = g_i conj(g_j)), from which the coefficients of the adjoint fringe
//     pass are laid out directly in that kernel's MFMA operand order;
//   dL/dg_a = sum_{(a, j)} c_aj g_j conj(V_aj) + sum_{(i, a)} conj(c_ia) g_i V_ia.
// One 256-thread block per (t, nu) keeps the gains and unique visibilities of
// that slice in LDS; every reduction runs in a fixed order.
#include "batch.hpp"
#include "objects.hpp"

namespace bv {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// Dynamic LDS up to which the per-baseline terms are staged on chip (three
// complex values per baseline: 61 dishes, 1830 baselines, 46 KB).
constexpr size_t kGainsSortedLds = 64 * 1024;

struct GainArgs {
  int nt, nf, nbl, nubl, nant;
  float inv_sig2;
  const int2* bl_ant;
  const int* bl_u;
  const int4* bl_pos;
  const int* u_off;
  const int* u_list;
  const int* a_off;
  const int* a_list;
  const float2* vu;
  const float2* gains;
  const float2* din;
  float2* vis_out;
  double* chi_part;
  float* gco;
  float2* g_part;
  const int4* cplan;
  int gstride;
  int split;   // the adjoint multiplies the coefficients as FP16 hi + lo pairs
  int tslab;   // consecutive times per block
};

// Sum of v over groups of `width` consecutive lanes (width a power of two
// dividing 64), in a fixed butterfly order; every lane of a group gets the sum.
__device__ __forceinline__ float2 group_sum(float2 v, int width) {
  for (int o = 1; o < width; o <<= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  return v;
}

// Largest power of two <= 256 / n, at most 16: threads that share one list.
__host__ __device__ inline int lanes_per_item(int n) {
  int w = 1;
  while (w < 16 && 2 * w * n <= 256) w <<= 1;
  return w;
}

// FP16 hi + lo pair of x: x ~ hi + lo with hi = fp16(x), lo = fp16(x - hi).
__device__ __forceinline__ void split_f16(float x, _Float16& hi, _Float16& lo) {
  hi = static_cast<_Float16>(x);
  lo = static_cast<_Float16>(x - static_cast<float>(hi));
}
__device__ __forceinline__ float pack_f16(_Float16 a, _Float16 b) {
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(float, h2{a, b});
}

// Sum of x[e] for e = r.x, r.x + w, ... < r.y as four interleaved partial
// sums (e, e + w, e + 2w, e + 3w), added in a fixed order at the end.
__device__ __forceinline__ float2 lds_sum4(const float2* x, int2 r, int w) {
  float2 p0 = make_float2(0.f, 0.f), p1 = p0, p2 = p0, p3 = p0;
  int e = r.x;
  for (; e + 3 * w < r.y; e += 4 * w) {
    const float2 a = x[e], b = x[e + w], c = x[e + 2 * w], d = x[e + 3 * w];
    p0.x += a.x; p0.y += a.y;
    p1.x += b.x; p1.y += b.y;
    p2.x += c.x; p2.y += c.y;
    p3.x += d.x; p3.y += d.y;
  }
  for (; e < r.y; e += w) {
    p0.x += x[e].x;
    p0.y += x[e].y;
  }
  return make_float2((p0.x + p1.x) + (p2.x + p3.x), (p0.y + p1.y) + (p2.y + p3.y));
}

// Adjoint coefficients of one (t, nu) slice from the collapsed omega in LDS.
// The coefficient matrix G[r][c], r = 16 i + (row in tile) = 2 (n - 1) + (Re /
// Im of alpha^n), c = 16 kt + (column in tile) = 2 (m - 1) + (Re / Im of beta^m):
//   G = w+r + w-r (Re Re), w-r - w+r (Im Im), w-i - w+i (Re Im), -w+i - w-i (Im Re),
// w+- = omega(n, +-m).  Where the tile has a free row (adj_axis_in_tile), row
// r = 2 dtile holds the beta-axis coefficients: omega(0, m).re in column
// 2 (m - 1) and -omega(0, m).im in column 2 (m - 1) + 1.
//
// FP32 layout: entry ((i * rt + kt) * 64 + l) * 4 + s holds G[r][c] with
// r = 16 i + (l & 15), c = 16 kt + 4 (l >> 4) + s (lane l's A operand of the
// four FP32 MFMA steps of tile (i, kt)).  Then the alpha-axis accumulator
// inputs (16 rt floats, below), then for n = 1..dtile (omega(n, 0).re,
// omega(n, 0).im, omega(0, n).re, omega(0, n).im).
//
// Split layout: G is scaled by a power of two s (|s G| < 2^14) and stored as
// FP16 hi + lo pairs.  Per tile (i, kt), 64 lanes x 8 halves: lane l = (row
// l & 15, group g = l >> 4) holds, in slot j, hi(s G[r][16 kt + 8 g + j]) for
// g < 2 and lo(s G[r][16 kt + 8 (g - 2) + j]) for g >= 2 (the A operand of one
// K = 32 MFMA against [B_hi; B_hi], giving G_hi B_hi + G_lo B_hi).  Then per
// tile 64 lanes x 4 halves: hi(s G[r][16 kt + 4 g + j]) (the A operand of one
// K = 16 MFMA against B_lo).  Then the alpha-axis inputs times s, the axis
// coefficients (unscaled) and 1 / s.
//
// The layout depends only on the field, so where every entry comes from is
// worked out once on the host (coef_plan): entry e holds one or two values
// g = +-omega[a].c +- omega[b].c (c = Re or Im, either source may be absent),
// combined as its kind says.
enum CoefKind : int { kCoefZero = 0, kCoefPlain = 1, kCoefScaled = 2, kCoefPackHi = 3, kCoefPackLo = 4,
                      kCoefInvScale = 5 };

// One value of a plan entry: sources a, b (unique index + 1, 0 = none) in
// `src`, and in `fl` the component (bit 0) and the negations of a (bit 1) and
// b (bit 2).
struct CoefTerm {
  int a = 0, b = 0, comp = 0, na = 0, nb = 0;
};

static int4 pack_plan(int kind, const CoefTerm& t0, const CoefTerm& t1) {
  int4 p;
  p.x = t0.a | (t0.b << 16);
  p.y = t1.a | (t1.b << 16);
  p.z = kind | (t0.comp << 4) | (t0.na << 5) | (t0.nb << 6) | (t1.comp << 7) | (t1.na << 8) |
        (t1.nb << 9);
  p.w = 0;
  return p;
}

std::vector<int4> coef_plan(const std::vector<int>& ulut, int extent, int dtile, bool split,
                            int gstride) {
  const int lw = 2 * extent + 1;
  auto src = [&](int n1, int n2) {   // unique index + 1 of lattice (n1, n2), 0 if none
    if (n1 > extent || n2 > extent || n2 < -extent) return 0;
    const int u = ulut[n1 * lw + n2 + extent];
    return u >= 0 ? u + 1 : 0;
  };
  const bool axis_row = adj_axis_in_tile(dtile);
  auto gterm = [&](int r, int c) {   // G[r][c] as +-omega(n, m).comp +- omega(n, -m).comp
    CoefTerm t;
    const int n = (r >> 1) + 1, m = (c >> 1) + 1;
    if (axis_row && r == 2 * dtile && m <= dtile) {
      // beta-axis row, against the pixel operand's row of ones: Re(omega(0, m)
      // beta^m) = omega.re Re(beta^m) - omega.im Im(beta^m)
      t.a = src(0, m);
      t.comp = c & 1;
      t.na = c & 1;
      return t;
    }
    if (n > dtile || m > dtile) return t;
    t.a = src(n, m);
    t.b = src(n, -m);
    const int pr = r & 1, pc = c & 1;
    if (pr == 0 && pc == 0) {          // w+r + w-r
      t.comp = 0;
    } else if (pr == 1 && pc == 1) {   // w-r - w+r
      t.comp = 0;
      t.na = 1;
    } else if (pr == 0 && pc == 1) {   // w-i - w+i
      t.comp = 1;
      t.na = 1;
    } else {                           // -w+i - w-i
      t.comp = 1;
      t.na = 1;
      t.nb = 1;
    }
    return t;
  };
  const int rt = fringe_tiles(dtile);
  const int ntile = rt * rt;
  const int nmat = ntile * (split ? 384 : 256);
  std::vector<int4> plan(gstride, pack_plan(kCoefZero, CoefTerm{}, CoefTerm{}));
  for (int e = 0; e < gstride; ++e) {
    if (e < nmat) {
      if (!split) {
        const int s4 = e & 3, l = (e >> 2) & 63, blk = e >> 8;
        const int i = blk / rt, kt = blk - i * rt;
        plan[e] = pack_plan(kCoefPlain, gterm(16 * i + (l & 15), 16 * kt + 4 * (l >> 4) + s4), CoefTerm{});
      } else if (e < ntile * 256) {   // K = 32 operand: two halves per float
        const int q = e & 3, l = (e >> 2) & 63, blk = e >> 8;
        const int i = blk / rt, kt = blk - i * rt, g = l >> 4, r = 16 * i + (l & 15);
        const int c = 16 * kt + 8 * (g & 1) + 2 * q;
        plan[e] = pack_plan(g < 2 ? kCoefPackHi : kCoefPackLo, gterm(r, c), gterm(r, c + 1));
      } else {                        // K = 16 operand: hi halves
        const int e2 = e - ntile * 256;
        const int q = e2 & 1, l = (e2 >> 1) & 63, blk = e2 >> 7;
        const int i = blk / rt, kt = blk - i * rt, g = l >> 4, r = 16 * i + (l & 15);
        const int c = 16 * kt + 4 * g + 2 * q;
        plan[e] = pack_plan(kCoefPackHi, gterm(r, c), gterm(r, c + 1));
      }
    } else if (e < nmat + 16 * rt) {
      // alpha-axis accumulator input of row tile i, lane group grp: rows
      // 16 i + 4 grp + 0..3 are (Re, Im) of the powers n = 8 i + 2 grp + 1
      // and n + 1, whose coefficients are (Re, -Im) of omega(n, 0)
      const int idx = e - nmat, i = idx >> 4, grp = (idx >> 2) & 3, comp = idx & 3;
      const int n = 8 * i + 2 * grp + (comp >> 1) + 1;
      if (n <= dtile) {
        CoefTerm t;
        t.a = src(n, 0);
        t.comp = comp & 1;
        t.na = comp & 1;
        plan[e] = pack_plan(kCoefScaled, t, CoefTerm{});
      }
    } else if (e < nmat + 16 * rt + 4 * dtile) {
      const int idx = e - nmat - 16 * rt, n = idx / 4 + 1, comp = idx & 3;
      CoefTerm t;
      t.a = comp < 2 ? src(n, 0) : src(0, n);
      t.comp = comp & 1;
      plan[e] = pack_plan(kCoefPlain, t, CoefTerm{});
    } else if (split && e == nmat + 16 * rt + 4 * dtile) {
      plan[e] = pack_plan(kCoefInvScale, CoefTerm{}, CoefTerm{});
    }
  }
  return plan;
}

__device__ __forceinline__ float coef_term(const float2* om, int src, int comp, int neg) {
  if (src == 0) return 0.f;
  const float2 o = om[src - 1];
  const float v = comp ? o.y : o.x;
  return neg ? -v : v;
}

// Plan entries a thread of a 256-thread block holds in registers for a whole
// slab (entries tid and tid + 256); the rest are read per slice.
constexpr int kPlanRegs = 2;

__device__ __forceinline__ void write_coefficients(const GainArgs& a, const float2* om, size_t slice,
                                                   int tid, const int4* plan_r) {
  // split layout: power-of-two scale from the largest |omega| component
  // (|G| <= 2 max |omega|), found by the whole block
  float scale = 1.0f;
  if (a.split) {
    __shared__ float red_max[4];
    float mx = 0.f;
    for (int u = tid; u < a.nubl; u += blockDim.x) mx = fmaxf(mx, fmaxf(fabsf(om[u].x), fabsf(om[u].y)));
    for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if ((tid & 63) == 0) red_max[tid >> 6] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(red_max[0], red_max[1]), fmaxf(red_max[2], red_max[3]));
    __syncthreads();   // red_max is reused by the next slice of this block
    if (mx > 0.f && isfinite(mx)) {
      int ex;
      frexpf(mx, &ex);   // mx < 2^ex, so |G| <= 2 mx < 2^(ex + 1)
      scale = ldexpf(1.0f, min(100, 13 - ex));
    }
  }
  float* G = a.gco + slice * a.gstride;
  auto entry = [&](int e, const int4 p) {
    const int kind = p.z & 15;
    const float g0 = coef_term(om, p.x & 0xffff, (p.z >> 4) & 1, (p.z >> 5) & 1) +
                     coef_term(om, p.x >> 16, (p.z >> 4) & 1, (p.z >> 6) & 1);
    float val = 0.f;
    if (kind == kCoefPlain) {
      val = g0;
    } else if (kind == kCoefScaled) {
      val = scale * g0;
    } else if (kind == kCoefPackHi || kind == kCoefPackLo) {
      const float g1 = coef_term(om, p.y & 0xffff, (p.z >> 7) & 1, (p.z >> 8) & 1) +
                       coef_term(om, p.y >> 16, (p.z >> 7) & 1, (p.z >> 9) & 1);
      _Float16 h0, l0, h1, l1;
      split_f16(scale * g0, h0, l0);
      split_f16(scale * g1, h1, l1);
      val = kind == kCoefPackHi ? pack_f16(h0, h1) : pack_f16(l0, l1);
    } else if (kind == kCoefInvScale) {
      val = 1.0f / scale;
    }
    G[e] = val;
  };
#pragma unroll
  for (int q = 0; q < kPlanRegs; ++q) {
    const int e = tid + 256 * q;
    if (e < a.gstride) entry(e, plan_r[q]);
  }
  for (int e = tid + 256 * kPlanRegs; e < a.gstride; e += 256) entry(e, a.cplan[e]);
}

// Gains pass over (t, nu) slices.  Pass 1 walks the physical baselines in
// order (the data reads are coalesced), forming the model, the chi^2 terms and
// the cotangent of every baseline.
//
// SORTED (fields of up to kGainsMaxPerThread * 256 baselines whose staging
// fits in LDS): a block handles `tslab` consecutive times of one channel and
// keeps its baselines' table entries in registers across them.  Pass 1 also
// forms each baseline's contribution to its unique baseline's omega and to its
// two antennas' gradients and stores them in LDS at the baseline's positions
// in the per-unique and per-antenna lists, so the sums that follow run over
// contiguous LDS ranges.  Otherwise (one slice per block) the sums walk the
// lists and recompute the terms.  Each list gets `w` lanes that combine their
// partial sums with a fixed butterfly, so every result has a fixed order.
constexpr int kGainsMaxPerThread = 8;

template <bool SORTED, int MODE>
struct KGains {
  using Args = GainArgs;
  static constexpr int kThreads = 256, kWaves = 1;
  static __device__ void run(const GainArgs& a, const Blk& B);
};

template <bool SORTED, int MODE>
__device__ void KGains<SORTED, MODE>::run(const GainArgs& a, const Blk& B) {
  static_assert(!(SORTED && MODE == kGainFwd), "the forward mode walks the baselines once");
  constexpr bool kCot = MODE == kGainAdj || MODE == kGainMap;   // cotangent given
  extern __shared__ float2 sm[];
  float2* g = sm;              // [nant]
  float2* v = sm + a.nant;     // [nubl]
  float2* om = v + a.nubl;     // [nubl] collapsed coefficients omega_u
  float2* tu = om + a.nubl;    // [nbl] omega terms in u_list order (SORTED)
  float2* ta = tu + a.nbl;     // [2 nbl] antenna terms in a_list order (SORTED)
  __shared__ double red[4];
  const int f = B.x, tid = threadIdx.x;
  const int t0 = B.y * a.tslab, t1 = min(a.nt, t0 + a.tslab);
  for (int i = tid; i < a.nant; i += 256) g[i] = a.gains[static_cast<size_t>(f) * a.nant + i];
  int2 ij_r[SORTED ? kGainsMaxPerThread : 1];
  int uc_r[SORTED ? kGainsMaxPerThread : 1];
  int4 pos_r[SORTED ? kGainsMaxPerThread : 1];
  if (SORTED) {
#pragma unroll
    for (int q = 0; q < kGainsMaxPerThread; ++q) {
      const int k = tid + 256 * q;
      if (k < a.nbl) {
        ij_r[q] = a.bl_ant[k];
        uc_r[q] = a.bl_u[k];
        pos_r[q] = a.bl_pos[k];
      }
    }
  }
  // this thread's first plan entries, the same for every slice
  int4 plan_r[kPlanRegs];
#pragma unroll
  for (int q = 0; q < kPlanRegs; ++q) {
    const int e = tid + 256 * q;
    plan_r[q] = e < a.gstride ? a.cplan[e] : int4{0, 0, 0, 0};
  }
  // SORTED: the lane group of each unique baseline and antenna, and its list's
  // range, are the same for every slice of the slab (one list per group:
  // lanes_per_item(n) * n <= 256 for the n <= 256 this path admits)
  const int wu = lanes_per_item(a.nubl), wa = lanes_per_item(a.nant);
  const int u_mine = tid / wu, a_mine = tid / wa;
  int2 u_rng = make_int2(0, 0), a_rng = make_int2(0, 0);
  if (SORTED) {
    if (u_mine < a.nubl) u_rng = make_int2(a.u_off[u_mine] + (tid & (wu - 1)), a.u_off[u_mine + 1]);
    if (a_mine < a.nant) a_rng = make_int2(a.a_off[a_mine] + (tid & (wa - 1)), a.a_off[a_mine + 1]);
  }
  auto omega_term = [&](bool neg, float2 c, float2 G) {
    return neg ? cmul(c, conjf2(G)) : cmul(conjf2(c), G);
  };
  // antenna terms through h = c conj(V): role 0 (antenna i of (i, j)) takes
  // h g_j, role 1 (antenna j) takes conj(h) g_i
  auto ant_term = [&](int role, int2 ij, float2 h) {
    return role ? cmul(conjf2(h), g[ij.x]) : cmul(h, g[ij.y]);
  };
  // SORTED: the next slice's data and unique visibilities are loaded into
  // registers while the current one is processed
  float2 d_r[SORTED ? kGainsMaxPerThread : 1], v_r = make_float2(0.f, 0.f);
  auto fetch = [&](int t) {
    const size_t sl = static_cast<size_t>(t) * a.nf + f;
#pragma unroll
    for (int q = 0; q < kGainsMaxPerThread; ++q) {
      const int k = tid + 256 * q;
      if (k < a.nbl) d_r[q] = a.din[sl * a.nbl + k];
    }
    if (tid < a.nubl) v_r = a.vu[sl * a.nubl + tid];
  };
  if (SORTED && t0 < t1) fetch(t0);
  // residual r = d - m in FP32 (one rounding of a difference of two FP32
  // values), its square summed in FP64
  auto cot_from = [&](float2 dk, float2 m, double& acc) {
    if (kCot) return dk;
    const float rx = dk.x - m.x, ry = dk.y - m.y;
    if (MODE == kGainChi2) acc += static_cast<double>(__builtin_fmaf(rx, rx, ry * ry));
    return make_float2(-2.f * a.inv_sig2 * rx, -2.f * a.inv_sig2 * ry);
  };
  for (int t = t0; t < t1; ++t) {
    const size_t slice = static_cast<size_t>(t) * a.nf + f;
    __syncthreads();   // the previous slice is done with v, om, tu, ta
    float2 dcur[SORTED ? kGainsMaxPerThread : 1];
    if (SORTED) {
      if (tid < a.nubl) v[tid] = v_r;
#pragma unroll
      for (int q = 0; q < kGainsMaxPerThread; ++q) dcur[q] = d_r[q];
      __syncthreads();
      if (t + 1 < t1) fetch(t + 1);
    } else {
      for (int u = tid; u < a.nubl; u += 256) v[u] = a.vu[slice * a.nubl + u];
      __syncthreads();
    }
    const float2* din = a.din + slice * a.nbl;
    auto vis_of = [&](int k) {
      const int u = a.bl_u[k];
      return u >= 0 ? v[u] : conjf2(v[~u]);
    };
    auto gprod = [&](int k) {
      const int2 ij = a.bl_ant[k];
      return cmul(g[ij.x], conjf2(g[ij.y]));
    };
    if (MODE == kGainFwd) {
      float2* out = a.vis_out + slice * a.nbl;
      for (int k = tid; k < a.nbl; k += 256) out[k] = cmul(gprod(k), vis_of(k));
      continue;
    }
    double acc = 0.0;
    if (SORTED) {
#pragma unroll
      for (int q = 0; q < kGainsMaxPerThread; ++q) {
        const int k = tid + 256 * q;
        if (k < a.nbl) {
          const int2 ij = ij_r[q];
          const int ucode = uc_r[q];
          const float2 G = cmul(g[ij.x], conjf2(g[ij.y]));
          const float2 vk = ucode >= 0 ? v[ucode] : conjf2(v[~ucode]);
          const float2 c = cot_from(dcur[q], kCot ? make_float2(0.f, 0.f) : cmul(G, vk), acc);
          tu[pos_r[q].x] = omega_term(ucode < 0, c, G);
          if (MODE != kGainMap) {
            const float2 h = cmul(c, conjf2(vk));
            ta[pos_r[q].y] = ant_term(0, ij, h);
            ta[pos_r[q].z] = ant_term(1, ij, h);
          }
        }
      }
    } else if (MODE == kGainChi2) {
      // four baselines' global loads at once, then their terms, added in
      // baseline order
      int k = tid;
      for (; k + 3 * 256 < a.nbl; k += 4 * 256) {
        float2 d4[4];
        int2 ij4[4];
        int uc4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          d4[q] = din[k + 256 * q];
          ij4[q] = a.bl_ant[k + 256 * q];
          uc4[q] = a.bl_u[k + 256 * q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float2 G = cmul(g[ij4[q].x], conjf2(g[ij4[q].y]));
          const float2 vk = uc4[q] >= 0 ? v[uc4[q]] : conjf2(v[~uc4[q]]);
          cot_from(d4[q], cmul(G, vk), acc);
        }
      }
      for (; k < a.nbl; k += 256) cot_from(din[k], cmul(gprod(k), vis_of(k)), acc);
    }
    if (MODE == kGainChi2) {
      for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
      if ((tid & 63) == 0) red[tid >> 6] = acc;
    }
    __syncthreads();
    if (MODE == kGainChi2 && tid == 0)
      a.chi_part[slice] = ((red[0] + red[1]) + (red[2] + red[3])) * static_cast<double>(a.inv_sig2);
    if (SORTED) {
      // one list per lane group; four interleaved partial sums keep four LDS
      // reads in flight
      const float2 o = group_sum(lds_sum4(tu, u_rng, wu), wu);
      if (u_mine < a.nubl && (tid & (wu - 1)) == 0) om[u_mine] = o;
      if (MODE != kGainMap) {
        const float2 sg = group_sum(lds_sum4(ta, a_rng, wa), wa);
        if (a_mine < a.nant && (tid & (wa - 1)) == 0) a.g_part[slice * a.nant + a_mine] = sg;
      }
    } else {
      double unused = 0.0;
      // One list entry's baseline data: the list code and the gathered data,
      // antenna pair and unique-baseline code of its baseline.  The walks
      // below gather kWalk entries at once (the gathers depend on the list
      // read, so one entry at a time would wait out two memory latencies per
      // entry) and then add their terms in list order.
      struct Ent { int code; float2 d; int2 ij; int uc; };
      constexpr int kWalk = 8;
      auto gather = [&](const int* list, int e) {
        Ent x;
        x.code = list[e];
        const int k = x.code >> 1;
        x.d = din[k];
        x.ij = a.bl_ant[k];
        x.uc = a.bl_u[k];
        return x;
      };
      auto vis_e = [&](const Ent& x) { return x.uc >= 0 ? v[x.uc] : conjf2(v[~x.uc]); };
      auto gprod_e = [&](const Ent& x) { return cmul(g[x.ij.x], conjf2(g[x.ij.y])); };
      auto uterm = [&](const Ent& x) {
        const float2 G = gprod_e(x);
        const float2 c = cot_from(x.d, kCot ? make_float2(0.f, 0.f) : cmul(G, vis_e(x)), unused);
        return omega_term(x.code & 1, c, G);
      };
      auto aterm = [&](const Ent& x) {
        const float2 vk = vis_e(x);
        const float2 c = cot_from(x.d, kCot ? make_float2(0.f, 0.f) : cmul(gprod_e(x), vk), unused);
        return ant_term(x.code & 1, x.ij, cmul(c, conjf2(vk)));
      };
      // sum of term(entry) over list[e0], list[e0 + w], ... < list[e1], in order
      auto walk = [&](const int* list, int e0, int e1, int w, auto term) {
        float2 o = make_float2(0.f, 0.f);
        int e = e0;
        for (; e + (kWalk - 1) * w < e1; e += kWalk * w) {
          Ent x[kWalk];
#pragma unroll
          for (int q = 0; q < kWalk; ++q) x[q] = gather(list, e + q * w);
#pragma unroll
          for (int q = 0; q < kWalk; ++q) {
            const float2 tq = term(x[q]);
            o.x += tq.x;
            o.y += tq.y;
          }
        }
        for (; e < e1; e += w) {
          const float2 tq = term(gather(list, e));
          o.x += tq.x;
          o.y += tq.y;
        }
        return o;
      };
      const int w = lanes_per_item(a.nubl), sub = tid & (w - 1);
      for (int base = 0; base < a.nubl; base += 256 / w) {
        const int u = base + tid / w;
        float2 o = make_float2(0.f, 0.f);
        if (u < a.nubl) o = walk(a.u_list, a.u_off[u] + sub, a.u_off[u + 1], w, uterm);
        o = group_sum(o, w);
        if (u < a.nubl && sub == 0) om[u] = o;
      }
      if (MODE != kGainMap) {
        const int w2 = lanes_per_item(a.nant), sub2 = tid & (w2 - 1);
        for (int base = 0; base < a.nant; base += 256 / w2) {
          const int ant = base + tid / w2;
          float2 sg = make_float2(0.f, 0.f);
          if (ant < a.nant) sg = walk(a.a_list, a.a_off[ant] + sub2, a.a_off[ant + 1], w2, aterm);
          sg = group_sum(sg, w2);
          if (ant < a.nant && sub2 == 0) a.g_part[slice * a.nant + ant] = sg;
        }
      }
    }
    __syncthreads();
    write_coefficients(a, om, slice, tid, plan_r);
  }
}

// Sum of x[0..n) by one 1024-thread block in a fixed order: four independent
// strided partial sums per thread, then a butterfly per wave and the 16 wave
// totals in index order.  Valid in thread 0.
template <class T>
__device__ double block_sum(const T* __restrict__ x, int n, double* red) {
  const int tid = threadIdx.x;
  double p[4] = {0.0, 0.0, 0.0, 0.0};
  int i = tid;
  for (; i + 3 * 1024 < n; i += 4 * 1024) {
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] += static_cast<double>(x[i + q * 1024]);
  }
  for (int q = 0; i < n; i += 1024, ++q) p[q & 3] += static_cast<double>(x[i]);
  double acc = (p[0] + p[1]) + (p[2] + p[3]);
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  double tot = 0.0;
  if (tid == 0)
    for (int w = 0; w < 16; ++w) tot += red[w];
  return tot;
}

// grad_gains[f][a] = sum_t g_part[t][f][a]; block nblk - 2 totals chi^2 and
// block nblk - 1 dL/dF, in FP64.
struct ReduceArgs {
  int nt, nf, nant, nfpart, with_chi2;
  const double* chi_part;
  double* chi2;
  const float2* g_part;
  float2* grad_gains;
  const float* f_part;
  float* grad_fwhm;
};

struct KReduceGrads {
  using Args = ReduceArgs;
  static constexpr int kThreads = 1024, kWaves = 1;
  static __device__ void run(const ReduceArgs& a, const Blk& B);
};

__device__ void KReduceGrads::run(const ReduceArgs& a, const Blk& B) {
  const int nt = a.nt, nf = a.nf, nant = a.nant, nfpart = a.nfpart, with_chi2 = a.with_chi2;
  const double* __restrict__ chi_part = a.chi_part;
  double* chi2 = a.chi2;
  const float2* __restrict__ g_part = a.g_part;
  float2* grad_gains = a.grad_gains;
  const float* __restrict__ f_part = a.f_part;
  float* grad_fwhm = a.grad_fwhm;
  const int tid = threadIdx.x;
  if (B.x + 2 < B.nx) {
    // eight lanes per output: lane j of the group sums the times t = j mod 8
    // (two interleaved partial sums, so its loads are all in flight), then
    // the group adds its lanes in a fixed butterfly order
    const int idx = B.x * (1024 / 8) + (tid >> 3), j = tid & 7;
    if (grad_gains == nullptr) return;   // uniform over the launch
    const bool live = idx < nf * nant;
    const size_t stride = static_cast<size_t>(nf) * nant;
    float2 p0 = make_float2(0.f, 0.f), p1 = p0;
    if (live) {
      int t = j;
      for (; t + 8 < nt; t += 16) {
        const float2 v0 = g_part[static_cast<size_t>(t) * stride + idx];
        const float2 v1 = g_part[static_cast<size_t>(t + 8) * stride + idx];
        p0.x += v0.x;
        p0.y += v0.y;
        p1.x += v1.x;
        p1.y += v1.y;
      }
      if (t < nt) {
        const float2 v0 = g_part[static_cast<size_t>(t) * stride + idx];
        p0.x += v0.x;
        p0.y += v0.y;
      }
    }
    float2 s = make_float2(p0.x + p1.x, p0.y + p1.y);
    for (int o = 1; o < 8; o <<= 1) {
      s.x += __shfl_xor(s.x, o);
      s.y += __shfl_xor(s.y, o);
    }
    if (live && j == 0) grad_gains[idx] = s;
    return;
  }
  // the last two blocks: chi^2 and dL/dF, side by side
  __shared__ double red[16];
  if (B.x + 2 == B.nx) {
    if (with_chi2) {
      const double tot = block_sum(chi_part, nt * nf, red);
      if (tid == 0) *chi2 = tot;
    }
  } else if (grad_fwhm != nullptr) {
    const double tot = block_sum(f_part, nfpart, red);
    if (tid == 0) *grad_fwhm = static_cast<float>(tot);
  }
}

void launch_gains(const vis_field* f, GainMode mode, const float2* vu, const float2* gains,
                  const float2* din, float sigma_n, float2* vis_out, double* chi_part, float* gco,
                  float2* g_part, hipStream_t st) {
  GainArgs a;
  a.nt = f->n_time;
  a.nf = f->n_freq;
  a.nbl = f->n_bl;
  a.nubl = f->n_ubl;
  a.nant = f->n_ant;
  a.inv_sig2 = sigma_n > 0.f ? 1.0f / (sigma_n * sigma_n) : 0.f;
  a.bl_ant = f->tab.bl_ant;
  a.bl_u = f->tab.bl_u;
  a.bl_pos = f->tab.bl_pos;
  a.u_off = f->tab.u_off;
  a.u_list = f->tab.u_list;
  a.a_off = f->tab.a_off;
  a.a_list = f->tab.a_list;
  a.vu = vu;
  a.gains = gains;
  a.din = din;
  a.vis_out = vis_out;
  a.chi_part = chi_part;
  a.gco = gco;
  a.g_part = g_part;
  a.cplan = f->tab.cplan;
  a.gstride = f->gstride;
  a.split = fringe_split(f);
  const size_t lds = sizeof(float2) * (f->n_ant + 2 * f->n_ubl);
  BV_REQUIRE(lds <= 48 * 1024, VIS_EINVAL, "field too large for the gains pass LDS budget");
  const size_t lds_sorted = lds + 3 * sizeof(float2) * f->n_bl;
  ProfScope ps(&f->prof, "k_gains", st);
  StageScope sc(kStageGains);
  if (mode != kGainFwd && lds_sorted <= kGainsSortedLds && f->n_bl <= 256 * kGainsMaxPerThread &&
      f->n_ubl <= 256 && f->n_ant <= 256) {
    // enough times per block that the grid is about one round of resident blocks
    const long slots = static_cast<long>(f->n_cu) * std::max<long>(1, (160 * 1024) / static_cast<long>(lds_sorted + 64));
    a.tslab = std::max(1, std::min(f->n_time, ceil_div(static_cast<long>(f->n_time) * f->n_freq, slots)));
    dim3 grid(f->n_freq, ceil_div(f->n_time, a.tslab));
    if (mode == kGainChi2)
      launch_k<KGains<true, kGainChi2>>(grid, lds_sorted, a, st, "k_gains");
    else if (mode == kGainAdj)
      launch_k<KGains<true, kGainAdj>>(grid, lds_sorted, a, st, "k_gains");
    else
      launch_k<KGains<true, kGainMap>>(grid, lds_sorted, a, st, "k_gains");
  } else {
    a.tslab = 1;
    dim3 grid(f->n_freq, f->n_time);
    if (mode == kGainFwd)
      launch_k<KGains<false, kGainFwd>>(grid, lds, a, st, "k_gains");
    else if (mode == kGainChi2)
      launch_k<KGains<false, kGainChi2>>(grid, lds, a, st, "k_gains");
    else if (mode == kGainAdj)
      launch_k<KGains<false, kGainAdj>>(grid, lds, a, st, "k_gains");
    else
      launch_k<KGains<false, kGainMap>>(grid, lds, a, st, "k_gains");
  }
}

void launch_reduce_grads(const vis_field* f, bool with_chi2, const double* chi_part, double* chi2,
                         const float2* g_part, float2* grad_gains, const float* f_part,
                         float* grad_fwhm, hipStream_t st) {
  const int nblk = (grad_gains != nullptr ? ceil_div(static_cast<long>(f->n_freq) * f->n_ant, 1024 / 8) : 0) + 2;
  ProfScope ps(&f->prof, "k_reduce_grads", st);
  const ReduceArgs a{f->n_time, f->n_freq, f->n_ant, f->n_freq * f->n_chunks, with_chi2 ? 1 : 0,
                     chi_part, chi2, g_part, grad_gains, f_part, grad_fwhm};
  launch_k<KReduceGrads>(dim3(nblk), 0, a, st, "k_reduce_grads");
}

}  // namespace bv
