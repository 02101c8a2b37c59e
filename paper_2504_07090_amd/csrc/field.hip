// Basis (Y) generation and field set-up: geometry tables computed once per
// observation in FP64 on the host ("cached mode": coordinate transforms are
// prepared once and reused by every evaluation), then uploaded.
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <map>
#include <utility>
#include <vector>

#include "batch.hpp"
#include "objects.hpp"

namespace bv {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
void clear_error() { g_err[0] = '\0'; }

// ------------------------------------------------------------- profiler --
hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  BV_HIP(hipEventCreate(&e));
  return e;
}

void Profiler::drain() {
  for (auto& r : pending) {
    BV_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    BV_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    auto& t = totals[r.name];
    t.first += 1;
    t.second += ms;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
}

Profiler::~Profiler() {
  for (auto& r : pending) {
    (void)hipEventSynchronize(r.b);
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

ProfScope::ProfScope(Profiler* p_, const char* n, hipStream_t s) : p(p_), name(n), st(s) {
  // a recorded (batched) launch runs later as part of a shared grid: no timing
  if (p && p->on && thread_recorder() == nullptr) {
    a = p->get();
    BV_HIP(hipEventRecord(a, st));
  }
}

ProfScope::~ProfScope() {
  if (a != nullptr) {
    hipEvent_t b = nullptr;
    try {
      b = p->get();
    } catch (...) {
      p->pool.push_back(a);
      return;
    }
    if (hipEventRecord(b, st) == hipSuccess) {
      p->pending.push_back(Profiler::Rec{name, a, b});
      if (p->pending.size() > 4096) {
        try { p->drain(); } catch (...) {}
      }
    } else {
      p->pool.push_back(a);
      p->pool.push_back(b);
    }
  }
}

// ---------------------------------------------------------------- basis --
// Normalised associated Legendre values lambda_lm(z) = sqrt((2l+1)/(4 pi)
// (l-m)!/(l+m)!) P_l^m(z) (no Condon-Shortley phase), stored triangular
// [l(l+1)/2 + m].  Built column by column in m: the diagonal from
// lambda_mm = sqrt((2m+1)/(2m)) sqrt(1-z^2) lambda_{m-1,m-1}, then upward in l
// with the three-term recurrence whose coefficients keep every value
// normalised (no factorials are ever formed, App. A).
static void legendre_ring(int lmax, double z, double* out) {
  const double s = std::sqrt(std::max(0.0, 1.0 - z * z));
  double diag = 1.0 / std::sqrt(4.0 * kPi);
  for (int m = 0; m <= lmax; ++m) {
    if (m > 0) diag *= std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
    double prev2 = 0.0, prev1 = diag;
    out[m * (m + 1) / 2 + m] = diag;
    for (int l = m + 1; l <= lmax; ++l) {
      const double ll = l, mm = m;
      const double a = std::sqrt((4.0 * ll * ll - 1.0) / (ll * ll - mm * mm));
      const double b = (l - 1 > m)
                           ? std::sqrt(((ll - 1) * (ll - 1) - mm * mm) / (4.0 * (ll - 1) * (ll - 1) - 1.0))
                           : 0.0;
      const double cur = a * (z * prev1 - b * prev2);
      out[l * (l + 1) / 2 + m] = cur;
      prev2 = prev1;
      prev1 = cur;
    }
  }
}

__global__ void __launch_bounds__(256) k_make_basis(int nphi, int n_modes, int kpad, int ntri,
                                                    const double* __restrict__ lam,
                                                    const double* __restrict__ trig,  // [nphi][2*(lmax+1)]
                                                    int lmax, float* y32, __hip_bfloat16* ybh,
                                                    __hip_bfloat16* ybl, _Float16* yhh, _Float16* yhl) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (c >= kpad) return;
  const int j = p / nphi, k = p - j * nphi;
  double y = 0.0;
  if (c < n_modes) {
    int l = static_cast<int>(sqrtf(static_cast<float>(c)));
    while ((l + 1) * (l + 1) <= c) ++l;
    while (l * l > c) --l;
    const int m = c - l * l - l;
    const int am = m < 0 ? -m : m;
    const double lv = lam[static_cast<size_t>(j) * ntri + l * (l + 1) / 2 + am];
    const double* tr = trig + static_cast<size_t>(k) * 2 * (lmax + 1);
    if (m == 0) y = lv;
    else if (m > 0) y = 1.4142135623730951 * lv * tr[2 * am];
    else y = 1.4142135623730951 * lv * tr[2 * am + 1];
  }
  const size_t o = static_cast<size_t>(p) * kpad + c;
  if (y32) y32[o] = static_cast<float>(y);
  if (ybh) {
    const __hip_bfloat16 h = __float2bfloat16(static_cast<float>(y));
    ybh[o] = h;
    ybl[o] = __float2bfloat16(static_cast<float>(y - static_cast<double>(__bfloat162float(h))));
  }
  if (yhh) {
    const _Float16 h = static_cast<_Float16>(static_cast<float>(y));
    yhh[o] = h;
    yhl[o] = static_cast<_Float16>(static_cast<float>((y - static_cast<double>(static_cast<float>(h))) * 2048.0));
  }
}

static void carve_basis(vis_basis* b, Carver& cv) {
  const size_t n = static_cast<size_t>(b->n_pix) * b->kpad;
  b->y32 = (b->storage & 1u) ? cv.take<float>(n) : nullptr;
  b->ybh = (b->storage & 2u) ? cv.take<__hip_bfloat16>(n) : nullptr;
  b->ybl = (b->storage & 2u) ? cv.take<__hip_bfloat16>(n) : nullptr;
  b->yhh = (b->storage & 4u) ? cv.take<_Float16>(n) : nullptr;
  b->yhl = (b->storage & 4u) ? cv.take<_Float16>(n) : nullptr;
  // staging tables for the generator (Legendre values per ring, cos/sin per column)
  const size_t ntri = static_cast<size_t>(b->lmax + 1) * (b->lmax + 2) / 2;
  b->lam = cv.take<double>(static_cast<size_t>(b->nz) * ntri);
  b->trig = cv.take<double>(static_cast<size_t>(b->nphi) * 2 * (b->lmax + 1));
  if (b->storage & 8u) {
    size_t nl = 0;
    for (int m = 0; m <= b->lmax; ++m) nl += static_cast<size_t>(b->nz) * sep_lpad(b->lmax, m);
    b->sep_lam = cv.take<float>(nl);
    b->sep_loff = cv.take<int>(static_cast<size_t>(b->lmax) + 2);
    b->sep_tt = cv.take<float>(static_cast<size_t>(b->nphi_b) * b->kaz_t);
  }
}

static void basis_shape(const vis_basis_desc* d, vis_basis* b) {
  BV_REQUIRE(d != nullptr, VIS_EINVAL, "null basis descriptor");
  BV_REQUIRE(d->grid_nz >= 2 && d->grid_nz <= 8192 && d->grid_nphi >= 4 && d->grid_nphi <= 16384,
             VIS_EINVAL, "grid %d x %d out of range", d->grid_nz, d->grid_nphi);
  BV_REQUIRE(d->lmax >= 0 && d->lmax <= 512, VIS_EINVAL, "lmax %d out of range [0, 512]", d->lmax);
  BV_REQUIRE(d->storage != 0 && (d->storage & ~15u) == 0, VIS_EINVAL, "bad storage flags 0x%x",
             d->storage);
  b->nz = d->grid_nz;
  b->nphi = d->grid_nphi;
  b->lmax = d->lmax;
  b->n_pix = d->grid_nz * d->grid_nphi;
  b->n_modes = (d->lmax + 1) * (d->lmax + 1);
  b->kpad = static_cast<int>(round_up(b->n_modes, 64));
  b->storage = d->storage;
  b->kaz_t = static_cast<int>(round_up(2 * d->lmax + 1 + 2 * kSepPad, 4));
  b->nphi_b = static_cast<int>(round_up(b->nphi, kSepStep));
}

// ---------------------------------------------------------------- field --
struct HostGeometry {
  std::vector<std::pair<int, int>> ubl;  // canonical (n1, n2), sorted
  std::vector<int> bl_i, bl_j, bl_u, bl_sign;
  int extent = 0;
  std::vector<int> vpix;                 // visible pixel indices
  int nv_pad = 0;
  std::vector<double> p1, p2;            // [t][nv_pad]
  std::vector<float> th2;                // [t][nv_pad]
  std::vector<int> tlo, thi;             // per chunk
  std::vector<int> tchunk_off, tchunk;   // CSR per time
  double vis_pix_time = 0.0;             // sum over t of visible pixel count
};

static void validate_field(const vis_basis* basis, const vis_field_desc* d) {
  BV_REQUIRE(basis != nullptr && d != nullptr, VIS_EINVAL, "null basis or field descriptor");
  BV_REQUIRE(d->n_ant >= 2 && d->n_ant <= 1024, VIS_EINVAL, "n_ant %d out of range [2, 1024]",
             d->n_ant);
  BV_REQUIRE(d->ant_lattice && d->freq_hz && d->lst_rad, VIS_EINVAL, "null descriptor array");
  BV_REQUIRE(d->n_freq >= 1 && d->n_freq <= 4096, VIS_EINVAL, "n_freq %d out of range", d->n_freq);
  BV_REQUIRE(d->n_time >= 1 && d->n_time <= 4096, VIS_EINVAL, "n_time %d out of range", d->n_time);
  BV_REQUIRE(d->lmax >= 0 && d->lmax <= basis->lmax, VIS_EINVAL,
             "field lmax %d exceeds the basis lmax %d", d->lmax, basis->lmax);
  BV_REQUIRE(d->lattice_e1_m[2] == 0.0 && d->lattice_e2_m[2] == 0.0, VIS_EINVAL,
             "lattice basis must be horizontal (U = 0): the array is assumed coplanar");
  const double cross = d->lattice_e1_m[0] * d->lattice_e2_m[1] - d->lattice_e1_m[1] * d->lattice_e2_m[0];
  BV_REQUIRE(std::fabs(cross) > 1e-9, VIS_EINVAL, "lattice basis vectors are parallel");
  for (int f = 0; f < d->n_freq; ++f)
    BV_REQUIRE(std::isfinite(d->freq_hz[f]) && d->freq_hz[f] > 0.0, VIS_EINVAL,
               "frequency %d is not positive", f);
  for (int t = 0; t < d->n_time; ++t)
    BV_REQUIRE(std::isfinite(d->lst_rad[t]), VIS_EINVAL, "lst %d not finite", t);
  BV_REQUIRE(std::isfinite(d->latitude_rad) && std::fabs(d->latitude_rad) <= kPi / 2, VIS_EINVAL,
             "latitude out of range");
  BV_REQUIRE(d->beam_ref_hz > 0.0, VIS_EINVAL, "beam_ref_hz must be positive");
  BV_REQUIRE(d->precision == VIS_FP32 || d->precision == VIS_BF16X3 || d->precision == VIS_FP16X3,
             VIS_EINVAL, "precision %d is not one of VIS_FP32, VIS_BF16X3, VIS_FP16X3", d->precision);
  BV_REQUIRE(d->synthesis == VIS_SYNTH_DENSE || d->synthesis == VIS_SYNTH_SEPARABLE, VIS_EINVAL,
             "synthesis %d is not one of VIS_SYNTH_DENSE, VIS_SYNTH_SEPARABLE", d->synthesis);
  if (d->synthesis == VIS_SYNTH_SEPARABLE) {
    // the separable synthesis itself runs in FP32 at every precision; a split
    // precision then applies to the fringe products only
    BV_REQUIRE((basis->storage & 8u) != 0, VIS_EINVAL,
               "the basis was created without the separable factor tables (storage bit 3)");
  } else {
    const uint32_t need = d->precision == VIS_FP32 ? 1u : d->precision == VIS_BF16X3 ? 2u : 4u;
    BV_REQUIRE((basis->storage & need) != 0, VIS_EINVAL,
               "the basis was created without the storage this precision needs");
  }
}

static HostGeometry build_geometry(const vis_basis* basis, const vis_field_desc* d) {
  HostGeometry g;
  const int na = d->n_ant;
  // baselines (i < j), lattice differences, canonical sign
  std::map<std::pair<int, int>, int> index;
  std::vector<std::pair<int, int>> canon;
  for (int i = 0; i < na; ++i)
    for (int j = i + 1; j < na; ++j) {
      int a = d->ant_lattice[2 * i] - d->ant_lattice[2 * j];
      int b = d->ant_lattice[2 * i + 1] - d->ant_lattice[2 * j + 1];
      BV_REQUIRE(a != 0 || b != 0, VIS_EINVAL, "antennas %d and %d share a lattice site", i, j);
      int s = 1;
      if (!(a > 0 || (a == 0 && b > 0))) { a = -a; b = -b; s = -1; }
      g.bl_i.push_back(i);
      g.bl_j.push_back(j);
      g.bl_sign.push_back(s);
      canon.emplace_back(a, b);
      index[{a, b}] = 0;
      g.extent = std::max(g.extent, std::max(std::abs(a), std::abs(b)));
    }
  BV_REQUIRE(g.extent <= kMaxExtent, VIS_EINVAL, "lattice extent %d exceeds %d", g.extent, kMaxExtent);
  int u = 0;
  for (auto& kv : index) { kv.second = u++; g.ubl.push_back(kv.first); }
  for (auto& c : canon) g.bl_u.push_back(index[c]);

  // directions of every pixel at every time
  const int nz = basis->nz, nphi = basis->nphi, npix = basis->n_pix, nt = d->n_time;
  const double cphi = std::cos(d->latitude_rad), sphi = std::sin(d->latitude_rad);
  std::vector<double> E(static_cast<size_t>(nt) * npix), N(E.size()), U(E.size());
  std::vector<int> first(npix, -1), last(npix, -1), nup(npix, 0);   // times above the horizon
  for (int t = 0; t < nt; ++t)
    for (int j = 0; j < nz; ++j) {
      const double z = -1.0 + (j + 0.5) * 2.0 / nz;
      const double cd = std::sqrt(std::max(0.0, 1.0 - z * z)), sd = z;
      for (int k = 0; k < nphi; ++k) {
        const double alpha = (k + 0.5) * 2.0 * kPi / nphi;
        const double h = d->lst_rad[t] - alpha;
        const double ch = std::cos(h), sh = std::sin(h);
        const size_t o = static_cast<size_t>(t) * npix + j * nphi + k;
        E[o] = -cd * sh;
        N[o] = cphi * sd - sphi * cd * ch;
        U[o] = sphi * sd + cphi * cd * ch;
        if (U[o] > 0.0) {
          const int p = j * nphi + k;
          if (first[p] < 0) first[p] = t;
          last[p] = t;
          ++nup[p];
        }
      }
    }
  // Visible slots: the pixels above the horizon at every time first, in pixel
  // order, then the others ordered by the first and the last time they are
  // up.  Chunks of 64 slots of the second group then hold pixels that are up
  // over similar times, so the chunks a time visits (forward) and the times a
  // chunk visits (adjoint) carry few slots below the horizon, whose terms are
  // exactly zero (61 dishes, 60 times: 0.3% of the visited slots instead of
  // 6.8% in plain pixel order).
  for (int p = 0; p < npix; ++p)
    if (nup[p] == nt) g.vpix.push_back(p);
  {
    std::vector<int> rest;
    for (int p = 0; p < npix; ++p)
      if (nup[p] > 0 && nup[p] < nt) rest.push_back(p);
    std::sort(rest.begin(), rest.end(), [&](int a, int b) {
      return first[a] != first[b] ? first[a] < first[b] : last[a] != last[b] ? last[a] < last[b] : a < b;
    });
    g.vpix.insert(g.vpix.end(), rest.begin(), rest.end());
  }
  // The adjoint fringe grid deals tiles of kAdjChunkTile chunks (all
  // channels) to the XCDs in contiguous ranges and a chunk costs one step per
  // time in its range, so the chunks are regrouped into tiles of equal mean
  // cost: longest first, each to the tile of lowest mean so far that has
  // room.  The last, possibly partial chunk keeps its place (the padding
  // slots stay at the end).
  {
    const int nv0 = static_cast<int>(g.vpix.size());
    const int nck = (nv0 + kChunk - 1) / kChunk;
    if (nck > 2) {
      std::vector<int> cost(nck);
      for (int c = 0; c < nck; ++c) {
        int lo = nt, hi = -1;
        for (int k = c * kChunk; k < std::min(nv0, (c + 1) * kChunk); ++k) {
          lo = std::min(lo, first[g.vpix[k]]);
          hi = std::max(hi, last[g.vpix[k]]);
        }
        cost[c] = hi - lo + 1;
      }
      const int ntile = (nck + kAdjChunkTile - 1) / kAdjChunkTile;
      std::vector<int> room(ntile, kAdjChunkTile), size(ntile, kAdjChunkTile);
      size[ntile - 1] = room[ntile - 1] = nck - (ntile - 1) * kAdjChunkTile;
      std::vector<long> load(ntile, 0);
      std::vector<std::vector<int>> tiles(ntile);
      room[ntile - 1] -= 1;                      // the last chunk, placed at the end
      load[ntile - 1] += cost[nck - 1];
      std::vector<int> order(nck - 1);
      for (int c = 0; c < nck - 1; ++c) order[c] = c;
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
      for (int c : order) {
        int best = -1;
        for (int tt = 0; tt < ntile; ++tt) {
          if (room[tt] == 0) continue;
          // lower mean cost per chunk of the tile's capacity (cross-multiplied)
          if (best < 0 || load[tt] * size[best] < load[best] * size[tt]) best = tt;
        }
        tiles[best].push_back(c);
        load[best] += cost[c];
        room[best] -= 1;
      }
      tiles[ntile - 1].push_back(nck - 1);
      std::vector<int> vp;
      vp.reserve(nv0);
      for (const auto& tl : tiles)
        for (int c : tl)
          for (int k = c * kChunk; k < std::min(nv0, (c + 1) * kChunk); ++k) vp.push_back(g.vpix[k]);
      g.vpix.swap(vp);
    }
  }
  BV_REQUIRE(!g.vpix.empty(), VIS_EINVAL, "no pixel is above the horizon at any time");
  const int nv = static_cast<int>(g.vpix.size());
  g.nv_pad = static_cast<int>(round_up(nv, kChunk));
  const int nchunks = g.nv_pad / kChunk;
  g.p1.assign(static_cast<size_t>(nt) * g.nv_pad, 0.0);
  g.p2.assign(g.p1.size(), 0.0);
  g.th2.assign(g.p1.size(), kBelowHorizon);
  g.tlo.assign(nchunks, nt);
  g.thi.assign(nchunks, -1);
  std::vector<std::vector<int>> active(nt);
  const double* e1 = d->lattice_e1_m;
  const double* e2 = d->lattice_e2_m;
  for (int t = 0; t < nt; ++t) {
    for (int c = 0; c < nchunks; ++c) {
      bool any = false;
      for (int q = 0; q < kChunk; ++q) {
        const int k = c * kChunk + q;
        if (k >= nv) break;
        const size_t o = static_cast<size_t>(t) * npix + g.vpix[k];
        const size_t w = static_cast<size_t>(t) * g.nv_pad + k;
        g.p1[w] = (e1[0] * E[o] + e1[1] * N[o]) / kCLight;
        g.p2[w] = (e2[0] * E[o] + e2[1] * N[o]) / kCLight;
        if (U[o] > 0.0) {
          const double th = std::acos(std::min(1.0, U[o]));
          g.th2[w] = static_cast<float>(th * th);
          any = true;
          g.vis_pix_time += 1.0;
        }
      }
      if (any) {
        active[t].push_back(c);
        g.tlo[c] = std::min(g.tlo[c], t);
        g.thi[c] = std::max(g.thi[c], t);
      }
    }
  }
  g.tchunk_off.push_back(0);
  for (int t = 0; t < nt; ++t) {
    for (int c : active[t]) g.tchunk.push_back(c);
    g.tchunk_off.push_back(static_cast<int>(g.tchunk.size()));
  }
  return g;
}

static void carve_field(vis_field* f, Carver& cv, int n_tchunk) {
  const size_t nt = f->n_time, nfq = f->n_freq, nvp = f->nv_pad;
  auto& T = f->tab;
  T.dnu = cv.take<float>(nfq);
  T.sigr = cv.take<float>(nfq);
  T.vpix = cv.take<int>(nvp);
  T.q1 = cv.take<float2>(nt * nvp);
  T.q2 = cv.take<float2>(nt * nvp);
  T.th2 = cv.take<float>(nt * nvp);
  T.chunk_t = cv.take<int2>(f->n_chunks);
  T.tchunk_off = cv.take<int>(nt + 1);
  T.tchunk = cv.take<int>(std::max(1, n_tchunk));
  T.bl_ant = cv.take<int2>(f->n_bl);
  T.bl_u = cv.take<int>(f->n_bl);
  T.bl_pos = cv.take<int4>(f->n_bl);
  T.u_off = cv.take<int>(f->n_ubl + 1);
  T.u_list = cv.take<int>(f->n_bl);
  T.a_off = cv.take<int>(f->n_ant + 1);
  T.a_list = cv.take<int>(2 * static_cast<size_t>(f->n_bl));
  T.ubl_nm = cv.take<int2>(f->n_ubl);
  T.ulut = cv.take<int>(static_cast<size_t>(f->extent + 1) * (2 * f->extent + 1));
  T.cplan = cv.take<int4>(f->gstride);
  auto& S = f->scr;
  const size_t kpad = f->basis->kpad;
  const bool dense = f->synthesis == VIS_SYNTH_DENSE;
  S.img = cv.take<float>(nfq * nvp);
  if (dense) S.apad = cv.take<float>(static_cast<size_t>(round_up(f->n_freq, 64)) * kpad);
  S.dimg = cv.take<float>(nfq * nvp);
  T.vidx = cv.take<int>(f->basis->n_pix);
  if (!dense) {
    S.sep_g = cv.take<float>(static_cast<size_t>(f->basis->nz) * f->kaz * nfq);
    S.sep_dfull = cv.take<float>(static_cast<size_t>(f->basis->nz) * nfq * f->basis->nphi_b);
    S.sep_at = cv.take<float>(static_cast<size_t>(f->n_modes) * nfq);
    T.sep_kb_off = cv.take<int>(f->basis->nz + 1);
    const size_t nkb_max = static_cast<size_t>(f->basis->nz) * ceil_div(f->basis->nphi, kSepStep);
    T.sep_kb = cv.take<int>(nkb_max);
    T.sep_kb_ring = cv.take<int>(nkb_max);
    T.sep_voff = cv.take<int>(nvp);
  }
  if (f->precision != VIS_FP32) {
    const size_t nfp = static_cast<size_t>(round_up(f->n_freq, 64));
    S.dsplit = cv.take<float>(nfp * nvp);
    S.rscale = cv.take<float>(nfp);
    S.rmax = cv.take<float>(nfp * ceil_div(std::max<long>(kpad, nvp), 2048));
    S.fscale = cv.take<float>(nfq * kScaleParts);
  }
  S.vu = cv.take<float2>(nt * nfq * f->n_ubl);
  S.gco = cv.take<float>(nt * nfq * static_cast<size_t>(f->gstride));
  S.chi_part = cv.take<double>(nt * nfq);
  S.g_part = cv.take<float2>(nt * nfq * f->n_ant);
  S.f_part = cv.take<float>(nfq * f->n_chunks);
  if (dense)
    S.a_part = cv.take<float>(std::max(static_cast<size_t>(f->asplit) * nfq * kpad,
                                       static_cast<size_t>(f->fsplit) * nfq * nvp));
}

static int choose_asplit(int n_freq, int kpad, int nv_pad) {
  const int tiles = ceil_div(n_freq, 64) * (kpad / 64);
  int s = std::max(1, ceil_div(1024, tiles));
  s = std::min(s, std::max(1, nv_pad / 512));
  return std::min(s, 64);
}

static void fill_shape(vis_field* f, const vis_basis* basis, const vis_field_desc* d,
                       const HostGeometry& g) {
  f->basis = basis;
  f->n_ant = d->n_ant;
  f->n_bl = static_cast<int>(g.bl_i.size());
  f->n_ubl = static_cast<int>(g.ubl.size());
  f->n_freq = d->n_freq;
  f->n_time = d->n_time;
  f->lmax = d->lmax;
  f->n_modes = (d->lmax + 1) * (d->lmax + 1);
  f->nv = static_cast<int>(g.vpix.size());
  f->nv_pad = g.nv_pad;
  f->n_chunks = g.nv_pad / kChunk;
  f->n_tchunk = static_cast<int>(g.tchunk.size());
  f->extent = g.extent;
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
      f->n_cu = ncu;
  }
  f->dtile = fringe_tile_extent(g.extent);
  f->precision = d->precision;
  f->gstride = adj_coef_stride(f->dtile, fringe_split(f));
  f->synthesis = d->synthesis;
  f->kaz = static_cast<int>(round_up(2 * d->lmax + 1, 4));
  f->d_omega = 4.0 * kPi / basis->n_pix;
  f->beam_ref_hz = d->beam_ref_hz;
  f->fwd_macs = g.vis_pix_time * f->n_ubl * d->n_freq;
  f->asplit = choose_asplit(d->n_freq, basis->kpad, g.nv_pad);
  {
    // forward synthesis: split the modes until the grid holds ~3072 blocks
    // (about four rounds of the 3 resident 52-KB-LDS blocks per CU), so the
    // last partial round is short, keeping at least 512 modes per split
    const int tiles = ceil_div(d->n_freq, 64) * (g.nv_pad / 64);
    const int nm = (d->lmax + 1) * (d->lmax + 1);
    f->fsplit = std::max(1, std::min(ceil_div(3072, std::max(1, tiles)), std::max(1, nm / 512)));
  }
  // tuning overrides (split-K factors of the two synthesis GEMMs)
  if (const char* e = getenv("BV_FSPLIT")) f->fsplit = std::max(1, std::min(64, atoi(e)));
  if (const char* e = getenv("BV_ASPLIT")) f->asplit = std::max(1, std::min(64, atoi(e)));
}

template <class T>
static void up(T* dst, const std::vector<T>& src, hipStream_t st) {
  if (!src.empty())
    BV_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

}  // namespace bv

using namespace bv;

extern "C" {

const char* vis_last_error(void) { return g_err; }
const char* vis_version(void) { return "bayesvis 0.1 (gfx950)"; }

vis_status vis_basis_workspace_bytes(const vis_basis_desc* desc, size_t* bytes) {
  return guarded([&] {
    BV_REQUIRE(bytes != nullptr, VIS_EINVAL, "null output");
    vis_basis b;
    basis_shape(desc, &b);
    Carver cv;
    carve_basis(&b, cv);
    *bytes = cv.used;
  });
}

vis_status vis_basis_create(const vis_basis_desc* desc, void* ws, size_t bytes, void* stream,
                            vis_basis** out) {
  vis_basis* b = nullptr;
  vis_status st = guarded([&] {
    BV_REQUIRE(out != nullptr && ws != nullptr, VIS_EINVAL, "null workspace or output");
    b = new vis_basis();
    basis_shape(desc, b);
    Carver cv{static_cast<char*>(ws), bytes, 0};
    carve_basis(b, cv);
    const int ntri = (b->lmax + 1) * (b->lmax + 2) / 2;
    std::vector<double> lam(static_cast<size_t>(b->nz) * ntri), trig(static_cast<size_t>(b->nphi) * 2 * (b->lmax + 1));
    for (int j = 0; j < b->nz; ++j) legendre_ring(b->lmax, -1.0 + (j + 0.5) * 2.0 / b->nz, &lam[static_cast<size_t>(j) * ntri]);
    for (int k = 0; k < b->nphi; ++k) {
      const double alpha = (k + 0.5) * 2.0 * kPi / b->nphi;
      for (int m = 0; m <= b->lmax; ++m) {
        trig[static_cast<size_t>(k) * 2 * (b->lmax + 1) + 2 * m] = std::cos(m * alpha);
        trig[static_cast<size_t>(k) * 2 * (b->lmax + 1) + 2 * m + 1] = std::sin(m * alpha);
      }
    }
    hipStream_t s = as_stream(stream);
    double* dlam = b->lam;
    double* dtrig = b->trig;
    BV_HIP(hipMemcpyAsync(dlam, lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice, s));
    BV_HIP(hipMemcpyAsync(dtrig, trig.data(), trig.size() * sizeof(double), hipMemcpyHostToDevice, s));
    if (b->storage & 7u) {
      dim3 grid(ceil_div(b->kpad, 256), b->n_pix);
      k_make_basis<<<grid, 256, 0, s>>>(b->nphi, b->n_modes, b->kpad, ntri, dlam, dtrig, b->lmax,
                                        b->y32, b->ybh, b->ybl, b->yhh, b->yhl);
      check_launch("k_make_basis");
    }
    std::vector<float> sl, stt;   // host staging, alive until the stream synchronises
    std::vector<int> loff;
    if (b->storage & 8u) {
      // separable factors: Y(j, k; l, m) = lambda_l|m|(z_j) T_m(alpha_k)
      // Legendre factors in m-major blocks: block m holds nz rows of l = m .. lmax
      loff.assign(static_cast<size_t>(b->lmax) + 2, 0);
      for (int m = 0; m <= b->lmax; ++m) loff[m + 1] = loff[m] + b->nz * sep_lpad(b->lmax, m);
      sl.assign(static_cast<size_t>(loff[b->lmax + 1]), 0.f);
      for (int m = 0; m <= b->lmax; ++m)
        for (int j = 0; j < b->nz; ++j)
          for (int l = m; l <= b->lmax; ++l)
            sl[static_cast<size_t>(loff[m]) + static_cast<size_t>(j) * sep_lpad(b->lmax, m) + (l - m)] =
                static_cast<float>(lam[static_cast<size_t>(j) * ntri + static_cast<size_t>(l) * (l + 1) / 2 + m]);
      BV_HIP(hipMemcpyAsync(b->sep_loff, loff.data(), loff.size() * sizeof(int), hipMemcpyHostToDevice, s));
      stt.assign(static_cast<size_t>(b->nphi_b) * b->kaz_t, 0.f);
      for (int k = 0; k < b->nphi; ++k) {
        const double* tr = &trig[static_cast<size_t>(k) * 2 * (b->lmax + 1)];
        for (int m = -b->lmax; m <= b->lmax; ++m) {
          const int am = m < 0 ? -m : m;
          const double v = m == 0 ? 1.0 : m > 0 ? std::sqrt(2.0) * tr[2 * am] : std::sqrt(2.0) * tr[2 * am + 1];
          const int c = m + b->lmax + kSepPad;
          stt[static_cast<size_t>(c) * b->nphi_b + k] = static_cast<float>(v);
        }
      }
      BV_HIP(hipMemcpyAsync(b->sep_lam, sl.data(), sl.size() * sizeof(float), hipMemcpyHostToDevice, s));
      BV_HIP(hipMemcpyAsync(b->sep_tt, stt.data(), stt.size() * sizeof(float), hipMemcpyHostToDevice, s));
    }
    BV_HIP(hipStreamSynchronize(s));
    *out = b;
  });
  if (st != VIS_OK) delete b;
  return st;
}

vis_status vis_basis_destroy(vis_basis* basis) {
  delete basis;
  return VIS_OK;
}

vis_status vis_field_workspace_bytes(const vis_basis* basis, const vis_field_desc* desc,
                                     size_t* bytes) {
  return guarded([&] {
    BV_REQUIRE(bytes != nullptr, VIS_EINVAL, "null output");
    validate_field(basis, desc);
    HostGeometry g = build_geometry(basis, desc);
    vis_field f;
    fill_shape(&f, basis, desc, g);
    Carver cv;
    carve_field(&f, cv, f.n_tchunk);
    *bytes = cv.used;
  });
}

vis_status vis_field_create(const vis_basis* basis, const vis_field_desc* desc, void* ws,
                            size_t bytes, void* stream, vis_field** out) {
  vis_field* f = nullptr;
  vis_status st = guarded([&] {
    BV_REQUIRE(out != nullptr && ws != nullptr, VIS_EINVAL, "null workspace or output");
    validate_field(basis, desc);
    HostGeometry g = build_geometry(basis, desc);
    f = new vis_field();
    fill_shape(f, basis, desc, g);
    Carver cv{static_cast<char*>(ws), bytes, 0};
    carve_field(f, cv, f->n_tchunk);
    hipStream_t s = as_stream(stream);
    const int nchunks = f->n_chunks;
    std::vector<double> freq(desc->freq_hz, desc->freq_hz + desc->n_freq);
    std::vector<int> vpix(g.vpix);
    vpix.resize(g.nv_pad, 0);
    std::vector<int2> chunk_t(nchunks);
    for (int c = 0; c < nchunks; ++c) chunk_t[c] = make_int2(g.tlo[c], g.thi[c]);
    std::vector<int2> bl_ant(f->n_bl);
    std::vector<int> bl_u(f->n_bl);
    for (int k = 0; k < f->n_bl; ++k) {
      bl_ant[k] = make_int2(g.bl_i[k], g.bl_j[k]);
      bl_u[k] = g.bl_sign[k] > 0 ? g.bl_u[k] : ~g.bl_u[k];
    }
    std::vector<int4> bl_pos(f->n_bl, make_int4(0, 0, 0, 0));
    std::vector<int> u_off(f->n_ubl + 1, 0), u_list(f->n_bl);
    for (int k = 0; k < f->n_bl; ++k) u_off[g.bl_u[k] + 1]++;
    for (int u = 0; u < f->n_ubl; ++u) u_off[u + 1] += u_off[u];
    {
      std::vector<int> fill(u_off.begin(), u_off.end() - 1);
      for (int k = 0; k < f->n_bl; ++k) {
        bl_pos[k].x = fill[g.bl_u[k]];
        u_list[fill[g.bl_u[k]]++] = (k << 1) | (g.bl_sign[k] < 0);
      }
    }
    std::vector<int> a_off(f->n_ant + 1, 0), a_list(2 * static_cast<size_t>(f->n_bl));
    for (int k = 0; k < f->n_bl; ++k) { a_off[g.bl_i[k] + 1]++; a_off[g.bl_j[k] + 1]++; }
    for (int a = 0; a < f->n_ant; ++a) a_off[a + 1] += a_off[a];
    {
      std::vector<int> fill(a_off.begin(), a_off.end() - 1);
      for (int k = 0; k < f->n_bl; ++k) {
        bl_pos[k].y = fill[g.bl_i[k]];
        a_list[fill[g.bl_i[k]]++] = (k << 1) | 0;
        bl_pos[k].z = fill[g.bl_j[k]];
        a_list[fill[g.bl_j[k]]++] = (k << 1) | 1;
      }
    }
    const int D = f->extent;
    std::vector<int2> ubl_nm(f->n_ubl);
    std::vector<int> ulut(static_cast<size_t>(D + 1) * (2 * D + 1), -1);
    for (int u = 0; u < f->n_ubl; ++u) {
      ubl_nm[u] = make_int2(g.ubl[u].first, g.ubl[u].second);
      ulut[g.ubl[u].first * (2 * D + 1) + g.ubl[u].second + D] = u;
    }
    auto& T = f->tab;
    // Phase tables: nu_f p = nu_c p + (nu_f - nu_c) p.  The large part is
    // reduced modulo 1 here in FP64 (|y| <= 1/2, one rounding to FP32); the
    // kernels add the small part with one FP32 fma, |nu_f - nu_c| p being at
    // most half the band times the longest lattice delay.
    double fmin = freq[0], fmax = freq[0];
    for (double v : freq) {
      fmin = std::min(fmin, v);
      fmax = std::max(fmax, v);
    }
    const double nu_c = 0.5 * (fmin + fmax);
    std::vector<float> dnu(f->n_freq), sigr(f->n_freq);
    for (int k = 0; k < f->n_freq; ++k) {
      dnu[k] = static_cast<float>(freq[k] - nu_c);
      sigr[k] = static_cast<float>(desc->beam_ref_hz / freq[k] * kFwhmToSigma);
    }
    auto phase_table = [&](const std::vector<double>& p) {
      std::vector<float2> q(p.size());
      for (size_t i = 0; i < p.size(); ++i) {
        const double x = nu_c * p[i];
        q[i] = make_float2(static_cast<float>(x - std::rint(x)), static_cast<float>(p[i]));
      }
      return q;
    };
    up(T.dnu, dnu, s);
    up(T.sigr, sigr, s);
    up(T.vpix, vpix, s);
    // named: the host buffers of the copies stay alive until the stream is synchronised
    const std::vector<float2> q1 = phase_table(g.p1), q2 = phase_table(g.p2);
    up(T.q1, q1, s);
    up(T.q2, q2, s);
    up(T.th2, g.th2, s);
    up(T.chunk_t, chunk_t, s);
    up(T.tchunk_off, g.tchunk_off, s);
    up(T.tchunk, g.tchunk, s);
    up(T.bl_ant, bl_ant, s);
    up(T.bl_u, bl_u, s);
    up(T.bl_pos, bl_pos, s);
    up(T.u_off, u_off, s);
    up(T.u_list, u_list, s);
    up(T.a_off, a_off, s);
    up(T.a_list, a_list, s);
    up(T.ubl_nm, ubl_nm, s);
    up(T.ulut, ulut, s);
    const std::vector<int4> cplan = coef_plan(ulut, f->extent, f->dtile, fringe_split(f), f->gstride);
    up(T.cplan, cplan, s);
    // the padded tail of the sky scratch must stay finite (it is multiplied by a zero beam)
    BV_HIP(hipMemsetAsync(f->scr.img, 0, sizeof(float) * f->n_freq * f->nv_pad, s));
    std::vector<int> vidx(basis->n_pix, -1);
    for (int k = 0; k < f->nv; ++k) vidx[g.vpix[k]] = k;
    up(T.vidx, vidx, s);
    // named, like the tables above, until the stream is synchronised
    std::vector<int> kb_off, kb, kb_ring, voff;
    if (f->synthesis == VIS_SYNTH_SEPARABLE) {
      // rows of the Legendre stage beyond 2 lmax + 1 are never written: keep them zero
      BV_HIP(hipMemsetAsync(f->scr.sep_g, 0,
                            sizeof(float) * basis->nz * f->kaz * f->n_freq, s));
      // the adjoint writes dL/dI only at pixels above the horizon at some time;
      // the others stay zero
      BV_HIP(hipMemsetAsync(f->scr.sep_dfull, 0,
                            sizeof(float) * basis->nz * f->n_freq * static_cast<size_t>(basis->nphi_b), s));
      // the column batches of each ring that the azimuthal stages visit
      kb_off.assign(1, 0);
      for (int j = 0; j < basis->nz; ++j) {
        for (int k0 = 0; k0 < basis->nphi; k0 += kSepStep) {
          bool any = false;
          for (int k = k0; k < std::min(basis->nphi, k0 + kSepStep); ++k)
            any = any || vidx[static_cast<size_t>(j) * basis->nphi + k] >= 0;
          if (any) {
            kb.push_back(k0);
            kb_ring.push_back(j);
          }
        }
        kb_off.push_back(static_cast<int>(kb.size()));
      }
      f->sep_nkb = static_cast<int>(kb.size());
      up(T.sep_kb_off, kb_off, s);
      up(T.sep_kb, kb, s);
      up(T.sep_kb_ring, kb_ring, s);
      BV_REQUIRE(static_cast<double>(basis->nz) * f->n_freq * basis->nphi_b < 2147483647.0, VIS_EINVAL,
                 "separable dL/dI rows of %d x %d x %d floats exceed 32-bit offsets", basis->nz, f->n_freq,
                 basis->nphi_b);
      voff.assign(f->nv_pad, 0);
      for (int k = 0; k < f->nv; ++k) {
        const int p = g.vpix[k];
        voff[k] = (p / basis->nphi) * f->n_freq * basis->nphi_b + p % basis->nphi;
      }
      up(T.sep_voff, voff, s);
    }
    BV_HIP(hipStreamSynchronize(s));
    *out = f;
  });
  if (st != VIS_OK) delete f;
  return st;
}

vis_status vis_field_get_info(const vis_field* f, vis_field_info* info) {
  return guarded([&] {
    BV_REQUIRE(f != nullptr && info != nullptr, VIS_EINVAL, "null argument");
    info->n_ant = f->n_ant;
    info->n_bl = f->n_bl;
    info->n_ubl = f->n_ubl;
    info->n_freq = f->n_freq;
    info->n_time = f->n_time;
    info->n_pix = f->basis->n_pix;
    info->n_modes = f->n_modes;
    info->n_pix_visible = f->nv;
    info->lattice_extent = f->extent;
    info->synthesis = f->synthesis;
    info->precision = f->precision;
    info->d_omega = f->d_omega;
    info->fwd_macs = f->fwd_macs;
  });
}

vis_status vis_field_destroy(vis_field* f) {
  delete f;
  return VIS_OK;
}

vis_status vis_profile_enable(vis_field* f, int32_t enable) {
  return guarded([&] {
    BV_REQUIRE(f != nullptr, VIS_EINVAL, "null field");
    f->prof.on = enable != 0;
  });
}

vis_status vis_profile_read(vis_field* f, vis_kernel_time* out, int32_t max, int32_t* n_out,
                            int32_t reset) {
  return guarded([&] {
    BV_REQUIRE(f != nullptr && n_out != nullptr && (out != nullptr || max == 0), VIS_EINVAL,
               "null argument");
    f->prof.drain();
    int n = 0;
    for (auto& kv : f->prof.totals) {
      if (n >= max) break;
      snprintf(out[n].name, sizeof(out[n].name), "%s", kv.first.c_str());
      out[n].launches = kv.second.first;
      out[n].total_ms = kv.second.second;
      ++n;
    }
    *n_out = n;
    if (reset) f->prof.totals.clear();
  });
}

}  // extern "C"
