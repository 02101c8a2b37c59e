// Leapfrog / Hamiltonian kernels for HMC with a diagonal mass matrix and,
// optionally, dense per-channel gain blocks (further below).
//
// Sec. 4.2 and App. B: with M = diag(1 / minv) the kinetic energy is
// K = sum minv p^2 / 2, the drift is dq = eps minv p, and momenta are drawn as
// p = z / sqrt(minv), z ~ N(0, 1).  One leapfrog step is
//     p <- p - eps/2 grad U(q);  q <- q + eps minv p;  p <- p - eps/2 grad U(q),
// and a trajectory ends with a Metropolis test on H = U + K (FP64).
// The potential is U = chi^2 / 2 + sum a^2 / (2 C) + sum |g - 1|^2 / (2 v_g)
// (Gaussian priors; flat in F), so grad U = grad chi^2 / 2 + a / C + (g - 1) / v_g.
//
// Momenta come from Philox-4x32-10 (Salmon et al. 2011): counter (block,
// trajectory, stream, 0), key (seed lo, seed hi); each 4-word output gives
// four normals by the Box-Muller transform.  The Metropolis uniform is word 0
// of counter (0xFFFFFFFF, trajectory, stream, 1).  All per-chain reductions
// run in a fixed order, so a chain's trajectory does not depend on which
// other chains share its batch.
#include "hmc.hpp"
#include "philox.hpp"

namespace bv {

// grad U at element i from its chi^2 gradient gchi and the priors (cvar: the
// prior variance of a sky coefficient, unused for other elements); adds the
// prior part of U to acc_u.
__device__ __forceinline__ float grad_potential_v(const HmcTask& T, int i, float q, float gchi, float cvar,
                                                  double& acc_u) {
  float g = 0.5f * gchi;
  if (i < T.nalm) {
    g += q / cvar;
    acc_u += 0.5 * static_cast<double>(q) * q / cvar;
  } else if (i >= T.goff && i < T.goff + T.ngain) {
    const float dg = q - ((i - T.goff) % 2 == 0 ? 1.0f : 0.0f);
    g += dg * T.gvar_inv;
    acc_u += 0.5 * static_cast<double>(dg) * dg * T.gvar_inv;
  }
  return g;
}
__device__ __forceinline__ float grad_potential(const HmcTask& T, int i, float q, double& acc_u) {
  return grad_potential_v(T, i, q, T.gchi[i], i < T.nalm ? T.cvar[i] : 1.f, acc_u);
}

// Sums N values over the block in a fixed order (wave butterflies, then the
// four wave totals in order); every thread receives the totals.
template <int N>
__device__ void block_sum_n(double v[N], double* lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) lds[w * N + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = ((lds[k] + lds[N + k]) + lds[2 * N + k]) + lds[3 * N + k];
  __syncthreads();
}

// ---------------------------------------------------------------- NUTS --
// Sec. 4.2: the No-U-Turn sampler (Hoffman & Gelman 2014) with multinomial
// sampling inside each subtree and biased progressive sampling across
// doublings (Betancourt 2017).  A trajectory grows by doublings; doubling j
// adds 2^j leapfrog steps in a direction drawn from Philox counter
// (j, trajectory, stream, 2), starting from the trajectory's end on that
// side.  Every step is one tick: the element kernel moves the state, the
// evaluation gives the gradient, the element kernel kicks and forms the
// partial dot products of the U-turn checks, the finalize kernel takes the
// decisions in FP64 and the apply pass acts on them.  The U-turn checks of
// the subtree being built use the checkpoint scheme of iterative NUTS
// (Phan, Pradhan & Jankowiak 2019): at an even leaf n its momentum and the
// running momentum sum are stored in checkpoint popcount(n >> 1); at an odd
// leaf the spans that end at n (one per trailing one bit of n) are checked
// against checkpoints popcount(n >> 1) - ones + 1 .. popcount(n >> 1).  A span
// with end momenta p_a, p_b and momentum sum r turns when
// (M^-1 p_a).(r - (p_a + p_b)/2) <= 0 or (M^-1 p_b).(r - (p_a + p_b)/2) <= 0.
// With dense gain mass blocks the velocities M^-1 p of the gain elements come
// from k_hmc_gainblk's triangular solves and are stored for the trajectory
// ends and the checkpoints (the elementwise kernels never form them).

__device__ __forceinline__ int nuts_direction(const HmcTask& T, int j) {
  const uint4 x = philox10(make_uint4(static_cast<uint32_t>(j), T.traj, T.stream, 2u),
                           make_uint2(static_cast<uint32_t>(T.seed), static_cast<uint32_t>(T.seed >> 32)));
  return (x.x & 1u) ? 1 : -1;
}

__device__ __forceinline__ double philox_unit(const HmcTask& T, uint32_t c0, uint32_t c3) {
  return unit_open(philox10(make_uint4(c0, T.traj, T.stream, c3),
                            make_uint2(static_cast<uint32_t>(T.seed), static_cast<uint32_t>(T.seed >> 32))).x);
}

// checkpoints checked at leaf n (empty for even n)
__device__ __forceinline__ void nuts_ckpt_range(int leaf, int& lo, int& hi) {
  lo = 0;
  hi = -1;
  if (leaf & 1) {
    hi = __popc(static_cast<unsigned>(leaf) >> 1);
    lo = hi - __builtin_ctz(~static_cast<unsigned>(leaf)) + 1;
  }
}

__device__ void nuts_elem(const HmcTask& T, int lb, double* lds, int phase) {
  HmcState* st = T.st;
  const bool begin = (T.op & kOpBegin) != 0;
  // gains of a chain with dense gain blocks: momentum draw, drift and kinetic
  // energy come from k_hmc_gainblk, as do the velocities M^-1 p of the U-turn
  // checks (phase 1 forms those dots once the current velocity exists)
  const bool dense = T.lrow != nullptr;
  if (phase == 1 && !(dense && (T.op & kOpNutsPost))) return;
  if (T.op & kOpNutsApply) {
    if (!st->act) return;                            // nothing decided this tick
  } else if (!begin && st->done) {
    return;                                          // finished: a no-op step
  }
  const bool dots = phase == 1 || (!dense && (T.op & kOpNutsPost));
  const float eps = st->eps;
  float* V = T.nuts;
  const size_t vs = static_cast<size_t>(T.vstride);
  auto vec = [&](int k) { return V + static_cast<size_t>(k) * vs; };
  const int dir = begin ? nuts_direction(T, 0) : st->dir;
  const int leaf = begin ? 0 : st->leaf;
  const int depth = begin ? 0 : st->depth;
  const float e = dir > 0 ? eps : -eps;
  int ck_lo, ck_hi;
  nuts_ckpt_range(leaf, ck_lo, ck_hi);
  const bool last = leaf == (1 << depth) - 1;
  const int beg = lb * kHmcPerBlock;
  double acc[kNutsDots + 3];   // dots, then U, K, K0
#pragma unroll
  for (int k = 0; k < kNutsDots + 3; ++k) acc[k] = 0.0;
  // decisions of the finalize kernel (apply pass)
  const int a_cand = st->act_cand, a_ckpt = st->act_ckpt, a_merge = st->act_merge,
            a_prop = st->act_prop, a_finish = st->act_finish, a_dir = st->act_dir;
  for (int i0 = beg + threadIdx.x * 4; i0 < beg + kHmcPerBlock; i0 += kHmcThreads * 4) {
    float z[4];
    if (phase == 0 && (T.op & kOpNutsPre) && begin)
      normals4(T.seed, T.stream, T.traj, static_cast<uint32_t>(i0 >> 2), z);
#pragma unroll
    for (int el = 0; el < 4; ++el) {
      const int i = i0 + el;
      if (i >= T.len) break;
      if (i >= T.nalm && i < T.goff) continue;  // alignment padding: never touched
      const float mi = T.minv[i];
      const bool dg = dense && i >= T.goff && i < T.goff + T.ngain;
      if (phase == 0 && (T.op & kOpNutsPre)) {
        float q = T.q[i], p = T.p[i], g = T.grad[i];
        if (begin) {
          T.q0[i] = q;
          T.grad0[i] = g;
          vec(kNqL)[i] = q; vec(kNqR)[i] = q; vec(kNqP)[i] = q;
          vec(kNgL)[i] = g; vec(kNgR)[i] = g; vec(kNgP)[i] = g;
          vec(kNrhos)[i] = 0.f;
          if (!dg) {   // dense gains: drawn, and their ends and sums set, by k_hmc_gainblk
            p = z[el] * rsqrtf(mi);
            acc[kNutsDots + 2] += 0.5 * static_cast<double>(mi) * p * p;
            vec(kNpL)[i] = p; vec(kNpR)[i] = p;
            vec(kNrho)[i] = p;
          }
        } else if (leaf == 0) {   // a new subtree starts at the end on its side
          q = vec(dir > 0 ? kNqR : kNqL)[i];
          p = vec(dir > 0 ? kNpR : kNpL)[i];
          g = vec(dir > 0 ? kNgR : kNgL)[i];
          T.grad[i] = g;
        }
        if (!dg) {
          p -= 0.5f * e * g;
          q += e * mi * p;
        }
        T.q[i] = q;
        T.p[i] = p;
      }
      if (phase == 0 && (T.op & kOpNutsPost)) {
        const float q = T.q[i];
        const float g = grad_potential(T, i, q, acc[kNutsDots]);
        const float p = T.p[i] - 0.5f * e * g;
        if (!dg) acc[kNutsDots + 1] += 0.5 * static_cast<double>(mi) * p * p;
        T.grad[i] = g;
        T.p[i] = p;
      }
      if (dots) {
        // velocity M^-1 of a momentum: stored for dense gains, minv p otherwise
        const float p = T.p[i];
        const float vnow = dg ? vec(kNvN)[i] : mi * p;
        const float rs = vec(kNrhos)[i] + p;   // subtree momentum sum with this leaf
#pragma unroll
        for (int c = 0; c < kNutsMaxDepth; ++c) {
          if (c >= ck_lo && c <= ck_hi) {
            const float cp = vec(kNckp + c)[i];
            const float vc = dg ? vec(kNckv + c)[i] : mi * cp;
            const float adj = rs - vec(kNckr + c)[i] + 0.5f * (cp - p);
            acc[2 * c] += static_cast<double>(vc) * adj;
            acc[2 * c + 1] += static_cast<double>(vnow) * adj;
          }
        }
        if (last) {   // whole-trajectory check, used if this leaf completes the subtree
          const float po = vec(dir > 0 ? kNpL : kNpR)[i];
          const float vo = dg ? vec(dir > 0 ? kNvL : kNvR)[i] : mi * po;
          const float adj = vec(kNrho)[i] + rs - 0.5f * (po + p);
          acc[2 * kNutsMaxDepth] += static_cast<double>(vo) * adj;
          acc[2 * kNutsMaxDepth + 1] += static_cast<double>(vnow) * adj;
        }
      }
      if (T.op & kOpNutsApply) {
        const float q = T.q[i], p = T.p[i], g = T.grad[i];
        const float rs = vec(kNrhos)[i] + p;
        if (a_cand) {
          vec(kNqC)[i] = q;
          vec(kNgC)[i] = g;
        }
        if (a_ckpt >= 0) {
          vec(kNckp + a_ckpt)[i] = p;
          vec(kNckr + a_ckpt)[i] = rs;
          if (dg) vec(kNckv + a_ckpt)[i] = vec(kNvN)[i];
        }
        if (a_merge) {
          if (a_prop) {
            vec(kNqP)[i] = vec(kNqC)[i];
            vec(kNgP)[i] = vec(kNgC)[i];
          }
          vec(kNrho)[i] += rs;
          vec(kNrhos)[i] = 0.f;
          vec(a_dir > 0 ? kNqR : kNqL)[i] = q;
          vec(a_dir > 0 ? kNpR : kNpL)[i] = p;
          vec(a_dir > 0 ? kNgR : kNgL)[i] = g;
          if (dg) vec(a_dir > 0 ? kNvR : kNvL)[i] = vec(kNvN)[i];
        } else {
          vec(kNrhos)[i] = rs;
        }
        if (a_finish) {
          T.q[i] = vec(kNqP)[i];
          T.grad[i] = vec(kNgP)[i];
        }
      }
    }
  }
  if (T.op & kOpNutsApply) return;
  block_sum_n<kNutsDots + 3>(acc, lds);
  if (threadIdx.x != 0) return;
  if (phase == 0 && (T.op & kOpNutsPre) && begin) {
    T.part_k0[lb] = acc[kNutsDots + 2];
    if (lb == 0) {
      st->u0 = st->u;
      st->chi2_0 = st->chi2;
      st->u_prop = st->u;
      st->chi2_prop = st->chi2;
      st->logw = 0.0;
      st->logw_sub = -INFINITY;
      st->acc_sum = 0.0;
      st->depth = 0;
      st->leaf = 0;
      st->dir = dir;
      st->nsteps = 0;
      st->done = 0;
      st->moved = 0;
      st->act = 0;
    }
  }
  if (phase == 0 && (T.op & kOpNutsPost)) {
    T.part_u[lb] = acc[kNutsDots];
    T.part_k[lb] = acc[kNutsDots + 1];
  }
  if (dots) {
#pragma unroll
    for (int k = 0; k < kNutsDots; ++k) T.part_nuts[static_cast<size_t>(lb) * kNutsDots + k] = acc[k];
  }
}

__device__ __forceinline__ int find_task(const int* __restrict__ blk0, int ntask, int b) {
  // blk0 is an exclusive prefix over tasks of their block counts
  int lo = 0, hi = ntask - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk0[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int kNutsOps = kOpNutsPre | kOpNutsPost | kOpNutsApply;

// The NUTS element work; the same task tables as k_hmc_elem, whose tasks it skips.
__global__ void __launch_bounds__(kHmcThreads)
k_nuts_elem(const HmcTask* __restrict__ tasks, int ntask, const int* __restrict__ blk0, int phase) {
  __shared__ double red_n[4 * (kNutsDots + 3)];
  const int k = find_task(blk0, ntask, blockIdx.x);
  const HmcTask T = tasks[k];
  const int lb = blockIdx.x - blk0[k];
  if (lb >= T.nblk || !(T.op & kNutsOps)) return;
  nuts_elem(T, lb, red_n, phase);
}

// One parameter's leapfrog work on register values: q, p and g come in as
// stored (g = grad U at q) and go out updated; mi = minv, gchi and cvar are
// its chi^2 gradient and prior variance (cvar read only for sky coefficients).
__device__ __forceinline__ void hmc_elem_one(const HmcTask& T, int i, float eps, float z, float mi,
                                             float gchi, float cvar, bool dense, float& q, float& p,
                                             float& g, double& acc_u, double& acc_k, double& acc_k0) {
  if ((T.op & kOpBegin) && !dense) {
    p = z * rsqrtf(mi);
    acc_k0 += 0.5 * static_cast<double>(mi) * p * p;
  }
  if ((T.op & kOpKickDrift) && !dense) {
    p -= 0.5f * eps * g;
    q += eps * mi * p;
  }
  if (T.op & (kOpPost | kOpInit)) {
    // assemble grad U from the chi^2 gradient and the priors
    g = grad_potential_v(T, i, q, gchi, cvar, acc_u);
    if (T.op & kOpPost) {
      p -= 0.5f * eps * g;
      if (!dense) acc_k += 0.5 * static_cast<double>(mi) * p * p;
    }
  }
}

typedef float hv4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) hv4 ghv4;   // global, not flat
__device__ __forceinline__ hv4 ld4(const float* a, int i) { return *(const ghv4*)(a + i); }
__device__ __forceinline__ void st4(float* a, int i, hv4 v) { *(ghv4*)(a + i) = v; }

// One block handles kHmcPerBlock consecutive parameters of one chain, a group
// of four consecutive ones per thread.  A group that lies wholly among the
// sky coefficients, or wholly among the gains, moves through 16-byte loads
// and stores (the chain's vectors start 256-byte aligned); any other group
// (a boundary, the last parameter) goes element by element, and groups in
// the alignment padding between the two are never touched.  Either way each
// element runs hmc_elem_one in index order, so the sums do not depend on the
// path.
static_assert(kHmcPerBlock == 4 * kHmcThreads, "one group of four parameters per thread");
__global__ void __launch_bounds__(kHmcThreads)
k_hmc_elem(const HmcTask* __restrict__ tasks, int ntask, const int* __restrict__ blk0) {
  __shared__ double red[4 * 3];   // block_sum_n<3> wave totals
  const int k = find_task(blk0, ntask, blockIdx.x);
  const HmcTask T = tasks[k];
  const int lb = blockIdx.x - blk0[k];
  if (lb >= T.nblk || (T.op & kNutsOps)) return;
  HmcState* st = T.st;
  const float eps = st->eps;
  double acc_u = 0.0, acc_k = 0.0, acc_k0 = 0.0;
  if ((T.op & kOpRestore) != 0 && st->restore == 0) return;
  const int i0 = lb * kHmcPerBlock + threadIdx.x * 4;
  const bool in_alm = i0 + 4 <= T.nalm;
  const bool in_gain = i0 >= T.goff && i0 + 4 <= T.goff + T.ngain;
  const bool padding = i0 >= T.nalm && i0 + 4 <= T.goff;
  if (i0 < T.len && !padding) {
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    if (T.op & kOpBegin) normals4(T.seed, T.stream, T.traj, static_cast<uint32_t>(i0 >> 2), z);
    if ((in_alm || in_gain) && i0 + 4 <= T.len) {
      if (T.op & kOpRestore) {
        st4(T.q, i0, ld4(T.q0, i0));
        st4(T.grad, i0, ld4(T.grad0, i0));
      } else {
        const bool dense = in_gain && T.lrow != nullptr;
        const bool post = (T.op & (kOpPost | kOpInit)) != 0;
        const hv4 q4 = ld4(T.q, i0), p4 = ld4(T.p, i0), mi = ld4(T.minv, i0), g4 = ld4(T.grad, i0);
        const hv4 gc = post ? ld4(T.gchi, i0) : hv4{0.f, 0.f, 0.f, 0.f};
        const hv4 cv = post && in_alm ? ld4(T.cvar, i0) : hv4{1.f, 1.f, 1.f, 1.f};
        if (T.op & kOpBegin) {
          st4(T.q0, i0, q4);
          st4(T.grad0, i0, g4);
        }
        float q[4] = {q4.x, q4.y, q4.z, q4.w}, p[4] = {p4.x, p4.y, p4.z, p4.w};
        float g[4] = {g4.x, g4.y, g4.z, g4.w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
          hmc_elem_one(T, i0 + e, eps, z[e], mi[e], gc[e], cv[e], dense, q[e], p[e], g[e], acc_u, acc_k, acc_k0);
        if (T.op & kOpKickDrift) st4(T.q, i0, hv4{q[0], q[1], q[2], q[3]});
        if (post) st4(T.grad, i0, hv4{g[0], g[1], g[2], g[3]});
        st4(T.p, i0, hv4{p[0], p[1], p[2], p[3]});
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + e;
        if (i >= T.len) break;
        if (i >= T.nalm && i < T.goff) continue;  // alignment padding: never touched
        if (T.op & kOpRestore) {
          T.q[i] = T.q0[i];
          T.grad[i] = T.grad0[i];
          continue;
        }
        // gains under a dense block mass: momentum draw, drift and kinetic
        // energy belong to k_hmc_gainblk, which runs after this kernel
        const bool dense = T.lrow != nullptr && i >= T.goff && i < T.goff + T.ngain;
        const bool post = (T.op & (kOpPost | kOpInit)) != 0;
        float q = T.q[i], p = T.p[i], g = T.grad[i];
        if (T.op & kOpBegin) {
          T.q0[i] = q;
          T.grad0[i] = g;
        }
        hmc_elem_one(T, i, eps, z[e], T.minv[i], post ? T.gchi[i] : 0.f,
                     post && i < T.nalm ? T.cvar[i] : 1.f, dense, q, p, g, acc_u, acc_k, acc_k0);
        if (T.op & kOpKickDrift) T.q[i] = q;
        if (post) T.grad[i] = g;
        T.p[i] = p;
      }
    }
  }
  if (T.op & kOpRestore) return;
  double sums[3] = {acc_u, acc_k, acc_k0};
  block_sum_n<3>(sums, red);   // fixed order: wave butterflies, then the four wave totals
  const double su = sums[0], sk = sums[1], sk0 = sums[2];
  if (threadIdx.x == 0) {
    if (T.op & (kOpPost | kOpInit)) T.part_u[lb] = su;
    if (T.op & kOpPost) T.part_k[lb] = sk;
    if (T.op & kOpBegin) {
      T.part_k0[lb] = sk0;
      if (lb == 0) {
        st->u0 = st->u;
        st->chi2_0 = st->chi2;
      }
    }
  }
}

// ------------------------------------------------ dense gain mass blocks --
// App. B: with M_f = L L^T the kinetic energy is K = z^T z / 2 where L z = p
// (forward substitution), the velocity is M^-1 p = L^-T z (backward
// substitution after the forward one) and momenta are drawn as p = L z0; the
// inverse of M is never formed.  One wave owns one channel's block and lane l
// holds rows 4l .. 4l+3.  A sweep walks the columns in order (column-oriented
// substitution): the pivot of column j is broadcast from the lane that holds
// row j, and every lane updates its four rows from one 16-byte load of that
// column, issued kGainPrefetch columns ahead.  Blocks are padded to a
// multiple of kGainPrefetch rows with identity rows, which leave the solves
// unchanged, so the unrolled sweep needs no bounds test.
constexpr int kGainPrefetch = kGainBlockPad;

enum Sweep : int { kSweepForward, kSweepBackward, kSweepProduct };

__device__ __forceinline__ float lane_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// At m + j * nb4 sit the nb4 entries that column step j multiplies: column j
// of L (forward solve L y = x, product y = L x; from the transposed copy) or
// row j of L (backward solve L^T y = x; from the row-major copy).  rd holds
// 1 / L_ii of the lane's rows; nb4 is a multiple of kGainPrefetch.  x is consumed.  The loads are unconditional
// (the zero triangle is read too) so that the prefetch ring never waits on a
// branch; lanes past the block read its last four rows and their results
// are discarded by the caller.
template <int MODE>
__device__ void sweep(const float* __restrict__ m, int nb4, float x[4], const float rd[4],
                      float y[4]) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  typedef const __attribute__((address_space(1))) v4f gv4f;   // global, not flat
  const int lane = threadIdx.x & 63;
  const int i0 = min(4 * lane, nb4 - 4);
  y[0] = y[1] = y[2] = y[3] = 0.f;
  auto fetch = [&](int s) {
    s = min(s, nb4 - 1);
    const int j = MODE == kSweepBackward ? nb4 - 1 - s : s;
    return *(gv4f*)(m + static_cast<size_t>(j) * nb4 + i0);
  };
  // the prologue loads stay in ring order, so that at the loop head the wait
  // for slot u is the same whether the loop was entered or repeated
  v4f c[kGainPrefetch];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < kGainPrefetch; ++u) {
    c[u] = fetch(u);
    __builtin_amdgcn_sched_barrier(0);
  }
  for (int s0 = 0; s0 < nb4; s0 += kGainPrefetch) {
#pragma unroll
    for (int u = 0; u < kGainPrefetch; ++u) {
      {
        const int j = MODE == kSweepBackward ? nb4 - 1 - (s0 + u) : s0 + u;
        const int comp = MODE == kSweepBackward ? 3 - (u & 3) : (u & 3);   // j & 3
        const int jl = j >> 2;
        const float cc[4] = {c[u].x, c[u].y, c[u].z, c[u].w};
        if (MODE == kSweepProduct) {
          const float zj = lane_bcast(x[comp], jl);
#pragma unroll
          for (int r = 0; r < 4; ++r) y[r] = fmaf(cc[r], zj, y[r]);
        } else {
          const float piv = x[comp] * rd[comp];
          const float zj = lane_bcast(piv, jl);
          if (lane == jl) y[comp] = piv;
#pragma unroll
          for (int r = 0; r < 4; ++r) x[r] = fmaf(-cc[r], zj, x[r]);
        }
        // refill the slot just consumed, kGainPrefetch columns ahead.  The
        // scheduling barrier keeps the load after the slot's last use (so it
        // reuses the slot's registers and the ring needs no copies that would
        // wait on the load); the empty asm keeps the optimizer from turning
        // the ring into loads at the loop head.
        __builtin_amdgcn_sched_barrier(0);
        c[u] = fetch(s0 + u + kGainPrefetch);
        asm volatile("" ::: "memory");
      }
    }
  }
}

__device__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ float pick4(const float z[4], int k) {
  return k == 0 ? z[0] : k == 1 ? z[1] : k == 2 ? z[2] : z[3];
}

__global__ void __launch_bounds__(64)
k_hmc_gainblk(const HmcTask* __restrict__ tasks, int ntask, const int* __restrict__ chan0) {
  int lo = 0, hi = ntask - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (chan0[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const HmcTask T = tasks[lo];
  const int f = b - chan0[lo];
  if (T.lrow == nullptr || f >= T.nchan) return;   // uniform over the wave
  // NUTS chains: steps after the device ended the trajectory are no-ops, and
  // the leapfrog runs in the doubling's direction
  const bool nuts = T.nuts != nullptr;
  if (nuts && !(T.op & kOpBegin) && T.st->done) return;
  const int lane = threadIdx.x;
  const int nb = T.nb, nb4 = T.nb4;
  const size_t mo = static_cast<size_t>(f) * nb4 * nb4;
  const float* lr = T.lrow + mo;
  const float* lc = T.lcol + mo;
  const int e0 = T.goff + f * nb;     // layout index of the block's first element
  const float eps = nuts && T.st->dir < 0 ? -T.st->eps : T.st->eps;
  const bool kick = (T.op & (kOpKickDrift | kOpNutsPre)) != 0;
  auto nvec = [&](int k) { return T.nuts + static_cast<size_t>(k) * T.vstride + e0; };
  float rd[4], p[4], x[4], y[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * lane + r;
    rd[r] = i < nb4 ? 1.0f / lr[static_cast<size_t>(i) * nb4 + i] : 1.0f;
    p[r] = i < nb ? T.p[e0 + i] : 0.f;
  }
  if (T.op & kOpBegin) {
    // z0 takes the same normals a diagonal mass would use for these elements
    double k0 = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * lane + r;
      x[r] = 0.f;
      if (i < nb) {
        const int e = e0 + i;
        float z4[4];
        normals4(T.seed, T.stream, T.traj, static_cast<uint32_t>(e >> 2), z4);
        x[r] = pick4(z4, e & 3);
        k0 += 0.5 * static_cast<double>(x[r]) * x[r];
      }
    }
    sweep<kSweepProduct>(lc, nb4, x, rd, p);   // p = L z0, K0 = |z0|^2 / 2
    k0 = wave_sum_f64(k0);
    if (lane == 0) T.part_k0g[f] = k0;
    if (nuts) {
      // both trajectory ends start here: momentum, momentum sum and velocity L^-T z0
      sweep<kSweepBackward>(lr, nb4, x, rd, y);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * lane + r;
        if (i < nb) {
          nvec(kNpL)[i] = p[r];
          nvec(kNpR)[i] = p[r];
          nvec(kNrho)[i] = p[r];
          nvec(kNvL)[i] = y[r];
          nvec(kNvR)[i] = y[r];
        }
      }
    }
  }
  if (kick) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * lane + r;
      if (i < nb) p[r] -= 0.5f * eps * T.grad[e0 + i];
      x[r] = p[r];
    }
    sweep<kSweepForward>(lc, nb4, x, rd, y);    // L z = p
    sweep<kSweepBackward>(lr, nb4, y, rd, x);   // L^T v = z
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * lane + r;
      if (i < nb) T.q[e0 + i] += eps * x[r];
    }
  }
  if (T.op & (kOpEnd | kOpNutsPost)) {
    // kinetic energy of the momentum after the closing half kick (every NUTS
    // leaf needs it; fixed-length HMC only at the trajectory end) and, for
    // NUTS, the velocity L^-T z of the U-turn checks
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = p[r];
    sweep<kSweepForward>(lc, nb4, x, rd, y);
    double k = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) k += 0.5 * static_cast<double>(y[r]) * y[r];
    k = wave_sum_f64(k);
    if (lane == 0) T.part_kg[f] = k;
    if (T.op & kOpNutsPost) {
      sweep<kSweepBackward>(lr, nb4, y, rd, x);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * lane + r;
        if (i < nb) nvec(kNvN)[i] = x[r];
      }
    }
  }
  if ((T.op & kOpBegin) || kick) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * lane + r;
      if (i < nb) T.p[e0 + i] = p[r];
    }
  }
}

// Row-major padded copy and transposed copy of the caller's factors; only
// the lower triangle is read.
__global__ void __launch_bounds__(256)
k_gain_mass_setup(const float* __restrict__ chol, int nb, int nb4, float* __restrict__ lrow,
                  float* __restrict__ lcol, int* __restrict__ bad) {
  const int i = blockIdx.x;
  const size_t f = blockIdx.y;
  for (int j = threadIdx.x; j < nb4; j += blockDim.x) {
    float v = i == j ? 1.0f : 0.0f;
    if (i < nb && j <= i) {
      v = chol[(f * nb + i) * nb + j];
      if (!isfinite(v) || (i == j && !(v > 0.0f))) *bad = 1;
    }
    lrow[(f * nb4 + i) * nb4 + j] = v;
    lcol[(f * nb4 + j) * nb4 + i] = v;
  }
}

__device__ __forceinline__ double log_add_exp(double a, double b) {
  const double m = fmax(a, b);
  if (m == -INFINITY) return m;
  return m + log1p(exp(-fabs(a - b)));
}

// Decisions of one NUTS step, in FP64 on one thread (see the NUTS notes above).
__device__ void nuts_finalize(const HmcTask& T, double* lds) {
  HmcState* st = T.st;
  if (st->done) {   // a step scheduled after the trajectory finished
    if (threadIdx.x == 0) {
      st->act = 0;
      st->finished_now = 0;
      *T.st_out = *st;
    }
    return;
  }
  double v[kNutsDots + 3];   // dots, U, K, K0
#pragma unroll
  for (int k = 0; k < kNutsDots + 3; ++k) v[k] = 0.0;
  for (int b = threadIdx.x; b < T.nblk; b += kHmcThreads) {
#pragma unroll
    for (int k = 0; k < kNutsDots; ++k) v[k] += T.part_nuts[static_cast<size_t>(b) * kNutsDots + k];
    v[kNutsDots] += T.part_u[b];
    v[kNutsDots + 1] += T.part_k[b];
    v[kNutsDots + 2] += T.part_k0[b];
  }
  if (T.lrow != nullptr) {   // kinetic energies of the dense gain blocks
    for (int c = threadIdx.x; c < T.nchan; c += kHmcThreads) {
      v[kNutsDots + 1] += T.part_kg[c];
      v[kNutsDots + 2] += T.part_k0g[c];
    }
  }
  block_sum_n<kNutsDots + 3>(v, lds);
  if (threadIdx.x != 0) return;
  const double u = 0.5 * st->chi2 + v[kNutsDots];
  const double h0 = st->u0 + v[kNutsDots + 2];
  const double h = u + v[kNutsDots + 1];
  const int s = st->nsteps;
  if (s == 0) st->h_prop = h0;       // the proposal starts as the initial state
  st->nsteps = s + 1;
  st->acc_sum += isfinite(h) && isfinite(h0) ? exp(fmin(0.0, h0 - h)) : 0.0;
  st->act = 1;
  st->act_dir = st->dir;
  st->act_cand = 0;
  st->act_ckpt = -1;
  st->act_merge = 0;
  st->act_prop = 0;
  st->act_finish = 0;
  st->finished_now = 0;
  bool finish = false;
  if (!isfinite(h0) || !isfinite(h) || h - h0 > 1000.0) {
    finish = true;   // divergent leaf: its subtree is discarded
  } else {
    const double lw = h0 - h;
    const double lws = log_add_exp(st->logw_sub, lw);
    // multinomial candidate of the subtree, in progressive form
    if (philox_unit(T, static_cast<uint32_t>(s), 3u) < exp(lw - lws)) {
      st->act_cand = 1;
      st->u_cand = u;
      st->chi2_cand = st->chi2;
      st->h_cand = h;
    }
    st->logw_sub = lws;
    const int leaf = st->leaf;
    if ((leaf & 1) == 0) {
      st->act_ckpt = __popc(static_cast<unsigned>(leaf) >> 1);
    } else {
      int lo, hi;
      nuts_ckpt_range(leaf, lo, hi);
#pragma unroll
      for (int c = 0; c < kNutsMaxDepth; ++c)
        if (c >= lo && c <= hi && (v[2 * c] <= 0.0 || v[2 * c + 1] <= 0.0)) finish = true;   // a span turned
    }
    if (!finish && leaf == (1 << st->depth) - 1) {
      // subtree complete: biased progressive sampling, then the whole-trajectory check
      st->act_merge = 1;
      if (philox_unit(T, static_cast<uint32_t>(st->depth), 4u) < exp(fmin(0.0, lws - st->logw))) {
        st->act_prop = 1;
        st->u_prop = st->u_cand;
        st->chi2_prop = st->chi2_cand;
        st->h_prop = st->h_cand;
        st->moved = 1;
      }
      st->logw = log_add_exp(st->logw, lws);
      if (v[2 * kNutsMaxDepth] <= 0.0 || v[2 * kNutsMaxDepth + 1] <= 0.0 ||
          st->depth + 1 >= T.nuts_depth) {
        finish = true;
      } else {
        st->depth += 1;
        st->leaf = 0;
        st->dir = nuts_direction(T, st->depth);
        st->logw_sub = -INFINITY;
      }
    } else if (!finish) {
      st->leaf = leaf + 1;
    }
  }
  if (finish) {
    st->act_finish = 1;
    st->done = 1;
    st->finished_now = 1;
    st->u = st->u_prop;
    st->chi2 = st->chi2_prop;
    st->h0 = h0;
    st->h1 = st->h_prop;
    st->accepted = st->moved;
    st->status = isfinite(h0) ? 0 : -6;
    st->eps_used = st->eps;
    const double stat = st->acc_sum / st->nsteps;
    st->accept_stat = static_cast<float>(stat);
    if (st->adapt) {
      const float e = st->eps;
      st->eps = stat < 0.2 ? e / 1.2f : fminf(st->eps0, 1.2f * e);
    }
  } else {
    st->u = u;
  }
  *T.st_out = *st;
}

// One block per task: totals in FP64, Hamiltonian and Metropolis test at the
// end of a trajectory, step-size adaptation.
__global__ void __launch_bounds__(kHmcThreads)
k_hmc_finalize(const HmcTask* __restrict__ tasks) {
  __shared__ double red[4 * 3];   // block_sum_n<3> wave totals
  __shared__ double red_n[4 * (kNutsDots + 3)];
  const HmcTask T = tasks[blockIdx.x];
  HmcState* st = T.st;
  if (T.op & kOpNutsPost) {
    nuts_finalize(T, red_n);
    return;
  }
  double su = 0.0, sk = 0.0, sk0 = 0.0;
  for (int i = threadIdx.x; i < T.nblk; i += kHmcThreads) {
    su += T.part_u[i];
    if (T.op & kOpEnd) {
      sk += T.part_k[i];
      sk0 += T.part_k0[i];
    }
  }
  if ((T.op & kOpEnd) && T.lrow != nullptr) {
    for (int f = threadIdx.x; f < T.nchan; f += kHmcThreads) {
      sk += T.part_kg[f];
      sk0 += T.part_k0g[f];
    }
  }
  double sums[3] = {su, sk, sk0};
  block_sum_n<3>(sums, red);
  su = sums[0];
  sk = sums[1];
  sk0 = sums[2];
  if (threadIdx.x != 0) return;
  const double u = 0.5 * st->chi2 + su;
  st->u = u;
  st->restore = 0;
  if (!(T.op & kOpEnd)) {
    // a non-finite potential at the chain's own (accepted) position is an
    // error; mid-trajectory it is a divergence, rejected at the trajectory end
    if ((T.op & kOpInit) && !isfinite(u)) st->status = -6;
    *T.st_out = *st;
    return;
  }
  const double h0 = st->u0 + sk0;
  const double h1 = u + sk;
  st->h0 = h0;
  st->h1 = h1;
  const double un = unit_open(philox10(make_uint4(0xFFFFFFFFu, T.traj, T.stream, 1u),
                                       make_uint2(static_cast<uint32_t>(T.seed),
                                                  static_cast<uint32_t>(T.seed >> 32))).x);
  const bool finite = isfinite(h0) && isfinite(h1);
  const double acc_prob = finite ? exp(fmin(0.0, h0 - h1)) : 0.0;
  const int accepted = finite && un < acc_prob;
  st->accepted = accepted;
  st->accept_stat = static_cast<float>(acc_prob);
  st->status = isfinite(h0) ? 0 : -6;
  st->eps_used = st->eps;
  if (!accepted) {
    st->restore = 1;
    st->u = st->u0;
    st->chi2 = st->chi2_0;
  }
  if (st->adapt) {
    const float e = st->eps;
    st->eps = acc_prob < 0.2 ? e / 1.2f : fminf(st->eps0, 1.2f * e);
  }
  *T.st_out = *st;
}

void launch_hmc_elem(const HmcTask* tasks_dev, int ntask, const int* blk0_dev, int nblocks,
                     hipStream_t st) {
  if (ntask == 0 || nblocks == 0) return;
  k_hmc_elem<<<nblocks, kHmcThreads, 0, st>>>(tasks_dev, ntask, blk0_dev);
  check_launch("k_hmc_elem");
}

void launch_hmc_gainblk(const HmcTask* tasks_dev, int ntask, const int* chan0_dev, int nchan,
                        hipStream_t st) {
  if (ntask == 0 || nchan == 0) return;
  k_hmc_gainblk<<<nchan, 64, 0, st>>>(tasks_dev, ntask, chan0_dev);
  check_launch("k_hmc_gainblk");
}

void launch_gain_mass_setup(const float* chol, int nchan, int nb, int nb4, float* lrow,
                            float* lcol, int* bad, hipStream_t st) {
  if (nchan == 0) return;
  k_gain_mass_setup<<<dim3(nb4, nchan), 256, 0, st>>>(chol, nb, nb4, lrow, lcol, bad);
  check_launch("k_gain_mass_setup");
}

void launch_nuts_elem(const HmcTask* tasks_dev, int ntask, const int* blk0_dev, int nblocks,
                      hipStream_t st, int phase) {
  if (ntask == 0 || nblocks == 0) return;
  k_nuts_elem<<<nblocks, kHmcThreads, 0, st>>>(tasks_dev, ntask, blk0_dev, phase);
  check_launch("k_nuts_elem");
}

void launch_hmc_finalize(const HmcTask* tasks_dev, int ntask, hipStream_t st) {
  if (ntask == 0) return;
  k_hmc_finalize<<<ntask, kHmcThreads, 0, st>>>(tasks_dev);
  check_launch("k_hmc_finalize");
}

}  // namespace bv
