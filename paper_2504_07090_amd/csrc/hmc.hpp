// Internal structures of the HMC kernels and the serving runtime.
#pragma once

#include "objects.hpp"

namespace bv {

constexpr int kHmcThreads = 256;
constexpr int kHmcPerBlock = 1024;   // parameters per elementwise block (4 per thread)
constexpr int kGainBlockMax = 256;   // largest dense gain block (2 n_ant)
constexpr int kGainBlockPad = 16;    // dense gain blocks are padded to a multiple of this
constexpr int kNutsMaxDepth = 10;    // NUTS doublings (at most 2^10 - 1 leapfrog steps)
// per-block NUTS partials: U-turn dots of every checkpoint (two each), then
// the two dots of the whole-trajectory check
constexpr int kNutsDots = 2 * kNutsMaxDepth + 2;
// NUTS vectors of a chain, each of the chain's padded length: the trajectory
// ends (q, p, grad on the left and right), the subtree candidate and the
// proposal (q, grad), the momentum sums of the trajectory and of the subtree
// being built, then kNutsMaxDepth checkpoint momenta and momentum sums.
// Chains with dense gain mass blocks also keep velocities M^-1 p of the gain
// elements (of the current state, of both ends and of every checkpoint),
// which the U-turn checks need and which only the block solves give.
enum NutsVec : int {
  kNqL, kNpL, kNgL, kNqR, kNpR, kNgR, kNqC, kNgC, kNqP, kNgP, kNrho, kNrhos, kNckp,
  kNckr = kNckp + kNutsMaxDepth, kNutsVecs = kNckr + kNutsMaxDepth,
  kNvN = kNutsVecs, kNvL, kNvR, kNckv, kNutsVecsDense = kNckv + kNutsMaxDepth
};

enum HmcOp : int {
  kOpBegin = 1,        // draw p, save q0 / grad0, K0 partials
  kOpKickDrift = 2,    // p -= eps/2 grad; q += eps minv p
  kOpPost = 4,         // grad = grad chi^2 / 2 + prior; p -= eps/2 grad; U, K partials
  kOpInit = 8,         // grad and U partials at the initial position, no kick
  kOpEnd = 16,         // finalize: this evaluation ends a trajectory
  kOpRestore = 32,     // q = q0, grad = grad0 if the trajectory was rejected
  // NUTS chains (the same launches, other element work)
  kOpNutsPre = 64,     // new subtree: start from the end on its side; kick + drift by dir * eps
  kOpNutsPost = 128,   // grad, kick, U / K partials and the U-turn dots
  kOpNutsApply = 256   // act on the finalize decisions (candidate, checkpoint, merge, finish)
};

// Device-resident scalars of one chain.
struct HmcState {
  double chi2;       // chi^2 at q (written by the evaluation)
  double chi2_0;     // chi^2 at the start of the current trajectory
  double u, u0;      // potential at q / at the trajectory start
  double h0, h1;     // Hamiltonian before / after the last finished trajectory
  float eps, eps0, eps_used;
  int adapt;
  int accepted, restore, status;
  int pad;
  // NUTS (zero for fixed-length HMC)
  double logw, logw_sub;      // log total weight of the trajectory / of the subtree being built
  double acc_sum;             // sum over leaves of min(1, exp(H0 - H))
  double u_cand, chi2_cand, h_cand, u_prop, chi2_prop, h_prop;
  int depth, dir, leaf, nsteps;
  int done;                   // trajectory finished; steps until the next start are no-ops
  int finished_now;           // this step finished it (the host reports the result)
  int act;                    // this step's decisions are to be applied
  int act_cand, act_ckpt, act_merge, act_prop, act_finish;
  int act_dir;                // direction of the step being applied (the merge updates that end)
  int moved;
  float accept_stat;
};

// One chain's work in one kernel launch.
struct HmcTask {
  float* q;
  float* p;
  float* grad;       // grad U at q
  const float* gchi; // grad chi^2 at q (evaluation output)
  const float* minv;
  float* q0;
  float* grad0;
  const float* cvar; // prior variance of the sky coefficients
  double* part_u;
  double* part_k;
  double* part_k0;
  HmcState* st;
  HmcState* st_out;  // finalize copies the state here (pinned host memory) for the host
  // dense per-channel gain mass blocks M_f = L_f L_f^T (null: diagonal minv)
  const float* lrow;  // [n_freq][nb4][nb4] L row-major, padded with identity rows
  const float* lcol;  // the same blocks transposed (L column-major)
  double* part_kg;    // [n_freq] kinetic-energy partials of the gain blocks
  double* part_k0g;
  int nchan, nb, nb4; // channels, block size 2 n_ant, padded size (multiple of kGainBlockPad)
  float* nuts;        // NUTS vectors (null for fixed-length HMC), kNutsVecs x vstride floats
  double* part_nuts;  // [nblk][kNutsDots]
  int nuts_depth, vstride;
  uint64_t seed;
  int len, nalm, goff, ngain;
  float gvar_inv;
  int op, nblk;
  uint32_t stream, traj;
};

void launch_hmc_elem(const HmcTask* tasks_dev, int ntask, const int* blk0_dev, int nblocks,
                     hipStream_t st);
// One wave per (task, channel) of the tasks with dense gain blocks; chan0 is
// an exclusive prefix over tasks of their channel counts (0 for tasks
// without dense blocks).
void launch_hmc_gainblk(const HmcTask* tasks_dev, int ntask, const int* chan0_dev, int nchan,
                        hipStream_t st);
// Admission: pads / transposes the caller's factors and flags a non-positive
// or non-finite diagonal or a non-finite entry in *bad.
void launch_gain_mass_setup(const float* chol, int nchan, int nb, int nb4, float* lrow,
                            float* lcol, int* bad, hipStream_t st);
// NUTS element work over the same task tables (skips fixed-length HMC tasks,
// which k_hmc_elem handles and this kernel's tasks skip in turn).
// phase 0: the task's own op; phase 1: the U-turn dot products of NUTS chains
// with dense gain blocks (after k_hmc_gainblk has formed the current velocity).
void launch_nuts_elem(const HmcTask* tasks_dev, int ntask, const int* blk0_dev, int nblocks,
                      hipStream_t st, int phase = 0);
void launch_hmc_finalize(const HmcTask* tasks_dev, int ntask, hipStream_t st);

}  // namespace bv
