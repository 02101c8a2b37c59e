// Continuous-batching HMC server.
//
// Each admitted chain owns a slice of the caller's arena holding its
// position q, momentum p, gradients, inverse mass diagonal, trajectory-start
// copies, prior variances, reduction partials and a small FP64 state block.
// A worker thread runs "ticks": every chain with work left contributes one
// chi^2 + gradient request (one leapfrog step) to the tick; a tick is one
// batched elementwise launch (kick / drift / momentum draw), the evaluations,
// one batched post-kick launch, one FP64 finalize launch (energies,
// Metropolis test, step-size adaptation) and a batched restore launch.
// A fixed-length trajectory has n_leapfrog steps, so the host knows its step
// schedule in advance; a NUTS trajectory ends when the device decides, and a
// step the host scheduled after that runs as a no-op.  By default the next
// tick is built once the current one completes (one tick in flight); with
// inflight_ticks = 2 it is built and queued while the current one runs.
// Results are read back through pinned staging.  Chains admitted or
// submitted while a tick is in flight join the next tick.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "hmc.hpp"

#include "../../include/bayesvis_serve.h"

namespace bv {

static uint64_t now_ns() {
  return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                   std::chrono::steady_clock::now().time_since_epoch())
                                   .count());
}

struct ChainLayout {
  int nalm, goff, ngain, len, nblk;
  int nchan = 0, nb = 0, nb4 = 0;   // dense gain blocks (nchan = 0: none)
  size_t off_q, off_p, off_grad, off_gchi, off_minv, off_q0, off_grad0, off_cvar;
  size_t off_pu, off_pk, off_pk0, off_state;
  size_t off_lrow = 0, off_lcol = 0, off_pkg = 0, off_pk0g = 0, off_flag = 0;
  int vstride = 0;                  // NUTS vectors (vstride = 0: fixed-length HMC)
  size_t off_nuts = 0, off_pnuts = 0;
  size_t bytes;
};

static ChainLayout chain_layout(const vis_field* f, bool dense_gains, bool nuts) {
  ChainLayout L;
  L.nalm = f->n_freq * f->n_modes;
  L.goff = static_cast<int>(round_up(L.nalm, 64));
  L.ngain = 2 * f->n_freq * f->n_ant;
  L.len = L.goff + L.ngain + 1;
  L.nblk = ceil_div(L.len, kHmcPerBlock);
  Carver cv;
  auto at = [&](size_t bytes) {
    size_t off = (cv.used + 255) / 256 * 256;
    cv.used = off + bytes;
    return off;
  };
  const size_t vf = sizeof(float) * static_cast<size_t>(L.len);
  L.off_q = at(vf);
  L.off_p = at(vf);
  L.off_grad = at(vf);
  L.off_gchi = at(vf);
  L.off_minv = at(vf);
  L.off_q0 = at(vf);
  L.off_grad0 = at(vf);
  L.off_cvar = at(sizeof(float) * static_cast<size_t>(L.nalm));
  L.off_pu = at(sizeof(double) * L.nblk);
  L.off_pk = at(sizeof(double) * L.nblk);
  L.off_pk0 = at(sizeof(double) * L.nblk);
  L.off_state = at(sizeof(HmcState));
  if (dense_gains) {
    L.nchan = f->n_freq;
    L.nb = 2 * f->n_ant;
    L.nb4 = static_cast<int>(round_up(L.nb, kGainBlockPad));
    const size_t mb = sizeof(float) * static_cast<size_t>(L.nchan) * L.nb4 * L.nb4;
    L.off_lrow = at(mb);
    L.off_lcol = at(mb);
    L.off_pkg = at(sizeof(double) * L.nchan);
    L.off_pk0g = at(sizeof(double) * L.nchan);
    L.off_flag = at(sizeof(int));
  }
  if (nuts) {
    L.vstride = static_cast<int>(round_up(L.len, 64));
    const int nvec = dense_gains ? kNutsVecsDense : kNutsVecs;
    L.off_nuts = at(sizeof(float) * static_cast<size_t>(nvec) * L.vstride);
    L.off_pnuts = at(sizeof(double) * static_cast<size_t>(L.nblk) * kNutsDots);
  }
  L.bytes = round_up(cv.used, 256);
  return L;
}

// First-fit allocator over the arena in 256-byte granules.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  std::list<std::pair<size_t, size_t>> free_list;  // (offset, size), sorted
  void init(char* b, size_t c) {
    base = b;
    cap = c;
    free_list.clear();
    free_list.emplace_back(0, c);
  }
  long alloc(size_t n) {
    n = round_up(n, 256);
    for (auto it = free_list.begin(); it != free_list.end(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first;
        it->first += n;
        it->second -= n;
        if (it->second == 0) free_list.erase(it);
        return static_cast<long>(off);
      }
    }
    return -1;
  }
  void release(size_t off, size_t n) {
    n = round_up(n, 256);
    auto it = free_list.begin();
    while (it != free_list.end() && it->first < off) ++it;
    it = free_list.insert(it, {off, n});
    auto nx = std::next(it);
    if (nx != free_list.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_list.erase(nx);
    }
    if (it != free_list.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_list.erase(it);
      }
    }
  }
};

struct Chain {
  int id = -1;
  const vis_field* field = nullptr;
  const float2* data = nullptr;
  float sigma_n = 1.f;
  float gvar_inv = 0.f;
  int n_leapfrog = 1;
  int nuts_depth = 0;         // > 0: NUTS with at most this many doublings
  uint64_t seed = 0;
  uint32_t stream = 0;
  ChainLayout L{};
  long off = -1;
  char* base = nullptr;
  // host-side schedule (advanced when a tick is enqueued)
  bool initialised = false;   // initial gradient evaluation enqueued
  int pending = 0;            // trajectories submitted, not yet started
  int step = 0;               // leapfrog steps done in the running trajectory (0 = none running)
  int traj_started = 0;       // trajectories begun
  bool running = false;
  bool releasing = false;
  bool failed = false;
  int inflight = 0;           // ticks in flight that include this chain
  std::deque<uint64_t> traj_submit_ns;
  HmcState* st() const { return reinterpret_cast<HmcState*>(base + L.off_state); }
  float* ptr(size_t o) const { return reinterpret_cast<float*>(base + o); }
};

struct TickEntry {
  struct Chain* c;
  bool init;        // gradient at the admitted position (no leapfrog step)
  bool first;       // first step of a trajectory: draw the momentum
  bool ends;        // last step of a trajectory: energies and Metropolis test
  bool nuts;        // a NUTS step (the device decides where the trajectory ends)
  int traj;
  uint64_t t_enqueue;
};

struct Tick {
  std::vector<TickEntry> entries;
  hipEvent_t done = nullptr;
  int slot = 0;
};

// Pinned host staging + device table slots, one per in-flight tick.
struct Slot {
  // pinned, one allocation laid out like the device copy (task tables, then
  // prefixes) so a tick uploads both with one copy
  HmcTask* host_tasks = nullptr;     // [4][max_batch] task tables (owns the allocation)
  int* host_blk = nullptr;           // [kPrefixes][max_batch + 1] block prefixes (inside it)
  size_t table_bytes = 0;
  // pinned, fine-grained: [max_batch] states, written by the finalize kernel
  // straight over the bus (no read-back copy) and read after the tick's event
  HmcState* host_states = nullptr;
  HmcTask* dev_tasks = nullptr;      // in the arena
  int* dev_blk = nullptr;
  // argument tables and workgroup entries of the batched evaluation launches
  unsigned char* host_batch = nullptr;   // pinned
  unsigned char* dev_batch = nullptr;    // in the arena
  size_t batch_bytes = 0;
};

constexpr int kSlots = 3;
// block prefixes of a tick: pre, post and restore/apply elementwise launches,
// then the channel prefixes of the pre and post gain-block launches
constexpr int kPrefixes = 5;
constexpr int kSubStreams = 4;   // evaluation streams of a multi-stream tick (hardware queues)
// staging of the batched evaluation launches: at most this many launches per
// evaluation, each with an argument block of at most LaunchRec::args bytes
constexpr int kMaxLaunchesPerEval = 16;
inline size_t batch_stage_bytes(int max_batch) {
  return round_up(static_cast<size_t>(max_batch) * kMaxLaunchesPerEval *
                      (sizeof(LaunchRec::args) + sizeof(BatchEntry) + 64) +
                  64 * 1024, 256);
}

}  // namespace bv

using namespace bv;

struct hmc_server {
  hmc_server_config cfg{};
  hipStream_t stream = nullptr;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  std::vector<Chain*> chains;         // by id (nullptr once released)
  std::deque<hmc_result> results;
  std::deque<Tick> inflight;
  Slot slots[kSlots];
  int next_slot = 0;
  int rr = 0;                         // round-robin start
  int depth = 1;                      // ticks queued on the device at once
  hipStream_t sub[kSubStreams] = {};
  hipEvent_t ev_pre = nullptr;
  hipEvent_t ev_sub[kSubStreams] = {};
  std::vector<uint64_t> req_latency_ns;
  uint64_t n_requests = 0;
  vis_status worker_status = VIS_OK;
  std::string worker_error;

  void run();
  bool build_tick(Tick& t);
  void enqueue(Tick& t);
  void complete(Tick& t);
};

namespace {

void hip_or_throw(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    set_error("%s: %s", what, hipGetErrorString(e));
    throw Failure{VIS_EDEVICE};
  }
}

}  // namespace

bool hmc_server::build_tick(Tick& t) {
  const int n = static_cast<int>(chains.size());
  for (int k = 0; k < n && static_cast<int>(t.entries.size()) < cfg.max_batch; ++k) {
    Chain* c = chains[(rr + k) % n];
    if (c == nullptr || c->releasing || c->failed) continue;
    TickEntry e{c, false, false, false, c->nuts_depth > 0, 0, now_ns()};
    if (!c->initialised) {
      c->initialised = true;
      e.init = true;
      e.traj = -1;
    } else if (c->running) {
      c->step += 1;
      e.traj = c->traj_started - 1;
    } else if (c->pending > 0) {
      c->pending -= 1;
      c->running = true;
      c->step = 1;
      c->traj_started += 1;
      e.first = true;
      e.traj = c->traj_started - 1;
    } else {
      continue;
    }
    if (e.init) e.nuts = false;
    // fixed-length HMC knows its last step; a NUTS chain runs until the host
    // reads back that the device finished the trajectory
    if (!e.init && !e.nuts && c->step == c->n_leapfrog) {
      e.ends = true;
      c->running = false;
      c->step = 0;
    }
    c->inflight += 1;
    t.entries.push_back(e);
  }
  if (n > 0) rr = (rr + 1) % n;
  return !t.entries.empty();
}

void hmc_server::enqueue(Tick& t) {
  Slot& S = slots[t.slot];
  const int nb = cfg.max_batch;
  HmcTask* pre = S.host_tasks;
  HmcTask* post = S.host_tasks + nb;
  HmcTask* fin = S.host_tasks + 2 * nb;
  HmcTask* rst = S.host_tasks + 3 * nb;
  int* pre_blk = S.host_blk;
  int* post_blk = S.host_blk + (nb + 1);
  int* pre_chan = S.host_blk + 3 * (nb + 1);
  int* post_chan = S.host_blk + 4 * (nb + 1);
  int npre = 0, npost = 0, nrst = 0, bpre = 0, bpost = 0, cpre = 0, cpost = 0;
  int nuts_tasks = 0, hmc_tasks = 0, nuts_dense = 0;
  std::vector<const Chain*> evs;
  for (const TickEntry& e : t.entries) {
    Chain* c = e.c;
    HmcTask T{};
    T.q = c->ptr(c->L.off_q);
    T.p = c->ptr(c->L.off_p);
    T.grad = c->ptr(c->L.off_grad);
    T.gchi = c->ptr(c->L.off_gchi);
    T.minv = c->ptr(c->L.off_minv);
    T.q0 = c->ptr(c->L.off_q0);
    T.grad0 = c->ptr(c->L.off_grad0);
    T.cvar = c->ptr(c->L.off_cvar);
    T.part_u = reinterpret_cast<double*>(c->base + c->L.off_pu);
    T.part_k = reinterpret_cast<double*>(c->base + c->L.off_pk);
    T.part_k0 = reinterpret_cast<double*>(c->base + c->L.off_pk0);
    T.st = c->st();
    T.st_out = S.host_states + npost;
    T.seed = c->seed;
    T.len = c->L.len;
    T.nalm = c->L.nalm;
    T.goff = c->L.goff;
    T.ngain = c->L.ngain;
    T.gvar_inv = c->gvar_inv;
    T.nblk = c->L.nblk;
    if (c->L.nchan > 0) {
      T.lrow = c->ptr(c->L.off_lrow);
      T.lcol = c->ptr(c->L.off_lcol);
      T.part_kg = reinterpret_cast<double*>(c->base + c->L.off_pkg);
      T.part_k0g = reinterpret_cast<double*>(c->base + c->L.off_pk0g);
      T.nchan = c->L.nchan;
      T.nb = c->L.nb;
      T.nb4 = c->L.nb4;
    }
    if (c->L.vstride > 0) {
      T.nuts = c->ptr(c->L.off_nuts);
      T.part_nuts = reinterpret_cast<double*>(c->base + c->L.off_pnuts);
      T.nuts_depth = c->nuts_depth;
      T.vstride = c->L.vstride;
    }
    T.stream = c->stream;
    T.traj = static_cast<uint32_t>(e.traj < 0 ? 0 : e.traj);
    if (e.nuts) ++nuts_tasks; else ++hmc_tasks;
    if (e.nuts && c->L.nchan > 0) ++nuts_dense;
    const bool is_init = e.init;
    // pre-evaluation: momentum draw at a trajectory start, then kick + drift
    if (!is_init) {
      HmcTask P = T;
      P.op = (e.nuts ? kOpNutsPre : kOpKickDrift) | (e.first ? kOpBegin : 0);
      pre_blk[npre] = bpre;
      pre_chan[npre] = cpre;
      pre[npre++] = P;
      bpre += P.nblk;
      cpre += c->L.nchan;
    }
    HmcTask Q = T;
    Q.op = is_init ? kOpInit : e.nuts ? kOpNutsPost : (kOpPost | (e.ends ? kOpEnd : 0));
    post_blk[npost] = bpost;
    post_chan[npost] = cpost;
    post[npost] = Q;
    fin[npost] = Q;
    npost++;
    bpost += Q.nblk;
    // the gain blocks' kinetic energy: at a fixed-length trajectory's end, at
    // every NUTS step (with the velocity of the U-turn checks)
    if (e.ends || (e.nuts && !is_init)) cpost += c->L.nchan;
    if (e.ends || (e.nuts && !is_init)) {
      HmcTask R = T;
      R.op = e.nuts ? kOpNutsApply : kOpRestore;
      rst[nrst++] = R;
    }
    evs.push_back(c);
  }
  pre_blk[npre] = bpre;
  post_blk[npost] = bpost;
  pre_chan[npre] = cpre;
  post_chan[npost] = cpost;
  // restore tasks reuse the post block prefix layout of their own list
  std::vector<int> rst_blk(nrst + 1, 0);
  for (int i = 0; i < nrst; ++i) rst_blk[i + 1] = rst_blk[i] + rst[i].nblk;
  int* rst_blk_host = S.host_blk + 2 * (nb + 1);
  std::memcpy(rst_blk_host, rst_blk.data(), sizeof(int) * (nrst + 1));

  hip_or_throw(hipMemcpyAsync(S.dev_tasks, S.host_tasks, S.table_bytes, hipMemcpyHostToDevice, stream),
               "task table upload");
  if (hmc_tasks) launch_hmc_elem(S.dev_tasks, npre, S.dev_blk, bpre, stream);
  if (nuts_tasks) launch_nuts_elem(S.dev_tasks, npre, S.dev_blk, bpre, stream);
  launch_hmc_gainblk(S.dev_tasks, npre, S.dev_blk + 3 * (nb + 1), cpre, stream);
  // evaluations.  Batched (cfg.batched == 1): every kernel of the evaluation
  // sequence runs as one grid over all chains of the tick that need it (the
  // chains grouped by their kernel sequence, one grid per launch of the
  // sequence, each group on a stream of its own).  Multi-stream
  // (cfg.batched == 2): each chain's sequence is launched on its own, spread
  // over several streams so that kernels of different fields overlap.
  if (cfg.batched == 1 && !evs.empty()) {
    Recorder rec;
    struct Install {
      explicit Install(Recorder* r) { thread_recorder() = r; }
      ~Install() { thread_recorder() = nullptr; }
    };
    {
      Install in(&rec);
      for (const Chain* c : evs) {
        rec.begin_eval();
        const float* q = c->ptr(c->L.off_q);
        float* g = c->ptr(c->L.off_gchi);
        const vis_status s = chi2_and_grad(
            c->field, reinterpret_cast<const vis_c64*>(c->data), c->sigma_n, q,
            reinterpret_cast<const vis_c64*>(q + c->L.goff), q + c->L.len - 1, &c->st()->chi2, g,
            reinterpret_cast<vis_c64*>(g + c->L.goff), g + c->L.len - 1, stream);
        if (s != VIS_OK) throw Failure{s};
      }
    }
    hipEvent_t evs_b[kSubStreams + 1];
    for (int i = 0; i < kSubStreams; ++i) evs_b[i] = ev_sub[i];
    evs_b[kSubStreams] = ev_pre;
    run_batched(rec, S.host_batch, S.dev_batch, S.batch_bytes, stream, kSubStreams, sub, evs_b);
    evs.clear();
  }
  const int nsub = (cfg.batched == 2 && evs.size() > 1) ? std::min<int>(kSubStreams, evs.size()) : 0;
  if (nsub > 0) {
    hip_or_throw(hipEventRecord(ev_pre, stream), "event record");
    for (int i = 0; i < nsub; ++i) hip_or_throw(hipStreamWaitEvent(sub[i], ev_pre, 0), "stream wait");
  }
  for (size_t k = 0; k < evs.size(); ++k) {
    const Chain* c = evs[k];
    const float* q = c->ptr(c->L.off_q);
    float* g = c->ptr(c->L.off_gchi);
    hipStream_t es = nsub > 0 ? sub[k % nsub] : stream;
    const vis_status s = chi2_and_grad(
        c->field, reinterpret_cast<const vis_c64*>(c->data), c->sigma_n, q,
        reinterpret_cast<const vis_c64*>(q + c->L.goff), q + c->L.len - 1, &c->st()->chi2, g,
        reinterpret_cast<vis_c64*>(g + c->L.goff), g + c->L.len - 1, es);
    if (s != VIS_OK) throw Failure{s};
  }
  for (int i = 0; i < nsub; ++i) {
    hip_or_throw(hipEventRecord(ev_sub[i], sub[i]), "event record");
    hip_or_throw(hipStreamWaitEvent(stream, ev_sub[i], 0), "stream wait");
  }
  launch_hmc_elem(S.dev_tasks + nb, npost, S.dev_blk + (nb + 1), bpost, stream);
  if (nuts_tasks) launch_nuts_elem(S.dev_tasks + nb, npost, S.dev_blk + (nb + 1), bpost, stream);
  launch_hmc_gainblk(S.dev_tasks + nb, npost, S.dev_blk + 4 * (nb + 1), cpost, stream);
  if (nuts_dense)   // U-turn dots of NUTS chains with dense gain blocks (need the velocities)
    launch_nuts_elem(S.dev_tasks + nb, npost, S.dev_blk + (nb + 1), bpost, stream, 1);
  launch_hmc_finalize(S.dev_tasks + 2 * nb, npost, stream);
  if (hmc_tasks)
    launch_hmc_elem(S.dev_tasks + 3 * nb, nrst, S.dev_blk + 2 * (nb + 1), rst_blk[nrst], stream);
  if (nuts_tasks)
    launch_nuts_elem(S.dev_tasks + 3 * nb, nrst, S.dev_blk + 2 * (nb + 1), rst_blk[nrst], stream);
  // the finalize kernel has written every chain's state into host_states; the
  // event orders the host's reads after it
  hip_or_throw(hipEventRecord(t.done, stream), "event record");
}

void hmc_server::complete(Tick& t) {
  hip_or_throw(hipEventSynchronize(t.done), "tick wait");
  const uint64_t tnow = now_ns();
  Slot& S = slots[t.slot];
  std::lock_guard<std::mutex> lk(mu);
  for (size_t i = 0; i < t.entries.size(); ++i) {
    const TickEntry& e = t.entries[i];
    Chain* c = e.c;
    c->inflight -= 1;
    req_latency_ns.push_back(tnow - e.t_enqueue);
    n_requests += 1;
    const HmcState& hs = S.host_states[i];
    const bool bad = hs.status != 0;
    const bool nuts_end = e.nuts && hs.finished_now;
    // a NUTS trajectory ends within 2^depth - 1 steps; the bound guards the schedule
    const bool overrun = e.nuts && !hs.finished_now && c->running &&
                         c->step > (1 << c->nuts_depth) + 2 * kSlots;
    if (nuts_end) {
      c->running = false;
      c->step = 0;
    }
    if ((e.ends || nuts_end || bad || overrun) && !c->failed) {
      hmc_result r{};
      r.chain = c->id;
      r.trajectory = e.traj;
      r.accepted = bad || overrun ? 0 : hs.accepted;
      r.status = overrun ? VIS_EDEVICE : bad ? VIS_ENUMERIC : VIS_OK;
      r.h0 = hs.h0;
      r.h1 = hs.h1;
      r.chi2 = hs.chi2;
      r.eps = hs.eps_used;
      r.n_grad = e.init ? 1 : e.nuts ? hs.nsteps : c->n_leapfrog;
      r.tree_depth = e.nuts ? hs.depth + 1 : 0;
      r.accept_stat = hs.accept_stat;
      if (!e.init && !c->traj_submit_ns.empty()) {
        r.t_submit_ns = c->traj_submit_ns.front();
        c->traj_submit_ns.pop_front();
      }
      r.t_done_ns = tnow;
      results.push_back(r);
      if (bad || overrun) {
        // a non-finite energy stops this chain only; its queued work is dropped
        c->failed = true;
        c->pending = 0;
        c->running = false;
        c->traj_submit_ns.clear();
      }
    }
    if (c->releasing && c->inflight == 0 && c->off >= 0) {
      arena.release(static_cast<size_t>(c->off), c->L.bytes);
      c->off = -1;
      chains[c->id] = nullptr;
      delete c;
    }
  }
  cv_done.notify_all();
}

void hmc_server::run() {
  try {
    while (true) {
      Tick t;
      {
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
          if (stop && inflight.empty()) return;
          if (!stop && static_cast<int>(inflight.size()) < depth && build_tick(t)) break;
          if (!inflight.empty()) break;
          cv_work.wait_for(lk, std::chrono::milliseconds(5));
        }
      }
      const bool built = !t.entries.empty();
      if (built) {
        t.slot = next_slot;
        next_slot = (next_slot + 1) % kSlots;
        hip_or_throw(hipEventCreateWithFlags(&t.done, hipEventDisableTiming), "event create");
        enqueue(t);
        inflight.push_back(std::move(t));
      }
      // keep at most `depth` ticks in flight; complete the oldest when full or
      // when nothing new could be scheduled
      if (!inflight.empty() && (static_cast<int>(inflight.size()) >= depth || !built)) {
        Tick& old = inflight.front();
        complete(old);
        (void)hipEventDestroy(old.done);
        inflight.pop_front();
      }
    }
  } catch (const Failure& f) {
    std::lock_guard<std::mutex> lk(mu);
    worker_status = f.code;
    worker_error = vis_last_error();
    stop = true;
    cv_done.notify_all();
  }
}

extern "C" {

size_t hmc_chain_footprint_bytes(const vis_field* field) {
  if (field == nullptr) return 0;
  return chain_layout(field, false, false).bytes;
}

size_t hmc_chain_footprint_dense_gain_bytes(const vis_field* field) {
  if (field == nullptr) return 0;
  return chain_layout(field, true, false).bytes;
}

size_t hmc_chain_footprint_nuts_bytes(const vis_field* field) {
  if (field == nullptr) return 0;
  return chain_layout(field, false, true).bytes;
}

size_t hmc_chain_footprint_nuts_dense_gain_bytes(const vis_field* field) {
  if (field == nullptr) return 0;
  return chain_layout(field, true, true).bytes;
}

vis_status hmc_server_create(const hmc_server_config* cfg, void* arena_dev, size_t arena_bytes,
                             void* stream, hmc_server** out) {
  hmc_server* s = nullptr;
  vis_status st = guarded([&] {
    BV_REQUIRE(cfg && out && arena_dev, VIS_EINVAL, "null argument");
    BV_REQUIRE(cfg->max_chains >= 1 && cfg->max_chains <= 4096, VIS_EINVAL, "max_chains out of range");
    BV_REQUIRE(cfg->max_batch >= 1 && cfg->max_batch <= 1024, VIS_EINVAL, "max_batch out of range");
    BV_REQUIRE(cfg->inflight_ticks >= 0 && cfg->inflight_ticks <= kSlots - 1, VIS_EINVAL,
               "inflight_ticks must be 0, 1 or 2");
    BV_REQUIRE(cfg->batched >= 0 && cfg->batched <= 2, VIS_EINVAL, "batched must be 0, 1 or 2");
    s = new hmc_server();
    s->cfg = *cfg;
    s->depth = cfg->inflight_ticks == 2 ? 2 : 1;
    s->stream = as_stream(stream);
    const int nb = cfg->max_batch;
    const size_t task_bytes = round_up(sizeof(HmcTask) * 4 * nb, 256);
    const size_t blk_bytes = round_up(sizeof(int) * kPrefixes * (nb + 1), 256);
    const size_t bb = cfg->batched == 1 ? batch_stage_bytes(nb) : 0;
    const size_t per = task_bytes + blk_bytes + bb;
    const size_t reserve = kSlots * per;
    BV_REQUIRE(arena_bytes > reserve, VIS_ENOMEM, "arena smaller than the %zu-byte tick tables",
               reserve);
    char* base = static_cast<char*>(arena_dev);
    for (int i = 0; i < kSlots; ++i) {
      Slot& S = s->slots[i];
      S.dev_tasks = reinterpret_cast<HmcTask*>(base + i * per);
      S.dev_blk = reinterpret_cast<int*>(base + i * per + task_bytes);
      S.table_bytes = task_bytes + blk_bytes;
      BV_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.host_tasks), S.table_bytes));
      S.host_blk = reinterpret_cast<int*>(reinterpret_cast<char*>(S.host_tasks) + task_bytes);
      BV_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.host_states), sizeof(HmcState) * nb,
                           hipHostMallocCoherent));
      std::memset(S.host_tasks, 0, S.table_bytes);
      if (bb > 0) {
        S.dev_batch = reinterpret_cast<unsigned char*>(base + i * per + task_bytes + blk_bytes);
        S.batch_bytes = bb;
        BV_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.host_batch), bb));
      }
    }
    s->arena.init(base + reserve, arena_bytes - reserve);
    if (cfg->batched != 0) {
      for (int i = 0; i < kSubStreams; ++i) {
        BV_HIP(hipStreamCreateWithFlags(&s->sub[i], hipStreamNonBlocking));
        BV_HIP(hipEventCreateWithFlags(&s->ev_sub[i], hipEventDisableTiming));
      }
      BV_HIP(hipEventCreateWithFlags(&s->ev_pre, hipEventDisableTiming));
    }
    s->chains.reserve(cfg->max_chains);
    s->worker = std::thread([s] { s->run(); });
    *out = s;
  });
  if (st != VIS_OK && s != nullptr) {
    for (auto& S : s->slots) {
      if (S.host_tasks) (void)hipHostFree(S.host_tasks);
      if (S.host_states) (void)hipHostFree(S.host_states);
      if (S.host_batch) (void)hipHostFree(S.host_batch);
    }
    delete s;
  }
  return st;
}

vis_status hmc_chain_admit(hmc_server* s, const hmc_chain_init* in, int32_t* chain_id) {
  return guarded([&] {
    BV_REQUIRE(s && in && chain_id, VIS_EINVAL, "null argument");
    BV_REQUIRE(in->field && in->data && in->q0 && in->minv && in->alm_prior_var, VIS_EINVAL,
               "null pointer in chain init");
    BV_REQUIRE(in->n_leapfrog >= 1 && in->n_leapfrog <= 100000, VIS_EINVAL, "n_leapfrog out of range");
    BV_REQUIRE(in->eps > 0.f && in->sigma_n > 0.f && in->gain_prior_sigma > 0.f, VIS_EINVAL,
               "eps, sigma_n and gain_prior_sigma must be positive");
    const bool dense = in->gain_chol != nullptr;
    BV_REQUIRE(in->nuts_max_depth >= 0 && in->nuts_max_depth <= kNutsMaxDepth, VIS_EINVAL,
               "nuts_max_depth must be in [0, %d]", kNutsMaxDepth);
    BV_REQUIRE(!dense || 2 * in->field->n_ant <= kGainBlockMax, VIS_EINVAL,
               "dense gain mass blocks hold at most %d antennas (field has %d)",
               kGainBlockMax / 2, in->field->n_ant);
    const ChainLayout L = chain_layout(in->field, dense, in->nuts_max_depth > 0);
    Chain* c = nullptr;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      BV_REQUIRE(s->worker_status == VIS_OK, s->worker_status, "server failed: %s",
                 s->worker_error.c_str());
      int live = 0;
      for (Chain* x : s->chains) {
        if (x == nullptr) continue;
        ++live;
        BV_REQUIRE(x->field != in->field, VIS_EINVAL,
                   "field already used by chain %d (each chain needs its own field)", x->id);
      }
      if (live >= s->cfg.max_chains) {
        set_error("request table full (%d chains)", s->cfg.max_chains);
        throw Failure{VIS_EAGAIN};
      }
      const long off = s->arena.alloc(L.bytes);
      if (off < 0) {
        set_error("arena has no room for a %zu-byte chain now", L.bytes);
        throw Failure{VIS_EAGAIN};
      }
      c = new Chain();
      c->off = off;
      c->base = s->arena.base + off;
      c->L = L;
      c->field = in->field;
      c->data = reinterpret_cast<const float2*>(in->data);
      c->sigma_n = in->sigma_n;
      c->gvar_inv = 2.0f / (in->gain_prior_sigma * in->gain_prior_sigma);
      c->n_leapfrog = in->n_leapfrog;
      c->nuts_depth = in->nuts_max_depth;
      c->seed = in->seed;
      c->stream = in->stream_id;
      c->releasing = true;  // not schedulable until its buffers are initialised
      c->id = static_cast<int>(s->chains.size());
      s->chains.push_back(c);
    }
    // initialise the chain's buffers on a private stream, then publish it
    hipStream_t cs = nullptr;
    BV_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const size_t vf = sizeof(float) * L.len;
    BV_HIP(hipMemsetAsync(c->base, 0, L.bytes, cs));
    BV_HIP(hipMemcpyAsync(c->ptr(L.off_q), in->q0, vf, hipMemcpyDeviceToDevice, cs));
    BV_HIP(hipMemcpyAsync(c->ptr(L.off_minv), in->minv, vf, hipMemcpyDeviceToDevice, cs));
    BV_HIP(hipMemcpyAsync(c->ptr(L.off_cvar), in->alm_prior_var, sizeof(float) * L.nalm,
                          hipMemcpyDeviceToDevice, cs));
    int bad = 0;
    if (dense) {
      int* flag = reinterpret_cast<int*>(c->base + L.off_flag);
      launch_gain_mass_setup(in->gain_chol, L.nchan, L.nb, L.nb4, c->ptr(L.off_lrow),
                             c->ptr(L.off_lcol), flag, cs);
      BV_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, cs));
    }
    HmcState hs{};
    hs.eps = hs.eps0 = hs.eps_used = in->eps;
    hs.adapt = in->adapt_step ? 1 : 0;
    BV_HIP(hipMemcpyAsync(c->st(), &hs, sizeof(HmcState), hipMemcpyHostToDevice, cs));
    BV_HIP(hipStreamSynchronize(cs));
    (void)hipStreamDestroy(cs);
    if (bad) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->arena.release(static_cast<size_t>(c->off), c->L.bytes);
      s->chains[c->id] = nullptr;
      delete c;
      BV_REQUIRE(false, VIS_EINVAL,
                 "gain_chol: non-finite entry or non-positive diagonal in the lower triangle");
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      c->releasing = false;
      *chain_id = c->id;
    }
    s->cv_work.notify_all();
  });
}

vis_status hmc_submit(hmc_server* s, int32_t id, int32_t n) {
  return guarded([&] {
    BV_REQUIRE(s != nullptr && n >= 0, VIS_EINVAL, "bad argument");
    std::lock_guard<std::mutex> lk(s->mu);
    BV_REQUIRE(id >= 0 && id < static_cast<int>(s->chains.size()) && s->chains[id] != nullptr &&
                   !s->chains[id]->releasing,
               VIS_ENOTFOUND, "unknown chain %d", id);
    Chain* c = s->chains[id];
    BV_REQUIRE(!c->failed, VIS_ENUMERIC, "chain %d stopped after a non-finite energy", id);
    const uint64_t t = now_ns();
    c->pending += n;
    for (int i = 0; i < n; ++i) c->traj_submit_ns.push_back(t);
    s->cv_work.notify_all();
  });
}

vis_status hmc_poll(hmc_server* s, hmc_result* out, int32_t max, int32_t* n_out, int32_t timeout_ms) {
  return guarded([&] {
    BV_REQUIRE(s && n_out && (out || max == 0), VIS_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->results.empty() && timeout_ms > 0 && s->worker_status == VIS_OK)
      s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                          [&] { return !s->results.empty() || s->worker_status != VIS_OK; });
    BV_REQUIRE(s->worker_status == VIS_OK, s->worker_status, "server failed: %s",
               s->worker_error.c_str());
    int n = 0;
    while (n < max && !s->results.empty()) {
      out[n++] = s->results.front();
      s->results.pop_front();
    }
    *n_out = n;
  });
}

vis_status hmc_chain_position(hmc_server* s, int32_t id, float* q_out, void* stream) {
  return guarded([&] {
    BV_REQUIRE(s && q_out, VIS_EINVAL, "null argument");
    Chain* c = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      BV_REQUIRE(id >= 0 && id < static_cast<int>(s->chains.size()) && s->chains[id] != nullptr,
                 VIS_ENOTFOUND, "unknown chain %d", id);
      c = s->chains[id];
      BV_REQUIRE(!c->running && c->pending == 0, VIS_EAGAIN, "chain %d still has work queued", id);
      // a tick built before the host saw the chain's last result (a NUTS step
      // that the device turns into a no-op) may still be in flight: wait for it
      s->cv_done.wait_for(lk, std::chrono::seconds(30), [&] {
        return s->chains[id] != c || c->inflight == 0 || s->worker_status != VIS_OK;
      });
      BV_REQUIRE(s->chains[id] == c, VIS_ENOTFOUND, "chain %d was released", id);
      BV_REQUIRE(c->inflight == 0, VIS_EAGAIN, "chain %d still has work in flight", id);
    }
    // the server stream orders this copy after the chain's last tick
    BV_HIP(hipMemcpyAsync(q_out, c->ptr(c->L.off_q), sizeof(float) * c->L.len,
                          hipMemcpyDeviceToDevice, s->stream));
    BV_HIP(hipStreamSynchronize(s->stream));
    (void)stream;
  });
}

vis_status hmc_chain_release(hmc_server* s, int32_t id) {
  return guarded([&] {
    BV_REQUIRE(s != nullptr, VIS_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    BV_REQUIRE(id >= 0 && id < static_cast<int>(s->chains.size()) && s->chains[id] != nullptr,
               VIS_ENOTFOUND, "unknown chain %d", id);
    Chain* c = s->chains[id];
    c->releasing = true;
    c->pending = 0;
    c->running = false;
    if (c->inflight == 0) {
      s->arena.release(static_cast<size_t>(c->off), c->L.bytes);
      c->off = -1;
      s->chains[id] = nullptr;
      delete c;
    }
  });
}

vis_status hmc_server_stats(hmc_server* s, hmc_stats* out, int32_t reset) {
  return guarded([&] {
    BV_REQUIRE(s && out, VIS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<uint64_t> v = s->req_latency_ns;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      if (v.empty()) return 0.0;
      const size_t i = std::min(v.size() - 1, static_cast<size_t>(q * (v.size() - 1) + 0.5));
      return static_cast<double>(v[i]) * 1e-6;
    };
    out->requests = static_cast<int64_t>(s->n_requests);
    out->p10_ms = pct(0.10);
    out->p50_ms = pct(0.50);
    out->p90_ms = pct(0.90);
    out->p99_ms = pct(0.99);
    out->max_ms = v.empty() ? 0.0 : static_cast<double>(v.back()) * 1e-6;
    size_t used = 0;
    for (auto& fr : s->arena.free_list) used += fr.second;
    out->arena_free_bytes = static_cast<int64_t>(used);
    int live = 0;
    for (Chain* c : s->chains) live += c != nullptr;
    out->live_chains = live;
    if (reset) {
      s->req_latency_ns.clear();
      s->n_requests = 0;
    }
  });
}

vis_status hmc_server_destroy(hmc_server* s) {
  if (s == nullptr) return VIS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (Chain* c : s->chains) delete c;
  for (int i = 0; i < kSubStreams; ++i) {
    if (s->sub[i]) (void)hipStreamDestroy(s->sub[i]);
    if (s->ev_sub[i]) (void)hipEventDestroy(s->ev_sub[i]);
  }
  if (s->ev_pre) (void)hipEventDestroy(s->ev_pre);
  for (auto& S : s->slots) {
    if (S.host_tasks) (void)hipHostFree(S.host_tasks);
    if (S.host_states) (void)hipHostFree(S.host_states);
    if (S.host_batch) (void)hipHostFree(S.host_batch);
  }
  delete s;
  return VIS_OK;
}

}  // extern "C"
