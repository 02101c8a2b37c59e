// Batched launches: one grid that covers the same kernel's work for many
// evaluations (many fields) at once.
//
// Every kernel of the evaluation path is written as a body that takes its
// arguments as one struct and its workgroup position as a Blk (block index
// and grid size of its own launch).  A plain launch runs the body with
// blockIdx / gridDim.  A batched launch concatenates the grids of several
// evaluations: evaluation r owns workgroups [start_r, start_r + nx ny nz),
// start_r a multiple of 8, so that each workgroup runs on the XCD it would
// occupy in its own launch (the dispatcher deals workgroups round-robin over
// the 8 XCDs) and the bodies' XCD-aware tile maps keep their meaning.  Each
// workgroup finds its evaluation by binary search over the starts, rebuilds
// its 3-D position in x-fastest order and runs the same body on that
// evaluation's arguments, so every evaluation computes exactly what its own
// launch would, whatever else shares the grid.
//
// The launchers record instead of launching while a Recorder is installed on
// the calling thread; run_batched sorts the recorded evaluations into classes
// with the same launch sequence (same kernel instantiations in the same
// order) and issues, per class, one batched launch per position of that
// sequence, in order, each class on a stream of its own.
#pragma once

#include <cstring>
#include <vector>

#include "common.hpp"

namespace bv {

struct Blk {
  int x, y, z;
  int nx, ny, nz;
};

__device__ __forceinline__ Blk blk_here() {
  return Blk{static_cast<int>(blockIdx.x), static_cast<int>(blockIdx.y), static_cast<int>(blockIdx.z),
             static_cast<int>(gridDim.x), static_cast<int>(gridDim.y), static_cast<int>(gridDim.z)};
}

struct BatchEntry {
  int start;        // first workgroup (multiple of 8); entry n is a sentinel with start = total
  int nx, ny, nz;   // the evaluation's own grid
};

__device__ __forceinline__ int batch_find(const BatchEntry* __restrict__ e, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (e[mid].start <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Kernel descriptor K: `using Args = ...;`, `static constexpr int kThreads`,
// `static constexpr int kWaves` (minimum waves per EU to aim for; 0 = no hint)
// and `static __device__ void run(const Args&, const Blk&)`.
template <class K>
__global__ void __launch_bounds__(K::kThreads) __attribute__((amdgpu_waves_per_eu(K::kWaves)))
k_one(typename K::Args a) {
  K::run(a, blk_here());
}

template <class K>
__global__ void __launch_bounds__(K::kThreads) __attribute__((amdgpu_waves_per_eu(K::kWaves)))
k_many(const typename K::Args* __restrict__ args, const BatchEntry* __restrict__ ent, int n) {
  const int b = static_cast<int>(blockIdx.x);
  // uniform over the workgroup: the evaluation's arguments load into scalar
  // registers (kernel-argument style) rather than per-lane registers
  const int r = __builtin_amdgcn_readfirstlane(batch_find(ent, n, b));
  const BatchEntry e = ent[r];
  const int l = b - e.start;
  const int per_z = e.nx * e.ny;
  if (l >= per_z * e.nz) return;   // workgroups padding the evaluation to a multiple of 8
  const int z = l / per_z, rem = l - z * per_z;
  const int y = rem / e.nx, x = rem - y * e.nx;
  // read through the constant address space: the table is never written while
  // the kernel runs, so the compiler may re-load fields at their uses instead
  // of holding all of them in registers (as it does for kernel arguments)
#if defined(__HIP_DEVICE_COMPILE__)
  typedef const typename K::Args __attribute__((address_space(4))) ConstArgs;
  const ConstArgs* ca = (const ConstArgs*)(reinterpret_cast<uintptr_t>(args));
  const typename K::Args a = ca[r];
#else   // the host pass only checks the body; the address space is a device notion
  const typename K::Args a = args[r];
#endif
  K::run(a, Blk{x, y, z, e.nx, e.ny, e.nz});
}

// Stages of one evaluation, in execution order.
enum Stage : int {
  kStageSynthFwd = 0, kStageFringeFwd = 1, kStageGains = 2, kStageFringeAdj = 3,
  kStageReduce = 4, kStageSynthAdj = 5, kNumStages = 6
};

// One recorded launch (type-erased).
struct LaunchRec {
  int stage = 0, pos = 0;
  const void* kid = nullptr;   // identifies the kernel (and its instantiation)
  void (*many)(const void* args_dev, const BatchEntry* ent_dev, int n, int total, size_t lds,
               hipStream_t st) = nullptr;
  size_t args_size = 0;
  unsigned char args[512];
  dim3 grid;
  size_t lds = 0;
};

struct Recorder {
  std::vector<std::vector<LaunchRec>> evals;   // launches of each evaluation, in order
  int cur = -1;
  int stage = 0;
  int pos = 0;
  void begin_eval() {
    evals.emplace_back();
    cur = static_cast<int>(evals.size()) - 1;
    stage = 0;
    pos = 0;
  }
  void set_stage(int s) {
    if (s != stage) {
      stage = s;
      pos = 0;
    }
  }
};

// The recorder of the calling thread, or nullptr (launch immediately).
Recorder*& thread_recorder();

// Marks the stage of the launches that follow (no effect without a recorder).
struct StageScope {
  explicit StageScope(int s) {
    if (Recorder* r = thread_recorder()) r->set_stage(s);
  }
};

template <class K>
void many_launcher(const void* args_dev, const BatchEntry* ent_dev, int n, int total, size_t lds,
                   hipStream_t st) {
  k_many<K><<<total, K::kThreads, lds, st>>>(static_cast<const typename K::Args*>(args_dev), ent_dev, n);
}

template <class K>
struct KernelId {
  static const char tag;
};
template <class K>
const char KernelId<K>::tag = 0;

// Launch K over `grid` now, or record it for a batched launch.
template <class K>
void launch_k(dim3 grid, size_t lds, const typename K::Args& a, hipStream_t st, const char* name) {
  if (static_cast<long>(grid.x) * grid.y * grid.z == 0) return;
  if (Recorder* r = thread_recorder()) {
    static_assert(sizeof(typename K::Args) <= sizeof(LaunchRec::args), "argument block too large");
    LaunchRec rec;
    rec.stage = r->stage;
    rec.pos = r->pos++;
    rec.kid = &KernelId<K>::tag;
    rec.many = &many_launcher<K>;
    rec.args_size = sizeof(typename K::Args);
    std::memcpy(rec.args, &a, sizeof(typename K::Args));
    rec.grid = grid;
    rec.lds = lds;
    r->evals[r->cur].push_back(rec);
    return;
  }
  k_one<K><<<grid, K::kThreads, lds, st>>>(a);
  check_launch(name);
}

// Batched execution of a recorder's evaluations on `st`.  The argument tables
// and entries of all launches are packed into `host_stage` (pinned) and
// uploaded with one copy to `dev_stage`; throws Failure{VIS_ENOMEM} when they
// do not fit `stage_bytes`.  Different classes of evaluations share no data:
// with `nsub` > 0 side streams they run concurrently on `sub` (heaviest class
// first, each to the least loaded side stream), started after the upload and
// joined into `st` by events (`ev` holds nsub + 1 events).
void run_batched(Recorder& rec, unsigned char* host_stage, unsigned char* dev_stage,
                 size_t stage_bytes, hipStream_t st, int nsub = 0, const hipStream_t* sub = nullptr,
                 const hipEvent_t* ev = nullptr);

}  // namespace bv
