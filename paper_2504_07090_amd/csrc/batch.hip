// Batched execution of recorded evaluation sequences (see batch.hpp).
#include <algorithm>
#include <map>
#include <tuple>

#include "batch.hpp"

namespace bv {

Recorder*& thread_recorder() {
  static thread_local Recorder* r = nullptr;
  return r;
}

namespace {

struct Group {
  int stage, pos;
  const void* kid;
  std::vector<const LaunchRec*> recs;   // one per evaluation that has this launch
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

void run_batched(Recorder& rec, unsigned char* host_stage, unsigned char* dev_stage,
                 size_t stage_bytes, hipStream_t st, int nsub, const hipStream_t* sub,
                 const hipEvent_t* ev) {
  // groups keyed by (stage, position in stage, kernel), in first-seen order of
  // the kernels within one (stage, position)
  std::map<std::tuple<int, int, int>, Group> groups;
  std::map<std::pair<int, int>, std::vector<const void*>> kid_order;
  for (const auto& ev : rec.evals) {
    for (const LaunchRec& L : ev) {
      auto& order = kid_order[{L.stage, L.pos}];
      int k = 0;
      while (k < static_cast<int>(order.size()) && order[k] != L.kid) ++k;
      if (k == static_cast<int>(order.size())) order.push_back(L.kid);
      Group& g = groups[{L.stage, L.pos, k}];
      g.stage = L.stage;
      g.pos = L.pos;
      g.kid = L.kid;
      g.recs.push_back(&L);
    }
  }
  // pack every group's argument table and entries into the staging buffer
  struct Packed {
    const Group* g;
    size_t args_off, ent_off;
    int n, total;
    size_t lds;
  };
  std::vector<Packed> packed;
  size_t used = 0;
  for (const auto& kv : groups) {
    const Group& g = kv.second;
    const int n = static_cast<int>(g.recs.size());
    const size_t asz = g.recs[0]->args_size;
    Packed p{&g, 0, 0, n, 0, 0};
    p.args_off = align_up(used, 256);
    p.ent_off = align_up(p.args_off + asz * n, 64);
    used = p.ent_off + sizeof(BatchEntry) * n;
    BV_REQUIRE(used <= stage_bytes, VIS_ENOMEM, "batched launch tables exceed %zu bytes", stage_bytes);
    BatchEntry* ent = reinterpret_cast<BatchEntry*>(host_stage + p.ent_off);
    long start = 0;
    for (int i = 0; i < n; ++i) {
      const LaunchRec* L = g.recs[i];
      std::memcpy(host_stage + p.args_off + asz * i, L->args, asz);
      const long blocks = static_cast<long>(L->grid.x) * L->grid.y * L->grid.z;
      ent[i] = BatchEntry{static_cast<int>(start), static_cast<int>(L->grid.x),
                          static_cast<int>(L->grid.y), static_cast<int>(L->grid.z)};
      start += round_up(blocks, 8);
      p.lds = std::max(p.lds, L->lds);
    }
    BV_REQUIRE(start < (1L << 31), VIS_EINVAL, "batched launch of %ld workgroups", start);
    p.total = static_cast<int>(start);
    packed.push_back(p);
  }
  if (packed.empty()) return;
  BV_HIP(hipMemcpyAsync(dev_stage, host_stage, used, hipMemcpyHostToDevice, st));
  auto launch = [&](const Packed& p, hipStream_t s) {
    const LaunchRec* L0 = p.g->recs[0];
    L0->many(dev_stage + p.args_off, reinterpret_cast<const BatchEntry*>(dev_stage + p.ent_off), p.n,
             p.total, p.lds, s);
    check_launch("batched evaluation kernel");
  };
  // levels: runs of groups with equal (stage, position); the map keeps them adjacent
  for (size_t i = 0; i < packed.size();) {
    size_t j = i + 1;
    while (j < packed.size() && packed[j].g->stage == packed[i].g->stage &&
           packed[j].g->pos == packed[i].g->pos)
      ++j;
    const int width = static_cast<int>(j - i);
    if (nsub == 0 || width == 1) {
      for (size_t k = i; k < j; ++k) launch(packed[k], st);
    } else {
      const int used_sub = std::min(nsub, width - 1);
      BV_HIP(hipEventRecord(ev[nsub], st));
      for (int q = 0; q < used_sub; ++q) BV_HIP(hipStreamWaitEvent(sub[q], ev[nsub], 0));
      // the first group stays on the main stream, the others go round-robin
      for (size_t k = i; k < j; ++k) {
        const int q = static_cast<int>(k - i);
        launch(packed[k], q == 0 ? st : sub[(q - 1) % used_sub]);
      }
      for (int q = 0; q < used_sub; ++q) {
        BV_HIP(hipEventRecord(ev[q], sub[q]));
        BV_HIP(hipStreamWaitEvent(st, ev[q], 0));
      }
    }
    i = j;
  }
}

}  // namespace bv
