// Batched execution of recorded evaluation sequences (see batch.hpp).
#include <algorithm>

#include "batch.hpp"

namespace bv {

Recorder*& thread_recorder() {
  static thread_local Recorder* r = nullptr;
  return r;
}

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

void run_batched(Recorder& rec, unsigned char* host_stage, unsigned char* dev_stage,
                 size_t stage_bytes, hipStream_t st, int nsub, const hipStream_t* sub,
                 const hipEvent_t* ev) {
  // Classes: evaluations whose launch sequences are the same kernel
  // instantiations in the same order (same lattice extent, precision and
  // synthesis).  A class runs as one grid per launch position, in order, on a
  // stream of its own; different classes share no data and overlap.
  std::vector<std::vector<int>> classes;   // evaluation indices
  std::vector<const std::vector<LaunchRec>*> reps;
  auto same_seq = [](const std::vector<LaunchRec>& a, const std::vector<LaunchRec>& b) {
    if (a.size() != b.size()) return false;
    for (size_t k = 0; k < a.size(); ++k)
      if (a[k].kid != b[k].kid || a[k].stage != b[k].stage || a[k].pos != b[k].pos) return false;
    return true;
  };
  for (int e = 0; e < static_cast<int>(rec.evals.size()); ++e) {
    const auto& seq = rec.evals[e];
    if (seq.empty()) continue;
    size_t c = 0;
    while (c < classes.size() && !same_seq(*reps[c], seq)) ++c;
    if (c == classes.size()) {
      classes.emplace_back();
      reps.push_back(&seq);
    }
    classes[c].push_back(e);
  }
  if (classes.empty()) return;
  // pack every (class, launch position) table: the evaluations' arguments and
  // their workgroup ranges
  struct Packed {
    const LaunchRec* rec0;
    size_t args_off, ent_off;
    int n, total;
    size_t lds;
  };
  std::vector<std::vector<Packed>> packed(classes.size());
  size_t used = 0;
  for (size_t c = 0; c < classes.size(); ++c) {
    const auto& members = classes[c];
    const size_t nlaunch = reps[c]->size();
    for (size_t k = 0; k < nlaunch; ++k) {
      const int n = static_cast<int>(members.size());
      const size_t asz = (*reps[c])[k].args_size;
      Packed p{&(*reps[c])[k], 0, 0, n, 0, 0};
      p.args_off = align_up(used, 256);
      p.ent_off = align_up(p.args_off + asz * n, 64);
      used = p.ent_off + sizeof(BatchEntry) * n;
      BV_REQUIRE(used <= stage_bytes, VIS_ENOMEM, "batched launch tables exceed %zu bytes", stage_bytes);
      BatchEntry* ent = reinterpret_cast<BatchEntry*>(host_stage + p.ent_off);
      long start = 0;
      for (int i = 0; i < n; ++i) {
        const LaunchRec& L = rec.evals[members[i]][k];
        std::memcpy(host_stage + p.args_off + asz * i, L.args, asz);
        const long blocks = static_cast<long>(L.grid.x) * L.grid.y * L.grid.z;
        ent[i] = BatchEntry{static_cast<int>(start), static_cast<int>(L.grid.x),
                            static_cast<int>(L.grid.y), static_cast<int>(L.grid.z)};
        start += round_up(blocks, 8);
        p.lds = std::max(p.lds, L.lds);
      }
      BV_REQUIRE(start < (1L << 31), VIS_EINVAL, "batched launch of %ld workgroups", start);
      p.total = static_cast<int>(start);
      packed[c].push_back(p);
    }
  }
  BV_HIP(hipMemcpyAsync(dev_stage, host_stage, used, hipMemcpyHostToDevice, st));
  auto launch = [&](const Packed& p, hipStream_t s) {
    p.rec0->many(dev_stage + p.args_off, reinterpret_cast<const BatchEntry*>(dev_stage + p.ent_off),
                 p.n, p.total, p.lds, s);
    check_launch("batched evaluation kernel");
  };
  const int nclass = static_cast<int>(classes.size());
  if (nsub == 0 || nclass == 1) {
    for (int c = 0; c < nclass; ++c)
      for (const Packed& p : packed[c]) launch(p, st);
    return;
  }
  // Classes go to the side streams only: streams created one after another
  // get distinct hardware queues (as many as the side streams, up to the
  // queue count), while the caller's stream may share one with them, and two
  // classes on one queue run one after the other.  Heaviest class first, each
  // to the side stream with the least work so far.
  std::vector<double> work(nclass, 0.0);
  for (int c = 0; c < nclass; ++c)
    for (int e : classes[c])
      for (const LaunchRec& L : rec.evals[e]) work[c] += static_cast<double>(L.grid.x) * L.grid.y * L.grid.z;
  std::vector<int> order(nclass);
  for (int c = 0; c < nclass; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  const int used_sub = std::min(nsub, nclass);
  std::vector<double> load(used_sub, 0.0);
  BV_HIP(hipEventRecord(ev[nsub], st));   // the tables are on the device
  for (int q = 0; q < used_sub; ++q) BV_HIP(hipStreamWaitEvent(sub[q], ev[nsub], 0));
  for (int c : order) {
    const int q = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
    load[q] += work[c];
    for (const Packed& p : packed[c]) launch(p, sub[q]);
  }
  for (int q = 0; q < used_sub; ++q) {
    BV_HIP(hipEventRecord(ev[q], sub[q]));
    BV_HIP(hipStreamWaitEvent(st, ev[q], 0));
  }
}

}  // namespace bv
