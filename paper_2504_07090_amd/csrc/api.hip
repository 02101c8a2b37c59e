// Evaluation entry points of the C ABI: vis_forward, vis_adjoint, chi2_and_grad.
// Each is a fixed stream-ordered sequence of kernel launches; nothing returns
// to the host.
#include <mutex>

#include "batch.hpp"
#include "objects.hpp"

using namespace bv;

namespace {

void check_field(const vis_field* f) {
  BV_REQUIRE(f != nullptr, VIS_EINVAL, "null field");
}

}  // namespace

namespace bv {

void forward_core(const vis_field* f, const float* alm, const float* fwhm, hipStream_t s) {
  { StageScope sc(kStageSynthFwd); launch_synth_fwd(f, alm, f->scr.img, s); }
  { StageScope sc(kStageFringeFwd); launch_fringe_fwd(f, f->scr.img, fwhm, f->scr.vu, s); }
}

void adjoint_tail(const vis_field* f, const float* fwhm, float* grad_alm, float2* grad_gains,
                  float* grad_fwhm, bool with_chi2, double* chi2, hipStream_t s) {
  // separable fields: the adjoint fringe pass writes dL/dI straight into the
  // full-grid layout that the azimuthal adjoint stage reads
  const bool full = f->synthesis == VIS_SYNTH_SEPARABLE;
  {
    StageScope sc(kStageFringeAdj);
    launch_fringe_adj(f, f->scr.img, fwhm, f->scr.gco, full ? nullptr : f->scr.dimg, f->scr.f_part, s,
                      full ? f->scr.sep_dfull : nullptr);
  }
  {
    // one launch for the gain gradient, chi^2 and dL/dF (the gains pass's
    // partials are complete before the fringe pass, dL/dF's after it)
    StageScope sc(kStageReduce);
    launch_reduce_grads(f, with_chi2, f->scr.chi_part, chi2, f->scr.g_part, grad_gains, f->scr.f_part,
                        grad_fwhm, s);
  }
  if (grad_alm != nullptr) {
    StageScope sc(kStageSynthAdj);
    launch_synth_adj(f, full ? nullptr : f->scr.dimg, grad_alm, s);
  }
}

}  // namespace bv

namespace {

// Scratch of chi2_filtered_and_grad_noalloc: one array per GPU, in the code
// object's device memory, held until the process ends.  Host code never
// passes `scratch` itself to a kernel (on the host it names a stand-in, not
// the device copy); it uses the device address looked up once per device.
static __device__ __align__(256) unsigned char scratch[VIS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device, with that device current).
void* noalloc_scratch() {
  int dev = 0;
  BV_HIP(hipGetDevice(&dev));
  BV_REQUIRE(dev >= 0 && dev < kMaxDevices, VIS_EDEVICE, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    void* p = nullptr;
    BV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    BV_REQUIRE(p != nullptr, VIS_EDEVICE, "no device address for the static scratch array");
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}

}  // namespace

extern "C" {

vis_status vis_forward(const vis_field* f, const float* alm, const vis_c64* gains,
                       const float* fwhm, vis_c64* vis, void* stream) {
  return guarded([&] {
    check_field(f);
    BV_REQUIRE(alm && gains && fwhm && vis, VIS_EINVAL, "null device pointer");
    hipStream_t s = as_stream(stream);
    forward_core(f, alm, fwhm, s);
    launch_gains(f, kGainFwd, f->scr.vu, reinterpret_cast<const float2*>(gains), nullptr, 0.f,
                 reinterpret_cast<float2*>(vis), nullptr, nullptr, nullptr, s);
  });
}

vis_status vis_adjoint(const vis_field* f, const float* alm, const vis_c64* gains,
                       const float* fwhm, const vis_c64* dvis, float* grad_alm,
                       vis_c64* grad_gains, float* grad_fwhm, void* stream) {
  return guarded([&] {
    check_field(f);
    BV_REQUIRE(alm && gains && fwhm && dvis, VIS_EINVAL, "null device pointer");
    BV_REQUIRE(grad_alm && grad_gains && grad_fwhm, VIS_EINVAL, "null gradient output");
    hipStream_t s = as_stream(stream);
    forward_core(f, alm, fwhm, s);
    launch_gains(f, kGainAdj, f->scr.vu, reinterpret_cast<const float2*>(gains),
                 reinterpret_cast<const float2*>(dvis), 0.f, nullptr, nullptr, f->scr.gco,
                 f->scr.g_part, s);
    adjoint_tail(f, fwhm, grad_alm, reinterpret_cast<float2*>(grad_gains), grad_fwhm, false,
                 nullptr, s);
  });
}

vis_status chi2_and_grad(const vis_field* f, const vis_c64* data, float sigma_n, const float* alm,
                         const vis_c64* gains, const float* fwhm, double* chi2, float* grad_alm,
                         vis_c64* grad_gains, float* grad_fwhm, void* stream) {
  return guarded([&] {
    check_field(f);
    BV_REQUIRE(data && alm && gains && fwhm && chi2, VIS_EINVAL, "null device pointer");
    BV_REQUIRE(sigma_n > 0.f && sigma_n < 3.0e38f, VIS_EINVAL, "sigma_n must be positive and finite");
    hipStream_t s = as_stream(stream);
    forward_core(f, alm, fwhm, s);
    launch_gains(f, kGainChi2, f->scr.vu, reinterpret_cast<const float2*>(gains),
                 reinterpret_cast<const float2*>(data), sigma_n, nullptr, f->scr.chi_part,
                 f->scr.gco, f->scr.g_part, s);
    const bool any_grad = grad_alm || grad_gains || grad_fwhm;
    if (!any_grad) {
      StageScope sc(kStageReduce);
      launch_reduce_grads(f, true, f->scr.chi_part, chi2, nullptr, nullptr, nullptr, nullptr, s);
      return;
    }
    adjoint_tail(f, fwhm, grad_alm, reinterpret_cast<float2*>(grad_gains), grad_fwhm, true, chi2, s);
  });
}

vis_status vis_make_map(const vis_field* f, const vis_c64* data, const vis_c64* gains,
                        const float* fwhm, float* map, float* weight, void* stream) {
  return guarded([&] {
    check_field(f);
    BV_REQUIRE(data && gains && fwhm && map, VIS_EINVAL, "null device pointer");
    hipStream_t s = as_stream(stream);
    launch_gains(f, kGainMap, f->scr.vu, reinterpret_cast<const float2*>(gains),
                 reinterpret_cast<const float2*>(data), 0.f, nullptr, nullptr, f->scr.gco, nullptr, s);
    launch_fringe_adj(f, f->scr.img, fwhm, f->scr.gco, f->scr.dimg, f->scr.f_part, s);
    launch_map_finish(f, gains, fwhm, map, weight, s);
  });
}

vis_status chi2_filtered_and_grad(const vis_field* f, const vis_filter* flt, const vis_c64* data,
                                  float sigma_n, const float* alm, const vis_c64* gains,
                                  const float* fwhm, double* chi2, float* grad_alm,
                                  vis_c64* grad_gains, float* grad_fwhm, void* work,
                                  size_t work_bytes, void* stream) {
  return guarded([&] {
    check_field(f);
    BV_REQUIRE(data && alm && gains && fwhm && chi2 && work, VIS_EINVAL, "null device pointer");
    BV_REQUIRE(sigma_n > 0.f && sigma_n < 3.0e38f, VIS_EINVAL, "sigma_n must be positive and finite");
    const FilteredWork w = carve_filtered_work(f, work, work_bytes);
    hipStream_t s = as_stream(stream);
    forward_core(f, alm, fwhm, s);
    launch_gains(f, kGainFwd, f->scr.vu, reinterpret_cast<const float2*>(gains), nullptr, 0.f, w.m,
                 nullptr, nullptr, nullptr, s);
    launch_filter_chi2(f, flt, reinterpret_cast<const float2*>(data), sigma_n, w, chi2, s);
    if (!(grad_alm || grad_gains || grad_fwhm)) return;
    launch_filter_cot(f, flt, w, s);
    launch_gains(f, kGainAdj, f->scr.vu, reinterpret_cast<const float2*>(gains), w.m, 0.f, nullptr,
                 nullptr, f->scr.gco, f->scr.g_part, s);
    adjoint_tail(f, fwhm, grad_alm, reinterpret_cast<float2*>(grad_gains), grad_fwhm, false, nullptr, s);
  });
}

vis_status chi2_filtered_and_grad_noalloc(const vis_field* f, const vis_filter* flt,
                                          const vis_c64* data, float sigma_n, const float* alm,
                                          const vis_c64* gains, const float* fwhm, double* chi2,
                                          float* grad_alm, vis_c64* grad_gains, float* grad_fwhm,
                                          void* stream) {
  return guarded([&] {
    check_field(f);
    const size_t need = carve_filtered_work(f, nullptr, 0).bytes;
    BV_REQUIRE(need <= VIS_NOALLOC_SCRATCH_BYTES, VIS_ENOMEM,
               "the field needs %zu bytes of scratch; the static array holds %zu", need,
               static_cast<size_t>(VIS_NOALLOC_SCRATCH_BYTES));
    void* work = noalloc_scratch();
    // the same sequence as chi2_filtered_and_grad over the static array (its
    // kernels write every scratch element they read, so nothing is cleared)
    const vis_status st = chi2_filtered_and_grad(f, flt, data, sigma_n, alm, gains, fwhm, chi2,
                                                 grad_alm, grad_gains, grad_fwhm, work,
                                                 VIS_NOALLOC_SCRATCH_BYTES, stream);
    if (st != VIS_OK) throw Failure{st};
  });
}

}  // extern "C"
