// Internal helpers of the bayesvis library: status/error plumbing, workspace
// carving, small device utilities.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/bayesvis.h"

namespace bv {

// ---------------------------------------------------------------- errors --
void set_error(const char* fmt, ...);
void clear_error();

struct Failure {
  vis_status code;
};

#define BV_REQUIRE(cond, code, ...)          \
  do {                                       \
    if (!(cond)) {                           \
      ::bv::set_error(__VA_ARGS__);          \
      throw ::bv::Failure{code};             \
    }                                        \
  } while (0)

#define BV_HIP(expr)                                                            \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::bv::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                      __FILE__, __LINE__);                                      \
      throw ::bv::Failure{VIS_EDEVICE};                                         \
    }                                                                           \
  } while (0)

// Runs f(); converts Failure / std exceptions into a status code.
template <class F>
vis_status guarded(F&& f) {
  try {
    clear_error();
    f();
    return VIS_OK;
  } catch (const Failure& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return VIS_ENOMEM;
  } catch (...) {
    set_error("unexpected internal error");
    return VIS_EDEVICE;
  }
}

// Launch check: catches invalid launch configurations immediately.
inline void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch %s failed: %s", what, hipGetErrorString(e));
    throw Failure{VIS_EDEVICE};
  }
}

// ------------------------------------------------------------- workspace --
// Bump allocator over a caller-provided device buffer.  With base == nullptr
// it only measures (used by the *_workspace_bytes queries).
struct Carver {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  template <class T>
  T* take(size_t count, size_t align = 256) {
    size_t off = (used + align - 1) / align * align;
    size_t bytes = count * sizeof(T);
    used = off + bytes;
    if (base == nullptr) return nullptr;
    BV_REQUIRE(used <= cap, VIS_ENOMEM, "workspace too small: need at least %zu bytes, have %zu",
               used, cap);
    return reinterpret_cast<T*>(base + off);
  }
};

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int ceil_div(long a, long b) { return static_cast<int>((a + b - 1) / b); }
inline long round_up(long a, long b) { return (a + b - 1) / b * b; }

// -------------------------------------------------------------- constants --
constexpr double kCLight = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
// sigma of a Gaussian = FWHM / (2 sqrt(2 ln 2))
constexpr double kFwhmToSigma = 0.42466090014400953;
constexpr double kLn2 = 0.69314718055994531;

constexpr int kChunk = 64;        // pixels per fringe chunk (one wavefront)
constexpr int kAdjChunkTile = 32; // chunks per tile of the adjoint fringe grid (with 16 channel groups)
constexpr int kScaleParts = 16;   // row segments of the split forward's sky maxima
constexpr int kMaxExtent = 16;    // max |lattice difference| supported
constexpr int kSepPad = 4;        // zero azimuthal columns on each side of the separable T table
constexpr int kSepStep = 32;      // columns per batch of the separable azimuthal stages
// row length of the separable Legendre table's block for order m (l = m .. lmax, zero-padded)
__host__ __device__ inline int sep_lpad(int lmax, int m) { return (lmax - m + 1 + 7) / 8 * 8; }
constexpr float kBelowHorizon = 1e30f;  // theta^2 marker: beam exactly 0

}  // namespace bv
