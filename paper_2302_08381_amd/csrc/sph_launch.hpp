// Internal interface between the C ABI (sph_api.cpp) and the kernel
// translation units.  Not installed; the public interface is include/sph.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sph {

// Largest supported l_max (the m-extent of the widest kernel bucket).
constexpr int kMaxLmax = 32;

// Kernel parameters of the forward / batched kernel (one struct argument so
// the same layout serves direct launches and graph kernel nodes).
struct FwdParams {
  const void* xyz;        // [n,3]
  int64_t n;              // points
  int32_t L;              // l_max (runtime-degree kernels)
  void* Y;                // [n,K]
  void* dY;               // [n,3,K] or null
  const void* gY;         // [n,K] or null (fused backward)
  void* gxyz;             // [n,3] (required iff gY)
  const int64_t* offsets; // CSR offsets or null (no validation)
  int64_t n_env;
  int32_t* status;        // device status word or null
};

struct BwdParams {
  const void* dY;
  const void* gY;
  int64_t n;
  int32_t K;
  void* gxyz;
};

struct DbwdParams {
  const void* xyz;
  const void* gY;
  const void* v;
  int64_t n;
  int32_t L;
  void* ggY;   // nullable
  void* gxyz2; // nullable
};

// Number of LDS budget variants per forward kernel (autotuner choice).
constexpr int kNumBudgetVariants = 2;

// A kernel's host stub, the LDS bytes of one 64-point staging tile for the
// l_max it was looked up with (forward: the launch passes one tile, or two
// with the fused backward, as dynamic LDS; double backward: one tile;
// backward: static LDS, 0), and the per-point LDS budget in elements.
struct KernelInfo {
  const void* fn;
  size_t tile_lds_bytes;
  int budget;
};

// Per element type (suffix f32 / f64).  The kernel serves every l_max up to
// its m-extent bucket.  fn == nullptr when the arguments are out of range.
KernelInfo fwd_info_f32(int L, int normalize, int variant);
KernelInfo fwd_info_f64(int L, int normalize, int variant);
KernelInfo bwd_info_f32(int L);
KernelInfo bwd_info_f64(int L);
KernelInfo dbwd_info_f32(int L, int normalize);
KernelInfo dbwd_info_f64(int L, int normalize);

constexpr int kBwdPointsPerBlock = 16;
constexpr int kPointsPerBlock = 64;
constexpr int kBlock = 64;

}  // namespace sph
