// C ABI of libsph (declared in include/sph.h): argument validation, kernel
// dispatch, launch shapes, and the batched path's hipGraph cache and
// launch-variant autotuner.
#include "sph.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "sph_launch.hpp"

namespace {

thread_local std::string g_last_error;

int32_t fail(int32_t code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int32_t ok() {
  g_last_error.clear();
  return SPH_OK;
}

int32_t device_fail(hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(SPH_ERR_DEVICE, m);
}

size_t elem_size(int32_t dtype) { return dtype == SPH_F64 ? 8 : 4; }

int32_t check_common(int64_t n, int32_t l_max, int32_t dtype) {
  if (n < 0) return fail(SPH_ERR_INVALID, "n must be >= 0");
  if (l_max < 0 || l_max > sph::kMaxLmax)
    return fail(SPH_ERR_LMAX, "l_max must be in [0, " + std::to_string(sph::kMaxLmax) + "]");
  if (dtype != SPH_F32 && dtype != SPH_F64) return fail(SPH_ERR_INVALID, "dtype must be SPH_F32 or SPH_F64");
  return SPH_OK;
}

int32_t check_norm(int32_t normalize) {
  if (normalize != 0 && normalize != 1) return fail(SPH_ERR_INVALID, "normalize must be 0 or 1");
  return SPH_OK;
}

// Byte range [p, p+bytes) of a buffer, for overlap checks.
struct Range {
  const void* p;
  size_t bytes;
  const char* name;
};

int32_t check_no_overlap(std::initializer_list<Range> outs, std::initializer_list<Range> all) {
  for (const Range& o : outs) {
    if (o.p == nullptr || o.bytes == 0) continue;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(o.p), a1 = a0 + o.bytes;
    for (const Range& b : all) {
      if (b.p == nullptr || b.bytes == 0 || b.p == o.p) continue;
      const uintptr_t b0 = reinterpret_cast<uintptr_t>(b.p), b1 = b0 + b.bytes;
      if (a0 < b1 && b0 < a1)
        return fail(SPH_ERR_INVALID, std::string(o.name) + " overlaps " + b.name);
    }
  }
  return SPH_OK;
}

// The forward kernel for a set of outputs: values only (one lane per point)
// unless dY is stored or the backward is fused (four lanes per point).
// variant: see sph::FwdVariant (fn == nullptr where it does not exist).
sph::KernelInfo fwd_info(int32_t dtype, int L, int norm, bool store_dy, bool fused,
                         int variant = sph::kVarDefault) {
  using KF = sph::KernelInfo (*)(int, int);
  static constexpr KF kValues[2][2] = {{sph::fwd_values_f32_n0, sph::fwd_values_f32_n1},
                                       {sph::fwd_values_f64_n0, sph::fwd_values_f64_n1}};
  static constexpr KF kDerivs[2][2][sph::kNumDerivModes] = {
      {{sph::fwd_derivs_f32_n0_m0, sph::fwd_derivs_f32_n0_m1, sph::fwd_derivs_f32_n0_m2},
       {sph::fwd_derivs_f32_n1_m0, sph::fwd_derivs_f32_n1_m1, sph::fwd_derivs_f32_n1_m2}},
      {{sph::fwd_derivs_f64_n0_m0, sph::fwd_derivs_f64_n0_m1, sph::fwd_derivs_f64_n0_m2},
       {sph::fwd_derivs_f64_n1_m0, sph::fwd_derivs_f64_n1_m1, sph::fwd_derivs_f64_n1_m2}}};
  const int d = dtype == SPH_F64 ? 1 : 0;
  const int n = norm ? 1 : 0;
  if (!store_dy && !fused) return kValues[d][n](L, variant);
  const int mode = !fused ? sph::kDerivStore : (store_dy ? sph::kDerivFusedStore : sph::kDerivFused);
  return kDerivs[d][n][mode](L, variant);
}
sph::KernelInfo bwd_info(int32_t dtype, int L) {
  return dtype == SPH_F64 ? sph::bwd_info_f64(L) : sph::bwd_info_f32(L);
}
sph::KernelInfo dbwd_info(int32_t dtype, int L, int norm) {
  return dtype == SPH_F64 ? sph::dbwd_info_f64(L, norm) : sph::dbwd_info_f32(L, norm);
}

// Kernels whose dynamic LDS exceeds the default limit get the attribute once.
std::mutex g_attr_mu;
std::map<std::pair<int, const void*>, size_t> g_attr_set;

hipError_t ensure_lds(const void* fn, size_t bytes) {
  if (bytes <= 48 * 1024) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_attr_mu);
  auto key = std::make_pair(dev, fn);
  auto it = g_attr_set.find(key);
  if (it != g_attr_set.end() && it->second >= bytes) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
  if (e == hipSuccess) g_attr_set[key] = bytes;
  return e;
}

int num_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
    return 256;
  return n;
}

hipError_t launch(const void* fn, unsigned grid, unsigned block, size_t lds, void* params,
                  hipStream_t s) {
  void* args[] = {params};
  hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Blocks of a kernel that are resident on one CU at once (from the runtime's
// occupancy for this block size and LDS), cached per device and kernel.  A
// loop-over-tiles grid must not exceed this times the CUs: blocks beyond it
// wait for a whole round.
std::mutex g_occ_mu;
std::map<std::tuple<int, const void*, int, size_t>, int> g_occ;

int resident_per_cu(const void* fn, int block, size_t lds) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lk(g_occ_mu);
  const auto key = std::make_tuple(dev, fn, block, lds);
  auto it = g_occ.find(key);
  if (it != g_occ.end()) return it->second;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess || per_cu <= 0) per_cu = 1;
  (void)hipGetLastError();
  g_occ[key] = per_cu;
  return per_cu;
}

// Grid of a plain forward call: one tile per block.  Blocks that each write
// one tile and exit keep the chip's concurrent stores on a compact, advancing
// address range; a resident grid of blocks looping over tiles spreads them
// over as many separate streams as there are blocks and writes measurably
// slower.  Beyond 2^31 - 1 tiles the kernels loop over the rest.
int64_t plain_grid(int64_t tiles) { return std::max<int64_t>(1, std::min<int64_t>(tiles, 0x7fffffff)); }

// ------------------------------------------------------------ batched path
struct BatchKey {
  int dev, dtype, L, norm, store_dy, bwd;
  bool operator<(const BatchKey& o) const {
    return std::tie(dev, dtype, L, norm, store_dy, bwd) <
           std::tie(o.dev, o.dtype, o.L, o.norm, o.store_dy, o.bwd);
  }
};

// Kernel variant (sph::FwdVariant: unrolled with its default tile, unrolled
// on a 16-point tile, or the run-time-degree kernel) and persistent-grid
// size: blocks_per_cu * CUs blocks loop over the tiles; 0 means one tile per
// block (a plain grid).
struct Choice {
  int variant = sph::kVarDefault;
  int blocks_per_cu = 8;
};

const char* variant_name(int v) {
  switch (v) {
    case sph::kVarDefault: return "default";
    case sph::kVarTile16: return "tile16";
    case sph::kVarRuntime: return "runtime_degree";
    case sph::kVarSplit: return "degree_split";
    case sph::kVarLane: return "one_lane";
    default: return "?";
  }
}

// One instantiated single-node graph per (combination, kernel, LDS size).
// The grid is not part of the key: every call rewrites the node's grid and
// arguments, so a caller whose point count changes from call to call (a
// neighbour list that changes every step) reuses one graph.  Every kernel
// walks its tiles with a grid-stride loop, so any grid is correct.
struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node = nullptr;
};

std::mutex g_batch_mu;
std::map<BatchKey, Choice> g_choice;
std::map<std::tuple<BatchKey, const void*, size_t>, GraphEntry> g_graphs;
int g_use_graph = 1;
int g_autotune = 1;
bool g_cache_loaded = false;

constexpr int kBpcCandidates[] = {2, 4, 8, 16, 0};

std::string cache_path() {
  const char* p = std::getenv("SPH_AUTOTUNE_CACHE");
  return p ? std::string(p) : std::string();
}

// Cache file: one line per combination,
//   dtype L normalize store_dY backward variant blocks_per_cu
// Unreadable or malformed lines are ignored (defaults apply).
void load_cache_locked() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  const std::string path = cache_path();
  if (path.empty()) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    int dt, L, nm, sd, bw, v, b;
    if (!(is >> dt >> L >> nm >> sd >> bw >> v >> b)) continue;
    if (dt < 0 || dt > 1 || L < 0 || L > sph::kMaxLmax || nm < 0 || nm > 1 || sd < 0 || sd > 1 || bw < 0 ||
        bw > 1 || v < 0 || v >= sph::kNumFwdVariants || b < 0 || b > 64)
      continue;
    if (fwd_info(dt == 1 ? SPH_F64 : SPH_F32, L, nm, sd != 0, bw != 0, v).fn == nullptr) continue;
    for (int dev = 0; dev < 64; ++dev) g_choice[BatchKey{dev, dt, L, nm, sd, bw}] = Choice{v, b};
  }
}

void save_cache_locked() {
  const std::string path = cache_path();
  if (path.empty()) return;
  std::ofstream f(path, std::ios::trunc);
  if (!f) return;
  for (const auto& kv : g_choice) {
    if (kv.first.dev != 0) continue;
    f << kv.first.dtype << ' ' << kv.first.L << ' ' << kv.first.norm << ' ' << kv.first.store_dy << ' '
      << kv.first.bwd << ' ' << kv.second.variant << ' ' << kv.second.blocks_per_cu << '\n';
  }
}

unsigned batched_grid(const sph::KernelInfo& ki, int64_t n, int bpc) {
  const int64_t tiles = ceil_div(n, ki.tile_points);
  const int64_t g = bpc > 0 ? std::min<int64_t>(tiles, int64_t(num_cus()) * bpc) : tiles;
  return static_cast<unsigned>(std::max<int64_t>(1, g));
}

// Times every kernel variant of the combination with every persistent-grid
// size on the caller's buffers (the kernel is a pure function of its inputs,
// so repeated runs leave the right result) and returns the fastest.
// Synchronises the host.
Choice autotune(int32_t dtype, int L, int norm, bool store_dy, bool fused, sph::FwdParams params,
                hipStream_t s) {
  Choice best;
  float best_ms = 1e30f;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return best;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return best;
  }
  const void* tried[sph::kNumFwdVariants] = {};
  for (int v = 0; v < sph::kNumFwdVariants; ++v) {
    const sph::KernelInfo ki = fwd_info(dtype, L, norm, store_dy, fused, v);
    if (ki.fn == nullptr) continue;
    bool seen = false;  // two variants may name one kernel
    for (int u = 0; u < v; ++u) seen = seen || tried[u] == ki.fn;
    tried[v] = ki.fn;
    if (seen) continue;
    const size_t lds = fused ? ki.lds_bytes_bwd : ki.lds_bytes;
    if (ensure_lds(ki.fn, lds) != hipSuccess) continue;
    for (int bpc : kBpcCandidates) {
      const unsigned grid = batched_grid(ki, params.n, bpc);
      sph::FwdParams p = params;
      if (launch(ki.fn, grid, ki.block, lds, &p, s) != hipSuccess) continue;  // warm-up
      (void)hipEventRecord(e0, s);
      constexpr int reps = 3;
      bool okr = true;
      for (int r = 0; r < reps && okr; ++r) okr = launch(ki.fn, grid, ki.block, lds, &p, s) == hipSuccess;
      (void)hipEventRecord(e1, s);
      if (!okr || hipEventSynchronize(e1) != hipSuccess) continue;
      float ms = 0;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) continue;
      if (ms < best_ms) {
        best_ms = ms;
        best = Choice{v, bpc};
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGetLastError();
  return best;
}

}  // namespace

extern "C" {

int32_t sph_num_components(int32_t l_max) { return l_max < 0 ? -1 : (l_max + 1) * (l_max + 1); }

int32_t sph_max_lmax(void) { return sph::kMaxLmax; }

const char* sph_status_string(int32_t status) {
  switch (status) {
    case SPH_OK: return "success";
    case SPH_ERR_NULL: return "a required pointer is NULL";
    case SPH_ERR_INVALID: return "invalid argument";
    case SPH_ERR_LMAX: return "l_max out of range";
    case SPH_ERR_OFFSETS: return "inconsistent CSR offsets";
    case SPH_ERR_DEVICE: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* sph_last_error(void) { return g_last_error.c_str(); }

const char* sph_version(void) { return "1.0.0 gfx950"; }

int32_t sph_compute_with_gradients(const void* xyz, int64_t n, int32_t l_max, int32_t normalize,
                                   int32_t dtype, void* Y, void* dY, void* stream) {
  int32_t st = check_common(n, l_max, dtype);
  if (st != SPH_OK) return st;
  if ((st = check_norm(normalize)) != SPH_OK) return st;
  if (n == 0) return ok();
  if (xyz == nullptr || Y == nullptr) return fail(SPH_ERR_NULL, "xyz and Y are required");
  const size_t w = elem_size(dtype);
  const size_t K = static_cast<size_t>(sph_num_components(l_max));
  const size_t un = static_cast<size_t>(n);
  if ((st = check_no_overlap({{Y, un * K * w, "Y"}, {dY, un * 3 * K * w, "dY"}},
                             {{xyz, un * 3 * w, "xyz"}, {Y, un * K * w, "Y"}, {dY, un * 3 * K * w, "dY"}})) !=
      SPH_OK)
    return st;
  const sph::KernelInfo ki = fwd_info(dtype, l_max, normalize, dY != nullptr, false);
  if (ki.fn == nullptr) return fail(SPH_ERR_INVALID, "no kernel for these arguments");
  hipError_t e = ensure_lds(ki.fn, ki.lds_bytes);
  if (e != hipSuccess) return device_fail(e, "hipFuncSetAttribute");
  sph::FwdParams p{xyz, n, l_max, Y, dY, nullptr, nullptr, nullptr, 0, nullptr};
  const int64_t grid = plain_grid(ceil_div(n, ki.tile_points));
  e = launch(ki.fn, static_cast<unsigned>(grid), ki.block, ki.lds_bytes, &p,
             static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "forward launch");
  return ok();
}

int32_t sph_compute(const void* xyz, int64_t n, int32_t l_max, int32_t normalize, int32_t dtype, void* Y,
                    void* stream) {
  return sph_compute_with_gradients(xyz, n, l_max, normalize, dtype, Y, nullptr, stream);
}

int32_t sph_backward(const void* dY, const void* grad_Y, int64_t n, int32_t l_max, int32_t dtype,
                     void* grad_xyz, void* stream) {
  int32_t st = check_common(n, l_max, dtype);
  if (st != SPH_OK) return st;
  if (n == 0) return ok();
  if (dY == nullptr || grad_Y == nullptr || grad_xyz == nullptr)
    return fail(SPH_ERR_NULL, "dY, grad_Y and grad_xyz are required");
  const size_t w = elem_size(dtype);
  const size_t K = static_cast<size_t>(sph_num_components(l_max));
  const size_t un = static_cast<size_t>(n);
  if ((st = check_no_overlap({{grad_xyz, un * 3 * w, "grad_xyz"}},
                             {{dY, un * 3 * K * w, "dY"}, {grad_Y, un * K * w, "grad_Y"}})) != SPH_OK)
    return st;
  const sph::KernelInfo ki = bwd_info(dtype, l_max);
  if (ki.fn == nullptr) return fail(SPH_ERR_INVALID, "no kernel for these arguments");
  sph::BwdParams p{dY, grad_Y, n, static_cast<int32_t>(K), grad_xyz};
  hipError_t e = ensure_lds(ki.fn, ki.lds_bytes);
  if (e != hipSuccess) return device_fail(e, "hipFuncSetAttribute");
  int64_t grid = ceil_div(n, ki.tile_points);
  if (ki.blocks_per_cu > 0)  // a resident grid looping over tiles
    grid = std::min<int64_t>(grid, int64_t(num_cus()) * resident_per_cu(ki.fn, ki.block, ki.lds_bytes));
  if (grid > 0x7fffffff) return fail(SPH_ERR_INVALID, "n too large for one launch");
  e = launch(ki.fn, static_cast<unsigned>(grid), ki.block, ki.lds_bytes, &p, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "backward launch");
  return ok();
}

int32_t sph_double_backward(const void* xyz, const void* grad_Y, const void* v, int64_t n, int32_t l_max,
                            int32_t normalize, int32_t dtype, void* grad_grad_Y, void* grad_xyz2,
                            void* stream) {
  int32_t st = check_common(n, l_max, dtype);
  if (st != SPH_OK) return st;
  if ((st = check_norm(normalize)) != SPH_OK) return st;
  if (n == 0 || (grad_grad_Y == nullptr && grad_xyz2 == nullptr)) return ok();
  if (xyz == nullptr || grad_Y == nullptr || v == nullptr)
    return fail(SPH_ERR_NULL, "xyz, grad_Y and v are required");
  const size_t w = elem_size(dtype);
  const size_t K = static_cast<size_t>(sph_num_components(l_max));
  const size_t un = static_cast<size_t>(n);
  if ((st = check_no_overlap(
           {{grad_grad_Y, un * K * w, "grad_grad_Y"}, {grad_xyz2, un * 3 * w, "grad_xyz2"}},
           {{xyz, un * 3 * w, "xyz"}, {grad_Y, un * K * w, "grad_Y"}, {v, un * 3 * w, "v"},
            {grad_grad_Y, un * K * w, "grad_grad_Y"}, {grad_xyz2, un * 3 * w, "grad_xyz2"}})) != SPH_OK)
    return st;
  const sph::KernelInfo ki = dbwd_info(dtype, l_max, normalize);
  if (ki.fn == nullptr) return fail(SPH_ERR_INVALID, "no kernel for these arguments");
  hipError_t e = ensure_lds(ki.fn, ki.lds_bytes);
  if (e != hipSuccess) return device_fail(e, "hipFuncSetAttribute");
  sph::DbwdParams p{xyz, grad_Y, v, n, l_max, grad_grad_Y, grad_xyz2};
  const int64_t grid = ceil_div(n, ki.tile_points);
  if (grid > 0x7fffffff) return fail(SPH_ERR_INVALID, "n too large for one launch");
  e = launch(ki.fn, static_cast<unsigned>(grid), ki.block, ki.lds_bytes, &p,
             static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "double backward launch");
  return ok();
}

int32_t sph_compute_with_hessians(const void* xyz, int64_t n, int32_t l_max, int32_t normalize, int32_t dtype,
                                  void* Y, void* dY, void* d2Y, void* stream) {
  int32_t st = check_common(n, l_max, dtype);
  if (st != SPH_OK) return st;
  if ((st = check_norm(normalize)) != SPH_OK) return st;
  if (n == 0) return ok();
  if (xyz == nullptr || Y == nullptr || d2Y == nullptr) return fail(SPH_ERR_NULL, "xyz, Y and d2Y are required");
  const size_t w = elem_size(dtype);
  const size_t K = static_cast<size_t>(sph_num_components(l_max));
  const size_t un = static_cast<size_t>(n);
  if ((st = check_no_overlap({{Y, un * K * w, "Y"}, {dY, un * 3 * K * w, "dY"}, {d2Y, un * 9 * K * w, "d2Y"}},
                             {{xyz, un * 3 * w, "xyz"}, {Y, un * K * w, "Y"}, {dY, un * 3 * K * w, "dY"},
                              {d2Y, un * 9 * K * w, "d2Y"}})) != SPH_OK)
    return st;
  const sph::KernelInfo kf = fwd_info(dtype, l_max, normalize, dY != nullptr, false);
  const sph::KernelInfo kh = dtype == SPH_F64 ? sph::hess_info_f64(l_max, normalize)
                                              : sph::hess_info_f32(l_max, normalize);
  if (kf.fn == nullptr || kh.fn == nullptr) return fail(SPH_ERR_INVALID, "no kernel for these arguments");
  hipError_t e = ensure_lds(kf.fn, kf.lds_bytes);
  if (e == hipSuccess) e = ensure_lds(kh.fn, kh.lds_bytes);
  if (e != hipSuccess) return device_fail(e, "hipFuncSetAttribute");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // values and first derivatives: the forward kernel of sph_compute_with_gradients
  sph::FwdParams pf{xyz, n, l_max, Y, dY, nullptr, nullptr, nullptr, 0, nullptr};
  e = launch(kf.fn, static_cast<unsigned>(plain_grid(ceil_div(n, kf.tile_points))), kf.block, kf.lds_bytes, &pf, s);
  if (e != hipSuccess) return device_fail(e, "forward launch");
  sph::HessParams ph{xyz, n, l_max, d2Y};
  e = launch(kh.fn, static_cast<unsigned>(plain_grid(ceil_div(n, kh.tile_points))), kh.block, kh.lds_bytes, &ph, s);
  if (e != hipSuccess) return device_fail(e, "hessian launch");
  return ok();
}

int32_t sph_e3nn_coordinates(const void* xyz, int64_t n, int32_t dtype, void* xyz_p, void* stream) {
  if (n < 0) return fail(SPH_ERR_INVALID, "n must be >= 0");
  if (dtype != SPH_F32 && dtype != SPH_F64) return fail(SPH_ERR_INVALID, "dtype must be SPH_F32 or SPH_F64");
  if (n == 0) return ok();
  if (xyz == nullptr || xyz_p == nullptr) return fail(SPH_ERR_NULL, "xyz and xyz_p are required");
  const size_t bytes = static_cast<size_t>(n) * 3 * elem_size(dtype);
  int32_t st;
  if (xyz_p != xyz &&
      (st = check_no_overlap({{xyz_p, bytes, "xyz_p"}}, {{xyz, bytes, "xyz"}, {xyz_p, bytes, "xyz_p"}})) != SPH_OK)
    return st;
  const hipError_t e = sph::e3nn_coordinates_launch(dtype == SPH_F64, xyz, n, xyz_p, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "e3nn coordinates launch");
  return ok();
}

int32_t sph_e3nn_convert(int64_t n, int32_t l_max, int32_t normalization, int32_t dtype, void* Y, void* dY,
                         void* stream) {
  int32_t st = check_common(n, l_max, dtype);
  if (st != SPH_OK) return st;
  if (normalization < 0 || normalization > 2)
    return fail(SPH_ERR_INVALID, "normalization must be 0 (integral), 1 (component) or 2 (norm)");
  if (n == 0) return ok();
  if (Y == nullptr) return fail(SPH_ERR_NULL, "Y is required");
  const size_t w = elem_size(dtype);
  const size_t K = static_cast<size_t>(sph_num_components(l_max));
  const size_t un = static_cast<size_t>(n);
  if ((st = check_no_overlap({{Y, un * K * w, "Y"}, {dY, un * 3 * K * w, "dY"}},
                             {{Y, un * K * w, "Y"}, {dY, un * 3 * K * w, "dY"}})) != SPH_OK)
    return st;
  const hipError_t e =
      sph::e3nn_convert_launch(dtype == SPH_F64, n, l_max, normalization, Y, dY, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "e3nn convert launch");
  return ok();
}

int32_t sph_radial_expansion(const void* xyz, const int64_t* offsets, int64_t n_env, int64_t n_points,
                             const void* R, int32_t n_max, int32_t l_max, int32_t normalize, int32_t dtype,
                             void* c, int32_t* status, void* stream) {
  int32_t st = check_common(n_points, l_max, dtype);
  if (st != SPH_OK) return st;
  if ((st = check_norm(normalize)) != SPH_OK) return st;
  if (n_env < 0) return fail(SPH_ERR_INVALID, "n_env must be >= 0");
  if (n_max < 1 || n_max > 64) return fail(SPH_ERR_INVALID, "n_max must be in [1, 64]");
  if (offsets == nullptr) return fail(SPH_ERR_NULL, "offsets is required");
  if (n_env > 0 && c == nullptr) return fail(SPH_ERR_NULL, "c is required");
  if (n_points > 0 && (xyz == nullptr || R == nullptr)) return fail(SPH_ERR_NULL, "xyz and R are required");
  if (n_env == 0 && status == nullptr) return ok();
  const size_t w = elem_size(dtype);
  const size_t K = static_cast<size_t>(sph_num_components(l_max));
  const size_t un = static_cast<size_t>(n_points), ue = static_cast<size_t>(n_env);
  const size_t nr = static_cast<size_t>(l_max + 1) * static_cast<size_t>(n_max);
  if ((st = check_no_overlap({{c, ue * n_max * K * w, "c"}, {status, status ? size_t(4) : size_t(0), "status"}},
                             {{xyz, un * 3 * w, "xyz"}, {R, un * nr * w, "R"},
                              {offsets, (ue + 1) * 8, "offsets"}, {c, ue * n_max * K * w, "c"},
                              {status, status ? size_t(4) : size_t(0), "status"}})) != SPH_OK)
    return st;
  const sph::KernelInfo ki = dtype == SPH_F64 ? sph::expand_info_f64(l_max, normalize, n_max)
                                              : sph::expand_info_f32(l_max, normalize, n_max);
  if (ki.fn == nullptr) return fail(SPH_ERR_INVALID, "no kernel for these arguments");
  // The largest chunk (points per LDS tile) within 64 KiB, two blocks per
  // CU; else an 8-point chunk within the 160 KiB of one CU.
  auto lds_of = [&](int chunk) {
    return dtype == SPH_F64 ? sph::expand_lds_bytes<double>(l_max, n_max, chunk)
                            : sph::expand_lds_bytes<float>(l_max, n_max, chunk);
  };
  int chunk = 128;
  while (chunk > 8 && lds_of(chunk) > 64 * 1024) chunk /= 2;
  const size_t lds = lds_of(chunk);
  if (lds > 160 * 1024) return fail(SPH_ERR_INVALID, "l_max and n_max need more LDS than one block has");
  hipError_t e = ensure_lds(ki.fn, lds);
  if (e != hipSuccess) return device_fail(e, "hipFuncSetAttribute");
  sph::ExpandParams p{xyz, R, offsets, n_env, n_points, l_max, n_max, chunk, c, status};
  // a resident grid: each block walks its environments as a pipeline
  const int64_t resident = static_cast<int64_t>(num_cus()) * resident_per_cu(ki.fn, ki.block, lds);
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(n_env, std::max<int64_t>(resident, 1)));
  e = launch(ki.fn, static_cast<unsigned>(grid), ki.block, lds, &p, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "radial expansion launch");
  return ok();
}

int32_t sph_radial_expansion_backward(const void* xyz, const int64_t* offsets, int64_t n_env, int64_t n_points,
                                      const void* R, int32_t n_max, int32_t l_max, int32_t normalize,
                                      int32_t dtype, const void* grad_c, void* grad_xyz, void* grad_R,
                                      int32_t* status, void* stream) {
  int32_t st = check_common(n_points, l_max, dtype);
  if (st != SPH_OK) return st;
  if ((st = check_norm(normalize)) != SPH_OK) return st;
  if (n_env < 0) return fail(SPH_ERR_INVALID, "n_env must be >= 0");
  if (n_max < 1 || n_max > 16) return fail(SPH_ERR_INVALID, "n_max must be in [1, 16]");
  if (offsets == nullptr) return fail(SPH_ERR_NULL, "offsets is required");
  if (n_env > 0 && grad_c == nullptr) return fail(SPH_ERR_NULL, "grad_c is required");
  if (n_points > 0 && (xyz == nullptr || R == nullptr)) return fail(SPH_ERR_NULL, "xyz and R are required");
  if ((n_env == 0 || (grad_xyz == nullptr && grad_R == nullptr)) && status == nullptr) return ok();
  const size_t w = elem_size(dtype);
  const size_t K = static_cast<size_t>(sph_num_components(l_max));
  const size_t un = static_cast<size_t>(n_points), ue = static_cast<size_t>(n_env);
  const size_t nr = static_cast<size_t>(l_max + 1) * static_cast<size_t>(n_max);
  const size_t sb = status ? size_t(4) : size_t(0);
  if ((st = check_no_overlap({{grad_xyz, un * 3 * w, "grad_xyz"}, {grad_R, un * nr * w, "grad_R"},
                              {status, sb, "status"}},
                             {{xyz, un * 3 * w, "xyz"}, {R, un * nr * w, "R"}, {offsets, (ue + 1) * 8, "offsets"},
                              {grad_c, ue * n_max * K * w, "grad_c"}, {grad_xyz, un * 3 * w, "grad_xyz"},
                              {grad_R, un * nr * w, "grad_R"}, {status, sb, "status"}})) != SPH_OK)
    return st;
  const sph::KernelInfo ki = dtype == SPH_F64 ? sph::expand_bwd_info_f64(l_max, normalize, n_max)
                                              : sph::expand_bwd_info_f32(l_max, normalize, n_max);
  if (ki.fn == nullptr) return fail(SPH_ERR_INVALID, "no kernel for these arguments");
  if (ki.lds_bytes > 160 * 1024) return fail(SPH_ERR_INVALID, "l_max and n_max need more LDS than one block has");
  hipError_t e = ensure_lds(ki.fn, ki.lds_bytes);
  if (e != hipSuccess) return device_fail(e, "hipFuncSetAttribute");
  sph::ExpandBwdParams p{xyz, R, offsets, n_env, n_points, l_max, n_max, grad_c, grad_xyz, grad_R, status,
                         ki.slices};
  // a resident grid of one-wave blocks, each block's lane groups
  // (tile_points of them) walking their own environments
  const int64_t resident = static_cast<int64_t>(num_cus()) * resident_per_cu(ki.fn, ki.block, ki.lds_bytes);
  const int64_t grid =
      std::max<int64_t>(1, std::min<int64_t>(ceil_div(n_env, ki.tile_points), std::max<int64_t>(resident, 1)));
  e = launch(ki.fn, static_cast<unsigned>(grid), ki.block, ki.lds_bytes, &p, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "radial expansion backward launch");
  return ok();
}

int32_t sph_batched_set_options(int32_t use_graph, int32_t autotune) {
  if ((use_graph != 0 && use_graph != 1) || (autotune != 0 && autotune != 1))
    return fail(SPH_ERR_INVALID, "options must be 0 or 1");
  std::lock_guard<std::mutex> lk(g_batch_mu);
  g_use_graph = use_graph;
  g_autotune = autotune;
  return ok();
}

int32_t sph_batched_get_config(int32_t l_max, int32_t normalize, int32_t dtype, int32_t store_dY,
                               int32_t with_backward, char* buf, int32_t len) {
  if (buf == nullptr || len <= 0) return fail(SPH_ERR_NULL, "buf is required");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lk(g_batch_mu);
  auto it = g_choice.find(BatchKey{dev, dtype, l_max, normalize, store_dY ? 1 : 0, with_backward ? 1 : 0});
  if (it == g_choice.end()) return fail(SPH_ERR_INVALID, "no configuration chosen yet");
  const sph::KernelInfo ki =
      fwd_info(dtype, l_max, normalize, store_dY != 0, with_backward != 0, it->second.variant);
  std::snprintf(buf, static_cast<size_t>(len), "kernel=%s blocks_per_cu=%d tile_points=%d",
                variant_name(it->second.variant), it->second.blocks_per_cu, ki.tile_points);
  return ok();
}

int32_t sph_batched_set_config(int32_t l_max, int32_t normalize, int32_t dtype, int32_t store_dY,
                               int32_t with_backward, int32_t variant, int32_t blocks_per_cu) {
  int32_t st = check_common(0, l_max, dtype);
  if (st != SPH_OK) return st;
  if ((st = check_norm(normalize)) != SPH_OK) return st;
  if ((store_dY != 0 && store_dY != 1) || (with_backward != 0 && with_backward != 1))
    return fail(SPH_ERR_INVALID, "store_dY and with_backward must be 0 or 1");
  if (variant < 0 || variant >= sph::kNumFwdVariants) return fail(SPH_ERR_INVALID, "unknown variant");
  if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(SPH_ERR_INVALID, "blocks_per_cu must be in 0..64");
  if (fwd_info(dtype, l_max, normalize, store_dY != 0, with_backward != 0, variant).fn == nullptr)
    return fail(SPH_ERR_INVALID, "this variant does not exist for the combination");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  (void)hipGetLastError();
  std::lock_guard<std::mutex> lk(g_batch_mu);
  load_cache_locked();
  g_choice[BatchKey{dev, dtype, l_max, normalize, store_dY, with_backward}] = Choice{variant, blocks_per_cu};
  return ok();
}

int32_t sph_batched_compute(const void* xyz, const int64_t* offsets, int64_t n_env, int64_t n_points,
                            int32_t l_max, int32_t normalize, int32_t dtype, void* Y, void* dY,
                            const void* grad_Y, void* grad_xyz, int32_t* status, void* stream) {
  int32_t st = check_common(n_points, l_max, dtype);
  if (st != SPH_OK) return st;
  if ((st = check_norm(normalize)) != SPH_OK) return st;
  if (n_env < 0) return fail(SPH_ERR_INVALID, "n_env must be >= 0");
  if (offsets == nullptr) return fail(SPH_ERR_NULL, "offsets is required");
  if (grad_Y != nullptr && grad_xyz == nullptr) return fail(SPH_ERR_NULL, "grad_xyz is required with grad_Y");
  if (grad_Y == nullptr && grad_xyz != nullptr) return fail(SPH_ERR_INVALID, "grad_xyz given without grad_Y");
  if (n_points > 0 && (xyz == nullptr || Y == nullptr)) return fail(SPH_ERR_NULL, "xyz and Y are required");
  if (n_points == 0 && status == nullptr) return ok();
  const size_t w = elem_size(dtype);
  const size_t K = static_cast<size_t>(sph_num_components(l_max));
  const size_t un = static_cast<size_t>(n_points);
  if ((st = check_no_overlap({{Y, un * K * w, "Y"}, {dY, un * 3 * K * w, "dY"}, {grad_xyz, un * 3 * w, "grad_xyz"},
                              {status, 4, "status"}},
                             {{xyz, un * 3 * w, "xyz"}, {offsets, (static_cast<size_t>(n_env) + 1) * 8, "offsets"},
                              {Y, un * K * w, "Y"}, {dY, un * 3 * K * w, "dY"}, {grad_Y, un * K * w, "grad_Y"},
                              {grad_xyz, un * 3 * w, "grad_xyz"}, {status, 4, "status"}})) != SPH_OK)
    return st;

  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  e = hipStreamIsCapturing(s, &cap);
  if (e != hipSuccess) return device_fail(e, "hipStreamIsCapturing");
  const bool capturing = cap != hipStreamCaptureStatusNone;

  const bool bwd = grad_Y != nullptr;
  const BatchKey key{dev, dtype, l_max, normalize, dY != nullptr ? 1 : 0, bwd ? 1 : 0};
  sph::FwdParams p{xyz, n_points, l_max, Y, dY, grad_Y, grad_xyz, offsets, n_env, status};

  if (fwd_info(dtype, l_max, normalize, dY != nullptr, bwd).fn == nullptr)
    return fail(SPH_ERR_INVALID, "no kernel for these arguments");

  std::lock_guard<std::mutex> lk(g_batch_mu);
  load_cache_locked();
  Choice ch;
  auto it = g_choice.find(key);
  if (it != g_choice.end()) {
    ch = it->second;
  } else if (g_autotune && !capturing && n_points >= int64_t(64) * 256) {
    ch = autotune(dtype, l_max, normalize, dY != nullptr, bwd, p, s);
    g_choice[key] = ch;
    save_cache_locked();
  }
  // Otherwise (tuning off, a capture in progress, or too few points to time)
  // this call uses the defaults and records nothing, so a later large call
  // outside a capture still tunes the combination.
  const sph::KernelInfo ki = fwd_info(dtype, l_max, normalize, dY != nullptr, bwd, ch.variant);
  if (ki.fn == nullptr) return fail(SPH_ERR_INVALID, "no kernel for the chosen variant");
  const size_t lds = bwd ? ki.lds_bytes_bwd : ki.lds_bytes;
  e = ensure_lds(ki.fn, lds);
  if (e != hipSuccess) return device_fail(e, "hipFuncSetAttribute");
  const unsigned grid = batched_grid(ki, n_points, ch.blocks_per_cu);

  if (!g_use_graph || capturing) {
    e = launch(ki.fn, grid, ki.block, lds, &p, s);
    if (e != hipSuccess) return device_fail(e, "batched launch");
    return ok();
  }

  // One graph per (combination, kernel, LDS); later calls set the kernel
  // node's grid and arguments and replay it.
  auto gkey = std::make_tuple(key, ki.fn, lds);
  GraphEntry& g = g_graphs[gkey];
  void* args[] = {&p};
  hipKernelNodeParams np{};
  np.blockDim = dim3(ki.block);
  np.gridDim = dim3(grid);
  np.func = const_cast<void*>(ki.fn);
  np.kernelParams = args;
  np.sharedMemBytes = static_cast<unsigned>(lds);
  np.extra = nullptr;
  if (g.exec == nullptr) {
    if ((e = hipGraphCreate(&g.graph, 0)) != hipSuccess) return device_fail(e, "hipGraphCreate");
    if ((e = hipGraphAddKernelNode(&g.node, g.graph, nullptr, 0, &np)) != hipSuccess) {
      (void)hipGraphDestroy(g.graph);
      g = GraphEntry{};
      return device_fail(e, "hipGraphAddKernelNode");
    }
    if ((e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0)) != hipSuccess) {
      (void)hipGraphDestroy(g.graph);
      g = GraphEntry{};
      return device_fail(e, "hipGraphInstantiate");
    }
  } else {
    if ((e = hipGraphExecKernelNodeSetParams(g.exec, g.node, &np)) != hipSuccess)
      return device_fail(e, "hipGraphExecKernelNodeSetParams");
  }
  if ((e = hipGraphLaunch(g.exec, s)) != hipSuccess) return device_fail(e, "hipGraphLaunch");
  return ok();
}

}  // extern "C"
