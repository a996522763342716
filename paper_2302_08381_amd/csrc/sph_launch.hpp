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

// Explicit Hessians (k_hess).
struct HessParams {
  const void* xyz;  // [n,3]
  int64_t n;
  int32_t L;
  void* d2Y;        // [n,3,3,K]
};

// Radial expansion over CSR environments (k_expand).
struct ExpandParams {
  const void* xyz;         // [n,3]
  const void* R;           // [n, L+1, n_max]
  const int64_t* offsets;  // [n_env+1]
  int64_t n_env;
  int64_t n;               // points (offsets[n_env] when consistent)
  int32_t L;
  int32_t n_max;
  int32_t chunk;           // points per LDS chunk (<= 128)
  void* c;                 // [n_env, n_max, K]
  int32_t* status;         // device status word or null
};

// LDS layout of one block (elements of T):
//   Y tile:   chunk rows of stride expand_ystride(K) (odd: conflict-free
//             column reads and row writes)
//   R tile:   chunk rows of (L+1) * NP, NP = n_max rounded up to the
//             accumulator width (4 or 8), zero padded, so each thread's
//             channels are aligned 16-byte vectors
//   C tile:   NP * K partial sums
__host__ __device__ constexpr int expand_ystride(int K) { return K | 1; }
__host__ __device__ constexpr int expand_np(int n_max, int acc) { return (n_max + acc - 1) / acc * acc; }
// Channels per accumulator item: 8 where 4 would need more than one pass of
// the block's 128 threads over the (column, channel group) items and there
// are more than 4 channels; else 4.  (Measured on 20 000 environments with 8
// channels: 8 is faster at l_max 8 and 12, 4 at l_max 3 and 6.)
__host__ __device__ constexpr int expand_acc(int L, int n_max) {
  return n_max > 4 && (L + 1) * (L + 1) * expand_np(n_max, 4) / 4 > 128 ? 8 : 4;
}
template <typename T>
__host__ __device__ constexpr size_t expand_lds_bytes(int L, int n_max, int chunk) {
  const int K = (L + 1) * (L + 1);
  // the Y tile is rounded to 16 bytes so the R tile starts aligned
  const size_t ytile = (static_cast<size_t>(chunk) * expand_ystride(K) * sizeof(T) + 15) & ~size_t(15);
  const int np = expand_np(n_max, expand_acc(L, n_max));
  return ytile + sizeof(T) * (static_cast<size_t>(chunk) * (L + 1) * np + static_cast<size_t>(np) * K);
}

// Backward of the radial expansion (k_expand_bwd).
struct ExpandBwdParams {
  const void* xyz;         // [n,3]
  const void* R;           // [n, L+1, n_max]
  const int64_t* offsets;  // [n_env+1]
  int64_t n_env;
  int64_t n;
  int32_t L;
  int32_t n_max;
  const void* gc;          // [n_env, n_max, K] upstream gradient of c
  void* gxyz;              // [n,3] or null
  void* gR;                // [n, L+1, n_max] or null
  int32_t* status;         // device status word or null
  int32_t slices;          // G slices per lane group: 2 (chunks may span two environments) or 1
};
// Row stride (elements) of the backward's LDS radial tile: (L+1) * np
// channels, padded so that a row spans an odd number of 16-byte vectors
// (lanes reading their rows as 16-byte vectors hit distinct banks).
template <typename T>
__host__ __device__ constexpr int expand_bwd_row_stride(int L, int np) {
  constexpr int W = 16 / static_cast<int>(sizeof(T));
  const int s = (L + 1) * np;
  return (s / W) % 2 == 1 ? s : s + W;
}
// LDS of one backward block (one wave in groups of gs lanes): each group's
// environment gradients G as [K][np], `slices` of them (two where a chunk
// may span two environments), and, when staged, its radial tile of gs rows.
template <typename T>
__host__ __device__ constexpr size_t expand_bwd_lds_bytes(int L, int np, int gs, bool stage, int slices = 2) {
  const int K = (L + 1) * (L + 1);
  const size_t per = static_cast<size_t>(slices) * K * np +
                     (stage ? static_cast<size_t>(gs) * expand_bwd_row_stride<T>(L, np) : 0);
  return sizeof(T) * static_cast<size_t>(64 / gs) * per;
}

// A kernel's host stub, its dynamic LDS bytes (for the l_max it was looked
// up with), and for the forward with derivatives the LDS bytes when the
// backward is fused (the extra upstream-gradient tile); tile_points is the
// number of points one block covers per tile and block its threads.
struct KernelInfo {
  const void* fn;
  size_t lds_bytes;
  size_t lds_bytes_bwd;
  int tile_points;
  int block;
  int blocks_per_cu = 0;  // plain calls: 1: a resident grid (occupancy x CUs) loops over tiles; 0: one tile per block
  int slices = 0;         // the expansion backward: G slices per lane group
};

// Per element type (suffix f32 / f64) and normalisation; fn == nullptr when
// the arguments are out of range or the variant does not exist for l_max.
//   values:      Y only (one lane per point, 64-point tiles, 64 threads)
//   derivatives: four lanes per point, 32- or 16-point tiles (one lane per point
//                and 64-point tiles for the one-lane kernel); mode
//                kDerivStore (Y and dY), kDerivFusedStore (Y, dY and the
//                fused backward), kDerivFused (Y and the fused backward)
// Variants (the batched autotuner's candidates; two may name one kernel):
//   kVarDefault  the one-lane kernel for l_max <= 1; else the compile-time
//                (unrolled) kernel where one exists, on its
//                default tile (32 points on two waves for float l_max <= 8,
//                the degree-split tile where that measured faster, else 16
//                points on one wave), else the run-time-degree kernel (with
//                each group's degrees split between two waves unless the
//                backward is fused)
//   kVarTile16   the compile-time kernel on an unsplit 16-point, one-wave tile
//   kVarRuntime  the unsplit run-time-degree (not unrolled) kernel
//   kVarSplit    a degree-split kernel: the compile-time one (float l_max
//                9..12, double 4..8) or the run-time-degree one (larger
//                l_max, no fused backward)
//   kVarLane     l_max <= 3: one lane per point, 64-point one-wave tiles
enum DerivMode { kDerivStore = 0, kDerivFusedStore = 1, kDerivFused = 2, kNumDerivModes = 3 };
enum FwdVariant { kVarDefault = 0, kVarTile16 = 1, kVarRuntime = 2, kVarSplit = 3, kVarLane = 4, kNumFwdVariants = 5 };
KernelInfo fwd_values_f32_n0(int L, int variant);
KernelInfo fwd_values_f32_n1(int L, int variant);
KernelInfo fwd_values_f64_n0(int L, int variant);
KernelInfo fwd_values_f64_n1(int L, int variant);
KernelInfo fwd_derivs_f32_n0_m0(int L, int variant);
KernelInfo fwd_derivs_f32_n0_m1(int L, int variant);
KernelInfo fwd_derivs_f32_n0_m2(int L, int variant);
KernelInfo fwd_derivs_f32_n1_m0(int L, int variant);
KernelInfo fwd_derivs_f32_n1_m1(int L, int variant);
KernelInfo fwd_derivs_f32_n1_m2(int L, int variant);
KernelInfo fwd_derivs_f64_n0_m0(int L, int variant);
KernelInfo fwd_derivs_f64_n0_m1(int L, int variant);
KernelInfo fwd_derivs_f64_n0_m2(int L, int variant);
KernelInfo fwd_derivs_f64_n1_m0(int L, int variant);
KernelInfo fwd_derivs_f64_n1_m1(int L, int variant);
KernelInfo fwd_derivs_f64_n1_m2(int L, int variant);
KernelInfo bwd_info_f32(int L);
KernelInfo bwd_info_f64(int L);
KernelInfo dbwd_info_f32(int L, int normalize);
KernelInfo dbwd_info_f64(int L, int normalize);
// Explicit Hessians: the run-time-degree kernel of the m-extent bucket of L,
// with a two-wave degree-split block where the nine rows of a point fit one
// group of degrees; tile_points = 16.
KernelInfo hess_info_f32(int L, int normalize);
KernelInfo hess_info_f64(int L, int normalize);
// Radial expansion: the compile-time kernel of L (float L <= 12, double
// L <= 8), else the one of the m-extent bucket of L (run-time degree), with
// the accumulator width expand_acc(L, n_max);
// lds_bytes is left 0 (it depends on n_max and the chunk, see
// expand_lds_bytes), block = 128 threads.
KernelInfo expand_info_f32(int L, int normalize, int n_max);
KernelInfo expand_info_f64(int L, int normalize, int n_max);
// Its backward: channels padded to 8 or 16 (n_max <= 16); tile_points holds
// the lane groups per block, slices the G slices per group (two unless two
// do not fit one block's LDS).
KernelInfo expand_bwd_info_f32(int L, int normalize, int n_max);
KernelInfo expand_bwd_info_f64(int L, int normalize, int n_max);
// e3nn's conventions: the permuted coordinates and the in-place conversion
// of Y and dY (dtype64: double, else float).
hipError_t e3nn_coordinates_launch(int dtype64, const void* xyz, int64_t n, void* out, hipStream_t s);
hipError_t e3nn_convert_launch(int dtype64, int64_t n, int L, int normalization, void* Y, void* dY,
                               hipStream_t s);

}  // namespace sph
