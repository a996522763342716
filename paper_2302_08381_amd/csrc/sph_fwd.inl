// Forward kernel: Y, optionally dY, optionally the fused backward
// gxyz = sum_k gY_k dY_k, over 64-point tiles with a grid-stride loop (one
// tile per block for plain calls, a persistent grid for the batched entry).
//
// Per tile and per group of degrees, four passes (value, d/dx, d/dy, d/dz)
// each emit one component of every point of the tile into the lane's LDS row
// and copy the tile out; the derivative passes are skipped when neither dY
// nor the fused backward is requested.
#pragma once

#include "sph_device.hpp"
#include "sph_launch.hpp"

namespace sph {

// Per-point LDS budgets (elements of one component of one group of degrees)
// offered to the autotuner.
template <typename T>
inline constexpr int kBudgets[kNumBudgetVariants] = {84, 170};
template <>
inline constexpr int kBudgets<double>[kNumBudgetVariants] = {66, 84};

template <typename T, int MM, bool NORM, int COMP>
__device__ __forceinline__ void fwd_pass(const Point<T>& pt, int la, int lb, int kb, int S, T* st,
                                         int lane) {
  T prev[MM + 3], cur[MM + 3];
  if constexpr (COMP != 0) q_row<T, MM>(la - 1, pt.ez, pt.rxy2, prev);
  T* row = st + lane * S - kb;
#pragma unroll 1
  for (int l = la; l < lb; ++l) {
    q_row<T, MM>(l, pt.ez, pt.rxy2, cur);
    emit_row<T, MM, COMP, NORM>(l, prev, cur, pt.ex, pt.ey, pt.ez, pt.inv_r,
                                [&](int k, T v) { row[k] = v; });
    if constexpr (COMP != 0) copy_row<T, MM>(l, cur, prev);
  }
}

// One group of degrees [la, lb) for one tile.
template <typename T, int MM, bool NORM>
__device__ __forceinline__ void fwd_group(const Point<T>& pt, int la, int lb, int K, int64_t p0, int np,
                                          const FwdParams& P, T* st, T* sg, T (&acc)[3], int lane) {
  const int kb = la * la;
  const int cnt = lb * lb - kb;
  const int S = cnt | 1;
  const bool store_dy = P.dY != nullptr;
  const bool bwd = P.gY != nullptr;

  if (bwd) {
    const T* src = static_cast<const T*>(P.gY) + p0 * K + kb;
    copy_in(sg, S, src, K, cnt, np, lane, aligned16(src));
  }
  fwd_pass<T, MM, NORM, 0>(pt, la, lb, kb, S, st, lane);
  __syncthreads();
  {
    T* dst = static_cast<T*>(P.Y) + p0 * K + kb;
    copy_out(st, S, dst, K, cnt, np, lane, aligned16(dst));
  }
  __syncthreads();
  if (!store_dy && !bwd) return;

  auto finish = [&](int a) {
    __syncthreads();
    if (bwd) {
      const T* gr = sg + lane * S;
      const T* dr = st + lane * S;
      T s = T(0);
      for (int j = 0; j < cnt; ++j) s += gr[j] * dr[j];
      acc[a] += s;
    }
    if (store_dy) {
      T* dst = static_cast<T*>(P.dY) + p0 * 3 * K + a * K + kb;
      copy_out(st, S, dst, 3 * K, cnt, np, lane, false);
    }
    __syncthreads();
  };
  fwd_pass<T, MM, NORM, 1>(pt, la, lb, kb, S, st, lane);
  finish(0);
  fwd_pass<T, MM, NORM, 2>(pt, la, lb, kb, S, st, lane);
  finish(1);
  fwd_pass<T, MM, NORM, 3>(pt, la, lb, kb, S, st, lane);
  finish(2);
}

// CSR consistency check, done by block 0 only (single writer, no atomics).
__device__ __forceinline__ void check_offsets(const FwdParams& P, int lane) {
  bool ok = true;
  const int64_t* o = P.offsets;
  for (int64_t i = lane; i < P.n_env; i += kWave) ok = ok && (o[i] <= o[i + 1]);
  if (lane == 0) ok = ok && (o[0] == 0) && (o[P.n_env] == P.n);
  const bool all_ok = __all(ok);
  if (lane == 0) P.status[0] = all_ok ? 0 : 4 /* SPH_ERR_OFFSETS */;
}

// MM: m-extent bucket (l_max <= MM); BUDGET: LDS elements per point.
// Dynamic LDS: one staging tile of 64 * stride(L) elements, two with the
// fused backward (the host sizes it from make_plan).
template <typename T, int MM, bool NORM, int BUDGET>
__global__ __launch_bounds__(kWave) void k_fwd(FwdParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const int L = P.L;
  const int K = (L + 1) * (L + 1);
  const int smax = plan_stride(L, BUDGET);
  T* st = reinterpret_cast<T*>(smem);
  T* sg = st + kWave * smax;

  if (P.status != nullptr && blockIdx.x == 0) check_offsets(P, lane);

  const T* xyz = static_cast<const T*>(P.xyz);
  for (int64_t tile = blockIdx.x; tile * kWave < P.n; tile += gridDim.x) {
    const int64_t p0 = tile * kWave;
    const int np = static_cast<int>(P.n - p0 < kWave ? P.n - p0 : kWave);
    T x = T(0), y = T(0), z = T(0);
    if (lane < np) {
      const T* q = xyz + (p0 + lane) * 3;
      x = q[0];
      y = q[1];
      z = q[2];
    }
    const Point<T> pt = make_point<T, NORM>(x, y, z);
    T acc[3] = {T(0), T(0), T(0)};
    for (int la = 0; la <= L;) {
      const int lb = group_end(la, L, BUDGET);
      fwd_group<T, MM, NORM>(pt, la, lb, K, p0, np, P, st, sg, acc, lane);
      la = lb;
    }
    if (P.gY != nullptr && lane < np) {
      T* g = static_cast<T*>(P.gxyz) + (p0 + lane) * 3;
      g[0] = acc[0];
      g[1] = acc[1];
      g[2] = acc[2];
    }
  }
}

}  // namespace sph
