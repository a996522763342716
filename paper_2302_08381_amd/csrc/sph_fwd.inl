// Values-only forward (sph_compute, and the batched entry without
// derivatives): one lane per point, 64-point tiles, grid-stride loop.
// Each lane writes the values of a group of degrees into its LDS row; the
// wave copies the tile out (with one group of degrees the tile is one
// contiguous block of Y and goes out with 16-byte stores).
#pragma once

#include "sph_device.hpp"
#include "sph_launch.hpp"

namespace sph {

// Per-point LDS budget (elements of one group of degrees).
template <typename T>
inline constexpr int kValueBudget = 84;
template <>
inline constexpr int kValueBudget<double> = 66;

// CSR consistency check, done by block 0 only (single writer, no atomics).
__device__ __forceinline__ void check_offsets(const FwdParams& P, int lane) {
  bool ok = true;
  const int64_t* o = P.offsets;
  for (int64_t i = lane; i < P.n_env; i += kWave) ok = ok && (o[i] <= o[i + 1]);
  if (lane == 0) ok = ok && (o[0] == 0) && (o[P.n_env] == P.n);
  const bool all_ok = __all(ok);
  if (lane == 0) P.status[0] = all_ok ? 0 : 4 /* SPH_ERR_OFFSETS */;
}

template <typename T, int MM, bool NORM, bool UNROLL>
__device__ __forceinline__ void emit_values(const Point<T>& pt, int la, int lb, T* row) {
  constexpr int UR = UNROLL ? 64 : 1;
  T cur[MM + 3], unused[MM + 3];
#pragma unroll UR
  for (int l = la; l < lb; ++l) {
    q_row_any<T, MM, UNROLL>(l, pt.ez, pt.rxy2, cur);
    emit_row<T, MM, 0, NORM>(l, unused, cur, pt.ex, pt.ey, pt.ez, pt.inv_r,
                             [&](int k, T v) { row[k] = v; });
  }
}

template <typename T, int MM, bool NORM, int LA, int LB>
__device__ __forceinline__ void values_group_ct(const Point<T>& pt, int K, int64_t p0, int np, int lane,
                                                const FwdParams& P, T* st) {
  constexpr int kb = LA * LA;
  constexpr int cnt = LB * LB - kb;
  constexpr int S = cnt | 1;
  T* row = st + lane * S - kb;
  T cur[MM + 3], unused[MM + 3];
#pragma unroll
  for (int l = LA; l < LB; ++l) {
    q_row<T, MM>(l, pt.ez, pt.rxy2, cur);
    emit_row<T, MM, 0, NORM>(l, unused, cur, pt.ex, pt.ey, pt.ez, pt.inv_r, [&](int k, T v) { row[k] = v; });
  }
  __syncthreads();
  T* dst = static_cast<T*>(P.Y) + p0 * K + kb;
  if constexpr (S == cnt && kb == 0) {
    if (np == kWave && aligned16(dst)) {
      copy_out_full<T, kWave * cnt / Vec16<T>::n>(st, dst, lane);
      __syncthreads();
      return;
    }
  }
  copy_out(st, S, dst, K, cnt, np, lane, aligned16(dst));
  __syncthreads();
}

template <typename T, int MM, bool NORM, int LT, int... Gs>
__device__ __forceinline__ void values_groups_ct(std::integer_sequence<int, Gs...>, const Point<T>& pt, int K,
                                                 int64_t p0, int np, int lane, const FwdParams& P, T* st) {
  constexpr Plan PL = make_plan(LT, kValueBudget<T>);
  (values_group_ct<T, MM, NORM, PL.lo[Gs], PL.hi[Gs]>(pt, K, p0, np, lane, P, st), ...);
}

// LT >= 0: l_max = LT at compile time (MM = LT); LT < 0: l_max = P.L <= MM.
// Dynamic LDS: 64 rows of stride(L) elements.
template <typename T, int MM, int LT, bool NORM>
__global__ __launch_bounds__(kWave) void k_fwd(FwdParams P) {
  constexpr int B = kValueBudget<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  T* st = reinterpret_cast<T*>(smem);
  const int lane = threadIdx.x;
  const int L = LT >= 0 ? LT : P.L;
  const int K = (L + 1) * (L + 1);

  if (P.status != nullptr && blockIdx.x == 0) check_offsets(P, lane);

  const T* xyz = static_cast<const T*>(P.xyz);
  // The coordinates of the block's next tile are loaded while the current
  // tile is processed.
  auto load_point = [&](int64_t tile, T& x, T& y, T& z) {
    const int64_t i = tile * kWave + lane;
    x = y = z = T(0);
    if (i < P.n) {
      const T* q = xyz + i * 3;
      x = q[0];
      y = q[1];
      z = q[2];
    }
  };
  T nx, ny, nz;
  load_point(blockIdx.x, nx, ny, nz);
  for (int64_t tile = blockIdx.x; tile * kWave < P.n; tile += gridDim.x) {
    const int64_t p0 = tile * kWave;
    const int np = static_cast<int>(P.n - p0 < kWave ? P.n - p0 : kWave);
    const T x = nx, y = ny, z = nz;
    load_point(tile + gridDim.x, nx, ny, nz);
    const Point<T> pt = make_point<T, NORM>(x, y, z);
    auto group = [&](int la, int lb, auto unroll_c) {
      constexpr bool UN = decltype(unroll_c)::value;
      const int kb = la * la;
      const int cnt = lb * lb - kb;
      const int S = cnt | 1;
      emit_values<T, MM, NORM, UN>(pt, la, lb, st + lane * S - kb);
      __syncthreads();
      T* dst = static_cast<T*>(P.Y) + p0 * K + kb;
      copy_out(st, S, dst, K, cnt, np, lane, aligned16(dst));
      __syncthreads();
    };
    if constexpr (LT >= 0) {
      constexpr Plan PL = make_plan(LT, B);
      values_groups_ct<T, MM, NORM, LT>(std::make_integer_sequence<int, PL.ng>{}, pt, K, p0, np, lane, P, st);
    } else {
      for (int la = 0; la <= L;) {
        const int lb = group_end(la, L, B);
        group(la, lb, std::false_type{});
        la = lb;
      }
    }
  }
}

}  // namespace sph
