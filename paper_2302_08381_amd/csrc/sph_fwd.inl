// Values-only forward (sph_compute, and the batched entry without
// derivatives): one lane per point, 64-point tiles, grid-stride loop.
// Each lane writes the values of a group of degrees into its LDS row; the
// wave copies the tile out (with one group of degrees the tile is one
// contiguous block of Y and goes out with 16-byte stores).
#pragma once

#include "sph_device.hpp"
#include "sph_launch.hpp"

namespace sph {

// Per-point LDS budget (elements of one group of degrees): one group up to
// l_max = 12 (float) or 8 (double), a 64-row tile of about 44 KB whose rows
// are contiguous in global memory.
template <typename T>
inline constexpr int kValueBudget = 172;
template <>
inline constexpr int kValueBudget<double> = 86;

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

template <typename T, int MM, bool NORM, bool FAST, bool WHOLE, int LA, int LB>
__device__ __forceinline__ void values_group_ct(const Point<T>& pt, int K, int64_t p0, int np, int lane,
                                                const FwdParams& P, T* st) {
  constexpr int kb = LA * LA;
  constexpr int cnt = LB * LB - kb;
  constexpr int S = row_stride<T>(cnt, WHOLE);
  T* row = st + lane * S - kb;
  T cur[MM + 3], unused[MM + 3];
#pragma unroll
  for (int l = LA; l < LB; ++l) {
    q_row<T, MM>(l, pt.ez, pt.rxy2, cur);
    emit_row<T, MM, 0, NORM>(l, unused, cur, pt.ex, pt.ey, pt.ez, pt.inv_r, [&](int k, T v) { row[k] = v; });
  }
  __syncthreads();
  T* dst = static_cast<T*>(P.Y) + p0 * K + kb;
  if constexpr (FAST) {
    static_assert(WHOLE && kb == 0, "fast path needs one group of whole rows");
    constexpr int W = Vec16<T>::n;
    constexpr int CV = S == cnt ? 1 : cnt / W, SV = S == cnt ? 1 : S / W;
    copy_out_full<T, kWave * cnt / W, kWave, CV, SV>(st, dst, lane);
  } else {
    copy_out(st, S, dst, K, cnt, np, lane, aligned16(dst));
  }
  __syncthreads();
}

template <typename T, int MM, bool NORM, bool FAST, int LT, int... Gs>
__device__ __forceinline__ void values_groups_ct(std::integer_sequence<int, Gs...>, const Point<T>& pt, int K,
                                                 int64_t p0, int np, int lane, const FwdParams& P, T* st) {
  constexpr Plan PL = make_plan(LT, kValueBudget<T>);
  (values_group_ct<T, MM, NORM, FAST, PL.ng == 1, PL.lo[Gs], PL.hi[Gs]>(pt, K, p0, np, lane, P, st), ...);
}

template <typename T, int LT>
constexpr bool values_has_fast() {
  if constexpr (LT < 0) {
    return false;
  } else {
    constexpr Plan PL = make_plan(LT, kValueBudget<T>);
    constexpr int K = (LT + 1) * (LT + 1);
    return PL.ng == 1 && (K % 2 == 1 || K % Vec16<T>::n == 0);
  }
}

// LT >= 0: l_max = LT at compile time (MM = LT); LT < 0: l_max = P.L <= MM.
// Dynamic LDS: 64 rows of stride(L) elements.  Full tiles of a one-group
// plan run one straight path with the next tile's coordinates loaded ahead
// (see k_fwd4); the ragged tile and unaligned outputs take the general path.
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
  auto tile_body = [&](int64_t tile, T x, T y, T z, auto fast_c) {
    constexpr bool FAST = decltype(fast_c)::value;
    const int64_t p0 = tile * kWave;
    const int np = FAST ? kWave : static_cast<int>(P.n - p0 < kWave ? P.n - p0 : kWave);
    const Point<T> pt = make_point<T, NORM>(x, y, z);
    if constexpr (LT >= 0) {
      constexpr Plan PL = make_plan(LT, B);
      values_groups_ct<T, MM, NORM, FAST, LT>(std::make_integer_sequence<int, PL.ng>{}, pt, K, p0, np, lane, P,
                                              st);
    } else {
      for (int la = 0; la <= L;) {
        const int lb = group_end(la, L, B);
        const int kb = la * la;
        const int cnt = lb * lb - kb;
        const int S = row_stride<T>(cnt, cnt == K);
        emit_values<T, MM, NORM, false>(pt, la, lb, st + lane * S - kb);
        __syncthreads();
        T* dst = static_cast<T*>(P.Y) + p0 * K + kb;
        copy_out(st, S, dst, K, cnt, np, lane, aligned16(dst));
        __syncthreads();
        la = lb;
      }
    }
  };
  auto load_point = [&](int64_t i, T& x, T& y, T& z) {
    const T* q = xyz + i * 3;
    x = q[0];
    y = q[1];
    z = q[2];
  };

  constexpr bool kFast = values_has_fast<T, LT>();
  const int64_t slot = xcd_slot(blockIdx.x, gridDim.x);  // first tile of this block
  if (kFast && aligned16(P.Y)) {
    const int64_t nfull = P.n / kWave;
    if (slot < nfull) {
      T nx, ny, nz;
      load_point(slot * kWave + lane, nx, ny, nz);
      for (int64_t tile = slot; tile < nfull; tile += gridDim.x) {
        const T x = nx, y = ny, z = nz;
        const int64_t nt = tile + gridDim.x < nfull ? tile + gridDim.x : tile;
        load_point(nt * kWave + lane, nx, ny, nz);
        tile_body(tile, x, y, z, std::integral_constant<bool, kFast>{});
      }
    }
    if (P.n % kWave != 0 && nfull % gridDim.x == slot) {
      T x = T(0), y = T(0), z = T(0);
      if (nfull * kWave + lane < P.n) load_point(nfull * kWave + lane, x, y, z);
      tile_body(nfull, x, y, z, std::false_type{});
    }
  } else {
    for (int64_t tile = slot; tile * kWave < P.n; tile += gridDim.x) {
      T x = T(0), y = T(0), z = T(0);
      if (tile * kWave + lane < P.n) load_point(tile * kWave + lane, x, y, z);
      tile_body(tile, x, y, z, std::false_type{});
    }
  }
}

}  // namespace sph
