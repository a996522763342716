// Forward with derivatives for small l_max (<= 3): one lane per point.
//
// At l_max <= 3 a point has at most 16 columns, so one lane forms the
// values and all three derivative rows of its point (the compile-time
// recursion unrolls into a short straight sequence of products with
// literal coefficients) and a 64-point tile needs one wave.  The quad-lane
// kernel spends four lanes, a two-wave block and a block barrier on a tile of
// 32 points, which at these sizes is mostly per-tile overhead.
//
// LDS tile laid out like global memory: 64 value rows (the tile's block of
// Y) followed by 192 derivative rows (dY[p][a]), rows of stride S.  Rows
// leave as 16-byte stores.  The fused backward adds, in lane p,
// grad_xyz[p][a] = sum_k gY[p,k] dY[p,a,k] from the gY tile (loaded to
// registers before the emission, committed to LDS after it) and the
// derivative rows in LDS, so dY is read back from LDS and never from memory.
#pragma once

#include "sph_device.hpp"
#include "sph_fwd.inl"
#include "sph_launch.hpp"

namespace sph {

constexpr int kLaneMaxL = 3;  // largest l_max of the one-lane kernel

template <typename T, int LT, bool NORM, bool FUSED, bool STORE, bool FAST>
__device__ __forceinline__ void fwd1_tile(const Point<T>& pt, int64_t p0, int np, int lane, const FwdParams& P,
                                          T* st) {
  constexpr int PT = kWave;
  constexpr int K = (LT + 1) * (LT + 1);
  constexpr int S = row_stride<T>(K, true);
  constexpr int W = Vec16<T>::n;
  constexpr int CV = S == K ? 1 : K / W, SV = S == K ? 1 : S / W;
  T* sg = st + 4 * PT * S;  // gY tile (fused)
  TilePrefetch<T, FUSED && FAST ? PT * K / W : 1, kWave, CV, SV> gpre;
  if constexpr (FUSED && FAST) gpre.prefetch(static_cast<const T*>(P.gY) + p0 * K, lane);

  T* yrow = st + lane * S;
  T* drow = st + (PT + 3 * lane) * S;
  T prev[LT + 3], cur[LT + 3];
#pragma unroll
  for (int l = 0; l <= LT; ++l) {
    copy_row<T, LT>(l - 1, cur, prev);
    q_row<T, LT>(l, pt.ez, pt.rxy2, cur);
    emit_row<T, LT, 0, NORM>(l, prev, cur, pt.ex, pt.ey, pt.ez, pt.inv_r, [&](int k, T v) { yrow[k] = v; });
    emit_row<T, LT, 1, NORM>(l, prev, cur, pt.ex, pt.ey, pt.ez, pt.inv_r, [&](int k, T v) { drow[k] = v; });
    emit_row<T, LT, 2, NORM>(l, prev, cur, pt.ex, pt.ey, pt.ez, pt.inv_r, [&](int k, T v) { drow[S + k] = v; });
    emit_row<T, LT, 3, NORM>(l, prev, cur, pt.ex, pt.ey, pt.ez, pt.inv_r,
                             [&](int k, T v) { drow[2 * S + k] = v; });
  }
  if constexpr (FUSED) {
    if constexpr (FAST) {
      gpre.commit(sg, lane);
    } else {
      const T* src = static_cast<const T*>(P.gY) + p0 * K;
      copy_in<kWave>(sg, S, src, K, K, np, lane, aligned16(src));
    }
  }
  __syncthreads();
  if constexpr (FUSED) {
    const T* g = sg + lane * S;
    T a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const T gk = g[k];
      a0 += gk * drow[k];
      a1 += gk * drow[S + k];
      a2 += gk * drow[2 * S + k];
    }
    if (lane < np) {
      T* gx = static_cast<T*>(P.gxyz) + (p0 + lane) * 3;
      gx[0] = a0;
      gx[1] = a1;
      gx[2] = a2;
    }
  }
  T* ydst = static_cast<T*>(P.Y) + p0 * K;
  T* ddst = STORE ? static_cast<T*>(P.dY) + p0 * 3 * K : nullptr;
  if constexpr (FAST) {
    copy_out_full<T, PT * K / W, kWave, CV, SV>(st, ydst, lane);
    if constexpr (STORE) copy_out_full<T, 3 * PT * K / W, kWave, CV, SV>(st + PT * S, ddst, lane);
  } else {
    copy_out(st, S, ydst, K, K, np, lane, aligned16(ydst));
    if constexpr (STORE) copy_out(st + PT * S, S, ddst, K, K, 3 * np, lane, aligned16(ddst));
  }
  __syncthreads();
}

// l_max = LT <= 3 at compile time.  One wave per block, a 64-point tile per
// loop step.  Dynamic LDS: 4 * 64 rows of row_stride(K) elements, plus 64
// rows for the gY tile when FUSED.  The loop structure is that of k_fwd4:
// full tiles run one straight path with the next tile's coordinates loaded
// ahead; the ragged last tile and unaligned outputs take the general path.
template <typename T, int LT, bool NORM, bool FUSED, bool STORE>
__global__ __launch_bounds__(kWave) void k_fwd1(FwdParams P) {
  static_assert(LT >= 0 && LT <= kLaneMaxL, "one-lane kernel: l_max <= 3");
  constexpr int PT = kWave;
  constexpr int K = (LT + 1) * (LT + 1);
  constexpr int W = Vec16<T>::n;
  extern __shared__ __align__(16) unsigned char smem[];
  T* st = reinterpret_cast<T*>(smem);
  const int lane = threadIdx.x;

  if (P.status != nullptr && blockIdx.x == 0) check_offsets(P, lane);

  const T* xyz = static_cast<const T*>(P.xyz);
  auto tile_body = [&](int64_t tile, T x, T y, T z, auto fast_c) {
    constexpr bool FAST = decltype(fast_c)::value;
    const int64_t p0 = tile * PT;
    const int np = FAST ? PT : static_cast<int>(P.n - p0 < PT ? P.n - p0 : PT);
    fwd1_tile<T, LT, NORM, FUSED, STORE, FAST>(make_point<T, NORM>(x, y, z), p0, np, lane, P, st);
  };
  auto load_point = [&](int64_t i, T& x, T& y, T& z) {
    const T* q = xyz + i * 3;
    x = q[0];
    y = q[1];
    z = q[2];
  };

  // whole tiles are whole numbers of 16-byte vectors for every K
  static_assert((PT * K) % W == 0, "tile of whole vectors");
  const bool aligned = aligned16(P.Y) && (!STORE || aligned16(P.dY)) && (!FUSED || aligned16(P.gY));
  const int64_t slot = xcd_slot(blockIdx.x, gridDim.x);
  if (aligned) {
    const int64_t nfull = P.n / PT;
    if (slot < nfull) {
      T nx, ny, nz;
      load_point(slot * PT + lane, nx, ny, nz);
      for (int64_t tile = slot; tile < nfull; tile += gridDim.x) {
        const T x = nx, y = ny, z = nz;
        const int64_t nt = tile + gridDim.x < nfull ? tile + gridDim.x : tile;
        load_point(nt * PT + lane, nx, ny, nz);
        tile_body(tile, x, y, z, std::true_type{});
      }
    }
    if (P.n % PT != 0 && nfull % gridDim.x == slot) {
      T x = T(0), y = T(0), z = T(0);
      if (nfull * PT + lane < P.n) load_point(nfull * PT + lane, x, y, z);
      tile_body(nfull, x, y, z, std::false_type{});
    }
  } else {
    for (int64_t tile = slot; tile * PT < P.n; tile += gridDim.x) {
      T x = T(0), y = T(0), z = T(0);
      if (tile * PT + lane < P.n) load_point(tile * PT + lane, x, y, z);
      tile_body(tile, x, y, z, std::false_type{});
    }
  }
}

}  // namespace sph
