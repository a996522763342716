// Backward (vector-Jacobian product) with stored derivatives:
//   gxyz[i,a] = sum_k gY[i,k] dY[i,a,k]
// A streaming contraction (no MFMA: one short dot product per point and
// axis).  A block of NW waves takes 16 NW points: two waves (32 points) for
// float with K <= 86, whose share of gY and dY is then a whole number of
// 128-byte lines for odd K, and one wave (16 points) otherwise.  The gY rows
// and the 3 x 16 NW dY rows of those points are copied into LDS with coalesced
// (16-byte when possible) loads in balanced chunks of at most KC columns (the
// tile stays near 44 KB), kBwdBatch loads in flight per thread: deep enough
// that one round trip covers a chunk, since at the occupancy the LDS tile
// allows the kernel is bound by read latency.  Thread (p, q) then sums
// columns k = q (mod 4) of point p for the three axes, and the four partial
// sums are combined with two lane exchanges.  The summation order is fixed,
// so the result is deterministic.
#pragma once

#include "sph_device.hpp"
#include "sph_launch.hpp"

namespace sph {

// Columns per chunk for blocks of NW waves.
template <typename T, int NW>
constexpr int bwd_chunk() {
  return (std::is_same_v<T, float> ? 172 : 86) / NW;
}
// Waves per block for K components.
template <typename T>
constexpr int bwd_waves(int K) {
  return (std::is_same_v<T, float> && K <= bwd_chunk<T, 2>()) ? 2 : 1;
}

// LDS stride (elements per row) that holds every chunk of K columns for
// blocks of NW waves: the rows of one whole-row chunk, or the odd width of
// the balanced chunks.  The dynamic LDS of a block is 4 * 16 NW rows of it.
template <typename T, int NW>
__host__ __device__ constexpr int bwd_stride(int K) {
  const int KC = bwd_chunk<T, NW>();
  const int nch = (K + KC - 1) / KC;
  const int ch = (K + nch - 1) / nch;
  return nch == 1 ? row_stride<T>(K, true) : (ch | 1);
}
constexpr int kBwdBatch = 16;
// Loads in flight per thread for a one-chunk tile (gY and dY together):
// measured best at 32 for float (two-wave blocks) and 48 for double (one-wave
// blocks, 40.5 vectors per thread at l_max = 8); other depths are slower.
template <typename T>
inline constexpr int kBwdPairBatch = std::is_same_v<T, float> ? 32 : 48;
// The pipelined loop over tiles (see k_bwd): float two-wave blocks (20.25
// vectors per thread at l_max = 8, batches of 24 and two waves per SIMD, no
// spills) and double one-wave blocks (batches of 48).
template <typename T, int NW>
inline constexpr bool kBwdPipe = !std::is_same_v<T, float> || NW == 2;
template <typename T>
inline constexpr int kBwdPipeBatch = std::is_same_v<T, float> ? 24 : 48;

template <typename T, int NW>
__global__ __launch_bounds__(kWave * NW)
__attribute__((amdgpu_waves_per_eu(std::is_same_v<T, float> && kBwdPipe<T, NW> ? 2 : 1))) void k_bwd(BwdParams P) {
  constexpr int PP = 16 * NW;   // points per block
  constexpr int NT = kWave * NW;
  constexpr int KC = bwd_chunk<T, NW>();
  extern __shared__ __align__(16) unsigned char smem[];
  const int K = P.K;
  T* sg = reinterpret_cast<T*>(smem);            // PP rows
  T* sd = sg + PP * bwd_stride<T, NW>(K);        // 3 PP rows
  const int lane = threadIdx.x;
  const int pl = lane >> 2;
  const int q = lane & 3;
  const int nch = (K + KC - 1) / KC;
  const int ch = (K + nch - 1) / nch;  // balanced chunk width, <= KC

  // sum over columns k = q (mod 4) of point pl, then over the four lanes
  auto reduce = [&](int S, int cnt, T& a0, T& a1, T& a2) {
    const T* g = sg + pl * S;
    const T* d0 = sd + (3 * pl) * S;
    const T* d1 = d0 + S;
    const T* d2 = d1 + S;
#pragma unroll 4
    for (int k = q; k < cnt; k += 4) {
      const T gv = g[k];
      a0 += gv * d0[k];
      a1 += gv * d1[k];
      a2 += gv * d2[k];
    }
  };
  auto finish = [&](int64_t p0, int np, T a0, T a1, T a2) {
    a0 += __shfl_xor(a0, 1);
    a1 += __shfl_xor(a1, 1);
    a2 += __shfl_xor(a2, 1);
    a0 += __shfl_xor(a0, 2);
    a1 += __shfl_xor(a1, 2);
    a2 += __shfl_xor(a2, 2);
    if (pl < np && q < 3) {
      const T v = (q == 0) ? a0 : (q == 1 ? a1 : a2);
      static_cast<T*>(P.gxyz)[(p0 + pl) * 3 + q] = v;
    }
  };
  // one tile, any shape: chunks of columns through LDS
  auto general_tile = [&](int64_t p0) {
    const int np = static_cast<int>(P.n - p0 < PP ? P.n - p0 : PP);
    const T* gY = static_cast<const T*>(P.gY) + p0 * K;
    const T* dY = static_cast<const T*>(P.dY) + p0 * 3 * K;
    T a0 = T(0), a1 = T(0), a2 = T(0);
    for (int kc0 = 0; kc0 < K; kc0 += ch) {
      const int cnt = (K - kc0) < ch ? (K - kc0) : ch;
      const int S = row_stride<T>(cnt, cnt == K);
      if (cnt == K && S == K && aligned16(gY) && aligned16(dY)) {
        // one chunk of whole rows: the gY and dY blocks share the round trips
        // (where the pipelined loop exists this is only the ragged last tile:
        // a small batch keeps the kernel's registers for the loop)
        copy_in_pair<NT, kBwdPipe<T, NW> ? 8 : kBwdPairBatch<T>>(sg, gY, np * K, sd, dY, 3 * np * K, lane);
      } else {
        copy_in<NT, kBwdBatch>(sg, S, gY + kc0, K, cnt, np, lane, aligned16(gY + kc0));
        copy_in<NT, kBwdBatch>(sd, S, dY + kc0, K, cnt, 3 * np, lane, aligned16(dY + kc0));
      }
      __syncthreads();
      if (pl < np) reduce(S, cnt, a0, a1, a2);
      __syncthreads();
    }
    finish(p0, np, a0, a1, a2);
  };

  // Full tiles of one contiguous chunk whose gY and dY fit one register batch
  // (the block's 16-byte vectors, nva + nvb <= NT * NB) run a loop over tiles
  // (the host launches a resident grid) that loads tile t + G into registers
  // while it reduces tile t from LDS, so the loads stay in flight across
  // tiles.  N = 1e6, l_max = 8: double 514 -> 437 us on the resident grid;
  // float 226 -> 202 us at one tile per block (the batch in registers, then
  // one commit to LDS, against the batched copy of general_tile).
  using V = typename Vec16<T>::type;
  constexpr int W = Vec16<T>::n;
  constexpr int NB = kBwdPipeBatch<T>;
  constexpr bool kPipe = kBwdPipe<T, NW>;
  const int nva = PP * K / W, nvb = 3 * nva, nv = nva + nvb;
  const int64_t nfull = P.n / PP;
  const bool pipe = kPipe && K <= KC && row_stride<T>(K, true) == K && (PP * K) % W == 0 && nv <= NT * NB &&
                    aligned16(P.gY) && aligned16(P.dY);
  int64_t tile = blockIdx.x;
  if constexpr (kPipe) {
   if (pipe) {
    V v[NB];
    auto issue = [&](int64_t t) {
      const V* ga = reinterpret_cast<const V*>(static_cast<const T*>(P.gY) + t * PP * K);
      const V* gb = reinterpret_cast<const V*>(static_cast<const T*>(P.dY) + t * PP * 3 * K);
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int i = lane + u * NT;
        if (i < nv) v[u] = __builtin_nontemporal_load(i < nva ? ga + i : gb + (i - nva));
      }
    };
    V* la = reinterpret_cast<V*>(sg);
    V* lb = reinterpret_cast<V*>(sd);
    if (tile < nfull) issue(tile);
    for (; tile < nfull; tile += gridDim.x) {
      // Wait for the whole batch once, on every path: with the waits left to
      // the compiler, the stores below (each under its own lane condition)
      // leave the batch possibly in flight on the skipped paths, and every
      // load of the next batch then waits for all loads before it.
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int i = lane + u * NT;
        if (i < nv) *(i < nva ? la + i : lb + (i - nva)) = v[u];
      }
      __syncthreads();
      if (tile + gridDim.x < nfull) issue(tile + gridDim.x);
      T a0 = T(0), a1 = T(0), a2 = T(0);
      reduce(K, K, a0, a1, a2);
      finish(tile * PP, PP, a0, a1, a2);
      __syncthreads();
    }
   }
  }
  for (; tile * PP < P.n; tile += gridDim.x) general_tile(tile * PP);
}

}  // namespace sph
