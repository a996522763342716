// Radial expansion over CSR environments (Sec. I, Eq. expansion):
//   c[e, n, l^2+l+m] = sum over the points j of environment e of
//                      R[j, l, n] * Y_l^m(x_j)
// with the radial values R[j, l, n] supplied by the caller.  The harmonics
// never leave the chip: one block takes one environment at a time, writes
// the values of a chunk of its points into an LDS tile (one thread per
// point, the values-only emission), copies the chunk's radial values next to
// it, and contracts the two tiles into per-thread accumulators; partial sums
// of environments longer than one chunk wait in LDS.
#pragma once

#include "sph_device.hpp"
#include "sph_fwd.inl"  // emit_values
#include "sph_launch.hpp"

namespace sph {

constexpr int kExpandThreads = 128;  // two waves
constexpr int kExpandAcc = 4;        // radial channels per accumulator item
constexpr int kExpandRBatch = 32;    // radial values in flight per thread

// Environment e's point range, clamped into [0, n] so that inconsistent
// offsets (reported through the status word) never index out of bounds.
__device__ __forceinline__ void env_range(const int64_t* o, int64_t e, int64_t n, int64_t& b, int64_t& t) {
  int64_t lo = o[e], hi = o[e + 1];
  lo = lo < 0 ? 0 : (lo > n ? n : lo);
  hi = hi < lo ? lo : (hi > n ? n : hi);
  b = lo;
  t = hi;
}

template <typename T, int MM, bool NORM>
__global__ __launch_bounds__(kExpandThreads) void k_expand(ExpandParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int L = P.L;
  const int K = (L + 1) * (L + 1);
  const int SY = expand_ystride(K);
  const int NM = P.n_max;
  const int NP = expand_np(NM);
  const int RS = (L + 1) * NP;  // R tile row stride
  const int JC = P.chunk;
  T* sY = reinterpret_cast<T*>(smem);
  T* sR = reinterpret_cast<T*>(smem + ((static_cast<size_t>(JC) * SY * sizeof(T) + 15) & ~size_t(15)));
  T* sC = sR + static_cast<size_t>(JC) * RS;
  const T* xyz = static_cast<const T*>(P.xyz);
  const T* R = static_cast<const T*>(P.R);
  T* c = static_cast<T*>(P.c);
  const int items = K * (NP / kExpandAcc);

  // CSR consistency, by the first wave of block 0 (one writer, no atomics)
  if (P.status != nullptr && blockIdx.x == 0 && tid < kWave) {
    bool ok = true;
    for (int64_t i = tid; i < P.n_env; i += kWave) ok = ok && (P.offsets[i] <= P.offsets[i + 1]);
    if (tid == 0) ok = ok && P.offsets[0] == 0 && P.offsets[P.n_env] == P.n;
    const bool all_ok = __all(ok);
    if (tid == 0) P.status[0] = all_ok ? 0 : 4 /* SPH_ERR_OFFSETS */;
  }

  for (int64_t e = blockIdx.x; e < P.n_env; e += gridDim.x) {
    int64_t b, t;
    env_range(P.offsets, e, P.n, b, t);
    T* ce = c + e * NM * K;
    for (int64_t j0 = b; j0 < t; j0 += JC) {
      const int cnt = static_cast<int>(t - j0 < JC ? t - j0 : JC);
      // The chunk's radial values (global rows [j][l][n], contiguous): the
      // first batch of loads is issued before the harmonics are computed so
      // that its latency hides behind them.  Indices past the chunk load its
      // last element again (in bounds, never stored), which keeps the loads
      // unconditional.
      const int nrv = cnt * (L + 1) * NM;
      const T* Rg = R + j0 * (L + 1) * NM;
      T rb[kExpandRBatch];
      auto rload = [&](int base) {
#pragma unroll
        for (int u = 0; u < kExpandRBatch; ++u) {
          const int i = base + tid + u * kExpandThreads;
          rb[u] = Rg[i < nrv ? i : nrv - 1];
        }
      };
      auto rstore = [&](int base) {
        __builtin_amdgcn_s_waitcnt(kWaitVmem0);  // one wait for the whole batch
#pragma unroll
        for (int u = 0; u < kExpandRBatch; ++u) {
          const int i = base + tid + u * kExpandThreads;
          if (i < nrv) {
            const int row = NP == NM ? 0 : i / NM;
            sR[NP == NM ? i : row * NP + (i - row * NM)] = rb[u];
          }
        }
      };
      rload(0);
      // the chunk's harmonics, one thread per point
      if (tid < cnt) {
        const T* q = xyz + (j0 + tid) * 3;
        const Point<T> pt = make_point<T, NORM>(q[0], q[1], q[2]);
        emit_values<T, MM, NORM, false>(pt, 0, L + 1, sY + tid * SY);
      }
      rstore(0);
      for (int base = kExpandRBatch * kExpandThreads; base < nrv; base += kExpandRBatch * kExpandThreads) {
        rload(base);
        rstore(base);
      }
      if (NP != NM) {
        const int nr = cnt * (L + 1);
        const int pad = NP - NM;
        for (int i = tid; i < nr * pad; i += kExpandThreads) {
          const int row = i / pad;
          sR[row * NP + NM + (i - row * pad)] = T(0);
        }
      }
      __syncthreads();
      for (int it = tid; it < items; it += kExpandThreads) {
        const int g = it / K;
        const int k = it - g * K;
        int l = static_cast<int>(sqrtf(static_cast<float>(k)));
        l += (l + 1) * (l + 1) <= k ? 1 : 0;
        l -= l * l > k ? 1 : 0;
        T a[kExpandAcc];
#pragma unroll
        for (int u = 0; u < kExpandAcc; ++u) a[u] = j0 == b ? T(0) : sC[(g * kExpandAcc + u) * K + k];
        using V = typename Vec16<T>::type;
        constexpr int W = Vec16<T>::n;
        const T* yc = sY + k;
        const T* rc = sR + l * NP + g * kExpandAcc;  // 16-byte aligned
#pragma unroll 4
        for (int j = 0; j < cnt; ++j) {
          const T y = yc[j * SY];
          const V* r = reinterpret_cast<const V*>(rc + j * RS);
#pragma unroll
          for (int h = 0; h < kExpandAcc / W; ++h) {
            const V rv = r[h];
#pragma unroll
            for (int u = 0; u < W; ++u) a[h * W + u] += rv[u] * y;
          }
        }
        if (j0 + JC >= t) {
#pragma unroll
          for (int u = 0; u < kExpandAcc; ++u)
            if (g * kExpandAcc + u < NM) ce[(g * kExpandAcc + u) * K + k] = a[u];
        } else {
#pragma unroll
          for (int u = 0; u < kExpandAcc; ++u) sC[(g * kExpandAcc + u) * K + k] = a[u];
        }
      }
      __syncthreads();
    }
    if (t == b) {  // empty environment
      for (int i = tid; i < NM * K; i += kExpandThreads) ce[i] = T(0);
    }
  }
}

}  // namespace sph
