// Radial expansion over CSR environments (Sec. I, Eq. expansion):
//   c[e, n, l^2+l+m] = sum over the points j of environment e of
//                      R[j, l, n] * Y_l^m(x_j)
// with the radial values R[j, l, n] supplied by the caller, and its
// backward.  The harmonics never leave the chip.  Forward: a block takes one
// environment at a time, writes the values of a chunk of its points into an
// LDS tile, copies the chunk's radial values next to it, and contracts the
// two tiles into per-thread accumulators; partial sums of environments
// longer than one chunk wait in LDS.  Backward: one thread per point, see
// k_expand_bwd.
#pragma once

#include "sph_device.hpp"
#include "sph_fwd.inl"  // emit_values
#include "sph_launch.hpp"

namespace sph {

constexpr int kExpandThreads = 128;  // two waves
// radial values in flight per thread (one batch covers a 64-point chunk of
// l_max = 8 with 8 channels in float, a 32-point one in double)
template <typename T>
inline constexpr int kExpandRBatch = std::is_same_v<T, float> ? 40 : 24;

// Environment e's point range, clamped into [0, n] so that inconsistent
// offsets (reported through the status word) never index out of bounds.
__device__ __forceinline__ void env_range(const int64_t* o, int64_t e, int64_t n, int64_t& b, int64_t& t) {
  int64_t lo = o[e], hi = o[e + 1];
  lo = lo < 0 ? 0 : (lo > n ? n : lo);
  hi = hi < lo ? lo : (hi > n ? n : hi);
  b = lo;
  t = hi;
}

// Values of degrees [la, lb) of one point into its LDS row.  LT >= 0: the
// degree loop is unrolled to LT with compile-time degrees (each row's
// coefficients fold to literals), every row behind a uniform range check;
// LT < 0: the run-time-degree rows of the m-extent bucket MM.
template <typename T, int MM, int LT, bool NORM>
__device__ __forceinline__ void expand_rows(const Point<T>& pt, int la, int lb, T* row) {
  if constexpr (LT >= 0) {
    T cur[LT + 3], unused[LT + 3];
#pragma unroll
    for (int l = 0; l <= LT; ++l) {
      if (l < la || l >= lb) continue;
      q_row<T, LT>(l, pt.ez, pt.rxy2, cur);
      emit_row<T, LT, 0, NORM>(l, unused, cur, pt.ex, pt.ey, pt.ez, pt.inv_r, [&](int k, T v) { row[k] = v; });
    }
  } else {
    emit_values<T, MM, NORM, false>(pt, la, lb, row);
  }
}

// ACC: radial channels per accumulator item (4 or 8; see expand_acc).
template <typename T, int MM, int LT, bool NORM, int ACC>
__global__ __launch_bounds__(kExpandThreads) void k_expand(ExpandParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int L = LT >= 0 ? LT : P.L;
  const int K = (L + 1) * (L + 1);
  const int SY = expand_ystride(K);
  const int NM = P.n_max;
  const int NP = expand_np(NM, ACC);
  const int RS = (L + 1) * NP;  // R tile row stride
  const int JC = P.chunk;
  T* sY = reinterpret_cast<T*>(smem);
  T* sR = reinterpret_cast<T*>(smem + ((static_cast<size_t>(JC) * SY * sizeof(T) + 15) & ~size_t(15)));
  T* sC = sR + static_cast<size_t>(JC) * RS;
  const T* xyz = static_cast<const T*>(P.xyz);
  const T* R = static_cast<const T*>(P.R);
  T* c = static_cast<T*>(P.c);
  const int items = K * (NP / ACC);

  // CSR consistency, by the first wave of block 0 (one writer, no atomics)
  if (P.status != nullptr && blockIdx.x == 0 && tid < kWave) {
    bool ok = true;
    for (int64_t i = tid; i < P.n_env; i += kWave) ok = ok && (P.offsets[i] <= P.offsets[i + 1]);
    if (tid == 0) ok = ok && P.offsets[0] == 0 && P.offsets[P.n_env] == P.n;
    const bool all_ok = __all(ok);
    if (tid == 0) P.status[0] = all_ok ? 0 : 4 /* SPH_ERR_OFFSETS */;
  }

  // The block walks its chunks (environment e = blockIdx.x, + gridDim.x,
  // ...; points j0 .. j0 + JC of each) as a pipeline: the coordinates and
  // the first radial batch of chunk i + 1 are loaded into registers while
  // chunk i's harmonics are computed and contracted.  Indices past a chunk
  // load its last element again (in bounds, never stored), which keeps the
  // loads unconditional.  Empty environments get their zeros as the walk
  // passes them.
  constexpr int RB = kExpandRBatch<T>;
  int64_t e = blockIdx.x, b = 0, t = 0, j0 = 0;
  // moves (e, b, t, j0) to the next chunk at or after environment e (j0 =
  // start of e when fresh); false when the block has no chunk left
  auto seek = [&](bool fresh) {
    if (!fresh) {
      j0 += JC;
      if (j0 < t) return true;
      e += gridDim.x;
    }
    for (; e < P.n_env; e += gridDim.x) {
      env_range(P.offsets, e, P.n, b, t);
      j0 = b;
      if (t > b) return true;
      T* ce = c + e * NM * K;
      for (int i = tid; i < NM * K; i += kExpandThreads) ce[i] = T(0);
    }
    return false;
  };
  T px = T(0), py = T(0), pz = T(0);
  T rb[RB];
  auto issue = [&]() {  // coordinates and first radial batch of chunk (e, j0)
    const int cnt = static_cast<int>(t - j0 < JC ? t - j0 : JC);
    const int64_t jp = j0 + (tid % JC < cnt ? tid % JC : cnt - 1);
    px = xyz[jp * 3 + 0];
    py = xyz[jp * 3 + 1];
    pz = xyz[jp * 3 + 2];
    const int nrv = cnt * (L + 1) * NM;
    const T* Rg = R + j0 * (L + 1) * NM;
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int i = tid + u * kExpandThreads;
      rb[u] = Rg[i < nrv ? i : nrv - 1];
    }
  };
  auto rstore = [&](int base, int nrv) {
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int i = base + tid + u * kExpandThreads;
      if (i < nrv) {
        const int row = NP == NM ? 0 : i / NM;
        sR[NP == NM ? i : row * NP + (i - row * NM)] = rb[u];
      }
    }
  };

  bool more = seek(true);
  if (more) issue();
  while (more) {
    const int cnt = static_cast<int>(t - j0 < JC ? t - j0 : JC);
    const int nrv = cnt * (L + 1) * NM;
    const int64_t cb = b, ct = t, c0 = j0;
    T* ce = c + e * NM * K;
    // this chunk's loads: one wait for all of them
    __builtin_amdgcn_s_waitcnt(kWaitVmem0);
    rstore(0, nrv);
    const T x = px, y = py, z = pz;
    // radial values past the first batch (chunks of more than RB * 128)
    for (int base = RB * kExpandThreads; base < nrv; base += RB * kExpandThreads) {
      const T* Rg = R + c0 * (L + 1) * NM;
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int i = base + tid + u * kExpandThreads;
        rb[u] = Rg[i < nrv ? i : nrv - 1];
      }
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);
      rstore(base, nrv);
    }
    if (NP != NM) {
      const int nr = cnt * (L + 1);
      const int pad = NP - NM;
      for (int i = tid; i < nr * pad; i += kExpandThreads) {
        const int row = i / pad;
        sR[row * NP + NM + (i - row * pad)] = T(0);
      }
    }
    // the next chunk's loads fly during this chunk's arithmetic
    more = seek(false);
    if (more) issue();
    // The chunk's harmonics: point tid % JC, degrees [la, lb) of part
    // tid / JC.  A chunk narrower than the block splits each point's degrees
    // into 128 / JC parts of equal row counts (each row starts its own
    // recursion, so any part can start at any degree), keeping every thread
    // busy.
    if (tid % JC < cnt) {
      const int parts = kExpandThreads / JC;
      const int part = tid / JC;
      const int per = (L + 1 + parts - 1) / parts;
      const int la = part * per;
      const int lb = la + per < L + 1 ? la + per : L + 1;
      if (la < lb) {
        const Point<T> pt = make_point<T, NORM>(x, y, z);
        expand_rows<T, MM, LT, NORM>(pt, la, lb, sY + (tid % JC) * SY);
      }
    }
    __syncthreads();
    const bool last = c0 + JC >= ct;
    bool done = false;
    if constexpr (LT >= 0 && LT <= 4) {
      // Fewer items than threads (small l_max): the chunk's points are split
      // into S parts, each summed by its own thread; parts 1..S-1 leave their
      // sums in the (then free) radial tile and part 0 adds them in order.
      const int S = items > kExpandThreads / 2 ? 1
                    : (items > kExpandThreads / 4 ? 2 : 4);
      const bool split = S > 1 && JC * RS >= (S - 1) * items * ACC;
      const int nparts = split ? S : 1;
      const int jper = (cnt + nparts - 1) / nparts;
      using V = typename Vec16<T>::type;
      constexpr int W = Vec16<T>::n;
      auto item_sum = [&](int k, int g, int l, int ja, int jb, T (&a)[ACC]) {
        const T* yc = sY + k;
        const T* rc = sR + l * NP + g * ACC;  // 16-byte aligned (NP, ACC multiples of 4)
#pragma unroll 4
        for (int j = ja; j < jb; ++j) {
          const T yv = yc[j * SY];
          const V* r = reinterpret_cast<const V*>(rc + j * RS);
#pragma unroll
          for (int h = 0; h < ACC / W; ++h) {
            const V rv = r[h];
#pragma unroll
            for (int u = 0; u < W; ++u) a[h * W + u] += rv[u] * yv;
          }
        }
      };
      auto degree_of = [](int k) {
        int l = static_cast<int>(sqrtf(static_cast<float>(k)));
        l += (l + 1) * (l + 1) <= k ? 1 : 0;
        l -= l * l > k ? 1 : 0;
        return l;
      };
      auto finish_item = [&](int k, int g, T (&a)[ACC]) {
        if (last) {
#pragma unroll
          for (int u = 0; u < ACC; ++u)
            if (g * ACC + u < NM) ce[(g * ACC + u) * K + k] = a[u];
        } else {
#pragma unroll
          for (int u = 0; u < ACC; ++u) sC[(g * ACC + u) * K + k] = a[u];
        }
      };
      if (split) {
          const int it = tid % items;
          const int part = tid / items;
          const int g = it / K;
          const int k = it - g * K;
          T a[ACC];
#pragma unroll
          for (int u = 0; u < ACC; ++u) a[u] = T(0);
          if (part < S) {
            const int ja = part * jper;
            const int jb = ja + jper < cnt ? ja + jper : cnt;
            item_sum(k, g, degree_of(k), ja, jb, a);
          }
          __syncthreads();  // every read of the radial tile is done
          T* sP = sR;
          if (part >= 1 && part < S) {
#pragma unroll
            for (int u = 0; u < ACC; ++u) sP[((part - 1) * items + it) * ACC + u] = a[u];
          }
          __syncthreads();
          if (part == 0) {
            for (int q = 1; q < S; ++q) {
#pragma unroll
              for (int u = 0; u < ACC; ++u) a[u] += sP[((q - 1) * items + it) * ACC + u];
            }
            if (c0 != cb) {
#pragma unroll
              for (int u = 0; u < ACC; ++u) a[u] += sC[(g * ACC + u) * K + k];
            }
            finish_item(k, g, a);
          }
        done = true;
      }
    }
    if (!done) {
      for (int it = tid; it < items; it += kExpandThreads) {
        const int g = it / K;
        const int k = it - g * K;
        int l = static_cast<int>(sqrtf(static_cast<float>(k)));
        l += (l + 1) * (l + 1) <= k ? 1 : 0;
        l -= l * l > k ? 1 : 0;
        T a[ACC];
#pragma unroll
        for (int u = 0; u < ACC; ++u) a[u] = c0 == cb ? T(0) : sC[(g * ACC + u) * K + k];
        using V = typename Vec16<T>::type;
        constexpr int W = Vec16<T>::n;
        const T* yc = sY + k;
        const T* rc = sR + l * NP + g * ACC;  // 16-byte aligned (NP, ACC multiples of 4)
#pragma unroll 4
        for (int j = 0; j < cnt; ++j) {
          const T yv = yc[j * SY];
          const V* r = reinterpret_cast<const V*>(rc + j * RS);
#pragma unroll
          for (int h = 0; h < ACC / W; ++h) {
            const V rv = r[h];
#pragma unroll
            for (int u = 0; u < W; ++u) a[h * W + u] += rv[u] * yv;
          }
        }
        if (last) {
#pragma unroll
          for (int u = 0; u < ACC; ++u)
            if (g * ACC + u < NM) ce[(g * ACC + u) * K + k] = a[u];
        } else {
#pragma unroll
          for (int u = 0; u < ACC; ++u) sC[(g * ACC + u) * K + k] = a[u];
        }
      }
    }
    __syncthreads();
  }
}

// Backward of the expansion for an upstream gradient G = dL/dc (chain rule):
//   grad_R[j, l, n] = sum_m G[e, n, l^2+l+m] Y_l^m(x_j)
//   grad_xyz[j, a]  = sum_k gY[j, k] dY_k/dx_a(x_j),
//                     gY[j, k] = sum_n G[e, n, k] R[j, l(k), n]
// One thread per point, the environment's G in LDS ([k][channel], read as
// 16-byte vectors, the same address for every thread).  Degree by degree the
// thread forms the value row (grad_R and gY of the row, gY kept in its LDS
// row) and then the three derivative rows (Eq. iter-deri), so neither Y nor
// dY is stored.  NPC: channels padded to a multiple of 4 held in registers.
template <typename T, int MM, int LT, bool NORM, int NPC>
__global__ __launch_bounds__(kExpandThreads) void k_expand_bwd(ExpandBwdParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int M = LT >= 0 ? LT : MM;
  constexpr bool CT = LT >= 0;
  using V = typename Vec16<T>::type;
  constexpr int W = Vec16<T>::n;
  const int tid = threadIdx.x;
  const int L = LT >= 0 ? LT : P.L;
  const int K = (L + 1) * (L + 1);
  const int NM = P.n_max;
  const int TS = (2 * L + 1) | 1;
  T* sG = reinterpret_cast<T*>(smem);
  T* sT = sG + static_cast<size_t>(K) * NPC + tid * TS;  // this thread's row
  const T* xyz = static_cast<const T*>(P.xyz);
  const T* R = static_cast<const T*>(P.R);
  const T* gc = static_cast<const T*>(P.gc);
  T* gxyz = static_cast<T*>(P.gxyz);
  T* gR = static_cast<T*>(P.gR);

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
    if (t == b) continue;
    __syncthreads();  // the previous environment's G is no longer read
    const T* ge = gc + e * NM * K;
    for (int i = tid; i < NPC * K; i += kExpandThreads) {
      const int n = i / K;
      const int k = i - n * K;
      sG[k * NPC + n] = n < NM ? ge[i] : T(0);
    }
    __syncthreads();
    for (int64_t j = b + tid; j < t; j += kExpandThreads) {
      const Point<T> pt = make_point<T, NORM>(xyz[j * 3], xyz[j * 3 + 1], xyz[j * 3 + 2]);
      T prev[M + 3], cur[M + 3];
#pragma unroll
      for (int m = 0; m < M + 3; ++m) prev[m] = T(0);
      T g0 = T(0), g1 = T(0), g2 = T(0);
      const T* Rj = R + j * (L + 1) * NM;
      auto row = [&](int l) {
        q_row_any<T, M, CT>(l, pt.ez, pt.rxy2, cur);
        T r[NPC], acc[NPC];
#pragma unroll
        for (int n = 0; n < NPC; ++n) {
          r[n] = n < NM ? Rj[l * NM + n] : T(0);
          acc[n] = T(0);
        }
        const int kb = l * l;
        emit_row<T, M, 0, NORM>(l, prev, cur, pt.ex, pt.ey, pt.ez, pt.inv_r, [&](int k, T v) {
          const V* gv = reinterpret_cast<const V*>(sG + k * NPC);
          T gy = T(0);
#pragma unroll
          for (int h = 0; h < NPC / W; ++h) {
            const V g = gv[h];
#pragma unroll
            for (int u = 0; u < W; ++u) {
              gy += g[u] * r[h * W + u];
              acc[h * W + u] += g[u] * v;
            }
          }
          sT[k - kb] = gy;
        });
        if (gR != nullptr) {
          T* out = gR + (j * (L + 1) + l) * NM;
#pragma unroll
          for (int n = 0; n < NPC; ++n)
            if (n < NM) out[n] = acc[n];
        }
        emit_row<T, M, 1, NORM>(l, prev, cur, pt.ex, pt.ey, pt.ez, pt.inv_r,
                                [&](int k, T d) { g0 += sT[k - kb] * d; });
        emit_row<T, M, 2, NORM>(l, prev, cur, pt.ex, pt.ey, pt.ez, pt.inv_r,
                                [&](int k, T d) { g1 += sT[k - kb] * d; });
        emit_row<T, M, 3, NORM>(l, prev, cur, pt.ex, pt.ey, pt.ez, pt.inv_r,
                                [&](int k, T d) { g2 += sT[k - kb] * d; });
#pragma unroll
        for (int m = 0; m < M + 3; ++m) prev[m] = cur[m];  // row l - 1 of the next degree
      };
      if constexpr (CT) {
#pragma unroll
        for (int l = 0; l <= LT; ++l) row(l);
      } else {
        for (int l = 0; l <= L; ++l) row(l);
      }
      if (gxyz != nullptr) {
        gxyz[j * 3 + 0] = g0;
        gxyz[j * 3 + 1] = g1;
        gxyz[j * 3 + 2] = g2;
      }
    }
  }
}

}  // namespace sph
