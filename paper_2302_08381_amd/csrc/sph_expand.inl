// Radial expansion over CSR environments (Sec. I, Eq. expansion):
//   c[e, n, l^2+l+m] = sum over the points j of environment e of
//                      R[j, l, n] * Y_l^m(x_j)
// with the radial values R[j, l, n] supplied by the caller, and its
// backward.  The harmonics never leave the chip.  Forward: a block takes one
// environment at a time, writes the values of a chunk of its points into an
// LDS tile, copies the chunk's radial values next to it, and contracts the
// two tiles into per-thread accumulators; partial sums of environments
// longer than one chunk wait in LDS.  Backward: one lane per point, see
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

// First e in [0, n_env] with o[e] >= p, found by the W lanes base .. base+W-1
// of the wave together: each round probes W evenly spaced offsets at once and
// keeps the gap where the comparison turns, so log_W(n_env) rounds of one
// dependent load replace log_2(n_env).  Every lane of the wave must call it
// (it votes across the wave); each group gets its own answer.  With offsets
// that are not sorted the result is still in [0, n_env].
__device__ __forceinline__ int64_t group_lower_bound(const int64_t* o, int64_t n_env, int64_t p, int gl, int base,
                                                     int W) {
  int rounds = 1;  // the same for every lane: W^rounds > n_env
  for (int64_t span = W; span <= n_env; span *= W) ++rounds;
  const unsigned long long gmask = W == 64 ? ~0ull : ((1ull << W) - 1) << base;
  int64_t lo = 0, hi = n_env;
  for (int r = 0; r < rounds; ++r) {
    const int64_t step = (hi - lo + W - 1) / W;
    const int64_t q = lo + gl * step;
    const bool less = step > 0 && q < hi && o[q] < p;
    const int c = __popcll(__ballot(less) & gmask);
    if (step > 0) {  // the answer is in (q_{c-1}, q_c]
      const int64_t qc = lo + c * step;
      const int64_t nhi = qc < hi ? qc : hi;
      const int64_t nlo = c > 0 ? lo + (c - 1) * step + 1 : lo;
      lo = nlo < nhi ? nlo : nhi;
      hi = nhi;
    }
  }
  return lo;
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

  // The blocks split the points evenly: block g of G takes the environments
  // that start in points [g n / G, (g+1) n / G) (found by searching the
  // offsets; every environment has one start, so each goes to exactly one
  // block; see kEven for small l_max).  The block walks its chunks (up to
  // JC consecutive points, within one environment or across the end of one
  // into the next, see shape) as a pipeline: the coordinates and the first
  // radial batch
  // of chunk i + 1 are loaded into registers while chunk i's harmonics are
  // computed and contracted.  Indices past a chunk load its last element
  // again (in bounds, never stored), which keeps the loads unconditional.
  // Empty environments get their zeros as the walk passes them.
  constexpr int RB = kExpandRBatch<T>;
  // Small l_max (the kernels whose items are split across threads) keeps
  // the interleaved walk, environments blockIdx.x + i gridDim.x: there the
  // even split measured 12 % slower (l_max 3: 98-103 against 85-91 us),
  // while it is 8-11 % faster at l_max 8 and 12.
  constexpr bool kEven = !(LT >= 0 && LT <= 4);
  const int64_t G = gridDim.x, g = blockIdx.x;
  int64_t e = g, e_end = P.n_env, b = 0, t = 0, j0 = 0;
  const int64_t estep = kEven ? 1 : G;
  if constexpr (kEven) {
    // each wave finds both ends at once: lanes 0..31 the start, 32..63 the end
    const int wl = tid % kWave, half = wl / 32;
    const int64_t bound = group_lower_bound(P.offsets, P.n_env, (g + half) * P.n / G, wl % 32, half * 32, 32);
    e = __shfl(bound, 0);
    e_end = g + 1 == G ? P.n_env : __shfl(bound, 32);
  }
  // the first non-empty environment at or after e (j0 = its start); false
  // when the block has none left
  auto scan = [&]() {
    for (; e < e_end; e += estep) {
      env_range(P.offsets, e, P.n, b, t);
      j0 = b;
      if (t > b) return true;
      T* ce = c + e * NM * K;
      for (int i = tid; i < NM * K; i += kExpandThreads) ce[i] = T(0);
    }
    return false;
  };
  // The chunk at (e, j0): cnt points from j0.  With the even split, a chunk
  // that reaches the end of e runs on into environment e + 1 when that one
  // starts there and is not empty (span; e's points are the first cut,
  // e + 1 ends at t2): chunks that stopped at every environment's end were
  // two thirds full on environments of 8..128 points at 64-point chunks.
  auto shape = [&](int& cnt, int& cut, bool& span, int64_t& t2) {
    cnt = static_cast<int>(t - j0 < JC ? t - j0 : JC);
    cut = cnt;
    span = false;
    if constexpr (kEven) {
      if (cnt < JC && e + 1 < e_end) {
        int64_t b2 = 0, tn = 0;
        env_range(P.offsets, e + 1, P.n, b2, tn);
        if (b2 == t && tn > b2) {
          span = true;
          t2 = tn;
          cnt = static_cast<int>(tn - j0 < JC ? tn - j0 : JC);
        }
      }
    }
  };
  // moves the walk past the chunk it has just done; false when the block
  // has no chunk left
  auto advance = [&](int cnt, bool span, int64_t t2) {
    if (span) {  // now inside e + 1 (the even split walks with estep = 1)
      ++e;
      b = t;
      t = t2;
      j0 += cnt;
    } else {
      j0 += JC;
    }
    if (j0 < t) return true;
    e += estep;
    return scan();
  };
  T px = T(0), py = T(0), pz = T(0);
  // The radial batch: RB values per thread, as RB / W 16-byte vectors when
  // the channels fill whole vectors and R is 16-byte aligned (no vector
  // crosses a row; without padding the tile is a copy of the global block,
  // with it each vector goes to its row's padded slot), else element by
  // element into the padded rows.
  using RV = typename Vec16<T>::type;
  constexpr int RW = Vec16<T>::n;
  static_assert(RB % RW == 0, "whole radial vectors");
  constexpr int RBV = RB / RW;
  const bool rvec = NM % RW == 0 && aligned16(R);
  RV rb[RBV];
  auto rload = [&](const T* Rg, int base, int nrv) {  // values base .. base + RB * 128 of the chunk
    if (rvec) {
      const RV* g = reinterpret_cast<const RV*>(Rg);
      const int nv = nrv / RW;
#pragma unroll
      for (int u = 0; u < RBV; ++u) {
        const int i = base / RW + tid + u * kExpandThreads;
        rb[u] = g[i < nv ? i : nv - 1];
      }
    } else {
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int i = base + tid + u * kExpandThreads;
        rb[u / RW][u % RW] = Rg[i < nrv ? i : nrv - 1];
      }
    }
  };
  auto issue = [&]() {  // coordinates and first radial batch of chunk (e, j0)
    int cnt = 0, cut = 0;
    bool span = false;
    int64_t t2 = 0;
    shape(cnt, cut, span, t2);
    const int64_t jp = j0 + (tid % JC < cnt ? tid % JC : cnt - 1);
    px = xyz[jp * 3 + 0];
    py = xyz[jp * 3 + 1];
    pz = xyz[jp * 3 + 2];
    rload(R + j0 * (L + 1) * NM, 0, cnt * (L + 1) * NM);
  };
  auto rstore = [&](int base, int nrv) {
    if (rvec) {
      RV* sv = reinterpret_cast<RV*>(sR);
      const int nv = nrv / RW;
      if (NP == NM) {
#pragma unroll
        for (int u = 0; u < RBV; ++u) {
          const int i = base / RW + tid + u * kExpandThreads;
          if (i < nv) sv[i] = rb[u];
        }
      } else {
        // vector i = row * mv + cv goes to row * pv + cv, running counters
        const int mv = NM / RW, pv = NP / RW;
        int i = base / RW + tid;
        int row = i / mv, cv = i - row * mv;
        const int qs = kExpandThreads / mv, rq = kExpandThreads - qs * mv;
#pragma unroll
        for (int u = 0; u < RBV; ++u) {
          if (i < nv) sv[row * pv + cv] = rb[u];
          i += kExpandThreads;
          row += qs;
          cv += rq;
          if (cv >= mv) {
            cv -= mv;
            ++row;
          }
        }
      }
    } else {
      // element i = row * NM + ch goes to row * NP + ch; one division per
      // batch, then running counters (the thread's elements are
      // kExpandThreads apart)
      int i = base + tid;
      int row = i / NM, ch = i - row * NM;
      const int qs = kExpandThreads / NM, rq = kExpandThreads - qs * NM;
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        if (i < nrv) sR[NP == NM ? i : row * NP + ch] = rb[u / RW][u % RW];
        i += kExpandThreads;
        row += qs;
        ch += rq;
        if (ch >= NM) {
          ch -= NM;
          ++row;
        }
      }
    }
  };

  bool more = scan();
  if (more) issue();
  while (more) {
    int cnt = 0, cut = 0;
    bool span = false;
    int64_t ct2 = 0;
    shape(cnt, cut, span, ct2);
    const int nrv = cnt * (L + 1) * NM;
    const int64_t cb = b, ct = t, c0 = j0;
    T* ce = c + e * NM * K;
    T* ce2 = span ? ce + NM * K : nullptr;  // environment e + 1
    // this chunk's loads: one wait for all of them
    __builtin_amdgcn_s_waitcnt(kWaitVmem0);
    rstore(0, nrv);
    const T x = px, y = py, z = pz;
    // radial values past the first batch (chunks of more than RB * 128)
    for (int base = RB * kExpandThreads; base < nrv; base += RB * kExpandThreads) {
      rload(R + c0 * (L + 1) * NM, base, nrv);
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
    more = advance(cnt, span, ct2);
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
        auto sum = [&](int ja, int jb) {
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
        auto to_c = [&](T* cc) {
#pragma unroll
          for (int u = 0; u < ACC; ++u)
            if (g * ACC + u < NM) cc[(g * ACC + u) * K + k] = a[u];
        };
        auto to_partial = [&]() {
#pragma unroll
          for (int u = 0; u < ACC; ++u) sC[(g * ACC + u) * K + k] = a[u];
        };
        sum(0, cut);
        if (!span) {
          if (last)
            to_c(ce);
          else
            to_partial();
        } else {
          // e ends in this chunk; e + 1 starts at point cut
          to_c(ce);
#pragma unroll
          for (int u = 0; u < ACC; ++u) a[u] = T(0);
          sum(cut, cnt);
          if (c0 + cnt >= ct2)
            to_c(ce2);
          else
            to_partial();
        }
      }
    }
    __syncthreads();
  }
}

// One point of the expansion backward: grad_R of every degree and grad_xyz.
// The point's radial values come from one of three sources:
//   SRC = 0: its row in an LDS tile, [degree][NPC channels] (zero padded);
//            grad_R goes back into the same slots, degree by degree, after
//            they are read;
//   SRC = 1: global memory as 16-byte vectors (channels = NPC, 16-byte
//            aligned), in one of two register buffers, the next degree's
//            loads issued before this degree's arithmetic.  Plain loads: a
//            lane reads its 16-byte pieces of a row over several degrees,
//            and with the nontemporal hint the lines left L2 between them
//            and were fetched again (20-30 % slower);
//   SRC = 2: global memory element by element (loading a degree ahead, as
//            for SRC = 1, was 1-4 % slower: the second buffer costs
//            occupancy);
//   SRC = 3: as SRC = 1 where the channels need padding but still fill
//            whole 16-byte vectors (NM a multiple of 4 floats or 2
//            doubles, so every degree's row stays 16-byte aligned): the
//            vectors past NM are zeros, never loaded or stored.
template <typename T, int MM, bool NORM, int NPC, int SRC>
__device__ __forceinline__ void expand_bwd_point(const T* __restrict__ xyz, const T* __restrict__ R,
                                                 const T* __restrict__ sG, T* __restrict__ sRow,
                                                 T* __restrict__ gxyz, T* __restrict__ gR, int64_t j, int L,
                                                 int NM) {
  using V = typename Vec16<T>::type;
  constexpr int W = Vec16<T>::n;
  constexpr int NV = NPC / W;
  constexpr T kIS2 = T(kInvSqrt2d);
  const CoefTable<T>& C = coef<T>();
  const Point<T> pt = make_point<T, NORM>(xyz[j * 3], xyz[j * 3 + 1], xyz[j * 3 + 2]);
  const T ex = pt.ex, ey = pt.ey, ez = pt.ez;
  // order-m factors: c_m, s_m, m c_{m-1}, m s_{m-1} (buckets up to m = 12)
  constexpr bool kTab = MM <= 12;
  constexpr int MT = kTab ? MM + 1 : 1;
  T tc[MT], ts[MT], tmc[MT], tms[MT];
  if constexpr (kTab) {
    T s1 = T(0), c1 = T(1), s0 = T(0), c0 = T(1);
#pragma unroll
    for (int m = 0; m <= MM; ++m) {
      if (m > 0) {
        const T sn = ex * s0 + ey * c0;
        const T cn = ex * c0 - ey * s0;
        s1 = s0;
        c1 = c0;
        s0 = sn;
        c0 = cn;
      }
      tc[m] = c0;
      ts[m] = s0;
      tmc[m] = T(m) * c1;
      tms[m] = T(m) * s1;
    }
  }
  T prev[MM + 3], cur[MM + 3];
#pragma unroll
  for (int m = 0; m < MM + 3; ++m) prev[m] = T(0);
  T g0 = T(0), g1 = T(0), g2 = T(0);
  const T* Rj = R + j * (L + 1) * NM;
  T* gRj = gR != nullptr ? gR + j * (L + 1) * NM : nullptr;
  V ra[NV], rb[NV];
  auto load_r = [&](int l, V (&dst)[NV]) {
    if constexpr (SRC == 1) {
#pragma unroll
      for (int h = 0; h < NV; ++h) dst[h] = reinterpret_cast<const V*>(Rj + l * NPC)[h];
    } else {
      const V* g = reinterpret_cast<const V*>(Rj + l * NM);
#pragma unroll
      for (int h = 0; h < NV; ++h) {
        V v;
#pragma unroll
        for (int u = 0; u < W; ++u) v[u] = T(0);
        dst[h] = h * W < NM ? g[h] : v;
      }
    }
  };
  // degree l; SRC = 1: radial values in rc, the next degree's loads issued
  // into rx first (unconditionally: the last degree loads itself again, so
  // the wait analysis sees one path)
  auto degree = [&](int l, const V (&rc)[NV], V (&rx)[NV]) {
    if constexpr (SRC == 1 || SRC == 3) load_r(l < L ? l + 1 : l, rx);
    // the degree's derivative coefficients, fetched together before any
    // column: scalar loads share their wait counter with LDS reads, so a
    // fetch next to each column would drain every G read in flight
    T kg[MM + 1], kz[MM + 1];
#pragma unroll
    for (int m = 0; m <= MM; ++m) {
      kg[m] = C.gxy[l][m];
      kz[m] = C.gz[l][m];
    }
    q_row_rt<T, MM>(l, ez, pt.rxy2, cur);
    T r[NPC], acc[NPC];
    if constexpr (SRC == 0) {
      const V* sv = reinterpret_cast<const V*>(sRow + l * NPC);
#pragma unroll
      for (int h = 0; h < NV; ++h) {
        const V v = sv[h];
#pragma unroll
        for (int u = 0; u < W; ++u) r[h * W + u] = v[u];
      }
    }
#pragma unroll
    for (int n = 0; n < NPC; ++n) {
      if constexpr (SRC == 1 || SRC == 3) r[n] = rc[n / W][n % W];
      if constexpr (SRC == 2) r[n] = n < NM ? Rj[l * NM + n] : T(0);
      acc[n] = T(0);
    }
    const int k0 = l * l + l;
    // sums over the row of gY times the scaled derivatives and the value;
    // normalised, d Y = (d Yt - l u Yt) / r, so the row adds
    // (S_d - l u S_Y) / r once instead of normalising every column
    T sx = T(0), sy = T(0), sz = T(0), sY = T(0);
    // one column: value Yt and scaled derivatives (dx, dy, dz)
    auto col = [&](int k, T Yt, T dx, T dy, T dz) {
      const V* gv = reinterpret_cast<const V*>(sG + k * NPC);
      T gy = T(0);
#pragma unroll
      for (int h = 0; h < NV; ++h) {
        const V g = gv[h];
#pragma unroll
        for (int u = 0; u < W; ++u) {
          gy += g[u] * r[h * W + u];
          acc[h * W + u] += g[u] * Yt;
        }
      }
      sx += gy * dx;
      sy += gy * dy;
      sz += gy * dz;
      if constexpr (NORM) sY += gy * Yt;
    };
    T s1 = T(0), c1 = T(1);  // s_{m-1}, c_{m-1}
    T s0 = T(0), c0 = T(1);  // s_m, c_m
#pragma unroll
    for (int m = 0; m <= MM; ++m) {
      if (m > l) continue;  // no early exit: keeps the loop fully unrolled
      T c, sm, mc, ms;
      if constexpr (kTab) {
        const int mt = kTab ? m : 0;
        c = tc[mt];
        sm = ts[mt];
        mc = tmc[mt];
        ms = tms[mt];
      } else {
        if (m > 0) {
          const T sn = ex * s0 + ey * c0;
          const T cn = ex * c0 - ey * s0;
          s1 = s0;
          c1 = c0;
          s0 = sn;
          c0 = cn;
        }
        c = c0;
        sm = s0;
        mc = T(m) * c1;
        ms = T(m) * s1;
      }
      const T q = cur[m];
      const T Tm = (m <= l - 2) ? kg[m] * prev[m + 1] : T(0);
      const T Cz = (m <= l - 1) ? kz[m] * prev[m] : T(0);
      const T xt = ex * Tm, yt = ey * Tm;
      if (m == 0) {
        col(k0, q * kIS2, xt * kIS2, yt * kIS2, Cz * kIS2);
      } else {
        col(k0 + m, q * c, xt * c + q * mc, yt * c - q * ms, Cz * c);
        col(k0 - m, q * sm, xt * sm + q * ms, yt * sm + q * mc, Cz * sm);
      }
    }
    if constexpr (NORM) {
      const T lY = T(l) * sY;
      g0 += (sx - lY * ex) * pt.inv_r;
      g1 += (sy - lY * ey) * pt.inv_r;
      g2 += (sz - lY * ez) * pt.inv_r;
    } else {
      g0 += sx;
      g1 += sy;
      g2 += sz;
    }
    if (gRj != nullptr) {
      if constexpr (SRC == 0) {
        V* sv = reinterpret_cast<V*>(sRow + l * NPC);
#pragma unroll
        for (int h = 0; h < NV; ++h) {
          V v;
#pragma unroll
          for (int u = 0; u < W; ++u) v[u] = acc[h * W + u];
          sv[h] = v;
        }
      } else if constexpr (SRC == 1) {
#pragma unroll
        for (int h = 0; h < NV; ++h) {
          V v;
#pragma unroll
          for (int u = 0; u < W; ++u) v[u] = acc[h * W + u];
          reinterpret_cast<V*>(gRj + l * NPC)[h] = v;
        }
      } else if constexpr (SRC == 3) {
#pragma unroll
        for (int h = 0; h < NV; ++h) {
          if (h * W < NM) {
            V v;
#pragma unroll
            for (int u = 0; u < W; ++u) v[u] = acc[h * W + u];
            reinterpret_cast<V*>(gRj + l * NM)[h] = v;
          }
        }
      } else {
#pragma unroll
        for (int n = 0; n < NPC; ++n)
          if (n < NM) gRj[l * NM + n] = acc[n];
      }
    }
    copy_row<T, MM>(MM, cur, prev);
  };
  if constexpr (SRC == 1 || SRC == 3) load_r(0, ra);
  // two degrees per trip, the radial buffers alternating
#pragma unroll 1
  for (int l = 0; l <= L; l += 2) {
    degree(l, ra, rb);
    if (l + 1 <= L) degree(l + 1, rb, ra);
  }
  if (gxyz != nullptr) {
    gxyz[j * 3 + 0] = g0;
    gxyz[j * 3 + 1] = g1;
    gxyz[j * 3 + 2] = g2;
  }
}

// Copies of one group's radial tile between global rows [cnt][L+1][NM]
// (contiguous from src) and LDS rows of stride RS, [L+1][NPC] each (NPC >= NM,
// the padding channels zero).  MODE 2 (NM == NPC, 16-byte aligned global
// rows): the block as contiguous 16-byte vectors, a batch of them in flight
// per lane.  MODE 1 (NM a whole number of vectors, aligned) and 0 (else):
// each lane keeps one slot of U channels (a vector, or one element) and
// walks the tile's rows, a batch in flight.  GS lanes of the group take
// part (lane gl).
template <typename T, int NPC, int GS, int MODE>
__device__ __forceinline__ void expand_tile_in(T* __restrict__ sR, int RS, const T* __restrict__ src, int cnt,
                                               int L, int NM, int gl) {
  if constexpr (MODE == 2) {
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::n;
    constexpr int NB = 6;
    const int RV = (L + 1) * NPC / W;  // vectors per row
    const int nv = cnt * RV;
    const V* g = reinterpret_cast<const V*>(src);
    int p = gl / RV, c = gl - (gl / RV) * RV;
    const int qs = GS / RV, rq = GS - qs * RV;
    for (int i0 = gl; i0 < nv; i0 += GS * NB) {
      V v[NB];
      int o[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        o[u] = p * RS + c * W;
        if (i0 + u * GS < nv) v[u] = __builtin_nontemporal_load(g + i0 + u * GS);
        p += qs;
        c += rq;
        if (c >= RV) {
          c -= RV;
          ++p;
        }
      }
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (i0 + u * GS < nv) *reinterpret_cast<V*>(sR + o[u]) = v[u];
    }
  } else {
    // lane gl keeps the slot of channels n .. n + U - 1 (n = (gl % SL) U)
    // and walks the rows r = p (L+1) + l of the tile, GS / SL rows per step,
    // NB loads in flight; the slots past NM get zeros
    constexpr int U = MODE == 1 ? Vec16<T>::n : 1;
    using E = std::conditional_t<U == 1, T, typename Vec16<T>::type>;
    constexpr int SL = NPC / U;
    static_assert(GS % SL == 0, "whole rows per step");
    constexpr int RPS = GS / SL;
    constexpr int NB = 8;
    E zero;
    if constexpr (U == 1) {
      zero = T(0);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) zero[u] = T(0);
    }
    const int n = (gl % SL) * U, L1 = L + 1, rows = cnt * L1;
    int p = (gl / SL) / L1, l = gl / SL - p * L1;
    const int qs = RPS / L1, rq = RPS - qs * L1;
    for (int r0 = gl / SL; r0 < rows; r0 += RPS * NB) {
      E v[NB];
      int o[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int r = r0 + u * RPS;
        o[u] = p * RS + l * NPC + n;
        v[u] = r < rows && n < NM ? *reinterpret_cast<const E*>(src + r * NM + n) : zero;
        p += qs;
        l += rq;
        if (l >= L1) {
          l -= L1;
          ++p;
        }
      }
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (r0 + u * RPS < rows) *reinterpret_cast<E*>(sR + o[u]) = v[u];
    }
  }
}

template <typename T, int NPC, int GS, int MODE>
__device__ __forceinline__ void expand_tile_out(const T* __restrict__ sR, int RS, T* __restrict__ dst, int cnt,
                                                int L, int NM, int gl) {
  if constexpr (MODE == 2) {
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::n;
    const int RV = (L + 1) * NPC / W;
    const int nv = cnt * RV;
    V* g = reinterpret_cast<V*>(dst);
    int p = gl / RV, c = gl - (gl / RV) * RV;
    const int qs = GS / RV, rq = GS - qs * RV;
    for (int i = gl; i < nv; i += GS) {
      g[i] = *reinterpret_cast<const V*>(sR + p * RS + c * W);
      p += qs;
      c += rq;
      if (c >= RV) {
        c -= RV;
        ++p;
      }
    }
  } else {
    // the walk of expand_tile_in: a slot of U channels per lane, GS / SL
    // rows a step
    constexpr int U = MODE == 1 ? Vec16<T>::n : 1;
    using E = std::conditional_t<U == 1, T, typename Vec16<T>::type>;
    constexpr int SL = NPC / U;
    constexpr int RPS = GS / SL;
    const int n = (gl % SL) * U, L1 = L + 1, rows = cnt * L1;
    int p = (gl / SL) / L1, l = gl / SL - p * L1;
    const int qs = RPS / L1, rq = RPS - qs * L1;
    if (n < NM) {
      for (int r = gl / SL; r < rows; r += RPS) {
        *reinterpret_cast<E*>(dst + r * NM + n) = *reinterpret_cast<const E*>(sR + p * RS + l * NPC + n);
        p += qs;
        l += rq;
        if (l >= L1) {
          l -= L1;
          ++p;
        }
      }
    }
  }
}

// Backward of the expansion for an upstream gradient G = dL/dc (chain rule):
//   grad_R[j, l, n] = sum_m G[e, n, l^2+l+m] Y_l^m(x_j)
//   grad_xyz[j, a]  = sum_k gY[j, k] dY_k/dx_a(x_j),
//                     gY[j, k] = sum_n G[e, n, k] R[j, l(k), n]
// One lane per point; neither Y nor dY is stored.  A block is one wave split
// into 64 / GS groups of GS lanes, each walking its own run of environments
// (an even share of the points) in chunks of GS consecutive points.  A chunk
// may span the end of one environment and the start of the next: the group
// keeps the G of both in two LDS slices ([k][channel], read as 16-byte
// vectors) and each lane reads the slice of its own point's environment.
// Chunks that stopped at every environment's end would leave a fifth of the
// lanes idle on environments of 8..128 points (a third with 64 lanes); where
// two slices would not fit one block's LDS (P.slices = 1) they do stop.  Per
// point, one pass per degree forms every value and derivative of the row at
// once (Eq. iter-deri with the order-m factors tabulated once per point),
// contracts it with G and the point's radial values of that degree, and
// produces the degree's grad_R.  STAGE: each chunk's radial rows arrive in
// an LDS tile by coalesced 16-byte copies and its grad_R leaves the same
// way; otherwise every lane reads and writes its own rows.  NPC: channels
// padded to a multiple of 4 (8 or 16).
template <typename T, int MM, bool NORM, int NPC, int GS, bool STAGE>
__global__ __launch_bounds__(kWave) void k_expand_bwd(ExpandBwdParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NG = kWave / GS;
  const int lane = threadIdx.x;
  const int grp = lane / GS, gl = lane % GS;
  const int L = P.L;
  const int K = (L + 1) * (L + 1);
  const int NM = P.n_max;
  const int RS = expand_bwd_row_stride<T>(L, NPC);
  const size_t slice = static_cast<size_t>(K) * NPC;
  const int nsl = P.slices;  // 2: chunks may span two environments
  T* sG = reinterpret_cast<T*>(smem) +
          static_cast<size_t>(grp) * (nsl * slice + (STAGE ? static_cast<size_t>(GS) * RS : 0));
  T* sR = sG + nsl * slice;
  const T* xyz = static_cast<const T*>(P.xyz);
  const T* R = static_cast<const T*>(P.R);
  const T* gc = static_cast<const T*>(P.gc);
  T* gxyz = static_cast<T*>(P.gxyz);
  T* gR = static_cast<T*>(P.gR);
  // radial rows as whole 16-byte vectors: every padded channel present and
  // both radial arrays 16-byte aligned (uniform); vpart: the channels fill
  // whole vectors short of the padding
  const bool aligned = aligned16(R) && (gR == nullptr || aligned16(gR));
  const bool vec = NM == NPC && aligned;
  const bool vpart = NM % Vec16<T>::n == 0 && aligned;

  if (P.status != nullptr && blockIdx.x == 0) {
    bool ok = true;
    for (int64_t i = lane; i < P.n_env; i += kWave) ok = ok && (P.offsets[i] <= P.offsets[i + 1]);
    if (lane == 0) ok = ok && P.offsets[0] == 0 && P.offsets[P.n_env] == P.n;
    const bool all_ok = __all(ok);
    if (lane == 0) P.status[0] = all_ok ? 0 : 4 /* SPH_ERR_OFFSETS */;
  }

  // The groups split the points evenly: group g of G takes the environments
  // that start in points [g n / G, (g+1) n / G) (found by searching the
  // offsets; every environment has one start, so each goes to exactly one
  // group), which keeps the two groups of a wave and all waves equally busy.
  // Group state: environment e, its range [b, t), the chunk start j0
  // (b <= j0 < t), and which environment each G slice holds.
  const int64_t G = static_cast<int64_t>(gridDim.x) * NG, g = static_cast<int64_t>(blockIdx.x) * NG + grp;
  int64_t e = group_lower_bound(P.offsets, P.n_env, g * P.n / G, gl, grp * GS, GS);
  const int64_t e_last = group_lower_bound(P.offsets, P.n_env, (g + 1) * P.n / G, gl, grp * GS, GS);
  const int64_t e_end = g + 1 == G ? P.n_env : e_last;
  int64_t b = 0, t = 0, j0 = 0;
  // first non-empty environment at or after ee (e_end if none), its range
  auto next_nonempty = [&](int64_t ee, int64_t& bb, int64_t& tt) {
    for (; ee < e_end; ++ee) {
      env_range(P.offsets, ee, P.n, bb, tt);
      if (tt > bb) break;
    }
    return ee;
  };
  e = next_nonempty(e, b, t);
  j0 = b;
  int se = 0;                         // the slice of environment e
  int64_t in_cur = -1, in_oth = -1;  // environments whose G slices se, 1 - se hold
  // G of one environment into a slice, [n][k] -> [k][n] (padding channels
  // zero): per column k of the lane, all NPC channels are loaded before any
  // is stored, so their latencies overlap (one wait per column, no division)
  auto load_slice = [&](int sl, int64_t env) {
    const T* ge = gc + env * NM * K;
    T* dst = sG + sl * slice;
    for (int k = gl; k < K; k += GS) {
      T v[NPC];
#pragma unroll
      for (int n = 0; n < NPC; ++n) v[n] = n < NM ? ge[n * K + k] : T(0);
      using V = typename Vec16<T>::type;
      constexpr int W = Vec16<T>::n;
      V* d = reinterpret_cast<V*>(dst + k * NPC);
#pragma unroll
      for (int h = 0; h < NPC / W; ++h) {
        V w;
#pragma unroll
        for (int u = 0; u < W; ++u) w[u] = v[h * W + u];
        d[h] = w;
      }
    }
  };
  while (__any(e < e_end)) {
    const bool active = e < e_end;
    // the chunk: GS points from j0, running into the next non-empty
    // environment e2 when e ends first and e2 starts where e ends
    int64_t b2 = 0, t2 = 0, e2 = e_end;
    int cnt = 0;
    if (active) {
      cnt = static_cast<int>(t - j0 < GS ? t - j0 : GS);
      if (cnt < GS && nsl == 2) {
        e2 = next_nonempty(e + 1, b2, t2);
        if (e2 < e_end && b2 == t)
          cnt = static_cast<int>(t2 - j0 < GS ? t2 - j0 : GS);
        else
          e2 = e_end;
      }
    }
    const bool span = e2 < e_end;
    __syncthreads();  // every read of the previous chunk's slices and tile is done
    if (active) {
      if (in_cur != e) {
        load_slice(se, e);
        in_cur = e;
      }
      if (span && in_oth != e2) {
        load_slice(1 - se, e2);
        in_oth = e2;
      }
    }
    if constexpr (STAGE) {
      if (active) {
        const T* src = R + j0 * (L + 1) * NM;
        if (vec)
          expand_tile_in<T, NPC, GS, 2>(sR, RS, src, cnt, L, NM, gl);
        else if (vpart)
          expand_tile_in<T, NPC, GS, 1>(sR, RS, src, cnt, L, NM, gl);
        else
          expand_tile_in<T, NPC, GS, 0>(sR, RS, src, cnt, L, NM, gl);
      }
    }
    __syncthreads();
    const int64_t j = j0 + gl;
    if (active && gl < cnt) {
      const T* sGj = sG + (j < t ? se : 1 - se) * slice;
      if constexpr (STAGE)
        expand_bwd_point<T, MM, NORM, NPC, 0>(xyz, R, sGj, sR + gl * RS, gxyz, gR, j, L, NM);
      else if (vec)
        expand_bwd_point<T, MM, NORM, NPC, 1>(xyz, R, sGj, nullptr, gxyz, gR, j, L, NM);
      else if (vpart)
        expand_bwd_point<T, MM, NORM, NPC, 3>(xyz, R, sGj, nullptr, gxyz, gR, j, L, NM);
      else
        expand_bwd_point<T, MM, NORM, NPC, 2>(xyz, R, sGj, nullptr, gxyz, gR, j, L, NM);
    }
    if constexpr (STAGE) {
      if (gR != nullptr) {
        __syncthreads();  // the group's grad_R rows are in the tile
        if (active) {
          T* dst = gR + j0 * (L + 1) * NM;
          if (vec)
            expand_tile_out<T, NPC, GS, 2>(sR, RS, dst, cnt, L, NM, gl);
          else if (vpart)
            expand_tile_out<T, NPC, GS, 1>(sR, RS, dst, cnt, L, NM, gl);
          else
            expand_tile_out<T, NPC, GS, 0>(sR, RS, dst, cnt, L, NM, gl);
        }
      }
    }
    // advance the group past the chunk
    if (active) {
      j0 += cnt;
      if (span) {  // the chunk ended inside e2 (or at its end): e2 becomes e
        e = e2;
        b = b2;
        t = t2;
        se = 1 - se;
        const int64_t h = in_cur;
        in_cur = in_oth;
        in_oth = h;
      }
      if (j0 >= t) {  // e done: the next non-empty environment
        e = next_nonempty(e + 1, b, t);
        j0 = b;
      }
    }
  }
}

}  // namespace sph
