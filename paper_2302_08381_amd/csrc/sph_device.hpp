// Device building blocks shared by the libsph kernels (gfx950, wave64).
//
// One lane owns one point.  For every degree l the lane builds the row
// Qt_l^0..Qt_l^l from scratch by the folded downward-in-m recursion (rows are
// independent of each other, Eq. iter-q-alt), and s_m, c_m by Eq. iter-sc
// while walking m upward.  A row together with the previous one (and the one
// before, for second derivatives) gives every value and derivative of degree
// l (Eqs. real-sh-cartesian and iter-deri).
//
// Output staging: values of one component (Y, d/dx, d/dy or d/dz) for a
// group of consecutive degrees are written by each lane into its own row of
// an LDS tile ([64 points][stride]); the wave then copies the tile out so
// that consecutive lanes write consecutive addresses of the point-major
// global arrays.  An odd LDS stride keeps the per-lane writes free of bank
// conflicts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "sph_coeffs.hpp"

namespace sph {

constexpr int kWave = 64;
// s_waitcnt operand (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt in
// 6:4, lgkmcnt in 11:8) that waits for every vector-memory access and leaves
// the other counters unconstrained.
constexpr int kWaitVmem0 = 0x0F70;

constexpr CoefTable<float> kCoefF = make_coef_table<float>();
constexpr CoefTable<double> kCoefD = make_coef_table<double>();

template <typename T>
__device__ __forceinline__ constexpr const CoefTable<T>& coef();
template <>
__device__ __forceinline__ constexpr const CoefTable<float>& coef<float>() { return kCoefF; }
template <>
__device__ __forceinline__ constexpr const CoefTable<double>& coef<double>() { return kCoefD; }

// 16-byte native vectors (clang ext_vector_type, usable with the
// nontemporal builtins).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = f32x4;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  using type = f64x2;
  static constexpr int n = 2;
};

// Streaming 16-byte stores of whole output tiles: a buffer store with the
// system-scope (sc1) and nontemporal (nt) cache-policy bits.  On MI355X it
// writes the forward's tiles 2-4 % faster than a plain nontemporal store
// (float and double Y+dY, values only), and the default policy is slower
// still.  The buffer resource covers [base, base + bytes); the hardware drops
// any store past its end.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kStreamStorePolicy = 16 | 2;  // sc1 | nt

__device__ __forceinline__ __amdgpu_buffer_rsrc_t stream_rsrc(void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, bytes, 0x00020000);
}

template <typename V>
__device__ __forceinline__ void stream_store16(const V& v, __amdgpu_buffer_rsrc_t rs, int byte_off) {
  static_assert(sizeof(V) == 16, "16-byte vector");
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rs, byte_off, 0, kStreamStorePolicy);
}

// ------------------------------------------------------------ group plans
// Consecutive degrees are grouped so that one component of one group fits
// the per-point LDS budget (in elements).  A single degree larger than the
// budget forms a group of its own.
struct Plan {
  int ng;
  int lo[kMaxL + 1];  // first degree of group g
  int hi[kMaxL + 1];  // one past the last degree
  int stride;         // LDS elements per point (odd)
};

__host__ __device__ constexpr Plan make_plan(int L, int budget) {
  Plan p{};
  p.ng = 0;
  int mx = 1;
  int la = 0;
  while (la <= L) {
    int lb = la + 1;
    while (lb <= L && (lb + 1) * (lb + 1) - la * la <= budget) ++lb;
    p.lo[p.ng] = la;
    p.hi[p.ng] = lb;
    ++p.ng;
    const int cnt = lb * lb - la * la;
    if (cnt > mx) mx = cnt;
    la = lb;
  }
  p.stride = (mx % 2 == 0) ? mx + 1 : mx;
  return p;
}

// LDS stride (elements per point) of the largest group for l_max = L; the
// same value as make_plan(L, budget).stride without the per-group arrays.
__host__ __device__ constexpr int plan_stride(int L, int budget) {
  int mx = 1;
  for (int la = 0; la <= L;) {
    int lb = la + 1;
    while (lb <= L && (lb + 1) * (lb + 1) - la * la <= budget) ++lb;
    const int cnt = lb * lb - la * la;
    if (cnt > mx) mx = cnt;
    la = lb;
  }
  return (mx % 2 == 0) ? mx + 1 : mx;
}

// End (exclusive) of the group of degrees starting at la.
__host__ __device__ constexpr int group_end(int la, int L, int budget) {
  int lb = la + 1;
  while (lb <= L && (lb + 1) * (lb + 1) - la * la <= budget) ++lb;
  return lb;
}

// LDS row stride (elements) of a group of cnt columns.  An odd cnt is its
// own stride: the rows stay contiguous and one column written by a wave hits
// distinct banks.  An even group that spans whole rows (one group of degrees)
// keeps rows that start on 16-byte boundaries, so the tile can still leave
// with 16-byte stores: cnt itself when cnt / W is odd (contiguous rows), else
// cnt + W.  Partial-row groups of even cnt: cnt + 1.
template <typename T>
__host__ __device__ constexpr int row_stride(int cnt, bool whole_rows) {
  constexpr int W = 16 / static_cast<int>(sizeof(T));
  if (cnt % 2 == 1) return cnt;
  if (!whole_rows || cnt % W != 0) return cnt + 1;
  return ((cnt / W) % 2 == 1) ? cnt : cnt + W;
}

// LDS stride per point of the plan for l_max = L: row_stride of the whole
// row for a one-group plan, the odd plan stride otherwise.
template <typename T>
__host__ __device__ constexpr int tile_stride(int L, int budget) {
  if (group_end(0, L, budget) > L) return row_stride<T>((L + 1) * (L + 1), true);
  return plan_stride(L, budget);
}

// m-extent buckets: a kernel instantiated for MM serves every l_max <= MM
// (its m loops are unrolled to MM and exit at the row's degree).
constexpr int kNumBuckets = 8;
constexpr int kBuckets[kNumBuckets] = {2, 4, 6, 8, 12, 16, 24, 32};
__host__ __device__ constexpr int bucket_index(int L) {
  for (int i = 0; i < kNumBuckets; ++i)
    if (L <= kBuckets[i]) return i;
  return -1;
}

// ------------------------------------------------------------ recursions
// Row l of the folded polynomials: q[m] = Qt_l^m for 0 <= m <= l (l <= MM).
// Entries m > l are left untouched: no caller reads them (every read of a
// neighbouring row is guarded by the degree conditions of its formula).
// l < 0 writes nothing.
template <typename T, int MM>
__device__ __forceinline__ void q_row(int l, T z, T rxy2, T (&q)[MM + 3]) {
  const CoefTable<T>& C = coef<T>();
#pragma unroll
  for (int m = MM; m >= 0; --m) {
    if (m > l) continue;
    if (m == l) {
      q[m] = C.qll[l];
    } else if (m == l - 1) {
      q[m] = (C.b1[l][m] * z) * q[m + 1];
    } else {
      q[m] = (C.b1[l][m] * z) * q[m + 1] + (C.b2[l][m] * rxy2) * q[m + 2];
    }
  }
}

// The same row for a run-time degree, without branches: every slot m <= MM
// is computed (the folded coefficients are 0 for m >= l, so slots past the
// row come out 0) and the row start is a select.  Branches on a run-time
// degree here would make the compiler merge the stores into a dynamically
// indexed one and move the row to scratch memory.
template <typename T, int MM>
__device__ __forceinline__ void q_row_rt(int l, T z, T rxy2, T (&q)[MM + 3]) {
  const CoefTable<T>& C = coef<T>();
  const T qll = (l >= 0) ? C.qll[l < 0 ? 0 : l] : T(0);
  const int li = l < 0 ? 0 : l;
  q[MM + 1] = T(0);
  q[MM + 2] = T(0);
#pragma unroll
  for (int m = MM; m >= 0; --m) {
    const T t = (C.b1[li][m] * z) * q[m + 1] + (C.b2[li][m] * rxy2) * q[m + 2];
    q[m] = (m == l) ? qll : t;
  }
}

// Row of either kind: compile-time degrees take the branchy form (it folds),
// run-time degrees the branch-free one.
template <typename T, int MM, bool CT>
__device__ __forceinline__ void q_row_any(int l, T z, T rxy2, T (&q)[MM + 3]) {
  if constexpr (CT)
    q_row<T, MM>(l, z, rxy2, q);
  else
    q_row_rt<T, MM>(l, z, rxy2, q);
}

// dst[m] = src[m] for m <= l.
template <typename T, int MM>
__device__ __forceinline__ void copy_row(int l, const T (&src)[MM + 3], T (&dst)[MM + 3]) {
#pragma unroll
  for (int m = 0; m <= MM; ++m) {
    if (m > l) continue;  // no early exit: keeps the loop fully unrolled
    dst[m] = src[m];
  }
}

// Component ids of a pass: 0 = value, 1..3 = d/dx, d/dy, d/dz.
// emit_row calls sink(k, value) for every column k = l^2 + l + m of degree l.
//   (ex, ey, ez): evaluation point (x/r for the normalised harmonics)
//   inv_r:        1/r (normalised only; 0 at the origin)
// Scaled derivatives (Eq. iter-deri and the product rule), with
// Tm = gxy * Qt_{l-1}^{m+1}, Cm = gz * Qt_{l-1}^m:
//   d/dx: x Tm {c_m, s_m} + m Qt_l^m {c_{m-1}, s_{m-1}}
//   d/dy: y Tm {c_m, s_m} + m Qt_l^m {-s_{m-1}, c_{m-1}}
//   d/dz: Cm {c_m, s_m}
// Normalised (chain rule through u = x/r): (d_a(u) - l u_a Y(u)) / r.
template <typename T, int MM, int COMP, bool NORM, typename Sink>
__device__ __forceinline__ void emit_row(int l, const T (&prev)[MM + 3], const T (&cur)[MM + 3],
                                         T ex, T ey, T ez, T inv_r, Sink&& sink) {
  const CoefTable<T>& C = coef<T>();
  constexpr T kIS2 = T(kInvSqrt2d);
  const int k0 = l * l + l;
  T lu = T(0);
  if constexpr (NORM && COMP != 0) lu = T(l) * (COMP == 1 ? ex : (COMP == 2 ? ey : ez));
  T sp = T(0), cp = T(1);  // s_{m-1}, c_{m-1}
  T s = T(0), c = T(1);    // s_m, c_m
#pragma unroll
  for (int m = 0; m <= MM; ++m) {
    if (m > l) continue;  // no early exit: keeps the loop fully unrolled
    if (m > 0) {
      const T sn = ex * s + ey * c;
      const T cn = ex * c - ey * s;
      sp = s;
      cp = c;
      s = sn;
      c = cn;
    }
    const T q = cur[m];
    if constexpr (COMP == 0) {
      if (m == 0) {
        sink(k0, q * kIS2);
      } else {
        sink(k0 + m, q * c);
        sink(k0 - m, q * s);
      }
    } else {
      T Tm = T(0), Cm = T(0);
      if (COMP != 3 && m <= l - 2) Tm = C.gxy[l][m] * prev[m + 1];
      if (COMP == 3 && m <= l - 1) Cm = C.gz[l][m] * prev[m];
      if (m == 0) {
        T d = (COMP == 1) ? ex * Tm : (COMP == 2 ? ey * Tm : Cm);
        d *= kIS2;
        if constexpr (NORM) d = (d - lu * (q * kIS2)) * inv_r;
        sink(k0, d);
      } else {
        const T mq = T(m) * q;
        T dp, dm;
        if constexpr (COMP == 1) {
          const T xt = ex * Tm;
          dp = xt * c + mq * cp;
          dm = xt * s + mq * sp;
        } else if constexpr (COMP == 2) {
          const T yt = ey * Tm;
          dp = yt * c - mq * sp;
          dm = yt * s + mq * cp;
        } else {
          dp = Cm * c;
          dm = Cm * s;
        }
        if constexpr (NORM) {
          dp = (dp - lu * (q * c)) * inv_r;
          dm = (dm - lu * (q * s)) * inv_r;
        }
        sink(k0 + m, dp);
        sink(k0 - m, dm);
      }
    }
  }
}

// ------------------------------------------------------------ evaluation point
template <typename T>
struct Point {
  T ex, ey, ez;  // evaluation point
  T rxy2;        // ex^2 + ey^2
  T inv_r;       // normalised only
};

template <typename T, bool NORM>
__device__ __forceinline__ Point<T> make_point(T x, T y, T z) {
  Point<T> p;
  if constexpr (NORM) {
    const T r = sqrt(x * x + y * y + z * z);
    // r == 0 -> inv_r = 0: every l >= 1 value and every derivative vanishes,
    // Y_0^0 keeps its constant.  NaN stays NaN.
    const T ir = (r == T(0)) ? T(0) : T(1) / r;
    p.ex = x * ir;
    p.ey = y * ir;
    p.ez = z * ir;
    p.inv_r = ir;
  } else {
    p.ex = x;
    p.ey = y;
    p.ez = z;
    p.inv_r = T(0);
  }
  p.rxy2 = p.ex * p.ex + p.ey * p.ey;
  return p;
}

// ------------------------------------------------------------ LDS <-> global
// Copies between an LDS tile (rows of stride S) and global rows (stride
// gstride): for row p < rows and j < cnt, dst[p * gstride + j] <-> st[p * S + j].
// NT threads of the block take part (lane = thread index < NT).  With
// gstride == cnt == S (one contiguous block) and a 16-byte aligned global
// pointer the copy uses 16-byte accesses.  Each lane keeps NB accesses in
// flight before it waits, so LDS and memory latency is paid once per batch
// rather than once per element.
constexpr int kBatch = 4;

template <int NT = kWave, int NB = kBatch, typename T>
__device__ __forceinline__ void copy_out(const T* __restrict__ st, int S, T* __restrict__ dst,
                                         int gstride, int cnt, int rows, int lane, bool vec) {
  const int total = rows * cnt;
  constexpr int W = Vec16<T>::n;
  if (vec && gstride == cnt && S != cnt && cnt % W == 0 && S % W == 0) {
    // whole rows, 16-byte aligned LDS rows with padding: vector i of the
    // block is vector (i / CV, i % CV) of the tile, walked incrementally
    using V = typename Vec16<T>::type;
    const int CV = cnt / W, SV = S / W;
    const int nv = rows * CV;
    const V* sv = reinterpret_cast<const V*>(st);
    const __amdgpu_buffer_rsrc_t rs = stream_rsrc(dst, nv * 16);
    int r = lane / CV, c = lane - r * CV;
    const int qs = NT / CV, rq = NT - qs * CV;
    for (int i0 = lane; i0 < nv; i0 += NT * NB) {
      V v[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        if (i0 + u * NT < nv) v[u] = sv[r * SV + c];
        r += qs;
        c += rq;
        if (c >= CV) {
          c -= CV;
          ++r;
        }
      }
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (i0 + u * NT < nv) stream_store16(v[u], rs, (i0 + u * NT) * 16);
    }
    return;
  }
  if (vec && gstride == cnt && S == cnt) {
    using V = typename Vec16<T>::type;
    const int nv = total / W;
    const V* sv = reinterpret_cast<const V*>(st);
    const __amdgpu_buffer_rsrc_t rs = stream_rsrc(dst, nv * 16);
    for (int i0 = lane; i0 < nv; i0 += NT * NB) {
      V v[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (i0 + u * NT < nv) v[u] = sv[i0 + u * NT];
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (i0 + u * NT < nv) stream_store16(v[u], rs, (i0 + u * NT) * 16);
    }
    for (int j = nv * W + lane; j < total; j += NT) __builtin_nontemporal_store(st[j], dst + j);
    return;
  }
  if (gstride != cnt && cnt >= 2 * W) {
    // Partial rows (one group of degrees).  Every row segment holds at least
    // M = floor((cnt - W + 1) / W) whole aligned 16-byte vectors, starting
    // after its head (the elements before its first aligned one); they leave
    // with 16-byte stores.  The other R = cnt - W M elements of the row (its
    // head and its tail) leave one by one.  Default cache policy: L2 merges
    // the partial lines at segment ends.  All stores go through a buffer
    // resource that covers exactly the rows' span.
    using V = typename Vec16<T>::type;
    const int M = (cnt - (W - 1)) / W;
    const int R = cnt - W * M;
    const int a0 = static_cast<int>((reinterpret_cast<uintptr_t>(dst) / sizeof(T)) % W);
    const int gm = gstride % W;
    const __amdgpu_buffer_rsrc_t rsr = stream_rsrc(dst, static_cast<int>(((rows - 1) * gstride + cnt) * sizeof(T)));
    {
      int r = lane / M, j = lane - r * M;
      const int qs = NT / M, rq = NT - qs * M;
      for (int i = lane; i < rows * M; i += NT) {
        const int c0 = (W - (a0 + r * gm) % W) % W + W * j;  // first column of the vector
        V v;
#pragma unroll
        for (int t = 0; t < W; ++t) v[t] = st[r * S + c0 + t];
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rsr,
                                               static_cast<int>((r * gstride + c0) * sizeof(T)), 0, 0);
        r += qs;
        j += rq;
        if (j >= M) {
          j -= M;
          ++r;
        }
      }
    }
    {
      int r = lane / R, e = lane - r * R;
      const int qs = NT / R, rq = NT - qs * R;
      for (int i = lane; i < rows * R; i += NT) {
        const int head = (W - (a0 + r * gm) % W) % W;
        const int c = e < head ? e : e + W * M;  // the head, then the tail after the middle
        const int off = static_cast<int>((r * gstride + c) * sizeof(T));
        if constexpr (sizeof(T) == 4)
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, st[r * S + c]), rsr, off, 0, 0);
        else
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, st[r * S + c]), rsr, off, 0, 0);
        r += qs;
        e += rq;
        if (e >= R) {
          e -= R;
          ++r;
        }
      }
    }
    return;
  }
  int p = lane / cnt;
  int k = lane - p * cnt;
  const int qs = NT / cnt;
  const int rs = NT - qs * cnt;
  for (int j0 = lane; j0 < total; j0 += NT * NB) {
    T v[NB];
    int off[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      off[u] = p * gstride + k;
      if (j0 + u * NT < total) v[u] = st[p * S + k];
      p += qs;
      k += rs;
      if (k >= cnt) {
        k -= cnt;
        ++p;
      }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (j0 + u * NT < total) dst[off[u]] = v[u];  // partial lines: let L2 merge them
  }
}

template <int NT = kWave, int NB = kBatch, typename T>
__device__ __forceinline__ void copy_in(T* __restrict__ st, int S, const T* __restrict__ src,
                                        int gstride, int cnt, int rows, int lane, bool vec) {
  const int total = rows * cnt;
  constexpr int W = Vec16<T>::n;
  if (vec && gstride == cnt && S != cnt && cnt % W == 0 && S % W == 0) {
    // whole rows into padded, 16-byte aligned LDS rows (as in copy_out)
    using V = typename Vec16<T>::type;
    const int CV = cnt / W, SV = S / W;
    const int nv = rows * CV;
    V* sv = reinterpret_cast<V*>(st);
    const V* dv = reinterpret_cast<const V*>(src);
    int r = lane / CV, c = lane - r * CV;
    const int qs = NT / CV, rq = NT - qs * CV;
    for (int i0 = lane; i0 < nv; i0 += NT * NB) {
      V v[NB];
      int o[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        o[u] = r * SV + c;
        if (i0 + u * NT < nv) v[u] = __builtin_nontemporal_load(dv + i0 + u * NT);
        r += qs;
        c += rq;
        if (c >= CV) {
          c -= CV;
          ++r;
        }
      }
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (i0 + u * NT < nv) sv[o[u]] = v[u];
    }
    return;
  }
  if (vec && gstride == cnt && S == cnt) {
    using V = typename Vec16<T>::type;
    const int nv = total / W;
    V* sv = reinterpret_cast<V*>(st);
    const V* dv = reinterpret_cast<const V*>(src);
    for (int i0 = lane; i0 < nv; i0 += NT * NB) {
      V v[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (i0 + u * NT < nv) v[u] = __builtin_nontemporal_load(dv + i0 + u * NT);
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (i0 + u * NT < nv) sv[i0 + u * NT] = v[u];
    }
    for (int j = nv * W + lane; j < total; j += NT) st[j] = __builtin_nontemporal_load(src + j);
    return;
  }
  int p = lane / cnt;
  int k = lane - p * cnt;
  const int qs = NT / cnt;
  const int rs = NT - qs * cnt;
  for (int j0 = lane; j0 < total; j0 += NT * NB) {
    T v[NB];
    int off[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      off[u] = p * S + k;
      if (j0 + u * NT < total) v[u] = __builtin_nontemporal_load(src + (p * gstride + k));
      p += qs;
      k += rs;
      if (k >= cnt) {
        k -= cnt;
        ++p;
      }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (j0 + u * NT < total) st[off[u]] = v[u];
  }
}

// Two contiguous global blocks a[0, na) and b[0, nb) (16-byte aligned) into
// two LDS blocks, as one list of 16-byte vectors with NB per thread in flight:
// both blocks share the memory round trips.  Elements past the last whole
// vector of each block are copied one by one.
template <int NT, int NB, typename T>
__device__ __forceinline__ void copy_in_pair(T* __restrict__ sa, const T* __restrict__ a, int na,
                                             T* __restrict__ sb, const T* __restrict__ b, int nb, int lane) {
  using V = typename Vec16<T>::type;
  constexpr int W = Vec16<T>::n;
  const int nva = na / W, nvb = nb / W;
  const int nv = nva + nvb;
  const V* ga = reinterpret_cast<const V*>(a);
  const V* gb = reinterpret_cast<const V*>(b);
  V* la = reinterpret_cast<V*>(sa);
  V* lb = reinterpret_cast<V*>(sb);
  for (int i0 = lane; i0 < nv; i0 += NT * NB) {
    V v[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int i = i0 + u * NT;
      if (i < nv) v[u] = __builtin_nontemporal_load(i < nva ? ga + i : gb + (i - nva));
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int i = i0 + u * NT;
      if (i < nv) *(i < nva ? la + i : lb + (i - nva)) = v[u];
    }
  }
  for (int j = nva * W + lane; j < na; j += NT) sa[j] = __builtin_nontemporal_load(a + j);
  for (int j = nvb * W + lane; j < nb; j += NT) sb[j] = __builtin_nontemporal_load(b + j);
}

// A full tile of whole rows, loaded in two halves so that the memory latency
// overlaps other work: prefetch() issues the 16-byte loads of NV vectors of
// src into registers (NT threads, thread lane), commit() writes them to LDS
// rows of SV vectors (CV per row: the same row geometry as copy_out_full).
template <typename T, int NV, int NT, int CV = 1, int SV = 1>
struct TilePrefetch {
  using V = typename Vec16<T>::type;
  static constexpr int kPer = (NV + NT - 1) / NT;
  V v[kPer];
  __device__ __forceinline__ void prefetch(const T* __restrict__ src, int lane) {
    const V* g = reinterpret_cast<const V*>(src);
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      if (u < NV / NT || lane + u * NT < NV) v[u] = __builtin_nontemporal_load(g + lane + u * NT);
  }
  __device__ __forceinline__ void commit(T* __restrict__ st, int lane) const {
    V* d = reinterpret_cast<V*>(st);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int i = lane + u * NT;
      if (u < NV / NT || i < NV) d[CV == SV ? i : (i / CV) * SV + i % CV] = v[u];
    }
  }
};

// Full-tile contiguous copy with compile-time size: NV 16-byte vectors from
// LDS to global by NT threads, kBatchFull in flight per lane, no predication
// except on the last, partial sweep.
constexpr int kBatchFull = 8;

// CV, SV: 16-byte vectors per row in global memory and in LDS (SV > CV for
// padded LDS rows; vector i of the block is LDS vector (i / CV) SV + i % CV).
template <typename T, int NV, int NT = kWave, int CV = 1, int SV = 1>
__device__ __forceinline__ void copy_out_full(const T* __restrict__ st, T* __restrict__ dst, int lane) {
  using V = typename Vec16<T>::type;
  const V* sv = reinterpret_cast<const V*>(st);
  const __amdgpu_buffer_rsrc_t rs = stream_rsrc(dst, NV * 16);
  constexpr int kSweeps = (NV + NT - 1) / NT;
  auto at = [](int i) { return CV == SV ? i : (i / CV) * SV + i % CV; };
#pragma unroll
  for (int s0 = 0; s0 < kSweeps; s0 += kBatchFull) {
    V v[kBatchFull];
#pragma unroll
    for (int u = 0; u < kBatchFull; ++u) {
      const int sw = s0 + u;
      if (sw < kSweeps && (sw < NV / NT || lane + sw * NT < NV)) v[u] = sv[at(lane + sw * NT)];
    }
#pragma unroll
    for (int u = 0; u < kBatchFull; ++u) {
      const int sw = s0 + u;
      if (sw < kSweeps && (sw < NV / NT || lane + sw * NT < NV))
        stream_store16(v[u], rs, (lane + sw * NT) * 16);
    }
  }
}

// Block index -> tile slot, a permutation of [0, G) that gives the blocks
// dispatched to one XCD (workgroups go to the 8 XCDs round-robin) one
// contiguous range of slots, so each XCD writes one long run of output
// instead of every eighth tile.  Correct for any dispatch order.  Measured on
// the forward with derivatives at l_max = 8: 231.6 -> 208.0 us (float),
// 446 -> 438 us (double); values only 58.0 -> 56.9 us.  The backward, which
// reads, is 2 % slower in this order and keeps the plain one.
constexpr int kNumXcd = 8;

__device__ __forceinline__ int64_t xcd_slot(int64_t b, int64_t G) {
  const int64_t x = b % kNumXcd, j = b / kNumXcd;
  const int64_t q = G / kNumXcd, rem = G % kNumXcd;
  return x * q + (x < rem ? x : rem) + j;
}

__device__ __forceinline__ bool aligned16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

}  // namespace sph
