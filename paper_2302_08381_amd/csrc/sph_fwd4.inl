// Forward with derivatives, four lanes per point.
//
// A block of one or two waves takes a tile of 16 or 32 points; thread 4p + r
// evaluates point p of the tile and emits component r of it: r = 0 the
// values, r = 1, 2, 3 the d/dx, d/dy, d/dz derivatives.  Every lane runs the
// same instructions (the four components differ only in per-lane weights, so
// nothing diverges):
//
//   value(+m) = A c_m + B P+ ,  value(-m) = A s_m + B P-
//   A = w_q Qt_l^m + w_t Tm + w_c Cm        (Tm = gxy Qt_{l-1}^{m+1}, Cm = gz Qt_{l-1}^m)
//   B = w_b m Qt_l^m,  P+ = a1 c_{m-1} + a2 s_{m-1},  P- = a1 s_{m-1} - a2 c_{m-1}
//
// with (w_q, w_t, w_c, w_b, a1, a2) = (1, 0, 0, 0, -, -) for the values,
// (0, x, 0, 1, 1, 0) for d/dx, (0, y, 0, 1, 0, -1) for d/dy and
// (0, 0, 1, 0, -, -) for d/dz, which restates Eqs. real-sh-cartesian and
// iter-deri with the product rule.  For the normalised harmonics the chain
// rule (d_a Yt(u) - l u_a Yt(u)) / r folds into A -> (A - l u_a Qt) / r and
// B -> B / r.
//
// The LDS tile is laid out exactly as the global arrays: the P value rows
// (the points' Y rows) followed by 3P derivative rows (dY[p][a]); with one
// group of degrees both blocks are contiguous in global memory and are
// copied out with 16-byte stores.  Tiles whose share of Y and dY is a whole
// number of 128-byte lines write no cache line from two blocks; a line split
// between blocks costs write bandwidth.  The fused backward (batched entry) adds
// sum_k gY[p,k] dY[p,a,k] in thread 4p + a + 1, which then owns
// grad_xyz[p,a].
#pragma once

#include "sph_device.hpp"
#include "sph_fwd.inl"
#include "sph_launch.hpp"

namespace sph {

// Waves per block.  Float kernels for a compile-time l_max <= 8 (K <= 81)
// take a 32-point tile on two waves, which makes each block's share of Y and
// dY a whole number of 128-byte lines (32 K and 96 K floats, K odd).  Every
// other kernel takes a 16-point tile on one wave so that the one-group LDS
// tile of a larger K still fits; for double a 16-point share is already a
// whole number of lines.  LT < 0: run-time l_max.
template <typename T>
constexpr int quad_waves(int LT) {
  return (std::is_same_v<T, float> && LT >= 0 && LT <= 8) ? 2 : 1;
}
constexpr int kQuadWavePoints = 16;  // points per wave (four lanes per point)

// Per-point LDS budget (elements of one component of one group of degrees).
// A one-wave tile (64 rows) then stays near 44 KB, and l_max <= 12 (float)
// or l_max <= 8 (double) is evaluated as one group of degrees, whose rows are
// contiguous in global memory.  Larger l_max split into groups of degrees
// whose partial rows are written with 4-byte stores.
template <typename T>
inline constexpr int kQuadBudget = 172;
template <>
inline constexpr int kQuadBudget<double> = 86;

template <typename T>
struct Role {
  T wq, wt, wc, wb, a1, a2;  // weights of the unified formula
  T lu;                      // u_a (normalised; times l per degree), 0 for the values
  T sc;                      // 1/r for normalised derivatives, else 1
};

template <typename T, bool NORM>
__device__ __forceinline__ Role<T> make_role(int r, const Point<T>& pt) {
  Role<T> ro;
  ro.wq = (r == 0) ? T(1) : T(0);
  ro.wt = (r == 1) ? pt.ex : ((r == 2) ? pt.ey : T(0));
  ro.wc = (r == 3) ? T(1) : T(0);
  ro.a1 = (r == 1) ? T(1) : T(0);
  ro.a2 = (r == 2) ? T(-1) : T(0);
  T sc = T(1);
  T lu = T(0);
  if constexpr (NORM) {
    if (r != 0) {
      sc = pt.inv_r;
      lu = (r == 1) ? pt.ex : ((r == 2) ? pt.ey : pt.ez);
    }
  }
  ro.wb = (r == 1 || r == 2) ? sc : T(0);
  ro.sc = sc;
  ro.lu = lu;
  return ro;
}

// Emit degrees [la, lb) of this lane's component into row[k] (row is the
// lane's LDS row shifted by -kb).  UNROLL: the degree loop has compile-time
// bounds and is unrolled.
template <typename T, int MM, bool NORM>
__device__ __forceinline__ void emit4_row(int l, const Role<T>& ro, const Point<T>& pt,
                                          const T (&prev)[MM + 3], const T (&cur)[MM + 3], T* row) {
  const CoefTable<T>& C = coef<T>();
  constexpr T kIS2 = T(kInvSqrt2d);
  const int k0 = l * l + l;
  T lu = T(0);
  if constexpr (NORM) lu = T(l) * ro.lu;
  T sp = T(0), cp = T(1);
  T s = T(0), c = T(1);
#pragma unroll
  for (int m = 0; m <= MM; ++m) {
    if (m > l) continue;  // no early exit: keeps the loop fully unrolled
    if (m > 0) {
      const T sn = pt.ex * s + pt.ey * c;
      const T cn = pt.ex * c - pt.ey * s;
      sp = s;
      cp = c;
      s = sn;
      c = cn;
    }
    const T q = cur[m];
    const T Tm = (m <= l - 2) ? C.gxy[l][m] * prev[m + 1] : T(0);
    const T Cm = (m <= l - 1) ? C.gz[l][m] * prev[m] : T(0);
    T A = q * ro.wq + Tm * ro.wt + Cm * ro.wc;
    if constexpr (NORM) A = (A - lu * q) * ro.sc;
    if (m == 0) {
      row[k0] = A * kIS2;
    } else {
      const T B = q * (T(m) * ro.wb);
      const T Pp = cp * ro.a1 + sp * ro.a2;
      const T Pm = sp * ro.a1 - cp * ro.a2;
      row[k0 + m] = A * c + B * Pp;
      row[k0 - m] = A * s + B * Pm;
    }
  }
}

// Emit degrees [la, lb) of this lane's component into row[k] (row is the
// lane's LDS row shifted by -kb).  UNROLL: the degree loop has compile-time
// bounds and is unrolled.
template <typename T, int MM, bool NORM, bool UNROLL>
__device__ __forceinline__ void emit4(const Role<T>& ro, const Point<T>& pt, int la, int lb, T* row) {
  constexpr int UR = UNROLL ? 64 : 1;
  T prev[MM + 3], cur[MM + 3];
  q_row_any<T, MM, UNROLL>(la - 1, pt.ez, pt.rxy2, prev);
#pragma unroll UR
  for (int l = la; l < lb; ++l) {
    q_row_any<T, MM, UNROLL>(l, pt.ez, pt.rxy2, cur);
    emit4_row<T, MM, NORM>(l, ro, pt, prev, cur, row);
    copy_row<T, MM>(UNROLL ? l : MM, cur, prev);
  }
}

// The lane's terms of order m that do not depend on the degree: c_m, s_m and
// the product-rule factors m w_b P+(m), m w_b P-(m) (m <= MM, compile-time).
template <typename T, int MM>
struct MTerms {
  T c[MM + 1], s[MM + 1], bp[MM + 1], bm[MM + 1];
};

template <typename T, int MM>
__device__ __forceinline__ void make_mterms(const Role<T>& ro, const Point<T>& pt, MTerms<T, MM>& t) {
  t.c[0] = T(1);
  t.s[0] = T(0);
  t.bp[0] = T(0);
  t.bm[0] = T(0);
#pragma unroll
  for (int m = 1; m <= MM; ++m) {
    const T cp = t.c[m - 1], sp = t.s[m - 1];
    t.s[m] = pt.ex * sp + pt.ey * cp;
    t.c[m] = pt.ex * cp - pt.ey * sp;
    const T w = T(m) * ro.wb;
    t.bp[m] = w * (cp * ro.a1 + sp * ro.a2);
    t.bm[m] = w * (sp * ro.a1 - cp * ro.a2);
  }
}

// emit4_row with the m terms tabulated and the weights pre-scaled:
//   A = q ql + wts gxy Qt_{l-1}^{m+1} + wcs gz Qt_{l-1}^m,
//   ql = (w_q - l u_a) s,  wts = w_t s,  wcs = w_c s   (s = 1/r or 1),
// the same A as emit4_row (the chain-rule correction folded into ql), and
//   value(+m) = A c_m + q bp_m,  value(-m) = A s_m + q bm_m.
template <typename T, int MM>
__device__ __forceinline__ void emit4_row_tab(int l, T ql, T wts, T wcs, const MTerms<T, MM>& t,
                                              const T (&prev)[MM + 3], const T (&cur)[MM + 3], T* row) {
  const CoefTable<T>& C = coef<T>();
  constexpr T kIS2 = T(kInvSqrt2d);
  const int k0 = l * l + l;
#pragma unroll
  for (int m = 0; m <= MM; ++m) {
    if (m > l) continue;  // no early exit: keeps the loop fully unrolled
    const T q = cur[m];
    T A = q * ql;
    if (m <= l - 2) A += (C.gxy[l][m] * prev[m + 1]) * wts;
    if (m <= l - 1) A += (C.gz[l][m] * prev[m]) * wcs;
    if (m == 0) {
      row[k0] = A * kIS2;
    } else {
      row[k0 + m] = A * t.c[m] + q * t.bp[m];
      row[k0 - m] = A * t.s[m] + q * t.bm[m];
    }
  }
}

// Degrees [LA, LB) known at compile time: the degree loop unrolls fully,
// every coefficient is a literal and the terms of order m are computed once.
template <typename T, int MM, bool NORM, int LA, int LB>
__device__ __forceinline__ void emit4_ct(const Role<T>& ro, const Point<T>& pt, T* row) {
  T prev[MM + 3], cur[MM + 3];
  MTerms<T, MM> t;
  make_mterms<T, MM>(ro, pt, t);
  const T wqs = ro.wq * ro.sc, lus = ro.lu * ro.sc;
  const T wts = ro.wt * ro.sc, wcs = ro.wc * ro.sc;
  if constexpr (LA >= 1) q_row<T, MM>(LA - 1, pt.ez, pt.rxy2, prev);
#pragma unroll
  for (int l = LA; l < LB; ++l) {
    q_row<T, MM>(l, pt.ez, pt.rxy2, cur);
    const T ql = NORM ? wqs - T(l) * lus : wqs;
    emit4_row_tab<T, MM>(l, ql, wts, wcs, t, prev, cur, row);
    copy_row<T, MM>(l, cur, prev);
  }
}

template <typename T, int NW, int MM, bool NORM, bool UNROLL, bool FUSED, bool STORE>
__device__ __forceinline__ void fwd4_group(const Role<T>& ro, const Point<T>& pt, int la, int lb, int K,
                                           int64_t p0, int np, int lane, int lrow, const FwdParams& P,
                                           T* st, T* sg, T& acc) {
  constexpr int PT = kQuadWavePoints * NW;
  constexpr int NT = kWave * NW;
  const int kb = la * la;
  const int cnt = lb * lb - kb;
  const int S = row_stride<T>(cnt, cnt == K);
  constexpr bool bwd = FUSED;
  const int p = lane >> 2;
  if (bwd) {
    const T* src = static_cast<const T*>(P.gY) + p0 * K + kb;
    copy_in<NT>(sg, S, src, K, cnt, np, lane, aligned16(src));
  }
  emit4<T, MM, NORM, UNROLL>(ro, pt, la, lb, st + lrow * S - kb);
  __syncthreads();
  if (bwd) {
    // derivative lanes: sum_k gY[p,k] dY[p,a,k] over this group
    const T* gr = sg + p * S;
    const T* dr = st + lrow * S;
    T s0 = T(0), s1 = T(0);
    int j = 0;
    for (; j + 1 < cnt; j += 2) {
      s0 += gr[j] * dr[j];
      s1 += gr[j + 1] * dr[j + 1];
    }
    if (j < cnt) s0 += gr[j] * dr[j];
    acc += s0 + s1;
  }
  {
    T* dst = static_cast<T*>(P.Y) + p0 * K + kb;
    copy_out<NT>(st, S, dst, K, cnt, np, lane, aligned16(dst));
  }
  if constexpr (STORE) {
    T* dst = static_cast<T*>(P.dY) + p0 * 3 * K + kb;
    copy_out<NT>(st + PT * S, S, dst, K, cnt, 3 * np, lane, aligned16(dst));
  }
  __syncthreads();
}

// A group of degrees [la, lb) of a run-time l_max with its degrees split
// between the block's two waves at the degree that balances the columns:
// wave h emits [la, ls) or [ls, lb) of every point (uniform per wave), both
// store the group.  Values and derivatives only (no fused backward).
template <typename T, int MM, bool NORM, bool STORE>
__device__ __forceinline__ void fwd4_group_split_rt(const Role<T>& ro, const Point<T>& pt, int la, int lb, int K,
                                                    int64_t p0, int np, int tid, int half, int lrow,
                                                    const FwdParams& P, T* st) {
  constexpr int PT = kQuadWavePoints;
  constexpr int NT = 2 * kWave;
  const int kb = la * la;
  const int cnt = lb * lb - kb;
  const int S = row_stride<T>(cnt, cnt == K);
  int ls = la + 1;  // first degree of wave 1
  while (ls < lb && 2 * (ls * ls - kb) < cnt) ++ls;
  if (half == 0)
    emit4<T, MM, NORM, false>(ro, pt, la, ls, st + lrow * S - kb);
  else
    emit4<T, MM, NORM, false>(ro, pt, ls, lb, st + lrow * S - kb);
  __syncthreads();
  {
    T* dst = static_cast<T*>(P.Y) + p0 * K + kb;
    copy_out<NT>(st, S, dst, K, cnt, np, tid, aligned16(dst));
  }
  if constexpr (STORE) {
    T* dst = static_cast<T*>(P.dY) + p0 * 3 * K + kb;
    copy_out<NT>(st + PT * S, S, dst, K, cnt, 3 * np, tid, aligned16(dst));
  }
  __syncthreads();
}

// One compile-time group of degrees [LA, LB).  FAST: a full tile of
// a one-group plan with 16-byte aligned outputs, copied out with the
// fixed-size unpredicated copy; otherwise the general copy.
template <typename T, int NW, int MM, bool NORM, bool FUSED, bool STORE, bool FAST, bool WHOLE, int LA, int LB>
__device__ __forceinline__ void fwd4_group_ct(const Role<T>& ro, const Point<T>& pt, int K, int64_t p0, int np,
                                              int lane, int lrow, const FwdParams& P, T* st, T* sg, T& acc) {
  constexpr int PT = kQuadWavePoints * NW;
  constexpr int NT = kWave * NW;
  constexpr int kb = LA * LA;
  constexpr int cnt = LB * LB - kb;
  constexpr int S = row_stride<T>(cnt, WHOLE);
  constexpr int W = Vec16<T>::n;
  const int p = lane >> 2;
  // full tiles: the upstream-gradient tile is loaded into registers before
  // the emission and written to LDS after it, so its latency is hidden
  constexpr bool kPre = FUSED && FAST;
  constexpr int GCV = S == cnt ? 1 : cnt / W, GSV = S == cnt ? 1 : S / W;
  TilePrefetch<T, kPre ? PT * cnt / W : 1, NT, GCV, GSV> gpre;
  if constexpr (kPre) {
    gpre.prefetch(static_cast<const T*>(P.gY) + p0 * K, lane);
  } else if constexpr (FUSED) {
    const T* src = static_cast<const T*>(P.gY) + p0 * K + kb;
    copy_in<NT>(sg, S, src, K, cnt, np, lane, aligned16(src));
  }
  emit4_ct<T, MM, NORM, LA, LB>(ro, pt, st + lrow * S - kb);
  if constexpr (kPre) gpre.commit(sg, lane);
  __syncthreads();
  if constexpr (FUSED) {
    const T* gr = sg + p * S;
    const T* dr = st + lrow * S;
    T s0 = T(0), s1 = T(0);
#pragma unroll
    for (int j = 0; j + 1 < cnt; j += 2) {
      s0 += gr[j] * dr[j];
      s1 += gr[j + 1] * dr[j + 1];
    }
    if constexpr (cnt % 2 == 1) s0 += gr[cnt - 1] * dr[cnt - 1];
    acc += s0 + s1;
  }
  T* ydst = static_cast<T*>(P.Y) + p0 * K + kb;
  T* ddst = STORE ? static_cast<T*>(P.dY) + p0 * 3 * K + kb : nullptr;
  if constexpr (FAST) {
    static_assert(WHOLE && kb == 0, "fast path needs one group of whole rows");
    constexpr int CV = S == cnt ? 1 : cnt / W, SV = S == cnt ? 1 : S / W;
    copy_out_full<T, PT * cnt / W, NT, CV, SV>(st, ydst, lane);
    if constexpr (STORE)
      copy_out_full<T, 3 * PT * cnt / W, NT, CV, SV>(st + PT * S, ddst, lane);
  } else {
    copy_out<NT>(st, S, ydst, K, cnt, np, lane, aligned16(ydst));
    if constexpr (STORE)
      copy_out<NT>(st + PT * S, S, ddst, K, cnt, 3 * np, lane, aligned16(ddst));
  }
  __syncthreads();
}

template <typename T, int NW, int MM, bool NORM, bool FUSED, bool STORE, bool FAST, int LT, int... Gs>
__device__ __forceinline__ void fwd4_groups_ct(std::integer_sequence<int, Gs...>, const Role<T>& ro,
                                               const Point<T>& pt, int K, int64_t p0, int np, int lane,
                                               int lrow, const FwdParams& P, T* st, T* sg, T& acc) {
  constexpr Plan PL = make_plan(LT, kQuadBudget<T>);
  (fwd4_group_ct<T, NW, MM, NORM, FUSED, STORE, FAST, PL.ng == 1, PL.lo[Gs], PL.hi[Gs]>(ro, pt, K, p0, np, lane,
                                                                                       lrow, P, st, sg, acc),
   ...);
}

// Degree at which a one-group tile of compile-time l_max LT is split between
// two waves: the l with l^2 (columns below it) closest to K/2.
template <int LT>
constexpr int split_degree() {
  constexpr int K = (LT + 1) * (LT + 1);
  int best = 1;
  for (int l = 1; l <= LT; ++l) {
    const int d = 2 * l * l - K, db = 2 * best * best - K;
    if ((d < 0 ? -d : d) < (db < 0 ? -db : db)) best = l;
  }
  return best;
}

// A one-group 16-point tile whose degrees are split between the block's two
// waves: wave 0 emits degrees [0, LS) and wave 1 degrees [LS, LT] of every
// point (the branch is uniform per wave), both store the tile.  Twice the
// waves of a one-wave tile on the same LDS, for kernels whose tile takes
// most of a CU's LDS.  tid: thread of the block (0..127); lane: quad lane
// within the wave.  FUSED: each wave sums gY.dY over its own columns; wave 1
// leaves its partial sum in sacc[lane] for wave 0 (read after the final
// barrier).
template <typename T, int MM, bool NORM, bool FUSED, bool STORE, bool FAST, int LT>
__device__ __forceinline__ void fwd4_tile_split(const Role<T>& ro, const Point<T>& pt, int64_t p0, int np,
                                                int tid, int half, int lane, int lrow, const FwdParams& P,
                                                T* st, T* sg, T* sacc, T& acc) {
  constexpr int PT = kQuadWavePoints;
  constexpr int NT = 2 * kWave;
  constexpr int K = (LT + 1) * (LT + 1);
  constexpr int S = row_stride<T>(K, true);
  constexpr int LS = split_degree<LT>();
  constexpr int KS = LS * LS;  // first column of wave 1
  const int p = lane >> 2;
  constexpr int W = Vec16<T>::n;
  constexpr bool kPre = FUSED && FAST;  // as in fwd4_group_ct
  constexpr int GCV = S == K ? 1 : K / W, GSV = S == K ? 1 : S / W;
  TilePrefetch<T, kPre ? PT * K / W : 1, NT, GCV, GSV> gpre;
  if constexpr (kPre) {
    gpre.prefetch(static_cast<const T*>(P.gY) + p0 * K, tid);
  } else if constexpr (FUSED) {
    const T* src = static_cast<const T*>(P.gY) + p0 * K;
    copy_in<NT>(sg, S, src, K, K, np, tid, aligned16(src));
  }
  T* row = st + lrow * S;
  if (half == 0)
    emit4_ct<T, LS - 1, NORM, 0, LS>(ro, pt, row);
  else
    emit4_ct<T, MM, NORM, LS, LT + 1>(ro, pt, row);
  if constexpr (kPre) gpre.commit(sg, tid);
  __syncthreads();
  if constexpr (FUSED) {
    const T* gr = sg + p * S;
    T s0 = T(0), s1 = T(0);
    if (half == 0) {
#pragma unroll
      for (int j = 0; j < KS; ++j) ((j & 1) ? s1 : s0) += gr[j] * row[j];
      acc += s0 + s1;
    } else {
#pragma unroll
      for (int j = KS; j < K; ++j) ((j & 1) ? s1 : s0) += gr[j] * row[j];
      sacc[lane] = s0 + s1;
    }
  }
  T* ydst = static_cast<T*>(P.Y) + p0 * K;
  T* ddst = STORE ? static_cast<T*>(P.dY) + p0 * 3 * K : nullptr;
  if constexpr (FAST) {
    constexpr int CV = S == K ? 1 : K / W, SV = S == K ? 1 : S / W;
    copy_out_full<T, PT * K / W, NT, CV, SV>(st, ydst, tid);
    if constexpr (STORE) copy_out_full<T, 3 * PT * K / W, NT, CV, SV>(st + PT * S, ddst, tid);
  } else {
    copy_out<NT>(st, S, ydst, K, K, np, tid, aligned16(ydst));
    if constexpr (STORE) copy_out<NT>(st + PT * S, S, ddst, K, K, 3 * np, tid, aligned16(ddst));
  }
  __syncthreads();
}

// Whether a compile-time l_max has a single contiguous group (the fast
// full-tile path).
template <typename T, int LT>
constexpr bool quad_has_fast() {
  if constexpr (LT < 0) {
    return false;
  } else {
    constexpr Plan PL = make_plan(LT, kQuadBudget<T>);
    constexpr int K = (LT + 1) * (LT + 1);
    return PL.ng == 1 && (K % 2 == 1 || K % Vec16<T>::n == 0);
  }
}

// LT >= 0: l_max = LT known at compile time (MM = LT, degree loops unrolled);
// LT < 0: l_max = P.L <= MM at run time.  NW waves per block (a tile of
// 16 NW points; quad_waves gives the default); DS = 2: the degrees of a
// one-wave tile split between two waves (fwd4_tile_split).  FUSED: the
// backward is fused
// (P.gY, P.gxyz); STORE: dY is written.  Dynamic LDS: 4 PT rows of
// stride(L) elements, plus PT rows for the upstream-gradient tile when FUSED.
//
// Full tiles of a one-group plan run a single straight path per tile: the
// next tile's coordinates are loaded first and the tile's stores follow, so
// the wait for that load leaves the stores in flight (loads and stores
// retire in order on one counter).  A branch in the loop whose paths issue
// different numbers of memory operations would turn that wait into a drain
// of every store of the tile, so the ragged last tile and unaligned outputs
// take a separate general path.
template <typename T, int MM, int LT, bool NORM, bool FUSED, bool STORE, int NW, int DS>
__global__ __launch_bounds__(kWave * NW * DS) void k_fwd4(FwdParams P) {
  static_assert(DS == 1 || (DS == 2 && NW == 1 && (LT >= 0 || !FUSED)),
                "degree split: one-wave tiles; run-time l_max without the fused backward");
  constexpr int PT = kQuadWavePoints * NW;  // points per tile
  constexpr int NQ = kWave * NW;            // quad lanes: four per point, also the tile's rows
  constexpr int B = kQuadBudget<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;  // 0 .. NQ * DS - 1
  const int lane = DS == 1 ? tid : tid % NQ;
  const int half = DS == 1 ? 0 : tid / NQ;
  const int L = LT >= 0 ? LT : P.L;
  const int K = (L + 1) * (L + 1);
  const int smax = tile_stride<T>(L, B);
  T* st = reinterpret_cast<T*>(smem);
  T* sg = st + NQ * smax;
  T* sacc = sg + PT * smax;  // degree split, fused: wave 1's partial sums
  const int p = lane >> 2;
  const int r = lane & 3;
  const int lrow = (r == 0) ? p : PT + 3 * p + (r - 1);

  if (P.status != nullptr && blockIdx.x == 0 && tid < kWave) check_offsets(P, tid);

  const T* xyz = static_cast<const T*>(P.xyz);
  auto tile_body = [&](int64_t tile, T x, T y, T z, auto fast_c) {
    constexpr bool FAST = decltype(fast_c)::value;
    const int64_t p0 = tile * PT;
    const int np = FAST ? PT : static_cast<int>(P.n - p0 < PT ? P.n - p0 : PT);
    const Point<T> pt = make_point<T, NORM>(x, y, z);
    const Role<T> ro = make_role<T, NORM>(r, pt);
    T acc = T(0);
    if constexpr (DS == 2 && LT < 0) {
      for (int la = 0; la <= L;) {
        const int lb = group_end(la, L, B);
        fwd4_group_split_rt<T, MM, NORM, STORE>(ro, pt, la, lb, K, p0, np, tid, half, lrow, P, st);
        la = lb;
      }
    } else if constexpr (DS == 2) {
      static_assert(make_plan(LT, B).ng == 1, "degree split needs one group of degrees");
      fwd4_tile_split<T, MM, NORM, FUSED, STORE, FAST, LT>(ro, pt, p0, np, tid, half, lane, lrow, P, st, sg, sacc,
                                                           acc);
    } else if constexpr (LT >= 0) {
      constexpr Plan PL = make_plan(LT, B);
      fwd4_groups_ct<T, NW, MM, NORM, FUSED, STORE, FAST, LT>(std::make_integer_sequence<int, PL.ng>{}, ro, pt, K,
                                                          p0, np, lane, lrow, P, st, sg, acc);
    } else {
      for (int la = 0; la <= L;) {
        const int lb = group_end(la, L, B);
        fwd4_group<T, NW, MM, NORM, false, FUSED, STORE>(ro, pt, la, lb, K, p0, np, lane, lrow, P, st, sg, acc);
        la = lb;
      }
    }
    if constexpr (FUSED) {
      if constexpr (DS == 2) acc += sacc[lane];
      if (half == 0 && r > 0 && p < np) static_cast<T*>(P.gxyz)[(p0 + p) * 3 + (r - 1)] = acc;
    }
  };
  auto load_point = [&](int64_t i, T& x, T& y, T& z) {
    const T* q = xyz + i * 3;
    x = q[0];
    y = q[1];
    z = q[2];
  };

  constexpr bool kFast = quad_has_fast<T, LT>();
  const bool aligned = aligned16(P.Y) && (!STORE || aligned16(P.dY)) && (!FUSED || aligned16(P.gY));
  const int64_t slot = xcd_slot(blockIdx.x, gridDim.x);  // first tile of this block
  if (kFast && aligned) {
    const int64_t nfull = P.n / PT;
    if (slot < nfull) {
      T nx, ny, nz;
      load_point(slot * PT + p, nx, ny, nz);
      for (int64_t tile = slot; tile < nfull; tile += gridDim.x) {
        const T x = nx, y = ny, z = nz;
        // next full tile (clamped, so the load is unconditional)
        const int64_t nt = tile + gridDim.x < nfull ? tile + gridDim.x : tile;
        load_point(nt * PT + p, nx, ny, nz);
        tile_body(tile, x, y, z, std::integral_constant<bool, kFast>{});
      }
    }
    if (P.n % PT != 0 && nfull % gridDim.x == slot) {
      T x = T(0), y = T(0), z = T(0);
      if (nfull * PT + p < P.n) load_point(nfull * PT + p, x, y, z);
      tile_body(nfull, x, y, z, std::false_type{});
    }
  } else {
    for (int64_t tile = slot; tile * PT < P.n; tile += gridDim.x) {
      T x = T(0), y = T(0), z = T(0);
      if (tile * PT + p < P.n) load_point(tile * PT + p, x, y, z);
      tile_body(tile, x, y, z, std::false_type{});
    }
  }
}

}  // namespace sph
