// Double backward: for v = dL'/d(gxyz),
//   ggY[i,k]   = sum_a v[i,a] dY[i,a,k]
//   gxyz2[i,b] = sum_k gY[i,k] sum_a v[i,a] d2Y[i,k]/(dx_a dx_b)
// One lane per point, 64-point tiles.  Nothing of the Hessian reaches memory:
// for every column the lane forms the Hessian-vector product H_k v in
// registers from three consecutive rows of the folded polynomials and
// accumulates gY_k H_k v.
//
// Second derivatives by applying Eq. iter-deri twice:
//   H(Qt) v = ( Tm vx + x W, Tm vy + y W, W1 rho + W0 vz ),
//     rho = x vx + y vy,  W = W2 rho + W1 vz,
//     Tm = gxy Qt_{l-1}^{m+1}, W2 = h2 Qt_{l-2}^{m+2}, W1 = h1 Qt_{l-2}^{m+1},
//     W0 = h0 Qt_{l-2}^m;
//   grad c_m = m (c_{m-1}, -s_{m-1}, 0),  grad s_m = m (s_{m-1}, c_{m-1}, 0),
//   H(c_m) = m(m-1) [[c_{m-2}, -s_{m-2}], [-s_{m-2}, -c_{m-2}]] (x-y block),
//   H(s_m) = m(m-1) [[s_{m-2},  c_{m-2}], [ c_{m-2}, -s_{m-2}]],
// and the product rule H(Qt t) v = t H(Qt) v + grad Qt (grad t . v)
//   + grad t (grad Qt . v) + Qt H(t) v.
// Normalised harmonics Y(x) = Yt(x/r): with u = x/r, g = grad Yt(u),
//   grad Y = (g - l Yt u) / r,
//   H Y v = [ H Yt v - l (g (u.v) + u (g.v)) - l Yt v + l(l+2) Yt u (u.v) ] / r^2.
#pragma once

#include "sph_device.hpp"
#include "sph_launch.hpp"

namespace sph {

// Per-point LDS budget: one group of degrees up to l_max = 12 (float) or 8
// (double), a 64-row tile of about 44 KB whose rows are contiguous in global
// memory.
template <typename T>
inline constexpr int kDbwdBudget = 172;
template <>
inline constexpr int kDbwdBudget<double> = 86;

template <typename T>
struct DbwdAcc {
  T hx, hy, hz;  // sum_k gY_k H_k v (at the evaluation point)
};

template <typename T, int MM, bool NORM>
__device__ __forceinline__ void dbwd_group(const Point<T>& pt, T vx, T vy, T vz, int la, int lb,
                                           int kb, int S, T* st, bool write_gg, DbwdAcc<T>& A,
                                           int lane) {
  const CoefTable<T>& C = coef<T>();
  constexpr T kIS2 = T(kInvSqrt2d);
  const T ex = pt.ex, ey = pt.ey, ez = pt.ez;
  const T rho = ex * vx + ey * vy;
  const T uv = rho + ez * vz;  // u.v (normalised: ex = u)
  // Terms of order m that do not depend on the degree, tabulated once per
  // point for buckets up to m = 12 (a few dozen registers):
  //   c_m, s_m;  m c_{m-1}, m s_{m-1} (gradients of c_m, s_m);
  //   tv = grad(c_m).v, grad(s_m).v;  hA, hB with H(c_m) v = (hA, -hB),
  //   H(s_m) v = (hB, hA)  (m(m-1) times the rotated (c_{m-2}, s_{m-2})).
  constexpr bool kTab = MM <= 12;
  constexpr int MT = kTab ? MM + 1 : 1;
  T tc[MT], ts[MT], tmc[MT], tms[MT], tvc[MT], tvs[MT], thA[MT], thB[MT];
  if constexpr (kTab) {
    T s2 = T(0), c2 = T(0), s1 = T(0), c1 = T(1), s0 = T(0), c0 = T(1);
#pragma unroll
    for (int m = 0; m <= MM; ++m) {
      if (m > 0) {
        const T sn = ex * s0 + ey * c0;
        const T cn = ex * c0 - ey * s0;
        s2 = s1;
        c2 = c1;
        s1 = s0;
        c1 = c0;
        s0 = sn;
        c0 = cn;
      }
      const T fm = T(m), fmm = T(m * (m - 1));
      tc[m] = c0;
      ts[m] = s0;
      tmc[m] = fm * c1;
      tms[m] = fm * s1;
      tvc[m] = tmc[m] * vx - tms[m] * vy;
      tvs[m] = tms[m] * vx + tmc[m] * vy;
      thA[m] = fmm * (c2 * vx - s2 * vy);
      thB[m] = fmm * (s2 * vx + c2 * vy);
    }
  }
  T pp[MM + 3], prev[MM + 3], cur[MM + 3];
  q_row_rt<T, MM>(la - 2, ez, pt.rxy2, pp);
  q_row_rt<T, MM>(la - 1, ez, pt.rxy2, prev);
  T* row = st + lane * S - kb;
#pragma unroll 1
  for (int l = la; l < lb; ++l) {
    q_row_rt<T, MM>(l, ez, pt.rxy2, cur);
    const int k0 = l * l + l;
    T Sgv = T(0), Sgx = T(0), Sgy = T(0), Sgz = T(0), Sy = T(0);
    const T luv = T(l) * uv;  // normalised: grad Y . v = (grad Yt . v - l (u.v) Yt) / r
    auto process = [&](int k, T Yt, T gx, T gy, T gz, T gv, T hx, T hy, T hz) {
      const T w = row[k];
      if (write_gg) {
        T gg = gv;
        if constexpr (NORM) gg = (gv - luv * Yt) * pt.inv_r;
        row[k] = gg;
      }
      A.hx += w * hx;
      A.hy += w * hy;
      A.hz += w * hz;
      if constexpr (NORM) {
        Sgv += w * gv;
        Sgx += w * gx;
        Sgy += w * gy;
        Sgz += w * gz;
        Sy += w * Yt;
      }
    };
    T s2 = T(0), c2 = T(0);  // s_{m-2}, c_{m-2}
    T s1 = T(0), c1 = T(1);  // s_{m-1}, c_{m-1}
    T s0 = T(0), c0 = T(1);  // s_m, c_m
#pragma unroll
    for (int m = 0; m <= MM; ++m) {
      if (m > l) continue;  // no early exit: keeps the loop fully unrolled
      if (!kTab && m > 0) {
        const T sn = ex * s0 + ey * c0;
        const T cn = ex * c0 - ey * s0;
        s2 = s1;
        c2 = c1;
        s1 = s0;
        c1 = c0;
        s0 = sn;
        c0 = cn;
      }
      const T q = cur[m];
      const T Tm = (m <= l - 2) ? C.gxy[l][m] * prev[m + 1] : T(0);
      const T Cz = (m <= l - 1) ? C.gz[l][m] * prev[m] : T(0);
      const T W2 = (m <= l - 4) ? C.h2[l][m] * pp[m + 2] : T(0);
      const T W1 = (m <= l - 3) ? C.h1[l][m] * pp[m + 1] : T(0);
      const T W0 = (m <= l - 2) ? C.h0[l][m] * pp[m] : T(0);
      const T Qx = ex * Tm, Qy = ey * Tm;  // grad Qt = (Qx, Qy, Cz)
      const T W = W2 * rho + W1 * vz;
      const T Hx = Tm * vx + ex * W;  // H(Qt) v
      const T Hy = Tm * vy + ey * W;
      const T Hz = W1 * rho + W0 * vz;
      const T gQv = Tm * rho + Cz * vz;  // grad Qt . v
      if (m == 0) {
        process(k0, q * kIS2, Qx * kIS2, Qy * kIS2, Cz * kIS2, gQv * kIS2, Hx * kIS2,
                Hy * kIS2, Hz * kIS2);
      } else if constexpr (kTab) {
        // The columns k0 + m (t = c_m, grad t = (mc, -ms), H(t) v = (hA, -hB))
        // and k0 - m (t = s_m, grad t = (ms, mc), H(t) v = (hB, hA)) of one
        // order, taken together: everything accumulated is linear in their
        // weights wp, wm, so the pair folds into P = wp c + wm s and five
        // like combinations before it meets the row's Hessian terms.
        const int mt = kTab ? m : 0;
        const T c = tc[mt], sm = ts[mt], mc = tmc[mt], ms = tms[mt];
        const T hA = thA[mt], hB = thB[mt], tvp = tvc[mt], tvm = tvs[mt];
        const int kp = k0 + m, km = k0 - m;
        const T wp = row[kp], wm = row[km];
        if (write_gg) {  // grad Y . v of each column
          T ggp = c * gQv + q * tvp, ggm = sm * gQv + q * tvm;
          if constexpr (NORM) {
            ggp = (ggp - luv * (q * c)) * pt.inv_r;
            ggm = (ggm - luv * (q * sm)) * pt.inv_r;
          }
          row[kp] = ggp;
          row[km] = ggm;
        }
        const T P = wp * c + wm * sm;
        const T Pt = wp * tvp + wm * tvm;
        const T Pm = wp * mc + wm * ms;
        const T Pn = wm * mc - wp * ms;
        const T Ph = wp * hA + wm * hB;
        const T Pk = wm * hA - wp * hB;
        A.hx += Hx * P + Qx * Pt + gQv * Pm + q * Ph;
        A.hy += Hy * P + Qy * Pt + gQv * Pn + q * Pk;
        A.hz += Hz * P + Cz * Pt;
        if constexpr (NORM) {
          Sgx += Qx * P + q * Pm;
          Sgy += Qy * P + q * Pn;
          Sgz += Cz * P;
          Sgv += gQv * P + q * Pt;
          Sy += q * P;
        }
      } else {
        const T fm = T(m);
        const T fmm = T(m * (m - 1));
        {  // +m: t = c_m
          const T tx = fm * c1, ty = -fm * s1;  // grad c_m
          const T tv = tx * vx + ty * vy;
          const T htx = fmm * (c2 * vx - s2 * vy);
          const T hty = fmm * (-s2 * vx - c2 * vy);
          const T gx = c0 * Qx + q * tx;
          const T gy = c0 * Qy + q * ty;
          const T gz = c0 * Cz;
          const T gv = c0 * gQv + q * tv;
          const T hx = c0 * Hx + Qx * tv + tx * gQv + q * htx;
          const T hy = c0 * Hy + Qy * tv + ty * gQv + q * hty;
          const T hz = c0 * Hz + Cz * tv;
          process(k0 + m, q * c0, gx, gy, gz, gv, hx, hy, hz);
        }
        {  // -m: t = s_m
          const T tx = fm * s1, ty = fm * c1;  // grad s_m
          const T tv = tx * vx + ty * vy;
          const T htx = fmm * (s2 * vx + c2 * vy);
          const T hty = fmm * (c2 * vx - s2 * vy);
          const T gx = s0 * Qx + q * tx;
          const T gy = s0 * Qy + q * ty;
          const T gz = s0 * Cz;
          const T gv = s0 * gQv + q * tv;
          const T hx = s0 * Hx + Qx * tv + tx * gQv + q * htx;
          const T hy = s0 * Hy + Qy * tv + ty * gQv + q * hty;
          const T hz = s0 * Hz + Cz * tv;
          process(k0 - m, q * s0, gx, gy, gz, gv, hx, hy, hz);
        }
      }
    }
    if constexpr (NORM) {
      const T fl = T(l);
      const T a = fl * (fl + T(2)) * Sy * uv;
      A.hx += -fl * (Sgx * uv + ex * Sgv) - fl * Sy * vx + a * ex;
      A.hy += -fl * (Sgy * uv + ey * Sgv) - fl * Sy * vy + a * ey;
      A.hz += -fl * (Sgz * uv + ez * Sgv) - fl * Sy * vz + a * ez;
    }
    copy_row<T, MM>(MM, prev, pp);
    copy_row<T, MM>(MM, cur, prev);
  }
}

// MM: m-extent bucket (l_max <= MM).  Dynamic LDS: 64 * stride(L) elements.
// DS = 2 (one group of degrees only): a block of two waves on the 64-point
// tile, wave h emitting degrees [0, LS) or [LS, l_max] of every point (LS
// balances the columns; the branch is uniform per wave).  Both waves copy the
// tiles, and wave 1 hands its Hessian sums to wave 0 through 3 * 64 more LDS
// elements.  Twice the waves per CU at the same LDS for this VALU-heavy
// kernel.
template <typename T, int MM, bool NORM, int DS>
__global__ __launch_bounds__(kWave * DS) void k_dbwd(DbwdParams P) {
  constexpr int B = kDbwdBudget<T>;
  constexpr int NT = kWave * DS;
  extern __shared__ __align__(16) unsigned char smem[];
  T* st = reinterpret_cast<T*>(smem);
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int half = tid / kWave;
  const int L = P.L;
  const int K = (L + 1) * (L + 1);
  const int64_t p0 = static_cast<int64_t>(blockIdx.x) * kWave;
  if (p0 >= P.n) return;
  const int np = static_cast<int>(P.n - p0 < kWave ? P.n - p0 : kWave);
  T x = T(0), y = T(0), z = T(0), vx = T(0), vy = T(0), vz = T(0);
  if (lane < np) {
    const T* q = static_cast<const T*>(P.xyz) + (p0 + lane) * 3;
    x = q[0];
    y = q[1];
    z = q[2];
    const T* w = static_cast<const T*>(P.v) + (p0 + lane) * 3;
    vx = w[0];
    vy = w[1];
    vz = w[2];
  }
  const Point<T> pt = make_point<T, NORM>(x, y, z);
  const bool write_gg = P.ggY != nullptr;
  DbwdAcc<T> A{T(0), T(0), T(0)};
  if constexpr (DS == 2) {
    const int S = row_stride<T>(K, true);
    int LS = 1;  // smallest degree with LS^2 >= K / 2
    while (LS <= L && 2 * LS * LS < K) ++LS;
    const T* src = static_cast<const T*>(P.gY) + p0 * K;
    copy_in<NT>(st, S, src, K, K, np, tid, aligned16(src));
    __syncthreads();
    if (half == 0)
      dbwd_group<T, MM, NORM>(pt, vx, vy, vz, 0, LS, 0, S, st, write_gg, A, lane);
    else
      dbwd_group<T, MM, NORM>(pt, vx, vy, vz, LS, L + 1, 0, S, st, write_gg, A, lane);
    T* sacc = st + kWave * S;
    if (half == 1) {
      sacc[lane] = A.hx;
      sacc[kWave + lane] = A.hy;
      sacc[2 * kWave + lane] = A.hz;
    }
    __syncthreads();
    if (write_gg) {
      T* dst = static_cast<T*>(P.ggY) + p0 * K;
      copy_out<NT>(st, S, dst, K, K, np, tid, aligned16(dst));
    }
    if (half == 1) return;
    A.hx += sacc[lane];
    A.hy += sacc[kWave + lane];
    A.hz += sacc[2 * kWave + lane];
  } else {
    for (int la = 0; la <= L;) {
      const int lb = group_end(la, L, B);
      const int kb = la * la;
      const int cnt = lb * lb - kb;
      const int S = row_stride<T>(cnt, cnt == K);
      const T* src = static_cast<const T*>(P.gY) + p0 * K + kb;
      copy_in(st, S, src, K, cnt, np, lane, aligned16(src));
      __syncthreads();
      dbwd_group<T, MM, NORM>(pt, vx, vy, vz, la, lb, kb, S, st, write_gg, A, lane);
      __syncthreads();
      if (write_gg) {
        T* dst = static_cast<T*>(P.ggY) + p0 * K + kb;
        copy_out(st, S, dst, K, cnt, np, lane, aligned16(dst));
        __syncthreads();
      }
      la = lb;
    }
  }
  if (P.gxyz2 != nullptr && lane < np) {
    T s = T(1);
    if constexpr (NORM) s = pt.inv_r * pt.inv_r;
    T* g = static_cast<T*>(P.gxyz2) + (p0 + lane) * 3;
    g[0] = A.hx * s;
    g[1] = A.hy * s;
    g[2] = A.hz * s;
  }
}

}  // namespace sph
