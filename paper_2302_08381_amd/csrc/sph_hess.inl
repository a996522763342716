// Explicit second derivatives: d2Y[i][a][b][k] = d^2 Y_k / (dx_a dx_b) at
// point i, the full symmetric 3x3 block of every column (Sec. II: the
// Cartesian recursion gives derivatives of any order by applying Eq.
// iter-deri again).
//
// Mapping: a 16-point tile per block, four lanes per point.  Lane (p, a)
// forms row a of the Hessian of every column of point p, i.e. the
// Hessian-vector product H_k e_a, with the same algebra as the double
// backward:
//   H(Qt) v = ( Tm vx + x W, Tm vy + y W, W1 rho + W0 vz ),
//     rho = x vx + y vy,  W = W2 rho + W1 vz,
//     Tm = gxy Qt_{l-1}^{m+1}, W2 = h2 Qt_{l-2}^{m+2}, W1 = h1 Qt_{l-2}^{m+1},
//     W0 = h0 Qt_{l-2}^m,
// the product rule with the order-m factor t = c_m or s_m
//   H(Qt t) v = t H(Qt) v + grad Qt (grad t . v) + grad t (grad Qt . v)
//               + Qt H(t) v,
// and, for the normalised harmonics Y(x) = Yt(u), u = x/r,
//   H Y v = [ H Yt v - l (g (u.v) + u (g.v)) - l Yt v + l(l+2) Yt u (u.v) ] / r^2
// with g = grad Yt(u).  The fourth lane of each point has no row (v = 0) and
// only helps with the stores.  Rows go into an LDS tile laid out like the
// global block [16 points][3][3][K], so the tile leaves as contiguous 16-byte
// stores.  Where the nine rows of a point exceed the per-point budget the
// degrees are taken in groups and each group's partial rows are stored.
#pragma once

#include "sph_device.hpp"
#include "sph_launch.hpp"

namespace sph {

constexpr int kHessPoints = 16;  // points per tile (four lanes each)

// Per-point LDS budget of one of the nine rows (elements): one group of
// degrees up to l_max = 8 (float) or 5 (double), a tile of about 47 KB.
template <typename T>
inline constexpr int kHessBudget = 86;
template <>
inline constexpr int kHessBudget<double> = 43;

// Degrees [la, lb) of one point's Hessian row a (v = e_a; v = 0 for the lane
// without a row) into the LDS rows at `out` (three rows of stride S, column
// k at out[k - kb]).
template <typename T, int MM, bool NORM>
__device__ __forceinline__ void hess_rows(const Point<T>& pt, T vx, T vy, T vz, bool has_row, int la,
                                          int lb, int kb, int S, T* out) {
  const CoefTable<T>& C = coef<T>();
  constexpr T kIS2 = T(kInvSqrt2d);
  const T ex = pt.ex, ey = pt.ey, ez = pt.ez;
  const T rho = ex * vx + ey * vy;
  const T uv = rho + ez * vz;  // u . v (normalised: ex = u)
  const T ir2 = pt.inv_r * pt.inv_r;
  // order-m terms tabulated once per point (buckets up to m = 12):
  //   c_m, s_m;  m c_{m-1}, m s_{m-1};  grad(c_m).v, grad(s_m).v;
  //   hA, hB with H(c_m) v = (hA, -hB), H(s_m) v = (hB, hA)
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
  T* row = out - kb;
#pragma unroll 1
  for (int l = la; l < lb; ++l) {
    q_row_rt<T, MM>(l, ez, pt.rxy2, cur);
    const int k0 = l * l + l;
    // normalised: H Y v = [h - l (g (u.v) + u (g.v)) - l Yt v + l(l+2) Yt u (u.v)] / r^2
    //                   = [h - luv g - lu (g.v) - bv Yt] / r^2 per component,
    // with the degree's luv = l (u.v), lu = l u, bv = l v - l(l+2) (u.v) u
    T luv = T(0), lux = T(0), luy = T(0), luz = T(0), bx = T(0), by = T(0), bz = T(0);
    if constexpr (NORM) {
      const T fl = T(l), A = T(l) * T(l + 2) * uv;
      luv = fl * uv;
      lux = fl * ex;
      luy = fl * ey;
      luz = fl * ez;
      bx = fl * vx - A * ex;
      by = fl * vy - A * ey;
      bz = fl * vz - A * ez;
    }
    // Yt, g = grad Yt, gv = g.v, h = H(Yt) v of column k
    auto put = [&](int k, T Yt, T gx, T gy, T gz, T gv, T hx, T hy, T hz) {
      if constexpr (NORM) {
        hx = (hx - luv * gx - lux * gv - bx * Yt) * ir2;
        hy = (hy - luv * gy - luy * gv - by * Yt) * ir2;
        hz = (hz - luv * gz - luz * gv - bz * Yt) * ir2;
      }
      if (has_row) {
        row[k] = hx;
        row[S + k] = hy;
        row[2 * S + k] = hz;
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
        put(k0, q * kIS2, Qx * kIS2, Qy * kIS2, Cz * kIS2, gQv * kIS2, Hx * kIS2, Hy * kIS2, Hz * kIS2);
      } else {
        T c, sm, mc, ms, tvp, tvm, hA, hB;
        if constexpr (kTab) {
          const int mt = kTab ? m : 0;
          c = tc[mt];
          sm = ts[mt];
          mc = tmc[mt];
          ms = tms[mt];
          tvp = tvc[mt];
          tvm = tvs[mt];
          hA = thA[mt];
          hB = thB[mt];
        } else {
          const T fm = T(m), fmm = T(m * (m - 1));
          c = c0;
          sm = s0;
          mc = fm * c1;
          ms = fm * s1;
          tvp = mc * vx - ms * vy;
          tvm = ms * vx + mc * vy;
          hA = fmm * (c2 * vx - s2 * vy);
          hB = fmm * (s2 * vx + c2 * vy);
        }
        {  // +m: t = c_m, grad t = (mc, -ms, 0), H(t) v = (hA, -hB, 0)
          const T gx = c * Qx + q * mc;
          const T gy = c * Qy - q * ms;
          const T gz = c * Cz;
          const T gv = c * gQv + q * tvp;
          const T hx = c * Hx + Qx * tvp + mc * gQv + q * hA;
          const T hy = c * Hy + Qy * tvp - ms * gQv - q * hB;
          const T hz = c * Hz + Cz * tvp;
          put(k0 + m, q * c, gx, gy, gz, gv, hx, hy, hz);
        }
        {  // -m: t = s_m, grad t = (ms, mc, 0), H(t) v = (hB, hA, 0)
          const T gx = sm * Qx + q * ms;
          const T gy = sm * Qy + q * mc;
          const T gz = sm * Cz;
          const T gv = sm * gQv + q * tvm;
          const T hx = sm * Hx + Qx * tvm + ms * gQv + q * hB;
          const T hy = sm * Hy + Qy * tvm + mc * gQv + q * hA;
          const T hz = sm * Hz + Cz * tvm;
          put(k0 - m, q * sm, gx, gy, gz, gv, hx, hy, hz);
        }
      }
    }
    copy_row<T, MM>(MM, prev, pp);
    copy_row<T, MM>(MM, cur, prev);
  }
}

// MM: m-extent bucket (l_max <= MM).  DS = 2 (one group of degrees only): a
// block of two waves on the tile, wave h forming degrees [0, LS) or
// [LS, l_max] (LS balances the columns; the branch is uniform per wave), both
// waves storing the tile.  Dynamic LDS: 16 * 9 * stride elements.
template <typename T, int MM, bool NORM, int DS>
__global__ __launch_bounds__(kWave * DS) void k_hess(HessParams P) {
  constexpr int B = kHessBudget<T>;
  constexpr int NT = kWave * DS;
  constexpr int PT = kHessPoints;
  extern __shared__ __align__(16) unsigned char smem[];
  T* st = reinterpret_cast<T*>(smem);
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int half = tid / kWave;
  const int p = lane / 4, a = lane % 4;
  const int L = P.L;
  const int K = (L + 1) * (L + 1);
  const T vx = a == 0 ? T(1) : T(0), vy = a == 1 ? T(1) : T(0), vz = a == 2 ? T(1) : T(0);
  T* d2 = static_cast<T*>(P.d2Y);
  const int64_t ntiles = (P.n + PT - 1) / PT;
  for (int64_t tile = xcd_slot(blockIdx.x, gridDim.x); tile < ntiles; tile += gridDim.x) {
    const int64_t p0 = tile * PT;
    const int np = static_cast<int>(P.n - p0 < PT ? P.n - p0 : PT);
    T x = T(0), y = T(0), z = T(0);
    if (p < np) {
      const T* q = static_cast<const T*>(P.xyz) + (p0 + p) * 3;
      x = q[0];
      y = q[1];
      z = q[2];
    }
    const Point<T> pt = make_point<T, NORM>(x, y, z);
    const bool has_row = a < 3 && p < np;
    T* dst = d2 + p0 * 9 * K;
    if constexpr (DS == 2) {
      const int S = row_stride<T>(K, true);
      int LS = 1;  // smallest degree with LS^2 >= K / 2
      while (LS <= L && 2 * LS * LS < K) ++LS;
      T* out = st + (p * 9 + a * 3) * S;
      if (half == 0)
        hess_rows<T, MM, NORM>(pt, vx, vy, vz, has_row, 0, LS, 0, S, out);
      else
        hess_rows<T, MM, NORM>(pt, vx, vy, vz, has_row, LS, L + 1, 0, S, out);
      __syncthreads();
      copy_out<NT>(st, S, dst, K, K, np * 9, tid, aligned16(dst));
      __syncthreads();
    } else {
      for (int la = 0; la <= L;) {
        const int lb = group_end(la, L, B);
        const int kb = la * la;
        const int cnt = lb * lb - kb;
        const int S = row_stride<T>(cnt, cnt == K);
        hess_rows<T, MM, NORM>(pt, vx, vy, vz, has_row, la, lb, kb, S, st + (p * 9 + a * 3) * S);
        __syncthreads();
        copy_out(st, S, dst + kb, K, cnt, np * 9, lane, aligned16(dst + kb));
        __syncthreads();
        la = lb;
      }
    }
  }
}

}  // namespace sph
