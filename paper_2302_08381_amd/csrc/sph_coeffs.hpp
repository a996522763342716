// Compile-time coefficient tables for the folded Cartesian recursion.
//
// Notation of arXiv:2302.08381, Sec. II and App. C.  With the prefactor
// F_l^m of Eq. Flm folded into the polynomial, Qt_l^m = F_l^m Q_l^m, the
// solid harmonic of Eq. real-sh-cartesian becomes
//     r^l Y_l^m = Qt_l^{|m|} * { s_|m| (m<0), 1/sqrt2 (m=0), c_m (m>0) }.
// Every entry below is an exact function of (l, m) evaluated in double at
// compile time; the float table is the double table rounded once.
//
// Row start (App. C prefactor recursion combined with Q_l^l of Eq. iter-q):
//     Qt_0^0 = 1/sqrt(2 pi),   Qt_l^l = Qt_{l-1}^{l-1} sqrt((2l+1)/(2l)).
// Downward in m (Eq. iter-q-alt; the printed form lacks an overall minus
// sign, the form used here follows from the three-term relation of the
// Ferrers functions and is checked by the oracle tests):
//     Q_l^m = -( 2(m+1) z Q_l^{m+1} + r_xy^2 Q_l^{m+2} ) / ((l+m+1)(l-m))
// which, with a_{l,m} = sqrt((l+m+1)(l-m)) and F_l^{m+1} = -F_l^m / a_{l,m},
// folds into
//     Qt_l^m = b1 z Qt_l^{m+1} + b2 r_xy^2 Qt_l^{m+2},
//     b1 = 2(m+1)/a_{l,m},  b2 = -a_{l,m+1}/a_{l,m}.
// Derivatives (Eq. iter-deri) need prefactor ratios between rows:
//     d/dx Q_l^m = x Q_{l-1}^{m+1}      -> gxy = F_l^m / F_{l-1}^{m+1}
//                = -sqrt((2l+1)/(2l-1) (l-m)(l-m-1))
//     d/dz Q_l^m = (l+m) Q_{l-1}^m      -> gz = (l+m) F_l^m / F_{l-1}^m
//                = sqrt((2l+1)/(2l-1) (l-m)(l+m))
// and, applying Eq. iter-deri twice (second derivatives for the double
// backward):
//     d2/dx2 Q_l^m  = Q_{l-1}^{m+1} + x^2 Q_{l-2}^{m+2}
//     d2/dxdz Q_l^m = x (l+m) Q_{l-2}^{m+1}
//     d2/dz2 Q_l^m  = (l+m)(l+m-1) Q_{l-2}^m
//  -> h2 = F_l^m/F_{l-2}^{m+2}           =  sqrt((2l+1)/(2l-3) (l-m)(l-m-1)(l-m-2)(l-m-3))
//     h1 = (l+m) F_l^m/F_{l-2}^{m+1}     = -sqrt((2l+1)/(2l-3) (l-m)(l-m-1)(l-m-2)(l+m))
//     h0 = (l+m)(l+m-1) F_l^m/F_{l-2}^m  =  sqrt((2l+1)/(2l-3) (l-m)(l-m-1)(l+m)(l+m-1))
// Entries whose lower-row polynomial does not exist (m beyond the row) are 0.
#pragma once

#include <bit>
#include <cstdint>

namespace sph {

constexpr int kMaxL = 32;
constexpr int kCols = kMaxL + 3;  // m index range with two zero guards

// sqrt in double at compile time: exponent-halving start + Newton steps,
// finished by a one-ulp correction so the result is the correctly rounded root
// for the arguments used here (positive, moderate).
constexpr double csqrt(double x) {
  if (!(x > 0.0)) return 0.0;
  const uint64_t bits = std::bit_cast<uint64_t>(x);
  const int64_t e = static_cast<int64_t>((bits >> 52) & 0x7ff) - 1023;
  const int64_t he = e / 2;
  double g = std::bit_cast<double>(static_cast<uint64_t>(he + 1023) << 52);
  for (int i = 0; i < 12; ++i) g = 0.5 * (g + x / g);
  // nudge by one ulp toward the better candidate
  const double up = std::bit_cast<double>(std::bit_cast<uint64_t>(g) + 1);
  const double dn = std::bit_cast<double>(std::bit_cast<uint64_t>(g) - 1);
  auto err = [x](double c) { double d = c * c - x; return d < 0 ? -d : d; };
  if (err(up) < err(g)) g = up;
  if (err(dn) < err(g)) g = dn;
  return g;
}

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kInvSqrt2d = 0.70710678118654752440084436210484903;

template <typename T>
struct CoefTable {
  T qll[kMaxL + 1];
  T b1[kMaxL + 1][kCols];
  T b2[kMaxL + 1][kCols];
  T gxy[kMaxL + 1][kCols];
  T gz[kMaxL + 1][kCols];
  T h2[kMaxL + 1][kCols];
  T h1[kMaxL + 1][kCols];
  T h0[kMaxL + 1][kCols];
};

constexpr double a_lm(int l, int m) {  // sqrt((l+m+1)(l-m)), 0 outside 0<=m<l
  if (m < 0 || m >= l) return 0.0;
  return csqrt(double(l + m + 1) * double(l - m));
}

template <typename T>
constexpr CoefTable<T> make_coef_table() {
  CoefTable<T> t{};
  double q = csqrt(1.0 / (2.0 * kPi));
  for (int l = 0; l <= kMaxL; ++l) {
    if (l > 0) q *= csqrt(double(2 * l + 1) / double(2 * l));
    t.qll[l] = static_cast<T>(q);
    for (int m = 0; m < kCols; ++m) {
      double b1 = 0, b2 = 0, gxy = 0, gz = 0, h2 = 0, h1 = 0, h0 = 0;
      if (m < l) {
        const double a = a_lm(l, m);
        b1 = 2.0 * double(m + 1) / a;
        b2 = -a_lm(l, m + 1) / a;  // a_{l,l} = 0 for m = l-1
      }
      if (l >= 1) {
        const double rr = double(2 * l + 1) / double(2 * l - 1);
        if (m <= l - 2) gxy = -csqrt(rr * double(l - m) * double(l - m - 1));
        if (m <= l - 1) gz = csqrt(rr * double(l - m) * double(l + m));
      }
      if (l >= 2) {
        const double rr = double(2 * l + 1) / double(2 * l - 3);
        if (m <= l - 4)
          h2 = csqrt(rr * double(l - m) * double(l - m - 1) * double(l - m - 2) * double(l - m - 3));
        if (m <= l - 3)
          h1 = -csqrt(rr * double(l - m) * double(l - m - 1) * double(l - m - 2) * double(l + m));
        if (m <= l - 2)
          h0 = csqrt(rr * double(l - m) * double(l - m - 1) * double(l + m) * double(l + m - 1));
      }
      t.b1[l][m] = static_cast<T>(b1);
      t.b2[l][m] = static_cast<T>(b2);
      t.gxy[l][m] = static_cast<T>(gxy);
      t.gz[l][m] = static_cast<T>(gz);
      t.h2[l][m] = static_cast<T>(h2);
      t.h1[l][m] = static_cast<T>(h1);
      t.h0[l][m] = static_cast<T>(h0);
    }
  }
  return t;
}

}  // namespace sph
