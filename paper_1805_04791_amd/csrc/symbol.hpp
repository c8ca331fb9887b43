// Device evaluation of the truncated-kernel transform and operator symbols,
// used by the table precompute.
//
// The free-space kernel exp(i omega r)/(4 pi r) (eq. Vw; omega = 0 is eq. Vo)
// cut off at r = R has the radial transform
//     G^(s) = (1/s) int_0^R exp(i omega r) sin(s r) dr.
// With A = (omega + s) R and B = (omega - s) R it equals
//     G^(s) = (R / (2 s)) [ (v(A) - v(B)) - i (c(A) - c(B)) ],
//     c(a) = sin(a)/a,  v(a) = 2 sin^2(a/2)/a   (c(0) = 1, v(0) = 0),
// which is regular at s = omega.  At s = 0,
//     G^(0) = int_0^R r exp(i omega r) dr = [exp(i omega R)(1 - i omega R) - 1]/omega^2,
// summed as its Taylor series in omega R below 1/2.
// Symbols (forward transform exp(-i s.x)):
//     grad div V: -s_a s_b G^;  (grad div + omega^2) V: (omega^2 delta_ab - s_a s_b) G^;
//     curl V: (i s G^) x .
#pragma once

#include "cx.hpp"

namespace vie {

// MAXWELL: 6 D entries then 3 curl entries; DIV: the 3 entries i s_b G^ (the
// symbol of div V, and of curl V as (i s G^) x)
enum { SYM_GRAD = 0, SYM_MAXWELL = 1, SYM_DIV = 2 };

__device__ __forceinline__ double sinc_dev(double a) { return a == 0.0 ? 1.0 : sin(a) / a; }
__device__ __forceinline__ double vers_dev(double a) {
  if (a == 0.0) return 0.0;
  double h = sin(0.5 * a);
  return 2.0 * h * h / a;
}

__device__ inline c128 ghat_dev(double s, double w, double R) {
  if (s == 0.0) {
    const double wR = w * R;
    if (fabs(wR) < 0.5) {
      // sum_k (i w)^k R^{k+2} / (k! (k+2))
      double tr = 1.0, ti = 0.0;  // (i w)^k / k!
      double sr = 0.0, si = 0.0;
      double Rp = R * R;
      for (int k = 0; k < 24; ++k) {
        sr += tr * Rp / (k + 2);
        si += ti * Rp / (k + 2);
        const double nr = -ti * w / (k + 1), ni = tr * w / (k + 1);
        tr = nr;
        ti = ni;
        Rp *= R;
      }
      return {sr, si};
    }
    double sn, cs;
    sincos(wR, &sn, &cs);
    // e (1 - i wR) - 1, e = cs + i sn
    const double re = cs + sn * wR - 1.0;
    const double im = sn - cs * wR;
    return {re / (w * w), im / (w * w)};
  }
  const double A = (w + s) * R, B = (w - s) * R;
  const double dr = sinc_dev(A) - sinc_dev(B);
  const double di = vers_dev(A) - vers_dev(B);
  const double f = R / (2.0 * s);
  return {f * di, -f * dr};
}

// entry e of the symbol set at frequency (sx, sy, sz)
// SYM_GRAD:    e = 0..5 -> xx, yy, zz, xy, xz, yz of -s s^T G^
// SYM_MAXWELL: e = 0..5 -> (w^2 I - s s^T) G^,  e = 6..8 -> i s_b G^
// SYM_DIV:     e = 0..2 -> i s_b G^
__device__ inline c128 symbol_entry(int set, int e, double sx, double sy, double sz, double w, double R) {
  if (set == SYM_DIV) e += 6;
  const double s = sqrt(sx * sx + sy * sy + sz * sz);
  const c128 g = ghat_dev(s, w, R);
  const double sv[3] = {sx, sy, sz};
  if (e < 6) {
    const int a = e < 3 ? e : (e == 5 ? 1 : 0);
    const int b = e < 3 ? e : (e == 3 ? 1 : 2);
    double f = -sv[a] * sv[b];
    if (set == SYM_MAXWELL && a == b) f += w * w;
    return {f * g.re, f * g.im};
  }
  const double sb = sv[e - 6];
  return {-sb * g.im, sb * g.re};  // i s_b G^
}

// is entry e of the set odd in s_axis?
__host__ __device__ inline bool symbol_odd(int e, int axis);
__host__ __device__ inline bool symbol_odd_in_set(int set, int e, int axis) {
  return symbol_odd(set == SYM_DIV ? e + 6 : e, axis);
}

__host__ __device__ inline bool symbol_odd(int e, int axis) {
  if (e < 3) return false;
  if (e < 6) {
    const int a = (e == 5 ? 1 : 0);
    const int b = (e == 3 ? 1 : 2);
    return axis == a || axis == b;
  }
  return axis == e - 6;
}

}  // namespace vie
