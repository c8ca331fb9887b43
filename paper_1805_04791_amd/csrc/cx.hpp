// Complex arithmetic and compile-time helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

namespace vie {

template <typename R>
struct __attribute__((aligned(2 * sizeof(R)))) cx {
  R re, im;
};

using c64 = cx<float>;
using c128 = cx<double>;

template <typename R>
__host__ __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// acc + a * b and acc - a * b as chains of fused multiply-adds (four
// instructions, where a product followed by a complex add takes six)
__host__ __device__ __forceinline__ cx<float> cmad(cx<float> a, cx<float> b, cx<float> acc) {
  return {__builtin_fmaf(a.re, b.re, __builtin_fmaf(-a.im, b.im, acc.re)),
          __builtin_fmaf(a.re, b.im, __builtin_fmaf(a.im, b.re, acc.im))};
}
__host__ __device__ __forceinline__ cx<float> cmsb(cx<float> a, cx<float> b, cx<float> acc) {
  return cmad(-a, b, acc);
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> times_mi(cx<R> a) { return {a.im, -a.re}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> czero() { return {R(0), R(0)}; }
template <typename R>
__host__ __device__ __forceinline__ R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }

// precision conversion between storage and compute types
template <typename To, typename From>
__host__ __device__ __forceinline__ cx<To> cvt(cx<From> a) { return {To(a.re), To(a.im)}; }

// ---------------------------------------------------------------------------
// compile-time loops
// ---------------------------------------------------------------------------
template <int I>
using ic = std::integral_constant<int, I>;

template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(ic<B>{});
    static_for<B + 1, E>(f);
  }
}

// ---------------------------------------------------------------------------
// compile-time cos/sin of 2*pi*j/L, exact quadrant reduction + Taylor series
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ct_sin_series(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 16; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos_series(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 16; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
// returns cos(2 pi j / L) (want_sin=false) or sin(2 pi j / L)
constexpr double ct_trig(long j, long L, bool want_sin) {
  j %= L;
  if (j < 0) j += L;
  // 2 pi j / L = q * pi/2 + phi, phi in [0, pi/2)
  long q = (4 * j) / L;
  long r = 4 * j - q * L;  // in [0, L)
  double phi = (kPi / 2.0) * double(r) / double(L);
  // use the smaller half-angle for accuracy: phi in [0, pi/4] or complementary
  double c = 0, s = 0;
  if (2 * r <= L) {
    c = ct_cos_series(phi);
    s = ct_sin_series(phi);
  } else {
    double psi = (kPi / 2.0) * double(L - r) / double(L);
    c = ct_sin_series(psi);
    s = ct_cos_series(psi);
  }
  double cc = c, ss = s;
  switch (q & 3) {
    case 0: cc = c; ss = s; break;
    case 1: cc = -s; ss = c; break;
    case 2: cc = -c; ss = -s; break;
    default: cc = s; ss = -c; break;
  }
  return want_sin ? ss : cc;
}

// multiply by W_L^J (forward, W = exp(-2 pi i / L)) or W_L^{-J} (inverse)
template <int L, int J, bool INV, typename R>
__host__ __device__ __forceinline__ cx<R> twiddle_mul(cx<R> a) {
  constexpr int j = ((J % L) + L) % L;
  if constexpr (j == 0) {
    return a;
  } else if constexpr (4 * j == L) {
    return INV ? times_i(a) : times_mi(a);
  } else if constexpr (2 * j == L) {
    return -a;
  } else if constexpr (4 * j == 3 * L) {
    return INV ? times_mi(a) : times_i(a);
  } else {
    constexpr double c = ct_trig(j, L, false);
    constexpr double s = ct_trig(j, L, true);
    // forward: (c - i s), inverse: (c + i s)
    constexpr R wr = R(c);
    constexpr R wi = INV ? R(s) : R(-s);
    return {a.re * wr - a.im * wi, a.re * wi + a.im * wr};
  }
}

}  // namespace vie
