// Register-resident DFTs of small 2/3/5-smooth lengths (natural order in and out).
//
// Forward: X[k] = sum_n x[n] W^{nk}, W = exp(-2 pi i / L); inverse uses W^{-nk}
// and is unnormalised.  Lengths above 5 use one Cooley-Tukey split
// L = A * B (n = B n1 + n2, k = k1 + A k2) with compile-time twiddles; the
// index permutations are free because every index is a compile-time constant.
#pragma once

#include "cx.hpp"

namespace vie {

constexpr int dft_first_factor(int L) {
  if (L % 4 == 0 && L != 4) return 4;
  if (L % 2 == 0 && L != 2) return 2;
  if (L % 3 == 0 && L != 3) return 3;
  if (L % 5 == 0 && L != 5) return 5;
  return L;
}

template <int L, bool INV>
struct DFT;

template <bool INV>
struct DFT<1, INV> {
  template <typename R>
  __host__ __device__ __forceinline__ static void run(cx<R>*) {}
};

template <bool INV>
struct DFT<2, INV> {
  template <typename R>
  __host__ __device__ __forceinline__ static void run(cx<R>* v) {
    cx<R> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <bool INV>
struct DFT<3, INV> {
  template <typename R>
  __host__ __device__ __forceinline__ static void run(cx<R>* v) {
    constexpr R h = R(0.5);
    constexpr R s = R(0.86602540378443864676372317075294);  // sin(2 pi / 3)
    cx<R> a = v[0], b = v[1], c = v[2];
    cx<R> t = b + c;
    cx<R> m = a - h * t;
    cx<R> d = s * (b - c);
    v[0] = a + t;
    // forward: X1 = m - i d, X2 = m + i d
    v[1] = INV ? m + times_i(d) : m + times_mi(d);
    v[2] = INV ? m + times_mi(d) : m + times_i(d);
  }
};

template <bool INV>
struct DFT<4, INV> {
  template <typename R>
  __host__ __device__ __forceinline__ static void run(cx<R>* v) {
    cx<R> a = v[0], b = v[1], c = v[2], d = v[3];
    cx<R> s0 = a + c, d0 = a - c, s1 = b + d, d1 = b - d;
    v[0] = s0 + s1;
    v[2] = s0 - s1;
    // forward: X1 = d0 - i d1, X3 = d0 + i d1
    v[1] = INV ? d0 + times_i(d1) : d0 + times_mi(d1);
    v[3] = INV ? d0 + times_mi(d1) : d0 + times_i(d1);
  }
};

template <bool INV>
struct DFT<5, INV> {
  template <typename R>
  __host__ __device__ __forceinline__ static void run(cx<R>* v) {
    constexpr R c1 = R(0.30901699437494742410229341718282);   // cos(2 pi/5)
    constexpr R c2 = R(-0.80901699437494742410229341718282);  // cos(4 pi/5)
    constexpr R s1 = R(0.95105651629515357211643933337938);   // sin(2 pi/5)
    constexpr R s2 = R(0.58778525229247312916870595463907);   // sin(4 pi/5)
    cx<R> a = v[0];
    cx<R> t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
    cx<R> m1 = a + c1 * t1 + c2 * t2;
    cx<R> m2 = a + c2 * t1 + c1 * t2;
    cx<R> n1 = s1 * t3 + s2 * t4;
    cx<R> n2 = s2 * t3 - s1 * t4;
    v[0] = a + t1 + t2;
    if (INV) {
      v[1] = m1 + times_i(n1);
      v[4] = m1 + times_mi(n1);
      v[2] = m2 + times_i(n2);
      v[3] = m2 + times_mi(n2);
    } else {
      v[1] = m1 + times_mi(n1);
      v[4] = m1 + times_i(n1);
      v[2] = m2 + times_mi(n2);
      v[3] = m2 + times_i(n2);
    }
  }
};

template <int L, bool INV>
struct DFT {
  static_assert(dft_first_factor(L) != L, "unsupported DFT length (must be 2/3/5-smooth)");
  template <typename R>
  __host__ __device__ __forceinline__ static void run(cx<R>* v) {
    constexpr int A = dft_first_factor(L);
    constexpr int B = L / A;
    cx<R> t[L];
    static_for<0, B>([&](auto n2) {
      cx<R> u[A];
      static_for<0, A>([&](auto n1) { u[n1] = v[B * n1 + n2]; });
      DFT<A, INV>::run(u);
      static_for<0, A>([&](auto k1) {
        t[n2 * A + k1] = twiddle_mul<L, decltype(n2)::value * decltype(k1)::value, INV>(u[k1]);
      });
    });
    static_for<0, A>([&](auto k1) {
      cx<R> u[B];
      static_for<0, B>([&](auto n2) { u[n2] = t[n2 * A + k1]; });
      DFT<B, INV>::run(u);
      static_for<0, B>([&](auto k2) { v[k1 + A * k2] = u[k2]; });
    });
  }
};

}  // namespace vie
