// Complex arithmetic, compile-time roots of unity and small in-register DFTs
// for the CDNA4 FFT engine.  Everything here is device code or constexpr.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace sofft {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// a + b * c
template <typename T>
__host__ __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
  return {a.re + b.re * c.re - b.im * c.im, a.im + b.re * c.im + b.im * c.re};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.im, a.re}; }

// Precision changes between the storage type of a state (HBM, LDS) and the
// FP64 arithmetic every kernel does.
template <typename T>
__host__ __device__ __forceinline__ cx<T> narrow(cx<double> v) { return {T(v.re), T(v.im)}; }
template <typename T>
__host__ __device__ __forceinline__ cx<double> widen(cx<T> v) { return {double(v.re), double(v.im)}; }

// ---------------------------------------------------------------- constexpr trig
// Taylor series on [0, pi/4] with octant symmetry: about 1 ulp in double.
namespace ct {
constexpr double kPi4 = 0.785398163397448309615660845819875721;
constexpr double sin_small(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cos_small(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi num/den, num in [0, den).
constexpr double cos2pi(long num, long den) {
  const long o = (8 * num) / den, rem = 8 * num - o * den;
  const double phi = kPi4 * double(rem) / double(den);
  const double psi = kPi4 * double(den - rem) / double(den);
  switch (o) {
    case 0: return cos_small(phi);
    case 1: return sin_small(psi);
    case 2: return -sin_small(phi);
    case 3: return -cos_small(psi);
    case 4: return -cos_small(phi);
    case 5: return -sin_small(psi);
    case 6: return sin_small(phi);
    default: return cos_small(psi);
  }
}
constexpr double sin2pi(long num, long den) {
  const long o = (8 * num) / den, rem = 8 * num - o * den;
  const double phi = kPi4 * double(rem) / double(den);
  const double psi = kPi4 * double(den - rem) / double(den);
  switch (o) {
    case 0: return sin_small(phi);
    case 1: return cos_small(psi);
    case 2: return cos_small(phi);
    case 3: return sin_small(psi);
    case 4: return -sin_small(phi);
    case 5: return -cos_small(psi);
    case 6: return -cos_small(phi);
    default: return -sin_small(psi);
  }
}
}  // namespace ct

template <int... Is, typename F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// v * exp(SIGN * 2 pi i NUM/DEN), with exact handling of the multiples of pi/2.
template <int NUM, int DEN, int SIGN, typename T>
__device__ __forceinline__ cx<T> mul_root(cx<T> v) {
  constexpr int num = ((NUM % DEN) + DEN) % DEN;
  if constexpr (num == 0) {
    return v;
  } else if constexpr (2 * num == DEN) {
    return -v;
  } else if constexpr (4 * num == DEN) {
    return SIGN > 0 ? cx<T>{-v.im, v.re} : cx<T>{v.im, -v.re};
  } else if constexpr (4 * num == 3 * DEN) {
    return SIGN > 0 ? cx<T>{v.im, -v.re} : cx<T>{-v.im, v.re};
  } else {
    constexpr T c = T(ct::cos2pi(num, DEN));
    constexpr T s = T(SIGN * ct::sin2pi(num, DEN));
    return {v.re * c - v.im * s, v.re * s + v.im * c};
  }
}

// ---------------------------------------------------------------- small DFTs
// In place, natural order in and out: a_k <- sum_n a_n exp(SIGN 2 pi i n k / R).
template <int R, int SIGN, typename T>
struct DFT;

template <int SIGN, typename T>
struct DFT<1, SIGN, T> {
  static __device__ __forceinline__ void run(cx<T>*) {}
};

template <int SIGN, typename T>
struct DFT<2, SIGN, T> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    const cx<T> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
  }
};

template <int SIGN, typename T>
struct DFT<3, SIGN, T> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    constexpr T h = T(0.866025403784438646763723170752936183);  // sqrt(3)/2
    const cx<T> s = a[1] + a[2], d = a[1] - a[2];
    const cx<T> m = a[0] - T(0.5) * s;
    const cx<T> r = (T(SIGN) * h) * times_i(d);
    a[0] = a[0] + s;
    a[1] = m + r;
    a[2] = m - r;
  }
};

template <int SIGN, typename T>
struct DFT<4, SIGN, T> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    const cx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
    const cx<T> t2 = a[1] + a[3], t3 = a[1] - a[3];
    const cx<T> r = SIGN > 0 ? times_i(t3) : -times_i(t3);
    a[0] = t0 + t2;
    a[2] = t0 - t2;
    a[1] = t1 + r;
    a[3] = t1 - r;
  }
};

// Composite R = F * M (Cooley-Tukey in registers, constant twiddles).
template <int R, int SIGN, typename T>
struct DFT {
  static constexpr int F = (R % 4 == 0) ? 4 : ((R % 2 == 0) ? 2 : 3);
  static constexpr int M = R / F;
  static_assert(F * M == R && M > 1, "unsupported radix");
  static __device__ __forceinline__ void run(cx<T>* a) {
    cx<T> sub[F][M];
    static_for<F>([&](auto fc) {
      constexpr int f = decltype(fc)::value;
#pragma unroll
      for (int m = 0; m < M; ++m) sub[f][m] = a[F * m + f];
      DFT<M, SIGN, T>::run(sub[f]);
    });
    static_for<M>([&](auto kc) {
      constexpr int k1 = decltype(kc)::value;
      cx<T> t[F];
      static_for<F>([&](auto fc) {
        constexpr int f = decltype(fc)::value;
        t[f] = mul_root<f * k1, R, SIGN>(sub[f][k1]);
      });
      DFT<F, SIGN, T>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < F; ++k2) a[k1 + M * k2] = t[k2];
    });
  }
};

}  // namespace sofft
