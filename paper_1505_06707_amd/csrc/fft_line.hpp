// Register-resident Stockham FFT along one "line" (a row or a column of the
// grid), exchanging through LDS between radix stages.
//
// A line of N points is owned by TPL = N/P threads.  Thread t holds element
// t + TPL*s in register slot s (s < P): this is the layout in which the first
// stage reads its inputs, in which the last stage leaves its outputs (natural
// order), and in which rows and columns are loaded from and stored to HBM.
// Stage r (radix R, NS = product of the earlier radices) runs P/R butterflies
// per thread; butterfly j reads elements j + m N/R, which are slots b + m P/R of
// thread t, multiplies input m by w^(m (j mod NS)), w = exp(-+2 pi i/(NS R)),
// and writes output m to element (j/NS) NS R + j mod NS + m NS.  All stages but
// the last go through LDS; the last writes back to the same slots.
//
// The forward transform is sum_j x_j exp(-2 pi i j k/N) (no scaling), the
// inverse uses exp(+2 pi i j k/N) (no scaling).
#pragma once
#include "cx.hpp"

namespace sofft {

template <int... Rs>
struct Radices {};

// Points per thread and radix sequence per supported line length.
template <int N>
struct FFTShape;
template <> struct FFTShape<16>   { static constexpr int P = 4;  using R = Radices<4, 4>; };
template <> struct FFTShape<32>   { static constexpr int P = 4;  using R = Radices<4, 4, 2>; };
template <> struct FFTShape<48>   { static constexpr int P = 12; using R = Radices<12, 4>; };
template <> struct FFTShape<64>   { static constexpr int P = 8;  using R = Radices<8, 8>; };
template <> struct FFTShape<96>   { static constexpr int P = 24; using R = Radices<24, 4>; };
template <> struct FFTShape<128>  { static constexpr int P = 8;  using R = Radices<8, 4, 4>; };
template <> struct FFTShape<192>  { static constexpr int P = 24; using R = Radices<24, 8>; };
template <> struct FFTShape<256>  { static constexpr int P = 16; using R = Radices<16, 16>; };
template <> struct FFTShape<384>  { static constexpr int P = 24; using R = Radices<12, 4, 8>; };
template <> struct FFTShape<512>  { static constexpr int P = 8;  using R = Radices<8, 8, 8>; };
template <> struct FFTShape<768>  { static constexpr int P = 24; using R = Radices<24, 8, 4>; };
template <> struct FFTShape<1024> { static constexpr int P = 16; using R = Radices<16, 16, 4>; };
template <> struct FFTShape<2048> { static constexpr int P = 16; using R = Radices<16, 16, 8>; };
template <> struct FFTShape<4096> { static constexpr int P = 16; using R = Radices<16, 16, 16>; };

// Line storage in LDS: element e of this thread's line lives at lds[base + e*es].
template <typename T>
struct LineLDS {
  cx<T>* lds;
  int base;
  int es;
  __device__ __forceinline__ cx<T>& operator[](int e) const { return lds[base + e * es]; }
};

template <typename T, int N, int P, int SIGN, int NS, int R, int... REST>
__device__ __forceinline__ void fft_stage(cx<T> (&v)[P], const LineLDS<T>& L, int t,
                                          const cx<T>* __restrict__ tw) {
  constexpr int TPL = N / P;
  constexpr int B = P / R;
  static_assert(P % R == 0, "points per thread must be a multiple of every radix");
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + TPL * b;
    const int k = j % NS;
    cx<T> a[R];
#pragma unroll
    for (int m = 0; m < R; ++m) a[m] = v[b + m * B];
    if constexpr (NS > 1) {
      constexpr int step = N / (NS * R);
#pragma unroll
      for (int m = 1; m < R; ++m) {
        const cx<T> w = tw[m * k * step];
        a[m] = SIGN < 0 ? cmul(a[m], w) : cmulc(a[m], w);
      }
    }
    DFT<R, SIGN, T>::run(a);
    if constexpr (sizeof...(REST) == 0) {
#pragma unroll
      for (int m = 0; m < R; ++m) v[b + m * B] = a[m];
    } else {
      const int o = (j / NS) * NS * R + k;
#pragma unroll
      for (int m = 0; m < R; ++m) L[o + m * NS] = a[m];
    }
  }
  if constexpr (sizeof...(REST) > 0) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = L[t + TPL * s];
    __syncthreads();
    fft_stage<T, N, P, SIGN, NS * R, REST...>(v, L, t, tw);
  }
}

template <typename T, int N, int SIGN, int P, int... Rs>
__device__ __forceinline__ void fft_line_impl(cx<T> (&v)[P], const LineLDS<T>& L, int t,
                                              const cx<T>* __restrict__ tw, Radices<Rs...>) {
  fft_stage<T, N, P, SIGN, 1, Rs...>(v, L, t, tw);
}

// In-place FFT of the line held in v (layout above).  tw[u] = exp(-2 pi i u/N).
// Every thread of the block must call this (it contains block barriers).
template <typename T, int N, int SIGN>
__device__ __forceinline__ void fft_line(cx<T> (&v)[FFTShape<N>::P], const LineLDS<T>& L, int t,
                                         const cx<T>* __restrict__ tw) {
  fft_line_impl<T, N, SIGN>(v, L, t, tw, typename FFTShape<N>::R{});
}

}  // namespace sofft
