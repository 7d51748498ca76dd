// Line geometry of the 3D passes (propagation and stationary solver):
// indexing of psi[z][y][x], block shapes, and the origin and stride of the
// lines along each axis.
#pragma once
#include "line_fft.hpp"

namespace sofft {

__host__ __device__ __forceinline__ size_t idx3(int x, int y, int z, int nx, int ny) {
  return (size_t(z) * ny + y) * nx + x;
}

// Lines per block of a kinetic pass: eight adjacent lines (128-byte segments of
// complex128 in the strided passes), more for short lines so that a block
// holds at least one wavefront.
template <int N>
constexpr int k3_lines() {
  constexpr int tpl = N / Shape<N>::P;
  return tpl * 8 >= 64 ? 8 : 64 / tpl;
}
template <int N>
constexpr int k3_threads() {
  return k3_lines<N>() * (N / Shape<N>::P);
}

// Origin (pass-axis coordinate 0) and element stride of line g.  AXIS 0: the
// rows, g = y + ny z; AXIS 1: g = x + nx z, stride nx; AXIS 2: g = x + nx y,
// stride nx ny.  Consecutive g of the strided passes are adjacent in x.
template <int AXIS>
__device__ __forceinline__ void line_origin(int g, int nx, int ny, int& lx, int& ly, int& lz, size_t& ld) {
  if constexpr (AXIS == 0) {
    lx = 0;
    ly = g % ny;
    lz = g / ny;
    ld = 1;
  } else if constexpr (AXIS == 1) {
    lx = g % nx;
    ly = 0;
    lz = g / nx;
    ld = size_t(nx);
  } else {
    lx = g % nx;
    ly = g / nx;
    lz = 0;
    ld = size_t(nx) * ny;
  }
}

template <int AXIS>
__device__ __forceinline__ void node_of(int e, int lx, int ly, int lz, int& x, int& y, int& z) {
  x = AXIS == 0 ? e : lx;
  y = AXIS == 1 ? e : ly;
  z = AXIS == 2 ? e : lz;
}

// Dispatch on a 3D line length: EXPR_N evaluated with the constant N_.
#define SOFFT_3D_SWITCH(n, EXPR_N)                       \
  switch (n) {                                           \
    case 16: { constexpr int N_ = 16; return EXPR_N; }   \
    case 32: { constexpr int N_ = 32; return EXPR_N; }   \
    case 64: { constexpr int N_ = 64; return EXPR_N; }   \
    case 128: { constexpr int N_ = 128; return EXPR_N; } \
    case 256: { constexpr int N_ = 256; return EXPR_N; } \
    case 512: { constexpr int N_ = 512; return EXPR_N; } \
    default: break;                                      \
  }

}  // namespace sofft
