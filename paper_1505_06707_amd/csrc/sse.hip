// Stationary equation with ECS and its FFT-preconditioned conjugate-gradient
// solve (Sec. III), batched over energies, on CDNA4.
//
// A v = F^-1 K F v + C v + (U - E) v (Eq. linsys).  In 2D the kinetic term is
// additive, T_x v + T_y v, so A v takes two passes: the row pass writes
// w1 = T_x v + C_x v + (U - E) v, the column pass adds T_y v + C_y v.  The
// preconditioner P^-1 r = F^-1 (K - E)^-1 F r (Eq. PreconFFT) is a full 2D
// transform: forward along rows (fused into the residual update), forward,
// divide and inverse along columns, inverse along rows (fused with r^T z).
//
// COCG (the conjugate-gradient recurrences with the unconjugated form u^T v,
// which keep the complex symmetry of A and P^-1), per energy e:
//   row  K1: p = z + beta p (p = z on the first iteration), w1 = row part of A p
//   col  K2: w = w1 + column part of A p, partial sums of p^T w
//        K3: alpha = rho / p^T w
//   row  K4: x += alpha p, r -= alpha w, partial ||r||^2, s = FFT_x r
//   col  K5: s = IFFT_y (FFT_y s / ((k_x^2 + k_y^2)/2 - E)) / (n_x n_y)
//   row  K6: z = IFFT_x s, partial r^T z
//        K7: convergence test on ||r||/||f||, beta = rho'/rho
// Vectors are [nE][n_y][n_x] complex128; every kernel skips energies whose
// state is not the one it works on.  Partial sums are reduced in a fixed order,
// so results do not depend on scheduling.
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "line_fft.hpp"
#include "potential.hpp"
#include "internal.hpp"
#include "sse.hpp"

namespace sofft {

// Threads per block.  Column kernels (K2, K5): at most 1024; lines of 512
// points take 512 (4 adjacent columns, 64-byte segments), see sse_col_threads.
// Row kernels (K1, K4, K6): 512.  Smaller blocks let several of them, at
// different phases, share a CU, so one block's transforms overlap another's
// loads: measured 8-10% off the 512^2 solves against 1024-thread blocks, at
// 8 waves per SIMD for the plain kernels (<= 64 VGPRs; K1 needs 72 without
// the hint, which left one 1024-thread block per CU) and 4 for the banded
// ones (about 100 VGPRs).
constexpr int kSseThreads = 1024;
constexpr int kSseRowThreads = 512;
constexpr int kSseRowWaves = 8;
constexpr int kSseBandWaves = 4;
// Launch bound of the column kernels: radix-3 shapes (P = 12) are launched
// with at most half the threads (sse_lpb), which leaves them the registers
// they need (with the 1024 bound they spilled 130-175 VGPRs).
template <int N>
constexpr int sse_col_bound() { return Shape<N>::P == 4 ? kSseThreads : kSseThreads / 2; }
// Row kernels likewise; the wave hints apply to radix-4 shapes only (the
// radix-3 ones hold 12 points per thread and spilled under them).
template <int N>
constexpr int sse_row_bound() { return Shape<N>::P == 4 ? kSseRowThreads : kSseRowThreads / 2; }
template <int N, bool BANDED>
constexpr int sse_row_waves() { return Shape<N>::P == 4 ? (BANDED ? kSseBandWaves : kSseRowWaves) : 1; }

// Blocks of the solver's line passes take one contiguous band of lines per
// XCD (workgroups go round-robin over the 8 XCDs).  Rows: 1-2% per pass
// against block b on rows lpb b ...; columns: 4% against pairs of adjacent
// column blocks per XCD slot.  Block partial sums keep their block order.
__device__ __forceinline__ int xcd_block_sse(int b, int nblk) {
  if (nblk % 8 != 0) return b;
  return (b % 8) * (nblk / 8) + b / 8;
}

// ---------------------------------------------------------------- K1: row part of A v
template <int N>
__global__ void __launch_bounds__(sse_row_bound<N>(), (sse_row_waves<N, false>())) k_sse_row_mv(SseArgs a, int want, int mode) {
  constexpr int P = Shape<N>::P, TPL = N / P;
  const int e = blockIdx.y;
  CocgScalars& sc = a.sc[e];
  if (sc.state != want) return;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* lines = reinterpret_cast<cx<double>*>(smem);
  const int lpb = blockDim.x / TPL;
  const int l = threadIdx.x / TPL, t = threadIdx.x - l * TPL;
  const int row = xcd_block_sse(blockIdx.x, gridDim.x) * lpb + l;
  const bool live = row < a.ny;
  const int crow = live ? row : 0;
  const LineLDS<double> L{lines, l * a.lds_line_x, 1};
  const size_t off = size_t(e) * a.vec + size_t(crow) * N;
  const double E = a.E[e];
  cx<double> v[P], acc[P];
  if (mode == kRowIter) {
    const cx<double> beta = sc.beta;
    const bool first = sc.first != 0;
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const size_t i = off + t + TPL * s;
      const cx<double> zz = live ? a.z[i] : cx<double>{0.0, 0.0};
      v[s] = first ? zz : cfma(zz, beta, live ? a.p[i] : cx<double>{0.0, 0.0});
      if (live) a.p[i] = v[s];
    }
  } else {
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = live ? a.x[off + t + TPL * s] : cx<double>{0.0, 0.0};
  }
  // C_x v + (U - E) v, with the line in LDS for the neighbours
#pragma unroll
  for (int s = 0; s < P; ++s) L[t + TPL * s] = v[s];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int el = t + TPL * s;
    const cx<double> u = a.V[size_t(crow) * N + el] - cx<double>{E, 0.0};
    acc[s] = cmul(u, v[s]);
    if (a.mx > 0) acc[s] = acc[s] + c_apply(L, el, N, a.j0x, a.mx, a.cx_strip);
  }
  __syncthreads();
  // T_x v = F_x^-1 (k_x^2/2) F_x v
  fft<double, N, -1>(v, L, t, a.twx);
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const double k = kval(t + TPL * s, N, a.Lx);
    v[s] = (0.5 * k * k / N) * v[s];
  }
  fft<double, N, +1>(v, L, t, a.twx);
  if (live) {
#pragma unroll
    for (int s = 0; s < P; ++s) a.s[off + t + TPL * s] = acc[s] + v[s];
  }
}


// ---------------------------------------------------------------- K2: column part of A v
// (Holding p in registers for p^T w needs 90 VGPRs.  Reading p again after the
// transforms with 6 waves per SIMD, 80 VGPRs, measured 4% slower overall.)
template <int N>
__global__ void __launch_bounds__(sse_col_bound<N>()) k_sse_col_mv(SseArgs a, int want, int mode) {
  constexpr int P = Shape<N>::P, TPL = N / P;
  const int e = blockIdx.y;
  CocgScalars& sc = a.sc[e];
  if (sc.state != want) return;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* lines = reinterpret_cast<cx<double>*>(smem);
  const int lpb = blockDim.x / TPL;
  const int c = threadIdx.x % lpb, t = threadIdx.x / lpb;
  const int cb = xcd_block_sse(blockIdx.x, gridDim.x);
  const int col = cb * lpb + c;
  const bool live = col < a.nx;
  const int ccol = live ? col : 0;
  const LineLDS<double> L{lines, c, lpb};
  const size_t base = size_t(e) * a.vec + ccol, ld = size_t(a.nx);
  const cx<double>* in = mode == kRowIter ? a.p : a.x;
  cx<double> v[P], acc[P];
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const size_t i = base + size_t(t + TPL * s) * ld;
    v[s] = live ? in[i] : cx<double>{0.0, 0.0};
    acc[s] = live ? a.s[i] : cx<double>{0.0, 0.0};
  }
  if (a.my > 0) {
#pragma unroll
    for (int s = 0; s < P; ++s) L[t + TPL * s] = v[s];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < P; ++s) acc[s] = acc[s] + c_apply(L, t + TPL * s, N, a.j0y, a.my, a.cy_strip);
    __syncthreads();
  }
  cx<double> pv[P];
#pragma unroll
  for (int s = 0; s < P; ++s) pv[s] = v[s];
  fft<double, N, -1>(v, L, t, a.twy);
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const double k = kval(t + TPL * s, N, a.Ly);
    v[s] = (0.5 * k * k / N) * v[s];
  }
  fft<double, N, +1>(v, L, t, a.twy);
  cx<double> dot{0.0, 0.0};
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const cx<double> wv = acc[s] + v[s];
    if (live) {
      a.w[base + size_t(t + TPL * s) * ld] = wv;
      dot = cfma(dot, pv[s], wv);   // p^T w, unconjugated
    }
  }
  if (mode == kRowIter) {
    const cx<double> sum = block_sum(dot, lines);
    if (threadIdx.x == 0) a.part_pw[size_t(e) * a.nblk_col + blockIdx.x] = sum;
  }
}

// ---------------------------------------------------------------- K4: update and forward row FFT
template <int N, bool BANDED>
__global__ void __launch_bounds__(sse_row_bound<N>(), (sse_row_waves<N, BANDED>())) k_sse_row_upd(SseArgs a, int want, int mode) {
  constexpr int P = Shape<N>::P, TPL = N / P;
  const int e = blockIdx.y;
  CocgScalars& sc = a.sc[e];
  if (sc.state != want) return;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* lines = reinterpret_cast<cx<double>*>(smem);
  const int lpb = blockDim.x / TPL;
  const int l = threadIdx.x / TPL, t = threadIdx.x - l * TPL;
  const int row = xcd_block_sse(blockIdx.x, gridDim.x) * lpb + l;
  const bool live = row < a.ny;
  const int crow = live ? row : 0;
  const LineLDS<double> L{lines, l * a.lds_line_x, 1};
  const size_t off = size_t(e) * a.vec + size_t(crow) * N;
  const size_t foff = (a.f_per_energy ? size_t(e) * a.vec : 0) + size_t(crow) * N;
  cx<double> v[P];
  double rr = 0.0;
  const cx<double> alpha = sc.alpha;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const size_t i = off + t + TPL * s;
    cx<double> rv{0.0, 0.0};
    if (live) {
      if (mode == kUpdIter) {
        a.x[i] = cfma(a.x[i], alpha, a.p[i]);
        rv = a.r[i] - cmul(alpha, a.w[i]);
      } else if (mode == kUpdInit) {
        a.x[i] = cx<double>{0.0, 0.0};
        rv = a.f[foff + t + TPL * s];
      } else if (mode == kUpdTrue) {
        rv = a.f[foff + t + TPL * s] - a.w[i];
      } else {
        rv = a.r[i];
      }
      if (mode != kUpdCopy) a.r[i] = rv;
      rr += rv.re * rv.re + rv.im * rv.im;
    }
    v[s] = rv;
  }
  fft<double, N, -1>(v, L, t, a.twx);
  if constexpr (BANDED) band_apply<N>(v, L, t, a.bx_xr, a.bx_start, a.bx_width);   // X_x
  if (live) {
#pragma unroll
    for (int s = 0; s < P; ++s) a.s[off + t + TPL * s] = v[s];
  }
  const cx<double> sum = block_sum(cx<double>{rr, 0.0}, lines);
  if (threadIdx.x == 0) a.part_rr[size_t(e) * a.nblk_row + blockIdx.x] = sum.re;
}

// ---------------------------------------------------------------- K5: column part of P^-1
template <int N, bool BANDED>
__global__ void __launch_bounds__(sse_col_bound<N>()) k_sse_col_prec(SseArgs a, int want) {
  constexpr int P = Shape<N>::P, TPL = N / P;
  const int e = blockIdx.y;
  if (a.sc[e].state != want) return;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* lines = reinterpret_cast<cx<double>*>(smem);
  const int lpb = blockDim.x / TPL;
  const int c = threadIdx.x % lpb, t = threadIdx.x / lpb;
  const int col = xcd_block_sse(blockIdx.x, gridDim.x) * lpb + c;
  const bool live = col < a.nx;
  const int ccol = live ? col : 0;
  const LineLDS<double> L{lines, c, lpb};
  const size_t base = size_t(e) * a.vec + ccol, ld = size_t(a.nx);
  cx<double> v[P];
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = live ? a.s[base + size_t(t + TPL * s) * ld] : cx<double>{0.0, 0.0};
  fft<double, N, -1>(v, L, t, a.twy);
  const double kx = kval(ccol, a.nx, a.Lx), E = a.E[e];
  const double eta = a.eta ? a.eta[e] : 0.0;
  const double scale = 1.0 / (double(a.nx) * double(N));
  if constexpr (BANDED) {
    // X_y, then 1/(lambda_x + lambda_y - E), then X_y^T (Eq. PreconFFT_ECS in 2D)
    band_apply<N>(v, L, t, a.by_xr, a.by_start, a.by_width);
    const cx<double> lx = a.bx_lam[ccol];
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const cx<double> d = lx + a.by_lam[t + TPL * s] - cx<double>{E, 0.0};
      const double q = scale / (d.re * d.re + d.im * d.im);
      v[s] = cmul(v[s], cx<double>{q * d.re, -q * d.im});
    }
    band_apply<N>(v, L, t, a.by_xc, a.by_start, a.by_width);
  } else if (eta == 0.0) {   // uniform over the block (the plain kernels compile without the banded branch)
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const double ky = kval(t + TPL * s, N, a.Ly);
      const double d = 0.5 * (kx * kx + ky * ky) - E;   // (K - E), as printed in Eq. PreconFFT
      v[s] = (scale / d) * v[s];
    }
  } else {
    // Shifted divisor K - E - i eta: the symbol stays even in k, so P^-1 stays
    // complex symmetric and COCG applies unchanged.
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const double ky = kval(t + TPL * s, N, a.Ly);
      const double d = 0.5 * (kx * kx + ky * ky) - E;
      const double q = scale / (d * d + eta * eta);   // 1/(d - i eta) = (d + i eta)/(d^2 + eta^2)
      v[s] = cmul(v[s], cx<double>{q * d, q * eta});
    }
  }
  fft<double, N, +1>(v, L, t, a.twy);
  if (live) {
#pragma unroll
    for (int s = 0; s < P; ++s) a.s[base + size_t(t + TPL * s) * ld] = v[s];
  }
}

// ---------------------------------------------------------------- K6: inverse row FFT and r^T z
template <int N, bool BANDED>
__global__ void __launch_bounds__(sse_row_bound<N>(), (sse_row_waves<N, BANDED>())) k_sse_row_prec(SseArgs a, int want) {
  constexpr int P = Shape<N>::P, TPL = N / P;
  const int e = blockIdx.y;
  if (a.sc[e].state != want) return;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* lines = reinterpret_cast<cx<double>*>(smem);
  const int lpb = blockDim.x / TPL;
  const int l = threadIdx.x / TPL, t = threadIdx.x - l * TPL;
  const int row = xcd_block_sse(blockIdx.x, gridDim.x) * lpb + l;
  const bool live = row < a.ny;
  const int crow = live ? row : 0;
  const LineLDS<double> L{lines, l * a.lds_line_x, 1};
  const size_t off = size_t(e) * a.vec + size_t(crow) * N;
  cx<double> v[P], rv[P];
#pragma unroll
  for (int s = 0; s < P; ++s) {
    v[s] = live ? a.s[off + t + TPL * s] : cx<double>{0.0, 0.0};
    rv[s] = live ? a.r[off + t + TPL * s] : cx<double>{0.0, 0.0};
  }
  if constexpr (BANDED) band_apply<N>(v, L, t, a.bx_xc, a.bx_start, a.bx_width);   // X_x^T
  fft<double, N, +1>(v, L, t, a.twx);
  cx<double> dot{0.0, 0.0}, dot_old{0.0, 0.0};
#pragma unroll
  for (int s = 0; s < P; ++s) {
    if (live) {
      if (a.learned) dot_old = cfma(dot_old, rv[s], a.z[off + t + TPL * s]);   // r^T z of the last iteration
      a.z[off + t + TPL * s] = v[s];
      dot = cfma(dot, rv[s], v[s]);   // r^T z, unconjugated
    }
  }
  const cx<double> sum = block_sum(dot, lines);
  if (threadIdx.x == 0) a.part_rz[size_t(e) * a.nblk_row + blockIdx.x] = sum;
  if (a.learned) {
    const cx<double> so = block_sum(dot_old, lines);
    if (threadIdx.x == 0) a.part_rzo[size_t(e) * a.nblk_row + blockIdx.x] = so;
  }
}

// ---------------------------------------------------------------- learned correction hooks
// active[e] = the network corrects z of energy e in this round; lp_scale[e] =
// rms of r from the partial sums of ||r||^2.
__global__ void k_sse_lp_gate(SseArgs a, int want) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nE) return;
  const CocgScalars& sc = a.sc[e];
  const bool on = sc.state == want && !sc.fell_back;
  double rr = 0.0;
  for (int b = 0; b < a.nred_row; ++b) rr += a.part_rr[size_t(e) * a.nblk_row + b];
  a.active[e] = (on && rr > 0.0) ? 1 : 0;
  a.lp_scale[e] = sqrt(rr / double(a.vec));
}

// part_rz[e][b] = r^T z over block b's share of the grid, for the corrected energies.
__global__ void __launch_bounds__(256) k_sse_lp_dot(SseArgs a) {
  __shared__ cx<double> red[4];
  const int e = blockIdx.y;
  if (!a.active[e]) return;
  const size_t per = (a.vec + gridDim.x - 1) / gridDim.x;
  const size_t i0 = per * blockIdx.x, i1 = i0 + per < a.vec ? i0 + per : a.vec;
  cx<double> dot{0.0, 0.0};
  for (size_t i = i0 + threadIdx.x; i < i1; i += blockDim.x)
    dot = cfma(dot, a.r[size_t(e) * a.vec + i], a.z[size_t(e) * a.vec + i]);
  const cx<double> sum = block_sum(dot, red);
  if (threadIdx.x == 0) a.part_rz[size_t(e) * a.nblk_row + blockIdx.x] = sum;
}

// ---------------------------------------------------------------- scalar steps (one thread per energy)
// After the initial r = f, z = P^-1 r: ||f||^2, rho = r^T z.
__global__ void k_sse_init(SseArgs a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nE) return;
  CocgScalars& sc = a.sc[e];
  double ff = 0.0;
  cx<double> rz{0.0, 0.0};
  for (int b = 0; b < a.nred_row; ++b) {
    ff += a.part_rr[size_t(e) * a.nblk_row + b];
    rz = rz + a.part_rz[size_t(e) * a.nblk_row + b];
  }
  sc.ff = ff;
  sc.rr = ff;
  sc.rho = rz;
  sc.first = 1;
  sc.iters = 0;
  sc.restarts = 0;
  sc.true_res = 1.0;
  sc.state = ff > 0.0 ? int(kActive) : int(kDone);
  if (ff == 0.0) sc.true_res = 0.0;
  sc.best_rr = ff;
  sc.since = 0;
  sc.fell_back = 0;
  sc.fb_pending = 0;
}

// alpha = rho / p^T w.
__global__ void k_sse_alpha(SseArgs a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nE) return;
  CocgScalars& sc = a.sc[e];
  if (sc.state != kActive) return;
  cx<double> pw{0.0, 0.0};
  for (int b = 0; b < a.nred_col; ++b) pw = pw + a.part_pw[size_t(e) * a.nblk_col + b];
  if (cabs2(pw) == 0.0) {
    sc.alpha = {0.0, 0.0};
    sc.state = kBreakdown;
    return;
  }
  sc.alpha = cdiv(sc.rho, pw);
  sc.first = 0;
}


// Convergence test on the recurrence residual, then beta and rho.
__global__ void k_sse_beta(SseArgs a, double rtol, int maxit) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nE) return;
  CocgScalars& sc = a.sc[e];
  if (sc.state != kActive) return;
  double rr = 0.0;
  cx<double> rz{0.0, 0.0};
  for (int b = 0; b < a.nred_row; ++b) {
    rr += a.part_rr[size_t(e) * a.nblk_row + b];
    rz = rz + a.part_rz[size_t(e) * a.nblk_row + b];
  }
  sc.rr = rr;
  sc.iters += 1;
  if (rr <= rtol * rtol * sc.ff) {
    sc.state = kCheck;
    return;
  }
  if (sc.iters >= maxit) {
    sc.state = kMaxit;
    sc.true_res = sqrt(rr / sc.ff);
    return;
  }
  if (cabs2(sc.rho) == 0.0) {
    sc.state = kBreakdown;
    return;
  }
  if (a.learned && !sc.fell_back) {
    // flexible beta = r^T (z - z_old) / rho; fall back to the plain
    // preconditioner (from the true residual) after `patience` iterations
    // without a new minimum of ||r||
    if (rr < sc.best_rr) {
      sc.best_rr = rr;
      sc.since = 0;
    } else if (++sc.since >= a.patience) {
      sc.fell_back = 1;
      sc.fb_pending = 1;
      sc.state = kCheck;
      return;
    }
    cx<double> rzo{0.0, 0.0};
    for (int b = 0; b < a.nred_row; ++b) rzo = rzo + a.part_rzo[size_t(e) * a.nblk_row + b];
    sc.beta = cdiv(rz - rzo, sc.rho);
    sc.rho = rz;
    return;
  }
  // A recurrence residual that has made no new minimum for kStallIters
  // iterations has stagnated (in finite precision COCG can plateau on badly
  // conditioned systems): go to the true-residual check, which restarts the
  // recurrence from r = f - A x (counted as a restart).
  if (rr < sc.best_rr) {
    sc.best_rr = rr;
    sc.since = 0;
  } else if (++sc.since >= kStallIters) {
    sc.state = kCheck;
    return;
  }
  sc.beta = cdiv(rz, sc.rho);
  sc.rho = rz;
}

// After the true residual r = f - A x and z = P^-1 r of the energies that
// passed the recurrence test: accept, or restart from the true residual.
__global__ void k_sse_true(SseArgs a, double rtol, int maxit) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nE) return;
  CocgScalars& sc = a.sc[e];
  if (sc.state != kCheck) return;
  double rr = 0.0;
  cx<double> rz{0.0, 0.0};
  for (int b = 0; b < a.nred_row; ++b) {
    rr += a.part_rr[size_t(e) * a.nblk_row + b];
    rz = rz + a.part_rz[size_t(e) * a.nblk_row + b];
  }
  sc.true_res = sqrt(rr / sc.ff);
  const int fb = sc.fb_pending;
  sc.fb_pending = 0;
  if (rr <= rtol * rtol * sc.ff) {
    sc.state = kDone;
  } else if (sc.iters >= maxit || (!fb && sc.restarts >= kMaxRestarts)) {
    sc.state = kMaxit;
  } else {
    sc.rr = rr;
    sc.rho = rz;
    sc.first = 1;
    if (!fb) sc.restarts += 1;
    sc.best_rr = rr;
    sc.since = 0;
    sc.state = kActive;
  }
}

// U on the grid: soft-core at (z_x, z_y[, z_z]) plus field * x, or a caller's V0
// (v0 non-null) and W (w non-null) in their places.  zz null: a 2D grid (nz = 1).
__global__ void k_sse_potential(cx<double>* V, int nx, int ny, int nz, const cx<double>* zx, const cx<double>* zy,
                                const cx<double>* zz, const double* x, double charge, double a2, double field,
                                const cx<double>* v0, const double* w) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= size_t(nx) * ny * nz) return;
  const int jx = int(i % nx), jy = int((i / nx) % ny), jz = int(i / (size_t(nx) * ny));
  const double fw = field * (w ? w[i] : x[jx]);
  if (v0) {
    V[i] = v0[i] + cx<double>{fw, 0.0};
    return;
  }
  cx<double> s = cmul(zx[jx], zx[jx]) + cmul(zy[jy], zy[jy]) + cx<double>{a2, 0.0};
  if (zz) s = s + cmul(zz[jz], zz[jz]);
  V[i] = potential_value(s, charge, fw);
}

// ---------------------------------------------------------------- host side

static int64_t sse_lds_elems(int64_t n) {
  switch (n) {
#define SOFFT_SSE_LDS(N) \
  case N:                \
    return fft_lds_elems<N>();
    SOFFT_SSE_LDS(16) SOFFT_SSE_LDS(32) SOFFT_SSE_LDS(48) SOFFT_SSE_LDS(64) SOFFT_SSE_LDS(96)
    SOFFT_SSE_LDS(128) SOFFT_SSE_LDS(192) SOFFT_SSE_LDS(256) SOFFT_SSE_LDS(384) SOFFT_SSE_LDS(512)
    SOFFT_SSE_LDS(768) SOFFT_SSE_LDS(1024)
#undef SOFFT_SSE_LDS
    default:
      return 2 * n;
  }
}

template <typename K>
static sofft_status sse_set_lds(K kernel, size_t bytes) {
  return bytes > 65536 ? raise_lds_limit(reinterpret_cast<const void*>(kernel), 150 * 1024) : SOFFT_OK;
}


// Lines per block: up to 1024 threads (512 for the radix-3 shapes, which use
// more registers) and within the LDS budget.
static int sse_lpb(int64_t n, int lds_line, int threads) {
  const ShapeInfo sh = shape_info(n);
  const int tpl = int(n) / sh.P;
  const int cap = sh.P == 4 ? threads : threads / 2;
  const int unit = tpl >= 64 ? 1 : 64 / tpl;   // whole wavefronts (block sums assume them)
  int lpb = tpl >= cap ? 1 : cap / tpl;
  while (lpb > unit && size_t(lpb) * lds_line * sizeof(cx<double>) > size_t(150 * 1024)) --lpb;
  lpb -= lpb % unit;
  return lpb > 0 ? lpb : unit;
}

// Column kernels: lines of 512 points in blocks of 512 threads (the 1024-point
// lines keep 1024: four columns per block either way); others up to 1024.
static int sse_col_threads(int64_t n) {
  const ShapeInfo sh = shape_info(n);
  return (sh.P == 4 && n / sh.P == 128) ? 512 : kSseThreads;
}

template <int NX, int NY>
static sofft_status sse_launch(SseKernel k, const SseArgs& a, int want, int mode, hipStream_t s, Timing& tm) {
  constexpr int TPLX = NX / Shape<NX>::P, TPLY = NY / Shape<NY>::P;
  const int lpbx = sse_lpb(NX, a.lds_line_x, kSseRowThreads);
  const int lpby = sse_lpb(NY, a.lds_line_y, sse_col_threads(NY));
  const size_t ldsx = size_t(lpbx) * a.lds_line_x * sizeof(cx<double>);
  const size_t ldsy = size_t(lpby) * a.lds_line_y * sizeof(cx<double>);
  const dim3 grow(a.nblk_row, a.nE), gcol(a.nblk_col, a.nE);
  sofft_status st = SOFFT_OK;
  switch (k) {
    case kK1:
      if ((st = sse_set_lds(k_sse_row_mv<NX>, ldsx)) != SOFFT_OK) return st;
      if ((st = tm.begin(SOFFT_KERNEL_SSE_ROW_MV, s)) != SOFFT_OK) return st;
      k_sse_row_mv<NX><<<grow, lpbx * TPLX, ldsx, s>>>(a, want, mode);
      break;
    case kK2:
      if ((st = sse_set_lds(k_sse_col_mv<NY>, ldsy)) != SOFFT_OK) return st;
      if ((st = tm.begin(SOFFT_KERNEL_SSE_COL_MV, s)) != SOFFT_OK) return st;
      k_sse_col_mv<NY><<<gcol, lpby * TPLY, ldsy, s>>>(a, want, mode);
      break;
    case kK4:
      if (a.banded) {
        if ((st = sse_set_lds(k_sse_row_upd<NX, true>, ldsx)) != SOFFT_OK) return st;
        if ((st = tm.begin(SOFFT_KERNEL_SSE_ROW_UPD, s)) != SOFFT_OK) return st;
        k_sse_row_upd<NX, true><<<grow, lpbx * TPLX, ldsx, s>>>(a, want, mode);
      } else {
        if ((st = sse_set_lds(k_sse_row_upd<NX, false>, ldsx)) != SOFFT_OK) return st;
        if ((st = tm.begin(SOFFT_KERNEL_SSE_ROW_UPD, s)) != SOFFT_OK) return st;
        k_sse_row_upd<NX, false><<<grow, lpbx * TPLX, ldsx, s>>>(a, want, mode);
      }
      break;
    case kK5:
      if (a.banded) {
        if ((st = sse_set_lds(k_sse_col_prec<NY, true>, ldsy)) != SOFFT_OK) return st;
        if ((st = tm.begin(SOFFT_KERNEL_SSE_COL_PREC, s)) != SOFFT_OK) return st;
        k_sse_col_prec<NY, true><<<gcol, lpby * TPLY, ldsy, s>>>(a, want);
      } else {
        if ((st = sse_set_lds(k_sse_col_prec<NY, false>, ldsy)) != SOFFT_OK) return st;
        if ((st = tm.begin(SOFFT_KERNEL_SSE_COL_PREC, s)) != SOFFT_OK) return st;
        k_sse_col_prec<NY, false><<<gcol, lpby * TPLY, ldsy, s>>>(a, want);
      }
      break;
    case kK6:
      if (a.banded) {
        if ((st = sse_set_lds(k_sse_row_prec<NX, true>, ldsx)) != SOFFT_OK) return st;
        if ((st = tm.begin(SOFFT_KERNEL_SSE_ROW_PREC, s)) != SOFFT_OK) return st;
        k_sse_row_prec<NX, true><<<grow, lpbx * TPLX, ldsx, s>>>(a, want);
      } else {
        if ((st = sse_set_lds(k_sse_row_prec<NX, false>, ldsx)) != SOFFT_OK) return st;
        if ((st = tm.begin(SOFFT_KERNEL_SSE_ROW_PREC, s)) != SOFFT_OK) return st;
        k_sse_row_prec<NX, false><<<grow, lpbx * TPLX, ldsx, s>>>(a, want);
      }
      break;
  }
  SOFFT_HIP_TRY(hipGetLastError());
  return tm.end(s);
}

// Square grids and the rectangular shapes the tests use; more pairs can be
// added here.
static SseLauncher sse_launcher(int64_t nx, int64_t ny) {
#define SOFFT_SSE_PAIR(X, Y) \
  if (nx == X && ny == Y) return sse_launch<X, Y>;
  SOFFT_SSE_PAIR(16, 16) SOFFT_SSE_PAIR(32, 32) SOFFT_SSE_PAIR(64, 64) SOFFT_SSE_PAIR(128, 128)
  SOFFT_SSE_PAIR(256, 256) SOFFT_SSE_PAIR(384, 384) SOFFT_SSE_PAIR(512, 512) SOFFT_SSE_PAIR(768, 768)
  SOFFT_SSE_PAIR(1024, 1024) SOFFT_SSE_PAIR(64, 32) SOFFT_SSE_PAIR(32, 64) SOFFT_SSE_PAIR(128, 96)
  SOFFT_SSE_PAIR(96, 128) SOFFT_SSE_PAIR(256, 128) SOFFT_SSE_PAIR(48, 64)
#undef SOFFT_SSE_PAIR
  return nullptr;
}

// Solver region of the workspace: five vectors per energy, U on the grid,
// partial sums, scalars, the energies and divisor shifts.
struct SseSizes {
  size_t vec, bytes_vec;
  int llx, lly, nbr, nbc;
};
static SseSizes sse_sizes(const Plan& p) {
  const Axis& X = p.ax[0];
  const Axis& Y = p.ax[1];
  SseSizes z;
  if (p.prob.ndim == 3) {
    const Axis& Z = p.ax[2];
    z.vec = size_t(X.n) * Y.n * Z.n;
    z.bytes_vec = z.vec * sizeof(cx<double>);
    z.llx = z.lly = 0;
    sse3_blocks(X.n, Y.n, Z.n, &z.nbr, &z.nbc);
    return z;
  }
  z.vec = size_t(X.n) * Y.n;
  z.bytes_vec = z.vec * sizeof(cx<double>);
  z.llx = int(std::max<int64_t>(sse_lds_elems(X.n), 64));
  z.lly = int(std::max<int64_t>(sse_lds_elems(Y.n), 64));
  const int lpr = sse_lpb(X.n, z.llx, kSseRowThreads), lpc = sse_lpb(Y.n, z.lly, sse_col_threads(Y.n));
  z.nbr = int((Y.n + lpr - 1) / lpr);
  z.nbc = int((X.n + lpc - 1) / lpc);
  return z;
}

static size_t r256(size_t b) { return (b + 255) / 256 * 256; }

size_t sse_solver_bytes(const Plan& p, int nE) {
  if (p.prob.ndim == 1) return sse1_solver_bytes(nE);
  const SseSizes z = sse_sizes(p);
  return 5 * r256(z.bytes_vec * nE) + r256(z.bytes_vec) + r256(sizeof(double) * nE * z.nbr) +
         2 * r256(sizeof(cx<double>) * nE * z.nbr) + r256(sizeof(cx<double>) * nE * z.nbc) +
         r256(sizeof(CocgScalars) * nE) + r256(sizeof(int) * nE) + 3 * r256(sizeof(double) * nE);
}

static sofft_status sse_prepare(Plan& p, int nE, double field, SseArgs& a, hipStream_t s) {
  const Axis& X = p.ax[0];
  const Axis& Y = p.ax[1];
  WsLayout WL;
  sofft_status st0 = plan_ws_check(p, nE, &WL);
  if (st0 != SOFFT_OK) return st0;
  const SseSizes z = sse_sizes(p);
  const size_t vec = z.vec, bytes_vec = z.bytes_vec;
  const int llx = z.llx, lly = z.lly, nbr = z.nbr, nbc = z.nbc;
  char* q = ws_at(p, WL.solver);
  auto take = [&](size_t b) {
    char* r = q;
    q += r256(b);
    return r;
  };
  const bool three = p.prob.ndim == 3;
  const Axis& Z = p.ax[three ? 2 : 1];
  a.nx = int(X.n);
  a.ny = int(Y.n);
  a.nz = three ? int(Z.n) : 1;
  a.nE = nE;
  a.vec = vec;
  a.r = reinterpret_cast<cx<double>*>(take(bytes_vec * nE));
  a.p = reinterpret_cast<cx<double>*>(take(bytes_vec * nE));
  a.w = reinterpret_cast<cx<double>*>(take(bytes_vec * nE));
  a.z = reinterpret_cast<cx<double>*>(take(bytes_vec * nE));
  a.s = reinterpret_cast<cx<double>*>(take(bytes_vec * nE));
  cx<double>* V = reinterpret_cast<cx<double>*>(take(bytes_vec));
  a.V = V;
  a.part_rr = reinterpret_cast<double*>(take(sizeof(double) * nE * nbr));
  a.part_rz = reinterpret_cast<cx<double>*>(take(sizeof(cx<double>) * nE * nbr));
  a.part_pw = reinterpret_cast<cx<double>*>(take(sizeof(cx<double>) * nE * nbc));
  a.sc = reinterpret_cast<CocgScalars*>(take(sizeof(CocgScalars) * nE));
  a.part_rzo = reinterpret_cast<cx<double>*>(take(sizeof(cx<double>) * nE * nbr));
  a.active = reinterpret_cast<int*>(take(sizeof(int) * nE));
  a.lp_scale = reinterpret_cast<double*>(take(sizeof(double) * nE));
  a.E_dev = reinterpret_cast<double*>(take(sizeof(double) * nE));
  a.eta_dev = reinterpret_cast<double*>(take(sizeof(double) * nE));
  a.nblk_row = nbr;
  a.nblk_col = nbc;
  // the 3D passes reduce their partials into the first slot of each energy
  a.nred_row = three ? 1 : nbr;
  a.nred_col = three ? 1 : nbc;
  a.twx = static_cast<const cx<double>*>(X.tw64.p);
  a.twy = static_cast<const cx<double>*>(Y.tw64.p);
  a.Lx = X.L;
  a.Ly = Y.L;
  a.j0x = int(X.j0);
  a.mx = int(X.m);
  a.j0y = int(Y.j0);
  a.my = int(Y.m);
  a.cx_strip = static_cast<const cx<double>*>(X.cstrip64.p);
  a.cy_strip = static_cast<const cx<double>*>(Y.cstrip64.p);
  if (three) {
    a.twz = static_cast<const cx<double>*>(Z.tw64.p);
    a.Lz = Z.L;
    a.j0z = int(Z.j0);
    a.mz = int(Z.m);
    a.cz_strip = static_cast<const cx<double>*>(Z.cstrip64.p);
  }
  a.lds_line_x = llx;
  a.lds_line_y = lly;
  const int threads = 256;
  k_sse_potential<<<int((vec + threads - 1) / threads), threads, 0, s>>>(
      V, a.nx, a.ny, a.nz, static_cast<const cx<double>*>(X.z_dev.p), static_cast<const cx<double>*>(Y.z_dev.p),
      three ? static_cast<const cx<double>*>(Z.z_dev.p) : nullptr, static_cast<const double*>(X.x_dev.p),
      p.prob.charge, p.prob.a2, field,
      static_cast<const cx<double>*>(p.user_v0), p.user_w);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

static SseLauncher launcher_of(const Plan& p) {
  if (p.prob.ndim == 3) return sse3_launcher(p.ax[0].n, p.ax[1].n, p.ax[2].n);
  return sse_launcher(p.ax[0].n, p.ax[1].n);
}

static sofft_status sse_check_plan(const Plan& p) {
  if (p.prob.dtype != SOFFT_C128) {
    set_error("the stationary solver works on complex128 plans");
    return SOFFT_EUNSUPPORTED;
  }
  if (p.prob.ndim == 1) {
    if (sse1_supported(p.ax[0].n)) return SOFFT_OK;
    set_error("no 1D stationary-solver kernel for n = " + std::to_string(p.ax[0].n));
    return SOFFT_EUNSUPPORTED;
  }
  if (!launcher_of(p)) {
    std::string shape = std::to_string(p.ax[0].n) + " x " + std::to_string(p.ax[1].n);
    if (p.prob.ndim == 3) shape += " x " + std::to_string(p.ax[2].n);
    set_error("no stationary-solver kernels for a " + shape + " grid");
    return SOFFT_EUNSUPPORTED;
  }
  return SOFFT_OK;
}

// The tables of the banded preconditioner of every axis into the solver's arguments.
static sofft_status use_bands(Plan& p, SseArgs& a) {
  sofft_status st;
  for (int d = 0; d < p.prob.ndim; ++d)
    if ((st = ensure_bands(p.ax[d])) != SOFFT_OK) return st;
  const Axis &ax = p.ax[0], &ay = p.ax[1];
  a.banded = 1;
  a.bx_lam = static_cast<const cx<double>*>(ax.band_lam.p);
  a.bx_xr = static_cast<const cx<double>*>(ax.band_xr.p);
  a.bx_xc = static_cast<const cx<double>*>(ax.band_xc.p);
  a.bx_start = static_cast<const int*>(ax.band_start.p);
  a.bx_width = static_cast<const int*>(ax.band_width.p);
  a.by_lam = static_cast<const cx<double>*>(ay.band_lam.p);
  a.by_xr = static_cast<const cx<double>*>(ay.band_xr.p);
  a.by_xc = static_cast<const cx<double>*>(ay.band_xc.p);
  a.by_start = static_cast<const int*>(ay.band_start.p);
  a.by_width = static_cast<const int*>(ay.band_width.p);
  if (p.prob.ndim == 3) {
    const Axis& az = p.ax[2];
    a.bz_lam = static_cast<const cx<double>*>(az.band_lam.p);
    a.bz_xr = static_cast<const cx<double>*>(az.band_xr.p);
    a.bz_xc = static_cast<const cx<double>*>(az.band_xc.p);
    a.bz_start = static_cast<const int*>(az.band_start.p);
    a.bz_width = static_cast<const int*>(az.band_width.p);
  }
  return SOFFT_OK;
}

sofft_status sse_solve(Plan& p, const void* f, int f_per_energy, const double* E_host, int nE, double field,
                       void* x_out, double rtol, int maxit, sofft_solve_stats* stats, hipStream_t s, LpNet* lp,
                       int patience, const double* eta_host, int banded) {
  sofft_status st = sse_check_plan(p);
  if (st != SOFFT_OK) return st;
  if (p.prob.ndim != 2 && lp) {
    set_error("the learned correction works on 2D grids");
    return SOFFT_EUNSUPPORTED;
  }
  if (p.prob.ndim == 1)
    return sse1_run(p, 0, f, f_per_energy, E_host, nE, field, x_out, rtol, maxit, stats, s, eta_host, banded);
  SseArgs a{};
  if ((st = sse_prepare(p, nE, field, a, s)) != SOFFT_OK) return st;
  a.learned = lp ? 1 : 0;
  a.patience = patience;
  a.x = static_cast<cx<double>*>(x_out);
  a.f = static_cast<const cx<double>*>(f);
  a.f_per_energy = f_per_energy;
  // energies and shifts, in the solver region
  SOFFT_HIP_TRY(hipMemcpyAsync(a.E_dev, E_host, sizeof(double) * nE, hipMemcpyHostToDevice, s));
  a.E = a.E_dev;
  if (eta_host) {
    SOFFT_HIP_TRY(hipMemcpyAsync(a.eta_dev, eta_host, sizeof(double) * nE, hipMemcpyHostToDevice, s));
    a.eta = a.eta_dev;
  }
  if (banded && (st = use_bands(p, a)) != SOFFT_OK) return st;
  SseLauncher L = launcher_of(p);
  Timing& tm = p.timing;
  const int sb = (nE + 63) / 64;
  // learned correction of z = P^-1 r for the energies in state `want`, then r^T z
  // lp_live: some energy still iterates with the correction.  Once every
  // iterating energy has fallen back (the host sees it when it polls), the
  // hook and the r^T z_old term of the flexible beta are skipped: the gate
  // would mark no energy, and beta takes the plain form for fallen-back ones.
  bool lp_live = lp != nullptr;
  auto correct = [&](int want) -> sofft_status {
    if (!lp || !lp_live) return SOFFT_OK;
    k_sse_lp_gate<<<sb, 64, 0, s>>>(a, want);
    SOFFT_HIP_TRY(hipGetLastError());
    sofft_status q = lp_apply(*lp, a.r, a.z, nE, a.ny, a.nx, a.active, a.lp_scale, s);
    if (q != SOFFT_OK) return q;
    k_sse_lp_dot<<<dim3(a.nblk_row, nE), 256, 0, s>>>(a);
    SOFFT_HIP_TRY(hipGetLastError());
    return SOFFT_OK;
  };
  // r = f, x = 0, z = P^-1 r, rho = r^T z: run the set-up kernels on every
  // energy by marking them active first.
  std::vector<CocgScalars> init(nE);
  for (auto& c : init) {
    c = CocgScalars{};
    c.state = kActive;
  }
  SOFFT_HIP_TRY(hipMemcpyAsync(a.sc, init.data(), sizeof(CocgScalars) * nE, hipMemcpyHostToDevice, s));
  if ((st = L(kK4, a, kActive, kUpdInit, s, tm)) != SOFFT_OK) return st;
  if ((st = L(kK5, a, kActive, 0, s, tm)) != SOFFT_OK) return st;
  if ((st = L(kK6, a, kActive, 0, s, tm)) != SOFFT_OK) return st;
  if ((st = correct(kActive)) != SOFFT_OK) return st;
  k_sse_init<<<sb, 64, 0, s>>>(a);
  SOFFT_HIP_TRY(hipGetLastError());

  std::vector<CocgScalars> host(nE);
  const int poll = 4;
  for (int round = 0;; ++round) {
    // iterate until no energy is active
    for (int it = 0;; ++it) {
      if ((st = L(kK1, a, kActive, kRowIter, s, tm)) != SOFFT_OK) return st;
      if ((st = L(kK2, a, kActive, kRowIter, s, tm)) != SOFFT_OK) return st;
      k_sse_alpha<<<sb, 64, 0, s>>>(a);
      SOFFT_HIP_TRY(hipGetLastError());
      if ((st = L(kK4, a, kActive, kUpdIter, s, tm)) != SOFFT_OK) return st;
      if ((st = L(kK5, a, kActive, 0, s, tm)) != SOFFT_OK) return st;
      if ((st = L(kK6, a, kActive, 0, s, tm)) != SOFFT_OK) return st;
      if ((st = correct(kActive)) != SOFFT_OK) return st;
      k_sse_beta<<<sb, 64, 0, s>>>(a, rtol, maxit);
      SOFFT_HIP_TRY(hipGetLastError());
      if ((it + 1) % poll == 0) {
        SOFFT_HIP_TRY(hipMemcpyAsync(host.data(), a.sc, sizeof(CocgScalars) * nE, hipMemcpyDeviceToHost, s));
        SOFFT_HIP_TRY(hipStreamSynchronize(s));
        bool any = false, corrected = false;
        for (const auto& c : host) {
          any |= c.state == kActive;
          corrected |= (c.state == kActive || c.state == kCheck) && !c.fell_back;
        }
        if (lp_live && !corrected) {
          lp_live = false;
          a.learned = 0;
        }
        if (!any) break;
      }
    }
    // true residual of the energies that passed the recurrence test
    if ((st = L(kK1, a, kCheck, kRowTrue, s, tm)) != SOFFT_OK) return st;
    if ((st = L(kK2, a, kCheck, kRowTrue, s, tm)) != SOFFT_OK) return st;
    if ((st = L(kK4, a, kCheck, kUpdTrue, s, tm)) != SOFFT_OK) return st;
    if ((st = L(kK5, a, kCheck, 0, s, tm)) != SOFFT_OK) return st;
    if ((st = L(kK6, a, kCheck, 0, s, tm)) != SOFFT_OK) return st;
    if ((st = correct(kCheck)) != SOFFT_OK) return st;
    k_sse_true<<<sb, 64, 0, s>>>(a, rtol, maxit);
    SOFFT_HIP_TRY(hipGetLastError());
    SOFFT_HIP_TRY(hipMemcpyAsync(host.data(), a.sc, sizeof(CocgScalars) * nE, hipMemcpyDeviceToHost, s));
    SOFFT_HIP_TRY(hipStreamSynchronize(s));
    bool any = false;
    for (const auto& c : host) any |= c.state == kActive;
    if (!any) break;
  }
  sofft_status worst = SOFFT_OK;
  for (int e = 0; e < nE; ++e) {
    const CocgScalars& c = host[e];
    int code = SOFFT_OK;
    if (c.state == kMaxit) code = SOFFT_NOT_CONVERGED;
    if (c.state == kBreakdown) code = SOFFT_BREAKDOWN;
    if (stats) {
      stats[e].iterations = c.iters;
      stats[e].status = code;
      stats[e].rel_residual = c.state == kBreakdown ? std::sqrt(c.rr / c.ff) : c.true_res;
      stats[e].restarts = c.restarts;
      stats[e].fell_back = c.fell_back;
    }
    if (code != SOFFT_OK && worst == SOFFT_OK) worst = sofft_status(code);
  }
  return worst;
}

// Choose, per energy, the shift of the preconditioner's divisor from a set of
// candidates by short solves of the problem itself: every (energy, candidate)
// pair is one system of a batched solve limited to probe_iters iterations; a
// candidate that converges ranks by its iterations, the others after it by
// the residual they reached; breakdowns rank last; ties keep the earlier
// candidate.
sofft_status sse_tune_shift(Plan& p, const void* f, const double* E_host, int nE, double field,
                            const double* cand, int ncand, int probe_iters, double rtol, void* scratch_x,
                            double* eta_out, hipStream_t s) {
  const int n = nE * ncand;
  std::vector<double> Ex(n), ex(n);
  for (int e = 0; e < nE; ++e)
    for (int c = 0; c < ncand; ++c) {
      Ex[size_t(e) * ncand + c] = E_host[e];
      ex[size_t(e) * ncand + c] = cand[c];
    }
  std::vector<sofft_solve_stats> st(n);
  const sofft_status r = sse_solve(p, f, 0, Ex.data(), n, field, scratch_x, rtol, probe_iters, st.data(), s,
                                   nullptr, 0, ex.data());
  if (r != SOFFT_OK && r != SOFFT_NOT_CONVERGED && r != SOFFT_BREAKDOWN) return r;
  for (int e = 0; e < nE; ++e) {
    int best = 0;
    auto key = [&](int c) {
      const sofft_solve_stats& q = st[size_t(e) * ncand + c];
      if (q.status == SOFFT_OK) return std::make_pair(0, double(q.iterations));
      if (q.status == SOFFT_NOT_CONVERGED) return std::make_pair(1, q.rel_residual);
      return std::make_pair(2, 0.0);
    };
    for (int c = 1; c < ncand; ++c)
      if (key(c) < key(best)) best = c;
    eta_out[e] = cand[best];
  }
  return SOFFT_OK;
}

// w = A v (op 0) or w = P^-1 v (op 1) for one energy.
sofft_status sse_apply(Plan& p, int op, const void* v, void* w, double E, double field, hipStream_t s, double eta,
                       int banded) {
  sofft_status st = sse_check_plan(p);
  if (st != SOFFT_OK) return st;
  if (p.prob.ndim == 1)
    return sse1_run(p, op == 0 ? 1 : 2, v, 0, &E, 1, field, w, 0.0, 0, nullptr, s, eta != 0.0 ? &eta : nullptr,
                    banded);
  SseArgs a{};
  if ((st = sse_prepare(p, 1, field, a, s)) != SOFFT_OK) return st;
  SOFFT_HIP_TRY(hipMemcpyAsync(a.E_dev, &E, sizeof(double), hipMemcpyHostToDevice, s));
  a.E = a.E_dev;
  if (eta != 0.0) {
    SOFFT_HIP_TRY(hipMemcpyAsync(a.eta_dev, &eta, sizeof(double), hipMemcpyHostToDevice, s));
    a.eta = a.eta_dev;
  }
  if (banded && (st = use_bands(p, a)) != SOFFT_OK) return st;
  CocgScalars c{};
  c.state = kActive;
  SOFFT_HIP_TRY(hipMemcpyAsync(a.sc, &c, sizeof(c), hipMemcpyHostToDevice, s));
  SseLauncher L = launcher_of(p);
  const size_t bytes = a.vec * sizeof(cx<double>);
  if (op == 0) {
    a.x = const_cast<cx<double>*>(static_cast<const cx<double>*>(v));
    if ((st = L(kK1, a, kActive, kRowTrue, s, p.timing)) != SOFFT_OK) return st;
    if ((st = L(kK2, a, kActive, kRowTrue, s, p.timing)) != SOFFT_OK) return st;
    SOFFT_HIP_TRY(hipMemcpyAsync(w, a.w, bytes, hipMemcpyDeviceToDevice, s));
  } else {
    SOFFT_HIP_TRY(hipMemcpyAsync(a.r, v, bytes, hipMemcpyDeviceToDevice, s));
    if ((st = L(kK4, a, kActive, kUpdCopy, s, p.timing)) != SOFFT_OK) return st;
    if ((st = L(kK5, a, kActive, 0, s, p.timing)) != SOFFT_OK) return st;
    if ((st = L(kK6, a, kActive, 0, s, p.timing)) != SOFFT_OK) return st;
    SOFFT_HIP_TRY(hipMemcpyAsync(w, a.z, bytes, hipMemcpyDeviceToDevice, s));
  }
  return SOFFT_OK;
}

}  // namespace sofft
