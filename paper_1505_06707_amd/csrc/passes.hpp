// Device pieces shared by the propagation kernels of 1D, 2D (tdse.hip) and
// 3D grids (tdse3d.hip): the arguments of a line pass, the parallel cyclic
// reduction of the Crank-Nicolson factor on a strip, and state accesses.
#pragma once
#include "line_fft.hpp"

namespace sofft {

// A complex128 or complex64 state (T = double or float) is loaded from HBM,
// transformed and propagated in FP64 registers with FP64 tables, and rounded
// to T only when stored.  Line exchanges and the CN reduction go through LDS
// in FP64 (xch_t): an FP32 exchange for complex64 measured 3% faster and 3x
// the error.
template <typename T>
using xch_t = double;

template <typename T>
struct PassArgs {
  cx<T>* psi;              // the state (one run), or
  cx<T>* const* runs;      // device array of nruns states of the same shape
  const double* const* f_runs;   // device array of their f_mid rows (may be null)
  int nruns;               // runs of this shape (lines of a pass: nruns * ny or nruns * nx)
  int ntiles;              // blocks of lines over all runs
  const int64_t* step_base;      // device offset added to step (graph replays), or null
  int nx, ny;
  const cx<double>* tw;    // twiddles exp(-2 pi i u/n) of the pass axis
  const cx<double>* kin;   // kinetic phase (with 1/n) of the pass axis
  int do_pot;         // apply the potential half-step and the CN sweep
  const double* f_mid;     // f_mid of the single state
  int64_t step;
  double ht;          // dt/2
  double charge, a2;
  const double* x;        // x nodes
  const cx<double>* zx;   // z(x_j)
  const cx<double>* zy;   // z(y_j) (2D) or null
  const cx<double>* vph;  // exp(-i V0(z) dt/2) on the quadrant j < n/2 of each axis, [ny/2][nx/2]
                          // (1D: [nx/2]); node j reads entry vfold(j, n); null when V0 = 0
  int vfull;              // vph holds the whole grid, [ny][nx] (a caller's V0, no symmetry)
  const double* w;        // W of the field term f W on the grid, [ny][nx]; null: W = x
  int j0, m, levels;      // ECS strip of the pass axis
  int j0y, my;            // ECS strip of the y axis (row pass of a 2D grid)
  const cx<double>* alpha;
  const cx<double>* gamma;
  const cx<double>* binv;
  int lds_line;           // LDS elements (of xch_t<T>) reserved per line
};

// The static potential is even in x and in y on every contour (z(-x) = -z(x)
// enters V0 through z^2), so its phase table keeps one quadrant: node j of an
// axis of n nodes reads entry min(j, n - 1 - j), the mirror node on the
// negative side.
__host__ __device__ __forceinline__ int vfold(int j, int n) { return j < n - 1 - j ? j : n - 1 - j; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Crank-Nicolson solve B u = v on one line's strip by parallel cyclic
// reduction with the coefficients the host prepared (truncated once the
// couplings fall below FP64 rounding).  The host zeroes alpha where p - 2^l <
// 0 and gamma where p + 2^l >= m, so neighbours are read at clamped indices
// without branches; the next level's coefficients are fetched while the
// current level is reduced.  Levels ping-pong between [0, m) and [m, 2m); on
// entry [0, m) holds v, on exit u is in the buffer cn_result(m, levels).
//
// The positions of a line are split into groups of 64 (one per lane of a
// wavefront); k wavefronts share the line, wavefront q taking groups q, q + k,
// ... (the host keeps 2D strips at m <= 256, so at most 4 groups).  With k > 1
// the levels are separated by block barriers, with k = 1 by wavefront ones.
// G bounds the groups one wavefront takes (at most ceil(W/k) of the W groups
// a strip of a line of N points can hold); callers that know k at compile time
// pass it, which keeps the other groups' coefficients out of the registers.
constexpr int kPcrGroups = 4;
__host__ __device__ __forceinline__ int cn_result(int m, int levels) { return (levels & 1) ? 0 : m; }
template <int N>
__host__ __device__ constexpr int pcr_groups() {
  return N / 128 > 0 ? (N / 128 < kPcrGroups ? N / 128 : kPcrGroups) : 1;
}

template <typename T, int N, typename X, int G = pcr_groups<N>()>
__device__ __forceinline__ void pcr_line(const LineLDS<X>& Lw, int lane, int q, int k, const PassArgs<T>& a) {
  constexpr int W = G;
  const int m = a.m, levels = a.levels;
  const int ngroups = (m + 63) >> 6;
  int src = 0, dst = m;
  cx<double> al[W], ga[W];
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const int p = min(lane + 64 * (q + k * i), m - 1);
    if (levels > 0 && q + k * i < ngroups) {
      al[i] = a.alpha[p];
      ga[i] = a.gamma[p];
    }
  }
  for (int l = 0; l < levels; ++l) {
    const int st = 1 << l;
    const cx<double>* aln = a.alpha + size_t(l + 1 < levels ? l + 1 : l) * m;
    const cx<double>* gan = a.gamma + size_t(l + 1 < levels ? l + 1 : l) * m;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      if (q + k * i < ngroups) {   // uniform over the wavefront
        const int p0 = lane + 64 * (q + k * i), p = min(p0, m - 1);
        const cx<double> d = widen(Lw[src + p]) - cmul(al[i], widen(Lw[src + max(p - st, 0)])) -
                             cmul(ga[i], widen(Lw[src + min(p + st, m - 1)]));
        al[i] = aln[p];
        ga[i] = gan[p];
        if (p0 < m) Lw[dst + p] = narrow<X>(d);
      }
    }
    if (k > 1)
      __syncthreads();
    else
      wave_sync();
    const int tmp = src;
    src = dst;
    dst = tmp;
  }
#pragma unroll
  for (int i = 0; i < W; ++i) {
    if (q + k * i < ngroups) {
      const int p0 = lane + 64 * (q + k * i), p = min(p0, m - 1);
      const cx<double> u = cmul(a.binv[p], widen(Lw[src + p]));
      if (p0 < m) Lw[dst + p] = narrow<X>(u);
    }
  }
}

// One element of a state through a global-address-space pointer: the state
// pointer comes from a select (one state, or the batch's pointer table), so
// the compiler cannot prove it global and would emit flat accesses, which
// also count against the LDS counter that the pass's barriers wait on.
template <typename T>
__device__ __forceinline__ cx<T> gload(const cx<T>* p) {
  using V = T __attribute__((ext_vector_type(2)));
  const V v = *(const __attribute__((address_space(1))) V*)(p);
  return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void gstore(cx<T>* p, cx<T> c) {
  using V = T __attribute__((ext_vector_type(2)));
  V v;
  v.x = c.re;
  v.y = c.im;
  *(__attribute__((address_space(1))) V*)(p) = v;
}

}  // namespace sofft
