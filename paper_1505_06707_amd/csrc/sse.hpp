// State, arguments and device helpers shared by the stationary solver's 2D
// and 3D line kernels (batched COCG over energies, Sec. III).
#pragma once
#include "cx.hpp"
#include "line_fft.hpp"
#include "internal.hpp"

namespace sofft {

enum CocgState : int {
  kActive = 0,     // iterating
  kCheck = 1,      // recurrence residual below rtol: true residual pending
  kDone = 2,       // true residual below rtol
  kMaxit = 3,      // iteration limit reached
  kBreakdown = 4,  // rho or p^T A p vanished twice in a row
};

// Plain COCG restarts from the true residual after this many iterations
// without a new minimum of ||r||.  On the 512^2 TFECS workload (2000-6300
// iterations per energy) single energies otherwise stalled near 1e-6..1e-5;
// with 2000 the window is reached only by those, whereas 500 and 1000 also
// restarted (and slowed) healthy energies.
constexpr int kStallIters = 2000;
// Restarts from the true residual after which an energy stops as not converged.
constexpr int kMaxRestarts = 8;

struct CocgScalars {
  cx<double> rho, alpha, beta;
  double rr, ff, true_res;
  int state, iters, first, restarts;
  // flexible COCG with the learned correction
  double best_rr;
  int since, fell_back, fb_pending, pad_;
};

struct SseArgs {
  int nx, ny, nE;
  int nz;                      // 1 on 2D grids
  size_t vec;                  // n_x n_y n_z
  cx<double>* x;               // solution (caller's buffer)
  cx<double>* r;
  cx<double>* p;
  cx<double>* w;
  cx<double>* z;
  cx<double>* s;               // preconditioner spectrum; also w1 of A p
  const cx<double>* f;
  int f_per_energy;
  const cx<double>* V;         // U on the grid, [n_z][n_y][n_x]
  const double* E;             // [nE]
  const double* eta;           // [nE] shift of the preconditioner's divisor (K - E - i eta), or null
  // banded ECS eigen-preconditioner (Eq. PreconFFT_ECS) instead of Eq. PreconFFT when banded = 1;
  // per axis the tables of ensure_bands (x: rows of the grid, y: columns)
  int banded;
  const cx<double>* bx_lam;
  const cx<double>* bx_xr;
  const cx<double>* bx_xc;
  const int* bx_start;
  const int* bx_width;
  const cx<double>* by_lam;
  const cx<double>* by_xr;
  const cx<double>* by_xc;
  const int* by_start;
  const int* by_width;
  const cx<double>* bz_lam;    // z axis (3D grids)
  const cx<double>* bz_xr;
  const cx<double>* bz_xc;
  const int* bz_start;
  const int* bz_width;
  CocgScalars* sc;             // [nE]
  double* part_rr;             // [nE][nblk_row]
  cx<double>* part_rz;         // [nE][nblk_row]
  cx<double>* part_pw;         // [nE][nblk_col]
  int nblk_row, nblk_col;      // partial sums per energy: stride of the arrays above
  int nred_row, nred_col;      // leading partials that the scalar steps add (the 3D passes reduce first)
  const cx<double>* twx;       // FFT stage twiddles along x and y
  const cx<double>* twy;
  const cx<double>* twz;
  double Lx, Ly, Lz;
  int j0x, mx, j0y, my, j0z, mz;   // ECS strips
  const cx<double>* cx_strip;  // [C_{j,j-1} | C_{j,j} | C_{j,j+1}] on the x-strip
  const cx<double>* cy_strip;
  const cx<double>* cz_strip;
  int lds_line_x, lds_line_y;
  // learned correction (flexible COCG): off when learned = 0
  int learned, patience;
  cx<double>* part_rzo;        // [nE][nblk_row]: r^T z_old
  int* active;                 // [nE]: energies the network corrects this round
  double* lp_scale;            // [nE]: rms of r
  double* E_dev;               // [nE] workspace copies of the energies and shifts
  double* eta_dev;
};

enum RowMode : int { kRowIter = 0, kRowTrue = 1 };          // K1: input p (updated) or x
enum UpdMode : int { kUpdIter = 0, kUpdInit = 1, kUpdTrue = 2, kUpdCopy = 3 };

__device__ __forceinline__ double kval(int e, int n, double L) {
  const int m = e < n / 2 ? e : e - n;
  return 6.283185307179586476925286766559 * double(m) / L;
}

__device__ __forceinline__ cx<double> shfl_xor(cx<double> v, int mask) {
  return {__shfl_xor(v.re, mask), __shfl_xor(v.im, mask)};
}

// Sum over the block in a fixed order (wavefront butterflies, then the
// wavefront sums in index order); result valid in thread 0.  red: LDS
// scratch of blockDim.x/64 elements.  Contains block barriers.
__device__ __forceinline__ cx<double> block_sum(cx<double> v, cx<double>* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = v + shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  cx<double> acc{0.0, 0.0};
  if (threadIdx.x == 0)
    for (int w = 0; w < int(blockDim.x >> 6); ++w) acc = acc + red[w];
  return acc;
}

__device__ __forceinline__ double cabs2(cx<double> v) { return v.re * v.re + v.im * v.im; }

__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// C applied on the strip of a line held in LDS (plain layout): element e's
// row of C times the line, zero off the strip.
__device__ __forceinline__ cx<double> c_apply(const LineLDS<double>& L, int e, int n, int j0, int m,
                                              const cx<double>* cs) {
  int p = e - j0;
  if (p < 0) p += n;
  if (p >= m) return {0.0, 0.0};
  const int em = e == 0 ? n - 1 : e - 1, ep = e + 1 == n ? 0 : e + 1;
  return cmul(cs[p], L[em]) + cmul(cs[m + p], L[e]) + cmul(cs[2 * m + p], L[ep]);
}

// Block-diagonal multiply along a line in Fourier space (Eq. PreconFFT_ECS):
// v[n] <- sum_{i < width[n]} coef[i * N + n] v[start[n] + i], the line held
// as v[s] = element t + TPL s (natural FFT index order) and passed through the
// LDS view L.  Every thread of the block calls it (block barriers).
template <int N>
__device__ __forceinline__ void band_apply(cx<double> (&v)[Shape<N>::P], const LineLDS<double>& L, int t,
                                           const cx<double>* __restrict__ coef, const int* __restrict__ start,
                                           const int* __restrict__ width) {
  constexpr int P = Shape<N>::P, TPL = N / P;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < P; ++s) L[t + TPL * s] = v[s];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int n = t + TPL * s, st = start[n], w = width[n];
    cx<double> acc{0.0, 0.0};
    // four entries per round, loads issued together (w <= 19: at most 5 rounds)
    for (int i0 = 0; i0 < w; i0 += 4) {
      cx<double> c[4], x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = min(i0 + j, w - 1);
        c[j] = coef[size_t(i) * N + n];
        x[j] = L[st + i];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (i0 + j < w) acc = cfma(acc, c[j], x[j]);
    }
    v[s] = acc;
  }
  __syncthreads();
}

// The solver's passes, in the order of one COCG iteration (the 3D launcher
// maps each onto its own sequence of line passes).
enum SseKernel { kK1, kK2, kK4, kK5, kK6 };

using SseLauncher = sofft_status (*)(SseKernel, const SseArgs&, int, int, hipStream_t, Timing&);

// 3D launcher for an nx x ny x nz grid, or null when there are no kernels for it.
SseLauncher sse3_launcher(int64_t nx, int64_t ny, int64_t nz);
// Blocks per energy of the 3D x passes (nbr) and z pass (nbc): the partial sums they write.
void sse3_blocks(int64_t nx, int64_t ny, int64_t nz, int* nbr, int* nbc);

// 1D grids (sse1d.hip): one workgroup per energy runs the whole solve.  mode 0
// solves; mode 1 writes A f and mode 2 P^-1 f to x_out (one energy).
size_t sse1_solver_bytes(int nE);
bool sse1_supported(int64_t n);
sofft_status sse1_run(Plan& p, int mode, const void* f, int f_per_energy, const double* E_host, int nE, double field,
                      void* x_out, double rtol, int maxit, sofft_solve_stats* stats, hipStream_t s,
                      const double* eta_host, int banded);

}  // namespace sofft
