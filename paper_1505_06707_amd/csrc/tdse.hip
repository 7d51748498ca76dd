// Split-operator SO-FFT + ECS time step (Sec. II) on CDNA4.
//
// 2D: one step is two HBM round trips of the state.
//   row pass    (along x): FFT_x, e^{-i k_x^2 dt/2}, IFFT_x, e^{-iU dt/2}, CN(C_x)
//   column pass (along y): CN(C_y), e^{-iU dt/2}, FFT_y, e^{-i k_y^2 dt/2}, IFFT_y
// The kinetic half-steps that close one step and open the next share a pass
// (the same diagonal in k), so the first row pass and the last column pass use
// the half-step table, and one extra column pass before and one row pass after
// the loop apply the opening/closing K_y/2 and K_x/2.
// 1D: one workgroup keeps the whole line in registers/LDS for all steps.
#include <algorithm>
#include <mutex>
#include <vector>

#include "line_fft.hpp"
#include "passes.hpp"
#include "potential.hpp"
#include "internal.hpp"

namespace sofft {

// Crank-Nicolson on the ECS strip of a line held by the whole block (1D):
// y = 2 B^-1 v - v by parallel cyclic reduction, staged in the line's LDS
// storage (buffers [0, m) and [m, 2m)).  As in pcr_line, neighbours are read at
// clamped indices (the host zeroes the coefficients that reach past the strip)
// and the next level's coefficients are fetched during the current level.
template <typename T, int N, typename X>
__device__ __forceinline__ void cn_strip(cx<double> (&v)[Shape<N>::P], const LineLDS<X>& L, int t,
                                         const PassArgs<T>& a) {
  constexpr int P = Shape<N>::P, TPL = N / P;
  constexpr int MAXPOS = P / 2;   // strip positions per thread: the host keeps m <= N/2
  const int m = a.m;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int p = strip_pos<N>(t + TPL * s, a.j0);
    if (p < m) L[p] = narrow<X>(v[s]);
  }
  cx<double> al[MAXPOS], ga[MAXPOS];
  if (a.levels > 0) {
#pragma unroll
    for (int i = 0; i < MAXPOS; ++i) {
      const int p = min(t + TPL * i, m - 1);
      al[i] = a.alpha[p];
      ga[i] = a.gamma[p];
    }
  }
  __syncthreads();
  int src = 0, dst = m;
  for (int l = 0; l < a.levels; ++l) {
    const int st = 1 << l;
    const cx<double>* aln = a.alpha + size_t(l + 1 < a.levels ? l + 1 : l) * m;
    const cx<double>* gan = a.gamma + size_t(l + 1 < a.levels ? l + 1 : l) * m;
#pragma unroll
    for (int i = 0; i < MAXPOS; ++i) {
      const int p0 = t + TPL * i, p = min(p0, m - 1);
      const cx<double> d = widen(L[src + p]) - cmul(al[i], widen(L[src + max(p - st, 0)])) -
                           cmul(ga[i], widen(L[src + min(p + st, m - 1)]));
      al[i] = aln[p];
      ga[i] = gan[p];
      if (p0 < m) L[dst + p] = narrow<X>(d);
    }
    __syncthreads();
    const int tmp = src;
    src = dst;
    dst = tmp;
  }
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int p = strip_pos<N>(t + TPL * s, a.j0);
    if (p < m) v[s] = 2.0 * cmul(a.binv[p], widen(L[src + p])) - v[s];
  }
  __syncthreads();
}

// U/2 . C . U/2 along a line whose cross coordinate is fixed (1D): outside
// the strip the two half-steps are one multiply by the squared phase; on the
// strip the phase is parked in LDS (from 2m) across the CN.
template <typename T, int N, typename X, typename PhaseFn>
__device__ __forceinline__ void pot_cn_pot(cx<double> (&v)[Shape<N>::P], const LineLDS<X>& L, int t,
                                           const PassArgs<T>& a, PhaseFn phase) {
  constexpr int P = Shape<N>::P, TPL = N / P;
  const int m = a.m;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int e = t + TPL * s;
    const cx<double> ph = phase(e);
    const int p = strip_pos<N>(e, a.j0);
    if (p < m) {
      v[s] = cmul(v[s], ph);
      L[2 * m + p] = ph;
    } else {
      v[s] = cmul(v[s], cmul(ph, ph));
    }
  }
  if (m > 0) {
    cn_strip<T, N>(v, L, t, a);
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int e = t + TPL * s;
      const int p = strip_pos<N>(e, a.j0);
      if (p < m) {
        v[s] = cmul(v[s], widen(L[2 * m + p]));
      }
    }
    __syncthreads();
  }
}

// Row blocks have 256 threads (one 1024-point row, or several shorter ones):
// independent rows do not wait at each other's barriers, measured 17% faster
// per row pass than four rows per block.  Column blocks have 1024 threads
// (four 1024-point columns: 64-byte row segments).  P = 4 shapes keep <= 96
// VGPRs (5 waves per SIMD; 6 spilled and measured slower, 4 measured 5%
// slower); P = 12 shapes (radix 3) take at most 512 threads and need more
// registers: 168 VGPRs at 3 waves per SIMD (a few spills, measured faster for
// batches of such lines than 2 waves without spills).
constexpr int kRowThreads = 256;
constexpr int kColThreads = 1024;
template <int N>
constexpr int min_waves_per_simd() {
  return Shape<N>::P == 4 ? 5 : 3;
}
// Threads per block: THREADS (P = 12 shapes at most 512, so that two waves
// per SIMD leave them 256 VGPRs), and at least one whole line.
template <int N, int THREADS>
constexpr int block_threads() {
  constexpr int cap = Shape<N>::P == 4 ? THREADS : (THREADS < 512 ? THREADS : 512);
  return N / Shape<N>::P > cap ? N / Shape<N>::P : cap;
}
// Persistent variants (a loop over tiles) hold more live registers: at most
// 512 threads per block and two waves per SIMD, i.e. 256 VGPRs.
template <int N, int THREADS, bool PERSIST>
constexpr int kernel_threads() {
  return PERSIST && block_threads<N, THREADS>() > 512 ? 512 : block_threads<N, THREADS>();
}
template <int N, bool PERSIST>
constexpr int kernel_waves() {
  return PERSIST ? 2 : min_waves_per_simd<N>();
}
// Two LDS exchange buffers per line (fft2: one barrier per exchange instead of
// two) when they fit the LDS budget at the largest block of a row or column pass.
template <int N, typename X>
constexpr int fft_buffers() {
  constexpr int lines = block_threads<N, (kRowThreads > kColThreads ? kRowThreads : kColThreads)>() / (N / Shape<N>::P);
  constexpr size_t bytes = size_t(2) * lines * fft_lds_elems<N>() * sizeof(cx<X>);
  return (N <= 1024 && bytes <= 128 * 1024) ? 2 : 1;
}

// All lines of the block; line_of(ln) gives the LDS view of line ln.  With at
// least as many wavefronts as lines (and a multiple of them) every wavefront
// works on one line, k = nwaves / lines sharing it; otherwise wavefront w
// solves lines w, w + nwaves, ... alone.  Block barriers before and after.
template <typename T, int N, typename LineOf>
__device__ __forceinline__ void cn_block(int lpb, const PassArgs<T>& a, LineOf line_of) {
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;   // whole wavefronts
  constexpr int TPL = N / Shape<N>::P;
  if constexpr (TPL >= 64) {
    // blocks of whole lines (lpb = blockDim.x / TPL): the TPL/64 wavefronts of
    // a line share its strip, each taking at most ceil(W k / TPL) groups
    constexpr int k = TPL / 64, W = pcr_groups<N>();
    pcr_line<T, N, xch_t<T>, (W + k - 1) / k>(line_of(w / k), lane, w % k, k, a);
  } else if (nw >= lpb && nw % lpb == 0) {
    const int k = nw / lpb;
    pcr_line<T, N>(line_of(w / k), lane, w % k, k, a);
  } else {
    for (int ln = w; ln < lpb; ln += nw) pcr_line<T, N>(line_of(ln), lane, 0, 1, a);
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ cx<T>* run_state(const PassArgs<T>& a, int run) {
  return a.runs ? a.runs[run] : a.psi;
}
template <typename T>
__device__ __forceinline__ const double* run_field(const PassArgs<T>& a, int run) {
  return a.runs ? (a.f_runs ? a.f_runs[run] : nullptr) : a.f_mid;
}
template <typename T>
__device__ __forceinline__ int64_t pass_step(const PassArgs<T>& a) {
  return a.step + (a.step_base ? *a.step_base : 0);
}

// The lines of a pass (rows or columns of every run, run-major) are cut into
// tiles of blockDim.x / TPL lines.  Without PERSIST block b takes tile b (the
// grid has one block per tile); with it block b loops over tiles b,
// b + gridDim.x, ... (a persistent grid sized to the resident blocks).  The
// two are separate instantiations because the loop around the transforms
// costs the one-tile kernels their register allocation (spills).
template <bool PERSIST, typename Body>
__device__ __forceinline__ void run_tiles(int ntiles, Body& body) {
  if constexpr (PERSIST) {
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
      body(tile);
      __syncthreads();   // LDS is reused by the next tile
    }
  } else {
    body(blockIdx.x);
  }
}

// One-row blocks are assigned so that each XCD runs groups of RG consecutive
// rows, 64 KiB of state (block t runs on XCD t mod 8 and takes row
// 8 RG floor(t / 8 RG) + RG (t mod 8) + floor(t/8) mod RG): the column pass that
// follows then reads each XCD's rows in 64-KiB runs.  At 1024^2 complex128
// (RG = 4) this measured 17% faster per column pass than row t on block t;
// 8 to 128 rows per group measured slower there.  Blocks of several rows
// keep the identity map.
template <int RG>
__device__ __forceinline__ int xcd_rows(int tile, int lpb, int nlines, int ntiles) {
  if (lpb != 1 || nlines % (8 * RG) != 0 || ntiles != nlines) return tile;
  return 8 * RG * (tile / (8 * RG)) + RG * (tile & 7) + (tile >> 3) % RG;
}

// Block LDS layout of the 2D passes: [line 0][line 1]...; a block holds
// blockDim.x / TPL lines of a.lds_line elements.  FFT twiddles and CN
// coefficients are read from global memory (they stay in the vector L1).
// UP: the plan carries a caller's potential (a whole-grid V0 table and/or W
// in place of x); the other instantiations keep the soft-core path alone.
template <typename T, int N, bool PERSIST, bool UP = false>
__global__ void __launch_bounds__((kernel_threads<N, kRowThreads, PERSIST>()), (kernel_waves<N, PERSIST>())) k_row_pass(PassArgs<T> a) {
  using X = xch_t<T>;
  constexpr int P = Shape<N>::P, TPL = N / P;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<X>* lines = reinterpret_cast<cx<X>*>(smem);
  const int lpb = blockDim.x / TPL;
  const int l = threadIdx.x / TPL, t = threadIdx.x - l * TPL;
  const LineLDS<X> L{lines, l * a.lds_line, 1};
  const int nlines = a.nruns * a.ny;
  const bool cn = a.do_pot && a.m > 0;
  const int64_t step = pass_step(a);
  auto body = [&](int tile) {
    constexpr int RG = (65536 / int(N * sizeof(cx<T>))) > 1 ? (65536 / int(N * sizeof(cx<T>))) : 1;
    const int g = xcd_rows<RG>(tile, lpb, nlines, a.ntiles) * lpb + l;
    const bool live = g < nlines;
    const int gg = live ? g : 0;
    const int run = gg / a.ny, crow = gg - run * a.ny;
    cx<T>* line = run_state(a, run) + size_t(crow) * N;
    // branch-free global loads (dead lanes read row 0 of run 0 and store nothing)
    cx<double> v[P];
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = widen(gload(line + t + TPL * s));
    // kinetic factors, static potential phases and x of the field term are
    // fetched where they are used: held across the transforms they cost the
    // registers of a fifth wave per SIMD (P = 4) or 120 VGPRs (P = 12).
    cx<double> kin[P];
    auto load_kin = [&]() {
#pragma unroll
      for (int s = 0; s < P; ++s) kin[s] = a.kin[t + TPL * s];
    };
    cx<double> vps[P];
    double xs[P];
    double f = 0.0;
    auto load_pot = [&]() {
      if (a.do_pot) {
        if constexpr (UP) {
          const cx<double>* vrow =
              a.vph ? a.vph + (a.vfull ? size_t(crow) * N : size_t(vfold(crow, a.ny)) * (N / 2)) : nullptr;
          const double* wrow = a.w ? a.w + size_t(crow) * N : a.x;
#pragma unroll
          for (int s = 0; s < P; ++s) {
            const int e = t + TPL * s;
            vps[s] = vrow ? vrow[a.vfull ? e : vfold(e, N)] : cx<double>{1.0, 0.0};
            xs[s] = wrow[e];
          }
        } else {
          const cx<double>* vrow = a.vph ? a.vph + size_t(vfold(crow, a.ny)) * (N / 2) : nullptr;
#pragma unroll
          for (int s = 0; s < P; ++s) {
            vps[s] = vrow ? vrow[vfold(t + TPL * s, N)] : cx<double>{1.0, 0.0};
            xs[s] = a.x[t + TPL * s];
          }
        }
        const double* fm = run_field(a, run);
        f = fm ? fm[step] : 0.0;
      }
    };
    // A row of TPL <= 64 threads (TPL dividing 64) lies within one wavefront:
    // its exchanges then need wavefront barriers only, and the rows of a
    // block progress independently.
    constexpr bool wave_rows = TPL <= 64 && 64 % TPL == 0;
    if constexpr (fft_buffers<N, X>() == 2) {
      const LineLDS<X> Lb{lines, l * a.lds_line + fft_lds_elems<N>(), 1};
      constexpr bool swz = fft2_swizzle<N>();   // rows are contiguous in LDS
      fft2<X, N, -1, wave_rows, swz>(v, L, Lb, t, a.tw);
      load_kin();
#pragma unroll
      for (int s = 0; s < P; ++s) v[s] = cmul(v[s], kin[s]);
      fft2<X, N, +1, wave_rows, swz>(v, L, Lb, t, a.tw);
    } else {
      fft<X, N, -1, wave_rows>(v, L, t, a.tw);
      load_kin();
#pragma unroll
      for (int s = 0; s < P; ++s) v[s] = cmul(v[s], kin[s]);
      fft<X, N, +1, wave_rows>(v, L, t, a.tw);
    }
    load_pot();
    if (a.do_pot) {
      // Rows outside the y-strip get both potential half-steps here (C_y is the
      // identity on them); rows on it get the first, the column pass the second.
      // On the x-strip the phase waits in LDS (from 2m) across the CN.
      // exp(-i U dt/2) = exp(-i V0 dt/2) exp(-i f x dt/2)
      const bool both = strip_pos_rt(crow, a.j0y, a.ny) >= a.my;
      const int m = a.m;
      const double fh = f * a.ht;
#pragma unroll
      for (int s = 0; s < P; ++s) {
        const cx<double> ph = cmul(vps[s], expi(fh * xs[s], 0.0));
        const int p = strip_pos<N>(t + TPL * s, a.j0);
        if (p < m) {
          v[s] = cmul(v[s], ph);
          L[p] = narrow<X>(v[s]);
          if (both) L[2 * m + p] = ph;
        } else {
          v[s] = cmul(v[s], both ? cmul(ph, ph) : ph);
        }
      }
      if (cn) {
        cn_block<T, N>(lpb, a, [&](int ln) { return LineLDS<X>{lines, ln * a.lds_line, 1}; });
#pragma unroll
        for (int s = 0; s < P; ++s) {
          const int p = strip_pos<N>(t + TPL * s, a.j0);
          if (p < m) {
            v[s] = 2.0 * widen(L[cn_result(m, a.levels) + p]) - v[s];
            if (both) v[s] = cmul(v[s], widen(L[2 * m + p]));
          }
        }
      }
    }
    if (live) {
#pragma unroll
      for (int s = 0; s < P; ++s) gstore(line + t + TPL * s, narrow<T>(v[s]));
    }
  };
  run_tiles<PERSIST>(a.ntiles, body);
}

// Column blocks are assigned so that blocks of neighbouring columns run on one
// XCD (workgroups go round-robin over the 8 XCDs): the cg blocks whose columns
// share 128-byte lines then meet in the same L2.  A single grid takes groups
// of cg adjacent blocks per XCD slot (cg = 2 for 4 complex128 columns, 4 for
// complex64), measured faster than one block per slot (17% per step at 1024^2
// complex128) and than contiguous bands of columns per XCD (2%); at complex64,
// cg = 4 with RG = 8 measured 10% faster than cg = 2 with RG = 4.  Batches
// keep the bands (the groups measured 6% slower there).
// Slots (s of element t + TPL s) of a column that can hold y-strip nodes: the
// strip is symmetric and holds at most half of the nodes, so at most N/4 per
// side, i.e. one slot per side for P = 4 and three for P = 12.
template <int N>
__host__ __device__ constexpr int col_edge_slots() { return Shape<N>::P == 4 ? 1 : 3; }
// k-th edge slot, k < 2 SE: 0 .. SE-1, then P-SE .. P-1.
template <int P, int SE>
__device__ __forceinline__ constexpr int edge_slot(int k) { return k < SE ? k : P - 2 * SE + k; }

__device__ __forceinline__ int xcd_block(int b, int nblk, bool single, int cg) {
  if (single) return nblk % (8 * cg) != 0 ? b : 8 * cg * (b / (8 * cg)) + cg * (b & 7) + (b >> 3) % cg;
  return nblk % 8 != 0 ? b : (b % 8) * (nblk / 8) + b / 8;
}

template <typename T, int N, bool PERSIST, bool UP = false>
__global__ void __launch_bounds__((kernel_threads<N, kColThreads, PERSIST>()), (kernel_waves<N, PERSIST>())) k_col_pass(PassArgs<T> a) {
  using X = xch_t<T>;
  constexpr int P = Shape<N>::P, TPL = N / P;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<X>* lines = reinterpret_cast<cx<X>*>(smem);
  const int lpb = blockDim.x / TPL;
  const int c = threadIdx.x % lpb, t = threadIdx.x / lpb;
  const LineLDS<X> L{lines, c, lpb};
  const size_t ld = size_t(a.nx);
  const int nlines = a.nruns * a.nx;
  const bool cn = a.do_pot && a.m > 0;
  const int64_t step = pass_step(a);
  auto body = [&](int tile) {
    const int cg = max(1, 128 / (lpb * int(sizeof(cx<T>))));
    const int g = xcd_block(tile, a.ntiles, a.runs == nullptr, cg) * lpb + c;
    const bool live = g < nlines;
    const int gg = live ? g : 0;
    const int run = gg / a.nx, ccol = gg - run * a.nx;
    cx<T>* base = run_state(a, run) + ccol;
    // The y-strip lies in the first and last SE slots of a column (the host
    // checks it): those are loaded first, so the CN can start while the
    // interior slots are still in flight.
    constexpr int SE = col_edge_slots<N>();
    // The field, x of this column and the potential-table entries of the
    // strip are loaded before the state, and used after the state's loads are
    // issued, so that waiting for them does not wait for the state.
    double f = 0.0, xc = 0.0;
    cx<double> vps[2 * SE];
    double wv[2 * SE];
    if (cn) {
      const double* fm = run_field(a, run);
      f = fm ? fm[step] : 0.0;
      xc = a.x[ccol];
#pragma unroll
      for (int k = 0; k < 2 * SE; ++k) {
        const int e = t + TPL * edge_slot<P, SE>(k);
        const bool on = strip_pos<N>(e, a.j0) < a.m;
        if constexpr (UP) {
          vps[k] = (on && a.vph) ? a.vph[a.vfull ? size_t(e) * ld + ccol
                                                 : size_t(vfold(e, N)) * (a.nx / 2) + vfold(ccol, a.nx)]
                                 : cx<double>{1.0, 0.0};
          wv[k] = (on && a.w) ? a.w[size_t(e) * ld + ccol] : 0.0;
        } else {
          vps[k] = (on && a.vph) ? a.vph[size_t(vfold(e, N)) * (a.nx / 2) + vfold(ccol, a.nx)]
                                 : cx<double>{1.0, 0.0};
        }
      }
    }
    // Loads in storage precision; the interior slots are widened after the CN
    // (for complex64 a conversion right after its load would wait for it).
    cx<T> raw[P];
#pragma unroll
    for (int k = 0; k < 2 * SE; ++k) {
      const int s = edge_slot<P, SE>(k);
      raw[s] = gload(base + size_t(t + TPL * s) * ld);
    }
    __builtin_amdgcn_sched_barrier(0);   // keep the edge loads ahead of the interior ones
#pragma unroll
    for (int s = SE; s < P - SE; ++s) raw[s] = gload(base + size_t(t + TPL * s) * ld);
    __builtin_amdgcn_sched_barrier(0);   // and every load issued before the first wait
    cx<double> v[P];
#pragma unroll
    for (int k = 0; k < 2 * SE; ++k) {
      const int s = edge_slot<P, SE>(k);
      v[s] = widen(raw[s]);
    }
    if (cn) {
      // C_y and the second potential half-step, on the y-strip only.
      // exp(-i U dt/2) = exp(-i V0 dt/2) exp(-i f W dt/2); with W = x the
      // field factor is the same along the column
      const cx<double> lph = expi(f * xc * a.ht, 0.0);
#pragma unroll
      for (int k = 0; k < 2 * SE; ++k) {
        if constexpr (UP) {
          vps[k] = cmul(vps[k], a.w ? expi(f * wv[k] * a.ht, 0.0) : lph);
        } else {
          vps[k] = cmul(vps[k], lph);
        }
      }
      const int m = a.m;
      // The strips go to a contiguous area per column (odd stride 2m + 1), not
      // the interleaved FFT layout: one wavefront's positions are then
      // consecutive in LDS and the reduction is free of bank conflicts.
      const int cstride = 2 * m + 1;
      const LineLDS<X> Lc{lines, c * cstride, 1};
#pragma unroll
      for (int k = 0; k < 2 * SE; ++k) {
        const int s = edge_slot<P, SE>(k);
        const int p = strip_pos<N>(t + TPL * s, a.j0);
        if (p < m) Lc[p] = narrow<X>(v[s]);
      }
      cn_block<T, N>(lpb, a, [&](int ln) { return LineLDS<X>{lines, ln * cstride, 1}; });
#pragma unroll
      for (int k = 0; k < 2 * SE; ++k) {
        const int s = edge_slot<P, SE>(k);
        const int p = strip_pos<N>(t + TPL * s, a.j0);
        if (p < m) v[s] = cmul(2.0 * widen(Lc[cn_result(m, a.levels) + p]) - v[s], vps[k]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int s = SE; s < P - SE; ++s) v[s] = widen(raw[s]);
    // the kinetic factors: for P = 4 fetched before the transforms (latency
    // hidden behind them); the P = 12 shapes fetch them where they are used,
    // which keeps their column pass free of spills
    cx<double> kin[P];
    auto load_kin = [&]() {
#pragma unroll
      for (int s = 0; s < P; ++s) kin[s] = a.kin[t + TPL * s];
    };
    constexpr bool early_kin = P == 4;
    if constexpr (early_kin) load_kin();
    if constexpr (fft_buffers<N, X>() == 2) {
      const LineLDS<X> Lb{lines, c + fft_lds_elems<N>() * lpb, lpb};
      fft2<X, N, -1>(v, L, Lb, t, a.tw);
      if constexpr (!early_kin) load_kin();
#pragma unroll
      for (int s = 0; s < P; ++s) v[s] = cmul(v[s], kin[s]);
      fft2<X, N, +1>(v, L, Lb, t, a.tw);
    } else {
      fft<X, N, -1>(v, L, t, a.tw);
      if constexpr (!early_kin) load_kin();
#pragma unroll
      for (int s = 0; s < P; ++s) v[s] = cmul(v[s], kin[s]);
      fft<X, N, +1>(v, L, t, a.tw);
    }
    if (live) {
#pragma unroll
      for (int s = 0; s < P; ++s) gstore(base + size_t(t + TPL * s) * ld, narrow<T>(v[s]));
    }
  };
  run_tiles<PERSIST>(a.ntiles, body);
}

// 1D: the whole propagation in one workgroup; psi stays in registers.  LDS
// holds two exchange buffers (fft2); twiddles are read through the vector L1.
// The static potential phase exp(-i V0 dt/2) comes from the plan's table (or is
// 1 without a potential) and is multiplied by exp(-i f x dt/2) each step.
template <typename T, int N>
__global__ void __launch_bounds__(N / Shape<N>::P) k_tdse1d(PassArgs<T> a, const cx<double>* kin_half,
                                                             const cx<double>* kin_full, int64_t nsteps) {
  using X = xch_t<T>;
  constexpr int P = Shape<N>::P, TPL = N / P;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<X>* lds = reinterpret_cast<cx<X>*>(smem);   // [line (lds_line)][second exchange buffer (N)]
  const int t = threadIdx.x;
  const LineLDS<X> L{lds, 0, 1};
  const LineLDS<X> Lb{lds, a.lds_line, 1};
  cx<double> v[P];
  cx<double> kf[P];
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = widen(a.psi[t + TPL * s]);
#pragma unroll
  for (int s = 0; s < P; ++s) kf[s] = kin_half[t + TPL * s];
  constexpr bool swz = fft2_swizzle<N>();   // the line is contiguous in LDS
  fft2<X, N, -1, false, swz>(v, L, Lb, t, a.tw);
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = cmul(v[s], kf[s]);
  fft2<X, N, +1, false, swz>(v, L, Lb, t, a.tw);
  for (int64_t n = 0; n < nsteps; ++n) {
    const double fh = (a.f_mid ? a.f_mid[n] : 0.0) * a.ht;
    pot_cn_pot<T, N>(v, L, t, a, [&](int e) {
      const cx<double> ph = expi(fh * (a.w ? a.w[e] : a.x[e]), 0.0);
      return a.vph ? cmul(a.vph[a.vfull ? e : vfold(e, N)], ph) : ph;
    });
    const cx<double>* kin = n + 1 == nsteps ? kin_half : kin_full;
#pragma unroll
    for (int s = 0; s < P; ++s) kf[s] = kin[t + TPL * s];
    fft2<X, N, -1, false, swz>(v, L, Lb, t, a.tw);
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = cmul(v[s], kf[s]);
    fft2<X, N, +1, false, swz>(v, L, Lb, t, a.tw);
  }
#pragma unroll
  for (int s = 0; s < P; ++s) a.psi[t + TPL * s] = narrow<T>(v[s]);
}

// exp(-i V0(z_x, z_y) dt/2) (the static part of the potential phase) on the
// quadrant [hy][hx] of nodes j < n/2 per axis (hy = 1 in 1D).
__global__ void __launch_bounds__(256) k_vphase(cx<double>* out, int hx, int hy, const cx<double>* zx,
                                                const cx<double>* zy, double charge, double a2, double ht) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= size_t(hx) * hy) return;
  const int jx = int(i % hx), jy = int(i / hx);
  const cx<double> zy2 = zy ? cmul(zy[jy], zy[jy]) : cx<double>{0.0, 0.0};   // 1D: no y term
  out[i] = potential_phase(cmul(zx[jx], zx[jx]) + zy2 + cx<double>{a2, 0.0}, charge, 0.0, ht);
}

// exp(-i V0 dt/2) from a caller's V0 on the whole grid (n nodes).
__global__ void __launch_bounds__(256) k_vphase_user(cx<double>* out, const cx<double>* v0, size_t n, double ht) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cx<double> v = v0[i];
  out[i] = expi(v.re * ht, v.im * ht);
}

// The soft-core V0 = -charge / sqrt(z_x^2 [+ z_y^2] + a2) on the [ny][nx] grid.
__global__ void __launch_bounds__(256) k_softcore(cx<double>* out, int nx, int ny, const cx<double>* zx,
                                                  const cx<double>* zy, double charge, double a2) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= size_t(nx) * ny) return;
  const int jx = int(i % nx), jy = int(i / nx);
  const cx<double> zy2 = zy ? cmul(zy[jy], zy[jy]) : cx<double>{0.0, 0.0};
  out[i] = potential_value(cmul(zx[jx], zx[jx]) + zy2 + cx<double>{a2, 0.0}, charge, 0.0);
}

__global__ void k_step_add(int64_t* counter, int64_t delta, int set) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = set ? delta : *counter + delta;
}

// Per-run FP64 partial sums of |psi|^2: block (b, r) of a 64 x nruns grid.
template <typename T>
__global__ void __launch_bounds__(256) k_norm2_runs(const cx<T>* const* runs, int64_t n, double* partials) {
  __shared__ double red[256];
  const cx<T>* psi = runs[blockIdx.y];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const cx<T> v = psi[i];
    acc += double(v.re) * double(v.re) + double(v.im) * double(v.im);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[size_t(blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

template <typename T>
__global__ void __launch_bounds__(256) k_norm2(const cx<T>* psi, int64_t n, double* partials) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const cx<T> v = psi[i];
    acc += double(v.re) * double(v.re) + double(v.im) * double(v.im);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------- launchers

template <typename X>
static int64_t lds_elems_for(int64_t n) {
  switch (n) {
#define SOFFT_LDS_CASE(N) \
  case N:                 \
    return fft_buffers<N, X>() * fft_lds_elems<N>();
    SOFFT_LDS_CASE(16) SOFFT_LDS_CASE(32) SOFFT_LDS_CASE(48) SOFFT_LDS_CASE(64) SOFFT_LDS_CASE(96)
    SOFFT_LDS_CASE(128) SOFFT_LDS_CASE(192) SOFFT_LDS_CASE(256) SOFFT_LDS_CASE(384) SOFFT_LDS_CASE(512)
    SOFFT_LDS_CASE(768) SOFFT_LDS_CASE(1024) SOFFT_LDS_CASE(2048) SOFFT_LDS_CASE(4096)
#undef SOFFT_LDS_CASE
    default:
      return 2 * n;
  }
}

template <typename T>
static PassArgs<T> axis_args(Plan& p, int axis, void* psi, double dt, const cx<double>* vph) {
  Axis& A = p.ax[axis];
  PassArgs<T> a{};
  a.psi = static_cast<cx<T>*>(psi);
  a.nruns = 1;
  a.nx = int(p.ax[0].n);
  a.ny = p.prob.ndim == 2 ? int(p.ax[1].n) : 1;
  a.tw = static_cast<const cx<double>*>(A.tw64.p);
  a.ht = 0.5 * dt;
  a.charge = p.prob.charge;
  a.a2 = p.prob.a2;
  a.x = static_cast<const double*>(p.ax[0].x_dev.p);
  a.zx = static_cast<const cx<double>*>(p.ax[0].z_dev.p);
  a.zy = p.prob.ndim == 2 ? static_cast<const cx<double>*>(p.ax[1].z_dev.p) : nullptr;
  a.vph = vph;
  a.vfull = p.user_v0 != nullptr;
  a.w = p.user_w;
  a.j0 = int(A.j0);
  a.m = int(A.m);
  a.levels = A.levels;
  a.alpha = static_cast<const cx<double>*>(A.alpha64.p);
  a.gamma = static_cast<const cx<double>*>(A.gamma64.p);
  a.binv = static_cast<const cx<double>*>(A.binv64.p);
  a.lds_line = int(std::max<int64_t>(lds_elems_for<xch_t<T>>(A.n), 3 * A.m));
  // y-strip, used by the row pass to decide which rows take both half-steps
  a.j0y = p.prob.ndim == 2 ? int(p.ax[1].j0) : 0;
  a.my = p.prob.ndim == 2 ? int(p.ax[1].m) : 0;
  return a;
}

// LDS budget per block (MI355X has 160 KiB per CU; leave room for the runtime).
constexpr size_t kLdsBudget = 150 * 1024;

// Raise a kernel's dynamic LDS limit once (to the whole budget) the first time
// it needs more than the default 64 KiB.
template <typename K>
static sofft_status set_lds(K kernel, size_t bytes) {
  return bytes > 65536 ? raise_lds_limit(reinterpret_cast<const void*>(kernel), kLdsBudget) : SOFFT_OK;
}

#define SOFFT_LENGTH_SWITCH(n, FN, T, ...)        \
  switch (n) {                                    \
    case 16: return FN<T, 16>(__VA_ARGS__);       \
    case 32: return FN<T, 32>(__VA_ARGS__);       \
    case 48: return FN<T, 48>(__VA_ARGS__);       \
    case 64: return FN<T, 64>(__VA_ARGS__);       \
    case 96: return FN<T, 96>(__VA_ARGS__);       \
    case 128: return FN<T, 128>(__VA_ARGS__);     \
    case 192: return FN<T, 192>(__VA_ARGS__);     \
    case 256: return FN<T, 256>(__VA_ARGS__);     \
    case 384: return FN<T, 384>(__VA_ARGS__);     \
    case 512: return FN<T, 512>(__VA_ARGS__);     \
    case 768: return FN<T, 768>(__VA_ARGS__);     \
    case 1024: return FN<T, 1024>(__VA_ARGS__);   \
    default: break;                               \
  }

// Lines per block of a 2D pass with `threads` threads (at least one line),
// fewer when the lines' LDS would exceed the budget.  Blocks are whole
// wavefronts (the CN gives each wavefront whole lines), so with lines shorter
// than a wavefront lpb is a multiple of 64/TPL.
template <typename T, int N>
static int lines_per_block(int threads, int lds_line, size_t* lds_bytes) {
  constexpr int TPL = N / Shape<N>::P;
  constexpr int unit = TPL >= 64 ? 1 : 64 / TPL;
  int lpb = TPL >= threads ? 1 : threads / TPL;
  const size_t per_line = size_t(lds_line) * sizeof(cx<xch_t<T>>);
  while (lpb > unit && lpb * per_line > kLdsBudget) --lpb;
  lpb -= lpb % unit;
  *lds_bytes = size_t(lpb) * per_line;
  return (lpb == 0 || *lds_bytes > kLdsBudget) ? 0 : lpb;
}

template <typename T, int N, bool ROW, bool PERSIST>
static void* pass_kernel() {
  return ROW ? reinterpret_cast<void*>(k_row_pass<T, N, PERSIST>) : reinterpret_cast<void*>(k_col_pass<T, N, PERSIST>);
}

template <typename T, int N, bool ROW>
static sofft_status pass_set_lds(size_t lds) {
  sofft_status st = ROW ? set_lds(k_row_pass<T, N, false>, lds) : set_lds(k_col_pass<T, N, false>, lds);
  if (st == SOFFT_OK) st = ROW ? set_lds(k_row_pass<T, N, true>, lds) : set_lds(k_col_pass<T, N, true>, lds);
  if (st == SOFFT_OK)
    st = ROW ? set_lds(k_row_pass<T, N, false, true>, lds) : set_lds(k_col_pass<T, N, false, true>, lds);
  return st;
}

// One pass over the lines of every run in a (row pass if ROW, else column
// pass).  cfg.threads = 0 takes the default block size; cfg.grid = 0 launches
// one block per tile, otherwise at most cfg.grid blocks loop over the tiles.
template <typename T, int N, bool ROW>
static sofft_status pass(PassArgs<T> a, PassLaunch cfg, hipStream_t s, Timing* tm) {
  constexpr int TPL = N / Shape<N>::P;
  const bool want_persist = cfg.grid > 0;
  const int maxt = want_persist ? kernel_threads<N, ROW ? kRowThreads : kColThreads, true>()
                                : kernel_threads<N, ROW ? kRowThreads : kColThreads, false>();
  const int threads = cfg.threads > 0 ? std::min(cfg.threads, maxt) : maxt;
  size_t lds = 0;
  const int lpb = lines_per_block<T, N>(threads, a.lds_line, &lds);
  if (lpb == 0) {
    set_error("ECS strip too long for the LDS budget");
    return SOFFT_EUNSUPPORTED;
  }
  sofft_status st = pass_set_lds<T, N, ROW>(lds);
  if (st != SOFFT_OK) return st;
  if (!ROW && a.do_pot && a.m > 0) {
    // the column pass applies the CN to the edge slots only
    constexpr int SE = col_edge_slots<N>(), P = Shape<N>::P;
    for (int q = 0; q < a.m; ++q) {
      const int sl = ((a.j0 + q) % N) / TPL;
      if (sl >= SE && sl < P - SE) {
        set_error("ECS strip of the y axis reaches beyond the outer quarters of the axis");
        return SOFFT_EUNSUPPORTED;
      }
    }
  }
  const int lines = a.nruns * (ROW ? a.ny : a.nx);
  a.ntiles = (lines + lpb - 1) / lpb;
  // a caller's potential (single plans only) takes the one-block-per-tile grid
  const bool user = a.vfull || a.w;
  const bool persist = !user && want_persist && cfg.grid < a.ntiles;
  const int blocks = persist ? cfg.grid : a.ntiles;
  if (tm && (st = tm->begin(ROW ? SOFFT_KERNEL_ROW : SOFFT_KERNEL_COL, s)) != SOFFT_OK) return st;
  if (user) {
    if (ROW)
      k_row_pass<T, N, false, true><<<blocks, lpb * TPL, lds, s>>>(a);
    else
      k_col_pass<T, N, false, true><<<blocks, lpb * TPL, lds, s>>>(a);
  } else if (ROW) {
    if (persist)
      k_row_pass<T, N, true><<<blocks, lpb * TPL, lds, s>>>(a);
    else
      k_row_pass<T, N, false><<<blocks, lpb * TPL, lds, s>>>(a);
  } else {
    if (persist)
      k_col_pass<T, N, true><<<blocks, lpb * TPL, lds, s>>>(a);
    else
      k_col_pass<T, N, false><<<blocks, lpb * TPL, lds, s>>>(a);
  }
  SOFFT_HIP_TRY(hipGetLastError());
  return tm ? tm->end(s) : SOFFT_OK;
}

// Resident blocks per CU of a pass kernel at a block size (for persistent grids).
template <typename T, int N, bool ROW>
static sofft_status pass_occupancy(int lds_line, int threads, int* blocks_per_cu, int* block_threads_out) {
  constexpr int TPL = N / Shape<N>::P;
  constexpr int maxt = kernel_threads<N, ROW ? kRowThreads : kColThreads, true>();
  threads = threads > 0 ? std::min(threads, maxt) : maxt;
  size_t lds = 0;
  const int lpb = lines_per_block<T, N>(threads, lds_line, &lds);
  if (lpb == 0) {
    set_error("ECS strip too long for the LDS budget");
    return SOFFT_EUNSUPPORTED;
  }
  sofft_status st = pass_set_lds<T, N, ROW>(lds);
  if (st != SOFFT_OK) return st;
  int nb = 0;
  SOFFT_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pass_kernel<T, N, ROW, true>(), lpb * TPL, lds));
  *blocks_per_cu = nb;
  *block_threads_out = lpb * TPL;
  return SOFFT_OK;
}

#define SOFFT_PASS_SWITCH(n, EXPR_N)                                                  \
  switch (n) {                                                                        \
    case 16: { constexpr int N_ = 16; return EXPR_N; }                                \
    case 32: { constexpr int N_ = 32; return EXPR_N; }                                \
    case 48: { constexpr int N_ = 48; return EXPR_N; }                                \
    case 64: { constexpr int N_ = 64; return EXPR_N; }                                \
    case 96: { constexpr int N_ = 96; return EXPR_N; }                                \
    case 128: { constexpr int N_ = 128; return EXPR_N; }                              \
    case 192: { constexpr int N_ = 192; return EXPR_N; }                              \
    case 256: { constexpr int N_ = 256; return EXPR_N; }                              \
    case 384: { constexpr int N_ = 384; return EXPR_N; }                              \
    case 512: { constexpr int N_ = 512; return EXPR_N; }                              \
    case 768: { constexpr int N_ = 768; return EXPR_N; }                              \
    case 1024: { constexpr int N_ = 1024; return EXPR_N; }                            \
    default: break;                                                                   \
  }

template <typename T>
static sofft_status pass_n(bool row, const PassArgs<T>& a, PassLaunch cfg, hipStream_t s, Timing* tm) {
  const int n = row ? a.nx : a.ny;
  if (row) {
    SOFFT_PASS_SWITCH(n, (pass<T, N_, true>(a, cfg, s, tm)))
  } else {
    SOFFT_PASS_SWITCH(n, (pass<T, N_, false>(a, cfg, s, tm)))
  }
  set_error("unsupported 2D line length");
  return SOFFT_EUNSUPPORTED;
}

template <typename T>
static sofft_status occupancy_n(bool row, int n, int lds_line, int threads, int* nb, int* bt) {
  if (row) {
    SOFFT_PASS_SWITCH(n, (pass_occupancy<T, N_, true>(lds_line, threads, nb, bt)))
  } else {
    SOFFT_PASS_SWITCH(n, (pass_occupancy<T, N_, false>(lds_line, threads, nb, bt)))
  }
  set_error("unsupported 2D line length");
  return SOFFT_EUNSUPPORTED;
}

// The table of exp(-i V0 dt/2) for this dt (plans with a potential): one
// quadrant for the soft-core, the whole grid for a caller's V0.
// Bytes of the table of exp(-i V0 dt/2): one quadrant for the soft-core, the
// whole grid for a caller's V0; 0 when the plan has no potential.
size_t vphase_bytes(const Plan& p) {
  if (p.prob.charge == 0.0 && !p.user_v0) return 0;
  size_t full = 1, fold = 1;
  for (int d = 0; d < p.prob.ndim; ++d) {
    full *= size_t(p.ax[d].n);
    fold *= size_t(p.ax[d].n) / 2;
  }
  return (p.user_v0 ? full : fold) * sizeof(cx<double>);
}

// Write the table of exp(-i V0 dt/2) of the plan into `table` (vphase_bytes).
static sofft_status build_vphase(const Plan& p, double dt, cx<double>* table, hipStream_t s) {
  if (p.prob.ndim == 3 && !p.user_v0) return build_octant_vphase(p, dt, table, s);
  if (p.prob.ndim == 3) {
    const size_t n = size_t(p.ax[0].n) * p.ax[1].n * p.ax[2].n;
    k_vphase_user<<<unsigned((n + 255) / 256), 256, 0, s>>>(table, static_cast<const cx<double>*>(p.user_v0), n,
                                                          0.5 * dt);
    SOFFT_HIP_TRY(hipGetLastError());
    return SOFFT_OK;
  }
  const bool full = p.user_v0 != nullptr;
  const int ny = p.prob.ndim == 2 ? int(p.ax[1].n) : 1;
  const int hx = int(p.ax[0].n) / 2, hy = p.prob.ndim == 2 ? ny / 2 : 1;
  const size_t n = full ? size_t(p.ax[0].n) * ny : size_t(hx) * hy;
  if (full) {
    k_vphase_user<<<unsigned((n + 255) / 256), 256, 0, s>>>(table, static_cast<const cx<double>*>(p.user_v0), n,
                                                          0.5 * dt);
  } else {
    k_vphase<<<unsigned((n + 255) / 256), 256, 0, s>>>(table, hx, hy, static_cast<const cx<double>*>(p.ax[0].z_dev.p),
                                                       p.prob.ndim == 2 ? static_cast<const cx<double>*>(p.ax[1].z_dev.p)
                                                                        : nullptr,
                                                       p.prob.charge, p.prob.a2, 0.5 * dt);
  }
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

// The plan's table of exp(-i V0 dt/2) in its workspace, built once per dt (and
// per binding); *table is null when the plan has no potential.
sofft_status ensure_vphase(Plan& p, double dt, hipStream_t s, bool* changed, const cx<double>** table) {
  if (changed) *changed = false;
  if (table) *table = nullptr;
  WsLayout L;
  sofft_status st = plan_ws_check(p, 0, &L);
  if (st != SOFFT_OK) return st;
  if (vphase_bytes(p) == 0) return SOFFT_OK;
  cx<double>* t = reinterpret_cast<cx<double>*>(ws_at(p, L.vphase));
  if (table) *table = t;
  if (p.vphase_ht == 0.5 * dt) return SOFFT_OK;
  if ((st = build_vphase(p, dt, t, s)) != SOFFT_OK) return st;
  p.vphase_ht = 0.5 * dt;
  if (changed) *changed = true;
  return SOFFT_OK;
}

template <typename T>
static sofft_status propagate_2d(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                 const cx<double>* vph, hipStream_t s) {
  PassArgs<T> ra = axis_args<T>(p, 0, psi, dt, vph);
  PassArgs<T> ca = axis_args<T>(p, 1, psi, dt, vph);
  ra.f_mid = ca.f_mid = f_mid;
  const cx<double>* kxf = static_cast<const cx<double>*>(p.ax[0].kin_full64.p);
  const cx<double>* kxh = static_cast<const cx<double>*>(p.ax[0].kin_half64.p);
  const cx<double>* kyf = static_cast<const cx<double>*>(p.ax[1].kin_full64.p);
  const cx<double>* kyh = static_cast<const cx<double>*>(p.ax[1].kin_half64.p);
  const PassLaunch dflt{};
  sofft_status st;
  // opening K_y/2
  ca.do_pot = 0;
  ca.kin = kyh;
  if ((st = pass_n<T>(false, ca, dflt, s, &p.timing)) != SOFFT_OK) return st;
  ra.do_pot = ca.do_pot = 1;
  for (int64_t n = 0; n < nsteps; ++n) {
    ra.step = ca.step = n;
    ra.kin = n == 0 ? kxh : kxf;
    ca.kin = n + 1 == nsteps ? kyh : kyf;
    if ((st = pass_n<T>(true, ra, dflt, s, &p.timing)) != SOFFT_OK) return st;
    if ((st = pass_n<T>(false, ca, dflt, s, &p.timing)) != SOFFT_OK) return st;
  }
  // closing K_x/2
  ra.do_pot = 0;
  ra.kin = kxh;
  return pass_n<T>(true, ra, dflt, s, &p.timing);
}

sofft_status launch_pass(Plan& p, const PassRequest& rq, hipStream_t s) {
  const int axis = rq.row ? 0 : 1;
  const Axis& A = p.ax[axis];
  // the class plan's table, built by ensure_vphase for this dt
  const cx<double>* vph = vphase_bytes(p) && p.vphase_ht == 0.5 * rq.dt
                              ? reinterpret_cast<const cx<double>*>(ws_at(p, plan_ws_layout(p, 0).vphase))
                              : nullptr;
  const cx<double>* kin = static_cast<const cx<double>*>(rq.half_kinetic ? A.kin_half64.p : A.kin_full64.p);
  if (p.prob.dtype == SOFFT_C128) {
    PassArgs<double> a = axis_args<double>(p, axis, nullptr, rq.dt, vph);
    a.runs = reinterpret_cast<cx<double>* const*>(rq.runs);
    a.f_runs = rq.f_runs;
    a.nruns = rq.nruns;
    a.step = rq.step;
    a.step_base = rq.step_base;
    a.do_pot = rq.do_pot;
    a.kin = kin;
    return pass_n<double>(rq.row, a, rq.cfg, s, rq.timing);
  }
  PassArgs<float> a = axis_args<float>(p, axis, nullptr, rq.dt, vph);
  a.runs = reinterpret_cast<cx<float>* const*>(rq.runs);
  a.f_runs = rq.f_runs;
  a.nruns = rq.nruns;
  a.step = rq.step;
  a.step_base = rq.step_base;
  a.do_pot = rq.do_pot;
  a.kin = kin;
  return pass_n<float>(rq.row, a, rq.cfg, s, rq.timing);
}

sofft_status pass_residency(const Plan& p, bool row, int threads, int* blocks_per_cu, int* block_threads_out) {
  const Axis& A = p.ax[row ? 0 : 1];
  const int lds_line = p.prob.dtype == SOFFT_C128 ? int(std::max<int64_t>(lds_elems_for<xch_t<double>>(A.n), 3 * A.m))
                                                 : int(std::max<int64_t>(lds_elems_for<xch_t<float>>(A.n), 3 * A.m));
  return p.prob.dtype == SOFFT_C128 ? occupancy_n<double>(row, int(A.n), lds_line, threads, blocks_per_cu, block_threads_out)
                                    : occupancy_n<float>(row, int(A.n), lds_line, threads, blocks_per_cu, block_threads_out);
}

template <typename T, int N>
static sofft_status tdse1d(Plan& p, PassArgs<T> a, int64_t nsteps, hipStream_t s) {
  constexpr int TPL = N / Shape<N>::P;
  // the line (with room for the CN strip) and a second exchange buffer
  a.lds_line = int(std::max<int64_t>(fft_lds_elems<N>(), 3 * p.ax[0].m));
  const size_t lds = (size_t(a.lds_line) + fft_lds_elems<N>()) * sizeof(cx<xch_t<T>>);
  if (lds > kLdsBudget) {
    set_error("ECS strip too long for the LDS budget");
    return SOFFT_EUNSUPPORTED;
  }
  sofft_status st = set_lds(k_tdse1d<T, N>, lds);
  if (st != SOFFT_OK) return st;
  const Axis& A = p.ax[0];
  if ((st = p.timing.begin(SOFFT_KERNEL_1D, s)) != SOFFT_OK) return st;
  k_tdse1d<T, N><<<1, TPL, lds, s>>>(a, static_cast<const cx<double>*>(A.kin_half64.p),
                                    static_cast<const cx<double>*>(A.kin_full64.p), nsteps);
  SOFFT_HIP_TRY(hipGetLastError());
  return p.timing.end(s);
}

template <typename T>
static sofft_status propagate_1d(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                 const cx<double>* vph, hipStream_t s) {
  PassArgs<T> a = axis_args<T>(p, 0, psi, dt, vph);
  a.f_mid = f_mid;
  switch (p.ax[0].n) {
    case 2048: return tdse1d<T, 2048>(p, a, nsteps, s);
    case 4096: return tdse1d<T, 4096>(p, a, nsteps, s);
    default: break;
  }
  SOFFT_LENGTH_SWITCH(int(p.ax[0].n), tdse1d, T, p, a, nsteps, s)
  set_error("unsupported 1D length");
  return SOFFT_EUNSUPPORTED;
}

// Propagation with the potential-phase table `vph` (null: no potential).
static sofft_status propagate_with(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                   const cx<double>* vph, hipStream_t s) {
  const bool c128 = p.prob.dtype == SOFFT_C128;
  if (p.prob.ndim == 3) return launch_propagate_3d(p, psi, dt, nsteps, f_mid, vph, s);
  if (p.prob.ndim == 1)
    return c128 ? propagate_1d<double>(p, psi, dt, nsteps, f_mid, vph, s)
                : propagate_1d<float>(p, psi, dt, nsteps, f_mid, vph, s);
  return c128 ? propagate_2d<double>(p, psi, dt, nsteps, f_mid, vph, s)
              : propagate_2d<float>(p, psi, dt, nsteps, f_mid, vph, s);
}

sofft_status launch_propagate(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid, hipStream_t s) {
  const cx<double>* vph = nullptr;
  sofft_status st = ensure_vphase(p, dt, s, nullptr, &vph);
  if (st != SOFFT_OK) return st;
  return propagate_with(p, psi, dt, nsteps, f_mid, vph, s);
}

// ------------------------------------------------ propagation without allocation
// For callers that cannot allocate (graph capture, serving loops): the
// potential-phase table, the only scratch memory of a propagation, lives in a
// file-scope device array of kStaticScratchBytes that each GPU holds for the
// life of the process.  Its address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current; host
// code uses only that address.  Every call rebuilds the table (the array keeps
// whatever the last call on the GPU wrote), so calls that overlap on one GPU
// race.
constexpr size_t kStaticScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static sofft_status static_scratch(void** out) {
  static std::mutex mu;
  static std::vector<void*> per_device;
  int dev = -1;
  SOFFT_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (int(per_device.size()) <= dev) per_device.resize(dev + 1, nullptr);
  if (!per_device[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e));
      return SOFFT_EHIP;
    }
    per_device[dev] = ptr;
  }
  *out = per_device[dev];
  return SOFFT_OK;
}

sofft_status launch_propagate_static(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                     hipStream_t s) {
  const size_t need = vphase_bytes(p);
  if (need > kStaticScratchBytes) {
    set_error("the potential-phase table of this plan needs " + std::to_string(need) +
              " bytes, more than the " + std::to_string(kStaticScratchBytes) +
              " bytes of static scratch: use sofft_propagate with a bound workspace");
    return SOFFT_EUNSUPPORTED;
  }
  cx<double>* vph = nullptr;
  if (need) {
    void* base = nullptr;
    sofft_status st = static_scratch(&base);
    if (st != SOFFT_OK) return st;
    vph = static_cast<cx<double>*>(base);
    if ((st = build_vphase(p, dt, vph, s)) != SOFFT_OK) return st;
  }
  return propagate_with(p, psi, dt, nsteps, f_mid, vph, s);
}

sofft_status launch_norm2(Plan& p, const void* psi, double* out, hipStream_t s) {
  WsLayout L;
  sofft_status st = plan_ws_check(p, 0, &L);
  if (st != SOFFT_OK) return st;
  int64_t n = 1;
  for (int d = 0; d < p.prob.ndim; ++d) n *= p.ax[d].n;
  const int blocks = int(std::min<int64_t>(kNormBlocks, (n + 255) / 256));
  double* part = reinterpret_cast<double*>(ws_at(p, L.partials));
  if (p.prob.dtype == SOFFT_C128)
    k_norm2<double><<<blocks, 256, 0, s>>>(static_cast<const cx<double>*>(psi), n, part);
  else
    k_norm2<float><<<blocks, 256, 0, s>>>(static_cast<const cx<float>*>(psi), n, part);
  SOFFT_HIP_TRY(hipGetLastError());
  p.host_partials.resize(blocks);
  SOFFT_HIP_TRY(hipMemcpyAsync(p.host_partials.data(), part, blocks * sizeof(double), hipMemcpyDeviceToHost, s));
  SOFFT_HIP_TRY(hipStreamSynchronize(s));
  double acc = 0.0;
  for (int b = 0; b < blocks; ++b) acc += p.host_partials[b];
  *out = acc;
  return SOFFT_OK;
}

sofft_status launch_softcore(const Plan& p, double charge, double a2, void* out, hipStream_t s) {
  if (p.prob.ndim == 3) return launch_softcore_3d(p, charge, a2, out, s);
  const int nx = int(p.ax[0].n), ny = p.prob.ndim == 2 ? int(p.ax[1].n) : 1;
  const size_t n = size_t(nx) * ny;
  k_softcore<<<unsigned((n + 255) / 256), 256, 0, s>>>(
      static_cast<cx<double>*>(out), nx, ny, static_cast<const cx<double>*>(p.ax[0].z_dev.p),
      p.prob.ndim == 2 ? static_cast<const cx<double>*>(p.ax[1].z_dev.p) : nullptr, charge, a2);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

sofft_status launch_step_add(int64_t* counter, int64_t delta, bool set, hipStream_t s) {
  k_step_add<<<1, 64, 0, s>>>(counter, delta, set ? 1 : 0);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

sofft_status launch_norm2_runs(const void* const* runs_dev, int nruns, int64_t npoints, bool c128,
                               double* partials, hipStream_t s) {
  const dim3 grid(64, nruns);
  if (c128)
    k_norm2_runs<double><<<grid, 256, 0, s>>>(reinterpret_cast<const cx<double>* const*>(runs_dev), npoints, partials);
  else
    k_norm2_runs<float><<<grid, 256, 0, s>>>(reinterpret_cast<const cx<float>* const*>(runs_dev), npoints, partials);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

}  // namespace sofft
