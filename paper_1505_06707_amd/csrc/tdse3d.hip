// Split-operator SO-FFT + ECS step (Sec. II) on 3D grids.  The paper works in
// 1D and names the many-dimensional case as its next step; the 3D step reads
// the scheme separably: K = (k_x^2 + k_y^2 + k_z^2)/2, C = C_x + C_y + C_z and
// e^{-iC dt} = CN(C_x) CN(C_y) CN(C_z).
//
// The state psi[z][y][x] (x fastest) stays in HBM.  A step is three kinetic
// passes, one per axis (FFT, e^{-i k_a^2 dt/2}, inverse FFT), and three strip
// passes that apply the Crank-Nicolson factor of one axis on its ECS strip
// only (the nodes where C_a has a row, about a fifth of each axis).  The
// kinetic half-steps of consecutive steps are merged, as in 2D, and the two
// potential half-steps are fused into the kinetic passes around the strip
// passes: the z pass multiplies by e^{-iU dt/2} after its transforms, the x
// pass of the next step before them.  In time order:
//   Kx/2 Ky/2 [Kz/2, U/2] ( CNx CNy CNz [U/2, Kx] Ky [Kz, U/2] )... CNx CNy CNz [U/2, Kx/2] Ky/2 Kz/2
#include <algorithm>

#include "internal.hpp"
#include "line_fft.hpp"
#include "lines3d.hpp"
#include "passes.hpp"
#include "potential.hpp"

namespace sofft {
namespace {

template <typename T>
struct Pass3 {
  cx<T>* psi;
  int nx, ny, nz;
  int nlines;                 // lines of the pass: the product of the two other axis lengths
  const cx<double>* tw;       // twiddles of the pass axis
  const cx<double>* kin;      // kinetic phase of the pass axis (1/n folded in)
  // exp(-i U dt/2) with U = V0 + f W: the V0 factor from vph (the octant
  // [nz/2][ny/2][nx/2] of the soft-core, read at vfold of each index, or the
  // whole grid for a caller's V0), the field factor from W (null: W = x)
  const cx<double>* vph;
  int vfull;
  const double* w;
  const double* x;
  const double* f_mid;
  int64_t pre_step, post_step;   // field index of the factor before / after the transforms; < 0: none
  double ht;                     // dt/2
};

template <typename T>
__device__ __forceinline__ cx<double> phase3(const Pass3<T>& a, int x, int y, int z, double f) {
  cx<double> v{1.0, 0.0};
  if (a.vph)
    v = a.vfull ? a.vph[idx3(x, y, z, a.nx, a.ny)]
                : a.vph[idx3(vfold(x, a.nx), vfold(y, a.ny), vfold(z, a.nz), a.nx / 2, a.ny / 2)];
  const double W = a.w ? a.w[idx3(x, y, z, a.nx, a.ny)] : a.x[x];
  return cmul(v, expi(f * W * a.ht, 0.0));
}

// Kinetic pass along AXIS: [potential factor], FFT, e^{-i k^2 dt/2}, inverse
// FFT, [potential factor].  The row pass keeps a line's threads consecutive
// (its exchanges stay within a wavefront when the line does); the strided
// passes interleave the lines of a block so that neighbouring threads load
// neighbouring x.
template <typename T, int N, int AXIS>
__global__ void __launch_bounds__(k3_threads<N>()) k3_kinetic(Pass3<T> a) {
  constexpr int P = Shape<N>::P, TPL = N / P, LPB = k3_lines<N>(), E = fft_lds_elems<N>();
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* lds = reinterpret_cast<cx<double>*>(smem);
  int c, t;
  if constexpr (AXIS == 0) {
    c = threadIdx.x / TPL;
    t = threadIdx.x - c * TPL;
  } else {
    c = threadIdx.x % LPB;
    t = threadIdx.x / LPB;
  }
  // Each XCD takes one contiguous band of the pass's lines (workgroups go
  // round-robin over the 8 XCDs): measured 2.5% (complex128) and 4%
  // (complex64) faster per 256^3 step than block b on lines 8b..8b+7, and
  // faster than groups of 2 or 4 blocks per XCD slot.
  const int nb = gridDim.x, b = blockIdx.x;
  const int bb = nb % 8 ? b : (b % 8) * (nb / 8) + b / 8;
  const int g = bb * LPB + c;
  const bool live = g < a.nlines;
  int lx, ly, lz;
  size_t ld;
  line_origin<AXIS>(live ? g : 0, a.nx, a.ny, lx, ly, lz, ld);
  cx<T>* base = a.psi + idx3(lx, ly, lz, a.nx, a.ny);
  cx<double> v[P];
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = widen(gload(base + size_t(t + TPL * s) * ld));
  if (a.pre_step >= 0) {
    const double f = a.f_mid ? a.f_mid[a.pre_step] : 0.0;
#pragma unroll
    for (int s = 0; s < P; ++s) {
      int x, y, z;
      node_of<AXIS>(t + TPL * s, lx, ly, lz, x, y, z);
      v[s] = cmul(v[s], phase3(a, x, y, z, f));
    }
  }
  cx<double> kin[P];
#pragma unroll
  for (int s = 0; s < P; ++s) kin[s] = a.kin[t + TPL * s];
  constexpr bool wave = AXIS == 0 && TPL <= 64 && 64 % TPL == 0;
  const LineLDS<double> L = AXIS == 0 ? LineLDS<double>{lds, c * 2 * E, 1} : LineLDS<double>{lds, c, LPB};
  const LineLDS<double> Lb = AXIS == 0 ? LineLDS<double>{lds, c * 2 * E + E, 1} : LineLDS<double>{lds, c + E * LPB, LPB};
  constexpr bool swz = AXIS == 0 && fft2_swizzle<N>();   // x lines are contiguous in LDS
  fft2<double, N, -1, wave, swz>(v, L, Lb, t, a.tw);
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = cmul(v[s], kin[s]);
  fft2<double, N, +1, wave, swz>(v, L, Lb, t, a.tw);
  if (a.post_step >= 0) {
    const double f = a.f_mid ? a.f_mid[a.post_step] : 0.0;
#pragma unroll
    for (int s = 0; s < P; ++s) {
      int x, y, z;
      node_of<AXIS>(t + TPL * s, lx, ly, lz, x, y, z);
      v[s] = cmul(v[s], phase3(a, x, y, z, f));
    }
  }
  if (live) {
#pragma unroll
    for (int s = 0; s < P; ++s) gstore(base + size_t(t + TPL * s) * ld, narrow<T>(v[s]));
  }
}

// Crank-Nicolson on the ECS strip of every line along AXIS: y = 2 B^-1 v - v
// with B = 1 + i dt C/2 by parallel cyclic reduction (pcr_line), one
// wavefront per line, eight lines per block.  Only the strip nodes are read
// and written.  Loads and stores map neighbouring threads to neighbouring
// addresses (along the row for AXIS 0, across the eight adjacent lines
// otherwise); the reduction reads the strips from LDS, laid out per line with
// an odd stride 2m + 1.
constexpr int kCnLines = 8;

template <typename T, int N, int AXIS>
__global__ void __launch_bounds__(64 * kCnLines) k3_cn(Pass3<T> a, PassArgs<T> cn) {
  constexpr int G = kPcrGroups;   // strip positions per loading thread: m <= 256 = 64 G
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* lds = reinterpret_cast<cx<double>*>(smem);
  const int m = cn.m, stride = 2 * m + 1;
  int c, r;
  if constexpr (AXIS == 0) {
    c = threadIdx.x >> 6;
    r = threadIdx.x & 63;
  } else {
    c = threadIdx.x % kCnLines;
    r = threadIdx.x / kCnLines;
  }
  const int nbk = gridDim.x, bk = blockIdx.x;   // one band of lines per XCD, as the kinetic passes
  const int g = (nbk % 8 ? bk : (bk % 8) * (nbk / 8) + bk / 8) * kCnLines + c;
  const bool live = g < a.nlines;
  int lx, ly, lz;
  size_t ld;
  line_origin<AXIS>(live ? g : 0, a.nx, a.ny, lx, ly, lz, ld);
  cx<T>* base = a.psi + idx3(lx, ly, lz, a.nx, a.ny);
  cx<double> v[G];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    const int p = min(r + 64 * i, m - 1);   // clamped: in bounds for every lane
    v[i] = widen(gload(base + size_t((cn.j0 + p) % N) * ld));
    if (r + 64 * i < m) lds[c * stride + r + 64 * i] = v[i];
  }
  __syncthreads();
  {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    pcr_line<T, N>(LineLDS<double>{lds, w * stride, 1}, lane, 0, 1, cn);
  }
  __syncthreads();
  const int res = cn_result(m, cn.levels);
  if (live) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int p = r + 64 * i;
      if (p < m) gstore(base + size_t((cn.j0 + p) % N) * ld, narrow<T>(2.0 * lds[c * stride + res + p] - v[i]));
    }
  }
}

// exp(-i V0 dt/2) of the soft-core on the octant of nodes j < n/2 per axis.
__global__ void __launch_bounds__(256) k3_vphase(cx<double>* out, int hx, int hy, int hz, const cx<double>* zx,
                                                 const cx<double>* zy, const cx<double>* zz, double charge, double a2,
                                                 double ht) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= size_t(hx) * hy * hz) return;
  const int jx = int(i % hx), jy = int((i / hx) % hy), jz = int(i / (size_t(hx) * hy));
  const cx<double> s = cmul(zx[jx], zx[jx]) + cmul(zy[jy], zy[jy]) + cmul(zz[jz], zz[jz]) + cx<double>{a2, 0.0};
  out[i] = potential_phase(s, charge, 0.0, ht);
}

// The soft-core V0 = -charge / sqrt(z_x^2 + z_y^2 + z_z^2 + a2) on the whole grid.
__global__ void __launch_bounds__(256) k3_softcore(cx<double>* out, int nx, int ny, int nz, const cx<double>* zx,
                                                   const cx<double>* zy, const cx<double>* zz, double charge,
                                                   double a2) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= size_t(nx) * ny * nz) return;
  const int jx = int(i % nx), jy = int((i / nx) % ny), jz = int(i / (size_t(nx) * ny));
  const cx<double> s = cmul(zx[jx], zx[jx]) + cmul(zy[jy], zy[jy]) + cmul(zz[jz], zz[jz]) + cx<double>{a2, 0.0};
  out[i] = potential_value(s, charge, 0.0);
}

// ---------------------------------------------------------------- launchers

constexpr size_t kLds3Budget = 150 * 1024;

template <typename K>
sofft_status lds3(K kernel, size_t bytes) {
  return bytes > 65536 ? raise_lds_limit(reinterpret_cast<const void*>(kernel), kLds3Budget) : SOFFT_OK;
}

template <typename T, int N, int AXIS>
sofft_status kinetic_n(const Pass3<T>& a, hipStream_t s, Timing* tm) {
  constexpr int LPB = k3_lines<N>();
  const size_t lds = size_t(LPB) * 2 * fft_lds_elems<N>() * sizeof(cx<double>);
  sofft_status st = lds3(k3_kinetic<T, N, AXIS>, lds);
  if (st != SOFFT_OK) return st;
  const int blocks = (a.nlines + LPB - 1) / LPB;
  if ((st = tm->begin(SOFFT_KERNEL_3D_KINETIC, s)) != SOFFT_OK) return st;
  k3_kinetic<T, N, AXIS><<<blocks, k3_threads<N>(), lds, s>>>(a);
  SOFFT_HIP_TRY(hipGetLastError());
  return tm->end(s);
}

template <typename T, int N, int AXIS>
sofft_status cn_n(const Pass3<T>& a, const PassArgs<T>& cn, hipStream_t s, Timing* tm) {
  const size_t lds = size_t(kCnLines) * (2 * cn.m + 1) * sizeof(cx<double>);
  sofft_status st = lds3(k3_cn<T, N, AXIS>, lds);
  if (st != SOFFT_OK) return st;
  const int blocks = (a.nlines + kCnLines - 1) / kCnLines;
  if ((st = tm->begin(SOFFT_KERNEL_3D_STRIP, s)) != SOFFT_OK) return st;
  k3_cn<T, N, AXIS><<<blocks, 64 * kCnLines, lds, s>>>(a, cn);
  SOFFT_HIP_TRY(hipGetLastError());
  return tm->end(s);
}

template <typename T, int AXIS>
sofft_status kinetic(int n, const Pass3<T>& a, hipStream_t s, Timing* tm) {
  SOFFT_3D_SWITCH(n, (kinetic_n<T, N_, AXIS>(a, s, tm)))
  set_error("unsupported 3D line length");
  return SOFFT_EUNSUPPORTED;
}

template <typename T, int AXIS>
sofft_status cn(int n, const Pass3<T>& a, const PassArgs<T>& c, hipStream_t s, Timing* tm) {
  SOFFT_3D_SWITCH(n, (cn_n<T, N_, AXIS>(a, c, s, tm)))
  set_error("unsupported 3D line length");
  return SOFFT_EUNSUPPORTED;
}

template <typename T>
sofft_status propagate_3d(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                          const cx<double>* vph, hipStream_t s) {
  const int n[3] = {int(p.ax[0].n), int(p.ax[1].n), int(p.ax[2].n)};
  Pass3<T> a{};
  a.psi = static_cast<cx<T>*>(psi);
  a.nx = n[0];
  a.ny = n[1];
  a.nz = n[2];
  a.vph = vph;
  a.vfull = p.user_v0 != nullptr;
  a.w = p.user_w;
  a.x = static_cast<const double*>(p.ax[0].x_dev.p);
  a.f_mid = f_mid;
  a.ht = 0.5 * dt;
  // The potential factors are skipped when there is neither V0 nor a field.
  const bool pot = vph != nullptr || f_mid != nullptr;
  Pass3<T> ax[3];
  PassArgs<T> cnargs[3];
  for (int d = 0; d < 3; ++d) {
    ax[d] = a;
    ax[d].nlines = n[(d + 1) % 3] * n[(d + 2) % 3];
    ax[d].tw = static_cast<const cx<double>*>(p.ax[d].tw64.p);
    ax[d].pre_step = ax[d].post_step = -1;
    PassArgs<T>& c = cnargs[d];
    c = PassArgs<T>{};
    c.j0 = int(p.ax[d].j0);
    c.m = int(p.ax[d].m);
    c.levels = p.ax[d].levels;
    c.alpha = static_cast<const cx<double>*>(p.ax[d].alpha64.p);
    c.gamma = static_cast<const cx<double>*>(p.ax[d].gamma64.p);
    c.binv = static_cast<const cx<double>*>(p.ax[d].binv64.p);
  }
  auto kin_table = [&](int d, bool half) {
    return static_cast<const cx<double>*>(half ? p.ax[d].kin_half64.p : p.ax[d].kin_full64.p);
  };
  // The three kinetic passes of one merged K factor; pre / post: field index
  // of the potential factor before the x pass / after the z pass (< 0: none).
  auto kinetic_group = [&](bool half, int64_t pre, int64_t post) -> sofft_status {
    Pass3<T> qx = ax[0], qy = ax[1], qz = ax[2];
    qx.kin = kin_table(0, half);
    qy.kin = kin_table(1, half);
    qz.kin = kin_table(2, half);
    qx.pre_step = pot ? pre : -1;
    qz.post_step = pot ? post : -1;
    sofft_status st = kinetic<T, 0>(n[0], qx, s, &p.timing);
    if (st == SOFFT_OK) st = kinetic<T, 1>(n[1], qy, s, &p.timing);
    if (st == SOFFT_OK) st = kinetic<T, 2>(n[2], qz, s, &p.timing);
    return st;
  };
  auto cn_all = [&]() -> sofft_status {
    sofft_status st = SOFFT_OK;
    if (st == SOFFT_OK && cnargs[0].m > 0) st = cn<T, 0>(n[0], ax[0], cnargs[0], s, &p.timing);
    if (st == SOFFT_OK && cnargs[1].m > 0) st = cn<T, 1>(n[1], ax[1], cnargs[1], s, &p.timing);
    if (st == SOFFT_OK && cnargs[2].m > 0) st = cn<T, 2>(n[2], ax[2], cnargs[2], s, &p.timing);
    return st;
  };
  sofft_status st = kinetic_group(true, -1, 0);
  for (int64_t k = 0; k < nsteps && st == SOFFT_OK; ++k) {
    st = cn_all();
    if (st != SOFFT_OK) break;
    const bool last = k + 1 == nsteps;
    st = kinetic_group(last, k, last ? -1 : k + 1);
  }
  return st;
}

}  // namespace

// exp(-i V0 dt/2) of the soft-core on the octant [nz/2][ny/2][nx/2].
sofft_status build_octant_vphase(const Plan& p, double dt, cx<double>* table, hipStream_t s) {
  const size_t nx = size_t(p.ax[0].n), ny = size_t(p.ax[1].n), nz = size_t(p.ax[2].n);
  const size_t n = (nx / 2) * (ny / 2) * (nz / 2);
  k3_vphase<<<unsigned((n + 255) / 256), 256, 0, s>>>(
      table, int(nx / 2), int(ny / 2), int(nz / 2), static_cast<const cx<double>*>(p.ax[0].z_dev.p),
      static_cast<const cx<double>*>(p.ax[1].z_dev.p), static_cast<const cx<double>*>(p.ax[2].z_dev.p),
      p.prob.charge, p.prob.a2, 0.5 * dt);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

sofft_status launch_softcore_3d(const Plan& p, double charge, double a2, void* out, hipStream_t s) {
  const int nx = int(p.ax[0].n), ny = int(p.ax[1].n), nz = int(p.ax[2].n);
  const size_t n = size_t(nx) * ny * nz;
  k3_softcore<<<unsigned((n + 255) / 256), 256, 0, s>>>(
      static_cast<cx<double>*>(out), nx, ny, nz, static_cast<const cx<double>*>(p.ax[0].z_dev.p),
      static_cast<const cx<double>*>(p.ax[1].z_dev.p), static_cast<const cx<double>*>(p.ax[2].z_dev.p), charge, a2);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

sofft_status launch_propagate_3d(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                 const cx<double>* vph, hipStream_t s) {
  return p.prob.dtype == SOFFT_C128 ? propagate_3d<double>(p, psi, dt, nsteps, f_mid, vph, s)
                                    : propagate_3d<float>(p, psi, dt, nsteps, f_mid, vph, s);
}

}  // namespace sofft
