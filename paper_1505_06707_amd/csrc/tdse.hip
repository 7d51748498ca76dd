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

#include "fft_line.hpp"
#include "internal.hpp"

namespace sofft {

template <typename T>
struct PassArgs {
  cx<T>* psi;
  int nx, ny;
  const cx<T>* tw;    // twiddles exp(-2 pi i u/n) of the pass axis
  const cx<T>* kin;   // kinetic phase (with 1/n) of the pass axis
  int do_pot;         // apply the potential half-step and the CN sweep
  const double* f_mid;
  int64_t step;
  double ht;          // dt/2
  double charge, a2;
  const double* x;        // x nodes
  const cx<double>* zx;   // z(x_j)
  const cx<double>* zy;   // z(y_j) (2D) or null
  int j0, m, levels;      // ECS strip of the pass axis
  const cx<T>* alpha;
  const cx<T>* gamma;
  const cx<T>* binv;
  int lds_line;           // LDS elements reserved per line
};

// exp(-i U dt/2) with U = -charge/sqrt(s) + f x, s = sum z^2 + a2 (principal
// branch), evaluated in FP64.
__device__ __forceinline__ cx<double> potential_phase(cx<double> s, double charge, double fx, double ht) {
  double ure = fx, uim = 0.0;
  if (charge != 0.0) {
    if (s.im == 0.0 && s.re > 0.0) {
      ure -= charge / sqrt(s.re);
    } else {
      const double r = hypot(s.re, s.im);
      double wr, wi;
      if (s.re >= 0.0) {
        wr = sqrt(0.5 * (r + s.re));
        wi = s.im / (2.0 * wr);
      } else {
        wi = copysign(sqrt(0.5 * (r - s.re)), s.im);
        wr = s.im / (2.0 * wi);
      }
      // -charge / w = -charge conj(w) / |w|^2, |w|^2 = r
      ure -= charge * wr / r;
      uim += charge * wi / r;
    }
  }
  double sn, cs;
  sincos(ure * ht, &sn, &cs);
  const double mag = uim == 0.0 ? 1.0 : exp(uim * ht);
  return {mag * cs, -mag * sn};
}

template <typename T>
__device__ __forceinline__ cx<T> to(cx<double> v) {
  return {T(v.re), T(v.im)};
}

// Crank-Nicolson on the ECS strip of this line: y = 2 B^-1 v - v by parallel
// cyclic reduction with the coefficients prepared on the host.  The strip is
// staged in the line's LDS storage (two buffers of m elements).
template <typename T, int N, int P>
__device__ __forceinline__ void cn_strip(cx<T> (&v)[P], const LineLDS<T>& L, int t, const PassArgs<T>& a) {
  constexpr int TPL = N / P;
  const int m = a.m;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    int p = t + TPL * s - a.j0;
    if (p < 0) p += N;
    if (p < m) L[p] = v[s];
  }
  __syncthreads();
  int src = 0, dst = m;
  for (int l = 0; l < a.levels; ++l) {
    const int st = 1 << l;
    const cx<T>* al = a.alpha + size_t(l) * m;
    const cx<T>* ga = a.gamma + size_t(l) * m;
    for (int p = t; p < m; p += TPL) {
      cx<T> d = L[src + p];
      if (p >= st) d = d - cmul(al[p], L[src + p - st]);
      if (p + st < m) d = d - cmul(ga[p], L[src + p + st]);
      L[dst + p] = d;
    }
    __syncthreads();
    const int tmp = src;
    src = dst;
    dst = tmp;
  }
#pragma unroll
  for (int s = 0; s < P; ++s) {
    int p = t + TPL * s - a.j0;
    if (p < 0) p += N;
    if (p < m) v[s] = T(2) * cmul(a.binv[p], L[src + p]) - v[s];
  }
  __syncthreads();
}

template <typename T, int N>
__global__ void __launch_bounds__(256) k_row_pass(PassArgs<T> a) {
  constexpr int P = FFTShape<N>::P, TPL = N / P, LPB = 256 / TPL;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int l = threadIdx.x / TPL, t = threadIdx.x - l * TPL;
  const int row = blockIdx.x * LPB + l;
  const bool live = row < a.ny;
  const int crow = live ? row : 0;
  const LineLDS<T> L{lds, l * a.lds_line, 1};
  cx<T>* line = a.psi + size_t(crow) * N;
  cx<T> v[P];
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = live ? line[t + TPL * s] : cx<T>{T(0), T(0)};
  fft_line<T, N, -1>(v, L, t, a.tw);
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = cmul(v[s], a.kin[t + TPL * s]);
  fft_line<T, N, +1>(v, L, t, a.tw);
  if (a.do_pot) {
    const double f = a.f_mid ? a.f_mid[a.step] : 0.0;
    const cx<double> zy = a.zy ? a.zy[crow] : cx<double>{0.0, 0.0};
    const cx<double> zy2a = cmul(zy, zy) + cx<double>{a.a2, 0.0};
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int e = t + TPL * s;
      const cx<double> zx = a.zx[e];
      const cx<double> ph = potential_phase(cmul(zx, zx) + zy2a, a.charge, f * a.x[e], a.ht);
      v[s] = cmul(v[s], to<T>(ph));
    }
    if (a.m > 0) cn_strip<T, N, P>(v, L, t, a);
  }
  if (live) {
#pragma unroll
    for (int s = 0; s < P; ++s) line[t + TPL * s] = v[s];
  }
}

template <typename T, int N>
__global__ void __launch_bounds__(256) k_col_pass(PassArgs<T> a) {
  constexpr int P = FFTShape<N>::P, TPL = N / P, C = 256 / TPL;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int col = blockIdx.x * C + c;
  const bool live = col < a.nx;
  const int ccol = live ? col : 0;
  const LineLDS<T> L{lds, c, C};
  cx<T>* base = a.psi + ccol;
  const size_t ld = size_t(a.nx);
  cx<T> v[P];
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = live ? base[size_t(t + TPL * s) * ld] : cx<T>{T(0), T(0)};
  if (a.do_pot) {
    if (a.m > 0) cn_strip<T, N, P>(v, L, t, a);
    const double f = a.f_mid ? a.f_mid[a.step] : 0.0;
    const cx<double> zx = a.zx[ccol];
    const cx<double> zx2a = cmul(zx, zx) + cx<double>{a.a2, 0.0};
    const double fx = f * a.x[ccol];
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const cx<double> zy = a.zy[t + TPL * s];
      const cx<double> ph = potential_phase(zx2a + cmul(zy, zy), a.charge, fx, a.ht);
      v[s] = cmul(v[s], to<T>(ph));
    }
  }
  fft_line<T, N, -1>(v, L, t, a.tw);
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = cmul(v[s], a.kin[t + TPL * s]);
  fft_line<T, N, +1>(v, L, t, a.tw);
  if (live) {
#pragma unroll
    for (int s = 0; s < P; ++s) base[size_t(t + TPL * s) * ld] = v[s];
  }
}

// 1D: the whole propagation in one workgroup; psi stays in registers.
template <typename T, int N>
__global__ void __launch_bounds__(N / FFTShape<N>::P) k_tdse1d(PassArgs<T> a, const cx<T>* kin_half,
                                                                const cx<T>* kin_full, int64_t nsteps) {
  constexpr int P = FFTShape<N>::P, TPL = N / P;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  const int t = threadIdx.x;
  const LineLDS<T> L{lds, 0, 1};
  cx<T> v[P];
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = a.psi[t + TPL * s];
  fft_line<T, N, -1>(v, L, t, a.tw);
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = cmul(v[s], kin_half[t + TPL * s]);
  fft_line<T, N, +1>(v, L, t, a.tw);
  for (int64_t n = 0; n < nsteps; ++n) {
    const double f = a.f_mid ? a.f_mid[n] : 0.0;
    cx<T> ph[P];
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int e = t + TPL * s;
      const cx<double> z = a.zx[e];
      ph[s] = to<T>(potential_phase(cmul(z, z) + cx<double>{a.a2, 0.0}, a.charge, f * a.x[e], a.ht));
      v[s] = cmul(v[s], ph[s]);
    }
    if (a.m > 0) cn_strip<T, N, P>(v, L, t, a);
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = cmul(v[s], ph[s]);
    const cx<T>* kin = (n + 1 == nsteps) ? kin_half : kin_full;
    fft_line<T, N, -1>(v, L, t, a.tw);
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = cmul(v[s], kin[t + TPL * s]);
    fft_line<T, N, +1>(v, L, t, a.tw);
  }
#pragma unroll
  for (int s = 0; s < P; ++s) a.psi[t + TPL * s] = v[s];
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

template <typename T>
static const cx<T>* tab(const DevBuf& b64, const DevBuf& b32) {
  return static_cast<const cx<T>*>(std::is_same<T, double>::value ? b64.p : b32.p);
}

template <typename T>
static PassArgs<T> axis_args(Plan& p, int axis, void* psi, double dt) {
  Axis& A = p.ax[axis];
  PassArgs<T> a{};
  a.psi = static_cast<cx<T>*>(psi);
  a.nx = int(p.ax[0].n);
  a.ny = p.prob.ndim == 2 ? int(p.ax[1].n) : 1;
  a.tw = tab<T>(A.tw64, A.tw32);
  a.ht = 0.5 * dt;
  a.charge = p.prob.charge;
  a.a2 = p.prob.a2;
  a.x = static_cast<const double*>(p.ax[0].x_dev.p);
  a.zx = static_cast<const cx<double>*>(p.ax[0].z_dev.p);
  a.zy = p.prob.ndim == 2 ? static_cast<const cx<double>*>(p.ax[1].z_dev.p) : nullptr;
  a.j0 = int(A.j0);
  a.m = int(A.m);
  a.levels = A.levels;
  a.alpha = tab<T>(A.alpha64, A.alpha32);
  a.gamma = tab<T>(A.gamma64, A.gamma32);
  a.binv = tab<T>(A.binv64, A.binv32);
  a.lds_line = int(std::max<int64_t>(A.n, 2 * A.m));
  return a;
}

template <typename K>
static sofft_status set_lds(K kernel, size_t bytes) {
  if (bytes > 65536) {
    SOFFT_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  }
  return SOFFT_OK;
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

template <typename T, int N>
static sofft_status row_pass(const PassArgs<T>& a, hipStream_t s) {
  constexpr int TPL = N / FFTShape<N>::P, LPB = 256 / TPL;
  const size_t lds = size_t(LPB) * a.lds_line * sizeof(cx<T>);
  sofft_status st = set_lds(k_row_pass<T, N>, lds);
  if (st != SOFFT_OK) return st;
  const int blocks = (a.ny + LPB - 1) / LPB;
  k_row_pass<T, N><<<blocks, 256, lds, s>>>(a);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

template <typename T, int N>
static sofft_status col_pass(const PassArgs<T>& a, hipStream_t s) {
  constexpr int TPL = N / FFTShape<N>::P, C = 256 / TPL;
  const size_t lds = size_t(C) * a.lds_line * sizeof(cx<T>);
  sofft_status st = set_lds(k_col_pass<T, N>, lds);
  if (st != SOFFT_OK) return st;
  const int blocks = (a.nx + C - 1) / C;
  k_col_pass<T, N><<<blocks, 256, lds, s>>>(a);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

template <typename T>
static sofft_status row_pass_n(int n, const PassArgs<T>& a, hipStream_t s) {
  SOFFT_LENGTH_SWITCH(n, row_pass, T, a, s)
  set_error("unsupported row length");
  return SOFFT_EUNSUPPORTED;
}

template <typename T>
static sofft_status col_pass_n(int n, const PassArgs<T>& a, hipStream_t s) {
  SOFFT_LENGTH_SWITCH(n, col_pass, T, a, s)
  set_error("unsupported column length");
  return SOFFT_EUNSUPPORTED;
}

template <typename T>
static sofft_status propagate_2d(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                 hipStream_t s) {
  PassArgs<T> ra = axis_args<T>(p, 0, psi, dt);
  PassArgs<T> ca = axis_args<T>(p, 1, psi, dt);
  ra.f_mid = ca.f_mid = f_mid;
  const int nx = int(p.ax[0].n), ny = int(p.ax[1].n);
  const cx<T>* kxf = tab<T>(p.ax[0].kin_full64, p.ax[0].kin_full32);
  const cx<T>* kxh = tab<T>(p.ax[0].kin_half64, p.ax[0].kin_half32);
  const cx<T>* kyf = tab<T>(p.ax[1].kin_full64, p.ax[1].kin_full32);
  const cx<T>* kyh = tab<T>(p.ax[1].kin_half64, p.ax[1].kin_half32);
  sofft_status st;
  // opening K_y/2
  ca.do_pot = 0;
  ca.kin = kyh;
  if ((st = col_pass_n<T>(ny, ca, s)) != SOFFT_OK) return st;
  ra.do_pot = ca.do_pot = 1;
  for (int64_t n = 0; n < nsteps; ++n) {
    ra.step = ca.step = n;
    ra.kin = n == 0 ? kxh : kxf;
    ca.kin = n + 1 == nsteps ? kyh : kyf;
    if ((st = row_pass_n<T>(nx, ra, s)) != SOFFT_OK) return st;
    if ((st = col_pass_n<T>(ny, ca, s)) != SOFFT_OK) return st;
  }
  // closing K_x/2
  ra.do_pot = 0;
  ra.kin = kxh;
  return row_pass_n<T>(nx, ra, s);
}

template <typename T, int N>
static sofft_status tdse1d(Plan& p, const PassArgs<T>& a, int64_t nsteps, hipStream_t s) {
  constexpr int TPL = N / FFTShape<N>::P;
  const size_t lds = size_t(a.lds_line) * sizeof(cx<T>);
  sofft_status st = set_lds(k_tdse1d<T, N>, lds);
  if (st != SOFFT_OK) return st;
  const Axis& A = p.ax[0];
  k_tdse1d<T, N><<<1, TPL, lds, s>>>(a, tab<T>(A.kin_half64, A.kin_half32), tab<T>(A.kin_full64, A.kin_full32),
                                    nsteps);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

template <typename T>
static sofft_status propagate_1d(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                 hipStream_t s) {
  PassArgs<T> a = axis_args<T>(p, 0, psi, dt);
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

sofft_status launch_propagate_1d(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                 hipStream_t s) {
  return p.prob.dtype == SOFFT_C128 ? propagate_1d<double>(p, psi, dt, nsteps, f_mid, s)
                                    : propagate_1d<float>(p, psi, dt, nsteps, f_mid, s);
}

sofft_status launch_propagate_2d(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                 hipStream_t s) {
  return p.prob.dtype == SOFFT_C128 ? propagate_2d<double>(p, psi, dt, nsteps, f_mid, s)
                                    : propagate_2d<float>(p, psi, dt, nsteps, f_mid, s);
}

sofft_status launch_norm2(Plan& p, const void* psi, double* out, hipStream_t s) {
  int64_t n = p.ax[0].n * (p.prob.ndim == 2 ? p.ax[1].n : 1);
  const int blocks = int(std::min<int64_t>(1024, (n + 255) / 256));
  if (!p.partials.p || p.partials.bytes < blocks * sizeof(double)) {
    dev_free(p.partials);
    if (hipMalloc(&p.partials.p, 1024 * sizeof(double)) != hipSuccess) {
      p.partials.p = nullptr;
      set_error("hipMalloc failed");
      return SOFFT_ENOMEM;
    }
    p.partials.bytes = 1024 * sizeof(double);
  }
  double* part = static_cast<double*>(p.partials.p);
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

}  // namespace sofft
