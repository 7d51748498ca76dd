// Stationary equation with ECS in 1D (Sec. III, the setting of the paper's
// own numerical example in Sec. V) and its preconditioned COCG solve.
//
// A line of at most 4096 points fits one workgroup, so each energy is one
// workgroup that runs the whole solve on chip: x, r and p stay in registers
// (element t + TPL s of the line in slot s of thread t), the transforms and
// the neighbours of C go through LDS, and the bilinear forms are FP64 block
// sums in a fixed order.  One launch solves every energy; nothing returns to
// the host until all have finished.  Lines of fewer than 256 points have
// fewer than 64 threads: the block is then one wavefront of G = 64/TPL groups
// that each work on their own LDS copy of the line (the same values); only
// group 0 enters the sums and stores the result.
//   A v   = F^-1 (k^2/2) F v + C v + (U - E) v                 (Eq. linsys)
//   P^-1 r = F^-1 (k^2/2 - E)^-1 F r                             (Eq. PreconFFT)
//          = F^-1 (k^2/2 - E - i eta)^-1 F r                     (shifted divisor)
//          = F^-1 X^T (lambda - E)^-1 X F r                      (Eq. PreconFFT_ECS)
// The iteration is that of the batched 2D/3D solver: COCG with the
// unconjugated form, stop when ||r|| <= rtol ||f||, then the true residual
// f - A x, restarting from it while it exceeds rtol (also after kStallIters
// iterations without a new minimum of ||r||), at most kMaxRestarts restarts.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "line_fft.hpp"
#include "potential.hpp"
#include "sse.hpp"

namespace sofft {
namespace {

struct Sse1Args {
  int n, nE;
  int mode;                    // 0 solve; 1 w = A v; 2 w = P^-1 v (energy 0, v in f, w in x)
  const cx<double>* f;         // right-hand side [n] (shared) or [nE][n]
  int f_per_energy;
  cx<double>* x;               // [nE][n]
  const double* E;             // [nE]
  const double* eta;           // [nE] or null
  double rtol;
  int maxit;
  // U = V0(z) + field x, or a caller's V0 and W
  const cx<double>* z;
  const double* xg;
  const cx<double>* v0;
  const double* w;
  double charge, a2, field;
  const cx<double>* tw;
  double L;
  int j0, m;
  const cx<double>* cstrip;
  int banded;
  const cx<double>* lam;
  const cx<double>* xr;
  const cx<double>* xc;
  const int* bstart;
  const int* bwidth;
  sofft_solve_stats* stats;    // [nE], device
};

// Sum over the block, returned to every thread (block_sum, then a broadcast
// through red[0]).
__device__ __forceinline__ cx<double> block_sum_all(cx<double> v, cx<double>* red) {
  const cx<double> s = block_sum(v, red);
  __syncthreads();
  if (threadIdx.x == 0) red[0] = s;
  __syncthreads();
  const cx<double> out = red[0];
  __syncthreads();
  return out;
}

// Groups of TPL threads per block (whole wavefronts).
template <int N>
constexpr int sse1_groups() {
  constexpr int tpl = N / Shape<N>::P;
  return tpl >= 64 ? 1 : 64 / tpl;
}

// w = A v for the line held in v (element t + TPL s), U - E in um.
template <int N>
__device__ __forceinline__ void apply_A(const cx<double> (&v)[Shape<N>::P], cx<double> (&w)[Shape<N>::P],
                                        const cx<double> (&um)[Shape<N>::P], const LineLDS<double>& L, int t,
                                        const Sse1Args& a) {
  constexpr int P = Shape<N>::P, TPL = N / P;
  cx<double> q[P];
#pragma unroll
  for (int s = 0; s < P; ++s) {
    w[s] = cmul(um[s], v[s]);
    q[s] = v[s];
  }
  if (a.m > 0) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < P; ++s) L[t + TPL * s] = v[s];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < P; ++s) w[s] = w[s] + c_apply(L, t + TPL * s, N, a.j0, a.m, a.cstrip);
  }
  __syncthreads();
  fft<double, N, -1>(q, L, t, a.tw);
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const double k = kval(t + TPL * s, N, a.L);
    q[s] = (0.5 * k * k / N) * q[s];
  }
  fft<double, N, +1>(q, L, t, a.tw);
#pragma unroll
  for (int s = 0; s < P; ++s) w[s] = w[s] + q[s];
}

// z = P^-1 r.
template <int N, bool BANDED>
__device__ __forceinline__ void apply_P(const cx<double> (&r)[Shape<N>::P], cx<double> (&z)[Shape<N>::P],
                                        const LineLDS<double>& L, int t, double E, double eta, const Sse1Args& a) {
  constexpr int P = Shape<N>::P, TPL = N / P;
#pragma unroll
  for (int s = 0; s < P; ++s) z[s] = r[s];
  __syncthreads();
  fft<double, N, -1>(z, L, t, a.tw);
  constexpr double scale = 1.0 / N;
  if constexpr (BANDED) {
    band_apply<N>(z, L, t, a.xr, a.bstart, a.bwidth);   // X
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const cx<double> d = a.lam[t + TPL * s] - cx<double>{E, 0.0};
      const double q = scale / (d.re * d.re + d.im * d.im);
      z[s] = cmul(z[s], cx<double>{q * d.re, -q * d.im});
    }
    band_apply<N>(z, L, t, a.xc, a.bstart, a.bwidth);   // X^T
  } else {
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const double k = kval(t + TPL * s, N, a.L);
      const double d = 0.5 * k * k - E;   // (K - E), as printed in Eq. PreconFFT
      if (eta == 0.0) {
        z[s] = (scale / d) * z[s];
      } else {
        const double q = scale / (d * d + eta * eta);   // 1/(d - i eta)
        z[s] = cmul(z[s], cx<double>{q * d, q * eta});
      }
    }
  }
  fft<double, N, +1>(z, L, t, a.tw);
}

// u^T v (unconjugated) and ||u||^2 over the line, to every thread; only
// group 0 (own = true) contributes.
template <int N>
__device__ __forceinline__ cx<double> dot_all(const cx<double> (&u)[Shape<N>::P], const cx<double> (&v)[Shape<N>::P],
                                              bool own, cx<double>* red) {
  cx<double> d{0.0, 0.0};
#pragma unroll
  for (int s = 0; s < Shape<N>::P; ++s) d = cfma(d, u[s], v[s]);
  return block_sum_all(own ? d : cx<double>{0.0, 0.0}, red);
}

template <int N>
__device__ __forceinline__ double norm2_all(const cx<double> (&u)[Shape<N>::P], bool own, cx<double>* red) {
  double d = 0.0;
#pragma unroll
  for (int s = 0; s < Shape<N>::P; ++s) d += u[s].re * u[s].re + u[s].im * u[s].im;
  return block_sum_all(cx<double>{own ? d : 0.0, 0.0}, red).re;
}

template <int N, bool BANDED>
__global__ void __launch_bounds__(N / Shape<N>::P * sse1_groups<N>()) k_sse1d(Sse1Args a) {
  constexpr int P = Shape<N>::P, TPL = N / P, G = sse1_groups<N>(), LINE = fft_lds_elems<N>();
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* lds = reinterpret_cast<cx<double>*>(smem);   // [G lines][block-sum scratch]
  cx<double>* red = lds + G * LINE;
  const int g = threadIdx.x / TPL, t = threadIdx.x - g * TPL, e = blockIdx.x;
  const bool own = g == 0;
  const LineLDS<double> L{lds, g * LINE, 1};
  const double E = a.E[e];
  const double eta = a.eta ? a.eta[e] : 0.0;
  cx<double> um[P];   // U - E
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int j = t + TPL * s;
    const double fw = a.field * (a.w ? a.w[j] : a.xg[j]);
    const cx<double> u = a.v0 ? a.v0[j] + cx<double>{fw, 0.0}
                              : potential_value(cmul(a.z[j], a.z[j]) + cx<double>{a.a2, 0.0}, a.charge, fw);
    um[s] = u - cx<double>{E, 0.0};
  }
  const cx<double>* f = a.f + (a.f_per_energy ? size_t(e) * N : 0);
  cx<double>* xo = a.x + size_t(e) * N;
  cx<double> x[P], r[P], p[P], w[P];
  if (a.mode != 0) {   // one application to f: A (mode 1) or P^-1 (mode 2)
#pragma unroll
    for (int s = 0; s < P; ++s) r[s] = f[t + TPL * s];
    if (a.mode == 1)
      apply_A<N>(r, w, um, L, t, a);
    else
      apply_P<N, BANDED>(r, w, L, t, E, eta, a);
    if (own) {
#pragma unroll
      for (int s = 0; s < P; ++s) xo[t + TPL * s] = w[s];
    }
    return;
  }
#pragma unroll
  for (int s = 0; s < P; ++s) {
    r[s] = f[t + TPL * s];
    x[s] = {0.0, 0.0};
  }
  const double ff = norm2_all<N>(r, own, red);
  int iters = 0, restarts = 0, status = SOFFT_OK;
  double true_res = 0.0, rr = ff;
  if (ff > 0.0) {
    const double tol2 = a.rtol * a.rtol * ff;
    for (;;) {   // one recurrence from the current residual r
      apply_P<N, BANDED>(r, p, L, t, E, eta, a);   // p = z
      cx<double> rho = dot_all<N>(r, p, own, red);
      double best = rr;
      int since = 0;
      bool check = false;
      while (!check) {
        apply_A<N>(p, w, um, L, t, a);
        const cx<double> pw = dot_all<N>(p, w, own, red);
        if (pw.re * pw.re + pw.im * pw.im == 0.0) {
          status = SOFFT_BREAKDOWN;
          break;
        }
        const cx<double> alpha = cdiv(rho, pw);
#pragma unroll
        for (int s = 0; s < P; ++s) {
          x[s] = cfma(x[s], alpha, p[s]);
          r[s] = r[s] - cmul(alpha, w[s]);
        }
        rr = norm2_all<N>(r, own, red);
        ++iters;
        if (rr <= tol2) break;
        if (iters >= a.maxit) {
          status = SOFFT_NOT_CONVERGED;
          true_res = sqrt(rr / ff);
          break;
        }
        if (rr < best) {
          best = rr;
          since = 0;
        } else if (++since >= kStallIters) {
          check = true;   // stagnated: restart from the true residual
          break;
        }
        cx<double> z[P];
        apply_P<N, BANDED>(r, z, L, t, E, eta, a);
        const cx<double> rho1 = dot_all<N>(r, z, own, red);
        if (rho.re * rho.re + rho.im * rho.im == 0.0) {
          status = SOFFT_BREAKDOWN;
          break;
        }
        const cx<double> beta = cdiv(rho1, rho);
        rho = rho1;
#pragma unroll
        for (int s = 0; s < P; ++s) p[s] = cfma(z[s], beta, p[s]);
      }
      if (status != SOFFT_OK) break;
      // true residual r = f - A x
      apply_A<N>(x, w, um, L, t, a);
#pragma unroll
      for (int s = 0; s < P; ++s) r[s] = f[t + TPL * s] - w[s];
      rr = norm2_all<N>(r, own, red);
      true_res = sqrt(rr / ff);
      if (rr <= tol2) break;
      if (iters >= a.maxit || restarts >= kMaxRestarts) {
        status = SOFFT_NOT_CONVERGED;
        break;
      }
      ++restarts;
    }
    if (status == SOFFT_BREAKDOWN) true_res = sqrt(rr / ff);
  }
  if (own) {
#pragma unroll
    for (int s = 0; s < P; ++s) xo[t + TPL * s] = x[s];
  }
  if (threadIdx.x == 0) {
    sofft_solve_stats st{};
    st.iterations = iters;
    st.status = status;
    st.restarts = restarts;
    st.fell_back = 0;
    st.rel_residual = true_res;
    a.stats[e] = st;
  }
}

template <int N>
sofft_status launch1(const Sse1Args& a, hipStream_t s) {
  constexpr int G = sse1_groups<N>(), TPL = N / Shape<N>::P * G;   // threads per block
  const size_t lds = (size_t(G) * fft_lds_elems<N>() + TPL / 64) * sizeof(cx<double>);
  if (a.banded) {
    if (lds > 65536) {
      const sofft_status st = raise_lds_limit(reinterpret_cast<const void*>(k_sse1d<N, true>), 150 * 1024);
      if (st != SOFFT_OK) return st;
    }
    k_sse1d<N, true><<<a.nE, TPL, lds, s>>>(a);
  } else {
    if (lds > 65536) {
      const sofft_status st = raise_lds_limit(reinterpret_cast<const void*>(k_sse1d<N, false>), 150 * 1024);
      if (st != SOFFT_OK) return st;
    }
    k_sse1d<N, false><<<a.nE, TPL, lds, s>>>(a);
  }
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

sofft_status launch1_n(int64_t n, const Sse1Args& a, hipStream_t s) {
  switch (n) {
#define SOFFT_SSE1_CASE(N) \
  case N:                  \
    return launch1<N>(a, s);
    SOFFT_SSE1_CASE(16) SOFFT_SSE1_CASE(32) SOFFT_SSE1_CASE(48) SOFFT_SSE1_CASE(64) SOFFT_SSE1_CASE(96)
    SOFFT_SSE1_CASE(128) SOFFT_SSE1_CASE(192) SOFFT_SSE1_CASE(256) SOFFT_SSE1_CASE(384) SOFFT_SSE1_CASE(512)
    SOFFT_SSE1_CASE(768) SOFFT_SSE1_CASE(1024) SOFFT_SSE1_CASE(2048) SOFFT_SSE1_CASE(4096)
#undef SOFFT_SSE1_CASE
    default:
      set_error("no 1D stationary-solver kernel for n = " + std::to_string(n));
      return SOFFT_EUNSUPPORTED;
  }
}

size_t r256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

bool sse1_supported(int64_t n) {
  switch (n) {
    case 16: case 32: case 48: case 64: case 96: case 128: case 192: case 256: case 384: case 512: case 768:
    case 1024: case 2048: case 4096:
      return true;
    default:
      return false;
  }
}

size_t sse1_solver_bytes(int nE) {
  return r256(sizeof(sofft_solve_stats) * nE) + 2 * r256(sizeof(double) * nE);
}

// Solve (mode 0), or one application to f (mode 1: A, mode 2: P^-1, energy
// E_host[0], result in x_out), on a 1D complex128 plan.
sofft_status sse1_run(Plan& p, int mode, const void* f, int f_per_energy, const double* E_host, int nE, double field,
                      void* x_out, double rtol, int maxit, sofft_solve_stats* stats, hipStream_t s,
                      const double* eta_host, int banded) {
  WsLayout WL;
  sofft_status st = plan_ws_check(p, nE, &WL);
  if (st != SOFFT_OK) return st;
  char* q = ws_at(p, WL.solver);
  sofft_solve_stats* st_dev = reinterpret_cast<sofft_solve_stats*>(q);
  q += r256(sizeof(sofft_solve_stats) * nE);
  double* E_dev = reinterpret_cast<double*>(q);
  q += r256(sizeof(double) * nE);
  double* eta_dev = reinterpret_cast<double*>(q);
  Axis& X = p.ax[0];
  if (banded && (st = ensure_bands(X)) != SOFFT_OK) return st;
  SOFFT_HIP_TRY(hipMemcpyAsync(E_dev, E_host, sizeof(double) * nE, hipMemcpyHostToDevice, s));
  if (eta_host) SOFFT_HIP_TRY(hipMemcpyAsync(eta_dev, eta_host, sizeof(double) * nE, hipMemcpyHostToDevice, s));
  Sse1Args a{};
  a.n = int(X.n);
  a.nE = nE;
  a.mode = mode;
  a.f = static_cast<const cx<double>*>(f);
  a.f_per_energy = f_per_energy;
  a.x = static_cast<cx<double>*>(x_out);
  a.E = E_dev;
  a.eta = eta_host ? eta_dev : nullptr;
  a.rtol = rtol;
  a.maxit = maxit;
  a.z = static_cast<const cx<double>*>(X.z_dev.p);
  a.xg = static_cast<const double*>(X.x_dev.p);
  a.v0 = static_cast<const cx<double>*>(p.user_v0);
  a.w = p.user_w;
  a.charge = p.prob.charge;
  a.a2 = p.prob.a2;
  a.field = field;
  a.tw = static_cast<const cx<double>*>(X.tw64.p);
  a.L = X.L;
  a.j0 = int(X.j0);
  a.m = int(X.m);
  a.cstrip = static_cast<const cx<double>*>(X.cstrip64.p);
  a.banded = banded ? 1 : 0;
  if (banded) {
    a.lam = static_cast<const cx<double>*>(X.band_lam.p);
    a.xr = static_cast<const cx<double>*>(X.band_xr.p);
    a.xc = static_cast<const cx<double>*>(X.band_xc.p);
    a.bstart = static_cast<const int*>(X.band_start.p);
    a.bwidth = static_cast<const int*>(X.band_width.p);
  }
  a.stats = st_dev;
  Timing& tm = p.timing;
  if ((st = tm.begin(SOFFT_KERNEL_SSE_1D, s)) != SOFFT_OK) return st;
  if ((st = launch1_n(X.n, a, s)) != SOFFT_OK) return st;
  if ((st = tm.end(s)) != SOFFT_OK) return st;
  if (mode != 0) return SOFFT_OK;
  std::vector<sofft_solve_stats> host(nE);
  SOFFT_HIP_TRY(hipMemcpyAsync(host.data(), st_dev, sizeof(sofft_solve_stats) * nE, hipMemcpyDeviceToHost, s));
  SOFFT_HIP_TRY(hipStreamSynchronize(s));
  sofft_status worst = SOFFT_OK;
  for (int e = 0; e < nE; ++e) {
    if (stats) stats[e] = host[e];
    if (host[e].status != SOFFT_OK && worst == SOFFT_OK) worst = sofft_status(host[e].status);
  }
  return worst;
}

}  // namespace sofft
