// Stationary equation with ECS on 3D grids and its FFT-preconditioned COCG
// solve (Sec. III; the FFT preconditioner carries over to the many-dimensional
// case): A v = sum_a (T_a v + C_a v) + (U - E) v with T_a = F_a^-1 (k_a^2/2) F_a,
// and P^-1 r = F^-1 ((k_x^2 + k_y^2 + k_z^2)/2 - E)^-1 F r with the full 3D
// transform.
//
// The vectors are [nE][nz][ny][nx] complex128 in HBM.  The COCG iteration of
// the 2D solver (scalar steps, polling, restarts) runs unchanged; each of its
// passes becomes a sequence of line passes, one axis each:
//   K1   x: p = z + beta p, w1 = T_x p + C_x p + (U - E) p
//        y: w1 += T_y p + C_y p
//   K2   z: w = w1 + T_z p + C_z p, partial p^T w
//   K4   x: x += alpha p, r -= alpha w, partial ||r||^2, s = F_x r
//   K5   y: s = F_y s;  z: s = F_z^-1 (F_z s / (K - E)) / (nx ny nz);  y: s = F_y^-1 s
//   K6   x: z = F_x^-1 s, partial r^T z
// With the banded ECS eigen-preconditioner (Eq. PreconFFT_ECS, X = X_x (x) X_y
// (x) X_z) each forward transform is followed by the band multiply X_a of its
// axis, the divisor is lambda_x + lambda_y + lambda_z - E, and each inverse
// transform is preceded by X_a^T.
// Partial sums are one per block; a reduction kernel adds each energy's in a
// fixed order into its first slot, so the scalar steps read one value and the
// result does not depend on scheduling.
#include "internal.hpp"
#include "line_fft.hpp"
#include "lines3d.hpp"
#include "sse.hpp"

namespace sofft {
namespace {

enum Op3 : int { kMvX, kMvY, kMvZ, kUpdX, kFwdY, kDivZ, kInvY, kPrecX };

template <int OP>
constexpr int op_axis() {
  return (OP == kMvX || OP == kUpdX || OP == kPrecX) ? 0 : ((OP == kMvZ || OP == kDivZ) ? 2 : 1);
}

template <int N, int OP, bool BANDED = false>
__global__ void __launch_bounds__(k3_threads<N>()) k3_sse(SseArgs a, int want, int mode) {
  constexpr int AXIS = op_axis<OP>();
  constexpr int P = Shape<N>::P, TPL = N / P, LPB = k3_lines<N>(), E = fft_lds_elems<N>();
  const int e = blockIdx.y;
  const CocgScalars& sc = a.sc[e];
  if (sc.state != want) return;
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
  const int nlines = AXIS == 0 ? a.ny * a.nz : (AXIS == 1 ? a.nx * a.nz : a.nx * a.ny);
  // one contiguous band of lines per XCD (workgroups go round-robin over the
  // 8 XCDs): measured 5.5% faster per energy-iteration at 128^3 than block b
  // on lines LPB b ...; the block partial sums keep their block order
  const int nbk = gridDim.x, bk = blockIdx.x;
  const int g = (nbk % 8 ? bk : (bk % 8) * (nbk / 8) + bk / 8) * LPB + c;
  const bool live = g < nlines;
  int lx, ly, lz;
  size_t ld;
  line_origin<AXIS>(live ? g : 0, a.nx, a.ny, lx, ly, lz, ld);
  const size_t o = idx3(lx, ly, lz, a.nx, a.ny);   // line origin within one vector
  const size_t off = size_t(e) * a.vec + o;
  constexpr bool wave = AXIS == 0 && TPL <= 64 && 64 % TPL == 0;
  constexpr bool swz = AXIS == 0 && fft2_swizzle<N>();   // x lines are contiguous in LDS
  const LineLDS<double> L = AXIS == 0 ? LineLDS<double>{lds, c * 2 * E, 1} : LineLDS<double>{lds, c, LPB};
  const LineLDS<double> Lb =
      AXIS == 0 ? LineLDS<double>{lds, c * 2 * E + E, 1} : LineLDS<double>{lds, c + E * LPB, LPB};
  const cx<double>* tw = AXIS == 0 ? a.twx : (AXIS == 1 ? a.twy : a.twz);
  const double La = AXIS == 0 ? a.Lx : (AXIS == 1 ? a.Ly : a.Lz);
  const cx<double> zero{0.0, 0.0};
  cx<double> v[P];

  if constexpr (OP == kMvX || OP == kMvY || OP == kMvZ) {
    // ---- one axis of A v
    cx<double> acc[P];
    if (OP == kMvX && mode == kRowIter) {
      const cx<double> beta = sc.beta;
      const bool first = sc.first != 0;
#pragma unroll
      for (int s = 0; s < P; ++s) {
        const size_t i = off + size_t(t + TPL * s) * ld;
        const cx<double> zz = a.z[i];
        v[s] = first ? zz : cfma(zz, beta, a.p[i]);
        if (live) a.p[i] = v[s];
      }
    } else {
      const cx<double>* in = mode == kRowIter ? a.p : a.x;
#pragma unroll
      for (int s = 0; s < P; ++s) v[s] = in[off + size_t(t + TPL * s) * ld];
    }
    if constexpr (OP == kMvX) {
      const cx<double> En{a.E[e], 0.0};
#pragma unroll
      for (int s = 0; s < P; ++s) acc[s] = cmul(a.V[o + size_t(t + TPL * s)] - En, v[s]);
    } else {
#pragma unroll
      for (int s = 0; s < P; ++s) acc[s] = a.s[off + size_t(t + TPL * s) * ld];
    }
    const int m = AXIS == 0 ? a.mx : (AXIS == 1 ? a.my : a.mz);
    if (m > 0) {   // C_a v on the strip, with the line in LDS for the neighbours
      const int j0 = AXIS == 0 ? a.j0x : (AXIS == 1 ? a.j0y : a.j0z);
      const cx<double>* cs = AXIS == 0 ? a.cx_strip : (AXIS == 1 ? a.cy_strip : a.cz_strip);
#pragma unroll
      for (int s = 0; s < P; ++s) L[t + TPL * s] = v[s];
      __syncthreads();
#pragma unroll
      for (int s = 0; s < P; ++s) acc[s] = acc[s] + c_apply(L, t + TPL * s, N, j0, m, cs);
      __syncthreads();
    }
    cx<double> pv[P];
    if constexpr (OP == kMvZ) {
#pragma unroll
      for (int s = 0; s < P; ++s) pv[s] = v[s];
    }
    // T_a v = F_a^-1 (k_a^2/2) F_a v
    fft2<double, N, -1, wave, swz>(v, L, Lb, t, tw);
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const double k = kval(t + TPL * s, N, La);
      v[s] = (0.5 * k * k / N) * v[s];
    }
    fft2<double, N, +1, wave, swz>(v, L, Lb, t, tw);
    cx<double> dot = zero;
    if (live) {
#pragma unroll
      for (int s = 0; s < P; ++s) {
        const cx<double> wv = acc[s] + v[s];
        const size_t i = off + size_t(t + TPL * s) * ld;
        if constexpr (OP == kMvZ) {
          a.w[i] = wv;
          dot = cfma(dot, pv[s], wv);   // p^T w, unconjugated
        } else {
          a.s[i] = wv;
        }
      }
    }
    if constexpr (OP == kMvZ) {
      if (mode == kRowIter) {
        const cx<double> sum = block_sum(dot, lds);
        if (threadIdx.x == 0) a.part_pw[size_t(e) * a.nblk_col + blockIdx.x] = sum;
      }
    }
  } else if constexpr (OP == kUpdX) {
    // ---- x += alpha p, r -= alpha w (or the set-up / true-residual forms), s = F_x r
    const size_t foff = (a.f_per_energy ? size_t(e) * a.vec : 0) + o;
    const cx<double> alpha = sc.alpha;
    double rr = 0.0;
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const size_t i = off + size_t(t + TPL * s);
      cx<double> rv = zero;
      if (live) {
        if (mode == kUpdIter) {
          a.x[i] = cfma(a.x[i], alpha, a.p[i]);
          rv = a.r[i] - cmul(alpha, a.w[i]);
        } else if (mode == kUpdInit) {
          a.x[i] = zero;
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
    fft2<double, N, -1, wave, swz>(v, L, Lb, t, tw);
    if constexpr (BANDED) band_apply<N>(v, L, t, a.bx_xr, a.bx_start, a.bx_width);   // X_x
    if (live) {
#pragma unroll
      for (int s = 0; s < P; ++s) a.s[off + t + TPL * s] = v[s];
    }
    const cx<double> sum = block_sum(cx<double>{rr, 0.0}, lds);
    if (threadIdx.x == 0) a.part_rr[size_t(e) * a.nblk_row + blockIdx.x] = sum.re;
  } else if constexpr (OP == kFwdY || OP == kInvY || OP == kDivZ) {
    // ---- the y and z parts of the preconditioner's transform
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = a.s[off + size_t(t + TPL * s) * ld];
    if constexpr (OP == kFwdY) {
      fft2<double, N, -1, wave, swz>(v, L, Lb, t, tw);
      if constexpr (BANDED) band_apply<N>(v, L, t, a.by_xr, a.by_start, a.by_width);   // X_y
    } else if constexpr (OP == kInvY) {
      if constexpr (BANDED) band_apply<N>(v, L, t, a.by_xc, a.by_start, a.by_width);   // X_y^T
      fft2<double, N, +1, wave, swz>(v, L, Lb, t, tw);
    } else {
      fft2<double, N, -1, wave, swz>(v, L, Lb, t, tw);
      const double kx = kval(lx, a.nx, a.Lx), ky = kval(ly, a.ny, a.Ly), En = a.E[e];
      const double kxy = kx * kx + ky * ky;
      const double eta = a.eta ? a.eta[e] : 0.0;
      const double scale = 1.0 / (double(a.nx) * double(a.ny) * double(N));
      if constexpr (BANDED) {
        // X_z, then 1/(lambda_x + lambda_y + lambda_z - E), then X_z^T
        band_apply<N>(v, L, t, a.bz_xr, a.bz_start, a.bz_width);
        const cx<double> lxy = a.bx_lam[lx] + a.by_lam[ly] - cx<double>{En, 0.0};
#pragma unroll
        for (int s = 0; s < P; ++s) {
          const cx<double> dd = lxy + a.bz_lam[t + TPL * s];
          const double q = scale / (dd.re * dd.re + dd.im * dd.im);
          v[s] = cmul(v[s], cx<double>{q * dd.re, -q * dd.im});
        }
        band_apply<N>(v, L, t, a.bz_xc, a.bz_start, a.bz_width);
      } else if (eta == 0.0) {
#pragma unroll
        for (int s = 0; s < P; ++s) {
          const double kz = kval(t + TPL * s, N, a.Lz);
          const double d = 0.5 * (kxy + kz * kz) - En;   // (K - E), as printed in Eq. PreconFFT
          v[s] = (scale / d) * v[s];
        }
      } else {
        // shifted divisor K - E - i eta (even in k: P^-1 stays complex symmetric)
#pragma unroll
        for (int s = 0; s < P; ++s) {
          const double kz = kval(t + TPL * s, N, a.Lz);
          const double d = 0.5 * (kxy + kz * kz) - En;
          const double q = scale / (d * d + eta * eta);
          v[s] = cmul(v[s], cx<double>{q * d, q * eta});
        }
      }
      fft2<double, N, +1, wave, swz>(v, L, Lb, t, tw);
    }
    if (live) {
#pragma unroll
      for (int s = 0; s < P; ++s) a.s[off + size_t(t + TPL * s) * ld] = v[s];
    }
  } else {
    // ---- z = F_x^-1 s, partial r^T z
    cx<double> rv[P];
#pragma unroll
    for (int s = 0; s < P; ++s) {
      v[s] = a.s[off + t + TPL * s];
      rv[s] = a.r[off + t + TPL * s];
    }
    if constexpr (BANDED) band_apply<N>(v, L, t, a.bx_xc, a.bx_start, a.bx_width);   // X_x^T
    fft2<double, N, +1, wave, swz>(v, L, Lb, t, tw);
    cx<double> dot = zero;
    if (live) {
#pragma unroll
      for (int s = 0; s < P; ++s) {
        a.z[off + t + TPL * s] = v[s];
        dot = cfma(dot, rv[s], v[s]);   // r^T z, unconjugated
      }
    }
    const cx<double> sum = block_sum(dot, lds);
    if (threadIdx.x == 0) a.part_rz[size_t(e) * a.nblk_row + blockIdx.x] = sum;
  }
}

// part[e][0] = sum of part[e][0 .. n) in a fixed order (strided per thread,
// then block_sum), for the energies in state want.  Reading slot 0 precedes
// the write: the write follows block_sum's barriers.
constexpr int kReduceThreads = 256;

__device__ __forceinline__ cx<double> as_cx(double v) { return {v, 0.0}; }
__device__ __forceinline__ cx<double> as_cx(cx<double> v) { return v; }
__device__ __forceinline__ void put(double& d, cx<double> v) { d = v.re; }
__device__ __forceinline__ void put(cx<double>& d, cx<double> v) { d = v; }

template <typename V>
__global__ void __launch_bounds__(kReduceThreads) k3_reduce(V* part, int stride, int n, const CocgScalars* sc,
                                                            int want) {
  __shared__ cx<double> red[kReduceThreads / 64];
  const int e = blockIdx.x;
  if (sc[e].state != want) return;
  V* q = part + size_t(e) * stride;
  cx<double> acc{0.0, 0.0};
  for (int b = threadIdx.x; b < n; b += kReduceThreads) acc = acc + as_cx(q[b]);
  const cx<double> sum = block_sum(acc, red);
  if (threadIdx.x == 0) put(q[0], sum);
}

template <int N, int OP, bool BANDED>
sofft_status pass_n(const SseArgs& a, int want, int mode, hipStream_t s) {
  constexpr int AXIS = op_axis<OP>(), LPB = k3_lines<N>();
  const size_t lds = size_t(LPB) * 2 * fft_lds_elems<N>() * sizeof(cx<double>);
  if (lds > 65536) {
    sofft_status st = raise_lds_limit(reinterpret_cast<const void*>(k3_sse<N, OP, BANDED>), 150 * 1024);
    if (st != SOFFT_OK) return st;
  }
  const int nlines = AXIS == 0 ? a.ny * a.nz : (AXIS == 1 ? a.nx * a.nz : a.nx * a.ny);
  const dim3 grid((nlines + LPB - 1) / LPB, a.nE);
  k3_sse<N, OP, BANDED><<<grid, k3_threads<N>(), lds, s>>>(a, want, mode);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

// The preconditioner's passes have banded instantiations (a.banded); the
// matrix passes do not need them.
template <int OP>
constexpr bool has_banded() { return OP == kUpdX || OP == kFwdY || OP == kDivZ || OP == kInvY || OP == kPrecX; }

template <int OP>
sofft_status pass(const SseArgs& a, int want, int mode, hipStream_t s) {
  constexpr int AXIS = op_axis<OP>();
  const int n = AXIS == 0 ? a.nx : (AXIS == 1 ? a.ny : a.nz);
  if constexpr (has_banded<OP>()) {
    if (a.banded) {
      SOFFT_3D_SWITCH(n, (pass_n<N_, OP, true>(a, want, mode, s)))
      set_error("unsupported 3D line length");
      return SOFFT_EUNSUPPORTED;
    }
  }
  SOFFT_3D_SWITCH(n, (pass_n<N_, OP, false>(a, want, mode, s)))
  set_error("unsupported 3D line length");
  return SOFFT_EUNSUPPORTED;
}

template <typename V>
sofft_status reduce(V* part, int stride, const SseArgs& a, int want, hipStream_t s) {
  k3_reduce<V><<<a.nE, kReduceThreads, 0, s>>>(part, stride, stride, a.sc, want);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

sofft_status sse3_launch(SseKernel k, const SseArgs& a, int want, int mode, hipStream_t s, Timing& tm) {
  sofft_status st = SOFFT_OK;
  auto ok = [&](sofft_status q) { return (st = q) == SOFFT_OK; };
  switch (k) {
    case kK1:
      if (!ok(tm.begin(SOFFT_KERNEL_SSE_ROW_MV, s))) return st;
      if (ok(pass<kMvX>(a, want, mode, s))) ok(pass<kMvY>(a, want, mode, s));
      break;
    case kK2:
      if (!ok(tm.begin(SOFFT_KERNEL_SSE_COL_MV, s))) return st;
      if (ok(pass<kMvZ>(a, want, mode, s)) && mode == kRowIter) ok(reduce(a.part_pw, a.nblk_col, a, want, s));
      break;
    case kK4:
      if (!ok(tm.begin(SOFFT_KERNEL_SSE_ROW_UPD, s))) return st;
      if (ok(pass<kUpdX>(a, want, mode, s))) ok(reduce(a.part_rr, a.nblk_row, a, want, s));
      break;
    case kK5:
      if (!ok(tm.begin(SOFFT_KERNEL_SSE_COL_PREC, s))) return st;
      if (ok(pass<kFwdY>(a, want, mode, s)) && ok(pass<kDivZ>(a, want, mode, s))) ok(pass<kInvY>(a, want, mode, s));
      break;
    case kK6:
      if (!ok(tm.begin(SOFFT_KERNEL_SSE_ROW_PREC, s))) return st;
      if (ok(pass<kPrecX>(a, want, mode, s))) ok(reduce(a.part_rz, a.nblk_row, a, want, s));
      break;
  }
  if (st != SOFFT_OK) return st;
  return tm.end(s);
}

bool line_ok(int64_t n) { return n >= 16 && n <= 512 && (n & (n - 1)) == 0; }

}  // namespace

SseLauncher sse3_launcher(int64_t nx, int64_t ny, int64_t nz) {
  return line_ok(nx) && line_ok(ny) && line_ok(nz) ? sse3_launch : nullptr;
}

// Partial sums per energy of the 3D passes: one per block of the x passes
// (row) and of the z pass (col).
void sse3_blocks(int64_t nx, int64_t ny, int64_t nz, int* nbr, int* nbc) {
  auto lpb = [](int64_t n) -> int {
    SOFFT_3D_SWITCH(n, (k3_lines<N_>()))
    return 1;
  };
  *nbr = int((ny * nz + lpb(nx) - 1) / lpb(nx));
  *nbc = int((nx * ny + lpb(nz) - 1) / lpb(nz));
}

}  // namespace sofft
