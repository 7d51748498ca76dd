// Absorbing potentials of Sec. IV (CAP and TFAP), the alternatives to ECS
// that the paper compares it with: added to a caller's V0 table on an
// unscaled grid.
#include "cx.hpp"
#include "internal.hpp"

namespace sofft {

// Absorbing potentials of Sec. IV on one axis, at s = (|x| - r_s)/Dx_CS:
// CAP (Eq. CAP_via_q with the contour of Eq. qSECS, end angle pi/4)
//   E_cap [1 - exp(i pi s/2)];
// TFAP (Eqs. TFAP, yTFAP) -i (k_min^2/2) y(s), where the pole terms
//   4/(1-s)^2 - 4/(1+s)^2 are taken as 16 s/(1-s^2)^2 (the same function,
//   without the cancellation near s = 0).
struct AbsorberAxis {
  const double* x;
  int n;
  double r_s, width;
};
struct AbsorberArgs {
  AbsorberAxis ax[3];
  int ndim, kind;
  double param;
};

__device__ __forceinline__ cx<double> absorber_1d(double x, const AbsorberAxis& a, int kind, double param) {
  const double d = fabs(x) - a.r_s;
  if (!(d > 0.0)) return {0.0, 0.0};
  const double s = d / a.width;
  if (kind == SOFFT_ABSORBER_CAP) {
    double sn, cs;
    sincospi(0.5 * s, &sn, &cs);
    return {param * (1.0 - cs), -param * sn};
  }
  constexpr double c = 2.622057, c2 = c * c, c3 = c2 * c;
  const double u = 1.0 - s * s;
  const double y = ((c3 - 16.0) * s - (c3 - 17.0) * s * s * s + 16.0 * s / (u * u)) / c2;
  return {0.0, -0.5 * param * param * y};
}

// v0 += sum over axes of the absorber of its axis, on the [nz][ny][nx] grid.
__global__ void __launch_bounds__(256) k_add_absorber(cx<double>* v0, AbsorberArgs a) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t total = 1;
  for (int d = 0; d < a.ndim; ++d) total *= size_t(a.ax[d].n);
  if (i >= total) return;
  cx<double> u{0.0, 0.0};
  size_t r = i;
  for (int d = 0; d < a.ndim; ++d) {
    const int j = int(r % size_t(a.ax[d].n));
    r /= size_t(a.ax[d].n);
    u = u + absorber_1d(a.ax[d].x[j], a.ax[d], a.kind, a.param);
  }
  v0[i] = v0[i] + u;
}

sofft_status launch_absorber(const Plan& p, int kind, double param, void* v0, hipStream_t s) {
  AbsorberArgs a{};
  a.ndim = p.prob.ndim;
  a.kind = kind;
  a.param = param;
  size_t total = 1;
  for (int d = 0; d < a.ndim; ++d) {
    const Axis& A = p.ax[d];
    a.ax[d] = {static_cast<const double*>(A.x_dev.p), int(A.n), p.prob.R0[d], p.prob.L[d] / 2 - p.prob.R0[d]};
    total *= size_t(A.n);
  }
  k_add_absorber<<<unsigned((total + 255) / 256), 256, 0, s>>>(static_cast<cx<double>*>(v0), a);
  SOFFT_HIP_TRY(hipGetLastError());
  return SOFFT_OK;
}

}  // namespace sofft
