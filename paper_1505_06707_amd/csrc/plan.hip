// Host side of a plan: the grid, momenta, ECS contour, the remainder C and the
// Crank-Nicolson factor, FFT twiddles and kinetic phases (Sec. II), and their
// device copies.
#include <cmath>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "line_fft.hpp"

namespace sofft {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

sofft_status raise_lds_limit(const void* kernel, size_t limit) {
  static std::mutex mu;
  static std::vector<const void*> raised;
  std::lock_guard<std::mutex> lock(mu);
  if (std::find(raised.begin(), raised.end(), kernel) != raised.end()) return SOFFT_OK;
  SOFFT_HIP_TRY(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(limit)));
  raised.push_back(kernel);
  return SOFFT_OK;
}

sofft_status dev_reserve(DevBuf& b, size_t bytes) {
  if (b.p && b.bytes >= bytes) return SOFFT_OK;
  dev_free(b);
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    b.p = nullptr;
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
    return SOFFT_ENOMEM;
  }
  b.bytes = bytes;
  return SOFFT_OK;
}

sofft_status dev_upload(DevBuf& b, const void* host, size_t bytes) {
  if (!b.p || b.bytes < bytes) {
    set_error("internal: device table of " + std::to_string(b.bytes) + " bytes cannot take " +
              std::to_string(bytes));
    return SOFFT_EUNSUPPORTED;
  }
  SOFFT_HIP_TRY(hipMemcpy(b.p, host, bytes, hipMemcpyHostToDevice));
  return SOFFT_OK;
}

void dev_free(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

WsLayout plan_ws_layout(const Plan& p, int n_energies) {
  WsLayout L;
  size_t npts = 1;
  for (int d = 0; d < p.prob.ndim; ++d) npts *= size_t(p.ax[d].n);
  L.vphase = 0;
  L.partials = round256(npts * sizeof(cx<double>));
  L.solver = L.partials + round256(kNormBlocks * sizeof(double));
  L.solver_bytes = n_energies > 0 ? sse_solver_bytes(p, n_energies) : 0;
  L.total = L.solver + round256(L.solver_bytes);
  return L;
}

sofft_status plan_ws_check(const Plan& p, int n_energies, WsLayout* out) {
  const WsLayout L = plan_ws_layout(p, n_energies);
  if (!p.ws || p.ws_bytes < L.total) {
    set_error("the plan needs a bound workspace of " + std::to_string(L.total) + " bytes" +
              (n_energies > 0 ? " for " + std::to_string(n_energies) + " energies" : std::string()) +
              " (sofft_workspace_size, sofft_plan_bind); bound: " + std::to_string(p.ws ? p.ws_bytes : 0));
    return SOFFT_EWORKSPACE;
  }
  if (out) *out = L;
  return SOFFT_OK;
}

bool supported_length(int64_t n) {
  switch (n) {
    case 16: case 32: case 48: case 64: case 96: case 128: case 192: case 256: case 384: case 512:
    case 768: case 1024: case 2048: case 4096:
      return true;
    default:
      return false;
  }
}

// TFECS (Sec. IV, Eq. qTFECS): q = sqrt(1 + i y(s)), s = (|x| - R0)/(L/2 - R0),
// y(s) = alpha [(1 - s)^-2 - (1 + s)^-2 - 4 s], alpha carried by theta.  q is
// infinite at the box edge (s = 1); that point is represented by an infinite
// real part and only ever divides (1/q = 0 there).
static zc tfecs_q(double ax, const Axis& a) {
  const double s = (ax - a.R0) / (a.L / 2 - a.R0);
  if (s >= 1.0) return zc(INFINITY, 0.0);
  // alpha [(1 - s)^-2 - (1 + s)^-2 - 4 s] = 4 alpha s^3 (2 - s^2)/(1 - s^2)^2, the
  // second form free of cancellation at small s
  const double u = 1.0 - s * s;
  const double y = 4.0 * a.theta * s * s * s * (2.0 - s * s) / (u * u);
  return std::sqrt(zc(1.0, y));
}

// q(x) of the contour (Sec. IV): sharp rotation, smooth SECS (Eq. qSECS with
// end angle theta at the box edge), TFECS, or no scaling.
static zc contour_q(double x, const Axis& a) {
  const double ax = std::fabs(x);
  switch (a.contour) {
    case SOFFT_SECS:
      if (ax > a.R0) return std::polar(1.0, a.theta * (ax - a.R0) / (a.L / 2 - a.R0));
      return 1.0;
    case SOFFT_SHARP:
      if (ax - a.R0 > 1e-9 * a.h) return std::polar(1.0, a.theta);
      return 1.0;
    case SOFFT_TFECS:
      if (ax > a.R0) return tfecs_q(ax, a);
      return 1.0;
    default:
      return 1.0;
  }
}

// n-point Gauss-Legendre nodes and weights on [-1, 1]: roots of P_n by Newton's
// method from the usual cosine guesses, P_n and P_n' by the three-term
// recurrence.
static void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& w) {
  const double pi = 3.14159265358979323846;
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    t[i] = x;
    w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

// int_u0^u1 q for TFECS by composite 20-point Gauss-Legendre, 4 panels per
// call (the integrand is analytic on the interval: its singularity at the box
// edge lies at least half a cell beyond any node).
static zc tfecs_integral(double u0, double u1, const Axis& a) {
  static std::vector<double> t, w;
  if (t.empty()) gauss_legendre(20, t, w);
  zc acc = 0.0;
  const int panels = 4;
  const double hp = (u1 - u0) / panels;
  for (int k = 0; k < panels; ++k) {
    const double c = u0 + hp * (k + 0.5), r = hp / 2;
    for (size_t i = 0; i < t.size(); ++i) acc += w[i] * r * tfecs_q(c + r * t[i], a);
  }
  return acc;
}

// z(x) = int_0^x q (Sec. II, Eq. ECSintdef) in closed form for each contour.
static zc contour_z(double x, const Axis& a) {
  const double ax = std::fabs(x), sg = x < 0 ? -1.0 : 1.0;
  switch (a.contour) {
    case SOFFT_SECS:
      if (ax > a.R0) {
        const double D = a.L / 2 - a.R0;
        const double phi = a.theta * (ax - a.R0) / D;
        // D/(i theta) (e^{i phi} - 1) = (D/theta) (sin phi + i (1 - cos phi))
        return sg * zc(a.R0 + D / a.theta * std::sin(phi), D / a.theta * (1.0 - std::cos(phi)));
      }
      return x;
    case SOFFT_SHARP:
      if (ax - a.R0 > 1e-9 * a.h) return sg * (a.R0 + (ax - a.R0) * std::polar(1.0, a.theta));
      return x;
    case SOFFT_TFECS:
      // no closed form: callers integrate (tfecs_integral); see build_axis
      return x;
    default:
      return x;
  }
}

// a / q, and 0 where q is infinite (TFECS at the box edge).
static zc over_q(zc num, zc q) { return std::isinf(q.real()) ? zc(0.0) : num / q; }

sofft_status build_axis(Axis& a, int64_t n, double L, double R0, double theta, int contour) {
  a.n = n;
  a.L = L;
  a.h = L / double(n);
  a.R0 = R0;
  a.theta = theta;
  a.contour = contour;
  a.x.resize(n);
  a.xm.resize(n);
  a.k.resize(n);
  a.q.resize(n);
  a.qm.resize(n);
  a.z.resize(n);
  const double pi = 3.14159265358979323846;
  for (int64_t j = 0; j < n; ++j) {
    a.x[j] = -L / 2 + a.h * (double(j) + 0.5);   // cell centres
    a.xm[j] = -L / 2 + a.h * double(j + 1);      // x_{j+1/2}; the last one is the box edge
    const int64_t mm = j < n / 2 ? j : j - n;    // Eq. FFTbasis order, Nyquist negative
    a.k[j] = 2 * pi * double(mm) / L;
  }
  for (int64_t j = 0; j < n; ++j) {
    a.q[j] = contour_q(a.x[j], a);
    a.qm[j] = contour_q(a.xm[j], a);
    a.z[j] = contour_z(a.x[j], a);
  }
  if (contour == SOFFT_TFECS) {
    // z = sign(x) (R0 + int_R0^|x| q), accumulated node by node outward from
    // R0 on each side (the nodes are symmetric about 0).
    for (int side = 0; side < 2; ++side) {
      zc acc = 0.0;
      double prev = R0;
      for (int64_t i = 0; i < n; ++i) {
        const int64_t j = side ? i : n - 1 - i;   // outward: increasing |x|
        const double ax = std::fabs(a.x[j]);
        if ((side == 1 && a.x[j] < 0) || (side == 0 && a.x[j] > 0) || ax <= R0) continue;
        acc += tfecs_integral(prev, ax, a);
        prev = ax;
        a.z[j] = (a.x[j] < 0 ? -1.0 : 1.0) * (R0 + acc);
      }
    }
  }
  // C = K_s - K_FD from the three-point stencils of Eqs. Ks_FD and K_FD,
  // periodic in j: the midpoint left of node 0 is the box edge (index n-1).
  a.cdn.assign(n, 0.0);
  a.cdg.assign(n, 0.0);
  a.cup.assign(n, 0.0);
  const double c = 1.0 / (2.0 * a.h * a.h);
  std::vector<zc> qs(n);
  for (int64_t j = 0; j < n; ++j) qs[j] = 1.0 / std::sqrt(a.q[j]);
  for (int64_t j = 0; j < n; ++j) {
    const int64_t jp = (j + 1) % n, jm = (j + n - 1) % n;
    const zc qr = a.qm[j], ql = a.qm[jm];
    a.cup[j] = -over_q(c * qs[j] * qs[jp], qr) + c;
    a.cdn[j] = -over_q(c * qs[j] * qs[jm], ql) + c;
    a.cdg[j] = c * (1.0 / a.q[j]) * (over_q(1.0, qr) + over_q(1.0, ql)) - 2.0 * c;
  }
  // The strip: nodes whose row of C is non-zero.  It must be one cyclic run
  // that leaves part of the axis unscaled.
  std::vector<char> in(n, 0);
  int64_t cnt = 0;
  for (int64_t j = 0; j < n; ++j) {
    in[j] = (a.cdn[j] != 0.0 || a.cdg[j] != 0.0 || a.cup[j] != 0.0);
    cnt += in[j];
  }
  a.m = cnt;
  a.j0 = 0;
  if (cnt > 0) {
    if (cnt > n / 2) {
      set_error("the scaled region covers more than half of the axis; increase R0");
      return SOFFT_EUNSUPPORTED;
    }
    int64_t starts = 0;
    for (int64_t j = 0; j < n; ++j)
      if (in[j] && !in[(j + n - 1) % n]) {
        a.j0 = j;
        ++starts;
      }
    if (starts != 1) {
      set_error("the scaled region is not one contiguous run through the box edge");
      return SOFFT_EUNSUPPORTED;
    }
  }
  return SOFFT_OK;
}

template <typename T>
static std::vector<cx<T>> to_cx(const std::vector<zc>& v) {
  std::vector<cx<T>> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = {T(v[i].real()), T(v[i].imag())};
  return o;
}

// Every device table of an axis at its largest size: the tables that depend
// on dt (kinetic phases, PCR coefficients for at most ceil(log2 m) levels) are
// refilled in place when dt changes, so no call after sofft_plan_create
// allocates device memory.  Band tables only for plans that can solve.
static sofft_status reserve_axis(Axis& a, bool bands) {
  const size_t c = sizeof(cx<double>), n = size_t(a.n), m = size_t(std::max<int64_t>(a.m, 1));
  int maxlev = 1;
  while ((int64_t(1) << maxlev) < a.m) ++maxlev;
  sofft_status st;
  for (auto req : {std::make_pair(&a.tw64, n * c), std::make_pair(&a.x_dev, n * sizeof(double)),
                   std::make_pair(&a.z_dev, n * c), std::make_pair(&a.cstrip64, 3 * m * c),
                   std::make_pair(&a.kin_full64, n * c), std::make_pair(&a.kin_half64, n * c),
                   std::make_pair(&a.alpha64, size_t(maxlev) * m * c), std::make_pair(&a.gamma64, size_t(maxlev) * m * c),
                   std::make_pair(&a.binv64, m * c)})
    if ((st = dev_reserve(*req.first, req.second)) != SOFFT_OK) return st;
  if (bands)
    for (auto req : {std::make_pair(&a.band_lam, n * c), std::make_pair(&a.band_xr, size_t(kBandMax) * n * c),
                     std::make_pair(&a.band_xc, size_t(kBandMax) * n * c),
                     std::make_pair(&a.band_start, n * sizeof(int32_t)),
                     std::make_pair(&a.band_width, n * sizeof(int32_t))})
      if ((st = dev_reserve(*req.first, req.second)) != SOFFT_OK) return st;
  return SOFFT_OK;
}

sofft_status upload_static(Axis& a, bool bands) {
  sofft_status st0 = reserve_axis(a, bands);
  if (st0 != SOFFT_OK) return st0;
  // Stage twiddle tables of the line FFT (layout in line_fft.hpp), evaluated
  // in long double and rounded.
  const ShapeInfo sh = shape_info(a.n);
  std::vector<zc> tw(a.n, 0.0);
  const long double pil = 3.141592653589793238462643383279502884L;
  int64_t off = 0, ns = sh.R0;
  for (int s = 1; s <= sh.K; ++s) {
    const int64_t stride = a.n / (sh.RR * ns);
    for (int m = 1; m < sh.RR; ++m)
      for (int64_t k = 0; k < ns; ++k) {
        const int64_t u = (m * k * stride) % a.n;
        const long double ang = 2.0L * pil * (long double)u / (long double)a.n;
        tw[off + (m - 1) * ns + k] = zc(double(cosl(ang)), double(-sinl(ang)));
      }
    off += (sh.RR - 1) * ns;
    ns *= sh.RR;
  }
  auto t64 = to_cx<double>(tw);
  auto z64 = to_cx<double>(a.z);
  sofft_status st;
  // Rows of C on the strip, [C_{j,j-1} (m) | C_{j,j} (m) | C_{j,j+1} (m)] at
  // j = (j0 + p) mod n, for the stationary matrix-vector product.
  if (a.m > 0) {
    std::vector<zc> cs(3 * a.m);
    for (int64_t p = 0; p < a.m; ++p) {
      const int64_t j = (a.j0 + p) % a.n;
      cs[p] = a.cdn[j];
      cs[a.m + p] = a.cdg[j];
      cs[2 * a.m + p] = a.cup[j];
    }
    auto c64 = to_cx<double>(cs);
    if ((st = dev_upload(a.cstrip64, c64.data(), c64.size() * sizeof(c64[0]))) != SOFFT_OK) return st;
  }
  if ((st = dev_upload(a.tw64, t64.data(), t64.size() * sizeof(t64[0]))) != SOFFT_OK) return st;
  if ((st = dev_upload(a.x_dev, a.x.data(), a.x.size() * sizeof(double))) != SOFFT_OK) return st;
  if ((st = dev_upload(a.z_dev, z64.data(), z64.size() * sizeof(z64[0]))) != SOFFT_OK) return st;
  return SOFFT_OK;
}

// Kinetic phases exp(-i k^2 dt/2)/n and exp(-i k^2 dt/4)/n (the 1/n of the
// unscaled inverse FFT folded in), and the Crank-Nicolson system on the strip
// prepared for parallel cyclic reduction.
sofft_status ensure_dt(Axis& a, double dt) {
  if (a.have_dt && a.dt == dt) return SOFFT_OK;
  // Work already enqueued may still read the tables of the previous dt.
  if (a.have_dt) SOFFT_HIP_TRY(hipDeviceSynchronize());
  const int64_t n = a.n;
  std::vector<zc> kf(n), kh(n);
  for (int64_t j = 0; j < n; ++j) {
    const long double e = (long double)a.k[j] * (long double)a.k[j] / 2.0L * (long double)dt;
    kf[j] = zc(double(cosl(e) / n), double(-sinl(e) / n));
    kh[j] = zc(double(cosl(e / 2) / n), double(-sinl(e / 2) / n));
  }
  sofft_status st;
  {
    auto f64 = to_cx<double>(kf), h64 = to_cx<double>(kh);
    if ((st = dev_upload(a.kin_full64, f64.data(), n * sizeof(f64[0]))) != SOFFT_OK) return st;
    if ((st = dev_upload(a.kin_half64, h64.data(), n * sizeof(h64[0]))) != SOFFT_OK) return st;
  }
  // CN: y = (1 + i dt C/2)^-1 (1 - i dt C/2) v = 2 B^-1 v - v with B = 1 + i dt C/2.
  // B restricted to the strip is tridiagonal: a_p u_{p-1} + b_p u_p + c_p u_{p+1}.
  // PCR level l (stride s = 2^l) replaces row p by row p - alpha_p row(p-s)
  // - gamma_p row(p+s); after ceil(log2 m) levels B is diagonal.
  const int64_t m = a.m;
  a.levels = 0;
  if (m > 0) {
    const zc ih(0.0, 0.5 * dt);
    std::vector<zc> A(m), Bd(m), Cu(m);
    for (int64_t p = 0; p < m; ++p) {
      const int64_t j = (a.j0 + p) % n;
      A[p] = p > 0 ? ih * a.cdn[j] : 0.0;
      Bd[p] = 1.0 + ih * a.cdg[j];
      Cu[p] = p + 1 < m ? ih * a.cup[j] : 0.0;
    }
    // B is strongly diagonally dominant for the usual dt, and each level
    // squares the relative coupling: stop as soon as every remaining
    // |a_p/b_p|, |c_p/b_p| is below 1e-18, where dropping the couplings
    // changes u by less than FP64 rounding.  ceil(log2 m) levels at most.
    int levels = 0;
    std::vector<zc> al, ga;
    auto coupled = [&]() {
      for (int64_t p = 0; p < m; ++p)
        if (std::abs(A[p]) > 1e-18 * std::abs(Bd[p]) || std::abs(Cu[p]) > 1e-18 * std::abs(Bd[p])) return true;
      return false;
    };
    while ((int64_t(1) << levels) < m && coupled()) {
      const int64_t s = int64_t(1) << levels;
      std::vector<zc> A2(m), B2(m), C2(m);
      al.resize(size_t(levels + 1) * m);
      ga.resize(size_t(levels + 1) * m);
      for (int64_t p = 0; p < m; ++p) {
        const bool lo = p - s >= 0, hi = p + s < m;
        const zc alpha = lo ? A[p] / Bd[p - s] : 0.0;
        const zc gamma = hi ? Cu[p] / Bd[p + s] : 0.0;
        al[size_t(levels) * m + p] = alpha;
        ga[size_t(levels) * m + p] = gamma;
        A2[p] = lo ? -alpha * A[p - s] : 0.0;
        C2[p] = hi ? -gamma * Cu[p + s] : 0.0;
        B2[p] = Bd[p] - (lo ? alpha * Cu[p - s] : 0.0) - (hi ? gamma * A[p + s] : 0.0);
      }
      A.swap(A2);
      Bd.swap(B2);
      Cu.swap(C2);
      ++levels;
    }
    std::vector<zc> bi(m);
    for (int64_t p = 0; p < m; ++p) bi[p] = 1.0 / Bd[p];
    a.levels = levels;
    std::vector<zc> dummy(1, 0.0);
    const auto& alv = levels ? al : dummy;
    const auto& gav = levels ? ga : dummy;
    auto al64 = to_cx<double>(alv), ga64 = to_cx<double>(gav), bi64 = to_cx<double>(bi);
    if ((st = dev_upload(a.alpha64, al64.data(), al64.size() * sizeof(al64[0]))) != SOFFT_OK) return st;
    if ((st = dev_upload(a.gamma64, ga64.data(), ga64.size() * sizeof(ga64[0]))) != SOFFT_OK) return st;
    if ((st = dev_upload(a.binv64, bi64.data(), bi64.size() * sizeof(bi64[0]))) != SOFFT_OK) return st;
  }
  a.dt = dt;
  a.have_dt = true;
  return SOFFT_OK;
}

void free_axis(Axis& a) {
  for (DevBuf* b : {&a.tw64, &a.x_dev, &a.z_dev, &a.cstrip64, &a.kin_full64, &a.kin_half64, &a.alpha64,
                    &a.gamma64, &a.binv64, &a.band_lam, &a.band_xr, &a.band_xc, &a.band_start, &a.band_width})
    dev_free(*b);
  a.have_bands = false;
}

}  // namespace sofft

using namespace sofft;

struct sofft_plan : public Plan {};

namespace sofft {
Plan& plan_of(sofft_plan* p) { return *p; }
}  // namespace sofft

extern "C" {

const char* sofft_last_error(void) { return g_err.c_str(); }

int32_t sofft_version(void) { return 100; }

sofft_status sofft_plan_create(const sofft_problem* prob, sofft_plan** out) {
  if (!prob || !out) {
    set_error("null argument");
    return SOFFT_EINVAL;
  }
  *out = nullptr;
  const sofft_problem& p = *prob;
  if (p.ndim < 1 || p.ndim > 3) {
    set_error("ndim must be 1, 2 or 3");
    return SOFFT_EINVAL;
  }
  if (p.dtype != SOFFT_C128 && p.dtype != SOFFT_C64) {
    set_error("dtype must be SOFFT_C128 or SOFFT_C64");
    return SOFFT_EINVAL;
  }
  if (p.contour != SOFFT_SECS && p.contour != SOFFT_SHARP && p.contour != SOFFT_ECS_OFF &&
      p.contour != SOFFT_TFECS) {
    set_error("unknown contour");
    return SOFFT_EINVAL;
  }
  if ((p.contour == SOFFT_SECS || p.contour == SOFFT_SHARP) && !(p.theta > 0 && p.theta < 1.5707963267948966)) {
    set_error("theta must lie in (0, pi/2)");
    return SOFFT_EINVAL;
  }
  if (p.contour == SOFFT_TFECS && !(p.theta > 0 && std::isfinite(p.theta))) {
    set_error("the TFECS parameter alpha (theta) must be positive and finite");
    return SOFFT_EINVAL;
  }
  if (!(p.charge >= 0) || (p.charge > 0 && !(p.a2 > 0))) {
    set_error("charge must be >= 0 and a2 > 0 when charge > 0");
    return SOFFT_EINVAL;
  }
  for (int d = 0; d < p.ndim; ++d) {
    const bool pow2 = p.n[d] > 0 && (p.n[d] & (p.n[d] - 1)) == 0;
    if (!supported_length(p.n[d]) || (p.ndim == 2 && p.n[d] > 1024) || (p.ndim == 3 && (p.n[d] > 512 || !pow2))) {
      set_error("unsupported grid length " + std::to_string(p.n[d]));
      return SOFFT_EUNSUPPORTED;
    }
    if (!(p.L[d] > 0)) {
      set_error("box length must be positive");
      return SOFFT_EINVAL;
    }
    if (p.contour != SOFFT_ECS_OFF && !(p.R0[d] > 0 && p.R0[d] < p.L[d] / 2)) {
      set_error("R0 must lie in (0, L/2)");
      return SOFFT_EINVAL;
    }
  }
  sofft_plan* pl = new sofft_plan();
  pl->prob = p;
  // The 2D passes solve each line's ECS strip in one wavefront, four nodes per
  // lane: at most 256 strip nodes per axis.
  for (int d = 0; d < p.ndim; ++d) {
    sofft_status st = build_axis(pl->ax[d], p.n[d], p.L[d], p.R0[d], p.theta, p.contour);
    if (st == SOFFT_OK && p.ndim >= 2 && pl->ax[d].m > 256) {
      set_error("ECS strip of " + std::to_string(pl->ax[d].m) + " nodes exceeds 256 per axis in 2D and 3D; "
                "increase R0");
      st = SOFFT_EUNSUPPORTED;
    }
    if (st == SOFFT_OK && pl->ax[d].m > pl->ax[d].n / 2) {
      set_error("ECS strip of " + std::to_string(pl->ax[d].m) + " nodes exceeds half the axis; increase R0");
      st = SOFFT_EUNSUPPORTED;
    }
    if (st == SOFFT_OK) st = upload_static(pl->ax[d], p.dtype == SOFFT_C128);
    if (st != SOFFT_OK) {
      for (int e = 0; e < 3; ++e) free_axis(pl->ax[e]);
      delete pl;
      return st;
    }
  }
  *out = pl;
  return SOFFT_OK;
}

sofft_status sofft_plan_destroy(sofft_plan* plan) {
  if (!plan) return SOFFT_OK;
  for (int d = 0; d < 3; ++d) free_axis(plan->ax[d]);
  delete plan;
  return SOFFT_OK;
}

sofft_status sofft_workspace_size(const sofft_plan* plan, int32_t n_energies, int64_t* bytes) {
  if (!plan || !bytes || n_energies < 0) {
    set_error("bad argument to sofft_workspace_size");
    return SOFFT_EINVAL;
  }
  if (n_energies > 0 && plan->prob.dtype != SOFFT_C128) {
    set_error("the stationary solver works on complex128 plans");
    return SOFFT_EUNSUPPORTED;
  }
  *bytes = int64_t(plan_ws_layout(*plan, n_energies).total);
  return SOFFT_OK;
}

sofft_status sofft_plan_bind(sofft_plan* plan, void* workspace, int64_t bytes) {
  if (!plan || bytes < 0 || (workspace && (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)) {
    set_error("bad argument to sofft_plan_bind (the workspace must be 256-byte aligned)");
    return SOFFT_EINVAL;
  }
  plan->ws = workspace;
  plan->ws_bytes = workspace ? size_t(bytes) : 0;
  plan->vphase_ht = __builtin_nan("");   // the phase table is rebuilt in the new memory
  return SOFFT_OK;
}

sofft_status sofft_grid_nodes(const sofft_plan* plan, int32_t axis, double* x_host) {
  if (!plan || !x_host || axis < 0 || axis >= plan->prob.ndim) {
    set_error("bad argument to sofft_grid_nodes");
    return SOFFT_EINVAL;
  }
  std::memcpy(x_host, plan->ax[axis].x.data(), plan->ax[axis].x.size() * sizeof(double));
  return SOFFT_OK;
}

sofft_status sofft_strip_length(const sofft_plan* plan, int32_t axis, int64_t* m) {
  if (!plan || !m || axis < 0 || axis >= plan->prob.ndim) {
    set_error("bad argument to sofft_strip_length");
    return SOFFT_EINVAL;
  }
  *m = plan->ax[axis].m;
  return SOFFT_OK;
}

sofft_status sofft_propagate(sofft_plan* plan, void* psi, double dt, int64_t nsteps,
                             const double* f_mid, void* stream) {
  if (!plan || !psi || nsteps < 0 || !std::isfinite(dt)) {
    set_error("bad argument to sofft_propagate");
    return SOFFT_EINVAL;
  }
  if (nsteps == 0) return SOFFT_OK;
  for (int d = 0; d < plan->prob.ndim; ++d) {
    sofft_status st = ensure_dt(plan->ax[d], dt);
    if (st != SOFFT_OK) return st;
  }
  return launch_propagate(*plan, psi, dt, nsteps, f_mid, reinterpret_cast<hipStream_t>(stream));
}

sofft_status sofft_propagate_static(sofft_plan* plan, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                    void* stream) {
  if (!plan || !psi || nsteps < 0 || !std::isfinite(dt)) {
    set_error("bad argument to sofft_propagate_static");
    return SOFFT_EINVAL;
  }
  if (nsteps == 0) return SOFFT_OK;
  for (int d = 0; d < plan->prob.ndim; ++d) {
    sofft_status st = ensure_dt(plan->ax[d], dt);
    if (st != SOFFT_OK) return st;
  }
  return launch_propagate_static(*plan, psi, dt, nsteps, f_mid, reinterpret_cast<hipStream_t>(stream));
}

sofft_status sofft_set_potential(sofft_plan* plan, const void* v0, const double* w) {
  if (!plan) {
    set_error("bad argument to sofft_set_potential");
    return SOFFT_EINVAL;
  }
  plan->user_v0 = v0;
  plan->user_w = w;
  plan->vphase_ht = __builtin_nan("");   // the phase table follows V0
  return SOFFT_OK;
}

sofft_status sofft_make_softcore(const sofft_plan* plan, double charge, double a2, void* v0, void* stream) {
  if (!plan || !v0 || !std::isfinite(charge) || !std::isfinite(a2) || (charge != 0.0 && !(a2 > 0))) {
    set_error("bad argument to sofft_make_softcore");
    return SOFFT_EINVAL;
  }
  return launch_softcore(*plan, charge, a2, v0, reinterpret_cast<hipStream_t>(stream));
}

sofft_status sofft_add_absorber(const sofft_plan* plan, int32_t kind, double param, void* v0, void* stream) {
  if (!plan || !v0 || (kind != SOFFT_ABSORBER_CAP && kind != SOFFT_ABSORBER_TFAP) || !std::isfinite(param) ||
      !(param > 0)) {
    set_error("bad argument to sofft_add_absorber");
    return SOFFT_EINVAL;
  }
  const sofft_problem& p = plan->prob;
  for (int d = 0; d < p.ndim; ++d)
    if (!(p.R0[d] > 0 && p.R0[d] < p.L[d] / 2)) {
      set_error("the absorber needs 0 < R0 < L/2 on every axis");
      return SOFFT_EINVAL;
    }
  return launch_absorber(*plan, kind, param, v0, reinterpret_cast<hipStream_t>(stream));
}

sofft_status sofft_sse_solve(sofft_plan* plan, const void* f, int32_t f_per_energy, const double* E_host,
                             int32_t nE, double field, void* x_out, double rtol, int32_t maxit,
                             sofft_solve_stats* stats, void* stream) {
  if (!plan || !f || !E_host || nE <= 0 || !x_out || !(rtol > 0) || maxit <= 0 || !std::isfinite(field)) {
    set_error("bad argument to sofft_sse_solve");
    return SOFFT_EINVAL;
  }
  for (int e = 0; e < nE; ++e)
    if (!std::isfinite(E_host[e])) {
      set_error("energies must be finite");
      return SOFFT_EINVAL;
    }
  return sse_solve(*plan, f, f_per_energy, E_host, nE, field, x_out, rtol, maxit, stats,
                   reinterpret_cast<hipStream_t>(stream));
}

sofft_status sofft_sse_apply(sofft_plan* plan, int32_t op, const void* v, void* w, double E, double field,
                             void* stream) {
  if (!plan || !v || !w || (op != 0 && op != 1) || !std::isfinite(E) || !std::isfinite(field)) {
    set_error("bad argument to sofft_sse_apply");
    return SOFFT_EINVAL;
  }
  return sse_apply(*plan, op, v, w, E, field, reinterpret_cast<hipStream_t>(stream));
}

static bool shifts_ok(const double* eta, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(eta[i]) || eta[i] < 0.0) return false;
  return true;
}

sofft_status sofft_sse_solve_shifted(sofft_plan* plan, const void* f, int32_t f_per_energy, const double* E_host,
                                     const double* eta_host, int32_t nE, double field, void* x_out, double rtol,
                                     int32_t maxit, sofft_solve_stats* stats, void* stream) {
  if (!plan || !f || !E_host || !eta_host || nE <= 0 || !x_out || !(rtol > 0) || maxit <= 0 ||
      !std::isfinite(field)) {
    set_error("bad argument to sofft_sse_solve_shifted");
    return SOFFT_EINVAL;
  }
  for (int e = 0; e < nE; ++e)
    if (!std::isfinite(E_host[e])) {
      set_error("energies must be finite");
      return SOFFT_EINVAL;
    }
  if (!shifts_ok(eta_host, nE)) {
    set_error("shifts must be finite and >= 0");
    return SOFFT_EINVAL;
  }
  return sse_solve(*plan, f, f_per_energy, E_host, nE, field, x_out, rtol, maxit, stats,
                   reinterpret_cast<hipStream_t>(stream), nullptr, 0, eta_host);
}

sofft_status sofft_sse_apply_shifted(sofft_plan* plan, int32_t op, const void* v, void* w, double E, double eta,
                                     double field, void* stream) {
  if (!plan || !v || !w || (op != 0 && op != 1) || !std::isfinite(E) || !std::isfinite(field) ||
      !shifts_ok(&eta, 1)) {
    set_error("bad argument to sofft_sse_apply_shifted");
    return SOFFT_EINVAL;
  }
  return sse_apply(*plan, op, v, w, E, field, reinterpret_cast<hipStream_t>(stream), eta);
}

sofft_status sofft_sse_solve_banded(sofft_plan* plan, const void* f, int32_t f_per_energy, const double* E_host,
                                    int32_t nE, double field, void* x_out, double rtol, int32_t maxit,
                                    sofft_solve_stats* stats, void* stream) {
  if (!plan || !f || !E_host || nE <= 0 || !x_out || !(rtol > 0) || maxit <= 0 || !std::isfinite(field)) {
    set_error("bad argument to sofft_sse_solve_banded");
    return SOFFT_EINVAL;
  }
  for (int e = 0; e < nE; ++e)
    if (!std::isfinite(E_host[e])) {
      set_error("energies must be finite");
      return SOFFT_EINVAL;
    }
  return sse_solve(*plan, f, f_per_energy, E_host, nE, field, x_out, rtol, maxit, stats,
                   reinterpret_cast<hipStream_t>(stream), nullptr, 0, nullptr, 1);
}

sofft_status sofft_sse_apply_banded(sofft_plan* plan, int32_t op, const void* v, void* w, double E, double field,
                                    void* stream) {
  if (!plan || !v || !w || (op != 0 && op != 1) || !std::isfinite(E) || !std::isfinite(field)) {
    set_error("bad argument to sofft_sse_apply_banded");
    return SOFFT_EINVAL;
  }
  return sse_apply(*plan, op, v, w, E, field, reinterpret_cast<hipStream_t>(stream), 0.0, 1);
}

sofft_status sofft_sse_tune_shift(sofft_plan* plan, const void* f, const double* E_host, int32_t nE, double field,
                                  const double* eta_candidates, int32_t ncand, int32_t probe_iters, double rtol,
                                  void* scratch_x, double* eta_out, void* stream) {
  if (!plan || !f || !E_host || nE <= 0 || !eta_candidates || ncand <= 0 || probe_iters <= 0 ||
      !(rtol > 0) || !scratch_x || !eta_out || !std::isfinite(field)) {
    set_error("bad argument to sofft_sse_tune_shift");
    return SOFFT_EINVAL;
  }
  for (int e = 0; e < nE; ++e)
    if (!std::isfinite(E_host[e])) {
      set_error("energies must be finite");
      return SOFFT_EINVAL;
    }
  if (!shifts_ok(eta_candidates, ncand)) {
    set_error("shift candidates must be finite and >= 0");
    return SOFFT_EINVAL;
  }
  return sse_tune_shift(*plan, f, E_host, nE, field, eta_candidates, ncand, probe_iters, rtol, scratch_x, eta_out,
                        reinterpret_cast<hipStream_t>(stream));
}

sofft_status sofft_norm2(sofft_plan* plan, const void* psi, double* norm2_host, void* stream) {
  if (!plan || !psi || !norm2_host) {
    set_error("bad argument to sofft_norm2");
    return SOFFT_EINVAL;
  }
  return launch_norm2(*plan, psi, norm2_host, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"

// ---------------------------------------------------------------- timing aid
namespace sofft {

static hipEvent_t take_event(Timing& T) {
  if (!T.pool.empty()) {
    hipEvent_t e = T.pool.back();
    T.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

sofft_status Timing::begin(int kind, hipStream_t s) {
  if (!on) return SOFFT_OK;
  if (recs.size() >= 4096) {
    sofft_status st = drain();
    if (st != SOFFT_OK) return st;
  }
  Rec r{kind, take_event(*this), take_event(*this)};
  if (!r.a || !r.b) {
    set_error("hipEventCreate failed");
    return SOFFT_EHIP;
  }
  SOFFT_HIP_TRY(hipEventRecord(r.a, s));
  recs.push_back(r);
  return SOFFT_OK;
}

sofft_status Timing::end(hipStream_t s) {
  if (!on || recs.empty()) return SOFFT_OK;
  SOFFT_HIP_TRY(hipEventRecord(recs.back().b, s));
  return SOFFT_OK;
}

sofft_status Timing::drain() {
  for (auto& r : recs) {
    SOFFT_HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    SOFFT_HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    total_ms[r.kind] += ms;
    count[r.kind] += 1;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
  return SOFFT_OK;
}

void Timing::clear() {
  for (auto& r : recs) {
    (void)hipEventSynchronize(r.b);
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
  for (int k = 0; k < SOFFT_KERNEL_COUNT_; ++k) {
    total_ms[k] = 0;
    count[k] = 0;
  }
}

Timing::~Timing() {
  clear();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

}  // namespace sofft

extern "C" {

sofft_status sofft_timing_enable(sofft_plan* plan, int32_t enable) {
  if (!plan) {
    set_error("null plan");
    return SOFFT_EINVAL;
  }
  plan->timing.clear();
  plan->timing.on = enable != 0;
  return SOFFT_OK;
}

sofft_status sofft_timing_read(sofft_plan* plan, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!plan || !total_ms || !launches || kernel < 0 || kernel >= SOFFT_KERNEL_COUNT_) {
    set_error("bad argument to sofft_timing_read");
    return SOFFT_EINVAL;
  }
  sofft_status st = plan->timing.drain();
  if (st != SOFFT_OK) return st;
  *total_ms = plan->timing.total_ms[kernel];
  *launches = plan->timing.count[kernel];
  return SOFFT_OK;
}

}  // extern "C"
