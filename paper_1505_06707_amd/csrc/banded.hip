// Host side of the banded ECS eigen-preconditioner (Sec. III, Eqs.
// Prec_eigen_eq, K_l and PreconFFT_ECS): per axis, the spectrum is cut into
// bands of consecutive momenta; on each band the complex-symmetric block
//   [K_l]_{nm} = 1/2 k_n k_m Q(m - n),  Q(d) = (1/N) sum_j q_j^-2 e^{i 2 pi d x_j / L}
// (the Fourier-basis block of K_a = -1/2 d/dx q^-2 d/dx, Q by the grid
// quadrature) is diagonalised by a complex orthogonal X (X^T X = 1), and
// P^-1 = F^-1 X^T (Lambda - E)^-1 X F.  The device part lives in the stationary
// solver's preconditioner passes.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace sofft {

// The paper's split, in FFT index order: {0} and {N/2} alone; the positive
// momenta 1..N/2-1 from k_1 outward in bands of kBandWidth, the remainder joined
// to the band next to N/2; the negative momenta mirror the positive ones.
static std::vector<std::pair<int, int>> band_list(int n) {
  std::vector<std::pair<int, int>> out;   // (first index, width)
  const int half = n / 2, npos = half - 1;
  out.push_back({0, 1});
  out.push_back({half, 1});
  const int nfull = npos / kBandWidth;
  std::vector<std::pair<int, int>> pos;
  if (nfull == 0) {
    if (npos > 0) pos.push_back({1, npos});
  } else {
    for (int b = 0; b < nfull - 1; ++b) pos.push_back({1 + b * kBandWidth, kBandWidth});
    const int s = 1 + (nfull - 1) * kBandWidth;
    pos.push_back({s, half - s});
  }
  for (const auto& b : pos) {
    out.push_back(b);
    out.push_back({n - (b.first + b.second - 1), b.second});   // mirror: indices n - i
  }
  return out;
}

// Eigen-decomposition of a complex-symmetric w x w matrix A (row-major) by
// cyclic Jacobi rotations that are complex orthogonal (c^2 + s^2 = 1): the
// product V of the rotations satisfies V^T V = 1 and V^T A V = diag(lam), so
// the columns of V are eigenvectors already normalised by chi^T chi = 1.
// Returns false if a rotation is undefined (1 + t^2 = 0) or it does not converge.
static bool jacobi_complex_symmetric(int w, std::vector<zc> A, std::vector<zc>& lam, std::vector<zc>& V) {
  V.assign(size_t(w) * w, 0.0);
  for (int i = 0; i < w; ++i) V[size_t(i) * w + i] = 1.0;
  auto at = [&](int r, int c) -> zc& { return A[size_t(r) * w + c]; };
  double scale = 0.0;
  for (const zc& v : A) scale = std::max(scale, std::abs(v));
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < w; ++p)
      for (int q = p + 1; q < w; ++q) off = std::max(off, std::abs(at(p, q)));
    if (off <= 1e-15 * scale || scale == 0.0) {
      lam.resize(w);
      for (int i = 0; i < w; ++i) lam[i] = at(i, i);
      return true;
    }
    for (int p = 0; p < w; ++p)
      for (int q = p + 1; q < w; ++q) {
        const zc apq = at(p, q);
        if (std::abs(apq) <= 1e-300) continue;
        const zc theta = (at(q, q) - at(p, p)) / (2.0 * apq);
        const zc r = std::sqrt(theta * theta + 1.0);
        const zc den = std::abs(theta + r) >= std::abs(theta - r) ? theta + r : theta - r;
        const zc t = 1.0 / den;
        const zc cc = 1.0 + t * t;
        if (std::abs(cc) < 1e-12) return false;
        const zc c = 1.0 / std::sqrt(cc), s = t * c;
        at(p, p) -= t * apq;
        at(q, q) += t * apq;
        at(p, q) = 0.0;
        at(q, p) = 0.0;
        for (int k = 0; k < w; ++k) {
          if (k == p || k == q) continue;
          const zc akp = at(k, p), akq = at(k, q);
          at(k, p) = at(p, k) = c * akp - s * akq;
          at(k, q) = at(q, k) = s * akp + c * akq;
        }
        for (int k = 0; k < w; ++k) {
          const zc vkp = V[size_t(k) * w + p], vkq = V[size_t(k) * w + q];
          V[size_t(k) * w + p] = c * vkp - s * vkq;
          V[size_t(k) * w + q] = s * vkp + c * vkq;
        }
      }
  }
  return false;
}

sofft_status band_tables(const Axis& a, std::vector<zc>& lam, std::vector<zc>& xr, std::vector<zc>& xc,
                         std::vector<int32_t>& start, std::vector<int32_t>& width) {
  const int n = int(a.n);
  const double pi = 3.14159265358979323846;
  lam.assign(n, 0.0);
  xr.assign(size_t(kBandMax) * n, 0.0);
  xc.assign(size_t(kBandMax) * n, 0.0);
  start.assign(n, 0);
  width.assign(n, 0);
  // Q(d) for |d| < kBandMax by the grid quadrature
  std::vector<zc> Qd(2 * kBandMax - 1);
  for (int d = -(kBandMax - 1); d <= kBandMax - 1; ++d) {
    zc acc = 0.0;
    for (int j = 0; j < n; ++j) acc += std::exp(zc(0.0, 2 * pi * d * a.x[j] / a.L)) / (a.q[j] * a.q[j]);
    Qd[d + kBandMax - 1] = acc / double(n);
  }
  for (const auto& b : band_list(n)) {
    const int s0 = b.first, w = b.second;
    if (w > kBandMax) {
      set_error("internal: band wider than the table");
      return SOFFT_EUNSUPPORTED;
    }
    std::vector<zc> K(size_t(w) * w), ev, V;
    for (int i = 0; i < w; ++i)
      for (int j = 0; j < w; ++j)
        K[size_t(i) * w + j] = 0.5 * a.k[s0 + i] * a.k[s0 + j] * Qd[(j - i) + kBandMax - 1];
    if (!jacobi_complex_symmetric(w, K, ev, V)) {
      set_error("banded preconditioner: the eigen-decomposition of a band did not converge");
      return SOFFT_EUNSUPPORTED;
    }
    // X = V^T: row nu of X is eigenvector nu (column nu of V)
    for (int nu = 0; nu < w; ++nu) {
      const int n_idx = s0 + nu;
      lam[n_idx] = ev[nu];
      start[n_idx] = s0;
      width[n_idx] = w;
      for (int i = 0; i < w; ++i) {
        xr[size_t(i) * n + n_idx] = V[size_t(i) * w + nu];   // X[nu][i] = V[i][nu]
        xc[size_t(i) * n + n_idx] = V[size_t(nu) * w + i];   // X[i][nu] = V[nu][i]
      }
    }
  }
  return SOFFT_OK;
}

sofft_status ensure_bands(Axis& a) {
  if (a.have_bands) return SOFFT_OK;
  std::vector<zc> lam, xr, xc;
  std::vector<int32_t> st, wd;
  sofft_status s = band_tables(a, lam, xr, xc, st, wd);
  if (s != SOFFT_OK) return s;
  // The kernels transform with the plain DFT, exp(-2 pi i m j / n); the basis
  // of Sec. II has F_mj = exp(-i k_m x_j)/sqrt(n) = ph_m exp(-2 pi i m j / n)/sqrt(n)
  // with ph_m = exp(-i k_m x_0) on the cell-centred grid.  A diagonal divisor does
  // not see ph; X does: in the DFT basis it is X ph (columns scaled by ph_m)
  // and X^T becomes ph^-1 X^T (rows scaled by 1/ph_n).
  const int64_t n = a.n;
  std::vector<zc> ph(n);
  for (int64_t m = 0; m < n; ++m) ph[m] = std::exp(zc(0.0, -a.k[m] * a.x[0]));
  for (int64_t idx = 0; idx < n; ++idx)
    for (int i = 0; i < wd[idx]; ++i) {
      xr[size_t(i) * n + idx] *= ph[st[idx] + i];
      xc[size_t(i) * n + idx] /= ph[idx];
    }
  if ((s = dev_upload(a.band_lam, lam.data(), lam.size() * sizeof(zc))) != SOFFT_OK) return s;
  if ((s = dev_upload(a.band_xr, xr.data(), xr.size() * sizeof(zc))) != SOFFT_OK) return s;
  if ((s = dev_upload(a.band_xc, xc.data(), xc.size() * sizeof(zc))) != SOFFT_OK) return s;
  if ((s = dev_upload(a.band_start, st.data(), st.size() * sizeof(int32_t))) != SOFFT_OK) return s;
  if ((s = dev_upload(a.band_width, wd.data(), wd.size() * sizeof(int32_t))) != SOFFT_OK) return s;
  a.have_bands = true;
  return SOFFT_OK;
}

}  // namespace sofft

using namespace sofft;

extern "C" sofft_status sofft_band_tables(const sofft_problem* prob, int32_t axis, double* lambda_out,
                                          double* x_rows_out, int32_t* band_start, int32_t* band_width) {
  if (!prob || !lambda_out || !x_rows_out || !band_start || !band_width || axis < 0 || axis >= prob->ndim ||
      (prob->ndim != 1 && prob->ndim != 2)) {
    set_error("bad argument to sofft_band_tables");
    return SOFFT_EINVAL;
  }
  const int64_t n_ax = prob->n[axis];
  const bool known = prob->contour == SOFFT_SECS || prob->contour == SOFFT_SHARP ||
                     prob->contour == SOFFT_ECS_OFF || prob->contour == SOFFT_TFECS;
  if (n_ax < 4 || n_ax % 2 != 0 || n_ax > (1 << 20) || !(prob->L[axis] > 0) || !known || !(prob->theta > 0) ||
      (prob->contour != SOFFT_ECS_OFF && !(prob->R0[axis] > 0 && prob->R0[axis] < prob->L[axis] / 2))) {
    set_error("bad problem in sofft_band_tables");
    return SOFFT_EINVAL;
  }
  Axis a;
  sofft_status s = build_axis(a, n_ax, prob->L[axis], prob->R0[axis], prob->theta, prob->contour);
  if (s != SOFFT_OK) return s;
  std::vector<zc> lam, xr, xc;
  std::vector<int32_t> st, wd;
  if ((s = band_tables(a, lam, xr, xc, st, wd)) != SOFFT_OK) return s;
  const int64_t n = a.n;
  for (int64_t i = 0; i < n; ++i) {
    lambda_out[2 * i] = lam[i].real();
    lambda_out[2 * i + 1] = lam[i].imag();
    band_start[i] = st[i];
    band_width[i] = wd[i];
    for (int j = 0; j < kBandMax; ++j) {
      const zc v = xr[size_t(j) * n + i];
      x_rows_out[2 * (i * kBandMax + j)] = v.real();
      x_rows_out[2 * (i * kBandMax + j) + 1] = v.imag();
    }
  }
  return SOFFT_OK;
}
