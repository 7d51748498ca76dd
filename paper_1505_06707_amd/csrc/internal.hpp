// Internal declarations shared by the host plan code and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "cx.hpp"
#include "sofft.h"

namespace sofft {

using zc = std::complex<double>;

void set_error(const std::string& msg);

#define SOFFT_HIP_TRY(expr)                                                        \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::sofft::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));       \
      return SOFFT_EHIP;                                                           \
    }                                                                              \
  } while (0)

// Device copy of a host vector; owned by the plan.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// One Cartesian axis of a problem: host tables (built from Sec. II) and their
// device copies.
struct Axis {
  int64_t n = 0;
  double L = 0, h = 0, R0 = 0, theta = 0;
  int contour = SOFFT_SECS;
  std::vector<double> x, xm, k;
  std::vector<zc> q, qm, z;
  std::vector<zc> cdn, cdg, cup;  // C_{j,j-1}, C_{j,j}, C_{j,j+1}
  int64_t j0 = 0, m = 0;          // ECS strip: nodes (j0 + p) mod n, p < m

  // Device tables that do not depend on dt.  Every table is FP64: the
  // complex64 state is also transformed and propagated in FP64 arithmetic.
  DevBuf tw64, x_dev, z_dev, cstrip64;
  // Tables that depend on dt.
  double dt = 0;
  bool have_dt = false;
  int levels = 0;
  DevBuf kin_full64, kin_half64;
  DevBuf alpha64, gamma64, binv64;
  // Banded ECS eigen-preconditioner of this axis (built on first use).
  bool have_bands = false;
  DevBuf band_lam, band_xr, band_xc, band_start, band_width;
};

// Banded ECS eigen-preconditioner (banded.hip), Sec. III: bands of at most
// kBandMax consecutive momenta per axis.  Per FFT index n (n is the band row nu
// for X and the column m for X^T):
//   lam[n]                 eigenvalue of K_l belonging to row n
//   xr[i * n_axis + n]     X[n][s_n + i]   (i < w_n): y_n = sum_i xr v[s_n + i]
//   xc[i * n_axis + n]     X[s_n + i][n]   (i < w_n): z_n = sum_i xc y[s_n + i]
//   start[n] = s_n, width[n] = w_n of the band holding n
constexpr int kBandWidth = 10;
constexpr int kBandMax = 2 * kBandWidth - 1;
sofft_status band_tables(const Axis& a, std::vector<zc>& lam, std::vector<zc>& xr, std::vector<zc>& xc,
                         std::vector<int32_t>& start, std::vector<int32_t>& width);
sofft_status ensure_bands(Axis& a);

// Optional per-launch event timing (measurement aid).
struct Timing {
  bool on = false;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double total_ms[SOFFT_KERNEL_COUNT_] = {};
  int64_t count[SOFFT_KERNEL_COUNT_] = {};
  sofft_status begin(int kind, hipStream_t s);
  sofft_status end(hipStream_t s);
  sofft_status drain();
  void clear();
  ~Timing();
};

struct Plan {
  sofft_problem prob{};
  Axis ax[3];
  std::vector<double> host_partials;
  Timing timing;
  // Caller-owned device workspace (sofft_plan_bind); every buffer of O(grid)
  // size lives there, laid out by plan_ws_layout.
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // The workspace's potential-phase table holds exp(-i V0 dt/2) for the dt in
  // vphase_ht = dt/2 (NaN: not built, or the workspace changed since).
  double vphase_ht = __builtin_nan("");
  // A caller's potential U = V0 + f W (device, caller-owned): V0 complex
  // [ny][nx] in place of the soft-core, W real [ny][nx] in place of x; null:
  // the problem's own.
  const void* user_v0 = nullptr;
  const double* user_w = nullptr;
};

// Layout of a plan's caller workspace: the potential-phase table (the whole
// grid, complex128: room for a caller's V0), the norm partial sums, then the
// stationary solver's region for n_energies energies (none for 0).  Regions
// start on 256-byte boundaries.
struct WsLayout {
  size_t vphase = 0, partials = 0, solver = 0;
  size_t solver_bytes = 0;
  size_t total = 0;
};
constexpr int kNormBlocks = 1024;
WsLayout plan_ws_layout(const Plan& p, int n_energies);
// Checks that the bound workspace holds the layout for n_energies energies
// (SOFFT_EWORKSPACE with a message naming the size otherwise).
sofft_status plan_ws_check(const Plan& p, int n_energies, WsLayout* L);
inline char* ws_at(const Plan& p, size_t off) { return static_cast<char*>(p.ws) + off; }
// Bytes of the stationary solver's region for nE energies (sse.hip).
size_t sse_solver_bytes(const Plan& p, int nE);

// Table builders (plan.hip).
sofft_status build_axis(Axis& a, int64_t n, double L, double R0, double theta, int contour);
sofft_status upload_static(Axis& a, bool bands);
sofft_status ensure_dt(Axis& a, double dt);
void free_axis(Axis& a);
// Device tables of a plan are reserved once, in sofft_plan_create, at their
// largest size (dev_reserve); later calls only copy into them (dev_upload
// fails if the copy would not fit, which would be a library bug).
sofft_status dev_reserve(DevBuf& b, size_t bytes);
sofft_status dev_upload(DevBuf& b, const void* host, size_t bytes);
// Raise a kernel's dynamic LDS limit to `limit` bytes, once per kernel (the
// attribute belongs to the function; the call is made the first time a launch
// needs more than the default 64 KiB).  Thread-safe.
sofft_status raise_lds_limit(const void* kernel, size_t limit);
void dev_free(DevBuf& b);

// Launch shape of a 2D pass: threads per block (0 = default) and grid (0 =
// one block per tile of lines, else a persistent grid of at most that many
// blocks looping over the tiles).
struct PassLaunch {
  int threads = 0;
  int grid = 0;
};

// One row or column pass over the states of nruns runs that share a plan
// (batched propagation).  runs / f_runs are device arrays of nruns pointers;
// the field of run r at step s is f_runs[r][s + *step_base] (f_runs may be
// null: no field; step_base may be null: offset 0).
struct PassRequest {
  bool row = true;
  bool half_kinetic = false;
  int do_pot = 1;
  double dt = 0;
  void* const* runs = nullptr;
  const double* const* f_runs = nullptr;
  int nruns = 0;
  int64_t step = 0;
  const int64_t* step_base = nullptr;
  PassLaunch cfg;
  Timing* timing = nullptr;
};

// Launchers (tdse.hip).
// Propagation (1D or 2D) with the phase table in the plan's workspace, or in
// the library's static device scratch (no allocation, no workspace).
sofft_status launch_propagate(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid, hipStream_t s);
sofft_status launch_propagate_static(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                     hipStream_t s);
size_t vphase_bytes(const Plan& p);
// 3D grids (tdse3d.hip).
sofft_status launch_propagate_3d(Plan& p, void* psi, double dt, int64_t nsteps, const double* f_mid,
                                 const cx<double>* vph, hipStream_t s);
sofft_status build_octant_vphase(const Plan& p, double dt, cx<double>* table, hipStream_t s);
sofft_status launch_softcore_3d(const Plan& p, double charge, double a2, void* out, hipStream_t s);
sofft_status launch_norm2(Plan& p, const void* psi, double* out, hipStream_t s);
// V0 = -charge / sqrt(sum z^2 + a2) on the plan's grid into out (complex, [ny][nx]).
sofft_status launch_softcore(const Plan& p, double charge, double a2, void* out, hipStream_t s);
sofft_status launch_absorber(const Plan& p, int kind, double param, void* v0, hipStream_t s);
sofft_status launch_pass(Plan& p, const PassRequest& rq, hipStream_t s);
// Build or refresh the potential-phase table of a plan for dt (enqueued on s).
sofft_status ensure_vphase(Plan& p, double dt, hipStream_t s, bool* changed,
                           const cx<double>** table = nullptr);
sofft_status pass_residency(const Plan& p, bool row, int threads, int* blocks_per_cu, int* block_threads);
// *counter += delta by one device thread (graph-safe step offsets).
sofft_status launch_step_add(int64_t* counter, int64_t delta, bool set, hipStream_t s);
// partials[r * 64 + b] = partial sums of |psi_r|^2 (64 blocks per run), FP64.
sofft_status launch_norm2_runs(const void* const* runs_dev, int nruns, int64_t npoints, bool c128,
                               double* partials, hipStream_t s);
bool supported_length(int64_t n);

// Learned correction network (learned.hip).
struct LpNet;
sofft_status lp_apply(LpNet& net, const cx<double>* r, cx<double>* z, int B, int H, int W, const int* active,
                      const double* scale, hipStream_t s);

// Stationary solver (sse.hip).  lp = null: plain FFT preconditioner (COCG);
// otherwise flexible COCG with the learned correction and the fallback.
// eta_host (nE shifts, may be null): divisor K - E - i eta of the
// preconditioner per energy.
sofft_status sse_solve(Plan& p, const void* f, int f_per_energy, const double* E_host, int nE, double field,
                       void* x_out, double rtol, int maxit, sofft_solve_stats* stats, hipStream_t s,
                       LpNet* lp = nullptr, int patience = 0, const double* eta_host = nullptr, int banded = 0);
sofft_status sse_apply(Plan& p, int op, const void* v, void* w, double E, double field, hipStream_t s,
                       double eta = 0.0, int banded = 0);
sofft_status sse_tune_shift(Plan& p, const void* f, const double* E_host, int nE, double field,
                            const double* cand, int ncand, int probe_iters, double rtol, void* scratch_x,
                            double* eta_out, hipStream_t s);

}  // namespace sofft
