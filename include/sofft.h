/*
 * libsofft -- split-operator FFT propagation of the complex-scaled
 * Schroedinger equation and FFT-preconditioned conjugate gradients for the
 * stationary equation, for AMD Instinct MI355X (gfx950).
 *
 * Method: V. V. Serov and T. A. Sergeeva, "Solution of the Schroedinger
 * equation using exterior complex scaling and fast Fourier transform"
 * (arXiv:1505.06707).  Sec. II defines the grid, the Fourier basis, the ECS
 * contour and the split-operator step; Sec. III defines the stationary system
 * and its FFT preconditioner.
 *
 * Conventions shared by every call:
 *  - Grid (Sec. II, Eq. DVRgrid): on a box of length L per axis the nodes are
 *    the cell centres x_j = -L/2 + h (j + 1/2), h = L/n, j = 0..n-1.
 *  - Arrays are complex, interleaved (re, im), in device memory, row-major with
 *    x the fast axis: psi[(j_z * n_y + j_y) * n_x + j_x] (the z and y terms
 *    only in 3D and 2D).  Element type: double2 for
 *    SOFFT_C128 plans, float2 for SOFFT_C64 plans.
 *  - The values held are those of the scaled function psi~(x) = sqrt(q(x))
 *    psi(z(x)) (Sec. II, Eq. psi_zx).
 *  - Device buffers passed in are owned by the caller; the library never frees
 *    them.  Ownership of device memory:
 *      * a plan owns its small device tables (O(n) elements per axis: grid,
 *        contour, twiddles, kinetic phases, Crank-Nicolson coefficients, and
 *        for 2D complex128 plans the banded-preconditioner blocks), allocated
 *        once by sofft_plan_create at their largest size and freed by
 *        sofft_plan_destroy;
 *      * every buffer of the size of a grid or larger (potential-phase table,
 *        reduction partials, the stationary solver's vectors) lives in a
 *        workspace the caller allocates and binds (sofft_workspace_size,
 *        sofft_plan_bind; sofft_batch_workspace_size, sofft_batch_bind for
 *        batches).  After sofft_plan_create no call allocates device memory
 *        (the learned-correction object and batch creation aside: see there).
 *    A call that needs more workspace than is bound returns SOFFT_EWORKSPACE.
 *  - Work is enqueued on the HIP stream given as `stream` (NULL = the default
 *    stream) and is asynchronous unless the call writes to host memory.
 *  - Errors: negative status codes; nothing has been enqueued when one is
 *    returned, and sofft_last_error() (per thread) describes it.
 *  - Plans are not thread-safe: one host thread at a time per plan.
 */
#ifndef SOFFT_H_
#define SOFFT_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SOFFT_OK = 0,
  SOFFT_EINVAL = -1,        /* bad argument (null pointer, size, range) */
  SOFFT_EUNSUPPORTED = -2,  /* valid but not implemented (e.g. grid length) */
  SOFFT_EHIP = -3,          /* HIP runtime error */
  SOFFT_ENOMEM = -4,        /* device allocation failed */
  SOFFT_EWORKSPACE = -5,    /* no workspace bound, or smaller than the call needs */
  SOFFT_NOT_CONVERGED = 1,  /* solver hit maxit before rtol */
  SOFFT_BREAKDOWN = 2       /* COCG breakdown that a restart did not cure */
} sofft_status;

typedef enum { SOFFT_C128 = 0, SOFFT_C64 = 1 } sofft_dtype;

/* ECS contour q(x), Sec. IV.  SOFFT_SECS: q = exp(i theta (|x|-R0)/(L/2-R0))
 * for |x| > R0 (Eq. qSECS with the end angle pi/4 replaced by theta).
 * SOFFT_SHARP: q = exp(i theta) for |x| - R0 > 1e-9 h.  SOFFT_ECS_OFF: q = 1.
 * SOFFT_TFECS: q = sqrt(1 + i y(s)) for |x| > R0 (Eq. qTFECS), s = (|x|-R0)/(L/2-R0),
 * y(s) = alpha [(1-s)^-2 - (1+s)^-2 - 4s], with alpha passed as theta (> 0;
 * the paper uses 0.5).  q is infinite at the box edge, where the stencil of C
 * then does not couple; z(x) = int q is integrated numerically (composite
 * Gauss-Legendre) and is finite at every node. */
typedef enum { SOFFT_SECS = 0, SOFFT_SHARP = 1, SOFFT_ECS_OFF = 2, SOFFT_TFECS = 3 } sofft_contour;

/* The problem statement of Sec. II/III: grid, ECS radius and angle, and the
 * static part of U.  U(x, t) = V0(z(x)) + f(t) x with the soft-core Coulomb
 * V0 = -charge / sqrt(z_x^2 [+ z_y^2 [+ z_z^2]] + a2) evaluated on the complex contour
 * (principal branch) and the dipole term f(t) x at the real coordinate x
 * (polarisation along x).  charge = 0 switches V0 off. */
typedef struct {
  int32_t ndim;      /* 1, 2 or 3 */
  int32_t dtype;     /* sofft_dtype of psi */
  int64_t n[3];      /* nodes per axis: n[0] = n_x (fast), n[1] = n_y, n[2] = n_z (slowest) */
  double L[3];       /* box length per axis */
  double R0[3];      /* ECS radius per axis, 0 < R0 < L/2 (ignored if contour off) */
  double theta;      /* ECS angle, 0 < theta < pi/2 (SECS, sharp); alpha > 0 (TFECS) */
  int32_t contour;   /* sofft_contour */
  double charge;     /* soft-core strength (>= 0) */
  double a2;         /* soft-core parameter a^2 (> 0 if charge > 0) */
} sofft_problem;

typedef struct sofft_plan sofft_plan;

/* Message describing the last error on this host thread ("" if none). */
const char* sofft_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int32_t sofft_version(void);

/* Build a plan: grid, momenta, contour tables q, z, the ECS remainder
 * C = K_s - K_FD (Sec. II, Eqs. C_FD, Ks_FD, K_FD, periodic stencils) and FFT
 * twiddles, and copy them to the current device.  Supported n per axis:
 * 16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024 (1D and 2D), 2048,
 * 4096 (1D only), 16, 32, 64, 128, 256, 512 (3D).  The ECS strip (nodes where
 * C is non-zero) may hold at most half of the nodes of an axis, and at most
 * 256 nodes per axis in 2D and 3D.  3D: the paper is 1D and names the
 * many-dimensional case as its next step; the step is read separably,
 * K = (k_x^2 + k_y^2 + k_z^2)/2 and e^{-iC dt} = CN(C_x) CN(C_y) CN(C_z).
 * The stationary solver takes complex128 plans of any dimension (its learned
 * correction 2D only); batches take 2D plans.
 * Returns SOFFT_EINVAL / SOFFT_EUNSUPPORTED / SOFFT_ENOMEM / SOFFT_EHIP. */
sofft_status sofft_plan_create(const sofft_problem* prob, sofft_plan** out);

/* Free the plan and its device tables (after the work using it has finished).
 * A bound workspace stays the caller's. */
sofft_status sofft_plan_destroy(sofft_plan* plan);

/* Bytes of device workspace the plan needs for sofft_propagate, sofft_norm2
 * and, with n_energies > 0, for stationary solves and applications of up to
 * n_energies energies at once (complex128 plans; SOFFT_EUNSUPPORTED
 * otherwise).  About 16 bytes per grid point for propagation (the table of
 * exp(-i V0 dt/2), room for a caller's V0), plus about (5 n_energies + 1) 16
 * bytes per grid point for solves.  Host only: nothing is enqueued. */
sofft_status sofft_workspace_size(const sofft_plan* plan, int32_t n_energies, int64_t* bytes);

/* Bind a caller-owned device workspace of `bytes` bytes (256-byte aligned, on
 * the plan's device) to the plan; NULL unbinds.  The plan keeps the pointer
 * and lays out its buffers in it; the memory must stay valid, and must not be
 * used by anything else, while work enqueued on the plan can still run.
 * Binding again (another or the same memory) makes the next propagation
 * rebuild its potential-phase table.  Calls that need more than what is bound
 * (sofft_workspace_size) return SOFFT_EWORKSPACE and enqueue nothing. */
sofft_status sofft_plan_bind(sofft_plan* plan, void* workspace, int64_t bytes);

/* Copy the n[axis] node coordinates x_j (Sec. II, Eq. DVRgrid) to host memory. */
sofft_status sofft_grid_nodes(const sofft_plan* plan, int32_t axis, double* x_host);

/* Number of nodes on the ECS strip of an axis, i.e. the nodes where the
 * remainder C has a non-zero row (0 when ECS is off). */
sofft_status sofft_strip_length(const sofft_plan* plan, int32_t axis, int64_t* m);

/* Replace the potential of the plan by U(x, t) = V0(x) + f(t) W(x) (the
 * general U(z(x), t) of Sec. II, Eq. TDSE, with a dipole-like time dependence):
 *   v0  device, complex128 [n_y][n_x] (interleaved re, im), V0 already evaluated
 *       at the complex coordinates z(x) of the contour; NULL: the problem's
 *       soft-core (charge, a2)
 *   w   device, double [n_y][n_x], real; NULL: W = x (polarisation along x)
 * Both stay owned by the caller and are read, not copied: they must stay
 * valid, and unchanged, while propagations and solves on the plan use them
 * (W is read at every step; the phase table exp(-i V0 dt/2) is rebuilt from
 * V0 at the next propagation, or for a new dt).  Call again after changing
 * V0.  Applies to sofft_propagate and the sofft_sse_* solves and applications
 * (whose U is V0 + field W).  Takes effect for work enqueued after the call;
 * work already enqueued still reads the previous buffers, which must stay
 * valid until it finishes.  sofft_set_potential(plan, NULL, NULL) restores the
 * problem's potential.  Returns SOFFT_EINVAL for a NULL plan. */
sofft_status sofft_set_potential(sofft_plan* plan, const void* v0, const double* w);

/* Write the soft-core V0 = -charge / sqrt(z_x^2 [+ z_y^2] + a2) (principal
 * branch) on the plan's grid, at the contour coordinates z, into v0 (device,
 * complex128 [n_y][n_x]; caller-owned).  A helper for sofft_set_potential:
 * scale, shift or add to it before passing it there.  charge and a2 finite,
 * a2 > 0 unless charge = 0.  Asynchronous on the stream. */
sofft_status sofft_make_softcore(const sofft_plan* plan, double charge, double a2, void* v0, void* stream);

/* Complex absorbing potentials of Sec. IV, the alternatives to ECS that the
 * paper compares it with: a potential U_a added to U on a grid that is not
 * scaled (a plan with contour SOFFT_ECS_OFF, so q = 1 and z = x).  On each
 * axis, with r_s = R0[axis] (which must lie in (0, L/2) for this call even
 * though the contour is off), Dx_CS = L/2 - r_s and s = (|x| - r_s)/Dx_CS at
 * the real node x, U_a = 0 for |x| <= r_s and beyond:
 *   SOFFT_ABSORBER_CAP   U_a = E_cap [1 - q(x)^2] with q of Eq. qSECS (end
 *                        angle pi/4): E_cap [1 - exp(i pi s/2)] (Eq. CAP_via_q);
 *                        param = E_cap (the paper: 2)
 *   SOFFT_ABSORBER_TFAP  U_a = -i (k_min^2/2) y(s), y(s) = [a s - b s^3
 *                        + 4/(1-s)^2 - 4/(1+s)^2]/c^2, a = c^3 - 16,
 *                        b = c^3 - 17, c = 2.622057 (Eqs. TFAP, yTFAP);
 *                        param = k_min (the paper: 0.25)
 * On a grid of several dimensions the axis terms are summed.  The call ADDS
 * U_a to v0 (device, complex128, the plan's grid [n_z][n_y][n_x], caller-owned;
 * start it from sofft_make_softcore or zeros) and enqueues one kernel on the
 * stream; pass the result to sofft_set_potential.  The nodes stop half a cell
 * short of the box edge, so y(s) is finite at every node.  Returns
 * SOFFT_EINVAL for a NULL plan or v0, an unknown kind, param not finite and
 * positive, or an R0 outside (0, L/2). */
typedef enum { SOFFT_ABSORBER_CAP = 0, SOFFT_ABSORBER_TFAP = 1 } sofft_absorber;
sofft_status sofft_add_absorber(const sofft_plan* plan, int32_t kind, double param, void* v0, void* stream);

/* Advance psi (device, in place, n_x [* n_y] elements) by nsteps split-operator
 * steps of length dt (Sec. II):
 *   psi <- F^-1 e^{-iK dt/2} F  e^{-iU dt/2}  e^{-iC dt}  e^{-iU dt/2}  F^-1 e^{-iK dt/2} F  psi
 * with e^{-iC dt} by Crank-Nicolson, (1 + i dt C/2)^-1 (1 - i dt C/2), and U at
 * the step midpoint: f_mid[s] = f(t0 + (s + 1/2) dt) is read from device memory
 * (nsteps doubles; may be NULL when there is no field).  In 2D,
 * K = (k_x^2 + k_y^2)/2 and e^{-iC dt} = CN(C_x) CN(C_y).  Neighbouring kinetic
 * half-steps of consecutive steps are applied as one full step, which is exact.
 * dt may be negative (backward propagation).  nsteps = 0 is a no-op.  Needs
 * the workspace of sofft_workspace_size(plan, 0) bound (SOFFT_EWORKSPACE). */
sofft_status sofft_propagate(sofft_plan* plan, void* psi, double dt, int64_t nsteps,
                             const double* f_mid, void* stream);

/* sofft_propagate for callers that cannot allocate or bind device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same steps and kernels, with the one scratch buffer of a
 * propagation, the table of exp(-i V0 dt/2), in a static device array of
 * 8 MiB that the library holds on each GPU it runs on until the process ends
 * (no workspace needs to be bound; nothing is allocated by the call).  Every
 * call rebuilds the table there, so calls that overlap on one GPU (several
 * streams or host threads) race and must be serialised by the caller.  A
 * plan whose table exceeds 8 MiB (a caller's V0 on more than 2^19 grid
 * points; the soft-core table, a quarter of the grid, always fits) returns
 * SOFFT_EUNSUPPORTED.  The first call for a new dt copies the plan's
 * dt-dependent tables synchronously (make it outside a graph capture).
 * Results are bit-identical to sofft_propagate. */
sofft_status sofft_propagate_static(sofft_plan* plan, void* psi, double dt, int64_t nsteps,
                                    const double* f_mid, void* stream);

/* ||psi||^2 = sum |psi_j|^2 accumulated in FP64 (blocking: waits for the
 * stream).  Its partial sums use the bound workspace. */
sofft_status sofft_norm2(sofft_plan* plan, const void* psi, double* norm2_host, void* stream);

/* Outcome of one energy of sofft_sse_solve. */
typedef struct {
  int32_t iterations;    /* COCG iterations (all restarts included) */
  int32_t status;        /* SOFFT_OK, SOFFT_NOT_CONVERGED or SOFFT_BREAKDOWN */
  int32_t restarts;      /* restarts from the true residual */
  int32_t fell_back;     /* learned solve only: 1 if it switched to the plain preconditioner */
  double rel_residual;   /* ||f - A x|| / ||f||, recomputed from x (Hermitian 2-norm) */
} sofft_solve_stats;

/* Solve the stationary equation with exterior complex scaling of Sec. III,
 *   [K_s + U - E_j] x_j = f   (Eq. linsys: A = F^-1 K F + C + U - E I),
 * for nE energies at once by preconditioned conjugate gradients for the
 * complex-symmetric A (COCG: unconjugated u^T v) with the FFT preconditioner
 * P^-1 = F^-1 (K - E)^-1 F of Eq. PreconFFT, starting from x = 0.  U is the
 * static potential of the plan plus field * x (field = 0 after a pulse).
 * Iterations stop when ||r|| / ||f|| <= rtol (Hermitian 2-norm of the
 * recurrence residual); the residual is then recomputed as f - A x and the
 * iteration restarts from it while that exceeds rtol.  The same restart is
 * taken when the recurrence residual has made no new minimum for 2000
 * iterations (stagnation in finite precision); stats.restarts counts both,
 * and an energy stops as SOFFT_NOT_CONVERGED after 8 restarts.
 *   f       device, [n_y][n_x] (f_per_energy = 0, shared) or [nE][n_y][n_x]
 *           ([n_x] and [nE][n_x] on 1D plans, [n_z][n_y][n_x] and
 *           [nE][n_z][n_y][n_x] on 3D plans)
 *   E_host  host, nE energies
 *   x_out   device, [nE][n_y][n_x] ([nE][n_x] in 1D, [nE][n_z][n_y][n_x] in 3D), written
 *   stats   host, nE entries (may be NULL)
 * Complex128 plans of 1, 2 or 3 dimensions.  In 3D (Sec. III: the FFT
 * preconditioner carries over to the many-dimensional case)
 * K = (k_x^2 + k_y^2 + k_z^2)/2, C = C_x + C_y + C_z and P^-1 uses the full 3D
 * transform.  In 1D (the setting of the paper's example, Sec. V) every energy
 * is one workgroup that runs the whole iteration on chip: the call is one
 * launch, and its stats and x are final when it returns.  The bound
 * workspace must hold sofft_workspace_size(plan, nE) bytes (about
 * (5 nE + 1) 16 bytes per grid point).
 * Blocking: returns after the solve.  Returns SOFFT_OK when every energy met
 * rtol, else SOFFT_NOT_CONVERGED / SOFFT_BREAKDOWN (per energy in stats). */
sofft_status sofft_sse_solve(sofft_plan* plan, const void* f, int32_t f_per_energy, const double* E_host,
                             int32_t nE, double field, void* x_out, double rtol, int32_t maxit,
                             sofft_solve_stats* stats, void* stream);

/* One application of the stationary matrix (op 0: w = A v, Eq. linsys) or of
 * the FFT preconditioner (op 1: w = P^-1 v, Eq. PreconFFT) at energy E, on
 * device vectors [n_y][n_x] ([n_x] on 1D plans, [n_z][n_y][n_x] on 3D plans).  Needs the workspace of one energy
 * (sofft_workspace_size(plan, 1)).  Asynchronous on the stream. */
sofft_status sofft_sse_apply(sofft_plan* plan, int32_t op, const void* v, void* w, double E, double field,
                             void* stream);

/* sofft_sse_solve with a shifted divisor in the FFT preconditioner of
 * Eq. PreconFFT: P^-1 = F^-1 (K - E_j - i eta_j)^-1 F for energy j.  This is
 * not the paper's preconditioner (eta = 0 is).  The symbol stays even in k, so
 * P^-1 stays complex symmetric and the COCG recurrences of sofft_sse_solve
 * apply unchanged; the solution x_j of Eq. linsys is the same, only the
 * iteration count changes.
 *   eta_host  host, nE shifts, finite and >= 0 (an entry of 0 gives exactly the
 *             arithmetic of sofft_sse_solve for that energy)
 * Other arguments, workspace, blocking and status: as sofft_sse_solve;
 * SOFFT_EINVAL for a negative or non-finite shift. */
sofft_status sofft_sse_solve_shifted(sofft_plan* plan, const void* f, int32_t f_per_energy, const double* E_host,
                                     const double* eta_host, int32_t nE, double field, void* x_out, double rtol,
                                     int32_t maxit, sofft_solve_stats* stats, void* stream);

/* sofft_sse_apply with the shifted divisor (op 1: w = F^-1 (K - E - i eta)^-1 F v;
 * op 0 ignores eta).  eta finite and >= 0, else SOFFT_EINVAL.  Asynchronous. */
sofft_status sofft_sse_apply_shifted(sofft_plan* plan, int32_t op, const void* v, void* w, double E, double eta,
                                     double field, void* stream);

/* sofft_sse_solve with the banded ECS eigen-preconditioner of Sec. III,
 * Eq. PreconFFT_ECS, instead of Eq. PreconFFT: in 2D
 *   P^-1 = F^-1 (X_x (x) X_y)^T (lambda_x + lambda_y - E)^-1 (X_x (x) X_y) F,
 * and in 3D with X = X_x (x) X_y (x) X_z and lambda_x + lambda_y + lambda_z - E,
 * with X and lambda of each axis as sofft_band_tables describes (built on the
 * first call and kept by the plan).  Arguments, workspace, blocking and status
 * as sofft_sse_solve; SOFFT_EUNSUPPORTED if a band's eigen-decomposition fails. */
sofft_status sofft_sse_solve_banded(sofft_plan* plan, const void* f, int32_t f_per_energy, const double* E_host,
                                    int32_t nE, double field, void* x_out, double rtol, int32_t maxit,
                                    sofft_solve_stats* stats, void* stream);

/* sofft_sse_apply with the banded preconditioner (op 1: w = P^-1 v of
 * Eq. PreconFFT_ECS; op 0 as sofft_sse_apply).  Asynchronous. */
sofft_status sofft_sse_apply_banded(sofft_plan* plan, int32_t op, const void* v, void* w, double E, double field,
                                    void* stream);

/* The banded ECS eigen-preconditioner of Sec. III (Eqs. Prec_eigen_eq, K_l,
 * PreconFFT_ECS) for one axis of a problem, computed on the host (no device
 * work; the stationary solver builds the same tables itself).  The spectrum,
 * in FFT index order, is cut into bands: {k_0} and {k_N/2} alone, the positive
 * momenta from k_1 outward in bands of 10 with the remainder joined to the band
 * next to k_N/2 (at most 19), the negative momenta mirrored.  On each band
 * [K_l]_{nm} = 1/2 k_n k_m Q(m - n), Q(d) = (1/N) sum_j q_j^-2 exp(2 pi i d x_j / L),
 * is diagonalised by a complex orthogonal X (X^T X = 1).
 *   lambda_out   host, 2 n doubles: eigenvalue of the row n of X (re, im)
 *   x_rows_out   host, 2 n 19 doubles: row n of X restricted to its band,
 *                x_rows[n][i] = X[n][band_start[n] + i], i < band_width[n], zero-padded
 *   band_start, band_width  host, n int32 each
 * n = prob->n[axis], even and >= 4.  SOFFT_EINVAL for a bad problem;
 * SOFFT_EUNSUPPORTED if a band's eigen-decomposition fails. */
sofft_status sofft_band_tables(const sofft_problem* prob, int32_t axis, double* lambda_out, double* x_rows_out,
                               int32_t* band_start, int32_t* band_width);

/* Choose a divisor shift per energy for sofft_sse_solve_shifted by short
 * solves of the problem itself: all nE * ncand (energy, candidate) systems
 * run as one batched COCG limited to probe_iters iterations.  A candidate
 * that reaches rtol ranks by its iterations, the others after it by the
 * residual they reached, breakdowns last; ties keep the earlier candidate.
 *   f               device, [n_y][n_x], one right-hand side for all energies
 *   E_host          host, nE energies (finite)
 *   eta_candidates  host, ncand shifts, finite and >= 0
 *   scratch_x       device, nE * ncand * n_x * n_y complex128, overwritten
 *   eta_out         host, nE entries, written with the chosen candidates
 * The bound workspace must hold nE * ncand energies.  Blocking.  SOFFT_OK unless an argument is bad
 * (SOFFT_EINVAL) or a launch or allocation fails. */
sofft_status sofft_sse_tune_shift(sofft_plan* plan, const void* f, const double* E_host, int32_t nE, double field,
                                  const double* eta_candidates, int32_t ncand, int32_t probe_iters, double rtol,
                                  void* scratch_x, double* eta_out, void* stream);

/* ------------------------------------------------------------------ batches
 * Many independent 2D propagations of uneven size advanced together (the
 * step of Sec. II, as in sofft_propagate, applied to every run).  Runs with an
 * identical problem statement share one set of tables and are processed by
 * the same launches: one pass covers the lines of all of them.  Launch shapes
 * (threads per block; one block per tile of lines or a persistent grid of the
 * resident blocks) are chosen per shape on the first propagation by timing
 * the candidates on scratch states the batch allocates and frees.  Steady
 * steps are replayed from a captured HIP graph (one branch per shape). */
typedef struct sofft_batch sofft_batch;

/* nrun problems (host array), all 2D and of one dtype; each must be valid for
 * sofft_plan_create.  The batch owns the tables of its distinct shapes, two
 * small device pointer tables and a step counter per shape (allocated here),
 * one stream and event per shape. */
sofft_status sofft_batch_create(const sofft_problem* probs, int32_t nrun, sofft_batch** out);

/* Bytes of device workspace a batch needs: the potential-phase table of each
 * distinct shape, per-run norm partial sums, and scratch states of the size
 * of the largest shape's runs, on which the launch shapes are timed.  Host
 * only. */
sofft_status sofft_batch_workspace_size(const sofft_batch* b, int64_t* bytes);

/* Bind a caller-owned device workspace to a batch (256-byte aligned; NULL
 * unbinds), with the conditions of sofft_plan_bind.  sofft_batch_propagate
 * returns SOFFT_EWORKSPACE when less than sofft_batch_workspace_size is bound. */
sofft_status sofft_batch_bind(sofft_batch* b, void* workspace, int64_t bytes);

/* Free the batch (after the work using it has finished). */
sofft_status sofft_batch_destroy(sofft_batch* b);

/* Advance every run by nsteps steps of length dt.
 *   psi      host array of nrun device pointers; run r holds n_x n_y elements
 *            of its problem (layout and element type as in sofft_propagate)
 *   f_mid    device, [nrun][nsteps] doubles: f of run r at the midpoint of
 *            step s is f_mid[r * nsteps + s]; NULL when no run has a field
 *   norm2    host, nrun doubles: ||psi_r||^2 after the steps, accumulated in
 *            FP64 (NULL: not computed; when given the call blocks)
 * The call waits for the stream once, to upload the pointer tables; the steps
 * are otherwise asynchronous.  The first call with nsteps > 0 times the launch
 * shapes (a few passes per shape on scratch memory of the size of that
 * shape's runs).  Calls on one batch must not overlap. */
sofft_status sofft_batch_propagate(sofft_batch* b, void* const* psi, double dt, int64_t nsteps,
                                   const double* f_mid, double* norm2, void* stream);

/* Steady steps per captured graph replay (default 32; 0 = plain launches). */
sofft_status sofft_batch_set_graph_steps(sofft_batch* b, int32_t steps);

/* Launch shape of the row (pass 0) or column (pass 1) launches of the shape
 * that run belongs to: threads per block (256, 512 or 1024; the kernels clamp
 * it to what a line needs and the LDS holds) and grid (0 = one block per tile
 * of lines, else at most that many blocks loop over the tiles).  Setting a
 * shape marks it as tuned (no timing); reading returns zeros before tuning. */
sofft_status sofft_batch_set_launch_shape(sofft_batch* b, int32_t run, int32_t pass, int32_t threads,
                                          int32_t grid);
sofft_status sofft_batch_launch_shape(const sofft_batch* b, int32_t run, int32_t pass, int32_t* threads,
                                      int32_t* grid);

/* ------------------------------------------------------------------ learned correction
 * An addition to the method (not from the paper): a small network N corrects
 * the FFT preconditioner of Eq. PreconFFT,
 *     z = P^-1 r + s N(r/s, P^-1 r/s),   s = sqrt(mean |r|^2),
 * N = three periodic 3x3 convolutions with 4 -> 16 -> 16 -> 2 channels and a
 * ReLU after the first two.  Its inputs are Re and Im of r/s and of
 * P^-1 r/s; its outputs are Re and Im of the correction.  Activations are
 * FP16; the forward convolutions run on the matrix cores with FP32
 * accumulation; weights are kept as FP32 master values and used as FP16.
 * Parameters (sofft_lp_param_count() floats, host order): W1[9][16][4], b1[16],
 * W2[9][16][16], b2[16], W3[9][2][16], b3[2], with tap t = 3 (dy + 1) + dx + 1
 * reading the input at (y + dy, x + dx), periodic.  Grid widths must be
 * multiples of 16. */
typedef struct sofft_lp sofft_lp;

/* A network with zero weights (a zero correction).  It owns its parameters,
 * their gradient and the Adam moments (sofft_lp_param_count() floats each,
 * allocated here); activations and every other per-call buffer live in a
 * workspace the caller binds (sofft_lp_workspace_size, sofft_lp_bind). */
sofft_status sofft_lp_create(sofft_lp** out);

/* Bytes of workspace for calls on `batch` items of ny x nx pixels (forward,
 * loss, backward, the solver's correction with batch = nE) that may train on
 * npairs pairs (sofft_lp_train; 0 otherwise).  Host only. */
sofft_status sofft_lp_workspace_size(int64_t ny, int64_t nx, int32_t batch, int64_t npairs, int64_t* bytes);

/* Bind a caller-owned device workspace (256-byte aligned; NULL unbinds); the
 * conditions of sofft_plan_bind apply.  Calls needing more than is bound
 * return SOFFT_EWORKSPACE. */
sofft_status sofft_lp_bind(sofft_lp* lp, void* workspace, int64_t bytes);
sofft_status sofft_lp_destroy(sofft_lp* lp);
int32_t sofft_lp_param_count(void);

/* Copy the parameters from / to host memory (FP32, layout above).  Setting
 * them also clears the Adam moments. */
sofft_status sofft_lp_set_weights(sofft_lp* lp, const float* host);
sofft_status sofft_lp_get_weights(const sofft_lp* lp, float* host);

/* Forward pass on batch items b < batch: r and pz (= P^-1 r) device complex128
 * [batch][ny][nx]; out device FP32 [batch][ny][nx][2] (N's output, before the
 * scaling by s).  Asynchronous. */
sofft_status sofft_lp_forward(sofft_lp* lp, const void* r, const void* pz, int64_t ny, int64_t nx, int32_t batch,
                              float* out, void* stream);

/* Loss and gradient of one batch: loss = mean over items, pixels and the two
 * channels of (N - (e - pz)/s)^2; grad device FP32 [param_count], loss host.
 * Blocking. */
sofft_status sofft_lp_loss_grad(sofft_lp* lp, const void* r, const void* pz, const void* e, int64_t ny,
                                int64_t nx, int32_t batch, float* grad, double* loss, void* stream);

/* Gradients of the network for gradient checks: a forward pass on (r, pz)
 * as in sofft_lp_forward, then for the given dL/dN (dout, device FP32
 * [batch][ny][nx][2]) the input gradient din (device FP32 [batch][ny][nx][4],
 * with respect to the four packed input channels Re r/s, Im r/s, Re pz/s,
 * Im pz/s) and the parameter gradient dw (device FP32 [param_count], layout as
 * above).  Asynchronous. */
sofft_status sofft_lp_backward(sofft_lp* lp, const void* r, const void* pz, const float* dout, int64_t ny,
                               int64_t nx, int32_t batch, float* din, float* dw, void* stream);

/* Train on npairs (residual r_k, error e_k = x* - x_k) pairs of the plan's
 * grid, pair k at energy E_host[k] (P^-1 r is formed at that energy):
 * `epochs` passes over shuffled batches of `batch` pairs (order drawn from
 * `seed`), Adam with learning rate lr.  r, e: device complex128
 * [npairs][ny][nx].  loss_host: epochs entries (mean batch loss), may be NULL.
 * Blocking. */
sofft_status sofft_lp_train(sofft_lp* lp, sofft_plan* plan, const void* r, const void* e, const double* E_host,
                            int64_t npairs, int32_t epochs, int32_t batch, double lr, uint64_t seed,
                            double* loss_host, void* stream);

/* sofft_sse_solve with the corrected preconditioner in flexible COCG
 * (beta = r_{k+1}^T (z_{k+1} - z_k) / rho_k).  An energy whose recurrence
 * residual has not reached a new minimum for `patience` iterations continues
 * with the plain preconditioner from its true residual (stats.fell_back = 1).
 * 2D plans only (SOFFT_EUNSUPPORTED on a 3D plan). */
sofft_status sofft_sse_solve_learned(sofft_plan* plan, sofft_lp* lp, const void* f, int32_t f_per_energy,
                                     const double* E_host, int32_t nE, double field, void* x_out, double rtol,
                                     int32_t maxit, int32_t patience, sofft_solve_stats* stats, void* stream);

/* Kernels whose launches can be timed (see sofft_timing_*). */
typedef enum {
  SOFFT_KERNEL_ROW = 0,   /* 2D row pass (x lines) of the propagation */
  SOFFT_KERNEL_COL = 1,   /* 2D column pass (y lines) of the propagation */
  SOFFT_KERNEL_1D = 2,    /* 1D whole-propagation kernel */
  /* stationary solver; on 3D plans each kind times its group of line passes */
  SOFFT_KERNEL_SSE_ROW_MV = 3,    /* p update + row part of A p (3D: x and y parts) */
  SOFFT_KERNEL_SSE_COL_MV = 4,    /* column part of A p and p^T A p (3D: z part) */
  SOFFT_KERNEL_SSE_ROW_UPD = 5,   /* x, r update, ||r||^2, forward row FFT of r */
  SOFFT_KERNEL_SSE_COL_PREC = 6,  /* column FFT, divide by k^2/2 - E, inverse (3D: y, z, y) */
  SOFFT_KERNEL_SSE_ROW_PREC = 7,  /* inverse row FFT to z and r^T z */
  SOFFT_KERNEL_3D_KINETIC = 8,    /* 3D kinetic pass along one axis (with the potential factors) */
  SOFFT_KERNEL_3D_STRIP = 9,      /* 3D Crank-Nicolson on the ECS strip of one axis */
  SOFFT_KERNEL_SSE_1D = 10,       /* 1D stationary solve or application (one workgroup per energy) */
  SOFFT_KERNEL_COUNT_ = 16
} sofft_kernel;

/* Measurement aid: while enabled, every launch of the plan's kernels is
 * bracketed by a pair of HIP events on the launch stream.  Enabling clears the
 * accumulated record.  Not for production use: event pairs add a small gap
 * between launches. */
sofft_status sofft_timing_enable(sofft_plan* plan, int32_t enable);

/* Sum of the event-measured durations (milliseconds) and number of launches
 * of one kernel kind since timing was enabled.  Blocks until the recorded
 * events have completed. */
sofft_status sofft_timing_read(sofft_plan* plan, int32_t kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* SOFFT_H_ */
