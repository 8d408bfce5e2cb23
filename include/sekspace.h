/*
 * sekspace.h — C ABI of the MI355X (gfx950) Spectral Ewald k-space library.
 *
 * Problem (paper section 1, eqs. 1.1-1.3): N point charges q_n at x_n in the
 * periodic cube [0,L)^3.  The library evaluates the Fourier-space
 * (long-range) parts of the Ewald sums, eqs. (1.5)-(1.7):
 *     E   = (2 pi / L^3) sum_{k != 0} e^{-k^2/4xi^2} / k^2 |S(k)|^2,
 *     phi = dE/dq,   F = -dE/dx,
 * approximated by the Spectral Ewald method (section 4, Algorithm 1, Table 2):
 *   1. sort particles into tiles of the M^3 grid,
 *   2. spread truncated Gaussians (eq. 4.5) with P^3 support,
 *   3. forward 3D FFT,
 *   4. scale by e^{-(1-eta) k^2 / 4 xi^2} / k^2 (eq. 4.6) and reduce E,
 *   5. inverse 3D FFT,
 *   6. gather phi (eq. 4.9) and F (eq. 4.12 read as F = -dE/dx).
 * The SPME window (section 6, eqs. 6.1-6.3: cardinal B-splines of order p,
 * influence function B(k) e^{-k^2/4xi^2}/k^2) is the second window behind the
 * same calls.
 *
 * Units: Coulomb constant 1; multiply E, phi, F by e.g. 138.935 kJ mol^-1 nm
 * e^-2 (section 5 remark) or 332.0637 kcal mol^-1 A e^-2 as needed.
 *
 * Conventions shared by every call
 *   - All functions return se_status and never throw or abort.  Arguments are
 *     checked on the host, synchronously, before anything is enqueued; on an
 *     error nothing is enqueued and outputs are untouched.
 *     se_last_error() returns a message for the last failing call on the
 *     calling thread.
 *   - Device pointers are HIP device memory on the plan's device.  Arrays are
 *     contiguous and row-major: x[N][3] (AoS), q[N], phi[N], F[N][3], all of
 *     the plan's dtype (float for SE_FP32, double for SE_FP64).  E is always
 *     one double in device memory.
 *   - The library never frees or retains caller memory beyond a call.
 *   - Work is enqueued asynchronously on the plan's stream; calls return
 *     without synchronising.  Calls on one plan must not overlap in time from
 *     different host threads.
 *   - Positions may lie outside [0,L): they are wrapped periodically
 *     (section 1: the box is periodic).
 *   - The k = 0 mode is always dropped (section 1); a non-neutral charge set
 *     is accepted and no neutralising-background term is added, so that
 *     dE/dq = phi holds for any q.
 *   - NaN or Inf inputs are not detected: the results of that call are then
 *     unspecified, but no index derived from them leaves the grid or the
 *     plan's workspace, and the plan stays usable for the next call.
 */
#ifndef SEKSPACE_H
#define SEKSPACE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SE_OK = 0,
    SE_ERR_ARG = 1,          /* bad scalar argument, null pointer, N > n_max */
    SE_ERR_GRID = 2,         /* M not even, not 2^a 3^b 5^c, out of range, or M < P */
    SE_ERR_ETA = 3,          /* Gaussian shape eta outside (0,1) (section 4) */
    SE_ERR_UNSUPPORTED = 4,  /* window/precision/P combination not built */
    SE_ERR_WORKSPACE = 5,    /* device allocation failed, or a workspace too
                                small or misaligned for the plan           */
    SE_ERR_HIP = 6,          /* HIP runtime error while enqueueing; the
                                plan's workspace is then in an undefined
                                state (a launch may be missing from the
                                sequence): destroy the plan               */
    SE_ERR_STATE = 7         /* se_gather/se_backward before any se_forward,
                                or se_forward on a plan awaiting its
                                caller-owned workspace                     */
} se_status;

typedef enum { SE_WINDOW_GAUSSIAN = 0, SE_WINDOW_BSPLINE = 1 } se_window;
typedef enum { SE_FP32 = 0, SE_FP64 = 1 } se_dtype;

/* se_params.flags */
#define SE_FLAG_ADD_SELF 1u  /* add the self terms of eqs. (1.5)-(1.6):
                                phi += -2 xi q / sqrt(pi), E += -(xi/sqrt(pi)) sum q^2 */
#define SE_FLAG_TIMING 2u    /* record a HIP event pair around every kernel launch
                                (on the plan's stream) for se_plan_stage_times;
                                such a plan must not be captured in a graph      */
#define SE_FLAG_IK_FORCE 4u  /* F of se_gather (and the field of se_eval_targets)
                                by ik differentiation (section 3.1): the field
                                -grad Phi from -i k times the scaled spectrum,
                                three more inverse 3D FFTs in se_forward, then
                                a plain-window gather of each component, instead
                                of the analytic derivative of the window.  For
                                comparison: se_backward keeps the analytic
                                adjoint (the exact gradient of E).  Tiled
                                supports only (SE P <= 16, SPME).            */
#define SE_FLAG_CALLER_WORKSPACE 8u  /* se_plan_create allocates no device
                                memory: the caller attaches a workspace of
                                se_plan_workspace_size bytes with
                                se_plan_set_workspace before the first
                                se_forward (e.g. memory of a framework's
                                caching allocator)                           */

/* Kernel stages of one evaluation (se_plan_stage_times), in launch order
   apart from the fused plane passes at the end. */
enum {
    SE_STAGE_BIN_COUNT = 0,  /* tile of each particle, its rank in the tile  */
    SE_STAGE_BIN_SCAN,       /* tile offsets (exclusive scan of the counts);
                                a launch of its own only above 8192 tiles   */
    SE_STAGE_BIN_SCATTER,    /* write particles in tile order (and, up to
                                8192 tiles, the scan)                        */
    SE_STAGE_SPREAD,         /* step 2 (tile blocks)                          */
    SE_STAGE_FOLD,           /* step 2, tile blocks summed into the grid      */
    SE_STAGE_FFT_X,          /* step 3, real-to-complex along x              */
    SE_STAGE_FFT_Y,          /* step 3, along y                              */
    SE_STAGE_FFT_Z_SCALE,    /* steps 3-5 along z: FFT, scale + energy, IFFT */
    SE_STAGE_IFFT_Y,         /* step 5, along y                              */
    SE_STAGE_IFFT_X,         /* step 5, complex-to-real along x              */
    SE_STAGE_GATHER,         /* step 6 (se_gather or se_backward)            */
    SE_STAGE_FFT_XY,         /* step 3, x and y in one pass per z plane: in
                                place of FFT_X + FFT_Y where an M x (M/2+1)
                                plane fits in LDS (FP32 M <= 192, FP64
                                M <= 128, compiled sizes)                    */
    SE_STAGE_IFFT_YX,        /* step 5, the same in place of IFFT_Y + IFFT_X */
    SE_NUM_STAGES
};

typedef struct {
    int M;          /* grid points per side; even, 2^a 3^b 5^c, 8 <= M <= 512 */
    int P;          /* SE: Gaussian support points per side, even, 4..16
                       (FP64 also 18..24, on an untiled path: atomics into
                       the grid, no binning); SPME: B-spline order p, 3..8.
                       P <= M.                                              */
    double L;       /* box side, > 0                                         */
    double xi;      /* Ewald splitting parameter, > 0                        */
    double c;       /* SE shape constant of eq. (5.2); <= 0 selects 0.95     */
    int window;     /* se_window                                             */
    int dtype;      /* se_dtype: precision of inputs, outputs and arithmetic */
    unsigned flags; /* SE_FLAG_*                                             */
} se_params;

typedef struct se_plan se_plan;

/* Human-readable name of a status code (static storage). */
const char *se_status_string(se_status s);

/* Message for the last failing call on this thread ("" if none). */
const char *se_last_error(void);

/* Host only, no GPU needed.  Gaussian shape parameter of section 4 and
 * eq. (5.2): eta = (2 w xi / m)^2 with w = P h / 2, h = L / M, m = c sqrt(pi P),
 * i.e. eta = P L^2 xi^2 / (c^2 pi M^2).  Validates *prm like se_plan_create
 * (except device checks); for the B-spline window *eta is set to 0. */
se_status se_params_check(const se_params *prm, double *eta);

/* Host only, no GPU needed.  Device bytes a plan for up to n_max particles
 * allocates (grids, spectra, sorted particles, tables). */
se_status se_plan_workspace_size(const se_params *prm, int n_max, size_t *bytes);

/* Create a plan on the current HIP device for up to n_max particles.
 * hip_stream is a hipStream_t (NULL = the default stream).  The plan owns
 * its device workspace (one allocation of se_plan_workspace_size bytes,
 * made here and freed by se_plan_destroy), unless prm->flags holds
 * SE_FLAG_CALLER_WORKSPACE: then nothing is allocated on the device (and,
 * without SE_FLAG_TIMING, no HIP call is made) until se_plan_set_workspace. */
se_status se_plan_create(const se_params *prm, int n_max, void *hip_stream,
                         se_plan **out);

/* Attach a caller-owned workspace to a plan created with
 * SE_FLAG_CALLER_WORKSPACE.  The workspace holds everything an evaluation
 * keeps on the device: the grid (G, then the scaled grid Phi of eq. 4.9 that
 * se_gather and se_backward read), the spread tile blocks, the half
 * spectrum, the sorted particles and the plan's tables.  dev_ptr: device memory on the plan's device, at least
 * se_plan_workspace_size(prm, n_max) bytes, 256-byte aligned; the caller
 * keeps it allocated and does not touch it while the plan's enqueued work
 * may use it, and frees it after se_plan_destroy (or after attaching another
 * workspace and waiting for the plan's stream).  The tables are written and
 * the tile counters cleared by a kernel enqueued on the plan's stream; the
 * stored grid of an earlier forward pass is not carried over
 * (se_gather/se_backward then return SE_ERR_STATE until the next se_forward).
 * SE_ERR_WORKSPACE if bytes is too small or dev_ptr misaligned, SE_ERR_ARG
 * for a NULL argument or a plan that owns its workspace; checked on the host
 * before any HIP call. */
se_status se_plan_set_workspace(se_plan *plan, void *dev_ptr, size_t bytes);

/* Change the stream later calls enqueue on. */
se_status se_plan_set_stream(se_plan *plan, void *hip_stream);

/* Read back the derived eta (0 for the B-spline window). */
se_status se_plan_eta(const se_plan *plan, double *eta);

/* Plans created with SE_FLAG_TIMING: wait for the recorded launches and
 * write to ms[0..n-1] (stage order above) the mean duration in milliseconds
 * of each stage's launches since the previous call (or since plan creation);
 * -1 for a stage not launched in that interval.  Every launch is counted: the
 * plan keeps a ring of event pairs per stage and, once a ring is full, waits
 * for the oldest pair before reusing it.  A timing plan must not be captured
 * into a HIP graph.  SE_ERR_STATE for plans without the flag. */
se_status se_plan_stage_times(se_plan *plan, double *ms, int n);

/* Release the plan and its workspace (synchronises its stream first). */
se_status se_plan_destroy(se_plan *plan);

/* Steps 1-5 of Algorithm 1: sort, spread, FFT, scale, energy, inverse FFT.
 * x: device [N][3], q: device [N] (plan dtype); E_dev: device double, set to
 * the k-space energy (plus the self energy with SE_FLAG_ADD_SELF).
 * 0 <= N <= n_max (N = 0 gives E = 0).  The scaled grid and the sorted
 * particles stay in the plan until the next se_forward on it; x and q are
 * not referenced after the call's work completes. */
se_status se_forward(se_plan *plan, int N, const void *x, const void *q,
                     double *E_dev);

/* Step 6 for the particles of the last se_forward: phi (device [N]) and F
 * (device [N][3]) in the caller's particle order; either may be NULL. */
se_status se_gather(se_plan *plan, void *phi, void *F);

/* se_forward followed by se_gather. */
se_status se_kspace(se_plan *plan, int N, const void *x, const void *q,
                    double *E_dev, void *phi, void *F);

/* se_kspace without a plan and without allocating, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Parameters as for se_plan_create
 * (prm->flags may hold SE_FLAG_ADD_SELF and SE_FLAG_IK_FORCE; SE_FLAG_TIMING
 * and SE_FLAG_CALLER_WORKSPACE are SE_ERR_ARG), arrays and outputs as for
 * se_kspace (device pointers; phi or F may be NULL; N >= 0), enqueued on
 * hip_stream (a hipStream_t, NULL = the default stream) of the current
 * device.  The workspace of the evaluation (se_plan_workspace_size(prm, N)
 * bytes) is carved out of a static array of 64 MiB that the library holds
 * on each device it runs on until the process ends; an evaluation needing
 * more is SE_ERR_WORKSPACE (checked on the host, nothing enqueued).  Every
 * call on a device shares that device's array: the tables and tile
 * counters are rewritten at the start of each call, and calls that overlap
 * in time on one device (other streams, other host threads) race.  The
 * first call on a device resolves the array's address there
 * (hipGetSymbolAddress; make it outside graph capture).  No hipMalloc,
 * hipFree or other allocating call is made. */
se_status se_kspace_noalloc(const se_params *prm, int N, const void *x, const void *q,
                            double *E_dev, void *phi, void *F, void *hip_stream);

/* Adjoint of se_forward for reverse-mode differentiation, reusing the stored
 * scaled grid (no re-spreading, no FFT):
 *     grad_x = gE * dE/dx = -gE * F,   grad_q = gE * dE/dq = gE * phi,
 * with gE read from device memory (one double).  grad_x device [N][3],
 * grad_q device [N]; either may be NULL. */
se_status se_backward(se_plan *plan, const double *gE_dev, void *grad_x,
                      void *grad_q);

/* Evaluation at points that are not sources.  Reserve room for up to nt_max
 * points (allocates; synchronises the plan's stream first).  SE_ERR_ARG if
 * nt_max < 1. */
se_status se_plan_reserve_targets(se_plan *plan, int nt_max);

/* The k-space potential and field of the charges of the last se_forward at
 * nt points xt (device [nt][3], plan dtype, wrapped periodically): a unit
 * test charge at each point gathers phi_t = sum_j Phi_j W(x_j - xt) (eq. 4.9,
 * no self term) and field_t = -grad phi_t (the force of eq. 4.12 per unit
 * charge), with the window and grid of the plan.  phi_t (device [nt]) or
 * field_t (device [nt][3]) may be NULL.  SE_ERR_STATE before the first
 * se_forward; SE_ERR_ARG if nt exceeds the reserved count.  Sources, the
 * stored grid and se_gather/se_backward are not affected. */
se_status se_eval_targets(se_plan *plan, int nt, const void *xt, void *phi_t, void *field_t);

/* ------------------------------------------------------------------------
 * Real-space part of the Ewald sums (section 1, eqs. 1.5-1.7, the erfc
 * terms), truncated at |r| < rc with the nearest periodic image:
 *     phi_m = sum_{n != m} q_n erfc(xi r)/r,
 *     F_m   = q_m sum_{n != m} q_n (2 xi/sqrt(pi) e^{-xi^2 r^2} + erfc(xi r)/r) r_vec/r^2,
 *     E     = 1/2 sum_m q_m phi_m,        r_vec = x_m - x_n.
 * The total Ewald sum is this plus se_forward/se_gather (k-space) plus the
 * self terms (SE_FLAG_ADD_SELF).  Same conventions as above (device arrays
 * x[N][3], q[N], phi[N], F[N][3] of the plan's dtype; E one device double;
 * asynchronous on the plan's stream; arguments checked on the host).
 * ------------------------------------------------------------------------ */
typedef struct se_rs_plan se_rs_plan;

/* A real-space plan on the current device for up to n_max particles in a
 * cube of side L.  Each se_rs_eval builds a cell list for its N: cells of
 * edge >= rc searched one cell to each side, or, where those of edge
 * >= rc/2 hold on average >= 10 particles (>= 5 when the coarse list has
 * fewer than 1024 cells), cells of edge >= rc/2 searched two to each side;
 * at most 64 cells per side (the coarse list alone where L >= 64 rc).
 * Requires
 * 0 < rc <= L/3 (SE_ERR_ARG otherwise), so at most one image of a pair lies
 * within rc.  The plan owns its workspace. */
se_status se_rs_plan_create(double L, double xi, double rc, int dtype, int n_max,
                            void *hip_stream, se_rs_plan **out);

/* Change the stream later calls enqueue on. */
se_status se_rs_plan_set_stream(se_rs_plan *plan, void *hip_stream);

/* E_dev, phi (device [N], may be NULL) and F (device [N][3], may be NULL)
 * of the real-space sum; 0 <= N <= n_max, N = 0 gives E = 0. */
se_status se_rs_eval(se_rs_plan *plan, int N, const void *x, const void *q,
                     double *E_dev, void *phi, void *F);

/* Release the plan (synchronises its stream first). */
se_status se_rs_plan_destroy(se_rs_plan *plan);

/* ------------------------------------------------------------------------
 * Parameters from an error tolerance (host only; no device, no plan).
 *
 * Error estimates for the potential, the energy or the force (kind =
 * SE_EST_POTENTIAL, SE_EST_ENERGY, SE_EST_FORCE), in the units of that
 * quantity with the Coulomb constant 1, for N charges with Q = sum q_n^2 in a
 * cube of side L.  The potential forms estimate the rms error per particle;
 * the force forms (which carry Q, not q_n sqrt(Q)) estimate the root of the
 * summed squared errors, sqrt(sum_n |dF_n|^2): divide by sqrt(N) for the
 * rms per particle.  Sources:
 *   - real-space truncation at rc: Kolafa-Perram, section 2.1 eq. 2.1;
 *   - Fourier truncation at |k| <= 2 pi kinf / L: section 2.1 eq. 2.2;
 *   - SE approximation error A e^{-pi P c^2/2} with A_phi = sqrt(Q xi L)/L,
 *     A_E = Q sqrt(xi L)/L, A_F = 4 pi Q sqrt(xi^3/L): sections 5.1-5.3.
 * The inversions solve an estimate = eps for xi (eq. 2.3) or kinf (eq. 2.4);
 * Lambert W is evaluated by Newton's method on w + ln w = ln z (exact to
 * rounding for every z > 0, no overflow for huge z).
 * All return SE_ERR_ARG for a non-finite or non-positive argument or an
 * unknown kind, and write the output only on success.
 * ------------------------------------------------------------------------ */
typedef enum {
  SE_EST_POTENTIAL = 0,
  SE_EST_ENERGY = 1,
  SE_EST_FORCE = 2
} se_est_kind;

se_status se_est_real_error(int kind, double Q, double L, double xi, double rc, double *err);
se_status se_est_fourier_error(int kind, double Q, double L, double xi, double kinf,
                               double *err);
/* xi at which the real-space estimate equals eps (eq. 2.3).  For the force
 * form SE_ERR_ARG also when eps exceeds the estimate's value at xi = 0
 * (every xi meets such a tolerance). */
se_status se_est_xi(int kind, double eps, double Q, double L, double rc, double *xi);
/* kinf at which the Fourier estimate equals eps (eq. 2.4). */
se_status se_est_kinf(int kind, double eps, double Q, double L, double xi, double *kinf);
/* SE approximation-error estimate at support P >= 1 and shape constant c
 * (c <= 0 selects 0.95). */
se_status se_est_se_error(int kind, double Q, double L, double xi, int P, double c,
                          double *err);
/* Smallest even P >= 2 whose SE estimate is <= eps (P is rounded up to an even
 * number, section 5.3); SE_ERR_ARG if none up to 64. */
se_status se_est_se_support(int kind, double eps, double Q, double L, double xi, double c,
                            int *P);

/* Runtime model, the form of section 7 extended by the terms a GPU launch
 * sequence has (seconds):
 *   t_real   = real_fixed + real_atom N + real_pair N nbar + real_cell ncells
 *              + real_test N ntest q,
 *   t_kspace = k_fixed + k_atom N + k_window N P^3 + k_block nt^3 (T+P-1)^3
 *              + k_grid M^3 + k_fft (M^3/2) ln(M^3/2),
 * with nbar = (4/3) pi rc^3 N / L^3 (section 7.1); for se_rs_eval's cell list
 * (nc cells per side searched w = 3 or 5 wide, as se_rs_plan_create
 * states) ncells = nc^3, ntest = w^3 (L/nc)^3 N / L^3 the
 * pairs it tests per particle and q = ceil(ncells/R) R / ncells the
 * work-group rounds on a 256-CU device with R cells resident at once
 * (FP32: 1024, or 1280 above 1024 cells; FP64: 512); T the tile edge
 * se_plan_create picks for (M, P, dtype) and nt = ceil(M/T) (the tile blocks
 * that spread, fold and gather move).  The paper's CPU model is
 * real_pair = c_real, k_window = c_sp-ga, k_grid = c_solve,
 * k_fft = c_fft-ifft, the rest 0. */
typedef struct {
  double real_fixed, real_atom, real_pair, real_cell, real_test;
  double k_fixed, k_atom, k_window, k_block, k_grid, k_fft;
} se_cost_model;

/* Constants fitted on an MI355X (one GPU, se_kspace with the SE window and
 * se_rs_eval, inputs resident in HBM) for dtype SE_FP32 or SE_FP64. */
se_status se_cost_model_mi355x(int dtype, se_cost_model *model);

/* The model's times for one configuration (SE window, shape constant 0.95
 * for the tile choice); SE_ERR_UNSUPPORTED when no tile edge fits (M, P) in
 * this precision.  t_real or t_kspace may be NULL. */
se_status se_cost_predict(const se_cost_model *model, int dtype, int N, double L, double rc,
                          int M, int P, double *t_real, double *t_kspace);

typedef struct {
  double rc, xi, kinf; /* chosen cutoff, Ewald parameter, Fourier cut        */
  int M, P;            /* grid size and Gaussian support for se_plan_create  */
  double eta;          /* P L^2 xi^2 / (c^2 pi M^2)                          */
  double t_real, t_kspace;                     /* model times (s)            */
  double est_real, est_fourier, est_approx;    /* estimates at the choice    */
} se_choice;

/* Cheapest SE parameters meeting tolerance eps (absolute rms error of the
 * kind) with each of the three error sources held to eps on its own: for
 * each of n_rc cutoffs rc_i = rc_min + i (rc_max - rc_min)/(n_rc - 1)
 * (rc_min alone when n_rc = 1), xi from eq. 2.3, kinf from eq. 2.4, M the
 * smallest size this library accepts (even, 8..512, 2^a 3^b 5^c) with
 * M >= 2 kinf (section 5.3) and eta <= 0.5 (the regime in which the
 * approximation estimate holds: it is derived at M ~ 4 xi L, where
 * eta = P/(16 pi c^2) < 0.36), P the smallest even support >= 4
 * meeting the SE estimate (at most 16); the cutoff of least modelled
 * t_real + t_kspace (se_cost_predict in precision dtype) wins (first on
 * ties).  Cutoffs above L/3 (the real-space plan's limit) or needing M > 512,
 * P > 16 or a tile that does not fit are skipped; SE_ERR_UNSUPPORTED if none
 * is left.  c <= 0 selects 0.95. */
se_status se_choose_params(int kind, double eps, int N, double Q, double L, double rc_min,
                           double rc_max, int n_rc, double c, int dtype,
                           const se_cost_model *model, se_choice *out);

#ifdef __cplusplus
}
#endif

#endif /* SEKSPACE_H */
