/*
 * rh.h -- C ABI of the MI355X (gfx950) relativistic-hydrodynamics hot path.
 *
 * The library advances the 3+1D ideal relativistic hydrodynamics equations in
 * conservation form (Sikorski et al., arXiv:1604.03360, Sec. 1, Eq. (1)) for the
 * conserved densities u = (E, Mx, My, Mz, N) on a Cartesian grid.  Each right-
 * hand-side evaluation is the semi-discrete operator L(u) of Eq. (2), with the
 * half-cell fluxes given by finite-difference WENO5 or WENO7 reconstruction
 * (Sec. 1.2) of Lax-Friedrichs-split physical fluxes, or by the MUSTA-FORCE
 * scheme with MUSCL reconstruction (Sec. 1.1); the ODE is integrated with the
 * third-order strong-stability-preserving Runge-Kutta method (Sec. 1).  The
 * equation of state is conformal, p = e/3, with N a passive conserved charge
 * (the paper's test fluids), or an ideal gas.
 *
 * Conventions shared by every call:
 *   - Fields are structure-of-arrays, [5][nz][ny][nx] with x fastest, in the
 *     order E, Mx, My, Mz, N (conserved) or e, vx, vy, vz, n (primitive).
 *   - Device pointers are HIP device addresses on the current device; the
 *     caller owns every buffer passed in (the library never frees them).
 *   - All work is enqueued asynchronously on the stream given to rh_bind
 *     (a hipStream_t passed as void*; NULL means the legacy default stream).
 *     Only rh_totals, rh_kernel_times, rh_plan_destroy and the batch calls
 *     that return host data synchronise that stream.
 *   - Every call returns RH_OK (0) or a negative rh_status; the message of
 *     the last failure on the calling thread is available from rh_last_error.
 *     No C++ exception crosses this interface.
 */
#ifndef RH_H
#define RH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int rh_status;
#define RH_OK         0
#define RH_E_INVAL   -1  /* invalid argument: bad sizes, widths, scheme, precision, boundary */
#define RH_E_NOMEM   -2  /* a library-owned device allocation failed */
#define RH_E_HIP     -3  /* a HIP runtime call or kernel launch failed (message has details) */
#define RH_E_STATE   -4  /* call out of order, e.g. stepping a plan with no bound buffers */
#define RH_E_NOTSUP  -5  /* valid request that this library does not support */
#define RH_E_PHYS    -6  /* strict mode: a primitive-recovery floor acted or a value is not finite */

/* Arithmetic of a plan.  RH_PREC_FP64: storage, stencil and Runge-Kutta in FP64.
 * RH_PREC_FP32: storage, stencil and Runge-Kutta in FP32, with the primitive
 * recovery (the velocity root solve) and the conservation totals in FP64. */
#define RH_PREC_FP64 0
#define RH_PREC_FP32 1

/* Boundary condition of one axis.  PERIODIC wraps; OUTFLOW copies the edge cell
 * into the ghost cells (zero gradient); HUBBLE fills ghost cells with the
 * analytic Hubble-like flow u^mu = x^mu/tau, tau = sqrt(t^2 - r^2),
 * e = e0 (t0/tau)^4, n = n0 (t0/tau)^3 at the Runge-Kutta stage time (Sec. 3).
 * An axis with one cell contributes nothing to L whatever its condition. */
#define RH_BC_PERIODIC 0
#define RH_BC_OUTFLOW  1
#define RH_BC_HUBBLE   2

/* Field kinds for rh_set_fields / rh_get_fields. */
#define RH_FIELDS_CONSERVED 0  /* E, Mx, My, Mz, N */
#define RH_FIELDS_PRIMITIVE 1  /* e, vx, vy, vz, n */

/* Kernel classes reported by rh_kernel_times. */
#define RH_KERNEL_SWEEP_X 0   /* x-direction WENO sweep */
#define RH_KERNEL_SWEEP_Y 1   /* y-direction WENO sweep */
#define RH_KERNEL_SWEEP_Z 2   /* z-direction WENO sweep */
#define RH_KERNEL_OTHER   3   /* combine, conversion, reduction and ideal-gas recovery kernels */
#define RH_KERNEL_ADJOINT 4   /* adjoint sweeps (all axes) */
#define RH_KERNEL_SWEEP_XY 5  /* fused x and y sweep (WENO5, and WENO7 in FP32; periodic x of
                                 64..256 cells, a multiple of 64): one launch in place of the x
                                 and y sweeps */
#define RH_KERNEL_STAGE 6     /* fused stage: x, y and z of L and the stage combine in one launch */
#define RH_KERNEL_CLASSES 7

/* Evaluation paths of L (rh_set_path, rh_batch_set_path).  RH_PATH_SWEEPS: one
 * directional sweep per axis (x, y, z; the x and y sweeps fused into one launch
 * where rh_kernel_times reports RH_KERNEL_SWEEP_XY) with an L accumulator in the
 * workspace.  RH_PATH_STAGE: one launch per Runge-Kutta stage evaluating all three
 * axes of L and the stage combine (no L accumulator).  For the WENO schemes with
 * global splitting and the conformal fluid both give bitwise the same results;
 * MUSTA-FORCE, local splitting and the ideal gas exist on RH_PATH_STAGE only.
 * RH_PATH_AUTO (the default) takes RH_PATH_SWEEPS for single grids where it
 * applies and RH_PATH_STAGE otherwise and for batches. */
#define RH_PATH_AUTO   0
#define RH_PATH_SWEEPS 1
#define RH_PATH_STAGE  2

/* Schemes (rh_grid_desc.scheme).  5 and 7: finite-difference WENO5 / WENO7
 * (Sec. 1.2) of Lax-Friedrichs-split fluxes.  RH_SCHEME_MUSTA: MUSTA-FORCE
 * (Sec. 1.1): MUSCL reconstruction of the conserved variables with a slope
 * limiter (2 ghost cells), then at every face k stages of the FORCE flux
 * F = (f_L + 2 f(u_M) + f_R)/4 - (u_R - u_L)/(4 lam), u_M = (u_L + u_R)/2 -
 * lam/2 (f_R - f_L), each stage but the last followed by u_L -= lam (F - f_L),
 * u_R -= lam (f_R - F), with lam = musta_cfl the local dt/dx over the light-speed
 * bound.  The paper names the method and its ingredients only; the stage
 * count, local Courant number and limiters offered are this library's
 * reading of it. */
#define RH_SCHEME_MUSTA 2

/* MUSCL slope limiters (MUSTA-FORCE): the slope of cell j from a = u_j - u_{j-1}
 * and b = u_{j+1} - u_j, zero where they differ in sign; NONE is first order. */
#define RH_LIMITER_MINMOD   0  /* the smaller of |a|, |b| */
#define RH_LIMITER_MC       1  /* min(2|a|, 2|b|, |a + b|/2) (monotonised central) */
#define RH_LIMITER_VANLEER  2  /* 2ab/(a + b) */
#define RH_LIMITER_SUPERBEE 3  /* max(min(2|a|, |b|), min(|a|, 2|b|)) */
#define RH_LIMITER_NONE     4  /* no slope */

/* Flux splitting of the WENO schemes.  GLOBAL: f+- = (F +- u)/2, alpha = 1 (the
 * light-speed bound; the paper's reading).  LOCAL: f+- = (F +- alpha u)/2 per
 * face, alpha the largest characteristic speed |lambda| over the face's 2r
 * stencil cells, from the acoustic eigenvalues of the flux Jacobian. */
#define RH_SPLIT_GLOBAL 0
#define RH_SPLIT_LOCAL  1

/* Equations of state.  CONFORMAL: p = e/3 (closed-form primitive recovery).
 * IDEAL: ideal gas with unit rest mass per unit charge, p = (gamma - 1)(e - n),
 * never below 0, c_s^2 = gamma p / (e + p); primitive recovery by a bracketed
 * FP64 Newton iteration for the speed, once per cell and evaluation of L (a
 * pass before the WENO stage).  HUBBLE boundaries need CONFORMAL. */
#define RH_EOS_CONFORMAL 0
#define RH_EOS_IDEAL     1

typedef struct rh_grid_desc {
    int nx, ny, nz;          /* cells per axis, each >= 1 */
    double dx, dy, dz;       /* cell widths, > 0 */
    double x0, y0, z0;       /* position of the centre of cell (0,0,0) (used by HUBBLE) */
    int scheme;              /* 5 (WENO5, 3 ghost cells), 7 (WENO7, 4 ghost cells) or RH_SCHEME_MUSTA */
    int precision;           /* RH_PREC_FP64 or RH_PREC_FP32 */
    int bc[3];               /* RH_BC_* for the x, y and z axes */
    double weno_eps;         /* epsilon of the nonlinear weights; 0 selects 1e-6 */
    double hubble_t0;        /* HUBBLE only: reference time t0 */
    double hubble_e0;        /* HUBBLE only: e at tau = t0 */
    double hubble_n0;        /* HUBBLE only: n at tau = t0 */
    int strict;              /* nonzero: rh_totals reports RH_E_PHYS when a floor acted */
    int limiter;             /* RH_SCHEME_MUSTA: RH_LIMITER_* (0 = minmod) */
    int musta_stages;        /* RH_SCHEME_MUSTA: FORCE evaluations per face, 1 .. 8; 0 selects 2 */
    double musta_cfl;        /* RH_SCHEME_MUSTA: local dt/dx of the stages, (0, 1]; 0 selects 0.9 */
    int flux_split;          /* WENO: RH_SPLIT_GLOBAL (0) or RH_SPLIT_LOCAL */
    int eos;                 /* RH_EOS_CONFORMAL (0) or RH_EOS_IDEAL */
    double eos_gamma;        /* RH_EOS_IDEAL: adiabatic index in (1, 2]; 0 selects 5/3 */
} rh_grid_desc;

typedef struct rh_plan rh_plan;

/* Message of the last failing call on this thread ("" if none).  Owned by the
 * library; valid until the next call on the same thread. */
const char* rh_last_error(void);

/* Library version string (static storage). */
const char* rh_version(void);

/* Create a plan for one grid (Eq. (2) on a Cartesian grid).  Validates the
 * description (axes of 1 .. 2^24 cells, one field below 4 GiB, the scheme and
 * its parameters) and allocates only small plan-owned device memory (counters
 * and reduction partials).  *out receives the plan; it is NULL on failure.
 * Floors (rh_totals counters[0]) are counted per cell and evaluation of L for
 * WENO, and per recovery of a face state (three per MUSTA stage, each face of
 * the grid once) for MUSTA-FORCE.
 * Errors: RH_E_INVAL (bad description), RH_E_NOTSUP (HUBBLE boundaries with the
 * ideal gas), RH_E_NOMEM, RH_E_HIP. */
rh_status rh_plan_create(rh_plan** out, const rh_grid_desc* desc);

/* Release a plan and its own device memory (after waiting for the plan's work
 * on its bound stream); never touches caller buffers.  NULL is ignored. */
void rh_plan_destroy(rh_plan* plan);

/* Bytes of one state: 5 * nx * ny * nz * (8 for FP64, 4 for FP32). */
size_t rh_state_bytes(const rh_plan* plan);

/* Bytes of the workspace the caller must provide to rh_bind: the two
 * intermediate Runge-Kutta stage states and the L accumulator (3 states).  The
 * adjoint calls use it as scratch (a six-field recovery pack); the ideal gas's
 * WENO stage keeps each cell's recovered (vx, vy, vz, p, c_s^2) in the slot of
 * the accumulator, which the fused stage does not otherwise use. */
size_t rh_workspace_bytes(const rh_plan* plan);

/* Bind caller-owned device buffers and a stream.  state: rh_state_bytes bytes,
 * the solution u^n, updated in place by rh_step.  workspace: rh_workspace_bytes
 * bytes, contents scratch.  Both must be 16-byte aligned and stay valid while
 * work of this plan is pending on the stream.  Rebinding is allowed at any
 * time between calls.  Errors: RH_E_INVAL (NULL or misaligned buffer). */
rh_status rh_bind(rh_plan* plan, void* state, void* workspace, void* stream);

/* Write the bound state from FP64 device fields src[5][nz][ny][nx] of the given
 * kind.  PRIMITIVE input is converted to conserved variables in FP64
 * (E = (e+p) g^2 - p, M = (e+p) g^2 v, N = n g, g = 1/sqrt(1-v^2), p from the
 * plan's equation of state) and then rounded to the plan precision.  Asynchronous.
 * Errors: RH_E_STATE (unbound), RH_E_INVAL (kind). */
rh_status rh_set_fields(rh_plan* plan, const double* src, int kind);

/* Read the bound state into FP64 device fields dst[5][nz][ny][nx].  PRIMITIVE
 * output runs the plan's FP64 primitive recovery (closed form for p = e/3,
 * Newton for the ideal gas; the same recovery as the kernels).  Asynchronous.
 * Errors: RH_E_STATE, RH_E_INVAL. */
rh_status rh_get_fields(rh_plan* plan, double* dst, int kind);

/* Evaluate L(u) of Eq. (2) for the bound state at physical time t (t matters
 * only for HUBBLE boundaries) into the caller's device buffer L_out, which has
 * the plan precision and layout [5][nz][ny][nx] and must not alias the bound
 * buffers.  Directions are accumulated in the order x, y, z.  Asynchronous.
 * Errors: RH_E_STATE (unbound), RH_E_INVAL (NULL or aliasing L_out). */
rh_status rh_apply_L(rh_plan* plan, double t, void* L_out);

/* Advance the bound state by n_steps steps of the Shu-Osher SSP-RK3 method
 * (Sec. 1): u1 = u + dt L(u, t); u2 = 3/4 u + 1/4 (u1 + dt L(u1, t+dt));
 * u <- 1/3 u + 2/3 (u2 + dt L(u2, t+dt/2)), the last stage evaluated as
 * u + c (v - u) with v = u2 + dt L(u2) and c = 2/3 in the plan precision.  The
 * combine of each stage is fused into its last directional sweep (or into the
 * stage kernel).  *t_inout is the physical time of the
 * state (used for HUBBLE boundaries) and is advanced by n_steps*dt on return
 * (host-side; the device work is asynchronous).  n_steps == 0 is a no-op.
 * Errors: RH_E_INVAL (dt <= 0, n_steps < 0, NULL t_inout), RH_E_STATE, RH_E_HIP. */
rh_status rh_step(rh_plan* plan, double dt, int n_steps, double* t_inout);

/* Conservation diagnostics of the bound state: out[0..4] = FP64 sums of E, Mx,
 * My, Mz and N over all cells (deterministic fixed-order two-pass reduction,
 * not multiplied by the cell volume).  counters (may be NULL) receives
 * [0] = primitive recoveries that hit a floor (E below 1e-12, or |M| at or
 * above the velocity cap) since the plan was created or last reset, counted
 * once per cell and evaluation of L (so one SSP-RK3 step counts a floored
 * cell of each of its three stage inputs once) and once per cell read back by
 * rh_get_fields(PRIMITIVE); grids with no axis longer than one cell evaluate
 * no recovery and count nothing; [1] = cells of the bound state with a
 * non-finite conserved value.  Synchronises the stream.
 * Errors: RH_E_STATE, RH_E_HIP, RH_E_PHYS (strict plans only). */
rh_status rh_totals(rh_plan* plan, double out[5], long long counters[2]);

/* The integrals of E, Mx, My, Mz and N over the grid (the conserved charges of
 * Eq. (1)): the sums of rh_totals times the cell volume dx dy dz.  counters,
 * synchronisation and errors as rh_totals (on RH_E_PHYS out is still filled). */
rh_status rh_totals_integrated(rh_plan* plan, double out[5], long long counters[2]);

/* Replay steps from graphs (enable != 0): rh_step then captures one SSP-RK3
 * step (its sweep launches, Sec. 1) into a hipGraph on first use, and four
 * steps into another once a call asks for at least four; a call replays the
 * four-step graph while four or more steps remain and the one-step graph for
 * the rest (one graph launch per four steps saves the idle time between
 * launches).  The graphs are rebuilt when dt or the bound buffers change.
 * Results are bitwise those of eager launches.  Plans with an analytic
 * boundary, and steps taken while per-launch timing is on, run eagerly.
 * Errors: RH_E_INVAL (NULL plan). */
rh_status rh_set_graph(rh_plan* plan, int enable);

/* Select the evaluation path (RH_PATH_*) of every later call that evaluates L
 * (rh_apply_L, rh_step, rh_step_store and the stage recomputation of
 * rh_step_vjp).  Drops a captured step graph.
 * Errors: RH_E_INVAL (unknown path), RH_E_NOTSUP (RH_PATH_SWEEPS for MUSTA-FORCE,
 * local splitting or the ideal gas). */
rh_status rh_set_path(rh_plan* plan, int path);

/* The path the plan's evaluations take now (RH_PATH_SWEEPS or RH_PATH_STAGE). */
rh_status rh_get_path(const rh_plan* plan, int* path);

/* Launch shape of the fused stage: tile_x (16, or 32 for WENO5) cells along x by 256/tile_x
 * along y per block (MUSTA-FORCE: 16 x 15), and the z segment each block rolls
 * along (seg_z >= 1; 0 selects a default for the grid, clamped to nz).  Drops a
 * captured step graph.  rh_get_stage_tuning reports the shape in use (the
 * segment resolved).  Errors: RH_E_INVAL, RH_E_NOTSUP (tile_x 32 for WENO7 or
 * MUSTA-FORCE). */
rh_status rh_set_stage_tuning(rh_plan* plan, int tile_x, int seg_z);
rh_status rh_get_stage_tuning(const rh_plan* plan, int* tile_x, int* seg_z);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): the totals of
 * rh_totals for a state given directly, with no plan and no host transfer.
 * state: device buffer [5][ncell] of the given precision (RH_PREC_*), ncell
 * cells, 1 <= ncell with one field of at most RH_NOALLOC_MAX_BYTES bytes.
 * out_dev: caller-owned device buffer of 6 doubles, receiving the FP64 sums
 * of E, Mx, My, Mz and N (the deterministic two-pass reduction of rh_totals,
 * so the same bits rh_totals returns for the same state) and, in out_dev[5],
 * the number of cells with a non-finite value.  Enqueued on stream (a
 * hipStream_t as void*, NULL = legacy default stream) of the current device;
 * nothing is allocated: the reduction partials live in a library-owned static
 * device array of 6 x 512 doubles (24 KiB) per GPU, whose address is looked up
 * on the first call on each device.  Every call on one GPU shares that array,
 * so calls that can overlap on one GPU (different streams, or threads without
 * ordering) race; calls on one stream are ordered and safe.
 * Errors: RH_E_INVAL (NULL pointer, unknown precision, ncell out of range),
 * RH_E_NOTSUP (device index above 63), RH_E_HIP. */
#define RH_NOALLOC_MAX_BYTES 4294967295LL
rh_status rh_totals_noalloc(const void* state, int precision, long long ncell, double* out_dev,
                            void* stream);

/* Reset the floor counter reported by rh_totals to zero (asynchronous). */
rh_status rh_reset_counters(rh_plan* plan);

/* Enable (nonzero) or disable per-kernel timing with HIP events recorded on
 * the bound stream around every launch.  Enabling clears earlier records. */
rh_status rh_set_timing(rh_plan* plan, int enable);

/* Per kernel class (RH_KERNEL_*): total milliseconds and number of launches
 * recorded since timing was enabled.  ms_out and launches_out hold n entries
 * (n <= RH_KERNEL_CLASSES).  Synchronises the stream. */
rh_status rh_kernel_times(rh_plan* plan, double* ms_out, long long* launches_out, int n);

/* ------------------------------------------------------------------------
 * Adjoint (reverse-mode derivative) of L and of one SSP-RK3 step.  The paper
 * integrates du/dt = L(u) (Sec. 1, Eq. (2)); these calls give the transposed
 * Jacobians needed to differentiate a run with respect to its initial state.
 * The derivative is that of the discrete scheme actually computed, including
 * the WENO nonlinear weights (Sec. 1.2) and the primitive-recovery floors.
 * They cover the WENO schemes with the conformal fluid and global splitting
 * (RH_E_NOTSUP otherwise).
 * ------------------------------------------------------------------------ */

/* out = J(u)^T w, J = dL/du of Eq. (2) at state u and time t.  u, w and out are
 * device buffers of the plan precision and layout [5][nz][ny][nx]; out must
 * not alias u or w, and none of them may alias the bound workspace, whose
 * contents this call overwrites (it holds the per-cell recovery pack).
 * Asynchronous on the bound stream.  Errors: RH_E_STATE (unbound),
 * RH_E_INVAL (NULL or aliasing). */
rh_status rh_apply_vjp(rh_plan* plan, double t, const void* u, const void* w, void* out);

/* Bytes of the scratch buffer rh_step_vjp needs (three states). */
size_t rh_vjp_workspace_bytes(const rh_plan* plan);

/* Adjoint of one SSP-RK3 step taken from u_n at time t with step dt:
 * ubar_out = (d u_{n+1} / d u_n)^T ubar_in.  The stage states u1, u2 are
 * recomputed into scratch (rh_vjp_workspace_bytes), then
 *   b2 = 2/3 b + 2/3 dt J(u2)^T b,  b1 = 1/4 b2 + 1/4 dt J(u1)^T b2,
 *   ubar_out = 1/3 b + 3/4 b2 + b1 + dt J(u_n)^T b1   (b = ubar_in),
 * with J(u2) at t + dt/2, J(u1) at t + dt, J(u_n) at t; the weights 2/3 and
 * 1/3 are c and 1 - c of the forward's last stage.  The plan must be bound;
 * its workspace is overwritten (recomputation and recovery pack) and may
 * not alias any operand.  ubar_out may alias ubar_in.  Errors: RH_E_STATE
 * (unbound), RH_E_INVAL. */
rh_status rh_step_vjp(rh_plan* plan, double t, double dt, const void* u_n, const void* ubar_in,
                      void* ubar_out, void* scratch);

/* One SSP-RK3 step of the bound state, exactly as rh_step with n_steps = 1,
 * that also leaves its two intermediate stage states u1 (after stage 1) and
 * u2 (after stage 2) in stages, a caller-owned device buffer of two states
 * [2][5][nz][ny][nx], for a later rh_step_vjp_stored.  *t_inout advances by dt.
 * Errors: RH_E_STATE (unbound), RH_E_INVAL (NULL, dt <= 0, aliasing). */
rh_status rh_step_store(rh_plan* plan, double dt, double* t_inout, void* stages);

/* n_steps SSP-RK3 steps of the bound state (bitwise as rh_step with the same
 * n_steps) that keep, for every step k, the state it started from and its two
 * stage states: store is a caller-owned device buffer of 3 * n_steps states,
 * [n_steps][3][5][nz][ny][nx] = (u_k, u1_k, u2_k), so that step k's adjoint is
 * rh_step_vjp_stored(plan, t_k, dt, store_k, store_k + one state, ...) with t_k
 * the time of step k as rh_step takes it (*t_inout on entry with dt added k
 * times).  *t_inout advances by n_steps * dt, as in rh_step; n_steps == 0 is a
 * no-op (store may then be NULL).  Asynchronous on the bound stream (the steps run eagerly, not from the
 * step graph; a failed call leaves the steps before it done and *t_inout
 * unchanged).  Errors: RH_E_STATE (unbound), RH_E_INVAL (NULL, dt <= 0,
 * n_steps < 0, store aliasing the bound state or workspace). */
rh_status rh_step_store_n(rh_plan* plan, double dt, int n_steps, double* t_inout, void* store);

/* The adjoint of rh_step_vjp with the stage states supplied instead of
 * recomputed: stages holds u1, u2 of the step taken from u_n at time t (as
 * written by rh_step_store), scratch is two states.  Same result as
 * rh_step_vjp up to rounding order; the bound workspace is overwritten and may
 * not alias any operand.  Errors: RH_E_STATE (unbound), RH_E_INVAL. */
rh_status rh_step_vjp_stored(rh_plan* plan, double t, double dt, const void* u_n, const void* stages,
                             const void* ubar_in, void* ubar_out, void* scratch);

/* ------------------------------------------------------------------------
 * Event-by-event ensembles (batched grids).  The paper's motivation is
 * event-by-event simulation of many independent collisions (abstract and
 * Sec. 1 introduction); a batch advances many independent grids together with
 * one launch per Runge-Kutta stage covering every grid (RH_PATH_STAGE, the
 * default), or one launch per directional sweep and stage (RH_PATH_SWEEPS).
 * ------------------------------------------------------------------------ */
typedef struct rh_batch rh_batch;

/* Create a batch of n_grids independent grids.  All descriptions must share
 * scheme, precision, equation of state (and gamma), flux splitting and the
 * MUSTA-FORCE parameters (RH_E_INVAL otherwise) and have at least 2 cells on
 * every axis (RH_E_NOTSUP otherwise).  Each grid's state occupies elements [offset_g, offset_g +
 * 5*ncell_g) of one concatenated buffer, in the single-grid layout
 * [5][nz][ny][nx]; offsets are multiples of 64 elements. */
rh_status rh_batch_create(rh_batch** out, int n_grids, const rh_grid_desc* descs);

/* Release a batch (library-owned memory only; NULL is ignored). */
void rh_batch_destroy(rh_batch* batch);

/* offsets[0 .. n_grids]: element offset of every grid's state in the
 * concatenated buffer; offsets[n_grids] is the total element count. */
rh_status rh_batch_offsets(const rh_batch* batch, long long* offsets);

/* Bytes of the concatenated state, and of the workspace (3 such buffers). */
size_t rh_batch_state_bytes(const rh_batch* batch);
size_t rh_batch_workspace_bytes(const rh_batch* batch);

/* Bind caller-owned device buffers (16-byte aligned) and a stream, as rh_bind. */
rh_status rh_batch_bind(rh_batch* batch, void* state, void* workspace, void* stream);

/* As rh_set_fields / rh_get_fields, on FP64 device buffers laid out with the
 * batch offsets (total element count from rh_batch_offsets). */
rh_status rh_batch_set_fields(rh_batch* batch, const double* src, int kind);
rh_status rh_batch_get_fields(rh_batch* batch, double* dst, int kind);

/* Advance every grid n_steps SSP-RK3 steps of size dt (Sec. 1).  On the
 * default path each stage is one launch covering all grids (x, y and z of L
 * and the stage combine); with RH_PATH_SWEEPS it is three (x, y, z sweeps).
 * With graphs enabled the launches of one step are captured once in a
 * hipGraph and replayed.  Errors as rh_step. */
rh_status rh_batch_step(rh_batch* batch, double dt, int n_steps, double* t_inout);

/* Per-grid FP64 totals out[n_grids][5] (E, Mx, My, Mz, N) and counters as
 * rh_totals.  Synchronises the stream. */
rh_status rh_batch_totals(rh_batch* batch, double* out, long long counters[2]);

/* Per-grid integrals out[n_grids][5]: rh_batch_totals times each grid's cell
 * volume dx dy dz.  Errors as rh_batch_totals. */
rh_status rh_batch_totals_integrated(rh_batch* batch, double* out, long long counters[2]);

/* Enable (nonzero) or disable hipGraph capture and replay of whole steps.
 * Ignored (no graph) when any grid has a HUBBLE boundary, whose ghost values
 * depend on the stage time. */
rh_status rh_batch_set_graph(rh_batch* batch, int enable);

/* Evaluation path of the batch (RH_PATH_*; as rh_set_path).  Drops a captured
 * step graph.  Errors: RH_E_INVAL. */
rh_status rh_batch_set_path(rh_batch* batch, int path);
rh_status rh_batch_get_path(const rh_batch* batch, int* path);

/* Launch shape of the batched directional sweeps (RH_PATH_SWEEPS): x tile width
 * (64, 32 or 16 cells) and the rolling segment lengths along y and z (>= 4). */
rh_status rh_batch_set_tuning(rh_batch* batch, int tile_x, int seg_y, int seg_z);
rh_status rh_batch_get_tuning(const rh_batch* batch, int* tile_x, int* seg_y, int* seg_z);

/* Launch shape of the batched fused stage (RH_PATH_STAGE): x-y tile width (16
 * or 32 cells) and z segment (>= 1, clamped to each grid's nz). */
rh_status rh_batch_set_stage_tuning(rh_batch* batch, int tile_x, int seg_z);
rh_status rh_batch_get_stage_tuning(const rh_batch* batch, int* tile_x, int* seg_z);

/* Time the candidate launch shapes of the batch's path on the bound state
 * (evaluations of L into the workspace; the state is not modified) with HIP
 * events, keep the fastest and report it through rh_batch_get_stage_tuning
 * (fused stage) or rh_batch_get_tuning (sweeps).  reps >= 1 timed launches per
 * candidate.  Synchronises the stream. */
rh_status rh_batch_autotune(rh_batch* batch, int reps);

/* Per-kernel timing of batched launches, as rh_set_timing / rh_kernel_times. */
rh_status rh_batch_set_timing(rh_batch* batch, int enable);
rh_status rh_batch_kernel_times(rh_batch* batch, double* ms_out, long long* launches_out, int n);

#ifdef __cplusplus
}
#endif

#endif /* RH_H */
