/*
 * dcf.h -- C ABI of the differentiable compressible-flow library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the finite-volume right-hand side of the
 * compressible Navier-Stokes equations for cell-averaged conserved variables
 * (paper: Section 2.1, Eqs. (1)-(6)), fills halo cells to impose boundary
 * conditions (Section 3.2), integrates in time with the three-stage TVD
 * Runge-Kutta scheme (Section 2.1, text after Eq. (6)), and differentiates
 * whole trajectories with a hand-written adjoint so that boundary-condition
 * parameters can be optimised end to end (Section 1 and Section 3.2,
 * "Disturbance Wall").  Every step runs in HIP kernels; the host code only
 * validates arguments, carves the workspace and enqueues kernels.
 *
 * Conventions
 *  - Every function returns a dcf_status (0 = DCF_OK, < 0 error) and never
 *    throws or exits.  dcf_last_error() gives a thread-local message for the
 *    last failure.
 *  - Argument errors are detected on the host before anything is enqueued.
 *    Non-physical states met by the kernels (rho <= 0, p <= 0, T <= 0, or a
 *    non-finite value) set a flag that dcf_flags() reports.
 *  - "dev" pointers are device memory owned by the caller (for example torch
 *    tensors); they must stay valid until the work enqueued on `stream`
 *    completes.  "host" pointers are read before the call returns.
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is the
 *    null stream).  No call synchronises except dcf_flags(),
 *    dcf_gradient() (its segment loop reads nothing back, but it returns
 *    only after enqueueing every segment) and dcf_destroy().
 *  - A context is one solve (grid + gas + boundaries).  A context is not
 *    thread-safe; many contexts per process are fine.
 *
 * State layout: an interior-only, dense FP64 array U[nv][nz][ny][nx] with
 * nv = ndim + 2 conserved variables (rho, rho*u[, rho*v[, rho*w]], E),
 * x fastest (Eq. (2)).  Unused axes have n = 1.  Primitive input arrays are
 * P[5][nz][ny][nx] = (rho, u, v, w, p), unused velocities zero.
 */
#ifndef DCF_H
#define DCF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int dcf_status;
#define DCF_OK 0
#define DCF_EINVAL (-1)       /* invalid argument                              */
#define DCF_ENOMEM (-2)       /* workspace too small / host allocation failed   */
#define DCF_EDEVICE (-3)      /* HIP runtime error                              */
#define DCF_ENONPHYS (-4)     /* non-physical state flagged by a kernel         */
#define DCF_EBUDGET (-5)      /* request exceeds a memory budget                */
#define DCF_EUNSUPPORTED (-6) /* valid but unsupported combination              */

/* boundary kinds (Section 3.2: halo cells carry the boundary condition) */
#define DCF_BC_PERIODIC 0
#define DCF_BC_WALL 1      /* no-slip wall, isothermal or adiabatic                    */
#define DCF_BC_POROUS 2    /* wall with a Darcy transpiration strip                   */
#define DCF_BC_ZEROGRAD 3  /* zero-gradient extrapolation                             */
#define DCF_BC_DIRICHLET 4 /* prescribed primitive profile                            */
#define DCF_BC_DISTURB 5   /* wall with normal velocity A sin(2 pi kappa x), Eq. (8)   */

#define DCF_VISC_NONE 0
#define DCF_VISC_POWER 1      /* mu = mu_ref (T/T_ref)^omega                          */
#define DCF_VISC_SUTHERLAND 2 /* mu = mu_ref (T/T_ref)^1.5 (T_ref+S)/(T+S), Sec. 3.2 */

#define DCF_STRETCH_UNIFORM 0
#define DCF_STRETCH_TANH2 1 /* x = lo + L (1 - tanh(beta (1 - 2 s))/tanh beta)/2, s = xi/n */
#define DCF_STRETCH_TANH1 2 /* x = lo + L (1 + tanh(beta (s - 1))/tanh beta)           */

#define DCF_SOURCE_NONE 0
#define DCF_SOURCE_MASSFLUX 1 /* body force S = [0, f, 0, 0, f u], f = -<R_rhou>_V */

#define DCF_FLAG_NONPHYS 1u

typedef struct dcf_ctx dcf_ctx;

/* Grid (Section 2.2: a single-device domain of [Nx, Ny, Nz] interior cells
 * plus Nh = 3 halo layers per active axis; stretched Cartesian meshes,
 * Section 2).  Cell i of an axis spans xi in [i, i+1] of the map above. */
typedef struct {
  int ndim;            /* 1, 2 or 3                                        */
  int n[3];            /* interior cells per axis; 1 on unused axes        */
  double lo[3], hi[3]; /* axis extents                                     */
  int stretch[3];      /* DCF_STRETCH_*                                    */
  double beta[3];      /* tanh stretching parameter                        */
} dcf_grid;

/* Ideal gas and transport (Section 2.1: Fourier heat flux, Stokes stress;
 * Section 3.2: Sutherland law).  lambda = mu * cp / Pr, cp = gamma R/(gamma-1). */
typedef struct {
  double gamma, R, Pr;
  int visc_law;      /* DCF_VISC_*                                       */
  double mu_ref, T_ref;
  double visc_param; /* power-law exponent, or Sutherland constant S      */
} dcf_gas;

/* One face's boundary condition.  Faces: 0..5 = x-, x+, y-, y+, z-, z+. */
typedef struct {
  int kind;                 /* DCF_BC_*                                          */
  double T_wall;            /* wall kinds: temperature > 0, or 0 for adiabatic   */
  const double *dirichlet;  /* dev, DIRICHLET: [5][n_t2][n_t1] (rho,u,v,w,p)     */
  int porous_begin;         /* POROUS: strip [begin, end) along the face's first  */
  int porous_end;           /*   tangential axis, all cells along the second one  */
  double p_inf;             /* POROUS: reference pressure of the Darcy law        */
} dcf_bc;

/* ---- context ------------------------------------------------------------ */
/* Creates a context on the current HIP device, computes the grid metrics
 * with a kernel (the only allocation the library makes: O(nx+ny+nz)
 * doubles) and sets every face to DCF_BC_PERIODIC. */
dcf_status dcf_create(const dcf_grid *grid, const dcf_gas *gas, dcf_ctx **out);
dcf_status dcf_destroy(dcf_ctx *ctx);

/* nv, interior cell count and the byte size of one state array. */
dcf_status dcf_state_info(const dcf_ctx *ctx, int *nv, long *ncell, size_t *state_bytes);

/* Workspace: caller-owned device memory (256-byte aligned) of at least the
 * size reported for the same (mode, nsteps, seg_len).  mode 0 = forward
 * (rhs, rk3_step, dt, diagnostics, cost); mode 1 = adds vjp_step; mode 2 =
 * adds the trajectory gradient over exactly `nsteps` steps with checkpoints
 * every `seg_len` steps (dcf_gradient); mode 3 = as mode 2 and also keeps
 * the primitive box of every stage of a segment from the forward recompute,
 * so the reverse sweep recomputes nothing of the forward (3 seg_len more
 * boxes of memory; bitwise the same gradient).
 * nsteps/seg_len are ignored below mode 2.  The library keeps the pointer
 * until the next call, clears the parts that must start at zero (the call
 * returns once that is done) and owns the contents from then on: the caller
 * must not write into the workspace. */
dcf_status dcf_workspace_size(const dcf_ctx *ctx, int mode, int nsteps, int seg_len,
                              size_t *bytes);
dcf_status dcf_set_workspace(dcf_ctx *ctx, int mode, int nsteps, int seg_len, void *dev,
                             size_t bytes);

/* dcf_workspace_size for a grid and gas without a context: host arithmetic
 * only (no device call, no allocation), for schedulers that size requests
 * before admitting them.  The same validation as dcf_create. */
dcf_status dcf_workspace_size_for(const dcf_grid *grid, const dcf_gas *gas, int mode,
                                  int nsteps, int seg_len, size_t *bytes);

/* Boundary condition of one face (Section 3.2).  Periodic faces must be
 * set in pairs.  Walls mirror the velocity (u_g = -u_mirror, no slip) and
 * the pressure; isothermal walls (T_wall > 0) set T_g = 2 T_wall - T_mirror
 * and rho_g = p_g/(R T_g), adiabatic walls (T_wall = 0) mirror T and rho.
 * Porous: the wall-normal velocity along the inward normal is
 * v_w = -K_i (p_w - p_inf)/p_inf, p_w the pressure of the first interior
 * cell, and the ghost normal velocity is 2 v_w - u_mirror.  Disturbance
 * wall (Section 3.2, Eq. (8)): v_w = A sin(2 pi kappa x_c), x_c the centre
 * of the wall face along the face's first tangential axis (x for y walls,
 * y for x walls); A and kappa are boundary parameters (dcf_set_params), so
 * that gradients reach them.  At most one face may be porous.  Returns
 * DCF_EINVAL for an unknown kind, a negative or non-finite T_wall, or a
 * porous strip outside the face.  A call that changes the number of
 * boundary parameters clears them: set them again before stepping. */
dcf_status dcf_set_bc(dcf_ctx *ctx, int face, const dcf_bc *bc);

/* Boundary parameters theta (dev, nK doubles): the porous coefficients K_i
 * (strip index fastest), then (A, kappa) of every disturbance face in face
 * order.  These are the differentiable inputs of dcf_vjp_step and
 * dcf_gradient (dJ/dtheta has the same layout).  The library reads them
 * from the caller's memory at every launch. */
dcf_status dcf_set_params(dcf_ctx *ctx, const double *K_dev, int nK);
int dcf_num_params(const dcf_ctx *ctx);

/* Spatial scheme.  DCF_SCHEME_WENO5 (default): WENO5-JS reconstruction of
 * the primitives (Section 2.1, "WENO-type") with 4th-order central
 * dissipative fluxes.  DCF_SCHEME_TENO6A: the channel scheme of Section 3.1,
 * TENO6-A reconstruction (sixth-order linear weights, adaptive cut-off) with
 * the interpolation limiter (a face side whose reconstructed density or
 * pressure is not positive takes its own cell's primitives) and 6th-order
 * central dissipative fluxes (tangential derivatives three cells either
 * side).  Forward calls only: dcf_vjp_step, dcf_gradient and the batched
 * steps return DCF_EUNSUPPORTED for TENO6-A.  DCF_EINVAL for another value. */
#define DCF_SCHEME_WENO5 0
#define DCF_SCHEME_TENO6A 1
dcf_status dcf_set_scheme(dcf_ctx *ctx, int scheme);

/* Source term (Eq. (1), sum_i S_i): DCF_SOURCE_MASSFLUX is the body force
 * that holds the bulk momentum of a channel constant (the constant-mass-flux
 * forcing of Section 3.1's channel), with f = -<R_rhou>_V each stage. */
dcf_status dcf_set_source(dcf_ctx *ctx, int kind);

/* Wall-pressure cost face: j(U) = sum_i (A_i/A)(p_i - p_ref)^2 over the
 * cells next to `face` (-1 disables), A_i the wall-face area of cell i and A
 * their sum.  The paper optimises boundary-condition parameters end to end
 * against a scalar objective of the flow (Section 1, Section 3.2); this
 * time-averaged wall-pressure-fluctuation cost (average of j over the steps
 * of a trajectory, dcf_gradient) is the build's reading of that objective
 * for the porous-wall boundary layer. */
dcf_status dcf_set_cost(dcf_ctx *ctx, int face, double p_ref);

/* ---- forward ------------------------------------------------------------ */
/* U (dev, out) from primitives P (dev), Eq. (2); needs no workspace. */
dcf_status dcf_init_state(dcf_ctx *ctx, const double *P_dev, double *U_dev, void *stream);

/* R = dU/dt of Eq. (6) including the source; R has the layout of U. */
dcf_status dcf_rhs(dcf_ctx *ctx, const double *U_dev, double *R_dev, void *stream);

/* dt_dev[0] = min(dt_max, cfl / max_cells[sum_d (|u_d|+c)/dx_d
 *             + 2 nu_eff sum_d 1/dx_d^2]), nu_eff = max(4/3, gamma/Pr) mu/rho.
 * The paper's explicit TVD Runge-Kutta integration (Section 2.1, text after
 * Eq. (6)) needs a stable step but states no rule for it: this convective
 * plus viscous CFL limit is the build's reading.  DCF_EINVAL for cfl <= 0;
 * dt_max <= 0 means no cap. */
dcf_status dcf_compute_dt(dcf_ctx *ctx, const double *U_dev, double cfl, double dt_max,
                          double *dt_dev, void *stream);

/* One TVD-RK3 step (Shu-Osher form; Section 2.1, text after Eq. (6)) in
 * place, with dt read from dt_dev[0]. */
dcf_status dcf_rk3_step(dcf_ctx *ctx, double *U_dev, const double *dt_dev, void *stream);

/* dcf_rk3_step that also keeps its two inner stage states:
 * stages_dev[0..M) = U^(1) = U^n + dt R(U^n) and stages_dev[M..2M) = U^(2) =
 * 3/4 U^n + 1/4 (U^(1) + dt R(U^(1))), M = nv * ncell (dev, caller-owned,
 * 2 state arrays, may not overlap U).  Bitwise the same U^{n+1} as
 * dcf_rk3_step; the stage states are what dcf_vjp_step reads instead of
 * recomputing them. */
dcf_status dcf_rk3_step_keep(dcf_ctx *ctx, double *U_dev, const double *dt_dev,
                             double *stages_dev, void *stream);

/* dcf_rk3_step for callers that cannot allocate device memory or be handed
 * a workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The forward workspace of the step is laid out in a
 * static scratch array of DCF_NOALLOC_SCRATCH_BYTES bytes that each device
 * holds from the library's first use on it (dcf_create resolves its address)
 * until the process ends; the call allocates and frees nothing.  The context
 * needs no workspace (one it has is left untouched).  flags_dev (nullable
 * dev, one unsigned): the non-physical flags of the step's kernels are OR-ed
 * into it (the caller clears it); NULL discards them.  DCF_EBUDGET when the
 * case needs more than DCF_NOALLOC_SCRATCH_BYTES (its mode-0 workspace size,
 * dcf_workspace_size).  Results are bitwise those of dcf_rk3_step.  Every
 * call on one device shares that device's scratch, which keeps the last
 * call's contents (no buffer in it needs to start at zero: each is written
 * before it is read within one call): calls that overlap on one device
 * (other streams or host threads) race and must be serialised by the
 * caller. */
#define DCF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
dcf_status dcf_rk3_step_noalloc(dcf_ctx *ctx, double *U_dev, const double *dt_dev,
                                unsigned *flags_dev, void *stream);

/* dcf_rk3_step fused with the CFL step of the new state: the last stage's
 * update also reduces the signal rates of the cells it writes, and
 * dt_next_dev[0] = min(dt_max, cfl / max_cells sigma(U^{n+1})), bitwise the
 * value dcf_compute_dt(U^{n+1}) would give (dt_max <= 0: no cap).  dt_next
 * may alias dt (the step reads dt before it is overwritten). */
dcf_status dcf_rk3_step_cfl(dcf_ctx *ctx, double *U_dev, const double *dt_dev, double cfl,
                            double dt_max, double *dt_next_dev, void *stream);

/* nsteps calls of dcf_rk3_step_cfl with dt_next = dt, in one call: each
 * step advances U with dt_dev[0], then dt_dev[0] becomes the CFL step of
 * the new state.  Bitwise the same U and dt as the separate calls; cheaper,
 * since a step after the first starts from the primitive box the previous
 * step's last update wrote (U is not touched in between).  DCF_EINVAL for
 * nsteps < 1 or cfl <= 0. */
dcf_status dcf_rk3_steps_cfl(dcf_ctx *ctx, double *U_dev, double *dt_dev, int nsteps, double cfl,
                             double dt_max, void *stream);

/* ---- batched stepping (the serving loop's step launches) ---------------- */
/* Bytes of the device table dcf_batch_rk3_step needs for n solves. */
dcf_status dcf_batch_table_bytes(int n, size_t *bytes);

/* One TVD-RK3 step of each of n independent solves with one launch per
 * kernel and stage for the whole batch (the same kernels as dcf_rk3_step;
 * workgroup (x, y) works on tile x of solve y, so solves of different grid
 * sizes share a launch).  ctxs[i] (distinct contexts, workspaces set),
 * U[i] (dev, advanced in place), dt[i] (dev, one double each).  With
 * cfl > 0 each solve's CFL step is computed first into dt[i] (as
 * dcf_compute_dt), otherwise dt[i] is read.  table: caller-owned device
 * memory of dcf_batch_table_bytes(n) bytes, 16-byte aligned, rewritten by
 * this call (an asynchronous host-to-device copy on `stream`; not for graph
 * capture).  Results are bitwise those of n calls of dcf_rk3_step.  The
 * solves must share ndim and the viscous flag (else DCF_EUNSUPPORTED) and
 * carry no source term (DCF_EUNSUPPORTED). */
dcf_status dcf_batch_rk3_step(dcf_ctx *const *ctxs, double *const *U, double *const *dt, int n,
                              double cfl, void *table, size_t table_bytes, void *stream);

/* The two halves of dcf_batch_rk3_step, so that the step launches can be
 * captured in a HIP graph and replayed while the batch does not change.
 * dcf_batch_table_fill validates the batch as dcf_batch_rk3_step does and
 * writes its table into table_host (host memory of dcf_batch_table_bytes(n)
 * bytes, 16-byte aligned); host work only.  The caller copies it to device
 * memory (outside any capture).  dcf_batch_rk3_step_table enqueues the step
 * launches alone: they read the table from table_dev (dev, a copy of
 * table_host, which must stay unchanged while launches or graph replays that
 * use it are pending); table_host is read during the call for the launch
 * sizes.  It enqueues kernels only (no copy, no allocation), so it may be
 * captured; the contexts, states and steps named in the table must outlive
 * every replay.  Bitwise the same results as dcf_batch_rk3_step. */
dcf_status dcf_batch_table_fill(dcf_ctx *const *ctxs, double *const *U, double *const *dt, int n,
                                void *table_host, size_t table_bytes);
dcf_status dcf_batch_rk3_step_table(const void *table_dev, const void *table_host, int n,
                                    double cfl, void *stream);

/* out_dev[8] = (<rho|u|^2/2>_V, <mu|omega|^2>_V, total mass, total x/y/z
 * momentum, total energy, volume): the kinetic-energy and dissipation
 * history of a Taylor-Green vortex and the conserved totals of Eq. (1). */
dcf_status dcf_diagnostics(dcf_ctx *ctx, const double *U_dev, double *out_dev, void *stream);

/* ---- adjoint ------------------------------------------------------------ */
/* Vector-Jacobian product of one RK3 step U^n -> U^{n+1} with dt_dev[0]
 * held constant (the reverse-mode derivative through the solver that the
 * paper's end-to-end optimisation rests on, Section 1; the boundary
 * parameters of Section 3.2 are differentiable inputs): lam_n =
 * (dU^{n+1}/dU^n)^T lam_np1, and, when dJdK_dev is not NULL, dJdK_dev +=
 * (dU^{n+1}/dK)^T lam_np1.  stages_dev (nullable dev): the step's stage
 * states U^(1), U^(2) as dcf_rk3_step_keep writes them; NULL recomputes them
 * from U^n (two more right-hand sides).  Branches (HLLC wave-speed cases,
 * min/max) follow the primal; with the mass-flux source the body force's
 * dependence on the state (through every cell's x-momentum right-hand side)
 * is included.  lam_n may not alias lam_np1.  Workspace mode >= 1;
 * DCF_EUNSUPPORTED for the TENO6-A scheme. */
dcf_status dcf_vjp_step(dcf_ctx *ctx, const double *Un_dev, const double *stages_dev,
                        const double *dt_dev, const double *lam_np1_dev, double *lam_n_dev,
                        double *dJdK_dev, void *stream);

/* J_dev[0] += w * j(U) with j the wall-pressure cost of dcf_set_cost; when
 * g_dev is not NULL, g_dev += w * dj/dU.  DCF_EINVAL without a cost face. */
dcf_status dcf_cost_term(dcf_ctx *ctx, const double *U_dev, double w, double *J_dev,
                         double *g_dev, void *stream);

/* J = (1/nsteps) sum_{n=1..nsteps} j(U^n) over a fixed-dt trajectory from U0,
 * and its gradient with respect to K and U0 -- the gradient through a whole
 * simulated trajectory that end-to-end optimisation needs (Section 1) -- by
 * checkpointing every seg_len steps and recomputing each segment in reverse
 * (workspace mode 2 or 3, sized for this seg_len and at least nsteps); the last
 * segment keeps its states from the forward sweep and is not recomputed
 * (seg_len >= nsteps: no recompute at all).  Any output pointer may be NULL
 * except J_dev.  DCF_EINVAL without a cost face, for another seg_len or for
 * more steps than the workspace holds; DCF_EUNSUPPORTED for the TENO6-A
 * scheme. */
dcf_status dcf_gradient(dcf_ctx *ctx, const double *U0_dev, int nsteps, const double *dt_dev,
                        int seg_len, double *J_dev, double *dJdK_dev, double *dJdU0_dev,
                        void *stream);

/* ---- measurement ---------------------------------------------------------- */
/* Times `reps` back-to-back launches of one kernel family on `stream` with
 * HIP events and returns the mean duration in milliseconds (synchronises).
 * which: 0 primitive box + halos, 1/2/3 face fluxes along x/y/z, 4 the
 * divergence + RK stage update, 5 the cell-centred velocity derivatives,
 * 6 the last direction's fluxes fused with the divergence and stage update
 * (2D/3D without source term; the kernel dcf_rk3_step runs in place of 3 or
 * 2 and 4), 7 the x and y face fluxes of a 3D grid in one launch (the form
 * the step runs in place of 1 and 2), 8 the ghost cells of the primitive box
 * alone (stages 2 and 3 of such a step: the previous stage's update wrote
 * the interior).  5 and 9 are not used: the flux kernels compute the
 * cell-centred velocity derivatives while staging their tiles (no separate
 * derivative launch).  The inputs it needs (primitive box, face fluxes) are
 * computed from U once before timing.  DCF_EINVAL for an unknown `which` or
 * one the case does not have. */
dcf_status dcf_time_kernel(dcf_ctx *ctx, const double *U_dev, int which, int reps,
                           double *avg_ms, void *stream);

/* Launch probe: while armed, every launch of kernel family `which` (the ids of
 * dcf_time_kernel: 1 x fluxes of a 2D step, 6 fused last-direction flux +
 * update, 7 x + y fluxes of a 3D step, 8 ghost fill of stages after the
 * first (with the carried CFL reduction where a step follows another in one
 * call)) that the fused stepping calls (dcf_rk3_step,
 * dcf_rk3_step_cfl, dcf_rk3_steps_cfl) make is bracketed by a pair of HIP
 * events recorded on that call's stream, up to max_launches launches (later
 * ones are not recorded).  The events are created here and owned by the
 * context.  dcf_probe_end waits for the last recorded event, returns the
 * number of recorded launches and their mean duration in milliseconds, and
 * releases the events (a later dcf_probe_begin may arm again).  DCF_EINVAL for
 * an id that cannot be probed, max_launches outside [1, 2^20], arming twice or
 * ending an unarmed probe. */
dcf_status dcf_probe_begin(dcf_ctx *ctx, int which, int max_launches);
dcf_status dcf_probe_end(dcf_ctx *ctx, int *launches, double *avg_ms);

/* Incremental form of dcf_gradient, for schedulers that interleave many
 * solves: begin validates and records the request (same arguments as
 * dcf_gradient, J and dJdK zeroed on `stream`); advance enqueues at most
 * max_units units of work -- a forward step with its checkpoint and cost
 * term, a recomputed step of the current segment, or one reverse step (the
 * first nsteps units are the forward sweep, after which J is complete) -- and
 * sets *done once the reverse sweep has reached U0; finish copies dJ/dU0
 * (nullable).  Between calls nothing is read back; the host keeps only the
 * position in the trajectory. */
dcf_status dcf_gradient_begin(dcf_ctx *ctx, const double *U0_dev, int nsteps,
                              const double *dt_dev, int seg_len, double *J_dev, double *dJdK_dev,
                              void *stream);
dcf_status dcf_gradient_advance(dcf_ctx *ctx, int max_units, int *done, void *stream);
dcf_status dcf_gradient_finish(dcf_ctx *ctx, double *dJdU0_dev, void *stream);

/* ---- status ------------------------------------------------------------- */
/* Synchronises `stream`, returns and clears the kernel flags (DCF_FLAG_*). */
dcf_status dcf_flags(dcf_ctx *ctx, unsigned *flags_host, void *stream);
const char *dcf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DCF_H */
