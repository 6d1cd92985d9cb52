/*
 * oracle.h -- C interface of the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, obviously-correct
 * FP64 CPU implementation of the finite-volume right-hand side of the
 * compressible Navier-Stokes equations (paper, Section 2.1, Eqs. (1)-(6)),
 * the halo-cell boundary conditions (Section 3.2), the explicit TVD
 * Runge-Kutta integration (Section 2.1, text after Eq. (6)) and a dense,
 * forward-mode adjoint for tiny grids.  Only tests/, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header
 * or constant with the GPU library; the two meet only through seeded input
 * arrays.
 *
 * Array layouts (all FP64, caller-owned host memory):
 *   interior state U      [nv][nz][ny][nx], nv = ndim + 2
 *                         (rho, rho*u[, rho*v[, rho*w]], E)
 *   primitive input P     [5][nz][ny][nx]   (rho, u, v, w, p); unused
 *                         velocity components must be zero
 *   boundary parameters K [nK]: the porous coefficients, (porous_end -
 *                         porous_begin) * n_t2 of them, strip index fastest,
 *                         then (A, kappa) of every disturbance-wall face in
 *                         face order
 *   halo'd box            [nz + 2hz][ny + 2hy][nx + 2hx], h = 3 on active
 *                         axes and 0 on inactive ones
 */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_PERIODIC = 0,
  ORC_WALL = 1,      /* isothermal no-slip wall                            */
  ORC_POROUS = 2,    /* isothermal wall with Darcy transpiration strip     */
  ORC_ZEROGRAD = 3,  /* zero-gradient extrapolation                         */
  ORC_DIRICHLET = 4, /* prescribed primitive profile                        */
  ORC_DISTURB = 5    /* no-slip wall with prescribed normal velocity
                        A sin(2 pi kappa x_t) (Section 3.2, Eq. (8)); A and
                        kappa are boundary parameters (entries of K)         */
};

enum { ORC_VISC_NONE = 0, ORC_VISC_POWER = 1, ORC_VISC_SUTHERLAND = 2 };
enum { ORC_STRETCH_UNIFORM = 0, ORC_STRETCH_TANH2 = 1, ORC_STRETCH_TANH1 = 2 };
enum { ORC_SOURCE_NONE = 0, ORC_SOURCE_MASSFLUX = 1 };
/* Spatial scheme: WENO5-JS reconstruction with 4th-order central dissipative
 * fluxes, or the channel scheme of Section 3.1: TENO6-A reconstruction with
 * the interpolation limiter and 6th-order central dissipative fluxes. */
enum { ORC_SCHEME_WENO5 = 0, ORC_SCHEME_TENO6A = 1 };

typedef struct {
  int ndim;
  int n[3];              /* interior cells per axis (1 on inactive axes)     */
  double lo[3], hi[3];   /* domain extent per axis                          */
  int stretch[3];        /* ORC_STRETCH_*                                    */
  double beta[3];        /* tanh stretching parameter                        */
  double gamma, R, Pr;   /* ideal gas, specific gas constant, Prandtl number */
  int visc_law;          /* ORC_VISC_*                                       */
  double mu_ref, T_ref;  /* viscosity at the reference temperature          */
  double visc_param;     /* power-law exponent, or Sutherland constant       */
  int bc[6];             /* faces x-, x+, y-, y+, z-, z+                    */
  double T_wall[6];      /* wall temperature per face; 0 = adiabatic wall     */
  const double *dirichlet[6]; /* [5][n_t2][n_t1] per Dirichlet face          */
  int porous_face;       /* face carrying the porous strip, -1 for none      */
  int porous_begin, porous_end; /* strip range along the first tangential axis */
  double p_inf;          /* reference pressure of the Darcy law and the cost */
  int source;            /* ORC_SOURCE_*                                     */
  int cost_face;         /* face of the wall-pressure cost, -1 for none      */
  int scheme;            /* ORC_SCHEME_*                                     */
} orc_case;

int orc_nk(const orc_case *c);
long orc_ncells(const orc_case *c);
long orc_nbox(const orc_case *c);

void orc_grid(const orc_case *c, int axis, double *xf, double *dx, double *met_c,
              double *met_f);
double orc_weno5(double a, double b, double c, double d, double e);
/* TENO6-A value at the right face of cell c from (a, b, c, d, e, f) =
 * cells c-2 .. c+3; ct_out (nullable) receives the cut-off C_T it used and
 * w_out (nullable, 4) the weights of the candidates (S0 = c-1..c+1,
 * S1 = c..c+2, S2 = c-2..c, S3 = c..c+3). */
double orc_teno6a(const double *v, double *ct_out, double *w_out);
/* Its smoothness indicators beta0, beta1, beta2, beta3, beta6 (out[5]). */
void orc_teno6a_beta(const double *v, double *beta);
/* Central stencils of the dissipative fluxes on point values v at offsets
 * -3 .. 3: 6th-order face value, face derivative (face between offsets 0
 * and 1) and cell derivative (offset 0), then the same at 4th order. */
void orc_central_stencils(const double *v, double *out);
void orc_hllc(const double *qL, const double *qR, double gamma, double *F);

void orc_cons_from_prim(const orc_case *c, const double *P, double *U);
void orc_prims_halo(const orc_case *c, const double *K, const double *U, double *Qbox,
                    double *mubox);
void orc_rhs(const orc_case *c, const double *K, const double *U, double *R);
double orc_dt(const orc_case *c, const double *U, double cfl);
void orc_step(const orc_case *c, const double *K, double *U, double dt);
int orc_run(const orc_case *c, const double *K, double *U, int max_steps, double cfl,
            double dt_fixed, double t_end, double *t_out);
void orc_diag(const orc_case *c, const double *U, double *out);

double orc_cost_term(const orc_case *c, const double *U);
void orc_cost_term_grad(const orc_case *c, const double *U, double *g);
void orc_jvp_step(const orc_case *c, const double *K, const double *dK, const double *U,
                  const double *dU, double dt, double *U1, double *dU1);
void orc_vjp_step(const orc_case *c, const double *K, const double *U, double dt,
                  const double *lam, double *lamU, double *lamK);
double orc_gradient(const orc_case *c, const double *K, const double *U0, int nsteps,
                    double dt, double *dJdK, double *dJdU0);

/* OpenMP threads of the per-line loops: n > 0 sets them; returns the number
 * the next parallel loop will use. */
int orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
