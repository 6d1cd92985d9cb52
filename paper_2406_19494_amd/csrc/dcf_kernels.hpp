// dcf_kernels.hpp -- host-side launchers of the library's kernels.  Each
// launcher enqueues on `st` and returns the launch status.
#pragma once

#include "dcf_common.hpp"

namespace dcf {

constexpr int RED_BLOCKS = 1024;  // partial-sum slots of the two-pass reductions

hipError_t launch_metrics(int kind, double lo, double hi, double beta, int n, double *dx,
                          double *idx, double *mc, double *mf, double *xm, hipStream_t st);
hipError_t launch_init_state(const Dev &g, const double *P, double *U, hipStream_t st);
hipError_t launch_prim_halo(const Dev &g, const double *U, hipStream_t st);
hipError_t launch_fluxes(const Dev &g, hipStream_t st);
hipError_t launch_flux_dir(const Dev &g, int D, hipStream_t st);
hipError_t launch_grad(const Dev &g, hipStream_t st);
hipError_t launch_force(const Dev &g, double *part, double *force, hipStream_t st);
hipError_t launch_update(const Dev &g, const double *Un, const double *Uin, double *Uout,
                         double *Rout, const double *dt, double a, double b,
                         const double *force, hipStream_t st);
hipError_t launch_dt(const Dev &g, const double *U, double cfl, double dt_max, double *part,
                     double *dt, hipStream_t st);
hipError_t launch_diag(const Dev &g, const double *U, double *part, double *out,
                       hipStream_t st);
hipError_t launch_cost(const Dev &g, int face, double pref, const double *U, double w,
                       double *J, double *grad, hipStream_t st);
hipError_t launch_fill(double *p, double v, long n, hipStream_t st);
hipError_t launch_copy(double *dst, const double *src, long n, hipStream_t st);
hipError_t launch_axpy(double *y, double a, const double *x, long n, hipStream_t st);

}  // namespace dcf
