// dcf_adjoint.hpp -- buffers and entry of the hand-written adjoint (VJP) of
// one TVD-RK3 step.
#pragma once

#include "dcf_common.hpp"
#include "dcf_kernels.hpp"

namespace dcf {

struct AdjBuffers {
  double *Qb[NQ];   // adjoint of the primitive box (rho, u, v, w, p, T, mu)
  double *Gb[9];    // adjoint of cell-centred velocity derivatives d u_phi / d x_t (3 t + phi)
  double *Qby[NQ];  // 2D: the y-direction tiles' Qb contributions (no w), added to Qb's
                    // on ghost and interior cells; every cell read is written each stage
  double *Ub1, *Ub2;  // stage adjoints
  const double *Wb;  // stage-output adjoint of the stage being reversed
  double *fwb;       // (body force) Wb with the corrected x-momentum component
  const double *dtp; // step size (device)
  double bcoef;      // weight b of the stage's V + dt R(V) term
  double *src;      // body-force adjoint of a stage: f, f-bar = sum Rb_rhou + Rb_E u, volume
  double *spart;    // reduction partials of the body force and of its adjoint
  double *dpart;    // per-column partial sums of dJ/d(A, kappa), 4 per wall column
  long dcols;       // columns per disturbance-face partial array
  double *zero_begin;  // Qb and Gb are carved back to back: one clear (with the
                       // workspace) zeroes both
  long zero_count;
};

// Lays the adjoint buffers out in the workspace (or measures them).
template <class Carver> void carve_adjoint(Carver &cv, const Dev &g, AdjBuffers &a) {
  const size_t off0 = cv.off;
  for (int q = 0; q < NQ; ++q) a.Qb[q] = cv.template take<double>(g.nboxp);
  const bool visc = g.visc != VISC_NONE && g.ndim >= 2;
  for (int q = 0; q < 9; ++q)
    a.Gb[q] = (visc && q / 3 < g.ndim && q % 3 < g.ndim) ? cv.template take<double>(g.nboxp)
                                                           : nullptr;
  a.zero_begin = a.Qb[0];
  a.zero_count = (long)((cv.off - off0) / sizeof(double));
  for (int q = 0; q < NQ; ++q)
    a.Qby[q] = (g.ndim == 2 && q != QW) ? cv.template take<double>(g.nboxp) : nullptr;
  a.Ub1 = cv.template take<double>((long)g.nv * g.ncell);
  a.Ub2 = cv.template take<double>((long)g.nv * g.ncell);
  long cols = 1;
  for (int d = 0; d < g.ndim; ++d) {
    const int t1 = tan1(d), t2 = tan2(d);
    long n1 = t1 < d ? g.N[t1] : g.n[t1], n2 = t2 < d ? g.N[t2] : g.n[t2];
    cols = n1 * n2 > cols ? n1 * n2 : cols;
  }
  a.dcols = cols;
  a.dpart = cv.template take<double>(4 * cols);
  a.src = cv.template take<double>(4);
  a.fwb = cv.template take<double>((long)g.nv * g.ncell);
  a.spart = cv.template take<double>(2 * RED_BLOCKS);
}

// lam0 = (dU^{n+1}/dU^n)^T lam1 and dJdK += (dU^{n+1}/dK)^T lam1 (if not
// null).  U1 and U2 hold the stage states of Un (as the forward step made
// them).  With `boxes` (three contexts whose Q point at the cached primitive
// boxes of Un, U1, U2) nothing of the forward is recomputed; without, each
// stage's primitive box is recomputed into g.Q.
hipError_t vjp_step(Dev g, const AdjBuffers &a, const double *Un, const double *U1,
                    const double *U2, const double *dt, const double *lam1, double *lam0,
                    double *dJdK, hipStream_t st, const Dev *boxes = nullptr);

}  // namespace dcf
