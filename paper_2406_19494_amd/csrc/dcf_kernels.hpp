// dcf_kernels.hpp -- host-side launchers of the library's kernels.  Each
// launcher enqueues on `st` and returns the launch status.
#pragma once

#include "dcf_common.hpp"

namespace dcf {

constexpr int RED_BLOCKS = 1024;  // partial-sum slots of the two-pass reductions

// One solve of a batched step: its context, its buffers and the number of
// workgroups each kernel needs for it.  A device array of these is the tile
// table of the batched launches (workgroup (x, y) = tile x of solve y).
struct BatchEntry {
  Dev g;
  Dev gb;               // the same solve with the second primitive box (2D/3D stages
                        // alternate the two, as the single-solve step does)
  double *U, *U1, *U2;  // state (advanced in place) and the two stage states
  double *dt;           // step size (device, one double)
  double *part;         // reduction partials of the CFL step
  unsigned nb_prim, nb_ghost, nb_x, nb_upd, nb_dt;
  unsigned yz_nbx[3], yz_nby[3], yz_ntot[3];  // tile grids of the y and z fluxes
  unsigned fu_nbx, fu_nby, fu_ntot;           // tile grid of the fused last-direction kernel
  int nwmax;            // x-flux LDS window length
};

// Fills the per-kernel workgroup counts of an entry (host side).
void batch_entry_sizes(BatchEntry &e);
// One TVD-RK3 step of every solve in the table (tab_dev: device copy of
// tab_host), optionally preceded by the CFL step (cfl > 0).  All entries
// share ndim and the viscous flag and carry no source term.
hipError_t launch_batch_step(const BatchEntry *tab_dev, const BatchEntry *tab_host, int n,
                             double cfl, hipStream_t st);

hipError_t launch_metrics(int kind, double lo, double hi, double beta, int n, double *dx,
                          double *idx, double *mc, double *mf, double *xm, hipStream_t st);
// out[0] = dx[0] + dx[1] + ... + dx[n-1], summed in index order.
hipError_t launch_line_length(const double *dx, int n, double *out, hipStream_t st);
hipError_t launch_init_state(const Dev &g, const double *P, double *U, hipStream_t st);
hipError_t launch_prim_halo(const Dev &g, const double *U, hipStream_t st);
hipError_t launch_fluxes(const Dev &g, hipStream_t st);
hipError_t launch_flux_dir(const Dev &g, int D, hipStream_t st);
// x and y face fluxes of a 3D grid in one launch.
hipError_t launch_flux_xy(const Dev &g, hipStream_t st);
// Body force of the constant-mass-flux source from the boundary face fluxes
// of directions D < ndir (default: all; the others must be periodic).
hipError_t launch_force(const Dev &g, double *part, double *force, hipStream_t st, int ndir = -1);
// The same body force from the primitive box alone (boundary face fluxes
// evaluated here; bitwise launch_force's value over the flux kernels'
// fluxes).  part: 2 RED_BLOCKS doubles.
hipError_t launch_force_direct(const Dev &g, double *part, double *force, hipStream_t st);
// With dtpart (update_blocks(g) doubles) each block also writes the largest
// signal rate of its cells' new state (the CFL step of the next step).
hipError_t launch_update(const Dev &g, const double *Un, const double *Uin, double *Uout,
                         double *Rout, const double *dt, double a, double b,
                         const double *force, hipStream_t st, double *dtpart = nullptr);
unsigned update_blocks(const Dev &g);
// The whole right-hand side and stage update with the last direction's
// fluxes fused into the update (ndim >= 2, no source term): the other
// directions' fluxes, then one kernel for the last direction + update (the
// flux kernels compute the velocity derivatives they need while staging).
// With dtpart (flux_update_blocks(g) doubles) the CFL partials as above.
// With qo the kernel also writes the new state's primitives (and mu) into
// the interior of the box qo (same layout as g.Q, another buffer), as
// k_prim_interior would: the next stage then only fills the ghosts
// (launch_prim_ghost on a context whose Q is qo).  With force (the
// constant-mass-flux source; the last direction periodic) the body force is
// reduced into force (partials in part) before the fused kernel applies it.
// HIP event pairs around the launches of one kernel family (the ids of
// dcf_time_kernel) while armed: before/after record on the launch's stream,
// up to cap launches.  Host-side bookkeeping only.
struct Probe {
  int which = -1;
  hipEvent_t *ev = nullptr;  // 2 * cap events: start, end of each launch
  int cap = 0, n = 0;
  void before(int w, hipStream_t st) {
    if (w == which && n < cap) (void)hipEventRecord(ev[2 * n], st);
  }
  void after(int w, hipStream_t st) {
    if (w != which || n >= cap) return;
    (void)hipEventRecord(ev[2 * n + 1], st);
    ++n;
  }
};

// With pr the x+y or x flux (7 / 1) and fused update (6) launches are
// bracketed by its events.
hipError_t launch_fluxes_update(const Dev &g, const double *Un, const double *Uin,
                                double *Uout, const double *dt, double a, double b,
                                double *dtpart, hipStream_t st, const BoxOut &qo = BoxOut{},
                                double *part = nullptr, double *force = nullptr,
                                Probe *pr = nullptr);
unsigned flux_update_blocks(const Dev &g);
// The last direction's flux + update kernel alone (the other directions'
// fluxes already computed).
hipError_t launch_flux_update_last(const Dev &g, const double *Un, const double *Uin,
                                   double *Uout, const double *dt, double a, double b,
                                   double *dtpart, hipStream_t st, const BoxOut &qo = BoxOut{},
                                   const double *force = nullptr);
// Ghost cells of the box from its interior (the interior already filled).
hipError_t launch_prim_ghost(const Dev &g, hipStream_t st);
// launch_prim_ghost and launch_dt_final in one launch (the reduction reads
// part as left by earlier launches and writes dt for later ones).
hipError_t launch_prim_ghost_dt(const Dev &g, const double *part, int nparts, double cfl,
                               double dt_max, double *dt, hipStream_t st);
// The interior cells' primitives alone (the first launch of launch_prim_halo's
// two-launch form).
hipError_t launch_prim_interior(const Dev &g, const double *U, hipStream_t st);
hipError_t launch_dt_final(const double *part, int nparts, double cfl, double dt_max, double *dt,
                           hipStream_t st);
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
