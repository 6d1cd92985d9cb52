// dcf_forward.hip -- forward kernels: grid metrics, conversion to
// primitives fused with the halo fill, per-direction face fluxes, the fused
// divergence + source + TVD-RK3 stage update, and deterministic reductions
// (CFL time step, body force, diagnostics, wall-pressure cost).
#include <algorithm>

#include "dcf_kernels.hpp"

namespace dcf {

// ---------------------------------------------------------------------------
// Grid metrics of one axis (stretched Cartesian meshes, Section 2; the tanh
// law of Section 3.2).  Face i at xi = i, centre at xi = i + 1/2.
// ---------------------------------------------------------------------------
__device__ void axis_map(int kind, double lo, double hi, double beta, int n, double s, double *x,
                         double *dxdxi) {
  double L = hi - lo;
  if (kind == 1) {  // symmetric clustering toward both ends
    double a = beta * (1.0 - 2.0 * s);
    double th = tanh(beta);
    *x = lo + L * 0.5 * (1.0 - tanh(a) / th);
    double ch = cosh(a);
    *dxdxi = L * beta / (n * th * ch * ch);
  } else if (kind == 2) {  // clustering toward lo
    double a = beta * (s - 1.0);
    double th = tanh(beta);
    *x = lo + L * (1.0 + tanh(a) / th);
    double ch = cosh(a);
    *dxdxi = L * beta / (n * th * ch * ch);
  } else {
    *x = lo + L * s;
    *dxdxi = L / n;
  }
}

__global__ void k_metrics(int kind, double lo, double hi, double beta, int n, double *dx,
                          double *idx, double *mc, double *mf, double *xm) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  double x0, g0;
  axis_map(kind, lo, hi, beta, n, (double)i / n, &x0, &g0);
  mf[i] = 1.0 / g0;
  if (i < n) {
    double x1, g1, xc, gc;
    axis_map(kind, lo, hi, beta, n, (double)(i + 1) / n, &x1, &g1);
    axis_map(kind, lo, hi, beta, n, (i + 0.5) / n, &xc, &gc);
    dx[i] = x1 - x0;
    idx[i] = 1.0 / (x1 - x0);
    xm[i] = 0.5 * (x0 + x1);
    mc[i] = 1.0 / gc;
  }
}

// The cell widths of an axis summed in index order (one thread: the order of
// the sum is part of the value).  Widths are loaded 16 at a time, all loads
// of a group issued before its adds, so the sum waits for one memory round
// trip per group instead of one per cell.
__global__ void k_line_length(const double *dx, int n, double *out) {
  double L = 0.0;
  for (int i0 = 0; i0 < n; i0 += 16) {
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = i0 + u < n ? dx[i0 + u] : 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (i0 + u < n) L += t[u];
  }
  *out = L;
}

// ---------------------------------------------------------------------------
// Primitives from conserved variables (Eq. (2), ideal gas).
// ---------------------------------------------------------------------------
// From (rho, rho u, rho v, rho w, E) with zeros for unused momenta.
__device__ __forceinline__ void prim_of_state(const Dev &g, const double *s, double *q) {
  const int nd = g.ndim;
  double rho = s[0];
  double ir = rcp_nr(rho);
  double u = s[1] * ir;
  double v = nd >= 2 ? s[2] * ir : 0.0;
  double w = nd >= 3 ? s[3] * ir : 0.0;
  double E = s[4];
  double p = (g.gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v + w * w));
  q[QR] = rho;
  q[QU] = u;
  q[QV] = v;
  q[QW] = w;
  q[QP] = p;
  q[QT] = p * ir * g.iR;
}

__device__ __forceinline__ void cons_to_prim(const Dev &g, const double *U, long c, double *q) {
  const int nd = g.ndim;
  const long nc = g.ncell;
  double rho = U[c];
  double ir = rcp_nr(rho);
  double u = U[nc + c] * ir;
  double v = nd >= 2 ? U[2 * nc + c] * ir : 0.0;
  double w = nd >= 3 ? U[3 * nc + c] * ir : 0.0;
  double E = U[(long)(nd + 1) * nc + c];
  double p = (g.gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v + w * w));
  q[QR] = rho;
  q[QU] = u;
  q[QV] = v;
  q[QW] = w;
  q[QP] = p;
  q[QT] = p * ir * g.iR;
}

__global__ void k_init_state(Dev g, const double *P, double *U) {
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const long nc = g.ncell;
  const int nd = g.ndim;
  double rho = P[c], u = P[nc + c], v = P[2 * nc + c], w = P[3 * nc + c], p = P[4 * nc + c];
  U[c] = rho;
  U[nc + c] = rho * u;
  if (nd >= 2) U[2 * nc + c] = rho * v;
  if (nd >= 3) U[3 * nc + c] = rho * w;
  U[(long)(nd + 1) * nc + c] = p / (g.gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
}

// ---------------------------------------------------------------------------
// Primitive box with halos.  The halo fill of the paper (values assigned to
// halo cells, Section 3.2) is applied axis by axis, x then y then z, each
// over the full extent of the axes filled before; a ghost thread resolves
// that chain for its own cell: it follows the source cells back to the
// interior (or to a Dirichlet profile) and applies the per-axis ghost
// transforms in x, y, z order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ghost_source(int kind, int side, int m, int n) {
  if (kind == BC_PERIODIC) return side == 0 ? n - 1 - m : m;
  if (kind == BC_ZEROGRAD) return side == 0 ? 0 : n - 1;
  return side == 0 ? m : n - 1 - m;  // walls mirror
}

// Sources of the ghost chain: the conserved state (the source cell is
// converted here) or the primitive box once its interior is filled (the
// source's primitives and mu are copied).
struct FromState {
  const double *U;
  __device__ __forceinline__ void load(const Dev &g, const int *s, double *q, double &mu) const {
    cons_to_prim(g, U, ((long)s[2] * g.n[1] + s[1]) * g.n[0] + s[0], q);
    mu = -1.0;
  }
  __device__ __forceinline__ double pressure(const Dev &g, const int *w) const {
    double q[6];
    cons_to_prim(g, U, ((long)w[2] * g.n[1] + w[1]) * g.n[0] + w[0], q);
    return q[QP];
  }
};
struct FromBox {
  __device__ __forceinline__ void load(const Dev &g, const int *s, double *q, double &mu) const {
    const int nd = g.ndim;
    const long sb = bidx(g, s[0], s[1], s[2]);
    q[QR] = g.Q[QR][sb];
    q[QU] = g.Q[QU][sb];
    q[QV] = nd >= 2 ? g.Q[QV][sb] : 0.0;
    q[QW] = nd >= 3 ? g.Q[QW][sb] : 0.0;
    q[QP] = g.Q[QP][sb];
    if (g.visc != VISC_NONE) {
      q[QT] = g.Q[QT][sb];
      mu = g.Q[QMU][sb];
    } else {
      q[QT] = q[QP] / (q[QR] * g.R);
      mu = -1.0;
    }
  }
  __device__ __forceinline__ double pressure(const Dev &g, const int *w) const {
    return g.Q[QP][bidx(g, w[0], w[1], w[2])];
  }
};

// Ghost cell p (box index b) through the halo-fill chain: follow the source
// cells back to the interior (or to a Dirichlet profile), then apply the
// per-axis ghost transforms in x, y, z order; mu is recomputed unless the
// source's is still valid (copied and no transform changed T).
template <class Src>
__device__ __forceinline__ void ghost_chain(const Dev &g, const int *p, long b, const Src &src) {
  const int nd = g.ndim;
  int s[3] = {p[0], p[1], p[2]};
  int side[3] = {0, 0, 0};
  bool gh[3] = {false, false, false};
  int top = -1;
  for (int d = 0; d < nd; ++d) {
    if (p[d] < 0 || p[d] >= g.n[d]) {
      gh[d] = true;
      side[d] = p[d] < 0 ? 0 : 1;
      int m = side[d] == 0 ? -1 - p[d] : p[d] - g.n[d];
      int kind = g.bck[2 * d + side[d]];
      if (kind == BC_DIRICHLET)
        top = d;
      else
        s[d] = ghost_source(kind, side[d], m, g.n[d]);
    }
  }
  double q[6];
  double mu = -1.0;  // mu of the source while no transform changed T
  int start = 0;
  if (top >= 0) {
    const int d = top;
    const int t1 = tan1(d), t2 = tan2(d);
    int a = t1 < nd ? (t1 < d ? p[t1] : s[t1]) : 0;
    int bb = t2 < nd ? (t2 < d ? p[t2] : s[t2]) : 0;
    a = min(max(a, 0), g.n[t1] - 1);
    bb = min(max(bb, 0), g.n[t2] - 1);
    const long nt = (long)g.n[t1] * g.n[t2];
    const long o = (long)bb * g.n[t1] + a;
    const double *P = g.dir[2 * d + side[d]];
    q[QR] = P[o];
    q[QU] = P[nt + o];
    q[QV] = P[2 * nt + o];
    q[QW] = P[3 * nt + o];
    q[QP] = P[4 * nt + o];
    q[QT] = q[QP] / (q[QR] * g.R);
    mu = -1.0;  // recomputed below
    start = top + 1;
  } else {
    src.load(g, s, q, mu);  // the interior source cell
  }
  for (int d = start; d < nd; ++d) {
    if (!gh[d]) continue;
    const int face = 2 * d + side[d];
    const int kind = g.bck[face];
    if (!is_wall(kind)) continue;  // copies keep the value
    double src_n = q[QU + d];
    q[QU] = -q[QU];
    q[QV] = -q[QV];
    q[QW] = -q[QW];
    const int t1 = tan1(d), t2 = tan2(d);
    const int a = t1 < nd ? (t1 < d ? p[t1] : s[t1]) : 0;
    const int bb = t2 < nd ? (t2 < d ? p[t2] : s[t2]) : 0;
    const double sigma = side[d] == 0 ? 1.0 : -1.0;
    if (kind == BC_POROUS && face == g.pface) {
      if (a >= g.pb && a < g.pe && bb >= 0 && bb < g.n[t2]) {
        // Darcy transpiration through the porous strip: inward-normal
        // velocity -K (p_w - p_inf)/p_inf, p_w of the first interior cell.
        int w[3];
        w[d] = side[d] == 0 ? 0 : g.n[d] - 1;
        w[t1] = a;
        w[t2] = bb;
        const double pw = src.pressure(g, w);
        int kk = bb * (g.pe - g.pb) + (a - g.pb);
        double vn = -g.K[kk] * (pw - g.pinf) / g.pinf;
        q[QU + d] = 2.0 * sigma * vn - src_n;
      }
    } else if (kind == BC_DISTURB && a >= 0 && a < g.n[t1]) {
      // Disturbance wall (Section 3.2, Eq. (8)): prescribed inward-normal
      // velocity A sin(2 pi kappa x) at the wall-face centre, (A, kappa)
      // taken from the boundary parameters.
      const double *th = g.K + g.doff[face];
      double vn = th[0] * sin(2.0 * M_PI * g.xm[t1][a] * th[1]);
      q[QU + d] = 2.0 * sigma * vn - src_n;
    }
    if (g.Tw[face] > 0.0) {  // isothermal; adiabatic keeps rho and T
      double Tg = 2.0 * g.Tw[face] - q[QT];
      if (!(Tg > 0.0)) atomicOr(g.flags, 1u);
      q[QT] = Tg;
      q[QR] = q[QP] / (g.R * Tg);
      mu = -1.0;
    }
  }
  g.Q[QR][b] = q[QR];
  g.Q[QU][b] = q[QU];
  if (nd >= 2) g.Q[QV][b] = q[QV];
  if (nd >= 3) g.Q[QW][b] = q[QW];
  g.Q[QP][b] = q[QP];
  if (g.visc != VISC_NONE) {
    g.Q[QT][b] = q[QT];
    g.Q[QMU][b] = mu >= 0.0 ? mu : viscosity(g, q[QT]);
  }
}

// Interior cells: primitives of their own conserved state (x-fastest,
// coalesced).
__device__ __forceinline__ void prim_interior_body(const Dev &g, const double *U, unsigned t) {
  if (t >= (unsigned)g.ncell) return;
  const int nd = g.ndim;
  const unsigned n0 = g.n[0], n01 = n0 * (unsigned)g.n[1];
  const int k = (int)(t / n01), j = (int)((t % n01) / n0), i = (int)(t % n0);
  const long b = bidx(g, i, j, k);
  double q[6];
  cons_to_prim(g, U, (long)t, q);
  if (!(finite_pos(q[QR]) && finite_pos(q[QP]))) atomicOr(g.flags, 1u);
  g.Q[QR][b] = q[QR];
  g.Q[QU][b] = q[QU];
  if (nd >= 2) g.Q[QV][b] = q[QV];
  if (nd >= 3) g.Q[QW][b] = q[QW];
  g.Q[QP][b] = q[QP];
  if (g.visc != VISC_NONE) {
    g.Q[QT][b] = q[QT];
    g.Q[QMU][b] = viscosity(g, q[QT]);
  }
}

// Single-launch form (used when ghost cells are a small share of the box):
// threads [0, ncell) convert interior cells (x-fastest, coalesced, one
// branch for the whole wave); threads [ncell, nbox) fill the ghost cells,
// converting their source cell's state themselves.
__device__ __forceinline__ void prim_halo_body(const Dev &g, const double *U, unsigned t) {
  if (t >= (unsigned)g.nbox) return;
  if (t < (unsigned)g.ncell) {
    prim_interior_body(g, U, t);
    return;
  }
  int p[3];
  ghost_position(g, t - (unsigned)g.ncell, p);
  ghost_chain(g, p, bidx(g, p[0], p[1], p[2]), FromState{U});
}

__global__ void __launch_bounds__(256) k_prim_halo(Dev g, const double *U) {
  prim_halo_body(g, U, blockIdx.x * blockDim.x + threadIdx.x);
}


// Ghost cell number t (after k_prim_interior): follow the chain of sources
// back to an interior cell (or a Dirichlet profile), copy its primitives from
// the box and apply the per-axis ghost transforms in x, y, z order; mu is
// recomputed only where a transform changed T.

// Ghost cell number t, after k_prim_interior has filled the interior.
__device__ __forceinline__ void prim_ghost_body(const Dev &g, unsigned t) {
  if (t >= (unsigned)(g.nbox - g.ncell)) return;
  int p[3];
  ghost_position(g, t, p);
  ghost_chain(g, p, bidx(g, p[0], p[1], p[2]), FromBox{});
}

// Two-launch form (many ghost cells): interior cells, then the ghost cells
// copied from the interior ones.
__global__ void __launch_bounds__(256) k_prim_interior(Dev g, const double *U) {
  prim_interior_body(g, U, blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(256) k_prim_ghost(Dev g) {
  prim_ghost_body(g, blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Total flux F = F^c - F^d at one face of direction D (Eq. (6)), in the
// global 5-component layout (mass, x/y/z momentum, energy).  The stencil is
// read through accessors: P(q, o) is primitive q of the cell at offset o from
// the face (o = -3 .. 2; the face lies between offsets -1 and 0), Gv(k, o) is
// the k-th tangential velocity derivative of that cell (o = -2 .. 1; k = 2 r
// + 0: d u_t / d t, k = 2 r + 1: d u_D / d t, r over the active tangential
// axes).
// ---------------------------------------------------------------------------
template <int NDIM, int D, bool VISC, int SCH, class PA, class GA>
__device__ __forceinline__ void face_flux(const Dev &g, const PA &P, const GA &Gv, int f,
                                          double *G) {
  constexpr int T1 = tan1(D), T2 = tan2(D);
  constexpr int qi[5] = {QR, QU + D, QU + T1, QU + T2, QP};
  double qL[5], qR[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    if ((m == 2 && T1 >= NDIM) || (m == 3 && T2 >= NDIM)) {
      qL[m] = qR[m] = 0.0;
      continue;
    }
    double v0 = P(qi[m], -3), v1 = P(qi[m], -2), v2 = P(qi[m], -1);
    double v3 = P(qi[m], 0), v4 = P(qi[m], 1), v5 = P(qi[m], 2);
    if (SCH == SCHEME_TENO6A)
      teno6a_pair(v0, v1, v2, v3, v4, v5, qL[m], qR[m]);
    else
      weno5_pair(v0, v1, v2, v3, v4, v5, qL[m], qR[m]);
  }
  if (SCH == SCHEME_TENO6A) {
    // interpolation limiter: a side whose reconstructed density or pressure
    // is not positive takes its own cell's primitives (first order)
    if (!(qL[0] > 0.0 && qL[4] > 0.0))
#pragma unroll
      for (int m = 0; m < 5; ++m)
        qL[m] = ((m == 2 && T1 >= NDIM) || (m == 3 && T2 >= NDIM)) ? 0.0 : P(qi[m], -1);
    if (!(qR[0] > 0.0 && qR[4] > 0.0))
#pragma unroll
      for (int m = 0; m < 5; ++m)
        qR[m] = ((m == 2 && T1 >= NDIM) || (m == 3 && T2 >= NDIM)) ? 0.0 : P(qi[m], 0);
  }
  double Fc[5];
  hllc(qL, qR, g.gamma, g.gm1i, Fc);
  G[0] = Fc[0];
  G[1 + D] = Fc[1];
  G[1 + T1] = Fc[2];
  G[1 + T2] = Fc[3];
  G[4] = Fc[4];
  if (VISC && SCH == SCHEME_TENO6A) {
    // Dissipative flux (Eqs. (4)-(5), Fourier's law) from 6th-order central
    // interpolation / differences over the cells at offsets -3 .. 2.
    double vel[3][6], Tc[6], muc[6];
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      vel[0][o] = P(QU, o - 3);
      vel[1][o] = NDIM >= 2 ? P(QV, o - 3) : 0.0;
      vel[2][o] = NDIM >= 3 ? P(QW, o - 3) : 0.0;
      Tc[o] = P(QT, o - 3);
      muc[o] = P(QMU, o - 3);
    }
    const double mfD = g.mf[D][f];
    auto i6 = [](const double *x) { return interp6(x[0], x[1], x[2], x[3], x[4], x[5]); };
    auto d6 = [](const double *x) { return dface6(x[0], x[1], x[2], x[3], x[4], x[5]); };
    double muf = i6(muc);
    double uf[3], dn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uf[c] = i6(vel[c]);
      dn[c] = d6(vel[c]) * mfD;
    }
    double dT = d6(Tc) * mfD;
    double divt = 0.0, dtn[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int tt = r == 0 ? T1 : T2;
      if (tt >= NDIM) continue;
      double gt[6], gn[6];
#pragma unroll
      for (int o = 0; o < 6; ++o) {
        gt[o] = Gv(2 * r, o - 3);
        gn[o] = Gv(2 * r + 1, o - 3);
      }
      divt += i6(gt);
      dtn[tt] = i6(gn);
    }
    double tau[3] = {0.0, 0.0, 0.0};
    tau[D] = muf * ((4.0 / 3.0) * dn[D] - (2.0 / 3.0) * divt);
    if (T1 < NDIM) tau[T1] = muf * (dtn[T1] + dn[T1]);
    if (T2 < NDIM) tau[T2] = muf * (dtn[T2] + dn[T2]);
    double lam = muf * g.cpPr;
    double en = uf[0] * tau[0] + uf[1] * tau[1] + uf[2] * tau[2] + lam * dT;
    G[1] -= tau[0];
    G[2] -= tau[1];
    G[3] -= tau[2];
    G[4] -= en;
  } else if (VISC) {
    // Dissipative flux (Eqs. (4)-(5), Fourier's law) from 4th-order central
    // interpolation / differences over the cells at offsets -2 .. 1.
    double vel[3][4], Tc[4], muc[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      vel[0][o] = P(QU, o - 2);
      vel[1][o] = NDIM >= 2 ? P(QV, o - 2) : 0.0;
      vel[2][o] = NDIM >= 3 ? P(QW, o - 2) : 0.0;
      Tc[o] = P(QT, o - 2);
      muc[o] = P(QMU, o - 2);
    }
    const double mfD = g.mf[D][f];
    double muf = interp4(muc[0], muc[1], muc[2], muc[3]);
    double uf[3], dn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uf[c] = interp4(vel[c][0], vel[c][1], vel[c][2], vel[c][3]);
      dn[c] = dface4(vel[c][0], vel[c][1], vel[c][2], vel[c][3]) * mfD;
    }
    double dT = dface4(Tc[0], Tc[1], Tc[2], Tc[3]) * mfD;
    double divt = 0.0, dtn[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int tt = r == 0 ? T1 : T2;
      if (tt >= NDIM) continue;
      divt += interp4(Gv(2 * r, -2), Gv(2 * r, -1), Gv(2 * r, 0), Gv(2 * r, 1));
      dtn[tt] = interp4(Gv(2 * r + 1, -2), Gv(2 * r + 1, -1), Gv(2 * r + 1, 0), Gv(2 * r + 1, 1));
    }
    double tau[3] = {0.0, 0.0, 0.0};
    tau[D] = muf * ((4.0 / 3.0) * dn[D] - (2.0 / 3.0) * divt);
    if (T1 < NDIM) tau[T1] = muf * (dtn[T1] + dn[T1]);
    if (T2 < NDIM) tau[T2] = muf * (dtn[T2] + dn[T2]);
    double lam = muf * g.cpPr;
    double en = uf[0] * tau[0] + uf[1] * tau[1] + uf[2] * tau[2] + lam * dT;
    G[1] -= tau[0];
    G[2] -= tau[1];
    G[3] -= tau[2];
    G[4] -= en;
  }
}

// LDS slots: primitives rho,u,v,w,p,T,mu then the tangential derivatives.
// LDS slots of a flux tile: the primitives (rho, u, v, w, p, and T, mu when
// viscous), then the 2 (2D) or 4 (3D) cell-centred tangential velocity
// derivatives the dissipative flux needs, computed while staging.
template <int NDIM, bool VISC> struct Slots {
  static constexpr int NP = VISC ? 7 : 5;
  static constexpr int NG = VISC ? 2 * (NDIM - 1) : 0;
  static constexpr int NC = NP + NG;
};

__device__ __forceinline__ int slot_of(int q) { return q; }  // QR..QMU map 1:1

// Staged value of LDS slot `sl` of direction D at box cell b, position p: a
// primitive, or (sl >= NP) the derivative d u_phi / d x_t (slots NP + 2r +
// {0, 1}: t the r-th tangential axis, phi = t, then phi = D), 4th order
// (6th for the TENO6-A scheme) in index space times the analytic metric.  A
// staged cell's tangential positions are interior, so the stencil stays in
// the box (three ghost layers).
template <int NDIM, int D, bool VISC, int SCH>
__device__ __forceinline__ double stage_value(const Dev &g, int sl, long b, const int *p) {
  constexpr int NP = Slots<NDIM, VISC>::NP;
  if (sl < NP) return g.Q[sl][b];  // QR..QMU map 1:1
  constexpr int T1 = tan1(D), T2 = tan2(D);
  const int k = sl - NP, t = (k / 2) == 0 ? T1 : T2;
  const int phi = (k & 1) ? D : t;
  const double *A = g.Q[QU + phi];
  const long st = g.sb[t];
  const double mct = g.mc[t][p[t]];
  if (SCH == SCHEME_TENO6A)
    return dcell6(A[b - 3 * st], A[b - 2 * st], A[b - st], A[b + st], A[b + 2 * st],
                  A[b + 3 * st]) *
           mct;
  return dcell4(A[b - 2 * st], A[b - st], A[b + st], A[b + 2 * st]) * mct;
}

// ---------------------------------------------------------------------------
// x faces: the face index space ((k ny + j) (nx+1) + f) is cut into chunks of
// 256 consecutive faces; a chunk's stencil cells (each row segment widened by
// 3 + 2 cells) are staged in LDS once, then every thread computes one face
// from LDS.  Coalesced loads, one global read per staged value.
// ---------------------------------------------------------------------------
template <int NDIM, bool VISC, int SCH = SCHEME_WENO5>
__device__ __forceinline__ void flux_x_body(const Dev &g, int nwmax, unsigned bid, double *lds) {
  using S = Slots<NDIM, VISC>;
  const int nf = g.n[0] + 1;
  const unsigned total = (unsigned)g.fcount[0];
  const unsigned t0 = bid * 256u;
  const unsigned tl = min(t0 + 255u, total - 1u);
  const unsigned r0 = t0 / nf, f0 = t0 % nf;
  const unsigned rl = tl / nf;
  const int first_len = (nf - (int)f0) + 5;
  const int nw = (int)(tl - t0 + 1) + 5 * (int)(rl - r0 + 1);
  const unsigned ny = g.n[1];
  for (int w = threadIdx.x; w < nw; w += 256) {
    int seg, xc;
    if (w < first_len) {
      seg = 0;
      xc = (int)f0 - 3 + w;
    } else {
      const int q = w - first_len;
      seg = 1 + q / (nf + 5);
      xc = -3 + q % (nf + 5);
    }
    const unsigned r = r0 + seg;
    const int j = (int)(r % ny), k = (int)(r / ny);
    const long bx = bidx(g, xc, j, k);
    const int pc[3] = {xc, j, k};
#pragma unroll
    for (int sl = 0; sl < S::NC; ++sl) {
      if ((sl == QV && NDIM < 2) || (sl == QW && NDIM < 3)) continue;
      lds[sl * nwmax + w] = stage_value<NDIM, 0, VISC, SCH>(g, sl, bx, pc);
    }
  }
  __syncthreads();
  const unsigned t = t0 + threadIdx.x;
  if (t > tl) return;
  const unsigned r = t / nf;
  const int f = (int)(t % nf);
  const int w0 = (int)(t - t0) + 5 * (int)(r - r0) + 3;  // window index of offset 0
  auto P = [&](int q, int o) { return lds[slot_of(q) * nwmax + w0 + o]; };
  auto Gv = [&](int kk, int o) { return lds[(S::NP + kk) * nwmax + w0 + o]; };
  double G[5];
  face_flux<NDIM, 0, VISC, SCH>(g, P, Gv, f, G);
  if (!(fabs(G[0]) + fabs(G[4]) < 1.0e300)) atomicOr(g.flags, 1u);  // non-finite flux
  double *F = g.F[0];
  const long fc = g.fcount[0];
#pragma unroll
  for (int m = 0; m < 5; ++m) F[m * fc + t] = G[m];
}

// Occupancy target of the x / x+y flux launches: 5 waves per SIMD with
// WENO5-JS (no spill; the tiles are bound by per-wave latency, so the extra
// wave pays); the TENO6-A instantiations keep the compiler's own allocation
// (5 waves would spill there).
constexpr int flux_waves(int sch) { return sch == SCHEME_WENO5 ? 5 : 1; }

template <int NDIM, bool VISC, int SCH = SCHEME_WENO5>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(flux_waves(SCH))))
k_flux_x(Dev g, int nwmax) {
  extern __shared__ double lds[];
  flux_x_body<NDIM, VISC, SCH>(g, nwmax, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// y / z faces: 16 (x) x 16 (faces along D) tiles; the tile's 21 cells along D
// by 16 along x are staged in LDS per primitive / derivative.
// ---------------------------------------------------------------------------
template <int NDIM, bool VISC> struct YzTile {
  static constexpr int TX = 16, TD = 16, TR = TD + 5;
  using S = Slots<NDIM, VISC>;
  double lds[S::NC][TR][TX];
};

// Stages the tile's stencil cells (rows f0 - 3 .. f0 + 17 along D, x from
// i0, remaining axis at oc) and computes the flux of face f0 + ty at x
// i0 + tx into G; returns false for a thread outside the grid.
template <int NDIM, int D, bool VISC, int SCH = SCHEME_WENO5>
__device__ __forceinline__ bool yz_tile_face(const Dev &g, YzTile<NDIM, VISC> &T, int i0, int f0,
                                             int oc, double *G) {
  using Tl = YzTile<NDIM, VISC>;
  using S = typename Tl::S;
  constexpr int TX = Tl::TX, TR = Tl::TR;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int nD = g.n[D];
  // oc is the remaining axis' index: z for D = 1, y for D = 2
  for (int idx = threadIdx.x; idx < TR * TX; idx += 256) {
    const int a = idx / TX, x = idx % TX;
    const int i = i0 + x, s = f0 - 3 + a;
    if (i >= g.n[0] || s > nD + 2) continue;
    int p[3];
    p[0] = i;
    p[D] = s;
    p[3 - D] = oc;  // D = 1 -> axis 2, D = 2 -> axis 1
    const long bx = bidx(g, p[0], p[1], p[2]);
#pragma unroll
    for (int sl = 0; sl < S::NC; ++sl) {
      if ((sl == QV && NDIM < 2) || (sl == QW && NDIM < 3)) continue;
      T.lds[sl][a][x] = stage_value<NDIM, D, VISC, SCH>(g, sl, bx, p);
    }
  }
  __syncthreads();
  const int i = i0 + tx, f = f0 + ty;
  if (i >= g.n[0] || f > nD) return false;
  auto P = [&](int q, int o) { return T.lds[slot_of(q)][ty + 3 + o][tx]; };
  auto Gv = [&](int kk, int o) { return T.lds[S::NP + kk][ty + 3 + o][tx]; };
  face_flux<NDIM, D, VISC, SCH>(g, P, Gv, f, G);
  if (!(fabs(G[0]) + fabs(G[4]) < 1.0e300)) atomicOr(g.flags, 1u);  // non-finite flux
  return true;
}

template <int NDIM, int D, bool VISC, int SCH = SCHEME_WENO5>
__device__ __forceinline__ void flux_yz_tile(const Dev &g, YzTile<NDIM, VISC> &T, unsigned lin,
                                             unsigned ntot, unsigned nbx, unsigned nby) {
  // tiles along D are consecutive in the remapped order (they share 5 rows)
  const unsigned lg = xcd_remap(lin, ntot);
  const unsigned by = lg % nby, rest = lg / nby;
  const int i0 = (int)(rest % nbx) * YzTile<NDIM, VISC>::TX, oc = (int)(rest / nbx);
  const int f0 = (int)by * YzTile<NDIM, VISC>::TD;
  double G[5];
  if (!yz_tile_face<NDIM, D, VISC, SCH>(g, T, i0, f0, oc, G)) return;
  int p[3];
  p[0] = i0 + (int)(threadIdx.x % 16);
  p[D] = f0 + (int)(threadIdx.x / 16);
  p[3 - D] = oc;
  const long t = ((long)p[2] * g.fn[D][1] + p[1]) * g.fn[D][0] + p[0];
  double *F = g.F[D];
  const long fc = g.fcount[D];
#pragma unroll
  for (int m = 0; m < 5; ++m) F[m * fc + t] = G[m];
}

template <int NDIM, int D, bool VISC, int SCH = SCHEME_WENO5>
__device__ __forceinline__ void flux_yz_body(const Dev &g, unsigned lin, unsigned ntot,
                                             unsigned nbx, unsigned nby) {
  __shared__ YzTile<NDIM, VISC> T;
  flux_yz_tile<NDIM, D, VISC, SCH>(g, T, lin, ntot, nbx, nby);
}

// x and y faces of a 3D grid in one launch (the two are independent): the
// first ny_tiles workgroups take y tiles, the rest x chunks; both kinds
// share one dynamic LDS buffer.
template <bool VISC, int SCH = SCHEME_WENO5>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(flux_waves(SCH))))
k_flux_xy(Dev g, int nwmax, unsigned ny_tiles, unsigned nbx, unsigned nby, int remap_x) {
  extern __shared__ double lds[];
  if (blockIdx.x < ny_tiles)
    flux_yz_tile<3, 1, VISC, SCH>(g, *reinterpret_cast<YzTile<3, VISC> *>(lds), blockIdx.x,
                                  ny_tiles, nbx, nby);
  else {
    // x chunks: with remap_x in contiguous ranges per XCD (z slabs, as the
    // y tiles and the derivative launch before), so that a chunk finds what
    // that launch left in its XCD's L2; plain order otherwise
    const unsigned c = blockIdx.x - ny_tiles;
    flux_x_body<3, VISC, SCH>(g, nwmax, remap_x ? xcd_remap(c, gridDim.x - ny_tiles) : c, lds);
  }
}

template <int NDIM, int D, bool VISC, int SCH = SCHEME_WENO5>
__global__ void __launch_bounds__(256) k_flux_yz(Dev g) {
  const unsigned nbx = gridDim.x, nby = gridDim.y;
  flux_yz_body<NDIM, D, VISC, SCH>(g, blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z),
                                   nbx * nby * gridDim.z, nbx, nby);
}

// Index of the face left of cell (i, j, k) in direction D's face array.
__device__ __forceinline__ long face_index(const Dev &g, int D, int i, int j, int k) {
  return ((long)k * g.fn[D][1] + j) * g.fn[D][0] + i;
}

__device__ __forceinline__ double cell_volume(const Dev &g, int i, int j, int k) {
  double V = g.dx[0][i];
  if (g.ndim >= 2) V *= g.dx[1][j];
  if (g.ndim >= 3) V *= g.dx[2][k];
  return V;
}

// ---------------------------------------------------------------------------
// Deterministic block reductions (fixed tree for a fixed launch shape).
// ---------------------------------------------------------------------------
template <int NV, int BS = 256>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *sh /*[NV*BS]*/) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NV; ++q) sh[q * BS + t] = v[q];
  __syncthreads();
  for (int w = BS / 2; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int q = 0; q < NV; ++q) sh[q * BS + t] += sh[q * BS + t + w];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = sh[q * BS];
}

// Maximum over a 256-thread workgroup: within each 64-lane wavefront by lane
// exchanges, then over the 4 wavefronts through LDS (sh: 4 doubles).  The
// maximum is exact, so its value does not depend on the order.
__device__ __forceinline__ double block_max(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();  // a previous call's readers of sh are done
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = v;
  __syncthreads();
  return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// Body force, pass 1.  The volume-weighted sum of the unforced x-momentum
// right-hand side, sum_c V_c R_c = -sum_D sum_c A_D (F_D(c+1/2) - F_D(c-1/2))
// with A_D = V_c / dx_D constant along a grid line, telescopes along every
// line to its two boundary faces: -sum_lines A_D (F_D(n) - F_D(0)).  (On a
// periodic axis both boundary faces see the same stencil values, so their
// fluxes are equal and cancel.)  Per-block partial sums of that boundary
// term and of the volume, over one thread per boundary line.
// Directions D >= ndir are skipped (their faces not computed yet; the
// caller guarantees that their boundary terms vanish, as for a periodic
// direction, whose two boundary faces see the same stencil).  The grid and
// the line-to-thread map do not depend on ndir, so the sums are bitwise
// those over every direction.
__global__ void __launch_bounds__(256) k_force_partial(Dev g, double *part, int ndir) {
  __shared__ double sh[2 * 256];
  double v[2] = {0.0, 0.0};
  const int nd = g.ndim;
  long nl[3] = {0, 0, 0}, tot = 0;
  for (int D = 0; D < nd; ++D) {
    nl[D] = (long)g.n[tan1(D)] * g.n[tan2(D)];
    tot += nl[D];
  }
  for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < tot;
       x += (long)gridDim.x * blockDim.x) {
    int D = 0;
    long l = x;
    while (l >= nl[D]) l -= nl[D++];
    if (D >= ndir) continue;
    const int T1 = tan1(D), T2 = tan2(D);
    const int a = (int)(l % g.n[T1]), b = (int)(l / g.n[T1]);
    double A = 1.0;
    if (T1 < nd) A *= g.dx[T1][a];
    if (T2 < nd) A *= g.dx[T2][b];
    // a periodic direction's two boundary fluxes are equal: an exact zero,
    // not read
    if (!(g.bck[2 * D] == BC_PERIODIC && g.bck[2 * D + 1] == BC_PERIODIC)) {
      int p[3];
      p[T1] = a;
      p[T2] = b;
      p[D] = 0;
      const long f0 = ((long)p[2] * g.fn[D][1] + p[1]) * g.fn[D][0] + p[0];
      p[D] = g.n[D];
      const long f1 = ((long)p[2] * g.fn[D][1] + p[1]) * g.fn[D][0] + p[0];
      const double *F = g.F[D] + 1 * g.fcount[D];
      v[0] -= A * (F[f1] - F[f0]);
    }
    if (D == 0) {  // volume: sum over x-lines of A_x * line length
      v[1] += A * g.Lx;
    }
  }
  block_sum<2>(v, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = v[0];
    part[2 * blockIdx.x + 1] = v[1];
  }
}

// x-momentum flux of face f of direction D on the line through p (p[D]
// ignored), evaluated from the primitive box: face_flux with the cells read
// from the box instead of a staged tile (the same operands and arithmetic,
// so the value of the flux kernels bitwise).
template <int NDIM, int D, bool VISC, int SCH>
__device__ __forceinline__ double box_face_xmom_flux(const Dev &g, const int *p, int f) {
  constexpr int NP = Slots<NDIM, VISC>::NP;
  int pc[3] = {p[0], p[1], p[2]};
  pc[D] = f;
  const long b = bidx(g, pc[0], pc[1], pc[2]);
  const long s = g.sb[D];
  auto P = [&](int q, int o) { return g.Q[q][b + o * s]; };
  auto Gv = [&](int kk, int o) {
    int po[3] = {pc[0], pc[1], pc[2]};
    po[D] = f + o;
    return stage_value<NDIM, D, VISC, SCH>(g, NP + kk, b + o * s, po);
  };
  double G[5];
  face_flux<NDIM, D, VISC, SCH>(g, P, Gv, f, G);
  return G[1];
}

// Body force, pass 1, from the primitive box alone (the adjoint's stages
// have no face fluxes): the sums of k_force_partial over every direction,
// with each boundary flux evaluated by box_face_xmom_flux.  A periodic
// direction's two boundary faces see the same stencil values, so its terms
// are exact zeros (not evaluated) and the sums equal k_force_partial's
// bitwise.
template <int NDIM, bool VISC, int SCH>
__global__ void __launch_bounds__(256) k_force_direct(Dev g, double *part) {
  __shared__ double sh[2 * 256];
  double v[2] = {0.0, 0.0};
  long nl[3] = {0, 0, 0}, tot = 0;
  for (int D = 0; D < NDIM; ++D) {
    nl[D] = (long)g.n[tan1(D)] * g.n[tan2(D)];
    tot += nl[D];
  }
  for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < tot;
       x += (long)gridDim.x * blockDim.x) {
    int D = 0;
    long l = x;
    while (l >= nl[D]) l -= nl[D++];
    const int T1 = tan1(D), T2 = tan2(D);
    const int a = (int)(l % g.n[T1]), b = (int)(l / g.n[T1]);
    double A = 1.0;
    if (T1 < NDIM) A *= g.dx[T1][a];
    if (T2 < NDIM) A *= g.dx[T2][b];
    int p[3] = {0, 0, 0};
    p[T1] = a;
    p[T2] = b;
    double F0 = 0.0, F1 = 0.0;
    if (g.bck[2 * D] == BC_PERIODIC && g.bck[2 * D + 1] == BC_PERIODIC) {
      // equal fluxes: an exact zero either way, not evaluated
    } else if (D == 0) {
      F0 = box_face_xmom_flux<NDIM, 0, VISC, SCH>(g, p, 0);
      F1 = box_face_xmom_flux<NDIM, 0, VISC, SCH>(g, p, g.n[0]);
    } else if (NDIM >= 2 && D == 1) {
      F0 = box_face_xmom_flux<NDIM, NDIM >= 2 ? 1 : 0, VISC, SCH>(g, p, 0);
      F1 = box_face_xmom_flux<NDIM, NDIM >= 2 ? 1 : 0, VISC, SCH>(g, p, g.n[1]);
    } else if (NDIM >= 3) {
      F0 = box_face_xmom_flux<NDIM, NDIM >= 3 ? 2 : 0, VISC, SCH>(g, p, 0);
      F1 = box_face_xmom_flux<NDIM, NDIM >= 3 ? 2 : 0, VISC, SCH>(g, p, g.n[2]);
    }
    v[0] -= A * (F1 - F0);
    if (D == 0) {  // volume: sum over x-lines of A_x * line length
      v[1] += A * g.Lx;
    }
  }
  block_sum<2>(v, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = v[0];
    part[2 * blockIdx.x + 1] = v[1];
  }
}

// Body force, pass 2: f = -sum(V R_rhou)/sum(V).
__global__ void __launch_bounds__(256) k_force_final(const double *part, int nparts, double *f) {
  __shared__ double sh[2 * 256];
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += 256) {
    v[0] += part[2 * b];
    v[1] += part[2 * b + 1];
  }
  block_sum<2>(v, sh);
  if (threadIdx.x == 0) f[0] = -v[0] / v[1];
}

// Signal rate of one cell, sum_d (|u_d| + c)/dx_d + 2 nu_eff sum_d 1/dx_d^2
// (nu_eff = max(4/3, gamma/Pr) mu/rho); dt = cfl / max over cells.
__device__ __forceinline__ double cell_sigma(const Dev &g, const double *q, const int *pos) {
  double y;  // 1 / (rho cs)
  double cs = sound_speed(g.gamma, q[QR], q[QP], y);
  double conv = 0.0, inv2 = 0.0;
  for (int d = 0; d < g.ndim; ++d) {
    double id = g.idx[d][pos[d]];
    conv += (fabs(q[QU + d]) + cs) * id;
    inv2 += id * id;
  }
  double sig = conv;
  if (g.visc != VISC_NONE) {
    double mu = viscosity(g, q[QT]);
    double nu = fmax(4.0 / 3.0, g.gamma / g.Pr) * mu * (cs * y);  // mu / rho
    sig += 2.0 * nu * inv2;
  }
  if (!(sig < 1.0e300)) sig = 1.0e300;  // non-finite: flagged elsewhere
  return sig;
}

// ---------------------------------------------------------------------------
// Divergence of the face fluxes (Eq. (6)) plus the source, fused with the
// TVD-RK3 stage: Uout = a*Un + b*(Uin + dt*R).  With Rout != nullptr the
// kernel writes R instead (rhs evaluation).
// ---------------------------------------------------------------------------
// R_m -= (F_D(c+1/2) - F_D(c-1/2)) / dx_D for the directions D < upto,
// fluxes read from the face arrays (Eq. (6), the divergence).
__device__ __forceinline__ void flux_divergence(const Dev &g, int i, int j, int k, int upto,
                                                double *R) {
  for (int D = 0; D < upto; ++D) {
    long fl = face_index(g, D, i, j, k);
    long fr = fl + (D == 0 ? 1 : (D == 1 ? g.fn[1][0] : (long)g.fn[2][0] * g.fn[2][1]));
    int pos = D == 0 ? i : (D == 1 ? j : k);
    double id = g.idx[D][pos];
    const double *F = g.F[D];
    const long fc = g.fcount[D];
#pragma unroll
    for (int m = 0; m < 5; ++m) R[m] -= (F[m * fc + fr] - F[m * fc + fl]) * id;
  }
}

// The inputs of one cell's stage update: Un, Uin, dt and, with the body
// force, the force and the cell's velocity.  They are loaded together, before
// any store: Un or Uin may be Uout itself, so the compiler could not move a
// later component's loads above an earlier component's store, and each
// component would wait a full memory round trip.  (Issuing them before the
// face fluxes of the divergence as well measured no faster.)
template <int NDIM> struct CellIn {
  double un[NDIM + 2], ui[NDIM + 2], dt, f, u;
};

template <int NDIM>
__device__ __forceinline__ void load_cell(const Dev &g, const double *Un, const double *Uin,
                                          const double *dtp, const double *force, long c, int i,
                                          int j, int k, CellIn<NDIM> &in) {
  const long nc = g.ncell;
#pragma unroll
  for (int v = 0; v < NDIM + 2; ++v) {
    in.un[v] = Un[v * nc + c];
    in.ui[v] = Uin[v * nc + c];
  }
  in.dt = dtp[0];
  in.f = in.u = 0.0;
  if (g.source == SRC_MASSFLUX) {
    in.f = force[0];
    in.u = g.Q[QU][bidx(g, i, j, k)];
  }
}

// Source, then Uout = a Un + b (Uin + dt R) for cell c of an NDIM grid; the
// new state (rho, the three momenta, E; zeros for the unused ones) is left
// in st.
template <int NDIM>
__device__ __forceinline__ void stage_apply_t(const Dev &g, const CellIn<NDIM> &in, double *Uout,
                                              double a, double bcoef, long c, double *R,
                                              double *st) {
  constexpr int NV = NDIM + 2;
  if (g.source == SRC_MASSFLUX) {
    R[1] += in.f;
    R[4] += in.f * in.u;
  }
  const long nc = g.ncell;
  // conserved component v <- flux entry m
  double Rv[NV];
  Rv[0] = R[0];
  Rv[1] = R[1];
  if (NDIM >= 2) Rv[2] = R[2];
  if (NDIM >= 3) Rv[3] = R[3];
  Rv[NV - 1] = R[4];
#pragma unroll
  for (int v = 0; v < 5; ++v) st[v] = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double uo = a * in.un[v] + bcoef * (in.ui[v] + in.dt * Rv[v]);
    Uout[v * nc + c] = uo;
    st[v == NV - 1 ? 4 : v] = uo;
  }
}

// One cell's divergence + source + stage update of an NDIM grid (no barrier
// inside); returns the new state's signal rate when want_sigma.
template <int NDIM>
__device__ __forceinline__ double update_cell_t(const Dev &g, const double *Un, const double *Uin,
                                                double *Uout, const double *dtp, double a,
                                                double bcoef, const double *force, long c,
                                                int i, int j, int k, bool want_sigma) {
  double R[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  flux_divergence(g, i, j, k, NDIM, R);
  CellIn<NDIM> in;
  load_cell<NDIM>(g, Un, Uin, dtp, force, c, i, j, k, in);
  double st[5];
  stage_apply_t<NDIM>(g, in, Uout, a, bcoef, c, R, st);
  if (!want_sigma) return 0.0;
  double q[6];
  prim_of_state(g, st, q);
  const int pos[3] = {i, j, k};
  return cell_sigma(g, q, pos);
}

// One cell's divergence + source + stage update (or R itself into Rout).
__device__ __forceinline__ double update_cell(const Dev &g, const double *Un, const double *Uin,
                                              double *Uout, double *Rout, const double *dtp,
                                              double a, double bcoef, const double *force,
                                              unsigned cu, bool want_sigma) {
  const unsigned n0 = g.n[0], n01 = n0 * (unsigned)g.n[1];
  const int k = (int)(cu / n01), j = (int)((cu % n01) / n0), i = (int)(cu % n0);
  const int nd = g.ndim;
  const long c = (long)cu;
  if (!Rout) {
    if (nd == 3) return update_cell_t<3>(g, Un, Uin, Uout, dtp, a, bcoef, force, c, i, j, k,
                                         want_sigma);
    if (nd == 2) return update_cell_t<2>(g, Un, Uin, Uout, dtp, a, bcoef, force, c, i, j, k,
                                         want_sigma);
    return update_cell_t<1>(g, Un, Uin, Uout, dtp, a, bcoef, force, c, i, j, k, want_sigma);
  }
  double R[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  flux_divergence(g, i, j, k, nd, R);
  if (g.source == SRC_MASSFLUX) {
    double f = force[0];
    long b = bidx(g, i, j, k);
    R[1] += f;
    R[4] += f * g.Q[QU][b];
  }
  const long nc = g.ncell;
  double Rv[5];
  Rv[0] = R[0];
  Rv[1] = R[1];
  if (nd >= 2) Rv[2] = R[2];
  if (nd >= 3) Rv[3] = R[3];
  Rv[nd + 1] = R[4];
  for (int v = 0; v < nd + 2; ++v) Rout[v * nc + c] = Rv[v];
  return 0.0;
}

// With dtpart (uniform over the launch) every thread of the block reaches
// the block reduction of the new state's signal rates (the CFL step of the
// next step); the barrier sits outside any branch on the thread's cell.
__device__ __forceinline__ void update_body(const Dev &g, const double *Un, const double *Uin,
                                            double *Uout, double *Rout, const double *dtp,
                                            double a, double bcoef, const double *force,
                                            unsigned cu, double *dtpart = nullptr) {
  double sig = 0.0;
  if (cu < (unsigned)g.ncell)  // ncell < 2^31
    sig = update_cell(g, Un, Uin, Uout, Rout, dtp, a, bcoef, force, cu, dtpart != nullptr);
  if (dtpart) {
    __shared__ double shx[4];
    const double m = block_max(sig, shx);
    if (threadIdx.x == 0) dtpart[blockIdx.x] = m;
  }
}

__global__ void __launch_bounds__(256) k_update(Dev g, const double *Un, const double *Uin,
                                                double *Uout, double *Rout, const double *dtp,
                                                double a, double bcoef, const double *force,
                                                double *dtpart) {
  update_body(g, Un, Uin, Uout, Rout, dtp, a, bcoef, force, blockIdx.x * blockDim.x + threadIdx.x,
              dtpart);
}

// ---------------------------------------------------------------------------
// Faces of the last direction fused with the stage update (no source term):
// 16 x 16 face tiles advance by 15 cells along D, so the 15 cells between a
// tile's faces get their whole divergence, the last direction's fluxes from
// LDS and the other directions' from the face arrays.  The face values and
// the order of the sums are those of k_flux_yz + k_update.
// ---------------------------------------------------------------------------
template <int NDIM, int D, bool VISC, int SCH = SCHEME_WENO5>
__device__ __forceinline__ void flux_update_body(const Dev &g, unsigned lin, unsigned ntot,
                                                 unsigned nbx, unsigned nby, const double *Un,
                                                 const double *Uin, double *Uout,
                                                 const double *dtp, double a, double bcoef,
                                                 double *dtpart, unsigned bid,
                                                 BoxOut qo = BoxOut{},
                                                 const double *force = nullptr) {
  using Tl = YzTile<NDIM, VISC>;
  __shared__ Tl T;
  const unsigned lg = xcd_remap(lin, ntot);
  const unsigned by = lg % nby, rest = lg / nby;
  const int i0 = (int)(rest % nbx) * Tl::TX, oc = (int)(rest / nbx);
  const int f0 = (int)by * (Tl::TD - 1);
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double G[5];
  const bool valid = yz_tile_face<NDIM, D, VISC, SCH>(g, T, i0, f0, oc, G);
  __syncthreads();  // the staged stencil is no longer read: reuse it for the faces
  double(*fl)[16][16] = reinterpret_cast<double(*)[16][16]>(&T.lds[0][0][0]);
  if (valid)
#pragma unroll
    for (int m = 0; m < 5; ++m) fl[m][ty][tx] = G[m];
  __syncthreads();
  double sig = 0.0;
  const int i = i0 + tx, cD = f0 + ty;
  if (ty < Tl::TD - 1 && i < g.n[0] && cD < g.n[D]) {
    int p[3];
    p[0] = i;
    p[D] = cD;
    p[3 - D] = oc;
    if (NDIM == 2) p[2] = 0;
    const long c = ((long)p[2] * g.n[1] + p[1]) * g.n[0] + p[0];
    double R[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    flux_divergence(g, p[0], p[1], p[2], D, R);
    const double id = g.idx[D][cD];
#pragma unroll
    for (int m = 0; m < 5; ++m) R[m] -= (fl[m][ty + 1][tx] - fl[m][ty][tx]) * id;
    CellIn<NDIM> in;
    load_cell<NDIM>(g, Un, Uin, dtp, force, c, p[0], p[1], p[2], in);
    double st[5];
    stage_apply_t<NDIM>(g, in, Uout, a, bcoef, c, R, st);
    double q[6];
    if (dtpart || qo.Q[0]) prim_of_state(g, st, q);  // the new state's primitives
    if (dtpart) sig = cell_sigma(g, q, p);
    if (qo.Q[0]) {
      // the new state's primitives (the values just stored, converted as
      // k_prim_interior converts them) into the next stage's box
      if (!(finite_pos(q[QR]) && finite_pos(q[QP]))) atomicOr(g.flags, 1u);
      const long bx = bidx(g, p[0], p[1], p[2]);
      qo.Q[QR][bx] = q[QR];
      qo.Q[QU][bx] = q[QU];
      qo.Q[QV][bx] = q[QV];
      if (NDIM >= 3) qo.Q[QW][bx] = q[QW];
      qo.Q[QP][bx] = q[QP];
      if (VISC) {
        qo.Q[QT][bx] = q[QT];
        qo.Q[QMU][bx] = viscosity(g, q[QT]);
      }
    }
  }
  if (dtpart) {
    __shared__ double shx[4];
    const double m = block_max(sig, shx);
    if (threadIdx.x == 0) dtpart[bid] = m;
  }
}

template <int NDIM, bool VISC, int SCH = SCHEME_WENO5>
__global__ void __launch_bounds__(256) k_flux_update(Dev g, const double *Un, const double *Uin,
                                                     double *Uout, const double *dtp, double a,
                                                     double bcoef, double *dtpart, BoxOut qo,
                                                     const double *force) {
  constexpr int D = NDIM - 1;
  const unsigned nbx = gridDim.x, nby = gridDim.y;
  const unsigned lin = blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z);
  flux_update_body<NDIM, D, VISC, SCH>(g, lin, nbx * nby * gridDim.z, nbx, nby, Un, Uin, Uout,
                                       dtp, a, bcoef, dtpart, lin, qo, force);
}

// ---------------------------------------------------------------------------
// CFL time step: dt = min(dt_max, cfl / max_cells sigma).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dt_partial_body(const Dev &g, const double *U, double *part,
                                                unsigned bid, unsigned nblk) {
  __shared__ double sh[4];
  double smax = 0.0;
  for (long c = (long)bid * blockDim.x + threadIdx.x; c < g.ncell;
       c += (long)nblk * blockDim.x) {
    int pos[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]),
                  (int)(c / ((long)g.n[0] * g.n[1]))};
    double q[6];
    cons_to_prim(g, U, c, q);
    smax = fmax(smax, cell_sigma(g, q, pos));
  }
  smax = block_max(smax, sh);
  if (threadIdx.x == 0) part[bid] = smax;
}

__global__ void __launch_bounds__(256) k_dt_partial(Dev g, const double *U, double *part) {
  dt_partial_body(g, U, part, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void dt_final_body(const double *part, int nparts, double cfl,
                                              double dt_max, double *dt) {
  __shared__ double sh[4];
  double m = 0.0;
  int b = threadIdx.x;
  // 8 partials per thread loaded before they are combined (the same
  // sequence of maxima per thread as one at a time)
  for (; b + 7 * 256 < nparts; b += 8 * 256) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = part[b + u * 256];
#pragma unroll
    for (int u = 0; u < 8; ++u) m = fmax(m, t[u]);
  }
  for (; b < nparts; b += 256) m = fmax(m, part[b]);
  m = block_max(m, sh);
  if (threadIdx.x == 0) dt[0] = fmin(dt_max, cfl / m);
}

__global__ void __launch_bounds__(256) k_dt_final(const double *part, int nparts, double cfl,
                                                  double dt_max, double *dt) {
  dt_final_body(part, nparts, cfl, dt_max, dt);
}

// Ghost fill of a primitive box together with the CFL step reduction of the
// update before it, as workgroup 0 (its partial maxima are complete when the
// launch starts, and only later launches read the step).  Saves the launch
// of a one-workgroup kernel per step.
__global__ void __launch_bounds__(256) k_prim_ghost_dt(Dev g, const double *part, int nparts,
                                                       double cfl, double dt_max, double *dt) {
  if (blockIdx.x == 0) {
    dt_final_body(part, nparts, cfl, dt_max, dt);
    return;
  }
  prim_ghost_body(g, (blockIdx.x - 1) * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Diagnostics: volume means of kinetic energy and mu |omega|^2, and the
// conserved totals.  Needs the primitive box (vorticity from 4th-order
// cell-centred differences).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_diag_partial(Dev g, const double *U, double *part) {
  __shared__ double sh[8 * 256];
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long nc = g.ncell;
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < nc;
       c += (long)gridDim.x * blockDim.x) {
    int i = (int)(c % g.n[0]), j = (int)((c / g.n[0]) % g.n[1]),
        k = (int)(c / ((long)g.n[0] * g.n[1]));
    double V = cell_volume(g, i, j, k);
    long b = bidx(g, i, j, k);
    double rho = g.Q[QR][b], u = g.Q[QU][b];
    double vv = g.ndim >= 2 ? g.Q[QV][b] : 0.0, w = g.ndim >= 3 ? g.Q[QW][b] : 0.0;
    v[0] += V * 0.5 * rho * (u * u + vv * vv + w * w);
    if (g.ndim == 3) {
      int pos[3] = {i, j, k};
      auto D = [&](int q, int t) {
        const double *A = g.Q[q];
        long st = g.sb[t];
        return dcell4(A[b - 2 * st], A[b - st], A[b + st], A[b + 2 * st]) * g.mc[t][pos[t]];
      };
      double wx = D(QW, 1) - D(QV, 2);
      double wy = D(QU, 2) - D(QW, 0);
      double wz = D(QV, 0) - D(QU, 1);
      double mu = g.visc != VISC_NONE ? g.Q[QMU][b] : 0.0;
      v[1] += V * mu * (wx * wx + wy * wy + wz * wz);
    }
    v[2] += V * U[c];
    v[3] += V * U[nc + c];
    if (g.ndim >= 2) v[4] += V * U[2 * nc + c];
    if (g.ndim >= 3) v[5] += V * U[3 * nc + c];
    v[6] += V * U[(long)(g.ndim + 1) * nc + c];
    v[7] += V;
  }
  block_sum<8>(v, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q < 8; ++q) part[8 * blockIdx.x + q] = v[q];
}

__global__ void __launch_bounds__(256) k_diag_final(const double *part, int nparts, double *out) {
  __shared__ double sh[8 * 256];
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nparts; b += 256)
    for (int q = 0; q < 8; ++q) v[q] += part[8 * b + q];
  block_sum<8>(v, sh);
  if (threadIdx.x == 0) {
    out[0] = v[0] / v[7];
    out[1] = v[1] / v[7];
    for (int q = 2; q < 8; ++q) out[q] = v[q];
  }
}

// ---------------------------------------------------------------------------
// Wall-pressure cost term j(U) = sum_i (A_i/A)(p_i - p_ref)^2 over the cells
// next to the cost face, accumulated as J += w j; optional gradient
// g += w dj/dU.  One block; the face has O(n^2) cells.
// ---------------------------------------------------------------------------
// Wall-pressure cost term and its gradient: one block of 1024 threads, one
// wall face per thread and round (fixed reduction order: deterministic).
__global__ void __launch_bounds__(1024) k_cost(Dev g, int face, double pref, const double *U,
                                               double w, double *J, double *grad) {
  constexpr int BS = 1024;
  __shared__ double sh[2 * BS];
  const int d = face / 2, side = face % 2;
  const int t1 = tan1(d), t2 = tan2(d);
  const unsigned na = g.n[t1];
  const unsigned nface = na * (unsigned)g.n[t2];
  const int nd = g.ndim;
  const long nc = g.ncell;
  auto cell_of = [&](unsigned x, double &A) {
    const int a = (int)(x % na), bb = (int)(x / na);
    A = 1.0;
    if (t1 < nd) A *= g.dx[t1][a];
    if (t2 < nd) A *= g.dx[t2][bb];
    int p[3];
    p[d] = side == 0 ? 0 : g.n[d] - 1;
    p[t1] = a;
    p[t2] = bb;
    return ((long)p[2] * g.n[1] + p[1]) * g.n[0] + p[0];
  };
  // total area (fixed order), then the weighted sum
  double v[2] = {0.0, 0.0};
  for (unsigned x = threadIdx.x; x < nface; x += BS) {
    double A, q[6];
    cons_to_prim(g, U, cell_of(x, A), q);
    double dp = q[QP] - pref;
    v[0] += A * dp * dp;
    v[1] += A;
  }
  block_sum<2, BS>(v, sh);
  const double area = v[1];
  if (threadIdx.x == 0) J[0] += w * (v[0] / area);
  if (!grad) return;
  for (unsigned x = threadIdx.x; x < nface; x += BS) {
    double A;
    const long c = cell_of(x, A);
    double q[6];
    cons_to_prim(g, U, c, q);
    double s = w * (A / area) * 2.0 * (q[QP] - pref) * (g.gamma - 1.0);
    // p = (gamma-1)(E - |m|^2/(2 rho)): dp/drho = (gamma-1)|u|^2/2,
    // dp/dm_i = -(gamma-1) u_i, dp/dE = gamma-1
    double ke = 0.5 * (q[QU] * q[QU] + q[QV] * q[QV] + q[QW] * q[QW]);
    grad[c] += s * ke;
    grad[nc + c] -= s * q[QU];
    if (nd >= 2) grad[2 * nc + c] -= s * q[QV];
    if (nd >= 3) grad[3 * nc + c] -= s * q[QW];
    grad[(long)(nd + 1) * nc + c] += s;
  }
}

}  // namespace dcf

// ---------------------------------------------------------------------------
// Small elementwise helpers (fills and copies as kernels, so that a captured
// graph holds no memset or memcpy nodes).
// ---------------------------------------------------------------------------
namespace dcf {

__global__ void k_fill(double *p, double v, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = v;
}
// 16-byte stores for a 16-byte aligned array (the last element separately).
__global__ void k_fill2(double2 *p, double v, long n2, double *tail) {
  const double2 vv = make_double2(v, v);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x)
    p[i] = vv;
  if (tail && blockIdx.x == 0 && threadIdx.x == 0) *tail = v;
}
__global__ void k_copy(double *dst, const double *src, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
__global__ void k_axpy(double *y, double a, const double *x, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}

static inline unsigned grid_for(long n, int bs = 256) {
  long b = (n + bs - 1) / bs;
  return (unsigned)(b < 1 ? 1 : b);
}
static inline unsigned grid_capped(long n, int cap) {
  long b = (n + 255) / 256;
  if (b > cap) b = cap;
  return (unsigned)(b < 1 ? 1 : b);
}

hipError_t launch_fill(double *p, double v, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if ((((uintptr_t)p) & 15) == 0 && n >= 2)
    k_fill2<<<grid_capped(n / 2, 4096), 256, 0, st>>>((double2 *)p, v, n / 2,
                                                       (n & 1) ? p + n - 1 : nullptr);
  else
    k_fill<<<grid_capped(n, 4096), 256, 0, st>>>(p, v, n);
  return hipGetLastError();
}
hipError_t launch_copy(double *dst, const double *src, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_copy<<<grid_capped(n, 4096), 256, 0, st>>>(dst, src, n);
  return hipGetLastError();
}
hipError_t launch_axpy(double *y, double a, const double *x, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_axpy<<<grid_capped(n, 4096), 256, 0, st>>>(y, a, x, n);
  return hipGetLastError();
}

hipError_t launch_line_length(const double *dx, int n, double *out, hipStream_t st) {
  k_line_length<<<1, 1, 0, st>>>(dx, n, out);
  return hipGetLastError();
}
hipError_t launch_metrics(int kind, double lo, double hi, double beta, int n, double *dx,
                          double *idx, double *mc, double *mf, double *xm, hipStream_t st) {
  k_metrics<<<grid_for(n + 1), 256, 0, st>>>(kind, lo, hi, beta, n, dx, idx, mc, mf, xm);
  return hipGetLastError();
}
hipError_t launch_init_state(const Dev &g, const double *P, double *U, hipStream_t st) {
  k_init_state<<<grid_for(g.ncell), 256, 0, st>>>(g, P, U);
  return hipGetLastError();
}
hipError_t launch_prim_halo(const Dev &g, const double *U, hipStream_t st) {
  // few ghost cells: one launch; otherwise interior first, then the ghosts
  // copied from it (a second launch costs less than ghost threads that
  // convert their source state themselves)
  if ((g.nbox - g.ncell) * 10 <= g.nbox) {
    k_prim_halo<<<grid_for(g.nbox), 256, 0, st>>>(g, U);
  } else {
    k_prim_interior<<<grid_for(g.ncell), 256, 0, st>>>(g, U);
    k_prim_ghost<<<grid_for(g.nbox - g.ncell), 256, 0, st>>>(g);
  }
  return hipGetLastError();
}
static int x_window(const Dev &g) {
  const int nf = g.n[0] + 1;
  return 256 + 5 * ((255 + nf - 1) / nf + 1);
}

template <int NDIM, bool VISC>
static hipError_t launch_x(const Dev &g, hipStream_t st) {
  const int nw = x_window(g);
  const size_t shm = sizeof(double) * Slots<NDIM, VISC>::NC * nw;
  if (g.scheme == SCHEME_TENO6A)
    k_flux_x<NDIM, VISC, SCHEME_TENO6A><<<grid_for(g.fcount[0]), 256, shm, st>>>(g, nw);
  else
    k_flux_x<NDIM, VISC><<<grid_for(g.fcount[0]), 256, shm, st>>>(g, nw);
  return hipGetLastError();
}

template <bool VISC>
static hipError_t launch_xy(const Dev &g, hipStream_t st) {
  const int nw = x_window(g);
  const size_t shm = std::max(sizeof(double) * Slots<3, VISC>::NC * nw, sizeof(YzTile<3, VISC>));
  const unsigned nbx = (g.n[0] + 15) / 16, nby = (g.n[1] + 1 + 15) / 16;
  const unsigned ny_tiles = nbx * nby * (unsigned)g.n[2];
  // XCD-contiguous x chunks pay when the box's primitives and derivatives fit
  // in the 256 MB Infinity Cache (TGV 64^3: +1.3 % per step); on larger boxes
  // the plain order measured faster (channel 192x128x128: -0.5 % with it)
  const int remap_x = (double)g.nboxp * 8.0 * (NQ + 9) < 256.0 * 1024.0 * 1024.0;
  if (g.scheme == SCHEME_TENO6A)
    k_flux_xy<VISC, SCHEME_TENO6A><<<ny_tiles + grid_for(g.fcount[0]), 256, shm, st>>>(
        g, nw, ny_tiles, nbx, nby, remap_x);
  else
    k_flux_xy<VISC><<<ny_tiles + grid_for(g.fcount[0]), 256, shm, st>>>(g, nw, ny_tiles, nbx,
                                                                          nby, remap_x);
  return hipGetLastError();
}

hipError_t launch_flux_xy(const Dev &g, hipStream_t st) {
  if (g.ndim != 3) return hipErrorInvalidValue;
  return g.visc != VISC_NONE ? launch_xy<true>(g, st) : launch_xy<false>(g, st);
}

template <int NDIM, int D, bool VISC>
static hipError_t launch_yz(const Dev &g, hipStream_t st) {
  dim3 grid((g.n[0] + 15) / 16, (g.n[D] + 1 + 15) / 16, D == 1 ? g.n[2] : g.n[1]);
  if (g.scheme == SCHEME_TENO6A)
    k_flux_yz<NDIM, D, VISC, SCHEME_TENO6A><<<grid, 256, 0, st>>>(g);
  else
    k_flux_yz<NDIM, D, VISC><<<grid, 256, 0, st>>>(g);
  return hipGetLastError();
}

template <int NDIM, bool VISC>
static hipError_t launch_fu(const Dev &g, const double *Un, const double *Uin, double *Uout,
                            const double *dt, double a, double b, double *dtpart,
                            const BoxOut &qo, const double *force, hipStream_t st) {
  constexpr int D = NDIM - 1;
  dim3 grid((g.n[0] + 15) / 16, (g.n[D] + 14) / 15, D == 1 ? g.n[2] : g.n[1]);
  if (g.scheme == SCHEME_TENO6A)
    k_flux_update<NDIM, VISC, SCHEME_TENO6A><<<grid, 256, 0, st>>>(g, Un, Uin, Uout, dt, a, b,
                                                                   dtpart, qo, force);
  else
    k_flux_update<NDIM, VISC><<<grid, 256, 0, st>>>(g, Un, Uin, Uout, dt, a, b, dtpart, qo,
                                                    force);
  return hipGetLastError();
}

unsigned flux_update_blocks(const Dev &g) {
  if (g.ndim < 2) return 0;
  const int D = g.ndim - 1;
  return (unsigned)((g.n[0] + 15) / 16) * (unsigned)((g.n[D] + 14) / 15) *
         (unsigned)(D == 1 ? g.n[2] : g.n[1]);
}

hipError_t launch_flux_update_last(const Dev &g, const double *Un, const double *Uin,
                                   double *Uout, const double *dt, double a, double b,
                                   double *dtpart, hipStream_t st, const BoxOut &qo,
                                   const double *force) {
  const bool v = g.visc != VISC_NONE;
  if (g.ndim == 2)
    return v ? launch_fu<2, true>(g, Un, Uin, Uout, dt, a, b, dtpart, qo, force, st)
             : launch_fu<2, false>(g, Un, Uin, Uout, dt, a, b, dtpart, qo, force, st);
  if (g.ndim == 3)
    return v ? launch_fu<3, true>(g, Un, Uin, Uout, dt, a, b, dtpart, qo, force, st)
             : launch_fu<3, false>(g, Un, Uin, Uout, dt, a, b, dtpart, qo, force, st);
  return hipErrorInvalidValue;
}

hipError_t launch_fluxes_update(const Dev &g, const double *Un, const double *Uin,
                                double *Uout, const double *dt, double a, double b,
                                double *dtpart, hipStream_t st, const BoxOut &qo,
                                double *part, double *force, Probe *pr) {
  Probe none;
  Probe &p = pr ? *pr : none;
  const int w = g.ndim == 3 ? 7 : 1;
  p.before(w, st);
  hipError_t e = g.ndim == 3 ? launch_flux_xy(g, st) : launch_flux_dir(g, 0, st);
  p.after(w, st);
  // the body force from the boundary fluxes of the directions before the
  // last (the last one is periodic: its boundary terms vanish)
  if (e == hipSuccess && force) e = launch_force(g, part, force, st, g.ndim - 1);
  if (e != hipSuccess) return e;
  p.before(6, st);
  e = launch_flux_update_last(g, Un, Uin, Uout, dt, a, b, dtpart, st, qo, force);
  p.after(6, st);
  return e;
}

hipError_t launch_prim_ghost(const Dev &g, hipStream_t st) {
  if (g.nbox > g.ncell) k_prim_ghost<<<grid_for(g.nbox - g.ncell), 256, 0, st>>>(g);
  return hipGetLastError();
}

hipError_t launch_flux_dir(const Dev &g, int D, hipStream_t st) {
  const bool v = g.visc != VISC_NONE;
  switch (g.ndim * 10 + D) {
    case 10: return v ? launch_x<1, true>(g, st) : launch_x<1, false>(g, st);
    case 20: return v ? launch_x<2, true>(g, st) : launch_x<2, false>(g, st);
    case 21: return v ? launch_yz<2, 1, true>(g, st) : launch_yz<2, 1, false>(g, st);
    case 30: return v ? launch_x<3, true>(g, st) : launch_x<3, false>(g, st);
    case 31: return v ? launch_yz<3, 1, true>(g, st) : launch_yz<3, 1, false>(g, st);
    case 32: return v ? launch_yz<3, 2, true>(g, st) : launch_yz<3, 2, false>(g, st);
  }
  return hipErrorInvalidValue;
}
hipError_t launch_fluxes(const Dev &g, hipStream_t st) {
  hipError_t e;
  if (g.ndim == 3) {
    e = launch_flux_xy(g, st);
    return e != hipSuccess ? e : launch_flux_dir(g, 2, st);
  }
  for (int D = 0; D < g.ndim; ++D) {
    e = launch_flux_dir(g, D, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t launch_force(const Dev &g, double *part, double *force, hipStream_t st, int ndir) {
  long lines = 0;
  for (int D = 0; D < g.ndim; ++D) lines += (long)g.n[tan1(D)] * g.n[tan2(D)];
  unsigned nb = grid_capped(lines, RED_BLOCKS);
  k_force_partial<<<nb, 256, 0, st>>>(g, part, ndir < 0 ? g.ndim : ndir);
  k_force_final<<<1, 256, 0, st>>>(part, (int)nb, force);
  return hipGetLastError();
}
template <int NDIM, bool VISC>
static void launch_force_direct_t(const Dev &g, unsigned nb, double *part, hipStream_t st) {
  if (g.scheme == SCHEME_TENO6A)
    k_force_direct<NDIM, VISC, SCHEME_TENO6A><<<nb, 256, 0, st>>>(g, part);
  else
    k_force_direct<NDIM, VISC, SCHEME_WENO5><<<nb, 256, 0, st>>>(g, part);
}
hipError_t launch_force_direct(const Dev &g, double *part, double *force, hipStream_t st) {
  long lines = 0;
  for (int D = 0; D < g.ndim; ++D) lines += (long)g.n[tan1(D)] * g.n[tan2(D)];
  const unsigned nb = grid_capped(lines, RED_BLOCKS);
  const bool v = g.visc != VISC_NONE;
  switch (g.ndim) {
    case 1: v ? launch_force_direct_t<1, true>(g, nb, part, st)
              : launch_force_direct_t<1, false>(g, nb, part, st); break;
    case 2: v ? launch_force_direct_t<2, true>(g, nb, part, st)
              : launch_force_direct_t<2, false>(g, nb, part, st); break;
    default: v ? launch_force_direct_t<3, true>(g, nb, part, st)
               : launch_force_direct_t<3, false>(g, nb, part, st); break;
  }
  k_force_final<<<1, 256, 0, st>>>(part, (int)nb, force);
  return hipGetLastError();
}
hipError_t launch_update(const Dev &g, const double *Un, const double *Uin, double *Uout,
                         double *Rout, const double *dt, double a, double b,
                         const double *force, hipStream_t st, double *dtpart) {
  k_update<<<grid_for(g.ncell), 256, 0, st>>>(g, Un, Uin, Uout, Rout, dt, a, b, force, dtpart);
  return hipGetLastError();
}
unsigned update_blocks(const Dev &g) { return grid_for(g.ncell); }
hipError_t launch_dt_final(const double *part, int nparts, double cfl, double dt_max, double *dt,
                           hipStream_t st) {
  k_dt_final<<<1, 256, 0, st>>>(part, nparts, cfl, dt_max, dt);
  return hipGetLastError();
}
hipError_t launch_prim_interior(const Dev &g, const double *U, hipStream_t st) {
  k_prim_interior<<<grid_for(g.ncell), 256, 0, st>>>(g, U);
  return hipGetLastError();
}
hipError_t launch_prim_ghost_dt(const Dev &g, const double *part, int nparts, double cfl,
                               double dt_max, double *dt, hipStream_t st) {
  const unsigned nb = g.nbox > g.ncell ? grid_for(g.nbox - g.ncell) : 0u;
  k_prim_ghost_dt<<<nb + 1, 256, 0, st>>>(g, part, nparts, cfl, dt_max, dt);
  return hipGetLastError();
}
hipError_t launch_dt(const Dev &g, const double *U, double cfl, double dt_max, double *part,
                     double *dt, hipStream_t st) {
  unsigned nb = grid_capped(g.ncell, RED_BLOCKS);
  k_dt_partial<<<nb, 256, 0, st>>>(g, U, part);
  k_dt_final<<<1, 256, 0, st>>>(part, (int)nb, cfl, dt_max, dt);
  return hipGetLastError();
}
hipError_t launch_diag(const Dev &g, const double *U, double *part, double *out,
                       hipStream_t st) {
  unsigned nb = grid_capped(g.ncell, RED_BLOCKS);
  k_diag_partial<<<nb, 256, 0, st>>>(g, U, part);
  k_diag_final<<<1, 256, 0, st>>>(part, (int)nb, out);
  return hipGetLastError();
}
// ---------------------------------------------------------------------------
// Batched step: the same kernels over a table of solves (gridDim.y = solve).
// A workgroup beyond its solve's own count returns before any barrier.
// ---------------------------------------------------------------------------
__device__ __forceinline__ const double *stage_in(const BatchEntry &e, int stage) {
  return stage == 0 ? e.U : (stage == 1 ? e.U1 : e.U2);
}

__global__ void __launch_bounds__(256) kb_prim_interior(const BatchEntry *tab, int stage) {
  const BatchEntry &e = tab[blockIdx.y];
  if (blockIdx.x >= e.nb_prim) return;
  prim_interior_body(e.g, stage_in(e, stage), blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(256) kb_prim_ghost(const BatchEntry *tab) {
  const BatchEntry &e = tab[blockIdx.y];
  if (blockIdx.x >= e.nb_ghost) return;
  prim_ghost_body(e.g, blockIdx.x * blockDim.x + threadIdx.x);
}

template <int NDIM, bool VISC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(flux_waves(SCHEME_WENO5))))
kb_flux_x(const BatchEntry *tab) {
  extern __shared__ double lds[];
  const BatchEntry &e = tab[blockIdx.y];
  if (blockIdx.x >= e.nb_x) return;
  flux_x_body<NDIM, VISC>(e.g, e.nwmax, blockIdx.x, lds);
}

template <int NDIM, int D, bool VISC>
__global__ void __launch_bounds__(256) kb_flux_yz(const BatchEntry *tab) {
  const BatchEntry &e = tab[blockIdx.y];
  if (blockIdx.x >= e.yz_ntot[D]) return;
  flux_yz_body<NDIM, D, VISC>(e.g, blockIdx.x, e.yz_ntot[D], e.yz_nbx[D], e.yz_nby[D]);
}

__global__ void __launch_bounds__(256) kb_update(const BatchEntry *tab, int stage) {
  const BatchEntry &e = tab[blockIdx.y];
  if (blockIdx.x >= e.nb_upd) return;
  // Shu-Osher stages: U1 = U + dt R(U); U2 = 3/4 U + 1/4 (U1 + dt R(U1));
  // U = 1/3 U + 2/3 (U2 + dt R(U2))
  const double a = stage == 0 ? 0.0 : (stage == 1 ? 0.75 : 1.0 / 3.0);
  const double b = stage == 0 ? 1.0 : (stage == 1 ? 0.25 : 2.0 / 3.0);
  double *out = stage == 0 ? e.U1 : (stage == 1 ? e.U2 : e.U);
  update_body(e.g, e.U, stage_in(e, stage), out, nullptr, e.dt, a, b, nullptr,
              blockIdx.x * blockDim.x + threadIdx.x);
}

// The fused-step forms (2D/3D): stage s works on the box of g (s even) or gb
// (s odd); the update of stages 0 and 1 writes the next stage's interior.
__device__ __forceinline__ const Dev &stage_dev(const BatchEntry &e, int stage) {
  return (stage & 1) ? e.gb : e.g;
}

__global__ void __launch_bounds__(256) kb_prim_ghost_s(const BatchEntry *tab, int stage) {
  const BatchEntry &e = tab[blockIdx.y];
  if (blockIdx.x >= e.nb_ghost) return;
  prim_ghost_body(stage_dev(e, stage), blockIdx.x * blockDim.x + threadIdx.x);
}

template <bool VISC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(flux_waves(SCHEME_WENO5))))
kb_flux_xy(const BatchEntry *tab, int stage) {
  extern __shared__ double lds[];
  const BatchEntry &e = tab[blockIdx.y];
  const unsigned ny_tiles = e.yz_ntot[1];
  if (blockIdx.x >= ny_tiles + e.nb_x) return;
  const Dev &g = stage_dev(e, stage);
  if (blockIdx.x < ny_tiles)
    flux_yz_tile<3, 1, VISC>(g, *reinterpret_cast<YzTile<3, VISC> *>(lds), blockIdx.x, ny_tiles,
                             e.yz_nbx[1], e.yz_nby[1]);
  else
    flux_x_body<3, VISC>(g, e.nwmax, blockIdx.x - ny_tiles, lds);
}

template <bool VISC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(flux_waves(SCHEME_WENO5))))
kb_flux_x_s(const BatchEntry *tab, int stage) {
  extern __shared__ double lds[];
  const BatchEntry &e = tab[blockIdx.y];
  if (blockIdx.x >= e.nb_x) return;
  flux_x_body<2, VISC>(stage_dev(e, stage), e.nwmax, blockIdx.x, lds);
}

template <int NDIM, bool VISC>
__global__ void __launch_bounds__(256) kb_flux_update(const BatchEntry *tab, int stage) {
  const BatchEntry &e = tab[blockIdx.y];
  if (blockIdx.x >= e.fu_ntot) return;
  const double a = stage == 0 ? 0.0 : (stage == 1 ? 0.75 : 1.0 / 3.0);
  const double b = stage == 0 ? 1.0 : (stage == 1 ? 0.25 : 2.0 / 3.0);
  double *out = stage == 0 ? e.U1 : (stage == 1 ? e.U2 : e.U);
  BoxOut qo;
  if (stage < 2) {
    const Dev &gn = stage_dev(e, stage + 1);
#pragma unroll
    for (int q = 0; q < NQ; ++q) qo.Q[q] = gn.Q[q];
  }
  flux_update_body<NDIM, NDIM - 1, VISC>(stage_dev(e, stage), blockIdx.x, e.fu_ntot, e.fu_nbx,
                                         e.fu_nby, e.U, stage_in(e, stage), out, e.dt, a, b,
                                         nullptr, blockIdx.x, qo);
}

__global__ void __launch_bounds__(256) kb_dt_partial(const BatchEntry *tab) {
  const BatchEntry &e = tab[blockIdx.y];
  if (blockIdx.x >= e.nb_dt) return;
  dt_partial_body(e.g, e.U, e.part, blockIdx.x, e.nb_dt);
}

__global__ void __launch_bounds__(256) kb_dt_final(const BatchEntry *tab, double cfl) {
  const BatchEntry &e = tab[blockIdx.x];
  dt_final_body(e.part, (int)e.nb_dt, cfl, 1.0e300, e.dt);
}

void batch_entry_sizes(BatchEntry &e) {
  const Dev &g = e.g;
  e.nb_prim = grid_for(g.ncell);
  e.nb_ghost = g.nbox > g.ncell ? grid_for(g.nbox - g.ncell) : 0;
  e.nb_x = grid_for(g.fcount[0]);
  e.nb_upd = grid_for(g.ncell);
  e.nb_dt = grid_capped(g.ncell, RED_BLOCKS);
  e.nwmax = x_window(g);
  for (int D = 0; D < 3; ++D) {
    e.yz_nbx[D] = e.yz_nby[D] = e.yz_ntot[D] = 0;
    if (D == 0 || D >= g.ndim) continue;
    e.yz_nbx[D] = (g.n[0] + 15) / 16;
    e.yz_nby[D] = (g.n[D] + 1 + 15) / 16;
    e.yz_ntot[D] = e.yz_nbx[D] * e.yz_nby[D] * (D == 1 ? g.n[2] : g.n[1]);
  }
  e.fu_nbx = e.fu_nby = e.fu_ntot = 0;
  if (g.ndim >= 2) {
    const int D = g.ndim - 1;
    e.fu_nbx = (g.n[0] + 15) / 16;
    e.fu_nby = (g.n[D] + 14) / 15;
    e.fu_ntot = e.fu_nbx * e.fu_nby * (D == 1 ? g.n[2] : g.n[1]);
  }
}

template <int NDIM, bool VISC>
static hipError_t batch_step_t(const BatchEntry *tab, const BatchEntry *h, int n, double cfl,
                               hipStream_t st) {
  unsigned mp = 0, mh = 0, mx = 0, mu = 0, md = 0, my[3] = {0, 0, 0};
  int nw = 0;
  for (int i = 0; i < n; ++i) {
    mp = std::max(mp, h[i].nb_prim);
    mh = std::max(mh, h[i].nb_ghost);
    mx = std::max(mx, h[i].nb_x);
    mu = std::max(mu, h[i].nb_upd);
    md = std::max(md, h[i].nb_dt);
    nw = std::max(nw, h[i].nwmax);
    for (int D = 1; D < 3; ++D) my[D] = std::max(my[D], h[i].yz_ntot[D]);
  }
  const unsigned ny = (unsigned)n;
  if (cfl > 0.0) {
    kb_dt_partial<<<dim3(md, ny), 256, 0, st>>>(tab);
    kb_dt_final<<<ny, 256, 0, st>>>(tab, cfl);
  }
  const size_t shm = sizeof(double) * Slots<NDIM, VISC>::NC * nw;
  if (NDIM >= 2) {
    // the single-solve step's launch sequence, one launch per kernel for all
    unsigned mf = 0;
    for (int i = 0; i < n; ++i) mf = std::max(mf, h[i].fu_ntot);
    constexpr int ND = NDIM < 2 ? 2 : NDIM;
    const size_t shm_xy = std::max(shm, sizeof(YzTile<ND, VISC>));
    for (int stage = 0; stage < 3; ++stage) {
      if (stage == 0) kb_prim_interior<<<dim3(mp, ny), 256, 0, st>>>(tab, 0);
      if (mh) kb_prim_ghost_s<<<dim3(mh, ny), 256, 0, st>>>(tab, stage);
      if (NDIM == 3)
        kb_flux_xy<VISC><<<dim3(my[1] + mx, ny), 256, shm_xy, st>>>(tab, stage);
      else
        kb_flux_x_s<VISC><<<dim3(mx, ny), 256, shm, st>>>(tab, stage);
      kb_flux_update<ND, VISC><<<dim3(mf, ny), 256, 0, st>>>(tab, stage);
    }
    return hipGetLastError();
  }
  for (int stage = 0; stage < 3; ++stage) {
    kb_prim_interior<<<dim3(mp, ny), 256, 0, st>>>(tab, stage);
    if (mh) kb_prim_ghost<<<dim3(mh, ny), 256, 0, st>>>(tab);
    kb_flux_x<NDIM, VISC><<<dim3(mx, ny), 256, shm, st>>>(tab);
    if (NDIM >= 2) kb_flux_yz<NDIM < 2 ? 2 : NDIM, 1, VISC><<<dim3(my[1], ny), 256, 0, st>>>(tab);
    if (NDIM >= 3) kb_flux_yz<3, 2, VISC><<<dim3(my[2], ny), 256, 0, st>>>(tab);
    kb_update<<<dim3(mu, ny), 256, 0, st>>>(tab, stage);
  }
  return hipGetLastError();
}

hipError_t launch_batch_step(const BatchEntry *tab_dev, const BatchEntry *tab_host, int n,
                             double cfl, hipStream_t st) {
  const int nd = tab_host[0].g.ndim;
  const bool v = tab_host[0].g.visc != VISC_NONE;
  switch (nd) {
    case 1: return v ? batch_step_t<1, true>(tab_dev, tab_host, n, cfl, st)
                     : batch_step_t<1, false>(tab_dev, tab_host, n, cfl, st);
    case 2: return v ? batch_step_t<2, true>(tab_dev, tab_host, n, cfl, st)
                     : batch_step_t<2, false>(tab_dev, tab_host, n, cfl, st);
    case 3: return v ? batch_step_t<3, true>(tab_dev, tab_host, n, cfl, st)
                     : batch_step_t<3, false>(tab_dev, tab_host, n, cfl, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_cost(const Dev &g, int face, double pref, const double *U, double w,
                       double *J, double *grad, hipStream_t st) {
  k_cost<<<1, 1024, 0, st>>>(g, face, pref, U, w, J, grad);
  return hipGetLastError();
}

}  // namespace dcf
