/*
 * oracle.cpp -- CPU oracle for the finite-volume compressible Navier-Stokes
 * right-hand side, its halo-cell boundary conditions, TVD-RK3 stepping and a
 * dense forward-mode adjoint.
 *
 * TEST INFRASTRUCTURE ONLY: plain FP64 loops written for readability, not
 * speed.  Only tests/, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  Nothing here is shared with the GPU library.
 *
 * What the paper fixes and what this file follows:
 *   - conserved vector U = [rho, rho u, rho v, rho w, E], E = rho e + |u|^2 rho/2
 *     (Section 2.1, Eq. (2)); ideal gas with gamma (Section 3.2);
 *   - convective fluxes F^c, G^c, H^c (Eq. (3)); dissipative fluxes
 *     F^d, G^d, H^d with the energy entry sum_i u_i tau_ij - q_j (Eq. (4));
 *     Stokes-hypothesis stress (Eq. (5)); Fourier heat flux q = -lambda grad T;
 *   - the cell-averaged semi-discrete update (Eq. (6)):
 *       dU/dt = -sum_d (1/dx_d) [(F^c - F^d)_{+1/2} - (F^c - F^d)_{-1/2}] + S;
 *   - convective fluxes from a WENO-type reconstruction and an approximate
 *     Riemann solver, HLLC (Section 2.1 text after Eq. (6); Section 3.1),
 *     dissipative fluxes by central finite differences, time integration by an
 *     explicit TVD Runge-Kutta scheme (Section 2.1);
 *   - boundary conditions by assigning halo-cell values: no-slip wall,
 *     Dirichlet, zero-gradient (Section 3.2), plus a wall whose normal
 *     velocity is set inside the boundary class from parameters handed down by
 *     the solver, so that it is differentiable (Section 3.2, "Disturbance
 *     Wall"); stretched Cartesian meshes with a tanh law (Section 2, 3.2);
 *   - Sutherland viscosity (Section 3.2);
 *   - a domain of [Nx+2Nh, Ny+2Nh, Nz+2Nh] cells including halos (Section 2.2).
 *
 * Where the paper names a scheme but does not write it out, this file uses
 * the textbook definition:
 *   - WENO5-JS: Jiang & Shu, J. Comput. Phys. 126 (1996), eps = 1e-6, p = 2;
 *   - HLLC: Toro, Spruce & Speares, Shock Waves 4 (1994), Davis wave speeds;
 *   - TVD-RK3: Shu & Osher, J. Comput. Phys. 77 (1988);
 *   - 4th-order central interpolation/differences for the dissipative terms.
 * The readings taken where the paper is silent are listed in the design notes
 * of the repository (reconstruction variables, wave speeds, tie-breaking,
 * wall ghost states, Darcy law sign, body force, time step).
 */
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include <omp.h>

namespace {

/* ------------------------------------------------------------------------ */
/* Forward-mode dual number with one tangent.  Branches and min/max follow   */
/* the primal value, so derivatives are those of the branch taken.           */
/* ------------------------------------------------------------------------ */
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double a) : v(a), d(0.0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual &operator+=(Dual &a, Dual b) { a = a + b; return a; }
inline Dual &operator-=(Dual &a, Dual b) { a = a - b; return a; }
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
inline Dual pow(Dual a, double e) {
  return Dual(std::pow(a.v, e), e * std::pow(a.v, e - 1.0) * a.d);
}
inline Dual sin(Dual a) { return Dual(std::sin(a.v), std::cos(a.v) * a.d); }
inline double sqrt(double a) { return std::sqrt(a); }
inline double sin(double a) { return std::sin(a); }
inline double pow(double a, double e) { return std::pow(a, e); }
inline double val(double x) { return x; }
inline double val(const Dual &x) { return x.v; }

template <class T> inline T vmin(T a, T b) { return val(b) < val(a) ? b : a; }
template <class T> inline T vmax(T a, T b) { return val(b) > val(a) ? b : a; }

/* ------------------------------------------------------------------------ */
/* Grid: one axis.  Computational coordinate xi in [0, n], one cell per unit; */
/* faces at xi = i, centres at xi = i + 1/2, physical x = map(xi / n).        */
/* ------------------------------------------------------------------------ */
struct Axis {
  int n;
  std::vector<double> xf, dx, mc, mf; /* faces, widths, dxi/dx at centres, faces */
};

/* x(s) and dx/dxi for s = xi/n in [0,1].  Two tanh laws (stretched meshes,
 * Section 2 and Section 3.2): symmetric clustering at both ends (walls of a
 * channel) and one-sided clustering at lo (wall of a boundary layer). */
static void axis_map(int kind, double lo, double hi, double beta, int n, double s,
                     double *x, double *dxdxi) {
  double L = hi - lo;
  if (kind == ORC_STRETCH_TANH2) {
    double a = beta * (1.0 - 2.0 * s);
    double th = std::tanh(beta);
    *x = lo + L * 0.5 * (1.0 - std::tanh(a) / th);
    double ch = std::cosh(a);
    *dxdxi = L * beta / (n * th * ch * ch);
  } else if (kind == ORC_STRETCH_TANH1) {
    double a = beta * (s - 1.0);
    double th = std::tanh(beta);
    *x = lo + L * (1.0 + std::tanh(a) / th);
    double ch = std::cosh(a);
    *dxdxi = L * beta / (n * th * ch * ch);
  } else {
    *x = lo + L * s;
    *dxdxi = L / n;
  }
}

static Axis make_axis(const orc_case &c, int d) {
  Axis ax;
  ax.n = c.n[d];
  int n = ax.n;
  ax.xf.resize(n + 1);
  ax.dx.resize(n);
  ax.mc.resize(n);
  ax.mf.resize(n + 1);
  for (int i = 0; i <= n; ++i) {
    double x, g;
    axis_map(c.stretch[d], c.lo[d], c.hi[d], c.beta[d], n, (double)i / n, &x, &g);
    ax.xf[i] = x;
    ax.mf[i] = 1.0 / g;
  }
  for (int i = 0; i < n; ++i) {
    double x, g;
    axis_map(c.stretch[d], c.lo[d], c.hi[d], c.beta[d], n, (i + 0.5) / n, &x, &g);
    ax.mc[i] = 1.0 / g;
    ax.dx[i] = ax.xf[i + 1] - ax.xf[i];
  }
  return ax;
}

/* ------------------------------------------------------------------------ */
/* WENO5-JS (Jiang & Shu 1996): value at the right face of the centre cell c  */
/* from the cell values (a, b, c, d, e).                                      */
/* ------------------------------------------------------------------------ */
template <class T> T weno5(T a, T b, T c, T d, T e) {
  const double eps = 1e-6;
  T q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  T q1 = (-1.0 * b + 5.0 * c + 2.0 * d) / 6.0;
  T q2 = (2.0 * c + 5.0 * d - 1.0 * e) / 6.0;
  T s0a = a - 2.0 * b + c, s0b = a - 4.0 * b + 3.0 * c;
  T s1a = b - 2.0 * c + d, s1b = b - d;
  T s2a = c - 2.0 * d + e, s2b = 3.0 * c - 4.0 * d + e;
  T b0 = (13.0 / 12.0) * s0a * s0a + 0.25 * s0b * s0b;
  T b1 = (13.0 / 12.0) * s1a * s1a + 0.25 * s1b * s1b;
  T b2 = (13.0 / 12.0) * s2a * s2a + 0.25 * s2b * s2b;
  T a0 = 0.1 / ((eps + b0) * (eps + b0));
  T a1 = 0.6 / ((eps + b1) * (eps + b1));
  T a2 = 0.3 / ((eps + b2) * (eps + b2));
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

/* ------------------------------------------------------------------------ */
/* HLLC flux (Toro, Spruce & Speares 1994) in the face frame.  q = (rho,     */
/* u_n, u_t1, u_t2, p); F = (mass, normal momentum, t1 momentum, t2 momentum, */
/* energy).  Physical flux per Eq. (3); wave speeds after Davis.  Ties at     */
/* 0 <= S take the left-side branch.                                          */
/* ------------------------------------------------------------------------ */
template <class T> void hllc(const T *qL, const T *qR, double gamma, T *F) {
  T rL = qL[0], uL = qL[1], vL = qL[2], wL = qL[3], pL = qL[4];
  T rR = qR[0], uR = qR[1], vR = qR[2], wR = qR[3], pR = qR[4];
  T EL = pL / (gamma - 1.0) + 0.5 * rL * (uL * uL + vL * vL + wL * wL);
  T ER = pR / (gamma - 1.0) + 0.5 * rR * (uR * uR + vR * vR + wR * wR);
  T cL = sqrt(gamma * pL / rL);
  T cR = sqrt(gamma * pR / rR);
  T SL = vmin(uL - cL, uR - cR);
  T SR = vmax(uL + cL, uR + cR);
  T Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
         (rL * (SL - uL) - rR * (SR - uR));

  T FL[5] = {rL * uL, rL * uL * uL + pL, rL * uL * vL, rL * uL * wL, uL * (EL + pL)};
  T FR[5] = {rR * uR, rR * uR * uR + pR, rR * uR * vR, rR * uR * wR, uR * (ER + pR)};
  if (0.0 <= val(SL)) {
    for (int m = 0; m < 5; ++m) F[m] = FL[m];
    return;
  }
  if (val(SR) < 0.0) {
    for (int m = 0; m < 5; ++m) F[m] = FR[m];
    return;
  }
  bool left = (0.0 <= val(Ss));
  T r = left ? rL : rR, u = left ? uL : uR, v = left ? vL : vR, w = left ? wL : wR;
  T p = left ? pL : pR, E = left ? EL : ER, S = left ? SL : SR;
  const T *Fk = left ? FL : FR;
  T fac = r * (S - u) / (S - Ss);
  T Us[5] = {fac, fac * Ss, fac * v, fac * w,
             fac * (E / r + (Ss - u) * (Ss + p / (r * (S - u))))};
  T Uk[5] = {r, r * u, r * v, r * w, E};
  for (int m = 0; m < 5; ++m) F[m] = Fk[m] + S * (Us[m] - Uk[m]);
}

/* ------------------------------------------------------------------------ */
/* TENO6-A (targeted ENO with six points and adaptive dissipation; Fu, Hu &  */
/* Adams): value at the right face of cell i from v = cells i-2 .. i+3.      */
/* Steps, in the scheme's order:                                             */
/*  1. third-order candidates on S0 = {i-1,i,i+1}, S1 = {i,i+1,i+2},          */
/*     S2 = {i-2,i-1,i} and the fourth-order candidate on S3 = {i..i+3};     */
/*     linear weights d = (0.45, 0.3, 0.05, 0.2), the combination that is    */
/*     the sixth-order central reconstruction on the six points;             */
/*  2. Jiang-Shu smoothness indicators beta_k of the candidates and beta6 of  */
/*     the six-point polynomial; tau6 = |beta6 - (beta0 + beta2 + 4 beta1)/6| */
/*  3. scale separation gamma_k = (C + tau6 / (beta_k + eps))^q, C = 1,     */
/*     q = 6, eps = 1e-40, chi_k = gamma_k / sum gamma;                       */
/*  4. adaptive cut-off C_T = 10^-floor(b), b = alpha1 - alpha2 (1 - g(m)),   */
/*     g(m) = (1 - m)^4 (1 + 4 m), m = 1 - min(1, eta / C_r), with eta the    */
/*     smallest of Ren et al.'s smoothness measures of cells i-1 .. i+2:      */
/*     eta_j = (|2 D_{j+1/2} D_{j-1/2}| + e) / (D_{j+1/2}^2 + D_{j-1/2}^2 + e),  */
/*     D_{j+1/2} = v_{j+1} - v_j, e = 0.9 C_r xi^2 / (1 - 0.9 C_r);            */
/*     alpha1 = 10.5, alpha2 = 3.5, C_r = 0.17, xi = 1e-3 (so C_T runs from   */
/*     1e-10 in smooth regions to 1e-7 at discontinuities);                  */
/*  5. sharp cut-off delta_k = 0 if chi_k < C_T else 1, and                   */
/*     omega_k = d_k delta_k / sum_l d_l delta_l;                             */
/*  6. the value sum_k omega_k q_k.                                           */
/* The cut-off decisions are piecewise constant: a Dual carries the          */
/* derivative of the branch taken.                                           */
/* ------------------------------------------------------------------------ */
template <class T> inline T vabs(T x) { return val(x) < 0.0 ? -1.0 * x : x; }

template <class T> T teno6a(const T *v, double *ct_out = nullptr, double *w_out = nullptr) {
  const T a = v[0], b = v[1], c = v[2], d = v[3], e = v[4], f = v[5];
  /* 1 */
  T q[4] = {(-1.0 * b + 5.0 * c + 2.0 * d) / 6.0, (2.0 * c + 5.0 * d - 1.0 * e) / 6.0,
            (2.0 * a - 7.0 * b + 11.0 * c) / 6.0,
            (3.0 * c + 13.0 * d - 5.0 * e + 1.0 * f) / 12.0};
  const double dk[4] = {0.45, 0.3, 0.05, 0.2};
  /* 2 */
  T beta[4];
  {
    T s1 = b - 2.0 * c + d, t1 = b - d;
    T s2 = c - 2.0 * d + e, t2 = 3.0 * c - 4.0 * d + e;
    T s3 = a - 2.0 * b + c, t3 = a - 4.0 * b + 3.0 * c;
    beta[0] = (13.0 / 12.0) * s1 * s1 + 0.25 * t1 * t1;
    beta[1] = (13.0 / 12.0) * s2 * s2 + 0.25 * t2 * t2;
    beta[2] = (13.0 / 12.0) * s3 * s3 + 0.25 * t3 * t3;
    beta[3] = (c * (2107.0 * c - 9402.0 * d + 7042.0 * e - 1854.0 * f) +
               d * (11003.0 * d - 17246.0 * e + 4642.0 * f) +
               e * (7043.0 * e - 3882.0 * f) + 547.0 * f * f) / 240.0;
  }
  T beta6 = (271779.0 * a * a +
             a * (-2380800.0 * b + 4086352.0 * c - 3462252.0 * d + 1458762.0 * e -
                  245620.0 * f) +
             b * (5653317.0 * b - 20427884.0 * c + 17905032.0 * d - 7727988.0 * e +
                  1325006.0 * f) +
             c * (19510972.0 * c - 35817664.0 * d + 15929912.0 * e - 2792660.0 * f) +
             d * (17195652.0 * d - 15880404.0 * e + 2863984.0 * f) +
             e * (3824847.0 * e - 1429976.0 * f) + 139633.0 * f * f) / 120960.0;
  T tau6 = vabs(beta6 - (beta[0] + beta[2] + 4.0 * beta[1]) / 6.0);
  /* 3 */
  T gam[4];
  T gsum = T(0.0);
  for (int k = 0; k < 4; ++k) {
    T r = 1.0 + tau6 / (beta[k] + 1e-40);
    gam[k] = r * r * r * r * r * r;
    gsum += gam[k];
  }
  /* 4 */
  const double Cr = 0.17, xi = 1e-3, alpha1 = 10.5, alpha2 = 3.5;
  const double eps_eta = 0.9 * Cr * xi * xi / (1.0 - 0.9 * Cr);
  double eta = 1e300;
  for (int j = 1; j <= 4; ++j) { /* cells i-1 .. i+2 = v[1] .. v[4] */
    double dm = val(v[j]) - val(v[j - 1]), dp = val(v[j + 1]) - val(v[j]);
    double ej = (std::fabs(2.0 * dp * dm) + eps_eta) / (dp * dp + dm * dm + eps_eta);
    eta = std::min(eta, ej);
  }
  double m = 1.0 - std::min(1.0, eta / Cr);
  double gm = std::pow(1.0 - m, 4.0) * (1.0 + 4.0 * m);
  double bbar = alpha1 - alpha2 * (1.0 - gm);
  double CT = std::pow(10.0, -std::floor(bbar));
  if (ct_out) *ct_out = CT;
  /* 5, 6 */
  double wsum = 0.0, w[4];
  for (int k = 0; k < 4; ++k) {
    double chi = val(gam[k]) / val(gsum);
    w[k] = chi < CT ? 0.0 : dk[k];
    wsum += w[k];
  }
  T out = T(0.0);
  for (int k = 0; k < 4; ++k) {
    if (w_out) w_out[k] = w[k] / wsum;
    out += (w[k] / wsum) * q[k];
  }
  return out;
}

/* 6th-order central interpolation to a face and derivatives (index space):
 * face value and face derivative from the six cells around the face, cell
 * derivative from the cells three either side. */
template <class T> inline T interp6(T a, T b, T c, T d, T e, T f) {
  return (3.0 * a - 25.0 * b + 150.0 * c + 150.0 * d - 25.0 * e + 3.0 * f) / 256.0;
}
template <class T> inline T dface6(T a, T b, T c, T d, T e, T f) {
  return (2250.0 * (d - c) - 125.0 * (e - b) + 9.0 * (f - a)) / 1920.0;
}
template <class T> inline T dcell6(T m3, T m2, T m1, T p1, T p2, T p3) {
  return (45.0 * (p1 - m1) - 9.0 * (p2 - m2) + (p3 - m3)) / 60.0;
}

/* 4th-order central interpolation to a face and derivatives (index space). */
template <class T> inline T interp4(T a, T b, T c, T d) {
  return (-1.0 * a + 9.0 * b + 9.0 * c - 1.0 * d) / 16.0;
}
template <class T> inline T dface4(T a, T b, T c, T d) {
  return (27.0 * (c - b) - (d - a)) / 24.0;
}
template <class T> inline T dcell4(T m2, T m1, T p1, T p2) {
  return (8.0 * (p1 - m1) - (p2 - m2)) / 12.0;
}

/* ------------------------------------------------------------------------ */
/* The solver on one case, templated on the scalar (double or Dual).         */
/* ------------------------------------------------------------------------ */
/* Position in the boundary-parameter vector K of the first parameter of
 * face `face` if it is a disturbance wall: the porous coefficients come
 * first, then (A, kappa) of each disturbance face in face order.  With
 * face = 2 ndim it is the length of K. */
static int disturb_offset(const orc_case *c, int face) {
  int o = 0;
  if (c->porous_face >= 0) {
    int d = c->porous_face / 2;
    int t2 = d == 2 ? 1 : 2;
    o = (c->porous_end - c->porous_begin) * c->n[t2];
  }
  for (int f = 0; f < face && f < 6; ++f)
    if (c->bc[f] == ORC_DISTURB) o += 2;
  return o;
}

template <class T> struct Solver {
  const orc_case &c;
  int nd, nv;
  int n[3], h[3], N[3];
  long ncell, nbox;
  Axis ax[3];
  std::vector<T> Q[6]; /* rho, u, v, w, p, T on the halo'd box */
  std::vector<T> MU;   /* dynamic viscosity on the halo'd box  */
  const T *K;          /* porous coefficients                  */
  double cp;

  explicit Solver(const orc_case &cs) : c(cs), K(nullptr) {
    nd = c.ndim;
    nv = nd + 2;
    for (int d = 0; d < 3; ++d) {
      n[d] = c.n[d];
      h[d] = d < nd ? 3 : 0;
      N[d] = n[d] + 2 * h[d];
      ax[d] = make_axis(c, d);
    }
    ncell = (long)n[0] * n[1] * n[2];
    nbox = (long)N[0] * N[1] * N[2];
    for (int q = 0; q < 6; ++q) Q[q].assign(nbox, T(0.0));
    MU.assign(nbox, T(0.0));
    cp = c.gamma * c.R / (c.gamma - 1.0);
  }

  bool viscous() const { return c.visc_law != ORC_VISC_NONE; }
  long bid(int i, int j, int k) const {
    return ((long)(k + h[2]) * N[1] + (j + h[1])) * N[0] + (i + h[0]);
  }
  long cid(int i, int j, int k) const { return ((long)k * n[1] + j) * n[0] + i; }
  static int t1(int d) { return d == 0 ? 1 : 0; }
  static int t2(int d) { return d == 2 ? 1 : 2; }
  /* box index of the cell at position s along axis d and (a, b) along t1, t2 */
  long at(int d, int s, int a, int b) const {
    int p[3];
    p[d] = s;
    p[t1(d)] = a;
    p[t2(d)] = b;
    return bid(p[0], p[1], p[2]);
  }
  /* conserved component index of the 5-component flux entry m */
  int cons_index(int m) const {
    if (m == 0) return 0;
    if (m == 4) return nd + 1;
    return (m <= nd) ? m : -1;
  }

  T viscosity(T Tt) const {
    if (c.visc_law == ORC_VISC_POWER) return c.mu_ref * pow(Tt / c.T_ref, c.visc_param);
    if (c.visc_law == ORC_VISC_SUTHERLAND) {
      /* Sutherland law (Section 3.2) */
      T t = Tt / c.T_ref;
      double s = c.visc_param / c.T_ref;
      return c.mu_ref * t * sqrt(t) * (1.0 + s) / (t + s);
    }
    return T(0.0);
  }

  /* Primitive variables of the interior cells from U (Eq. (2)). */
  void prims_interior(const T *U) {
    const double g = c.gamma;
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j)
        for (int i = 0; i < n[0]; ++i) {
          long ci = cid(i, j, k), b = bid(i, j, k);
          T rho = U[0 * ncell + ci];
          T u = U[1 * ncell + ci] / rho;
          T v = nd >= 2 ? U[2 * ncell + ci] / rho : T(0.0);
          T w = nd >= 3 ? U[3 * ncell + ci] / rho : T(0.0);
          T E = U[(long)(nd + 1) * ncell + ci];
          T p = (g - 1.0) * (E - 0.5 * rho * (u * u + v * v + w * w));
          Q[0][b] = rho;
          Q[1][b] = u;
          Q[2][b] = v;
          Q[3][b] = w;
          Q[4][b] = p;
          Q[5][b] = p / (rho * c.R);
        }
  }

  /* Halo cells of axis d (Section 3.2: boundary conditions are imposed by
   * assigning halo-cell values).  Axes are filled in the order x, y, z; each
   * fill covers the full extent of the axes filled before it, which defines
   * edge and corner halos. Ghost layer m mirrors interior layer m. */
  void fill_axis(int d) {
    int lo1 = 0, hi1 = n[t1(d)], lo2 = 0, hi2 = n[t2(d)];
    if (t1(d) < d) { lo1 = -h[t1(d)]; hi1 = n[t1(d)] + h[t1(d)]; }
    if (t2(d) < d) { lo2 = -h[t2(d)]; hi2 = n[t2(d)] + h[t2(d)]; }
    for (int side = 0; side < 2; ++side) {
      int face = 2 * d + side;
      int kind = c.bc[face];
      for (int m = 0; m < 3; ++m) {
        int g = side == 0 ? -1 - m : n[d] + m;
        for (int b = lo2; b < hi2; ++b)
          for (int a = lo1; a < hi1; ++a) {
            long G = at(d, g, a, b);
            if (kind == ORC_PERIODIC) {
              long S = at(d, side == 0 ? n[d] - 1 - m : m, a, b);
              for (int q = 0; q < 6; ++q) Q[q][G] = Q[q][S];
            } else if (kind == ORC_ZEROGRAD) {
              long S = at(d, side == 0 ? 0 : n[d] - 1, a, b);
              for (int q = 0; q < 6; ++q) Q[q][G] = Q[q][S];
            } else if (kind == ORC_DIRICHLET) {
              int ac = std::min(std::max(a, 0), n[t1(d)] - 1);
              int bc = std::min(std::max(b, 0), n[t2(d)] - 1);
              long nt = (long)n[t1(d)] * n[t2(d)];
              long o = (long)bc * n[t1(d)] + ac;
              const double *P = c.dirichlet[face];
              Q[0][G] = P[0 * nt + o];
              Q[1][G] = P[1 * nt + o];
              Q[2][G] = P[2 * nt + o];
              Q[3][G] = P[3 * nt + o];
              Q[4][G] = P[4 * nt + o];
              Q[5][G] = Q[4][G] / (Q[0][G] * c.R);
            } else { /* no-slip wall: isothermal or adiabatic, optionally porous
                        or with a prescribed normal velocity */
              long S = at(d, side == 0 ? m : n[d] - 1 - m, a, b);
              T vel[3] = {-1.0 * Q[1][S], -1.0 * Q[2][S], -1.0 * Q[3][S]};
              double sigma = side == 0 ? 1.0 : -1.0;
              if (kind == ORC_POROUS && face == c.porous_face && a >= c.porous_begin &&
                  a < c.porous_end && b >= 0 && b < n[t2(d)]) {
                /* Darcy transpiration: wall-normal velocity along the inward
                 * normal is -K (p_w - p_inf)/p_inf, p_w from the first
                 * interior cell of this column. */
                long W = at(d, side == 0 ? 0 : n[d] - 1, a, b);
                int kk = b * (c.porous_end - c.porous_begin) + (a - c.porous_begin);
                T vn = -1.0 * K[kk] * (Q[4][W] - c.p_inf) / c.p_inf;
                vel[d] = 2.0 * sigma * vn - Q[1 + d][S];
              }
              if (kind == ORC_DISTURB && a >= 0 && a < n[t1(d)]) {
                /* Disturbance wall: v_n = A sin(2 pi kappa x) at the centre
                 * of the wall face along the first tangential axis; A and
                 * kappa are boundary parameters. */
                const Axis &ta = ax[t1(d)];
                double xc = 0.5 * (ta.xf[a] + ta.xf[a + 1]);
                int o = disturb_offset(&c, face);
                T vn = K[o] * sin(2.0 * M_PI * xc * K[o + 1]);
                vel[d] = 2.0 * sigma * vn - Q[1 + d][S];
              }
              T p = Q[4][S];
              if (c.T_wall[face] > 0.0) { /* isothermal */
                T Tg = 2.0 * c.T_wall[face] - Q[5][S];
                Q[0][G] = p / (c.R * Tg);
                Q[5][G] = Tg;
              } else { /* adiabatic: temperature and density mirror */
                Q[0][G] = Q[0][S];
                Q[5][G] = Q[5][S];
              }
              Q[1][G] = vel[0];
              Q[2][G] = vel[1];
              Q[3][G] = vel[2];
              Q[4][G] = p;
            }
          }
      }
    }
  }

  void build_prims(const T *U) {
    prims_interior(U);
    for (int d = 0; d < nd; ++d) fill_axis(d);
    if (viscous())
      for (long b = 0; b < nbox; ++b) MU[b] = viscosity(Q[5][b]);
  }

  /* Tangential derivative along axis t of primitive q at box cell with
   * position (s along d, a, b); the cell's index along t is pos. */
  T dtan(int q, int d, int t, int s, int a, int b) const {
    int p[3];
    p[d] = s;
    p[t1(d)] = a;
    p[t2(d)] = b;
    int pos = p[t];
    auto val_at = [&](int off) {
      int r[3] = {p[0], p[1], p[2]};
      r[t] += off;
      return Q[q][bid(r[0], r[1], r[2])];
    };
    if (c.scheme == ORC_SCHEME_TENO6A)
      return dcell6(val_at(-3), val_at(-2), val_at(-1), val_at(1), val_at(2), val_at(3)) *
             ax[t].mc[pos];
    return dcell4(val_at(-2), val_at(-1), val_at(1), val_at(2)) * ax[t].mc[pos];
  }

  /* Total flux (F^c - F^d) at face f (between cells f-1 and f) of axis d,
   * in the global 5-component layout. */
  void face_flux(int d, int f, int a, int b, T *out) const {
    const int qi[5] = {0, 1 + d, 1 + t1(d), 1 + t2(d), 4};
    T qL[5], qR[5];
    for (int m = 0; m < 5; ++m) {
      const std::vector<T> &A = Q[qi[m]];
      T v0 = A[at(d, f - 3, a, b)], v1 = A[at(d, f - 2, a, b)], v2 = A[at(d, f - 1, a, b)];
      T v3 = A[at(d, f, a, b)], v4 = A[at(d, f + 1, a, b)], v5 = A[at(d, f + 2, a, b)];
      if (c.scheme == ORC_SCHEME_TENO6A) {
        T six[6] = {v0, v1, v2, v3, v4, v5}, mir[6] = {v5, v4, v3, v2, v1, v0};
        qL[m] = teno6a(six);
        qR[m] = teno6a(mir);
      } else {
        qL[m] = weno5(v0, v1, v2, v3, v4);
        qR[m] = weno5(v5, v4, v3, v2, v1);
      }
    }
    if (c.scheme == ORC_SCHEME_TENO6A) {
      /* interpolation limiter: a side whose reconstructed density or
       * pressure is not positive takes the first-order state, the primitives
       * of its own cell */
      if (!(val(qL[0]) > 0.0 && val(qL[4]) > 0.0))
        for (int m = 0; m < 5; ++m) qL[m] = Q[qi[m]][at(d, f - 1, a, b)];
      if (!(val(qR[0]) > 0.0 && val(qR[4]) > 0.0))
        for (int m = 0; m < 5; ++m) qR[m] = Q[qi[m]][at(d, f, a, b)];
    }
    T Fc[5];
    hllc(qL, qR, c.gamma, Fc);
    T G[5];
    G[0] = Fc[0];
    G[1 + d] = Fc[1];
    G[1 + t1(d)] = Fc[2];
    G[1 + t2(d)] = Fc[3];
    G[4] = Fc[4];
    if (viscous() && c.scheme == ORC_SCHEME_TENO6A) {
      /* Dissipative flux, Eqs. (4)-(5) and Fourier's law, 6th-order central
       * over the six cells f-3 .. f+2. */
      auto cellq = [&](int q, int s) { return Q[q][at(d, s, a, b)]; };
      auto fval = [&](int q) {
        return interp6(cellq(q, f - 3), cellq(q, f - 2), cellq(q, f - 1), cellq(q, f),
                       cellq(q, f + 1), cellq(q, f + 2));
      };
      auto fder = [&](int q) {
        return dface6(cellq(q, f - 3), cellq(q, f - 2), cellq(q, f - 1), cellq(q, f),
                      cellq(q, f + 1), cellq(q, f + 2)) * ax[d].mf[f];
      };
      T muf = interp6(MU[at(d, f - 3, a, b)], MU[at(d, f - 2, a, b)], MU[at(d, f - 1, a, b)],
                      MU[at(d, f, a, b)], MU[at(d, f + 1, a, b)], MU[at(d, f + 2, a, b)]);
      T uf[3] = {fval(1), fval(2), fval(3)};
      T dn[3] = {fder(1), fder(2), fder(3)};
      T dT = fder(5);
      T tau[3] = {T(0.0), T(0.0), T(0.0)};
      T divt = T(0.0);
      T dtn[3] = {T(0.0), T(0.0), T(0.0)};
      const int tt[2] = {t1(d), t2(d)};
      for (int r = 0; r < 2; ++r) {
        int t = tt[r];
        if (t >= nd) continue;
        T g_tt[6], g_tn[6];
        for (int o = 0; o < 6; ++o) {
          g_tt[o] = dtan(1 + t, d, t, f - 3 + o, a, b);
          g_tn[o] = dtan(1 + d, d, t, f - 3 + o, a, b);
        }
        divt += interp6(g_tt[0], g_tt[1], g_tt[2], g_tt[3], g_tt[4], g_tt[5]);
        dtn[t] = interp6(g_tn[0], g_tn[1], g_tn[2], g_tn[3], g_tn[4], g_tn[5]);
      }
      tau[d] = muf * ((4.0 / 3.0) * dn[d] - (2.0 / 3.0) * divt);
      for (int r = 0; r < 2; ++r) {
        int t = tt[r];
        if (t >= nd) continue;
        tau[t] = muf * (dtn[t] + dn[t]);
      }
      T lam = muf * cp / c.Pr;
      T en = uf[0] * tau[0] + uf[1] * tau[1] + uf[2] * tau[2] + lam * dT;
      G[1] -= tau[0];
      G[2] -= tau[1];
      G[3] -= tau[2];
      G[4] -= en;
    } else if (viscous()) {
      /* Dissipative flux, Eqs. (4)-(5) and Fourier's law, 4th-order central. */
      auto cellq = [&](int q, int s) { return Q[q][at(d, s, a, b)]; };
      auto fval = [&](int q) {
        return interp4(cellq(q, f - 2), cellq(q, f - 1), cellq(q, f), cellq(q, f + 1));
      };
      auto fder = [&](int q) {
        return dface4(cellq(q, f - 2), cellq(q, f - 1), cellq(q, f), cellq(q, f + 1)) *
               ax[d].mf[f];
      };
      T muf = interp4(MU[at(d, f - 2, a, b)], MU[at(d, f - 1, a, b)], MU[at(d, f, a, b)],
                      MU[at(d, f + 1, a, b)]);
      T uf[3] = {fval(1), fval(2), fval(3)};
      T dn[3] = {fder(1), fder(2), fder(3)}; /* normal derivative of u, v, w */
      T dT = fder(5);
      /* tangential derivatives: cell-centred, then interpolated to the face */
      T tau[3] = {T(0.0), T(0.0), T(0.0)};
      T divt = T(0.0);
      T dtn[3] = {T(0.0), T(0.0), T(0.0)}; /* d u_n / d t at the face */
      const int tt[2] = {t1(d), t2(d)};
      for (int r = 0; r < 2; ++r) {
        int t = tt[r];
        if (t >= nd) continue;
        T g_tt[4], g_tn[4];
        for (int o = 0; o < 4; ++o) {
          g_tt[o] = dtan(1 + t, d, t, f - 2 + o, a, b);
          g_tn[o] = dtan(1 + d, d, t, f - 2 + o, a, b);
        }
        divt += interp4(g_tt[0], g_tt[1], g_tt[2], g_tt[3]);
        dtn[t] = interp4(g_tn[0], g_tn[1], g_tn[2], g_tn[3]);
      }
      tau[d] = muf * ((4.0 / 3.0) * dn[d] - (2.0 / 3.0) * divt);
      for (int r = 0; r < 2; ++r) {
        int t = tt[r];
        if (t >= nd) continue;
        tau[t] = muf * (dtn[t] + dn[t]);
      }
      T lam = muf * cp / c.Pr;
      T en = uf[0] * tau[0] + uf[1] * tau[1] + uf[2] * tau[2] + lam * dT;
      G[1] -= tau[0];
      G[2] -= tau[1];
      G[3] -= tau[2];
      G[4] -= en;
    }
    for (int m = 0; m < 5; ++m) out[m] = G[m];
  }

  /* Semi-discrete right-hand side, Eq. (6). */
  void rhs(const T *U, T *R) {
    build_prims(U);
    for (long x = 0; x < (long)nv * ncell; ++x) R[x] = T(0.0);
    for (int d = 0; d < nd; ++d) {
      int na = n[t1(d)], nb = n[t2(d)];
#pragma omp parallel for collapse(2) schedule(static)
      for (int b = 0; b < nb; ++b)
        for (int a = 0; a < na; ++a) {
          std::vector<T> F((size_t)(n[d] + 1) * 5);
          for (int f = 0; f <= n[d]; ++f) face_flux(d, f, a, b, &F[(size_t)f * 5]);
          for (int s = 0; s < n[d]; ++s) {
            int p[3];
            p[d] = s;
            p[t1(d)] = a;
            p[t2(d)] = b;
            long ci = cid(p[0], p[1], p[2]);
            for (int m = 0; m < 5; ++m) {
              int v = cons_index(m);
              if (v < 0) continue;
              R[(long)v * ncell + ci] -=
                  (F[(size_t)(s + 1) * 5 + m] - F[(size_t)s * 5 + m]) / ax[d].dx[s];
            }
          }
        }
    }
    if (c.source == ORC_SOURCE_MASSFLUX) {
      /* Constant-mass-flux body force S = [0, f, 0, 0, f u]: f cancels the
       * volume-weighted mean of the x-momentum right-hand side. */
      T sum = T(0.0);
      double vol = 0.0;
      for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
          for (int i = 0; i < n[0]; ++i) {
            double V = cell_volume(i, j, k);
            sum += V * R[1 * ncell + cid(i, j, k)];
            vol += V;
          }
      T f = -1.0 * sum / vol;
      for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
          for (int i = 0; i < n[0]; ++i) {
            long ci = cid(i, j, k);
            R[1 * ncell + ci] += f;
            R[(long)(nd + 1) * ncell + ci] += f * Q[1][bid(i, j, k)];
          }
    }
  }

  double cell_volume(int i, int j, int k) const {
    double V = ax[0].dx[i];
    if (nd >= 2) V *= ax[1].dx[j];
    if (nd >= 3) V *= ax[2].dx[k];
    return V;
  }

  /* Three-stage TVD Runge-Kutta (Shu & Osher 1988). */
  void step(T *U, double dt) {
    long M = (long)nv * ncell;
    std::vector<T> U1(M), U2(M), R(M);
    rhs(U, R.data());
    for (long x = 0; x < M; ++x) U1[x] = U[x] + dt * R[x];
    rhs(U1.data(), R.data());
    for (long x = 0; x < M; ++x) U2[x] = 0.75 * U[x] + 0.25 * (U1[x] + dt * R[x]);
    rhs(U2.data(), R.data());
    for (long x = 0; x < M; ++x) U[x] = (1.0 / 3.0) * U[x] + (2.0 / 3.0) * (U2[x] + dt * R[x]);
  }

  /* Wall-pressure cost term sum_i (A_i / A) (p_i - p_inf)^2 over the cells
   * adjacent to the cost face. */
  T cost_term(const T *U) {
    prims_interior(U);
    int face = c.cost_face;
    if (face < 0) return T(0.0);
    int d = face / 2, side = face % 2;
    int s = side == 0 ? 0 : n[d] - 1;
    T sum = T(0.0);
    double area = 0.0;
    for (int b = 0; b < n[t2(d)]; ++b)
      for (int a = 0; a < n[t1(d)]; ++a) {
        double A = 1.0;
        if (t1(d) < nd) A *= ax[t1(d)].dx[a];
        if (t2(d) < nd) A *= ax[t2(d)].dx[b];
        T dp = Q[4][at(d, s, a, b)] - c.p_inf;
        sum += A * dp * dp;
        area += A;
      }
    return sum / area;
  }
};

template <class T> void copy_in(const double *src, T *dst, long n) {
  for (long i = 0; i < n; ++i) dst[i] = T(src[i]);
}

} // namespace

/* ======================================================================== */
/* C entry points                                                           */
/* ======================================================================== */
extern "C" {

int orc_nk(const orc_case *c) { return disturb_offset(c, 2 * c->ndim); }

long orc_ncells(const orc_case *c) { return (long)c->n[0] * c->n[1] * c->n[2]; }

long orc_nbox(const orc_case *c) {
  long s = 1;
  for (int d = 0; d < 3; ++d) s *= c->n[d] + (d < c->ndim ? 6 : 0);
  return s;
}

void orc_grid(const orc_case *c, int axis, double *xf, double *dx, double *met_c,
              double *met_f) {
  Axis a = make_axis(*c, axis);
  for (int i = 0; i <= a.n; ++i) {
    xf[i] = a.xf[i];
    met_f[i] = a.mf[i];
  }
  for (int i = 0; i < a.n; ++i) {
    dx[i] = a.dx[i];
    met_c[i] = a.mc[i];
  }
}

double orc_weno5(double a, double b, double c, double d, double e) {
  return weno5<double>(a, b, c, d, e);
}

double orc_teno6a(const double *v, double *ct_out, double *w_out) {
  return teno6a<double>(v, ct_out, w_out);
}

void orc_teno6a_beta(const double *v, double *beta) {
  /* the smoothness indicators teno6a forms (step 2): beta0..beta3, beta6 */
  const double a = v[0], b = v[1], c = v[2], d = v[3], e = v[4], f = v[5];
  double s1 = b - 2.0 * c + d, t1 = b - d;
  double s2 = c - 2.0 * d + e, t2 = 3.0 * c - 4.0 * d + e;
  double s3 = a - 2.0 * b + c, t3 = a - 4.0 * b + 3.0 * c;
  beta[0] = (13.0 / 12.0) * s1 * s1 + 0.25 * t1 * t1;
  beta[1] = (13.0 / 12.0) * s2 * s2 + 0.25 * t2 * t2;
  beta[2] = (13.0 / 12.0) * s3 * s3 + 0.25 * t3 * t3;
  beta[3] = (c * (2107.0 * c - 9402.0 * d + 7042.0 * e - 1854.0 * f) +
             d * (11003.0 * d - 17246.0 * e + 4642.0 * f) + e * (7043.0 * e - 3882.0 * f) +
             547.0 * f * f) / 240.0;
  beta[4] = (271779.0 * a * a +
             a * (-2380800.0 * b + 4086352.0 * c - 3462252.0 * d + 1458762.0 * e -
                  245620.0 * f) +
             b * (5653317.0 * b - 20427884.0 * c + 17905032.0 * d - 7727988.0 * e +
                  1325006.0 * f) +
             c * (19510972.0 * c - 35817664.0 * d + 15929912.0 * e - 2792660.0 * f) +
             d * (17195652.0 * d - 15880404.0 * e + 2863984.0 * f) +
             e * (3824847.0 * e - 1429976.0 * f) + 139633.0 * f * f) / 120960.0;
}

void orc_central_stencils(const double *v, double *out) {
  /* v = point values at offsets -3 .. 3 (v[3] at offset 0): out[0..2] =
   * 6th-order face value, face derivative (face between offsets 0 and 1,
   * from offsets -2 .. 3) and cell derivative at offset 0; out[3..5] the
   * same at 4th order */
  out[0] = interp6(v[1], v[2], v[3], v[4], v[5], v[6]);
  out[1] = dface6(v[1], v[2], v[3], v[4], v[5], v[6]);
  out[2] = dcell6(v[0], v[1], v[2], v[4], v[5], v[6]);
  out[3] = interp4(v[2], v[3], v[4], v[5]);
  out[4] = dface4(v[2], v[3], v[4], v[5]);
  out[5] = dcell4(v[1], v[2], v[4], v[5]);
}

void orc_hllc(const double *qL, const double *qR, double gamma, double *F) {
  hllc<double>(qL, qR, gamma, F);
}

/* Conserved variables from primitives (Eq. (2), ideal gas). */
void orc_cons_from_prim(const orc_case *c, const double *P, double *U) {
  long nc = orc_ncells(c);
  int nd = c->ndim;
  for (long x = 0; x < nc; ++x) {
    double rho = P[0 * nc + x], u = P[1 * nc + x], v = P[2 * nc + x], w = P[3 * nc + x];
    double p = P[4 * nc + x];
    U[0 * nc + x] = rho;
    U[1 * nc + x] = rho * u;
    if (nd >= 2) U[2 * nc + x] = rho * v;
    if (nd >= 3) U[3 * nc + x] = rho * w;
    U[(long)(nd + 1) * nc + x] = p / (c->gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
  }
}

void orc_prims_halo(const orc_case *c, const double *K, const double *U, double *Qbox,
                    double *mubox) {
  Solver<double> s(*c);
  s.K = K;
  s.build_prims(U);
  for (int q = 0; q < 6; ++q)
    std::memcpy(Qbox + (long)q * s.nbox, s.Q[q].data(), sizeof(double) * s.nbox);
  if (mubox) std::memcpy(mubox, s.MU.data(), sizeof(double) * s.nbox);
}

void orc_rhs(const orc_case *c, const double *K, const double *U, double *R) {
  Solver<double> s(*c);
  s.K = K;
  s.rhs(U, R);
}

/* Time step from the CFL condition: dt = CFL / max over cells of
 * sum_d (|u_d| + c)/dx_d + 2 nu_eff sum_d 1/dx_d^2, nu_eff = max(4/3, gamma/Pr) mu/rho. */
double orc_dt(const orc_case *c, const double *U, double cfl) {
  Solver<double> s(*c);
  s.prims_interior(U);
  double smax = 0.0;
  for (int k = 0; k < s.n[2]; ++k)
    for (int j = 0; j < s.n[1]; ++j)
      for (int i = 0; i < s.n[0]; ++i) {
        long b = s.bid(i, j, k);
        double rho = s.Q[0][b], p = s.Q[4][b];
        double cs = std::sqrt(c->gamma * p / rho);
        int pos[3] = {i, j, k};
        double conv = 0.0, inv2 = 0.0;
        for (int d = 0; d < s.nd; ++d) {
          double dx = s.ax[d].dx[pos[d]];
          conv += (std::fabs(s.Q[1 + d][b]) + cs) / dx;
          inv2 += 1.0 / (dx * dx);
        }
        double sig = conv;
        if (s.viscous()) {
          double mu = s.viscosity(s.Q[5][b]);
          double nu = std::max(4.0 / 3.0, c->gamma / c->Pr) * mu / rho;
          sig += 2.0 * nu * inv2;
        }
        smax = std::max(smax, sig);
      }
  return cfl / smax;
}

void orc_step(const orc_case *c, const double *K, double *U, double dt) {
  Solver<double> s(*c);
  s.K = K;
  s.step(U, dt);
}

int orc_run(const orc_case *c, const double *K, double *U, int max_steps, double cfl,
            double dt_fixed, double t_end, double *t_out) {
  Solver<double> s(*c);
  s.K = K;
  double t = 0.0;
  int steps = 0;
  while (steps < max_steps) {
    if (t_end > 0.0 && t >= t_end) break;
    double dt = dt_fixed > 0.0 ? dt_fixed : orc_dt(c, U, cfl);
    if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
    s.step(U, dt);
    t += dt;
    ++steps;
  }
  if (t_out) *t_out = t;
  return steps;
}

/* Volume means: out = [E_k, eps, total mass, total x/y/z momentum, total
 * energy, volume].  E_k = <rho |u|^2 / 2>, eps = <mu |omega|^2> with the
 * vorticity from cell-centred 4th-order differences of the halo'd velocity. */
void orc_diag(const orc_case *c, const double *U, double *out) {
  Solver<double> s(*c);
  std::vector<double> K0(orc_nk(c) + 1, 0.0);
  s.K = K0.data();
  s.build_prims(U);
  double ek = 0.0, eps = 0.0, vol = 0.0, tot[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < s.n[2]; ++k)
    for (int j = 0; j < s.n[1]; ++j)
      for (int i = 0; i < s.n[0]; ++i) {
        double V = s.cell_volume(i, j, k);
        long b = s.bid(i, j, k), ci = s.cid(i, j, k);
        double rho = s.Q[0][b], u = s.Q[1][b], v = s.Q[2][b], w = s.Q[3][b];
        ek += V * 0.5 * rho * (u * u + v * v + w * w);
        if (s.nd == 3) {
          /* derivative of velocity component q along axis t at this cell */
          auto D = [&](int q, int t) { return s.dtan(q, 0, t, i, j, k); };
          double wx = D(3, 1) - D(2, 2);
          double wy = D(1, 2) - D(3, 0);
          double wz = D(2, 0) - D(1, 1);
          eps += V * s.MU[b] * (wx * wx + wy * wy + wz * wz);
        }
        for (int v2 = 0; v2 < s.nv; ++v2) tot[v2] += V * U[(long)v2 * s.ncell + ci];
        vol += V;
      }
  out[0] = ek / vol;
  out[1] = eps / vol;
  out[2] = tot[0];
  out[3] = tot[1];
  out[4] = s.nd >= 2 ? tot[2] : 0.0;
  out[5] = s.nd >= 3 ? tot[3] : 0.0;
  out[6] = tot[s.nd + 1];
  out[7] = vol;
}

double orc_cost_term(const orc_case *c, const double *U) {
  Solver<double> s(*c);
  return s.cost_term(U);
}

/* Gradient of the cost term with respect to U, one dual tangent per entry. */
void orc_cost_term_grad(const orc_case *c, const double *U, double *g) {
  long M = (long)(c->ndim + 2) * orc_ncells(c);
  Solver<Dual> s(*c);
  std::vector<Dual> Ud(M);
  copy_in(U, Ud.data(), M);
  for (long x = 0; x < M; ++x) {
    Ud[x].d = 1.0;
    g[x] = s.cost_term(Ud.data()).d;
    Ud[x].d = 0.0;
  }
}

/* Jacobian-vector product of one RK3 step with respect to (U, K). */
void orc_jvp_step(const orc_case *c, const double *K, const double *dK, const double *U,
                  const double *dU, double dt, double *U1, double *dU1) {
  long M = (long)(c->ndim + 2) * orc_ncells(c);
  int nk = orc_nk(c);
  Solver<Dual> s(*c);
  std::vector<Dual> Ud(M), Kd(nk + 1);
  for (long x = 0; x < M; ++x) Ud[x] = Dual(U[x], dU ? dU[x] : 0.0);
  for (int x = 0; x < nk; ++x) Kd[x] = Dual(K[x], dK ? dK[x] : 0.0);
  s.K = Kd.data();
  s.step(Ud.data(), dt);
  for (long x = 0; x < M; ++x) {
    U1[x] = Ud[x].v;
    dU1[x] = Ud[x].d;
  }
}

/* Vector-Jacobian product of one RK3 step: lam^T J, with J assembled column
 * by column from dual-number JVPs (tiny grids only). */
void orc_vjp_step(const orc_case *c, const double *K, const double *U, double dt,
                  const double *lam, double *lamU, double *lamK) {
  long M = (long)(c->ndim + 2) * orc_ncells(c);
  int nk = orc_nk(c);
  long ncol = M + nk;
#pragma omp parallel for schedule(dynamic)
  for (long col = 0; col < ncol; ++col) {
    Solver<Dual> s(*c);
    std::vector<Dual> Ud(M), Kd(nk + 1);
    for (long x = 0; x < M; ++x) Ud[x] = Dual(U[x], x == col ? 1.0 : 0.0);
    for (int x = 0; x < nk; ++x) Kd[x] = Dual(K[x], (M + x) == col ? 1.0 : 0.0);
    s.K = Kd.data();
    s.step(Ud.data(), dt);
    double acc = 0.0;
    for (long x = 0; x < M; ++x) acc += lam[x] * Ud[x].d;
    if (col < M)
      lamU[col] = acc;
    else
      lamK[col - M] = acc;
  }
}

/* J = (1/Nt) sum_{n=1..Nt} cost_term(U^n) over a fixed-dt trajectory and its
 * gradient with respect to K and U^0 by reverse accumulation of dense VJPs. */
double orc_gradient(const orc_case *c, const double *K, const double *U0, int nsteps,
                    double dt, double *dJdK, double *dJdU0) {
  long M = (long)(c->ndim + 2) * orc_ncells(c);
  int nk = orc_nk(c);
  std::vector<std::vector<double>> traj(nsteps + 1, std::vector<double>(M));
  std::memcpy(traj[0].data(), U0, sizeof(double) * M);
  double J = 0.0;
  for (int s = 1; s <= nsteps; ++s) {
    traj[s] = traj[s - 1];
    orc_step(c, K, traj[s].data(), dt);
    J += orc_cost_term(c, traj[s].data()) / nsteps;
  }
  std::vector<double> lam(M), g(M), lamU(M), lamK(nk + 1);
  for (int x = 0; x < nk; ++x) dJdK[x] = 0.0;
  orc_cost_term_grad(c, traj[nsteps].data(), g.data());
  for (long x = 0; x < M; ++x) lam[x] = g[x] / nsteps;
  for (int s = nsteps; s >= 1; --s) {
    orc_vjp_step(c, K, traj[s - 1].data(), dt, lam.data(), lamU.data(), lamK.data());
    for (int x = 0; x < nk; ++x) dJdK[x] += lamK[x];
    if (s - 1 >= 1) {
      orc_cost_term_grad(c, traj[s - 1].data(), g.data());
      for (long x = 0; x < M; ++x) lam[x] = lamU[x] + g[x] / nsteps;
    } else {
      for (long x = 0; x < M; ++x) lam[x] = lamU[x];
    }
  }
  std::memcpy(dJdU0, lam.data(), sizeof(double) * M);
  return J;
}

int orc_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}

} /* extern "C" */
