// dcf_common.hpp -- device-side data structures and the per-face numerics of
// the finite-volume compressible Navier-Stokes right-hand side (gfx950, FP64).
//
// Paper correspondence:
//   conserved vector and total energy ............ Section 2.1, Eq. (2)
//   convective fluxes F^c, G^c, H^c ................ Eq. (3)
//   dissipative fluxes (stress, heat flux) ......... Eqs. (4)-(5), Fourier law
//   semi-discrete update with cell widths .......... Eq. (6)
//   WENO-type reconstruction + HLLC Riemann solver . Section 2.1 / Section 3.1
//   halo-cell boundary conditions .................. Section 3.2
// Schemes named but not written out in the paper use their published
// definitions: WENO5-JS (Jiang & Shu 1996, eps = 1e-6, power 2), HLLC
// (Toro, Spruce & Speares 1994) with Davis wave speeds, 4th-order central
// differences for the dissipative fluxes, and three-stage TVD Runge-Kutta
// (Shu & Osher 1988).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dcf {

constexpr int NH = 3;  // halo layers per active axis (Section 2.2)

enum : int {
  BC_PERIODIC = 0, BC_WALL = 1, BC_POROUS = 2, BC_ZEROGRAD = 3, BC_DIRICHLET = 4, BC_DISTURB = 5
};
__host__ __device__ __forceinline__ bool is_wall(int k) {
  return k == BC_WALL || k == BC_POROUS || k == BC_DISTURB;
}
enum : int { VISC_NONE = 0, VISC_POWER = 1, VISC_SUTHERLAND = 2 };
enum : int { SRC_NONE = 0, SRC_MASSFLUX = 1 };
enum : int { SCHEME_WENO5 = 0, SCHEME_TENO6A = 1 };
enum : int { QR = 0, QU = 1, QV = 2, QW = 3, QP = 4, QT = 5, QMU = 6, NQ = 7 };

// Everything a kernel needs about one solve, passed by value.
struct Dev {
  int ndim, nv;
  int n[3], h[3], N[3];  // interior cells, halo layers, box cells per axis
  int ho[3];             // array index of interior cell 0 along each axis
  long ncell, nbox;      // interior cells; box cells (N0 N1 N2)
  long nboxp;            // elements of one box array (rows padded to 16 doubles)
  long sb[3];            // box strides per axis
  // grid metrics per axis (device arrays): widths, 1/width, dxi/dx at
  // centres (n) and at faces (n+1)
  const double *dx[3], *idx[3], *mc[3], *mf[3];
  const double *xm[3];   // cell-centre coordinates (midpoint of the two faces)
  double Lx;             // the x cell widths summed in index order (an x line's length)
  // gas
  double gamma, R, Pr, cp, mu_ref, T_ref, vparam;
  double gm1i, cpPr;     // 1/(gamma - 1) and cp/Pr
  double iR, iTref;      // 1/R and 1/T_ref
  int visc;
  // boundaries
  int bck[6];
  double Tw[6];          // wall temperature; 0 = adiabatic wall
  int doff[6];           // disturbance wall: offset of (A, kappa) in K, else -1
  const double *dir[6];
  int pface, pb, pe;
  double pinf;
  const double *K;       // boundary parameters: porous K_i, then (A, kappa) per disturbance face
  int source;
  // workspace
  double *Q[NQ];         // primitive box arrays
  double *F[3];          // face fluxes per direction, 5 components each
  long fcount[3];        // faces per direction (component stride of F)
  int fn[3][3];          // face-array extents per direction
  unsigned *flags;
  int scheme;            // SCHEME_WENO5 or SCHEME_TENO6A (face reconstruction and
                         // order of the central dissipative stencils)
};

// Primitive box arrays a kernel writes besides its main output (null Q[0]:
// none).
struct BoxOut {
  double *Q[NQ] = {};
};

__device__ __forceinline__ bool finite_pos(double x) { return x > 0.0 && x < 1.0e300; }

// Box arrays: interior cell 0 of each row sits on a 128-byte boundary (x
// offset 16 doubles, row pitch a multiple of 16), so tiles of 16 cells along
// x load whole cache lines.
__host__ __device__ __forceinline__ long bidx(const Dev &g, int i, int j, int k) {
  return (long)(k + g.ho[2]) * g.sb[2] + (long)(j + g.ho[1]) * g.sb[1] + (i + g.ho[0]);
}

// Box position of ghost cell number gi (ghost cells enumerated z-plane by
// z-plane: whole halo planes, then per interior plane its halo rows and the
// 2 h0 x-halo cells of each interior row).
__host__ __device__ __forceinline__ void ghost_position(const Dev &g, unsigned gi, int p[3]) {
  const unsigned N0 = g.N[0], h0 = g.h[0], h1 = g.h[1], h2 = g.h[2];
  const unsigned n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const unsigned plane = N0 * (unsigned)g.N[1];
  const unsigned lowz = h2 * plane, inner = plane - n0 * n1;
  unsigned x, y, z;
  if (gi < lowz || gi >= lowz + n2 * inner) {  // a whole halo plane
    const unsigned r0 = gi < lowz ? gi : gi - n2 * inner;
    z = r0 / plane;
    if (gi >= lowz) z += n2;
    const unsigned r = r0 % plane;
    y = r / N0;
    x = r % N0;
  } else {
    const unsigned r0 = gi - lowz;
    z = h2 + r0 / inner;
    unsigned r = r0 % inner;
    const unsigned lowy = h1 * N0, mid = 2u * h0;
    if (r < lowy) {
      y = r / N0;
      x = r % N0;
    } else if (r < lowy + n1 * mid) {
      r -= lowy;
      y = h1 + r / mid;
      const unsigned m = r % mid;
      x = m < h0 ? m : n0 + m;
    } else {
      r -= lowy + n1 * mid;
      y = h1 + n1 + r / N0;
      x = r % N0;
    }
  }
  p[0] = (int)x - g.h[0];
  p[1] = (int)y - g.h[1];
  p[2] = (int)z - g.h[2];
}

// Reciprocal from the hardware estimate refined by two Newton-Raphson steps
// e = 1 - x r, r <- r + r e (each squares the relative error): within about
// an ulp of 1/x for normal x, at half the instructions of an IEEE division.
// Zero or non-finite x gives a non-finite result.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/sqrt(x) for normal x > 0, likewise: the hardware estimate and two Newton
// steps y <- y + y (1 - x y^2) / 2.  Negative x gives NaN.
__device__ __forceinline__ double rsq_nr(double x) {
  const double hx = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  y = fma(y, fma(-hx * y, y, 0.5), y);
  return fma(y, fma(-hx * y, y, 0.5), y);
}

// Sound speed c = sqrt(gamma p / rho), written gamma p y with
// y = 1 / sqrt(gamma p rho) = 1 / (rho c) so that it needs no division.
__device__ __forceinline__ double sound_speed(double gamma, double rho, double p, double &y) {
  const double gp = gamma * p;
  y = rsq_nr(gp * rho);
  return gp * y;
}
__device__ __forceinline__ double sound_speed(double gamma, double rho, double p) {
  double y;
  return sound_speed(gamma, rho, p, y);
}

// Dynamic viscosity: power law, or Sutherland's law (Section 3.2).
__device__ __forceinline__ double viscosity(const Dev &g, double T) {
  // (T/T_ref)^omega as exp(omega log(T/T_ref)): a few ulp, half the cost of pow
  if (g.visc == VISC_POWER) return g.mu_ref * exp(g.vparam * log(T * g.iTref));
  if (g.visc == VISC_SUTHERLAND) {
    // t^{3/2} (1 + s) / (t + s) with t^{3/2} = t^2 / sqrt(t)
    double t = T * g.iTref;
    double s = g.vparam * g.iTref;
    return g.mu_ref * (1.0 + s) * (t * t * rsq_nr(t)) * rcp_nr(t + s);
  }
  return 0.0;
}

// WENO5-JS (Section 2.1): both reconstructions at the face between v2 and
// v3, left-biased from v0..v4 and right-biased from v5..v1.  The nonlinear
// weights d_k / (eps + beta_k)^2 are normalised after multiplying through by
// the product of the three denominators, and the two values share one
// reciprocal: y_L = N_L D_R r, y_R = N_R D_L r with r = 1 / (6 D_L D_R)
// (the candidates are kept at six times the third-order reconstructions).
// The mirrored stencils share work: the left stencils (1..3) and (2..4) are
// the right stencils (3..1) and (4..2), with the same second differences, and
// the left candidates 1 and 2 equal the right candidates 2 and 1.
__device__ __forceinline__ void weno5_pair(double v0, double v1, double v2, double v3, double v4,
                                           double v5, double &yl, double &yr) {
  const double eps = 1.0e-6;
  const double c1312 = 13.0 / 12.0;
  // second differences over cells (0,1,2), (1,2,3), (2,3,4), (3,4,5)
  const double d0 = v0 - 2.0 * v1 + v2, d1 = v1 - 2.0 * v2 + v3;
  const double d2 = v2 - 2.0 * v3 + v4, d3 = v3 - 2.0 * v4 + v5;
  // candidates: qa left 0, qb left 1 = right 2, qc left 2 = right 1, qd right 0
  const double qa = 2.0 * v0 - 7.0 * v1 + 11.0 * v2;
  const double qb = -v1 + 5.0 * v2 + 2.0 * v3;
  const double qc = 2.0 * v2 + 5.0 * v3 - v4;
  const double qd = 2.0 * v5 - 7.0 * v4 + 11.0 * v3;
  // first-derivative terms of the smoothness indicators, per side
  const double sl0 = v0 - 4.0 * v1 + 3.0 * v2, sl1 = v1 - v3, sl2 = 3.0 * v2 - 4.0 * v3 + v4;
  const double sr0 = v5 - 4.0 * v4 + 3.0 * v3, sr1 = v4 - v2, sr2 = 3.0 * v3 - 4.0 * v2 + v1;
  // u_k = (eps + beta_k)^2 / d_k, the square of (eps + beta_k) / sqrt(d_k)
  // with 1 / sqrt(d_k) folded into the constants (d = 0.1, 0.6, 0.3); the
  // weights d_k / (eps + beta_k)^2 times the product of all three
  // denominators are then the products of the other two u (the common
  // factor d_0 d_1 d_2 cancels in the normalisation)
  constexpr double is1 = 3.162277660168379, is6 = 1.2909944487358056,
                   is3 = 1.8257418583505538;  // 1 / sqrt(d_k)
  auto usq = [&](double r, double s, double sc) {
    const double t = fma(c1312 * sc * r, r, fma(0.25 * sc * s, s, eps * sc));
    return t * t;
  };
  const double ul0 = usq(d0, sl0, is1), ul1 = usq(d1, sl1, is6), ul2 = usq(d2, sl2, is3);
  const double ur0 = usq(d3, sr0, is1), ur1 = usq(d2, sr1, is6), ur2 = usq(d1, sr2, is3);
  const double wl0 = ul1 * ul2, wl1 = ul0 * ul2, wl2 = ul0 * ul1;
  const double wr0 = ur1 * ur2, wr1 = ur0 * ur2, wr2 = ur0 * ur1;
  const double nl = wl0 * qa + wl1 * qb + wl2 * qc, dl = wl0 + wl1 + wl2;
  const double nr = wr0 * qd + wr1 * qc + wr2 * qb, dr = wr0 + wr1 + wr2;
  const double r = rcp_nr(6.0 * dl * dr);
  yl = nl * dr * r;
  yr = nr * dl * r;
}

// HLLC flux in the face frame.  q = (rho, u_n, u_t1, u_t2, p) on each side;
// F = (mass, normal momentum, t1 momentum, t2 momentum, energy).  Ties at
// 0 <= S select the left-side state.  Star state written with one
// reciprocal r = 1/(S_K - S*):
//   U*_K = r [rho (S-u), rho (S-u) S*, rho (S-u) v, rho (S-u) w,
//             E (S-u) + (S*-u)(rho (S-u) S* + p)].
__device__ __forceinline__ void hllc(const double *qL, const double *qR, double gamma,
                                     double gm1i, double *F) {
  double rL = qL[0], uL = qL[1], vL = qL[2], wL = qL[3], pL = qL[4];
  double rR = qR[0], uR = qR[1], vR = qR[2], wR = qR[3], pR = qR[4];
  double EL = pL * gm1i + 0.5 * rL * (uL * uL + vL * vL + wL * wL);
  double ER = pR * gm1i + 0.5 * rR * (uR * uR + vR * vR + wR * wR);
  double cL = sound_speed(gamma, rL, pL);
  double cR = sound_speed(gamma, rR, pR);
  double SL = fmin(uL - cL, uR - cR);
  double SR = fmax(uL + cL, uR + cR);
  double mL = rL * (SL - uL), mR = rR * (SR - uR);
  double Ss = (pR - pL + uL * mL - uR * mR) * rcp_nr(mL - mR);
  if (0.0 <= SL) {
    F[0] = rL * uL;
    F[1] = rL * uL * uL + pL;
    F[2] = rL * uL * vL;
    F[3] = rL * uL * wL;
    F[4] = uL * (EL + pL);
    return;
  }
  if (SR < 0.0) {
    F[0] = rR * uR;
    F[1] = rR * uR * uR + pR;
    F[2] = rR * uR * vR;
    F[3] = rR * uR * wR;
    F[4] = uR * (ER + pR);
    return;
  }
  const bool left = (0.0 <= Ss);
  double r = left ? rL : rR, u = left ? uL : uR, v = left ? vL : vR, w = left ? wL : wR;
  double p = left ? pL : pR, E = left ? EL : ER, S = left ? SL : SR, m = left ? mL : mR;
  double inv = rcp_nr(S - Ss);
  double Us0 = m * inv;
  double Us4 = (E * (S - u) + (Ss - u) * (m * Ss + p)) * inv;
  double fm = r * u;
  F[0] = fm + S * (Us0 - r);
  F[1] = fm * u + p + S * (Us0 * Ss - fm);
  F[2] = fm * v + S * (Us0 * v - r * v);
  F[3] = fm * w + S * (Us0 * w - r * w);
  F[4] = u * (E + p) + S * (Us4 - E);
}

// TENO6-A (Fu, Hu & Adams: targeted ENO, six points, adaptive dissipation):
// both reconstructions at the face between v2 and v3, the left one centred on
// v2 (cells v0 .. v5) and the right one its mirror image centred on v3 (cells
// v5 .. v0).  Per side, with (a .. f) the six cells and c the centre:
// third-order candidates on (b c d), (c d e) and (a b c) and a fourth-order
// one on (c d e f), sixth-order linear weights (0.45, 0.3, 0.05, 0.2); the
// Jiang-Shu indicators of the candidates and of the six-point polynomial
// (integrals over the centre cell) give tau6 = |b6 - (b0 + b2 + 4 b1) / 6|
// and the measures gamma_k = (1 + tau6 / (b_k + 1e-40))^6; a candidate whose
// share gamma_k / sum gamma is below the cut-off C_T is dropped (tested as
// gamma_k < C_T sum gamma), the kept ones are combined with their linear
// weights renormalised.
// C_T = 10^-floor(10.5 - 3.5 (1 - (1-m)^4 (1+4m))), m = 1 - min(1, eta/0.17),
// eta the smallest of Ren's measures (|2 a b| + e) / (a^2 + b^2 + e) over the
// neighbouring differences (a, b) of the four inner cells,
// e = 0.9 * 0.17 * (1e-3)^2 / (1 - 0.9 * 0.17); the mirrored differences give
// the same measures, so C_T is shared by both sides.  Reciprocals are the
// refined hardware ones (no IEEE division).
__device__ __forceinline__ void teno6a_pair(double v0, double v1, double v2, double v3, double v4,
                                            double v5, double &yl, double &yr) {
  double ct;
  {
    const double Cr = 0.17, xi = 1.0e-3;
    const double ee = 0.9 * Cr * xi * xi / (1.0 - 0.9 * Cr);
    const double d0 = v1 - v0, d1 = v2 - v1, d2 = v3 - v2, d3 = v4 - v3, d4 = v5 - v4;
    auto ren = [&](double dm, double dp) {
      return (fabs(2.0 * dp * dm) + ee) * rcp_nr(fma(dp, dp, fma(dm, dm, ee)));
    };
    const double eta = fmin(fmin(ren(d0, d1), ren(d1, d2)), fmin(ren(d2, d3), ren(d3, d4)));
    const double m = 1.0 - fmin(1.0, eta * (1.0 / Cr));
    const double om = 1.0 - m, om2 = om * om;
    const double bbar = 10.5 - 3.5 * (1.0 - om2 * om2 * (1.0 + 4.0 * m));
    const int k = (int)floor(bbar);
    ct = k >= 10 ? 1.0e-10 : (k == 9 ? 1.0e-9 : (k == 8 ? 1.0e-8 : 1.0e-7));
  }
  auto side = [ct](double a, double b, double c, double d, double e, double f) {
    constexpr double c1312 = 13.0 / 12.0;
    const double s0 = b - 2.0 * c + d, t0 = b - d;
    const double s1 = c - 2.0 * d + e, t1 = 3.0 * c - 4.0 * d + e;
    const double s2 = a - 2.0 * b + c, t2 = a - 4.0 * b + 3.0 * c;
    const double b0 = fma(c1312 * s0, s0, 0.25 * t0 * t0);
    const double b1 = fma(c1312 * s1, s1, 0.25 * t1 * t1);
    const double b2 = fma(c1312 * s2, s2, 0.25 * t2 * t2);
    const double b3 = (c * (2107.0 * c - 9402.0 * d + 7042.0 * e - 1854.0 * f) +
                       d * (11003.0 * d - 17246.0 * e + 4642.0 * f) +
                       e * (7043.0 * e - 3882.0 * f) + 547.0 * f * f) * (1.0 / 240.0);
    const double b6 =
        (a * (271779.0 * a - 2380800.0 * b + 4086352.0 * c - 3462252.0 * d + 1458762.0 * e -
              245620.0 * f) +
         b * (5653317.0 * b - 20427884.0 * c + 17905032.0 * d - 7727988.0 * e +
              1325006.0 * f) +
         c * (19510972.0 * c - 35817664.0 * d + 15929912.0 * e - 2792660.0 * f) +
         d * (17195652.0 * d - 15880404.0 * e + 2863984.0 * f) +
         e * (3824847.0 * e - 1429976.0 * f) + 139633.0 * f * f) * (1.0 / 120960.0);
    const double tau = fabs(b6 - (b0 + b2 + 4.0 * b1) * (1.0 / 6.0));
    auto gam = [tau](double beta) {
      const double r = fma(tau, rcp_nr(beta + 1.0e-40), 1.0);
      const double r2 = r * r;
      return r2 * r2 * r2;
    };
    const double g0 = gam(b0), g1 = gam(b1), g2 = gam(b2), g3 = gam(b3);
    const double lim = ct * (g0 + g1 + g2 + g3);
    const double w0 = g0 < lim ? 0.0 : 0.45, w1 = g1 < lim ? 0.0 : 0.3;
    const double w2 = g2 < lim ? 0.0 : 0.05, w3 = g3 < lim ? 0.0 : 0.2;
    // candidates: (b c d), (c d e), (a b c), (c d e f)
    const double q0 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
    const double q1 = (2.0 * c + 5.0 * d - e) * (1.0 / 6.0);
    const double q2 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
    const double q3 = (3.0 * c + 13.0 * d - 5.0 * e + f) * (1.0 / 12.0);
    return (w0 * q0 + w1 * q1 + w2 * q2 + w3 * q3) * rcp_nr(w0 + w1 + w2 + w3);
  };
  yl = side(v0, v1, v2, v3, v4, v5);
  yr = side(v5, v4, v3, v2, v1, v0);
}

// 6th-order central interpolation and derivatives in index space: face value
// and face derivative from the six cells around a face, cell derivative from
// three cells either side.
__device__ __forceinline__ double interp6(double a, double b, double c, double d, double e,
                                          double f) {
  return (150.0 * (c + d) - 25.0 * (b + e) + 3.0 * (a + f)) * (1.0 / 256.0);
}
__device__ __forceinline__ double dface6(double a, double b, double c, double d, double e,
                                         double f) {
  return (2250.0 * (d - c) - 125.0 * (e - b) + 9.0 * (f - a)) * (1.0 / 1920.0);
}
__device__ __forceinline__ double dcell6(double m3, double m2, double m1, double p1, double p2,
                                         double p3) {
  return (45.0 * (p1 - m1) - 9.0 * (p2 - m2) + (p3 - m3)) * (1.0 / 60.0);
}

// 4th-order central interpolation and derivatives in index space.
__device__ __forceinline__ double interp4(double a, double b, double c, double d) {
  return (9.0 * (b + c) - (a + d)) * (1.0 / 16.0);
}
__device__ __forceinline__ double dface4(double a, double b, double c, double d) {
  return (27.0 * (c - b) - (d - a)) * (1.0 / 24.0);
}
__device__ __forceinline__ double dcell4(double m2, double m1, double p1, double p2) {
  return (8.0 * (p1 - m1) - (p2 - m2)) * (1.0 / 12.0);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  This bijection of [0, nb) gives XCD x a contiguous range of logical
// tile indices, so neighbouring tiles that share halo cells meet in one L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned L, unsigned nb) {
  const unsigned x = L % 8u, i = L / 8u, per = nb / 8u, rem = nb % 8u;
  return x < rem ? x * (per + 1u) + i : rem * (per + 1u) + (x - rem) * per + i;
}

// As xcd_remap, but spreading chunks of C consecutive logical tiles round
// robin over the XCDs (chunk k on XCD k mod 8): tiles of one chunk share an
// L2 while the work of any region is spread over all XCDs.  Blocks past the
// last whole round of 8 chunks keep their index.
__device__ __forceinline__ unsigned xcd_chunk_remap(unsigned P, unsigned nb, unsigned C) {
  const unsigned full = nb / (8u * C) * (8u * C);
  if (P >= full) return P;
  const unsigned x = P % 8u, i = P / 8u;
  return ((i / C) * 8u + x) * C + i % C;
}

__host__ __device__ __forceinline__ constexpr int tan1(int d) { return d == 0 ? 1 : 0; }
__host__ __device__ __forceinline__ constexpr int tan2(int d) { return d == 2 ? 1 : 2; }

}  // namespace dcf
