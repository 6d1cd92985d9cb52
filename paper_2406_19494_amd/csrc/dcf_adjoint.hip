// dcf_adjoint.hip -- hand-written reverse mode (VJP) of one TVD-RK3 step of
// the finite-volume right-hand side (Eq. (6)), through the halo-cell boundary
// conditions including the differentiable porous wall (Section 3.2), so that
// gradients of a cost along a trajectory reach the wall parameters (the
// end-to-end optimisation of Section 1).
//
// Per stage (state V, stage output W = a Un + b (V + dt R(V))), given the
// stage-output adjoint Wb:
//   Rb = b dt Wb,  Fb(face) = Rb(right cell)/dx - Rb(left cell)/dx (formed
//                  per face from Wb inside the flux adjoint kernels),
//   Qb = sum over faces of (dF/dQ)^T Fb        (convective + dissipative),
//   Qb += D_t^T Gb   (tangential derivatives were cell-centred, then
//                     interpolated: their adjoint Gb is gathered along t),
//   Tb += mu'(T) mub, then the halo fill is transposed axis by axis in the
//   reverse order z, y, x (ghost adjoints fold into their sources and, for
//   the porous wall, into dJ/dK), and Vb = b Wb + (dQ/dU)^T Qb.
// Every scatter of the reverse pass is done as a deterministic gather: face
// adjoints are accumulated in LDS tiles offset by offset (one writer per
// cell per phase), and the tile only writes the cells all of whose faces it
// computed; no atomics anywhere, so results are bitwise reproducible.
#include "dcf_adjoint.hpp"
#include "dcf_kernels.hpp"

namespace dcf {

// Tile shape of direction D (TF faces per line x TW lines = 256 threads):
// x-faces run along the lanes (64 x 4); y and z tiles take 8 neighbouring
// x-lines so that a cell row is read and written in 64-byte segments
// (32 x 8, at the price of more faces recomputed at tile edges).
template <int D> struct TileShape {
  static constexpr int TF = D == 0 ? 64 : 32;
  static constexpr int TW = 256 / TF;
};
__host__ inline int tile_faces(int D) { return D == 0 ? 64 : 32; }

// ---------------------------------------------------------------------------
// Reverse of WENO5-JS: g[0..4] += d y / d (a..e) * yb.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void weno5_vjp(double a, double b, double c, double d, double e,
                                          double yb, double *g) {
  // the forward in the form the face flux evaluates it: t_k = (eps +
  // beta_k) / sqrt(d_k), u_k = t_k^2, weights w_k = u_i u_j (i, j != k),
  // candidates q_k at six times the third-order values, y = N / (6 W)
  const double eps = 1.0e-6;
  const double c1312 = 13.0 / 12.0;
  constexpr double is1 = 3.162277660168379, is6 = 1.2909944487358056,
                   is3 = 1.8257418583505538;  // 1 / sqrt(d_k), d = 0.1, 0.6, 0.3
  double q0 = 2.0 * a - 7.0 * b + 11.0 * c;
  double q1 = -b + 5.0 * c + 2.0 * d;
  double q2 = 2.0 * c + 5.0 * d - e;
  double r0 = a - 2.0 * b + c, s0 = a - 4.0 * b + 3.0 * c;
  double r1 = b - 2.0 * c + d, s1 = b - d;
  double r2 = c - 2.0 * d + e, s2 = 3.0 * c - 4.0 * d + e;
  double t0 = fma(c1312 * is1 * r0, r0, fma(0.25 * is1 * s0, s0, eps * is1));
  double t1 = fma(c1312 * is6 * r1, r1, fma(0.25 * is6 * s1, s1, eps * is6));
  double t2 = fma(c1312 * is3 * r2, r2, fma(0.25 * is3 * s2, s2, eps * is3));
  double u0 = t0 * t0, u1 = t1 * t1, u2 = t2 * t2;
  double w0 = u1 * u2, w1 = u0 * u2, w2 = u0 * u1;
  double iW = rcp_nr(6.0 * (w0 + w1 + w2));
  double y6 = 6.0 * ((w0 * q0 + w1 * q1 + w2 * q2) * iW);
  double Nb = yb * iW;
  double q0b = Nb * w0, q1b = Nb * w1, q2b = Nb * w2;
  double w0b = Nb * (q0 - y6), w1b = Nb * (q1 - y6), w2b = Nb * (q2 - y6);
  double u0b = w1b * u2 + w2b * u1;
  double u1b = w0b * u2 + w2b * u0;
  double u2b = w0b * u1 + w1b * u0;
  double t0b = 2.0 * t0 * u0b, t1b = 2.0 * t1 * u1b, t2b = 2.0 * t2 * u2b;
  // d t_k / d r_k = 2 (13/12) r_k / sqrt(d_k), d t_k / d s_k = s_k / (2 sqrt(d_k))
  double r0b = (2.0 * c1312 * is1) * r0 * t0b, s0b = (0.5 * is1) * s0 * t0b;
  double r1b = (2.0 * c1312 * is6) * r1 * t1b, s1b = (0.5 * is6) * s1 * t1b;
  double r2b = (2.0 * c1312 * is3) * r2 * t2b, s2b = (0.5 * is3) * s2 * t2b;
  g[0] += 2.0 * q0b + r0b + s0b;
  g[1] += -7.0 * q0b - q1b - 2.0 * r0b - 4.0 * s0b + r1b + s1b;
  g[2] += 11.0 * q0b + 5.0 * q1b + 2.0 * q2b + r0b + 3.0 * s0b - 2.0 * r1b + r2b + 3.0 * s2b;
  g[3] += 2.0 * q1b + 5.0 * q2b + r1b - s1b - 2.0 * r2b - 4.0 * s2b;
  g[4] += -q2b + r2b + s2b;
}

// Reverse of the physical flux of one state (Eq. (3), face frame).
__device__ __forceinline__ void phys_flux_vjp(const double *q, double gm1i, const double *Fb,
                                              double *qb) {
  double r = q[0], u = q[1], v = q[2], w = q[3], p = q[4];
  double k2 = u * u + v * v + w * w;
  double E = p * gm1i + 0.5 * r * k2;
  double Eb = Fb[4] * u;
  qb[0] += Fb[0] * u + Fb[1] * u * u + Fb[2] * u * v + Fb[3] * u * w + Eb * 0.5 * k2;
  qb[1] += Fb[0] * r + 2.0 * Fb[1] * r * u + Fb[2] * r * v + Fb[3] * r * w + Fb[4] * (E + p) +
           Eb * r * u;
  qb[2] += Fb[2] * r * u + Eb * r * v;
  qb[3] += Fb[3] * r * u + Eb * r * w;
  qb[4] += Fb[1] + Fb[4] * u + Eb * gm1i;
}

// Reverse of the HLLC flux (same branch choices as the forward: Davis wave
// speeds with the left candidate kept on ties, 0 <= S selects the left side).
__device__ void hllc_vjp(const double *qL, const double *qR, double gamma, double gm1i,
                         const double *Fb, double *qLb, double *qRb) {
  double rL = qL[0], uL = qL[1], vL = qL[2], wL = qL[3], pL = qL[4];
  double rR = qR[0], uR = qR[1], vR = qR[2], wR = qR[3], pR = qR[4];
  double EL = pL * gm1i + 0.5 * rL * (uL * uL + vL * vL + wL * wL);
  double ER = pR * gm1i + 0.5 * rR * (uR * uR + vR * vR + wR * wR);
  // wave speeds, star speed and star reciprocal in the forward's arithmetic
  // (same branch decisions)
  double yL, yR;  // 1 / (rho c) per side
  double cL = sound_speed(gamma, rL, pL, yL);
  double cR = sound_speed(gamma, rR, pR, yR);
  double aL = uL - cL, bL = uR - cR;
  const bool selL = bL < aL;
  double SL = selL ? bL : aL;
  double aR = uL + cL, bR = uR + cR;
  const bool selR = bR > aR;
  double SR = selR ? bR : aR;
  for (int m = 0; m < 5; ++m) qLb[m] = qRb[m] = 0.0;
  if (0.0 <= SL) {
    phys_flux_vjp(qL, gm1i, Fb, qLb);
    return;
  }
  if (SR < 0.0) {
    phys_flux_vjp(qR, gm1i, Fb, qRb);
    return;
  }
  double mL = rL * (SL - uL), mR = rR * (SR - uR);
  double Nn = pR - pL + uL * mL - uR * mR, Dd = mL - mR;
  const double iDd = rcp_nr(Dd);
  double Ss = Nn * iDd;
  const bool left = (0.0 <= Ss);
  double r = left ? rL : rR, u = left ? uL : uR, v = left ? vL : vR, w = left ? wL : wR;
  double p = left ? pL : pR, E = left ? EL : ER, S = left ? SL : SR, m = left ? mL : mR;
  double inv = rcp_nr(S - Ss);
  double Us0 = m * inv;
  double A4 = m * Ss + p;
  double N4 = E * (S - u) + (Ss - u) * A4;
  double Us4 = N4 * inv;
  double fm = r * u;
  const double F0 = Fb[0], F1 = Fb[1], F2 = Fb[2], F3 = Fb[3], F4 = Fb[4];
  double Sb = F0 * (Us0 - r) + F1 * (Us0 * Ss - fm) + F2 * (Us0 * v - r * v) +
              F3 * (Us0 * w - r * w) + F4 * (Us4 - E);
  double Us0b = S * (F0 + F1 * Ss + F2 * v + F3 * w);
  double Ssb = F1 * S * Us0;
  double Us4b = S * F4;
  double fmb = F0 + F1 * (u - S) + F2 * v + F3 * w;
  double rb = -S * (F0 + F2 * v + F3 * w);
  double ub = F1 * fm + F4 * (E + p);
  double vb = F2 * (fm + S * Us0 - S * r);
  double wb = F3 * (fm + S * Us0 - S * r);
  double pb = F1 + F4 * u;
  double Eb = F4 * (u - S);
  double N4b = Us4b * inv, invb = Us4b * N4;
  Eb += N4b * (S - u);
  Sb += N4b * E;
  ub -= N4b * (E + A4);
  Ssb += N4b * (A4 + (Ss - u) * m);
  double mb = N4b * (Ss - u) * Ss;
  pb += N4b * (Ss - u);
  mb += Us0b * inv;
  invb += Us0b * m;
  double db = -invb * inv * inv;
  Sb += db;
  Ssb -= db;
  rb += fmb * u;
  ub += fmb * r;
  pb += Eb * gm1i;
  rb += Eb * 0.5 * (u * u + v * v + w * w);
  ub += Eb * r * u;
  vb += Eb * r * v;
  wb += Eb * r * w;
  double *qKb = left ? qLb : qRb;
  qKb[0] += rb;
  qKb[1] += ub;
  qKb[2] += vb;
  qKb[3] += wb;
  qKb[4] += pb;
  double mLb = left ? mb : 0.0, mRb = left ? 0.0 : mb;
  double SLb = left ? Sb : 0.0, SRb = left ? 0.0 : Sb;
  double Nnb = Ssb * iDd, Ddb = -Ssb * Ss * iDd;
  qRb[4] += Nnb;
  qLb[4] -= Nnb;
  qLb[1] += Nnb * mL;
  mLb += Nnb * uL + Ddb;
  qRb[1] -= Nnb * mR;
  mRb += -Nnb * uR - Ddb;
  qLb[0] += mLb * (SL - uL);
  SLb += mLb * rL;
  qLb[1] -= mLb * rL;
  qRb[0] += mRb * (SR - uR);
  SRb += mRb * rR;
  qRb[1] -= mRb * rR;
  double cLb = 0.0, cRb = 0.0;
  if (selL) {
    qRb[1] += SLb;
    cRb -= SLb;
  } else {
    qLb[1] += SLb;
    cLb -= SLb;
  }
  if (selR) {
    qRb[1] += SRb;
    cRb += SRb;
  } else {
    qLb[1] += SRb;
    cLb += SRb;
  }
  // c = sqrt(gamma p / rho): dc/dp = gamma / (2 rho c) = gamma y / 2 and
  // dc/drho = -c / (2 rho) = -c^2 y / 2
  qLb[4] += cLb * (0.5 * gamma) * yL;
  qLb[0] -= cLb * (0.5 * cL * cL) * yL;
  qRb[4] += cRb * (0.5 * gamma) * yR;
  qRb[0] -= cRb * (0.5 * cR * cR) * yR;
}

// Flux adjoint at face f of direction D from the stage-output adjoint Wb:
// with Rb = b dt Wb (the right-hand-side adjoint, 5-component flux layout),
// Fb[m] = Rb_m(cell f)/dx_f - Rb_m(cell f-1)/dx_{f-1}.  (With the body
// force A.Wb is the copy k_force_adj_apply corrected.)
template <int NDIM>
__device__ __forceinline__ void face_adjoint(const Dev &g, const AdjBuffers &A, int D,
                                             const int *pos, int f, double *Fb) {
  const long nc = g.ncell;
  const double s = A.bcoef * A.dtp[0];
  const long vo[5] = {0, nc, 2 * nc, 3 * nc, (long)(NDIM + 1) * nc};
  // both cells' loads are issued unconditionally (at clamped positions, in
  // bounds) and together; only the sums depend on the cell existing
  const bool hr = f < g.n[D], hl = f >= 1;
  int cpos[3] = {pos[0], pos[1], pos[2]};
  cpos[D] = hr ? f : g.n[D] - 1;
  const long cr = ((long)cpos[2] * g.n[1] + cpos[1]) * g.n[0] + cpos[0];
  cpos[D] = hl ? f - 1 : 0;
  const long cl = ((long)cpos[2] * g.n[1] + cpos[1]) * g.n[0] + cpos[0];
  const double idr = g.idx[D][hr ? f : g.n[D] - 1], idl = g.idx[D][hl ? f - 1 : 0];
  double wr[5], wl[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const bool on = m < 2 || m == 4 || m <= NDIM;
    wr[m] = on ? A.Wb[vo[m] + cr] : 0.0;
    wl[m] = on ? A.Wb[vo[m] + cl] : 0.0;
  }
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    Fb[m] = 0.0;
    if (!(m < 2 || m == 4 || m <= NDIM)) continue;
    const double r = Fb[m] + (s * wr[m]) * idr;
    Fb[m] = hr ? r : Fb[m];
    const double l = Fb[m] - (s * wl[m]) * idl;
    Fb[m] = hl ? l : Fb[m];
  }
}

// Tile geometry for direction D: tile index -> first face and line origin.
struct Tile {
  int f0;       // first face of the tile along D
  int c0, c1;   // cells written by the tile along D: [c0, c1)
  int line[3];  // tangential position of this thread's line (pos[D] unused)
  int lane_line, lane_face;
  long lg;      // line group of the tile
  bool line_ok;
  bool valid;   // the workgroup has a tile
};

// P: the workgroup's index among the nb workgroups of direction D (the
// hardware index modulo 8 must equal P modulo 8: the XCD order below assumes
// it); t.valid is false for workgroups beyond the direction's tile count
template <int OLO, int OHI, int D>
__device__ __forceinline__ Tile make_tile(const Dev &g, unsigned P, unsigned nb) {
  constexpr int TF = TileShape<D>::TF, TW = TileShape<D>::TW;
  constexpr int SPAN = OHI - OLO;
  constexpr int CPT = TF - SPAN;  // cells completed per tile line
  const int T1 = tan1(D), T2 = tan2(D);
  const int nt1 = g.n[T1], nt2 = g.n[T2];
  const int cmin = OLO;                         // first cell receiving contributions
  const int ncell_line = g.n[D] + 1 + SPAN;     // cells [OLO, n + OHI]
  const int tiles_d = (ncell_line + CPT - 1) / CPT;
  const long lines = (long)nt1 * nt2;
  // y/z tiles: the two line groups that share each 128-byte row segment (and
  // the tiles along D of both, which share halo rows) run on one XCD, with
  // such chunks dealt round robin so that every XCD gets wall and free-stream
  // regions alike; x tiles keep the hardware order
  long tile = D == 0 ? P : xcd_chunk_remap(P, nb, 2u * tiles_d);
  int td = (int)(tile % tiles_d);
  long lg = tile / tiles_d;  // line group
  Tile t;
  t.valid = tile < (long)tiles_d * ((lines + TW - 1) / TW);
  const int tid = threadIdx.x;
  if (D == 0) {
    t.lane_face = tid % TF;
    t.lane_line = tid / TF;
  } else {
    t.lane_line = tid % TW;
    t.lane_face = tid / TW;
  }
  long ln = lg * TW + t.lane_line;  // line index over (t1 fastest, t2)
  t.line_ok = ln < lines;
  int a = t.line_ok ? (int)(ln % nt1) : 0;
  int bq = t.line_ok ? (int)(ln / nt1) : 0;
  t.line[D] = 0;
  t.line[T1] = a;
  t.line[T2] = bq;
  t.c0 = cmin + td * CPT;
  t.c1 = min(t.c0 + CPT, g.n[D] + OHI + 1);
  t.f0 = t.c0 - OHI;
  t.lg = lg;
  return t;
}

template <int OLO, int OHI>
__host__ inline unsigned tile_count(const Dev &g, int D) {
  const int TF = tile_faces(D), TW = 256 / TF;
  constexpr int SPAN = OHI - OLO;
  const int CPT = TF - SPAN;
  const int ncell_line = g.n[D] + 1 + SPAN;
  const long tiles_d = (ncell_line + CPT - 1) / CPT;
  const long lines = (long)g.n[tan1(D)] * g.n[tan2(D)];
  return (unsigned)(tiles_d * ((lines + TW - 1) / TW));
}

// ---------------------------------------------------------------------------
// Adjoint of the fluxes along D, one tile of faces per workgroup:
//  * convective: WENO5-JS + HLLC reversed per face, contributions to the
//    cells f-3 .. f+2 (rho, velocity, p);
//  * dissipative (VISC): the face stress / heat flux reversed to face-level
//    adjoints, expanded over the cells f-2 .. f+1 into velocity, T, mu and
//    the adjoint Gb of the cell-centred tangential velocity derivatives.
// Both share the face adjoint from Wb and one LDS window of cells
// (f0-3 .. f0+TF+1 per line); the tile writes each completed cell once.
// ---------------------------------------------------------------------------
// LDS of one tile: the accumulators (NCH channels x TW lines x NCW window
// cells) and, along y and z, the staging rows of the convective gather.
template <int NDIM, int D, bool VISC> struct DirLds {
  static constexpr int TF = TileShape<D>::TF, TW = TileShape<D>::TW;
  static constexpr int NOFF = 6, NCW = TF + 5;
  static constexpr int CP = 1 + NDIM, CT = 2 + NDIM, CMU = 3 + NDIM, CG = 4 + NDIM;
  static constexpr int NCH = VISC ? CG + 2 * (NDIM - 1) : CP + 1;
  static constexpr int BF = D == 0 ? TF : TF + 4;
  static constexpr int ACC = NCH * TW * NCW;
  static constexpr int BUF = D == 0 ? 0 : NOFF * TW * BF;
  static constexpr int SIZE = ACC + BUF;  // doubles
};

// One tile of direction D.  SIDE: the tile writes its completed cells' Qb
// contributions to the side arrays Qby (set, never added) instead of adding
// them to Qb, so that it can run concurrently with the x tiles that set Qb;
// k_tangential_vjp (ghost cells) and k_interior_vjp (interior cells) add the
// two.
template <int NDIM, int D, bool VISC, bool SIDE>
__device__ __forceinline__ void dir_vjp_tile(const Dev &g, const AdjBuffers &A, unsigned P,
                                             unsigned nb, double *lds) {
  using L = DirLds<NDIM, D, VISC>;
  constexpr int OLO = -3, OHI = 2, NOFF = L::NOFF, SPAN = OHI - OLO;
  constexpr int TF = L::TF, TW = L::TW;
  constexpr int NCW = L::NCW;  // window cells per line
  constexpr int T1 = tan1(D), T2 = tan2(D);
  // accumulator channels, active axes only: rho, the NDIM global velocity
  // components, p, then T, mu and Gb(T1,T1), Gb(T1,D) (Gb(T2,T2), Gb(T2,D))
  // for each active tangential axis when viscous.  In 2D this is 8 channels,
  // which keeps a y tile within a fifth of the CU's LDS (5 blocks per CU).
  constexpr int CP = L::CP, CT = L::CT, CMU = L::CMU, CG = L::CG;
  constexpr int NCH = L::NCH;
  // y/z tiles: a row stride of 36 doubles puts the 8 lines x 4 faces of a
  // half-wave on distinct LDS banks
  constexpr int BF = L::BF;
  auto acc = reinterpret_cast<double (*)[TW][NCW]>(lds);
  auto buf = reinterpret_cast<double (*)[TW][BF]>(lds + L::ACC);
  static_assert(NCH * TW * NCW == L::ACC, "accumulator layout");
  Tile t = make_tile<OLO, OHI, D>(g, P, nb);
  if (!t.valid) return;  // uniform across the workgroup
  for (int i = threadIdx.x; i < NCH * TW * NCW; i += 256) (&acc[0][0][0])[i] = 0.0;
  // x tiles: each wavefront holds the 64 faces of one line and its lanes
  // are the only writers of that line's window, one lane per cell in the
  // convective gather, so after this barrier that gather uses lane shuffles
  // and no barrier
  if (D == 0) __syncthreads();

  const int f = t.f0 + t.lane_face;
  const bool active = t.line_ok && f >= 0 && f <= g.n[D];
  const int qi[5] = {QR, QU + D, QU + T1, QU + T2, QP};
  constexpr int ch[5] = {0, 1 + D, 1 + T1, 1 + T2, CP};  // face frame -> channel (active m)
  double qLb[5] = {0, 0, 0, 0, 0}, qRb[5] = {0, 0, 0, 0, 0};
  double Fb[5] = {0, 0, 0, 0, 0};
  long base = 0;
  const long s = g.sb[D];
  if (active) {
    int pos[3] = {t.line[0], t.line[1], t.line[2]};
    pos[D] = f;
    face_adjoint<NDIM>(g, A, D, pos, f, Fb);
    base = bidx(g, pos[0], pos[1], pos[2]);
    double qL[5], qR[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const bool act = !((m == 2 && T1 >= NDIM) || (m == 3 && T2 >= NDIM));
      if (!act) {
        qL[m] = qR[m] = 0.0;
        continue;
      }
      const double *Qm = g.Q[qi[m]];
      double v0 = Qm[base - 3 * s], v1 = Qm[base - 2 * s], v2 = Qm[base - s];
      double v3 = Qm[base], v4 = Qm[base + s], v5 = Qm[base + 2 * s];
      weno5_pair(v0, v1, v2, v3, v4, v5, qL[m], qR[m]);
    }
    double Fr[5] = {Fb[0], Fb[1 + D], Fb[1 + T1], Fb[1 + T2], Fb[4]};
    hllc_vjp(qL, qR, g.gamma, g.gm1i, Fr, qLb, qRb);
  }
  // convective, per component: reverse the two reconstructions, stage the
  // contributions to cells f-3 .. f+2 in LDS, then gather them per window
  // cell in a fixed order of faces (deterministic, no atomics)
  for (int m = 0; m < 5; ++m) {
    const bool act = !((m == 2 && T1 >= NDIM) || (m == 3 && T2 >= NDIM));
    if (!act) continue;  // uniform across the block
    double c[NOFF] = {0, 0, 0, 0, 0, 0};
    if (active) {
      const double *Qm = g.Q[qi[m]];
      double v0 = Qm[base - 3 * s], v1 = Qm[base - 2 * s], v2 = Qm[base - s];
      double v3 = Qm[base], v4 = Qm[base + s], v5 = Qm[base + 2 * s];
      double gL[5] = {0, 0, 0, 0, 0}, gR[5] = {0, 0, 0, 0, 0};
      // an upwind (supersonic) face leaves one side without adjoint
      if (qLb[m] != 0.0) weno5_vjp(v0, v1, v2, v3, v4, qLb[m], gL);
      if (qRb[m] != 0.0) weno5_vjp(v5, v4, v3, v2, v1, qRb[m], gR);
      c[0] = gL[0];
      c[1] = gL[1] + gR[4];
      c[2] = gL[2] + gR[3];
      c[3] = gL[3] + gR[2];
      c[4] = gL[4] + gR[1];
      c[5] = gR[0];
    }
    if (D == 0) {
      // window cell w = L (and w = 64 + L for the last SPAN cells) takes
      // offset o from lane w - o, in the order of the LDS gather below
      const int L = t.lane_face;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int o = 0; o < NOFF; ++o) {
        const double v0 = __shfl(c[o], L - o);
        const double v1 = __shfl(c[o], TF + L - o);
        if (L >= o) s0 += v0;
        if (o > L) s1 += v1;
      }
      acc[ch[m]][t.lane_line][L] += s0;
      if (L < SPAN) acc[ch[m]][t.lane_line][TF + L] += s1;
      continue;
    }
#pragma unroll
    for (int o = 0; o < NOFF; ++o) buf[o][t.lane_line][t.lane_face] = c[o];
    __syncthreads();
    for (int i = threadIdx.x; i < TW * NCW; i += 256) {
      const int ll = i / NCW, w = i % NCW;
      double sum = 0.0;
#pragma unroll
      for (int o = 0; o < NOFF; ++o) {
        const int fl = w - o;  // face (lane) whose offset o lands on window cell w
        if (fl >= 0 && fl < TF) sum += buf[o][ll][fl];
      }
      acc[ch[m]][ll][w] += sum;
    }
    __syncthreads();
  }
  if constexpr (VISC) {
    // face-level adjoints of the dissipative flux
    double ufb[3] = {0, 0, 0}, dnb[3] = {0, 0, 0}, dTb = 0.0, mufb = 0.0;
    double divtb = 0.0, dtnb[3] = {0, 0, 0};
    double mfD = 0.0;
    if (active) {
      double vel[3][4], Tc[4], muc[4];
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        long cb = base + (o - 2) * s;
        vel[0][o] = g.Q[QU][cb];
        vel[1][o] = NDIM >= 2 ? g.Q[QV][cb] : 0.0;
        vel[2][o] = NDIM >= 3 ? g.Q[QW][cb] : 0.0;
        Tc[o] = g.Q[QT][cb];
        muc[o] = g.Q[QMU][cb];
      }
      mfD = g.mf[D][f];
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
        // cell-centred tangential derivatives d u_tt / d x_tt and d u_D /
        // d x_tt of the stage's primitive box, with the operands and
        // arithmetic of the forward flux kernels (the same values bitwise)
        const double *Ut = g.Q[QU + tt], *Ud = g.Q[QU + D];
        const long stt = g.sb[tt];
        const double mct = g.mc[tt][t.line[tt]];
        double gtt[4], gtn[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
          long cb = base + (o - 2) * s;
          gtt[o] = dcell4(Ut[cb - 2 * stt], Ut[cb - stt], Ut[cb + stt], Ut[cb + 2 * stt]) * mct;
          gtn[o] = dcell4(Ud[cb - 2 * stt], Ud[cb - stt], Ud[cb + stt], Ud[cb + 2 * stt]) * mct;
        }
        divt += interp4(gtt[0], gtt[1], gtt[2], gtt[3]);
        dtn[tt] = interp4(gtn[0], gtn[1], gtn[2], gtn[3]);
      }
      double brk[3] = {0.0, 0.0, 0.0};
      brk[D] = (4.0 / 3.0) * dn[D] - (2.0 / 3.0) * divt;
      if (T1 < NDIM) brk[T1] = dtn[T1] + dn[T1];
      if (T2 < NDIM) brk[T2] = dtn[T2] + dn[T2];
      double tau[3] = {muf * brk[0], muf * brk[1], muf * brk[2]};
      const double cpPr = g.cpPr;
      double lam = muf * cpPr;
      // reverse
      double enb = -Fb[4];
      double taub[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        taub[c] = -Fb[1 + c] + enb * uf[c];
        ufb[c] = enb * tau[c];
      }
      double lamb = enb * dT;
      dTb = enb * lam;
      mufb = lamb * cpPr + taub[0] * brk[0] + taub[1] * brk[1] + taub[2] * brk[2];
      dnb[D] = taub[D] * muf * (4.0 / 3.0);
      divtb = -taub[D] * muf * (2.0 / 3.0);
      if (T1 < NDIM) {
        dtnb[T1] = taub[T1] * muf;
        dnb[T1] = taub[T1] * muf;
      }
      if (T2 < NDIM) {
        dtnb[T2] = taub[T2] * muf;
        dnb[T2] = taub[T2] * muf;
      }
    }
    // cells f-2 .. f+1 are window cells lane_face + 1 .. lane_face + 4; one
    // offset at a time so that no two faces update a cell together
    const double I4[4] = {-1.0 / 16.0, 9.0 / 16.0, 9.0 / 16.0, -1.0 / 16.0};
    const double D4[4] = {1.0 / 24.0, -27.0 / 24.0, 27.0 / 24.0, -1.0 / 24.0};
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      if (active) {
        const int w = t.lane_face + 1 + o;
        const int ll = t.lane_line;
        const double dm = D4[o] * mfD, im = I4[o];
#pragma unroll
        for (int c = 0; c < NDIM; ++c) acc[1 + c][ll][w] += ufb[c] * im + dnb[c] * dm;
        acc[CT][ll][w] += dTb * dm;
        acc[CMU][ll][w] += mufb * im;
        if constexpr (T1 < NDIM) {
          acc[CG][ll][w] += divtb * im;
          acc[CG + 1][ll][w] += dtnb[T1] * im;
        }
        if constexpr (T2 < NDIM) {
          acc[CG + 2][ll][w] += divtb * im;
          acc[CG + 3][ll][w] += dtnb[T2] * im;
        }
      }
      // neighbouring faces update the same cells at consecutive offsets
      __syncthreads();
    }
  }
  if (D == 0 && !VISC) __syncthreads();  // every line's window complete before the write-out
  // write the completed cells: window cell w <-> cell t.f0 + OLO + w
  for (int i = threadIdx.x; i < TW * NCW; i += 256) {
    // x-lines: consecutive threads take consecutive cells of a line;
    // otherwise consecutive lines (x-neighbours) of one cell position
    const int ll = D == 0 ? i / NCW : i % TW, w = D == 0 ? i % NCW : i / TW;
    const int cell = t.f0 + OLO + w;
    if (cell < t.c0 || cell >= t.c1) continue;
    long ln = t.lg * TW + ll;
    if (ln >= (long)g.n[T1] * g.n[T2]) continue;
    int p[3];
    p[D] = cell;
    p[T1] = (int)(ln % g.n[T1]);
    p[T2] = (int)(ln / g.n[T1]);
    const long b = bidx(g, p[0], p[1], p[2]);
    const bool ghost = cell < 0 || cell >= g.n[D];
    if constexpr (SIDE) {
      A.Qby[QR][b] = acc[0][ll][w];
#pragma unroll
      for (int c = 0; c < NDIM; ++c) A.Qby[QU + c][b] = acc[1 + c][ll][w];
      A.Qby[QP][b] = acc[CP][ll][w];
      if constexpr (VISC) {
        A.Qby[QT][b] = acc[CT][ll][w];
        A.Qby[QMU][b] = acc[CMU][ll][w];
      } else {
        A.Qby[QT][b] = 0.0;
      }
    } else if (D == 0 || ghost) {
      // first writer of this cell in the stage: set every component the
      // later kernels accumulate into
      A.Qb[QR][b] = acc[0][ll][w];
#pragma unroll
      for (int c = 0; c < NDIM; ++c) A.Qb[QU + c][b] = acc[1 + c][ll][w];
      A.Qb[QP][b] = acc[CP][ll][w];
      if constexpr (VISC) {
        A.Qb[QT][b] = acc[CT][ll][w];
        A.Qb[QMU][b] = acc[CMU][ll][w];
      } else {
        A.Qb[QT][b] = 0.0;
      }
    } else {
      A.Qb[QR][b] += acc[0][ll][w];
#pragma unroll
      for (int c = 0; c < NDIM; ++c) A.Qb[QU + c][b] += acc[1 + c][ll][w];
      A.Qb[QP][b] += acc[CP][ll][w];
      if constexpr (VISC) {
        A.Qb[QT][b] += acc[CT][ll][w];
        A.Qb[QMU][b] += acc[CMU][ll][w];
      }
    }
    if constexpr (VISC) {
      // derivative adjoints: d u_D / d x_t is this kernel's alone (set); the
      // diagonal d u_t / d x_t is shared with the kernel of every earlier
      // direction other than t, which covered the cells interior along D
      constexpr bool sh1 = D >= 2 || (D == 1 && T1 != 0), sh2 = D >= 2 || (D == 1 && T2 != 0);
      if constexpr (T1 < NDIM) {
        double &d1 = A.Gb[3 * T1 + T1][b];
        d1 = (sh1 && !ghost ? d1 : 0.0) + acc[CG][ll][w];
        A.Gb[3 * T1 + D][b] = acc[CG + 1][ll][w];
      }
      if constexpr (T2 < NDIM) {
        double &d2 = A.Gb[3 * T2 + T2][b];
        d2 = (sh2 && !ghost ? d2 : 0.0) + acc[CG + 2][ll][w];
        A.Gb[3 * T2 + D][b] = acc[CG + 3][ll][w];
      }
    }
  }
}

// One direction per launch (1D, 3D).
template <int NDIM, int D, bool VISC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NDIM == 2 ? 5 : 4)))
k_dir_vjp(Dev g, AdjBuffers A) {
  __shared__ double lds[DirLds<NDIM, D, VISC>::SIZE];
  dir_vjp_tile<NDIM, D, VISC, false>(g, A, blockIdx.x, gridDim.x, lds);
}

// 2D: the x and y tiles of a stage in one launch, so that the two directions'
// tiles share the CUs (each alone leaves the FP64 units idle while its
// workgroups wait on memory).  Workgroups are dealt in groups of 8, x and y
// alternating while both have tiles left: group c of a direction holds its
// tiles 8c .. 8c+7, so that a tile's index modulo 8 is its hardware index
// modulo 8 (its XCD) as in a launch of its own.  The y tiles write their cell
// contributions to Qby; the x tiles set Qb.
template <bool VISC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
k_dir_vjp_xy(Dev g, AdjBuffers A, unsigned nx, unsigned ny) {
  constexpr int SX = DirLds<2, 0, VISC>::SIZE, SY = DirLds<2, 1, VISC>::SIZE;
  __shared__ double lds[SX > SY ? SX : SY];
  const unsigned grp = blockIdx.x / 8u, r = blockIdx.x % 8u;
  const unsigned cx = (nx + 7u) / 8u, cy = (ny + 7u) / 8u, cm = cx < cy ? cx : cy;
  unsigned dir, ci;
  if (grp < 2u * cm) {
    dir = grp % 2u;
    ci = grp / 2u;
  } else {
    dir = cx > cy ? 0u : 1u;
    ci = grp - cm;
  }
  const unsigned P = ci * 8u + r;
  if (dir == 0u) dir_vjp_tile<2, 0, VISC, false>(g, A, P, 8u * cx, lds);
  else dir_vjp_tile<2, 1, VISC, true>(g, A, P, 8u * cy, lds);
}

// ---------------------------------------------------------------------------
// Gather of the tangential-derivative adjoints (transpose of the
// cell-centred 4th-order difference along t), then mu'(T) folding: on the
// ghost cells in a launch of their own (the halo transposes read them), on
// the interior cells inside k_interior_vjp.
// ---------------------------------------------------------------------------
// d mu / dT from T and mu(T): omega mu / T (power law), mu (1.5/t - 1/(t+s))
// / T_ref with t = T/T_ref, s = S/T_ref (Sutherland).
__device__ __forceinline__ double dviscosity(const Dev &g, double T, double mu) {
  if (g.visc == VISC_POWER) return g.vparam * mu / T;
  if (g.visc == VISC_SUTHERLAND) {
    double t = T / g.T_ref;
    double s = g.vparam / g.T_ref;
    return mu * (1.5 / t - 1.0 / (t + s)) / g.T_ref;
  }
  return 0.0;
}

// Gather of the tangential-derivative adjoints at box cell p: y = x + k along
// t contributes coef(k) mc(y) Gb(y); the metric factors of the (at most
// four) neighbours along each axis are shared by the NDIM velocity components.
// INTERIOR: p is an interior cell (else a box cell of the ghost layers).
template <int NDIM, bool INTERIOR>
__device__ __forceinline__ void tangential_gather(const Dev &g, const AdjBuffers &A, const int *p,
                                                  long b, double *add) {
  constexpr int ks[4] = {-1, 1, -2, 2};
  constexpr double cf[4] = {8.0 / 12.0, -8.0 / 12.0, -1.0 / 12.0, 1.0 / 12.0};
  // Every load is issued first, so all of them are in flight together, then
  // the terms of the interior neighbours are summed in the order of the
  // definition (selects, no branches).  A neighbour that is not an interior
  // cell reads the cell itself and the metric at the cell's (clamped)
  // position instead, in bounds either way; an interior cell's neighbours
  // all lie in the box (two of its three ghost layers at most).
  double mct[NDIM][4], gv[NDIM][4][NDIM];
  bool in[NDIM][4];
#pragma unroll
  for (int t = 0; t < NDIM; ++t) {
    const long st = g.sb[t];
    const int pt = INTERIOR ? p[t] : min(max(p[t], 0), g.n[t] - 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int yt = p[t] + ks[r];
      in[t][r] = yt >= 0 && yt < g.n[t];
      mct[t][r] = g.mc[t][in[t][r] ? yt : pt];
      const long bb = (INTERIOR || in[t][r]) ? b + ks[r] * st : b;
#pragma unroll
      for (int phi = 0; phi < NDIM; ++phi) gv[t][r][phi] = A.Gb[3 * t + phi][bb];
    }
  }
#pragma unroll
  for (int phi = 0; phi < NDIM; ++phi) add[phi] = 0.0;
#pragma unroll
  for (int t = 0; t < NDIM; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double w = cf[r] * mct[t][r];
#pragma unroll
      for (int phi = 0; phi < NDIM; ++phi) {
        const double sum = add[phi] + w * gv[t][r][phi];
        add[phi] = in[t][r] ? sum : add[phi];
      }
    }
}

// Adjoint components carried through the halo fill: rho, the active
// velocities, p, T (mu-bar is folded into T-bar first).
template <int NDIM> struct HaloQ {
  static constexpr int nq = NDIM + 3;
  static constexpr int qs[6] = {QR, QU, NDIM >= 2 ? QV : QP,
                                NDIM == 3 ? QW : (NDIM == 2 ? QP : QT), NDIM == 3 ? QP : QT, QT};
};

// Ghost cell number t (0 <= t < nbox - ncell) -> its box position: the z
// ghost planes, then the y ghost rows of the interior planes, then the x
// ghost cells of the interior rows (x fastest within each part).
__device__ __forceinline__ void ghost_cell(const Dev &g, long t, int *p) {
  const long N0 = g.N[0], N1 = g.N[1];
  const int h0 = g.h[0], h1 = g.h[1], h2 = g.h[2];
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const long cz = 2L * h2 * N0 * N1;
  if (t < cz) {
    const long pl = t / (N0 * N1), rem = t % (N0 * N1);
    p[2] = pl < h2 ? (int)pl - h2 : n2 + (int)pl - h2;
    p[1] = (int)(rem / N0) - h1;
    p[0] = (int)(rem % N0) - h0;
    return;
  }
  t -= cz;
  const long cy = 2L * h1 * N0 * n2;
  if (t < cy) {
    const long row = t / N0;
    const int rr = (int)(row % (2 * h1));
    p[2] = (int)(row / (2 * h1));
    p[1] = rr < h1 ? rr - h1 : n1 + rr - h1;
    p[0] = (int)(t % N0) - h0;
    return;
  }
  t -= cy;
  const int c = (int)(t % (2 * h0));
  const long line = t / (2 * h0);
  p[2] = (int)(line / n1);
  p[1] = (int)(line % n1);
  p[0] = c < h0 ? c - h0 : n0 + c - h0;
}

// Ghost cells, before the halo transposes read them: the y tiles' side
// arrays (2D; on the y ghosts interior along x, which no x tile writes, they
// are the whole value), the tangential gather, and mu'(T) folded into T.
// Interior cells take the same three steps in k_interior_vjp.
template <int NDIM>
__global__ void __launch_bounds__(64) k_tangential_vjp(Dev g, AdjBuffers A) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.nbox - g.ncell) return;
  int p[3];
  ghost_cell(g, t, p);
  const long b = bidx(g, p[0], p[1], p[2]);
  const bool visc = g.visc != VISC_NONE;
  // every load first (Qb, Qby and Gb may overlap as far as the compiler
  // knows, which would serialise loads behind stores), then the stores
  // 2D: a y ghost's adjoint is the y tiles' side array (x ghosts: x tiles only)
  const bool side = NDIM == 2 && p[0] >= 0 && p[0] < g.n[0];
  const bool gather = NDIM >= 2 && A.Gb[0] != nullptr;
  // every active component is read (from the side array or from Qb; both
  // exist for each of them), whichever of them the stores below use
  double qb[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q == QW && NDIM < 3) {
      qb[q] = 0.0;
      continue;
    }
    const double x = (side ? A.Qby[q] : A.Qb[q])[b];
    qb[q] = side ? 0.0 + x : x;
  }
  double add[NDIM];
  if (gather) tangential_gather<NDIM, false>(g, A, p, b, add);
  const double Tq = g.Q[QT][b], muq = g.Q[QMU][b];  // (every box array exists)
  const double dmu = visc ? dviscosity(g, Tq, muq) : 0.0;
  if (side) {
#pragma unroll
    for (int i = 0; i < HaloQ<NDIM>::nq; ++i) {
      const int q = HaloQ<NDIM>::qs[i];
      A.Qb[q][b] = qb[q];
    }
    if (visc) A.Qb[QMU][b] = qb[QMU];
  }
  if (gather) {
#pragma unroll
    for (int phi = 0; phi < NDIM; ++phi) {
      qb[QU + phi] += add[phi];
      A.Qb[QU + phi][b] = qb[QU + phi];
    }
  }
  if (visc) A.Qb[QT][b] = qb[QT] + dmu * qb[QMU];
}

// Source cell of ghost layer m (0 nearest the face) on side `side` of an axis
// of n cells: the cell the forward halo fill copies (and mirrors) into it.
__device__ __forceinline__ int halo_source(int kind, int side, int m, int n) {
  if (kind == BC_PERIODIC) return side == 0 ? n - 1 - m : m;
  if (kind == BC_ZEROGRAD) return side == 0 ? 0 : n - 1;
  return side == 0 ? m : n - 1 - m;
}

// A ghost adjoint mapped to its contribution to the source: copies pass
// through; walls: p_g = p_s, u_g = -u_s (plus a prescribed normal part that
// depends on the state only through the porous p_w, taken separately);
// isothermal: rho_g = p_g / (R T_g), T_g = 2 T_w - T_s; adiabatic:
// rho_g = rho_s, T_g = T_s.  rg, pg: the ghost's density and pressure.
template <int NDIM>
__device__ __forceinline__ void ghost_transform(const Dev &g, bool wall, bool iso,
                                                const double *gbm, double rg, double pg,
                                                double *cs) {
  constexpr int nq = HaloQ<NDIM>::nq, iP = nq - 2, iT = nq - 1;
#pragma unroll
  for (int i = 0; i < nq; ++i) cs[i] = gbm[i];
  if (!wall) return;
#pragma unroll
  for (int c = 0; c < NDIM; ++c) cs[1 + c] = -gbm[1 + c];
  if (iso) {
    const double rb = gbm[0];
    cs[0] = 0.0;
    cs[iP] = gbm[iP] + rb * rg / pg;
    cs[iT] = -(gbm[iT] - rb * rg * rg * g.R / pg);
  }
}

// ---------------------------------------------------------------------------
// Transpose of the halo fill along axis d, folding ghost adjoints (complete
// after k_tangential_vjp) into their sources, axes in the order z, y, x.
// When the two sides' sources cannot coincide (n >= 6) a thread takes one
// ghost layer of one side of a column (its ghost and its source are its own
// cells); the zero-gradient copy (three layers, one source) and the porous /
// disturbance terms (which sum the three layers' normal-velocity adjoints)
// are taken by the layer-0 thread.  Short axes (n < 6) keep one thread per
// column doing both sides and every layer in turn.
// ---------------------------------------------------------------------------
__host__ inline long halo_vjp_threads(const Dev &g, int d) {
  const int t1 = tan1(d), t2 = tan2(d);
  const long n1 = t1 < d ? g.N[t1] : g.n[t1];
  const long n2 = t2 < d ? g.N[t2] : g.n[t2];
  return (g.n[d] >= 6 ? 6 : 1) * n1 * n2;
}

template <int NDIM>
__global__ void __launch_bounds__(64) k_halo_vjp(Dev g, AdjBuffers A, int d, double *dJdK) {
  using H = HaloQ<NDIM>;
  constexpr int nq = H::nq, iP = nq - 2;
  const int t1 = tan1(d), t2 = tan2(d);
  int lo1 = 0, n1 = g.n[t1], lo2 = 0, n2 = g.n[t2];
  if (t1 < d) { lo1 = -g.h[t1]; n1 = g.N[t1]; }
  if (t2 < d) { lo2 = -g.h[t2]; n2 = g.N[t2]; }
  const long ncol = (long)n1 * n2;
  const bool split = g.n[d] >= 6;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (split ? 6 : 1) * ncol) return;
  // thread -> (column, side, layer): columns fastest, then side, then layer
  const long col = split ? tid % ncol : tid;
  const int r = split ? (int)(tid / ncol) : 0;
  const int side_lo = split ? r % 2 : 0, side_hi = split ? side_lo + 1 : 2;
  const int mlo = split ? r / 2 : 0, mhi = split ? mlo + 1 : 3;
  const int a = lo1 + (int)(col % n1), bq = lo2 + (int)(col / n1);
  const int n = g.n[d];
  // ghost cells of this column that are ghosts along another axis too (edges
  // and corners of the box) are written only by the tangential-derivative
  // adjoint and by the transposes of later axes: this kernel, their last
  // reader, clears them for the next stage.  Every other cell the adjoint
  // reads is set afresh each stage by the flux adjoints.
  const bool edge = a < 0 || a >= g.n[t1] || bq < 0 || bq >= g.n[t2];
  for (int side = side_lo; side < side_hi; ++side) {
    const int face = 2 * d + side;
    const int kind = g.bck[face];
    const bool merged = kind == BC_ZEROGRAD;  // every layer copies one cell
    const bool distinct = !merged && n >= 3;  // three distinct sources
    // layers of this side that this thread folds
    int m0 = mlo, m1 = mhi;
    if (!distinct && kind != BC_DIRICHLET) {
      if (m0 > 0) continue;  // the layer-0 thread folds the whole column
      m1 = 3;
    }
    auto mine = [&](int m) { return m >= m0 && m < m1; };
    int pG[3][3];
    long G[3], S[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int gd = side == 0 ? -1 - m : n + m, sd = halo_source(kind, side, m, n);
      int ps[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {  // no dynamic register index
        pG[m][e] = e == d ? gd : (e == t1 ? a : bq);
        ps[e] = e == d ? sd : pG[m][e];
      }
      G[m] = bidx(g, pG[m][0], pG[m][1], pG[m][2]);
      S[m] = bidx(g, ps[0], ps[1], ps[2]);
    }
    if (kind == BC_DIRICHLET) {  // ghost adjoints discarded
      if (edge)
#pragma unroll
        for (int m = 0; m < 3; ++m)
          if (mine(m))
#pragma unroll
            for (int i = 0; i < nq; ++i) A.Qb[H::qs[i]][G[m]] = 0.0;
      continue;
    }
    const double sigma = side == 0 ? 1.0 : -1.0;
    const bool wall = is_wall(kind);
    const bool iso = wall && g.Tw[face] > 0.0;
    // porous and disturbance columns are never edge columns, so the layer-0
    // thread reads the other layers' ghosts while no thread clears them
    const bool porous = kind == BC_POROUS && face == g.pface && a >= g.pb && a < g.pe &&
                        bq >= 0 && bq < g.n[t2] && m0 == 0;
    const bool disturb = kind == BC_DISTURB && dJdK && a >= 0 && a < g.n[t1] && m0 == 0;
    const bool allgn = porous || disturb;  // needs every layer's normal-velocity adjoint
    double gb[3][6] = {}, sv[3][6] = {}, rg[3] = {}, pg[3] = {}, gn[3] = {};
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (mine(m)) {
#pragma unroll
        for (int i = 0; i < nq; ++i) gb[m][i] = A.Qb[H::qs[i]][G[m]];
        gn[m] = gb[m][1];  // gb[m][1 + d], without a dynamic register index
#pragma unroll
        for (int c = 1; c < NDIM; ++c)
          if (c == d) gn[m] = gb[m][1 + c];
      } else if (allgn) {
        gn[m] = A.Qb[QU + d][G[m]];
      }
    }
    if (merged) {
#pragma unroll
      for (int i = 0; i < nq; ++i) sv[0][i] = A.Qb[H::qs[i]][S[0]];
    } else if (distinct) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
        if (mine(m))
#pragma unroll
          for (int i = 0; i < nq; ++i) sv[m][i] = A.Qb[H::qs[i]][S[m]];
    }
    if (iso) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
        if (mine(m)) {
          rg[m] = g.Q[QR][G[m]];
          pg[m] = g.Q[QP][G[m]];
        }
    }
    int kk = 0;
    double pw = 0.0, Kk = 0.0, kb0 = 0.0;
    if (porous) {
      kk = bq * (g.pe - g.pb) + (a - g.pb);
      pw = g.Q[QP][S[0]];
      Kk = g.K[kk];
      if (dJdK) kb0 = dJdK[kk];
    }
    double xd = 0.0, th0 = 0.0, th1 = 0.0;
    if (disturb) {
      xd = g.xm[t1][a];
      th0 = g.K[g.doff[face]];
      th1 = g.K[g.doff[face] + 1];
    }
    double cs[3][6] = {};
    double vsum = 0.0;  // sum over the column's ghosts of the normal-velocity adjoint
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (wall) vsum += gn[m];
      if (mine(m)) ghost_transform<NDIM>(g, wall, iso, gb[m], rg[m], pg[m], cs[m]);
    }
    if (porous) {
      // v_g[d] = 2 sigma v_n - v_s[d], v_n = -K (p_w - p_inf)/p_inf; the
      // wall cell W is the source of ghost layer 0
      double kb = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double vnb = 2.0 * sigma * gn[m];
        cs[0][iP] += -Kk / g.pinf * vnb;
        kb += -(pw - g.pinf) / g.pinf * vnb;
      }
      if (dJdK) dJdK[kk] = kb0 + kb;
    }
    if (edge)
#pragma unroll
      for (int m = 0; m < 3; ++m)
        if (mine(m))
#pragma unroll
          for (int i = 0; i < nq; ++i) A.Qb[H::qs[i]][G[m]] = 0.0;
    // fold into the sources
    if (merged) {
#pragma unroll
      for (int i = 0; i < nq; ++i)
        A.Qb[H::qs[i]][S[0]] = sv[0][i] + ((cs[0][i] + cs[1][i]) + cs[2][i]);
    } else if (distinct) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
        if (mine(m))
#pragma unroll
          for (int i = 0; i < nq; ++i) A.Qb[H::qs[i]][S[m]] = sv[m][i] + cs[m][i];
    } else {  // n < 3: sources may repeat, accumulate layer by layer
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int i = 0; i < nq; ++i) A.Qb[H::qs[i]][S[m]] += cs[m][i];
    }
    if (kind == BC_DISTURB && dJdK && m0 == 0) {
      // v_g[d] = 2 sigma A sin(phi) - v_s[d], phi = 2 pi kappa x: per-column
      // partials of dJ/dA and dJ/dkappa, summed over columns by k_disturb_sum
      double dA = 0.0, dk = 0.0;
      if (disturb) {
        const double ph = 2.0 * M_PI * xd * th1;
        const double w = 2.0 * sigma * vsum;
        dA = w * sin(ph);
        dk = w * th0 * cos(ph) * 2.0 * M_PI * xd;
      }
      A.dpart[(2 * side) * A.dcols + col] = dA;
      A.dpart[(2 * side + 1) * A.dcols + col] = dk;
    }
  }
}

// dJ/d(A, kappa) += column sums of k_halo_vjp's partials for one disturbance
// face (one block, fixed summation order: deterministic).
__global__ void __launch_bounds__(256) k_disturb_sum(const double *part, long cols, double *out) {
  __shared__ double sh[2][256];
  double v[2] = {0.0, 0.0};
  for (long i = threadIdx.x; i < cols; i += 256) {
    v[0] += part[i];
    v[1] += part[cols + i];
  }
  sh[0][threadIdx.x] = v[0];
  sh[1][threadIdx.x] = v[1];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] += sh[0][0];
    out[1] += sh[1][0];
  }
}

// ---------------------------------------------------------------------------
// Mass-flux body force of a stage, adjoint side: the source adds f to the
// x-momentum and f u to the energy right-hand side of every cell, so with
// Rb = b dt Wb, f-bar = sum_c (Rb_rhou(c) + Rb_E(c) u(c)); also the volume
// W = sum_c V_c.  Two passes, fixed-shape trees (deterministic): src[1] =
// f-bar, src[2] = W.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_force_adj_partial(Dev g, AdjBuffers A) {
  __shared__ double sh[2][256];
  const double s = A.bcoef * A.dtp[0];
  const long nc = g.ncell;
  const int nd = g.ndim;
  const unsigned n0 = g.n[0], n01 = n0 * (unsigned)g.n[1];
  double v[2] = {0.0, 0.0};
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < nc;
       c += (long)gridDim.x * blockDim.x) {
    const unsigned cu = (unsigned)c;
    const int k = (int)(cu / n01), j = (int)((cu % n01) / n0), i = (int)(cu % n0);
    const double rb1 = s * A.Wb[nc + c], rbE = s * A.Wb[(long)(nd + 1) * nc + c];
    v[0] += rb1 + rbE * g.Q[QU][bidx(g, i, j, k)];
    double V = g.dx[0][i];
    if (nd >= 2) V *= g.dx[1][j];
    if (nd >= 3) V *= g.dx[2][k];
    v[1] += V;
  }
  sh[0][threadIdx.x] = v[0];
  sh[1][threadIdx.x] = v[1];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    A.spart[2 * blockIdx.x] = sh[0][0];
    A.spart[2 * blockIdx.x + 1] = sh[1][0];
  }
}

// With the mass-flux body force f = -sum_c V_c R_rhou(c) / W every cell's
// x-momentum right-hand side also carries the force's dependence on the
// face fluxes: its adjoint gets -f-bar V_c / W (between the cells of a line
// these terms cancel in the face adjoints, leaving the boundary faces, as in
// the forward's boundary-flux form).  Written as a copy of the stage-output
// adjoint whose x-momentum component is Wb_rhou - f-bar V_c / (W b dt); the
// flux adjoints read the copy (the other kernels the stage's own Wb).
__global__ void __launch_bounds__(256) k_force_adj_apply(Dev g, AdjBuffers A, double *Wc) {
  const unsigned cu = blockIdx.x * blockDim.x + threadIdx.x;
  if (cu >= (unsigned)g.ncell) return;
  const long nc = g.ncell;
  const int nd = g.ndim;
  const unsigned n0 = g.n[0], n01 = n0 * (unsigned)g.n[1];
  const int k = (int)(cu / n01), j = (int)((cu % n01) / n0), i = (int)(cu % n0);
  double V = g.dx[0][i];
  if (nd >= 2) V *= g.dx[1][j];
  if (nd >= 3) V *= g.dx[2][k];
  const double s = A.bcoef * A.dtp[0];
  for (int v = 0; v < nd + 2; ++v) {
    const double w = A.Wb[(long)v * nc + cu];
    Wc[(long)v * nc + cu] = v == 1 ? w - (A.src[1] / A.src[2]) * V / s : w;
  }
}

__global__ void __launch_bounds__(256) k_force_adj_final(AdjBuffers A, int nparts) {
  __shared__ double sh[2][256];
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += 256) {
    v[0] += A.spart[2 * b];
    v[1] += A.spart[2 * b + 1];
  }
  sh[0][threadIdx.x] = v[0];
  sh[1][threadIdx.x] = v[1];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    A.src[1] = sh[0][0];
    A.src[2] = sh[1][0];
  }
}

// ---------------------------------------------------------------------------
// Interior: Vb = b Wb + (dQ/dU)^T Qb, with Q = (rho, u, v, w, p, T(p, rho)).
// In the first stage (fold != 0, V = Un) Vb also takes the Un terms of the
// later stages' combinations, a3 W3 + a2 W2 (their output adjoints, still
// held), so no accumulator crosses the stages.
// ---------------------------------------------------------------------------
template <int NDIM>
__global__ void __launch_bounds__(256) k_interior_vjp(Dev g, AdjBuffers A, const double *V,
                                                      const double *Wb, double a, double b,
                                                      double *Vb, const double *w3, double a3,
                                                      const double *w2, double a2, int fold) {
  constexpr int nd = NDIM;
  const unsigned cu = blockIdx.x * blockDim.x + threadIdx.x;  // ncell < 2^31
  if (cu >= (unsigned)g.ncell) return;
  const long c = cu;
  const long nc = g.ncell;
  const unsigned n0 = g.n[0], n01 = n0 * (unsigned)g.n[1];
  const int k = (int)(cu / n01), j = (int)((cu % n01) / n0), i = (int)(cu % n0);
  const long bx = bidx(g, i, j, k);
  // the cell's state and stage-output adjoints (and the fold's inputs)
  // first: every load of the kernel before the first store (Vb may be an
  // input array as far as the compiler knows), as few round trips as the
  // branches allow
  double Vc[nd + 2], wv[nd + 2], f3[nd + 2], f2[nd + 2];
#pragma unroll
  for (int v = 0; v < nd + 2; ++v) {
    const long x = (long)v * nc + c;
    Vc[v] = V[x];
    wv[v] = Wb[x];
    f3[v] = fold ? w3[x] : 0.0;
    f2[v] = fold ? w2[x] : 0.0;
  }
  // the primitive adjoint of the cell: the flux adjoints' (x tiles plus, in
  // 2D, the y tiles' side arrays) with the halo transposes' contributions,
  // the tangential gather, and mu'(T) folded into T
  double rb = A.Qb[QR][bx], pb = A.Qb[QP][bx], Tb = A.Qb[QT][bx];
  double ub[3] = {A.Qb[QU][bx], nd >= 2 ? A.Qb[QV][bx] : 0.0, nd >= 3 ? A.Qb[QW][bx] : 0.0};
  const bool visc = g.visc != VISC_NONE;
  double mub = visc ? A.Qb[QMU][bx] : 0.0;
  if constexpr (NDIM == 2) {
    rb += A.Qby[QR][bx];
    ub[0] += A.Qby[QU][bx];
    ub[1] += A.Qby[QV][bx];
    pb += A.Qby[QP][bx];
    Tb += A.Qby[QT][bx];
    if (visc) mub += A.Qby[QMU][bx];
  }
  if (NDIM >= 2 && A.Gb[0] != nullptr) {
    const int pc[3] = {i, j, k};
    double add[NDIM];
    tangential_gather<NDIM, true>(g, A, pc, bx, add);
#pragma unroll
    for (int phi = 0; phi < NDIM; ++phi) ub[phi] += add[phi];
  }
  const double Tq = g.Q[QT][bx], muq = g.Q[QMU][bx];  // (every box array exists)
  if (visc) Tb += dviscosity(g, Tq, muq) * mub;
  if (g.source == SRC_MASSFLUX)  // energy source f u: u-bar += Rb_E f
    ub[0] += (A.bcoef * A.dtp[0] * wv[nd + 1]) * A.src[0];
  double rho = Vc[0];
  double ir = 1.0 / rho;
  double u[3] = {Vc[1] * ir, nd >= 2 ? Vc[2] * ir : 0.0, nd >= 3 ? Vc[3] * ir : 0.0};
  double E = Vc[nd + 1];
  double k2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double p = (g.gamma - 1.0) * (E - 0.5 * rho * k2);
  double T = p / (rho * g.R);
  pb += Tb / (rho * g.R);
  rb -= Tb * T * ir;
  const double gm1 = g.gamma - 1.0;
  double Ub[5];
  Ub[0] = rb + gm1 * 0.5 * k2 * pb;
#pragma unroll
  for (int d = 0; d < nd; ++d) {
    Ub[1 + d] = ub[d] * ir - gm1 * u[d] * pb;
    Ub[0] -= ub[d] * u[d] * ir;
  }
  Ub[nd + 1] = gm1 * pb;
#pragma unroll
  for (int v = 0; v < nd + 2; ++v) {
    const long x = (long)v * nc + c;
    const double w = wv[v];
    double vb = b * w + Ub[v];
    if (fold) {
      const double accv = ((0.0 + a3 * f3[v]) + a2 * f2[v]) + a * w;
      Vb[x] = accv + vb;
    } else {
      Vb[x] = vb;
    }
  }
}

// ---------------------------------------------------------------------------
// Host sequencing.
// ---------------------------------------------------------------------------
using AdjKernel = void (*)(Dev, AdjBuffers);

static AdjKernel dir_kernel(int nd, int D, bool visc) {
  if (nd == 1) return visc ? k_dir_vjp<1, 0, true> : k_dir_vjp<1, 0, false>;
  if (D == 0) return visc ? k_dir_vjp<3, 0, true> : k_dir_vjp<3, 0, false>;
  if (D == 1) return visc ? k_dir_vjp<3, 1, true> : k_dir_vjp<3, 1, false>;
  return visc ? k_dir_vjp<3, 2, true> : k_dir_vjp<3, 2, false>;
}

static inline unsigned blocks(long n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

#define DCF_TRY(x)                    \
  do {                                \
    hipError_t e_ = (x);              \
    if (e_ != hipSuccess) return e_;  \
  } while (0)

// dJ/d(A, kappa) of the disturbance faces of axis d from the per-column
// partials its halo transpose wrote.
static hipError_t disturb_sums(const Dev &g, const AdjBuffers &A, int d, double *dJdK,
                               hipStream_t st) {
  if (!dJdK) return hipSuccess;
  const int t1 = tan1(d), t2 = tan2(d);
  const long n1 = t1 < d ? g.N[t1] : g.n[t1];
  const long n2 = t2 < d ? g.N[t2] : g.n[t2];
  for (int side = 0; side < 2; ++side) {
    const int face = 2 * d + side;
    if (g.bck[face] != BC_DISTURB) continue;
    k_disturb_sum<<<1, 256, 0, st>>>(A.dpart + 2 * side * A.dcols, n1 * n2, dJdK + g.doff[face]);
    DCF_TRY(hipGetLastError());
  }
  return hipSuccess;
}

// Reverse of one stage: Vb = b Wb + R'(V)^T (b dt Wb), accumulators as in
// k_interior_vjp.  Needs g.Q to hold nothing on entry (recomputed here), and
// the adjoint boxes (Qb, Gb) zero wherever no kernel of a stage writes them
// (cleared once with the workspace; the kernels keep it so).
static hipError_t stage_vjp(const Dev &g, const AdjBuffers &A0, const double *V, const double *Wb,
                            const double *dt, double a, double b, double *Vb,
                            const double *w3, double a3, const double *w2, double a2,
                            int fold, double *dJdK,
                            hipStream_t st, bool have_box) {
  const bool visc = g.visc != VISC_NONE;
  AdjBuffers A = A0;
  A.Wb = Wb;
  A.dtp = dt;
  A.bcoef = b;
  if (!have_box) DCF_TRY(launch_prim_halo(g, V, st));  // the stage's primitive box
  if (g.source == SRC_MASSFLUX) {
    // the stage's body force f (as the forward stage computed it), f-bar,
    // and the x-momentum adjoint corrected for the force's dependence
    DCF_TRY(launch_force_direct(g, A.spart, A.src, st));
    const unsigned nb = (unsigned)std::min<long>((g.ncell + 255) / 256, RED_BLOCKS);
    k_force_adj_partial<<<nb, 256, 0, st>>>(g, A);
    k_force_adj_final<<<1, 256, 0, st>>>(A, (int)nb);
    k_force_adj_apply<<<blocks(g.ncell), 256, 0, st>>>(g, A, A.fwb);
    DCF_TRY(hipGetLastError());
    A.Wb = A.fwb;  // for the flux adjoints; k_interior_vjp takes Wb itself
  }
  if (g.ndim == 2) {
    const unsigned nx = tile_count<-3, 2>(g, 0), ny = tile_count<-3, 2>(g, 1);
    const unsigned nblk = 8u * ((nx + 7u) / 8u + (ny + 7u) / 8u);
    auto k = visc ? k_dir_vjp_xy<true> : k_dir_vjp_xy<false>;
    k<<<nblk, 256, 0, st>>>(g, A, nx, ny);
    DCF_TRY(hipGetLastError());
  } else {
    for (int D = 0; D < g.ndim; ++D) {
      hipLaunchKernelGGL(dir_kernel(g.ndim, D, visc), dim3(tile_count<-3, 2>(g, D)), dim3(256),
                         0, st, g, A);
      DCF_TRY(hipGetLastError());
    }
  }
  if ((visc || g.ndim == 2) && g.nbox > g.ncell) {  // 2D: also the y tiles' side arrays
    auto tk = g.ndim == 1 ? k_tangential_vjp<1>
                          : (g.ndim == 2 ? k_tangential_vjp<2> : k_tangential_vjp<3>);
    tk<<<(unsigned)((g.nbox - g.ncell + 63) / 64), 64, 0, st>>>(g, A);
    DCF_TRY(hipGetLastError());
  }
  // the halo transposes, axes z, y, x
  for (int d = g.ndim - 1; d >= 0; --d) {
    auto hk = g.ndim == 1 ? k_halo_vjp<1> : (g.ndim == 2 ? k_halo_vjp<2> : k_halo_vjp<3>);
    const long nt = halo_vjp_threads(g, d);
    hk<<<(unsigned)((nt + 63) / 64), 64, 0, st>>>(g, A, d, dJdK);
    DCF_TRY(hipGetLastError());
    DCF_TRY(disturb_sums(g, A, d, dJdK, st));
  }
  auto ik = g.ndim == 1 ? k_interior_vjp<1> : (g.ndim == 2 ? k_interior_vjp<2> : k_interior_vjp<3>);
  ik<<<blocks(g.ncell), 256, 0, st>>>(g, A, V, Wb, a, b, Vb, w3, a3, w2, a2, fold);
  return hipGetLastError();
}

hipError_t vjp_step(Dev g, const AdjBuffers &A, const double *Un, const double *U1,
                    const double *U2, const double *dt, const double *lam1, double *lam0,
                    double *dJdK, hipStream_t st, const Dev *boxes) {
  const bool have = boxes != nullptr;  // stage boxes cached by the forward recompute
  const Dev &g3 = have ? boxes[2] : g, &g2 = have ? boxes[1] : g, &g1 = have ? boxes[0] : g;
  // stage 3: W = Un/3 + 2/3 (U2 + dt R(U2))
  DCF_TRY(stage_vjp(g3, A, U2, lam1, dt, 1.0 / 3.0, 2.0 / 3.0, A.Ub2, nullptr, 0.0, nullptr, 0.0,
                    0, dJdK, st, have));
  // stage 2: W = 3/4 Un + 1/4 (U1 + dt R(U1))
  DCF_TRY(stage_vjp(g2, A, U1, A.Ub2, dt, 0.75, 0.25, A.Ub1, nullptr, 0.0, nullptr, 0.0, 0, dJdK,
                    st, have));
  // stage 1: W = Un + dt R(Un)
  // (Un enters stage 3 with weight 1/3 and stage 2 with 3/4)
  DCF_TRY(stage_vjp(g1, A, Un, A.Ub1, dt, 0.0, 1.0, lam0, lam1, 1.0 / 3.0, A.Ub2, 0.75, 1, dJdK,
                    st, have));
  return hipSuccess;
}

}  // namespace dcf
