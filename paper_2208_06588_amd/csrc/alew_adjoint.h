// Discrete adjoint of one SSP-RK3 stage (reverse mode, written by hand).
//
// Stage s maps q^(s-1) to
//   q^(s) = [a_s J^n q^n + b_s (J^(s-1) q^(s-1) + dt R(q^(s-1)))] / J^(s),
//   R = A + alpha D,   alpha = max over faces and traces of |u - w| + sqrt(g h).
// Given lambda^(s) = dL/dq^(s), with mu = lambda^(s) / J^(s) and rho = b_s dt mu:
//   dL/dq^n     += a_s J^n mu
//   dL/dq^(s-1)  = b_s J^(s-1) mu + (dR/dq^(s-1))^T rho,
// where the alpha part enters through lambda_alpha = sum_j rho_j . D_j, sent to
// the one trace that attains alpha (first face, left trace first, as a scan in
// face order finds it).  Everything that switches is frozen to the forward
// values: detector class, limiter activity and its argmin, |.| signs, dry
// cut-offs, the argmax.  The mesh and the step sizes do not depend on the
// state.
//
// Work split per stage (gather form, no floating-point atomics):
//   k_adj_fused   per tile: forward reconstruction and limiter of its cells and
//                 a two-cell halo, face adjoints without the alpha term, reverse
//                 of limiter and reconstruction, stencil contributions summed in
//                 LDS, lambda^(s-1) of the owned cells, and the tile's part of
//                 lambda_alpha;
//   k_adj_fold    contributions to ghost cells onto their source cells;
//   k_adj_lsum    lambda_alpha per instance (tile parts in tile order);
//   k_adj_patch   the alpha term: one trace per instance (found by the forward
//                 records), through the limiter and reconstruction of its cell.
// The alpha term is linear in the adjoints given the frozen switches, so it can
// be added after the rest.
#pragma once

#include "alew_kernels.h"

namespace alew_dev {

struct AdjBufs {
  const int64_t* cell_off;
  int64_t S;
  int32_t ninst;
  int32_t pad;
  const double* q;     // [3][S] stage input q^(s-1) (eta, hu, b)
  const double* akeyd; // [ninst] 2 f + side of the trace attaining alpha (forward record)
  const double* x;     // [S+ninst] x^n
  const double* w;     // [S+ninst] w^n
  const double* scal;  // [ninst][8] t, dt, alpha_1..3, dx_0..2 of the step
  double* lam;         // [3][S] lambda^(s)
  double* lam_out;     // [3][S] lambda^(s-1) (a different buffer: tiles read
                       // lambda^(s) of their halo cells while others write)
  double* lbase;       // [3][S] adjoint of q^n accumulated over the stages
  double* lalpha;      // [ninst]
  double* lpart;       // [fused tiles] per-tile parts of lambda_alpha
};

__device__ __forceinline__ double stage_a(int s) { return s == 1 ? 0.0 : (s == 2 ? 0.75 : 1.0 / 3.0); }
__device__ __forceinline__ double stage_b(int s) { return s == 1 ? 1.0 : (s == 2 ? 0.25 : 2.0 / 3.0); }

// Widths of cell k at the stage meshes: Jn, J^(s-1), J^(s).
__device__ __forceinline__ void stage_widths(const double* x, const double* w, int64_t k, double dt,
                                             int s, double& Jn, double& Jin, double& Jout) {
  Jn = x[k + 1] - x[k];
  const double dw = w[k + 1] - w[k];
  const double J1 = Jn + dt * dw;
  const double J2 = 0.75 * Jn + 0.25 * (J1 + dt * dw);
  const double J3 = (1.0 / 3.0) * Jn + (2.0 / 3.0) * (J2 + dt * dw);
  Jin = s == 1 ? Jn : (s == 2 ? J1 : J2);
  Jout = s == 1 ? J1 : (s == 2 ? J2 : J3);
}

// ----------------------------------------------------------------------------
// Reverse of one face: adjoints of the flux pieces (from the neighbouring
// cells' rho) onto the two limited traces.
// ----------------------------------------------------------------------------
struct TraceAdj {
  double h, m, b;
};

__device__ __forceinline__ void face_vjp(double hl, double ml, double bl, double hr, double mr,
                                         double br, double w, double alpha, double g, double dry,
                                         const double rl[3], const double rr[3], double etal_bar,
                                         double etar_bar, TraceAdj& Ll, TraceAdj& Lr) {
  // adjoints of F1, F2, G, B1, B2 at this face
  const double lF1 = rr[0] - rl[0];
  const double lF2 = rr[1] - rl[1];
  const double lG = rr[2] - rl[2];
  const double lB2 = 0.5 * g * (rl[1] - rr[1]);
  const double lB1 = -g * etal_bar * rl[1] + g * etar_bar * rr[1];
  const bool wl = hl > dry, wr = hr > dry;
  const double mlp = wl ? ml : 0.0, mrp = wr ? mr : 0.0;
  const double ihl = wl ? frcp(hl) : 0.0, ihr = wr ? frcp(hr) : 0.0;
  const double ul = wl ? ml * ihl : 0.0, ur = wr ? mr * ihr : 0.0;
  double lel = 0.5 * alpha * lF1, ler = -0.5 * alpha * lF1;
  const double lHl1 = 0.5 * lF1, lHr1 = 0.5 * lF1;
  const double lHl2 = 0.5 * lF2, lHr2 = 0.5 * lF2;
  double lmlp = 0.5 * alpha * lF2, lmrp = -0.5 * alpha * lF2;
  double lbl = (-0.5 * w + 0.5 * alpha) * lG + 0.5 * lB1 + bl * lB2;
  double lbr = (-0.5 * w - 0.5 * alpha) * lG + 0.5 * lB1 + br * lB2;
  // H1 = m' - w eta
  lmlp += lHl1; lel += -w * lHl1;
  lmrp += lHr1; ler += -w * lHr1;
  // H2 = m' u + g h^2 / 2 - w m'
  lmlp += (ul - w) * lHl2;
  lmrp += (ur - w) * lHr2;
  double lul = mlp * lHl2, lur = mrp * lHr2;
  double lhl = g * hl * lHl2, lhr = g * hr * lHr2;
  // u = m'/h on wet traces
  if (wl) { lmlp += lul * ihl; lhl += -(ul * ihl) * lul; }
  if (wr) { lmrp += lur * ihr; lhr += -(ur * ihr) * lur; }
  // eta = h + b
  lhl += lel; lbl += lel;
  lhr += ler; lbr += ler;
  Ll.h = lhl; Ll.m = wl ? lmlp : 0.0; Ll.b = lbl;
  Lr.h = lhr; Lr.m = wr ? lmrp : 0.0; Lr.b = lbr;
}

// Reverse of one face of the hydrostatic form (face_flux_hydro): the left
// cell's residual takes -(F1, F2 + cl, G) and the right cell's +(F1, F2 + cr,
// G), each with the alpha jump; alpha is a constant here (its own adjoint
// goes through the trace that attains it).  max(bl, br) at a tie takes bl.
__device__ __forceinline__ void face_vjp_hydro(double hl, double ml, double bl, double hr,
                                               double mr, double br, double w, double alpha,
                                               double g, double dry, const double rl[3],
                                               const double rr[3], TraceAdj& Ll, TraceAdj& Lr) {
  const double lF1 = rr[0] - rl[0];
  const double lF2 = rr[1] - rl[1];
  const double lG = rr[2] - rl[2];
  const double lcl = -rl[1], lcr = rr[1];
  const bool wl = hl > dry, wr = hr > dry;
  const double mlp = wl ? ml : 0.0, mrp = wr ? mr : 0.0;
  const double el = hl + bl, er = hr + br;
  const bool lmax = bl >= br;
  const double bmax = lmax ? bl : br;
  const double xl = el - bmax, xr = er - bmax;
  const double hsl = xl > 0.0 ? xl : 0.0, hsr = xr > 0.0 ? xr : 0.0;
  const bool sl = hsl > dry, sr = hsr > dry;
  const double ihsl = sl ? frcp(hsl) : 0.0, ihsr = sr ? frcp(hsr) : 0.0;
  const double usl = sl ? mlp * ihsl : 0.0, usr = sr ? mrp * ihsr : 0.0;
  // F1 = (m'l - w el + m'r - w er)/2 - alpha/2 (er - el)
  double lel = 0.5 * (alpha - w) * lF1, ler = -0.5 * (alpha + w) * lF1;
  double lmlp = 0.5 * lF1, lmrp = 0.5 * lF1;
  // alpha part of the momentum: -alpha/2 (m'r - m'l)
  lmlp += 0.5 * alpha * lF2;
  lmrp -= 0.5 * alpha * lF2;
  // F2 = (m'l usl + g/2 hsl^2 - w m'l + m'r usr + g/2 hsr^2 - w m'r)/2, usl = m'l/hsl
  const double A = 0.5 * lF2;
  lmlp += A * ((sl ? 2.0 * usl : 0.0) - w);
  lmrp += A * ((sr ? 2.0 * usr : 0.0) - w);
  double lhsl = A * (g * hsl - (sl ? usl * usl : 0.0));
  double lhsr = A * (g * hsr - (sr ? usr * usr : 0.0));
  // cl = g/2 (hl^2 - hsl^2), cr = g/2 (hr^2 - hsr^2)
  double lhl = g * hl * lcl, lhr = g * hr * lcr;
  lhsl -= g * hsl * lcl;
  lhsr -= g * hsr * lcr;
  // hs = max(e - bmax, 0)
  double lbmax = 0.0;
  if (xl >= 0.0) { lel += lhsl; lbmax -= lhsl; }
  if (xr >= 0.0) { ler += lhsr; lbmax -= lhsr; }
  // G = -w (bl + br)/2 - alpha/2 (br - bl)
  double lbl = (-0.5 * w + 0.5 * alpha) * lG, lbr = (-0.5 * w - 0.5 * alpha) * lG;
  if (lmax) lbl += lbmax; else lbr += lbmax;
  // e = h + b
  lhl += lel; lbl += lel;
  lhr += ler; lbr += ler;
  Ll.h = lhl; Ll.m = wl ? lmlp : 0.0; Ll.b = lbl;
  Lr.h = lhr; Lr.m = wr ? lmrp : 0.0; Lr.b = lbr;
}

// Reverse of hydro_source: cotangents of the eta and b values at the four
// Gauss-Lobatto points from the cotangent lS of the source.
__device__ __forceinline__ void hydro_source_vjp(double g, const double e[4], const double b[4],
                                                 double lS, double le[4], double lb[4]) {
  const double PHI = 1.6180339887498948482, PHI1 = 0.6180339887498948482;
  const double R5 = 2.2360679774997896964;
  const double D[4][4] = {{-6.0, 5.0 * PHI, -5.0 * PHI1, 1.0},
                          {-PHI, 0.0, R5, -PHI1},
                          {PHI1, -R5, 0.0, PHI},
                          {-1.0, 5.0 * PHI1, -5.0 * PHI, 6.0}};
  const double om[4] = {1.0, 5.0, 5.0, 1.0};
  const double lq = (-g / 12.0) * lS;
  double d[4], gq[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    d[mu] = D[mu][0] * b[0] + D[mu][1] * b[1] + D[mu][2] * b[2] + D[mu][3] * b[3];
    gq[mu] = om[mu] * (e[mu] - b[mu]);
  }
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    double t = -om[nu] * d[nu];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) t += gq[mu] * D[mu][nu];
    le[nu] = lq * om[nu] * d[nu];
    lb[nu] = lq * t;
  }
}

// Adjoint of alpha = |u - w| + sqrt(g max(h,0)) at the trace that attains it.
__device__ __forceinline__ void alpha_trace_vjp(double h, double m, double w, double g, double dry,
                                                double lalpha, TraceAdj& L) {
  const bool wet = h > dry;
  const double ih = wet ? frcp(h) : 0.0;
  const double u = wet ? m * ih : 0.0;
  const double d = u - w;
  const double sg = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
  const double lu = sg * lalpha;
  if (wet) { L.m += lu * ih; L.h += -(u * ih) * lu; }
  if (h > 0.0) {
    const double sq = sqrt(g * h);
    if (sq > 0.0) L.h += g * (0.5 / sq) * lalpha;
  }
}

// ----------------------------------------------------------------------------
// Reverse of the positivity limiter (1D eq. (3.20)-(3.21), Remark 4.1).
// o: unlimited traces.  In: adjoints of the limited traces; out: adjoints of
// the unlimited traces, plus the cell means.  hu_lim as in limit_cell.
// ----------------------------------------------------------------------------
__device__ __forceinline__ void limit_vjp(double hbar, double mbar, double pp_eps, const CellRecon& o,
                                          TraceAdj& LL, TraceAdj& LR, double& lhbar,
                                          double& lmbar, bool hu_lim = true) {
  if (hbar <= 0.0) {
    // h' = hbar, m' = mbar (hu_lim), b' = (h + b) - hbar
    lhbar += LL.h + LR.h - LL.b - LR.b;
    LL.h = LL.b;
    LR.h = LR.b;
    if (hu_lim) {
      lmbar += LL.m + LR.m;
      LL.m = 0.0;
      LR.m = 0.0;
    }
    return;
  }
  const double s1 = 1.0 / 12.0;
  const double delta = (hbar - s1 * o.hL - s1 * o.hR) * (1.0 / (1.0 - 2.0 * s1));
  double mn = o.hL;
  int which = 0;
  if (delta < mn) { mn = delta; which = 1; }
  if (o.hR < mn) { mn = o.hR; which = 2; }
  const bool eps_const = pp_eps < hbar;
  const double epsj = eps_const ? pp_eps : hbar;
  if (!(mn < epsj)) return;  // identity
  const double iden = frcp(hbar - mn);
  double Phi = (hbar - epsj) * iden;
  const bool clamped = Phi > 1.0;
  if (clamped) Phi = 1.0;
  // b' = (h + b) - h'  ->  total adjoint of h' is lh' - lb'
  const double lhLt = LL.h - LL.b, lhRt = LR.h - LR.b;
  double lPhi = (o.hL - hbar) * lhLt + (o.hR - hbar) * lhRt;
  double lhL = LL.b + Phi * lhLt;
  double lhR = LR.b + Phi * lhRt;
  lhbar += (1.0 - Phi) * (lhLt + lhRt);
  double lmL = LL.m, lmR = LR.m;
  if (hu_lim) {
    lPhi += (o.mL - mbar) * LL.m + (o.mR - mbar) * LR.m;
    lmL = Phi * LL.m;
    lmR = Phi * LR.m;
    lmbar += (1.0 - Phi) * (LL.m + LR.m);
  }
  if (!clamped) {
    lhbar += lPhi * ((eps_const ? 1.0 : 0.0) - Phi) * iden;
    const double lmn = lPhi * Phi * iden;
    if (which == 0) lhL += lmn;
    else if (which == 2) lhR += lmn;
    else {
      const double ld = lmn * (1.0 / (1.0 - 2.0 * s1));
      lhbar += ld;
      lhL -= s1 * ld;
      lhR -= s1 * ld;
    }
  }
  LL.h = lhL; LL.m = lmL;  // LL.b unchanged: b enters only through eta = h + b
  LR.h = lhR; LR.m = lmR;
}

// ----------------------------------------------------------------------------
// Reverse of recon_cell.  Recomputes the forward values, then propagates the
// adjoints of the unlimited traces (L, R) and of rint onto the stencil data.
// ----------------------------------------------------------------------------
struct ReconAdjOut {
  double lv[5], lh[5], lm[5], lb[5];
  double letabar;
};

// The 5-cell quartic Q = ubar + a1 y + a2 (y^2 - 1/12) + a3 y^3 + a4 (y^4 -
// 1/80) of one variable from its stencil coefficients B_r, C_r (as
// recon_cell: a3, a4 from stencils 0 and 2 by the 2x2 system of their
// coefficients on y^3 and y^4 - 1/80, a1, a2 from stencil 1), with the
// geometry recomputed from the widths; and the reverse of that map.
struct QuartGeo {
  double qi[4], qb[4];
};
__device__ __forceinline__ void quartic_geo(const double* __restrict__ J5, double iJ0,
                                            QuartGeo& Q) {
  double M1[4], M2[4], M3[4], M4[4];
  stencil_moments(J5, iJ0, M1, M2, M3, M4);
  const int C1[3] = {2, 1, 0}, C2[3] = {3, 2, 1};
  double B3[3], C3[3], B4[3], C4[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int c1 = C1[r], c2 = C2[r];
    const double idet = frcp(M1[c1] * M2[c2] - M1[c2] * M2[c1]);
    const double kb1 = M2[c2] * idet, kb2 = -M2[c1] * idet;
    const double kc1 = -M1[c2] * idet, kc2 = M1[c1] * idet;
    B3[r] = kb1 * M3[c1] + kb2 * M3[c2];
    C3[r] = kc1 * M3[c1] + kc2 * M3[c2];
    B4[r] = kb1 * M4[c1] + kb2 * M4[c2];
    C4[r] = kc1 * M4[c1] + kc2 * M4[c2];
  }
  const double g00 = B3[0] - B3[2], g01 = B4[0] - B4[2];
  const double g10 = C3[0] - C3[2], g11 = C4[0] - C4[2];
  const double igd = frcp(g00 * g11 - g01 * g10);
  Q.qi[0] = g11 * igd; Q.qi[1] = -g01 * igd; Q.qi[2] = -g10 * igd; Q.qi[3] = g00 * igd;
  Q.qb[0] = B3[1]; Q.qb[1] = B4[1]; Q.qb[2] = C3[1]; Q.qb[3] = C4[1];
}
__device__ __forceinline__ void quartic_b(const double* __restrict__ J5, double iJ0,
                                          const double* Bx, const double* Cx, double* a) {
  QuartGeo Q;
  quartic_geo(J5, iJ0, Q);
  const double dB = Bx[0] - Bx[2], dC = Cx[0] - Cx[2];
  a[2] = Q.qi[0] * dB + Q.qi[1] * dC;
  a[3] = Q.qi[2] * dB + Q.qi[3] * dC;
  a[0] = Bx[1] - (a[2] * Q.qb[0] + a[3] * Q.qb[1]);
  a[1] = Cx[1] - (a[2] * Q.qb[2] + a[3] * Q.qb[3]);
}
__device__ __forceinline__ void quartic_b_rev(const double* __restrict__ J5, double iJ0,
                                              const double* la, double* lBx, double* lCx) {
  QuartGeo Q;
  quartic_geo(J5, iJ0, Q);
  lBx[1] += la[0];
  lCx[1] += la[1];
  const double l2 = la[2] - (la[0] * Q.qb[0] + la[1] * Q.qb[2]);
  const double l3 = la[3] - (la[0] * Q.qb[1] + la[1] * Q.qb[3]);
  const double ldB = Q.qi[0] * l2 + Q.qi[2] * l3, ldC = Q.qi[1] * l2 + Q.qi[3] * l3;
  lBx[0] += ldB; lBx[2] -= ldB;
  lCx[0] += ldC; lCx[2] -= ldC;
}

// HR: the interior values of eta and b (points 1, 2) take the cotangents
// le[mu], lb[mu] of the hydrostatic source instead of the special-source term.
template <bool HR = false>
__device__ __forceinline__ void recon_cell_vjp(const double* __restrict__ v5,
                                               const double* __restrict__ h5,
                                               const double* __restrict__ m5,
                                               const double* __restrict__ b5,
                                               const double* __restrict__ J5, double Dx,
                                               double eps, double etabar, const TraceAdj& LL,
                                               const TraceAdj& LR, double lrint,
                                               ReconAdjOut& out, const double* hle = nullptr,
                                               const double* hlb = nullptr) {
  // ---------------- forward (as recon_cell) ----------------
  const double J0 = J5[2];
  const double iJ0 = frcp(J0);
  double M1[4], M2[4], M3[4], M4[4];
  stencil_moments(J5, iJ0, M1, M2, M3, M4);
  const int C1[3] = {2, 1, 0}, C2[3] = {3, 2, 1};
  double kb1[3], kb2[3], kc1[3], kc2[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int c1 = C1[r], c2 = C2[r];
    const double idet = frcp(M1[c1] * M2[c2] - M1[c2] * M2[c1]);
    kb1[r] = M2[c2] * idet;
    kb2[r] = -M2[c1] * idet;
    kc1[r] = -M1[c2] * idet;
    kc2[r] = M1[c1] * idet;
  }
  const double q = 0.22360679774997896964;
  const double q3 = 0.011180339887498948482;
  const double yv[4] = {-0.5, -q, q, 0.5};
  const double p2v[4] = {1.0 / 6.0, -1.0 / 30.0, -1.0 / 30.0, 1.0 / 6.0};
  const double f3v[4] = {-0.125, -q3, q3, 0.125};
  const double f4v[4] = {0.05, -0.01, -0.01, 0.05};
  double d[4][3];
  {
    double B3[3], C3[3], B4[3], C4[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int c1 = C1[r], c2 = C2[r];
      B3[r] = kb1[r] * M3[c1] + kb2[r] * M3[c2];
      C3[r] = kc1[r] * M3[c1] + kc2[r] * M3[c2];
      B4[r] = kb1[r] * M4[c1] + kb2[r] * M4[c2];
      C4[r] = kc1[r] * M4[c1] + kc2[r] * M4[c2];
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      double e3[3], e4[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        e3[r] = B3[r] * yv[mu] + C3[r] * p2v[mu] - f3v[mu];
        e4[r] = B4[r] * yv[mu] + C4[r] * p2v[mu] - f4v[mu];
      }
      const double x0 = e3[1] * e4[2] - e3[2] * e4[1];
      const double x1 = e3[2] * e4[0] - e3[0] * e4[2];
      const double x2 = e3[0] * e4[1] - e3[1] * e4[0];
      const double is = frcp(x0 + x1 + x2);
      d[mu][0] = x0 * is;
      d[mu][1] = x1 * is;
      d[mu][2] = x2 * is;
    }
  }
  const int idx[4] = {0, 1, 3, 4};
  double dv[4], dh[4], dm[4], db[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    dv[c] = v5[idx[c]] - v5[2];
    dh[c] = h5[idx[c]] - h5[2];
    dm[c] = m5[idx[c]] - m5[2];
    db[c] = b5[idx[c]] - b5[2];
  }
  double Bv[3], Cv[3], Bh[3], Ch[3], Bm[3], Cm[3], Bb[3], Cb[3], beta[3];
  const double kap = Dx * iJ0;
  const double kapC = kap * (1.0 / 3.0) + 4.0 * kap * kap * kap;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int c1 = C1[r], c2 = C2[r];
    Bv[r] = kb1[r] * dv[c1] + kb2[r] * dv[c2];
    Cv[r] = kc1[r] * dv[c1] + kc2[r] * dv[c2];
    Bh[r] = kb1[r] * dh[c1] + kb2[r] * dh[c2];
    Ch[r] = kc1[r] * dh[c1] + kc2[r] * dh[c2];
    Bm[r] = kb1[r] * dm[c1] + kb2[r] * dm[c2];
    Cm[r] = kc1[r] * dm[c1] + kc2[r] * dm[c2];
    Bb[r] = kb1[r] * db[c1] + kb2[r] * db[c2];
    Cb[r] = kc1[r] * db[c1] + kc2[r] * db[c2];
    beta[r] = (kap * (Bv[r] * Bv[r]) + kapC * (Cv[r] * Cv[r])) +
              (kap * (Bm[r] * Bm[r]) + kapC * (Cm[r] * Cm[r]));
  }
  const double tau = fabs(beta[0] - beta[2]);
  const double betaA = (beta[0] + beta[1] + beta[2]) * (1.0 / 3.0);
  const double ibA = frcp(betaA + eps);
  const double gam = tau * ibA;
  const int cls = (gam <= 0.5) ? 0 : ((gam >= 1.0) ? 2 : 1);
  double K[3] = {1.0, 1.0, 1.0}, z[3] = {0.0, 0.0, 0.0}, ib[3] = {0.0, 0.0, 0.0};
  if (cls != 0) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      ib[r] = frcp(beta[r] + eps);
      z[r] = tau * ib[r];
      K[r] = 1.0 + z[r] * z[r];
    }
  }
  const double Mg = 2.0 * gam - 1.0;
  // b_x (special source) by the rule of recon_cell: the slopes weighted by ph
  // plus (1 - mq) corr, corr = Q_b' - (the slopes weighted by the linear
  // weights), mq = 0 (smooth), Mg (transition), 1 (non-smooth).  For the
  // smooth class the whole special-source term is reversed after the point
  // loop, through the quartics (nothing of it is held across the loop); the
  // transition class keeps corr and its cotangent at the 4 points.
  const double mq = cls == 0 ? 0.0 : (cls == 1 ? Mg : 1.0);
  double corr[4] = {0, 0, 0, 0}, lab[4] = {0, 0, 0, 0};
  if (!HR && cls == 1) {
    double ab[4];
    quartic_b(J5, iJ0, Bb, Cb, ab);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const double y = yv[mu];
      const double wd = ((d[mu][0] * Bb[0] + d[mu][1] * Bb[1] + d[mu][2] * Bb[2]) +
                         2.0 * y * (d[mu][0] * Cb[0] + d[mu][1] * Cb[1] + d[mu][2] * Cb[2])) * iJ0;
      corr[mu] = (ab[0] + (2.0 * y) * ab[1] + (3.0 * y * y) * ab[2] + (4.0 * y * y * y) * ab[3]) * iJ0 - wd;
    }
  }
  // ---------------- reverse ----------------
  double lBv[3] = {0, 0, 0}, lCv[3] = {0, 0, 0}, lBh[3] = {0, 0, 0}, lCh[3] = {0, 0, 0};
  double lBm[3] = {0, 0, 0}, lCm[3] = {0, 0, 0}, lBb[3] = {0, 0, 0}, lCb[3] = {0, 0, 0};
  double lK[3] = {0, 0, 0}, lMg = 0.0;
  double lh0 = 0.0, lm0 = 0.0, lb0 = 0.0, letab = 0.0;
  double isa_mu[4] = {0, 0, 0, 0};
  const double wgl[4] = {1.0 / 12.0, 5.0 / 12.0, 5.0 / 12.0, 1.0 / 12.0};
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    // forward weights at this point
    double ph[3], phN[3] = {0, 0, 0}, sa = 1.0;
    if (cls == 0) {
      ph[0] = d[mu][0]; ph[1] = d[mu][1]; ph[2] = d[mu][2];
    } else {
      const double a0 = d[mu][0] * K[0], a1 = d[mu][1] * K[1], a2 = d[mu][2] * K[2];
      sa = a0 + a1 + a2;
      const double ia = frcp(sa);
      isa_mu[mu] = ia;
      phN[0] = a0 * ia; phN[1] = a1 * ia; phN[2] = a2 * ia;
#pragma unroll
      for (int r = 0; r < 3; ++r) ph[r] = cls == 1 ? Mg * phN[r] + (1.0 - Mg) * d[mu][r] : phN[r];
    }
    const double y = yv[mu], p2 = p2v[mu];
    double sBh = 0, sCh = 0, sBb = 0, sCb = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      sBh += ph[r] * Bh[r]; sCh += ph[r] * Ch[r];
      sBb += ph[r] * Bb[r]; sCb += ph[r] * Cb[r];
    }
    const double hv = h5[2] + (sBh * y + sCh * p2);
    const double bv = b5[2] + (sBb * y + sCb * p2);
    const double bxv = (sBb + 2.0 * y * sCb) * iJ0 + (1.0 - mq) * corr[mu];
    // adjoints of the values at this point
    double lhv = 0.0, lmv = 0.0, lbv = 0.0, lbx = 0.0;
    if (mu == 0) { lhv += LL.h; lmv += LL.m; lbv += LL.b; }
    if (mu == 3) { lhv += LR.h; lmv += LR.m; lbv += LR.b; }
    if (HR) {
      // eta = h + b and b at the interior points feed the hydrostatic source
      if (mu == 1 || mu == 2) { lhv += hle[mu]; lbv += hle[mu] + hlb[mu]; }
    } else if (cls != 0) {
      // rint = sum_mu (w_mu J0) ((h + b) - etabar) b_x
      const double cw = wgl[mu] * J0;
      lhv += lrint * cw * bxv;
      lbv += lrint * cw * bxv;
      lbx += lrint * cw * ((hv + bv) - etabar);
      letab -= lrint * cw * bxv;
    }
    // v = v0 + (sB y + sC p2); b_x = (sB_b + 2 y sC_b) / J0
    lh0 += lhv; lm0 += lmv; lb0 += lbv;
    if (cls == 1) {
      // b_x's correction (1 - Mg) corr onto Mg, onto the linear weights'
      // slopes here and onto the quartic's coefficients (reversed after the
      // loop)
      const double lq = (1.0 - Mg) * lbx * iJ0;
      lMg -= corr[mu] * lbx;
      lab[0] += lq; lab[1] += (2.0 * y) * lq; lab[2] += (3.0 * y * y) * lq;
      lab[3] += (4.0 * y * y * y) * lq;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        lBb[r] -= d[mu][r] * lq;
        lCb[r] -= d[mu][r] * (2.0 * y * lq);
      }
    }
    const double lsBh = y * lhv, lsCh = p2 * lhv;
    const double lsBm = y * lmv, lsCm = p2 * lmv;
    const double lsBb = y * lbv + iJ0 * lbx, lsCb = p2 * lbv + 2.0 * y * iJ0 * lbx;
    double lph[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      lph[r] = Bh[r] * lsBh + Ch[r] * lsCh + Bm[r] * lsBm + Cm[r] * lsCm + Bb[r] * lsBb +
               Cb[r] * lsCb;
      lBh[r] += ph[r] * lsBh; lCh[r] += ph[r] * lsCh;
      lBm[r] += ph[r] * lsBm; lCm[r] += ph[r] * lsCm;
      lBb[r] += ph[r] * lsBb; lCb[r] += ph[r] * lsCb;
    }
    if (cls != 0) {
      double lphN[3];
      if (cls == 1) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          lphN[r] = Mg * lph[r];
          lMg += (phN[r] - d[mu][r]) * lph[r];
        }
      } else {
        lphN[0] = lph[0]; lphN[1] = lph[1]; lphN[2] = lph[2];
      }
      const double dotp = phN[0] * lphN[0] + phN[1] * lphN[1] + phN[2] * lphN[2];
#pragma unroll
      for (int r = 0; r < 3; ++r) lK[r] += d[mu][r] * ((lphN[r] - dotp) * isa_mu[mu]);
    }
  }
  if (!HR && cls != 2) {
    // reverse of the quartic parts: for the smooth class the special-source
    // term sum_mu (w_mu J0) (eta_mu - etabar) Q_b'(y_mu) / J0 with eta_mu =
    // ubar_h + ubar_b + Q_h(y_mu) + Q_b(y_mu) (the smooth values are the
    // quartics'); for the transition class corr = Q_b' - weighted slopes
    asm volatile("" ::: "memory");
    if (cls == 0) {
      double ab[4];
      quartic_b(J5, iJ0, Bb, Cb, ab);
      double ah[4], lah[4] = {0, 0, 0, 0};
      quartic_b(J5, iJ0, Bh, Ch, ah);
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        const double y = yv[mu], p2 = p2v[mu], f3 = f3v[mu], f4 = f4v[mu];
        const double dy2 = 2.0 * y, dy3 = 3.0 * y * y, dy4 = 4.0 * y * y * y;
        const double eta = (h5[2] + (ah[0] * y + ah[1] * p2 + ah[2] * f3 + ah[3] * f4)) +
                           (b5[2] + (ab[0] * y + ab[1] * p2 + ab[2] * f3 + ab[3] * f4));
        const double bxv = (ab[0] + dy2 * ab[1] + dy3 * ab[2] + dy4 * ab[3]) * iJ0;
        const double cw = wgl[mu] * J0;
        const double le = lrint * cw * bxv;      // onto h and b at the point
        const double lbx = lrint * cw * (eta - etabar);
        letab -= le;
        lh0 += le;
        lb0 += le;
        lah[0] += y * le; lah[1] += p2 * le; lah[2] += f3 * le; lah[3] += f4 * le;
        const double lbj = iJ0 * lbx;
        lab[0] += y * le + lbj;
        lab[1] += p2 * le + dy2 * lbj;
        lab[2] += f3 * le + dy3 * lbj;
        lab[3] += f4 * le + dy4 * lbj;
      }
      quartic_b_rev(J5, iJ0, lah, lBh, lCh);
    }
    quartic_b_rev(J5, iJ0, lab, lBb, lCb);
  }
  double lbeta[3] = {0, 0, 0}, ltau = 0.0;
  if (cls != 0) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double lz = 2.0 * z[r] * lK[r];
      ltau += lz * ib[r];
      lbeta[r] -= lz * z[r] * ib[r];
    }
  }
  if (cls == 1) {
    const double lgam = 2.0 * lMg;
    ltau += lgam * ibA;
    const double lbA = -lgam * gam * ibA;
#pragma unroll
    for (int r = 0; r < 3; ++r) lbeta[r] += lbA * (1.0 / 3.0);
  }
  {
    const double dd = beta[0] - beta[2];
    const double sg = dd > 0.0 ? 1.0 : (dd < 0.0 ? -1.0 : 0.0);
    lbeta[0] += sg * ltau;
    lbeta[2] -= sg * ltau;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    lBv[r] += 2.0 * kap * Bv[r] * lbeta[r];
    lCv[r] += 2.0 * kapC * Cv[r] * lbeta[r];
    lBm[r] += 2.0 * kap * Bm[r] * lbeta[r];
    lCm[r] += 2.0 * kapC * Cm[r] * lbeta[r];
  }
  double ldv[4] = {0, 0, 0, 0}, ldh[4] = {0, 0, 0, 0}, ldm[4] = {0, 0, 0, 0}, ldb[4] = {0, 0, 0, 0};
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int c1 = C1[r], c2 = C2[r];
    ldv[c1] += kb1[r] * lBv[r] + kc1[r] * lCv[r]; ldv[c2] += kb2[r] * lBv[r] + kc2[r] * lCv[r];
    ldh[c1] += kb1[r] * lBh[r] + kc1[r] * lCh[r]; ldh[c2] += kb2[r] * lBh[r] + kc2[r] * lCh[r];
    ldm[c1] += kb1[r] * lBm[r] + kc1[r] * lCm[r]; ldm[c2] += kb2[r] * lBm[r] + kc2[r] * lCm[r];
    ldb[c1] += kb1[r] * lBb[r] + kc1[r] * lCb[r]; ldb[c2] += kb2[r] * lBb[r] + kc2[r] * lCb[r];
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) { out.lv[k] = 0; out.lh[k] = 0; out.lm[k] = 0; out.lb[k] = 0; }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    out.lv[idx[c]] += ldv[c]; out.lv[2] -= ldv[c];
    out.lh[idx[c]] += ldh[c]; out.lh[2] -= ldh[c];
    out.lm[idx[c]] += ldm[c]; out.lm[2] -= ldm[c];
    out.lb[idx[c]] += ldb[c]; out.lb[2] -= ldb[c];
  }
  out.lh[2] += lh0;
  out.lm[2] += lm0;
  out.lb[2] += lb0;
  out.letabar = letab;
}

// ----------------------------------------------------------------------------
// Kernels of the reverse stage
// ----------------------------------------------------------------------------
struct AdjTile {
  int32_t inst;
  int32_t pad;
  int64_t c0;
  int64_t co;  // cell offset of the instance
  int64_t n;   // cells of the instance
};

// lambda_alpha of each instance from its fused tiles' parts (the tiles of
// instance i are tfirst[i] .. tfirst[i+1]-1): one wave per instance, lane l
// sums the parts l, l+64, ... and the lanes are combined by a fixed butterfly,
// so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_adj_lsum(AdjBufs ab, const int64_t* __restrict__ tfirst) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= ab.ninst) return;
  double acc = 0.0;
  for (int64_t k = tfirst[i] + lane; k < tfirst[i + 1]; k += 64) acc += ab.lpart[k];
  acc = wave_sum(acc);
  if (lane == 0) ab.lalpha[i] = acc;
}


// ----------------------------------------------------------------------------
// Fused reverse stage.  A tile owns the TB = B - 6 cells [c0, c0 + TB) and
// recomputes two cells of halo on each side, so that every stencil
// contribution to an owned cell is formed inside the tile and summed in LDS:
//   slots      cells c0-5 .. c0+B-2        (stencil data, rho)
//   thread t   reconstructs cell j = c0-3+t (forward, limited traces),
//              owns the face at node j,
//              for 1 <= t <= B-2 takes the reverse of cell j (limiter and
//              reconstruction), writing its 5 x 3 stencil contributions.
// Contributions to ghost cells (only the first and the last tile of an
// instance see them) go to a per-instance buffer and are folded onto their
// source cells by k_adj_fold, so tiles never add into each other's cells.
// ----------------------------------------------------------------------------
template <int B>
struct SmemAdjF {
  double e[B + 4], m[B + 4], b[B + 4], J[B + 4];
  double rho[3][B + 4];
  union {
    double tr[6][B];   // limited traces (faces)
    double cl[15][B];  // stencil contributions of the reversed cells
  } u;
  double lf[6][B];
  double B1[B];
  double wn[B + 4];   // node speed at the left node of slot q (nodes 0..n)
  double jd[3][B];    // jumps of eta, hu, b at the faces (alpha coefficients)
  // owned slots (loaded with the stencil, used by the last phase):
  double mu[3][B];    // lambda^(s) / J^(s)
  double lb[3][B];    // lambda of q^n accumulated up to this stage
};

// gfold layout: [ninst][2 ends][3 ghost cells][3 components], ends: left
// ghosts -3..-1, right ghosts n..n+2.
// Stencil slot q of a fused tile (cell k = c0 - 5 + q): the stage input, the
// stage width and rho = b_s dt lambda^(s) / J^(s) into LDS; for an owned cell
// also the pieces the last phase combines, and its part of lambda_alpha.  All
// loads of a thread's slots are issued before the first use.
struct AdjSlotRaw {
  double x0, x1, w0, w1, wk, e, m, b, l0, l1, l2, lb0, lb1, lb2;
  double ms;
  bool in, real, own;
};

__device__ __forceinline__ AdjSlotRaw adj_slot_load(const AdjBufs& ab, const Consts& cs,
                                                    const double* x, const double* w, int64_t co,
                                                    int64_t n, int64_t k, int64_t own_beg,
                                                    int64_t own_end, int s) {
  AdjSlotRaw r;
  r.in = k >= -3 && k < n + 3;
  r.real = k >= 0 && k < n;
  r.own = r.real && k >= own_beg && k < own_end;
  r.x0 = r.x1 = r.w0 = r.w1 = 0.0;
  r.e = r.m = r.b = 0.0;
  r.l0 = r.l1 = r.l2 = r.lb0 = r.lb1 = r.lb2 = 0.0;
  r.ms = 1.0;
  r.wk = (k >= 0 && k <= n) ? w[k] : 0.0;
  if (r.in) {
    const int64_t src = ghost_src(cs.bc, n, k, r.ms);
    r.x0 = x[src]; r.x1 = x[src + 1]; r.w0 = w[src]; r.w1 = w[src + 1];
    const int64_t g = co + src;
    r.e = ab.q[g]; r.m = ab.q[ab.S + g]; r.b = ab.q[2 * ab.S + g];
    if (r.real) {
      r.l0 = ab.lam[g]; r.l1 = ab.lam[ab.S + g]; r.l2 = ab.lam[2 * ab.S + g];
    }
    if (r.own && s != 3) {
      r.lb0 = ab.lbase[g]; r.lb1 = ab.lbase[ab.S + g]; r.lb2 = ab.lbase[2 * ab.S + g];
    }
  }
  return r;
}

// Widths and LDS stores of a loaded slot.
template <int B>
__device__ __forceinline__ void adj_slot_put(const AdjSlotRaw& r, int q, double dt, int s,
                                             SmemAdjF<B>& sm) {
  double e = 0, m = 0, b = 0, J = 1, r0 = 0, r1 = 0, r2 = 0;
  if (r.in) {
    // the widths of stage_widths() from the raw node values
    const double Jn = r.x1 - r.x0;
    const double dw = r.w1 - r.w0;
    const double J1 = Jn + dt * dw;
    const double J2 = 0.75 * Jn + 0.25 * (J1 + dt * dw);
    const double J3 = (1.0 / 3.0) * Jn + (2.0 / 3.0) * (J2 + dt * dw);
    const double Jin = s == 1 ? Jn : (s == 2 ? J1 : J2);
    const double Jout = s == 1 ? J1 : (s == 2 ? J2 : J3);
    const double bs = stage_b(s);
    e = r.e;
    m = r.m * r.ms;
    b = r.b;
    J = Jin;
    if (r.real) {
      const double rf = bs * dt / Jout;
      r0 = rf * r.l0;
      r1 = rf * r.l1;
      r2 = rf * r.l2;
    }
    if (r.own) {
      const double mu[3] = {r.l0 / Jout, r.l1 / Jout, r.l2 / Jout};
      const double lbv[3] = {r.lb0, r.lb1, r.lb2};
      const double as = stage_a(s);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sm.mu[c][q] = mu[c];
        const double base = as * Jn * mu[c];
        sm.lb[c][q] = s == 3 ? base : lbv[c] + base;
      }
    }
  }
  sm.e[q] = e; sm.m[q] = m; sm.b[q] = b; sm.J[q] = J;
  sm.rho[0][q] = r0; sm.rho[1][q] = r1; sm.rho[2][q] = r2;
  sm.wn[q] = r.wk;
}

template <int B, bool HR>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(2))) void k_adj_fused(AdjBufs ab, Consts cs,
                                                 const AdjTile* __restrict__ tiles, int s,
                                                 double* __restrict__ gfold) {
  constexpr int TB = B - 6;
  __shared__ SmemAdjF<B> sm;
  const AdjTile tl = tiles[blockIdx.x];
  const int i = tl.inst;
  const int64_t co = tl.co, n = tl.n, no = co + i;
  const int64_t c0 = tl.c0;
  const int t = threadIdx.x;
  const double* x = ab.x + no;
  const double* w = ab.w + no;
  // 1. stencil data and rho for cells c0-5 .. c0+B-2 (slots 0 .. B+3); the
  // owned cells c0 .. c0+TB-1 are the slots 5 .. TB+4
  const int64_t own_end = c0 + TB < n ? c0 + TB : n;
  const AdjSlotRaw ra0 = adj_slot_load(ab, cs, x, w, co, n, c0 - 5 + t, c0, own_end, s);
  const bool ext = t < 4;
  AdjSlotRaw ra1;
  if (ext) ra1 = adj_slot_load(ab, cs, x, w, co, n, c0 - 5 + B + t, c0, own_end, s);
  // per-instance scalars of the step (not written during the reverse sweep)
  typedef const __attribute__((address_space(4))) double* cdbl;
  const cdbl sc8 = (cdbl)ab.scal + (int64_t)i * 8;
  const double dt = sc8[1];
  const double alpha = sc8[1 + s];
  const double dx = sc8[5 + (s - 1)];
  adj_slot_put<B>(ra0, t, dt, s, sm);
  if (ext) adj_slot_put<B>(ra1, B + t, dt, s, sm);
  lds_sync();
  // 2. forward reconstruction and limiter of cell j = c0 - 3 + t (stencil slots t .. t+4)
  const int64_t j = c0 - 3 + t;
  const bool active = (j >= -1) && (j <= n);
  CellRecon o, ou;
  double h5[5], v5[5];
  double Dx = dx;
  if (active) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      h5[k] = sm.e[t + k] - sm.b[t + k];
      v5[k] = (cs.flags & F_BETA_FROM_H) ? h5[k] : sm.e[t + k];
    }
    if (cs.flags & F_BETA_LOCAL) Dx = sm.J[t + 2];
    recon_cell<HR>(v5, h5, &sm.m[t], &sm.b[t], &sm.J[t], frcp(sm.J[t + 2]), Dx, cs.weno_eps,
                   sm.e[t + 2], o);
    ou = o;
    limit_cell(h5[2], sm.m[t + 2], cs.pp_eps, o, !(cs.flags & F_NO_HU_LIMIT));
    sm.u.tr[0][t] = o.hL; sm.u.tr[1][t] = o.mL; sm.u.tr[2][t] = o.bL;
    sm.u.tr[3][t] = o.hR; sm.u.tr[4][t] = o.mR; sm.u.tr[5][t] = o.bR;
  }
  lds_sync();
  // 3. face at node j between cells j-1 (slot t+1) and j (slot t+2)
  if (t >= 1 && j >= 0 && j <= n) {
    const double rl[3] = {sm.rho[0][t + 1], sm.rho[1][t + 1], sm.rho[2][t + 1]};
    const double rr[3] = {sm.rho[0][t + 2], sm.rho[1][t + 2], sm.rho[2][t + 2]};
    const double hl = sm.u.tr[3][t - 1], ml = sm.u.tr[4][t - 1], bl = sm.u.tr[5][t - 1];
    const double hr = sm.u.tr[0][t], mr = sm.u.tr[1][t], br = sm.u.tr[2][t];
    TraceAdj Ll, Lr;
    if (HR)
      face_vjp_hydro(hl, ml, bl, hr, mr, br, sm.wn[t + 2], alpha, cs.g, cs.dry_eps, rl, rr, Ll, Lr);
    else
      face_vjp(hl, ml, bl, hr, mr, br, sm.wn[t + 2], alpha, cs.g, cs.dry_eps, rl, rr, sm.e[t + 1],
               sm.e[t + 2], Ll, Lr);
    sm.lf[0][t] = Ll.h; sm.lf[1][t] = Ll.m; sm.lf[2][t] = Ll.b;
    sm.lf[3][t] = Lr.h; sm.lf[4][t] = Lr.m; sm.lf[5][t] = Lr.b;
    sm.B1[t] = 0.5 * (bl + br);
    // the jumps of the forward face (its alpha coefficients), dry momenta cut
    sm.jd[0][t] = (hr + br) - (hl + bl);
    sm.jd[1][t] = (hr > cs.dry_eps ? mr : 0.0) - (hl > cs.dry_eps ? ml : 0.0);
    sm.jd[2][t] = br - bl;
  }
  lds_sync();  // the traces are dead from here on: their LDS takes the contributions
  // 4. reverse of cell j for 1 <= t <= B-2; contributions to stencil slots t .. t+4
  double cv[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) cv[k] = 0.0;
  if (t >= 1 && t <= B - 2 && active) {
    TraceAdj LL{0, 0, 0}, LR{0, 0, 0};
    if (j >= 0) { LL.h = sm.lf[3][t]; LL.m = sm.lf[4][t]; LL.b = sm.lf[5][t]; }
    if (j < n) { LR.h = sm.lf[0][t + 1]; LR.m = sm.lf[1][t + 1]; LR.b = sm.lf[2][t + 1]; }
    double lrint = 0.0, letabar = 0.0;
    double hle[4] = {0.0, 0.0, 0.0, 0.0}, hlb[4] = {0.0, 0.0, 0.0, 0.0};
    if (j >= 0 && j < n) {
      const double rm = sm.rho[1][t + 2];
      if (HR) {
        // hydrostatic source of the cell: limited end traces, interior values
        const double ev[4] = {o.hL + o.bL, o.e1, o.e2, o.hR + o.bR};
        const double bv[4] = {o.bL, o.b1, o.b2, o.bR};
        hydro_source_vjp(cs.g, ev, bv, rm, hle, hlb);
        LL.h += hle[0]; LL.b += hle[0] + hlb[0];
        LR.h += hle[3]; LR.b += hle[3] + hlb[3];
      } else {
        lrint = -cs.g * rm;
        letabar += -cs.g * rm * (sm.B1[t + 1] - sm.B1[t]);
      }
    }
    double lhbar = 0.0, lmbar = 0.0;
    limit_vjp(h5[2], sm.m[t + 2], cs.pp_eps, ou, LL, LR, lhbar, lmbar, !(cs.flags & F_NO_HU_LIMIT));
    ReconAdjOut ra;
    recon_cell_vjp<HR>(v5, h5, &sm.m[t], &sm.b[t], &sm.J[t], Dx, cs.weno_eps, sm.e[t + 2], LL, LR,
                       lrint, ra, hle, hlb);
    const bool vh = (cs.flags & F_BETA_FROM_H) != 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double lh = ra.lh[k] + (vh ? ra.lv[k] : 0.0);
      double le = lh + (vh ? 0.0 : ra.lv[k]);
      double lb = ra.lb[k] - lh;
      double lm = ra.lm[k];
      if (k == 2) {
        le += lhbar + letabar + ra.letabar;
        lb -= lhbar;
        lm += lmbar;
      }
      cv[3 * k + 0] = le; cv[3 * k + 1] = lm; cv[3 * k + 2] = lb;
    }
  }
#pragma unroll
  for (int k = 0; k < 15; ++k) sm.u.cl[k][t] = cv[k];
  lds_sync();
  // 5. owned cell k = c0 + t: slot i = t + 5 collects offset o from the cell of thread i - o;
  // its faces are those of threads t + 3 and t + 4
  double lap = 0.0;  // rho . D of the owned cell (part of lambda_alpha)
  if (t < TB && c0 + t < n) {
    const int64_t g = co + c0 + t;
    const int si = t + 5;
    const double bs = stage_b(s), Jin = sm.J[si];
    double acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double mu = sm.mu[c][si];
      const double Dc = 0.5 * (sm.jd[c][t + 4] - sm.jd[c][t + 3]);
      lap += (bs * dt * mu) * Dc;
      acc[c] = bs * Jin * mu;
    }
#pragma unroll
    for (int oo = 0; oo < 5; ++oo) {
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += sm.u.cl[3 * oo + c][si - oo];
    }
    double* lo = ab.lam_out;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double lb = sm.lb[c][si];
      if (s == 1) {
        lo[c * ab.S + g] = acc[c] + lb;
      } else {
        lo[c * ab.S + g] = acc[c];
        ab.lbase[c * ab.S + g] = lb;
      }
    }
  }
  // ghost cells: the first tile has the left ones (slots 2..4), the last tile
  // the right ones (slots n-c0+5 .. n-c0+7)
  const int gi = t % 3, gc = (t / 3) % 3, gend = t / 9;  // t < 18: 2 ends x 3 cells x 3 comps
  if (t < 18) {
    const bool mine = gend == 0 ? (c0 == 0) : (c0 + TB >= n);
    if (mine) {
      const int64_t kg = gend == 0 ? (-3 + gi) : (n + gi);
      const int si = (int)(kg - (c0 - 5));
      double acc = 0.0;
#pragma unroll
      for (int oo = 0; oo < 5; ++oo) {
        const int tv = si - oo;
        if (tv >= 0 && tv < B) acc += sm.u.cl[3 * oo + gc][tv];
      }
      gfold[(((int64_t)i * 2 + gend) * 3 + gi) * 3 + gc] = acc;
    }
  }
  double rv[1] = {lap};
  const int op[1] = {2};
  block_reduce<B, 1>(rv, op, sm.lf[0]);
  if (t == 0) ab.lpart[blockIdx.x] = rv[0];
}

// The alpha term of the reverse stage: lambda_alpha times the derivative of
// the LF speed at the trace that attains it, through the limiter and the
// reconstruction of that trace's cell (a ghost cell at an end is possible),
// added onto lambda^(s-1) after k_adj_fused and k_adj_fold.  One thread per
// instance.
__global__ __launch_bounds__(64) void k_adj_patch(AdjBufs ab, Consts cs, int s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ab.ninst) return;
  const double lal = ab.lalpha[i];
  const double kd = ab.akeyd[i];
  if (lal == 0.0 || !(kd >= 0.0 && kd < 1e18)) return;
  const int64_t co = ab.cell_off[i], n = ab.cell_off[i + 1] - co, no = co + i;
  const int64_t key = (int64_t)kd;
  const int64_t f = key >> 1;
  const int side = (int)(key & 1);
  if (f < 0 || f > n) return;
  const int64_t cc = side ? f : f - 1;  // the cell whose trace it is (-1 .. n)
  const double* x = ab.x + no;
  const double* w = ab.w + no;
  const double dt = ab.scal[(int64_t)i * 8 + 1];
  double Dx = ab.scal[(int64_t)i * 8 + 5 + (s - 1)];
  double e5[5], m5[5], b5[5], J5[5], h5[5], v5[5], ms5[5];
  int64_t src5[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double ms;
    const int64_t src = ghost_src(cs.bc, n, cc - 2 + k, ms);
    double Jn, Jin, Jout;
    stage_widths(x, w, src, dt, s, Jn, Jin, Jout);
    const int64_t g = co + src;
    e5[k] = ab.q[g];
    m5[k] = ab.q[ab.S + g] * ms;
    b5[k] = ab.q[2 * ab.S + g];
    J5[k] = Jin;
    src5[k] = src;
    ms5[k] = ms;
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    h5[k] = e5[k] - b5[k];
    v5[k] = (cs.flags & F_BETA_FROM_H) ? h5[k] : e5[k];
  }
  if (cs.flags & F_BETA_LOCAL) Dx = J5[2];
  CellRecon o;
  recon_cell(v5, h5, m5, b5, J5, frcp(J5[2]), Dx, cs.weno_eps, e5[2], o);
  const CellRecon ou = o;
  limit_cell(h5[2], m5[2], cs.pp_eps, o, !(cs.flags & F_NO_HU_LIMIT));
  TraceAdj LL{0, 0, 0}, LR{0, 0, 0};
  if (side == 0) alpha_trace_vjp(o.hR, o.mR, w[f], cs.g, cs.dry_eps, lal, LR);
  else alpha_trace_vjp(o.hL, o.mL, w[f], cs.g, cs.dry_eps, lal, LL);
  double lhbar = 0.0, lmbar = 0.0;
  limit_vjp(h5[2], m5[2], cs.pp_eps, ou, LL, LR, lhbar, lmbar, !(cs.flags & F_NO_HU_LIMIT));
  ReconAdjOut ra;
  recon_cell_vjp(v5, h5, m5, b5, J5, Dx, cs.weno_eps, e5[2], LL, LR, 0.0, ra);
  const bool vh = (cs.flags & F_BETA_FROM_H) != 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double lh = ra.lh[k] + (vh ? ra.lv[k] : 0.0);
    double le = lh + (vh ? 0.0 : ra.lv[k]);
    double lb = ra.lb[k] - lh;
    double lm = ra.lm[k];
    if (k == 2) {
      le += lhbar + ra.letabar;
      lb -= lhbar;
      lm += lmbar;
    }
    const int64_t g = co + src5[k];
    ab.lam_out[g] += le;
    ab.lam_out[ab.S + g] += ms5[k] * lm;
    ab.lam_out[2 * ab.S + g] += lb;
  }
}

// Ghost-cell contributions onto their source cells (after k_adj_fused); one
// thread per instance, fixed order.
__global__ void k_adj_fold(AdjBufs ab, Consts cs, const double* __restrict__ gfold) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ab.ninst) return;
  const int64_t co = ab.cell_off[i], n = ab.cell_off[i + 1] - co;
  for (int gend = 0; gend < 2; ++gend)
    for (int gi = 0; gi < 3; ++gi) {
      const int64_t kg = gend == 0 ? (-3 + gi) : (n + gi);
      double ms;
      const int64_t src = ghost_src(cs.bc, n, kg, ms);
      const double* v = gfold + (((int64_t)i * 2 + gend) * 3 + gi) * 3;
      const int64_t g = co + src;
      ab.lam_out[g] += v[0];
      ab.lam_out[ab.S + g] += ms * v[1];
      ab.lam_out[2 * ab.S + g] += v[2];
    }
}

}  // namespace alew_dev
