// MI355X (gfx950) kernels and C ABI of the 2D extension: the well-balanced
// ALE-WENO hybrid scheme with the special source-term treatment (Sec. 2-4 in
// two dimensions) on a tensor-product moving mesh, whose nodes move along each
// logical direction on their own,
//     x_i(t) = xi_i + Ax sin(2 pi kx xi_i) sin(omx t),
//     y_j(t) = eta_j + Ay sin(2 pi ky eta_j) sin(omy t),
// so that every cell stays a rectangle [x_i, x_i+1] x [y_j, y_j+1].
//
// One stage of the modified SSP-RK3 of eq. (3.14) with the area recurrence of
// eq. (3.15) (div(w) J = dA/dt = dwx dy + dx dwy on the stage mesh) is two
// kernels:
//  * x-sweep (a work-group per row segment): finishes the previous stage's
//    update on every cell it stages in LDS (the global Lax-Friedrichs speed of
//    that stage is known only after it), writes the stage state, and runs the
//    hybrid WENO reconstruction of Sec. 2.2 along x on each cell's 5-cell row
//    stencil: h, hu, hv, b and db/dx, averaged over the cell's y-extent, at
//    the 4 Gauss-Lobatto abscissae of the cell (20 line values per cell, SoA
//    planes in HBM), and the cell's x-class.
//  * y-sweep (a wavefront per strip of 62 columns, marching up a chunk of
//    rows): reconstructs the line values along y at every abscissa (4 sweeps
//    per cell) to the 4 x 4 tensor Gauss-Lobatto points, evaluates the
//    Lax-Friedrichs edge fluxes at the 4 points of each edge (left edges with
//    the left neighbour's traces taken by a lane shuffle, bottom edges with the
//    cell below's traces kept in registers from the previous row), the bottom's
//    ALE flux, the special source (edge terms B1, B2 and the 4 x 4 interior
//    rule), and writes the right-hand side split as Rc + alpha Rd with the
//    stage's largest trace speed taken by one atomic max per wavefront.
// A single work-group computes the step's size, node speeds, stage widths and
// the reconstruction geometry of every column and row at the three stage
// meshes (the geometry of a tensor-product mesh depends on the column or the
// row only), and an epilogue kernel finishes the third stage.  Every step is
// 8 launches; a status word in device memory stops the remaining launches of
// a run once it reaches t_end or max_steps.  No MFMA: nothing here is a dense
// contraction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "alew.h"
#include "alew_device.h"

using namespace alew_dev;

alew_status alew_set_error(alew_status s, const char* msg);  // alew.hip

namespace alew2d {

// Geometry table of one column (x) or row (y) at one stage mesh: the stencil
// maps B_r = kb1 du_c1 + kb2 du_c2, C_r = kc1 du_c1 + kc2 du_c2 in the
// zero-mean basis (y, y^2 - 1/12) of the cell, the linear weights at the 4
// Gauss-Lobatto points, the indicator factors Dx / width and its y^2
// counterpart, and 1 / width.  SoA: field f of entry e at stage s is
// T[(f * 3 + s) * n_entries + e].
enum { GF_KB1 = 0, GF_KB2 = 3, GF_KC1 = 6, GF_KC2 = 9, GF_D = 12, GF_KAP = 24, GF_KAPC = 25,
       GF_IJ = 26, GF_QI = 27, GF_QB = 31, NGF = 35 };

constexpr int STRIP = 62;  // columns owned by a y-sweep wavefront (64 lanes, one ring each side)
constexpr int XB = 256;    // x-sweep work-group (row segment)
constexpr int KB = 1024;   // kinematics work-group
constexpr unsigned long long CLS_SIG_MUL = 1099511628211ull;

struct State2 {
  double t, dt, t_end, dt_min, dt_max;
  double Dx[3], Dy[3];
  int64_t steps, max_steps;
  unsigned long long alpha[3];  // bits of each stage's LF speed (non-negative: integer max)
  unsigned long long n_class[3];
  unsigned long long n_limited;
  int32_t status, done, timed, pad;
};

struct K2 {
  double g, cfl, eps, dry;
  double Ax, kx, omx, Ay, ky, omy;
  double Vx, Vy;  // uniform node translation
  int32_t bcx, bcy, nx, ny;
  int64_t N, LW, PL4;  // cells; row length of the line-value planes, 4 x their cells
  double* qa;         // [4][N] step state (eta, hu, hv, b)
  double* qs0;        // [4][N] stage states (even / odd stages)
  double* qs1;
  double* L;          // [5][ny][LW][4] line values (h, hu, hv, b, db/dx) at the 4 abscissae
  uint8_t* xcls;      // [ny][LW]
  double* Rc;         // [4][N] right-hand side: Rc + alpha Rd
  double* Rd;
  double *dx0, *dwx, *dy0, *dwy, *wx, *wy;
  double *Gx, *Gy;    // geometry tables, entries nx + 2 (columns -1..nx), ny + 2
  double *x, *y;
  const double *xi, *yi;
  State2* st;
  uint8_t* cls;                // [3][N] classes of the last step (or NULL)
  uint32_t* ccount;            // [3][N] class counts over the run (or NULL)
  unsigned long long* csig;    // [N] class sequence signatures (or NULL)
  double* part;                // [2][ny] row sums of the mass diagnostics
  double* spart;               // [nspart] work-group maxima of the wave speed (next dt)
  int64_t nspart;
};

__device__ __forceinline__ int wrapi(int bc, int n, int k) {
  if (k >= 0 && k < n) return k;
  if (bc == BC_PERIODIC) return ((k % n) + n) % n;
  return k < 0 ? 0 : n - 1;
}

constexpr double GLW[4] = {1.0 / 12.0, 5.0 / 12.0, 5.0 / 12.0, 1.0 / 12.0};

// stage constants of eq. (3.14): Q^(s+1) = CA_s Q^n + CB_s (Q^(s) + dt R^(s)) on
// the stage mesh at t_n + TAU_s
__device__ __forceinline__ double CA(int s) { return s == 0 ? 0.0 : (s == 1 ? 0.75 : 1.0 / 3.0); }
__device__ __forceinline__ double CB(int s) { return s == 0 ? 1.0 : (s == 1 ? 0.25 : 2.0 / 3.0); }
__device__ __forceinline__ double TAU(int s, double dt) { return s == 0 ? 0.0 : (s == 1 ? dt : 0.5 * dt); }

// Areas J^(0..S) of cell (i, j) by the recurrence of eq. (3.15).
template <int S>
__device__ __forceinline__ void jrec(double dx0, double dwx, double dy0, double dwy, double dt,
                                     double (&J)[S + 1]) {
  J[0] = dx0 * dy0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double ta = TAU(s, dt);
    const double dxs = dx0 + ta * dwx, dys = dy0 + ta * dwy;
    const double dA = dwx * dys + dxs * dwy;
    J[s + 1] = CA(s) * J[0] + CB(s) * (J[s] + dt * dA);
  }
}

// The state of stage S (S >= 1) of one cell from the stage-(S-1) state, its
// right-hand side Rc + alpha Rd and the step state.
template <int S>
__device__ __forceinline__ void stage_update(const K2& k, int64_t c, double dx0, double dwx,
                                             double dy0, double dwy, double dt, double alpha,
                                             const double* __restrict__ qprev, double (&q)[4],
                                             double& Jn) {
  double J[S + 1];
  jrec<S>(dx0, dwx, dy0, dwy, dt, J);
  Jn = J[S];
  const double iJS = frcp(J[S]);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double R = k.Rc[v * k.N + c] + alpha * k.Rd[v * k.N + c];
    const double Q = CA(S - 1) * (J[0] * k.qa[v * k.N + c]) +
                     CB(S - 1) * (J[S - 1] * qprev[v * k.N + c] + dt * R);
    q[v] = Q * iJS;
  }
}

struct Geo {
  double kb1[3], kb2[3], kc1[3], kc2[3], d[4][3], kap, kapC, iJ;
  // the quartic's fields (GF_QI, GF_QB), read where the sweep needs them
  const double* tq;
  int64_t tst;
};

__device__ __forceinline__ void load_geo(const double* __restrict__ T, int64_t ne, int s, int64_t e,
                                         Geo& G) {
  auto f = [&](int fld) { return T[((int64_t)fld * 3 + s) * ne + e]; };
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    G.kb1[r] = f(GF_KB1 + r);
    G.kb2[r] = f(GF_KB2 + r);
    G.kc1[r] = f(GF_KC1 + r);
    G.kc2[r] = f(GF_KC2 + r);
  }
#pragma unroll
  for (int mu = 0; mu < 4; ++mu)
#pragma unroll
    for (int r = 0; r < 3; ++r) G.d[mu][r] = f(GF_D + mu * 3 + r);
  G.kap = f(GF_KAP);
  G.kapC = f(GF_KAPC);
  G.iJ = f(GF_IJ);
  G.tq = T + ((int64_t)GF_QI * 3 + s) * ne + e;
  G.tst = 3 * ne;
}

// B_r, C_r of the three candidate stencils of one variable (Sec. 2.2, Step 1)
__device__ __forceinline__ void stencil_bc(const Geo& G, const double* u, double* B, double* C) {
  const double du[4] = {u[0] - u[2], u[1] - u[2], u[3] - u[2], u[4] - u[2]};
  const int C1[3] = {2, 1, 0}, C2[3] = {3, 2, 1};
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    B[r] = G.kb1[r] * du[C1[r]] + G.kb2[r] * du[C2[r]];
    C[r] = G.kc1[r] * du[C1[r]] + G.kc2[r] * du[C2[r]];
  }
}

// One sweep of the dimension-by-dimension reconstruction on a 5-cell stencil
// along one direction: indicators of eq. (2.10) summed over (eta, hu, hv),
// the detector class, the hybrid weights at the 4 Gauss-Lobatto points
// shared by every variable; values of h, hu, hv, b (and of an extra variable
// with EXT) at the points, and b's derivative along the sweep: the 5-cell
// quartic's where the class is smooth, the stencil slopes weighted by the
// WENO-Z weights where it is not, blended by M(gamma) in the transition class
// (as in 1D).
template <bool EXT>
__device__ __forceinline__ int sweep(const Geo& G, double eps, const double* e5, const double* m5,
                                     const double* n5, const double* h5, const double* b5,
                                     const double* x5, double (&oh)[4], double (&om)[4],
                                     double (&on)[4], double (&ob)[4], double (&od)[4],
                                     double (&ox)[4]) {
  double beta[3];
  {
    double Be[3], Ce[3];
    stencil_bc(G, e5, Be, Ce);
#pragma unroll
    for (int r = 0; r < 3; ++r) beta[r] = G.kap * (Be[r] * Be[r]) + G.kapC * (Ce[r] * Ce[r]);
  }
  double Bm[3], Cm[3], Bn[3], Cn[3], Bh[3], Ch[3], Bb[3], Cb[3], Bx[3], Cx[3];
  stencil_bc(G, m5, Bm, Cm);
  stencil_bc(G, n5, Bn, Cn);
#pragma unroll
  for (int r = 0; r < 3; ++r)
    beta[r] = (beta[r] + (G.kap * (Bm[r] * Bm[r]) + G.kapC * (Cm[r] * Cm[r]))) +
              (G.kap * (Bn[r] * Bn[r]) + G.kapC * (Cn[r] * Cn[r]));
  stencil_bc(G, h5, Bh, Ch);
  stencil_bc(G, b5, Bb, Cb);
  if (EXT) stencil_bc(G, x5, Bx, Cx);
  const double tau = fabs(beta[0] - beta[2]);
  const double betaA = (beta[0] + beta[1] + beta[2]) * (1.0 / 3.0);
  const double gam = tau * frcp(betaA + eps);
  const int cls = (gam <= 0.5) ? 0 : ((gam >= 1.0) ? 2 : 1);
  double K[3] = {1.0, 1.0, 1.0};
  if (cls != 0) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double z = tau * frcp(beta[r] + eps);
      K[r] = 1.0 + z * z;
    }
  }
  const double Mg = 2.0 * gam - 1.0;
  const double q = 0.22360679774997896964;  // sqrt(5)/10
  const double yv[4] = {-0.5, -q, q, 0.5};
  const double p2v[4] = {1.0 / 6.0, -1.0 / 30.0, -1.0 / 30.0, 1.0 / 6.0};
  // b's derivative: the quartic's (smooth and transition classes) first, at
  // all 4 points; its geometry is loaded here, not with the rest (registers)
  if (cls != 2) {
    asm volatile("" ::: "memory");
    double qi[4], qb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      qi[i] = G.tq[i * G.tst];
      qb[i] = G.tq[(i + GF_QB - GF_QI) * G.tst];
    }
    const double dB = Bb[0] - Bb[2], dC = Cb[0] - Cb[2];
    const double a3 = qi[0] * dB + qi[1] * dC;
    const double a4 = qi[2] * dB + qi[3] * dC;
    const double a1 = Bb[1] - (a3 * qb[0] + a4 * qb[1]);
    const double a2 = Cb[1] - (a3 * qb[2] + a4 * qb[3]);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const double y = yv[mu];
      od[mu] = (a1 + (2.0 * y) * a2 + (3.0 * y * y) * a3 + (4.0 * y * y * y) * a4) * G.iJ;
    }
  }
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    double ph[3];
    if (cls == 0) {
#pragma unroll
      for (int r = 0; r < 3; ++r) ph[r] = G.d[mu][r];
    } else {
      const double a0 = G.d[mu][0] * K[0], a1 = G.d[mu][1] * K[1], a2 = G.d[mu][2] * K[2];
      const double ia = frcp(a0 + a1 + a2);
      ph[0] = a0 * ia;
      ph[1] = a1 * ia;
      ph[2] = a2 * ia;
      // the WENO-Z weighted slopes of b: the derivative (non-smooth) or its
      // Mg part (transition)
      double sBn = 0.0, sCn = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        sBn += ph[r] * Bb[r];
        sCn += ph[r] * Cb[r];
      }
      const double wN = (sBn + 2.0 * yv[mu] * sCn) * G.iJ;
      od[mu] = cls == 2 ? wN : Mg * wN + (1.0 - Mg) * od[mu];
      if (cls == 1) {
#pragma unroll
        for (int r = 0; r < 3; ++r) ph[r] = Mg * ph[r] + (1.0 - Mg) * G.d[mu][r];
      }
    }
    auto val = [&](const double* B, const double* C, double u2) {
      double sB = 0.0, sC = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        sB += ph[r] * B[r];
        sC += ph[r] * C[r];
      }
      return u2 + (sB * yv[mu] + sC * p2v[mu]);
    };
    oh[mu] = val(Bh, Ch, h5[2]);
    om[mu] = val(Bm, Cm, m5[2]);
    on[mu] = val(Bn, Cn, n5[2]);
    ob[mu] = val(Bb, Cb, b5[2]);
    if (EXT) ox[mu] = val(Bx, Cx, x5[2]);
  }
  return cls;
}

// One sweep of the scheme without well-balancing: (eta, hu, hv) in the local
// characteristic variables of the sweep direction (DIR 0: x, 1: y), from the
// eigenvectors of that direction's flux Jacobian at the mean state (hb, mxb,
// myb): eigenvalues u_n -+ c, u_n, right eigenvectors (1, u_n - c, u_t),
// (0, 0, 1), (1, u_n + c, u_t) in (eta, m_n, m_t); the identity where hb <=
// dry.  Each characteristic variable and b are swept as scalars with their
// own indicators, class and weights (sweep on one variable); b's derivative
// and (EXT) the extra lines take b's weights.  Outputs as sweep's (h = eta -
// b); returns the largest of the four classes.
template <int DIR, bool EXT>
__device__ __forceinline__ int sweep_char(const Geo& G, double eps, double g, double dry,
                                          double hb, double mxb, double myb, const double* e5,
                                          const double* m5, const double* n5, const double* b5,
                                          const double* x5, double (&oh)[4], double (&om)[4],
                                          double (&on)[4], double (&ob)[4], double (&od)[4],
                                          double (&ox)[4]) {
  const bool chr = hb > dry;
  double un = 0.0, ut = 0.0, c = 0.0, i2c = 0.0;
  if (chr) {
    const double ih = frcp(hb);
    un = (DIR == 0 ? mxb : myb) * ih;
    ut = (DIR == 0 ? myb : mxb) * ih;
    c = fsqrt(g * hb);
    i2c = 0.5 * frcp(c);
  }
  double w0[5], w1[5], w2[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double mn = DIR == 0 ? m5[k] : n5[k], mt = DIR == 0 ? n5[k] : m5[k];
    if (chr) {
      w0[k] = ((un + c) * e5[k] - mn) * i2c;
      w1[k] = mt - ut * e5[k];
      w2[k] = ((c - un) * e5[k] + mn) * i2c;
    } else {
      w0[k] = e5[k];
      w1[k] = mt;
      w2[k] = mn;
    }
  }
  const double z5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double a0[4], a1[4], a2[4], t[4], u[4];
  int cl = sweep<false>(G, eps, w0, z5, z5, w0, w0, nullptr, a0, t, t, t, u, u);
  cl = max(cl, sweep<false>(G, eps, w1, z5, z5, w1, w1, nullptr, a1, t, t, t, u, u));
  cl = max(cl, sweep<false>(G, eps, w2, z5, z5, w2, w2, nullptr, a2, t, t, t, u, u));
  cl = max(cl, sweep<EXT>(G, eps, b5, z5, z5, b5, b5, x5, t, u, u, ob, od, ox));
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    double e, mn, mt;
    if (chr) {
      e = a0[mu] + a2[mu];
      mn = (un - c) * a0[mu] + (un + c) * a2[mu];
      mt = ut * a0[mu] + a1[mu] + ut * a2[mu];
    } else {
      e = a0[mu];
      mt = a1[mu];
      mn = a2[mu];
    }
    oh[mu] = e - ob[mu];
    om[mu] = DIR == 0 ? mn : mt;
    on[mu] = DIR == 0 ? mt : mn;
  }
  return cl;
}

// Lax-Friedrichs flux of eq. (3.13) for F.n - (w.n) q at one edge point,
// split as C + alpha D (D = -jump / 2), the bottom's ALE flux of eq. (3.17)
// likewise, the edge terms B1 = (b- + b+)/2 and B2 = (b-^2 + b+^2)/2 of the
// special source, weighted by wt; amax takes both traces' speeds
// |u.n - w.n| + sqrt(g h).  Traces with h <= dry carry zero discharge.
// HYD: the hydrostatic reconstruction (eq. (4.4)-(4.6)): the momentum fluxes
// of the starred states (h* = max(0, eta - max(b-, b+)), discharges kept),
// and the pressure corrections g/2 (h^2 - h*^2) of the side a (left / below:
// PL) and c (PR); the eta component of the starred flux plus theta is the
// plain one exactly, so C, D of eta are the plain ones; no B1, B2.
template <int DIR, bool HYD = false>
__device__ __forceinline__ void lf_point(double g, double dry, double w, double wt, double ah,
                                         double am, double an, double ab, double ch, double cm,
                                         double cn, double cb, double (&C)[4], double (&D)[4],
                                         double& B1, double& B2, double& amax, double& PL,
                                         double& PR) {
  if (!(ah > dry)) { am = 0.0; an = 0.0; }
  if (!(ch > dry)) { cm = 0.0; cn = 0.0; }
  double ua = 0.0, va = 0.0, uc = 0.0, vc = 0.0;
  if (ah > dry) { const double r = frcp(ah); ua = am * r; va = an * r; }
  if (ch > dry) { const double r = frcp(ch); uc = cm * r; vc = cn * r; }
  const double ea = ah + ab, ec = ch + cb;
  // depths and velocities of the momentum fluxes
  double pa = ah, pc = ch, usa = ua, vsa = va, usc = uc, vsc = vc;
  if (HYD) {
    const double bm = fmax(ab, cb);
    pa = fmax(0.0, ea - bm);
    pc = fmax(0.0, ec - bm);
    usa = 0.0; vsa = 0.0; usc = 0.0; vsc = 0.0;
    if (pa > dry) { const double r = frcp(pa); usa = am * r; vsa = an * r; }
    if (pc > dry) { const double r = frcp(pc); usc = cm * r; vsc = cn * r; }
    PL += wt * (0.5 * g * (ah * ah - pa * pa));
    PR += wt * (0.5 * g * (ch * ch - pc * pc));
  }
  double Ha[3], Hc[3];
  if (DIR == 0) {
    Ha[0] = am - w * ea; Ha[1] = am * usa + 0.5 * g * pa * pa - w * am; Ha[2] = am * vsa - w * an;
    Hc[0] = cm - w * ec; Hc[1] = cm * usc + 0.5 * g * pc * pc - w * cm; Hc[2] = cm * vsc - w * cn;
  } else {
    Ha[0] = an - w * ea; Ha[1] = an * usa - w * am; Ha[2] = an * vsa + 0.5 * g * pa * pa - w * an;
    Hc[0] = cn - w * ec; Hc[1] = cn * usc - w * cm; Hc[2] = cn * vsc + 0.5 * g * pc * pc - w * cn;
  }
  const double jump[3] = {ec - ea, cm - am, cn - an};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    C[q] += wt * (0.5 * (Ha[q] + Hc[q]));
    D[q] += wt * (-0.5 * jump[q]);
  }
  C[3] += wt * (-0.5 * w * (ab + cb));
  D[3] += wt * (-0.5 * (cb - ab));
  if (!HYD) {
    B1 += wt * (0.5 * (ab + cb));
    B2 += wt * (0.5 * (ab * ab + cb * cb));
  }
  const double una = DIR == 0 ? ua : va, unc = DIR == 0 ? uc : vc;
  const double sa = fabs(una - w) + fsqrt(g * fmax(ah, 0.0));
  const double sc = fabs(unc - w) + fsqrt(g * fmax(ch, 0.0));
  amax = fmax(amax, fmax(sa, sc));
}

// Value of lane (l & ~3) + perm[l & 3] within each quad of lanes (DPP quad_perm;
// CTRL = perm0 | perm1 << 2 | perm2 << 4 | perm3 << 6): 0xB1 swaps neighbours,
// 0x4E swaps pairs.
template <int CTRL>
__device__ __forceinline__ double quad_perm(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// sum over a quad, the same bits in its four lanes ((a + b) + (c + d) with the
// pair sums commuted)
__device__ __forceinline__ double quad_sum(double v) {
  v += quad_perm<0xB1>(v);
  return v + quad_perm<0x4E>(v);
}
__device__ __forceinline__ double quad_min(double v) {
  v = fmin(v, quad_perm<0xB1>(v));
  return fmin(v, quad_perm<0x4E>(v));
}
__device__ __forceinline__ int quad_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false));
  return max(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false));
}

// Positivity limiter across one direction of a rectangle (eq. (3.21)-(3.22)
// split by direction): Phi from the cell mean depth hbar, the Gauss-Lobatto
// quadratures q0, q1 of the depth along the cell's two edges across that
// direction and the smallest edge value mn; delta, the mean of the interior
// lines, follows from hbar = s1 q0 + s1 q1 + (1 - 2 s1) delta.  Phi = 1 where
// min(mn, delta) >= eps = min(1e-11, hbar); 0 where hbar <= 0.
__device__ __forceinline__ double limiter_phi(double hbar, double q0, double q1, double mn) {
  if (!(hbar > 0.0)) return 0.0;
  const double s1 = GLW[0];
  const double delta = (hbar - s1 * q0 - s1 * q1) * (1.0 / (1.0 - 2.0 * s1));
  mn = fmin(mn, delta);
  const double epsj = fmin(1e-11, hbar);
  if (!(mn < epsj)) return 1.0;
  return fmin(1.0, (hbar - epsj) * frcp(hbar - mn));
}
// A trace moved towards the cell means by Phi; b follows eta (Remark 4.1), or
// (KEEPB: the scheme without well-balancing) keeps its value.
template <bool KEEPB = false>
__device__ __forceinline__ void limit_trace(double Phi, double hbar, double mbar, double nbar,
                                            double& h, double& m, double& n, double& b) {
  if (Phi == 1.0) return;
  const double eta = h + b;
  h = Phi * (h - hbar) + hbar;
  m = Phi * (m - mbar) + mbar;
  n = Phi * (n - nbar) + nbar;
  if (!KEEPB) b = eta - h;
}

// ----------------------------------------------------------------------------
// kernels
// ----------------------------------------------------------------------------
// Step state from the caller's arrays: eta = h + b; work-group maxima of the
// wave speed max(|u|, |v|) + sqrt(g h) for the first step size.  Grid:
// (ceil(nx / 256), ny), as the step epilogue's.
__global__ void __launch_bounds__(256) k2_prep(K2 k, const double* __restrict__ h,
                                               const double* __restrict__ hu,
                                               const double* __restrict__ hv,
                                               const double* __restrict__ b) {
  const int i = (int)blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  double s = 0.0;
  if (i < k.nx) {
    const int64_t c = i + (int64_t)k.nx * j;
    const double bb = b[c], m = hu[c], n = hv[c], e = h[c] + bb;
    const double hh = e - bb;
    k.qa[c] = e;
    k.qa[k.N + c] = m;
    k.qa[2 * k.N + c] = n;
    k.qa[3 * k.N + c] = bb;
    double u = 0.0, v = 0.0;
    if (hh > k.dry) { u = m / hh; v = n / hh; }
    s = fmax(fabs(u), fabs(v)) + fsqrt(k.g * fmax(hh, 0.0));
  }
  __shared__ double red[4];
  double v1[1] = {s};
  const int op[1] = {0};
  block_reduce<256, 1>(v1, op, red);
  if (threadIdx.x == 0) k.spart[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = v1[0];
}

// Sums over row j of area x eta and area x b (one work-group per row, fixed
// order), for the conservation diagnostics.
__global__ void __launch_bounds__(256) k2_mass_rows(K2 k) {
  const int j = blockIdx.x;
  const double dy = k.y[j + 1] - k.y[j];
  double me = 0.0, mb = 0.0;
  for (int i = threadIdx.x; i < k.nx; i += 256) {
    const int64_t c = i + (int64_t)k.nx * j;
    const double A = (k.x[i + 1] - k.x[i]) * dy;
    me += A * k.qa[c];
    mb += A * k.qa[3 * k.N + c];
  }
  __shared__ double red[8];
  double v[2] = {me, mb};
  const int op[2] = {2, 2};
  block_reduce<256, 2>(v, op, red);
  if (threadIdx.x == 0) {
    k.part[j] = v[0];
    k.part[k.ny + j] = v[1];
  }
}

__global__ void __launch_bounds__(256) k2_mass_sum(K2 k, double* __restrict__ out) {
  double me = 0.0, mb = 0.0;
  for (int j = threadIdx.x; j < k.ny; j += 256) {
    me += k.part[j];
    mb += k.part[k.ny + j];
  }
  __shared__ double red[8];
  double v[2] = {me, mb};
  const int op[2] = {2, 2};
  block_reduce<256, 2>(v, op, red);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    out[1] = v[1];
  }
}

// Step kinematics (one work-group): stop test, step size
// dt = CFL / ((s + Wx) / min dx + (s + Wy) / min dy) (the CFL condition
// eq. (3.19) sums over the cell's four edges), s the larger of the means'
// max(|u|, |v|) + sqrt(g h) and the previous step's Lax-Friedrichs alpha
// (eq. (3.13), taken on the traces; zero at a run's first step), Wx, Wy the
// largest node speeds of each direction; node speeds (the chords of the
// prescribed maps over [t, t + dt]), widths and their increments, stage
// Dx / Dy of the indicators, the geometry tables of the three stage meshes,
// and the nodes of t + dt.
__global__ void __launch_bounds__(KB) k2_kin(K2 k) {
  State2& S = *k.st;
  __shared__ int s_go;
  __shared__ double s_dt, s_t;
  __shared__ double red[5 * (KB / 64)];
  const int tid = threadIdx.x;
  if (tid == 0) {
    bool stop = S.status != 0 || S.done != 0;
    if (!stop && S.max_steps > 0 && S.steps >= S.max_steps) stop = true;
    if (!stop && S.timed && !(S.t < S.t_end)) stop = true;
    if (!stop && !S.timed && S.max_steps <= 0) stop = true;
    if (stop) S.done = 1;
    s_go = stop ? 0 : 1;
    s_t = S.t;
  }
  __syncthreads();
  if (!s_go) return;
  const int nx = k.nx, ny = k.ny;
  const double t = s_t;
  const double TP = 2.0 * M_PI;
  double dxmin = INFINITY, dymin = INFINITY, Wx = 0.0, Wy = 0.0, smax = 0.0;
  for (int64_t e = tid; e < k.nspart; e += KB) smax = fmax(smax, k.spart[e]);
  for (int i = tid; i < nx; i += KB) dxmin = fmin(dxmin, k.x[i + 1] - k.x[i]);
  for (int j = tid; j < ny; j += KB) dymin = fmin(dymin, k.y[j + 1] - k.y[j]);
  const double cx = k.Ax * k.omx * cos(k.omx * t), cy = k.Ay * k.omy * cos(k.omy * t);
  for (int i = tid; i <= nx; i += KB) Wx = fmax(Wx, fabs(k.Vx + cx * sin(TP * k.kx * k.xi[i])));
  for (int j = tid; j <= ny; j += KB) Wy = fmax(Wy, fabs(k.Vy + cy * sin(TP * k.ky * k.yi[j])));
  {
    double v[5] = {dxmin, dymin, Wx, Wy, smax};
    const int op[5] = {1, 1, 0, 0, 0};
    block_reduce<KB, 5>(v, op, red);
    dxmin = v[0];
    dymin = v[1];
    Wx = v[2];
    Wy = v[3];
    smax = v[4];
  }
  if (tid == 0) {
    // the previous step's alpha of its three stages (bits of non-negative
    // doubles; zeroed when a run starts)
    for (int s = 0; s < 3; ++s) smax = fmax(smax, bitsd(S.alpha[s]));
    double dt = k.cfl / ((smax + Wx) / dxmin + (smax + Wy) / dymin);
    if (S.timed && t + dt > S.t_end) dt = S.t_end - t;
    s_dt = dt;
    S.dt = dt;
    S.dt_min = fmin(S.dt_min, dt);
    S.dt_max = fmax(S.dt_max, dt);
    S.alpha[0] = S.alpha[1] = S.alpha[2] = 0ull;
  }
  __syncthreads();
  const double dt = s_dt;
  // chord of the map's time factor over [t, t + dt]
  const double fx = 2.0 * cos(k.omx * (t + 0.5 * dt)) * sin(0.5 * k.omx * dt) / dt;
  const double fy = 2.0 * cos(k.omy * (t + 0.5 * dt)) * sin(0.5 * k.omy * dt) / dt;
  for (int i = tid; i <= nx; i += KB) k.wx[i] = k.Vx + k.Ax * sin(TP * k.kx * k.xi[i]) * fx;
  for (int j = tid; j <= ny; j += KB) k.wy[j] = k.Vy + k.Ay * sin(TP * k.ky * k.yi[j]) * fy;
  __syncthreads();
  if (tid == 0) {
    if (k.bcx == BC_PERIODIC) k.wx[nx] = k.wx[0];
    if (k.bcy == BC_PERIODIC) k.wy[ny] = k.wy[0];
  }
  __syncthreads();
  for (int i = tid; i < nx; i += KB) {
    k.dx0[i] = k.x[i + 1] - k.x[i];
    k.dwx[i] = k.wx[i + 1] - k.wx[i];
  }
  for (int j = tid; j < ny; j += KB) {
    k.dy0[j] = k.y[j + 1] - k.y[j];
    k.dwy[j] = k.wy[j + 1] - k.wy[j];
  }
  __syncthreads();
  // largest width of each stage mesh per direction (Dx of the indicators)
  double mx[3] = {0.0, 0.0, 0.0}, my[3] = {0.0, 0.0, 0.0};
  for (int i = tid; i < nx; i += KB)
#pragma unroll
    for (int s = 0; s < 3; ++s) mx[s] = fmax(mx[s], k.dx0[i] + TAU(s, dt) * k.dwx[i]);
  for (int j = tid; j < ny; j += KB)
#pragma unroll
    for (int s = 0; s < 3; ++s) my[s] = fmax(my[s], k.dy0[j] + TAU(s, dt) * k.dwy[j]);
  {
    double v[3] = {mx[0], mx[1], mx[2]};
    const int op[3] = {0, 0, 0};
    block_reduce<KB, 3>(v, op, red);
    mx[0] = v[0]; mx[1] = v[1]; mx[2] = v[2];
    double u[3] = {my[0], my[1], my[2]};
    block_reduce<KB, 3>(u, op, red);
    my[0] = u[0]; my[1] = u[1]; my[2] = u[2];
  }
  if (tid == 0)
    for (int s = 0; s < 3; ++s) {
      S.Dx[s] = mx[s];
      S.Dy[s] = my[s];
    }
  // geometry of every column -1..nx and row -1..ny at each stage mesh
  const int ex = nx + 2, ey = ny + 2;
  for (int e = tid; e < 3 * (ex + ey); e += KB) {
    const bool isx = e < 3 * ex;
    const int ee = isx ? e : e - 3 * ex;
    const int ne = isx ? ex : ey;
    const int s = ee / ne, a = ee % ne - 1;
    const int n = isx ? nx : ny, bc = isx ? k.bcx : k.bcy;
    const double* w0 = isx ? k.dx0 : k.dy0;
    const double* dw = isx ? k.dwx : k.dwy;
    double J5[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const int m = wrapi(bc, n, a - 2 + q);
      J5[q] = w0[m] + TAU(s, dt) * dw[m];
    }
    const double iJ = 1.0 / J5[2];
    CellGeom G;
    cell_geom(J5, iJ, isx ? mx[s] : my[s], G);
    // a negative linear weight (Sec. 2.2, after Step 4) is not split in 2D: the
    // run reports it after this step
    if (G.sgn >> 31) atomicOr(&k.st->status, SB_NEGWEIGHT);
    double* T = isx ? k.Gx : k.Gy;
    auto put = [&](int fld, double v) { T[((int64_t)fld * 3 + s) * ne + (a + 1)] = v; };
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      put(GF_KB1 + r, G.kb1[r]);
      put(GF_KB2 + r, G.kb2[r]);
      put(GF_KC1 + r, G.kc1[r]);
      put(GF_KC2 + r, G.kc2[r]);
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
      for (int r = 0; r < 3; ++r) put(GF_D + mu * 3 + r, G.d[mu][r]);
    put(GF_KAP, G.kap);
    put(GF_KAPC, G.kapC);
    put(GF_IJ, iJ);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      put(GF_QI + i, G.qi[i]);
      put(GF_QB + i, G.qb[i]);
    }
  }
  // nodes of t + dt (every read of the old nodes is behind the barriers above)
  for (int i = tid; i <= nx; i += KB) k.x[i] = k.x[i] + dt * k.wx[i];
  for (int j = tid; j <= ny; j += KB) k.y[j] = k.y[j] + dt * k.wy[j];
  if (tid == 0) {
    S.t = t + dt;
    S.steps = S.steps + 1;
  }
}

// x-sweep of stage S: a work-group of XB threads outputs the line values of
// columns i0 .. i0 + XB - 1 (i0 = blockIdx.x XB - 1, columns -1..nx) of row
// blockIdx.y from the XB + 4 stage states staged in LDS.
template <int S, int SCH>
__global__ void __launch_bounds__(XB) k2_xsweep(K2 k) {
  constexpr bool NWB = SCH == 2;  // characteristic sweeps of the scheme without well-balancing
  const State2& St = *k.st;
  if (St.done) return;
  __shared__ double sv[4][XB + 4];
  const int j = blockIdx.y, tid = threadIdx.x;
  const int i0 = (int)blockIdx.x * XB - 1;
  const int nx = k.nx;
  const double dt = St.dt;
  const double* qprev = (S & 1) ? k.qs0 : k.qs1;  // stage S-1's state
  double* qcur = (S & 1) ? k.qs1 : k.qs0;
  const double dy0 = k.dy0[j], dwy = k.dwy[j];
  const double alpha = S > 0 ? bitsd(St.alpha[S > 0 ? S - 1 : 0]) : 0.0;
  for (int kk = tid; kk < XB + 4; kk += XB) {
    const int ic = i0 - 2 + kk;
    const int iw = wrapi(k.bcx, nx, ic);
    const int64_t c = iw + (int64_t)nx * j;
    double q[4];
    if (S == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) q[v] = k.qa[v * k.N + c];
    } else {
      double Jn;
      stage_update<S>(k, c, k.dx0[iw], k.dwx[iw], dy0, dwy, dt, alpha, qprev, q, Jn);
      if (ic == iw && kk >= 2 && kk < XB + 2 && !(Jn > 0.0)) atomicOr(&k.st->status, SB_MESH);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sv[v][kk] = q[v];
    if (ic == iw && kk >= 2 && kk < XB + 2)
#pragma unroll
      for (int v = 0; v < 4; ++v) qcur[v * k.N + c] = q[v];
  }
  __syncthreads();
  const int i = i0 + tid;
  if (i > nx) return;
  double e5[5], m5[5], n5[5], b5[5], h5[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    e5[q] = sv[0][tid + q];
    m5[q] = sv[1][tid + q];
    n5[q] = sv[2][tid + q];
    b5[q] = sv[3][tid + q];
    h5[q] = e5[q] - b5[q];
  }
  Geo G;
  load_geo(k.Gx, nx + 2, S, i + 1, G);
  double oh[4], om[4], on[4], ob[4], od[4], ox[4];
  int cls;
  if (NWB)
    cls = sweep_char<0, false>(G, k.eps, k.g, k.dry, h5[2], m5[2], n5[2], e5, m5, n5, b5, nullptr,
                               oh, om, on, ob, od, ox);
  else
    cls = sweep<false>(G, k.eps, e5, m5, n5, h5, b5, nullptr, oh, om, on, ob, od, ox);
  const uint32_t o = (uint32_t)j * (uint32_t)k.LW + (uint32_t)(i + 1);
  double* __restrict__ Lh = k.L;
  double* __restrict__ Lm = k.L + k.PL4;
  double* __restrict__ Ln = k.L + 2 * k.PL4;
  double* __restrict__ Lb = k.L + 3 * k.PL4;
  double* __restrict__ Lx = k.L + 4 * k.PL4;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    Lh[o * 4u + mu] = oh[mu];
    Lm[o * 4u + mu] = om[mu];
    Ln[o * 4u + mu] = on[mu];
    Lb[o * 4u + mu] = ob[mu];
    Lx[o * 4u + mu] = od[mu];
  }
  k.xcls[o] = (uint8_t)cls;
}

// y-sweep of stage S: a work-group of 256 threads marches up rows j0-1 .. j1
// of its strip of 64 columns (column 62 blockIdx.x + slot - 1; slots 0 and 63
// are the strip's ring columns), four threads per column: thread q of a
// column reconstructs along y at abscissa q, evaluates the bottom edge at
// point q (against the top trace it kept from the row below) and the left
// edge at point q (against the left neighbour's right traces, through LDS);
// the column's four threads then sum the edge points and the source terms by
// quad shuffles, and thread q writes component q of the right-hand side.
// Rows j0-1 and j1 give only the traces of the edges below row j0 and above
// row j1 - 1.
template <int S, int SCH>
__global__ void __launch_bounds__(256) k2_ysweep(K2 k, int rows) {
  // SCH 0: special source term; 1: hydrostatic reconstruction; 2: without
  // well-balancing (characteristic sweeps, -g h grad b, b kept by the limiter)
  constexpr bool HYD = SCH == 1, NWB = SCH == 2;
  const State2& St = *k.st;
  if (St.done) return;
  __shared__ double sL[64][4][4];  // left traces of each column at point nu: h, hu, hv, b
  __shared__ double sR[64][4][4];  // right traces
  __shared__ double sF[64][12];    // left-edge sums of each column: C[4], D[4], B1, B2
  const int t = threadIdx.x, cs = t >> 2, q = t & 3;
  const int nx = k.nx, ny = k.ny;
  const int i = STRIP * (int)blockIdx.x + cs - 1;
  const int j0 = (int)blockIdx.y * rows, j1 = min(j0 + rows, ny);
  const bool own_col = cs >= 1 && cs <= STRIP && i >= 0 && i < nx;
  const bool xedge = cs >= 1 && i >= 0 && i <= nx;  // this column's left edge exists
  const bool ycol = i >= 0 && i < nx;
  const int ic = min(max(i, -1), nx);               // slots past the ring load a valid column
  const uint32_t lc = (uint32_t)(ic + 1);
  // 32-bit offsets from uniform plane pointers (the context caps the grid at
  // 2^26 cells, so every offset here stays below 2^29 elements)
  const uint32_t lo = lc * 4u + (uint32_t)q, rowL = 4u * (uint32_t)k.LW;
  const double* __restrict__ Lh = k.L;
  const double* __restrict__ Lm = k.L + k.PL4;
  const double* __restrict__ Ln = k.L + 2 * k.PL4;
  const double* __restrict__ Lb = k.L + 3 * k.PL4;
  const double* __restrict__ Lx = k.L + 4 * k.PL4;
  const double dt = St.dt, tau = TAU(S, dt), g = k.g, dry = k.dry;
  const double* qcur = (S & 1) ? k.qs1 : k.qs0;
  const int iw = min(max(i, 0), nx - 1);
  const double dxs = k.dx0[iw] + tau * k.dwx[iw];
  const double wxl = k.wx[min(max(i, 0), nx)];
  const double wq = GLW[q];
  // HYD: row q of the cubic's differentiation matrix at the Gauss-Lobatto
  // points (cell coordinate in [0, 1]; the rows hydro_source applies)
  constexpr double PHI = 1.6180339887498948482, PHI1 = 0.6180339887498948482;
  constexpr double R5 = 2.2360679774997896964;
  const double dq0 = q == 0 ? -6.0 : q == 1 ? -PHI : q == 2 ? PHI1 : -1.0;
  const double dq1 = q == 0 ? 5.0 * PHI : q == 1 ? 0.0 : q == 2 ? -R5 : 5.0 * PHI1;
  const double dq2 = q == 0 ? -5.0 * PHI1 : q == 1 ? R5 : q == 2 ? 0.0 : -5.0 * PHI;
  const double dq3 = q == 0 ? 1.0 : q == 1 ? -PHI1 : q == 2 ? PHI : 6.0;
  double amax = 0.0;
  unsigned ncl[3] = {0u, 0u, 0u}, nlim = 0u;
  bool negd = false;
  double th = 0.0, tm = 0.0, tn = 0.0, tb = 0.0;  // top trace at abscissa q, row below
  double Pc = 0.0, Pd = 0.0;  // component q of the previous row's partial right-hand side
  double etab_p = 0.0;
  for (int jr = j0 - 1; jr <= j1; ++jr) {
    const bool first = jr == j0 - 1, last = jr == j1;
    const bool body = !first && !last;
    Geo G;
    load_geo(k.Gy, ny + 2, S, jr + 1, G);
    const int jw = wrapi(k.bcy, ny, jr);
    const double dys = k.dy0[jw] + tau * k.dwy[jw];
    const double wyb = k.wy[min(max(jr, 0), ny)];
    const uint32_t c = (uint32_t)(ycol ? i : 0) + (uint32_t)nx * (uint32_t)jw;
    const double etab = body && ycol ? qcur[c] : 0.0;
    // means of the cell (ring and ghost cells: their source cells) for the limiter
    const uint32_t cm = (uint32_t)wrapi(k.bcx, nx, ic) + (uint32_t)nx * (uint32_t)jw;
    const double hbar = qcur[cm] - qcur[3 * (uint32_t)k.N + cm];
    const double mbar = qcur[(uint32_t)k.N + cm], nbar = qcur[2 * (uint32_t)k.N + cm];
    // reconstruction along y at abscissa q: point values at nu = 0..3
    double oh[4], om[4], on[4], ob[4], od[4], ox[4];
    int cl;
    {
      double h5[5], m5[5], n5[5], b5[5], x5[5], e5[5];
#pragma unroll
      for (int r = 0; r < 5; ++r) {
        const uint32_t o = (uint32_t)wrapi(k.bcy, ny, jr - 2 + r) * rowL + lo;
        h5[r] = Lh[o];
        m5[r] = Lm[o];
        n5[r] = Ln[o];
        b5[r] = Lb[o];
        x5[r] = Lx[o];
        e5[r] = h5[r] + b5[r];
      }
      if (NWB)
        cl = sweep_char<1, true>(G, k.eps, g, dry, hbar, mbar, nbar, e5, m5, n5, b5, x5, oh, om,
                                 on, ob, od, ox);
      else
        cl = sweep<true>(G, k.eps, e5, m5, n5, h5, b5, x5, oh, om, on, ob, od, ox);
    }
    double ix = 0.0, iy = 0.0;
    if (body && HYD) {
      // the line sources of the hydrostatic reconstruction (the 1D source on
      // every Gauss-Lobatto line) from the unlimited values: this lane's part
      // of each x-line (point nu; b of the line from the quad's four lanes),
      // and its own y-line's, each with its abscissa's weight
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) {
        const double d = dq0 * quad_perm<0x00>(ob[nu]) + dq1 * quad_perm<0x55>(ob[nu]) +
                         dq2 * quad_perm<0xAA>(ob[nu]) + dq3 * quad_perm<0xFF>(ob[nu]);
        ix += GLW[nu] * (oh[nu] * d);
      }
      ix *= wq;
      iy = wq * hydro_source(g, oh[0] + ob[0], oh[1] + ob[1], oh[2] + ob[2], oh[3] + ob[3], ob[0],
                             ob[1], ob[2], ob[3]);
    } else if (body && NWB) {
      // -g h grad b at the 4 points of this abscissa (the unlimited values)
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) {
        ix += (wq * GLW[nu]) * (oh[nu] * ox[nu]);
        iy += (wq * GLW[nu]) * (oh[nu] * od[nu]);
      }
    } else if (body) {
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) {
        const double e = oh[nu] + ob[nu];
        ix += (wq * GLW[nu]) * ((e - etab) * ox[nu]);
        iy += (wq * GLW[nu]) * ((e - etab) * od[nu]);
      }
    }
    // positivity limiter, per direction (the source above keeps the unlimited
    // values): across x on the left and right edges (threads 0 and 3 hold
    // them), across y on the bottom and top edges (point q of each here);
    // both factors from the unlimited values
    double p1, p2;
    {
      const double qb = quad_sum(wq * oh[0]), qt = quad_sum(wq * oh[3]);
      p1 = limiter_phi(hbar, qb, qt, quad_min(fmin(oh[0], oh[3])));
      double ql = 0.0, mnl = oh[0];
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) {
        ql += GLW[nu] * oh[nu];
        mnl = fmin(mnl, oh[nu]);
      }
      const double q0 = quad_perm<0x00>(ql), q3 = quad_perm<0xFF>(ql);
      const double m0 = quad_perm<0x00>(mnl), m3 = quad_perm<0xFF>(mnl);
      p2 = limiter_phi(hbar, q0, q3, fmin(m0, m3));
    }
    const bool limited = p1 != 1.0 || p2 != 1.0;
    // the left / right edge traces (corners included) limited across x
    if (q == 0 || q == 3) {
      double (*dst)[4] = q == 0 ? sL[cs] : sR[cs];
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) {
        double hh = oh[nu], mm = om[nu], nn = on[nu], bb = ob[nu];
        limit_trace<NWB>(p2, hbar, mbar, nbar, hh, mm, nn, bb);
        dst[nu][0] = hh; dst[nu][1] = mm; dst[nu][2] = nn; dst[nu][3] = bb;
      }
    }
    // the bottom / top traces at point q limited across y
    limit_trace<NWB>(p1, hbar, mbar, nbar, oh[0], om[0], on[0], ob[0]);
    limit_trace<NWB>(p1, hbar, mbar, nbar, oh[3], om[3], on[3], ob[3]);
    // bottom edge (node jr) at point q: the cell below's top trace
    double Cy[4] = {0, 0, 0, 0}, Dy[4] = {0, 0, 0, 0}, B1y = 0.0, B2y = 0.0;
    double PLy = 0.0, PRy = 0.0;  // HYD: pressure corrections below / above the edge
    if (!first) {
      double am = 0.0;
      lf_point<1, HYD>(g, dry, wyb, wq, th, tm, tn, tb, oh[0], om[0], on[0], ob[0], Cy, Dy, B1y,
                       B2y, am, PLy, PRy);
      if (ycol) amax = fmax(amax, am);
    }
    th = oh[3]; tm = om[3]; tn = on[3]; tb = ob[3];
    __syncthreads();
    // left edge (node i) at point q: the left neighbour's right trace
    double Cx[4] = {0, 0, 0, 0}, Dx[4] = {0, 0, 0, 0}, B1x = 0.0, B2x = 0.0;
    double PLx = 0.0, PRx = 0.0;  // HYD: pressure corrections left / right of the edge
    if (body && cs >= 1) {
      double am = 0.0;
      lf_point<0, HYD>(g, dry, wxl, wq, sR[cs - 1][q][0], sR[cs - 1][q][1], sR[cs - 1][q][2],
                       sR[cs - 1][q][3], sL[cs][q][0], sL[cs][q][1], sL[cs][q][2], sL[cs][q][3],
                       Cx, Dx, B1x, B2x, am, PLx, PRx);
      if (xedge) amax = fmax(amax, am);
    }
    // sums over the column's four points (every thread of the quad gets them)
    auto qsum = [](double v) { return quad_sum(v); };
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Cy[r] = qsum(Cy[r]) * dxs; Dy[r] = qsum(Dy[r]) * dxs;
      Cx[r] = qsum(Cx[r]) * dys; Dx[r] = qsum(Dx[r]) * dys;
    }
    if (HYD) {
      PLy = qsum(PLy) * dxs; PRy = qsum(PRy) * dxs;
      PLx = qsum(PLx) * dys; PRx = qsum(PRx) * dys;
    } else {
      B1y = qsum(B1y) * dxs; B2y = qsum(B2y) * dxs;
      B1x = qsum(B1x) * dys; B2x = qsum(B2x) * dys;
    }
    ix = qsum(ix);
    iy = qsum(iy);
    const int ymax = quad_max(cl);
    // publish the left-edge sums: the right edge of the column to the left
    {
      const double fv[12] = {Cx[0], Cx[1], Cx[2], Cx[3], Dx[0], Dx[1], Dx[2], Dx[3], B1x, B2x,
                             PLx, 0.0};
#pragma unroll
      for (int r = 0; r < 3; ++r) sF[cs][q + 4 * r] = fv[q + 4 * r];
    }
    __syncthreads();
    const int cn = min(cs + 1, 63);
    // component q of: C, D of the bottom (this row) edge, and the right edge
    const double Cyq = q == 0 ? Cy[0] : q == 1 ? Cy[1] : q == 2 ? Cy[2] : Cy[3];
    const double Dyq = q == 0 ? Dy[0] : q == 1 ? Dy[1] : q == 2 ? Dy[2] : Dy[3];
    const double Cxq = q == 0 ? Cx[0] : q == 1 ? Cx[1] : q == 2 ? Cx[2] : Cx[3];
    const double Dxq = q == 0 ? Dx[0] : q == 1 ? Dx[1] : q == 2 ? Dx[2] : Dx[3];
    const double Crq = sF[cn][q], Drq = sF[cn][4 + q];
    const double B1r = sF[cn][8], B2r = sF[cn][9];
    const double PLr = sF[cn][10];  // HYD: this cell's correction on its right edge
    if (!first) {
      // the previous row is complete: its top edge is this row's bottom edge
      const int jp = jr - 1;
      if (own_col && jp >= j0) {
        const uint32_t cp = (uint32_t)q * (uint32_t)k.N + (uint32_t)i + (uint32_t)nx * (uint32_t)jp;
        double rc = Pc - Cyq;
        if (q == 2 && !NWB) rc += HYD ? -PLy : 0.5 * g * B2y - g * etab_p * B1y;
        k.Rc[cp] = rc;
        k.Rd[cp] = Pd - Dyq;
      }
    }
    if (body) {
      const double area = dxs * dys;
      Pc = -(Crq - Cxq) + Cyq;
      if (HYD) {
        if (q == 1) Pc += (PRx - PLr) - g * dys * ix;
        if (q == 2) Pc += PRy + dxs * iy;
      } else if (NWB) {
        if (q == 1) Pc += -g * area * ix;
        if (q == 2) Pc += -g * area * iy;
      } else {
        if (q == 1) Pc += 0.5 * g * (B2r - B2x) - g * etab * (B1r - B1x) - g * area * ix;
        if (q == 2) Pc += -0.5 * g * B2y + g * etab * B1y - g * area * iy;
      }
      Pd = -(Drq - Dxq) + Dyq;
      etab_p = etab;
      if (own_col && q == 0) {
        const int cls = max(ymax, (int)k.xcls[(uint32_t)jr * (uint32_t)k.LW + lc]);
        ncl[cls] += 1u;
        if (limited) nlim += 1u;
        if (hbar < -1e-11) negd = true;
        const int64_t cc = i + (int64_t)nx * jr;
        if (k.cls) k.cls[S * k.N + cc] = (uint8_t)cls;
        if (k.ccount) k.ccount[cls * k.N + cc] += 1u;
        if (k.csig) k.csig[cc] = k.csig[cc] * CLS_SIG_MUL + (unsigned long long)(cls + 1);
      }
    }
  }
  // one atomic per wavefront for the stage's speed and the class counts
  amax = wave_max(amax);
  if ((t & 63) == 0) amax_pos(&k.st->alpha[S], amax);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const unsigned n = wave_usum(ncl[r]);
    if ((t & 63) == 0 && n) atomicAdd(&k.st->n_class[r], (unsigned long long)n);
  }
  const unsigned nl = wave_usum(nlim);
  if ((t & 63) == 0 && nl) atomicAdd(&k.st->n_limited, (unsigned long long)nl);
  if (negd) atomicOr(&k.st->status, SB_NEGDEPTH);
}

// Step epilogue: the third stage's update into the step state, the finite
// check and the work-group maxima of the next step's wave speed.  Grid:
// (ceil(nx / 256), ny).
__global__ void __launch_bounds__(256) k2_fin(K2 k) {
  const State2& St = *k.st;
  if (St.done) return;
  const int i = (int)blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  double s = 0.0;
  bool bad = false;
  if (i < k.nx) {
    const int64_t c = i + (int64_t)k.nx * j;
    double q[4], Jn;
    stage_update<3>(k, c, k.dx0[i], k.dwx[i], k.dy0[j], k.dwy[j], St.dt, bitsd(St.alpha[2]), k.qs0,
                    q, Jn);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      k.qa[v * k.N + c] = q[v];
      bad = bad || !isfinite(q[v]);
    }
    const double hh = q[0] - q[3];
    double u = 0.0, v = 0.0;
    if (hh > k.dry) { u = q[1] / hh; v = q[2] / hh; }
    s = fmax(fabs(u), fabs(v)) + fsqrt(k.g * fmax(hh, 0.0));
  }
  if (bad) atomicOr(&k.st->status, SB_NONFINITE);
  __shared__ double red[4];
  double v1[1] = {s};
  const int op[1] = {0};
  block_reduce<256, 1>(v1, op, red);
  if (threadIdx.x == 0) k.spart[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = v1[0];
}

// Caller's arrays from the step state: h = eta - b, hu, hv, b.
__global__ void __launch_bounds__(256) k2_out(K2 k, double* __restrict__ h, double* __restrict__ hu,
                                              double* __restrict__ hv, double* __restrict__ b) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k.N) return;
  const double e = k.qa[c], bb = k.qa[3 * k.N + c];
  h[c] = e - bb;
  hu[c] = k.qa[k.N + c];
  hv[c] = k.qa[2 * k.N + c];
  b[c] = bb;
}

}  // namespace alew2d

// ============================================================================
// host side
// ============================================================================
using namespace alew2d;

struct alew2d_ctx {
  hipStream_t stream = nullptr;
  int64_t max_nx = 0, max_ny = 0;
  double *qa = nullptr, *qs0 = nullptr, *qs1 = nullptr, *L = nullptr, *Rc = nullptr, *Rd = nullptr;
  uint8_t* xcls = nullptr;
  double *dx0 = nullptr, *dwx = nullptr, *dy0 = nullptr, *dwy = nullptr, *wx = nullptr, *wy = nullptr;
  double *Gx = nullptr, *Gy = nullptr, *part = nullptr, *mass = nullptr, *spart = nullptr;
  State2* st = nullptr;
  State2* st_h = nullptr;  // pinned
  double* mass_h = nullptr;  // pinned [4]
  int rows = 16;           // rows per y-sweep wavefront
  int check_every = 8;     // steps between stop checks of a timed run
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
  // per-kernel timing (alew2d_set_kernel_timing): an event pair around every
  // launch of a step, summed per kind after the call
  int ktime_on = 0;
  std::vector<hipEvent_t> kt_ev;
  std::vector<int> kt_kind;
  double kt_ms[4] = {0, 0, 0, 0};
  int64_t kt_n[4] = {0, 0, 0, 0};
};

namespace {

alew_status fail2(alew_status s, const std::string& m) { return alew_set_error(s, m.c_str()); }

#define HIPCHK2(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail2(ALEW_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

alew_status map_bits(int bits) {
  if (bits & SB_MESH) return ALEW_E_MESH;
  if (bits & SB_NEGDEPTH) return ALEW_E_NEGDEPTH;
  if (bits & SB_NONFINITE) return ALEW_E_NONFINITE;
  if (bits & SB_NEGWEIGHT) return ALEW_E_NEGWEIGHT;
  return bits ? ALEW_E_HIP : ALEW_OK;
}

}  // namespace

extern "C" {

alew_status alew2d_create(alew2d_ctx** out, int64_t max_nx, int64_t max_ny, void* hip_stream) {
  if (!out) return fail2(ALEW_E_ARG, "ctx output pointer is NULL");
  *out = nullptr;
  if (max_nx < 5 || max_ny < 5) return fail2(ALEW_E_ARG, "max_nx >= 5 and max_ny >= 5 required");
  if (max_nx > (1 << 24) || max_ny > 65535 || max_nx * max_ny > ((int64_t)1 << 26))
    return fail2(ALEW_E_ARG, "max_nx <= 2^24, max_ny <= 65535 and max_nx * max_ny <= 2^26 required");
  alew2d_ctx* c = new alew2d_ctx();
  c->stream = (hipStream_t)hip_stream;
  c->max_nx = max_nx;
  c->max_ny = max_ny;
  const int64_t N = max_nx * max_ny, PL = (max_nx + 2) * max_ny;
  auto alloc = [&](void** p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; };
  bool ok = alloc((void**)&c->qa, 4 * N * 8) && alloc((void**)&c->qs0, 4 * N * 8) &&
            alloc((void**)&c->qs1, 4 * N * 8) && alloc((void**)&c->L, 20 * PL * 8) &&
            alloc((void**)&c->Rc, 4 * N * 8) && alloc((void**)&c->Rd, 4 * N * 8) &&
            alloc((void**)&c->xcls, PL) && alloc((void**)&c->dx0, max_nx * 8) &&
            alloc((void**)&c->dwx, max_nx * 8) && alloc((void**)&c->dy0, max_ny * 8) &&
            alloc((void**)&c->dwy, max_ny * 8) && alloc((void**)&c->wx, (max_nx + 1) * 8) &&
            alloc((void**)&c->wy, (max_ny + 1) * 8) &&
            alloc((void**)&c->Gx, (size_t)NGF * 3 * (max_nx + 2) * 8) &&
            alloc((void**)&c->Gy, (size_t)NGF * 3 * (max_ny + 2) * 8) &&
            alloc((void**)&c->part, 2 * max_ny * 8) && alloc((void**)&c->mass, 4 * 8) &&
            alloc((void**)&c->spart, ((max_nx + 255) / 256) * max_ny * 8) &&
            alloc((void**)&c->st, sizeof(State2));
  ok = ok && hipHostMalloc((void**)&c->st_h, sizeof(State2), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c->mass_h, 4 * 8, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipEventCreate(&c->ev0) == hipSuccess && hipEventCreate(&c->ev1) == hipSuccess;
  if (!ok) {
    alew2d_destroy(c);
    return fail2(ALEW_E_NOMEM, "device allocation failed");
  }
  *out = c;
  return ALEW_OK;
}

void alew2d_destroy(alew2d_ctx* c) {
  if (!c) return;
  void* ps[] = {c->qa, c->qs0, c->qs1, c->L, c->Rc, c->Rd, c->xcls, c->dx0, c->dwx, c->dy0,
                c->dwy, c->wx, c->wy, c->Gx, c->Gy, c->part, c->mass, c->spart, c->st};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (c->st_h) (void)hipHostFree(c->st_h);
  if (c->mass_h) (void)hipHostFree(c->mass_h);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->kt_ev) (void)hipEventDestroy(e);
  delete c;
}

alew_status alew2d_set_kernel_timing(alew2d_ctx* c, int on) {
  if (!c) return fail2(ALEW_E_ARG, "ctx is NULL");
  c->ktime_on = on ? 1 : 0;
  return ALEW_OK;
}

alew_status alew2d_kernel_timing(const alew2d_ctx* c, int which, double* ms, int64_t* launches) {
  if (!c || !ms || !launches || which < 0 || which > 3)
    return fail2(ALEW_E_ARG, "ctx, which in 0..3 and output pointers required");
  *ms = c->kt_ms[which];
  *launches = c->kt_n[which];
  return ALEW_OK;
}

alew_status alew2d_set_stream(alew2d_ctx* c, void* s) {
  if (!c) return fail2(ALEW_E_ARG, "ctx is NULL");
  c->stream = (hipStream_t)s;
  return ALEW_OK;
}

alew_status alew2d_set_launch(alew2d_ctx* c, int32_t rows, int32_t check_every) {
  if (!c) return fail2(ALEW_E_ARG, "ctx is NULL");
  if (rows < 1 || rows > 4096 || check_every < 1 || check_every > 4096)
    return fail2(ALEW_E_ARG, "rows and check_every must lie in [1, 4096]");
  c->rows = rows;
  c->check_every = check_every;
  return ALEW_OK;
}

alew_status alew2d_last_timing(const alew2d_ctx* c, double* ms) {
  if (!c || !ms) return fail2(ALEW_E_ARG, "NULL argument");
  *ms = c->last_ms;
  return ALEW_OK;
}

alew_status alew2d_run(alew2d_ctx* c, const alew2d_params* p, int64_t nx, int64_t ny, double* h,
                       double* hu, double* hv, double* b, double* x, double* y, const double* xi,
                       const double* yi, double t0, double t_end, int64_t max_steps, uint8_t* cls,
                       uint32_t* cls_count, uint64_t* cls_sig, alew2d_stats* stats) {
  if (!c || !p) return fail2(ALEW_E_ARG, "ctx or params is NULL");
  if (nx < 5 || ny < 5 || nx > c->max_nx || ny > c->max_ny)
    return fail2(ALEW_E_ARG, "need 5 <= nx <= max_nx and 5 <= ny <= max_ny of the context");
  if (!h || !hu || !hv || !b || !x || !y || !xi || !yi)
    return fail2(ALEW_E_ARG, "state, node and reference-node arrays are required");
  if (!(p->g > 0.0) || !(p->cfl > 0.0) || !(p->weno_eps > 0.0) || !(p->dry_eps >= 0.0))
    return fail2(ALEW_E_ARG, "g, cfl, weno_eps > 0 and dry_eps >= 0 required");
  if ((p->bcx != ALEW_BC_PERIODIC && p->bcx != ALEW_BC_TRANSMISSIVE) ||
      (p->bcy != ALEW_BC_PERIODIC && p->bcy != ALEW_BC_TRANSMISSIVE))
    return fail2(ALEW_E_UNSUPPORTED, "2D boundaries: periodic or transmissive");
  if (p->flags & ~(ALEW_F_HYDROSTATIC | ALEW_F_NONWB))
    return fail2(ALEW_E_UNSUPPORTED, "the 2D flags are HYDROSTATIC and NONWB");
  if ((p->flags & ALEW_F_HYDROSTATIC) && (p->flags & ALEW_F_NONWB))
    return fail2(ALEW_E_ARG, "HYDROSTATIC and NONWB select different schemes");
  const int sch = (p->flags & ALEW_F_HYDROSTATIC) ? 1 : (p->flags & ALEW_F_NONWB) ? 2 : 0;
  if (!std::isfinite(p->Vx) || !std::isfinite(p->Vy))
    return fail2(ALEW_E_ARG, "the node translation Vx, Vy must be finite");
  if (!std::isfinite(t0) || std::isnan(t_end) || max_steps < 0)
    return fail2(ALEW_E_ARG, "t0 finite, t_end not NaN and max_steps >= 0 required");
  K2 k{};
  k.g = p->g; k.cfl = p->cfl; k.eps = p->weno_eps; k.dry = p->dry_eps;
  k.Ax = p->Ax; k.kx = p->kx; k.omx = p->omx; k.Ay = p->Ay; k.ky = p->ky; k.omy = p->omy;
  k.Vx = p->Vx; k.Vy = p->Vy;
  k.bcx = p->bcx; k.bcy = p->bcy; k.nx = (int32_t)nx; k.ny = (int32_t)ny;
  k.N = nx * ny; k.LW = nx + 2; k.PL4 = 4 * (nx + 2) * ny;
  k.qa = c->qa; k.qs0 = c->qs0; k.qs1 = c->qs1; k.L = c->L; k.xcls = c->xcls; k.Rc = c->Rc;
  k.Rd = c->Rd; k.dx0 = c->dx0; k.dwx = c->dwx; k.dy0 = c->dy0; k.dwy = c->dwy; k.wx = c->wx;
  k.wy = c->wy; k.Gx = c->Gx; k.Gy = c->Gy; k.x = x; k.y = y; k.xi = xi; k.yi = yi; k.st = c->st;
  k.cls = cls; k.ccount = cls_count; k.csig = (unsigned long long*)cls_sig; k.part = c->part;
  const dim3 gc((unsigned)((nx + 255) / 256), (unsigned)ny);  // per-cell kernels
  k.spart = c->spart;
  k.nspart = (int64_t)gc.x * gc.y;
  const bool timed = t_end > t0;
  State2& S = *c->st_h;
  std::memset(&S, 0, sizeof(S));
  S.t = t0;
  S.t_end = t_end;
  S.dt_min = INFINITY;
  S.dt_max = 0.0;
  S.max_steps = max_steps;
  S.timed = timed ? 1 : 0;
  hipStream_t st = c->stream;
  HIPCHK2(hipMemcpyAsync(c->st, &S, sizeof(S), hipMemcpyHostToDevice, st));
  const int64_t N = k.N;
  const unsigned nb = (unsigned)((N + 255) / 256);
  HIPCHK2(hipEventRecord(c->ev0, st));
  hipLaunchKernelGGL(k2_prep, gc, dim3(256), 0, st, k, h, hu, hv, b);
  hipLaunchKernelGGL(k2_mass_rows, dim3((unsigned)ny), dim3(256), 0, st, k);
  hipLaunchKernelGGL(k2_mass_sum, dim3(1), dim3(256), 0, st, k, c->mass);
  const dim3 gx((unsigned)((nx + 2 + XB - 1) / XB), (unsigned)ny);
  const dim3 gy((unsigned)((nx + STRIP - 1) / STRIP), (unsigned)((ny + c->rows - 1) / c->rows));
  const int rows = c->rows;
  // kernel timing: event pairs (created on first use, reused by later calls)
  size_t kt_used = 0;
  for (int q = 0; q < 4; ++q) { c->kt_ms[q] = 0.0; c->kt_n[q] = 0; }
  c->kt_kind.clear();
  auto mark = [&](int kind, bool begin) -> alew_status {
    if (!c->ktime_on) return ALEW_OK;
    if (kt_used == c->kt_ev.size()) {
      hipEvent_t e;
      HIPCHK2(hipEventCreate(&e));
      c->kt_ev.push_back(e);
    }
    HIPCHK2(hipEventRecord(c->kt_ev[kt_used++], st));
    if (begin) c->kt_kind.push_back(kind);
    return ALEW_OK;
  };
  auto one_step = [&]() -> alew_status {
    alew_status r = ALEW_OK;
    auto timed_launch = [&](int kind, auto&& launch) {
      if (r == ALEW_OK) r = mark(kind, true);
      launch();
      if (r == ALEW_OK) r = mark(kind, false);
    };
    timed_launch(0, [&] { hipLaunchKernelGGL(k2_kin, dim3(1), dim3(KB), 0, st, k); });
    timed_launch(1, [&] {
      if (sch == 2) hipLaunchKernelGGL((k2_xsweep<0, 2>), gx, dim3(XB), 0, st, k);
      else hipLaunchKernelGGL((k2_xsweep<0, 0>), gx, dim3(XB), 0, st, k);
    });
    timed_launch(2, [&] {
      if (sch == 1) hipLaunchKernelGGL((k2_ysweep<0, 1>), gy, dim3(256), 0, st, k, rows);
      else if (sch == 2) hipLaunchKernelGGL((k2_ysweep<0, 2>), gy, dim3(256), 0, st, k, rows);
      else hipLaunchKernelGGL((k2_ysweep<0, 0>), gy, dim3(256), 0, st, k, rows);
    });
    timed_launch(1, [&] {
      if (sch == 2) hipLaunchKernelGGL((k2_xsweep<1, 2>), gx, dim3(XB), 0, st, k);
      else hipLaunchKernelGGL((k2_xsweep<1, 0>), gx, dim3(XB), 0, st, k);
    });
    timed_launch(2, [&] {
      if (sch == 1) hipLaunchKernelGGL((k2_ysweep<1, 1>), gy, dim3(256), 0, st, k, rows);
      else if (sch == 2) hipLaunchKernelGGL((k2_ysweep<1, 2>), gy, dim3(256), 0, st, k, rows);
      else hipLaunchKernelGGL((k2_ysweep<1, 0>), gy, dim3(256), 0, st, k, rows);
    });
    timed_launch(1, [&] {
      if (sch == 2) hipLaunchKernelGGL((k2_xsweep<2, 2>), gx, dim3(XB), 0, st, k);
      else hipLaunchKernelGGL((k2_xsweep<2, 0>), gx, dim3(XB), 0, st, k);
    });
    timed_launch(2, [&] {
      if (sch == 1) hipLaunchKernelGGL((k2_ysweep<2, 1>), gy, dim3(256), 0, st, k, rows);
      else if (sch == 2) hipLaunchKernelGGL((k2_ysweep<2, 2>), gy, dim3(256), 0, st, k, rows);
      else hipLaunchKernelGGL((k2_ysweep<2, 0>), gy, dim3(256), 0, st, k, rows);
    });
    timed_launch(3, [&] { hipLaunchKernelGGL(k2_fin, gc, dim3(256), 0, st, k); });
    return r;
  };
  int64_t launched = 0;
  if (!timed) {
    for (; launched < max_steps; ++launched) {
      const alew_status r = one_step();
      if (r != ALEW_OK) return r;
    }
  } else {
    while (true) {
      for (int q = 0; q < c->check_every; ++q) {
        const alew_status r = one_step();
        if (r != ALEW_OK) return r;
      }
      launched += c->check_every;
      HIPCHK2(hipGetLastError());
      HIPCHK2(hipMemcpyAsync(c->st_h, c->st, sizeof(State2), hipMemcpyDeviceToHost, st));
      HIPCHK2(hipStreamSynchronize(st));
      if (c->st_h->done || c->st_h->status) break;
      if (max_steps > 0 && launched >= max_steps) break;
    }
  }
  HIPCHK2(hipGetLastError());
  hipLaunchKernelGGL(k2_out, dim3(nb), dim3(256), 0, st, k, h, hu, hv, b);
  hipLaunchKernelGGL(k2_mass_rows, dim3((unsigned)ny), dim3(256), 0, st, k);
  hipLaunchKernelGGL(k2_mass_sum, dim3(1), dim3(256), 0, st, k, c->mass + 2);
  HIPCHK2(hipEventRecord(c->ev1, st));
  HIPCHK2(hipGetLastError());
  HIPCHK2(hipMemcpyAsync(c->st_h, c->st, sizeof(State2), hipMemcpyDeviceToHost, st));
  HIPCHK2(hipMemcpyAsync(c->mass_h, c->mass, 4 * 8, hipMemcpyDeviceToHost, st));
  HIPCHK2(hipStreamSynchronize(st));
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) c->last_ms = ms;
  for (size_t q = 0; q < c->kt_kind.size(); ++q) {
    float m = 0.0f;
    HIPCHK2(hipEventElapsedTime(&m, c->kt_ev[2 * q], c->kt_ev[2 * q + 1]));
    c->kt_ms[c->kt_kind[q]] += m;
    c->kt_n[c->kt_kind[q]] += 1;
  }
  const State2& R = *c->st_h;
  const alew_status status = map_bits(R.status);
  if (stats) {
    stats->steps = R.steps;
    stats->t = R.t;
    stats->dt_min = R.steps > 0 ? R.dt_min : 0.0;
    stats->dt_max = R.dt_max;
    stats->mass0 = c->mass_h[0];
    stats->mass_b0 = c->mass_h[1];
    stats->mass = c->mass_h[2];
    stats->mass_b = c->mass_h[3];
    for (int q = 0; q < 3; ++q) stats->n_class[q] = (int64_t)R.n_class[q];
    stats->n_limited = (int64_t)R.n_limited;
    stats->status = (int32_t)status;
  }
  if (status != ALEW_OK)
    return fail2(status, status == ALEW_E_MESH       ? "a cell area became non-positive"
                         : status == ALEW_E_NEGDEPTH  ? "a mean depth below -1e-11"
                         : status == ALEW_E_NEGWEIGHT ? "a negative linear weight on the stage mesh"
                                                      : "non-finite state");
  return ALEW_OK;
}

}  // extern "C"
