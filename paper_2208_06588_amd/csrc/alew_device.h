// Device building blocks of the FP64 ALE-WENO stage for gfx950.
//
// Layout: every per-cell quantity is a plain FP64 array (SoA).  A work-group of
// B threads handles a tile of B-2 consecutive cells of one instance: it stages
// the B+4 cells of the stencils (3 halo cells each side) in LDS, reconstructs
// the B cells c0-1 .. c0+B-2 (one per thread), exchanges the limited traces
// through LDS, evaluates the B-1 interface fluxes, and updates the B-2 owned
// cells.  The global Lax-Friedrichs speed of the stage (eq. (3.13)) is not
// known until every trace of the instance exists, so the update is split as
// RHS = A + alpha * D: the stage writes
//     P = a_s Q^n + b_s (J^(s-1) q^(s-1) + dt A)   and   D,
// and the next stage (or the step epilogue) forms Q^(s) = P + b_s dt alpha D
// while loading.  No MFMA: nothing here is a dense contraction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace alew_dev {

enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2 };
enum { MESH_GIVEN = 0, MESH_SINE = 1, MESH_PAPER = 2, MESH_FLUID = 3, MESH_ALIGNED = 4 };
// Meshes moved by a prescribed map X(xi, t) = xi + A S(xi) sin(omega t).
__host__ __device__ __forceinline__ bool prescribed(int mesh) {
  return mesh == MESH_SINE || mesh == MESH_PAPER || mesh == MESH_ALIGNED;
}
enum {
  F_BETA_LOCAL = 1, F_BETA_FROM_H = 2, F_HYDROSTATIC = 4, F_ALPHA_CELLAVG = 8, F_NO_HU_LIMIT = 16,
  F_W_TANGENT = 32, F_NONWB = 64, F_SPLIT = 128
};
// Scheme of a stage kernel (a template parameter): the special source-term
// treatment (Sec. 4.2), the hydrostatic reconstruction (Sec. 4.1), or the
// ALE-WENO scheme of Sec. 3 without well-balancing, with characteristic
// reconstruction; SCH_SPLIT added: negative linear weights split (a separate
// instantiation, so that the other kernels carry none of its registers).
enum { SCH_SPECIAL = 0, SCH_HYDRO = 1, SCH_NONWB = 2, SCH_SPLIT = 4 };
// status bits (combined per instance; mapped to alew_status on the host)
enum {
  SB_MESH = 1, SB_NEGDEPTH = 2, SB_NONFINITE = 4, SB_NEGWEIGHT = 8, SB_SEQUENCE = 16,
  SB_CAPACITY = 32
};

struct Consts {
  double g, cfl, weno_eps, pp_eps;
  double mesh_A, mesh_k, mesh_omega, dry_eps;
  int32_t bc, mesh, flags, bottom;
  double bp[4];
};

enum { BOT_ALE = 0, BOT_STEP = 1, BOT_GAUSS = 2, BOT_SIN2 = 3, BOT_BUMP = 4, BOT_PARABOLA = 5 };

// Average of the analytic bottom over [xl, xr] (the L2 projection of eq.
// (3.16) onto one cell): closed forms of the integral where the bottom has
// one, the 5-point Gauss-Legendre rule (exact to degree 9) for the Gaussian.
__device__ __forceinline__ double bottom_avg(const Consts& cs, double xl, double xr) {
  const double* p = cs.bp;
  const double L = xr - xl;
  switch (cs.bottom) {
    case BOT_STEP: {
      const double a = xl > p[1] ? xl : p[1], b = xr < p[2] ? xr : p[2];
      return b > a ? p[0] * ((b - a) / L) : 0.0;
    }
    case BOT_GAUSS: {
      const double r1 = 0.90617984593866399280, r2 = 0.53846931010568309104;
      const double w0 = 0.56888888888888888889, w1 = 0.23692688505618908751,
                   w2 = 0.47862867049936646804;
      const double m = 0.5 * (xl + xr), hw = 0.5 * L;
      auto f = [&](double x) { const double z = x - p[2]; return exp(-p[1] * (z * z)); };
      const double s = w0 * f(m) + w1 * (f(m - r1 * hw) + f(m + r1 * hw)) +
                       w2 * (f(m - r2 * hw) + f(m + r2 * hw));
      return p[0] * (0.5 * s);
    }
    case BOT_SIN2: {
      // sin^2 = (1 - cos 2 pi k x) / 2; the difference of sines over the cell by
      // the sum-to-product identity (no cancellation on small cells)
      const double k = M_PI * p[1];
      return p[0] * (0.5 - cos(k * (xl + xr)) * sin(k * L) / (2.0 * k * L));
    }
    case BOT_BUMP: {
      const double a = xl > p[2] - p[1] ? xl : p[2] - p[1];
      const double b = xr < p[2] + p[1] ? xr : p[2] + p[1];
      if (!(b > a)) return 0.0;
      const double k = M_PI / p[1];
      // int of cos(k (x - c)) over [a, b] = 2 cos(k (m - c)) sin(k (b - a) / 2) / k
      const double I = 2.0 * cos(k * (0.5 * (a + b) - p[2])) * sin(0.5 * k * (b - a)) / k;
      return p[0] * ((I + (b - a)) / L);
    }
    case BOT_PARABOLA:
      return p[0] * ((xl * xl + xl * xr + xr * xr) / (3.0 * p[1] * p[1]));
    default:
      return 0.0;
  }
}

// Per-instance scalars.  Reduction slots hold IEEE bit patterns so that
// integer atomics give order-independent max/min.
struct Inst {
  double t, t0, t_end, dt;
  double alpha[3];  // LF speed of stages 1..3
  double dx[3];     // Dx of the indicators at stages 1..3
  double smax;      // max_i |S(xi_i)| of the prescribed map
  double wscale;    // node speed of this step = wscale * w[] (w[] holds A S(xi) for the map)
  double dt_min, dt_max;
  double mass_eta0, mass_b0, mass_eta, mass_b;
  int64_t steps, max_steps;
  int32_t active, status;
  unsigned long long r_speed, r_minJ, r_maxJ, r_W;  // for the next step size
  unsigned long long r_hmin;                        // ordered key of min depth
  unsigned long long n_class[3], n_limited, n_negweight;
};

// Per-tile results.  Every tile writes its record with plain stores; a small
// kernel then reduces the records of each instance in tile order (one wave
// per instance), so no tile ever waits on, or queues behind, a shared address
// and every sum is taken in a fixed order.
//   stage record: LF speed, max next width, classes S/T/N, limited, negative
//                 weights, status bits, (records kept) first face trace
//                 attaining the tile's LF speed, unused
//   plain record: max speed, min width, max width, min depth, node-speed
//                 bound (or shape bound), two mass sums, unused
enum { SREC = 10, PREC = 8 };

// ----------------------------------------------------------------------------
// order-independent atomics on doubles
// ----------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long dbits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}
__device__ __forceinline__ double bitsd(unsigned long long u) {
  return __longlong_as_double((long long)u);
}
// total-order key for doubles of either sign (min via unsigned compare)
__device__ __forceinline__ unsigned long long okey(double v) {
  unsigned long long u = dbits(v);
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double okey_inv(unsigned long long k) {
  unsigned long long u = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
  return bitsd(u);
}
__device__ __forceinline__ void amax_pos(unsigned long long* p, double v) {
  atomicMax(p, dbits(v));
}

__device__ __forceinline__ unsigned hiword(double x) {
  return (unsigned)(__double_as_longlong(x) >> 32);
}

// Reciprocal: the hardware estimate r (relative error below 2^-24 on gfx950)
// refined by one third-order step, r (1 + e + e^2) with e = 1 - x r, whose
// error is of order e^3 (every divisor here is a positive width, depth or sum).
__device__ __forceinline__ double frcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// Square root of x >= 0 for the wave speeds: the hardware estimate y of
// 1/sqrt(x) (relative error below 2^-23 on gfx950), one Goldschmidt step for
// g ~ sqrt(x) and h ~ 1/(2 sqrt(x)), then two residual corrections
// g += (x - g^2) h.  Correctly rounded on [2^-45, 2^15] (4M samples), within
// a few ulp below; x = 0 gives 0 (the estimate is capped at 2^600).  A NaN
// stays NaN.  No rescaling of tiny arguments or class tests, unlike the
// library square root.
__device__ __forceinline__ double fsqrt(double x) {
  const double y = __builtin_fmin(__builtin_amdgcn_rsq(x), 0x1p600);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

// max / min of two values as one VALU instruction.  fmax / fmin on operands
// the compiler cannot prove canonical (loads, selects, lane shuffles) first
// quiet each operand with an extra instruction; no operand here can be a
// signalling NaN, and a quiet NaN operand gives the other one as fmax / fmin
// do.  The compiler inserts no wait states around inline asm, so the asm
// carries its own: one before (a transcendental result, e.g. of v_rsq_f64,
// needs one instruction before a VALU reads it) and two after (a DPP read of
// a VALU result needs two).  The nops cost issue slots of this wave only.
__device__ __forceinline__ double vmax(double a, double b) {
  double r;
  asm("s_nop 0\n\tv_max_f64 %0, %1, %2\n\ts_nop 1" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double vmin(double a, double b) {
  double r;
  asm("s_nop 0\n\tv_min_f64 %0, %1, %2\n\ts_nop 1" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// ----------------------------------------------------------------------------
// wave64 / work-group reductions (result in every thread)
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = vmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = vmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= (unsigned)__shfl_xor((int)v, o, 64);
  return v;
}
__device__ __forceinline__ unsigned wave_usum(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Work-group barrier for LDS traffic only: each wave waits for its own LDS
// accesses (s_waitcnt lgkmcnt(0); the vector-memory and export counters are
// left at their maxima), not for global loads, stores or direct-to-LDS copies
// still in flight.  The signal fences keep the compiler from moving memory
// accesses across the barrier.  Used only where the waves exchange data
// through LDS that they wrote with ordinary LDS stores.
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Reduce NV values per thread across the work-group.  op[k]: 0 max, 1 min, 2 sum.
template <int B, int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const int (&op)[NV], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k)
    v[k] = op[k] == 0 ? wave_max(v[k]) : (op[k] == 1 ? wave_min(v[k]) : wave_sum(v[k]));
  lds_sync();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wid * NV + k] = v[k];
  }
  lds_sync();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double r = red[k];
    for (int q = 1; q < B / 64; ++q) {
      double o = red[q * NV + k];
      r = op[k] == 0 ? vmax(r, o) : (op[k] == 1 ? vmin(r, o) : r + o);
    }
    v[k] = r;
  }
}

// ----------------------------------------------------------------------------
// boundary conditions (3 ghost cells per side)
// ----------------------------------------------------------------------------
__device__ __forceinline__ int64_t ghost_src(int bc, int64_t n, int64_t k, double& msign) {
  msign = 1.0;
  if (k >= 0 && k < n) return k;
  if (bc == BC_PERIODIC) {
    int64_t r = k % n;
    return r < 0 ? r + n : r;
  }
  if (bc == BC_TRANSMISSIVE) return k < 0 ? 0 : n - 1;
  msign = -1.0;
  return k < 0 ? -1 - k : 2 * n - 1 - k;
}

// ----------------------------------------------------------------------------
// Reconstruction of one cell (Sec. 2.2, Steps 1-4 with eq. (2.10)).
//
// Geometry in the cell's own normalised coordinate y = (x - x_j)/Delta_j,
// cell j = [-1/2, 1/2].  Each stencil quadratic is written as
//   p_r(y) = ubar_j + B_r y + C_r (y^2 - 1/12)
// (both basis functions have zero mean on cell j, so the average of cell j is
// matched by construction); B_r, C_r come from the 2x2 system matching the
// averages of the other two cells of the stencil.  The linear weights at each
// evaluation point are the unique weights (summing to one) under which the
// combination of the three quadratics also reproduces the cubic y^3 and the
// quartic y^4 - 1/80: with e_r^(3), e_r^(4) the errors of stencil r on those two
// functions, d is the normalised cross product e^(3) x e^(4).  That is the
// 5-cell quartic condition of Step 1, in a form with 3x3 work per point.
// ----------------------------------------------------------------------------
// Nonlinear weights at a point whose linear weights d include a negative one:
// the splitting of Shi, Hu & Shu (J. Comput. Phys. 175, 2002) with theta = 3.
// gp_r = (d_r + 3 |d_r|) / 2 and gm_r = gp_r - d_r are both non-negative
// (gp - gm = d); each group, normalised to sum one, gets the WENO-Z factors K,
// and the weights are sp w+_r - sm w-_r (sp, sm the group sums), which add up
// to one and stay in [-sm, sp] however the factors vary.  With w+_r =
// gp_r K_r / sum_s gp_s K_s (and likewise w-), the weights are
// K_r (cp gp_r - cm gm_r), cp = sp / sum gp K, cm = sm / sum gm K.  Kept out of
// line: it runs only on meshes with negative linear weights, and inlined it
// would cost the stage kernel registers on every mesh.
__device__ __forceinline__ void split_weights(const double* d, const double* K, double* ph) {
  double gp[3], gm[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    gp[r] = 0.5 * (d[r] + 3.0 * fabs(d[r]));
    gm[r] = gp[r] - d[r];
  }
  const double sp = gp[0] + gp[1] + gp[2], sm = gm[0] + gm[1] + gm[2];
  const double cp = sp / (gp[0] * K[0] + gp[1] * K[1] + gp[2] * K[2]);
  const double cm = sm / (gm[0] * K[0] + gm[1] * K[1] + gm[2] * K[2]);
#pragma unroll
  for (int r = 0; r < 3; ++r) ph[r] = K[r] * (cp * gp[r] - cm * gm[r]);
}

struct CellRecon {
  double hL, mL, bL, hR, mR, bR;  // unlimited traces
  double rint;                    // sum_mu w_mu (eta_mu - etabar) b_x(x_mu) * Delta_j
  double e1, e2, b1, b2;          // eta and b at the two interior Gauss-Lobatto points
                                  // (hydrostatic reconstruction only)
  int cls;
  int negw;
};

// Averages over the neighbour cells j-2, j-1, j+1, j+2 (slots 0..3) of y,
// y^2 - 1/12, y^3 and y^4 - 1/80, with y the coordinate in which cell j is
// [-1/2, 1/2].  A cell of centre c and width w averages y^2 to c^2 + w^2/12,
// y^3 to c^3 + c w^2/4 and y^4 to c^4 + c^2 w^2/2 + w^4/80.
__device__ __forceinline__ void stencil_moments(const double* __restrict__ J5, double iJ0,
                                                double* M1, double* M2, double* M3, double* M4) {
  const double w[4] = {J5[0] * iJ0, J5[1] * iJ0, J5[3] * iJ0, J5[4] * iJ0};
  const double em1 = -0.5 - w[1], ep1 = 0.5 + w[2];
  const double c[4] = {em1 - 0.5 * w[0], -0.5 - 0.5 * w[1], 0.5 + 0.5 * w[2], ep1 + 0.5 * w[3]};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double c2 = c[k] * c[k], w2 = w[k] * w[k];
    M1[k] = c[k];
    M2[k] = fma(w2, 1.0 / 12.0, c2) - 1.0 / 12.0;
    M3[k] = c[k] * fma(w2, 0.25, c2);
    M4[k] = fma(c2, fma(w2, 0.5, c2), fma(w2 * w2, 0.0125, -0.0125));
  }
}

// v5: eta (or h under F_BETA_FROM_H: chosen by the caller), stencil order
// cells j-2..j+2; iJ0 = frcp(J5[2]).  HR: instead of the special-source
// quadrature term, keep eta and b at the two interior points.
template <bool HR = false>
__device__ __forceinline__ void recon_cell(const double* __restrict__ v5,  // indicator var
                                           const double* __restrict__ h5,
                                           const double* __restrict__ m5,
                                           const double* __restrict__ b5,
                                           const double* __restrict__ J5, double iJ0, double Dx,
                                           double eps, double etabar, CellRecon& o,
                                           bool split = false) {
  const double J0 = J5[2];
  double M1[4], M2[4], M3[4], M4[4];  // cells j-2, j-1, j+1, j+2
  stencil_moments(J5, iJ0, M1, M2, M3, M4);
  // stencil r uses neighbour slots (c1, c2): r=0 -> (j+1, j+2), r=1 -> (j-1, j+1),
  // r=2 -> (j-2, j-1)
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
  // linear weights at the 4 Gauss-Lobatto points y = -1/2, -q, q, 1/2
  const double q = 0.22360679774997896964;       // sqrt(5)/10
  const double q3 = 0.011180339887498948482;     // q^3
  const double yv[4] = {-0.5, -q, q, 0.5};
  const double p2v[4] = {1.0 / 6.0, -1.0 / 30.0, -1.0 / 30.0, 1.0 / 6.0};
  const double f3v[4] = {-0.125, -q3, q3, 0.125};
  const double f4v[4] = {0.05, -0.01, -0.01, 0.05};
  // error coefficients of the stencils on y^3 and y^4 - 1/80 (the weights are
  // formed point by point below)
  double B3[3], C3[3], B4[3], C4[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int c1 = C1[r], c2 = C2[r];
    B3[r] = kb1[r] * M3[c1] + kb2[r] * M3[c2];
    C3[r] = kc1[r] * M3[c1] + kc2[r] * M3[c2];
    B4[r] = kb1[r] * M4[c1] + kb2[r] * M4[c2];
    C4[r] = kc1[r] * M4[c1] + kc2[r] * M4[c2];
  }
  unsigned sgn = 0u;  // OR of the high words: bit 31 set if some weight is negative
  // per-variable stencil coefficients
  double dv[4], dh[4], dm[4], db[4];
  {
    const int idx[4] = {0, 1, 3, 4};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      dv[c] = v5[idx[c]] - v5[2];
      dh[c] = h5[idx[c]] - h5[2];
      dm[c] = m5[idx[c]] - m5[2];
      db[c] = b5[idx[c]] - b5[2];
    }
  }
  double Bh[3], Ch[3], Bm[3], Cm[3], Bb[3], Cb[3], beta[3];
  const double kap = Dx * iJ0;
  const double kapC = kap * (1.0 / 3.0) + 4.0 * kap * kap * kap;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int c1 = C1[r], c2 = C2[r];
    const double Bv = kb1[r] * dv[c1] + kb2[r] * dv[c2];
    const double Cv = kc1[r] * dv[c1] + kc2[r] * dv[c2];
    Bh[r] = kb1[r] * dh[c1] + kb2[r] * dh[c2];
    Ch[r] = kc1[r] * dh[c1] + kc2[r] * dh[c2];
    Bm[r] = kb1[r] * dm[c1] + kb2[r] * dm[c2];
    Cm[r] = kc1[r] * dm[c1] + kc2[r] * dm[c2];
    Bb[r] = kb1[r] * db[c1] + kb2[r] * db[c2];
    Cb[r] = kc1[r] * db[c1] + kc2[r] * db[c2];
    // Dx int (p')^2 + Dx^3 int (p'')^2 over cell j, summed over the two equations
    beta[r] = (kap * (Bv * Bv) + kapC * (Cv * Cv)) + (kap * (Bm[r] * Bm[r]) + kapC * (Cm[r] * Cm[r]));
  }
  // Step 2: detector
  const double tau = fabs(beta[0] - beta[2]);
  const double betaA = (beta[0] + beta[1] + beta[2]) * (1.0 / 3.0);
  const double gam = tau * frcp(betaA + eps);
  const int cls = (gam <= 0.5) ? 0 : ((gam >= 1.0) ? 2 : 1);
  // Steps 3-4 at the 4 points: h, m, b at the end points (traces); at every
  // point the term of the interior Gauss-Lobatto quadrature of
  // (eta - etabar) b_x, weights (1,5,5,1)/12, summed in point order
  const double wgl[4] = {1.0 / 12.0, 5.0 / 12.0, 5.0 / 12.0, 1.0 / 12.0};
  double ri = 0.0;
  // The smooth class combines the stencils with the linear weights, which is
  // the 5-cell quartic Q = ubar + a1 y + a2 (y^2 - 1/12) + a3 y^3 +
  // a4 (y^4 - 1/80) itself.  Each stencil quadratic reproduces the first two
  // terms and projects the last two: B_r = a1 + a3 B3_r + a4 B4_r and
  // C_r = a2 + a3 C3_r + a4 C4_r, so stencils 0 and 2 give a3, a4 (a 2x2
  // system that only depends on the geometry) and stencil 1 gives a1, a2.
  // b_x of the smooth class is Q_b' / Delta_j.
  // the 2x2 matrix of stencils 0 and 2 (formed where used: kept live across
  // the point loops it would cost registers)
  auto gmat = [&](double* g) {
    g[0] = B3[0] - B3[2]; g[1] = B4[0] - B4[2];
    g[2] = C3[0] - C3[2]; g[3] = C4[0] - C4[2];
  };
  auto quartic = [&](const double* Bx, const double* Cx, const double* g, double igd, double* a) {
    const double dB = Bx[0] - Bx[2], dC = Cx[0] - Cx[2];
    a[2] = (g[3] * dB - g[1] * dC) * igd;
    a[3] = (g[0] * dC - g[2] * dB) * igd;
    a[0] = Bx[1] - (a[2] * B3[1] + a[3] * B4[1]);
    a[1] = Cx[1] - (a[2] * C3[1] + a[3] * C4[1]);
  };
  // Q' at the 4 points from its even and odd parts
  auto qslope = [&](const double* a, double* bx) {
    const double ee = a[0] + 0.75 * a[2], oe = a[1] + 0.5 * a[3];
    const double ei = a[0] + 0.15 * a[2], oi = (2.0 * q) * a[1] + (4.0 * q3) * a[3];
    bx[0] = (ee - oe) * iJ0;
    bx[1] = (ei - oi) * iJ0;
    bx[2] = (ei + oi) * iJ0;
    bx[3] = (ee + oe) * iJ0;
  };
  // Where no width of the stencil is more than four times another, every
  // linear weight at the 4 points is positive (smallest 0.011, at widths
  // (4, 4, 4, 1, 1)): a smooth cell there needs neither the weights nor their
  // sign test and evaluates Q directly.
  const double jmax = vmax(vmax(vmax(J5[0], J5[1]), vmax(J5[3], J5[4])), J0);
  const double jmin = vmin(vmin(vmin(J5[0], J5[1]), vmin(J5[3], J5[4])), J0);
  if (cls == 0 && jmax <= 4.0 * jmin) {
    double g[4];
    gmat(g);
    const double igd = frcp(g[0] * g[3] - g[1] * g[2]);
    double ah[4], ab[4], am[4], bx[4];
    quartic(Bh, Ch, g, igd, ah);
    quartic(Bb, Cb, g, igd, ab);
    quartic(Bm, Cm, g, igd, am);
    qslope(ab, bx);
    // values at -1/2, -q, q, 1/2: even part a2 p2 + a4 f4, odd part a1 y + a3 y^3
    auto vals = [&](double v0, const double* a, double* v) {
      const double ee = a[1] * (1.0 / 6.0) + a[3] * 0.05, oe = a[0] * 0.5 + a[2] * 0.125;
      const double ei = a[1] * (-1.0 / 30.0) + a[3] * (-0.01), oi = a[0] * q + a[2] * q3;
      v[0] = v0 + (ee - oe);
      v[1] = v0 + (ei - oi);
      v[2] = v0 + (ei + oi);
      v[3] = v0 + (ee + oe);
    };
    double hv[4], bv[4];
    vals(h5[2], ah, hv);
    vals(b5[2], ab, bv);
    if (HR) {
      o.e1 = hv[1] + bv[1]; o.b1 = bv[1];
      o.e2 = hv[2] + bv[2]; o.b2 = bv[2];
    } else {
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) ri += (wgl[mu] * J0) * (((hv[mu] + bv[mu]) - etabar) * bx[mu]);
    }
    o.hL = hv[0]; o.bL = bv[0]; o.hR = hv[3]; o.bR = bv[3];
    const double em = am[1] * (1.0 / 6.0) + am[3] * 0.05, om = am[0] * 0.5 + am[2] * 0.125;
    o.mL = m5[2] + (em - om);
    o.mR = m5[2] + (em + om);
    o.rint = ri;
    o.cls = 0;
    o.negw = 0;
    return;
  }
  // linear weights d_r at point mu
  auto lin_weights = [&](int mu, double* d) {
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
    d[0] = x0 * is;
    d[1] = x1 * is;
    d[2] = x2 * is;
    sgn |= hiword(d[0]) | hiword(d[1]) | hiword(d[2]);
  };
  // reconstructed values at point mu with the weights ph_r; b_x given (bxg)
  // or, non-smooth class, the stencil slopes weighted by ph
  auto at_point = [&](int mu, const double* ph, double bxg) {
    const double y = yv[mu], p2 = p2v[mu];
    double sBh = 0, sCh = 0, sBm = 0, sCm = 0, sBb = 0, sCb = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      sBh += ph[r] * Bh[r];
      sCh += ph[r] * Ch[r];
      sBm += ph[r] * Bm[r];
      sCm += ph[r] * Cm[r];
      sBb += ph[r] * Bb[r];
      sCb += ph[r] * Cb[r];
    }
    const double hv = h5[2] + (sBh * y + sCh * p2);
    const double bv = b5[2] + (sBb * y + sCb * p2);
    if (HR) {
      if (mu == 1) { o.e1 = hv + bv; o.b1 = bv; }
      if (mu == 2) { o.e2 = hv + bv; o.b2 = bv; }
    } else {
      const double bxv = cls == 2 ? (sBb + 2.0 * y * sCb) * iJ0 : bxg;
      ri += (wgl[mu] * J0) * (((hv + bv) - etabar) * bxv);
    }
    if (mu == 0) { o.hL = hv; o.mL = m5[2] + (sBm * y + sCm * p2); o.bL = bv; }
    if (mu == 3) { o.hR = hv; o.mR = m5[2] + (sBm * y + sCm * p2); o.bR = bv; }
  };
  // one branch per cell (not per point)
  if (cls == 0) {
    // smooth cell on a stencil with widths further apart: the weights (and
    // their sign test) at every point, b_x the quartic's
    double bx[4] = {0.0, 0.0, 0.0, 0.0};
    if (!HR) {
      double g[4], ab[4];
      gmat(g);
      quartic(Bb, Cb, g, frcp(g[0] * g[3] - g[1] * g[2]), ab);
      qslope(ab, bx);
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      double d[3];
      lin_weights(mu, d);
      at_point(mu, d, bx[mu]);
    }
  } else {
    double K[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double z = tau * frcp(beta[r] + eps);
      K[r] = 1.0 + z * z;
    }
    const double Mg = 2.0 * gam - 1.0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      double d[3], ph[3];
      lin_weights(mu, d);
      if (__builtin_expect(split && ((hiword(d[0]) | hiword(d[1]) | hiword(d[2])) >> 31), 0)) {
        split_weights(d, K, ph);
      } else {
        const double a0 = d[0] * K[0], a1 = d[1] * K[1], a2 = d[2] * K[2];
        const double ia = frcp(a0 + a1 + a2);
        ph[0] = a0 * ia;
        ph[1] = a1 * ia;
        ph[2] = a2 * ia;
      }
      double bxg = 0.0;
      if (cls == 1) {
        // transition: b_x = Mg (WENO-Z weighted slopes) + (1 - Mg) Q' (the
        // quartic recomputed at each point: a rare class, no registers held
        // across the loop)
        const double y = yv[mu];
        const double wN = HR ? 0.0
                             : ((ph[0] * Bb[0] + ph[1] * Bb[1] + ph[2] * Bb[2]) +
                                2.0 * y * (ph[0] * Cb[0] + ph[1] * Cb[1] + ph[2] * Cb[2])) * iJ0;
#pragma unroll
        for (int r = 0; r < 3; ++r) ph[r] = Mg * ph[r] + (1.0 - Mg) * d[r];
        if (!HR) {
          double g[4], ab[4];
          gmat(g);
          quartic(Bb, Cb, g, frcp(g[0] * g[3] - g[1] * g[2]), ab);
          const double qd = ab[0] + (2.0 * y) * ab[1] + (3.0 * y * y) * ab[2] +
                            (4.0 * y * y * y) * ab[3];
          bxg = Mg * wN + (1.0 - Mg) * (qd * iJ0);
        }
      }
      at_point(mu, ph, bxg);
    }
  }
  o.rint = ri;
  o.cls = cls;
  o.negw = (int)(sgn >> 31);
}

// ----------------------------------------------------------------------------
// Reconstruction with weights of its own for each variable (the scheme of
// Sec. 3 without well-balancing): the geometry of the cell (stencil maps and
// the linear weights at the 4 Gauss-Lobatto points) is shared, and each
// variable gets its indicators, detector class and hybrid weights (Sec. 2.2,
// Steps 2-4 for a scalar).
// ----------------------------------------------------------------------------
struct CellGeom {
  double kb1[3], kb2[3], kc1[3], kc2[3];  // B_r, C_r from the two other averages of stencil r
  double d[4][3];                         // linear weights at the 4 points
  double dd[4][3];                        // their derivatives d/dy at the 4 points
  double kap, kapC;                       // Dx / Delta_j and the y^2 indicator factor
  // the 5-cell quartic's a3, a4 = qi (B_0 - B_2, C_0 - C_2) and a1 = B_1 -
  // a3 qb[0] - a4 qb[1], a2 = C_1 - a3 qb[2] - a4 qb[3] (see recon_cell)
  double qi[4], qb[4];
  unsigned sgn;                           // OR of the weights' high words (sign bit)
};

__device__ __forceinline__ void cell_geom(const double* __restrict__ J5, double iJ0, double Dx,
                                          CellGeom& G) {
  double M1[4], M2[4], M3[4], M4[4];
  stencil_moments(J5, iJ0, M1, M2, M3, M4);
  const int C1[3] = {2, 1, 0}, C2[3] = {3, 2, 1};
  double B3[3], C3[3], B4[3], C4[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int c1 = C1[r], c2 = C2[r];
    const double idet = frcp(M1[c1] * M2[c2] - M1[c2] * M2[c1]);
    G.kb1[r] = M2[c2] * idet;
    G.kb2[r] = -M2[c1] * idet;
    G.kc1[r] = -M1[c2] * idet;
    G.kc2[r] = M1[c1] * idet;
    B3[r] = G.kb1[r] * M3[c1] + G.kb2[r] * M3[c2];
    C3[r] = G.kc1[r] * M3[c1] + G.kc2[r] * M3[c2];
    B4[r] = G.kb1[r] * M4[c1] + G.kb2[r] * M4[c2];
    C4[r] = G.kc1[r] * M4[c1] + G.kc2[r] * M4[c2];
  }
  const double q = 0.22360679774997896964, q3 = 0.011180339887498948482;
  const double yv[4] = {-0.5, -q, q, 0.5};
  const double p2v[4] = {1.0 / 6.0, -1.0 / 30.0, -1.0 / 30.0, 1.0 / 6.0};
  const double f3v[4] = {-0.125, -q3, q3, 0.125};
  const double f4v[4] = {0.05, -0.01, -0.01, 0.05};
  unsigned sgn = 0u;
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
    G.d[mu][0] = x0 * is;
    G.d[mu][1] = x1 * is;
    G.d[mu][2] = x2 * is;
    sgn |= hiword(G.d[mu][0]) | hiword(G.d[mu][1]) | hiword(G.d[mu][2]);
    // d_r' = (x_r' - d_r X') / X with X = x_0 + x_1 + x_2 (quotient rule), the
    // error vectors differentiated term by term
    const double y = yv[mu];
    double g3[3], g4[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      g3[r] = B3[r] + 2.0 * C3[r] * y - 3.0 * y * y;
      g4[r] = B4[r] + 2.0 * C4[r] * y - 4.0 * y * y * y;
    }
    const double y0 = g3[1] * e4[2] + e3[1] * g4[2] - g3[2] * e4[1] - e3[2] * g4[1];
    const double y1 = g3[2] * e4[0] + e3[2] * g4[0] - g3[0] * e4[2] - e3[0] * g4[2];
    const double y2 = g3[0] * e4[1] + e3[0] * g4[1] - g3[1] * e4[0] - e3[1] * g4[0];
    const double Xp = y0 + y1 + y2;
    G.dd[mu][0] = (y0 - G.d[mu][0] * Xp) * is;
    G.dd[mu][1] = (y1 - G.d[mu][1] * Xp) * is;
    G.dd[mu][2] = (y2 - G.d[mu][2] * Xp) * is;
  }
  G.sgn = sgn;
  G.kap = Dx * iJ0;
  G.kapC = G.kap * (1.0 / 3.0) + 4.0 * G.kap * G.kap * G.kap;
  {
    const double g00 = B3[0] - B3[2], g01 = B4[0] - B4[2];
    const double g10 = C3[0] - C3[2], g11 = C4[0] - C4[2];
    const double igd = frcp(g00 * g11 - g01 * g10);
    G.qi[0] = g11 * igd; G.qi[1] = -g01 * igd;
    G.qi[2] = -g10 * igd; G.qi[3] = g00 * igd;
    G.qb[0] = B3[1]; G.qb[1] = B4[1]; G.qb[2] = C3[1]; G.qb[3] = C4[1];
  }
}

// Values of one variable at the 4 points (and, with der, its x-derivative);
// returns the variable's class.
__device__ __forceinline__ int recon_scalar(const CellGeom& G, const double* u5, double eps,
                                            double iJ0, double* val, double* der,
                                            bool split = false) {
  const int C1[3] = {2, 1, 0}, C2[3] = {3, 2, 1};
  const double du[4] = {u5[0] - u5[2], u5[1] - u5[2], u5[3] - u5[2], u5[4] - u5[2]};
  double Bv[3], Cv[3], beta[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    Bv[r] = G.kb1[r] * du[C1[r]] + G.kb2[r] * du[C2[r]];
    Cv[r] = G.kc1[r] * du[C1[r]] + G.kc2[r] * du[C2[r]];
    beta[r] = G.kap * (Bv[r] * Bv[r]) + G.kapC * (Cv[r] * Cv[r]);
  }
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
  const double q = 0.22360679774997896964;
  const double yv[4] = {-0.5, -q, q, 0.5};
  const double p2v[4] = {1.0 / 6.0, -1.0 / 30.0, -1.0 / 30.0, 1.0 / 6.0};
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    double ph[3], pn[3] = {0.0, 0.0, 0.0};
    if (cls == 0) {
#pragma unroll
      for (int r = 0; r < 3; ++r) ph[r] = G.d[mu][r];
    } else {
      if (__builtin_expect(split && ((hiword(G.d[mu][0]) | hiword(G.d[mu][1]) | hiword(G.d[mu][2])) >> 31), 0)) {
        split_weights(G.d[mu], K, ph);
      } else {
        const double a0 = G.d[mu][0] * K[0], a1 = G.d[mu][1] * K[1], a2 = G.d[mu][2] * K[2];
        const double ia = frcp(a0 + a1 + a2);
        ph[0] = a0 * ia;
        ph[1] = a1 * ia;
        ph[2] = a2 * ia;
      }
      pn[0] = ph[0]; pn[1] = ph[1]; pn[2] = ph[2];
      if (cls == 1) {
#pragma unroll
        for (int r = 0; r < 3; ++r) ph[r] = Mg * ph[r] + (1.0 - Mg) * G.d[mu][r];
      }
    }
    double sB = 0.0, sC = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      sB += ph[r] * Bv[r];
      sC += ph[r] * Cv[r];
    }
    val[mu] = u5[2] + (sB * yv[mu] + sC * p2v[mu]);
    if (der) {
      // the derivative of the reconstruction: where it is the 5-cell quartic
      // sum_r d_r p_r (smooth class), sum_r (d_r' p_r + d_r p_r') (fourth
      // order; the weighted stencil derivatives alone are second order); the
      // WENO-Z weighted stencil slopes where it is not, blended by Mg in the
      // transition class
      double dq = 0.0;
      if (cls != 2) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
          dq += G.d[mu][r] * (Bv[r] + 2.0 * yv[mu] * Cv[r]) +
                G.dd[mu][r] * (Bv[r] * yv[mu] + Cv[r] * p2v[mu]);
      }
      if (cls == 0) {
        der[mu] = dq * iJ0;
      } else {
        double sBn = 0.0, sCn = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          sBn += pn[r] * Bv[r];
          sCn += pn[r] * Cv[r];
        }
        const double wN = (sBn + 2.0 * yv[mu] * sCn) * iJ0;
        der[mu] = cls == 2 ? wN : Mg * wN + (1.0 - Mg) * (dq * iJ0);
      }
    }
  }
  return cls;
}

// Cell of the scheme without well-balancing: (eta, hu) reconstructed in the
// characteristic variables of the cell's mean state (eigenvectors of the flux
// Jacobian, (1, u -+ c); component-wise where the mean depth is at most dry),
// b with weights of its own.  Traces of h = eta - b, hu and b; rint = the
// source integral of -g (eta - b) b_x over the cell by the 4-point
// Gauss-Lobatto rule with the unlimited values.  The class is the largest of
// the three variables' classes.
__device__ __forceinline__ void recon_cell_char(const double* __restrict__ e5,
                                                const double* __restrict__ m5,
                                                const double* __restrict__ b5,
                                                const double* __restrict__ J5, double iJ0, double Dx,
                                                double eps, double g, double dry, CellRecon& o,
                                                bool split = false) {
  CellGeom G;
  cell_geom(J5, iJ0, Dx, G);
  const double hb = e5[2] - b5[2];
  const bool chr = hb > dry;
  double u = 0.0, c = 0.0, w1[5], w2[5];
  if (chr) {
    u = m5[2] * frcp(hb);
    c = fsqrt(g * hb);
    const double i2c = 0.5 * frcp(c);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      w1[k] = ((u + c) * e5[k] - m5[k]) * i2c;
      w2[k] = ((c - u) * e5[k] + m5[k]) * i2c;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 5; ++k) { w1[k] = e5[k]; w2[k] = m5[k]; }
  }
  double v1[4], v2[4], bv[4], bx[4];
  const int c1 = recon_scalar(G, w1, eps, iJ0, v1, nullptr, split);
  const int c2 = recon_scalar(G, w2, eps, iJ0, v2, nullptr, split);
  const int cb = recon_scalar(G, b5, eps, iJ0, bv, bx, split);
  const double wgl[4] = {1.0 / 12.0, 5.0 / 12.0, 5.0 / 12.0, 1.0 / 12.0};
  double ri = 0.0, ev[4], mv[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    ev[mu] = chr ? v1[mu] + v2[mu] : v1[mu];
    mv[mu] = chr ? (u - c) * v1[mu] + (u + c) * v2[mu] : v2[mu];
    ri += (wgl[mu] * J5[2]) * ((-g) * ((ev[mu] - bv[mu]) * bx[mu]));
  }
  o.hL = ev[0] - bv[0]; o.mL = mv[0]; o.bL = bv[0];
  o.hR = ev[3] - bv[3]; o.mR = mv[3]; o.bR = bv[3];
  o.rint = ri;
  o.cls = c1 > c2 ? c1 : c2;
  if (cb > o.cls) o.cls = cb;
  o.negw = (int)(G.sgn >> 31);
}

// ----------------------------------------------------------------------------
// Positivity limiter, 1D form of eq. (3.20)-(3.21); bottom traces by Remark 4.1.
// The hu traces are scaled by the same Phi about their mean unless hu_lim is
// false (then the limiter acts on h, and through Remark 4.1 on b, only).
// Returns 1 when the traces were modified.
// ----------------------------------------------------------------------------
// keep_b: the bottom traces stay and eta follows h (the scheme without
// well-balancing); by default eta stays and b follows h (Remark 4.1).
__device__ __forceinline__ int limit_cell(double hbar, double mbar, double pp_eps, CellRecon& o,
                                          bool hu_lim = true, bool keep_b = false) {
  if (hbar <= 0.0) {
    const double eL = o.hL + o.bL, eR = o.hR + o.bR;
    o.hL = hbar; o.hR = hbar;
    if (hu_lim) { o.mL = mbar; o.mR = mbar; }
    if (!keep_b) {
      o.bL = eL - o.hL;
      o.bR = eR - o.hR;
    }
    return 1;
  }
  const double s1 = 1.0 / 12.0;
  const double delta = (hbar - s1 * o.hL - s1 * o.hR) * (1.0 / (1.0 - 2.0 * s1));
  double mn = o.hL;
  if (delta < mn) mn = delta;
  if (o.hR < mn) mn = o.hR;
  const double epsj = (pp_eps < hbar) ? pp_eps : hbar;
  if (!(mn < epsj)) return 0;
  double Phi = (hbar - epsj) * frcp(hbar - mn);
  if (Phi > 1.0) Phi = 1.0;
  const double eL = o.hL + o.bL, eR = o.hR + o.bR;
  o.hL = Phi * (o.hL - hbar) + hbar;
  o.hR = Phi * (o.hR - hbar) + hbar;
  if (hu_lim) {
    o.mL = Phi * (o.mL - mbar) + mbar;
    o.mR = Phi * (o.mR - mbar) + mbar;
  }
  if (!keep_b) {
    o.bL = eL - o.hL;
    o.bR = eR - o.hR;
  }
  return 1;
}

// ----------------------------------------------------------------------------
// Interface flux pieces (eq. (3.13), (3.17), (4.9)) for left trace (cell i-1's
// right trace) and right trace (cell i's left trace) at node speed w.
// F_hat = Fc - alpha/2 * jump; the alpha part is applied later.
// ----------------------------------------------------------------------------
struct Face {
  double Fc1, Fc2, Gc, je, jm, jb, B1, B2;
  double speed;   // max over both traces of |u - w| + sqrt(g h)
  double sl, sr;  // the two trace speeds
};

__device__ __forceinline__ void face_flux(double hl, double ml, double bl, double hr, double mr,
                                          double br, double w, double g, double dry, Face& f) {
  const double el = hl + bl, er = hr + br;
  double ul = 0.0, ur = 0.0;
  if (hl > dry) ul = ml * frcp(hl); else ml = 0.0;
  if (hr > dry) ur = mr * frcp(hr); else mr = 0.0;
  const double Hl1 = ml - w * el;
  const double Hl2 = ml * ul + 0.5 * g * hl * hl - w * ml;
  const double Hr1 = mr - w * er;
  const double Hr2 = mr * ur + 0.5 * g * hr * hr - w * mr;
  f.Fc1 = 0.5 * (Hl1 + Hr1);
  f.Fc2 = 0.5 * (Hl2 + Hr2);
  f.Gc = -0.5 * w * (bl + br);
  f.je = er - el;
  f.jm = mr - ml;
  f.jb = br - bl;
  f.B1 = 0.5 * (bl + br);
  f.B2 = 0.5 * (bl * bl + br * br);
  const double sl = fabs(ul - w) + fsqrt(g * vmax(hl, 0.0));
  const double sr = fabs(ur - w) + fsqrt(g * vmax(hr, 0.0));
  f.speed = vmax(sl, sr);
  f.sl = sl;
  f.sr = sr;
}

// Hydrostatic reconstruction (Sec. 4.1, eq. (4.2)-(4.3)) at the face between
// a left cell (own right trace hl, ml, bl) and a right cell (own left trace
// hr, mr, br).  h* = max(0, eta - max(bl, br)) on both sides, the discharge
// kept; the momentum flux of the starred states is Fc2 (same for both cells),
// and each cell adds the pressure correction g/2 (h^2 - h*^2) of its own trace
// (cl for the left cell, cr for the right one).  The eta flux of eq. (4.2)
// reduces to the unmodified one: the theta term undoes the starred eta in
// the central part and in the alpha jump.  Fc1, Gc, the jumps and the speeds
// are those of face_flux (alpha from the unstarred traces).
struct FaceHR {
  double Fc1, Fc2, Gc, je, jm, jb, cl, cr;
  double speed, sl, sr;
};

__device__ __forceinline__ void face_flux_hydro(double hl, double ml, double bl, double hr, double mr,
                                                double br, double w, double g, double dry, FaceHR& f) {
  const double el = hl + bl, er = hr + br;
  double ul = 0.0, ur = 0.0;
  if (hl > dry) ul = ml * frcp(hl); else ml = 0.0;
  if (hr > dry) ur = mr * frcp(hr); else mr = 0.0;
  const double bmax = vmax(bl, br);
  const double hsl = vmax(el - bmax, 0.0), hsr = vmax(er - bmax, 0.0);
  const double usl = hsl > dry ? ml * frcp(hsl) : 0.0;
  const double usr = hsr > dry ? mr * frcp(hsr) : 0.0;
  const double g2 = 0.5 * g;
  f.Fc1 = 0.5 * ((ml - w * el) + (mr - w * er));
  f.Fc2 = 0.5 * ((ml * usl + g2 * hsl * hsl - w * ml) + (mr * usr + g2 * hsr * hsr - w * mr));
  f.Gc = -0.5 * w * (bl + br);
  f.je = er - el;
  f.jm = mr - ml;
  f.jb = br - bl;
  f.cl = g2 * (hl * hl - hsl * hsl);
  f.cr = g2 * (hr * hr - hsr * hsr);
  const double sl = fabs(ul - w) + fsqrt(g * vmax(hl, 0.0));
  const double sr = fabs(ur - w) + fsqrt(g * vmax(hr, 0.0));
  f.speed = vmax(sl, sr);
  f.sl = sl;
  f.sr = sr;
}

// Hydrostatic source of one cell (after eq. (4.3)): the integral over the cell
// of -g (eta_h - b_h) d b_h / dx, eta_h and b_h the cubics through the values
// at the 4 Gauss-Lobatto points (e0, b0 the left trace, e3, b3 the right one).
// In the cell coordinate s in [0,1] the width cancels; the 4-point
// Gauss-Lobatto rule (weights 1, 5, 5, 1 over 12) is exact for the degree-5
// integrand, and d b_h / ds at the points is the cubic's differentiation
// matrix, whose entries are 6, 1, sqrt 5 and multiples of the golden ratio
// phi and of phi - 1.
__device__ __forceinline__ double hydro_source(double g, double e0, double e1, double e2, double e3,
                                               double b0, double b1, double b2, double b3) {
  const double PHI = 1.6180339887498948482, PHI1 = 0.6180339887498948482;
  const double R5 = 2.2360679774997896964;
  const double d0 = -6.0 * b0 + 5.0 * PHI * b1 - 5.0 * PHI1 * b2 + b3;
  const double d1 = -PHI * b0 + R5 * b2 - PHI1 * b3;
  const double d2 = PHI1 * b0 - R5 * b1 + PHI * b3;
  const double d3 = -b0 + 5.0 * PHI1 * b1 - 5.0 * PHI * b2 + 6.0 * b3;
  const double q = ((e0 - b0) * d0 + (e3 - b3) * d3) + 5.0 * ((e1 - b1) * d1 + (e2 - b2) * d2);
  return (-g / 12.0) * q;
}

}  // namespace alew_dev
