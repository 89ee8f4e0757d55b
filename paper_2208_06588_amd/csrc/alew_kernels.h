// Tile bodies shared by the stage-launch engine and the persistent engine.
#pragma once

#include "alew_device.h"

namespace alew_dev {

// Records kept by the forward recomputation of the adjoint (all NULL otherwise).
struct Dump {
  double* q;     // [3 stages][3 comps][S]: stage inputs q^(s-1)
  double* D;     // [3][3][S]: alpha coefficient of the residual
  double* fs;    // [3 stages][2 sides][S + ninst]: trace speeds |u - w| + sqrt(g h) per face
  double* xw;    // [2][S + ninst]: x^n and w^n of the step
  double* scal;       // [ninst][8] of this step: t, dt, alpha_1..3, dx_0..2
  double* scal_next;  // the next step's record (t, dt, dx_0 are set at step end)
};

// Buffers of a packed batch.  Component c of a 3-vector array V lives at
// V + c * S, S = total cell count.  Node arrays hold ncell+1 entries per
// instance (node offset of instance i = cell_off[i] + i).
struct Bufs {
  const int64_t* cell_off;
  double* eta;  // state eta (scratch; h is formed on exit)
  double* m;    // state hu (caller's array)
  double* b;    // state b (caller's array)
  double* xa;   // nodes, even steps read xa, write xb
  double* xb;
  const double* xi;
  double* w;    // node speeds (times Inst::wscale); for the prescribed map A S(xi)
  double* P0;   // stage buffers: stages 1 and 3 write (P0, D0), stage 2 writes (P1, D1)
  double* D0;
  double* P1;
  double* D1;
  uint8_t* cls;  // optional [3][S] classes of the current step
  Inst* inst;
  const double* dts;  // optional frozen step sizes [ninst][dts_stride]
  double* dt_log;     // optional [ninst][dts_stride]
  int64_t dts_stride;
  int64_t S;
  int32_t ninst;
  int32_t pad;
  Dump dump;
};

// Per-instance view used by the tile bodies.
struct View {
  int64_t n, co, no;  // cells, cell offset, node offset
  const double* x;    // nodes of this step (x^n)
  double* xnew;       // nodes of the next step
};

__device__ __forceinline__ View make_view(const Bufs& bf, int i, const Inst& I) {
  View v;
  v.co = bf.cell_off[i];
  v.n = bf.cell_off[i + 1] - v.co;
  v.no = v.co + i;
  const bool odd = (I.steps & 1) != 0;
  v.x = (odd ? bf.xb : bf.xa) + v.no;
  v.xnew = (odd ? bf.xa : bf.xb) + v.no;
  return v;
}

struct StageScal {
  int s;           // 1..3
  double dt, cprev, dx, as, bs;
  double wsc;      // node speed = wsc * w[]
};

// Block-level results of a stage tile.
struct StageRes {
  double alpha, maxJ;
  unsigned ncls0, ncls1, ncls2, nlim, nneg;
  int status;
};

template <int B>
struct SmemStage {
  double e[B + 4], m[B + 4], b[B + 4], J[B + 4];
  double tr[6][B];
  double fl[8][B];
  double red[(B / 64) * 8];
  unsigned cnt[8];  // class S/T/N, limited, negative weight, status bits
};

// Stage-input state (eta, hu, b) and width of cell k (ghosts mapped).
__device__ __forceinline__ void load_stage_cell(const Bufs& bf, const Consts& cs, const View& v,
                                                const StageScal& sc, int64_t k, double& e,
                                                double& m, double& b, double& J, int& st) {
  double ms;
  const int64_t src = ghost_src(cs.bc, v.n, k, ms);
  const double Jn = v.x[src + 1] - v.x[src];
  const int64_t g = v.co + src;
  if (sc.s == 1) {
    J = Jn;
    e = bf.eta[g];
    m = bf.m[g] * ms;
    b = bf.b[g];
  } else {
    const double dw = bf.w[v.no + src + 1] * sc.wsc - bf.w[v.no + src] * sc.wsc;
    const double J1 = Jn + sc.dt * dw;
    J = (sc.s == 2) ? J1 : 0.75 * Jn + 0.25 * (J1 + sc.dt * dw);
    const double* P = (sc.s == 2) ? bf.P0 : bf.P1;
    const double* D = (sc.s == 2) ? bf.D0 : bf.D1;
    const double iJ = frcp(J);
    e = (P[g] + sc.cprev * D[g]) * iJ;
    m = ((P[bf.S + g] + sc.cprev * D[bf.S + g]) * iJ) * ms;
    b = (P[2 * bf.S + g] + sc.cprev * D[2 * bf.S + g]) * iJ;
  }
  if (!(J > 0.0)) st |= SB_MESH;
}

// One stage over the tile of owned cells [c0, c0 + B - 2) of one instance.
template <int B>
__device__ __forceinline__ StageRes stage_tile(const Bufs& bf, const Consts& cs, const View& v,
                                               const StageScal& sc, int64_t c0,
                                               SmemStage<B>& sm, uint8_t* cls_inst) {
  const int t = threadIdx.x;
  int st = 0;
  if (t < 8) sm.cnt[t] = 0u;
  // 1. stencil data for cells c0-3 .. c0+B
  for (int i = t; i < B + 4; i += B) {
    const int64_t k = c0 - 3 + i;
    double e = 0, m = 0, b = 0, J = 1;
    if (k >= -3 && k < v.n + 3) load_stage_cell(bf, cs, v, sc, k, e, m, b, J, st);
    sm.e[i] = e; sm.m[i] = m; sm.b[i] = b; sm.J[i] = J;
  }
  __syncthreads();
  // 2. reconstruct cell j = c0 - 1 + t (cells -1 and n are ghosts for the end faces)
  const int64_t j = c0 - 1 + t;
  const bool active = (j >= -1) && (j <= v.n);
  const bool owned = (t >= 1) && (t <= B - 2) && (j < v.n);
  CellRecon o;
  double ebar = 0, hbar = 0, mbar = 0, bbar = 0, Jj = 1;
  bool lim_owned = false, neg_cell = false;
  int cls_owned = -1;
  if (active) {
    double h5[5], v5[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      h5[k] = sm.e[t + k] - sm.b[t + k];
      v5[k] = (cs.flags & F_BETA_FROM_H) ? h5[k] : sm.e[t + k];
    }
    ebar = sm.e[t + 2]; mbar = sm.m[t + 2]; bbar = sm.b[t + 2]; hbar = h5[2]; Jj = sm.J[t + 2];
    const double Dx = (cs.flags & F_BETA_LOCAL) ? Jj : sc.dx;
    recon_cell(v5, h5, &sm.m[t], &sm.b[t], &sm.J[t], Dx, cs.weno_eps, ebar, o);
    const int lim = limit_cell(hbar, mbar, cs.pp_eps, o);
    if (owned) {
      cls_owned = o.cls;
      lim_owned = lim != 0;
      if (hbar < -cs.pp_eps) st |= SB_NEGDEPTH;
      if (cls_inst) cls_inst[j] = (uint8_t)o.cls;
    }
    if (o.negw && (owned || j == -1 || j == v.n)) { neg_cell = true; st |= SB_NEGWEIGHT; }
    sm.tr[0][t] = o.hL; sm.tr[1][t] = o.mL; sm.tr[2][t] = o.bL;
    sm.tr[3][t] = o.hR; sm.tr[4][t] = o.mR; sm.tr[5][t] = o.bR;
  }
  __syncthreads();
  // 3. face at node k = j (between cells j-1 and j), t = 1 .. B-1
  double fspeed = 0.0;
  if (t >= 1 && j >= 0 && j <= v.n) {
    Face f;
    face_flux(sm.tr[3][t - 1], sm.tr[4][t - 1], sm.tr[5][t - 1], sm.tr[0][t], sm.tr[1][t],
              sm.tr[2][t], bf.w[v.no + j] * sc.wsc, cs.g, cs.dry_eps, f);
    sm.fl[0][t] = f.Fc1; sm.fl[1][t] = f.Fc2; sm.fl[2][t] = f.Gc; sm.fl[3][t] = f.je;
    sm.fl[4][t] = f.jm; sm.fl[5][t] = f.jb; sm.fl[6][t] = f.B1; sm.fl[7][t] = f.B2;
    fspeed = f.speed;
    if (bf.dump.fs) {
      const int64_t NN = bf.S + bf.ninst;
      bf.dump.fs[(int64_t)(2 * (sc.s - 1)) * NN + v.no + j] = f.sl;
      bf.dump.fs[(int64_t)(2 * (sc.s - 1) + 1) * NN + v.no + j] = f.sr;
    }
  }
  __syncthreads();
  // 4. owned cells: residual split, stage combination
  double maxJ = 0.0;
  if (owned) {
    const double g = cs.g;
    const double Ae = -(sm.fl[0][t + 1] - sm.fl[0][t]);
    const double S = 0.5 * g * (sm.fl[7][t + 1] - sm.fl[7][t]) - g * ebar * (sm.fl[6][t + 1] - sm.fl[6][t]) - g * o.rint;
    const double Am = -(sm.fl[1][t + 1] - sm.fl[1][t]) + S;
    const double Ab = -(sm.fl[2][t + 1] - sm.fl[2][t]);
    const double De = 0.5 * (sm.fl[3][t + 1] - sm.fl[3][t]);
    const double Dm = 0.5 * (sm.fl[4][t + 1] - sm.fl[4][t]);
    const double Db = 0.5 * (sm.fl[5][t + 1] - sm.fl[5][t]);
    const int64_t gi = v.co + j;
    const double Jn = v.x[j + 1] - v.x[j];
    const double dw = bf.w[v.no + j + 1] * sc.wsc - bf.w[v.no + j] * sc.wsc;
    double Pe, Pm, Pb;
    if (sc.s == 1) {
      Pe = Jj * ebar + sc.dt * Ae;
      Pm = Jj * mbar + sc.dt * Am;
      Pb = Jj * bbar + sc.dt * Ab;
    } else {
      const double Qe = Jn * bf.eta[gi], Qm = Jn * bf.m[gi], Qb = Jn * bf.b[gi];
      Pe = sc.as * Qe + sc.bs * (Jj * ebar + sc.dt * Ae);
      Pm = sc.as * Qm + sc.bs * (Jj * mbar + sc.dt * Am);
      Pb = sc.as * Qb + sc.bs * (Jj * bbar + sc.dt * Ab);
    }
    double* Po = (sc.s == 2) ? bf.P1 : bf.P0;
    double* Do = (sc.s == 2) ? bf.D1 : bf.D0;
    Po[gi] = Pe; Po[bf.S + gi] = Pm; Po[2 * bf.S + gi] = Pb;
    Do[gi] = De; Do[bf.S + gi] = Dm; Do[2 * bf.S + gi] = Db;
    if (bf.dump.q) {
      const int64_t o = (int64_t)(3 * (sc.s - 1)) * bf.S + gi;
      bf.dump.q[o] = ebar; bf.dump.q[o + bf.S] = mbar; bf.dump.q[o + 2 * bf.S] = bbar;
      bf.dump.D[o] = De; bf.dump.D[o + bf.S] = Dm; bf.dump.D[o + 2 * bf.S] = Db;
    }
    const double Jnext = sc.as * Jn + sc.bs * (Jj + sc.dt * dw);
    maxJ = Jnext;
    if (!(Jnext > 0.0)) st |= SB_MESH;
  }
  // counters: one ballot per wave, summed in LDS
  {
    const unsigned long long b0 = __ballot(cls_owned == 0), b1 = __ballot(cls_owned == 1);
    const unsigned long long b2 = __ballot(cls_owned == 2), bl = __ballot(lim_owned);
    const unsigned long long bn = __ballot(neg_cell);
    if ((t & 63) == 0) {
      atomicAdd(&sm.cnt[0], (unsigned)__popcll(b0));
      atomicAdd(&sm.cnt[1], (unsigned)__popcll(b1));
      atomicAdd(&sm.cnt[2], (unsigned)__popcll(b2));
      if (bl) atomicAdd(&sm.cnt[3], (unsigned)__popcll(bl));
      if (bn) atomicAdd(&sm.cnt[4], (unsigned)__popcll(bn));
    }
    if (st) atomicOr(&sm.cnt[5], (unsigned)st);
  }
  double rv[2] = {fspeed, maxJ};
  const int op[2] = {0, 0};
  block_reduce<B, 2>(rv, op, sm.red);
  StageRes res;
  res.alpha = rv[0];
  res.maxJ = rv[1];
  res.ncls0 = sm.cnt[0]; res.ncls1 = sm.cnt[1]; res.ncls2 = sm.cnt[2];
  res.nlim = sm.cnt[3]; res.nneg = sm.cnt[4];
  res.status = (int)sm.cnt[5];
  __syncthreads();
  return res;
}

// Step epilogue over cells [c0, c0+B): q^{n+1}, x^{n+1}, and the reductions
// that size the next step.
struct FinalRes {
  double speed, minJ, maxJ, hmin;
  int status;
};

template <int B>
__device__ __forceinline__ FinalRes final_tile(const Bufs& bf, const Consts& cs, const View& v,
                                               double dt, double alpha3, double wsc, int64_t c0,
                                               double* red) {
  const int t = threadIdx.x;
  const int64_t j = c0 + t;
  int st = 0;
  double speed = 0.0, minJ = INFINITY, maxJ = 0.0, hmin = INFINITY;
  if (j < v.n) {
    const double x0 = v.x[j], x1 = v.x[j + 1];
    const double w0 = bf.w[v.no + j] * wsc, w1 = bf.w[v.no + j + 1] * wsc;
    const double Jn = x1 - x0, dw = w1 - w0;
    const double J1 = Jn + dt * dw;
    const double J2 = 0.75 * Jn + 0.25 * (J1 + dt * dw);
    const double J3 = (1.0 / 3.0) * Jn + (2.0 / 3.0) * (J2 + dt * dw);
    const double c = (2.0 / 3.0) * dt * alpha3;
    const int64_t gi = v.co + j;
    const double iJ3 = frcp(J3);
    const double e = (bf.P0[gi] + c * bf.D0[gi]) * iJ3;
    const double m = (bf.P0[bf.S + gi] + c * bf.D0[bf.S + gi]) * iJ3;
    const double b = (bf.P0[2 * bf.S + gi] + c * bf.D0[2 * bf.S + gi]) * iJ3;
    bf.eta[gi] = e; bf.m[gi] = m; bf.b[gi] = b;
    const double xn0 = x0 + dt * w0, xn1 = x1 + dt * w1;
    if (bf.dump.xw) {
      const int64_t NN = bf.S + bf.ninst;
      bf.dump.xw[v.no + j] = x0;
      bf.dump.xw[NN + v.no + j] = w0;
      if (j == v.n - 1) {
        bf.dump.xw[v.no + v.n] = x1;
        bf.dump.xw[NN + v.no + v.n] = w1;
      }
    }
    v.xnew[j] = xn0;
    if (j == v.n - 1) v.xnew[v.n] = xn1;
    const double Jnew = xn1 - xn0;
    const double h = e - b;
    const double u = h > cs.dry_eps ? m / h : 0.0;
    speed = fabs(u) + sqrt(cs.g * fmax(h, 0.0));
    minJ = Jnew; maxJ = Jnew; hmin = h;
    if (!(J3 > 0.0) || !(Jnew > 0.0)) st |= SB_MESH;
    if (!isfinite(e) || !isfinite(m) || !isfinite(b)) st |= SB_NONFINITE;
    if (h < -cs.pp_eps) st |= SB_NEGDEPTH;
  }
  double rv[4] = {speed, minJ, maxJ, hmin};
  const int op[4] = {0, 1, 0, 1};
  block_reduce<B, 4>(rv, op, red);
  __syncthreads();
  if (t == 0) red[0] = 0.0;
  __syncthreads();
  if (st) atomicOr((int*)&red[0], st);
  __syncthreads();
  FinalRes r;
  r.speed = rv[0]; r.minJ = rv[1]; r.maxJ = rv[2]; r.hmin = rv[3];
  r.status = *(int*)&red[0];
  __syncthreads();
  return r;
}

// Shape function of the prescribed mesh map.
__device__ __forceinline__ double mesh_shape(const Consts& cs, double xi, double x0, double x1) {
  if (cs.mesh == MESH_SINE) return sin(2.0 * M_PI * cs.mesh_k * xi);
  const double L = x1 - x0;
  return (xi - x1) * (xi - x0) / (3.0 * L * L);
}

// Chord factor of the prescribed map over the step [t, t+dt] (eq. (2.1)):
// (sin(om (t+dt)) - sin(om t)) / dt = 2 cos(om (t + dt/2)) sin(om dt/2) / dt;
// the node speed is (A S(xi)) times this factor.
__device__ __forceinline__ double chord_factor(const Consts& cs, double t, double dt) {
  const double om = cs.mesh_omega;
  return 2.0 * cos(om * (t + 0.5 * dt)) * sin(0.5 * om * dt) / dt;
}

// Fluid-following node speeds for nodes [k0, k0+B): node average of the cell
// velocities, two [1/4,1/2,1/4] passes, end nodes fixed (unless periodic).
template <int B>
__device__ __forceinline__ double wfluid_tile(const Bufs& bf, const Consts& cs, const View& v,
                                              int64_t k0, double* su /* B+6 */,
                                              double* sv /* B+4 */, double* red) {
  const int t = threadIdx.x;
  const bool per = cs.bc == BC_PERIODIC;
  const int64_t n = v.n;
  // cell velocities of cells k0-3 .. k0+B+2
  for (int i = t; i < B + 6; i += B) {
    const int64_t c = k0 - 3 + i;
    double u = 0.0;
    int64_t cc = c;
    if (per) { cc = c % n; if (cc < 0) cc += n; }
    if (cc >= 0 && cc < n) {
      const int64_t g = v.co + cc;
      const double h = bf.eta[g] - bf.b[g];
      u = h > cs.dry_eps ? bf.m[g] / h : 0.0;
    }
    su[i] = u;
  }
  __syncthreads();
  // level 0 at nodes k0-2 .. k0+B+1 (index i <-> node k0-2+i); node k sits between
  // cells k-1 and k (su index k-k0+3)
  auto endnode = [&](int64_t k) { return !per && (k <= 0 || k >= n); };
  for (int i = t; i < B + 4; i += B) {
    const int64_t k = k0 - 2 + i;
    sv[i] = endnode(k) ? 0.0 : 0.5 * (su[i] + su[i + 1]);
  }
  __syncthreads();
  // two smoothing passes; pass 1 on nodes k0-1 .. k0+B, pass 2 on k0 .. k0+B-1
  double a = 0.0;
  for (int i = t; i < B + 2; i += B) {
    const int64_t k = k0 - 1 + i;
    su[i] = endnode(k) ? 0.0 : 0.25 * sv[i] + 0.5 * sv[i + 1] + 0.25 * sv[i + 2];
  }
  __syncthreads();
  {
    const int64_t k = k0 + t;
    a = endnode(k) ? 0.0 : 0.25 * su[t] + 0.5 * su[t + 1] + 0.25 * su[t + 2];
  }
  double wabs = 0.0;
  const int64_t k = k0 + t;
  if (k <= n) {
    bf.w[v.no + k] = a;
    wabs = fabs(a);
  }
  double rv[1] = {wabs};
  const int op[1] = {0};
  __syncthreads();
  block_reduce<B, 1>(rv, op, red);
  __syncthreads();
  return rv[0];
}

// Time-step rule of the scheme: dt from the reductions of the previous epilogue.
__device__ __forceinline__ double next_dt(const Inst& I, const Consts& cs, const double* dts,
                                          int64_t dts_stride, int i) {
  double dt;
  if (dts) {
    dt = dts[(int64_t)i * dts_stride + I.steps];
  } else {
    double W;
    if (cs.mesh == MESH_SINE || cs.mesh == MESH_PAPER)
      W = fabs(cs.mesh_A * cs.mesh_omega * cos(cs.mesh_omega * I.t)) * I.smax;
    else
      W = bitsd(I.r_W);
    dt = cs.cfl * bitsd(I.r_minJ) / (bitsd(I.r_speed) + W);
  }
  if (I.t_end > I.t0 && I.t + dt > I.t_end) dt = I.t_end - I.t;
  return dt;
}

__device__ __forceinline__ bool inst_done(const Inst& I) {
  if (I.status & (SB_MESH | SB_NEGDEPTH | SB_NONFINITE)) return true;
  if (I.max_steps > 0 && I.steps >= I.max_steps) return true;
  if (I.t_end > I.t0 && !(I.t < I.t_end)) return true;
  if (!(I.t_end > I.t0) && I.max_steps <= 0) return true;
  return false;
}

}  // namespace alew_dev
