// MI355X (gfx950) library for the 1D well-balanced ALE-WENO hybrid scheme
// (special source-term treatment, or the hydrostatic reconstruction under
// F_HYDROSTATIC: a template parameter of the stage, persistent and reverse
// kernels): kernels and the C ABI declared in include/alew.h.
//
// Two engines run the same tile bodies (alew_kernels.h):
//  * stage launches: each kernel covers every tile of every active instance;
//    every tile writes a record of its results (LF speed, widths, counts,
//    status), and the per-instance reductions of the records (maxima, minima,
//    integer counts: order independent) run as small launches between the
//    stage kernels.  One time step is 9-10 launches; a 2-step sequence is
//    replayed as a hipGraph.
//  * persistent: one launch runs a whole ragged batch.  A work-group takes the
//    next instance from a device queue (largest first), runs all of its steps
//    with work-group reductions only, and takes the next one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <type_traits>
#include <string>
#include <vector>

#include "alew.h"
#include "alew_adjoint.h"
#include "alew_kernels.h"

using namespace alew_dev;

// ============================================================================
// kernels
// ============================================================================
// Items per plain tile (set-up, step epilogue, finish): independent of the
// stage kernels' work-group size.
constexpr int PB = 256;
// Fewest cells a stage tile owns over every supported shape (block 64, one
// cell per thread, compact tiles: 64 slots, 58 owned); sizes the tile tables.
constexpr int64_t MIN_OWN = 58;

struct Tile {
  int32_t inst;
  int32_t rec;  // index of the tile's result record (stage or plain table)
  int64_t c0;
  int64_t co;   // cell offset of the instance
  int64_t n;    // cells of the instance
};

// Start of a call: eta = h + b, reductions for the first step, shape bound of
// the prescribed map, initial masses.  Plain tiles: B items per tile over the
// n+1 nodes of each instance.
template <int B>
__global__ __launch_bounds__(B) void k_prep(Bufs bf, Consts cs, const Tile* __restrict__ tiles,
                                            const double* __restrict__ h_in,
                                            const double* __restrict__ wgiven) {
  __shared__ double red[(B / 64) * 8];
  const Tile tl = tiles[blockIdx.x];
  Inst& I = bf.inst[tl.inst];
  View v = make_view(bf, tl.inst, I);
  const int64_t j = tl.c0 + threadIdx.x;
  double speed = 0, minJ = INFINITY, maxJ = 0, hmin = INFINITY, me = 0, mb = 0, sabs = 0;
  if (j < v.n) {
    const int64_t g = v.co + j;
    // an analytic bottom: its projection onto the initial cells replaces b
    const double b = cs.bottom != BOT_ALE ? bottom_avg(cs, v.x[j], v.x[j + 1]) : bf.b[g];
    if (cs.bottom != BOT_ALE) bf.b[g] = b;
    const double h = h_in[g], m = bf.m[g];
    const double e = h + b;
    bf.eta[g] = e;
    const double J = v.x[j + 1] - v.x[j];
    const double hh = e - b;
    const double u = hh > cs.dry_eps ? m / hh : 0.0;
    speed = fabs(u) + fsqrt(cs.g * vmax(hh, 0.0));
    minJ = J; maxJ = J; hmin = hh;
    me = J * e; mb = J * b;
    if (!(J > 0.0)) atomicOr(&I.status, (int)SB_MESH);
    if (!isfinite(h) || !isfinite(m) || !isfinite(b)) atomicOr(&I.status, (int)SB_NONFINITE);
  }
  if (j <= v.n) {
    if (prescribed(cs.mesh)) {
      // the map's node amplitudes A S(xi); periodic meshes repeat node 0 at node n
      const double* xi = bf.xi + v.no;
      const int64_t jj = (cs.bc == BC_PERIODIC && j == v.n) ? 0 : j;
      const double S = mesh_shape(cs, xi[jj], xi[0], xi[v.n]);
      bf.w[v.no + j] = cs.mesh_A * S;
      sabs = fabs(mesh_shape(cs, xi[j], xi[0], xi[v.n]));
    } else if (cs.mesh == MESH_GIVEN && wgiven) {
      const double wv = wgiven[j];
      bf.w[v.no + j] = wv;
      sabs = fabs(wv);
    }
  }
  double rv[7] = {speed, minJ, maxJ, hmin, sabs, me, mb};
  const int op[7] = {0, 1, 0, 1, 0, 2, 2};
  block_reduce<B, 7>(rv, op, red);
  if (threadIdx.x == 0) {
    double* r = bf.prec + (int64_t)tl.rec * PREC;
#pragma unroll
    for (int k = 0; k < 7; ++k) r[k] = rv[k];
  }
}

template <int B>
__global__ __launch_bounds__(B) void k_wfluid(Bufs bf, Consts cs, const Tile* __restrict__ tiles) {
  __shared__ double su[B + 6], sv[B + 4], red[(B / 64) * 8];
  const Tile tl = tiles[blockIdx.x];
  Inst& I = bf.inst[tl.inst];
  if (!I.active) return;
  View v = make_view(bf, tl.inst, I);
  const double W = wfluid_tile<B>(bf, cs, v, tl.c0, su, sv, red);
  if (threadIdx.x == 0) bf.prec[(int64_t)tl.rec * PREC + 4] = W;
}

// Stage input of b under the L2 projection of eq. (3.16): the previous stage
// left P_b, D_b of the ALE bottom update in its stage buffers; they become the
// projection onto the mesh of stage s (x^n + tau w, tau = dt for stage 2 and
// dt / 2 for stage 3) times the stage width (the recurrence of eq. (3.15), as
// the stage kernel forms it) with D_b = 0, so the stage kernel's b is the
// projection.  Cells [c0, c0 + B) of one instance.
__device__ __forceinline__ void project_cell(const Bufs& bf, const Consts& cs, const View& v,
                                             int64_t j, int s, double dt, double wsc) {
  const double x0 = v.x[j], x1 = v.x[j + 1];
  const double w0 = bf.w[v.no + j] * wsc, w1 = bf.w[v.no + j + 1] * wsc;
  const double Jn = x1 - x0, dw = w1 - w0;
  const double J1 = Jn + dt * dw;
  const double J = (s == 2) ? J1 : 0.75 * Jn + 0.25 * (J1 + dt * dw);
  const double tau = (s == 2) ? dt : 0.5 * dt;
  const double bp = bottom_avg(cs, x0 + tau * w0, x1 + tau * w1);
  const int64_t g = v.co + j;
  double* P = (s == 2) ? bf.P0 : bf.P1;
  double* D = (s == 2) ? bf.D0 : bf.D1;
  P[2 * bf.S + g] = bp * J;
  D[2 * bf.S + g] = 0.0;
}

template <int B>
__global__ __launch_bounds__(B) void k_project(Bufs bf, Consts cs, const Tile* __restrict__ tiles,
                                               int s, int par) {
  const Tile tl = tiles[blockIdx.x];
  View v;
  v.n = tl.n;
  v.co = tl.co;
  v.no = tl.co + tl.inst;
  v.x = (par ? bf.xb : bf.xa) + v.no;
  v.xnew = (par ? bf.xa : bf.xb) + v.no;
  const Inst& I = bf.inst[tl.inst];
  if (!I.active) return;
  const int64_t j = tl.c0 + threadIdx.x;
  if (j < v.n) project_cell(bf, cs, v, j, s, I.dt, I.wscale);
}

// Result record of one stage tile.
__device__ __forceinline__ void publish_stage(const Bufs& bf, int rec, const StageRes& r) {
  double* d = bf.srec + (int64_t)rec * SREC;
  d[0] = r.alpha;
  d[1] = r.maxJ;
  d[2] = (double)r.ncls0;
  d[3] = (double)r.ncls1;
  d[4] = (double)r.ncls2;
  d[5] = (double)r.nlim;
  d[6] = (double)r.nneg;
  d[7] = (double)r.status;
  d[8] = r.akey;
}

// Stage s of one tile; par is the parity of the step (x^n in xa or xb).
// NOEXT: tiles of TB slots (TB - 6 owned cells) instead of TB + 4 slots.
template <int B, int CPT, bool NOEXT, int SCH>
__global__ __launch_bounds__(B) void k_stage(Bufs bf, Consts cs, const Tile* __restrict__ tiles,
                                             int s, int par) {
  constexpr int TB = B * CPT;
  constexpr int NR = NOEXT ? TB - 4 : TB;
  __shared__ SmemStage<B, CPT> sm;
  const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  View v;
  int st = 0;
  if (tile_inner<NOEXT ? TB : TB + 4>(tl.n, tl.c0)) {
    v.n = tl.n;
    v.co = tl.co;
    v.no = tl.co + tl.inst;
    v.x = (par ? bf.xb : bf.xa) + v.no;
    v.xnew = (par ? bf.xa : bf.xb) + v.no;
    const bool on =
        (s == 1) ? stage_load_direct<B, CPT, true, NOEXT>(bf, v, tl.inst, s, par, tl.c0, sm, st)
                 : stage_load_direct<B, CPT, false, NOEXT>(bf, v, tl.inst, s, par, tl.c0, sm, st);
    if (!on) return;
  } else {
    const Inst& I = bf.inst[tl.inst];
    if (!I.active) return;
    v = make_view(bf, tl.inst, I);
    load_tile_edge<B, CPT, NOEXT>(bf, cs, v, stage_scal(I, s), tl.c0, sm, st);
  }
  // read again after the two paths join, so that they stay scalar
  const StageScal sc = stage_scal_const(bf.inst, tl.inst, s);
  lds_sync();
  uint8_t* cl = bf.cls ? bf.cls + (int64_t)(s - 1) * bf.S + v.co : nullptr;
  const StageRes r = stage_compute<B, CPT, NR, SCH>(bf, cs, v, sc, tl.c0, sm, cl, st, (int)threadIdx.x);
  if (threadIdx.x == 0) publish_stage(bf, tl.rec, r);
}

template <int B>
// par is the parity of the step (x^n in xa or xb); the cell loads go out
// before the instance record is read (scalar loads through the constant
// address space: no instance record is written while this kernel runs).
__global__ __launch_bounds__(B) void k_final(Bufs bf, Consts cs, const Tile* __restrict__ tiles,
                                             int par) {
  __shared__ double red[(B / 64) * 8];
  const Tile tl = tiles[blockIdx.x];
  View v;
  v.n = tl.n;
  v.co = tl.co;
  v.no = tl.co + tl.inst;
  v.x = (par ? bf.xb : bf.xa) + v.no;
  v.xnew = (par ? bf.xa : bf.xb) + v.no;
  const int64_t j = tl.c0 + threadIdx.x;
  const bool cell = j < v.n;
  FinalRaw raw;
  if (cell) raw = final_load(bf, v, j);
  typedef const __attribute__((address_space(4))) Inst* cinst;
  const cinst I = (cinst)bf.inst + tl.inst;
  if (!I->active) return;
  int st = ((int)(I->steps & 1) != par) ? SB_SEQUENCE : 0;
  double speed = 0.0, minJ = INFINITY, maxJ = 0.0, hmin = INFINITY;
  if (cell)
    final_cell(bf, cs, v, j, raw, I->dt, I->alpha[2], I->wscale, speed, minJ, maxJ, hmin, st);
  const FinalRes r = final_reduce<B>(speed, minJ, maxJ, hmin, st, red);
  if (threadIdx.x == 0) {
    double* d = bf.prec + (int64_t)tl.rec * PREC;
    d[0] = r.speed; d[1] = r.minJ; d[2] = r.maxJ; d[3] = r.hmin;
    if (r.status) atomicOr(&bf.inst[tl.inst].status, r.status);  // rare: a failed cell
  }
}

// Per-instance scalar work between launches (one work-group, loops over instances).
__device__ void reset_step_slots(Inst& I) {
  I.r_speed = 0ull;
  I.r_minJ = dbits(INFINITY);
  I.r_maxJ = 0ull;
  I.r_W = 0ull;
}

// End of a step (first = false) and size of the next one.
__device__ void boundary_update(Inst& I, const Consts& cs, const Bufs& bf, int i, bool first) {
  if (!I.active) return;
  if (!first) {
    I.t = I.t + I.dt;
    I.steps += 1;
    I.dt_min = fmin(I.dt_min, I.dt);
    I.dt_max = fmax(I.dt_max, I.dt);
  }
  if (inst_done(I)) {
    I.active = 0;
    return;
  }
  // the frozen step sizes and the step log hold dts_stride entries per
  // instance: an instance that needs more steps stops with a status bit
  if ((bf.dts || bf.dt_log) && I.steps >= bf.dts_stride) {
    I.status |= SB_CAPACITY;
    I.active = 0;
    return;
  }
  const double dt = next_dt(I, cs, bf.dts, bf.dts_stride, i);
  // a step that cannot advance the clock ends the instance (no endless loops)
  if (!(dt > 0.0) || !(dt < INFINITY) || I.steps >= 100000000ll) {
    I.status |= SB_NONFINITE;
    I.active = 0;
    return;
  }
  I.dt = dt;
  if (prescribed(cs.mesh))
    I.wscale = (cs.flags & F_W_TANGENT) ? cs.mesh_omega * cos(cs.mesh_omega * I.t)
                                        : chord_factor(cs, I.t, dt);
  else
    I.wscale = 1.0;
  if (bf.dt_log) bf.dt_log[(int64_t)i * bf.dts_stride + I.steps] = dt;
  I.dx[0] = bitsd(I.r_maxJ);
  if (bf.dump.scal_next) {
    bf.dump.scal_next[(int64_t)i * 8 + 0] = I.t;
    bf.dump.scal_next[(int64_t)i * 8 + 1] = dt;
    bf.dump.scal_next[(int64_t)i * 8 + 5] = I.dx[0];
  }
  reset_step_slots(I);
}

// End of a step (first: start of a call): step results of each instance from
// its plain-tile records, then boundary_update.
struct PlainSum {
  double sp, mnJ, mxJ, hm, w4, me, mb;
};

__device__ __forceinline__ PlainSum reduce_plain_recs(const double* recs, int64_t k0, int64_t k1,
                                                      bool first, int lane) {
  double sp = 0.0, mnJ = INFINITY, mxJ = 0.0, hm = INFINITY, w4 = 0.0, me = 0.0, mb = 0.0;
  for (int64_t k = k0 + lane; k < k1; k += 64) {
    const double* q = recs + k * PREC;
    sp = fmax(sp, q[0]);
    mnJ = fmin(mnJ, q[1]);
    mxJ = fmax(mxJ, q[2]);
    hm = fmin(hm, q[3]);
    w4 = fmax(w4, q[4]);
    if (first) { me += q[5]; mb += q[6]; }
  }
  PlainSum r;
  r.sp = wave_max(sp); r.mnJ = wave_min(mnJ); r.mxJ = wave_max(mxJ); r.hm = wave_min(hm);
  r.w4 = wave_max(w4);
  r.me = first ? wave_sum(me) : 0.0;
  r.mb = first ? wave_sum(mb) : 0.0;
  return r;
}

__device__ __forceinline__ void put_plain_sum(double* q, const PlainSum& r) {
  q[0] = r.sp; q[1] = r.mnJ; q[2] = r.mxJ; q[3] = r.hm; q[4] = r.w4; q[5] = r.me; q[6] = r.mb;
}

__device__ __forceinline__ void apply_boundary(const Bufs& bf, const Consts& cs, int i,
                                               bool first, const PlainSum& r) {
  Inst& I = bf.inst[i];
  I.r_speed = dbits(r.sp);
  I.r_minJ = dbits(r.mnJ);
  I.r_maxJ = dbits(r.mxJ);
  const unsigned long long hk = okey(r.hm);
  if (hk < I.r_hmin) I.r_hmin = hk;
  if (first) {
    I.mass_eta0 = r.me;
    I.mass_b0 = r.mb;
    if (prescribed(cs.mesh)) I.smax = r.w4;
  }
  if (cs.mesh == MESH_GIVEN || cs.mesh == MESH_FLUID) I.r_W = dbits(r.w4);
  boundary_update(I, cs, bf, i, first);
}

// One wave per plain-record chunk; a chunk that holds a whole instance
// finishes it, others leave a partial result.
__global__ __launch_bounds__(256) void k_boundary(Bufs bf, Consts cs, int64_t nchunks, int first) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= nchunks) return;
  const RChunk ch = bf.pchunk[c];
  if (!bf.inst[ch.inst].active) return;
  const PlainSum r = reduce_plain_recs(bf.prec, ch.k0, ch.k1, first != 0, lane);
  if (lane == 0) {
    if (ch.whole) apply_boundary(bf, cs, ch.inst, first != 0, r);
    else put_plain_sum(bf.pcrec + c * PREC, r);
  }
}

// Second pass for instances split over several chunks (one wave per instance;
// the masses of a split instance are summed chunk by chunk, in chunk order).
__global__ __launch_bounds__(256) void k_boundary_split(Bufs bf, Consts cs, int first) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= bf.ninst) return;
  if (!bf.inst[i].active || bf.pcfirst[i + 1] - bf.pcfirst[i] < 2) return;
  const PlainSum r = reduce_plain_recs(bf.pcrec, bf.pcfirst[i], bf.pcfirst[i + 1], first != 0, lane);
  if (lane == 0) apply_boundary(bf, cs, i, first != 0, r);
}

// Stage results of an instance from records [k0, k1) (tile records, or the
// partial results of its chunks: same layout), reduced by one wave.
struct StageSum {
  double a, mj, ak;
  unsigned n0, n1, n2, nl, nn, stt;
};

__device__ __forceinline__ StageSum reduce_stage_recs(const double* recs, int64_t k0, int64_t k1,
                                                      bool keys, int lane) {
  StageSum r;
  double a = 0.0, mj = 0.0;
  unsigned n0 = 0u, n1 = 0u, n2 = 0u, nl = 0u, nn = 0u, stt = 0u;
  for (int64_t k = k0 + lane; k < k1; k += 64) {
    const double* q = recs + k * SREC;
    a = fmax(a, q[0]);
    mj = fmax(mj, q[1]);
    n0 += (unsigned)q[2]; n1 += (unsigned)q[3]; n2 += (unsigned)q[4];
    nl += (unsigned)q[5]; nn += (unsigned)q[6];
    stt |= (unsigned)q[7];
  }
  r.a = wave_max(a); r.mj = wave_max(mj);
  r.n0 = wave_usum(n0); r.n1 = wave_usum(n1); r.n2 = wave_usum(n2);
  r.nl = wave_usum(nl); r.nn = wave_usum(nn); r.stt = wave_or(stt);
  double ak = 1e300;
  if (keys) {
    // first face trace attaining alpha: smallest key among the records whose
    // LF speed is the reduced one
    for (int64_t k = k0 + lane; k < k1; k += 64) {
      const double* q = recs + k * SREC;
      if (q[0] == r.a) ak = fmin(ak, q[8]);
    }
    ak = wave_min(ak);
  }
  r.ak = ak;
  return r;
}

__device__ __forceinline__ void put_stage_sum(double* q, const StageSum& r) {
  q[0] = r.a; q[1] = r.mj;
  q[2] = (double)r.n0; q[3] = (double)r.n1; q[4] = (double)r.n2;
  q[5] = (double)r.nl; q[6] = (double)r.nn; q[7] = (double)r.stt; q[8] = r.ak;
}

__device__ __forceinline__ void apply_stage(const Bufs& bf, int i, int s, const StageSum& r) {
  Inst& I = bf.inst[i];
  I.alpha[s - 1] = r.a;
  if (s < 3) I.dx[s] = r.mj;
  I.n_class[0] += r.n0; I.n_class[1] += r.n1; I.n_class[2] += r.n2;
  I.n_limited += r.nl; I.n_negweight += r.nn;
  if (r.stt) I.status |= (int)r.stt;
  if (bf.dump.scal) {
    bf.dump.scal[(int64_t)i * 8 + 1 + s] = I.alpha[s - 1];
    if (s < 3) bf.dump.scal[(int64_t)i * 8 + 5 + s] = I.dx[s];
  }
  if (bf.dump.akey) bf.dump.akey[(int64_t)(s - 1) * bf.ninst + i] = r.ak;
}

// After stage s: one wave per record chunk; a chunk that holds a whole
// instance sets the instance's stage results, others leave a partial result.
__global__ __launch_bounds__(256) void k_after_stage(Bufs bf, int64_t nchunks, int s) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= nchunks) return;
  const RChunk ch = bf.schunk[c];
  if (!bf.inst[ch.inst].active) return;
  const StageSum r = reduce_stage_recs(bf.srec, ch.k0, ch.k1, bf.dump.akey != nullptr, lane);
  if (lane == 0) {
    if (ch.whole) apply_stage(bf, ch.inst, s, r);
    else put_stage_sum(bf.screc + c * SREC, r);
  }
}

// Second pass for instances split over several chunks (one wave per instance).
__global__ __launch_bounds__(256) void k_after_stage_split(Bufs bf, int s) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= bf.ninst) return;
  if (!bf.inst[i].active || bf.scfirst[i + 1] - bf.scfirst[i] < 2) return;
  const StageSum r =
      reduce_stage_recs(bf.screc, bf.scfirst[i], bf.scfirst[i + 1], bf.dump.akey != nullptr, lane);
  if (lane == 0) apply_stage(bf, i, s, r);
}

// End of a call: h = eta - b, final nodes back into the caller's array, masses.
template <int B>
__global__ __launch_bounds__(B) void k_finish(Bufs bf, Consts cs, const Tile* __restrict__ tiles,
                                              double* __restrict__ h_out,
                                              double* __restrict__ x_out) {
  __shared__ double red[(B / 64) * 8];
  const Tile tl = tiles[blockIdx.x];
  Inst& I = bf.inst[tl.inst];
  View v = make_view(bf, tl.inst, I);
  const int64_t j = tl.c0 + threadIdx.x;
  double me = 0, mb = 0;
  if (j <= v.n) x_out[v.no + j] = v.x[j];
  if (j < v.n) {
    const int64_t g = v.co + j;
    const double e = bf.eta[g], b = bf.b[g];
    h_out[g] = e - b;
    const double J = v.x[j + 1] - v.x[j];
    me = J * e;
    mb = J * b;
  }
  double rv[2] = {me, mb};
  const int op[2] = {2, 2};
  block_reduce<B, 2>(rv, op, red);
  if (threadIdx.x == 0) {
    bf.prec[(int64_t)tl.rec * PREC + 5] = rv[0];
    bf.prec[(int64_t)tl.rec * PREC + 6] = rv[1];
  }
}

// Final masses of each instance from the plain-tile records of k_finish.
__global__ __launch_bounds__(256) void k_masses(Bufs bf) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= bf.ninst) return;
  double me = 0.0, mb = 0.0;
  for (int64_t k = bf.pfirst[i] + lane; k < bf.pfirst[i + 1]; k += 64) {
    me += bf.prec[k * PREC + 5];
    mb += bf.prec[k * PREC + 6];
  }
  me = wave_sum(me);
  mb = wave_sum(mb);
  if (lane == 0) {
    bf.inst[i].mass_eta = me;
    bf.inst[i].mass_b = mb;
  }
}

__global__ void k_zero_u32(unsigned* p) { *p = 0u; }

// Number of active instances, and (act non-NULL) one activity byte per instance.
__global__ __launch_bounds__(1024) void k_count_active(Bufs bf, int* __restrict__ n_active,
                                                      uint8_t* __restrict__ act) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int c = 0;
  for (int i = threadIdx.x; i < bf.ninst; i += blockDim.x) {
    const int a = bf.inst[i].active ? 1 : 0;
    c += a;
    if (act) act[i] = (uint8_t)a;
  }
  atomicAdd(&cnt, c);
  __syncthreads();
  if (threadIdx.x == 0) *n_active = cnt;
}

// Persistent engine: one launch for the whole batch.  A work-group of B
// threads runs the stage tiles of its instance one after the other, CPT cells
// per thread (tiles of B * CPT cells, B * CPT - 2 owned).
template <int B, int CPT, int SCH>
__global__ __launch_bounds__(B) void k_persistent(Bufs bf, Consts cs,
                                                  const int32_t* __restrict__ order,
                                                  unsigned* __restrict__ queue,
                                                  int32_t steps_limit) {
  __shared__ SmemStage<B, CPT> sm;
  __shared__ Inst sI;
  __shared__ int s_idx;
  __shared__ double su[B + 6], sv[B + 4], red[(B / 64) * 8];
  for (;;) {
    if (threadIdx.x == 0) s_idx = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int qi = s_idx;
    if (qi >= bf.ninst) break;
    const int i = order[qi];
    if (threadIdx.x == 0) sI = bf.inst[i];
    __syncthreads();
    int launched = 0;
    while (sI.active && (steps_limit <= 0 || launched < steps_limit)) {
      const View v = make_view(bf, i, sI);
      const double dt = sI.dt;
      unsigned long long c_cls[3] = {0, 0, 0}, c_lim = 0, c_neg = 0;
      int st = 0;
      for (int s = 1; s <= 3; ++s) {
        const StageScal sc = stage_scal(sI, s);
        double amax = 0.0, jmax = 0.0;
        for (int64_t c0 = 0; c0 < v.n; c0 += B * CPT - 2) {
          StageRes r = stage_tile<B, CPT, SCH>(bf, cs, v, sc, c0, sm, nullptr);
          amax = fmax(amax, r.alpha);
          jmax = fmax(jmax, r.maxJ);
          c_cls[0] += r.ncls0; c_cls[1] += r.ncls1; c_cls[2] += r.ncls2;
          c_lim += r.nlim; c_neg += r.nneg;
          st |= r.status;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
          sI.alpha[s - 1] = amax;
          if (s < 3) sI.dx[s] = jmax;
        }
        if (cs.bottom != BOT_ALE && s < 3)
          for (int64_t j = threadIdx.x; j < v.n; j += B) project_cell(bf, cs, v, j, s + 1, dt, sI.wscale);
        __syncthreads();
      }
      double fsp = 0.0, fminJ = INFINITY, fmaxJ = 0.0, fhmin = INFINITY;
      for (int64_t c0 = 0; c0 < v.n; c0 += B) {
        FinalRes r = final_tile<B>(bf, cs, v, dt, sI.alpha[2], sI.wscale, c0, red);
        fsp = fmax(fsp, r.speed);
        fminJ = fmin(fminJ, r.minJ);
        fmaxJ = fmax(fmaxJ, r.maxJ);
        fhmin = fmin(fhmin, r.hmin);
        st |= r.status;
      }
      __syncthreads();
      double Wf = 0.0;
      if (cs.mesh == MESH_FLUID) {
        // the node speeds of the next step follow the new state
        View vn = v;
        vn.x = v.xnew;
        for (int64_t k0 = 0; k0 <= v.n; k0 += B)
          Wf = fmax(Wf, wfluid_tile<B>(bf, cs, vn, k0, su, sv, red));
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        sI.n_class[0] += c_cls[0];
        sI.n_class[1] += c_cls[1];
        sI.n_class[2] += c_cls[2];
        sI.n_limited += c_lim;
        sI.n_negweight += c_neg;
        sI.status |= st;
        sI.r_speed = dbits(fsp);
        sI.r_minJ = dbits(fminJ);
        sI.r_maxJ = dbits(fmaxJ);
        if (cs.mesh == MESH_FLUID) sI.r_W = dbits(Wf);
        const unsigned long long hk = okey(fhmin);
        if (hk < sI.r_hmin) sI.r_hmin = hk;
        boundary_update(sI, cs, bf, i, false);
      }
      __syncthreads();
      ++launched;
    }
    if (threadIdx.x == 0) bf.inst[i] = sI;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// adjoint driver kernels
// ---------------------------------------------------------------------------
// Mean depth at the final time in the cell containing each gauge (first cell
// whose right node lies beyond the gauge, at most the last cell).
__global__ void k_gauge(Bufs bf, int64_t ngauge, const double* __restrict__ gx,
                        double* __restrict__ gh, int64_t* __restrict__ gcell) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)bf.ninst * ngauge) return;
  const int i = (int)(id / ngauge);
  const Inst& I = bf.inst[i];
  const View v = make_view(bf, i, I);
  const double xg = gx[id];
  int64_t lo = 0, hi = v.n - 1;  // smallest c with xg < x[c+1], capped at n-1
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (xg < v.x[mid + 1]) hi = mid; else lo = mid + 1;
  }
  const int64_t g = v.co + lo;
  gcell[id] = g;
  if (gh) gh[id] = bf.eta[g] - bf.b[g];
}

// Seed of the reverse sweep: each gauge adds its cotangent to its cell's eta and
// b adjoints.  One thread per instance walks the instance's gauges in order, so
// gauges sharing a cell add in a fixed order (instances own disjoint cells).
__global__ void k_gauge_seed(int64_t ninst, int64_t ngauge, int64_t S,
                             const int64_t* __restrict__ gcell, const double* __restrict__ gbar,
                             double* __restrict__ lam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  for (int64_t k = i * ngauge; k < (i + 1) * ngauge; ++k) {
    const int64_t g = gcell[k];
    lam[g] += gbar[k];           // d hbar / d eta
    lam[2 * S + g] -= gbar[k];   // d hbar / d b
  }
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) p[id] = v;
}

// dL/dh0 = lambda_eta, dL/dhu0 = lambda_hu, dL/db0 = lambda_b + lambda_eta (eta = h + b)
__global__ void k_adj_out(int64_t S, const double* __restrict__ lam, double* __restrict__ dh,
                          double* __restrict__ dhu, double* __restrict__ db) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= S) return;
  dh[g] = lam[g];
  dhu[g] = lam[S + g];
  db[g] = lam[2 * S + g] + lam[g];
}

// Record (t, dt, dx_0) of the first step of a recomputed segment.
__global__ void k_seed_scal(Bufs bf, double* __restrict__ scal) {
  for (int i = threadIdx.x; i < bf.ninst; i += blockDim.x) {
    const Inst& I = bf.inst[i];
    scal[(int64_t)i * 8 + 0] = I.t;
    scal[(int64_t)i * 8 + 1] = I.dt;
    scal[(int64_t)i * 8 + 5] = I.dx[0];
  }
}

// ============================================================================
// host side
// ============================================================================
namespace {

thread_local std::string g_err;

alew_status fail(alew_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                             \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(ALEW_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct GraphKey {
  std::vector<char> bytes;
  bool operator==(const GraphKey& o) const { return bytes == o.bytes; }
};

}  // namespace

// Message setter for the other translation units of the library (the 2D
// entry points): same thread-local message as alew_last_error() returns.
__attribute__((visibility("hidden"))) alew_status alew_set_error(alew_status s, const char* msg) {
  return fail(s, msg);
}

struct alew_ctx {
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // capture stream for graphs
  int64_t max_cells = 0, max_inst = 0;
  double *eta = nullptr, *P0 = nullptr, *D0 = nullptr, *P1 = nullptr, *D1 = nullptr;
  double *w = nullptr, *xa = nullptr, *xb = nullptr;
  Inst* inst = nullptr;
  Inst* inst_h = nullptr;  // pinned
  int64_t* cell_off_d = nullptr;
  int32_t* order_d = nullptr;
  unsigned* queue_d = nullptr;
  int* nactive_d = nullptr;
  int* nactive_h = nullptr;  // pinned
  double* dt1_d = nullptr;   // step size of alew_step
  double* dt1_h = nullptr;   // pinned staging
  Tile* tiles_stage_d = nullptr;
  Tile* tiles_plain_d = nullptr;
  Tile* tiles_edge_d = nullptr;   // stage tiles touching an instance end
  Tile* tiles_inner_d = nullptr;  // ghost-free stage tiles
  double* srec = nullptr;          // per-tile stage results
  double* prec = nullptr;          // per-tile step results
  int64_t* sfirst_d = nullptr;     // [max_inst+1] first stage / plain tile of each instance
  int64_t* pfirst_d = nullptr;
  int64_t* scfirst_d = nullptr;    // [max_inst+1] first stage / plain record chunk
  int64_t* pcfirst_d = nullptr;
  RChunk* schunk_d = nullptr;      // record chunks (at most one per tile)
  RChunk* pchunk_d = nullptr;
  double* screc = nullptr;         // partial results of split instances
  double* pcrec = nullptr;
  int64_t n_schunks = 0, n_pchunks = 0;
  uint8_t* act_d = nullptr;        // [max_inst] activity bytes (k_count_active)
  uint8_t* act_h = nullptr;        // pinned copy
  int64_t tables_ninst = 0;        // instances with tiles in the current tables
  int64_t tables_cells = 0;        // their cells
  bool tables_masked = false;      // tables hold only the instances active at a check
  std::vector<uint8_t> cached_mask;
  bool split_s = false, split_p = false;  // some instance has several chunks
  int64_t cap_stage = 0, cap_plain = 0;  // tile table capacities (set in alew_create)
  int64_t n_tiles_edge = 0, n_tiles_inner = 0;
  int n_cu = 0;
  std::vector<int64_t> cell_off_h;  // cached batch layout
  int cached_B = 0, cached_TB = 0;
  bool cached_noext = false;
  bool tiles_noext = false;  // stage tiles of TB slots (TB - 6 owned): compact tiles
  int64_t n_tiles_stage = 0, n_tiles_plain = 0;
  alew_launch launch{0, 0, 0, 1, 0, 0};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around the compute launches of a call
  // per-kernel timing (alew_set_kernel_timing): event pairs around launches
  int ktime_on = 0;
  bool ktime_rec = false;  // recording in the current call
  std::vector<hipEvent_t> kt_ev;
  std::vector<int> kt_kind;
  std::vector<double> kt_cells;
  size_t kt_used = 0;
  // adjoint workspace (allocated by the first alew_adjoint call, grown on demand)
  double* adj_ws = nullptr;
  size_t adj_ws_bytes = 0;
  double last_ms = 0.0;
  int64_t last_launches = 0;
  // graph of a 2-step sequence (stage-launch engine)
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  GraphKey gkey;
};

namespace {

// Scheme of the stage kernels from the flags.
int scheme_of(const Consts& cs) {
  if (cs.flags & F_HYDROSTATIC) return SCH_HYDRO;
  if (cs.flags & F_NONWB) return SCH_NONWB;
  return SCH_SPECIAL;
}

Consts make_consts(const alew_params* p) {
  Consts c;
  c.g = p->g; c.cfl = p->cfl; c.weno_eps = p->weno_eps; c.pp_eps = p->pp_eps;
  c.mesh_A = p->mesh_A; c.mesh_k = p->mesh_k; c.mesh_omega = p->mesh_omega; c.dry_eps = p->dry_eps;
  c.bc = p->bc; c.mesh = p->mesh; c.flags = p->flags; c.bottom = p->bottom;
  for (int k = 0; k < 4; ++k) c.bp[k] = p->bottom_p[k];
  return c;
}

alew_status check_params(const alew_params* p) {
  if (!p) return fail(ALEW_E_ARG, "params is NULL");
  if (!(p->g > 0) || !(p->cfl > 0) || !(p->weno_eps > 0) || !(p->pp_eps >= 0) || !(p->dry_eps >= 0))
    return fail(ALEW_E_ARG, "g, cfl, weno_eps must be > 0 and pp_eps, dry_eps >= 0");
  if (p->bc < 0 || p->bc > 2) return fail(ALEW_E_ARG, "unknown boundary type");
  if (p->mesh < 0 || p->mesh > ALEW_MESH_ALIGNED) return fail(ALEW_E_ARG, "unknown mesh mode");
  if (prescribed(p->mesh) && !(p->mesh_omega == p->mesh_omega))
    return fail(ALEW_E_ARG, "mesh_omega is NaN");
  if (p->mesh == ALEW_MESH_ALIGNED && !(std::isfinite(p->bottom_p[1]) && std::isfinite(p->bottom_p[2])))
    return fail(ALEW_E_ARG, "the ALIGNED mesh needs finite roots bottom_p[1], bottom_p[2]");
  if ((p->flags & ALEW_F_HYDROSTATIC) && (p->flags & ALEW_F_NONWB))
    return fail(ALEW_E_ARG, "HYDROSTATIC and NONWB select different schemes");
  if (p->bottom < 0 || p->bottom > ALEW_BOTTOM_PARABOLA) return fail(ALEW_E_ARG, "unknown bottom");
  if ((p->bottom == ALEW_BOTTOM_BUMP || p->bottom == ALEW_BOTTOM_PARABOLA) && !(p->bottom_p[1] > 0))
    return fail(ALEW_E_ARG, "bottom_p[1] must be > 0 for BUMP and PARABOLA");
  return ALEW_OK;
}

// Work-group size: block 0 = 64 for the stage-launch engine (one-wave tiles,
// no barrier across SIMDs), 256 for the persistent engine.
int pick_block(const alew_ctx* c, int engine) {
  const int b = c->launch.block;
  if (b == 64 || b == 128 || b == 256 || b == 512) return b;
  return engine == 1 ? 256 : 64;
}

// Cells per thread of the stage-launch engine (block 512 runs one; 0 = two
// for block 64, else one).
int pick_cpt(const alew_ctx* c, int B) {
  const int k = c->launch.cells_per_thread;
  if (B > 256) return 1;
  if (k == 0) return B == 64 ? 2 : 1;
  return k == 2 ? 2 : 1;
}

// (Re)build the tile tables for a batch layout, block size B and stage tile
// width TB: TB + 4 stencil slots and TB - 2 owned cells per stage tile, or
// with noext TB slots and TB - 6 owned cells; B items per plain tile.  With a
// host mask (one byte per instance) only the instances marked active get
// tiles; the others have empty record ranges.
alew_status build_tiles(alew_ctx* c, const int64_t* cell_off, int64_t ninst, int B, int TB,
                        bool noext, const uint8_t* mask = nullptr) {
  std::vector<int64_t> off(cell_off, cell_off + ninst + 1);
  std::vector<uint8_t> mk;
  if (mask) mk.assign(mask, mask + ninst);
  if (off == c->cell_off_h && c->cached_B == B && c->cached_TB == TB && c->cached_noext == noext &&
      mk == c->cached_mask)
    return ALEW_OK;
  const int64_t own = noext ? TB - 6 : TB - 2;
  const int64_t NS = noext ? TB : TB + 4;
  // stage tiles carry their index in the full stage table as record index (the
  // end-tile and ghost-free tables are subsets of it); plain tiles their own
  std::vector<Tile> ts, tp, te, tin;
  std::vector<int64_t> sfirst(ninst + 1, 0), pfirst(ninst + 1, 0);
  int64_t tab_ninst = 0, tab_cells = 0;
  for (int64_t i = 0; i < ninst; ++i) {
    const int64_t n = off[i + 1] - off[i];
    sfirst[i] = (int64_t)ts.size();
    pfirst[i] = (int64_t)tp.size();
    if (mask && !mask[i]) continue;
    tab_ninst += 1;
    tab_cells += n;
    for (int64_t c0 = 0; c0 < n; c0 += own) {
      const Tile tl{(int32_t)i, (int32_t)ts.size(), c0, off[i], n};
      ts.push_back(tl);
      // same test as tile_inner() on the device
      const bool inner = c0 >= 3 && c0 + NS - 4 < n && n < (int64_t(1) << 28);
      (inner ? tin : te).push_back(tl);
    }
    for (int64_t c0 = 0; c0 <= n; c0 += B)
      tp.push_back(Tile{(int32_t)i, (int32_t)tp.size(), c0, off[i], n});
  }
  sfirst[ninst] = (int64_t)ts.size();
  pfirst[ninst] = (int64_t)tp.size();
  if (ts.size() >= (size_t)INT32_MAX || tp.size() >= (size_t)INT32_MAX)
    return fail(ALEW_E_ARG, "too many tiles");
  // the tables were sized in alew_create for the smallest stage tile (no
  // allocation here); the caller's capacity checks keep them within bounds
  if ((int64_t)ts.size() > c->cap_stage || (int64_t)tp.size() > c->cap_plain)
    return fail(ALEW_E_ARG, "internal: tile tables exceed the context capacity");
  // record chunks: up to RCHUNK consecutive records of one instance
  auto chunk = [&](const std::vector<int64_t>& first, std::vector<RChunk>& out,
                   std::vector<int64_t>& cfirst, bool& split) {
    split = false;
    for (int64_t i = 0; i < ninst; ++i) {
      cfirst[i] = (int64_t)out.size();
      const int64_t a = first[i], e = first[i + 1];
      const int32_t whole = e - a <= RCHUNK ? 1 : 0;
      if (!whole) split = true;
      for (int64_t k0 = a; k0 < e; k0 += RCHUNK)
        out.push_back(RChunk{(int32_t)i, whole, k0, std::min<int64_t>(k0 + RCHUNK, e)});
    }
    cfirst[ninst] = (int64_t)out.size();
  };
  std::vector<RChunk> sch, pch;
  std::vector<int64_t> scfirst(ninst + 1, 0), pcfirst(ninst + 1, 0);
  bool split_s = false, split_p = false;
  chunk(sfirst, sch, scfirst, split_s);
  chunk(pfirst, pch, pcfirst, split_p);
  HIPCHK(hipMemcpyAsync(c->scfirst_d, scfirst.data(), scfirst.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->pcfirst_d, pcfirst.data(), pcfirst.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->schunk_d, sch.data(), sch.size() * sizeof(RChunk), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->pchunk_d, pch.data(), pch.size() * sizeof(RChunk), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->sfirst_d, sfirst.data(), sfirst.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->pfirst_d, pfirst.data(), pfirst.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->tiles_stage_d, ts.data(), ts.size() * sizeof(Tile), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->tiles_plain_d, tp.data(), tp.size() * sizeof(Tile), hipMemcpyHostToDevice, c->stream));
  if (!te.empty())
    HIPCHK(hipMemcpyAsync(c->tiles_edge_d, te.data(), te.size() * sizeof(Tile), hipMemcpyHostToDevice, c->stream));
  if (!tin.empty())
    HIPCHK(hipMemcpyAsync(c->tiles_inner_d, tin.data(), tin.size() * sizeof(Tile), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->cell_off_d, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  // largest work first for the persistent queue
  std::vector<int32_t> order(ninst);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return (off[a + 1] - off[a]) > (off[b + 1] - off[b]);
  });
  HIPCHK(hipMemcpyAsync(c->order_d, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->cell_off_h = off;
  c->cached_B = B;
  c->cached_TB = TB;
  c->cached_noext = noext;
  c->cached_mask = mk;
  c->tiles_noext = noext;
  c->tables_ninst = tab_ninst;
  c->tables_cells = tab_cells;
  c->tables_masked = mask != nullptr;
  c->n_tiles_stage = (int64_t)ts.size();
  c->n_tiles_plain = (int64_t)tp.size();
  c->n_tiles_edge = (int64_t)te.size();
  c->n_tiles_inner = (int64_t)tin.size();
  c->n_schunks = (int64_t)sch.size();
  c->n_pchunks = (int64_t)pch.size();
  c->split_s = split_s;
  c->split_p = split_p;
  if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
  if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
  return ALEW_OK;
}

Bufs make_bufs(alew_ctx* c, int64_t S, int64_t ninst, double* hu, double* b, const double* xi,
               uint8_t* cls, const double* dts, double* dt_log, int64_t dts_stride,
               uint32_t* ccount = nullptr, uint64_t* csig = nullptr) {
  Bufs bf;
  bf.cell_off = c->cell_off_d;
  bf.eta = c->eta; bf.m = hu; bf.b = b;
  bf.xa = c->xa; bf.xb = c->xb; bf.xi = xi; bf.w = c->w;
  bf.P0 = c->P0; bf.D0 = c->D0; bf.P1 = c->P1; bf.D1 = c->D1;
  bf.cls = cls; bf.inst = c->inst;
  bf.ccount = ccount; bf.csig = (unsigned long long*)csig;
  bf.dts = dts; bf.dt_log = dt_log; bf.dts_stride = dts_stride;
  bf.S = S; bf.ninst = (int32_t)ninst; bf.pad = 0;
  bf.srec = c->srec; bf.prec = c->prec;
  bf.sfirst = c->sfirst_d; bf.pfirst = c->pfirst_d;
  bf.schunk = c->schunk_d; bf.pchunk = c->pchunk_d;
  bf.scfirst = c->scfirst_d; bf.pcfirst = c->pcfirst_d;
  bf.screc = c->screc; bf.pcrec = c->pcrec;
  bf.dump = Dump{nullptr, nullptr, nullptr, nullptr, nullptr};
  return bf;
}

// Event pair around a launch for per-kernel timing (kind 1: epilogue; 2, 3, 4:
// the stage launch of RK stage 1, 2, 3).
int kt_begin(alew_ctx* c, hipStream_t st, int kind, double cells) {
  if (!c->ktime_rec) return -1;
  const size_t k = c->kt_used;
  if (2 * k + 2 > c->kt_ev.size()) {
    for (int q = 0; q < 2; ++q) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      c->kt_ev.push_back(e);
    }
    c->kt_kind.push_back(0);
    c->kt_cells.push_back(0.0);
  }
  c->kt_kind[k] = kind;
  c->kt_cells[k] = cells;
  (void)hipEventRecord(c->kt_ev[2 * k], st);
  c->kt_used = k + 1;
  return (int)k;
}
void kt_end(alew_ctx* c, hipStream_t st, int k) {
  if (k >= 0) (void)hipEventRecord(c->kt_ev[2 * (size_t)k + 1], st);
}

// Per-instance reductions of the stage and plain tile records: a wave per
// record chunk, and a second pass only when some instance is split.
void launch_after_stage(const alew_ctx* c, const Bufs& bf, hipStream_t st, int s) {
  hipLaunchKernelGGL(k_after_stage, dim3((unsigned)((c->n_schunks + 3) / 4)), dim3(256), 0, st, bf,
                     c->n_schunks, s);
  if (c->split_s)
    hipLaunchKernelGGL(k_after_stage_split, dim3((unsigned)((bf.ninst + 3) / 4)), dim3(256), 0, st,
                       bf, s);
}

void launch_boundary(const alew_ctx* c, const Bufs& bf, const Consts& cs, hipStream_t st,
                     int first) {
  hipLaunchKernelGGL(k_boundary, dim3((unsigned)((c->n_pchunks + 3) / 4)), dim3(256), 0, st, bf, cs,
                     c->n_pchunks, first);
  if (c->split_p)
    hipLaunchKernelGGL(k_boundary_split, dim3((unsigned)((bf.ninst + 3) / 4)), dim3(256), 0, st, bf,
                       cs, first);
}

template <int B, int CPT>
void launch_step_seq(alew_ctx* c, const Bufs& bf, const Consts& cs, hipStream_t st, int64_t step) {
  const int par = (int)(step & 1);
  const dim3 gs((unsigned)c->n_tiles_stage), gp((unsigned)c->n_tiles_plain);
  const int sch = scheme_of(cs);
  for (int s = 1; s <= 3; ++s) {
    const int kt = kt_begin(c, st, 1 + s, (double)c->tables_cells);
#define ALEW_STAGE(NX, SC)                                                                      \
  hipLaunchKernelGGL((k_stage<B, CPT, NX, SC>), gs, dim3(B), 0, st, bf, cs, c->tiles_stage_d, s, par)
    if (cs.flags & F_SPLIT) {
      // split negative weights: the automatic tile shape only (the driver
      // forces it), so that no other shape carries the split's registers
      if constexpr (B == 64 && CPT == 2) {
        if (sch == SCH_HYDRO) ALEW_STAGE(false, SCH_HYDRO | SCH_SPLIT);
        else if (sch == SCH_NONWB) ALEW_STAGE(false, SCH_NONWB | SCH_SPLIT);
        else ALEW_STAGE(false, SCH_SPECIAL | SCH_SPLIT);
      }
    } else if (c->tiles_noext) {
      if (sch == SCH_HYDRO) ALEW_STAGE(true, SCH_HYDRO);
      else if (sch == SCH_NONWB) ALEW_STAGE(true, SCH_NONWB);
      else ALEW_STAGE(true, SCH_SPECIAL);
    } else {
      if (sch == SCH_HYDRO) ALEW_STAGE(false, SCH_HYDRO);
      else if (sch == SCH_NONWB) ALEW_STAGE(false, SCH_NONWB);
      else ALEW_STAGE(false, SCH_SPECIAL);
    }
#undef ALEW_STAGE
    kt_end(c, st, kt);
    launch_after_stage(c, bf, st, s);
    if (cs.bottom != BOT_ALE && s < 3)
      hipLaunchKernelGGL(k_project<PB>, dim3((unsigned)c->n_tiles_plain), dim3(PB), 0, st, bf, cs,
                         c->tiles_plain_d, s + 1, par);
  }
  const int kf = kt_begin(c, st, 1, (double)c->tables_cells);
  hipLaunchKernelGGL(k_final<PB>, gp, dim3(PB), 0, st, bf, cs, c->tiles_plain_d, par);
  kt_end(c, st, kf);
  if (cs.mesh == MESH_FLUID)
    hipLaunchKernelGGL(k_wfluid<PB>, gp, dim3(PB), 0, st, bf, cs, c->tiles_plain_d);
  launch_boundary(c, bf, cs, st, 0);
}

// Step sequence for a run-time tile shape (block B, CPT cells per thread).
void launch_step_shape(alew_ctx* c, int B, int CPT, const Bufs& bf, const Consts& cs,
                       hipStream_t st, int64_t step) {
  if (B == 64)
    CPT == 2 ? launch_step_seq<64, 2>(c, bf, cs, st, step) : launch_step_seq<64, 1>(c, bf, cs, st, step);
  else if (B == 128)
    CPT == 2 ? launch_step_seq<128, 2>(c, bf, cs, st, step) : launch_step_seq<128, 1>(c, bf, cs, st, step);
  else if (B == 512)
    launch_step_seq<512, 1>(c, bf, cs, st, step);
  else
    CPT == 2 ? launch_step_seq<256, 2>(c, bf, cs, st, step) : launch_step_seq<256, 1>(c, bf, cs, st, step);
}

GraphKey make_key(const Bufs& bf, const Consts& cs, int B, int CPT, const alew_ctx* c) {
  GraphKey k;
  auto put = [&](const void* p, size_t n) {
    const char* q = (const char*)p;
    k.bytes.insert(k.bytes.end(), q, q + n);
  };
  put(&bf, sizeof(bf));
  put(&cs, sizeof(cs));
  put(&B, sizeof(B));
  put(&CPT, sizeof(CPT));
  put(&c->tiles_noext, sizeof(bool));
  put(&c->n_tiles_stage, sizeof(int64_t));
  put(&c->n_tiles_plain, sizeof(int64_t));
  put(&c->n_schunks, sizeof(int64_t));
  put(&c->n_pchunks, sizeof(int64_t));
  put(&c->split_s, sizeof(bool));
  put(&c->split_p, sizeof(bool));
  put(&c->tables_cells, sizeof(int64_t));
  return k;
}

template <int B, int CPT>
alew_status run_stage_engine(alew_ctx* c, const Bufs& bf, const Consts& cs, int64_t max_iters) {
  const bool use_graph = c->launch.use_graph != 0 && !c->ktime_on;
  c->kt_used = 0;
  c->ktime_rec = c->ktime_on != 0;
  const int check_every = 8;  // 2-step graphs between host checks
  auto ensure_graph = [&]() -> hipError_t {
    if (!use_graph) return hipSuccess;
    GraphKey key = make_key(bf, cs, B, CPT, c);
    if (c->gexec && key == c->gkey) return hipSuccess;
    if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
    if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    // the graph starts at an even step and holds two
    launch_step_seq<B, CPT>(c, bf, cs, c->cap_stream, 0);
    launch_step_seq<B, CPT>(c, bf, cs, c->cap_stream, 1);
    e = hipStreamEndCapture(c->cap_stream, &c->graph);
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return e;
    c->gkey = key;
    return hipSuccess;
  };
  HIPCHK(ensure_graph());
  int64_t it = 0;
  c->last_launches = 0;
  if (c->ev0) HIPCHK(hipEventRecord(c->ev0, c->stream));
  while (it < max_iters) {
    for (int k = 0; k < check_every && it < max_iters; ++k) {
      if (use_graph) {
        HIPCHK(hipGraphLaunch(c->gexec, c->stream));
        it += 2;
      } else {
        launch_step_seq<B, CPT>(c, bf, cs, c->stream, it);
        it += 1;
      }
      c->last_launches += 1;
    }
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(1024), 0, c->stream, bf, c->nactive_d, c->act_d);
    HIPCHK(hipMemcpyAsync(c->nactive_h, c->nactive_d, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t na = *c->nactive_h;
    if (na == 0) break;
    // once half of the instances in the tile tables are done, the tables keep
    // only the active ones: a done instance's tiles would still load their
    // stencils before reading that the instance is done
    if (2 * na <= c->tables_ninst) {
      HIPCHK(hipMemcpyAsync(c->act_h, c->act_d, (size_t)bf.ninst, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      alew_status ts = build_tiles(c, c->cell_off_h.data(), bf.ninst, c->cached_B, c->cached_TB,
                                   c->cached_noext, c->act_h);
      if (ts != ALEW_OK) return ts;
      HIPCHK(ensure_graph());
    }
  }
  c->ktime_rec = false;
  c->last_ms = 0.0;
  if (c->ev0 && c->ev1) {  // a context without events (the allocation-free step) skips timing
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    HIPCHK(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_ms = ms;
  }
  return ALEW_OK;
}

template <int B, int CPT>
alew_status run_persistent(alew_ctx* c, const Bufs& bf, const Consts& cs, int64_t ninst) {
  int dev = 0, ncu = 0, per_cu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int sch = scheme_of(cs);
  if (sch == SCH_HYDRO)
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<B, CPT, SCH_HYDRO>, B, 0));
  else if (sch == SCH_NONWB)
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<B, CPT, SCH_NONWB>, B, 0));
  else
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<B, CPT, SCH_SPECIAL>, B, 0));
  int64_t grid = (int64_t)std::max(1, ncu) * std::max(1, per_cu);
  grid = std::min<int64_t>(grid, ninst);
  const int limit = c->launch.steps_per_launch;
  c->last_launches = 0;
  double total = 0.0;
  for (;;) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, c->stream, c->queue_d);
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    if (sch == SCH_HYDRO)
      hipLaunchKernelGGL((k_persistent<B, CPT, SCH_HYDRO>), dim3((unsigned)grid), dim3(B), 0,
                         c->stream, bf, cs, c->order_d, c->queue_d, limit);
    else if (sch == SCH_NONWB)
      hipLaunchKernelGGL((k_persistent<B, CPT, SCH_NONWB>), dim3((unsigned)grid), dim3(B), 0,
                         c->stream, bf, cs, c->order_d, c->queue_d, limit);
    else
      hipLaunchKernelGGL((k_persistent<B, CPT, SCH_SPECIAL>), dim3((unsigned)grid), dim3(B), 0,
                         c->stream, bf, cs, c->order_d, c->queue_d, limit);
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    total += ms;
    c->last_launches += 1;
    if (limit <= 0) break;
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(1024), 0, c->stream, bf, c->nactive_d, nullptr);
    HIPCHK(hipMemcpyAsync(c->nactive_h, c->nactive_d, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (*c->nactive_h == 0) break;
  }
  c->last_ms = total;
  return ALEW_OK;
}

template <int B>
alew_status run_persist(alew_ctx* c, const Bufs& bf, const Consts& cs, int64_t ninst, int cpt) {
  if constexpr (B <= 256) {
    if (cpt == 2) return run_persistent<B, 2>(c, bf, cs, ninst);
  }
  return run_persistent<B, 1>(c, bf, cs, ninst);
}

template <int B>
alew_status run_stages(alew_ctx* c, const Bufs& bf, const Consts& cs, int64_t max_iters, int cpt) {
  if constexpr (B <= 256) {
    if (cpt == 2) return run_stage_engine<B, 2>(c, bf, cs, max_iters);
  }
  return run_stage_engine<B, 1>(c, bf, cs, max_iters);
}

alew_status map_status(int bits) {
  if (bits & SB_MESH) return ALEW_E_MESH;
  if (bits & SB_NONFINITE) return ALEW_E_NONFINITE;
  if (bits & SB_NEGDEPTH) return ALEW_E_NEGDEPTH;
  if (bits & SB_NEGWEIGHT) return ALEW_E_NEGWEIGHT;
  if (bits & SB_CAPACITY) return ALEW_E_CAPACITY;
  if (bits & SB_SEQUENCE) return ALEW_E_UNSUPPORTED;  // instances of a batch out of step
  return ALEW_OK;
}

// Shared driver of alew_step and alew_run.
alew_status drive(alew_ctx* c, const alew_params* p, int64_t ninst, const int64_t* cell_off,
                  double* h, double* hu, double* b, double* x, const double* xi,
                  const double* wgiven, const double* t0, const double* t_end,
                  const int64_t* max_steps, const double* dts, double* dt_log, int64_t dts_stride,
                  uint8_t* cls, uint32_t* ccount, uint64_t* csig, alew_stats* stats, int engine) {
  alew_status ps = check_params(p);
  if (ps != ALEW_OK) return ps;
  if (!c) return fail(ALEW_E_ARG, "ctx is NULL");
  if (ninst <= 0 || !cell_off) return fail(ALEW_E_ARG, "ninst <= 0 or cell_off is NULL");
  if (ninst > c->max_inst) return fail(ALEW_E_ARG, "ninst exceeds the context capacity");
  if (!h || !hu || !b || !x) return fail(ALEW_E_ARG, "state or node array is NULL");
  if (prescribed(p->mesh) && !xi)
    return fail(ALEW_E_ARG, "xi is required for the prescribed mesh");
  if (p->mesh == ALEW_MESH_GIVEN && !wgiven) return fail(ALEW_E_ARG, "w is required for MESH_GIVEN");
  if (cell_off[0] != 0) return fail(ALEW_E_ARG, "cell_off[0] must be 0");
  for (int64_t i = 0; i < ninst; ++i)
    if (cell_off[i + 1] - cell_off[i] < 5) return fail(ALEW_E_ARG, "every instance needs >= 5 cells");
  const int64_t S = cell_off[ninst];
  if (S > c->max_cells) return fail(ALEW_E_ARG, "total cells exceed the context capacity");
  if ((dts || dt_log) && dts_stride <= 0) return fail(ALEW_E_ARG, "dts_stride must be > 0");
  if ((ccount == nullptr) != (csig == nullptr))
    return fail(ALEW_E_ARG, "cls_count and cls_sig go together");
  // split negative weights: the stage engine in its automatic tile shape
  const bool split = (p->flags & ALEW_F_SPLIT) != 0;
  if (split) engine = 2;
  const int B = split ? 64 : pick_block(c, engine);
  const int CPT = split ? 2 : pick_cpt(c, B);
  const bool noext = !split && engine != 1 && c->launch.compact_tiles == 1;
  alew_status ts = build_tiles(c, cell_off, ninst, PB, B * CPT, noext);
  if (ts != ALEW_OK) return ts;
  // per-instance scalars
  int64_t max_iters = 0;
  for (int64_t i = 0; i < ninst; ++i) {
    Inst& I = c->inst_h[i];
    std::memset(&I, 0, sizeof(Inst));
    I.t0 = t0 ? t0[i] : 0.0;
    I.t = I.t0;
    I.t_end = t_end ? t_end[i] : 0.0;
    I.max_steps = max_steps ? max_steps[i] : 0;
    I.active = 1;
    I.dt_min = INFINITY;
    I.dt_max = 0.0;
    I.r_minJ = 0x7ff0000000000000ull;  // +inf
    I.r_hmin = 0xffffffffffffffffull;
    if (I.max_steps > 0) max_iters = std::max(max_iters, I.max_steps);
    else if (I.t_end > I.t0) max_iters = std::max<int64_t>(max_iters, INT64_MAX / 4);
  }
  HIPCHK(hipMemcpyAsync(c->inst, c->inst_h, ninst * sizeof(Inst), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->xa, x, (S + ninst) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  Bufs bf = make_bufs(c, S, ninst, hu, b, xi, cls, dts, dt_log, dts_stride, ccount, csig);
  const Consts cs = make_consts(p);
  const dim3 gp((unsigned)c->n_tiles_plain);
#define ALEW_DISPATCH(BB)                                                                       \
  do {                                                                                          \
    hipLaunchKernelGGL(k_prep<PB>, gp, dim3(PB), 0, c->stream, bf, cs, c->tiles_plain_d, h, wgiven); \
    if (cs.mesh == MESH_FLUID)                                                                  \
      hipLaunchKernelGGL(k_wfluid<PB>, gp, dim3(PB), 0, c->stream, bf, cs, c->tiles_plain_d);  \
    launch_boundary(c, bf, cs, c->stream, 1);                                                 \
    HIPCHK(hipGetLastError());                                                                  \
    alew_status rs = (engine == 1) ? run_persist<BB>(c, bf, cs, ninst, CPT)                     \
                                   : run_stages<BB>(c, bf, cs, max_iters, CPT);                 \
    if (rs != ALEW_OK) return rs;                                                               \
    if (c->tables_masked) { /* every instance's tiles again for the finish */                   \
      rs = build_tiles(c, cell_off, ninst, PB, B * CPT, noext);                                 \
      if (rs != ALEW_OK) return rs;                                                             \
    }                                                                                           \
    hipLaunchKernelGGL(k_finish<PB>, gp, dim3(PB), 0, c->stream, bf, cs, c->tiles_plain_d, h, x); \
    hipLaunchKernelGGL(k_masses, dim3((unsigned)((ninst + 3) / 4)), dim3(256), 0, c->stream, bf); \
  } while (0)
  if (B == 64) ALEW_DISPATCH(64);
  else if (B == 128) ALEW_DISPATCH(128);
  else if (B == 512) ALEW_DISPATCH(512);
  else ALEW_DISPATCH(256);
#undef ALEW_DISPATCH
  HIPCHK(hipGetLastError());
  // statistics and status
  HIPCHK(hipMemcpyAsync(c->inst_h, c->inst, ninst * sizeof(Inst), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  alew_status worst = ALEW_OK;
  for (int64_t i = 0; i < ninst; ++i) {
    const Inst& I = c->inst_h[i];
    const alew_status si = map_status(I.status);
    if (si != ALEW_OK && (worst == ALEW_OK || worst == ALEW_E_NEGWEIGHT)) worst = si;
    if (stats) {
      alew_stats& S_ = stats[i];
      std::memset(&S_, 0, sizeof(S_));
      S_.steps = I.steps;
      for (int k = 0; k < 3; ++k) S_.n_class[k] = (int64_t)I.n_class[k];
      S_.n_limited = (int64_t)I.n_limited;
      S_.n_negweight = (int64_t)I.n_negweight;
      S_.t = I.t;
      S_.dt_min = I.dt_min;
      S_.dt_max = I.dt_max;
      unsigned long long k = I.r_hmin;
      unsigned long long u = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
      double hm;
      std::memcpy(&hm, &u, sizeof(hm));
      S_.h_min = hm;
      S_.mass_eta0 = I.mass_eta0;
      S_.mass_eta = I.mass_eta;
      S_.mass_b0 = I.mass_b0;
      S_.mass_b = I.mass_b;
      S_.status = (int32_t)si;
    }
  }
  if (worst != ALEW_OK) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "device reported status %d", (int)worst);
    g_err = buf;
  }
  return worst;
}

// Workspace of alew_adjoint (in doubles): hu and b of the run, checkpoints
// (state, nodes, instance records) every K steps, the per-step records of one
// segment (q of the three stages, x^n and w^n, step scalars, argmax keys),
// and the adjoint state, reverse-tile table and per-instance sums.
constexpr int ADJ_OWN = 250;  // owned cells of a fused reverse-stage tile
struct AdjLayout {
  size_t n_ck, n_ckI, per_step, n_seg, n_at, bytes;
};
AdjLayout adj_layout(int64_t S, int64_t ninst, int64_t n_atiles, int64_t nsteps, int64_t K,
                     int64_t ngauge) {
  AdjLayout L;
  const int64_t nck = (nsteps + K - 1) / K;
  const int64_t NN = S + ninst;
  const size_t n_state = 2 * (size_t)S;
  L.n_ck = (size_t)nck * (3 * S + NN);
  L.n_ckI = (size_t)nck * ninst * sizeof(Inst) / 8 + 1;
  L.per_step = 9 * (size_t)S + 2 * (size_t)NN + 11 * (size_t)ninst;
  L.n_seg = (size_t)(K + 1) * L.per_step;
  L.n_at = (sizeof(AdjTile) / 8) * (size_t)n_atiles;
  const size_t n_adj = 9 * (size_t)S + (size_t)ninst + (size_t)ninst * ngauge +
                       18 * (size_t)ninst + L.n_at + (size_t)n_atiles + (size_t)ninst + 1;
  L.bytes = (n_state + L.n_ck + L.n_ckI + L.n_seg + n_adj) * 8;
  return L;
}

alew_status adj_reserve(alew_ctx* c, size_t bytes) {
  if (c->adj_ws) (void)hipFree(c->adj_ws);
  c->adj_ws = nullptr;
  c->adj_ws_bytes = 0;
  if (hipMalloc(&c->adj_ws, bytes) != hipSuccess) return fail(ALEW_E_NOMEM, "adjoint workspace");
  c->adj_ws_bytes = bytes;
  return ALEW_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free step: alew_step's scratch in a file-scope device array
// ---------------------------------------------------------------------------
constexpr int64_t NA_CELLS = 65536;  // largest instance of alew_step_noalloc
constexpr int NA_MAXDEV = 64;
constexpr size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr int64_t NA_CAP_STAGE = (NA_CELLS + MIN_OWN - 1) / MIN_OWN + 1;
constexpr int64_t NA_CAP_PLAIN = NA_CELLS / PB + 2;
constexpr size_t NA_BYTES =
    al256(NA_CELLS * 8) + 4 * al256(3 * NA_CELLS * 8) + 3 * al256((NA_CELLS + 1) * 8) +
    al256(sizeof(Inst)) + 5 * al256(2 * sizeof(int64_t)) + 4 * al256(8) + al256(8) +
    3 * al256(NA_CAP_STAGE * sizeof(Tile)) + al256(NA_CAP_PLAIN * sizeof(Tile)) +
    2 * al256(NA_CAP_STAGE * SREC * 8) + 2 * al256(NA_CAP_PLAIN * PREC * 8) +
    al256(NA_CAP_STAGE * sizeof(RChunk)) + al256(NA_CAP_PLAIN * sizeof(RChunk));

}  // namespace

// One copy per GPU, held until the process ends.  Host code never uses this
// name for the memory: it takes the device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {

struct NoallocDev {
  bool ready = false;
  alew_ctx ctx;                // device pointers into scratch; no events, no graph
  Inst inst_h;                 // host copies (pageable: nothing is allocated)
  double dt1_h = 0.0;
  int nactive_h = 0;
  uint8_t act_h = 0;
};
NoallocDev g_na[NA_MAXDEV];
std::mutex g_na_mu[NA_MAXDEV];

// Point the context's buffers into the device array at base (same order and
// sizes as NA_BYTES).
alew_status noalloc_setup(NoallocDev& d, char* base) {
  alew_ctx* c = &d.ctx;
  size_t off = 0;
  auto take = [&](auto** p, size_t bytes) {
    *p = reinterpret_cast<std::remove_reference_t<decltype(*p)>>(base + off);
    off += al256(bytes);
  };
  const int64_t S = NA_CELLS, Nn = NA_CELLS + 1;
  take(&c->eta, S * 8);
  take(&c->P0, 3 * S * 8); take(&c->D0, 3 * S * 8); take(&c->P1, 3 * S * 8); take(&c->D1, 3 * S * 8);
  take(&c->w, Nn * 8); take(&c->xa, Nn * 8); take(&c->xb, Nn * 8);
  take(&c->inst, sizeof(Inst));
  take(&c->cell_off_d, 2 * sizeof(int64_t)); take(&c->sfirst_d, 2 * sizeof(int64_t));
  take(&c->pfirst_d, 2 * sizeof(int64_t)); take(&c->scfirst_d, 2 * sizeof(int64_t));
  take(&c->pcfirst_d, 2 * sizeof(int64_t));
  take(&c->order_d, 8); take(&c->queue_d, 8); take(&c->nactive_d, 8); take(&c->act_d, 8);
  take(&c->dt1_d, 8);
  take(&c->tiles_stage_d, NA_CAP_STAGE * sizeof(Tile));
  take(&c->tiles_edge_d, NA_CAP_STAGE * sizeof(Tile));
  take(&c->tiles_inner_d, NA_CAP_STAGE * sizeof(Tile));
  take(&c->tiles_plain_d, NA_CAP_PLAIN * sizeof(Tile));
  take(&c->srec, NA_CAP_STAGE * SREC * 8); take(&c->screc, NA_CAP_STAGE * SREC * 8);
  take(&c->prec, NA_CAP_PLAIN * PREC * 8); take(&c->pcrec, NA_CAP_PLAIN * PREC * 8);
  take(&c->schunk_d, NA_CAP_STAGE * sizeof(RChunk));
  take(&c->pchunk_d, NA_CAP_PLAIN * sizeof(RChunk));
  if (off > NA_BYTES) return fail(ALEW_E_ARG, "internal: static scratch layout");
  c->max_cells = NA_CELLS;
  c->max_inst = 1;
  c->cap_stage = NA_CAP_STAGE;
  c->cap_plain = NA_CAP_PLAIN;
  c->inst_h = &d.inst_h;
  c->dt1_h = &d.dt1_h;
  c->nactive_h = &d.nactive_h;
  c->act_h = &d.act_h;
  return ALEW_OK;
}

}  // namespace


// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* alew_last_error(void) { return g_err.c_str(); }

alew_status alew_last_timing(const alew_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return fail(ALEW_E_ARG, "NULL argument");
  *ms = c->last_ms;
  *launches = c->last_launches;
  return ALEW_OK;
}
alew_status alew_set_kernel_timing(alew_ctx* c, int on) {
  if (!c) return fail(ALEW_E_ARG, "ctx is NULL");
  c->ktime_on = on != 0;
  return ALEW_OK;
}

alew_status alew_kernel_timing(const alew_ctx* c, int which, double* ms, int64_t* launches,
                               double* cells) {
  if (!c || !ms || !launches || !cells) return fail(ALEW_E_ARG, "NULL argument");
  if (which < 0 || which > 4) return fail(ALEW_E_ARG, "which must be 0 to 4");
  double tot = 0.0, cel = 0.0;
  int64_t n = 0;
  for (size_t k = 0; k < c->kt_used; ++k) {
    const int kd = c->kt_kind[k];
    if (which == 0 ? kd < 2 : kd != which) continue;
    float e = 0.f;
    HIPCHK(hipEventElapsedTime(&e, c->kt_ev[2 * k], c->kt_ev[2 * k + 1]));
    tot += e;
    cel += c->kt_cells[k];
    ++n;
  }
  *ms = tot;
  *launches = n;
  *cells = cel;
  return ALEW_OK;
}

const char* alew_version(void) { return "alew 0.1 gfx950 fp64"; }

alew_status alew_create(alew_ctx** out, int64_t max_cells, int64_t max_inst, void* hip_stream) {
  if (!out) return fail(ALEW_E_ARG, "ctx output pointer is NULL");
  *out = nullptr;
  if (max_cells < 5 || max_inst < 1) return fail(ALEW_E_ARG, "max_cells >= 5 and max_inst >= 1 required");
  alew_ctx* c = new alew_ctx();
  c->stream = (hipStream_t)hip_stream;
  c->max_cells = max_cells;
  c->max_inst = max_inst;
  const int64_t S = max_cells, Nn = max_cells + max_inst;
  auto alloc = [&](void** p, size_t bytes) -> bool { return hipMalloc(p, bytes) == hipSuccess; };
  bool ok = alloc((void**)&c->eta, S * 8) && alloc((void**)&c->P0, 3 * S * 8) &&
            alloc((void**)&c->D0, 3 * S * 8) && alloc((void**)&c->P1, 3 * S * 8) &&
            alloc((void**)&c->D1, 3 * S * 8) && alloc((void**)&c->w, Nn * 8) &&
            alloc((void**)&c->xa, Nn * 8) && alloc((void**)&c->xb, Nn * 8) &&
            alloc((void**)&c->inst, max_inst * sizeof(Inst)) &&
            alloc((void**)&c->cell_off_d, (max_inst + 1) * sizeof(int64_t)) &&
            alloc((void**)&c->sfirst_d, (max_inst + 1) * sizeof(int64_t)) &&
            alloc((void**)&c->pfirst_d, (max_inst + 1) * sizeof(int64_t)) &&
            alloc((void**)&c->scfirst_d, (max_inst + 1) * sizeof(int64_t)) &&
            alloc((void**)&c->pcfirst_d, (max_inst + 1) * sizeof(int64_t)) &&
            alloc((void**)&c->order_d, max_inst * sizeof(int32_t)) &&
            alloc((void**)&c->queue_d, sizeof(unsigned)) && alloc((void**)&c->nactive_d, sizeof(int)) &&
            alloc((void**)&c->act_d, max_inst) &&
            alloc((void**)&c->dt1_d, sizeof(double));
  // tile tables, result records and record chunks, sized for the smallest
  // stage tile (64 slots, 58 owned cells) and the plain tiles (256 items over
  // the n + 1 nodes of each instance)
  c->cap_stage = (max_cells + MIN_OWN - 1) / MIN_OWN + max_inst;
  c->cap_plain = max_cells / PB + max_inst + 1;
  const int64_t cs_ = c->cap_stage, cp_ = c->cap_plain;
  ok = ok && alloc((void**)&c->tiles_stage_d, cs_ * sizeof(Tile)) &&
       alloc((void**)&c->tiles_edge_d, cs_ * sizeof(Tile)) &&
       alloc((void**)&c->tiles_inner_d, cs_ * sizeof(Tile)) &&
       alloc((void**)&c->tiles_plain_d, cp_ * sizeof(Tile)) &&
       alloc((void**)&c->srec, cs_ * SREC * sizeof(double)) &&
       alloc((void**)&c->screc, cs_ * SREC * sizeof(double)) &&
       alloc((void**)&c->prec, cp_ * PREC * sizeof(double)) &&
       alloc((void**)&c->pcrec, cp_ * PREC * sizeof(double)) &&
       alloc((void**)&c->schunk_d, cs_ * sizeof(RChunk)) &&
       alloc((void**)&c->pchunk_d, cp_ * sizeof(RChunk));
  ok = ok && hipHostMalloc((void**)&c->dt1_h, sizeof(double), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c->inst_h, max_inst * sizeof(Inst), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c->nactive_h, sizeof(int), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c->act_h, max_inst, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreate(&c->ev0) == hipSuccess && hipEventCreate(&c->ev1) == hipSuccess;
  if (!ok) {
    alew_destroy(c);
    return fail(ALEW_E_NOMEM, "device allocation failed");
  }
  *out = c;
  return ALEW_OK;
}

void alew_destroy(alew_ctx* c) {
  if (!c) return;
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  void* ps[] = {c->eta, c->P0, c->D0, c->P1, c->D1, c->w, c->xa, c->xb, c->inst, c->cell_off_d,
                c->order_d, c->queue_d, c->nactive_d, c->tiles_stage_d, c->tiles_plain_d,
                c->tiles_edge_d, c->tiles_inner_d, c->srec, c->prec, c->sfirst_d, c->pfirst_d,
                c->scfirst_d, c->pcfirst_d, c->schunk_d, c->pchunk_d, c->screc, c->pcrec, c->act_d,
                c->dt1_d,
                c->adj_ws};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (c->inst_h) (void)hipHostFree(c->inst_h);
  if (c->dt1_h) (void)hipHostFree(c->dt1_h);
  if (c->nactive_h) (void)hipHostFree(c->nactive_h);
  if (c->act_h) (void)hipHostFree(c->act_h);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->kt_ev) (void)hipEventDestroy(e);
  delete c;
}

alew_status alew_set_stream(alew_ctx* c, void* s) {
  if (!c) return fail(ALEW_E_ARG, "ctx is NULL");
  c->stream = (hipStream_t)s;
  return ALEW_OK;
}

alew_status alew_set_launch(alew_ctx* c, const alew_launch* l) {
  if (!c || !l) return fail(ALEW_E_ARG, "ctx or launch is NULL");
  if (l->engine < 0 || l->engine > 2) return fail(ALEW_E_ARG, "unknown engine");
  if (l->block != 0 && l->block != 64 && l->block != 128 && l->block != 256 && l->block != 512)
    return fail(ALEW_E_ARG, "block must be 0, 64, 128, 256 or 512");
  if (l->cells_per_thread < 0 || l->cells_per_thread > 2)
    return fail(ALEW_E_ARG, "cells_per_thread must be 0, 1 or 2");
  if (l->compact_tiles < 0 || l->compact_tiles > 1)
    return fail(ALEW_E_ARG, "compact_tiles must be 0 or 1");
  c->launch = *l;
  return ALEW_OK;
}

alew_status alew_get_launch(const alew_ctx* c, alew_launch* l) {
  if (!c || !l) return fail(ALEW_E_ARG, "ctx or launch is NULL");
  *l = c->launch;
  return ALEW_OK;
}

alew_status alew_step(alew_ctx* c, const alew_params* p, int64_t ncell, double* h, double* hu,
                      double* b, double* x, const double* xi, const double* w, double t, double dt,
                      double t_end, uint8_t* cls, alew_stats* stats) {
  if (!c) return fail(ALEW_E_ARG, "ctx is NULL");
  if (ncell < 5) return fail(ALEW_E_ARG, "ncell must be >= 5");
  const int64_t off[2] = {0, ncell};
  const int64_t one = 1;
  const double tend = t_end;
  const double* dts = nullptr;
  if (dt > 0) {
    HIPCHK(hipStreamSynchronize(c->stream));  // the staging buffer may still be in use
    *c->dt1_h = dt;
    HIPCHK(hipMemcpyAsync(c->dt1_d, c->dt1_h, sizeof(double), hipMemcpyHostToDevice, c->stream));
    dts = c->dt1_d;
  }
  const alew_launch keep = c->launch;
  c->launch.engine = 2;
  c->launch.use_graph = 0;
  alew_stats st;
  alew_status r = drive(c, p, 1, off, h, hu, b, x, xi, w, &t, &tend, &one, dts, nullptr,
                        dts ? 1 : 0, cls, nullptr, nullptr, &st, 2);
  c->launch = keep;
  if (stats) *stats = st;
  return r;
}

alew_status alew_step_noalloc(const alew_params* p, int64_t ncell, double* h, double* hu, double* b,
                              double* x, const double* xi, const double* w, double t, double dt,
                              double t_end, uint8_t* cls, alew_stats* stats, void* hip_stream) {
  if (ncell < 5) return fail(ALEW_E_ARG, "ncell must be >= 5");
  if (ncell > NA_CELLS)
    return fail(ALEW_E_ARG, "alew_step_noalloc: ncell exceeds the static scratch maximum of " +
                                std::to_string(NA_CELLS) + " cells");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NA_MAXDEV) return fail(ALEW_E_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_na_mu[dev]);
  NoallocDev& d = g_na[dev];
  if (!d.ready) {
    // once per device, with the device current: the address of this GPU's copy
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    alew_status ls = noalloc_setup(d, (char*)ptr);
    if (ls != ALEW_OK) return ls;
    d.ready = true;
  }
  alew_ctx* c = &d.ctx;
  c->stream = (hipStream_t)hip_stream;
  const int64_t off[2] = {0, ncell};
  const int64_t one = 1;
  const double tend = t_end;
  const double* dts = nullptr;
  if (dt > 0) {
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, c->stream, c->dt1_d, (int64_t)1, dt);
    dts = c->dt1_d;
  }
  c->launch = alew_launch{2, 0, 0, 0, 0, 0};
  alew_stats st;
  alew_status r = drive(c, p, 1, off, h, hu, b, x, xi, w, &t, &tend, &one, dts, nullptr,
                        dts ? 1 : 0, cls, nullptr, nullptr, &st, 2);
  if (stats) *stats = st;
  return r;
}

alew_status alew_run(alew_ctx* c, const alew_params* p, int64_t ninst, const int64_t* cell_off,
                     double* h, double* hu, double* b, double* x, const double* xi,
                     const double* t0, const double* t_end, const int64_t* max_steps,
                     const double* dts, double* dt_log, int64_t dts_stride, uint32_t* cls_count,
                     uint64_t* cls_sig, alew_stats* stats) {
  if (p && p->mesh == ALEW_MESH_GIVEN) return fail(ALEW_E_UNSUPPORTED, "alew_run needs a SINE, PAPER, ALIGNED or FLUID mesh");
  if (!c) return fail(ALEW_E_ARG, "ctx is NULL");
  int engine = c->launch.engine;
  if (engine == 0) engine = 2;
  std::vector<alew_stats> tmp;
  if (!stats) { tmp.resize(ninst > 0 ? ninst : 1); stats = tmp.data(); }
  return drive(c, p, ninst, cell_off, h, hu, b, x, xi, nullptr, t0, t_end, max_steps, dts, dt_log,
               dts_stride, nullptr, cls_count, cls_sig, stats, engine);
}

alew_status alew_adjoint_reserve(alew_ctx* c, int64_t nsteps, int64_t ckpt_every, int64_t ngauge) {
  if (!c) return fail(ALEW_E_ARG, "ctx is NULL");
  if (nsteps < 1 || ngauge < 1) return fail(ALEW_E_ARG, "nsteps and ngauge must be >= 1");
  const int64_t K = ckpt_every > 0 ? ckpt_every : 16;
  const int64_t nat = c->max_cells / ADJ_OWN + c->max_inst;
  const AdjLayout L = adj_layout(c->max_cells, c->max_inst, nat, nsteps, K, ngauge);
  if (L.bytes <= c->adj_ws_bytes) return ALEW_OK;
  return adj_reserve(c, L.bytes);
}

alew_status alew_adjoint(alew_ctx* c, const alew_params* p, int64_t ninst,
                         const int64_t* cell_off, const double* h0, const double* hu0,
                         const double* b0, const double* x0, const double* xi, double t0,
                         int64_t nsteps, const double* dts, int64_t ckpt_every, int64_t ngauge,
                         const double* gauge_x, double* gauge_h, const double* gauge_bar,
                         double* dh0, double* dhu0, double* db0) {
  alew_status ps = check_params(p);
  if (ps != ALEW_OK) return ps;
  if (!c) return fail(ALEW_E_ARG, "ctx is NULL");
  if (!prescribed(p->mesh))
    return fail(ALEW_E_UNSUPPORTED, "the adjoint needs a prescribed (SINE, PAPER or ALIGNED) mesh");
  if (p->flags & ALEW_F_ALPHA_CELLAVG)
    return fail(ALEW_E_UNSUPPORTED, "the adjoint takes the LF speed over the face traces");
  if (p->flags & ALEW_F_NONWB)
    return fail(ALEW_E_UNSUPPORTED, "the adjoint covers the well-balanced schemes");
  if (p->bottom != ALEW_BOTTOM_ALE)
    return fail(ALEW_E_UNSUPPORTED, "the adjoint differentiates with respect to an evolved bottom");
  if (ninst <= 0 || ninst > c->max_inst || !cell_off) return fail(ALEW_E_ARG, "bad ninst / cell_off");
  if (!h0 || !hu0 || !b0 || !x0 || !xi || !dts) return fail(ALEW_E_ARG, "NULL input array");
  if (nsteps < 1) return fail(ALEW_E_ARG, "nsteps must be >= 1");
  if (ngauge < 1 || !gauge_x) return fail(ALEW_E_ARG, "gauges required");
  if (gauge_bar && (!dh0 || !dhu0 || !db0)) return fail(ALEW_E_ARG, "gradient outputs required");
  if (cell_off[0] != 0) return fail(ALEW_E_ARG, "cell_off[0] must be 0");
  for (int64_t i = 0; i < ninst; ++i)
    if (cell_off[i + 1] - cell_off[i] < 5) return fail(ALEW_E_ARG, "every instance needs >= 5 cells");
  const int64_t S = cell_off[ninst];
  if (S > c->max_cells) return fail(ALEW_E_ARG, "total cells exceed the context capacity");
  const int64_t K = ckpt_every > 0 ? ckpt_every : 16;
  const int64_t nck = (nsteps + K - 1) / K;
  const int64_t NN = S + ninst;
  // forward passes in the stage-launch engine's tile shape
  const int B = pick_block(c, 2), CPT = pick_cpt(c, B);
  alew_status ts = build_tiles(c, cell_off, ninst, PB, B * CPT, c->launch.compact_tiles == 1);
  if (ts != ALEW_OK) return ts;
  // tiles of the fused reverse stage: ADJ_OWN owned cells each (256 threads)
  constexpr int BA = 256, TBA = ADJ_OWN;
  std::vector<AdjTile> atiles;
  for (int64_t i = 0; i < ninst; ++i)
    for (int64_t c0 = 0; c0 < cell_off[i + 1] - cell_off[i]; c0 += TBA)
      atiles.push_back(AdjTile{(int32_t)i, 0, c0, cell_off[i], cell_off[i + 1] - cell_off[i]});
  const AdjLayout L = adj_layout(S, ninst, (int64_t)atiles.size(), nsteps, K, ngauge);
  if (L.bytes > c->adj_ws_bytes) {
    alew_status rs = adj_reserve(c, L.bytes);
    if (rs != ALEW_OK) return rs;
  }
  const size_t n_ck = L.n_ck, n_ckI = L.n_ckI, per_step = L.per_step, n_seg = L.n_seg,
               n_at = L.n_at;
  double* wp = c->adj_ws;
  double* st_m = wp; wp += S;
  double* st_b = wp; wp += S;
  double* ck = wp; wp += n_ck;
  Inst* ckI = (Inst*)wp; wp += n_ckI;
  double* seg = wp; wp += n_seg;
  double* lam = wp; wp += 3 * S;
  double* lam2 = wp; wp += 3 * S;
  double* lbase = wp; wp += 3 * S;
  double* gfold = wp; wp += 18 * ninst;
  AdjTile* atiles_d = (AdjTile*)wp; wp += n_at;
  double* lalpha = wp; wp += ninst;
  double* lpart = wp; wp += atiles.size();
  int64_t* tfirst_d = (int64_t*)wp; wp += ninst + 1;
  int64_t* gcell = (int64_t*)wp; wp += ninst * ngauge;
  hipStream_t st = c->stream;
  // per-instance scalars: nsteps frozen steps from t0
  for (int64_t i = 0; i < ninst; ++i) {
    Inst& I = c->inst_h[i];
    std::memset(&I, 0, sizeof(Inst));
    I.t0 = t0; I.t = t0; I.t_end = 0.0; I.max_steps = nsteps; I.active = 1;
    I.dt_min = INFINITY; I.dt_max = 0.0;
    I.r_minJ = 0x7ff0000000000000ull;
    I.r_hmin = 0xffffffffffffffffull;
  }
  HIPCHK(hipMemcpyAsync(c->inst, c->inst_h, ninst * sizeof(Inst), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(c->xa, x0, NN * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(st_m, hu0, S * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(st_b, b0, S * 8, hipMemcpyDeviceToDevice, st));
  Bufs bf = make_bufs(c, S, ninst, st_m, st_b, xi, nullptr, dts, nullptr, nsteps);
  // the reverse sweep differentiates the unsplit weights: a negative linear
  // weight is reported (ALEW_E_NEGWEIGHT), never split
  Consts cs = make_consts(p);
  cs.flags &= ~F_SPLIT;
  const dim3 gp((unsigned)c->n_tiles_plain);
  auto step_dump = [&](int64_t slot) {
    Dump d;
    double* base = seg + slot * per_step;
    d.q = base;
    d.xw = base + 9 * S;
    d.scal = base + 9 * S + 2 * NN;
    d.akey = d.scal + 8 * ninst;
    d.scal_next = d.scal + per_step;
    return d;
  };
  auto xbuf_of = [&](int64_t k) { return (k & 1) ? c->xb : c->xa; };
  hipLaunchKernelGGL(k_prep<256>, gp, dim3(256), 0, st, bf, cs, c->tiles_plain_d, h0, nullptr);
  launch_boundary(c, bf, cs, st, 1);
  // forward with checkpoints; when a gradient follows, the last segment keeps
  // its records right away (the reverse sweep starts there)
  const int64_t qlast = nck - 1, klast = qlast * K;
  const bool keep_last = gauge_bar != nullptr;
  for (int64_t k = 0; k < nsteps; ++k) {
    if (k % K == 0 && !(keep_last && k / K == qlast)) {
      const int64_t q = k / K;
      double* cq = ck + q * (3 * S + NN);
      HIPCHK(hipMemcpyAsync(cq, c->eta, S * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(cq + S, st_m, S * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(cq + 2 * S, st_b, S * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(cq + 3 * S, xbuf_of(k), NN * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(ckI + q * ninst, c->inst, ninst * sizeof(Inst), hipMemcpyDeviceToDevice, st));
    }
    if (keep_last && k >= klast) {
      if (k == klast)
        hipLaunchKernelGGL(k_seed_scal, dim3(1), dim3(1024), 0, st, bf, step_dump(0).scal);
      Bufs bd = bf;
      bd.dump = step_dump(k - klast);
      launch_step_shape(c, B, CPT, bd, cs, st, k);
    } else {
      launch_step_shape(c, B, CPT, bf, cs, st, k);
    }
  }
  HIPCHK(hipGetLastError());
  const int64_t ng = ninst * ngauge;
  const unsigned gb = (unsigned)((ng + 255) / 256);
  hipLaunchKernelGGL(k_gauge, dim3(gb), dim3(256), 0, st, bf, ngauge, gauge_x, gauge_h, gcell);
  HIPCHK(hipMemcpyAsync(c->inst_h, c->inst, ninst * sizeof(Inst), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int64_t i = 0; i < ninst; ++i) {
    const alew_status si = map_status(c->inst_h[i].status);
    if (si != ALEW_OK && si != ALEW_E_NEGWEIGHT) return fail(si, "forward run of the adjoint failed");
    if (c->inst_h[i].steps != nsteps) return fail(ALEW_E_ARG, "forward run stopped early");
  }
  if (!gauge_bar) return ALEW_OK;
  // reverse sweep
  const unsigned g3 = (unsigned)((3 * S + 255) / 256);
  hipLaunchKernelGGL(k_fill, dim3(g3), dim3(256), 0, st, lam, 3 * S, 0.0);
  hipLaunchKernelGGL(k_gauge_seed, dim3((unsigned)((ninst + 255) / 256)), dim3(256), 0, st, ninst,
                     ngauge, S, gcell, gauge_bar, lam);
  AdjBufs ab;
  ab.cell_off = c->cell_off_d; ab.S = S; ab.ninst = (int32_t)ninst; ab.pad = 0;
  ab.lam = lam; ab.lam_out = lam2; ab.lbase = lbase; ab.lalpha = lalpha;
  ab.lpart = lpart;
  {
    // first fused tile of each instance
    std::vector<int64_t> tf(ninst + 1, 0);
    for (int64_t i = 0; i < ninst; ++i)
      tf[i + 1] = tf[i] + (cell_off[i + 1] - cell_off[i] + TBA - 1) / TBA;
    if (tf[ninst] != (int64_t)atiles.size()) return fail(ALEW_E_ARG, "internal: fused tile count");
    HIPCHK(hipMemcpyAsync(tfirst_d, tf.data(), tf.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(atiles_d, atiles.data(), atiles.size() * sizeof(AdjTile),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  const dim3 ga((unsigned)atiles.size());
  const unsigned gfb = (unsigned)((ninst + 255) / 256);
  for (int64_t q = nck - 1; q >= 0; --q) {
    const int64_t k0 = q * K, k1 = std::min(nsteps, k0 + K);
    if (q != qlast) {  // recompute the segment from its checkpoint, keeping records
      double* cq = ck + q * (3 * S + NN);
      HIPCHK(hipMemcpyAsync(c->eta, cq, S * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(st_m, cq + S, S * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(st_b, cq + 2 * S, S * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(xbuf_of(k0), cq + 3 * S, NN * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(c->inst, ckI + q * ninst, ninst * sizeof(Inst), hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(k_seed_scal, dim3(1), dim3(1024), 0, st, bf, step_dump(0).scal);
      for (int64_t k = k0; k < k1; ++k) {
        Bufs bd = bf;
        bd.dump = step_dump(k - k0);
        launch_step_shape(c, B, CPT, bd, cs, st, k);
      }
    }
    for (int64_t k = k1 - 1; k >= k0; --k) {
      const Dump d = step_dump(k - k0);
      ab.x = d.xw; ab.w = d.xw + NN; ab.scal = d.scal;
      for (int s3 = 3; s3 >= 1; --s3) {
        ab.q = d.q + (int64_t)3 * (s3 - 1) * S;
        ab.akeyd = d.akey + (int64_t)(s3 - 1) * ninst;
        if (cs.flags & F_HYDROSTATIC)
          hipLaunchKernelGGL((k_adj_fused<BA, true>), ga, dim3(BA), 0, st, ab, cs, atiles_d, s3,
                             gfold);
        else
          hipLaunchKernelGGL((k_adj_fused<BA, false>), ga, dim3(BA), 0, st, ab, cs, atiles_d, s3,
                             gfold);
        hipLaunchKernelGGL(k_adj_fold, dim3(gfb), dim3(256), 0, st, ab, cs, gfold);
        hipLaunchKernelGGL(k_adj_lsum, dim3((unsigned)((ninst + 3) / 4)), dim3(256), 0, st, ab, tfirst_d);
        hipLaunchKernelGGL(k_adj_patch, dim3((unsigned)((ninst + 63) / 64)), dim3(64), 0, st, ab, cs, s3);
        std::swap(ab.lam, ab.lam_out);
      }
    }
    HIPCHK(hipGetLastError());
  }
  const unsigned g1 = (unsigned)((S + 255) / 256);
  hipLaunchKernelGGL(k_adj_out, dim3(g1), dim3(256), 0, st, S, ab.lam, dh0, dhu0, db0);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return ALEW_OK;
}

}  // extern "C"
