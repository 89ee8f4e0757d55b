// Tile bodies shared by the stage-launch engine and the persistent engine.
#pragma once

#include "alew_device.h"

namespace alew_dev {

// Records kept by the forward recomputation of the adjoint (all NULL otherwise).
struct Dump {
  double* q;     // [3 stages][3 comps][S]: stage inputs q^(s-1)
  double* akey;  // [3 stages][ninst]: 2 f + side of the first face trace attaining alpha
  double* xw;    // [2][S + ninst]: x^n and w^n of the step
  double* scal;       // [ninst][8] of this step: t, dt, alpha_1..3, dx_0..2
  double* scal_next;  // the next step's record (t, dt, dx_0 are set at step end)
};

// Up to RCHUNK consecutive tile records of one instance, reduced by one wave.
// An instance with more records has several chunks; their partial results are
// reduced by a second pass (max, min and integer sums: order-free, exact).
enum { RCHUNK = 512 };
struct RChunk {
  int32_t inst;
  int32_t whole;  // 1 if the chunk holds every record of its instance
  int64_t k0, k1;
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
  // optional class record of a run: per-cell counts of stages classified
  // S / T / N ([3][S]) and a signature of each cell's class sequence ([S]),
  // csig <- csig * CLS_SIG_MUL + class + 1 (mod 2^64) at every stage
  uint32_t* ccount;
  unsigned long long* csig;
  Inst* inst;
  const double* dts;  // optional frozen step sizes [ninst][dts_stride]
  double* dt_log;     // optional [ninst][dts_stride]
  int64_t dts_stride;
  int64_t S;
  int32_t ninst;
  int32_t pad;
  double* srec;            // [stage tiles][SREC] per-tile stage results
  double* prec;            // [plain tiles][PREC] per-tile step results
  const int64_t* sfirst;   // [ninst+1] first stage tile of each instance
  const int64_t* pfirst;   // [ninst+1] first plain tile of each instance
  const RChunk* schunk;    // record chunks of the stage / plain tables
  const RChunk* pchunk;
  const int64_t* scfirst;  // [ninst+1] first stage / plain chunk of each instance
  const int64_t* pcfirst;
  double* screc;           // [stage chunks][SREC] partial results of split instances
  double* pcrec;           // [plain chunks][PREC]
  Dump dump;
};

// Multiplier of the class-sequence signature (odd, so that every class
// sequence of a cell maps to its own residue far more often than not).
constexpr unsigned long long CLS_SIG_MUL = 1099511628211ull;

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

// Scalars of stage s of an instance.
__device__ __forceinline__ StageScal stage_scal(const Inst& I, int s) {
  StageScal sc;
  sc.s = s;
  sc.dt = I.dt;
  sc.as = s == 1 ? 0.0 : (s == 2 ? 0.75 : 1.0 / 3.0);
  sc.bs = s == 1 ? 1.0 : (s == 2 ? 0.25 : 2.0 / 3.0);
  const double bprev = s == 2 ? 1.0 : 0.25;
  sc.cprev = s == 1 ? 0.0 : bprev * I.dt * I.alpha[s - 2];
  sc.dx = I.dx[s - 1];
  sc.wsc = I.wscale;
  return sc;
}

// Block-level results of a stage tile.
struct StageRes {
  double alpha, maxJ;
  double akey;  // (records kept) first face trace of the tile attaining its alpha
  unsigned ncls0, ncls1, ncls2, nlim, nneg;
  int status;
};

// LDS of a stage tile: B threads, CPT cells per thread, TB = B * CPT cells
// reconstructed per tile (TB - 2 of them owned).
template <int B, int CPT>
struct SmemStage {
  static constexpr int TB = B * CPT;
  static constexpr int NW = B / 64;
  // Stencil slot i holds cell k = c0 - 3 + i (ghosts mapped).  The stencil
  // arrays are dead once the traces are formed, so the face values reuse them.
  union {
    struct {
      double e[TB + 4], m[TB + 4], b[TB + 4], J[TB + 4], iJ[TB + 4];
    } in;
    double fl[7][TB];
  } u;
  double wn[TB + 4];     // node speed at the left node of slot i (nodes 0..n)
  double qn[3][TB + 4];  // a_s Q^n of owned slots (stages 2 and 3)
  double Jx[TB + 4];     // the width this stage produces, a_s J^n + b_s (J + dt dw)
  double xr[CPT * NW][3];  // right traces of the last lane of each wave
  double red[NW * 8];
  unsigned cntw[NW][8];  // per wave: class S/T/N, limited, negative weight, status bits
};

// 32-bit byte offsets from a work-group-uniform base (instances of fewer than
// 2^28 cells), so every load of a slot shares one offset register.
__device__ __forceinline__ double ldo(const double* base, unsigned off) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + off);
}

// Work-group b of a G-group launch is dispatched to XCD b mod 8; this maps
// the groups of each XCD onto one contiguous eighth of the tile table, so
// that neighbouring tiles, whose stencils share the cache lines at the tile
// ends, run on the same XCD and meet in its L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G) {
  const int64_t x = b & 7, q = G >> 3, r = G & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// Stage inputs of one stencil slot from its raw loads: x^n and w of the two
// nodes, and either q^n (stage 1) or P, D of the previous stage together with
// q^n of the cell (stages 2, 3).  ms = -1 mirrors hu (reflective ghosts).
template <class SM>
__device__ __forceinline__ void put_slot(const StageScal& sc, int i, double ms, bool real,
                                         double x0, double x1, double w0r, double w1r,
                                         double a0, double a1, double a2, double d0, double d1,
                                         double d2, double q0, double q1, double q2, SM& sm,
                                         int& st) {
  const double Jn = x1 - x0;
  const double w0 = w0r * sc.wsc;
  const double dw = w1r * sc.wsc - w0;
  double J, iJ, e, m, b, qe = 0.0, qm = 0.0, qb = 0.0;
  if (sc.s == 1) {
    J = Jn;
    iJ = frcp(J);
    e = a0;
    m = a1 * ms;
    b = a2;
  } else {
    const double J1 = Jn + sc.dt * dw;
    J = (sc.s == 2) ? J1 : 0.75 * Jn + 0.25 * (J1 + sc.dt * dw);
    iJ = frcp(J);
    e = (a0 + sc.cprev * d0) * iJ;
    m = ((a1 + sc.cprev * d1) * iJ) * ms;
    b = (a2 + sc.cprev * d2) * iJ;
    if (real) {
      qe = sc.as * (Jn * q0);
      qm = sc.as * (Jn * q1);
      qb = sc.as * (Jn * q2);
    }
  }
  if (!(J > 0.0)) st |= SB_MESH;
  sm.u.in.e[i] = e; sm.u.in.m[i] = m; sm.u.in.b[i] = b; sm.u.in.J[i] = J; sm.u.in.iJ[i] = iJ;
  sm.Jx[i] = sc.as * Jn + sc.bs * (J + sc.dt * dw);
  sm.qn[0][i] = qe; sm.qn[1][i] = qm; sm.qn[2][i] = qb;
  if (real) sm.wn[i] = w0;
}

// Raw values of one ghost-free stencil slot: x^n and w at its two nodes, and
// q^n (first stage) or P, D of the previous stage and q^n (later stages).
struct RawSlot {
  double x0, x1, w0, w1, a0, a1, a2, d0, d1, d2, q0, q1, q2;
};

// Issue the loads of the ghost-free slot at byte offset o of the instance.
// P, D are the previous stage's rows (unused in the first stage).
template <bool FIRST>
__device__ __forceinline__ RawSlot raw_inner(const Bufs& bf, const View& v, const double* P,
                                             const double* D, unsigned o) {
  RawSlot r;
  const double* ws = bf.w + v.no;
  r.x0 = ldo(v.x, o); r.x1 = ldo(v.x, o + 8u);
  r.w0 = ldo(ws, o); r.w1 = ldo(ws, o + 8u);
  const double* eta = bf.eta + v.co;
  const double* hu = bf.m + v.co;
  const double* bb = bf.b + v.co;
  if (FIRST) {
    r.a0 = ldo(eta, o); r.a1 = ldo(hu, o); r.a2 = ldo(bb, o);
    r.d0 = 0.0; r.d1 = 0.0; r.d2 = 0.0;
    r.q0 = 0.0; r.q1 = 0.0; r.q2 = 0.0;
  } else {
    const int64_t S = bf.S;
    r.a0 = ldo(P, o); r.a1 = ldo(P + S, o); r.a2 = ldo(P + 2 * S, o);
    r.d0 = ldo(D, o); r.d1 = ldo(D + S, o); r.d2 = ldo(D + 2 * S, o);
    r.q0 = ldo(eta, o); r.q1 = ldo(hu, o); r.q2 = ldo(bb, o);
  }
  return r;
}

template <class SM>
__device__ __forceinline__ void put_raw(const StageScal& sc, int i, const RawSlot& r, SM& sm,
                                        int& st) {
  put_slot(sc, i, 1.0, true, r.x0, r.x1, r.w0, r.w1, r.a0, r.a1, r.a2, r.d0, r.d1, r.d2, r.q0,
           r.q1, r.q2, sm, st);
}

// Ghost-free tile: every load of the thread's slots (and of the four slots
// past the last thread) is issued before the first of them is used, so a
// tile waits for memory once.
template <int B, int CPT, bool FIRST, class SM>
__device__ __forceinline__ void load_tile_inner(const Bufs& bf, const View& v, const StageScal& sc,
                                                int64_t c0, SM& sm, int& st) {
  constexpr int TB = B * CPT;
  const int t = threadIdx.x;
  const double* P = ((sc.s == 2) ? bf.P0 : bf.P1) + v.co;
  const double* D = ((sc.s == 2) ? bf.D0 : bf.D1) + v.co;
  RawSlot r[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
    r[c] = raw_inner<FIRST>(bf, v, P, D, (unsigned)(c0 - 3 + t + c * B) * 8u);
  const bool ext = t < 4;
  RawSlot rx;
  if (ext) rx = raw_inner<FIRST>(bf, v, P, D, (unsigned)(c0 - 3 + TB + t) * 8u);
#pragma unroll
  for (int c = 0; c < CPT; ++c) put_raw(sc, t + c * B, r[c], sm, st);
  if (ext) put_raw(sc, TB + t, rx, sm, st);
}

// Slot of a tile that touches an end of the instance: ghosts mapped by the
// boundary condition; slots beyond the ghosts get a harmless placeholder.
template <class SM>
__device__ __forceinline__ void load_slot_edge(const Bufs& bf, const Consts& cs, const View& v,
                                               const StageScal& sc, int64_t k, int i, SM& sm,
                                               int& st) {
  sm.wn[i] = (k == v.n) ? bf.w[v.no + v.n] * sc.wsc : 0.0;
  if (k >= -3 && k < v.n + 3) {
    double ms;
    const int64_t src = ghost_src(cs.bc, v.n, k, ms);
    const bool real = k >= 0 && k < v.n;
    const double x0 = v.x[src], x1 = v.x[src + 1];
    const double w0 = bf.w[v.no + src], w1 = bf.w[v.no + src + 1];
    const int64_t g = v.co + src;
    if (sc.s == 1) {
      put_slot(sc, i, ms, real, x0, x1, w0, w1, bf.eta[g], bf.m[g], bf.b[g], 0.0, 0.0, 0.0, 0.0,
               0.0, 0.0, sm, st);
    } else {
      const double* P = (sc.s == 2) ? bf.P0 : bf.P1;
      const double* D = (sc.s == 2) ? bf.D0 : bf.D1;
      const int64_t S = bf.S;
      put_slot(sc, i, ms, real, x0, x1, w0, w1, P[g], P[S + g], P[2 * S + g], D[g], D[S + g],
               D[2 * S + g], bf.eta[g], bf.m[g], bf.b[g], sm, st);
    }
  } else {
    sm.u.in.e[i] = 0.0; sm.u.in.m[i] = 0.0; sm.u.in.b[i] = 0.0;
    sm.u.in.J[i] = 1.0; sm.u.in.iJ[i] = 1.0; sm.Jx[i] = 0.0;
    sm.qn[0][i] = 0.0; sm.qn[1][i] = 0.0; sm.qn[2][i] = 0.0;
  }
}

// True if every stencil slot of the tile at c0 is a real cell.
// NS stencil slots per tile (TB + 4 with the extra slots, TB without).
template <int NS>
__device__ __forceinline__ bool tile_inner(int64_t n, int64_t c0) {
  return c0 >= 3 && c0 + NS - 4 < n && n < (int64_t(1) << 28);
}

// Tile that touches an end of the instance, slot by slot (with or without
// the four slots past the last thread).
template <int B, int CPT, bool NOEXT = false>
__device__ __forceinline__ void load_tile_edge(const Bufs& bf, const Consts& cs, const View& v,
                                               const StageScal& sc, int64_t c0,
                                               SmemStage<B, CPT>& sm, int& st) {
  constexpr int TB = B * CPT;
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < CPT; ++c) load_slot_edge(bf, cs, v, sc, c0 - 3 + t + c * B, t + c * B, sm, st);
  if (!NOEXT && t < 4) load_slot_edge(bf, cs, v, sc, c0 - 3 + TB + t, TB + t, sm, st);
}

// Phase 1 of a stage tile: stencil data for cells c0-3 .. c0+TB in LDS.
template <int B, int CPT>
__device__ __forceinline__ void stage_load(const Bufs& bf, const Consts& cs, const View& v,
                                           const StageScal& sc, int64_t c0,
                                           SmemStage<B, CPT>& sm, int& st) {
  constexpr int TB = B * CPT;
  const int t = threadIdx.x;
  if (tile_inner<TB + 4>(v.n, c0)) {
    if (sc.s == 1)
      load_tile_inner<B, CPT, true>(bf, v, sc, c0, sm, st);
    else
      load_tile_inner<B, CPT, false>(bf, v, sc, c0, sm, st);
  } else {
    load_tile_edge<B, CPT>(bf, cs, v, sc, c0, sm, st);
  }
}

// Value of lane (lane - 1) of a double (lane 0 keeps its own): two DPP row
// moves with the wave-wide right shift by one lane, no LDS traffic.
__device__ __forceinline__ double shfl_prev(double x, int lane) {
  (void)lane;
  const long long u = __double_as_longlong(x);
  const int lo0 = (int)(u & 0xffffffffll), hi0 = (int)(u >> 32);
  const int lo = __builtin_amdgcn_update_dpp(lo0, lo0, 0x138, 0xf, 0xf, false);  // wave_shr:1
  const int hi = __builtin_amdgcn_update_dpp(hi0, hi0, 0x138, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Phases 2-4 of a stage tile (the stencil data is in LDS and visible to the
// whole work-group): reconstruction and limiter per cell, interface fluxes,
// residual split and stage combination of the owned cells, and the tile's
// reductions.  Thread t handles the tile cells t + c B, c < CPT.  NR tile
// cells are reconstructed (NR - 2 owned): TB with the four extra stencil
// slots loaded, TB - 4 without them.
template <int B, int CPT, int NR = B * CPT, int SCH = SCH_SPECIAL>
__device__ __forceinline__ StageRes stage_compute(const Bufs& bf, const Consts& cs, const View& v,
                                                  const StageScal& sc, int64_t c0,
                                                  SmemStage<B, CPT>& sm, uint8_t* cls_inst,
                                                  int st, int t) {
  constexpr bool HR = (SCH & 3) == SCH_HYDRO;
  constexpr bool NWB = (SCH & 3) == SCH_NONWB;
  constexpr bool split = (SCH & SCH_SPLIT) != 0;
  constexpr int TB = B * CPT;
  constexpr int NW = B / 64;
  const int lane = t & 63, wv = t >> 6;
  // 2. reconstruct tile cell i (cell j = c0 - 1 + i; cells -1 and n are ghosts
  // for the end faces); one cell after the other.  The left state of the face
  // at node j is the right trace of cell j-1: from the previous lane, or for
  // lane 0 through LDS after the barrier.
  double rint[CPT], ebar[CPT], mbar[CPT], bbar[CPT], Jj[CPT];
  double tl0[CPT], tl1[CPT], tl2[CPT], tp0[CPT], tp1[CPT], tp2[CPT];
  unsigned n0 = 0, n1 = 0, n2 = 0, nl = 0, nn = 0;
  // tile-local bounds (work-group uniform): tile cell i is cell c0 - 1 + i, so
  // it is a real cell or an end ghost for i <= iact, owned for 1 <= i <= iown;
  // ighr is the tile index of the right ghost (cell n), if in the tile
  const int64_t nrel = v.n - c0;
  static_assert(NR == TB || NR == TB - 4, "tile cells reconstructed");
  const int iact = (int)(nrel + 1 < NR - 1 ? nrel + 1 : NR - 1);
  const int iown = (int)(nrel < NR - 2 ? nrel : NR - 2);
  const int ighr = (nrel + 1 < NR) ? (int)(nrel + 1) : -1;
  const bool lghost = c0 == 0;
  uint8_t* cls_tile = cls_inst ? cls_inst + c0 : nullptr;  // tile cell i at [i - 1]
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int i = t + c * B;
    const bool active = i <= iact;
    const bool owned = (i >= 1) && (i <= iown);
    int cls_owned = -1;
    bool lim_owned = false, neg_cell = false;
    rint[c] = 0.0; ebar[c] = 0.0; mbar[c] = 0.0; bbar[c] = 0.0; Jj[c] = 1.0;
    double hR = 0.0, mR = 0.0, bR = 0.0;
    tl0[c] = 0.0; tl1[c] = 0.0; tl2[c] = 0.0;
    if (active) {
      CellRecon o;
      const double* se = sm.u.in.e + i;
      const double* sb = sm.u.in.b + i;
      double h5[5], v5[5];
      // indicator variable: h (fb = 1) or eta (fb = 0), exact either way
      const double fb = (cs.flags & F_BETA_FROM_H) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        h5[k] = se[k] - sb[k];
        v5[k] = fma(-fb, sb[k], se[k]);
      }
      const double hbar = h5[2];
      ebar[c] = se[2]; mbar[c] = sm.u.in.m[i + 2]; bbar[c] = sb[2]; Jj[c] = sm.u.in.J[i + 2];
      const double Dx = (cs.flags & F_BETA_LOCAL) ? Jj[c] : sc.dx;
      if (NWB)
        recon_cell_char(se, sm.u.in.m + i, sb, sm.u.in.J + i, sm.u.in.iJ[i + 2], Dx, cs.weno_eps,
                        cs.g, cs.dry_eps, o, split);
      else
        recon_cell<HR>(v5, h5, sm.u.in.m + i, sb, sm.u.in.J + i, sm.u.in.iJ[i + 2], Dx,
                       cs.weno_eps, ebar[c], o, split);
      const int lim = limit_cell(hbar, mbar[c], cs.pp_eps, o, !(cs.flags & F_NO_HU_LIMIT), NWB);
      // HR: the cell's hydrostatic source from its limited traces (eta kept by
      // the limiter) and the interior values; NWB: the source integral; else
      // the special-source term
      rint[c] = HR ? hydro_source(cs.g, o.hL + o.bL, o.e1, o.e2, o.hR + o.bR, o.bL, o.b1, o.b2, o.bR)
                   : o.rint;
      if (owned) {
        cls_owned = o.cls;
        lim_owned = lim != 0;
        if (hbar < -cs.pp_eps) st |= SB_NEGDEPTH;
        if (cls_tile) cls_tile[i - 1] = (uint8_t)o.cls;
        if (bf.ccount) {
          const int64_t g = v.co + c0 - 1 + i;
          bf.ccount[(int64_t)o.cls * bf.S + g] += 1u;
          bf.csig[g] = bf.csig[g] * CLS_SIG_MUL + (unsigned long long)(o.cls + 1);
        }
      }
      if (o.negw && (owned || (lghost && i == 0) || i == ighr)) {
        neg_cell = true;
        if (!split) st |= SB_NEGWEIGHT;  // split weights: counted, not an error
      }
      tl0[c] = o.hL; tl1[c] = o.mL; tl2[c] = o.bL;
      hR = o.hR; mR = o.mR; bR = o.bR;
    }
    tp0[c] = shfl_prev(hR, lane); tp1[c] = shfl_prev(mR, lane); tp2[c] = shfl_prev(bR, lane);
    if (lane == 63) {
      sm.xr[c * NW + wv][0] = hR; sm.xr[c * NW + wv][1] = mR; sm.xr[c * NW + wv][2] = bR;
    }
    // counters: one ballot per wave
    n0 += (unsigned)__popcll(__ballot(cls_owned == 0));
    n1 += (unsigned)__popcll(__ballot(cls_owned == 1));
    n2 += (unsigned)__popcll(__ballot(cls_owned == 2));
    nl += (unsigned)__popcll(__ballot(lim_owned));
    nn += (unsigned)__popcll(__ballot(neg_cell));
    // keep the reconstructions of different cells apart in the schedule (register pressure)
    if (CPT > 1) __builtin_amdgcn_sched_barrier(0);
  }
  lds_sync();
  // 3. face at node j of tile cell i (between cells j-1 and j), i = 1 .. TB-1
  // LF speed: over the limited face traces, or (ALPHA_CELLAVG) over the cell
  // averages of the stage input and the two node speeds of each owned cell
  const bool a_cell = (cs.flags & F_ALPHA_CELLAVG) != 0;
  double fspeed = 0.0;
  double fsl[CPT], fsr[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int i = t + c * B;
    fsl[c] = -1.0; fsr[c] = -1.0;
    if (i >= 1 && i <= iact) {
      if (lane == 0) {
        const int q = c * NW + wv - 1;
        tp0[c] = sm.xr[q][0]; tp1[c] = sm.xr[q][1]; tp2[c] = sm.xr[q][2];
      }
      if (HR) {
        // momentum flux as seen by the left cell (fl[1]) and by the right one (fl[6])
        FaceHR f;
        face_flux_hydro(tp0[c], tp1[c], tp2[c], tl0[c], tl1[c], tl2[c], sm.wn[i + 2], cs.g,
                        cs.dry_eps, f);
        sm.u.fl[0][i] = f.Fc1; sm.u.fl[1][i] = f.Fc2 + f.cl; sm.u.fl[2][i] = f.Gc;
        sm.u.fl[3][i] = f.je; sm.u.fl[4][i] = f.jm; sm.u.fl[5][i] = f.jb;
        sm.u.fl[6][i] = f.Fc2 + f.cr;
        if (!a_cell) fspeed = vmax(fspeed, f.speed);
        fsl[c] = f.sl;
        fsr[c] = f.sr;
      } else {
        Face f;
        face_flux(tp0[c], tp1[c], tp2[c], tl0[c], tl1[c], tl2[c], sm.wn[i + 2], cs.g, cs.dry_eps, f);
        // the g/2 b^2 part of the special source joins the momentum flux at the
        // face (one LDS array less; still water still cancels to round-off)
        sm.u.fl[0][i] = f.Fc1;
        sm.u.fl[1][i] = NWB ? f.Fc2 : f.Fc2 - 0.5 * cs.g * f.B2;
        sm.u.fl[2][i] = f.Gc;
        sm.u.fl[3][i] = f.je; sm.u.fl[4][i] = f.jm; sm.u.fl[5][i] = f.jb; sm.u.fl[6][i] = f.B1;
        if (!a_cell) fspeed = vmax(fspeed, f.speed);
        fsl[c] = f.sl;
        fsr[c] = f.sr;
      }
    }
  }
  lds_sync();
  // 4. owned cells: residual split, stage combination
  double maxJ = 0.0;
  const int64_t gt = v.co + c0 - 1;  // global index of tile cell 0
  const int64_t NS = bf.S;
  double* Po = ((sc.s == 2) ? bf.P1 : bf.P0) + gt;
  double* Do = ((sc.s == 2) ? bf.D1 : bf.D0) + gt;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int i = t + c * B;
    if ((i >= 1) && (i <= iown)) {
      const double g = cs.g;
      const double(*fl)[TB] = sm.u.fl;
      const double eb = ebar[c], mb = mbar[c], bb = bbar[c], Jc = Jj[c];
      const double Ae = -(fl[0][i + 1] - fl[0][i]);
      const double Am = HR ? -(fl[1][i + 1] - fl[6][i]) + rint[c]
                           : (NWB ? -(fl[1][i + 1] - fl[1][i]) + rint[c]
                                  : -(fl[1][i + 1] - fl[1][i]) - g * eb * (fl[6][i + 1] - fl[6][i]) -
                                        g * rint[c]);
      const double Ab = -(fl[2][i + 1] - fl[2][i]);
      const double De = 0.5 * (fl[3][i + 1] - fl[3][i]);
      const double Dm = 0.5 * (fl[4][i + 1] - fl[4][i]);
      const double Db = 0.5 * (fl[5][i + 1] - fl[5][i]);
      double Pe, Pm, Pb;
      if (sc.s == 1) {
        Pe = Jc * eb + sc.dt * Ae;
        Pm = Jc * mb + sc.dt * Am;
        Pb = Jc * bb + sc.dt * Ab;
      } else {
        Pe = sm.qn[0][i + 2] + sc.bs * (Jc * eb + sc.dt * Ae);
        Pm = sm.qn[1][i + 2] + sc.bs * (Jc * mb + sc.dt * Am);
        Pb = sm.qn[2][i + 2] + sc.bs * (Jc * bb + sc.dt * Ab);
      }
      Po[i] = Pe; (Po + NS)[i] = Pm; (Po + 2 * NS)[i] = Pb;
      Do[i] = De; (Do + NS)[i] = Dm; (Do + 2 * NS)[i] = Db;
      if (bf.dump.q) {
        const int64_t o = (int64_t)(3 * (sc.s - 1)) * NS + gt + i;
        bf.dump.q[o] = eb; bf.dump.q[o + NS] = mb; bf.dump.q[o + 2 * NS] = bb;
      }
      if (a_cell) {
        const double hc = eb - bb;
        const double uc = hc > cs.dry_eps ? mb * frcp(hc) : 0.0;
        const double du = vmax(fabs(uc - sm.wn[i + 2]), fabs(uc - sm.wn[i + 3]));
        fspeed = vmax(fspeed, du + fsqrt(g * vmax(hc, 0.0)));
      }
      const double Jnext = sm.Jx[i + 2];
      maxJ = vmax(maxJ, Jnext);
      if (!(Jnext > 0.0)) st |= SB_MESH;
    }
  }
  // per-wave counts and status bits (wave-uniform), plain LDS stores
  unsigned stw = 0u;
#pragma unroll
  for (int bit = 1; bit <= SB_SEQUENCE; bit <<= 1)
    if (__ballot((st & bit) != 0)) stw |= (unsigned)bit;
  if (lane == 0) {
    sm.cntw[wv][0] = n0; sm.cntw[wv][1] = n1; sm.cntw[wv][2] = n2;
    sm.cntw[wv][3] = nl; sm.cntw[wv][4] = nn; sm.cntw[wv][5] = stw;
  }
  double rv[2] = {fspeed, maxJ};
  const int op[2] = {0, 0};
  block_reduce<B, 2>(rv, op, sm.red);
  StageRes res;
  res.alpha = rv[0];
  res.maxJ = rv[1];
  res.akey = 0.0;
  if (bf.dump.akey) {
    // first face trace of the tile (left trace first) whose speed is the tile's alpha
    double kmin = 1e300;
#pragma unroll
    for (int c = CPT - 1; c >= 0; --c) {
      const double j2 = 2.0 * (double)(c0 - 1 + t + c * B);
      if (fsr[c] == rv[0]) kmin = j2 + 1.0;
      if (fsl[c] == rv[0]) kmin = j2;
    }
    double kv[1] = {kmin};
    const int kop[1] = {1};
    block_reduce<B, 1>(kv, kop, sm.red);
    res.akey = kv[0];
  }
  res.ncls0 = 0u; res.ncls1 = 0u; res.ncls2 = 0u; res.nlim = 0u; res.nneg = 0u;
  unsigned sta = 0u;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    res.ncls0 += sm.cntw[w][0]; res.ncls1 += sm.cntw[w][1]; res.ncls2 += sm.cntw[w][2];
    res.nlim += sm.cntw[w][3]; res.nneg += sm.cntw[w][4];
    sta |= sm.cntw[w][5];
  }
  res.status = (int)sta;
  lds_sync();
  return res;
}

// One stage over the tile of owned cells [c0, c0 + TB - 2) of one instance.
template <int B, int CPT, int SCH>
__device__ __forceinline__ StageRes stage_tile(const Bufs& bf, const Consts& cs, const View& v,
                                               const StageScal& sc, int64_t c0,
                                               SmemStage<B, CPT>& sm, uint8_t* cls_inst) {
  int st = 0;
  stage_load<B, CPT>(bf, cs, v, sc, c0, sm, st);
  lds_sync();
  return stage_compute<B, CPT, B * CPT, SCH>(bf, cs, v, sc, c0, sm, cls_inst, st, (int)threadIdx.x);
}

// Scalars of stage s of instance i read through the constant address space
// (scalar loads; no instance record is written while a stage kernel runs).
__device__ __forceinline__ StageScal stage_scal_const(const Inst* inst, int i, int s) {
  typedef const __attribute__((address_space(4))) Inst* cinst;
  const cinst I = (cinst)inst + i;
  StageScal sc;
  sc.s = s;
  sc.dt = I->dt;
  sc.as = s == 1 ? 0.0 : (s == 2 ? 0.75 : 1.0 / 3.0);
  sc.bs = s == 1 ? 1.0 : (s == 2 ? 0.25 : 2.0 / 3.0);
  sc.cprev = s == 1 ? 0.0 : (s == 2 ? 1.0 : 0.25) * sc.dt * I->alpha[s == 1 ? 0 : s - 2];
  sc.dx = I->dx[s - 1];
  sc.wsc = I->wscale;
  return sc;
}

// Phase 1 of a ghost-free tile of the stage-launch engine, whose instance
// offsets come with the tile: the loads of the tile are issued before the
// instance record is read, so the two latencies overlap.  The instance
// scalars are read through the constant address space (scalar loads whose
// wait does not wait for the tile's vector loads): no instance record is
// written while a stage kernel runs.  par is the parity of the step, the same
// for every active instance of a batch (all of them start together and step
// together).  Returns false for an inactive instance.
template <int B, int CPT, bool FIRST, bool NOEXT>
__device__ __forceinline__ bool stage_load_direct(const Bufs& bf, const View& v, int inst, int s,
                                                  int par, int64_t c0, SmemStage<B, CPT>& sm,
                                                  int& st) {
  constexpr int TB = B * CPT;
  const int t = threadIdx.x;
  const double* P = ((s == 2) ? bf.P0 : bf.P1) + v.co;
  const double* D = ((s == 2) ? bf.D0 : bf.D1) + v.co;
  RawSlot r[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
    r[c] = raw_inner<FIRST>(bf, v, P, D, (unsigned)(c0 - 3 + t + c * B) * 8u);
  const bool ext = !NOEXT && t < 4;
  RawSlot rx;
  if (ext) rx = raw_inner<FIRST>(bf, v, P, D, (unsigned)(c0 - 3 + TB + t) * 8u);
  typedef const __attribute__((address_space(4))) Inst* cinst;
  const cinst I = (cinst)bf.inst + inst;
  if (!I->active) return false;
  // an instance out of step with the batch would have read the wrong nodes
  if ((int)(I->steps & 1) != par) st |= SB_SEQUENCE;
  const StageScal sc = stage_scal_const(bf.inst, inst, s);
#pragma unroll
  for (int c = 0; c < CPT; ++c) put_raw(sc, t + c * B, r[c], sm, st);
  if (ext) put_raw(sc, TB + t, rx, sm, st);
  return true;
}

// Step epilogue over cells [c0, c0+B): q^{n+1}, x^{n+1}, and the reductions
// that size the next step.
struct FinalRes {
  double speed, minJ, maxJ, hmin;
  int status;
};

// Raw values of cell j: its two nodes and node speeds, P and D of stage 3.
struct FinalRaw {
  double x0, x1, w0, w1, p0, p1, p2, d0, d1, d2;
};

__device__ __forceinline__ FinalRaw final_load(const Bufs& bf, const View& v, int64_t j) {
  FinalRaw r;
  r.x0 = v.x[j]; r.x1 = v.x[j + 1];
  r.w0 = bf.w[v.no + j]; r.w1 = bf.w[v.no + j + 1];
  const int64_t gi = v.co + j;
  r.p0 = bf.P0[gi]; r.p1 = bf.P0[bf.S + gi]; r.p2 = bf.P0[2 * bf.S + gi];
  r.d0 = bf.D0[gi]; r.d1 = bf.D0[bf.S + gi]; r.d2 = bf.D0[2 * bf.S + gi];
  return r;
}

// New state and nodes of cell j (< n) from its raw values; the cell's part
// of the reductions and its status bits.
__device__ __forceinline__ void final_cell(const Bufs& bf, const Consts& cs, const View& v,
                                           int64_t j, const FinalRaw& r, double dt, double alpha3,
                                           double wsc, double& speed, double& minJ, double& maxJ,
                                           double& hmin, int& st) {
  const double x0 = r.x0, x1 = r.x1;
  const double w0 = r.w0 * wsc, w1 = r.w1 * wsc;
  const double Jn = x1 - x0, dw = w1 - w0;
  const double J1 = Jn + dt * dw;
  const double J2 = 0.75 * Jn + 0.25 * (J1 + dt * dw);
  const double J3 = (1.0 / 3.0) * Jn + (2.0 / 3.0) * (J2 + dt * dw);
  const double c = (2.0 / 3.0) * dt * alpha3;
  const int64_t gi = v.co + j;
  const double iJ3 = frcp(J3);
  const double xn0 = x0 + dt * w0, xn1 = x1 + dt * w1;
  const double e = (r.p0 + c * r.d0) * iJ3;
  const double m = (r.p1 + c * r.d1) * iJ3;
  // an analytic bottom: its projection onto the new cell (eq. (3.16))
  const double b = cs.bottom != BOT_ALE ? bottom_avg(cs, xn0, xn1) : (r.p2 + c * r.d2) * iJ3;
  bf.eta[gi] = e; bf.m[gi] = m; bf.b[gi] = b;
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
  speed = fabs(u) + fsqrt(cs.g * vmax(h, 0.0));
  minJ = Jnew; maxJ = Jnew; hmin = h;
  if (!(J3 > 0.0) || !(Jnew > 0.0)) st |= SB_MESH;
  if (!isfinite(e) || !isfinite(m) || !isfinite(b)) st |= SB_NONFINITE;
  if (h < -cs.pp_eps) st |= SB_NEGDEPTH;
}

// Reductions of an epilogue tile; the status bits through one ballot per
// bit and wave.  red holds B / 64 * 8 doubles (its first slots are reused).
template <int B>
__device__ __forceinline__ FinalRes final_reduce(double speed, double minJ, double maxJ,
                                                 double hmin, int st, double* red) {
  constexpr int NW = B / 64;
  const int t = threadIdx.x;
  unsigned stw = 0u;
#pragma unroll
  for (int bit = 1; bit <= SB_SEQUENCE; bit <<= 1)
    if (__ballot((st & bit) != 0)) stw |= (unsigned)bit;
  double rv[4] = {speed, minJ, maxJ, hmin};
  const int op[4] = {0, 1, 0, 1};
  block_reduce<B, 4>(rv, op, red);
  __shared__ unsigned stws[NW];
  if ((t & 63) == 0) stws[t >> 6] = stw;
  __syncthreads();
  FinalRes r;
  r.speed = rv[0]; r.minJ = rv[1]; r.maxJ = rv[2]; r.hmin = rv[3];
  unsigned sa = 0u;
#pragma unroll
  for (int w = 0; w < NW; ++w) sa |= stws[w];
  r.status = (int)sa;
  __syncthreads();
  return r;
}

template <int B>
__device__ __forceinline__ FinalRes final_tile(const Bufs& bf, const Consts& cs, const View& v,
                                               double dt, double alpha3, double wsc, int64_t c0,
                                               double* red) {
  const int64_t j = c0 + threadIdx.x;
  int st = 0;
  double speed = 0.0, minJ = INFINITY, maxJ = 0.0, hmin = INFINITY;
  if (j < v.n) {
    const FinalRaw r = final_load(bf, v, j);
    final_cell(bf, cs, v, j, r, dt, alpha3, wsc, speed, minJ, maxJ, hmin, st);
  }
  return final_reduce<B>(speed, minJ, maxJ, hmin, st, red);
}

// Shape function of the prescribed mesh map.
// PAPER: eq. (5.1).  ALIGNED: eq. (5.14), which also vanishes at the step
// bottom's jump points bp[1], bp[2] (nodes placed there never move).
__device__ __forceinline__ double mesh_shape(const Consts& cs, double xi, double x0, double x1) {
  if (cs.mesh == MESH_SINE) return sin(2.0 * M_PI * cs.mesh_k * xi);
  const double L = x1 - x0;
  const double q = (xi - x1) * (xi - x0);
  if (cs.mesh == MESH_ALIGNED) return q * (xi - cs.bp[1]) * (xi - cs.bp[2]) / (3.0 * L * L * L * L);
  return q / (3.0 * L * L);
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
    if (prescribed(cs.mesh))
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
