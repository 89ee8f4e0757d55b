/*
 * alew.h -- C ABI of the MI355X (gfx950) library for the 1D well-balanced
 * ALE-WENO hybrid finite-volume scheme of Zhang, Xia & Xu, "Structure-preserving
 * finite volume arbitrary Lagrangian-Eulerian WENO schemes for the shallow water
 * equations" (special source-term variant, Sec. 4.2; the hydrostatic
 * reconstruction of Sec. 4.1 and the scheme of Sec. 3 without well-balancing
 * by flag), and its 2D tensor-product extension (alew2d_*, below).
 *
 * One time step is the modified SSP-RK3 of eq. (3.14) with the width recurrence
 * of eq. (3.15).  Each stage evaluates the semi-discrete right-hand side
 * eq. (3.11)-(3.12): hybrid WENO reconstruction with the smooth/transition/
 * non-smooth detector (Sec. 2.2, eq. (2.7)-(2.10)), the positivity limiter of
 * eq. (3.20)-(3.21) with Remark 4.1, the Lax-Friedrichs flux of F(q) - w q with
 * the global speed of eq. (3.13), the ALE bottom flux of eq. (3.17) and the
 * well-balanced source of eq. (4.7)-(4.10).  Everything is FP64.
 *
 * Conventions shared by every entry point
 *  - Array arguments are DEVICE pointers to contiguous FP64 (or int64/uint8)
 *    data unless the comment says "host".  The caller owns them; the library
 *    never frees or keeps them after the call returns.
 *  - State arrays are cell averages: h (depth), hu (discharge), b (bottom), one
 *    value per cell.  Nodes x hold ncell+1 positions per instance; xi holds the
 *    reference node positions of the prescribed mesh map
 *    X(xi,t) = xi + mesh_A * S(xi) * sin(mesh_omega * t).
 *  - Ragged batches are packed: instance i owns cells [cell_off[i],
 *    cell_off[i+1]) and nodes [cell_off[i] + i, cell_off[i+1] + i].
 *  - Work is enqueued on the context's HIP stream.  Calls that return stats
 *    synchronise that stream before returning.
 *  - Errors: argument errors return at once (ALEW_E_ARG); errors found on the
 *    device (non-positive width, negative mean depth below -pp_eps, non-finite
 *    values, negative linear weight) stop the affected instance and are
 *    returned by the call (and per instance in stats).  alew_last_error()
 *    returns a message for the calling thread's last non-OK return.
 *  - One context per host thread and stream; contexts are independent.
 */
#ifndef ALEW_H
#define ALEW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct alew_ctx alew_ctx;

typedef enum {
  ALEW_OK = 0,
  ALEW_E_ARG = 1,         /* bad argument (NULL, size, enum, ...)                  */
  ALEW_E_MESH = 2,        /* a cell width <= 0 (assumption (A1) of Sec. 2.1)        */
  ALEW_E_NEGDEPTH = 3,    /* a mean depth below -pp_eps (Property 3.1 violated)     */
  ALEW_E_NONFINITE = 4,   /* NaN or Inf in the state                               */
  ALEW_E_HIP = 5,         /* HIP runtime error                                     */
  ALEW_E_NOMEM = 6,       /* device allocation failed                              */
  ALEW_E_UNSUPPORTED = 7, /* combination not supported by this entry point; also an
                           * instance of a batch out of step with the others (the
                           * stage kernels take one node-buffer parity per launch) */
  ALEW_E_NEGWEIGHT = 8,   /* a negative linear weight d_r (Sec. 2.2, after Step 4)
                           * without ALEW_F_SPLIT                                 */
  ALEW_E_CAPACITY = 9     /* the step-size buffer of alew_run (dts or dt_log) holds
                           * fewer than the steps an instance needed: the instance
                           * stopped there, before its t_end / max_steps            */
} alew_status;

enum { ALEW_BC_PERIODIC = 0, ALEW_BC_TRANSMISSIVE = 1, ALEW_BC_REFLECTIVE = 2 };

/* Mesh motion.  GIVEN: node speeds w supplied by the caller (alew_step only).
 * SINE: S(xi) = sin(2 pi mesh_k xi).  PAPER: S(xi) = (xi - xi_N)(xi - xi_0) /
 * (3 (xi_N - xi_0)^2), eq. (5.1) with mesh_A = 1, mesh_omega = 2 pi / t_end.
 * ALIGNED: S(xi) = (xi - xi_N)(xi - xi_0)(xi - p1)(xi - p2) / (3 (xi_N - xi_0)^4)
 * with p1 = bottom_p[1], p2 = bottom_p[2] (the STEP bottom's jump points),
 * eq. (5.14) of Example 5.5: a node placed on a jump point stays on it, so the
 * projection of eq. (3.16) never averages across the jump (the cell count of
 * the example's domain [0, 1500] must be a multiple of 8 for 562.5 and 937.5
 * to be nodes).
 * For SINE, PAPER and ALIGNED the node speed of a step is the chord of eq. (2.1),
 * (X(xi, t+dt) - X(xi, t)) / dt.  FLUID: node speeds follow the fluid (average
 * of the two adjacent cell velocities, two passes of [1/4,1/2,1/4] smoothing,
 * fixed end nodes unless periodic). */
enum {
  ALEW_MESH_GIVEN = 0, ALEW_MESH_SINE = 1, ALEW_MESH_PAPER = 2, ALEW_MESH_FLUID = 3, ALEW_MESH_ALIGNED = 4
};

/* flags */
enum {
  ALEW_F_BETA_LOCAL = 1,  /* Dx in the indicators = the cell's own width instead of
                             the max width of the stage mesh (Sec. 2.2, Step 1)     */
  ALEW_F_BETA_FROM_H = 2, /* indicators on (h, hu) instead of (eta, hu)             */
  ALEW_F_HYDROSTATIC = 4, /* well-balanced scheme with the hydrostatic reconstruction
                             of Sec. 4.1, eq. (4.2)-(4.3), instead of the special
                             source-term treatment of eq. (4.4)-(4.6): at each face
                             h* = max(0, eta - max(b-, b+)) on both sides, the
                             discharge kept, the momentum flux of the starred states
                             plus each cell's pressure correction g/2 (h^2 - h*^2);
                             the source is the integral of -g (eta_h - b_h) b_h' with
                             eta_h, b_h the cubics through the values at the 4
                             Gauss-Lobatto points.  The eta and b equations are those
                             of the default scheme.  Every entry point and engine
                             (alew_step, alew_run, alew_adjoint).                  */
  /* Alternative readings of points the paper leaves open (the defaults are the
   * readings the oracle and the library take without flags):                     */
  ALEW_F_ALPHA_CELLAVG = 8,  /* Lax-Friedrichs speed of eq. (3.13) taken over the cell
                                averages of the stage input instead of the limited
                                face traces: max over the cells j of an instance of
                                max(|u_j - w_{j-1/2}|, |u_j - w_{j+1/2}|) + sqrt(g h_j)
                                (u_j = hu_j / h_j if h_j > dry_eps, else 0); not
                                with alew_adjoint                                     */
  ALEW_F_NO_HU_LIMIT = 16,   /* the positivity limiter of eq. (3.20)-(3.21) scales the
                                h traces (and the b traces through Remark 4.1) only;
                                by default the hu traces are scaled by the same Phi
                                about the cell mean of hu                             */
  ALEW_F_W_TANGENT = 32,     /* prescribed meshes: the node speed of a step is the
                                map's time derivative at the start of the step,
                                A S(xi) omega cos(omega t_n), instead of the chord of
                                eq. (2.1) (nodes then leave the map by O(dt^2) a step) */
  ALEW_F_NONWB = 64          /* the ALE-WENO scheme of Sec. 3 without well-balancing,
                                eq. (3.11)-(3.13): (eta, hu) reconstructed in the local
                                characteristic variables of each cell's mean state (the
                                eigenvectors (1, u -+ c) of the flux Jacobian;
                                component-wise where the mean depth is at most dry_eps),
                                b reconstructed with weights of its own, every variable
                                with its own indicators and detector class (the class
                                reported for a cell is the largest of the three); the
                                source term is the integral of -g (eta - b) b_x over the
                                cell by the 4-point Gauss-Lobatto rule on the unlimited
                                values; the positivity limiter changes h and keeps the b
                                traces.  alew_step and alew_run only; not with
                                ALEW_F_HYDROSTATIC                                     */
  ,
  ALEW_F_SPLIT = 128         /* negative linear weights (the remark after Step 4 of
                                Sec. 2.2): by default a negative weight is reported
                                (ALEW_E_NEGWEIGHT, counted in n_negweight).  With
                                this flag, at a point whose linear weights include a
                                negative one, the nonlinear weights of the
                                transition and non-smooth classes come from the
                                splitting of Shi, Hu & Shu (2002, theta = 3): a
                                positive and a negative group, each with its own
                                nonlinear weights; such cell-stages are counted and
                                the run goes on.  Runs the stage engine in its
                                automatic tile shape.  alew_step and alew_run;
                                alew_adjoint ignores it (and reports)              */
};

/* Bottom topography (Sec. 3.3).  ALE (default): the cell averages of b are a
 * state variable evolved by the ALE scheme of eq. (3.17) from the b the caller
 * passes.  The other kinds give b(x) in closed form, and the cell averages are
 * its L2 projection onto the moving cells, eq. (3.16): at every stage on the
 * stage's mesh (t_n, t_{n+1}, t_{n+1/2}) and at the end of every step on the
 * new mesh; the b array's input values are not used, and it receives the
 * projection onto the final mesh.  Parameters bottom_p[0..3]:
 *   STEP      b = p0 on [p1, p2], 0 elsewhere
 *   GAUSS     b = p0 exp(-p1 (x - p2)^2)
 *   SIN2      b = p0 sin^2(pi p1 x)
 *   BUMP      b = p0 (cos(pi (x - p2) / p1) + 1) for |x - p2| < p1, else 0
 *   PARABOLA  b = p0 (x / p1)^2 */
enum {
  ALEW_BOTTOM_ALE = 0, ALEW_BOTTOM_STEP = 1, ALEW_BOTTOM_GAUSS = 2, ALEW_BOTTOM_SIN2 = 3,
  ALEW_BOTTOM_BUMP = 4, ALEW_BOTTOM_PARABOLA = 5
};

typedef struct {
  double g;          /* gravitational constant (9.812 in Sec. 5)                       */
  double cfl;        /* CFL number of the time-step rule                               */
  double weno_eps;   /* epsilon of eq. (2.7)-(2.8) (1e-6; 1e-9 for Example 5.4)         */
  double pp_eps;     /* positivity epsilon of eq. (3.20) (1e-11)                        */
  double mesh_A, mesh_k, mesh_omega;   /* prescribed mesh map (see above)            */
  double dry_eps;    /* trace depth below which u = hu = 0 in the flux (1e-8)          */
  int32_t bc;        /* ALEW_BC_*                                                      */
  int32_t mesh;      /* ALEW_MESH_*                                                    */
  int32_t flags;     /* ALEW_F_*                                                       */
  int32_t bottom;    /* ALEW_BOTTOM_* (0: evolved by eq. (3.17))                       */
  double bottom_p[4];  /* parameters of the analytic bottom                           */
} alew_params;

typedef struct {
  int64_t steps;          /* time steps taken                                          */
  int64_t n_class[3];     /* cell-stages classified smooth / transition / non-smooth   */
  int64_t n_limited;      /* cell-stages where the positivity limiter acted            */
  int64_t n_negweight;    /* cell-stages with a negative linear weight                  */
  double t;               /* time reached                                               */
  double dt_min, dt_max;  /* step sizes used                                            */
  double h_min;           /* smallest mean depth seen (initial and after every step)    */
  double mass_eta0, mass_eta;  /* sum_j Delta_j eta_j at start and end                  */
  double mass_b0, mass_b;      /* sum_j Delta_j b_j at start and end                    */
  int32_t status;         /* alew_status of this instance                               */
  int32_t pad;
} alew_stats;

/* Launch configuration (normally chosen by the autotuner).
 * engine 0 = automatic (the stage launches), 1 = persistent (one launch runs a
 * whole ragged batch, a work-group per instance, instances taken largest first
 * from a device queue), 2 = stage launches (every tile of every instance in
 * each stage kernel).
 * block: work-group size (64, 128, 256 or 512; 0 = 64 for the stage launches,
 * 256 for the persistent engine).
 * steps_per_launch: persistent engine, steps per launch before control returns to
 * the host (0 = until every instance is done).
 * use_graph: stage-launch engine, replay the launches of a step as a hipGraph.
 * cells_per_thread: stage-launch engine, cells each thread reconstructs per
 * tile (1 or 2; 0 = 2 for block 64, else 1); a tile spans block *
 * cells_per_thread cells.
 * compact_tiles: stage-launch engine: 0 = a stage tile of T = block x
 * cells_per_thread cells loads T + 4 stencil slots (the first four threads load
 * the last four) and owns T - 2 cells (default); 1 = it loads T slots, one per
 * cell a thread handles, and owns T - 6 cells. */
typedef struct {
  int32_t engine;
  int32_t block;
  int32_t steps_per_launch;
  int32_t use_graph;
  int32_t cells_per_thread;
  int32_t compact_tiles;
} alew_launch;

/* Create a context able to run up to max_cells cells in up to max_inst instances.
 * The scratch memory of alew_step and alew_run (state and stage buffers, tile
 * tables and result records: about 120 bytes per cell) is allocated here;
 * alew_step and alew_run never allocate device memory.  alew_adjoint's larger
 * workspace is allocated by alew_adjoint_reserve, or by the first alew_adjoint
 * call that needs more than the context holds.
 * hip_stream: hipStream_t to enqueue on (NULL = default stream). */
alew_status alew_create(alew_ctx** ctx, int64_t max_cells, int64_t max_inst, void* hip_stream);
void alew_destroy(alew_ctx* ctx);
alew_status alew_set_stream(alew_ctx* ctx, void* hip_stream);
alew_status alew_set_launch(alew_ctx* ctx, const alew_launch* launch);
alew_status alew_get_launch(const alew_ctx* ctx, alew_launch* launch);

/* One time step of one instance (eq. (3.14)-(3.15)).
 * h, hu, b [ncell] and x [ncell+1] are updated in place.  xi [ncell+1] is
 * required for SINE/PAPER/ALIGNED meshes; w [ncell+1] is required for GIVEN (node
 * speeds over the step; w[ncell] must equal w[0] when periodic).
 * dt > 0 fixes the step; dt <= 0 selects the CFL rule
 *   dt = cfl * min_j Delta_j / (max_j(|u_j| + sqrt(g h_j)) + max_i |W_i|),
 * W the node speed at t.  If t_end > t the step is clipped to end at t_end.
 * cls [3*ncell] (optional) receives the detector class of every cell at each
 * stage (0 smooth, 1 transition, 2 non-smooth).  stats (host, optional)
 * receives the step statistics; stats->t is the new time.  ncell >= 5. */
alew_status alew_step(alew_ctx* ctx, const alew_params* p, int64_t ncell, double* h, double* hu,
                      double* b, double* x, const double* xi, const double* w, double t, double dt,
                      double t_end, uint8_t* cls, alew_stats* stats);

/* For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid hipMalloc): the step of alew_step without a context and without
 * any allocation.  Its scratch (state and stage buffers, tile tables, result
 * records: about 8.7 MB) is a file-scope device array of the library, one copy
 * per GPU, held until the process ends.  Arguments, results and errors as
 * alew_step; ncell <= 65536 (larger: ALEW_E_ARG).  hip_stream: the stream to
 * enqueue on (NULL = default stream); the call returns after its work on that
 * stream is done.  Every call on a GPU uses that GPU's one array, which keeps
 * the last call's contents; the library serializes the calls on a GPU with a
 * lock, and two calls whose work overlapped on one GPU would race. */
alew_status alew_step_noalloc(const alew_params* p, int64_t ncell, double* h, double* hu, double* b,
                              double* x, const double* xi, const double* w, double t, double dt,
                              double t_end, uint8_t* cls, alew_stats* stats, void* hip_stream);

/* Run a ragged batch of independent instances.
 * cell_off (host) [ninst+1]; h, hu, b, x, xi packed as described above.
 * t0, t_end, max_steps (host) [ninst], each may be NULL: instance i starts at
 * t0[i] (0) and advances until t_end[i] (if > t0[i]) and/or max_steps[i] steps
 * (if > 0).  dts (device, optional) [ninst * dts_stride] fixes the step sizes
 * (the CFL rule is used when NULL).  dt_log (device, optional)
 * [ninst * dts_stride] receives the step sizes used.  With either of them an
 * instance that would need more than dts_stride steps stops after dts_stride
 * steps with ALEW_E_CAPACITY.
 * cls_count, cls_sig (device, optional, both or neither): a record of the
 * detector class (Sec. 2.2, Step 2) of every cell at every stage of the run,
 * accumulated onto what the arrays hold (zero them for a fresh record):
 * cls_count [3 * S] (S = cell_off[ninst]) counts the stages at which cell g
 * was classified smooth (cls_count[g]), transition (cls_count[S + g]) or
 * non-smooth (cls_count[2 S + g]); cls_sig [S] is a signature of the cell's
 * class sequence: at every stage, in time order,
 *     cls_sig[g] = cls_sig[g] * 1099511628211 + class + 1   (mod 2^64),
 * class 0 smooth, 1 transition, 2 non-smooth.
 * stats (host, optional) [ninst].  mesh must be SINE, PAPER, ALIGNED or FLUID. */
alew_status alew_run(alew_ctx* ctx, const alew_params* p, int64_t ninst, const int64_t* cell_off,
                     double* h, double* hu, double* b, double* x, const double* xi,
                     const double* t0, const double* t_end, const int64_t* max_steps,
                     const double* dts, double* dt_log, int64_t dts_stride, uint32_t* cls_count,
                     uint64_t* cls_sig, alew_stats* stats);

/* Discrete adjoint of alew_run with frozen step sizes (prescribed mesh).
 * Forward: from (h0, hu0, b0, x0) at time t0 run nsteps steps of sizes dts
 * (device, [ninst * nsteps]); gauge_h (device, out) [ninst * ngauge] receives the mean
 * depth at the final time of the cell containing gauge_x (device)
 * [ninst * ngauge] (positions in the final mesh).
 * Reverse: with gauge_bar (device) [ninst * ngauge] = dL/d gauge_h, writes
 * dh0, dhu0, db0 (device) [sum ncell] = dL/d (h0, hu0, b0).  The detector class,
 * the limiter's active set and argmin, the argmax of the LF speed, |.| signs and
 * dry cut-offs are frozen to the forward pass.  The forward is checkpointed every
 * ckpt_every steps and recomputed segment by segment (ckpt_every <= 0: 16).
 * gauge_h may be computed without the reverse pass by passing gauge_bar = NULL.
 * Checkpoints and per-step records of one segment live in the context's
 * adjoint workspace (alew_adjoint_reserve); a call that needs more than the
 * workspace holds allocates a larger one first.  ALEW_F_ALPHA_CELLAVG is not
 * supported here (ALEW_E_UNSUPPORTED). */
alew_status alew_adjoint(alew_ctx* ctx, const alew_params* p, int64_t ninst,
                         const int64_t* cell_off, const double* h0, const double* hu0,
                         const double* b0, const double* x0, const double* xi, double t0,
                         int64_t nsteps,
                         const double* dts, int64_t ckpt_every, int64_t ngauge,
                         const double* gauge_x, double* gauge_h, const double* gauge_bar,
                         double* dh0, double* dhu0, double* db0);

/* Allocate alew_adjoint's workspace ahead of time for runs of up to nsteps
 * steps with checkpoints every ckpt_every steps (<= 0: 16) and up to ngauge
 * gauges per instance, at the context's max_cells and max_inst.  A later
 * alew_adjoint call within these sizes allocates nothing.  The workspace is
 * about (3 + 26 ckpt_every) * 8 bytes per cell plus 40 bytes per cell for each
 * checkpoint. */
alew_status alew_adjoint_reserve(alew_ctx* ctx, int64_t nsteps, int64_t ckpt_every,
                                 int64_t ngauge);

/* Device time of the compute launches of the last alew_step/alew_run on this
 * context, measured with HIP events recorded on the context's stream around
 * them: the persistent kernel launches (engine 1, launches = kernel launches)
 * or the step sequences (engine 2, launches = graph or sequence launches).
 * ms and launches are host pointers. */
alew_status alew_last_timing(const alew_ctx* ctx, double* ms, int64_t* launches);

/* Per-kernel timing of the stage-launch engine.  With on != 0, later
 * alew_step/alew_run calls launch the step sequence without a graph and record
 * a HIP event pair on the context's stream around every stage launch (all
 * stage kernels of one RK stage) and every step-epilogue launch (new state, nodes and
 * step-size reductions).  It adds an event pair per launch and is off by
 * default. */
alew_status alew_set_kernel_timing(alew_ctx* ctx, int on);

/* Totals of the last call with kernel timing on.  which: 0 = stage launches,
 * 1 = step epilogues, 2, 3, 4 = the stage launches of RK stage 1, 2, 3 (stage 1
 * reads the step's state; stages 2 and 3 also the previous stage's partial
 * updates).  ms: summed device time; launches: number of launches;
 * cells: summed batch cells over those launches (every launch covers the whole
 * batch; tiles of instances already finished return at once).  Host pointers. */
alew_status alew_kernel_timing(const alew_ctx* ctx, int which, double* ms, int64_t* launches,
                               double* cells);

/* ------------------------------------------------------------------------
 * 2D extension: the special source-term scheme by default (Sec. 2-4 in two
 * dimensions: eq. (3.11)-(3.15) with the 2D flux, eq. (4.7)-(4.10) with the
 * 4 x 4 Gauss-Lobatto rule on the cell and 4 Gauss-Lobatto points per edge),
 * the hydrostatic reconstruction or the scheme without well-balancing by flag
 * (see alew2d_params.flags below), on a
 * tensor-product moving mesh of rectangles: node i of the x-direction at
 * x_i(t) = xi_i + Ax sin(2 pi kx xi_i) sin(omx t), node j of the y-direction at
 * y_j(t) = yi_j + Ay sin(2 pi ky yi_j) sin(omy t); the node speeds of a step
 * are the chords (X(t + dt) - X(t)) / dt.  The reconstruction runs dimension by
 * dimension (Sec. 2.2 along x on cell averages, then along y on the line
 * values): indicators summed over (eta, hu, hv), one class per sweep (the
 * cell's class is the largest of its x-sweep's and its four y-sweeps').
 * Step size (the CFL condition eq. (3.19) sums over the four edges):
 * dt = cfl / ((s + Wx) / min dx + (s + Wy) / min dy), Wx, Wy the largest node
 * speeds of each direction at t, s the larger of the means' largest
 * max(|u|, |v|) + sqrt(g h) and the previous step's Lax-Friedrichs alpha
 * (eq. (3.13), on the traces; none at a call's first step).  Positivity: the
 * limiter of eq. (3.20) split by direction as eq. (3.21)-(3.22) (the bottom
 * and top edge traces limited together, the left and right ones together,
 * each with the interior mean from the Gauss-Lobatto identity and
 * eps = min(1e-11, hbar); hu, hv towards their means by the same factor, b
 * following eta); traces with h <= dry_eps carry zero discharge; a mean depth
 * below -1e-11 is ALEW_E_NEGDEPTH.  flags = ALEW_F_HYDROSTATIC selects the
 * hydrostatic reconstruction of Sec. 4.1 (eq. (4.4)-(4.6)) instead of the
 * special source term: at each edge point the momentum fluxes of the starred
 * states (h* = max(0, eta - max(b-, b+)), discharges kept) and each cell's
 * pressure correction g/2 (h^2 - h*^2) of its own trace; the cell source is the
 * 1D hydrostatic source (the cubic through the 4 Gauss-Lobatto values of b,
 * eta - b times its derivative, by the 4-point rule) on every Gauss-Lobatto
 * line of the cell, weighted by the other direction's rule.  flags =
 * ALEW_F_NONWB selects the scheme of Sec. 3 without well-balancing: in each
 * sweep (eta, hu, hv) in the local characteristic variables of the sweep
 * direction (the flux Jacobian's eigenvectors at the cell's mean state; the
 * identity where the mean depth is at most dry_eps), each characteristic
 * variable and b with their own indicators, class and weights; the plain
 * flux; the source -g h grad b by the 4 x 4 Gauss-Lobatto rule; the limiter
 * keeps the bottom traces.  Both flags together are ALEW_E_ARG, other flags
 * ALEW_E_UNSUPPORTED.  State arrays are [ny][nx] (cell (i, j) at
 * i + nx j), device FP64; nodes x [nx + 1], y [ny + 1] in place; reference
 * nodes xi [nx + 1], yi [ny + 1].
 * ------------------------------------------------------------------------ */
typedef struct alew2d_ctx alew2d_ctx;

typedef struct {
  double g, cfl, weno_eps, dry_eps; /* 9.812, 0.6, 1e-6, 1e-8                      */
  double Ax, kx, omx;               /* x-node map                                  */
  double Ay, ky, omy;               /* y-node map                                  */
  int32_t bcx, bcy;                 /* ALEW_BC_PERIODIC or ALEW_BC_TRANSMISSIVE    */
  int32_t flags, pad;               /* 0, ALEW_F_HYDROSTATIC or ALEW_F_NONWB        */
  double Vx, Vy;                    /* uniform node translation: x_i(t) adds Vx t,
                                       y_j(t) adds Vy t (Example 5.7's w = (1, 0)) */
} alew2d_params;

typedef struct {
  int64_t steps;
  double t, dt_min, dt_max;
  double mass0, mass_b0, mass, mass_b; /* sums of area x eta and area x b, start / end */
  int64_t n_class[3];                  /* cells x stages per class over the run        */
  int64_t n_limited;                   /* cells x stages where the limiter acted       */
  int32_t status, pad;
} alew2d_stats;

/* Context for grids up to max_nx x max_ny cells (max_nx <= 2^24, max_ny <=
 * 65535, product <= 2^26): allocates about 340 bytes per cell of device
 * workspace; alew2d_run allocates nothing. */
alew_status alew2d_create(alew2d_ctx** ctx, int64_t max_nx, int64_t max_ny, void* hip_stream);
void alew2d_destroy(alew2d_ctx* ctx);
alew_status alew2d_set_stream(alew2d_ctx* ctx, void* hip_stream);
/* rows: rows of cells per y-sweep wavefront (default 16); check_every: steps
 * between the host's stop checks of a run with t_end (default 8). */
alew_status alew2d_set_launch(alew2d_ctx* ctx, int32_t rows, int32_t check_every);

/* Advance from t0 until t_end (if > t0) and/or max_steps steps (if > 0).
 * h, hu, hv, b [nx * ny] and x, y are updated in place.  cls (device, optional)
 * [3 * nx * ny] receives the classes of every cell at the three stages of the
 * last step; cls_count (device, optional) [3 * nx * ny] and cls_sig (device,
 * optional) [nx * ny] accumulate a record of every stage as alew_run's do.
 * stats (host, optional).  Errors: ALEW_E_ARG / ALEW_E_UNSUPPORTED before any
 * work; ALEW_E_MESH (a non-positive area), ALEW_E_NEGDEPTH, ALEW_E_NONFINITE or
 * ALEW_E_NEGWEIGHT
 * (a negative linear weight on a stage mesh; not split in 2D) stop the run
 * after the step that met them, with the state of that step in the arrays. */
alew_status alew2d_run(alew2d_ctx* ctx, const alew2d_params* p, int64_t nx, int64_t ny,
                       double* h, double* hu, double* hv, double* b, double* x, double* y,
                       const double* xi, const double* yi, double t0, double t_end,
                       int64_t max_steps, uint8_t* cls, uint32_t* cls_count, uint64_t* cls_sig,
                       alew2d_stats* stats);

/* Device time (ms, host pointer) of the last alew2d_run, from HIP events on the
 * context's stream around its launches. */
alew_status alew2d_last_timing(const alew2d_ctx* ctx, double* ms);

/* Per-kernel timing: with on != 0 later alew2d_run calls record a HIP event
 * pair on the context's stream around every launch of a step (off by
 * default).  alew2d_kernel_timing returns the summed device time (ms) and the
 * number of launches of the last call per kind: which = 0 step kinematics,
 * 1 x-sweeps, 2 y-sweeps (edge fluxes, source, right-hand side), 3 step
 * epilogues.  Host pointers. */
alew_status alew2d_set_kernel_timing(alew2d_ctx* ctx, int on);
alew_status alew2d_kernel_timing(const alew2d_ctx* ctx, int which, double* ms, int64_t* launches);

/* Message for the calling thread's last non-OK status ("" if none). */
const char* alew_last_error(void);

/* Library version string. */
const char* alew_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ALEW_H */
