/*
 * Oracle for the 1D well-balanced ALE-WENO hybrid scheme with the special
 * source-term treatment (Zhang, Xia & Xu, "Structure-preserving finite volume
 * arbitrary Lagrangian-Eulerian WENO schemes for the shallow water equations").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, serial FP64 CPU version of
 * the scheme.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it, to check the GPU library against it.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * Style: every quantity is computed from its definition in the paper, in the
 * paper's order.  Polynomials are obtained by solving the cell-average
 * matching systems with Gaussian elimination, integrals by exact Gauss
 * quadrature, and there is no fusion, blocking or reordering.  Built with
 * -ffp-contract=off (no FMA contraction), IEEE division and sqrt.
 *
 * The forward scheme is written once as templates over the scalar type, so
 * that the same code also runs on a reverse-mode tape scalar (AD below).
 * That gives the exact discrete adjoint of this oracle, with every branch
 * (detector class, limiter activity, argmin/argmax, |.| signs, dry cut-offs)
 * taken from the forward values.
 *
 * Readings of points the paper leaves open:
 *  R1  Dx in the smoothness indicators is the global max cell width of the
 *      stage mesh (Sec. 2.2, Step 1 defines Dx^n as max_j Delta_j^n); flag
 *      FLAG_BETA_LOCAL switches to the cell's own width.
 *  R2  Class ties: smooth if gamma <= 1/2, non-smooth if gamma >= 1, else
 *      transition (Sec. 2.2, Step 2; the printed intervals overlap).
 *  R3  tau, gamma and the WENO-Z weights use the beta summed over the two
 *      equations (eq. (2.10)), taken on the equilibrium variables (eta, hu)
 *      of eq. (3.2); b is not an equation.  The polynomials themselves are
 *      built on (h, hu) and b (Sec. 4.1).  This is the reading under which
 *      the still-water test over the step bottom (Table 5.5) stays at
 *      round-off; indicators on (h, hu) lose it near the step.  Flag
 *      FLAG_BETA_FROM_H selects indicators on (h, hu).
 *  R4  Well-balanced reconstruction is component-wise on (h, hu) and b with
 *      shared weights (Sec. 4.1 items 1-2); no characteristic projection.
 *  R5  Linear weights on non-uniform cells come from the two outermost
 *      coefficients of the 5-cell quartic; a negative one is counted and
 *      reported as an error (no splitting).
 *  R6  Lax-Friedrichs alpha: per stage, global over all interfaces and both
 *      limited traces (eq. (3.13): "taken globally").
 *  R7  Time step: dt = CFL * min_j J_j / (max_j(|u_j| + sqrt(g h_j)) + max|W|),
 *      W the node speed of the mesh at t_n; clipped to t_end.
 *  R8  Prescribed mesh X(xi,t) = xi + A S(xi) sin(omega t): node velocity is
 *      the chord (X(t_{n+1}) - X(t_n))/dt of eq. (2.1), evaluated with the
 *      sum-to-product identity.  Periodic meshes use w_N = w_0.
 *  R9  Stage widths follow the recurrence of eq. (3.15) (1D: div(w) J = dw_j).
 *  R10 Limiter (eq. (3.20)-(3.21), 1D): delta from the Gauss-Lobatto mean
 *      identity (eq. (A.3)), m = min(h^L, delta, h^R), active only when
 *      m < eps_j; hu traces scaled by the same Phi about the mean; the bottom
 *      traces follow Remark 4.1 (b = eta - h_new).
 *  R11 Dry cut-off at traces: u = hu/h if h > dry_eps, else u = 0 and hu = 0.
 *      The limiter only bounds trace depths below by eps = 1e-11; dividing
 *      by depths that small makes the global alpha explode (Moses's second
 *      problem reaches alpha ~ 3e3 against ~10 physical at its second step),
 *      so the cut-off has its own tolerance (default 1e-8).  Setting u = 0
 *      at a trace keeps |u - w| <= alpha there, which is all the positivity
 *      argument of Appendix A uses.  A mean depth is reported negative only
 *      below -eps: dry cells (h = 0) carry round-off of either sign because
 *      h = eta - b is the difference of two separately updated means.
 *  R12 Special source (eq. (4.8)-(4.10), 1D): B1, B2 from the limited bottom
 *      traces; the interior integral uses the 4-point Gauss-Lobatto rule with
 *      the unlimited hybrid values of eta = h + b and of d b/dx: the
 *      derivative of b's reconstruction, i.e. where the class is smooth the
 *      derivative of the 5-cell quartic (the smooth class's reconstruction,
 *      eq. (2.10) with the linear weights, is that quartic at every point);
 *      in the non-smooth class the weighted stencil slopes sum_r phi_r p_r'
 *      (the weights change from point to point and no single polynomial is
 *      formed); in the transition class M times the WENO-Z weighted slopes
 *      plus (1 - M) times the quartic's, the blend of eq. (2.8) applied to
 *      the two parts, so that b_x, like the values, is continuous where the
 *      class changes.
 *  R13 Bottom evolves by the ALE scheme of eq. (3.17) (the paper's default).
 *  R14 Ghost cells: 3 per side.  Periodic wraps; transmissive copies the
 *      boundary cell (values and width); reflective mirrors with hu negated.
 *  R15 The state carried through a run is (eta, hu, b); h = eta - b is
 *      formed on entry and on exit of each library call.
 *  R16 A mean depth counts as negative only below -eps (the end of R11).
 *  R17 Hydrostatic reconstruction (Sec. 4.1, eq. (4.2)-(4.3) in 1D; flag
 *      FLAG_HYDROSTATIC).  At each face of cell j, q- is the cell's own
 *      limited trace and q+ the neighbour's, n the outward normal (+1 on the
 *      right face, -1 on the left).  h*+- = max(0, eta+- - max(b+, b-)),
 *      eta*+- = h*+- + b+-, q*+- = (eta*+-, (hu)+-): the discharge is kept as
 *      printed.  The momentum flux of q* uses u* = (hu)/h* where h* > dry_eps
 *      (R11), else 0.  H^mod = H(q*-, q*+, n) + (theta, (g/2 (eta- - b-)^2 -
 *      g/2 (h*-)^2) n), H the Lax-Friedrichs flux of eq. (3.13) with the
 *      alpha of R6 (taken on the traces q+-, not q*+-).  The bottom keeps the
 *      ALE flux of R13.
 *  R18 Hydrostatic source (the sentence after eq. (4.3)): "fourth-order
 *      polynomials" are read as the cubics (four coefficients) eta_h, b_h
 *      that interpolate the values at the 4 Gauss-Lobatto points of the cell
 *      (the limited traces at the two ends, the unlimited hybrid values
 *      inside).  A degree-4 polynomial is not fixed by these values and the
 *      cell average: the 4-point Gauss-Lobatto rule is exact to degree 5, so
 *      the average follows from the point values.  The integral of
 *      -g (eta_h - b_h) d b_h / dx over the cell is taken by the 5-point
 *      Gauss-Legendre rule, exact for the degree-5 integrand.
 *  Alternative readings, each behind a flag (the defaults are R6, R10, R8):
 *  R19 FLAG_ALPHA_CELLAVG: the Lax-Friedrichs speed of a stage is taken over the
 *      cell averages of the stage input (eq. (3.13) names u, v without saying
 *      where): max over the cells j of max(|u_j - w_{j-1/2}|, |u_j - w_{j+1/2}|)
 *      + sqrt(g h_j), u_j = hu_j / h_j if h_j > dry_eps, else 0.
 *  R20 FLAG_NO_HU_LIMIT: the limiter of eq. (3.20)-(3.21) acts on h (and on b
 *      through Remark 4.1) only; the hu traces stay as reconstructed.
 *  R21 FLAG_W_TANGENT: the node speed of a step on a prescribed map is the map's
 *      time derivative at the start of the step, dX/dt(xi, t_n), instead of the
 *      chord of eq. (2.1).
 *  R22 FLAG_NONWB: the scheme of Sec. 3 without well-balancing.  q = (eta, hu)
 *      is reconstructed in local characteristic variables (the remark after
 *      Step 4 of Sec. 2.2 prefers them for systems) taken from the eigenvectors
 *      of the flux Jacobian at the cell's own mean state; where the mean depth
 *      is at most dry_eps the reconstruction is component-wise.  Each
 *      characteristic variable and b (needed for the bottom flux of eq. (3.17)
 *      and the source) get their own indicators, class and weights.  The
 *      source integral of r(q, b) over the cell uses the 4-point Gauss-Lobatto
 *      rule of the limiter on the unlimited values (b_x: the derivative of b's
 *      hybrid reconstruction as in R12, with b's own class; the quartic's
 *      derivative is fourth order where the weighted candidate derivatives
 *      are second order only).  The limiter acts on h = eta - b and keeps the
 *      bottom traces (Remark 4.1 is stated for the well-balanced schemes; here
 *      a flat bottom stays flat).
 *  R23 params.bottom != ALE: the bottom is an analytic b(x) and its cell
 *      averages are the L2 projection of eq. (3.16) onto the moving cells,
 *      taken on the mesh of every stage (t_n, t_{n+1}, t_{n+1/2}, the meshes of
 *      eq. (3.14)) and on the new mesh at the end of the step, instead of the
 *      ALE evolution of eq. (3.17); the initial b is the projection onto the
 *      initial cells.  The integral is taken by the 5-point Gauss-Legendre
 *      rule on the smooth pieces of b.
 *  R29 Negative linear weights (the remark after Step 4 of Sec. 2.2 asks for
 *      a special treatment): by default a point whose linear weights include
 *      a negative one is counted and the run reports ST_NEGWEIGHT (the weights
 *      are used as they are).  FLAG_SPLIT: the nonlinear weights of the
 *      transition and non-smooth classes at such a point come from the
 *      splitting of Shi, Hu & Shu (2002) with theta = 3 (nonlinear_weights
 *      below), the smooth class keeps the linear weights (a linear
 *      combination needs no positivity), and the run goes on.  In 2D a
 *      negative weight on a stage mesh ends the run with ST_NEGWEIGHT after
 *      the step that met it (that step's sweeps use the split weights).
 *  R31 2D FLAG_HYDROSTATIC: the scheme of eq. (4.4)-(4.6) on the
 *      tensor-product mesh: at each of the 4 Gauss-Lobatto points of an edge
 *      the flux of the starred states q* = (eta*, hu, hv) (h* = max(0, eta -
 *      max(b-, b+)), velocities hu / h*, hv / h*), theta added to the eta
 *      component, and the pressure correction g/2 (h^2 - h*^2) of each cell's
 *      own trace on its normal momentum; the reconstruction, the bottom flux and
 *      alpha are the special source-term scheme's.  The paper leaves the 2D
 *      source to the 1D construction ("similar"): here the 1D source of R18
 *      (the cubic interpolants of eta and b through the 4 point values, their
 *      integral by 5-point Gauss-Legendre) on every x-line (points nu) and
 *      y-line (points mu) of the cell, weighted by the other direction's
 *      Gauss-Lobatto rule; the point values are the unlimited ones, as for
 *      the special source (R28).  Still water is kept line by line: the edge
 *      and cell rules share the points.
 *  R32 2D FLAG_NONWB: the scheme of Sec. 3 without well-balancing on the
 *      tensor-product mesh, as R22 in each sweep: q = (eta, hu, hv) in the
 *      local characteristic variables of the sweep direction (the flux
 *      Jacobian's eigenvectors at the cell's mean state; the x-sweep of a
 *      row's cell at that cell's mean, the y-sweep of every abscissa at the
 *      cell's mean), each characteristic variable and b with their own
 *      indicators, class and weights (b's x-derivative lines in the y-sweep
 *      with b's weights), the identity frame where the mean depth is at most
 *      dry_eps; the plain Lax-Friedrichs flux; the source -g h grad b by the
 *      4 x 4 Gauss-Lobatto rule on the unlimited values (b_x, b_y the
 *      derivatives of b's reconstructions, R12); the limiter keeps the bottom
 *      traces (as R22).
 *  R34 2D translation (Example 5.7): the node maps take a uniform velocity
 *      as well, X = xi + Vx t + Ax sin(2 pi kx xi) sin(omx t) (y likewise);
 *      the node speeds are the chords, Vx plus the sine part's.
 *  R30 MESH_ALIGNED: the quartic map of eq. (5.14) (Example 5.5), the map of
 *      eq. (5.1) times (xi - p1)(xi - p2) / (xmax - xmin)^2 with p1, p2 the
 *      step bottom's jump points bottom_p[1], bottom_p[2]: a node placed on a
 *      jump point stays there, so the projection of eq. (3.16) never averages
 *      across a jump.  With the example's 100 uniform cells on [0, 1500] the
 *      jump points 562.5 = 3L/8 and 937.5 = 5L/8 lie inside cells; a cell
 *      count that is a multiple of 8 puts them on nodes.
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

namespace orc {

/* ------------------------------------------------------------------------ */
/* Reverse-mode tape scalar                                                  */
/* ------------------------------------------------------------------------ */
struct TapeNode { int64_t a, b; double da, db; };
static std::vector<TapeNode>* g_tape = nullptr;

struct AD {
  double v;
  int64_t i;  /* tape index, -1 = constant */
  AD() : v(0.0), i(-1) {}
  AD(double x) : v(x), i(-1) {}
};

static inline AD node(double v, int64_t a, double da, int64_t b, double db) {
  AD r;
  r.v = v;
  if (a < 0 && b < 0) { r.i = -1; return r; }
  r.i = (int64_t)g_tape->size();
  g_tape->push_back({a, b, da, db});
  return r;
}
static inline AD make_input(double v) {
  AD r;
  r.v = v;
  r.i = (int64_t)g_tape->size();
  g_tape->push_back({-1, -1, 0.0, 0.0});
  return r;
}
static inline AD operator+(const AD& x, const AD& y) { return node(x.v + y.v, x.i, 1.0, y.i, 1.0); }
static inline AD operator-(const AD& x, const AD& y) { return node(x.v - y.v, x.i, 1.0, y.i, -1.0); }
static inline AD operator*(const AD& x, const AD& y) { return node(x.v * y.v, x.i, y.v, y.i, x.v); }
static inline AD operator/(const AD& x, const AD& y) {
  double q = x.v / y.v;
  return node(q, x.i, 1.0 / y.v, y.i, -q / y.v);
}
static inline AD operator-(const AD& x) { return node(-x.v, x.i, -1.0, -1, 0.0); }
static inline AD sqrt(const AD& x) {
  double s = std::sqrt(x.v);
  return node(s, x.i, s > 0.0 ? 0.5 / s : 0.0, -1, 0.0);
}
static inline AD fabs(const AD& x) {
  double d = x.v > 0.0 ? 1.0 : (x.v < 0.0 ? -1.0 : 0.0);
  return node(std::fabs(x.v), x.i, d, -1, 0.0);
}
static inline double val(double x) { return x; }
static inline double val(const AD& x) { return x.v; }
using std::sqrt;
using std::fabs;

/* ------------------------------------------------------------------------ */
/* Parameters, statistics                                                    */
/* ------------------------------------------------------------------------ */
enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2 };
enum { MESH_GIVEN = 0, MESH_SINE = 1, MESH_PAPER = 2, MESH_FLUID = 3, MESH_ALIGNED = 4 };
enum { ST_OK = 0, ST_ARG = 1, ST_MESH = 2, ST_NEGDEPTH = 3, ST_NONFINITE = 4, ST_NEGWEIGHT = 8 };

enum {
  FLAG_BETA_LOCAL = 1, FLAG_BETA_FROM_H = 2, FLAG_HYDROSTATIC = 4, FLAG_ALPHA_CELLAVG = 8,
  FLAG_NO_HU_LIMIT = 16, FLAG_W_TANGENT = 32, FLAG_NONWB = 64, FLAG_SPLIT = 128
};

struct Params {
  double g, cfl, weno_eps, pp_eps;
  double mesh_A, mesh_k, mesh_omega, dry_eps;
  int32_t bc, mesh, flags, bottom;
  double bottom_p[4];
};

/* ------------------------------------------------------------------------ */
/* Sec. 3.3, eq. (3.16): L2 projection of an analytic bottom b(x) (R23)       */
/* ------------------------------------------------------------------------ */
enum { BOTTOM_ALE = 0, BOTTOM_STEP = 1, BOTTOM_GAUSS = 2, BOTTOM_SIN2 = 3, BOTTOM_BUMP = 4,
       BOTTOM_PARABOLA = 5 };

static double bottom_value(const Params& P, double x) {
  const double* p = P.bottom_p;
  switch (P.bottom) {
    case BOTTOM_STEP: return (x >= p[1] && x <= p[2]) ? p[0] : 0.0;
    case BOTTOM_GAUSS: return p[0] * std::exp(-p[1] * (x - p[2]) * (x - p[2]));
    case BOTTOM_SIN2: {
      double s = std::sin(M_PI * p[1] * x);
      return p[0] * s * s;
    }
    case BOTTOM_BUMP:
      return std::fabs(x - p[2]) < p[1] ? p[0] * (std::cos(M_PI * (x - p[2]) / p[1]) + 1.0) : 0.0;
    case BOTTOM_PARABOLA: return p[0] * (x / p[1]) * (x / p[1]);
    default: return 0.0;
  }
}

/* Average of b over [xl, xr]: the 5-point Gauss-Legendre rule on 16 equal
 * parts of every piece between the points where b is not smooth (exact for
 * the step and the parabola; for the smooth pieces the composite rule is
 * accurate to round-off also on cells as wide as the bump itself). */
static double bottom_average(const Params& P, double xl, double xr) {
  static const double r[5] = {-0.90617984593866399280, -0.53846931010568309104, 0.0,
                              0.53846931010568309104, 0.90617984593866399280};
  static const double w[5] = {0.23692688505618908751, 0.47862867049936646804,
                              0.56888888888888888889, 0.47862867049936646804,
                              0.23692688505618908751};
  std::vector<double> cuts = {xl};
  const double* p = P.bottom_p;
  double br[2] = {0.0, 0.0};
  int nb = 0;
  if (P.bottom == BOTTOM_STEP) { br[0] = p[1]; br[1] = p[2]; nb = 2; }
  if (P.bottom == BOTTOM_BUMP) { br[0] = p[2] - p[1]; br[1] = p[2] + p[1]; nb = 2; }
  for (int k = 0; k < nb; ++k)
    if (br[k] > xl && br[k] < xr) cuts.push_back(br[k]);
  cuts.push_back(xr);
  std::sort(cuts.begin(), cuts.end());
  double I = 0.0;
  const int parts = 16;
  for (size_t k = 0; k + 1 < cuts.size(); ++k) {
    for (int e = 0; e < parts; ++e) {
      const double a = cuts[k] + (cuts[k + 1] - cuts[k]) * e / parts;
      const double b = cuts[k] + (cuts[k + 1] - cuts[k]) * (e + 1) / parts;
      const double m = 0.5 * (a + b), hw = 0.5 * (b - a);
      double s = 0.0;
      for (int q = 0; q < 5; ++q) s = s + w[q] * bottom_value(P, m + r[q] * hw);
      I = I + s * hw;
    }
  }
  return I / (xr - xl);
}

struct Stats {
  int64_t steps;
  int64_t n_class[3];
  int64_t n_limited, n_negweight;
  double t, dt_min, dt_max, h_min;
  double mass_eta0, mass_eta, mass_b0, mass_b;
  int32_t status, pad;
};

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra: Gaussian elimination with partial pivoting    */
/* ------------------------------------------------------------------------ */
/* Inverse of the n x n row-major matrix A into Ainv. */
static void invert(int n, const double* A, double* Ainv) {
  double M[5][10];
  for (int r = 0; r < n; ++r) {
    for (int c = 0; c < n; ++c) M[r][c] = A[r * n + c];
    for (int c = 0; c < n; ++c) M[r][n + c] = (r == c) ? 1.0 : 0.0;
  }
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(M[r][k]) > std::fabs(M[p][k])) p = r;
    if (p != k)
      for (int c = 0; c < 2 * n; ++c) std::swap(M[k][c], M[p][c]);
    double piv = M[k][k];
    for (int c = 0; c < 2 * n; ++c) M[k][c] = M[k][c] / piv;
    for (int r = 0; r < n; ++r) {
      if (r == k) continue;
      double f = M[r][k];
      if (f == 0.0) continue;
      for (int c = 0; c < 2 * n; ++c) M[r][c] = M[r][c] - f * M[k][c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) Ainv[r * n + c] = M[r][n + c];
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.2, Step 1: stencil polynomials and linear weights on moving cells  */
/* ------------------------------------------------------------------------ */
/* Evaluation points in cell j, in the coordinate s = (x - x_{j-1/2}) / Delta_j:
 * the 4-point Gauss-Lobatto nodes on [0,1] (Sec. 3.4.1 with k = 4 >= (5+2)/2). */
static const double kS[4] = {0.0, 0.5 - 0.1 * 2.2360679774997896964,
                             0.5 + 0.1 * 2.2360679774997896964, 1.0};
/* Gauss-Lobatto weights (sum 1). */
static const double kGLW[4] = {1.0 / 12.0, 5.0 / 12.0, 5.0 / 12.0, 1.0 / 12.0};

struct CellGeo {
  double J;            /* width of the cell                                    */
  double a[3][3][3];   /* a[r][p][i]: coefficient of s^p in u_r, per average i  */
  double c[3][4][3];   /* c[r][mu][i]: u_r(x_mu) = sum_i c[r][mu][i] ubar_{j-r+i} */
  double cd[3][4][3];  /* same for d u_r/dx at x_mu                            */
  double d[4][3];      /* linear weights d_r(x_mu)                              */
  double cq[4][5];     /* dP/dx at x_mu of the 5-cell quartic P, per average     */
};

/* Mean over [a,b] of s^p. */
static double mean_pow(double a, double b, int p) {
  return (std::pow(b, p + 1) - std::pow(a, p + 1)) / ((p + 1) * (b - a));
}

/* wid[k] = width of cell j-2+k, k = 0..4. */
static void cell_geometry(const double wid[5], CellGeo& G) {
  const double Jj = wid[2];
  G.J = Jj;
  double E[6];
  E[2] = 0.0;
  E[3] = 1.0;
  E[1] = -wid[1] / Jj;
  E[0] = E[1] - wid[0] / Jj;
  E[4] = 1.0 + wid[3] / Jj;
  E[5] = E[4] + wid[4] / Jj;
  /* Small stencils s_r(j) = {T_{j-r}, T_{j-r+1}, T_{j-r+2}}, r = 0,1,2:
   * the quadratic whose averages over the three cells equal the data. */
  for (int r = 0; r < 3; ++r) {
    double M[9], Mi[9];
    for (int i = 0; i < 3; ++i) {
      int k = 2 - r + i; /* cell index 0..4 within the big stencil */
      for (int p = 0; p < 3; ++p) M[i * 3 + p] = mean_pow(E[k], E[k + 1], p);
    }
    invert(3, M, Mi);
    for (int p = 0; p < 3; ++p)
      for (int i = 0; i < 3; ++i) G.a[r][p][i] = Mi[p * 3 + i];
    for (int mu = 0; mu < 4; ++mu) {
      double s = kS[mu];
      for (int i = 0; i < 3; ++i) {
        double v = 0.0, dv = 0.0;
        for (int p = 0; p < 3; ++p) v = v + std::pow(s, p) * Mi[p * 3 + i];
        for (int p = 1; p < 3; ++p) dv = dv + p * std::pow(s, p - 1) * Mi[p * 3 + i];
        G.c[r][mu][i] = v;
        G.cd[r][mu][i] = dv / Jj;
      }
    }
  }
  /* Big stencil S_j = {T_{j-2}, ..., T_{j+2}}: the quartic matching all five
   * averages.  Linear weights with sum_r d_r u_r = quartic: cell j+2 appears
   * only in u_0 (as its third average), cell j-2 only in u_2 (first average). */
  double M5[25], M5i[25];
  for (int k = 0; k < 5; ++k)
    for (int p = 0; p < 5; ++p) M5[k * 5 + p] = mean_pow(E[k], E[k + 1], p);
  invert(5, M5, M5i);
  for (int mu = 0; mu < 4; ++mu) {
    double s = kS[mu];
    double Cm2 = 0.0, Cp2 = 0.0;
    for (int p = 0; p < 5; ++p) {
      Cm2 = Cm2 + std::pow(s, p) * M5i[p * 5 + 0];
      Cp2 = Cp2 + std::pow(s, p) * M5i[p * 5 + 4];
    }
    double d0 = Cp2 / G.c[0][mu][2];
    double d2 = Cm2 / G.c[2][mu][0];
    G.d[mu][0] = d0;
    G.d[mu][2] = d2;
    G.d[mu][1] = 1.0 - d0 - d2;
    /* derivative of the quartic at the point: d/dx = (1/J) d/ds */
    for (int k = 0; k < 5; ++k) {
      double dv = 0.0;
      for (int p = 1; p < 5; ++p) dv = dv + p * std::pow(s, p - 1) * M5i[p * 5 + k];
      G.cq[mu][k] = dv / Jj;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.2, Steps 2-4 with eq. (2.10): hybrid WENO values in one cell       */
/* ------------------------------------------------------------------------ */
enum { CLS_S = 0, CLS_T = 1, CLS_N = 2 };

template <class T>
struct Recon {
  T h[4], m[4], b[4]; /* hybrid values at the 4 Gauss-Lobatto points */
  T bx[4];            /* hybrid value of d b / dx at the same points  */
  int cls;
  int negw;
};

/* 3-point Gauss-Legendre rule on [0,1] (exact to degree 5). */
static const double kGLeg_s[3] = {0.5 - 0.5 * 0.77459666924148337704, 0.5,
                                  0.5 + 0.5 * 0.77459666924148337704};
static const double kGLeg_w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

/* Smoothness indicator of one stencil polynomial for one variable (Step 2):
 * sum_{l=1,2} Dx^{2l-1} * integral over cell j of (d^l u_r / dx^l)^2. */
template <class T>
static T beta_one(const CellGeo& G, int r, const T v[3], double Dx) {
  T a1 = 0.0, a2 = 0.0;
  for (int i = 0; i < 3; ++i) {
    a1 = a1 + G.a[r][1][i] * v[i];
    a2 = a2 + G.a[r][2][i] * v[i];
  }
  const double J = G.J;
  /* u_r(x) = a0 + a1 s + a2 s^2 with s = (x - x_{j-1/2})/J. */
  T I1 = 0.0;
  for (int q = 0; q < 3; ++q) {
    T du = (a1 + 2.0 * a2 * kGLeg_s[q]) / J;
    I1 = I1 + kGLeg_w[q] * J * (du * du);
  }
  T d2u = 2.0 * a2 / (J * J);
  T I2 = J * (d2u * d2u);
  return Dx * I1 + (Dx * Dx * Dx) * I2;
}

/* v[5]: the first indicator variable (eta by default, see R3). */
/* Nonlinear weights at one point from the linear weights d[3] and the factors
 * K_r = 1 + (tau / (beta_r + eps))^2 of eq. (2.9).  With a negative linear
 * weight and split set (R29), the weights are split into a positive group
 * gp_r = (d_r + 3 |d_r|) / 2 and a negative group gm_r = gp_r - d_r (both
 * non-negative, gp - gm = d), each normalised to sum one and given its own
 * nonlinear weights; the point value is sp (positive group's value) -
 * sm (negative group's value), sp, sm the group sums: the splitting of Shi,
 * Hu & Shu (J. Comput. Phys. 175, 2002) with theta = 3. */
template <class T>
static void nonlinear_weights(const double d[3], const T K[3], bool split, T phi[3]) {
  const bool neg = d[0] < 0.0 || d[1] < 0.0 || d[2] < 0.0;
  if (neg && split) {
    double gp[3], gm[3], sp = 0.0, sm = 0.0;
    for (int r = 0; r < 3; ++r) {
      gp[r] = 0.5 * (d[r] + 3.0 * std::fabs(d[r]));
      gm[r] = gp[r] - d[r];
      sp = sp + gp[r];
      sm = sm + gm[r];
    }
    T ap[3], am[3];
    for (int r = 0; r < 3; ++r) {
      ap[r] = (gp[r] / sp) * K[r];
      am[r] = (gm[r] / sm) * K[r];
    }
    T SP = ap[0] + ap[1] + ap[2], SM = am[0] + am[1] + am[2];
    for (int r = 0; r < 3; ++r) phi[r] = sp * (ap[r] / SP) - sm * (am[r] / SM);
    return;
  }
  T a[3];
  for (int r = 0; r < 3; ++r) a[r] = d[r] * K[r];
  T sum = a[0] + a[1] + a[2];
  for (int r = 0; r < 3; ++r) phi[r] = a[r] / sum;
}

template <class T>
static void reconstruct(const CellGeo& G, double Dx, double eps, const T v[5], const T h[5],
                        const T m[5], const T b[5], Recon<T>& o, bool split = true) {
  /* Step 2: indicators summed over the two equations, detector. */
  T beta[3];
  for (int r = 0; r < 3; ++r) {
    T vv[3] = {v[2 - r], v[3 - r], v[4 - r]};
    T mv[3] = {m[2 - r], m[3 - r], m[4 - r]};
    beta[r] = beta_one(G, r, vv, Dx) + beta_one(G, r, mv, Dx);
  }
  T tau = fabs(beta[0] - beta[2]);
  T betaA = (beta[0] + beta[1] + beta[2]) / 3.0;
  T gamma = tau / (betaA + eps);
  int cls;
  if (val(gamma) <= 0.5) cls = CLS_S;
  else if (val(gamma) >= 1.0) cls = CLS_N;
  else cls = CLS_T;
  o.cls = cls;
  o.negw = 0;
  /* Steps 3-4 at each point. */
  for (int mu = 0; mu < 4; ++mu) {
    T phi[3], phiS[3]; /* weights of the values and of the slope's WENO part */
    for (int r = 0; r < 3; ++r)
      if (G.d[mu][r] < 0.0) o.negw = 1;
    if (cls == CLS_S) {
      for (int r = 0; r < 3; ++r) phi[r] = G.d[mu][r];
      for (int r = 0; r < 3; ++r) phiS[r] = 0.0;
    } else {
      T Kf[3];
      for (int r = 0; r < 3; ++r) {
        T q = tau / (beta[r] + eps);
        Kf[r] = 1.0 + q * q;
      }
      T phiN[3];
      nonlinear_weights(G.d[mu], Kf, split, phiN);
      for (int r = 0; r < 3; ++r) phiS[r] = phiN[r];
      if (cls == CLS_N) {
        for (int r = 0; r < 3; ++r) phi[r] = phiN[r];
      } else {
        T M = 2.0 * gamma - 1.0;
        for (int r = 0; r < 3; ++r) phi[r] = M * phiN[r] + (1.0 - M) * G.d[mu][r];
      }
    }
    T vh = 0.0, vm = 0.0, vb = 0.0, vbx = 0.0;
    for (int r = 0; r < 3; ++r) {
      T ph = 0.0, pm = 0.0, pb = 0.0, pbx = 0.0;
      for (int i = 0; i < 3; ++i) {
        ph = ph + G.c[r][mu][i] * h[2 - r + i];
        pm = pm + G.c[r][mu][i] * m[2 - r + i];
        pb = pb + G.c[r][mu][i] * b[2 - r + i];
        pbx = pbx + G.cd[r][mu][i] * b[2 - r + i];
      }
      vh = vh + phi[r] * ph;
      vm = vm + phi[r] * pm;
      vb = vb + phi[r] * pb;
      vbx = vbx + phiS[r] * pbx;
    }
    /* R12: b_x is the derivative of b's reconstruction.  The linear part of
     * eq. (2.10) is the quartic of the big stencil at every point, so its
     * slope is the quartic's derivative; the WENO-Z part has weights that
     * change from point to point, and its slope is taken as the weighted
     * stencil slopes.  Smooth: the quartic's; transition: M times the
     * weighted slopes plus (1 - M) times the quartic's (continuous at both
     * class edges); non-smooth: the weighted slopes. */
    if (cls != CLS_N) {
      T vq = 0.0;
      for (int k = 0; k < 5; ++k) vq = vq + G.cq[mu][k] * b[k];
      if (cls == CLS_S) {
        vbx = vq;
      } else {
        T M = 2.0 * gamma - 1.0;
        vbx = M * vbx + (1.0 - M) * vq;
      }
    }
    o.h[mu] = vh;
    o.m[mu] = vm;
    o.b[mu] = vb;
    o.bx[mu] = vbx;
  }
}

/* Non-well-balanced scheme of Sec. 3 (R22): the equilibrium variables
 * q = (eta, hu) reconstructed in local characteristic variables (the remark
 * after Step 4 of Sec. 2.2), b on its own.  The flux Jacobian of f(q) with
 * respect to q at fixed b has the eigenvalues u -+ c, c = sqrt(g h), and the
 * right eigenvectors (1, u - c), (1, u + c); the characteristic variables of
 * the 5 stencil averages are taken with the left eigenvectors of cell j's
 * mean state, each is reconstructed as a scalar with its own indicators,
 * class and weights (Steps 1-4), and the point values are mapped back with
 * the right eigenvectors.  Where the mean depth is at most dry_eps the frame
 * is the identity.  o.h holds h = eta - b at the points, o.bx the derivative
 * of b's reconstruction; o.cls the largest of the three classes. */
template <class T>
static void reconstruct_char(const CellGeo& G, double Dx, double eps, double g, double dry,
                             const T eta[5], const T m[5], const T b[5], Recon<T>& o,
                             bool split = true) {
  T zero[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  T hbar = eta[2] - b[2];
  bool chr = val(hbar) > dry;
  T u = 0.0, c = 0.0;
  T w1[5], w2[5];
  if (chr) {
    u = m[2] / hbar;
    c = sqrt(g * hbar);
    for (int k = 0; k < 5; ++k) {
      /* rows of the inverse of R = [[1, 1], [u - c, u + c]] */
      w1[k] = ((u + c) * eta[k] - m[k]) / (2.0 * c);
      w2[k] = ((c - u) * eta[k] + m[k]) / (2.0 * c);
    }
  } else {
    for (int k = 0; k < 5; ++k) {
      w1[k] = eta[k];
      w2[k] = m[k];
    }
  }
  Recon<T> r1, r2, rb;
  reconstruct(G, Dx, eps, w1, w1, zero, w1, r1, split);
  reconstruct(G, Dx, eps, w2, w2, zero, w2, r2, split);
  /* b_x as R12: where b is smooth its reconstruction is the 5-cell quartic
   * P (linear weights) and b_x its derivative, fourth order (the weighted
   * stencil derivatives sum_r d_r p_r' leave out sum_r d_r' p_r and are
   * second order only); blended in the transition class */
  reconstruct(G, Dx, eps, b, b, zero, b, rb, split);
  for (int mu = 0; mu < 4; ++mu) {
    T e, mm;
    if (chr) {
      e = r1.h[mu] + r2.h[mu];
      mm = (u - c) * r1.h[mu] + (u + c) * r2.h[mu];
    } else {
      e = r1.h[mu];
      mm = r2.h[mu];
    }
    o.h[mu] = e - rb.h[mu];
    o.m[mu] = mm;
    o.b[mu] = rb.h[mu];
    o.bx[mu] = rb.bx[mu];
  }
  o.cls = std::max(r1.cls, std::max(r2.cls, rb.cls));
  o.negw = r1.negw | r2.negw | rb.negw;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.4.2, eq. (3.20)-(3.21) in 1D, with Remark 4.1                      */
/* ------------------------------------------------------------------------ */
template <class T>
struct Traces {
  T hL, mL, bL, hR, mR, bR;
};

/* Returns 1 if the limiter modified the traces, 2 if hbar < 0.  hu_lim = false
 * (FLAG_NO_HU_LIMIT) leaves the hu traces as reconstructed. */
template <class T>
static int limit_cell(T hbar, T mbar, const Recon<T>& o, double pp_eps, Traces<T>& tr,
                      bool hu_lim = true, bool keep_b = false) {
  tr.hL = o.h[0]; tr.mL = o.m[0]; tr.bL = o.b[0];
  tr.hR = o.h[3]; tr.mR = o.m[3]; tr.bR = o.b[3];
  const double s1 = kGLW[0];
  if (val(hbar) <= 0.0) {
    /* Phi = 0: the traces collapse onto the cell mean. */
    T etaL = tr.hL + tr.bL, etaR = tr.hR + tr.bR;
    tr.hL = hbar; tr.hR = hbar;
    if (hu_lim) { tr.mL = mbar; tr.mR = mbar; }
    if (!keep_b) {
      tr.bL = etaL - tr.hL;
      tr.bR = etaR - tr.hR;
    }
    return val(hbar) < 0.0 ? 2 : 1;
  }
  /* Interior mean delta from hbar = s1 hL + s1 hR + (1 - 2 s1) delta. */
  T delta = (hbar - s1 * tr.hL - s1 * tr.hR) / (1.0 - 2.0 * s1);
  T mn = tr.hL;
  if (val(delta) < val(mn)) mn = delta;
  if (val(tr.hR) < val(mn)) mn = tr.hR;
  T epsj = (pp_eps < val(hbar)) ? T(pp_eps) : hbar;
  if (!(val(mn) < val(epsj))) return 0;
  T Phi = (hbar - epsj) / (hbar - mn);
  if (val(Phi) > 1.0) Phi = 1.0;
  T etaL = tr.hL + tr.bL, etaR = tr.hR + tr.bR;
  tr.hL = Phi * (tr.hL - hbar) + hbar;
  tr.hR = Phi * (tr.hR - hbar) + hbar;
  if (hu_lim) {
    tr.mL = Phi * (tr.mL - mbar) + mbar;
    tr.mR = Phi * (tr.mR - mbar) + mbar;
  }
  if (!keep_b) {
    tr.bL = etaL - tr.hL;
    tr.bR = etaR - tr.hR;
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Residual of the semi-discrete scheme (eq. (3.11)-(3.13), (3.17),          */
/* (4.7)-(4.10)), 1D: RHS_j for (eta, hu, b)                                 */
/* ------------------------------------------------------------------------ */
struct Counters {
  int64_t n_class[3];
  int64_t n_limited, n_negweight;
  int negdepth;
};

/* Source cell and hu sign of extended index k in [-3, n+2] (R14). */
static void ghost_map(int bc, int n, int k, int& src, double& msign) {
  msign = 1.0;
  if (k >= 0 && k < n) { src = k; return; }
  if (bc == BC_PERIODIC) {
    src = ((k % n) + n) % n;
  } else if (bc == BC_TRANSMISSIVE) {
    src = k < 0 ? 0 : n - 1;
  } else {
    src = k < 0 ? -1 - k : 2 * n - 1 - k;
    msign = -1.0;
  }
}

template <class T>
struct TraceFlux {
  T h, m, b, eta, u;
};

template <class T>
static TraceFlux<T> trace_state(T h, T m, T b, double dry_eps) {
  TraceFlux<T> s;
  s.h = h;
  s.b = b;
  s.eta = h + b;
  if (val(h) > dry_eps) {
    s.m = m;
    s.u = m / h;
  } else {
    s.m = 0.0;
    s.u = 0.0;
  }
  return s;
}

/* ------------------------------------------------------------------------ */
/* Hydrostatic reconstruction (Sec. 4.1, eq. (4.2)-(4.3)), readings R17-R18   */
/* ------------------------------------------------------------------------ */
/* H^mod of eq. (4.2) at one face of a cell: q- its own trace, q+ the
 * neighbour's, nrm the outward normal, w the node speed.  Components eta, hu. */
template <class T>
static void hydro_face_flux(const Params& P, const TraceFlux<T>& qm, const TraceFlux<T>& qp,
                            double nrm, double w, T alpha, T& H1, T& H2) {
  /* max(b-, b+), ties resolved by the face's orientation (its left trace
   * first), so that both cells of the face take the same branch */
  const TraceFlux<T>& fl = nrm > 0.0 ? qm : qp;
  const TraceFlux<T>& fr = nrm > 0.0 ? qp : qm;
  T bmax = (val(fl.b) >= val(fr.b)) ? fl.b : fr.b;
  T hsm = qm.eta - bmax, hsp = qp.eta - bmax;
  if (val(hsm) < 0.0) hsm = 0.0;
  if (val(hsp) < 0.0) hsp = 0.0;
  T esm = hsm + qm.b, esp = hsp + qp.b;
  T usm = 0.0, usp = 0.0;
  if (val(hsm) > P.dry_eps) usm = qm.m / hsm;
  if (val(hsp) > P.dry_eps) usp = qp.m / hsp;
  /* calH(w, q*) . n for both states, then the Lax-Friedrichs flux */
  T Hm1 = nrm * (qm.m - w * esm);
  T Hp1 = nrm * (qp.m - w * esp);
  T Hm2 = nrm * (qm.m * usm + 0.5 * P.g * hsm * hsm - w * qm.m);
  T Hp2 = nrm * (qp.m * usp + 0.5 * P.g * hsp * hsp - w * qp.m);
  H1 = 0.5 * (Hm1 + Hp1) - 0.5 * alpha * (esp - esm);
  H2 = 0.5 * (Hm2 + Hp2) - 0.5 * alpha * (qp.m - qm.m);
  T theta = 0.5 * (w * nrm + alpha) * (esp - qp.eta) + 0.5 * (w * nrm - alpha) * (esm - qm.eta);
  T hm = qm.eta - qm.b;
  H1 = H1 + theta;
  H2 = H2 + (0.5 * P.g * hm * hm - 0.5 * P.g * hsm * hsm) * nrm;
}

/* 5-point Gauss-Legendre rule on [0,1] (exact to degree 9). */
static const double kGL5_s[5] = {0.5 - 0.5 * 0.90617984593866399280, 0.5 - 0.5 * 0.53846931010568309104,
                                 0.5, 0.5 + 0.5 * 0.53846931010568309104,
                                 0.5 + 0.5 * 0.90617984593866399280};
static const double kGL5_w[5] = {0.5 * 0.23692688505618908751, 0.5 * 0.47862867049936646804,
                                 0.5 * 0.56888888888888888889, 0.5 * 0.47862867049936646804,
                                 0.5 * 0.23692688505618908751};

/* Inverse of the interpolation system of R18 in the cell coordinate
 * s in [0,1]: p(s) = sum_k c_k s^k, k = 0..3, with p at the 4 Gauss-Lobatto
 * points kS. */
struct InterpInverse {
  double a[16];
  InterpInverse() {
    double A[16];
    for (int r = 0; r < 4; ++r)
      for (int k = 0; k < 4; ++k) A[r * 4 + k] = std::pow(kS[r], k);
    invert(4, A, a);
  }
};
static const double* hydro_interp_inverse() {
  static const InterpInverse inv;  /* initialised once, thread-safe */
  return inv.a;
}

/* R18: integral over cell j of -g (eta_h - b_h) d b_h / dx.  ev, bv: values
 * at the 4 Gauss-Lobatto points.  With x = x_{j-1/2} + s J, dx = J ds and
 * d/dx = (1/J) d/ds, so J drops out. */
template <class T>
static T hydro_source(double g, const T ev[4], const T bv[4]) {
  const double* Ai = hydro_interp_inverse();
  T ce[4], cb[4];
  for (int k = 0; k < 4; ++k) {
    ce[k] = 0.0;
    cb[k] = 0.0;
    for (int r = 0; r < 4; ++r) {
      ce[k] = ce[k] + Ai[k * 4 + r] * ev[r];
      cb[k] = cb[k] + Ai[k * 4 + r] * bv[r];
    }
  }
  T S = 0.0;
  for (int q = 0; q < 5; ++q) {
    const double s = kGL5_s[q];
    T eh = 0.0, bh = 0.0, dbh = 0.0;
    for (int k = 3; k >= 0; --k) {
      eh = eh * s + ce[k];
      bh = bh * s + cb[k];
      if (k >= 1) dbh = dbh * s + (double)k * cb[k];
    }
    S = S + kGL5_w[q] * ((-g) * (eh - bh) * dbh);
  }
  return S;
}

template <class T>
static void residual(const Params& P, int n, const T* eta, const T* m, const T* b, const double* J,
                     const double* w, T* R, double* alpha_out, uint8_t* cls, Counters& cnt) {
  const int G = 3, NE = n + 2 * G;
  std::vector<T> he(NE), me(NE), be(NE), etae(NE);
  std::vector<double> Je(NE);
  for (int k = -G; k < n + G; ++k) {
    int src;
    double ms;
    ghost_map(P.bc, n, k, src, ms);
    etae[k + G] = eta[src];
    be[k + G] = b[src];
    he[k + G] = eta[src] - b[src];
    me[k + G] = ms * m[src];
    Je[k + G] = J[src];
  }
  double Dx = 0.0;
  for (int j = 0; j < n; ++j) Dx = std::max(Dx, J[j]);
  /* Cells -1..n: reconstruction and limiter. */
  const int NC = n + 2;
  std::vector<Recon<T>> rec(NC);
  std::vector<Traces<T>> tr(NC);
  for (int j = -1; j <= n; ++j) {
    double wid[5];
    T vs[5], hs[5], ms5[5], bs[5];
    for (int k = 0; k < 5; ++k) {
      wid[k] = Je[j - 2 + k + G];
      hs[k] = he[j - 2 + k + G];
      ms5[k] = me[j - 2 + k + G];
      bs[k] = be[j - 2 + k + G];
      vs[k] = (P.flags & FLAG_BETA_FROM_H) ? hs[k] : etae[j - 2 + k + G];
    }
    CellGeo geo;
    cell_geometry(wid, geo);
    double dxr = (P.flags & FLAG_BETA_LOCAL) ? wid[2] : Dx;
    const bool nonwb = (P.flags & FLAG_NONWB) != 0;
    const bool split = (P.flags & FLAG_SPLIT) != 0;
    if (nonwb) {
      T es[5];
      for (int k = 0; k < 5; ++k) es[k] = etae[j - 2 + k + G];
      reconstruct_char(geo, dxr, P.weno_eps, P.g, P.dry_eps, es, ms5, bs, rec[j + 1], split);
    } else {
      reconstruct(geo, dxr, P.weno_eps, vs, hs, ms5, bs, rec[j + 1], split);
    }
    int lim = limit_cell(he[j + G], me[j + G], rec[j + 1], P.pp_eps, tr[j + 1],
                         !(P.flags & FLAG_NO_HU_LIMIT), nonwb);
    if (j >= 0 && j < n) {
      cnt.n_class[rec[j + 1].cls] += 1;
      if (cls) cls[j] = (uint8_t)rec[j + 1].cls;
      if (lim) cnt.n_limited += 1;
      if (val(he[j + G]) < -P.pp_eps) cnt.negdepth = 1;
    }
    if (rec[j + 1].negw) cnt.n_negweight += 1;
  }
  /* Interface i (0..n) lies between cell i-1 (its right trace) and cell i
   * (its left trace).  Global LF speed over all interfaces and both traces. */
  std::vector<TraceFlux<T>> Lt(n + 1), Rt(n + 1);
  T alpha = 0.0;
  for (int i = 0; i <= n; ++i) {
    const Traces<T>& a = tr[i];     /* cell i-1 */
    const Traces<T>& c = tr[i + 1]; /* cell i   */
    Lt[i] = trace_state(a.hR, a.mR, a.bR, P.dry_eps);
    Rt[i] = trace_state(c.hL, c.mL, c.bL, P.dry_eps);
    T hl = Lt[i].h, hr = Rt[i].h;
    if (val(hl) < 0.0) hl = 0.0;
    if (val(hr) < 0.0) hr = 0.0;
    T sl = fabs(Lt[i].u - w[i]) + sqrt(P.g * hl);
    T sr = fabs(Rt[i].u - w[i]) + sqrt(P.g * hr);
    if (P.flags & FLAG_ALPHA_CELLAVG) continue;
    if (val(sl) > val(alpha)) alpha = sl;
    if (val(sr) > val(alpha)) alpha = sr;
  }
  if (P.flags & FLAG_ALPHA_CELLAVG) {
    /* R19: the speed over the cell averages of the cells and their two nodes */
    for (int j = 0; j < n; ++j) {
      T hc = eta[j] - b[j];
      T uc = 0.0;
      if (val(hc) > P.dry_eps) uc = m[j] / hc;
      if (val(hc) < 0.0) hc = 0.0;
      T cg = sqrt(P.g * hc);
      T sa = fabs(uc - w[j]) + cg;
      T sb = fabs(uc - w[j + 1]) + cg;
      if (val(sa) > val(alpha)) alpha = sa;
      if (val(sb) > val(alpha)) alpha = sb;
    }
  }
  if (alpha_out) *alpha_out = val(alpha);
  /* Numerical fluxes (eq. (3.13), (3.17)) and bottom averages (eq. (4.9)). */
  std::vector<T> F1(n + 1), F2(n + 1), Gb(n + 1), B1(n + 1), B2(n + 1);
  for (int i = 0; i <= n; ++i) {
    const TraceFlux<T>& l = Lt[i];
    const TraceFlux<T>& r = Rt[i];
    const double wi = w[i];
    T Hl1 = l.m - wi * l.eta;
    T Hl2 = l.m * l.u + 0.5 * P.g * l.h * l.h - wi * l.m;
    T Hr1 = r.m - wi * r.eta;
    T Hr2 = r.m * r.u + 0.5 * P.g * r.h * r.h - wi * r.m;
    F1[i] = 0.5 * (Hl1 + Hr1) - 0.5 * alpha * (r.eta - l.eta);
    F2[i] = 0.5 * (Hl2 + Hr2) - 0.5 * alpha * (r.m - l.m);
    Gb[i] = -0.5 * wi * (l.b + r.b) - 0.5 * alpha * (r.b - l.b);
    B1[i] = 0.5 * (l.b + r.b);
    B2[i] = 0.5 * (l.b * l.b + r.b * r.b);
  }
  if (P.flags & FLAG_HYDROSTATIC) {
    /* Residuals with the hydrostatic reconstruction (R17-R18): each cell sums
     * H^mod over its two faces with outward normals; the bottom keeps Gb. */
    for (int j = 0; j < n; ++j) {
      T He_r, Hm_r, He_l, Hm_l;
      hydro_face_flux(P, Lt[j + 1], Rt[j + 1], +1.0, w[j + 1], alpha, He_r, Hm_r);
      hydro_face_flux(P, Rt[j], Lt[j], -1.0, w[j], alpha, He_l, Hm_l);
      const Recon<T>& o = rec[j + 1];
      T ev[4] = {Rt[j].eta, o.h[1] + o.b[1], o.h[2] + o.b[2], Lt[j + 1].eta};
      T bv[4] = {Rt[j].b, o.b[1], o.b[2], Lt[j + 1].b};
      R[j] = -(He_r + He_l);
      R[n + j] = -(Hm_r + Hm_l) + hydro_source(P.g, ev, bv);
      R[2 * n + j] = -(Gb[j + 1] - Gb[j]);
    }
    return;
  }
  if (P.flags & FLAG_NONWB) {
    /* Residuals of the scheme of Sec. 3 (eq. (3.11)-(3.12)): the fluxes and the
     * integral of the source r(q, b) = (0, -g (eta - b) b_x) over the cell by
     * the 4-point Gauss-Lobatto rule on the unlimited reconstructed values. */
    for (int j = 0; j < n; ++j) {
      const Recon<T>& o = rec[j + 1];
      T S = 0.0;
      for (int mu = 0; mu < 4; ++mu)
        S = S + (kGLW[mu] * J[j]) * ((-P.g) * (o.h[mu] * o.bx[mu]));
      R[j] = -(F1[j + 1] - F1[j]);
      R[n + j] = -(F2[j + 1] - F2[j]) + S;
      R[2 * n + j] = -(Gb[j + 1] - Gb[j]);
    }
    return;
  }
  /* Residuals with the special source (eq. (4.7)-(4.10)). */
  for (int j = 0; j < n; ++j) {
    const Recon<T>& o = rec[j + 1];
    T etabar = eta[j];
    T rint = 0.0;
    for (int mu = 0; mu < 4; ++mu) {
      T etamu = o.h[mu] + o.b[mu];
      rint = rint + (kGLW[mu] * J[j]) * (P.g * (etamu - etabar) * o.bx[mu]);
    }
    T S = 0.5 * P.g * (B2[j + 1] - B2[j]) - P.g * etabar * (B1[j + 1] - B1[j]) - rint;
    R[j] = -(F1[j + 1] - F1[j]);
    R[n + j] = -(F2[j + 1] - F2[j]) + S;
    R[2 * n + j] = -(Gb[j + 1] - Gb[j]);
  }
}

/* ------------------------------------------------------------------------ */
/* Mesh motion                                                               */
/* ------------------------------------------------------------------------ */
static double mesh_shape(const Params& P, double xi, double xmin, double xmax) {
  if (P.mesh == MESH_SINE) return std::sin(2.0 * M_PI * P.mesh_k * xi);
  double L = xmax - xmin;
  /* eq. (5.14): the quartic that also vanishes at the two jump points of the
   * step bottom (bottom_p[1], bottom_p[2]), so that nodes placed there stay
   * there: (xi - xmax)(xi - xmin)(xi - p1)(xi - p2) / (3 (xmax - xmin)^4) */
  if (P.mesh == MESH_ALIGNED)
    return (xi - xmax) * (xi - xmin) * (xi - P.bottom_p[1]) * (xi - P.bottom_p[2]) /
           (3.0 * L * L * L * L);
  /* eq. (5.1): (xi - xmax)(xi - xmin) / (3 (xmax - xmin)^2) */
  return (xi - xmax) * (xi - xmin) / (3.0 * L * L);
}

static bool prescribed_mesh(const Params& P) {
  return P.mesh == MESH_SINE || P.mesh == MESH_PAPER || P.mesh == MESH_ALIGNED;
}

/* Node speeds for the step [t, t+dt]. */
template <class T>
static void mesh_velocity(const Params& P, int n, const T* eta, const T* m, const T* b,
                          const double* xi, const double* w_given, double t, double dt, double* w) {
  if (P.mesh == MESH_GIVEN) {
    for (int i = 0; i <= n; ++i) w[i] = w_given[i];
  } else if (prescribed_mesh(P)) {
    /* Chord of X(xi,t) = xi + A S(xi) sin(omega t) over the step (eq. (2.1)):
     * (sin(om(t+dt)) - sin(om t))/dt = 2 cos(om(t+dt/2)) sin(om dt/2)/dt. */
    double om = P.mesh_omega;
    double fac = 2.0 * std::cos(om * (t + 0.5 * dt)) * std::sin(0.5 * om * dt) / dt;
    /* R21: the map's time derivative at t instead of the chord */
    if (P.flags & FLAG_W_TANGENT) fac = om * std::cos(om * t);
    for (int i = 0; i <= n; ++i) w[i] = P.mesh_A * mesh_shape(P, xi[i], xi[0], xi[n]) * fac;
  } else {
    /* Fluid-following mesh: node average of the cell velocities, two passes
     * of [1/4, 1/2, 1/4] smoothing, fixed boundary nodes (non-periodic). */
    std::vector<double> u(n), v(n + 1), v2(n + 1);
    for (int j = 0; j < n; ++j) {
      double hb = val(eta[j]) - val(b[j]);
      u[j] = hb > P.dry_eps ? val(m[j]) / hb : 0.0;
    }
    for (int i = 0; i <= n; ++i) {
      if (P.bc == BC_PERIODIC) {
        int l = (i - 1 + n) % n, r = i % n;
        v[i] = 0.5 * (u[l] + u[r]);
      } else {
        v[i] = (i == 0 || i == n) ? 0.0 : 0.5 * (u[i - 1] + u[i]);
      }
    }
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i <= n; ++i) {
        if (P.bc == BC_PERIODIC) {
          int l = (i - 1 + n) % n, r = (i + 1) % n;
          int c = i % n;
          v2[i] = 0.25 * v[l] + 0.5 * v[c] + 0.25 * v[r];
        } else {
          v2[i] = (i == 0 || i == n) ? 0.0 : 0.25 * v[i - 1] + 0.5 * v[i] + 0.25 * v[i + 1];
        }
      }
      v.swap(v2);
    }
    for (int i = 0; i <= n; ++i) w[i] = v[i];
  }
  if (P.bc == BC_PERIODIC) w[n] = w[0];
}

/* Largest node speed of the mesh at time t, for the time-step rule (R7). */
template <class T>
static double mesh_speed_bound(const Params& P, int n, const T* eta, const T* m, const T* b,
                               const double* xi, const double* w_given, double t) {
  double W = 0.0;
  if (P.mesh == MESH_GIVEN) {
    for (int i = 0; i <= n; ++i) W = std::max(W, std::fabs(w_given[i]));
  } else if (prescribed_mesh(P)) {
    double Smax = 0.0;
    for (int i = 0; i <= n; ++i) Smax = std::max(Smax, std::fabs(mesh_shape(P, xi[i], xi[0], xi[n])));
    W = std::fabs(P.mesh_A * P.mesh_omega * std::cos(P.mesh_omega * t)) * Smax;
  } else {
    std::vector<double> wf(n + 1);
    mesh_velocity(P, n, eta, m, b, xi, w_given, t, 1.0, wf.data());
    for (int i = 0; i <= n; ++i) W = std::max(W, std::fabs(wf[i]));
  }
  return W;
}

/* ------------------------------------------------------------------------ */
/* One time step: eq. (3.14)-(3.15) in 1D                                    */
/* ------------------------------------------------------------------------ */
template <class T>
static double cfl_dt(const Params& P, int n, const T* eta, const T* m, const T* b, const double* x,
                     const double* xi, const double* w_given, double t) {
  double Jmin = INFINITY, smax = 0.0;
  for (int j = 0; j < n; ++j) {
    Jmin = std::min(Jmin, x[j + 1] - x[j]);
    double hb = val(eta[j]) - val(b[j]);
    double u = hb > P.dry_eps ? val(m[j]) / hb : 0.0;
    double s = std::fabs(u) + std::sqrt(P.g * std::max(hb, 0.0));
    smax = std::max(smax, s);
  }
  double W = mesh_speed_bound(P, n, eta, m, b, xi, w_given, t);
  return P.cfl * Jmin / (smax + W);
}

template <class T>
static int step(const Params& P, int n, T* eta, T* m, T* b, double* x, const double* xi,
                const double* w_given, double* w_used, double& t, double dt, uint8_t* cls,
                Counters& cnt) {
  std::vector<double> J0(n), w(n + 1), dw(n);
  for (int j = 0; j < n; ++j) {
    J0[j] = x[j + 1] - x[j];
    if (!(J0[j] > 0.0)) return ST_MESH;
  }
  mesh_velocity(P, n, eta, m, b, xi, w_given, t, dt, w.data());
  for (int j = 0; j < n; ++j) dw[j] = w[j + 1] - w[j];
  /* Base state Q^n = J^n q^n. */
  std::vector<T> Qn(3 * n), q(3 * n), Rv(3 * n);
  for (int j = 0; j < n; ++j) {
    Qn[j] = J0[j] * eta[j];
    Qn[n + j] = J0[j] * m[j];
    Qn[2 * n + j] = J0[j] * b[j];
    q[j] = eta[j];
    q[n + j] = m[j];
    q[2 * n + j] = b[j];
  }
  std::vector<double> Js = J0, Jn(n);
  const double ca[3] = {0.0, 0.75, 1.0 / 3.0};
  const double cb[3] = {1.0, 0.25, 2.0 / 3.0};
  /* stage meshes t_n, t_{n+1}, t_{n+1/2} (eq. (3.14)): nodes x + tau w */
  const double tau[3] = {0.0, dt, 0.5 * dt};
  for (int s = 0; s < 3; ++s) {
    for (int j = 0; j < n; ++j)
      if (!(Js[j] > 0.0)) return ST_MESH;
    if (P.bottom != BOTTOM_ALE)  /* R23: b is the projection onto the stage mesh */
      for (int j = 0; j < n; ++j)
        q[2 * n + j] = bottom_average(P, x[j] + tau[s] * w[j], x[j + 1] + tau[s] * w[j + 1]);
    double alpha;
    residual(P, n, q.data(), q.data() + n, q.data() + 2 * n, Js.data(), w.data(), Rv.data(), &alpha,
             cls ? cls + (size_t)s * n : nullptr, cnt);
    for (int j = 0; j < n; ++j) Jn[j] = ca[s] * J0[j] + cb[s] * (Js[j] + dt * dw[j]);
    for (int v = 0; v < 3; ++v)
      for (int j = 0; j < n; ++j) {
        T Q = ca[s] * Qn[v * n + j] + cb[s] * (Js[j] * q[v * n + j] + dt * Rv[v * n + j]);
        q[v * n + j] = Q / Jn[j];
      }
    Js = Jn;
  }
  for (int j = 0; j < n; ++j) {
    eta[j] = q[j];
    m[j] = q[n + j];
    b[j] = q[2 * n + j];
  }
  for (int i = 0; i <= n; ++i) x[i] = x[i] + dt * w[i];
  if (P.bottom != BOTTOM_ALE)
    for (int j = 0; j < n; ++j) b[j] = bottom_average(P, x[j], x[j + 1]);
  if (w_used)
    for (int i = 0; i <= n; ++i) w_used[i] = w[i];
  t = t + dt;
  int st = ST_OK;
  if (cnt.negdepth) st = ST_NEGDEPTH;
  for (int j = 0; j < n; ++j) {
    if (!std::isfinite(val(eta[j])) || !std::isfinite(val(m[j])) || !std::isfinite(val(b[j])))
      st = ST_NONFINITE;
    if (val(eta[j]) - val(b[j]) < -P.pp_eps && st == ST_OK) st = ST_NEGDEPTH;
  }
  if (cnt.n_negweight && st == ST_OK && !(P.flags & FLAG_SPLIT)) st = ST_NEGWEIGHT;
  return st;
}

static void mass(int n, const double* eta, const double* b, const double* x, double& me, double& mb) {
  me = 0.0;
  mb = 0.0;
  for (int j = 0; j < n; ++j) {
    double J = x[j + 1] - x[j];
    me = me + J * eta[j];
    mb = mb + J * b[j];
  }
}


/* ======================================================================== */
/* 2D extension on a tensor-product moving mesh (R24-R28)                    */
/* ======================================================================== */
/* R24 Mesh: the nodes move along each logical direction on its own,
 *     x_i(t) = xi_i + Ax sin(2 pi kx xi_i) sin(omx t) and
 *     y_j(t) = eta_j + Ay sin(2 pi ky eta_j) sin(omy t), so the cells are
 *     rectangles [x_i, x_{i+1}] x [y_j, y_{j+1}] of moving widths; node speeds
 *     are the chords of eq. (2.1) per direction.
 * R25 Reconstruction (Sec. 2.2 in two dimensions): dimension by dimension.  An
 *     x-sweep of row j (the 1D hybrid procedure on the widths dx_{i-2..i+2})
 *     gives, from the cell averages, the y-line averages at the 4 Gauss-Lobatto
 *     abscissae of cell i; a y-sweep of those line averages over the rows
 *     j-2..j+2 (widths dy) gives the point values at the 4 x 4 tensor
 *     Gauss-Lobatto points of the cell.  Each sweep has its own indicators,
 *     class and hybrid weights, on (eta, hu, hv) summed (eq. (2.10), d = 3),
 *     shared by h, hu, hv and b; b_x is the y-sweep of the x-derivative line
 *     values, b_y the derivative in the y-sweep of b, each derivative taken
 *     as in 1D (R12: the 5-cell quartic's where the sweep's class is smooth,
 *     blended by M with the WENO-Z weighted slopes in the transition class).  Dx of the indicators is
 *     the largest width in the sweep's direction.  The class of a cell is the
 *     largest of its x-sweep's and its four y-sweeps' classes.
 * R26 Fluxes: the Lax-Friedrichs flux of eq. (3.13) at the 4 Gauss-Lobatto
 *     points of every edge (corners included; the rule is exact to degree 5),
 *     alpha global over all edge points and both traces; the bottom's ALE flux
 *     of eq. (3.17); the special source of eq. (4.7)-(4.10) with B1, B2 on the
 *     edges and the interior term by the 4 x 4 Gauss-Lobatto rule on the cell
 *     (its geometric area at the stage time) with the unlimited values.
 * R27 Time: eq. (3.14) with the area recurrence eq. (3.15), div(w) J taken as
 *     dA/dt = dwx_i dy_j(t_s) + dx_i(t_s) dwy_j on the stage mesh t_s.  Step
 *     size dt = CFL / ((s + Wx) / min dx + (s + Wy) / min dy): the CFL
 *     condition eq. (3.19) sums over the four edges of the cell, so both
 *     directions share the budget; Wx, Wy the largest
 *     node speeds of each direction at t_n; s the larger of the largest
 *     max(|u|, |v|) + sqrt(g h) over the cell means and the previous step's
 *     Lax-Friedrichs alpha (the largest of its three stages; 0 at the first
 *     step of a run).  Eq. (3.19) bounds dt by the alpha of eq. (3.13),
 *     taken on the traces, which a step knows only after its stages: near a
 *     wet-dry front a corner trace of small depth carries |hu / h| far above
 *     the means' speeds, and a step size from the means alone then breaks
 *     the condition by orders of magnitude (Example 5.9 on 50 x 50 cells
 *     reaches alpha ~ 9e3 against ~ 20 and negative depths within ten
 *     steps).
 * R28 Positivity: the limiter of eq. (3.20) split by direction as
 *     eq. (3.21)-(3.22) prescribe, on the rectangle's Gauss-Lobatto
 *     points: the bottom and top edge traces of a cell are limited together
 *     with delta1 (the mean of the interior rows from the Gauss-Lobatto
 *     identity), the left and right edge traces with delta2, each with its own
 *     Phi and eps = min(1e-11, hbar) (limit_edges2); hu, hv move to their means
 *     by the same Phi and b follows eta (Remark 4.1); the source keeps the
 *     unlimited point values.  A mean depth below -1e-11 ends the run
 *     (ST_NEGDEPTH).  Traces with h <= dry_eps carry u = v = 0 and hu = hv = 0
 *     in the flux as in 1D.  Boundaries periodic or transmissive in each
 *     direction. */
struct Params2 {
  double g, cfl, weno_eps, dry_eps;
  double Ax, kx, omx, Ay, ky, omy;
  int32_t bcx, bcy, flags, pad;
  double Vx, Vy;  /* a uniform translation of the nodes (R34) */
};

/* One sweep: 5 cells along a direction (widths wid), indicator variables
 * (eta, hu, hv) and the variables reconstructed with the shared weights at the
 * 4 Gauss-Lobatto points of the middle cell: out[0..3] = h, hu, hv, b,
 * out[4] = db/ds (derivative along the sweep), out[5] = the extra variable
 * (if ext5 is not NULL).  Returns the class. */
static int sweep2(const CellGeo& G, double Dx, double eps, const double e5[5], const double mx5[5],
                  const double my5[5], const double h5[5], const double b5[5], const double* ext5,
                  double out[6][4]) {
  double beta[3];
  for (int r = 0; r < 3; ++r) {
    double ev[3] = {e5[2 - r], e5[3 - r], e5[4 - r]};
    double xv[3] = {mx5[2 - r], mx5[3 - r], mx5[4 - r]};
    double yv[3] = {my5[2 - r], my5[3 - r], my5[4 - r]};
    beta[r] = beta_one(G, r, ev, Dx) + beta_one(G, r, xv, Dx) + beta_one(G, r, yv, Dx);
  }
  double tau = std::fabs(beta[0] - beta[2]);
  double betaA = (beta[0] + beta[1] + beta[2]) / 3.0;
  double gamma = tau / (betaA + eps);
  int cls = gamma <= 0.5 ? CLS_S : (gamma >= 1.0 ? CLS_N : CLS_T);
  const double* var[6] = {h5, mx5, my5, b5, b5, ext5};
  for (int mu = 0; mu < 4; ++mu) {
    double phi[3], pn[3] = {0.0, 0.0, 0.0};
    if (cls == CLS_S) {
      for (int r = 0; r < 3; ++r) phi[r] = G.d[mu][r];
    } else {
      double Kf[3];
      for (int r = 0; r < 3; ++r) {
        double q = tau / (beta[r] + eps);
        Kf[r] = 1.0 + q * q;
      }
      nonlinear_weights(G.d[mu], Kf, false, pn);
      for (int r = 0; r < 3; ++r)
        phi[r] = cls == CLS_N ? pn[r] : (2.0 * gamma - 1.0) * pn[r] + (1.0 - (2.0 * gamma - 1.0)) * G.d[mu][r];
    }
    for (int v = 0; v < 6; ++v) {
      if (!var[v]) continue;
      double acc = 0.0;
      for (int r = 0; r < 3; ++r) {
        double pr = 0.0;
        for (int i = 0; i < 3; ++i)
          pr = pr + (v == 4 ? G.cd[r][mu][i] : G.c[r][mu][i]) * var[v][2 - r + i];
        acc = acc + (v == 4 ? pn[r] : phi[r]) * pr;
      }
      out[v][mu] = acc;
    }
    /* b's derivative as in 1D (R12): the quartic's where the class is smooth,
     * blended with the WENO-Z weighted slopes by M in the transition class */
    if (cls != CLS_N) {
      double vq = 0.0;
      for (int k = 0; k < 5; ++k) vq = vq + G.cq[mu][k] * b5[k];
      const double M = 2.0 * gamma - 1.0;
      out[4][mu] = cls == CLS_S ? vq : M * out[4][mu] + (1.0 - M) * vq;
    }
  }
  return cls;
}

/* R32: one sweep of the scheme without well-balancing.  q = (eta, m_x, m_y)
 * in the local characteristic variables of the sweep direction (dir 0: x,
 * 1: y), taken from the eigenvectors of that direction's flux Jacobian at the
 * mean state (hbar, mxbar, mybar) given: with u_n, u_t the normal and
 * tangential velocities and c = sqrt(g hbar), the eigenvalues u_n - c, u_n,
 * u_n + c have the right eigenvectors (1, u_n - c, u_t), (0, 0, 1),
 * (1, u_n + c, u_t) in (eta, m_n, m_t); where hbar <= dry the frame is the
 * identity.  Each characteristic variable and b are swept as scalars with
 * their own indicators, class and weights (sweep2 on one variable); the
 * extra variable (b's x-derivative lines in the y-sweep) takes b's weights.
 * out as sweep2's (h = eta - b); returns the largest of the four classes. */
static int sweep2_char(const CellGeo& G, double Dx, double eps, double g, double dry, int dir,
                       double hbar, double mxbar, double mybar, const double e5[5],
                       const double mx5[5], const double my5[5], const double b5[5],
                       const double* ext5, double out[6][4]) {
  const double zero[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const bool chr = hbar > dry;
  double un = 0.0, ut = 0.0, c = 0.0;
  if (chr) {
    un = (dir == 0 ? mxbar : mybar) / hbar;
    ut = (dir == 0 ? mybar : mxbar) / hbar;
    c = std::sqrt(g * hbar);
  }
  double w[3][5];
  for (int k = 0; k < 5; ++k) {
    const double mn = dir == 0 ? mx5[k] : my5[k], mt = dir == 0 ? my5[k] : mx5[k];
    if (chr) {
      /* rows of the inverse of the right-eigenvector matrix */
      w[0][k] = ((un + c) * e5[k] - mn) / (2.0 * c);
      w[1][k] = mt - ut * e5[k];
      w[2][k] = ((c - un) * e5[k] + mn) / (2.0 * c);
    } else {
      w[0][k] = e5[k];
      w[1][k] = mt;
      w[2][k] = mn;
    }
  }
  double ow[3][6][4], ob[6][4];
  int cmax = 0;
  for (int q = 0; q < 3; ++q)
    cmax = std::max(cmax, sweep2(G, Dx, eps, w[q], zero, zero, w[q], w[q], nullptr, ow[q]));
  cmax = std::max(cmax, sweep2(G, Dx, eps, b5, zero, zero, b5, b5, ext5, ob));
  for (int mu = 0; mu < 4; ++mu) {
    const double a0 = ow[0][0][mu], a1 = ow[1][0][mu], a2 = ow[2][0][mu];
    double e, mn, mt;
    if (chr) {
      e = a0 + a2;
      mn = (un - c) * a0 + (un + c) * a2;
      mt = ut * a0 + a1 + ut * a2;
    } else {
      e = a0;
      mt = a1;
      mn = a2;
    }
    out[0][mu] = e - ob[0][mu];
    out[1][mu] = dir == 0 ? mn : mt;
    out[2][mu] = dir == 0 ? mt : mn;
    out[3][mu] = ob[0][mu];
    out[4][mu] = ob[4][mu];
    out[5][mu] = ob[5][mu];
  }
  return cmax;
}

struct Counters2 {
  int64_t n_class[3];
  int negw;  /* a negative linear weight on a stage mesh (R29) */
  int64_t n_limited;  /* owned cells where the limiter acted in either direction */
  int negdepth;       /* an owned mean depth below -1e-11 */
};

/* R28: the positivity limiter of eq. (3.20) in one direction of a rectangle
 * (eq. (3.21) / (3.22)): the traces h, hu, hv, b at the
 * 4 points of the cell's two edges across that direction, e[side][k][var].
 * delta is the mean of the interior lines from the Gauss-Lobatto identity
 * hbar = s1 (edge quadrature, side 0) + s1 (side 1) + (1 - 2 s1) delta;
 * m = min(edge values, delta); where m < eps = min(1e-11, hbar) the depths,
 * hu and hv move towards the cell means by Phi = (hbar - eps) / (hbar - m) and
 * the bottom follows eta (Remark 4.1).  Returns 1 if it acted. */
static int limit_edges2(double hbar, double mbar, double nbar, double e[2][4][4],
                        bool keep_b = false) {
  const double s1 = kGLW[0], PPE = 1e-11;
  double eta[2][4];
  for (int sd = 0; sd < 2; ++sd)
    for (int k = 0; k < 4; ++k) eta[sd][k] = e[sd][k][0] + e[sd][k][3];
  double Phi;
  if (hbar <= 0.0) {
    Phi = 0.0;
  } else {
    double q[2] = {0.0, 0.0};
    for (int sd = 0; sd < 2; ++sd)
      for (int k = 0; k < 4; ++k) q[sd] = q[sd] + kGLW[k] * e[sd][k][0];
    const double delta = (hbar - s1 * q[0] - s1 * q[1]) / (1.0 - 2.0 * s1);
    double mn = delta;
    for (int sd = 0; sd < 2; ++sd)
      for (int k = 0; k < 4; ++k) mn = std::min(mn, e[sd][k][0]);
    const double epsj = std::min(PPE, hbar);
    if (!(mn < epsj)) return 0;
    Phi = std::min(1.0, (hbar - epsj) / (hbar - mn));
  }
  for (int sd = 0; sd < 2; ++sd)
    for (int k = 0; k < 4; ++k) {
      double* t = e[sd][k];
      t[0] = Phi * (t[0] - hbar) + hbar;
      t[1] = Phi * (t[1] - mbar) + mbar;
      t[2] = Phi * (t[2] - nbar) + nbar;
      if (!keep_b) t[3] = eta[sd][k] - t[0];
    }
  return 1;
}

static int wrap_index(int bc, int n, int k) {
  if (k >= 0 && k < n) return k;
  if (bc == BC_PERIODIC) return ((k % n) + n) % n;
  return k < 0 ? 0 : n - 1;
}

/* Residual (eta, hu, hv, b) of the 2D scheme on the stage mesh: widths dx[nx],
 * dy[ny] at the stage time, node speeds wx[nx+1], wy[ny+1].  Returns alpha. */
static double residual2(const Params2& P, int nx, int ny, const double* eta, const double* mx,
                        const double* my, const double* b, const double* dx, const double* dy,
                        const double* wx, const double* wy, double* R, uint8_t* cls,
                        Counters2& cnt) {
  const int G = 3, EX = nx + 2 * G, EY = ny + 2 * G;
  const bool nwb = (P.flags & FLAG_NONWB) != 0;  /* R32 */
  auto cell = [&](int i, int j) { return wrap_index(P.bcx, nx, i) + nx * wrap_index(P.bcy, ny, j); };
  auto wdx = [&](int i) { return dx[wrap_index(P.bcx, nx, i)]; };
  auto wdy = [&](int j) { return dy[wrap_index(P.bcy, ny, j)]; };
  double Dxg = 0.0, Dyg = 0.0;
  for (int i = 0; i < nx; ++i) Dxg = std::max(Dxg, dx[i]);
  for (int j = 0; j < ny; ++j) Dyg = std::max(Dyg, dy[j]);
  /* the geometry of an x-sweep depends on the column only, of a y-sweep on
   * the row only (tensor-product mesh): one per column i in -1..nx and row j
   * in -1..ny */
  std::vector<CellGeo> Gx(nx + 2), Gy(ny + 2);
  for (int i = -1; i <= nx; ++i) {
    double wid[5];
    for (int k = 0; k < 5; ++k) wid[k] = wdx(i - 2 + k);
    cell_geometry(wid, Gx[i + 1]);
  }
  for (int j = -1; j <= ny; ++j) {
    double wid[5];
    for (int k = 0; k < 5; ++k) wid[k] = wdy(j - 2 + k);
    cell_geometry(wid, Gy[j + 1]);
  }
  for (const std::vector<CellGeo>* T : {&Gx, &Gy})
    for (const CellGeo& g : *T)
      for (int mu = 0; mu < 4; ++mu)
        for (int r = 0; r < 3; ++r)
          if (g.d[mu][r] < 0.0) cnt.negw = 1;
  /* x-sweeps: line values L[(i, j)][var][mu] for i in -1..nx, j in -3..ny+2 */
  const int LX = nx + 2, LY = ny + 6;
  std::vector<double> L((size_t)LX * LY * 5 * 4);
  std::vector<int> xcls((size_t)LX * LY);
  auto Lat = [&](int i, int j, int v, int mu) -> double& {
    return L[((((size_t)(j + 3) * LX + (i + 1)) * 5) + v) * 4 + mu];
  };
  for (int j = -3; j <= ny + 2; ++j)
    for (int i = -1; i <= nx; ++i) {
      double e5[5], x5[5], y5[5], h5[5], b5[5];
      for (int k = 0; k < 5; ++k) {
        const int c = cell(i - 2 + k, j);
        e5[k] = eta[c]; x5[k] = mx[c]; y5[k] = my[c]; b5[k] = b[c]; h5[k] = eta[c] - b[c];
      }
      double out[6][4];
      xcls[(size_t)(j + 3) * LX + (i + 1)] =
          nwb ? sweep2_char(Gx[i + 1], Dxg, P.weno_eps, P.g, P.dry_eps, 0, h5[2], x5[2], y5[2],
                            e5, x5, y5, b5, nullptr, out)
              : sweep2(Gx[i + 1], Dxg, P.weno_eps, e5, x5, y5, h5, b5, nullptr, out);
      for (int v = 0; v < 5; ++v)
        for (int mu = 0; mu < 4; ++mu) Lat(i, j, v, mu) = out[v][mu];
    }
  /* y-sweeps: point values V[(i, j)][var][mu][nu] for i in -1..nx, j in -1..ny;
   * var: h, hu, hv, b, b_x, b_y */
  const int VX = nx + 2, VY = ny + 2;
  std::vector<double> V((size_t)VX * VY * 6 * 16);
  auto Vat = [&](int i, int j, int v, int mu, int nu) -> double& {
    return V[((((size_t)(j + 1) * VX + (i + 1)) * 6) + v) * 16 + mu * 4 + nu];
  };
  for (int j = -1; j <= ny; ++j)
    for (int i = -1; i <= nx; ++i) {
      int cmax = xcls[(size_t)(j + 3) * LX + (i + 1)];
      for (int mu = 0; mu < 4; ++mu) {
        double e5[5], x5[5], y5[5], h5[5], b5[5], d5[5];
        for (int k = 0; k < 5; ++k) {
          const int jj = j - 2 + k;
          h5[k] = Lat(i, jj, 0, mu); x5[k] = Lat(i, jj, 1, mu); y5[k] = Lat(i, jj, 2, mu);
          b5[k] = Lat(i, jj, 3, mu); d5[k] = Lat(i, jj, 4, mu);
          e5[k] = h5[k] + b5[k];
        }
        double out[6][4];
        const int cc = cell(i, j);
        int c = nwb ? sweep2_char(Gy[j + 1], Dyg, P.weno_eps, P.g, P.dry_eps, 1, eta[cc] - b[cc],
                                  mx[cc], my[cc], e5, x5, y5, b5, d5, out)
                    : sweep2(Gy[j + 1], Dyg, P.weno_eps, e5, x5, y5, h5, b5, d5, out);
        cmax = std::max(cmax, c);
        for (int nu = 0; nu < 4; ++nu) {
          Vat(i, j, 0, mu, nu) = out[0][nu];
          Vat(i, j, 1, mu, nu) = out[1][nu];
          Vat(i, j, 2, mu, nu) = out[2][nu];
          Vat(i, j, 3, mu, nu) = out[3][nu];
          Vat(i, j, 4, mu, nu) = out[5][nu];  /* b_x: y-sweep of the x-derivative lines */
          Vat(i, j, 5, mu, nu) = out[4][nu];  /* b_y */
        }
      }
      if (i >= 0 && i < nx && j >= 0 && j < ny) {
        cnt.n_class[cmax] += 1;
        if (cls) cls[i + nx * j] = (uint8_t)cmax;
      }
    }
  /* R28: limited edge traces of every cell -1..nx x -1..ny: the left and
   * right edges (points nu) limited across x, the bottom and top edges
   * (points mu) across y; the point values V stay unlimited for the source */
  std::vector<double> TX((size_t)VX * VY * 32), TY((size_t)VX * VY * 32);
  auto TXat = [&](int i, int j, int sd, int k, int v) -> double& {
    return TX[((((size_t)(j + 1) * VX + (i + 1)) * 2 + sd) * 4 + k) * 4 + v];
  };
  auto TYat = [&](int i, int j, int sd, int k, int v) -> double& {
    return TY[((((size_t)(j + 1) * VX + (i + 1)) * 2 + sd) * 4 + k) * 4 + v];
  };
  for (int j = -1; j <= ny; ++j)
    for (int i = -1; i <= nx; ++i) {
      const int c = cell(i, j);
      const double hbar = eta[c] - b[c];
      double ex[2][4][4], ey[2][4][4];
      for (int sd = 0; sd < 2; ++sd)
        for (int k = 0; k < 4; ++k)
          for (int v = 0; v < 4; ++v) {
            ex[sd][k][v] = Vat(i, j, v, sd ? 3 : 0, k);
            ey[sd][k][v] = Vat(i, j, v, k, sd ? 3 : 0);
          }
      const int lx = limit_edges2(hbar, mx[c], my[c], ex, nwb);
      const int ly = limit_edges2(hbar, mx[c], my[c], ey, nwb);
      for (int sd = 0; sd < 2; ++sd)
        for (int k = 0; k < 4; ++k)
          for (int v = 0; v < 4; ++v) {
            TXat(i, j, sd, k, v) = ex[sd][k][v];
            TYat(i, j, sd, k, v) = ey[sd][k][v];
          }
      if (i >= 0 && i < nx && j >= 0 && j < ny) {
        if (lx || ly) cnt.n_limited += 1;
        if (hbar < -1e-11) cnt.negdepth = 1;
      }
    }
  /* traces at an edge point: h, hu, hv, b of one side; dir 0: the x-edge
   * point nu of the left (mu = 0) or right (mu = 3) edge, dir 1: the y-edge
   * point mu of the bottom (nu = 0) or top (nu = 3) edge */
  struct Tr { double h, m1, m2, b; };
  auto trace_x = [&](int i, int j, int sd, int nu) {
    Tr t{TXat(i, j, sd, nu, 0), TXat(i, j, sd, nu, 1), TXat(i, j, sd, nu, 2), TXat(i, j, sd, nu, 3)};
    if (!(t.h > P.dry_eps)) { t.m1 = 0.0; t.m2 = 0.0; }
    return t;
  };
  auto trace_y = [&](int i, int j, int mu, int nu) {
    const int sd = nu == 3 ? 1 : 0;
    Tr t{TYat(i, j, sd, mu, 0), TYat(i, j, sd, mu, 1), TYat(i, j, sd, mu, 2), TYat(i, j, sd, mu, 3)};
    if (!(t.h > P.dry_eps)) { t.m1 = 0.0; t.m2 = 0.0; }
    return t;
  };
  auto speed = [&](const Tr& t, int dir, double w) {
    double un = 0.0;
    if (t.h > P.dry_eps) un = (dir == 0 ? t.m1 : t.m2) / t.h;
    return std::fabs(un - w) + std::sqrt(P.g * std::max(t.h, 0.0));
  };
  double alpha = 0.0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i <= nx; ++i)
      for (int nu = 0; nu < 4; ++nu) {
        alpha = std::max(alpha, speed(trace_x(i - 1, j, 1, nu), 0, wx[i]));
        alpha = std::max(alpha, speed(trace_x(i, j, 0, nu), 0, wx[i]));
      }
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int mu = 0; mu < 4; ++mu) {
        alpha = std::max(alpha, speed(trace_y(i, j - 1, mu, 3), 1, wy[j]));
        alpha = std::max(alpha, speed(trace_y(i, j, mu, 0), 1, wy[j]));
      }
  /* edge integrals: flux (eta, hu, hv), bottom flux, B1, B2; with the
   * hydrostatic reconstruction (R31) also the pressure corrections of the
   * cell on the left / below (PL) and on the right / above (PR) */
  const bool hydro = (P.flags & FLAG_HYDROSTATIC) != 0;
  struct EdgeI { double F[3], Gb, B1, B2, PL, PR; };
  auto edge = [&](const Tr& l, const Tr& r, int dir, double w, double len, const double* wts,
                  int npt, const Tr* L_, const Tr* R_) {
    EdgeI e{{0, 0, 0}, 0, 0, 0, 0, 0};
    (void)l; (void)r;
    for (int k = 0; k < npt; ++k) {
      const Tr& a = L_[k];
      const Tr& c = R_[k];
      if (hydro) {
        /* eq. (4.5)-(4.6): the flux of the starred states, theta on the eta
         * component, each side's pressure correction g/2 (h^2 - h*^2) */
        const double bm = std::max(a.b, c.b);
        const double ea = a.h + a.b, ec = c.h + c.b;
        const double hsa = std::max(0.0, ea - bm), hsc = std::max(0.0, ec - bm);
        const double esa = hsa + a.b, esc = hsc + c.b;
        double usa = 0.0, vsa = 0.0, usc = 0.0, vsc = 0.0;
        if (hsa > P.dry_eps) { usa = a.m1 / hsa; vsa = a.m2 / hsa; }
        if (hsc > P.dry_eps) { usc = c.m1 / hsc; vsc = c.m2 / hsc; }
        double Ha[3], Hc[3];
        if (dir == 0) {
          Ha[0] = a.m1 - w * esa; Ha[1] = a.m1 * usa + 0.5 * P.g * hsa * hsa - w * a.m1; Ha[2] = a.m1 * vsa - w * a.m2;
          Hc[0] = c.m1 - w * esc; Hc[1] = c.m1 * usc + 0.5 * P.g * hsc * hsc - w * c.m1; Hc[2] = c.m1 * vsc - w * c.m2;
        } else {
          Ha[0] = a.m2 - w * esa; Ha[1] = a.m2 * usa - w * a.m1; Ha[2] = a.m2 * vsa + 0.5 * P.g * hsa * hsa - w * a.m2;
          Hc[0] = c.m2 - w * esc; Hc[1] = c.m2 * usc - w * c.m1; Hc[2] = c.m2 * vsc + 0.5 * P.g * hsc * hsc - w * c.m2;
        }
        const double jump[3] = {esc - esa, c.m1 - a.m1, c.m2 - a.m2};
        const double theta = 0.5 * (w + alpha) * (esc - ec) + 0.5 * (w - alpha) * (esa - ea);
        for (int q = 0; q < 3; ++q)
          e.F[q] = e.F[q] + wts[k] * (0.5 * (Ha[q] + Hc[q]) - 0.5 * alpha * jump[q]);
        e.F[0] = e.F[0] + wts[k] * theta;
        e.Gb = e.Gb + wts[k] * (-0.5 * w * (a.b + c.b) - 0.5 * alpha * (c.b - a.b));
        e.PL = e.PL + wts[k] * (0.5 * P.g * a.h * a.h - 0.5 * P.g * hsa * hsa);
        e.PR = e.PR + wts[k] * (0.5 * P.g * c.h * c.h - 0.5 * P.g * hsc * hsc);
        continue;
      }
      double ua = a.h > P.dry_eps ? a.m1 / a.h : 0.0, va = a.h > P.dry_eps ? a.m2 / a.h : 0.0;
      double uc = c.h > P.dry_eps ? c.m1 / c.h : 0.0, vc = c.h > P.dry_eps ? c.m2 / c.h : 0.0;
      double ea = a.h + a.b, ec = c.h + c.b;
      double Ha[3], Hc[3];
      if (dir == 0) {
        Ha[0] = a.m1 - w * ea; Ha[1] = a.m1 * ua + 0.5 * P.g * a.h * a.h - w * a.m1; Ha[2] = a.m1 * va - w * a.m2;
        Hc[0] = c.m1 - w * ec; Hc[1] = c.m1 * uc + 0.5 * P.g * c.h * c.h - w * c.m1; Hc[2] = c.m1 * vc - w * c.m2;
      } else {
        Ha[0] = a.m2 - w * ea; Ha[1] = a.m2 * ua - w * a.m1; Ha[2] = a.m2 * va + 0.5 * P.g * a.h * a.h - w * a.m2;
        Hc[0] = c.m2 - w * ec; Hc[1] = c.m2 * uc - w * c.m1; Hc[2] = c.m2 * vc + 0.5 * P.g * c.h * c.h - w * c.m2;
      }
      double jump[3] = {ec - ea, c.m1 - a.m1, c.m2 - a.m2};
      for (int q = 0; q < 3; ++q)
        e.F[q] = e.F[q] + wts[k] * (0.5 * (Ha[q] + Hc[q]) - 0.5 * alpha * jump[q]);
      e.Gb = e.Gb + wts[k] * (-0.5 * w * (a.b + c.b) - 0.5 * alpha * (c.b - a.b));
      e.B1 = e.B1 + wts[k] * (0.5 * (a.b + c.b));
      e.B2 = e.B2 + wts[k] * (0.5 * (a.b * a.b + c.b * c.b));
    }
    for (int q = 0; q < 3; ++q) e.F[q] = e.F[q] * len;
    e.Gb = e.Gb * len; e.B1 = e.B1 * len; e.B2 = e.B2 * len;
    e.PL = e.PL * len; e.PR = e.PR * len;
    return e;
  };
  std::vector<EdgeI> EXs((size_t)(nx + 1) * ny), EYs((size_t)nx * (ny + 1));
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i <= nx; ++i) {
      Tr Ls[4], Rs[4];
      for (int nu = 0; nu < 4; ++nu) { Ls[nu] = trace_x(i - 1, j, 1, nu); Rs[nu] = trace_x(i, j, 0, nu); }
      EXs[(size_t)j * (nx + 1) + i] = edge(Ls[0], Rs[0], 0, wx[i], dy[j], kGLW, 4, Ls, Rs);
    }
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i) {
      Tr Ls[4], Rs[4];
      for (int mu = 0; mu < 4; ++mu) { Ls[mu] = trace_y(i, j - 1, mu, 3); Rs[mu] = trace_y(i, j, mu, 0); }
      EYs[(size_t)j * nx + i] = edge(Ls[0], Rs[0], 1, wy[j], dx[i], kGLW, 4, Ls, Rs);
    }
  const size_t N = (size_t)nx * ny;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t c = (size_t)i + (size_t)nx * j;
      const EdgeI& el = EXs[(size_t)j * (nx + 1) + i];
      const EdgeI& er = EXs[(size_t)j * (nx + 1) + i + 1];
      const EdgeI& eb = EYs[(size_t)j * nx + i];
      const EdgeI& et = EYs[(size_t)(j + 1) * nx + i];
      const double etab = eta[c];
      double ix = 0.0, iy = 0.0;
      for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu) {
          double e = Vat(i, j, 0, mu, nu) + Vat(i, j, 3, mu, nu);
          ix = ix + (kGLW[mu] * kGLW[nu]) * ((e - etab) * Vat(i, j, 4, mu, nu));
          iy = iy + (kGLW[mu] * kGLW[nu]) * ((e - etab) * Vat(i, j, 5, mu, nu));
        }
      const double area = dx[i] * dy[j];
      double Sx = 0.5 * P.g * (er.B2 - el.B2) - P.g * etab * (er.B1 - el.B1) - P.g * area * ix;
      double Sy = 0.5 * P.g * (et.B2 - eb.B2) - P.g * etab * (et.B1 - eb.B1) - P.g * area * iy;
      if (hydro) {
        /* R31: the 1D source of R18 on every Gauss-Lobatto line of the cell
         * (x-lines at the points nu, y-lines at the points mu), weighted by
         * the other direction's rule; the pressure corrections of the cell's
         * own traces on its four edges */
        Sx = 0.0;
        Sy = 0.0;
        for (int k = 0; k < 4; ++k) {
          double ex_[4], bx_[4], ey_[4], by_[4];
          for (int l = 0; l < 4; ++l) {
            ex_[l] = Vat(i, j, 0, l, k) + Vat(i, j, 3, l, k);
            bx_[l] = Vat(i, j, 3, l, k);
            ey_[l] = Vat(i, j, 0, k, l) + Vat(i, j, 3, k, l);
            by_[l] = Vat(i, j, 3, k, l);
          }
          Sx = Sx + kGLW[k] * dy[j] * hydro_source(P.g, ex_, bx_);
          Sy = Sy + kGLW[k] * dx[i] * hydro_source(P.g, ey_, by_);
        }
        Sx = Sx - er.PL + el.PR;
        Sy = Sy - et.PL + eb.PR;
      }
      if (nwb) {
        /* R32: -g h grad b by the 4 x 4 Gauss-Lobatto rule on the unlimited
         * point values (b_x, b_y: the derivatives of b's reconstructions) */
        double sx = 0.0, sy = 0.0;
        for (int mu = 0; mu < 4; ++mu)
          for (int nu = 0; nu < 4; ++nu) {
            const double wgt = kGLW[mu] * kGLW[nu], hh = Vat(i, j, 0, mu, nu);
            sx = sx + wgt * (hh * Vat(i, j, 4, mu, nu));
            sy = sy + wgt * (hh * Vat(i, j, 5, mu, nu));
          }
        Sx = -P.g * area * sx;
        Sy = -P.g * area * sy;
      }
      R[c] = -(er.F[0] - el.F[0]) - (et.F[0] - eb.F[0]);
      R[N + c] = -(er.F[1] - el.F[1]) - (et.F[1] - eb.F[1]) + Sx;
      R[2 * N + c] = -(er.F[2] - el.F[2]) - (et.F[2] - eb.F[2]) + Sy;
      R[3 * N + c] = -(er.Gb - el.Gb) - (et.Gb - eb.Gb);
    }
  return alpha;
}

static double chord2(double A, double om, double t, double dt) {
  (void)A;
  return 2.0 * std::cos(om * (t + 0.5 * dt)) * std::sin(0.5 * om * dt) / dt;
}

/* One step of the 2D scheme (R27).  State eta, mx, my, b [nx*ny] in place;
 * nodes x [nx+1], y [ny+1] in place; xi, yi the reference nodes. */
static int step2(const Params2& P, int nx, int ny, double* eta, double* mx, double* my, double* b,
                 double* x, double* y, const double* xi, const double* yi, double& t, double dt,
                 uint8_t* cls, Counters2& cnt, double& alpha_max) {
  const size_t N = (size_t)nx * ny;
  std::vector<double> wx(nx + 1), wy(ny + 1);
  const double fx = chord2(P.Ax, P.omx, t, dt), fy = chord2(P.Ay, P.omy, t, dt);
  for (int i = 0; i <= nx; ++i) wx[i] = P.Vx + P.Ax * std::sin(2.0 * M_PI * P.kx * xi[i]) * fx;
  for (int j = 0; j <= ny; ++j) wy[j] = P.Vy + P.Ay * std::sin(2.0 * M_PI * P.ky * yi[j]) * fy;
  if (P.bcx == BC_PERIODIC) wx[nx] = wx[0];
  if (P.bcy == BC_PERIODIC) wy[ny] = wy[0];
  std::vector<double> dx0(nx), dy0(ny), dwx(nx), dwy(ny);
  for (int i = 0; i < nx; ++i) { dx0[i] = x[i + 1] - x[i]; dwx[i] = wx[i + 1] - wx[i]; }
  for (int j = 0; j < ny; ++j) { dy0[j] = y[j + 1] - y[j]; dwy[j] = wy[j + 1] - wy[j]; }
  std::vector<double> J0(N), Js(N), Jn(N), Qn(4 * N), q(4 * N), Rv(4 * N);
  double* st[4] = {eta, mx, my, b};
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t c = (size_t)i + (size_t)nx * j;
      J0[c] = dx0[i] * dy0[j];
      for (int v = 0; v < 4; ++v) {
        Qn[v * N + c] = J0[c] * st[v][c];
        q[v * N + c] = st[v][c];
      }
    }
  Js = J0;
  const double ca[3] = {0.0, 0.75, 1.0 / 3.0};
  const double cb[3] = {1.0, 0.25, 2.0 / 3.0};
  const double tau[3] = {0.0, dt, 0.5 * dt};
  std::vector<double> dxs(nx), dys(ny);
  for (int s = 0; s < 3; ++s) {
    for (int i = 0; i < nx; ++i) dxs[i] = dx0[i] + tau[s] * dwx[i];
    for (int j = 0; j < ny; ++j) dys[j] = dy0[j] + tau[s] * dwy[j];
    for (size_t c = 0; c < N; ++c)
      if (!(Js[c] > 0.0)) return ST_MESH;
    const double alpha =
        residual2(P, nx, ny, q.data(), q.data() + N, q.data() + 2 * N, q.data() + 3 * N,
                  dxs.data(), dys.data(), wx.data(), wy.data(), Rv.data(),
                  cls ? cls + (size_t)s * N : nullptr, cnt);
    alpha_max = std::max(alpha_max, alpha);
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t c = (size_t)i + (size_t)nx * j;
        const double dA = dwx[i] * dys[j] + dxs[i] * dwy[j];
        Jn[c] = ca[s] * J0[c] + cb[s] * (Js[c] + dt * dA);
      }
    for (int v = 0; v < 4; ++v)
      for (size_t c = 0; c < N; ++c) {
        double Q = ca[s] * Qn[v * N + c] + cb[s] * (Js[c] * q[v * N + c] + dt * Rv[v * N + c]);
        q[v * N + c] = Q / Jn[c];
      }
    Js = Jn;
  }
  for (int v = 0; v < 4; ++v)
    for (size_t c = 0; c < N; ++c) st[v][c] = q[v * N + c];
  for (int i = 0; i <= nx; ++i) x[i] = x[i] + dt * wx[i];
  for (int j = 0; j <= ny; ++j) y[j] = y[j] + dt * wy[j];
  t = t + dt;
  if (cnt.negdepth) return ST_NEGDEPTH;
  for (size_t c = 0; c < N; ++c)
    for (int v = 0; v < 4; ++v)
      if (!std::isfinite(st[v][c])) return ST_NONFINITE;
  return cnt.negw ? ST_NEGWEIGHT : ST_OK;
}

static double cfl_dt2(const Params2& P, int nx, int ny, const double* eta, const double* mx,
                      const double* my, const double* b, const double* x, const double* y,
                      const double* xi, const double* yi, double t, double alpha_prev) {
  double dxmin = INFINITY, dymin = INFINITY, smax = 0.0;
  for (int i = 0; i < nx; ++i) dxmin = std::min(dxmin, x[i + 1] - x[i]);
  for (int j = 0; j < ny; ++j) dymin = std::min(dymin, y[j + 1] - y[j]);
  for (size_t c = 0; c < (size_t)nx * ny; ++c) {
    double h = eta[c] - b[c];
    double u = h > P.dry_eps ? mx[c] / h : 0.0, v = h > P.dry_eps ? my[c] / h : 0.0;
    smax = std::max(smax, std::max(std::fabs(u), std::fabs(v)) + std::sqrt(P.g * std::max(h, 0.0)));
  }
  double Wx = 0.0, Wy = 0.0;
  for (int i = 0; i <= nx; ++i)
    Wx = std::max(Wx, std::fabs(P.Vx + P.Ax * P.omx * std::cos(P.omx * t) * std::sin(2.0 * M_PI * P.kx * xi[i])));
  for (int j = 0; j <= ny; ++j)
    Wy = std::max(Wy, std::fabs(P.Vy + P.Ay * P.omy * std::cos(P.omy * t) * std::sin(2.0 * M_PI * P.ky * yi[j])));
  smax = std::max(smax, alpha_prev);
  return P.cfl / ((smax + Wx) / dxmin + (smax + Wy) / dymin);
}
}  // namespace orc

/* ======================================================================== */
/* C interface (ctypes)                                                      */
/* ======================================================================== */
using namespace orc;

extern "C" {

/* Geometry of one cell from the widths of cells j-2..j+2: d[4][3], c[3][4][3],
 * cd[3][4][3], a[3][3][3]. */
int orc_geometry(const double* wid5, double* d, double* c, double* cd, double* a) {
  CellGeo G;
  cell_geometry(wid5, G);
  if (d) std::memcpy(d, G.d, sizeof(G.d));
  if (c) std::memcpy(c, G.c, sizeof(G.c));
  if (cd) std::memcpy(cd, G.cd, sizeof(G.cd));
  if (a) std::memcpy(a, G.a, sizeof(G.a));
  return 0;
}

/* Unlimited hybrid reconstruction of one cell.  v5 is the first indicator
 * variable (eta, or h under FLAG_BETA_FROM_H).  out[16] = h[4], m[4], b[4],
 * bx[4]; beta_out[3] (may be NULL); returns the class (0 S, 1 T, 2 N). */
int orc_reconstruct(const double* wid5, const double* v5, const double* h5, const double* m5,
                    const double* b5, double Dx, double eps, double* out, double* beta_out,
                    double* gamma_out) {
  CellGeo G;
  cell_geometry(wid5, G);
  Recon<double> o;
  reconstruct(G, Dx, eps, v5, h5, m5, b5, o);
  for (int mu = 0; mu < 4; ++mu) {
    out[mu] = o.h[mu];
    out[4 + mu] = o.m[mu];
    out[8 + mu] = o.b[mu];
    out[12 + mu] = o.bx[mu];
  }
  if (beta_out || gamma_out) {
    double beta[3];
    for (int r = 0; r < 3; ++r) {
      double hv[3] = {v5[2 - r], v5[3 - r], v5[4 - r]};
      double mv[3] = {m5[2 - r], m5[3 - r], m5[4 - r]};
      beta[r] = beta_one(G, r, hv, Dx) + beta_one(G, r, mv, Dx);
      if (beta_out) beta_out[r] = beta[r];
    }
    if (gamma_out) {
      double tau = std::fabs(beta[0] - beta[2]);
      *gamma_out = tau / ((beta[0] + beta[1] + beta[2]) / 3.0 + eps);
    }
  }
  return o.cls;
}

/* Reconstruction of one cell of the scheme without well-balancing (R22):
 * out[16] = h[4], hu[4], b[4], b_x[4] at the 4 Gauss-Lobatto points; returns
 * the cell's class (the largest of the three variables' classes). */
int orc_reconstruct_char(const double* wid5, const double* eta5, const double* m5,
                         const double* b5, double Dx, double eps, double g, double dry,
                         double* out) {
  CellGeo G;
  cell_geometry(wid5, G);
  Recon<double> o;
  reconstruct_char(G, Dx, eps, g, dry, eta5, m5, b5, o);
  for (int mu = 0; mu < 4; ++mu) {
    out[mu] = o.h[mu];
    out[4 + mu] = o.m[mu];
    out[8 + mu] = o.b[mu];
    out[12 + mu] = o.bx[mu];
  }
  return o.cls;
}

/* Cell average of the analytic bottom over [xl, xr] (R23, eq. (3.16)). */
double orc_bottom_average(const Params* P, double xl, double xr) {
  return bottom_average(*P, xl, xr);
}

/* Positivity limiter on given traces.  in[6] = hL, mL, bL, hR, mR, bR;
 * out[6] same order; hu_lim = 0 leaves the hu traces alone (R20).
 * Returns 0 untouched, 1 limited, 2 negative mean. */
int orc_limit(double hbar, double mbar, const double* in, double pp_eps, int hu_lim, double* out) {
  Recon<double> o;
  for (int mu = 0; mu < 4; ++mu) { o.h[mu] = 0; o.m[mu] = 0; o.b[mu] = 0; o.bx[mu] = 0; }
  o.h[0] = in[0]; o.m[0] = in[1]; o.b[0] = in[2];
  o.h[3] = in[3]; o.m[3] = in[4]; o.b[3] = in[5];
  Traces<double> tr;
  int r = limit_cell(hbar, mbar, o, pp_eps, tr, hu_lim != 0);
  out[0] = tr.hL; out[1] = tr.mL; out[2] = tr.bL;
  out[3] = tr.hR; out[4] = tr.mR; out[5] = tr.bR;
  return r;
}

/* Hydrostatic source of one cell (R18) from eta and b at the 4 Gauss-Lobatto
 * points of the cell (ends first and last). */
double orc_hydro_source(double g, const double* ev, const double* bv) {
  double e[4], b[4];
  for (int k = 0; k < 4; ++k) { e[k] = ev[k]; b[k] = bv[k]; }
  return hydro_source(g, e, b);
}

/* Residual RHS_j (3n: eta, hu, b) of the state (eta, hu, b) on widths J and
 * node speeds w.  Returns the LF speed in *alpha. */
int orc_residual(const Params* P, int64_t n, const double* eta, const double* m, const double* b,
                 const double* J, const double* w, double* R, double* alpha, uint8_t* cls) {
  Counters cnt{};
  residual(*P, (int)n, eta, m, b, J, w, R, alpha, cls, cnt);
  return 0;
}

/* Node speed used by a step [t, t+dt] (mesh modes other than GIVEN). */
int orc_mesh_velocity(const Params* P, int64_t n, const double* h, const double* hu, const double* b,
                      const double* xi, double t, double dt, double* w) {
  std::vector<double> eta(n);
  for (int64_t j = 0; j < n; ++j) eta[j] = h[j] + b[j];
  mesh_velocity(*P, (int)n, eta.data(), hu, b, xi, (const double*)nullptr, t, dt, w);
  return 0;
}

static void stats_init(Stats* S) {
  if (!S) return;
  std::memset(S, 0, sizeof(Stats));
  S->dt_min = INFINITY;
  S->dt_max = 0.0;
  S->h_min = INFINITY;
}

/* Run from t0 until t_end (if t_end > t0) or for max_steps steps (if > 0).
 * If dts != NULL it gives the step sizes (frozen); otherwise the CFL rule.
 * h, hu, b [n] and x [n+1] are updated in place; t_out receives the time.
 * w_given [n+1] is the node speed for MESH_GIVEN.  cls (optional) receives
 * the class of every cell, stage and step: [max_steps][3][n]. */
int orc_run(const Params* P, int64_t n_, double* h, double* hu, double* b, double* x,
            const double* xi, const double* w_given, double t0, double t_end, int64_t max_steps,
            const double* dts, double* t_out, uint8_t* cls, Stats* S) {
  const int n = (int)n_;
  if (n < 5 || !P || !h || !hu || !b || !x) return ST_ARG;
  if (P->mesh < MESH_GIVEN || P->mesh > MESH_ALIGNED) return ST_ARG;
  if (P->mesh != MESH_GIVEN && !xi) return ST_ARG;
  if (P->mesh == MESH_GIVEN && !w_given) return ST_ARG;
  stats_init(S);
  if (P->bottom != BOTTOM_ALE)  /* R23: the projection onto the initial cells */
    for (int j = 0; j < n; ++j) b[j] = bottom_average(*P, x[j], x[j + 1]);
  std::vector<double> eta(n);
  for (int j = 0; j < n; ++j) eta[j] = h[j] + b[j];
  double t = t0;
  if (S) {
    mass(n, eta.data(), b, x, S->mass_eta0, S->mass_b0);
    for (int j = 0; j < n; ++j) S->h_min = std::min(S->h_min, h[j]);
  }
  int st = ST_OK;
  int64_t k = 0;
  const bool timed = t_end > t0;
  while (true) {
    if (max_steps > 0 && k >= max_steps) break;
    if (timed && !(t < t_end)) break;
    if (!timed && max_steps <= 0) break;
    double dt;
    if (dts) dt = dts[k];
    else dt = cfl_dt(*P, n, eta.data(), hu, b, x, xi, w_given, t);
    if (timed && t + dt > t_end) dt = t_end - t;
    Counters cnt{};
    st = step(*P, n, eta.data(), hu, b, x, xi, w_given, (double*)nullptr, t, dt,
              cls ? cls + (size_t)k * 3 * n : nullptr, cnt);
    if (S) {
      S->steps += 1;
      for (int c = 0; c < 3; ++c) S->n_class[c] += cnt.n_class[c];
      S->n_limited += cnt.n_limited;
      S->n_negweight += cnt.n_negweight;
      S->dt_min = std::min(S->dt_min, dt);
      S->dt_max = std::max(S->dt_max, dt);
      for (int j = 0; j < n; ++j) S->h_min = std::min(S->h_min, eta[j] - b[j]);
    }
    ++k;
    if (st != ST_OK && st != ST_NEGWEIGHT) break;
  }
  for (int j = 0; j < n; ++j) h[j] = eta[j] - b[j];
  if (t_out) *t_out = t;
  if (S) {
    S->t = t;
    mass(n, eta.data(), b, x, S->mass_eta, S->mass_b);
    S->status = st;
  }
  return st;
}

/* Discrete adjoint of a run with frozen step sizes dts[nsteps] (prescribed
 * mesh): gauge_h[g] = hbar of the cell containing gauge_x[g] at the final
 * time; returns d/d(h0, hu0, b0) of sum_g gauge_bar[g] * gauge_h[g]. */
int orc_adjoint(const Params* P, int64_t n_, const double* h0, const double* hu0, const double* b0,
                const double* x0, const double* xi, double t0, int64_t nsteps, const double* dts,
                int64_t ngauge, const double* gauge_x, double* gauge_h, const double* gauge_bar,
                double* dh0, double* dhu0, double* db0) {
  const int n = (int)n_;
  if (n < 5 || P->mesh == MESH_FLUID || P->mesh == MESH_GIVEN) return ST_ARG;
  if (P->bottom != BOTTOM_ALE) return ST_ARG;
  std::vector<TapeNode> tape;
  tape.reserve(1 << 20);
  g_tape = &tape;
  std::vector<AD> eta(n), m(n), b(n), hin(n), muin(n), bin(n);
  for (int j = 0; j < n; ++j) {
    hin[j] = make_input(h0[j]);
    muin[j] = make_input(hu0[j]);
    bin[j] = make_input(b0[j]);
  }
  for (int j = 0; j < n; ++j) {
    eta[j] = hin[j] + bin[j];
    m[j] = muin[j];
    b[j] = bin[j];
  }
  std::vector<double> x(x0, x0 + n + 1);
  double t = t0;
  int st = ST_OK;
  for (int64_t k = 0; k < nsteps; ++k) {
    Counters cnt{};
    st = step(*P, n, eta.data(), m.data(), b.data(), x.data(), xi, (const double*)nullptr,
              (double*)nullptr, t, dts[k], (uint8_t*)nullptr, cnt);
    if (st != ST_OK && st != ST_NEGWEIGHT) break;
  }
  /* gauge readings first: they add nodes to the tape */
  std::vector<AD> hgs(ngauge);
  for (int64_t gI = 0; gI < ngauge; ++gI) {
    double xg = gauge_x[gI];
    int c = 0;
    while (c < n - 1 && !(xg < x[c + 1])) ++c;
    hgs[gI] = eta[c] - b[c];
    if (gauge_h) gauge_h[gI] = hgs[gI].v;
  }
  std::vector<double> adj(tape.size(), 0.0);
  for (int64_t gI = 0; gI < ngauge; ++gI)
    if (hgs[gI].i >= 0) adj[hgs[gI].i] += gauge_bar[gI];
  for (int64_t k = (int64_t)tape.size() - 1; k >= 0; --k) {
    double a = adj[k];
    if (a == 0.0) continue;
    const TapeNode& nd = tape[k];
    if (nd.a >= 0) adj[nd.a] += nd.da * a;
    if (nd.b >= 0) adj[nd.b] += nd.db * a;
  }
  for (int j = 0; j < n; ++j) {
    dh0[j] = adj[hin[j].i];
    dhu0[j] = adj[muin[j].i];
    db0[j] = adj[bin[j].i];
  }
  g_tape = nullptr;
  return st;
}


/* 2D tensor-product run (R24-R28): state h, hu, hv, b [nx*ny] (cell (i, j) at
 * i + nx j) and nodes x [nx+1], y [ny+1] in place, xi, yi the reference nodes;
 * from t0 until t_end (if > t0) and/or max_steps steps.  cls (optional)
 * [max_steps][3][nx*ny].  n_class (optional) [3]. */
int orc2_run(const Params2* P, int64_t nx_, int64_t ny_, double* h, double* hu, double* hv,
             double* b, double* x, double* y, const double* xi, const double* yi, double t0,
             double t_end, int64_t max_steps, double* t_out, int64_t* steps_out, uint8_t* cls,
             int64_t* n_class, double* mass /* [4]: eta, b at start and end */,
             int64_t* n_limited, double* dts_out /* step sizes of the first dts_cap steps */,
             int64_t dts_cap) {
  const int nx = (int)nx_, ny = (int)ny_;
  if (nx < 5 || ny < 5) return ST_ARG;
  if ((P->flags & FLAG_HYDROSTATIC) && (P->flags & FLAG_NONWB)) return ST_ARG;
  const size_t N = (size_t)nx * ny;
  std::vector<double> eta(N);
  for (size_t c = 0; c < N; ++c) eta[c] = h[c] + b[c];
  auto masses = [&](double& me, double& mb) {
    me = 0.0; mb = 0.0;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t c = (size_t)i + (size_t)nx * j;
        const double A = (x[i + 1] - x[i]) * (y[j + 1] - y[j]);
        me = me + A * eta[c];
        mb = mb + A * b[c];
      }
  };
  if (mass) masses(mass[0], mass[1]);
  double t = t0;
  int64_t k = 0;
  int st = ST_OK;
  Counters2 cnt{{0, 0, 0}, 0, 0, 0};
  double alpha_prev = 0.0;  /* the previous step's largest stage alpha (R27) */
  const bool timed = t_end > t0;
  while (true) {
    if (max_steps > 0 && k >= max_steps) break;
    if (timed && !(t < t_end)) break;
    if (!timed && max_steps <= 0) break;
    double dt = cfl_dt2(*P, nx, ny, eta.data(), hu, hv, b, x, y, xi, yi, t, alpha_prev);
    if (timed && t + dt > t_end) dt = t_end - t;
    if (dts_out && k < dts_cap) dts_out[k] = dt;
    alpha_prev = 0.0;
    st = step2(*P, nx, ny, eta.data(), hu, hv, b, x, y, xi, yi, t, dt,
               cls ? cls + (size_t)k * 3 * N : nullptr, cnt, alpha_prev);
    ++k;
    if (st != ST_OK) break;
  }
  for (size_t c = 0; c < N; ++c) h[c] = eta[c] - b[c];
  if (mass) masses(mass[2], mass[3]);
  if (t_out) *t_out = t;
  if (steps_out) *steps_out = k;
  if (n_class)
    for (int c = 0; c < 3; ++c) n_class[c] = cnt.n_class[c];
  if (n_limited) *n_limited = cnt.n_limited;
  return st;
}

/* Nonlinear weights of one point (eq. (2.9), with the splitting of R29 when
 * split != 0 and a linear weight is negative): d[3] linear weights, K[3] the
 * factors 1 + (tau / (beta_r + eps))^2; phi[3] out. */
void orc_nonlinear_weights(const double* d, const double* K, int split, double* phi) {
  nonlinear_weights(d, K, split != 0, phi);
}

/* The directional limiter of R28 on one cell's two opposite edges:
 * e[2][4][4] = (side, point, h/hu/hv/b), limited in place; returns 1 if it
 * acted. */
int orc2_limit_edges(double hbar, double mbar, double nbar, double* e) {
  double t[2][4][4];
  for (int k = 0; k < 32; ++k) t[k / 16][(k / 4) % 4][k % 4] = e[k];
  const int r = limit_edges2(hbar, mbar, nbar, t);
  for (int k = 0; k < 32; ++k) e[k] = t[k / 16][(k / 4) % 4][k % 4];
  return r;
}

/* One 2D reconstruction sweep (R25) on 5 cells: out[6][4] as sweep2. */
int orc2_sweep(const double* wid5, double Dx, double eps, const double* e5, const double* mx5,
               const double* my5, const double* h5, const double* b5, const double* ext5,
               double* out) {
  double o[6][4] = {{0}};
  CellGeo G;
  cell_geometry(wid5, G);
  int c = sweep2(G, Dx, eps, e5, mx5, my5, h5, b5, ext5, o);
  for (int v = 0; v < 6; ++v)
    for (int mu = 0; mu < 4; ++mu) out[v * 4 + mu] = o[v][mu];
  return c;
}

/* Residual of the 2D scheme (eta, hu, hv, b) [4][nx*ny]; returns alpha. */
double orc2_residual(const Params2* P, int64_t nx, int64_t ny, const double* eta, const double* hu,
                     const double* hv, const double* b, const double* dx, const double* dy,
                     const double* wx, const double* wy, double* R) {
  Counters2 cnt{{0, 0, 0}, 0, 0, 0};
  return residual2(*P, (int)nx, (int)ny, eta, hu, hv, b, dx, dy, wx, wy, R, nullptr, cnt);
}
}  /* extern "C" */
