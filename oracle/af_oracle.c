/*
 * af_oracle.c -- TEST INFRASTRUCTURE ONLY (see af_oracle.h).
 *
 * Plain FP64 reference of one step of the fully discrete Active Flux method for the 2D
 * Euler equations, arXiv 2508.06273.  Every function follows the paper's formulas in the
 * paper's order; nothing is blocked, fused or reordered.  Where the paper is silent the
 * reading used is stated at the function.  Circle integrals of the evolution operators are
 * computed by composite Gauss-Legendre quadrature on the arcs into which the grid lines
 * through the degree of freedom cut the circle (each arc lies in one cell, where the data
 * is a polynomial); with sub-arcs of at most pi/8 and 10 nodes the quadrature error is
 * far below FP64 rounding for the degree-6 trigonometric integrands that arise.
 */
#include "af_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------------------ */
/* Physics (paper Sec. 2: fluxes f, g and the ideal-gas equation of state)               */
/* ------------------------------------------------------------------------------------ */
void or_p2c(const double U[4], double gamma, double Q[4]) {
  Q[0] = U[0];
  Q[1] = U[0] * U[1];
  Q[2] = U[0] * U[2];
  Q[3] = U[3] / (gamma - 1.0) + 0.5 * U[0] * (U[1] * U[1] + U[2] * U[2]);
}

void or_c2p(const double Q[4], double gamma, double U[4]) {
  U[0] = Q[0];
  U[1] = Q[1] / Q[0];
  U[2] = Q[2] / Q[0];
  U[3] = (gamma - 1.0) * (Q[3] - 0.5 * (Q[1] * Q[1] + Q[2] * Q[2]) / Q[0]);
}

/* f(q) and g(q) written in primitive variables */
static void flux_f(const double U[4], double gamma, double F[4]) {
  double E = U[3] / (gamma - 1.0) + 0.5 * U[0] * (U[1] * U[1] + U[2] * U[2]);
  F[0] = U[0] * U[1];
  F[1] = U[0] * U[1] * U[1] + U[3];
  F[2] = U[0] * U[1] * U[2];
  F[3] = U[1] * (E + U[3]);
}

static void flux_g(const double U[4], double gamma, double G[4]) {
  double E = U[3] / (gamma - 1.0) + 0.5 * U[0] * (U[1] * U[1] + U[2] * U[2]);
  G[0] = U[0] * U[2];
  G[1] = U[0] * U[1] * U[2];
  G[2] = U[0] * U[2] * U[2] + U[3];
  G[3] = U[2] * (E + U[3]);
}

/* Admissible: positive density and pressure.  A zero (or NaN) value counts as failing,
 * because the sound speed of a linearisation state divides by rho and needs p > 0. */
static int admissible(const double U[4]) { return U[0] > 0.0 && U[3] > 0.0; }

static double sound(const double U[4], double gamma) { return sqrt(gamma * U[3] / U[0]); }

/* ------------------------------------------------------------------------------------ */
/* Corollary 1: correction term C(x, y, t_n, tau) = tau^2/2 * V(U, U_x, U_y)              */
/* ------------------------------------------------------------------------------------ */
void or_corr(const double U[4], const double Ux[4], const double Uy[4], double gamma,
             double tau, double out[4]) {
  double rho = U[0], u = U[1], v = U[2], p = U[3];
  double rx = Ux[0], ux = Ux[1], vx = Ux[2], px = Ux[3];
  double ry = Uy[0], uy = Uy[1], vy = Uy[2], py = Uy[3];
  double f1 = ux * ux + uy * vx;
  double f2 = uy * vx + vy * vy;
  double g1 = px * (gamma * (ux + vy) + ux) + py * vx;
  double g2 = py * (gamma * (ux + vy) + vy) + px * uy;
  double h1 = (rx * px + ry * py) / rho;
  double h2 = (rx * u + ry * v) / (rho * rho);
  double V[4];
  V[0] = rho * (f1 + f2) + u * (rx * (2.0 * ux + vy) + ry * vx) +
         v * (rx * uy + ry * (ux + 2.0 * vy)) - h1;
  V[1] = u * f1 + v * uy * (ux + vy) + g1 / rho - px * h2;
  V[2] = v * f2 + u * vx * (ux + vy) + g2 / rho - py * h2;
  V[3] = u * g1 + v * g2 + gamma * p * (f1 + f2 - h1 / rho);
  for (int k = 0; k < 4; ++k) out[k] = 0.5 * tau * tau * V[k];
}

/* ------------------------------------------------------------------------------------ */
/* Gauss-Legendre nodes on [-1,1] (Newton iteration on the Legendre recurrence)           */
/* ------------------------------------------------------------------------------------ */
void or_gl(int n, double* x, double* w) {
  for (int k = 0; k < n; ++k) {
    double z = cos(PI * (k + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int m = 2; m <= n; ++m) {
        double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int m = 2; m <= n; ++m) {
        double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[k] = z;
    w[k] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* ------------------------------------------------------------------------------------ */
/* Grid access with boundary treatment (paper Sec. 4, implementation of boundary          */
/* conditions), one ghost layer:                                                          */
/*   periodic: index wrap;                                                               */
/*   outflow:  piecewise constant extrapolation, read as a DOF-wise copy of the nearest    */
/*             boundary value;                                                            */
/*   wall:     the ghost DOF is the mirror image of the interior DOF at the same distance  */
/*             from the wall line, with the normal velocity (momentum) negated;           */
/*   inflow:   the ghost DOF holds the given inflow state.                                */
/* At a domain corner the x rule is applied first, then the y rule.                        */
/* ------------------------------------------------------------------------------------ */
typedef struct {
  const or_cfg* c; /* points at cn */
  or_cfg cn;       /* the caller's configuration with the side kinds completed */
  const double *A, *K, *X, *Y;
  int nkx, nky;
  double* Uc; /* centre values of cells -1..nx x -1..ny */
  double* Ub; /* primitive Simpson averages of the same cells */
  long long cnt[OR_NCOUNTERS];
  int gl_n;
  double glx[64], glw[64];
} ctx;

/* index i on an axis of n cells (line = 1: the grid lines 0..n, else the cells 0..n-1) with
 * boundary kinds lo, hi: the interior index that supplies the value, and in *side the side
 * whose rule then applies (-1: none, 0: lo, 1: hi) */
static int axis_map(int i, int n, int line, int lo, int hi, int* side) {
  const int last = line ? n : n - 1;
  *side = -1;
  if (lo == OR_BC_PERIODIC) return ((i % n) + n) % n;
  if (i < 0) {
    *side = 0;
    i = (lo == OR_BC_WALL) ? (line ? -i : -1 - i) : 0;
  } else if (i > last) {
    *side = 1;
    i = (hi == OR_BC_WALL) ? (line ? 2 * n - i : 2 * n - 1 - i) : last;
  }
  if (i < 0) i = 0;
  if (i > last) i = last;
  return i;
}

/* ghost rules on a value fetched through axis_map (sx, sy: the sides that apply, -1: none):
 * solid walls first (the normal velocity, or momentum, negated), then inflow (the side's
 * state replaces the value; the y side's if both apply) */
static void apply_sides(const or_cfg* c, int sx, int sy, int conserved, double o[4]) {
  if (sx >= 0 && c->bc[sx] == OR_BC_WALL) o[1] = -o[1];
  if (sy >= 0 && c->bc[2 + sy] == OR_BC_WALL) o[2] = -o[2];
  for (int axis = 0; axis < 2; ++axis) {
    const int side = axis ? sy : sx;
    if (side < 0) continue;
    const int s = 2 * axis + side;
    if (c->bc[s] != OR_BC_INFLOW) continue;
    if (conserved) or_p2c(c->inflow[s], c->gamma, o);
    else memcpy(o, c->inflow[s], sizeof(double) * 4);
  }
}

/* value of array `a` (4 variables of rows x width) at (i, j); xl, yl: lines or cells */
static void get_dof(const ctx* C, const double* a, int width, int rows, int i, int j, int xl,
                    int yl, int conserved, double o[4]) {
  const or_cfg* c = C->c;
  int sx, sy;
  const int ii = axis_map(i, c->nx, xl, c->bc[0], c->bc[1], &sx);
  const int jj = axis_map(j, c->ny, yl, c->bc[2], c->bc[3], &sy);
  for (int v = 0; v < 4; ++v) o[v] = a[(size_t)v * rows * width + (size_t)jj * width + ii];
  apply_sides(c, sx, sy, conserved, o);
}

/* Kind of cell (i, j), one layer of ghosts:
 *   CELL_OWN    interior, or a ghost beyond outflow (reconstructed from its own nodes);
 *   CELL_INFLOW a ghost beyond an inflow side: every point value, the centre included, is
 *               the inflow state;
 *   CELL_MIRROR a ghost beyond a solid wall (and no inflow side): the mirror image about the
 *               wall line of the cell (*si, *sj), whose velocity components in *flips (bit 0:
 *               u, bit 1: v) are negated. */
enum { CELL_OWN = 0, CELL_INFLOW = 1, CELL_MIRROR = 2 };
static int cell_kind(const or_cfg* c, int i, int j, int* si, int* sj, int* flips) {
  int sx, sy;
  const int mi = axis_map(i, c->nx, 0, c->bc[0], c->bc[1], &sx);
  const int mj = axis_map(j, c->ny, 0, c->bc[2], c->bc[3], &sy);
  *si = i; *sj = j; *flips = 0;
  if ((sx >= 0 && c->bc[sx] == OR_BC_INFLOW) || (sy >= 0 && c->bc[2 + sy] == OR_BC_INFLOW))
    return CELL_INFLOW;
  if (sx >= 0 && c->bc[sx] == OR_BC_WALL) { *si = mi; *flips |= 1; }
  if (sy >= 0 && c->bc[2 + sy] == OR_BC_WALL) { *sj = mj; *flips |= 2; }
  return *flips ? CELL_MIRROR : CELL_OWN;
}
static int wrap_line(int i, int n, int per) {
  if (per) return ((i % n) + n) % n;
  return i < 0 ? 0 : (i > n ? n : i);
}

static void getA(const ctx* C, int i, int j, double o[4]) {
  get_dof(C, C->A, C->c->nx, C->c->ny, i, j, 0, 0, 1, o);
}
static void getK(const ctx* C, int i, int j, double o[4]) {
  get_dof(C, C->K, C->nkx, C->nky, i, j, 1, 1, 0, o);
}
static void getX(const ctx* C, int i, int j, double o[4]) {
  get_dof(C, C->X, C->nkx, C->c->ny, i, j, 1, 0, 0, o);
}
static void getY(const ctx* C, int i, int j, double o[4]) {
  get_dof(C, C->Y, C->c->nx, C->nky, i, j, 0, 1, 0, o);
}
/* cells -2 .. n+1 in each direction: the shock indicators reach two cells beyond a DOF */
static size_t ghost_index(const ctx* C, int i, int j) {
  return (size_t)(j + 2) * (C->c->nx + 4) + (i + 2);
}

/* The nine nodes of cell (i,j): W[a][b], a = x-position (0 left, 1 centre, 2 right),
 * b = y-position; the centre node is the point value U_c obtained by inverting Simpson. */
static void cell_nodes(const ctx* C, int i, int j, double W[3][3][4], int with_centre) {
  getK(C, i, j, W[0][0]);
  getK(C, i + 1, j, W[2][0]);
  getK(C, i, j + 1, W[0][2]);
  getK(C, i + 1, j + 1, W[2][2]);
  getX(C, i, j, W[0][1]);
  getX(C, i + 1, j, W[2][1]);
  getY(C, i, j, W[1][0]);
  getY(C, i, j + 1, W[1][2]);
  if (with_centre) memcpy(W[1][1], C->Uc + 4 * ghost_index(C, i, j), sizeof(double) * 4);
}

/* Paper Sec. 2: the conserved point value at the cell midpoint by inverting Simpson's rule,
 * its primitive value U_c, and the primitive cell average U-bar by Simpson's rule.
 * Reading: if U_c is not admissible, the centre node falls back to C2P(Q-bar). */
static int prep_cell(ctx* C, int i, int j, double Uc[4], double Ub[4], int count) {
  const or_cfg* c = C->c;
  double g = c->gamma, W[3][3][4], Qn[3][3][4], Qb[4], Qc[4];
  cell_nodes(C, i, j, W, 0);
  /* a ghost cell beyond an inflow side: its point values, the centre included, are the
   * inflow state (Sec. 4.3); its average is then the Simpson average of its nodes */
  int si, sj, fl;
  if (cell_kind(c, i, j, &si, &sj, &fl) == CELL_INFLOW) {
    int sx, sy;
    double o[4] = {0, 0, 0, 0};
    axis_map(i, c->nx, 0, c->bc[0], c->bc[1], &sx);
    axis_map(j, c->ny, 0, c->bc[2], c->bc[3], &sy);
    apply_sides(c, sx, sy, 0, o);
    memcpy(Uc, o, sizeof(o));
    for (int v = 0; v < 4; ++v) {
      double corners = W[0][0][v] + W[2][0][v] + W[0][2][v] + W[2][2][v];
      double edges = W[0][1][v] + W[2][1][v] + W[1][0][v] + W[1][2][v];
      Ub[v] = (corners + 4.0 * edges + 16.0 * Uc[v]) / 36.0;
    }
    return 0;
  }
  getA(C, i, j, Qb);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (!(a == 1 && b == 1)) or_p2c(W[a][b], g, Qn[a][b]);
  for (int v = 0; v < 4; ++v) {
    double corners = Qn[0][0][v] + Qn[2][0][v] + Qn[0][2][v] + Qn[2][2][v];
    double edges = Qn[0][1][v] + Qn[2][1][v] + Qn[1][0][v] + Qn[1][2][v];
    Qc[v] = (36.0 * Qb[v] - corners - 4.0 * edges) / 16.0;
  }
  or_c2p(Qc, g, Uc);
  if (!admissible(Uc)) {
    or_c2p(Qb, g, Uc);
    if (count) C->cnt[2]++;
  }
  for (int v = 0; v < 4; ++v) {
    double corners = W[0][0][v] + W[2][0][v] + W[0][2][v] + W[2][2][v];
    double edges = W[0][1][v] + W[2][1][v] + W[1][0][v] + W[1][2][v];
    Ub[v] = (corners + 4.0 * edges + 16.0 * Uc[v]) / 36.0;
  }
  return admissible(Qb) ? 0 : -1;
}

/* Globally continuous piecewise quadratic reconstruction: in each cell the biquadratic
 * Lagrange interpolant of its nine nodes (local coordinates xi, eta in [-1/2, 1/2]). */
static void lagr(double s, double l[3]) {
  l[0] = 2.0 * s * s - s;
  l[1] = 1.0 - 4.0 * s * s;
  l[2] = 2.0 * s * s + s;
}
static void recon_eval(const ctx* C, int i, int j, double x, double y, double out[4]) {
  const or_cfg* c = C->c;
  int si, sj, fl;
  if (cell_kind(c, i, j, &si, &sj, &fl) == CELL_MIRROR) {
    /* the reflected point in the mirrored cell; the wall lines are x0, x0 + nx dx, ... */
    if (fl & 1) x = 2.0 * (c->x0 + (i < 0 ? 0 : c->nx) * c->dx) - x;
    if (fl & 2) y = 2.0 * (c->y0 + (j < 0 ? 0 : c->ny) * c->dy) - y;
    recon_eval(C, si, sj, x, y, out);
    if (fl & 1) out[1] = -out[1];
    if (fl & 2) out[2] = -out[2];
    return;
  }
  double W[3][3][4], lx[3], ly[3];
  cell_nodes(C, i, j, W, 1);
  double xc = c->x0 + (i + 0.5) * c->dx, yc = c->y0 + (j + 0.5) * c->dy;
  lagr((x - xc) / c->dx, lx);
  lagr((y - yc) / c->dy, ly);
  for (int v = 0; v < 4; ++v) {
    double s = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) s += W[a][b][v] * lx[a] * ly[b];
    out[v] = s;
  }
}

/* ------------------------------------------------------------------------------------ */
/* Evolution operators EG2 (eq. EG2) and EG1 (the first-order operator of the same       */
/* family, used on piecewise constant data in Algorithm 3).                               */
/* ------------------------------------------------------------------------------------ */
typedef struct {
  const ctx* C;    /* grid data (NULL for a callback field) */
  int rec;         /* 0: cpq reconstruction, 1: pc data (U-bar) */
  int kind, ci, cj;
  or_field_cb cb;
} field_t;

/* value of the data on an arc that lies in the cell on side (right, top) of the DOF */
static void field_arc(const field_t* F, int right, int top, double x, double y, double o[4]) {
  if (F->cb) { F->cb(x, y, o); return; }
  int i = F->ci, j = F->cj;
  if (F->kind == OR_KIND_K) { i = F->ci - 1 + right; j = F->cj - 1 + top; }
  if (F->kind == OR_KIND_X) { i = F->ci - 1 + right; }
  if (F->kind == OR_KIND_Y) { j = F->cj - 1 + top; }
  if (F->rec == 0) recon_eval(F->C, i, j, x, y, o);
  else memcpy(o, F->C->Ub + 4 * ghost_index(F->C, i, j), sizeof(double) * 4);
}

/* Value at the foot point P' = (x, y) = (xb - u' tau, yb - v' tau).  The cpq data are
 * continuous, so on a grid line either side gives the value.  For pc data a foot point on a
 * grid line takes the mean of the cells whose closure contains it (reading of the paper).
 * P' - (xb, yb) = -tau (u', v') exactly, so the side of P' is read from the signs of u' and
 * v' (tau > 0): the rounded coordinates can equal xb or yb while P' lies off the line. */
static void field_point(const field_t* F, double xb, double yb, int vline, int hline,
                        double x, double y, double up, double vp, double o[4]) {
  if (F->cb || F->rec == 0) {
    field_arc(F, x >= xb, y >= yb, x, y, o);
    return;
  }
  int xs[2], ys[2], nxs = 1, nys = 1;
  xs[0] = up < 0.0;
  ys[0] = vp < 0.0;
  if (vline && up == 0.0) { xs[0] = 0; xs[1] = 1; nxs = 2; }
  if (hline && vp == 0.0) { ys[0] = 0; ys[1] = 1; nys = 2; }
  double acc[4] = {0, 0, 0, 0}, t[4];
  for (int a = 0; a < nxs; ++a)
    for (int b = 0; b < nys; ++b) {
      field_arc(F, xs[a], ys[b], x, y, t);
      for (int v = 0; v < 4; ++v) acc[v] += t[v];
    }
  for (int v = 0; v < 4; ++v) o[v] = acc[v] / (nxs * nys);
}

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* order 2: EG2; order 1: EG1.  The integrals run over the circle Q(theta) = P' + c' tau
 * (cos theta, sin theta) of the linearised system with state lin = (rho', u', v', p'). */
static int eg_generic(const field_t* F, int order, double xb, double yb, int vline, int hline,
                      const double lin[4], double tau, double gamma, int gl_n,
                      const double* glx, const double* glw, double hmin, double out[4]) {
  if (!admissible(lin)) return OR_ERR_NONPHYSICAL;
  double rp = lin[0], up = lin[1], vp = lin[2], pp = lin[3];
  double cp = sqrt(gamma * pp / rp);
  double fu = fabs(up), fv = fabs(vp);
  if (hmin > 0.0 && ((fu > fv ? fu : fv) + cp) * tau >= 0.5 * hmin) return OR_ERR_CFL;
  double Px = xb - up * tau, Py = yb - vp * tau, r = cp * tau;

  /* angles where the circle crosses the grid lines through the DOF */
  double th[4];
  int n = 0;
  if (vline && r > 0.0) {
    double d = (xb - Px) / r;
    if (fabs(d) < 1.0) {
      double a = acos(d);
      th[n++] = a;
      th[n++] = 2.0 * PI - a;
    }
  }
  if (hline && r > 0.0) {
    double e = (yb - Py) / r;
    if (fabs(e) < 1.0) {
      double b = asin(e);
      th[n++] = b < 0.0 ? b + 2.0 * PI : b;
      th[n++] = PI - b;
    }
  }
  qsort(th, n, sizeof(double), cmp_double);
  double start[5], stop[5];
  int narc = 0;
  if (n == 0) {
    start[0] = 0.0;
    stop[0] = 2.0 * PI;
    narc = 1;
  } else {
    for (int k = 0; k < n; ++k) {
      start[narc] = th[k];
      stop[narc] = (k + 1 < n) ? th[k + 1] : th[0] + 2.0 * PI;
      ++narc;
    }
  }

  /* integrals of the four integrands */
  double I[4] = {0, 0, 0, 0};
  for (int k = 0; k < narc; ++k) {
    double L = stop[k] - start[k];
    if (!(L > 0.0)) continue;
    double tm = 0.5 * (start[k] + stop[k]);
    int right = (Px + r * cos(tm)) > xb;
    int top = (Py + r * sin(tm)) > yb;
    int m = (int)ceil(L / (PI / 8.0));
    if (m < 1) m = 1;
    double h = L / m;
    for (int s = 0; s < m; ++s) {
      double a = start[k] + s * h;
      for (int q = 0; q < gl_n; ++q) {
        double t = a + 0.5 * h * (glx[q] + 1.0);
        double wq = 0.5 * h * glw[q];
        double C = cos(t), S = sin(t), d[4];
        field_arc(F, right, top, Px + r * C, Py + r * S, d);
        double u = d[1], v = d[2], p = d[3];
        if (order == 2) {
          I[0] += wq * (p / (cp * cp) - (rp / cp) * (u * C + v * S));
          I[1] += wq * (-p * C / (rp * cp) + u * (2.0 * C * C - 0.5) + 2.0 * v * S * C);
          I[2] += wq * (-p * S / (rp * cp) + 2.0 * u * S * C + v * (2.0 * S * S - 0.5));
          I[3] += wq * (p - rp * cp * (u * C + v * S));
        } else {
          I[0] += wq * (p / (cp * cp) - 2.0 * (rp / cp) * (u * C + v * S));
          I[1] += wq * (-2.0 * p * C / (rp * cp) + u * (3.0 * C * C - 1.0) + 3.0 * v * S * C);
          I[2] += wq * (-2.0 * p * S / (rp * cp) + 3.0 * u * S * C + v * (3.0 * S * S - 1.0));
          I[3] += wq * (p - 2.0 * rp * cp * (u * C + v * S));
        }
      }
    }
  }
  double P[4];
  field_point(F, xb, yb, vline, hline, Px, Py, up, vp, P);
  if (order == 2) {
    out[0] = P[0] - 2.0 * P[3] / (cp * cp) + I[0] / PI;
    out[1] = I[1] / PI;
    out[2] = I[2] / PI;
    out[3] = -P[3] + I[3] / PI;
  } else {
    out[0] = P[0] - P[3] / (cp * cp) + I[0] / (2.0 * PI);
    out[1] = 0.5 * P[1] + I[1] / (2.0 * PI);
    out[2] = 0.5 * P[2] + I[2] / (2.0 * PI);
    out[3] = I[3] / (2.0 * PI);
  }
  return OR_OK;
}

static void dof_pos(const or_cfg* c, int kind, int ci, int cj, double* xb, double* yb) {
  *xb = c->x0 + ci * c->dx;
  *yb = c->y0 + cj * c->dy;
  if (kind == OR_KIND_X) *yb += 0.5 * c->dy;
  if (kind == OR_KIND_Y) *xb += 0.5 * c->dx;
}

static int dof_eg(const ctx* C, int order, int rec, int kind, int ci, int cj,
                  const double lin[4], double tau, double out[4]) {
  const or_cfg* c = C->c;
  field_t F = {C, rec, kind, ci, cj, NULL};
  double xb, yb;
  dof_pos(c, kind, ci, cj, &xb, &yb);
  int vline = (kind != OR_KIND_Y), hline = (kind != OR_KIND_X);
  double hmin = c->dx < c->dy ? c->dx : c->dy;
  return eg_generic(&F, order, xb, yb, vline, hline, lin, tau, c->gamma, C->gl_n, C->glx,
                    C->glw, hmin, out);
}

/* ------------------------------------------------------------------------------------ */
/* Per-DOF ingredients                                                                    */
/* ------------------------------------------------------------------------------------ */
static void get_site(const ctx* C, int kind, int i, int j, double o[4]) {
  if (kind == OR_KIND_K) getK(C, i, j, o);
  else if (kind == OR_KIND_X) getX(C, i, j, o);
  else getY(C, i, j, o);
}

static const double* Ucell(const ctx* C, int i, int j) { return C->Uc + 4 * ghost_index(C, i, j); }
static const double* Ubcell(const ctx* C, int i, int j) { return C->Ub + 4 * ghost_index(C, i, j); }

/* Derivatives for C by centred differences of neighbouring point values or cell-centre
 * values (paper, remark after Algorithm 1); the stencils with spacing dx, dy that are
 * centred on the DOF are used. */
static void dof_derivs(const ctx* C, int kind, int i, int j, double Ux[4], double Uy[4]) {
  const or_cfg* c = C->c;
  double a[4], b[4];
  if (kind == OR_KIND_K) {
    getY(C, i, j, a); getY(C, i - 1, j, b);
    for (int v = 0; v < 4; ++v) Ux[v] = (a[v] - b[v]) / c->dx;
    getX(C, i, j, a); getX(C, i, j - 1, b);
    for (int v = 0; v < 4; ++v) Uy[v] = (a[v] - b[v]) / c->dy;
  } else if (kind == OR_KIND_X) {
    getK(C, i, j + 1, a); getK(C, i, j, b);
    for (int v = 0; v < 4; ++v) Uy[v] = (a[v] - b[v]) / c->dy;
    const double *p = Ucell(C, i, j), *q = Ucell(C, i - 1, j);
    for (int v = 0; v < 4; ++v) Ux[v] = (p[v] - q[v]) / c->dx;
  } else {
    getK(C, i + 1, j, a); getK(C, i, j, b);
    for (int v = 0; v < 4; ++v) Ux[v] = (a[v] - b[v]) / c->dx;
    const double *p = Ucell(C, i, j), *q = Ucell(C, i, j - 1);
    for (int v = 0; v < 4; ++v) Uy[v] = (p[v] - q[v]) / c->dy;
  }
}

/* Mean of the primitive averages of the cells adjacent to the DOF (eq. Un+1/2 and the
 * edge-midpoint variant after it). */
static void dof_avg_lin(const ctx* C, int kind, int i, int j, double o[4]) {
  for (int v = 0; v < 4; ++v) o[v] = 0.0;
  if (kind == OR_KIND_K) {
    const double *a = Ubcell(C, i - 1, j - 1), *b = Ubcell(C, i, j - 1),
                 *d = Ubcell(C, i - 1, j), *e = Ubcell(C, i, j);
    /* summed by rows: on a solid wall the ghost row (or the ghost cell of each row) is the
     * mirror image of the interior one, and this order gives the exact mean, whose normal
     * velocity is zero, so that EG1's foot point lies on the wall line (Sec. 4.3) */
    for (int v = 0; v < 4; ++v) o[v] = 0.25 * ((a[v] + b[v]) + (d[v] + e[v]));
  } else if (kind == OR_KIND_X) {
    const double *a = Ubcell(C, i - 1, j), *b = Ubcell(C, i, j);
    for (int v = 0; v < 4; ++v) o[v] = 0.5 * (a[v] + b[v]);
  } else {
    const double *a = Ubcell(C, i, j - 1), *b = Ubcell(C, i, j);
    for (int v = 0; v < 4; ++v) o[v] = 0.5 * (a[v] + b[v]);
  }
}

/* ------------------------------------------------------------------------------------ */
/* Indicators from the primitive cell averages U-bar at t_n                               */
/* ------------------------------------------------------------------------------------ */
/* Algorithm 2: across the cell pair (L, R) in the direction of velocity component `comp`
 * (1: u, x; 2: v, y) a characteristic speed w + c or w - c changes from positive to
 * negative (the same sign choice on both sides). */
static int transonic_pair(const double* L, const double* R, int comp, double gamma) {
  const double cl = sound(L, gamma), cr = sound(R, gamma);
  if (L[comp] + cl > 0.0 && R[comp] + cr < 0.0) return 1;
  if (L[comp] - cl > 0.0 && R[comp] - cr < 0.0) return 1;
  return 0;
}

/* Algorithm 2: indicator of the corner at (x0 + I dx, y0 + J dy), from the four cells around
 * it: the two rows in x, the two columns in y. */
static int transonic_corner(const ctx* C, int I, int J) {
  const double g = C->c->gamma;
  return transonic_pair(Ubcell(C, I - 1, J), Ubcell(C, I, J), 1, g) ||
         transonic_pair(Ubcell(C, I - 1, J - 1), Ubcell(C, I, J - 1), 1, g) ||
         transonic_pair(Ubcell(C, I - 1, J - 1), Ubcell(C, I - 1, J), 2, g) ||
         transonic_pair(Ubcell(C, I, J - 1), Ubcell(C, I, J), 2, g);
}

/* Algorithm 2: a corner uses its own indicator, an edge midpoint the larger of its two end
 * corners' indicators. */
static int transonic_dof(const ctx* C, int kind, int i, int j) {
  if (kind == OR_KIND_K) return transonic_corner(C, i, j);
  if (kind == OR_KIND_X) return transonic_corner(C, i, j) || transonic_corner(C, i, j + 1);
  return transonic_corner(C, i, j) || transonic_corner(C, i + 1, j);
}

/* Sec. 3.4: theta = exp(-phi1 phi2) of the edge-midpoint DOF between the cells k-1 and k of a
 * line of cells (axis 0: X site (k, j), the cells k-2 .. k+1 of row j; axis 1: Y site (i, k),
 * the cells k-2 .. k+1 of column i).  phi1: the larger of the two pressure sensors
 * |p_{m+1} - 2 p_m + p_{m-1}| / (p_{m+1} + 2 p_m + p_{m-1}) centred on the cells m = k and
 * m = k-1; phi2 = 2^max(|w| + c) over the cells k-1 and k, w the velocity component along the
 * axis.  Reading: with a non-admissible average among the four cells theta is 0. */
static double theta_edge(const ctx* C, int axis, int i, int j) {
  const double g = C->c->gamma;
  const double* U[4];
  for (int m = 0; m < 4; ++m)
    U[m] = axis == 0 ? Ubcell(C, i - 2 + m, j) : Ubcell(C, i, j - 2 + m);
  for (int m = 0; m < 4; ++m)
    if (!admissible(U[m])) return 0.0;
  const double p0 = U[0][3], p1 = U[1][3], p2 = U[2][3], p3 = U[3][3];
  double s_hi = fabs((p3 - 2.0 * p2 + p1) / (p3 + 2.0 * p2 + p1));  /* centred on cell k */
  double s_lo = fabs((p2 - 2.0 * p1 + p0) / (p2 + 2.0 * p1 + p0));  /* centred on cell k-1 */
  const double phi1 = s_hi > s_lo ? s_hi : s_lo;
  const int comp = 1 + axis;
  const double a = fabs(U[2][comp]) + sound(U[2], g), b = fabs(U[1][comp]) + sound(U[1], g);
  const double phi2 = pow(2.0, a > b ? a : b);
  return exp(-phi1 * phi2);
}

/* Sec. 3.4: theta of a DOF.  Edge midpoints: theta_edge; a corner: the smallest theta of the
 * four edge midpoints next to it (the x-edges above and below, the y-edges right and left). */
static double theta_dof(const ctx* C, int kind, int i, int j) {
  if (kind == OR_KIND_X) return theta_edge(C, 0, i, j);
  if (kind == OR_KIND_Y) return theta_edge(C, 1, i, j);
  double t = theta_edge(C, 0, i, j), u;
  u = theta_edge(C, 0, i, j - 1); if (u < t) t = u;
  u = theta_edge(C, 1, i, j);     if (u < t) t = u;
  u = theta_edge(C, 1, i - 1, j); if (u < t) t = u;
  return t;
}

/* Lax-Friedrichs point update (Algorithm 3, last resort), in conservative variables, on the
 * lattice of DOFs of the same kind: a dual cell of size dx x dy centred at the DOF, with
 * Rusanov fluxes between the DOF and its four same-kind neighbours; the time increment is
 * tau (dt/2 for the intermediate, dt for the new time level). */
static void lf_pair(const double UL[4], const double UR[4], int dir, double gamma, double o[4]) {
  double fL[4], fR[4], QL[4], QR[4];
  if (dir == 0) { flux_f(UL, gamma, fL); flux_f(UR, gamma, fR); }
  else { flux_g(UL, gamma, fL); flux_g(UR, gamma, fR); }
  or_p2c(UL, gamma, QL);
  or_p2c(UR, gamma, QR);
  double sL = fabs(UL[1 + dir]) + sound(UL, gamma), sR = fabs(UR[1 + dir]) + sound(UR, gamma);
  double al = sL > sR ? sL : sR;
  for (int v = 0; v < 4; ++v) o[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * al * (QR[v] - QL[v]);
}
static void dof_lf(const ctx* C, int kind, int i, int j, double tau, double out[4]) {
  const or_cfg* c = C->c;
  double U0[4], Ue[4], Uw[4], Un[4], Us[4], Q0[4], Fe[4], Fw[4], Gn[4], Gs[4], Q[4];
  get_site(C, kind, i, j, U0);
  get_site(C, kind, i + 1, j, Ue);
  get_site(C, kind, i - 1, j, Uw);
  get_site(C, kind, i, j + 1, Un);
  get_site(C, kind, i, j - 1, Us);
  or_p2c(U0, c->gamma, Q0);
  lf_pair(U0, Ue, 0, c->gamma, Fe);
  lf_pair(Uw, U0, 0, c->gamma, Fw);
  lf_pair(U0, Un, 1, c->gamma, Gn);
  lf_pair(Us, U0, 1, c->gamma, Gs);
  for (int v = 0; v < 4; ++v)
    Q[v] = Q0[v] - tau / c->dx * (Fe[v] - Fw[v]) - tau / c->dy * (Gn[v] - Gs[v]);
  or_c2p(Q, c->gamma, out);
}

/* Algorithm 3 applied to one high-order point value: EG1 on pc data with the averaged
 * linearisation, then Lax-Friedrichs. */
static int limit_point(ctx* C, int kind, int i, int j, double tau, double U[4],
                       long long* cnt) {
  if (admissible(U)) return OR_OK;
  double Ut[4];
  dof_avg_lin(C, kind, i, j, Ut);
  int used_lf = 1;
  if (admissible(Ut)) {
    double lo[4];
    int e = dof_eg(C, 1, 1, kind, i, j, Ut, tau, lo);
    if (e == OR_ERR_CFL) return e;
    cnt[0]++;
    if (e == OR_OK && admissible(lo)) {
      memcpy(U, lo, sizeof(lo));
      used_lf = 0;
    }
  }
  if (used_lf) {
    double lf[4];
    dof_lf(C, kind, i, j, tau, lf);
    cnt[1]++;
    memcpy(U, lf, sizeof(lf));
    if (!admissible(U)) return OR_ERR_NONPHYSICAL;
  }
  return OR_OK;
}

/* Sec. 3.4: U := theta U + (1 - theta) U_lo, with U_lo the EG1 value on piecewise constant
 * data over tau, linearised at the mean of the adjacent averages (as in Algorithm 3).
 * Reading: where that mean is not admissible, or EG1 fails for a reason other than the CFL
 * condition, U is kept (Algorithm 3 then takes care of its positivity). */
static int shock_blend(const ctx* C, int kind, int i, int j, double tau, double theta,
                       double U[4]) {
  double Ut[4], lo[4];
  dof_avg_lin(C, kind, i, j, Ut);
  if (!admissible(Ut)) return OR_OK;
  int e = dof_eg(C, 1, 1, kind, i, j, Ut, tau, lo);
  if (e == OR_ERR_CFL) return e;
  if (e != OR_OK) return OR_OK;
  for (int v = 0; v < 4; ++v) U[v] = theta * U[v] + (1.0 - theta) * lo[v];
  return OR_OK;
}

/* Does the DOF lie on a grid line that is a solid wall? */
static int on_wall(const or_cfg* c, int kind, int i, int j) {
  if (kind != OR_KIND_Y) {
    if (i == 0 && c->bc[0] == OR_BC_WALL) return 1;
    if (i == c->nx && c->bc[1] == OR_BC_WALL) return 1;
  }
  if (kind != OR_KIND_X) {
    if (j == 0 && c->bc[2] == OR_BC_WALL) return 1;
    if (j == c->ny && c->bc[3] == OR_BC_WALL) return 1;
  }
  return 0;
}

/* One point-value DOF: intermediate and new time level (Algorithm 1; Sec. 3.1 averaged
 * linearisation; simplified method eq. 1stStep), plus Algorithm 3 when the limiter is on. */
static int dof_update(ctx* C, int kind, int i, int j, double dt, double half[4],
                      double full[4], long long* cnt) {
  const or_cfg* c = C->c;
  double U0[4], V[4] = {0, 0, 0, 0}, Ch[4] = {0, 0, 0, 0}, Cf[4] = {0, 0, 0, 0}, lin[4];
  get_site(C, kind, i, j, U0);
  if (c->correction) {
    double Ux[4], Uy[4];
    dof_derivs(C, kind, i, j, Ux, Uy);
    or_corr(U0, Ux, Uy, c->gamma, 1.0, V); /* V = C(tau=1) = V/2 */
    for (int v = 0; v < 4; ++v) {
      Ch[v] = V[v] * (0.5 * dt) * (0.5 * dt);
      Cf[v] = V[v] * dt * dt;
    }
  }
  int e;
  if (c->mode == 0) {
    double q[4];
    e = dof_eg(C, 2, 0, kind, i, j, U0, 0.25 * dt, q);
    if (e != OR_OK) return e;
    if (admissible(q)) memcpy(lin, q, sizeof(q));
    else { memcpy(lin, U0, sizeof(U0)); cnt[3]++; }
  } else if (c->mode == 1) {
    /* on a solid wall the mean of the cell averages on both sides of the wall is replaced by
     * the point value itself (Sec. 4.3) */
    if (on_wall(c, kind, i, j)) memcpy(lin, U0, sizeof(U0));
    else dof_avg_lin(C, kind, i, j, lin);
  } else {
    memcpy(lin, U0, sizeof(U0));
  }
  const double theta = c->shock ? theta_dof(C, kind, i, j) : 1.0;
  e = dof_eg(C, 2, 0, kind, i, j, lin, 0.5 * dt, half);
  if (e != OR_OK) return e;
  for (int v = 0; v < 4; ++v) half[v] += Ch[v];
  if (theta < 1.0) {
    e = shock_blend(C, kind, i, j, 0.5 * dt, theta, half);
    if (e != OR_OK) return e;
  }
  if (c->limiter) {
    e = limit_point(C, kind, i, j, 0.5 * dt, half, cnt);
    if (e != OR_OK) return e;
  } else if (!admissible(half)) {
    return OR_ERR_NONPHYSICAL;
  }
  /* full step: linearised at U^{n+1/2}, or near a transonic shock at the mean of the adjacent
   * averages (Algorithm 2) */
  double linf[4];
  if (c->tsw && transonic_dof(C, kind, i, j)) {
    dof_avg_lin(C, kind, i, j, linf);
    cnt[5]++;
  } else {
    memcpy(linf, half, sizeof(linf));
  }
  e = dof_eg(C, 2, 0, kind, i, j, linf, dt, full);
  if (e != OR_OK) return e;
  for (int v = 0; v < 4; ++v) full[v] += Cf[v];
  if (theta < 1.0) {
    e = shock_blend(C, kind, i, j, dt, theta, full);
    if (e != OR_OK) return e;
  }
  if (c->limiter) {
    e = limit_point(C, kind, i, j, dt, full, cnt);
    if (e != OR_OK) return e;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Context set-up                                                                        */
/* ------------------------------------------------------------------------------------ */
static int ctx_init(ctx* C, const or_cfg* c, const double* A, const double* K,
                    const double* X, const double* Y) {
  memset(C, 0, sizeof(*C));
  C->cn = *c;
  /* periodicity follows per_x / per_y; on a non-periodic axis a side left at
   * OR_BC_PERIODIC is outflow */
  for (int s = 0; s < 4; ++s) {
    int per = s < 2 ? c->per_x : c->per_y;
    if (per) C->cn.bc[s] = OR_BC_PERIODIC;
    else if (C->cn.bc[s] == OR_BC_PERIODIC) C->cn.bc[s] = OR_BC_OUTFLOW;
  }
  C->c = &C->cn;
  C->A = A; C->K = K; C->X = X; C->Y = Y;
  C->nkx = c->nx + (c->per_x ? 0 : 1);
  C->nky = c->ny + (c->per_y ? 0 : 1);
  C->gl_n = c->gl_n > 0 ? c->gl_n : 10;
  if (C->gl_n > 64) C->gl_n = 64;
  or_gl(C->gl_n, C->glx, C->glw);
  size_t nc = (size_t)(c->nx + 4) * (c->ny + 4);
  C->Uc = (double*)malloc(sizeof(double) * 4 * nc);
  C->Ub = (double*)malloc(sizeof(double) * 4 * nc);
  if (!C->Uc || !C->Ub) return OR_ERR_ARG;
  int bad = 0;
  long long ccount = 0;
#pragma omp parallel for reduction(+ : bad, ccount) schedule(static)
  for (int j = -2; j <= c->ny + 1; ++j) {
    for (int i = -2; i <= c->nx + 1; ++i) {
      int si, sj, fl;
      if (cell_kind(C->c, i, j, &si, &sj, &fl) == CELL_MIRROR) continue;
      int phys = (i >= 0 && i < c->nx && j >= 0 && j < c->ny);
      ctx local = *C;
      memset(local.cnt, 0, sizeof(local.cnt));
      if (prep_cell(&local, i, j, C->Uc + 4 * ghost_index(C, i, j),
                    C->Ub + 4 * ghost_index(C, i, j), phys) != 0)
        bad += phys;
      ccount += local.cnt[2];
    }
  }
  C->cnt[2] += ccount;
  /* ghost cells beyond solid walls: the mirror images of the cells they face */
  for (int j = -2; j <= c->ny + 1; ++j)
    for (int i = -2; i <= c->nx + 1; ++i) {
      int si, sj, fl;
      if (cell_kind(C->c, i, j, &si, &sj, &fl) != CELL_MIRROR) continue;
      double* uc = C->Uc + 4 * ghost_index(C, i, j);
      double* ub = C->Ub + 4 * ghost_index(C, i, j);
      memcpy(uc, C->Uc + 4 * ghost_index(C, si, sj), sizeof(double) * 4);
      memcpy(ub, C->Ub + 4 * ghost_index(C, si, sj), sizeof(double) * 4);
      if (fl & 1) { uc[1] = -uc[1]; ub[1] = -ub[1]; }
      if (fl & 2) { uc[2] = -uc[2]; ub[2] = -ub[2]; }
    }
  return bad ? OR_ERR_NONPHYSICAL : OR_OK;
}

static void ctx_free(ctx* C) {
  free(C->Uc);
  free(C->Ub);
}

/* ------------------------------------------------------------------------------------ */
/* One time step                                                                         */
/* ------------------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------------------ */
/* Sec. 3.5: flux limiting of the cell averages.  Each face flux becomes                  */
/*   F_lim = gamma F_ho + (1 - gamma) F_lo,  gamma in [0, 1],                            */
/* with F_ho the Simpson flux (eq. F) and F_lo the local Lax-Friedrichs (Rusanov) flux of */
/* the t_n averages of the two cells.  gamma is chosen, following the positivity-         */
/* preserving flux limiting of Hu, Adams and Shu (J. Comput. Phys. 242, 2013) built on   */
/* Zhang and Shu, so that the averages of both cells stay admissible: the new average of  */
/* a cell is the mean of the four states Q_lo - 4 lambda_f s_f gamma_f (F_ho - F_lo)_f    */
/* (Q_lo: the cell's low-order update; s_f = +1 on the east and north faces, -1 on the    */
/* west and south faces; lambda_f = dt/dx or dt/dy), and gamma_f is the smallest over the */
/* face's two cells of the largest theta in [0, 1] for which that state has density and  */
/* pressure at least min(1e-13, the low-order update's).  The admissible theta of one     */
/* state form an interval containing 0 (density is linear and pressure concave along the */
/* segment), found by bisection.                                                          */
/* ------------------------------------------------------------------------------------ */
static void rusanov(const double QL[4], const double QR[4], int dir, double gamma, double o[4]) {
  double UL[4], UR[4], fL[4], fR[4];
  or_c2p(QL, gamma, UL);
  or_c2p(QR, gamma, UR);
  if (dir == 0) { flux_f(UL, gamma, fL); flux_f(UR, gamma, fR); }
  else { flux_g(UL, gamma, fL); flux_g(UR, gamma, fR); }
  const double aL = fabs(UL[1 + dir]) + sound(UL, gamma);
  const double aR = fabs(UR[1 + dir]) + sound(UR, gamma);
  const double al = aL > aR ? aL : aR;
  for (int v = 0; v < 4; ++v) o[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * al * (QR[v] - QL[v]);
}

/* density >= er and pressure >= ep */
static int above(const double Q[4], double gamma, double er, double ep) {
  if (!(Q[0] >= er)) return 0;
  const double p = (gamma - 1.0) * (Q[3] - 0.5 * (Q[1] * Q[1] + Q[2] * Q[2]) / Q[0]);
  return p >= ep;
}

/* largest theta in [0, 1] with Qlo + theta d above the floors (bisection, 60 halvings) */
static double flux_theta(const double Qlo[4], const double d[4], double gamma) {
  double Ulo[4];
  or_c2p(Qlo, gamma, Ulo);
  const double er = Qlo[0] < 1e-13 ? Qlo[0] : 1e-13;
  const double ep = Ulo[3] < 1e-13 ? Ulo[3] : 1e-13;
  double Q[4];
  for (int v = 0; v < 4; ++v) Q[v] = Qlo[v] + d[v];
  if (above(Q, gamma, er, ep)) return 1.0;
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 60; ++it) {
    const double m = 0.5 * (lo + hi);
    for (int v = 0; v < 4; ++v) Q[v] = Qlo[v] + m * d[v];
    if (above(Q, gamma, er, ep)) lo = m;
    else hi = m;
  }
  return lo;
}

double or_flux_theta(const double Qlo[4], const double d[4], double gamma) {
  return flux_theta(Qlo, d, gamma);
}

/* Limit the faces of all cells in place.  F[cell][face][v]: face 0 west, 1 east, 2 south,
 * 3 north (the high-order fluxes on entry, the limited ones on return; a face shared by two
 * cells holds the same value in both).  Returns the number of limited faces, or -1 if a
 * low-order update is not admissible. */
static long long limit_fluxes(const ctx* C, double dt, double* F) {
  const or_cfg* c = C->c;
  const int nx = c->nx, ny = c->ny;
  const double g = c->gamma, lam[2] = {dt / c->dx, dt / c->dy};
  const size_t ncell = (size_t)nx * ny;
  double* FL = (double*)malloc(sizeof(double) * 16 * ncell); /* low-order fluxes, same layout */
  double* TH = (double*)malloc(sizeof(double) * 4 * ncell);  /* theta per cell and face */
  int bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t cell = (size_t)j * nx + i;
      double Q[4], Qw[4], Qe[4], Qs[4], Qn[4];
      getA(C, i, j, Q);
      getA(C, i - 1, j, Qw);
      getA(C, i + 1, j, Qe);
      getA(C, i, j - 1, Qs);
      getA(C, i, j + 1, Qn);
      double* fl = FL + 16 * cell;
      rusanov(Qw, Q, 0, g, fl + 0);
      rusanov(Q, Qe, 0, g, fl + 4);
      rusanov(Qs, Q, 1, g, fl + 8);
      rusanov(Q, Qn, 1, g, fl + 12);
      double Qlo[4], Ulo[4];
      for (int v = 0; v < 4; ++v)
        Qlo[v] = Q[v] - lam[0] * (fl[4 + v] - fl[v]) - lam[1] * (fl[12 + v] - fl[8 + v]);
      or_c2p(Qlo, g, Ulo);
      if (!admissible(Ulo)) { bad++; continue; }
      const double* fh = F + 16 * cell;
      for (int face = 0; face < 4; ++face) {
        const double sgn = (face == 1 || face == 3) ? 1.0 : -1.0;
        double d[4];
        for (int v = 0; v < 4; ++v)
          d[v] = -4.0 * lam[face / 2] * sgn * (fh[4 * face + v] - fl[4 * face + v]);
        TH[4 * cell + face] = flux_theta(Qlo, d, g);
      }
    }
  long long nlim = -1;
  if (!bad) {
    nlim = 0;
    double* out = (double*)malloc(sizeof(double) * 16 * ncell);
#pragma omp parallel for reduction(+ : nlim) schedule(static)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t cell = (size_t)j * nx + i;
        for (int face = 0; face < 4; ++face) {
          /* the neighbour across the face and its face index; none beyond a non-periodic side */
          int ni = i + (face == 1) - (face == 0), nj = j + (face == 3) - (face == 2);
          const int per = face < 2 ? c->per_x : c->per_y;
          const int n = face < 2 ? nx : ny;
          const int k = face < 2 ? ni : nj;
          double gam = TH[4 * cell + face];
          if (per || (k >= 0 && k < n)) {
            ni = ((ni % nx) + nx) % nx;
            nj = ((nj % ny) + ny) % ny;
            const double t = TH[4 * ((size_t)nj * nx + ni) + (face ^ 1)];
            if (t < gam) gam = t;
          }
          for (int v = 0; v < 4; ++v) {
            const double fh = F[16 * cell + 4 * face + v], flo = FL[16 * cell + 4 * face + v];
            out[16 * cell + 4 * face + v] = gam < 1.0 ? gam * fh + (1.0 - gam) * flo : fh;
          }
          /* count each face once: west and south faces, and east / north at a closed side */
          if (gam < 1.0 && (face == 0 || face == 2 || (face == 1 && !c->per_x && i == nx - 1) ||
                            (face == 3 && !c->per_y && j == ny - 1)))
            nlim++;
        }
      }
    memcpy(F, out, sizeof(double) * 16 * ncell);
    free(out);
  }
  free(FL);
  free(TH);
  return nlim;
}

int or_step(const or_cfg* c, double* A, double* K, double* X, double* Y, double dt,
            long long* counters) {
  if (!c || c->nx < 1 || c->ny < 1 || !(dt >= 0.0)) return OR_ERR_ARG;
#ifdef _OPENMP
  if (c->nthreads > 0) omp_set_num_threads(c->nthreads);
#endif
  ctx C;
  int err = ctx_init(&C, c, A, K, X, Y);
  if (err != OR_OK) { ctx_free(&C); return err; }
  int nkx = C.nkx, nky = C.nky, nx = c->nx, ny = c->ny;
  double g = c->gamma;
  /* per-kind site counts and arrays of the three time levels */
  int nsite[3] = {nkx * nky, nkx * ny, nx * nky};
  int wid[3] = {nkx, nkx, nx};
  double* half[3];
  double* full[3];
  for (int k = 0; k < 3; ++k) {
    half[k] = (double*)malloc(sizeof(double) * 4 * nsite[k]);
    full[k] = (double*)malloc(sizeof(double) * 4 * nsite[k]);
  }
  long long cnt[OR_NCOUNTERS] = {0};
  cnt[2] = C.cnt[2];
  for (int kind = 0; kind < 3; ++kind) {
    long long c0 = 0, c1 = 0, c3 = 0, c5 = 0;
    int kerr = 0;
#pragma omp parallel for reduction(+ : c0, c1, c3, c5) schedule(dynamic, 16)
    for (int s = 0; s < nsite[kind]; ++s) {
      int i = s % wid[kind], j = s / wid[kind];
      double h[4], f[4];
      long long lc[OR_NCOUNTERS] = {0};
      int e = dof_update(&C, kind, i, j, dt, h, f, lc);
      if (e != OR_OK) {
        /* several failing DOFs: the most negative code wins (CFL before non-physical) */
#pragma omp critical
        { if (e < kerr) kerr = e; }
      }
      c0 += lc[0]; c1 += lc[1]; c3 += lc[3]; c5 += lc[5];
      for (int v = 0; v < 4; ++v) {
        half[kind][(size_t)v * nsite[kind] + s] = h[v];
        full[kind][(size_t)v * nsite[kind] + s] = f[v];
      }
    }
    cnt[0] += c0; cnt[1] += c1; cnt[3] += c3; cnt[5] += c5;
    if (kerr < err) err = kerr;
  }
  if (err == OR_OK) {
    /* Simpson space-time fluxes (eq. F) and the finite volume update (eq. 2dfvm) */
    double* Anew = (double*)malloc(sizeof(double) * 4 * nx * ny);
    double* FF = (double*)malloc(sizeof(double) * 16 * (size_t)nx * ny); /* [cell][face][v] */
    const double* lvl[3][3];
    for (int k = 0; k < 3; ++k) {
      lvl[k][1] = half[k];
      lvl[k][2] = full[k];
    }
    lvl[0][0] = K; lvl[1][0] = X; lvl[2][0] = Y;
    int bad = 0;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
      for (int i = 0; i < nx; ++i) {
        double* Fc = FF + 16 * ((size_t)j * nx + i);
        for (int q = 0; q < 16; ++q) Fc[q] = 0.0;
        const double wt[3] = {1.0, 4.0, 1.0};
        for (int t = 0; t < 3; ++t) {
          for (int face = 0; face < 4; ++face) {
            /* face 0: west (X site (i,j)), 1: east (X site (i+1,j)),
             * 2: south (Y site (i,j)), 3: north (Y site (i,j+1)) */
            int ii = (face == 1) ? i + 1 : i, jj = (face == 3) ? j + 1 : j;
            int lx = wrap_line(ii, nx, c->per_x), ly = wrap_line(jj, ny, c->per_y);
            int k0x, k0y, k1x, k1y, mk, mx, my;
            if (face < 2) { k0x = lx; k0y = j; k1x = lx; k1y = wrap_line(j + 1, ny, c->per_y); mk = 1; mx = lx; my = j; }
            else { k0x = i; k0y = ly; k1x = wrap_line(i + 1, nx, c->per_x); k1y = ly; mk = 2; mx = i; my = ly; }
            double Ua[4], Um[4], Ub[4], fa[4], fm[4], fb[4];
            for (int v = 0; v < 4; ++v) {
              Ua[v] = lvl[0][t][(size_t)v * nsite[0] + (size_t)k0y * nkx + k0x];
              Ub[v] = lvl[0][t][(size_t)v * nsite[0] + (size_t)k1y * nkx + k1x];
              Um[v] = lvl[mk][t][(size_t)v * nsite[mk] + (size_t)my * wid[mk] + mx];
            }
            if (face < 2) { flux_f(Ua, g, fa); flux_f(Um, g, fm); flux_f(Ub, g, fb); }
            else { flux_g(Ua, g, fa); flux_g(Um, g, fm); flux_g(Ub, g, fb); }
            for (int v = 0; v < 4; ++v) Fc[4 * face + v] += wt[t] * (fa[v] + 4.0 * fm[v] + fb[v]) / 36.0;
          }
        }
      }
    }
    if (c->flux_limiter) {
      const long long nlim = limit_fluxes(&C, dt, FF);
      if (nlim < 0) bad = 1;
      else cnt[6] += nlim;
    }
#pragma omp parallel for reduction(+ : bad) schedule(static)
    for (int j = 0; j < ny; ++j) {
      for (int i = 0; i < nx; ++i) {
        const double* Fc = FF + 16 * ((size_t)j * nx + i);
        const double *Fw = Fc, *Fe = Fc + 4, *Gs = Fc + 8, *Gn = Fc + 12;
        double Q[4];
        for (int v = 0; v < 4; ++v) {
          size_t idx = (size_t)v * nx * ny + (size_t)j * nx + i;
          Q[v] = A[idx] - dt / c->dx * (Fe[v] - Fw[v]) - dt / c->dy * (Gn[v] - Gs[v]);
          Anew[idx] = Q[v];
        }
        double U[4];
        or_c2p(Q, g, U);
        if (!admissible(U)) bad++;
      }
    }
    free(FF);
    if (bad) err = OR_ERR_NONPHYSICAL;
    if (err == OR_OK) {
      memcpy(A, Anew, sizeof(double) * 4 * nx * ny);
      memcpy(K, full[0], sizeof(double) * 4 * nsite[0]);
      memcpy(X, full[1], sizeof(double) * 4 * nsite[1]);
      memcpy(Y, full[2], sizeof(double) * 4 * nsite[2]);
    }
    free(Anew);
  }
  for (int k = 0; k < 3; ++k) { free(half[k]); free(full[k]); }
  if (counters)
    for (int k = 0; k < OR_NCOUNTERS; ++k) counters[k] += cnt[k];
  ctx_free(&C);
  return err;
}

/* ------------------------------------------------------------------------------------ */
/* Time step size: dt = CFL min(dx, dy) / max over all DOFs of (max(|u|,|v|) + c), with    */
/* the cell averages converted to primitive variables.                                   */
/* ------------------------------------------------------------------------------------ */
double or_max_speed(const or_cfg* c, const double* A, const double* K, const double* X,
                    const double* Y) {
  int nkx = c->nx + (c->per_x ? 0 : 1), nky = c->ny + (c->per_y ? 0 : 1);
  double smax = 0.0;
  const double* arr[3] = {K, X, Y};
  size_t n[3] = {(size_t)nkx * nky, (size_t)nkx * c->ny, (size_t)c->nx * nky};
  for (int k = 0; k < 3; ++k)
    for (size_t s = 0; s < n[k]; ++s) {
      double U[4] = {arr[k][s], arr[k][n[k] + s], arr[k][2 * n[k] + s], arr[k][3 * n[k] + s]};
      double fu = fabs(U[1]), fv = fabs(U[2]);
      double sp = (fu > fv ? fu : fv) + sound(U, c->gamma);
      if (sp > smax) smax = sp;
    }
  size_t nc = (size_t)c->nx * c->ny;
  for (size_t s = 0; s < nc; ++s) {
    double Q[4] = {A[s], A[nc + s], A[2 * nc + s], A[3 * nc + s]}, U[4];
    or_c2p(Q, c->gamma, U);
    double fu = fabs(U[1]), fv = fabs(U[2]);
    double sp = (fu > fv ? fu : fv) + sound(U, c->gamma);
    if (sp > smax) smax = sp;
  }
  return smax;
}

int or_run(const or_cfg* c, double* A, double* K, double* X, double* Y, double* t,
           double t_end, double cfl, long long max_steps, long long* steps,
           long long* counters) {
  long long n = 0;
  double h = c->dx < c->dy ? c->dx : c->dy;
  while (*t < t_end && (max_steps <= 0 || n < max_steps)) {
    double smax = or_max_speed(c, A, K, X, Y);
    if (!(smax > 0.0)) return OR_ERR_NONPHYSICAL;
    double dt = cfl * h / smax;
    if (*t + dt >= t_end) dt = t_end - *t;
    int e = or_step(c, A, K, X, Y, dt, counters);
    if (e != OR_OK) { if (steps) *steps = n; return e; }
    if (*t + dt >= t_end) *t = t_end; else *t += dt;
    ++n;
  }
  if (steps) *steps = n;
  return OR_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Exported pieces for the pins                                                           */
/* ------------------------------------------------------------------------------------ */
int or_prep_cell(const or_cfg* c, const double* A, const double* K, const double* X,
                 const double* Y, int i, int j, double Uc[4], double Ub[4]) {
  ctx C;
  int e = ctx_init(&C, c, A, K, X, Y);
  memcpy(Uc, Ucell(&C, i, j), sizeof(double) * 4);
  memcpy(Ub, Ubcell(&C, i, j), sizeof(double) * 4);
  ctx_free(&C);
  return e;
}

int or_eval_recon(const or_cfg* c, const double* A, const double* K, const double* X,
                  const double* Y, int i, int j, double x, double y, double out[4]) {
  ctx C;
  int e = ctx_init(&C, c, A, K, X, Y);
  recon_eval(&C, i, j, x, y, out);
  ctx_free(&C);
  return e;
}

int or_dof_eg(const or_cfg* c, const double* A, const double* K, const double* X,
              const double* Y, int order, int rec, int kind, int ci, int cj,
              const double lin[4], double tau, double out[4]) {
  ctx C;
  int e = ctx_init(&C, c, A, K, X, Y);
  if (e == OR_OK) e = dof_eg(&C, order, rec, kind, ci, cj, lin, tau, out);
  ctx_free(&C);
  return e;
}

int or_dof_update(const or_cfg* c, const double* A, const double* K, const double* X,
                  const double* Y, int kind, int ci, int cj, double dt, double half[4],
                  double full[4], long long* counters) {
  ctx C;
  int e = ctx_init(&C, c, A, K, X, Y);
  long long lc[OR_NCOUNTERS] = {0};
  if (e == OR_OK) e = dof_update(&C, kind, ci, cj, dt, half, full, lc);
  if (counters)
    for (int k = 0; k < OR_NCOUNTERS; ++k) counters[k] += lc[k] + (k == 2 ? C.cnt[2] : 0);
  ctx_free(&C);
  return e;
}

int or_indicators(const or_cfg* c, const double* A, const double* K, const double* X,
                  const double* Y, int kind, int ci, int cj, double* theta, int* tsw) {
  ctx C;
  int e = ctx_init(&C, c, A, K, X, Y);
  *theta = theta_dof(&C, kind, ci, cj);
  *tsw = transonic_dof(&C, kind, ci, cj);
  ctx_free(&C);
  return e;
}

int or_lf_point(const or_cfg* c, const double* A, const double* K, const double* X,
                const double* Y, int kind, int ci, int cj, double tau, double out[4]) {
  ctx C;
  int e = ctx_init(&C, c, A, K, X, Y);
  if (e == OR_OK) dof_lf(&C, kind, ci, cj, tau, out);
  ctx_free(&C);
  return e;
}

int or_eg_cb(int order, double xb, double yb, int vline, int hline, const double lin[4],
             double tau, double gamma, or_field_cb cb, int gl_n, double out[4]) {
  double glx[64], glw[64];
  if (gl_n <= 0) gl_n = 10;
  if (gl_n > 64) gl_n = 64;
  or_gl(gl_n, glx, glw);
  field_t F = {NULL, 0, OR_KIND_K, 0, 0, cb};
  return eg_generic(&F, order, xb, yb, vline, hline, lin, tau, gamma, gl_n, glx, glw, 0.0,
                    out);
}
