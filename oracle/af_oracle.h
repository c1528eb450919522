/*
 * af_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow FP64 CPU reference of one time step of the fully discrete third-order Active
 * Flux method for the 2D Euler equations (Chudzik, Helzel, Porfetye, arXiv 2508.06273).
 * Only tests/, the package smoke check and the CPU-baseline leg of bench.py use it; the HIP
 * library shares no code with it.
 *
 * Arrays are FP64, variable-major, unpadded (see the Python input module for the site
 * geometry):  A (4,ny,nx) conserved cell averages;  K (4,nky,nkx), X (4,ny,nkx),
 * Y (4,nky,nx) primitive point values, nkx = nx + !per_x, nky = ny + !per_y.
 */
#ifndef AF_ORACLE_H
#define AF_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int nx, ny;
  double x0, y0, dx, dy;
  double gamma;
  int per_x, per_y;    /* 1: periodic; 0: the sides of the axis follow bc[] */
  int mode;            /* 0: Algorithm 1; 1: averaged linearisation (Sec. 3.1); 2: simplified */
  int correction;      /* 1: add the Corollary 1 correction C */
  int limiter;         /* 1: bound-preserving point values (Algorithm 3) */
  int gl_n;            /* Gauss-Legendre nodes per sub-arc (0: default 10) */
  int nthreads;        /* OpenMP threads (0: runtime default) */
  /* boundary kind per side (left, right, bottom, top), OR_BC_* (Sec. 4.3).  On a periodic
   * axis bc[] is ignored; on a non-periodic axis OR_BC_PERIODIC (0) reads as outflow.
   * inflow[s]: primitive inflow state of side s (used when bc[s] == OR_BC_INFLOW). */
  int bc[4];
  double inflow[4][4];
  int tsw;             /* 1: Algorithm 2 (full step linearised at averages near transonic shocks) */
  int shock;           /* 1: shock-indicator blend of high- and low-order point values (Sec. 3.4) */
  int flux_limiter;    /* 1: flux limiting of the cell averages (Sec. 3.5) */
} or_cfg;
enum { OR_BC_PERIODIC = 0, OR_BC_OUTFLOW = 1, OR_BC_WALL = 2, OR_BC_INFLOW = 3 };

enum { OR_OK = 0, OR_ERR_ARG = -1, OR_ERR_NONPHYSICAL = -2, OR_ERR_CFL = -3 };
enum { OR_KIND_K = 0, OR_KIND_X = 1, OR_KIND_Y = 2 };
/* counters[0] EG1 fallbacks, [1] LF fallbacks, [2] centre-value fallbacks,
 * [3] Algorithm 1 inner-state fallbacks, [4] unused, [5] DOFs whose full step took the
 * transonic-shock linearisation (Algorithm 2), [6] faces whose flux was limited (Sec. 3.5),
 * [7] unused */
#define OR_NCOUNTERS 8

int or_step(const or_cfg* c, double* A, double* K, double* X, double* Y, double dt,
            long long* counters);
double or_max_speed(const or_cfg* c, const double* A, const double* K, const double* X,
                    const double* Y);
int or_run(const or_cfg* c, double* A, double* K, double* X, double* Y, double* t,
           double t_end, double cfl, long long max_steps, long long* steps,
           long long* counters);

/* pieces, exported for the pins */
void or_gl(int n, double* x, double* w);
void or_p2c(const double U[4], double gamma, double Q[4]);
void or_c2p(const double Q[4], double gamma, double U[4]);
void or_corr(const double U[4], const double Ux[4], const double Uy[4], double gamma,
             double tau, double out[4]);
int or_prep_cell(const or_cfg* c, const double* A, const double* K, const double* X,
                 const double* Y, int i, int j, double Uc[4], double Ub[4]);
int or_eval_recon(const or_cfg* c, const double* A, const double* K, const double* X,
                  const double* Y, int i, int j, double x, double y, double out[4]);
int or_dof_eg(const or_cfg* c, const double* A, const double* K, const double* X,
              const double* Y, int order, int rec, int kind, int ci, int cj,
              const double lin[4], double tau, double out[4]);
int or_dof_update(const or_cfg* c, const double* A, const double* K, const double* X,
                  const double* Y, int kind, int ci, int cj, double dt, double half[4],
                  double full[4], long long* counters);
/* Shock-indicator weight theta of a DOF (Sec. 3.4) and its transonic-shock flag
 * (Algorithm 2) from the t_n state. */
int or_indicators(const or_cfg* c, const double* A, const double* K, const double* X,
                  const double* Y, int kind, int ci, int cj, double* theta, int* tsw);
int or_lf_point(const or_cfg* c, const double* A, const double* K, const double* X,
                const double* Y, int kind, int ci, int cj, double tau, double out[4]);
/* Sec. 3.5: largest theta in [0, 1] for which Qlo + theta d keeps density and pressure at
 * least min(1e-13, those of Qlo) (conserved variables). */
double or_flux_theta(const double Qlo[4], const double d[4], double gamma);
typedef void (*or_field_cb)(double x, double y, double* out4);
int or_eg_cb(int order, double xb, double yb, int vline, int hline, const double lin[4],
             double tau, double gamma, or_field_cb cb, int gl_n, double out[4]);

#ifdef __cplusplus
}
#endif
#endif
