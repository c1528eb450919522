/*
 * sanitize_main.c -- TEST INFRASTRUCTURE ONLY: a program that runs the oracle's whole step
 * under the address and undefined-behaviour sanitizers (built and run by
 * tests/test_oracle_sanitize.py with gcc).  It steps small grids through every boundary kind,
 * linearisation mode and limiter option, and checks two invariants as it goes: a uniform
 * state is preserved to rounding, and on periodic grids the sums of the conserved averages
 * are conserved to rounding.  Exit status 0 when every run and check passes.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "af_oracle.h"

static unsigned long long g_state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* xorshift64*, uniform in [0, 1) */
  g_state ^= g_state >> 12;
  g_state ^= g_state << 25;
  g_state ^= g_state >> 27;
  return (double)((g_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

typedef struct {
  int nx, ny, nkx, nky;
  double *A, *K, *X, *Y;
} arrays;

static void fill(arrays* a, const double W0[4], double amp, double gamma) {
  const size_t na = (size_t)a->nx * a->ny, nk = (size_t)a->nkx * a->nky;
  const size_t nxs = (size_t)a->nkx * a->ny, nys = (size_t)a->nx * a->nky;
  double* pts[3] = {a->K, a->X, a->Y};
  const size_t n[3] = {nk, nxs, nys};
  for (int k = 0; k < 3; ++k)
    for (size_t s = 0; s < n[k]; ++s)
      for (int v = 0; v < 4; ++v)
        pts[k][v * n[k] + s] = W0[v] * (1.0 + amp * (urand() - 0.5)) + (v == 1 || v == 2 ? amp * (urand() - 0.5) : 0.0);
  for (size_t c = 0; c < na; ++c) {
    double U[4], Q[4];
    for (int v = 0; v < 4; ++v) U[v] = W0[v] * (1.0 + amp * (urand() - 0.5));
    or_p2c(U, gamma, Q);
    for (int v = 0; v < 4; ++v) a->A[v * na + c] = Q[v];
  }
}

static int alloc(arrays* a, int nx, int ny, int per_x, int per_y) {
  a->nx = nx; a->ny = ny;
  a->nkx = nx + !per_x; a->nky = ny + !per_y;
  a->A = malloc(sizeof(double) * 4 * nx * ny);
  a->K = malloc(sizeof(double) * 4 * a->nkx * a->nky);
  a->X = malloc(sizeof(double) * 4 * a->nkx * ny);
  a->Y = malloc(sizeof(double) * 4 * nx * a->nky);
  return a->A && a->K && a->X && a->Y;
}
static void release(arrays* a) { free(a->A); free(a->K); free(a->X); free(a->Y); }

/* equal to rounding: |x - y| <= 1e-13 max|y| */
static int same(const double* x, const double* y, size_t n) {
  double m = 0.0;
  for (size_t k = 0; k < n; ++k) m = fabs(y[k]) > m ? fabs(y[k]) : m;
  for (size_t k = 0; k < n; ++k)
    if (!(fabs(x[k] - y[k]) <= 1e-13 * m)) return 0;
  return 1;
}

int main(void) {
  int failures = 0, runs = 0;
  const double gamma = 1.4;
  const int kinds[][4] = {{0, 0, 0, 0}, {1, 1, 1, 1}, {2, 2, 2, 2}, {3, 1, 2, 2}, {0, 0, 2, 3}};
  for (int bk = 0; bk < 5; ++bk)
    for (int mode = 0; mode < 3; ++mode)
      for (int opt = 0; opt < 4; ++opt) {
        or_cfg c;
        memset(&c, 0, sizeof(c));
        c.nx = 11 + bk; c.ny = 9 + mode;
        c.dx = 1.0 / c.nx; c.dy = 1.0 / c.ny;
        c.gamma = gamma; c.mode = mode; c.correction = 1; c.gl_n = 6; c.nthreads = 2;
        for (int s = 0; s < 4; ++s) {
          c.bc[s] = kinds[bk][s];
          c.inflow[s][0] = 1.0; c.inflow[s][1] = 0.4; c.inflow[s][2] = 0.0; c.inflow[s][3] = 1.0;
        }
        c.per_x = kinds[bk][0] == 0; c.per_y = kinds[bk][2] == 0;
        c.limiter = opt >= 1; c.tsw = opt == 2; c.shock = opt == 2; c.flux_limiter = opt == 3;
        arrays a;
        if (!alloc(&a, c.nx, c.ny, c.per_x, c.per_y)) return 2;
        const double W0[4] = {1.0, 0.4, kinds[bk][2] == 2 ? 0.0 : -0.3, 1.0};
        fill(&a, W0, 0.05, gamma);
        const size_t na = (size_t)c.nx * c.ny;
        double m0[4] = {0, 0, 0, 0};
        for (int v = 0; v < 4; ++v)
          for (size_t k = 0; k < na; ++k) m0[v] += a.A[v * na + k];
        long long cnt[OR_NCOUNTERS] = {0}, steps = 0;
        double t = 0.0;
        const int e = or_run(&c, a.A, a.K, a.X, a.Y, &t, 1e9, 0.3, 6, &steps, cnt);
        ++runs;
        if (e != OR_OK || steps != 6) {
          printf("run bc=%d mode=%d opt=%d: error %d after %lld steps\n", bk, mode, opt, e, steps);
          ++failures;
        } else if (c.per_x && c.per_y) {
          for (int v = 0; v < 4; ++v) {
            double m1 = 0.0;
            for (size_t k = 0; k < na; ++k) m1 += a.A[v * na + k];
            if (fabs(m1 - m0[v]) > 1e-12 * (fabs(m0[v]) + 1.0)) {
              printf("conservation bc=%d mode=%d opt=%d var=%d: %.3e\n", bk, mode, opt, v, m1 - m0[v]);
              ++failures;
            }
          }
        }
        /* a uniform state is preserved (inflow sides carry the same state; no flow through
         * a wall) */
        const double Wu[4] = {1.0, bk == 2 ? 0.0 : 0.4, 0.0, 1.0};
        fill(&a, Wu, 0.0, gamma);
        arrays b;
        if (!alloc(&b, c.nx, c.ny, c.per_x, c.per_y)) return 2;
        memcpy(b.A, a.A, sizeof(double) * 4 * na);
        memcpy(b.K, a.K, sizeof(double) * 4 * a.nkx * a.nky);
        memcpy(b.X, a.X, sizeof(double) * 4 * a.nkx * a.ny);
        memcpy(b.Y, a.Y, sizeof(double) * 4 * a.nx * a.nky);
        const int e2 = or_step(&c, a.A, a.K, a.X, a.Y, 0.2 * c.dx, cnt);
        ++runs;
        if (e2 != OR_OK || !same(a.A, b.A, 4 * na) || !same(a.K, b.K, (size_t)4 * a.nkx * a.nky) ||
            !same(a.X, b.X, (size_t)4 * a.nkx * a.ny) || !same(a.Y, b.Y, (size_t)4 * a.nx * a.nky)) {
          printf("uniform state bc=%d mode=%d opt=%d: error %d or changed\n", bk, mode, opt, e2);
          ++failures;
        }
        release(&a);
        release(&b);
      }
  printf("%d runs, %d failures\n", runs, failures);
  return failures ? 1 : 0;
}
