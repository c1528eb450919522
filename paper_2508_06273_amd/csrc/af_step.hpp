// af_step.hpp -- device functions of one Active Flux step shared by the single-grid and the
// batched kernels: step control, halo staging and cell reconstruction, the point-value update
// of a tile (with the hand-off to the positivity fix-up), the fix-up of a tile, the
// conservative update of a cell and the wave-speed maximum of a state.
#pragma once
#include "af.h"
#include "af_kernels.hpp"

namespace af {

// AF_WAVES_F32 / AF_WAVES_F64 set the wavefronts per SIMD that the register allocation of the
// point kernels aims at (0: the compiler's choice).
#ifndef AF_WAVES_F32
#define AF_WAVES_F32 0
#endif
#ifndef AF_WAVES_F64
#define AF_WAVES_F64 0
#endif
#if AF_WAVES_F32 > 0
#define AF_ATTR_F32 __attribute__((amdgpu_waves_per_eu(AF_WAVES_F32)))
#else
#define AF_ATTR_F32
#endif
#if AF_WAVES_F64 > 0
#define AF_ATTR_F64 __attribute__((amdgpu_waves_per_eu(AF_WAVES_F64)))
#else
#define AF_ATTR_F64
#endif

constexpr int FIX_BLOCKS = 1024;     // fix-up workgroups (grid-stride over the listed tiles)
constexpr int UP_THREADS = 256;      // update kernel workgroup
constexpr int UP_MAX_BLOCKS = 65536;  // update kernel grid cap (grid-stride beyond it)

// ------------------------------------------------------------------------------------------
// Kernel 1: point values of one tile of 8x8 sites.
// ------------------------------------------------------------------------------------------
// Algorithm 3 applied to a high-order value U (tests in FP64).  Returns 0 or an error code.
template <class R, int KIND>
__device__ __forceinline__ int limit_value(const Smem<R>& S, const Params& P, const Geo<R>& G,
                                           const double* site, int a, int b, int cb,
                                           const double Ut[4], double tau, double U[4],
                                           DevState* dev) {
  if (admissible(U[0], U[3])) return 0;
  if (admissible(Ut[0], Ut[3])) {
    R d[4];
    const int e = eg1_pc<R, KIND>(S.ub, cb, Ut, R(tau), G, d);
    if (e == ERR_CFL) return e;
    atomicAdd(&dev->cnt[AF_CNT_EG1], 1ull);
    double lo[4];
    for (int v = 0; v < 4; ++v) lo[v] = Ut[v] + (double)d[v];
    if (e == 0 && admissible(lo[0], lo[3])) {
      for (int v = 0; v < 4; ++v) U[v] = lo[v];
      return 0;
    }
  }
  lf_update(site, a, b, tau, P, U);
  atomicAdd(&dev->cnt[AF_CNT_LF], 1ull);
  return admissible(U[0], U[3]) ? 0 : ERR_NONPHYS;
}

// Hand a DOF that needs Algorithm 3 to the fix-up pass: set its lane bit and list the tile.
__device__ __forceinline__ void mark_fix(const Bufs& B, int tile, int kind, int lane) {
  atomicOr(&B.fix_mask[4 * (long long)tile + kind], 1ull << lane);
  if (atomicExch(&B.fix_mask[4 * (long long)tile + 3], 1ull) == 0ull) {
    const unsigned int k = atomicAdd(B.fix_count, 1u);
    B.fix_list[k] = B.tile_base + tile;
  }
}

// One DOF through the rounds of the point update.  States are carried in FP64; the
// evolution operators work in the bulk type R on deviations from the linearisation state.
// FIX = false (main pass): a DOF whose value needs the positivity limiter is left to the
// fix-up pass, which keeps the rare limiter code out of the main kernel's registers.
// FIX = true (fix-up pass): the same computation with Algorithm 3 applied.
// Sec. 3.4: the low-order value U_lo = EG1 on the piecewise constant data, linearised at the mean
// Ut of the adjacent primitive averages.  On data constant in the four quadrants around the DOF
// the circle's centre and radius both scale with tau, so every arc angle, and EG1's value, is
// the same for tau = dt/2 and tau = dt: one evaluation serves both time levels; only the CFL
// check depends on tau.  Returns 0 (lo valid), 1 (no blend: Ut not admissible) or ERR_CFL.
template <class R, int KIND>
__device__ __forceinline__ int shock_low(const Smem<R>& S, const Geo<R>& G, int cb,
                                         const double Ut[4], double tau, double lo[4]) {
  if (!admissible(Ut[0], Ut[3])) return 1;
  R d[4];
  const int e = eg1_pc<R, KIND>(S.ub, cb, Ut, R(tau), G, d);
  if (e) return e;
#pragma unroll
  for (int v = 0; v < 4; ++v) lo[v] = Ut[v] + (double)d[v];
  return 0;
}

// eg1_pc's CFL condition for the linearisation state Ut over tau.
template <class R>
__device__ __forceinline__ bool eg1_cfl_fails(const Geo<R>& G, const double Ut[4], double tau) {
  const R rp = R(Ut[0]), up = R(Ut[1]), vp = R(Ut[2]), pp = R(Ut[3]);
  const R c = Math<R>::sqrt_(G.gamma * pp / rp);
  return (mx(absr(up), absr(vp)) + c) * R(tau) >= G.half_h;
}

template <class R, int KIND, bool FIX, bool IND>
__device__ __forceinline__ void evolve_dof(Smem<R>& S, const Ind* I, const Params& P,
                                           const Bufs& B, DevState* dev, int tile, int a, int b,
                                           int gi, int gj, double dt, double& speed) {
  const Geo<R> G = {R(P.idx), R(0.5 * P.dy * P.idx), R(P.gamma), R(0.5 * P.hmin), R(P.dx)};
  // 1 / tau of the three evaluations (tau = dt/4, dt/2, dt): powers of two times 1 / dt
  const double idt = 1.0 / dt;
  const double* site = (KIND == KIND_K) ? S.sk : (KIND == KIND_X ? S.sx : S.sy);
  const int s0 = sidx(a, b);
  double U0[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) U0[v] = site[v * NS + s0];

  // cells around the DOF and the neighbours of the derivative stencils
  int cb;
  R Ux[4], Uy[4];
  if constexpr (KIND == KIND_K) {
    cb = a + b * HC;  // cell (a-1, b-1)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Ux[v] = R((S.sy[v * NS + sidx(a, b)] - S.sy[v * NS + sidx(a - 1, b)]) * P.idx);
      Uy[v] = R((S.sx[v * NS + sidx(a, b)] - S.sx[v * NS + sidx(a, b - 1)]) * P.idy);
    }
  } else if constexpr (KIND == KIND_X) {
    cb = a + (b + 1) * HC;  // cell (a-1, b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Uy[v] = R((S.sk[v * NS + sidx(a, b + 1)] - S.sk[v * NS + sidx(a, b)]) * P.idy);
      Ux[v] = R((S.c0[v * NC + cb + 1] - S.c0[v * NC + cb]) * P.idx);
    }
  } else {
    cb = (a + 1) + b * HC;  // cell (a, b-1)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Ux[v] = R((S.sk[v * NS + sidx(a + 1, b)] - S.sk[v * NS + sidx(a, b)]) * P.idx);
      Uy[v] = R((S.c0[v * NC + cb + HC] - S.c0[v * NC + cb]) * P.idy);
    }
  }
  // mean of the adjacent primitive averages (read from LDS where it is used)
  auto avg_lin = [&](double Ut[4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if constexpr (KIND == KIND_K)
        Ut[v] = 0.25 * ((S.ub[v * NC + cb] + S.ub[v * NC + cb + 1]) +
                        (S.ub[v * NC + cb + HC] + S.ub[v * NC + cb + HC + 1]));
      else
        Ut[v] = 0.5 * (S.ub[v * NC + cb] + S.ub[v * NC + cb + (KIND == KIND_X ? 1 : HC)]);
    }
  };
  R Cv[4] = {R(0), R(0), R(0), R(0)};
  if (P.correction) {
    const R U0r[4] = {R(U0[0]), R(U0[1]), R(U0[2]), R(U0[3])};
    corr_half(U0r, Ux, Uy, G.gamma, Cv);
  }
  const double h2 = 0.25 * dt * dt, f2 = dt * dt;

  int e = 0;
  double lin[4];
  if (P.mode == LIN_AF3) {
    R dq[4];
    e = eg2<R, KIND>(S, cb, U0, R(0.25 * dt), R(4.0 * idt), G, dq);
    if (e) { set_err(dev, e); return; }
    double q[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = U0[v] + (double)dq[v];
    if (admissible(q[0], q[3])) {
#pragma unroll
      for (int v = 0; v < 4; ++v) lin[v] = q[v];
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) lin[v] = U0[v];
      if (!FIX) atomicAdd(&dev->cnt[AF_CNT_INNER], 1ull);
    }
  } else if (P.mode == LIN_AVG && !on_wall<KIND>(P, gi, gj)) {
    avg_lin(lin);
  } else {  // simplified method; and the averaged linearisation on a wall line (Sec. 4.3)
#pragma unroll
    for (int v = 0; v < 4; ++v) lin[v] = U0[v];
  }

  // indicators of this DOF (Sec. 3.4 theta; Algorithm 2 flag)
  double theta = 1.0;
  bool tsw = false;
  if constexpr (IND) {
    if (P.shock) {
      if constexpr (KIND == KIND_K)
        theta = mn(mn(I->thx[thx_idx(a, b)], I->thx[thx_idx(a, b - 1)]),
                   mn(I->thy[thy_idx(a, b)], I->thy[thy_idx(a - 1, b)]));
      else if constexpr (KIND == KIND_X)
        theta = I->thx[thx_idx(a, b)];
      else
        theta = I->thy[thy_idx(a, b)];
    }
    if (P.tsw) {
      if constexpr (KIND == KIND_K)
        tsw = I->flag[flag_idx(a, b)] != 0;
      else if constexpr (KIND == KIND_X)
        tsw = (I->flag[flag_idx(a, b)] | I->flag[flag_idx(a, b + 1)]) != 0;
      else
        tsw = (I->flag[flag_idx(a, b)] | I->flag[flag_idx(a + 1, b)]) != 0;
    }
  }

  double Uh[4], U1[4];
  {
    R d[4];
    e = eg2<R, KIND>(S, cb, lin, R(0.5 * dt), R(2.0 * idt), G, d);
    if (e) { set_err(dev, e); return; }
#pragma unroll
    for (int v = 0; v < 4; ++v) Uh[v] = lin[v] + (double)d[v] + h2 * (double)Cv[v];
  }
  // Sec. 3.4 blend of the intermediate value (U_lo is kept for the new time level)
  double lo[4], Ut[4];
  int lo_state = 1;  // 0: lo valid, 1: no blend
  if (IND && theta < 1.0) {
    avg_lin(Ut);
    lo_state = shock_low<R, KIND>(S, G, cb, Ut, 0.5 * dt, lo);
    if (lo_state == ERR_CFL) { set_err(dev, ERR_CFL); return; }
    if (lo_state == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) Uh[v] = theta * Uh[v] + (1.0 - theta) * lo[v];
    }
  }
  // positivity of the intermediate value (Algorithm 3)
  if (!admissible(Uh[0], Uh[3])) {
    if (!P.limiter) { set_err(dev, ERR_NONPHYS); return; }
    if constexpr (!FIX) {
      mark_fix(B, tile, KIND, threadIdx.x & 63);
      return;
    } else {
      double Ut[4];
      avg_lin(Ut);
      e = limit_value<R, KIND>(S, P, G, site, a, b, cb, Ut, 0.5 * dt, Uh, dev);
      if (e) { set_err(dev, e); return; }
    }
  }
  {
    // the new time level is linearised at U^{n+1/2}, or next to a transonic shock at the mean
    // of the adjacent averages (Algorithm 2)
    double lf[4];
    if (IND && tsw) {
      avg_lin(lf);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) lf[v] = Uh[v];
    }
    R d[4];
    e = eg2<R, KIND>(S, cb, lf, R(dt), R(idt), G, d);
    if (e) { set_err(dev, e); return; }
#pragma unroll
    for (int v = 0; v < 4; ++v) U1[v] = lf[v] + (double)d[v] + f2 * (double)Cv[v];
  }
  if (IND && lo_state == 0) {
    if (eg1_cfl_fails<R>(G, Ut, dt)) { set_err(dev, ERR_CFL); return; }
#pragma unroll
    for (int v = 0; v < 4; ++v) U1[v] = theta * U1[v] + (1.0 - theta) * lo[v];
  }
  if (P.limiter && !admissible(U1[0], U1[3])) {
    if constexpr (!FIX) {
      mark_fix(B, tile, KIND, threadIdx.x & 63);
      return;
    } else {
      double Ut[4];
      avg_lin(Ut);
      e = limit_value<R, KIND>(S, P, G, site, a, b, cb, Ut, dt, U1, dev);
      if (e) { set_err(dev, e); return; }
    }
  }

  // outputs: new point value, Simpson-in-time flux sums (weights 1, 4, 1 at t_n, t_n+1/2,
  // t_n+1), wave speed
  if (IND && tsw) atomicAdd(&dev->cnt[AF_CNT_TSW], 1ull);
  double* out = (KIND == KIND_K) ? B.K_out : (KIND == KIND_X ? B.X_out : B.Y_out);
  const long long o = (long long)gj * P.pP + gi;
#pragma unroll
  for (int v = 0; v < 4; ++v) out[v * P.sP + o] = U1[v];
  const double g1inv = P.g1inv;
  double Fs[4], Gs[4];
  {
#pragma clang fp contract(off)
    double F0[4], G0[4], F[4], Gq[4];
    flux_fg(U0, g1inv, F0, G0);
    flux_fg(Uh, g1inv, F, Gq);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Fs[v] = __builtin_fma(4.0, F[v], F0[v]);
      Gs[v] = __builtin_fma(4.0, Gq[v], G0[v]);
    }
    flux_fg(U1, g1inv, F, Gq);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Fs[v] += F[v];
      Gs[v] += Gq[v];
    }
  }
  const long long of = (long long)gj * P.pF + gi;
  if constexpr (KIND == KIND_K) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      B.FK[v * P.sF + of] = Fs[v];
      B.FK[(4 + v) * P.sF + of] = Gs[v];
    }
  } else if constexpr (KIND == KIND_X) {
#pragma unroll
    for (int v = 0; v < 4; ++v) B.FX[v * P.sF + of] = Fs[v];
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) B.FY[v * P.sF + of] = Gs[v];
  }
  if (admissible(U1[0], U1[3])) speed = mx(speed, wave_speed(U1, P.gamma));
}

// Step control of the point kernel: thread 0 decides and broadcasts through LDS, so that the
// decision is uniform over the block even if another block flags an error meanwhile.  One
// block per grid (`leader`) records dt and the run flags for the later kernels of the step.
// Returns false if the step does not run.
__device__ __forceinline__ bool step_dt(const Params& P, DevState* dev, double dt_host, int slot,
                                        bool leader, double* dt_out) {
  __shared__ double s_dt;
  __shared__ int s_run;
  if (threadIdx.x == 0) {
    int run = 1, last = 0;
    double dt = dt_host;
    if (dev->err) {
      run = 0;
    } else if (dev->steps >= dev->steps_limit) {
      run = 0;
      if (leader) dev->active = 0;
    } else if (!(dt_host > 0.0)) {
      const double t = dev->t, te = dev->t_end;
      const double smax = __longlong_as_double((long long)dev->smax[slot]);
      if (!(t < te)) {
        run = 0;
        if (leader) dev->active = 0;
      } else if (!(smax > 0.0) || !(smax < 1e300)) {
        run = 0;
        set_err(dev, ERR_NONPHYS);
      } else {
        dt = dev->cfl * P.hmin / smax;
        if (t + dt >= te) { dt = te - t; last = 1; }
      }
    }
    if (run && leader) {
      dev->dt = dt;
      dev->active = 1;
      dev->last = last;
    }
    s_dt = dt;
    s_run = run;
  }
  __syncthreads();
  *dt_out = s_dt;
  return s_run != 0;
}

// t_n point value of kind `kind` (0 K, 1 X, 2 Y) at the possibly ghost site (gi, gj), through
// the boundary rules.
__device__ __forceinline__ void fetch_site(const Params& P, const Bufs& B, int kind, int gi,
                                           int gj, double W[4]) {
  int si, sj, sx, sy;
  const double* src;
  if (kind == 0) {
    si = map_axis<true>(gi, P.nx, P.per_x, P.bc[0], P.bc[1], sx);
    sj = map_axis<true>(gj, P.ny, P.per_y, P.bc[2], P.bc[3], sy);
    src = B.K_in;
  } else if (kind == 1) {
    si = map_axis<true>(gi, P.nx, P.per_x, P.bc[0], P.bc[1], sx);
    sj = map_axis<false>(gj, P.ny, P.per_y, P.bc[2], P.bc[3], sy);
    src = B.X_in;
  } else {
    si = map_axis<false>(gi, P.nx, P.per_x, P.bc[0], P.bc[1], sx);
    sj = map_axis<true>(gj, P.ny, P.per_y, P.bc[2], P.bc[3], sy);
    src = B.Y_in;
  }
  const long long o = (long long)sj * P.pP + si;
#pragma unroll
  for (int v = 0; v < 4; ++v) W[v] = src[v * P.sP + o];
  if (sx >= 0 || sy >= 0) apply_sides(P, sx, sy, W);  // a ghost site
}

// Primitive Simpson average of the (possibly ghost, up to two layers) cell (i, j), with the
// cell preparation's rules and arithmetic: inverse Simpson for the centre value (deviation
// form, falling back to C2P of the average), inflow ghosts centred at the inflow state, wall
// ghosts the reflection of the cell they face.
__device__ __forceinline__ void prim_average(const Params& P, const Bufs& B, int i, int j,
                                             double ub[4]) {
  int sx, sy;
  const int gi = map_axis<false>(i, P.nx, P.per_x, P.bc[0], P.bc[1], sx);
  const int gj = map_axis<false>(j, P.ny, P.per_y, P.bc[2], P.bc[3], sy);
  const bool inflow = inflow_side(P, 0, sx) || inflow_side(P, 1, sy);
  const bool fx = !inflow && sx >= 0 && side_kind(P, sx) == BC_WALL;
  const bool fy = !inflow && sy >= 0 && side_kind(P, 2 + sy) == BC_WALL;
  const int ci = fx ? gi : i, cj = fy ? gj : j;
  const double g1inv = P.g1inv, gm1 = P.gamma - 1.0;
  double w[8][4];
  fetch_site(P, B, 0, ci, cj, w[0]);
  fetch_site(P, B, 0, ci + 1, cj, w[1]);
  fetch_site(P, B, 0, ci, cj + 1, w[2]);
  fetch_site(P, B, 0, ci + 1, cj + 1, w[3]);
  fetch_site(P, B, 1, ci, cj, w[4]);
  fetch_site(P, B, 1, ci + 1, cj, w[5]);
  fetch_site(P, B, 2, ci, cj, w[6]);
  fetch_site(P, B, 2, ci, cj + 1, w[7]);
  double Uc[4];
  if (inflow) {
#pragma unroll
    for (int v = 0; v < 4; ++v) Uc[v] = 0.0;
    apply_sides(P, sx, sy, Uc);
  } else {
    double Qb[4];
    const long long oa = (long long)gj * P.pA + gi;
#pragma unroll
    for (int v = 0; v < 4; ++v) Qb[v] = B.A_in[v * P.sA + oa];
    double Wr[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
      Wr[v] = (((w[0][v] + w[1][v]) + (w[2][v] + w[3][v])) +
               ((w[4][v] + w[5][v]) + (w[6][v] + w[7][v]))) * 0.125;
    double dQ[4];
    {
      double sK[4] = {0, 0, 0, 0}, sE[4] = {0, 0, 0, 0}, Q[4];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        p2c(w[k], g1inv, Q);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (k < 4) sK[v] += Qb[v] - Q[v];
          else sE[v] += Qb[v] - Q[v];
        }
      }
      p2c(Wr, g1inv, Q);
#pragma unroll
      for (int v = 0; v < 4; ++v) dQ[v] = (Qb[v] - Q[v]) + (sK[v] + 4.0 * sE[v]) * 0.0625;
    }
    c2p_dev(Wr, dQ, gm1, Uc);
    if (!admissible(Uc[0], Uc[3])) c2p_plain(Qb, gm1, Uc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double u = Uc[v];
    const double sK4 = ((w[0][v] - u) + (w[1][v] - u)) + ((w[2][v] - u) + (w[3][v] - u));
    const double sE4 = ((w[4][v] - u) + (w[5][v] - u)) + ((w[6][v] - u) + (w[7][v] - u));
    const double sv = ((fx && v == 1) || (fy && v == 2)) ? -1.0 : 1.0;
    ub[v] = sv * (u + (sK4 + 4.0 * sE4) * (1.0 / 36.0));
  }
}

// Primitive average of ring cell (a, b), -2 <= a, b <= TILE, component v.
template <class R>
__device__ __forceinline__ double ring_at(const Smem<R>& S, const Ind& I, int v, int a, int b) {
  const bool halo = a >= -1 && a < TILE && b >= -1 && b < TILE;
  const double* p = halo ? S.ub + (v * NC + cidx(a, b)) : I.outer + (v * NO + oidx(a, b));
  return *p;
}

// Algorithm 2: across the ring cells L = (al, bl) -> R = (ar, br) in the direction of velocity
// component comp (1: x, 2: y), w + c or w - c goes from positive to negative.
template <class R>
__device__ __forceinline__ bool transonic_pair(const Smem<R>& S, const Ind& I, int al, int bl,
                                               int ar, int br, int comp, double gamma) {
  const double cl = sqrt(gamma * ring_at(S, I, 3, al, bl) / ring_at(S, I, 0, al, bl));
  const double cr = sqrt(gamma * ring_at(S, I, 3, ar, br) / ring_at(S, I, 0, ar, br));
  const double wl = ring_at(S, I, comp, al, bl), wr = ring_at(S, I, comp, ar, br);
  return (wl + cl > 0.0 && wr + cr < 0.0) || (wl - cl > 0.0 && wr - cr < 0.0);
}

// Sec. 3.4: theta of the edge midpoint between ring cells 1 and 2 of the line of ring cells
// (a0, b0) + m (da, db), m = 0..3, velocity component comp along the line.
template <class R>
__device__ __forceinline__ double theta_edge(const Smem<R>& S, const Ind& I, int a0, int b0,
                                             int da, int db, int comp, double gamma) {
  double p[4], rho[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    rho[m] = ring_at(S, I, 0, a0 + m * da, b0 + m * db);
    p[m] = ring_at(S, I, 3, a0 + m * da, b0 + m * db);
    if (!admissible(rho[m], p[m])) return 0.0;
  }
  double a[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int k = 2 - m;  // cell k, then k-1
    a[m] = fabs(ring_at(S, I, comp, a0 + k * da, b0 + k * db)) + sqrt(gamma * p[k] / rho[k]);
  }
  const double s_hi = fabs((p[3] - 2.0 * p[2] + p[1]) / (p[3] + 2.0 * p[2] + p[1]));
  const double s_lo = fabs((p[2] - 2.0 * p[1] + p[0]) / (p[2] + 2.0 * p[1] + p[0]));
  const double phi1 = s_hi > s_lo ? s_hi : s_lo;
  const double phi2 = exp2(a[0] > a[1] ? a[0] : a[1]);
  return exp(-phi1 * phi2);
}

// Stage the primitive averages of the ring of cells -2 .. TILE around a tile (from the padded
// array written by the averaging pass; they replace the prep's own, so that one set of averages
// serves the linearisations and the indicators), then theta of the tile's edge midpoints and the
// transonic flags of its corners.  Ends with a barrier.
template <class R>
__device__ __forceinline__ void stage_indicators(Smem<R>& S, Ind& I, const Params& P,
                                                 const Bufs& B, int tile) {
  const int i0 = (tile % P.tiles_x) * TILE, j0 = (tile / P.tiles_x) * TILE;
  const int tid = threadIdx.x;
  for (int c = tid; c < NR; c += PT_THREADS) {
    const int a = c % RC - 2, b = c / RC - 2;
    // cells beyond the padded range are never read by a DOF of the grid
    const int gi = min(i0 + a, P.nx + 1), gj = min(j0 + b, P.ny + 1);
    const long long o = (long long)(gj + 2) * P.pU + (gi + 2);
    const bool halo = a >= -1 && a < TILE && b >= -1 && b < TILE;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double u = B.UB[v * P.sU + o];
      if (halo)
        S.ub[v * NC + cidx(a, b)] = u;
      else
        I.outer[v * NO + oidx(a, b)] = u;
    }
  }
  __syncthreads();
  const double g = P.gamma;
  for (int e = tid; e < (TILE + 1) * (TILE + 1) + 2 * TILE * (TILE + 1); e += PT_THREADS) {
    if (e < (TILE + 1) * (TILE + 1)) {
      // corner (a, b): cells (a-1 .. a) x (b-1 .. b)
      const int a = e % (TILE + 1), b = e / (TILE + 1);
      bool f = false;
      if (P.tsw)
        f = transonic_pair(S, I, a - 1, b, a, b, 1, g) ||
            transonic_pair(S, I, a - 1, b - 1, a, b - 1, 1, g) ||
            transonic_pair(S, I, a - 1, b - 1, a - 1, b, 2, g) ||
            transonic_pair(S, I, a, b - 1, a, b, 2, g);
      I.flag[flag_idx(a, b)] = f ? 1 : 0;
    } else if (e < (TILE + 1) * (TILE + 1) + TILE * (TILE + 1)) {
      // x-edge (a, b), a in 0..TILE-1, b in -1..TILE-1: cells a-2 .. a+1 of row b
      const int q = e - (TILE + 1) * (TILE + 1);
      const int a = q % TILE, b = q / TILE - 1;
      I.thx[thx_idx(a, b)] = P.shock ? theta_edge(S, I, a - 2, b, 1, 0, 1, g) : 1.0;
    } else {
      // y-edge (a, b), a in -1..TILE-1, b in 0..TILE-1: cells b-2 .. b+1 of column a
      const int q = e - (TILE + 1) * (TILE + 1) - TILE * (TILE + 1);
      const int a = q % (TILE + 1) - 1, b = q / (TILE + 1);
      I.thy[thy_idx(a, b)] = P.shock ? theta_edge(S, I, a, b - 2, 0, 1, 2, g) : 1.0;
    }
  }
  __syncthreads();
}

// Reconstruction of the halo cell c of the tile with corner (i0, j0): centre value, primitive
// Simpson average and monomial coefficients into LDS.  GHOST: the cell or its nodes may lie
// beyond the grid (boundary rules apply); otherwise every index is a plain interior one.
template <class R, bool GHOST>
__device__ __forceinline__ void prep_cell(Smem<R>& S, const Params& P, const Bufs& B,
                                          DevState* dev, int i0, int j0, int c, bool count) {
  const int a = c % HC - 1, b = c / HC - 1;
  int sx = -1, sy = -1, gi = i0 + a, gj = j0 + b;
  if constexpr (GHOST) {
    gi = map_axis<false>(i0 + a, P.nx, P.per_x, P.bc[0], P.bc[1], sx);
    gj = map_axis<false>(j0 + b, P.ny, P.per_y, P.bc[2], P.bc[3], sy);
  }
  // A ghost cell beyond an inflow side holds the inflow state (centre value below).  A ghost
  // cell beyond a solid wall is the mirror image of the cell (gi, gj) it faces: that cell's
  // reconstruction is built from its own nodes and average, then reflected (fx, fy).  Halo
  // cells more than one layer beyond the grid are never read; their node cell is only kept
  // inside the halo.
  const bool inflow = inflow_side(P, 0, sx) || inflow_side(P, 1, sy);
  const bool fx = !inflow && sx >= 0 && side_kind(P, sx) == BC_WALL;
  const bool fy = !inflow && sy >= 0 && side_kind(P, 2 + sy) == BC_WALL;
  const int an = fx ? min(max(gi - i0, -1), TILE - 1) : a;
  const int bn = fy ? min(max(gj - j0, -1), TILE - 1) : b;
  const double g1inv = P.g1inv, gm1 = P.gamma - 1.0;
  // node k of the cell: 0..3 corners K(a,b) K(a+1,b) K(a,b+1) K(a+1,b+1),
  // 4,5 X(a,b) X(a+1,b), 6,7 Y(a,b) Y(a,b+1)
  const double* nptr[8] = {S.sk + sidx(an, bn), S.sk + sidx(an + 1, bn),
                           S.sk + sidx(an, bn + 1), S.sk + sidx(an + 1, bn + 1),
                           S.sx + sidx(an, bn), S.sx + sidx(an + 1, bn),
                           S.sy + sidx(an, bn), S.sy + sidx(an, bn + 1)};
  auto node = [&](int k, double W[4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) W[v] = (double)nptr[k][v * NS];
  };
  double Qb[4];
  const long long oa = (long long)gj * P.pA + gi;
#pragma unroll
  for (int v = 0; v < 4; ++v) Qb[v] = B.A_in[v * P.sA + oa];
  // inverse Simpson for the centre value: Q_c = Q-bar + [sum_K (Q-bar - Q_k)
  //                                          + 4 sum_E (Q-bar - Q_e)] / 16,
  // converted to primitive variables by deviation from the lower-left corner node Wr (so that
  // equal nodes give the centre value Wr exactly)
  double dQ[4], Uc[4], Wr[4];
  {
    double sK[4] = {0, 0, 0, 0}, sE[4] = {0, 0, 0, 0}, W[4], Q[4], Qr[4];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      node(k, W);
      p2c(W, g1inv, Q);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (k == 0) { Wr[v] = W[v]; Qr[v] = Q[v]; }
        if (k < 4) sK[v] += Qb[v] - Q[v];
        else sE[v] += Qb[v] - Q[v];
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) dQ[v] = (Qb[v] - Qr[v]) + (sK[v] + 4.0 * sE[v]) * 0.0625;
  }
  c2p_dev(Wr, dQ, gm1, Uc);
  if (inflow) {
    // every point value of the ghost cell, the centre included, is the inflow state
#pragma unroll
    for (int v = 0; v < 4; ++v) Uc[v] = 0.0;
    apply_sides(P, sx, sy, Uc);
  } else if (!admissible(Uc[0], Uc[3])) {
    c2p_plain(Qb, gm1, Uc);
    const bool owned = a >= 0 && b >= 0 && (i0 + a) < P.nx && (j0 + b) < P.ny;
    if (owned && count) atomicAdd(&dev->cnt[AF_CNT_CENTRE], 1ull);
  }
  const double rho = P.aspect, rho2 = rho * rho;
  // primitive Simpson average and monomial coefficients, variable by variable
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = (double)nptr[k][v * NS];
    const double u = Uc[v];
    const double sK4 = ((w[0] - u) + (w[1] - u)) + ((w[2] - u) + (w[3] - u));
    const double sE4 = ((w[4] - u) + (w[5] - u)) + ((w[6] - u) + (w[7] - u));
    // reflection of a wall ghost: the normal velocity negated, and in the monomial
    // coefficients c_mn (of xi^m eta^n, k = 3m + n) the odd powers of the normal coordinate
    const double sv = ((fx && v == 1) || (fy && v == 2)) ? -1.0 : 1.0;
    S.ub[v * NC + c] = sv * (u + (sK4 + 4.0 * sE4) * (1.0 / 36.0));
    const double N[3][3] = {{w[0], w[4], w[2]}, {w[6], u, w[7]}, {w[1], w[5], w[3]}};
    double cm[9];
    nodes_to_monomials(N, cm);
    S.c0[v * NC + c] = sv * cm[0];
    // c_mn of xi^m eta^n -> coefficient of xi^m (eta dy/dx)^n: the circle integrals use
    // dx as the unit length in both directions
#pragma unroll
    for (int k = 1; k < 9; ++k) {
      const double sk = sv * ((fx && ((k / 3) & 1)) ? -1.0 : 1.0) *
                        ((fy && ((k % 3) & 1)) ? -1.0 : 1.0);
      S.ch[c * CS + v * 8 + k - 1] =
          (R)(sk * (k % 3 == 0 ? cm[k] : (k % 3 == 1 ? cm[k] * rho : cm[k] * rho2)));
    }
  }
}

// Stage the t_n point values of a tile's halo in LDS and build the halo cells'
// reconstructions.  Ends with a barrier.
template <class R>
__device__ __forceinline__ void stage_and_prep(Smem<R>& S, const Params& P, const Bufs& B,
                                               DevState* dev, int tile, bool count) {
  const int i0 = (tile % P.tiles_x) * TILE, j0 = (tile / P.tiles_x) * TILE;
  const int tid = threadIdx.x;
  // a tile whose halo (sites i0-1 .. i0+TILE, cells i0-1 .. i0+TILE-1, likewise in y) lies
  // inside the grid needs no boundary rule: the same for the whole block
  const bool inner = i0 >= 1 && j0 >= 1 && i0 + TILE <= P.nx - 1 && j0 + TILE <= P.ny - 1;
  // 1. stage the t_n point values of the halo (local sites -1 .. TILE) in LDS: one site per
  // thread, its K, X and Y values together (one index computation, twelve loads from the three
  // arrays at one offset)
  static_assert(NS <= PT_THREADS, "one halo site per thread");
  if (tid < NS) {
    const int a = tid % HS - 1, b = tid / HS - 1;
    double W[3][4];
    if (inner) {
      const long long o = (long long)(j0 + b) * P.pP + (i0 + a);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        W[0][v] = B.K_in[v * P.sP + o];
        W[1][v] = B.X_in[v * P.sP + o];
        W[2][v] = B.Y_in[v * P.sP + o];
      }
    } else {
#pragma unroll
      for (int kind = 0; kind < 3; ++kind) fetch_site(P, B, kind, i0 + a, j0 + b, W[kind]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      S.sk[v * NS + tid] = W[0][v];
      S.sx[v * NS + tid] = W[1][v];
      S.sy[v * NS + tid] = W[2][v];
    }
  }
  __syncthreads();

  // 2. cell reconstructions of the halo cells (local cells -1 .. TILE-1)
  for (int c = tid; c < NC; c += PT_THREADS) {
    if (inner)
      prep_cell<R, false>(S, P, B, dev, i0, j0, c, count);
    else
      prep_cell<R, true>(S, P, B, dev, i0, j0, c, count);
  }
  __syncthreads();
}

// Evolve the tile's own DOFs: wavefront 0 -> K; wavefront 1 -> X, then Y (an edge EG2 costs
// about 40 % of a corner EG2, so the two waves' loads are within about a fifth of each other).
// In the fix-up pass only the lanes listed in `mask` (per kind) run.
template <class R, bool FIX, bool IND>
__device__ __forceinline__ void evolve_tile(Smem<R>& S, const Ind* I, const Params& P,
                                            const Bufs& B, DevState* dev, int tile, double dt,
                                            const unsigned long long* mask, double& speed) {
  const int i0 = (tile % P.tiles_x) * TILE, j0 = (tile / P.tiles_x) * TILE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int a = lane % TILE, b = lane / TILE;
  const int gi = i0 + a, gj = j0 + b;
  auto listed = [&](int kind) { return !FIX || ((mask[kind] >> lane) & 1ull); };
  if (wave == 0) {
    if (listed(KIND_K) && gi < P.nkx && gj < P.nky)
      evolve_dof<R, KIND_K, FIX, IND>(S, I, P, B, dev, tile, a, b, gi, gj, dt, speed);
  } else {
    if (listed(KIND_X) && gi < P.nkx && gj < P.ny)
      evolve_dof<R, KIND_X, FIX, IND>(S, I, P, B, dev, tile, a, b, gi, gj, dt, speed);
    if (listed(KIND_Y) && gi < P.nx && gj < P.nky)
      evolve_dof<R, KIND_Y, FIX, IND>(S, I, P, B, dev, tile, a, b, gi, gj, dt, speed);
  }
}

// Workgroups are dealt to the eight XCDs in turn (block b to XCD b mod 8), and each XCD has its
// own L2.  Giving XCD x the contiguous tile range [x * ntiles/8, (x+1) * ntiles/8), in row
// order, keeps the halos that neighbouring tiles share in one L2.  A bijection on the tile
// indices (the last ntiles mod 8 tiles map to themselves).
__device__ __forceinline__ int tile_of_block(int b, int ntiles) {
  const int per = ntiles >> 3;
  if (b >= (per << 3)) return b;
  return (b & 7) * per + (b >> 3);
}

// One tile of the point kernel.  `slot` is the buffer index of the t_n state (its wave-speed
// maximum is smax[slot]; the new state's goes to smax[slot ^ 1]).
template <class R, bool IND = false>
__device__ __forceinline__ void points_body(Smem<R>& S, Ind* I, const Params& P, const Bufs& B,
                                            DevState* dev, double dt_host, int slot, int tile,
                                            bool leader) {
  double dt;
  if (!step_dt(P, dev, dt_host, slot, leader, &dt)) return;
  stage_and_prep(S, P, B, dev, tile, true);
  if constexpr (IND) stage_indicators(S, *I, P, B, tile);
  double speed = 0.0;
  evolve_tile<R, false, IND>(S, I, P, B, dev, tile, dt, nullptr, speed);
  block_max_atomic(speed, &dev->smax[slot ^ 1], S.red);
}

// Positivity fix-up of one listed tile: stage and prepare it again and recompute only the
// lanes flagged in its masks with Algorithm 3; then clear the masks.  Block-uniform `run`.
template <class R, bool IND = false>
__device__ __forceinline__ void fixup_tile(Smem<R>& S, Ind* I, const Params& P, const Bufs& B,
                                           DevState* dev, int tile, double dt, bool run,
                                           unsigned long long* mask, double& speed) {
  if (threadIdx.x < 3) mask[threadIdx.x] = B.fix_mask[4 * (long long)tile + threadIdx.x];
  __syncthreads();
  if (run) {
    stage_and_prep(S, P, B, dev, tile, false);
    if constexpr (IND) stage_indicators(S, *I, P, B, tile);
    evolve_tile<R, true, IND>(S, I, P, B, dev, tile, dt, mask, speed);
  }
  __syncthreads();
  if (threadIdx.x < 4) B.fix_mask[4 * (long long)tile + threadIdx.x] = 0ull;
}

// Conservative update (eqs. F and 2dfvm) of the two cells (i, j) and (i + 1, j), i even (the
// second only if i + 1 < nx): per cell the four Simpson face fluxes from the per-site
// Simpson-in-time sums, F = (f_K + 4 f_X + f_K') sums, then the FP64 update with
// lx = dt / (36 dx), ly = dt / (36 dy).  The east face of the first cell is the west face of
// the second, and site pairs (i, i + 1) are read with 16-byte loads (rows are aligned to 32
// doubles or more).  Returns false if a new average is not admissible; else raises `speed` to
// the new averages' wave speeds.
__device__ __forceinline__ bool update_pair(const Params& P, const double* __restrict__ A_in,
                                            double* __restrict__ A_out,
                                            const double* __restrict__ FK,
                                            const double* __restrict__ FX,
                                            const double* __restrict__ FY, double lx, double ly,
                                            int i, int j, double& speed) {
  const bool two = i + 1 < P.nx;
  const int jp = wrap_line(j + 1, P.ny, P.per_y);
  const int s1 = wrap_line(i + 1, P.nx, P.per_x);
  const int s2 = two ? wrap_line(i + 2, P.nx, P.per_x) : s1;
  const long long r0 = (long long)j * P.pF, r1 = (long long)jp * P.pF;
  const long long ra = (long long)j * P.pA;
  double Q0[4], Q1[4];
  if (two && s1 == i + 1) {
    // sites i, i + 1 adjacent in memory: 16-byte loads of the pairs
    auto ld = [](const double* a, long long o) {
      return *reinterpret_cast<const double2*>(a + o);
    };
    // every load first, then the arithmetic
    double2 f0[4], f1[4], g0[4], g1[4], x[4], y0[4], y1[4], a[4];
    double f20[4], f21[4], g20[4], x2[4], g21[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double* fk = FK + v * P.sF;
      const double* gk = FK + (4 + v) * P.sF;
      const double* fx = FX + v * P.sF;
      const double* fy = FY + v * P.sF;
      f0[v] = ld(fk, r0 + i); f1[v] = ld(fk, r1 + i);
      g0[v] = ld(gk, r0 + i); g1[v] = ld(gk, r1 + i);
      x[v] = ld(fx, r0 + i); y0[v] = ld(fy, r0 + i); y1[v] = ld(fy, r1 + i);
      a[v] = ld(A_in + v * P.sA, ra + i);
      f20[v] = fk[r0 + s2]; f21[v] = fk[r1 + s2]; g20[v] = gk[r0 + s2]; x2[v] = fx[r0 + s2];
      g21[v] = gk[r1 + s2];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double Fw = f0[v].x + 4.0 * x[v].x + f1[v].x;
      const double Fe = f0[v].y + 4.0 * x[v].y + f1[v].y;
      const double Gs = g0[v].x + 4.0 * y0[v].x + g0[v].y;
      const double Gn = g1[v].x + 4.0 * y1[v].x + g1[v].y;
      Q0[v] = a[v].x - lx * (Fe - Fw) - ly * (Gn - Gs);
      const double Fe1 = f20[v] + 4.0 * x2[v] + f21[v];
      const double Gs1 = g0[v].y + 4.0 * y0[v].y + g20[v];
      const double Gn1 = g1[v].y + 4.0 * y1[v].y + g21[v];
      Q1[v] = a[v].y - lx * (Fe1 - Fe) - ly * (Gn1 - Gs1);
      *reinterpret_cast<double2*>(A_out + v * P.sA + ra + i) = make_double2(Q0[v], Q1[v]);
    }
  } else {
    // the last cell of a row (one cell, or a periodic wrap between the two sites)
#pragma unroll 1
    for (int v = 0; v < 4; ++v) {
      const double* fk = FK + v * P.sF;
      const double* gk = FK + (4 + v) * P.sF;
      const double* fx = FX + v * P.sF;
      const double* fy = FY + v * P.sF;
      const double Fw = fk[r0 + i] + 4.0 * fx[r0 + i] + fk[r1 + i];
      const double Fe = fk[r0 + s1] + 4.0 * fx[r0 + s1] + fk[r1 + s1];
      const double Gs = gk[r0 + i] + 4.0 * fy[r0 + i] + gk[r0 + s1];
      const double Gn = gk[r1 + i] + 4.0 * fy[r1 + i] + gk[r1 + s1];
      Q0[v] = A_in[v * P.sA + ra + i] - lx * (Fe - Fw) - ly * (Gn - Gs);
      A_out[v * P.sA + ra + i] = Q0[v];
      if (two) {
        const double Fe1 = fk[r0 + s2] + 4.0 * fx[r0 + s2] + fk[r1 + s2];
        const double Gs1 = gk[r0 + s1] + 4.0 * fy[r0 + i + 1] + gk[r0 + s2];
        const double Gn1 = gk[r1 + s1] + 4.0 * fy[r1 + i + 1] + gk[r1 + s2];
        Q1[v] = A_in[v * P.sA + ra + i + 1] - lx * (Fe1 - Fe) - ly * (Gn1 - Gs1);
        A_out[v * P.sA + ra + i + 1] = Q1[v];
      }
    }
  }
  bool ok = true;
  double U[4];
  if (two) {
    c2p_plain(Q1, P.gamma - 1.0, U);
    if (!admissible(U[0], U[3])) ok = false;
    else speed = mx(speed, wave_speed(U, P.gamma));
  }
  c2p_plain(Q0, P.gamma - 1.0, U);
  if (!admissible(U[0], U[3])) return false;
  speed = mx(speed, wave_speed(U, P.gamma));
  return ok;
}

// Largest wave speed over the DOFs e0, e0 + stride, ... of a state (averages, then K, X, Y in
// storage order), for the time step before a run.  Non-admissible values do not enter.
__device__ __forceinline__ double state_speed(const Params& P, const double* __restrict__ A,
                                              const double* __restrict__ K,
                                              const double* __restrict__ X,
                                              const double* __restrict__ Y, long long e0,
                                              long long stride) {
  const long long n0 = (long long)P.nx * P.ny, n1 = (long long)P.nkx * P.nky,
                  n2 = (long long)P.nkx * P.ny, n3 = (long long)P.nx * P.nky;
  const long long ntot = n0 + n1 + n2 + n3;
  double speed = 0.0;
  for (long long e = e0; e < ntot; e += stride) {
    double U[4];
    if (e < n0) {
      const int i = (int)(e % P.nx), j = (int)(e / P.nx);
      double Q[4];
      for (int v = 0; v < 4; ++v) Q[v] = A[v * P.sA + (long long)j * P.pA + i];
      c2p_plain(Q, P.gamma - 1.0, U);
    } else {
      long long r = e - n0;
      const double* src;
      int w;
      if (r < n1) { src = K; w = P.nkx; }
      else if (r < n1 + n2) { src = X; w = P.nkx; r -= n1; }
      else { src = Y; w = P.nx; r -= n1 + n2; }
      const int i = (int)(r % w), j = (int)(r / w);
      for (int v = 0; v < 4; ++v) U[v] = src[v * P.sP + (long long)j * P.pP + i];
    }
    if (admissible(U[0], U[3])) speed = mx(speed, wave_speed(U, P.gamma));
  }
  return speed;
}

}  // namespace af

namespace af {

// ------------------------------------------------------------------------------------------
// Flux limiting of the cell averages (Sec. 3.5).  Each face flux becomes
// gamma F_ho + (1 - gamma) F_lo with F_lo the Rusanov flux of the t_n averages of the two
// cells; gamma is the smaller over the face's two cells of the largest theta in [0, 1] that
// keeps the cell's share Q_lo - 4 lambda s theta (F_ho - F_lo) of the new average above the
// density and pressure floors min(1e-13, those of Q_lo), Q_lo being the cell's low-order
// update (positivity-preserving limiting after Hu, Adams and Shu on Zhang and Shu).  The new
// average is the mean of the four shares, hence admissible.
// ------------------------------------------------------------------------------------------
// t_n average of the possibly ghost cell (i, j), one layer beyond the grid, by the side rules
// (periodic wrap, outflow copy, wall mirror with the normal momentum negated, inflow state).
__device__ __forceinline__ void ghost_avg(const Params& P, const double* __restrict__ A, int i,
                                          int j, double Q[4]) {
  int sx, sy;
  const int gi = map_axis<false>(i, P.nx, P.per_x, P.bc[0], P.bc[1], sx);
  const int gj = map_axis<false>(j, P.ny, P.per_y, P.bc[2], P.bc[3], sy);
  const long long o = (long long)gj * P.pA + gi;
#pragma unroll
  for (int v = 0; v < 4; ++v) Q[v] = A[v * P.sA + o];
  if (sx >= 0 && side_kind(P, sx) == BC_WALL) Q[1] = -Q[1];
  if (sy >= 0 && side_kind(P, 2 + sy) == BC_WALL) Q[2] = -Q[2];
  if (sx >= 0 && side_kind(P, sx) == BC_INFLOW) {
    double W[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) W[v] = side_inflow(P, sx, v);
    p2c(W, P.g1inv, Q);
  }
  if (sy >= 0 && side_kind(P, 2 + sy) == BC_INFLOW) {
    double W[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) W[v] = side_inflow(P, 2 + sy, v);
    p2c(W, P.g1inv, Q);
  }
}

// Rusanov flux between the conserved states QL, QR in direction dir (0: x, 1: y), scaled by
// 36 (the scale of the Simpson site sums the update works with).
__device__ __forceinline__ void rusanov36(const Params& P, const double QL[4], const double QR[4],
                                          int dir, double o[4]) {
  double UL[4], UR[4], FL[4], GL[4], FR[4], GR[4];
  const double gm1 = P.gamma - 1.0;
  c2p_plain(QL, gm1, UL);
  c2p_plain(QR, gm1, UR);
  flux_fg(UL, P.g1inv, FL, GL);
  flux_fg(UR, P.g1inv, FR, GR);
  const double aL = __builtin_fabs(UL[1 + dir]) + __builtin_sqrt(P.gamma * UL[3] / UL[0]);
  const double aR = __builtin_fabs(UR[1 + dir]) + __builtin_sqrt(P.gamma * UR[3] / UR[0]);
  const double al = mx(aL, aR);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double fl = dir ? GL[v] : FL[v], fr = dir ? GR[v] : FR[v];
    o[v] = 36.0 * (0.5 * (fl + fr) - 0.5 * al * (QR[v] - QL[v]));
  }
}

// density >= er and pressure >= ep
__device__ __forceinline__ bool above_floor(const double Q[4], double gm1, double er, double ep) {
  if (!(Q[0] >= er)) return false;
  const double p = gm1 * (Q[3] - 0.5 * (Q[1] * Q[1] + Q[2] * Q[2]) / Q[0]);
  return p >= ep;
}

// Largest theta in [0, 1] with Qlo + theta d above the floors: theta = 1 if that state is,
// else bisection (60 halvings; the admissible theta form an interval containing 0).
__device__ __forceinline__ double flux_theta(const double Qlo[4], const double d[4], double gm1,
                                             double plo) {
  const double er = mn(1e-13, Qlo[0]), ep = mn(1e-13, plo);
  double Q[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) Q[v] = Qlo[v] + d[v];
  if (above_floor(Q, gm1, er, ep)) return 1.0;
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 60; ++it) {
    const double m = 0.5 * (lo + hi);
#pragma unroll
    for (int v = 0; v < 4; ++v) Q[v] = Qlo[v] + m * d[v];
    if (above_floor(Q, gm1, er, ep)) lo = m;
    else hi = m;
  }
  return lo;
}

// Site sums of the four faces of cell (i, j), Simpson in space (F = f_K + 4 f_X + f_K'):
// S[0] west, S[1] east, S[2] south, S[3] north.
__device__ __forceinline__ void face_sums(const Params& P, const double* __restrict__ FK,
                                          const double* __restrict__ FX,
                                          const double* __restrict__ FY, int i, int j,
                                          double S[4][4]) {
  const int jp = wrap_line(j + 1, P.ny, P.per_y);
  const int ip = wrap_line(i + 1, P.nx, P.per_x);
  const long long r0 = (long long)j * P.pF, r1 = (long long)jp * P.pF;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double* fk = FK + v * P.sF;
    const double* gk = FK + (4 + v) * P.sF;
    const double* fx = FX + v * P.sF;
    const double* fy = FY + v * P.sF;
    S[0][v] = fk[r0 + i] + 4.0 * fx[r0 + i] + fk[r1 + i];
    S[1][v] = fk[r0 + ip] + 4.0 * fx[r0 + ip] + fk[r1 + ip];
    S[2][v] = gk[r0 + i] + 4.0 * fy[r0 + i] + gk[r0 + ip];
    S[3][v] = gk[r1 + i] + 4.0 * fy[r1 + i] + gk[r1 + ip];
  }
}

// Rusanov fluxes (x36) of the four faces of cell (i, j), same face order, and its average.
__device__ __forceinline__ void face_low(const Params& P, const double* __restrict__ A, int i,
                                         int j, double Q[4], double L[4][4]) {
  double Qw[4], Qe[4], Qs[4], Qn[4];
  ghost_avg(P, A, i, j, Q);
  ghost_avg(P, A, i - 1, j, Qw);
  ghost_avg(P, A, i + 1, j, Qe);
  ghost_avg(P, A, i, j - 1, Qs);
  ghost_avg(P, A, i, j + 1, Qn);
  rusanov36(P, Qw, Q, 0, L[0]);
  rusanov36(P, Q, Qe, 0, L[1]);
  rusanov36(P, Qs, Q, 1, L[2]);
  rusanov36(P, Q, Qn, 1, L[3]);
}

// theta of the four faces of cell (i, j); false if its low-order update is not admissible.
__device__ __forceinline__ bool cell_thetas(const Params& P, const double* __restrict__ A,
                                            const double* __restrict__ FK,
                                            const double* __restrict__ FX,
                                            const double* __restrict__ FY, double lx, double ly,
                                            int i, int j, double th[4]) {
  double S[4][4], L[4][4], Q[4], Qlo[4], Ulo[4];
  face_sums(P, FK, FX, FY, i, j, S);
  face_low(P, A, i, j, Q, L);
#pragma unroll
  for (int v = 0; v < 4; ++v) Qlo[v] = Q[v] - lx * (L[1][v] - L[0][v]) - ly * (L[3][v] - L[2][v]);
  c2p_plain(Qlo, P.gamma - 1.0, Ulo);
  if (!admissible(Ulo[0], Ulo[3])) return false;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const double sl = (f == 1 || f == 3) ? -4.0 : 4.0;  // -4 s_f
    const double lam = f < 2 ? lx : ly;
    double d[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) d[v] = sl * lam * (S[f][v] - L[f][v]);
    th[f] = flux_theta(Qlo, d, P.gamma - 1.0, Ulo[3]);
  }
  return true;
}

// Limited update of cell (i, j) from the thetas (4 planes of the cell layout).  Counts its west
// and south faces (and east / north at a closed side) in *nlim when limited.  Returns false if
// the new average is not admissible; else raises `speed`.
__device__ __forceinline__ bool update_limited(const Params& P, const double* __restrict__ A_in,
                                               double* __restrict__ A_out,
                                               const double* __restrict__ FK,
                                               const double* __restrict__ FX,
                                               const double* __restrict__ FY,
                                               const double* __restrict__ TH, double lx,
                                               double ly, int i, int j, double& speed,
                                               unsigned& nlim) {
  const long long st = (long long)P.ny * P.pA;  // theta plane stride
  auto th = [&](int f, int ci, int cj) { return TH[f * st + (long long)cj * P.pA + ci]; };
  double S[4][4], g[4];
  face_sums(P, FK, FX, FY, i, j, S);
  bool any = false;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    double t = th(f, i, j);
    const int ni = i + (f == 1) - (f == 0), nj = j + (f == 3) - (f == 2);
    const bool xf = f < 2;
    const int k = xf ? ni : nj, n = xf ? P.nx : P.ny;
    if ((xf ? P.per_x : P.per_y) || (k >= 0 && k < n)) {
      const int wi = wrap_per(ni < 0 ? ni + P.nx : ni, P.nx);
      const int wj = wrap_per(nj < 0 ? nj + P.ny : nj, P.ny);
      t = mn(t, th(f ^ 1, wi, wj));
    }
    g[f] = t;
    if (t < 1.0) {
      any = true;
      if (f == 0 || f == 2 || (f == 1 && !P.per_x && i == P.nx - 1) ||
          (f == 3 && !P.per_y && j == P.ny - 1))
        ++nlim;
    }
  }
  if (any) {
    double L[4][4], Q[4];
    face_low(P, A_in, i, j, Q, L);
#pragma unroll
    for (int f = 0; f < 4; ++f)
      if (g[f] < 1.0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) S[f][v] = g[f] * S[f][v] + (1.0 - g[f]) * L[f][v];
      }
  }
  const long long oa = (long long)j * P.pA + i;
  double Qn[4], U[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    Qn[v] = A_in[v * P.sA + oa] - lx * (S[1][v] - S[0][v]) - ly * (S[3][v] - S[2][v]);
    A_out[v * P.sA + oa] = Qn[v];
  }
  c2p_plain(Qn, P.gamma - 1.0, U);
  if (!admissible(U[0], U[3])) return false;
  speed = mx(speed, wave_speed(U, P.gamma));
  return true;
}

}  // namespace af
