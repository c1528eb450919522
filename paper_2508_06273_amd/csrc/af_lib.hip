// af_lib.hip -- kernels and host runtime of libaf.so (C ABI in include/af.h).
//
// Fully discrete third-order Active Flux method for the 2D Euler equations, arXiv 2508.06273.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "af.h"
#include "af_kernels.hpp"

namespace af {

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
__device__ __forceinline__ void mark_fix(const Bufs& B, DevState* dev, int tile, int kind,
                                         int lane) {
  atomicOr(&B.fix_mask[4 * (long long)tile + kind], 1ull << lane);
  if (atomicExch(&B.fix_mask[4 * (long long)tile + 3], 1ull) == 0ull) {
    const unsigned int k = atomicAdd(&dev->fix_count, 1u);
    B.fix_list[k] = tile;
  }
}

// One DOF through the rounds of the point update.  States are carried in FP64; the
// evolution operators work in the bulk type R on deviations from the linearisation state.
// FIX = false (main pass): a DOF whose value needs the positivity limiter is left to the
// fix-up pass, which keeps the rare limiter code out of the main kernel's registers.
// FIX = true (fix-up pass): the same computation with Algorithm 3 applied.
template <class R, int KIND, bool FIX>
__device__ __forceinline__ void evolve_dof(Smem<R>& S, const Params& P, const Bufs& B,
                                           DevState* dev, int tile, int a, int b, int gi,
                                           int gj, double dt, double& speed) {
  const Geo<R> G = {R(P.idx), R(0.5 * P.dy * P.idx), R(P.gamma), R(0.5 * P.hmin)};
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
    e = eg2<R, KIND>(S, cb, U0, R(0.25 * dt), G, dq);
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
  } else if (P.mode == LIN_AVG) {
    avg_lin(lin);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) lin[v] = U0[v];
  }

  double Uh[4], U1[4];
  {
    R d[4];
    e = eg2<R, KIND>(S, cb, lin, R(0.5 * dt), G, d);
    if (e) { set_err(dev, e); return; }
#pragma unroll
    for (int v = 0; v < 4; ++v) Uh[v] = lin[v] + (double)d[v] + h2 * (double)Cv[v];
  }
  // positivity of the intermediate value (Algorithm 3)
  if (!admissible(Uh[0], Uh[3])) {
    if (!P.limiter) { set_err(dev, ERR_NONPHYS); return; }
    if constexpr (!FIX) {
      mark_fix(B, dev, tile, KIND, threadIdx.x & 63);
      return;
    } else {
      double Ut[4];
      avg_lin(Ut);
      e = limit_value<R, KIND>(S, P, G, site, a, b, cb, Ut, 0.5 * dt, Uh, dev);
      if (e) { set_err(dev, e); return; }
    }
  }
  {
    R d[4];
    e = eg2<R, KIND>(S, cb, Uh, R(dt), G, d);
    if (e) { set_err(dev, e); return; }
#pragma unroll
    for (int v = 0; v < 4; ++v) U1[v] = Uh[v] + (double)d[v] + f2 * (double)Cv[v];
  }
  if (P.limiter && !admissible(U1[0], U1[3])) {
    if constexpr (!FIX) {
      mark_fix(B, dev, tile, KIND, threadIdx.x & 63);
      return;
    } else {
      double Ut[4];
      avg_lin(Ut);
      e = limit_value<R, KIND>(S, P, G, site, a, b, cb, Ut, dt, U1, dev);
      if (e) { set_err(dev, e); return; }
    }
  }

  // outputs: new point value, Simpson-in-time flux sums, wave speed
  double* out = (KIND == KIND_K) ? B.K_out : (KIND == KIND_X ? B.X_out : B.Y_out);
  const long long o = (long long)gj * P.pP + gi;
#pragma unroll
  for (int v = 0; v < 4; ++v) out[v * P.sP + o] = U1[v];
  const double g1inv = 1.0 / (P.gamma - 1.0);
  double Fs[4] = {0, 0, 0, 0}, Gs[4] = {0, 0, 0, 0};
  {
    double Ul[4], F[4], Gq[4];
#pragma unroll 1
    for (int lvl = 0; lvl < 3; ++lvl) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Ul[v] = lvl == 0 ? site[v * NS + s0] : (lvl == 1 ? Uh[v] : U1[v]);
      flux_fg(Ul, g1inv, F, Gq);
      const double w = lvl == 1 ? 4.0 : 1.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Fs[v] += w * F[v];
        Gs[v] += w * Gq[v];
      }
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
// decision is uniform over the block even if another block flags an error meanwhile.
// Returns false if the step does not run.
__device__ __forceinline__ bool step_dt(const Params& P, DevState* dev, double dt_host, int slot,
                                        double* dt_out) {
  __shared__ double s_dt;
  __shared__ int s_run;
  if (threadIdx.x == 0) {
    int run = 1, last = 0;
    double dt = dt_host;
    if (dev->err) {
      run = 0;
    } else if (!(dt_host > 0.0)) {
      const double t = dev->t, te = dev->t_end;
      const double smax = __longlong_as_double((long long)dev->smax[slot]);
      if (!(t < te)) {
        run = 0;
        if (blockIdx.x == 0) dev->active = 0;
      } else if (!(smax > 0.0) || !(smax < 1e300)) {
        run = 0;
        set_err(dev, ERR_NONPHYS);
      } else {
        dt = dev->cfl * P.hmin / smax;
        if (t + dt >= te) { dt = te - t; last = 1; }
      }
    }
    if (run && blockIdx.x == 0) {
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

// Stage the t_n point values of a tile's halo in LDS and build the halo cells'
// reconstructions.  Ends with a barrier.
template <class R>
__device__ __forceinline__ void stage_and_prep(Smem<R>& S, const Params& P, const Bufs& B,
                                               DevState* dev, int tile, bool count) {
  const int i0 = (tile % P.tiles_x) * TILE, j0 = (tile / P.tiles_x) * TILE;
  const int tid = threadIdx.x;

  // 1. stage the t_n point values of the halo (local sites -1 .. TILE) in LDS
  for (int e = tid; e < 3 * NS; e += PT_THREADS) {
    const int kind = e / NS, s = e % NS;
    const int a = s % HS - 1, b = s / HS - 1;
    const int gi = i0 + a, gj = j0 + b;
    int si, sj;
    const double* src;
    double* dst;
    if (kind == 0) {
      si = wrap_line(gi, P.nx, P.per_x); sj = wrap_line(gj, P.ny, P.per_y); src = B.K_in; dst = S.sk;
    } else if (kind == 1) {
      si = wrap_line(gi, P.nx, P.per_x); sj = wrap_cell(gj, P.ny, P.per_y); src = B.X_in; dst = S.sx;
    } else {
      si = wrap_cell(gi, P.nx, P.per_x); sj = wrap_line(gj, P.ny, P.per_y); src = B.Y_in; dst = S.sy;
    }
    const long long o = (long long)sj * P.pP + si;
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[v * NS + s] = src[v * P.sP + o];
  }
  __syncthreads();

  // 2. cell reconstructions of the halo cells (local cells -1 .. TILE-1)
  for (int c = tid; c < NC; c += PT_THREADS) {
    const int a = c % HC - 1, b = c / HC - 1;
    const int gi = wrap_cell(i0 + a, P.nx, P.per_x), gj = wrap_cell(j0 + b, P.ny, P.per_y);
    const double g1inv = 1.0 / (P.gamma - 1.0), gm1 = P.gamma - 1.0;
    // node k of the cell: 0..3 corners K(a,b) K(a+1,b) K(a,b+1) K(a+1,b+1),
    // 4,5 X(a,b) X(a+1,b), 6,7 Y(a,b) Y(a,b+1)
    const double* nptr[8] = {S.sk + sidx(a, b), S.sk + sidx(a + 1, b), S.sk + sidx(a, b + 1),
                        S.sk + sidx(a + 1, b + 1), S.sx + sidx(a, b), S.sx + sidx(a + 1, b),
                        S.sy + sidx(a, b), S.sy + sidx(a, b + 1)};
    auto node = [&](int k, double W[4]) {
#pragma unroll
      for (int v = 0; v < 4; ++v) W[v] = (double)nptr[k][v * NS];
    };
    double Qb[4];
    const long long oa = (long long)gj * P.pA + gi;
#pragma unroll
    for (int v = 0; v < 4; ++v) Qb[v] = B.A_in[v * P.sA + oa];
    // reference state: mean of the eight nodes (exact for equal nodes)
    double Wr[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Wr[v] = ((((double)nptr[0][v * NS] + (double)nptr[1][v * NS]) +
                ((double)nptr[2][v * NS] + (double)nptr[3][v * NS])) +
               (((double)nptr[4][v * NS] + (double)nptr[5][v * NS]) +
                ((double)nptr[6][v * NS] + (double)nptr[7][v * NS]))) * 0.125;
    }
    // inverse Simpson for the centre value: Q_c = Q-bar + [sum_K (Q-bar - Q_k)
    //                                          + 4 sum_E (Q-bar - Q_e)] / 16
    double dQ[4], Uc[4];
    {
      double sK[4] = {0, 0, 0, 0}, sE[4] = {0, 0, 0, 0}, W[4], Q[4];
      for (int k = 0; k < 8; ++k) {
        node(k, W);
        p2c(W, g1inv, Q);
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
    if (!admissible(Uc[0], Uc[3])) {
      c2p_plain(Qb, gm1, Uc);
      const bool owned = a >= 0 && b >= 0 && (i0 + a) < P.nx && (j0 + b) < P.ny;
      if (owned && count) atomicAdd(&dev->cnt[AF_CNT_CENTRE], 1ull);
    }
    const double rho = P.dx / P.dy, rho2 = rho * rho;
    // primitive Simpson average and monomial coefficients, one variable at a time
#pragma unroll 1
    for (int v = 0; v < 4; ++v) {
      double w[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) w[k] = (double)nptr[k][v * NS];
      const double u = Uc[v];
      const double sK4 = ((w[0] - u) + (w[1] - u)) + ((w[2] - u) + (w[3] - u));
      const double sE4 = ((w[4] - u) + (w[5] - u)) + ((w[6] - u) + (w[7] - u));
      S.ub[v * NC + c] = u + (sK4 + 4.0 * sE4) * (1.0 / 36.0);
      const double N[3][3] = {{w[0], w[4], w[2]}, {w[6], u, w[7]}, {w[1], w[5], w[3]}};
      double cm[9];
      nodes_to_monomials(N, cm);
      S.c0[v * NC + c] = cm[0];
      // c_mn of xi^m eta^n -> coefficient of xi^m (eta dy/dx)^n: the circle integrals use
      // dx as the unit length in both directions
#pragma unroll
      for (int k = 1; k < 9; ++k)
        S.ch[(v * 8 + k - 1) * NC + c] = (R)(k % 3 == 0 ? cm[k] : (k % 3 == 1 ? cm[k] * rho
                                                                              : cm[k] * rho2));
    }
  }
  __syncthreads();
}

// Evolve the tile's own DOFs: wavefront 0 -> K; wavefront 1 -> X, then Y (an edge EG2 costs
// well under half of a corner EG2, so the two waves are about equally loaded).  In the fix-up
// pass only the lanes listed in `mask` (per kind) run.
template <class R, bool FIX>
__device__ __forceinline__ void evolve_tile(Smem<R>& S, const Params& P, const Bufs& B,
                                            DevState* dev, int tile, double dt,
                                            const unsigned long long* mask, double& speed) {
  const int i0 = (tile % P.tiles_x) * TILE, j0 = (tile / P.tiles_x) * TILE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int a = lane % TILE, b = lane / TILE;
  const int gi = i0 + a, gj = j0 + b;
  auto listed = [&](int kind) { return !FIX || ((mask[kind] >> lane) & 1ull); };
  if (wave == 0) {
    if (listed(KIND_K) && gi < P.nkx && gj < P.nky)
      evolve_dof<R, KIND_K, FIX>(S, P, B, dev, tile, a, b, gi, gj, dt, speed);
  } else {
    if (listed(KIND_X) && gi < P.nkx && gj < P.ny)
      evolve_dof<R, KIND_X, FIX>(S, P, B, dev, tile, a, b, gi, gj, dt, speed);
    if (listed(KIND_Y) && gi < P.nx && gj < P.nky)
      evolve_dof<R, KIND_Y, FIX>(S, P, B, dev, tile, a, b, gi, gj, dt, speed);
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

template <class R>
__device__ __forceinline__ void points_body(Smem<R>& S, const Params& P, const Bufs& B,
                                            DevState* dev, double dt_host, int slot) {
  double dt;
  if (!step_dt(P, dev, dt_host, slot, &dt)) return;
  const int tile = tile_of_block(blockIdx.x, P.tiles_x * P.tiles_y);
  stage_and_prep(S, P, B, dev, tile, true);
  double speed = 0.0;
  evolve_tile<R, false>(S, P, B, dev, tile, dt, nullptr, speed);
  block_max_atomic(speed, &dev->smax[slot ^ 1], S.red);
}

// Positivity fix-up pass: the tiles listed by the main pass are staged again and only their
// flagged DOFs are recomputed with Algorithm 3.  Cheap when the list is empty.
template <class R>
__device__ __forceinline__ void fixup_body(Smem<R>& S, const Params& P, const Bufs& B,
                                           DevState* dev, int slot) {
  __shared__ unsigned long long mask[3];
  __shared__ int s_run;
  __shared__ unsigned int s_n;
  __shared__ double s_dt;
  if (threadIdx.x == 0) {
    s_run = !dev->err && dev->active;
    s_n = dev->fix_count;
    s_dt = dev->dt;
  }
  __syncthreads();
  const bool run = s_run != 0;
  const double dt = s_dt;
  const unsigned int n = s_n;
  double speed = 0.0;
  for (unsigned int k = blockIdx.x; k < n; k += gridDim.x) {
    const int tile = B.fix_list[k];
    if (threadIdx.x < 3) mask[threadIdx.x] = B.fix_mask[4 * (long long)tile + threadIdx.x];
    __syncthreads();
    if (run) {
      stage_and_prep(S, P, B, dev, tile, false);
      evolve_tile<R, true>(S, P, B, dev, tile, dt, mask, speed);
    }
    __syncthreads();
    if (threadIdx.x < 4) B.fix_mask[4 * (long long)tile + threadIdx.x] = 0ull;
  }
  if (n > blockIdx.x) block_max_atomic(speed, &dev->smax[slot ^ 1], S.red);
}

// One launch per step and precision.  AF_WAVES_F32 / AF_WAVES_F64 set the wavefronts per SIMD
// that the register allocation aims at (0: the compiler's choice).
#ifndef AF_WAVES_F32
#define AF_WAVES_F32 0
#endif
#ifndef AF_WAVES_F64
#define AF_WAVES_F64 3
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
__global__ __launch_bounds__(PT_THREADS) AF_ATTR_F32
void k_points_f32(Params P, Bufs B, DevState* dev, double dt_host, int slot) {
  __shared__ Smem<float> S;
  points_body<float>(S, P, B, dev, dt_host, slot);
}
__global__ __launch_bounds__(PT_THREADS) AF_ATTR_F64
void k_points_f64(Params P, Bufs B, DevState* dev, double dt_host, int slot) {
  __shared__ Smem<double> S;
  points_body<double>(S, P, B, dev, dt_host, slot);
}
__global__ __launch_bounds__(PT_THREADS) void k_fixup_f32(Params P, Bufs B, DevState* dev,
                                                         int slot) {
  __shared__ Smem<float> S;
  fixup_body<float>(S, P, B, dev, slot);
}
__global__ __launch_bounds__(PT_THREADS) void k_fixup_f64(Params P, Bufs B, DevState* dev,
                                                         int slot) {
  __shared__ Smem<double> S;
  fixup_body<double>(S, P, B, dev, slot);
}
constexpr int FIX_BLOCKS = 1024;

// ------------------------------------------------------------------------------------------
// Kernel 2: Simpson space-time fluxes and the conservative update of the averages.
// ------------------------------------------------------------------------------------------
constexpr int UP_THREADS = 256;
constexpr int UP_MAX_BLOCKS = 1024;

__global__ __launch_bounds__(UP_THREADS) void k_update(Params P, const double* __restrict__ A_in,
                                                      double* __restrict__ A_out,
                                                      const double* __restrict__ FK,
                                                      const double* __restrict__ FX,
                                                      const double* __restrict__ FY,
                                                      DevState* dev, int slot) {
  __shared__ double red[4];
  __shared__ int last_block;
  const bool run = !dev->err && dev->active;
  const double dt = dev->dt;
  const double lx = dt * P.idx * (1.0 / 36.0), ly = dt * P.idy * (1.0 / 36.0);
  double speed = 0.0;
  bool bad = false;
  if (run) {
    // rows of cells, 256 consecutive cells of a row per pass (coalesced)
    const int chunks_x = (P.nx + UP_THREADS - 1) / UP_THREADS;
    const long long nwork = (long long)chunks_x * P.ny;
    for (long long w = blockIdx.x; w < nwork; w += gridDim.x) {
      const int j = (int)(w / chunks_x);
      const int i = (int)(w % chunks_x) * UP_THREADS + threadIdx.x;
      if (i >= P.nx) continue;
      const int ip = wrap_line(i + 1, P.nx, P.per_x), jp = wrap_line(j + 1, P.ny, P.per_y);
      const long long kw0 = (long long)j * P.pF + i, kw1 = (long long)jp * P.pF + i;
      const long long ke0 = (long long)j * P.pF + ip, ke1 = (long long)jp * P.pF + ip;
      const long long oa = (long long)j * P.pA + i;
      double Q[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double* fk = FK + v * P.sF;
        const double* gk = FK + (4 + v) * P.sF;
        const double Fw = fk[kw0] + 4.0 * FX[v * P.sF + kw0] + fk[kw1];
        const double Fe = fk[ke0] + 4.0 * FX[v * P.sF + ke0] + fk[ke1];
        const double Gs = gk[kw0] + 4.0 * FY[v * P.sF + kw0] + gk[ke0];
        const double Gn = gk[kw1] + 4.0 * FY[v * P.sF + kw1] + gk[ke1];
        Q[v] = A_in[v * P.sA + oa] - lx * (Fe - Fw) - ly * (Gn - Gs);
        A_out[v * P.sA + oa] = Q[v];
      }
      double U[4];
      c2p_plain(Q, P.gamma - 1.0, U);
      if (!admissible(U[0], U[3])) bad = true;
      else speed = mx(speed, wave_speed(U, P.gamma));
    }
  }
  if (bad) set_err(dev, ERR_NONPHYS);
  {
    double v = speed;
    for (int off = 32; off > 0; off >>= 1) v = mx(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = mx(mx(red[0], red[1]), mx(red[2], red[3]));
    if (run) atomic_max_pos(&dev->smax[slot ^ 1], m);
    __threadfence();
    const unsigned int ticket = atomicAdd(&dev->done_blocks, 1u);
    last_block = (ticket == gridDim.x - 1);
  }
  __syncthreads();
  if (last_block && threadIdx.x == 0) {
    __threadfence();
    dev->done_blocks = 0;
    dev->fix_count = 0u;
    if (run && !atomicAdd(&dev->err, 0)) {
      dev->t = dev->last ? dev->t_end : dev->t + dt;
      dev->steps += 1;
      dev->smax[slot] = 0ull;
    }
  }
}

// Largest wave speed of the current state (averages and point values) into smax[slot].
__global__ void k_cfl(Params P, const double* __restrict__ A, const double* __restrict__ K,
                      const double* __restrict__ X, const double* __restrict__ Y, DevState* dev,
                      int slot) {
  __shared__ double red[4];
  const long long n0 = (long long)P.nx * P.ny, n1 = (long long)P.nkx * P.nky,
                  n2 = (long long)P.nkx * P.ny, n3 = (long long)P.nx * P.nky;
  const long long ntot = n0 + n1 + n2 + n3;
  double speed = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ntot;
       e += (long long)gridDim.x * blockDim.x) {
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
    // non-admissible values do not enter the time step (as NaN speeds would not)
    if (admissible(U[0], U[3])) speed = mx(speed, wave_speed(U, P.gamma));
  }
  block_max_atomic(speed, &dev->smax[slot], red);
}

}  // namespace af

// ==========================================================================================
// Host runtime
// ==========================================================================================
using namespace af;

struct af_handle {
  int nx = 0, ny = 0, per_x = 1, per_y = 1, nkx = 0, nky = 0;
  double x0 = 0, x1 = 1, y0 = 0, y1 = 1, dx = 1, dy = 1, gamma = 1.4;
  int prec = AF_PREC_FP64, mode = AF_LIN_AF3, correction = 1, limiter = 0;
  int graph_steps = 16;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  long long pA = 0, pP = 0, pF = 0;
  double* A[2] = {nullptr, nullptr};
  void* K[2] = {nullptr, nullptr};
  void* X[2] = {nullptr, nullptr};
  void* Y[2] = {nullptr, nullptr};
  double* FK = nullptr;
  double* FX = nullptr;
  double* FY = nullptr;
  unsigned long long* fix_mask = nullptr;
  int* fix_list = nullptr;
  DevState* dev = nullptr;
  int cur = 0;
  bool has_state = false;
  long long steps_base = 0;
  hipGraphExec_t gexec = nullptr;
  int gexec_steps = 0;
  // AF_OPT_TIMING: events around each kernel of every eager step
  int timing = 0;
  std::vector<hipEvent_t> ev;  // 3 per step: before points, between, after update
  double ms_points = 0.0, ms_update = 0.0;
  long long timed_steps = 0;
  double* stage = nullptr;  // pinned host staging buffer of host <-> device copies
  std::string err;
};

static std::string g_create_error;

static int fail(const af_handle* h, int code, const std::string& msg) {
  if (h) const_cast<af_handle*>(h)->err = msg;
  else g_create_error = msg;
  return code;
}

#define HIP_OK(call, h)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(h, e_ == hipErrorOutOfMemory ? AF_ERR_OOM : AF_ERR_DEVICE,         \
                  std::string(#call) + ": " + hipGetErrorString(e_));                \
  } while (0)


static Params make_params(const af_handle* h) {
  Params P;
  P.nx = h->nx; P.ny = h->ny; P.nkx = h->nkx; P.nky = h->nky;
  P.per_x = h->per_x; P.per_y = h->per_y;
  P.tiles_x = (h->nkx + TILE - 1) / TILE;
  P.tiles_y = (h->nky + TILE - 1) / TILE;
  P.dx = h->dx; P.dy = h->dy; P.idx = 1.0 / h->dx; P.idy = 1.0 / h->dy;
  P.gamma = h->gamma; P.hmin = std::min(h->dx, h->dy);
  P.mode = h->mode; P.correction = h->correction; P.limiter = h->limiter; P.pad = 0;
  P.pA = h->pA; P.sA = h->pA * h->ny;
  P.pP = h->pP; P.sP = h->pP * h->nky;
  P.pF = h->pF; P.sF = h->pF * h->nky;
  return P;
}

static void free_buffers(af_handle* h) {
  for (int k = 0; k < 2; ++k) {
    if (h->A[k]) (void)hipFree(h->A[k]);
    if (h->K[k]) (void)hipFree(h->K[k]);
    if (h->X[k]) (void)hipFree(h->X[k]);
    if (h->Y[k]) (void)hipFree(h->Y[k]);
    h->A[k] = nullptr; h->K[k] = h->X[k] = h->Y[k] = nullptr;
  }
  if (h->FK) (void)hipFree(h->FK);
  if (h->FX) (void)hipFree(h->FX);
  if (h->FY) (void)hipFree(h->FY);
  h->FK = h->FX = h->FY = nullptr;
  if (h->fix_mask) (void)hipFree(h->fix_mask);
  if (h->fix_list) (void)hipFree(h->fix_list);
  h->fix_mask = nullptr;
  h->fix_list = nullptr;
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  h->gexec = nullptr;
  h->gexec_steps = 0;
}

static int alloc_buffers(af_handle* h) {
  free_buffers(h);
  h->pA = (h->nx + 31) / 32 * 32;
  h->pP = (h->nkx + 63) / 64 * 64;
  h->pF = h->pP;
  const size_t na = (size_t)4 * h->pA * h->ny, np = (size_t)4 * h->pP * h->nky;
  const size_t nf = (size_t)h->pF * h->nky;
  for (int k = 0; k < 2; ++k) {
    HIP_OK(hipMalloc(&h->A[k], na * 8), h);
    HIP_OK(hipMalloc(&h->K[k], np * sizeof(double)), h);
    HIP_OK(hipMalloc(&h->X[k], np * sizeof(double)), h);
    HIP_OK(hipMalloc(&h->Y[k], np * sizeof(double)), h);
  }
  HIP_OK(hipMalloc(&h->FK, nf * 8 * 8), h);
  HIP_OK(hipMalloc(&h->FX, nf * 4 * 8), h);
  HIP_OK(hipMalloc(&h->FY, nf * 4 * 8), h);
  const size_t ntiles = (size_t)((h->nkx + TILE - 1) / TILE) * ((h->nky + TILE - 1) / TILE);
  HIP_OK(hipMalloc(&h->fix_mask, ntiles * 4 * sizeof(unsigned long long)), h);
  HIP_OK(hipMalloc(&h->fix_list, ntiles * sizeof(int)), h);
  HIP_OK(hipMemset(h->fix_mask, 0, ntiles * 4 * sizeof(unsigned long long)), h);
  h->has_state = false;
  return AF_OK;
}

extern "C" int af_create(const af_grid* grid, double gamma, const af_bc* bc, af_handle** out) {
  if (!out) return fail(nullptr, AF_ERR_INVALID_ARG, "af_create: out is NULL");
  *out = nullptr;
  if (!grid || !bc) return fail(nullptr, AF_ERR_INVALID_ARG, "af_create: NULL grid or bc");
  if (grid->nx < 2 || grid->ny < 2 || grid->nx > (1 << 16) || grid->ny > (1 << 16))
    return fail(nullptr, AF_ERR_INVALID_ARG, "af_create: nx, ny must be in [2, 65536]");
  if (!(grid->x1 > grid->x0) || !(grid->y1 > grid->y0))
    return fail(nullptr, AF_ERR_INVALID_ARG, "af_create: empty domain");
  if (!(gamma > 1.0)) return fail(nullptr, AF_ERR_INVALID_ARG, "af_create: gamma must be > 1");
  auto okbc = [](int k) { return k == AF_BC_PERIODIC || k == AF_BC_OUTFLOW; };
  if (!okbc(bc->left) || !okbc(bc->right) || !okbc(bc->bottom) || !okbc(bc->top))
    return fail(nullptr, AF_ERR_INVALID_ARG, "af_create: unknown boundary kind");
  if ((bc->left == AF_BC_PERIODIC) != (bc->right == AF_BC_PERIODIC) ||
      (bc->bottom == AF_BC_PERIODIC) != (bc->top == AF_BC_PERIODIC))
    return fail(nullptr, AF_ERR_INVALID_ARG, "af_create: periodic must pair on an axis");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(nullptr, AF_ERR_DEVICE, "af_create: no HIP device");
  af_handle* h = new af_handle();
  h->nx = grid->nx; h->ny = grid->ny;
  h->x0 = grid->x0; h->x1 = grid->x1; h->y0 = grid->y0; h->y1 = grid->y1;
  h->dx = (h->x1 - h->x0) / h->nx; h->dy = (h->y1 - h->y0) / h->ny;
  h->per_x = bc->left == AF_BC_PERIODIC; h->per_y = bc->bottom == AF_BC_PERIODIC;
  h->nkx = h->nx + (h->per_x ? 0 : 1); h->nky = h->ny + (h->per_y ? 0 : 1);
  h->gamma = gamma;
  int e = AF_OK;
  if (hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess)
    e = fail(h, AF_ERR_DEVICE, "af_create: hipStreamCreate");
  h->stream = h->own_stream;
  if (e == AF_OK) e = alloc_buffers(h);
  if (e == AF_OK) {
    hipError_t he = hipMalloc(&h->dev, sizeof(DevState));
    if (he != hipSuccess) e = fail(h, AF_ERR_OOM, "af_create: hipMalloc(dev)");
    else if (hipMemset(h->dev, 0, sizeof(DevState)) != hipSuccess)
      e = fail(h, AF_ERR_DEVICE, "af_create: hipMemset");
  }
  if (e != AF_OK) {
    g_create_error = h->err;
    free_buffers(h);
    if (h->dev) (void)hipFree(h->dev);
    if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
    delete h;
    return e;
  }
  *out = h;
  return AF_OK;
}

extern "C" void af_destroy(af_handle* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  free_buffers(h);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  if (h->dev) (void)hipFree(h->dev);
  if (h->stage) (void)hipHostFree(h->stage);
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  delete h;
}

extern "C" const char* af_last_error(const af_handle* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

extern "C" int64_t af_dof_count(const af_handle* h) {
  if (!h) return 0;
  return (int64_t)h->nx * h->ny + (int64_t)h->nkx * h->nky + (int64_t)h->nkx * h->ny +
         (int64_t)h->nx * h->nky;
}

extern "C" int af_set_option(af_handle* h, int key, int64_t value) {
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_set_option: NULL handle");
  switch (key) {
    case AF_OPT_PRECISION:
      if (value != AF_PREC_FP64 && value != AF_PREC_FP32)
        return fail(h, AF_ERR_INVALID_ARG, "af_set_option: precision must be FP64 or FP32");
      if (value != h->prec) {
        h->prec = (int)value;
        return alloc_buffers(h);
      }
      return AF_OK;
    case AF_OPT_LINEARISATION:
      if (value < 0 || value > 2) return fail(h, AF_ERR_INVALID_ARG, "af_set_option: bad mode");
      h->mode = (int)value;
      break;
    case AF_OPT_CORRECTION:
      if (value != 0 && value != 1) return fail(h, AF_ERR_INVALID_ARG, "af_set_option: 0 or 1");
      h->correction = (int)value;
      break;
    case AF_OPT_LIMITER:
      if (value != 0 && value != 1) return fail(h, AF_ERR_INVALID_ARG, "af_set_option: 0 or 1");
      h->limiter = (int)value;
      break;
    case AF_OPT_TIMING:
      if (value != 0 && value != 1) return fail(h, AF_ERR_INVALID_ARG, "af_set_option: 0 or 1");
      h->timing = (int)value;
      h->ms_points = h->ms_update = 0.0;
      h->timed_steps = 0;
      break;
    case AF_OPT_GRAPH_STEPS:
      if (value < 0 || value > 4096 || (value & 1))
        return fail(h, AF_ERR_INVALID_ARG, "af_set_option: graph steps must be even, 0..4096");
      h->graph_steps = (int)value;
      break;
    default:
      return fail(h, AF_ERR_INVALID_ARG, "af_set_option: unknown key");
  }
  if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; h->gexec_steps = 0; }
  return AF_OK;
}

extern "C" int af_set_stream(af_handle* h, void* s) {
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_set_stream: NULL handle");
  (void)hipStreamSynchronize(h->stream);
  h->stream = s ? (hipStream_t)s : h->own_stream;
  if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; h->gexec_steps = 0; }
  return AF_OK;
}

// Host <-> device copies go through a pinned staging buffer, in blocks of whole rows: one
// 2D copy per block between the padded device rows and the staging buffer, one memcpy between
// the staging buffer and the caller's array.  Synchronous on the handle's stream.
constexpr size_t STAGE_BYTES = 8u << 20;

static int ensure_stage(const af_handle* hc) {
  af_handle* h = const_cast<af_handle*>(hc);
  if (!h->stage) HIP_OK(hipHostMalloc((void**)&h->stage, STAGE_BYTES, hipHostMallocDefault), h);
  return AF_OK;
}

// One variable: host FP64 rows x cols (unpadded, row-major) <-> device FP64 rows x cols with
// a row pitch of `pitch` elements.
static int copy2d(const af_handle* h, bool to_device, double* dev, long long pitch, int rows,
                  int cols, double* host) {
  if (cols > pitch) return fail(h, AF_ERR_INVALID_ARG, "copy2d: cols exceed pitch");
  if (int e = ensure_stage(h)) return e;
  const size_t row_bytes = (size_t)cols * 8;
  const int block = (int)std::max<size_t>(1, STAGE_BYTES / row_bytes);
  for (int r0 = 0; r0 < rows; r0 += block) {
    const int nr = std::min(block, rows - r0);
    double* d = dev + (size_t)r0 * pitch;
    double* hst = host + (size_t)r0 * cols;
    if (to_device) {
      std::memcpy(h->stage, hst, (size_t)nr * row_bytes);
      HIP_OK(hipMemcpy2DAsync(d, pitch * 8, h->stage, row_bytes, row_bytes, (size_t)nr,
                              hipMemcpyHostToDevice, h->stream), h);
      HIP_OK(hipStreamSynchronize(h->stream), h);
    } else {
      HIP_OK(hipMemcpy2DAsync(h->stage, row_bytes, d, pitch * 8, row_bytes, (size_t)nr,
                              hipMemcpyDeviceToHost, h->stream), h);
      HIP_OK(hipStreamSynchronize(h->stream), h);
      std::memcpy(hst, h->stage, (size_t)nr * row_bytes);
    }
  }
  return AF_OK;
}

// The padded arrays store variable v at offset v * rows_alloc * pitch: copy one variable at a
// time.
static int copy4(const af_handle* h, bool to_device, void* dev, long long pitch, int rows_alloc,
                 int rows, int cols, double* host) {
  if (rows > rows_alloc) return fail(h, AF_ERR_INVALID_ARG, "copy4: rows exceed allocation");
  for (int v = 0; v < 4; ++v) {
    double* d = (double*)dev + (size_t)v * rows_alloc * pitch;
    if (int e = copy2d(h, to_device, d, pitch, rows, cols, host + (size_t)v * rows * cols))
      return e;
  }
  return AF_OK;
}

extern "C" int af_set_state(af_handle* h, const double* avg, const double* K, const double* X,
                            const double* Y, double t) {
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_set_state: NULL handle");
  if (!avg || !K || !X || !Y) return fail(h, AF_ERR_INVALID_ARG, "af_set_state: NULL array");
  if (!std::isfinite(t)) return fail(h, AF_ERR_INVALID_ARG, "af_set_state: t not finite");
  const size_t nc = (size_t)h->nx * h->ny;
  for (size_t k = 0; k < nc; ++k) {
    const double r = avg[k], E = avg[3 * nc + k];
    const double kin = 0.5 * (avg[nc + k] * avg[nc + k] + avg[2 * nc + k] * avg[2 * nc + k]) / r;
    if (!(r > 0.0) || !((h->gamma - 1.0) * (E - kin) > 0.0))
      return fail(h, AF_ERR_NONPHYSICAL, "af_set_state: non-admissible cell average");
  }
  h->cur = 0;
  int e;
  if ((e = copy4(h, true, h->A[0], h->pA, h->ny, h->ny, h->nx, const_cast<double*>(avg))))
    return e;
  if ((e = copy4(h, true, h->K[0], h->pP, h->nky, h->nky, h->nkx, const_cast<double*>(K))))
    return e;
  if ((e = copy4(h, true, h->X[0], h->pP, h->nky, h->ny, h->nkx, const_cast<double*>(X))))
    return e;
  if ((e = copy4(h, true, h->Y[0], h->pP, h->nky, h->nky, h->nx, const_cast<double*>(Y))))
    return e;
  DevState ds;
  std::memset(&ds, 0, sizeof(ds));
  ds.t = t;
  ds.t_end = t;
  HIP_OK(hipMemcpyAsync(h->dev, &ds, sizeof(ds), hipMemcpyHostToDevice, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  h->has_state = true;
  h->steps_base = 0;
  return AF_OK;
}

extern "C" int af_get_state(const af_handle* h, double* avg, double* K, double* X, double* Y,
                            double* t) {
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_get_state: NULL handle");
  if (!h->has_state) return fail(h, AF_ERR_INVALID_ARG, "af_get_state: no state set");
  const int c = h->cur;
  int e;
  if (avg && (e = copy4(h, false, h->A[c], h->pA, h->ny, h->ny, h->nx, avg))) return e;
  if (K && (e = copy4(h, false, h->K[c], h->pP, h->nky, h->nky, h->nkx, K))) return e;
  if (X && (e = copy4(h, false, h->X[c], h->pP, h->nky, h->ny, h->nkx, X))) return e;
  if (Y && (e = copy4(h, false, h->Y[c], h->pP, h->nky, h->nky, h->nx, Y))) return e;
  if (t) {
    DevState ds;
    HIP_OK(hipMemcpyAsync(&ds, h->dev, sizeof(ds), hipMemcpyDeviceToHost, h->stream), h);
    HIP_OK(hipStreamSynchronize(h->stream), h);
    *t = ds.t;
  }
  return AF_OK;
}

extern "C" int af_get_counters(const af_handle* h, int64_t* out) {
  if (!h || !out) return fail(h, AF_ERR_INVALID_ARG, "af_get_counters: NULL argument");
  DevState ds;
  HIP_OK(hipMemcpyAsync(&ds, h->dev, sizeof(ds), hipMemcpyDeviceToHost, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  for (int k = 0; k < AF_NCOUNTERS; ++k) out[k] = (int64_t)ds.cnt[k];
  out[AF_CNT_STEPS] = ds.steps;
  return AF_OK;
}

// enqueue one step reading buffer `in` (0/1); dt_host > 0 for a caller-given step
template <class R>
static void enqueue_step_t(af_handle* h, int in, double dt_host) {
  const Params P = make_params(h);
  const int out = in ^ 1;
  Bufs B;
  B.A_in = h->A[in]; B.A_out = h->A[out];
  B.K_in = (const double*)h->K[in]; B.X_in = (const double*)h->X[in];
  B.Y_in = (const double*)h->Y[in];
  B.K_out = (double*)h->K[out]; B.X_out = (double*)h->X[out]; B.Y_out = (double*)h->Y[out];
  B.FK = h->FK; B.FX = h->FX; B.FY = h->FY;
  B.fix_mask = h->fix_mask; B.fix_list = h->fix_list;
  const int ntiles = P.tiles_x * P.tiles_y;
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
  if (h->timing) {
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventCreate(&e2);
    (void)hipEventRecord(e0, h->stream);
  }
  if constexpr (sizeof(R) == 4)
    hipLaunchKernelGGL(k_points_f32, dim3(ntiles), dim3(PT_THREADS), 0, h->stream, P, B, h->dev,
                       dt_host, in);
  else
    hipLaunchKernelGGL(k_points_f64, dim3(ntiles), dim3(PT_THREADS), 0, h->stream, P, B, h->dev,
                       dt_host, in);
  if (h->limiter) {
    const int nb = std::min(ntiles, FIX_BLOCKS);
    if constexpr (sizeof(R) == 4)
      hipLaunchKernelGGL(k_fixup_f32, dim3(nb), dim3(PT_THREADS), 0, h->stream, P, B, h->dev, in);
    else
      hipLaunchKernelGGL(k_fixup_f64, dim3(nb), dim3(PT_THREADS), 0, h->stream, P, B, h->dev, in);
  }
  if (h->timing) (void)hipEventRecord(e1, h->stream);
  const long long nwork = (long long)((h->nx + UP_THREADS - 1) / UP_THREADS) * h->ny;
  const int gu = (int)std::min<long long>(nwork, UP_MAX_BLOCKS);
  hipLaunchKernelGGL(k_update, dim3(gu), dim3(UP_THREADS), 0, h->stream, P, (const double*)h->A[in],
                     h->A[out], (const double*)h->FK, (const double*)h->FX,
                     (const double*)h->FY, h->dev, in);
  if (h->timing) {
    (void)hipEventRecord(e2, h->stream);
    h->ev.push_back(e0);
    h->ev.push_back(e1);
    h->ev.push_back(e2);
  }
}

// fold recorded events into the kernel times (only steps that committed are counted)
static void collect_timing(af_handle* h, long long committed) {
  for (size_t k = 0; k + 2 < h->ev.size(); k += 3) {
    float a = 0.f, b = 0.f;
    if ((long long)(k / 3) < committed &&
        hipEventElapsedTime(&a, h->ev[k], h->ev[k + 1]) == hipSuccess &&
        hipEventElapsedTime(&b, h->ev[k + 1], h->ev[k + 2]) == hipSuccess) {
      h->ms_points += a;
      h->ms_update += b;
      h->timed_steps += 1;
    }
  }
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
}

static void enqueue_step(af_handle* h, int in, double dt_host) {
  if (h->prec == AF_PREC_FP32) enqueue_step_t<float>(h, in, dt_host);
  else enqueue_step_t<double>(h, in, dt_host);
}

static int read_dev(const af_handle* h, DevState* ds) {
  HIP_OK(hipMemcpyAsync(ds, h->dev, sizeof(*ds), hipMemcpyDeviceToHost, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  return AF_OK;
}

static const char* err_text(int code) {
  switch (code) {
    case ERR_NONPHYS: return "non-positive density or pressure";
    case ERR_CFL: return "time step too large: an evolution circle leaves its cells";
    default: return "device error";
  }
}

extern "C" int af_step(af_handle* h, double dt) {
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_step: NULL handle");
  if (!h->has_state) return fail(h, AF_ERR_INVALID_ARG, "af_step: no state set");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(h, AF_ERR_INVALID_ARG, "af_step: dt must be > 0");
  DevState ds;
  int e = read_dev(h, &ds);
  if (e) return e;
  if (ds.err) {
    ds.err = 0;
    HIP_OK(hipMemcpyAsync(&h->dev->err, &ds.err, sizeof(int), hipMemcpyHostToDevice, h->stream), h);
  }
  const long long before = ds.steps;
  enqueue_step(h, h->cur, dt);
  HIP_OK(hipGetLastError(), h);
  if ((e = read_dev(h, &ds))) return e;
  if (h->timing) collect_timing(h, ds.err ? 0 : 1);
  if (ds.err) return fail(h, ds.err, std::string("af_step: ") + err_text(ds.err));
  if (ds.steps != before + 1) return fail(h, AF_ERR_DEVICE, "af_step: step did not commit");
  h->cur ^= 1;
  return AF_OK;
}

extern "C" int af_run(af_handle* h, double t_end, double cfl, int64_t max_steps,
                      double* t_reached, int64_t* steps_taken) {
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_run: NULL handle");
  if (!h->has_state) return fail(h, AF_ERR_INVALID_ARG, "af_run: no state set");
  if (!(cfl > 0.0) || !(cfl < 0.5)) return fail(h, AF_ERR_INVALID_ARG, "af_run: cfl must be in (0, 0.5)");
  if (std::isnan(t_end)) return fail(h, AF_ERR_INVALID_ARG, "af_run: t_end is NaN");
  DevState ds;
  int e = read_dev(h, &ds);
  if (e) return e;
  const long long steps0 = ds.steps;
  ds.err = 0;
  ds.t_end = t_end;
  ds.cfl = cfl;
  ds.smax[0] = ds.smax[1] = 0ull;
  ds.done_blocks = 0;
  HIP_OK(hipMemcpyAsync(h->dev, &ds, sizeof(ds), hipMemcpyHostToDevice, h->stream), h);
  {
    const Params P = make_params(h);
    const int c = h->cur;
    hipLaunchKernelGGL(k_cfl, dim3(1024), dim3(256), 0, h->stream, P, (const double*)h->A[c],
                       (const double*)h->K[c], (const double*)h->X[c], (const double*)h->Y[c],
                       h->dev, c);
    HIP_OK(hipGetLastError(), h);
  }
  long long done = 0;
  while (true) {
    if ((e = read_dev(h, &ds))) return e;
    const long long executed = ds.steps - steps0;
    if (h->timing) collect_timing(h, executed - done);
    h->cur = (int)((h->cur + (executed - done)) & 1);
    done = executed;
    if (ds.err) {
      if (t_reached) *t_reached = ds.t;
      if (steps_taken) *steps_taken = done;
      return fail(h, ds.err, std::string("af_run: ") + err_text(ds.err));
    }
    if (!(ds.t < t_end) || (max_steps > 0 && done >= max_steps)) break;
    long long k = h->graph_steps > 0 ? h->graph_steps : 8;
    if (max_steps > 0) k = std::min<long long>(k, max_steps - done);
    if (h->cur == 1 && h->graph_steps > 0 && !h->timing) k = 1;  // graphs start at buffer 0
    if (!h->timing && k == h->graph_steps && h->graph_steps > 0 && h->cur == 0) {
      if (!h->gexec || h->gexec_steps != k) {
        if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
        hipGraph_t g;
        HIP_OK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), h);
        for (long long s = 0; s < k; ++s) enqueue_step(h, (int)(s & 1), 0.0);
        HIP_OK(hipStreamEndCapture(h->stream, &g), h);
        HIP_OK(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0), h);
        (void)hipGraphDestroy(g);
        h->gexec_steps = (int)k;
      }
      HIP_OK(hipGraphLaunch(h->gexec, h->stream), h);
    } else {
      for (long long s = 0; s < k; ++s) enqueue_step(h, (int)((h->cur + s) & 1), 0.0);
    }
    HIP_OK(hipGetLastError(), h);
  }
  if (t_reached) *t_reached = ds.t;
  if (steps_taken) *steps_taken = done;
  return AF_OK;
}

extern "C" int af_get_timing(const af_handle* h, double* out) {
  if (!h || !out) return fail(h, AF_ERR_INVALID_ARG, "af_get_timing: NULL argument");
  out[0] = h->ms_points;
  out[1] = h->ms_update;
  out[2] = (double)h->timed_steps;
  return AF_OK;
}
