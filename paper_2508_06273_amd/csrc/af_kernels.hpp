// af_kernels.hpp -- kernels of one Active Flux step (gfx950).
//
// One step = three launches (plus the positivity fix-up pass when the limiter is on):
//   k_points : per 8x8 tile of DOF sites, stage the t_n point values of a one-cell halo in
//              LDS, build the cell reconstructions of the 9x9 halo cells (inverse Simpson for
//              the centre value, primitive Simpson average, monomial coefficients), then evolve
//              the tile's own K, X and Y point values to the intermediate and new time levels
//              (wavefront 0: corners; wavefront 1: x-edges, then y-edges), hand DOFs that
//              need the positivity limiter to the fix-up pass, write U^{n+1} and
//              the per-site Simpson-in-time flux sums f(U^n) + 4 f(U^{n+1/2}) + f(U^{n+1}).
//   k_update : per cell, Simpson space-time face fluxes from the site sums and the
//              conservative FP64 update of the cell average (paper eqs. F and 2dfvm);
//   k_commit : one thread advances t and the step counter if the step ran without error.
// The point and update kernels accumulate the largest wave speed of the new state for the next
// step's time step.  With the shock indicators (Algorithm 2, Sec. 3.4) an averaging pass
// (k_avgprim) runs first and the point kernel's indicator variant replaces the default one.
#pragma once
#include "af_device.hpp"

namespace af {

enum { ERR_NONPHYS = -2, ERR_CFL = -3, ERR_SYNC = -4 };
enum { KIND_K = 0, KIND_X = 1, KIND_Y = 2 };
enum { LIN_AF3 = 0, LIN_AVG = 1, LIN_SIMPLE = 2 };
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_WALL = 2, BC_INFLOW = 3 };

constexpr int TILE = 8;        // sites per tile edge
constexpr int HS = TILE + 2;   // halo sites per edge (local -1 .. TILE)
constexpr int HC = TILE + 1;   // halo cells per edge (local -1 .. TILE-1)
constexpr int NS = HS * HS;    // 100
constexpr int NC = HC * HC;    // 81
// LDS words (of the bulk type) per halo cell of the monomial coefficients: 4 variables x 8,
// plus one so that lanes reading neighbouring cells fall into different banks.  All the
// coefficients of a cell and of its right neighbour then lie within reach of the
// immediate offsets of one paired LDS read: one address per cell pair, not per coefficient.
constexpr int CS = 4 * 8 + 1;
constexpr int PT_THREADS = 128;  // two wavefronts: corners; edges

// Device-resident step control.
struct DevState {
  double t, dt, t_end, cfl;
  unsigned long long smax[2];  // bit patterns of positive doubles (ordered like integers)
  int err;
  int active;
  int last;   // the running step was cut to land on t_end
  int pad0;
  long long steps;
  long long steps_limit;  // no step runs once steps reaches this
  unsigned long long cnt[8];
  unsigned int fix_count;  // tiles listed for the positivity fix-up pass of this step
  unsigned int pad2;
  int cur;                 // batched grids: buffer index of the current state
  int pad1;
};

struct Params {
  int nx, ny, nkx, nky, per_x, per_y;
  int tiles_x, tiles_y;
  double dx, dy, idx, idy, gamma, hmin;
  double g1inv, aspect;  // 1 / (gamma - 1) and dx / dy, formed on the host
  int mode, correction, limiter, pad;
  long long pA, sA;  // pitch and variable stride of the cell-average arrays (doubles)
  long long pP, sP;  // pitch and variable stride of the point-value arrays
  long long pF, sF;  // pitch and variable stride of the flux-sum arrays (doubles)
  int bc[4];         // boundary kind per side (left, right, bottom, top): BC_*
  double inflow[4][4];  // primitive inflow state per side (sides of kind BC_INFLOW)
  int tsw, shock;    // Algorithm 2; the shock-indicator blend of Sec. 3.4
  long long pU, sU;  // pitch and variable stride of the padded primitive averages
};

// Point values are stored in FP64 in both precisions (the bulk type only sets the arithmetic
// of the evolution operators).
struct Bufs {
  const double* A_in;
  double* A_out;
  const double* K_in;
  const double* X_in;
  const double* Y_in;
  double* K_out;
  double* X_out;
  double* Y_out;
  double* FK;  // 8 variables: f sums then g sums
  double* FX;  // 4: f sums
  double* FY;  // 4: g sums
  // positivity fix-up: per tile 3 lane masks (K, X, Y) and a listed flag; list of tiles
  // (numbered from tile_base), and its length
  unsigned long long* fix_mask;
  int* fix_list;
  unsigned int* fix_count;
  int tile_base;
  // primitive Simpson averages of the cells -2 .. nx+1 x -2 .. ny+1 (cell (i, j) at
  // (j + 2) * pU + i + 2), written before the point kernel when an indicator is on
  double* UB;
};

// Device-resident descriptor of a grid: geometry and options, and the buffers for each of the
// two buffer indices (t_n state in buffer `cur`, t_n+1 in `cur ^ 1`).  The point kernels read it
// through a pointer: passed by value, the parameters fill the scalar registers and spill.
struct GridDesc {
  Params P;
  Bufs B[2];
  int tile_base;  // batched grids: first global tile of the grid
};

// Periodic index of a (possibly ghost) cell or grid line, i >= -n.  The common case needs no
// integer division.
__device__ __forceinline__ int wrap_per(int i, int n) {
  if (i < 0) return i + n;
  if (i >= n) {
    i -= n;
    if (i >= n) i %= n;  // grids narrower than a tile
  }
  return i;
}
__device__ __forceinline__ int wrap_line(int i, int n, int per) {
  if (per) return wrap_per(i, n);
  return i < 0 ? 0 : (i > n ? n : i);
}

// Ghost data (Sec. 4 and 4.3).  map_axis gives, for a possibly ghost index i on an axis of n
// cells (LINE: the grid lines 0..n, else the cells 0..n-1), the index of the stored value that
// supplies it and, in `side`, the side whose rule then applies (-1: none, 0: low, 1: high).
// Periodic: wrap.  Outflow and inflow: the nearest boundary value (inflow then replaces it).
// Wall: the mirror image about the boundary line (line n - k <-> n + k, cell n - 1 - k <->
// n + k).  Indices stay in range for any i (grids narrower than a tile).
template <bool LINE>
__device__ __forceinline__ int map_axis(int i, int n, int per, int lo, int hi, int& side) {
  side = -1;
  if (per) return wrap_per(i, n);
  const int last = LINE ? n : n - 1;
  if (i < 0) {
    side = 0;
    i = (lo == BC_WALL) ? (LINE ? -i : -1 - i) : 0;
  } else if (i > last) {
    side = 1;
    i = (hi == BC_WALL) ? (LINE ? 2 * n - i : 2 * n - 1 - i) : last;
  }
  return i < 0 ? 0 : (i > last ? last : i);
}

// Kind and inflow state of side s (0 left, 1 right, 2 bottom, 3 top), by selects: indexing the
// kernel parameters with a runtime value makes the compiler copy them to scratch memory.
__device__ __forceinline__ int side_kind(const Params& P, int s) {
  return s == 0 ? P.bc[0] : (s == 1 ? P.bc[1] : (s == 2 ? P.bc[2] : P.bc[3]));
}
__device__ __forceinline__ double side_inflow(const Params& P, int s, int v) {
  return s == 0 ? P.inflow[0][v]
                : (s == 1 ? P.inflow[1][v] : (s == 2 ? P.inflow[2][v] : P.inflow[3][v]));
}

// Ghost rules on a value fetched through map_axis (sx, sy: the sides that apply, -1: none):
// solid walls first (the normal velocity, or momentum, negated), then inflow (the side's state
// replaces a primitive value; the y side's if both apply).
__device__ __forceinline__ void apply_sides(const Params& P, int sx, int sy, double o[4]) {
  if (sx >= 0 && side_kind(P, sx) == BC_WALL) o[1] = -o[1];
  if (sy >= 0 && side_kind(P, 2 + sy) == BC_WALL) o[2] = -o[2];
  if (sx >= 0 && side_kind(P, sx) == BC_INFLOW) {
#pragma unroll
    for (int v = 0; v < 4; ++v) o[v] = side_inflow(P, sx, v);
  }
  if (sy >= 0 && side_kind(P, 2 + sy) == BC_INFLOW) {
#pragma unroll
    for (int v = 0; v < 4; ++v) o[v] = side_inflow(P, 2 + sy, v);
  }
}

// Is side `side` of axis `axis` an inflow side?
__device__ __forceinline__ bool inflow_side(const Params& P, int axis, int side) {
  return side >= 0 && side_kind(P, 2 * axis + side) == BC_INFLOW;
}

// Does a DOF of kind KIND at (i, j) lie on a solid-wall line?
template <int KIND>
__device__ __forceinline__ bool on_wall(const Params& P, int i, int j) {
  bool w = false;
  if (KIND != KIND_Y)
    w = w || (i == 0 && P.bc[0] == BC_WALL) || (i == P.nx && P.bc[1] == BC_WALL);
  if (KIND != KIND_X)
    w = w || (j == 0 && P.bc[2] == BC_WALL) || (j == P.ny && P.bc[3] == BC_WALL);
  return w;
}

// Errors are negative; when several DOFs fail in one step the most negative code wins
// (AF_ERR_CFL = -3 before AF_ERR_NONPHYSICAL = -2), independent of the order of the waves.
__device__ __forceinline__ void set_err(DevState* d, int code) { atomicMin(&d->err, code); }

__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

// Max of a positive double into *target (bit patterns of positive doubles order like
// unsigned integers).  The current value is read first: once the maximum is reached almost no
// block issues the atomic, so thousands of blocks do not serialise on one address.
__device__ __forceinline__ void atomic_max_pos(unsigned long long* target, double m) {
  if (!(m > 0.0)) return;
  const unsigned long long b = dbits(m);
  if (b > __hip_atomic_load(target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(target, b);
}

// Block-wide max of a non-negative double, at most one atomic per block.
__device__ __forceinline__ void block_max_atomic(double v, unsigned long long* target,
                                                 double* red) {
  for (int off = 32; off > 0; off >>= 1) v = mx(v, __shfl_xor(v, off, 64));
  const int w = threadIdx.x / 64 + (threadIdx.y * blockDim.x) / 64;
  const int lane = (threadIdx.x + threadIdx.y * blockDim.x) & 63;
  if (lane == 0) red[w] = v;
  __syncthreads();
  const int nw = (blockDim.x * blockDim.y + 63) / 64;
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    double m = red[0];
    for (int k = 1; k < nw; ++k) m = mx(m, red[k]);
    atomic_max_pos(target, m);
  }
}

// ------------------------------------------------------------------------------------------
// Shared memory of a point tile.
// ------------------------------------------------------------------------------------------
template <class R> struct Smem {
  double c0[4 * NC];  // centre values U_c (constant monomial coefficient) [var][cell]
  R ch[NC * CS];      // other monomial coefficients c_01 .. c_22 [cell][var][coef-1]
  double ub[4 * NC];  // primitive Simpson averages [var][cell]
  double sk[4 * NS];  // t_n point values [var][site], local site (a,b) -> (a+1) + (b+1)*HS
  double sx[4 * NS];
  double sy[4 * NS];
  double red[4];
};

// Indicators of a tile (Algorithm 2, Sec. 3.4): the primitive averages of the ring of cells
// -2 .. TILE around it, theta of its x-edges (sites 0..TILE-1 x -1..TILE-1) and y-edges
// (-1..TILE-1 x 0..TILE-1), and the transonic flags of the corners 0..TILE x 0..TILE.  The ring
// cells -1 .. TILE-1 are the halo cells, whose averages live in Smem::ub; `outer` holds the
// layer around them.
constexpr int RC = TILE + 3;  // ring cells per edge (local -2 .. TILE)
constexpr int NR = RC * RC;
constexpr int NO = NR - NC;   // outer layer: 4 (TILE + 2) cells
struct Ind {
  double outer[4 * NO];
  double thx[TILE * (TILE + 1)];
  double thy[(TILE + 1) * TILE];
  unsigned char flag[(TILE + 1) * (TILE + 1)];
};
// outer-layer index of ring cell (a, b): bottom row, top row, then the left and right columns
__device__ __forceinline__ int oidx(int a, int b) {
  if (b == -2) return a + 2;
  if (b == TILE) return RC + a + 2;
  return 2 * RC + (a == -2 ? 0 : TILE + 1) + (b + 1);
}
__device__ __forceinline__ int thx_idx(int a, int b) { return a + (b + 1) * TILE; }
__device__ __forceinline__ int thy_idx(int a, int b) { return (a + 1) + b * (TILE + 1); }
__device__ __forceinline__ int flag_idx(int a, int b) { return a + b * (TILE + 1); }

__device__ __forceinline__ int sidx(int a, int b) { return (a + 1) + (b + 1) * HS; }
__device__ __forceinline__ int cidx(int a, int b) { return (a + 1) + (b + 1) * HC; }

// idx = 1/dx; hy = dy / (2 dx): half a cell in y in units of dx (the local frame of the circle
// integrals uses dx in both directions).
// An LDS pointer whose value the compiler cannot see through (p must point into LDS: it is
// converted to the LDS address space).  Reads at constant offsets from it fold the offsets into
// the LDS instructions; from a visible base computation the compiler instead rebuilds the full
// address for every read.
template <class T> __device__ __forceinline__ const T* lds_base(const T* p) {
  auto q = (__attribute__((address_space(3))) const T*)p;
  asm("" : "+v"(q));
  return (const T*)q;
}

template <class R> struct Geo {
  R idx, hy, gamma, half_h, dx;
};

// a / b in the bulk precision: IEEE division in FP64, hardware reciprocal (1 ulp) in FP32
template <class R> __device__ __forceinline__ R qdiv(R a, R b) { return a / b; }
template <> __device__ __forceinline__ float qdiv<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}

// ------------------------------------------------------------------------------------------
// EG2 at one DOF.  cb: LDS index of the lower-left cell around the DOF (K: cell (a-1,b-1);
// X: cell (a-1,b); Y: cell (a,b-1)); tau: the evolution time, itau = 1 / tau (the FP64 path
// forms 1 / (c' tau / dx) from it without a division).  Returns the deviation dU = EG2[U] - lin.
// ------------------------------------------------------------------------------------------
template <class R, int KIND>
__device__ __forceinline__ int eg2(const Smem<R>& S, int cb, const double lin64[4], R tau,
                                   R itau, const Geo<R>& G, R dU[4]) {
  using MA = Math<R>;
  // the coefficients of the lower-left cell and of the cell above it; their right neighbours
  // are constant offsets from them
  const R* __restrict__ chc = lds_base(S.ch + cb * CS);
  const R* __restrict__ chu = lds_base(S.ch + (cb + HC) * CS);
  const double* __restrict__ c0 = S.c0;
  const R rp = R(lin64[0]), up = R(lin64[1]), vp = R(lin64[2]), pp = R(lin64[3]);
  if (!admissible(rp, pp)) return ERR_NONPHYS;
  const R irho = qdiv(R(1), rp);
  const R c2 = G.gamma * pp * irho;
  R c, ic;
  if constexpr (sizeof(R) == 8) {
    ic = ::rsqrt(c2);  // 1/c without a square root and a division
    c = c2 * ic;
  } else {
    c = MA::sqrt_(c2);
    ic = qdiv(R(1), c);
  }
  if ((mx(absr(up), absr(vp)) + c) * tau >= G.half_h) return ERR_CFL;
  // foot point offset and circle radius in units of dx
  const R px = -up * tau * G.idx, py = -vp * tau * G.idx;
  const R ar = c * tau * G.idx;
  const R hy = G.hy;
  const R cMx = clamp1(up * ic), cMy = clamp1(vp * ic);
  const R pi = R(kPi);
  // deviation of a cell's centre value from the linearisation state, formed in FP64
  auto dev0 = [&](int var, int cell) { return R(c0[var * NC + cell] - lin64[var]); };
  Acc<R> A = {R(0), R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
  Mom<R> Mf;
  full_moments(Mf, ar);

  if constexpr (KIND == KIND_K) {
    // corner: the lower-left cell's polynomial P_LL on the full circle, plus (P_LR - P_LL) on
    // the right half (cos > u'/c'), (P_UL - P_LL) on the upper half (sin > v'/c') and
    // (P_UR - P_UL - P_LR + P_LL) on their intersection; in every cell the terms sum to the
    // cell's own polynomial.  The two halves are symmetric arcs (half their moments vanish);
    // only the upper-right arc set needs the general moments.
    const R sxx = MA::sqrt_(mx(R(0), R(1) - cMx * cMx));
    const R syy = MA::sqrt_(mx(R(0), R(1) - cMy * cMy));
    const R al = MA::acos_cs(cMx, sxx), be = MA::asin_cs(cMy, syy);
    const R Ly = pi - R(2) * be;
    // end points of the arcs on the circle of radius ar (the moments are those of that circle)
    const R cxa = ar * cMx, sxa = ar * sxx, sya = ar * syy, cya = ar * cMy, a2 = ar * ar;
    Mom<R> Mq;
    {
      // upper-right arc set: (-al, al) cap (be, pi - be), pieces for the shifts 0 and -2 pi
      Br<R> B;
      br_zero(B);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const R sh = t ? R(-2 * kPi) : R(0);
        const R lo2 = be + sh, hi2 = pi - be + sh;
        const bool l1 = -al >= lo2, h1 = al <= hi2;
        const R lo = l1 ? -al : lo2, hi = h1 ? al : hi2;
        const R Ca = l1 ? cxa : sya, Sa = l1 ? -sxa : cya;
        const R Cb = h1 ? cxa : -sya, Sb = h1 ? sxa : cya;
        br_piece(B, Ca, Sa, Cb, Sb, hi - lo);
      }
      moments(B, a2, Mq);
    }
    const int cLL = cb, cLR = cb + 1, cUL = cb + HC, cUR = cb + HC + 1;
    const R xl = px + R(0.5), xr = px - R(0.5), yb = py + hy, yt = py - hy;
    Mom<R> Mx, My;
    moments_sym_x(cxa, sxa, al, a2, Mx);
    moments_sym_y(sya, cya, Ly, a2, My);
#pragma unroll
    for (int var = 1; var < 4; ++var) {
      R t[9], r[9], w[9];
      circle_shift(dev0(var, cLL), chc + var * 8, 1, xl, yb, t);
      circle_shift(dev0(var, cLR), chc + CS + var * 8, 1, xr, yb, r);
#pragma unroll
      for (int i = 0; i < 9; ++i) w[i] = r[i] - t[i];  // P_LR - P_LL
      if (var == 3) { contract_p<3>(t, Mf, A); contract_p<1>(w, Mx, A); }
      if (var == 1) { contract_u<3>(t, Mf, A); contract_u<1>(w, Mx, A); }
      if (var == 2) { contract_v<3>(t, Mf, A); contract_v<1>(w, Mx, A); }
      circle_shift(dev0(var, cUL), chu + var * 8, 1, xl, yt, w);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const R d = w[i] - t[i];  // P_UL - P_LL
        w[i] = d;
        r[i] += d;  // P_LR + P_UL - P_LL
      }
      if (var == 3) contract_p<2>(w, My, A);
      if (var == 1) contract_u<2>(w, My, A);
      if (var == 2) contract_v<2>(w, My, A);
      circle_shift(dev0(var, cUR), chu + CS + var * 8, 1, xr, yt, w);
#pragma unroll
      for (int i = 0; i < 9; ++i) w[i] -= r[i];  // P_UR - P_UL - P_LR + P_LL
      if (var == 3) contract_p<0>(w, Mq, A);
      if (var == 1) contract_u<0>(w, Mq, A);
      if (var == 2) contract_v<0>(w, Mq, A);
    }
  } else {
    // edge: the low-side cell on the full circle plus, on the high-side arc, the difference of
    // the two cell polynomials (it vanishes on the grid line by continuity).  The high-side
    // arc is symmetric, so half of its moments vanish.
    Mom<R> M;
    if constexpr (KIND == KIND_X) {
      const R sxx = MA::sqrt_(mx(R(0), R(1) - cMx * cMx));
      moments_sym_x(ar * cMx, ar * sxx, MA::acos_cs(cMx, sxx), ar * ar, M);
    } else {
      const R syy = MA::sqrt_(mx(R(0), R(1) - cMy * cMy));
      moments_sym_y(ar * syy, ar * cMy, pi - R(2) * MA::asin_cs(cMy, syy), ar * ar, M);
    }
    const int cl = cb, chh = cb + (KIND == KIND_X ? 1 : HC);
    const R xl = (KIND == KIND_X) ? px + R(0.5) : px;
    const R yl = (KIND == KIND_X) ? py : py + hy;
    const R xh = (KIND == KIND_X) ? px - R(0.5) : px;
    const R yh = (KIND == KIND_X) ? py : py - hy;
    constexpr int SYM = (KIND == KIND_X) ? 1 : 2;
#pragma unroll
    for (int var = 1; var < 4; ++var) {
      R lo[9], hi[9];
      const R dl = dev0(var, cl);
      circle_shift(dl, chc + var * 8, 1, xl, yl, lo);
      circle_shift(dev0(var, chh), (KIND == KIND_X ? chc + CS : chu) + var * 8, 1, xh, yh, hi);
#pragma unroll
      for (int i = 0; i < 9; ++i) hi[i] -= lo[i];
      if (var == 3) { contract_p<3>(lo, Mf, A); contract_p<SYM>(hi, M, A); }
      if (var == 1) { contract_u<3>(lo, Mf, A); contract_u<SYM>(hi, M, A); }
      if (var == 2) { contract_v<3>(lo, Mf, A); contract_v<SYM>(hi, M, A); }
    }
  }

  // values at the foot point P'
  const int sxP = (KIND == KIND_Y) ? 0 : (up <= R(0) ? 1 : 0);
  const int syP = (KIND == KIND_X) ? 0 : (vp <= R(0) ? 1 : 0);
  const int cellP = cb + sxP + syP * HC;
  const R* chP = (syP ? chu : chc) + sxP * CS;
  const R xiP = (KIND == KIND_Y) ? px : px + R(0.5) - R(sxP);
  const R etaP = (KIND == KIND_X) ? py : py + (syP ? -hy : hy);
  const R drP = poly_eval(dev0(0, cellP), chP, 1, xiP, etaP);
  const R dpP = poly_eval(dev0(3, cellP), chP + 3 * 8, 1, xiP, etaP);

  // undo the moment scaling: first-order integrals carry a factor ar, second-order ar^2
  // 1 / ar: in FP64 from 1/c and the caller's 1/tau (no division), in FP32 by the hardware
  // reciprocal
  const R ia = (sizeof(R) == 8) ? ic * itau * G.dx : qdiv(R(1), ar), ia2 = ia * ia;
  const R IpC = A.IpC * ia, IpS = A.IpS * ia, Jr = A.Jr * ia;
  const R Ju = R(2) * A.Ua * ia2 - R(0.5) * A.Ub;
  const R Jv = R(2) * A.Va * ia2 - R(0.5) * A.Vb;
  const R ipi = R(1.0 / kPi);
  const R ic2 = ic * ic;
  const R irc = ic * irho;
  const R rc = rp * c;
  dU[0] = drP - R(2) * dpP * ic2 + ipi * (A.Ip * ic2 - rp * ic * Jr);
  dU[1] = ipi * (Ju - IpC * irc);
  dU[2] = ipi * (Jv - IpS * irc);
  dU[3] = -dpP + ipi * (A.Ip - rc * Jr);
  return 0;
}

// ------------------------------------------------------------------------------------------
// EG1 on piecewise constant data (the primitive cell averages), used by the positivity
// limiter.  Low moments only.  A foot point on a grid line takes the mean of the cells whose
// closure contains it.
// ------------------------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void low_moments(R Ca, R Sa, R Cb, R Sb, R L, R m[6]) {
  // m: M00, M10, M01, M20, M11, M02
  m[0] = L;
  m[1] = Sb - Sa;
  m[2] = Ca - Cb;
  const R cs = Cb * Sb - Ca * Sa;
  m[3] = R(0.5) * (cs + L);
  m[4] = R(-0.5) * (Cb * Cb - Ca * Ca);
  m[5] = R(0.5) * (L - cs);
}

template <class R>
__device__ __forceinline__ void low_piece(R a1, R c1a, R s1a, R b1, R c1b, R s1b, R a2, R c2a,
                                          R s2a, R b2, R c2b, R s2b, R m[6]) {
  const bool lo1 = a1 >= a2, hi1 = b1 <= b2;
  const R lo = lo1 ? a1 : a2, hi = hi1 ? b1 : b2;
  const R L = hi - lo;
  const R keep = L > R(0) ? R(1) : R(0);
  low_moments(lo1 ? c1a : c2a, lo1 ? s1a : s2a, hi1 ? c1b : c2b, hi1 ? s1b : s2b,
              L * keep, m);
#pragma unroll
  for (int k = 0; k < 6; ++k) m[k] *= keep;
}

template <class R, int KIND>
__device__ __forceinline__ int eg1_pc(const double* __restrict__ ub, int cb, const double* lin64,
                                      R tau, const Geo<R>& G, R dU[4]) {
  using MA = Math<R>;
  const R rp = R(lin64[0]), up = R(lin64[1]), vp = R(lin64[2]), pp = R(lin64[3]);
  if (!admissible(rp, pp)) return ERR_NONPHYS;
  const R c = MA::sqrt_(G.gamma * pp / rp);
  if ((mx(absr(up), absr(vp)) + c) * tau >= G.half_h) return ERR_CFL;
  const R ic = R(1) / c;
  const R cMx = clamp1(up * ic), cMy = clamp1(vp * ic);
  const R sxx = MA::sqrt_(mx(R(0), R(1) - cMx * cMx));
  const R syy = MA::sqrt_(mx(R(0), R(1) - cMy * cMy));
  const R al = MA::acos_cs(cMx, sxx), be = MA::asin_cs(cMy, syy);
  R Ip = 0, IpC = 0, IpS = 0, Jr = 0, Ku = 0, Kv = 0;
  // The data are constant on the quadrants (K) or halves (X, Y) around the DOF.  As for EG2,
  // split them into the low-side value on the full circle plus differences on the right half,
  // the upper half and their intersection: the full circle's moments are closed form, and only
  // the half circles (one arc each) and the quadrant need arc moments.
  auto piece = [&](double dp, double du, double dv, const R m[6]) {
    const R p = R(dp), u = R(du), v = R(dv);
    Ip += p * m[0];
    IpC += p * m[1];
    IpS += p * m[2];
    Jr += u * m[1] + v * m[2];
    Ku += u * (R(3) * m[3] - m[0]) + R(3) * v * m[4];
    Kv += R(3) * u * m[4] + v * (R(3) * m[5] - m[0]);
  };
  auto dev = [&](int cell, int var) { return ub[var * NC + cell] - lin64[var]; };
  const R twopi = R(2 * kPi), pi = R(kPi);
  const R mfull[6] = {twopi, R(0), R(0), pi, R(0), pi};
  R mr[6], mu[6];
  if (KIND != KIND_Y) low_moments(cMx, -sxx, cMx, sxx, R(2) * al, mr);   // right: (-al, al)
  if (KIND != KIND_X) low_moments(syy, cMy, -syy, cMy, pi - R(2) * be, mu);  // up: (be, pi-be)
  const int c00 = cb;                                 // low-side cell (left / lower)
  const int c10 = cb + 1, c01 = cb + HC, c11 = cb + HC + 1;
  piece(dev(c00, 3), dev(c00, 1), dev(c00, 2), mfull);
  if constexpr (KIND == KIND_X) {
    piece(dev(c10, 3) - dev(c00, 3), dev(c10, 1) - dev(c00, 1), dev(c10, 2) - dev(c00, 2), mr);
  } else if constexpr (KIND == KIND_Y) {
    piece(dev(c01, 3) - dev(c00, 3), dev(c01, 1) - dev(c00, 1), dev(c01, 2) - dev(c00, 2), mu);
  } else {
    piece(dev(c10, 3) - dev(c00, 3), dev(c10, 1) - dev(c00, 1), dev(c10, 2) - dev(c00, 2), mr);
    piece(dev(c01, 3) - dev(c00, 3), dev(c01, 1) - dev(c00, 1), dev(c01, 2) - dev(c00, 2), mu);
    // the upper right quadrant: (-al, al) and (be, pi - be), up to one turn apart
    R mq[6] = {0, 0, 0, 0, 0, 0};
    for (int k = -1; k <= 1; ++k) {
      R n[6];
      low_piece(-al, cMx, -sxx, al, cMx, sxx, be + R(k) * twopi, syy, cMy,
                pi - be + R(k) * twopi, -syy, cMy, n);
      for (int t = 0; t < 6; ++t) mq[t] += n[t];
    }
    auto d4 = [&](int var) { return ((ub[var * NC + c11] - ub[var * NC + c01]) -
                                     (ub[var * NC + c10] - ub[var * NC + c00])); };
    piece(d4(3), d4(1), d4(2), mq);
  }
  // foot point values (mean over the cells whose closure contains P')
  double P[4] = {0, 0, 0, 0};
  {
    const bool onx = (KIND != KIND_Y) && (up == R(0));
    const bool ony = (KIND != KIND_X) && (vp == R(0));
    const int sx0 = (KIND == KIND_Y) ? 0 : (up < R(0) ? 1 : 0);
    const int sy0 = (KIND == KIND_X) ? 0 : (vp < R(0) ? 1 : 0);
    int n = 0;
    for (int ox = 0; ox < 2; ++ox)
      for (int oy = 0; oy < 2; ++oy) {
        const int sx = onx ? ox : sx0, sy = ony ? oy : sy0;
        if ((!onx && ox) || (!ony && oy)) continue;
        const int cell = cb + (KIND == KIND_Y ? 0 : sx) + (KIND == KIND_X ? 0 : sy * HC);
        for (int v = 0; v < 4; ++v) P[v] += ub[v * NC + cell];
        ++n;
      }
    const double inv = 1.0 / n;
    for (int v = 0; v < 4; ++v) P[v] = P[v] * inv - lin64[v];
  }
  const R i2pi = R(0.5 / kPi);
  const R ic2 = ic * ic, irc = ic / rp;
  dU[0] = R(P[0]) - R(P[3]) * ic2 + i2pi * (Ip * ic2 - R(2) * rp * ic * Jr);
  dU[1] = R(0.5) * R(P[1]) + i2pi * (Ku - R(2) * IpC * irc);
  dU[2] = R(0.5) * R(P[2]) + i2pi * (Kv - R(2) * IpS * irc);
  dU[3] = i2pi * (Ip - R(2) * rp * c * Jr);
  return 0;
}

// ------------------------------------------------------------------------------------------
// Lax-Friedrichs point update on the lattice of same-kind DOFs (FP64), the last resort of
// the positivity limiter: a dual cell dx x dy centred at the DOF, Rusanov fluxes with the
// four same-kind neighbours, time increment tau.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void lf_flux(const double UL[4], const double UR[4], int dir,
                                        double gamma, double g1inv, double o[4]) {
  double FL[4], GL[4], FR[4], GR[4], QL[4], QR[4];
  flux_fg(UL, g1inv, FL, GL);
  flux_fg(UR, g1inv, FR, GR);
  p2c(UL, g1inv, QL);
  p2c(UR, g1inv, QR);
  const double sL = __builtin_fabs(UL[1 + dir]) + __builtin_sqrt(gamma * UL[3] / UL[0]);
  const double sR = __builtin_fabs(UR[1 + dir]) + __builtin_sqrt(gamma * UR[3] / UR[0]);
  const double al = mx(sL, sR);
  for (int v = 0; v < 4; ++v) {
    const double fl = dir ? GL[v] : FL[v], fr = dir ? GR[v] : FR[v];
    o[v] = 0.5 * (fl + fr) - 0.5 * al * (QR[v] - QL[v]);
  }
}

__device__ __noinline__ void lf_update(const double* __restrict__ site, int a, int b, double tau,
                                       const Params& P, double out[4]) {
  double U[5][4];
  const int nb[5][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}};
  for (int k = 0; k < 5; ++k)
    for (int v = 0; v < 4; ++v) U[k][v] = site[v * NS + sidx(a + nb[k][0], b + nb[k][1])];
  const double g1inv = P.g1inv;
  double Fe[4], Fw[4], Gn[4], Gs[4], Q0[4], Q[4];
  lf_flux(U[0], U[1], 0, P.gamma, g1inv, Fe);
  lf_flux(U[2], U[0], 0, P.gamma, g1inv, Fw);
  lf_flux(U[0], U[3], 1, P.gamma, g1inv, Gn);
  lf_flux(U[4], U[0], 1, P.gamma, g1inv, Gs);
  p2c(U[0], g1inv, Q0);
  for (int v = 0; v < 4; ++v)
    Q[v] = Q0[v] - tau * P.idx * (Fe[v] - Fw[v]) - tau * P.idy * (Gn[v] - Gs[v]);
  c2p_plain(Q, P.gamma - 1.0, out);
}

}  // namespace af
