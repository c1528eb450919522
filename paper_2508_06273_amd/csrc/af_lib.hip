// af_lib.hip -- kernels and host runtime of libaf.so (C ABI in include/af.h).
//
// Fully discrete third-order Active Flux method for the 2D Euler equations, arXiv 2508.06273.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "af.h"
#include "af_host.hpp"
#include "af_step.hpp"

namespace af {

// ------------------------------------------------------------------------------------------
// Kernel 1: point values, one workgroup per 8x8-site tile (XCD-aware tile order).  The _ind
// variants add the indicators of Algorithm 2 and Sec. 3.4.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(PT_THREADS) AF_ATTR_F32
void k_points_f32(const GridDesc* __restrict__ d, DevState* dev, double dt_host, int slot) {
  __shared__ Smem<float> S;
  const Params& P = d->P;
  const Bufs& B = d->B[slot];
  points_body<float>(S, nullptr, P, B, dev, dt_host, slot,
                     tile_of_block(blockIdx.x, P.tiles_x * P.tiles_y),
                     blockIdx.x == 0);
}
__global__ __launch_bounds__(PT_THREADS) AF_ATTR_F64
void k_points_f64(const GridDesc* __restrict__ d, DevState* dev, double dt_host, int slot) {
  __shared__ Smem<double> S;
  const Params& P = d->P;
  const Bufs& B = d->B[slot];
  points_body<double>(S, nullptr, P, B, dev, dt_host, slot,
                      tile_of_block(blockIdx.x, P.tiles_x * P.tiles_y),
                      blockIdx.x == 0);
}
template <class R>
__global__ __launch_bounds__(PT_THREADS) void k_points_ind(const GridDesc* __restrict__ d,
                                                           DevState* dev, double dt_host,
                                                           int slot) {
  __shared__ Smem<R> S;
  __shared__ Ind I;
  const Params& P = d->P;
  const Bufs& B = d->B[slot];
  points_body<R, true>(S, &I, P, B, dev, dt_host, slot,
                       tile_of_block(blockIdx.x, P.tiles_x * P.tiles_y),
                       blockIdx.x == 0);
}

// Primitive Simpson averages of the cells -2 .. nx+1 x -2 .. ny+1 for the indicators, one
// thread per cell (row-major, coalesced).
__global__ __launch_bounds__(256) void k_avgprim(Params P, Bufs B) {
  const int W = P.nx + 4;
  const long long n = (long long)W * (P.ny + 4);
  for (long long e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const int i = (int)(e % W) - 2, j = (int)(e / W) - 2;
    double ub[4];
    prim_average(P, B, i, j, ub);
    const long long o = (long long)(j + 2) * P.pU + (i + 2);
#pragma unroll
    for (int v = 0; v < 4; ++v) B.UB[v * P.sU + o] = ub[v];
  }
}

// Positivity fix-up pass over the tiles the point kernel listed.  Cheap when the list is empty.
template <class R, bool IND>
__device__ __forceinline__ void fixup_body(Smem<R>& S, Ind* I, const Params& P, const Bufs& B,
                                           DevState* dev, int slot) {
  __shared__ unsigned long long mask[3];
  __shared__ int s_run;
  __shared__ unsigned int s_n;
  __shared__ double s_dt;
  if (threadIdx.x == 0) {
    s_run = !dev->err && dev->active;
    s_n = *B.fix_count;
    s_dt = dev->dt;
  }
  __syncthreads();
  const unsigned int n = s_n;
  double speed = 0.0;
  for (unsigned int k = blockIdx.x; k < n; k += gridDim.x)
    fixup_tile<R, IND>(S, I, P, B, dev, B.fix_list[k], s_dt, s_run != 0, mask, speed);
  if (n > blockIdx.x) block_max_atomic(speed, &dev->smax[slot ^ 1], S.red);
}
__global__ __launch_bounds__(PT_THREADS) void k_fixup_f32(const GridDesc* __restrict__ d,
                                                         DevState* dev, int slot) {
  __shared__ Smem<float> S;
  fixup_body<float, false>(S, nullptr, d->P, d->B[slot], dev, slot);
}
__global__ __launch_bounds__(PT_THREADS) void k_fixup_f64(const GridDesc* __restrict__ d,
                                                         DevState* dev, int slot) {
  __shared__ Smem<double> S;
  fixup_body<double, false>(S, nullptr, d->P, d->B[slot], dev, slot);
}
template <class R>
__global__ __launch_bounds__(PT_THREADS) void k_fixup_ind(const GridDesc* __restrict__ d,
                                                          DevState* dev, int slot) {
  __shared__ Smem<R> S;
  __shared__ Ind I;
  fixup_body<R, true>(S, &I, d->P, d->B[slot], dev, slot);
}

// ------------------------------------------------------------------------------------------
// Kernel 2: Simpson space-time fluxes and the conservative update of the averages.  Rows of
// cells, 2 UP_THREADS consecutive cells of a row per work item, two neighbouring cells per
// thread (16-byte loads), about one item per workgroup.  Kernel 3 (one thread) then commits
// the step.
// ------------------------------------------------------------------------------------------
// Two waves per SIMD: the register budget lets every load of a cell pair be in flight before
// the first use (this HBM-bound kernel gains more from that than from occupancy).
__global__ __launch_bounds__(UP_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_update(Params P, const double* __restrict__ A_in, double* __restrict__ A_out,
              const double* __restrict__ FK, const double* __restrict__ FX,
              const double* __restrict__ FY, DevState* dev, int slot) {
  __shared__ double red[UP_THREADS / 64];
  const bool run = !dev->err && dev->active;
  const double dt = dev->dt;
  const double lx = dt * P.idx * (1.0 / 36.0), ly = dt * P.idy * (1.0 / 36.0);
  double speed = 0.0;
  bool bad = false;
  if (run) {
    const int chunks_x = (P.nx + 2 * UP_THREADS - 1) / (2 * UP_THREADS);
    const long long nwork = (long long)chunks_x * P.ny;
    for (long long w = blockIdx.x; w < nwork; w += gridDim.x) {
      const int j = (int)(w / chunks_x);
      const int i = (int)(w % chunks_x) * 2 * UP_THREADS + 2 * threadIdx.x;
      if (i < P.nx && !update_pair(P, A_in, A_out, FK, FX, FY, lx, ly, i, j, speed)) bad = true;
    }
  }
  if (bad) set_err(dev, ERR_NONPHYS);
  for (int off = 32; off > 0; off >>= 1) speed = mx(speed, __shfl_xor(speed, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = speed;
  __syncthreads();
  if (threadIdx.x == 0 && run) {
    double m = red[0];
    for (int k = 1; k < UP_THREADS / 64; ++k) m = mx(m, red[k]);
    atomic_max_pos(&dev->smax[slot ^ 1], m);
  }
}

// Flux limiting of the averages (Sec. 3.5), two passes replacing k_update: the face weights
// theta of every cell, then the limited update.  One thread per cell, rows of cells in order.
__global__ __launch_bounds__(256) void k_flux_theta(Params P, const double* __restrict__ A_in,
                                                    const double* __restrict__ FK,
                                                    const double* __restrict__ FX,
                                                    const double* __restrict__ FY,
                                                    double* __restrict__ TH, DevState* dev) {
  if (dev->err || !dev->active) return;
  const double dt = dev->dt;
  const double lx = dt * P.idx * (1.0 / 36.0), ly = dt * P.idy * (1.0 / 36.0);
  const long long n = (long long)P.nx * P.ny, st = (long long)P.ny * P.pA;
  bool bad = false;
  for (long long c = blockIdx.x * 256ll + threadIdx.x; c < n; c += (long long)gridDim.x * 256) {
    const int i = (int)(c % P.nx), j = (int)(c / P.nx);
    double th[4];
    if (!cell_thetas(P, A_in, FK, FX, FY, lx, ly, i, j, th)) {
      bad = true;
      continue;
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) TH[f * st + (long long)j * P.pA + i] = th[f];
  }
  if (bad) set_err(dev, ERR_NONPHYS);
}

__global__ __launch_bounds__(256) void k_update_lim(Params P, const double* __restrict__ A_in,
                                                    double* __restrict__ A_out,
                                                    const double* __restrict__ FK,
                                                    const double* __restrict__ FX,
                                                    const double* __restrict__ FY,
                                                    const double* __restrict__ TH,
                                                    DevState* dev, int slot) {
  __shared__ double red[4];
  __shared__ unsigned int s_lim;
  if (threadIdx.x == 0) s_lim = 0u;
  __syncthreads();
  const bool run = !dev->err && dev->active;
  const double dt = dev->dt;
  const double lx = dt * P.idx * (1.0 / 36.0), ly = dt * P.idy * (1.0 / 36.0);
  const long long n = (long long)P.nx * P.ny;
  double speed = 0.0;
  bool bad = false;
  unsigned nlim = 0;
  if (run) {
    for (long long c = blockIdx.x * 256ll + threadIdx.x; c < n; c += (long long)gridDim.x * 256) {
      const int i = (int)(c % P.nx), j = (int)(c / P.nx);
      if (!update_limited(P, A_in, A_out, FK, FX, FY, TH, lx, ly, i, j, speed, nlim)) bad = true;
    }
  }
  if (bad) set_err(dev, ERR_NONPHYS);
  if (nlim) atomicAdd(&s_lim, nlim);
  block_max_atomic(speed, &dev->smax[slot ^ 1], red);
  if (threadIdx.x == 0 && s_lim) atomicAdd(&dev->cnt[AF_CNT_FLUX], (unsigned long long)s_lim);
}

// Commit of a step (one thread): a step that ran without error advances t and the step
// counter and clears the wave-speed slot of the old state.
__global__ void k_commit(DevState* dev, int slot) {
  dev->fix_count = 0u;
  if (!dev->err && dev->active) {
    dev->t = dev->last ? dev->t_end : dev->t + dev->dt;
    dev->steps += 1;
    dev->smax[slot] = 0ull;
  }
}

// Admissibility of n conserved averages (variable-major, unpadded): sets *bad if any is not.
__global__ void k_check_avg(const double* __restrict__ avg, long long n, double gamma, int* bad) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    double Q[4] = {avg[k], avg[n + k], avg[2 * n + k], avg[3 * n + k]}, U[4];
    c2p_plain(Q, gamma - 1.0, U);
    if (!admissible(U[0], U[3])) atomicOr(bad, 1);
  }
}

// Largest wave speed of the current state (averages and point values) into smax[slot].
__global__ void k_cfl(Params P, const double* __restrict__ A, const double* __restrict__ K,
                      const double* __restrict__ X, const double* __restrict__ Y, DevState* dev,
                      int slot) {
  __shared__ double red[4];
  const double speed = state_speed(P, A, K, X, Y, blockIdx.x * (long long)blockDim.x + threadIdx.x,
                                   (long long)gridDim.x * blockDim.x);
  block_max_atomic(speed, &dev->smax[slot], red);
}

// ------------------------------------------------------------------------------------------
// Scratch memory of af_step_noalloc (no allocation at call time): step control, the grid
// descriptor, the fix-up masks and tile list, and the per-site flux sums, carved out of one file-scope array that
// every GPU the library runs on holds until the process ends.  Host code never passes the
// array's name to a kernel (in host code it is a stand-in, not a device address): it uses the
// address that hipGetSymbolAddress returns for the current device.
// ------------------------------------------------------------------------------------------
constexpr size_t NOALLOC_BYTES = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Write the device descriptor of a single grid (its parameters and the buffers of both buffer
// indices) from kernel arguments: no host copy, so it may be enqueued anywhere on a stream.
__global__ void k_write_desc(GridDesc* d, Params P, Bufs B0, Bufs B1) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    d->P = P;
    d->B[0] = B0;
    d->B[1] = B1;
    d->tile_base = 0;
  }
}

// Reset the step control (zero, no step limit) and clear n fix-up mask words.
__global__ void k_noalloc_init(DevState* dev, unsigned long long* mask, long long n) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t == 0) {
    unsigned long long* w = reinterpret_cast<unsigned long long*>(dev);
    for (size_t k = 0; k < sizeof(DevState) / 8; ++k) w[k] = 0ull;
    dev->steps_limit = LLONG_MAX;
  }
  for (long long k = t; k < n; k += (long long)gridDim.x * blockDim.x) mask[k] = 0ull;
}
static_assert(sizeof(DevState) % 8 == 0, "DevState is cleared as 64-bit words");

}  // namespace af

// ==========================================================================================
// Host runtime
// ==========================================================================================
using namespace af;

std::string g_create_error;

// ------------------------------------------------------------------------------------------
// Domain totals of the conserved variables (af_get_totals): two passes in a fixed order, so
// that the result does not depend on the scheduling: TOTAL_BLOCKS workgroups sum the cells
// b, b + TOTAL_BLOCKS * 256, ... of the row-major cell index (each of its 256 threads a
// strided share, then a fixed-order tree over the workgroup), one workgroup adds the partial
// sums in block order.  FP64 throughout.
namespace {
__global__ __launch_bounds__(256) void k_totals_partial(const double* __restrict__ A, long long pA,
                                                        long long sA, int nx, int ny,
                                                        double* __restrict__ partial) {
  __shared__ double red[4][256];
  const long long n = (long long)nx * ny;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long c = (long long)blockIdx.x * 256 + threadIdx.x; c < n;
       c += (long long)gridDim.x * 256) {
    const long long j = c / nx, i = c - j * nx;
    const long long o = j * pA + i;
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] += A[v * sA + o];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) red[v][threadIdx.x] = s[v];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int v = 0; v < 4; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[4 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}
__global__ void k_totals_final(const double* __restrict__ partial, int nblocks, double area,
                               double* __restrict__ out) {
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[4 * b + threadIdx.x];
    out[threadIdx.x] = s * area;
  }
}
}  // namespace

int reduce_totals(const af_handle* h, hipStream_t stream, const double* A, long long pA,
                  long long sA, int nx, int ny, double area, double* scratch, double* out) {
  hipLaunchKernelGGL(k_totals_partial, dim3(TOTAL_BLOCKS), dim3(256), 0, stream, A, pA, sA, nx,
                     ny, scratch);
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, stream, (const double*)scratch,
                     TOTAL_BLOCKS, area, scratch + 4 * TOTAL_BLOCKS);
  HIP_OK(hipGetLastError(), h);
  HIP_OK(hipMemcpyAsync(out, scratch + 4 * TOTAL_BLOCKS, 4 * sizeof(double),
                        hipMemcpyDeviceToHost, stream), h);
  HIP_OK(hipStreamSynchronize(stream), h);
  return AF_OK;
}

int fail(const af_handle* h, int code, const std::string& msg) {
  if (h) const_cast<af_handle*>(h)->err = msg;
  else g_create_error = msg;
  return code;
}

static Params make_params(const af_handle* h) {
  Params P;
  P.nx = h->nx; P.ny = h->ny; P.nkx = h->nkx; P.nky = h->nky;
  P.per_x = h->per_x; P.per_y = h->per_y;
  P.tiles_x = (h->nkx + TILE - 1) / TILE;
  P.tiles_y = (h->nky + TILE - 1) / TILE;
  P.dx = h->dx; P.dy = h->dy; P.idx = 1.0 / h->dx; P.idy = 1.0 / h->dy;
  P.gamma = h->gamma; P.hmin = std::min(h->dx, h->dy);
  P.g1inv = 1.0 / (h->gamma - 1.0); P.aspect = h->dx / h->dy;
  P.mode = h->mode; P.correction = h->correction; P.limiter = h->limiter; P.pad = 0;
  P.pA = h->pA; P.sA = h->pA * h->ny;
  P.pP = h->pP; P.sP = h->pP * h->nky;
  P.pF = h->pF; P.sF = h->pF * h->nky;
  fill_sides(h, 0, P);
  P.tsw = h->tsw; P.shock = h->shock;
  P.pU = h->pU; P.sU = h->pU * (h->ny + 4);
  return P;
}

void fill_sides(const af_handle* h, int g, Params& P) {
  const Sides& q = h->sides[g];
  for (int s = 0; s < 4; ++s) {
    P.bc[s] = q.bc[s];
    for (int v = 0; v < 4; ++v) P.inflow[s][v] = q.inflow[s][v];
  }
}

static Sides make_sides(const af_bc* bc) {
  Sides q;
  q.bc[0] = bc->left; q.bc[1] = bc->right; q.bc[2] = bc->bottom; q.bc[3] = bc->top;
  return q;
}

// Every inflow side of every grid has its state.
static int check_inflow(af_handle* h, const char* fn) {
  for (size_t g = 0; g < h->sides.size(); ++g)
    for (int s = 0; s < 4; ++s)
      if (h->sides[g].bc[s] == AF_BC_INFLOW && !((h->sides[g].set >> s) & 1u))
        return fail(h, AF_ERR_INVALID_ARG,
                    std::string(fn) + ": no inflow state for side " + std::to_string(s) +
                        " of grid " + std::to_string(g) + " (af_set_inflow)");
  return AF_OK;
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

static int check_grid(const af_grid* grid, const af_bc* bc, const char* fn) {
  const std::string f(fn);
  if (grid->nx < 2 || grid->ny < 2 || grid->nx > (1 << 16) || grid->ny > (1 << 16))
    return fail(nullptr, AF_ERR_INVALID_ARG, f + ": nx, ny must be in [2, 65536]");
  if (!std::isfinite(grid->x0) || !std::isfinite(grid->x1) || !std::isfinite(grid->y0) ||
      !std::isfinite(grid->y1))
    return fail(nullptr, AF_ERR_INVALID_ARG, f + ": domain bounds must be finite");
  if (!(grid->x1 > grid->x0) || !(grid->y1 > grid->y0))
    return fail(nullptr, AF_ERR_INVALID_ARG, f + ": empty domain");
  const double dx = (grid->x1 - grid->x0) / grid->nx, dy = (grid->y1 - grid->y0) / grid->ny;
  if (!std::isfinite(dx) || !std::isfinite(dy) || !(dx >= 1e-150) || !(dy >= 1e-150))
    return fail(nullptr, AF_ERR_INVALID_ARG, f + ": cell size not finite and positive");
  auto okbc = [](int k) { return k >= AF_BC_PERIODIC && k <= AF_BC_INFLOW; };
  if (!okbc(bc->left) || !okbc(bc->right) || !okbc(bc->bottom) || !okbc(bc->top))
    return fail(nullptr, AF_ERR_INVALID_ARG, f + ": unknown boundary kind");
  if ((bc->left == AF_BC_PERIODIC) != (bc->right == AF_BC_PERIODIC) ||
      (bc->bottom == AF_BC_PERIODIC) != (bc->top == AF_BC_PERIODIC))
    return fail(nullptr, AF_ERR_INVALID_ARG, f + ": periodic must pair on an axis");
  return AF_OK;
}

static void destroy_handle(af_handle* h) {
  free_buffers(h);
  batch_destroy(h);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  if (h->dev) (void)hipFree(h->dev);
  if (h->d_desc) (void)hipFree(h->d_desc);
  if (h->d_totals) (void)hipFree(h->d_totals);
  if (h->UB) (void)hipFree(h->UB);
  if (h->TH) (void)hipFree(h->TH);
  if (h->d_flag) (void)hipFree(h->d_flag);
  if (h->stage) (void)hipHostFree(h->stage);
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  delete h;
}

extern "C" int af_create(const af_grid* grid, double gamma, const af_bc* bc, af_handle** out) {
  if (!out) return fail(nullptr, AF_ERR_INVALID_ARG, "af_create: out is NULL");
  *out = nullptr;
  if (!grid || !bc) return fail(nullptr, AF_ERR_INVALID_ARG, "af_create: NULL grid or bc");
  if (int e = check_grid(grid, bc, "af_create")) return e;
  if (!(gamma > 1.0) || !std::isfinite(gamma))
    return fail(nullptr, AF_ERR_INVALID_ARG, "af_create: gamma must be finite and > 1");
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
  h->sides.assign(1, make_sides(bc));
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
  if (e == AF_OK && hipMalloc(&h->d_desc, sizeof(GridDesc)) != hipSuccess)
    e = fail(h, AF_ERR_OOM, "af_create: hipMalloc(desc)");
  if (e != AF_OK) {
    g_create_error = h->err;
    destroy_handle(h);
    return e;
  }
  *out = h;
  return AF_OK;
}

extern "C" int af_create_batch(int32_t n, const af_grid* grids, double gamma, const af_bc* bcs,
                               af_handle** out) {
  if (!out) return fail(nullptr, AF_ERR_INVALID_ARG, "af_create_batch: out is NULL");
  *out = nullptr;
  if (n < 1 || !grids || !bcs)
    return fail(nullptr, AF_ERR_INVALID_ARG, "af_create_batch: need n >= 1 grids and bcs");
  for (int k = 0; k < n; ++k)
    if (int e = check_grid(&grids[k], &bcs[k], "af_create_batch")) return e;
  if (!(gamma > 1.0) || !std::isfinite(gamma))
    return fail(nullptr, AF_ERR_INVALID_ARG, "af_create_batch: gamma must be finite and > 1");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(nullptr, AF_ERR_DEVICE, "af_create_batch: no HIP device");
  af_handle* h = new af_handle();
  h->gamma = gamma;
  for (int k = 0; k < n; ++k) h->sides.push_back(make_sides(&bcs[k]));
  int e = AF_OK;
  if (hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess)
    e = fail(h, AF_ERR_DEVICE, "af_create_batch: hipStreamCreate");
  h->stream = h->own_stream;
  if (e == AF_OK) e = batch_create(n, grids, gamma, bcs, h);
  if (e != AF_OK) {
    g_create_error = h->err;
    destroy_handle(h);
    return e;
  }
  *out = h;
  return AF_OK;
}

extern "C" int32_t af_batch_size(const af_handle* h) {
  if (!h) return 0;
  return h->batch ? batch_count(h) : 1;
}

extern "C" void af_destroy(af_handle* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  destroy_handle(h);
}

extern "C" const char* af_last_error(const af_handle* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

extern "C" int64_t af_dof_count(const af_handle* h) {
  if (!h) return 0;
  if (h->batch) return batch_dof_count(h);
  return (int64_t)h->nx * h->ny + (int64_t)h->nkx * h->nky + (int64_t)h->nkx * h->ny +
         (int64_t)h->nx * h->nky;
}

extern "C" int af_set_option(af_handle* h, int key, int64_t value) {
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_set_option: NULL handle");
  switch (key) {
    case AF_OPT_PRECISION:
      if (value != AF_PREC_FP64 && value != AF_PREC_FP32)
        return fail(h, AF_ERR_INVALID_ARG, "af_set_option: precision must be FP64 or FP32");
      h->prec = (int)value;  // storage is FP64 in both precisions: the state is kept
      break;
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
    case AF_OPT_AUTOTUNE:
      if (value != 0 && value != 1) return fail(h, AF_ERR_INVALID_ARG, "af_set_option: 0 or 1");
      h->autotune = (int)value;
      break;
    case AF_OPT_TRANSONIC:
    case AF_OPT_SHOCK_LIMITER:
      if (value != 0 && value != 1) return fail(h, AF_ERR_INVALID_ARG, "af_set_option: 0 or 1");
      if (value && h->batch) {
        if (int e = batch_alloc_indicators(h)) return e;
      } else if (value && !h->UB) {
        h->pU = (h->nx + 4 + 31) / 32 * 32;
        HIP_OK(hipMalloc(&h->UB, (size_t)4 * h->pU * (h->ny + 4) * sizeof(double)), h);
      }
      if (key == AF_OPT_TRANSONIC) h->tsw = (int)value;
      else h->shock = (int)value;
      break;
    case AF_OPT_FLUX_LIMITER:
      if (value != 0 && value != 1) return fail(h, AF_ERR_INVALID_ARG, "af_set_option: 0 or 1");
      if (value && h->batch)
        return fail(h, AF_ERR_INVALID_ARG,
                    "af_set_option: flux limiting is available on single-grid handles");
      if (value && !h->TH)
        HIP_OK(hipMalloc(&h->TH, (size_t)4 * h->pA * h->ny * sizeof(double)), h);
      h->flux_limiter = (int)value;
      break;
    case AF_OPT_TILE_ORDER:
    case AF_OPT_UPDATE_THREADS:
    case AF_OPT_STEP_KERNEL: {
      if (!h->batch) return fail(h, AF_ERR_INVALID_ARG, "af_set_option: batched handles only");
      int order = 0, threads = 0, kernel = 0;
      batch_get_schedule(h, &order, &threads, &kernel);
      if (value < 0 || value > 4096)
        return fail(h, AF_ERR_INVALID_ARG, "af_set_option: bad schedule value");
      if (key == AF_OPT_TILE_ORDER) order = (int)value;
      else if (key == AF_OPT_UPDATE_THREADS) threads = (int)value;
      else kernel = (int)value;
      return batch_set_schedule(h, order, threads, kernel);
    }
    case AF_OPT_SYNC_TIMEOUT_US: {
      if (!h->batch) return fail(h, AF_ERR_INVALID_ARG, "af_set_option: batched handles only");
      if (int e = batch_set_sync_timeout(h, value)) return e;
      break;  // a captured graph holds the old limit: rebuilt below
    }
    default:
      return fail(h, AF_ERR_INVALID_ARG, "af_set_option: unknown key");
  }
  if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; h->gexec_steps = 0; }
  h->desc_valid = false;
  batch_invalidate(h);
  return AF_OK;
}

extern "C" int af_get_option(const af_handle* h, int key, int64_t* value) {
  if (!h || !value) return fail(h, AF_ERR_INVALID_ARG, "af_get_option: NULL argument");
  int order = 0, threads = 0, kernel = 0;
  switch (key) {
    case AF_OPT_PRECISION: *value = h->prec; return AF_OK;
    case AF_OPT_LINEARISATION: *value = h->mode; return AF_OK;
    case AF_OPT_CORRECTION: *value = h->correction; return AF_OK;
    case AF_OPT_LIMITER: *value = h->limiter; return AF_OK;
    case AF_OPT_GRAPH_STEPS: *value = h->graph_steps; return AF_OK;
    case AF_OPT_TIMING: *value = h->timing; return AF_OK;
    case AF_OPT_AUTOTUNE: *value = h->autotune == 1; return AF_OK;
    case AF_OPT_TRANSONIC: *value = h->tsw; return AF_OK;
    case AF_OPT_SHOCK_LIMITER: *value = h->shock; return AF_OK;
    case AF_OPT_FLUX_LIMITER: *value = h->flux_limiter; return AF_OK;
    case AF_OPT_SYNC_TIMEOUT_US:
      if (!h->batch) return fail(h, AF_ERR_INVALID_ARG, "af_get_option: batched handles only");
      *value = batch_get_sync_timeout(h);
      return AF_OK;
    case AF_OPT_TILE_ORDER:
    case AF_OPT_UPDATE_THREADS:
    case AF_OPT_STEP_KERNEL:
      if (!h->batch) return fail(h, AF_ERR_INVALID_ARG, "af_get_option: batched handles only");
      batch_get_schedule(h, &order, &threads, &kernel);
      *value = key == AF_OPT_TILE_ORDER ? order : (key == AF_OPT_UPDATE_THREADS ? threads : kernel);
      return AF_OK;
    default:
      return fail(h, AF_ERR_INVALID_ARG, "af_get_option: unknown key");
  }
}

extern "C" int af_set_stream(af_handle* h, void* s) {
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_set_stream: NULL handle");
  (void)hipStreamSynchronize(h->stream);
  h->stream = s ? (hipStream_t)s : h->own_stream;
  h->desc_valid = false;  // rewritten on the new stream before its first step
  if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; h->gexec_steps = 0; }
  batch_invalidate(h);
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
int copy2d(const af_handle* h, bool to_device, double* dev, long long pitch, int rows,
                  int cols, double* host, bool user_dev) {
  if (cols > pitch) return fail(h, AF_ERR_INVALID_ARG, "copy2d: cols exceed pitch");
  if (user_dev) {
    const size_t row_bytes = (size_t)cols * 8;
    if (to_device)
      HIP_OK(hipMemcpy2DAsync(dev, pitch * 8, host, row_bytes, row_bytes, (size_t)rows,
                              hipMemcpyDeviceToDevice, h->stream), h);
    else
      HIP_OK(hipMemcpy2DAsync(host, row_bytes, dev, pitch * 8, row_bytes, (size_t)rows,
                              hipMemcpyDeviceToDevice, h->stream), h);
    HIP_OK(hipStreamSynchronize(h->stream), h);
    return AF_OK;
  }
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
int copy4(const af_handle* h, bool to_device, void* dev, long long pitch, int rows_alloc,
                 int rows, int cols, double* host, bool user_dev) {
  if (rows > rows_alloc) return fail(h, AF_ERR_INVALID_ARG, "copy4: rows exceed allocation");
  for (int v = 0; v < 4; ++v) {
    double* d = (double*)dev + (size_t)v * rows_alloc * pitch;
    if (int e = copy2d(h, to_device, d, pitch, rows, cols, host + (size_t)v * rows * cols,
                       user_dev))
      return e;
  }
  return AF_OK;
}

int check_avg_device(const af_handle* h, const double* avg, int nx, int ny, const char* fn) {
  af_handle* hm = const_cast<af_handle*>(h);
  if (!hm->d_flag) HIP_OK(hipMalloc(&hm->d_flag, sizeof(int)), h);
  HIP_OK(hipMemsetAsync(hm->d_flag, 0, sizeof(int), h->stream), h);
  const long long n = (long long)nx * ny;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_check_avg, dim3(blocks), dim3(256), 0, h->stream, avg, n, h->gamma,
                     hm->d_flag);
  HIP_OK(hipGetLastError(), h);
  int bad = 0;
  HIP_OK(hipMemcpyAsync(&bad, hm->d_flag, sizeof(int), hipMemcpyDeviceToHost, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  if (bad) return fail(h, AF_ERR_NONPHYSICAL, std::string(fn) + ": non-admissible cell average");
  return AF_OK;
}

static int set_state_impl(af_handle* h, int g, const double* avg, const double* K,
                          const double* X, const double* Y, double t, bool user_dev,
                          const char* fn) {
  const std::string f(fn);
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, f + ": NULL handle");
  if (h->batch) return batch_set_state(h, g, avg, K, X, Y, t, user_dev);
  if (g != 0) return fail(h, AF_ERR_INVALID_ARG, f + ": grid index must be 0");
  if (!avg || !K || !X || !Y) return fail(h, AF_ERR_INVALID_ARG, f + ": NULL array");
  if (!std::isfinite(t)) return fail(h, AF_ERR_INVALID_ARG, f + ": t not finite");
  if (user_dev) {
    if (int e = check_avg_device(h, avg, h->nx, h->ny, fn)) return e;
  } else {
    const size_t nc = (size_t)h->nx * h->ny;
    for (size_t k = 0; k < nc; ++k) {
      const double r = avg[k], E = avg[3 * nc + k];
      const double kin = 0.5 * (avg[nc + k] * avg[nc + k] + avg[2 * nc + k] * avg[2 * nc + k]) / r;
      if (!(r > 0.0) || !((h->gamma - 1.0) * (E - kin) > 0.0))
        return fail(h, AF_ERR_NONPHYSICAL, f + ": non-admissible cell average");
    }
  }
  h->cur = 0;
  int e;
  if ((e = copy4(h, true, h->A[0], h->pA, h->ny, h->ny, h->nx, const_cast<double*>(avg),
                 user_dev)))
    return e;
  if ((e = copy4(h, true, h->K[0], h->pP, h->nky, h->nky, h->nkx, const_cast<double*>(K),
                 user_dev)))
    return e;
  if ((e = copy4(h, true, h->X[0], h->pP, h->nky, h->ny, h->nkx, const_cast<double*>(X),
                 user_dev)))
    return e;
  if ((e = copy4(h, true, h->Y[0], h->pP, h->nky, h->nky, h->nx, const_cast<double*>(Y),
                 user_dev)))
    return e;
  DevState ds;
  std::memset(&ds, 0, sizeof(ds));
  ds.t = t;
  ds.t_end = t;
  ds.steps_limit = LLONG_MAX;
  HIP_OK(hipMemcpyAsync(h->dev, &ds, sizeof(ds), hipMemcpyHostToDevice, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  h->has_state = true;
  h->steps_base = 0;
  return AF_OK;
}

static int get_state_impl(const af_handle* h, int g, double* avg, double* K, double* X,
                          double* Y, double* t, bool user_dev, const char* fn) {
  const std::string f(fn);
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, f + ": NULL handle");
  if (h->batch) return batch_get_state(h, g, avg, K, X, Y, t, user_dev);
  if (g != 0) return fail(h, AF_ERR_INVALID_ARG, f + ": grid index must be 0");
  if (!h->has_state) return fail(h, AF_ERR_INVALID_ARG, f + ": no state set");
  const int c = h->cur;
  int e;
  if (avg && (e = copy4(h, false, h->A[c], h->pA, h->ny, h->ny, h->nx, avg, user_dev))) return e;
  if (K && (e = copy4(h, false, h->K[c], h->pP, h->nky, h->nky, h->nkx, K, user_dev))) return e;
  if (X && (e = copy4(h, false, h->X[c], h->pP, h->nky, h->ny, h->nkx, X, user_dev))) return e;
  if (Y && (e = copy4(h, false, h->Y[c], h->pP, h->nky, h->nky, h->nx, Y, user_dev))) return e;
  if (t) {
    DevState ds;
    HIP_OK(hipMemcpyAsync(&ds, h->dev, sizeof(ds), hipMemcpyDeviceToHost, h->stream), h);
    HIP_OK(hipStreamSynchronize(h->stream), h);
    *t = ds.t;
  }
  return AF_OK;
}

extern "C" int af_set_state(af_handle* h, const double* avg, const double* K, const double* X,
                            const double* Y, double t) {
  Range range("af_set_state");
  if (h && h->batch && batch_count(h) != 1)
    return fail(h, AF_ERR_INVALID_ARG, "af_set_state: batched handle, use af_set_state_grid");
  return set_state_impl(h, 0, avg, K, X, Y, t, false, "af_set_state");
}

extern "C" int af_get_state(const af_handle* h, double* avg, double* K, double* X, double* Y,
                            double* t) {
  Range range("af_get_state");
  if (h && h->batch && batch_count(h) != 1)
    return fail(h, AF_ERR_INVALID_ARG, "af_get_state: batched handle, use af_get_state_grid");
  return get_state_impl(h, 0, avg, K, X, Y, t, false, "af_get_state");
}

extern "C" int af_set_state_device(af_handle* h, int32_t g, const double* avg, const double* K,
                                   const double* X, const double* Y, double t) {
  Range range("af_set_state_device");
  return set_state_impl(h, g, avg, K, X, Y, t, true, "af_set_state_device");
}

extern "C" int af_get_state_device(const af_handle* h, int32_t g, double* avg, double* K,
                                   double* X, double* Y, double* t) {
  Range range("af_get_state_device");
  return get_state_impl(h, g, avg, K, X, Y, t, true, "af_get_state_device");
}

extern "C" int af_get_counters(const af_handle* h, int64_t* out) {
  if (!h || !out) return fail(h, AF_ERR_INVALID_ARG, "af_get_counters: NULL argument");
  if (h->batch) return batch_get_counters(h, out);
  DevState ds;
  HIP_OK(hipMemcpyAsync(&ds, h->dev, sizeof(ds), hipMemcpyDeviceToHost, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  for (int k = 0; k < AF_NCOUNTERS; ++k) out[k] = (int64_t)ds.cnt[k];
  out[AF_CNT_STEPS] = ds.steps;
  return AF_OK;
}

// Kernels of one step on the buffers B (t_n state in, t_n+1 state out), smax slot `slot`;
// dt_host > 0 for a caller-given step.  `desc` is the device copy of P with B as its buffers
// B[slot] (the point and fix-up kernels read it there).  Events e0/e1/e2 (nullable) bracket the
// point and the update kernels.
template <class R>
static void launch_step(const Params& P, const Bufs& B, const GridDesc* desc, DevState* dev,
                        bool limiter, bool ind, double dt_host, int slot, hipStream_t s,
                        hipEvent_t e0, hipEvent_t e1, hipEvent_t e2, double* TH = nullptr) {
  const int ntiles = P.tiles_x * P.tiles_y;
  if (e0) (void)hipEventRecord(e0, s);
  if (ind) {
    const long long n = (long long)(P.nx + 4) * (P.ny + 4);
    const int gb = (int)std::min<long long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_avgprim, dim3(gb), dim3(256), 0, s, P, B);
    hipLaunchKernelGGL(k_points_ind<R>, dim3(ntiles), dim3(PT_THREADS), 0, s, desc, dev,
                       dt_host, slot);
  } else if constexpr (sizeof(R) == 4) {
    hipLaunchKernelGGL(k_points_f32, dim3(ntiles), dim3(PT_THREADS), 0, s, desc, dev, dt_host,
                       slot);
  } else {
    hipLaunchKernelGGL(k_points_f64, dim3(ntiles), dim3(PT_THREADS), 0, s, desc, dev, dt_host,
                       slot);
  }
  if (limiter) {
    const int nb = std::min(ntiles, FIX_BLOCKS);
    if (ind)
      hipLaunchKernelGGL(k_fixup_ind<R>, dim3(nb), dim3(PT_THREADS), 0, s, desc, dev, slot);
    else if constexpr (sizeof(R) == 4)
      hipLaunchKernelGGL(k_fixup_f32, dim3(nb), dim3(PT_THREADS), 0, s, desc, dev, slot);
    else
      hipLaunchKernelGGL(k_fixup_f64, dim3(nb), dim3(PT_THREADS), 0, s, desc, dev, slot);
  }
  if (e1) (void)hipEventRecord(e1, s);
  if (TH) {
    const long long n = (long long)P.nx * P.ny;
    const int gb = (int)std::min<long long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_flux_theta, dim3(gb), dim3(256), 0, s, P, B.A_in, (const double*)B.FK,
                       (const double*)B.FX, (const double*)B.FY, TH, dev);
    hipLaunchKernelGGL(k_update_lim, dim3(gb), dim3(256), 0, s, P, B.A_in, B.A_out,
                       (const double*)B.FK, (const double*)B.FX, (const double*)B.FY,
                       (const double*)TH, dev, slot);
  } else {
    const long long nwork = (long long)((P.nx + 2 * UP_THREADS - 1) / (2 * UP_THREADS)) * P.ny;
    const int gu = (int)std::min<long long>(nwork, UP_MAX_BLOCKS);
    hipLaunchKernelGGL(k_update, dim3(gu), dim3(UP_THREADS), 0, s, P, B.A_in, B.A_out,
                       (const double*)B.FK, (const double*)B.FX, (const double*)B.FY, dev, slot);
  }
  hipLaunchKernelGGL(k_commit, dim3(1), dim3(1), 0, s, dev, slot);
  if (e2) (void)hipEventRecord(e2, s);
}

// Buffers of a step that reads buffer `in` (0/1) and writes the other.
static Bufs handle_bufs(const af_handle* h, int in) {
  const int out = in ^ 1;
  Bufs B;
  B.A_in = h->A[in]; B.A_out = h->A[out];
  B.K_in = (const double*)h->K[in]; B.X_in = (const double*)h->X[in];
  B.Y_in = (const double*)h->Y[in];
  B.K_out = (double*)h->K[out]; B.X_out = (double*)h->X[out]; B.Y_out = (double*)h->Y[out];
  B.FK = h->FK; B.FX = h->FX; B.FY = h->FY;
  B.fix_mask = h->fix_mask; B.fix_list = h->fix_list;
  B.fix_count = &h->dev->fix_count; B.tile_base = 0;
  B.UB = h->UB;
  return B;
}

// Bring the device descriptor up to date (enqueued on the handle's stream before the steps that
// read it; af_run calls this before it captures a graph).
static int ensure_desc(af_handle* h) {
  if (h->desc_valid) return AF_OK;
  hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(64), 0, h->stream, h->d_desc, make_params(h),
                     handle_bufs(h, 0), handle_bufs(h, 1));
  HIP_OK(hipGetLastError(), h);
  h->desc_valid = true;
  return AF_OK;
}

// enqueue one step reading buffer `in` (0/1); dt_host > 0 for a caller-given step
template <class R>
static void enqueue_step_t(af_handle* h, int in, double dt_host) {
  const Params P = make_params(h);
  const Bufs B = handle_bufs(h, in);
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
  if (h->timing) {
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventCreate(&e2);
  }
  launch_step<R>(P, B, h->d_desc, h->dev, h->limiter != 0, (h->tsw || h->shock), dt_host, in,
                 h->stream, e0, e1, e2, h->flux_limiter ? h->TH : nullptr);
  if (h->timing) {
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
  Range range("af_step");
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_step: NULL handle");
  if (int e = check_inflow(h, "af_step")) return e;
  if (h->batch) return batch_step(h, dt);
  if (!h->has_state) return fail(h, AF_ERR_INVALID_ARG, "af_step: no state set");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(h, AF_ERR_INVALID_ARG, "af_step: dt must be > 0");
  DevState ds;
  int e = read_dev(h, &ds);
  if (e) return e;
  ds.err = 0;
  ds.steps_limit = LLONG_MAX;
  HIP_OK(hipMemcpyAsync(h->dev, &ds, sizeof(ds), hipMemcpyHostToDevice, h->stream), h);
  const long long before = ds.steps;
  if ((e = ensure_desc(h))) return e;
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
  Range range("af_run");
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_run: NULL handle");
  if (int e = check_inflow(h, "af_run")) return e;
  if (h->batch) return batch_run(h, t_end, cfl, max_steps, t_reached, steps_taken);
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
  ds.steps_limit = max_steps > 0 ? steps0 + max_steps : LLONG_MAX;
  HIP_OK(hipMemcpyAsync(h->dev, &ds, sizeof(ds), hipMemcpyHostToDevice, h->stream), h);
  if ((e = ensure_desc(h))) return e;
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
    Range chunk("af_run: chunk of steps");
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

extern "C" int af_set_state_grid(af_handle* h, int32_t g, const double* avg, const double* K,
                                 const double* X, const double* Y, double t) {
  Range range("af_set_state_grid");
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_set_state_grid: NULL handle");
  if (!h->batch) {
    if (g != 0) return fail(h, AF_ERR_INVALID_ARG, "af_set_state_grid: bad grid index");
    return af_set_state(h, avg, K, X, Y, t);
  }
  return batch_set_state(h, g, avg, K, X, Y, t);
}

extern "C" int af_get_state_grid(const af_handle* h, int32_t g, double* avg, double* K, double* X,
                                 double* Y, double* t) {
  Range range("af_get_state_grid");
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_get_state_grid: NULL handle");
  if (!h->batch) {
    if (g != 0) return fail(h, AF_ERR_INVALID_ARG, "af_get_state_grid: bad grid index");
    return af_get_state(h, avg, K, X, Y, t);
  }
  return batch_get_state(h, g, avg, K, X, Y, t);
}

extern "C" int af_get_grid_info(const af_handle* h, int32_t g, double* t, int64_t* steps) {
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_get_grid_info: NULL handle");
  if (h->batch) return batch_grid_info(h, g, t, steps);
  if (g != 0) return fail(h, AF_ERR_INVALID_ARG, "af_get_grid_info: bad grid index");
  if (!h->has_state) return fail(h, AF_ERR_INVALID_ARG, "af_get_grid_info: no state set");
  DevState ds;
  HIP_OK(hipMemcpyAsync(&ds, h->dev, sizeof(ds), hipMemcpyDeviceToHost, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  if (t) *t = ds.t;
  if (steps) *steps = ds.steps;
  return AF_OK;
}

extern "C" int af_set_inflow(af_handle* h, int32_t g, int32_t side, const double* W) {
  if (!h) return fail(nullptr, AF_ERR_INVALID_ARG, "af_set_inflow: NULL handle");
  if (g < 0 || g >= (int)h->sides.size())
    return fail(h, AF_ERR_INVALID_ARG, "af_set_inflow: grid index out of range");
  if (side < 0 || side > 3) return fail(h, AF_ERR_INVALID_ARG, "af_set_inflow: bad side");
  if (h->sides[g].bc[side] != AF_BC_INFLOW)
    return fail(h, AF_ERR_INVALID_ARG, "af_set_inflow: side is not an inflow boundary");
  if (!W || !(W[0] > 0.0) || !(W[3] > 0.0) || !std::isfinite(W[0]) || !std::isfinite(W[1]) ||
      !std::isfinite(W[2]) || !std::isfinite(W[3]))
    return fail(h, AF_ERR_INVALID_ARG, "af_set_inflow: need finite W with rho > 0 and p > 0");
  for (int v = 0; v < 4; ++v) h->sides[g].inflow[side][v] = W[v];
  h->sides[g].set |= 1u << side;
  // the parameters are baked into captured graphs and the device descriptors
  if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; h->gexec_steps = 0; }
  h->desc_valid = false;
  batch_invalidate(h);
  return AF_OK;
}

// ==========================================================================================
// af_step_noalloc: one step on caller-owned device arrays with the file-scope scratch array
// ==========================================================================================
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(void** out) {
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= kMaxDevices)
    return fail(nullptr, AF_ERR_DEVICE, "af_step_noalloc: no current HIP device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(af::scratch));
    if (e != hipSuccess || !p)
      return fail(nullptr, AF_ERR_DEVICE,
                  std::string("af_step_noalloc: hipGetSymbolAddress(scratch): ") +
                      hipGetErrorString(e));
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return AF_OK;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

extern "C" int af_step_noalloc(const af_grid* grid, double gamma, const af_bc* bc,
                               const double* inflow, int32_t precision, int32_t linearisation,
                               int32_t correction, int32_t limiter, const double* avg_in,
                               const double* K_in, const double* X_in, const double* Y_in,
                               double* avg_out, double* K_out, double* X_out, double* Y_out,
                               int64_t pitch_avg, int64_t pitch_pts, double dt, void* stream,
                               int64_t* counters) {
  Range range("af_step_noalloc");
  const char* fn = "af_step_noalloc";
  if (!grid || !bc) return fail(nullptr, AF_ERR_INVALID_ARG, "af_step_noalloc: NULL grid or bc");
  if (int e = check_grid(grid, bc, fn)) return e;
  if (!(gamma > 1.0) || !std::isfinite(gamma))
    return fail(nullptr, AF_ERR_INVALID_ARG, "af_step_noalloc: gamma must be finite and > 1");
  if ((precision != AF_PREC_FP64 && precision != AF_PREC_FP32) || linearisation < 0 ||
      linearisation > 2 || (correction != 0 && correction != 1) || (limiter != 0 && limiter != 1))
    return fail(nullptr, AF_ERR_INVALID_ARG, "af_step_noalloc: bad option value");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return fail(nullptr, AF_ERR_INVALID_ARG, "af_step_noalloc: dt must be > 0");
  const double* ins[4] = {avg_in, K_in, X_in, Y_in};
  const double* outs[4] = {avg_out, K_out, X_out, Y_out};
  for (int k = 0; k < 4; ++k) {
    if (!ins[k] || !outs[k]) return fail(nullptr, AF_ERR_INVALID_ARG, "af_step_noalloc: NULL array");
    if ((reinterpret_cast<uintptr_t>(ins[k]) | reinterpret_cast<uintptr_t>(outs[k])) & 15u)
      return fail(nullptr, AF_ERR_INVALID_ARG, "af_step_noalloc: arrays must be 16-byte aligned");
    for (int m = 0; m < 4; ++m)
      if (ins[k] == outs[m])
        return fail(nullptr, AF_ERR_INVALID_ARG, "af_step_noalloc: an output aliases an input");
  }
  const int nx = grid->nx, ny = grid->ny;
  const int per_x = bc->left == AF_BC_PERIODIC, per_y = bc->bottom == AF_BC_PERIODIC;
  const int nkx = nx + (per_x ? 0 : 1), nky = ny + (per_y ? 0 : 1);
  if (pitch_avg < nx || pitch_pts < nkx || (pitch_avg & 1) || (pitch_pts & 1))
    return fail(nullptr, AF_ERR_INVALID_ARG,
                "af_step_noalloc: need even pitches, pitch_avg >= nx, pitch_pts >= nx + 1 on "
                "a non-periodic x axis (>= nx otherwise)");
  Params P;
  P.nx = nx; P.ny = ny; P.nkx = nkx; P.nky = nky; P.per_x = per_x; P.per_y = per_y;
  P.tiles_x = (nkx + TILE - 1) / TILE;
  P.tiles_y = (nky + TILE - 1) / TILE;
  const double dx = (grid->x1 - grid->x0) / nx, dy = (grid->y1 - grid->y0) / ny;
  P.dx = dx; P.dy = dy; P.idx = 1.0 / dx; P.idy = 1.0 / dy;
  P.gamma = gamma; P.hmin = std::min(dx, dy);
  P.g1inv = 1.0 / (gamma - 1.0); P.aspect = dx / dy;
  P.mode = linearisation; P.correction = correction; P.limiter = limiter; P.pad = 0;
  P.pA = pitch_avg; P.sA = pitch_avg * ny;
  P.pP = pitch_pts; P.sP = pitch_pts * nky;
  P.pF = pitch_pts; P.sF = pitch_pts * nky;
  const int kinds[4] = {bc->left, bc->right, bc->bottom, bc->top};
  for (int s = 0; s < 4; ++s) {
    P.bc[s] = kinds[s];
    for (int v = 0; v < 4; ++v) P.inflow[s][v] = 0.0;
    if (kinds[s] == AF_BC_INFLOW) {
      if (!inflow || !(inflow[4 * s] > 0.0) || !(inflow[4 * s + 3] > 0.0))
        return fail(nullptr, AF_ERR_INVALID_ARG,
                    "af_step_noalloc: an inflow side needs a state with rho > 0 and p > 0");
      for (int v = 0; v < 4; ++v) P.inflow[s][v] = inflow[4 * s + v];
    }
  }
  P.tsw = 0; P.shock = 0; P.pU = 0; P.sU = 0;

  // scratch layout: step control, grid descriptor, fix-up masks (4 words per tile), fix-up
  // list, flux sums
  const size_t ntiles = (size_t)P.tiles_x * P.tiles_y;
  const size_t o_desc = align256(sizeof(DevState));
  const size_t o_mask = align256(o_desc + sizeof(GridDesc));
  const size_t o_list = align256(o_mask + ntiles * 4 * sizeof(unsigned long long));
  const size_t o_flux = align256(o_list + ntiles * sizeof(int));
  const size_t flux_words = (size_t)P.sF * 16;  // FK: 8 variables, FX: 4, FY: 4
  const size_t need = o_flux + flux_words * sizeof(double);
  if (need > NOALLOC_BYTES)
    return fail(nullptr, AF_ERR_INVALID_ARG,
                "af_step_noalloc: grid too large for the scratch array (" +
                    std::to_string(need) + " bytes needed, " + std::to_string(NOALLOC_BYTES) +
                    " available)");
  void* base = nullptr;
  if (int e = scratch_address(&base)) return e;
  unsigned char* sp = static_cast<unsigned char*>(base);
  DevState* dev = reinterpret_cast<DevState*>(sp);
  Bufs B;
  B.A_in = avg_in; B.A_out = avg_out;
  B.K_in = K_in; B.X_in = X_in; B.Y_in = Y_in;
  B.K_out = K_out; B.X_out = X_out; B.Y_out = Y_out;
  double* flux = reinterpret_cast<double*>(sp + o_flux);
  B.FK = flux; B.FX = flux + (size_t)P.sF * 8; B.FY = flux + (size_t)P.sF * 12;
  B.fix_mask = reinterpret_cast<unsigned long long*>(sp + o_mask);
  B.fix_list = reinterpret_cast<int*>(sp + o_list);
  B.fix_count = &dev->fix_count;
  B.tile_base = 0;
  B.UB = nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long nmask = (long long)ntiles * 4;
  const int ib = (int)std::min<long long>((nmask + 255) / 256, 1024);
  GridDesc* desc = reinterpret_cast<GridDesc*>(sp + o_desc);
  hipLaunchKernelGGL(k_noalloc_init, dim3(std::max(ib, 1)), dim3(256), 0, s, dev, B.fix_mask,
                     nmask);
  hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(64), 0, s, desc, P, B, B);
  if (precision == AF_PREC_FP32)
    launch_step<float>(P, B, desc, dev, limiter != 0, false, dt, 0, s, nullptr, nullptr,
                       nullptr);
  else
    launch_step<double>(P, B, desc, dev, limiter != 0, false, dt, 0, s, nullptr, nullptr,
                        nullptr);
  hipError_t he = hipGetLastError();
  if (he != hipSuccess)
    return fail(nullptr, AF_ERR_DEVICE, std::string("af_step_noalloc: launch: ") + hipGetErrorString(he));
  DevState ds;
  he = hipMemcpyAsync(&ds, dev, sizeof(ds), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess)
    return fail(nullptr, AF_ERR_DEVICE, std::string("af_step_noalloc: ") + hipGetErrorString(he));
  if (counters) {
    for (int k = 0; k < AF_NCOUNTERS; ++k) counters[k] = (int64_t)ds.cnt[k];
    counters[AF_CNT_STEPS] = ds.steps;
  }
  if (ds.err) return fail(nullptr, ds.err, std::string(fn) + ": " + err_text(ds.err));
  if (ds.steps != 1) return fail(nullptr, AF_ERR_DEVICE, "af_step_noalloc: step did not commit");
  return AF_OK;
}

// Domain totals of the conserved variables of the current state: out[0..3] = the sums over the
// grid's cells of rho, rho u, rho v and E times the cell area (deterministic; synchronous).
extern "C" int af_get_totals(const af_handle* h, int32_t g, double* out) {
  Range range("af_get_totals");
  if (!h || !out) return fail(h, AF_ERR_INVALID_ARG, "af_get_totals: NULL argument");
  af_handle* hm = const_cast<af_handle*>(h);
  if (!hm->d_totals)
    HIP_OK(hipMalloc(&hm->d_totals, (4 * TOTAL_BLOCKS + 4) * sizeof(double)), h);
  if (h->batch) return batch_totals(h, g, out);
  if (g != 0) return fail(h, AF_ERR_INVALID_ARG, "af_get_totals: grid index must be 0");
  if (!h->has_state) return fail(h, AF_ERR_INVALID_ARG, "af_get_totals: no state set");
  return reduce_totals(h, h->stream, h->A[h->cur], h->pA, h->pA * h->ny, h->nx, h->ny,
                       h->dx * h->dy, h->d_totals, out);
}
