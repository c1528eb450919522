// af_batch.hip -- many independent grids advanced together (af_create_batch in af.h).
//
// The grids' arrays are packed into one allocation per array kind.  Every step is one launch
// of each kernel for all grids: the point kernel runs one workgroup per 8x8-site tile of any
// grid (a per-tile table gives the grid), the update kernel one workgroup per row of cells of
// any grid, then a commit kernel advances each grid's time.  Each grid keeps its own time step
// (CFL from its own wave speeds), time, step limit and buffer index on the device, so the
// sequence of launches is the same for every step and is captured once in a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "af.h"
#include "af_host.hpp"
#include "af_step.hpp"

namespace af {

// Agent-scope load of a value another workgroup may have written earlier in the same launch.
__device__ __forceinline__ int ld_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __longlong_as_double(__hip_atomic_load(reinterpret_cast<const long long*>(p),
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Point kernel over the tiles of all grids.  Workgroup b evolves the tile block_tile[b] =
// (grid, tile within the grid): a permutation of the global tiles (the schedule, see
// set_order).  One table read names the grid, so the grid's descriptor and step control are
// the next loads and the first staging loads the ones after.
template <class R, bool IND = false>
__device__ __forceinline__ void batch_points(Smem<R>& S, Ind* I, const GridDesc* __restrict__ desc,
                                             const int2* __restrict__ block_tile,
                                             DevState* devs, double dt_host, int k) {
  const int2 gt = block_tile[k];
  const int g = __builtin_amdgcn_readfirstlane(gt.x);
  const int local = __builtin_amdgcn_readfirstlane(gt.y);
  const int cur = __builtin_amdgcn_readfirstlane(devs[g].cur);
  const Params& P = desc[g].P;
  const Bufs& B = desc[g].B[cur];
  points_body<R, IND>(S, I, P, B, devs + g, dt_host, cur, local, local == 0);
}

// The grid's descriptor seen through the constant address space, as a reference the step
// code takes like any other.  The host writes the descriptors before a launch and no kernel
// writes them, so loads from them may be taken as never clobbered; the compiler then issues
// the uniform ones as scalar loads.  Read through a plain pointer inside the persistent kernel,
// whose loop has atomics, fences and stores, the same loads become vector loads, kept in VGPRs
// and partly spilled (FP32 19 VGPRs spilled against 14, FP64 46 against 31).
typedef const __attribute__((address_space(4))) GridDesc ConstGridDesc;
__device__ __forceinline__ const GridDesc& const_desc(const GridDesc* d, int g) {
  ConstGridDesc* c = (ConstGridDesc*)d;
  return *(const GridDesc*)(c + g);
}

// The persistent kernel's point item: the split kernel's points_body with one addition: `pop`
// (a functor called by
// every thread) takes the workgroup's next item from its queue once the tile's sites are
// staged and prepared, so that the atomic's round trip overlaps the tile's arithmetic.  A grid
// that takes no step does no work and no pop; the caller then pops after the item.  Returns
// whether `pop` was called (uniform over the workgroup).
template <class R, bool IND, class Pop>
__device__ __forceinline__ bool batch_points_item(Smem<R>& S, Ind* I,
                                                  const GridDesc* __restrict__ desc,
                                                  const int2* __restrict__ block_tile,
                                                  DevState* devs, double dt_host, int k,
                                                  Pop& pop) {
  const int2 gt = block_tile[k];
  const int g = __builtin_amdgcn_readfirstlane(gt.x);
  const int local = __builtin_amdgcn_readfirstlane(gt.y);
  const int cur = __builtin_amdgcn_readfirstlane(devs[g].cur);
  const GridDesc& D = const_desc(desc, g);
  const Params& P = D.P;
  const Bufs& B = D.B[cur];
  DevState* dev = devs + g;
  double dt;
  bool popped = false;
  if (step_dt(P, dev, dt_host, cur, local == 0, &dt)) {
    stage_and_prep(S, P, B, dev, local, true);
    if constexpr (IND) stage_indicators(S, *I, P, B, local);
    pop();
    popped = true;
    double speed = 0.0;
    evolve_tile<R, false, IND>(S, I, P, B, dev, local, dt, nullptr, speed);
    block_max_atomic(speed, &dev->smax[cur ^ 1], S.red);
  }
  __syncthreads();  // the tile's LDS is free before the next item stages into it
  return popped;
}

__global__ __launch_bounds__(PT_THREADS) AF_ATTR_F32
void kb_points_f32(const GridDesc* __restrict__ desc, const int2* __restrict__ block_tile,
                   DevState* devs, double dt_host) {
  __shared__ Smem<float> S;
  batch_points<float>(S, nullptr, desc, block_tile, devs, dt_host, blockIdx.x);
}
__global__ __launch_bounds__(PT_THREADS) AF_ATTR_F64
void kb_points_f64(const GridDesc* __restrict__ desc, const int2* __restrict__ block_tile,
                   DevState* devs, double dt_host) {
  __shared__ Smem<double> S;
  batch_points<double>(S, nullptr, desc, block_tile, devs, dt_host, blockIdx.x);
}

// With the shock indicators (Algorithm 2, Sec. 3.4): the point kernel's indicator variant.  At
// least two waves per SIMD: left alone, the FP64 variant takes two registers more than that
// allows and runs one wave per SIMD.
template <class R>
__global__ __launch_bounds__(PT_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
void kb_points_ind(const GridDesc* __restrict__ desc, const int2* __restrict__ block_tile,
                   DevState* devs, double dt_host) {
  __shared__ Smem<R> S;
  __shared__ Ind I;
  batch_points<R, true>(S, &I, desc, block_tile, devs, dt_host, blockIdx.x);
}

// Primitive Simpson averages of every grid's padded cells (-2 .. nx+1 x -2 .. ny+1) from its
// current state: one workgroup per padded row (prow_grid: the grid of each padded row).
__device__ __forceinline__ void avgprim_row(const GridDesc* __restrict__ desc,
                                            const int* __restrict__ prow_grid,
                                            const int* __restrict__ prow_base, DevState* devs,
                                            int row) {
  const int g = prow_grid[row];
  const GridDesc& D = const_desc(desc, g);
  const Params& P = D.P;
  const Bufs& B = D.B[devs[g].cur];
  const int j = row - prow_base[g] - 2;
  for (int i = (int)threadIdx.x - 2; i < P.nx + 2; i += (int)blockDim.x) {
    double ub[4];
    prim_average(P, B, i, j, ub);
    const long long o = (long long)(j + 2) * P.pU + (i + 2);
#pragma unroll
    for (int v = 0; v < 4; ++v) B.UB[v * P.sU + o] = ub[v];
  }
}
__global__ __launch_bounds__(256) void kb_avgprim(const GridDesc* __restrict__ desc,
                                                  const int* __restrict__ prow_grid,
                                                  const int* __restrict__ prow_base,
                                                  DevState* devs) {
  avgprim_row(desc, prow_grid, prow_base, devs, blockIdx.x);
}

// Positivity fix-up over the global list of flagged tiles (entries are global tile indices).
// Entry k of the list: the tile's grid, buffers and step from the device state.
template <class R, bool IND = false>
__device__ __forceinline__ void fixup_entry(Smem<R>& S, Ind* I, const GridDesc* __restrict__ desc,
                                            const int* __restrict__ tile_grid, DevState* devs,
                                            const int* fix_list, unsigned int k) {
  __shared__ unsigned long long mask[3];
  __shared__ int s_g, s_cur, s_run, s_tile;
  __shared__ double s_dt;
  if (threadIdx.x == 0) {
    const int t = fix_list[k];
    const int g = tile_grid[t];
    s_g = g;
    s_tile = t - desc[g].tile_base;
    s_cur = devs[g].cur;
    s_run = !ld_agent(&devs[g].err) && ld_agent(&devs[g].active);
    s_dt = ld_agent(&devs[g].dt);
  }
  __syncthreads();
  const int g = __builtin_amdgcn_readfirstlane(s_g);
  const int cur = __builtin_amdgcn_readfirstlane(s_cur);
  const GridDesc& D = const_desc(desc, g);
  const Params& P = D.P;
  const Bufs& B = D.B[cur];
  double speed = 0.0;
  fixup_tile<R, IND>(S, I, P, B, devs + g, s_tile, s_dt, s_run != 0, mask, speed);
  block_max_atomic(speed, &devs[g].smax[cur ^ 1], S.red);
  __syncthreads();  // the next entry overwrites the shared values
}
template <class R, bool IND = false>
__device__ __forceinline__ void batch_fixup(Smem<R>& S, Ind* I, const GridDesc* __restrict__ desc,
                                            const int* __restrict__ tile_grid, DevState* devs,
                                            const int* fix_list, const unsigned int* fix_count) {
  __shared__ unsigned int s_n;
  if (threadIdx.x == 0) s_n = *fix_count;
  __syncthreads();
  const unsigned int n = s_n;
  for (unsigned int k = blockIdx.x; k < n; k += gridDim.x)
    fixup_entry<R, IND>(S, I, desc, tile_grid, devs, fix_list, k);
}
__global__ __launch_bounds__(PT_THREADS)
void kb_fixup_f32(const GridDesc* __restrict__ desc, const int* __restrict__ tile_grid,
                  DevState* devs, const int* __restrict__ fix_list,
                  const unsigned int* fix_count) {
  __shared__ Smem<float> S;
  batch_fixup<float>(S, nullptr, desc, tile_grid, devs, fix_list, fix_count);
}
__global__ __launch_bounds__(PT_THREADS)
void kb_fixup_f64(const GridDesc* __restrict__ desc, const int* __restrict__ tile_grid,
                  DevState* devs, const int* __restrict__ fix_list,
                  const unsigned int* fix_count) {
  __shared__ Smem<double> S;
  batch_fixup<double>(S, nullptr, desc, tile_grid, devs, fix_list, fix_count);
}

template <class R>
__global__ __launch_bounds__(PT_THREADS)
void kb_fixup_ind(const GridDesc* __restrict__ desc, const int* __restrict__ tile_grid,
                  DevState* devs, const int* __restrict__ fix_list,
                  const unsigned int* fix_count) {
  __shared__ Smem<R> S;
  __shared__ Ind I;
  batch_fixup<R, true>(S, &I, desc, tile_grid, devs, fix_list, fix_count);
}

// Update kernel.  The cells of a grid are taken as pairs of neighbours in a row, numbered row by
// row, and cut into chunks of T pairs; in a grid of odd width the last cell of every row is left
// out of the pairs, and these cells form chunks of T rows of their own after the pair chunks (so
// that no wave mixes the paired and the single-cell code).  A work item is one chunk of one grid
// ((grid, chunk) in `items`), one workgroup per item in an XCD-aware order.  Lanes stay busy
// across the ends of short rows, and neighbouring workgroups read neighbouring memory.  The
// grid's largest new wave speed goes out by one atomic per item.
// Two waves per SIMD, as the single-grid update: the register budget lets every load of a cell
// pair be in flight before its first use (left alone, the compiler takes 116 registers for four
// waves and the loads go out in groups).
template <int T>
__device__ __forceinline__ void update_body(const Params& P, const Bufs& B, int2 it,
                                            DevState* dev, int cur, double* red) {
  // Set in the point phase, which a kernel boundary or (persistent kernel) a grid barrier
  // separates from this one: the barrier's acquire makes plain loads current, and they hit L2,
  // where agent-scope atomic loads would go to memory at every item.  An error flagged by
  // another update item meanwhile may be missed; the item then updates a state that is not
  // committed, and the codes combine by a minimum (set_err), whichever item came first.
  const bool run = !dev->err && dev->active;
  const double dt = dev->dt;
  const double lx = dt * P.idx * (1.0 / 36.0), ly = dt * P.idy * (1.0 / 36.0);
  // full pairs per row, their number and chunks (below 2^31: at most 65536 rows of 32768 pairs)
  const unsigned ppr = (unsigned)P.nx >> 1;
  const unsigned npair = ppr * (unsigned)P.ny;
  const unsigned nchunk = (npair + T - 1) / T;
  double speed = 0.0;
  bool bad = false;
  if (run) {
    int i = -1, j = 0;
    if ((unsigned)it.y < nchunk) {
      const unsigned pair = (unsigned)it.y * T + threadIdx.x;
      if (pair < npair) {
        j = (int)(pair / ppr);
        i = 2 * (int)(pair - (unsigned)j * ppr);
      }
    } else {  // the last cell of each row of a grid of odd width
      j = (int)(((unsigned)it.y - nchunk) * T + threadIdx.x);
      if (j < P.ny) i = P.nx - 1;
    }
    if (i >= 0 && !update_pair(P, B.A_in, B.A_out, B.FK, B.FX, B.FY, lx, ly, i, j, speed))
      bad = true;
  }
  if (bad) set_err(dev, ERR_NONPHYS);
  for (int off = 32; off > 0; off >>= 1) speed = mx(speed, __shfl_xor(speed, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = speed;
  __syncthreads();
  if (threadIdx.x == 0 && run) {
    double m = red[0];
    for (int k = 1; k < (T + 63) / 64; ++k) m = mx(m, red[k]);
    atomic_max_pos(&dev->smax[cur ^ 1], m);
  }
}
template <int T>
__device__ __forceinline__ void update_item(const GridDesc* __restrict__ desc, int2 it,
                                            DevState* devs, double* red) {
  const int g = __builtin_amdgcn_readfirstlane(it.x);
  DevState* dev = devs + g;
  const int cur = __builtin_amdgcn_readfirstlane(dev->cur);
  update_body<T>(desc[g].P, desc[g].B[cur], it, dev, cur, red);
}
// The persistent kernel's update item, with the descriptor read as in batch_points_item.
template <int T>
__device__ __forceinline__ void update_item_persistent(const GridDesc* __restrict__ desc,
                                                       int2 it, DevState* devs, double* red) {
  const int g = __builtin_amdgcn_readfirstlane(it.x);
  DevState* dev = devs + g;
  const int cur = __builtin_amdgcn_readfirstlane(dev->cur);
  const GridDesc& D = const_desc(desc, g);
  update_body<T>(D.P, D.B[cur], it, dev, cur, red);
}
template <int T>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(2, 2)))
void kb_update(const GridDesc* __restrict__ desc, const int2* __restrict__ items,
               int total_items, DevState* devs) {
  __shared__ double red[(T + 63) / 64];
  update_item<T>(desc, items[tile_of_block(blockIdx.x, total_items)], devs, red);
}

// Commit: every grid whose step ran without error advances t and its step counter, clears the
// wave-speed slot of the old state and switches to the other buffer.
__device__ __forceinline__ void commit_grid(DevState* d) {
  if (!d->err && d->active) {
    d->t = d->last ? d->t_end : d->t + d->dt;
    d->steps += 1;
    d->smax[d->cur] = 0ull;
    d->cur ^= 1;
  }
}
__global__ void kb_commit(DevState* devs, int n, unsigned int* fix_count) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) *fix_count = 0u;
  if (g < n) commit_grid(devs + g);
}

// Wave speed of every grid's current state into its smax[cur], before a run: `per` workgroups
// per grid.
__global__ void kb_cfl(const GridDesc* __restrict__ desc, DevState* devs, int per) {
  __shared__ double red[4];
  const int g = blockIdx.x / per, part = blockIdx.x % per;
  const Params& P = desc[g].P;
  const int cur = devs[g].cur;
  const Bufs& B = desc[g].B[cur];
  const double speed = state_speed(P, B.A_in, B.K_in, B.X_in, B.Y_in,
                                   (long long)part * blockDim.x + threadIdx.x,
                                   (long long)per * blockDim.x);
  block_max_atomic(speed, &devs[g].smax[cur], red);
}

// ------------------------------------------------------------------------------------------
// The whole step in one persistent launch (AF_STEP_PERSISTENT).
//
// A fixed grid of workgroups, no more than can be resident on the GPU at once, takes the step's
// work from device-side queues, phase after phase: the padded primitive averages (with the
// indicators), the tiles of the point kernel, the tiles listed for the positivity fix-up (with
// the limiter), the update items.  A grid-wide barrier separates the phases; the last workgroup
// to finish commits every grid and leaves the queues empty for the next launch.  Each phase's
// items are split over 8 queues, one per XCD (workgroup b runs on XCD b mod 8, and queue x
// holds items x, x + 8, x + 16, ...), so that the tile orders keep their meaning.  The point
// and update phases hand out every item by the queue's head counter, in order (resolve_pop);
// the indicator rows and the listed tiles go mostly by a fixed stride (next_item).  The grid
// is a multiple of 8 workgroups.  Every wait is bounded: a
// barrier not reached within the handle's limit on the 100 MHz wall clock (workgroups that
// were not all resident) flags `timeout`, and the step then ends every running grid with
// ERR_SYNC instead of committing it.
struct StepSync {
  unsigned int head[8 * 16];  // queue heads, 64 bytes apart
  unsigned int arrive, pad0[15];
  unsigned int gen, pad1[15];
  unsigned int done, pad2[15];
  unsigned int timeout, pad3[15];
};
constexpr unsigned int SYNC_MAX_POLLS = 1u << 26;  // a second bound, independent of the clock

// Relaxed agent-scope load of a counter: no cache invalidation (an acquire would invalidate the
// caches at every queue pop and every poll, and the tiles would lose their L2 halo reuse); the
// barrier orders the data with fences of its own.
__device__ __forceinline__ unsigned int ld_relaxed(const unsigned int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(unsigned int* p, unsigned int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Items of the other phases, m of them: queue x holds items x, x + 8, x + 16, ... below m
// (queue-local index j: item x + 8 j); the workgroups of XCD x (b mod 8 = x, wpq = nb / 8 of
// them) take the queue's first items by a fixed stride -- workgroup b takes j = b / 8,
// b / 8 + wpq, ... -- so that together they walk the queue in order, as the hardware
// dispatches a kernel's workgroups, with no atomic per item.  The last 2 wpq items of every
// queue are handed out one by one by its head counter, to the queue's own workgroups first and
// then to those whose queues are done.
__device__ __forceinline__ int queue_len(int m, int x) { return x < m ? (m - x + 7) >> 3 : 0; }
__device__ __forceinline__ int queue_tail(int m, int x, int wpq) {
  return min(queue_len(m, x), 2 * wpq);
}
// A tail item for a workgroup on XCD `xcd` (thread 0 only): an index in [0, m), or -1 once
// every tail is empty.
__device__ __forceinline__ int pop_tail(StepSync* s, int m, int xcd, int wpq) {
  for (int k = 0; k < 8; ++k) {
    const int x = (xcd + k) & 7;
    const unsigned int t = (unsigned int)queue_tail(m, x, wpq);
    if (t == 0u || ld_relaxed(&s->head[16 * x]) >= t) continue;
    const unsigned int p = atomicAdd(&s->head[16 * x], 1u);
    if (p < t) return x + 8 * (queue_len(m, x) - (int)t + (int)p);
  }
  return -1;
}

// The workgroup's next item of a phase with m items, the same for all its threads; `j` (thread
// 0's) is the workgroup's next fixed-stride index, b / 8 at the start of the phase, -1 once
// they are done.
__device__ __forceinline__ int next_item(StepSync* s, int m, int* s_item, int& j) {
  if (threadIdx.x == 0) {
    const int x = (int)(blockIdx.x & 7), wpq = (int)(gridDim.x >> 3);
    int k = -1;
    if (j >= 0) {
      if (j < queue_len(m, x) - queue_tail(m, x, wpq)) {
        k = x + 8 * j;
        j += wpq;
      } else {
        j = -1;
      }
    }
    if (k < 0) k = pop_tail(s, m, x, wpq);
    *s_item = k;
  }
  __syncthreads();
  const int k = *s_item;
  __syncthreads();  // read by all before thread 0 overwrites it
  return k;
}

// The point and update phases take every item through its queue's head counter: the p-th pop
// of queue x is item x + 8 p, so each XCD's items go out strictly in order, as the hardware
// dispatcher hands out a kernel's workgroups, and the items in flight on an XCD stay a narrow
// window of its range (the fixed stride lets the workgroups drift apart, and the tiles that
// share a halo are then no longer in L2 together).  `p` is the value the workgroup's atomic on
// its own head returned; once its queue is empty it takes items from the others.  -1 when all
// are empty.
__device__ __forceinline__ int resolve_pop(StepSync* s, int m, int xcd, unsigned int p) {
  if ((int)p < queue_len(m, xcd)) return xcd + 8 * (int)p;
  for (int k = 1; k < 8; ++k) {
    const int x = (xcd + k) & 7;
    const unsigned int t = (unsigned int)queue_len(m, x);
    if (t == 0u || ld_relaxed(&s->head[16 * x]) >= t) continue;
    const unsigned int q = atomicAdd(&s->head[16 * x], 1u);
    if (q < t) return x + 8 * (int)q;
  }
  return -1;
}

// Grid-wide barrier of the `nb` workgroups; the last to arrive empties the queues for the
// next phase.  Every wave releases its writes (agent scope) before the workgroup arrives and
// acquires the other workgroups' after it leaves.
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void grid_barrier(StepSync* s, unsigned int nb,
                                             unsigned long long limit_ticks) {
  fence_release();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int g = ld_relaxed(&s->gen);
    fence_release();  // the read of gen comes before the arrival
    if (atomicAdd(&s->arrive, 1u) == nb - 1) {
      for (int x = 0; x < 8; ++x) st_relaxed(&s->head[16 * x], 0u);
      st_relaxed(&s->arrive, 0u);
      __hip_atomic_fetch_add(&s->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const unsigned long long t0 = (unsigned long long)wall_clock64();
      for (unsigned int it = 0; ld_relaxed(&s->gen) == g; ++it) {
        __builtin_amdgcn_s_sleep(4);
        if ((unsigned long long)wall_clock64() - t0 > limit_ticks ||
            it >= SYNC_MAX_POLLS) {
          st_relaxed(&s->timeout, 1u);
          break;
        }
      }
    }
    fence_acquire();
  }
  __syncthreads();
  fence_acquire();
}

// The kernel's arguments, kept in LDS.  Read back inside every phase loop (after its barrier,
// so that the reads cannot be hoisted out of the loop) they are not live through the point
// phase: as kernel-argument registers held across the whole kernel they pushed the point
// phase into SGPR spills (v_readlane/v_writelane, VALU instructions in the hot code).
struct StepArgs {
  const GridDesc* desc;
  const int2* block_tile;
  const int2* items;
  const int* tile_grid;
  const int* prow_grid;
  const int* prow_base;
  DevState* devs;
  int* fix_list;
  unsigned int* fix_count;
  StepSync* sync;
  double dt_host;
  unsigned long long sync_ticks;  // barrier wait limit (100 MHz wall-clock ticks)
  int n_tiles, n_items, n_prows, n_grids;
};
// A pointer read from LDS, made wave-uniform (scalar loads through it stay possible).
template <class T> __device__ __forceinline__ T* uni(T* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)v);
  const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)(v >> 32));
  return (T*)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// `desc` and `block_tile` stay kernel arguments, read-only and __restrict__ (the descriptors are
// read through const_desc): through a pointer read back from LDS the compiler cannot tell that
// nothing writes them, and loads them with vector instructions.
template <class R, bool LIM, bool IND>
__device__ __forceinline__ void step_body(Smem<R>& S, Ind* I, const GridDesc* __restrict__ desc,
                                          const int2* __restrict__ block_tile,
                                          const StepArgs& arg) {
  __shared__ StepArgs A;
  __shared__ int s_item;
  __shared__ unsigned int s_n;
  __shared__ int s_last;
  if (threadIdx.x == 0) A = arg;
  __syncthreads();
  // A launch in which no grid can step (every grid stopped or failed: the rest of a run's last
  // graph chunk) leaves at once, instead of handing out every tile to find that out.  The test
  // is step_dt's, which would only clear the stopped grids' `active` flags, and the next launch
  // that steps sets every flag again before anything reads it.  All workgroups read the same
  // states, written by earlier launches, so they all leave or all stay.
  int can_step = 0;
  for (int g = threadIdx.x; g < uni(A.n_grids); g += blockDim.x) {
    const DevState* d = uni(A.devs) + g;
    can_step |= !d->err && d->steps < d->steps_limit && (A.dt_host > 0.0 || d->t < d->t_end);
  }
  if (!__syncthreads_or(can_step)) return;
  const unsigned int nb = gridDim.x;
  const int j0 = (int)(blockIdx.x >> 3);
  if constexpr (IND) {
    for (int k, j = j0; (k = next_item(uni(A.sync), uni(A.n_prows), &s_item, j)) >= 0;)
      avgprim_row(desc, uni(A.prow_grid), uni(A.prow_base), uni(A.devs), k);
    grid_barrier(uni(A.sync), nb, A.sync_ticks);
  }
  {
    StepSync* sy = uni(A.sync);
    const int m = uni(A.n_tiles), xcd = (int)(blockIdx.x & 7);
    if (threadIdx.x == 0) s_item = resolve_pop(sy, m, xcd, atomicAdd(&sy->head[16 * xcd], 1u));
    __syncthreads();
    int k = s_item;
    __syncthreads();
    while (k >= 0) {
      unsigned int p = 0u;  // thread 0's
      auto pop = [&]() {
        if (threadIdx.x == 0) p = atomicAdd(&sy->head[16 * xcd], 1u);
      };
      const bool popped = batch_points_item<R, IND>(S, I, desc, block_tile, uni(A.devs),
                                                    A.dt_host, k, pop);
      if (threadIdx.x == 0) {
        if (!popped) p = atomicAdd(&sy->head[16 * xcd], 1u);
        s_item = resolve_pop(sy, m, xcd, p);
      }
      __syncthreads();
      k = s_item;
      __syncthreads();
    }
  }
  grid_barrier(uni(A.sync), nb, A.sync_ticks);
  if constexpr (LIM) {
    if (threadIdx.x == 0) s_n = __hip_atomic_load(A.fix_count, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int nfix = (int)s_n;
    for (int k, j = j0; (k = next_item(uni(A.sync), nfix, &s_item, j)) >= 0;)
      fixup_entry<R, IND>(S, I, desc, uni(A.tile_grid), uni(A.devs), uni(A.fix_list),
                          (unsigned int)k);
    grid_barrier(uni(A.sync), nb, A.sync_ticks);
  }
  // update items, in order like the tiles (neighbouring rows share the flux sums of their
  // common sites); the next pop goes out before the item's loads
  {
    StepSync* sy = uni(A.sync);
    const int m = uni(A.n_items), xcd = (int)(blockIdx.x & 7);
    if (threadIdx.x == 0) s_item = resolve_pop(sy, m, xcd, atomicAdd(&sy->head[16 * xcd], 1u));
    __syncthreads();
    int k = s_item;
    __syncthreads();
    while (k >= 0) {
      unsigned int p = 0u;
      if (threadIdx.x == 0) p = atomicAdd(&sy->head[16 * xcd], 1u);
      update_item_persistent<PT_THREADS>(desc, uni(A.items)[tile_of_block(k, m)], uni(A.devs),
                                         S.red);
      if (threadIdx.x == 0) s_item = resolve_pop(sy, m, xcd, p);
      __syncthreads();
      k = s_item;
      __syncthreads();
    }
  }
  // the last workgroup to finish commits the step of every grid
  StepSync* sync = uni(A.sync);
  fence_release();
  __syncthreads();
  if (threadIdx.x == 0) {
    s_last = atomicAdd(&sync->done, 1u) == nb - 1;
    fence_acquire();
  }
  __syncthreads();
  if (!s_last) return;
  fence_acquire();
  const bool timed_out = ld_relaxed(&sync->timeout) != 0u;
  DevState* devs = uni(A.devs);
  const int ng = uni(A.n_grids);
  for (int g = threadIdx.x; g < ng; g += blockDim.x) {
    DevState* d = devs + g;
    if (timed_out) {
      // every running grid: an abandoned step may also have flagged other errors on the way
      if (d->active) set_err(d, ERR_SYNC);
    } else {
      commit_grid(d);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int x = 0; x < 8; ++x) st_relaxed(&sync->head[16 * x], 0u);
    st_relaxed(&sync->arrive, 0u);  // already 0 unless a barrier timed out
    st_relaxed(&sync->done, 0u);
    st_relaxed(&sync->timeout, 0u);
    st_relaxed(A.fix_count, 0u);
  }
}

#define AF_STEP_ARGS                                                                          \
  const GridDesc *__restrict__ desc, const int2 *__restrict__ block_tile, int n_tiles,       \
      const int2 *__restrict__ items, int n_items, const int *__restrict__ tile_grid,        \
      const int *__restrict__ prow_grid, const int *__restrict__ prow_base, int n_prows,     \
      DevState *devs, int n_grids, int *fix_list, unsigned int *fix_count, StepSync *sync,   \
      double dt_host, unsigned long long sync_ticks
#define AF_STEP_PASS                                                                          \
  desc, block_tile,                                                                           \
      StepArgs{desc, block_tile, items, tile_grid, prow_grid, prow_base, devs, fix_list,     \
               fix_count, sync, dt_host, sync_ticks, n_tiles, n_items, n_prows, n_grids}

// At least as many waves per SIMD as the point kernels get (left alone, the update phase's
// register budget lowers them: 3 -> 2 in FP32, 2 -> 1 in FP64).
template <bool LIM>
__global__ __launch_bounds__(PT_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
void kb_step_f32(AF_STEP_ARGS) {
  __shared__ Smem<float> S;
  step_body<float, LIM, false>(S, nullptr, AF_STEP_PASS);
}
template <bool LIM>
__global__ __launch_bounds__(PT_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
void kb_step_f64(AF_STEP_ARGS) {
  __shared__ Smem<double> S;
  step_body<double, LIM, false>(S, nullptr, AF_STEP_PASS);
}
template <class R, bool LIM>
__global__ __launch_bounds__(PT_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
void kb_step_ind(AF_STEP_ARGS) {
  __shared__ Smem<R> S;
  __shared__ Ind I;
  step_body<R, LIM, true>(S, &I, AF_STEP_PASS);
}

}  // namespace af

// ==========================================================================================
// Host side
// ==========================================================================================
struct BatchGrid {
  int nx, ny, per_x, per_y, nkx, nky;
  double x0, y0, dx, dy;
  long long pA, pP;        // row pitches (elements)
  size_t oA, oP, oF;       // element offsets of the grid in the packed arrays
  long long pU;            // row pitch of the padded primitive averages (indicators)
  size_t oU;               // element offset of those
  int tile_base, tiles_x, tiles_y;
  bool has_state;
};

struct Batch {
  int n = 0;
  std::vector<BatchGrid> g;
  double* A[2] = {nullptr, nullptr};
  double* K[2] = {nullptr, nullptr};
  double* X[2] = {nullptr, nullptr};
  double* Y[2] = {nullptr, nullptr};
  double* FK = nullptr;
  double* FX = nullptr;
  double* FY = nullptr;
  unsigned long long* fix_mask = nullptr;
  int* fix_list = nullptr;
  unsigned int* fix_count = nullptr;
  GridDesc* d_desc = nullptr;
  int* d_tile_grid = nullptr;
  int2* d_items = nullptr;       // update work items (grid, chunk of bu_threads cell pairs)
  int total_items = 0;           // for the current bu_threads
  double* UB = nullptr;          // padded primitive averages (allocated with the indicators)
  int* d_prow_grid = nullptr;    // grid of every padded row
  int* d_prow_base = nullptr;    // first padded row of every grid
  int total_prows = 0;
  DevState* d_devs = nullptr;
  int total_tiles = 0;
  bool desc_valid = false;
  // schedule: tile order of the point kernel (AF_ORDER_*), workgroup size of the update kernel
  int order = -1;
  int bu_threads = 128;
  int step_kernel = AF_STEP_SPLIT;    // AF_STEP_SPLIT or AF_STEP_PERSISTENT
  af::StepSync* d_sync = nullptr;     // queues and barrier of the persistent step kernel
  int2* d_items_p = nullptr;          // its update items (chunks of PT_THREADS cell pairs)
  int total_items_p = 0;
  int step_cap[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // resident workgroups per step-kernel variant
  int step_nb = 0;                              // workgroups of its next launches
  unsigned long long sync_ticks = 200000000ull;  // its barrier wait limit: 2 s at 100 MHz
  int2* d_block_tile = nullptr;       // (grid, tile within the grid) of every workgroup
  std::vector<long long> grid_tiles;  // tiles per grid (host copy for the orders)
  std::vector<int> tile_grid;         // grid of every global tile (host copy)
  hipGraphExec_t gexec = nullptr;
  int gexec_steps = 0;
};

static size_t round_up(size_t x, size_t m) { return (x + m - 1) / m * m; }

// Update work items for chunks of `pairs` cell pairs (and, in a grid of odd width, chunks of
// `pairs` rows for the last cell of each row): their number, and (with `out`) the table
// (grid, chunk) grid after grid.
static long long update_items(const Batch* b, int pairs, std::vector<int2>* out = nullptr) {
  long long total = 0;
  if (out) out->clear();
  for (int g = 0; g < b->n; ++g) {
    const BatchGrid& q = b->g[g];
    const long long npair = (long long)(q.nx / 2) * q.ny;
    const long long m = (npair + pairs - 1) / pairs + ((q.nx & 1) ? (q.ny + pairs - 1) / pairs : 0);
    if (out)
      for (long long c = 0; c < m; ++c) out->push_back(make_int2(g, (int)c));
    total += m;
  }
  return total;
}

static void batch_free(Batch* b) {
  for (int k = 0; k < 2; ++k) {
    for (double* p : {b->A[k], b->K[k], b->X[k], b->Y[k]})
      if (p) (void)hipFree(p);
  }
  for (void* p : {(void*)b->FK, (void*)b->FX, (void*)b->FY, (void*)b->fix_mask,
                  (void*)b->fix_list, (void*)b->fix_count, (void*)b->d_desc,
                  (void*)b->d_tile_grid, (void*)b->d_items, (void*)b->d_devs,
                  (void*)b->UB, (void*)b->d_prow_grid, (void*)b->d_prow_base,
                  (void*)b->d_block_tile, (void*)b->d_sync, (void*)b->d_items_p})
    if (p) (void)hipFree(p);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  delete b;
}

void batch_invalidate(af_handle* h) {
  if (!h->batch) return;
  h->batch->desc_valid = false;
  if (h->batch->gexec) {
    (void)hipGraphExecDestroy(h->batch->gexec);
    h->batch->gexec = nullptr;
    h->batch->gexec_steps = 0;
  }
}

int batch_count(const af_handle* h) { return h->batch ? h->batch->n : 1; }

// Padded primitive averages of every grid and the padded-row tables (the shock indicators).
int batch_alloc_indicators(af_handle* h) {
  Batch* b = h->batch;
  if (b->UB) return AF_OK;
  size_t nU = 0;
  std::vector<int> pg, pb((size_t)b->n);
  for (int k = 0; k < b->n; ++k) {
    BatchGrid& q = b->g[k];
    q.pU = (q.nx + 4 + 31) / 32 * 32;
    q.oU = nU;
    nU += round_up((size_t)4 * q.pU * (q.ny + 4), 64);
    pb[k] = (int)pg.size();
    pg.insert(pg.end(), (size_t)(q.ny + 4), k);
  }
  HIP_OK(hipMalloc(&b->UB, nU * sizeof(double)), h);
  HIP_OK(hipMalloc(&b->d_prow_grid, pg.size() * sizeof(int)), h);
  HIP_OK(hipMalloc(&b->d_prow_base, pb.size() * sizeof(int)), h);
  HIP_OK(hipMemcpy(b->d_prow_grid, pg.data(), pg.size() * sizeof(int), hipMemcpyHostToDevice), h);
  HIP_OK(hipMemcpy(b->d_prow_base, pb.data(), pb.size() * sizeof(int), hipMemcpyHostToDevice), h);
  b->total_prows = (int)pg.size();
  batch_invalidate(h);
  return AF_OK;
}

void batch_destroy(af_handle* h) {
  if (h->batch) batch_free(h->batch);
  h->batch = nullptr;
}

int batch_create(int n, const af_grid* grids, double gamma, const af_bc* bcs, af_handle* h) {
  Batch* b = new Batch();
  h->batch = b;
  b->n = n;
  b->g.resize(n);
  size_t nA = 0, nP = 0, nF = 0;
  long long tiles = 0;
  for (int k = 0; k < n; ++k) {
    const af_grid& G = grids[k];
    const af_bc& bc = bcs[k];
    BatchGrid& q = b->g[k];
    q.nx = G.nx; q.ny = G.ny;
    q.per_x = bc.left == AF_BC_PERIODIC; q.per_y = bc.bottom == AF_BC_PERIODIC;
    q.nkx = q.nx + (q.per_x ? 0 : 1); q.nky = q.ny + (q.per_y ? 0 : 1);
    q.x0 = G.x0; q.y0 = G.y0;
    q.dx = (G.x1 - G.x0) / G.nx; q.dy = (G.y1 - G.y0) / G.ny;
    q.pA = (q.nx + 31) / 32 * 32;
    q.pP = (q.nkx + 63) / 64 * 64;
    q.oA = nA; q.oP = nP; q.oF = nF;
    nA += round_up((size_t)4 * q.pA * q.ny, 64);
    nP += round_up((size_t)4 * q.pP * q.nky, 64);
    nF += round_up((size_t)q.pP * q.nky, 64);
    q.tiles_x = (q.nkx + TILE - 1) / TILE;
    q.tiles_y = (q.nky + TILE - 1) / TILE;
    q.tile_base = (int)tiles;
    q.pU = 0;
    q.oU = 0;
    tiles += (long long)q.tiles_x * q.tiles_y;
    q.has_state = false;
  }
  if (tiles > INT_MAX / 2)
    return fail(h, AF_ERR_INVALID_ARG, "af_create_batch: too many tiles");
  b->total_tiles = (int)tiles;
  for (int k = 0; k < 2; ++k) {
    HIP_OK(hipMalloc(&b->A[k], nA * 8), h);
    HIP_OK(hipMalloc(&b->K[k], nP * 8), h);
    HIP_OK(hipMalloc(&b->X[k], nP * 8), h);
    HIP_OK(hipMalloc(&b->Y[k], nP * 8), h);
  }
  HIP_OK(hipMalloc(&b->FK, nF * 8 * 8), h);
  HIP_OK(hipMalloc(&b->FX, nF * 4 * 8), h);
  HIP_OK(hipMalloc(&b->FY, nF * 4 * 8), h);
  HIP_OK(hipMalloc(&b->fix_mask, (size_t)tiles * 4 * sizeof(unsigned long long)), h);
  HIP_OK(hipMemset(b->fix_mask, 0, (size_t)tiles * 4 * sizeof(unsigned long long)), h);
  HIP_OK(hipMalloc(&b->fix_list, (size_t)tiles * sizeof(int)), h);
  HIP_OK(hipMalloc(&b->fix_count, sizeof(unsigned int)), h);
  HIP_OK(hipMemset(b->fix_count, 0, sizeof(unsigned int)), h);
  HIP_OK(hipMalloc(&b->d_desc, (size_t)n * sizeof(GridDesc)), h);
  HIP_OK(hipMalloc(&b->d_devs, (size_t)n * sizeof(DevState)), h);
  HIP_OK(hipMemset(b->d_devs, 0, (size_t)n * sizeof(DevState)), h);
  // the grid of every tile
  std::vector<int> tg((size_t)tiles);
  for (int k = 0; k < n; ++k) {
    const BatchGrid& q = b->g[k];
    std::fill(tg.begin() + q.tile_base, tg.begin() + q.tile_base + q.tiles_x * q.tiles_y, k);
  }
  b->grid_tiles.resize(n);
  for (int k = 0; k < n; ++k) b->grid_tiles[k] = (long long)b->g[k].tiles_x * b->g[k].tiles_y;
  HIP_OK(hipMalloc(&b->d_block_tile, tg.size() * sizeof(int2)), h);
  HIP_OK(hipMalloc(&b->d_tile_grid, tg.size() * sizeof(int)), h);
  HIP_OK(hipMemcpy(b->d_tile_grid, tg.data(), tg.size() * sizeof(int), hipMemcpyHostToDevice), h);
  b->tile_grid = tg;
  // update work items: room for the smallest chunk (64 pairs), which gives the most items
  if (update_items(b, 64) > INT_MAX / 2)
    return fail(h, AF_ERR_INVALID_ARG, "af_create_batch: too many cells");
  HIP_OK(hipMalloc(&b->d_items, (size_t)update_items(b, 64) * sizeof(int2)), h);
  {
    std::vector<int2> items;
    b->total_items_p = (int)update_items(b, PT_THREADS, &items);
    HIP_OK(hipMalloc(&b->d_items_p, items.size() * sizeof(int2)), h);
    HIP_OK(hipMemcpy(b->d_items_p, items.data(), items.size() * sizeof(int2),
                     hipMemcpyHostToDevice), h);
  }
  HIP_OK(hipMalloc(&b->d_sync, sizeof(StepSync)), h);
  HIP_OK(hipMemset(b->d_sync, 0, sizeof(StepSync)), h);
  (void)gamma;
  return batch_set_schedule(h, AF_ORDER_XCD, 128, AF_STEP_SPLIT);
}

// Workgroup-to-tile table of the point kernel for a tile order:
//   AF_ORDER_XCD     workgroups are dealt to the 8 XCDs in turn; XCD x takes the contiguous
//                    global tile range [x T/8, (x+1) T/8) (neighbouring tiles share its L2);
//   AF_ORDER_LINEAR  workgroup b takes tile b;
//   AF_ORDER_GRIDS   whole grids are packed onto the XCDs (largest first onto the least loaded),
//                    each XCD working through its grids' tiles in order; a short XCD queue is
//                    topped up from the longest.
static std::vector<int> block_tile_table(const Batch* b, int order) {
  const int T = b->total_tiles;
  std::vector<int> tab((size_t)T);
  if (order == AF_ORDER_LINEAR) {
    for (int k = 0; k < T; ++k) tab[k] = k;
  } else if (order == AF_ORDER_XCD) {
    const int per = T >> 3;
    for (int k = 0; k < T; ++k) tab[k] = k >= (per << 3) ? k : (k & 7) * per + (k >> 3);
  } else {
    std::vector<int> idx((size_t)b->n);
    for (int k = 0; k < b->n; ++k) idx[k] = k;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int x, int y) { return b->grid_tiles[x] > b->grid_tiles[y]; });
    std::vector<std::vector<int>> q(8);
    long long load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int gi : idx) {
      const int x = (int)(std::min_element(load, load + 8) - load);
      load[x] += b->grid_tiles[gi];
      const int base = b->g[gi].tile_base;
      for (long long t = 0; t < b->grid_tiles[gi]; ++t) q[x].push_back(base + (int)t);
    }
    size_t head[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < T; ++k) {
      int x = k & 7;
      if (head[x] >= q[x].size()) {
        size_t best = 0;
        for (int y = 0; y < 8; ++y)
          if (q[y].size() - head[y] > best) { best = q[y].size() - head[y]; x = y; }
      }
      tab[k] = q[x][head[x]++];
    }
  }
  return tab;
}

int batch_set_schedule(af_handle* h, int order, int bu_threads, int step_kernel) {
  Batch* b = h->batch;
  if (order != AF_ORDER_XCD && order != AF_ORDER_LINEAR && order != AF_ORDER_GRIDS)
    return fail(h, AF_ERR_INVALID_ARG, "af_set_option: unknown tile order");
  if (bu_threads != 64 && bu_threads != 128 && bu_threads != 256)
    return fail(h, AF_ERR_INVALID_ARG, "af_set_option: update threads must be 64, 128 or 256");
  if (step_kernel != AF_STEP_SPLIT && step_kernel != AF_STEP_PERSISTENT)
    return fail(h, AF_ERR_INVALID_ARG, "af_set_option: unknown step kernel");
  b->step_kernel = step_kernel;
  if (order != b->order) {
    const std::vector<int> tab = block_tile_table(b, order);
    std::vector<int2> gt(tab.size());
    for (size_t k = 0; k < tab.size(); ++k) {
      const int g = b->tile_grid[tab[k]];
      gt[k] = make_int2(g, tab[k] - b->g[g].tile_base);
    }
    HIP_OK(hipMemcpy(b->d_block_tile, gt.data(), gt.size() * sizeof(int2),
                     hipMemcpyHostToDevice), h);
    b->order = order;
  }
  if (bu_threads != b->bu_threads || b->total_items == 0) {
    std::vector<int2> items;
    b->total_items = (int)update_items(b, bu_threads, &items);
    HIP_OK(hipMemcpy(b->d_items, items.data(), items.size() * sizeof(int2),
                     hipMemcpyHostToDevice), h);
  }
  b->bu_threads = bu_threads;
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->gexec_steps = 0;
  }
  return AF_OK;
}

int batch_set_sync_timeout(af_handle* h, int64_t us) {
  if (us < 0 || us > 100000000)
    return fail(h, AF_ERR_INVALID_ARG, "af_set_option: sync timeout must be 0 .. 1e8 us");
  h->batch->sync_ticks = (unsigned long long)us * 100ull;
  return AF_OK;
}
int64_t batch_get_sync_timeout(const af_handle* h) {
  return (int64_t)(h->batch->sync_ticks / 100ull);
}

int batch_get_schedule(const af_handle* h, int* order, int* bu_threads, int* step_kernel) {
  *order = h->batch->order;
  *bu_threads = h->batch->bu_threads;
  *step_kernel = h->batch->step_kernel;
  return AF_OK;
}

// Descriptors of all grids for the handle's current options (uploaded before a step or run).
static int upload_desc(af_handle* h) {
  Batch* b = h->batch;
  if (b->desc_valid) return AF_OK;
  std::vector<GridDesc> d((size_t)b->n);
  for (int k = 0; k < b->n; ++k) {
    const BatchGrid& q = b->g[k];
    Params& P = d[k].P;
    P.nx = q.nx; P.ny = q.ny; P.nkx = q.nkx; P.nky = q.nky;
    P.per_x = q.per_x; P.per_y = q.per_y;
    P.tiles_x = q.tiles_x; P.tiles_y = q.tiles_y;
    P.dx = q.dx; P.dy = q.dy; P.idx = 1.0 / q.dx; P.idy = 1.0 / q.dy;
    P.gamma = h->gamma; P.hmin = std::min(q.dx, q.dy);
    P.g1inv = 1.0 / (h->gamma - 1.0); P.aspect = q.dx / q.dy;
    P.mode = h->mode; P.correction = h->correction; P.limiter = h->limiter; P.pad = 0;
    P.pA = q.pA; P.sA = q.pA * q.ny;
    P.pP = q.pP; P.sP = q.pP * q.nky;
    P.pF = q.pP; P.sF = q.pP * q.nky;
    fill_sides(h, k, P);
    P.tsw = h->tsw; P.shock = h->shock;
    P.pU = q.pU; P.sU = q.pU * (q.ny + 4);
    for (int in = 0; in < 2; ++in) {
      Bufs& B = d[k].B[in];
      const int out = in ^ 1;
      B.A_in = b->A[in] + q.oA; B.A_out = b->A[out] + q.oA;
      B.K_in = b->K[in] + q.oP; B.X_in = b->X[in] + q.oP; B.Y_in = b->Y[in] + q.oP;
      B.K_out = b->K[out] + q.oP; B.X_out = b->X[out] + q.oP; B.Y_out = b->Y[out] + q.oP;
      B.FK = b->FK + 8 * q.oF; B.FX = b->FX + 4 * q.oF; B.FY = b->FY + 4 * q.oF;
      B.fix_mask = b->fix_mask + 4 * (size_t)q.tile_base;
      B.fix_list = b->fix_list;
      B.fix_count = b->fix_count;
      B.UB = b->UB ? b->UB + q.oU : nullptr;
      B.tile_base = q.tile_base;
    }
    d[k].tile_base = q.tile_base;
  }
  HIP_OK(hipMemcpyAsync(b->d_desc, d.data(), d.size() * sizeof(GridDesc), hipMemcpyHostToDevice,
                        h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  b->desc_valid = true;
  return AF_OK;
}

int64_t batch_dof_count(const af_handle* h) {
  int64_t s = 0;
  for (const BatchGrid& q : h->batch->g)
    s += (int64_t)q.nx * q.ny + (int64_t)q.nkx * q.nky + (int64_t)q.nkx * q.ny +
         (int64_t)q.nx * q.nky;
  return s;
}

static int read_devs(const af_handle* h, std::vector<DevState>& ds) {
  const Batch* b = h->batch;
  ds.resize((size_t)b->n);
  HIP_OK(hipMemcpyAsync(ds.data(), b->d_devs, ds.size() * sizeof(DevState),
                        hipMemcpyDeviceToHost, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  return AF_OK;
}
static int write_devs(af_handle* h, const std::vector<DevState>& ds) {
  HIP_OK(hipMemcpyAsync(h->batch->d_devs, ds.data(), ds.size() * sizeof(DevState),
                        hipMemcpyHostToDevice, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  return AF_OK;
}

int batch_set_state(af_handle* h, int g, const double* avg, const double* K, const double* X,
                    const double* Y, double t, bool user_dev) {
  Batch* b = h->batch;
  if (g < 0 || g >= b->n) return fail(h, AF_ERR_INVALID_ARG, "af_set_state_grid: bad grid index");
  if (!avg || !K || !X || !Y) return fail(h, AF_ERR_INVALID_ARG, "af_set_state_grid: NULL array");
  if (!std::isfinite(t)) return fail(h, AF_ERR_INVALID_ARG, "af_set_state_grid: t not finite");
  BatchGrid& q = b->g[g];
  if (user_dev) {
    if (int e = check_avg_device(h, avg, q.nx, q.ny, "af_set_state_device")) return e;
  } else {
    const size_t nc = (size_t)q.nx * q.ny;
    for (size_t k = 0; k < nc; ++k) {
      const double r = avg[k], E = avg[3 * nc + k];
      const double kin = 0.5 * (avg[nc + k] * avg[nc + k] + avg[2 * nc + k] * avg[2 * nc + k]) / r;
      if (!(r > 0.0) || !((h->gamma - 1.0) * (E - kin) > 0.0))
        return fail(h, AF_ERR_NONPHYSICAL, "af_set_state_grid: non-admissible cell average");
    }
  }
  int e;
  if ((e = copy4(h, true, b->A[0] + q.oA, q.pA, q.ny, q.ny, q.nx, const_cast<double*>(avg),
                 user_dev)))
    return e;
  if ((e = copy4(h, true, b->K[0] + q.oP, q.pP, q.nky, q.nky, q.nkx, const_cast<double*>(K),
                 user_dev)))
    return e;
  if ((e = copy4(h, true, b->X[0] + q.oP, q.pP, q.nky, q.ny, q.nkx, const_cast<double*>(X),
                 user_dev)))
    return e;
  if ((e = copy4(h, true, b->Y[0] + q.oP, q.pP, q.nky, q.nky, q.nx, const_cast<double*>(Y),
                 user_dev)))
    return e;
  DevState ds;
  std::memset(&ds, 0, sizeof(ds));
  ds.t = t;
  ds.t_end = t;
  ds.steps_limit = LLONG_MAX;
  ds.cur = 0;
  HIP_OK(hipMemcpyAsync(b->d_devs + g, &ds, sizeof(ds), hipMemcpyHostToDevice, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  q.has_state = true;
  return AF_OK;
}

int batch_get_state(const af_handle* h, int g, double* avg, double* K, double* X, double* Y,
                    double* t, bool user_dev) {
  const Batch* b = h->batch;
  if (g < 0 || g >= b->n) return fail(h, AF_ERR_INVALID_ARG, "af_get_state_grid: bad grid index");
  const BatchGrid& q = b->g[g];
  if (!q.has_state) return fail(h, AF_ERR_INVALID_ARG, "af_get_state_grid: no state set");
  DevState ds;
  HIP_OK(hipMemcpyAsync(&ds, b->d_devs + g, sizeof(ds), hipMemcpyDeviceToHost, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  const int c = ds.cur;
  int e;
  if (avg && (e = copy4(h, false, b->A[c] + q.oA, q.pA, q.ny, q.ny, q.nx, avg, user_dev)))
    return e;
  if (K && (e = copy4(h, false, b->K[c] + q.oP, q.pP, q.nky, q.nky, q.nkx, K, user_dev)))
    return e;
  if (X && (e = copy4(h, false, b->X[c] + q.oP, q.pP, q.nky, q.ny, q.nkx, X, user_dev)))
    return e;
  if (Y && (e = copy4(h, false, b->Y[c] + q.oP, q.pP, q.nky, q.nky, q.nx, Y, user_dev)))
    return e;
  if (t) *t = ds.t;
  return AF_OK;
}

int batch_totals(const af_handle* h, int g, double* out) {
  const Batch* b = h->batch;
  if (g < 0 || g >= b->n) return fail(h, AF_ERR_INVALID_ARG, "af_get_totals: bad grid index");
  const BatchGrid& q = b->g[g];
  if (!q.has_state) return fail(h, AF_ERR_INVALID_ARG, "af_get_totals: no state set");
  DevState ds;
  HIP_OK(hipMemcpyAsync(&ds, b->d_devs + g, sizeof(ds), hipMemcpyDeviceToHost, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  return reduce_totals(h, h->stream, b->A[ds.cur] + q.oA, q.pA, q.pA * q.ny, q.nx, q.ny,
                       q.dx * q.dy, h->d_totals, out);
}

int batch_grid_info(const af_handle* h, int g, double* t, int64_t* steps) {
  const Batch* b = h->batch;
  if (g < 0 || g >= b->n) return fail(h, AF_ERR_INVALID_ARG, "af_get_grid_info: bad grid index");
  DevState ds;
  HIP_OK(hipMemcpyAsync(&ds, b->d_devs + g, sizeof(ds), hipMemcpyDeviceToHost, h->stream), h);
  HIP_OK(hipStreamSynchronize(h->stream), h);
  if (t) *t = ds.t;
  if (steps) *steps = ds.steps;
  return AF_OK;
}

int batch_get_counters(const af_handle* h, int64_t* out) {
  std::vector<DevState> ds;
  if (int e = read_devs(h, ds)) return e;
  for (int k = 0; k < AF_NCOUNTERS; ++k) out[k] = 0;
  for (const DevState& d : ds) {
    for (int k = 0; k < AF_NCOUNTERS; ++k)
      if (k != AF_CNT_STEPS) out[k] += (int64_t)d.cnt[k];
    out[AF_CNT_STEPS] = std::max<int64_t>(out[AF_CNT_STEPS], d.steps);
  }
  return AF_OK;
}

// Launch of one persistent step-kernel variant with nb workgroups.
template <class K>
static void launch_step(K kernel, const Batch* b, hipStream_t st, int nb, double dt_host) {
  hipLaunchKernelGGL(kernel, dim3(nb), dim3(PT_THREADS), 0, st, b->d_desc, b->d_block_tile,
                     b->total_tiles, b->d_items_p, b->total_items_p, b->d_tile_grid,
                     b->d_prow_grid, b->d_prow_base, b->total_prows, b->d_devs, b->n,
                     b->fix_list, b->fix_count, b->d_sync, dt_host, b->sync_ticks);
}
template <class R>
static void launch_step(const af_handle* h, int nb, double dt_host) {
  const Batch* b = h->batch;
  const bool lim = h->limiter != 0, ind = h->tsw || h->shock;
  if (ind) {
    if (lim) launch_step(kb_step_ind<R, true>, b, h->stream, nb, dt_host);
    else launch_step(kb_step_ind<R, false>, b, h->stream, nb, dt_host);
  } else if constexpr (sizeof(R) == 4) {
    if (lim) launch_step(kb_step_f32<true>, b, h->stream, nb, dt_host);
    else launch_step(kb_step_f32<false>, b, h->stream, nb, dt_host);
  } else {
    if (lim) launch_step(kb_step_f64<true>, b, h->stream, nb, dt_host);
    else launch_step(kb_step_f64<false>, b, h->stream, nb, dt_host);
  }
}

// Workgroups of the persistent step kernel for the handle's options (into b->step_nb): as many
// as the GPU holds at once -- every workgroup must be resident for the kernel's barriers -- or
// fewer if the step has fewer items.
template <class K>
static int resident_blocks(K kernel, int* per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kernel, PT_THREADS, 0) ==
                 hipSuccess
             ? AF_OK
             : AF_ERR_DEVICE;
}
static int prepare_step_kernel(af_handle* h) {
  Batch* b = h->batch;
  if (b->step_kernel != AF_STEP_PERSISTENT) return AF_OK;
  const bool lim = h->limiter != 0, ind = h->tsw || h->shock, f32 = h->prec == AF_PREC_FP32;
  int& cap = b->step_cap[(f32 ? 4 : 0) + (lim ? 2 : 0) + (ind ? 1 : 0)];
  if (cap == 0) {
    int dev = 0, ncu = 0, per = 0, e = AF_OK;
    HIP_OK(hipGetDevice(&dev), h);
    HIP_OK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), h);
    if (ind && f32) e = lim ? resident_blocks(kb_step_ind<float, true>, &per)
                            : resident_blocks(kb_step_ind<float, false>, &per);
    else if (ind) e = lim ? resident_blocks(kb_step_ind<double, true>, &per)
                          : resident_blocks(kb_step_ind<double, false>, &per);
    else if (f32) e = lim ? resident_blocks(kb_step_f32<true>, &per)
                          : resident_blocks(kb_step_f32<false>, &per);
    else e = lim ? resident_blocks(kb_step_f64<true>, &per) : resident_blocks(kb_step_f64<false>, &per);
    if (e != AF_OK || per < 1 || ncu < 1 || per * ncu < 8)
      return fail(h, AF_ERR_DEVICE, "persistent step kernel: occupancy query failed");
    cap = per * ncu / 8 * 8;
  }
  const int work = std::max({b->total_tiles, b->total_items_p, ind ? b->total_prows : 0});
  b->step_nb = std::max(1, std::min(cap, (work + 7) / 8 * 8));
  return AF_OK;
}

// One step of every grid: point kernel, fix-up (limiter on), update, commit; or all of it in
// one launch of the persistent step kernel.
// `ev` (nullable): three events recorded before the point kernel, between the fix-up and the
// update, and after the commit (with the persistent kernel: before it, and twice after it).
template <class R>
static void enqueue_batch_step(af_handle* h, double dt_host, hipEvent_t* ev) {
  Batch* b = h->batch;
  if (ev) (void)hipEventRecord(ev[0], h->stream);
  const bool ind = h->tsw || h->shock;
  if (b->step_kernel == AF_STEP_PERSISTENT) {
    launch_step<R>(h, b->step_nb, dt_host);
    if (ev) {
      (void)hipEventRecord(ev[1], h->stream);
      (void)hipEventRecord(ev[2], h->stream);
    }
    return;
  }
  if (ind) {
    hipLaunchKernelGGL(kb_avgprim, dim3(b->total_prows), dim3(256), 0, h->stream, b->d_desc,
                       b->d_prow_grid, b->d_prow_base, b->d_devs);
    hipLaunchKernelGGL(kb_points_ind<R>, dim3(b->total_tiles), dim3(PT_THREADS), 0, h->stream,
                       b->d_desc, b->d_block_tile, b->d_devs, dt_host);
  } else if constexpr (sizeof(R) == 4) {
    hipLaunchKernelGGL(kb_points_f32, dim3(b->total_tiles), dim3(PT_THREADS), 0, h->stream,
                       b->d_desc, b->d_block_tile, b->d_devs, dt_host);
  } else {
    hipLaunchKernelGGL(kb_points_f64, dim3(b->total_tiles), dim3(PT_THREADS), 0, h->stream,
                       b->d_desc, b->d_block_tile, b->d_devs, dt_host);
  }
  if (h->limiter) {
    const int nb = std::min(b->total_tiles, FIX_BLOCKS);
    if (ind)
      hipLaunchKernelGGL(kb_fixup_ind<R>, dim3(nb), dim3(PT_THREADS), 0, h->stream, b->d_desc,
                         b->d_tile_grid, b->d_devs, b->fix_list, b->fix_count);
    else if constexpr (sizeof(R) == 4)
      hipLaunchKernelGGL(kb_fixup_f32, dim3(nb), dim3(PT_THREADS), 0, h->stream, b->d_desc,
                         b->d_tile_grid, b->d_devs, b->fix_list, b->fix_count);
    else
      hipLaunchKernelGGL(kb_fixup_f64, dim3(nb), dim3(PT_THREADS), 0, h->stream, b->d_desc,
                         b->d_tile_grid, b->d_devs, b->fix_list, b->fix_count);
  }
  if (ev) (void)hipEventRecord(ev[1], h->stream);
  if (b->bu_threads == 64)
    hipLaunchKernelGGL(kb_update<64>, dim3(b->total_items), dim3(64), 0, h->stream, b->d_desc,
                       b->d_items, b->total_items, b->d_devs);
  else if (b->bu_threads == 256)
    hipLaunchKernelGGL(kb_update<256>, dim3(b->total_items), dim3(256), 0, h->stream, b->d_desc,
                       b->d_items, b->total_items, b->d_devs);
  else
    hipLaunchKernelGGL(kb_update<128>, dim3(b->total_items), dim3(128), 0, h->stream, b->d_desc,
                       b->d_items, b->total_items, b->d_devs);
  hipLaunchKernelGGL(kb_commit, dim3((b->n + 63) / 64), dim3(64), 0, h->stream, b->d_devs, b->n,
                     b->fix_count);
  if (ev) (void)hipEventRecord(ev[2], h->stream);
}
static void enqueue_batch(af_handle* h, double dt_host) {
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  if (h->timing) {
    for (hipEvent_t& e : ev) (void)hipEventCreate(&e);
  }
  if (h->prec == AF_PREC_FP32) enqueue_batch_step<float>(h, dt_host, h->timing ? ev : nullptr);
  else enqueue_batch_step<double>(h, dt_host, h->timing ? ev : nullptr);
  if (h->timing)
    for (hipEvent_t e : ev) h->ev.push_back(e);
}

// Mean times of the point and of the update kernel (ms) over `steps` eager steps of the run.
static int time_steps(af_handle* h, int steps, double* ms_points, double* ms_update) {
  std::vector<hipEvent_t> ev((size_t)3 * steps);
  for (hipEvent_t& e : ev) HIP_OK(hipEventCreate(&e), h);
  for (int s = 0; s < steps; ++s) {
    if (h->prec == AF_PREC_FP32) enqueue_batch_step<float>(h, 0.0, &ev[3 * s]);
    else enqueue_batch_step<double>(h, 0.0, &ev[3 * s]);
  }
  HIP_OK(hipStreamSynchronize(h->stream), h);
  double a = 0.0, c = 0.0;
  for (int s = 0; s < steps; ++s) {
    float x = 0.f, y = 0.f;
    (void)hipEventElapsedTime(&x, ev[3 * s], ev[3 * s + 1]);
    (void)hipEventElapsedTime(&y, ev[3 * s + 1], ev[3 * s + 2]);
    a += x;
    c += y;
  }
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  *ms_points = a / steps;
  *ms_update = c / steps;
  return AF_OK;
}

// Autotuner, on `per` steps of the run per trial (every schedule computes the same values):
// with separate kernels, time each tile order of the point kernel, then each workgroup size of
// the update kernel; then the persistent step kernel with each tile order.  Keeps the schedule
// with the shortest step.
static int autotune(af_handle* h, int per) {
  Batch* b = h->batch;
  const int orders[3] = {AF_ORDER_XCD, AF_ORDER_LINEAR, AF_ORDER_GRIDS};
  const int threads[3] = {64, 128, 256};
  double best = INFINITY, mp = 0.0, mu = 0.0;
  int best_order = b->order;
  if (int e = batch_set_schedule(h, b->order, b->bu_threads, AF_STEP_SPLIT)) return e;
  if (int e = time_steps(h, 1, &mp, &mu)) return e;  // warm-up
  for (int o : orders) {
    if (int e = batch_set_schedule(h, o, b->bu_threads, AF_STEP_SPLIT)) return e;
    if (int e = time_steps(h, per, &mp, &mu)) return e;
    if (mp < best) { best = mp; best_order = o; }
  }
  double split = INFINITY;
  int best_threads = b->bu_threads;
  for (int t : threads) {
    if (int e = batch_set_schedule(h, best_order, t, AF_STEP_SPLIT)) return e;
    if (int e = time_steps(h, per, &mp, &mu)) return e;
    if (mp + mu < split) { split = mp + mu; best_threads = t; }
  }
  double fused = INFINITY;
  int fused_order = best_order, e_warm = AF_OK;
  for (int o : orders) {
    if (int e = batch_set_schedule(h, o, best_threads, AF_STEP_PERSISTENT)) return e;
    if (int e = prepare_step_kernel(h)) return e;
    if (o == orders[0] && (e_warm = time_steps(h, 1, &mp, &mu))) return e_warm;
    if (int e = time_steps(h, per, &mp, &mu)) return e;
    if (mp + mu < fused) { fused = mp + mu; fused_order = o; }
  }
  if (fused < split) {
    if (int e = batch_set_schedule(h, fused_order, best_threads, AF_STEP_PERSISTENT)) return e;
    return prepare_step_kernel(h);
  }
  return batch_set_schedule(h, best_order, best_threads, AF_STEP_SPLIT);
}

// Add the event times of the first `used` enqueued steps (those in which some grid advanced;
// the launches after every grid has stopped return at once and are not counted).
static void collect_batch_timing(af_handle* h, long long used) {
  for (size_t k = 0; k + 2 < h->ev.size() && (long long)(k / 3) < used; k += 3) {
    float a = 0.f, c = 0.f;
    if (hipEventElapsedTime(&a, h->ev[k], h->ev[k + 1]) == hipSuccess &&
        hipEventElapsedTime(&c, h->ev[k + 1], h->ev[k + 2]) == hipSuccess) {
      h->ms_points += a;
      h->ms_update += c;
      h->timed_steps += 1;
    }
  }
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
}

static const char* batch_err_text(int code) {
  switch (code) {
    case ERR_NONPHYS: return "non-positive density or pressure";
    case ERR_CFL: return "time step too large: an evolution circle leaves its cells";
    case ERR_SYNC: return "persistent step kernel: a grid barrier timed out (not all workgroups "
                          "were resident); the step was not committed";
    default: return "device error";
  }
}

// the most negative error over the grids (CFL before NONPHYSICAL), and the first grid with it
static int first_error(const std::vector<DevState>& ds, int* grid) {
  int e = 0;
  for (size_t k = 0; k < ds.size(); ++k)
    if (ds[k].err < e) { e = ds[k].err; *grid = (int)k; }
  return e;
}

static int check_all_state(const af_handle* h, const char* fn) {
  for (const BatchGrid& q : h->batch->g)
    if (!q.has_state) return fail(h, AF_ERR_INVALID_ARG, std::string(fn) + ": a grid has no state");
  return AF_OK;
}

int batch_step(af_handle* h, double dt) {
  if (int e = check_all_state(h, "af_step")) return e;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(h, AF_ERR_INVALID_ARG, "af_step: dt must be > 0");
  if (int e = upload_desc(h)) return e;
  if (int e = prepare_step_kernel(h)) return e;
  std::vector<DevState> ds;
  if (int e = read_devs(h, ds)) return e;
  for (DevState& d : ds) {
    d.err = 0;
    d.steps_limit = LLONG_MAX;
  }
  if (int e = write_devs(h, ds)) return e;
  enqueue_batch(h, dt);
  HIP_OK(hipGetLastError(), h);
  std::vector<long long> before((size_t)h->batch->n);
  for (size_t k = 0; k < ds.size(); ++k) before[k] = ds[k].steps;
  if (int e = read_devs(h, ds)) return e;
  if (h->timing) {
    long long used = 0;
    for (size_t k = 0; k < ds.size(); ++k) used = std::max(used, ds[k].steps - before[k]);
    collect_batch_timing(h, used);
  }
  int g = 0;
  if (int e = first_error(ds, &g))
    return fail(h, e, "af_step: grid " + std::to_string(g) + ": " + batch_err_text(e));
  return AF_OK;
}

int batch_run(af_handle* h, double t_end, double cfl, int64_t max_steps, double* t_reached,
              int64_t* steps_taken) {
  if (int e = check_all_state(h, "af_run")) return e;
  if (!(cfl > 0.0) || !(cfl < 0.5)) return fail(h, AF_ERR_INVALID_ARG, "af_run: cfl must be in (0, 0.5)");
  if (std::isnan(t_end)) return fail(h, AF_ERR_INVALID_ARG, "af_run: t_end is NaN");
  Batch* b = h->batch;
  if (int e = upload_desc(h)) return e;
  if (int e = prepare_step_kernel(h)) return e;
  std::vector<DevState> ds;
  if (int e = read_devs(h, ds)) return e;
  std::vector<long long> steps0((size_t)b->n);
  for (int k = 0; k < b->n; ++k) {
    DevState& d = ds[k];
    steps0[k] = d.steps;
    d.err = 0;
    d.t_end = t_end;
    d.cfl = cfl;
    d.smax[0] = d.smax[1] = 0ull;
    d.active = 0;
    d.steps_limit = max_steps > 0 ? d.steps + max_steps : LLONG_MAX;
  }
  if (int e = write_devs(h, ds)) return e;
  const int per = 16;
  hipLaunchKernelGGL(kb_cfl, dim3(b->n * per), dim3(256), 0, h->stream, b->d_desc, b->d_devs, per);
  HIP_OK(hipGetLastError(), h);
  if (h->autotune == 1) {
    if (int e = autotune(h, 2)) return e;
    h->autotune = 2;  // done; the chosen schedule stays
    if (int e = read_devs(h, ds)) return e;
  }
  const long long chunk = h->graph_steps > 0 ? h->graph_steps : 8;
  std::vector<long long> before((size_t)b->n);
  while (true) {
    for (int k = 0; k < b->n; ++k) before[k] = ds[k].steps;
    // every grid stops by itself at t_end or at its step limit; the host only checks between
    // chunks whether any grid is still running or has failed.  No more steps are launched
    // than the step limit leaves to any running grid: a shorter rest goes out without a graph.
    long long n_launch = chunk;
    if (max_steps > 0) {
      long long rest = 0;
      for (int k = 0; k < b->n; ++k)
        if (!ds[k].err && ds[k].t < t_end) rest = std::max(rest, ds[k].steps_limit - ds[k].steps);
      n_launch = std::min(chunk, rest);
    }
    if (h->timing || n_launch < chunk) {
      for (long long s = 0; s < n_launch; ++s) enqueue_batch(h, 0.0);
    } else {
      if (!b->gexec || b->gexec_steps != chunk) {
        if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
        hipGraph_t gr;
        HIP_OK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), h);
        for (long long s = 0; s < chunk; ++s) enqueue_batch(h, 0.0);
        HIP_OK(hipStreamEndCapture(h->stream, &gr), h);
        HIP_OK(hipGraphInstantiate(&b->gexec, gr, nullptr, nullptr, 0), h);
        (void)hipGraphDestroy(gr);
        b->gexec_steps = (int)chunk;
      }
      HIP_OK(hipGraphLaunch(b->gexec, h->stream), h);
    }
    HIP_OK(hipGetLastError(), h);
    if (int e = read_devs(h, ds)) return e;
    if (h->timing) {
      long long used = 0;
      for (int k = 0; k < b->n; ++k) used = std::max(used, ds[k].steps - before[k]);
      collect_batch_timing(h, used);
    }
    double tmin = INFINITY;
    long long smax = 0;
    bool running = false;
    for (int k = 0; k < b->n; ++k) {
      tmin = std::min(tmin, ds[k].t);
      smax = std::max(smax, ds[k].steps - steps0[k]);
      if (ds[k].t < t_end && ds[k].steps < ds[k].steps_limit) running = true;
    }
    if (t_reached) *t_reached = tmin;
    if (steps_taken) *steps_taken = smax;
    int g = 0;
    if (int e = first_error(ds, &g))
      return fail(h, e, "af_run: grid " + std::to_string(g) + ": " + batch_err_text(e));
    if (!running) break;
  }
  return AF_OK;
}
