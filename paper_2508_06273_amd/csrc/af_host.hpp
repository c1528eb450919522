// af_host.hpp -- host-side state of a handle and helpers shared by the single-grid and the
// batched runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <string>
#include <vector>

#include "af.h"
#include "af_kernels.hpp"

using namespace af;

// A roctx range over a scope: the library's calls appear by name on the host timeline of
// `rocprofv3 --marker-trace`, around the kernels they enqueue; next to no cost without a
// profiler.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

struct Batch;  // batched grids (af_batch.hip)

// Boundary of one grid: kind per side (left, right, bottom, top; a periodic axis has
// AF_BC_PERIODIC on both sides) and the inflow states (`set`: bit s = inflow[s] given).
struct Sides {
  int bc[4] = {0, 0, 0, 0};
  double inflow[4][4] = {};
  unsigned set = 0;
};

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
  GridDesc* d_desc = nullptr;  // device copy of the parameters and buffers (point kernels)
  double* d_totals = nullptr;  // partial sums and result of af_get_totals (allocated on first use)
  bool desc_valid = false;
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
  Batch* batch = nullptr;   // several grids (af_create_batch); nullptr for one grid
  int autotune = 0;         // batched: 1 = tune the schedule at the next af_run, 2 = tuned
  std::vector<Sides> sides;  // per grid
  int* d_flag = nullptr;     // device flag of check_avg_device
  int tsw = 0, shock = 0;    // Algorithm 2; the shock-indicator blend
  double* UB = nullptr;      // padded primitive averages for the indicators
  int flux_limiter = 0;      // flux limiting of the averages (Sec. 3.5)
  double* TH = nullptr;      // its face weights: 4 planes of ny x pA
  long long pU = 0;
  std::string err;
};

// Error text of the last failed call (per handle; af_create's in a process-wide string).
extern std::string g_create_error;
int fail(const af_handle* h, int code, const std::string& msg);

#define HIP_OK(call, h)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(h, e_ == hipErrorOutOfMemory ? AF_ERR_OOM : AF_ERR_DEVICE,         \
                  std::string(#call) + ": " + hipGetErrorString(e_));                \
  } while (0)


// Host <-> device copies through the handle's pinned staging buffer (synchronous on the
// handle's stream): one variable of rows x cols (host unpadded, device with a row pitch), or
// the four variables of a padded array (variable v at offset v * rows_alloc * pitch).
// `user_dev`: the caller's array is in device memory (copied device to device, no staging).
int copy2d(const af_handle* h, bool to_device, double* dev, long long pitch, int rows, int cols,
           double* host, bool user_dev = false);
int copy4(const af_handle* h, bool to_device, void* dev, long long pitch, int rows_alloc,
          int rows, int cols, double* host, bool user_dev = false);
// Are all nx * ny conserved averages of the caller's device array (4 x ny x nx) admissible?
int check_avg_device(const af_handle* h, const double* avg, int nx, int ny, const char* fn);

// Boundary kinds and inflow states of grid g into P.
void fill_sides(const af_handle* h, int g, Params& P);

// Batched handles (af_batch.hip): the public entry points hand over to these when h->batch.
int batch_create(int n, const af_grid* grids, double gamma, const af_bc* bcs, af_handle* h);
void batch_destroy(af_handle* h);
int batch_count(const af_handle* h);
int batch_alloc_indicators(af_handle* h);
void batch_invalidate(af_handle* h);
int64_t batch_dof_count(const af_handle* h);
int batch_set_state(af_handle* h, int g, const double* avg, const double* K, const double* X,
                    const double* Y, double t, bool user_dev = false);
int batch_get_state(const af_handle* h, int g, double* avg, double* K, double* X, double* Y,
                    double* t, bool user_dev = false);
int batch_grid_info(const af_handle* h, int g, double* t, int64_t* steps);
int batch_get_counters(const af_handle* h, int64_t* out);
int batch_step(af_handle* h, double dt);
int batch_set_schedule(af_handle* h, int order, int bu_threads, int step_kernel);
int batch_get_schedule(const af_handle* h, int* order, int* bu_threads, int* step_kernel);
int batch_set_sync_timeout(af_handle* h, int64_t us);
int batch_totals(const af_handle* h, int g, double* out);
int64_t batch_get_sync_timeout(const af_handle* h);
int batch_run(af_handle* h, double t_end, double cfl, int64_t max_steps, double* t_reached,
              int64_t* steps_taken);

// Domain totals (sum over cells of the conserved averages, times the cell area) of one grid's
// averages A (4 variables at stride sA, rows at pitch pA), by the deterministic two-pass
// reduction of af_lib.hip; synchronous on `stream`.  `scratch`: TOTAL_BLOCKS * 4 + 4 doubles.
constexpr int TOTAL_BLOCKS = 256;
int reduce_totals(const af_handle* h, hipStream_t stream, const double* A, long long pA,
                  long long sA, int nx, int ny, double area, double* scratch, double* out);
