// pa_host.h -- host-side objects behind the opaque C-ABI handles, shared by
// api.cpp (validation, single-step entry points) and solve.cpp (graph-captured
// solves and batches).
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/pa.h"
#include "pa_internal.h"

namespace pa {
struct SolvePlan;   // solve.cpp: a captured, replayable solve of one or more instances
void free_plan(SolvePlan *plan);
}  // namespace pa

struct pa_context {
  int device = 0;
  pa::DeviceInfo info;
  hipStream_t stream = nullptr;          // library-internal work and graph capture
  pa::SolvePlan *batch_plan = nullptr;   // last pa_solve_batch plan (replayed when unchanged)
  void *scratch = nullptr;               // device address of the device's no-allocation scratch
};

struct pa_instance {
  pa_context *ctx = nullptr;
  pa::DevProblem p;
  int M = 1;
  double rho = 1.0;
  int T = 0;
  bool has_pos = false;
  // solve work buffers (grown on demand)
  int work_N = 0, work_G = -1;
  uint8_t *popA = nullptr, *popB = nullptr;
  float *fitA = nullptr, *fitB = nullptr;
  float *trace = nullptr;
  int32_t *best_idx = nullptr;
  float *best_fit = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  pa::SolvePlan *plan = nullptr;  // last pa_solve plan (replayed when params are unchanged)
};


namespace pa {
// Error reporting shared by the host files (thread-local message).
pa_status set_error(pa_status s, const char *fmt, ...);
pa_status hip_error(hipError_t e, const char *what);
pa_status validate_ga(const pa_instance *inst, const pa_ga_params *g);
DevGa ga_from_params(const pa_ga_params *g);
pa_status ensure_work(pa_instance *in, int N, int G);
pa_status use_device(pa_context *ctx);
// Launch shape of a class of instances for the generation kernel: threads
// per workgroup (maxK = the largest K of the class), and workgroups for
// ntasks tasks (0 when the table does not fit LDS).
int gen_class_block(int L, int TP, int mode, int maxK);
int gen_class_grid(int L, int TP, int mode, int block, int ntasks, int cus);
// Workgroups of the class's generation kernel at `block` threads that one CU
// holds at once (occupancy query, cached; 0 when none fits).
int gen_class_per_cu(int L, int TP, int mode, int block);
// Device address of the no-allocation scratch array of `device` (looked up
// once per device, with that device current); its lookup error otherwise.
hipError_t noalloc_scratch(int device, void **ptr);
}  // namespace pa
