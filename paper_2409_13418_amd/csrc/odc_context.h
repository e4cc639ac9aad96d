// Host-side state of an extraction context, shared by the extraction calls
// (odc_api.hip) and the serving loop (odc_server.hip).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/odc.h"
#include "odc_internal.h"

namespace odc {

// Device buffer that only grows.  Growing waits for the stream first, so no
// queued kernel still uses the old allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Scratch of one job slot.  A context owns its slots' buffers, except in a
// server lane, where each job's scratch is one block of the server's arena
// (ext), sized for ext_cap_edges crossing edges.
struct Slot {
  DevBuf grid;    // bit sets, word counts, prefixes, scan block sums
  DevBuf active;  // active-set arrays
  DevBuf mlpw;    // packed MLP weights
  DevBuf guard;   // bf16 guard queue
  DevBuf status;  // 9 x uint64
  int cap_edges = 0;
  bool guard_full = false;
  char* ext = nullptr;
  size_t ext_bytes = 0;
  int ext_cap_edges = 0;
};

constexpr int kMaxJobs = 1024;

}  // namespace odc

struct odc_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t capture_stream = nullptr;
  std::string err;
  std::vector<odc::Slot> slots;
  odc::DevBuf djobs, dweights, dgather, table;
  odc::Job* hjobs = nullptr;               // pinned
  const float** hweights = nullptr;        // pinned
  unsigned long long* hgather = nullptr;   // pinned, kGatherWords per job
  odc::LaunchCfg cfg;
  // autotuned launch shapes per (field kind, resolution bucket), filled by
  // odc_autotune; an extraction uses the entry of its dominant job, else cfg
  odc::LaunchCfg tuned[2][odc::kResBuckets];
  bool tuned_ok[2][odc::kResBuckets] = {};
  bool tuning = false;  // odc_autotune is timing candidates in cfg
  double cap_scale = 1.0;
  bool trace = false;  // record decision traces of the searches
  // the device's fixed scratch array (odc_mesh_extract_noalloc), and whether
  // the pending extract lives in it (then it is never regrown or rerun)
  void* fixed_scratch = nullptr;
  std::string fixed_err;
  bool pending_fixed = false;
  // timing
  bool timing = false;
  hipEvent_t ev[9] = {};
  // graph replay
  bool use_graph = false;
  hipGraphExec_t graph = nullptr;
  int graph_njobs = -1;
  odc::PipelineShape graph_shape;
  odc::LaunchCfg graph_cfg;
  const void* graph_ptrs[3] = {nullptr, nullptr, nullptr};
  // the pending batch (kept to rerun it after a scratch overflow)
  int pending = 0;
  std::vector<odc_field> p_fields;
  std::vector<odc_params> p_params;
  std::vector<odc_mesh_buffers> p_outs;
};

namespace odc {

// hipMalloc unless failure injection (odc_inject_alloc_failures) refuses it.
hipError_t device_alloc(void** p, size_t bytes);
// Sets ctx->err (when ctx is not NULL) and returns code.
int32_t ctx_fail(odc_context* ctx, int32_t code, const char* fmt, ...);
// Argument checks of one job.
int32_t validate_job(odc_context* ctx, const odc_field* f, const odc_params* p,
                     const odc_mesh_buffers* o);
// Crossing-edge capacity planned for a grid of N cells per axis.
int estimate_edges(double cap_scale, int N);
// Device scratch of one job with the given crossing-edge capacity.
size_t job_scratch_bytes(const odc_field* f, const odc_params* p, int cap_edges, bool guard_full);
// Uploads and launches n jobs on the context stream (asynchronous); the
// gathered counts land in ctx->hgather when the stream reaches that point.
int32_t enqueue_batch(odc_context* ctx, int n, const odc_field* fields, const odc_params* params,
                      const odc_mesh_buffers* outs);
// Counts of job k of the last batch, from ctx->hgather.
void fill_counts(const odc_context* ctx, int k, odc_mesh_counts* c);
// After a scratch overflow: the crossing-edge capacity job k needed, and
// whether its bf16 guard queue overflowed.
int needed_edges(const odc_context* ctx, int k, bool* guard_over);
// Whether job k of the last batch overflowed its scratch.
bool job_overflowed(const odc_context* ctx, int k);

}  // namespace odc
