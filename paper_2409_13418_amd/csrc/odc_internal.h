// Host-side declarations shared by the ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "odc_device.h"
#include "odc_job.h"
#include "odc_mlp.h"

namespace odc {

// Persistent grid sizes (blocks of 256 threads) per kind of kernel; chosen
// by the autotuner.
struct LaunchCfg {
  int grid_blocks = 2048;  // grid-wide passes: CSG labels, classification, compaction
  int elem_blocks = 4096;  // thread-per-element passes over active sets
  int mlp_blocks = 256;    // wavefront-per-32-elements MLP passes (LDS-bound: 1 block/CU)
  int scan_blocks = 512;
  int pack_blocks = 512;
};

// Resolution buckets of the autotuner's cache: res <= 64, <= 128, <= 256,
// above.
constexpr int kResBuckets = 4;
inline int res_bucket(int res) { return res <= 64 ? 0 : (res <= 128 ? 1 : (res <= 256 ? 2 : 3)); }

// Which kernels a launch needs.
struct PipelineShape {
  bool any_csg = false, any_mlp = false, any_mlp_fp32 = false, any_mlp_bf16 = false;
  bool any_mlp_x3 = false;  // split-bf16 precision
  bool any_grad = false;  // some job takes gradient normals
  bool any_coarse = false;  // some job evaluates its corners coarse to fine
};

// The whole path for njobs jobs in device memory; ev (9 events, or NULL)
// marks the stage boundaries.  No host synchronisation inside.
hipError_t launch_pipeline(const Job* d, int njobs, const PipelineShape& sh,
                           const float* const* d_weights, const uint32_t* table,
                           const LaunchCfg& cfg, hipEvent_t* ev, hipStream_t s);
// kGatherWords x uint64 per job: edges, pairs, cells, partition vertices,
// triangles, case-3 vertices, guard corners, fp64 cells | overflow << 32,
// 2D-search queries made (MLP), corner queries (adaptive evaluation),
// flipped faces
constexpr int kGatherWords = 11;
hipError_t launch_gather(const Job* d, int njobs, unsigned long long* out, hipStream_t s);
hipError_t launch_eval(const Job* d_job, const Job& h_job, const float* const* d_weights,
                       int precision, const float* xyz, int n, float* z, const LaunchCfg& cfg,
                       hipStream_t s);
hipError_t launch_partition_table(uint32_t* table, hipStream_t s);

}  // namespace odc
