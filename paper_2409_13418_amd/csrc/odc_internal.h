// Host-side declarations shared by the ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "odc_device.h"
#include "odc_mlp.h"

namespace odc {

// Device state of one meshing job: inputs, active sets and outputs.
struct Job {
  Grid g;
  int kind;            // ODC_FIELD_*
  int precision;       // ODC_PREC_*
  const float* prims;  // CSG
  int n_prims;
  Mlp mlp;             // MLP (packed weights in scratch)
  int iters_1d, lin1, bin1, lin2, bin2;
  float range1, range2, qef_tau, guard_logit;
  double fp64_cond;

  // corner labels
  uint32_t* labels;      // ceil(nc/32) words
  // crossing edges: mask, per-word count/prefix, list, 1D points
  uint32_t* emask;
  uint32_t* eprefix;     // exclusive prefix per word (+ total at [nwords])
  int* elist;
  float* et;
  // faces: active (>= 1 pair), ambiguous (2 pairs), flipped
  uint32_t* fact;
  uint32_t* famb;
  uint32_t* fflip;
  uint32_t* pprefix;     // pairs before each word (+ total)
  int* plist;            // face << 1 | slot
  double2* pf;           // 2D points, face-local (binary64: see search_pair)
  // cells
  uint32_t* cmask;
  uint32_t* cprefix;
  int* clist;
  uint32_t* cpm;         // partmap per active cell
  uint32_t* cnf;         // npart | flipmask << 4
  uint32_t* vbase;       // exclusive prefix of npart (+ total)
  float* vloc;           // 3 floats per partition vertex, cell-local
  // emission
  uint32_t* ecase;       // per crossing edge: case (0..3)
  uint32_t* tprefix;     // triangles before each crossing edge (+ total)
  uint32_t* c3prefix;    // case-3 vertices before each crossing edge (+ total)
  int4* quad;            // oriented vertex ids per crossing edge
  // outputs
  float* out_v;
  int64_t cap_v;
  int* out_t;
  int64_t cap_t;
  float* out_vloc;
  int* out_vref;
  // device counters: [0] guard corners, [1] fp64 cells, [2] queries
  unsigned long long* counters;
  uint32_t* guard_list;  // corners queued for fp32 re-evaluation
  int guard_cap;
  // host copies of active sizes (after classification)
  int n_edges, n_pairs, n_cells;
};

// scan: out[i] = sum in[0..i), out[n] = total (uint32); tmp >= scan_tmp_words(n)
size_t scan_tmp_words(int n);
hipError_t scan_exclusive(const uint32_t* in, uint32_t* out, int n, uint32_t* tmp,
                          hipStream_t s);

hipError_t launch_pack_mlp(const float* weights, int in_dim, int depth, float* w1f, float* whf,
                           v8bf* w1b, v8bf* whb, float* bias, float* wout, hipStream_t s);
hipError_t launch_labels(Job& j, hipStream_t s);
hipError_t launch_classify(Job& j, uint32_t* ecount, uint32_t* pcount, uint32_t* ccount,
                           const uint32_t* part_table, hipStream_t s);
hipError_t launch_compact(Job& j, hipStream_t s);
hipError_t launch_bisect(Job& j, hipStream_t s);
hipError_t launch_search2d(Job& j, hipStream_t s);
hipError_t launch_cell_count(Job& j, uint32_t* npart, const uint32_t* part_table, hipStream_t s);
hipError_t launch_cell_qef(Job& j, hipStream_t s);
hipError_t launch_emit_count(Job& j, uint32_t* ntri, uint32_t* n3, hipStream_t s);
hipError_t launch_emit_write(Job& j, hipStream_t s);
hipError_t launch_eval(int kind, int precision, const float* prims, int np, const Mlp& m,
                       const float* xyz, int n, float* z, hipStream_t s);

}  // namespace odc
