// One meshing job as the kernels see it, and the job-major work distribution
// shared by every kernel.
//
// A launch serves an array of jobs in device memory (one for odc_mesh_extract,
// many for odc_mesh_extract_batch).  Each kernel is persistent: a fixed grid of
// workers (threads, wavefronts or blocks) walks the jobs in order and, inside
// each job, the units of that stage; unit u of job k goes to worker
// (u + rot_k) mod W where rot_k counts the units of the jobs before k, so
// small jobs spread over the whole grid instead of piling onto the first
// workers.  Active-set sizes come from device memory (the scans' totals),
// clamped to the job's scratch capacities: nothing ever indexes past them,
// and an overflow is flagged for the host to grow the scratch and run again.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "odc_device.h"
#include "odc_mlp.h"

namespace odc {

// ablation bits of a job (the public ODC_ABL_* values)
constexpr int kAblLinear1D = 1, kAblGradNormals = 2, kAblMdcSplit = 4, kAblSdfInput = 8;

struct Job {
  Grid g;
  int kind;       // 0 CSG, 1 MLP
  int precision;  // 0 fp32, 1 bf16 guarded
  const float* prims;
  int n_prims;
  Mlp mlp;
  int iters_1d, lin1, bin1, lin2, bin2;
  float range1, range2, qef_tau, guard_logit;
  double fp64_cond;
  int ablation;   // ODC_ABL_* bits (0 = the method)
  int clamp;      // clamp 3D points into their cells
  // adaptive corner evaluation (coarse_step > 1): coarse grid of cn cells per
  // axis (cn + 1 corners); bit sets of the coarse corners' labels, of those
  // within the logit band, and of the marked coarse cells
  int coarse_step, cn;
  float coarse_band;
  uint32_t* cbits;
  uint32_t* cnear;
  uint32_t* cmark;
  int* wlist;  // the fine label words that need the field (count in status[5])

  int nw_c, nw_e, nw_f, nw_cell;       // words of the corner / edge / face / cell bit sets
  int cap_edges, cap_pairs, cap_cells;  // active-set scratch capacities

  // grid-wide bit sets and word counts / exclusive prefixes (+ total)
  uint32_t* labels;
  uint32_t* emask;
  uint32_t* ecount;
  uint32_t* eprefix;
  uint32_t* fact;  // faces with >= 1 pair
  uint32_t* famb;  // faces with 2 pairs
  uint32_t* fflip; // faces taking the manifold-fix pairing
  uint32_t* pcount;
  uint32_t* pprefix;
  uint32_t* cmask;
  uint32_t* ccount;
  uint32_t* cprefix;
  uint32_t* scan_tmp;

  // active sets
  int* elist;
  float* et;
  uint32_t* ecase;
  uint32_t* ntri;
  uint32_t* n3;
  uint32_t* tprefix;
  uint32_t* c3prefix;
  int4* quad;
  int* plist;
  double2* pf;
  int* clist;
  uint32_t* cpm;
  uint32_t* cnf;
  uint32_t* npart;
  uint32_t* vbase;
  float* vloc;
  float* egrad;  // dz/dx at each crossing edge's 1D point (gradient-normal ablation)
  // decision traces (NULL unless the context records them): the label of
  // every bisection query per crossing edge, and per pair the labels and the
  // evaluated-query mask of its 2D search
  uint32_t* etrace;
  unsigned long long* ptrace;

  // outputs (caller memory)
  float* out_v;
  int64_t cap_v;
  int* out_t;
  int64_t cap_t;
  float* out_vloc;
  int* out_vref;

  // [0] guard corners, [1] fp64 cells, [2] overflow, [3] 2D-search queries,
  // [4] corner queries, [5] listed fine words (adaptive evaluation),
  // [6] flipped faces, [7] 2D-search units taken, [8] bisection units taken
  unsigned long long* status;
  uint32_t* guard_list;
  int guard_cap;
};

__device__ __forceinline__ int clampi(uint32_t v, int cap) {
  return (int)v < cap ? (int)v : cap;
}
__device__ __forceinline__ int n_edges_of(const Job& J) {
  return clampi(J.eprefix[J.nw_e], J.cap_edges);
}
__device__ __forceinline__ int n_pairs_of(const Job& J) {
  return clampi(J.pprefix[J.nw_f], J.cap_pairs);
}
__device__ __forceinline__ int n_cells_of(const Job& J) {
  return clampi(J.cprefix[J.nw_cell], J.cap_cells);
}

// index of crossing edge `id` in the active list (clamped into the scratch)
__device__ __forceinline__ int edge_slot(const Job& J, int id) {
  const int r = rank_of(J.emask, J.eprefix, id);
  return r < J.cap_edges ? r : J.cap_edges - 1;
}
__device__ __forceinline__ int cell_slot(const Job& J, int id) {
  const int r = rank_of(J.cmask, J.cprefix, id);
  return r < J.cap_cells ? r : J.cap_cells - 1;
}
// first pair of face `f`
__device__ __forceinline__ int pair_slot(const Job& J, int f) {
  const int w = f >> 5;
  const uint32_t below = (1u << (f & 31)) - 1u;
  const int r = (int)J.pprefix[w] + __popc(J.fact[w] & below) + __popc(J.famb[w] & below);
  return r < J.cap_pairs - 1 ? r : J.cap_pairs - 2;
}

// Job-major distribution: calls body(J, u) for the units of every job that
// belong to `worker` out of W workers; nunits(J) gives a job's unit count
// (0 to skip the job).  Wave-uniform when worker and the counts are.
template <class NFn, class Body>
__device__ __forceinline__ void for_units(const Job* __restrict__ jobs, int njobs, int worker,
                                          int W, const NFn& nunits, const Body& body) {
  // The job records never change during a launch: reading them through the
  // constant address space lets the compiler keep their fields in scalar
  // registers across the global stores of the body.
  const __attribute__((address_space(4))) Job* cj =
      (const __attribute__((address_space(4))) Job*)jobs;
  long long rot = 0;
  for (int k = 0; k < njobs; ++k) {
    const Job& J = *(const Job*)&cj[k];
    const int n = nunits(J);
    if (n <= 0) continue;
    int u0 = (int)(((long long)worker - rot) % W);
    if (u0 < 0) u0 += W;
    for (int u = u0; u < n; u += W) body(J, u);
    rot += n;
  }
}

// Job-major distribution of whole unit streams: body(J, u0, W, count) gets
// the units u0, u0 + W, ... (count of them) of every job that belong to
// `worker`, the same units for_units would give it.
template <class NFn, class Body>
__device__ __forceinline__ void for_unit_streams(const Job* __restrict__ jobs, int njobs,
                                                 int worker, int W, const NFn& nunits,
                                                 const Body& body) {
  const __attribute__((address_space(4))) Job* cj =
      (const __attribute__((address_space(4))) Job*)jobs;
  long long rot = 0;
  for (int k = 0; k < njobs; ++k) {
    const Job& J = *(const Job*)&cj[k];
    const int n = nunits(J);
    if (n <= 0) continue;
    int u0 = (int)(((long long)worker - rot) % W);
    if (u0 < 0) u0 += W;
    if (u0 < n) body(J, u0, (n - u0 + W - 1) / W);
    rot += n;
  }
}

// A unit index drawn by the wavefront from a counter in device memory
// (wave-uniform; every lane must call it).
__device__ __forceinline__ int take_unit(unsigned long long* ctr) {
  int v = 0;
  if (lane_id() == 0) v = (int)atomicAdd(ctr, 1ull);
  return __builtin_amdgcn_readfirstlane(v);
}

// Job-major distribution by drawing: every wavefront takes part in every
// job and draws its units from the job's counter ctr(J) (cleared before the
// launch) until they run out, so wavefronts whose units run short take more
// of them and all end together.  body(J, u) runs wave-uniformly.
template <class NFn, class CFn, class Body>
__device__ __forceinline__ void for_units_drawn(const Job* __restrict__ jobs, int njobs,
                                                const NFn& nunits, const CFn& ctr,
                                                const Body& body) {
  const __attribute__((address_space(4))) Job* cj =
      (const __attribute__((address_space(4))) Job*)jobs;
  for (int k = 0; k < njobs; ++k) {
    const Job& J = *(const Job*)&cj[k];
    const int n = nunits(J);
    if (n <= 0) continue;
    for (int u = take_unit(ctr(J)); u < n; u = take_unit(ctr(J))) body(J, u);
  }
}

// Job-major distribution in contiguous chunks: body(J, u0, u1) gets units
// [u0, u1) of every job, the worker's share of ceil(n / W) consecutive units
// (for passes that walk their units in order, see BlockWalk).
template <class NFn, class Body>
__device__ __forceinline__ void for_unit_chunks(const Job* __restrict__ jobs, int njobs,
                                                int worker, int W, const NFn& nunits,
                                                const Body& body) {
  const __attribute__((address_space(4))) Job* cj =
      (const __attribute__((address_space(4))) Job*)jobs;
  long long rot = 0;
  for (int k = 0; k < njobs; ++k) {
    const Job& J = *(const Job*)&cj[k];
    const int n = nunits(J);
    if (n <= 0) continue;
    const int chunk = (n + W - 1) / W;
    const int used = (n + chunk - 1) / chunk;
    int w = (int)(((long long)worker - rot) % W);
    if (w < 0) w += W;
    if (w < used) {
      const int u0 = w * chunk;
      body(J, u0, n - u0 < chunk ? n : u0 + chunk);
    }
    rot += used;
  }
}

// Grid position of element e of the edges (one block per axis: N along the
// axis, N + 1 across it), the faces (N + 1 along the axis, N across) or the
// cells (one N^3 block), x fastest: set once with divisions, then moved 64
// elements at a time with carries.
struct BlockWalk {
  int N, kind;  // 0 edges, 1 faces, 2 cells
  int a, p[3], n[3];
  __device__ __forceinline__ void dims() {
#pragma unroll
    for (int d = 0; d < 3; ++d) n[d] = kind == 2 ? N : (((d == a) == (kind == 0)) ? N : N + 1);
  }
  __device__ __forceinline__ void init(const Grid& g, int k, int e) {
    N = g.N;
    kind = k;
    if (k == 0) {
      edge_pos(g, e, a, p);
    } else if (k == 1) {
      face_pos(g, e, a, p);
    } else {
      a = 0;
      p[0] = e % N;
      p[1] = (e / N) % N;
      p[2] = e / (N * N);
    }
    dims();
  }
  // the element 64 further on (past the last block the position is unused)
  __device__ __forceinline__ void advance64() {
    p[0] += 64;
    while (p[0] >= n[0]) {
      p[0] -= n[0];
      if (++p[1] >= n[1]) {
        p[1] = 0;
        if (++p[2] >= n[2]) {
          p[2] = 0;
          ++a;
          dims();
        }
      }
    }
  }
};

}  // namespace odc
