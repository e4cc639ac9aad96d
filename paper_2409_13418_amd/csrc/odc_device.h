// Device-side building blocks of the ODC path: grid indexing, binary32
// occupancy of CSG fields, face pairing and cube partitions.
//
// Conventions follow include/odc.h.  Everything that decides an occupancy
// label is written as explicit binary32 operations; the library is compiled
// with -ffp-contract=off so none of them fuse.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace odc {

constexpr int kPrimFloats = 20;
constexpr int kMaxRes = 512;

struct Grid {
  int N;          // cells per axis
  float lo[3];    // (float)lo
  float h;        // (float)(size / N)
  int nc;         // corners (N+1)^3
  int ea;         // edges per axis N(N+1)^2
  int fa;         // faces per axis (N+1)N^2
  int ncell;      // N^3
};

// ---------------------------------------------------------------- indexing
// Element i of a 3-vector, and updates of it, written as selects: a small
// array indexed at run time would otherwise be placed in scratch or LDS.
template <class T>
__device__ __forceinline__ T at3(const T v[3], int i) {
  return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]);
}
template <class T>
__device__ __forceinline__ void add_at3(T v[3], int i, T x) {
  v[0] = i == 0 ? v[0] + x : v[0];
  v[1] = i == 1 ? v[1] + x : v[1];
  v[2] = i == 2 ? v[2] + x : v[2];
}
template <class T>
__device__ __forceinline__ void set_at3(T v[3], int i, T x) {
  v[0] = i == 0 ? x : v[0];
  v[1] = i == 1 ? x : v[1];
  v[2] = i == 2 ? x : v[2];
}

__device__ __forceinline__ void other_axes(int a, int& b1, int& b2) {
  b1 = (a == 0) ? 1 : 0;
  b2 = (a == 2) ? 1 : 2;
}

__device__ __forceinline__ int corner_index(const Grid& g, int i, int j, int k) {
  return i + (g.N + 1) * (j + (g.N + 1) * k);
}

__device__ __forceinline__ int edge_index(const Grid& g, int a, int i, int j, int k) {
  const int N = g.N;
  if (a == 0) return i + N * (j + (N + 1) * k);
  if (a == 1) return g.ea + i + (N + 1) * (j + N * k);
  return 2 * g.ea + i + (N + 1) * (j + (N + 1) * k);
}

__device__ __forceinline__ void edge_pos(const Grid& g, int id, int& a, int p[3]) {
  a = id / g.ea;
  int r = id - a * g.ea;
  const int nx = (a == 0) ? g.N : g.N + 1;
  const int ny = (a == 1) ? g.N : g.N + 1;
  p[0] = r % nx;
  r /= nx;
  p[1] = r % ny;
  p[2] = r / ny;
}

__device__ __forceinline__ int face_index(const Grid& g, int a, int i, int j, int k) {
  const int N = g.N;
  if (a == 0) return i + (N + 1) * (j + N * k);
  if (a == 1) return g.fa + i + N * (j + (N + 1) * k);
  return 2 * g.fa + i + N * (j + N * k);
}

__device__ __forceinline__ void face_pos(const Grid& g, int id, int& a, int p[3]) {
  a = id / g.fa;
  int r = id - a * g.fa;
  const int nx = (a == 0) ? g.N + 1 : g.N;
  const int ny = (a == 1) ? g.N + 1 : g.N;
  p[0] = r % nx;
  r /= nx;
  p[1] = r % ny;
  p[2] = r / ny;
}

__device__ __forceinline__ int bit_of(const uint32_t* __restrict__ words, int i) {
  return (words[i >> 5] >> (i & 31)) & 1;
}

// rank of element i among the set bits of `mask`, given exclusive word prefixes
__device__ __forceinline__ int rank_of(const uint32_t* __restrict__ mask,
                                       const uint32_t* __restrict__ prefix, int i) {
  const uint32_t below = mask[i >> 5] & ((1u << (i & 31)) - 1u);
  return (int)prefix[i >> 5] + __popc(below);
}

// world position of a grid-unit point: x = lo + g*h, two binary32 ops per axis
__device__ __forceinline__ void grid_world(const Grid& g, const float gp[3], float x[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float gh = gp[a] * g.h;
    x[a] = g.lo[a] + gh;
  }
}

// ------------------------------------------------------------- CSG labels
// Primitive records stay unchanged for a whole launch.  Read through the
// constant address space, their (wave-uniform) fields come in through
// scalar loads, also in kernels that store to global memory while they
// evaluate the field.
typedef const __attribute__((address_space(4))) float PrimF;

__device__ __forceinline__ int prim_inside(const PrimF* __restrict__ p, const float x[3]) {
  const int type = (int)p[1];
  const float dx = x[0] - p[2];
  const float dy = x[1] - p[3];
  const float dz = x[2] - p[4];
  if (type == 0) {
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float d2 = (xx + yy) + zz;
    const float r2 = p[5] * p[5];
    return d2 < r2;
  }
  if (type == 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float t0 = p[8 + 3 * a] * dx, t1 = p[9 + 3 * a] * dy, t2 = p[10 + 3 * a] * dz;
      const float l = (t0 + t1) + t2;
      if (!(fabsf(l) < p[5 + a])) return 0;
    }
    return 1;
  }
  const float t0 = p[5] * dx, t1 = p[6] * dy, t2 = p[7] * dz;
  const float v = (t0 + t1) + t2;
  return v < 0.0f;
}

// Left fold over the primitives; a primitive whose operation cannot change
// the running result is skipped (booleans, so the result is unchanged).
__device__ __forceinline__ int csg_inside(const float* __restrict__ prims_, int n,
                                          const float x[3]) {
  const PrimF* prims = (const PrimF*)prims_;
  int acc = prim_inside(prims, x);
  for (int i = 1; i < n; ++i) {
    const PrimF* p = prims + kPrimFloats * i;
    const int op = (int)p[0];
    if ((op == 0) == (acc != 0)) continue;  // union of true / subtract or intersect of false
    const int b = prim_inside(p, x);
    acc = (op == 0) ? b : ((op == 1) ? !b : b);
  }
  return acc;
}

// A signed-distance bound of the CSG solid (negative inside): exact distances
// of the primitives (rotation rows orthonormal; a half-space's normal
// normalised), folded with min (union), max(a, -b) (subtract) and max
// (intersect).  The fold is 1-Lipschitz and its sign is the solid's label
// away from rounding, so where the labels of two points differ, each lies
// within their distance of a zero of it: |d| at a point bounds how close a
// label change can be.  Used only to mark coarse cells (adaptive corner
// evaluation); labels always come from csg_inside.
__device__ __forceinline__ float prim_distance(const PrimF* __restrict__ p, const float x[3]) {
  const int type = (int)p[1];
  const float dx = x[0] - p[2], dy = x[1] - p[3], dz = x[2] - p[4];
  if (type == 0) return sqrtf(dx * dx + dy * dy + dz * dz) - p[5];
  if (type == 1) {
    float out2 = 0.0f, inmax = -INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float l = p[8 + 3 * a] * dx + p[9 + 3 * a] * dy + p[10 + 3 * a] * dz;
      const float e = fabsf(l) - p[5 + a];
      out2 += e > 0.0f ? e * e : 0.0f;
      inmax = fmaxf(inmax, e);
    }
    return sqrtf(out2) + fminf(inmax, 0.0f);
  }
  const float nn = sqrtf(p[5] * p[5] + p[6] * p[6] + p[7] * p[7]);
  return (p[5] * dx + p[6] * dy + p[7] * dz) / nn;
}

__device__ __forceinline__ float csg_distance(const float* __restrict__ prims_, int n,
                                              const float x[3]) {
  const PrimF* prims = (const PrimF*)prims_;
  float acc = prim_distance(prims, x);
  for (int i = 1; i < n; ++i) {
    const PrimF* p = prims + kPrimFloats * i;
    const int op = (int)p[0];
    const float b = prim_distance(p, x);
    acc = op == 0 ? fminf(acc, b) : (op == 1 ? fmaxf(acc, -b) : fmaxf(acc, b));
  }
  return acc;
}

// --------------------------------------------------------- faces / cubes
// face-local corner lc = bu + 2 bv; face-local edges
// 0: lc0-lc1 (v=0), 1: lc2-lc3 (v=1), 2: lc0-lc2 (u=0), 3: lc1-lc3 (u=1)
__device__ __forceinline__ int face_crossing_mask(const int L[4]) {
  return (L[0] != L[1]) | ((L[2] != L[3]) << 1) | ((L[0] != L[2]) << 2) | ((L[1] != L[3]) << 3);
}

// Pairs of crossing face-local edges (App. A.1.1): two crossings make one
// pair; a checkerboard face pairs around its inside corners, or around its
// outside corners when flipped.  Returns the pair count, pairs sorted by
// first edge.
__device__ __forceinline__ int face_pairs(const int L[4], int flipped, int pa[2], int pb[2]) {
  const int m = face_crossing_mask(L);
  const int n = __popc(m);
  if (n == 0) return 0;
  if (n == 2) {
    const int e0 = __ffs(m) - 1;
    const int e1 = __ffs(m & ~(1 << e0)) - 1;
    pa[0] = e0;
    pb[0] = e1;
    return 1;
  }
  const int around03 = (L[0] == 1) != (flipped != 0);
  pa[0] = 0;
  pa[1] = 1;
  pb[0] = around03 ? 2 : 3;
  pb[1] = around03 ? 3 : 2;
  return 2;
}

// cell-local edge of axis `axis` with corner offsets off[]
__device__ __forceinline__ int cell_edge(int axis, const int off[3]) {
  int b1, b2;
  other_axes(axis, b1, b2);
  return 4 * axis + off[b1] + 2 * off[b2];
}

// cell-local edge of face-local edge fe on local face (normal a, side s)
__device__ __forceinline__ int face_to_cell_edge(int a, int s, int fe) {
  int u, v;
  other_axes(a, u, v);
  int off[3] = {0, 0, 0};
  off[a] = s;
  int axis;
  if (fe < 2) {
    axis = u;
    off[v] = fe;
  } else {
    axis = v;
    off[u] = fe - 2;
  }
  return cell_edge(axis, off);
}

__device__ __forceinline__ void cube_face_labels(int cfg, int a, int s, int L[4]) {
  int u, v;
  other_axes(a, u, v);
#pragma unroll
  for (int lc = 0; lc < 4; ++lc) {
    int off[3] = {0, 0, 0};
    off[a] = s;
    off[u] = lc & 1;
    off[v] = lc >> 1;
    L[lc] = (cfg >> (off[0] + 2 * off[1] + 4 * off[2])) & 1;
  }
}

__device__ __forceinline__ int cube_edge_crosses(int cfg, int le) {
  const int axis = le >> 2;
  int b1, b2;
  other_axes(axis, b1, b2);
  int off[3] = {0, 0, 0};
  off[b1] = le & 1;
  off[b2] = (le >> 1) & 1;
  const int c0 = off[0] + 2 * off[1] + 4 * off[2];
  off[axis] = 1;
  const int c1 = off[0] + 2 * off[1] + 4 * off[2];
  return ((cfg >> c0) & 1) != ((cfg >> c1) & 1);
}

// Cycles of the face-pair graph of one cube (App. A.1.1): partition index of
// each crossing edge, 2 bits per cell-local edge; returns the count.
__device__ inline int cube_partitions(int cfg, int flipmask, int& partmap) {
  int nb0[12], nb1[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) nb0[e] = nb1[e] = -1;
  for (int lf = 0; lf < 6; ++lf) {
    const int a = lf >> 1, s = lf & 1;
    int L[4], pa[2], pb[2];
    cube_face_labels(cfg, a, s, L);
    const int np = face_pairs(L, (flipmask >> lf) & 1, pa, pb);
    for (int q = 0; q < np; ++q) {
      const int e0 = face_to_cell_edge(a, s, pa[q]);
      const int e1 = face_to_cell_edge(a, s, pb[q]);
      if (nb0[e0] < 0) nb0[e0] = e1; else nb1[e0] = e1;
      if (nb0[e1] < 0) nb0[e1] = e0; else nb1[e1] = e0;
    }
  }
  int part[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) part[e] = -1;
  int np = 0;
  for (int e = 0; e < 12; ++e) {
    if (!cube_edge_crosses(cfg, e) || part[e] >= 0) continue;
    int cur = e;
    while (cur >= 0 && part[cur] < 0) {
      part[cur] = np;
      const int a = nb0[cur], b = nb1[cur];
      cur = (a >= 0 && part[a] < 0) ? a : ((b >= 0 && part[b] < 0) ? b : -1);
    }
    ++np;
  }
  int pm = 0;
  for (int e = 0; e < 12; ++e)
    if (part[e] >= 0) pm |= (part[e] & 3) << (2 * e);
  partmap = pm;
  return np;
}

}  // namespace odc
