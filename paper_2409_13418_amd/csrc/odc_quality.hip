// Self-intersections of a triangle mesh (a quality metric of Sec. 6 and of
// Table 3): the pairs of triangles that share no vertex and whose closed
// triangles intersect.
//
// Candidate pairs come from a uniform grid of cubes of side `cell`: every
// triangle is entered in each cube its bounding box overlaps, the entries are
// sorted by cube, and each pair of entries of one cube is tested there only
// if that cube holds the lowest corner of the two boxes' overlap, so every
// pair is tested once.  The test takes orientation determinants in binary64
// on binary32 inputs: the coordinate differences are exact (for coordinates
// of like magnitude) and only the products round, so rounding can decide a
// sign only for a nearly degenerate, touching configuration (a determinant
// within ~2^-50 of its terms).  A non-coplanar pair intersects iff an edge
// of one meets the other closed triangle; a coplanar pair, iff an edge pair
// crosses or a corner of one lies in the other, in the plane's projection.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "odc_context.h"

namespace odc {
namespace {

constexpr int kMaxCubesPerTriangle = 4096;
constexpr int kCubeBias = 1 << 20;  // cube coordinates within +-2^20 pack into 21 bits

__device__ __forceinline__ void tri_box(const float* v, const int* t, long long i, float lo[3],
                                        float hi[3]) {
  const int a = t[3 * i], b = t[3 * i + 1], c = t[3 * i + 2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float x = v[3 * (long long)a + k], y = v[3 * (long long)b + k], z = v[3 * (long long)c + k];
    lo[k] = fminf(x, fminf(y, z));
    hi[k] = fmaxf(x, fmaxf(y, z));
  }
}

__device__ __forceinline__ int cube_of(float x, float inv) { return (int)floorf(x * inv); }

__device__ __forceinline__ unsigned long long cube_key(int i, int j, int k) {
  return (unsigned long long)(i + kCubeBias) | ((unsigned long long)(j + kCubeBias) << 21) |
         ((unsigned long long)(k + kCubeBias) << 42);
}

// Cubes overlapped by triangle i (0 for an invalid or oversized triangle,
// which sets the matching bit of *flags).
__global__ void k_cube_count(const float* v, long long nv, const int* t, long long nt, float inv,
                             int* cnt, int* flags) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nt;
       i += (long long)gridDim.x * blockDim.x) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) ok = ok && t[3 * i + k] >= 0 && t[3 * i + k] < nv;
    if (!ok) {
      cnt[i] = 0;
      atomicOr(flags, 1);
      continue;
    }
    float lo[3], hi[3];
    tri_box(v, t, i, lo, hi);
    long long n = 1;
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      fin = fin && isfinite(lo[k]) && isfinite(hi[k]) && fabsf(lo[k] * inv) < kCubeBias &&
            fabsf(hi[k] * inv) < kCubeBias;
      n *= (long long)(cube_of(hi[k], inv) - cube_of(lo[k], inv) + 1);
    }
    if (!fin || n > kMaxCubesPerTriangle) {
      cnt[i] = 0;
      atomicOr(flags, 2);
      continue;
    }
    cnt[i] = (int)n;
  }
}

__global__ void k_cube_fill(const float* v, const int* t, long long nt, float inv, const int* cnt,
                            const long long* off, unsigned long long* keys, int* vals) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nt;
       i += (long long)gridDim.x * blockDim.x) {
    if (cnt[i] == 0) continue;
    float lo[3], hi[3];
    tri_box(v, t, i, lo, hi);
    int c0[3], c1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      c0[k] = cube_of(lo[k], inv);
      c1[k] = cube_of(hi[k], inv);
    }
    long long o = off[i];
    for (int z = c0[2]; z <= c1[2]; ++z)
      for (int y = c0[1]; y <= c1[1]; ++y)
        for (int x = c0[0]; x <= c1[0]; ++x) {
          keys[o] = cube_key(x, y, z);
          vals[o] = (int)i;
          ++o;
        }
  }
}

__device__ __forceinline__ double orient(const double a[3], const double b[3], const double c[3],
                                         const double d[3]) {
  const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  const double p[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  const double q[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
  return u[0] * (p[1] * q[2] - p[2] * q[1]) + u[1] * (p[2] * q[0] - p[0] * q[2]) +
         u[2] * (p[0] * q[1] - p[1] * q[0]);
}

// segment pq against closed triangle ABC when pq does not lie in its plane
__device__ bool segment_meets(const double p[3], const double q[3], const double A[3],
                              const double B[3], const double C[3]) {
  const double s1 = orient(A, B, C, p), s2 = orient(A, B, C, q);
  if ((s1 > 0.0 && s2 > 0.0) || (s1 < 0.0 && s2 < 0.0) || (s1 == 0.0 && s2 == 0.0)) return false;
  const double o1 = orient(p, q, A, B), o2 = orient(p, q, B, C), o3 = orient(p, q, C, A);
  return (o1 >= 0.0 && o2 >= 0.0 && o3 >= 0.0) || (o1 <= 0.0 && o2 <= 0.0 && o3 <= 0.0);
}

__device__ __forceinline__ double orient2(const double a[2], const double b[2], const double c[2]) {
  return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

__device__ bool in_triangle2(const double p[2], const double T[3][2]) {
  const double a = orient2(T[0], T[1], p), b = orient2(T[1], T[2], p), c = orient2(T[2], T[0], p);
  return (a >= 0.0 && b >= 0.0 && c >= 0.0) || (a <= 0.0 && b <= 0.0 && c <= 0.0);
}

__device__ bool segments_cross2(const double a[2], const double b[2], const double c[2],
                                const double d[2]) {
  const double o1 = orient2(a, b, c), o2 = orient2(a, b, d), o3 = orient2(c, d, a),
               o4 = orient2(c, d, b);
  if (((o1 > 0.0 && o2 < 0.0) || (o1 < 0.0 && o2 > 0.0)) &&
      ((o3 > 0.0 && o4 < 0.0) || (o3 < 0.0 && o4 > 0.0)))
    return true;
  // collinear touching: an endpoint on the other segment
  auto on = [](const double p[2], const double q[2], const double r[2], double o) {
    return o == 0.0 && fmin(p[0], q[0]) <= r[0] && r[0] <= fmax(p[0], q[0]) &&
           fmin(p[1], q[1]) <= r[1] && r[1] <= fmax(p[1], q[1]);
  };
  return on(a, b, c, o1) || on(a, b, d, o2) || on(c, d, a, o3) || on(c, d, b, o4);
}

__device__ bool triangles_meet(const double P[3][3], const double Q[3][3]) {
  const bool coplanar = orient(P[0], P[1], P[2], Q[0]) == 0.0 &&
                        orient(P[0], P[1], P[2], Q[1]) == 0.0 &&
                        orient(P[0], P[1], P[2], Q[2]) == 0.0;
  if (!coplanar) {
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      if (segment_meets(P[e], P[(e + 1) % 3], Q[0], Q[1], Q[2])) return true;
      if (segment_meets(Q[e], Q[(e + 1) % 3], P[0], P[1], P[2])) return true;
    }
    return false;
  }
  // project onto the coordinate plane most parallel to the triangles
  const double u[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
  const double w[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
  const double n[3] = {fabs(u[1] * w[2] - u[2] * w[1]), fabs(u[2] * w[0] - u[0] * w[2]),
                       fabs(u[0] * w[1] - u[1] * w[0])};
  const int drop = n[0] >= n[1] && n[0] >= n[2] ? 0 : (n[1] >= n[2] ? 1 : 2);
  // kept coordinates i0 < i1 (selects, not indexing: the arrays stay in
  // registers)
  double p2[3][2], q2[3][2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    p2[k][0] = drop == 0 ? P[k][1] : P[k][0];
    p2[k][1] = drop == 2 ? P[k][1] : P[k][2];
    q2[k][0] = drop == 0 ? Q[k][1] : Q[k][0];
    q2[k][1] = drop == 2 ? Q[k][1] : Q[k][2];
  }
#pragma unroll
  for (int e = 0; e < 3; ++e)
#pragma unroll
    for (int f = 0; f < 3; ++f)
      if (segments_cross2(p2[e], p2[(e + 1) % 3], q2[f], q2[(f + 1) % 3])) return true;
  return in_triangle2(p2[0], q2) || in_triangle2(q2[0], p2);
}

__global__ void __launch_bounds__(256) k_cube_pairs(const float* v, const int* t, float inv,
                             const unsigned long long* keys, const int* vals, long long ne,
                             unsigned long long* count) {
  unsigned long long mine = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < ne;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long key = keys[i];
    const int a = vals[i];
    float la[3], ha[3];
    tri_box(v, t, a, la, ha);
    for (long long j = i + 1; j < ne && keys[j] == key; ++j) {
      const int b = vals[j];
      bool shared = false;
#pragma unroll
      for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) shared = shared || t[3 * (long long)a + x] == t[3 * (long long)b + y];
      if (shared) continue;
      float lb[3], hb[3];
      tri_box(v, t, b, lb, hb);
      bool overlap = true;
      int cm[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float m = fmaxf(la[k], lb[k]);
        overlap = overlap && m <= fminf(ha[k], hb[k]);
        cm[k] = cube_of(m, inv);
      }
      if (!overlap || cube_key(cm[0], cm[1], cm[2]) != key) continue;
      double P[3][3], Q[3][3];
#pragma unroll
      for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          P[x][k] = (double)v[3 * (long long)t[3 * (long long)a + x] + k];
          Q[x][k] = (double)v[3 * (long long)t[3 * (long long)b + x] + k];
        }
      if (triangles_meet(P, Q)) ++mine;
    }
  }
  if (mine) atomicAdd(count, mine);
}

}  // namespace
}  // namespace odc

using namespace odc;

#define QTRY(expr)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      rc = ctx_fail(ctx, ODC_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));              \
      goto done;                                                                            \
    }                                                                                       \
  } while (0)

extern "C" int32_t odc_count_self_intersections(odc_context* ctx, const float* vertices,
                                                int64_t n_vertices, const int32_t* triangles,
                                                int64_t n_triangles, double cell,
                                                int64_t* count) {
  if (!ctx || !count) return ODC_ERR_INVALID_ARG;
  *count = 0;
  if (!(cell > 0.0) || n_vertices < 0 || n_triangles < 0 || n_triangles >= (1LL << 31) ||
      (n_triangles > 0 && (!vertices || !triangles)))
    return ctx_fail(ctx, ODC_ERR_INVALID_ARG,
                    "self-intersections need device vertices/triangles and cell > 0");
  if (n_triangles < 2) return ODC_OK;
  int32_t rc = ODC_OK;
  const hipStream_t s = ctx->stream;
  const float inv = (float)(1.0 / cell);
  const int blocks = 2048, threads = 256;
  int *cnt = nullptr, *flags = nullptr, *vals = nullptr, *vals2 = nullptr;
  long long* off = nullptr;
  unsigned long long *keys = nullptr, *keys2 = nullptr, *dcount = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  long long total = 0;
  int hflags = 0;
  unsigned long long hcount = 0;
  long long last_off = 0;
  int last_cnt = 0;
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx_fail(ctx, ODC_ERR_HIP, "hipSetDevice");
  QTRY(hipMalloc(&cnt, sizeof(int) * n_triangles));
  QTRY(hipMalloc(&off, sizeof(long long) * n_triangles));
  QTRY(hipMalloc(&flags, sizeof(int)));
  QTRY(hipMalloc(&dcount, sizeof(unsigned long long)));
  QTRY(hipMemsetAsync(flags, 0, sizeof(int), s));
  QTRY(hipMemsetAsync(dcount, 0, sizeof(unsigned long long), s));
  k_cube_count<<<blocks, threads, 0, s>>>(vertices, n_vertices, triangles, n_triangles, inv, cnt,
                                          flags);
  QTRY(hipGetLastError());
  QTRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt, off, (int)n_triangles, s));
  QTRY(hipMalloc(&tmp, tmp_bytes));
  QTRY(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, off, (int)n_triangles, s));
  QTRY(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s));
  QTRY(hipMemcpyAsync(&last_off, off + n_triangles - 1, sizeof(long long), hipMemcpyDeviceToHost, s));
  QTRY(hipMemcpyAsync(&last_cnt, cnt + n_triangles - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  QTRY(hipStreamSynchronize(s));
  if (hflags & 1) {
    rc = ctx_fail(ctx, ODC_ERR_INVALID_ARG, "a triangle references a vertex outside 0..%lld",
                  (long long)n_vertices - 1);
    goto done;
  }
  if (hflags & 2) {
    rc = ctx_fail(ctx, ODC_ERR_INVALID_ARG,
                  "a triangle is not finite or spans more than %d cubes of side %g",
                  kMaxCubesPerTriangle, cell);
    goto done;
  }
  total = last_off + last_cnt;
  if (total >= (1LL << 31)) {
    rc = ctx_fail(ctx, ODC_ERR_INVALID_ARG, "%lld grid entries: choose a larger cell", total);
    goto done;
  }
  if (total > 1) {
    QTRY(hipMalloc(&keys, sizeof(unsigned long long) * total));
    QTRY(hipMalloc(&keys2, sizeof(unsigned long long) * total));
    QTRY(hipMalloc(&vals, sizeof(int) * total));
    QTRY(hipMalloc(&vals2, sizeof(int) * total));
    k_cube_fill<<<blocks, threads, 0, s>>>(vertices, triangles, n_triangles, inv, cnt, off, keys,
                                           vals);
    QTRY(hipGetLastError());
    size_t sort_bytes = 0;
    QTRY(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, keys, keys2, vals, vals2,
                                            (int)total, 0, 63, s));
    if (sort_bytes > tmp_bytes) {
      QTRY(hipFree(tmp));
      tmp = nullptr;
      QTRY(hipMalloc(&tmp, sort_bytes));
      tmp_bytes = sort_bytes;
    }
    QTRY(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, keys2, vals, vals2, (int)total,
                                            0, 63, s));
    k_cube_pairs<<<blocks, threads, 0, s>>>(vertices, triangles, inv, keys2, vals2, total, dcount);
    QTRY(hipGetLastError());
  }
  QTRY(hipMemcpyAsync(&hcount, dcount, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  QTRY(hipStreamSynchronize(s));
  *count = (int64_t)hcount;
done:
  (void)hipStreamSynchronize(s);
  (void)hipFree(cnt);
  (void)hipFree(off);
  (void)hipFree(flags);
  (void)hipFree(dcount);
  (void)hipFree(tmp);
  (void)hipFree(keys);
  (void)hipFree(keys2);
  (void)hipFree(vals);
  (void)hipFree(vals2);
  return rc;
}
