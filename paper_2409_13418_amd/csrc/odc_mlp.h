// Occupancy of an MLP field evaluated by one wavefront for 32 query points at
// a time on the CDNA4 matrix cores.
//
// Layout.  Queries are the N (column) dimension of the MFMA tiles: lane l
// and lane l+32 hold query l%32.  A layer computes out^T = W in^T, so the
// weights are the A operand (streamed from memory in a pre-packed fragment
// order) and the activations are the B operand.  The accumulator of a 32x32
// tile holds, in lane l and register r, output row 8(r/4) + 4(l/32) + r%4 of
// column l%32; the next layer consumes exactly those registers as its B
// operand, which fixes a permutation of the K index that the packed weights
// absorb.  Activations therefore never leave registers.
//
//  fp32 path  v_mfma_f32_32x32x2_f32: K block b (2 rows), lane half h gives
//             row 2b+h.  Hidden-layer virtual K row (b = 16T + i, h) is
//             physical neuron 32T + 8(i/4) + 4h + i%4.
//  bf16 path  v_mfma_f32_32x32x16_bf16: K block b (16 rows), lane half h
//             gives rows 16b + 8h + j, j < 8.  Hidden-layer virtual row
//             (b = 2T + beta, h, j) is physical neuron 32T + 16 beta +
//             8(j/4) + 4h + j%4, taken from accumulator register 8 beta + j.
//
// Both paths end with the same binary32 output dot product (fixed order)
// and the same sdf term, so a query the bf16 path hands to the fp32 path
// gets bit-for-bit the fp32 path's logit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace odc {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kWidth = 256;
constexpr int kMaxDepth = 8;
constexpr int kMaxInDim = 45;
constexpr int kHiddenBlocksF32 = kWidth / 2;    // 128 K blocks of 2
constexpr int kHiddenBlocksBF16 = kWidth / 16;  // 16 K blocks of 16

struct Mlp {
  const float* w1f;  // [kb1f][8][64]            layer 1, fp32 fragments
  const float* whf;  // [depth-1][128][8][64]    hidden layers, fp32 fragments
  const v8bf* w1b;   // [kb1b][8][64]            layer 1, bf16 fragments
  const v8bf* whb;   // [depth-1][16][8][64]     hidden layers, bf16 fragments
  const float* bias; // [depth][256]
  const float* wout; // [256]
  const float* spheres;
  float bout;
  float sdf_gain, out_scale;
  int n_spheres, depth, in_dim, kb1f, kb1b;
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Feature k of gamma(x): (x, y, z), then per band j: sin(2^j pi x_a), a < 3,
// then cos(2^j pi x_a); 0 past in_dim.  The argument 2^j x is exact.
__device__ __forceinline__ float mlp_feature(int k, const float x[3], int in_dim) {
  if (k >= in_dim) return 0.0f;
  if (k < 3) return k == 0 ? x[0] : (k == 1 ? x[1] : x[2]);
  const int r = k - 3;
  const int band = r / 6;
  const int w = r - 6 * band;
  const int axis = w % 3;
  const float xa = axis == 0 ? x[0] : (axis == 1 ? x[1] : x[2]);
  const float arg = xa * (float)(1 << band);
  return w >= 3 ? cospif(arg) : sinpif(arg);
}

// z = out_scale * y - sdf_gain * sdf, from the two half-wave partial sums
__device__ __forceinline__ float mlp_finish(const Mlp& M, float part, const float x[3]) {
  const float other = __shfl_xor(part, 32);
  const float y0 = (lane_id() < 32) ? (part + other) : (other + part);
  const float y = y0 + M.bout;
  float sdf = INFINITY;
  for (int s = 0; s < M.n_spheres; ++s) {
    const float* sp = M.spheres + 4 * s;
    const float dx = x[0] - sp[0], dy = x[1] - sp[1], dz = x[2] - sp[2];
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float d = sqrtf((xx + yy) + zz) - sp[3];
    sdf = fminf(sdf, d);
  }
  const float mt = M.out_scale * y;
  const float st = M.sdf_gain * sdf;
  return mt - st;
}

// binary32 logit of this lane's query (all 64 lanes must be active).
// `act` is this wavefront's LDS region of kActWords floats: between layers
// each lane parks its 128 activations there ([K block][lane], conflict-free)
// and reads them back one K block at a time as B operands.  A lane only ever
// reads what it wrote itself, so no synchronisation is involved; the point
// is to free 128 registers per lane for the weight-fragment prefetch.
constexpr int kActWords = kHiddenBlocksF32 * 64;

__device__ __forceinline__ float mlp_logit_fp32(const Mlp& M, const float x[3],
                                                float* __restrict__ act) {
  const int lane = lane_id();
  const int h = lane >> 5;
  v16f acc[8];
#pragma unroll
  for (int R = 0; R < 8; ++R) acc[R] = (v16f){};
  for (int b = 0; b < M.kb1f; ++b) {
    const float bv = mlp_feature(2 * b + h, x, M.in_dim);
    const float* wp = M.w1f + (size_t)b * 8 * 64 + lane;
#pragma unroll
    for (int R = 0; R < 8; ++R)
      acc[R] = __builtin_amdgcn_mfma_f32_32x32x2f32(wp[R * 64], bv, acc[R], 0, 0, 0);
  }
  for (int l = 1; l < M.depth; ++l) {
    const float* bl = M.bias + (l - 1) * kWidth;
#pragma unroll
    for (int T = 0; T < 8; ++T)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int n = 32 * T + 8 * (i >> 2) + 4 * h + (i & 3);
        act[(16 * T + i) * 64 + lane] = fmaxf(acc[T][i] + bl[n], 0.0f);
      }
#pragma unroll
    for (int R = 0; R < 8; ++R) acc[R] = (v16f){};
    const float* W = M.whf + (size_t)(l - 1) * kHiddenBlocksF32 * 8 * 64 + lane;
#pragma unroll 8
    for (int b = 0; b < kHiddenBlocksF32; ++b) {
      const float* wp = W + (size_t)b * 8 * 64;
      const float bv = act[b * 64 + lane];
#pragma unroll
      for (int R = 0; R < 8; ++R)
        acc[R] = __builtin_amdgcn_mfma_f32_32x32x2f32(wp[R * 64], bv, acc[R], 0, 0, 0);
    }
  }
  const float* bl = M.bias + (M.depth - 1) * kWidth;
  float part = 0.0f;
#pragma unroll
  for (int T = 0; T < 8; ++T)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int n = 32 * T + 8 * (i >> 2) + 4 * h + (i & 3);
      const float a = fmaxf(acc[T][i] + bl[n], 0.0f);
      const float p = M.wout[n] * a;
      part = part + p;
    }
  return mlp_finish(M, part, x);
}

// bf16 operands, fp32 accumulation (all 64 lanes must be active).  `act`
// is this wavefront's LDS region of kActBlocksBF16 * 64 eight-element bf16
// vectors, used as in the fp32 path.
constexpr int kActVecsBF16 = kHiddenBlocksBF16 * 64;

__device__ __forceinline__ float mlp_logit_bf16(const Mlp& M, const float x[3],
                                                v8bf* __restrict__ act) {
  const int lane = lane_id();
  const int h = lane >> 5;
  v16f acc[8];
#pragma unroll
  for (int R = 0; R < 8; ++R) acc[R] = (v16f){};
  for (int b = 0; b < M.kb1b; ++b) {
    v8bf bv;
#pragma unroll
    for (int j = 0; j < 8; ++j) bv[j] = (__bf16)mlp_feature(16 * b + 8 * h + j, x, M.in_dim);
    const v8bf* wp = M.w1b + (size_t)b * 8 * 64 + lane;
#pragma unroll
    for (int R = 0; R < 8; ++R)
      acc[R] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wp[R * 64], bv, acc[R], 0, 0, 0);
  }
  for (int l = 1; l < M.depth; ++l) {
    const float* bl = M.bias + (l - 1) * kWidth;
#pragma unroll
    for (int T = 0; T < 8; ++T)
#pragma unroll
      for (int beta = 0; beta < 2; ++beta) {
        v8bf v;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int i = 8 * beta + j;
          const int n = 32 * T + 8 * (i >> 2) + 4 * h + (i & 3);
          v[j] = (__bf16)fmaxf(acc[T][i] + bl[n], 0.0f);
        }
        act[(2 * T + beta) * 64 + lane] = v;
      }
#pragma unroll
    for (int R = 0; R < 8; ++R) acc[R] = (v16f){};
    const v8bf* W = M.whb + (size_t)(l - 1) * kHiddenBlocksBF16 * 8 * 64 + lane;
#pragma unroll 4
    for (int b = 0; b < kHiddenBlocksBF16; ++b) {
      const v8bf* wp = W + (size_t)b * 8 * 64;
      const v8bf bv = act[b * 64 + lane];
#pragma unroll
      for (int R = 0; R < 8; ++R)
        acc[R] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wp[R * 64], bv, acc[R], 0, 0, 0);
    }
  }
  const float* bl = M.bias + (M.depth - 1) * kWidth;
  float part = 0.0f;
#pragma unroll
  for (int T = 0; T < 8; ++T)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int n = 32 * T + 8 * (i >> 2) + 4 * h + (i & 3);
      const float a = fmaxf(acc[T][i] + bl[n], 0.0f);
      const float p = M.wout[n] * a;
      part = part + p;
    }
  return mlp_finish(M, part, x);
}

}  // namespace odc
