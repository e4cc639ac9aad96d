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
// absorb.  Between layers the activations are parked in LDS (see
// mlp_logit_fp32), which frees registers for the weight prefetch.
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
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kWidth = 256;
constexpr int kMaxDepth = 8;
constexpr int kMaxInDim = 45;
constexpr int kHiddenBlocksF32 = kWidth / 2;    // 128 K blocks of 2
constexpr int kHiddenBlocksBF16 = kWidth / 16;  // 16 K blocks of 16
// Layer-1 K blocks, padded with zero weights to whole groups of 4 so that one
// register ring streams layer 1 and the hidden layers alike (they are
// contiguous in memory); at most 6 (fp32) and 1 (bf16) groups.
__host__ __device__ constexpr int kb1_fp32(int in_dim) { return ((in_dim + 1) / 2 + 3) / 4 * 4; }
__host__ __device__ constexpr int kb1_bf16(int in_dim) { return ((in_dim + 15) / 16 + 3) / 4 * 4; }
constexpr int kMaxGroups1F32 = kb1_fp32(45) / 4;
constexpr int kMaxGroups1BF16 = kb1_bf16(45) / 4;

// Pointers that are known to address device global memory.  The kernels
// read the job records from memory, so the pointers inside are generic; a
// load through a generic pointer is a flat load, which also counts against
// the LDS wait counter and stalls the LDS/matrix-core pipeline.  Weight
// reads therefore go through global-qualified copies.
#define ODC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const ODC_GLOBAL T* gmem(const T* p) {
  return (const ODC_GLOBAL T*)p;
}
// Read-only for the whole launch (biases, output weights, sdf spheres: the
// packing runs in an earlier kernel): wave-uniform reads through the
// constant address space become scalar loads.
#define ODC_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const ODC_CONST T* cmem(const T* p) {
  return (const ODC_CONST T*)p;
}

// A raw buffer resource over `bytes` bytes at p (gfx9 descriptor word 3).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t weight_stream(const void* p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ v4f ring_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

struct Mlp {
  const float* w1f;  // [kb1f][8][64]            layer 1, fp32 fragments
  const float* whf;  // [depth-1][128][8][64]    hidden layers, fp32 fragments
  const v8bf* w1b;   // [kb1b][8][64]            layer 1, bf16 fragments
  const v8bf* whb;   // [depth-1][16][8][64]     hidden layers, bf16 fragments
  const float* bias; // [depth][256]
  const float* wout; // [256]
  const float* spheres;
  const float* bout;  // the output bias, read in place from the caller's weights
  float sdf_gain, out_scale;
  int n_spheres, depth, in_dim, kb1f, kb1b;
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Entry of a per-neuron vector (bias, output weights) for accumulator
// register i of tile T in lane half h: neuron 32 T + 8 (i/4) + 4 h + i%4.
// Both candidates are wave-uniform (scalar loads); the lane half selects.
__device__ __forceinline__ float bias_of(const ODC_CONST float* v, int T, int i, int h) {
  const int n0 = 32 * T + 8 * (i >> 2) + (i & 3);
  const float lo = v[n0], hi = v[n0 + 4];
  return h ? hi : lo;
}

// Feature k of gamma(x): (x, y, z), then per band j: sin(2^j pi x_a), a < 3,
// then cos(2^j pi x_a); 0 past in_dim.  The argument is taken in
// revolutions, a = 2^(j-1) x_a (exact), reduced exactly to [-1/2, 1/2] by
// subtracting the nearest integer, and handed to the hardware sine and
// cosine (absolute error ~1.2e-7 against the correctly rounded sin(pi t)
// on this range: about two binary32 ulps of a value near 1).
__device__ __forceinline__ float mlp_feature(int k, const float x[3], int in_dim) {
  if (k >= in_dim) return 0.0f;
  if (k < 3) return k == 0 ? x[0] : (k == 1 ? x[1] : x[2]);
  const int r = k - 3;
  const int band = r / 6;
  const int w = r - 6 * band;
  const int axis = w % 3;
  const float xa = axis == 0 ? x[0] : (axis == 1 ? x[1] : x[2]);
  const float a = xa * (float)(1 << band) * 0.5f;  // sin(pi t) = sin(2 pi (t / 2))
  const float rev = a - __builtin_rintf(a);
  return w >= 3 ? __builtin_amdgcn_cosf(rev) : __builtin_amdgcn_sinf(rev);
}

// |x - c| - r of one sphere (c, r): squared distance by fused multiply-adds,
// hardware square root (within 1 ulp).
__device__ __forceinline__ float sphere_term(const ODC_CONST float* sp, const float x[3]) {
  const float dx = x[0] - sp[0], dy = x[1] - sp[1], dz = x[2] - sp[2];
  const float q = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
  return __builtin_amdgcn_sqrtf(q) - sp[3];
}

// z = out_scale * y - sdf_gain * sdf, from the two half-wave partial sums
__device__ __forceinline__ float mlp_finish(const Mlp& M, float part, const float x[3]) {
  const float other = __shfl_xor(part, 32);
  const float y0 = (lane_id() < 32) ? (part + other) : (other + part);
  const float y = y0 + *cmem(M.bout);
  // spheres four at a time (one 16-dword scalar load each), then the rest
  const ODC_CONST float* sp = cmem(M.spheres);
  float sdf = INFINITY;
  int s = 0;
  for (; s + 4 <= M.n_spheres; s += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) sdf = fminf(sdf, sphere_term(sp + 4 * (s + u), x));
  }
  for (; s < M.n_spheres; ++s) sdf = fminf(sdf, sphere_term(sp + 4 * s, x));
  const float mt = M.out_scale * y;
  const float st = M.sdf_gain * sdf;
  return mt - st;
}

// binary32 logit of this lane's query (all 64 lanes must be active).
//
// Between layers each lane parks its 128 pre-activations in `act` (this
// wavefront's LDS region of kActWords floats) as 32 four-element vectors,
// [group G = 4T + g][lane] holding accumulator registers 4g..4g+3 of tile T,
// and reads them back one group of four K blocks at a time.  Group G of a
// layer's input is, for lane half h, neurons 8G + 4h + d (d < 4) of the
// previous layer, so its bias (and, after the last layer, its output
// weights) is the four contiguous floats at 8G + 4h: one vector load per
// group, applied with the ReLU as the B operands are formed.  A lane only
// reads what it wrote itself, so no synchronisation is involved; parking
// frees 128 registers per lane for the weight prefetch.
constexpr int kActWords = kHiddenBlocksF32 * 64;
constexpr int kGroupsF32 = kHiddenBlocksF32 / 4;  // 32 groups of 4 K blocks

// Weight fragments stream through a ring of kPrefetchF32 K blocks held in
// registers: the load of block b + kPrefetchF32 is issued as block b is
// consumed, so each load has about kPrefetchF32 x 8 matrix-core
// instructions (~2000 cycles) to arrive.  A lane's eight fp32 fragments of a
// K block are packed as two 16-byte vectors: two load instructions per
// block.  Layer 1 (padded to whole groups of kPrefetchF32 blocks) and the
// hidden layers are contiguous in memory and the ring runs straight through
// them; the packed buffer carries kPrefetchF32 blocks of padding after the
// last layer for the overrun.  The bias vector of the next group rides with
// the refill of each group's first block.
constexpr int kPrefetchF32 = 4;
static_assert(kPrefetchF32 == 4, "one ring turn per group of four K blocks");

__device__ __forceinline__ float mlp_logit_fp32(const Mlp& M, const float x[3],
                                                float* __restrict__ act) {
  const int lane = lane_id();
  const int h = lane >> 5;
  // The offset is an opaque zero so that the ring's first loads stay here:
  // hoisted out of a caller's query loop they would pin 32 registers for its
  // whole length.
  int zero = 0;
  asm volatile("" : "+v"(zero));
  // layer 1, then the hidden layers: lane l's fragments of K block b are two
  // 16-byte vectors (tiles 0-3 and 4-7) at vector index (2b + q) * 64 + l
  // (buffer loads: the lane's byte offset stays in one register and the
  // block offset is scalar, so the stream costs no vector address arithmetic)
  const __amdgpu_buffer_rsrc_t ws = weight_stream(
      M.w1f, ((size_t)M.kb1f + (size_t)(M.depth - 1) * kHiddenBlocksF32 + kPrefetchF32) * 2048);
  const int voff = (lane + zero) * 16;
  auto S = [&](int vec) -> v4f { return ring_load(ws, voff, vec * 1024); };
  // bias of layer l, group G, this lane half: vector (l * 64 + 2G + h)
  const ODC_GLOBAL v4f* Bv = (const ODC_GLOBAL v4f*)gmem(M.bias) + h + zero;
  v4f* act4 = reinterpret_cast<v4f*>(act);
  v4f wr[kPrefetchF32][2];
#pragma unroll
  for (int d = 0; d < kPrefetchF32; ++d)
#pragma unroll
    for (int q = 0; q < 2; ++q) wr[d][q] = S(2 * d + q);
  const v16f zacc = {};
  v16f acc[8];
  // layer 1: B operand = Fourier features computed in registers; the first
  // block starts the accumulators from zero (every layer has one)
  // Each block's B operand is formed while the previous block's matrix
  // instructions run (no VALU-to-MFMA dependency at the block boundary).
  const int ng = M.kb1f / kPrefetchF32;
  float bv = mlp_feature(h, x, M.in_dim);
#pragma unroll
  for (int gi = 0; gi < kMaxGroups1F32; ++gi) {
    if (gi == 0 || gi < ng) {
#pragma unroll
      for (int d = 0; d < kPrefetchF32; ++d) {
        const int b = gi * kPrefetchF32 + d;
#pragma unroll
        for (int R = 0; R < 8; ++R)
          acc[R] = __builtin_amdgcn_mfma_f32_32x32x2f32(wr[d][R >> 2][R & 3], bv,
                                                        b == 0 ? zacc : acc[R], 0, 0, 0);
        bv = mlp_feature(2 * (b + 1) + h, x, M.in_dim);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 2; ++q) wr[d][q] = S((b + kPrefetchF32) * 2 + q);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  v4f bq[2];
  bq[0] = Bv[0];  // layer 1's bias, group 0
  for (int l = 1; l < M.depth; ++l) {
    // park the pre-activations of layer l
#pragma unroll
    for (int T = 0; T < 8; ++T)
#pragma unroll
      for (int g = 0; g < 4; ++g)
        act4[(4 * T + g) * 64 + lane] =
            (v4f){acc[T][4 * g], acc[T][4 * g + 1], acc[T][4 * g + 2], acc[T][4 * g + 3]};
    // block b of this layer is block kb1f + (l-1)*128 + b of the stream
    const int wn = (M.kb1f + (l - 1) * kHiddenBlocksF32 + kPrefetchF32) * 2;
    const ODC_GLOBAL v4f* Bn = Bv + (size_t)(l - 1) * 64;
    v4f an = act4[lane];
    bv = fmaxf(an[0] + bq[0][0], 0.0f);
    // fully unrolled: a loop back-edge here makes the wait-count insertion
    // drain every load in flight at the top of each trip
#pragma unroll
    for (int G = 0; G < kGroupsF32; ++G) {
      const v4f a = an;
      an = act4[((G + 1) & (kGroupsF32 - 1)) * 64 + lane];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int b = 4 * G + d;
#pragma unroll
        for (int R = 0; R < 8; ++R)
          acc[R] = __builtin_amdgcn_mfma_f32_32x32x2f32(wr[d][R >> 2][R & 3], bv,
                                                        b == 0 ? zacc : acc[R], 0, 0, 0);
        // the next block's operand (after the last group: unused)
        bv = d < 3 ? fmaxf(a[d + 1] + bq[G & 1][d + 1], 0.0f)
                   : fmaxf(an[0] + bq[(G + 1) & 1][0], 0.0f);
        // refill the slot just consumed (same registers: no copies); the
        // first block's refill also fetches the next group's bias (after the
        // last group: group 0 of the next layer, or of the output layer)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 2; ++q) wr[d][q] = S(wn + b * 2 + q);
        if (d == 0) bq[(G + 1) & 1] = G + 1 < kGroupsF32 ? Bn[2 * (G + 1)] : Bn[64];
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // output layer: y = sum_n wout[n] relu(pre_n + bias_n), lane half h taking
  // neurons 8G + 4h + d, in the order (G, d)
  const ODC_GLOBAL v4f* Bl = Bv + (size_t)(M.depth - 1) * 64;
  const ODC_GLOBAL v4f* Wo = (const ODC_GLOBAL v4f*)gmem(M.wout) + h + zero;
  float part = 0.0f;
#pragma unroll
  for (int G0 = 0; G0 < kGroupsF32; G0 += 8) {
    v4f bb[8], wo[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      bb[u] = Bl[2 * (G0 + u)];
      wo[u] = Wo[2 * (G0 + u)];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int G = G0 + u, T = G >> 2, g = G & 3;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const float a = fmaxf(acc[T][4 * g + d] + bb[u][d], 0.0f);
        part = __builtin_fmaf(wo[u][d], a, part);
      }
    }
  }
  return mlp_finish(M, part, x);
}

// bf16 operands, fp32 accumulation (all 64 lanes must be active).  `act`
// is this wavefront's LDS region of kActBlocksBF16 * 64 eight-element bf16
// vectors, used as in the fp32 path.
constexpr int kActVecsBF16 = kHiddenBlocksBF16 * 64;
// Ring depth of the bf16 hidden-layer weight stream (K blocks of 16 rows;
// 32 registers per block), as in the fp32 path.
constexpr int kPrefetchBF16 = 4;

__device__ __forceinline__ float mlp_logit_bf16(const Mlp& M, const float x[3],
                                                v8bf* __restrict__ act) {
  const int lane = lane_id();
  const int h = lane >> 5;
  int zero = 0;  // keeps the ring prologue here (see mlp_logit_fp32)
  asm volatile("" : "+v"(zero));
  // layer 1, then the hidden layers, through a buffer resource as in the
  // fp32 path: vector (8b + R) of the stream holds tile R of K block b
  const __amdgpu_buffer_rsrc_t ws = weight_stream(
      M.w1b, ((size_t)M.kb1b + (size_t)(M.depth - 1) * kHiddenBlocksBF16 + kPrefetchBF16) * 8192);
  const int voff = (lane + zero) * 16;
  auto S = [&](int vec) -> v8bf {
    return __builtin_bit_cast(v8bf, __builtin_amdgcn_raw_buffer_load_b128(ws, voff, vec * 1024, 0));
  };
  v8bf wr[kPrefetchBF16][8];
#pragma unroll
  for (int d = 0; d < kPrefetchBF16; ++d)
#pragma unroll
    for (int R = 0; R < 8; ++R) wr[d][R] = S(d * 8 + R);
  v16f acc[8];
#pragma unroll
  for (int R = 0; R < 8; ++R) acc[R] = (v16f){};
  const int ng = M.kb1b / kPrefetchBF16;
#pragma unroll
  for (int gi = 0; gi < kMaxGroups1BF16; ++gi) {
    if (gi < ng) {
#pragma unroll
      for (int d = 0; d < kPrefetchBF16; ++d) {
        const int b = gi * kPrefetchBF16 + d;
        v8bf bv;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          bv[j] = (__bf16)mlp_feature(16 * b + 8 * h + j, x, M.in_dim);
#pragma unroll
        for (int R = 0; R < 8; ++R)
          acc[R] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wr[d][R], bv, acc[R], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int R = 0; R < 8; ++R) wr[d][R] = S((b + kPrefetchBF16) * 8 + R);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  for (int l = 1; l < M.depth; ++l) {
    // scalar bias reads: vector loads here would queue behind the ring's
    // refills and wait for all of them
    const ODC_CONST float* bl = cmem(M.bias) + (l - 1) * kWidth;
#pragma unroll
    for (int T = 0; T < 8; ++T) {
#pragma unroll
      for (int beta = 0; beta < 2; ++beta) {
        v8bf v;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int i = 8 * beta + j;
          v[j] = (__bf16)fmaxf(acc[T][i] + bias_of(bl, T, i, h), 0.0f);
        }
        act[(2 * T + beta) * 64 + lane] = v;
      }
      acc[T] = (v16f){};
    }
    const int wn = (M.kb1b + (l - 1) * kHiddenBlocksBF16 + kPrefetchBF16) * 8;
    v8bf bvn = act[lane];
#pragma unroll
    for (int b0 = 0; b0 < kHiddenBlocksBF16; b0 += kPrefetchBF16) {
#pragma unroll
      for (int d = 0; d < kPrefetchBF16; ++d) {
        const int b = b0 + d;
        const v8bf bv = bvn;
        bvn = act[((b + 1) & (kHiddenBlocksBF16 - 1)) * 64 + lane];
#pragma unroll
        for (int R = 0; R < 8; ++R)
          acc[R] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wr[d][R], bv, acc[R], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int R = 0; R < 8; ++R) wr[d][R] = S(wn + b * 8 + R);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  const ODC_CONST float* bl = cmem(M.bias) + (M.depth - 1) * kWidth;
  const ODC_CONST float* wo = cmem(M.wout);
  float part = 0.0f;
#pragma unroll
  for (int T = 0; T < 8; ++T) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const float a = fmaxf(acc[T][i] + bias_of(bl, T, i, h), 0.0f);
      const float p = bias_of(wo, T, i, h) * a;
      part = part + p;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  return mlp_finish(M, part, x);
}

}  // namespace odc
