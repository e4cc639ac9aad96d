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
//             row 2b+h.  Layer-1 block b is input pair b (below); hidden-layer
//             virtual K row (b = 16T + i, h) is physical neuron
//             32T + 8(i/4) + 4h + i%4.
//  bf16 path  v_mfma_f32_32x32x16_bf16: K block b (16 rows), lane half h
//             gives rows 16b + 8h + j, j < 8.  Layer-1 row (b, h, j) is member
//             h of input pair 8b + j; hidden-layer virtual row
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
// Layer-1 inputs gamma(x): (x, y, z), then per band j: sin(2^j pi x_a),
// a < 3, then cos(2^j pi x_a).  The matrix cores consume them in pairs, lane
// half h taking member h: pair 0 = (x, y), pair 1 = (z, none), pair
// 2 + 3j + a = (sin, cos)(2^j pi x_a).  The packed layer-1 weights follow
// this order (feature_of_pair), so both halves run the same instructions.
__host__ __device__ constexpr int feature_of_pair(int p, int h) {
  return p == 0 ? h : (p == 1 ? (h ? -1 : 2) : 3 + 6 * ((p - 2) / 3) + 3 * h + (p - 2) % 3);
}
__host__ __device__ constexpr int n_pairs(int in_dim) { return (in_dim + 1) / 2; }
// every input of gamma is a member of exactly one of the first n_pairs pairs
constexpr bool pairs_cover(int in_dim) {
  for (int k = 0; k < in_dim; ++k) {
    int n = 0;
    for (int p = 0; p < n_pairs(in_dim); ++p)
      for (int h = 0; h < 2; ++h) n += feature_of_pair(p, h) == k;
    if (n != 1) return false;
  }
  for (int p = 0; p < n_pairs(in_dim); ++p)
    for (int h = 0; h < 2; ++h)
      if (feature_of_pair(p, h) >= in_dim) return false;
  return true;
}
static_assert(pairs_cover(3) && pairs_cover(9) && pairs_cover(39) && pairs_cover(45),
              "input pairs must cover gamma exactly");

// Layer-1 K blocks, padded with zero weights to whole groups of 4 so that one
// register ring streams layer 1 and the hidden layers alike (they are
// contiguous in memory); at most 6 (fp32) and 1 (bf16) groups.
__host__ __device__ constexpr int kb1_fp32(int in_dim) { return (n_pairs(in_dim) + 3) / 4 * 4; }
__host__ __device__ constexpr int kb1_bf16(int in_dim) { return ((n_pairs(in_dim) + 7) / 8 + 3) / 4 * 4; }
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
  // the second and third bf16 terms of every weight (w = w0 + w1 + w2
  // exactly, w0 = the fragments above), laid out as w1b then whb: the
  // split-bf16 evaluation only (else NULL)
  const v8bf* wx1;
  const v8bf* wx2;
  const float* bias; // [depth][256]
  const float* wout; // [256]
  const float* spheres;
  const float* bout;  // the output bias, read in place from the caller's weights
  float sdf_gain, out_scale;
  int n_spheres, depth, in_dim, kb1f, kb1b;
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Sum of an int over the 64 lanes of the wavefront (every lane gets it).
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Entry of a per-neuron vector (bias, output weights) for accumulator
// register i of tile T in lane half h: neuron 32 T + 8 (i/4) + 4 h + i%4.
// Both candidates are wave-uniform (scalar loads); the lane half selects.
__device__ __forceinline__ float bias_of(const ODC_CONST float* v, int T, int i, int h) {
  const int n0 = 32 * T + 8 * (i >> 2) + (i & 3);
  const float lo = v[n0], hi = v[n0 + 4];
  return h ? hi : lo;
}

// The phase in revolutions, 2^(j-1) x_a (exact), reduced exactly to
// [-1/2, 1/2] by subtracting the nearest integer.
__device__ __forceinline__ float pair_phase(int p, const float x[3]) {
  const int q = p - 2, j = q / 3, a = q % 3;
  const float t = x[a] * (j == 0 ? 0.5f : (float)(1 << (j - 1)));
  return t - __builtin_rintf(t);
}

// binary32 member h of pair p: the hardware sine or cosine of the reduced
// phase (absolute error ~1.2e-7 against the correctly rounded value on this
// range: about two binary32 ulps of a value near 1).
__device__ __forceinline__ float pair_feature(int p, int h, const float x[3]) {
  if (p == 0) return h ? x[1] : x[0];
  if (p == 1) return h ? 0.0f : x[2];
  const float r = pair_phase(p, x);
  return h ? __builtin_amdgcn_cosf(r) : __builtin_amdgcn_sinf(r);
}

// The same for the bf16 path (inputs rounded to bf16, relative error 2^-9):
// cos(2 pi r) = sin(2 pi (r + 1/4)), one transcendental for either half;
// the added quarter rounds by at most 2^-25 revolutions.
__device__ __forceinline__ float pair_feature_fast(int p, float quarter_h, int h,
                                                   const float x[3]) {
  if (p == 0) return h ? x[1] : x[0];
  if (p == 1) return h ? 0.0f : x[2];
  return __builtin_amdgcn_sinf(pair_phase(p, x) + quarter_h);
}

// Forward-mode differentiation (the gradient-normal ablation): lane l's
// column l%32 is channel ch = l%4 of query (l%32)/4; channel 0 carries the
// value, channel 1 + d the derivative along x_d.  Member h of pair p in
// channel ch:
__device__ __forceinline__ float pair_tangent(int p, int h, int ch, const float x[3]) {
  const int d = ch - 1;
  if (p == 0) return ch == 0 ? (h ? x[1] : x[0]) : ((h ? d == 1 : d == 0) ? 1.0f : 0.0f);
  if (p == 1) return ch == 0 ? (h ? 0.0f : x[2]) : ((!h && d == 2) ? 1.0f : 0.0f);
  const int q = p - 2, j = q / 3, a = q % 3;
  const float r = pair_phase(p, x);
  const float sn = __builtin_amdgcn_sinf(r), cs = __builtin_amdgcn_cosf(r);
  // d/dx_a sin(pi 2^j x_a) = pi 2^j cos(pi 2^j x_a); the cosine's is -pi 2^j sin
  const float w = (float)(3.14159265358979323846 * (double)(1 << j));
  if (ch == 0) return h ? cs : sn;
  return d == a ? (h ? -w * sn : w * cs) : 0.0f;
}

// The value of lane 4k of this lane's quad (DPP quad permutation 0,0,0,0).
__device__ __forceinline__ float quad_lead(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x00, 0xF, 0xF, false));
}

// B operand of a hidden layer from a parked pre-activation a and its bias b:
// relu(a + b) for values; for derivative channels a where the value's
// pre-activation is positive (the ReLU's derivative, 0 at 0), else 0.
template <bool kTan>
__device__ __forceinline__ float relu_operand(float a, float b, int ch) {
  const float s = a + b;
  if constexpr (!kTan) {
    return fmaxf(s, 0.0f);
  } else {
    const float lead = quad_lead(s);
    return ch == 0 ? fmaxf(s, 0.0f) : (lead > 0.0f ? a : 0.0f);
  }
}

// |x - c| - r of one sphere (c, r): squared distance by fused multiply-adds,
// hardware square root (within 1 ulp).
__device__ __forceinline__ float sphere_term(float cx, float cy, float cz, float r,
                                             const float x[3]) {
  const float dx = x[0] - cx, dy = x[1] - cy, dz = x[2] - cz;
  const float q = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
  return __builtin_amdgcn_sqrtf(q) - r;
}

// z = out_scale * y - sdf_gain * sdf, from the two half-wave partial sums
template <bool kTan = false>
__device__ __forceinline__ float mlp_finish(const Mlp& M, float part, const float x[3]) {
  const float other = __shfl_xor(part, 32);
  const float y0 = (lane_id() < 32) ? (part + other) : (other + part);
  if constexpr (kTan) {
    // derivative channels: out_scale dy/dx_d - sdf_gain (x_d - c_d)/|x - c|
    // through the nearest sphere (the first in index order on a tie)
    const ODC_CONST float* sp = cmem(M.spheres);
    float sdf = INFINITY, near[3] = {0.0f, 0.0f, 0.0f}, dist = 1.0f;
    for (int s = 0; s < M.n_spheres; ++s) {
      const float dx = x[0] - sp[4 * s], dy = x[1] - sp[4 * s + 1], dz = x[2] - sp[4 * s + 2];
      const float r = __builtin_amdgcn_sqrtf(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
      const float dd = r - sp[4 * s + 3];
      if (dd < sdf) {
        sdf = dd;
        near[0] = dx;
        near[1] = dy;
        near[2] = dz;
        dist = r;
      }
    }
    const int ch = lane_id() & 3;
    if (ch == 0) return M.out_scale * (y0 + *cmem(M.bout)) - M.sdf_gain * sdf;
    const float nd = ch == 1 ? near[0] : (ch == 2 ? near[1] : near[2]);
    return M.out_scale * y0 - (dist > 0.0f ? M.sdf_gain * (nd / dist) : 0.0f);
  }
  const float y = y0 + *cmem(M.bout);
  // spheres four at a time (one 16-dword scalar load each, issued one group
  // ahead of its use), then the rest
  const ODC_CONST float* sp = cmem(M.spheres);
  const int n4 = M.n_spheres & ~3;
  float sdf = INFINITY;
  if (n4 > 0) {
    float c[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) c[j] = sp[j];
    for (int s = 0; s < n4; s += 4) {
      const int sn = s + 4 < n4 ? s + 4 : s;
      float nx[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) nx[j] = sp[4 * sn + j];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        sdf = fminf(sdf, sphere_term(c[4 * u], c[4 * u + 1], c[4 * u + 2], c[4 * u + 3], x));
#pragma unroll
      for (int j = 0; j < 16; ++j) c[j] = nx[j];
    }
  }
  for (int s = n4; s < M.n_spheres; ++s)
    sdf = fminf(sdf, sphere_term(sp[4 * s], sp[4 * s + 1], sp[4 * s + 2], sp[4 * s + 3], x));
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

// Output layer of either path from the last layer's pre-activations in the
// accumulators: y = sum_n wout[n] relu(pre_n + bias_n), lane half h taking
// neurons 8G + 4h + d in the order (G, d), then the sdf term.
//
// ob: lane l's share of the last layer's biases and the output weights
// (vectors l of each, loaded by the caller well ahead); they go through the
// wavefront's LDS region, free once the last layer's accumulators are
// final, so that the output layer waits on LDS and not on memory.
template <bool kTan = false>
__device__ __forceinline__ float mlp_output(const Mlp& M, const v16f (&acc)[8], int h,
                                            const v4f (&ob)[2], v4f* __restrict__ act4,
                                            const float x[3]) {
  const int ch = lane_id() & 3;
  act4[lane_id()] = ob[0];
  act4[64 + lane_id()] = ob[1];
  const v4f* Bl = act4 + h;
  const v4f* Wo = act4 + 64 + h;
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
        const float a = relu_operand<kTan>(acc[T][4 * g + d], bb[u][d], ch);
        part = __builtin_fmaf(wo[u][d], a, part);
      }
    }
  }
  return mlp_finish<kTan>(M, part, x);
}

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

//
// kTan: forward-mode differentiation instead (8 queries of 4 channels each,
// see pair_tangent); lane l returns channel l%4 of query (l%32)/4: the logit,
// then dz/dx, dz/dy, dz/dz.
template <bool kTan = false>
__device__ __forceinline__ float mlp_logit_fp32(const Mlp& M, const float x[3],
                                                float* __restrict__ act) {
  const int lane = lane_id();
  const int h = lane >> 5;
  const int ch = lane & 3;
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
  // vector base + c of the stream, base a multiple of 4 and c a constant:
  // c mod 4 KB goes into the load's immediate offset, so the four vectors of
  // two K blocks share one scalar offset (one scalar add per two blocks)
  auto S = [&](int base, int c) -> v4f {
    return ring_load(ws, voff + (c & 3) * 1024, (base + (c & ~3)) * 1024);
  };
  // bias of layer l, group G, this lane half: vector (l * 64 + 2G + h)
  const ODC_GLOBAL v4f* Bv = (const ODC_GLOBAL v4f*)gmem(M.bias) + h + zero;
  v4f* act4 = reinterpret_cast<v4f*>(act);
  // layer 1's bias, group 0, fetched ahead of the ring so that waiting for
  // it at the first hidden layer does not drain the ring
  v4f bq[2];
  bq[0] = Bv[0];
  v4f wr[kPrefetchF32][2];
#pragma unroll
  for (int d = 0; d < kPrefetchF32; ++d)
#pragma unroll
    for (int q = 0; q < 2; ++q) wr[d][q] = S(0, 2 * d + q);
  const v16f zacc = {};
  v16f acc[8];
  // layer 1: B operand = Fourier features computed in registers; the first
  // block starts the accumulators from zero (every layer has one)
  // Each block's B operand is formed while the previous block's matrix
  // instructions run (no VALU-to-MFMA dependency at the block boundary).
  const int ng = M.kb1f / kPrefetchF32;
  auto feature = [&](int p) { return kTan ? pair_tangent(p, h, ch, x) : pair_feature(p, h, x); };
  float bv = feature(0);
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
        bv = feature(b + 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 2; ++q) wr[d][q] = S(2 * kPrefetchF32, 2 * b + q);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // the output layer's biases and weights (this lane's vectors), loaded
  // when the last layer starts
  v4f ob[2] = {};
  const ODC_GLOBAL v4f* Ob = (const ODC_GLOBAL v4f*)gmem(M.bias) + (size_t)(M.depth - 1) * 64 + zero;
  const ODC_GLOBAL v4f* Ow = (const ODC_GLOBAL v4f*)gmem(M.wout) + zero;
  if (M.depth == 1) {
    ob[0] = Ob[lane];
    ob[1] = Ow[lane];
  }
  for (int l = 1; l < M.depth; ++l) {
    if (l == M.depth - 1) {
      ob[0] = Ob[lane];
      ob[1] = Ow[lane];
    }
    // park the pre-activations of layer l
#pragma unroll
    for (int T = 0; T < 8; ++T)
#pragma unroll
      for (int g = 0; g < 4; ++g)
        act4[(4 * T + g) * 64 + lane] =
            (v4f){acc[T][4 * g], acc[T][4 * g + 1], acc[T][4 * g + 2], acc[T][4 * g + 3]};
    // block b of this layer is block kb1f + (l-1)*128 + b of the stream
    // (kb1f is a multiple of 4, so wn is one of 8)
    const int wn = (M.kb1f + (l - 1) * kHiddenBlocksF32 + kPrefetchF32) * 2;
    const ODC_GLOBAL v4f* Bn = Bv + (size_t)(l - 1) * 64;
    v4f an = act4[lane];
    bv = relu_operand<kTan>(an[0], bq[0][0], ch);
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
        bv = d < 3 ? relu_operand<kTan>(a[d + 1], bq[G & 1][d + 1], ch)
                   : relu_operand<kTan>(an[0], bq[(G + 1) & 1][0], ch);
        // refill the slot just consumed (same registers: no copies); the
        // first block's refill also fetches the next group's bias (after the
        // last group: group 0 of the next layer, or of the output layer)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 2; ++q) wr[d][q] = S(wn, 2 * b + q);
        if (d == 0) bq[(G + 1) & 1] = G + 1 < kGroupsF32 ? Bn[2 * (G + 1)] : Bn[64];
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  return mlp_output<kTan>(M, acc, h, ob, act4, x);
}

// bf16 evaluation (corner pass): a K block b of a hidden layer takes, in
// lane half h, neurons 16b + 4h + (0..3) and 16b + 8 + 4h + (0..3); its B
// operand is bf16(relu(pre + bias)) (bf16_operand).
// Ring depth of the bf16 weight stream (K blocks of 16 rows; 32 registers
// per block), as in the fp32 path.
constexpr int kPrefetchBF16 = 4;

// ReLU of two packed bf16 values: a bf16 is below zero exactly when its bits
// read as a negative 16-bit integer, so a packed signed max against 0 maps
// negatives (and -0) to +0 and keeps the rest.  Rounding to bf16 is
// monotonic and keeps 0, so this equals rounding relu(v).
__device__ __forceinline__ v8bf relu_bf16(v8bf v) {
  typedef short v8s __attribute__((ext_vector_type(8)));
  const v8s z = {};
  return __builtin_bit_cast(v8bf, __builtin_elementwise_max(__builtin_bit_cast(v8s, v), z));
}

// Two floats to a packed bf16 pair in one instruction (round to nearest even).
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  typedef float v2f __attribute__((ext_vector_type(2)));
  typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f){a, b}, v2bf));
}

__device__ __forceinline__ v8bf bf16_operand(v4f a0, v4f a1, v4f t0, v4f t1) {
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  const v4f s0 = a0 + t0, s1 = a1 + t1;
  const v4u p = {pack_bf16(s0[0], s0[1]), pack_bf16(s0[2], s0[3]), pack_bf16(s1[0], s1[1]),
                 pack_bf16(s1[2], s1[3])};
  return relu_bf16(__builtin_bit_cast(v8bf, p));
}

// LDS wait and workgroup barrier: this wavefront's LDS operations are
// complete, and the other wavefronts' are once it returns.
__device__ __forceinline__ void lds_block_sync() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// ---------------------------------------------------------- bf16 ping-pong
// The bf16 evaluation of 128 queries by the four wavefronts of a 256-thread
// workgroup, split by output tiles (wavefront w computes tiles 2w and 2w + 1,
// neurons 64w..64w + 63, of every layer, streaming only those tiles' weight
// fragments: two 16-byte loads per lane per K block), with the queries in two
// groups of 64: group g = sets 2g and 2g + 1 (set s = the 32 queries of
// wavefront s).  The groups take turns on the matrix cores.  While group 0
// runs layer k, the wavefront converts group 1's layer k - 1 accumulators
// into group 1's layer-k operands, bf16(relu(pre + bias)), and while group
// 1 runs layer k it converts group 0's layer-k accumulators.  Each phase's
// conversions thus run in the shadow of the other group's matrix
// instructions instead of between layers.  A barrier separates the phases
// (2 per layer): a group's LDS operands are rewritten only after every
// wavefront has read them.
//
// The weight fragments stream through a ring of kPPRing K blocks in
// registers, each slot reloaded with the block kPPRing ahead as soon as its
// matrix instructions are issued; the ring runs on into the next phase and,
// after the last, into the next call's layer 1, so a call starts with its
// weights loaded.  Biases and output weights are staged in LDS
// (stage_bias_wout), so the matrix loop issues no vector memory load but the
// weight refills.  At most 128 accumulator and 128 other registers per lane
// let two workgroups share a compute unit: one's matrix instructions run
// while the other converts, waits at a barrier or computes the output.
//
// The output layer sums, per wavefront, its 64 neurons for each set (group
// 0's in the shadow of group 1's last layer); the four partial sums then add
// in wavefront order, y = ((y_0 + y_1) + y_2) + y_3, followed by the output
// bias, out_scale and the sdf term as in mlp_finish.
//
// All four wavefronts of the workgroup must call it together, for the same
// field (2 depth + 2 barriers per call); `lds` is the workgroup's
// kPPLdsBytes with the field staged at kPPBiasOff, `wave` the wavefront's
// index in the workgroup.
constexpr int kPPOpBytes = 2 * kHiddenBlocksBF16 * 64 * 16;  // one group's operands: 32 KB
constexpr int kPPPartOff = 2 * kPPOpBytes;                   // [set][wave][32] floats
constexpr int kPPBiasOff = kPPPartOff + 4 * 4 * 32 * 4;      // depth x 256 biases, then w_out
constexpr int kPPLdsBytes = kPPBiasOff + (kMaxDepth + 1) * kWidth * 4;
constexpr int kB1 = kMaxGroups1BF16 * kPrefetchBF16;  // layer-1 K blocks
static_assert(kb1_bf16(3) == kB1 && kb1_bf16(kMaxInDim) == kB1, "one layer-1 block count");

// Copies the field's biases (depth x 256) and output weights (256) to dst
// (LDS); all 256 threads call it, then a barrier before they are read.
__device__ __forceinline__ void stage_bias_wout(const Mlp& M, char* dst_bytes) {
  v4f* dst = reinterpret_cast<v4f*>(dst_bytes);
  const ODC_GLOBAL v4f* Bsrc = (const ODC_GLOBAL v4f*)gmem(M.bias);
  const ODC_GLOBAL v4f* Wsrc = (const ODC_GLOBAL v4f*)gmem(M.wout);
  const int nb = M.depth * 64;
  for (int i = (int)threadIdx.x; i < nb + 64; i += 256) dst[i] = i < nb ? Bsrc[i] : Wsrc[i - nb];
}

// The weight stream of the ping-pong evaluation: tile 2 wave + j of stream
// block b (layer 1's kB1 blocks, then each hidden layer's NB; blocks past the
// end read as zero).
struct PPStream {
  __amdgpu_buffer_rsrc_t ws;
  int voff, wave;
  __device__ __forceinline__ PPStream(const Mlp& M, int wave_) : wave(wave_) {
    ws = weight_stream(M.w1b, ((size_t)kB1 + (size_t)(M.depth - 1) * kHiddenBlocksBF16 +
                               kPrefetchBF16) * 8192);
    voff = lane_id() * 16;
  }
  __device__ __forceinline__ v8bf operator()(int b, int j) const {
    return __builtin_bit_cast(
        v8bf, __builtin_amdgcn_raw_buffer_load_b128(ws, voff, (b * 8 + 2 * wave + j) * 1024, 0));
  }
};
constexpr int kPPRing = 4;  // weight ring slots (K blocks)

// Loads the ring for a call's first phase: layer 1's blocks.
__device__ __forceinline__ void pp_prime(const PPStream& S, v8bf (&W)[kPPRing][2]) {
#pragma unroll
  for (int b = 0; b < kPPRing; ++b)
#pragma unroll
    for (int j = 0; j < 2; ++j) W[b][j] = S(b, j);
}

// W: the weight ring, loaded by pp_prime before the first call for a field;
// each call leaves it loaded for the next.
__device__ __forceinline__ float mlp_logit_bf16_pp(const Mlp& M, const float x[3],
                                                   char* __restrict__ lds, int wave,
                                                   const PPStream& S, v8bf (&W)[kPPRing][2]) {
  const int lane = lane_id();
  const int h = lane >> 5;
  constexpr int NB = kHiddenBlocksBF16;
  static_assert(kB1 == kPPRing, "layer 1 fills the ring exactly");
  // operand vector of set s (0, 1) of group g, K block b
  auto op = [&](int g, int s, int b) -> v8bf* {
    return reinterpret_cast<v8bf*>(lds + g * kPPOpBytes) + (s * NB + b) * 64 + lane;
  };
  float* const part = reinterpret_cast<float*>(lds + kPPPartOff);
  const v4f* const bias4 = reinterpret_cast<const v4f*>(lds + kPPBiasOff) + h;
  // layer-1 operands of this wavefront's queries (set = wave)
  {
    const float quarter_h = h ? 0.25f : 0.0f;
#pragma unroll
    for (int b = 0; b < kB1; ++b) {
      typedef uint32_t v4u __attribute__((ext_vector_type(4)));
      v4u p;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        p[j] = pack_bf16(pair_feature_fast(8 * b + 2 * j, quarter_h, h, x),
                         pair_feature_fast(8 * b + 2 * j + 1, quarter_h, h, x));
      *op(wave >> 1, wave & 1, b) = __builtin_bit_cast(v8bf, p);
    }
  }
  lds_block_sync();
  const v16f zacc = {};
  v16f acc[4][2];  // [set][tile]
  float ps[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  // Side work k (0..7) done in the shadow of the other group's phase: operand
  // vector k of group g for the next layer (side 1, layer bias lb), or a
  // slice of group g's output sums (side 2).  Its two bias (or bias and
  // output weight) vectors are read from LDS before the block's matrix
  // instructions and used after them.
  struct SideIn {
    v4f t0, t1;
  };
  auto side_load = [&](auto side_c, int k, int lb) __attribute__((always_inline)) -> SideIn {
    constexpr int side = decltype(side_c)::value;
    SideIn r{};
    if constexpr (side == 1) {
      const int j = (k >> 1) & 1, beta = k & 1;
      const int b = 2 * (2 * wave + j) + beta;
      const v4f* Bl = bias4 + lb * 64;
      r.t0 = Bl[4 * b];
      r.t1 = Bl[4 * b + 2];
    } else if constexpr (side == 2) {
      const int G = 4 * (2 * wave + (k >> 2)) + (k & 3);
      r.t0 = bias4[(M.depth - 1) * 64 + 2 * G];
      r.t1 = bias4[M.depth * 64 + 2 * G];
    }
    return r;
  };
  auto side_run = [&](auto side_c, auto g_c, int k, const SideIn& in)
      __attribute__((always_inline)) {
    constexpr int side = decltype(side_c)::value;
    constexpr int g = decltype(g_c)::value;
    if constexpr (side == 1) {
      const int s = k >> 2, j = (k >> 1) & 1, beta = k & 1;
      const int b = 2 * (2 * wave + j) + beta;
      const v16f& a = acc[2 * g + s][j];
      const v4f a0 = {a[8 * beta], a[8 * beta + 1], a[8 * beta + 2], a[8 * beta + 3]};
      const v4f a1 = {a[8 * beta + 4], a[8 * beta + 5], a[8 * beta + 6], a[8 * beta + 7]};
      *op(g, s, b) = bf16_operand(a0, a1, in.t0, in.t1);
    } else if constexpr (side == 2) {
      const int j = k >> 2, gq = k & 3;
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int d = 0; d < 4; ++d)
          ps[2 * g + s] = __builtin_fmaf(
              in.t1[d], fmaxf(acc[2 * g + s][j][4 * gq + d] + in.t0[d], 0.0f), ps[2 * g + s]);
    }
  };
  using G0 = std::integral_constant<int, 0>;
  using G1 = std::integral_constant<int, 1>;
  using Side0 = std::integral_constant<int, 0>;
  using Side1 = std::integral_constant<int, 1>;
  using Side2 = std::integral_constant<int, 2>;
  // one phase: group g's matrix work over the nblk blocks of stream blocks
  // rb.., each block's operands read one block ahead, and side work for the
  // other group.  After block b's matrix instructions its slot is reloaded
  // with the block kPPRing ahead: of this phase while there is one, then of
  // the next phase (stream blocks rn..).
  auto phase = [&](auto g_c, auto nblk_c, auto side_c, int rb, int rn, int lb)
      __attribute__((always_inline)) {
    constexpr int g = decltype(g_c)::value;
    constexpr int nblk = decltype(nblk_c)::value;
    constexpr int side = decltype(side_c)::value;
    constexpr int per = nblk >= 8 ? 1 : 8 / nblk;  // side slices per block (every other, if 1)
    using OG = std::integral_constant<int, 1 - g>;
    v8bf bo[2], bn[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) bo[s] = *op(g, s, 0);
#pragma unroll
    for (int b = 0; b < nblk; ++b) {
      const int nb = b + 1 < nblk ? b + 1 : b;
      const int d = b % kPPRing;
      constexpr int nsl = side == 0 ? 0 : per;
      const bool has = side != 0 && (nblk < 8 || (b & 1) == 0);
      SideIn in[per];
      if (has) {
#pragma unroll
        for (int i = 0; i < nsl; ++i) in[i] = side_load(side_c, nblk >= 8 ? b >> 1 : b * per + i, lb);
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) bn[s] = *op(g, s, nb);
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[2 * g + s][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              W[d][j], bo[s], b == 0 ? zacc : acc[2 * g + s][j], 0, 0, 0);
      if (has) {
#pragma unroll
        for (int i = 0; i < nsl; ++i)
          side_run(side_c, OG{}, nblk >= 8 ? b >> 1 : b * per + i, in[i]);
      }
      __builtin_amdgcn_sched_barrier(0);
      const int sb = b + kPPRing < nblk ? rb + b + kPPRing : rn + b + kPPRing - nblk;
#pragma unroll
      for (int j = 0; j < 2; ++j) W[d][j] = S(sb, j);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < 2; ++s) bo[s] = bn[s];
    }
  };
  using L1 = std::integral_constant<int, kB1>;
  using LH = std::integral_constant<int, NB>;
  const int D = M.depth;
  // stream block of hidden layer k's first block (k >= 1)
  auto hb = [&](int k) { return kB1 + (k - 1) * NB; };
  // layer 1 (k = 0); the last phase reloads the ring with layer 1 for the
  // next call
  phase(G0{}, L1{}, Side0{}, 0, 0, 0);
  lds_block_sync();
  if (D > 1) phase(G1{}, L1{}, Side1{}, 0, hb(1), 0);
  else phase(G1{}, L1{}, Side2{}, 0, 0, 0);
  lds_block_sync();
  for (int k = 1; k < D; ++k) {
    phase(G0{}, LH{}, Side1{}, hb(k), hb(k), k - 1);
    lds_block_sync();
    if (k + 1 < D) phase(G1{}, LH{}, Side1{}, hb(k), hb(k + 1), k);
    else phase(G1{}, LH{}, Side2{}, hb(k), 0, k);
    lds_block_sync();
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) side_run(Side2{}, G1{}, k, side_load(Side2{}, k, 0));
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float t = ps[s] + __shfl_xor(ps[s], 32);
    if (h == 0) part[(s * 4 + wave) * 32 + lane] = t;
  }
  lds_block_sync();
  const float* pp = part + wave * 4 * 32 + (lane & 31);
  const float y = ((pp[0] + pp[32]) + pp[64]) + pp[96];
  return mlp_finish(M, h ? 0.0f : y, x);
}

// ---------------------------------------------------------- split bf16
// Evaluation at binary32 accuracy on the bf16 matrix cores.  Every weight is
// split exactly into three bf16 terms, w = w0 + w1 + w2 (each the rounded
// remainder of the previous: 8 + 8 + 8 significant bits), and so is every
// activation, a = a0 + a1 + a2.  A layer accumulates in binary32 the six
// products w_i a_j with i + j <= 2, smallest first.  Each product of two
// bf16 numbers is exact in binary32, and the three terms left out are each
// below 2^-24 |w a|: the result carries the error of binary32 arithmetic,
// not bf16's.  Six bf16 matrix instructions cost about 0.4 of one fp32 one
// for the same K rows.
//
// The four wavefronts of a 256-thread workgroup evaluate 128 queries
// together (set s = the 32 queries of wavefront s), split by output tiles
// as in the bf16 corner pass: wavefront w computes tiles 2w, 2w + 1 of every
// layer for all four sets, streaming only those tiles' three weight terms.
// Layer inputs are exchanged through LDS as binary32 activations,
// relu(pre + bias), in the bf16 B-operand order: [set][K block][half][lane]
// vectors of four (128 KB); each wavefront splits them into three bf16
// operands as it reads them.  Biases and output weights are staged in LDS by the caller
// (x3_stage) before the first call for a field.  The output layer sums, per
// wavefront, its 64 neurons for the four sets; the four partial sums then
// add in wavefront order, y = ((y_0 + y_1) + y_2) + y_3, followed by the
// output bias, out_scale and the sdf term as in mlp_finish.
constexpr int kX3OpBytes = 4 * kHiddenBlocksBF16 * 64 * 32;    // 128 KB
constexpr int kX3PartOff = kX3OpBytes;                          // [set][wave][32] floats
constexpr int kX3BiasOff = kX3PartOff + 4 * 4 * 32 * 4;          // (depth + 1) x 256 floats
constexpr int kX3VoteOff = kX3BiasOff + (kMaxDepth + 1) * kWidth * 4;
constexpr int kX3LdsBytes = kX3VoteOff + 2 * 4 * 4;              // two vote slots of 4 ints
constexpr int kX3Ring = 2;  // weight ring depth in K blocks (each ~1500 matrix cycles)

// Stages the field's biases and output weights in the workgroup's LDS; all
// 256 threads call it, then a barrier, before x3 evaluations of the field.
__device__ __forceinline__ void x3_stage(const Mlp& M, char* lds) {
  stage_bias_wout(M, lds + kX3BiasOff);
}

// Eight binary32 values to the three bf16 terms of each (exact split).
__device__ __forceinline__ void split3(v4f lo, v4f hi, v8bf& a0, v8bf& a1, v8bf& a2) {
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  auto pk = [](v4f a, v4f b) -> v4u {
    return (v4u){pack_bf16(a[0], a[1]), pack_bf16(a[2], a[3]), pack_bf16(b[0], b[1]),
                 pack_bf16(b[2], b[3])};
  };
  // a packed pair back to binary32: the low half shifted up, the high half masked
  auto un = [](v4u p, v4f& a, v4f& b) {
    a = (v4f){__builtin_bit_cast(float, p[0] << 16), __builtin_bit_cast(float, p[0] & 0xffff0000u),
              __builtin_bit_cast(float, p[1] << 16), __builtin_bit_cast(float, p[1] & 0xffff0000u)};
    b = (v4f){__builtin_bit_cast(float, p[2] << 16), __builtin_bit_cast(float, p[2] & 0xffff0000u),
              __builtin_bit_cast(float, p[3] << 16), __builtin_bit_cast(float, p[3] & 0xffff0000u)};
  };
  const v4u p0 = pk(lo, hi);
  v4f f0, f1;
  un(p0, f0, f1);
  const v4f r0 = lo - f0, r1 = hi - f1;
  const v4u p1 = pk(r0, r1);
  v4f g0, g1;
  un(p1, g0, g1);
  const v4u p2 = pk(r0 - g0, r1 - g1);
  a0 = __builtin_bit_cast(v8bf, p0);
  a1 = __builtin_bit_cast(v8bf, p1);
  a2 = __builtin_bit_cast(v8bf, p2);
}

// The logit of this lane's query (lanes l and l + 32 hold query l % 32);
// all four wavefronts call together.  2 depth + 1 barriers.
__device__ __forceinline__ float mlp_logit_x3(const Mlp& M, const float x[3], char* __restrict__ lds,
                                              int wave) {
  const int lane = lane_id();
  const int h = lane >> 5;
  int zero = 0;  // keeps the stream prologue here (see mlp_logit_fp32)
  asm volatile("" : "+v"(zero));
  v4f* const opnd = reinterpret_cast<v4f*>(lds);  // [set][block][half][lane]
  float* const part = reinterpret_cast<float*>(lds + kX3PartOff);
  const v4f* const bias4 = reinterpret_cast<const v4f*>(lds + kX3BiasOff);
  // half k (rows 4k..4k+3 of the lane's eight) of set `set`, K block b
  auto op = [&](int set, int b, int k) -> v4f* {
    return opnd + ((set * kHiddenBlocksBF16 + b) * 2 + k) * 64 + lane;
  };
  const size_t stream = ((size_t)kPrefetchBF16 + (size_t)(M.depth - 1) * kHiddenBlocksBF16 +
                         kPrefetchBF16) * 8192;
  const __amdgpu_buffer_rsrc_t w0s = weight_stream(M.w1b, stream);
  const __amdgpu_buffer_rsrc_t w1s = weight_stream(M.wx1, stream);
  const __amdgpu_buffer_rsrc_t w2s = weight_stream(M.wx2, stream);
  const int voff = (lane + zero) * 16;
  auto S = [&](__amdgpu_buffer_rsrc_t r, int b, int j) -> v8bf {
    return __builtin_bit_cast(
        v8bf, __builtin_amdgcn_raw_buffer_load_b128(r, voff, (b * 8 + 2 * wave + j) * 1024, 0));
  };
  // ring of kX3Ring K blocks: [slot][tile j][term]
  v8bf wr[kX3Ring][2][3];
  auto refill = [&](int d, int b) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      wr[d][j][0] = S(w0s, b, j);
      wr[d][j][1] = S(w1s, b, j);
      wr[d][j][2] = S(w2s, b, j);
    }
  };
#pragma unroll
  for (int d = 0; d < kX3Ring; ++d) refill(d, d);
  // layer-1 inputs of this wavefront's queries: K block b, lane half h, row
  // j = member h of input pair 8b + j (binary32 features)
#pragma unroll
  for (int b = 0; b < kPrefetchBF16; ++b) {
    v4f f[2];
#pragma unroll
    for (int j = 0; j < 8; ++j) f[j >> 2][j & 3] = pair_feature(8 * b + j, h, x);
    *op(wave, b, 0) = f[0];
    *op(wave, b, 1) = f[1];
  }
  lds_block_sync();
  const v16f zacc = {};
  v16f acc[4][2];
  // one layer: stream blocks base..base+nblk-1 (the ring continues into the
  // next layer's first blocks; the streams carry padding after the last)
  auto layer = [&](int base, auto nblk_c) {
    constexpr int nblk = decltype(nblk_c)::value;
#pragma unroll
    for (int i = 0; i < nblk; ++i) {
      const int d = i % kX3Ring;
#pragma unroll
      for (int set = 0; set < 4; ++set) {
        v8bf a0, a1, a2;
        split3(*op(set, i, 0), *op(set, i, 1), a0, a1, a2);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          v16f c = i == 0 ? zacc : acc[set][j];
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wr[d][j][2], a0, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wr[d][j][1], a1, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wr[d][j][0], a2, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wr[d][j][1], a0, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wr[d][j][0], a1, c, 0, 0, 0);
          acc[set][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wr[d][j][0], a0, c, 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      refill(d, base + i + kX3Ring);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  using L1 = std::integral_constant<int, kPrefetchBF16>;
  using LH = std::integral_constant<int, kHiddenBlocksBF16>;
  layer(0, L1{});
  const v4f* Bg = bias4 + h;
  for (int l = 1; l < M.depth; ++l) {
    lds_block_sync();  // every wavefront's reads of this layer's inputs are done
    // this wavefront's share of layer l's inputs: operand block b = 2 T + beta
    const v4f* Bl = Bg + (size_t)(l - 1) * 64;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int beta = 0; beta < 2; ++beta) {
        const int b = 2 * (2 * wave + j) + beta;
        const v4f t0 = Bl[4 * b], t1 = Bl[4 * b + 2];
#pragma unroll
        for (int set = 0; set < 4; ++set) {
          const v16f& a = acc[set][j];
          const v4f a0 = {a[8 * beta], a[8 * beta + 1], a[8 * beta + 2], a[8 * beta + 3]};
          const v4f a1 = {a[8 * beta + 4], a[8 * beta + 5], a[8 * beta + 6], a[8 * beta + 7]};
          const v4f s0 = a0 + t0, s1 = a1 + t1;
          *op(set, b, 0) =
              (v4f){fmaxf(s0[0], 0.0f), fmaxf(s0[1], 0.0f), fmaxf(s0[2], 0.0f), fmaxf(s0[3], 0.0f)};
          *op(set, b, 1) =
              (v4f){fmaxf(s1[0], 0.0f), fmaxf(s1[1], 0.0f), fmaxf(s1[2], 0.0f), fmaxf(s1[3], 0.0f)};
        }
      }
    lds_block_sync();  // layer l's inputs are complete
    layer(kPrefetchBF16 + (l - 1) * kHiddenBlocksBF16, LH{});
  }
  // output sums over this wavefront's 64 neurons (tile 2 wave + j, register
  // group G' = 4 h-interleaved neurons 32 T + 8 G' + 4 h + d), lane halves combined
  {
    const v4f* Bl = Bg + (size_t)(M.depth - 1) * 64;
    const v4f* Wo = bias4 + (size_t)M.depth * 64 + h;
    float ps[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int gq = 0; gq < 4; ++gq) {
        const int G = 4 * (2 * wave + j) + gq;
        const v4f bb = Bl[2 * G], wo = Wo[2 * G];
#pragma unroll
        for (int set = 0; set < 4; ++set)
#pragma unroll
          for (int d = 0; d < 4; ++d)
            ps[set] = __builtin_fmaf(wo[d], fmaxf(acc[set][j][4 * gq + d] + bb[d], 0.0f), ps[set]);
      }
#pragma unroll
    for (int set = 0; set < 4; ++set) {
      const float t = ps[set] + __shfl_xor(ps[set], 32);
      if (h == 0) part[(set * 4 + wave) * 32 + lane] = t;
    }
  }
  lds_block_sync();
  const float* pp = part + wave * 4 * 32 + (lane & 31);
  const float y = ((pp[0] + pp[32]) + pp[64]) + pp[96];
  return mlp_finish(M, h ? 0.0f : y, x);
}

// Workgroup-wide "may skip": 1 when every lane of the four wavefronts
// passes unneeded != 0.  Alternating vote slots (`parity`, flipped by the
// caller each vote) let a fast wavefront write the next vote while a slow
// one still reads this one; one barrier.
__device__ __forceinline__ int x3_vote_all(char* lds, int wave, int parity, int unneeded) {
  int* slot = reinterpret_cast<int*>(lds + kX3VoteOff) + 4 * parity;
  const int mine = __all(unneeded);
  if (lane_id() == 0) slot[wave] = mine;
  lds_block_sync();
  return slot[0] & slot[1] & slot[2] & slot[3];
}

}  // namespace odc
