// HIP kernels of the ODC path for gfx950 and their launchers.
//
// Stage map (paper sections in brackets):
//   labels            (a) phi' at every corner, bit-packed          [Sec. 3]
//   classify/compact  crossing edges, face pairs, active cells      [Sec. 3, App. A.1.1]
//   bisect            (b) 1D points                                 [Sec. 5.1]
//   search2d          (c) 2D points                                 [Sec. 5.2, App. A.1.3-A.1.4]
//   cell_count/qef    (d) partitions, normals, QEF 3D points        [App. A.1.1, Sec. 5.3, Eq. 2]
//   emit              (e) quads, intersection-free split            [Sec. 4, App. A.1.5]
//
// Every kernel is persistent and job-major (odc_job.h): one launch per stage
// serves all jobs of a batch.  Grid-wide passes (labels of analytic fields,
// classification) give each wavefront 64 consecutive elements and pack the
// results with a ballot into two 32-bit words.  Passes over the compacted
// active sets run one thread per element for analytic fields; MLP fields run
// one wavefront per 32 elements so that each occupancy query of a search is a
// 32-column matrix-core batch (odc_mlp.h).
#include "odc_internal.h"

namespace odc {

constexpr int kBlock = 256;

__device__ __forceinline__ int gthread() { return blockIdx.x * kBlock + threadIdx.x; }
__device__ __forceinline__ int nthreads() { return gridDim.x * kBlock; }
__device__ __forceinline__ int gwave() { return (blockIdx.x * kBlock + threadIdx.x) >> 6; }
__device__ __forceinline__ int nwaves() { return gridDim.x * (kBlock / 64); }

__device__ __forceinline__ void store_ballot(uint64_t b, int first_elem_of_wave, int nwords,
                                             uint32_t* __restrict__ dst) {
  const int lane = lane_id();
  const int w0 = first_elem_of_wave >> 5;
  if (lane == 0 && w0 < nwords) dst[w0] = (uint32_t)b;
  if (lane == 32 && w0 + 1 < nwords) dst[w0 + 1] = (uint32_t)(b >> 32);
}

// ------------------------------------------------------------------ scans
// Exclusive scans of per-job uint32 arrays, out[n] = total.  Which array:
//   0 crossing-edge word counts, 1 pair word counts, 2 active-cell word counts,
//   3 partitions per active cell, 4 triangles per crossing edge,
//   5 case-3 vertices per crossing edge.
template <int S>
__device__ __forceinline__ void scan_arrays(const Job& J, const uint32_t*& in, uint32_t*& out,
                                            int& n) {
  if (S == 0) { in = J.ecount; out = J.eprefix; n = J.nw_e; }
  if (S == 1) { in = J.pcount; out = J.pprefix; n = J.nw_f; }
  if (S == 2) { in = J.ccount; out = J.cprefix; n = J.nw_cell; }
  if (S == 3) { in = J.npart; out = J.vbase; n = n_cells_of(J); }
  if (S == 4) { in = J.ntri; out = J.tprefix; n = n_edges_of(J); }
  if (S == 5) { in = J.n3; out = J.c3prefix; n = n_edges_of(J); }
}

template <int S>
__device__ __forceinline__ int scan_blocks_of(const Job& J) {
  const uint32_t* in;
  uint32_t* out;
  int n;
  scan_arrays<S>(J, in, out, n);
  return (n + 1023) >> 10;
}

template <int S>
__global__ __launch_bounds__(256) void k_scan_reduce(const Job* __restrict__ jobs, int njobs) {
  __shared__ uint32_t sh[256];
  for_units(jobs, njobs, blockIdx.x, gridDim.x,
            [](const Job& J) { return scan_blocks_of<S>(J); },
            [&](const Job& J, int blk) {
              const uint32_t* in;
              uint32_t* out;
              int n;
              scan_arrays<S>(J, in, out, n);
              const int base = blk * 1024;
              uint32_t s = 0;
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                const int i = base + threadIdx.x + k * 256;
                if (i < n) s += in[i];
              }
              sh[threadIdx.x] = s;
              __syncthreads();
              for (int off = 128; off > 0; off >>= 1) {
                if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
                __syncthreads();
              }
              if (threadIdx.x == 0) J.scan_tmp[blk] = sh[0];
              __syncthreads();
            });
}

template <int S>
__global__ __launch_bounds__(1024) void k_scan_blocks(const Job* __restrict__ jobs, int njobs) {
  __shared__ uint32_t sh[1024];
  for_units(jobs, njobs, blockIdx.x, gridDim.x, [](const Job&) { return 1; },
            [&](const Job& J, int) {
              const uint32_t* in;
              uint32_t* out;
              int n;
              scan_arrays<S>(J, in, out, n);
              const int nb = (n + 1023) >> 10;
              uint32_t carry = 0;
              const int t = threadIdx.x;
              for (int base = 0; base < nb; base += 1024) {
                const int i = base + t;
                const uint32_t v = i < nb ? J.scan_tmp[i] : 0u;
                sh[t] = v;
                __syncthreads();
                for (int off = 1; off < 1024; off <<= 1) {
                  const uint32_t x = t >= off ? sh[t - off] : 0u;
                  __syncthreads();
                  sh[t] += x;
                  __syncthreads();
                }
                if (i < nb) J.scan_tmp[i] = carry + sh[t] - v;
                carry += sh[1023];
                __syncthreads();
              }
              if (t == 0) out[n] = carry;
              __syncthreads();
            });
}

template <int S>
__global__ __launch_bounds__(256) void k_scan_apply(const Job* __restrict__ jobs, int njobs) {
  __shared__ uint32_t sh[256];
  for_units(jobs, njobs, blockIdx.x, gridDim.x,
            [](const Job& J) { return scan_blocks_of<S>(J); },
            [&](const Job& J, int blk) {
              const uint32_t* in;
              uint32_t* out;
              int n;
              scan_arrays<S>(J, in, out, n);
              const int t = threadIdx.x;
              const int base = blk * 1024 + 4 * t;
              uint32_t v[4], s = 0;
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                v[k] = (base + k < n) ? in[base + k] : 0u;
                s += v[k];
              }
              sh[t] = s;
              __syncthreads();
              for (int off = 1; off < 256; off <<= 1) {
                const uint32_t x = t >= off ? sh[t - off] : 0u;
                __syncthreads();
                sh[t] += x;
                __syncthreads();
              }
              uint32_t run = J.scan_tmp[blk] + sh[t] - s;
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                if (base + k < n) out[base + k] = run;
                run += v[k];
              }
              __syncthreads();
            });
}

template <int S>
static void scan(const Job* d, int njobs, const LaunchCfg& cfg, hipStream_t s) {
  k_scan_reduce<S><<<cfg.scan_blocks, 256, 0, s>>>(d, njobs);
  k_scan_blocks<S><<<njobs < 64 ? njobs : 64, 1024, 0, s>>>(d, njobs);
  k_scan_apply<S><<<cfg.scan_blocks, 256, 0, s>>>(d, njobs);
}

// ------------------------------------------------------------ MLP weights
// Packs the binary32 weights into the fragment orders of odc_mlp.h.
// Term t (0, 1, 2) of the exact three-term bf16 split of a binary32 weight:
// each term is the remainder of the previous ones rounded to bf16.
__device__ __forceinline__ __bf16 bf16_term(float w, int t) {
  const __bf16 w0 = (__bf16)w;
  if (t == 0) return w0;
  const float r = w - (float)w0;
  const __bf16 w1 = (__bf16)r;
  if (t == 1) return w1;
  return (__bf16)(r - (float)w1);
}

__device__ void pack_mlp(const float* __restrict__ w, int in_dim, int depth, long long id,
                         float* __restrict__ w1f, float* __restrict__ whf,
                         v8bf* __restrict__ w1b, v8bf* __restrict__ whb,
                         float* __restrict__ bias, float* __restrict__ wout,
                         v8bf* __restrict__ wx1, v8bf* __restrict__ wx2) {
  const int kb1f = kb1_fp32(in_dim), kb1b = kb1_bf16(in_dim);
  const size_t l1 = (size_t)kWidth * in_dim;
  const size_t hid = (size_t)kWidth * kWidth;
  const long long n_w1f = (long long)kb1f * 8 * 64;
  const long long n_whf = (long long)(depth - 1) * kHiddenBlocksF32 * 8 * 64;
  const long long n_w1b = (long long)kb1b * 8 * 64;
  const long long n_whb = (long long)(depth - 1) * kHiddenBlocksBF16 * 8 * 64;
  {
    long long r = id;
    // fp32 fragments: for K block b, lane l holds the values of tiles
    // R = 4q + c (c < 4) as one 16-byte vector at float offset
    // ((2b + q) * 64 + l) * 4 + c, so a lane loads its 8 tiles with 2 loads
    if (r < n_w1f) {
      const int c = r % 4, lane = (r / 4) % 64, q = (r / 256) % 2, b = (int)(r / 512);
      const int R = 4 * q + c;
      const int row = 32 * R + (lane & 31), k = feature_of_pair(b, lane >> 5);
      w1f[r] = k >= 0 && k < in_dim ? w[(size_t)row * in_dim + k] : 0.0f;
      return;
    }
    r -= n_w1f;
    if (r < n_whf) {
      const int c = r % 4, lane = (r / 4) % 64, q = (r / 256) % 2;
      const int R = 4 * q + c, b = (int)((r / 512) % kHiddenBlocksF32);
      const int l = (int)(r / (512LL * kHiddenBlocksF32));
      const int row = 32 * R + (lane & 31), h = lane >> 5;
      const int T = b >> 4, i = b & 15;
      const int n = 32 * T + 8 * (i >> 2) + 4 * h + (i & 3);
      const float* W = w + l1 + kWidth + (size_t)l * (hid + kWidth);
      whf[r] = W[(size_t)row * kWidth + n];
      return;
    }
    r -= n_whf;
    if (r < n_w1b) {
      const int lane = r % 64, R = (r / 64) % 8, b = (int)(r / 512);
      const int row = 32 * R + (lane & 31), h = lane >> 5;
      v8bf v;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = feature_of_pair(8 * b + j, h);
        v[j] = (__bf16)(k >= 0 && k < in_dim ? w[(size_t)row * in_dim + k] : 0.0f);
      }
      w1b[r] = v;
      return;
    }
    r -= n_w1b;
    if (r < n_whb) {
      const int lane = r % 64, R = (r / 64) % 8, b = (int)((r / 512) % kHiddenBlocksBF16);
      const int l = (int)(r / (512LL * kHiddenBlocksBF16));
      const int row = 32 * R + (lane & 31), h = lane >> 5;
      const int T = b >> 1, beta = b & 1;
      const float* W = w + l1 + kWidth + (size_t)l * (hid + kWidth);
      v8bf v;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int n = 32 * T + 16 * beta + 8 * (j >> 2) + 4 * h + (j & 3);
        v[j] = (__bf16)W[(size_t)row * kWidth + n];
      }
      whb[r] = v;
      return;
    }
    r -= n_whb;
    if (r < (long long)depth * kWidth) {
      const int l = (int)(r / kWidth), n = (int)(r % kWidth);
      const size_t off = (l == 0) ? l1 : l1 + kWidth + (size_t)(l - 1) * (hid + kWidth) + hid;
      bias[r] = w[off + n];
      return;
    }
    r -= (long long)depth * kWidth;
    if (r < kWidth) {
      wout[r] = w[l1 + kWidth + (size_t)(depth - 1) * (hid + kWidth) + r];
      return;
    }
    r -= kWidth;
    // the second and third bf16 terms, in the order of the bf16 fragments
    // (layer 1, then the hidden layers): term 1 + r / (n_w1b + n_whb)
    const long long nb = n_w1b + n_whb;
    if (r >= 2 * nb) return;
    const int t = 1 + (int)(r / nb);
    r %= nb;
    v8bf* dst = t == 1 ? wx1 : wx2;
    v8bf v;
    if (r < n_w1b) {
      const int lane = r % 64, R = (r / 64) % 8, b = (int)(r / 512);
      const int row = 32 * R + (lane & 31), h = lane >> 5;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = feature_of_pair(8 * b + j, h);
        v[j] = bf16_term(k >= 0 && k < in_dim ? w[(size_t)row * in_dim + k] : 0.0f, t);
      }
    } else {
      const long long q = r - n_w1b;
      const int lane = q % 64, R = (q / 64) % 8, b = (int)((q / 512) % kHiddenBlocksBF16);
      const int l = (int)(q / (512LL * kHiddenBlocksBF16));
      const int row = 32 * R + (lane & 31), h = lane >> 5;
      const int T = b >> 1, beta = b & 1;
      const float* W = w + l1 + kWidth + (size_t)l * (hid + kWidth);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int n = 32 * T + 16 * beta + 8 * (j >> 2) + 4 * h + (j & 3);
        v[j] = bf16_term(W[(size_t)row * kWidth + n], t);
      }
    }
    dst[r] = v;
  }
}


__device__ __forceinline__ long long pack_units(const Job& J) {
  if (J.kind != 1) return 0;
  const int d = J.mlp.depth;
  const long long nb = (long long)(J.mlp.kb1b + (d - 1) * kHiddenBlocksBF16) * 512;
  return (long long)(J.mlp.kb1f + (d - 1) * kHiddenBlocksF32) * 512 + nb +
         (long long)(d + 1) * kWidth + (J.mlp.wx1 ? 2 * nb : 0);
}

__global__ __launch_bounds__(256) void k_pack(const Job* __restrict__ jobs, int njobs,
                                              const float* const* __restrict__ weights) {
  for (int k = 0; k < njobs; ++k) {
    const Job& J = jobs[k];
    const long long n = pack_units(J);
    for (long long id = gthread(); id < n; id += nthreads())
      pack_mlp(weights[k], J.mlp.in_dim, J.mlp.depth, id, const_cast<float*>(J.mlp.w1f),
               const_cast<float*>(J.mlp.whf), const_cast<v8bf*>(J.mlp.w1b),
               const_cast<v8bf*>(J.mlp.whb), const_cast<float*>(J.mlp.bias),
               const_cast<float*>(J.mlp.wout), const_cast<v8bf*>(J.mlp.wx1),
               const_cast<v8bf*>(J.mlp.wx2));
  }
}

// ------------------------------------------------------------------ status
__global__ void k_clear_status(const Job* __restrict__ jobs, int njobs) {
  for (int k = gthread(); k < njobs; k += nthreads()) {
    jobs[k].status[0] = 0;
    jobs[k].status[1] = 0;
    jobs[k].status[2] = 0;
    jobs[k].status[3] = 0;
    jobs[k].status[4] = 0;
    jobs[k].status[5] = 0;
    jobs[k].status[6] = 0;
    jobs[k].status[7] = 0;
    jobs[k].status[8] = 0;
  }
}

// per job: raw totals and status for the host (kGatherWords x uint64)
__global__ void k_gather(const Job* __restrict__ jobs, int njobs,
                         unsigned long long* __restrict__ out) {
  for (int k = gthread(); k < njobs; k += nthreads()) {
    const Job& J = jobs[k];
    unsigned long long* o = out + kGatherWords * k;
    const int ne = n_edges_of(J), nc = n_cells_of(J);
    o[0] = J.eprefix[J.nw_e];
    o[1] = J.pprefix[J.nw_f];
    o[2] = J.cprefix[J.nw_cell];
    o[3] = J.vbase[nc];
    o[4] = J.tprefix[ne];
    o[5] = J.c3prefix[ne];
    o[6] = J.status[0];
    o[7] = J.status[1] | (J.status[2] << 32);
    o[8] = J.status[3];
    o[9] = J.status[4];
    o[10] = J.status[6];
  }
}

// ------------------------------------------- (a) adaptive corner evaluation
// With coarse_step S > 1 the field is first evaluated on the corners of the
// coarse grid (every S-th fine corner per axis), a coarse cell is marked when
// its corners' labels differ or one lies within the logit band, and the fine
// corner passes evaluate only corners of marked cells (whole units of 32 to
// 128 corners); every other corner takes its unmarked coarse cell's common
// label.

__device__ __forceinline__ int coarse_corners(const Job& J) {
  return (J.cn + 1) * (J.cn + 1) * (J.cn + 1);
}

// Binary32 labels of the coarse corners, 32 per wavefront, and whether each
// lies within the band: |z| < coarse_band for MLP fields, a CSG distance
// bound below the coarse cell's diagonal for CSG fields.
__global__ __launch_bounds__(256) void k_coarse_labels(const Job* __restrict__ jobs, int njobs) {
  __shared__ __align__(16) float act_lds[kBlock / 64][kActWords];
  float* act = act_lds[threadIdx.x >> 6];
  for_units(jobs, njobs, gwave(), nwaves(),
            [](const Job& J) { return J.coarse_step ? (coarse_corners(J) + 31) >> 5 : 0; },
            [&](const Job& J, int t) {
              const int ncc = coarse_corners(J), c1 = J.cn + 1, S = J.coarse_step;
              const int lane = lane_id();
              const int q = t * 32 + (lane & 31);
              const bool valid = q < ncc;
              const int qq = valid ? q : ncc - 1;
              const float gp[3] = {(float)(S * (qq % c1)), (float)(S * ((qq / c1) % c1)),
                                   (float)(S * (qq / (c1 * c1)))};
              float x[3];
              grid_world(J.g, gp, x);
              int lab, near = 0;
              if (J.kind == 0) {
                lab = csg_inside(J.prims, J.n_prims, x);
                near = fabsf(csg_distance(J.prims, J.n_prims, x)) < J.coarse_band;
              } else {
                const float z = mlp_logit_fp32(J.mlp, x, act);
                lab = z > 0.0f;
                near = fabsf(z) < J.coarse_band;
              }
              const uint64_t bl = __ballot(valid && lane < 32 && lab);
              const uint64_t bn = __ballot(valid && lane < 32 && near);
              if (lane == 0) {
                J.cbits[t] = (uint32_t)bl;
                J.cnear[t] = (uint32_t)bn;
                atomicAdd(&J.status[4], (unsigned long long)min(32, ncc - t * 32));
              }
            });
}

// Marked coarse cells: corners' labels differ, or one is within the band.
__global__ __launch_bounds__(256) void k_coarse_mark(const Job* __restrict__ jobs, int njobs) {
  for_units(jobs, njobs, gwave(), nwaves(),
            [](const Job& J) { return J.coarse_step ? (J.cn * J.cn * J.cn + 63) >> 6 : 0; },
            [&](const Job& J, int u) {
              const int cn = J.cn, c1 = cn + 1;
              const int cell = u * 64 + lane_id();
              int m = 0;
              if (cell < cn * cn * cn) {
                const int i = cell % cn, j = (cell / cn) % cn, k = cell / (cn * cn);
                int ones = 0, near = 0;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                  const int q = (i + (d & 1)) + c1 * ((j + ((d >> 1) & 1)) + c1 * (k + (d >> 2)));
                  ones += bit_of(J.cbits, q);
                  near |= bit_of(J.cnear, q);
                }
                m = (ones != 0 && ones != 8) || near;
              }
              const uint64_t b = __ballot(m);
              const int lane = lane_id();
              if (lane == 0) J.cmark[2 * u] = (uint32_t)b;
              if (lane == 32) J.cmark[2 * u + 1] = (uint32_t)(b >> 32);
            });
}

// Coarse cells holding fine coordinate p along an axis: lo..hi (two when p
// lies on a coarse plane inside the grid).
__device__ __forceinline__ void coarse_span(int p, int S, int cn, int& lo, int& hi) {
  lo = p > 0 ? (p - 1) / S : 0;
  hi = p / S < cn - 1 ? p / S : cn - 1;
}

// Whether some corner of fine corners c0..c1 (one word) lies in a marked
// coarse cell: the word's row segments against the marked bit set.
__device__ __forceinline__ bool word_needed(const Job& J, int c0, int c1) {
  const int n1 = J.g.N + 1, S = J.coarse_step, cn = J.cn;
  for (int r = c0 / n1; r <= c1 / n1; ++r) {
    const int xa = r == c0 / n1 ? c0 % n1 : 0, xb = r == c1 / n1 ? c1 % n1 : n1 - 1;
    int jl, jh, kl, kh, il, ih, t;
    coarse_span(r % n1, S, cn, jl, jh);
    coarse_span(r / n1, S, cn, kl, kh);
    coarse_span(xa, S, cn, il, t);
    coarse_span(xb, S, cn, t, ih);
    for (int k = kl; k <= kh; ++k)
      for (int j = jl; j <= jh; ++j)
        for (int i = il; i <= ih; ++i)
          if (bit_of(J.cmark, i + cn * (j + cn * k))) return true;
  }
  return false;
}

// The common coarse label of the unmarked coarse cells holding corner c.
__device__ __forceinline__ int corner_fill(const Job& J, int c) {
  const int n1 = J.g.N + 1, S = J.coarse_step, cn = J.cn, c1 = cn + 1;
  int lo[3], hi;
  coarse_span(c % n1, S, cn, lo[0], hi);
  coarse_span((c / n1) % n1, S, cn, lo[1], hi);
  coarse_span(c / (n1 * n1), S, cn, lo[2], hi);
  return bit_of(J.cbits, lo[0] + c1 * (lo[1] + c1 * lo[2]));
}

// The fine words (32 corners) that need the field, i.e. hold a corner of a
// marked coarse cell, are appended to J.wlist (count in status[5]); every
// other word takes its corners' coarse labels here.
__global__ __launch_bounds__(256) void k_fine_plan(const Job* __restrict__ jobs, int njobs) {
  for_units(jobs, njobs, gwave(), nwaves(),
            [](const Job& J) { return J.coarse_step ? (J.nw_c + 63) >> 6 : 0; },
            [&](const Job& J, int u) {
              const int lane = lane_id();
              const int t = u * 64 + lane;
              bool need = false;
              if (t < J.nw_c) {
                const int c0 = t * 32, c1 = (c0 + 32 < J.g.nc ? c0 + 32 : J.g.nc) - 1;
                need = word_needed(J, c0, c1);
                if (!need) {
                  uint32_t w = 0;
                  for (int c = c0; c <= c1; ++c) w |= (uint32_t)corner_fill(J, c) << (c - c0);
                  J.labels[t] = w;
                }
              }
              const uint64_t b = __ballot(need);
              unsigned long long base = 0;
              if (lane == 0 && b) {
                base = atomicAdd(&J.status[5], (unsigned long long)__popcll(b));
                // the listed words' corners are the fine corner queries (the
                // last word of the grid may be partial)
                const int lw = J.nw_c - 1 - u * 64;  // the grid's last word, if in this wave
                const bool last = lw >= 0 && lw < 64 && ((b >> lw) & 1ull);
                const int tail = J.g.nc - (J.nw_c - 1) * 32;
                atomicAdd(&J.status[4],
                          (unsigned long long)(32 * __popcll(b) - (last ? 32 - tail : 0)));
              }
              base = __shfl(base, 0);
              if (need) J.wlist[base + __popcll(b & ((1ull << lane) - 1ull))] = t;
            });
}

// Corner words of stage (a): all of them, or with adaptive evaluation the
// listed ones (n of them); fine_word maps a unit's word index to the word
// (past the end: nw_c, no word).
__device__ __forceinline__ int fine_words(const Job& J) {
  return J.coarse_step ? (int)J.status[5] : J.nw_c;
}
__device__ __forceinline__ int fine_word(const Job& J, int n, int i) {
  return J.coarse_step ? (i < n ? J.wlist[i] : J.nw_c) : i;
}

// ------------------------------------------------------------- (a) labels
// CSG corners, two words per wavefront (lane half h takes word 2u + h).
__global__ __launch_bounds__(256) void k_labels_csg(const Job* __restrict__ jobs, int njobs) {
  for_units(jobs, njobs, gwave(), nwaves(),
            [](const Job& J) { return J.kind == 0 ? (fine_words(J) + 1) >> 1 : 0; },
            [&](const Job& J, int u) {
              const Grid& g = J.g;
              const int lane = lane_id();
              const int t = fine_word(J, fine_words(J), 2 * u + (lane >> 5));
              const int c = t * 32 + (lane & 31);
              int lab = 0;
              if (t < J.nw_c && c < g.nc) {
                const int n1 = g.N + 1;
                const float gp[3] = {(float)(c % n1), (float)((c / n1) % n1),
                                     (float)(c / (n1 * n1))};
                float x[3];
                grid_world(g, gp, x);
                lab = csg_inside(J.prims, J.n_prims, x);
              }
              const uint64_t b = __ballot(lab);
              if ((lane & 31) == 0 && t < J.nw_c) J.labels[t] = (uint32_t)(lane ? b >> 32 : b);
            });
}

// MLP corners, 32 per wavefront.  fp32: each wavefront takes label words on
// its own.  bf16 (guard-band corners queued for fp32 re-evaluation): the four
// wavefronts of a workgroup evaluate their 128 corners together
// (mlp_logit_bf16_pp), so they take four consecutive words together
// (workgroup-uniform units, a wavefront past the end evaluating a clamped
// dummy) and every call is made by all four; two such workgroups share a
// compute unit (one wavefront of each per SIMD), so one's matrix work fills
// the other's waits.
// ADAPT: the jobs with adaptive corner evaluation (their listed words only),
// else the others (every word); separate kernels keep the list handling out
// of the plain pass's registers.
template <int BF16, bool ADAPT>
__global__ __launch_bounds__(256, BF16 ? 2 : 1) void k_labels_mlp(const Job* __restrict__ jobs,
                                                                 int njobs) {
  static_assert(kBlock == 256, "the bf16 evaluation takes four wavefronts");
  __shared__ __align__(16) float act_lds[BF16 ? 1 : kBlock / 64][BF16 ? 4 : kActWords];
  __shared__ __align__(16) char pp_lds[BF16 ? kPPLdsBytes : 16];
  // wave-uniform (the loads' scalar offsets depend on it)
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  float* act = act_lds[BF16 ? 0 : wave];
  auto body = [&](const Job& J, int t, float z) {
    const Grid& g = J.g;
    const int lane = lane_id();
    const bool unit = t < J.nw_c;
    const int c = t * 32 + (lane & 31);
    const bool valid = unit && c < g.nc;
    const uint64_t b = __ballot(valid && z > 0.0f);
    if (unit && lane == 0) J.labels[t] = (uint32_t)b;
    if (BF16) {
      const bool q = valid && lane < 32 && fabsf(z) < J.guard_logit;
      const uint64_t qb = __ballot(q);
      if (qb) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&J.status[0], (unsigned long long)__popcll(qb));
        base = __shfl(base, 0);
        if (q) {
          const unsigned long long r = base + __popcll(qb & ((1ull << lane) - 1ull));
          if (r < (unsigned long long)J.guard_cap) J.guard_list[r] = (uint32_t)c;
          else J.status[2] = 1;  // queue full: rerun with room for every corner
        }
      }
    }
  };
  // world position of corner word t's lane
  auto position = [&](const Job& J, int t, float x[3]) {
    const Grid& g = J.g;
    const int c = t * 32 + (lane_id() & 31);
    const int cc = t < J.nw_c && c < g.nc ? c : g.nc - 1;
    const int n1 = g.N + 1;
    const float gp[3] = {(float)(cc % n1), (float)((cc / n1) % n1), (float)(cc / (n1 * n1))};
    grid_world(g, gp, x);
  };
  // bf16 corners also for the split-bf16 precision (2); both re-evaluate
  // their guard band in fp32 (k_relabel_fp32), so their corner signs are
  // the fp32 path's
  const auto mine = [](const Job& J) {
    return J.kind == 1 && (BF16 ? J.precision >= 1 : J.precision == 0) &&
           (J.coarse_step != 0) == ADAPT;
  };
  auto n_words = [](const Job& J) { return ADAPT ? (int)J.status[5] : J.nw_c; };
  auto word_at = [](const Job& J, int n, int i) {
    return ADAPT ? (i < n ? J.wlist[i] : J.nw_c) : i;
  };
  if constexpr (BF16) {
    // the field's biases and output weights are staged, and the weight ring
    // primed, once per job
    for_unit_streams(jobs, njobs, (int)blockIdx.x, (int)gridDim.x,
                     [&](const Job& J) { return mine(J) ? (n_words(J) + 3) >> 2 : 0; },
                     [&](const Job& J, int u0, int count) {
                       lds_block_sync();  // the previous job's reads are done
                       stage_bias_wout(J.mlp, pp_lds + kPPBiasOff);
                       const PPStream S(J.mlp, wave);
                       v8bf W[kPPRing][2];
                       pp_prime(S, W);
                       lds_block_sync();
                       // the listed words' indices are read one call ahead
                       const int nw = n_words(J);
                       int tn = word_at(J, nw, 4 * u0 + wave);
                       for (int i = 0; i < count; ++i) {
                         const int t = tn;
                         if (i + 1 < count)
                           tn = word_at(J, nw, 4 * (u0 + (i + 1) * (int)gridDim.x) + wave);
                         float x[3];
                         position(J, t, x);
                         body(J, t, mlp_logit_bf16_pp(J.mlp, x, pp_lds, wave, S, W));
                       }
                     });
  } else {
    for_units(jobs, njobs, gwave(), nwaves(),
              [&](const Job& J) { return mine(J) ? n_words(J) : 0; },
              [&](const Job& J, int i) {
                const int t = word_at(J, n_words(J), i);
                float x[3];
                position(J, t, x);
                body(J, t, mlp_logit_fp32(J.mlp, x, act));
              });
  }
}

// fp32 re-evaluation of the corners queued by the bf16 pass
__global__ __launch_bounds__(256) void k_relabel_fp32(const Job* __restrict__ jobs, int njobs) {
  __shared__ __align__(16) float act_lds[kBlock / 64][kActWords];
  float* act = act_lds[threadIdx.x >> 6];
  for_units(jobs, njobs, gwave(), nwaves(),
            [](const Job& J) {
              if (J.kind != 1 || J.precision == 0) return 0;
              const unsigned long long n = J.status[0];
              const int m = (int)(n < (unsigned long long)J.guard_cap ? n : J.guard_cap);
              return (m + 31) >> 5;
            },
            [&](const Job& J, int t) {
              const Grid& g = J.g;
              const unsigned long long nq = J.status[0];
              const int n = (int)(nq < (unsigned long long)J.guard_cap ? nq : J.guard_cap);
              const int lane = lane_id();
              const int xi = t * 32 + (lane & 31);
              const bool valid = xi < n;
              const int c = (int)J.guard_list[valid ? xi : n - 1];
              const int n1 = g.N + 1;
              const float gp[3] = {(float)(c % n1), (float)((c / n1) % n1),
                                   (float)(c / (n1 * n1))};
              float x[3];
              grid_world(g, gp, x);
              const float z = mlp_logit_fp32(J.mlp, x, act);
              if (valid && lane < 32) {
                const uint32_t bit = 1u << (c & 31);
                if (z > 0.0f) atomicOr(&J.labels[c >> 5], bit);
                else atomicAnd(&J.labels[c >> 5], ~bit);
              }
            });
}

// ---------------------------------------------------------- classification
// The classification passes walk contiguous chunks of 64-element units,
// each lane carrying its element's grid position from unit to unit
// (BlockWalk): the per-element index divisions would otherwise dominate
// these passes.
__global__ __launch_bounds__(256) void k_classify_edges(const Job* __restrict__ jobs, int njobs) {
  for_unit_chunks(jobs, njobs, gwave(), nwaves(),
                  [](const Job& J) { return (3 * J.g.ea + 63) >> 6; },
                  [&](const Job& J, int u0, int u1) {
                    const Grid& g = J.g;
                    const int lane = lane_id();
                    BlockWalk w;
                    w.init(g, 0, u0 * 64 + lane);
                    for (int u = u0; u < u1; ++u, w.advance64()) {
                      const int e = u * 64 + lane;
                      int x = 0;
                      if (e < 3 * g.ea) {
                        const int c0 = corner_index(g, w.p[0], w.p[1], w.p[2]);
                        const int step =
                            w.a == 0 ? 1 : (w.a == 1 ? g.N + 1 : (g.N + 1) * (g.N + 1));
                        x = bit_of(J.labels, c0) != bit_of(J.labels, c0 + step);
                      }
                      const uint64_t b = __ballot(x);
                      store_ballot(b, u * 64, J.nw_e, J.emask);
                      const int w0 = u * 2;
                      if (lane == 0 && w0 < J.nw_e) J.ecount[w0] = __popc((uint32_t)b);
                      if (lane == 32 && w0 + 1 < J.nw_e)
                        J.ecount[w0 + 1] = __popc((uint32_t)(b >> 32));
                    }
                  });
}

// labels of the 8 corners of cell (i,j,k): bit lc = x + 2y + 4z
__device__ __forceinline__ int cell_config(const Grid& g, const uint32_t* __restrict__ L, int i,
                                           int j, int k) {
  const int c = corner_index(g, i, j, k);
  const int n1 = g.N + 1, n2 = n1 * n1;
  return bit_of(L, c) | (bit_of(L, c + 1) << 1) | (bit_of(L, c + n1) << 2) |
         (bit_of(L, c + n1 + 1) << 3) | (bit_of(L, c + n2) << 4) | (bit_of(L, c + n2 + 1) << 5) |
         (bit_of(L, c + n2 + n1) << 6) | (bit_of(L, c + n2 + n1 + 1) << 7);
}

__device__ __forceinline__ void face_labels(const Grid& g, const uint32_t* __restrict__ L, int a,
                                            const int p[3], int out[4]) {
  int u, v;
  other_axes(a, u, v);
#pragma unroll
  for (int lc = 0; lc < 4; ++lc) {
    int q[3] = {p[0], p[1], p[2]};
    add_at3(q, u, lc & 1);
    add_at3(q, v, lc >> 1);
    out[lc] = bit_of(L, corner_index(g, q[0], q[1], q[2]));
  }
}

// Manifold fix (App. A.1.1): an ambiguous face whose plain partitions merge
// its two pairs in both adjacent cells takes the other pairing.
__device__ inline int face_flip(const Grid& g, const uint32_t* __restrict__ L,
                                const uint32_t* __restrict__ table, int a, const int p[3]) {
  if (p[a] <= 0 || p[a] >= g.N) return 0;
  int merged = 1;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    int c[3] = {p[0], p[1], p[2]};
    int s_in_cell = 0;
    if (side == 0) {
      c[a] -= 1;
      s_in_cell = 1;
    }
    const int cfg = cell_config(g, L, c[0], c[1], c[2]);
    const uint32_t pm = table[cfg] & 0xFFFFFFu;
    const int e0 = face_to_cell_edge(a, s_in_cell, 0);
    const int e1 = face_to_cell_edge(a, s_in_cell, 1);
    if (((pm >> (2 * e0)) & 3u) != ((pm >> (2 * e1)) & 3u)) merged = 0;
  }
  return merged;
}

__global__ __launch_bounds__(256) void k_classify_faces(const Job* __restrict__ jobs, int njobs,
                                                        const uint32_t* __restrict__ table) {
  for_unit_chunks(jobs, njobs, gwave(), nwaves(),
                  [](const Job& J) { return (3 * J.g.fa + 63) >> 6; },
                  [&](const Job& J, int u0, int u1) {
                    const Grid& g = J.g;
                    const int lane = lane_id();
                    BlockWalk w;
                    w.init(g, 1, u0 * 64 + lane);
                    int flips = 0;  // wave-uniform
                    for (int u = u0; u < u1; ++u, w.advance64()) {
                      const int f = u * 64 + lane;
                      int act = 0, amb = 0, flip = 0;
                      if (f < 3 * g.fa) {
                        int Lf[4];
                        face_labels(g, J.labels, w.a, w.p, Lf);
                        const int n = __popc(face_crossing_mask(Lf));
                        act = n > 0;
                        amb = n == 4;
                        if (amb) flip = face_flip(g, J.labels, table, w.a, w.p);
                      }
                      const uint64_t ba = __ballot(act), bb = __ballot(amb), bf = __ballot(flip);
                      store_ballot(ba, u * 64, J.nw_f, J.fact);
                      store_ballot(bb, u * 64, J.nw_f, J.famb);
                      store_ballot(bf, u * 64, J.nw_f, J.fflip);
                      flips += __popcll(bf);
                      const int w0 = u * 2;
                      if (lane == 0 && w0 < J.nw_f)
                        J.pcount[w0] = __popc((uint32_t)ba) + __popc((uint32_t)bb);
                      if (lane == 32 && w0 + 1 < J.nw_f)
                        J.pcount[w0 + 1] =
                            __popc((uint32_t)(ba >> 32)) + __popc((uint32_t)(bb >> 32));
                    }
                    if (lane == 0 && flips)
                      atomicAdd(&J.status[6], (unsigned long long)flips);
                  });
}

__global__ __launch_bounds__(256) void k_classify_cells(const Job* __restrict__ jobs, int njobs) {
  for_unit_chunks(jobs, njobs, gwave(), nwaves(),
                  [](const Job& J) { return (J.g.ncell + 63) >> 6; },
                  [&](const Job& J, int u0, int u1) {
                    const Grid& g = J.g;
                    const int lane = lane_id();
                    BlockWalk w;
                    w.init(g, 2, u0 * 64 + lane);
                    for (int u = u0; u < u1; ++u, w.advance64()) {
                      const int c = u * 64 + lane;
                      int x = 0;
                      if (c < g.ncell) {
                        const int cfg = cell_config(g, J.labels, w.p[0], w.p[1], w.p[2]);
                        x = cfg != 0 && cfg != 255;
                      }
                      const uint64_t b = __ballot(x);
                      store_ballot(b, u * 64, J.nw_cell, J.cmask);
                      const int w0 = u * 2;
                      if (lane == 0 && w0 < J.nw_cell) J.ccount[w0] = __popc((uint32_t)b);
                      if (lane == 32 && w0 + 1 < J.nw_cell)
                        J.ccount[w0 + 1] = __popc((uint32_t)(b >> 32));
                    }
                  });
}

// ------------------------------------------------------------ compaction
// Lists in ascending id order; entries past the capacity are dropped and the
// job is flagged for a larger scratch.
__global__ __launch_bounds__(256) void k_compact(const Job* __restrict__ jobs, int njobs) {
  for_units(jobs, njobs, gthread(), nthreads(),
            [](const Job& J) { return J.nw_e + J.nw_f + J.nw_cell; },
            [&](const Job& J, int u) {
              if (u < J.nw_e) {
                uint32_t m = J.emask[u];
                int o = (int)J.eprefix[u];
                while (m) {
                  const int b = __ffs(m) - 1;
                  if (o < J.cap_edges) J.elist[o] = u * 32 + b;
                  else J.status[2] = 1;
                  ++o;
                  m &= m - 1u;
                }
                return;
              }
              u -= J.nw_e;
              if (u < J.nw_f) {
                uint32_t m = J.fact[u];
                const uint32_t a2 = J.famb[u];
                int o = (int)J.pprefix[u];
                while (m) {
                  const int b = __ffs(m) - 1;
                  const int f = u * 32 + b;
                  if (o < J.cap_pairs) J.plist[o] = f << 1;
                  else J.status[2] = 1;
                  ++o;
                  if ((a2 >> b) & 1u) {
                    if (o < J.cap_pairs) J.plist[o] = (f << 1) | 1;
                    else J.status[2] = 1;
                    ++o;
                  }
                  m &= m - 1u;
                }
                return;
              }
              u -= J.nw_f;
              uint32_t m = J.cmask[u];
              int o = (int)J.cprefix[u];
              while (m) {
                const int b = __ffs(m) - 1;
                if (o < J.cap_cells) J.clist[o] = u * 32 + b;
                else J.status[2] = 1;
                ++o;
                m &= m - 1u;
              }
            });
}

// --------------------------------------------------------- label functors
struct CsgLabel {
  const Grid* g;
  const float* prims;
  int n;
  __device__ __forceinline__ int operator()(const float gp[3]) const {
    float x[3];
    grid_world(*g, gp, x);
    return csg_inside(prims, n, x);
  }
};

// wave-cooperative: every lane of the wave must call it together
struct MlpLabel {
  const Grid* g;
  const Mlp* m;
  float* act;  // this wavefront's LDS activation region
  __device__ __forceinline__ int operator()(const float gp[3]) const {
    float x[3];
    grid_world(*g, gp, x);
    return mlp_logit_fp32(*m, x, act) > 0.0f;
  }
  // whether any lane of the wavefront (which evaluates together) has a query
  __device__ __forceinline__ bool any(bool q) const { return __any(q); }
};

// workgroup-cooperative (split-bf16 evaluation): the four wavefronts of the
// workgroup call it together, each for its 32 elements
struct X3Label {
  const Grid* g;
  const Mlp* m;
  char* lds;
  int wave;
  mutable int parity;
  __device__ __forceinline__ int operator()(const float gp[3]) const {
    float x[3];
    grid_world(*g, gp, x);
    return mlp_logit_x3(*m, x, lds, wave) > 0.0f;
  }
  // whether any lane of the workgroup (which evaluates together) has a query
  __device__ __forceinline__ bool any(bool q) const {
    parity ^= 1;
    return !x3_vote_all(lds, wave, parity, !q);
  }
};

// ------------------------------------------------------------ (b) 1D points
// Bisection (Sec. 5.1): k halvings of [0,1] keeping distinct end labels; the
// point is the middle of the final bracket.
// `bits` receives the label of every query (bit it for halving it), the
// decision trace that a checker can replay.
template <class Lab>
__device__ __forceinline__ float bisect_edge(const Job& j, const Lab& lab, int id,
                                             uint32_t& bits) {
  int a, p[3];
  edge_pos(j.g, id, a, p);
  const int l0 = bit_of(j.labels, corner_index(j.g, p[0], p[1], p[2]));
  float lo = 0.0f, hi = 1.0f;
  bits = 0u;
  for (int it = 0; it < j.iters_1d; ++it) {
    const float mid = (lo + hi) * 0.5f;
    float gp[3] = {(float)p[0], (float)p[1], (float)p[2]};
    gp[a] = (float)p[a] + mid;
    const int l = lab(gp);
    bits |= (uint32_t)l << it;
    if (l == l0) lo = mid;
    else hi = mid;
  }
  return (lo + hi) * 0.5f;
}

__global__ __launch_bounds__(256) void k_bisect_csg(const Job* __restrict__ jobs, int njobs) {
  for_units(jobs, njobs, gthread(), nthreads(),
            [](const Job& J) { return J.kind == 0 ? n_edges_of(J) : 0; },
            [&](const Job& J, int x) {
              if (J.ablation & kAblLinear1D) {
                // Eq. 1 on binary occupancy: psi = +-1/2 at the two ends
                J.et[x] = 0.5f;
                return;
              }
              CsgLabel lab{&J.g, J.prims, J.n_prims};
              uint32_t bits;
              J.et[x] = bisect_edge(J, lab, J.elist[x], bits);
              if (J.etrace) J.etrace[x] = bits;
            });
}

// Eq. 1 (the linear-1D ablation): psi = phi - 1/2 = tanh(z/2)/2 at the two
// corners of the edge (z itself for SDF input), t = psi0 / (psi0 - psi1),
// binary32.
__device__ __forceinline__ float linear_edge_mlp(const Job& J, int e, float* act) {
  int a, p[3];
  edge_pos(J.g, e, a, p);
  float psi[2];
#pragma unroll 1
  for (int end = 0; end < 2; ++end) {
    const float gp[3] = {(float)p[0], (float)p[1], (float)p[2]};
    float x[3];
    grid_world(J.g, gp, x);
    const float z = mlp_logit_fp32(J.mlp, x, act);
    psi[end] = (J.ablation & kAblSdfInput) ? z : 0.5f * tanhf(0.5f * z);
    add_at3(p, a, 1);
  }
  return psi[0] / (psi[0] - psi[1]);
}

__global__ __launch_bounds__(256) void k_bisect_mlp(const Job* __restrict__ jobs, int njobs) {
  __shared__ __align__(16) float act_lds[kBlock / 64][kActWords];
  float* act = act_lds[threadIdx.x >> 6];
  for_units_drawn(jobs, njobs,
            [](const Job& J) {
              return J.kind == 1 && J.precision != 2 ? (n_edges_of(J) + 31) >> 5 : 0;
            },
            [](const Job& J) { return &J.status[8]; },
            [&](const Job& J, int t) {
              const int ne = n_edges_of(J);
              const int lane = lane_id();
              const int x = t * 32 + (lane & 31);
              const bool valid = x < ne;
              const int e = J.elist[valid ? x : ne - 1];
              float tt;
              uint32_t bits = 0u;
              if (J.ablation & kAblLinear1D) {
                tt = linear_edge_mlp(J, e, act);
              } else {
                MlpLabel lab{&J.g, &J.mlp, act};
                tt = bisect_edge(J, lab, e, bits);
              }
              if (valid && lane < 32) {
                J.et[x] = tt;
                if (J.etrace) J.etrace[x] = bits;
              }
            });
}

// Split-bf16 evaluation (precision 2): a workgroup takes 128 crossing edges,
// 32 per wavefront, and the four evaluate each bisection query together.
__global__ __launch_bounds__(256) void k_bisect_x3(const Job* __restrict__ jobs, int njobs) {
  __shared__ __align__(16) char lds[kX3LdsBytes];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for_units(jobs, njobs, (int)blockIdx.x, (int)gridDim.x,
            [](const Job& J) { return J.kind == 1 && J.precision == 2 ? (n_edges_of(J) + 127) >> 7 : 0; },
            [&](const Job& J, int t) {
              lds_block_sync();  // the previous unit's reads of the staged field are done
              x3_stage(J.mlp, lds);
              lds_block_sync();
              const int ne = n_edges_of(J);
              const int lane = lane_id();
              const int x = t * 128 + wave * 32 + (lane & 31);
              const bool valid = x < ne;
              const int e = J.elist[valid ? x : ne - 1];
              X3Label lab{&J.g, &J.mlp, lds, wave, 0};
              uint32_t bits;
              const float tt = bisect_edge(J, lab, e, bits);
              if (valid && lane < 32) {
                J.et[x] = tt;
                if (J.etrace) J.etrace[x] = bits;
              }
            });
}

// Gradient of the logit at each crossing edge's 1D point (the gradient-normal
// ablation, Eq. 2), by forward-mode differentiation on the matrix cores:
// 8 edges per wavefront pass, 4 channels each (value and 3 derivatives).
__global__ __launch_bounds__(256) void k_grad_mlp(const Job* __restrict__ jobs, int njobs) {
  __shared__ __align__(16) float act_lds[kBlock / 64][kActWords];
  float* act = act_lds[threadIdx.x >> 6];
  for_units(jobs, njobs, gwave(), nwaves(),
            [](const Job& J) {
              return (J.kind == 1 && (J.ablation & kAblGradNormals)) ? (n_edges_of(J) + 7) >> 3
                                                                      : 0;
            },
            [&](const Job& J, int t) {
              const int ne = n_edges_of(J);
              const int lane = lane_id();
              const int q = (lane & 31) >> 2, ch = lane & 3;
              const int x = t * 8 + q;
              const bool valid = x < ne;
              const int xi = valid ? x : ne - 1;
              int a, p[3];
              edge_pos(J.g, J.elist[xi], a, p);
              float gp[3] = {(float)p[0], (float)p[1], (float)p[2]};
              set_at3(gp, a, (float)at3(p, a) + J.et[xi]);
              float w[3];
              grid_world(J.g, gp, w);
              const float v = mlp_logit_fp32<true>(J.mlp, w, act);
              if (valid && lane < 32 && ch != 0) J.egrad[3 * x + ch - 1] = v;
            });
}

// ------------------------------------------------------------ (c) 2D points
struct FaceFrame {
  int a, u, v;
  int p[3];
};

__device__ __forceinline__ void face_edge_point(int fe, float t, float P[2]) {
  P[0] = fe < 2 ? t : (float)(fe - 2);
  P[1] = fe < 2 ? (float)fe : t;
}

__device__ __forceinline__ int face_edge_global(const Grid& g, const FaceFrame& fr, int fe) {
  int q[3] = {fr.p[0], fr.p[1], fr.p[2]};
  int axis;
  if (fe < 2) {
    axis = fr.u;
    add_at3(q, fr.v, fe);
  } else {
    axis = fr.v;
    add_at3(q, fr.u, fe - 2);
  }
  return edge_index(g, axis, q[0], q[1], q[2]);
}

// One line-binary search (App. A.1.3) driven one query at a time: samples
// p0 + (R i / N) d for i = 1..N; the first whose label differs from s0 (else
// i = N) bounds the bracket; then halvings compare the middle with the near
// end, which keeps the label s0.
struct LineBinary {
  float p0[2], d[2];
  float R, nr, fa;
  int nl, s0, istar, found;
  __device__ __forceinline__ void start(const float a[2], const float dir[2], int s, float r,
                                        int n) {
    p0[0] = a[0];
    p0[1] = a[1];
    d[0] = dir[0];
    d[1] = dir[1];
    s0 = s;
    R = r;
    nl = n;
    istar = n;
    found = 0;
  }
  __device__ __forceinline__ float param(int k) const {
    return k < nl ? (R * (float)(k + 1)) / (float)nl : (nr + fa) * 0.5f;
  }
  __device__ __forceinline__ void point(float s, float P[2]) const {
    const float su = s * d[0], sv = s * d[1];
    P[0] = p0[0] + su;
    P[1] = p0[1] + sv;
  }
  __device__ __forceinline__ void consume(int k, float s, int lab) {
    if (k < nl) {
      if (lab != s0 && !found) {
        istar = k + 1;
        found = 1;
      }
      if (k == nl - 1) {
        nr = (istar == 1) ? 0.0f : (R * (float)(istar - 1)) / (float)nl;
        fa = (R * (float)istar) / (float)nl;
      }
    } else {
      // both ends written through selects: a store whose address depends on
      // the label would keep the state out of registers
      const bool keep = lab == s0;
      nr = keep ? s : nr;
      fa = keep ? fa : s;
    }
  }
};

// The three steps of Sec. 5.2 for pair `slot` of face `face`, as a resumable
// sequence of 1 + (lin1 + bin1) + 2 (lin2 + bin2) occupancy queries: next()
// gives the grid point of the next query the pair needs, take() consumes its
// label, result() is the 2D point once next() reports the end.  A driver
// can thus interleave the queries of many pairs (one lane per pair, each at
// its own place in its sequence) into one batched evaluation.
//
// With `skip`, queries the method does not need are passed over: a linear
// sample after its ray's first label change (the change already fixed i*),
// and step 2 when step 1 ends at m (the point is m).  Without it every query
// of the sequence is made (the results are the same).
//
// Query q of the sequence (0 = m, then step 1's ray, then step 2's two rays)
// sets bit q of `evald` when it is evaluated and bit q of `bits` to its
// label: the decision trace that a checker can replay.  `need` counts the
// queries made.
struct PairSearch {
  FaceFrame fr;
  float P1[2], P2[2], m[2], q[2], q1[2], H[4];
  float s1, cs;
  LineBinary lb;
  int lmask, sm, n1, n2, total, step, ck, need;
  uint64_t bits, evald;

  __device__ __forceinline__ void init(const Job& j, int face, int slot) {
    const Grid& g = j.g;
    face_pos(g, face, fr.a, fr.p);
    other_axes(fr.a, fr.u, fr.v);
    int L[4], pa[2], pb[2];
    face_labels(g, j.labels, fr.a, fr.p, L);
    face_pairs(L, bit_of(j.fflip, face), pa, pb);
    lmask = L[0] | (L[1] << 1) | (L[2] << 2) | (L[3] << 3);
    const int fa = slot ? pa[1] : pa[0], fb = slot ? pb[1] : pb[0];
    const float t1 = j.et[edge_slot(j, face_edge_global(g, fr, fa))];
    const float t2 = j.et[edge_slot(j, face_edge_global(g, fr, fb))];
    face_edge_point(fa, t1, P1);
    face_edge_point(fb, t2, P2);
    // which side of the chord a corner lies on does not depend on t in
    // (0,1); it is evaluated at t = 1/2, where the products are exact
    face_edge_point(fa, 0.5f, H);
    face_edge_point(fb, 0.5f, H + 2);
    m[0] = (P1[0] + P2[0]) * 0.5f;
    m[1] = (P1[1] + P2[1]) * 0.5f;
    q[0] = m[0];
    q[1] = m[1];
    q1[0] = q1[1] = 0.0f;
    s1 = 0.0f;
    sm = 0;
    n1 = j.lin1 + j.bin1;
    n2 = j.lin2 + j.bin2;
    total = 1 + n1 + 2 * n2;
    step = 0;
    need = 0;
    bits = 0ull;
    evald = 0ull;
  }

  // the ray transitions after the query at `step` (Sec. 5.2 steps 1 and 2)
  __device__ __forceinline__ void after(const Job& j) {
    if (step == n1) {
      // end of step 1: q; step 2 starts towards P1
      s1 = lb.nr;
      lb.point(s1, q);
      const float wu = P1[0] - m[0], wv = P1[1] - m[1];
      const float ww = wu * wu, vv = wv * wv;
      const float lw = sqrtf(ww + vv);
      const float uh[2] = {wu / lw, wv / lw};
      lb.start(q, uh, sm, j.range2, j.lin2);
    } else if (step == n1 + n2) {
      lb.point(lb.nr, q1);
      const float un[2] = {-lb.d[0], -lb.d[1]};
      lb.start(q, un, sm, j.range2, j.lin2);
    }
  }

  __device__ __forceinline__ bool next(const Job& j, bool skip, float gp[3]) {
    while (step < total) {
      float P[2];
      if (step == 0) {
        P[0] = m[0];
        P[1] = m[1];
      } else {
        if (skip && step > n1 && s1 == 0.0f) {  // step 1 ended at m
          step = total;
          break;
        }
        // index of the query within its own ray
        const int k =
            step <= n1 ? step - 1 : (step <= n1 + n2 ? step - 1 - n1 : step - 1 - n1 - n2);
        if (skip && k < lb.nl && lb.found) {
          // the ray's remaining linear samples cannot move the bracket: go
          // straight to its last one, whose bookkeeping fixes the bracket
          // (the label is unused)
          step += lb.nl - 1 - k;
          lb.consume(lb.nl - 1, 0.0f, 0);
          after(j);
          ++step;
          continue;
        }
        const float s = lb.param(k);
        ck = k;
        cs = s;
        lb.point(s, P);
      }
      gp[0] = (float)fr.p[0];
      gp[1] = (float)fr.p[1];
      gp[2] = (float)fr.p[2];
      add_at3(gp, fr.u, P[0]);
      add_at3(gp, fr.v, P[1]);
      return true;
    }
    return false;
  }

  __device__ __forceinline__ void take(const Job& j, int l) {
    if (step < 64) {  // sequences longer than 64 queries are not traced
      evald |= 1ull << step;
      bits |= (uint64_t)l << step;
    }
    ++need;
    if (step == 0) {
      // step 1: the ray from m orthogonal to l, towards a corner whose label
      // differs from m's; when both sides qualify, the side of the corner the
      // pair cuts off
      sm = l;
      const float du = P2[0] - P1[0], dv = P2[1] - P1[1];
      const float dd = du * du, ee = dv * dv;
      const float len = sqrtf(dd + ee);
      const float perp[2] = {-dv / len, du / len};  // left of P1 -> P2
      int nleft = 0, nright = 0, dleft = 0, dright = 0;
#pragma unroll
      for (int lc = 0; lc < 4; ++lc) {
        const float cu = (float)(lc & 1), cv = (float)(lc >> 1);
        const float cr = (H[2] - H[0]) * (cv - H[1]) - (H[3] - H[1]) * (cu - H[0]);
        const int differs = ((lmask >> lc) & 1) != sm;
        if (cr > 0.0f) {
          ++nleft;
          dleft |= differs;
        } else {
          ++nright;
          dright |= differs;
        }
      }
      const int go_left =
          (dleft && !dright) ? 1 : ((dright && !dleft) ? 0 : (nleft <= nright ? 1 : 0));
      const float d[2] = {go_left ? perp[0] : -perp[0], go_left ? perp[1] : -perp[1]};
      lb.start(m, d, sm, j.range1, j.lin1);
    } else {
      lb.consume(ck, cs, l);
      after(j);
    }
    ++step;
  }

  __device__ __forceinline__ double2 result() const {
    if (s1 == 0.0f) return make_double2(m[0], m[1]);
    float q2[2];
    lb.point(lb.nr, q2);
    // step 3: intersection of line(P1,q1) and line(P2,q2).  On smooth
    // surfaces l1 and l2 are nearly parallel (sin ~ 1e-4), where binary32
    // differences of the inputs alone move the apex by 1e-7/sin; the solve
    // is binary64 (the differences of binary32 inputs are then exact) and
    // the point is kept in binary64: where a cell cuts a tiny corner, its 2D
    // points sit within 1e-5 of their 1D points near face coordinate 1, below
    // binary32 resolution there relative to the distance that sets the normal.
    const double Au = (double)q1[0] - (double)P1[0], Av = (double)q1[1] - (double)P1[1];
    const double Bu = (double)q2[0] - (double)P2[0], Bv = (double)q2[1] - (double)P2[1];
    const double det = Au * Bv - Av * Bu;
    if (det == 0.0) return make_double2(q[0], q[1]);
    const double Du = (double)P2[0] - (double)P1[0], Dv = (double)P2[1] - (double)P1[1];
    const double alpha = (Du * Bv - Dv * Bu) / det;
    return make_double2((double)P1[0] + alpha * Au, (double)P1[1] + alpha * Av);
  }
};

// Analytic fields: one thread per pair, making the queries the pair needs
// (the early exits of PairSearch), counted per wavefront into status[3].
// The job-major distribution of for_units, written out so that the whole
// wavefront sums its count after each job's pairs.
__global__ __launch_bounds__(256) void k_search2d_csg(const Job* __restrict__ jobs, int njobs) {
  const __attribute__((address_space(4))) Job* cj =
      (const __attribute__((address_space(4))) Job*)jobs;
  const int worker = gthread(), W = nthreads();
  long long rot = 0;
  for (int k = 0; k < njobs; ++k) {
    const Job& J = *(const Job*)&cj[k];
    const int n = J.kind == 0 ? n_pairs_of(J) : 0;
    if (n <= 0) continue;
    int u0 = (int)(((long long)worker - rot) % W);
    if (u0 < 0) u0 += W;
    int need = 0;
    for (int x = u0; x < n; x += W) {
      CsgLabel lab{&J.g, J.prims, J.n_prims};
      const int rec = J.plist[x];
      PairSearch ps;
      ps.init(J, rec >> 1, rec & 1);
      float gp[3];
      while (ps.next(J, true, gp)) ps.take(J, lab(gp));
      J.pf[x] = ps.result();
      if (J.ptrace) {
        J.ptrace[2 * x] = ps.bits;
        J.ptrace[2 * x + 1] = ps.evald;
      }
      need += ps.need;
    }
    const int nsum = wave_sum(need);
    if (lane_id() == 0 && nsum) atomicAdd(&J.status[3], (unsigned long long)nsum);
    rot += n;
  }
}

// MLP fields: a wavefront keeps 32 pairs in flight, one per lane (lanes
// l and l + 32 mirror each other: they hold the two K halves of one query
// column), and evaluates the next query of all of them at once.  A lane whose
// pair ends takes the next pair of the wavefront's stream at once, so lanes
// do not wait for the slowest pair of a group, and each pair makes only the
// queries it needs.  The stream is the pairs of the units this worker owns
// (units of `per_unit` pairs; this wavefront's 32 of each start at `off`):
// units u0, u0 + W, ... (n_units of them), or, with kDyn, units of the job's
// n_units taken from its counter `ctr` as the wavefront needs them, so
// wavefronts that draw short pairs take more units and all end together.
// `lab.any` ends the loop when no lane of the evaluating group has a query.
template <class Lab, bool kDyn = false>
__device__ __forceinline__ void search_stream(const Job& J, const Lab& lab, int u0, int W,
                                              int n_units, int per_unit, int off,
                                              unsigned long long* ctr = nullptr) {
  const int np = n_pairs_of(J);
  const int lane = lane_id(), ln = lane & 31;
  const int slen = n_units * 32;
  int next = 0, have = 0, x = 0, need = 0;
  // kDyn: the units of stream slots next / 32 and the one after
  int ub0 = 0, ub1 = 0;
  if (kDyn) {
    ub0 = take_unit(ctr);
    ub1 = take_unit(ctr);
  }
  PairSearch ps;
  while (true) {
    float gp[3] = {0.0f, 0.0f, 0.0f};
    bool q = false;
    if (have) {
      q = ps.next(J, true, gp);
      if (!q) {
        if (lane < 32) {
          J.pf[x] = ps.result();
          if (J.ptrace) {
            J.ptrace[2 * x] = ps.bits;
            J.ptrace[2 * x + 1] = ps.evald;
          }
        }
        need += ps.need;
        have = 0;
      }
    }
    // refill: the free lanes (the same in both halves) take the next pairs
    const uint32_t free_lanes = (uint32_t)__ballot(!have);
    if (free_lanes != 0u && (kDyn ? ub0 < n_units : next < slen)) {
      const int pos = next + __popc(free_lanes & ((1u << ln) - 1u));
      const int slot0 = next >> 5;
      next += __popc(free_lanes);
      // at most 32 lanes are free, so pos lies in slot0 or the slot after
      const int unit = kDyn ? ((pos >> 5) == slot0 ? ub0 : ub1) : u0 + (pos >> 5) * W;
      if (kDyn && (next >> 5) != slot0) {
        ub0 = ub1;
        ub1 = take_unit(ctr);
      }
      if (!have && (kDyn ? unit < n_units : pos < slen)) {
        const int xi = unit * per_unit + off + (pos & 31);
        if (xi < np) {
          x = xi;
          const int rec = J.plist[x];
          ps.init(J, rec >> 1, rec & 1);
          have = 1;
          q = ps.next(J, true, gp);  // m: always made
        }
      }
    }
    if (!lab.any(q)) break;
    const int l = lab(gp);
    if (q) ps.take(J, l);
  }
  const int nsum = wave_sum(lane < 32 ? need : 0);
  if (lane == 0 && nsum) atomicAdd(&J.status[3], (unsigned long long)nsum);
}

// Every wavefront takes part in every job, drawing units of 32 pairs from
// the job's counter (status[7]) until they run out.
__global__ __launch_bounds__(256) void k_search2d_mlp(const Job* __restrict__ jobs, int njobs) {
  __shared__ __align__(16) float act_lds[kBlock / 64][kActWords];
  float* act = act_lds[threadIdx.x >> 6];
  const __attribute__((address_space(4))) Job* cj =
      (const __attribute__((address_space(4))) Job*)jobs;
  for (int k = 0; k < njobs; ++k) {
    const Job& J = *(const Job*)&cj[k];
    if (!(J.kind == 1 && J.precision != 2 && !(J.ablation & kAblGradNormals))) continue;
    const int nu = (n_pairs_of(J) + 31) >> 5;
    if (nu == 0) continue;
    MlpLabel lab{&J.g, &J.mlp, act};
    search_stream<MlpLabel, true>(J, lab, 0, 0, nu, 32, 0, &J.status[7]);
  }
}

// Split-bf16 evaluation (precision 2): a workgroup keeps 128 pairs in
// flight, 32 per wavefront, and the four evaluate each round of queries
// together; it stops when none of the four has a query left.
// Every workgroup takes part in every job; each wavefront draws its units
// of 32 pairs from the job's counter (status[7]) on its own, and the four
// keep evaluating together until none of them has a query.
__global__ __launch_bounds__(256) void k_search2d_x3(const Job* __restrict__ jobs, int njobs) {
  __shared__ __align__(16) char lds[kX3LdsBytes];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const __attribute__((address_space(4))) Job* cj =
      (const __attribute__((address_space(4))) Job*)jobs;
  for (int k = 0; k < njobs; ++k) {
    const Job& J = *(const Job*)&cj[k];
    if (!(J.kind == 1 && J.precision == 2)) continue;
    const int nu = (n_pairs_of(J) + 31) >> 5;
    if (nu == 0) continue;
    lds_block_sync();  // the previous job's reads of the staged field are done
    x3_stage(J.mlp, lds);
    lds_block_sync();
    X3Label lab{&J.g, &J.mlp, lds, wave, 0};
    search_stream<X3Label, true>(J, lab, 0, 0, nu, 32, 0, &J.status[7]);
  }
}

// ----------------------------------------------------- (d) partitions, QEF
__device__ __forceinline__ void cell_of(const Grid& g, int cid, int c[3]) {
  c[0] = cid % g.N;
  c[1] = (cid / g.N) % g.N;
  c[2] = cid / (g.N * g.N);
}

__device__ __forceinline__ int cell_flipmask(const Grid& g, const uint32_t* __restrict__ fflip,
                                             const int c[3]) {
  int fm = 0;
#pragma unroll
  for (int lf = 0; lf < 6; ++lf) {
    const int a = lf >> 1;
    int q[3] = {c[0], c[1], c[2]};
    q[a] += lf & 1;
    fm |= bit_of(fflip, face_index(g, a, q[0], q[1], q[2])) << lf;
  }
  return fm;
}

__global__ __launch_bounds__(256) void k_cell_count(const Job* __restrict__ jobs, int njobs,
                                                    const uint32_t* __restrict__ table) {
  for_units(jobs, njobs, gthread(), nthreads(), [](const Job& J) { return n_cells_of(J); },
            [&](const Job& J, int x) {
              int c[3];
              cell_of(J.g, J.clist[x], c);
              const int cfg = cell_config(J.g, J.labels, c[0], c[1], c[2]);
              const int fm = cell_flipmask(J.g, J.fflip, c);
              int pm, np;
              if (fm == 0) {
                pm = (int)(table[cfg] & 0xFFFFFFu);
                np = (int)(table[cfg] >> 24);
              } else {
                np = cube_partitions(cfg, fm, pm);
              }
              J.cpm[x] = (uint32_t)pm;
              J.cnf[x] = (uint32_t)(np | (fm << 4));
              J.npart[x] = (uint32_t)np;
            });
}

template <typename T>
__device__ void jacobi3(T A[3][3], T V[3][3], T ev[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) V[i][k] = (i == k) ? T(1) : T(0);
  const T eps = sizeof(T) == 4 ? T(1e-7) : T(1e-18);
  for (int sweep = 0; sweep < 32; ++sweep) {
    const T off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
    const T diag = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
    if (off == T(0) || off <= eps * diag) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      if (A[p][q] == T(0)) continue;
      const T theta = (A[q][q] - A[p][p]) / (T(2) * A[p][q]);
      const T t = (theta >= T(0) ? T(1) : T(-1)) / (fabs(theta) + sqrt(theta * theta + T(1)));
      const T cs = T(1) / sqrt(t * t + T(1)), sn = t * cs;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T akp = A[k][p], akq = A[k][q];
        A[k][p] = cs * akp - sn * akq;
        A[k][q] = sn * akp + cs * akq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T apk = A[p][k], aqk = A[q][k];
        A[p][k] = cs * apk - sn * aqk;
        A[q][k] = sn * apk + cs * aqk;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T vkp = V[k][p], vkq = V[k][q];
        V[k][p] = cs * vkp - sn * vkq;
        V[k][q] = sn * vkp + cs * vkq;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) ev[i] = A[i][i];
}

// 2D point (cell-local 3D) of the pair on local face (fa, side) that holds
// cell-local edge le.
__device__ __forceinline__ void cell_face_point(const Job& j, const int c[3], int fm, int fa,
                                                int side, int le, double out[3]) {
  const Grid& g = j.g;
  int q[3] = {c[0], c[1], c[2]};
  q[fa] += side;
  const int face = face_index(g, fa, q[0], q[1], q[2]);
  int L[4], pa[2], pb[2];
  face_labels(g, j.labels, fa, q, L);
  const int np = face_pairs(L, (fm >> (2 * fa + side)) & 1, pa, pb);
  // face-local index of the edge
  const int ax = le >> 2;
  int b1, b2;
  other_axes(ax, b1, b2);
  const int off_b1 = le & 1, off_b2 = (le >> 1) & 1;
  int u, v;
  other_axes(fa, u, v);
  const int other = (b1 == fa) ? b2 : b1;
  const int off_other = (b1 == fa) ? off_b2 : off_b1;
  const int fe = (ax == u) ? off_other : 2 + off_other;
  (void)v;
  int slot = 0;
  for (int k = 0; k < np; ++k)
    if (pa[k] == fe || pb[k] == fe) slot = k;
  const double2 pf = j.pf[pair_slot(j, face) + slot];
  out[fa] = (double)side;
  out[u] = pf.x;
  out[v] = pf.y;
  (void)other;
}

// Normal of crossing edge le of cell c (Sec. 5.3): the cross product of the
// directions from its 1D point to the 2D points on the cell's two faces that
// hold it.  The differences are taken in binary64 from the binary64 2D points
// and then rounded to T.  Returns false for a zero cross product.
__device__ __forceinline__ bool edge_plane(const Job& j, const int c[3], int fm, int le,
                                           double pe[3], double n[3]) {
  const int ax = le >> 2;
  int b1, b2;
  other_axes(ax, b1, b2);
  int off[3] = {0, 0, 0};
  off[b1] = le & 1;
  off[b2] = (le >> 1) & 1;
  const int gid = edge_index(j.g, ax, c[0] + off[0], c[1] + off[1], c[2] + off[2]);
  const float t = j.et[edge_slot(j, gid)];
  double ped[3] = {(double)off[0], (double)off[1], (double)off[2]};
  ped[ax] = (double)t;
  double f1[3], f2[3];
  cell_face_point(j, c, fm, b1, off[b1], le, f1);
  cell_face_point(j, c, fm, b2, off[b2], le, f2);
  double d1[3], d2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    pe[k] = ped[k];
    d1[k] = f1[k] - ped[k];
    d2[k] = f2[k] - ped[k];
  }
  n[0] = d1[1] * d2[2] - d1[2] * d2[1];
  n[1] = d1[2] * d2[0] - d1[0] * d2[2];
  n[2] = d1[0] * d2[1] - d1[1] * d2[0];
  const double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  if (!(nl > 0.0)) return false;
#pragma unroll
  for (int k = 0; k < 3; ++k) n[k] /= nl;
  return true;
}

// QEF of one partition (Eq. 2 with normals from 2D points, Sec. 5.3) in
// cell-local coordinates: mass point c of the 1D points, A = sum n n^T,
// b = sum n n.(p_e - c), x = c + A^+_tau b with eigenvalues below
// tau * max dropped.  The planes, A, b and the residual are binary64; T is
// the precision of the eigen-decomposition.  With T = float the solve is
// one pseudo-inverse application plus one refinement step on the binary64
// residual, x += A^+_tau (b - A x): the retained eigenvalues can be as small
// as tau * max, which would amplify the binary32 rounding of the
// decomposition ~1/tau-fold, and the refinement removes that.  The
// refinement cannot repair the kept subspace itself, which a binary32
// decomposition resolves only to ~2^-24 lambda_max / gap (Davis-Kahan; gap =
// smallest kept minus largest dropped eigenvalue): measured errors reach
// 3 * 2^-24 / gap cell widths.  Returns false when T is float and either the
// normal matrix's condition number exceeds fp64_cond (including a singular
// matrix) or, with an eigenvalue dropped, gap < kQefMinGap lambda_max (error
// bound 3.6e-6 cell widths); the caller then redoes the decomposition in
// binary64.
// The gradient-normal ablation's plane at crossing edge le of cell c: the
// 1D point and the normalised logit gradient there (binary64 from the
// binary32 gradient).  Returns false for a zero gradient.
__device__ __forceinline__ bool edge_grad_plane(const Job& j, const int c[3], int le, double pe[3],
                                                double n[3]) {
  const int ax = le >> 2;
  int b1, b2;
  other_axes(ax, b1, b2);
  int off[3] = {0, 0, 0};
  off[b1] = le & 1;
  off[b2] = (le >> 1) & 1;
  const int gid = edge_index(j.g, ax, c[0] + off[0], c[1] + off[1], c[2] + off[2]);
  const int es = edge_slot(j, gid);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    pe[k] = (double)off[k];
    n[k] = (double)j.egrad[3 * es + k];
  }
  pe[ax] = (double)j.et[es];
  const double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  if (!(nl > 0.0)) return false;
#pragma unroll
  for (int k = 0; k < 3; ++k) n[k] /= nl;
  return true;
}

constexpr float kQefMinGap = 0.05f;

template <typename T>
__device__ bool qef_partition(const Job& j, const int c[3], int cfg, int fm, uint32_t pm,
                              int part, double x[3]) {
  // pass 1: mass point of the 1D points
  double cs[3] = {0, 0, 0};
  int cnt = 0;
  for (int le = 0; le < 12; ++le) {
    if (!cube_edge_crosses(cfg, le) || (int)((pm >> (2 * le)) & 3u) != part) continue;
    const int ax = le >> 2;
    int b1, b2;
    other_axes(ax, b1, b2);
    int off[3] = {0, 0, 0};
    off[b1] = le & 1;
    off[b2] = (le >> 1) & 1;
    const int gid = edge_index(j.g, ax, c[0] + off[0], c[1] + off[1], c[2] + off[2]);
    double pe[3] = {(double)off[0], (double)off[1], (double)off[2]};
    pe[ax] = (double)j.et[edge_slot(j, gid)];
#pragma unroll
    for (int k = 0; k < 3; ++k) cs[k] += pe[k];
    ++cnt;
  }
  double cm[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    cm[k] = cs[k] / (double)(cnt > 0 ? cnt : 1);
    x[k] = cm[k];
  }
  // pass 2: planes
  double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, b[3] = {0, 0, 0};
  int used = 0;
  for (int le = 0; le < 12; ++le) {
    if (!cube_edge_crosses(cfg, le) || (int)((pm >> (2 * le)) & 3u) != part) continue;
    double pe[3], n[3];
    if (j.ablation & kAblGradNormals) {
      if (!edge_grad_plane(j, c, le, pe, n)) continue;
    } else if (!edge_plane(j, c, fm, le, pe, n)) {
      continue;
    }
    const double dd = n[0] * (pe[0] - cm[0]) + n[1] * (pe[1] - cm[1]) + n[2] * (pe[2] - cm[2]);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      b[r] += n[r] * dd;
#pragma unroll
      for (int k = 0; k < 3; ++k) A[r][k] += n[r] * n[k];
    }
    ++used;
  }
  if (used == 0) return true;
  T M[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[r][k] = (T)A[r][k];
  T V[3][3], ev[3];
  jacobi3<T>(M, V, ev);
  const T lmax = fmax(ev[0], fmax(ev[1], ev[2]));
  const T lmin = fmin(ev[0], fmin(ev[1], ev[2]));
  if (sizeof(T) == 4 && (lmin <= T(0) || (double)lmax > j.fp64_cond * (double)lmin)) return false;
  const T thr = (T)j.qef_tau * lmax;
  if (sizeof(T) == 4) {
    T kept_min = lmax, dropped_max = T(-1);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (ev[k] >= thr) kept_min = fmin(kept_min, ev[k]);
      else dropped_max = fmax(dropped_max, ev[k]);
    }
    if (dropped_max >= T(0) && kept_min - dropped_max < T(kQefMinGap) * lmax) return false;
  }
  double y[3] = {0, 0, 0};
  for (int pass = 0; pass < 2; ++pass) {
    double r[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) r[q] = b[q] - (A[q][0] * y[0] + A[q][1] * y[1] + A[q][2] * y[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (!(ev[k] >= thr) || ev[k] <= T(0)) continue;
      const double vr = (double)V[0][k] * r[0] + (double)V[1][k] * r[1] + (double)V[2][k] * r[2];
#pragma unroll
      for (int a = 0; a < 3; ++a) y[a] += (double)V[a][k] * vr / (double)ev[k];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] += y[a];
  return true;
}

__global__ __launch_bounds__(256) void k_cell_qef(const Job* __restrict__ jobs, int njobs) {
  for_units(jobs, njobs, gthread(), nthreads(), [](const Job& J) { return n_cells_of(J); },
            [&](const Job& J, int x) {
              const int cid = J.clist[x];
              int c[3];
              cell_of(J.g, cid, c);
              const int cfg = cell_config(J.g, J.labels, c[0], c[1], c[2]);
              const uint32_t pm = J.cpm[x];
              const int np = (int)(J.cnf[x] & 15u), fm = (int)(J.cnf[x] >> 4);
              const int vb = (int)J.vbase[x];
              int fp64 = 0;
              for (int part = 0; part < np; ++part) {
                double xd[3];
                if (!qef_partition<float>(J, c, cfg, fm, pm, part, xd)) {
                  qef_partition<double>(J, c, cfg, fm, pm, part, xd);
                  ++fp64;
                }
                if (J.clamp)
                  for (int a = 0; a < 3; ++a) xd[a] = fmin(fmax(xd[a], 0.0), 1.0);
                const float v[3] = {(float)xd[0], (float)xd[1], (float)xd[2]};
                const int vid = vb + part;
                J.vloc[3 * vid] = v[0];
                J.vloc[3 * vid + 1] = v[1];
                J.vloc[3 * vid + 2] = v[2];
                if (vid < J.cap_v) {
                  const float gp[3] = {(float)c[0] + v[0], (float)c[1] + v[1], (float)c[2] + v[2]};
                  float w[3];
                  grid_world(J.g, gp, w);
                  J.out_v[3 * vid] = w[0];
                  J.out_v[3 * vid + 1] = w[1];
                  J.out_v[3 * vid + 2] = w[2];
                  if (J.out_vloc) {
                    J.out_vloc[3 * vid] = v[0];
                    J.out_vloc[3 * vid + 1] = v[1];
                    J.out_vloc[3 * vid + 2] = v[2];
                  }
                  if (J.out_vref) J.out_vref[vid] = corner_index(J.g, c[0], c[1], c[2]);
                }
              }
              if (fp64) atomicAdd(&J.status[1], (unsigned long long)fp64);
            });
}

// --------------------------------------------------------------- (e) emit
__device__ __forceinline__ float triple3(const float a[3], const float b[3], const float c[3]) {
  const float x = b[1] * c[2] - b[2] * c[1];
  const float y = b[2] * c[0] - b[0] * c[2];
  const float z = b[0] * c[1] - b[1] * c[0];
  return a[0] * x + a[1] * y + a[2] * z;
}

__global__ __launch_bounds__(256) void k_emit_count(const Job* __restrict__ jobs, int njobs) {
  for_units(jobs, njobs, gthread(), nthreads(), [](const Job& J) { return n_edges_of(J); },
            [&](const Job& J, int x) {
              const Grid& g = J.g;
              int a, p[3];
              edge_pos(g, J.elist[x], a, p);
              const int b = (a + 1) % 3, cc = (a + 2) % 3;
              const int OFFB[4] = {0, -1, -1, 0}, OFFC[4] = {0, 0, -1, -1};
              int vid[4];
              float P[4][3];
              for (int q = 0; q < 4; ++q) {
                int c[3] = {p[0], p[1], p[2]};
                c[b] += OFFB[q];
                c[cc] += OFFC[q];
                if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= g.N || c[1] >= g.N || c[2] >= g.N) {
                  J.ecase[x] = 0;
                  J.ntri[x] = 0;
                  J.n3[x] = 0;
                  return;
                }
                const int ci = cell_slot(J, c[0] + g.N * (c[1] + g.N * c[2]));
                int off[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
                const int le = cell_edge(a, off);
                const int part = (int)((J.cpm[ci] >> (2 * le)) & 3u);
                vid[q] = (int)J.vbase[ci] + part;
#pragma unroll
                for (int k = 0; k < 3; ++k) P[q][k] = (float)(c[k] - p[k]) + J.vloc[3 * vid[q] + k];
              }
              const int lower_in = bit_of(J.labels, corner_index(g, p[0], p[1], p[2]));
              // c1..c4 counter-clockwise about +a; reversed when the inside end is the upper one
              const int ord[4] = {0, lower_in ? 1 : 3, 2, lower_in ? 3 : 1};
              float Q[4][3], pin[3] = {0, 0, 0}, pout[3] = {0, 0, 0};
              (lower_in ? pout : pin)[a] = 1.0f;
              int4 qd;
              int* qv = &qd.x;
              for (int q = 0; q < 4; ++q) {
                qv[q] = vid[ord[q]];
#pragma unroll
                for (int k = 0; k < 3; ++k) Q[q][k] = P[ord[q]][k];
              }
              // App. A.1.5: vertex k concave against v_out (Eq. A1) or v_in (Eq. A2)
              int concave[4];
              for (int k = 0; k < 4; ++k) {
                const int kp = (k + 3) & 3, kn = (k + 1) & 3;
                float u0[3], u1[3], u2[3], w0[3], w1[3], w2[3];
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                  u0[t] = Q[k][t] - pout[t];
                  u1[t] = Q[kp][t] - pout[t];
                  u2[t] = Q[kn][t] - pout[t];
                  w0[t] = Q[k][t] - pin[t];
                  w1[t] = Q[kp][t] - pin[t];
                  w2[t] = Q[kn][t] - pin[t];
                }
                concave[k] = (triple3(u0, u1, u2) < 0.0f) || (triple3(w0, w1, w2) > 0.0f);
              }
              int cs = 3;
              if ((J.ablation & kAblMdcSplit) || (!concave[1] && !concave[3])) cs = 1;
              else if (!concave[0] && !concave[2]) cs = 2;
              J.ecase[x] = (uint32_t)cs;
              J.quad[x] = qd;
              J.ntri[x] = cs == 3 ? 4u : 2u;
              J.n3[x] = cs == 3 ? 1u : 0u;
            });
}

__global__ __launch_bounds__(256) void k_emit_write(const Job* __restrict__ jobs, int njobs) {
  for_units(jobs, njobs, gthread(), nthreads(), [](const Job& J) { return n_edges_of(J); },
            [&](const Job& J, int x) {
              const int cs = (int)J.ecase[x];
              if (cs == 0) return;
              const int4 qd = J.quad[x];
              const int t0 = (int)J.tprefix[x];
              int tri[4][3];
              int nt = 2;
              if (cs == 1) {
                tri[0][0] = qd.x; tri[0][1] = qd.y; tri[0][2] = qd.z;
                tri[1][0] = qd.x; tri[1][1] = qd.z; tri[1][2] = qd.w;
              } else if (cs == 2) {
                tri[0][0] = qd.x; tri[0][1] = qd.y; tri[0][2] = qd.w;
                tri[1][0] = qd.y; tri[1][1] = qd.z; tri[1][2] = qd.w;
              } else {
                const int nvp = (int)J.vbase[n_cells_of(J)];
                const int ve = nvp + (int)J.c3prefix[x];
                const int qv[4] = {qd.x, qd.y, qd.z, qd.w};
                for (int k = 0; k < 4; ++k) {
                  tri[k][0] = ve;
                  tri[k][1] = qv[k];
                  tri[k][2] = qv[(k + 1) & 3];
                }
                nt = 4;
                if (ve < J.cap_v) {
                  int a, p[3];
                  edge_pos(J.g, J.elist[x], a, p);
                  const float t = J.et[x];
                  float gp[3] = {(float)p[0], (float)p[1], (float)p[2]};
                  gp[a] = (float)p[a] + t;
                  float w[3];
                  grid_world(J.g, gp, w);
                  J.out_v[3 * ve] = w[0];
                  J.out_v[3 * ve + 1] = w[1];
                  J.out_v[3 * ve + 2] = w[2];
                  if (J.out_vloc) {
                    J.out_vloc[3 * ve] = a == 0 ? t : 0.0f;
                    J.out_vloc[3 * ve + 1] = a == 1 ? t : 0.0f;
                    J.out_vloc[3 * ve + 2] = a == 2 ? t : 0.0f;
                  }
                  if (J.out_vref) J.out_vref[ve] = corner_index(J.g, p[0], p[1], p[2]);
                }
              }
              for (int k = 0; k < nt; ++k) {
                if (t0 + k >= J.cap_t) break;
                J.out_t[3 * (t0 + k)] = tri[k][0];
                J.out_t[3 * (t0 + k) + 1] = tri[k][1];
                J.out_t[3 * (t0 + k) + 2] = tri[k][2];
              }
            });
}

// ------------------------------------------------------------ pipeline
// The whole path for njobs jobs (device array d): one launch per stage and
// no host synchronisation, so a stream capture of it replays as one graph.
hipError_t launch_pipeline(const Job* d, int njobs, const PipelineShape& sh,
                           const float* const* d_weights, const uint32_t* table,
                           const LaunchCfg& cfg, hipEvent_t* ev, hipStream_t s) {
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], s);
  };
  k_clear_status<<<4, kBlock, 0, s>>>(d, njobs);
  if (sh.any_mlp) k_pack<<<cfg.pack_blocks, kBlock, 0, s>>>(d, njobs, d_weights);
  mark(0);
  if (sh.any_coarse) {
    k_coarse_labels<<<cfg.mlp_blocks, kBlock, 0, s>>>(d, njobs);
    k_coarse_mark<<<cfg.grid_blocks, kBlock, 0, s>>>(d, njobs);
    k_fine_plan<<<cfg.grid_blocks, kBlock, 0, s>>>(d, njobs);
  }
  if (sh.any_csg) k_labels_csg<<<cfg.grid_blocks, kBlock, 0, s>>>(d, njobs);
  if (sh.any_mlp_fp32) k_labels_mlp<0, false><<<cfg.mlp_blocks, kBlock, 0, s>>>(d, njobs);
  if (sh.any_mlp_fp32 && sh.any_coarse)
    k_labels_mlp<0, true><<<cfg.mlp_blocks, kBlock, 0, s>>>(d, njobs);
  if (sh.any_mlp_bf16 || sh.any_mlp_x3)
    k_labels_mlp<1, false><<<2 * cfg.mlp_blocks, kBlock, 0, s>>>(d, njobs);
  if ((sh.any_mlp_bf16 || sh.any_mlp_x3) && sh.any_coarse)
    k_labels_mlp<1, true><<<2 * cfg.mlp_blocks, kBlock, 0, s>>>(d, njobs);
  if (sh.any_mlp_bf16 || sh.any_mlp_x3)
    k_relabel_fp32<<<cfg.mlp_blocks, kBlock, 0, s>>>(d, njobs);
  mark(1);
  k_classify_edges<<<cfg.grid_blocks, kBlock, 0, s>>>(d, njobs);
  k_classify_faces<<<cfg.grid_blocks, kBlock, 0, s>>>(d, njobs, table);
  k_classify_cells<<<cfg.grid_blocks, kBlock, 0, s>>>(d, njobs);
  scan<0>(d, njobs, cfg, s);
  scan<1>(d, njobs, cfg, s);
  scan<2>(d, njobs, cfg, s);
  mark(2);
  k_compact<<<cfg.grid_blocks, kBlock, 0, s>>>(d, njobs);
  mark(3);
  if (sh.any_csg) k_bisect_csg<<<cfg.elem_blocks, kBlock, 0, s>>>(d, njobs);
  if (sh.any_mlp_fp32 || sh.any_mlp_bf16) k_bisect_mlp<<<cfg.mlp_blocks, kBlock, 0, s>>>(d, njobs);
  if (sh.any_mlp_x3) k_bisect_x3<<<cfg.mlp_blocks, kBlock, 0, s>>>(d, njobs);
  mark(4);
  if (sh.any_csg) k_search2d_csg<<<cfg.elem_blocks, kBlock, 0, s>>>(d, njobs);
  if (sh.any_mlp_fp32 || sh.any_mlp_bf16)
    k_search2d_mlp<<<cfg.mlp_blocks, kBlock, 0, s>>>(d, njobs);
  if (sh.any_mlp_x3) k_search2d_x3<<<cfg.mlp_blocks, kBlock, 0, s>>>(d, njobs);
  if (sh.any_grad) k_grad_mlp<<<cfg.mlp_blocks, kBlock, 0, s>>>(d, njobs);
  mark(5);
  k_cell_count<<<cfg.elem_blocks, kBlock, 0, s>>>(d, njobs, table);
  scan<3>(d, njobs, cfg, s);
  mark(6);
  k_cell_qef<<<cfg.elem_blocks, kBlock, 0, s>>>(d, njobs);
  mark(7);
  k_emit_count<<<cfg.elem_blocks, kBlock, 0, s>>>(d, njobs);
  scan<4>(d, njobs, cfg, s);
  scan<5>(d, njobs, cfg, s);
  k_emit_write<<<cfg.elem_blocks, kBlock, 0, s>>>(d, njobs);
  mark(8);
  return hipGetLastError();
}

hipError_t launch_gather(const Job* d, int njobs, unsigned long long* out, hipStream_t s) {
  k_gather<<<4, kBlock, 0, s>>>(d, njobs, out);
  return hipGetLastError();
}

// ------------------------------------------------------------ field eval
__global__ __launch_bounds__(256) void k_eval_csg(const float* __restrict__ prims, int np,
                                                  const float* __restrict__ xyz, int n,
                                                  float* __restrict__ z) {
  for (int i = gthread(); i < n; i += nthreads()) {
    const float x[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
    z[i] = csg_inside(prims, np, x) ? 1.0f : -1.0f;
  }
}

__global__ __launch_bounds__(256) void k_eval_fp32(const Job* __restrict__ job,
                                                   const float* __restrict__ xyz, int n,
                                                   float* __restrict__ z) {
  __shared__ __align__(16) float act_lds[kBlock / 64][kActWords];
  float* act = act_lds[threadIdx.x >> 6];
  const Mlp& m = job->mlp;
  const int lane = lane_id();
  for (int t = gwave(); t * 32 < n; t += nwaves()) {
    const int i = t * 32 + (lane & 31);
    const int k = i < n ? i : n - 1;
    const float x[3] = {xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]};
    const float v = mlp_logit_fp32(m, x, act);
    if (i < n && lane < 32) z[i] = v;
  }
}

// the bf16 evaluation of the corner pass (mlp_logit_bf16_pp), 128 points per
// workgroup
__global__ __launch_bounds__(256, 2) void k_eval_bf16(const Job* __restrict__ job,
                                                   const float* __restrict__ xyz, int n,
                                                   float* __restrict__ z) {
  __shared__ __align__(16) char lds[kPPLdsBytes];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const Mlp& m = job->mlp;
  const int lane = lane_id();
  stage_bias_wout(m, lds + kPPBiasOff);
  const PPStream S(m, wave);
  v8bf W[kPPRing][2];
  pp_prime(S, W);
  lds_block_sync();
  for (int t = blockIdx.x; t * 128 < n; t += gridDim.x) {
    const int i = t * 128 + wave * 32 + (lane & 31);
    const int k = i < n ? i : n - 1;
    const float x[3] = {xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]};
    const float v = mlp_logit_bf16_pp(m, x, lds, wave, S, W);
    if (i < n && lane < 32) z[i] = v;
  }
}

__global__ __launch_bounds__(256) void k_eval_x3(const Job* __restrict__ job,
                                                 const float* __restrict__ xyz, int n,
                                                 float* __restrict__ z) {
  __shared__ __align__(16) char lds[kX3LdsBytes];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const Mlp& m = job->mlp;
  const int lane = lane_id();
  x3_stage(m, lds);
  lds_block_sync();
  for (int t = blockIdx.x; t * 128 < n; t += gridDim.x) {
    const int i = t * 128 + wave * 32 + (lane & 31);
    const int k = i < n ? i : n - 1;
    const float x[3] = {xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]};
    const float v = mlp_logit_x3(m, x, lds, wave);
    if (i < n && lane < 32) z[i] = v;
  }
}

hipError_t launch_eval(const Job* d_job, const Job& h_job, const float* const* d_weights,
                       int precision, const float* xyz, int n, float* z, const LaunchCfg& cfg,
                       hipStream_t s) {
  if (h_job.kind == 0) {
    k_eval_csg<<<cfg.elem_blocks, kBlock, 0, s>>>(h_job.prims, h_job.n_prims, xyz, n, z);
  } else {
    k_pack<<<cfg.pack_blocks, kBlock, 0, s>>>(d_job, 1, d_weights);
    if (precision == 0) k_eval_fp32<<<cfg.mlp_blocks, kBlock, 0, s>>>(d_job, xyz, n, z);
    else if (precision == 1) k_eval_bf16<<<2 * cfg.mlp_blocks, kBlock, 0, s>>>(d_job, xyz, n, z);
    else k_eval_x3<<<cfg.mlp_blocks, kBlock, 0, s>>>(d_job, xyz, n, z);
  }
  return hipGetLastError();
}

// R6 partition table: partmap | npart << 24 for each cube configuration
__global__ void k_partition_table(uint32_t* table) {
  const int cfg = threadIdx.x;
  if (cfg >= 256) return;
  int pm;
  const int np = cube_partitions(cfg, 0, pm);
  table[cfg] = (uint32_t)pm | ((uint32_t)np << 24);
}

hipError_t launch_partition_table(uint32_t* table, hipStream_t s) {
  k_partition_table<<<1, 256, 0, s>>>(table);
  return hipGetLastError();
}

}  // namespace odc
