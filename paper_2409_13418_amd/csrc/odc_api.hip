// C ABI of libodc.so (include/odc.h): contexts, per-job scratch, batches,
// graph replay, the autotuner and the stage timers.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include <atomic>
#include <mutex>

#include "odc_context.h"

using namespace odc;

namespace {

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Scratch of odc_mesh_extract_noalloc: one fixed array per GPU, alive until
// the process ends.  Host code never uses its name as an address: each
// device's copy is resolved once (fixed_scratch_of) and that pointer is what
// kernels and copies get.
constexpr size_t kFixedScratchBytes = size_t(192) << 20;
static __device__ __align__(256) char scratch[kFixedScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void* g_fixed_ptr[kMaxDevices] = {};

// Failure injection for tests of the error paths (odc_inject_alloc_failures):
// the number of device allocations still allowed, or -1 for no limit.
std::atomic<long long> g_alloc_allowed{-1};

}  // namespace

hipError_t odc::device_alloc(void** p, size_t bytes) {
  long long left = g_alloc_allowed.load();
  while (left >= 0) {
    if (left == 0) {
      *p = nullptr;
      return hipErrorOutOfMemory;
    }
    if (g_alloc_allowed.compare_exchange_weak(left, left - 1)) break;
  }
  return hipMalloc(p, bytes);
}

extern "C" int32_t odc_inject_alloc_failures(int32_t after) {
  g_alloc_allowed.store(after < 0 ? -1 : after);
  return ODC_OK;
}

int32_t odc::ctx_fail(odc_context* ctx, int32_t code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}
#define fail odc::ctx_fail

#define HIP_TRY(ctx, expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(ctx, ODC_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                              \
  } while (0)

#define TRY(expr)                \
  do {                           \
    int32_t r_ = (expr);         \
    if (r_ != ODC_OK) return r_; \
  } while (0)

static void drop_graph(odc_context* ctx) {
  if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
  ctx->graph = nullptr;
  ctx->graph_njobs = -1;
}

static int32_t ensure(odc_context* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return ODC_OK;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  drop_graph(ctx);  // a captured graph may reference the old allocation
  if (b.p) HIP_TRY(ctx, hipFree(b.p));
  b.p = nullptr;
  b.bytes = 0;
  const size_t want = bytes + bytes / 4;
  if (device_alloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(ctx, ODC_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed", want);
  }
  b.bytes = want;
  return ODC_OK;
}

template <class T>
static T* P(DevBuf& b) {
  return reinterpret_cast<T*>(b.p);
}

extern "C" const char* odc_status_string(int32_t s) {
  switch (s) {
    case ODC_OK: return "ok";
    case ODC_ERR_INVALID_ARG: return "invalid argument";
    case ODC_ERR_OUT_OF_MEMORY: return "out of device memory";
    case ODC_ERR_CAPACITY: return "output capacity exceeded";
    case ODC_ERR_HIP: return "HIP runtime error";
    case ODC_ERR_UNSUPPORTED: return "unsupported field";
    case ODC_ERR_BUSY: return "busy";
    default: return "unknown status";
  }
}

extern "C" const char* odc_last_error(const odc_context* ctx) {
  return ctx ? ctx->err.c_str() : "no context";
}

extern "C" void odc_params_default(odc_params* p, int32_t res) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->lo[0] = p->lo[1] = p->lo[2] = -0.5;
  p->size = 1.0;
  p->res = res;
  p->iters_1d = 15;
  p->lin1 = 4;
  p->bin1 = 11;
  p->lin2 = 3;
  p->bin2 = 12;
  p->range1 = 0.8f;
  p->range2 = (float)(sqrt(2.0) / 2.0);
  p->qef_tau = 1e-2f;
  p->fp64_cond = 1e6;
  p->precision = ODC_PREC_FP32;
  p->guard_logit = (float)(2.0 * atanh(0.02));
}

// The device address of this device's fixed scratch array, looked up once
// per device (with that device current) and kept.
static int32_t fixed_scratch_of(odc_context* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return fail(ctx, ODC_ERR_UNSUPPORTED, "device index %d above %d", ctx->device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_fixed_mu);
  if (!g_fixed_ptr[ctx->device]) {
    void* ptr = nullptr;
    HIP_TRY(ctx, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(ctx, ODC_ERR_HIP, "fixed scratch array has no device address");
    g_fixed_ptr[ctx->device] = ptr;
  }
  ctx->fixed_scratch = g_fixed_ptr[ctx->device];
  return ODC_OK;
}

extern "C" int32_t odc_context_create(int32_t device, void* stream, odc_context** out) {
  if (!out) return ODC_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return ODC_ERR_INVALID_ARG;
  }
  odc_context* ctx = new odc_context();
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return ODC_ERR_HIP;
  }
  int32_t rc = ODC_OK;
  if (stream) {
    ctx->stream = (hipStream_t)stream;
  } else if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) == hipSuccess) {
    ctx->own_stream = true;
  } else {
    rc = ODC_ERR_HIP;
  }
  if (rc == ODC_OK && hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) !=
                          hipSuccess)
    rc = ODC_ERR_HIP;
  if (rc == ODC_OK &&
      (hipHostMalloc((void**)&ctx->hjobs, kMaxJobs * sizeof(Job), hipHostMallocDefault) !=
           hipSuccess ||
       hipHostMalloc((void**)&ctx->hweights, kMaxJobs * sizeof(float*), hipHostMallocDefault) !=
           hipSuccess ||
       hipHostMalloc((void**)&ctx->hgather, kMaxJobs * kGatherWords * sizeof(unsigned long long),
                     hipHostMallocDefault) != hipSuccess))
    rc = ODC_ERR_OUT_OF_MEMORY;
  if (rc == ODC_OK) rc = ensure(ctx, ctx->table, 256 * sizeof(uint32_t));
  if (rc == ODC_OK) rc = ensure(ctx, ctx->djobs, kMaxJobs * sizeof(Job));
  if (rc == ODC_OK) rc = ensure(ctx, ctx->dweights, kMaxJobs * sizeof(float*));
  if (rc == ODC_OK) rc = ensure(ctx, ctx->dgather, kMaxJobs * kGatherWords * sizeof(unsigned long long));
  if (rc == ODC_OK && launch_partition_table(P<uint32_t>(ctx->table), ctx->stream) != hipSuccess)
    rc = ODC_ERR_HIP;
  // only odc_mesh_extract_noalloc needs the fixed array: a failed lookup is
  // kept as its error instead of failing the context
  if (rc == ODC_OK && fixed_scratch_of(ctx) != ODC_OK) {
    ctx->fixed_err = ctx->err;
    (void)hipGetLastError();
  }
  if (rc == ODC_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) rc = ODC_ERR_HIP;
  if (rc != ODC_OK) {
    odc_context_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return ODC_OK;
}

static void free_buf(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

extern "C" void odc_context_destroy(odc_context* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  drop_graph(ctx);
  for (Slot& s : ctx->slots) {
    free_buf(s.grid);
    free_buf(s.active);
    free_buf(s.mlpw);
    free_buf(s.guard);
    free_buf(s.status);
  }
  free_buf(ctx->djobs);
  free_buf(ctx->dweights);
  free_buf(ctx->dgather);
  free_buf(ctx->table);
  if (ctx->hjobs) (void)hipHostFree(ctx->hjobs);
  if (ctx->hweights) (void)hipHostFree(ctx->hweights);
  if (ctx->hgather) (void)hipHostFree(ctx->hgather);
  for (hipEvent_t& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

int32_t odc::validate_job(odc_context* ctx, const odc_field* f, const odc_params* p,
                          const odc_mesh_buffers* o) {
  if (!f || !p || !o) return fail(ctx, ODC_ERR_INVALID_ARG, "NULL field, params or buffers");
  if (p->res < 1 || p->res > kMaxRes)
    return fail(ctx, ODC_ERR_INVALID_ARG, "res %d outside 1..%d", p->res, kMaxRes);
  if (!(p->size > 0.0) || !isfinite(p->size) || !isfinite(p->lo[0]) || !isfinite(p->lo[1]) ||
      !isfinite(p->lo[2]))
    return fail(ctx, ODC_ERR_INVALID_ARG, "domain must be finite with size > 0");
  if (p->iters_1d < 1 || p->iters_1d > 23)
    return fail(ctx, ODC_ERR_INVALID_ARG, "iters_1d %d outside 1..23", p->iters_1d);
  if (p->lin1 < 1 || p->lin2 < 1 || p->bin1 < 0 || p->bin2 < 0 || p->lin1 > 64 ||
      p->lin2 > 64 || p->bin1 > 30 || p->bin2 > 30)
    return fail(ctx, ODC_ERR_INVALID_ARG, "line-binary sample/halving counts out of range");
  if (!(p->range1 > 0.0f) || !(p->range2 > 0.0f))
    return fail(ctx, ODC_ERR_INVALID_ARG, "search ranges must be positive");
  if (!(p->qef_tau >= 0.0f) || !(p->qef_tau < 1.0f))
    return fail(ctx, ODC_ERR_INVALID_ARG, "qef_tau outside [0,1)");
  if (p->precision != ODC_PREC_FP32 && p->precision != ODC_PREC_BF16_GUARDED &&
      p->precision != ODC_PREC_BF16_X3)
    return fail(ctx, ODC_ERR_INVALID_ARG, "unknown precision %d", p->precision);
  if (p->precision == ODC_PREC_BF16_X3 && p->ablation)
    return fail(ctx, ODC_ERR_UNSUPPORTED,
                "the ablation baselines run on the fp32 and bf16-guarded precisions");
  if (!(p->guard_logit > 0.0f) || !isfinite(p->guard_logit))
    return fail(ctx, ODC_ERR_INVALID_ARG, "guard_logit must be finite and positive");
  if (!(p->fp64_cond > 0.0) || isnan(p->fp64_cond))
    return fail(ctx, ODC_ERR_INVALID_ARG, "fp64_cond must be positive");
  if (p->ablation &
      ~(ODC_ABL_LINEAR_1D | ODC_ABL_GRAD_NORMALS | ODC_ABL_MDC_SPLIT | ODC_ABL_SDF_INPUT))
    return fail(ctx, ODC_ERR_INVALID_ARG, "unknown ablation bits 0x%x", p->ablation);
  if ((p->ablation & ODC_ABL_SDF_INPUT) && !(p->ablation & ODC_ABL_LINEAR_1D))
    return fail(ctx, ODC_ERR_INVALID_ARG, "SDF input applies to linear 1D points only");
  if (p->clamp_vertices != 0 && p->clamp_vertices != 1)
    return fail(ctx, ODC_ERR_INVALID_ARG, "clamp_vertices must be 0 or 1");
  if (p->coarse_step < 0 || p->coarse_step > 64 ||
      (p->coarse_step > 1 && p->res % p->coarse_step != 0))
    return fail(ctx, ODC_ERR_INVALID_ARG,
                "coarse_step must be 0, 1, or 2..64 dividing res (%d, res %d)", p->coarse_step,
                p->res);
  if (!(p->coarse_band >= 0.0f) || !isfinite(p->coarse_band))
    return fail(ctx, ODC_ERR_INVALID_ARG, "coarse_band must be finite and >= 0");
  if ((p->ablation & ODC_ABL_GRAD_NORMALS) && f->kind != ODC_FIELD_MLP)
    return fail(ctx, ODC_ERR_UNSUPPORTED, "gradient normals need an MLP field");
  if ((o->cap_vertices > 0 && !o->vertices) || (o->cap_triangles > 0 && !o->triangles) ||
      o->cap_vertices < 0 || o->cap_triangles < 0)
    return fail(ctx, ODC_ERR_INVALID_ARG, "NULL output buffer with non-zero capacity");
  if (f->kind == ODC_FIELD_CSG) {
    if (!f->prims || f->n_prims < 1)
      return fail(ctx, ODC_ERR_INVALID_ARG, "CSG field needs at least one primitive");
  } else if (f->kind == ODC_FIELD_MLP) {
    if (!f->weights || !f->spheres || f->n_spheres < 1)
      return fail(ctx, ODC_ERR_INVALID_ARG, "MLP field needs weights and sdf spheres");
    if (f->width != kWidth || f->depth < 1 || f->depth > kMaxDepth || f->n_bands < 0 ||
        f->in_dim != 3 + 6 * f->n_bands || f->in_dim > kMaxInDim)
      return fail(ctx, ODC_ERR_UNSUPPORTED,
                  "MLP kernels need width 256, depth 1..8 and in_dim = 3 + 6 n_bands <= 45");
  } else {
    return fail(ctx, ODC_ERR_INVALID_ARG, "unknown field kind %d", f->kind);
  }
  return ODC_OK;
}

// Active-set capacity for a grid of N cells per axis: crossing edges of a
// surface scale with its area; 12 N^2 leaves a third of headroom over the
// benchmark fields (5.5 N^2 for the MLP field, 7.3 N^2 for the CSG field),
// and an overflow grows the scale for the rest of the context's life.
int odc::estimate_edges(double cap_scale, int N) {
  const double e = (12.0 * N * N + 4096.0) * cap_scale;
  const double total = 3.0 * N * (double)(N + 1) * (N + 1);
  return (int)(e < total ? e : total) + 64;
}

namespace {

// Scalar fields of a job: grid, field, parameters, bit-set sizes and
// active-set capacities for ce crossing edges.
void job_scalars(Job& J, const odc_field* f, const odc_params* p, int ce) {
  memset(&J, 0, sizeof(J));
  const int N = p->res;
  J.g.N = N;
  for (int a = 0; a < 3; ++a) J.g.lo[a] = (float)p->lo[a];
  J.g.h = (float)(p->size / (double)N);
  J.g.nc = (N + 1) * (N + 1) * (N + 1);
  J.g.ea = N * (N + 1) * (N + 1);
  J.g.fa = (N + 1) * N * N;
  J.g.ncell = N * N * N;
  J.kind = f->kind;
  J.precision = f->kind == ODC_FIELD_MLP ? p->precision : 0;
  J.prims = f->prims;
  J.n_prims = f->n_prims;
  J.iters_1d = p->iters_1d;
  J.lin1 = p->lin1;
  J.bin1 = p->bin1;
  J.lin2 = p->lin2;
  J.bin2 = p->bin2;
  J.range1 = p->range1;
  J.range2 = p->range2;
  J.qef_tau = p->qef_tau;
  J.guard_logit = p->guard_logit;
  J.fp64_cond = p->fp64_cond;
  J.ablation = p->ablation;
  J.clamp = p->clamp_vertices;
  J.coarse_step = p->coarse_step > 1 ? p->coarse_step : 0;
  J.cn = J.coarse_step ? N / J.coarse_step : 0;
  // CSG: the band is a distance, the coarse cell's diagonal (the condition
  // under which marking by the distance bound is exact), with a margin
  J.coarse_band = f->kind == ODC_FIELD_CSG
                      ? (float)(sqrt(3.0) * J.coarse_step * (p->size / N) * 1.001 + 1e-6)
                      : p->coarse_band;
  J.nw_c = (J.g.nc + 31) / 32;
  J.nw_e = (3 * J.g.ea + 31) / 32;
  J.nw_f = (3 * J.g.fa + 31) / 32;
  J.nw_cell = (J.g.ncell + 31) / 32;
  J.cap_edges = ce;
  J.cap_pairs = 2 * ce + 64;
  J.cap_cells = ce + ce / 2 + 64;
}

// Byte sizes of a job's scratch regions (each a multiple of 256).
struct Layout {
  size_t grid[17];
  size_t active[19];
  size_t grid_total = 0, active_total = 0;
  size_t mlpw = 0, guard = 0, status = 0;
  int guard_cap = 0;
  size_t n_w1f = 0, n_whf = 0, n_w1b = 0, n_whb = 0;
  size_t total() const { return grid_total + active_total + mlpw + guard + status; }
};

Layout job_layout(const Job& J, const odc_field* f, bool guard_full, bool trace) {
  Layout L;
  int nscan = J.nw_e;
  const int others[4] = {J.nw_f, J.nw_cell, J.cap_edges + 1, J.cap_cells + 1};
  for (int v : others) nscan = v > nscan ? v : nscan;
  L.grid[0] = align_up((size_t)J.nw_c * 4);                 // labels
  L.grid[1] = L.grid[2] = align_up((size_t)J.nw_e * 4);     // emask, ecount
  L.grid[3] = align_up((size_t)(J.nw_e + 1) * 4);           // eprefix
  L.grid[4] = L.grid[5] = L.grid[6] = L.grid[7] = align_up((size_t)J.nw_f * 4);
  L.grid[8] = align_up((size_t)(J.nw_f + 1) * 4);
  L.grid[9] = L.grid[10] = align_up((size_t)J.nw_cell * 4);
  L.grid[11] = align_up((size_t)(J.nw_cell + 1) * 4);
  L.grid[12] = align_up((size_t)((nscan + 1023) / 1024 + 2) * 4);
  // adaptive corner evaluation: coarse corner labels and band bits, marked coarse cells
  const size_t c1 = J.coarse_step ? (size_t)J.cn + 1 : 0;
  L.grid[13] = L.grid[14] = align_up((c1 * c1 * c1 + 31) / 32 * 4);
  L.grid[15] = J.coarse_step ? align_up(((size_t)J.cn * J.cn * J.cn + 63) / 64 * 8) : 0;
  L.grid[16] = J.coarse_step ? align_up((size_t)J.nw_c * 4) : 0;  // listed fine words
  for (size_t x : L.grid) L.grid_total += x;
  const size_t ne = (size_t)J.cap_edges, np = (size_t)J.cap_pairs, nc = (size_t)J.cap_cells;
  const size_t asz[16] = {align_up(ne * 4),          align_up(ne * 4),
                          align_up(ne * 4),          align_up(ne * 4),
                          align_up(ne * 4),          align_up((ne + 1) * 4),
                          align_up((ne + 1) * 4),    align_up(ne * sizeof(int4)),
                          align_up(np * 4),          align_up(np * sizeof(double2)),
                          align_up(nc * 4),          align_up(nc * 4),
                          align_up(nc * 4),          align_up(nc * 4),
                          align_up((nc + 1) * 4),    align_up(nc * 12 * sizeof(float))};
  for (int i = 0; i < 16; ++i) {
    L.active[i] = asz[i];
    L.active_total += asz[i];
  }
  L.active[16] = (J.ablation & kAblGradNormals) ? align_up(ne * 3 * sizeof(float)) : 0;
  L.active[17] = trace ? align_up(ne * 4) : 0;
  L.active[18] = trace ? align_up(np * 16) : 0;
  L.active_total += L.active[16] + L.active[17] + L.active[18];
  L.status = align_up(9 * sizeof(unsigned long long));
  if (f->kind == ODC_FIELD_MLP) {
    const int kb1f = kb1_fp32(f->in_dim), kb1b = kb1_bf16(f->in_dim), d = f->depth;
    L.n_w1f = (size_t)kb1f * 512;
    L.n_whf = ((size_t)(d - 1) * kHiddenBlocksF32 + kPrefetchF32) * 512;  // + ring overrun
    L.n_w1b = (size_t)kb1b * 512;
    L.n_whb = ((size_t)(d - 1) * kHiddenBlocksBF16 + kPrefetchBF16) * 512;  // + ring overrun
    // the split-bf16 precision adds the second and third bf16 weight terms
    const size_t x3 = J.precision == ODC_PREC_BF16_X3 ? 2 * (L.n_w1b + L.n_whb) * 16 : 0;
    L.mlpw = align_up((L.n_w1f + L.n_whf) * 4 + (L.n_w1b + L.n_whb) * 16 +
                      (size_t)(d + 1) * kWidth * 4 + x3);
    if (J.precision == ODC_PREC_BF16_GUARDED || J.precision == ODC_PREC_BF16_X3) {
      // corners in the guard band are ~1% of a grid; the queue holds 1/16 of
      // the corners unless an earlier run of this job overflowed it
      L.guard_cap = guard_full ? J.g.nc : (J.g.nc / 16 > 4096 ? J.g.nc / 16 : J.g.nc);
      L.guard = align_up((size_t)L.guard_cap * 4);
    }
  }
  return L;
}

// Points the job's arrays into its scratch regions.
void job_bind(Job& J, const Layout& L, const odc_field* f, char* grid, char* active, char* mlpw,
              char* guard, char* status) {
  uint32_t** gp[17] = {&J.labels, &J.emask,  &J.ecount,   &J.eprefix, &J.fact,  &J.famb,
                       &J.fflip,  &J.pcount, &J.pprefix,  &J.cmask,   &J.ccount, &J.cprefix,
                       &J.scan_tmp, &J.cbits, &J.cnear,   &J.cmark,
                       reinterpret_cast<uint32_t**>(&J.wlist)};
  size_t off = 0;
  for (int i = 0; i < 17; ++i) {
    *gp[i] = (uint32_t*)(grid + off);
    off += L.grid[i];
  }
  if (!J.coarse_step) {
    J.cbits = J.cnear = J.cmark = nullptr;
    J.wlist = nullptr;
  }
  void** ap[19] = {(void**)&J.elist,    (void**)&J.et,    (void**)&J.ecase, (void**)&J.ntri,
                   (void**)&J.n3,       (void**)&J.tprefix, (void**)&J.c3prefix,
                   (void**)&J.quad,     (void**)&J.plist, (void**)&J.pf,    (void**)&J.clist,
                   (void**)&J.cpm,      (void**)&J.cnf,   (void**)&J.npart, (void**)&J.vbase,
                   (void**)&J.vloc,     (void**)&J.egrad, (void**)&J.etrace,
                   (void**)&J.ptrace};
  off = 0;
  for (int i = 0; i < 19; ++i) {
    *ap[i] = active + off;
    off += L.active[i];
  }
  if (!(J.ablation & kAblGradNormals)) J.egrad = nullptr;
  if (!L.active[17]) J.etrace = nullptr;
  if (!L.active[18]) J.ptrace = nullptr;
  J.status = (unsigned long long*)status;
  if (f->kind == ODC_FIELD_MLP) {
    const int d = f->depth;
    float* w1f = (float*)mlpw;
    float* whf = w1f + L.n_w1f;
    v8bf* w1b = (v8bf*)(whf + L.n_whf);
    v8bf* whb = w1b + L.n_w1b;
    float* bias = (float*)(whb + L.n_whb);
    Mlp& m = J.mlp;
    m.w1f = w1f;
    m.whf = whf;
    m.w1b = w1b;
    m.whb = whb;
    m.bias = bias;
    m.wout = bias + (size_t)d * kWidth;
    m.spheres = f->spheres;
    m.bout = f->weights + (size_t)kWidth * f->in_dim + kWidth +
             (size_t)(d - 1) * (kWidth * kWidth + kWidth) + kWidth;
    m.sdf_gain = f->sdf_gain;
    m.out_scale = f->out_scale;
    m.n_spheres = f->n_spheres;
    m.depth = d;
    m.in_dim = f->in_dim;
    m.kb1f = kb1_fp32(f->in_dim);
    m.kb1b = kb1_bf16(f->in_dim);
    m.wx1 = m.wx2 = nullptr;
    if (J.precision == ODC_PREC_BF16_X3) {
      v8bf* x1 = (v8bf*)(bias + (size_t)(d + 1) * kWidth);
      m.wx1 = x1;
      m.wx2 = x1 + L.n_w1b + L.n_whb;
    }
    if (J.precision == ODC_PREC_BF16_GUARDED || J.precision == ODC_PREC_BF16_X3) {
      J.guard_list = (uint32_t*)guard;
      J.guard_cap = L.guard_cap;
    }
  }
}

}  // namespace

size_t odc::job_scratch_bytes(const odc_field* f, const odc_params* p, int cap_edges,
                              bool guard_full) {
  Job J;
  job_scalars(J, f, p, cap_edges);
  return job_layout(J, f, guard_full, false).total();
}

// Fills job k (host mirror) and points it into its slot's scratch: the
// context's own growing buffers, or the slot's block of a server arena.
static int32_t setup_job(odc_context* ctx, int k, const odc_field* f, const odc_params* p,
                         const odc_mesh_buffers* o, int cap_edges_min) {
  Slot& S = ctx->slots[k];
  Job& J = ctx->hjobs[k];
  const int N = p->res;
  int ce;
  if (S.ext) {
    ce = S.ext_cap_edges;
  } else {
    ce = estimate_edges(ctx->cap_scale, N);
    if (ce < cap_edges_min) ce = cap_edges_min;
    const int all = 3 * N * (N + 1) * (N + 1) + 64;
    if (ce < S.cap_edges && S.cap_edges <= all) ce = S.cap_edges;
    S.cap_edges = ce;
  }
  job_scalars(J, f, p, ce);
  const Layout L = job_layout(J, f, S.guard_full, ctx->trace && !S.ext);
  if (S.ext) {
    if (L.total() > S.ext_bytes)
      return fail(ctx, ODC_ERR_OUT_OF_MEMORY, "job needs %zu bytes of scratch, block has %zu",
                  L.total(), S.ext_bytes);
    char* b = S.ext;
    job_bind(J, L, f, b, b + L.grid_total, b + L.grid_total + L.active_total,
             b + L.grid_total + L.active_total + L.mlpw,
             b + L.grid_total + L.active_total + L.mlpw + L.guard);
  } else {
    TRY(ensure(ctx, S.grid, L.grid_total));
    TRY(ensure(ctx, S.active, L.active_total));
    TRY(ensure(ctx, S.status, L.status));
    if (L.mlpw) TRY(ensure(ctx, S.mlpw, L.mlpw));
    if (L.guard) TRY(ensure(ctx, S.guard, L.guard));
    job_bind(J, L, f, P<char>(S.grid), P<char>(S.active), P<char>(S.mlpw), P<char>(S.guard),
             P<char>(S.status));
  }
  ctx->hweights[k] = f->kind == ODC_FIELD_MLP ? f->weights : nullptr;
  if (o) {
    J.out_v = o->vertices;
    J.cap_v = o->cap_vertices;
    J.out_t = o->triangles;
    J.cap_t = o->cap_triangles;
    J.out_vloc = o->vertices_local;
    J.out_vref = o->vertex_ref;
  }
  return ODC_OK;
}

static PipelineShape shape_of(odc_context* ctx, int n) {
  PipelineShape sh;
  for (int k = 0; k < n; ++k) {
    const Job& J = ctx->hjobs[k];
    if (J.kind == 0) sh.any_csg = true;
    if (J.coarse_step) sh.any_coarse = true;
    if (J.kind == 1) {
      sh.any_mlp = true;
      if (J.precision == 0) sh.any_mlp_fp32 = true;
      else if (J.precision == 1) sh.any_mlp_bf16 = true;
      else sh.any_mlp_x3 = true;
      if (J.ablation & kAblGradNormals) sh.any_grad = true;
    }
  }
  return sh;
}

static bool same_shape(const PipelineShape& a, const PipelineShape& b) {
  return a.any_csg == b.any_csg && a.any_mlp == b.any_mlp && a.any_mlp_fp32 == b.any_mlp_fp32 &&
         a.any_mlp_bf16 == b.any_mlp_bf16 && a.any_mlp_x3 == b.any_mlp_x3 &&
         a.any_grad == b.any_grad && a.any_coarse == b.any_coarse;
}
static bool same_cfg(const LaunchCfg& a, const LaunchCfg& b) {
  return a.grid_blocks == b.grid_blocks && a.elem_blocks == b.elem_blocks &&
         a.mlp_blocks == b.mlp_blocks && a.scan_blocks == b.scan_blocks &&
         a.pack_blocks == b.pack_blocks;
}

// The launch shape for the n jobs in ctx->hjobs: the autotuned entry of the
// dominant job's (field kind, resolution bucket) when there is one, else the
// context's.  The dominant job is the largest MLP job if any (its matrix
// stages dominate), else the largest job.
static const LaunchCfg& cfg_for(const odc_context* ctx, int n) {
  if (ctx->tuning || n <= 0) return ctx->cfg;
  int best = 0;
  for (int k = 1; k < n; ++k) {
    const Job& a = ctx->hjobs[k];
    const Job& b = ctx->hjobs[best];
    if (a.kind > b.kind || (a.kind == b.kind && a.g.N > b.g.N)) best = k;
  }
  const Job& J = ctx->hjobs[best];
  const int kind = J.kind == 1 ? 1 : 0, rb = res_bucket(J.g.N);
  return ctx->tuned_ok[kind][rb] ? ctx->tuned[kind][rb] : ctx->cfg;
}

// Uploads the job array and launches the whole path for n jobs: directly, or
// by replaying a captured graph (the kernels read everything from the job
// array, so one graph serves every batch of the same size and kinds).
static int32_t run_batch(odc_context* ctx, int n) {
  hipStream_t s = ctx->stream;
  const Job* d = P<Job>(ctx->djobs);
  const float* const* dw = P<const float*>(ctx->dweights);
  HIP_TRY(ctx, hipMemcpyAsync(P<Job>(ctx->djobs), ctx->hjobs, n * sizeof(Job),
                              hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(P<const float*>(ctx->dweights), ctx->hweights,
                              n * sizeof(float*), hipMemcpyHostToDevice, s));
  const PipelineShape sh = shape_of(ctx, n);
  const LaunchCfg& cfg = cfg_for(ctx, n);
  if (ctx->use_graph && !ctx->timing) {
    const void* ptrs[3] = {ctx->djobs.p, ctx->dweights.p, ctx->table.p};
    const bool reuse = ctx->graph && ctx->graph_njobs == n && same_shape(ctx->graph_shape, sh) &&
                       same_cfg(ctx->graph_cfg, cfg) && ptrs[0] == ctx->graph_ptrs[0] &&
                       ptrs[1] == ctx->graph_ptrs[1] && ptrs[2] == ctx->graph_ptrs[2];
    if (!reuse) {
      drop_graph(ctx);
      hipGraph_t g = nullptr;
      HIP_TRY(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
      hipError_t le = launch_pipeline(d, n, sh, dw, P<uint32_t>(ctx->table), cfg, nullptr,
                                      ctx->capture_stream);
      hipError_t ce = hipStreamEndCapture(ctx->capture_stream, &g);
      if (le != hipSuccess || ce != hipSuccess)
        return fail(ctx, ODC_ERR_HIP, "graph capture failed: %s / %s", hipGetErrorString(le),
                    hipGetErrorString(ce));
      hipError_t ie = hipGraphInstantiate(&ctx->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        ctx->graph = nullptr;
        return fail(ctx, ODC_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
      }
      ctx->graph_njobs = n;
      ctx->graph_shape = sh;
      ctx->graph_cfg = cfg;
      for (int i = 0; i < 3; ++i) ctx->graph_ptrs[i] = ptrs[i];
    }
    HIP_TRY(ctx, hipGraphLaunch(ctx->graph, s));
  } else {
    HIP_TRY(ctx, launch_pipeline(d, n, sh, dw, P<uint32_t>(ctx->table), cfg,
                                 ctx->timing ? ctx->ev : nullptr, s));
  }
  HIP_TRY(ctx, launch_gather(d, n, P<unsigned long long>(ctx->dgather), s));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->hgather, P<unsigned long long>(ctx->dgather),
                              n * kGatherWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  return ODC_OK;
}

int32_t odc::enqueue_batch(odc_context* ctx, int n, const odc_field* fields,
                           const odc_params* params, const odc_mesh_buffers* outs) {
  if (!ctx) return ODC_ERR_INVALID_ARG;
  if (n < 1 || n > kMaxJobs) return fail(ctx, ODC_ERR_INVALID_ARG, "batch size %d", n);
  if (!fields || !params || !outs) return fail(ctx, ODC_ERR_INVALID_ARG, "NULL arrays");
  for (int k = 0; k < n; ++k) TRY(validate_job(ctx, &fields[k], &params[k], &outs[k]));
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  // the host mirrors are reused: wait for the previous batch's uploads
  if (ctx->pending) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if ((int)ctx->slots.size() < n) ctx->slots.resize(n);
  // the host job mirrors are rewritten from here on: a failure abandons the
  // previous batch too (nothing of it is pending any more)
  ctx->pending = 0;
  for (int k = 0; k < n; ++k) TRY(setup_job(ctx, k, &fields[k], &params[k], &outs[k], 0));
  TRY(run_batch(ctx, n));
  ctx->pending = n;
  ctx->pending_fixed = false;
  ctx->p_fields.assign(fields, fields + n);
  ctx->p_params.assign(params, params + n);
  ctx->p_outs.assign(outs, outs + n);
  return ODC_OK;
}

extern "C" int32_t odc_mesh_extract(odc_context* ctx, const odc_field* field,
                                    const odc_params* params, const odc_mesh_buffers* out) {
  return enqueue_batch(ctx, 1, field, params, out);
}

// The job record and scratch layout of the allocation-free variant: the
// planned crossing-edge capacity, cut to what the fixed array holds; fails
// (OUT_OF_MEMORY) when even 4096 crossing edges do not fit.  Host only.
static int32_t plan_fixed(odc_context* ctx, const odc_field* f, const odc_params* p,
                          double cap_scale, Job& J, Layout& L) {
  const int N = p->res;
  int ce = estimate_edges(cap_scale, N);
  job_scalars(J, f, p, ce);
  L = job_layout(J, f, false, false);
  if (L.total() <= kFixedScratchBytes) return ODC_OK;
  job_scalars(J, f, p, 64);
  const Layout L0 = job_layout(J, f, false, false);
  job_scalars(J, f, p, 65536 + 64);
  const Layout L1 = job_layout(J, f, false, false);
  const double per_edge = (double)(L1.total() - L0.total()) / 65536.0;
  const double room = (double)kFixedScratchBytes - (double)L0.total();
  ce = room > per_edge * 4096 ? 64 + (int)(room / per_edge) - 256 : 0;
  if (ce < 4096)
    return fail(ctx, ODC_ERR_OUT_OF_MEMORY,
                "res %d needs %zu bytes of scratch beyond the active sets; the fixed array "
                "holds %zu",
                N, L0.total(), kFixedScratchBytes);
  job_scalars(J, f, p, ce);
  L = job_layout(J, f, false, false);
  while (L.total() > kFixedScratchBytes && ce > 4096) {
    ce -= 1024;
    job_scalars(J, f, p, ce);
    L = job_layout(J, f, false, false);
  }
  if (L.total() > kFixedScratchBytes)
    return fail(ctx, ODC_ERR_OUT_OF_MEMORY, "res %d does not fit the fixed scratch of %zu bytes",
                N, kFixedScratchBytes);
  return ODC_OK;
}

extern "C" int32_t odc_plan_scratch(const odc_field* f, const odc_params* p, int64_t* bytes,
                                    int32_t* fits_fixed) {
  if (!bytes) return ODC_ERR_INVALID_ARG;
  odc_mesh_buffers o;
  memset(&o, 0, sizeof(o));
  TRY(validate_job(nullptr, f, p, &o));
  Job J;
  job_scalars(J, f, p, estimate_edges(1.0, p->res));
  *bytes = (int64_t)job_layout(J, f, false, false).total();
  if (fits_fixed) {
    Layout L;
    *fits_fixed = plan_fixed(nullptr, f, p, 1.0, J, L) == ODC_OK;
  }
  return ODC_OK;
}

// The allocation-free variant: the job's scratch is carved out of the
// device's fixed array, no graph is captured, and an overflow is reported
// rather than regrown.  Nothing here allocates: the job record goes through
// the context's pinned mirror into its device job array (both made at
// context creation).
extern "C" int32_t odc_mesh_extract_noalloc(odc_context* ctx, const odc_field* f,
                                            const odc_params* p, const odc_mesh_buffers* o) {
  if (!ctx) return ODC_ERR_INVALID_ARG;
  TRY(validate_job(ctx, f, p, o));
  if (!ctx->fixed_scratch)
    return fail(ctx, ODC_ERR_HIP, "fixed scratch unavailable: %s", ctx->fixed_err.c_str());
  Job& J = ctx->hjobs[0];
  Layout L;
  TRY(plan_fixed(ctx, f, p, ctx->cap_scale, J, L));
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (ctx->pending) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  ctx->pending = 0;
  char* b = (char*)ctx->fixed_scratch;
  job_bind(J, L, f, b, b + L.grid_total, b + L.grid_total + L.active_total,
           b + L.grid_total + L.active_total + L.mlpw,
           b + L.grid_total + L.active_total + L.mlpw + L.guard);
  J.out_v = o->vertices;
  J.cap_v = o->cap_vertices;
  J.out_t = o->triangles;
  J.cap_t = o->cap_triangles;
  J.out_vloc = o->vertices_local;
  J.out_vref = o->vertex_ref;
  ctx->hweights[0] = f->kind == ODC_FIELD_MLP ? f->weights : nullptr;
  hipStream_t s = ctx->stream;
  HIP_TRY(ctx, hipMemcpyAsync(P<Job>(ctx->djobs), ctx->hjobs, sizeof(Job),
                              hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(P<const float*>(ctx->dweights), ctx->hweights, sizeof(float*),
                              hipMemcpyHostToDevice, s));
  const PipelineShape sh = shape_of(ctx, 1);
  HIP_TRY(ctx, launch_pipeline(P<Job>(ctx->djobs), 1, sh, P<const float*>(ctx->dweights),
                               P<uint32_t>(ctx->table), cfg_for(ctx, 1),
                               ctx->timing ? ctx->ev : nullptr, s));
  HIP_TRY(ctx, launch_gather(P<Job>(ctx->djobs), 1, P<unsigned long long>(ctx->dgather), s));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->hgather, P<unsigned long long>(ctx->dgather),
                              kGatherWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  ctx->pending = 1;
  ctx->pending_fixed = true;
  return ODC_OK;
}

extern "C" int32_t odc_mesh_extract_batch(odc_context* ctx, int32_t n, const odc_field* fields,
                                          const odc_params* params,
                                          const odc_mesh_buffers* outs) {
  return enqueue_batch(ctx, n, fields, params, outs);
}

bool odc::job_overflowed(const odc_context* ctx, int k) {
  return (ctx->hgather[kGatherWords * k + 7] >> 32) != 0;
}

int odc::needed_edges(const odc_context* ctx, int k, bool* guard_over) {
  const unsigned long long* o = ctx->hgather + kGatherWords * k;
  if (guard_over) *guard_over = o[6] > (unsigned long long)ctx->hjobs[k].guard_cap;
  long long need = (long long)o[0];
  if ((long long)((o[1] + 1) / 2) > need) need = (long long)((o[1] + 1) / 2);
  if ((long long)(o[2] * 2 / 3) > need) need = (long long)(o[2] * 2 / 3);
  need += need / 8 + 64;
  const long long all = 3LL * ctx->hjobs[k].g.ea + 64;
  return (int)(need < all ? need : all);
}

// Waits for the pending batch; a job whose active sets outgrew its scratch is
// given room for what it needed and the batch runs again.
static int32_t finish(odc_context* ctx) {
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  for (int attempt = 0;; ++attempt) {
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const int n = ctx->pending;
    bool over = false;
    for (int k = 0; k < n; ++k) over |= job_overflowed(ctx, k);
    if (!over) return ODC_OK;
    if (ctx->pending_fixed) {
      bool gover = false;
      const int need = needed_edges(ctx, 0, &gover);
      return fail(ctx, ODC_ERR_OUT_OF_MEMORY,
                  gover ? "the bf16 guard queue in the fixed scratch overflowed"
                        : "active sets need %d crossing edges; the fixed scratch held %d",
                  need, ctx->hjobs[0].cap_edges);
    }
    if (attempt >= 2) return fail(ctx, ODC_ERR_OUT_OF_MEMORY, "scratch overflow persists");
    for (int k = 0; k < n; ++k) {
      bool gover = false;
      const int need = needed_edges(ctx, k, &gover);
      if (gover) ctx->slots[k].guard_full = true;
      const double est = 12.0 * ctx->p_params[k].res * ctx->p_params[k].res + 4096.0;
      if (need > est * ctx->cap_scale) ctx->cap_scale = need / est;
      TRY(setup_job(ctx, k, &ctx->p_fields[k], &ctx->p_params[k], &ctx->p_outs[k], need));
    }
    TRY(run_batch(ctx, n));
  }
}

void odc::fill_counts(const odc_context* ctx, int k, odc_mesh_counts* c) {
  const unsigned long long* o = ctx->hgather + kGatherWords * k;
  const Job& J = ctx->hjobs[k];
  memset(c, 0, sizeof(*c));
  c->n_active_edges = (int64_t)o[0];
  c->n_pairs = (int64_t)o[1];
  c->n_active_cells = (int64_t)o[2];
  c->n_case3 = (int64_t)o[5];
  c->n_vertices = (int64_t)o[3] + c->n_case3;
  c->n_triangles = (int64_t)o[4];
  c->n_guard_corners = (int64_t)o[6];
  c->n_fp64_cells = (int64_t)(o[7] & 0xFFFFFFFFull);
  // occupancy queries: every corner, the bf16 guard's fp32 repeats, the 1D
  // points (two corner queries each for linear points), the 2D searches'
  // queries, the ones the pairs needed, counted on the device (none with
  // gradient normals, whose passes are not occupancy queries)
  const bool grad = (J.ablation & kAblGradNormals) != 0;
  c->n_search2d_needed = grad ? -1 : (int64_t)o[8];
  c->n_search2d_queries = grad ? 0 : (int64_t)o[8];
  c->n_corner_queries = J.coarse_step ? (int64_t)o[9] : (int64_t)J.g.nc;
  c->n_queries = c->n_corner_queries + c->n_guard_corners +
                 c->n_active_edges * ((J.ablation & kAblLinear1D) ? 2 : J.iters_1d) +
                 c->n_search2d_queries;
  c->n_flipped_faces = (int64_t)o[10];
}

extern "C" int32_t odc_mesh_sync_batch(odc_context* ctx, int32_t n, odc_mesh_counts* counts) {
  if (!ctx || !counts) return ODC_ERR_INVALID_ARG;
  if (!ctx->pending) return fail(ctx, ODC_ERR_INVALID_ARG, "no extract to wait for");
  if (n != ctx->pending)
    return fail(ctx, ODC_ERR_INVALID_ARG, "pending batch has %d jobs", ctx->pending);
  TRY(finish(ctx));
  int32_t rc = ODC_OK;
  for (int k = 0; k < n; ++k) {
    fill_counts(ctx, k, &counts[k]);
    if (counts[k].n_vertices > ctx->p_outs[k].cap_vertices ||
        counts[k].n_triangles > ctx->p_outs[k].cap_triangles)
      rc = fail(ctx, ODC_ERR_CAPACITY, "job %d needs %lld vertices and %lld triangles", k,
                (long long)counts[k].n_vertices, (long long)counts[k].n_triangles);
  }
  return rc;
}

extern "C" int32_t odc_mesh_sync(odc_context* ctx, odc_mesh_counts* c) {
  if (!ctx || !c) return ODC_ERR_INVALID_ARG;
  if (ctx->pending != 1) return fail(ctx, ODC_ERR_INVALID_ARG, "no single extract pending");
  return odc_mesh_sync_batch(ctx, 1, c);
}

extern "C" int32_t odc_get_job_intermediate(odc_context* ctx, int32_t job, int32_t which,
                                            void* dst, int64_t cap_bytes, int64_t* n) {
  if (!ctx || !n) return ODC_ERR_INVALID_ARG;
  if (!ctx->pending) return fail(ctx, ODC_ERR_INVALID_ARG, "no extract yet");
  if (job < 0 || job >= ctx->pending)
    return fail(ctx, ODC_ERR_INVALID_ARG, "job %d outside the last batch of %d", job,
                ctx->pending);
  TRY(finish(ctx));
  const Job& J = ctx->hjobs[job];
  const unsigned long long* o = ctx->hgather + kGatherWords * job;
  const void* src = nullptr;
  int64_t count = 0, elem = 4;
  switch (which) {
    case 0: src = J.labels; count = J.nw_c; break;
    case 1: src = J.elist; count = (int64_t)o[0]; break;
    case 2: src = J.et; count = (int64_t)o[0]; break;
    case 3: src = J.plist; count = (int64_t)o[1]; break;
    case 4: src = J.pf; count = (int64_t)o[1]; elem = 16; break;
    case 5: src = J.clist; count = (int64_t)o[2]; break;
    case 6: src = J.cpm; count = (int64_t)o[2]; break;
    case 7: src = J.cnf; count = (int64_t)o[2]; break;
    case 8: src = J.vbase; count = (int64_t)o[2]; break;
    case 9: src = J.ecase; count = (int64_t)o[0]; break;
    case 10:
      src = J.egrad;
      count = J.egrad ? (int64_t)o[0] : 0;
      elem = 12;
      break;
    case 11:
    case 12:
      if (which == 11 ? !J.etrace : !J.ptrace)
        return fail(ctx, ODC_ERR_INVALID_ARG, "decision traces were not recorded");
      if (which == 12 && 1 + (J.lin1 + J.bin1) + 2 * (J.lin2 + J.bin2) > 64)
        return fail(ctx, ODC_ERR_UNSUPPORTED, "2D searches of more than 64 queries are not traced");
      src = which == 11 ? (const void*)J.etrace : (const void*)J.ptrace;
      count = (int64_t)o[which == 11 ? 0 : 1];
      elem = which == 11 ? 4 : 16;
      break;
    default: return fail(ctx, ODC_ERR_INVALID_ARG, "unknown intermediate %d", which);
  }
  *n = count;
  if (count * elem > cap_bytes)
    return fail(ctx, ODC_ERR_CAPACITY, "intermediate %d needs %lld bytes", which,
                (long long)(count * elem));
  if (count > 0) {
    if (!dst) return fail(ctx, ODC_ERR_INVALID_ARG, "NULL destination");
    HIP_TRY(ctx, hipMemcpyAsync(dst, src, (size_t)(count * elem), hipMemcpyDeviceToDevice,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  return ODC_OK;
}

extern "C" int32_t odc_get_intermediate(odc_context* ctx, int32_t which, void* dst,
                                        int64_t cap_bytes, int64_t* n) {
  return odc_get_job_intermediate(ctx, 0, which, dst, cap_bytes, n);
}

extern "C" int32_t odc_context_set_trace(odc_context* ctx, int32_t enable) {
  if (!ctx) return ODC_ERR_INVALID_ARG;
  if ((enable != 0) != ctx->trace) {
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    drop_graph(ctx);  // the job layout changes
  }
  ctx->trace = enable != 0;
  return ODC_OK;
}

extern "C" int32_t odc_context_set_timing(odc_context* ctx, int32_t enable) {
  if (!ctx) return ODC_ERR_INVALID_ARG;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (enable && !ctx->ev[0])
    for (hipEvent_t& e : ctx->ev) HIP_TRY(ctx, hipEventCreate(&e));
  ctx->timing = enable != 0;
  return ODC_OK;
}

extern "C" int32_t odc_context_set_graph(odc_context* ctx, int32_t enable) {
  if (!ctx) return ODC_ERR_INVALID_ARG;
  if (!enable) drop_graph(ctx);
  ctx->use_graph = enable != 0;
  return ODC_OK;
}

extern "C" int32_t odc_get_stage_times(odc_context* ctx, float* ms, int32_t cap, int32_t* n) {
  if (!ctx || !n) return ODC_ERR_INVALID_ARG;
  *n = 8;
  if (!ctx->timing || !ctx->pending)
    return fail(ctx, ODC_ERR_INVALID_ARG, "stage timing is off or nothing was extracted");
  if (cap < 8 || !ms) return fail(ctx, ODC_ERR_CAPACITY, "need room for 8 stage times");
  HIP_TRY(ctx, hipEventSynchronize(ctx->ev[8]));
  for (int i = 0; i < 8; ++i)
    HIP_TRY(ctx, hipEventElapsedTime(&ms[i], ctx->ev[i], ctx->ev[i + 1]));
  return ODC_OK;
}

extern "C" int32_t odc_field_eval(odc_context* ctx, const odc_field* f, int32_t precision,
                                  const float* xyz, int64_t n, float* z) {
  if (!ctx) return ODC_ERR_INVALID_ARG;
  if (n < 0 || n > (1LL << 30) || (n > 0 && (!xyz || !z)))
    return fail(ctx, ODC_ERR_INVALID_ARG, "bad point count or NULL buffers");
  if (precision != ODC_PREC_FP32 && precision != ODC_PREC_BF16_GUARDED &&
      precision != ODC_PREC_BF16_X3)
    return fail(ctx, ODC_ERR_INVALID_ARG, "unknown precision %d", precision);
  odc_params p;
  odc_params_default(&p, 1);
  p.precision = precision;  // the split-bf16 evaluation needs its weight terms packed
  odc_mesh_buffers o;
  memset(&o, 0, sizeof(o));
  TRY(validate_job(ctx, f, &p, &o));
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (n == 0) return ODC_OK;
  if (ctx->pending) TRY(finish(ctx));
  ctx->pending = 0;
  ctx->pending_fixed = false;
  if (ctx->slots.empty()) ctx->slots.resize(1);
  TRY(setup_job(ctx, 0, f, &p, &o, 0));
  HIP_TRY(ctx, hipMemcpyAsync(P<Job>(ctx->djobs), ctx->hjobs, sizeof(Job),
                              hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(P<const float*>(ctx->dweights), ctx->hweights, sizeof(float*),
                              hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, launch_eval(P<Job>(ctx->djobs), ctx->hjobs[0], P<const float*>(ctx->dweights),
                           precision, xyz, (int)n, z, ctx->cfg, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return ODC_OK;
}

// ------------------------------------------------------------- autotuner
// Picks the persistent grid sizes for one field by timing the stages they
// drive: grid-wide passes, thread-per-element passes and MLP passes.  The
// result is cached for the field's (kind, resolution bucket) and becomes the
// context's default.
extern "C" int32_t odc_autotune(odc_context* ctx, const odc_field* f, const odc_params* p,
                                int32_t* chosen) {
  if (!ctx || !f || !p) return ODC_ERR_INVALID_ARG;
  odc_mesh_buffers o;
  memset(&o, 0, sizeof(o));
  TRY(validate_job(ctx, f, p, &o));
  const bool was_timing = ctx->timing;
  TRY(odc_context_set_timing(ctx, 1));
  struct Tuning {  // timing candidates in ctx->cfg, bypassing the cache
    odc_context* c;
    ~Tuning() { c->tuning = false; }
  } tuning{ctx};
  ctx->tuning = true;
  const int kind = f->kind == ODC_FIELD_MLP ? 1 : 0, rb = res_bucket(p->res);
  if (ctx->tuned_ok[kind][rb]) ctx->cfg = ctx->tuned[kind][rb];
  auto time_stages = [&](float st[8]) -> int32_t {
    TRY(enqueue_batch(ctx, 1, f, p, &o));
    TRY(finish(ctx));
    HIP_TRY(ctx, hipEventSynchronize(ctx->ev[8]));
    for (int i = 0; i < 8; ++i) HIP_TRY(ctx, hipEventElapsedTime(&st[i], ctx->ev[i], ctx->ev[i + 1]));
    return ODC_OK;
  };
  float st[8];
  TRY(time_stages(st));  // warm-up at the current configuration
  const int grid_c[4] = {512, 1024, 2048, 4096};
  const int elem_c[4] = {1024, 2048, 4096, 8192};
  const int mlp_c[2] = {256, 512};
  LaunchCfg best = ctx->cfg;
  float bt = 1e30f;
  for (int v : grid_c) {
    ctx->cfg.grid_blocks = v;
    TRY(time_stages(st));
    const float t = st[1] + st[2] + (f->kind == ODC_FIELD_CSG ? st[0] : 0.0f);
    if (t < bt) { bt = t; best.grid_blocks = v; }
  }
  ctx->cfg.grid_blocks = best.grid_blocks;
  bt = 1e30f;
  for (int v : elem_c) {
    ctx->cfg.elem_blocks = v;
    TRY(time_stages(st));
    const float t = st[5] + st[6] + st[7] + (f->kind == ODC_FIELD_CSG ? st[3] + st[4] : 0.0f);
    if (t < bt) { bt = t; best.elem_blocks = v; }
  }
  ctx->cfg.elem_blocks = best.elem_blocks;
  if (f->kind == ODC_FIELD_MLP) {
    bt = 1e30f;
    for (int v : mlp_c) {
      ctx->cfg.mlp_blocks = v;
      TRY(time_stages(st));
      const float t = st[0] + st[3] + st[4];
      if (t < bt) { bt = t; best.mlp_blocks = v; }
    }
  }
  ctx->cfg = best;
  ctx->tuned[kind][rb] = best;
  ctx->tuned_ok[kind][rb] = true;
  if (!was_timing) ctx->timing = false;
  if (chosen) {
    chosen[0] = best.grid_blocks;
    chosen[1] = best.elem_blocks;
    chosen[2] = best.mlp_blocks;
  }
  return ODC_OK;
}

extern "C" int32_t odc_set_launch_config(odc_context* ctx, const int32_t* cfg3) {
  if (!ctx || !cfg3) return ODC_ERR_INVALID_ARG;
  if (cfg3[0] < 1 || cfg3[1] < 1 || cfg3[2] < 1 || cfg3[0] > 65536 || cfg3[1] > 65536 ||
      cfg3[2] > 65536)
    return fail(ctx, ODC_ERR_INVALID_ARG, "grid sizes must be in 1..65536");
  ctx->cfg.grid_blocks = cfg3[0];
  ctx->cfg.elem_blocks = cfg3[1];
  ctx->cfg.mlp_blocks = cfg3[2];
  memset(ctx->tuned_ok, 0, sizeof(ctx->tuned_ok));  // an explicit shape overrides the cache
  return ODC_OK;
}

extern "C" int32_t odc_get_launch_config(const odc_context* ctx, int32_t kind, int32_t res,
                                         int32_t* cfg3, int32_t* tuned) {
  if (!ctx || !cfg3 || (kind != ODC_FIELD_CSG && kind != ODC_FIELD_MLP) || res < 1)
    return ODC_ERR_INVALID_ARG;
  const int rb = res_bucket(res);
  const bool ok = ctx->tuned_ok[kind][rb];
  const LaunchCfg& c = ok ? ctx->tuned[kind][rb] : ctx->cfg;
  cfg3[0] = c.grid_blocks;
  cfg3[1] = c.elem_blocks;
  cfg3[2] = c.mlp_blocks;
  if (tuned) *tuned = ok ? 1 : 0;
  return ODC_OK;
}
