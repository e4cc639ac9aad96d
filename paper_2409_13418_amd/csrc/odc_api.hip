// C ABI of libodc.so (include/odc.h): context, scratch and stage orchestration.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "../../include/odc.h"
#include "odc_internal.h"

namespace odc {
hipError_t launch_partition_table(uint32_t* table, hipStream_t s);
}

using namespace odc;

namespace {

// Device buffer that only grows.  Growing waits for the stream first, so no
// kernel still uses the old allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct odc_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // scratch
  DevBuf labels, emask, ecount, eprefix, fact, famb, fflip, pcount, pprefix, cmask, ccount,
      cprefix, scan_tmp, counters, guard, elist, et, ecase, ntri, n3, tprefix, c3prefix, quad,
      plist, pf, clist, cpm, cnf, npart, vbase, vloc, mlpw, table;
  // pinned readback: [0..2] active sizes, [3] partition vertices, [4] triangles,
  // [5] case-3, [6..8] counters
  uint64_t* host = nullptr;
  Job job;
  bool pending = false;
  int64_t cap_v = 0, cap_t = 0;
  bool timing = false;
  hipEvent_t ev[9] = {};
};

static int32_t fail(odc_context* ctx, int32_t code, const char* fmt, ...) {
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

#define HIP_TRY(ctx, expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(ctx, ODC_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                              \
  } while (0)

static int32_t ensure(odc_context* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return ODC_OK;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (b.p) HIP_TRY(ctx, hipFree(b.p));
  b.p = nullptr;
  b.bytes = 0;
  const size_t want = bytes + bytes / 4;
  if (hipMalloc(&b.p, want) != hipSuccess) {
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
  if (stream) {
    ctx->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return ODC_ERR_HIP;
    }
    ctx->own_stream = true;
  }
  if (hipHostMalloc((void**)&ctx->host, 16 * sizeof(uint64_t), hipHostMallocDefault) !=
      hipSuccess) {
    odc_context_destroy(ctx);
    return ODC_ERR_OUT_OF_MEMORY;
  }
  memset(ctx->host, 0, 16 * sizeof(uint64_t));
  int32_t rc = ensure(ctx, ctx->table, 256 * sizeof(uint32_t));
  if (rc == ODC_OK && launch_partition_table(P<uint32_t>(ctx->table), ctx->stream) != hipSuccess)
    rc = ODC_ERR_HIP;
  if (rc == ODC_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) rc = ODC_ERR_HIP;
  if (rc != ODC_OK) {
    odc_context_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return ODC_OK;
}

extern "C" void odc_context_destroy(odc_context* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  DevBuf* bufs[] = {&ctx->labels, &ctx->emask, &ctx->ecount, &ctx->eprefix, &ctx->fact,
                    &ctx->famb, &ctx->fflip, &ctx->pcount, &ctx->pprefix, &ctx->cmask,
                    &ctx->ccount, &ctx->cprefix, &ctx->scan_tmp, &ctx->counters, &ctx->guard,
                    &ctx->elist, &ctx->et, &ctx->ecase, &ctx->ntri, &ctx->n3, &ctx->tprefix,
                    &ctx->c3prefix, &ctx->quad, &ctx->plist, &ctx->pf, &ctx->clist, &ctx->cpm,
                    &ctx->cnf, &ctx->npart, &ctx->vbase, &ctx->vloc, &ctx->mlpw, &ctx->table};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (ctx->host) (void)hipHostFree(ctx->host);
  for (hipEvent_t& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

static int32_t validate(odc_context* ctx, const odc_field* f, const odc_params* p,
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
  if (p->precision != ODC_PREC_FP32 && p->precision != ODC_PREC_BF16_GUARDED)
    return fail(ctx, ODC_ERR_INVALID_ARG, "unknown precision %d", p->precision);
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

#define TRY(expr)                     \
  do {                                \
    int32_t r_ = (expr);              \
    if (r_ != ODC_OK) return r_;      \
  } while (0)

static int32_t mark(odc_context* ctx, int i) {
  if (!ctx->timing) return ODC_OK;
  HIP_TRY(ctx, hipEventRecord(ctx->ev[i], ctx->stream));
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

extern "C" int32_t odc_get_stage_times(odc_context* ctx, float* ms, int32_t cap, int32_t* n) {
  if (!ctx || !n) return ODC_ERR_INVALID_ARG;
  *n = 8;
  if (!ctx->timing || !ctx->pending)
    return fail(ctx, ODC_ERR_INVALID_ARG, "stage timing is off or nothing was extracted");
  if (cap < 8 || !ms) return fail(ctx, ODC_ERR_CAPACITY, "need room for 8 stage times");
  HIP_TRY(ctx, hipEventSynchronize(ctx->ev[8]));
  for (int i = 0; i < 8; ++i) HIP_TRY(ctx, hipEventElapsedTime(&ms[i], ctx->ev[i], ctx->ev[i + 1]));
  return ODC_OK;
}

// Packs the MLP weights into the fragment orders of the matrix-core
// evaluators (context scratch) and fills m.
static int32_t prepare_mlp(odc_context* ctx, const odc_field* f, Mlp& m) {
  hipStream_t s = ctx->stream;
  const int kb1f = (f->in_dim + 1) / 2, kb1b = (f->in_dim + 15) / 16, d = f->depth;
  const size_t n_w1f = (size_t)kb1f * 512, n_whf = (size_t)(d - 1) * kHiddenBlocksF32 * 512;
  const size_t n_w1b = (size_t)kb1b * 512, n_whb = (size_t)(d - 1) * kHiddenBlocksBF16 * 512;
  const size_t bytes = (n_w1f + n_whf) * 4 + (n_w1b + n_whb) * 16 + (size_t)(d + 1) * kWidth * 4;
  TRY(ensure(ctx, ctx->mlpw, bytes));
  char* base = P<char>(ctx->mlpw);
  float* w1f = (float*)base;
  float* whf = w1f + n_w1f;
  v8bf* w1b = (v8bf*)(whf + n_whf);
  v8bf* whb = w1b + n_w1b;
  float* bias = (float*)(whb + n_whb);
  float* wout = bias + (size_t)d * kWidth;
  HIP_TRY(ctx, launch_pack_mlp(f->weights, f->in_dim, d, w1f, whf, w1b, whb, bias, wout, s));
  m.w1f = w1f;
  m.whf = whf;
  m.w1b = w1b;
  m.whb = whb;
  m.bias = bias;
  m.wout = wout;
  m.spheres = f->spheres;
  m.sdf_gain = f->sdf_gain;
  m.out_scale = f->out_scale;
  m.n_spheres = f->n_spheres;
  m.depth = d;
  m.in_dim = f->in_dim;
  m.kb1f = kb1f;
  m.kb1b = kb1b;
  // b_out is read back once: the weights are caller data of fixed layout
  const size_t bout_off = (size_t)kWidth * f->in_dim + kWidth +
                          (size_t)(d - 1) * (kWidth * kWidth + kWidth) + kWidth;
  float bout = 0.0f;
  HIP_TRY(ctx, hipMemcpyAsync(&bout, f->weights + bout_off, sizeof(float),
                              hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  m.bout = bout;
  return ODC_OK;
}

extern "C" int32_t odc_mesh_extract(odc_context* ctx, const odc_field* f, const odc_params* p,
                                    const odc_mesh_buffers* o) {
  if (!ctx) return ODC_ERR_INVALID_ARG;
  TRY(validate(ctx, f, p, o));
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  Job& j = ctx->job;
  j = Job();
  const int N = p->res;
  j.g.N = N;
  for (int a = 0; a < 3; ++a) j.g.lo[a] = (float)p->lo[a];
  j.g.h = (float)(p->size / (double)N);
  j.g.nc = (N + 1) * (N + 1) * (N + 1);
  j.g.ea = N * (N + 1) * (N + 1);
  j.g.fa = (N + 1) * N * N;
  j.g.ncell = N * N * N;
  j.kind = f->kind;
  j.precision = p->precision;
  j.prims = f->prims;
  j.n_prims = f->n_prims;
  j.iters_1d = p->iters_1d;
  j.lin1 = p->lin1;
  j.bin1 = p->bin1;
  j.lin2 = p->lin2;
  j.bin2 = p->bin2;
  j.range1 = p->range1;
  j.range2 = p->range2;
  j.qef_tau = p->qef_tau;
  j.guard_logit = p->guard_logit;
  j.fp64_cond = p->fp64_cond;

  const int nw_c = (j.g.nc + 31) / 32;
  const int nw_e = (3 * j.g.ea + 31) / 32;
  const int nw_f = (3 * j.g.fa + 31) / 32;
  const int nw_cell = (j.g.ncell + 31) / 32;
  int nw_max = nw_e > nw_f ? nw_e : nw_f;
  if (nw_cell > nw_max) nw_max = nw_cell;

  TRY(ensure(ctx, ctx->labels, (size_t)nw_c * 4));
  TRY(ensure(ctx, ctx->emask, (size_t)nw_e * 4));
  TRY(ensure(ctx, ctx->ecount, (size_t)nw_e * 4));
  TRY(ensure(ctx, ctx->eprefix, (size_t)(nw_e + 1) * 4));
  TRY(ensure(ctx, ctx->fact, (size_t)nw_f * 4));
  TRY(ensure(ctx, ctx->famb, (size_t)nw_f * 4));
  TRY(ensure(ctx, ctx->fflip, (size_t)nw_f * 4));
  TRY(ensure(ctx, ctx->pcount, (size_t)nw_f * 4));
  TRY(ensure(ctx, ctx->pprefix, (size_t)(nw_f + 1) * 4));
  TRY(ensure(ctx, ctx->cmask, (size_t)nw_cell * 4));
  TRY(ensure(ctx, ctx->ccount, (size_t)nw_cell * 4));
  TRY(ensure(ctx, ctx->cprefix, (size_t)(nw_cell + 1) * 4));
  TRY(ensure(ctx, ctx->counters, 4 * sizeof(unsigned long long)));
  j.labels = P<uint32_t>(ctx->labels);
  j.emask = P<uint32_t>(ctx->emask);
  j.eprefix = P<uint32_t>(ctx->eprefix);
  j.fact = P<uint32_t>(ctx->fact);
  j.famb = P<uint32_t>(ctx->famb);
  j.fflip = P<uint32_t>(ctx->fflip);
  j.pprefix = P<uint32_t>(ctx->pprefix);
  j.cmask = P<uint32_t>(ctx->cmask);
  j.cprefix = P<uint32_t>(ctx->cprefix);
  j.counters = P<unsigned long long>(ctx->counters);

  if (f->kind == ODC_FIELD_MLP) {
    TRY(prepare_mlp(ctx, f, j.mlp));
    if (p->precision == ODC_PREC_BF16_GUARDED) {
      TRY(ensure(ctx, ctx->guard, (size_t)j.g.nc * 4));
      j.guard_list = P<uint32_t>(ctx->guard);
      j.guard_cap = j.g.nc;
    }
  }
  HIP_TRY(ctx, hipMemsetAsync(j.counters, 0, 4 * sizeof(unsigned long long), s));

  // (a) corner labels, then classification and the three scans
  TRY(mark(ctx, 0));
  HIP_TRY(ctx, launch_labels(j, s));
  TRY(mark(ctx, 1));
  TRY(ensure(ctx, ctx->scan_tmp, scan_tmp_words(nw_max) * 4));
  uint32_t* tmp = P<uint32_t>(ctx->scan_tmp);
  HIP_TRY(ctx, launch_classify(j, P<uint32_t>(ctx->ecount), P<uint32_t>(ctx->pcount),
                               P<uint32_t>(ctx->ccount), P<uint32_t>(ctx->table), s));
  HIP_TRY(ctx, scan_exclusive(P<uint32_t>(ctx->ecount), j.eprefix, nw_e, tmp, s));
  HIP_TRY(ctx, scan_exclusive(P<uint32_t>(ctx->pcount), j.pprefix, nw_f, tmp, s));
  HIP_TRY(ctx, scan_exclusive(P<uint32_t>(ctx->ccount), j.cprefix, nw_cell, tmp, s));
  TRY(mark(ctx, 2));
  uint32_t tot[3];
  HIP_TRY(ctx, hipMemcpyAsync(&tot[0], j.eprefix + nw_e, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(&tot[1], j.pprefix + nw_f, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(&tot[2], j.cprefix + nw_cell, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  j.n_edges = (int)tot[0];
  j.n_pairs = (int)tot[1];
  j.n_cells = (int)tot[2];

  const size_t ne = (size_t)j.n_edges + 1, np = (size_t)j.n_pairs + 1,
               nc = (size_t)j.n_cells + 1;
  TRY(ensure(ctx, ctx->elist, ne * 4));
  TRY(ensure(ctx, ctx->et, ne * 4));
  TRY(ensure(ctx, ctx->ecase, ne * 4));
  TRY(ensure(ctx, ctx->ntri, ne * 4));
  TRY(ensure(ctx, ctx->n3, ne * 4));
  TRY(ensure(ctx, ctx->tprefix, (ne + 1) * 4));
  TRY(ensure(ctx, ctx->c3prefix, (ne + 1) * 4));
  TRY(ensure(ctx, ctx->quad, ne * sizeof(int4)));
  TRY(ensure(ctx, ctx->plist, np * 4));
  TRY(ensure(ctx, ctx->pf, np * sizeof(double2)));
  TRY(ensure(ctx, ctx->clist, nc * 4));
  TRY(ensure(ctx, ctx->cpm, nc * 4));
  TRY(ensure(ctx, ctx->cnf, nc * 4));
  TRY(ensure(ctx, ctx->npart, nc * 4));
  TRY(ensure(ctx, ctx->vbase, (nc + 1) * 4));
  TRY(ensure(ctx, ctx->vloc, nc * 4 * 3 * sizeof(float)));
  TRY(ensure(ctx, ctx->scan_tmp, scan_tmp_words((int)(ne > nc ? ne : nc)) * 4));
  tmp = P<uint32_t>(ctx->scan_tmp);
  j.elist = P<int>(ctx->elist);
  j.et = P<float>(ctx->et);
  j.ecase = P<uint32_t>(ctx->ecase);
  j.tprefix = P<uint32_t>(ctx->tprefix);
  j.c3prefix = P<uint32_t>(ctx->c3prefix);
  j.quad = P<int4>(ctx->quad);
  j.plist = P<int>(ctx->plist);
  j.pf = P<double2>(ctx->pf);
  j.clist = P<int>(ctx->clist);
  j.cpm = P<uint32_t>(ctx->cpm);
  j.cnf = P<uint32_t>(ctx->cnf);
  j.vbase = P<uint32_t>(ctx->vbase);
  j.vloc = P<float>(ctx->vloc);
  j.out_v = o->vertices;
  j.cap_v = o->cap_vertices;
  j.out_t = o->triangles;
  j.cap_t = o->cap_triangles;
  j.out_vloc = o->vertices_local;
  j.out_vref = o->vertex_ref;

  HIP_TRY(ctx, launch_compact(j, s));
  TRY(mark(ctx, 3));
  // (b) 1D points, (c) 2D points
  HIP_TRY(ctx, launch_bisect(j, s));
  TRY(mark(ctx, 4));
  HIP_TRY(ctx, launch_search2d(j, s));
  TRY(mark(ctx, 5));
  // (d) partitions, vertex numbering, QEF
  HIP_TRY(ctx, launch_cell_count(j, P<uint32_t>(ctx->npart), P<uint32_t>(ctx->table), s));
  HIP_TRY(ctx, scan_exclusive(P<uint32_t>(ctx->npart), j.vbase, j.n_cells, tmp, s));
  TRY(mark(ctx, 6));
  HIP_TRY(ctx, launch_cell_qef(j, s));
  TRY(mark(ctx, 7));
  // (e) emission
  HIP_TRY(ctx, launch_emit_count(j, P<uint32_t>(ctx->ntri), P<uint32_t>(ctx->n3), s));
  HIP_TRY(ctx, scan_exclusive(P<uint32_t>(ctx->ntri), j.tprefix, j.n_edges, tmp, s));
  HIP_TRY(ctx, scan_exclusive(P<uint32_t>(ctx->n3), j.c3prefix, j.n_edges, tmp, s));
  HIP_TRY(ctx, launch_emit_write(j, s));
  TRY(mark(ctx, 8));

  uint64_t* h = ctx->host;
  memset(h, 0, 16 * sizeof(uint64_t));
  h[0] = tot[0];
  h[1] = tot[1];
  h[2] = tot[2];
  HIP_TRY(ctx, hipMemcpyAsync(&h[3], j.vbase + j.n_cells, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(&h[4], j.tprefix + j.n_edges, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(&h[5], j.c3prefix + j.n_edges, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(&h[6], j.counters, 3 * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
  ctx->pending = true;
  ctx->cap_v = o->cap_vertices;
  ctx->cap_t = o->cap_triangles;
  return ODC_OK;
}

// number of set bits in the flip words (read once per sync; diagnostics only)
static int32_t count_flips(odc_context* ctx, int64_t* out) {
  const Job& j = ctx->job;
  const int nw_f = (3 * j.g.fa + 31) / 32;
  std::string tmp;
  uint32_t* host = (uint32_t*)malloc((size_t)nw_f * 4);
  if (!host) return fail(ctx, ODC_ERR_OUT_OF_MEMORY, "host allocation failed");
  hipError_t e = hipMemcpy(host, j.fflip, (size_t)nw_f * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    free(host);
    return fail(ctx, ODC_ERR_HIP, "flip readback: %s", hipGetErrorString(e));
  }
  int64_t n = 0;
  for (int i = 0; i < nw_f; ++i) n += __builtin_popcount(host[i]);
  free(host);
  *out = n;
  return ODC_OK;
}

extern "C" int32_t odc_mesh_sync(odc_context* ctx, odc_mesh_counts* c) {
  if (!ctx || !c) return ODC_ERR_INVALID_ARG;
  if (!ctx->pending) return fail(ctx, ODC_ERR_INVALID_ARG, "no extract to wait for");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  const uint64_t* h = ctx->host;
  const Job& j = ctx->job;
  memset(c, 0, sizeof(*c));
  c->n_active_edges = (int64_t)h[0];
  c->n_pairs = (int64_t)h[1];
  c->n_active_cells = (int64_t)h[2];
  c->n_case3 = (int64_t)h[5];
  c->n_vertices = (int64_t)h[3] + c->n_case3;
  c->n_triangles = (int64_t)h[4];
  c->n_guard_corners = (int64_t)h[6];
  c->n_fp64_cells = (int64_t)h[7];
  const int64_t per_pair = 1 + (j.lin1 + j.bin1) + 2 * (j.lin2 + j.bin2);
  c->n_queries = (int64_t)j.g.nc + c->n_guard_corners + c->n_active_edges * j.iters_1d +
                 c->n_pairs * per_pair;
  TRY(count_flips(ctx, &c->n_flipped_faces));
  if (c->n_vertices > ctx->cap_v || c->n_triangles > ctx->cap_t)
    return fail(ctx, ODC_ERR_CAPACITY, "mesh needs %lld vertices and %lld triangles",
                (long long)c->n_vertices, (long long)c->n_triangles);
  return ODC_OK;
}

extern "C" int32_t odc_get_intermediate(odc_context* ctx, int32_t which, void* dst,
                                        int64_t cap_bytes, int64_t* n) {
  if (!ctx || !n) return ODC_ERR_INVALID_ARG;
  if (!ctx->pending) return fail(ctx, ODC_ERR_INVALID_ARG, "no extract yet");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  const Job& j = ctx->job;
  const void* src = nullptr;
  int64_t count = 0, elem = 4;
  switch (which) {
    case 0: src = j.labels; count = (j.g.nc + 31) / 32; break;
    case 1: src = j.elist; count = j.n_edges; break;
    case 2: src = j.et; count = j.n_edges; break;
    case 3: src = j.plist; count = j.n_pairs; break;
    case 4: src = j.pf; count = j.n_pairs; elem = 16; break;
    case 5: src = j.clist; count = j.n_cells; break;
    case 6: src = j.cpm; count = j.n_cells; break;
    case 7: src = j.cnf; count = j.n_cells; break;
    case 8: src = j.vbase; count = j.n_cells; break;
    case 9: src = j.ecase; count = j.n_edges; break;
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

extern "C" int32_t odc_field_eval(odc_context* ctx, const odc_field* f, int32_t precision,
                                  const float* xyz, int64_t n, float* z) {
  if (!ctx) return ODC_ERR_INVALID_ARG;
  if (n < 0 || n > (1LL << 30) || (n > 0 && (!xyz || !z)))
    return fail(ctx, ODC_ERR_INVALID_ARG, "bad point count or NULL buffers");
  if (precision != ODC_PREC_FP32 && precision != ODC_PREC_BF16_GUARDED)
    return fail(ctx, ODC_ERR_INVALID_ARG, "unknown precision %d", precision);
  odc_params p;
  odc_params_default(&p, 1);
  odc_mesh_buffers o;
  memset(&o, 0, sizeof(o));
  TRY(validate(ctx, f, &p, &o));
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  Mlp m = Mlp();
  if (f->kind == ODC_FIELD_MLP) TRY(prepare_mlp(ctx, f, m));
  HIP_TRY(ctx, launch_eval(f->kind, precision, f->prims, f->n_prims, m, xyz, (int)n, z,
                           ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return ODC_OK;
}
