/*
 * odc.h -- C ABI of libodc.so: Occupancy-Based Dual Contouring on one AMD
 * MI355X (gfx950).
 *
 * Method: Hwang & Sung, "Occupancy-Based Dual Contouring", SIGGRAPH Asia
 * 2024.  Problem statement (Sec. 3): an occupancy function phi and a uniform
 * grid over a cubic domain go in; a Manifold-Dual-Contouring mesh comes out.
 * The path: (a) phi' at every grid corner; (b) the 1D point of every crossing
 * edge by bisection (Sec. 5.1); (c) 2D points of every crossing-edge pair on
 * a face by three line-binary searches (Sec. 5.2, App. A.1.3-A.1.4); (d) per
 * cell partitions of the crossing edges (App. A.1.1), normals from the 2D
 * points (Sec. 5.3) and the QEF of Eq. 2 for each partition's 3D point;
 * (e) MDC quads split by the intersection-free rule (App. A.1.5).
 *
 * Memory: every pointer inside odc_field and odc_mesh_buffers is DEVICE
 * memory owned by the caller; it must stay valid until odc_mesh_sync (or the
 * stream work) completes.  Scratch belongs to the context.  Nothing is freed
 * across the ABI.  Calls never throw; every call returns an odc_status and
 * leaves a message in odc_last_error().  A context is not thread-safe: one
 * host thread at a time.
 *
 * Grid conventions (N = res cells per axis, corners 0..N):
 *   corner (i,j,k) id = i + (N+1)(j + (N+1)k); cell id = i + N(j + Nk)
 *   x-edges id = i + N(j + (N+1)k), then y-edges Ex + i + (N+1)(j + Nk),
 *   then z-edges Ex + Ey + i + (N+1)(j + (N+1)k), Ex = Ey = N(N+1)^2
 *   faces with normal x: i + (N+1)(j + Nk); normal y: Fx + i + N(j + (N+1)k);
 *   normal z: Fx + Fy + i + N(j + Nk), Fx = Fy = (N+1)N^2
 */
#ifndef ODC_H
#define ODC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ODC_OK = 0,
  ODC_ERR_INVALID_ARG = 1,   /* a NULL pointer, a size or parameter out of range */
  ODC_ERR_OUT_OF_MEMORY = 2, /* scratch could not be allocated */
  ODC_ERR_CAPACITY = 3,      /* output buffers too small; counts hold the sizes needed */
  ODC_ERR_HIP = 4,           /* a HIP runtime call failed; see odc_last_error */
  ODC_ERR_UNSUPPORTED = 5,   /* a field shape the kernels do not implement */
  ODC_ERR_BUSY = 6           /* reserved */
} odc_status;

typedef struct odc_context odc_context;

/* Occupancy field (Sec. 3: phi': R^3 -> {0,1}).  Two kinds:
 *  ODC_FIELD_CSG  analytic primitives, n_prims records of 20 floats:
 *                 [0] op (0 union, 1 subtract, 2 intersect; left fold, first ignored)
 *                 [1] type (0 sphere, 1 box, 2 half-space) [2..4] centre c
 *                 [5..7] sphere radius at [5] | box half extents | half-space normal
 *                 [8..16] box rotation rows R (box-local = R (x - c))
 *                 Labels are decided in binary32: sphere (dx^2+dy^2)+dz^2 < r*r;
 *                 box |(R_a0 dx + R_a1 dy) + R_a2 dz| < half_a; half-space
 *                 (n_x dx + n_y dy) + n_z dz < 0.
 *  ODC_FIELD_MLP  phi = sigmoid(z), z = out_scale * MLP(gamma(x)) - sdf_gain * sdf(x);
 *                 gamma(x) = (x, sin(2^k pi x), cos(2^k pi x)), k < n_bands
 *                 (in_dim = 3 + 6 n_bands <= 45); depth hidden ReLU layers of
 *                 width 256; weights binary32: W1[256][in_dim], b1[256], then
 *                 (W[256][256], b[256]) per further layer, w_out[256], b_out;
 *                 sdf = min over n_spheres spheres (cx,cy,cz,r) of |x-c| - r.
 *                 Inside iff z > 0 (phi > 0.5, strict). */
enum { ODC_FIELD_CSG = 0, ODC_FIELD_MLP = 1 };

typedef struct {
  int32_t kind;
  const float* prims;   /* CSG records, device */
  int32_t n_prims;
  const float* weights; /* MLP weights, device */
  int32_t in_dim, width, depth, n_bands;
  const float* spheres; /* MLP sdf spheres, device, 4 floats each */
  int32_t n_spheres;
  float sdf_gain, out_scale;
} odc_field;

/* Evaluation precision for MLP fields (ignored for CSG).
 *  FP32           every query in binary32 on matrix cores (fp32 MFMA).
 *  BF16_GUARDED   corner queries in bf16 on matrix cores with fp32
 *                 accumulation; any corner whose bf16 logit lies within
 *                 guard_logit of zero is re-evaluated by the fp32 path, and the
 *                 searches of (b) and (c), whose queries sit at the surface,
 *                 use the fp32 path directly.
 *  BF16_X3        corner queries and their guard exactly as BF16_GUARDED,
 *                 so every corner sign, and with them the crossing edges,
 *                 face pairs, active cells and faces, are the FP32 path's;
 *                 every search query of (b) and (c) at binary32 accuracy on
 *                 the bf16 matrix cores: weights and activations each split
 *                 exactly into three bf16 terms, the six products of terms
 *                 i + j <= 2 accumulated in binary32 (the three left out are
 *                 each at most about 2^-24 of the product).  Search logits
 *                 agree with the FP32 path's to binary32 rounding, not bit
 *                 for bit, so 1D/2D points (and vertices) may differ from
 *                 its at decisions within that rounding of the threshold.
 *                 The method only (ablation bits: UNSUPPORTED). */
enum { ODC_PREC_FP32 = 0, ODC_PREC_BF16_GUARDED = 1, ODC_PREC_BF16_X3 = 2 };

typedef struct {
  double lo[3];          /* domain minimum corner */
  double size;           /* domain edge length; h = size / res */
  int32_t res;           /* cells per axis, 1..512 */
  int32_t iters_1d;      /* bisection halvings per crossing edge, 1..23 (paper: 15) */
  int32_t lin1, bin1;    /* step-1 line-binary search: samples, halvings (4, 11) */
  int32_t lin2, bin2;    /* step-2 line-binary searches (3, 12) */
  float range1, range2;  /* search ranges in cell widths (0.8, sqrt(2)/2) */
  float qef_tau;         /* QEF eigenvalue truncation relative to the largest (1e-2) */
  double fp64_cond;      /* QEF redone in binary64 above this condition number (1e6); > 0 */
  int32_t precision;     /* ODC_PREC_* */
  float guard_logit;     /* bf16 guard band on z: 2 atanh(0.02) for |phi - 0.5| < 0.01;
                          * finite and > 0.  The guarded labels equal the fp32 path's
                          * when the bf16 logit error stays below the band; that is
                          * measured for the fields of this library's tests (< half the
                          * band), not known for arbitrary weights */
  int32_t ablation;      /* 0 = the method; ODC_ABL_* bits select Table 3's baselines */
  int32_t clamp_vertices; /* 1: clamp each 3D point into its cell.  The paper is silent
                          * and the method leaves them where the QEF puts them (0);
                          * clamping keeps the intersection-free split's envelope
                          * argument valid (fewer self-intersections) */
  int32_t coarse_step;   /* adaptive corner evaluation (the paper leaves adaptive
                          * resolution to future work; this is one reading of it, for
                          * the evaluation only: the mesh stays on the uniform grid).
                          * 0 or 1: every corner is evaluated.  S in 2..64 (res a
                          * multiple of S): the field is first evaluated (binary32) on
                          * the corners of the coarse grid of S x S x S cells; a coarse
                          * cell is marked when its 8 corners' labels differ or (MLP)
                          * one of them has |z| < coarse_band; only fine corners in
                          * marked coarse cells are evaluated (in blocks of 32 to 128
                          * consecutive corners), every other corner takes the common
                          * label of its unmarked coarse cell.  Exact, i.e. the same
                          * labels as S = 0, when no unmarked coarse cell holds a
                          * label change: for MLP fields whenever coarse_band >=
                          * L sqrt(3) S h for a bound L on |grad z| (not checked);
                          * for CSG fields always: a coarse corner is in the band when
                          * a signed-distance bound of the solid (the primitives'
                          * exact distances folded with min/max, 1-Lipschitz) is
                          * below sqrt(3) S h there. */
  float coarse_band;     /* logit band of the coarse marking (MLP; >= 0, finite; CSG
                          * fields ignore it) */
} odc_params;

/* Ablation baselines (Sec. 4 and Table 3): each bit replaces one step of the
 * method with Manifold Dual Contouring's.
 *  LINEAR_1D     1D points by Eq. 1 from psi = phi - 1/2 = tanh(z/2)/2 at the
 *                edge's corners (binary32; 1/2 for a CSG field)
 *  GRAD_NORMALS  QEF normals = the logit's gradient at the 1D point (Eq. 2),
 *                by forward-mode differentiation through the network on the
 *                matrix cores; no 2D points are searched.  MLP fields only
 *                (UNSUPPORTED otherwise)
 *  MDC_SPLIT     every quad split as case 1 of App. A.1.5 (no case 3)
 *  SDF_INPUT     with LINEAR_1D only (INVALID_ARG otherwise): the field is a
 *                signed distance psi (inside where psi < 0, the DeepSDF
 *                results of S.3.5) carried as its logit z = -psi (say
 *                out_scale = -1 and sdf_gain = 0 take the network's output as
 *                psi), so Eq. 1 interpolates z itself rather than tanh(z/2)/2.
 *                The method proper needs no flag for such a field: it reads
 *                only the sign of z.  No effect on CSG fields (t = 1/2). */
enum { ODC_ABL_LINEAR_1D = 1, ODC_ABL_GRAD_NORMALS = 2, ODC_ABL_MDC_SPLIT = 4,
       ODC_ABL_SDF_INPUT = 8 };

/* Output buffers (device, caller-owned).  vertices: 3 floats per vertex,
 * world coordinates.  triangles: 3 int32 vertex ids each, oriented so the
 * normal points from inside to outside.  vertices_local / vertex_ref are
 * optional (NULL): a vertex's offset in cell widths from grid corner
 * vertex_ref (binary32), exact enough to compare at 512^3. */
typedef struct {
  float* vertices;
  int64_t cap_vertices;
  int32_t* triangles;
  int64_t cap_triangles;
  float* vertices_local;
  int32_t* vertex_ref;
} odc_mesh_buffers;

typedef struct {
  int64_t n_vertices;      /* partition vertices + case-3 vertices */
  int64_t n_triangles;
  int64_t n_active_edges;  /* crossing edges */
  int64_t n_pairs;         /* crossing-edge pairs on faces (2D points) */
  int64_t n_active_cells;
  int64_t n_case3;         /* quads split into four triangles */
  int64_t n_flipped_faces; /* ambiguous faces given the manifold-fix pairing */
  int64_t n_fp64_cells;    /* QEF solves redone in binary64 */
  int64_t n_guard_corners; /* bf16 corner queries re-evaluated in fp32 */
  int64_t n_queries;       /* occupancy queries issued (corners, guard repeats, searches) */
  int64_t n_search2d_queries; /* of which in the 2D searches: the queries each pair needs
                                 (= n_search2d_needed) */
  int64_t n_search2d_needed;  /* the 2D-search queries the method itself needs, summed
                                 over pairs (m; per ray the linear samples up to the first
                                 label change and the halvings; no step-2 rays when step 1
                                 ends at m), at most n_pairs x (1 + lin1 + bin1 +
                                 2 (lin2 + bin2)).  -1 with gradient normals (no 2D
                                 searches). */
  int64_t n_corner_queries;   /* corner queries of stage (a): (res + 1)^3, or with
                                 coarse_step > 1 the coarse corners plus the fine corners
                                 evaluated (the bf16 guard's repeats not included) */
} odc_mesh_counts;

/* Status text (static storage). */
const char* odc_status_string(int32_t status);
/* Detail of the last failure on this context (context-owned, valid until the next call). */
const char* odc_last_error(const odc_context* ctx);

/* Creates a context on HIP device `device`.  hip_stream: a hipStream_t to
 * enqueue on, or NULL for a context-owned stream (default priority). */
int32_t odc_context_create(int32_t device, void* hip_stream, odc_context** out);
void odc_context_destroy(odc_context* ctx);

/* Fills the paper's parameters (App. A.1.4, Sec. 5.1) for res cells over [lo, lo+size]^3. */
void odc_params_default(odc_params* p, int32_t res);

/* Meshes one field.  Enqueues the whole path on the context stream with no
 * host synchronisation (active sets live in context scratch sized from the
 * resolution; see odc_mesh_sync).  Errors: INVALID_ARG for bad params,
 * NULL pointers with non-zero capacity, or an MLP without weights;
 * UNSUPPORTED for MLP width != 256, depth outside 1..8 or in_dim > 45;
 * OUT_OF_MEMORY; HIP. */
int32_t odc_mesh_extract(odc_context* ctx, const odc_field* field, const odc_params* params,
                         const odc_mesh_buffers* out);

/* Waits for the last extract and reports its counts.  ODC_ERR_CAPACITY if
 * the vertices or triangles did not fit: nothing beyond the capacities was
 * written and the counts hold the sizes needed.  If the active sets outgrew
 * the context's scratch, the extraction is redone with enough scratch before
 * returning (the scratch estimate then grows for later calls). */
int32_t odc_mesh_sync(odc_context* ctx, odc_mesh_counts* counts);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid it): odc_mesh_extract whose
 * scratch (bit sets, active sets, packed weights, guard queue, counters)
 * lives in one fixed device array of 192 MiB per GPU, held from library load
 * until the process ends.  No hipMalloc, hipFree or allocating library call
 * is made, and no graph is captured.  The crossing-edge capacity is the
 * planned estimate, cut to what the array holds (a 256^3 grid fits; 512^3
 * does not: OUT_OF_MEMORY with the sizes, before anything is launched).
 * Asynchronous; wait with odc_mesh_sync, which then never regrows or reruns:
 * active sets or a bf16 guard queue that outgrow the array give
 * OUT_OF_MEMORY (the counts still hold what was found).  Every call on a GPU shares that GPU's array and
 * leaves its contents there until the next call: calls on one GPU that
 * overlap (several contexts or streams) race, and an earlier extract's
 * intermediates are gone after the next one.  Same arguments and errors as
 * odc_mesh_extract otherwise. */
int32_t odc_mesh_extract_noalloc(odc_context* ctx, const odc_field* field,
                                 const odc_params* params, const odc_mesh_buffers* out);

/* Device scratch that an extraction of this field and grid needs, computed on
 * the host alone (no device, no context): *bytes = what odc_mesh_extract
 * allocates for it at the planned crossing-edge capacity (bit sets over the
 * grid, active sets, packed weights, guard queue); *fits_fixed (may be NULL)
 * = 1 when odc_mesh_extract_noalloc accepts it.  For planning a server's
 * arena or a caller's memory.  Errors: the argument checks of
 * odc_mesh_extract; INVALID_ARG for a NULL bytes. */
int32_t odc_plan_scratch(const odc_field* field, const odc_params* params, int64_t* bytes,
                         int32_t* fits_fixed);

/* Failure injection for tests of the error paths: after `after` more device
 * allocations by the library (context scratch, server arenas), every further
 * one fails as if the device were out of memory, until called again with
 * after < 0 (no limit, the default).  The calls that needed the memory return
 * OUT_OF_MEMORY and leave their context usable.  Process-wide. */
int32_t odc_inject_alloc_failures(int32_t after);

/* Batched meshing: n fields (each with its own params and output buffers) in
 * one launch per stage -- persistent kernels walk all jobs of the batch, so
 * many small or uneven shapes fill the GPU together.  Asynchronous; results
 * are identical to meshing each field alone.  n is 1..1024.  The same errors
 * as odc_mesh_extract, per job. */
int32_t odc_mesh_extract_batch(odc_context* ctx, int32_t n, const odc_field* fields,
                               const odc_params* params, const odc_mesh_buffers* outs);
/* Waits for the batch; counts[k] for job k.  ODC_ERR_CAPACITY if any job's
 * outputs did not fit (its counts then hold the sizes needed). */
int32_t odc_mesh_sync_batch(odc_context* ctx, int32_t n, odc_mesh_counts* counts);

/* Graph replay.  When enabled (and stage timing is off), the launch sequence
 * of a batch is captured once into a hipGraph and replayed for every later
 * batch of the same size and field kinds; the kernels read all job data from
 * device memory, so one graph serves any fields and resolutions. */
int32_t odc_context_set_graph(odc_context* ctx, int32_t enable);

/* Autotuner: times the extraction of `field` under candidate persistent grid
 * sizes (grid-wide passes, per-element passes, matrix-core passes) and
 * writes the fastest of each to chosen[3] (may be NULL).  The result is
 * cached per (field kind, resolution bucket: res <= 64, <= 128, <= 256,
 * above) and becomes the context's default: an extraction or batch uses the
 * cached entry of its dominant job (the largest MLP job, else the largest
 * job), else the default.  Synchronous. */
int32_t odc_autotune(odc_context* ctx, const odc_field* field, const odc_params* params,
                     int32_t* chosen);
/* Sets the three grid sizes (blocks of 256 threads) directly as the default
 * and clears the autotuner's cache. */
int32_t odc_set_launch_config(odc_context* ctx, const int32_t* grid_elem_mlp_blocks);
/* The grid sizes an extraction whose dominant job has field kind `kind` and
 * `res` cells per axis would use (cfg3[3]), and whether they come from the
 * autotuner's cache (*tuned = 1; may be NULL).  Errors: INVALID_ARG. */
int32_t odc_get_launch_config(const odc_context* ctx, int32_t kind, int32_t res, int32_t* cfg3,
                              int32_t* tuned);

/* Copies an intermediate array of the last extract (after odc_mesh_sync) into
 * dst (device memory of cap_bytes).  *n receives the element count.
 *  0 corner label words   uint32 per 32 corners, bit c%32 of word c/32 (1 = inside)
 *  1 crossing edge ids    int32, ascending
 *  2 1D points            float t per crossing edge, from the lower corner
 *  3 pair records         int32 face id << 1 | slot, ascending
 *  4 2D points            double2 face-local (u,v) per pair (u,v: the two other axes, ascending)
 *  5 active cell ids      int32, ascending
 *  6 cell partition map   uint32: 2 bits per cell-local edge (crossing edges only)
 *  7 cell counts          uint32: npart | flipmask << 4 (bit lf: local face 2*axis+side)
 *  8 vertex base          int32 per active cell
 *  9 emission case        int32 per crossing edge: 0 none, 1, 2, 3
 * 10 edge gradients       3 floats per crossing edge: dz/dx at the 1D point (world
 *                         units; ODC_ABL_GRAD_NORMALS only, else 0 elements)
 * 11 1D decision trace    uint32 per crossing edge: bit i = the label (1 inside) that
 *                         query i of its bisection returned (Sec. 5.1)
 * 12 2D decision trace    2 x uint64 per pair: [0] bit q = the label of query q of its
 *                         search, [1] bit q set when query q was evaluated.  Queries in
 *                         order: q = 0 the midpoint m, then step 1's ray (lin1 samples,
 *                         bin1 halvings), then step 2's ray towards the pair's first
 *                         1D point and the opposite ray (lin2 + bin2 each) (Sec. 5.2,
 *                         App. A.1.3).  A linear sample that cannot move any bracket of
 *                         the wavefront's pairs may be skipped (bit clear in [1]).
 * 11 and 12 exist only when odc_context_set_trace was on for the extract (else
 * INVALID_ARG); 12 only for searches of at most 64 queries (else UNSUPPORTED).
 * Errors: INVALID_ARG for an unknown `which`; CAPACITY when cap_bytes is too small. */
int32_t odc_get_intermediate(odc_context* ctx, int32_t which, void* dst, int64_t cap_bytes,
                             int64_t* n);
/* The same for job `job` (0-based) of the last batch.  INVALID_ARG when job is
 * outside the last batch. */
int32_t odc_get_job_intermediate(odc_context* ctx, int32_t job, int32_t which, void* dst,
                                 int64_t cap_bytes, int64_t* n);

/* Decision traces.  When enabled, later extracts on this context also record
 * the label of every occupancy query of the 1D and 2D searches (intermediates
 * 11 and 12), so that a checker can replay the searches' branches.  Costs
 * 4 bytes of scratch per crossing edge and 16 per pair, and one store per
 * element; off by default.  Server lanes never record them. */
int32_t odc_context_set_trace(odc_context* ctx, int32_t enable);

/* Self-intersections of a triangle mesh (the quality metric of Sec. 6 and
 * Table 3): the number of pairs of triangles that share no vertex and whose
 * closed triangles intersect, counted on the context's GPU.  vertices:
 * n_vertices x 3 floats, triangles: n_triangles x 3 int32 (device memory,
 * caller-owned).  cell > 0 is the side of the uniform grid that finds
 * candidate pairs (the meshing grid's cell width suits this library's
 * meshes; the count does not depend on it).  Allocates and frees temporary
 * device memory and synchronises the context's stream.
 * Errors: INVALID_ARG for bad arguments, a vertex index out of range, a
 * non-finite triangle or one spanning more than 4096 grid cubes. */
int32_t odc_count_self_intersections(odc_context* ctx, const float* vertices, int64_t n_vertices,
                                     const int32_t* triangles, int64_t n_triangles, double cell,
                                     int64_t* count);

/* Evaluates the field at n world points (xyz: device, 3 floats each) into z
 * (device, n floats): for MLP fields the logit z (inside iff z > 0) computed
 * by the same matrix-core code as the meshing path in the given precision
 * (ODC_PREC_BF16_GUARDED here means the plain bf16 evaluation, without the
 * fp32 re-check; ODC_PREC_BF16_X3 the split-bf16 evaluation of the
 * searches); for CSG fields +1 inside, -1 outside.  Synchronous.
 * Errors: INVALID_ARG, UNSUPPORTED (as for odc_mesh_extract), HIP. */
int32_t odc_field_eval(odc_context* ctx, const odc_field* field, int32_t precision,
                       const float* xyz, int64_t n, float* z);

/* Stage timing.  When enabled, odc_mesh_extract records HIP events on the
 * context stream between stages; after odc_mesh_sync, odc_get_stage_times
 * writes the device time of each stage in milliseconds:
 *  0 (a) corner labels (incl. the fp32 re-evaluation of the bf16 guard band)
 *  1 classification and scans (crossing edges, face pairs, active cells)
 *  2 compaction of the active sets
 *  3 (b) 1D points          4 (c) 2D points
 *  5 (d) partitions and vertex numbering     6 (d) normals and QEF
 *  7 (e) emission
 * *n receives the number of stages (8).  Errors: INVALID_ARG when timing is
 * off or no extract has completed; CAPACITY when cap < 8. */
int32_t odc_context_set_timing(odc_context* ctx, int32_t enable);
int32_t odc_get_stage_times(odc_context* ctx, float* ms, int32_t cap, int32_t* n);

/* ------------------------------------------------------------- serving
 * A request loop with continuous batching on the context's GPU.  The server
 * owns n_lanes extraction contexts (each with its own stream) and one device
 * arena of hbm_budget_bytes for job scratch.  A scheduler thread admits
 * queued jobs in arrival order into idle lanes as long as each job's scratch
 * footprint (bit sets over the grid plus its active-set capacity) fits in
 * the free arena, up to max_batch jobs and max_batch_corners grid corners
 * per batch (a lone job may exceed the corner limit), and launches them as
 * one batch (odc_mesh_extract_batch semantics).  Jobs arriving while other
 * batches run are admitted as lanes and arena memory free up.  A job whose
 * active sets outgrow the planned capacity is requeued at the head with the
 * capacity it needed.  The server takes the context's launch configuration
 * (e.g. after odc_autotune) at creation; the context itself stays free for
 * other use.
 *
 * Every device pointer of a submitted job (field data, output buffers) must
 * stay valid until odc_server_wait returns for its ticket.  submit, poll,
 * wait and the statistics calls may come from any host threads; destroy
 * must not overlap any other call on the server.  destroy waits for the
 * batches in flight and drops queued jobs. */
typedef struct odc_server odc_server;

/* Admission order.  FIFO: arrival order, and a job that does not fit in the
 * free arena blocks the jobs behind it.  SHORTEST: the queued job with the
 * smallest estimated work first (grid corners plus crossing-edge searches,
 * weighted by field kind), skipping jobs that do not fit; a job waiting
 * longer than age_ms goes before all others and is not skipped.  BANDED:
 * SHORTEST, and a batch also skips jobs estimated at more than `band` times
 * its first job (a batch ends with its slowest job, so small jobs are not
 * held behind large ones); aged jobs are never skipped. */
enum { ODC_SERVE_FIFO = 0, ODC_SERVE_SHORTEST = 1, ODC_SERVE_BANDED = 2 };

typedef struct {
  int64_t hbm_budget_bytes;  /* scratch arena (>= 1 MiB) */
  int32_t n_lanes;           /* batches in flight at once, 1..8; 0 = 2 */
  int32_t max_batch;         /* jobs per batch; 0 = 16 */
  int64_t max_batch_corners; /* grid corners per batch; 0 = 2^25 */
  int32_t policy;            /* ODC_SERVE_FIFO (0), ODC_SERVE_SHORTEST or ODC_SERVE_BANDED */
  float age_ms;              /* SHORTEST, BANDED: waiting time that promotes a job; 0 = 1000 */
  float band;                /* BANDED: cost ratio a batch admits (> 1); 0 = 8 */
} odc_server_config;

typedef struct {
  int32_t status;            /* odc_status of the job (CAPACITY: counts hold the sizes needed) */
  int32_t attempts;          /* launches of the job (> 1 after a scratch overflow) */
  odc_mesh_counts counts;
  double submit_ms;          /* host steady clock, ms since the server started */
  double admit_ms;           /* last admission into a lane */
  double done_ms;            /* completion seen by the scheduler */
} odc_request_result;

typedef struct {
  int64_t submitted, completed, failed; /* since the last reset */
  int64_t queued, in_flight;            /* now */
  int64_t batches;
  int64_t active_cells;                 /* summed over completed jobs */
  double p50_ms, p99_ms, mean_ms, max_ms; /* latency = done - submit, nearest rank */
  double window_s;                      /* from the reset to the last completion */
  double cells_per_s;                   /* active_cells / window_s */
  int64_t arena_bytes, arena_peak_bytes;
} odc_server_stats;

/* Errors: INVALID_ARG for a bad configuration; OUT_OF_MEMORY when the arena
 * cannot be allocated. */
int32_t odc_server_create(odc_context* ctx, const odc_server_config* cfg, odc_server** out);
void odc_server_destroy(odc_server* server);
const char* odc_server_last_error(const odc_server* server);
/* Scratch bytes a job would be admitted with. */
int32_t odc_server_footprint(odc_server* server, const odc_field* field,
                             const odc_params* params, int64_t* bytes);
/* Queues one job and returns at once.  Errors: the argument checks of
 * odc_mesh_extract; OUT_OF_MEMORY when the job's footprint exceeds the
 * whole arena. */
int32_t odc_server_submit(odc_server* server, const odc_field* field, const odc_params* params,
                          const odc_mesh_buffers* out, uint64_t* ticket);
/* *done = 1 once the job has finished (successfully or not). */
int32_t odc_server_poll(odc_server* server, uint64_t ticket, int32_t* done);
/* Blocks until the job has finished, writes its result and releases the
 * ticket.  The call's own status is INVALID_ARG for an unknown ticket; the
 * job's status is in result->status. */
int32_t odc_server_wait(odc_server* server, uint64_t ticket, odc_request_result* result);
/* Latency and throughput of the jobs submitted since the last reset. */
int32_t odc_server_get_stats(odc_server* server, odc_server_stats* stats);
int32_t odc_server_reset_stats(odc_server* server);

#ifdef __cplusplus
}
#endif
#endif
