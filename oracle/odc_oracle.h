/*
 * odc_oracle.h -- plain, slow CPU oracle for Occupancy-Based Dual Contouring
 * (Hwang & Sung, "Occupancy-Based Dual Contouring", SIGGRAPH Asia 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the GPU path: the two only
 * see the same seeded field arrays.
 *
 * Arithmetic.  Geometry after the searches (2D-point line intersection,
 * normals, QEF, intersection-free quad splitting) is binary64.  Where floating
 * point decides an integer -- an occupancy label -- the decision is taken in
 * the kernel's precision, binary32, with the operation order spelled out in
 * odc_oracle.c (the paper never fixes a precision).  For analytic (CSG) fields
 * that makes every label reproducible bit for bit.  For MLP fields the oracle
 * evaluates the network in binary64 and marks a decision a near-tie when the
 * logit lies within `mlp_tie_eps` of zero: both outcomes are then correct.
 *
 * Conventions (grid of `res` cells per axis, corners 0..res):
 *   corner (i,j,k) id = i + (N+1)(j + (N+1)k)
 *   x-edge id = i + N(j + (N+1)k); y-edges follow, id = Ex + i + (N+1)(j + Nk);
 *   z-edges follow, id = Ex + Ey + i + (N+1)(j + (N+1)k)
 *   face with normal x at (i,j,k): id = i + (N+1)(j + Nk); normal y: Fx + i + N(j + (N+1)k);
 *   normal z: Fx + Fy + i + N(j + Nk)
 *   cell id = i + N(j + Nk)
 *   cell-local corner = x + 2y + 4z; cell-local edge = 4*axis + o1 + 2*o2 with
 *   (o1,o2) the offsets along the two other axes in increasing axis order;
 *   face-local axes (u,v) = the two other axes in increasing order; face-local
 *   edges 0:(v=0,along u) 1:(v=1,along u) 2:(u=0,along v) 3:(u=1,along v).
 */
#ifndef ODC_ORACLE_H
#define ODC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FIELD_CSG = 0, ORC_FIELD_MLP = 1 };
enum { ORC_OP_UNION = 0, ORC_OP_SUBTRACT = 1, ORC_OP_INTERSECT = 2 };
enum { ORC_PRIM_SPHERE = 0, ORC_PRIM_BOX = 1, ORC_PRIM_HALFSPACE = 2 };
#define ORC_PRIM_FLOATS 20

typedef struct {
  int kind;                 /* ORC_FIELD_CSG or ORC_FIELD_MLP */
  /* CSG: n_prims records of 20 floats:
   *   [0] op  [1] type  [2..4] centre c
   *   [5..7] sphere: radius at [5]; box: half extents; halfspace: normal n
   *   [8..16] box rotation rows R (local = R (x - c)); [17..19] unused */
  const float* prims;
  int n_prims;
  /* MLP: W1[width][in], b1[width], (W_l[width][width], b_l[width]) for
   * l = 2..depth, w_out[width], b_out[1]; all binary32. */
  const float* weights;
  int in_dim, width, depth, n_bands;
  const float* spheres;     /* n_spheres x (cx, cy, cz, r) */
  int n_spheres;
  double sdf_gain, out_scale;
  double mlp_tie_eps;       /* |logit| below this is a near-tie */
} orc_field;

/* Replay of an implementation under test (staged parity).  The paper fixes
 * no precision, so where the oracle's own occupancy decision is a near-tie
 * (|logit| < mlp_tie_eps) both branches are correct; an implementation that
 * records the branch it took at every query lets the oracle follow that
 * branch there and check every other decision against it.  Orders are the
 * canonical ones above; arrays are host memory owned by the caller; any
 * array may be NULL (no trace for that stage).
 *   label_words   corner labels, bit c%32 of word c/32 (1 = inside)
 *   labels_given  1: take label_words as the corner labels without evaluating
 *                 the field (for topology from labels checked elsewhere)
 *   edge_id[n_edges]   crossing edges, ascending; edge_bits[x] bit i = the
 *                 label of bisection query i (Sec. 5.1)
 *   pair_rec[n_pairs]  face id << 1 | slot, ascending; pair_bits[2x] bit q =
 *                 the label of 2D-search query q, pair_bits[2x+1] bit q = query
 *                 q was evaluated.  q = 0 is m, then step 1's lin1 samples and
 *                 bin1 halvings, then step 2's ray towards the first 1D point
 *                 and the opposite ray, lin2 + bin2 each (Sec. 5.2, App. A.1.3);
 *                 queries past the 64th are untraced.
 *   staged        1: the 2D searches start from edge_t (the implementation's
 *                 1D points) and the QEF takes edge_t and pair_pf (its 2D
 *                 points), and with gradient normals edge_grad (its dz/dx at
 *                 each 1D point, 3 per crossing edge), instead of the
 *                 oracle's own; the outputs still hold the oracle's own 1D
 *                 and 2D points.
 * Counters (outputs, accumulated over calls): adopted = near-tie decisions
 * that took the recorded branch; mismatched = decisions away from a near-tie
 * that differ from the recorded one (a failure of the implementation);
 * unmatched = oracle elements with no trace entry (their decisions stay the
 * oracle's own). */
typedef struct {
  const uint32_t* label_words;
  int labels_given;
  int64_t n_edges;
  const int32_t* edge_id;
  const uint32_t* edge_bits;
  const float* edge_t;
  int64_t n_pairs;
  const int32_t* pair_rec;
  const uint64_t* pair_bits;
  const double* pair_pf;
  const float* edge_grad;
  int staged;
  int64_t adopted, mismatched, unmatched;
} orc_trace;

typedef struct {
  double lo[3];
  double size;              /* edge length of the cubic domain */
  int res;                  /* cells per axis */
  int iters_1d;             /* bisection steps per crossing edge */
  int lin1, bin1, lin2, bin2;
  float range1, range2;     /* line-binary ranges, in cell widths */
  double qef_tau;           /* eigenvalue truncation, relative to the largest */
  double ic_tie_tol;        /* vertex uncertainty (cell widths) for IC near-ties */
  int n_threads;            /* 0 = all */
  int ablation;             /* 0 = the method; else ORC_ABL_* bits (Table 3 baselines) */
  int clamp;                /* 1: clamp each 3D point into its cell (the method leaves it) */
  int topology_only;        /* 1: labels, crossing edges, pairs, flips, cells, partitions and
                             * vertex numbering only (no searches, 3D points or triangles) */
  orc_trace* trace;         /* NULL, or the replay above */
} orc_params;

/* Ablation baselines (Sec. 4 / Table 3), each replacing one step of the
 * method with Manifold Dual Contouring's:
 *   LINEAR_1D     1D points by Eq. 1 from psi = phi - 1/2 at the corners
 *   GRAD_NORMALS  QEF normals = the field gradient at the 1D point (Eq. 2;
 *                 MLP fields only), no 2D points
 *   MDC_SPLIT     every quad split as case 1 (no intersection-free split) */
enum { ORC_ABL_LINEAR_1D = 1, ORC_ABL_GRAD_NORMALS = 2, ORC_ABL_MDC_SPLIT = 4,
       /* with LINEAR_1D: the field's logit is a signed distance (SDF input,
        * inside where z > 0), and Eq. 1 interpolates z itself */
       ORC_ABL_SDF_INPUT = 8 };

typedef struct {
  int res;
  /* corners */
  int64_t n_corners;
  uint8_t* corner_label;    /* 1 = inside */
  uint8_t* corner_tie;
  /* crossing edges, ascending id */
  int64_t n_edges;
  int32_t* edge_id;
  double* edge_t;           /* parameter from the lower corner, in (0,1) */
  int32_t* edge_tie_step;   /* first bisection step that was a near-tie, 0 = none */
  uint32_t* edge_bits;      /* bit i: the label taken at bisection query i (as orc_trace) */
  /* face pairs, ascending (face id, slot) */
  int64_t n_pairs;
  int32_t* pair_face;
  int32_t* pair_info;       /* slot | fe_a<<4 | fe_b<<8 | flipped<<12 | (q==m)<<13 | ambiguous<<14 */
  double* pair_pf;          /* face-local (u,v) */
  uint8_t* pair_tie;        /* own decisions or an input 1D point had a near-tie */
  double* pair_sin;         /* |sin| of the angle between l1 and l2 (1 when q == m) */
  uint64_t* pair_bits;      /* per pair: labels taken, queried mask (as orc_trace) */
  int64_t n_flipped_faces;
  /* active cells, ascending id */
  int64_t n_cells;
  int32_t* cell_id;
  int32_t* cell_npart;
  int32_t* cell_partmap;    /* 2 bits per cell-local edge: partition index (crossing edges only) */
  int32_t* cell_flipmask;   /* bit lf set: local face lf uses the flipped pairing */
  int32_t* cell_vbase;
  uint8_t* cell_tie;
  /* vertices: partitions (cells ascending, partitions in order), then case-3 */
  int64_t n_vertices;
  double* vert;             /* grid units */
  uint8_t* vert_tie;
  double* vert_kappa;       /* largest/smallest eigenvalue of the normal matrix */
  double* vert_gap;         /* smallest (kept - dropped) eigenvalue gap / largest; inf if none dropped */
  /* emission, one entry per crossing edge */
  int32_t* edge_case;       /* 0 = no quad (grid boundary), 1, 2, 3 */
  uint8_t* edge_case_tie;
  int64_t n_case3;
  int64_t n_tris;
  int32_t* tris;
} orc_mesh;

/* Near-tie flags (corner_tie, edge_tie_step, pair_tie, cell_tie, vert_tie,
 * edge_case_tie) mark decisions the oracle could not fix: with a trace, a
 * near-tie that took the recorded branch is fixed and not flagged.
 * Full pipeline.  Returns 0 on success, <0 on invalid input. */
int orc_mesh_extract(const orc_field* f, const orc_params* p, orc_mesh* out);
void orc_mesh_free(orc_mesh* m);

/* Single-element entry points used for sampled checks on large grids.  Each
 * recomputes what it needs from the field alone. */
int orc_label_world(const orc_field* f, const float xyz[3], int* tie, double* margin);
int orc_corner_label(const orc_field* f, const orc_params* p, int i, int j, int k, int* tie);
/* t of a crossing edge; returns -1 if the edge does not cross. */
double orc_edge_point(const orc_field* f, const orc_params* p, int64_t edge_id, int* tie_step);
/* 2D point of pair `slot` on face `face_id` (after the manifold flip).
 * Returns the number of pairs on the face, or -1 if slot is out of range. */
int orc_pair_point(const orc_field* f, const orc_params* p, int64_t face_id, int slot,
                   double pf[2], int* info, int* tie);
/* Vertices of one cell: returns the partition count (0 if inactive);
 * verts receives up to 4 grid-unit points, partmap the edge map. */
int orc_cell_vertices(const orc_field* f, const orc_params* p, int64_t cell_id,
                      double* verts, int* partmap, int* tie, double* kappa);

/* Building blocks exposed for pinning tests. */
/* Logit z and its gradient dz/dx at a binary64 point of an MLP field (NAN
 * for other fields).  margin (may be NULL) receives the distance to a switch
 * of the gradient's formula: [0] the gap between the two nearest spheres'
 * distances, [1] the smallest |pre-activation| of any ReLU. */
double orc_logit_grad(const orc_field* f, const double x[3], double grad[3], double margin[2]);
/* Line-binary search along a face-local ray on face `face_id` (FP32 ray
 * geometry as in the search).  Returns the near parameter s; q receives the point. */
float orc_line_binary(const orc_field* f, const orc_params* p, int64_t face_id,
                      const float p0[2], const float dir[2], int s0,
                      float range, int n_lin, int n_bin, float q[2], int* tie);
/* Partitions of a cube configuration (bit c = label of cell-local corner c)
 * with a face-flip mask: returns the partition count and fills partmap
 * (2 bits per cell-local edge, meaningful for crossing edges only). */
int orc_cube_partitions(int config, int flipmask, int* partmap);
/* Truncated pseudo-inverse QEF: n planes (normal, point) in rows of 6. */
void orc_qef_solve(int n, const double* planes, double tau, double out[3], double* kappa);
/* Self-intersections: the number of pairs of triangles sharing no vertex
 * whose closed triangles intersect (brute force over all pairs). */
int64_t orc_self_intersections(const float* vertices, int64_t n_vertices, const int32_t* tris,
                               int64_t n_tris);
/* Intersection-free split of an oriented quad; returns case 1..3. */
int orc_ic_case(const double q[4][3], const double pin[3], const double pout[3],
                double tol, int* tie);

#ifdef __cplusplus
}
#endif
#endif
