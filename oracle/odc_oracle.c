/*
 * odc_oracle.c -- plain CPU oracle for Occupancy-Based Dual Contouring.
 *
 * TEST INFRASTRUCTURE ONLY (see odc_oracle.h).  Written for a reader holding
 * the paper: every step names the section it follows.  No blocking, fusion or
 * reordering beyond what the method states; loops are the obvious ones.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math (x86-64 SSE, so
 * every float operation below is one IEEE binary32 operation).
 */
#include "odc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Grid indexing (problem statement, Sec. 3: vertices, edges, cells).       */
/* ------------------------------------------------------------------------ */

static void other_axes(int a, int* b1, int* b2) {
  if (a == 0) { *b1 = 1; *b2 = 2; }
  else if (a == 1) { *b1 = 0; *b2 = 2; }
  else { *b1 = 0; *b2 = 1; }
}

static int64_t corner_id(int N, int i, int j, int k) {
  return (int64_t)i + (int64_t)(N + 1) * ((int64_t)j + (int64_t)(N + 1) * k);
}

static int64_t edges_per_axis(int N) { return (int64_t)N * (N + 1) * (N + 1); }
static int64_t faces_per_axis(int N) { return (int64_t)(N + 1) * N * N; }

/* edge of axis a starting at corner pos[] */
static int64_t edge_id(int N, int a, const int pos[3]) {
  int64_t E = edges_per_axis(N);
  if (a == 0) return pos[0] + (int64_t)N * (pos[1] + (int64_t)(N + 1) * pos[2]);
  if (a == 1) return E + pos[0] + (int64_t)(N + 1) * (pos[1] + (int64_t)N * pos[2]);
  return 2 * E + pos[0] + (int64_t)(N + 1) * (pos[1] + (int64_t)(N + 1) * pos[2]);
}

static void edge_decode(int N, int64_t id, int* a, int pos[3]) {
  int64_t E = edges_per_axis(N);
  *a = (int)(id / E);
  int64_t r = id - (int64_t)(*a) * E;
  int nx = (*a == 0) ? N : N + 1;
  int ny = (*a == 1) ? N : N + 1;
  pos[0] = (int)(r % nx);
  r /= nx;
  pos[1] = (int)(r % ny);
  pos[2] = (int)(r / ny);
}

/* face with normal a at min corner pos[] */
static int64_t face_id(int N, int a, const int pos[3]) {
  int64_t F = faces_per_axis(N);
  if (a == 0) return pos[0] + (int64_t)(N + 1) * (pos[1] + (int64_t)N * pos[2]);
  if (a == 1) return F + pos[0] + (int64_t)N * (pos[1] + (int64_t)(N + 1) * pos[2]);
  return 2 * F + pos[0] + (int64_t)N * (pos[1] + (int64_t)N * pos[2]);
}

static void face_decode(int N, int64_t id, int* a, int pos[3]) {
  int64_t F = faces_per_axis(N);
  *a = (int)(id / F);
  int64_t r = id - (int64_t)(*a) * F;
  int nx = (*a == 0) ? N + 1 : N;
  int ny = (*a == 1) ? N + 1 : N;
  pos[0] = (int)(r % nx);
  r /= nx;
  pos[1] = (int)(r % ny);
  pos[2] = (int)(r / ny);
}

static int64_t cell_id(int N, int i, int j, int k) {
  return (int64_t)i + (int64_t)N * ((int64_t)j + (int64_t)N * k);
}

/* ------------------------------------------------------------------------ */
/* Occupancy phi' (Sec. 3; binarisation of App. A.2.2).                     */
/* ------------------------------------------------------------------------ */

/* World position of a grid-unit point, binary32: x = lo + g*h (two ops). */
static void grid_to_world(const orc_params* p, const float g[3], float x[3]) {
  float h = (float)(p->size / (double)p->res);
  for (int a = 0; a < 3; ++a) {
    float lo = (float)p->lo[a];
    float gh = g[a] * h;
    x[a] = lo + gh;
  }
}

/* One CSG primitive, binary32, operation order fixed. */
static int prim_inside(const float* pr, const float x[3]) {
  int type = (int)pr[1];
  float dx = x[0] - pr[2];
  float dy = x[1] - pr[3];
  float dz = x[2] - pr[4];
  if (type == ORC_PRIM_SPHERE) {
    float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    float d2 = (xx + yy) + zz;
    float r2 = pr[5] * pr[5];
    return d2 < r2;
  }
  if (type == ORC_PRIM_BOX) {
    for (int a = 0; a < 3; ++a) {
      const float* R = pr + 8 + 3 * a;
      float t0 = R[0] * dx, t1 = R[1] * dy, t2 = R[2] * dz;
      float l = (t0 + t1) + t2;
      if (!(fabsf(l) < pr[5 + a])) return 0;
    }
    return 1;
  }
  /* half-space through c with outward normal n: inside where n.(x-c) < 0 */
  {
    float t0 = pr[5] * dx, t1 = pr[6] * dy, t2 = pr[7] * dz;
    float v = (t0 + t1) + t2;
    return v < 0.0f;
  }
}

/* Left fold of the primitive list: ((p0 op1 p1) op2 p2) ... */
static int csg_label(const orc_field* f, const float x[3]) {
  int acc = prim_inside(f->prims, x);
  for (int i = 1; i < f->n_prims; ++i) {
    const float* pr = f->prims + (size_t)ORC_PRIM_FLOATS * i;
    int b = prim_inside(pr, x);
    int op = (int)pr[0];
    if (op == ORC_OP_UNION) acc = acc || b;
    else if (op == ORC_OP_SUBTRACT) acc = acc && !b;
    else acc = acc && b;
  }
  return acc;
}

/* Logit z(x) of an MLP field (App. B network: gamma, depth ReLU layers, a
 * linear output; then the sdf term), in binary64 at a binary64 point.
 *   z = out_scale * y(gamma(x)) - sdf_gain * sdf(x)
 * gamma(x) = (x, sin(2^k pi x), cos(2^k pi x)), k = 0..n_bands-1,
 * sdf = min over spheres of (|x - c| - r).
 * With grad != NULL also dz/dx by reverse-mode differentiation: the ReLU's
 * derivative is 0 where its input is <= 0 (the forward pass keeps exactly
 * the positive inputs), and the sdf term differentiates through its nearest
 * sphere (the first in index order on a tie). */
static double mlp_eval_m(const orc_field* f, const double x[3], double grad[3], double margin[2]);
static double mlp_eval(const orc_field* f, const double x[3], double grad[3]) {
  return mlp_eval_m(f, x, grad, NULL);
}

/* As mlp_eval; margin (if not NULL) receives how far the gradient is from a
 * switch: [0] the gap between the two nearest spheres' distances, [1] the
 * smallest |pre-activation| of any ReLU. */
static double mlp_eval_m(const orc_field* f, const double x[3], double grad[3], double margin[2]) {
  const int in = f->in_dim, W = f->width, D = f->depth;
  double* act = (double*)malloc(sizeof(double) * ((size_t)in + (size_t)D * W));
  double* pre = (double*)malloc(sizeof(double) * (size_t)D * W);
  for (int a = 0; a < 3; ++a) act[a] = x[a];
  for (int k = 0; k < f->n_bands; ++k) {
    double s = ldexp(1.0, k);
    for (int a = 0; a < 3; ++a) {
      act[3 + 6 * k + a] = sin(M_PI * (s * x[a]));
      act[3 + 6 * k + 3 + a] = cos(M_PI * (s * x[a]));
    }
  }
  /* layer l reads its input at act + off_in[l] and writes its output after it */
  const float* w = f->weights;
  const float* Wl_of[64];
  size_t off = 0;
  int n_in = in;
  for (int l = 0; l < D; ++l) {
    const float* Wl = w;
    const float* bl = w + (size_t)W * n_in;
    Wl_of[l] = Wl;
    double* hin = act + off;
    double* hout = act + off + n_in;
    for (int j = 0; j < W; ++j) {
      double acc = bl[j];
      for (int i = 0; i < n_in; ++i) acc += (double)Wl[(size_t)j * n_in + i] * hin[i];
      pre[(size_t)l * W + j] = acc;
      hout[j] = acc > 0.0 ? acc : 0.0;
    }
    w = bl + W;
    off += n_in;
    n_in = W;
  }
  const double* hlast = act + off;
  double y = w[W];
  for (int i = 0; i < W; ++i) y += (double)w[i] * hlast[i];
  double sdf = INFINITY, sdf2 = INFINITY, dnear[3] = {0, 0, 0}, rnear = 0.0;
  for (int s = 0; s < f->n_spheres; ++s) {
    const float* sp = f->spheres + 4 * s;
    double dx = x[0] - sp[0], dy = x[1] - sp[1], dz = x[2] - sp[2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double d = r - sp[3];
    if (d >= sdf && d < sdf2) sdf2 = d;
    if (d < sdf) {
      sdf2 = sdf;
      sdf = d;
      dnear[0] = dx;
      dnear[1] = dy;
      dnear[2] = dz;
      rnear = r;
    }
  }
  if (margin) {
    margin[0] = sdf2 - sdf;
    double mp = INFINITY;
    for (size_t i = 0; i < (size_t)D * W; ++i) mp = fmin(mp, fabs(pre[i]));
    margin[1] = mp;
  }
  if (grad) {
    /* g = dz/d(pre-activation) of the current layer, walked down */
    double* g = (double*)malloc(sizeof(double) * (size_t)(W > in ? W : in));
    double* gn = (double*)malloc(sizeof(double) * (size_t)(W > in ? W : in));
    for (int j = 0; j < W; ++j)
      g[j] = pre[(size_t)(D - 1) * W + j] > 0.0 ? f->out_scale * (double)w[j] : 0.0;
    for (int l = D - 1; l >= 0; --l) {
      const int ni = l == 0 ? in : W;
      for (int i = 0; i < ni; ++i) {
        double acc = 0.0;
        for (int j = 0; j < W; ++j) acc += (double)Wl_of[l][(size_t)j * ni + i] * g[j];
        gn[i] = acc;
      }
      if (l > 0)
        for (int i = 0; i < W; ++i) g[i] = pre[(size_t)(l - 1) * W + i] > 0.0 ? gn[i] : 0.0;
    }
    /* gn = dz/dgamma; chain through gamma */
    for (int a = 0; a < 3; ++a) {
      double d = gn[a];
      for (int k = 0; k < f->n_bands; ++k) {
        double s = ldexp(1.0, k);
        d += gn[3 + 6 * k + a] * M_PI * s * cos(M_PI * (s * x[a]));
        d -= gn[3 + 6 * k + 3 + a] * M_PI * s * sin(M_PI * (s * x[a]));
      }
      if (rnear > 0.0) d -= f->sdf_gain * dnear[a] / rnear;
      grad[a] = d;
    }
    free(g);
    free(gn);
  }
  free(act);
  free(pre);
  return f->out_scale * y - f->sdf_gain * sdf;
}

static double mlp_logit(const orc_field* f, const float xf[3]) {
  double x[3] = {xf[0], xf[1], xf[2]};
  return mlp_eval(f, x, NULL);
}

double orc_logit_grad(const orc_field* f, const double x[3], double grad[3], double margin[2]) {
  if (f->kind != ORC_FIELD_MLP || f->depth > 64) return NAN;
  return mlp_eval_m(f, x, grad, margin);
}

int orc_label_world(const orc_field* f, const float xyz[3], int* tie, double* margin) {
  if (f->kind == ORC_FIELD_CSG) {
    if (tie) *tie = 0;
    if (margin) *margin = INFINITY;
    return csg_label(f, xyz);
  }
  double z = mlp_logit(f, xyz);
  if (tie) *tie = fabs(z) < f->mlp_tie_eps;
  if (margin) *margin = z;
  return z > 0.0; /* phi > 0.5, strict */
}

static int label_grid(const orc_field* f, const orc_params* p, const float g[3], int* tie) {
  float x[3];
  grid_to_world(p, g, x);
  return orc_label_world(f, x, tie, NULL);
}

/* ------------------------------------------------------------------------ */
/* Replay of an implementation under test (see orc_trace).                  */
/* ------------------------------------------------------------------------ */

/* One decision: the oracle's own label `own` (*tie set when it is a
 * near-tie) against the recorded label `theirs` when `have`.  A near-tie
 * follows the recorded branch and is then fixed (*tie cleared); any other
 * decision stays the oracle's and a disagreement is counted. */
static int decide(orc_trace* tr, int own, int* tie, int have, int theirs) {
  if (!tr || !have) return own;
  if (*tie) {
    *tie = 0;
#pragma omp atomic
    tr->adopted += 1;
    return theirs;
  }
  if (own != theirs) {
#pragma omp atomic
    tr->mismatched += 1;
  }
  return own;
}

static void count_unmatched(orc_trace* tr) {
#pragma omp atomic
  tr->unmatched += 1;
}

/* index of v in the ascending array a[n], or -1 */
static int64_t find_sorted(const int32_t* a, int64_t n, int64_t v) {
  int64_t lo = 0, hi = n - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (a[mid] == v) return mid;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

/* the implementation's slot of crossing edge eid, or -1 */
static int64_t trace_edge_slot(const orc_trace* tr, int64_t eid) {
  if (!tr || !tr->edge_id) return -1;
  return find_sorted(tr->edge_id, tr->n_edges, eid);
}

/* the implementation's slot of pair `slot` of face fid, or -1 */
static int64_t trace_pair_slot(const orc_trace* tr, int64_t fid, int slot) {
  if (!tr || !tr->pair_rec) return -1;
  return find_sorted(tr->pair_rec, tr->n_pairs, fid * 2 + slot);
}

int orc_corner_label(const orc_field* f, const orc_params* p, int i, int j, int k, int* tie) {
  orc_trace* tr = p->trace;
  int64_t c = corner_id(p->res, i, j, k);
  int theirs = tr && tr->label_words ? (int)((tr->label_words[c >> 5] >> (c & 31)) & 1u) : 0;
  if (tr && tr->label_words && tr->labels_given) {
    if (tie) *tie = 0;
    return theirs;
  }
  float g[3] = {(float)i, (float)j, (float)k};
  int t = 0;
  int lab = label_grid(f, p, g, &t);
  lab = decide(tr, lab, &t, tr && tr->label_words, theirs);
  if (tie) *tie = t;
  return lab;
}

/* ------------------------------------------------------------------------ */
/* 1D point: binary search on a crossing edge (Sec. 5.1).                  */
/* The bracket [a,b] keeps distinct end labels; after `iters` halvings the   */
/* point is the middle of the final bracket.                                */
/* ------------------------------------------------------------------------ */

static double bisect_edge(const orc_field* f, const orc_params* p, int a, const int pos[3],
                          int label0, int* tie_step, uint32_t* own_bits) {
  double lo_t = 0.0, hi_t = 1.0;
  *tie_step = 0;
  if (own_bits) *own_bits = 0u;
  /* the implementation's recorded labels for this edge, when replaying */
  orc_trace* tr = p->trace;
  const uint32_t* rec = NULL;
  if (tr && tr->edge_bits) {
    int64_t x = trace_edge_slot(tr, edge_id(p->res, a, pos));
    if (x >= 0) rec = tr->edge_bits + x;
    else count_unmatched(tr);
  }
  for (int it = 1; it <= p->iters_1d; ++it) {
    double mid = 0.5 * (lo_t + hi_t);
    float g[3] = {(float)pos[0], (float)pos[1], (float)pos[2]};
    float fm = (float)mid;
    g[a] = (float)pos[a] + fm;
    int tie = 0;
    int lab = label_grid(f, p, g, &tie);
    lab = decide(tr, lab, &tie, rec != NULL, rec ? (int)((*rec >> (it - 1)) & 1u) : 0);
    if (own_bits) *own_bits |= (uint32_t)lab << (it - 1);
    if (tie && *tie_step == 0) *tie_step = it;
    if (lab == label0) lo_t = mid;
    else hi_t = mid;
  }
  return 0.5 * (lo_t + hi_t);
}

/* MDC's 1D point (Eq. 1) from continuous occupancy, the ablation baseline:
 * psi = phi - 1/2 at the edge's two corners, written psi = tanh(z/2)/2 for
 * phi = sigmoid(z) (the same number, without the cancellation near 1/2), and
 * t = psi(lower) / (psi(lower) - psi(upper)).  A CSG field's occupancy is
 * the label itself, so t = 1/2. */
static double linear_edge(const orc_field* f, const orc_params* p, int a, const int pos[3]) {
  int up[3] = {pos[0], pos[1], pos[2]};
  up[a] += 1;
  double psi[2];
  for (int e = 0; e < 2; ++e) {
    const int* q = e == 0 ? pos : up;
    if (f->kind == ORC_FIELD_CSG) {
      psi[e] = orc_corner_label(f, p, q[0], q[1], q[2], NULL) - 0.5;
    } else {
      float g[3] = {(float)q[0], (float)q[1], (float)q[2]}, x[3];
      grid_to_world(p, g, x);
      const double z = mlp_logit(f, x);
      psi[e] = (p->ablation & ORC_ABL_SDF_INPUT) ? z : 0.5 * tanh(0.5 * z);
    }
  }
  return psi[0] / (psi[0] - psi[1]);
}

static double edge_point_mode(const orc_field* f, const orc_params* p, int a, const int pos[3],
                              int label0, int* tie_step, uint32_t* own_bits) {
  if (p->ablation & ORC_ABL_LINEAR_1D) {
    *tie_step = 0;
    return linear_edge(f, p, a, pos);
  }
  return bisect_edge(f, p, a, pos, label0, tie_step, own_bits);
}

double orc_edge_point(const orc_field* f, const orc_params* p, int64_t eid, int* tie_step) {
  int N = p->res, a, pos[3];
  edge_decode(N, eid, &a, pos);
  int up[3] = {pos[0], pos[1], pos[2]};
  up[a] += 1;
  int l0 = orc_corner_label(f, p, pos[0], pos[1], pos[2], NULL);
  int l1 = orc_corner_label(f, p, up[0], up[1], up[2], NULL);
  if (l0 == l1) return -1.0;
  return edge_point_mode(f, p, a, pos, l0, tie_step, NULL);
}

/* ------------------------------------------------------------------------ */
/* Faces: crossing edges and their pairing (App. A.1.1).                    */
/* ------------------------------------------------------------------------ */

/* face-local corner lc = bu + 2 bv; face-local edges:
 * 0: lc0-lc1 (v=0), 1: lc2-lc3 (v=1), 2: lc0-lc2 (u=0), 3: lc1-lc3 (u=1) */
static const int FE_CORNERS[4][2] = {{0, 1}, {2, 3}, {0, 2}, {1, 3}};

/* Pairs of crossing face-local edges.  Two crossings: one pair.  Four
 * crossings (diagonal corners equal): one pair around each inside corner,
 * or around each outside corner when `flipped`.  Returns the pair count;
 * pairs are ordered by their first edge. */
static int face_pairs(const int L[4], int flipped, int pairs[2][2]) {
  int cross[4], n = 0;
  for (int e = 0; e < 4; ++e) {
    cross[e] = L[FE_CORNERS[e][0]] != L[FE_CORNERS[e][1]];
    n += cross[e];
  }
  if (n == 0) return 0;
  if (n == 2) {
    int k = 0;
    for (int e = 0; e < 4; ++e)
      if (cross[e]) pairs[0][k++] = e;
    return 1;
  }
  /* corner 0 touches edges 0,2; corner 3 touches 1,3; corner 1: 0,3; corner 2: 1,2 */
  int around_03 = (L[0] == 1) != (flipped != 0);
  if (around_03) {
    pairs[0][0] = 0; pairs[0][1] = 2;
    pairs[1][0] = 1; pairs[1][1] = 3;
  } else {
    pairs[0][0] = 0; pairs[0][1] = 3;
    pairs[1][0] = 1; pairs[1][1] = 2;
  }
  return 2;
}

/* Geometry of a global face: normal a, min corner pos, face-local axes u,v. */
typedef struct {
  int a, u, v;
  int pos[3];
} face_geom;

static face_geom face_geometry(int N, int64_t fid) {
  face_geom g;
  face_decode(N, fid, &g.a, g.pos);
  other_axes(g.a, &g.u, &g.v);
  return g;
}

static void face_corner_pos(const face_geom* g, int lc, int out[3]) {
  out[0] = g->pos[0]; out[1] = g->pos[1]; out[2] = g->pos[2];
  out[g->u] += lc & 1;
  out[g->v] += (lc >> 1) & 1;
}

static int64_t face_edge_global(int N, const face_geom* g, int fe) {
  int pos[3] = {g->pos[0], g->pos[1], g->pos[2]};
  int axis;
  if (fe == 0) axis = g->u;
  else if (fe == 1) { axis = g->u; pos[g->v] += 1; }
  else if (fe == 2) axis = g->v;
  else { axis = g->v; pos[g->u] += 1; }
  return edge_id(N, axis, pos);
}

/* Face-local position of the 1D point of face-local edge fe with parameter t. */
static void face_edge_point(int fe, float t, float P[2]) {
  if (fe == 0) { P[0] = t; P[1] = 0.0f; }
  else if (fe == 1) { P[0] = t; P[1] = 1.0f; }
  else if (fe == 2) { P[0] = 0.0f; P[1] = t; }
  else { P[0] = 1.0f; P[1] = t; }
}

/* ------------------------------------------------------------------------ */
/* Cube partitions: cycles of the face-pair graph (App. A.1.1, Fig. A1).    */
/* ------------------------------------------------------------------------ */

static int cell_local_edge(int axis, const int off[3]) {
  int b1, b2;
  other_axes(axis, &b1, &b2);
  return 4 * axis + off[b1] + 2 * off[b2];
}

/* cell-local edge of face-local edge fe on local face (normal a, side s) */
static int face_edge_to_cell_edge(int a, int s, int fe) {
  int u, v, off[3] = {0, 0, 0}, axis;
  other_axes(a, &u, &v);
  off[a] = s;
  if (fe == 0) { axis = u; off[v] = 0; }
  else if (fe == 1) { axis = u; off[v] = 1; }
  else if (fe == 2) { axis = v; off[u] = 0; }
  else { axis = v; off[u] = 1; }
  return cell_local_edge(axis, off);
}

/* labels of the face-local corners of local face (a, s) in a cube config */
static void face_labels_from_config(int config, int a, int s, int L[4]) {
  int u, v;
  other_axes(a, &u, &v);
  for (int lc = 0; lc < 4; ++lc) {
    int off[3] = {0, 0, 0};
    off[a] = s;
    off[u] = lc & 1;
    off[v] = (lc >> 1) & 1;
    int c = off[0] + 2 * off[1] + 4 * off[2];
    L[lc] = (config >> c) & 1;
  }
}

static int edge_crosses_config(int config, int le) {
  int axis = le / 4, b1, b2, off[3] = {0, 0, 0};
  other_axes(axis, &b1, &b2);
  off[b1] = le & 1;
  off[b2] = (le >> 1) & 1;
  int c0 = off[0] + 2 * off[1] + 4 * off[2];
  off[axis] = 1;
  int c1 = off[0] + 2 * off[1] + 4 * off[2];
  return ((config >> c0) & 1) != ((config >> c1) & 1);
}

int orc_cube_partitions(int config, int flipmask, int* partmap_out) {
  int nb[12][2], deg[12];
  for (int e = 0; e < 12; ++e) { deg[e] = 0; nb[e][0] = nb[e][1] = -1; }
  for (int lf = 0; lf < 6; ++lf) {
    int a = lf / 2, s = lf % 2, L[4], pairs[2][2];
    face_labels_from_config(config, a, s, L);
    int np = face_pairs(L, (flipmask >> lf) & 1, pairs);
    for (int q = 0; q < np; ++q) {
      int e0 = face_edge_to_cell_edge(a, s, pairs[q][0]);
      int e1 = face_edge_to_cell_edge(a, s, pairs[q][1]);
      nb[e0][deg[e0]++] = e1;
      nb[e1][deg[e1]++] = e0;
    }
  }
  int part[12], npart = 0;
  for (int e = 0; e < 12; ++e) part[e] = -1;
  for (int e = 0; e < 12; ++e) {
    if (!edge_crosses_config(config, e) || part[e] >= 0) continue;
    /* walk the cycle through e; e is its smallest edge since lower ones are done */
    int cur = e;
    while (cur >= 0 && part[cur] < 0) {
      part[cur] = npart;
      int nxt = -1;
      for (int q = 0; q < deg[cur]; ++q)
        if (part[nb[cur][q]] < 0) { nxt = nb[cur][q]; break; }
      cur = nxt;
    }
    ++npart;
  }
  int pm = 0;
  for (int e = 0; e < 12; ++e)
    if (part[e] >= 0) pm |= (part[e] & 3) << (2 * e);
  if (partmap_out) *partmap_out = pm;
  return npart;
}

/* ------------------------------------------------------------------------ */
/* Manifold fix (App. A.1.1): an ambiguous face shared by two cells whose   */
/* plain partitions both merge its two pairs would make one dual edge carry */
/* four quads; such a face takes the other pairing in both cells.           */
/* ------------------------------------------------------------------------ */

static int cell_config(const orc_field* f, const orc_params* p, const uint8_t* labels,
                       const int c[3]) {
  int N = p->res, cfg = 0;
  for (int lc = 0; lc < 8; ++lc) {
    int i = c[0] + (lc & 1), j = c[1] + ((lc >> 1) & 1), k = c[2] + ((lc >> 2) & 1);
    int lab = labels ? labels[corner_id(N, i, j, k)] : orc_corner_label(f, p, i, j, k, NULL);
    cfg |= lab << lc;
  }
  return cfg;
}

static void face_labels_global(const orc_field* f, const orc_params* p, const uint8_t* labels,
                               const face_geom* g, int L[4]) {
  for (int lc = 0; lc < 4; ++lc) {
    int c[3];
    face_corner_pos(g, lc, c);
    L[lc] = labels ? labels[corner_id(p->res, c[0], c[1], c[2])]
                   : orc_corner_label(f, p, c[0], c[1], c[2], NULL);
  }
}

/* 1 if the ambiguous face takes the flipped pairing. */
static int face_flip(const orc_field* f, const orc_params* p, const uint8_t* labels,
                     const face_geom* g) {
  int N = p->res;
  if (g->pos[g->a] <= 0 || g->pos[g->a] >= N) return 0; /* only one cell */
  int L[4], pairs[2][2];
  face_labels_global(f, p, labels, g, L);
  if (face_pairs(L, 0, pairs) != 2) return 0;
  int merged_both = 1;
  for (int side = 0; side < 2; ++side) {
    /* side 0: the cell below (face is its side 1); side 1: the cell above */
    int c[3] = {g->pos[0], g->pos[1], g->pos[2]};
    int s_in_cell = 1;
    if (side == 0) c[g->a] -= 1;
    else s_in_cell = 0;
    int cfg = cell_config(f, p, labels, c), pm;
    orc_cube_partitions(cfg, 0, &pm);
    int e0 = face_edge_to_cell_edge(g->a, s_in_cell, pairs[0][0]);
    int e1 = face_edge_to_cell_edge(g->a, s_in_cell, pairs[1][0]);
    int p0 = (pm >> (2 * e0)) & 3, p1 = (pm >> (2 * e1)) & 3;
    if (p0 != p1) merged_both = 0;
  }
  return merged_both;
}

/* ------------------------------------------------------------------------ */
/* 2D point search (Sec. 5.2; line-binary search App. A.1.3; parameters     */
/* App. A.1.4).  Ray geometry and query points are binary32 so that both    */
/* implementations query the same points; the final intersection is        */
/* binary64.                                                                 */
/* ------------------------------------------------------------------------ */

static int label_face_point(const orc_field* f, const orc_params* p, const face_geom* g,
                            const float P[2], int* tie) {
  float gp[3];
  gp[g->a] = (float)g->pos[g->a];
  gp[g->u] = (float)g->pos[g->u] + P[0];
  gp[g->v] = (float)g->pos[g->v] + P[1];
  return label_grid(f, p, gp, tie);
}

static void ray_point(const float p0[2], const float d[2], float s, float out[2]) {
  float su = s * d[0], sv = s * d[1];
  out[0] = p0[0] + su;
  out[1] = p0[1] + sv;
}

/* Samples p_i = p0 + (R i / N) d, i = 1..N; the first i whose label differs
 * from s0 (or N if none) bounds [p_{i-1}, p_i]; then n_bin halvings compare
 * the middle with the near end.  Returns the near parameter. */
/* A recorded 2D search (replay): its two trace words and the index of this
 * search's first query in them. */
typedef struct {
  const uint64_t* w; /* [0] labels, [1] evaluated mask; NULL when not replaying */
  int q0;
  uint64_t own[2];   /* the oracle's own decisions, in the same encoding */
} pair_rec_t;

static int recorded(const pair_rec_t* r, int q, int* theirs) {
  if (!r || !r->w || q >= 64 || !((r->w[1] >> q) & 1u)) return 0;
  *theirs = (int)((r->w[0] >> q) & 1u);
  return 1;
}

static void record_own(pair_rec_t* r, int q, int lab) {
  if (!r || q >= 64) return;
  r->own[0] |= (uint64_t)lab << q;
  r->own[1] |= 1ull << q;
}

static float line_binary(const orc_field* f, const orc_params* p, const face_geom* g,
                         const float p0[2], const float d[2], int s0, float R, int n_lin,
                         int n_bin, float q[2], int* tie_any, pair_rec_t* rec) {
  int istar = n_lin, found = 0, theirs = 0, have;
  for (int i = 1; i <= n_lin; ++i) {
    float s = (R * (float)i) / (float)n_lin;
    float P[2];
    ray_point(p0, d, s, P);
    int tie = 0;
    int lab = label_face_point(f, p, g, P, &tie);
    have = recorded(rec, rec ? rec->q0 + i - 1 : 0, &theirs);
    lab = decide(p->trace, lab, &tie, have, theirs);
    record_own(rec, rec ? rec->q0 + i - 1 : 0, lab);
    /* samples after the first label change cannot move the bracket */
    if (tie && !found) *tie_any = 1;
    if (lab != s0 && !found) { istar = i; found = 1; }
  }
  float near_s = (istar == 1) ? 0.0f : (R * (float)(istar - 1)) / (float)n_lin;
  float far_s = (R * (float)istar) / (float)n_lin;
  for (int it = 0; it < n_bin; ++it) {
    float mid = (near_s + far_s) * 0.5f;
    float P[2];
    ray_point(p0, d, mid, P);
    int tie = 0;
    int lab = label_face_point(f, p, g, P, &tie);
    have = recorded(rec, rec ? rec->q0 + n_lin + it : 0, &theirs);
    lab = decide(p->trace, lab, &tie, have, theirs);
    record_own(rec, rec ? rec->q0 + n_lin + it : 0, lab);
    if (tie) *tie_any = 1;
    if (lab == s0) near_s = mid;
    else far_s = mid;
  }
  ray_point(p0, d, near_s, q);
  return near_s;
}

float orc_line_binary(const orc_field* f, const orc_params* p, int64_t fid, const float p0[2],
                      const float dir[2], int s0, float range, int n_lin, int n_bin, float q[2],
                      int* tie) {
  face_geom g = face_geometry(p->res, fid);
  int t = 0;
  float s = line_binary(f, p, &g, p0, dir, s0, range, n_lin, n_bin, q, &t, NULL);
  if (tie) *tie = t;
  return s;
}

/* Exact side of corner c relative to the directed line P1->P2: sign of the
 * cross product, evaluated in binary64 where the inputs are exact. */
static int corner_side_left(const float P1[2], const float P2[2], int lc) {
  double cu = lc & 1, cv = (lc >> 1) & 1;
  double du = (double)P2[0] - P1[0], dv = (double)P2[1] - P1[1];
  double cr = du * (cv - P1[1]) - dv * (cu - P1[0]);
  return cr > 0.0;
}

typedef struct {
  double pf[2];
  int qm;        /* q coincided with m */
  int tie;
  uint64_t bits[2]; /* the decisions taken: labels, queried mask (as a trace) */
  double sinang; /* |sin| of the angle between l1 and l2 */
} pair_result;

/* The three steps of Sec. 5.2 for the pair (P1 on fe_a, P2 on fe_b). */
static pair_result search_pair(const orc_field* f, const orc_params* p, const face_geom* g,
                               const int L[4], const float P1[2], const float P2[2],
                               const uint64_t* trace_words) {
  pair_result r;
  int tie_any = 0, tie = 0, theirs = 0;
  pair_rec_t rec = {trace_words, 0, {0, 0}};
  /* Step 1: m, its label, and the ray from m orthogonal to l. */
  float m[2] = {(P1[0] + P2[0]) * 0.5f, (P1[1] + P2[1]) * 0.5f};
  int sm = label_face_point(f, p, g, m, &tie);
  int have = recorded(&rec, 0, &theirs);
  sm = decide(p->trace, sm, &tie, have, theirs);
  record_own(&rec, 0, sm);
  if (tie) tie_any = 1;
  float du = P2[0] - P1[0], dv = P2[1] - P1[1];
  float len = sqrtf(du * du + dv * dv);
  float perp[2] = {-dv / len, du / len}; /* points to the left of P1->P2 */
  int nleft = 0, nright = 0, dleft = 0, dright = 0;
  for (int lc = 0; lc < 4; ++lc) {
    int left = corner_side_left(P1, P2, lc);
    if (left) { ++nleft; if (L[lc] != sm) dleft = 1; }
    else { ++nright; if (L[lc] != sm) dright = 1; }
  }
  int go_left;
  if (dleft && !dright) go_left = 1;
  else if (dright && !dleft) go_left = 0;
  else go_left = nleft <= nright; /* both qualify: the cut-off corner's side */
  float d[2] = {go_left ? perp[0] : -perp[0], go_left ? perp[1] : -perp[1]};
  float q[2];
  rec.q0 = 1;
  float s1 = line_binary(f, p, g, m, d, sm, p->range1, p->lin1, p->bin1, q, &tie_any, &rec);
  if (s1 == 0.0f) {
    r.pf[0] = m[0]; r.pf[1] = m[1];
    r.qm = 1; r.tie = tie_any; r.sinang = 1.0;
    r.bits[0] = rec.own[0]; r.bits[1] = rec.own[1];
    return r;
  }
  /* Step 2: rays from q parallel to l, towards P1 and towards P2. */
  float wu = P1[0] - m[0], wv = P1[1] - m[1];
  float lw = sqrtf(wu * wu + wv * wv);
  float uh[2] = {wu / lw, wv / lw};
  float un[2] = {-uh[0], -uh[1]};
  float q1[2], q2[2];
  rec.q0 = 1 + p->lin1 + p->bin1;
  line_binary(f, p, g, q, uh, sm, p->range2, p->lin2, p->bin2, q1, &tie_any, &rec);
  rec.q0 = 1 + p->lin1 + p->bin1 + p->lin2 + p->bin2;
  line_binary(f, p, g, q, un, sm, p->range2, p->lin2, p->bin2, q2, &tie_any, &rec);
  /* Step 3: intersection of line(P1,q1) and line(P2,q2). */
  double Au = (double)q1[0] - P1[0], Av = (double)q1[1] - P1[1];
  double Bu = (double)q2[0] - P2[0], Bv = (double)q2[1] - P2[1];
  double det = Au * Bv - Av * Bu;
  r.qm = 0;
  r.tie = tie_any;
  r.bits[0] = rec.own[0];
  r.bits[1] = rec.own[1];
  if (det == 0.0) {
    r.pf[0] = q[0]; r.pf[1] = q[1];
    r.sinang = 0.0;
    return r;
  }
  double Du = (double)P2[0] - P1[0], Dv = (double)P2[1] - P1[1];
  double alpha = (Du * Bv - Dv * Bu) / det;
  r.pf[0] = P1[0] + alpha * Au;
  r.pf[1] = P1[1] + alpha * Av;
  r.sinang = fabs(det) / (sqrt(Au * Au + Av * Av) * sqrt(Bu * Bu + Bv * Bv));
  return r;
}

/* ------------------------------------------------------------------------ */
/* QEF (Sec. 4, Eq. 2) with a truncated pseudo-inverse about the mass point */
/* ------------------------------------------------------------------------ */

/* Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix. */
static void jacobi3(double A[3][3], double V[3][3], double ev[3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j);
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
    double diag = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
    if (off == 0.0 || off <= 1e-18 * diag) break;
    for (int pq = 0; pq < 3; ++pq) {
      int pi = pq == 2 ? 1 : 0, qi = pq == 0 ? 1 : 2;
      if (A[pi][qi] == 0.0) continue;
      double theta = (A[qi][qi] - A[pi][pi]) / (2.0 * A[pi][qi]);
      double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      for (int k = 0; k < 3; ++k) { /* A <- A J */
        double akp = A[k][pi], akq = A[k][qi];
        A[k][pi] = c * akp - s * akq;
        A[k][qi] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) { /* A <- J^T A */
        double apk = A[pi][k], aqk = A[qi][k];
        A[pi][k] = c * apk - s * aqk;
        A[qi][k] = s * apk + c * aqk;
      }
      for (int k = 0; k < 3; ++k) {
        double vkp = V[k][pi], vkq = V[k][qi];
        V[k][pi] = c * vkp - s * vkq;
        V[k][qi] = s * vkp + c * vkq;
      }
    }
  }
  for (int i = 0; i < 3; ++i) ev[i] = A[i][i];
}

/* argmin_x sum (n.(x - p))^2 = mass point + A^+_tau r; returns the vertex.
 * Sets *trunc_tie when an eigenvalue sits at the truncation threshold. */
static void qef_solve(int n, const double* pl, double tau, double out[3], double* kappa,
                      int* trunc_tie, double* gap) {
  double c[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) c[a] += pl[6 * i + 3 + a];
  for (int a = 0; a < 3; ++a) c[a] /= (n > 0 ? n : 1);
  double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, b[3] = {0, 0, 0};
  int used = 0;
  for (int i = 0; i < n; ++i) {
    const double* nn = pl + 6 * i;
    if (nn[0] == 0.0 && nn[1] == 0.0 && nn[2] == 0.0) continue;
    ++used;
    double d = nn[0] * (pl[6 * i + 3] - c[0]) + nn[1] * (pl[6 * i + 4] - c[1]) +
               nn[2] * (pl[6 * i + 5] - c[2]);
    for (int r = 0; r < 3; ++r) {
      b[r] += nn[r] * d;
      for (int s = 0; s < 3; ++s) A[r][s] += nn[r] * nn[s];
    }
  }
  if (trunc_tie) *trunc_tie = 0;
  if (gap) *gap = INFINITY;
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2];
  if (used == 0) { if (kappa) *kappa = INFINITY; return; }
  double V[3][3], ev[3];
  jacobi3(A, V, ev);
  double lmax = fmax(ev[0], fmax(ev[1], ev[2]));
  double lmin = fmin(ev[0], fmin(ev[1], ev[2]));
  if (kappa) *kappa = lmin > 0.0 ? lmax / lmin : INFINITY;
  /* smallest distance between a kept and a dropped eigenvalue, relative to
   * the largest: how well a decomposition's rounding separates the kept
   * subspace (the solution's sensitivity to it grows as 1/gap) */
  if (gap) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        int keep_i = ev[i] >= tau * lmax && ev[i] > 0.0;
        int keep_j = ev[j] >= tau * lmax && ev[j] > 0.0;
        if (keep_i && !keep_j) *gap = fmin(*gap, (ev[i] - ev[j]) / lmax);
      }
  }
  for (int k = 0; k < 3; ++k) {
    if (trunc_tie && fabs(ev[k] - tau * lmax) <= 1e-5 * lmax) *trunc_tie = 1;
    if (!(ev[k] >= tau * lmax) || ev[k] <= 0.0) continue;
    double vb = V[0][k] * b[0] + V[1][k] * b[1] + V[2][k] * b[2];
    for (int a = 0; a < 3; ++a) out[a] += V[a][k] * vb / ev[k];
  }
}

void orc_qef_solve(int n, const double* planes, double tau, double out[3], double* kappa) {
  qef_solve(n, planes, tau, out, kappa, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Intersection-free quad split (Sec. 5.4; App. A.1.5, Eqs. A1-A2).          */
/* ------------------------------------------------------------------------ */

static double triple(const double a[3], const double b[3], const double c[3], double* scale) {
  double x = b[1] * c[2] - b[2] * c[1];
  double y = b[2] * c[0] - b[0] * c[2];
  double z = b[0] * c[1] - b[1] * c[0];
  double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  double nb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  double nc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  *scale = nb * nc + na * nc + na * nb;
  return a[0] * x + a[1] * y + a[2] * z;
}

int orc_ic_case(const double q[4][3], const double pin[3], const double pout[3], double tol,
                int* tie) {
  int concave[4];
  int t = 0;
  for (int k = 0; k < 4; ++k) {
    int kp = (k + 3) % 4, kn = (k + 1) % 4;
    double a[3], b[3], c[3], sc;
    for (int x = 0; x < 3; ++x) {
      a[x] = q[k][x] - pout[x];
      b[x] = q[kp][x] - pout[x];
      c[x] = q[kn][x] - pout[x];
    }
    double to = triple(a, b, c, &sc); /* Eq. A1 */
    if (fabs(to) <= 2.0 * tol * sc) t = 1;
    for (int x = 0; x < 3; ++x) {
      a[x] = q[k][x] - pin[x];
      b[x] = q[kp][x] - pin[x];
      c[x] = q[kn][x] - pin[x];
    }
    double ti = triple(a, b, c, &sc); /* Eq. A2 */
    if (fabs(ti) <= 2.0 * tol * sc) t = 1;
    concave[k] = (to < 0.0) || (ti > 0.0);
  }
  if (tie) *tie = t;
  if (!concave[1] && !concave[3]) return 1;
  if (!concave[0] && !concave[2]) return 2;
  return 3;
}

/* ------------------------------------------------------------------------ */
/* 3D points of one cell (Sec. 5.3): normals from each 1D point's two       */
/* neighbouring 2D points inside this cell, then the QEF per partition.     */
/* ------------------------------------------------------------------------ */

/* The recorded trace words of pair `slot` of face fid (replay), or NULL. */
static const uint64_t* trace_pair_words(orc_trace* tr, int64_t fid, int slot) {
  if (!tr || !tr->pair_bits) return NULL;
  int64_t x = trace_pair_slot(tr, fid, slot);
  if (x < 0) {
    count_unmatched(tr);
    return NULL;
  }
  return tr->pair_bits + 2 * x;
}

/* Staged inputs: the implementation's 1D point of edge eid (returns 1), or 0. */
static int staged_edge_t(const orc_trace* tr, int64_t eid, double* t) {
  if (!tr || !tr->staged || !tr->edge_t) return 0;
  int64_t x = trace_edge_slot(tr, eid);
  if (x < 0) return 0;
  *t = tr->edge_t[x];
  return 1;
}

/* Staged inputs: the implementation's 2D point of pair `slot` of face fid. */
static int staged_pair_pf(const orc_trace* tr, int64_t fid, int slot, double pf[2]) {
  if (!tr || !tr->staged || !tr->pair_pf) return 0;
  int64_t x = trace_pair_slot(tr, fid, slot);
  if (x < 0) return 0;
  pf[0] = tr->pair_pf[2 * x];
  pf[1] = tr->pair_pf[2 * x + 1];
  return 1;
}

typedef struct {
  /* lookups the cell needs; the full pipeline supplies tables, single-cell
   * queries compute on demand */
  const orc_field* f;
  const orc_params* p;
  const uint8_t* labels;          /* may be NULL */
  const int32_t* edge_index;      /* edge id -> crossing-edge index, or NULL */
  const double* edge_t;
  const int32_t* edge_tie;
  const int32_t* face_first_pair; /* face id -> first pair index (-1), or NULL */
  const double* pair_pf;
  const uint8_t* pair_tie;
  const uint8_t* face_flip;       /* face id -> flip flag, or NULL */
} cell_ctx;

static double ctx_edge_t(const cell_ctx* cx, int64_t eid, int* tie) {
  double st;
  if (staged_edge_t(cx->p->trace, eid, &st)) {
    *tie = 0;
    return st;
  }
  if (cx->edge_index) {
    int32_t ix = cx->edge_index[eid];
    *tie = cx->edge_tie[ix] != 0;
    return cx->edge_t[ix];
  }
  int ts = 0;
  double t = orc_edge_point(cx->f, cx->p, eid, &ts);
  *tie = ts != 0;
  return t;
}

static int ctx_face_flip(const cell_ctx* cx, int64_t fid) {
  if (cx->face_flip) return cx->face_flip[fid];
  face_geom g = face_geometry(cx->p->res, fid);
  return face_flip(cx->f, cx->p, cx->labels, &g);
}

/* 2D point of the pair `slot` of face fid, computed from scratch. */
static pair_result compute_pair(const orc_field* f, const orc_params* p, const uint8_t* labels,
                                int64_t fid, int slot, int flipped, int* info, int* edge_ties) {
  int N = p->res;
  face_geom g = face_geometry(N, fid);
  int L[4], pairs[2][2];
  face_labels_global(f, p, labels, &g, L);
  int np = face_pairs(L, flipped, pairs);
  int fa = pairs[slot][0], fb = pairs[slot][1];
  int ta = 0, tb = 0;
  int64_t ea = face_edge_global(N, &g, fa), eb = face_edge_global(N, &g, fb);
  double t1, t2;
  if (!staged_edge_t(p->trace, ea, &t1)) t1 = orc_edge_point(f, p, ea, &ta);
  if (!staged_edge_t(p->trace, eb, &t2)) t2 = orc_edge_point(f, p, eb, &tb);
  float P1[2], P2[2];
  face_edge_point(fa, (float)t1, P1);
  face_edge_point(fb, (float)t2, P2);
  pair_result r = search_pair(f, p, &g, L, P1, P2, trace_pair_words(p->trace, fid, slot));
  if (info)
    *info = slot | (fa << 4) | (fb << 8) | (flipped << 12) | (r.qm << 13) | ((np == 2) << 14);
  if (edge_ties) *edge_ties = (ta != 0) || (tb != 0);
  return r;
}

static void ctx_pair_pf(const cell_ctx* cx, int64_t fid, int slot, double pf[2], int* tie) {
  if (staged_pair_pf(cx->p->trace, fid, slot, pf)) {
    *tie = 0;
    return;
  }
  if (cx->face_first_pair) {
    int32_t ix = cx->face_first_pair[fid] + slot;
    pf[0] = cx->pair_pf[2 * ix];
    pf[1] = cx->pair_pf[2 * ix + 1];
    *tie = cx->pair_tie[ix] != 0;
    return;
  }
  int et = 0;
  pair_result r = compute_pair(cx->f, cx->p, cx->labels, fid, slot, ctx_face_flip(cx, fid),
                               NULL, &et);
  pf[0] = r.pf[0];
  pf[1] = r.pf[1];
  *tie = r.tie || et;
}

/* Computes the partitions and vertices of cell c; returns the count. */
static int cell_solve(const cell_ctx* cx, const int c[3], double* verts, int* partmap_out,
                      int* flipmask_out, int* tie_out, double* kappa_out, double* gap_out) {
  const orc_params* p = cx->p;
  int N = p->res;
  int cfg = cell_config(cx->f, p, cx->labels, c);
  if (cfg == 0 || cfg == 255) return 0;
  int flipmask = 0;
  for (int lf = 0; lf < 6; ++lf) {
    int a = lf / 2, s = lf % 2, pos[3] = {c[0], c[1], c[2]};
    pos[a] += s;
    if (ctx_face_flip(cx, face_id(N, a, pos))) flipmask |= 1 << lf;
  }
  int pm;
  int npart = orc_cube_partitions(cfg, flipmask, &pm);
  int tie = 0;
  double kmax = 0.0;
  for (int part = 0; part < npart; ++part) {
    double planes[12 * 6];
    int n = 0;
    for (int le = 0; le < 12; ++le) {
      if (!edge_crosses_config(cfg, le) || ((pm >> (2 * le)) & 3) != part) continue;
      int axis = le / 4, b1, b2, off[3] = {0, 0, 0};
      other_axes(axis, &b1, &b2);
      off[b1] = le & 1;
      off[b2] = (le >> 1) & 1;
      int gpos[3] = {c[0] + off[0], c[1] + off[1], c[2] + off[2]};
      int et = 0;
      double t = ctx_edge_t(cx, edge_id(N, axis, gpos), &et);
      tie |= et;
      double pe[3] = {off[0], off[1], off[2]};
      pe[axis] = t;
      double* row = planes + 6 * n;
      if (p->ablation & ORC_ABL_GRAD_NORMALS) {
        /* Eq. 2 with the field's gradient at the 1D point (the ablation
         * baseline); the query point is built as the searches build theirs */
        float g[3] = {(float)gpos[0], (float)gpos[1], (float)gpos[2]}, xw[3];
        g[axis] = (float)gpos[axis] + (float)t;
        grid_to_world(p, g, xw);
        double xd[3] = {xw[0], xw[1], xw[2]}, gr[3];
        const orc_trace* st = p->trace;
        int64_t sx = st && st->staged && st->edge_grad ? trace_edge_slot(st, edge_id(N, axis, gpos))
                                                       : -1;
        if (sx >= 0)  /* staged: the implementation's gradient */
          for (int q = 0; q < 3; ++q) gr[q] = st->edge_grad[3 * sx + q];
        else
          mlp_eval(cx->f, xd, gr);
        double gl = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
        for (int q = 0; q < 3; ++q) {
          row[q] = gl > 0.0 ? gr[q] / gl : 0.0;
          row[3 + q] = pe[q];
        }
        ++n;
        continue;
      }
      /* the two faces of this cell that contain the edge */
      double pfs[2][3];
      for (int w = 0; w < 2; ++w) {
        int fa = w == 0 ? b1 : b2;
        int side = off[fa];
        int fpos[3] = {c[0], c[1], c[2]};
        fpos[fa] += side;
        int64_t fid = face_id(N, fa, fpos);
        /* which pair of that face holds this edge */
        face_geom g = face_geometry(N, fid);
        int L[4], pairs[2][2];
        face_labels_global(cx->f, p, cx->labels, &g, L);
        int np = face_pairs(L, (flipmask >> (2 * fa + side)) & 1, pairs);
        int slot = -1;
        for (int q = 0; q < np; ++q)
          for (int k = 0; k < 2; ++k)
            if (face_edge_to_cell_edge(fa, side, pairs[q][k]) == le) slot = q;
        double pf[2];
        int pt = 0;
        ctx_pair_pf(cx, fid, slot, pf, &pt);
        tie |= pt;
        int u, v;
        other_axes(fa, &u, &v);
        pfs[w][fa] = side;
        pfs[w][u] = pf[0];
        pfs[w][v] = pf[1];
      }
      double a1[3], a2[3];
      for (int x = 0; x < 3; ++x) {
        a1[x] = pfs[0][x] - pe[x];
        a2[x] = pfs[1][x] - pe[x];
      }
      double nn[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2],
                      a1[0] * a2[1] - a1[1] * a2[0]};
      double nl = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
      for (int x = 0; x < 3; ++x) {
        row[x] = nl > 0.0 ? nn[x] / nl : 0.0;
        row[3 + x] = pe[x];
      }
      ++n;
    }
    double x[3], kap, gp;
    int tt = 0;
    qef_solve(n, planes, p->qef_tau, x, &kap, &tt, &gp);
    if (gap_out) gap_out[part] = gp;
    tie |= tt;
    if (kap > kmax) kmax = kap;
    if (p->clamp)
      for (int a = 0; a < 3; ++a) x[a] = fmin(fmax(x[a], 0.0), 1.0);
    for (int a = 0; a < 3; ++a) verts[3 * part + a] = c[a] + x[a];
    if (kappa_out) kappa_out[part] = kap;
  }
  /* corners whose label is itself a near-tie (the full pipeline has them) */
  if (cx->f->kind == ORC_FIELD_MLP && !cx->labels) {
    for (int lc = 0; lc < 8; ++lc) {
      int t = 0;
      orc_corner_label(cx->f, p, c[0] + (lc & 1), c[1] + ((lc >> 1) & 1), c[2] + ((lc >> 2) & 1),
                       &t);
      tie |= t;
    }
  }
  if (partmap_out) *partmap_out = pm;
  if (flipmask_out) *flipmask_out = flipmask;
  if (tie_out) *tie_out = tie;
  return npart;
}

int orc_pair_point(const orc_field* f, const orc_params* p, int64_t fid, int slot, double pf[2],
                   int* info, int* tie) {
  face_geom g = face_geometry(p->res, fid);
  int L[4], pairs[2][2];
  face_labels_global(f, p, NULL, &g, L);
  int flipped = face_flip(f, p, NULL, &g);
  int np = face_pairs(L, flipped, pairs);
  if (slot < 0 || slot >= np) return -1;
  int et = 0;
  pair_result r = compute_pair(f, p, NULL, fid, slot, flipped, info, &et);
  pf[0] = r.pf[0];
  pf[1] = r.pf[1];
  if (tie) *tie = r.tie || et;
  return np;
}

int orc_cell_vertices(const orc_field* f, const orc_params* p, int64_t cid, double* verts,
                      int* partmap, int* tie, double* kappa) {
  cell_ctx cx;
  memset(&cx, 0, sizeof(cx));
  cx.f = f;
  cx.p = p;
  int N = p->res;
  int c[3] = {(int)(cid % N), (int)((cid / N) % N), (int)(cid / ((int64_t)N * N))};
  return cell_solve(&cx, c, verts, partmap, NULL, tie, kappa, NULL);
}

/* ------------------------------------------------------------------------ */
/* Full pipeline                                                            */
/* ------------------------------------------------------------------------ */

static int valid_params(const orc_field* f, const orc_params* p) {
  if (!f || !p) return 0;
  if (p->res < 1 || p->res > 1024) return 0;
  if (!(p->size > 0.0)) return 0;
  if (p->iters_1d < 1 || p->iters_1d > 23) return 0;
  if (p->lin1 < 1 || p->lin2 < 1 || p->bin1 < 0 || p->bin2 < 0) return 0;
  if (f->kind == ORC_FIELD_CSG && (f->n_prims < 1 || !f->prims)) return 0;
  if (f->kind == ORC_FIELD_MLP && (!f->weights || f->depth < 1 || f->width < 1)) return 0;
  if (p->ablation &
      ~(ORC_ABL_LINEAR_1D | ORC_ABL_GRAD_NORMALS | ORC_ABL_MDC_SPLIT | ORC_ABL_SDF_INPUT))
    return 0;
  if ((p->ablation & ORC_ABL_SDF_INPUT) && !(p->ablation & ORC_ABL_LINEAR_1D)) return 0;
  if ((p->ablation & ORC_ABL_GRAD_NORMALS) && (f->kind != ORC_FIELD_MLP || f->depth > 64)) return 0;
  return 1;
}

#define ALLOC(ptr, n) ((ptr) = calloc((size_t)((n) > 0 ? (n) : 1), sizeof(*(ptr))))

int orc_mesh_extract(const orc_field* f, const orc_params* p, orc_mesh* m) {
  memset(m, 0, sizeof(*m));
  if (!valid_params(f, p)) return -1;
  if (f->kind == ORC_FIELD_MLP && 3 + 6 * f->n_bands != f->in_dim) return -1;
#ifdef _OPENMP
  /* n_threads = 0: the process default (OMP_NUM_THREADS or all cores), also
   * after an earlier call asked for fewer */
  static int default_threads = 0;
#pragma omp critical(orc_threads)
  {
    if (default_threads == 0) default_threads = omp_get_max_threads();
  }
  omp_set_num_threads(p->n_threads > 0 ? p->n_threads : default_threads);
#endif
  int N = p->res;
  m->res = N;
  int64_t NC = (int64_t)(N + 1) * (N + 1) * (N + 1);
  int64_t NE = 3 * edges_per_axis(N), NF = 3 * faces_per_axis(N), NCELL = (int64_t)N * N * N;

  /* corners */
  m->n_corners = NC;
  ALLOC(m->corner_label, NC);
  ALLOC(m->corner_tie, NC);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t id = 0; id < NC; ++id) {
    int i = (int)(id % (N + 1)), j = (int)((id / (N + 1)) % (N + 1)),
        k = (int)(id / ((int64_t)(N + 1) * (N + 1)));
    int tie = 0;
    m->corner_label[id] = (uint8_t)orc_corner_label(f, p, i, j, k, &tie);
    m->corner_tie[id] = (uint8_t)tie;
  }
  const uint8_t* lab = m->corner_label;

  /* crossing edges (Sec. 3) */
  int32_t* eidx;
  ALLOC(eidx, NE);
  int64_t ne = 0;
  for (int64_t e = 0; e < NE; ++e) {
    int a, pos[3];
    edge_decode(N, e, &a, pos);
    int up[3] = {pos[0], pos[1], pos[2]};
    up[a] += 1;
    if (lab[corner_id(N, pos[0], pos[1], pos[2])] != lab[corner_id(N, up[0], up[1], up[2])])
      eidx[e] = (int32_t)ne++;
    else
      eidx[e] = -1;
  }
  m->n_edges = ne;
  ALLOC(m->edge_id, ne);
  ALLOC(m->edge_t, ne);
  ALLOC(m->edge_tie_step, ne);
  ALLOC(m->edge_bits, ne);
  for (int64_t e = 0; e < NE; ++e)
    if (eidx[e] >= 0) m->edge_id[eidx[e]] = (int32_t)e;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t x = 0; x < ne; ++x) {
    if (p->topology_only) continue;
    int a, pos[3], ts = 0;
    edge_decode(N, m->edge_id[x], &a, pos);
    int l0 = lab[corner_id(N, pos[0], pos[1], pos[2])];
    m->edge_t[x] = edge_point_mode(f, p, a, pos, l0, &ts, m->edge_bits + x);
    m->edge_tie_step[x] = ts;
  }

  /* faces: pairs and manifold flips */
  int32_t* ffirst;
  uint8_t* fflip;
  ALLOC(ffirst, NF);
  ALLOC(fflip, NF);
  uint8_t* fcount;
  ALLOC(fcount, NF);
  int64_t np = 0;
  for (int64_t fid = 0; fid < NF; ++fid) {
    face_geom g = face_geometry(N, fid);
    int L[4], pairs[2][2];
    face_labels_global(f, p, lab, &g, L);
    int c = face_pairs(L, 0, pairs);
    fcount[fid] = (uint8_t)c;
    ffirst[fid] = c ? (int32_t)np : -1;
    if (c == 2) {
      fflip[fid] = (uint8_t)face_flip(f, p, lab, &g);
      m->n_flipped_faces += fflip[fid];
    }
    np += c;
  }
  m->n_pairs = np;
  ALLOC(m->pair_face, np);
  ALLOC(m->pair_info, np);
  ALLOC(m->pair_pf, 2 * np);
  ALLOC(m->pair_tie, np);
  ALLOC(m->pair_sin, np);
  ALLOC(m->pair_bits, 2 * np);
  for (int64_t fid = 0; fid < NF; ++fid)
    for (int s = 0; s < fcount[fid]; ++s) m->pair_face[ffirst[fid] + s] = (int32_t)fid;
  free(fcount);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t x = 0; x < np; ++x) {
    int64_t fid = m->pair_face[x];
    int slot = (int)(x - ffirst[fid]);
    face_geom g = face_geometry(N, fid);
    int L[4], pairs[2][2];
    face_labels_global(f, p, lab, &g, L);
    int npf = face_pairs(L, fflip[fid], pairs);
    int fa = pairs[slot][0], fb = pairs[slot][1];
    int64_t ga = face_edge_global(N, &g, fa), gb = face_edge_global(N, &g, fb);
    int32_t ia = eidx[ga], ib = eidx[gb];
    double t1 = m->edge_t[ia], t2 = m->edge_t[ib];
    staged_edge_t(p->trace, ga, &t1); /* the implementation's 1D points when staged */
    staged_edge_t(p->trace, gb, &t2);
    float P1[2], P2[2];
    face_edge_point(fa, (float)t1, P1);
    face_edge_point(fb, (float)t2, P2);
    pair_result r;
    if (p->topology_only || (p->ablation & ORC_ABL_GRAD_NORMALS)) {
      /* gradient normals need no 2D points */
      memset(&r, 0, sizeof(r));
      r.pf[0] = r.pf[1] = NAN;
    } else {
      r = search_pair(f, p, &g, L, P1, P2, trace_pair_words(p->trace, fid, slot));
    }
    m->pair_pf[2 * x] = r.pf[0];
    m->pair_pf[2 * x + 1] = r.pf[1];
    int ctie = 0;
    for (int lc = 0; lc < 4; ++lc) {
      int cp[3];
      face_corner_pos(&g, lc, cp);
      ctie |= m->corner_tie[corner_id(N, cp[0], cp[1], cp[2])];
    }
    m->pair_tie[x] = (uint8_t)(r.tie || ctie || m->edge_tie_step[ia] || m->edge_tie_step[ib]);
    m->pair_sin[x] = r.sinang;
    m->pair_bits[2 * x] = r.bits[0];
    m->pair_bits[2 * x + 1] = r.bits[1];
    m->pair_info[x] = slot | (fa << 4) | (fb << 8) | (fflip[fid] << 12) | (r.qm << 13) |
                      ((npf == 2) << 14);
  }

  /* active cells */
  int64_t nc = 0;
  int32_t* cidx;
  ALLOC(cidx, NCELL);
  for (int64_t cid = 0; cid < NCELL; ++cid) {
    int c[3] = {(int)(cid % N), (int)((cid / N) % N), (int)(cid / ((int64_t)N * N))};
    int cfg = cell_config(f, p, lab, c);
    cidx[cid] = (cfg != 0 && cfg != 255) ? (int32_t)nc++ : -1;
  }
  m->n_cells = nc;
  ALLOC(m->cell_id, nc);
  ALLOC(m->cell_npart, nc);
  ALLOC(m->cell_partmap, nc);
  ALLOC(m->cell_flipmask, nc);
  ALLOC(m->cell_vbase, nc);
  ALLOC(m->cell_tie, nc);
  for (int64_t cid = 0; cid < NCELL; ++cid)
    if (cidx[cid] >= 0) m->cell_id[cidx[cid]] = (int32_t)cid;
  double* cverts;
  double* ckap;
  double* cgap;
  uint8_t* ctie;
  ALLOC(cverts, 12 * nc);
  ALLOC(ckap, 4 * nc);
  ALLOC(cgap, 4 * nc);
  ALLOC(ctie, nc);
  int32_t* etie;
  ALLOC(etie, ne);
  for (int64_t x = 0; x < ne; ++x) etie[x] = m->edge_tie_step[x];
  cell_ctx cx;
  cx.f = f;
  cx.p = p;
  cx.labels = lab;
  cx.edge_index = eidx;
  cx.edge_t = m->edge_t;
  cx.edge_tie = etie;
  cx.face_first_pair = ffirst;
  cx.pair_pf = m->pair_pf;
  cx.pair_tie = m->pair_tie;
  cx.face_flip = fflip;
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t x = 0; x < nc; ++x) {
    int64_t cid = m->cell_id[x];
    int c[3] = {(int)(cid % N), (int)((cid / N) % N), (int)(cid / ((int64_t)N * N))};
    int pm, fm, tie = 0, npart;
    if (p->topology_only) {
      /* partitions only: the cell's configuration, its faces' flips, cycles */
      fm = 0;
      for (int lf = 0; lf < 6; ++lf) {
        int a = lf / 2, sd = lf % 2, pos[3] = {c[0], c[1], c[2]};
        pos[a] += sd;
        if (fflip[face_id(N, a, pos)]) fm |= 1 << lf;
      }
      npart = orc_cube_partitions(cell_config(f, p, lab, c), fm, &pm);
    } else {
      npart = cell_solve(&cx, c, cverts + 12 * x, &pm, &fm, &tie, ckap + 4 * x, cgap + 4 * x);
    }
    m->cell_npart[x] = npart;
    m->cell_partmap[x] = pm;
    m->cell_flipmask[x] = fm;
    /* corner ties in the cell (cell_solve checks them through the field) */
    for (int lc = 0; lc < 8; ++lc)
      tie |= m->corner_tie[corner_id(N, c[0] + (lc & 1), c[1] + ((lc >> 1) & 1),
                                     c[2] + ((lc >> 2) & 1))];
    m->cell_tie[x] = (uint8_t)tie;
  }
  int64_t nv = 0;
  for (int64_t x = 0; x < nc; ++x) {
    m->cell_vbase[x] = (int32_t)nv;
    nv += m->cell_npart[x];
  }

  /* emission (Sec. 4 polygonization; IC split of App. A.1.5) */
  ALLOC(m->edge_case, ne);
  ALLOC(m->edge_case_tie, ne);
  int32_t(*quad)[4];
  quad = calloc((size_t)(ne > 0 ? ne : 1), sizeof(*quad));
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t x = 0; x < ne; ++x) {
    if (p->topology_only) { m->edge_case[x] = 0; continue; }
    int a, pos[3];
    edge_decode(N, m->edge_id[x], &a, pos);
    int b = (a + 1) % 3, cc = (a + 2) % 3;
    static const int OFF[4][2] = {{0, 0}, {-1, 0}, {-1, -1}, {0, -1}};
    int cells[4][3], ok = 1;
    for (int q = 0; q < 4; ++q) {
      for (int y = 0; y < 3; ++y) cells[q][y] = pos[y];
      cells[q][b] += OFF[q][0];
      cells[q][cc] += OFF[q][1];
      for (int y = 0; y < 3; ++y)
        if (cells[q][y] < 0 || cells[q][y] >= N) ok = 0;
    }
    if (!ok) { m->edge_case[x] = 0; continue; }
    int vid[4], tie = 0;
    double P[4][3];
    for (int q = 0; q < 4; ++q) {
      int64_t cid = cell_id(N, cells[q][0], cells[q][1], cells[q][2]);
      int32_t ci = cidx[cid];
      int off[3];
      for (int y = 0; y < 3; ++y) off[y] = pos[y] - cells[q][y];
      int le = cell_local_edge(a, off);
      int part = (m->cell_partmap[ci] >> (2 * le)) & 3;
      vid[q] = m->cell_vbase[ci] + part;
      for (int y = 0; y < 3; ++y) P[q][y] = cverts[12 * ci + 3 * part + y];
      tie |= m->cell_tie[ci];
    }
    int lower_in = lab[corner_id(N, pos[0], pos[1], pos[2])];
    int ord[4] = {0, 1, 2, 3};
    if (!lower_in) { ord[1] = 3; ord[3] = 1; } /* c1, c4, c3, c2 */
    double Q[4][3], pin[3], pout[3];
    for (int q = 0; q < 4; ++q) {
      quad[x][q] = vid[ord[q]];
      for (int y = 0; y < 3; ++y) Q[q][y] = P[ord[q]][y];
    }
    for (int y = 0; y < 3; ++y) pin[y] = pout[y] = pos[y];
    if (lower_in) pout[a] += 1.0;
    else pin[a] += 1.0;
    int it = 0;
    if (p->ablation & ORC_ABL_MDC_SPLIT) {
      m->edge_case[x] = 1; /* the plain two-triangle split (ablation baseline) */
      m->edge_case_tie[x] = 0;
    } else {
      m->edge_case[x] = orc_ic_case(Q, pin, pout, p->ic_tie_tol, &it);
      m->edge_case_tie[x] = (uint8_t)(tie || it);
    }
  }
  int64_t n3 = 0, nt = 0;
  for (int64_t x = 0; x < ne; ++x) {
    if (m->edge_case[x] == 3) ++n3;
    nt += m->edge_case[x] == 0 ? 0 : (m->edge_case[x] == 3 ? 4 : 2);
  }
  m->n_case3 = n3;
  m->n_vertices = nv + n3;
  m->n_tris = nt;
  ALLOC(m->vert, 3 * m->n_vertices);
  ALLOC(m->vert_tie, m->n_vertices);
  ALLOC(m->vert_kappa, m->n_vertices);
  ALLOC(m->vert_gap, m->n_vertices);
  ALLOC(m->tris, 3 * nt);
  for (int64_t x = 0; x < nc; ++x)
    for (int q = 0; q < m->cell_npart[x]; ++q) {
      int64_t v = m->cell_vbase[x] + q;
      for (int y = 0; y < 3; ++y) m->vert[3 * v + y] = cverts[12 * x + 3 * q + y];
      m->vert_tie[v] = m->cell_tie[x];
      m->vert_kappa[v] = ckap[4 * x + q];
      m->vert_gap[v] = cgap[4 * x + q];
    }
  int64_t v3 = nv, tw = 0;
  for (int64_t x = 0; x < ne; ++x) {
    int cs = m->edge_case[x];
    if (cs == 0) continue;
    int32_t* T = m->tris + 3 * tw;
    const int32_t* Qd = quad[x];
    if (cs == 1) {
      T[0] = Qd[0]; T[1] = Qd[1]; T[2] = Qd[2];
      T[3] = Qd[0]; T[4] = Qd[2]; T[5] = Qd[3];
      tw += 2;
    } else if (cs == 2) {
      T[0] = Qd[0]; T[1] = Qd[1]; T[2] = Qd[3];
      T[3] = Qd[1]; T[4] = Qd[2]; T[5] = Qd[3];
      tw += 2;
    } else {
      int a, pos[3];
      edge_decode(N, m->edge_id[x], &a, pos);
      double te = m->edge_t[x];
      staged_edge_t(p->trace, m->edge_id[x], &te);
      for (int y = 0; y < 3; ++y) m->vert[3 * v3 + y] = pos[y];
      m->vert[3 * v3 + a] += te;
      m->vert_tie[v3] = (uint8_t)(m->edge_tie_step[x] != 0);
      m->vert_kappa[v3] = 0.0;
      m->vert_gap[v3] = INFINITY;
      for (int q = 0; q < 4; ++q) {
        T[3 * q] = (int32_t)v3;
        T[3 * q + 1] = Qd[q];
        T[3 * q + 2] = Qd[(q + 1) % 4];
      }
      ++v3;
      tw += 4;
    }
  }
  free(quad);
  free(cverts);
  free(ckap);
  free(cgap);
  free(ctie);
  free(etie);
  free(cidx);
  free(ffirst);
  free(fflip);
  free(eidx);
  return 0;
}

void orc_mesh_free(orc_mesh* m) {
  void* ptrs[] = {m->corner_label, m->corner_tie, m->edge_id, m->edge_t, m->edge_tie_step,
                  m->edge_bits, m->pair_bits,
                  m->pair_face, m->pair_info, m->pair_pf, m->pair_tie, m->pair_sin,
                  m->cell_id, m->cell_npart, m->cell_partmap, m->cell_flipmask, m->cell_vbase,
                  m->cell_tie, m->vert, m->vert_tie, m->vert_kappa, m->vert_gap, m->edge_case,
                  m->edge_case_tie, m->tris};
  for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) free(ptrs[i]);
  memset(m, 0, sizeof(*m));
}

/* ------------------------------------------------------------------------ */
/* Self-intersections (a quality metric of Sec. 6): pairs of triangles that  */
/* share no vertex and whose closed triangles intersect, by brute force over */
/* all pairs.  Non-coplanar pairs: an edge of one meets the other triangle, */
/* found by solving p + s (q - p) = A + u (B - A) + v (C - A) with Cramer's  */
/* rule.  Coplanar pairs: no separating axis among the six edge normals in   */
/* the common plane.                                                         */
/* ------------------------------------------------------------------------ */

static void sub3(const double a[3], const double b[3], double o[3]) {
  for (int k = 0; k < 3; ++k) o[k] = a[k] - b[k];
}
static void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* segment pq against triangle ABC, the triangle's plane not containing pq */
static int segment_hits_triangle(const double p[3], const double q[3], const double A[3],
                                 const double B[3], const double C[3]) {
  double d[3], e1[3], e2[3], r[3];
  sub3(q, p, d);
  sub3(B, A, e1);
  sub3(C, A, e2);
  sub3(p, A, r);
  /* [e1 e2 -d] (u v s)^T = r */
  double md[3] = {-d[0], -d[1], -d[2]}, c12[3];
  cross3(e1, e2, c12);
  double det = dot3(c12, md);
  if (det == 0.0) return 0; /* parallel to the plane */
  double t1[3], t2[3], t3[3];
  cross3(r, e2, t1);
  cross3(e1, r, t2);
  double u = dot3(t1, md) / det;
  double v = dot3(t2, md) / det;
  cross3(e1, e2, t3);
  double s = dot3(t3, r) / det;
  return s >= 0.0 && s <= 1.0 && u >= 0.0 && v >= 0.0 && u + v <= 1.0;
}

static int coplanar_overlap(const double P[3][3], const double Q[3][3], const double n[3]) {
  /* separating-axis test: axes n x (edge) of both triangles */
  for (int w = 0; w < 2; ++w) {
    const double(*T)[3] = w == 0 ? P : Q;
    for (int e = 0; e < 3; ++e) {
      double ed[3], ax[3];
      sub3(T[(e + 1) % 3], T[e], ed);
      cross3(n, ed, ax);
      double pmin = INFINITY, pmax = -INFINITY, qmin = INFINITY, qmax = -INFINITY;
      for (int k = 0; k < 3; ++k) {
        double a = dot3(ax, P[k]), b = dot3(ax, Q[k]);
        pmin = fmin(pmin, a); pmax = fmax(pmax, a);
        qmin = fmin(qmin, b); qmax = fmax(qmax, b);
      }
      if (pmax < qmin || qmax < pmin) return 0;
    }
  }
  return 1;
}

static int triangles_intersect(const double P[3][3], const double Q[3][3]) {
  double e1[3], e2[3], n[3];
  sub3(P[1], P[0], e1);
  sub3(P[2], P[0], e2);
  cross3(e1, e2, n);
  int coplanar = 1;
  for (int k = 0; k < 3; ++k) {
    double r[3];
    sub3(Q[k], P[0], r);
    if (dot3(n, r) != 0.0) coplanar = 0;
  }
  if (coplanar) return coplanar_overlap(P, Q, n);
  for (int e = 0; e < 3; ++e) {
    if (segment_hits_triangle(P[e], P[(e + 1) % 3], Q[0], Q[1], Q[2])) return 1;
    if (segment_hits_triangle(Q[e], Q[(e + 1) % 3], P[0], P[1], P[2])) return 1;
  }
  return 0;
}

int64_t orc_self_intersections(const float* vertices, int64_t n_vertices, const int32_t* tris,
                               int64_t n_tris) {
  (void)n_vertices;
  int64_t count = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : count)
  for (int64_t a = 0; a < n_tris; ++a) {
    double P[3][3], lo[3], hi[3];
    for (int k = 0; k < 3; ++k)
      for (int c = 0; c < 3; ++c) P[k][c] = vertices[3 * (int64_t)tris[3 * a + k] + c];
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmin(P[0][c], fmin(P[1][c], P[2][c]));
      hi[c] = fmax(P[0][c], fmax(P[1][c], P[2][c]));
    }
    for (int64_t b = a + 1; b < n_tris; ++b) {
      int shared = 0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) shared |= tris[3 * a + i] == tris[3 * b + j];
      if (shared) continue;
      double Q[3][3];
      int apart = 0;
      for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 3; ++c) Q[k][c] = vertices[3 * (int64_t)tris[3 * b + k] + c];
      for (int c = 0; c < 3; ++c) {
        double ql = fmin(Q[0][c], fmin(Q[1][c], Q[2][c])), qh = fmax(Q[0][c], fmax(Q[1][c], Q[2][c]));
        if (qh < lo[c] || ql > hi[c]) apart = 1;
      }
      if (!apart && triangles_intersect(P, Q)) ++count;
    }
  }
  return count;
}
