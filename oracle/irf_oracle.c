/*
 * FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see irf_oracle.h).
 *
 * Paper: Majercik, Marrs, Spjut, McGuire, "Scaling Probe-Based Real-Time
 * Dynamic Global Illumination for Production" (JCGT / arXiv 2009.10796).
 * Sections are cited by title:
 *   "Overview of the algorithm"   -> Build/Init, Probe Query, Probe Update,
 *                                    and the hysteresis update equation (Eq. U)
 *   "Self-shadow bias ..."         -> Eq. 1 and the backface-ray rule
 *   "Probe States"                 -> states, full initialization algorithm
 *   "Multiple Probe Volumes"       -> cascade blending
 * Readings where the paper is silent follow the published base method
 * (DDGI, Majercik et al. 2019); the GPU path takes the same readings.
 *
 * Plain, unblocked loops: every function follows the definition it cites.
 */
#include "irf_oracle.h"

#include <float.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>

/* Arithmetic type of the value path (octahedral map, ray directions,
   shading, blend, query).  The oracle is double.  The same source built with
   -DORC_REAL=float (and single-precision constants) is a float32 evaluation
   of the same steps, used only to check the oracle's own float32
   sensitivity estimate (kappa) as an error bound.  Nearest-hit search,
   flags, classification and the adjoint stay double in both builds; every
   interface array is double in both (a float32 build rounds what it reads). */
#ifndef ORC_REAL
#define ORC_REAL double
#endif
typedef ORC_REAL real;

#define EPS_B 1e-4   /* barycentric margin for flags */
#define EPS_T 1e-6   /* relative distance margin for flags */
#define U32 (1.0 / 16777216.0)

/* ------------------------------------------------------------------ vec3 */
static inline double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static inline void sub3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static inline void cross3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double len3(const double a[3]) { return sqrt(dot3(a, a)); }
static inline void normalize3(double a[3]) {
  double l = len3(a);
  if (l > 0) { a[0] /= l; a[1] /= l; a[2] /= l; }
  else { a[0] = a[1] = a[2] = 0; }
}
static inline double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }
static inline double signnz(double x) { return x >= 0.0 ? 1.0 : -1.0; }

/* the same helpers in the value-path type */
static inline real dot3r(const real a[3], const real b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void sub3r(const real a[3], const real b[3], real r[3]) {
  r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static inline void cross3r(const real a[3], const real b[3], real r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
static inline real len3r(const real a[3]) { return sqrt(dot3r(a, a)); }
static inline void normalize3r(real a[3]) {
  real l = len3r(a);
  if (l > 0) { a[0] /= l; a[1] /= l; a[2] /= l; }
  else { a[0] = a[1] = a[2] = 0; }
}
static inline real clampr(real x, real lo, real hi) { return x < lo ? lo : (x > hi ? hi : x); }
static inline real signnzr(real x) { return x >= 0 ? 1 : -1; }
static inline void load3r(const double a[3], real r[3]) { r[0] = (real)a[0]; r[1] = (real)a[1]; r[2] = (real)a[2]; }

/* ------------------------------------------------------------------ scene */
typedef struct {
  double lo[3], hi[3];
  int32_t left, right;  /* children, -1 for leaves */
  int32_t first, count; /* range in s->order for leaves */
} onode;

struct orc_scene {
  int64_t nt;
  double* v;          /* [T][3][3] triangle vertices */
  int32_t* material;  /* [T] */
  int32_t* object;    /* [T] */
  int32_t nm;
  double* albedo;     /* [M][3] */
  double* emission;   /* [M][3] */
  double* specular;   /* [M][3] mirror reflectance (second-order glossy), zeros unless set */
  int32_t* order;     /* triangle ids in leaf order */
  onode* nodes;
  int64_t nnodes, cap;
  int32_t nobj;       /* number of dynamic objects (ids 1..nobj) */
  double* obj_lo;     /* [nobj+1][3] */
  double* obj_hi;
};

static const double* tri_v(const orc_scene* s, int64_t t, int k) { return s->v + (t * 3 + k) * 3; }

static void tri_box(const orc_scene* s, int32_t t, double lo[3], double hi[3]) {
  /* triangle bounds inflated so that every point within EPS_B (barycentric)
     of the triangle is inside; the flag pass relies on it */
  double e = 0;
  for (int k = 0; k < 3; k++) {
    double d[3];
    sub3(tri_v(s, t, (k + 1) % 3), tri_v(s, t, k), d);
    double l = len3(d);
    if (l > e) e = l;
  }
  e = 4.0 * EPS_B * e + 1e-9;
  for (int a = 0; a < 3; a++) {
    lo[a] = INFINITY; hi[a] = -INFINITY;
    for (int k = 0; k < 3; k++) {
      double x = tri_v(s, t, k)[a];
      if (x < lo[a]) lo[a] = x;
      if (x > hi[a]) hi[a] = x;
    }
    lo[a] -= e; hi[a] += e;
  }
}

static int32_t new_node(orc_scene* s) {
  if (s->nnodes == s->cap) {
    s->cap = s->cap ? s->cap * 2 : 1024;
    s->nodes = (onode*)realloc(s->nodes, (size_t)s->cap * sizeof(onode));
  }
  return (int32_t)s->nnodes++;
}

static double* g_cent; /* build-time centroid table, used by the comparator */
static int g_axis;
static int cmp_cent(const void* a, const void* b) {
  double ca = g_cent[*(const int32_t*)a * 3 + g_axis];
  double cb = g_cent[*(const int32_t*)b * 3 + g_axis];
  if (ca < cb) return -1;
  if (ca > cb) return 1;
  return (*(const int32_t*)a) - (*(const int32_t*)b);
}

/* median split on the widest centroid axis; exact accelerator only */
static int32_t build(orc_scene* s, int32_t first, int32_t count) {
  int32_t id = new_node(s);
  onode n;
  for (int a = 0; a < 3; a++) { n.lo[a] = INFINITY; n.hi[a] = -INFINITY; }
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t i = first; i < first + count; i++) {
    double lo[3], hi[3];
    int32_t t = s->order[i];
    tri_box(s, t, lo, hi);
    for (int a = 0; a < 3; a++) {
      if (lo[a] < n.lo[a]) n.lo[a] = lo[a];
      if (hi[a] > n.hi[a]) n.hi[a] = hi[a];
      double c = g_cent[t * 3 + a];
      if (c < clo[a]) clo[a] = c;
      if (c > chi[a]) chi[a] = c;
    }
  }
  n.left = n.right = -1;
  n.first = first;
  n.count = count;
  if (count > 4) {
    int axis = 0;
    for (int a = 1; a < 3; a++)
      if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    g_axis = axis;
    qsort(s->order + first, (size_t)count, sizeof(int32_t), cmp_cent);
    int32_t half = count / 2;
    n.left = build(s, first, half);
    n.right = build(s, first + half, count - half);
    n.count = 0;
  }
  s->nodes[id] = n;
  return id;
}

orc_scene* orc_scene_create(const float* vertices, int64_t n_vertices, const uint32_t* indices,
                            int64_t n_tris, const uint32_t* tri_material, const uint32_t* tri_object,
                            const float* albedo, const float* emission, int32_t n_materials) {
  (void)n_vertices;
  orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
  s->nt = n_tris;
  s->v = (double*)malloc(sizeof(double) * 9 * (size_t)(n_tris ? n_tris : 1));
  s->material = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_tris ? n_tris : 1));
  s->object = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_tris ? n_tris : 1));
  s->order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_tris ? n_tris : 1));
  s->nobj = 0;
  for (int64_t t = 0; t < n_tris; t++) {
    for (int k = 0; k < 3; k++)
      for (int a = 0; a < 3; a++) s->v[(t * 3 + k) * 3 + a] = (double)vertices[(size_t)indices[t * 3 + k] * 3 + a];
    s->material[t] = (int32_t)tri_material[t];
    s->object[t] = tri_object ? (int32_t)tri_object[t] : 0;
    if (s->object[t] > s->nobj) s->nobj = s->object[t];
    s->order[t] = (int32_t)t;
  }
  s->nm = n_materials;
  s->albedo = (double*)malloc(sizeof(double) * 3 * (size_t)(n_materials ? n_materials : 1));
  s->emission = (double*)malloc(sizeof(double) * 3 * (size_t)(n_materials ? n_materials : 1));
  s->specular = (double*)calloc(3 * (size_t)(n_materials ? n_materials : 1), sizeof(double));
  for (int32_t m = 0; m < 3 * n_materials; m++) {
    s->albedo[m] = albedo[m];
    s->emission[m] = emission[m];
  }
  s->obj_lo = (double*)malloc(sizeof(double) * 3 * (size_t)(s->nobj + 1));
  s->obj_hi = (double*)malloc(sizeof(double) * 3 * (size_t)(s->nobj + 1));
  for (int32_t o = 0; o <= s->nobj; o++)
    for (int a = 0; a < 3; a++) { s->obj_lo[o * 3 + a] = INFINITY; s->obj_hi[o * 3 + a] = -INFINITY; }
  for (int64_t t = 0; t < n_tris; t++) {
    int32_t o = s->object[t];
    for (int k = 0; k < 3; k++)
      for (int a = 0; a < 3; a++) {
        double x = tri_v(s, t, k)[a];
        if (x < s->obj_lo[o * 3 + a]) s->obj_lo[o * 3 + a] = x;
        if (x > s->obj_hi[o * 3 + a]) s->obj_hi[o * 3 + a] = x;
      }
  }
  if (n_tris > 0) {
    g_cent = (double*)malloc(sizeof(double) * 3 * (size_t)n_tris);
    for (int64_t t = 0; t < n_tris; t++)
      for (int a = 0; a < 3; a++)
        g_cent[t * 3 + a] = (tri_v(s, t, 0)[a] + tri_v(s, t, 1)[a] + tri_v(s, t, 2)[a]) / 3.0;
    build(s, 0, (int32_t)n_tris);
    free(g_cent);
    g_cent = NULL;
  }
  return s;
}

void orc_scene_free(orc_scene* s) {
  if (!s) return;
  free(s->v); free(s->material); free(s->object); free(s->order); free(s->nodes);
  free(s->albedo); free(s->emission); free(s->specular); free(s->obj_lo); free(s->obj_hi);
  free(s);
}

int64_t orc_scene_bvh_nodes(const orc_scene* s) { return s->nnodes; }

void orc_scene_set_specular(orc_scene* s, const double* specular) {
  for (int32_t m = 0; m < 3 * s->nm; m++) s->specular[m] = specular[m];
}

void orc_scene_set_emission(orc_scene* s, const double* emission) {
  for (int32_t m = 0; m < 3 * s->nm; m++) s->emission[m] = emission[m];
}

/* ---------------------------------------------------------- intersection */
/* Plane intersection of ray o + t d with triangle t (Moller-Trumbore):
   returns 0 if the ray is parallel to the plane, else t and the three
   barycentric coordinates (negative outside the triangle). */
static int plane_hit(const orc_scene* s, int32_t tri, const double o[3], const double d[3],
                     double* t, double* bmin) {
  const double *v0 = tri_v(s, tri, 0), *v1 = tri_v(s, tri, 1), *v2 = tri_v(s, tri, 2);
  double e1[3], e2[3], p[3], q[3], sv[3];
  sub3(v1, v0, e1);
  sub3(v2, v0, e2);
  cross3(d, e2, p);
  double det = dot3(e1, p);
  if (det == 0.0) return 0;
  double inv = 1.0 / det;
  sub3(o, v0, sv);
  double u = dot3(sv, p) * inv;
  cross3(sv, e1, q);
  double v = dot3(d, q) * inv;
  *t = dot3(e2, q) * inv;
  double b0 = 1.0 - u - v;
  double m = b0 < u ? b0 : u;
  *bmin = m < v ? m : v;
  return 1;
}

static int box_hit(const onode* n, const double o[3], const double d[3], double tmax) {
  double t0 = 0.0, t1 = tmax;
  for (int a = 0; a < 3; a++) {
    if (d[a] == 0.0) {
      if (o[a] < n->lo[a] || o[a] > n->hi[a]) return 0;
      continue;
    }
    double ta = (n->lo[a] - o[a]) / d[a], tb = (n->hi[a] - o[a]) / d[a];
    if (ta > tb) { double x = ta; ta = tb; tb = x; }
    if (ta > t0) t0 = ta;
    if (tb < t1) t1 = tb;
    if (t0 > t1) return 0;
  }
  return 1;
}

static int skip_tri(const orc_scene* s, int32_t t, int32_t static_only) {
  return static_only && s->object[t] != 0;
}

/* Visits every leaf triangle whose (inflated) box meets the ray within
   [0, *tlim]; the callback may shrink *tlim. brute: visit all triangles. */
typedef void (*visit_fn)(const orc_scene* s, int32_t tri, const double o[3], const double d[3],
                         void* ctx, double* tlim);

static void traverse(const orc_scene* s, const double o[3], const double d[3], double* tlim,
                     int32_t static_only, int brute, visit_fn f, void* ctx) {
  if (s->nt == 0) return;
  if (brute) {
    for (int64_t t = 0; t < s->nt; t++)
      if (!skip_tri(s, (int32_t)t, static_only)) f(s, (int32_t)t, o, d, ctx, tlim);
    return;
  }
  int32_t stack[256];
  int sp = 0;
  stack[sp++] = 0;
  while (sp) {
    const onode* n = &s->nodes[stack[--sp]];
    double lim = isinf(*tlim) ? INFINITY : *tlim * (1.0 + 4.0 * EPS_T) + 1e-12;
    if (!box_hit(n, o, d, lim)) continue;
    if (n->left < 0) {
      for (int32_t i = n->first; i < n->first + n->count; i++) {
        int32_t t = s->order[i];
        if (!skip_tri(s, t, static_only)) f(s, t, o, d, ctx, tlim);
      }
    } else {
      stack[sp++] = n->left;
      stack[sp++] = n->right;
    }
  }
}

typedef struct { double t; int32_t tri; } closest_ctx;

static void visit_closest(const orc_scene* s, int32_t tri, const double o[3], const double d[3],
                          void* vctx, double* tlim) {
  closest_ctx* c = (closest_ctx*)vctx;
  double t, bmin;
  if (!plane_hit(s, tri, o, d, &t, &bmin)) return;
  if (!(t > 0.0) || bmin < 0.0) return;
  if (t < c->t || (t == c->t && tri < c->tri)) {
    c->t = t;
    c->tri = tri;
    *tlim = t;
  }
}

typedef struct { double t; int32_t tri; int32_t flags; } flag_ctx;

static void visit_flags(const orc_scene* s, int32_t tri, const double o[3], const double d[3],
                        void* vctx, double* tlim) {
  (void)tlim;
  flag_ctx* c = (flag_ctx*)vctx;
  if (tri == c->tri) return;
  double t, bmin;
  if (!plane_hit(s, tri, o, d, &t, &bmin)) return;
  if (!(t > 0.0)) return;
  if (c->tri >= 0 && t > c->t * (1.0 + EPS_T)) return;
  if (bmin >= 0.0) {
    if (c->tri >= 0 && fabs(t - c->t) <= EPS_T * c->t) c->flags |= ORC_F_TIE;
  } else if (bmin > -EPS_B) {
    c->flags |= ORC_F_NEARMISS;
  }
}

static void trace_impl(const orc_scene* s, const double o[3], const double d[3], int32_t static_only,
                       int brute, orc_hit* hit) {
  closest_ctx c = {INFINITY, -1};
  double tlim = INFINITY;
  traverse(s, o, d, &tlim, static_only, brute, visit_closest, &c);
  flag_ctx f = {c.t, c.tri, 0};
  double tl2 = c.tri >= 0 ? c.t : INFINITY;
  traverse(s, o, d, &tl2, static_only, brute, visit_flags, &f);
  hit->tri = c.tri;
  hit->t = c.t;
  hit->bmin = 0.0;
  hit->flags = f.flags;
  if (c.tri >= 0) {
    double t, bmin;
    plane_hit(s, c.tri, o, d, &t, &bmin);
    hit->bmin = bmin;
    if (bmin < EPS_B) hit->flags |= ORC_F_GRAZE;
    double e1[3], e2[3], n[3];
    sub3(tri_v(s, c.tri, 1), tri_v(s, c.tri, 0), e1);
    sub3(tri_v(s, c.tri, 2), tri_v(s, c.tri, 0), e2);
    cross3(e1, e2, n);
    if (fabs(dot3(n, d)) < 1e-5 * len3(n) * len3(d)) hit->flags |= ORC_F_EDGEON;
  }
}

void orc_trace(const orc_scene* s, const double o[3], const double d[3], int32_t static_only, orc_hit* hit) {
  trace_impl(s, o, d, static_only, 0, hit);
}
void orc_trace_brute(const orc_scene* s, const double o[3], const double d[3], int32_t static_only,
                     orc_hit* hit) {
  trace_impl(s, o, d, static_only, 1, hit);
}
void orc_trace_batch(const orc_scene* s, int64_t n, const double* o, const double* d,
                     int32_t static_only, int32_t brute, orc_hit* hits) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; i++) trace_impl(s, o + 3 * i, d + 3 * i, static_only, brute, &hits[i]);
}

/* Shadow ray: is any triangle (either side) hit at 0 < t < tmax?  ambiguous
   is set when a float32 tracer could decide otherwise. */
typedef struct { double tmax; int occ; int robust; int amb; } shadow_ctx;

static void visit_shadow(const orc_scene* s, int32_t tri, const double o[3], const double d[3],
                         void* vctx, double* tlim) {
  shadow_ctx* c = (shadow_ctx*)vctx;
  if (c->robust) return;
  double t, bmin;
  if (!plane_hit(s, tri, o, d, &t, &bmin)) return;
  if (!(t > -EPS_T)) return;
  double hi = isinf(c->tmax) ? INFINITY : c->tmax * (1.0 + EPS_T);
  if (t > hi) return;
  double lo_amb = isinf(c->tmax) ? INFINITY : c->tmax * (1.0 - EPS_T);
  int inside = bmin >= 0.0 && t > 0.0 && t < c->tmax;
  if (inside) c->occ = 1;
  if (inside && bmin >= EPS_B && t < lo_amb && t > EPS_T) {
    c->robust = 1;
    *tlim = 0.0; /* stop: the decision is settled */
    return;
  }
  if (fabs(bmin) < EPS_B || (bmin >= 0.0 && (t >= lo_amb || t <= EPS_T))) c->amb = 1;
}

static int occluded(const orc_scene* s, const double o[3], const double d[3], double tmax, int* amb) {
  shadow_ctx c = {tmax, 0, 0, 0};
  double tlim = tmax;
  traverse(s, o, d, &tlim, 0, 0, visit_shadow, &c);
  *amb = c.robust ? 0 : c.amb;
  return c.occ;
}

/* -------------------------------------------------------------- octahedral */
/* Octahedral map of the unit sphere onto [-1,1]^2 (Cigolle et al. 2014),
   used for the probe tiles (Section "Probe Representation" and Table 2). */
static void oct_encode_r(const real v[3], real p[2]) {
  real l1 = fabs(v[0]) + fabs(v[1]) + fabs(v[2]);
  real x = v[0] / l1, y = v[1] / l1;
  if (v[2] < 0.0) {
    real nx = (1.0 - fabs(y)) * signnzr(x);
    real ny = (1.0 - fabs(x)) * signnzr(y);
    x = nx;
    y = ny;
  }
  p[0] = x;
  p[1] = y;
}

static void oct_decode_r(const real p[2], real v[3]) {
  real x = p[0], y = p[1];
  real z = 1.0 - fabs(x) - fabs(y);
  if (z < 0.0) {
    real nx = (1.0 - fabs(y)) * signnzr(x);
    real ny = (1.0 - fabs(x)) * signnzr(y);
    x = nx;
    y = ny;
  }
  v[0] = x; v[1] = y; v[2] = z;
  normalize3r(v);
}

void orc_oct_encode(const double v[3], double p[2]) {
  real vr[3], pr[2];
  load3r(v, vr);
  oct_encode_r(vr, pr);
  p[0] = pr[0];
  p[1] = pr[1];
}

void orc_oct_decode(const double p[2], double v[3]) {
  real pr[2] = {(real)p[0], (real)p[1]}, vr[3];
  oct_decode_r(pr, vr);
  for (int a = 0; a < 3; a++) v[a] = vr[a];
}

/* interior cell (x, y) of an m x m tile covers [-1,1]^2 in k = m-2 cells */
static void texel_direction_r(int32_t m, int32_t x, int32_t y, real v[3]) {
  int32_t k = m - 2;
  real p[2] = {(real)2.0 * ((x - 1) + (real)0.5) / k - 1, (real)2.0 * ((y - 1) + (real)0.5) / k - 1};
  oct_decode_r(p, v);
}

void orc_texel_direction(int32_t m, int32_t x, int32_t y, double v[3]) {
  real vr[3];
  texel_direction_r(m, x, y, vr);
  for (int a = 0; a < 3; a++) v[a] = vr[a];
}

/* The one-texel border repeats the cell across the octahedral seam: the
   edge p_y = -1 folds onto itself mirrored in x (and likewise for the other
   edges); corners take the diagonally opposite interior corner. */
void orc_border_source(int32_t m, int32_t x, int32_t y, int32_t* sx, int32_t* sy) {
  int32_t k = m - 2;
  int bx = (x == 0 || x == k + 1), by = (y == 0 || y == k + 1);
  if (bx && by) {
    *sx = (x == 0) ? k : 1;
    *sy = (y == 0) ? k : 1;
  } else if (by) {
    *sx = k + 1 - x;
    *sy = (y == 0) ? 1 : k;
  } else if (bx) {
    *sx = (x == 0) ? 1 : k;
    *sy = k + 1 - y;
  } else {
    *sx = x;
    *sy = y;
  }
}

static void sample_tile_r(const double* tile, int32_t m, int32_t nch, const real v[3], real* out) {
  int32_t k = m - 2;
  real p[2];
  oct_encode_r(v, p);
  real cx = 1.0 + (0.5 * p[0] + 0.5) * k - 0.5;
  real cy = 1.0 + (0.5 * p[1] + 0.5) * k - 0.5;
  int32_t x0 = (int32_t)floor(cx), y0 = (int32_t)floor(cy);
  if (x0 < 0) x0 = 0;
  if (x0 > k) x0 = k;
  if (y0 < 0) y0 = 0;
  if (y0 > k) y0 = k;
  real fx = clampr(cx - x0, 0.0, 1.0), fy = clampr(cy - y0, 0.0, 1.0);
  for (int c = 0; c < nch; c++) {
    real a = tile[(y0 * m + x0) * nch + c], b = tile[(y0 * m + x0 + 1) * nch + c];
    real cc = tile[((y0 + 1) * m + x0) * nch + c], dd = tile[((y0 + 1) * m + x0 + 1) * nch + c];
    out[c] = (1 - fy) * ((1 - fx) * a + fx * b) + fy * ((1 - fx) * cc + fx * dd);
  }
}

void orc_sample_tile(const double* tile, int32_t m, int32_t nch, const double v[3], double* out) {
  real vr[3], o[4];
  load3r(v, vr);
  sample_tile_r(tile, m, nch, vr, o);
  for (int c = 0; c < nch; c++) out[c] = o[c];
}

/* -------------------------------------------------------------------- rays */
/* Spherical Fibonacci point i of n (Keinert et al. 2015), rotated by the
   frame's random rotation (Section "Probe Update"). */
void orc_sf_direction(int32_t i, int32_t n, const float R[9], double out[3]) {
  /* the fractional part of i * phi is taken in double in both builds: it
     has to be exact (in float32 the product loses the fraction's low bits) */
  const double phi = (1.0 + sqrt((double)5)) / 2.0;
  double f = (double)i * phi;
  double frac = f - floor(f);
  real z = 1.0 - (2.0 * i + 1.0) / n;
  real r = sqrt(fmax((real)0.0, 1.0 - z * z));
  real a = (real)2.0 * (real)M_PI * (real)frac;
  real sf[3] = {r * cos(a), r * sin(a), z};
  for (int row = 0; row < 3; row++)
    out[row] = (real)R[row * 3 + 0] * sf[0] + (real)R[row * 3 + 1] * sf[1] + (real)R[row * 3 + 2] * sf[2];
}

/* ------------------------------------------------------------------- blend */
/* Eq. U with the normalisation that makes it the weighted *average* the text
   describes: texel' = a*texel + (1-a) * sum(w L) / sum(w), w = max(0, n.w)
   for irradiance and max(0, n.w)^p for mean distance and distance^2.  The
   border is copied from the blended interior afterwards. */
void orc_blend_probe(int32_t n, const double* omega, const double* rgb, const double* d,
                     double cos_power, double alpha_irr, double alpha_dist,
                     double* irr, double* dist) {
  orc_blend_probe_k(n, omega, rgb, NULL, d, NULL, cos_power, alpha_irr, alpha_dist, 1.0, 0, irr, dist, NULL, NULL);
}

void orc_blend_probe_ex(int32_t n, const double* omega, const double* rgb, const double* d, double cos_power,
                        double alpha_irr, double alpha_dist, double gamma, int32_t thresholds, double* irr,
                        double* dist) {
  orc_blend_probe_k(n, omega, rgb, NULL, d, NULL, cos_power, alpha_irr, alpha_dist, gamma, thresholds, irr, dist,
                    NULL, NULL);
}

/* Section "Fast Convergence Heuristics": the irradiance hysteresis of one
   texel given the largest per-channel change between the new (encoded) value
   and the stored one: lowered by 0.15 (not below 0) above a change of 0.25,
   and 0 above 0.8 (the probe is taken to see a new distribution). */
static real texel_hysteresis(real alpha, real change) {
  real a = alpha;
  if (change > 0.25) a = fmax((real)0.0, a - (real)0.15);
  if (change > 0.8) a = 0.0;
  return a;
}

void orc_blend_probe_k(int32_t n, const double* omega, const double* rgb, const double* rgb_kappa, const double* d,
                       const double* d_kappa, double cos_power, double alpha_irr, double alpha_dist, double gamma,
                       int32_t thresholds, double* irr, double* dist, double* irr_k, double* dist_k) {
  for (int32_t y = 1; y <= 6; y++)
    for (int32_t x = 1; x <= 6; x++) {
      real nt[3], W = 0, acc[3] = {0, 0, 0};
      texel_direction_r(8, x, y, nt);
      const double ntd[3] = {nt[0], nt[1], nt[2]};
      for (int32_t r = 0; r < n; r++) {
        real om[3];
        load3r(omega + 3 * r, om);
        real w = fmax((real)0.0, dot3r(nt, om));
        W += w;
        for (int c = 0; c < 3; c++) acc[c] += w * (real)rgb[3 * r + c];
      }
      if (!(W > 0.0)) continue;
      double* t = &irr[(y * 8 + x) * 3];
      real nv[3], enc[3];
      double kn[3], kenc[3];
      for (int c = 0; c < 3; c++) {
        nv[c] = acc[c] / W;
        /* Section "Perception-based exponential encoding": the stored value
           is the new mean raised to 1/gamma; the hysteresis then blends in
           the encoded domain */
        enc[c] = gamma != 1.0 ? pow(fmax(nv[c], (real)0.0), (real)(1.0 / gamma)) : nv[c];
        if (irr_k) {
          double kw = 0.0, kr = 0.0;
          for (int32_t r = 0; r < n; r++) {
            double cw = dot3(ntd, omega + 3 * r);
            double w = fmax(0.0, cw);
            if (cw > -8.0 * U32) kw += fabs(rgb[3 * r + c] - nv[c]) * 8.0;
            if (rgb_kappa) kr += w * rgb_kappa[3 * r + c];
          }
          kn[c] = kw / W + kr / W + 8.0 * fabs((double)nv[c]);
          if (gamma != 1.0) {
            /* the encoded value's range over the linear value's error bound */
            double e = 8.0 * U32 * kn[c];
            double hi = pow(fmax((double)nv[c], 0.0) + e, 1.0 / gamma), lo = pow(fmax(nv[c] - e, 0.0), 1.0 / gamma);
            kenc[c] = fmax(hi - enc[c], enc[c] - lo) / (8.0 * U32) + 8.0 * enc[c];
          } else {
            kenc[c] = kn[c];
          }
        }
      }
      real a = alpha_irr;
      double flip = 0.0;
      if (thresholds) {
        real change = 0.0;
        for (int c = 0; c < 3; c++) change = fmax(change, fabs(enc[c] - (real)t[c]));
        a = texel_hysteresis(alpha_irr, change);
        if (irr_k) {
          /* a float32 evaluation may see the change on the other side of a
             threshold: the jump between the two outcomes enters the
             sensitivity */
          double dc = 0.0;
          for (int c = 0; c < 3; c++) dc = fmax(dc, 8.0 * U32 * (kenc[c] + irr_k[(y * 8 + x) * 3 + c]) + 4.0 * U32);
          double a_lo = texel_hysteresis(alpha_irr, change + dc), a_hi = texel_hysteresis(alpha_irr, change - dc);
          flip = a_hi - a_lo;
        }
      }
      for (int c = 0; c < 3; c++) {
        if (irr_k) {
          double* kt = &irr_k[(y * 8 + x) * 3 + c];
          *kt = a * (*kt) + (1.0 - a) * kenc[c] + 4.0 * fabs(t[c]) + flip * fabs(t[c] - enc[c]) / (8.0 * U32);
        }
        real tc = t[c];
        t[c] = a * tc + (1 - a) * enc[c];
      }
    }
  for (int32_t y = 1; y <= 14; y++)
    for (int32_t x = 1; x <= 14; x++) {
      real nt[3], W = 0, m1 = 0, m2 = 0;
      texel_direction_r(16, x, y, nt);
      const double ntd[3] = {nt[0], nt[1], nt[2]};
      for (int32_t r = 0; r < n; r++) {
        real om[3];
        load3r(omega + 3 * r, om);
        real w = pow(fmax((real)0.0, dot3r(nt, om)), (real)cos_power);
        real dr = d[r];
        W += w;
        m1 += w * dr;
        m2 += w * dr * dr;
      }
      if (W > 0.0) {
        double* t = &dist[(y * 16 + x) * 2];
        real n1 = m1 / W, n2 = m2 / W;
        if (dist_k) {
          double k1 = 0.0, k2 = 0.0;
          for (int32_t r = 0; r < n; r++) {
            double cw = dot3(ntd, omega + 3 * r);
            if (cw <= -8.0 * U32) continue;
            /* |dw/dc| * 8u with w = c^p */
            double dw = cos_power * pow(fmax(cw, 8.0 * U32), cos_power - 1.0) * 8.0;
            k1 += fabs(d[r] - n1) * dw;
            k2 += fabs(d[r] * d[r] - n2) * dw;
            if (d_kappa && cw > 0.0) {
              /* the ray's own distance error */
              double w = pow(cw, cos_power);
              k1 += w * d_kappa[r];
              k2 += w * 2.0 * fabs(d[r]) * d_kappa[r];
            }
          }
          double* kt = &dist_k[(y * 16 + x) * 2];
          kt[0] = alpha_dist * kt[0] + (1.0 - alpha_dist) * (k1 / W + 8.0 * fabs((double)n1)) + 4.0 * fabs(t[0]);
          kt[1] = alpha_dist * kt[1] + (1.0 - alpha_dist) * (k2 / W + 8.0 * fabs((double)n2)) + 4.0 * fabs(t[1]);
        }
        real ad = alpha_dist, t0 = t[0], t1 = t[1];
        t[0] = ad * t0 + (1 - ad) * n1;
        t[1] = ad * t1 + (1 - ad) * n2;
      }
    }
  for (int32_t y = 0; y < 8; y++)
    for (int32_t x = 0; x < 8; x++) {
      int32_t sx, sy;
      orc_border_source(8, x, y, &sx, &sy);
      if (sx != x || sy != y)
        for (int c = 0; c < 3; c++) {
          irr[(y * 8 + x) * 3 + c] = irr[(sy * 8 + sx) * 3 + c];
          if (irr_k) irr_k[(y * 8 + x) * 3 + c] = irr_k[(sy * 8 + sx) * 3 + c];
        }
    }
  for (int32_t y = 0; y < 16; y++)
    for (int32_t x = 0; x < 16; x++) {
      int32_t sx, sy;
      orc_border_source(16, x, y, &sx, &sy);
      if (sx != x || sy != y)
        for (int c = 0; c < 2; c++) {
          dist[(y * 16 + x) * 2 + c] = dist[(sy * 16 + sx) * 2 + c];
          if (dist_k) dist_k[(y * 16 + x) * 2 + c] = dist_k[(sy * 16 + sx) * 2 + c];
        }
    }
}

/* ------------------------------------------------------------------- query */
/* smallest and largest value of the four bilinear taps (diagnostics for the
   float32 sensitivity estimate only) */
static void footprint_range(const double* tile, int32_t m, int32_t nch, const double v[3], double* lo, double* hi) {
  int32_t k = m - 2;
  double p[2];
  orc_oct_encode(v, p);
  double cx = 1.0 + (0.5 * p[0] + 0.5) * k - 0.5;
  double cy = 1.0 + (0.5 * p[1] + 0.5) * k - 0.5;
  int32_t x0 = (int32_t)floor(cx), y0 = (int32_t)floor(cy);
  if (x0 < 0) x0 = 0;
  if (x0 > k) x0 = k;
  if (y0 < 0) y0 = 0;
  if (y0 > k) y0 = k;
  for (int c = 0; c < nch; c++) {
    double a = tile[(y0 * m + x0) * nch + c], b = tile[(y0 * m + x0 + 1) * nch + c];
    double cc = tile[((y0 + 1) * m + x0) * nch + c], dd = tile[((y0 + 1) * m + x0 + 1) * nch + c];
    lo[c] = fmin(fmin(a, b), fmin(cc, dd));
    hi[c] = fmax(fmax(a, b), fmax(cc, dd));
  }
}
static int64_t vol_probes(const orc_volume* V) { return (int64_t)V->counts[0] * V->counts[1] * V->counts[2]; }

static int64_t wrap(int64_t i, int64_t n) { return ((i % n) + n) % n; }

/* Logical grid index of storage slot q (Section "Tracking Windows": a
   tracking volume is a circular buffer; the slot of logical probe i along an
   axis is (i + phase) mod n). */
static void logical_index(const orc_volume* V, int64_t q, int64_t g[3]) {
  int64_t s[3] = {q % V->counts[0], (q / V->counts[0]) % V->counts[1], q / ((int64_t)V->counts[0] * V->counts[1])};
  for (int a = 0; a < 3; a++) g[a] = wrap(s[a] - V->phase[a], V->counts[a]);
}

/* Storage slot of logical probe (i, j, k). */
static int64_t storage_index(const orc_volume* V, int64_t i, int64_t j, int64_t k) {
  return wrap(i + V->phase[0], V->counts[0]) +
         (int64_t)V->counts[0] * (wrap(j + V->phase[1], V->counts[1]) + (int64_t)V->counts[1] * wrap(k + V->phase[2], V->counts[2]));
}

static void probe_position_r(const orc_volume* V, int64_t q, real P[3]) {
  int64_t g[3];
  logical_index(V, q, g);
  for (int a = 0; a < 3; a++) {
    P[a] = (real)V->origin[a] + (real)g[a] * (real)V->spacing[a];
    if (V->offsets) P[a] += (real)V->offsets[q * 3 + a];
  }
}

static void probe_position(const orc_volume* V, int64_t q, double P[3]) {
  real Pr[3];
  probe_position_r(V, q, Pr);
  for (int a = 0; a < 3; a++) P[a] = Pr[a];
}

/* Section "Multiple Probe Volumes": a volume's weight falls linearly from 1
   to 0 over its last grid cell along each axis (product over axes).  For a
   volume that tracks the camera the transition region is tightened by one
   cell and centred on the camera. */
static real volume_weight(const orc_volume* V, const real X[3]) {
  real wv = 1.0;
  for (int a = 0; a < 3; a++) {
    real sp = V->spacing[a];
    if (V->tracking) {
      real h = (real)0.5 * (real)(V->counts[a] - 1) - 1;
      wv *= clampr(h - fabs(X[a] - (real)V->camera[a]) / sp, 0.0, 1.0);
    } else {
      real u = (X[a] - (real)V->origin[a]) / sp;
      wv *= clampr(fmin(u, (real)(V->counts[a] - 1) - u), 0.0, 1.0);
    }
  }
  return wv;
}

static int sampled_state(uint8_t s) { return s == ORC_AWAKE || s == ORC_VIGILANT; }

/* Section "Probe Query": the 8 probes of the cage around X, each weighted by
   trilinear x backface x visibility; the visibility test (one-sided
   Chebyshev on the mean/mean^2 distance texels) is taken at X moved by the
   self-shadow bias of Eq. 1.  Result: normalised weighted sum of the
   irradiance texels sampled in direction n.  kap receives the absolute
   sensitivity of the result to float32 rounding (units of 2^-24). */
static void volume_query(const orc_volume* V, int64_t base, const real X[3], const real n[3],
                         const real wo[3], const real look[3], real out[3], double kap[3], int32_t* cage,
                         int32_t* ncage) {
  real u[3], f[3];
  int64_t g[3];
  real D = fmin((real)V->spacing[0], fmin((real)V->spacing[1], (real)V->spacing[2]));
  real Xb[3];
  for (int a = 0; a < 3; a++) {
    u[a] = (X[a] - (real)V->origin[a]) / (real)V->spacing[a];
    real fl = floor(u[a]);
    g[a] = (int64_t)clampr(fl, 0.0, (real)(V->counts[a] - 2));
    f[a] = clampr(u[a] - (real)g[a], 0.0, 1.0);
    Xb[a] = X[a] + ((real)0.2 * n[a] + (real)0.8 * wo[a]) * ((real)0.75 * D) * (real)V->bias;
  }
  real w[8], e[8][3], W = 0;
  double ek[8][3], sens[8];
  int32_t ids[8];
  int used = 0;
  for (int c = 0; c < 8; c++) {
    int cb[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    int64_t q = storage_index(V, g[0] + cb[0], g[1] + cb[1], g[2] + cb[2]);
    if (!sampled_state(V->states[q])) continue;
    real wt = 1.0;
    for (int a = 0; a < 3; a++) wt *= cb[a] ? f[a] : 1 - f[a];
    real P[3], toP[3];
    probe_position_r(V, q, P);
    sub3r(P, X, toP);
    normalize3r(toP);
    real h = (1 + dot3r(n, toP)) * (real)0.5;
    real wb = h * h + (real)0.2;
    real z[3];
    sub3r(Xb, P, z);
    real r = len3r(z);
    real wv = 1.0;
    double s = 8.0;
    if (r > 0.0) {
      real zd[3] = {z[0] / r, z[1] / r, z[2] / r}, mm[2];
      sample_tile_r(V->dist + q * 16 * 16 * 2, 16, 2, zd, mm);
      if (r > mm[0]) {
        real var = fmax(mm[1] - mm[0] * mm[0], (real)0.0);
        real dl = r - mm[0];
        real ch = var / (var + dl * dl);
        wv = pow(ch, (real)V->cheb_power);
        /* relative float32 sensitivity of the Chebyshev weight (units of u):
           the bilinear position (k * few u of a texel) and the rounding of
           mu, mu2 and r enter through the cancellations mu2 - mu^2, r - mu */
        double zdd[3] = {zd[0], zd[1], zd[2]}, lo[2], hi[2];
        footprint_range(V->dist + q * 16 * 16 * 2, 16, 2, zdd, lo, hi);
        double dmu = 4.0 * fabs((double)mm[0]) + 32.0 * (hi[0] - lo[0]);
        double dmu2 = 4.0 * fabs((double)mm[1]) + 32.0 * (hi[1] - lo[1]);
        if (V->dist_kappa) {
          /* the float32 atlas itself differs by its texels' sensitivity */
          double kk[2];
          orc_sample_tile(V->dist_kappa + q * 16 * 16 * 2, 16, 2, zdd, kk);
          dmu += kk[0];
          dmu2 += kk[1];
        }
        double dvar = dmu2 + 2.0 * fabs((double)mm[0]) * dmu + 4.0 * (fabs((double)mm[1]) + (double)mm[0] * mm[0]);
        double ddl = 4.0 * r + dmu;
        if (var > 0.0)
          s += V->cheb_power * (1.0 - ch) * (dvar / var + 2.0 * ddl / dl);
        else
          s = INFINITY; /* zero variance: float32 rounding decides the weight */
      }
    }
    ids[used] = (int32_t)(base + q);
    w[used] = wt * wb * wv;
    sens[used] = s;
    sample_tile_r(V->irr + q * 8 * 8 * 3, 8, 3, look, e[used]);
    if (V->irr_kappa) {
      double lk[3] = {look[0], look[1], look[2]};
      orc_sample_tile(V->irr_kappa + q * 8 * 8 * 3, 8, 3, lk, ek[used]);
    } else {
      ek[used][0] = ek[used][1] = ek[used][2] = 0.0;
    }
    if (V->gamma != 1.0f) {
      /* Section "Perception-based exponential encoding": each probe's sample
         is decoded to the power gamma/2, so the cage blend runs on a
         gamma-2 curve; the normalised result is squared back below */
      real h2 = (real)0.5 * (real)V->gamma;
      for (int k = 0; k < 3; k++) {
        real ev = fmax(e[used][k], (real)0.0);
        real dec = pow(ev, h2);
        double ee = (16.0 * fabs((double)e[used][k]) + ek[used][k]) * U32;
        double hi = pow((double)ev + ee, (double)h2), lo = pow(fmax((double)ev - ee, 0.0), (double)h2);
        ek[used][k] = fmax(hi - dec, dec - lo) / U32;
        e[used][k] = dec;
      }
    }
    W += w[used];
    used++;
  }
  for (int c = 0; c < 3; c++) { out[c] = 0.0; kap[c] = 0.0; }
  if (ncage) *ncage = 0;
  const int sq = V->gamma != 1.0f;
  if (!(W > 0.0)) {
    /* no visible probe: float32 may find tiny positive weights */
    for (int i = 0; i < used; i++)
      for (int c = 0; c < 3; c++)
        kap[c] = fmax(kap[c], (sq ? (double)e[i][c] * e[i][c] : fabs((double)e[i][c])) / U32);
    return;
  }
  for (int i = 0; i < used; i++)
    for (int c = 0; c < 3; c++) out[c] += w[i] * e[i][c];
  for (int c = 0; c < 3; c++) out[c] /= W;
  /* a weight whose relative float32 sensitivity reaches 1 (its Chebyshev
     variance below the float32 resolution of mu2 - mu^2) may be zero in
     float32; if that holds for every probe that carries weight, float32 may
     find no probe with weight, and the query is then zero (the mirror of
     the W = 0 case above) */
  int all_fragile = 1;
  for (int i = 0; i < used; i++)
    if (w[i] > 0.0 && !(sens[i] * U32 >= 1.0)) all_fragile = 0;
  for (int i = 0; i < used; i++) {
    for (int c = 0; c < 3; c++) {
      double dv = fabs((double)e[i][c] - (double)out[c]);
      double term = isinf(sens[i]) ? (dv > 0 ? dv / U32 : 0.0) : ((double)w[i] / W) * dv * sens[i];
      kap[c] += term + ((double)w[i] / W) * (16.0 * fabs((double)e[i][c]) + ek[i][c]);
    }
    if (w[i] > 0.0 && cage && ncage && *ncage < 8) cage[(*ncage)++] = ids[i];
  }
  if (all_fragile)
    for (int c = 0; c < 3; c++) kap[c] += fabs((double)out[c]) / U32;
  if (sq)
    for (int c = 0; c < 3; c++) {
      kap[c] = 2.0 * fabs((double)out[c]) * kap[c] + 8.0 * (double)out[c] * out[c];
      out[c] = out[c] * out[c];
    }
}

/* Section "Multiple Probe Volumes": volumes are visited from most to least
   dense; a volume's weight falls linearly from 1 to 0 across its last grid
   cell on every axis (product over axes); weights accumulate until they
   reach 1; the sparsest volume takes whatever weight remains.  `look`: the
   direction the probes' texels are sampled in (the normal for irradiance;
   see orc_query_look). */
static void query_look_r(const orc_volume* vols, int32_t nvol, const real X[3], const real n[3], const real wo[3],
                         const real look[3], real out[3], double kappa[3], int32_t* cage, int32_t* n_cage) {
  real Wt = 0.0;
  int64_t base = 0;
  for (int c = 0; c < 3; c++) { out[c] = 0.0; kappa[c] = 0.0; }
  if (n_cage) *n_cage = 0;
  for (int32_t v = 0; v < nvol; v++) {
    const orc_volume* V = &vols[v];
    if (Wt >= 1.0) break;
    real wv = volume_weight(V, X);
    real wuse = (v == nvol - 1) ? 1 - Wt : fmin(wv, 1 - Wt);
    if (wuse > 0.0) {
      real ev[3];
      double kv[3];
      int32_t cg[8], nc = 0;
      volume_query(V, base, X, n, wo, look, ev, kv, cg, &nc);
      for (int c = 0; c < 3; c++) {
        out[c] += wuse * ev[c];
        kappa[c] += wuse * kv[c] + 4.0 * fabs((double)(wuse * ev[c]));
      }
      if (cage && n_cage)
        for (int i = 0; i < nc && *n_cage < ORC_CAGE; i++) cage[(*n_cage)++] = cg[i];
      Wt += wuse;
    }
    base += vol_probes(V);
  }
}

void orc_query(const orc_volume* vols, int32_t nvol, const double X[3], const double n[3],
               const double wo[3], double out[3], double kappa[3], int32_t* cage, int32_t* n_cage) {
  orc_query_look(vols, nvol, X, n, wo, n, out, kappa, cage, n_cage);
}

/* The query with the probes' texels sampled in direction `look` instead of
   the normal (the cage weights still use X, n and w_o): the probes' filtered
   radiance around `look`. */
void orc_query_look(const orc_volume* vols, int32_t nvol, const double X[3], const double n[3],
                    const double wo[3], const double look[3], double out[3], double kappa[3], int32_t* cage,
                    int32_t* n_cage) {
  real Xr[3], nr[3], wr[3], lr[3], o[3];
  load3r(X, Xr);
  load3r(n, nr);
  load3r(wo, wr);
  load3r(look, lr);
  query_look_r(vols, nvol, Xr, nr, wr, lr, o, kappa, cage, n_cage);
  for (int c = 0; c < 3; c++) out[c] = o[c];
}

void orc_query_batch(const orc_volume* vols, int32_t nvol, int64_t nq, const float* pos,
                     const float* nrm, const float* view, double* out, double* kappa) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < nq; i++) {
    double X[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    double n[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
    double w[3] = {view[3 * i], view[3 * i + 1], view[3 * i + 2]};
    orc_query(vols, nvol, X, n, w, out + 3 * i, kappa + 3 * i, NULL, NULL);
  }
}

/* ----------------------------------------------------------------- shading */
/* Lambertian radiance leaving front-face hit X (geometric normal ng) toward
   -w, given which shadow rays are unblocked (bit l of vis): emission plus
   albedo x (direct irradiance / pi + previous-frame probe irradiance). */
static void front_radiance(const orc_scene* s, const orc_lights* L, const orc_volume* vols, int32_t nvol, int32_t m,
                           const real X[3], const real ng[3], const real w[3], uint32_t vis, real rgb[3],
                           double kq[3], int32_t* cage, int32_t* n_cage) {
  real direct[3] = {0, 0, 0};
  real xmax = fmax(fabs(X[0]), fmax(fabs(X[1]), fabs(X[2])));
  real eps = (real)1e-4 * fmax((real)1.0, xmax);
  real Xs[3] = {X[0] + eps * ng[0], X[1] + eps * ng[1], X[2] + eps * ng[2]};
  int32_t li = 0;
  for (int32_t l = 0; l < L->n_dir; l++, li++) {
    if (!(vis >> li & 1u)) continue;
    real dl[3] = {L->dir_to_light[3 * l], L->dir_to_light[3 * l + 1], L->dir_to_light[3 * l + 2]};
    real c = dot3r(ng, dl);
    for (int k = 0; k < 3; k++) direct[k] += (real)L->dir_irradiance[3 * l + k] * c;
  }
  for (int32_t l = 0; l < L->n_point; l++, li++) {
    if (!(vis >> li & 1u)) continue;
    real u[3] = {L->point_pos[3 * l] - Xs[0], L->point_pos[3 * l + 1] - Xs[1], L->point_pos[3 * l + 2] - Xs[2]};
    real dist = len3r(u);
    real c = dot3r(ng, u) / dist;
    for (int k = 0; k < 3; k++) direct[k] += (real)L->point_intensity[3 * l + k] * c / (dist * dist);
  }
  real wo[3] = {-w[0], -w[1], -w[2]}, ind[3] = {0, 0, 0};
  for (int k = 0; k < 3; k++) kq[k] = 0.0;
  if (nvol > 0) query_look_r(vols, nvol, X, ng, wo, ng, ind, kq, cage, n_cage);
  for (int k = 0; k < 3; k++)
    rgb[k] = (real)s->emission[m * 3 + k] + (real)s->albedo[m * 3 + k] * (direct[k] / (real)M_PI + ind[k]);
}

/* Shadow rays of a front-face hit X (geometric normal ng) toward every
   light on its front side, from the hit lifted off the surface; any
   triangle, either side, occludes.  Sets bit l of vis for an unblocked light
   and ORC_F_SHADOW in flags for an ambiguous shadow ray. */
static void hit_visibility(const orc_scene* s, const orc_lights* L, const real X[3], const real ng[3],
                           uint32_t* vis, int32_t* flags) {
  real xmax = fmax(fabs(X[0]), fmax(fabs(X[1]), fabs(X[2])));
  real eps = (real)1e-4 * fmax((real)1.0, xmax);
  real Xs[3] = {X[0] + eps * ng[0], X[1] + eps * ng[1], X[2] + eps * ng[2]};
  double Xsd[3] = {Xs[0], Xs[1], Xs[2]};
  int32_t li = 0;
  for (int32_t l = 0; l < L->n_dir; l++, li++) {
    real dl[3] = {L->dir_to_light[3 * l], L->dir_to_light[3 * l + 1], L->dir_to_light[3 * l + 2]};
    if (dot3r(ng, dl) <= 0.0) continue;
    double dld[3] = {dl[0], dl[1], dl[2]};
    int amb = 0;
    if (!occluded(s, Xsd, dld, INFINITY, &amb)) *vis |= 1u << li;
    if (amb) *flags |= ORC_F_SHADOW;
  }
  for (int32_t l = 0; l < L->n_point; l++, li++) {
    real u[3] = {L->point_pos[3 * l] - Xs[0], L->point_pos[3 * l + 1] - Xs[1], L->point_pos[3 * l + 2] - Xs[2]};
    real dist = len3r(u);
    if (!(dist > 0.0)) continue;
    real uh[3] = {u[0] / dist, u[1] / dist, u[2] / dist};
    if (dot3r(ng, uh) <= 0.0) continue;
    double uhd[3] = {uh[0], uh[1], uh[2]};
    int amb = 0;
    if (!occluded(s, Xsd, uhd, dist * (1.0 - 1e-6), &amb)) *vis |= 1u << li;
    if (amb) *flags |= ORC_F_SHADOW;
  }
}

/* geometric normal of triangle t (counter-clockwise front face) */
static void tri_normal_r(const orc_scene* s, int32_t t, real ng[3]) {
  real v0[3], v1[3], v2[3], e1[3], e2[3];
  load3r(tri_v(s, t, 0), v0);
  load3r(tri_v(s, t, 1), v1);
  load3r(tri_v(s, t, 2), v2);
  sub3r(v1, v0, e1);
  sub3r(v2, v0, e2);
  cross3r(e1, e2, ng);
  normalize3r(ng);
}

/* Section "Probe Update" (hit shading) and the backface rule of the
   self-shadow-bias section: a miss sees the sky at the distance clamp; a
   backface records radiance 0 and 20 % of its distance; a front face is
   shaded Lambertian with shadowed direct light, its emission and the
   previous frame's probe irradiance at the hit. */
/* float32 sensitivity (units of u) of a ray's recorded distance: the hit
   distance's error along the ray, t (8 / |cos| + 16) from the direction and
   the arithmetic plus 32 |o| / |cos| from the rounding of the origin's
   coordinates (|o| its largest), scaled by 0.2 for a backface, unless the
   distance sits at the clamp beyond that error */
static double ray_distance_kappa(const orc_ray_record* rr, double dmax, double omag) {
  if (rr->tri < 0) return 0.0;
  double c = fmax(rr->cosi, 1e-6);
  double terr = rr->t * (8.0 / c + 16.0) + 32.0 * omag / c;
  int back = rr->d == fmin(0.2 * rr->t, dmax) && 0.2 * rr->t < rr->t && rr->d < rr->t;
  double tt = back ? 0.2 * rr->t : rr->t, err = back ? 0.2 * terr : terr;
  return tt <= dmax * (1.0 + 4.0 * U32) + err * U32 ? err : 0.0;
}

static void shade_ray_body(const orc_scene* s, const orc_lights* L, const orc_volume* vols, int32_t nvol,
                           const double o[3], const double w[3], double dmax, uint8_t force, int32_t force_tri,
                           uint32_t force_vis, orc_ray_record* rec);

static void shade_ray_impl(const orc_scene* s, const orc_lights* L, const orc_volume* vols, int32_t nvol,
                           const double o[3], const double w[3], double dmax, uint8_t force, int32_t force_tri,
                           uint32_t force_vis, orc_ray_record* rec) {
  shade_ray_body(s, L, vols, nvol, o, w, dmax, force, force_tri, force_vis, rec);
  rec->d_kappa = ray_distance_kappa(rec, dmax, fmax(fabs(o[0]), fmax(fabs(o[1]), fabs(o[2]))));
}

static void shade_ray_body(const orc_scene* s, const orc_lights* L, const orc_volume* vols, int32_t nvol,
                           const double o[3], const double w[3], double dmax, uint8_t force, int32_t force_tri,
                           uint32_t force_vis, orc_ray_record* rec) {
  orc_hit h;
  orc_trace(s, o, w, 0, &h);
  memset(rec, 0, sizeof(*rec));
  for (int i = 0; i < ORC_CAGE; i++) rec->cage[i] = -1;
  if (force & 1) {
    /* the hit is given (another tracer's decision on a ray this oracle
       flags): a miss, or triangle force_tri at the exact distance of its
       plane along the ray */
    h.flags |= ORC_F_FORCED;
    if (force_tri < 0 || force_tri >= s->nt) {
      h.tri = -1;
      h.t = INFINITY;
    } else if (force_tri != h.tri) {
      double t, bmin;
      if (plane_hit(s, force_tri, o, w, &t, &bmin) && t > 0.0) {
        h.tri = force_tri;
        h.t = t;
      } else {
        h.flags |= ORC_F_FORCE_INVALID;
      }
    }
  }
  rec->tri = h.tri;
  rec->t = h.t;
  rec->flags = h.flags;
  if (h.tri < 0) {
    for (int c = 0; c < 3; c++) rec->rgb[c] = L->sky[c];
    rec->d = dmax;
    return;
  }
  real ng[3], wr[3], orr[3];
  tri_normal_r(s, h.tri, ng);
  load3r(w, wr);
  load3r(o, orr);
  double ngd[3] = {ng[0], ng[1], ng[2]};
  rec->cosi = fabs(dot3(w, ngd)) / len3(w);
  real t = h.t;
  if (dot3r(wr, ng) > 0.0) {
    rec->d = fmin((real)0.2 * t, (real)dmax);
    return;
  }
  rec->d = fmin(t, (real)dmax);
  real X[3];
  for (int a = 0; a < 3; a++) X[a] = orr[a] + t * wr[a];
  int32_t m = s->material[h.tri];
  hit_visibility(s, L, X, ng, &rec->vis, &rec->flags);
  if (force & 2) {
    rec->vis = force_vis;
    rec->flags |= ORC_F_FORCED;
  }
  double kq[3];
  real rgb[3];
  front_radiance(s, L, vols, nvol, m, X, ng, wr, rec->vis, rgb, kq, rec->cage, &rec->n_cage);
  for (int k = 0; k < 3; k++) rec->rgb[k] = rgb[k];
  /* float32 sensitivity: the query's own, rounding of the sum, and, by
     finite differences of the shading at the scale of each error, (i) the
     hit distance's error along the ray (about t u / |cos|), (ii) the
     rounding of the hit point's coordinates (about 2 u of the largest
     coordinate, per axis) and (iii) the direction error of a float32
     normal (about 4 u (1 + |e1| |e2| / |e1 x e2|), along two tangents) */
  double ep = fmin(1e-2, U32 * (8.0 / fmax(rec->cosi, 1e-6) + 16.0));
  real X2[3], rgb2[3];
  double kq2[3], fd[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < 3; a++) X2[a] = orr[a] + t * (real)(1.0 + ep) * wr[a];
  front_radiance(s, L, vols, nvol, m, X2, ng, wr, rec->vis, rgb2, kq2, NULL, NULL);
  for (int k = 0; k < 3; k++) fd[k] += fabs((double)rgb2[k] - rec->rgb[k]);
  double xmag = 0.0;
  for (int a = 0; a < 3; a++) xmag = fmax(xmag, fmax(fabs((double)X[a]), fabs(o[a])));
  for (int a = 0; a < 3; a++) {
    for (int b = 0; b < 3; b++) X2[b] = X[b];
    X2[a] += (real)(2.0 * U32 * xmag);
    front_radiance(s, L, vols, nvol, m, X2, ng, wr, rec->vis, rgb2, kq2, NULL, NULL);
    for (int k = 0; k < 3; k++) fd[k] += fabs((double)rgb2[k] - rec->rgb[k]);
  }
  {
    double e1[3], e2[3], c[3], tg[2][3];
    sub3(tri_v(s, h.tri, 1), tri_v(s, h.tri, 0), e1);
    sub3(tri_v(s, h.tri, 2), tri_v(s, h.tri, 0), e2);
    cross3(e1, e2, c);
    double en = 4.0 * U32 * (1.0 + len3(e1) * len3(e2) / fmax(len3(c), 1e-30));
    /* two unit tangents of the normal */
    int ax = fabs(ngd[0]) < fabs(ngd[1]) ? (fabs(ngd[0]) < fabs(ngd[2]) ? 0 : 2) : (fabs(ngd[1]) < fabs(ngd[2]) ? 1 : 2);
    double ea[3] = {0.0, 0.0, 0.0};
    ea[ax] = 1.0;
    cross3(ngd, ea, tg[0]);
    normalize3(tg[0]);
    cross3(ngd, tg[0], tg[1]);
    for (int j = 0; j < 2; j++) {
      real n2[3];
      for (int b = 0; b < 3; b++) n2[b] = (real)(ngd[b] + en * tg[j][b]);
      normalize3r(n2);
      front_radiance(s, L, vols, nvol, m, X, n2, wr, rec->vis, rgb2, kq2, NULL, NULL);
      for (int k = 0; k < 3; k++) fd[k] += fabs((double)rgb2[k] - rec->rgb[k]);
    }
  }
  for (int k = 0; k < 3; k++) rec->kappa[k] = s->albedo[m * 3 + k] * kq[k] + 8.0 * fabs(rec->rgb[k]) + fd[k] / U32;
}

void orc_shade_ray(const orc_scene* s, const orc_lights* L, const orc_volume* vols, int32_t nvol,
                   const double o[3], const double w[3], double dmax, orc_ray_record* rec) {
  shade_ray_impl(s, L, vols, nvol, o, w, dmax, 0, -1, 0, rec);
}

/* Section "Second Order Glossy": the mirror reflection ray of a surface
   point X (normal n, direction toward the viewer v) from X lifted off the
   surface; its hit is shaded as a probe-ray hit (emission, albedo times
   direct light over pi plus the probes' irradiance) plus the hit material's
   mirror reflectance times the probes' filtered radiance in the hit's own
   mirror direction -- the second and later glossy bounces come from the
   probes instead of further rays.  A miss sees the sky; a backface is
   black.  kappa: float32 sensitivity as for a probe ray. */
static void glossy_front(const orc_scene* s, const orc_lights* L, const orc_volume* vols, int32_t nvol, int32_t m,
                         const real Y[3], const real ng[3], const real r[3], uint32_t vis, real rgb[3],
                         double kap[3], int32_t* cage, int32_t* n_cage) {
  double kq[3], kg[3];
  front_radiance(s, L, vols, nvol, m, Y, ng, r, vis, rgb, kq, cage, n_cage);
  real c = dot3r(ng, r);
  real r2[3] = {r[0] - (real)2.0 * c * ng[0], r[1] - (real)2.0 * c * ng[1], r[2] - (real)2.0 * c * ng[2]};
  real wo[3] = {-r[0], -r[1], -r[2]}, g[3];
  query_look_r(vols, nvol, Y, ng, wo, r2, g, kg, NULL, NULL);
  for (int k = 0; k < 3; k++) {
    rgb[k] += (real)s->specular[m * 3 + k] * g[k];
    kap[k] = s->albedo[m * 3 + k] * kq[k] + s->specular[m * 3 + k] * kg[k];
  }
}

void orc_glossy(const orc_scene* s, const orc_lights* L, const orc_volume* vols, int32_t nvol, const double X[3],
                const double n[3], const double v[3], orc_ray_record* rec) {
  real Xr[3], nr[3], vr[3];
  load3r(X, Xr);
  load3r(n, nr);
  load3r(v, vr);
  real c = dot3r(nr, vr);
  real r[3] = {(real)2.0 * c * nr[0] - vr[0], (real)2.0 * c * nr[1] - vr[1], (real)2.0 * c * nr[2] - vr[2]};
  normalize3r(r);
  real xmax = fmax(fabs(Xr[0]), fmax(fabs(Xr[1]), fabs(Xr[2])));
  real eps = (real)1e-4 * fmax((real)1.0, xmax);
  real o[3] = {Xr[0] + eps * nr[0], Xr[1] + eps * nr[1], Xr[2] + eps * nr[2]};
  double od[3] = {o[0], o[1], o[2]}, rd[3] = {r[0], r[1], r[2]};
  orc_hit h;
  orc_trace(s, od, rd, 0, &h);
  memset(rec, 0, sizeof(*rec));
  for (int i = 0; i < ORC_CAGE; i++) rec->cage[i] = -1;
  rec->tri = h.tri;
  rec->t = h.t;
  rec->flags = h.flags;
  if (h.tri < 0) {
    for (int k = 0; k < 3; k++) rec->rgb[k] = L->sky[k];
    return;
  }
  real ng[3];
  tri_normal_r(s, h.tri, ng);
  double ngd[3] = {ng[0], ng[1], ng[2]};
  rec->cosi = fabs(dot3(rd, ngd));
  if (dot3r(r, ng) > 0.0) return;   /* backface: black */
  real t = h.t, Y[3];
  for (int a = 0; a < 3; a++) Y[a] = o[a] + t * r[a];
  int32_t m = s->material[h.tri];
  hit_visibility(s, L, Y, ng, &rec->vis, &rec->flags);
  double kap[3];
  real rgb[3];
  glossy_front(s, L, vols, nvol, m, Y, ng, r, rec->vis, rgb, kap, rec->cage, &rec->n_cage);
  for (int k = 0; k < 3; k++) rec->rgb[k] = rgb[k];
  /* the hit point's float32 error along the ray, and the reflection
     direction's (about u per component over the distance t) */
  double ep = fmin(1e-2, U32 * (8.0 / fmax(rec->cosi, 1e-6) + 16.0 + 8.0 / fmax(h.t, 1e-6)));
  real Y2[3], rgb2[3];
  double kap2[3];
  for (int a = 0; a < 3; a++) Y2[a] = o[a] + t * (real)(1.0 + ep) * r[a];
  glossy_front(s, L, vols, nvol, m, Y2, ng, r, rec->vis, rgb2, kap2, NULL, NULL);
  for (int k = 0; k < 3; k++) rec->kappa[k] = kap[k] + 8.0 * fabs(rec->rgb[k]) + fabs((double)rgb2[k] - rec->rgb[k]) / U32;
}

void orc_glossy_batch(const orc_scene* s, const orc_lights* L, const orc_volume* vols, int32_t nvol, int64_t n,
                      const float* pos, const float* nrm, const float* view, orc_ray_record* recs) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; i++) {
    double X[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    double nn[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
    double v[3] = {view[3 * i], view[3 * i + 1], view[3 * i + 2]};
    orc_glossy(s, L, vols, nvol, X, nn, v, &recs[i]);
  }
}

/* ----------------------------------------------------------------- states */
static void expanded_object_boxes(const orc_scene* s, const orc_volume* V, double* lo, double* hi) {
  double D = fmin((double)V->spacing[0], fmin((double)V->spacing[1], (double)V->spacing[2]));
  double bias = 0.75 * D * (double)V->bias;
  for (int32_t o = 1; o <= s->nobj; o++)
    for (int a = 0; a < 3; a++) {
      lo[o * 3 + a] = s->obj_lo[o * 3 + a] - ((double)V->spacing[a] + bias);
      hi[o * 3 + a] = s->obj_hi[o * 3 + a] + ((double)V->spacing[a] + bias);
    }
}

static int inside_any(const orc_scene* s, const double* lo, const double* hi, const double P[3]) {
  for (int32_t o = 1; o <= s->nobj; o++) {
    if (isinf(s->obj_lo[o * 3])) continue;
    int in = 1;
    for (int a = 0; a < 3; a++) in &= (P[a] >= lo[o * 3 + a] && P[a] <= hi[o * 3 + a]);
    if (in) return 1;
  }
  return 0;
}

/* Section "Full Probe Initialization Algorithm", steps 1-2: distance-only
   rays against static geometry; a probe that sees more than 25 % backfaces
   is inside geometry (Off); a front face closer than the probe spacing makes
   it Newly Vigilant, otherwise it sleeps; sleeping probes inside the box of
   a dynamic object (grown by one cell and the self-shadow bias) become Newly
   Awake. */
/* One probe's classification (steps 1-2): K x N distance-only rays against
   static triangles from its position. */
static uint8_t classify_probe(const orc_scene* s, const orc_volume* V, int64_t q, const float* rotations, int32_t K,
                              const double* lo, const double* hi, int32_t* n_back, int32_t* n_flagged,
                              double* t_front) {
  double smax = fmax((double)V->spacing[0], fmax((double)V->spacing[1], (double)V->spacing[2]));
  double Pq[3];
  probe_position(V, q, Pq);
  int32_t back = 0, flagged = 0;
  double tf = INFINITY;
  for (int32_t k = 0; k < K; k++)
    for (int32_t r = 0; r < V->rays; r++) {
      double w[3];
      orc_sf_direction(r, V->rays, rotations + 9 * k, w);
      orc_hit h;
      orc_trace(s, Pq, w, 1, &h);
      if (h.flags) flagged++;
      if (h.tri < 0) continue;
      double e1[3], e2[3], ng[3];
      sub3(tri_v(s, h.tri, 1), tri_v(s, h.tri, 0), e1);
      sub3(tri_v(s, h.tri, 2), tri_v(s, h.tri, 0), e2);
      cross3(e1, e2, ng);
      if (dot3(w, ng) > 0.0) back++;
      else if (h.t < tf) tf = h.t;
    }
  uint8_t st;
  if ((double)back / ((double)K * V->rays) > 0.25) st = ORC_OFF;
  else if (tf < smax) st = ORC_NEWLY_VIGILANT;
  else st = ORC_SLEEPING;
  if (st == ORC_SLEEPING && inside_any(s, lo, hi, Pq)) st = ORC_NEWLY_AWAKE;
  if (n_back) *n_back = back;
  if (n_flagged) *n_flagged = flagged;
  if (t_front) *t_front = tf;
  return st;
}

void orc_classify(const orc_scene* s, orc_volume* vols, int32_t nvol, const float* rotations,
                  int32_t K, int32_t* n_back, int32_t* n_flagged, double* t_front) {
  int64_t base = 0;
  for (int32_t v = 0; v < nvol; v++) {
    orc_volume* V = &vols[v];
    int64_t P = vol_probes(V);
    double* lo = (double*)malloc(sizeof(double) * 3 * (size_t)(s->nobj + 1));
    double* hi = (double*)malloc(sizeof(double) * 3 * (size_t)(s->nobj + 1));
    expanded_object_boxes(s, V, lo, hi);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < P; q++)
      V->states[q] = classify_probe(s, V, q, rotations, K, lo, hi, n_back ? n_back + base + q : NULL,
                                    n_flagged ? n_flagged + base + q : NULL, t_front ? t_front + base + q : NULL);
    free(lo);
    free(hi);
    base += P;
  }
}

/* Section "Tracking Windows": the window follows the camera in whole cells;
   a plane leaving behind the camera is reused for the plane entering in
   front (circular buffer), and its probes start over through the state
   machine (reset texels and offsets, classification). */
void orc_track_volume(const orc_scene* s, orc_volume* V, const float camera[3], const float* rotations, int32_t K,
                      int32_t* shift_out) {
  int64_t lo_new[3], hi_new[3];
  int32_t shift[3];
  for (int a = 0; a < 3; a++) {
    double sp = (double)V->spacing[a];
    double center = (double)V->origin[a] + 0.5 * (double)(V->counts[a] - 1) * sp;
    double d = (double)camera[a] - center;
    int32_t k = 0;
    while (d > sp) {
      k++;
      d -= sp;
    }
    while (d < -sp) {
      k--;
      d += sp;
    }
    shift[a] = k;
    V->origin[a] = (float)((double)V->origin[a] + (double)k * sp);
    V->phase[a] = (int32_t)wrap((int64_t)V->phase[a] + k, V->counts[a]);
    int64_t n = V->counts[a], m = k > 0 ? (k < n ? k : n) : (-k < n ? -k : n);
    if (k > 0) { lo_new[a] = n - m; hi_new[a] = n - 1; }
    else if (k < 0) { lo_new[a] = 0; hi_new[a] = m - 1; }
    else { lo_new[a] = 1; hi_new[a] = 0; }   /* empty */
    V->camera[a] = camera[a];
  }
  if (shift_out)
    for (int a = 0; a < 3; a++) shift_out[a] = shift[a];
  double* blo = (double*)malloc(sizeof(double) * 3 * (size_t)(s->nobj + 1));
  double* bhi = (double*)malloc(sizeof(double) * 3 * (size_t)(s->nobj + 1));
  expanded_object_boxes(s, V, blo, bhi);
  int64_t P = vol_probes(V);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < P; q++) {
    int64_t g[3];
    logical_index(V, q, g);
    int fresh = 0;
    for (int a = 0; a < 3; a++) fresh |= g[a] >= lo_new[a] && g[a] <= hi_new[a];
    if (!fresh) continue;
    for (int i = 0; i < 192; i++) V->irr[q * 192 + i] = 0.0;
    for (int i = 0; i < 512; i++) V->dist[q * 512 + i] = 0.0;
    if (V->irr_kappa)
      for (int i = 0; i < 192; i++) V->irr_kappa[q * 192 + i] = 0.0;
    if (V->dist_kappa)
      for (int i = 0; i < 512; i++) V->dist_kappa[q * 512 + i] = 0.0;
    if (V->offsets)
      for (int a = 0; a < 3; a++) ((float*)V->offsets)[q * 3 + a] = 0.0f;
    V->states[q] = classify_probe(s, V, q, rotations, K, blo, bhi, NULL, NULL, NULL);
  }
  free(blo);
  free(bhi);
}

/* ------------------------------------------------------- probe relocation */
/* Section "Probe Position Adjustment": iterations of the offset optimizer,
   each tracing the probe's rays against static geometry under one rotation.
   A probe that sees more than 25 % backfaces moves along the vector to its
   closest backface, scaled as far as the per-axis offset limit allows (less
   1e-3 of the scale); it moves only if that scale exceeds 1, i.e. only if it
   gets through the backface.  Otherwise, unless the farthest and closest
   front faces lie within 60 degrees of each other (one surface seen), it
   moves min(0.2, distance) toward the farthest front face.  Readings of the
   listing: the direction used in the 60-degree test is the farthest front
   face's ray direction; a probe for which neither branch applies keeps its
   offset; a front-face move that would leave the offset limit is not taken;
   an axis along which the backface vector has no component does not limit
   the scale.  Offsets are kept in float32 between iterations.  ambiguous[q]
   (may be NULL) gets bit i set when iteration i's decision for probe q
   depends on something a float32 tracer may see otherwise (a flagged ray
   near an extreme, a tie, a count or a dot product at its threshold). */
static double axis_scale(double cur, double lim, double v) {
  if (v == 0.0) return INFINITY;
  return fmax((lim - cur) / v, (-lim - cur) / v);
}

void orc_optimize_offsets(const orc_scene* s, orc_volume* V, const float* rotations, int32_t iterations,
                          double offset_limit, int32_t* ambiguous) {
  int64_t P = vol_probes(V);
  float* offsets = (float*)V->offsets;
  const int32_t N = V->rays;
  double lim[3];
  for (int a = 0; a < 3; a++) lim[a] = offset_limit * (double)V->spacing[a];
  if (ambiguous)
    for (int64_t q = 0; q < P; q++) ambiguous[q] = 0;
  for (int32_t it = 0; it < iterations; it++) {
    const float* R = rotations + 9 * it;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < P; q++) {
      double Pq[3];
      probe_position(V, q, Pq);
      int32_t back = 0, n_flag = 0, flag_miss = 0;
      double tcb = INFINITY, tcf = INFINITY, tff = -1.0;
      int32_t rcb = -1, rcf = -1, rff = -1;
      double* ts = (double*)malloc(sizeof(double) * (size_t)N);
      int8_t* kind = (int8_t*)malloc((size_t)N); /* 0 miss, 1 front, 2 back */
      int32_t* fl = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
      for (int32_t r = 0; r < N; r++) {
        double w[3];
        orc_sf_direction(r, N, R, w);
        orc_hit h;
        orc_trace(s, Pq, w, 1, &h);
        fl[r] = h.flags;
        if (h.flags) {
          n_flag++;
          if (h.tri < 0) flag_miss = 1;
        }
        kind[r] = 0;
        ts[r] = h.t;
        if (h.tri < 0) continue;
        double e1[3], e2[3], ng[3];
        sub3(tri_v(s, h.tri, 1), tri_v(s, h.tri, 0), e1);
        sub3(tri_v(s, h.tri, 2), tri_v(s, h.tri, 0), e2);
        cross3(e1, e2, ng);
        if (dot3(w, ng) > 0.0) {
          kind[r] = 2;
          back++;
          if (h.t < tcb) { tcb = h.t; rcb = r; }
        } else {
          kind[r] = 1;
          if (h.t < tcf) { tcf = h.t; rcf = r; }
          if (h.t > tff) { tff = h.t; rff = r; }
        }
      }
      double cur[3] = {offsets[3 * q], offsets[3 * q + 1], offsets[3 * q + 2]};
      double nw[3] = {cur[0], cur[1], cur[2]};
      int amb = flag_miss;
      /* the count decides the branch: ambiguous if flagged rays could move it across */
      if (abs(4 * back - N) <= 4 * n_flag) amb = 1;
      if (4 * back > N) {
        /* near-ties or flagged rays at the closest backface */
        for (int32_t r = 0; r < N; r++)
          if (kind[r] == 2 && r != rcb && ts[r] <= tcb * (1.0 + 1e-6)) amb = 1;
          else if (fl[r] && ts[r] <= tcb * (1.0 + 1e-4)) amb = 1;
        double w[3];
        orc_sf_direction(rcb, N, R, w);
        double v[3] = {w[0] * tcb, w[1] * tcb, w[2] * tcb};
        double sc = INFINITY;
        for (int a = 0; a < 3; a++) sc = fmin(sc, axis_scale(cur[a], lim[a], v[a]));
        sc -= 1e-3;
        if (fabs(sc - 1.0) < 1e-5 * fmax(1.0, fabs(sc))) amb = 1;
        if (sc > 1.0)
          for (int a = 0; a < 3; a++) nw[a] = cur[a] + v[a] * sc;
      } else if (rff >= 0) {
        for (int32_t r = 0; r < N; r++) {
          if (kind[r] == 1 && r != rcf && ts[r] <= tcf * (1.0 + 1e-6)) amb = 1;
          if (kind[r] == 1 && r != rff && ts[r] >= tff * (1.0 - 1e-6)) amb = 1;
          if (fl[r] && (ts[r] <= tcf * (1.0 + 1e-4) || ts[r] >= tff * (1.0 - 1e-4))) amb = 1;
        }
        double wf[3], wc[3];
        orc_sf_direction(rff, N, R, wf);
        orc_sf_direction(rcf, N, R, wc);
        double c = dot3(wf, wc);
        if (fabs(c - 0.5) < 1e-5) amb = 1;
        if (!(c > 0.5)) {
          double step = fmin(0.2, tff), cand[3];
          int inside = 1;
          for (int a = 0; a < 3; a++) {
            cand[a] = cur[a] + step * wf[a];
            if (fabs(cand[a]) > lim[a]) inside = 0;
            if (fabs(fabs(cand[a]) - lim[a]) < 1e-6 * lim[a]) amb = 1;
          }
          if (inside)
            for (int a = 0; a < 3; a++) nw[a] = cand[a];
        }
      }
      for (int a = 0; a < 3; a++) offsets[3 * q + a] = (float)nw[a];
      if (ambiguous && amb) ambiguous[q] |= 1 << it;
      free(ts);
      free(kind);
      free(fl);
    }
  }
}

/* Per-frame state step: sleeping probes near a dynamic object wake (Newly
   Awake); awake probes no longer near any dynamic object go back to sleep. */
void orc_state_step(const orc_scene* s, orc_volume* vols, int32_t nvol) {
  for (int32_t v = 0; v < nvol; v++) {
    orc_volume* V = &vols[v];
    double* lo = (double*)malloc(sizeof(double) * 3 * (size_t)(s->nobj + 1));
    double* hi = (double*)malloc(sizeof(double) * 3 * (size_t)(s->nobj + 1));
    expanded_object_boxes(s, V, lo, hi);
    for (int64_t q = 0; q < vol_probes(V); q++) {
      double P[3];
      probe_position(V, q, P);
      int in = inside_any(s, lo, hi, P);
      if (V->states[q] == ORC_SLEEPING && in) V->states[q] = ORC_NEWLY_AWAKE;
      else if (V->states[q] == ORC_AWAKE && !in) V->states[q] = ORC_SLEEPING;
    }
    free(lo);
    free(hi);
  }
}

static int active_state(uint8_t s) {
  return s == ORC_NEWLY_AWAKE || s == ORC_NEWLY_VIGILANT || s == ORC_AWAKE || s == ORC_VIGILANT;
}

/* One frame (Section "Probe Update" and the last two steps of the full
   initialization): state step; every active probe traces its rotated
   spherical-Fibonacci rays and shades them against the previous atlases of
   all volumes; only then are all probes blended (hysteresis 0 for Newly
   states) and Newly states promoted. */
int64_t orc_update_frame(const orc_scene* s, const orc_lights* L, orc_volume* vols, int32_t nvol,
                         const float R[9], orc_ray_record* records, int64_t capacity) {
  return orc_update_frame_forced(s, L, vols, nvol, R, records, capacity, 0, NULL, NULL, NULL);
}

int64_t orc_update_frame_forced(const orc_scene* s, const orc_lights* L, orc_volume* vols, int32_t nvol,
                                const float R[9], orc_ray_record* records, int64_t capacity, int64_t n_force,
                                const uint8_t* force, const int32_t* force_tri, const uint32_t* force_vis) {
  orc_state_step(s, vols, nvol);
  /* previous atlases and states, read by hit shading */
  orc_volume* prev = (orc_volume*)malloc(sizeof(orc_volume) * (size_t)(nvol ? nvol : 1));
  int64_t total_rays = 0;
  for (int32_t v = 0; v < nvol; v++) {
    prev[v] = vols[v];
    int64_t P = vol_probes(&vols[v]);
    prev[v].irr = (double*)malloc(sizeof(double) * (size_t)P * 192);
    prev[v].dist = (double*)malloc(sizeof(double) * (size_t)P * 512);
    prev[v].states = (uint8_t*)malloc((size_t)P);
    memcpy(prev[v].irr, vols[v].irr, sizeof(double) * (size_t)P * 192);
    memcpy(prev[v].dist, vols[v].dist, sizeof(double) * (size_t)P * 512);
    memcpy(prev[v].states, vols[v].states, (size_t)P);
    for (int64_t q = 0; q < P; q++)
      if (active_state(vols[v].states[q])) total_rays += vols[v].rays;
  }
  orc_ray_record* rec = (orc_ray_record*)malloc(sizeof(orc_ray_record) * (size_t)(total_rays ? total_rays : 1));
  int64_t off = 0;
  for (int32_t v = 0; v < nvol; v++) {
    orc_volume* V = &vols[v];
    int64_t P = vol_probes(V);
    int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)P);
    int64_t na = 0;
    for (int64_t q = 0; q < P; q++) slot[q] = active_state(V->states[q]) ? na++ : -1;
    double dmax = V->dmax;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < P; q++) {
      if (slot[q] < 0) continue;
      double Pq[3];
      probe_position(V, q, Pq);
      for (int32_t r = 0; r < V->rays; r++) {
        double w[3];
        orc_sf_direction(r, V->rays, R, w);
        int64_t i = off + slot[q] * V->rays + r;
        uint8_t fm = (force && i < n_force) ? force[i] : 0;
        shade_ray_impl(s, L, prev, nvol, Pq, w, dmax, fm, fm ? force_tri[i] : -1, fm ? force_vis[i] : 0, &rec[i]);
      }
    }
    off += na * V->rays;
    free(slot);
  }
  /* blend */
  off = 0;
  for (int32_t v = 0; v < nvol; v++) {
    orc_volume* V = &vols[v];
    int64_t P = vol_probes(V);
    int32_t N = V->rays;
    double* omega = (double*)malloc(sizeof(double) * 3 * (size_t)N);
    for (int32_t r = 0; r < N; r++) orc_sf_direction(r, N, R, omega + 3 * r);
    int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)P);
    int64_t na = 0;
    for (int64_t q = 0; q < P; q++) slot[q] = active_state(V->states[q]) ? na++ : -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < P; q++) {
      if (slot[q] < 0) continue;
      double* rgb = (double*)malloc(sizeof(double) * 3 * (size_t)N);
      double* rk = (double*)malloc(sizeof(double) * 3 * (size_t)N);
      double* d = (double*)malloc(sizeof(double) * (size_t)N);
      double* dk = (double*)malloc(sizeof(double) * (size_t)N);
      for (int32_t r = 0; r < N; r++) {
        const orc_ray_record* rr = &rec[off + slot[q] * N + r];
        for (int c = 0; c < 3; c++) {
          rgb[3 * r + c] = rr->rgb[c];
          rk[3 * r + c] = rr->kappa[c];
        }
        d[r] = rr->d;
        dk[r] = rr->d_kappa;
      }
      int fresh = V->states[q] == ORC_NEWLY_AWAKE || V->states[q] == ORC_NEWLY_VIGILANT;
      orc_blend_probe_k(N, omega, rgb, rk, d, dk, (double)V->cos_power, fresh ? 0.0 : (double)V->alpha_irr,
                        fresh ? 0.0 : (double)V->alpha_dist, (double)V->gamma, V->texel_thresholds,
                        V->irr + q * 192, V->dist + q * 512,
                        V->irr_kappa ? V->irr_kappa + q * 192 : NULL, V->dist_kappa ? V->dist_kappa + q * 512 : NULL);
      free(rgb);
      free(rk);
      free(d);
      free(dk);
    }
    for (int64_t q = 0; q < P; q++) {
      if (V->states[q] == ORC_NEWLY_AWAKE) V->states[q] = ORC_AWAKE;
      else if (V->states[q] == ORC_NEWLY_VIGILANT) V->states[q] = ORC_VIGILANT;
    }
    off += na * N;
    free(omega);
    free(slot);
  }
  if (records) memcpy(records, rec, sizeof(orc_ray_record) * (size_t)(total_rays < capacity ? total_rays : capacity));
  free(rec);
  for (int32_t v = 0; v < nvol; v++) {
    free(prev[v].irr);
    free(prev[v].dist);
    free(prev[v].states);
  }
  free(prev);
  return total_rays;
}

/* ================================================================ adjoint */
/* Reverse pass of the query and of one update frame with the ray hits and
   shadow decisions of the forward frame held fixed (the quantities are then
   smooth functions of emission and texels, except at the Chebyshev branch
   point r = mu where the weight is C1). */

static void footprint(int32_t m, const double v[3], int32_t* x0, int32_t* y0, double* fx, double* fy) {
  int32_t k = m - 2;
  double p[2];
  orc_oct_encode(v, p);
  double cx = 1.0 + (0.5 * p[0] + 0.5) * k - 0.5;
  double cy = 1.0 + (0.5 * p[1] + 0.5) * k - 0.5;
  *x0 = (int32_t)floor(cx);
  *y0 = (int32_t)floor(cy);
  if (*x0 < 0) *x0 = 0;
  if (*x0 > k) *x0 = k;
  if (*y0 < 0) *y0 = 0;
  if (*y0 > k) *y0 = k;
  *fx = clampd(cx - *x0, 0.0, 1.0);
  *fy = clampd(cy - *y0, 0.0, 1.0);
}

/* adds g (nch channels) to the four bilinear taps of direction v */
static void scatter_tile(double* gtile, int32_t m, int32_t nch, const double v[3], const double* g) {
  int32_t x0, y0;
  double fx, fy;
  footprint(m, v, &x0, &y0, &fx, &fy);
  const double bw[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
  const int32_t idx[4] = {y0 * m + x0, y0 * m + x0 + 1, (y0 + 1) * m + x0, (y0 + 1) * m + x0 + 1};
  for (int t = 0; t < 4; t++)
    for (int c = 0; c < nch; c++) gtile[idx[t] * nch + c] += bw[t] * g[c];
}

/* The terms of a query's gradient, one per (texel, tap), before they are
   added into the gradient atlases.  Keeping them apart lets the reverse pass
   also report, per texel, the sum of the magnitudes of its terms and how far
   float32 evaluation of the same terms may move them (a finite difference
   over the float32 error of each input of the Chebyshev factor, of the
   irradiance values and of the hit point).  Those two are test
   infrastructure for judging a float32 implementation; the gradient does not
   depend on them. */
typedef struct {
  int32_t vol, dist;   /* volume; 0: irradiance texel (3 channels), 1: distance texel (2) */
  int64_t elem;        /* offset of the texel's first channel in its atlas */
  double g[3], a[3];   /* gradient terms; magnitude bounds of the same terms */
} term;

typedef struct {
  int32_t n, cap;
  term* t;
} term_list;

static term* term_push(term_list* L) {
  if (L->n == L->cap) {
    L->cap = L->cap ? 2 * L->cap : 256;
    L->t = (term*)realloc(L->t, sizeof(term) * (size_t)L->cap);
  }
  term* t = &L->t[L->n++];
  memset(t, 0, sizeof(*t));
  return t;
}

/* the four bilinear taps of direction v in a tile with nch channels */
static void push_taps(term_list* L, int32_t vol, int32_t dist, int64_t tile_elem, int32_t m, int32_t nch,
                      const double v[3], const double* g, const double* a) {
  int32_t x0, y0;
  double fx, fy;
  footprint(m, v, &x0, &y0, &fx, &fy);
  const double bw[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
  const int32_t idx[4] = {y0 * m + x0, y0 * m + x0 + 1, (y0 + 1) * m + x0, (y0 + 1) * m + x0 + 1};
  for (int k = 0; k < 4; k++) {
    term* t = term_push(L);
    t->vol = vol;
    t->dist = dist;
    t->elem = tile_elem + (int64_t)idx[k] * nch;
    for (int c = 0; c < nch; c++) {
      t->g[c] = bw[k] * g[c];
      t->a[c] = bw[k] * a[c];
    }
  }
}

/* Perturbations of the float32 inputs, in multiples of their error bound:
   [0] mu, [1] mu2 (with the rounding of mu2 - mu^2), [2] r, [3] the sampled
   irradiance (alternating in sign over the cage, which moves e_i - E). */
typedef struct {
  double mu, mu2, r, e;
} perturb;

/* Reverse pass of one volume's cage query (forward: volume_query): the
   normalised weighted average of Eq. with the backface factor, the
   Chebyshev factor of the visibility section and the self-shadow bias of
   Eq. 1; g is dLoss/dE for this volume's share, ga its magnitude bound. */
static void volume_query_terms(const orc_volume* V, int32_t vol, const double X[3], const double n[3],
                               const double wo[3], const double g[3], const double ga[3], const perturb* pt,
                               term_list* L) {
  double u[3], f[3], Xb[3];
  int64_t gi[3];
  double D = fmin((double)V->spacing[0], fmin((double)V->spacing[1], (double)V->spacing[2]));
  for (int a = 0; a < 3; a++) {
    u[a] = (X[a] - (double)V->origin[a]) / (double)V->spacing[a];
    gi[a] = (int64_t)clampd(floor(u[a]), 0.0, (double)(V->counts[a] - 2));
    f[a] = clampd(u[a] - (double)gi[a], 0.0, 1.0);
    Xb[a] = X[a] + (0.2 * n[a] + 0.8 * wo[a]) * (0.75 * D) * (double)V->bias;
  }
  double w[8], e[8][3], wtb[8], zd[8][3], mmv[8][2], rr[8];
  int64_t qs[8];
  int cheb[8];
  int used = 0;
  double W = 0.0;
  for (int c = 0; c < 8; c++) {
    int cb[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    int64_t q = storage_index(V, gi[0] + cb[0], gi[1] + cb[1], gi[2] + cb[2]);
    if (!sampled_state(V->states[q])) continue;
    double wt = 1.0;
    for (int a = 0; a < 3; a++) wt *= cb[a] ? f[a] : 1.0 - f[a];
    double P[3], toP[3];
    probe_position(V, q, P);
    sub3(P, X, toP);
    normalize3(toP);
    double h = (1.0 + dot3(n, toP)) * 0.5;
    double wb = h * h + 0.2;
    double z[3];
    sub3(Xb, P, z);
    double r = len3(z);
    double wv = 1.0;
    cheb[used] = 0;
    if (r > 0.0) {
      for (int a = 0; a < 3; a++) zd[used][a] = z[a] / r;
      orc_sample_tile(V->dist + q * 512, 16, 2, zd[used], mmv[used]);
      if (pt) {
        /* float32 error bounds of the sampled moments and of r, as in the
           forward query's sensitivity */
        double lo[2], hi[2], kk[2] = {0.0, 0.0};
        footprint_range(V->dist + q * 512, 16, 2, zd[used], lo, hi);
        if (V->dist_kappa) orc_sample_tile(V->dist_kappa + q * 512, 16, 2, zd[used], kk);
        double m0 = mmv[used][0], m1 = mmv[used][1];
        double dmu = (4.0 * fabs(m0) + 32.0 * (hi[0] - lo[0]) + kk[0]) * U32;
        double dmu2 = (4.0 * fabs(m1) + 32.0 * (hi[1] - lo[1]) + kk[1] + 4.0 * (fabs(m1) + m0 * m0)) * U32;
        mmv[used][0] = m0 + pt->mu * dmu;
        mmv[used][1] = m1 + pt->mu2 * dmu2;
        r += pt->r * 4.0 * r * U32;
      }
      if (r > mmv[used][0]) {
        double var = fmax(mmv[used][1] - mmv[used][0] * mmv[used][0], 0.0);
        double dl = r - mmv[used][0];
        wv = pow(var / (var + dl * dl), (double)V->cheb_power);
        cheb[used] = 1;
      }
    }
    rr[used] = r;
    qs[used] = q;
    wtb[used] = wt * wb;
    w[used] = wt * wb * wv;
    orc_sample_tile(V->irr + q * 192, 8, 3, n, e[used]);
    if (pt && pt->e != 0.0) {
      double ek[3] = {0.0, 0.0, 0.0};
      if (V->irr_kappa) orc_sample_tile(V->irr_kappa + q * 192, 8, 3, n, ek);
      double sg = (used & 1) ? -pt->e : pt->e;
      for (int c = 0; c < 3; c++) e[used][c] += sg * (16.0 * fabs(e[used][c]) + ek[c]) * U32;
    }
    W += w[used];
    used++;
  }
  if (!(W > 0.0)) return;
  double E[3] = {0, 0, 0};
  for (int i = 0; i < used; i++)
    for (int c = 0; c < 3; c++) E[c] += w[i] * e[i][c] / W;
  for (int i = 0; i < used; i++) {
    /* dE/de_i = w_i / W, through the bilinear taps of the irradiance tile */
    double ge[3], gea[3];
    for (int c = 0; c < 3; c++) {
      ge[c] = g[c] * w[i] / W;
      gea[c] = ga[c] * w[i] / W;
    }
    push_taps(L, vol, 0, qs[i] * 192, 8, 3, n, ge, gea);
    if (!cheb[i]) continue;
    /* dE/dw_i = (e_i - E) / W; w_i = wt wb ch^k with ch = var / (var + dl^2),
       var = max(mu2 - mu^2, 0), dl = r - mu */
    double gw = 0.0, gwa = 0.0;
    for (int c = 0; c < 3; c++) {
      gw += g[c] * (e[i][c] - E[c]) / W;
      gwa += ga[c] * (fabs(e[i][c]) + fabs(E[c])) / W;
    }
    double mu = mmv[i][0], mu2 = mmv[i][1];
    double raw = mu2 - mu * mu;
    double var = fmax(raw, 0.0);
    double dl = rr[i] - mu;
    double den = var + dl * dl;
    double ch = var / den;
    double dch_dvar = dl * dl / (den * den);
    double dch_ddl = -2.0 * dl * var / (den * den);
    double dvar_dmu = raw > 0.0 ? -2.0 * mu : 0.0, dvar_dmu2 = raw > 0.0 ? 1.0 : 0.0;
    double k = (double)V->cheb_power;
    double dwv_dch = k * pow(ch, k - 1.0);
    double cmu = wtb[i] * dwv_dch * (dch_dvar * dvar_dmu - dch_ddl);
    double cmu2 = wtb[i] * dwv_dch * dch_dvar * dvar_dmu2;
    double gd[2] = {gw * cmu, gw * cmu2}, gda[2] = {gwa * fabs(cmu), gwa * fabs(cmu2)};
    push_taps(L, vol, 1, qs[i] * 512, 16, 2, zd[i], gd, gda);
  }
}

/* Section "Multiple Probe Volumes": the same share of dE as the forward
   blend of volumes gives each volume */
static void query_terms(const orc_volume* vols, int32_t nvol, const double X[3], const double n[3],
                        const double wo[3], const double gout[3], const double gabs[3], const perturb* pt,
                        term_list* L) {
  double Wt = 0.0;
  for (int32_t v = 0; v < nvol; v++) {
    const orc_volume* V = &vols[v];
    if (Wt >= 1.0) break;
    real Xr[3];
    load3r(X, Xr);
    double wv = volume_weight(V, Xr);
    double wuse = (v == nvol - 1) ? 1.0 - Wt : fmin(wv, 1.0 - Wt);
    if (wuse > 0.0) {
      double g[3] = {wuse * gout[0], wuse * gout[1], wuse * gout[2]};
      double ga[3] = {wuse * gabs[0], wuse * gabs[1], wuse * gabs[2]};
      volume_query_terms(V, v, X, n, wo, g, ga, pt, L);
      Wt += wuse;
    }
  }
}

static double* texel_ptr(double** arrays, const term* t) { return arrays[t->vol] + t->elem; }

static void add_terms(const term_list* L, double** gi, double** gd, double** ai, double** ad) {
  for (int32_t j = 0; j < L->n; j++) {
    const term* t = &L->t[j];
    int nch = t->dist ? 2 : 3;
    double* g = texel_ptr(t->dist ? gd : gi, t);
    for (int c = 0; c < nch; c++) g[c] += t->g[c];
    if (ai && ad) {
      double* a = texel_ptr(t->dist ? ad : ai, t);
      for (int c = 0; c < nch; c++) a[c] += t->a[c];
    }
  }
}

static int term_cmp(const void* pa, const void* pb) {
  const term* a = (const term*)pa;
  const term* b = (const term*)pb;
  if (a->vol != b->vol) return a->vol < b->vol ? -1 : 1;
  if (a->dist != b->dist) return a->dist < b->dist ? -1 : 1;
  if (a->elem != b->elem) return a->elem < b->elem ? -1 : 1;
  return 0;
}

/* per texel: sums the terms of L (sorted, duplicates merged in place) */
static void merge_terms(term_list* L) {
  if (L->n == 0) return;
  qsort(L->t, (size_t)L->n, sizeof(term), term_cmp);
  int32_t o = 0;
  for (int32_t j = 1; j < L->n; j++) {
    if (term_cmp(&L->t[o], &L->t[j]) == 0) {
      for (int c = 0; c < 3; c++) {
        L->t[o].g[c] += L->t[j].g[c];
        L->t[o].a[c] += L->t[j].a[c];
      }
    } else {
      L->t[++o] = L->t[j];
    }
  }
  L->n = o + 1;
}

/* adds |per-texel terms of A - per-texel terms of B| (both merged) */
static void add_abs_diff(const term_list* A, const term_list* B, double** si, double** sd) {
  int32_t i = 0, j = 0;
  while (i < A->n || j < B->n) {
    int cmp = i == A->n ? 1 : j == B->n ? -1 : term_cmp(&A->t[i], &B->t[j]);
    const term* t = cmp <= 0 ? &A->t[i] : &B->t[j];
    double* s = texel_ptr(t->dist ? sd : si, t);
    for (int c = 0; c < (t->dist ? 2 : 3); c++) {
      double va = cmp <= 0 ? A->t[i].g[c] : 0.0, vb = cmp >= 0 ? B->t[j].g[c] : 0.0;
      s[c] += fabs(va - vb);
    }
    if (cmp <= 0) i++;
    if (cmp >= 0) j++;
  }
}

/* gradient, magnitudes and float32 sensitivities of one query at X; a hit
   point X2 (or NULL) is X moved by its own float32 error */
static void query_backward_full(const orc_volume* vols, int32_t nvol, const double X[3], const double X2[3],
                                const double n[3], const double wo[3], const double g[3], const double ga[3],
                                const orc_grads* G) {
  term_list L0 = {0, 0, NULL};
  query_terms(vols, nvol, X, n, wo, g, ga, NULL, &L0);
  add_terms(&L0, G->g_irr, G->g_dist, G->a_irr, G->a_dist);
  if (G->s_irr && G->s_dist) {
    merge_terms(&L0);
    static const perturb P[8] = {{1, 0, 0, 0}, {-1, 0, 0, 0}, {0, 1, 0, 0}, {0, -1, 0, 0},
                                 {0, 0, 1, 0}, {0, 0, -1, 0}, {0, 0, 0, 1}, {0, 0, 0, -1}};
    term_list Lp = {0, 0, NULL};
    for (int k = 0; k < 8; k++) {
      Lp.n = 0;
      query_terms(vols, nvol, X, n, wo, g, ga, &P[k], &Lp);
      merge_terms(&Lp);
      add_abs_diff(&L0, &Lp, G->s_irr, G->s_dist);
    }
    if (X2) {
      Lp.n = 0;
      query_terms(vols, nvol, X2, n, wo, g, ga, NULL, &Lp);
      merge_terms(&Lp);
      add_abs_diff(&L0, &Lp, G->s_irr, G->s_dist);
    }
    free(Lp.t);
  }
  free(L0.t);
}

void orc_query_backward(const orc_volume* vols, int32_t nvol, const double X[3], const double n[3],
                        const double wo[3], const double gout[3], const orc_grads* G) {
  double ga[3] = {fabs(gout[0]), fabs(gout[1]), fabs(gout[2])};
  query_backward_full(vols, nvol, X, NULL, n, wo, gout, ga, G);
}

void orc_update_backward(const orc_scene* s, const orc_volume* prev, int32_t nvol, const float R[9],
                         const orc_ray_record* records, const orc_grads* Gnew, const orc_grads* Gprev,
                         double* g_emission) {
  int64_t off = 0;
  const int mag = Gprev->a_irr && Gprev->a_dist;
  for (int32_t v = 0; v < nvol; v++) {
    const orc_volume* V = &prev[v];
    int64_t P = vol_probes(V);
    int32_t N = V->rays;
    double* omega = (double*)malloc(sizeof(double) * 3 * (size_t)N);
    double* gL = (double*)malloc(sizeof(double) * 3 * (size_t)N);
    double* gLa = (double*)malloc(sizeof(double) * 3 * (size_t)N);
    for (int32_t r = 0; r < N; r++) orc_sf_direction(r, N, R, omega + 3 * r);
    for (int64_t q = 0; q < P; q++) {
      const double* gi = Gnew->g_irr[v] + q * 192;
      const double* gd = Gnew->g_dist[v] + q * 512;
      /* magnitude bounds of the upstream gradient: given, else |g| */
      double ain[192], adn[512];
      for (int i = 0; i < 192; i++) ain[i] = Gnew->a_irr ? Gnew->a_irr[v][q * 192 + i] : fabs(gi[i]);
      for (int i = 0; i < 512; i++) adn[i] = Gnew->a_dist ? Gnew->a_dist[v][q * 512 + i] : fabs(gd[i]);
      double* pi = Gprev->g_irr[v] + q * 192;
      double* pd = Gprev->g_dist[v] + q * 512;
      double* pia = mag ? Gprev->a_irr[v] + q * 192 : NULL;
      double* pda = mag ? Gprev->a_dist[v] + q * 512 : NULL;
      if (!active_state(V->states[q])) {
        /* not updated this frame: output texels are the input texels */
        for (int i = 0; i < 192; i++) pi[i] += gi[i];
        for (int i = 0; i < 512; i++) pd[i] += gd[i];
        if (mag) {
          for (int i = 0; i < 192; i++) pia[i] += ain[i];
          for (int i = 0; i < 512; i++) pda[i] += adn[i];
        }
        continue;
      }
      int fresh = V->states[q] == ORC_NEWLY_AWAKE || V->states[q] == ORC_NEWLY_VIGILANT;
      double ai = fresh ? 0.0 : (double)V->alpha_irr, ad = fresh ? 0.0 : (double)V->alpha_dist;
      /* border texels repeat interior texels: fold their gradients */
      double fi[192], fd[512], fia[192], fda[512];
      memset(fi, 0, sizeof(fi));
      memset(fd, 0, sizeof(fd));
      memset(fia, 0, sizeof(fia));
      memset(fda, 0, sizeof(fda));
      for (int32_t y = 0; y < 8; y++)
        for (int32_t x = 0; x < 8; x++) {
          int32_t sx, sy;
          orc_border_source(8, x, y, &sx, &sy);
          for (int c = 0; c < 3; c++) {
            fi[(sy * 8 + sx) * 3 + c] += gi[(y * 8 + x) * 3 + c];
            fia[(sy * 8 + sx) * 3 + c] += ain[(y * 8 + x) * 3 + c];
          }
        }
      for (int32_t y = 0; y < 16; y++)
        for (int32_t x = 0; x < 16; x++) {
          int32_t sx, sy;
          orc_border_source(16, x, y, &sx, &sy);
          for (int c = 0; c < 2; c++) {
            fd[(sy * 16 + sx) * 2 + c] += gd[(y * 16 + x) * 2 + c];
            fda[(sy * 16 + sx) * 2 + c] += adn[(y * 16 + x) * 2 + c];
          }
        }
      for (int32_t r = 0; r < 3 * N; r++) gL[r] = gLa[r] = 0.0;
      for (int32_t y = 1; y <= 6; y++)
        for (int32_t x = 1; x <= 6; x++) {
          double nt[3], W = 0.0;
          orc_texel_direction(8, x, y, nt);
          for (int32_t r = 0; r < N; r++) W += fmax(0.0, dot3(nt, omega + 3 * r));
          const int e0 = (y * 8 + x) * 3;
          double keep = W > 0.0 ? ai : 1.0;
          for (int c = 0; c < 3; c++) {
            pi[e0 + c] += keep * fi[e0 + c];
            if (mag) pia[e0 + c] += keep * fia[e0 + c];
          }
          if (!(W > 0.0)) continue;
          for (int32_t r = 0; r < N; r++) {
            double wr = fmax(0.0, dot3(nt, omega + 3 * r)) / W;
            for (int c = 0; c < 3; c++) {
              gL[3 * r + c] += (1.0 - ai) * wr * fi[e0 + c];
              gLa[3 * r + c] += (1.0 - ai) * wr * fia[e0 + c];
            }
          }
        }
      for (int32_t y = 1; y <= 14; y++)
        for (int32_t x = 1; x <= 14; x++) {
          double nt[3], W = 0.0;
          orc_texel_direction(16, x, y, nt);
          for (int32_t r = 0; r < N; r++) W += pow(fmax(0.0, dot3(nt, omega + 3 * r)), (double)V->cos_power);
          const int e0 = (y * 16 + x) * 2;
          double keep = W > 0.0 ? ad : 1.0;
          for (int c = 0; c < 2; c++) {
            pd[e0 + c] += keep * fd[e0 + c];
            if (mag) pda[e0 + c] += keep * fda[e0 + c];
          }
        }
      /* ray radiance -> emission and previous-frame irradiance at the hit */
      double Pq[3];
      probe_position(V, q, Pq);
      for (int32_t r = 0; r < N; r++, off++) {
        const orc_ray_record* rec = &records[off];
        if (rec->tri < 0) continue;
        double e1[3], e2[3], ng[3];
        sub3(tri_v(s, rec->tri, 1), tri_v(s, rec->tri, 0), e1);
        sub3(tri_v(s, rec->tri, 2), tri_v(s, rec->tri, 0), e2);
        cross3(e1, e2, ng);
        normalize3(ng);
        const double* w = omega + 3 * r;
        if (dot3(w, ng) > 0.0) continue;
        int32_t m = s->material[rec->tri];
        for (int c = 0; c < 3; c++) g_emission[m * 3 + c] += gL[3 * r + c];
        double X[3], X2[3], wo[3] = {-w[0], -w[1], -w[2]};
        /* the hit point moved by its float32 error along the ray, as for
           the forward shading's sensitivity */
        double ep = fmin(1e-2, U32 * (8.0 / fmax(rec->cosi, 1e-6) + 16.0));
        for (int a = 0; a < 3; a++) {
          X[a] = Pq[a] + rec->t * w[a];
          X2[a] = Pq[a] + rec->t * (1.0 + ep) * w[a];
        }
        double gq[3], gqa[3];
        for (int c = 0; c < 3; c++) {
          gq[c] = s->albedo[m * 3 + c] * gL[3 * r + c];
          gqa[c] = s->albedo[m * 3 + c] * gLa[3 * r + c];
        }
        query_backward_full(prev, nvol, X, X2, ng, wo, gq, gqa, Gprev);
      }
    }
    free(omega);
    free(gL);
    free(gLa);
  }
}
