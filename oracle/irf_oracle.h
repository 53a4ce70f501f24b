/*
 * FP64 CPU oracle of the probe update and probe query of the irradiance
 * field with visibility (Majercik et al., "Scaling Probe-Based Real-Time
 * Dynamic Global Illumination for Production").
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, plain reference that the
 * GPU library is checked against.  It shares no code, header, table or
 * helper with the GPU library, and nothing in the product may link or call
 * it; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.
 *
 * All arithmetic is IEEE double.  Inputs arrive as the same float32 arrays
 * that the GPU library receives and are promoted on entry.  (A second build
 * of the same source with -DORC_REAL=float evaluates the value path in
 * float32; it exists only to check the float32 sensitivity estimates kappa
 * that the records and texels carry.)
 */
#ifndef IRF_ORACLE_H
#define IRF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* probe states (Section "Probe States") */
enum { ORC_OFF = 0, ORC_SLEEPING = 1, ORC_NEWLY_AWAKE = 2, ORC_NEWLY_VIGILANT = 3,
       ORC_AWAKE = 4, ORC_VIGILANT = 5 };

/* ray flags: where a float32 tracer may legitimately decide differently */
enum {
  ORC_F_GRAZE = 1,     /* closest hit lies within eps_b of a triangle edge      */
  ORC_F_TIE = 2,       /* another hit within eps_t * t of the closest           */
  ORC_F_NEARMISS = 4,  /* a triangle missed by less than eps_b before t(1+eps_t) */
  ORC_F_EDGEON = 8,    /* ray nearly parallel to the hit plane (face side unsure) */
  ORC_F_SHADOW = 16,   /* at least one shadow ray of this hit is ambiguous       */
  ORC_F_FORCED = 32,   /* hit or shadow decisions given by the caller            */
  ORC_F_FORCE_INVALID = 64 /* the given triangle is not hit by the ray's line    */
};

typedef struct orc_scene orc_scene;

orc_scene* orc_scene_create(const float* vertices, int64_t n_vertices,
                            const uint32_t* indices, int64_t n_tris,
                            const uint32_t* tri_material, const uint32_t* tri_object,
                            const float* albedo, const float* emission, int32_t n_materials);
void orc_scene_free(orc_scene* s);
void orc_scene_set_emission(orc_scene* s, const double* emission); /* [M][3] */
void orc_scene_set_specular(orc_scene* s, const double* specular); /* [M][3], mirror reflectance */
int64_t orc_scene_bvh_nodes(const orc_scene* s);

typedef struct {
  int32_t n_dir;
  const float* dir_to_light;    /* [n_dir][3] */
  const float* dir_irradiance;  /* [n_dir][3] */
  int32_t n_point;
  const float* point_pos;       /* [n_point][3] */
  const float* point_intensity; /* [n_point][3] */
  float sky[3];
} orc_lights;

typedef struct {
  float origin[3];
  float spacing[3];
  int32_t counts[3];
  int32_t rays;
  float alpha_irr, alpha_dist;
  float cos_power;
  float bias;         /* B of the self-shadow bias */
  float dmax;         /* distance clamp */
  int32_t cheb_power;
  double* irr;        /* [P][8][8][3]   */
  double* dist;       /* [P][16][16][2] */
  uint8_t* states;    /* [P] */
  const float* offsets; /* [P][3] or NULL */
  double* irr_kappa;  /* [P][8][8][3] or NULL: float32 sensitivity of each texel (units of u) */
  double* dist_kappa; /* [P][16][16][2] or NULL */
  float gamma;        /* perception encoding exponent of irradiance texels; 1 = linear */
  int32_t texel_thresholds; /* per-texel hysteresis thresholds on irradiance: 0 / 1 */
  int32_t phase[3];   /* tracking window: storage slot of logical probe i is (i + phase) mod n */
  int32_t tracking;   /* 1: the volume tracks the camera (window + camera-centred blend weight) */
  float camera[3];    /* camera position for the blend weight of a tracking volume */
} orc_volume;

typedef struct {
  int32_t tri;       /* original triangle id, -1 on miss */
  int32_t flags;
  double t;          /* hit distance (INFINITY on miss) */
  double bmin;       /* smallest barycentric of the hit */
} orc_hit;

#define ORC_CAGE 16
typedef struct {
  int32_t tri;
  int32_t flags;
  double t;
  double rgb[3];
  double d;
  uint32_t vis;          /* bit l: shadow ray to light l unoccluded */
  int32_t n_cage;        /* probes that carried weight in the hit's query */
  int32_t cage[ORC_CAGE];/* global probe ids (volume base + q); -1 pads */
  double kappa[3];       /* absolute float32 sensitivity of rgb (units of u) */
  double cosi;           /* |cos| of the angle between ray and hit plane (0 on a miss) */
  double d_kappa;        /* absolute float32 sensitivity of d (units of u) */
} orc_ray_record;

/* ---- octahedral map (Cigolle et al. 2014), square [-1,1]^2 ---- */
void orc_oct_encode(const double v[3], double p[2]);
void orc_oct_decode(const double p[2], double v[3]);
/* direction of interior cell (x, y), 1 <= x, y <= m-2, of an m x m tile */
void orc_texel_direction(int32_t m, int32_t x, int32_t y, double v[3]);
/* source cell of border cell (x, y) of an m x m tile */
void orc_border_source(int32_t m, int32_t x, int32_t y, int32_t* sx, int32_t* sy);
/* bilinear sample of an m x m tile with nch channels in direction v */
void orc_sample_tile(const double* tile, int32_t m, int32_t nch, const double v[3], double* out);

/* ---- rays ---- */
void orc_sf_direction(int32_t i, int32_t n, const float R[9], double out[3]);

/* ---- nearest hit ---- */
void orc_trace(const orc_scene* s, const double o[3], const double d[3], int32_t static_only,
               orc_hit* hit);
void orc_trace_brute(const orc_scene* s, const double o[3], const double d[3], int32_t static_only,
                     orc_hit* hit);
void orc_trace_batch(const orc_scene* s, int64_t n, const double* o, const double* d,
                     int32_t static_only, int32_t brute, orc_hit* hits);

/* ---- blend of one probe (Eq. U, cos and cos^p weights, hysteresis) ---- */
void orc_blend_probe(int32_t n, const double* omega, const double* rgb, const double* d,
                     double cos_power, double alpha_irr, double alpha_dist,
                     double* irr_tile, double* dist_tile);
/* the same blend, also carrying the float32 sensitivity of every texel
   (units of u): the rays' own (rgb_kappa [n][3] and d_kappa [n], may be NULL), the weights'
   (a float32 cosine is off by about 8 u absolute) and rounding; kappa tiles
   blend with the same hysteresis as the texels */
void orc_blend_probe_k(int32_t n, const double* omega, const double* rgb, const double* rgb_kappa, const double* d,
                       const double* d_kappa, double cos_power, double alpha_irr, double alpha_dist, double gamma,
                       int32_t thresholds, double* irr_tile, double* dist_tile, double* irr_kappa, double* dist_kappa);
/* the blend with the convergence refinements of the sections on perception
   encoding and fast convergence: irradiance texels store the new mean raised
   to 1/gamma (gamma = 1: linear), and with thresholds != 0 the irradiance
   hysteresis of a texel drops by 0.15 when its largest per-channel change (in
   stored units) exceeds 0.25 and to 0 when it exceeds 0.8 */
void orc_blend_probe_ex(int32_t n, const double* omega, const double* rgb, const double* d, double cos_power,
                        double alpha_irr, double alpha_dist, double gamma, int32_t thresholds, double* irr_tile,
                        double* dist_tile);

/* ---- query E(X, n, w_o) over cascaded volumes ---- */
void orc_query(const orc_volume* vols, int32_t nvol, const double X[3], const double n[3],
               const double wo[3], double out[3], double kappa[3],
               int32_t* cage, int32_t* n_cage);
void orc_query_batch(const orc_volume* vols, int32_t nvol, int64_t nq, const float* pos,
                     const float* nrm, const float* view, double* out, double* kappa);

/* ---- probe states ---- */
void orc_classify(const orc_scene* s, orc_volume* vols, int32_t nvol, const float* rotations,
                  int32_t K, int32_t* n_back, int32_t* n_flagged, double* t_front);
void orc_state_step(const orc_scene* s, orc_volume* vols, int32_t nvol);

/* ---- one update frame for all volumes; records (optional) receive, per
   volume in order, per active probe in index order, per ray, one record ---- */
int64_t orc_update_frame(const orc_scene* s, const orc_lights* L, orc_volume* vols, int32_t nvol,
                         const float R[9], orc_ray_record* records, int64_t capacity);
/* the same frame with some rays' decisions given (the parity protocol: on a
   ray this oracle flags, another tracer's hit and shadow decisions are
   adopted and everything downstream is recomputed).  For record index
   i < n_force: bit 0 of force[i] takes force_tri[i] (-1: a miss) as the
   ray's nearest hit, at the exact distance of that triangle's plane; bit 1
   takes force_vis[i] as its shadow-ray bits.  Flags keep this oracle's own
   flags plus ORC_F_FORCED. */
int64_t orc_update_frame_forced(const orc_scene* s, const orc_lights* L, orc_volume* vols, int32_t nvol,
                                const float R[9], orc_ray_record* records, int64_t capacity, int64_t n_force,
                                const uint8_t* force, const int32_t* force_tri, const uint32_t* force_vis);

/* ---- tracking window (Section "Tracking Windows") ----
   Moves V's window toward the camera: along each axis, while the camera is
   more than one spacing from the window centre, the window shifts one cell
   toward it; the plane left behind is reused (circular buffer) for the new
   plane in front, whose probes are reset (zero texels and offsets) and
   classified with the K rotations as in orc_classify.  Stores the camera for
   the blend weight.  shift (int32[3], may be NULL) receives the cells moved. */
void orc_track_volume(const orc_scene* s, orc_volume* V, const float camera[3], const float* rotations, int32_t K,
                      int32_t* shift);

/* ---- probe relocation (Section "Probe Position Adjustment") ----
   iterations rotations [iterations][9]; offsets of V (float32 [P][3]) are
   updated in place; offset_limit is a fraction of the spacing per axis;
   ambiguous [P] (or NULL): bit i set when iteration i's decision for the
   probe depends on something float32 may decide otherwise. */
void orc_optimize_offsets(const orc_scene* s, orc_volume* V, const float* rotations, int32_t iterations,
                          double offset_limit, int32_t* ambiguous);

/* ---- adjoint, ray hits and shadow decisions held fixed ----
   Per volume v: g_irr[v] / g_dist[v] are [P][8][8][3] / [P][16][16][2]
   float64 arrays; everything accumulates (+=).  Optional (NULL to skip):
   a_*: per texel, the sum of the magnitudes of the terms that make up its
   gradient (with the upstream gradient replaced by its magnitude bound);
   s_*: per texel, how far the terms move when the float32 inputs of the
   query (sampled moments, r, irradiance, hit point) move by their float32
   error bounds.  a_ and s_ are test infrastructure for judging a float32
   implementation; they do not change the gradient. */
typedef struct {
  double** g_irr;
  double** g_dist;
  double** a_irr;
  double** a_dist;
  double** s_irr;
  double** s_dist;
} orc_grads;

void orc_query_backward(const orc_volume* vols, int32_t nvol, const double X[3], const double n[3],
                        const double wo[3], const double gout[3], const orc_grads* G);
/* Backward of one update frame.  prev: the frame's input atlases and the
   states after the frame's state step (before promotion); records: the
   frame's ray records (per volume in order, per active probe, per ray);
   Gnew: dLoss/d(output atlases) in g_*, with magnitude bounds in a_* (NULL:
   |g|); accumulates dLoss/d(input atlases) into Gprev (a_*, s_* optional)
   and dLoss/d(emission) into g_emission [M][3]. */
void orc_update_backward(const orc_scene* s, const orc_volume* prev, int32_t nvol, const float R[9],
                         const orc_ray_record* records, const orc_grads* Gnew, const orc_grads* Gprev,
                         double* g_emission);

/* ---- query with the texels sampled in direction `look` (filtered radiance) ---- */
void orc_query_look(const orc_volume* vols, int32_t nvol, const double X[3], const double n[3],
                    const double wo[3], const double look[3], double out[3], double kappa[3], int32_t* cage,
                    int32_t* n_cage);

/* ---- second-order glossy (Section "Second Order Glossy"): the mirror ray of
   surface point X (normal n, toward-viewer v) and its shaded hit, whose own
   mirror bounce is the probes' filtered radiance; record fields as for a
   probe ray (d unused) ---- */
void orc_glossy(const orc_scene* s, const orc_lights* L, const orc_volume* vols, int32_t nvol, const double X[3],
                const double n[3], const double v[3], orc_ray_record* rec);
void orc_glossy_batch(const orc_scene* s, const orc_lights* L, const orc_volume* vols, int32_t nvol, int64_t n,
                      const float* pos, const float* nrm, const float* view, orc_ray_record* recs);

/* ---- shading of a single ray from o along w (exposed for pins) ---- */
void orc_shade_ray(const orc_scene* s, const orc_lights* L, const orc_volume* vols, int32_t nvol,
                   const double o[3], const double w[3], double dmax, orc_ray_record* rec);

#ifdef __cplusplus
}
#endif
#endif
