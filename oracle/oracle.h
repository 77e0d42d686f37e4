/*
 * CPU oracle for photon-path verification (Moreau, Doggett, Sintorn,
 * "Path Verification for Dynamic Indirect Illumination").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * Plain, slow, brute force, FP64.  Segment and ray queries test every
 * triangle of the relevant objects; consecutive triangles are grouped in
 * chunks of at most 32 whose padded FP64 bounding boxes are used as a
 * pre-reject, which cannot change any result.
 *
 * Path store seen by the oracle (plain layout; the test harness converts):
 *   pos    float [B][N][3]   photon x_{r+1} in row r
 *   hit    uint  [B][N]      global triangle id of the photon, ~0 when empty
 *   energy float [B][N][3]   arriving flux (RGB) of the photon
 *   radius float [B][N]
 *   origin float [N][3]      world-space light sample x_0
 *   info   uint  [N]         bits 0..21 cell, 22..25 segment count,
 *                            26..29 retrace start, 30 replace, 31 reuse light
 */
#ifndef PV_ORACLE_H
#define PV_ORACLE_H
#include <stdint.h>

typedef struct {
  int64_t n_tris;
  const float* verts;        /* [n_tris][9] world vertices at the current frame */
  const uint32_t* tri_obj;   /* [n_tris] object id, 0 = static world */
  const uint32_t* tri_mat;   /* [n_tris] material id */
  int32_t n_obj;
  const uint8_t* obj_moved;  /* [n_obj] transform changed since last frame */
  const float* albedo;       /* [n_mat][3] */
  int32_t n_lights;
  const float* light_xf;     /* [L][12] current rigid transform of each light */
  const float* light_half;   /* [L][2] half extents in light-local u, v */
  const float* light_power;  /* [L][3] */
  const uint8_t* light_moved;/* [L] */
  const int64_t* light_base; /* [L+1] path ranges per light */
  double eps_end;            /* endpoint tolerance, scene units */
  double eps_close;          /* AreClose tolerance, scene units */
  double band_verify;        /* ambiguity band for verification decisions */
  double band_trace;         /* ambiguity band for traced rays */
  float radius;              /* radius written on new photons */
  int32_t verify_boxes;      /* 1: a segment is invalid once it reaches a moved object's box */
  double band_box;           /* ambiguity band of that box decision */
  const int32_t* dm;         /* NULL, or the distribution-map grid {gu, gv, rings, sectors}: new
                                light samples are drawn inside the cell of their path */
  const int32_t* light_kind; /* NULL (all 0), or [L] emission of each light: 0 rectangle / point
                                light (cosine-weighted hemisphere), 1 spot light, 2 camera */
  const float* light_param;  /* [L][2]: spot: cos of the cone half-angle; camera: tangents of the
                                half field of view along u and v */
  int32_t energy_test;       /* Equation 2's E_N: 0 albedo of the new vertex (arrival side); 1 also
                                times the ratio of the kept direction's cosines at the new and the
                                old vertex (BRDF-weighted) */
} or_scene;

/* light kinds (emission set of a light of zero extent) */
#define OR_LIGHT_AREA 0
#define OR_LIGHT_SPOT 1
#define OR_LIGHT_CAMERA 2

typedef struct {
  int64_t n_paths;
  int32_t B;
  float* pos;
  uint32_t* hit;
  float* energy;
  float* radius;
  float* origin;
  uint32_t* info;
} or_store;

/* ambiguity flags (per path) */
#define OR_AMB_EDGE 1u
#define OR_AMB_END 2u
#define OR_AMB_LIGHT 4u
#define OR_AMB_TIE 8u
#define OR_AMB_HEMI 16u
#define OR_AMB_CLOSE 32u
#define OR_AMB_BOX 64u
#define OR_AMB_CELL 128u
#define OR_AMB_EQ2 256u

#endif
