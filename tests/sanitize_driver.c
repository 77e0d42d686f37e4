/*
 * Host sanitizer run of the CPU oracle (test infrastructure): built together
 * with oracle/oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer
 * by tests/test_oracle_sanitizers.py, it drives every entry point the tests
 * use on a small procedural scene and exits 0 when the run completes.  Any
 * sanitizer report aborts the program with a non-zero status.
 *
 * Scene: a closed unit box (static world, two materials), one moving
 * axis-aligned cube of side 0.12 (object 1), one rectangle light under the
 * ceiling facing down; frame 1 moves the cube and the light.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

/* oracle entry points the tests reach through ctypes (declared in oracle.c) */
void or_verify(const or_scene* s, or_store* st, uint32_t* amb, int32_t* examined);
void or_retrace(const or_scene* s, or_store* st, float T, uint64_t seed, uint64_t frame, uint32_t* amb,
                int32_t* traces);
void or_dm_update(const or_scene* s, or_store* st, uint64_t seed, uint64_t frame, uint32_t* dm_c,
                  uint32_t* dm_pruned, uint32_t* amb);
int64_t or_dm_cells(const float* half, int32_t kind, const int32_t* dm);
void or_energy_forward(const or_scene* s, int64_t N, int32_t B, const uint32_t* hit, const uint32_t* info,
                       const double* albedo, const double* power, double* E);
void or_energy_backward(const or_scene* s, int64_t N, int32_t B, const uint32_t* hit, const uint32_t* info,
                        const double* albedo, const double* power, const double* gE, int32_t n_mat,
                        double* g_albedo, double* g_power);
void or_transform(int64_t n_verts, const float* local, const float* m, float* out);
uint32_t or_info_make(uint32_t cell, uint32_t nseg, uint32_t start, uint32_t replace, uint32_t reuse);

/* the 12 triangles of the box [lo, hi] (two per face), 9 floats each */
static void box_tris(const float lo[3], const float hi[3], float* out) {
  const float c[8][3] = {{lo[0], lo[1], lo[2]}, {hi[0], lo[1], lo[2]}, {hi[0], hi[1], lo[2]},
                         {lo[0], hi[1], lo[2]}, {lo[0], lo[1], hi[2]}, {hi[0], lo[1], hi[2]},
                         {hi[0], hi[1], hi[2]}, {lo[0], hi[1], hi[2]}};
  const int f[12][3] = {{0, 1, 2}, {0, 2, 3}, {4, 6, 5}, {4, 7, 6}, {0, 4, 5}, {0, 5, 1},
                        {3, 2, 6}, {3, 6, 7}, {0, 3, 7}, {0, 7, 4}, {1, 5, 6}, {1, 6, 2}};
  for (int t = 0; t < 12; ++t)
    for (int v = 0; v < 3; ++v) memcpy(out + 9 * t + 3 * v, c[f[t][v]], 3 * sizeof(float));
}

enum { NS = 12, ND = 12, NT = NS + ND, N_PATHS = 600, B = 5, N_MAT = 2 };

int main(void) {
  float stat[NS * 9], loc[ND * 9], verts[2][NT * 9];
  const float blo[3] = {0, 0, 0}, bhi[3] = {1, 1, 1};
  const float clo[3] = {-0.06f, -0.06f, -0.06f}, chi[3] = {0.06f, 0.06f, 0.06f};
  box_tris(blo, bhi, stat);
  box_tris(clo, chi, loc);
  /* cube transforms of frames 0 and 1: a small rotation about y, then a shift */
  float oxf[2][12];
  for (int fr = 0; fr < 2; ++fr) {
    const double a = 0.3 + 0.05 * fr, ca = cos(a), sa = sin(a);
    const float m[12] = {(float)ca, 0, (float)sa, 0.5f + 0.04f * fr, 0, 1, 0, 0.45f,
                         (float)-sa, 0, (float)ca, 0.5f};
    memcpy(oxf[fr], m, sizeof(m));
    memcpy(verts[fr], stat, sizeof(stat));
    or_transform(3 * ND, loc, oxf[fr], verts[fr] + 9 * NS);
  }
  uint32_t tri_obj[NT], tri_mat[NT];
  for (int t = 0; t < NT; ++t) {
    tri_obj[t] = t < NS ? 0u : 1u;
    tri_mat[t] = (uint32_t)(t % N_MAT);
  }
  const float albedo_f[N_MAT * 3] = {0.7f, 0.6f, 0.5f, 0.4f, 0.5f, 0.6f};
  /* light: u along x, v along z, normal -y, centre under the ceiling */
  float lxf[2][12] = {{1, 0, 0, 0.5f, 0, 0, -1, 0.97f, 0, 1, 0, 0.5f},
                      {1, 0, 0, 0.52f, 0, 0, -1, 0.97f, 0, 1, 0, 0.49f}};
  const float lhalf[2] = {0.08f, 0.08f}, lpow[3] = {1.0f, 0.9f, 0.8f};
  const int64_t lbase[2] = {0, N_PATHS};
  uint8_t omoved[2][2] = {{0, 0}, {0, 1}}, lmoved[2] = {0, 1};

  or_scene sc[2];
  for (int fr = 0; fr < 2; ++fr) {
    memset(&sc[fr], 0, sizeof(or_scene));
    sc[fr].n_tris = NT;
    sc[fr].verts = verts[fr];
    sc[fr].tri_obj = tri_obj;
    sc[fr].tri_mat = tri_mat;
    sc[fr].n_obj = 2;
    sc[fr].obj_moved = omoved[fr];
    sc[fr].albedo = albedo_f;
    sc[fr].n_lights = 1;
    sc[fr].light_xf = lxf[fr];
    sc[fr].light_half = lhalf;
    sc[fr].light_power = lpow;
    sc[fr].light_moved = &lmoved[fr];
    sc[fr].light_base = lbase;
    sc[fr].eps_end = 1e-4;
    sc[fr].eps_close = 1e-3;
    sc[fr].band_verify = 1e-6;
    sc[fr].band_trace = 1e-5;
    sc[fr].radius = 0.01f;
    sc[fr].band_box = 1e-6;
  }
  const size_t rows = (size_t)B * N_PATHS;
  float* pos = calloc(rows * 3, sizeof(float));
  uint32_t* hit = calloc(rows, sizeof(uint32_t));
  float* energy = calloc(rows * 3, sizeof(float));
  float* radius = calloc(rows, sizeof(float));
  float* origin = calloc((size_t)N_PATHS * 3, sizeof(float));
  uint32_t* info = calloc(N_PATHS, sizeof(uint32_t));
  uint32_t* amb = calloc(N_PATHS, sizeof(uint32_t));
  int32_t* cnt = calloc(N_PATHS, sizeof(int32_t));
  if (!pos || !hit || !energy || !radius || !origin || !info || !amb || !cnt) return 2;
  or_store st = {N_PATHS, B, pos, hit, energy, radius, origin, info};
  const uint64_t seed = 11;

  /* frame 0: every path a new light sample, traced to B photons */
  for (int p = 0; p < N_PATHS; ++p) info[p] = or_info_make(0, 0, 0, 1, 0);
  or_retrace(&sc[0], &st, -1.0f, seed, 0, amb, cnt);
  int64_t photons = 0;
  for (int p = 0; p < N_PATHS; ++p) photons += (info[p] >> 22) & 15u;
  if (photons == 0) {
    fprintf(stderr, "frame 0 traced no photon\n");
    return 3;
  }
  /* frame 1: triangle test, then the error-based re-trace */
  or_verify(&sc[1], &st, amb, cnt);
  or_retrace(&sc[1], &st, 0.01f, seed, 1, amb, cnt);
  /* the paper's box test and the cosine-ratio energy test on the same store */
  sc[1].verify_boxes = 1;
  sc[1].energy_test = 1;
  or_verify(&sc[1], &st, amb, cnt);
  or_retrace(&sc[1], &st, 0.01f, seed, 2, amb, cnt);
  sc[1].verify_boxes = 0;
  sc[1].energy_test = 0;
  /* distribution maps: cells, prune, fill, then the re-trace of the re-sampled paths */
  const int32_t dm[4] = {2, 2, 2, 4};
  sc[1].dm = dm;
  const int64_t cells = or_dm_cells(lhalf, 0, dm);
  uint32_t* dm_c = calloc((size_t)cells, sizeof(uint32_t));
  uint32_t* dm_p = calloc((size_t)cells, sizeof(uint32_t));
  if (!dm_c || !dm_p) return 2;
  or_dm_update(&sc[1], &st, seed, 3, dm_c, dm_p, amb);
  or_retrace(&sc[1], &st, 0.01f, seed, 3, amb, cnt);
  sc[1].dm = NULL;
  /* spot light and camera emitters (zero extent) */
  const float zero_half[2] = {0, 0};
  for (int kind = 1; kind <= 2; ++kind) {
    const int32_t k = kind;
    const float param[2] = {kind == 1 ? 0.8f : 0.5f, kind == 1 ? 0.0f : 0.4f};
    sc[1].light_half = zero_half;
    sc[1].light_kind = &k;
    sc[1].light_param = param;
    or_verify(&sc[1], &st, amb, cnt);
    or_retrace(&sc[1], &st, 0.01f, seed, 4 + kind, amb, cnt);
  }
  sc[1].light_half = lhalf;
  sc[1].light_kind = NULL;
  sc[1].light_param = NULL;
  /* differentiation form */
  double alb[N_MAT * 3], pw[3], ga[N_MAT * 3], gp[3];
  for (int i = 0; i < N_MAT * 3; ++i) alb[i] = albedo_f[i];
  for (int i = 0; i < 3; ++i) pw[i] = lpow[i];
  double* E = calloc(rows * 3, sizeof(double));
  double* gE = calloc(rows * 3, sizeof(double));
  if (!E || !gE) return 2;
  for (size_t i = 0; i < rows * 3; ++i) gE[i] = 1.0 + (double)(i % 7);
  or_energy_forward(&sc[1], N_PATHS, B, hit, info, alb, pw, E);
  or_energy_backward(&sc[1], N_PATHS, B, hit, info, alb, pw, gE, N_MAT, ga, gp);
  double sum = 0;
  for (int i = 0; i < N_MAT * 3; ++i) sum += ga[i];
  if (!isfinite(sum)) return 4;
  free(E);
  free(gE);
  free(dm_c);
  free(dm_p);
  free(pos);
  free(hit);
  free(energy);
  free(radius);
  free(origin);
  free(info);
  free(amb);
  free(cnt);
  printf("sanitized oracle run done: %lld photons at frame 0\n", (long long)photons);
  return 0;
}
