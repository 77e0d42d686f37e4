/*
 * CPU oracle for photon-path verification.  TEST INFRASTRUCTURE ONLY: see
 * oracle.h.  Every function states the passage of the paper it follows
 * (Moreau, Doggett, Sintorn, "Path Verification for Dynamic Indirect
 * Illumination") or the published method it restates.
 *
 * Readings taken where the paper is silent (each is also listed in the design
 * notes of the repository):
 *  - photons store their position in place of the incoming direction; the
 *    incoming direction is the difference of consecutive positions;
 *  - a segment is blocked by a triangle (two-sided) crossed strictly inside
 *    the open interval (eps_end, L - eps_end) of its length L;
 *  - only objects whose transform changed are tested; a segment whose end
 *    photon lies on a moved object is invalid;
 *  - a light with both half extents 0 is a point light emitting cosine-
 *    weighted about its normal; Section 3.1's point-light update moves the
 *    origin to the light's new position, re-aims segment 0 at the first
 *    photon (lost when that leaves the emitting side) and replaces the
 *    shadow-map test by a visibility segment against every triangle;
 *  - the box mode (Section 3.2's own, conservative test) uses the exact box
 *    of each moved object's current world triangles and the same interval
 *    (eps_end, L - eps_end) of the segment; the error-based walk after it
 *    tests the first invalid segment against the moved triangles before
 *    tracing it, unless its origin moved (Section 3.3's box-without-triangle
 *    case);
 *  - world vertices are fp32(fma(m0,x,fma(m1,y,fma(m2,z,t)))) evaluated in FP64;
 *  - random numbers come from Philox4x64-10 keyed (seed, 0) with counter
 *    (path, frame, vertex, tag); uniforms are the top 24 bits times 2^-24;
 *  - cosine-weighted directions: Shirley-Chiu concentric map lifted to the
 *    hemisphere (Malley), tangent frame from Duff et al. 2017;
 *  - no Russian roulette: paths run to B photons or to a ray that escapes.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define HIT_NONE 0xffffffffu
#define CHUNK 32
#define T_FAR 16.0

/* ------------------------------------------------------------------------ */
/* path information word (Section 4: cell 22 bits, segment count 4 bits,     */
/* retrace start 4 bits, replace 1 bit, reuse light 1 bit)                   */

static uint32_t info_cell(uint32_t w) { return w & 0x3fffffu; }
static uint32_t info_nseg(uint32_t w) { return (w >> 22) & 15u; }
static uint32_t info_start(uint32_t w) { return (w >> 26) & 15u; }
static uint32_t info_replace(uint32_t w) { return (w >> 30) & 1u; }
static uint32_t info_reuse(uint32_t w) { return (w >> 31) & 1u; }
static uint32_t info_make(uint32_t cell, uint32_t nseg, uint32_t start, uint32_t replace,
                          uint32_t reuse) {
  return (cell & 0x3fffffu) | ((nseg & 15u) << 22) | ((start & 15u) << 26) |
         ((replace & 1u) << 30) | ((reuse & 1u) << 31);
}

uint32_t or_info_make(uint32_t cell, uint32_t nseg, uint32_t start, uint32_t replace,
                      uint32_t reuse) {
  return info_make(cell, nseg, start, replace, reuse);
}

/* ------------------------------------------------------------------------ */
/* small FP64 vector helpers                                                 */

static void sub3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
static void load3f(const float* p, double o[3]) { o[0] = p[0]; o[1] = p[1]; o[2] = p[2]; }
static void store3f(float* p, const double o[3]) {
  p[0] = (float)o[0]; p[1] = (float)o[1]; p[2] = (float)o[2];
}
static double clamp01(double x) { return x < 0 ? 0 : (x > 1 ? 1 : x); }

/* ------------------------------------------------------------------------ */
/* Transform of dynamic-object vertices (Section 3.2 needs the current       */
/* frame's geometry; rounding fixed by the reading above).                   */

void or_transform(int64_t n_verts, const float* local, const float* m, float* out) {
  for (int64_t i = 0; i < n_verts; ++i) {
    double x = local[3 * i], y = local[3 * i + 1], z = local[3 * i + 2];
    for (int r = 0; r < 3; ++r) {
      double v = fma((double)m[4 * r + 0], x,
                     fma((double)m[4 * r + 1], y, fma((double)m[4 * r + 2], z, (double)m[4 * r + 3])));
      out[3 * i + r] = (float)v;
    }
  }
}

/* moved <=> any of the 12 floats differs bitwise */
int or_xf_moved(const float* a, const float* b) {
  return memcmp(a, b, 12 * sizeof(float)) != 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), restated from its      */
/* published definition: ten rounds of two 64x64->128 multiplies, the key     */
/* bumped by the Weyl constants between rounds.                              */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void or_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, &hi0, &lo0);
    mulhilo64(M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0; k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in [0,1): top 24 bits, exactly representable in FP32 */
static double u24(uint64_t x) { return (double)(x >> 40) * (1.0 / 16777216.0); }

static void draw4(uint64_t seed, uint64_t path, uint64_t frame, uint64_t vertex, uint64_t tag,
                  double u[4]) {
  uint64_t ctr[4] = {path, frame, vertex, tag}, key[2] = {seed, 0}, r[4];
  or_philox4x64(ctr, key, r);
  for (int i = 0; i < 4; ++i) u[i] = u24(r[i]);
}

/* Shirley & Chiu 1997 concentric square-to-disk map, lifted to the cosine-  */
/* weighted hemisphere (Malley's method): returns local (x, y, z), z >= 0.   */
void or_cosine_local(double u1, double u2, double out[3]) {
  double a = 2.0 * u1 - 1.0, b = 2.0 * u2 - 1.0, r, phi;
  const double PI = 3.14159265358979323846;
  if (a == 0.0 && b == 0.0) {
    r = 0.0; phi = 0.0;
  } else if (fabs(a) > fabs(b)) {
    r = a; phi = (PI / 4.0) * (b / a);
  } else {
    r = b; phi = PI / 2.0 - (PI / 4.0) * (a / b);
  }
  double x = r * cos(phi), y = r * sin(phi);
  /* height on the unit sphere above the disk point at radius |r| */
  double ar = fabs(r);
  double z2 = (1.0 - ar) * (1.0 + ar);
  out[0] = x; out[1] = y; out[2] = z2 > 0.0 ? sqrt(z2) : 0.0;
}

/* Duff, Burgess, Christensen, Hery, Kensler, Liani, Villemin, "Building an  */
/* Orthonormal Basis, Revisited", JCGT 2017: tangents t, b of unit normal n. */
void or_onb(const double n[3], double t[3], double b[3]) {
  double sign = n[2] >= 0.0 ? 1.0 : -1.0;
  double a = -1.0 / (sign + n[2]);
  double c = n[0] * n[1] * a;
  t[0] = 1.0 + sign * n[0] * n[0] * a; t[1] = sign * c; t[2] = -sign * n[0];
  b[0] = c; b[1] = sign + n[1] * n[1] * a; b[2] = -n[1];
}

/* cosine-weighted direction about unit normal n */
void or_cosine_dir(double u1, double u2, const double n[3], double out[3]) {
  double l[3], t[3], b[3];
  or_cosine_local(u1, u2, l);
  or_onb(n, t, b);
  for (int i = 0; i < 3; ++i) out[i] = l[0] * t[i] + l[1] * b[i] + l[2] * n[i];
}

/* ------------------------------------------------------------------------ */
/* Geometry predicates                                                        */

/* Moller & Trumbore 1997, two-sided, FP64: line o + t d against triangle.   */
/* Returns 1 with (t,u,v) when det != 0 (plane crossing); inside-ness is      */
/* left to the caller (u >= 0, v >= 0, u + v <= 1).                          */
static int mt_plane(const double o[3], const double d[3], const double v0[3], const double v1[3],
                    const double v2[3], double* t, double* u, double* v) {
  double e1[3], e2[3], p[3], s[3], q[3];
  sub3(v1, v0, e1);
  sub3(v2, v0, e2);
  cross3(d, e2, p);
  double det = dot3(e1, p);
  if (det == 0.0) return 0;
  double inv = 1.0 / det;
  sub3(o, v0, s);
  *u = dot3(s, p) * inv;
  cross3(s, e1, q);
  *v = dot3(d, q) * inv;
  *t = dot3(e2, q) * inv;
  return 1;
}

static int inside_uv(double u, double v) { return u >= 0.0 && v >= 0.0 && u + v <= 1.0; }

/* Exported for tests: 1 if the segment a->b is blocked by the triangle in   */
/* the sense of Section 3.2 with an endpoint tolerance eps.                  */
int or_segment_blocked_tri(const double a[3], const double b[3], const double* tri, double eps) {
  double d[3], t, u, v;
  sub3(b, a, d);
  double L = norm3(d);
  if (!mt_plane(a, d, tri, tri + 3, tri + 6, &t, &u, &v)) return 0;
  double s = t * L;
  return inside_uv(u, v) && s > eps && s < L - eps;
}

/* Closest distance between segments p0p1 and q0q1 (Ericson, Real-Time       */
/* Collision Detection, 2005, section 5.1.9), FP64.                          */
double or_segseg_dist(const double p0[3], const double p1[3], const double q0[3], const double q1[3]) {
  double d1[3], d2[3], r[3];
  sub3(p1, p0, d1);
  sub3(q1, q0, d2);
  sub3(p0, q0, r);
  double a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r);
  double s, t;
  if (a <= 1e-300 && e <= 1e-300) {
    s = t = 0.0;
  } else if (a <= 1e-300) {
    s = 0.0; t = clamp01(f / e);
  } else {
    double c = dot3(d1, r);
    if (e <= 1e-300) {
      t = 0.0; s = clamp01(-c / a);
    } else {
      double b = dot3(d1, d2), den = a * e - b * b;
      s = den != 0.0 ? clamp01((b * f - c * e) / den) : 0.0;
      t = (b * s + f) / e;
      if (t < 0.0) {
        t = 0.0; s = clamp01(-c / a);
      } else if (t > 1.0) {
        t = 1.0; s = clamp01((b - c) / a);
      }
    }
  }
  double c1[3], c2[3], w[3];
  for (int i = 0; i < 3; ++i) { c1[i] = p0[i] + d1[i] * s; c2[i] = q0[i] + d2[i] * t; }
  sub3(c1, c2, w);
  return norm3(w);
}

static double tri_edge_dist(const double s0[3], const double s1[3], const double v[9]) {
  double m = or_segseg_dist(s0, s1, v, v + 3);
  double m2 = or_segseg_dist(s0, s1, v + 3, v + 6);
  double m3 = or_segseg_dist(s0, s1, v + 6, v);
  if (m2 < m) m = m2;
  if (m3 < m) m = m3;
  return m;
}

/* ------------------------------------------------------------------------ */
/* exactness-preserving pre-reject: chunks of consecutive same-object tris   */

typedef struct {
  double lo[3], hi[3];
  int64_t first;
  int32_t count;
  uint32_t obj;
} chunk_t;

typedef struct {
  const or_scene* s;
  chunk_t* ch;
  int64_t n_ch;
  double* obox;  /* [n_obj][6] box (lo, hi) of each object's world triangles */
} accel_t;

static void accel_build(accel_t* a, const or_scene* s) {
  a->s = s;
  a->obox = (double*)malloc(sizeof(double) * 6 * (size_t)(s->n_obj > 0 ? s->n_obj : 1));
  for (int32_t o = 0; o < s->n_obj; ++o)
    for (int k = 0; k < 3; ++k) {
      a->obox[6 * o + k] = INFINITY;
      a->obox[6 * o + 3 + k] = -INFINITY;
    }
  for (int64_t t = 0; t < s->n_tris; ++t) {
    const uint32_t o = s->tri_obj[t];
    if (o == 0 || (int32_t)o >= s->n_obj) continue;
    for (int v = 0; v < 3; ++v)
      for (int k = 0; k < 3; ++k) {
        const double x = s->verts[9 * t + 3 * v + k];
        if (x < a->obox[6 * o + k]) a->obox[6 * o + k] = x;
        if (x > a->obox[6 * o + 3 + k]) a->obox[6 * o + 3 + k] = x;
      }
  }
  a->ch = (chunk_t*)malloc(sizeof(chunk_t) * (size_t)(s->n_tris / 1 + 1));
  a->n_ch = 0;
  int64_t t = 0;
  while (t < s->n_tris) {
    chunk_t* c = &a->ch[a->n_ch++];
    c->first = t;
    c->obj = s->tri_obj[t];
    c->count = 0;
    for (int k = 0; k < 3; ++k) { c->lo[k] = INFINITY; c->hi[k] = -INFINITY; }
    while (t < s->n_tris && c->count < CHUNK && s->tri_obj[t] == c->obj) {
      for (int v = 0; v < 3; ++v)
        for (int k = 0; k < 3; ++k) {
          double x = s->verts[9 * t + 3 * v + k];
          if (x < c->lo[k]) c->lo[k] = x;
          if (x > c->hi[k]) c->hi[k] = x;
        }
      ++c->count;
      ++t;
    }
  }
}

static void accel_free(accel_t* a) {
  free(a->ch);
  free(a->obox);
}

/* does o + t d, t in [t0, t1], come within pad of the box? (slab test)      */
static int seg_box(const double o[3], const double d[3], double t0, double t1, const double lo[3],
                   const double hi[3], double pad) {
  for (int k = 0; k < 3; ++k) {
    double l = lo[k] - pad, h = hi[k] + pad;
    if (l > h) return 0; /* a box shrunk to nothing */
    if (d[k] == 0.0) {
      if (o[k] < l || o[k] > h) return 0;
    } else {
      double ta = (l - o[k]) / d[k], tb = (h - o[k]) / d[k];
      if (ta > tb) { double x = ta; ta = tb; tb = x; }
      if (ta > t0) t0 = ta;
      if (tb < t1) t1 = tb;
      if (t0 > t1) return 0;
    }
  }
  return 1;
}

static void tri_verts(const or_scene* s, int64_t t, double v[9]) {
  for (int i = 0; i < 9; ++i) v[i] = s->verts[9 * t + i];
}

/* ------------------------------------------------------------------------ */
/* Section 3.2: is segment a->b blocked by a triangle of a moved object (of   */
/* any object and the static world when 'all': a point light's visibility)?  */
/* Result: 0 clear, 1 blocked.  *amb |= flags when some triangle lies within  */
/* the band of the decision (edge or endpoint) and no triangle blocks it      */
/* with margin.                                                               */

static int seg_blocked(const accel_t* A, const double a[3], const double b[3], double band, int all,
                       uint32_t* amb) {
  const or_scene* s = A->s;
  double d[3];
  sub3(b, a, d);
  double L = norm3(d);
  if (L <= 0.0) return 0;
  double e = s->eps_end;
  double tlo = (e - band) / L, thi = (L - e + band) / L;
  if (tlo < 0) tlo = 0;
  if (thi > 1) thi = 1;
  if (tlo > thi) return 0;
  double s0[3], s1[3];
  for (int i = 0; i < 3; ++i) { s0[i] = a[i] + tlo * d[i]; s1[i] = a[i] + thi * d[i]; }
  int blocked = 0, certain = 0;
  uint32_t local_amb = 0;
  for (int64_t c = 0; c < A->n_ch && !certain; ++c) {
    const chunk_t* ch = &A->ch[c];
    if (!all && (ch->obj == 0 || !s->obj_moved[ch->obj])) continue;
    if (!seg_box(a, d, tlo, thi, ch->lo, ch->hi, band + 1e-9)) continue;
    for (int64_t t = ch->first; t < ch->first + ch->count; ++t) {
      double v[9], tt, u, w;
      tri_verts(s, t, v);
      double ed = tri_edge_dist(s0, s1, v);
      int near_edge = ed <= band;
      int hit = 0, near_end = 0;
      if (mt_plane(a, d, v, v + 3, v + 6, &tt, &u, &w)) {
        double dist = tt * L;
        int in = inside_uv(u, w);
        hit = in && dist > e && dist < L - e;
        near_end = in && (fabs(dist - e) <= band || fabs(dist - (L - e)) <= band);
      }
      if (hit) blocked = 1;
      if (hit && !near_edge && !near_end) { certain = 1; break; }
      if (near_edge) local_amb |= OR_AMB_EDGE;
      if (near_end) local_amb |= OR_AMB_END;
    }
  }
  if (!certain) *amb |= local_amb;
  return blocked;
}

/* ------------------------------------------------------------------------ */
/* Section 3.2's own test: does segment a->b, over the part (eps_end,         */
/* L - eps_end) of its length L, reach the bounding box of a moved object?     */
/* The decision is taken on the exact boxes and interval; *amb gets           */
/* OR_AMB_BOX when growing, or shrinking, every box and the interval by the   */
/* band would change it.                                                      */

static int seg_reaches_moved_box(const accel_t* A, const double a[3], const double b[3], double band,
                                 uint32_t* amb) {
  const or_scene* s = A->s;
  double d[3];
  sub3(b, a, d);
  double L = norm3(d);
  if (L <= 0.0) return 0;
  double e = s->eps_end;
  int hit = 0, grown = 0, shrunk = 0;
  for (int32_t o = 1; o < s->n_obj; ++o) {
    if (!s->obj_moved[o]) continue;
    const double* lo = A->obox + 6 * o;
    const double* hi = lo + 3;
    if (e <= L - e) hit |= seg_box(a, d, e / L, (L - e) / L, lo, hi, 0.0);
    grown |= seg_box(a, d, (e - band) / L, (L - e + band) / L, lo, hi, band);
    if (e + band <= L - e - band) shrunk |= seg_box(a, d, (e + band) / L, (L - e - band) / L, lo, hi, -band);
  }
  if (grown != shrunk) *amb |= OR_AMB_BOX;
  return hit;
}

/* ------------------------------------------------------------------------ */
/* Closest hit over every triangle (static and dynamic), two-sided, with the  */
/* ray o + t w (w unit), t > eps_end.  Ties at equal t: lowest triangle id.   */

typedef struct {
  double t;
  int64_t tri;
} hit_t;

static hit_t closest_hit(const accel_t* A, const double o[3], const double w[3], double band,
                         uint32_t* amb) {
  const or_scene* s = A->s;
  double e = s->eps_end;
  hit_t h = {INFINITY, -1};
  for (int64_t c = 0; c < A->n_ch; ++c) {
    const chunk_t* ch = &A->ch[c];
    double tmax = h.tri >= 0 ? h.t : T_FAR;
    if (!seg_box(o, w, e, tmax, ch->lo, ch->hi, 1e-9)) continue;
    for (int64_t t = ch->first; t < ch->first + ch->count; ++t) {
      double v[9], tt, u, vv;
      tri_verts(s, t, v);
      if (!mt_plane(o, w, v, v + 3, v + 6, &tt, &u, &vv)) continue;
      if (!inside_uv(u, vv) || !(tt > e)) continue;
      if (tt < h.t || (tt == h.t && t < h.tri)) { h.t = tt; h.tri = t; }
    }
  }
  /* ambiguity: any triangle edge within band of the travelled ray, a second
     surface within band of the hit distance, or a crossing within band of
     eps_end */
  double tend = h.tri >= 0 ? h.t + band : T_FAR;
  double s0[3], s1[3];
  for (int i = 0; i < 3; ++i) { s0[i] = o[i] + (e - band) * w[i]; s1[i] = o[i] + tend * w[i]; }
  for (int64_t c = 0; c < A->n_ch; ++c) {
    const chunk_t* ch = &A->ch[c];
    if (!seg_box(o, w, e - band, tend, ch->lo, ch->hi, band + 1e-9)) continue;
    for (int64_t t = ch->first; t < ch->first + ch->count; ++t) {
      double v[9], tt, u, vv;
      tri_verts(s, t, v);
      if (tri_edge_dist(s0, s1, v) <= band) *amb |= OR_AMB_EDGE;
      if (mt_plane(o, w, v, v + 3, v + 6, &tt, &u, &vv) && inside_uv(u, vv)) {
        if (fabs(tt - e) <= band) *amb |= OR_AMB_END;
        if (t != h.tri && h.tri >= 0 && fabs(tt - h.t) <= band) *amb |= OR_AMB_TIE;
      }
    }
  }
  return h;
}

/* geometric normal of a triangle (unit, FP64) */
static void tri_normal(const or_scene* s, int64_t t, double n[3]) {
  double v[9], e1[3], e2[3];
  tri_verts(s, t, v);
  sub3(v + 3, v, e1);
  sub3(v + 6, v, e2);
  cross3(e1, e2, n);
  double l = norm3(n);
  for (int i = 0; i < 3; ++i) n[i] /= l;
}

/* ------------------------------------------------------------------------ */
/* Section 3.1, "Update path origins" for an area light: keep the outgoing    */
/* direction, intersect it with the moved light's plane; invalid when the     */
/* new origin falls outside the light or the direction leaves its back side.  */

static void light_frame(const float* xf, double c[3], double eu[3], double ev[3], double n[3]) {
  for (int r = 0; r < 3; ++r) {
    eu[r] = xf[4 * r + 0];
    ev[r] = xf[4 * r + 1];
    n[r] = xf[4 * r + 2];
    c[r] = xf[4 * r + 3];
  }
  double l = norm3(n);
  for (int r = 0; r < 3; ++r) n[r] /= l;
}

/* whether the unit direction d (light frame eu, ev, n) lies in the emission */
/* set of a zero-extent light of kind 'kind' (flags decisions within band)    */
static int emits(int32_t kind, const float* param, const double eu[3], const double ev[3],
                 const double n[3], const double d[3], double band, uint32_t* amb) {
  const double z = dot3(d, n);
  if (fabs(z) <= band) *amb |= OR_AMB_LIGHT;
  if (!(z > 0.0)) return 0;
  if (kind == OR_LIGHT_SPOT) {
    /* inside the cone: cos of the angle to the axis at least param[0] */
    if (fabs(z - param[0]) <= band) *amb |= OR_AMB_LIGHT;
    return z >= param[0];
  }
  if (kind == OR_LIGHT_CAMERA) {
    /* through the near plane at unit distance: |x / z| <= tu, |y / z| <= tv */
    const double a = dot3(d, eu) / z, b = dot3(d, ev) / z;
    if (fabs(fabs(a) - param[0]) <= band || fabs(fabs(b) - param[1]) <= band) *amb |= OR_AMB_LIGHT;
    return fabs(a) <= param[0] && fabs(b) <= param[1];
  }
  return 1;
}

int or_light_update(const float* xf, const float* half, int32_t kind, const float* param, const double x0[3],
                    const double x1[3], double eps, double band, double out[3], uint32_t* amb) {
  double c[3], eu[3], ev[3], n[3], w[3];
  light_frame(xf, c, eu, ev, n);
  if (half[0] == 0.0f && half[1] == 0.0f) {
    /* point, spot or camera: the sample is the light's new position and     */
    /* segment 0 is re-aimed at the first photon; it must be longer than eps */
    /* and leave within the emission set (its visibility is tested by the    */
    /* caller)                                                               */
    sub3(x1, c, w);
    double len = norm3(w);
    if (fabs(len - eps) <= band) *amb |= OR_AMB_LIGHT;
    if (!(len > eps)) return 0;
    for (int i = 0; i < 3; ++i) w[i] /= len;
    if (!emits(kind, param, eu, ev, n, w, band, amb)) return 0;
    for (int i = 0; i < 3; ++i) out[i] = c[i];
    return 1;
  }
  sub3(x1, x0, w);
  double len = norm3(w);
  if (len <= 0.0) return 0;
  for (int i = 0; i < 3; ++i) w[i] /= len;
  double dn = dot3(w, n);
  if (fabs(dn) <= band) *amb |= OR_AMB_LIGHT;
  if (!(dn > 0.0)) return 0;
  double q[3];
  sub3(x1, c, q);
  double sdist = dot3(q, n) / dn;
  if (fabs(sdist - eps) <= band) *amb |= OR_AMB_LIGHT;
  if (!(sdist > eps)) return 0;
  double p[3];
  for (int i = 0; i < 3; ++i) p[i] = x1[i] - sdist * w[i];
  double r[3];
  sub3(p, c, r);
  double u = dot3(r, eu), v = dot3(r, ev);
  if (fabs(fabs(u) - half[0]) <= band || fabs(fabs(v) - half[1]) <= band) *amb |= OR_AMB_LIGHT;
  if (!(fabs(u) <= half[0] && fabs(v) <= half[1])) return 0;
  for (int i = 0; i < 3; ++i) out[i] = p[i];
  return 1;
}

static int32_t lkind(const or_scene* s, int l) { return s->light_kind ? s->light_kind[l] : OR_LIGHT_AREA; }
static const float* lparam(const or_scene* s, int l) {
  static const float none[2] = {0.0f, 0.0f};
  return s->light_param ? s->light_param + 2 * l : none;
}

static int light_of(const or_scene* s, int64_t p) {
  for (int l = 0; l < s->n_lights; ++l)
    if (p >= s->light_base[l] && p < s->light_base[l + 1]) return l;
  return -1;
}

/* ------------------------------------------------------------------------ */
/* path vertex access: x_0 = origin, x_j = row j-1                            */

static void vtx(const or_store* st, int64_t p, int j, double o[3]) {
  if (j == 0)
    load3f(st->origin + 3 * p, o);
  else
    load3f(st->pos + 3 * ((int64_t)(j - 1) * st->n_paths + p), o);
}
static uint32_t vhit(const or_store* st, int64_t p, int j) {
  return st->hit[(int64_t)(j - 1) * st->n_paths + p];
}
static int hit_on_moved(const or_scene* s, uint32_t h) {
  if (h == HIT_NONE || (int64_t)h >= s->n_tris) return 0;
  uint32_t o = s->tri_obj[h];
  return o != 0 && s->obj_moved[o];
}

/* ------------------------------------------------------------------------ */
/* Dynamic occlusions (Section 3.2) preceded by the origin update (Section   */
/* 3.1), per path, by definition: segments are tested in order from the one  */
/* leaving the light, and the first invalid one and all later ones are        */
/* scheduled for re-tracing.  The origin is rewritten for moved lights and    */
/* the information word gets replace / start / reuse-light.                   */

static void verify_path(const or_scene* s, const accel_t* A, or_store* st, int64_t p,
                        uint32_t* amb_out, int32_t* examined_out) {
  const double band = s->band_verify;
  uint32_t w = st->info[p];
  uint32_t n = info_nseg(w), cell = info_cell(w);
  uint32_t a = 0;
  int ex = 0, done = 0;
  int l = light_of(s, p);
  uint32_t out = info_make(cell, n, 0, 0, 0);
  int visibility = 0; /* segment 0 is tested against every triangle */
  if (l >= 0 && s->light_moved[l]) {
    double x0[3], x1[3], nx[3];
    if (n == 0) {
      done = 1; /* no photon to aim at: a new light sample is drawn */
    } else {
      vtx(st, p, 0, x0);
      vtx(st, p, 1, x1);
      if (or_light_update(s->light_xf + 12 * l, s->light_half + 2 * l, lkind(s, l), lparam(s, l), x0, x1,
                          s->eps_end, band, nx, &a)) {
        store3f(st->origin + 3 * p, nx);
        visibility = s->light_half[2 * l] == 0.0f && s->light_half[2 * l + 1] == 0.0f;
      } else {
        done = 1;
      }
    }
    if (done) out = info_make(cell, n, 0, 1, 0);
  }
  for (uint32_t j = 0; j < n && !done; ++j) {
    double xa[3], xb[3];
    vtx(st, p, (int)j, xa);
    vtx(st, p, (int)j + 1, xb);
    ++ex;
    int inv = hit_on_moved(s, vhit(st, p, (int)j + 1));
    if (!inv && s->verify_boxes) inv = seg_reaches_moved_box(A, xa, xb, s->band_box, &a);
    if (!inv) {
      if (j == 0 && visibility)
        inv = seg_blocked(A, xa, xb, band, 1, &a); /* every triangle: the point light's visibility */
      else if (!s->verify_boxes)
        inv = seg_blocked(A, xa, xb, band, 0, &a); /* the moved objects' triangles */
    }
    if (inv) {
      out = info_make(cell, n, j, 1, 1);
      done = 1;
    }
  }
  st->info[p] = out;
  *amb_out = a;
  *examined_out = ex;
}

/* all paths; out: amb[p] flags, examined[p] segments examined */
void or_verify(const or_scene* s, or_store* st, uint32_t* amb, int32_t* examined) {
  accel_t A;
  accel_build(&A, s);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t p = 0; p < st->n_paths; ++p) verify_path(s, &A, st, p, &amb[p], &examined[p]);
  accel_free(&A);
}

/* only the listed paths (a sample); amb / examined indexed like the list */
void or_verify_list(const or_scene* s, or_store* st, const int64_t* list, int64_t n_list,
                    uint32_t* amb, int32_t* examined) {
  accel_t A;
  accel_build(&A, s);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n_list; ++i) verify_path(s, &A, st, list[i], &amb[i], &examined[i]);
  accel_free(&A);
}

/* stand-alone segment query for tests: returns 0/1, amb flags */
int or_segment_query(const or_scene* s, const double a[3], const double b[3], uint32_t* amb) {
  accel_t A;
  accel_build(&A, s);
  int r = seg_blocked(&A, a, b, s->band_verify, 0, amb);
  accel_free(&A);
  return r;
}

/* stand-alone closest-hit query for tests */
int64_t or_closest_query(const or_scene* s, const double o[3], const double w[3], double* t,
                         uint32_t* amb) {
  accel_t A;
  accel_build(&A, s);
  hit_t h = closest_hit(&A, o, w, s->band_trace, amb);
  accel_free(&A);
  *t = h.t;
  return h.tri;
}

/* ------------------------------------------------------------------------ */
/* Re-tracing (Section 3.2 naive; Section 3.3 / Algorithm 1 error-based)     */

typedef struct {
  const or_scene* s;
  const accel_t* A;
  or_store* st;
  uint64_t seed;
  uint64_t frame;
  float T;
} rctx;

static void put_photon(or_store* st, int64_t p, int row, const double x[3], uint32_t hit,
                       const float e[3], float radius) {
  int64_t i = (int64_t)row * st->n_paths + p;
  store3f(st->pos + 3 * i, x);
  st->hit[i] = hit;
  st->energy[3 * i + 0] = e[0];
  st->energy[3 * i + 1] = e[1];
  st->energy[3 * i + 2] = e[2];
  st->radius[i] = radius;
}

static void clear_rows(or_store* st, int64_t p, int from) {
  for (int r = from; r < st->B; ++r) {
    int64_t i = (int64_t)r * st->n_paths + p;
    st->pos[3 * i] = st->pos[3 * i + 1] = st->pos[3 * i + 2] = 0.0f;
    st->hit[i] = HIT_NONE;
    st->energy[3 * i] = st->energy[3 * i + 1] = st->energy[3 * i + 2] = 0.0f;
    st->radius[i] = 0.0f;
  }
}

static void energy_row(const or_store* st, int64_t p, int row, float e[3]) {
  int64_t i = (int64_t)row * st->n_paths + p;
  e[0] = st->energy[3 * i]; e[1] = st->energy[3 * i + 1]; e[2] = st->energy[3 * i + 2];
}

/* E_next = E (x) albedo, per channel, rounded to FP32 (the product of two    */
/* FP32 numbers is exact in FP64, so this is the FP32 product)                */
static void reflect(const or_scene* s, const float e[3], uint32_t tri, float out[3]) {
  const float* rho = s->albedo + 3 * s->tri_mat[tri];
  for (int c = 0; c < 3; ++c) out[c] = (float)((double)e[c] * (double)rho[c]);
}

/* Trace new bounces from photon row 'row0' (vertex x_{row0+1}) with energy  */
/* e_row0 already stored, sampling cosine-weighted directions, up to B.      */
/* w_in: direction that arrived at that vertex.  Returns the photon count.   */
static int naive_tail(rctx* c, int64_t p, int row0, const double x_in[3], const double w_in[3],
                      uint32_t tri_in, const float e_in[3], uint32_t* amb, int* traces) {
  double x[3] = {x_in[0], x_in[1], x_in[2]}, w[3] = {w_in[0], w_in[1], w_in[2]};
  uint32_t tri = tri_in;
  float e[3] = {e_in[0], e_in[1], e_in[2]};
  int row = row0;
  while (row + 1 < c->st->B) {
    double n[3], u[4], wn[3];
    tri_normal(c->s, tri, n);
    if (dot3(n, w) > 0.0)
      for (int i = 0; i < 3; ++i) n[i] = -n[i];
    draw4(c->seed, (uint64_t)p, c->frame, (uint64_t)(row + 1), 1, u);
    or_cosine_dir(u[0], u[1], n, wn);
    hit_t h = closest_hit(c->A, x, wn, c->s->band_trace, amb);
    ++*traces;
    if (h.tri < 0) break;
    double xn[3];
    for (int i = 0; i < 3; ++i) xn[i] = x[i] + h.t * wn[i];
    float en[3];
    reflect(c->s, e, tri, en);
    ++row;
    put_photon(c->st, p, row, xn, (uint32_t)h.tri, en, c->s->radius);
    for (int i = 0; i < 3; ++i) { x[i] = xn[i]; w[i] = wn[i]; }
    tri = (uint32_t)h.tri;
    e[0] = en[0]; e[1] = en[1]; e[2] = en[2];
  }
  return row + 1;
}

/* Trace segment k from x_k along direction w and continue naively.          */
/* Writes photons rows k.., returns the photon count.                          */
static int naive_from(rctx* c, int64_t p, int k, const double xk[3], const double w[3],
                      uint32_t* amb, int* traces) {
  const or_scene* s = c->s;
  or_store* st = c->st;
  int l = light_of(s, p);
  hit_t h = closest_hit(c->A, xk, w, s->band_trace, amb);
  ++*traces;
  if (h.tri < 0) return k;
  double xn[3];
  for (int i = 0; i < 3; ++i) xn[i] = xk[i] + h.t * w[i];
  float en[3];
  if (k == 0) {
    int64_t Nl = s->light_base[l + 1] - s->light_base[l];
    for (int ch = 0; ch < 3; ++ch) en[ch] = (float)((double)s->light_power[3 * l + ch] / (double)Nl);
  } else {
    float ek[3];
    energy_row(st, p, k - 1, ek);
    reflect(s, ek, vhit(st, p, k), en);
  }
  put_photon(st, p, k, xn, (uint32_t)h.tri, en, s->radius);
  return naive_tail(c, p, k, xn, w, (uint32_t)h.tri, en, amb, traces);
}

/* new light sample, from one Philox draw (tag 0): position uniform on the  */
/* rectangle (the centre for a zero-extent light); direction cosine-weighted  */
/* about the light normal, restricted for a spot light to its cone (the disk  */
/* point scaled to the cone's radius sin(theta) before the lift, which keeps  */
/* the cosine weighting inside the cone), and for a camera uniform on the     */
/* near plane at unit distance, |x| <= tu, |y| <= tv                          */
void or_light_sample(const float* xf, const float* half, int32_t kind, const float* param, uint64_t seed,
                     uint64_t path, uint64_t frame, double x0[3], double w[3]) {
  double u[4], c[3], eu[3], ev[3], n[3], l[3];
  draw4(seed, path, frame, 0, 0, u);
  light_frame(xf, c, eu, ev, n);
  double a = (2.0 * u[0] - 1.0) * half[0], b = (2.0 * u[1] - 1.0) * half[1];
  for (int i = 0; i < 3; ++i) x0[i] = c[i] + a * eu[i] + b * ev[i];
  if (kind == OR_LIGHT_CAMERA) {
    const double x = (2.0 * u[0] - 1.0) * param[0], y = (2.0 * u[1] - 1.0) * param[1];
    const double len = sqrt(x * x + y * y + 1.0);
    for (int i = 0; i < 3; ++i) w[i] = (x * eu[i] + y * ev[i] + n[i]) / len;
    return;
  }
  or_cosine_local(u[2], u[3], l);
  if (kind == OR_LIGHT_SPOT) {
    const double sr = sqrt((1.0 - (double)param[0]) * (1.0 + (double)param[0]));
    l[0] *= sr;
    l[1] *= sr;
    const double r2 = l[0] * l[0] + l[1] * l[1];
    l[2] = sqrt(1.0 - r2 > 0.0 ? 1.0 - r2 : 0.0);
  }
  for (int i = 0; i < 3; ++i) w[i] = l[0] * eu[i] + l[1] * ev[i] + l[2] * n[i];
}

/* ------------------------------------------------------------------------ */
/* Distribution maps (Section 3.1).  The light's surface and its set of       */
/* outgoing directions are partitioned into cells; DM_T holds the targeted     */
/* number of paths per cell, DM_C the number of existing paths.  Reading of    */
/* the parametrisation the paper leaves open: a rectangle's cell is a          */
/* position cell of a gu x gv grid over its local (u, v), times a direction    */
/* cell of the unit disk of the direction's local (x, y) components, cut into  */
/* 'rings' rings of equal area (equal steps of x^2 + y^2) and 'sectors'       */
/* sectors of equal angle.  Cosine-weighted emission is uniform on that disk   */
/* (Malley's method), so every cell of a light is equally likely; a point      */
/* light has the direction cells only.  Cell index:                            */
/* ((iu * gv + iv) * rings + ring) * sectors + sector.                         */

static const double PI_D = 3.14159265358979323846;

static int dm_point(const float* half) { return half[0] == 0.0f && half[1] == 0.0f; }

/* a camera's cells are a gu x gv grid over its near plane (the pixels); a  */
/* spot light's direction cells cover the disk of its cone, radius          */
/* sin(theta), in the same rings (equal area) and sectors                   */
int64_t or_dm_cells(const float* half, int32_t kind, const int32_t* dm) {
  if (kind == OR_LIGHT_CAMERA) return (int64_t)dm[0] * dm[1];
  return (int64_t)(dm_point(half) ? 1 : dm[0] * dm[1]) * dm[2] * dm[3];
}

/* DM_T: the light's paths spread evenly, the first N mod C cells one more */
static int64_t dm_target_of(int64_t n_paths, int64_t n_cells, int64_t c) {
  return n_paths / n_cells + (c < n_paths % n_cells ? 1 : 0);
}
void or_dm_target(int64_t n_cells, int64_t n_paths, uint32_t* target) {
  for (int64_t c = 0; c < n_cells; ++c) target[c] = (uint32_t)dm_target_of(n_paths, n_cells, c);
}

/* distance of x to the nearest integer */
static double frac_dist(double x) { return fabs(x - floor(x + 0.5)); }

/* The cell of a light sample (origin x0 on the light, unit direction w), or  */
/* -1 when the parametrisation has no value for it (origin off the rectangle, */
/* direction not on the emitting side).  Decisions within 'band' of a cell    */
/* boundary (in scene units on the light, in disk units for the direction)    */
/* set OR_AMB_CELL.                                                           */
int64_t or_dm_cell(const float* xf, const float* half, int32_t kind, const float* param, const int32_t* dm,
                   const double x0[3], const double w[3], double band, uint32_t* amb) {
  double c[3], eu[3], ev[3], n[3];
  light_frame(xf, c, eu, ev, n);
  if (kind == OR_LIGHT_CAMERA) {
    const double z = dot3(w, n);
    if (fabs(z) <= band) *amb |= OR_AMB_CELL;
    if (!(z > 0.0)) return -1;
    const double fu = (dot3(w, eu) / z + param[0]) / (2.0 * param[0]) * dm[0];
    const double fv = (dot3(w, ev) / z + param[1]) / (2.0 * param[1]) * dm[1];
    if (!(fu >= 0.0 && fu <= dm[0] && fv >= 0.0 && fv <= dm[1])) return -1;
    if (frac_dist(fu) * (2.0 * param[0] / dm[0]) <= band || frac_dist(fv) * (2.0 * param[1] / dm[1]) <= band)
      *amb |= OR_AMB_CELL;
    int64_t iu = (int64_t)floor(fu), iv = (int64_t)floor(fv);
    if (iu > dm[0] - 1) iu = dm[0] - 1;
    if (iv > dm[1] - 1) iv = dm[1] - 1;
    return iu * dm[1] + iv;
  }
  /* squared radius of the direction disk: 1, or sin^2 of a spot's cone */
  const double s2 = kind == OR_LIGHT_SPOT ? (1.0 - (double)param[0]) * (1.0 + (double)param[0]) : 1.0;
  const int point = dm_point(half);
  const int gu = point ? 1 : dm[0], gv = point ? 1 : dm[1], nr = dm[2], ns = dm[3];
  int64_t iu = 0, iv = 0;
  if (!point) {
    double r[3];
    sub3(x0, c, r);
    const double u = dot3(r, eu), v = dot3(r, ev);
    const double fu = (u + half[0]) / (2.0 * half[0]) * gu, fv = (v + half[1]) / (2.0 * half[1]) * gv;
    if (!(fu >= 0.0 && fu <= gu && fv >= 0.0 && fv <= gv)) return -1;
    if (frac_dist(fu) * (2.0 * half[0] / gu) <= band || frac_dist(fv) * (2.0 * half[1] / gv) <= band)
      *amb |= OR_AMB_CELL;
    iu = (int64_t)floor(fu);
    iv = (int64_t)floor(fv);
    if (iu > gu - 1) iu = gu - 1;
    if (iv > gv - 1) iv = gv - 1;
  }
  const double x = dot3(w, eu), y = dot3(w, ev), z = dot3(w, n);
  if (fabs(z) <= band) *amb |= OR_AMB_CELL;
  if (!(z > 0.0)) return -1;
  const double rho2 = x * x + y * y, rho = sqrt(rho2);
  const double fr = rho2 / s2 * nr;
  if (frac_dist(fr) / nr * s2 <= band) *amb |= OR_AMB_CELL;
  if (kind == OR_LIGHT_SPOT && !(fr <= nr)) return -1; /* outside the cone */
  int64_t ring = (int64_t)floor(fr);
  if (ring > nr - 1) ring = nr - 1;
  const double phi = atan2(y, x);  /* (-pi, pi] */
  const double fs = (phi + PI_D) / (2.0 * PI_D) * ns;
  if (rho <= band || rho * frac_dist(fs) * (2.0 * PI_D / ns) <= band) *amb |= OR_AMB_CELL;
  int64_t sector = (int64_t)floor(fs);
  if (sector > ns - 1) sector = ns - 1;
  if (sector < 0) sector = 0;
  return ((iu * gv + iv) * nr + ring) * ns + sector;
}

/* A new light sample inside cell 'cell' (Section 3.1, "Fill DM_C": sampling */
/* restricted to the cell): position uniform in the cell's part of the        */
/* rectangle, disk point uniform in the cell's ring and sector (uniform in     */
/* x^2 + y^2 and in angle), lifted to the hemisphere; one Philox draw, tag 0. */
void or_dm_sample(const float* xf, const float* half, int32_t kind, const float* param, const int32_t* dm,
                  int64_t cell, uint64_t seed, uint64_t path, uint64_t frame, double x0[3], double w[3]) {
  double u[4], c[3], eu[3], ev[3], n[3];
  draw4(seed, path, frame, 0, 0, u);
  light_frame(xf, c, eu, ev, n);
  if (kind == OR_LIGHT_CAMERA) {
    /* uniform in the pixel's part of the near plane */
    const int64_t iu = cell / dm[1], iv = cell % dm[1];
    const double x = -param[0] + ((double)iu + u[0]) * (2.0 * param[0] / dm[0]);
    const double y = -param[1] + ((double)iv + u[1]) * (2.0 * param[1] / dm[1]);
    const double len = sqrt(x * x + y * y + 1.0);
    for (int i = 0; i < 3; ++i) {
      x0[i] = c[i];
      w[i] = (x * eu[i] + y * ev[i] + n[i]) / len;
    }
    return;
  }
  const double s2 = kind == OR_LIGHT_SPOT ? (1.0 - (double)param[0]) * (1.0 + (double)param[0]) : 1.0;
  const int point = dm_point(half);
  const int64_t gv = point ? 1 : dm[1], nr = dm[2], ns = dm[3];
  const int64_t gu = point ? 1 : dm[0];
  const int64_t sector = cell % ns, ring = (cell / ns) % nr, pc = cell / (ns * nr);
  const int64_t iv = pc % gv, iu = pc / gv;
  if (point) {
    for (int i = 0; i < 3; ++i) x0[i] = c[i];
  } else {
    const double a = -half[0] + ((double)iu + u[0]) * (2.0 * half[0] / (double)gu);
    const double b = -half[1] + ((double)iv + u[1]) * (2.0 * half[1] / (double)gv);
    for (int i = 0; i < 3; ++i) x0[i] = c[i] + a * eu[i] + b * ev[i];
  }
  const double rho2 = ((double)ring + u[2]) / (double)nr * s2, rho = sqrt(rho2);
  const double phi = -PI_D + ((double)sector + u[3]) * (2.0 * PI_D / (double)ns);
  const double lx = rho * cos(phi), ly = rho * sin(phi), lz = sqrt(1.0 - rho2 > 0.0 ? 1.0 - rho2 : 0.0);
  for (int i = 0; i < 3; ++i) w[i] = lx * eu[i] + ly * ev[i] + lz * n[i];
}

/* offset of light l's cells in the maps of all lights */
static int64_t dm_offset(const or_scene* s, int l) {
  int64_t off = 0;
  for (int i = 0; i < l; ++i) off += or_dm_cells(s->light_half + 2 * i, lkind(s, i), s->dm);
  return off;
}

/* The three distribution-map steps of Section 3.1 after the origin update,  */
/* in the paper's order, on the whole store:                                  */
/*  Compute DM_C: every path whose light sample survived the update counts in */
/*    its cell (a moved light's sample gets its cell from its updated origin  */
/*    and its kept direction; a path the parametrisation cannot place is      */
/*    marked for re-sampling; otherwise the stored cell);                     */
/*  Prune paths: in a cell with DM_C > DM_T each path is pruned with          */
/*    probability (DM_C - DM_T) / DM_C (Equation 1), decided in FP32 against  */
/*    one Philox uniform (vertex 0, tag 2), all decisions taken with the      */
/*    counts before any pruning and the counts lowered afterwards (the two    */
/*    passes of Section 4);                                                   */
/*  Fill DM_C: the paths to re-sample (replace without reuse-light: lost by  */
/*    the update, pruned, or all of them at the first frame), in path order,  */
/*    are given the cells still below target: the i-th re-sampled path of a   */
/*    light takes the cell where the running sum of the deficits              */
/*    max(0, DM_T - DM_C) passes i.                                           */
/* dm_c / dm_pruned (all lights' cells) receive the counts of the first step  */
/* and the pruned paths per cell.                                             */
void or_dm_update(const or_scene* s, or_store* st, uint64_t seed, uint64_t frame, uint32_t* dm_c,
                  uint32_t* dm_pruned, uint32_t* amb) {
  const int32_t* dm = s->dm;
  const int64_t total = dm_offset(s, s->n_lights);
  memset(dm_c, 0, sizeof(uint32_t) * total);
  memset(dm_pruned, 0, sizeof(uint32_t) * total);
  /* Compute DM_C */
  for (int64_t p = 0; p < st->n_paths; ++p) {
    const int l = light_of(s, p);
    if (l < 0) continue;
    uint32_t w = st->info[p];
    if (info_replace(w) && !info_reuse(w)) continue;
    int64_t cell = info_cell(w);
    if (s->light_moved[l]) {
      double x0[3], x1[3], d[3];
      vtx(st, p, 0, x0);
      vtx(st, p, 1, x1);
      sub3(x1, x0, d);
      const double len = norm3(d);
      for (int i = 0; i < 3; ++i) d[i] /= len;
      cell = or_dm_cell(s->light_xf + 12 * l, s->light_half + 2 * l, lkind(s, l), lparam(s, l), dm, x0, d,
                        s->band_verify, &amb[p]);
      if (cell < 0) {
        st->info[p] = info_make(0, info_nseg(w), 0, 1, 0);
        continue;
      }
      st->info[p] = info_make((uint32_t)cell, info_nseg(w), info_start(w), info_replace(w), info_reuse(w));
    }
    dm_c[dm_offset(s, l) + cell] += 1;
  }
  /* Prune paths (Equation 1) */
  for (int64_t p = 0; p < st->n_paths; ++p) {
    const int l = light_of(s, p);
    if (l < 0) continue;
    const uint32_t w = st->info[p];
    if (info_replace(w) && !info_reuse(w)) continue;
    const int64_t at = dm_offset(s, l) + info_cell(w);
    const int64_t cells = or_dm_cells(s->light_half + 2 * l, lkind(s, l), dm);
    const uint32_t tgt = (uint32_t)dm_target_of(s->light_base[l + 1] - s->light_base[l], cells, info_cell(w));
    const uint32_t C = dm_c[at];
    if (C <= tgt) continue;
    double u[4];
    draw4(seed, (uint64_t)p, frame, 0, 2, u);
    const float prob = (float)(C - tgt) / (float)C;
    if ((float)u[0] < prob) {
      st->info[p] = info_make(info_cell(w), info_nseg(w), 0, 1, 0);
      dm_pruned[at] += 1;
    }
  }
  /* Fill DM_C */
  for (int l = 0; l < s->n_lights; ++l) {
    const int64_t off = dm_offset(s, l), cells = or_dm_cells(s->light_half + 2 * l, lkind(s, l), dm);
    const int64_t Nl = s->light_base[l + 1] - s->light_base[l];
    int64_t c = 0, run = 0, i = 0;
    for (int64_t p = s->light_base[l]; p < s->light_base[l + 1]; ++p) {
      const uint32_t w = st->info[p];
      if (!(info_replace(w) && !info_reuse(w))) continue;
      /* advance to the cell whose running deficit sum passes i */
      while (c < cells) {
        const int64_t tgt = dm_target_of(Nl, cells, c);
        const int64_t have = (int64_t)dm_c[off + c] - (int64_t)dm_pruned[off + c];
        const int64_t def = tgt > have ? tgt - have : 0;
        if (run + def > i) break;
        run += def;
        ++c;
      }
      const int64_t cell = c < cells ? c : i % cells;
      st->info[p] = info_make((uint32_t)cell, info_nseg(w), info_start(w), 1, 0);
      ++i;
    }
  }
}

/* Section 3.3 energy test, Equation 2, per channel, inclusive, evaluated in */
/* FP32 (the precision of the stored energies).                              */
int or_eq2(const float en[3], const float eo[3], float T) {
  for (int c = 0; c < 3; ++c) {
    volatile float d = en[c] - eo[c];
    volatile float te = T * eo[c];
    volatile float mte = -te;
    if (!(mte <= d && d <= te)) return 0;
  }
  return 1;
}

static void retrace_path(rctx* c, int64_t p, uint32_t* amb, int* traces) {
  const or_scene* s = c->s;
  or_store* st = c->st;
  uint32_t w = st->info[p];
  uint32_t n = info_nseg(w), k = info_start(w), cell = info_cell(w);
  int newn;
  *traces = 0;
  if (!info_replace(w)) return;
  if (k == 0 && !info_reuse(w)) {
    int l = light_of(s, p);
    double x0[3], w0[3];
    if (s->dm)
      or_dm_sample(s->light_xf + 12 * l, s->light_half + 2 * l, lkind(s, l), lparam(s, l), s->dm, info_cell(w),
                   c->seed, (uint64_t)p, c->frame, x0, w0);
    else
      or_light_sample(s->light_xf + 12 * l, s->light_half + 2 * l, lkind(s, l), lparam(s, l), c->seed,
                      (uint64_t)p, c->frame, x0, w0);
    store3f(st->origin + 3 * p, x0);
    double x0f[3];
    vtx(st, p, 0, x0f);
    newn = naive_from(c, p, 0, x0f, w0, amb, traces);
  } else if (c->T < 0.0f) {
    double xa[3], xb[3], d[3];
    vtx(st, p, (int)k, xa);
    vtx(st, p, (int)k + 1, xb);
    sub3(xb, xa, d);
    double L = norm3(d);
    for (int i = 0; i < 3; ++i) d[i] /= L;
    newn = naive_from(c, p, (int)k, xa, d, amb, traces);
  } else {
    /* Algorithm 1 with the readings: trace iff blocked, origin moved, or end
       photon on a moved object; after an accepted re-hit that lands within
       eps_close of the old vertex, the following segment is kept without a
       trace when it is itself clear.  Segment k itself is known to be
       blocked after the triangle test; after the box test (Section 3.2's
       own) it only reached a moved object's box, and Section 3.3 casts no
       visibility ray for a segment that the object's box crosses but none of
       its triangles: when segment k's origin is unchanged (k > 0, or the
       light did not move) the walk first checks it against the triangles. */
    int l = light_of(s, p);
    int origin_moved = k == 0 && l >= 0 && s->light_moved[l];
    int j = (int)k, need = !(s->verify_boxes && !origin_moved);
    newn = (int)n;
    while (j < newn) {
      double xa[3], xb[3];
      vtx(st, p, j, xa);
      vtx(st, p, j + 1, xb);
      if (!need) {
        int inv = hit_on_moved(s, vhit(st, p, j + 1));
        if (!inv) inv = seg_blocked(c->A, xa, xb, s->band_trace, 0, amb);
        if (!inv) { ++j; continue; }
      }
      double d[3];
      sub3(xb, xa, d);
      double L = norm3(d);
      for (int i = 0; i < 3; ++i) d[i] /= L;
      hit_t h = closest_hit(c->A, xa, d, s->band_trace, amb);
      ++*traces;
      if (h.tri < 0) { newn = j; break; }
      double hp[3];
      for (int i = 0; i < 3; ++i) hp[i] = xa[i] + h.t * d[i];
      if (j == newn - 1) {
        float e[3];
        energy_row(st, p, j, e);
        put_photon(st, p, j, hp, (uint32_t)h.tri, e, s->radius);
        break;
      }
      /* energy reflected at the new hit towards the old next photon */
      double xc[3], d2[3], nh[3];
      vtx(st, p, j + 2, xc);
      sub3(xc, hp, d2);
      tri_normal(s, h.tri, nh);
      double c1 = dot3(d, nh), l2 = norm3(d2);
      double c2 = l2 > 0 ? dot3(d2, nh) / l2 : 0.0;
      if (fabs(c1) <= s->band_trace || fabs(c2) <= s->band_trace) *amb |= OR_AMB_HEMI;
      float ein[3], en[3], eo[3];
      energy_row(st, p, j, ein);
      energy_row(st, p, j + 1, eo);
      if (c1 * c2 < 0.0)
        reflect(s, ein, (uint32_t)h.tri, en);
      else
        en[0] = en[1] = en[2] = 0.0f;
      if (s->energy_test == 1 && c1 * c2 < 0.0) {
        /* BRDF(Segment, NextSeg) weighted by how the kept direction was       */
        /* sampled: a diffuse bounce drawn cosine-weighted at the old vertex    */
        /* carries the albedo; the same next photon reached from the new vertex */
        /* carries the albedo times the ratio of the kept direction's cosines   */
        /* at the new and at the old vertex (reading of the cosine ratio)       */
        double no[3], d3[3];
        tri_normal(s, vhit(st, p, j + 1), no);
        sub3(xc, xb, d3);
        const double l3 = norm3(d3);
        const double co = l3 > 0.0 ? fabs(dot3(d3, no)) / l3 : 0.0;
        if (co <= s->band_trace) *amb |= OR_AMB_HEMI;
        const double ratio = co > 0.0 ? fabs(c2) / co : 0.0;
        for (int ch = 0; ch < 3; ++ch) {
          en[ch] = (float)((double)en[ch] * ratio);
          /* Equation 2 near its bound: the kernels form the ratio in FP32 */
          const double dd = fabs((double)en[ch] - (double)eo[ch]), te = (double)c->T * (double)eo[ch];
          if (fabs(dd - te) <= 1e-5 * fabs((double)eo[ch])) *amb |= OR_AMB_EQ2;
        }
      }
      if (!or_eq2(en, eo, c->T)) {
        /* energies differ: keep the new hit and resample from it */
        float ej[3];
        energy_row(st, p, j, ej);
        put_photon(st, p, j, hp, (uint32_t)h.tri, ej, s->radius);
        newn = naive_tail(c, p, j, hp, d, (uint32_t)h.tri, ej, amb, traces);
        break;
      }
      double dd[3];
      sub3(hp, xb, dd);
      double dist = norm3(dd);
      if (fabs(dist - s->eps_close) <= s->band_trace) *amb |= OR_AMB_CLOSE;
      uint32_t old_hit = vhit(st, p, j + 1);
      if (dist <= s->eps_close && !hit_on_moved(s, (uint32_t)h.tri) && !hit_on_moved(s, old_hit) &&
          !hit_on_moved(s, vhit(st, p, j + 2)) &&
          !seg_blocked(c->A, xb, xc, s->band_trace, 0, amb)) {
        j += 2;
        need = 0;
        continue;
      }
      float ej[3];
      energy_row(st, p, j, ej);
      put_photon(st, p, j, hp, (uint32_t)h.tri, ej, s->radius);
      ++j;
      need = 1;
    }
  }
  clear_rows(st, p, newn);
  st->info[p] = info_make(cell, (uint32_t)newn, 0, 0, 0);
}

/* Re-trace every path whose replace bit is set (store updated in place).    */
/* T < 0: naive re-tracing from the first invalid segment (Section 3.2);     */
/* T >= 0: the error-based walk (Section 3.3, Algorithm 1, Equation 2).      */
void or_retrace(const or_scene* s, or_store* st, float T, uint64_t seed, uint64_t frame,
                uint32_t* amb, int32_t* traces) {
  accel_t A;
  accel_build(&A, s);
  rctx c = {s, &A, st, seed, frame, T};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < st->n_paths; ++p) {
    uint32_t a = 0;
    int tr = 0;
    retrace_path(&c, p, &a, &tr);
    amb[p] = a;
    traces[p] = tr;
  }
  accel_free(&A);
}

/* Re-trace only the listed paths (a sample), same semantics. */
void or_retrace_list(const or_scene* s, or_store* st, float T, uint64_t seed, uint64_t frame,
                     const int64_t* list, int64_t n_list, uint32_t* amb, int32_t* traces) {
  accel_t A;
  accel_build(&A, s);
  rctx c = {s, &A, st, seed, frame, T};
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n_list; ++i) {
    uint32_t a = 0;
    int tr = 0;
    retrace_path(&c, list[i], &a, &tr);
    amb[i] = a;
    traces[i] = tr;
  }
  accel_free(&A);
}

/* ------------------------------------------------------------------------ */
/* Differentiation form: deposited energy of every photon recomputed from    */
/* the materials along its path, E_{p,j} = (Phi_l / N_l) prod_{i<j} rho(x_i), */
/* and its gradients with respect to albedo and light power, FP64.           */

void or_energy_forward(const or_scene* s, int64_t N, int32_t B, const uint32_t* hit,
                       const uint32_t* info, const double* albedo, const double* power,
                       double* E /* [B][N][3] */) {
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < N; ++p) {
    int l = light_of(s, p);
    double Nl = (double)(s->light_base[l + 1] - s->light_base[l]);
    uint32_t n = info_nseg(info[p]);
    double e[3];
    for (int c = 0; c < 3; ++c) e[c] = power[3 * l + c] / Nl;
    for (int r = 0; r < B; ++r) {
      int64_t i = (int64_t)r * N + p;
      if ((uint32_t)r < n) {
        if (r > 0) {
          uint32_t m = s->tri_mat[hit[(int64_t)(r - 1) * N + p]];
          for (int c = 0; c < 3; ++c) e[c] *= albedo[3 * m + c];
        }
        for (int c = 0; c < 3; ++c) E[3 * i + c] = e[c];
      } else {
        for (int c = 0; c < 3; ++c) E[3 * i + c] = 0.0;
      }
    }
  }
}

/* L = sum g . E; dL/drho_{m,c} = sum over photons j and vertices i<j with    */
/* material m of g_{j,c} E_{j,c} / rho_{m,c}; dL/dPhi_{l,c} = sum g E / Phi.  */
/* Written with the division so that it is the plain derivative of the       */
/* product; requires rho, Phi > 0.  Serial accumulation in FP64.             */
void or_energy_backward(const or_scene* s, int64_t N, int32_t B, const uint32_t* hit,
                        const uint32_t* info, const double* albedo, const double* power,
                        const double* gE, int32_t n_mat, double* g_albedo, double* g_power) {
  double* E = (double*)malloc(sizeof(double) * 3 * (size_t)N * (size_t)B);
  or_energy_forward(s, N, B, hit, info, albedo, power, E);
  memset(g_albedo, 0, sizeof(double) * 3 * (size_t)n_mat);
  memset(g_power, 0, sizeof(double) * 3 * (size_t)s->n_lights);
  for (int64_t p = 0; p < N; ++p) {
    int l = light_of(s, p);
    uint32_t n = info_nseg(info[p]);
    for (uint32_t j = 0; j < n; ++j) {
      int64_t ij = (int64_t)j * N + p;
      for (int c = 0; c < 3; ++c) {
        double ge = gE[3 * ij + c] * E[3 * ij + c];
        g_power[3 * l + c] += ge / power[3 * l + c];
        for (uint32_t i = 1; i <= j; ++i) {
          uint32_t m = s->tri_mat[hit[(int64_t)(i - 1) * N + p]];
          g_albedo[3 * m + c] += ge / albedo[3 * m + c];
        }
      }
    }
  }
  free(E);
}
