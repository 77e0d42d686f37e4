// Device-side data structures and inline routines of the path-verification
// library (gfx950).  Included by every .hip translation unit of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pv.h"

namespace pv {

// Pointers read from the scene descriptor are generic; casting them to the
// global address space lets the compiler emit global (not flat) memory
// instructions, which do not make LDS accesses (the traversal stack) wait for
// outstanding memory loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define PV_GLOBAL __attribute__((address_space(1)))
#define PV_LDS __attribute__((address_space(3)))
#else
#define PV_GLOBAL
#define PV_LDS
#endif
template <typename T>
__device__ __forceinline__ PV_GLOBAL T* G(T* p) {
  return (PV_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const PV_GLOBAL T* G(const T* p) {
  return (const PV_GLOBAL T*)p;
}

constexpr int kBlock = 256;        // threads per block of the streaming kernels
constexpr int kLdsStack = 16;      // traversal stack entries per lane held in LDS
constexpr int kPrivStack = 48;     // further entries per lane in private memory
constexpr uint32_t kHitNone = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// information word (Section 4): 22-bit cell, 4-bit count, 4-bit start,
// replace bit, reuse-light bit
__host__ __device__ inline uint32_t info_nseg(uint32_t w) { return (w >> 22) & 15u; }
__host__ __device__ inline uint32_t info_start(uint32_t w) { return (w >> 26) & 15u; }
__host__ __device__ inline uint32_t info_replace(uint32_t w) { return (w >> 30) & 1u; }
__host__ __device__ inline uint32_t info_reuse(uint32_t w) { return (w >> 31) & 1u; }
__host__ __device__ inline uint32_t info_cell(uint32_t w) { return w & 0x3fffffu; }
__host__ __device__ inline uint32_t info_pack(uint32_t cell, uint32_t nseg, uint32_t start,
                                              uint32_t replace, uint32_t reuse) {
  return (cell & 0x3fffffu) | ((nseg & 15u) << 22) | ((start & 15u) << 26) | ((replace & 1u) << 30) |
         ((reuse & 1u) << 31);
}

// ---------------------------------------------------------------------------
// BVH2 node: both child boxes stored in the parent (one 64-byte line).
//   a = lo0.xyz hi0.x, b = hi0.yz lo1.xy, c = lo1.z hi1.xyz, d = (child0, child1, parent, -)
// child >= 0: internal node index; child < 0: leaf, ~child = first_tri << 3 | (count-1)
struct alignas(16) Node {
  float4 a, b, c;
  int4 d;
};

__host__ __device__ inline int leaf_code(uint32_t first, uint32_t count) {
  return ~(int)((first << 3) | (count - 1));
}
__host__ __device__ inline uint32_t leaf_first(int code) { return ((uint32_t)~code) >> 3; }
__host__ __device__ inline uint32_t leaf_count(int code) { return (((uint32_t)~code) & 7u) + 1u; }

// Triangle record in BVH leaf order: t0 = (v0, id), t1 = (v1, material), t2 = (v2, 0).
struct alignas(16) Tri {
  float4 t0, t1, t2;
};

// ---------------------------------------------------------------------------
// scene as seen by kernels (one entry per scene of a batch; plain calls use one)
struct ObjDev {
  uint32_t gbase;      // global triangle id of its first triangle (upload order)
  uint32_t n_tris;
  uint32_t tri_base;   // first record in the dynamic Tri / local arrays (leaf order)
  uint32_t node_base;  // first node of its hierarchy in the dynamic node array
  uint32_t n_nodes;    // internal nodes of its hierarchy
  uint32_t lvl_base;   // first entry of its level offsets (n_levels + 1 entries)
  int32_t root;        // root child code (absolute node index, or leaf code)
  uint32_t n_levels;   // depth levels holding internal nodes
};

struct LightDev {
  float half[2];
  float power[3];
  uint32_t path_base, path_count;
  uint32_t pad;
};

struct LeafRec {          // a leaf of a hierarchy built on the host
  uint32_t first, count;  // triangle records
  int32_t parent;         // parent node, -1 when the leaf is the root
  uint32_t side;          // 0 = child0 of its parent, 1 = child1
};

struct SceneDev {
  // static world
  const Node* snodes;
  const Tri* stris;
  int32_t sroot;          // child code of the static root
  uint32_t n_static;
  // dynamic objects
  Node* dnodes;
  Tri* dtris;
  const float* dlocal;    // [n][9] object-space vertices in leaf order
  const uint32_t* dtri_gid;  // [n] global id of each leaf-order triangle
  const uint32_t* dlevel_nodes;  // internal nodes of each object, deepest level first
  const uint32_t* dlevel_off;    // per object: offsets of its levels in dlevel_nodes
  const ObjDev* objs;
  uint32_t n_obj;
  uint32_t n_dyn_tris;
  float* obj_aabb;        // [n_obj][6] world boxes (lo, hi)
  float* obj_xf_cur;      // [n_obj][12]
  float* obj_xf_prev;
  uint32_t* obj_moved;    // [n_obj]
  // lights
  const LightDev* lights;
  float* light_xf_cur;    // [L][12]
  float* light_xf_prev;
  uint32_t* light_moved;  // [L]
  uint32_t n_lights;
  // materials
  const float* albedo;      // [M][3]
  const uint32_t* tri_mat;  // [T] by global id
  uint32_t n_tris_total;
  // store
  float4* pos;
  float4* energy;
  float* origin;
  uint32_t* info;
  uint32_t stride, n_paths, B;
  float eps_end, eps_close, radius;
  uint32_t gpath_base;    // offset of this scene's paths in the work-queue id space
  uint32_t n_blocks;      // path blocks of the bound store
  uint32_t count_base;    // first entry of this scene's (row, block) photon counts
  uint32_t* state;        // [1] first-frame flag of the scene
};

// ---------------------------------------------------------------------------
// small vector helpers (FP32)
__device__ inline float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ inline float3 sub(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline float3 add(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ inline float3 mul(float3 a, float s) { return f3(a.x * s, a.y * s, a.z * s); }
__device__ inline float dot(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline float3 cross(float3 a, float3 b) {
  return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ inline float length(float3 a) { return sqrtf(dot(a, a)); }
__device__ inline float3 xyz(float4 v) { return f3(v.x, v.y, v.z); }
__device__ inline float comp(float3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// ---------------------------------------------------------------------------
// ray / segment query state
struct Ray {
  float3 o, d, inv;   // origin, direction (not necessarily unit), 1/direction
  float tmin, tmax;   // open interval of the parameter
  int kx, ky, kz;     // watertight-test axis permutation
  float sx, sy, sz;   // shear constants
};

__device__ inline Ray make_ray(float3 o, float3 d, float tmin, float tmax) {
  Ray r;
  r.o = o;
  r.d = d;
  const float tiny = 1e-30f;
  float dx = fabsf(d.x) > tiny ? d.x : copysignf(tiny, d.x);
  float dy = fabsf(d.y) > tiny ? d.y : copysignf(tiny, d.y);
  float dz = fabsf(d.z) > tiny ? d.z : copysignf(tiny, d.z);
  r.inv = f3(1.0f / dx, 1.0f / dy, 1.0f / dz);
  r.tmin = tmin;
  r.tmax = tmax;
  // Woop, Benthin, Wald 2013: largest |d| component becomes z
  float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  if (comp(d, kz) < 0.0f) {
    int t = kx;
    kx = ky;
    ky = t;
  }
  r.kx = kx;
  r.ky = ky;
  r.kz = kz;
  float dkz = comp(d, kz);
  r.sx = comp(d, kx) / dkz;
  r.sy = comp(d, ky) / dkz;
  r.sz = 1.0f / dkz;
  return r;
}

// Slab test of one box against the ray's current [tmin, tmax]; returns the
// entry parameter or +inf.
__device__ inline float box_entry(float lx, float ly, float lz, float hx, float hy, float hz, const Ray& r,
                                  float tmax) {
  float tx0 = (lx - r.o.x) * r.inv.x, tx1 = (hx - r.o.x) * r.inv.x;
  float ty0 = (ly - r.o.y) * r.inv.y, ty1 = (hy - r.o.y) * r.inv.y;
  float tz0 = (lz - r.o.z) * r.inv.z, tz1 = (hz - r.o.z) * r.inv.z;
  float t0 = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), r.tmin));
  float t1 = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
  return t0 <= t1 ? t0 : __builtin_inff();
}

// Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013), two-sided.
// Returns true with *t when the triangle is crossed at a parameter strictly
// inside (tmin, tmax).  The edge functions are evaluated without contraction
// so that triangles sharing an edge see the same value with opposite sign.
__device__ inline bool tri_hit(const Ray& r, float3 v0, float3 v1, float3 v2, float tmax, float* t_out) {
  float3 A = sub(v0, r.o), B = sub(v1, r.o), C = sub(v2, r.o);
  float Akz = comp(A, r.kz), Bkz = comp(B, r.kz), Ckz = comp(C, r.kz);
  float Ax = comp(A, r.kx) - r.sx * Akz, Ay = comp(A, r.ky) - r.sy * Akz;
  float Bx = comp(B, r.kx) - r.sx * Bkz, By = comp(B, r.ky) - r.sy * Bkz;
  float Cx = comp(C, r.kx) - r.sx * Ckz, Cy = comp(C, r.ky) - r.sy * Ckz;
  float U = __fsub_rn(__fmul_rn(Cx, By), __fmul_rn(Cy, Bx));
  float V = __fsub_rn(__fmul_rn(Ax, Cy), __fmul_rn(Ay, Cx));
  float W = __fsub_rn(__fmul_rn(Bx, Ay), __fmul_rn(By, Ax));
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    // exact-zero edge function: re-evaluate in double precision (same paper)
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
  if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
  float det = U + V + W;
  if (det == 0.0f) return false;
  float Az = r.sz * Akz, Bz = r.sz * Bkz, Cz = r.sz * Ckz;
  float T = U * Az + V * Bz + W * Cz;
  if (det < 0.0f) {
    T = -T;
    det = -det;
  }
  if (!(T > r.tmin * det) || !(T < tmax * det)) return false;
  *t_out = T / det;
  return true;
}

// ---------------------------------------------------------------------------
// traversal stack: the top kLdsStack entries of each lane in LDS (column per
// lane, conflict-free), deeper entries in private memory.
struct Stack {
  PV_LDS uint32_t* lds;  // &shared[0][lane]; entry i at lds[i * kBlock]
  int sp;
  int32_t priv[kPrivStack];
  __device__ inline void push(int32_t v) {
    if (sp < kLdsStack)
      lds[sp * kBlock] = (uint32_t)v;
    else
      priv[sp - kLdsStack] = v;
    ++sp;
  }
  __device__ inline int32_t pop() {
    --sp;
    return sp < kLdsStack ? (int32_t)lds[sp * kBlock] : priv[sp - kLdsStack];
  }
};

// Any-hit over one hierarchy; true when some triangle is crossed inside the
// ray's open interval.  'root' is a child code relative to 'nodes'/'tris'.
__device__ inline bool bvh_any(const Node* __restrict__ nodes_in, const Tri* __restrict__ tris_in, int32_t root,
                               const Ray& r, Stack& st) {
  const PV_GLOBAL Node* nodes = G(nodes_in);
  const PV_GLOBAL Tri* tris = G(tris_in);
  float t;
  int base = st.sp;
  int32_t cur = root;
  while (true) {
    if (cur < 0) {
      uint32_t f = leaf_first(cur), n = leaf_count(cur);
      for (uint32_t i = 0; i < n; ++i) {
        Tri tr = tris[f + i];
        if (tri_hit(r, xyz(tr.t0), xyz(tr.t1), xyz(tr.t2), r.tmax, &t)) {
          st.sp = base;
          return true;
        }
      }
      if (st.sp == base) return false;
      cur = st.pop();
      continue;
    }
    Node nd = nodes[cur];
    float e0 = box_entry(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, r, r.tmax);
    float e1 = box_entry(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, r, r.tmax);
    bool h0 = e0 != __builtin_inff(), h1 = e1 != __builtin_inff();
    if (h0 && h1) {
      int32_t nearc = e0 <= e1 ? nd.d.x : nd.d.y, farc = e0 <= e1 ? nd.d.y : nd.d.x;
      st.push(farc);
      cur = nearc;
    } else if (h0) {
      cur = nd.d.x;
    } else if (h1) {
      cur = nd.d.y;
    } else {
      if (st.sp == base) return false;
      cur = st.pop();
    }
  }
}

// Closest hit over one hierarchy: shrinks *tbest, records the record index.
__device__ inline void bvh_closest(const Node* __restrict__ nodes_in, const Tri* __restrict__ tris_in, int32_t root,
                                   const Ray& r, Stack& st, float* tbest, uint32_t* gid_best,
                                   uint32_t* rec_best, const Tri** set_best) {
  const PV_GLOBAL Node* nodes = G(nodes_in);
  const PV_GLOBAL Tri* tris = G(tris_in);
  float t;
  int base = st.sp;
  int32_t cur = root;
  while (true) {
    if (cur < 0) {
      uint32_t f = leaf_first(cur), n = leaf_count(cur);
      for (uint32_t i = 0; i < n; ++i) {
        Tri tr = tris[f + i];
        if (tri_hit(r, xyz(tr.t0), xyz(tr.t1), xyz(tr.t2), *tbest, &t)) {
          // tri_hit only reports crossings strictly closer than *tbest
          *tbest = t;
          *gid_best = __float_as_uint(tr.t0.w);
          *rec_best = f + i;
          *set_best = tris_in;
        }
      }
      if (st.sp == base) return;
      cur = st.pop();
      continue;
    }
    Node nd = nodes[cur];
    float tb = *tbest;
    float e0 = box_entry(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, r, tb);
    float e1 = box_entry(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, r, tb);
    bool h0 = e0 != __builtin_inff(), h1 = e1 != __builtin_inff();
    if (h0 && h1) {
      int32_t nearc = e0 <= e1 ? nd.d.x : nd.d.y, farc = e0 <= e1 ? nd.d.y : nd.d.x;
      st.push(farc);
      cur = nearc;
    } else if (h0) {
      cur = nd.d.x;
    } else if (h1) {
      cur = nd.d.y;
    } else {
      if (st.sp == base) return;
      cur = st.pop();
    }
  }
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) from its published
// definition; uniforms are the top 24 bits of each word times 2^-24.
__device__ inline void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

__device__ inline void draw4(uint64_t seed, uint64_t path, uint64_t frame, uint64_t vertex, uint64_t tag,
                             float u[4]) {
  uint64_t c[4] = {path, frame, vertex, tag};
  philox4x64(c, seed, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = (float)(uint32_t)(c[i] >> 40) * (1.0f / 16777216.0f);
}

// Shirley-Chiu concentric map to the unit disk, lifted to the cosine-weighted
// hemisphere (Malley): local (x, y, z).
__device__ inline float3 cosine_local(float u1, float u2) {
  float a = 2.0f * u1 - 1.0f, b = 2.0f * u2 - 1.0f, r, phi;
  const float PI4 = 0.78539816339744830962f;
  if (a == 0.0f && b == 0.0f) {
    r = 0.0f;
    phi = 0.0f;
  } else if (fabsf(a) > fabsf(b)) {
    r = a;
    phi = PI4 * (b / a);
  } else {
    r = b;
    phi = 2.0f * PI4 - PI4 * (a / b);
  }
  float x = r * cosf(phi), y = r * sinf(phi);
  // height above the disk point at radius |r|; (1-|r|) is exact for |r| >= 1/2
  float ar = fabsf(r);
  float z2 = (1.0f - ar) * (1.0f + ar);
  return f3(x, y, z2 > 0.0f ? sqrtf(z2) : 0.0f);
}

// Tangent frame of a unit normal (Duff et al., JCGT 2017).
__device__ inline void onb(float3 n, float3* t, float3* b) {
  float sign = n.z >= 0.0f ? 1.0f : -1.0f;
  float a = -1.0f / (sign + n.z);
  float c = n.x * n.y * a;
  *t = f3(1.0f + sign * n.x * n.x * a, sign * c, -sign * n.x);
  *b = f3(c, sign + n.y * n.y * a, -n.y);
}

}  // namespace pv
