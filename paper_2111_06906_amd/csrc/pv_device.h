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
// Traversal stack: entries per lane, all in LDS (dynamic shared memory sized
// per launch from the scene's hierarchy depths).  A depth-first walk holds at
// most one entry per internal ancestor of the node it visits, plus the
// sentinel at the bottom, and writes the far child one slot above the top:
// a walk through a top-level tree of depth t into a hierarchy of depth d needs
// t + d + 2 entries.
constexpr int kMaxStack = 40;
constexpr int kTopDepth = 7;  // top-level tree depth bound (the static root beside a median split of <= 64 objects)
constexpr int kMaxDepth = kMaxStack - kTopDepth - 2;
static_assert((1 << (kTopDepth - 1)) >= PV_MAX_OBJECTS, "top-level depth bound");
__host__ __device__ inline uint32_t stack_entries(uint32_t top_depth, uint32_t depth) {
  return top_depth + depth + 2;
}
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
  uint32_t tri_base;   // first record of the object in the object-space vertex arrays
  uint32_t node_base;  // first node of its hierarchy in the scene's node array
  uint32_t n_nodes;    // internal nodes of its hierarchy
  uint32_t lvl_base;   // first entry of its level offsets (n_levels + 1 entries)
  int32_t root;        // root child code in the scene's node / triangle arrays (current hierarchy)
  uint32_t n_levels;   // depth levels holding internal nodes
  int32_t sah_root;    // root of the upload-time topology (refit each frame)
  uint32_t lbvh_base;  // first node of its region for the per-frame rebuilt radix tree
  int32_t oroot;       // root of the upload-time topology with object-space boxes
  uint32_t pad_;
};

struct LightDev {
  float half[2];
  float power[3];
  uint32_t path_base, path_count;
  int32_t kind;     // PV_LIGHT_AREA / PV_LIGHT_SPOT / PV_LIGHT_CAMERA
  float param[2];   // spot: cos of the cone half-angle; camera: tan of the half field of view along u, v
  uint32_t pad[2];
};

struct LeafRec {          // a leaf of a hierarchy built on the host
  uint32_t first, count;  // triangle records
  int32_t parent;         // parent node, -1 when the leaf is the root
  uint32_t side;          // 0 = child0 of its parent, 1 = child1
};

// One hierarchy per scene: the static world's nodes, then every object's
// nodes, then two top-level trees rebuilt each frame (one over the static root
// and all object roots, one over the moved objects only).  Child codes and
// leaf triangle indices are absolute in the scene's node and triangle arrays,
// so one traversal loop serves every query.
constexpr uint32_t kTopNodes = PV_MAX_OBJECTS;  // internal nodes of one top-level tree
constexpr int32_t kRootNone = INT32_MIN;        // empty tree; never a leaf code (< 2^28 triangles)

struct SceneDev {
  Node* nodes;            // [static][objects][2 x kTopNodes]
  Tri* tris;              // [static][objects], leaf order
  int32_t* top;           // [2] per frame: root of the whole scene, root of the moved objects
  uint32_t top_base;      // first top-level node
  uint32_t n_static;
  int32_t sroot;          // static root code (kRootNone without static triangles)
  float sbox[6];          // static world box (lo, hi)
  // dynamic objects
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
  // per internal node of the objects' upload-time topologies (nodes
  // [obj_node_first, obj_node_first + n_obj_nodes) of the scene): the
  // dynamic-record ranges of its two children (a subtree holds a contiguous
  // run of the leaf order), and its object
  const uint4* dspan;
  const uint32_t* dspan_obj;
  uint32_t obj_node_first, n_obj_nodes;
  // the same topologies with fixed object-space boxes (padded for the error
  // of mapping a world segment into object space), nodes [onode_first,
  // onode_first + n_obj_nodes); ObjDev::oroot is an object's root among them
  uint32_t onode_first;
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
  uint32_t verify_boxes;  // 1: a segment that reaches a moved object's box is invalid (no triangle test)
  uint32_t energy_test;   // Equation 2's E_N: PV_ENERGY_ALBEDO or PV_ENERGY_COSINE_RATIO
  const uint32_t* gid_rec;  // [T] record of each global triangle id in the leaf-order triangle array
  float eps_end, eps_close, radius;
  uint32_t gpath_base;    // offset of this scene's paths in the work-queue id space
  uint32_t n_blocks;      // path blocks of the bound store
  uint32_t count_base;    // first entry of this scene's (row, block) photon counts
  uint32_t tile_base;     // first path tile (block of kBlock paths) of this scene
  uint32_t task_base;     // first entry of this scene's tile regions of verification tasks
  uint32_t* state;        // [1] first-frame flag of the scene
  // distribution maps (Section 3.1): grid {gu, gv, rings, sectors}, dm[0] = 0
  // when none; first cell of each light in the maps of all lights
  int32_t dm[4];
  uint32_t dm_off[PV_MAX_LIGHTS + 1];
};

// Device scratch of the per-frame object hierarchy rebuild (linear BVH over
// 30-bit Morton codes): sort keys (object << 30 | Morton code of the
// triangle's centroid) and values (dynamic triangle record) in two buffers,
// per-tile digit counts (and their scan for large sorts), parent links of the
// radix trees, a pyramid of box unions over the sorted triangles (level l
// entry k: positions [k 2^l, (k+1) 2^l)), each object's tree depth and
// centroid box.
struct LbvhWork {
  uint64_t* key[2];
  uint32_t* val[2];
  uint32_t* hist;        // [256][tiles] digit counts of a sort pass
  uint32_t* hoff;        // their exclusive scan (sorts of more than kFusedTiles tiles)
  uint32_t* htotal;      // [1]
  uint32_t* scan_tmp;    // scan_tmp_words(256 * tiles)
  int32_t* parent_leaf;  // [n_dyn] by sorted position: parent node (scene index)
  int32_t* parent_node;  // [nodes] parent node, -1 at an object's root
  float4* pyr;           // [2 * pyr_entries]: lo, hi of each pyramid entry
  uint32_t* odepth;      // [n_obj] deepest leaf of each rebuilt tree
  float* cbox;           // [n_obj][6] centroid bounds
  uint32_t n_dyn;        // dynamic triangles of the scene
  uint32_t first_node;   // scene node index of the first rebuilt node
  uint32_t n_nodes;      // rebuilt nodes of all objects
};

// first entry of pyramid level l over n positions (level sizes n, ceil(n/2), ...)
__host__ __device__ inline uint32_t pyr_level(uint32_t n, int l) {
  uint32_t off = 0, m = n;
  for (int i = 0; i < l; ++i) {
    off += m;
    m = (m + 1) / 2;
  }
  return off;
}
// entries of the whole pyramid (levels down to a single entry)
__host__ __device__ inline uint32_t pyr_entries(uint32_t n) {
  uint32_t off = 0, m = n;
  while (m > 1) {
    off += m;
    m = (m + 1) / 2;
  }
  return off + m;
}

// Verification work lists (device scratch).  A task is one segment whose ray
// reaches a moved object's box: (global path id << 4) | segment.  Each path
// tile first writes its tasks into a region of its own; a scan of the
// per-tile counts and a gather make them one list.  No atomics are needed:
// device-wide atomics on one word from thousands of blocks serialise.
struct VerifyWork {
  uint32_t* tmp;     // tasks by tile: region of a tile = kBlock * B entries
  uint32_t* tasks;   // compacted tasks
  uint32_t* tcount;  // [tiles] tasks of each tile
  uint32_t* toff;    // [tiles] their offsets in the compacted list
  uint32_t* total;   // [1] tasks in all
  uint32_t* first;   // [paths] first invalid segment found so far (global path id)
  uint32_t* part;    // per-block statistics: [scan blocks][4], then [finish blocks][2]
  uint32_t* deal;    // [kDealGroups * kDealStride] refill counters of the traversal
};

// Persistent kernels take their work lists a refill at a time from one of
// kDealGroups counters (a wave uses counter wave mod kDealGroups, each
// counter on its own 128-byte line); counter g deals the list's chunks
// g, g + kDealGroups, ... in order.
constexpr uint32_t kDealGroups = 64;
constexpr uint32_t kDealStride = 32;

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
  float3 oi;          // -o / d per axis: slab parameters are fma(bound, inv, oi)
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
  r.oi = f3(-(o.x * r.inv.x), -(o.y * r.inv.y), -(o.z * r.inv.z));
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
// entry parameter or +inf.  A slab parameter is one fused multiply-add,
// bound * (1/d) - o/d; its error (relative 2^-24 of o/d, i.e. about 6e-8 of
// the origin's coordinates in distance) stays far inside the 1e-6 padding of
// every stored box, so the test remains conservative.
__device__ inline float box_entry(float lx, float ly, float lz, float hx, float hy, float hz, const Ray& r,
                                  float tmax) {
  float tx0 = fmaf(lx, r.inv.x, r.oi.x), tx1 = fmaf(hx, r.inv.x, r.oi.x);
  float ty0 = fmaf(ly, r.inv.y, r.oi.y), ty1 = fmaf(hy, r.inv.y, r.oi.y);
  float tz0 = fmaf(lz, r.inv.z, r.oi.z), tz1 = fmaf(hz, r.inv.z, r.oi.z);
  float t0 = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), r.tmin));
  float t1 = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
  return t0 <= t1 ? t0 : __builtin_inff();
}

// Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013), two-sided.
// Returns true with *t when the triangle is crossed at a parameter strictly
// inside (tmin, tmax).  The edge functions are evaluated without contraction
// so that triangles sharing an edge see the same value with opposite sign.
// Written without early exits (the caller's loop stays one predicated block);
// only an exactly zero edge function takes the double-precision branch.
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
  const bool mixed = (U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f);
  float det = U + V + W;
  float Az = r.sz * Akz, Bz = r.sz * Bkz, Cz = r.sz * Ckz;
  float T = U * Az + V * Bz + W * Cz;
  const bool neg = det < 0.0f;
  T = neg ? -T : T;
  det = neg ? -det : det;
  const bool ok = !mixed && det != 0.0f && T > r.tmin * det && T < tmax * det;
  *t_out = T / det;
  return ok;
}

// ---------------------------------------------------------------------------
// traversal stack column of one lane: entry i at col[i * kBlock] (a column per
// lane of a kBlock-wide LDS array, conflict-free)
using StackCol = PV_LDS int32_t*;

struct Hit {
  float t;       // ray parameter of the closest crossing (tmax when none)
  uint32_t gid;  // its global triangle id, kHitNone when none
  uint32_t rec;  // its record in the scene's triangle array
};

// Depth-first walk of the scene hierarchy from a root (near child first), in
// resumable form for persistent kernels.  any = stop at the first crossing
// inside the ray's open interval; otherwise the closest crossing.  The state
// of one lane's query survives between calls, and a call returns as soon as
// this lane's walk is finished or fewer than 'min_active' lanes of the wave
// are still walking, so that finished lanes can take new work instead of
// idling until the longest walk of the wave ends (Aila and Laine 2009,
// dynamic ray fetch).
//
// The inner loop over internal nodes has no branch besides its exit: the far
// child is always written one slot above the top of the stack and the stack
// pointer moves by +1 (both children entered), 0 (one) or -1 (none: the top
// entry, read ahead, becomes the next node).  A sentinel at the bottom ends
// the walk.
struct Walk {
  int32_t cur;    // next node or leaf; kRootNone once the stack is exhausted
  int32_t leaf;   // a reached leaf whose test is postponed, 0 when none
  int sp;         // stack entries in use
  float tb;       // closest crossing so far (the ray's tmax initially)
  uint32_t gid;   // its global triangle id, kHitNone when none
  uint32_t rec;   // its record in the scene's triangle array
};

__device__ inline bool is_leaf(int32_t c) { return (uint32_t)c > 0x80000000u; }  // c < 0, c != kRootNone

__device__ inline bool walk_done(const Walk& w) { return w.cur == kRootNone && w.leaf == 0; }

__device__ inline void walk_start(Walk& w, int32_t root, float tmax, StackCol col) {
  col[0] = kRootNone;
  w.sp = 1;
  w.cur = root;
  w.leaf = 0;
  w.tb = tmax;
  w.gid = kHitNone;
  w.rec = 0;
}

// Speculative traversal (Aila and Laine 2009): a lane that reaches a leaf
// while holding none keeps it pending and continues with the next stack
// entry, until every lane still walking holds a leaf; then the wave tests
// leaves together.  Leaves are tested in the same depth-first order as
// without postponement and culling only uses an older (larger) closest
// distance, so the result is the same.
//
// Boxes are tested with the slab parameters (binv, boi) and triangles with
// the ray r itself: a walk through a rigid object's hierarchy in its own
// object space passes the object-space ray's parameters for the boxes, with
// the same parameter interval, while triangles stay in world space.
__device__ inline void walk_run(const PV_GLOBAL Node* __restrict__ nodes, const PV_GLOBAL Tri* __restrict__ tris,
                                const Ray& r, float3 binv, float3 boi, bool any, StackCol col, Walk& w,
                                int min_active) {
  int32_t cur = w.cur, leaf = w.leaf;
  // top: the stack's top entry (entry sp - 1); the far child goes one entry
  // above it.  Once the sentinel itself is taken top points one entry below
  // the column's first, which every launch allocates and nothing uses.
  StackCol top = col + (w.sp - 1) * kBlock;
  float tb = w.tb;
  uint32_t gid = w.gid, rec = w.rec;
  const float tmin = r.tmin;
  while (true) {
    while (cur >= 0) {
      const int32_t below = top[0];
      // node records are addressed by a 32-bit byte offset (arrays < 4 GiB)
      const Node nd = *(const PV_GLOBAL Node*)((const PV_GLOBAL char*)nodes + ((uint32_t)cur << 6));
      // slab entry and exit of both children; the query interval enters by
      // comparisons only (min/max with it would need canonical operands)
      float tx0 = fmaf(nd.a.x, binv.x, boi.x), tx1 = fmaf(nd.a.w, binv.x, boi.x);
      float ty0 = fmaf(nd.a.y, binv.y, boi.y), ty1 = fmaf(nd.b.x, binv.y, boi.y);
      float tz0 = fmaf(nd.a.z, binv.z, boi.z), tz1 = fmaf(nd.b.y, binv.z, boi.z);
      const float e0 = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fminf(tz0, tz1));
      const float x0 = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
      tx0 = fmaf(nd.b.z, binv.x, boi.x), tx1 = fmaf(nd.c.y, binv.x, boi.x);
      ty0 = fmaf(nd.b.w, binv.y, boi.y), ty1 = fmaf(nd.c.z, binv.y, boi.y);
      tz0 = fmaf(nd.c.x, binv.z, boi.z), tz1 = fmaf(nd.c.w, binv.z, boi.z);
      const float e1 = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fminf(tz0, tz1));
      const float x1 = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
      // the slab interval meets [tmin, tb]
      const bool a0 = e0 <= x0, b0 = e0 <= tb, c0 = x0 >= tmin;
      const bool a1 = e1 <= x1, b1 = e1 <= tb, c1 = x1 >= tmin;
      const bool le = e0 <= e1;
      const bool h0 = a0 && b0 && c0, h1 = a1 && b1 && c1;
      const bool near0 = h0 && (!h1 || le);  // a missed child comes last
      top[kBlock] = near0 ? nd.d.y : nd.d.x;
      const StackCol up = top + kBlock, down = top - kBlock;
      top = (h0 && h1) ? up : ((h0 || h1) ? top : down);
      cur = (h0 || h1) ? (near0 ? nd.d.x : nd.d.y) : below;
      // postpone a reached leaf and go on with the next stack entry (once the
      // sentinel itself was taken, cur is kRootNone and nothing is postponed)
      const int32_t next = top[0];
      const bool lf = is_leaf(cur), em = leaf == 0;
      const bool post = em && lf;
      leaf = post ? cur : leaf;
      cur = post ? next : cur;
      top = post ? top - kBlock : top;
      if (__ballot(leaf == 0) == 0) break;  // every lane still here holds a leaf
    }
    if (leaf == 0 && is_leaf(cur)) {
      leaf = cur;
      cur = top[0];
      top -= kBlock;
    }
    bool found = false;
    while (leaf != 0) {
      const uint32_t f = leaf_first(leaf), n = leaf_count(leaf);
      for (uint32_t i = f; i < f + n; ++i) {
        const Tri tr = tris[i];
        float t;
        const bool hit = tri_hit(r, xyz(tr.t0), xyz(tr.t1), xyz(tr.t2), tb, &t);
        tb = hit ? t : tb;
        gid = hit ? __float_as_uint(tr.t0.w) : gid;
        rec = hit ? i : rec;
        found |= hit;
      }
      // the current entry may itself be a leaf: test it next
      const bool again = is_leaf(cur) && !(found && any);
      leaf = again ? cur : 0;
      if (again) {
        cur = top[0];
        top -= kBlock;
      }
    }
    if (found && any) cur = kRootNone;
    if (cur == kRootNone) break;
    if (__popcll(__ballot(1)) < min_active) break;
  }
  w.cur = cur;
  w.leaf = leaf;
  w.sp = (int)(top - col) / kBlock + 1;
  w.tb = tb;
  w.gid = gid;
  w.rec = rec;
}

// the same walk with world-space boxes
__device__ inline void walk_run(const PV_GLOBAL Node* __restrict__ nodes, const PV_GLOBAL Tri* __restrict__ tris,
                                const Ray& r, bool any, StackCol col, Walk& w, int min_active) {
  walk_run(nodes, tris, r, r.inv, r.oi, any, col, w, min_active);
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

// ---------------------------------------------------------------------------
// Distribution maps (Section 3.1).  A light's emission is partitioned into
// cells: for a rectangle, a gu x gv grid over its local (u, v) times a grid of
// directions; for a point light, the directions only.  Directions are cut on
// the unit disk of their local (x, y) components (cosine-weighted emission is
// uniform there): 'rings' rings of equal area (equal steps of x^2 + y^2) and
// 'sectors' sectors of equal angle, so that every cell is equally likely.
// Cell index ((iu * gv + iv) * rings + ring) * sectors + sector.

__host__ __device__ inline bool dm_point(const float half[2]) { return half[0] == 0.0f && half[1] == 0.0f; }

__host__ __device__ inline uint32_t dm_cells(const float half[2], int32_t kind, const int32_t dm[4]) {
  if (kind == PV_LIGHT_CAMERA) return (uint32_t)dm[0] * (uint32_t)dm[1];  // pixel grid of the near plane
  return (uint32_t)(dm_point(half) ? 1 : dm[0] * dm[1]) * (uint32_t)dm[2] * (uint32_t)dm[3];
}

// squared radius of a light's direction disk: 1, or sin^2 of a spot's cone
__device__ inline float dm_disk2(int32_t kind, const float param[2]) {
  return kind == PV_LIGHT_SPOT ? (1.0f - param[0]) * (1.0f + param[0]) : 1.0f;
}

// DM_T: a light's paths spread evenly over its cells, the first N mod C
// cells one more
__host__ __device__ inline uint32_t dm_target(uint32_t n_paths, uint32_t cells, uint32_t c) {
  return n_paths / cells + (c < n_paths % cells ? 1u : 0u);
}

constexpr float kPiF = 3.14159265358979323846f;

// The cell of a light sample (origin x0 on the light, unit direction w), or
// -1 when the parametrisation has no value for it (origin off the rectangle,
// direction not on the emitting side).  xf: the light's 3x4 transform
// (columns eu, ev, n, centre).
__device__ inline int32_t dm_cell(const float* xf, const LightDev& lt, const int32_t dm[4], float3 x0, float3 w) {
  const float* half = lt.half;
  const float3 eu = f3(xf[0], xf[4], xf[8]), ev = f3(xf[1], xf[5], xf[9]);
  const float3 c = f3(xf[3], xf[7], xf[11]);
  float3 n = f3(xf[2], xf[6], xf[10]);
  n = mul(n, 1.0f / length(n));
  if (lt.kind == PV_LIGHT_CAMERA) {
    const float z = dot(w, n);
    if (!(z > 0.0f)) return -1;
    const float fu = (dot(w, eu) / z + lt.param[0]) / (2.0f * lt.param[0]) * (float)dm[0];
    const float fv = (dot(w, ev) / z + lt.param[1]) / (2.0f * lt.param[1]) * (float)dm[1];
    if (!(fu >= 0.0f && fu <= (float)dm[0] && fv >= 0.0f && fv <= (float)dm[1])) return -1;
    return min((int32_t)floorf(fu), dm[0] - 1) * dm[1] + min((int32_t)floorf(fv), dm[1] - 1);
  }
  const float s2 = dm_disk2(lt.kind, lt.param);
  const bool point = dm_point(half);
  const int32_t gu = point ? 1 : dm[0], gv = point ? 1 : dm[1], nr = dm[2], ns = dm[3];
  int32_t iu = 0, iv = 0;
  if (!point) {
    const float3 r = sub(x0, c);
    const float u = dot(r, eu), v = dot(r, ev);
    const float fu = (u + half[0]) / (2.0f * half[0]) * (float)gu;
    const float fv = (v + half[1]) / (2.0f * half[1]) * (float)gv;
    if (!(fu >= 0.0f && fu <= (float)gu && fv >= 0.0f && fv <= (float)gv)) return -1;
    iu = min((int32_t)floorf(fu), gu - 1);
    iv = min((int32_t)floorf(fv), gv - 1);
  }
  const float x = dot(w, eu), y = dot(w, ev), z = dot(w, n);
  if (!(z > 0.0f)) return -1;
  const float rho2 = x * x + y * y;
  const float fr = rho2 / s2 * (float)nr;
  if (lt.kind == PV_LIGHT_SPOT && !(fr <= (float)nr)) return -1;  // outside the cone
  const int32_t ring = min((int32_t)floorf(fr), nr - 1);
  const float phi = atan2f(y, x);  // [-pi, pi]
  const float fs = (phi + kPiF) / (2.0f * kPiF) * (float)ns;
  const int32_t sector = max(0, min((int32_t)floorf(fs), ns - 1));
  return ((iu * gv + iv) * nr + ring) * ns + sector;
}

// A new light sample inside cell 'cell' (Section 3.1, filling DM_C:
// sampling restricted to the cell): position uniform in the cell's part of
// the rectangle, disk point uniform in the cell's ring (in x^2 + y^2) and
// sector (in angle), lifted to the hemisphere; u: one Philox draw (tag 0).
__device__ inline void dm_sample(const float* xf, const LightDev& lt, const int32_t dm[4], uint32_t cell,
                                 const float u[4], float3* x0, float3* w) {
  const float* half = lt.half;
  const float3 eu = f3(xf[0], xf[4], xf[8]), ev = f3(xf[1], xf[5], xf[9]);
  const float3 c = f3(xf[3], xf[7], xf[11]);
  float3 n = f3(xf[2], xf[6], xf[10]);
  n = mul(n, 1.0f / length(n));
  if (lt.kind == PV_LIGHT_CAMERA) {
    // uniform in the pixel's part of the near plane
    const uint32_t iu = cell / (uint32_t)dm[1], iv = cell % (uint32_t)dm[1];
    const float x = -lt.param[0] + ((float)iu + u[0]) * (2.0f * lt.param[0] / (float)dm[0]);
    const float y = -lt.param[1] + ((float)iv + u[1]) * (2.0f * lt.param[1] / (float)dm[1]);
    *x0 = c;
    *w = mul(add(add(mul(eu, x), mul(ev, y)), n), 1.0f / sqrtf(x * x + y * y + 1.0f));
    return;
  }
  const float s2 = dm_disk2(lt.kind, lt.param);
  const bool point = dm_point(half);
  const uint32_t gu = point ? 1u : (uint32_t)dm[0], gv = point ? 1u : (uint32_t)dm[1];
  const uint32_t nr = (uint32_t)dm[2], ns = (uint32_t)dm[3];
  const uint32_t sector = cell % ns, ring = (cell / ns) % nr, pc = cell / (ns * nr);
  const uint32_t iv = pc % gv, iu = pc / gv;
  if (point) {
    *x0 = c;
  } else {
    const float a = -half[0] + ((float)iu + u[0]) * (2.0f * half[0] / (float)gu);
    const float b = -half[1] + ((float)iv + u[1]) * (2.0f * half[1] / (float)gv);
    *x0 = add(c, add(mul(eu, a), mul(ev, b)));
  }
  const float rho2 = ((float)ring + u[2]) / (float)nr * s2, rho = sqrtf(rho2);
  const float phi = -kPiF + ((float)sector + u[3]) * (2.0f * kPiF / (float)ns);
  // height over the disk point, sqrt(1 - rho^2), formed without cancellation
  // near the disk's rim: 1 - rho^2 = (1 - s2) + s2 (1 - t) for rho^2 = s2 t,
  // with 1 - t = ((nr - ring) - u) / nr and 1 - s2 the squared cone cosine
  const float om = ((float)(nr - ring) - u[2]) / (float)nr;
  const float c2 = lt.kind == PV_LIGHT_SPOT ? lt.param[0] * lt.param[0] : 0.0f;
  const float lx = rho * cosf(phi), ly = rho * sinf(phi), lz = sqrtf(fmaxf(c2 + s2 * om, 0.0f));
  *w = add(add(mul(eu, lx), mul(ev, ly)), mul(n, lz));
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
