// HIP kernels of the path-verification hot path (gfx950).
//
//   k_frame_begin   moved flags for objects / lights, transform history
//   k_update_objects  per moved object: world-space triangles (FP64 fma chain
//                   -> FP32) and level-by-level box refit of its hierarchy
//   k_verify        Section 3.1 origin update + Section 3.2 dynamic occlusions,
//                   first invalid segment, per-block replace counts
//   k_scan          exclusive scan of per-block counts (single block)
//   k_scatter_queue stable re-trace work queue (wave ballot + prefix)
//   k_mark_all      full invalidation (baseline / frame 0)
//   k_retrace       persistent re-trace over the device work queue
//   k_photon_count / k_photon_scatter   compaction of existing photons
//   k_energy_fwd / k_energy_bwd / k_reduce_partials   differentiation form
#include "pv_device.h"
#include "pv_launch.h"

namespace pv {

__device__ inline uint32_t lane_id() { return threadIdx.x & 63u; }
__device__ inline uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// block-wide sum of one value per thread (kBlock threads), result to all
__device__ inline unsigned long long block_sum_u64(unsigned long long v, unsigned long long* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long t = 0;
  for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// frame begin: one thread per (scene, object) and per (scene, light)

__global__ void k_frame_begin(SceneDev* scenes, int n_scenes, const float* const* obj_in,
                              const float* const* light_in) {
  int s = blockIdx.x;
  if (s >= n_scenes) return;
  SceneDev& S = scenes[s];
  const uint32_t first = S.state[0];
  for (uint32_t o = threadIdx.x; o < S.n_obj; o += blockDim.x) {
    const float* nw = obj_in[s] + 12 * o;
    float* cur = S.obj_xf_cur + 12 * o;
    float* prev = S.obj_xf_prev + 12 * o;
    uint32_t moved = first;
    for (int i = 0; i < 12; ++i) {
      float c = cur[i], n = nw[i];
      moved |= (__float_as_uint(c) != __float_as_uint(n)) ? 1u : 0u;
      prev[i] = c;
      cur[i] = n;
    }
    S.obj_moved[o] = moved;
  }
  for (uint32_t l = threadIdx.x; l < S.n_lights; l += blockDim.x) {
    const float* nw = light_in[s] + 12 * l;
    float* cur = S.light_xf_cur + 12 * l;
    float* prev = S.light_xf_prev + 12 * l;
    uint32_t moved = 0;  // a light's first placement does not invalidate anything
    if (!first) {
      for (int i = 0; i < 12; ++i) moved |= (__float_as_uint(cur[i]) != __float_as_uint(nw[i])) ? 1u : 0u;
    }
    for (int i = 0; i < 12; ++i) {
      prev[i] = cur[i];
      cur[i] = nw[i];
    }
    S.light_moved[l] = moved;
  }
  __syncthreads();
  if (threadIdx.x == 0) S.state[0] = 0;
}

// ---------------------------------------------------------------------------
// sparse transform update (one wave, n <= 64): row ids[i] of dst takes the 12
// floats m[i]; when an id repeats, its last entry wins; ids >= n_rows are
// skipped

__global__ __launch_bounds__(64) void k_scatter_xf(float* __restrict__ dst, uint32_t n_rows,
                                                   const uint32_t* __restrict__ ids,
                                                   const float* __restrict__ m, uint32_t n) {
  __shared__ uint32_t sid[64];
  const uint32_t i = threadIdx.x;
  const uint32_t id = i < n ? ids[i] : 0xFFFFFFFFu;
  sid[i] = id;
  __syncthreads();
  if (i >= n || id >= n_rows) return;
  for (uint32_t j = i + 1; j < n; ++j)
    if (sid[j] == id) return;
  for (int c = 0; c < 12; ++c) dst[12 * (size_t)id + c] = m[12 * (size_t)i + c];
}

hipError_t launch_scatter_xf(float* dst, uint32_t n_rows, const uint32_t* ids, const float* m, uint32_t n,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scatter_xf, dim3(1), dim3(64), 0, s, dst, n_rows, ids, m, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per moved object, one workgroup: world-space triangles (FP64 fma chain
// rounded to FP32), then the hierarchy's boxes level by level from the
// deepest internal nodes up (the topology, fixed for a rigid object, was
// built at upload), then the object's box.  No atomics: levels are separated
// by workgroup barriers.

__device__ inline float xform_coord(const float* m, int r, float x, float y, float z) {
  double v = fma((double)m[4 * r + 0], (double)x,
                 fma((double)m[4 * r + 1], (double)y, fma((double)m[4 * r + 2], (double)z, (double)m[4 * r + 3])));
  return (float)v;
}

__device__ inline float pad_lo(float x) { return x - (1e-6f + fabsf(x) * 1e-6f); }
__device__ inline float pad_hi(float x) { return x + (1e-6f + fabsf(x) * 1e-6f); }

// box (lo xyz, hi xyz) of a child: a leaf's padded triangle box, or the union
// of an internal node's two child boxes
__device__ inline void child_box(const SceneDev& S, int32_t code, float* b) {
  if (code < 0) {
    uint32_t f = leaf_first(code), c = leaf_count(code);
    float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    for (uint32_t i = f; i < f + c; ++i) {
      Tri t = S.tris[i];
      float4 vs[3] = {t.t0, t.t1, t.t2};
      for (int k = 0; k < 3; ++k) {
        lo[0] = fminf(lo[0], vs[k].x); hi[0] = fmaxf(hi[0], vs[k].x);
        lo[1] = fminf(lo[1], vs[k].y); hi[1] = fmaxf(hi[1], vs[k].y);
        lo[2] = fminf(lo[2], vs[k].z); hi[2] = fmaxf(hi[2], vs[k].z);
      }
    }
    for (int k = 0; k < 3; ++k) {
      b[k] = pad_lo(lo[k]);
      b[3 + k] = pad_hi(hi[k]);
    }
  } else {
    const Node nd = S.nodes[code];
    const float* f = reinterpret_cast<const float*>(&nd);
    for (int k = 0; k < 3; ++k) {
      b[k] = fminf(f[k], f[6 + k]);
      b[3 + k] = fmaxf(f[3 + k], f[9 + k]);
    }
  }
}

// world-space triangles of moved objects: one thread per triangle; a tile is
// (scene << 8 | object, first triangle of the object) for kBlock triangles
__global__ __launch_bounds__(kBlock) void k_transform(SceneDev* scenes, const uint2* tiles) {
  const uint2 tile = tiles[blockIdx.x];
  SceneDev& S = scenes[tile.x >> 8];
  const uint32_t o = tile.x & 0xffu;
  if (!S.obj_moved[o]) return;
  const ObjDev ob = S.objs[o];
  const uint32_t i = tile.y + threadIdx.x;
  if (i < ob.n_tris) {
    const float* m = S.obj_xf_cur + 12 * o;
    uint32_t rec = ob.tri_base + i;
    const float* v = S.dlocal + 9 * (size_t)rec;
    float w[9];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int r = 0; r < 3; ++r) w[3 * k + r] = xform_coord(m, r, v[3 * k], v[3 * k + 1], v[3 * k + 2]);
    uint32_t gid = S.dtri_gid[rec];
    Tri t;
    t.t0 = make_float4(w[0], w[1], w[2], __uint_as_float(gid));
    t.t1 = make_float4(w[3], w[4], w[5], __uint_as_float(S.tri_mat[gid]));
    t.t2 = make_float4(w[6], w[7], w[8], 0.0f);
    S.tris[S.n_static + rec] = t;
  }
}

// per moved object, one workgroup: the hierarchy's boxes level by level from
// the deepest internal nodes up, then the object's box
constexpr int kRefitBlock = 1024;  // the deepest levels of an object hold thousands of nodes

__global__ __launch_bounds__(kRefitBlock) void k_update_objects(SceneDev* scenes, const uint2* tiles) {
  uint2 tile = tiles[blockIdx.x];
  SceneDev& S = scenes[tile.x];
  const uint32_t o = tile.y;
  if (!S.obj_moved[o]) return;
  const ObjDev ob = S.objs[o];
  const uint32_t* off = S.dlevel_off + ob.lvl_base;
  for (uint32_t lv = 0; lv < ob.n_levels; ++lv) {
    const uint32_t e = off[lv + 1];
    for (uint32_t i = off[lv] + threadIdx.x; i < e; i += blockDim.x) {
      Node* nd = S.nodes + S.dlevel_nodes[i];
      int4 ch = nd->d;
      float b[12];
      child_box(S, ch.x, b);
      child_box(S, ch.y, b + 6);
      nd->a = make_float4(b[0], b[1], b[2], b[3]);
      nd->b = make_float4(b[4], b[5], b[6], b[7]);
      nd->c = make_float4(b[8], b[9], b[10], b[11]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    float b[6];
    child_box(S, ob.sah_root, b);
    for (int k = 0; k < 6; ++k) S.obj_aabb[6 * o + k] = b[k];
    const_cast<ObjDev*>(S.objs)[o].root = ob.sah_root;  // the refit topology is the current one
  }
}

// ---------------------------------------------------------------------------
// top-level trees, rebuilt each frame once the object boxes are current: one
// over the static root and every object root, one over the moved objects
// only (the set that verification and the walk's clearance tests query).
// The objects of a tree are split at their median along the widest axis of
// their box centres, recursively; the static hierarchy, whose box spans the
// scene and would widen every node above it, is the root's first child and
// the objects' tree the second (nearly every query enters the static side
// first).  One wave per tree, one lane per position of the item order, one
// level of the recursion per step: every range of the level is stably sorted
// by rank along its own axis, at once.  A range [lo, hi) splits at
// mid = (lo + hi) / 2, and each split position belongs to exactly one
// internal node, so node mid - 1 of the tree's block holds that range (node
// n - 1 the root above the static hierarchy).

constexpr int kTopLevels = kTopDepth - 1;  // median levels over <= PV_MAX_OBJECTS objects

__global__ __launch_bounds__(128) void k_build_top(SceneDev* scenes) {
  static_assert(PV_MAX_OBJECTS <= 64, "one lane per object");
  static_assert((1 << kTopLevels) >= PV_MAX_OBJECTS, "median levels");
  __shared__ float sbx[2][2][6][64];  // [tree][buffer][box component][position]
  __shared__ int32_t scode[2][2][64];
  SceneDev& S = scenes[blockIdx.x];
  const int which = threadIdx.x >> 6;  // tree of this wave
  const uint32_t lane = threadIdx.x & 63u;
  // items of the tree in object order (moved objects compacted by ballot)
  const bool have = lane < S.n_obj;
  const bool take = have && (which == 0 || S.obj_moved[lane] != 0);
  const uint64_t mm = __ballot(take);
  const uint32_t n = (uint32_t)__popcll(mm);
  if (take) {
    const uint32_t i = (uint32_t)__popcll(mm & lanemask_lt());
    for (int k = 0; k < 6; ++k) sbx[which][0][k][i] = S.obj_aabb[6 * lane + k];
    scode[which][0][i] = S.objs[lane].root;
  }
  __syncthreads();
  const uint32_t first = S.top_base + (uint32_t)which * kTopNodes;
  uint32_t lo = 0, hi = n;  // range of this lane's position
  int buf = 0;
  for (int level = 0; level < kTopLevels; ++level) {
    const float(*bx)[64] = sbx[which][buf];
    const bool live = lane < n && hi - lo >= 2;
    uint32_t dst = lane;
    if (live) {
      // widest axis of the range's box centres
      float clo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
      float chi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
      for (uint32_t q = lo; q < hi; ++q)
        for (int k = 0; k < 3; ++k) {
          const float c = 0.5f * (bx[k][q] + bx[3 + k][q]);
          clo[k] = fminf(clo[k], c);
          chi[k] = fmaxf(chi[k], c);
        }
      int ax = 0;
      for (int k = 1; k < 3; ++k)
        if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
      // stable rank along that axis
      const float mine = 0.5f * (bx[ax][lane] + bx[3 + ax][lane]);
      uint32_t rank = 0;
      for (uint32_t q = lo; q < hi; ++q) {
        const float c = 0.5f * (bx[ax][q] + bx[3 + ax][q]);
        rank += (c < mine || (c == mine && q < lane)) ? 1u : 0u;
      }
      dst = lo + rank;
    }
    float mb[6];
    for (int k = 0; k < 6; ++k) mb[k] = bx[k][lane];
    const int32_t mc = scode[which][buf][lane];
    if (lane < n) {
      for (int k = 0; k < 6; ++k) sbx[which][buf ^ 1][k][dst] = mb[k];
      scode[which][buf ^ 1][dst] = mc;
    }
    __syncthreads();
    buf ^= 1;
    if (live) {
      const uint32_t mid = (lo + hi) / 2;
      if (lane == lo) {  // one lane per range writes its node
        const float(*nb)[64] = sbx[which][buf];
        float cb[2][6];
        int32_t ch[2];
        for (int side = 0; side < 2; ++side) {
          const uint32_t a = side ? mid : lo, b = side ? hi : mid;
          for (int k = 0; k < 3; ++k) {
            cb[side][k] = __builtin_inff();
            cb[side][3 + k] = -__builtin_inff();
          }
          for (uint32_t q = a; q < b; ++q)
            for (int k = 0; k < 3; ++k) {
              cb[side][k] = fminf(cb[side][k], nb[k][q]);
              cb[side][3 + k] = fmaxf(cb[side][3 + k], nb[3 + k][q]);
            }
          ch[side] = b - a == 1 ? scode[which][buf][a] : (int32_t)(first + (a + b) / 2 - 1);
        }
        Node& nd = S.nodes[first + mid - 1];
        nd.a = make_float4(cb[0][0], cb[0][1], cb[0][2], cb[0][3]);
        nd.b = make_float4(cb[0][4], cb[0][5], cb[1][0], cb[1][1]);
        nd.c = make_float4(cb[1][2], cb[1][3], cb[1][4], cb[1][5]);
        nd.d = make_int4(ch[0], ch[1], -1, 0);
      }
      if (lane < mid) hi = mid;
      else lo = mid;
    }
  }
  if (lane != 0) return;
  // root of the objects' tree: its node, the single object, or none
  int32_t root = n == 0 ? kRootNone : (n == 1 ? scode[which][buf][0] : (int32_t)(first + n / 2 - 1));
  if (which == 0 && S.sroot != kRootNone && n > 0) {
    float ob[6] = {__builtin_inff(), __builtin_inff(), __builtin_inff(),
                   -__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    for (uint32_t q = 0; q < n; ++q)
      for (int k = 0; k < 3; ++k) {
        ob[k] = fminf(ob[k], sbx[0][buf][k][q]);
        ob[3 + k] = fmaxf(ob[3 + k], sbx[0][buf][3 + k][q]);
      }
    Node& nd = S.nodes[first + n - 1];
    nd.a = make_float4(S.sbox[0], S.sbox[1], S.sbox[2], S.sbox[3]);
    nd.b = make_float4(S.sbox[4], S.sbox[5], ob[0], ob[1]);
    nd.c = make_float4(ob[2], ob[3], ob[4], ob[5]);
    nd.d = make_int4(S.sroot, root, -1, 0);
    root = (int32_t)(first + n - 1);
  } else if (which == 0 && S.sroot != kRootNone) {
    root = S.sroot;
  }
  S.top[which] = root;
}

// ---------------------------------------------------------------------------
// verification (Sections 3.1 and 3.2)

// Moved objects of a scene in LDS: box corners with the object's global
// triangle id range in the w components (lo.w = first id, hi.w = count), and
// the same id ranges merged where consecutive moved objects' ids adjoin
// (run[k] = {first id, count}; one run when every object moves).
struct MovedSet {
  int n, nr;
  float4 lo[PV_MAX_OBJECTS], hi[PV_MAX_OBJECTS];
  uint2 run[PV_MAX_OBJECTS];
};

// the moved objects of the scene, compacted in object order by the first wave
// (at most PV_MAX_OBJECTS = 64 objects: one lane each)
__device__ inline void load_moved(const SceneDev& S, MovedSet& M) {
  static_assert(PV_MAX_OBJECTS <= 64, "one lane per object");
  if (threadIdx.x < 64) {
    const uint32_t o = threadIdx.x;
    const bool have = o < S.n_obj;
    const bool mv = have && G(S.obj_moved)[o] != 0;
    const uint64_t m = __ballot(mv);
    ObjDev ob{};
    if (have) ob = G(S.objs)[o];
    if (mv) {
      const uint32_t i = (uint32_t)__popcll(m & lanemask_lt());
      const PV_GLOBAL float* b = G(S.obj_aabb) + 6 * o;
      M.lo[i] = make_float4(b[0], b[1], b[2], __uint_as_float(ob.gbase));
      M.hi[i] = make_float4(b[3], b[4], b[5], __uint_as_float(ob.n_tris));
    }
    // runs: a moved object continues the run of the object before it when
    // that one moved too and its ids end where this one's begin
    const uint32_t end = ob.gbase + ob.n_tris;
    const uint32_t prev_end = __shfl_up(end, 1, 64);
    const bool cont = mv && o > 0 && ((m >> (o - 1)) & 1ull) && prev_end == ob.gbase;
    const bool start = mv && !cont;
    const uint64_t cm = __ballot(cont), sm = __ballot(start);
    const uint64_t after = o < 63 ? ~cm >> (o + 1) : 0ull;  // lanes past o that end a run
    const uint32_t last = o + (after ? (uint32_t)__ffsll((long long)after) - 1u : 63u - o);
    const uint32_t run_end = __shfl(end, (int)last, 64);
    if (start) M.run[__popcll(sm & lanemask_lt())] = make_uint2(ob.gbase, run_end - ob.gbase);
    if (o == 0) {
      M.n = (int)__popcll(m);
      M.nr = (int)__popcll(sm);
    }
  }
  __syncthreads();
}

// whether a stored hit id lies on a moved object (no early exit: the loop
// count is uniform over the block)
__device__ inline bool on_moved(const MovedSet& M, uint32_t hit) {
  bool mv = false;
  for (int k = 0; k < M.nr; ++k) mv |= hit - M.run[k].x < M.run[k].y;
  return mv;
}

// whether a segment's query reaches box [lo, hi] within its interval: the
// same decision as box_entry(...) != inf when tmin <= tmax, with the interval
// entering by comparisons (the slab parameters are fma results, so the
// min/max need no operand canonicalisation)
__device__ inline bool slab_hit(float4 lo, float4 hi, const Ray& r) {
  const float x0 = fmaf(lo.x, r.inv.x, r.oi.x), x1 = fmaf(hi.x, r.inv.x, r.oi.x);
  const float y0 = fmaf(lo.y, r.inv.y, r.oi.y), y1 = fmaf(hi.y, r.inv.y, r.oi.y);
  const float z0 = fmaf(lo.z, r.inv.z, r.oi.z), z1 = fmaf(hi.z, r.inv.z, r.oi.z);
  const float e = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), r.tmin));
  const float x = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), r.tmax));
  return e <= x;
}

// whether a ray reaches any moved object's box within its interval
__device__ inline bool reaches_moved_box(const MovedSet& M, const Ray& r) {
  bool h = false;
  for (int i = 0; i < M.n; ++i) {
    const float4 lo = M.lo[i], hi = M.hi[i];
    h |= box_entry(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, r, r.tmax) != __builtin_inff();
  }
  return h;
}

__device__ inline Ray segment_ray(float3 a, float3 b, float eps) {
  float3 d = sub(b, a);
  float L = length(d);
  float tmin = L > 0.0f ? eps / L : 1.0f;
  return make_ray(a, d, tmin, 1.0f - tmin);
}

// The box-test part of segment_ray, for filters only: 1/d from the hardware
// reciprocal (1 ulp) and the end tolerance shortened by 1e-5 relative.  Both
// move slab parameters by about 1e-7 of the segment or widen the tested
// interval, far inside the 1e-6 padding of every stored box, so a segment that
// crosses a triangle inside a box always reaches that box.
__device__ inline Ray segment_box_ray(float3 a, float3 b, float eps) {
  Ray r;
  const float3 d = sub(b, a);
  const float tiny = 1e-30f;
  // |d| raised to at least tiny, sign kept (the same values as a select)
  const float dx = copysignf(fmaxf(fabsf(d.x), tiny), d.x);
  const float dy = copysignf(fmaxf(fabsf(d.y), tiny), d.y);
  const float dz = copysignf(fmaxf(fabsf(d.z), tiny), d.z);
  r.inv = f3(__builtin_amdgcn_rcpf(dx), __builtin_amdgcn_rcpf(dy), __builtin_amdgcn_rcpf(dz));
  r.oi = f3(-(a.x * r.inv.x), -(a.y * r.inv.y), -(a.z * r.inv.z));
  const float L2 = dot(d, d);
  r.tmin = L2 > 0.0f ? eps * __builtin_amdgcn_rsqf(L2) * (1.0f - 1e-5f) : 1.0f;
  r.tmax = 1.0f - r.tmin;
  return r;
}

__device__ inline int light_of(const SceneDev& S, uint32_t p) {
  const PV_GLOBAL LightDev* lights = G(S.lights);
  for (uint32_t l = 0; l < S.n_lights; ++l)
    if (p - lights[l].path_base < lights[l].path_count) return (int)l;
  return -1;
}

// Section 3.1 for a rectangular area light: keep the outgoing direction and
// intersect it with the light's current plane.  A light with both half
// extents 0 is a point light: the sample becomes the light's new position and
// segment 0 is re-aimed at the first photon, which must lie on the emitting
// side farther than eps_end; *vis then asks for segment 0 to be tested
// against every triangle (the visibility the paper reads from a shadow map).
__device__ inline bool light_update(const SceneDev& S, int l, float3 x0, float3 x1, float3* out, bool* vis) {
  const PV_GLOBAL float* xf = G(S.light_xf_cur) + 12 * l;
  float3 eu = f3(xf[0], xf[4], xf[8]), ev = f3(xf[1], xf[5], xf[9]);
  float3 n = f3(xf[2], xf[6], xf[10]), c = f3(xf[3], xf[7], xf[11]);
  const PV_GLOBAL LightDev* lt = G(S.lights) + l;
  if (lt->half[0] == 0.0f && lt->half[1] == 0.0f) {
    const float3 w = sub(x1, c);
    const float z = dot(w, n);
    if (!(dot(w, w) > S.eps_end * S.eps_end) || !(z > 0.0f)) return false;
    const int32_t kind = lt->kind;
    if (kind == PV_LIGHT_SPOT) {
      // inside the cone: z / |w| >= cos of the half-angle
      if (!(z * __builtin_amdgcn_rsqf(dot(w, w) * dot(n, n)) >= lt->param[0])) return false;
    } else if (kind == PV_LIGHT_CAMERA) {
      // through the near plane: |u / z| <= tan_u, |v / z| <= tan_v (n unit length)
      const float zn = z * __builtin_amdgcn_rsqf(dot(n, n));
      if (!(fabsf(dot(w, eu)) <= lt->param[0] * zn && fabsf(dot(w, ev)) <= lt->param[1] * zn)) return false;
    }
    *out = c;
    *vis = true;
    return true;
  }
  // hardware reciprocal and reciprocal square root (about 1 ulp): the
  // decisions match the FP64 update outside its 1e-6 band, the new origin
  // within the position tolerance
  n = mul(n, __builtin_amdgcn_rsqf(dot(n, n)));
  float3 w = sub(x1, x0);
  const float l2 = dot(w, w);
  if (!(l2 > 0.0f)) return false;
  w = mul(w, __builtin_amdgcn_rsqf(l2));
  const float dn = dot(w, n);
  if (!(dn > 0.0f)) return false;
  const float sdist = dot(sub(x1, c), n) * __builtin_amdgcn_rcpf(dn);
  if (!(sdist > S.eps_end)) return false;
  float3 p = sub(x1, mul(w, sdist));
  float3 r = sub(p, c);
  float u = dot(r, eu), v = dot(r, ev);
  if (!(fabsf(u) <= lt->half[0] && fabsf(v) <= lt->half[1])) return false;
  *out = p;
  return true;
}

// The scene bases of a multi-scene launch (gbase[0..n_scenes]) copied to LDS
// by the whole block, so that the binary search of scene_of reads LDS (up to
// kLdsScenes scenes; larger batches keep reading global memory).  Ends with a
// barrier.
constexpr int kLdsScenes = 256;
__device__ inline const uint32_t* stage_gbase(const uint32_t* gbase, int n_scenes, uint32_t* sg) {
  if (n_scenes > kLdsScenes) return gbase;
  for (int i = (int)threadIdx.x; i <= n_scenes; i += (int)blockDim.x) sg[i] = gbase[i];
  __syncthreads();
  return sg;
}

// scene of a global path id: gbase[s] <= gp < gbase[s + 1]
__device__ inline uint32_t scene_of(const uint32_t* gbase, int n_scenes, uint32_t gp) {
  int lo = 0, hi = n_scenes;  // gbase[s] <= gp < gbase[s+1]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (gbase[mid] <= gp)
      lo = mid;
    else
      hi = mid;
  }
  return (uint32_t)lo;
}

// Work lists are dealt to the waves of a persistent grid dynamically, a
// refill at a time: a wave whose idle lanes want work adds their number to its
// group's counter (one device atomic per refill) and takes that many entries
// of the group's share, chunks g, g + kDealGroups, ... of kChunk entries, in
// list order.  Static shares per wave left a wave idle for 12% of a re-trace
// launch on average (the sums of ~340 path costs differ from wave to wave);
// one counter for all waves serialised the atomics on one word; with 64
// groups each counter sees a few hundred refills per launch.  The group's
// n-th entry (groups: kDealGroups, or one per wave for grids of fewer waves):
constexpr uint32_t kChunk = 64;
__device__ inline uint32_t group_entry(uint32_t g, uint32_t groups, uint32_t n) {
  return ((n / kChunk) * groups + g) * kChunk + n % kChunk;
}

constexpr uint32_t kNoEntry = 0xFFFFFFFFu;

// The entry a lane that wants work takes (kNoEntry once its group's share is
// exhausted).  Called by every lane of the wave.
__device__ inline uint32_t deal(uint32_t* __restrict__ ctrs, uint32_t wave, uint32_t count, bool want) {
  const uint64_t m = __ballot(want);
  if (!m) return kNoEntry;
  const uint32_t groups = min(kDealGroups, gridDim.x * (blockDim.x / 64));
  const uint32_t g = wave % groups;
  const uint32_t leader = (uint32_t)__ffsll((long long)m) - 1u;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(ctrs + g * kDealStride, (uint32_t)__popcll(m));
  base = __shfl(base, (int)leader, 64);
  if (!want) return kNoEntry;
  const uint32_t idx = group_entry(g, groups, base + (uint32_t)__popcll(m & lanemask_lt()));
  return idx < count ? idx : kNoEntry;
}

// the counters start at zero for a launch (cleared by a kernel that precedes
// it in the stream, so that the sequence can be captured in a graph)
__device__ inline void deal_reset(uint32_t* ctrs) {
  if (blockIdx.x == 0 && threadIdx.x < kDealGroups) ctrs[threadIdx.x * kDealStride] = 0;
}

// Verification runs as a short chain of kernels without atomics.
//  k_verify_scan (coalesced, lane per path, no traversal): origin update for
//    moved lights, the bounce rows read up front, endpoint test, and one task
//    per segment whose ray reaches a moved object's box, written into the
//    tile's own region; scanning stops at the first segment whose end photon
//    is on a moved object (that segment is invalid whatever lies before it).
//    Writes the information word as if no task were blocked (final for paths
//    without tasks) and the tile's replace count over those paths.
//  scan of the per-tile task counts, k_verify_gather: one compact task list.
//  k_verify_trace: the tasks as independent any-hit queries against the
//    moved objects, every lane busy; a blocked segment lowers its path's
//    first invalid segment (atomic minimum on that path's own word).
//  k_verify_finish: information words of the paths with tasks, whose replace
//    bits it adds to their tiles' counts (the work queue's block counts).
// The result equals the in-order test of Section 3.2: the first invalid
// segment is the minimum over blocked segments and the first moved endpoint.

constexpr int kPreRows = 8;  // bounce rows a lane loads before testing
// task segment field of a point light's visibility test of segment 0 (real
// segments are 0..14)
constexpr uint32_t kVisTask = 15;
static_assert(PV_MAX_BOUNCES <= 15, "segment indices below kVisTask");

__global__ __launch_bounds__(kBlock) void k_verify_scan(const SceneDev* __restrict__ scenes,
                                                        const uint2* __restrict__ tiles, VerifyWork W,
                                                        uint32_t* __restrict__ block_cnt, pv_stats* stats) {
  __shared__ MovedSet M;
  __shared__ unsigned long long sred[kBlock / 64];
  __shared__ uint32_t swt[kBlock / 64];
  uint2 tile = tiles[blockIdx.x];
  const SceneDev& S = scenes[tile.x];
  load_moved(S, M);
  const uint32_t tid = threadIdx.x;
  const uint32_t p = tile.y + tid;
  const bool active = p < S.n_paths;
  const size_t stride = S.stride;
  uint32_t n = 0, cell = 0, cap = 0, mask = 0, lost = 0;
  bool vis = false;  // a point light moved: segment 0 against every triangle
  if (active) {
    const PV_GLOBAL float4* pos = G(S.pos);
    PV_GLOBAL float* org = G(S.origin);
    uint32_t w = G(S.info)[p];
    n = min(info_nseg(w), S.B);
    cell = info_cell(w);
    cap = n;
    // the path's rows (up to kPreRows) are all requested before the first
    // is used, so their loads are in flight together
    float4 rows[kPreRows];
    const uint32_t nload = M.n > 0 ? n : min(n, 1u);  // the light update needs the first hit only
#pragma unroll
    for (int j = 0; j < kPreRows; ++j) {
      rows[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if ((uint32_t)j < nload) rows[j] = pos[(size_t)j * stride + p];
    }
    float3 a = f3(org[p], org[stride + p], org[2 * stride + p]);
    int l = light_of(S, p);
    if (l >= 0 && G(S.light_moved)[l]) {
      float3 na;
      if (n > 0 && light_update(S, l, a, xyz(rows[0]), &na, &vis)) {
        a = na;
        org[p] = na.x;
        org[stride + p] = na.y;
        org[2 * stride + p] = na.z;
      } else {
        lost = 1;
        cap = 0;
      }
    }
    if (!lost && M.n > 0) {
      // every segment of the path is tested (no early exit); the first
      // segment whose end photon lies on a moved object caps the scan.  The
      // loaded rows' segments are set up first, then each moved box is read
      // once and tested against all of them (rows past n are masked off).
      // Rows are tested up to the scene's bounce limit (uniform), not the
      // path's own count, so that no lane-dependent branch splits the loop.
      // Box hits are collected as wave masks (one per row, scalar registers).
      Ray rs[kPreRows];
      uint64_t hit[kPreRows];
      uint32_t mv = 0;
#pragma unroll
      for (int j = 0; j < kPreRows; ++j) {
        hit[j] = 0;
        if ((uint32_t)j < S.B) {
          const float3 b = xyz(rows[j]);
          rs[j] = segment_box_ray(a, b, S.eps_end);
          if (!(rs[j].tmin <= rs[j].tmax)) rs[j].tmin = __builtin_inff();  // nothing to test
          rs[j].tmin = __builtin_canonicalizef(rs[j].tmin);
          rs[j].tmax = __builtin_canonicalizef(rs[j].tmax);
          if (on_moved(M, __float_as_uint(rows[j].w))) mv |= 1u << j;
          a = b;
        }
      }
      for (int i = 0; i < M.n; ++i) {
        const float4 lo = M.lo[i], hi = M.hi[i];
#pragma unroll
        for (int j = 0; j < kPreRows; ++j)
          if ((uint32_t)j < S.B) hit[j] |= __builtin_amdgcn_ballot_w64(slab_hit(lo, hi, rs[j]));
      }
#pragma unroll
      for (int j = 0; j < kPreRows; ++j) mask |= (uint32_t)((hit[j] >> lane_id()) & 1ull) << j;
      uint32_t first_mv = min(n, mv ? (uint32_t)__ffs(mv) - 1u : n);
      for (uint32_t j = kPreRows; j < n; ++j) {
        const float4 row = pos[(size_t)j * stride + p];
        const float3 b = xyz(row);
        if (on_moved(M, __float_as_uint(row.w))) first_mv = min(first_mv, j);
        if (reaches_moved_box(M, segment_box_ray(a, b, S.eps_end))) mask |= 1u << j;
        a = b;
      }
      if (S.verify_boxes) {
        // Section 3.2's own test: the first segment that reaches a moved
        // box is invalid, no triangle is tested (rows past n masked off)
        mask &= (1u << n) - 1u;
        cap = min(first_mv, mask ? (uint32_t)__ffs(mask) - 1u : n);
        mask = 0;
      } else {
        cap = first_mv;
        mask &= (1u << cap) - 1u;
      }
    }
    // the visibility task (segment index kVisTask) replaces segment 0's own
    // test, which it covers; none when segment 0 is already invalid
    if (vis && cap > 0) mask = (mask & ~1u) | (1u << kVisTask);
  }
  // ---- tasks into the tile's region, in lane order
  const uint32_t nt = (uint32_t)__popc(mask);
  uint32_t x = nt;  // inclusive wave prefix of the task counts
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if ((int)lane_id() >= o) x += y;
  }
  const uint32_t wave = tid >> 6;
  if (lane_id() == 63) swt[wave] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (uint32_t w = 0; w < kBlock / 64; ++w) {
    before += w < wave ? swt[w] : 0u;
    all += swt[w];
  }
  if (tid == 0) W.tcount[blockIdx.x] = all;
  if (nt > 0) {
    const uint32_t gp = S.gpath_base + p;
    W.first[gp] = cap;
    PV_GLOBAL uint32_t* region =
        G(W.tmp) + S.task_base + (size_t)(blockIdx.x - S.tile_base) * kBlock * S.B;
    uint32_t t = before + x - nt;
    for (uint32_t m = mask; m; m &= m - 1) region[t++] = (gp << 4) | (uint32_t)(__ffs(m) - 1);
  }
  // ---- information word as if no task were blocked
  uint32_t ex = 0, inv = 0;
  if (active) {
    uint32_t out;
    if (lost) {
      out = info_pack(cell, n, 0, 1, 0);
    } else if (cap < n) {
      out = info_pack(cell, n, cap, 1, 1);
      ex = cap + 1;
    } else {
      out = info_pack(cell, n, 0, 0, 0);
      ex = n;
    }
    G(S.info)[p] = out;
    inv = info_replace(out);
    if (nt > 0) ex = inv = 0;  // counted by k_verify_finish
  }
  {
    // per-block counts go to their own slots and are summed by
    // k_verify_stats: one counter word shared by every block would serialise
    // thousands of atomics.  Each count is at most kBlock * 15 < 2^16 per
    // block, so the four travel as 16-bit fields of one sum.  The replace
    // count of the tile is one of them.
    static_assert(kBlock * 15 < (1 << 16), "16-bit fields");
    const unsigned long long packed = (unsigned long long)ex | ((unsigned long long)inv << 16) |
                                      ((unsigned long long)lost << 32) | ((unsigned long long)nt << 48);
    const unsigned long long sum = block_sum_u64(packed, sred);
    if (tid == 0) block_cnt[blockIdx.x] = (uint32_t)((sum >> 16) & 0xffffu);
    if (stats && tid == 0) {
      uint32_t* o = W.part + 4 * (size_t)blockIdx.x;
      o[0] = (uint32_t)(sum & 0xffffu);
      o[1] = (uint32_t)((sum >> 16) & 0xffffu);
      o[2] = (uint32_t)((sum >> 32) & 0xffffu);
      o[3] = (uint32_t)(sum >> 48);
    }
  }
}

// one block per path tile: its tasks to their place in the compacted list
__global__ __launch_bounds__(kBlock) void k_verify_gather(const SceneDev* __restrict__ scenes,
                                                          const uint2* __restrict__ tiles, VerifyWork W) {
  const SceneDev& S = scenes[tiles[blockIdx.x].x];
  const uint32_t n = W.tcount[blockIdx.x];
  const PV_GLOBAL uint32_t* src = G(W.tmp) + S.task_base + (size_t)(blockIdx.x - S.tile_base) * kBlock * S.B;
  PV_GLOBAL uint32_t* dst = G(W.tasks) + W.toff[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < n; i += kBlock) dst[i] = src[i];
  deal_reset(W.deal);
}

// Persistent: a lane whose walk has finished takes the wave's next task
// (dealt by deal()) while the other lanes continue.

template <bool kSingle>
__global__ __launch_bounds__(kBlock) void k_verify_trace(const SceneDev* __restrict__ scenes,
                                                         const uint32_t* __restrict__ gbase, int n_scenes,
                                                         VerifyWork W, int min_active) {
  extern __shared__ int32_t sstack[];  // traversal stacks, launch-time size
  __shared__ MovedSet M;                // single scene: the moved objects' boxes
  __shared__ int32_t mroot[PV_MAX_OBJECTS];  // and their hierarchies' roots
  // their upload-time topologies with object-space boxes (kRootNone: walk in
  // world space) and the inverse of their current transforms (rows of the
  // inverse 3x3, then the translation)
  __shared__ int32_t moroot[PV_MAX_OBJECTS];
  __shared__ float minv[PV_MAX_OBJECTS][12];
  const StackCol col = (StackCol)(sstack + kBlock + threadIdx.x);  // entry 0 of the column; entry -1 spare
  if (kSingle) {
    if (threadIdx.x < 64) {
      const SceneDev& S0 = scenes[0];
      const uint32_t o = threadIdx.x;
      const bool mv = o < S0.n_obj && G(S0.obj_moved)[o] != 0;
      const uint64_t mm = __ballot(mv);
      if (mv) {
        const uint32_t i = (uint32_t)__popcll(mm & lanemask_lt());
        const ObjDev ob = G(S0.objs)[o];
        mroot[i] = ob.root;
        // inverse of the 3x3 part by cofactors in FP64
        const PV_GLOBAL float* x = G(S0.obj_xf_cur) + 12 * o;
        const double m0 = x[0], m1 = x[1], m2 = x[2], m4 = x[4], m5 = x[5], m6 = x[6];
        const double m8 = x[8], m9 = x[9], m10 = x[10];
        const double c00 = m5 * m10 - m6 * m9, c01 = m2 * m9 - m1 * m10, c02 = m1 * m6 - m2 * m5;
        const double det = m0 * c00 + m4 * c01 + m8 * c02;
        const bool ok = fabs(det) > 1e-12 && isfinite(det);
        const double id = ok ? 1.0 / det : 0.0;
        minv[i][0] = (float)(c00 * id);
        minv[i][1] = (float)(c01 * id);
        minv[i][2] = (float)(c02 * id);
        minv[i][3] = (float)((m6 * m8 - m4 * m10) * id);
        minv[i][4] = (float)((m0 * m10 - m2 * m8) * id);
        minv[i][5] = (float)((m2 * m4 - m0 * m6) * id);
        minv[i][6] = (float)((m4 * m9 - m5 * m8) * id);
        minv[i][7] = (float)((m1 * m8 - m0 * m9) * id);
        minv[i][8] = (float)((m0 * m5 - m1 * m4) * id);
        minv[i][9] = x[3];
        minv[i][10] = x[7];
        minv[i][11] = x[11];
        moroot[i] = ok ? ob.oroot : kRootNone;
      }
    }
    load_moved(scenes[0], M);  // ends with a barrier
  }
  __shared__ uint32_t sgb[kSingle ? 1 : kLdsScenes + 1];
  if (!kSingle) gbase = stage_gbase(gbase, n_scenes, sgb);
  const uint32_t total = *W.total;
  const uint32_t wave = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  Walk w;
  w.cur = kRootNone;
  w.leaf = 0;
  Ray r;
  float3 binv = f3(0.0f, 0.0f, 0.0f), boi = binv;  // slab parameters of the walk's boxes
  uint32_t gp = 0, j = 0;
  bool busy = false, drained = false;
  const SceneDev* S = scenes;
  while (true) {
    // lanes without a task take the next ones; a task whose path already
    // failed at an earlier segment is dropped (the minimum only decreases)
    const bool want = !busy && !drained;
    if (__ballot(want)) {
      const uint32_t t = deal(W.deal, wave, total, want);
      if (want) {
        if (t == kNoEntry) {
          drained = true;
        } else {
          const uint32_t tk = G(W.tasks)[t];
          gp = tk >> 4;
          j = tk & 15u;
          const bool vis = j == kVisTask;  // segment 0 against the whole scene
          if (vis) j = 0;
          if (j < __hip_atomic_load(&W.first[gp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            S = scenes + (kSingle ? 0u : scene_of(gbase, n_scenes, gp));
            const uint32_t q = gp - S->gpath_base;
            const size_t stride = S->stride;
            const PV_GLOBAL float* org = G(S->origin);
            const float3 a = j == 0 ? f3(org[q], org[stride + q], org[2 * stride + q])
                                    : xyz(G(S->pos)[(size_t)(j - 1) * stride + q]);
            const float3 b = xyz(G(S->pos)[(size_t)j * stride + q]);
            r = segment_ray(a, b, S->eps_end);
            binv = r.inv;
            boi = r.oi;
            int32_t root = G(S->top)[1];
            if (kSingle && !vis) {
              // the objects whose boxes the segment reaches, from LDS: one
              // object is walked from its own root (its box is the only one
              // of the moved-object tree the ray enters); several, through
              // the moved-object tree; none, not at all
              uint32_t nh = 0;
              int only = 0;
              for (int i = 0; i < M.n; ++i) {
                const float4 lo = M.lo[i], hi = M.hi[i];
                const bool h = box_entry(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, r, r.tmax) != __builtin_inff();
                nh += h ? 1u : 0u;
                only = h ? i : only;
              }
              root = nh == 0 ? kRootNone : (nh == 1 ? mroot[only] : root);
              if (nh == 1 && moroot[only] != kRootNone) {
                // a rigid object is walked in its own space: the segment
                // mapped by the inverse transform (same parameter interval)
                // meets the fixed object-space boxes, which are tighter than
                // the world boxes of the rotated nodes; triangles are still
                // tested in world space
                const float* mi = minv[only];
                const float3 ta = sub(a, f3(mi[9], mi[10], mi[11])), tb = sub(b, f3(mi[9], mi[10], mi[11]));
                const float3 oa = f3(mi[0] * ta.x + mi[1] * ta.y + mi[2] * ta.z,
                                     mi[3] * ta.x + mi[4] * ta.y + mi[5] * ta.z,
                                     mi[6] * ta.x + mi[7] * ta.y + mi[8] * ta.z);
                const float3 ob = f3(mi[0] * tb.x + mi[1] * tb.y + mi[2] * tb.z,
                                     mi[3] * tb.x + mi[4] * tb.y + mi[5] * tb.z,
                                     mi[6] * tb.x + mi[7] * tb.y + mi[8] * tb.z);
                const float3 od = sub(ob, oa);
                const float tiny = 1e-30f;
                const float dx = copysignf(fmaxf(fabsf(od.x), tiny), od.x);
                const float dy = copysignf(fmaxf(fabsf(od.y), tiny), od.y);
                const float dz = copysignf(fmaxf(fabsf(od.z), tiny), od.z);
                binv = f3(__builtin_amdgcn_rcpf(dx), __builtin_amdgcn_rcpf(dy), __builtin_amdgcn_rcpf(dz));
                boi = f3(-(oa.x * binv.x), -(oa.y * binv.y), -(oa.z * binv.z));
                root = moroot[only];
              }
            }
            if (vis) root = G(S->top)[0];
            walk_start(w, root, r.tmax, col);
            busy = root != kRootNone;
          }
        }
      }
    }
    if (__ballot(busy) == 0) {
      if (__ballot(!drained) == 0) break;
      continue;
    }
    if (busy) {
      walk_run(G(S->nodes), G(S->tris), r, binv, boi, true, col, w, min_active);
      if (walk_done(w)) {
        if (w.gid != kHitNone) atomicMin(&W.first[gp], j);
        busy = false;
      }
    }
  }
}

// The tasks of a path are adjacent in the list: the thread holding a path's
// first task writes its information word.
// The replace bits are added to the tiles' counts with one atomic per tile a
// wave's lanes reach (a wave's tasks belong to one or two tiles of paths).
template <bool kSingle>
__global__ __launch_bounds__(kBlock) void k_verify_finish(const SceneDev* __restrict__ scenes,
                                                          const uint32_t* __restrict__ gbase, int n_scenes,
                                                          VerifyWork W, uint32_t* __restrict__ block_cnt,
                                                          uint32_t n_scan_blocks, pv_stats* stats) {
  __shared__ unsigned long long sred[kBlock / 64];
  __shared__ uint32_t sgb[kSingle ? 1 : kLdsScenes + 1];
  if (!kSingle) gbase = stage_gbase(gbase, n_scenes, sgb);
  const uint32_t total = *W.total;
  uint32_t ex = 0, inv = 0;
  // the lanes of a wave hold consecutive tasks: they stay in step and leave
  // the loop together except in its last round
  for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < total; t += gridDim.x * kBlock) {
    const uint32_t gp = G(W.tasks)[t] >> 4;
    uint32_t tile = kNoEntry;  // the tile whose count this lane raises
    if (!(t > 0 && (G(W.tasks)[t - 1] >> 4) == gp)) {
      uint32_t s = 0;
      if (!kSingle) s = scene_of(gbase, n_scenes, gp);
      const SceneDev& S = scenes[s];
      const uint32_t q = gp - S.gpath_base;
      const uint32_t w = G(S.info)[q];  // as written by the scan
      const uint32_t n = info_nseg(w), k = G(W.first)[gp];
      if (k < n) {
        G(S.info)[q] = info_pack(info_cell(w), n, k, 1, 1);
        ex += k + 1;
        inv += 1;
        tile = S.tile_base + q / kBlock;
      } else {
        ex += n;
      }
    }
    while (true) {
      const uint64_t m = __ballot(tile != kNoEntry);
      if (!m) break;
      const int leader = __ffsll((long long)m) - 1;
      const uint32_t lt = __shfl(tile, leader, 64);
      const uint64_t same = __ballot(tile == lt);
      if ((int)lane_id() == leader) atomicAdd(block_cnt + lt, (uint32_t)__popcll(same));
      if (tile == lt) tile = kNoEntry;
    }
  }
  if (stats) {
    // both counts of a block fit 32 bits (at most 15 and 1 per path): one sum
    const unsigned long long sum = block_sum_u64((unsigned long long)ex | ((unsigned long long)inv << 32), sred);
    if (threadIdx.x == 0) {
      uint32_t* o = W.part + 4 * (size_t)n_scan_blocks + 2 * (size_t)blockIdx.x;
      o[0] = (uint32_t)(sum & 0xffffffffull);
      o[1] = (uint32_t)(sum >> 32);
    }
  }
}

// sum of the per-block statistics of one verification call into pv_stats
// (a few blocks, each adding its part with one atomic per counter)
__global__ __launch_bounds__(1024) void k_verify_stats(const uint32_t* __restrict__ part, uint32_t n_scan,
                                                       uint32_t n_fin, pv_stats* stats) {
  __shared__ unsigned long long sh[4][1024 / 64];
  unsigned long long a[4] = {0, 0, 0, 0};
  const uint4* __restrict__ p4 = reinterpret_cast<const uint4*>(part);  // one record per scan block
  const uint32_t step = gridDim.x * blockDim.x;
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_scan; b += step) {
    const uint4 r = p4[b];
    a[0] += r.x;
    a[1] += r.y;
    a[2] += r.z;
    a[3] += r.w;
  }
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_fin; b += step)
    for (int k = 0; k < 2; ++k) a[k] += part[4 * (size_t)n_scan + 2 * (size_t)b + k];
  for (int k = 0; k < 4; ++k) {
    for (int o = 32; o > 0; o >>= 1) a[k] += __shfl_down(a[k], o, 64);
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = a[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k)
      for (uint32_t w = 0; w < blockDim.x / 64; ++w) t[k] += sh[k][w];
    atomicAdd(&stats->segments_examined, t[0]);
    atomicAdd(&stats->paths_invalid, t[1]);
    atomicAdd(&stats->paths_light_lost, t[2]);
    atomicAdd(&stats->verify_box_hits, t[3]);
  }
}

// ---------------------------------------------------------------------------
// exclusive scan of n counts by one block of 1024 threads; total -> *total

__global__ __launch_bounds__(1024) void k_scan(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, uint32_t n,
                                               uint32_t* total) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t carry_sh;
  if (threadIdx.x == 0) carry_sh = 0;
  __syncthreads();
  for (uint32_t base = 0; base < n; base += 1024) {
    uint32_t i = base + threadIdx.x;
    uint32_t v = i < n ? in[i] : 0u;
    // inclusive wave scan
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t y = __shfl_up(x, o, 64);
      if ((int)lane_id() >= o) x += y;
    }
    if (lane_id() == 63) wsum[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x < 16) {
      uint32_t s = wsum[threadIdx.x];
      for (int o = 1; o < 16; o <<= 1) {
        uint32_t y = __shfl_up(s, o, 64);
        if ((int)threadIdx.x >= o) s += y;
      }
      wsum[threadIdx.x] = s;  // inclusive over waves
    }
    __syncthreads();
    uint32_t wpre = (threadIdx.x >> 6) ? wsum[(threadIdx.x >> 6) - 1] : 0u;
    uint32_t carry = carry_sh;
    if (i < n) out[i] = carry + wpre + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry_sh = carry + wsum[15];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *total = carry_sh;
  }
}

// Exclusive scan of count arrays: each block scans a tile of kScanTile
// entries, kScanPer rows of 1024 read and written coalesced (row k of the tile
// is entries k * 1024 .. k * 1024 + 1023).  Every row is scanned within its
// waves, then one pass over the (row, wave) totals in entry order gives each
// wave its offset.  One tile (the per-tile counts of a few million paths) is
// the whole scan in one launch; longer arrays add k_scan over the tile totals
// and k_scan_add.
constexpr uint32_t kScanPer = 16;
constexpr uint32_t kScanTile = 1024 * kScanPer;

__global__ __launch_bounds__(1024) void k_scan_tiles(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                     uint32_t n, uint32_t* __restrict__ tile_sums) {
  static_assert(kScanPer * 16 == 256, "four waves scan the (row, wave) totals");
  __shared__ uint32_t part[kScanPer * 16];  // (row, wave) totals, then their exclusive offsets
  __shared__ uint32_t qsum[4];
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
  const uint32_t base = blockIdx.x * kScanTile + tid;
  uint32_t v[kScanPer], x[kScanPer];
#pragma unroll
  for (uint32_t k = 0; k < kScanPer; ++k) {
    const uint32_t i = base + k * 1024;
    v[k] = i < n ? in[i] : 0u;
    x[k] = v[k];
  }
  for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; ++k) {
      const uint32_t y = __shfl_up(x[k], o, 64);
      if ((int)lane >= o) x[k] += y;
    }
  }
  if (lane == 63) {
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; ++k) part[k * 16 + wave] = x[k];
  }
  __syncthreads();
  uint32_t a = 0, q = 0;
  if (tid < 256) {
    a = part[tid];
    q = a;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(q, o, 64);
      if ((int)lane >= o) q += y;
    }
    if (lane == 63) qsum[wave] = q;
  }
  __syncthreads();
  if (tid < 256) {
    uint32_t pre = 0;
    for (uint32_t w = 0; w < wave; ++w) pre += qsum[w];
    part[tid] = pre + q - a;
  }
  if (tid == 0) tile_sums[blockIdx.x] = qsum[0] + qsum[1] + qsum[2] + qsum[3];
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < kScanPer; ++k) {
    const uint32_t i = base + k * 1024;
    if (i < n) out[i] = part[k * 16 + wave] + x[k] - v[k];
  }
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t* __restrict__ out, uint32_t n,
                                                  const uint32_t* __restrict__ tile_off) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_off[i / kScanTile];
}

// stable queue: ascending global path ids with the replace bit
__global__ __launch_bounds__(kBlock) void k_scatter_queue(const SceneDev* __restrict__ scenes, const uint2* __restrict__ tiles,
                                                          const uint32_t* __restrict__ offsets, uint32_t* __restrict__ queue) {
  __shared__ uint32_t wcnt[kBlock / 64];
  uint2 tile = tiles[blockIdx.x];
  const SceneDev& S = scenes[tile.x];
  uint32_t p = tile.y + threadIdx.x;
  bool flag = p < S.n_paths && info_replace(S.info[p]);
  uint64_t bal = __ballot(flag);
  if (lane_id() == 0) wcnt[threadIdx.x >> 6] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t pre = 0;
  for (uint32_t w = 0; w < (threadIdx.x >> 6); ++w) pre += wcnt[w];
  if (flag) queue[offsets[blockIdx.x] + pre + (uint32_t)__popcll(bal & lanemask_lt())] = S.gpath_base + p;
}

// full invalidation: every path replace=1, start=0, reuse_light=0; queue = all
__global__ __launch_bounds__(kBlock) void k_mark_all(const SceneDev* __restrict__ scenes, const uint2* __restrict__ tiles,
                                                     uint32_t* __restrict__ block_cnt) {
  __shared__ unsigned long long sred[kBlock / 64];
  uint2 tile = tiles[blockIdx.x];
  const SceneDev& S = scenes[tile.x];
  uint32_t p = tile.y + threadIdx.x;
  uint32_t f = 0;
  if (p < S.n_paths) {
    uint32_t w = S.info[p];
    S.info[p] = info_pack(info_cell(w), info_nseg(w), 0, 1, 0);
    f = 1;
  }
  unsigned long long c = block_sum_u64(f, sred);
  if (threadIdx.x == 0) block_cnt[blockIdx.x] = (uint32_t)c;
}

// ---------------------------------------------------------------------------
// re-tracing (Section 3.2 naive, Section 3.3 / Algorithm 1 error-based)

constexpr float kTFar = 16.0f;

__device__ inline float3 hit_normal(const SceneDev& S, const Hit& h) {
  Tri t = G(S.tris)[h.rec];
  float3 v0 = xyz(t.t0), v1 = xyz(t.t1), v2 = xyz(t.t2);
  float3 n = cross(sub(v1, v0), sub(v2, v0));
  return mul(n, 1.0f / length(n));
}

__device__ inline uint32_t hit_material(const SceneDev& S, const Hit& h) {
  return __float_as_uint(G(S.tris)[h.rec].t1.w);
}

__device__ inline float3 vertex(const SceneDev& S, uint32_t p, uint32_t j) {
  const size_t stride = S.stride;
  const PV_GLOBAL float* org = G(S.origin);
  if (j == 0) return f3(org[p], org[stride + p], org[2 * stride + p]);
  return xyz(G(S.pos)[(size_t)(j - 1) * stride + p]);
}

__device__ inline uint32_t vertex_hit(const SceneDev& S, uint32_t p, uint32_t j) {
  return __float_as_uint(G(S.pos)[(size_t)(j - 1) * S.stride + p].w);
}

__device__ inline float3 energy_row(const SceneDev& S, uint32_t p, uint32_t row) {
  return xyz(G(S.energy)[(size_t)row * S.stride + p]);
}

__device__ inline void put_photon(const SceneDev& S, uint32_t p, uint32_t row, float3 x, uint32_t gid, float3 e) {
  size_t i = (size_t)row * S.stride + p;
  G(S.pos)[i] = make_float4(x.x, x.y, x.z, __uint_as_float(gid));
  G(S.energy)[i] = make_float4(e.x, e.y, e.z, S.radius);
}

// material of a stored hit id (ids beyond the scene map to material 0)
__device__ inline uint32_t mat_of(const SceneDev& S, uint32_t hit) {
  return hit < S.n_tris_total ? G(S.tri_mat)[hit] : 0u;
}

__device__ inline float3 reflect_energy(const SceneDev& S, float3 e, uint32_t mat) {
  const PV_GLOBAL float* rho = G(S.albedo) + 3 * mat;
  return f3(__fmul_rn(e.x, rho[0]), __fmul_rn(e.y, rho[1]), __fmul_rn(e.z, rho[2]));
}

__device__ inline bool eq2(float3 en, float3 eo, float T) {
  float d0 = __fsub_rn(en.x, eo.x), d1 = __fsub_rn(en.y, eo.y), d2 = __fsub_rn(en.z, eo.z);
  float t0 = __fmul_rn(T, eo.x), t1 = __fmul_rn(T, eo.y), t2 = __fmul_rn(T, eo.z);
  return (-t0 <= d0 && d0 <= t0) && (-t1 <= d1 && d1 <= t1) && (-t2 <= d2 && d2 <= t2);
}

__device__ inline bool on_moved_obj(const SceneDev& S, uint32_t hit) {
  if (hit == kHitNone || hit < S.n_static) return false;
  for (uint32_t o = 0; o < S.n_obj; ++o) {
    const ObjDev ob = G(S.objs)[o];
    if (hit - ob.gbase < ob.n_tris) return G(S.obj_moved)[o] != 0;
  }
  return false;
}

// Object id ranges, moved flags and light path ranges of the scene of a
// single-scene launch, staged in LDS once per workgroup for the state
// machine's lookups.
struct SceneTab {
  uint32_t obj_lo[PV_MAX_OBJECTS], obj_n[PV_MAX_OBJECTS], obj_mv[PV_MAX_OBJECTS];
  uint32_t light_base[PV_MAX_LIGHTS], light_n[PV_MAX_LIGHTS];
  uint32_t n_obj, n_lights;
};

__device__ inline void load_tab(const SceneDev& S, SceneTab& T) {
  const uint32_t i = threadIdx.x;
  if (i < S.n_obj) {
    const ObjDev ob = G(S.objs)[i];
    T.obj_lo[i] = ob.gbase;
    T.obj_n[i] = ob.n_tris;
    T.obj_mv[i] = G(S.obj_moved)[i];
  }
  if (i < S.n_lights) {
    T.light_base[i] = G(S.lights)[i].path_base;
    T.light_n[i] = G(S.lights)[i].path_count;
  }
  if (i == 0) {
    T.n_obj = S.n_obj;
    T.n_lights = S.n_lights;
  }
  __syncthreads();
}

__device__ inline bool on_moved_obj(const PV_LDS SceneTab& T, uint32_t hit) {
  bool mv = false;  // no early exit: the loop count is uniform
  for (uint32_t o = 0; o < T.n_obj; ++o) mv |= (hit - T.obj_lo[o] < T.obj_n[o]) && T.obj_mv[o] != 0;
  return mv;  // kHitNone and static ids lie in no object range
}

__device__ inline int light_of(const PV_LDS SceneTab& T, uint32_t p) {
  int l = -1;
  for (uint32_t i = 0; i < T.n_lights; ++i) l = (p - T.light_base[i] < T.light_n[i]) ? (int)i : l;
  return l;
}

__device__ inline void clear_rows(const SceneDev& S, uint32_t p, uint32_t from) {
  for (uint32_t r = from; r < S.B; ++r) {
    size_t i = (size_t)r * S.stride + p;
    G(S.pos)[i] = make_float4(0.0f, 0.0f, 0.0f, __uint_as_float(kHitNone));
    G(S.energy)[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
}

__device__ inline float3 normalize3(float3 v) { return mul(v, 1.0f / length(v)); }


// Re-trace state machine: every iteration each busy lane issues exactly one
// query (closest hit over the scene, or any hit against the moved objects),
// then advances its path; lanes whose path is finished take the next path of
// the work queue (persistent while-while scheme, Aila & Laine 2009).
enum : uint32_t {
  ST_IDLE = 0,   // needs a path
  ST_FIRST,      // trace segment k from x (direction w), naive continuation
  ST_TAIL,       // sample a bounce from photon 'row' and trace it
  ST_WCHECK,     // walk: is segment j (origin unchanged) still valid?
  ST_WTRACE,     // walk: trace segment j
  ST_WSKIP,      // walk: accepted close re-hit; is segment j+1 clear?
  ST_END         // queue exhausted
};

struct Lane {
  const SceneDev* S;
  uint32_t p, mode, n, k, cell, j, newn, row, mat, hgid;
  int l;
  float3 x, w, ntri, e, hp;
};

__device__ inline void finish(Lane& L) {
  clear_rows(*L.S, L.p, L.newn);
  G(L.S->info)[L.p] = info_pack(L.cell, L.newn, 0, 0, 0);
  L.mode = ST_IDLE;
}

// after writing photon 'row' (position x, triangle normal, material, energy):
// continue sampling or finish
__device__ inline void to_tail(Lane& L) {
  if (L.row + 1 < L.S->B) {
    L.mode = ST_TAIL;
  } else {
    L.newn = L.row + 1;
    finish(L);
  }
}

__device__ inline void start_path(Lane& L, float T, uint64_t seed, uint32_t frame, const PV_LDS SceneTab* tab) {
  const SceneDev& S = *L.S;
  uint32_t w = G(S.info)[L.p];
  L.n = min(info_nseg(w), S.B);
  L.k = info_start(w);
  L.cell = info_cell(w);
  L.l = tab ? light_of(*tab, L.p) : light_of(S, L.p);
  bool reuse = info_reuse(w) != 0;
  if (!info_replace(w) || L.l < 0) {
    L.mode = ST_IDLE;
    return;
  }
  if (L.k >= L.n) {
    L.k = 0;
    reuse = false;
  }
  if (L.k == 0 && !reuse) {
    // new light sample: position uniform on the rectangle, direction
    // cosine-weighted about the light normal (one Philox draw, tag 0)
    const PV_GLOBAL float* xf = G(S.light_xf_cur) + 12 * L.l;
    const PV_GLOBAL LightDev* lt = G(S.lights) + L.l;
    float3 eu = f3(xf[0], xf[4], xf[8]), ev = f3(xf[1], xf[5], xf[9]);
    float3 nl = normalize3(f3(xf[2], xf[6], xf[10])), c = f3(xf[3], xf[7], xf[11]);
    float u[4];
    draw4(seed, L.p, frame, 0, 0, u);
    float3 x0;
    const LightDev ld = *lt;
    if (S.dm[0] > 0) {
      // distribution maps: the sample is drawn inside the path's cell
      dm_sample((const float*)xf, ld, S.dm, L.cell, u, &x0, &L.w);
    } else if (ld.kind == PV_LIGHT_CAMERA) {
      // uniform over the near plane at unit distance
      const float x = (2.0f * u[0] - 1.0f) * ld.param[0], y = (2.0f * u[1] - 1.0f) * ld.param[1];
      x0 = c;
      L.w = mul(add(add(mul(eu, x), mul(ev, y)), nl), 1.0f / sqrtf(x * x + y * y + 1.0f));
    } else {
      float a = (2.0f * u[0] - 1.0f) * ld.half[0], b = (2.0f * u[1] - 1.0f) * ld.half[1];
      x0 = add(c, add(mul(eu, a), mul(ev, b)));
      float3 lc = cosine_local(u[2], u[3]);
      if (ld.kind == PV_LIGHT_SPOT) {
        // the disk point scaled to the cone's radius, then lifted: with the
        // unit disk's height z0, 1 - sr^2 r^2 = cos^2 + sr^2 z0^2 (no
        // cancellation near the cone's rim)
        const float sr = sqrtf((1.0f - ld.param[0]) * (1.0f + ld.param[0]));
        const float z0 = lc.z;
        lc.x *= sr;
        lc.y *= sr;
        lc.z = sqrtf(ld.param[0] * ld.param[0] + (sr * sr) * (z0 * z0));
      }
      L.w = add(add(mul(eu, lc.x), mul(ev, lc.y)), mul(nl, lc.z));
    }
    const size_t stride = S.stride;
    PV_GLOBAL float* org = G(S.origin);
    org[L.p] = x0.x;
    org[stride + L.p] = x0.y;
    org[2 * stride + L.p] = x0.z;
    L.x = x0;
    L.mode = ST_FIRST;
  } else if (T < 0.0f) {
    L.x = vertex(S, L.p, L.k);
    L.w = normalize3(sub(vertex(S, L.p, L.k + 1), L.x));
    L.mode = ST_FIRST;
  } else {
    L.j = L.k;
    L.newn = L.n;
    // After the triangle test segment k is known to be blocked.  After the
    // box test it only reached a moved object's box, and Section 3.3 casts no
    // ray for a segment that the box crosses but no triangle: with its origin
    // unchanged the walk first checks it against the moved triangles.
    const bool origin_moved = L.k == 0 && G(S.light_moved)[L.l] != 0;
    L.mode = (S.verify_boxes && !origin_moved) ? ST_WCHECK : ST_WTRACE;
  }
}

template <bool kSingle, int kWaves>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWaves))) void k_retrace(const SceneDev* __restrict__ scenes, const uint32_t* __restrict__ gbase,
                                                    int n_scenes, const uint32_t* __restrict__ queue,
                                                    const uint32_t* __restrict__ qcount, float T,
                                                    uint64_t seed, uint32_t frame_arg, const uint32_t* frame_ptr,
                                                    pv_stats* stats, int min_active, uint32_t* __restrict__ deal_ctr) {
  extern __shared__ int32_t sstack[];  // traversal stacks, launch-time size
  __shared__ unsigned long long sred[kBlock / 64];
  __shared__ SceneTab stab;
  const StackCol col = (StackCol)(sstack + kBlock + threadIdx.x);  // entry 0 of the column; entry -1 spare
  const uint32_t frame = frame_ptr ? *frame_ptr : frame_arg;
  uint32_t n_rays = 0, n_photons = 0, n_acc = 0, n_trunc = 0;
  const PV_LDS SceneTab* tab = nullptr;
  if (kSingle) {
    load_tab(scenes[0], stab);
    tab = (const PV_LDS SceneTab*)&stab;
  }
  __shared__ uint32_t sgb[kSingle ? 1 : kLdsScenes + 1];
  if (!kSingle) gbase = stage_gbase(gbase, n_scenes, sgb);
  // the work queue, dealt by deal() from the counters 'deal_ctr'
  const uint32_t count = *qcount;
  const uint32_t wave = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  Lane L;
  L.S = scenes;
  L.mode = ST_IDLE;
  L.p = 0;
  Ray r;             // the lane's current query
  Walk wk;           // its walk through the hierarchy
  wk.cur = kRootNone;
  wk.leaf = 0;
  bool tracing = false, any = false;
  while (true) {
    // refill idle lanes from the queue
    const bool want = L.mode == ST_IDLE;
    if (__ballot(want)) {
      const uint32_t qi = deal(deal_ctr, wave, count, want);
      if (want) {
        if (qi != kNoEntry) {
          uint32_t gp = G(queue)[qi];
          if (kSingle) {
            L.p = gp;
          } else {
            uint32_t s = scene_of(gbase, n_scenes, gp);
            L.S = scenes + s;
            L.p = gp - gbase[s];
          }
          start_path(L, T, seed, frame, tab);
          // a path without the replace bit is skipped (stays idle this round)
        } else {
          L.mode = ST_END;
        }
      }
    }
    if (__ballot(L.mode != ST_END && L.mode != ST_IDLE) == 0) {
      if (__ballot(L.mode == ST_IDLE) == 0) break;
      continue;
    }
    const SceneDev& S = kSingle ? scenes[0] : *L.S;
    const bool busy = L.mode != ST_IDLE && L.mode != ST_END;
    // ---- a lane with a path and no walk in progress starts its next query
    if (busy && !tracing) {
      any = false;
      float3 qo = L.x, qd = L.w;
      float tmin = S.eps_end, tmax = kTFar;
      if (L.mode == ST_TAIL) {
        float3 nrm = dot(L.ntri, L.w) > 0.0f ? mul(L.ntri, -1.0f) : L.ntri;
        float u[4];
        draw4(seed, L.p, frame, L.row + 1, 1, u);
        float3 lc = cosine_local(u[0], u[1]);
        float3 tt, bb;
        onb(nrm, &tt, &bb);
        qd = add(add(mul(tt, lc.x), mul(bb, lc.y)), mul(nrm, lc.z));
      } else if (L.mode == ST_WCHECK || L.mode == ST_WTRACE || L.mode == ST_WSKIP) {
        uint32_t sj = L.mode == ST_WSKIP ? L.j + 1 : L.j;
        const float3 xa = vertex(S, L.p, sj), xb = vertex(S, L.p, sj + 1);
        if (L.mode == ST_WCHECK && (tab ? on_moved_obj(*tab, vertex_hit(S, L.p, sj + 1))
                                        : on_moved_obj(S, vertex_hit(S, L.p, sj + 1))))
          L.mode = ST_WTRACE;
        qo = xa;
        if (L.mode == ST_WTRACE) {
          qd = normalize3(sub(xb, xa));
        } else {
          // any hit of the segment xa -> xb against the moved objects
          any = true;
          qd = sub(xb, xa);
          float len = length(qd);
          tmin = len > 0.0f ? S.eps_end / len : 1.0f;
          tmax = 1.0f - tmin;
        }
      }
      r = make_ray(qo, qd, tmin, tmax);
      walk_start(wk, G(S.top)[any ? 1 : 0], tmax, col);
      tracing = true;
      if (!any) ++n_rays;
    }
    if (tracing) walk_run(G(S.nodes), G(S.tris), r, any, col, wk, min_active);
    if (!tracing || !walk_done(wk)) continue;
    // ---- the walk is finished: its query's ray is r (origin xa of a walk
    // segment, direction of a sampled bounce)
    tracing = false;
    Hit h;
    h.t = wk.tb;
    h.gid = wk.gid;
    h.rec = wk.rec;
    const float3 wn = r.d, qd = r.d, xa = r.o;
    // ---- advance the state machine with the result
    const bool hit = h.gid != kHitNone;
    switch (L.mode) {
      case ST_FIRST: {
        if (!hit) {
          ++n_trunc;
          L.newn = L.k;
          finish(L);
          break;
        }
        float3 xn = add(L.x, mul(L.w, h.t));
        float3 en;
        if (L.k == 0) {
          const PV_GLOBAL LightDev* lt = G(S.lights) + L.l;
          float N = (float)lt->path_count;
          en = f3(__fdiv_rn(lt->power[0], N), __fdiv_rn(lt->power[1], N), __fdiv_rn(lt->power[2], N));
        } else {
          en = reflect_energy(S, energy_row(S, L.p, L.k - 1), mat_of(S, vertex_hit(S, L.p, L.k)));
        }
        put_photon(S, L.p, L.k, xn, h.gid, en);
        ++n_photons;
        L.x = xn;
        L.ntri = hit_normal(S, h);
        L.mat = hit_material(S, h);
        L.e = en;
        L.row = L.k;
        to_tail(L);
        break;
      }
      case ST_TAIL: {
        if (!hit) {
          ++n_trunc;
          L.newn = L.row + 1;
          finish(L);
          break;
        }
        float3 xn = add(L.x, mul(wn, h.t));
        float3 en = reflect_energy(S, L.e, L.mat);
        L.row += 1;
        put_photon(S, L.p, L.row, xn, h.gid, en);
        ++n_photons;
        L.x = xn;
        L.w = wn;
        L.ntri = hit_normal(S, h);
        L.mat = hit_material(S, h);
        L.e = en;
        to_tail(L);
        break;
      }
      case ST_WCHECK: {
        if (hit) {
          L.mode = ST_WTRACE;
        } else if (++L.j >= L.newn) {
          finish(L);
        }
        break;
      }
      case ST_WTRACE: {
        if (!hit) {
          ++n_trunc;
          L.newn = L.j;
          finish(L);
          break;
        }
        float3 hp = add(xa, mul(qd, h.t));
        float3 ej = energy_row(S, L.p, L.j);
        if (L.j == L.newn - 1) {
          put_photon(S, L.p, L.j, hp, h.gid, ej);
          ++n_photons;
          finish(L);
          break;
        }
        float3 xc = vertex(S, L.p, L.j + 2);
        float3 d2 = sub(xc, hp);
        float3 nh = hit_normal(S, h);
        float c1 = dot(qd, nh), l2 = length(d2);
        float c2 = l2 > 0.0f ? dot(d2, nh) / l2 : 0.0f;
        uint32_t mat = hit_material(S, h);
        float3 en = (c1 * c2 < 0.0f) ? reflect_energy(S, ej, mat) : f3(0.0f, 0.0f, 0.0f);
        if (S.energy_test == PV_ENERGY_COSINE_RATIO && c1 * c2 < 0.0f) {
          // the kept direction's cosine at the new vertex over the one at the
          // old vertex (its stored triangle, from x_{j+1} to x_{j+2})
          const Tri to = G(S.tris)[G(S.gid_rec)[vertex_hit(S, L.p, L.j + 1)]];
          const float3 no = cross(sub(xyz(to.t1), xyz(to.t0)), sub(xyz(to.t2), xyz(to.t0)));
          const float3 d3 = sub(xc, vertex(S, L.p, L.j + 1));
          const float den = fabsf(dot(d3, no)), num = fabsf(c2) * length(d3) * length(no);
          const float ratio = den > 0.0f ? num / den : 0.0f;
          en = mul(en, ratio);
        }
        float3 eo = energy_row(S, L.p, L.j + 1);
        if (!eq2(en, eo, T)) {
          // energies differ: keep the new hit and re-sample the rest
          put_photon(S, L.p, L.j, hp, h.gid, ej);
          ++n_photons;
          L.x = hp;
          L.w = qd;
          L.ntri = nh;
          L.mat = mat;
          L.e = ej;
          L.row = L.j;
          to_tail(L);
          break;
        }
        ++n_acc;
        float dist = length(sub(hp, vertex(S, L.p, L.j + 1)));
        auto moved = [&](uint32_t hit) { return tab ? on_moved_obj(*tab, hit) : on_moved_obj(S, hit); };
        if (dist <= S.eps_close && !moved(h.gid) && !moved(vertex_hit(S, L.p, L.j + 1)) &&
            !moved(vertex_hit(S, L.p, L.j + 2))) {
          L.hp = hp;
          L.hgid = h.gid;
          L.mode = ST_WSKIP;  // the next segment must also be clear
          break;
        }
        put_photon(S, L.p, L.j, hp, h.gid, ej);
        ++n_photons;
        ++L.j;
        L.mode = ST_WTRACE;
        break;
      }
      case ST_WSKIP: {
        if (!hit) {
          L.j += 2;
          if (L.j >= L.newn)
            finish(L);
          else
            L.mode = ST_WCHECK;
        } else {
          put_photon(S, L.p, L.j, L.hp, L.hgid, energy_row(S, L.p, L.j));
          ++n_photons;
          ++L.j;
          L.mode = ST_WTRACE;
        }
        break;
      }
      default:
        break;
    }
  }
  if (stats) {
    unsigned long long a = block_sum_u64(n_rays, sred);
    unsigned long long b = block_sum_u64(n_photons, sred);
    unsigned long long c = block_sum_u64(n_acc, sred);
    unsigned long long d = block_sum_u64(n_trunc, sred);
    if (threadIdx.x == 0) {
      atomicAdd(&stats->rays_traced, a);
      atomicAdd(&stats->photons_written, b);
      atomicAdd(&stats->reuse_accepted, c);
      atomicAdd(&stats->paths_truncated, d);
    }
  }
}

// ---------------------------------------------------------------------------
// compaction of existing photons: counts per (row, block), scan, scatter

__global__ __launch_bounds__(kBlock) void k_photon_count(const SceneDev* __restrict__ scenes, const uint2* __restrict__ tiles,
                                                         uint32_t* __restrict__ counts) {
  __shared__ uint32_t wc[PV_MAX_BOUNCES][kBlock / 64];
  uint2 tile = tiles[blockIdx.x];
  const SceneDev& S = scenes[tile.x];
  uint32_t p = tile.y + threadIdx.x;
  uint32_t n = p < S.n_paths ? min(info_nseg(S.info[p]), S.B) : 0u;
  for (uint32_t r = 0; r < S.B; ++r) {
    uint64_t bal = __ballot(n > r);
    if (lane_id() == 0) wc[r][threadIdx.x >> 6] = (uint32_t)__popcll(bal);
  }
  __syncthreads();
  if (threadIdx.x < S.B) {
    uint32_t c = 0;
    for (int w = 0; w < kBlock / 64; ++w) c += wc[threadIdx.x][w];
    counts[S.count_base + threadIdx.x * S.n_blocks + tile.y / kBlock] = c;
  }
}

__global__ __launch_bounds__(kBlock) void k_photon_scatter(const SceneDev* __restrict__ scenes, const uint2* __restrict__ tiles,
                                                           const uint32_t* __restrict__ offsets,
                                                           float* __restrict__ out_pos, float* __restrict__ out_e,
                                                           uint32_t capacity) {
  __shared__ uint32_t wcnt[kBlock / 64];
  uint32_t r = blockIdx.y;
  uint2 tile = tiles[blockIdx.x];
  const SceneDev& S = scenes[tile.x];
  if (r >= S.B) return;
  uint32_t p = tile.y + threadIdx.x;
  bool flag = p < S.n_paths && min(info_nseg(S.info[p]), S.B) > r;
  uint64_t bal = __ballot(flag);
  if (lane_id() == 0) wcnt[threadIdx.x >> 6] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t pre = 0;
  for (uint32_t w = 0; w < (threadIdx.x >> 6); ++w) pre += wcnt[w];
  if (!flag) return;
  uint32_t idx = offsets[S.count_base + r * S.n_blocks + tile.y / kBlock] + pre + (uint32_t)__popcll(bal & lanemask_lt());
  if (idx >= capacity) return;
  size_t i = (size_t)r * S.stride + p;
  float4 x = S.pos[i], e = S.energy[i];
  out_pos[3 * (size_t)idx + 0] = x.x;
  out_pos[3 * (size_t)idx + 1] = x.y;
  out_pos[3 * (size_t)idx + 2] = x.z;
  out_e[3 * (size_t)idx + 0] = e.x;
  out_e[3 * (size_t)idx + 1] = e.y;
  out_e[3 * (size_t)idx + 2] = e.z;
}

// ---------------------------------------------------------------------------
// differentiation form

__global__ __launch_bounds__(kBlock) void k_energy_fwd(const SceneDev* __restrict__ scenes, const uint2* __restrict__ tiles,
                                                       const float* __restrict__ albedo, const float* __restrict__ power,
                                                       float* __restrict__ E) {
  uint2 tile = tiles[blockIdx.x];
  const SceneDev& S = scenes[tile.x];
  uint32_t p = tile.y + threadIdx.x;
  if (p >= S.n_paths) return;
  uint32_t n = min(info_nseg(S.info[p]), S.B);
  int l = light_of(S, p);
  if (l < 0) return;
  float N = (float)S.lights[l].path_count;
  float3 e = f3(__fdiv_rn(power[3 * l], N), __fdiv_rn(power[3 * l + 1], N), __fdiv_rn(power[3 * l + 2], N));
  const size_t np = S.n_paths;
  for (uint32_t r = 0; r < S.B; ++r) {
    float* o = E + 3 * ((size_t)r * np + p);
    if (r < n) {
      if (r > 0) {
        uint32_t m = mat_of(S, __float_as_uint(S.pos[(size_t)(r - 1) * S.stride + p].w));
        e = f3(__fmul_rn(e.x, albedo[3 * m]), __fmul_rn(e.y, albedo[3 * m + 1]), __fmul_rn(e.z, albedo[3 * m + 2]));
      }
      o[0] = e.x;
      o[1] = e.y;
      o[2] = e.z;
    } else {
      o[0] = o[1] = o[2] = 0.0f;
    }
  }
}

// One thread per path.  With P_j = prod_{i<j} rho_i (photon j has energy
// Phi/N * P_j) and R_i = g_{i+1} + rho_{i+1} R_{i+1} (R_{n-1} = 0, photon
// rows 0..n-1, vertex i = row i), the contribution of vertex i to the
// albedo gradient is Phi/N * P_i * R_i (division free), and the power
// gradient is sum_j g_j P_j / N.  Block partials go to
// partial[block][M*3 + L*3], which a fixed-order FP64 reduction sums across
// blocks; inside a block the contributions meet in FP32 LDS atomics, whose
// order follows the scheduling, so the gradients agree from run to run only
// to FP32 rounding of those sums, not bit for bit.
__global__ __launch_bounds__(kBlock) void k_energy_bwd(const SceneDev* __restrict__ scenes, const uint2* __restrict__ tiles,
                                                       const float* __restrict__ albedo, const float* __restrict__ power,
                                                       const float* __restrict__ gE, uint32_t n_mat,
                                                       float* __restrict__ partial) {
  extern __shared__ float acc[];  // n_mat*3 + n_lights*3
  uint2 tile = tiles[blockIdx.x];
  const SceneDev& S = scenes[tile.x];
  const uint32_t width = 3 * (n_mat + S.n_lights);
  for (uint32_t i = threadIdx.x; i < width; i += blockDim.x) acc[i] = 0.0f;
  __syncthreads();
  uint32_t p = tile.y + threadIdx.x;
  if (p < S.n_paths) {
    uint32_t n = min(info_nseg(S.info[p]), S.B);
    int l = light_of(S, p);
    if (l < 0) n = 0;
    float N = l >= 0 ? (float)S.lights[l].path_count : 1.0f;
    const size_t np = S.n_paths;
    uint32_t mats[PV_MAX_BOUNCES];
    for (uint32_t r = 0; r + 1 < n; ++r) mats[r] = mat_of(S, __float_as_uint(S.pos[(size_t)r * S.stride + p].w));
    for (int c = 0; c < 3; ++c) {
      // prefix products P_r for r = 0..n-1
      float P[PV_MAX_BOUNCES];
      float pr = 1.0f;
      float gp = 0.0f;
      for (uint32_t r = 0; r < n; ++r) {
        if (r > 0) pr *= albedo[3 * mats[r - 1] + c];
        P[r] = pr;
        gp += gE[3 * ((size_t)r * np + p) + c] * pr;
      }
      if (n == 0) break;
      atomicAdd(&acc[3 * n_mat + 3 * l + c], gp / N);
      float scale = power[3 * l + c] / N;
      float R = 0.0f;
      for (int i = (int)n - 2; i >= 0; --i) {
        // R_i = g_{i+1} + rho_{i+1} R_{i+1}
        float g1 = gE[3 * ((size_t)(i + 1) * np + p) + c];
        float rho1 = (i + 1 <= (int)n - 2) ? albedo[3 * mats[i + 1] + c] : 0.0f;
        R = g1 + rho1 * R;
        atomicAdd(&acc[3 * mats[i] + c], scale * P[i] * R);
      }
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < width; i += blockDim.x) partial[(size_t)blockIdx.x * width + i] = acc[i];
}

__global__ void k_reduce_partials(const float* __restrict__ partial, uint32_t n_blocks, uint32_t width,
                                  float* __restrict__ g_albedo, uint32_t n_mat3, float* __restrict__ g_power) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= width) return;
  double s = 0.0;
  for (uint32_t b = 0; b < n_blocks; ++b) s += (double)partial[(size_t)b * width + i];
  if (i < n_mat3)
    g_albedo[i] = (float)s;
  else
    g_power[i - n_mat3] = (float)s;
}

// ---------------------------------------------------------------------------
// Re-trace work order.  A path's re-trace costs up to one ray per segment from
// its first invalid one on, so the queue (ascending path ids, as the caller
// sees it) is handed to the persistent re-trace kernel reordered by that
// segment, smallest first (a stable counting sort over kOrderBuckets
// buckets): the refills deal the long paths first and the last refills of a
// launch are short paths, so the waves finish closer together.

constexpr uint32_t kOrderTile = 2048;  // queue entries per tile of the reorder
constexpr int kOrderBuckets = 8;

__device__ inline uint32_t order_bucket(const SceneDev* scenes, const uint32_t* gbase, int n_scenes, uint32_t gp) {
  const uint32_t s = scene_of(gbase, n_scenes, gp);
  const SceneDev& S = scenes[s];
  const uint32_t w = G(S.info)[gp - gbase[s]];
  const uint32_t n = min(info_nseg(w), S.B), k = info_start(w);
  return min(k < n ? k : 0u, (uint32_t)kOrderBuckets - 1u);  // k >= n: a new light sample, a full path
}

__global__ __launch_bounds__(kBlock) void k_order_hist(const SceneDev* __restrict__ scenes,
                                                       const uint32_t* __restrict__ gbase, int n_scenes,
                                                       const uint32_t* __restrict__ queue,
                                                       const uint32_t* __restrict__ qcount, uint32_t* __restrict__ hist,
                                                       uint32_t tiles) {
  __shared__ uint32_t h[kOrderBuckets];
  __shared__ uint32_t sgb[kLdsScenes + 1];
  if (n_scenes > 1) gbase = stage_gbase(gbase, n_scenes, sgb);  // uniform
  if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t count = *qcount, base = blockIdx.x * kOrderTile;
  const uint32_t end = min(base + kOrderTile, count);
  for (uint32_t e = base + threadIdx.x; e < end; e += kBlock)
    atomicAdd(&h[order_bucket(scenes, gbase, n_scenes, queue[e])], 1u);
  __syncthreads();
  if (threadIdx.x < kOrderBuckets) hist[threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// stable scatter of one tile: entries in index order, kBlock at a time; an
// entry's slot is its (bucket, tile) start plus the entries of its bucket
// placed by earlier rounds, lower waves and lower lanes (ballots over the
// bucket's bits)
__global__ __launch_bounds__(kBlock) void k_order_scatter(const SceneDev* __restrict__ scenes,
                                                          const uint32_t* __restrict__ gbase, int n_scenes,
                                                          const uint32_t* __restrict__ queue,
                                                          const uint32_t* __restrict__ qcount,
                                                          const uint32_t* __restrict__ hoff, uint32_t tiles,
                                                          uint32_t* __restrict__ out, uint32_t* __restrict__ deal_ctr) {
  constexpr int kWaves = kBlock / 64;
  static_assert(kOrderBuckets == 8, "three bucket bits");
  __shared__ uint32_t run[kOrderBuckets];
  __shared__ uint32_t wc[kWaves][kOrderBuckets];
  __shared__ uint32_t sgb[kLdsScenes + 1];
  deal_reset(deal_ctr);  // the re-trace that follows deals from these
  if (n_scenes > 1) gbase = stage_gbase(gbase, n_scenes, sgb);  // uniform
  const uint32_t count = *qcount, base = blockIdx.x * kOrderTile;
  if (base >= count) return;  // uniform over the block
  const uint32_t tid = threadIdx.x, w = tid >> 6;
  if (tid < kOrderBuckets) run[tid] = hoff[tid * tiles + blockIdx.x];
  for (uint32_t r = 0; r < kOrderTile / kBlock; ++r) {
    __syncthreads();
    if (tid < kWaves * kOrderBuckets) wc[tid / kOrderBuckets][tid % kOrderBuckets] = 0;
    __syncthreads();
    const uint32_t e = base + r * kBlock + tid;
    const bool valid = e < count;
    uint32_t gp = 0, b = 0;
    if (valid) {
      gp = queue[e];
      b = order_bucket(scenes, gbase, n_scenes, gp);
    }
    uint64_t peers = __ballot(valid);
    for (int bit = 0; bit < 3; ++bit) {
      const bool set = ((b >> bit) & 1u) != 0;
      const uint64_t m = __ballot(valid && set);
      peers &= set ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
    if (valid && rank == 0) wc[w][b] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t before = 0;
      for (uint32_t q = 0; q < w; ++q) before += wc[q][b];
      out[run[b] + before + rank] = gp;
    }
    __syncthreads();
    if (tid < kOrderBuckets) {
      uint32_t add = 0;
      for (int q = 0; q < kWaves; ++q) add += wc[q][tid];
      run[tid] += add;
    }
  }
}

uint32_t order_tiles(uint32_t max_entries) { return (max_entries + kOrderTile - 1) / kOrderTile; }

// ---------------------------------------------------------------------------
// launch wrappers (host side)

hipError_t launch_frame_begin(SceneDev* scenes, int n_scenes, const float* const* obj_in,
                              const float* const* light_in, hipStream_t s) {
  hipLaunchKernelGGL(k_frame_begin, dim3(n_scenes), dim3(64), 0, s, scenes, n_scenes, obj_in, light_in);
  return hipGetLastError();
}

hipError_t launch_update_objects(SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, const uint2* xf_tiles,
                                 uint32_t n_xf_tiles, hipStream_t s) {
  if (!n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_transform, dim3(n_xf_tiles), dim3(kBlock), 0, s, scenes, xf_tiles);
  hipLaunchKernelGGL(k_update_objects, dim3(n_tiles), dim3(kRefitBlock), 0, s, scenes, tiles);
  return hipGetLastError();
}

hipError_t launch_transform_objects(SceneDev* scenes, const uint2* xf_tiles, uint32_t n_xf_tiles, hipStream_t s) {
  if (!n_xf_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_transform, dim3(n_xf_tiles), dim3(kBlock), 0, s, scenes, xf_tiles);
  return hipGetLastError();
}

hipError_t launch_build_top(SceneDev* scenes, int n_scenes, hipStream_t s) {
  if (n_scenes <= 0) return hipSuccess;
  k_build_top<<<n_scenes, 128, 0, s>>>(scenes);
  return hipGetLastError();
}

// the stack columns of a block, plus one spare entry below each column (a walk
// whose sentinel was taken points there)
static size_t stack_bytes(uint32_t entries) { return (size_t)(entries + 1) * kBlock * sizeof(int32_t); }

uint32_t verify_finish_blocks(uint32_t trace_blocks) { return std::max(1u, trace_blocks / 2); }

hipError_t launch_verify(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, const uint32_t* gbase,
                         int n_scenes, VerifyWork W, uint32_t* block_cnt, pv_stats* stats, uint32_t stack,
                         uint32_t trace_blocks, int min_active, uint32_t* scan_tmp, hipStream_t s) {
  if (!n_tiles) return hipSuccess;
  if (stack < 2 || stack > (uint32_t)kMaxStack || trace_blocks == 0 || min_active < 1 || min_active > 64)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_verify_scan, dim3(n_tiles), dim3(kBlock), 0, s, scenes, tiles, W, block_cnt, stats);
  hipError_t e = launch_scan(W.tcount, W.toff, n_tiles, W.total, scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_verify_gather, dim3(n_tiles), dim3(kBlock), 0, s, scenes, tiles, W);
  const dim3 gt(trace_blocks), gf(verify_finish_blocks(trace_blocks));
  if (n_scenes == 1) {
    hipLaunchKernelGGL(k_verify_trace<true>, gt, dim3(kBlock), stack_bytes(stack), s, scenes, gbase, n_scenes, W,
                       min_active);
    hipLaunchKernelGGL(k_verify_finish<true>, gf, dim3(kBlock), 0, s, scenes, gbase, n_scenes, W, block_cnt, n_tiles,
                       stats);
  } else {
    hipLaunchKernelGGL(k_verify_trace<false>, gt, dim3(kBlock), stack_bytes(stack), s, scenes, gbase, n_scenes, W,
                       min_active);
    hipLaunchKernelGGL(k_verify_finish<false>, gf, dim3(kBlock), 0, s, scenes, gbase, n_scenes, W, block_cnt, n_tiles,
                       stats);
  }
  if (stats) {
    const uint32_t sb = std::min(16u, (std::max(n_tiles, gf.x) + 1023) / 1024);
    hipLaunchKernelGGL(k_verify_stats, dim3(sb), dim3(1024), 0, s, W.part, n_tiles, gf.x, stats);
  }
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total,
                       uint32_t* tile_tmp, hipStream_t s) {
  if (n <= kScanTile) {  // one tile: its total is the scan's
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, in, out, n, total);
    return hipGetLastError();
  }
  if (!tile_tmp) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, in, out, n, total);
    return hipGetLastError();
  }
  // tile_tmp holds 2 * ceil(n / kScanTile) words: tile sums, then their offsets
  const uint32_t tiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(1024), 0, s, in, out, n, tile_tmp);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, tile_tmp, tile_tmp + tiles, tiles, total);
  hipLaunchKernelGGL(k_scan_add, dim3((n + 255) / 256), dim3(256), 0, s, out, n, tile_tmp + tiles);
  return hipGetLastError();
}

uint32_t scan_tmp_words(uint32_t n) { return 2 * ((n + kScanTile - 1) / kScanTile) + 2; }

hipError_t launch_scatter_queue(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, const uint32_t* offsets,
                                uint32_t* queue, hipStream_t s) {
  if (!n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_queue, dim3(n_tiles), dim3(kBlock), 0, s, scenes, tiles, offsets, queue);
  return hipGetLastError();
}

hipError_t launch_mark_all(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, uint32_t* block_cnt,
                           hipStream_t s) {
  if (!n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_mark_all, dim3(n_tiles), dim3(kBlock), 0, s, scenes, tiles, block_cnt);
  return hipGetLastError();
}

// variant v selects the occupancy target of the re-trace kernel (waves per
// SIMD the compiler must allow): 0 -> 4, 1 -> 5, 2 -> 6, 3 -> 8
template <bool kSingle>
static void retrace_variant(int v, dim3 g, size_t lds, hipStream_t s, const SceneDev* scenes, const uint32_t* gbase, int n_scenes,
                            const uint32_t* queue, const uint32_t* qcount, float T, uint64_t seed,
                            uint32_t frame, const uint32_t* frame_ptr, pv_stats* stats, int min_active,
                            uint32_t* deal_ctr) {
  switch (v) {
    case 1:
      hipLaunchKernelGGL((k_retrace<kSingle, 5>), g, dim3(kBlock), lds, s, scenes, gbase, n_scenes, queue, qcount,
                         T, seed, frame, frame_ptr, stats, min_active, deal_ctr);
      break;
    case 2:
      hipLaunchKernelGGL((k_retrace<kSingle, 6>), g, dim3(kBlock), lds, s, scenes, gbase, n_scenes, queue, qcount,
                         T, seed, frame, frame_ptr, stats, min_active, deal_ctr);
      break;
    case 3:
      hipLaunchKernelGGL((k_retrace<kSingle, 8>), g, dim3(kBlock), lds, s, scenes, gbase, n_scenes, queue, qcount,
                         T, seed, frame, frame_ptr, stats, min_active, deal_ctr);
      break;
    default:
      hipLaunchKernelGGL((k_retrace<kSingle, 4>), g, dim3(kBlock), lds, s, scenes, gbase, n_scenes, queue, qcount,
                         T, seed, frame, frame_ptr, stats, min_active, deal_ctr);
      break;
  }
}

hipError_t launch_retrace(const SceneDev* scenes, const uint32_t* gbase, int n_scenes, const uint32_t* queue_in,
                          const uint32_t* qcount, float T, uint64_t seed, uint32_t frame,
                          const uint32_t* frame_ptr, pv_stats* stats, uint32_t n_blocks, int variant, uint32_t stack,
                          int min_active, const OrderWork& O, hipStream_t s) {
  if (stack < 2 || stack > (uint32_t)kMaxStack || min_active < 1 || min_active > 64) return hipErrorInvalidValue;
  // the queue reordered by first invalid segment (see k_order_hist)
  hipLaunchKernelGGL(k_order_hist, dim3(O.tiles), dim3(kBlock), 0, s, scenes, gbase, n_scenes, queue_in, qcount, O.hist,
                     O.tiles);
  hipError_t e = launch_scan(O.hist, O.hoff, kOrderBuckets * O.tiles, O.htotal, O.scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_order_scatter, dim3(O.tiles), dim3(kBlock), 0, s, scenes, gbase, n_scenes, queue_in, qcount,
                     O.hoff, O.tiles, O.queue, O.deal);
  const uint32_t* queue = O.queue;
  if (n_scenes == 1)
    retrace_variant<true>(variant, dim3(n_blocks), stack_bytes(stack), s, scenes, gbase, n_scenes, queue, qcount, T, seed, frame,
                          frame_ptr, stats, min_active, O.deal);
  else
    retrace_variant<false>(variant, dim3(n_blocks), stack_bytes(stack), s, scenes, gbase, n_scenes, queue, qcount, T, seed, frame,
                           frame_ptr, stats, min_active, O.deal);
  return hipGetLastError();
}

hipError_t launch_photon_count(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, uint32_t* counts,
                               hipStream_t s) {
  if (!n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_photon_count, dim3(n_tiles), dim3(kBlock), 0, s, scenes, tiles, counts);
  return hipGetLastError();
}

hipError_t launch_photon_scatter(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, uint32_t B,
                                 const uint32_t* offsets, float* out_pos, float* out_e, uint32_t capacity,
                                 hipStream_t s) {
  if (!n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_photon_scatter, dim3(n_tiles, B), dim3(kBlock), 0, s, scenes, tiles, offsets, out_pos, out_e,
                     capacity);
  return hipGetLastError();
}

// photon ranges of the scenes of a batch: base[s] = offsets[count_base of s],
// base[n] = total
__global__ void k_scene_photon_base(const SceneDev* __restrict__ scenes, int n_scenes, const uint32_t* __restrict__ offsets,
                                    const uint32_t* __restrict__ total, uint32_t* __restrict__ base) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_scenes) base[i] = offsets[scenes[i].count_base];
  if (i == n_scenes) base[i] = *total;
}

hipError_t launch_scene_photon_base(const SceneDev* scenes, int n_scenes, const uint32_t* offsets, const uint32_t* total,
                                    uint32_t* base, hipStream_t s) {
  hipLaunchKernelGGL(k_scene_photon_base, dim3((n_scenes + 64) / 64), dim3(64), 0, s, scenes, n_scenes, offsets, total,
                     base);
  return hipGetLastError();
}

hipError_t launch_energy_fwd(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, const float* albedo,
                             const float* power, float* E, hipStream_t s) {
  if (!n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_energy_fwd, dim3(n_tiles), dim3(kBlock), 0, s, scenes, tiles, albedo, power, E);
  return hipGetLastError();
}

hipError_t launch_energy_bwd(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, const float* albedo,
                             const float* power, const float* gE, uint32_t n_mat, uint32_t n_lights, float* partial,
                             float* g_albedo, float* g_power, hipStream_t s) {
  uint32_t width = 3 * (n_mat + n_lights);
  if (n_tiles) {
    hipLaunchKernelGGL(k_energy_bwd, dim3(n_tiles), dim3(kBlock), width * sizeof(float), s, scenes, tiles, albedo,
                       power, gE, n_mat, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_reduce_partials, dim3((width + 255) / 256), dim3(256), 0, s, partial, n_tiles, width, g_albedo,
                     3 * n_mat, g_power);
  return hipGetLastError();
}

}  // namespace pv
