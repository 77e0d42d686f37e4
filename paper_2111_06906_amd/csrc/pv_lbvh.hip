// Per-frame rebuild of the dynamic objects' hierarchies on the device: a
// linear BVH (Karras, "Maximizing Parallelism in the Construction of BVHs,
// Octrees, and k-d Trees", HPG 2012) over 30-bit Morton codes of the
// triangles' centroids, quantised in each object's centroid box.
//
//   k_lbvh_bounds   one workgroup per object: centroid box of its triangles
//   k_lbvh_keys     one thread per dynamic triangle: key (object << 30 |
//                   Morton code), value (its record)
//   k_lbvh_hist /   stable least-significant-digit radix sort of the keys,
//   launch_scan /   8 bits per pass: digit counts per tile, their scan, and a
//   k_lbvh_scatter  scatter that keeps the order of equal digits (wave ballots
//                   rank the keys of one digit inside a wave)
//   k_lbvh_nodes    one thread per internal node of each object's radix tree:
//                   its key range and split (the object's keys are contiguous
//                   after the sort); equal keys are ordered by position
//   k_lbvh_boxes    one thread per leaf climbs towards the root; at each node
//                   the second child to finish computes the node's boxes and
//                   height (an arrival counter per node; no thread ever waits)
//
// Leaves hold one triangle and name its record directly, so triangles are
// never moved.  A radix tree can be deeper than the traversal stack allows
// (up to 30 + ceil(log2 n) levels: the common prefix of a node's keys grows
// from a node to its children, and the varying key bits are the Morton code
// and the position); an object whose rebuilt tree is deeper than the depth
// allowance keeps its refit upload-time topology for the frame.
#include "pv_launch.h"

namespace pv {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr uint32_t kSortTile = kSortThreads * kSortItems;  // keys per sort tile
constexpr int kDigits = 256;
constexpr int kSortPasses = 5;  // 8-bit digits over the 36 key bits (6 object + 30 Morton)
static_assert(kSortThreads == kDigits, "one thread per digit in the tile histograms");
static_assert(PV_MAX_OBJECTS <= 64, "object ids fit the 6 key bits above the Morton code");

__device__ inline uint32_t lane_of() { return threadIdx.x & 63u; }
__device__ inline uint64_t lanes_below() { return (1ull << lane_of()) - 1ull; }

__device__ inline float pad_lo(float x) { return x - (1e-6f + fabsf(x) * 1e-6f); }
__device__ inline float pad_hi(float x) { return x + (1e-6f + fabsf(x) * 1e-6f); }

// object of a dynamic triangle record: the last object whose first record is
// not after it (records are grouped by object, in object order)
__device__ inline uint32_t object_of_record(const SceneDev& S, uint32_t r) {
  uint32_t lo = 0, hi = S.n_obj;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (S.objs[mid].tri_base <= r)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__device__ inline float3 centroid(const Tri& t) {
  const float s = 1.0f / 3.0f;
  return make_float3((t.t0.x + t.t1.x + t.t2.x) * s, (t.t0.y + t.t1.y + t.t2.y) * s, (t.t0.z + t.t1.z + t.t2.z) * s);
}

// 10 bits spread to every third bit
__device__ inline uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ inline uint32_t quantise(float c, float lo, float hi) {
  const float ext = hi - lo;
  const float u = ext > 0.0f ? (c - lo) / ext : 0.0f;
  return min((uint32_t)fmaxf(u * 1024.0f, 0.0f), 1023u);
}

}  // namespace

__global__ __launch_bounds__(1024) void k_lbvh_bounds(const SceneDev* __restrict__ scenes, LbvhWork W) {
  __shared__ float red[6][1024 / 64];
  const SceneDev& S = scenes[0];
  const uint32_t o = blockIdx.x;
  const ObjDev ob = S.objs[o];
  float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
  float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
  for (uint32_t i = threadIdx.x; i < ob.n_tris; i += blockDim.x) {
    const float3 c = centroid(S.tris[S.n_static + ob.tri_base + i]);
    lo[0] = fminf(lo[0], c.x), lo[1] = fminf(lo[1], c.y), lo[2] = fminf(lo[2], c.z);
    hi[0] = fmaxf(hi[0], c.x), hi[1] = fmaxf(hi[1], c.y), hi[2] = fmaxf(hi[2], c.z);
  }
  for (int off = 32; off > 0; off >>= 1)
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], off, 64));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off, 64));
    }
  const uint32_t w = threadIdx.x >> 6;
  if (lane_of() == 0)
    for (int k = 0; k < 3; ++k) {
      red[k][w] = lo[k];
      red[3 + k][w] = hi[k];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = (int)threadIdx.x;
    float v = red[k][0];
    for (uint32_t q = 1; q < blockDim.x / 64; ++q) v = k < 3 ? fminf(v, red[k][q]) : fmaxf(v, red[k][q]);
    W.cbox[6 * o + k] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_lbvh_keys(const SceneDev* __restrict__ scenes, LbvhWork W) {
  const SceneDev& S = scenes[0];
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= W.n_dyn) return;
  const uint32_t o = object_of_record(S, r);
  const float3 c = centroid(S.tris[S.n_static + r]);
  const float* b = W.cbox + 6 * o;
  const uint32_t m = (spread3(quantise(c.x, b[0], b[3])) << 2) | (spread3(quantise(c.y, b[1], b[4])) << 1) |
                     spread3(quantise(c.z, b[2], b[5]));
  W.key[0][r] = ((uint64_t)o << 30) | m;
  W.val[0][r] = r;
}

// digit counts of one tile, stored digit-major (hist[digit * tiles + tile]),
// so that an exclusive scan gives every (digit, tile) its first output slot
__global__ __launch_bounds__(kSortThreads) void k_lbvh_hist(const uint64_t* __restrict__ key, uint32_t n, int shift,
                                                            uint32_t* __restrict__ hist, uint32_t tiles) {
  __shared__ uint32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kSortTile;
  for (int s = 0; s < kSortItems; ++s) {
    const uint32_t e = base + (uint32_t)s * kSortThreads + threadIdx.x;
    if (e < n) atomicAdd(&h[(uint32_t)(key[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: keys are taken in index order, kSortThreads at
// a time; a key's slot is the scanned start of its (digit, tile), plus the
// keys of its digit placed by earlier rounds, by lower waves of this round and
// by lower lanes of its wave (lanes of equal digit found by ballots over the
// digit's bits).
__global__ __launch_bounds__(kSortThreads) void k_lbvh_scatter(const uint64_t* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                               uint32_t n, int shift, const uint32_t* __restrict__ hoff,
                                                               uint32_t tiles) {
  constexpr int kWaves = kSortThreads / 64;
  __shared__ uint32_t run[kDigits];
  __shared__ uint32_t wc[kWaves][kDigits];
  const uint32_t tid = threadIdx.x, w = tid >> 6;
  run[tid] = hoff[tid * tiles + blockIdx.x];
  const uint32_t base = blockIdx.x * kSortTile;
  for (int s = 0; s < kSortItems; ++s) {
    for (int q = 0; q < kWaves; ++q) wc[q][tid] = 0;
    __syncthreads();
    const uint32_t e = base + (uint32_t)s * kSortThreads + tid;
    const bool valid = e < n;
    uint64_t k = 0;
    uint32_t v = 0, d = 0;
    if (valid) {
      k = kin[e];
      v = vin[e];
      d = (uint32_t)(k >> shift) & 255u;
    }
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const bool bit = ((d >> b) & 1u) != 0;
      const uint64_t set = __ballot(valid && bit);
      peers &= bit ? set : ~set;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lanes_below());
    if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t before = 0;
      for (uint32_t q = 0; q < w; ++q) before += wc[q][d];
      const uint32_t pos = run[d] + before + rank;
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < kWaves; ++q) add += wc[q][tid];
    run[tid] += add;
  }
}

namespace {

// length of the common prefix of the keys at positions i and j of an object's
// sorted range (ties broken by position); -1 outside the range
__device__ inline int prefix(const uint64_t* __restrict__ key, uint32_t start, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  const uint64_t a = key[start + (uint32_t)i], b = key[start + (uint32_t)j];
  if (a != b) return __clzll((long long)(a ^ b));
  return 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_lbvh_nodes(SceneDev* __restrict__ scenes, LbvhWork W,
                                                       const uint64_t* __restrict__ key,
                                                       const uint32_t* __restrict__ val) {
  SceneDev& S = scenes[0];
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= W.n_dyn) return;
  const uint32_t o = (uint32_t)(key[g] >> 30);
  const ObjDev ob = S.objs[o];
  const uint32_t start = ob.tri_base;
  const int n = (int)ob.n_tris;
  const int i = (int)(g - start);
  if (n < 2 || i >= n - 1) return;
  // direction of the node's range and its far end
  const int d = prefix(key, start, n, i, i + 1) > prefix(key, start, n, i, i - 1) ? 1 : -1;
  const int dmin = prefix(key, start, n, i, i - d);
  int lmax = 2;
  while (prefix(key, start, n, i, i + lmax * d) > dmin) lmax *= 2;
  int l = 0;
  for (int t = lmax / 2; t >= 1; t /= 2)
    if (prefix(key, start, n, i, i + (l + t) * d) > dmin) l += t;
  const int j = i + l * d;
  // split: the last position sharing more than the range's common prefix with i
  const int dnode = prefix(key, start, n, i, j);
  int s = 0;
  for (int t = (l + 1) / 2;; t = (t + 1) / 2) {
    if (prefix(key, start, n, i, i + (s + t) * d) > dnode) s += t;
    if (t == 1) break;
  }
  const int split = i + s * d + min(d, 0);
  const uint32_t node = ob.lbvh_base + (uint32_t)i;
  int32_t ch[2];
  for (int side = 0; side < 2; ++side) {
    const int c = split + side;
    const bool leaf = side == 0 ? min(i, j) == c : max(i, j) == c;
    if (leaf) {
      ch[side] = leaf_code(S.n_static + val[start + (uint32_t)c], 1);
      W.parent_leaf[start + (uint32_t)c] = (int32_t)node;
    } else {
      ch[side] = (int32_t)(ob.lbvh_base + (uint32_t)c);
      W.parent_node[ob.lbvh_base + (uint32_t)c - W.first_node] = (int32_t)node;
    }
  }
  S.nodes[node].d = make_int4(ch[0], ch[1], -1, 0);
  W.flag[node - W.first_node] = 0;
  if (i == 0) W.parent_node[node - W.first_node] = -1;
}

namespace {

__device__ inline void tri_box(const Tri& t, float* b) {
  b[0] = pad_lo(fminf(fminf(t.t0.x, t.t1.x), t.t2.x));
  b[1] = pad_lo(fminf(fminf(t.t0.y, t.t1.y), t.t2.y));
  b[2] = pad_lo(fminf(fminf(t.t0.z, t.t1.z), t.t2.z));
  b[3] = pad_hi(fmaxf(fmaxf(t.t0.x, t.t1.x), t.t2.x));
  b[4] = pad_hi(fmaxf(fmaxf(t.t0.y, t.t1.y), t.t2.y));
  b[5] = pad_hi(fmaxf(fmaxf(t.t0.z, t.t1.z), t.t2.z));
}

// box of a child while the hierarchy is being built: a leaf's padded triangle
// box, or the union of a node's two child boxes, which another thread of this
// launch wrote (read at device scope, past this compute unit's cache)
__device__ inline void rebuilt_child_box(const SceneDev& S, int32_t code, float* b) {
  if (code < 0) {
    tri_box(S.tris[leaf_first(code)], b);
    return;
  }
  const uint32_t* w = reinterpret_cast<const uint32_t*>(S.nodes + code);
  float f[12];
  for (int k = 0; k < 12; ++k)
    f[k] = __uint_as_float(__hip_atomic_load(w + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  for (int k = 0; k < 3; ++k) {
    b[k] = fminf(f[k], f[6 + k]);
    b[3 + k] = fmaxf(f[3 + k], f[9 + k]);
  }
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_lbvh_boxes(SceneDev* __restrict__ scenes, LbvhWork W,
                                                       const uint64_t* __restrict__ key,
                                                       const uint32_t* __restrict__ val, uint32_t max_depth) {
  SceneDev& S = scenes[0];
  ObjDev* objs = const_cast<ObjDev*>(S.objs);
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= W.n_dyn) return;
  const uint32_t o = (uint32_t)(key[g] >> 30);
  if (S.objs[o].n_tris == 1) {
    const int32_t leaf = leaf_code(S.n_static + val[g], 1);
    float b[6];
    tri_box(S.tris[leaf_first(leaf)], b);
    for (int k = 0; k < 6; ++k) S.obj_aabb[6 * o + k] = b[k];
    objs[o].root = leaf;
    return;
  }
  int32_t p = W.parent_leaf[g];
  while (true) {
    // the first child to arrive stops; the second builds the node: every
    // node is completed exactly once, after both of its children
    __threadfence();
    if (atomicAdd(&W.flag[(uint32_t)p - W.first_node], 1u) == 0u) return;
    __threadfence();
    Node& nd = S.nodes[p];
    const int4 ch = nd.d;
    float b[12];
    rebuilt_child_box(S, ch.x, b);
    rebuilt_child_box(S, ch.y, b + 6);
    nd.a = make_float4(b[0], b[1], b[2], b[3]);
    nd.b = make_float4(b[4], b[5], b[6], b[7]);
    nd.c = make_float4(b[8], b[9], b[10], b[11]);
    uint32_t h = 0;  // levels below this node
    for (int side = 0; side < 2; ++side) {
      const int32_t c = side ? ch.y : ch.x;
      const uint32_t hc = c < 0 ? 0u
                                : __hip_atomic_load(&W.height[(uint32_t)c - W.first_node], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
      h = max(h, hc + 1);
    }
    W.height[(uint32_t)p - W.first_node] = h;
    const int32_t up = W.parent_node[(uint32_t)p - W.first_node];
    if (up < 0) {
      // the rebuilt tree replaces the refit topology only within the depth
      // the traversal stacks were sized for
      if (h <= max_depth) {
        for (int k = 0; k < 3; ++k) {
          S.obj_aabb[6 * o + k] = fminf(b[k], b[6 + k]);
          S.obj_aabb[6 * o + 3 + k] = fmaxf(b[3 + k], b[9 + k]);
        }
        objs[o].root = p;
      }
      return;
    }
    p = up;
  }
}

hipError_t launch_rebuild_objects(SceneDev* scenes, LbvhWork W, uint32_t n_obj, uint32_t max_depth, hipStream_t s) {
  if (!W.n_dyn || !n_obj) return hipSuccess;
  hipLaunchKernelGGL(k_lbvh_bounds, dim3(n_obj), dim3(1024), 0, s, scenes, W);
  const uint32_t nb = (W.n_dyn + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_lbvh_keys, dim3(nb), dim3(kBlock), 0, s, scenes, W);
  const uint32_t tiles = lbvh_sort_tiles(W.n_dyn);
  int src = 0;
  for (int pass = 0; pass < kSortPasses; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(k_lbvh_hist, dim3(tiles), dim3(kSortThreads), 0, s, W.key[src], W.n_dyn, shift, W.hist, tiles);
    hipError_t e = launch_scan(W.hist, W.hoff, kDigits * tiles, W.htotal, W.scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lbvh_scatter, dim3(tiles), dim3(kSortThreads), 0, s, W.key[src], W.val[src], W.key[src ^ 1],
                       W.val[src ^ 1], W.n_dyn, shift, W.hoff, tiles);
    src ^= 1;
  }
  hipLaunchKernelGGL(k_lbvh_nodes, dim3(nb), dim3(kBlock), 0, s, scenes, W, W.key[src], W.val[src]);
  hipLaunchKernelGGL(k_lbvh_boxes, dim3(nb), dim3(kBlock), 0, s, scenes, W, W.key[src], W.val[src], max_depth);
  return hipGetLastError();
}

uint32_t lbvh_sort_tiles(uint32_t n_dyn) { return (n_dyn + kSortTile - 1) / kSortTile; }

}  // namespace pv
