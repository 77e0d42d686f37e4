// Per-frame rebuild of the dynamic objects' hierarchies on the device: a
// linear BVH (Karras, "Maximizing Parallelism in the Construction of BVHs,
// Octrees, and k-d Trees", HPG 2012) over 30-bit Morton codes of the
// triangles' centroids, quantised in each object's centroid box.
//
//   k_lbvh_bounds   one workgroup per object: centroid box of its triangles
//   k_lbvh_keys     one thread per dynamic triangle: key (object << 30 |
//                   Morton code), value (its record)
//   k_lbvh_hist /   stable least-significant-digit radix sort of the keys, 8
//   k_lbvh_scatter  bits per pass: digit counts per tile, then a scatter that
//                   keeps the order of equal digits (wave ballots rank the keys
//                   of one digit inside a wave); the scatter scans the counts
//                   itself when there are few tiles
//   k_lbvh_leaves / padded triangle boxes in sorted order and a pyramid of
//   k_lbvh_pyramid  their unions over aligned power-of-two blocks
//   k_lbvh_nodes    one thread per internal node of each object's radix tree:
//                   its key range and split (the object's keys are contiguous
//                   after the sort; equal keys are ordered by position), and
//                   its two child boxes as unions over the children's position
//                   ranges, each assembled from O(log n) pyramid entries: no
//                   node waits for another
//   k_lbvh_depth    one thread per leaf counts its ancestors
//   k_lbvh_finish   one thread per object: the rebuilt tree becomes the
//                   object's hierarchy unless it is deeper than the traversal
//                   stacks allow (up to 30 + ceil(log2 n) levels are possible:
//                   the common prefix of a node's keys grows from a node to its
//                   children); the refit upload-time topology serves otherwise
//
// Leaves hold one triangle and name its record directly, so triangles are
// never moved.  The boxes are the same unions of the same padded triangle
// boxes that a bottom-up refit computes.
#include "pv_launch.h"

namespace pv {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr uint32_t kSortTile = kSortThreads * kSortItems;  // keys per sort tile
constexpr int kDigits = 256;
constexpr int kSortPasses = 5;          // 8-bit digits over the 36 key bits (6 object + 30 Morton)
constexpr uint32_t kFusedTiles = 256;   // up to this many tiles the scatter scans the counts itself
constexpr int kLowLevels = 8;           // pyramid levels built inside one 256-entry workgroup
constexpr uint32_t kDepthGuard = 64;    // > 30 + 28: no radix tree here is that deep
static_assert(kSortThreads == kDigits, "one thread per digit in the tile histograms");
static_assert(kBlock == (1 << kLowLevels), "one workgroup of the leaf kernel spans the low pyramid levels");
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

struct Box {
  float3 lo, hi;
};

__device__ inline Box empty_box() {
  return {make_float3(__builtin_inff(), __builtin_inff(), __builtin_inff()),
          make_float3(-__builtin_inff(), -__builtin_inff(), -__builtin_inff())};
}

__device__ inline Box join(const Box& a, const Box& b) {
  return {make_float3(fminf(a.lo.x, b.lo.x), fminf(a.lo.y, b.lo.y), fminf(a.lo.z, b.lo.z)),
          make_float3(fmaxf(a.hi.x, b.hi.x), fmaxf(a.hi.y, b.hi.y), fmaxf(a.hi.z, b.hi.z))};
}

// a leaf's box: the padded box of its triangle (as the refit computes it)
__device__ inline Box tri_box(const Tri& t) {
  return {make_float3(pad_lo(fminf(fminf(t.t0.x, t.t1.x), t.t2.x)), pad_lo(fminf(fminf(t.t0.y, t.t1.y), t.t2.y)),
                      pad_lo(fminf(fminf(t.t0.z, t.t1.z), t.t2.z))),
          make_float3(pad_hi(fmaxf(fmaxf(t.t0.x, t.t1.x), t.t2.x)), pad_hi(fmaxf(fmaxf(t.t0.y, t.t1.y), t.t2.y)),
                      pad_hi(fmaxf(fmaxf(t.t0.z, t.t1.z), t.t2.z)))};
}

__device__ inline Box pyr_get(const float4* pyr, uint32_t i) {
  const float4 a = pyr[2 * i], b = pyr[2 * i + 1];
  return {make_float3(a.x, a.y, a.z), make_float3(b.x, b.y, b.z)};
}

__device__ inline void pyr_put(float4* pyr, uint32_t i, const Box& v) {
  pyr[2 * i] = make_float4(v.lo.x, v.lo.y, v.lo.z, 0.0f);
  pyr[2 * i + 1] = make_float4(v.hi.x, v.hi.y, v.hi.z, 0.0f);
}

// union of the boxes at sorted positions [a, b) from the pyramid: at each
// level the blocks at the range's ragged ends, then one level up.  The
// entries of four levels are loaded before any of them is joined, so their
// loads are in flight together (min and max: the order of the joins does not
// change the box).
__device__ inline Box range_box(const float4* pyr, uint32_t n, uint32_t a, uint32_t b) {
  Box r = empty_box();
  uint32_t off = 0, m = n;
  while (a < b) {
    Box e[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool ta = a < b && (a & 1u) != 0u;
      e[2 * k] = ta ? pyr_get(pyr, off + a) : empty_box();
      a += ta ? 1u : 0u;
      const bool tb = a < b && (b & 1u) != 0u;
      e[2 * k + 1] = tb ? pyr_get(pyr, off + b - 1u) : empty_box();
      b -= tb ? 1u : 0u;
      a >>= 1;
      b >>= 1;
      off += m;
      m = (m + 1) / 2;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) r = join(r, e[k]);
  }
  return r;
}

// length of the common prefix of the keys at positions i and j of an object's
// sorted range (ties broken by position); -1 outside the range
__device__ inline int prefix(const uint64_t* __restrict__ key, uint32_t start, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  const uint64_t a = key[start + (uint32_t)i], b = key[start + (uint32_t)j];
  if (a != b) return __clzll((long long)(a ^ b));
  return 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
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
  if (threadIdx.x == 0) W.odepth[o] = 0;
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
// a time; a key's slot is the first slot of its (digit, tile), plus the keys
// of its digit placed by earlier rounds, by lower waves of this round and by
// lower lanes of its wave (lanes of equal digit found by ballots over the
// digit's bits).  hoff == nullptr: the first slots are computed here from the
// raw counts (all digits' totals, scanned, plus this digit's count in the
// earlier tiles).
__global__ __launch_bounds__(kSortThreads) void k_lbvh_scatter(const uint64_t* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                               uint32_t n, int shift, const uint32_t* __restrict__ hist,
                                                               const uint32_t* __restrict__ hoff, uint32_t tiles) {
  constexpr int kWaves = kSortThreads / 64;
  __shared__ uint32_t run[kDigits];
  __shared__ uint32_t wc[kWaves][kDigits];
  const uint32_t tid = threadIdx.x, w = tid >> 6;
  if (hoff) {
    run[tid] = hoff[tid * tiles + blockIdx.x];
  } else {
    uint32_t tot = 0, mine = 0;
    for (uint32_t t = 0; t < tiles; ++t) {
      const uint32_t c = hist[tid * tiles + t];
      tot += c;
      mine += t < blockIdx.x ? c : 0u;
    }
    uint32_t x = tot;  // inclusive scan of the digit totals: waves, then wave sums
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if ((int)lane_of() >= o) x += y;
    }
    if (lane_of() == 63) wc[0][w] = x;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t q = 0; q < w; ++q) before += wc[0][q];
    run[tid] = before + x - tot + mine;
  }
  const uint32_t base = blockIdx.x * kSortTile;
  for (int s = 0; s < kSortItems; ++s) {
    __syncthreads();
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

// level 0 of the pyramid (padded triangle boxes in sorted order, or in record
// order when val is null) and the levels 1..kLowLevels of each aligned
// 256-position block
__global__ __launch_bounds__(kBlock) void k_lbvh_leaves(const SceneDev* __restrict__ scenes, LbvhWork W,
                                                        const uint32_t* __restrict__ val) {
  __shared__ float3 slo[kBlock], shi[kBlock];
  const SceneDev& S = scenes[0];
  const uint32_t n = W.n_dyn;
  const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
  Box b = empty_box();
  if (g < n) {
    b = tri_box(S.tris[S.n_static + (val ? val[g] : g)]);
    pyr_put(W.pyr, g, b);
  }
  uint32_t off = 0, m = n;
  for (int l = 1; l <= kLowLevels; ++l) {
    off += m;
    m = (m + 1) / 2;
    slo[threadIdx.x] = b.lo;
    shi[threadIdx.x] = b.hi;
    __syncthreads();
    const uint32_t cnt = (uint32_t)kBlock >> l;
    if (threadIdx.x < cnt) {
      const uint32_t i = 2 * threadIdx.x;
      b = join(Box{slo[i], shi[i]}, Box{slo[i + 1], shi[i + 1]});
      const uint32_t k = (blockIdx.x * kBlock >> l) + threadIdx.x;
      if (k < m) pyr_put(W.pyr, off + k, b);
    }
    __syncthreads();
  }
}

// the pyramid levels above kLowLevels, one workgroup
__global__ __launch_bounds__(1024) void k_lbvh_pyramid(LbvhWork W) {
  const uint32_t n = W.n_dyn;
  uint32_t off = pyr_level(n, kLowLevels), m = (n + (1u << kLowLevels) - 1) >> kLowLevels;
  while (m > 1) {
    const uint32_t up = (m + 1) / 2;
    for (uint32_t k = threadIdx.x; k < up; k += blockDim.x) {
      Box b = pyr_get(W.pyr, off + 2 * k);
      if (2 * k + 1 < m) b = join(b, pyr_get(W.pyr, off + 2 * k + 1));
      pyr_put(W.pyr, off + m + k, b);
    }
    __syncthreads();
    off += m;
    m = up;
  }
}

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
  const int first = min(i, j), last = max(i, j);
  const uint32_t node = ob.lbvh_base + (uint32_t)i;
  int32_t ch[2];
  for (int side = 0; side < 2; ++side) {
    const int c = split + side;
    const bool leaf = side == 0 ? first == c : last == c;
    if (leaf) {
      ch[side] = leaf_code(S.n_static + val[start + (uint32_t)c], 1);
      W.parent_leaf[start + (uint32_t)c] = (int32_t)node;
    } else {
      ch[side] = (int32_t)(ob.lbvh_base + (uint32_t)c);
      W.parent_node[ob.lbvh_base + (uint32_t)c - W.first_node] = (int32_t)node;
    }
  }
  const Box b0 = range_box(W.pyr, W.n_dyn, start + (uint32_t)first, start + (uint32_t)split + 1);
  const Box b1 = range_box(W.pyr, W.n_dyn, start + (uint32_t)split + 1, start + (uint32_t)last + 1);
  Node& nd = S.nodes[node];
  nd.a = make_float4(b0.lo.x, b0.lo.y, b0.lo.z, b0.hi.x);
  nd.b = make_float4(b0.hi.y, b0.hi.z, b1.lo.x, b1.lo.y);
  nd.c = make_float4(b1.lo.z, b1.hi.x, b1.hi.y, b1.hi.z);
  nd.d = make_int4(ch[0], ch[1], -1, 0);
  if (i == 0) W.parent_node[node - W.first_node] = -1;
}

// depth of every leaf (its internal ancestors), maximum per object
__global__ __launch_bounds__(kBlock) void k_lbvh_depth(const SceneDev* __restrict__ scenes, LbvhWork W,
                                                       const uint64_t* __restrict__ key) {
  const SceneDev& S = scenes[0];
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = g < W.n_dyn;
  uint32_t o = 0, depth = 0;
  if (valid) {
    o = (uint32_t)(key[g] >> 30);
    // every non-root node has one parent and the root none, so the climb
    // ends at the root; the step bound (above any radix tree's depth over
    // 2^28 triangles) only keeps a damaged tree from looping
    if (S.objs[o].n_tris > 1)
      for (int32_t p = W.parent_leaf[g]; p >= 0 && depth < kDepthGuard; p = W.parent_node[(uint32_t)p - W.first_node])
        ++depth;
  }
  // one atomic per wave when the wave's leaves share an object
  const uint64_t act = __ballot(valid);
  if (!act) return;
  const uint32_t lead = (uint32_t)__ffsll((long long)act) - 1u;
  const uint32_t o0 = __shfl(o, (int)lead, 64);
  if (__ballot(valid && o != o0) == 0) {
    uint32_t m = valid ? depth : 0u;
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor(m, off, 64));
    if (lane_of() == lead) atomicMax(&W.odepth[o0], m);
  } else if (valid) {
    atomicMax(&W.odepth[o], depth);
  }
}

__global__ void k_lbvh_finish(SceneDev* __restrict__ scenes, LbvhWork W, const uint32_t* __restrict__ val,
                              uint32_t max_depth) {
  SceneDev& S = scenes[0];
  ObjDev* objs = const_cast<ObjDev*>(S.objs);
  const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= S.n_obj) return;
  const ObjDev ob = S.objs[o];
  Box b;
  int32_t root;
  if (ob.n_tris == 1) {
    root = leaf_code(S.n_static + val[ob.tri_base], 1);
    b = tri_box(S.tris[leaf_first(root)]);
  } else {
    // the rebuilt tree replaces the refit topology only within the depth the
    // traversal stacks were sized for
    if (W.odepth[o] > max_depth) return;
    root = (int32_t)ob.lbvh_base;
    b = range_box(W.pyr, W.n_dyn, ob.tri_base, ob.tri_base + ob.n_tris);
  }
  S.obj_aabb[6 * o + 0] = b.lo.x;
  S.obj_aabb[6 * o + 1] = b.lo.y;
  S.obj_aabb[6 * o + 2] = b.lo.z;
  S.obj_aabb[6 * o + 3] = b.hi.x;
  S.obj_aabb[6 * o + 4] = b.hi.y;
  S.obj_aabb[6 * o + 5] = b.hi.z;
  objs[o].root = root;
}

// Per-frame refit of the upload-time topologies of the moved objects: every
// node's two child boxes are unions over the children's leaf-order record
// ranges, read from the pyramid over the records (a subtree holds a
// contiguous run of the leaf order), so no node waits for its children.
// The unions equal those of a level-by-level refit bit for bit: the padding
// is monotone, so the padded box of a union is the union of padded boxes.
__global__ __launch_bounds__(kBlock) void k_refit_nodes(SceneDev* __restrict__ scenes, LbvhWork W) {
  SceneDev& S = scenes[0];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n_obj_nodes || !S.obj_moved[S.dspan_obj[i]]) return;
  const uint4 r = S.dspan[i];
  const Box b0 = range_box(W.pyr, W.n_dyn, r.x, r.y), b1 = range_box(W.pyr, W.n_dyn, r.z, r.w);
  Node& nd = S.nodes[S.obj_node_first + i];
  nd.a = make_float4(b0.lo.x, b0.lo.y, b0.lo.z, b0.hi.x);
  nd.b = make_float4(b0.hi.y, b0.hi.z, b1.lo.x, b1.lo.y);
  nd.c = make_float4(b1.lo.z, b1.hi.x, b1.hi.y, b1.hi.z);
}

// each moved object's box (the union of its records) and its refit topology
// as its current hierarchy
__global__ void k_refit_objects(SceneDev* __restrict__ scenes, LbvhWork W) {
  SceneDev& S = scenes[0];
  ObjDev* objs = const_cast<ObjDev*>(S.objs);
  const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= S.n_obj || !S.obj_moved[o]) return;
  const ObjDev ob = S.objs[o];
  const Box b = range_box(W.pyr, W.n_dyn, ob.tri_base, ob.tri_base + ob.n_tris);
  S.obj_aabb[6 * o + 0] = b.lo.x;
  S.obj_aabb[6 * o + 1] = b.lo.y;
  S.obj_aabb[6 * o + 2] = b.lo.z;
  S.obj_aabb[6 * o + 3] = b.hi.x;
  S.obj_aabb[6 * o + 4] = b.hi.y;
  S.obj_aabb[6 * o + 5] = b.hi.z;
  objs[o].root = ob.sah_root;
}

hipError_t launch_refit_objects(SceneDev* scenes, LbvhWork W, uint32_t n_obj, uint32_t n_obj_nodes, hipStream_t s) {
  if (!W.n_dyn || !n_obj) return hipSuccess;
  const uint32_t nb = (W.n_dyn + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_lbvh_leaves, dim3(nb), dim3(kBlock), 0, s, scenes, W, nullptr);
  if (W.n_dyn > (1u << kLowLevels)) hipLaunchKernelGGL(k_lbvh_pyramid, dim3(1), dim3(1024), 0, s, W);
  if (n_obj_nodes)
    hipLaunchKernelGGL(k_refit_nodes, dim3((n_obj_nodes + kBlock - 1) / kBlock), dim3(kBlock), 0, s, scenes, W);
  hipLaunchKernelGGL(k_refit_objects, dim3((n_obj + 63) / 64), dim3(64), 0, s, scenes, W);
  return hipGetLastError();
}

uint32_t lbvh_sort_tiles(uint32_t n_dyn) { return (n_dyn + kSortTile - 1) / kSortTile; }

// the leaf kernel writes levels 1..kLowLevels even where the pyramid has
// fewer levels (their entries past the top are never read)
uint32_t lbvh_pyramid_entries(uint32_t n_dyn) {
  return std::max(pyr_entries(n_dyn), pyr_level(n_dyn, kLowLevels + 1));
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
    const uint32_t* hoff = nullptr;
    if (tiles > kFusedTiles) {
      hipError_t e = launch_scan(W.hist, W.hoff, kDigits * tiles, W.htotal, W.scan_tmp, s);
      if (e != hipSuccess) return e;
      hoff = W.hoff;
    }
    hipLaunchKernelGGL(k_lbvh_scatter, dim3(tiles), dim3(kSortThreads), 0, s, W.key[src], W.val[src], W.key[src ^ 1],
                       W.val[src ^ 1], W.n_dyn, shift, W.hist, hoff, tiles);
    src ^= 1;
  }
  hipLaunchKernelGGL(k_lbvh_leaves, dim3(nb), dim3(kBlock), 0, s, scenes, W, W.val[src]);
  if (W.n_dyn > (1u << kLowLevels)) hipLaunchKernelGGL(k_lbvh_pyramid, dim3(1), dim3(1024), 0, s, W);
  hipLaunchKernelGGL(k_lbvh_nodes, dim3(nb), dim3(kBlock), 0, s, scenes, W, W.key[src], W.val[src]);
  hipLaunchKernelGGL(k_lbvh_depth, dim3(nb), dim3(kBlock), 0, s, scenes, W, W.key[src]);
  hipLaunchKernelGGL(k_lbvh_finish, dim3((n_obj + 63) / 64), dim3(64), 0, s, scenes, W, W.val[src], max_depth);
  return hipGetLastError();
}

}  // namespace pv
