// Host side of the C-ABI: contexts, scene upload with host-built hierarchy
// topology, scratch reservation and the per-frame calls.  Every public
// function validates its arguments before enqueuing anything and never lets a
// C++ exception escape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pv_device.h"
#include "pv_launch.h"

// Fixed device scratch of pv_compact_photons_noalloc: the photon counts per
// (bounce row, path block), their exclusive offsets and the scan's tile sums.
// Each device holds its own copy until the process ends.  Host code never
// uses this name as an address: it takes the current device's address from
// hipGetSymbolAddress (fixed_scratch below) and passes that to the kernels.
constexpr uint32_t kFixedScratchWords = (1u << 20) / 4;  // 1 MiB
static __device__ __align__(256) uint32_t scratch[kFixedScratchWords];

using pv::LeafRec;
using pv::LightDev;
using pv::Node;
using pv::ObjDev;
using pv::SceneDev;
using pv::Tri;

namespace {

thread_local std::string g_create_error;

struct Alloc {
  std::vector<void*> ptrs;
  ~Alloc() { release(); }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

}  // namespace

struct pv_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  uint32_t* fixed_scratch = nullptr;  // this device's copy of 'scratch'

  int n_cu = 256;
  std::string err;
  // scene
  bool uploaded = false, frame_started = false;
  Alloc scene_mem;
  SceneDev hs{};               // host image of the descriptor
  SceneDev* d_scene = nullptr; // device descriptor (one entry)
  uint32_t* d_state = nullptr; // first-frame flag
  uint2* d_obj_tiles = nullptr;  // (scene, object) for the object update kernel
  uint32_t n_obj_tiles = 0;
  uint2* d_xf_tiles = nullptr;   // (scene << 8 | object, first triangle) for the transform kernel
  uint32_t n_xf_tiles = 0;
  const float** d_in_ptrs = nullptr;  // [2]: object / light transform inputs of the frame
  // transforms of the next frame, written sparsely by pv_update_transforms /
  // pv_update_lights (and densely by pv_frame_begin); a pending update begins
  // the frame at the next call that reads the scene
  float *d_obj_staged = nullptr, *d_light_staged = nullptr;
  bool xf_pending = false;
  uint32_t n_materials = 0, n_lights = 0, n_objects = 0;
  std::vector<uint32_t> h_obj_tris;  // triangles per object
  uint32_t stack_entries = 2;  // traversal stack per lane: whole-scene queries
  uint32_t stack_moved = 2;    // traversal stack per lane: queries against the moved objects
  // deepest leaves: static world, upload-time object topologies, rebuilt
  // object hierarchies (bound), whole-scene top-level tree
  uint32_t static_depth = 0, obj_depth = 0, lbvh_depth = 0, top_depth = 0;
  pv::LbvhWork lw{};          // scratch of the per-frame object rebuild
  bool object_rebuild = false;  // PV_TUNE_OBJECT_REBUILD
  bool verify_boxes = false;    // pv_set_verify_mode
  int32_t energy_test = 0;      // pv_set_energy_test
  bool point_lights = false;    // a light of zero extent: verification walks the whole scene
  bool lbvh_used = false;       // a rebuilt hierarchy may be current: stacks sized for it
  std::vector<uint32_t> h_light_paths;  // filled at binding
  // scratch
  bool reserved = false;
  Alloc res_mem;
  uint32_t max_paths = 0, max_bounces = 0, max_blocks = 0;
  uint2* d_path_tiles = nullptr;
  uint32_t *d_block_cnt = nullptr, *d_offsets = nullptr, *d_queue = nullptr, *d_qcount = nullptr,
           *d_pcounts = nullptr, *d_poffsets = nullptr, *d_gbase = nullptr,
           *d_scan_tmp = nullptr;
  float* d_partial = nullptr;
  uint32_t* d_scan_tmp_c = nullptr;  // scan scratch of the overlapped photon compaction
  // overlapped compaction (pv_compact_photons_async): the event its stream
  // records when done, waited for by the next work that conflicts with it
  hipEvent_t ev_store = nullptr, ev_compact = nullptr;
  bool compact_pending = false;
  pv::VerifyWork vw{};  // verification task lists
  pv::OrderWork ow{};   // re-trace work order
  // distribution maps (pv_set_distribution_map)
  bool dm_enabled = false;
  uint32_t dm_cells = 0;  // cells of all lights
  Alloc dm_mem;
  pv::DmWork dw{};
  // tuning (pv_set_tuning / pv_autotune)
  int retrace_variant = 0;
  // defaults: the settings the autotuner picks on the 3M-path, 380k-triangle
  // interior (twice the workgroups that fit at once: the later ones take
  // what is left of the dealt work lists)
  int retrace_blocks_per_cu = 8;
  int walk_min_active = 40;  // a wave's re-trace walk yields once fewer lanes are still walking
  int verify_blocks_per_cu = 8;  // persistent verification traversal workgroups per compute unit
  int verify_min_active = 16;    // yield threshold of the verification walks
  float tune_report[7] = {0, 0, 0, 0, 0, 0, 0};  // pv_autotune_report
  // bound store
  bool bound = false;
  bool counts_ready = false;   // per-block replace counts written by verify
  bool queue_stale = false;    // verify ran after the last queue build
  pv_path_store bstore{};
};

struct pv_batch {
  pv_ctx* owner = nullptr;  // contexts[0]: stream and error message
  hipStream_t stream = nullptr;      // the owner's stream (the caller's ordering)
  hipStream_t cap_stream = nullptr;  // the batch's own stream: graphs cannot be captured on the null stream
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  uint32_t n = 0;
  Alloc mem;
  SceneDev* d_scenes = nullptr;
  uint2 *d_path_tiles = nullptr, *d_obj_tiles = nullptr, *d_xf_tiles = nullptr;
  uint32_t n_path_tiles = 0, n_obj_tiles = 0, n_xf_tiles = 0;
  uint32_t *d_block_cnt = nullptr, *d_offsets = nullptr, *d_queue = nullptr, *d_qcount = nullptr,
           *d_gbase = nullptr, *d_pcounts = nullptr, *d_poffsets = nullptr, *d_ptotal = nullptr, *d_pbase = nullptr,
           *d_frame = nullptr, *d_scan_tmp = nullptr;
  uint32_t n_counts = 0;
  pv::VerifyWork vw{};
  pv::OrderWork ow{};
  float *d_out_pos = nullptr, *d_out_en = nullptr;
  uint32_t capacity = 0;
  const float** d_obj_in = nullptr;
  const float** d_light_in = nullptr;
  float T = -1.0f;
  uint64_t seed = 0;
  uint32_t retrace_blocks = 0;
  uint32_t stack_entries = 2, stack_moved = 2;  // largest of the scenes'
  uint32_t max_bounces = 1;                      // largest B of the scenes' stores (photon rows)
  bool captured = false;
  pv_stats* captured_stats = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // several frames per launch (pv_batch_frames): frame numbers and per-frame
  // transform pointer tables, and the graph of that many frames
  std::vector<uint32_t> n_obj;  // objects of each scene
  Alloc tab_mem;
  uint32_t tab_frames = 0;      // frames the tables hold
  uint32_t* d_frames = nullptr;
  const float** d_obj_tab = nullptr;
  const float** d_light_tab = nullptr;
  uint32_t multi_k = 0;         // frames of the captured graph (0: none)
  pv_stats* multi_stats = nullptr;
  hipGraph_t multi_graph = nullptr;
  hipGraphExec_t multi_exec = nullptr;
  // distribution maps of the scenes whose context had one when the batch was
  // created (Section 3.1's update after verification, on batch-owned scratch)
  struct Dm {
    uint32_t scene, tile_base, n_tiles, cells, n_lights;
    pv::DmWork D;
  };
  std::vector<Dm> dms;
  ~pv_batch() {
    if (multi_exec) (void)hipGraphExecDestroy(multi_exec);
    if (multi_graph) (void)hipGraphDestroy(multi_graph);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace {

// Device address of 'scratch' on device 'dev', which must be current: looked
// up once per device and kept (every context of a device shares the array).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};

hipError_t fixed_scratch(int dev, uint32_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Layout of the fixed scratch for n = path blocks x bounce rows counts:
// counts [0, a), offsets [a, 2a), scan tile sums [2a, 2a + scan_tmp_words(n))
// with a = n rounded up to 64 words; returns the words it needs.
uint64_t fixed_layout(uint64_t n, uint64_t* a) {
  *a = (n + 63) / 64 * 64;
  return 2 * *a + pv::scan_tmp_words((uint32_t)std::min<uint64_t>(n, 0xFFFFFFFFull));
}

pv_status fail(pv_ctx* c, pv_status code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define CK(call)                                                                                     \
  do {                                                                                               \
    hipError_t e_ = (call);                                                                          \
    if (e_ != hipSuccess) return fail(ctx, PV_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
hipError_t dalloc(Alloc& a, T** out, size_t count) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return e;
  a.ptrs.push_back(p);
  *out = static_cast<T*>(p);
  return hipSuccess;
}

template <typename T>
hipError_t upload(Alloc& a, T** out, const T* src, size_t count, hipStream_t s) {
  hipError_t e = dalloc(a, out, count);
  if (e != hipSuccess || count == 0) return e;
  return hipMemcpyAsync(*out, src, count * sizeof(T), hipMemcpyHostToDevice, s);
}

// ---------------------------------------------------------------------------
// hierarchy topology on the host: 30-bit Morton codes of triangle centroids,
// sorted, split top-down at the highest differing code bit (the binary radix
// tree of the sorted codes; equal codes split at the middle), nodes numbered
// in depth-first order so the left child of an internal node follows it.

uint32_t expand10(uint32_t v) {
  v &= 1023u;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

struct HostBvh {
  std::vector<Node> nodes;
  std::vector<uint32_t> order;   // leaf position -> input triangle
  std::vector<LeafRec> leaves;   // first/parent relative
  std::vector<int32_t> parent;   // per node: parent*2+side or -1
  int32_t root = 0;
  uint32_t max_depth = 0;        // deepest leaf (root = 0)
};

constexpr uint32_t kMaxDepth = (uint32_t)pv::kMaxDepth;
// paths per context or batch: verification tasks carry a path index in 28 bits
constexpr uint32_t kMaxPaths = 1u << 28;

inline uint32_t ceil_log2(uint32_t n) { return n <= 1 ? 0u : 32u - (uint32_t)__builtin_clz(n - 1); }

// Both builders split at the middle of the range once an unbalanced split
// could push a leaf below depth kMaxDepth: a range of cnt items at depth d
// with d + ceil_log2(cnt) <= kMaxDepth keeps that property under a middle
// split, so every leaf stays within the bound (root: ceil_log2(n) <= kMaxDepth).
inline bool must_halve(uint32_t depth, uint32_t cnt) { return depth + ceil_log2(cnt) + 1 > kMaxDepth; }

HostBvh build_topology(const float* v9, uint32_t n, uint32_t leaf_max) {
  HostBvh h;
  std::vector<uint32_t> code(n);
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  std::vector<float> cen(3 * (size_t)n);
  for (uint32_t i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      float c = (v9[9 * (size_t)i + k] + v9[9 * (size_t)i + 3 + k] + v9[9 * (size_t)i + 6 + k]) / 3.0f;
      cen[3 * (size_t)i + k] = c;
      lo[k] = std::min(lo[k], c);
      hi[k] = std::max(hi[k], c);
    }
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
      float ext = hi[k] - lo[k];
      float u = ext > 0 ? (cen[3 * (size_t)i + k] - lo[k]) / ext : 0.5f;
      q[k] = (uint32_t)std::min(1023.0f, std::max(0.0f, u * 1024.0f));
    }
    code[i] = (expand10(q[0]) << 2) | (expand10(q[1]) << 1) | expand10(q[2]);
  }
  h.order.resize(n);
  for (uint32_t i = 0; i < n; ++i) h.order[i] = i;
  std::stable_sort(h.order.begin(), h.order.end(), [&](uint32_t a, uint32_t b) { return code[a] < code[b]; });
  std::vector<uint32_t> sc(n);
  for (uint32_t i = 0; i < n; ++i) sc[i] = code[h.order[i]];

  struct Item {
    uint32_t lo, hi;
    int32_t parent;
    uint32_t side;
    uint32_t depth;
  };
  std::vector<Item> stack;
  stack.push_back({0, n - 1, -1, 0, 0});
  auto set_child = [&](int32_t parent, uint32_t side, int32_t childcode) {
    if (parent < 0)
      h.root = childcode;
    else if (side == 0)
      h.nodes[parent].d.x = childcode;
    else
      h.nodes[parent].d.y = childcode;
  };
  while (!stack.empty()) {
    Item it = stack.back();
    stack.pop_back();
    uint32_t cnt = it.hi - it.lo + 1;
    h.max_depth = std::max(h.max_depth, it.depth);
    if (cnt <= leaf_max) {
      set_child(it.parent, it.side, pv::leaf_code(it.lo, cnt));
      h.leaves.push_back({it.lo, cnt, it.parent, it.side});
      continue;
    }
    uint32_t split;
    if (sc[it.lo] == sc[it.hi] || must_halve(it.depth, cnt)) {
      split = (it.lo + it.hi) / 2;
    } else {
      int bit = 31 - __builtin_clz(sc[it.lo] ^ sc[it.hi]);
      uint32_t a = it.lo + 1, b = it.hi;  // first index with the bit set
      while (a < b) {
        uint32_t m = (a + b) / 2;
        if ((sc[m] >> bit) & 1u)
          b = m;
        else
          a = m + 1;
      }
      split = a - 1;
    }
    int32_t id = (int32_t)h.nodes.size();
    Node nd{};
    nd.d = make_int4(0, 0, it.parent < 0 ? -1 : it.parent * 2 + (int)it.side, 0);
    h.nodes.push_back(nd);
    h.parent.push_back(nd.d.z);
    set_child(it.parent, it.side, id);
    stack.push_back({split + 1, it.hi, id, 1, it.depth + 1});
    stack.push_back({it.lo, split, id, 0, it.depth + 1});
  }
  return h;
}

// Static world: binned surface-area-heuristic split (16 bins per axis) of
// the centroid range, with a leaf of at most 8 triangles when splitting does
// not pay; a median split where the depth bound requires it.
HostBvh build_sah(const float* v9, uint32_t n) {
  HostBvh h;
  constexpr int K = 16;
  constexpr uint32_t kLeafMax = 8, kMinSplit = 2;
  struct Box {
    float lo[3], hi[3];
    void reset() {
      for (int k = 0; k < 3; ++k) {
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
      }
    }
    void grow(const Box& b) {
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], b.lo[k]);
        hi[k] = std::max(hi[k], b.hi[k]);
      }
    }
    float area() const {
      float d[3];
      for (int k = 0; k < 3; ++k) d[k] = std::max(0.0f, hi[k] - lo[k]);
      return d[0] * d[1] + d[1] * d[2] + d[2] * d[0];
    }
  };
  std::vector<Box> tb(n);
  std::vector<float> cen(3 * (size_t)n);
  for (uint32_t i = 0; i < n; ++i) {
    tb[i].reset();
    for (int v = 0; v < 3; ++v)
      for (int k = 0; k < 3; ++k) {
        float x = v9[9 * (size_t)i + 3 * v + k];
        tb[i].lo[k] = std::min(tb[i].lo[k], x);
        tb[i].hi[k] = std::max(tb[i].hi[k], x);
      }
    for (int k = 0; k < 3; ++k) cen[3 * (size_t)i + k] = 0.5f * (tb[i].lo[k] + tb[i].hi[k]);
  }
  h.order.resize(n);
  for (uint32_t i = 0; i < n; ++i) h.order[i] = i;
  struct Item {
    uint32_t lo, hi;  // [lo, hi)
    int32_t parent;
    uint32_t side, depth;
  };
  std::vector<Item> stack;
  stack.push_back({0, n, -1, 0, 0});
  auto set_child = [&](int32_t parent, uint32_t side, int32_t code) {
    if (parent < 0)
      h.root = code;
    else if (side == 0)
      h.nodes[parent].d.x = code;
    else
      h.nodes[parent].d.y = code;
  };
  while (!stack.empty()) {
    Item it = stack.back();
    stack.pop_back();
    uint32_t cnt = it.hi - it.lo;
    h.max_depth = std::max(h.max_depth, it.depth);
    Box nb, cb;
    nb.reset();
    cb.reset();
    for (uint32_t i = it.lo; i < it.hi; ++i) {
      uint32_t t = h.order[i];
      nb.grow(tb[t]);
      Box c;
      for (int k = 0; k < 3; ++k) c.lo[k] = c.hi[k] = cen[3 * (size_t)t + k];
      cb.grow(c);
    }
    uint32_t mid = it.lo;
    bool leaf = cnt < kMinSplit;
    if (!leaf) {
      int best_axis = -1, best_s = 0;
      float best = INFINITY;
      if (!must_halve(it.depth, cnt)) {
        for (int ax = 0; ax < 3; ++ax) {
          float ext = cb.hi[ax] - cb.lo[ax];
          if (!(ext > 0)) continue;
          Box bb[K];
          uint32_t bc[K] = {0};
          for (int b = 0; b < K; ++b) bb[b].reset();
          for (uint32_t i = it.lo; i < it.hi; ++i) {
            uint32_t t = h.order[i];
            int b = std::min(K - 1, (int)((cen[3 * (size_t)t + ax] - cb.lo[ax]) / ext * K));
            bb[b].grow(tb[t]);
            ++bc[b];
          }
          float ra[K];
          uint32_t rc[K];
          Box acc;
          acc.reset();
          uint32_t c = 0;
          for (int b = K - 1; b > 0; --b) {
            acc.grow(bb[b]);
            c += bc[b];
            ra[b] = acc.area();
            rc[b] = c;
          }
          acc.reset();
          c = 0;
          for (int b = 0; b < K - 1; ++b) {
            acc.grow(bb[b]);
            c += bc[b];
            if (c == 0 || rc[b + 1] == 0) continue;
            float cost = acc.area() * c + ra[b + 1] * rc[b + 1];
            if (cost < best) {
              best = cost;
              best_axis = ax;
              best_s = b + 1;
            }
          }
        }
      }
      float leaf_cost = nb.area() * cnt;
      float split_cost = best + nb.area();  // one traversal step plus the children
      if (best_axis >= 0 && (split_cost < leaf_cost || cnt > kLeafMax)) {
        float ext = cb.hi[best_axis] - cb.lo[best_axis];
        auto first = h.order.begin() + it.lo, last = h.order.begin() + it.hi;
        auto m = std::partition(first, last, [&](uint32_t t) {
          int b = std::min(K - 1, (int)((cen[3 * (size_t)t + best_axis] - cb.lo[best_axis]) / ext * K));
          return b < best_s;
        });
        mid = (uint32_t)(m - h.order.begin());
      } else if (cnt <= kLeafMax) {
        leaf = true;
      }
      if (!leaf && (mid == it.lo || mid == it.hi)) {
        // median split along the widest centroid axis
        int ax = 0;
        for (int k = 1; k < 3; ++k)
          if (cb.hi[k] - cb.lo[k] > cb.hi[ax] - cb.lo[ax]) ax = k;
        mid = it.lo + cnt / 2;
        std::nth_element(h.order.begin() + it.lo, h.order.begin() + mid, h.order.begin() + it.hi,
                         [&](uint32_t a, uint32_t b) { return cen[3 * (size_t)a + ax] < cen[3 * (size_t)b + ax]; });
      }
    }
    if (leaf) {
      set_child(it.parent, it.side, pv::leaf_code(it.lo, cnt));
      h.leaves.push_back({it.lo, cnt, it.parent, it.side});
      continue;
    }
    int32_t id = (int32_t)h.nodes.size();
    Node nd{};
    nd.d = make_int4(0, 0, it.parent < 0 ? -1 : it.parent * 2 + (int)it.side, 0);
    h.nodes.push_back(nd);
    h.parent.push_back(nd.d.z);
    set_child(it.parent, it.side, id);
    stack.push_back({mid, it.hi, id, 1, it.depth + 1});
    stack.push_back({it.lo, mid, id, 0, it.depth + 1});
  }
  return h;
}

inline float pad_lo(float x) { return x - (1e-6f + std::fabs(x) * 1e-6f); }
inline float pad_hi(float x) { return x + (1e-6f + std::fabs(x) * 1e-6f); }

// Extra padding of the object-space boxes: a world segment mapped into object
// space in FP32 (inverse transform) is off by a few units of 2^-24 of its
// distance from the object's origin, at most about 4e-6 for coordinates up
// to 10 scene units; 1e-5 keeps every object-space box conservative.
constexpr float kObjSpacePad = 1e-5f;

// child boxes of every node from leaf-order vertices (static world, or an
// object in its own space with 'extra' added to the padding)
void host_boxes(HostBvh& h, const float* v9_leaf_order, float extra = 0.0f) {
  auto leaf_box = [&](int32_t code, float* b) {
    uint32_t f = pv::leaf_first(code), c = pv::leaf_count(code);
    for (int k = 0; k < 3; ++k) {
      b[k] = INFINITY;
      b[3 + k] = -INFINITY;
    }
    for (uint32_t i = f; i < f + c; ++i)
      for (int v = 0; v < 3; ++v)
        for (int k = 0; k < 3; ++k) {
          float x = v9_leaf_order[9 * (size_t)i + 3 * v + k];
          b[k] = std::min(b[k], x);
          b[3 + k] = std::max(b[3 + k], x);
        }
    for (int k = 0; k < 3; ++k) {
      b[k] = pad_lo(b[k]) - extra;
      b[3 + k] = pad_hi(b[3 + k]) + extra;
    }
  };
  std::vector<float> nb(6 * h.nodes.size());
  for (int64_t i = (int64_t)h.nodes.size() - 1; i >= 0; --i) {
    Node& nd = h.nodes[i];
    float cb[2][6];
    int32_t ch[2] = {nd.d.x, nd.d.y};
    for (int s = 0; s < 2; ++s) {
      if (ch[s] < 0)
        leaf_box(ch[s], cb[s]);
      else
        std::memcpy(cb[s], &nb[6 * (size_t)ch[s]], sizeof(cb[s]));
    }
    float* f = reinterpret_cast<float*>(&nd);
    std::memcpy(f, cb[0], 6 * sizeof(float));
    std::memcpy(f + 6, cb[1], 6 * sizeof(float));
    for (int k = 0; k < 3; ++k) {
      nb[6 * i + k] = std::min(cb[0][k], cb[1][k]);
      nb[6 * i + 3 + k] = std::max(cb[0][3 + k], cb[1][3 + k]);
    }
  }
}

bool finite_all(const float* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

std::vector<uint2> make_tiles(uint32_t scene, uint32_t n) {
  std::vector<uint2> t;
  for (uint32_t f = 0; f < n; f += pv::kBlock) t.push_back(make_uint2(scene, f));
  return t;
}

uint32_t path_blocks(uint32_t n) { return (n + pv::kBlock - 1) / pv::kBlock; }

// transform tiles of a scene's objects: (scene << 8 | object, first triangle)
std::vector<uint2> xf_tiles(uint32_t scene, const uint32_t* obj_tris, uint32_t n_objects) {
  std::vector<uint2> t;
  for (uint32_t o = 0; o < n_objects; ++o)
    for (uint32_t f = 0; f < obj_tris[o]; f += pv::kBlock) t.push_back(make_uint2((scene << 8) | o, f));
  return t;
}

// grid of the verification traversal kernel (persistent, grid-stride)
constexpr int kMaxVerifyBlocksPerCu = 32;
uint32_t verify_blocks(const pv_ctx* ctx) { return (uint32_t)(ctx->n_cu * ctx->verify_blocks_per_cu); }
// the largest traversal grid any tuning can pick (sizes the statistics slots)
uint32_t verify_blocks_max(const pv_ctx* ctx) { return (uint32_t)(ctx->n_cu * kMaxVerifyBlocksPerCu); }

// Work that writes what an overlapped compaction reads (the photon rows and
// segment counts, the scene descriptor) or reuses its scratch is ordered
// after it on the context's stream.
pv_status wait_compaction(pv_ctx* ctx) {
  if (!ctx->compact_pending) return PV_OK;
  ctx->compact_pending = false;
  CK(hipStreamWaitEvent(ctx->stream, ctx->ev_compact, 0));
  return PV_OK;
}

pv_status bind_store(pv_ctx* ctx, const pv_path_store* st) {
  if (!ctx->uploaded) return fail(ctx, PV_ERR_STATE, "no scene uploaded");
  if (!ctx->reserved) return fail(ctx, PV_ERR_STATE, "pv_reserve has not been called");
  if (!st) return fail(ctx, PV_ERR_ARG, "store is NULL");
  if (!st->d_pos_hit || !st->d_energy || !st->d_origin || !st->d_info)
    return fail(ctx, PV_ERR_ARG, "store has a NULL array");
  if (st->max_bounces < 1 || st->max_bounces > PV_MAX_BOUNCES)
    return fail(ctx, PV_ERR_ARG, "max_bounces out of range 1..15");
  if (st->stride < st->n_paths || st->stride % 64 != 0)
    return fail(ctx, PV_ERR_ARG, "stride must be >= n_paths and a multiple of 64");
  if (st->n_paths > ctx->max_paths || st->max_bounces > ctx->max_bounces)
    return fail(ctx, PV_ERR_CAPACITY, "store exceeds the reserved size");
  if (((uintptr_t)st->d_pos_hit | (uintptr_t)st->d_energy) & 15u)
    return fail(ctx, PV_ERR_ARG, "pos_hit / energy must be 16-byte aligned");
  if (ctx->bound && std::memcmp(&ctx->bstore, st, sizeof(*st)) == 0) return PV_OK;
  if (pv_status w = wait_compaction(ctx)) return w;
  // light path ranges must cover the store exactly
  uint32_t total = 0;
  for (uint32_t l = 0; l < ctx->n_lights; ++l) total += ctx->h_light_paths[l];
  if (total != st->n_paths) return fail(ctx, PV_ERR_ARG, "light path counts do not add up to n_paths");
  ctx->hs.pos = static_cast<float4*>(st->d_pos_hit);
  ctx->hs.energy = static_cast<float4*>(st->d_energy);
  ctx->hs.origin = st->d_origin;
  ctx->hs.info = st->d_info;
  ctx->hs.stride = st->stride;
  ctx->hs.n_paths = st->n_paths;
  ctx->hs.B = st->max_bounces;
  ctx->hs.n_blocks = path_blocks(st->n_paths);
  ctx->hs.count_base = 0;
  ctx->hs.gpath_base = 0;
  ctx->hs.tile_base = 0;
  ctx->hs.task_base = 0;
  CK(hipMemcpyAsync(ctx->d_scene, &ctx->hs, sizeof(SceneDev), hipMemcpyHostToDevice, ctx->stream));
  uint32_t gb[2] = {0, st->n_paths};
  CK(hipMemcpyAsync(ctx->d_gbase, gb, sizeof(gb), hipMemcpyHostToDevice, ctx->stream));
  ctx->bstore = *st;
  ctx->bound = true;
  ctx->counts_ready = false;
  return PV_OK;
}

}  // namespace

// Traversal stack entries per lane: the top-level tree above the deepest
// hierarchy a query can enter (a rebuilt object hierarchy once one may be
// current: objects that did not move since keep theirs).
static void size_stacks(pv_ctx* ctx) {
  const uint32_t od = ctx->lbvh_used ? std::max(ctx->obj_depth, ctx->lbvh_depth) : ctx->obj_depth;
  ctx->stack_entries = pv::stack_entries(ctx->top_depth, std::max(ctx->static_depth, od));
  ctx->stack_moved = pv::stack_entries(ceil_log2(ctx->n_objects), od);
  // a point light's visibility test walks the whole scene during verification
  if (ctx->point_lights) ctx->stack_moved = std::max(ctx->stack_moved, ctx->stack_entries);
}

// Invariants of a hierarchy over leaf-order vertices: leaves partition the
// triangles, every stored child box contains its subtree, depth <= bound.
bool check_hierarchy(const HostBvh& h, const float* v9_leaf_order, uint32_t n) {
  std::vector<uint8_t> seen(n, 0);
  struct It {
    int32_t code;
    float box[6];
  };
  std::vector<It> st;
  float inf_box[6] = {-INFINITY, -INFINITY, -INFINITY, INFINITY, INFINITY, INFINITY};
  It r;
  r.code = h.root;
  std::memcpy(r.box, inf_box, sizeof(inf_box));
  st.push_back(r);
  auto inside = [](const float* inner_lo_hi, const float* outer) {
    for (int k = 0; k < 3; ++k)
      if (inner_lo_hi[k] < outer[k] || inner_lo_hi[3 + k] > outer[3 + k]) return false;
    return true;
  };
  while (!st.empty()) {
    It it = st.back();
    st.pop_back();
    if (it.code < 0) {
      uint32_t f = pv::leaf_first(it.code), c = pv::leaf_count(it.code);
      for (uint32_t i = f; i < f + c; ++i) {
        if (i >= n || seen[i]) return false;
        seen[i] = 1;
        for (int v = 0; v < 3; ++v) {
          const float* x = v9_leaf_order + 9 * (size_t)i + 3 * v;
          float b[6] = {x[0], x[1], x[2], x[0], x[1], x[2]};
          if (!inside(b, it.box)) return false;
        }
      }
      continue;
    }
    if ((size_t)it.code >= h.nodes.size()) return false;
    const Node& nd = h.nodes[it.code];
    const float* f = reinterpret_cast<const float*>(&nd);
    for (int side = 0; side < 2; ++side) {
      It ch;
      ch.code = side ? nd.d.y : nd.d.x;
      std::memcpy(ch.box, f + 6 * side, 6 * sizeof(float));
      if (!inside(ch.box, it.box)) return false;
      st.push_back(ch);
    }
  }
  for (uint32_t i = 0; i < n; ++i)
    if (!seen[i]) return false;
  return true;
}

// ===========================================================================
extern "C" {

pv_status pv_hierarchy_info(const float* h_verts, uint32_t n, int32_t kind, uint32_t* out) {
  if (!h_verts || !out || n == 0 || (kind != 0 && kind != 1)) return PV_ERR_ARG;
  try {
    HostBvh h = kind == 0 ? build_sah(h_verts, n) : build_topology(h_verts, n, 2);
    std::vector<float> v9(9 * (size_t)n);
    for (uint32_t i = 0; i < n; ++i) std::memcpy(&v9[9 * (size_t)i], h_verts + 9 * (size_t)h.order[i], 36);
    host_boxes(h, v9.data());
    out[0] = (uint32_t)h.nodes.size();
    out[1] = (uint32_t)h.leaves.size();
    out[2] = h.max_depth;
    out[3] = (check_hierarchy(h, v9.data(), n) && h.max_depth <= kMaxDepth) ? 1u : 0u;
    return PV_OK;
  } catch (...) {
    return PV_ERR_OOM;
  }
}


const char* pv_version(void) { return "pv-mi355x 0.1 (gfx950)"; }

uint64_t pv_store_bytes(uint64_t n_paths, uint32_t max_bounces) {
  return n_paths * (32ull * max_bounces + 4ull + 12ull);
}

uint32_t pv_info_pack(uint32_t cell, uint32_t nseg, uint32_t start, uint32_t replace, uint32_t reuse) {
  return pv::info_pack(cell, nseg, start, replace, reuse);
}

void pv_info_unpack(uint32_t w, uint32_t* cell, uint32_t* nseg, uint32_t* start, uint32_t* replace,
                    uint32_t* reuse) {
  if (cell) *cell = pv::info_cell(w);
  if (nseg) *nseg = pv::info_nseg(w);
  if (start) *start = pv::info_start(w);
  if (replace) *replace = pv::info_replace(w);
  if (reuse) *reuse = pv::info_reuse(w);
}

const char* pv_last_error(const pv_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

pv_status pv_create(pv_ctx** out, void* hip_stream) {
  if (!out) {
    g_create_error = "out is NULL";
    return PV_ERR_ARG;
  }
  *out = nullptr;
  pv_ctx* ctx = new (std::nothrow) pv_ctx();
  if (!ctx) {
    g_create_error = "host allocation failed";
    return PV_ERR_OOM;
  }
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipGetDevice(&ctx->device);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, ctx->device);
  if (e != hipSuccess) {
    g_create_error = std::string("no HIP device: ") + hipGetErrorString(e);
    delete ctx;
    return PV_ERR_HIP;
  }
  ctx->n_cu = prop.multiProcessorCount;
  // the library's fixed scratch on this (current) device
  if ((e = fixed_scratch(ctx->device, &ctx->fixed_scratch)) != hipSuccess) {
    g_create_error = std::string("fixed scratch: hipGetSymbolAddress: ") + hipGetErrorString(e);
    delete ctx;
    return PV_ERR_HIP;
  }
  *out = ctx;
  return PV_OK;
}

pv_status pv_create_config(pv_ctx** out, const pv_config* cfg, void* hip_stream) {
  if (!cfg) {
    if (out) *out = nullptr;
    g_create_error = "cfg is NULL";
    return PV_ERR_ARG;
  }
  if (cfg->verify_mode != PV_VERIFY_TRIANGLES && cfg->verify_mode != PV_VERIFY_BOXES) {
    if (out) *out = nullptr;
    g_create_error = "verify_mode out of range";
    return PV_ERR_ARG;
  }
  pv_status st = pv_create(out, hip_stream);
  if (st) return st;
  pv_ctx* ctx = *out;
  if (!st) st = pv_set_verify_mode(ctx, cfg->verify_mode);
  if (!st) st = pv_set_tuning(ctx, PV_TUNE_OBJECT_REBUILD, cfg->object_rebuild);
  if (!st && cfg->max_paths) st = pv_reserve(ctx, cfg->max_paths, cfg->max_bounces);
  if (st) {
    g_create_error = ctx->err;
    pv_destroy(ctx);
    *out = nullptr;
  }
  return st;
}

void pv_destroy(pv_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ev_compact) (void)hipEventSynchronize(ctx->ev_compact);
  if (ctx->ev_store) (void)hipEventDestroy(ctx->ev_store);
  if (ctx->ev_compact) (void)hipEventDestroy(ctx->ev_compact);
  delete ctx;
}

pv_status pv_upload_scene(pv_ctx* ctx, const pv_scene_desc* d) {
  if (!ctx) return PV_ERR_ARG;
  try {
    if (!d) return fail(ctx, PV_ERR_ARG, "desc is NULL");
    if (d->n_objects > PV_MAX_OBJECTS) return fail(ctx, PV_ERR_ARG, "too many dynamic objects");
    if (d->n_lights < 1 || d->n_lights > PV_MAX_LIGHTS) return fail(ctx, PV_ERR_ARG, "n_lights out of range 1..8");
    if (d->n_materials < 1 || !d->h_albedo) return fail(ctx, PV_ERR_ARG, "no materials");
    if (d->n_static && (!d->h_static_verts || !d->h_static_mat)) return fail(ctx, PV_ERR_ARG, "static arrays NULL");
    if (!d->h_light_half || !d->h_light_power) return fail(ctx, PV_ERR_ARG, "light arrays NULL");
    for (uint32_t l = 0; l < d->n_lights; ++l) {
      const float hu = d->h_light_half[2 * l], hv = d->h_light_half[2 * l + 1];
      if (!((hu > 0.0f && hv > 0.0f) || (hu == 0.0f && hv == 0.0f)))
        return fail(ctx, PV_ERR_ARG, "light half extents must both be positive (rectangle) or both 0 (point light)");
      const int32_t kind = d->h_light_kind ? d->h_light_kind[l] : PV_LIGHT_AREA;
      if (kind != PV_LIGHT_AREA) {
        if (kind != PV_LIGHT_SPOT && kind != PV_LIGHT_CAMERA) return fail(ctx, PV_ERR_ARG, "unknown light kind");
        if (hu != 0.0f || hv != 0.0f) return fail(ctx, PV_ERR_ARG, "spot lights and cameras have zero extents");
        if (!d->h_light_param) return fail(ctx, PV_ERR_ARG, "light parameters NULL");
        const float p0 = d->h_light_param[2 * l], p1 = d->h_light_param[2 * l + 1];
        if (kind == PV_LIGHT_SPOT && !(p0 >= 0.0f && p0 < 1.0f))
          return fail(ctx, PV_ERR_ARG, "spot cone cosine out of range [0, 1)");
        if (kind == PV_LIGHT_CAMERA && !(p0 > 0.0f && p1 > 0.0f && std::isfinite(p0) && std::isfinite(p1)))
          return fail(ctx, PV_ERR_ARG, "camera field-of-view tangents must be positive");
      }
    }
    if (!(d->eps_end > 0.0f) || !(d->eps_close >= 0.0f)) return fail(ctx, PV_ERR_ARG, "bad tolerances");
    uint64_t n_dyn = 0;
    for (uint32_t o = 0; o < d->n_objects; ++o) {
      if (!d->h_obj_tris || d->h_obj_tris[o] == 0) return fail(ctx, PV_ERR_ARG, "object without triangles");
      n_dyn += d->h_obj_tris[o];
    }
    if (n_dyn && (!d->h_obj_verts || !d->h_obj_mat)) return fail(ctx, PV_ERR_ARG, "object arrays NULL");
    if ((uint64_t)d->n_static + n_dyn >= (1ull << 28)) return fail(ctx, PV_ERR_ARG, "too many triangles");
    if (d->n_static + n_dyn == 0) return fail(ctx, PV_ERR_ARG, "empty scene");
    if (!finite_all(d->h_static_verts, 9 * (size_t)d->n_static) || !finite_all(d->h_obj_verts, 9 * n_dyn))
      return fail(ctx, PV_ERR_ARG, "non-finite vertex");
    for (uint64_t i = 0; i < d->n_static; ++i)
      if (d->h_static_mat[i] >= d->n_materials) return fail(ctx, PV_ERR_ARG, "static material id out of range");
    for (uint64_t i = 0; i < n_dyn; ++i)
      if (d->h_obj_mat[i] >= d->n_materials) return fail(ctx, PV_ERR_ARG, "object material id out of range");

    if (pv_status w = wait_compaction(ctx)) return w;
    CK(hipStreamSynchronize(ctx->stream));
    ctx->scene_mem.release();
    ctx->uploaded = ctx->frame_started = ctx->bound = false;
    ctx->dm_mem.release();  // a new scene has no distribution map
    ctx->dm_enabled = false;
    ctx->dm_cells = 0;
    hipStream_t s = ctx->stream;
    Alloc& A = ctx->scene_mem;
    SceneDev hs{};
    const uint32_t S = d->n_static;
    const uint32_t T = S + (uint32_t)n_dyn;

    // materials by global triangle id
    std::vector<uint32_t> tri_mat(T);
    for (uint32_t i = 0; i < S; ++i) tri_mat[i] = d->h_static_mat[i];
    for (uint64_t i = 0; i < n_dyn; ++i) tri_mat[S + i] = d->h_obj_mat[i];
    uint32_t* d_tri_mat;
    CK(upload(A, &d_tri_mat, tri_mat.data(), T, s));
    float* d_albedo;
    CK(upload(A, &d_albedo, d->h_albedo, 3 * (size_t)d->n_materials, s));
    hs.tri_mat = d_tri_mat;
    hs.albedo = d_albedo;
    hs.n_tris_total = T;

    // static world: topology + boxes on the host
    std::vector<Node> nodes;  // static, then objects, then the top-level trees
    std::vector<Tri> stris;
    hs.n_static = S;
    hs.sroot = pv::kRootNone;
    uint32_t depth = 0, obj_depth = 0;  // deepest leaf: all hierarchies, object hierarchies
    for (int k = 0; k < 3; ++k) {
      hs.sbox[k] = INFINITY;
      hs.sbox[3 + k] = -INFINITY;
    }
    if (S) {
      HostBvh hb = build_sah(d->h_static_verts, S);
      std::vector<float> v9(9 * (size_t)S);
      stris.resize(S);
      for (uint32_t i = 0; i < S; ++i) {
        const float* v = d->h_static_verts + 9 * (size_t)hb.order[i];
        std::memcpy(&v9[9 * (size_t)i], v, 9 * sizeof(float));
        uint32_t gid = hb.order[i];
        stris[i].t0 = make_float4(v[0], v[1], v[2], 0.0f);
        stris[i].t1 = make_float4(v[3], v[4], v[5], 0.0f);
        stris[i].t2 = make_float4(v[6], v[7], v[8], 0.0f);
        std::memcpy(&stris[i].t0.w, &gid, 4);
        std::memcpy(&stris[i].t1.w, &tri_mat[gid], 4);
      }
      if (hb.max_depth > kMaxDepth) return fail(ctx, PV_ERR_CAPACITY, "static hierarchy too deep");
      depth = std::max(depth, hb.max_depth);
      host_boxes(hb, v9.data());
      nodes = std::move(hb.nodes);
      hs.sroot = hb.root;
      for (size_t i = 0; i < v9.size(); ++i) {
        const int k = (int)(i % 3);
        hs.sbox[k] = std::min(hs.sbox[k], v9[i]);
        hs.sbox[3 + k] = std::max(hs.sbox[3 + k], v9[i]);
      }
      for (int k = 0; k < 3; ++k) {
        hs.sbox[k] = pad_lo(hs.sbox[k]);
        hs.sbox[3 + k] = pad_hi(hs.sbox[3 + k]);
      }
    }

    const uint32_t static_depth = depth;
    // dynamic objects: topology in object space, boxes refit per frame
    std::vector<ObjDev> objs(d->n_objects);
    std::vector<float> dlocal(9 * n_dyn);
    std::vector<uint32_t> dgid(n_dyn);
    std::vector<uint32_t> level_nodes, level_off;
    std::vector<uint4> dspan;          // per object node: its children's record ranges
    std::vector<uint32_t> dspan_obj;   // and its object
    std::vector<Node> onodes;          // the objects' topologies with object-space boxes
    const uint32_t obj_node_first = (uint32_t)nodes.size();
    uint32_t tri_base = 0, gbase = S;
    for (uint32_t o = 0; o < d->n_objects; ++o) {
      uint32_t n = d->h_obj_tris[o];
      const float* v = d->h_obj_verts + 9 * (size_t)tri_base;
      HostBvh hb = build_sah(v, n);  // topology in object space, boxes refit each frame
      if (hb.max_depth > kMaxDepth) return fail(ctx, PV_ERR_CAPACITY, "object hierarchy too deep");
      depth = std::max(depth, hb.max_depth);
      obj_depth = std::max(obj_depth, hb.max_depth);
      uint32_t node_base = (uint32_t)nodes.size();
      auto rebase = [&](int32_t c) {
        return c >= 0 ? c + (int32_t)node_base
                      : pv::leaf_code(pv::leaf_first(c) + S + tri_base, pv::leaf_count(c));
      };
      // depth of every internal node (parents precede children in the node order)
      std::vector<uint32_t> depth(hb.nodes.size(), 0);
      uint32_t maxd = 0;
      for (size_t i = 0; i < hb.nodes.size(); ++i) {
        int32_t par = hb.parent[i];
        depth[i] = par < 0 ? 0 : depth[par >> 1] + 1;
        maxd = std::max(maxd, depth[i]);
      }
      ObjDev& ob = objs[o];
      ob.lvl_base = (uint32_t)level_off.size();
      ob.n_levels = hb.nodes.empty() ? 0 : maxd + 1;
      for (int64_t lv = (int64_t)maxd; lv >= 0 && !hb.nodes.empty(); --lv) {
        level_off.push_back((uint32_t)level_nodes.size());
        for (size_t i = 0; i < hb.nodes.size(); ++i)
          if (depth[i] == (uint32_t)lv) level_nodes.push_back(node_base + (uint32_t)i);
      }
      level_off.push_back((uint32_t)level_nodes.size());
      for (Node nd : hb.nodes) {
        nd.d.x = rebase(nd.d.x);
        nd.d.y = rebase(nd.d.y);
        if (nd.d.z >= 0) nd.d.z += 2 * (int32_t)node_base;
        nodes.push_back(nd);
      }
      // children's leaf-order ranges, children before parents (a parent
      // precedes its children in the node order)
      {
        std::vector<uint2> span(hb.nodes.size());
        auto child_span = [&](int32_t c) {
          if (c < 0) return make_uint2(pv::leaf_first(c), pv::leaf_first(c) + pv::leaf_count(c));
          return span[(size_t)c];
        };
        const size_t at = dspan.size();
        dspan.resize(at + hb.nodes.size());
        dspan_obj.resize(at + hb.nodes.size(), o);
        for (size_t k = hb.nodes.size(); k-- > 0;) {
          const uint2 a = child_span(hb.nodes[k].d.x), b = child_span(hb.nodes[k].d.y);
          if (a.y != b.x) return fail(ctx, PV_ERR_STATE, "object topology is not in leaf order");
          span[k] = make_uint2(a.x, b.y);
          dspan[at + k] = make_uint4(tri_base + a.x, tri_base + a.y, tri_base + b.x, tri_base + b.y);
        }
      }
      for (uint32_t i = 0; i < n; ++i) {
        std::memcpy(&dlocal[9 * (size_t)(tri_base + i)], v + 9 * (size_t)hb.order[i], 9 * sizeof(float));
        dgid[tri_base + i] = gbase + hb.order[i];
      }
      ob.gbase = gbase;
      ob.n_tris = n;
      ob.tri_base = tri_base;
      ob.node_base = node_base;
      ob.n_nodes = (uint32_t)hb.nodes.size();
      ob.root = rebase(hb.root);
      {
        // the same topology with fixed object-space boxes; internal child
        // codes count from the region's start until it is placed below
        std::vector<float> lv9(9 * (size_t)n);
        for (uint32_t i = 0; i < n; ++i)
          std::memcpy(&lv9[9 * (size_t)i], v + 9 * (size_t)hb.order[i], 9 * sizeof(float));
        HostBvh os = hb;
        host_boxes(os, lv9.data(), kObjSpacePad);
        const int32_t obase = (int32_t)onodes.size();
        auto orebase = [&](int32_t c) { return c >= 0 ? c + obase : rebase(c); };
        for (Node nd : os.nodes) {
          nd.d.x = orebase(nd.d.x);
          nd.d.y = orebase(nd.d.y);
          nd.d.z = -1;
          onodes.push_back(nd);
        }
        ob.oroot = orebase(hb.root);
      }
      tri_base += n;
      gbase += n;
    }
    // regions of the per-frame rebuilt hierarchies (a radix tree over an
    // object's n triangles has n - 1 internal nodes), after the topologies
    const uint32_t lbvh_first = (uint32_t)nodes.size();
    for (uint32_t o = 0; o < d->n_objects; ++o) {
      objs[o].sah_root = objs[o].root;
      objs[o].lbvh_base = (uint32_t)nodes.size();
      nodes.resize(nodes.size() + (objs[o].n_tris - 1), Node{});
    }
    const uint32_t lbvh_nodes = (uint32_t)nodes.size() - lbvh_first;
    // traversal addresses node records by a 32-bit byte offset
    if ((nodes.size() + 2 * (size_t)pv::kTopNodes) * sizeof(Node) > (size_t)UINT32_MAX)
      return fail(ctx, PV_ERR_CAPACITY, "too many hierarchy nodes");
    hs.top_base = (uint32_t)nodes.size();
    nodes.resize(nodes.size() + 2 * (size_t)pv::kTopNodes, Node{});
    // the object-space copies after the top-level trees
    hs.onode_first = (uint32_t)nodes.size();
    for (Node nd : onodes) {
      if (nd.d.x >= 0) nd.d.x += (int32_t)hs.onode_first;
      if (nd.d.y >= 0) nd.d.y += (int32_t)hs.onode_first;
      nodes.push_back(nd);
    }
    for (ObjDev& ob : objs)
      if (ob.oroot >= 0) ob.oroot += (int32_t)hs.onode_first;
    if (nodes.size() * sizeof(Node) > (size_t)UINT32_MAX) return fail(ctx, PV_ERR_CAPACITY, "too many hierarchy nodes");
    Node* d_nodes;
    Tri* d_tris;
    float* d_dlocal;
    uint32_t *d_dgid, *d_lnodes, *d_loff;
    ObjDev* d_objs;
    CK(upload(A, &d_nodes, nodes.data(), nodes.size(), s));
    CK(dalloc(A, &d_tris, (size_t)S + n_dyn));
    if (S) CK(hipMemcpyAsync(d_tris, stris.data(), sizeof(Tri) * S, hipMemcpyHostToDevice, s));
    const int32_t no_roots[2] = {pv::kRootNone, pv::kRootNone};  // set per frame by the top-level build
    CK(upload(A, &hs.top, no_roots, 2, s));
    CK(upload(A, &d_dlocal, dlocal.data(), dlocal.size(), s));
    CK(upload(A, &d_dgid, dgid.data(), dgid.size(), s));
    {
      // record of each global triangle id in the leaf-order arrays (the
      // refit topology's order, which k_transform keeps current)
      std::vector<uint32_t> grec((size_t)S + n_dyn, 0u);
      for (uint32_t i = 0; i < S; ++i) {
        uint32_t g;
        std::memcpy(&g, &stris[i].t0.w, 4);
        grec[g] = i;
      }
      for (size_t k = 0; k < dgid.size(); ++k) grec[dgid[k]] = S + (uint32_t)k;
      uint32_t* d_grec;
      CK(upload(A, &d_grec, grec.data(), grec.size(), s));
      hs.gid_rec = d_grec;
    }
    CK(upload(A, &d_lnodes, level_nodes.data(), level_nodes.size(), s));
    CK(upload(A, &d_loff, level_off.data(), level_off.size(), s));
    CK(upload(A, &d_objs, objs.data(), objs.size(), s));
    hs.obj_node_first = obj_node_first;
    hs.n_obj_nodes = (uint32_t)dspan.size();
    if (!dspan.empty()) {
      uint4* d_span;
      uint32_t* d_span_obj;
      CK(upload(A, &d_span, dspan.data(), dspan.size(), s));
      CK(upload(A, &d_span_obj, dspan_obj.data(), dspan_obj.size(), s));
      hs.dspan = d_span;
      hs.dspan_obj = d_span_obj;
    }
    pv::LbvhWork lw{};
    if (n_dyn) {
      const uint32_t nd = (uint32_t)n_dyn, tiles = pv::lbvh_sort_tiles(nd);
      for (int b = 0; b < 2; ++b) {
        CK(dalloc(A, &lw.key[b], nd));
        CK(dalloc(A, &lw.val[b], nd));
      }
      CK(dalloc(A, &lw.hist, 256 * (size_t)tiles));
      CK(dalloc(A, &lw.hoff, 256 * (size_t)tiles));
      CK(dalloc(A, &lw.htotal, 1));
      CK(dalloc(A, &lw.scan_tmp, pv::scan_tmp_words(256 * tiles)));
      CK(dalloc(A, &lw.parent_leaf, nd));
      CK(dalloc(A, &lw.parent_node, std::max(lbvh_nodes, 1u)));
      CK(dalloc(A, &lw.pyr, 2 * (size_t)pv::lbvh_pyramid_entries(nd)));
      CK(dalloc(A, &lw.odepth, d->n_objects));
      CK(dalloc(A, &lw.cbox, 6 * (size_t)d->n_objects));
      lw.n_dyn = nd;
      lw.first_node = lbvh_first;
      lw.n_nodes = lbvh_nodes;
    }
    hs.nodes = d_nodes;
    hs.tris = d_tris;
    hs.dlocal = d_dlocal;
    hs.dtri_gid = d_dgid;
    hs.dlevel_nodes = d_lnodes;
    hs.dlevel_off = d_loff;
    hs.objs = d_objs;
    hs.n_obj = d->n_objects;
    hs.n_dyn_tris = (uint32_t)n_dyn;
    CK(dalloc(A, &hs.obj_aabb, 6 * (size_t)d->n_objects));
    CK(dalloc(A, &hs.obj_xf_cur, 12 * (size_t)d->n_objects));
    CK(dalloc(A, &hs.obj_xf_prev, 12 * (size_t)d->n_objects));
    CK(dalloc(A, &hs.obj_moved, d->n_objects));

    // lights (path ranges filled at store binding time)
    std::vector<LightDev> lights(d->n_lights);
    for (uint32_t l = 0; l < d->n_lights; ++l) {
      lights[l].half[0] = d->h_light_half[2 * l];
      lights[l].half[1] = d->h_light_half[2 * l + 1];
      for (int c = 0; c < 3; ++c) lights[l].power[c] = d->h_light_power[3 * l + c];
      lights[l].path_base = lights[l].path_count = 0;
      lights[l].kind = d->h_light_kind ? d->h_light_kind[l] : PV_LIGHT_AREA;
      lights[l].param[0] = lights[l].kind != PV_LIGHT_AREA ? d->h_light_param[2 * l] : 0.0f;
      lights[l].param[1] = lights[l].kind != PV_LIGHT_AREA ? d->h_light_param[2 * l + 1] : 0.0f;
      lights[l].pad[0] = lights[l].pad[1] = 0;
    }
    LightDev* d_lights;
    CK(upload(A, &d_lights, lights.data(), lights.size(), s));
    hs.lights = d_lights;
    hs.n_lights = d->n_lights;
    CK(dalloc(A, &hs.light_xf_cur, 12 * (size_t)d->n_lights));
    CK(dalloc(A, &hs.light_xf_prev, 12 * (size_t)d->n_lights));
    CK(dalloc(A, &hs.light_moved, d->n_lights));
    hs.verify_boxes = ctx->verify_boxes ? 1u : 0u;
    hs.energy_test = (uint32_t)ctx->energy_test;
    hs.eps_end = d->eps_end;
    hs.eps_close = d->eps_close;
    hs.radius = d->photon_radius;
    hs.gpath_base = 0;

    CK(dalloc(A, &ctx->d_scene, 1));
    CK(dalloc(A, &ctx->d_state, 1));
    hs.state = ctx->d_state;
    uint32_t one = 1;
    CK(hipMemcpyAsync(ctx->d_state, &one, 4, hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(ctx->d_scene, &hs, sizeof(hs), hipMemcpyHostToDevice, s));
    std::vector<uint2> ot;
    for (uint32_t o = 0; o < d->n_objects; ++o) ot.push_back(make_uint2(0, o));
    CK(upload(A, &ctx->d_obj_tiles, ot.data(), ot.size(), s));
    ctx->n_obj_tiles = (uint32_t)ot.size();
    std::vector<uint2> xt = xf_tiles(0, d->h_obj_tris, d->n_objects);
    CK(upload(A, &ctx->d_xf_tiles, xt.data(), xt.size(), s));
    ctx->n_xf_tiles = (uint32_t)xt.size();
    CK(dalloc(A, &ctx->d_in_ptrs, 2));
    // staged transforms start as identities (every object and light moves at
    // the first frame anyway); the host copy lives until the synchronisation
    const float id12[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
    std::vector<float> ident(12 * (size_t)std::max(std::max(d->n_objects, d->n_lights), 1u));
    for (size_t i = 0; i < ident.size(); ++i) ident[i] = id12[i % 12];
    CK(upload(A, &ctx->d_obj_staged, ident.data(), 12 * (size_t)std::max(d->n_objects, 1u), s));
    CK(upload(A, &ctx->d_light_staged, ident.data(), 12 * (size_t)d->n_lights, s));
    ctx->xf_pending = false;
    CK(hipStreamSynchronize(s));
    ctx->hs = hs;
    ctx->n_materials = d->n_materials;
    ctx->n_lights = d->n_lights;
    ctx->n_objects = d->n_objects;
    ctx->h_obj_tris.assign(d->h_obj_tris, d->h_obj_tris + d->n_objects);
    // the whole-scene top-level tree: the static root beside a median split
    // of the objects (or either alone); the moved-object tree: a median split
    ctx->top_depth = S && d->n_objects ? 1u + ceil_log2(d->n_objects) : ceil_log2(d->n_objects);
    ctx->static_depth = static_depth;
    ctx->obj_depth = obj_depth;
    ctx->lbvh_depth = d->n_objects ? (uint32_t)kMaxDepth : 0;
    ctx->lw = lw;
    ctx->lbvh_used = ctx->object_rebuild;
    ctx->point_lights = false;
    for (uint32_t l = 0; l < d->n_lights; ++l)
      ctx->point_lights |= d->h_light_half[2 * l] == 0.0f && d->h_light_half[2 * l + 1] == 0.0f;
    size_stacks(ctx);
    ctx->h_light_paths.assign(d->n_lights, 0);
    ctx->uploaded = true;
    return PV_OK;
  } catch (const std::exception& e) {
    return fail(ctx, PV_ERR_OOM, std::string("host exception: ") + e.what());
  }
}

// Paths per light: light l owns paths [sum_{i<l} counts[i], ... + counts[l]).
pv_status pv_set_light_paths(pv_ctx* ctx, const uint32_t* h_counts) {
  if (!ctx) return PV_ERR_ARG;
  if (!ctx->uploaded) return fail(ctx, PV_ERR_STATE, "no scene uploaded");
  if (!h_counts) return fail(ctx, PV_ERR_ARG, "counts is NULL");
  std::vector<LightDev> lights(ctx->n_lights);
  CK(hipMemcpy(lights.data(), ctx->hs.lights, sizeof(LightDev) * ctx->n_lights, hipMemcpyDeviceToHost));
  uint32_t base = 0;
  for (uint32_t l = 0; l < ctx->n_lights; ++l) {
    lights[l].path_base = base;
    lights[l].path_count = h_counts[l];
    ctx->h_light_paths[l] = h_counts[l];
    base += h_counts[l];
  }
  CK(hipMemcpy(const_cast<LightDev*>(ctx->hs.lights), lights.data(), sizeof(LightDev) * ctx->n_lights,
               hipMemcpyHostToDevice));
  ctx->bound = false;
  return PV_OK;
}

pv_status pv_reserve(pv_ctx* ctx, uint32_t max_paths, uint32_t max_bounces) {
  if (!ctx) return PV_ERR_ARG;
  if (max_paths == 0 || max_paths > kMaxPaths) return fail(ctx, PV_ERR_ARG, "max_paths out of range");
  if (max_bounces < 1 || max_bounces > PV_MAX_BOUNCES) return fail(ctx, PV_ERR_ARG, "max_bounces out of range");
  try {
    if (pv_status w = wait_compaction(ctx)) return w;
    CK(hipStreamSynchronize(ctx->stream));
    ctx->res_mem.release();
    ctx->reserved = ctx->bound = false;
    if (ctx->dm_enabled) {  // the maps' per-tile scratch follows the reserved size: set them again
      ctx->dm_mem.release();
      ctx->dm_enabled = false;
      ctx->dm_cells = 0;
      std::memset(ctx->hs.dm, 0, sizeof(ctx->hs.dm));
    }
    Alloc& A = ctx->res_mem;
    uint32_t nb = path_blocks(max_paths);
    std::vector<uint2> tiles = make_tiles(0, max_paths);
    CK(upload(A, &ctx->d_path_tiles, tiles.data(), tiles.size(), ctx->stream));
    CK(dalloc(A, &ctx->d_block_cnt, nb));
    CK(dalloc(A, &ctx->d_offsets, nb));
    CK(dalloc(A, &ctx->d_queue, max_paths));
    ctx->ow.tiles = pv::order_tiles(max_paths);
    CK(dalloc(A, &ctx->ow.queue, max_paths));
    CK(dalloc(A, &ctx->ow.hist, 8 * (size_t)ctx->ow.tiles));
    CK(dalloc(A, &ctx->ow.hoff, 8 * (size_t)ctx->ow.tiles));
    CK(dalloc(A, &ctx->ow.htotal, 1));
    CK(dalloc(A, &ctx->ow.scan_tmp, pv::scan_tmp_words(8 * ctx->ow.tiles)));
    CK(dalloc(A, &ctx->ow.deal, (size_t)pv::kDealGroups * pv::kDealStride));
    CK(dalloc(A, &ctx->d_qcount, 1));
    CK(dalloc(A, &ctx->d_pcounts, (size_t)nb * max_bounces));
    CK(dalloc(A, &ctx->d_poffsets, (size_t)nb * max_bounces));
    CK(dalloc(A, &ctx->d_gbase, 2));
    CK(dalloc(A, &ctx->d_partial, (size_t)nb * 3 * (256 + PV_MAX_LIGHTS)));
    CK(dalloc(A, &ctx->d_scan_tmp, pv::scan_tmp_words(nb * max_bounces)));
    CK(dalloc(A, &ctx->d_scan_tmp_c, pv::scan_tmp_words(nb * max_bounces)));
    const size_t task_cap = (size_t)nb * pv::kBlock * max_bounces;  // a region of kBlock * B per tile
    CK(dalloc(A, &ctx->vw.tmp, task_cap));
    CK(dalloc(A, &ctx->vw.tasks, task_cap));
    CK(dalloc(A, &ctx->vw.tcount, nb));
    CK(dalloc(A, &ctx->vw.toff, nb));
    CK(dalloc(A, &ctx->vw.total, 1));
    CK(dalloc(A, &ctx->vw.deal, (size_t)pv::kDealGroups * pv::kDealStride));
    CK(dalloc(A, &ctx->vw.first, max_paths));
    CK(dalloc(A, &ctx->vw.part, 4 * (size_t)nb + 2 * (size_t)pv::verify_finish_blocks(verify_blocks_max(ctx))));
    CK(hipMemsetAsync(ctx->d_qcount, 0, 4, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    ctx->max_paths = max_paths;
    ctx->max_bounces = max_bounces;
    ctx->max_blocks = nb;
    ctx->reserved = true;
    return PV_OK;
  } catch (const std::exception& e) {
    return fail(ctx, PV_ERR_OOM, std::string("host exception: ") + e.what());
  }
}

namespace {

// Start a frame with the given transform arrays (the staged ones when both
// are NULL): moved flags, world triangles of the moved objects, their boxes,
// the top-level trees.
pv_status begin_frame(pv_ctx* ctx, const float* d_obj_xf, const float* d_light_xf) {
  if (!d_obj_xf && !d_light_xf) {
    d_obj_xf = ctx->d_obj_staged;
    d_light_xf = ctx->d_light_staged;
  } else {
    // the staged arrays follow the dense ones, for later sparse updates
    if (ctx->n_objects)
      CK(hipMemcpyAsync(ctx->d_obj_staged, d_obj_xf, 48 * (size_t)ctx->n_objects, hipMemcpyDeviceToDevice,
                        ctx->stream));
    CK(hipMemcpyAsync(ctx->d_light_staged, d_light_xf, 48 * (size_t)ctx->n_lights, hipMemcpyDeviceToDevice,
                      ctx->stream));
  }
  ctx->xf_pending = false;
  const float* in[2] = {d_obj_xf, d_light_xf};
  CK(hipMemcpyAsync(ctx->d_in_ptrs, in, sizeof(in), hipMemcpyHostToDevice, ctx->stream));
  CK(pv::launch_frame_begin(ctx->d_scene, 1, ctx->d_in_ptrs, ctx->d_in_ptrs + 1, ctx->stream));
  // world triangles of the moved objects, then their topologies' boxes as
  // unions over leaf-order ranges
  CK(pv::launch_transform_objects(ctx->d_scene, ctx->d_xf_tiles, ctx->n_xf_tiles, ctx->stream));
  CK(pv::launch_refit_objects(ctx->d_scene, ctx->lw, ctx->n_objects, ctx->hs.n_obj_nodes, ctx->stream));
  // rebuild mode: every object's hierarchy rebuilt from its current
  // triangles; the refit topology (kept current above) stays the hierarchy of
  // an object whose rebuilt tree is too deep for the traversal stacks
  if (ctx->object_rebuild)
    CK(pv::launch_rebuild_objects(ctx->d_scene, ctx->lw, ctx->n_objects, ctx->lbvh_depth, ctx->stream));
  CK(pv::launch_build_top(ctx->d_scene, 1, ctx->stream));
  ctx->frame_started = true;
  return PV_OK;
}

// A sparse transform update since the last frame begins the next frame.
pv_status commit_pending(pv_ctx* ctx) {
  if (!ctx->xf_pending) return PV_OK;
  return begin_frame(ctx, nullptr, nullptr);
}

pv_status update_staged(pv_ctx* ctx, float* staged, uint32_t n_rows, uint32_t max_n, uint32_t n,
                        const uint32_t* d_ids, const float* d_m3x4, const char* what) {
  if (!ctx) return PV_ERR_ARG;
  if (!ctx->uploaded) return fail(ctx, PV_ERR_STATE, "no scene uploaded");
  if (n > max_n) return fail(ctx, PV_ERR_ARG, std::string("more ") + what + " updates than " + what + "s");
  if (n && (!d_ids || !d_m3x4)) return fail(ctx, PV_ERR_ARG, "id or matrix array is NULL");
  if (n) CK(pv::launch_scatter_xf(staged, n_rows, d_ids, d_m3x4, n, ctx->stream));
  ctx->xf_pending = true;
  return PV_OK;
}

}  // namespace

pv_status pv_frame_begin(pv_ctx* ctx, const float* d_obj_xf, const float* d_light_xf) {
  if (!ctx) return PV_ERR_ARG;
  if (!ctx->uploaded) return fail(ctx, PV_ERR_STATE, "no scene uploaded");
  const bool staged = !d_obj_xf && !d_light_xf;
  if (!staged && ((ctx->n_objects && !d_obj_xf) || !d_light_xf))
    return fail(ctx, PV_ERR_ARG, "transform array is NULL");
  return begin_frame(ctx, d_obj_xf, d_light_xf);
}

pv_status pv_update_transforms(pv_ctx* ctx, uint32_t n, const uint32_t* d_obj_ids, const float* d_m3x4) {
  return update_staged(ctx, ctx ? ctx->d_obj_staged : nullptr, ctx ? ctx->n_objects : 0, PV_MAX_OBJECTS, n,
                       d_obj_ids, d_m3x4, "object");
}

pv_status pv_update_lights(pv_ctx* ctx, uint32_t n, const uint32_t* d_light_ids, const float* d_m3x4) {
  return update_staged(ctx, ctx ? ctx->d_light_staged : nullptr, ctx ? ctx->n_lights : 0, PV_MAX_LIGHTS, n,
                       d_light_ids, d_m3x4, "light");
}

pv_status pv_verify_paths(pv_ctx* ctx, const pv_path_store* store, pv_stats* d_stats) {
  if (!ctx) return PV_ERR_ARG;
  pv_status st = bind_store(ctx, store);
  if (st) return st;
  if ((st = commit_pending(ctx))) return st;
  if (!ctx->frame_started) return fail(ctx, PV_ERR_STATE, "no transforms given (pv_frame_begin or pv_update_*)");
  uint32_t nb = path_blocks(store->n_paths);
  CK(pv::launch_verify(ctx->d_scene, ctx->d_path_tiles, nb, ctx->d_gbase, 1, ctx->vw, ctx->d_block_cnt, d_stats,
                       ctx->stack_moved, verify_blocks(ctx), ctx->verify_min_active, ctx->d_scan_tmp, ctx->stream));
  ctx->counts_ready = true;
  ctx->queue_stale = true;
  return PV_OK;
}

pv_status pv_build_queue(pv_ctx* ctx, const pv_path_store* store) {
  if (!ctx) return PV_ERR_ARG;
  pv_status st = bind_store(ctx, store);
  if (st) return st;
  if (!ctx->counts_ready) return fail(ctx, PV_ERR_STATE, "pv_verify_paths has not been called");
  uint32_t nb = path_blocks(store->n_paths);
  CK(pv::launch_scan(ctx->d_block_cnt, ctx->d_offsets, nb, ctx->d_qcount, ctx->d_scan_tmp, ctx->stream));
  CK(pv::launch_scatter_queue(ctx->d_scene, ctx->d_path_tiles, nb, ctx->d_offsets, ctx->d_queue, ctx->stream));
  ctx->queue_stale = false;
  return PV_OK;
}

pv_status pv_queue_all(pv_ctx* ctx, const pv_path_store* store) {
  if (!ctx) return PV_ERR_ARG;
  pv_status st = bind_store(ctx, store);
  if (st) return st;
  if ((st = wait_compaction(ctx))) return st;
  uint32_t nb = path_blocks(store->n_paths);
  CK(pv::launch_mark_all(ctx->d_scene, ctx->d_path_tiles, nb, ctx->d_block_cnt, ctx->stream));
  CK(pv::launch_scan(ctx->d_block_cnt, ctx->d_offsets, nb, ctx->d_qcount, ctx->d_scan_tmp, ctx->stream));
  CK(pv::launch_scatter_queue(ctx->d_scene, ctx->d_path_tiles, nb, ctx->d_offsets, ctx->d_queue, ctx->stream));
  ctx->queue_stale = false;
  return PV_OK;
}

pv_status pv_copy_queue(pv_ctx* ctx, uint32_t* d_out, uint32_t capacity, uint32_t* d_count) {
  if (!ctx) return PV_ERR_ARG;
  if (!ctx->reserved) return fail(ctx, PV_ERR_STATE, "pv_reserve has not been called");
  if (!d_out || !d_count) return fail(ctx, PV_ERR_ARG, "output is NULL");
  uint32_t n = std::min(capacity, ctx->bound ? ctx->bstore.n_paths : 0u);
  if (n) CK(hipMemcpyAsync(d_out, ctx->d_queue, 4 * (size_t)n, hipMemcpyDeviceToDevice, ctx->stream));
  CK(hipMemcpyAsync(d_count, ctx->d_qcount, 4, hipMemcpyDeviceToDevice, ctx->stream));
  return PV_OK;
}

pv_status pv_retrace_paths(pv_ctx* ctx, const pv_path_store* store, float threshold, uint64_t seed, uint32_t frame,
                           pv_stats* d_stats) {
  if (!ctx) return PV_ERR_ARG;
  pv_status st = bind_store(ctx, store);
  if (st) return st;
  if (std::isnan(threshold)) return fail(ctx, PV_ERR_ARG, "threshold is NaN");
  if ((st = commit_pending(ctx))) return st;
  if (!ctx->frame_started) return fail(ctx, PV_ERR_STATE, "no transforms given (pv_frame_begin or pv_update_*)");
  // the paths the last verification replaced, unless the queue was built since
  if (ctx->queue_stale && (st = pv_build_queue(ctx, store))) return st;
  if ((st = wait_compaction(ctx))) return st;
  uint32_t blocks = (uint32_t)(ctx->n_cu * ctx->retrace_blocks_per_cu);
  CK(pv::launch_retrace(ctx->d_scene, ctx->d_gbase, 1, ctx->d_queue, ctx->d_qcount, threshold, seed,
                        frame, nullptr, d_stats, blocks, ctx->retrace_variant, ctx->stack_entries,
                        ctx->walk_min_active, ctx->ow, ctx->stream));
  return PV_OK;
}

pv_status pv_set_tuning(pv_ctx* ctx, int32_t key, int32_t value) {
  if (!ctx) return PV_ERR_ARG;
  if (key == PV_TUNE_RETRACE_VARIANT) {
    if (value < 0 || value > 3) return fail(ctx, PV_ERR_ARG, "re-trace variant out of range 0..3");
    ctx->retrace_variant = value;
  } else if (key == PV_TUNE_RETRACE_BLOCKS_PER_CU) {
    if (value < 1 || value > 64) return fail(ctx, PV_ERR_ARG, "blocks per CU out of range 1..64");
    ctx->retrace_blocks_per_cu = value;
  } else if (key == PV_TUNE_WALK_MIN_ACTIVE) {
    if (value < 1 || value > 64) return fail(ctx, PV_ERR_ARG, "walk minimum active lanes out of range 1..64");
    ctx->walk_min_active = value;
  } else if (key == PV_TUNE_VERIFY_BLOCKS_PER_CU) {
    if (value < 1 || value > kMaxVerifyBlocksPerCu) return fail(ctx, PV_ERR_ARG, "verify blocks per CU out of range 1..32");
    ctx->verify_blocks_per_cu = value;
  } else if (key == PV_TUNE_VERIFY_MIN_ACTIVE) {
    if (value < 1 || value > 64) return fail(ctx, PV_ERR_ARG, "verify minimum active lanes out of range 1..64");
    ctx->verify_min_active = value;
  } else if (key == PV_TUNE_OBJECT_REBUILD) {
    if (value != 0 && value != 1) return fail(ctx, PV_ERR_ARG, "object rebuild is 0 or 1");
    ctx->object_rebuild = value == 1;
    if (ctx->object_rebuild && !ctx->lbvh_used) {
      ctx->lbvh_used = true;
      size_stacks(ctx);
    }
  } else {
    return fail(ctx, PV_ERR_ARG, "unknown tuning key");
  }
  return PV_OK;
}

pv_status pv_set_verify_mode(pv_ctx* ctx, int32_t mode) {
  if (!ctx) return PV_ERR_ARG;
  if (mode != PV_VERIFY_TRIANGLES && mode != PV_VERIFY_BOXES)
    return fail(ctx, PV_ERR_ARG, "verify mode is PV_VERIFY_TRIANGLES or PV_VERIFY_BOXES");
  ctx->verify_boxes = mode == PV_VERIFY_BOXES;
  ctx->hs.verify_boxes = ctx->verify_boxes ? 1u : 0u;
  if (pv_status w = wait_compaction(ctx)) return w;
  if (ctx->uploaded)  // stream-ordered after the work already enqueued
    CK(hipMemcpyAsync(ctx->d_scene, &ctx->hs, sizeof(SceneDev), hipMemcpyHostToDevice, ctx->stream));
  return PV_OK;
}

pv_status pv_set_energy_test(pv_ctx* ctx, int32_t mode) {
  if (!ctx) return PV_ERR_ARG;
  if (mode != PV_ENERGY_ALBEDO && mode != PV_ENERGY_COSINE_RATIO)
    return fail(ctx, PV_ERR_ARG, "energy test is PV_ENERGY_ALBEDO or PV_ENERGY_COSINE_RATIO");
  ctx->energy_test = mode;
  ctx->hs.energy_test = (uint32_t)mode;
  if (pv_status w = wait_compaction(ctx)) return w;
  if (ctx->uploaded)  // stream-ordered after the work already enqueued
    CK(hipMemcpyAsync(ctx->d_scene, &ctx->hs, sizeof(SceneDev), hipMemcpyHostToDevice, ctx->stream));
  return PV_OK;
}

pv_status pv_set_distribution_map(pv_ctx* ctx, const int32_t* h_grid) {
  if (!ctx) return PV_ERR_ARG;
  if (!ctx->uploaded) return fail(ctx, PV_ERR_STATE, "no scene uploaded");
  if (!ctx->reserved) return fail(ctx, PV_ERR_STATE, "pv_reserve has not been called");
  if (pv_status w = wait_compaction(ctx)) return w;
  CK(hipStreamSynchronize(ctx->stream));  // the maps' scratch may be in use
  ctx->dm_mem.release();
  ctx->dw = pv::DmWork{};
  ctx->dm_enabled = false;
  ctx->dm_cells = 0;
  std::memset(ctx->hs.dm, 0, sizeof(ctx->hs.dm));
  std::memset(ctx->hs.dm_off, 0, sizeof(ctx->hs.dm_off));
  if (h_grid) {
    for (int k = 0; k < 4; ++k)
      if (h_grid[k] < 1 || h_grid[k] > 4096) return fail(ctx, PV_ERR_ARG, "grid sizes out of range 1..4096");
    std::vector<LightDev> lights(ctx->n_lights);
    CK(hipMemcpy(lights.data(), ctx->hs.lights, sizeof(LightDev) * ctx->n_lights, hipMemcpyDeviceToHost));
    uint64_t total = 0;
    uint32_t off[PV_MAX_LIGHTS + 1] = {0};
    for (uint32_t l = 0; l < ctx->n_lights; ++l) {
      const uint64_t c = lights[l].kind == PV_LIGHT_CAMERA
                             ? (uint64_t)h_grid[0] * h_grid[1]
                             : (uint64_t)(pv::dm_point(lights[l].half) ? 1 : (uint64_t)h_grid[0] * h_grid[1]) *
                                   (uint64_t)h_grid[2] * h_grid[3];
      if (c > (1u << 22)) return fail(ctx, PV_ERR_ARG, "more than 2^22 cells for a light (22-bit cell field)");
      off[l] = (uint32_t)total;
      total += c;
    }
    if (total > (1u << 24)) return fail(ctx, PV_ERR_ARG, "more than 2^24 cells in all");
    off[ctx->n_lights] = (uint32_t)total;
    const uint32_t cells = (uint32_t)total, tiles = ctx->max_blocks;
    Alloc& A = ctx->dm_mem;
    pv::DmWork& D = ctx->dw;
    CK(dalloc(A, &D.dm_c, cells));
    CK(dalloc(A, &D.pruned, cells));
    CK(dalloc(A, &D.def, cells));
    CK(dalloc(A, &D.dex, (size_t)cells + 1));
    CK(dalloc(A, &D.tcnt, tiles));
    CK(dalloc(A, &D.toff, tiles));
    CK(dalloc(A, &D.ttotal, 1));
    CK(dalloc(A, &D.rank0, PV_MAX_LIGHTS));
    CK(dalloc(A, &D.scan_tmp, pv::scan_tmp_words(cells)));
    CK(dalloc(A, &D.scan_tmp2, pv::scan_tmp_words(tiles)));
    for (int k = 0; k < 4; ++k) ctx->hs.dm[k] = h_grid[k];
    std::memcpy(ctx->hs.dm_off, off, sizeof(off));
    ctx->dm_cells = cells;
    ctx->dm_enabled = true;
  }
  // stream-ordered after the work already enqueued
  CK(hipMemcpyAsync(ctx->d_scene, &ctx->hs, sizeof(SceneDev), hipMemcpyHostToDevice, ctx->stream));
  return PV_OK;
}

pv_status pv_update_distribution(pv_ctx* ctx, const pv_path_store* store, uint64_t seed, uint32_t frame,
                                 uint32_t* d_dm_c, uint32_t* d_pruned) {
  if (!ctx) return PV_ERR_ARG;
  pv_status st = bind_store(ctx, store);
  if (st) return st;
  if (!ctx->dm_enabled) return fail(ctx, PV_ERR_STATE, "no distribution map (pv_set_distribution_map)");
  if ((st = commit_pending(ctx))) return st;
  if (!ctx->frame_started) return fail(ctx, PV_ERR_STATE, "no transforms given (pv_frame_begin or pv_update_*)");
  if ((st = wait_compaction(ctx))) return st;
  const uint32_t nb = path_blocks(store->n_paths);
  CK(pv::launch_dm_update(ctx->d_scene, ctx->d_scene, ctx->d_path_tiles, nb, ctx->dm_cells, ctx->n_lights, ctx->dw,
                          ctx->d_block_cnt, seed, frame, nullptr, ctx->stream));
  if (d_dm_c)
    CK(hipMemcpyAsync(d_dm_c, ctx->dw.dm_c, 4 * (size_t)ctx->dm_cells, hipMemcpyDeviceToDevice, ctx->stream));
  if (d_pruned)
    CK(hipMemcpyAsync(d_pruned, ctx->dw.pruned, 4 * (size_t)ctx->dm_cells, hipMemcpyDeviceToDevice, ctx->stream));
  ctx->counts_ready = true;
  ctx->queue_stale = true;
  return PV_OK;
}

uint32_t pv_distribution_cells(const pv_ctx* ctx) { return ctx && ctx->dm_enabled ? ctx->dm_cells : 0u; }

pv_status pv_object_hierarchy_info(pv_ctx* ctx, uint32_t obj, uint32_t* out) {
  if (!ctx) return PV_ERR_ARG;
  if (!out) return fail(ctx, PV_ERR_ARG, "out is NULL");
  if (!ctx->uploaded) return fail(ctx, PV_ERR_STATE, "no scene uploaded");
  if (obj >= ctx->n_objects) return fail(ctx, PV_ERR_ARG, "object index out of range");
  try {
    if (pv_status st = commit_pending(ctx)) return st;
    CK(hipStreamSynchronize(ctx->stream));
    const SceneDev& hs = ctx->hs;
    ObjDev ob;
    CK(hipMemcpy(&ob, hs.objs + obj, sizeof(ObjDev), hipMemcpyDeviceToHost));
    std::vector<Node> nodes(hs.top_base);
    CK(hipMemcpy(nodes.data(), hs.nodes, sizeof(Node) * nodes.size(), hipMemcpyDeviceToHost));
    const uint32_t first = hs.n_static + ob.tri_base;
    std::vector<Tri> tris(ob.n_tris);
    CK(hipMemcpy(tris.data(), hs.tris + first, sizeof(Tri) * tris.size(), hipMemcpyDeviceToHost));
    // walk the current hierarchy from the object's root: its internal nodes
    // lie in the object's topology or rebuild region, its leaves partition the
    // object's triangle records, every box on the way to a leaf contains that
    // leaf's triangles, and no leaf is deeper than the stack allows
    const bool in_rebuild = ob.root >= 0 && (uint32_t)ob.root >= ob.lbvh_base;
    const uint32_t lo = in_rebuild ? ob.lbvh_base : ob.node_base;
    const uint32_t hi = in_rebuild ? ob.lbvh_base + (ob.n_tris - 1) : ob.node_base + ob.n_nodes;
    struct It {
      int32_t code;
      uint32_t depth;
      float box[6];
    };
    std::vector<It> st;
    std::vector<uint8_t> seen(ob.n_tris, 0);
    st.push_back({ob.root, 0, {-INFINITY, -INFINITY, -INFINITY, INFINITY, INFINITY, INFINITY}});
    uint32_t n_int = 0, n_leaf = 0, max_depth = 0;
    bool ok = true;
    auto inside = [](const float* in6, const float* out6) {
      for (int k = 0; k < 3; ++k)
        if (in6[k] < out6[k] || in6[3 + k] > out6[3 + k]) return false;
      return true;
    };
    while (!st.empty() && ok) {
      const It it = st.back();
      st.pop_back();
      max_depth = std::max(max_depth, it.depth);
      if (it.code < 0) {
        ++n_leaf;
        const uint32_t f = pv::leaf_first(it.code), c = pv::leaf_count(it.code);
        for (uint32_t i = f; i < f + c && ok; ++i) {
          if (i < first || i - first >= ob.n_tris || seen[i - first]) {
            ok = false;
            break;
          }
          seen[i - first] = 1;
          const Tri& t = tris[i - first];
          const float4 v[3] = {t.t0, t.t1, t.t2};
          for (int q = 0; q < 3; ++q) {
            const float b[6] = {v[q].x, v[q].y, v[q].z, v[q].x, v[q].y, v[q].z};
            if (!inside(b, it.box)) ok = false;
          }
        }
        continue;
      }
      if ((uint32_t)it.code < lo || (uint32_t)it.code >= hi || n_int > ob.n_tris) {
        ok = false;
        break;
      }
      ++n_int;
      const Node& nd = nodes[it.code];
      const float* f = reinterpret_cast<const float*>(&nd);
      for (int side = 0; side < 2; ++side) {
        It ch;
        ch.code = side ? nd.d.y : nd.d.x;
        ch.depth = it.depth + 1;
        std::memcpy(ch.box, f + 6 * side, sizeof(ch.box));
        if (!inside(ch.box, it.box)) ok = false;
        st.push_back(ch);
      }
    }
    for (uint32_t i = 0; i < ob.n_tris && ok; ++i)
      if (!seen[i]) ok = false;
    const uint32_t allowed = ctx->lbvh_used ? std::max(ctx->obj_depth, ctx->lbvh_depth) : ctx->obj_depth;
    out[0] = n_int;
    out[1] = n_leaf;
    out[2] = max_depth;
    out[3] = (ok && max_depth <= allowed) ? 1u : 0u;
    out[4] = in_rebuild ? 1u : 0u;
    return PV_OK;
  } catch (const std::bad_alloc&) {
    return fail(ctx, PV_ERR_OOM, "host allocation failed");
  }
}

pv_status pv_get_tuning(const pv_ctx* ctx, int32_t key, int32_t* value) {
  if (!ctx || !value) return PV_ERR_ARG;
  if (key == PV_TUNE_RETRACE_VARIANT)
    *value = ctx->retrace_variant;
  else if (key == PV_TUNE_RETRACE_BLOCKS_PER_CU)
    *value = ctx->retrace_blocks_per_cu;
  else if (key == PV_TUNE_WALK_MIN_ACTIVE)
    *value = ctx->walk_min_active;
  else if (key == PV_TUNE_VERIFY_BLOCKS_PER_CU)
    *value = ctx->verify_blocks_per_cu;
  else if (key == PV_TUNE_VERIFY_MIN_ACTIVE)
    *value = ctx->verify_min_active;
  else if (key == PV_TUNE_OBJECT_REBUILD)
    *value = ctx->object_rebuild ? 1 : 0;
  else
    return PV_ERR_ARG;
  return PV_OK;
}

pv_status pv_autotune(pv_ctx* ctx, const pv_path_store* store, float threshold, uint64_t seed, uint32_t frame,
                      float* out_ms) {
  if (!ctx) return PV_ERR_ARG;
  pv_status st = bind_store(ctx, store);
  if (st) return st;
  if (std::isnan(threshold)) return fail(ctx, PV_ERR_ARG, "threshold is NaN");
  if ((st = commit_pending(ctx))) return st;
  if (!ctx->frame_started) return fail(ctx, PV_ERR_STATE, "no transforms given (pv_frame_begin or pv_update_*)");
  // the paths the last verification replaced, unless the queue was built since
  if (ctx->queue_stale && (st = pv_build_queue(ctx, store))) return st;
  if ((st = wait_compaction(ctx))) return st;
  const size_t rows = (size_t)store->max_bounces * store->stride;
  const size_t b_pos = 16 * rows, b_en = 16 * rows, b_or = 12 * (size_t)store->stride, b_in = 4 * (size_t)store->stride;
  char* backup = nullptr;
  CK(hipMalloc(&backup, b_pos + b_en + b_or + b_in));
  hipStream_t s = ctx->stream;
  auto copy_store = [&](bool save) -> hipError_t {
    void* dev[4] = {store->d_pos_hit, store->d_energy, store->d_origin, store->d_info};
    size_t sz[4] = {b_pos, b_en, b_or, b_in};
    size_t off = 0;
    for (int i = 0; i < 4; ++i) {
      hipError_t e = save ? hipMemcpyAsync(backup + off, dev[i], sz[i], hipMemcpyDeviceToDevice, s)
                          : hipMemcpyAsync(dev[i], backup + off, sz[i], hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
      off += sz[i];
    }
    return hipSuccess;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = copy_store(true);
  if (err == hipSuccess) err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  const uint32_t nb = path_blocks(store->n_paths);
  // every trial is timed kTuneReps times on the restored store; the median
  // decides, and the spread (max - min) / median of each trial is recorded
  constexpr int kTuneReps = 3;
  float rep_ms[kTuneReps];
  auto median_spread = [&](float* spread) {
    float a = rep_ms[0], b = rep_ms[1], c = rep_ms[2];
    const float lo = std::min(a, std::min(b, c)), hi = std::max(a, std::max(b, c));
    const float med = a + b + c - lo - hi;
    *spread = med > 0.0f ? (hi - lo) / med : 0.0f;
    return med;
  };
  float rep_spread = 0.0f;
  std::memset(ctx->tune_report, 0, sizeof(ctx->tune_report));
  // one trial: restore the store, verify + queue, time the re-trace
  auto trial = [&](int v, int bpc, int min_active, float* ms_out) -> hipError_t {
    hipError_t e = hipSuccess;
    for (int rep = 0; rep < kTuneReps && e == hipSuccess; ++rep) {
      e = copy_store(false);
      if (e == hipSuccess)
        e = pv::launch_verify(ctx->d_scene, ctx->d_path_tiles, nb, ctx->d_gbase, 1, ctx->vw, ctx->d_block_cnt,
                              nullptr, ctx->stack_moved, verify_blocks(ctx), ctx->verify_min_active, ctx->d_scan_tmp, s);
      if (e == hipSuccess)
        e = pv::launch_scan(ctx->d_block_cnt, ctx->d_offsets, nb, ctx->d_qcount, ctx->d_scan_tmp, s);
      if (e == hipSuccess)
        e = pv::launch_scatter_queue(ctx->d_scene, ctx->d_path_tiles, nb, ctx->d_offsets, ctx->d_queue, s);
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      if (e == hipSuccess)
        e = pv::launch_retrace(ctx->d_scene, ctx->d_gbase, 1, ctx->d_queue, ctx->d_qcount, threshold,
                               seed, frame, nullptr, nullptr, (uint32_t)(ctx->n_cu * bpc), v, ctx->stack_entries,
                               min_active, ctx->ow, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      rep_ms[rep] = ms;
    }
    *ms_out = e == hipSuccess ? median_spread(&rep_spread) : INFINITY;
    ctx->tune_report[6] += 1.0f;
    ctx->tune_report[5] = std::max(ctx->tune_report[5], rep_spread);
    return e;
  };
  // a later candidate (larger grid, higher occupancy target or threshold)
  // replaces the best one only when it is clearly faster: near-ties between
  // grids measured on one frame did not carry over to later frames
  constexpr float kTuneMargin = 0.99f;
  // verification: traversal grid x yield threshold, each timed on the restored store
  float best_verify = INFINITY;
  {
    int bv_b = ctx->verify_blocks_per_cu, bv_m = ctx->verify_min_active;
    // (with work dealt a refill at a time, workgroups beyond residency simply
    // start later and take what is left)
    const int vgrids[4] = {4, 8, 16, 32}, vmins[4] = {8, 16, 32, 48};
    for (int gi = 0; gi < 4 && err == hipSuccess; ++gi) {
      for (int mi = 0; mi < 4 && err == hipSuccess; ++mi) {
        ctx->verify_blocks_per_cu = vgrids[gi];
        ctx->verify_min_active = vmins[mi];
        for (int rep = 0; rep < kTuneReps && err == hipSuccess; ++rep) {
          err = copy_store(false);
          if (err == hipSuccess) err = hipEventRecord(e0, s);
          if (err == hipSuccess)
            err = pv::launch_verify(ctx->d_scene, ctx->d_path_tiles, nb, ctx->d_gbase, 1, ctx->vw, ctx->d_block_cnt,
                                    nullptr, ctx->stack_moved, verify_blocks(ctx), ctx->verify_min_active,
                                    ctx->d_scan_tmp, s);
          if (err == hipSuccess) err = hipEventRecord(e1, s);
          if (err == hipSuccess) err = hipEventSynchronize(e1);
          float ms = 0;
          if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
          rep_ms[rep] = ms;
        }
        if (err != hipSuccess) break;
        float spread = 0.0f;
        const float t_med = median_spread(&spread);
        ctx->tune_report[6] += 1.0f;
        ctx->tune_report[2] = std::max(ctx->tune_report[2], spread);
        if (t_med < best_verify * kTuneMargin) {
          best_verify = t_med;
          ctx->tune_report[1] = spread;
          bv_b = vgrids[gi];
          bv_m = vmins[mi];
        }
      }
    }
    ctx->verify_blocks_per_cu = bv_b;
    ctx->verify_min_active = bv_m;
  }
  // re-trace: occupancy variant x grid at the current yield threshold, then the threshold
  float best = INFINITY;
  int best_v = ctx->retrace_variant, best_b = ctx->retrace_blocks_per_cu, best_m = ctx->walk_min_active;
  const int grids[4] = {4, 8, 16, 32};
  for (int v = 0; v < 4 && err == hipSuccess; ++v) {
    for (int gi = 0; gi < 4 && err == hipSuccess; ++gi) {
      float ms = INFINITY;
      err = trial(v, grids[gi], best_m, &ms);
      if (ms < best * kTuneMargin) {
        best = ms;
        ctx->tune_report[4] = rep_spread;
        best_v = v;
        best_b = grids[gi];
      }
    }
  }
  const int mins[6] = {8, 16, 24, 32, 40, 48};
  for (int mi = 0; mi < 6 && err == hipSuccess; ++mi) {
    float ms = INFINITY;
    err = trial(best_v, best_b, mins[mi], &ms);
    if (ms < best * kTuneMargin) {
      best = ms;
      ctx->tune_report[4] = rep_spread;
      best_m = mins[mi];
    }
  }
  if (err == hipSuccess) err = copy_store(false);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(backup);
  CK(err);
  ctx->retrace_variant = best_v;
  ctx->retrace_blocks_per_cu = best_b;
  ctx->walk_min_active = best_m;
  ctx->counts_ready = false;
  ctx->tune_report[0] = best_verify;
  ctx->tune_report[3] = best;
  if (out_ms) *out_ms = best;
  return PV_OK;
}

pv_status pv_autotune_report(const pv_ctx* ctx, float* h_out) {
  if (!ctx || !h_out) return PV_ERR_ARG;
  std::memcpy(h_out, ctx->tune_report, sizeof(ctx->tune_report));
  return PV_OK;
}

pv_status pv_compact_photons(pv_ctx* ctx, const pv_path_store* store, float* d_out_pos, float* d_out_energy,
                             uint32_t capacity, uint32_t* d_count) {
  if (!ctx) return PV_ERR_ARG;
  pv_status st = bind_store(ctx, store);
  if (st) return st;
  if (!d_count || (capacity && (!d_out_pos || !d_out_energy))) return fail(ctx, PV_ERR_ARG, "output is NULL");
  if ((st = wait_compaction(ctx))) return st;
  uint32_t nb = path_blocks(store->n_paths);
  CK(pv::launch_photon_count(ctx->d_scene, ctx->d_path_tiles, nb, ctx->d_pcounts, ctx->stream));
  CK(pv::launch_scan(ctx->d_pcounts, ctx->d_poffsets, nb * store->max_bounces, d_count, ctx->d_scan_tmp,
                     ctx->stream));
  CK(pv::launch_photon_scatter(ctx->d_scene, ctx->d_path_tiles, nb, store->max_bounces, ctx->d_poffsets, d_out_pos,
                               d_out_energy, capacity, ctx->stream));
  return PV_OK;
}

pv_status pv_compact_photons_noalloc(pv_ctx* ctx, const pv_path_store* store, float* d_out_pos,
                                     float* d_out_energy, uint32_t capacity, uint32_t* d_count) {
  if (!ctx) return PV_ERR_ARG;
  if (!store) return fail(ctx, PV_ERR_ARG, "store is NULL");
  if (store->max_bounces < 1 || store->max_bounces > PV_MAX_BOUNCES)
    return fail(ctx, PV_ERR_ARG, "max_bounces out of range 1..15");
  // the size check comes first: a store too large for the fixed scratch is
  // rejected before anything is bound or enqueued
  const uint64_t n = (uint64_t)path_blocks(store->n_paths) * store->max_bounces;
  uint64_t a = 0;
  if (fixed_layout(n, &a) > kFixedScratchWords)
    return fail(ctx, PV_ERR_CAPACITY,
                "store too large for the fixed compaction scratch: " + std::to_string(n) +
                    " (path blocks of 256) x (bounce rows) counts, at most " +
                    std::to_string(PV_NOALLOC_MAX_COUNTS));
  if (!ctx->fixed_scratch) return fail(ctx, PV_ERR_STATE, "fixed scratch unavailable");
  pv_status st = bind_store(ctx, store);
  if (st) return st;
  if (!d_count || (capacity && (!d_out_pos || !d_out_energy))) return fail(ctx, PV_ERR_ARG, "output is NULL");
  if ((st = wait_compaction(ctx))) return st;
  // every word the kernels read is written earlier in the same call, so
  // nothing is cleared; the scratch keeps the last call's contents
  uint32_t* counts = ctx->fixed_scratch;
  uint32_t* offsets = counts + a;
  uint32_t* tmp = offsets + a;
  const uint32_t nb = path_blocks(store->n_paths);
  CK(pv::launch_photon_count(ctx->d_scene, ctx->d_path_tiles, nb, counts, ctx->stream));
  CK(pv::launch_scan(counts, offsets, (uint32_t)n, d_count, tmp, ctx->stream));
  CK(pv::launch_photon_scatter(ctx->d_scene, ctx->d_path_tiles, nb, store->max_bounces, offsets, d_out_pos,
                               d_out_energy, capacity, ctx->stream));
  return PV_OK;
}

pv_status pv_compact_photons_async(pv_ctx* ctx, const pv_path_store* store, float* d_out_pos,
                                   float* d_out_energy, uint32_t capacity, uint32_t* d_count, void* hip_stream) {
  if (!ctx) return PV_ERR_ARG;
  pv_status st = bind_store(ctx, store);
  if (st) return st;
  if (!d_count || (capacity && (!d_out_pos || !d_out_energy))) return fail(ctx, PV_ERR_ARG, "output is NULL");
  if ((st = wait_compaction(ctx))) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (!ctx->ev_store) CK(hipEventCreateWithFlags(&ctx->ev_store, hipEventDisableTiming));
  if (!ctx->ev_compact) CK(hipEventCreateWithFlags(&ctx->ev_compact, hipEventDisableTiming));
  // after everything enqueued on the context's stream so far
  CK(hipEventRecord(ctx->ev_store, ctx->stream));
  CK(hipStreamWaitEvent(s, ctx->ev_store, 0));
  uint32_t nb = path_blocks(store->n_paths);
  CK(pv::launch_photon_count(ctx->d_scene, ctx->d_path_tiles, nb, ctx->d_pcounts, s));
  CK(pv::launch_scan(ctx->d_pcounts, ctx->d_poffsets, nb * store->max_bounces, d_count, ctx->d_scan_tmp_c, s));
  CK(pv::launch_photon_scatter(ctx->d_scene, ctx->d_path_tiles, nb, store->max_bounces, ctx->d_poffsets, d_out_pos,
                               d_out_energy, capacity, s));
  CK(hipEventRecord(ctx->ev_compact, s));
  ctx->compact_pending = true;
  return PV_OK;
}

pv_status pv_energy_forward(pv_ctx* ctx, const pv_path_store* store, const float* d_albedo, const float* d_power,
                            float* d_E) {
  if (!ctx) return PV_ERR_ARG;
  pv_status st = bind_store(ctx, store);
  if (st) return st;
  if (!d_albedo || !d_power || !d_E) return fail(ctx, PV_ERR_ARG, "NULL argument");
  CK(pv::launch_energy_fwd(ctx->d_scene, ctx->d_path_tiles, path_blocks(store->n_paths), d_albedo, d_power, d_E,
                           ctx->stream));
  return PV_OK;
}

pv_status pv_energy_backward(pv_ctx* ctx, const pv_path_store* store, const float* d_albedo, const float* d_power,
                             const float* d_gE, float* d_g_albedo, float* d_g_power) {
  if (!ctx) return PV_ERR_ARG;
  pv_status st = bind_store(ctx, store);
  if (st) return st;
  if (!d_albedo || !d_power || !d_gE || !d_g_albedo || !d_g_power) return fail(ctx, PV_ERR_ARG, "NULL argument");
  if (ctx->n_materials > 256) return fail(ctx, PV_ERR_CAPACITY, "backward supports at most 256 materials");
  CK(pv::launch_energy_bwd(ctx->d_scene, ctx->d_path_tiles, path_blocks(store->n_paths), d_albedo, d_power, d_gE,
                           ctx->n_materials, ctx->n_lights, ctx->d_partial, d_g_albedo, d_g_power, ctx->stream));
  return PV_OK;
}

// ---------------------------------------------------------------------------
// batched form: every phase of a frame is one launch over all scenes

// one frame of every scene on the batch's capture stream: transforms from the
// device pointer tables obj_in / light_in, frame number from frame_ptr
static pv_status batch_enqueue(pv_batch* b, pv_stats* d_stats, const float* const* obj_in,
                               const float* const* light_in, const uint32_t* frame_ptr) {
  pv_ctx* ctx = b->owner;
  hipStream_t st = b->cap_stream;
  CK(pv::launch_frame_begin(b->d_scenes, (int)b->n, obj_in, light_in, st));
  if (b->n == 1) {
    // one scene (its context is the owner): the plain frame's refit, the
    // topologies' boxes as unions over leaf-order ranges, with many more
    // threads than the per-object level-by-level refit and the same boxes
    CK(pv::launch_transform_objects(b->d_scenes, b->d_xf_tiles, b->n_xf_tiles, st));
    CK(pv::launch_refit_objects(b->d_scenes, ctx->lw, ctx->n_objects, ctx->hs.n_obj_nodes, st));
  } else {
    CK(pv::launch_update_objects(b->d_scenes, b->d_obj_tiles, b->n_obj_tiles, b->d_xf_tiles, b->n_xf_tiles, st));
  }
  CK(pv::launch_build_top(b->d_scenes, (int)b->n, st));
  CK(pv::launch_verify(b->d_scenes, b->d_path_tiles, b->n_path_tiles, b->d_gbase, (int)b->n, b->vw, b->d_block_cnt,
                       d_stats, b->stack_moved, verify_blocks(ctx), ctx->verify_min_active, b->d_scan_tmp, st));
  // distribution maps: compute DM_C, prune, fill, scene by scene (each
  // rewrites its own tiles' replace counts before the queue is built)
  for (const pv_batch::Dm& d : b->dms)
    CK(pv::launch_dm_update(b->d_scenes, b->d_scenes + d.scene, b->d_path_tiles + d.tile_base, d.n_tiles, d.cells,
                            d.n_lights, d.D, b->d_block_cnt + d.tile_base, b->seed, 0, frame_ptr, st));
  CK(pv::launch_scan(b->d_block_cnt, b->d_offsets, b->n_path_tiles, b->d_qcount, b->d_scan_tmp, st));
  CK(pv::launch_scatter_queue(b->d_scenes, b->d_path_tiles, b->n_path_tiles, b->d_offsets, b->d_queue, st));
  CK(pv::launch_retrace(b->d_scenes, b->d_gbase, (int)b->n, b->d_queue, b->d_qcount, b->T, b->seed, 0,
                        frame_ptr, d_stats, (uint32_t)(ctx->n_cu * ctx->retrace_blocks_per_cu), ctx->retrace_variant,
                        b->stack_entries, ctx->walk_min_active, b->ow, st));
  CK(pv::launch_photon_count(b->d_scenes, b->d_path_tiles, b->n_path_tiles, b->d_pcounts, st));
  CK(pv::launch_scan(b->d_pcounts, b->d_poffsets, b->n_counts, b->d_ptotal, b->d_scan_tmp, st));
  CK(pv::launch_photon_scatter(b->d_scenes, b->d_path_tiles, b->n_path_tiles, b->max_bounces, b->d_poffsets,
                               b->d_out_pos, b->d_out_en, b->capacity, st));
  CK(pv::launch_scene_photon_base(b->d_scenes, (int)b->n, b->d_poffsets, b->d_ptotal, b->d_pbase, st));
  return PV_OK;
}

pv_status pv_batch_create(pv_batch** out, pv_ctx* const* contexts, const pv_path_store* stores, uint32_t n,
                          const float* const* d_obj_xf, const float* const* d_light_xf, float threshold,
                          uint64_t seed) {
  if (!out || !contexts || !stores || n == 0 || !d_obj_xf || !d_light_xf) return PV_ERR_ARG;
  *out = nullptr;
  pv_ctx* ctx = contexts[0];
  if (!ctx) return PV_ERR_ARG;
  if (std::isnan(threshold)) return fail(ctx, PV_ERR_ARG, "threshold is NaN");
  try {
    pv_batch* b = new pv_batch();
    b->owner = ctx;
    b->stream = ctx->stream;
    b->n = n;
    b->T = threshold;
    b->seed = seed;
    b->retrace_blocks = (uint32_t)ctx->n_cu * 8;
    std::vector<SceneDev> table(n);
    std::vector<uint2> ptiles, otiles, xtiles;
    std::vector<uint32_t> gbase(n + 1, 0);
    uint64_t total_paths = 0, counts = 0, cap = 0, task_cap = 0;
    for (uint32_t i = 0; i < n; ++i) {
      pv_ctx* c = contexts[i];
      const pv_path_store* st = &stores[i];
      auto bad = [&](const char* m) {
        delete b;
        return fail(ctx, PV_ERR_ARG, std::string("batch scene ") + std::to_string(i) + ": " + m);
      };
      if (!c || !c->uploaded) return bad("context without a scene");
      if (c->compact_pending) {  // an overlapped compaction still reads this store
        if (hipEventSynchronize(c->ev_compact) != hipSuccess) return bad("overlapped compaction failed");
        c->compact_pending = false;
      }
      if (!st->d_pos_hit || !st->d_energy || !st->d_origin || !st->d_info) return bad("store has a NULL array");
      if (st->max_bounces < 1 || st->max_bounces > PV_MAX_BOUNCES) return bad("max_bounces out of range");
      if (st->stride < st->n_paths || st->stride % 64 != 0) return bad("bad stride");
      if ((c->n_objects && !d_obj_xf[i]) || !d_light_xf[i]) return bad("transform array is NULL");
      b->n_obj.push_back(c->n_objects);
      uint32_t lp = 0;
      for (uint32_t l = 0; l < c->n_lights; ++l) lp += c->h_light_paths[l];
      if (lp != st->n_paths) return bad("light path counts do not add up to n_paths");
      b->stack_entries = std::max(b->stack_entries, c->stack_entries);
      b->max_bounces = std::max(b->max_bounces, st->max_bounces);
      b->stack_moved = std::max(b->stack_moved, c->stack_moved);
      SceneDev hs = c->hs;
      hs.pos = static_cast<float4*>(st->d_pos_hit);
      hs.energy = static_cast<float4*>(st->d_energy);
      hs.origin = st->d_origin;
      hs.info = st->d_info;
      hs.stride = st->stride;
      hs.n_paths = st->n_paths;
      hs.B = st->max_bounces;
      hs.n_blocks = path_blocks(st->n_paths);
      hs.count_base = (uint32_t)counts;
      hs.gpath_base = (uint32_t)total_paths;
      hs.tile_base = (uint32_t)ptiles.size();
      hs.task_base = (uint32_t)task_cap;
      table[i] = hs;
      if (c->dm_enabled)
        b->dms.push_back(pv_batch::Dm{i, hs.tile_base, hs.n_blocks, c->dm_cells, c->n_lights, pv::DmWork{}});
      gbase[i] = (uint32_t)total_paths;
      for (uint2 t : make_tiles(i, st->n_paths)) ptiles.push_back(t);
      for (uint32_t o = 0; o < c->n_objects; ++o) otiles.push_back(make_uint2(i, o));
      for (uint2 t : xf_tiles(i, c->h_obj_tris.data(), c->n_objects)) xtiles.push_back(t);
      total_paths += st->n_paths;
      counts += (uint64_t)hs.n_blocks * st->max_bounces;
      cap += (uint64_t)st->n_paths * st->max_bounces;
      task_cap += (uint64_t)hs.n_blocks * pv::kBlock * st->max_bounces;
    }
    gbase[n] = (uint32_t)total_paths;
    if (total_paths > kMaxPaths || cap >= (1ull << 32) || task_cap >= (1ull << 32)) {
      delete b;
      return fail(ctx, PV_ERR_CAPACITY, "batch too large");
    }
    Alloc& A = b->mem;
    hipStream_t s = b->stream;
    auto chk = [&](hipError_t e) { return e == hipSuccess; };
    bool ok = chk(upload(A, &b->d_scenes, table.data(), n, s)) && chk(upload(A, &b->d_path_tiles, ptiles.data(), ptiles.size(), s)) &&
              chk(upload(A, &b->d_obj_tiles, otiles.data(), otiles.size(), s)) &&
              chk(upload(A, &b->d_xf_tiles, xtiles.data(), xtiles.size(), s)) &&
              chk(upload(A, &b->d_gbase, gbase.data(), gbase.size(), s)) &&
              chk(dalloc(A, &b->d_block_cnt, ptiles.size())) && chk(dalloc(A, &b->d_offsets, ptiles.size())) &&
              chk(dalloc(A, &b->d_queue, total_paths)) && chk(dalloc(A, &b->d_qcount, 1)) &&
              chk(dalloc(A, &b->d_pcounts, counts)) &&
              chk(dalloc(A, &b->d_poffsets, counts)) && chk(dalloc(A, &b->d_ptotal, 1)) &&
              chk(dalloc(A, &b->d_pbase, n + 1)) && chk(dalloc(A, &b->d_frame, 1)) &&
              chk(dalloc(A, &b->d_scan_tmp, pv::scan_tmp_words((uint32_t)std::max<uint64_t>(counts, ptiles.size())))) &&
              chk(dalloc(A, &b->d_out_pos, 3 * cap)) && chk(dalloc(A, &b->d_out_en, 3 * cap)) &&
              chk(dalloc(A, &b->vw.tmp, task_cap)) && chk(dalloc(A, &b->vw.tasks, task_cap)) &&
              chk(dalloc(A, &b->vw.tcount, ptiles.size())) && chk(dalloc(A, &b->vw.toff, ptiles.size())) &&
              chk(dalloc(A, &b->vw.total, 1)) && chk(dalloc(A, &b->vw.first, total_paths)) &&
              (b->ow.tiles = pv::order_tiles((uint32_t)total_paths), true) &&
              chk(dalloc(A, &b->ow.queue, total_paths)) && chk(dalloc(A, &b->ow.hist, 8 * (size_t)b->ow.tiles)) &&
              chk(dalloc(A, &b->ow.hoff, 8 * (size_t)b->ow.tiles)) && chk(dalloc(A, &b->ow.htotal, 1)) &&
              chk(dalloc(A, &b->ow.scan_tmp, pv::scan_tmp_words(8 * b->ow.tiles))) &&
              chk(dalloc(A, &b->ow.deal, (size_t)pv::kDealGroups * pv::kDealStride)) &&
              chk(dalloc(A, &b->vw.deal, (size_t)pv::kDealGroups * pv::kDealStride)) &&
              chk(dalloc(A, &b->vw.part, 4 * ptiles.size() + 2 * (size_t)pv::verify_finish_blocks(verify_blocks_max(ctx)))) &&
              chk(upload(A, &b->d_obj_in, const_cast<const float**>(d_obj_xf), n, s)) &&
              chk(upload(A, &b->d_light_in, const_cast<const float**>(d_light_xf), n, s));
    for (pv_batch::Dm& d : b->dms) {
      pv::DmWork& D = d.D;
      ok = ok && chk(dalloc(A, &D.dm_c, d.cells)) && chk(dalloc(A, &D.pruned, d.cells)) &&
           chk(dalloc(A, &D.def, d.cells)) && chk(dalloc(A, &D.dex, (size_t)d.cells + 1)) &&
           chk(dalloc(A, &D.tcnt, d.n_tiles)) && chk(dalloc(A, &D.toff, d.n_tiles)) && chk(dalloc(A, &D.ttotal, 1)) &&
           chk(dalloc(A, &D.rank0, PV_MAX_LIGHTS)) && chk(dalloc(A, &D.scan_tmp, pv::scan_tmp_words(d.cells))) &&
           chk(dalloc(A, &D.scan_tmp2, pv::scan_tmp_words(d.n_tiles)));
    }
    if (!ok || hipStreamSynchronize(s) != hipSuccess) {
      delete b;
      return fail(ctx, PV_ERR_OOM, "batch allocation failed");
    }
    if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
      delete b;
      return fail(ctx, PV_ERR_HIP, "batch stream/event creation failed");
    }
    b->n_path_tiles = (uint32_t)ptiles.size();
    b->n_obj_tiles = (uint32_t)otiles.size();
    b->n_xf_tiles = (uint32_t)xtiles.size();
    b->n_counts = (uint32_t)counts;
    b->capacity = (uint32_t)cap;
    *out = b;
    return PV_OK;
  } catch (const std::exception& e) {
    return fail(ctx, PV_ERR_OOM, std::string("host exception: ") + e.what());
  }
}

void pv_batch_destroy(pv_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  if (b->cap_stream) (void)hipStreamSynchronize(b->cap_stream);
  delete b;
}

pv_status pv_batch_frame(pv_batch* b, uint32_t frame, pv_stats* d_stats) {
  if (!b) return PV_ERR_ARG;
  pv_ctx* ctx = b->owner;
  CK(hipMemcpyAsync(b->d_frame, &frame, sizeof(frame), hipMemcpyHostToDevice, b->stream));
  // the frame runs on the batch's stream, ordered after everything the caller
  // enqueued on the owner's stream and before anything enqueued there later
  CK(hipEventRecord(b->ev_in, b->stream));
  CK(hipStreamWaitEvent(b->cap_stream, b->ev_in, 0));
  if (!b->captured || b->captured_stats != d_stats) {
    if (b->exec) {
      CK(hipGraphExecDestroy(b->exec));
      b->exec = nullptr;
    }
    if (b->graph) {
      CK(hipGraphDestroy(b->graph));
      b->graph = nullptr;
    }
    CK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    pv_status st = batch_enqueue(b, d_stats, b->d_obj_in, b->d_light_in, b->d_frame);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (st != PV_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    CK(e);
    b->graph = g;
    CK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->captured = true;
    b->captured_stats = d_stats;
  }
  CK(hipGraphLaunch(b->exec, b->cap_stream));
  CK(hipEventRecord(b->ev_out, b->cap_stream));
  CK(hipStreamWaitEvent(b->stream, b->ev_out, 0));
  return PV_OK;
}

pv_status pv_batch_frames(pv_batch* b, uint32_t first_frame, uint32_t k, const float* const* d_obj_xf,
                          const float* const* d_light_xf, pv_stats* d_stats) {
  if (!b) return PV_ERR_ARG;
  pv_ctx* ctx = b->owner;
  if (k == 0 || k > PV_BATCH_MAX_FRAMES) return fail(ctx, PV_ERR_ARG, "frame count out of range");
  if (!d_obj_xf || !d_light_xf) return fail(ctx, PV_ERR_ARG, "NULL transform table");
  for (uint32_t f = 0; f < k; ++f)
    for (uint32_t i = 0; i < b->n; ++i)
      if ((b->n_obj[i] && !d_obj_xf[(size_t)f * b->n + i]) || !d_light_xf[(size_t)f * b->n + i])
        return fail(ctx, PV_ERR_ARG, "transform array is NULL");
  if (first_frame > UINT32_MAX - (k - 1)) return fail(ctx, PV_ERR_ARG, "frame numbers overflow");
  if (k > b->tab_frames) {
    // larger tables: nothing enqueued may still read or write the old ones
    CK(hipStreamSynchronize(b->stream));
    CK(hipStreamSynchronize(b->cap_stream));
    if (b->multi_exec) CK(hipGraphExecDestroy(b->multi_exec));
    if (b->multi_graph) CK(hipGraphDestroy(b->multi_graph));
    b->multi_exec = nullptr;
    b->multi_graph = nullptr;
    b->multi_k = 0;
    b->tab_mem.release();
    b->tab_frames = 0;
    CK(dalloc(b->tab_mem, &b->d_frames, k));
    CK(dalloc(b->tab_mem, &b->d_obj_tab, (size_t)k * b->n));
    CK(dalloc(b->tab_mem, &b->d_light_tab, (size_t)k * b->n));
    b->tab_frames = k;
  }
  std::vector<uint32_t> frames(k);
  for (uint32_t f = 0; f < k; ++f) frames[f] = first_frame + f;
  CK(hipMemcpyAsync(b->d_frames, frames.data(), sizeof(uint32_t) * k, hipMemcpyHostToDevice, b->stream));
  CK(hipMemcpyAsync(b->d_obj_tab, d_obj_xf, sizeof(float*) * k * b->n, hipMemcpyHostToDevice, b->stream));
  CK(hipMemcpyAsync(b->d_light_tab, d_light_xf, sizeof(float*) * k * b->n, hipMemcpyHostToDevice, b->stream));
  CK(hipEventRecord(b->ev_in, b->stream));
  CK(hipStreamWaitEvent(b->cap_stream, b->ev_in, 0));
  if (b->multi_k != k || b->multi_stats != d_stats) {
    if (b->multi_exec) CK(hipGraphExecDestroy(b->multi_exec));
    if (b->multi_graph) CK(hipGraphDestroy(b->multi_graph));
    b->multi_exec = nullptr;
    b->multi_graph = nullptr;
    b->multi_k = 0;
    CK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    pv_status st = PV_OK;
    for (uint32_t f = 0; f < k && st == PV_OK; ++f)
      st = batch_enqueue(b, d_stats, b->d_obj_tab + (size_t)f * b->n, b->d_light_tab + (size_t)f * b->n,
                         b->d_frames + f);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (st != PV_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    CK(e);
    b->multi_graph = g;
    CK(hipGraphInstantiate(&b->multi_exec, b->multi_graph, nullptr, nullptr, 0));
    b->multi_k = k;
    b->multi_stats = d_stats;
  }
  CK(hipGraphLaunch(b->multi_exec, b->cap_stream));
  CK(hipEventRecord(b->ev_out, b->cap_stream));
  CK(hipStreamWaitEvent(b->stream, b->ev_out, 0));
  return PV_OK;
}

pv_status pv_batch_set_transforms(pv_batch* b, const float* const* d_obj_xf, const float* const* d_light_xf) {
  if (!b || !d_obj_xf || !d_light_xf) return PV_ERR_ARG;
  pv_ctx* ctx = b->owner;
  CK(hipMemcpyAsync(b->d_obj_in, d_obj_xf, sizeof(float*) * b->n, hipMemcpyHostToDevice, b->stream));
  CK(hipMemcpyAsync(b->d_light_in, d_light_xf, sizeof(float*) * b->n, hipMemcpyHostToDevice, b->stream));
  return PV_OK;
}

pv_status pv_batch_copy_photons(pv_batch* b, float* d_pos, float* d_energy, uint32_t capacity,
                                uint32_t* d_scene_base) {
  if (!b || !d_scene_base || (capacity && (!d_pos || !d_energy))) return PV_ERR_ARG;
  pv_ctx* ctx = b->owner;
  uint32_t n = std::min(capacity, b->capacity);
  if (n) {
    CK(hipMemcpyAsync(d_pos, b->d_out_pos, 12 * (size_t)n, hipMemcpyDeviceToDevice, b->stream));
    CK(hipMemcpyAsync(d_energy, b->d_out_en, 12 * (size_t)n, hipMemcpyDeviceToDevice, b->stream));
  }
  CK(hipMemcpyAsync(d_scene_base, b->d_pbase, 4 * (size_t)(b->n + 1), hipMemcpyDeviceToDevice, b->stream));
  return PV_OK;
}

}  // extern "C"
