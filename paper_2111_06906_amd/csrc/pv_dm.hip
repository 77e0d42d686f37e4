// Distribution maps of Section 3.1 on the device: after the origin update
// (verification), "Compute DM_C" counts the paths of every cell, "Prune
// paths" re-samples paths of over-full cells with the probability of
// Equation 1, and "Fill DM_C" gives the paths to re-sample the cells still
// below their target; the re-trace then draws their new light samples inside
// those cells.  All kernels take path tiles (scene, first path) of kBlock
// paths; counts are integer and every decision is either an integer or an
// FP32 comparison taken the same way by the CPU oracle.
#include "pv_device.h"
#include "pv_launch.h"

namespace pv {

namespace {

__device__ inline uint32_t lane() { return threadIdx.x & 63u; }
__device__ inline uint64_t lanes_below() { return (1ull << lane()) - 1ull; }

__device__ inline int light_index(const SceneDev& S, uint32_t p) {
  const PV_GLOBAL LightDev* lights = G(S.lights);
  for (uint32_t l = 0; l < S.n_lights; ++l)
    if (p - lights[l].path_base < lights[l].path_count) return (int)l;
  return -1;
}

// a path re-sampled from its light: replace without reuse of the light sample
__device__ inline bool resampled(uint32_t w) { return info_replace(w) && !info_reuse(w); }

// cells of all lights counted in LDS when they fit (one atomic per path into
// LDS, one per non-empty cell and block into global memory)
constexpr uint32_t kLdsCells = 8192;

__device__ inline void hist_add(uint32_t* lds, bool use_lds, uint32_t* glob, uint32_t cell) {
  if (use_lds)
    atomicAdd(lds + cell, 1u);
  else
    atomicAdd(glob + cell, 1u);
}

__device__ inline void hist_flush(const uint32_t* lds, uint32_t* glob, uint32_t cells) {
  __syncthreads();
  for (uint32_t c = threadIdx.x; c < cells; c += kBlock)
    if (lds[c]) atomicAdd(glob + c, lds[c]);
}

}  // namespace

// zero the per-cell counts (a kernel, so that the sequence can be captured)
__global__ __launch_bounds__(kBlock) void k_dm_clear(uint32_t* __restrict__ a, uint32_t* __restrict__ b,
                                                     uint32_t cells) {
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < cells; i += gridDim.x * kBlock) {
    a[i] = 0;
    b[i] = 0;
  }
}

// Compute DM_C: every path whose light sample survived the origin update
// counts in its cell; a moved light's path takes the cell of its updated
// origin and kept direction, and one the parametrisation cannot place is
// marked for re-sampling.
__global__ __launch_bounds__(kBlock) void k_dm_count(const SceneDev* __restrict__ scenes,
                                                     const uint2* __restrict__ tiles, uint32_t* __restrict__ dm_c) {
  __shared__ uint32_t h[kLdsCells];
  const uint2 tile = tiles[blockIdx.x];
  const SceneDev& S = scenes[tile.x];
  const uint32_t cells = S.dm_off[S.n_lights];
  const bool use_lds = cells <= kLdsCells;
  if (use_lds)
    for (uint32_t c = threadIdx.x; c < cells; c += kBlock) h[c] = 0;
  __syncthreads();
  const uint32_t p = tile.y + threadIdx.x;
  if (p < S.n_paths) {
    const int l = light_index(S, p);
    uint32_t w = G(S.info)[p];
    if (l >= 0 && !resampled(w)) {
      uint32_t cell = info_cell(w);
      bool ok = true;
      if (G(S.light_moved)[l]) {
        const size_t stride = S.stride;
        const PV_GLOBAL float* org = G(S.origin);
        const float3 x0 = f3(org[p], org[stride + p], org[2 * stride + p]);
        const float3 x1 = xyz(G(S.pos)[p]);
        const float3 d = sub(x1, x0);
        const float len = length(d);
        const float* xf = G(S.light_xf_cur) + 12 * l;
        const LightDev lt = G(S.lights)[l];
        const int32_t c = len > 0.0f ? dm_cell(xf, lt, S.dm, x0, mul(d, 1.0f / len)) : -1;
        ok = c >= 0;
        if (ok) {
          cell = (uint32_t)c;
          w = info_pack(cell, info_nseg(w), info_start(w), info_replace(w), info_reuse(w));
        } else {
          w = info_pack(0, info_nseg(w), 0, 1, 0);
        }
        G(S.info)[p] = w;
      }
      if (ok) hist_add(h, use_lds, dm_c, S.dm_off[l] + cell);
    }
  }
  if (use_lds) hist_flush(h, dm_c, cells);
}

// Prune paths (Equation 1): a path of a cell holding C > DM_T paths is
// re-sampled with probability (C - DM_T) / C, decided in FP32 against one
// Philox uniform (vertex 0, tag 2); all decisions use the counts before any
// pruning (Section 4's two passes: decide, then count the pruned paths).
__global__ __launch_bounds__(kBlock) void k_dm_prune(const SceneDev* __restrict__ scenes,
                                                     const uint2* __restrict__ tiles, const uint32_t* __restrict__ dm_c,
                                                     uint32_t* __restrict__ pruned, uint64_t seed, uint32_t frame,
                                                     const uint32_t* __restrict__ frame_ptr) {
  __shared__ uint32_t h[kLdsCells];
  if (frame_ptr) frame = *frame_ptr;  // a captured frame reads its number from device memory
  const uint2 tile = tiles[blockIdx.x];
  const SceneDev& S = scenes[tile.x];
  const uint32_t cells = S.dm_off[S.n_lights];
  const bool use_lds = cells <= kLdsCells;
  if (use_lds)
    for (uint32_t c = threadIdx.x; c < cells; c += kBlock) h[c] = 0;
  __syncthreads();
  const uint32_t p = tile.y + threadIdx.x;
  if (p < S.n_paths) {
    const int l = light_index(S, p);
    const uint32_t w = G(S.info)[p];
    if (l >= 0 && !resampled(w)) {
      const LightDev lt = G(S.lights)[l];
      const uint32_t at = S.dm_off[l] + info_cell(w);
      const uint32_t tgt = dm_target(lt.path_count, S.dm_off[l + 1] - S.dm_off[l], info_cell(w));
      const uint32_t C = dm_c[at];
      if (C > tgt) {
        float u[4];
        draw4(seed, p, frame, 0, 2, u);
        const float prob = __fdiv_rn((float)(C - tgt), (float)C);
        if (u[0] < prob) {
          G(S.info)[p] = info_pack(info_cell(w), info_nseg(w), 0, 1, 0);
          hist_add(h, use_lds, pruned, at);
        }
      }
    }
  }
  if (use_lds) hist_flush(h, pruned, cells);
}

// deficit of every cell, max(0, DM_T - (DM_C - pruned)), for the scan
__global__ __launch_bounds__(kBlock) void k_dm_deficit(const SceneDev* __restrict__ scenes,
                                                       const uint32_t* __restrict__ dm_c,
                                                       const uint32_t* __restrict__ pruned,
                                                       uint32_t* __restrict__ def) {
  const SceneDev& S = scenes[0];
  const uint32_t cells = S.dm_off[S.n_lights];
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < cells; i += gridDim.x * kBlock) {
    uint32_t l = 0;
    while (l + 1 < S.n_lights && i >= S.dm_off[l + 1]) ++l;
    const uint32_t c = i - S.dm_off[l];
    const uint32_t tgt = dm_target(G(S.lights)[l].path_count, S.dm_off[l + 1] - S.dm_off[l], c);
    const uint32_t have = dm_c[i] - pruned[i];
    def[i] = tgt > have ? tgt - have : 0u;
  }
}

// re-sampled paths per tile (the ranks of the fill)
__global__ __launch_bounds__(kBlock) void k_dm_flags(const SceneDev* __restrict__ scenes,
                                                     const uint2* __restrict__ tiles, uint32_t* __restrict__ tcnt) {
  __shared__ uint32_t ws[kBlock / 64];
  const uint2 tile = tiles[blockIdx.x];
  const SceneDev& S = scenes[tile.x];
  const uint32_t p = tile.y + threadIdx.x;
  const bool f = p < S.n_paths && light_index(S, p) >= 0 && resampled(G(S.info)[p]);
  const uint64_t b = __ballot(f);
  if (lane() == 0) ws[threadIdx.x >> 6] = (uint32_t)__popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int i = 0; i < kBlock / 64; ++i) t += ws[i];
    tcnt[blockIdx.x] = t;
  }
}

// rank of each light's first path among the re-sampled paths of the store:
// the scanned count of the tiles before its first path's tile plus the
// re-sampled paths of that tile ahead of it (one wave per light, a ballot
// per 64 of those paths)
__global__ __launch_bounds__(64) void k_dm_rank0(const SceneDev* __restrict__ scenes,
                                                 const uint32_t* __restrict__ toff, uint32_t* __restrict__ rank0) {
  const SceneDev& S = scenes[0];
  const uint32_t l = blockIdx.x;
  if (l >= S.n_lights) return;
  const uint32_t base = G(S.lights)[l].path_base;
  const uint32_t t0 = base / kBlock * kBlock;
  uint32_t r = 0;
  for (uint32_t q0 = t0; q0 < base; q0 += 64) {
    const uint32_t q = q0 + lane();
    const bool f = q < base && light_index(S, q) >= 0 && resampled(G(S.info)[q]);
    r += (uint32_t)__popcll(__ballot(f));
  }
  if (lane() == 0) rank0[l] = (base / kBlock < S.n_blocks ? toff[base / kBlock] : 0u) + r;
}

// Fill DM_C: the i-th re-sampled path of a light (path order) takes the cell
// where the running sum of the deficits passes i ('dex': exclusive scan of
// the deficits of all cells, dex[cells] their total); also the tile's
// replace count for the work queue.
__global__ __launch_bounds__(kBlock) void k_dm_fill(const SceneDev* __restrict__ scenes,
                                                    const uint2* __restrict__ tiles, const uint32_t* __restrict__ dex,
                                                    const uint32_t* __restrict__ toff,
                                                    const uint32_t* __restrict__ rank0,
                                                    uint32_t* __restrict__ block_cnt) {
  __shared__ uint32_t ws[kBlock / 64], wr[kBlock / 64];
  const uint2 tile = tiles[blockIdx.x];
  const SceneDev& S = scenes[tile.x];
  const uint32_t p = tile.y + threadIdx.x;
  const bool have = p < S.n_paths;
  const int l = have ? light_index(S, p) : -1;
  uint32_t w = have ? G(S.info)[p] : 0u;
  const bool f = l >= 0 && resampled(w);
  const uint64_t b = __ballot(f);
  const uint64_t rb = __ballot(have && info_replace(w));
  if (lane() == 0) {
    ws[threadIdx.x >> 6] = (uint32_t)__popcll(b);
    wr[threadIdx.x >> 6] = (uint32_t)__popcll(rb);
  }
  __syncthreads();
  uint32_t before = 0;
  for (uint32_t i = 0; i < (threadIdx.x >> 6); ++i) before += ws[i];
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int i = 0; i < kBlock / 64; ++i) t += wr[i];
    block_cnt[blockIdx.x] = t;  // resampled paths already carry the replace bit
  }
  if (!f) return;
  const uint32_t i = toff[blockIdx.x] + before + (uint32_t)__popcll(b & lanes_below()) - rank0[l];
  const uint32_t lo = S.dm_off[l], cells = S.dm_off[l + 1] - lo, base = dex[lo];
  // first cell c of the light with dex[c + 1] - dex[lo] > i
  uint32_t a = 0, e = cells;
  while (a < e) {
    const uint32_t m = (a + e) >> 1;
    if (dex[lo + m + 1] - base > i)
      e = m;
    else
      a = m + 1;
  }
  const uint32_t cell = a < cells ? a : i % cells;
  G(S.info)[p] = info_pack(cell, info_nseg(w), info_start(w), 1, 0);
}

hipError_t launch_dm_update(const SceneDev* table, const SceneDev* scene, const uint2* tiles, uint32_t n_tiles,
                            uint32_t cells, uint32_t n_lights, const DmWork& D, uint32_t* block_cnt, uint64_t seed,
                            uint32_t frame, const uint32_t* frame_ptr, hipStream_t s) {
  if (!n_tiles || !cells) return hipSuccess;
  if (n_lights < 1 || n_lights > PV_MAX_LIGHTS) return hipErrorInvalidValue;
  const uint32_t cb = std::min(1024u, (cells + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_dm_clear, dim3(cb), dim3(kBlock), 0, s, D.dm_c, D.pruned, cells);
  hipLaunchKernelGGL(k_dm_count, dim3(n_tiles), dim3(kBlock), 0, s, table, tiles, D.dm_c);
  hipLaunchKernelGGL(k_dm_prune, dim3(n_tiles), dim3(kBlock), 0, s, table, tiles, D.dm_c, D.pruned, seed, frame,
                     frame_ptr);
  hipLaunchKernelGGL(k_dm_deficit, dim3(cb), dim3(kBlock), 0, s, scene, D.dm_c, D.pruned, D.def);
  hipError_t e = launch_scan(D.def, D.dex, cells, D.dex + cells, D.scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dm_flags, dim3(n_tiles), dim3(kBlock), 0, s, table, tiles, D.tcnt);
  e = launch_scan(D.tcnt, D.toff, n_tiles, D.ttotal, D.scan_tmp2, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dm_rank0, dim3(n_lights), dim3(64), 0, s, scene, D.toff, D.rank0);
  hipLaunchKernelGGL(k_dm_fill, dim3(n_tiles), dim3(kBlock), 0, s, table, tiles, D.dex, D.toff, D.rank0,
                     block_cnt);
  return hipGetLastError();
}

}  // namespace pv
