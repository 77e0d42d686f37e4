// Host-callable launch wrappers of the library's kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "pv_device.h"

namespace pv {

// rows ids[i] of dst (n_rows rows of 12 floats) take m[i] (n <= 64; the last
// entry of a repeated id wins, ids >= n_rows are skipped)
hipError_t launch_scatter_xf(float* dst, uint32_t n_rows, const uint32_t* ids, const float* m, uint32_t n,
                             hipStream_t s);
hipError_t launch_frame_begin(SceneDev* scenes, int n_scenes, const float* const* obj_in,
                              const float* const* light_in, hipStream_t s);
// moved objects: world triangles (xf_tiles: (scene << 8 | object, first
// triangle) per kBlock triangles), then their hierarchies' boxes (tiles:
// (scene, object))
hipError_t launch_update_objects(SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, const uint2* xf_tiles,
                                 uint32_t n_xf_tiles, hipStream_t s);
// world triangles of the moved objects only (xf_tiles as above)
hipError_t launch_transform_objects(SceneDev* scenes, const uint2* xf_tiles, uint32_t n_xf_tiles, hipStream_t s);
// boxes of the moved objects' upload-time topologies (one scene) as unions
// over leaf-order ranges (the box pyramid of W), their object boxes and roots
hipError_t launch_refit_objects(SceneDev* scenes, LbvhWork W, uint32_t n_obj, uint32_t n_obj_nodes, hipStream_t s);
// every object's hierarchy rebuilt from its current world triangles (one
// scene): linear BVH over Morton codes, into the objects' rebuild regions; an
// object whose tree is deeper than max_depth keeps its current hierarchy
hipError_t launch_rebuild_objects(SceneDev* scenes, LbvhWork W, uint32_t n_obj, uint32_t max_depth, hipStream_t s);
// sort tiles of the rebuild for n_dyn triangles (W.hist holds 256 per tile)
uint32_t lbvh_sort_tiles(uint32_t n_dyn);
// entries of W.pyr (two float4 each) for n_dyn triangles
uint32_t lbvh_pyramid_entries(uint32_t n_dyn);
hipError_t launch_build_top(SceneDev* scenes, int n_scenes, hipStream_t s);
// Verification of every path of the tiles: scan, task list, traversal of the
// box-hit segments, information words of the paths with tasks, per-tile
// replace counts into block_cnt.  'gbase' / 'n_scenes': scene path ranges
// (global path ids); 'stack': traversal stack entries per lane (stack_entries
// of the moved objects' hierarchy depths, at most kMaxStack); 'trace_blocks':
// grid of the traversal kernel; 'min_active': its walk yield threshold;
// 'scan_tmp': scan_tmp_words(n_tiles) words.
hipError_t launch_verify(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, const uint32_t* gbase,
                         int n_scenes, VerifyWork W, uint32_t* block_cnt, pv_stats* stats, uint32_t stack,
                         uint32_t trace_blocks, int min_active, uint32_t* scan_tmp, hipStream_t s);
// blocks of the finishing kernel for a traversal grid (sizes W.part: 4 words
// per path tile plus 2 per finishing block)
uint32_t verify_finish_blocks(uint32_t trace_blocks);
hipError_t launch_scan(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total,
                       uint32_t* tile_tmp, hipStream_t s);
uint32_t scan_tmp_words(uint32_t n);
hipError_t launch_scatter_queue(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, const uint32_t* offsets,
                                uint32_t* queue, hipStream_t s);
hipError_t launch_mark_all(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, uint32_t* block_cnt,
                           hipStream_t s);
// Scratch of the re-trace's work order: the reordered queue (as many entries
// as the queue can hold), bucket counts per tile and their scan.
struct OrderWork {
  uint32_t* queue;     // [max entries]
  uint32_t* hist;      // [8 * tiles]
  uint32_t* hoff;      // [8 * tiles]
  uint32_t* htotal;    // [1]
  uint32_t* scan_tmp;  // scan_tmp_words(8 * tiles)
  uint32_t* deal;      // [kDealGroups * kDealStride] refill counters of the re-trace
  uint32_t tiles;      // order_tiles(max entries)
};
uint32_t order_tiles(uint32_t max_entries);
// queue_in / qcount: the work queue (ascending path ids) and its length; the
// paths are re-traced in the order of their first invalid segment
hipError_t launch_retrace(const SceneDev* scenes, const uint32_t* gbase, int n_scenes, const uint32_t* queue_in,
                          const uint32_t* qcount, float T, uint64_t seed, uint32_t frame,
                          const uint32_t* frame_ptr, pv_stats* stats, uint32_t n_blocks, int variant, uint32_t stack,
                          int min_active, const OrderWork& O, hipStream_t s);
hipError_t launch_photon_count(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, uint32_t* counts,
                               hipStream_t s);
hipError_t launch_photon_scatter(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, uint32_t B,
                                 const uint32_t* offsets, float* out_pos, float* out_e, uint32_t capacity,
                                 hipStream_t s);
hipError_t launch_scene_photon_base(const SceneDev* scenes, int n_scenes, const uint32_t* offsets, const uint32_t* total,
                                    uint32_t* base, hipStream_t s);
// Scratch of the distribution-map update (cells: all lights' cells)
struct DmWork {
  uint32_t* dm_c;      // [cells] paths counted per cell (Compute DM_C)
  uint32_t* pruned;    // [cells] paths pruned per cell
  uint32_t* def;       // [cells] deficits
  uint32_t* dex;       // [cells + 1] their exclusive scan, then the total
  uint32_t* tcnt;      // [tiles] re-sampled paths per path tile
  uint32_t* toff;      // [tiles] their exclusive scan
  uint32_t* ttotal;    // [1]
  uint32_t* rank0;     // [PV_MAX_LIGHTS] rank of each light's first path among the re-sampled ones
  uint32_t* scan_tmp;  // scan_tmp_words(cells)
  uint32_t* scan_tmp2; // scan_tmp_words(tiles)
};
// Compute DM_C, prune (Equation 1), fill (Section 3.1) on one scene's store
// (information words updated, tiles' replace counts into block_cnt[0 ..
// n_tiles)).  tiles index the descriptor table 'table', and every tile names
// the same scene, 'scene'; the frame number is *frame_ptr when frame_ptr is
// not NULL (graph replays), else 'frame'.
hipError_t launch_dm_update(const SceneDev* table, const SceneDev* scene, const uint2* tiles, uint32_t n_tiles,
                            uint32_t cells, uint32_t n_lights, const DmWork& D, uint32_t* block_cnt, uint64_t seed,
                            uint32_t frame, const uint32_t* frame_ptr, hipStream_t s);
hipError_t launch_energy_fwd(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, const float* albedo,
                             const float* power, float* E, hipStream_t s);
hipError_t launch_energy_bwd(const SceneDev* scenes, const uint2* tiles, uint32_t n_tiles, const float* albedo,
                             const float* power, const float* gE, uint32_t n_mat, uint32_t n_lights, float* partial,
                             float* g_albedo, float* g_power, hipStream_t s);

}  // namespace pv
