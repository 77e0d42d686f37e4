/*
 * pv.h -- C-ABI of the MI355X photon-path verification library.
 *
 * Implements the per-frame hot path of Moreau, Doggett and Sintorn, "Path
 * Verification for Dynamic Indirect Illumination": photon paths stored by the
 * previous frame are verified against the current frame's dynamic geometry
 * and moving area or point lights, and each invalidated path is re-traced from its
 * first invalid segment, optionally keeping path tails whose reflected energy
 * stays within the error threshold of Equation 2.
 *
 * Conventions for every call:
 *  - Pointers named d_* are DEVICE pointers (HIP global memory on the
 *    context's device); h_* are HOST pointers.  Scene data passed at upload is
 *    copied; the path store and outputs stay caller-owned and must remain
 *    valid until the context's stream has completed the call.
 *  - All work is enqueued on the context's stream (the one given to
 *    pv_create; pv_compact_photons_async also uses the caller's stream); no
 *    call synchronises the stream except pv_upload_scene, pv_set_light_paths
 *    and pv_reserve.
 *  - Return value: PV_OK (0) or a negative PV_ERR_* code.  Argument errors are
 *    detected on the host before anything is enqueued; pv_last_error() then
 *    describes the problem.  Faults of enqueued work surface as PV_ERR_HIP on
 *    a later call that synchronises.  No C++ exception crosses this boundary.
 *  - One context per stream/thread; calls on one context are not thread safe.
 *  - Verify, queue, re-trace and compaction calls allocate nothing: their
 *    scratch space is reserved by pv_reserve, so they may be captured in a
 *    HIP graph.
 *
 * Path store (Section 4 of the paper, with the photon position stored in place
 * of the incoming direction, which is the difference of consecutive
 * positions): paths are columns, bounce rows are contiguous, so all lanes that
 * load the i-th photon of their path touch consecutive memory.
 *   pos_hit [B][stride] float4 {x, y, z, hit}: photon x_{r+1} in row r;
 *           hit = global triangle id (bit pattern in .w), 0xFFFFFFFF = none
 *   energy  [B][stride] float4 {r, g, b, radius}: flux arriving at the photon
 *   origin  [3][stride] float: world-space light sample x_0 (x row, y row, z row)
 *   info    [stride] uint32 (Section 4 path-information word):
 *           bits 0..21 distribution-map cell (pv_set_distribution_map; kept
 *           unchanged without maps),
 *           22..25 segment count n (0..15),
 *           26..29 first segment to re-trace, 30 replace, 31 reuse light
 *   Paths [light_base[l], light_base[l+1]) belong to light l.
 *
 * Global triangle ids: static triangles first (0..S-1, upload order), then
 * each dynamic object's triangles in upload order.
 */
#ifndef PV_H
#define PV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pv_ctx pv_ctx;
typedef struct pv_batch pv_batch;
typedef int32_t pv_status;

enum {
  PV_OK = 0,
  PV_ERR_ARG = -1,      /* invalid argument (null pointer, size out of range) */
  PV_ERR_OOM = -2,      /* device allocation failed */
  PV_ERR_HIP = -3,      /* a HIP runtime call failed */
  PV_ERR_CAPACITY = -4, /* request exceeds what pv_reserve provided */
  PV_ERR_STATE = -5     /* call out of order (e.g. verify before upload) */
};

#define PV_MAX_BOUNCES 15   /* 4-bit segment count of the information word */
#define PV_MAX_OBJECTS 64   /* dynamic objects per scene */
#define PV_MAX_LIGHTS 8
#define PV_HIT_NONE 0xFFFFFFFFu

typedef struct {
  uint32_t n_paths;       /* columns in use */
  uint32_t max_bounces;   /* B, rows, 1..PV_MAX_BOUNCES */
  uint32_t stride;        /* floats4 between rows; >= n_paths, multiple of 64 */
  void* d_pos_hit;        /* float4 [B][stride] */
  void* d_energy;         /* float4 [B][stride] */
  float* d_origin;        /* float  [3][stride] */
  uint32_t* d_info;       /* uint32 [stride] */
} pv_path_store;

/* Scene description for pv_upload_scene; every pointer is a HOST pointer and
 * is copied.  Vertices are float[9] per triangle (v0, v1, v2).  Dynamic
 * objects are rigid and given in object space; their placement comes from
 * pv_frame_begin each frame. */
typedef struct {
  uint32_t n_static;             /* static triangles */
  const float* h_static_verts;   /* [n_static][9] world space */
  const uint32_t* h_static_mat;  /* [n_static] material ids */
  uint32_t n_objects;            /* dynamic objects, <= PV_MAX_OBJECTS */
  const uint32_t* h_obj_tris;    /* [n_objects] triangle counts */
  const float* h_obj_verts;      /* [sum obj_tris][9] object space, objects in order */
  const uint32_t* h_obj_mat;     /* [sum obj_tris] material ids */
  uint32_t n_materials;
  const float* h_albedo;         /* [n_materials][3] diffuse albedo rho */
  uint32_t n_lights;             /* lights, <= PV_MAX_LIGHTS */
  const float* h_light_half;     /* [n_lights][2] half extents along local u, v: both > 0 for a
                                    rectangular area light, both 0 for a point light (PV_ERR_ARG
                                    otherwise); both emit cosine-weighted about the local z axis */
  const float* h_light_power;    /* [n_lights][3] radiant power Phi */
  float eps_end;                 /* segment endpoint tolerance (scene units) */
  float eps_close;               /* AreClose tolerance of Algorithm 1 (scene units) */
  float photon_radius;           /* radius written into new photons */
  const int32_t* h_light_kind;   /* NULL (every light PV_LIGHT_AREA), or [n_lights]: the emission of
                                    a light of zero extent (Section 3.1's spotlight; the camera of
                                    Section 7's camera paths), PV_ERR_ARG for a nonzero kind with
                                    nonzero extents or out-of-range parameters */
  const float* h_light_param;    /* [n_lights][2] with h_light_kind: PV_LIGHT_SPOT {cos of the cone
                                    half-angle in [0, 1), unused}; PV_LIGHT_CAMERA {tan of the half
                                    field of view along local u, along local v}, both > 0 */
} pv_scene_desc;

/* Emission of a light (h_light_kind).  PV_LIGHT_AREA: a rectangle, or a point
 * light for zero extents, cosine-weighted about the local z axis.
 * PV_LIGHT_SPOT: a point emitting cosine-weighted inside the cone of
 * directions within the half-angle about local z.  PV_LIGHT_CAMERA: a point
 * emitting uniformly over its near plane at unit distance along local z,
 * |x| <= tan_u, |y| <= tan_v (a pinhole camera whose paths are camera paths;
 * its distribution map is the pixel grid of that plane).  A moved spot or
 * camera, like a moved point light, re-aims segment 0 from its new position
 * at the first photon and keeps the path only when the new direction lies in
 * its emission set; segment 0 is then tested against every triangle. */
enum { PV_LIGHT_AREA = 0, PV_LIGHT_SPOT = 1, PV_LIGHT_CAMERA = 2 };

/* Device counters accumulated by the calls that take a pv_stats* (may be
 * NULL).  Zero them (device memory) before the frame if per-frame values are
 * wanted. */
typedef struct {
  unsigned long long segments_examined;  /* segments tested by verify */
  unsigned long long paths_invalid;      /* paths given the replace bit */
  unsigned long long paths_light_lost;   /* of those: origin left the moved light */
  unsigned long long rays_traced;        /* closest-hit rays of the re-trace */
  unsigned long long photons_written;    /* photons written by the re-trace */
  unsigned long long reuse_accepted;     /* Equation 2 acceptances (error-based walk) */
  unsigned long long paths_truncated;    /* re-traced paths ending on an escaping ray */
  unsigned long long verify_box_hits;    /* segments traversed by verify: those reaching a moved object's box
                                            (none in the box mode), and point-light visibility segments */
} pv_stats;

/* --- context ----------------------------------------------------------- */

/* Create a context on the current HIP device; all work goes to 'hip_stream'
 * (a hipStream_t; NULL = the null stream). */
pv_status pv_create(pv_ctx** out, void* hip_stream);

/* Options fixed when a context is created (pv_create_config). */
typedef struct {
  uint32_t max_paths;     /* > 0: scratch reserved now, as by pv_reserve(max_paths, max_bounces);
                             0: call pv_reserve before the first store */
  uint32_t max_bounces;   /* rows of the stores (1..PV_MAX_BOUNCES) when max_paths > 0 */
  int32_t verify_mode;    /* PV_VERIFY_TRIANGLES or PV_VERIFY_BOXES (pv_set_verify_mode) */
  int32_t object_rebuild; /* 0 or 1 (PV_TUNE_OBJECT_REBUILD) */
} pv_config;

/* pv_create followed by the settings of *cfg (host pointer, read during the
 * call).  On any error no context is returned (*out = NULL) and
 * pv_last_error(NULL) describes it; PV_ERR_ARG for an option out of range,
 * PV_ERR_OOM when the reservation fails.  Synchronises when it reserves. */
pv_status pv_create_config(pv_ctx** out, const pv_config* cfg, void* hip_stream);
void pv_destroy(pv_ctx* ctx);
/* Last error message of the context (or of the last failed pv_create when ctx
 * is NULL).  Valid until the next call on the context. */
const char* pv_last_error(const pv_ctx* ctx);

/* Copy the scene to the device and build its bounding-volume hierarchies
 * (static world and one per rigid dynamic object, topology in object space).
 * Synchronises the stream.  Replaces any previous scene. */
pv_status pv_upload_scene(pv_ctx* ctx, const pv_scene_desc* desc);

/* Paths per light: light l owns the next h_counts[l] paths of the store,
 * lights in order, so E_1 = Phi_l / h_counts[l] (photon power of Section 3).
 * Synchronises.  The counts must add up to the n_paths of every store used
 * afterwards. */
pv_status pv_set_light_paths(pv_ctx* ctx, const uint32_t* h_counts);

/* Reserve scratch (work queue, per-block counters, verification task lists:
 * about 4 * max_paths * (max_bounces + 4) bytes) for stores of up to
 * max_paths paths (1 .. 2^28) and max_bounces rows.  Synchronises.  Must
 * precede verify/queue/retrace/compact calls. */
pv_status pv_reserve(pv_ctx* ctx, uint32_t max_paths, uint32_t max_bounces);

/* --- per frame --------------------------------------------------------- */

/* Section 3 (dynamic objects, dynamic lights): start a frame with new rigid
 * transforms.  d_obj_xf: [n_objects][12] device floats, row-major 3x4 [R|t]
 * (world = R p + t); d_light_xf: [n_lights][12] rigid light transforms (light
 * local z = emitting normal, the light is the rectangle |u|<=hu, |v|<=hv of
 * its local z=0 plane, or its local origin for a point light).  An object or light is "moved" when any of its 12
 * floats differs bitwise from the previous frame's; the first call marks
 * everything moved.  Then transforms the moved objects' triangles to world
 * space (each coordinate the FP64 evaluation of fma(r0,x,fma(r1,y,fma(r2,z,t)))
 * rounded to FP32) and refits their hierarchies. */
pv_status pv_frame_begin(pv_ctx* ctx, const float* d_obj_xf, const float* d_light_xf);
/* (With both arrays NULL, pv_frame_begin starts the frame with the context's
 * staged transforms below.) */

/* Section 3 (dynamic objects, dynamic lights) by id: stage new rigid
 * transforms for some objects (lights) of the next frame.  d_obj_ids /
 * d_light_ids: n DEVICE uint32 ids; d_m3x4: n DEVICE float[12] matrices in the
 * layout of pv_frame_begin.  Entries whose id is not below the scene's object
 * (light) count are skipped; of a repeated id the last entry is taken.  Ids
 * not named keep their staged transform: the last one given by this call or
 * by pv_frame_begin, identity before any.  n <= PV_MAX_OBJECTS
 * (PV_MAX_LIGHTS), else PV_ERR_ARG; PV_ERR_STATE before pv_upload_scene.
 * Stream-ordered, allocates nothing, may be captured.  The next
 * pv_verify_paths, pv_retrace_paths, pv_autotune or pv_object_hierarchy_info
 * first begins the frame with the staged transforms, as pv_frame_begin(ctx,
 * NULL, NULL) would; an object or light counts as moved when its staged
 * matrix differs bitwise from the previous frame's. */
pv_status pv_update_transforms(pv_ctx* ctx, uint32_t n, const uint32_t* d_obj_ids, const float* d_m3x4);
pv_status pv_update_lights(pv_ctx* ctx, uint32_t n, const uint32_t* d_light_ids, const float* d_m3x4);

/* Sections 3.1 and 3.2 (update path origins, dynamic occlusions): for each
 * path of a moved light, keep the outgoing direction and move x_0 onto the
 * light's new plane (invalid when outside the rectangle or behind the light:
 * replace=1, start=0, reuse_light=0); for a point light, x_0 becomes the
 * light's new position and segment 0 is re-aimed at the first photon (invalid
 * as above when that is not farther than eps_end on the emitting side), and
 * segment 0 is then tested against every triangle, static ones included (a
 * visibility ray in place of the paper's shadow map); then test the segments in order from the
 * light against every triangle of the moved objects (two-sided, hit strictly
 * inside (eps_end, L-eps_end)), a segment also being invalid when its end
 * photon lies on a moved object; the first invalid segment k gives replace=1,
 * start=k, reuse_light=1.  The store's info and origin are rewritten, and the
 * per-block counts of replaced paths are left for pv_build_queue. */
pv_status pv_verify_paths(pv_ctx* ctx, const pv_path_store* store, pv_stats* d_stats);

/* Section 4 (pruned-paths array, here the re-trace work list): compact the
 * ids of the paths whose replace bit was set by the last pv_verify_paths into
 * the context's work queue, in ascending order (stable ballot + prefix-sum
 * compaction), so that re-tracing packs active paths into few waves. */
pv_status pv_build_queue(pv_ctx* ctx, const pv_path_store* store);

/* Full invalidation (the paper's baseline, and frame 0): mark every path
 * replace=1, start=0, reuse_light=0 and queue them all. */
pv_status pv_queue_all(pv_ctx* ctx, const pv_path_store* store);

/* Copy the current work queue: d_out receives up to 'capacity' path ids,
 * *d_count (device) the queue length. */
pv_status pv_copy_queue(pv_ctx* ctx, uint32_t* d_out, uint32_t capacity, uint32_t* d_count);

/* Re-trace the queued paths (Section 3.2 / 3.3).  threshold < 0: naive --
 * re-trace from the first invalid segment along its stored direction, then
 * sample cosine-weighted diffuse bounces up to B photons (energy multiplied by
 * the albedo at each bounce, E_1 = Phi_l / N_l).  threshold >= 0: the
 * error-based walk of Algorithm 1 with Equation 2 evaluated per channel in
 * FP32 against the stored energies.  Random numbers: Philox4x64-10 keyed
 * (seed, 0), counter (path, frame, vertex, tag).  When pv_verify_paths ran
 * after the last pv_build_queue / pv_queue_all, the queue of its replaced
 * paths is built first (as pv_build_queue would). */
pv_status pv_retrace_paths(pv_ctx* ctx, const pv_path_store* store, float threshold, uint64_t seed,
                           uint32_t frame, pv_stats* d_stats);

/* Kernel tuning of a context.  PV_TUNE_RETRACE_VARIANT (0..3): occupancy
 * target of the re-trace kernel (4, 5, 6, 8 waves per SIMD; higher targets
 * trade registers for private-memory spills); PV_TUNE_RETRACE_BLOCKS_PER_CU
 * (1..64): persistent re-trace workgroups per compute unit;
 * PV_TUNE_WALK_MIN_ACTIVE (1..64): a wave's re-trace walk yields to take new
 * queries once fewer of its 64 lanes are still walking;
 * PV_TUNE_VERIFY_BLOCKS_PER_CU (1..32) and PV_TUNE_VERIFY_MIN_ACTIVE (1..64):
 * the same two choices for the verification traversal;
 * PV_TUNE_OBJECT_REBUILD (0 or 1): 0 (default) refits each moved object's
 * upload-time topology (binned surface-area heuristic, object space) in
 * pv_frame_begin; 1 also rebuilds every object's hierarchy on the device each
 * frame, as a linear BVH (30-bit Morton codes of the triangle centroids, radix
 * sort, radix tree by Karras 2012, boxes bottom-up), which becomes the
 * object's hierarchy unless it is deeper than 31 levels (then the refit
 * topology serves that frame).  Once mode 1 was set, the traversal stacks stay
 * sized for 31-level object hierarchies.  Results do not depend on the
 * tuning. */
enum {
  PV_TUNE_RETRACE_VARIANT = 0,
  PV_TUNE_RETRACE_BLOCKS_PER_CU = 1,
  PV_TUNE_WALK_MIN_ACTIVE = 2,
  PV_TUNE_VERIFY_BLOCKS_PER_CU = 3,
  PV_TUNE_VERIFY_MIN_ACTIVE = 4,
  PV_TUNE_OBJECT_REBUILD = 5
};
pv_status pv_set_tuning(pv_ctx* ctx, int32_t key, int32_t value);
pv_status pv_get_tuning(const pv_ctx* ctx, int32_t key, int32_t* value);

/* Test of the dynamic-occlusion step (Section 3.2) used by pv_verify_paths.
 * PV_VERIFY_TRIANGLES (default): a segment is invalid when a triangle of a
 * moved object crosses it within (eps_end, L - eps_end).  PV_VERIFY_BOXES: the
 * paper's conservative test, a segment is invalid once that part of it
 * reaches the bounding box of a moved object (the box is the object's stored
 * world box, padded by 1e-6 + 1e-6 |x| per coordinate); it invalidates every
 * path the triangle test does, at the same or an earlier segment, and traces
 * nothing.  Both tests take the first moved end photon and the origin update
 * of Section 3.1 alike; Algorithm 1's own checks in pv_retrace_paths stay
 * triangle-exact.  Takes effect for the context's next verification (a batch
 * takes each context's mode when it is created).  PV_ERR_ARG for any other
 * value. */
enum { PV_VERIFY_TRIANGLES = 0, PV_VERIFY_BOXES = 1 };
pv_status pv_set_verify_mode(pv_ctx* ctx, int32_t mode);

/* Equation 2's E_N in the error-based walk (Algorithm 1's
 * BRDF(Segment, NextSeg)).  PV_ENERGY_ALBEDO (default): the energy arriving
 * at the new vertex times its albedo when the kept outgoing direction leaves
 * on the arrival side, else 0.  PV_ENERGY_COSINE_RATIO: that value times the
 * ratio of the kept direction's cosine at the new vertex to its cosine at the
 * old vertex (whose stored triangle gives the normal): a diffuse bounce drawn
 * cosine-weighted at the old vertex, reached from the new one.  Takes effect
 * for the context's next re-trace.  PV_ERR_ARG for any other value. */
enum { PV_ENERGY_ALBEDO = 0, PV_ENERGY_COSINE_RATIO = 1 };
pv_status pv_set_energy_test(pv_ctx* ctx, int32_t mode);

/* --- distribution maps (Section 3.1) -------------------------------------- */

/* Section 3.1's distribution maps: each light's emission is partitioned into
 * cells and the number of paths per cell kept at its target DM_T.
 * h_grid (host) = {gu, gv, rings, sectors}, each 1..4096: a rectangle's cells
 * are a gu x gv grid over its local (u, v) times the direction cells, a point
 * light's the direction cells only; directions are cut on the unit disk of
 * their local (x, y) components into 'rings' rings of equal area and
 * 'sectors' sectors of equal angle (cosine-weighted emission is uniform
 * there, so every cell is equally likely); cell index
 * ((iu * gv + iv) * rings + ring) * sectors + sector, stored in bits 0..21 of
 * the information word.  DM_T of cell c of a light with N paths and C cells:
 * N / C, plus one for c < N mod C.  NULL disables the maps.  Requires an
 * uploaded scene and pv_reserve (a later pv_reserve or pv_upload_scene
 * disables them again).  Allocates and synchronises.  PV_ERR_ARG for sizes out
 * of range or more than 2^22 cells per light (2^24 in all). */
pv_status pv_set_distribution_map(pv_ctx* ctx, const int32_t* h_grid);
/* Cells of all lights of the context's maps (0 when none). */
uint32_t pv_distribution_cells(const pv_ctx* ctx);
/* Section 3.1's three steps after the origin update (call after
 * pv_verify_paths, or after pv_queue_all at the first frame, and before
 * pv_build_queue / pv_retrace_paths):
 *  Compute DM_C: every path whose light sample survived counts in its cell;
 *    a moved light's path takes the cell of its updated origin and kept
 *    direction, and one that has no cell is re-sampled;
 *  Prune paths: a path of a cell holding C > DM_T paths is re-sampled with
 *    probability (C - DM_T) / C (Equation 1), decided in FP32 against one
 *    Philox uniform (key seed, counter (path, frame, 0, 2)), all with the
 *    counts before pruning (two passes, Section 4);
 *  Fill DM_C: the i-th re-sampled path of a light (path order: lost, pruned,
 *    or all of them at the first frame) takes the cell where the running sum
 *    of the deficits max(0, DM_T - (DM_C - pruned)) passes i.
 * Re-sampled paths get replace = 1, reuse-light = 0 and their cell; the next
 * pv_retrace_paths draws their light samples inside the cell.  d_dm_c /
 * d_pruned (device, nullable, [pv_distribution_cells]) receive the counts of
 * the first step and the pruned paths per cell.  Single-scene calls only (the
 * batched form has no maps).  PV_ERR_STATE without maps. */
pv_status pv_update_distribution(pv_ctx* ctx, const pv_path_store* store, uint64_t seed, uint32_t frame,
                                 uint32_t* d_dm_c, uint32_t* d_pruned);

/* Autotuner: with the current frame (after pv_frame_begin) and the given
 * store, on a snapshot of the store: time verification (median of three runs
 * each) for every traversal grid (4, 8, 16, 32 workgroups per CU) and yield
 * threshold (8, 16, 32, 48);
 * then, after verification and queue building, time the re-trace for every
 * re-trace variant and persistent grid size (4, 8, 16, 32 workgroups per CU),
 * then for yield thresholds 8..48.  Keeps the fastest settings in the
 * context and restores the store.  Allocates a temporary copy of the store
 * and synchronises.  *out_ms (host, optional) receives the best re-trace
 * time. */
pv_status pv_autotune(pv_ctx* ctx, const pv_path_store* store, float threshold, uint64_t seed, uint32_t frame,
                      float* out_ms);
/* Timings of the context's last pv_autotune (every trial is timed three
 * times; its median decides): h_out[7] (host) receives the chosen
 * verification setting's median ms, its spread (max - min) / median, the
 * largest spread of any verification trial, the chosen re-trace setting's
 * median ms, its spread, the largest spread of any re-trace trial, and the
 * number of trials.  Zeros before the first autotuning. */
pv_status pv_autotune_report(const pv_ctx* ctx, float* h_out);

/* Section 4 (the photon map a splatting renderer consumes): existing photons
 * in (row, path) order; d_out_pos / d_out_energy receive float[3] per photon
 * (at most 'capacity' written), *d_count the true count.  The call never
 * synchronises, so it cannot know the count when it returns: an output too
 * small for the photons is reported only through *d_count > capacity (the
 * first 'capacity' photons are written), never as PV_ERR_CAPACITY. */
pv_status pv_compact_photons(pv_ctx* ctx, const pv_path_store* store, float* d_out_pos,
                             float* d_out_energy, uint32_t capacity, uint32_t* d_count);

/* For callers that cannot allocate device memory at all (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * compaction, same outputs and argument errors as pv_compact_photons, with
 * its scratch (photon counts per bounce row and 256-path block, their
 * offsets, the scan's tile sums) in a fixed 1 MiB array of the library
 * instead of the context's reserved scratch.  The call allocates nothing.
 * Limit: path blocks x bounce rows, ceil(n_paths / 256) * max_bounces, at most
 * PV_NOALLOC_MAX_COUNTS (e.g. 4.79 M paths of 7 rows); a larger store returns
 * PV_ERR_CAPACITY before anything is enqueued.  The array is one per device,
 * shared by every context and call on that device and held until the process
 * ends; each call overwrites what it reads, so nothing needs clearing, but
 * calls that overlap on one device (other streams, other threads) race on it
 * and must be ordered by the caller. */
#define PV_NOALLOC_MAX_COUNTS 131008u
pv_status pv_compact_photons_noalloc(pv_ctx* ctx, const pv_path_store* store, float* d_out_pos,
                                     float* d_out_energy, uint32_t capacity, uint32_t* d_count);

/* The same compaction, overlapped with the next frame: enqueued on the
 * caller's 'hip_stream' behind everything already on the context's stream (an
 * event), with scan scratch of its own, so that it runs beside the next
 * frame's pv_frame_begin, pv_verify_paths and pv_build_queue (they write no
 * photon row, no segment count and no scratch it uses).  The context's next
 * pv_retrace_paths, pv_queue_all, compaction, autotuning, verify-mode change,
 * store rebinding, pv_reserve or pv_upload_scene waits for it on the context's
 * stream (an event); consumers of d_out_pos / d_out_energy / d_count order
 * themselves after 'hip_stream'.  Same outputs and errors as
 * pv_compact_photons. */
pv_status pv_compact_photons_async(pv_ctx* ctx, const pv_path_store* store, float* d_out_pos,
                                   float* d_out_energy, uint32_t capacity, uint32_t* d_count, void* hip_stream);

/* --- differentiation form ------------------------------------------------ */

/* Deposited energy of every photon recomputed from the path's materials:
 * E[r][p][c] = Phi_{l,c}/N_l * prod_{i=1..r} albedo[m(x_i)][c] for r < n_p, else 0.
 * d_albedo [n_materials][3], d_power [n_lights][3], d_E [B][n_paths][3]. */
pv_status pv_energy_forward(pv_ctx* ctx, const pv_path_store* store, const float* d_albedo,
                            const float* d_power, float* d_E);
/* Gradients of L = sum gE * E with the validity masks held fixed.
 * d_gE [B][n_paths][3]; outputs d_g_albedo [n_materials][3], d_g_power [n_lights][3]
 * (overwritten). */
pv_status pv_energy_backward(pv_ctx* ctx, const pv_path_store* store, const float* d_albedo,
                             const float* d_power, const float* d_gE, float* d_g_albedo,
                             float* d_g_power);

/* --- batched form -------------------------------------------------------- */

/* Group n uploaded contexts, each with its path store (the store binding of
 * the batch is fixed), so that one call runs a whole frame of every scene with
 * one launch per phase: transform + refit, verification, work queue (one
 * queue over all scenes), re-trace (one persistent launch) and photon
 * compaction into a batch-owned buffer.  d_obj_xf[i] / d_light_xf[i] are the
 * device transform arrays of scene i (layout of pv_frame_begin) whose
 * addresses stay fixed; the caller rewrites their contents before each frame.
 * threshold and seed as in pv_retrace_paths.  Frames are ordered on the
 * stream of contexts[0] (they run on a stream of the batch's own, which may
 * be captured, fenced with events); every context must have been uploaded with pv_set_light_paths
 * matching its store.  A context that has a distribution map when the batch
 * is created (pv_set_distribution_map) keeps it in the batch: every frame
 * runs pv_update_distribution's steps for that scene after verification,
 * with the batch's seed and the frame's number, on batch-owned scratch (a map
 * set or cleared on the context later does not reach the batch).  Results are
 * bit-identical to the per-context calls (pv_verify_paths, pv_update_distribution
 * for a scene with a map, pv_retrace_paths).
 * Synchronises.  Errors are reported through pv_last_error(contexts[0]). */
pv_status pv_batch_create(pv_batch** out, pv_ctx* const* contexts, const pv_path_store* stores, uint32_t n,
                          const float* const* d_obj_xf, const float* const* d_light_xf, float threshold,
                          uint64_t seed);
void pv_batch_destroy(pv_batch* b);
/* One frame of every scene.  The first call (and any call with a different
 * d_stats) captures the frame into a HIP graph; later calls replay it, with
 * the frame number read from device memory.  Never synchronises. */
pv_status pv_batch_frame(pv_batch* b, uint32_t frame, pv_stats* d_stats);
/* Frames first_frame .. first_frame + k - 1 of every scene, in order, with one
 * graph launch (the batched form over frames as well as scenes: each frame is
 * the sequence pv_batch_frame runs, Sections 3.2 and 3.3 in turn, and a frame
 * verifies the paths the one before it wrote).  d_obj_xf / d_light_xf are
 * host arrays of k * n device pointers, frame-major (frame f of scene i at
 * [f * n + i]), each a transform array of pv_frame_begin's layout; a scene
 * without objects may pass NULL for its object arrays.  The tables and frame
 * numbers are copied (stream-ordered) before the launch, so the caller may
 * reuse the host arrays at once; the device arrays they point to must hold
 * their transforms until the launch has run.  The graph is captured on the
 * first call and again when k or d_stats changes (a larger k than any before
 * also synchronises the owner's and the batch's streams once, to grow the
 * tables); later calls replay it.  Photon compaction runs in every frame, so the buffer that
 * pv_batch_copy_photons reads holds the last frame's photons.  Results are
 * bit-identical to k calls of pv_batch_frame.  1 <= k <= PV_BATCH_MAX_FRAMES,
 * else PV_ERR_ARG; a NULL table or a NULL light array (or object array of a
 * scene with objects) is PV_ERR_ARG.  Never synchronises otherwise. */
#define PV_BATCH_MAX_FRAMES 1024u
pv_status pv_batch_frames(pv_batch* b, uint32_t first_frame, uint32_t k, const float* const* d_obj_xf,
                          const float* const* d_light_xf, pv_stats* d_stats);
/* Point the batch at other per-scene transform arrays for the next frames
 * (host arrays of n device pointers, copied; stream-ordered, no
 * synchronisation, no graph re-capture: the frame reads the pointer tables
 * from device memory). */
pv_status pv_batch_set_transforms(pv_batch* b, const float* const* d_obj_xf, const float* const* d_light_xf);
/* Copy the last frame's photon compaction of the batch: positions and
 * energies (float[3] each) of every existing photon, scene by scene, each in
 * (row, path) order (at most 'capacity' photons), and d_scene_base[0..n]: the
 * first photon of each scene and, last, the total.  Device buffers. */
pv_status pv_batch_copy_photons(pv_batch* b, float* d_pos, float* d_energy, uint32_t capacity,
                                uint32_t* d_scene_base);

/* --- host utilities ------------------------------------------------------ */

/* Bytes of the store layout for n paths and B rows (Table 1 of the paper
 * counts 32 B per photon, 4 B path information and 12 B origin per path). */
uint64_t pv_store_bytes(uint64_t n_paths, uint32_t max_bounces);
/* Build, on the host, the hierarchy the library builds for n triangles
 * (h_verts [n][9]; kind 0 = static world, binned surface-area heuristic;
 * kind 1 = dynamic object, Morton-order radix split) and check it:
 * out[0] internal nodes, out[1] leaves, out[2] depth of the deepest leaf,
 * out[3] = 1 when the leaves partition the triangles, every child box
 * contains its subtree and the depth fits the traversal stack. */
pv_status pv_hierarchy_info(const float* h_verts, uint32_t n, int32_t kind, uint32_t* out);
/* Check the current hierarchy of dynamic object 'obj' on the device (after
 * pv_frame_begin; synchronises the context's stream and copies the scene's
 * nodes and the object's triangles to the host): out[0] internal nodes,
 * out[1] leaves, out[2] depth of the deepest leaf, out[3] = 1 when the leaves
 * partition the object's triangles, every box on the way to a leaf contains
 * its triangles and the depth fits the traversal stack, out[4] = 1 when the
 * hierarchy is the per-frame rebuilt one (PV_TUNE_OBJECT_REBUILD), 0 for the
 * refit upload-time topology.  PV_ERR_ARG for an object index out of range,
 * PV_ERR_STATE before a scene upload. */
pv_status pv_object_hierarchy_info(pv_ctx* ctx, uint32_t obj, uint32_t* out);
/* Pack / unpack the path-information word. */
uint32_t pv_info_pack(uint32_t cell, uint32_t nseg, uint32_t start, uint32_t replace, uint32_t reuse);
void pv_info_unpack(uint32_t w, uint32_t* cell, uint32_t* nseg, uint32_t* start, uint32_t* replace,
                    uint32_t* reuse);
/* Library version string. */
const char* pv_version(void);

#ifdef __cplusplus
}
#endif
#endif
