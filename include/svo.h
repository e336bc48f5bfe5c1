/*
 * svo.h -- C ABI of the animated sparse-voxel-octree ray tracer for MI355X
 * (gfx950).
 *
 * The library traces rays R(t) = o + t d, t in [tmin, tmax] (paper Eq. 1)
 * through one octree pool whose interior nodes may carry affine transforms.
 * A transformed node starts a new frame: its subtree is a rigid body placed
 * by a parent-relative forward map A_s (rotation, translation, anisotropic
 * scale, or any invertible affine map).  The octree is never rebuilt when
 * transforms change; each ray is mapped into a frame's local coordinates
 * instead (Sec. 3: inverse-transform the ray, Fig. 1; Eq. 2-3: the local ray
 * keeps the world parameter t).  The first hit reports the voxel id, t and
 * the surface normal, the per-pixel fields of the paper's hit buffer
 * (Sec. 4.3).
 *
 * Conventions for every entry point:
 *   - Return SVO_OK (0) or a negative svo_status; nothing throws or aborts
 *     across the ABI.  svo_last_error() gives a message for the calling
 *     thread's last failure.
 *   - "host" pointers are read during the call only and may be reused on
 *     return; "device" pointers must stay valid until the stream work that
 *     uses them has completed.  The caller owns both.  The library owns the
 *     device copies of pools and transform tables.
 *   - Work is stream ordered on the hipStream_t passed as `void* stream`
 *     (NULL = the null stream).  Calls on one context are not thread safe.
 *
 * ------------------------------------------------------------------------
 * Pool format (one uint64 per node, little endian):
 *   bits  0..7   child mask m; octant i = x | y << 1 | z << 2, where x, y, z
 *                select the upper half of the cell along that axis
 *   bits  8..31  c24: offset of the first child relative to this node
 *   bits 32..63  word1
 *   m == 0                  solid leaf; the whole cell is solid; word1 is
 *                           free (RGBA8 colour by convention); c24 unused
 *   m != 0, word1 bit 31    transformed node; slot s = word1 & 0x7fffffff;
 *                           children start at slot_child[s]; c24 unused
 *   m != 0, c24 == 0xffffff far pointer: children start at word1
 *   m != 0, otherwise       children start at node_index + c24 (c24 >= 1)
 * The k-th set bit of m (in octant order) is the child at start + k.  The
 * cell of a child is the parent cell halved on every axis; the world root
 * cell is [root_min, root_min + root_size)^3 and the root frame of slot s is
 * the cube slot_cell[s] = (min x, min y, min z, size) in that slot's local
 * coordinates.  A node reached through more than one parent (DAG sharing,
 * instancing) must not contain transformed nodes.  Leaves are boxes closed
 * on every side.
 *
 * Hit semantics (identical to the CPU oracle's definition):
 *   frame F0 = the world tree without its transformed subtrees; frame F_s =
 *   the subtree of slot s without nested transformed subtrees; the world map
 *   of F_s is W_s = W_parent(s) o A_s.  A leaf box B of frame F is hit at
 *   t = max(t_near, tmin) when the ray meets W_F(B) within [tmin, tmax];
 *   the result is the smallest such t over all frames (ties: smaller slot,
 *   then smaller node index).  id = node index of the leaf, inst = slot of
 *   its frame (SVO_NONE for F0), normal = outward normal of the entry face
 *   (the inverse transpose of W_F applied to the local face normal,
 *   normalised), zero when the ray starts inside the leaf.  A miss returns
 *   id = inst = SVO_NONE, t = +inf, normal = 0.  Rays with a non-finite
 *   component, a direction below 2^-100 in every component or tmin > tmax
 *   miss.  The direction is never
 *   renormalised: t is in units of the caller's d.
 *
 * The device computes in FP32.  Rays within a few ulps of an edge, a face
 * or a tie may resolve to a neighbouring voxel (a "grazing" ray).
 */
#ifndef SVO_H
#define SVO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SVO_ABI_VERSION 1

typedef enum {
    SVO_OK = 0,
    SVO_EINVAL = -1,   /* invalid argument, malformed pool or singular transform */
    SVO_ENOMEM = -2,   /* host or device allocation failed */
    SVO_EDEVICE = -3,  /* a HIP runtime call failed */
    SVO_ERANGE = -4,   /* a size is beyond a documented limit */
    SVO_EBUSY = -5,    /* resource still in use */
    SVO_ESTATE = -6    /* call not valid in the current state */
} svo_status;

#define SVO_NONE 0xFFFFFFFFu        /* miss id / inst; world frame; empty world root */
#define SVO_STEP_LIMIT 0xFFFFFFFEu  /* id of a ray that exceeded the per-ray step limit */
#define SVO_MAX_DEPTH 20u           /* levels below any frame root */
#define SVO_MAX_SLOTS 1023u         /* transform slots per scene (all frame records live in LDS) */
#define SVO_MAX_INLINE_NEST 4u      /* slots entered in place may nest this deep */

typedef struct svo_ctx svo_ctx;     /* opaque: device, pools, transform tables, work queues */
typedef uint32_t svo_scene;         /* scene handle, 0 is never valid */

/* What validation found out about a pool (host-only; svo_validate). */
typedef struct {
    uint64_t n_nodes;
    uint32_t n_frames;        /* 1 (world) + number of referenced slots */
    uint32_t world_height;    /* levels below the world root (0: root is a leaf or the world is empty) */
    uint32_t max_height;      /* largest frame height */
    uint32_t max_nesting;     /* deepest chain of nested slots (0: no slot) */
    uint32_t n_shared;        /* nodes referenced from more than one parent */
    uint32_t reserved;
} svo_pool_info;

/* How the current transforms classify a scene's frames (svo_get_scene_stats). */
typedef struct {
    uint64_t device_bytes;    /* pool + transform tables */
    uint32_t n_slots;
    uint32_t n_frames;        /* 1 (world) + referenced slots */
    uint32_t n_inline;        /* slots entered in place by the walk */
    uint32_t n_candidates;    /* slots traced from their own roots */
    uint32_t stack_levels;    /* traversal stack entries per lane */
    uint32_t nest_levels;     /* deepest chain of in-place frames */
} svo_scene_stats;

/* Kernel configuration; svo_tune() picks one, svo_set_config() sets one.
   Zero fields select the library defaults.  A launch whose tables do not
   fit the device's LDS per work-group under it halves lds_cache_nodes, then
   lowers waves_per_block (to a multiple of 4, then by one), before it
   reports SVO_ERANGE; results never depend on the configuration. */
typedef struct {
    uint32_t waves_per_block;   /* 1..16 wavefronts (64 lanes) per work-group */
    uint32_t blocks_per_cu;     /* work-groups per compute unit of the persistent grid (capped by what LDS and 32 waves per CU let reside) */
    uint32_t lds_cache_nodes;   /* first N pool nodes (the top levels, breadth-first) kept in LDS */
    uint32_t refill_lanes;      /* 0 or 64: a wave takes 64-ray tiles; 1..63: claim new rays once that many lanes are idle */
    uint32_t step_limit;        /* cell advances plus candidate selections per ray before SVO_STEP_LIMIT */
    uint32_t claim_tiles;       /* 64-ray tiles a wave takes from the work queue at once (0: 2; at most 64) */
    uint32_t sorted_candidates; /* 0: 16; 1..64: a job with at most this many candidate frames orders them by
                                   entry with a per-lane sorted table (the depth sort of Sec. 4.2), one with more
                                   through the box hierarchy over their world boxes (a scene whose table travels
                                   in the kernel arguments always takes the sorted table) */
    uint32_t tile_order;        /* 0: slow tiles first, 1: the plain claim order.  With 0, a one-job trace with
                                   whole-tile claims (refill_lanes 0 or 64; not the hit buffer) lists the 64-ray
                                   tiles whose slowest ray took the most walk steps (about the slowest 12 %) in
                                   its work queue's state, and the next trace of the same rays on the same
                                   stream hands those tiles to its waves first, so that the launch's longest
                                   chains start at its beginning instead of setting its end.  Order only:
                                   results are the same. */
} svo_config;

/* ABI version the library was built with (SVO_ABI_VERSION). */
int svo_abi_version(void);

/* Message for the calling thread's last failed call ("" if none).  The
   string stays valid until the thread's next library call. */
const char* svo_last_error(void);

/* Create a context on HIP device `device_ordinal` (makes it current while
   the library works).  *out is set to NULL on failure.  Infrastructure: no
   passage of the paper defines it. */
int svo_create(svo_ctx** out, int device_ordinal);

/* Free every scene, buffer and stream resource of the context after
   waiting for its device work.  NULL is a no-op.  Infrastructure: no
   passage of the paper defines it. */
void svo_destroy(svo_ctx* ctx);

/* Host-only pool check (no device needed).  nodes: host, n_nodes entries.
   root: index of the world root, or SVO_NONE for an empty world.
   max_depth: reject frames deeper than this (<= SVO_MAX_DEPTH).
   slot_child: host, n_slots child-group starts.  Checks every rule of the
   pool format above: child groups inside the pool, c24 != 0, slots in range
   and used by at most one node, no cycles, no transformed root, depth, and
   the DAG rule.  info may be NULL.  SVO_EINVAL on a malformed pool,
   SVO_ERANGE on a limit. */
int svo_validate(const uint64_t* nodes, uint64_t n_nodes, uint32_t root, uint32_t max_depth,
                 const uint32_t* slot_child, uint32_t n_slots, svo_pool_info* info);

/* Validate a pool and copy it to the device (synchronous).  root_min[3],
   root_size: world root cell.  slot_cell: host, n_slots * 4 floats (local
   root cell min xyz, edge length > 0).  Every slot starts with the identity
   transform.  *out receives the scene handle.  The parent frame of each slot
   (its nesting) is read from the pool itself: the slot whose subtree holds
   the transformed node, or the world, so it is not an argument.  The scene
   of independent SVOs with transforms is the paper's (Sec. 3), placed here
   on nodes; the upload itself is infrastructure. */
int svo_upload(svo_ctx* ctx, const uint64_t* nodes, uint64_t n_nodes, uint32_t root, const float root_min[3],
               float root_size, uint32_t max_depth, const uint32_t* slot_child, const float* slot_cell,
               uint32_t n_slots, svo_scene* out);

/* Release a scene's device memory after its queued work has finished.
   Infrastructure: no passage of the paper defines it. */
int svo_free_scene(svo_ctx* ctx, svo_scene scene);

/* Device bytes the scene holds (pool + transform tables), for admission.
   Infrastructure: no passage of the paper defines it (the paper sizes its
   SVOs and transforms in memory, Sec. 5.2). */
int svo_scene_bytes(svo_ctx* ctx, svo_scene scene, uint64_t* bytes);

/* Classification of the scene's frames under its latest transforms. */
int svo_get_scene_stats(svo_ctx* ctx, svo_scene scene, svo_scene_stats* out);

/* Set the parent-relative forward maps of slots [first_slot, first_slot +
   count).  fwd_3x4: host, count * 12 floats, row-major 3x4 [L | b] with
   x_parent = L x_local + b (paper Eq. 3 inverts this per frame; nested slots
   compose).  The library composes and inverts in FP64 on the host and packs
   one 64-byte FP32 record per frame, plus its exact (FP64) map, from which
   a hit's entry t and face are recomputed.  A scene of at most 10 slots carries
   that table to each trace in the kernel arguments: this call then does no
   device work, and every trace keeps the transforms current when it was
   enqueued, on any stream.  A larger scene's table is copied on `stream`;
   traces enqueued on `stream` afterwards see the new transforms, earlier
   ones the old (two device tables alternate; a copy into a table that
   traces on other streams may still read waits for them on the device, so
   `stream` may stall behind them but no trace reads a half-written table;
   svo_trace_batch jobs read the host staging when they are packed).  A slot whose moved cell stays
   inside its static cell (with a margin of 1e-5 cell) is entered in place
   when the walk reaches it (at most SVO_MAX_INLINE_NEST deep); every other
   slot is traced as a separate candidate in order of its root-cell entry.
   SVO_EINVAL on a non-finite or singular map or slots out of range. */
int svo_set_transforms(svo_ctx* ctx, svo_scene scene, uint32_t first_slot, uint32_t count, const float* fwd_3x4,
                       void* stream);

/* Trace n rays.  rays: device, n * 8 floats per ray (ox, oy, oz, tmin, dx,
   dy, dz, tmax), 16-byte aligned.  Outputs (device, n entries each): out_id
   (required), out_inst (nullable), out_t (required), out_normal (nullable,
   n * 3 floats).  n == 0 is a no-op.  The kernel never reads outside the
   pool, the rays or the outputs; ray contents are not validated (see the
   hit semantics above).  Traces on different streams of one context may
   overlap (each stream has its own work queue, up to 64 streams). */
int svo_trace_rays(svo_ctx* ctx, svo_scene scene, const float* rays, uint64_t n, uint32_t* out_id,
                   uint32_t* out_inst, float* out_t, float* out_normal, void* stream);

/* Trace as svo_trace_rays in a counting build of the kernel, for tests and
   measurement (the memory a traversal reads per node and per transform,
   Sec. 5.2); results are identical to svo_trace_rays.  counts: device, 3 *
   n uint32, zeroed by the caller: counts[i] = node records ray i read (each
   frame walked counts its root record once, then every pool node the walk
   loads), counts[n + i] = frames walked, counts[2n + i] += 1 per result
   write (exactly 1 when every ray is claimed and written once).  trail:
   nullable device uint32 array of trail_cap * n: trail[k * n + i] = pool
   index of ray i's k-th node load for k < trail_cap, bit 31 set when it came
   from the LDS copy of the pool prefix.  Errors: as svo_trace_rays;
   SVO_EINVAL without counts, SVO_ERANGE above 2^31 - 1 rays or a trail over
   2^40 entries. */
int svo_trace_rays_counted(svo_ctx* ctx, svo_scene scene, const float* rays, uint64_t n, uint32_t* out_id,
                           uint32_t* out_inst, float* out_t, float* out_normal, uint32_t* counts, uint32_t* trail,
                           uint32_t trail_cap, void* stream);

/* Trace with the hit buffer of the previous frame (Sec. 4.3, applied to
   transforms on nodes): on entry the outputs hold the results of an
   earlier svo_trace_rays / svo_trace_rays_reuse of the same rays against
   the same scene, under any transforms; on return they hold the results
   under the current transforms, identical to svo_trace_rays.  A ray whose
   previous result is a hit in the static world frame (inst == SVO_NONE) or
   a miss keeps it unchanged when no moved frame -- a transformed subtree
   entered in place or traced as a candidate -- can lie in front of it (the
   ray's entry into its moved root cell, after its bounding sphere and the
   candidate hierarchy's boxes, tested up to the previous hit with the
   current transforms); every other ray is traced
   again.  The static world never changes, so this is exact.  out_inst is
   required (it is read); out_normal may be NULL only if it was NULL before.
   retraced: nullable device uint64 to which the number of rays traced again
   is added (the caller zeroes it).  The caller guarantees the rays and
   outputs are those of the earlier trace; anything else gives undefined
   (but in-bounds) results.  Errors as for svo_trace_rays. */
int svo_trace_rays_reuse(svo_ctx* ctx, svo_scene scene, const float* rays, uint64_t n, uint32_t* out_id,
                         uint32_t* out_inst, float* out_t, float* out_normal, uint64_t* retraced, void* stream);

/* Pinhole camera: the primary rays of svo_generate_primary_rays, and of a
   camera trace (svo_trace_camera, svo_job.camera), which makes the same rays
   inside the trace kernel instead of reading them.  forward, right and up are
   unit vectors (right = forward x up); pixel (i, j), j counted from the top
   row, sample s has direction normalize(forward + sx right + sy up) with
   sx = ((i + fx) / width * 2 - 1) tan_half_fov * width / height and
   sy = (1 - (j + fy) / height * 2) tan_half_fov, where (fx, fy) = (1/2, 1/2)
   unless jitter is set, in which case they are hashed from (seed, pixel,
   sample) into [0, 1).  Every ray has origin eye, tmin 0 and tmax +inf.
   Ray order: tiled -- 8x8 pixel tiles, tile rows top to bottom, tiles left
   to right, pixels row-major inside a tile, partial edge tiles holding only
   in-image pixels; otherwise row-major pixels.  The samples of one pixel
   are consecutive.  One pixel sample per ray, the paper's per-pixel form
   (Fig. 5). */
typedef struct {
    float eye[3];
    float forward[3];
    float right[3];
    float up[3];
    float tan_half_fov;
    uint32_t width, height;
    uint32_t samples;         /* rays per pixel, >= 1 */
    uint32_t seed;
    uint32_t jitter;          /* 0: pixel centres */
    uint32_t tiled;           /* 1: 8x8 pixel tiles (see below), 0: rows */
    uint32_t reserved;
} svo_camera;

/* One job of a batched launch: rays traced against one scene under one set
   of transforms. */
typedef struct {
    svo_scene scene;
    const float* fwd_3x4;     /* host, n_slots * 12 floats (every slot of the scene, parent-relative,
                                 as in svo_set_transforms), or NULL for the scene's current transforms */
    const float* rays;        /* device, n * 8 floats, 16-byte aligned; NULL with a camera */
    uint64_t n;               /* rays; with a camera width * height * samples */
    uint32_t* out_id;         /* device outputs, as in svo_trace_rays */
    uint32_t* out_inst;       /* nullable */
    float* out_t;
    float* out_normal;        /* nullable */
    const svo_camera* camera; /* host, nullable: the job's rays are made in the trace kernel from this
                                 camera (read when the call packs the job), in the camera's ray order */
} svo_job;

/* Trace several jobs -- rays of many requests, scenes and animation frames
   -- in one persistent launch: the work queue spans every job's rays, each
   ray walks its own job's scene under its own transforms (one pixel/ray as in
   the paper's per-pixel algorithm, Fig. 5).  Results are identical to one
   svo_trace_rays per job.  At most 256 non-empty jobs and 2047 frame
   records (1 + n_slots per job) per call; jobs with n == 0 are skipped.  The
   job table is packed on the host into pinned memory and copied on `stream`
   (a ring of four tables; a fifth call waits for the first to finish); a
   single job of a scene of at most 10 slots instead takes its frame table in
   the kernel arguments, with no copy. */
int svo_trace_batch(svo_ctx* ctx, const svo_job* jobs, uint32_t n_jobs, void* stream);

/* Trace the primary rays of a camera (width * height * samples rays, in the
   camera's ray order) without a ray buffer: the trace kernel makes each ray
   from the camera where svo_trace_rays would read it (Eq. 1; Fig. 5, one
   pixel sample per ray); results are identical to svo_generate_primary_rays
   followed by svo_trace_rays.  cam: host, read during the call.  Outputs as
   in svo_trace_rays, width * height * samples entries.  Errors: as
   svo_trace_rays; SVO_EINVAL for a bad camera (zero size or samples, a
   field of view that is not finite and positive), SVO_ERANGE for a side
   above 2^20 pixels or more than 0xff000000 rays. */
int svo_trace_camera(svo_ctx* ctx, svo_scene scene, const svo_camera* cam, uint32_t* out_id, uint32_t* out_inst,
                     float* out_t, float* out_normal, void* stream);

/* svo_trace_batch without device allocation, for callers that cannot
   allocate: code under HIP graph capture, tight serving loops, harnesses
   that forbid hipMalloc.  Same jobs, limits and results as svo_trace_batch,
   but the work queue and the launch's tables live in one fixed scratch
   array per device inside the library (264 KiB: an 8.25 KiB work queue,
   then 256 KiB of tables), held until the process ends; the call allocates
   no device or pinned memory.  The tables are packed into pinned staging
   that svo_create set up and copied on `stream`; the call waits on the host
   until the previous call's copy has read that staging.  Each call first
   clears the queue with a small kernel on `stream`.  Every call on a device,
   from any context, shares that device's scratch, which keeps the last
   call's contents: calls that overlap on one device race (order them on one
   stream).  Errors: as svo_trace_batch, and SVO_ERANGE (nothing enqueued)
   when the batch's job, frame, candidate, sphere, exact-map and hierarchy
   records exceed 256 KiB (about 1,400 frame records). */
int svo_trace_batch_static(svo_ctx* ctx, const svo_job* jobs, uint32_t n_jobs, void* stream);

/* Composite traced hits into an RGBA8 image (the colour field of the
   paper's hit buffer, Sec. 4.3; images like its Fig. 6).  prim_id: device,
   width * height * samples ids of primary rays in ray order (8x8 tiles when
   tiled != 0, else row-major; `samples` consecutive rays per pixel, as
   svo_generate_primary_rays makes them).  ao_id: device, k ids per primary
   ray (consecutive, as svo_generate_ao_rays makes them), or NULL when k ==
   0.  In integers: a sample whose primary id is a node of `scene` has the
   RGB of that leaf's word1 and, with occ of its k AO rays blocked (id !=
   SVO_NONE), weight (F k + (1000 - F)(k - occ)) / (1000 k), F =
   ambient_permille (weight 1 when k == 0); any other id (a miss, a step
   limit) takes background_rgba with weight 1.  Each channel is the mean of
   colour * weight over the pixel's samples, rounded half up; alpha 255.
   out_rgba: device, width * height uint32, row-major (R in the low byte).
   Errors: SVO_EINVAL (unknown scene, NULL buffer, ambient_permille > 1000),
   SVO_ERANGE (samples 0 or > 1024, k > 64, a side above 2^20 pixels, more
   than 0xff000000 samples), SVO_EDEVICE. */
int svo_shade(svo_ctx* ctx, svo_scene scene, const uint32_t* prim_id, const uint32_t* ao_id, uint32_t width,
              uint32_t height, uint32_t samples, uint32_t tiled, uint32_t k, uint32_t ambient_permille,
              uint32_t background_rgba, uint32_t* out_rgba, void* stream);

/* ------------------------------------------------------------------------
 * Launch plans: a batched launch whose kernel arguments are fixed when the
 * plan is created, so that one svo_plan_launch can be captured into a HIP
 * graph (hipStreamBeginCapture, torch.cuda.graph) and replayed for every
 * later batch.  Rays of many requests and scenes then run in one persistent
 * launch per replay (one pixel/ray, Fig. 5), with no per-step launch setup;
 * the jobs of each replay come from the plan's pinned staging table as it is
 * when the replay's copy executes.  Results are identical to svo_trace_batch
 * with the same jobs.
 */
typedef struct svo_plan svo_plan;

/* Capacity of a plan. */
typedef struct {
    uint32_t max_jobs;        /* 1..256 non-empty jobs per launch */
    uint32_t max_frames;      /* 1..2047 frame records per launch; a job takes 1 + n_slots of its scene */
    uint32_t reserved[2];     /* zero */
} svo_plan_limits;

/* Create a plan for jobs on the given scenes (host array of n_scenes >= 1
   handles).  The scenes fix the plan's traversal-stack and frame-nesting
   capacity (bounds that hold under any transforms), the LDS candidate table
   and the pool whose prefix is cached in LDS (the first scene's).  The
   kernel configuration is the first scene's tuned one if it has one, else
   the context's.  Allocates a device table, pinned staging of the same
   size and a private work queue (zeroed; synchronous).  Errors: SVO_EINVAL
   (NULL argument, unknown scene, non-zero reserved field), SVO_ERANGE
   (limits out of range, or the plan's LDS footprint exceeds the device's
   even with no node cache and one wave per work-group), SVO_ENOMEM,
   SVO_EDEVICE.  *out is NULL on
   failure. */
int svo_plan_create(svo_ctx* ctx, const svo_scene* scenes, uint32_t n_scenes, const svo_plan_limits* limits,
                    svo_plan** out);

/* Pack jobs (host array, as for svo_trace_batch) into the plan's staging
   table, host only.  Every non-empty job's scene must be one of the plan's
   scenes; jobs without transforms use their scene's current ones, read now.
   Waits until the plan's last eager launch has copied the staging.  After a
   launch captured into a graph the library cannot see replays: the caller
   must not call this while a replay may still be copying (wait for an event
   recorded after the replay).  n_jobs == 0 (or only empty jobs) makes the
   next launch trace nothing.  Errors: SVO_EINVAL (bad job, foreign scene),
   SVO_ERANGE (more jobs, frame records or rays than the plan holds). */
int svo_plan_set_jobs(svo_ctx* ctx, svo_plan* plan, const svo_job* jobs, uint32_t n_jobs);

/* Enqueue the plan's launch on `stream`: a copy of the whole staging table
   to the device table, then the persistent trace kernel on the plan's own
   work queue (the kernel resets it on exit).  Allocates nothing and does not
   synchronise the host, so it may be captured; a captured copy reads the
   staging at every replay.  Launches of one plan must not overlap (one
   stream, or ordered streams).  Errors: SVO_EINVAL, SVO_EDEVICE. */
int svo_plan_launch(svo_ctx* ctx, svo_plan* plan, void* stream);

/* Wait for the plan's eager launches and free it.  Graphs holding a
   captured launch of the plan must not be replayed afterwards.  NULL is a
   no-op. */
int svo_plan_destroy(svo_ctx* ctx, svo_plan* plan);

/* Current kernel configuration of the context / replace it (validated).
   svo_set_config also drops every scene's tuned configuration. */
int svo_get_config(svo_ctx* ctx, svo_config* cfg);
int svo_set_config(svo_ctx* ctx, const svo_config* cfg);

/* Autotuner.  Times candidate kernel configurations on n device sample rays
   against `scene` under its current transforms, in two stages: the launch
   shape (waves per work-group, work-groups per CU, LDS pool-prefix size),
   then lane refill, tiles per work-queue claim and the candidate ordering
   (sorted table or hierarchy) for the fastest shape, then five times longer timings of that winner, the first
   stage's winner and the next two shapes.  Infrastructure: no passage of the paper defines it.  Keeps
   the fastest for that scene -- later svo_trace_rays calls on it use it, and
   a batch uses it when that scene holds most of the batch's rays -- and
   writes it to *best (nullable).  Results never depend on the
   configuration, only speed does.  Allocates and frees its own scratch
   outputs and synchronises `stream`; not for use inside a timed loop. */
int svo_tune(svo_ctx* ctx, svo_scene scene, const float* sample_rays, uint64_t n, void* stream, svo_config* best);


/* Write width * height * samples primary rays (8 floats each, tmin = 0,
   tmax = +inf) to out_rays (device, 16-byte aligned) on `stream`, in the
   camera's ray order (svo_camera).  SVO_ERANGE for a side above 2^20
   pixels or more than 0xff000000 rays. */
int svo_generate_primary_rays(svo_ctx* ctx, const svo_camera* cam, float* out_rays, void* stream);

/* Ambient-occlusion rays from primary hits: for each of the n primary rays
   (device, 8 floats each) with hit t (device, n floats) and normal (device,
   n * 3 floats) as svo_trace_rays returns them, write k rays to out_rays
   (device, n * k * 8 floats, 16-byte aligned): origin p + offset *
   max(1, |p|inf) * normal with p = o + t d, a cosine-weighted direction
   about the normal (seeded, counter-based: ray (i, j) depends only on seed,
   i and j), tmin = 0, tmax = radius.  A primary miss or a start inside a
   voxel (zero normal) yields k rays with tmin > tmax, which trace as misses. */
int svo_generate_ao_rays(svo_ctx* ctx, const float* rays, const float* t, const float* normal, uint64_t n, uint32_t k,
                         uint32_t seed, float radius, float offset, float* out_rays, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SVO_H */
