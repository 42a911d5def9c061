/*
 * mrs.h -- C ABI of libmrs, a multi-resolution Monte Carlo renderer for
 * AMD Instinct MI355X (gfx950).
 *
 * The library renders the two inputs of the hybrid method of "Fast Monte Carlo
 * Rendering via Multi-Resolution Sampling" (Sec. 4): a high-resolution,
 * low-spp image (HRLS) and a low-resolution, high-spp image (LRHS), each with
 * albedo / normal / depth feature buffers (Sec. 4, first paragraph: HRLS carries
 * RGB plus extra layers; LRHS carries RGB).  The images are produced by a
 * Monte Carlo path tracer (Sec. 3.2 renders with one; Sec. 1 motivates the
 * ray-count cost) that this library implements on the GPU.
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers (HBM).  Everything else is host
 *    memory.  Device outputs are owned by the caller (e.g. torch tensors);
 *    the library never frees them.  *_create functions copy their host inputs,
 *    which the caller may free on return.
 *  - All GPU work is enqueued asynchronously on the stream set with
 *    mrs_set_stream (default: the null stream).  Results are visible after
 *    mrs_sync() or any later synchronisation of that stream.
 *  - Functions return mrs_status and never throw or abort.  On failure,
 *    mrs_last_error() returns a thread-local message.  Arguments are validated
 *    before any work is enqueued: a call that fails validation writes nothing.
 *    Asynchronous device faults are reported by the next call or by mrs_sync.
 *  - Images are row-major, row 0 at the top, channels interleaved (HWC), FP32.
 *  - Destroy functions accept NULL.
 */
#ifndef MRS_H_
#define MRS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mrs_status {
  MRS_OK = 0,
  MRS_ERR_INVALID_ARGUMENT = 1,
  MRS_ERR_OUT_OF_MEMORY = 2,
  MRS_ERR_DEVICE = 3,
  MRS_ERR_NOT_READY = 4,
  MRS_ERR_UNSUPPORTED = 5
} mrs_status;

/* ------------------------------------------------------------------ scenes */

typedef enum mrs_material_kind {
  MRS_LAMBERT = 0, /* f = color / pi */
  MRS_GGX = 1,     /* GGX microfacet reflection (Walter et al. 2007), F0 = color,
                      roughness alpha, separable Smith G, Schlick Fresnel */
  MRS_EMITTER = 2  /* pure emitter: no BSDF; a path ends on it */
} mrs_material_kind;

/* 32 bytes.  Any kind may also emit `emission` from its front face. */
typedef struct mrs_material {
  int32_t kind;
  float color[3];
  float alpha;
  float emission[3];
} mrs_material;

/* 56 bytes.  Parallelogram light y = corner + u*edge_u + v*edge_v, u,v in
 * [0,1); it emits from the side edge_u x edge_v points to.  tri[] names the
 * two scene triangles that carry its geometry; those triangles are excluded
 * from its shadow rays and do not add emission when reached by a BSDF ray
 * (next-event estimation accounts for them). */
typedef struct mrs_quad_light {
  float corner[3];
  float edge_u[3];
  float edge_v[3];
  float emission[3];
  int32_t tri[2];
} mrs_quad_light;

/* Pinhole camera.  Forward f = normalize(look_at - pos), right r =
 * normalize(f x up), vertical v = r x f, vfov_deg the full vertical angle. */
typedef struct mrs_camera {
  float pos[3];
  float look_at[3];
  float up[3];
  float vfov_deg;
} mrs_camera;

#define MRS_TRI_SMOOTH 1u /* shade with the interpolated per-corner normals */

typedef struct mrs_scene_desc {
  int32_t num_tris;             /* 0 .. 2^24 - 2; 0 gives an environment-only scene */
  const float* vertices;        /* host, num_tris*9: v0, v1, v2 (xyz each) */
  const float* normals;         /* host, num_tris*9 per-corner normals, or NULL */
  const uint32_t* tri_material; /* host, num_tris indices into materials */
  const uint32_t* tri_flags;    /* host, num_tris MRS_TRI_* bits, or NULL */
  int32_t num_materials;
  const mrs_material* materials;
  int32_t num_lights; /* 0..255 */
  const mrs_quad_light* lights;
  float env[3]; /* constant environment radiance seen by rays that miss */
  mrs_camera camera;
} mrs_scene_desc;

typedef struct mrs_scene mrs_scene; /* opaque: device copy of the scene + LBVH */

/* Thread-local message of the last failed call ("" if none). */
const char* mrs_last_error(void);

/* Stream for all later work of this thread (a hipStream_t; NULL = null stream). */
mrs_status mrs_set_stream(void* hip_stream);

/* Wait for all work on the current stream; reports asynchronous faults. */
mrs_status mrs_sync(void);

/* Copies the scene to the device.  Fails with INVALID_ARGUMENT on NULL arrays
 * (when num_tris > 0), material or light indices out of range, or non-finite
 * vertices; OUT_OF_MEMORY if device allocation fails. */
mrs_status mrs_scene_create(const mrs_scene_desc* desc, mrs_scene** out);
mrs_status mrs_scene_destroy(mrs_scene* scene);

/* Builds the scene's BVH on the device, with the builder that
 * mrs_tuning.bvh_builder selects:
 *   MRS_BVH_LBVH  the linear BVH of Karras (HPG 2012): 30-bit Morton codes of
 *                 triangle centroids in the centroid bounds, keys
 *                 (morton << 32 | prim) sorted by a device radix sort, one
 *                 internal node per adjacent key pair from common-prefix
 *                 lengths, leaf-to-root box refit with atomic visit counters;
 *   MRS_BVH_PLOC  (default) agglomerative clustering over the same Morton
 *                 order (Meister & Bittner, TVCG 2018): nearest neighbours by
 *                 union surface area within 12 places, mutual pairs merge,
 *                 until one cluster is left; laid out depth first.  A tree
 *                 deeper than 64 levels, or one that needs more than 256
 *                 clustering rounds (chains), falls back to MRS_BVH_LBVH.
 * Then either is collapsed into the four-wide BVH that rendering traverses.
 * Every builder gives the same closest hits and images, bitwise (traversal
 * culls conservatively and breaks ties by primitive id); they differ in speed.
 * Idempotent.  Enqueued on the current stream. */
#define MRS_BVH_LBVH 0
#define MRS_BVH_PLOC 1
mrs_status mrs_build_bvh(mrs_scene* scene);
/* The builder that made the scene's BVH (MRS_BVH_*); MRS_ERR_NOT_READY before
 * mrs_build_bvh. */
mrs_status mrs_scene_bvh_builder(const mrs_scene* scene, int32_t* builder);

/* Renders W x H pixels at spp samples each, paths of at most max_depth bounces
 * (vertex 0 is the camera hit; next-event estimation at vertices
 * 0..max_depth-1), Russian roulette from vertex 3, Philox4x32-10 random
 * numbers keyed by seed and counted by (pixel, sample, dimension).
 *   out_rgb_dev  H*W*3 FP32: per-pixel mean radiance over the samples, summed
 *                in sample order (FP64 sums when spp >= 1024, FP32 below).
 *   out_aux_dev  H*W*7 FP32 or NULL: mean first-hit albedo (3), shading normal
 *                facing the camera (3) and hit distance (1); zeros on a miss.
 * Limits: 1 <= W, H <= 16384, 1 <= spp <= 2^20, 0 <= max_depth <= 64, outputs
 * 4-byte aligned.  NOT_READY if the BVH has not been built. */
mrs_status mrs_render(const mrs_scene* scene, int32_t W, int32_t H, int32_t spp,
                      int32_t max_depth, uint64_t seed, float* out_rgb_dev, float* out_aux_dev);

typedef struct mrs_render_opts {
  int32_t rr_start;   /* first vertex with Russian roulette (default 3) */
  int32_t x0, y0;     /* window origin in the W x H image (default 0, 0) */
  int32_t win_w;      /* window size; 0 = the whole image */
  int32_t win_h;
  int32_t accum_fp64; /* -1 auto (spp >= 1024), 0 FP32 sums, 1 FP64 sums */
  int32_t mis;        /* 0 (default): quad lights by next-event estimation only (E8);
                         1: next-event estimation and BSDF sampling of the quad lights
                         combined by multiple importance sampling, power heuristic
                         (Veach & Guibas 1995): a BSDF ray that reaches a listed light
                         at vertex b >= 1 adds its emission weighted against the
                         light-sampling density.  Finding that light scans the scene's
                         light list. */
  float lens_radius;  /* thin lens (depth of field): radius of the lens disk; 0 = pinhole */
  float focus_dist;   /* distance of the focal plane along the view axis (> 0 with a lens) */
  float cam_motion[3]; /* camera translation over the shutter (motion blur); 0 = still.
                         A sample's ray leaves from pos + tau * cam_motion + a point of
                         the lens disk (uniforms d2, d3: radius R sqrt(u2), angle
                         2 pi u3) towards the point where the pinhole ray of its pixel
                         point meets the focal plane; tau = word 0 of Philox with
                         counter (p, s, 0, 4), drawn only for a moving camera. */
  float* out_sumsq_dev; /* optional win_h*win_w*3: sum over samples of L^2 */
  float* out_layers_dev; /* optional win_h*win_w*9: the render layers of Sec. 3.1
                         (Eqs. 1-2; no subsurface or transmission lobes here), per
                         pixel the sample means of (0..2) the radiance emitted towards
                         the camera at the first vertex (emitters, or the environment
                         when the camera ray misses), (3..5) the rest of the radiance
                         of samples whose first vertex is Lambert (diffuse) and (6..8)
                         GGX (glossy).  The three add up to the rgb output up to
                         rounding; a non-finite sample counts as zero in all of them.
                         Uses the accumulation precision of the render. */
} mrs_render_opts;

/* Fills `opts` with the defaults listed above. */
void mrs_render_opts_default(mrs_render_opts* opts);

/* mrs_render with options.  A window renders pixels (x0..x0+win_w-1,
 * y0..y0+win_h-1) of the W x H image into win_h*win_w outputs; random numbers
 * use full-image pixel indices, so a window is bitwise a crop of the full
 * image. */
mrs_status mrs_render_ex(const mrs_scene* scene, int32_t W, int32_t H, int32_t spp,
                         int32_t max_depth, uint64_t seed, const mrs_render_opts* opts,
                         float* out_rgb_dev, float* out_aux_dev);

/* mrs_render_ex for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, validation and results -- bitwise those of mrs_render_ex --
 * but the call performs no device allocation.  Its workspace is a fixed array
 * in the library's device code (each GPU that loads the library holds its own
 * copy, about 170 MB, until the process ends): at most 2^18 resident paths
 * (any spp: the render loops over super-chunks), 512 traversal blocks, the
 * caller's stream only (no internal sub-chunk streams), and 2^19 * 13 * 8
 * bytes (54.5 MB) of pixel sums: 13 values per window pixel (22 with render
 * layers) at 8 bytes with FP64 sums (spp >= 1024) or 4 with FP32 sums, i.e.
 * windows of up to 2^19 pixels with FP64 sums, 2^20 with FP32 sums; a larger
 * window returns INVALID_ARGUMENT before anything is enqueued (render such
 * images in windows: a window is bitwise a crop of the full image).  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other threads) race and must
 * be ordered by the caller.  Its counters are not added to mrs_get_counters
 * and its kernels are not timed by mrs_profile_*. */
mrs_status mrs_render_ex_noalloc(const mrs_scene* scene, int32_t W, int32_t H, int32_t spp,
                                 int32_t max_depth, uint64_t seed, const mrs_render_opts* opts,
                                 float* out_rgb_dev, float* out_aux_dev);

/* ------------------------------------------------------------ batches */

/* One render of a batch: the arguments of mrs_render_ex. */
typedef struct mrs_job {
  const mrs_scene* scene;
  int32_t W, H, spp, max_depth;
  uint64_t seed;
  mrs_render_opts opts;
  float* out_rgb_dev;
  float* out_aux_dev; /* or NULL */
} mrs_job;

typedef struct mrs_batch mrs_batch; /* opaque: job table, accumulators, workspace */

/* Validates 1..255 jobs (each as mrs_render_ex would), uploads the job table
 * and reserves every buffer the batch needs (synchronous).  Jobs may differ in
 * scene, resolution, window, spp and depth.  The paths of all jobs form one
 * index space, so each stage of the wavefront (generate, extend, shade, shadow,
 * accumulate, resolve) is one launch over every job's live work: small jobs
 * share the GPU instead of running one after another.  Each job's outputs are
 * bitwise those of the same mrs_render_ex call.  The scenes must outlive the
 * batch. */
mrs_status mrs_batch_create(const mrs_job* jobs, int32_t n, mrs_batch** out);
/* Enqueues the batch on the current stream.  The batch owns its path
 * workspace, sized with the tuning in force at mrs_batch_create (later
 * mrs_set_tuning calls do not affect it), so this performs no allocation and
 * no host synchronisation and can be captured in a HIP graph.  Two renders of
 * one batch must not overlap (same stream, or ordered by events). */
mrs_status mrs_batch_render(mrs_batch* batch);
/* mrs_batch_render in two calls, for frame pipelines.  _begin enqueues the
 * render on the current stream up to its last per-pixel sums: the wavefront
 * runs on the library's sub-chunk streams from there on.  _end, on the same
 * stream, enqueues those sums and the resolve; until then the caller's stream
 * may take other work, which runs concurrently with the render (e.g. the
 * fusion network on the previous frame's images).  The batch's outputs are
 * written only by _end, so work enqueued between the two calls may still read
 * them (the previous frame's values).  Errors (MRS_ERR_INVALID_ARGUMENT, no
 * effect): _begin while a render of the batch is begun and not ended, _end
 * with none begun or on another stream.  Begin + end is mrs_batch_render,
 * bitwise.  No allocation, no host synchronisation. */
mrs_status mrs_batch_render_begin(mrs_batch* batch);
mrs_status mrs_batch_render_end(mrs_batch* batch);
/* The start of the batch's next render, marked ahead of its launches, for frame
 * pipelines: on the current stream, clears the batch's per-pixel sums and marks
 * the point the render's sub-chunk streams start from.  The next
 * mrs_batch_render_begin (or mrs_batch_render) on the same stream then starts
 * its wavefront from that point, so work enqueued on the stream between the two
 * calls (e.g. the fusion of the previous frame, enqueued before the ~50
 * launches of the wavefront) runs beside the render instead of before it.
 * Seeds set after the fork undo it (the next begin forks again); a begin on
 * another stream ignores it.  Same results, no allocation, no host
 * synchronisation.  Error (MRS_ERR_INVALID_ARGUMENT, no effect): a render of the
 * batch begun and not ended. */
mrs_status mrs_batch_render_fork(mrs_batch* batch);
/* Replaces the seed of every job (seeds[i] for job i, as many as the batch
 * has jobs): enqueues a small update of the device job table on the current
 * stream, ordered before later renders of the batch.  No allocation. */
mrs_status mrs_batch_set_seeds(mrs_batch* batch, const uint64_t* seeds);
/* Synchronises the device, then frees the batch.  NULL is accepted. */
mrs_status mrs_batch_destroy(mrs_batch* batch);

/* Single renders use a path workspace per stream (renders on different
 * streams run concurrently; a built scene is read-only).  A workspace grows on
 * the first render that needs more room (hipMalloc, so not under graph
 * capture: run the same call shapes on the capturing stream once first) and is
 * kept until this call, which synchronises the device and frees them all. */
mrs_status mrs_release_workspaces(void);

/* Counters accumulated by every stream since the last reset (synchronises
 * the current stream):
 * [0] non-finite samples replaced by 0, [1] closest-hit rays, [2] shadow rays,
 * [3] traversal stack entries spilled from LDS to global memory,
 * [4] paths started, [5] stack overflows (must be 0),
 * [6] closest-hit node visits, [7] closest-hit triangle tests,
 * [8] shadow node visits, [9] shadow triangle tests,
 * [10] / [11] most node visits + triangle tests of one closest-hit / shadow ray,
 * [12] / [13] closest-hit / shadow rays traced by the path-tail kernel (also
 * included in [1] / [2]), [14] / [15] its node visits / triangle tests
 * ([6]..[11], [14], [15] only while work counting is on, see
 * mrs_set_count_work; [6]..[9] cover the wavefront kernels only). */
#define MRS_NUM_COUNTERS 16
mrs_status mrs_get_counters(int64_t out[MRS_NUM_COUNTERS], int32_t reset);

/* Work counting: while on, traversal kernels also count node visits and
 * triangle tests (a slower variant of the same kernels; results identical). */
mrs_status mrs_set_count_work(int32_t on);

/* Kernel timing with HIP events recorded on the launch stream around every
 * launch of the library's kernels, by kernel id:
 * 0 generate, 1 extend (closest hit), 2 shade, 3 shadow (any hit),
 * 4 accumulate, 5 resolve, 6 network input preparation, 7 network HR input conv,
 * 8 network LR convs (lrhs, fuse, trunk, up), 9 network HR output conv,
 * 10 training forward, 11 training backward, 12 Adam + weight refresh,
 * 13 path tail (bounces from mrs_tuning.tail_bounce on), 14..15 reserved.
 * mrs_profile_enable(1) clears the totals and starts recording;
 * mrs_profile_read synchronises and returns, per id, the summed milliseconds
 * and the launch count of the launches recorded so far.
 * mrs_profile_select(mask) limits the recording to the ids whose bit is set
 * in mask (default: all), so that a timed run pays for the events of the
 * kernels it reports only. */
#define MRS_NUM_KERNEL_IDS 16
mrs_status mrs_profile_enable(int32_t on);
mrs_status mrs_profile_select(uint32_t mask);
mrs_status mrs_profile_read(double ms_out[MRS_NUM_KERNEL_IDS],
                            int64_t launches_out[MRS_NUM_KERNEL_IDS]);

/* Tuning knobs (performance only; results do not depend on them). */
typedef struct mrs_tuning {
  int32_t chunk_paths;  /* paths resident at once (default 1<<23, at most 1<<26) */
  int32_t trace_blocks; /* grid size of traversal kernels (default 8192) */
  int32_t schedule;     /* traversal queue: 0 grid-stride (default), 1 per-wave
                           dynamic fetch from a device counter */
  int32_t bvh_leaf_max; /* triangles a BVH4 leaf may group, 1..4 (default 3);
                           applies to scenes built afterwards */
  int32_t streams;      /* 1..4 (default 3): a render's resident paths are cut into
                           this many sub-chunks, traced concurrently on internal
                           streams shared by the library (joined back into the
                           caller's stream before the per-pixel sums) */
  int32_t tail_bounce;  /* 1..65 (default 3): bounces from this one on are traced
                           path by path in one launch (65: never) */
  int32_t bvh_builder;  /* MRS_BVH_PLOC (default) or MRS_BVH_LBVH; applies to
                           scenes built afterwards */
  int32_t conv_small_tiles; /* 0..2^30 (default 128): a 3x3 network conv whose
                           output has fewer 16x16-pixel tiles than this (over
                           the batch) runs on 16x8 tiles of 4 waves with its
                           output channels split over blocks; otherwise on
                           16x16 tiles of 8 waves (0: always the large tiles).
                           Both sum in the same order: outputs are bitwise
                           the same */
  int32_t queue_sort;   /* 1 (default): the shade kernel orders each block's
                           appended rays by direction octant and its shadow rays
                           by light, so that a wave of the next traversal holds
                           alike rays; 0: in lane order */
  int32_t bvh_quantized; /* 1: traversal reads the 64-byte copy of each BVH4
                           node whose child boxes are 8-bit steps from the node's
                           origin, rounded outward with a margin; 0 (default):
                           the 128-byte nodes with FP32 boxes.  Same hits */
  int32_t wave_extend;  /* 0..65 (default 1): closest-hit rays of the bounces
                           below this one are traced a wave at a time (the 64
                           rays of a wave walk one tree order together; node
                           loads, stack and child order shared by the wave),
                           the rest lane by lane.  Same hits */
  int32_t wave_shadow;  /* 0..65 (default 0): the same for shadow rays */
  int32_t net_fused_blocks; /* 1 (default): each residual block of the 16-block
                           network's trunk runs as one kernel (both convs, the
                           intermediate kept in LDS) when the LR image has at
                           least conv_small_tiles 16x16 tiles; 0: two conv
                           launches.  Bitwise the same */
} mrs_tuning;
mrs_status mrs_get_tuning(mrs_tuning* out);
mrs_status mrs_set_tuning(const mrs_tuning* t);

/* ------------------------------------------------------------ fusion network */

/* The HRLS + LRHS fusion network of the hybrid method (paper Sec. 4, Fig. 3):
 *   h0  = ReLU(conv3x3 10->64) on HRLS (rgb, albedo, normal, depth)    HR
 *   fl  = ReLU(conv3x3 3->64) on LRHS rgb                               LR
 *   F0  = ReLU(conv1x1 [fl, unshuffle4(h0)] 1088->64)   (deshuffle + fuse)
 *   r  <- r + 0.1 conv3x3(ReLU(conv3x3(r))) x 16, r_0 = F0   (trunk)
 *   FDF = r_16 + F0                                      (global residual)
 *   out = conv3x3 [shuffle4(ReLU(conv3x3 64->256 FDF)), h0] 80->3    HR
 * Every conv is 3x3 except the 1x1 fuse, ReLU after every conv but the last
 * (Sec. 4, implementation details).  Inputs are preprocessed on the device:
 * RGB clipped to [0, 100] (Sec. 3.2) then log1p, depth log1p, albedo and normal
 * as rendered.  unshuffle by r maps HR pixel (rY+i, rX+j) channel c to LR
 * channel (i r + j) C + c; shuffle is its inverse.  Convolutions run as BF16
 * MFMA implicit GEMMs with FP32 accumulation; the residual stream is FP32.
 * Parameters: MRS_NET_NUM_PARAMS FP32 values, layer by layer (hrls, lrhs, fuse,
 * res0a, res0b, ..., res15b, up, rec), each weight [C_out][C_in][k][k] then
 * bias [C_out]. */
typedef struct mrs_net mrs_net;
#define MRS_NET_NUM_PARAMS 1408883

/* Network architectures:
 * MRS_NET_RES16  the network above (16 residual blocks).
 * MRS_NET_RDG    the paper's own network (Sec. 4, Fig. 4):
 *   h0   = ReLU(conv3x3 10->64) on HRLS                              HR
 *   fl   = ReLU(conv3x3 3->64) on LRHS                               LR
 *   F0   = ReLU(conv1x1 [fl, DSF(DSF(h0))] 1088->64)   two stacked stride-2
 *          deshuffles: HR pixel (4Y+I, 4X+J) channel c -> LR channel
 *          (2 (I>>1) + (J>>1)) 256 + (2 (I&1) + (J&1)) 64 + c
 *   RDB: x_c = ReLU(conv3x3 [x_0 .. x_{c-1}] -> 64) for c = 1..3, output
 *        x_0 + conv3x3 [x_0 .. x_3] 256->64 (no ReLU before the block's skip)
 *   F_g  = RDB^5(F_{g-1}) + F_{g-1} for g = 1..3 (residual dense groups)
 *   FDF  = F_3 + F0
 *   UP   = twice: shuffle2(ReLU(conv3x3 64->256))   (sub-pixel, ESPCN)
 *   out  = conv3x3 UP(FDF) 64->3                                     HR
 *   Parameters (MRS_NET_RDG_NUM_PARAMS): hrls, lrhs, fuse, g0b0c0 .. g0b0c3,
 *   g0b1c0, ..., g2b4c3, up0, up1, rec, each weight [C_out][C_in][k][k] then
 *   bias [C_out]; conv c of a block reads channels [x_0, .., x_{c}] in that
 *   order.  mrs_net_init scales the bound of each block's last conv and of rec by 0.1. */
#define MRS_NET_RES16 0
#define MRS_NET_RDG 1
#define MRS_NET_RDG_NUM_PARAMS 5907907
/* The paper's network at x2 and x8 (Sec. 4: D stacked stride-2 deshuffles for
 * scale 2^D, as many upscaling steps; the fuse conv reads 64 + 64 4^D
 * channels): 5,711,043 and 6,252,227 parameters (up0..up{D-1}).  W and H (and
 * the LRHS image, W/s x H/s) must be multiples of the scale s. */
#define MRS_NET_RDG_X2 2
#define MRS_NET_RDG_X8 3
/* The x4 networks with the HRLS render layers as inputs (Sec. 4, first
 * paragraph: I_HRLS is RGB plus albedo, normal, diffuse, specular and variance
 * layers; the layers are those of Sec. 3.1): the HRLS input conv reads 16
 * channels instead of 10 -- log1p of the clipped RGB, albedo (3), normal (3),
 * log1p of the clipped diffuse and glossy layers (3 + 3), and log1p of the
 * per-sample variance averaged over RGB, mean_c(sumsq_c / spp - rgb_c^2)
 * clamped to [0, 1e4] (1); depth is not an input.  Everything else is the
 * network of MRS_NET_RES16 / MRS_NET_RDG; 1,412,339 / 5,911,363 parameters.
 * These networks read the layers from the buffers bound with
 * mrs_net_bind_layers; every fuse / train / gradient call on them returns
 * NOT_READY until some are bound. */
#define MRS_NET_RES16_LAYERS 4
#define MRS_NET_RDG_LAYERS 5

int64_t mrs_net_num_params(void);                 /* MRS_NET_RES16's count */
int64_t mrs_net_arch_num_params(int32_t arch);     /* -1 for an unknown arch */
mrs_status mrs_net_create(mrs_net** out); /* MRS_NET_RES16; parameters unset: mrs_fuse is NOT_READY */
/* A network of the given architecture; INVALID_ARGUMENT for an unknown one. */
mrs_status mrs_net_create_arch(int32_t arch, mrs_net** out);
mrs_status mrs_net_destroy(mrs_net* net);
/* Binds the HRLS render layers that the MRS_NET_*_LAYERS networks read in every
 * later mrs_fuse / mrs_fuse_batch / mrs_train_step(_ex) / mrs_net_loss_grad(_ex)
 * / mrs_net_backward call: layers_dev B*H*W*9 FP32 (emission, diffuse, glossy:
 * a render's out_layers_dev) and sumsq_dev B*H*W*3 FP32 (its out_sumsq_dev),
 * laid out like hrls_rgb_dev of those calls, and spp the render's samples per
 * pixel.  The buffers stay owned by the caller and must hold the B, W and H of
 * each call that reads them.  NULL, NULL, 0 unbinds.  INVALID_ARGUMENT for a
 * network without layer inputs, NULL or misaligned buffers or spp < 1. */
mrs_status mrs_net_bind_layers(mrs_net* net, const float* layers_dev, const float* sumsq_dev,
                               int32_t spp);

/* He-uniform weights (bound sqrt(6 / fan_in)) from Philox4x32-10 with key seed,
 * counter (parameter index lo, hi, 0, 2); zero biases.  On the device. */
mrs_status mrs_net_init(mrs_net* net, uint64_t seed);
/* Copies `count` (= MRS_NET_NUM_PARAMS) FP32 masters from host memory and
 * refreshes the packed BF16 weights; synchronises. */
mrs_status mrs_net_set_params(mrs_net* net, const float* params_host, int64_t count);
mrs_status mrs_net_get_params(const mrs_net* net, float* params_host, int64_t count);

/* I_SR = Net(I_LRHS, I_HRLS) for one frame: hrls_rgb_dev H*W*3, hrls_aux_dev
 * H*W*7 (as written by mrs_render), lrhs_rgb_dev (H/4)*(W/4)*3, out_rgb_dev
 * H*W*3, all FP32 HWC device buffers.  W, H multiples of 4.  The network's
 * activations live in a per-net device arena grown on demand; calls on one
 * net must not overlap.  NOT_READY without parameters. */
mrs_status mrs_fuse(mrs_net* net, const float* hrls_rgb_dev, const float* hrls_aux_dev,
                    const float* lrhs_rgb_dev, int32_t W, int32_t H, float* out_rgb_dev);
/* The same for B frames stored one after the other (NHWC). */
mrs_status mrs_fuse_batch(mrs_net* net, int32_t B, const float* hrls_rgb_dev,
                          const float* hrls_aux_dev, const float* lrhs_rgb_dev, int32_t W,
                          int32_t H, float* out_rgb_dev);

/* One training step: forward on B frames (saving activations), L1 loss
 * mean |I_SR - clip(target, 0, 100)| reduced in FP64, backward through every
 * layer (BF16 MFMA data and weight gradients, FP32 accumulation), then Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the FP32 masters and
 * a refresh of the BF16 copies.  Buffers as for mrs_fuse_batch plus target_dev
 * B*H*W*3.  If loss_host is not NULL the stream is synchronised and the loss
 * of this step (before the update) is written there.  B*W*H <= 2^26. */
mrs_status mrs_train_step(mrs_net* net, int32_t B, const float* hrls_rgb_dev,
                          const float* hrls_aux_dev, const float* lrhs_rgb_dev,
                          const float* target_dev, int32_t W, int32_t H, float lr,
                          double* loss_host);

/* Forward + loss + backward without an update: the FP32 gradient of every
 * parameter (MRS_NET_NUM_PARAMS, master layout) to grad_host, the loss to
 * loss_host and the network output to out_dev (each optional).  Synchronises. */
mrs_status mrs_net_loss_grad(mrs_net* net, int32_t B, const float* hrls_rgb_dev,
                             const float* hrls_aux_dev, const float* lrhs_rgb_dev,
                             const float* target_dev, int32_t W, int32_t H, float* grad_host,
                             double* loss_host, float* out_dev);

/* Forward (saving activations) and backward from a caller-supplied output
 * gradient dL/dI_SR (grad_out_dev, FP32 B*H*W*3 device buffer, used as BF16)
 * in place of a built-in loss: for any loss computed outside the library.
 * Writes the FP32 gradient of every parameter (master layout) to grad_host if
 * not NULL.  Synchronises. */
mrs_status mrs_net_backward(mrs_net* net, int32_t B, const float* hrls_rgb_dev,
                            const float* hrls_aux_dev, const float* lrhs_rgb_dev, int32_t W,
                            int32_t H, const float* grad_out_dev, float* grad_host);

/* Losses and optimisers of mrs_train_step_ex.
 * MRS_LOSS_L1      mean |I_SR - t| (t = clip(target, 0, 100)).
 * MRS_LOSS_ROBUST  the paper's robust loss (Sec. 4): mean |d| / (beta + |d|),
 *                  d = I_SR - t, beta > 0 (the paper uses 0.1); gradient
 *                  sign(d) beta / (beta + |d|)^2 / N.  Reduced in FP64.
 * MRS_OPT_ADAM     Adam as in mrs_train_step (counts its own steps).
 * MRS_OPT_SGD      w -= lr g (the paper's optimiser). */
#define MRS_LOSS_L1 0
#define MRS_LOSS_ROBUST 1
#define MRS_OPT_ADAM 0
#define MRS_OPT_SGD 1
typedef struct mrs_train_opts {
  int32_t loss;
  float beta;
  int32_t optimizer;
  float lr;
} mrs_train_opts;

/* mrs_train_step with a choice of loss and optimiser; INVALID_ARGUMENT for an
 * unknown loss or optimiser, beta <= 0 with the robust loss, or lr <= 0. */
mrs_status mrs_train_step_ex(mrs_net* net, int32_t B, const float* hrls_rgb_dev,
                             const float* hrls_aux_dev, const float* lrhs_rgb_dev,
                             const float* target_dev, int32_t W, int32_t H,
                             const mrs_train_opts* opts, double* loss_host);
/* mrs_net_loss_grad with a choice of loss (beta as in mrs_train_opts). */
mrs_status mrs_net_loss_grad_ex(mrs_net* net, int32_t B, const float* hrls_rgb_dev,
                                const float* hrls_aux_dev, const float* lrhs_rgb_dev,
                                const float* target_dev, int32_t W, int32_t H, int32_t loss,
                                float beta, float* grad_host, double* loss_host,
                                float* out_dev);

/* Checkpoint state: FP32 masters, Adam first and second moments, step count
 * (host arrays of `count` = MRS_NET_NUM_PARAMS floats).  set_state then
 * continuing is bitwise the same as never having stopped. */
mrs_status mrs_net_get_state(const mrs_net* net, float* params, float* adam_m, float* adam_v,
                             int64_t count, int64_t* step);
mrs_status mrs_net_set_state(mrs_net* net, const float* params, const float* adam_m,
                             const float* adam_v, int64_t count, int64_t step);

/* Checkpoint files (training resume).  mrs_net_save writes the state of
 * mrs_net_get_state plus a caller-defined data counter (e.g. the position in
 * the training data order) to `path`: a 48-byte little-endian header -- magic
 * "MRSCKPT\0", u32 version 1, i32 architecture (MRS_NET_*), i64 parameter
 * count, i64 Adam step, u64 data counter, u32 CRC-32 (IEEE 802.3) of the body,
 * u32 CRC-32 of the 44 header bytes before it -- then the body: the FP32
 * masters, Adam m and Adam v, `count` values each.  It writes `path`.tmp and
 * renames it over `path`, so a failed save leaves an existing file intact.
 * Synchronises the current stream.  NOT_READY without parameters; DEVICE if
 * the file cannot be written.
 * mrs_net_load reads and checks the whole file (magic, both checksums,
 * version, the net's architecture and count, exact length) before it changes
 * anything: any mismatch returns INVALID_ARGUMENT and leaves the net as it
 * was.  Then it sets the state as mrs_net_set_state does and stores the data
 * counter in *data_counter (if not NULL).  Save, load and continue training is
 * bitwise the same as never having stopped. */
mrs_status mrs_net_save(const mrs_net* net, const char* path, uint64_t data_counter);
mrs_status mrs_net_load(mrs_net* net, const char* path, uint64_t* data_counter);

/* ------------------------------------------------------------ metrics */

/* Evaluation metrics of the paper (Sec. 5) between two FP32 device images of
 * `count` values (pixels x channels, scene-linear):
 *   out[0] = MSE of the sRGB values (Eq. 3: 0 for l <= 0, 12.92 l up to
 *            0.0031308, 1.055 l^(1/2.4) - 0.055 below 1, then 1),
 *   out[1] = PSNR = 10 log10(1 / out[0]) (peak 1; +inf when equal),
 *   out[2] = RelMSE = mean of lambda1 (img - ref)^2 / (ref^2 + lambda2)
 *            (the paper uses 0.5 and 0.01 on its dataset).
 * FP64 accumulation in a fixed order; synchronises the stream. */
mrs_status mrs_image_metrics(const float* img_dev, const float* ref_dev, int64_t count,
                             double lambda1, double lambda2, double out[3]);

/* ------------------------------------------------------- debug / test hooks */

/* FP32 copy of an activation of the last mrs_fuse on `net`: which 0 = F0,
 * 1 = FDF, each B*(H/4)*(W/4)*64 values (count must match).  Synchronises. */
mrs_status mrs_debug_net_activation(const mrs_net* net, int32_t which, float* out_host,
                                    int64_t count);

/* Launches of each network conv kernel since the last reset, counted on the
 * host when enqueued (so a captured graph counts once): [0] 3x3 LDS conv on
 * 16x8 tiles, 64-channel input chunks, output channels split over blocks;
 * [1] 3x3 LDS conv on 16x16 tiles, 64-channel chunks; [2] / [3] the same with
 * 16 / 8 input channels (the HR and LR input convs); [4] / [5] 3x3 LDS convs
 * with fewer than 64 output channels (80 / 64 input channels: the
 * reconstruction convs); [6] / [7] the direct implicit-GEMM conv (64 / 16
 * output channels per block: the 1x1 fuse conv and shapes the LDS kernels do
 * not take); [8] / [9] the data-gradient convs of training on the LDS conv
 * (16x8 / 16x16 tiles; the others run a direct implicit GEMM, not counted);
 * [10] a residual block of the trunk as one kernel (two 3x3 convs, counted
 * once).  reset != 0 clears the counts after reading them. */
#define MRS_NUM_CONV_KINDS 11
mrs_status mrs_debug_conv_launches(int64_t out[MRS_NUM_CONV_KINDS], int32_t reset);

/* Philox4x32-10 on the device: out_dev[4i..4i+3] = philox(ctr_dev[4i..4i+3],
 * key_dev[2i..2i+1]) for i < n.  For bitwise checks against the host. */
mrs_status mrs_debug_philox(int32_t n, const uint32_t* ctr_dev, const uint32_t* key_dev,
                            uint32_t* out_dev);

/* Closest hit through the LBVH for n rays: origins/directions as xyz float
 * triples, skip_dev[i] a primitive to exclude (-1 for none) or NULL.
 * Writes t (inf on a miss), primitive (-1 on a miss) and barycentrics b1, b2. */
mrs_status mrs_debug_closest_hit(const mrs_scene* scene, int32_t n, const float* o_dev,
                                 const float* d_dev, const int32_t* skip_dev, float* t_dev,
                                 int32_t* prim_dev, float* b_dev);

/* Copies the LBVH to host memory for invariant checks.  nodes_host receives
 * (num_tris-1) records of 16 floats: left box lo xyz, hi xyz, right box lo
 * xyz, hi xyz, then left/right child references as uint32 bit patterns (bit 31
 * set = leaf, low bits = leaf slot), 2 pad words.  leaf_prim_host receives
 * num_tris primitive ids in leaf order; morton_host the sorted Morton codes.
 * Any pointer may be NULL.  Synchronises. */
mrs_status mrs_debug_bvh(const mrs_scene* scene, float* nodes_host, int32_t* leaf_prim_host,
                         uint32_t* morton_host, int32_t* root_ref_host);

/* Copies the four-wide BVH the renderer traverses (collapsed from the LBVH).
 * nodes_host (NULL to query the count) receives count records of 32 floats:
 * child boxes lo.x[4], lo.y[4], lo.z[4], hi.x[4], hi.y[4], hi.z[4], then 4
 * child references as uint32 bit patterns (0xffffffff = no child; bit 31 set
 * = leaf: bits 24..25 = count - 1, bits 0..23 = first leaf slot, covering
 * leaf slots first .. first + count - 1; otherwise a node index), 4 pad words.
 * root_ref is a reference in the same encoding; leaf_max is the grouping
 * limit the build used.  Synchronises. */
mrs_status mrs_debug_bvh4(const mrs_scene* scene, float* nodes_host, int32_t* count,
                          uint32_t* root_ref, int32_t* leaf_max);

#ifdef __cplusplus
}
#endif

#endif /* MRS_H_ */
