/*
 * sg.h -- C ABI of the MI355X (gfx950) stereo volume ray caster.
 *
 * Direct volume ray casting through a bricked, multiresolution (octree LOD)
 * volume, following syGlass (arXiv 1804.08197): Sec 5.1 (ray casting with the
 * emission-absorption model and early ray termination), Sec 5.2 (octree
 * blocks in a multi-resolution pyramid, top-down LOD selection, front-to-back
 * block order), Sec 5.3 (one render per eye of a head-mounted display),
 * Sec 4.1/4.2 (volume chunks uploaded to a GPU-resident cache), Sec 5.6
 * (pre-multiplied alpha output; rays ending at the depth of opaque geometry),
 * Sec 6 (cut plane and region-of-interest tools) and Sec 8 (transfer
 * functions, multichannel).
 *
 * Conventions shared by every call
 *  - World space is level-0 voxel units: voxel (i, j, k) covers
 *    [i, i+1) x [j, j+1) x [k, k+1) with its value at the centre; the volume
 *    box is [0, dims]. Voxel arrays are x fastest.
 *  - Every function returns an sg_status and never throws. Argument and state
 *    errors are reported synchronously; asynchronous device errors surface on
 *    a later call or on stream synchronisation. sg_last_error() gives a
 *    thread-local description of the last failure.
 *  - hip_stream is a hipStream_t (NULL = the default stream). Device work is
 *    enqueued on it in order; device pointers passed in are read or written
 *    in that stream order.
 *  - Ownership: the library owns everything it allocates for a volume (brick
 *    pool, page table, transfer functions, per-view scratch); the caller owns
 *    its inputs and output buffers. A volume is not thread-safe; distinct
 *    volumes are independent.
 *  - There is no CPU fallback: without a usable gfx950 device the calls that
 *    need one return SG_ERR_DEVICE.
 */
#ifndef SG_H
#define SG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SG_ABI_VERSION 5

typedef enum {
  SG_OK = 0,
  SG_ERR_INVALID_ARG = -1,   /* NULL, out of range, NaN or inconsistent input */
  SG_ERR_OUT_OF_MEMORY = -2, /* device allocation failed (e.g. pool > HBM)   */
  SG_ERR_DEVICE = -3,        /* no device, or a HIP runtime call failed        */
  SG_ERR_STATE = -4,         /* call not valid now (e.g. no transfer function) */
  SG_ERR_UNSUPPORTED = -5    /* valid request the library does not implement  */
} sg_status;

typedef enum { SG_U8 = 1, SG_U16 = 2 } sg_dtype;

/* Order of the voxels inside a pool slot, sg_volume_desc.layout. Images are
 * bit-identical under both; only their speed differs.
 *  - SG_LAYOUT_LINEAR: x fastest, rows padded to a multiple of 4 bytes.
 *  - SG_LAYOUT_MICROBLOCK: the slot is cut into 4x4x4-voxel blocks (the
 *    stored edge rounded up to a multiple of 4), each block contiguous
 *    (x fastest inside it) and the blocks in x-fastest order: a block of
 *    16-bit voxels is one 128-byte cache line, so a brick region staged for
 *    the rays of a screen tile reads whole lines (large volumes rendered
 *    by the staged kernel: about 4x fewer bytes fetched from HBM than rows
 *    of the linear layout). */
typedef enum { SG_LAYOUT_LINEAR = 0, SG_LAYOUT_MICROBLOCK = 1 } sg_layout;

/* Optical models (Sec 5.1), sg_render_params.model. */
typedef enum {
  SG_MODEL_EMISSION_ABSORPTION = 0, /* C += (1-A) a rgb, A += (1-A) a with
                                       a = 1 - exp(-rho s); early termination */
  SG_MODEL_EMISSION_ONLY = 1,       /* C += rgb s, rgb the summed emission of
                                       the channels; A stays 0 (Sec 5.6)     */
  SG_MODEL_MAX_INTENSITY = 2        /* per channel the largest trilinear value
                                       along the ray; C = summed emission of
                                       those maxima, A = 0                   */
} sg_model;

/* sg_render_params.flags */
enum {
  SG_LOD = 1u << 0,        /* screen-space LOD cut (Sec 5.2); without it every
                              node is rendered at level lod_bias             */
  SG_SKIP_EMPTY = 1u << 1, /* skip nodes that cannot contribute: zero opacity
                              (emission-absorption), zero emission
                              (emission-only), a stored maximum no larger than
                              the ray's running maxima (maximum intensity);
                              the image is the same either way              */
  SG_GATHER = 1u << 2      /* tuning/testing: trilinear stencils read the brick
                              pool directly instead of LDS-staged brick tiles;
                              the image is bit-identical either way          */
};

typedef struct sg_volume sg_volume; /* opaque */

/* Volume geometry. The brick pool holds, for every channel and timepoint,
 * every node of the pyramid: level L has dims ceil(dims / 2^L) voxels,
 * split into bricks of brick^3 core voxels stored with a one-voxel apron
 * ((brick+2)^3 voxels per slot). */
typedef struct {
  int32_t dims[3];    /* level-0 voxels per axis, >= 1                        */
  int32_t channels;   /* 1..4                                                 */
  int32_t timepoints; /* >= 1                                                 */
  int32_t dtype;      /* sg_dtype                                             */
  int32_t brick;      /* core edge: power of two in [2, 256]                  */
  int32_t levels;     /* pyramid levels, 1..16 (1 = no pyramid)               */
  int32_t device;     /* HIP device ordinal                                   */
  int32_t cache_slots; /* 0: every node of every channel and timepoint has a
                          pool slot. > 0: the pool is a cache of this many
                          slots (out-of-core mode, see sg_cache_put)         */
  int32_t layout;     /* sg_layout of the pool slots                          */
} sg_volume_desc;

/* One eye / camera (Sec 5.1: one ray per pixel; Sec 5.3: one view per eye).
 * The camera looks down its own -z axis. cam_to_world is row-major 4x4 with
 * the eye position in its last column (m[3], m[7], m[11]) and a rotation in
 * its upper-left 3x3. The image plane at distance 1 spans
 * [tan_left, tan_right] x [tan_bottom, tan_top] (asymmetric frusta allowed);
 * pixel (x, y) has its centre at tangent
 *   (sx, sy) = (tan_left + (x + 0.5) / width * (tan_right - tan_left),
 *               tan_top  - (y + 0.5) / height * (tan_top - tan_bottom)),
 * row 0 at the top.
 * Wrapped space (Sec 5.3: rays spread uniformly over the image the lens
 * distortion is applied to): with lens = {k1, k2, cx, cy} not both k zero,
 * each pixel's tangent is moved radially about (cx, cy):
 *   (sx, sy) <- (cx, cy) + (sx - cx, sy - cy) * (1 + k1 r^2 + k2 r^4),
 *   r^2 = (sx - cx)^2 + (sy - cy)^2.
 * The LOD pixel angle stays (tan_top - tan_bottom) / height.
 * ray_limit (Sec 5.6: rays end at the distance of opaque geometry read from
 * a depth texture): NULL, or a device float [height][width] of distances
 * along each pixel's ray from the eye (level-0 units); samples lie in front
 * of it (+inf or NaN: no limit). Read in stream order; ignored by
 * sg_get_lod_cut.
 * tile_any: NULL, or a device uint8 [(height + 7) / 8][(width + 7) / 8]
 * that the render fills, one byte per 8x8-pixel block of the image (block
 * (bx, by) holds pixels 8 bx .. 8 bx + 7, 8 by .. 8 by + 7): 1 if any of its
 * pixels has a nonzero output RGBA (background included) or, when depth is
 * written, a finite depth; else 0: a content mask of the image for passes
 * that run over it later. The mask describes the pixels of each block only:
 * a consumer whose output at a pixel depends on neighbouring pixels (a
 * filter or a network with a receptive field) must dilate it by that reach
 * itself. */
typedef struct {
  double cam_to_world[16];
  double tan_left, tan_right, tan_bottom, tan_top;
  int32_t width, height; /* >= 1 */
  double lens[4];        /* k1, k2, cx, cy; all 0 = rectilinear           */
  const float *ray_limit;
  uint8_t *tile_any;
} sg_view;

typedef struct {
  double step_voxels;   /* sample spacing in voxels of the sampled level (0.5),
                           in [1/64, 64]                                      */
  double ert_alpha;     /* stop a ray once its alpha >= this (0.99); > 1 = off */
  double lod_tau_px;    /* LOD: largest voxel footprint in pixels (1.0)        */
  double background[4]; /* premultiplied RGBA composited under the volume     */
  double depth_alpha;   /* depth output: first sample with alpha >= this (0.5) */
  int32_t lod_bias;     /* finest level used (0 = full resolution)            */
  int32_t timepoint;    /* 0 .. timepoints-1                                  */
  uint32_t flags;       /* SG_LOD | SG_SKIP_EMPTY | SG_GATHER                 */
  int32_t model;        /* sg_model                                           */
  /* Clipping of every ray (Sec 6): cut plane j keeps the points p with
   * nx px + ny py + nz pz + w <= 0 (planes[j] = {nx, ny, nz, w}, finite,
   * normal not zero); with roi_on only the box roi = {lo x, y, z, hi x, y, z}
   * (level-0 units, lo <= hi) is kept. */
  int32_t n_planes;     /* 0..4                                              */
  int32_t roi_on;       /* 0 or 1                                            */
  double planes[4][4];
  double roi[6];
} sg_render_params;

/* Optional instrumentation of one render (sg_render_views_stats). */
typedef struct {
  int32_t *const *samples; /* in: per view a device int32 [height*width]
                              buffer for per-pixel sample counts, or NULL    */
  uint64_t total_samples;  /* out: samples evaluated over all views          */
  uint64_t microblocks;    /* out: distinct 4^3 voxel blocks (per channel and
                              level) read by the trilinear stencils          */
  uint64_t node_visits;    /* out: (wave, node) pairs sampled (staged kernel)
                              or (ray, node) segments sampled (gather)       */
  uint64_t slabs;          /* out: LDS staging passes (staged kernel)        */
  uint64_t staged_bytes;   /* out: bytes copied from the pool into LDS       */
  uint64_t node_lanes;     /* out: staged kernel: sum over (wave, node) visits
                              of the lanes whose ray is in that node         */
  uint64_t loop_iterations; /* out: staged kernel: wave iterations of the
                              sample loops (LDS and pool reads); the lane
                              utilisation of the loops is
                              total_samples / (64 * loop_iterations)        */
  uint64_t pool_samples;   /* out: staged kernel: samples whose stencils read
                              the pool, not LDS (the node's rays share no
                              dominant direction, or one layer of the slab
                              does not fit the staging space)               */
  uint64_t slab_retries;   /* out: staged kernel: slab sizes tried beyond the
                              first (the region did not fit)               */
  uint64_t alive_lanes;    /* out: staged kernel: sum over (wave, node) visits
                              of the lanes whose ray is still in flight (in
                              that node or in another)                      */
  uint64_t wide_slabs;     /* out: staged kernel: slabs whose region rows
                              were wider than one 64-lane copy pass (bricks
                              of 128 voxels or more), copied chunk by chunk */
} sg_render_stats;

/* Create a volume on desc->device (Sec 4.2: the GPU-side store of volume
 * chunks; Sec 5.2: blocks of every level of the multi-resolution pyramid):
 * allocates the brick pool for every channel, timepoint and node (or
 * cache_slots slots), the page table (node -> pool slot) and the per-node
 * value ranges. The pool starts zeroed.
 * Errors: SG_ERR_INVALID_ARG (bad desc, out NULL), SG_ERR_OUT_OF_MEMORY,
 * SG_ERR_DEVICE. On success *out owns all of it until sg_volume_destroy. */
sg_status sg_volume_create(const sg_volume_desc *desc, sg_volume **out);

/* Release every device allocation of vol (after synchronising its device):
 * the end of the GPU store of Sec 4.2. vol must not be used afterwards. */
sg_status sg_volume_destroy(sg_volume *vol);

/* Upload n brick cores of one (channel, timepoint, level) into the pool
 * (Sec 4.1: decompressed chunks uploaded to the GPU; Sec 4.2: GPU cache).
 *   coords : host int32 [n][3] brick indices (bx, by, bz) at that level
 *   src    : n consecutive cores of brick^3 voxels (x fastest) of the
 *            volume's dtype; a host pointer (copied before the call returns)
 *            or, if src_on_device, a device pointer read in stream order.
 * Core voxels outside the level's extent (partial bricks at the far faces)
 * are ignored: commit replaces them by the clamped edge values.
 * Marks the channel/timepoint for commit (apron fill, value ranges). */
sg_status sg_upload_bricks(sg_volume *vol, int32_t channel, int32_t timepoint,
                           int32_t level, int32_t n, const int32_t *coords,
                           const void *src, int32_t src_on_device,
                           void *hip_stream);

/* Build levels 1..levels-1 of one (channel, timepoint) from its level-0
 * cores on the device (Sec 5.2 multi-resolution pyramid): each coarse voxel
 * is (sum of its 2x2x2 children + 4) >> 3, child indices clamped to the
 * finer level. Marks the channel/timepoint for commit. */
sg_status sg_build_lod(sg_volume *vol, int32_t channel, int32_t timepoint,
                       void *hip_stream);

/* Finish pending uploads/builds on the device (Sec 5.2: every block of the
 * pyramid samples on its own, so each carries the neighbour voxels its
 * trilinear stencils reach; Sec 5.1: blocks whose opacity is zero under the
 * transfer function contribute nothing): fill every brick's apron (and
 * out-of-extent core voxels) with clamped neighbour values, recompute
 * per-brick min/max, and recompute empty-node flags. sg_render_views calls
 * this itself when something is pending. Errors: SG_ERR_INVALID_ARG (vol
 * NULL), SG_ERR_DEVICE. Asynchronous on hip_stream. */
sg_status sg_volume_commit(sg_volume *vol, void *hip_stream);

/* Set the transfer function of a channel (Sec 5.1 tau and T; Sec 8):
 * rgba is a host float [n_entries][4] table, copied before return: r, g, b
 * are the emitted colour, a the extinction per level-0 voxel length. Entry
 * k sits at raw value domain_lo + k/(n_entries-1) * (domain_hi - domain_lo);
 * lookups interpolate linearly and clamp at both ends.
 * n_entries in [2, 1024], all entries finite, extinction >= 0,
 * domain_hi > domain_lo. Every channel of a volume uses the same n_entries.
 * The device copy and the empty flags are refreshed in stream order by the
 * next commit or render. */
sg_status sg_set_transfer_function(sg_volume *vol, int32_t channel,
                                   const float *rgba, int32_t n_entries,
                                   double domain_lo, double domain_hi);

/* Render n_views views in one launch sequence on hip_stream (Sec 5.1-5.3):
 * per view an LOD cut (Sec 5.2), then per pixel a ray through the cut's
 * nodes front to back, trilinear samples every step_voxels * 2^L level-0
 * units inside the clipped ray interval, transfer-function lookup, the
 * optical model's accumulation (emission-absorption compositing with early
 * termination by default), background composited underneath
 * (C + (1 - A) bg, A + (1 - A) bg.a).
 *   views    : host array [n_views]
 *   out_rgba : host array [n_views] of device float pointers, each
 *              [height][width][4] premultiplied RGBA, row 0 = top
 *   out_depth: NULL, or host array [n_views] of device float pointers (or
 *              NULL entries), each [height][width]: distance along the ray
 *              of the first sample whose alpha >= depth_alpha, +inf if none
 *              (always +inf under the emission-only and maximum-intensity
 *              models, whose alpha stays 0)
 * Asynchronous: returns after enqueueing. Requires a transfer function for
 * every channel (SG_ERR_STATE otherwise). n_views in [1, 4096]. */
sg_status sg_render_views(sg_volume *vol, int32_t n_views, const sg_view *views,
                          const sg_render_params *params, float *const *out_rgba,
                          float *const *out_depth, void *hip_stream);

/* sg_render_views whose execution is decided on the device: enable is a
 * device int32 read by the render's kernels when they run (stream order);
 * nonzero renders exactly as sg_render_views, zero makes every kernel return
 * at once, so the outputs keep their contents (and a cache volume records no
 * requests or uses). For decisions taken by earlier device work without a
 * host round trip, such as the upsampler's fallback to the full-resolution
 * render (sg_up_forward_flag). enable must not be NULL
 * (SG_ERR_INVALID_ARG). */
sg_status sg_render_views_if(sg_volume *vol, int32_t n_views, const sg_view *views,
                             const sg_render_params *params, float *const *out_rgba,
                             float *const *out_depth, const int32_t *enable,
                             void *hip_stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): sg_render_views
 * with every piece of per-render scratch -- the view table, the persistent
 * grid's tile queues and the per-view cut maps -- in a static device array
 * of 4 MiB that each GPU the library runs on holds until the process ends.
 * The call makes no hipMalloc, hipFree or other allocating call; it enqueues
 * the same kernels as sg_render_views and renders the same image bit for
 * bit. Limits and requirements:
 *   - n_views in [1, 4];
 *   - n_views x (level-0 brick grid cells) x 4 bytes <= 4 MiB - 8 KiB (e.g.
 *     a 2048^3 volume in 64^3 bricks: 32^3 cells, 128 KiB per view);
 *     larger requests fail with SG_ERR_INVALID_ARG;
 *   - the volume must be committed (sg_volume_commit after uploads, pyramid
 *     builds or transfer-function changes), else SG_ERR_STATE;
 *   - kernel timing (sg_set_kernel_timing) does not record these renders.
 * Every call on one GPU uses that GPU's single scratch array, which keeps
 * the last call's contents (each call rewrites what it reads): calls whose
 * device work may overlap on one GPU -- on different streams without
 * ordering between them -- race, and must be serialised by the caller.
 * Other errors as sg_render_views. Asynchronous on hip_stream. */
sg_status sg_render_views_noalloc(sg_volume *vol, int32_t n_views, const sg_view *views,
                                  const sg_render_params *params, float *const *out_rgba,
                                  float *const *out_depth, void *hip_stream);

/* Sort-last compositing of one view's part images (Sec 5.1: the over
 * operator is associative, so renders of disjoint parts of the volume
 * combine): parts[k] is the premultiplied RGBA image (float4 per pixel,
 * row-major, view->width x view->height, device memory, 16-byte aligned) of
 * the render of box k alone, rendered on a zero background with the region
 * of interest set to that box; boxes holds 6 host doubles per part (lo x, y,
 * z, hi x, y, z; level-0 voxel units; the boxes must not overlap). Per
 * pixel the parts whose box the pixel's ray crosses are combined front over
 * back in the order the ray enters the boxes, C = sum_k (prod_{j<k} (1 -
 * A_j)) C_k and A likewise, into out_rgba (same layout; may not alias a
 * part). 1 <= n_parts <= 8. The ray of each pixel is the renderer's (same
 * FP64 arithmetic, lens included). Errors: SG_ERR_INVALID_ARG for NULL or
 * misaligned pointers, a bad view, n_parts out of range, non-finite or empty
 * boxes. Asynchronous on hip_stream; runs on the current device. */
sg_status sg_composite_over(const sg_view *view, int32_t n_parts,
                            const float *const *parts, const double *boxes,
                            float *out_rgba, void *hip_stream);

/* Same render with instrumentation (per-pixel sample counts, total samples,
 * distinct micro-blocks read). Synchronises hip_stream before returning so
 * that the host counters are valid. Slower; for tests and measurement. */
sg_status sg_render_views_stats(sg_volume *vol, int32_t n_views,
                                const sg_view *views,
                                const sg_render_params *params,
                                float *const *out_rgba, float *const *out_depth,
                                sg_render_stats *stats, void *hip_stream);

/* The LOD cut of one view (Sec 5.2) as computed on the device, for checking:
 * nodes receives the cut's node identifiers sorted ascending, each
 *   (level << 60) | (bx << 40) | (by << 20) | bz,
 * and empty[i] (if not NULL) the skip flag of nodes[i] at params->timepoint
 * for params->model (zero opacity, zero emission, or 0 for maximum
 * intensity, whose skips depend on the ray).
 * *n_nodes is the capacity on input and the cut size on output; if the cut
 * is larger nothing is written and SG_ERR_INVALID_ARG is returned with the
 * needed size in *n_nodes. Host buffers; synchronises hip_stream. */
sg_status sg_get_lod_cut(sg_volume *vol, const sg_view *view,
                         const sg_render_params *params, uint64_t *nodes,
                         int32_t *n_nodes, uint8_t *empty, void *hip_stream);

/* Instrumentation: while enabled, every render of vol records HIP events
 * on its stream around the cut-map kernel and around the ray-casting kernel.
 * sg_get_kernel_timing synchronises those events and returns the number of
 * renders recorded and the summed kernel milliseconds (cut map, ray cast)
 * since the last query or enable, then clears the record. */
sg_status sg_set_kernel_timing(sg_volume *vol, int32_t enable);
sg_status sg_get_kernel_timing(sg_volume *vol, int32_t *renders,
                               double *cutmap_ms, double *raycast_ms);

/* ---------------------------------------------------------------------
 * Launch configuration and autotuning (batched uneven views, Sec 5.3 per-eye
 * rendering at scale). A wave renders 8x8 pixels; the knobs below change
 * only how that work is laid out on the device, never a sample position, so
 * every configuration renders the same image bit for bit.
 */
typedef struct {
  int32_t kernel;      /* 0 = staged (brick regions copied to LDS per wave),
                          1 = gather (stencils read the brick pool)          */
  int32_t tile;        /* workgroup screen tile edge in pixels: 8, 16, 32
                          (1, 4 or 4 waves per workgroup; at 32 each wave
                          renders four 8x8 tiles in turn)                  */
  int32_t block;       /* edge in pixels of the screen blocks dealt to the
                          XCDs in turn: 32, 64 or 128, >= tile              */
  int32_t stage_bytes; /* LDS staging bytes per wave (staged): 1024..32768,
                          a multiple of 16                                 */
  int32_t persistent;  /* 1: one resident grid whose waves take 8x8 tiles
                          from per-XCD queues; 0: one workgroup per tile    */
} sg_launch_config;
/* Default: {0, 16, 64, 8192, 0}. NULL config restores the default.
 * Errors: SG_ERR_INVALID_ARG (out of range), SG_ERR_UNSUPPORTED (the tile's
 * LDS need exceeds 160 KiB). SG_GATHER in a render's flags overrides
 * `kernel` for that render. */
sg_status sg_set_launch_config(sg_volume *vol, const sg_launch_config *config);
sg_status sg_get_launch_config(const sg_volume *vol, sg_launch_config *config);
/* Time launch configurations on this render (coordinate descent over the
 * five fields, two sweeps, each candidate timed over `repeats` renders after
 * one warm-up render, with events on hip_stream) and keep the fastest as the
 * volume's configuration. out_rgba receives the renders. best and best_ms
 * (either may be NULL) receive the choice and its time per render.
 * Synchronises hip_stream. SG_GATHER must be clear (the kernel is tuned). */
sg_status sg_autotune(sg_volume *vol, int32_t n_views, const sg_view *views,
                      const sg_render_params *params, float *const *out_rgba,
                      int32_t repeats, sg_launch_config *best, double *best_ms,
                      void *hip_stream);

/* ---------------------------------------------------------------------
 * Render graphs: a render prepared once as a HIP graph (cut-map kernel,
 * queue reset when persistent, ray-casting kernel) and replayed per frame
 * without host-side preparation. The graph owns its view table, cut map
 * and queues; it keeps the volume's launch configuration, the params and
 * the output pointers given at creation. Between launches the views may be
 * re-posed (same sizes); transfer-function tables and brick contents may
 * change (they are read at replay), but a different table size or value
 * domain makes sg_render_graph_launch return SG_ERR_STATE. Launches of one
 * graph must not overlap (they share its scratch); the volume must outlive
 * the graph. */
typedef struct sg_render_graph sg_render_graph; /* opaque */
sg_status sg_render_graph_create(sg_volume *vol, int32_t n_views,
                                 const sg_view *views,
                                 const sg_render_params *params,
                                 float *const *out_rgba, float *const *out_depth,
                                 sg_render_graph **out);
/* New camera poses / lens / ray limits for the next launches (view sizes
 * must match creation). Stream-ordered on hip_stream. */
sg_status sg_render_graph_set_views(sg_render_graph *graph, const sg_view *views,
                                    void *hip_stream);
/* Commit pending volume work, then replay the graph on hip_stream. */
sg_status sg_render_graph_launch(sg_render_graph *graph, void *hip_stream);
/* Synchronises the device, then frees the graph and its scratch. */
sg_status sg_render_graph_destroy(sg_render_graph *graph);

/* ---------------------------------------------------------------------
 * Out-of-core mode (cache_slots > 0; Sec 4.2 GPU chunk cache, Sec 5.2
 * request queue and coarser fallback, Sec 5.4 time series). The pool holds
 * cache_slots bricks; which (channel, timepoint, node) are resident is the
 * caller's loading decision, driven by the requests renders make:
 *  - a render's LOD traversal descends from a block that does not suit into
 *    its children only when every existing child is resident for every
 *    channel at the render's timepoint; otherwise it renders the block one
 *    level coarser and requests the missing children;
 *  - every top-level node must be resident at the render's timepoint
 *    (SG_ERR_STATE otherwise);
 *  - each render stamps the slots of the nodes it uses with a frame number;
 *    when sg_cache_put needs a slot and none is free it evicts the slot with
 *    the oldest stamp (a min-heap over stamps), never a top-level node's;
 *  - sg_upload_bricks and sg_build_lod are not available (SG_ERR_UNSUPPORTED):
 *    bricks arrive whole, apron included, at every level;
 *  - render graphs are not available for such volumes.
 * All cache calls are ordered on hip_stream after earlier work (evicting a
 * slot an enqueued render still reads is safe only in stream order). */
/* Store n bricks of one (channel, timepoint, level): src holds n regions of
 * (brick+2)^3 voxels (x fastest), each the core [brick*b - 1, brick*b+brick]
 * per axis with indices clamped to the level (the one-voxel apron), from a
 * host pointer (copied before return) or a device pointer. coords: host
 * int32 [n][3]. Bricks already resident are overwritten in place. Errors:
 * SG_ERR_UNSUPPORTED (not a cache volume), SG_ERR_OUT_OF_MEMORY (n larger
 * than the slots that can be freed). */
sg_status sg_cache_put(sg_volume *vol, int32_t channel, int32_t timepoint,
                       int32_t level, int32_t n, const int32_t *coords,
                       const void *src, int32_t src_on_device, void *hip_stream);
/* As sg_cache_put, with brick i's region ((brick+2)^3 voxels, x fastest) at
 * srcs[i]: for a CPU-memory tier that keeps every chunk on its own (Sec 4.2:
 * a host cache beside the GPU cache). Each run of regions that lie back to
 * back in memory (srcs[i+1] = srcs[i] + region bytes) is copied by one DMA
 * into the library's staging buffer (the memory kind of every pointer is
 * looked up: page-locked host memory moves at the bus rate, pageable host
 * memory through the runtime's bounce buffers, device memory directly), then
 * all n are stored as by sg_cache_put. srcs: host array of n pointers, none
 * NULL; coords as in sg_cache_put. The regions are consumed before return.
 * Errors as sg_cache_put. */
sg_status sg_cache_put_scattered(sg_volume *vol, int32_t channel, int32_t timepoint,
                                 int32_t level, int32_t n, const int32_t *coords,
                                 const void *const *srcs, void *hip_stream);
/* Nodes requested by renders since the last call, then cleared: ids[i]
 * packed as in sg_get_lod_cut, timepoints[i] its timepoint (every channel
 * of it is wanted). *n is the capacity on input, the count on output
 * (nothing is written and SG_ERR_INVALID_ARG returned, with the count, if
 * too small). Host buffers; synchronises hip_stream. */
sg_status sg_cache_requests(sg_volume *vol, uint64_t *ids, int32_t *timepoints,
                            int32_t *n, void *hip_stream);
typedef struct {
  int64_t capacity;   /* pool slots                                         */
  int64_t resident;   /* slots holding a brick                              */
  int64_t uploads;    /* bricks stored by sg_cache_put                      */
  int64_t evictions;  /* bricks dropped to make room                        */
  int64_t frame;      /* renders so far (the stamp of the latest)           */
} sg_cache_info;
sg_status sg_cache_get_info(const sg_volume *vol, sg_cache_info *info);
/* Whether node (level, b) of (channel, timepoint) is resident: *resident =
 * 1 or 0. */
sg_status sg_cache_resident(const sg_volume *vol, int32_t channel, int32_t timepoint,
                            int32_t level, const int32_t b[3], int32_t *resident);

/* ---------------------------------------------------------------------
 * Import of an out-of-core volume (Sec 4.1: chunks of the volume made once
 * at several resolutions; Sec 4.2: chunks move whole between the CPU and GPU
 * caches). These work on plain device arrays of voxels of type dtype
 * (SG_U8 or SG_U16), x fastest (indexed [z][y][x]), need no volume and run
 * on the current device, asynchronously on hip_stream. */
/* One coarser level of the resolution pyramid (Sec 5.2): src has src_dims
 * voxels (each in [1, 2^20]); dst receives ceil(src_dims / 2) voxels, voxel
 * g = (sum of the 2x2x2 children 2g + delta, each child index clamped to
 * src_dims - 1, + 4) >> 3 -- the rule sg_build_lod applies to a resident
 * volume. src and dst are caller-owned device buffers and must not overlap.
 * Errors: SG_ERR_INVALID_ARG (NULL pointer, bad dtype or dims, overlap),
 * SG_ERR_DEVICE. */
sg_status sg_pyramid_level(int32_t dtype, const int32_t src_dims[3], const void *src,
                           void *dst, void *hip_stream);
/* Whole bricks of one level in the form sg_cache_put takes: out receives n
 * regions of (brick+2)^3 voxels, x fastest; region i holds the level's
 * voxels brick*b_i - 1 .. brick*b_i + brick per axis with indices clamped
 * to [0, dims - 1] (the core and its one-voxel apron).
 *   dims  : host int32 [3], the level's voxels per axis, each in [1, 2^20]
 *   level : device array of the level
 *   brick : core edge, a power of two in [2, 256]
 *   coords: host int32 [n][3] brick indices (bx, by, bz), each inside the
 *           level's brick grid ceil(dims / brick); consumed before return
 *   out   : device buffer of n (brick+2)^3 voxels, caller-owned
 * n = 0 does nothing. Errors: SG_ERR_INVALID_ARG (NULL pointer, bad dtype,
 * dims or brick, n < 0, a coordinate outside the grid),
 * SG_ERR_OUT_OF_MEMORY / SG_ERR_DEVICE (staging of the coordinates). */
sg_status sg_brick_regions(int32_t dtype, const int32_t dims[3], const void *level,
                           int32_t brick, int32_t n, const int32_t *coords, void *out,
                           void *hip_stream);

/* Bytes of device memory the volume holds (pool, tables, scratch). */
sg_status sg_volume_memory(const sg_volume *vol, uint64_t *bytes);

const char *sg_status_string(sg_status s); /* static string, never NULL */
const char *sg_last_error(void);           /* thread-local, never NULL  */
int32_t sg_abi_version(void);              /* SG_ABI_VERSION            */

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
