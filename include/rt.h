/*
 * rt.h -- C ABI of the MI355X (gfx950) direct-volume-rendering raycaster.
 *
 * The library renders a scalar volume on a Cartesian grid (arXiv:1211.5595,
 * Section 2.1) by image-order ray casting (Section 4.1): one viewing ray per
 * pixel, intersected with the volume, sampled at evenly spaced points,
 * classified by a colour+opacity transfer function (Sections 2.6 and 6) and
 * combined by a ray function -- compositing as in Section 4.2, eqs. (1)-(5),
 * or one of the other ray functions listed in Section 4.1.
 *
 * Conventions shared by every entry point
 *   - Volume: node-centred grid, node (i,j,k) at (i*sx, j*sy, k*sz) mm;
 *     source arrays are C-order [z][y][x] (x fastest); dims = {nx, ny, nz},
 *     each >= 2.  The volume is the closed box [0,(n-1)s] per axis.
 *   - Sampling: dt = step_vox * min(spacing) mm along a unit ray; samples at
 *     the midpoints of the dt-segments of the clipped chord, plus one at the
 *     midpoint of the remaining partial segment (length r) whose opacity is
 *     1-(1-a)^(r/dt).  Trilinear interpolation with clamp-to-edge.
 *   - Classification: post-classification; x = clamp((v-vmin)/(vmax-vmin),
 *     0, 1)*(K-1), linear interpolation between table entries floor(x) and
 *     floor(x)+1.  Table colours are non-premultiplied.
 *   - Compositing: front-to-back, C += T*a*c, T *= 1-a; stop after the first
 *     sample with 1-T >= alpha_cutoff (early ray termination).  Output pixel
 *     = (C + T*bg.rgb, (1-T) + T*bg.a), premultiplied, float32 RGBA.
 *   - Image: H x W x 4 float32, row-major, row 0 at the top; pixel (i,j) is
 *     sampled at its centre; aspect ratio W/H.
 *   - Arithmetic: float32 (float-float pairs for ray set-up and fixed-point
 *     sample positions); no float64 on the device.
 *
 * Memory ownership
 *   The caller allocates and owns every device buffer (volume storage,
 *   transfer-function storage, images, workspaces) and keeps it alive until
 *   the handle using it is destroyed and all work queued on it has finished.
 *   Handles (rt_volume, rt_tf, rt_batch_plan) are small host objects owned by
 *   the library; destroy them with the matching rt_destroy_* call.
 *
 * Streams
 *   Every call that touches the device is ordered on the caller's stream
 *   (a hipStream_t passed as void*; NULL = the null stream).  No call
 *   synchronises the device unless its comment says so.
 *
 * Errors
 *   Every function returns an rt_status and never aborts.  rt_last_error()
 *   returns a thread-local message for the last failing call on the calling
 *   thread.  Launch failures are reported synchronously as RT_ERR_DEVICE; an
 *   asynchronous device fault surfaces at the caller's next synchronisation.
 */
#ifndef RTVOL_RT_H
#define RTVOL_RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RT_OK = 0,
    RT_ERR_INVALID_ARG = 1,   /* null pointer, bad size, bad camera, ... */
    RT_ERR_OUT_OF_MEMORY = 2, /* a caller-provided buffer is too small */
    RT_ERR_DEVICE = 3,        /* a HIP runtime call failed */
    RT_ERR_UNSUPPORTED = 4    /* valid request outside what the library supports */
} rt_status;

/* Storage (and source) element types of a volume. */
typedef enum {
    RT_U8 = 0,              /* unsigned 8-bit integers, converted exactly */
    RT_U16 = 1,             /* unsigned 16-bit integers, converted exactly */
    RT_F16 = 2,             /* IEEE half; conversion from other types rounds to nearest even */
    RT_F32 = 3,             /* IEEE single */
    RT_U8_BRICKSCALED = 4,  /* storage only: 8-bit codes with a (lo, scale) per brick of B^3 cells */
    RT_U15 = 5,             /* storage only, RT_LAYOUT_CELLS only, from RT_U8/RT_U16 sources: integers
                             * 0..32767 (larger values are clamped to 32767, so 15-bit data such as
                             * 12-bit MRI is converted exactly); each cell keeps its x-neighbour corner
                             * pairs as (c0, c1 - c0), which saves one conversion per pair in the marcher.
                             * Images are bit-identical to RT_U16 for the same (unclamped) data. */
    RT_U12 = 6              /* storage only, RT_LAYOUT_CELLS only, from RT_U8/RT_U16 sources: integers
                             * 0..4096 (larger values are clamped to 4096, so 12-bit data is converted
                             * exactly), each stored as the IEEE half of (value - 2048), which is exact
                             * on that range.  The marcher interpolates the halves with mixed-precision
                             * fused multiply-adds and no conversions; all arithmetic is binary32.
                             * Images match RT_U16 to within binary32 rounding (not bit for bit: the
                             * interpolation runs on values shifted by 2048). */
} rt_dtype;

/* Device layouts of a volume.  All of them add a one-node replicated border
 * on every face so that clamp-to-edge holds without per-sample clamping. */
typedef enum {
    RT_LAYOUT_CELLS = 0,  /* every cell's 8 corners contiguous, cells in 2x2x2 blocks; any storage type
                           * (the only layout of RT_U15 and RT_U12).
                           * 8 values per cell (8x the grid); for RT_U8_BRICKSCALED the codes of a
                           * cell use its owning brick's (lo, scale), kept once per 2x2x2 block */
    RT_LAYOUT_LINEAR = 1, /* RT_U8/RT_U16/RT_F16/RT_F32: the bordered grid in C order (1x the grid) */
    RT_LAYOUT_BRICKS = 2, /* RT_U8_BRICKSCALED: per brick the codes of local nodes -1..B+1 ((B+3)^3) */
    RT_LAYOUT_POLY = 3,   /* RT_U8/RT_U16: every cell stores the 8 coefficients of its trilinear polynomial
                           * as binary32 (exact for integer data), cells in 2x2x2 blocks (32 B per cell);
                           * a sample then costs 7 fused multiply-adds */
    RT_LAYOUT_QUADS = 4   /* RT_U16/RT_U12: quad bricks.  A quad is the 2x2 nodes of a padded cell column at one
                           * padded layer (8 bytes); a brick holds 2x2 columns by 4 layers (128 bytes, 3 cells
                           * deep, consecutive bricks in z sharing a layer), so a sample's cell is the quads of
                           * its two layers, one 16-byte load, in the cell layout's word order: images equal
                           * those of RT_LAYOUT_CELLS of the same storage type bit for bit, in 2/3 of the
                           * memory (5.3 bytes of storage per 16-bit value against 8).  At most 65533 slices,
                           * 2^20 bricks per z-brick slice, 2 GiB in all. */
} rt_layout;

/* Ray functions (Section 4.1 list; Section 2.4 for maximum intensity and
 * X-ray projection).  The three projections visit every sample of the ray's
 * lattice (weight 1, and r/dt for the partial last segment; no early
 * termination), reduce the interpolated values to one scalar, classify it
 * once and lay it over the background with the table's opacity a:
 * out.rgb = a*rgb + (1-a)*bg.rgb, out.a = a + (1-a)*bg.a (bg when the ray
 * misses).  The maximum takes the partial sample whatever its weight. */
typedef enum {
    RT_COMPOSITE = 0,  /* emission-absorption compositing, Section 4.2 */
    RT_MIP = 1,        /* maximum interpolated value along the ray */
    RT_XRAY = 2,       /* dt times the weighted sum of the values (the chord's line integral) */
    RT_AVERAGE = 3,    /* weighted mean of the values */
    RT_ISO = 4,        /* first crossing of an iso-value, shaded (below) */
    RT_THRESHOLD = 5   /* compositing of the samples inside a value window (below) */
} rt_ray_function;
/* RT_THRESHOLD composites as RT_COMPOSITE with every sample whose
 * interpolated value lies outside [iso_value, iso_high] transparent (it still
 * counts as a processed sample); needs finite iso_value <= iso_high.
 * RT_ISO: the first lattice sample whose value reaches iso_value is the hit;
 * the hit point is refined by linear interpolation from the sample before it
 * (unless it is the ray's first sample); the normal n is the descent direction
 * of the trilinear field from central differences over +-1/2 cell per axis
 * (scaled by the spacing); the pixel is opaque, rgb = c * (0.2 + 0.8 |n.d|)
 * with c the table colour at iso_value and d the ray direction (a headlight),
 * alpha = 1; a ray that never reaches iso_value shows the background.  The
 * sample count of a hit is the hit sample's index + 1.  Empty-space skipping
 * applies to compositing and thresholding only. */

/* Look-at camera (Section 6: camera settings).  w = normalize(center-eye),
 * u = normalize(w x up), v = u x w.  Invalid when eye == center or up is
 * parallel to w.  perspective != 0: pinhole at eye with full vertical field
 * of view fovy_deg in (0, 180).  perspective == 0: parallel rays along w
 * through a window of half-height ortho_half_height (> 0) mm centred on eye. */
typedef struct {
    double eye[3], center[3], up[3];
    int perspective;
    double fovy_deg;
    double ortho_half_height;
} rt_camera;

typedef struct rt_volume rt_volume;
typedef struct rt_tf rt_tf;
typedef struct rt_batch_plan rt_batch_plan;

/* Optional per-render settings; a NULL pointer or zeroed struct selects the
 * defaults. */
typedef struct {
    unsigned long long* sample_counter; /* device, nullable: atomically += samples processed */
    int32_t* pixel_counts;              /* device, nullable: H*W samples processed per pixel */
    int ray_function;                   /* rt_ray_function; 0 = compositing */
    float iso_value;                    /* RT_ISO iso-value; RT_THRESHOLD window low */
    float iso_high;                     /* RT_THRESHOLD window high */
    int tile_w, tile_h;                 /* ray tile of one wavefront, tile_w*tile_h == 64; 0 = 8x8 */
    int waves_per_block;                /* wavefronts per workgroup, 1..16; 0 = default: 16 for
                                         * batches; for rt_render the most (up to 16) that still
                                         * give every compute unit a workgroup */
    int skip_empty;                     /* compositing: nonzero leaps over empty space (see below) */
    int tile_order;                     /* 1: a workgroup renders a compact block of tiles (cache
                                         * locality across the rays of a block: the better order when
                                         * many views share the GPU); 2: its wavefronts take tiles
                                         * spread over the view (tile = block + blocks * wavefront), so
                                         * the long rays of the middle of an image share a SIMD with
                                         * short ones (lower latency when one view has the GPU to
                                         * itself); 0: 2 for rt_render, 1 for batches and plans.
                                         * Images are identical in every order. */
    double opacity_unit_distance;       /* > 0 (mm): the table's opacities are per this distance
                                         * and are corrected to the sample spacing,
                                         * a' = 1 - (1 - a)^(dt / unit), entry by entry when the
                                         * table is staged (compositing and thresholding; the
                                         * paper's compositing, Section 4.2, uses the table opacity
                                         * per sample, which is the default 0) */
    int batch_form;                     /* batch plans: 0 = by size: a batch of at most
                                         * rt_batch_latency_pixels() pixels takes the latency form
                                         * (one workgroup per block of tiles, workgroups sized to the
                                         * batch as rt_render sizes them to a view, the single-view
                                         * kernel's occupancy), a larger one the persistent form;
                                         * 1 = always persistent; 2 = always the latency form.
                                         * Images are identical in either form. */
} rt_render_opts;

/* Empty-space skipping (compositing only).  Each volume keeps, per skip brick
 * of 8^3 cells (larger for very large volumes, so that a volume has at most
 * 65536 of them), the range of values its samples can take; each transfer
 * function keeps a running count of its entries with nonzero opacity.  A
 * brick whose range (widened by a few units in the last place, and by one
 * table entry each side) touches only zero-opacity entries is empty: its
 * samples leave the accumulated colour and transmittance unchanged, bit for
 * bit.  With skip_empty set, a wavefront whose live rays all sit in empty
 * bricks advances every ray to the last sample it has in its brick in one
 * step.  Images and per-pixel sample counts (skipped samples included) are
 * identical to rendering without it. */

/* ---------------------------------------------------------------------------
 * Volume data (Section 2.1: samples f(x,y,z,d) on a Cartesian grid; slices
 * with thickness and gaps, Section 1, give an anisotropic spacing).
 * ------------------------------------------------------------------------- */

/* Device bytes needed to hold a volume of `dims` with element type `storage`
 * in `layout`, followed by the value ranges of its empty-space skip bricks
 * (8 bytes per brick, 256-byte aligned).  brick is the brick edge B in cells (8, 16 or 32) for
 * RT_U8_BRICKSCALED and must be 0 otherwise.  Errors: RT_ERR_INVALID_ARG
 * (bad dims, layout or brick, NULL), RT_ERR_UNSUPPORTED (volume too large for
 * 32-bit addressing: 4 GiB of storage). */
rt_status rt_volume_bytes(const int64_t dims[3], int storage, int layout, int brick, size_t* bytes);

/* Convert a device-resident source array (C-order [z][y][x] of src_dtype,
 * one of RT_U8/RT_U16/RT_F16/RT_F32) into element type `storage` and
 * `layout` (rt_layout) in the caller's device buffer dev_buf
 * (>= rt_volume_bytes bytes, 256-byte aligned), on `stream`.  For
 * RT_U8_BRICKSCALED each brick of brick^3 cells gets lo = minimum and
 * scale = (maximum-lo)/255 over its nodes (high halo included) and every
 * node the code rint((v-lo)/scale), all binary32; a sample is decoded with
 * the brick that owns its cell.  The source may be freed once the stream has
 * passed this call.  *out receives the handle.
 * Errors: RT_ERR_INVALID_ARG (NULL, dims < 2, non-finite or non-positive
 * spacing, storage/src combination such as F32 -> U8), RT_ERR_OUT_OF_MEMORY
 * (dev_buf_bytes too small), RT_ERR_DEVICE (launch failure). */
rt_status rt_create_volume(const void* src_dev, int src_dtype, const int64_t dims[3], const double spacing[3],
                           int storage, int layout, int brick, void* dev_buf, size_t dev_buf_bytes, void* stream,
                           rt_volume** out);
rt_status rt_destroy_volume(rt_volume* vol);

/* ---------------------------------------------------------------------------
 * Transfer function (Sections 2.6 and 6: colour and scalar-opacity transfer
 * functions), held as one K x 4 RGBA table over the value window
 * [vmin, vmax].
 * ------------------------------------------------------------------------- */

/* Device bytes for a K-entry table (K in [2, 4096]): the K x 4 float table
 * (256-byte aligned) and K+2 int32 running counts of its nonzero-opacity
 * entries, used by empty-space skipping. */
rt_status rt_tf_bytes(int K, size_t* bytes);

/* Create (*tf == NULL) or update in place (*tf != NULL) a transfer function:
 * the host table rgba[K][4] (each value in [0,1]) is copied into a pinned,
 * coherent buffer owned by the handle, which a small kernel on `stream` reads
 * into dev_buf (>= rt_tf_bytes(K), 16-byte aligned; no runtime memory copy is
 * made); the call does not wait for the upload, and
 * the caller's table may be reused as soon as it returns.  An update keeps
 * dev_buf (pass NULL or the same buffer) and may change K while
 * rt_tf_bytes(K) still fits dev_buf and the handle's pinned buffer (sized by
 * the K it was created with), so a handle created with 4096 entries takes any
 * table without allocating; it waits only for this handle's previous upload,
 * and renders that read the table must be ordered after it (same stream, or
 * an event).
 * Errors: RT_ERR_INVALID_ARG (NULL, K outside [2,4096], vmax <= vmin,
 * non-finite or out-of-range entries, changed buffer),
 * RT_ERR_OUT_OF_MEMORY (buffer too small), RT_ERR_DEVICE. */
rt_status rt_set_transfer_function(rt_tf** tf, const float* rgba, int K, double vmin, double vmax, void* dev_buf,
                                   size_t dev_buf_bytes, void* stream);
rt_status rt_destroy_tf(rt_tf* tf);

/* ---------------------------------------------------------------------------
 * Rendering (Section 4.1: ray path, values along the ray, ray function).
 * ------------------------------------------------------------------------- */

/* Render one image of `volume` into out_dev (H*W*4 float32, device).  dims
 * must equal the volume's dims; spacing (> 0) may differ from the one given
 * at creation (geometry only).  step_vox > 0 in units of the finest spacing;
 * alpha_cutoff in (0, 1] (1 = stop only at full opacity).  bg_rgba may be
 * NULL (transparent black).  One kernel launch on `stream`.
 * Errors: RT_ERR_INVALID_ARG (NULL, size/camera/step/cutoff out of range,
 * dims mismatch, unknown ray function, invalid threshold window or
 * iso-value), RT_ERR_UNSUPPORTED (tile shape not built),
 * RT_ERR_DEVICE (launch failure). */
rt_status rt_render(const rt_volume* volume, const int64_t dims[3], const double spacing[3], const rt_tf* tf,
                    const rt_camera* camera, int width, int height, double step_vox, double alpha_cutoff,
                    const float bg_rgba[4], float* out_dev, const rt_render_opts* opts, void* stream);

/* One view of a batch. */
typedef struct {
    const rt_volume* volume;
    const rt_tf* tf;
    rt_camera camera;
    int width, height;
    double step_vox, alpha_cutoff;
    float bg_rgba[4];
    float* out_dev;           /* H*W*4 float32, device */
    int32_t* pixel_counts;    /* device, nullable */
    int ray_function;         /* rt_ray_function of this view; 0 = compositing */
    float iso_value, iso_high;
    int skip_empty;           /* compositing: leap over empty space (as rt_render_opts.skip_empty) */
    double opacity_unit_distance; /* as rt_render_opts.opacity_unit_distance (0 = none) */
} rt_render_job;

/* Workspace bytes for batches of up to max_jobs views (max_jobs >= 1). */
rt_status rt_batch_workspace_bytes(int max_jobs, size_t* bytes);

/* Render n views (of possibly different volumes, transfer functions, ray
 * functions and sizes; all volumes of one storage type and layout; each job
 * selects its own ray function, the ray-function fields of opts are not used)
 * in one persistent launch that pulls
 * ray tiles from a device work queue.  Writes the job table into `workspace`
 * (>= rt_batch_workspace_bytes(n)) on `stream` through the arguments of small
 * fill kernels (no runtime memory copy); the job array may be reused
 * once the call returns.  A workspace holds one batch at a time: batches that
 * may run at once (on different streams) need workspaces of their own.  Results are bitwise identical to rt_render of each
 * view.  Errors: as rt_render, plus RT_ERR_OUT_OF_MEMORY (workspace too
 * small) and RT_ERR_UNSUPPORTED (mixed storage types or layouts). */
rt_status rt_render_batch(const rt_render_job* jobs, int n, void* workspace, size_t ws_bytes,
                          unsigned long long* sample_counter, const rt_render_opts* opts, void* stream);

/* A batch plan: the persistent launch captured once into a HIP graph over a
 * fixed workspace, replayed for every batch of up to max_jobs views of one
 * storage type and layout.  rt_batch_plan_launch writes the job table into the
 * workspace through the arguments of small fill kernels on `stream` (outside the
 * graph; no runtime memory copy) and launches the graph on `stream` -- or, for
 * a batch small enough for the latency form (opts->batch_form), launches that
 * form's kernel directly, its grid the batch's block count (up to 6 views with
 * the job table in its own arguments).  Calls on one plan must not run
 * concurrently.  A plan created with opts->skip_empty set skips empty space
 * for the jobs whose skip_empty is set; a plan created without it never skips
 * (the images are the same either way). */
rt_status rt_batch_plan_create(int max_jobs, int storage, int layout, void* workspace, size_t ws_bytes,
                               const rt_render_opts* opts, rt_batch_plan** out);
/* Pixels (summed over a batch's views) up to which a plan with batch_form 0
 * takes the latency form on the current device. */
long long rt_batch_latency_pixels(void);
rt_status rt_batch_plan_launch(rt_batch_plan* plan, const rt_render_job* jobs, int n,
                               unsigned long long* sample_counter, void* stream);
rt_status rt_batch_plan_destroy(rt_batch_plan* plan);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid device allocation): rt_render_batch
 * with its workspace in a device array inside the library instead of a
 * caller buffer.  Takes at most 64 jobs (RT_ERR_UNSUPPORTED above that,
 * before any device work); otherwise arguments, errors and results are those
 * of rt_render_batch, images bitwise identical.  The header, block prefix and
 * job table are delivered to the array by small kernels whose arguments carry
 * them (about 52 KB of device memory per GPU, held until the process ends),
 * so the call makes no device or pinned-host allocation and no copy from
 * pageable memory.  The array of the current device is used; `stream` must
 * belong to it.  Every call on one GPU shares that array: calls that may
 * overlap on one GPU (other threads, other streams) race and must be ordered
 * by the caller. */
rt_status rt_render_batch_noalloc(const rt_render_job* jobs, int n, unsigned long long* sample_counter,
                                  const rt_render_opts* opts, void* stream);

/* ---------------------------------------------------------------------------
 * Diagnostics
 * ------------------------------------------------------------------------- */
const char* rt_status_string(rt_status status);
const char* rt_last_error(void);
/* Library version string (static). */
const char* rt_version(void);

#ifdef __cplusplus
}
#endif
#endif
