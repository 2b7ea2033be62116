/*
 * rt_serve.h -- serving runtime of the raycaster (C ABI).
 *
 * Render requests against resident volumes (rt.h) are admitted by a device
 * memory budget and batched as they arrive -- continuous batching: whenever
 * one of the server's streams is free, every queued request whose image fits
 * the free part of the image pool (first come, first served: the head of the
 * queue waits for memory rather than being overtaken) goes into one launch of
 * that stream's captured batch plan, so requests that arrive while others
 * render are started as soon as a stream and memory free up and their work
 * overlaps on the device.  A batch also closes before its images would
 * exceed 16 x rt_batch_latency_pixels() pixels in all (one request at least),
 * so a burst of arrivals is split over the streams rather than finishing as
 * one long launch; batches up to rt_batch_latency_pixels() take the plans'
 * latency form.  A server thread inside the library uploads the
 * requests' transfer functions, launches, and retires finished batches;
 * callers only submit, wait and release.  Every image is bitwise the image
 * rt_render gives for the same request alone (the batched launch renders each
 * view exactly as a single launch does).
 *
 * This is not a method of the paper (which renders one view at a time for an
 * interactive user); it is the request loop of a rendering service built on
 * the same ray caster.
 *
 * Memory: the caller allocates one device arena (rt_server_arena_bytes) that
 * holds, per stream, the batch workspace and max_batch transfer-function
 * slots of 4096 entries, followed by the image pool.  The
 * image pool is the admission budget: a request holds W*H*16 bytes of it
 * (rounded up to 256) from admission until the caller releases it.  Host
 * memory: a pinned, coherent staging buffer per table slot, and a host copy of
 * each stream's job table.  The request path makes no runtime memory copy:
 * tables and job tables reach the device through small kernels.
 *
 * Threads: every entry point may be called from any thread.  Volumes must stay
 * alive until the requests that use them are released.  A request submitted
 * to an empty queue while a stream is free is launched by rt_server_submit in
 * the caller's thread (saving the server thread's wake-up); every other
 * request is launched by the server thread.
 */
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "rt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_server rt_server;

/* One render request.  The table is copied by rt_server_submit; the request
 * struct and the table may be reused as soon as the call returns. */
typedef struct {
    const rt_volume* volume;   /* resident, of the server's storage type and layout */
    const float* tf_rgba;      /* host table, tf_entries x 4 floats in [0, 1] */
    int tf_entries;            /* K in [2, 4096] */
    double tf_vmin, tf_vmax;   /* value window of the table (vmin < vmax) */
    rt_camera camera;
    int width, height;         /* image size, each in [1, 32768] */
    double step_vox, alpha_cutoff;
    float bg_rgba[4];
    int ray_function;          /* rt_ray_function */
    float iso_value, iso_high; /* as in rt_render_opts */
    double opacity_unit_distance; /* as in rt_render_opts (0 = none) */
} rt_request;

enum {
    RT_REQ_QUEUED = 0,  /* waiting for a stream or for image memory */
    RT_REQ_RUNNING = 1, /* in a launched batch */
    RT_REQ_DONE = 2,    /* image ready in the pool until released */
    RT_REQ_FAILED = 3   /* status says why; nothing to read */
};

typedef struct {
    int state;                          /* RT_REQ_* */
    rt_status status;                   /* RT_OK, or the failure of the request's batch */
    float* image_dev;                   /* DONE: H x W x 4 float32 in the image pool, else NULL */
    double t_submit, t_launch, t_done;  /* CLOCK_MONOTONIC seconds, 0 until reached: queued, taken from
                                         * the queue into a batch (in queue order), seen complete */
    int batch_size;                     /* requests in the launch that rendered it */
} rt_request_info;

typedef struct {
    unsigned long long submitted, completed, failed, batches;
    size_t pool_bytes, pool_in_use, pool_peak; /* image pool: size, held now, most ever held */
    int queued, running;
} rt_server_stats;

/* Arena bytes for n_streams in [1, 8] streams, batches of max_batch in
 * [1, 256] requests and an image pool of image_pool_bytes (>= 256). */
rt_status rt_server_arena_bytes(int n_streams, int max_batch, size_t image_pool_bytes, size_t* bytes);

/* Create a server for volumes of one storage type and layout on the current
 * device.  opts selects the launch shape, tile order, batch form and
 * empty-space skipping of the batch plans; opts->sample_counter, when not
 * NULL, is a device counter every batch atomically adds its composited samples
 * to (no copy back: read it on the device or after the server is idle); the
 * pixel-count and ray-function fields are not used (each request carries its
 * own ray function).  arena_dev is
 * 256-byte aligned device memory of at least rt_server_arena_bytes(...) bytes,
 * owned by the caller and kept until rt_server_destroy returns.  Starts the
 * server thread.  Errors: RT_ERR_INVALID_ARG (sizes, storage/layout, opts,
 * alignment), RT_ERR_OUT_OF_MEMORY (arena too small), RT_ERR_DEVICE. */
rt_status rt_server_create(int n_streams, int max_batch, int storage, int layout, const rt_render_opts* opts,
                           void* arena_dev, size_t arena_bytes, size_t image_pool_bytes, rt_server** out);

/* Queue one request; *ticket identifies it until released.  The request is
 * checked as rt_render would check it (no device work).  Errors:
 * RT_ERR_INVALID_ARG (NULL, invalid request, volume of another storage type or
 * layout, server shutting down), RT_ERR_OUT_OF_MEMORY (the image is larger
 * than the whole pool). */
rt_status rt_server_submit(rt_server* server, const rt_request* req, uint64_t* ticket);

/* Wait until the request is DONE or FAILED, or timeout_s seconds have passed
 * (timeout_s < 0: no limit; 0: just look), and fill *info with its state.
 * Errors: RT_ERR_INVALID_ARG (NULL, unknown or released ticket). */
rt_status rt_server_wait(rt_server* server, uint64_t ticket, double timeout_s, rt_request_info* info);

/* Give back a DONE or FAILED request: its image memory returns to the pool
 * (the image must not be read afterwards) and the ticket becomes unknown.
 * Errors: RT_ERR_INVALID_ARG (NULL, unknown ticket, request still queued or
 * running). */
rt_status rt_server_release(rt_server* server, uint64_t ticket);

rt_status rt_server_get_stats(rt_server* server, rt_server_stats* stats);

/* Finish every queued and running request (a queued request that can never
 * be admitted because unreleased images hold the pool fails with
 * RT_ERR_OUT_OF_MEMORY), stop the server thread and free the server's streams,
 * plans, table handles and host buffers.  Images of unreleased requests stay
 * in the caller's arena.  No other call on the server may run concurrently
 * with this one or follow it. */
rt_status rt_server_destroy(rt_server* server);

#ifdef __cplusplus
}
#endif
