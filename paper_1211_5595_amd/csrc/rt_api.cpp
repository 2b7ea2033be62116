// rt_api.cpp -- host runtime behind include/rt.h: argument validation,
// handle lifetime, view set-up in binary64 (rounded to float-float for the
// device), launches on the caller's stream, batch plans captured in HIP
// graphs.  See rt.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rt.h"
#include "rt_internal.h"

using namespace rtv;

struct rt_volume {
    VolDev dev;
    int64_t dims[3];
    double spacing[3];
    int storage;
    int brick;
};

struct rt_tf {
    const float4* dev;
    int K;
    double vmin, vmax;
    size_t bytes;
    void* staging;      // pinned, coherent host copy of the table for the asynchronous upload
    const void* staging_dev;  // its device-side address
    size_t staging_bytes;
    hipEvent_t copied;  // recorded after the upload on the caller's stream
    bool pending;
};

struct rt_batch_plan {
    int max_jobs;
    int kind;
    int form;       // rt_render_opts.batch_form
    bool skip;      // opts->skip_empty at creation
    LaunchShape ls;
    LaunchShape ls_lat;  // the latency form's tile and order (waves set per batch)
    int grid;
    void* ws;
    size_t ws_bytes;
    hipGraph_t graph;
    hipGraphExec_t exec;
    void* staging;  // host copy of header + prefix + job table, in the workspace's layout
    size_t staging_bytes;
};

namespace {

thread_local std::string g_last_error;

rt_status fail(rt_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

rt_status hip_fail(hipError_t e, const char* what) {
    return fail(RT_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool finite3(const double a[3]) { return std::isfinite(a[0]) && std::isfinite(a[1]) && std::isfinite(a[2]); }

int elem_bytes(int kind) {
    switch (kind) {
        case ST_U8: return 1;
        case ST_U16: return 2;
        case ST_F16: return 2;
        case ST_F32: return 4;
        case ST_U15: return 2;
        case ST_U12: return 2;
        default: return 0;
    }
}

// Which layouts a storage type can be held in.
bool layout_allowed(int storage, int layout) {
    switch (storage) {
        case RT_U8: return layout == RT_LAYOUT_CELLS || layout == RT_LAYOUT_LINEAR || layout == RT_LAYOUT_POLY;
        case RT_U16:
            return layout == RT_LAYOUT_CELLS || layout == RT_LAYOUT_LINEAR || layout == RT_LAYOUT_POLY ||
                   layout == RT_LAYOUT_QUADS;
        case RT_F16:
        case RT_F32: return layout == RT_LAYOUT_CELLS || layout == RT_LAYOUT_LINEAR;
        case RT_U8_BRICKSCALED: return layout == RT_LAYOUT_CELLS || layout == RT_LAYOUT_BRICKS;
        case RT_U15: return layout == RT_LAYOUT_CELLS;
        case RT_U12: return layout == RT_LAYOUT_CELLS || layout == RT_LAYOUT_QUADS;
        default: return false;
    }
}

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

// Transfer-function buffer: the K x 4 table, then (256-aligned) K+2 running
// counts nz[j] of the entries i < j with nonzero opacity over the table
// extended by a copy of its last entry (the lookup reads entries j0, j0+1).
size_t tf_nz_offset(int K) { return round256((size_t)K * 16); }
size_t tf_layout_bytes(int K) { return tf_nz_offset(K) + round256((size_t)(K + 2) * 4); }

struct Layout {
    size_t total;             // bytes
    size_t data_offset;       // start of the grid / cells / codes
    size_t data_bytes;
    size_t par_bytes;         // U8B cells: per-block (lo, scale)
    size_t brick_par_offset;  // U8B cells: per-brick (lo, scale) used while encoding
    uint32_t sy, sz, brick_bytes;
    int32_t nb[3];            // cell blocks (CELLS) or bricks (BRICKS) per axis
    int32_t brick_nb[3];      // U8B cells: bricks per axis
    int32_t bshift;
    int32_t layout;
    size_t ess_offset;        // skip-brick value ranges (float2 each), after everything else
    int32_t enb[3];
    int32_t eshift;
    size_t sup_offset;        // super-brick ranges, after the skip-brick ranges
    int32_t snb[3];
};

rt_status compute_data_layout(const int64_t dims[3], int storage, int layout, int brick, Layout& L);

// Skip bricks: 2^eshift padded cells per axis (cells 0..n), the smallest
// power of two from 8 up that keeps the count within kMaxSkipBricks.
rt_status compute_layout(const int64_t dims[3], int storage, int layout, int brick, Layout& L) {
    rt_status st = compute_data_layout(dims, storage, layout, brick, L);
    if (st != RT_OK) return st;
    for (L.eshift = 3;; ++L.eshift) {
        size_t nbt = 1;
        for (int a = 0; a < 3; ++a) {
            L.enb[a] = (int32_t)(((size_t)dims[a] + 1 + ((size_t)1 << L.eshift) - 1) >> L.eshift);
            nbt *= (size_t)L.enb[a];
        }
        if (nbt <= (size_t)kMaxSkipBricks) {
            L.ess_offset = L.total;
            L.sup_offset = round256(L.ess_offset + nbt * sizeof(float2));
            size_t nst = 1;
            for (int a = 0; a < 3; ++a) {
                L.snb[a] = (L.enb[a] + 3) / 4;
                nst *= (size_t)L.snb[a];
            }
            L.total = round256(L.sup_offset + nst * sizeof(float2));
            return RT_OK;
        }
    }
}

rt_status compute_data_layout(const int64_t dims[3], int storage, int layout, int brick, Layout& L) {
    if (!dims) return fail(RT_ERR_INVALID_ARG, "dims is NULL");
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 2 || dims[a] > (1 << 20)) return fail(RT_ERR_INVALID_ARG, "each dimension must be in [2, 2^20]");
    std::memset(&L, 0, sizeof(L));
    if (storage < RT_U8 || storage > RT_U12) return fail(RT_ERR_INVALID_ARG, "unknown storage type");
    const bool u8b = storage == RT_U8_BRICKSCALED;
    if (!layout_allowed(storage, layout)) return fail(RT_ERR_INVALID_ARG, "layout not available for this storage type");
    if (u8b) {
        if (brick != 8 && brick != 16 && brick != 32)
            return fail(RT_ERR_INVALID_ARG, "brick-scaled storage needs brick 8, 16 or 32");
    } else if (brick != 0) {
        return fail(RT_ERR_INVALID_ARG, "brick must be 0 unless the storage is brick-scaled");
    }
    if (u8b && layout == RT_LAYOUT_BRICKS) {
        size_t nbt = 1;
        for (int a = 0; a < 3; ++a) {
            L.nb[a] = (int32_t)((dims[a] - 1 + brick - 1) / brick);
            nbt *= (size_t)L.nb[a];
        }
        const size_t S = (size_t)brick + 3;
        L.sy = (uint32_t)S;
        L.sz = (uint32_t)(S * S);
        L.brick_bytes = (uint32_t)(S * S * S);
        L.bshift = brick == 8 ? 3 : (brick == 16 ? 4 : 5);
        L.layout = LAYOUT_BRICKS;
        L.data_offset = round256(nbt * sizeof(float2));
        L.data_bytes = nbt * S * S * S;
        if (nbt >= ((size_t)1 << 24) || L.data_bytes >= ((size_t)1 << 31))
            return fail(RT_ERR_UNSUPPORTED, "volume too large for 32-bit brick addressing");
        L.total = round256(L.data_offset + L.data_bytes);
        return RT_OK;
    }
    if (u8b) {
        // [block (lo, scale) x ncb][codes 64 B x ncb][brick (lo, scale) x nbricks]
        size_t nbt = 1, ncb = 1;
        for (int a = 0; a < 3; ++a) {
            L.nb[a] = (int32_t)((dims[a] + 1) / 2 + 1);  // shifted cell blocks covering padded cells 0..n
            L.brick_nb[a] = (int32_t)((dims[a] - 1 + brick - 1) / brick);
            ncb *= (size_t)L.nb[a];
            nbt *= (size_t)L.brick_nb[a];
        }
        L.bshift = brick == 8 ? 3 : (brick == 16 ? 4 : 5);
        L.layout = LAYOUT_CELLS;
        L.par_bytes = round256(ncb * sizeof(float2));
        L.data_offset = L.par_bytes;
        L.data_bytes = ncb * 64;
        L.brick_par_offset = round256(L.data_offset + L.data_bytes);
        if (ncb >= ((size_t)1 << 24) || L.data_bytes > 0xffffffffull)
            return fail(RT_ERR_UNSUPPORTED, "volume too large for the cell-packed layout (4 GiB)");
        L.total = round256(L.brick_par_offset + nbt * sizeof(float2));
        return RT_OK;
    }
    const int e = layout == RT_LAYOUT_POLY ? 4 : elem_bytes(storage);  // poly cells hold binary32 coefficients
    const size_t px = (size_t)dims[0] + 2, py = (size_t)dims[1] + 2, pz = (size_t)dims[2] + 2;
    L.data_offset = 0;
    if (layout == RT_LAYOUT_CELLS || layout == RT_LAYOUT_POLY) {
        L.layout = layout == RT_LAYOUT_POLY ? LAYOUT_POLY : LAYOUT_CELLS;
        size_t nbt = 1;
        for (int a = 0; a < 3; ++a) {
            L.nb[a] = (int32_t)((dims[a] + 2) / 2);  // padded cells 0..n, rounded up to pairs
            nbt *= (size_t)L.nb[a];
        }
        L.data_bytes = nbt * 8 * 8 * (size_t)e;
        if (nbt >= ((size_t)1 << 24) || L.data_bytes > 0xffffffffull)
            return fail(RT_ERR_UNSUPPORTED, "volume too large for the cell-packed layout (4 GiB)");
        // cell-index strides of the y and z block coordinates (24-bit multiplies in the marcher)
        if (8 * (size_t)L.nb[0] * L.nb[1] >= ((size_t)1 << 24))
            return fail(RT_ERR_UNSUPPORTED, "slice too large for the cell-packed layout (24-bit strides)");
        L.sy = (uint32_t)(8 * (size_t)L.nb[0] - 4);
        L.sz = (uint32_t)(8 * (size_t)L.nb[0] * L.nb[1] - 8);
    } else if (layout == RT_LAYOUT_QUADS) {
        // quad bricks: 2x2 padded cell columns (0..n in x and y) by 4 padded
        // layers, 128 B each, 3 cells deep (consecutive z-bricks share a
        // layer); 8-byte-unit strides below 2^24, byte offsets below 2^31
        L.layout = LAYOUT_QUADS;
        L.nb[0] = (int32_t)((dims[0] + 2) / 2);
        L.nb[1] = (int32_t)((dims[1] + 2) / 2);
        L.nb[2] = (int32_t)((dims[2] + 3) / 3);
        if (dims[2] + 2 >= 65536) return fail(RT_ERR_UNSUPPORTED, "more than 65533 slices in the quad layout");
        const size_t slice = (size_t)L.nb[0] * L.nb[1];
        if (slice * 16 >= ((size_t)1 << 24))
            return fail(RT_ERR_UNSUPPORTED, "slice too large for the quad layout (24-bit strides)");
        L.sy = (uint32_t)(16 * (size_t)L.nb[0] - 16);  // y-brick stride less the in-brick y step, 8 B units
        L.sz = (uint32_t)(16 * slice - 3);                // z-brick stride less 3 layers, 8 B units
        L.data_bytes = slice * L.nb[2] * 128;
        if (L.data_bytes >= ((size_t)1 << 31)) return fail(RT_ERR_UNSUPPORTED, "volume larger than 2 GiB of storage");
    } else {
        L.layout = LAYOUT_LINEAR;
        L.sy = (uint32_t)(px * e);
        L.sz = (uint32_t)(px * py * e);
        if (px * py * e >= ((size_t)1 << 24)) return fail(RT_ERR_UNSUPPORTED, "slice too large for 24-bit addressing");
        L.data_bytes = px * py * pz * e;
        if (L.data_bytes >= ((size_t)1 << 31)) return fail(RT_ERR_UNSUPPORTED, "volume larger than 2 GiB of storage");
    }
    L.total = round256(L.data_bytes);
    return RT_OK;
}

ff to_ff(double x) {
    ff r;
    r.hi = (float)x;
    r.lo = (float)(x - (double)r.hi);
    return r;
}

void cross(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
double norm(const double a[3]) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

enum { LAUNCH_SINGLE = 0, LAUNCH_BATCH = 1, LAUNCH_BATCH_SKIP = 2 };

void set_waves(LaunchShape& ls, int waves) {
    ls.waves = waves;
    ls.bw = waves >= 8 ? 4 : (waves == 4 ? 2 : waves);  // 8 = 4x2, 12 = 4x3, 16 = 4x4 tiles
    ls.bh = waves / ls.bw;
}

// launch: LAUNCH_SINGLE (rt_render: spread tiles by default), LAUNCH_BATCH
// (the fixed-step batched kernel: 12-wavefront workgroups by default, at most
// 12) or LAUNCH_BATCH_SKIP (the batched kernel with empty-space skipping).
rt_status make_shape(const rt_render_opts* opts, int launch, LaunchShape& ls) {
    const bool single_view = launch == LAUNCH_SINGLE;
    int tw = 8, th = 8, waves = launch == LAUNCH_BATCH ? 12 : 16;
    if (opts) {
        if (opts->tile_w || opts->tile_h) {
            tw = opts->tile_w;
            th = opts->tile_h;
        }
        if (opts->waves_per_block) waves = opts->waves_per_block;
        if (opts->tile_order < 0 || opts->tile_order > 2)
            return fail(RT_ERR_INVALID_ARG, "tile_order must be 0, 1 or 2");
    }
    const int order = opts ? opts->tile_order : 0;
    ls.order = order == 2 || (order == 0 && single_view) ? 1 : 0;  // 1 = spread
    if (tw <= 0 || th <= 0 || tw * th != 64 || (tw & (tw - 1)))
        return fail(RT_ERR_UNSUPPORTED, "tile must be tile_w x tile_h = 64 with tile_w a power of two");
    if (waves != 1 && waves != 2 && waves != 4 && waves != 8 && waves != 12 && waves != 16)
        return fail(RT_ERR_UNSUPPORTED, "waves_per_block must be 1, 2, 4, 8, 12 or 16");
    if (launch == LAUNCH_BATCH && waves > 12)
        return fail(RT_ERR_UNSUPPORTED, "a batched launch without empty-space skipping takes at most 12 waves per "
                                        "workgroup");
    ls.tile_w = tw;
    ls.tile_h = th;
    set_waves(ls, waves);
    return RT_OK;
}

// Compute units of the current device (queried once per device).
int cu_count() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cache[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

// Default wavefronts per workgroup of a single view: as many as keep every
// compute unit busy -- a 16-wavefront workgroup fills a CU's four SIMDs, so a
// view of fewer tiles than 16 per CU would leave CUs idle.
int default_waves_for_tiles(long long tiles) {
    const long long per_cu = tiles / std::max(cu_count(), 1);
    int waves = 1;
    while (waves < 16 && 2LL * waves <= per_cu) waves *= 2;
    return waves;
}
int default_waves(int W, int H, const LaunchShape& ls) {
    return default_waves_for_tiles((long long)((W + ls.tile_w - 1) / ls.tile_w) * ((H + ls.tile_h - 1) / ls.tile_h));
}
// Ray tiles of a batch's views (sizes not yet checked: non-positive counts 0).
long long batch_tiles(const rt_render_job* jobs, int n, const LaunchShape& ls) {
    long long t = 0;
    for (int i = 0; i < n; ++i)
        if (jobs[i].width > 0 && jobs[i].height > 0)
            t += (long long)((jobs[i].width + ls.tile_w - 1) / ls.tile_w) * ((jobs[i].height + ls.tile_h - 1) / ls.tile_h);
    return t;
}
// Batches up to this many pixels take a plan's latency form by default: the
// rays the single-view kernel's occupancy (4 wavefronts per SIMD) holds at
// once on every compute unit.
long long latency_pixels() { return (long long)cu_count() * 4 * 4 * 64; }

rt_status make_view(const rt_volume* vol, const int64_t dims[3], const double spacing[3], const rt_tf* tf,
                    const rt_camera* cam, int W, int H, double step_vox, double cutoff, const float* bg,
                    float* out, int32_t* counts, const LaunchShape& ls, int ray_function, float iso_value,
                    float iso_high, int skip_empty, double opacity_unit, ViewDesc& v) {
    if (!vol || !tf || !cam || !out) return fail(RT_ERR_INVALID_ARG, "NULL volume, transfer function, camera or output");
    if (dims)
        for (int a = 0; a < 3; ++a)
            if (dims[a] != vol->dims[a]) return fail(RT_ERR_INVALID_ARG, "dims differ from the volume's dims");
    double sp[3];
    for (int a = 0; a < 3; ++a) {
        sp[a] = spacing ? spacing[a] : vol->spacing[a];
        if (!(sp[a] > 0.0) || !std::isfinite(sp[a])) return fail(RT_ERR_INVALID_ARG, "spacing must be finite and > 0");
    }
    if (W < 1 || H < 1 || W > 32768 || H > 32768) return fail(RT_ERR_INVALID_ARG, "image size must be in [1, 32768]");
    if (!(step_vox > 0.0) || !std::isfinite(step_vox)) return fail(RT_ERR_INVALID_ARG, "step must be finite and > 0");
    if (!(cutoff > 0.0 && cutoff <= 1.0)) return fail(RT_ERR_INVALID_ARG, "alpha cutoff must be in (0, 1]");
    if (((uintptr_t)out & 15) != 0) return fail(RT_ERR_INVALID_ARG, "output must be 16-byte aligned");
    if (ray_function < RT_COMPOSITE || ray_function > RT_THRESHOLD)
        return fail(RT_ERR_INVALID_ARG, "unknown ray function");
    if (ray_function == RT_ISO && !std::isfinite(iso_value)) return fail(RT_ERR_INVALID_ARG, "iso-value must be finite");
    if (ray_function == RT_THRESHOLD &&
        !(std::isfinite(iso_value) && std::isfinite(iso_high) && iso_value <= iso_high))
        return fail(RT_ERR_INVALID_ARG, "threshold window must be finite with iso_value <= iso_high");
    if (!finite3(cam->eye) || !finite3(cam->center) || !finite3(cam->up))
        return fail(RT_ERR_INVALID_ARG, "camera vectors must be finite");
    double f[3] = {cam->center[0] - cam->eye[0], cam->center[1] - cam->eye[1], cam->center[2] - cam->eye[2]};
    const double fl = norm(f);
    if (!(fl > 0.0)) return fail(RT_ERR_INVALID_ARG, "camera eye equals center");
    double w[3] = {f[0] / fl, f[1] / fl, f[2] / fl}, s[3], u[3], vv[3];
    cross(w, cam->up, s);
    const double sl = norm(s);
    if (!(sl >= 1e-12 * norm(cam->up)) || !(sl > 0.0)) return fail(RT_ERR_INVALID_ARG, "camera up is parallel to the view");
    for (int a = 0; a < 3; ++a) u[a] = s[a] / sl;
    cross(u, w, vv);
    double scale;
    if (cam->perspective) {
        if (!(cam->fovy_deg > 0.0 && cam->fovy_deg < 180.0)) return fail(RT_ERR_INVALID_ARG, "fovy must be in (0, 180)");
        scale = std::tan(0.5 * cam->fovy_deg * M_PI / 180.0) / (double)H;
    } else {
        if (!(cam->ortho_half_height > 0.0) || !std::isfinite(cam->ortho_half_height))
            return fail(RT_ERR_INVALID_ARG, "orthographic half-height must be finite and > 0");
        scale = cam->ortho_half_height / (double)H;
    }
    if (bg)
        for (int c = 0; c < 4; ++c)
            if (!std::isfinite(bg[c])) return fail(RT_ERR_INVALID_ARG, "background must be finite");
    if (!(opacity_unit >= 0.0) || !std::isfinite(opacity_unit))
        return fail(RT_ERR_INVALID_ARG, "opacity unit distance must be finite and >= 0");
    const double dt = step_vox * std::min(sp[0], std::min(sp[1], sp[2]));
    double diag2 = 0.0;
    for (int a = 0; a < 3; ++a) diag2 += std::pow((double)(vol->dims[a] - 1) * sp[a], 2);
    if (std::sqrt(diag2) / dt + 2.0 > (double)(1 << 30)) return fail(RT_ERR_INVALID_ARG, "step too small for the volume");

    std::memset(&v, 0, sizeof(v));
    for (int a = 0; a < 3; ++a) {
        v.eye[a] = to_ff(cam->eye[a]);
        v.w[a] = to_ff(w[a]);
        v.U[a] = to_ff(scale * u[a]);
        v.V[a] = to_ff(scale * vv[a]);
        v.inv_sp[a] = to_ff(1.0 / sp[a]);
        v.box_hi[a] = to_ff((double)(vol->dims[a] - 1) * sp[a]);
        const double eq = cam->eye[a] / sp[a] + 1.0;
        v.eye_q[a] = to_ff(eq);
        v.U_q[a] = to_ff(scale * u[a] / sp[a]);
        v.V_q[a] = to_ff(scale * vv[a] / sp[a]);
        v.w_q[a] = to_ff(w[a] / sp[a]);
        v.face_lo_q[a] = to_ff(1.0 - eq);
        v.face_hi_q[a] = to_ff((double)vol->dims[a] - eq);
    }
    v.dt = to_ff(dt);
    v.inv_dt = to_ff(1.0 / dt);
    v.thr = (float)(1.0 - cutoff);
    for (int c = 0; c < 4; ++c) v.bg[c] = bg ? bg[c] : 0.0f;
    v.W = W;
    v.H = H;
    v.perspective = cam->perspective ? 1 : 0;
    v.tiles_x = (W + ls.tile_w - 1) / ls.tile_w;
    v.tiles_y = (H + ls.tile_h - 1) / ls.tile_h;
    v.blocks_x = (v.tiles_x + ls.bw - 1) / ls.bw;
    v.nblocks = v.blocks_x * ((v.tiles_y + ls.bh - 1) / ls.bh);
    v.ray_function = ray_function;
    v.iso_lo = iso_value;
    v.iso_hi = iso_high;
    v.vol = vol->dev;
    v.tf = tf->dev;
    v.tf_nz = reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(tf->dev) + tf_nz_offset(tf->K));
    v.skip_empty = (skip_empty && (ray_function == RT_COMPOSITE || ray_function == RT_THRESHOLD)) ? 1 : 0;
    v.K = tf->K;
    const double ta = (double)(tf->K - 1) / (tf->vmax - tf->vmin);
    v.tf_a = (float)ta;
    v.tf_b = (float)(-tf->vmin * ta);
    v.alpha_exp = (opacity_unit > 0.0 && (ray_function == RT_COMPOSITE || ray_function == RT_THRESHOLD))
                      ? (float)(dt / opacity_unit)
                      : 0.0f;
    v.out = out;
    v.counts = counts;
    return RT_OK;
}

// Host buffer for a one-off batch's header, prefix and job table (the fill
// launches take the bytes with their arguments, so it is free again at once).
thread_local std::vector<unsigned char> g_staging;

size_t prefix_bytes() { return kBatchPrefixBytes; }

size_t batch_ws_bytes(int max_jobs) { return kBatchHeaderBytes + prefix_bytes() + (size_t)max_jobs * sizeof(ViewDesc); }

// Validate n jobs and fill their view descriptions descs[0..n) and block
// prefix prefix[0..n] (prefix[i] = first workgroup block of job i).
rt_status build_batch_into(const rt_render_job* jobs, int n, const LaunchShape& ls, int* kind, int* max_k,
                           ViewDesc* descs, int* prefix) {
    if (!jobs || n < 1) return fail(RT_ERR_INVALID_ARG, "empty batch");
    if (n > kMaxBatchJobs) return fail(RT_ERR_UNSUPPORTED, "too many jobs in one batch");
    prefix[0] = 0;
    *kind = -1;
    *max_k = 2;
    for (int i = 0; i < n; ++i) {
        const rt_render_job& J = jobs[i];
        if (!J.volume) return fail(RT_ERR_INVALID_ARG, "job without volume");
        rt_status st = make_view(J.volume, nullptr, nullptr, J.tf, &J.camera, J.width, J.height, J.step_vox,
                                 J.alpha_cutoff, J.bg_rgba, J.out_dev, J.pixel_counts, ls, J.ray_function,
                                 J.iso_value, J.iso_high, J.skip_empty, J.opacity_unit_distance, descs[i]);
        if (st != RT_OK) return fail(st, "job " + std::to_string(i) + ": " + g_last_error);
        const int k = J.volume->dev.kind * 8 + J.volume->dev.layout;  // storage type and layout
        if (*kind < 0) *kind = k;
        if (k != *kind) return fail(RT_ERR_UNSUPPORTED, "all volumes of a batch must share one storage type and layout");
        *max_k = std::max(*max_k, J.tf->K);
        const long long next = (long long)prefix[i] + descs[i].nblocks;
        if (next >= (1LL << 31)) return fail(RT_ERR_UNSUPPORTED, "batch too large");
        prefix[i + 1] = (int)next;
    }
    return RT_OK;
}

rt_status build_batch(const rt_render_job* jobs, int n, const LaunchShape& ls, int* kind,
                      int* max_k, std::vector<ViewDesc>& descs, std::vector<int>& prefix) {
    if (!jobs || n < 1) return fail(RT_ERR_INVALID_ARG, "empty batch");
    if (n > kMaxBatchJobs) return fail(RT_ERR_UNSUPPORTED, "too many jobs in one batch");
    descs.resize(n);
    prefix.assign(n + 1, 0);
    return build_batch_into(jobs, n, ls, kind, max_k, descs.data(), prefix.data());
}

// The workspace header of a batch of n jobs.
void make_batch_header(void* h, int n, int total_blocks, int max_k, unsigned long long* counter) {
    BatchHeader hdr;
    std::memset(&hdr, 0, sizeof(hdr));
    hdr.queue = 0;
    hdr.n_jobs = (unsigned)n;
    hdr.total_blocks = (unsigned)total_blocks;
    hdr.tf_lds_entries = max_k + 1;
    hdr.counter = counter;
    std::memset(h, 0, kBatchHeaderBytes);
    std::memcpy(h, &hdr, sizeof(hdr));
}

// Header, prefix and job table for n jobs into host memory `h` (the
// workspace image to copy).
void write_batch_host(void* h, const std::vector<ViewDesc>& descs, const std::vector<int>& prefix, int max_k,
                      unsigned long long* counter) {
    char* b = static_cast<char*>(h);
    make_batch_header(b, (int)descs.size(), prefix.back(), max_k, counter);
    std::memcpy(b + kBatchHeaderBytes, prefix.data(), prefix.size() * sizeof(int));
    std::memcpy(b + kBatchHeaderBytes + prefix_bytes(), descs.data(), descs.size() * sizeof(ViewDesc));
}

size_t batch_copy_bytes(int n) { return kBatchHeaderBytes + prefix_bytes() + (size_t)n * sizeof(ViewDesc); }

// A batch's header, block prefix and job table reach the device workspace
// through the arguments of small fill kernels (the runtime copies kernel
// arguments when the launch call is made, so the host buffer is free at once):
// no runtime memory copy on the launch path, where a small host-to-device
// copy has been seen to block its caller for milliseconds.
constexpr int kFillPayload = 3584;  // table bytes per fill launch (kernel arguments stay under 4 KiB)

struct FillChunk {
    uint32_t dst_offset;   // first segment: byte offset in the workspace, 16-byte aligned
    uint32_t bytes;        // multiple of 16
    uint32_t dst_offset2;  // second segment, from data + bytes
    uint32_t bytes2;       // multiple of 16; bytes + bytes2 <= kFillPayload
    uint4 data[kFillPayload / 16];
};

__global__ void __launch_bounds__(256) fill_workspace_kernel(unsigned char* __restrict__ ws, const FillChunk c) {
    for (uint32_t i = threadIdx.x; i * 16u < c.bytes + c.bytes2; i += blockDim.x) {
        const uint32_t o = i * 16u;
        const uint32_t d = o < c.bytes ? c.dst_offset + o : c.dst_offset2 + (o - c.bytes);
        *reinterpret_cast<uint4*>(ws + d) = c.data[i];
    }
}

// A table's upload: the device reads the pinned, coherent staging copy
// directly (n16 16-byte units), so no runtime copy runs on the request path.
__global__ void __launch_bounds__(256) upload_table_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                           uint32_t n16) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n16) dst[i] = src[i];
}

// Copy bytes_a from host a to ws + 0 and bytes_b from host b to ws + off_b
// (each rounded up to 16; the sources must be readable that far, off_b
// 16-byte aligned) in fill launches on stream s, as few as the payload allows.
hipError_t fill_workspace(unsigned char* ws, const void* a, size_t bytes_a, size_t off_b, const void* b,
                          size_t bytes_b, hipStream_t s) {
    const unsigned char* pa = static_cast<const unsigned char*>(a);
    const unsigned char* pb = static_cast<const unsigned char*>(b);
    size_t ra = (bytes_a + 15) & ~(size_t)15, rb = (bytes_b + 15) & ~(size_t)15;
    size_t da = 0, db = 0;  // bytes of each sent so far
    while (da < ra || db < rb) {
        FillChunk c;
        const size_t na = std::min(ra - da, (size_t)kFillPayload);
        const size_t nb = std::min(rb - db, (size_t)kFillPayload - na);
        c.dst_offset = (uint32_t)da;
        c.bytes = (uint32_t)na;
        c.dst_offset2 = (uint32_t)(off_b + db);
        c.bytes2 = (uint32_t)nb;
        if (na) std::memcpy(c.data, pa + da, na);
        if (nb) std::memcpy(reinterpret_cast<unsigned char*>(c.data) + na, pb + db, nb);
        hipLaunchKernelGGL(fill_workspace_kernel, dim3(1), dim3(256), 0, s, ws, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        da += na;
        db += nb;
    }
    return hipSuccess;
}

int layout_code(int layout) {
    return layout == RT_LAYOUT_LINEAR   ? LAYOUT_LINEAR
           : layout == RT_LAYOUT_BRICKS ? LAYOUT_BRICKS
           : layout == RT_LAYOUT_POLY   ? LAYOUT_POLY
           : layout == RT_LAYOUT_QUADS ? LAYOUT_QUADS
                                        : LAYOUT_CELLS;
}

}  // namespace

namespace rtv {

// Every value in [0, 1] (NaN fails): a branch-free pass the compiler
// vectorizes, as tables of 16384 values are checked on every request.
bool unit_range(const float* v, size_t n) {
    int bad = 0;
    for (size_t i = 0; i < n; ++i) bad |= !(v[i] >= 0.0f) | !(v[i] <= 1.0f);
    return bad == 0;
}


int storage_layout_kind(int storage, int layout) {
    if (storage < RT_U8 || storage > RT_U12 || !layout_allowed(storage, layout)) return -1;
    return (storage == RT_U8_BRICKSCALED ? ST_U8B : storage) * 8 + layout_code(layout);
}

int volume_kind(const rt_volume* vol) { return vol ? vol->dev.kind * 8 + vol->dev.layout : -1; }

int set_last_error(int status, const char* msg) { return fail(static_cast<rt_status>(status), msg); }

int check_request(const rt_volume* vol, int K, double vmin, double vmax, const void* camera, int W, int H,
                  double step_vox, double cutoff, const float* bg, const float* out, int ray_function,
                  float iso_value, float iso_high, double opacity_unit, int* kind) {
    if (K < 2 || K > kMaxK) return fail(RT_ERR_INVALID_ARG, "K must be in [2, 4096]");
    if (!std::isfinite(vmin) || !std::isfinite(vmax) || !(vmax > vmin)) return fail(RT_ERR_INVALID_ARG, "need vmin < vmax");
    rt_tf probe;  // geometry and table size only: never read on the device
    std::memset(&probe, 0, sizeof(probe));
    probe.dev = reinterpret_cast<const float4*>((uintptr_t)256);
    probe.K = K;
    probe.vmin = vmin;
    probe.vmax = vmax;
    LaunchShape ls;
    rt_status st = make_shape(nullptr, LAUNCH_BATCH_SKIP, ls);  // any valid shape: only the view is checked
    if (st != RT_OK) return st;
    ViewDesc v;
    st = make_view(vol, nullptr, nullptr, &probe, static_cast<const rt_camera*>(camera), W, H, step_vox, cutoff, bg,
                   const_cast<float*>(out), nullptr, ls, ray_function, iso_value, iso_high, 0, opacity_unit, v);
    if (st != RT_OK) return st;
    if (kind) *kind = volume_kind(vol);
    return RT_OK;
}

}  // namespace rtv

extern "C" {

const char* rt_status_string(rt_status s) {
    switch (s) {
        case RT_OK: return "ok";
        case RT_ERR_INVALID_ARG: return "invalid argument";
        case RT_ERR_OUT_OF_MEMORY: return "buffer too small";
        case RT_ERR_DEVICE: return "device error";
        case RT_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* rt_last_error(void) { return g_last_error.c_str(); }

const char* rt_version(void) { return "rtvol 0.1 gfx950"; }

rt_status rt_volume_bytes(const int64_t dims[3], int storage, int layout, int brick, size_t* bytes) {
    if (!bytes) return fail(RT_ERR_INVALID_ARG, "bytes is NULL");
    Layout L;
    rt_status st = compute_layout(dims, storage, layout, brick, L);
    if (st != RT_OK) return st;
    *bytes = L.total;
    return RT_OK;
}

rt_status rt_create_volume(const void* src_dev, int src_dtype, const int64_t dims[3], const double spacing[3],
                           int storage, int layout, int brick, void* dev_buf, size_t dev_buf_bytes, void* stream,
                           rt_volume** out) {
    if (!out) return fail(RT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!src_dev || !dev_buf || !spacing) return fail(RT_ERR_INVALID_ARG, "NULL source, buffer or spacing");
    if (src_dtype < RT_U8 || src_dtype > RT_F32) return fail(RT_ERR_INVALID_ARG, "source type must be U8, U16, F16 or F32");
    for (int a = 0; a < 3; ++a)
        if (!(spacing[a] > 0.0) || !std::isfinite(spacing[a])) return fail(RT_ERR_INVALID_ARG, "spacing must be finite and > 0");
    Layout L;
    rt_status st = compute_layout(dims, storage, layout, brick, L);
    if (st != RT_OK) return st;
    if (dev_buf_bytes < L.total) return fail(RT_ERR_OUT_OF_MEMORY, "volume buffer smaller than rt_volume_bytes");
    if (((uintptr_t)dev_buf & 255) != 0) return fail(RT_ERR_INVALID_ARG, "volume buffer must be 256-byte aligned");
    if (storage != RT_U8_BRICKSCALED) {
        const bool ok = storage == RT_F16 || storage == RT_F32 || (storage == RT_U16 && src_dtype <= RT_U16) ||
                        (storage == RT_U8 && src_dtype == RT_U8) || ((storage == RT_U15 || storage == RT_U12) && src_dtype <= RT_U16);
        if (!ok) return fail(RT_ERR_INVALID_ARG, "conversion to this storage type would lose information");
        if (layout == RT_LAYOUT_POLY && src_dtype > RT_U16)
            return fail(RT_ERR_INVALID_ARG, "the polynomial layout needs integer source data");
    }
    const int32_t n[3] = {(int32_t)dims[0], (int32_t)dims[1], (int32_t)dims[2]};
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(dev_buf);
    hipError_t e;
    if (storage == RT_U8_BRICKSCALED && L.layout == LAYOUT_CELLS)
        e = launch_relayout_u8b_cells(src_dev, src_dtype, n, brick, L.brick_nb,
                                      reinterpret_cast<float2*>(base + L.brick_par_offset), L.nb,
                                      reinterpret_cast<float2*>(base),
                                      reinterpret_cast<unsigned char*>(base + L.data_offset), s);
    else if (storage == RT_U8_BRICKSCALED)
        e = launch_relayout_u8b(src_dev, src_dtype, n, brick, L.nb, reinterpret_cast<float2*>(base),
                                reinterpret_cast<unsigned char*>(base + L.data_offset), s);
    else if (L.layout == LAYOUT_CELLS)
        e = launch_relayout_cells(src_dev, src_dtype, storage, n, L.nb, base, s);
    else if (L.layout == LAYOUT_POLY)
        e = launch_relayout_poly(src_dev, src_dtype, n, L.nb, base, s);
    else if (L.layout == LAYOUT_QUADS)
        e = launch_relayout_quads(src_dev, src_dtype, storage, n, L.nb, base, s);
    else
        e = launch_relayout_linear(src_dev, src_dtype, storage, n, base, s);
    if (e != hipSuccess) return hip_fail(e, "relayout launch");
    rt_volume* v = new (std::nothrow) rt_volume;
    if (!v) return fail(RT_ERR_OUT_OF_MEMORY, "host allocation failed");
    std::memset(v, 0, sizeof(*v));
    v->dev.data = reinterpret_cast<const unsigned char*>(base + L.data_offset);
    v->dev.brick_par = storage == RT_U8_BRICKSCALED ? reinterpret_cast<const float2*>(base) : nullptr;
    v->dev.data_bytes = (uint32_t)L.data_bytes;
    v->dev.sy = L.sy;
    v->dev.sz = L.sz;
    v->dev.brick_bytes = L.brick_bytes;
    for (int a = 0; a < 3; ++a) {
        v->dev.n[a] = n[a];
        v->dev.nb[a] = L.nb[a];
        v->dims[a] = dims[a];
        v->spacing[a] = spacing[a];
    }
    v->dev.bshift = L.bshift;
    v->dev.kind = storage == RT_U8_BRICKSCALED ? ST_U8B : storage;
    v->dev.layout = L.layout;
    v->dev.ess_range = reinterpret_cast<const float2*>(base + L.ess_offset);
    for (int a = 0; a < 3; ++a) v->dev.enb[a] = L.enb[a];
    v->dev.eshift = L.eshift;
    v->dev.esy = (uint32_t)L.enb[0];
    v->dev.esz = (uint32_t)(L.enb[0] * L.enb[1]);
    v->dev.ess_super = reinterpret_cast<const float2*>(base + L.sup_offset);
    for (int a = 0; a < 3; ++a) v->dev.snb[a] = L.snb[a];
    v->dev.ssy = (uint32_t)L.snb[0];
    v->dev.ssz = (uint32_t)(L.snb[0] * L.snb[1]);
    v->storage = storage;
    v->brick = brick;
    e = launch_skip_ranges(v->dev, s);
    if (e != hipSuccess) {
        delete v;
        return hip_fail(e, "skip-range launch");
    }
    *out = v;
    return RT_OK;
}

rt_status rt_destroy_volume(rt_volume* vol) {
    delete vol;
    return RT_OK;
}

rt_status rt_tf_bytes(int K, size_t* bytes) {
    if (!bytes) return fail(RT_ERR_INVALID_ARG, "bytes is NULL");
    if (K < 2 || K > kMaxK) return fail(RT_ERR_INVALID_ARG, "K must be in [2, 4096]");
    *bytes = tf_layout_bytes(K);
    return RT_OK;
}

rt_status rt_set_transfer_function(rt_tf** tf, const float* rgba, int K, double vmin, double vmax, void* dev_buf,
                                   size_t dev_buf_bytes, void* stream) {
    if (!tf || !rgba) return fail(RT_ERR_INVALID_ARG, "NULL handle pointer or table");
    if (K < 2 || K > kMaxK) return fail(RT_ERR_INVALID_ARG, "K must be in [2, 4096]");
    if (!std::isfinite(vmin) || !std::isfinite(vmax) || !(vmax > vmin)) return fail(RT_ERR_INVALID_ARG, "need vmin < vmax");
    if (!unit_range(rgba, 4 * (size_t)K)) return fail(RT_ERR_INVALID_ARG, "table entries must be in [0, 1]");
    const size_t need = tf_layout_bytes(K);
    rt_tf* t = *tf;
    if (t) {
        if (dev_buf && dev_buf != (const void*)t->dev) return fail(RT_ERR_INVALID_ARG, "an update must keep the buffer");
        if (need > t->bytes || need > t->staging_bytes)
            return fail(RT_ERR_OUT_OF_MEMORY, "table larger than the handle's device or staging buffer");
    } else {
        if (!dev_buf) return fail(RT_ERR_INVALID_ARG, "NULL device buffer");
        if (dev_buf_bytes < need) return fail(RT_ERR_OUT_OF_MEMORY, "transfer-function buffer smaller than rt_tf_bytes");
        if (((uintptr_t)dev_buf & 15) != 0) return fail(RT_ERR_INVALID_ARG, "transfer-function buffer must be 16-byte aligned");
        t = new (std::nothrow) rt_tf;
        if (!t) return fail(RT_ERR_OUT_OF_MEMORY, "host allocation failed");
        std::memset(t, 0, sizeof(*t));
        t->dev = static_cast<const float4*>(dev_buf);
        t->K = K;
        t->bytes = dev_buf_bytes;
        t->staging_bytes = need;
        hipError_t e = hipHostMalloc(&t->staging, need, hipHostMallocCoherent);
        void* sd = nullptr;
        if (e == hipSuccess) e = hipHostGetDevicePointer(&sd, t->staging, 0);
        t->staging_dev = sd;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&t->copied, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (t->staging) (void)hipHostFree(t->staging);
            delete t;
            return hip_fail(e, "transfer-function staging");
        }
    }
    if (t->pending) {  // the previous upload of this table must have left the staging buffer
        hipError_t e = hipEventSynchronize(t->copied);
        if (e != hipSuccess) return hip_fail(e, "waiting for the previous table upload");
        t->pending = false;
    }
    std::memcpy(t->staging, rgba, (size_t)K * 16);
    int32_t* nz = reinterpret_cast<int32_t*>(static_cast<char*>(t->staging) + tf_nz_offset(K));
    nz[0] = 0;
    for (int j = 0; j <= K; ++j) nz[j + 1] = nz[j] + (rgba[4 * std::min(j, K - 1) + 3] > 0.0f ? 1 : 0);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint32_t n16 = (uint32_t)(need / 16);  // need is a multiple of 256
    hipLaunchKernelGGL(upload_table_kernel, dim3((n16 + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<uint4*>(const_cast<float4*>(t->dev)),
                       static_cast<const uint4*>(t->staging_dev), n16);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(t->copied, s);
    if (e != hipSuccess) {
        if (!*tf) {
            (void)hipEventDestroy(t->copied);
            (void)hipHostFree(t->staging);
            delete t;
        }
        return hip_fail(e, "transfer-function copy");
    }
    t->pending = true;
    t->K = K;
    t->vmin = vmin;
    t->vmax = vmax;
    *tf = t;
    return RT_OK;
}

rt_status rt_destroy_tf(rt_tf* tf) {
    if (!tf) return RT_OK;
    if (tf->pending) (void)hipEventSynchronize(tf->copied);
    if (tf->copied) (void)hipEventDestroy(tf->copied);
    if (tf->staging) (void)hipHostFree(tf->staging);
    delete tf;
    return RT_OK;
}

rt_status rt_render(const rt_volume* volume, const int64_t dims[3], const double spacing[3], const rt_tf* tf,
                    const rt_camera* camera, int width, int height, double step_vox, double alpha_cutoff,
                    const float bg_rgba[4], float* out_dev, const rt_render_opts* opts, void* stream) {
    if (!dims) return fail(RT_ERR_INVALID_ARG, "dims is NULL");
    LaunchShape ls;
    rt_status st = make_shape(opts, LAUNCH_SINGLE, ls);
    if (st != RT_OK) return st;
    if ((!opts || opts->waves_per_block == 0) && width > 0 && height > 0)
        set_waves(ls, default_waves(width, height, ls));
    ViewDesc v;
    st = make_view(volume, dims, spacing, tf, camera, width, height, step_vox, alpha_cutoff, bg_rgba, out_dev,
                   opts ? opts->pixel_counts : nullptr, ls, opts ? opts->ray_function : 0,
                   opts ? opts->iso_value : 0.0f, opts ? opts->iso_high : 0.0f, opts ? opts->skip_empty : 0,
                   opts ? opts->opacity_unit_distance : 0.0, v);
    if (st != RT_OK) return st;
    hipError_t e = launch_march_plain(v, ls, opts ? opts->sample_counter : nullptr, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return RT_OK;
}

rt_status rt_batch_workspace_bytes(int max_jobs, size_t* bytes) {
    if (!bytes) return fail(RT_ERR_INVALID_ARG, "bytes is NULL");
    if (max_jobs < 1 || max_jobs > kMaxBatchJobs) return fail(RT_ERR_INVALID_ARG, "max_jobs must be in [1, 4096]");
    *bytes = batch_ws_bytes(max_jobs);
    return RT_OK;
}

rt_status rt_render_batch(const rt_render_job* jobs, int n, void* workspace, size_t ws_bytes,
                          unsigned long long* sample_counter, const rt_render_opts* opts, void* stream) {
    if (!workspace) return fail(RT_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(RT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    bool any_skip = false;
    for (int i = 0; jobs && i < n && i <= kMaxBatchJobs; ++i) any_skip = any_skip || jobs[i].skip_empty;
    LaunchShape ls;
    rt_status st = make_shape(opts, any_skip ? LAUNCH_BATCH_SKIP : LAUNCH_BATCH, ls);
    if (st != RT_OK) return st;
    std::vector<ViewDesc> descs;
    std::vector<int> prefix;
    int kind, max_k;
    st = build_batch(jobs, n, ls, &kind, &max_k, descs, prefix);
    if (st != RT_OK) return st;
    if (ws_bytes < batch_ws_bytes(n)) return fail(RT_ERR_OUT_OF_MEMORY, "workspace smaller than rt_batch_workspace_bytes");
    const size_t bytes = batch_copy_bytes(n);
    if (g_staging.size() < bytes) g_staging.resize(bytes);
    void* h = g_staging.data();
    write_batch_host(h, descs, prefix, max_k, sample_counter);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // header and the n + 1 prefix entries, then the n job descriptions; the fill
    // launches take the bytes with their arguments, so the staging buffer is free
    unsigned char* hb = static_cast<unsigned char*>(h);
    hipError_t e = fill_workspace(static_cast<unsigned char*>(workspace), hb,
                                  kBatchHeaderBytes + (size_t)(n + 1) * sizeof(int), kBatchHeaderBytes + prefix_bytes(),
                                  hb + kBatchHeaderBytes + prefix_bytes(), (size_t)n * sizeof(ViewDesc), s);
    if (e != hipSuccess) return hip_fail(e, "job-table fill");
    const bool skip = any_skip;  // the kernel the shape was checked for
    const int grid = std::min(batch_persistent_grid(ls, max_k, skip), std::max(prefix.back(), 1));
    e = launch_march_batch(kind / 8, kind % 8, workspace, grid, ls, max_k, skip, s);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return RT_OK;
}

rt_status rt_batch_plan_create(int max_jobs, int storage, int layout, void* workspace, size_t ws_bytes,
                               const rt_render_opts* opts, rt_batch_plan** out) {
    if (!out) return fail(RT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!workspace) return fail(RT_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(RT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (max_jobs < 1 || max_jobs > kMaxBatchJobs) return fail(RT_ERR_INVALID_ARG, "max_jobs must be in [1, 4096]");
    if (ws_bytes < batch_ws_bytes(max_jobs)) return fail(RT_ERR_OUT_OF_MEMORY, "workspace smaller than rt_batch_workspace_bytes");
    if (storage < RT_U8 || storage > RT_U12) return fail(RT_ERR_INVALID_ARG, "unknown storage type");
    if (!layout_allowed(storage, layout)) return fail(RT_ERR_INVALID_ARG, "layout not available for this storage type");
    if (opts && (opts->batch_form < 0 || opts->batch_form > 2))
        return fail(RT_ERR_INVALID_ARG, "batch_form must be 0, 1 or 2");
    LaunchShape ls;
    rt_status st = make_shape(opts, opts && opts->skip_empty ? LAUNCH_BATCH_SKIP : LAUNCH_BATCH, ls);
    if (st != RT_OK) return st;
    rt_batch_plan* p = new (std::nothrow) rt_batch_plan;
    if (!p) return fail(RT_ERR_OUT_OF_MEMORY, "host allocation failed");
    std::memset(p, 0, sizeof(*p));
    p->max_jobs = max_jobs;
    p->kind = storage_layout_kind(storage, layout);
    p->form = opts ? opts->batch_form : 0;
    p->skip = opts && opts->skip_empty;
    p->ls = ls;
    // the latency form: rt_render's tile (8x8 unless given) in spread order
    st = make_shape(opts, LAUNCH_SINGLE, p->ls_lat);
    if (st != RT_OK) {
        delete p;
        return st;
    }
    p->ls_lat.order = 1;
    p->grid = batch_persistent_grid(ls, kMaxK, opts && opts->skip_empty);
    p->ws = workspace;
    p->ws_bytes = ws_bytes;
    hipStream_t cs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipStreamCreate");
    }
    // The graph holds the kernel alone: each launch first copies the job
    // table, whose header starts the block queue at zero.
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess)
        e = launch_march_batch(p->kind / 8, p->kind % 8, workspace, p->grid, ls, kMaxK, opts && opts->skip_empty, cs);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        delete p;
        return hip_fail(e, "batch graph capture");
    }
    p->graph = g;
    p->staging_bytes = batch_copy_bytes(max_jobs);
    p->staging = std::aligned_alloc(64, (p->staging_bytes + 63) & ~(size_t)63);
    if (!p->staging) {
        rt_batch_plan_destroy(p);
        return fail(RT_ERR_OUT_OF_MEMORY, "batch plan staging");
    }
    *out = p;
    return RT_OK;
}

long long rt_batch_latency_pixels(void) { return latency_pixels(); }

rt_status rt_batch_plan_launch(rt_batch_plan* p, const rt_render_job* jobs, int n, unsigned long long* sample_counter,
                               void* stream) {
    if (!p) return fail(RT_ERR_INVALID_ARG, "plan is NULL");
    if (n > p->max_jobs) return fail(RT_ERR_INVALID_ARG, "more jobs than the plan holds");
    if (!jobs || n < 1) return fail(RT_ERR_INVALID_ARG, "empty batch");
    long long pixels = 0;
    for (int i = 0; i < n; ++i) pixels += (long long)std::max(jobs[i].width, 0) * std::max(jobs[i].height, 0);
    const bool lat = p->form == 2 || (p->form == 0 && pixels <= latency_pixels());
    LaunchShape ls = p->ls;
    if (lat) {  // workgroups sized to the batch, as rt_render sizes them to a view
        ls = p->ls_lat;
        set_waves(ls, default_waves_for_tiles(batch_tiles(jobs, n, ls)));
    }
    std::vector<ViewDesc> descs;
    std::vector<int> prefix;
    int kind, max_k;
    rt_status st = build_batch(jobs, n, ls, &kind, &max_k, descs, prefix);
    if (st != RT_OK) return st;
    if (kind != p->kind) return fail(RT_ERR_INVALID_ARG, "jobs' storage type or layout differs from the plan's");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (lat && n == 1) {  // one view: the single-view kernel, as rt_render launches it
        hipError_t e = launch_march_plain(descs[0], ls, sample_counter, s);
        if (e != hipSuccess) return hip_fail(e, "latency-form launch");
        return RT_OK;
    }
    if (lat && n <= kSmallBatchJobs) {  // the job table travels in the kernel arguments
        SmallBatch b;
        std::memset(&b, 0, sizeof(b));
        for (int i = 0; i < n; ++i) b.v[i] = descs[i];
        for (int i = 0; i <= n; ++i) b.prefix[i] = prefix[i];
        b.n = n;
        b.tf_lds_entries = max_k + 1;
        b.counter = sample_counter;
        hipError_t e = launch_march_views_args(p->kind / 8, p->kind % 8, b, ls, p->skip, s);
        if (e != hipSuccess) return hip_fail(e, "latency-form launch");
        return RT_OK;
    }
    // header and the n + 1 prefix entries, then the n job descriptions
    write_batch_host(p->staging, descs, prefix, max_k, sample_counter);
    unsigned char* st_b = static_cast<unsigned char*>(p->staging);
    hipError_t e = fill_workspace(static_cast<unsigned char*>(p->ws), st_b,
                                  kBatchHeaderBytes + (size_t)(n + 1) * sizeof(int), kBatchHeaderBytes + prefix_bytes(),
                                  st_b + kBatchHeaderBytes + prefix_bytes(), (size_t)n * sizeof(ViewDesc), s);
    if (e != hipSuccess) return hip_fail(e, "job-table fill");
    if (lat) {
        e = launch_march_views(p->kind / 8, p->kind % 8, p->ws, prefix.back(), ls, max_k, p->skip, s);
        if (e != hipSuccess) return hip_fail(e, "latency-form launch");
        return RT_OK;
    }
    e = hipGraphLaunch(p->exec, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return RT_OK;
}

rt_status rt_batch_plan_destroy(rt_batch_plan* p) {
    if (!p) return RT_OK;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    std::free(p->staging);
    delete p;
    return RT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// rt_render_batch_noalloc: the batched launch with its workspace in this
// file's device array `scratch` (one copy per GPU, held until the process
// ends).  The header, block prefix and job table reach it through the
// arguments of small fill kernels (the runtime copies kernel arguments at
// launch), so the call needs no device or pinned host allocation and no copy
// from pageable memory.  Calls that overlap on one GPU share the array and
// race; each call rewrites the header, whose block queue word starts at zero.
// ---------------------------------------------------------------------------
namespace {

constexpr int kNoAllocMaxJobs = 64;
constexpr size_t kNoAllocDescOffset = kBatchHeaderBytes + kBatchPrefixBytes;
constexpr size_t kNoAllocBytes = kNoAllocDescOffset + (size_t)kNoAllocMaxJobs * sizeof(ViewDesc) + 16;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];  // device address of `scratch` per device, set on first use

// The current device's address of `scratch`, looked up once per device with
// that device current.
rt_status scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RT_ERR_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(RT_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return RT_OK;
}

}  // namespace

extern "C" {

rt_status rt_render_batch_noalloc(const rt_render_job* jobs, int n, unsigned long long* sample_counter,
                                  const rt_render_opts* opts, void* stream) {
    if (n > kNoAllocMaxJobs) return fail(RT_ERR_UNSUPPORTED, "rt_render_batch_noalloc takes at most 64 jobs");
    bool any_skip = false;
    for (int i = 0; jobs && i < n; ++i) any_skip = any_skip || jobs[i].skip_empty;
    LaunchShape ls;
    rt_status st = make_shape(opts, any_skip ? LAUNCH_BATCH_SKIP : LAUNCH_BATCH, ls);
    if (st != RT_OK) return st;
    // header + prefix, and the job table (one spare entry: the 16-byte
    // rounding of a copy stays inside the arrays)
    alignas(16) unsigned char head[kBatchHeaderBytes + ((kNoAllocMaxJobs + 1) * sizeof(int) + 15) / 16 * 16];
    alignas(16) ViewDesc descs[kNoAllocMaxJobs + 1];
    int* prefix = reinterpret_cast<int*>(head + kBatchHeaderBytes);
    int kind, max_k;
    st = build_batch_into(jobs, n, ls, &kind, &max_k, descs, prefix);
    if (st != RT_OK) return st;
    make_batch_header(head, n, prefix[n], max_k, sample_counter);
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != RT_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char* w = static_cast<unsigned char*>(ws);
    hipError_t e = fill_workspace(w, head, kBatchHeaderBytes + (size_t)(n + 1) * sizeof(int), kNoAllocDescOffset,
                                  descs, (size_t)n * sizeof(ViewDesc), s);
    if (e != hipSuccess) return hip_fail(e, "workspace fill");
    const int grid = std::min(batch_persistent_grid(ls, max_k, any_skip), std::max(prefix[n], 1));
    e = launch_march_batch(kind / 8, kind % 8, ws, grid, ls, max_k, any_skip, s);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return RT_OK;
}

}  // extern "C"
