// rt_internal.h -- structures shared by the library's host runtime and its
// HIP kernels.  Product code only; the reference oracle has its own header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct rt_volume;

namespace rtv {

// A float-float number: value = hi + lo with |lo| <= ulp(hi)/2.  Used for the
// per-ray set-up so that sample positions carry ~44 bits.
struct ff {
    float hi, lo;
};

enum StorageKind : int { ST_U8 = 0, ST_U16 = 1, ST_F16 = 2, ST_F32 = 3, ST_U8B = 4, ST_U15 = 5, ST_U12 = 6 };
// Ray functions as stored in a view descriptor (values of rt_ray_function).
enum RayFn : int { RT_FN_COMPOSITE = 0, RT_FN_MIP = 1, RT_FN_XRAY = 2, RT_FN_AVERAGE = 3, RT_FN_ISO = 4,
                   RT_FN_THRESHOLD = 5 };

enum LayoutKind : int { LAYOUT_CELLS = 0, LAYOUT_LINEAR = 1, LAYOUT_BRICKS = 2, LAYOUT_POLY = 3, LAYOUT_QUADS = 4 };

// Device view of a volume in storage layout.  All layouts work on the
// padded grid: nodes P = 0..n+1 per axis, node P holding node clamp(P-1)
// of the volume (one replicated border node on every face), so a sample a
// hair outside the box still finds 8 valid corners and clamp-to-edge holds.
//  LAYOUT_CELLS (U8/U16/F16/F32, default): every padded cell C = 0..n
//    stores its 8 corners contiguously (x fastest: c000 c100 c010 c110
//    c001 c101 c011 c111); cells are grouped in 2x2x2 blocks (one 128-byte
//    line for 16-bit storage), blocks in x-fastest order.  One vector load
//    per sample, and the cache lines a ray tile touches do not depend on
//    the viewing direction.
//    For U15 the 8 16-bit words of a cell are the x-pairs (c000, c100-c000),
//    (c010, c110-c010), (c001, c101-c001), (c011, c111-c011): the first of
//    each pair unsigned, the difference a signed 16-bit integer.
//  LAYOUT_POLY (U8/U16): like LAYOUT_CELLS, but a cell holds the binary32
//    coefficients p0, px, py, pz, pxy, pxz, pyz, pxyz of its trilinear
//    polynomial v = p0 + px fx + py fy + pz fz + pxy fx fy + pxz fx fz
//    + pyz fy fz + pxyz fx fy fz (sums of at most 8 integer corners: exact).
//  LAYOUT_LINEAR (U8/U16/F16/F32): the padded grid in C order.
//  LAYOUT_QUADS (U16/U12): the quad of a padded cell column (x, y) at a
//    padded layer z is its 4 nodes (x..x+1, y..y+1) at that layer, four
//    16-bit words, x fastest (for U12 the halves of value - 2048); a cell is
//    the quads of its two layers.  Quad bricks of 2x2 columns by 4 layers
//    hold 3 cells in z (z-brick b: layers 3b..3b+3, the last shared with
//    brick b+1), one 128-byte line each, x-fastest brick order; within a
//    brick column (y&1)*2 + (x&1) holds its 4 layers contiguously, so a
//    cell's quads are 16 consecutive bytes in the cell layout's word order.
//    nb: bricks per axis; sy = 16 nb[0] - 16 and sz = 16 nb[0] nb[1] - 3:
//    the y and z brick strides in 8-byte units less what the in-brick terms
//    already count (cell offset / 8 = 4x + 8y + z + 8 (x>>1) + sy (y>>1)
//    + sz (z/3)).
//    For U8B the cell blocks are shifted by one cell (block = (C+1)/2) so a
//    block never straddles a brick (B even); each block keeps the (lo,
//    scale) of the brick owning its cells in `brick_par` (8 B per block)
//    next to 64 B of codes.
//  LAYOUT_BRICKS (U8B): per brick of B^3 cells a (lo, scale) float2 and
//    (B+3)^3 codes for local nodes -1..B+1 (replicated beyond the volume).
struct VolDev {
    const unsigned char* data;  // grid, cells or codes
    const float2* brick_par;    // U8B: (lo, scale) per brick (BRICKS) or per cell block (CELLS)
    uint32_t data_bytes;        // size of `data` in bytes (buffer bound)
    uint32_t sy, sz;            // LINEAR: row / slice stride in bytes; BRICKS: (B+3), (B+3)^2
    uint32_t brick_bytes;       // BRICKS: (B+3)^3
    int32_t n[3];               // nodes per axis
    int32_t nb[3];              // CELLS: 2x2x2 cell blocks per axis; BRICKS: bricks per axis
    int32_t bshift;             // BRICKS: log2(B)
    int32_t kind;               // StorageKind
    int32_t layout;             // LayoutKind
    // Empty-space skipping: the padded cells 0..n per axis are grouped in skip
    // bricks of 2^eshift cells per axis; ess_range holds, per skip brick
    // (x fastest), the smallest and largest value the sampler can return for
    // a sample in one of its cells (NaN when a corner is NaN).
    const float2* ess_range;
    int32_t enb[3];             // skip bricks per axis
    int32_t eshift;
    uint32_t esy, esz;          // skip-brick index strides: enb[0], enb[0]*enb[1]
    // super-bricks of 4x4x4 skip bricks: the union of their bricks' ranges
    const float2* ess_super;
    int32_t snb[3];             // super-bricks per axis: ceil(enb / 4)
    uint32_t ssy, ssz;          // super-brick index strides
};
// At most this many skip bricks per volume (their empty bits fit in 8 KB of
// LDS).  Groups of 4x4x4 skip bricks (super-bricks) get a second mask, at most
// 544 words for any brick-grid shape within the limit (ceil(e/4) products).
static constexpr int kMaxSkipBricks = 65536;
static constexpr int kSkipWords = kMaxSkipBricks / 32;
static constexpr int kSuperWords = 544;
static constexpr int kSkipMaskBytes = (kSkipWords + kSuperWords) * 4;

// Everything one view needs; computed on the host in binary64, rounded to
// float-float.  Pixel (i,j) uses a = 2i+1-W, b = H-2j-1:
//   pinhole:      origin eye,              direction normalize(w + a*U + b*V)
//   orthographic: origin eye + a*U + b*V,  direction w
struct ViewDesc {
    ff eye[3];
    ff w[3];
    ff U[3];
    ff V[3];
    ff inv_sp[3];     // 1 / spacing
    ff box_hi[3];     // (n-1) * spacing, mm
    ff dt;            // sample spacing, mm
    ff inv_dt;        // 1 / dt
    // The same frame in padded index space (index = position / spacing + 1,
    // the volume box [1, n] per axis): eye, and per-pixel offsets U, V and the
    // orthographic direction w, each divided by the spacing; and, for the
    // pinhole (whose rays all start at the eye), the box faces relative to the
    // eye, 1 - eye_q and n - eye_q.
    ff eye_q[3];
    ff U_q[3], V_q[3], w_q[3];
    ff face_lo_q[3], face_hi_q[3];
    float thr;        // stop once transmittance T <= thr (= 1 - cutoff)
    float bg[4];
    int32_t W, H, perspective;
    int32_t tiles_x, tiles_y;   // ray tiles (of tile_w x tile_h pixels)
    int32_t blocks_x;           // workgroup blocks per block-row
    int32_t nblocks;            // workgroup blocks of this view
    int32_t ray_function;
    float iso_lo, iso_hi;       // RT_ISO: iso-value in iso_lo; RT_THRESHOLD: value window [iso_lo, iso_hi]
    VolDev vol;
    const float4* tf;           // K entries
    const int32_t* tf_nz;       // K+2 entries: nz[j] = number of table entries i < j (entry K = entry K-1) with alpha > 0
    int32_t skip_empty;         // nonzero: leap over skip bricks whose samples all have zero opacity
    int32_t K;
    float tf_a, tf_b;           // x = val*tf_a + tf_b, clamped to [0, K-1]
    float alpha_exp;            // > 0: table opacities corrected to a' = 1-(1-a)^alpha_exp when staged
    float* out;                 // H*W float4
    int32_t* counts;            // nullable
};

// Launch geometry common to the plain and batched marchers.
struct LaunchShape {
    int tile_w, tile_h;   // tile_w * tile_h == 64
    int waves;            // waves per workgroup
    int bw, bh;           // workgroup block in tiles: bw * bh == waves
    int order;            // 0: compact blocks; 1: tiles spread over the view (resolved from the options)
};

// Workspace layout of a batched launch (device memory owned by the caller).
//  [BatchHeader | 256 B][prefix: int[kMaxBatchJobs+1], 256-aligned][ViewDesc x n]
// prefix[i] = first workgroup block of view i, prefix[n] = total blocks.
struct BatchHeader {
    unsigned int queue;                 // next workgroup block to claim
    unsigned int n_jobs;
    unsigned int total_blocks;
    int32_t tf_lds_entries;             // max K over the jobs, +1
    unsigned long long* counter;        // nullable sample counter
};
static constexpr size_t kBatchHeaderBytes = 256;
static constexpr int kMaxBatchJobs = 4096;
static constexpr size_t kBatchPrefixBytes = ((size_t)(kMaxBatchJobs + 1) * sizeof(int) + 255) & ~(size_t)255;
static constexpr int kMaxK = 4096;

// Host launchers (march.hip / relayout.hip).
hipError_t launch_march_plain(const ViewDesc& v, const LaunchShape& ls, unsigned long long* counter,
                              hipStream_t s);
// Views, prefix, job count and counter pointer are read from the workspace,
// so one captured launch serves every batch that fits the workspace.
// skip: use the kernel with empty-space skipping (for the jobs that ask for it).
hipError_t launch_march_batch(int kind, int layout, void* workspace, int grid, const LaunchShape& ls, int max_k,
                              bool skip, hipStream_t s);
int batch_persistent_grid(const LaunchShape& ls, int max_k, bool skip);
// The latency form of a batch: one workgroup per block (blocks = the
// prefix's total), the job table read from the workspace as above.
hipError_t launch_march_views(int kind, int layout, void* workspace, int blocks, const LaunchShape& ls, int max_k,
                              bool skip, hipStream_t s);
// A latency-form batch of at most kSmallBatchJobs views carried whole in the
// kernel arguments (under 4 KiB): no job-table copy precedes the launch.
static constexpr int kSmallBatchJobs = 6;
struct SmallBatch {
    ViewDesc v[kSmallBatchJobs];
    int32_t prefix[kSmallBatchJobs + 1];  // prefix[i] = first block of view i, prefix[n] = blocks
    int32_t n;
    int32_t tf_lds_entries;               // max K over the views, +1
    unsigned long long* counter;          // nullable sample counter
};
hipError_t launch_march_views_args(int kind, int layout, const SmallBatch& b, const LaunchShape& ls, bool skip,
                                   hipStream_t s);

// Per skip brick value range of a volume in its storage layout (march.hip).
hipError_t launch_skip_ranges(const VolDev& vol, hipStream_t s);

hipError_t launch_relayout_linear(const void* src, int src_kind, int dst_kind, const int32_t n[3], void* dst,
                                  hipStream_t s);
hipError_t launch_relayout_cells(const void* src, int src_kind, int dst_kind, const int32_t n[3],
                                 const int32_t nb[3], void* dst, hipStream_t s);
hipError_t launch_relayout_quads(const void* src, int src_kind, int dst_kind, const int32_t n[3],
                                 const int32_t nb[3], void* dst, hipStream_t s);
hipError_t launch_relayout_poly(const void* src, int src_kind, const int32_t n[3], const int32_t nb[3], void* dst,
                                hipStream_t s);
hipError_t launch_relayout_u8b(const void* src, int src_kind, const int32_t n[3], int B, const int32_t nb[3],
                               float2* brick_par, unsigned char* codes, hipStream_t s);
// Cell-packed 8-bit codes: per-brick (lo, scale) into brick_par (nbricks),
// then codes and per-block parameters for the ncb cell blocks.
hipError_t launch_relayout_u8b_cells(const void* src, int src_kind, const int32_t n[3], int B, const int32_t nb[3],
                                     float2* brick_par, const int32_t ncb[3], float2* block_par,
                                     unsigned char* codes, hipStream_t s);

// Host-side helpers of rt_api.cpp used by the serving runtime (rt_serve.cpp).
// storage_layout_kind: the storage-type-and-layout code of a batch plan, -1
// when the pair does not exist.  check_request: the validation rt_render and
// the batch calls apply to one view, run without any device work (the table is
// given by its size and value window only); *kind receives the volume's code.
int storage_layout_kind(int storage, int layout);
bool unit_range(const float* v, size_t n);
int volume_kind(const rt_volume* vol);
// Record msg as the calling thread's rt_last_error(); returns status.
int set_last_error(int status, const char* msg);
int check_request(const rt_volume* vol, int K, double vmin, double vmax, const void* camera, int W, int H,
                  double step_vox, double cutoff, const float* bg, const float* out, int ray_function,
                  float iso_value, float iso_high, double opacity_unit, int* kind);

}  // namespace rtv
