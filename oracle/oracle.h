/*
 * oracle.h -- plain FP64 CPU reference raycaster.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness oracle for the
 * GPU raycaster.  Only the test-suite, the package smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * What it computes follows "Hardware-Accelerated Raycasting: Towards an
 * Effective Brain MRI Visualization" (Adeshina et al., arXiv:1211.5595):
 *   - Section 4.1: a viewing ray per image-plane pixel, intersected with the
 *     volume, sampled at evenly spaced points; the three ray-casting steps
 *     (ray path, values along the ray, ray function);
 *   - Section 2.6 / Section 6: classification by a colour and an opacity
 *     transfer function (here one RGBA table sampled at K points);
 *   - Section 3.2: trilinear resampling filter;
 *   - Section 4.2, eqs. (1)-(5): compositing as the discrete sum of attenuated
 *     emissions along the ray (emission-absorption model, no scattering);
 *   - Section 2.4 / Section 4.1: the other ray functions (maximum intensity
 *     projection, X-ray sum, average intensity, iso-surface, thresholding).
 * Every choice the paper leaves open (grid convention, sample placement,
 * transfer-function lookup, early termination, ...) is fixed as documented
 * next to each function in oracle.c.
 *
 * All arithmetic is IEEE binary64 except the 8-bit brick encoder, whose
 * integer decisions are taken in binary32 so that a binary32 implementation
 * can reproduce them exactly.
 */
#ifndef RTVOL_ORACLE_H
#define RTVOL_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_EINVAL 1

/* Ray functions (Section 4.1 list; Section 2.4 for MIP and X-ray). */
#define ORC_COMPOSITE 0   /* front-to-back emission-absorption compositing */
#define ORC_MIP 1         /* maximum interpolated value along the ray */
#define ORC_XRAY 2        /* dt times the weighted sum of the interpolated values */
#define ORC_AVERAGE 3     /* weighted mean of the interpolated values */
/* The three projections visit every lattice sample (weights 1, and r/dt for
 * the remainder), classify the resulting scalar once and lay it over the
 * background: out.rgb = a c + (1-a) bg.rgb, out.a = a + (1-a) bg.a. */
#define ORC_ISO 4         /* first crossing of an iso-value, shaded */
#define ORC_THRESHOLD 5   /* compositing restricted to a value window */
/* Thresholding composites like ORC_COMPOSITE with the samples whose value lies
 * outside [iso_value, iso_high] transparent.  The iso-surface is hit at the
 * first sample whose value reaches iso_value, refined linearly from the
 * previous sample; out.rgb = c * (0.2 + 0.8 |n.d|) with c the table colour at
 * iso_value, n the central-difference normal (+-1/2 voxel), d the ray
 * direction; out.a = 1; a miss gives the background.  Tie bit 3 marks a pixel
 * where a window or iso decision lies within 2^-20 of the interpolated
 * cell's largest corner magnitude (decided by rounding). */

typedef struct {
    double eye[3], center[3], up[3];
    int perspective;          /* 1 pinhole, 0 orthographic */
    double fovy_deg;          /* pinhole: full vertical field of view */
    double ortho_half_height; /* orthographic: half-height of the window, mm */
} orc_camera;

/* A scalar volume on a node-centred Cartesian grid: node (i,j,k) at
 * (i*sx, j*sy, k*sz) mm.  Either a plain field of node values (field != NULL)
 * or per-brick 8-bit codes (field == NULL, see orc_encode_u8_bricks). */
typedef struct {
    int64_t dims[3];          /* nx, ny, nz; each >= 2 */
    double spacing[3];        /* > 0 */
    const double* field;      /* nz*ny*nx node values, x fastest */
    int brick;                /* B for the coded form */
    const float* brick_lo;    /* per brick, [nbz][nby][nbx] */
    const float* brick_scale; /* per brick */
    const uint8_t* codes;     /* per brick (B+1)^3 node codes, x fastest */
} orc_volume;

typedef struct {
    const float* rgba;        /* K x 4, each in [0,1]; entry j <-> value vmin + j*(vmax-vmin)/(K-1) */
    int K;                    /* >= 2 */
    double vmin, vmax;        /* vmax > vmin */
} orc_tf;

typedef struct {
    int width, height;        /* image size, >= 1 */
    double step_vox;          /* sample spacing in units of the finest voxel spacing, > 0 */
    double cutoff;            /* early termination once accumulated opacity >= cutoff, in (0,1] */
    double bg[4];             /* premultiplied background RGBA behind the volume */
    int ray_function;         /* ORC_* */
    double iso_value;         /* ORC_ISO: iso-value; ORC_THRESHOLD: window low */
    double iso_high;          /* ORC_THRESHOLD: window high */
    double tie_delta;         /* half-width of the early-termination tie band (>= 0) */
    double opacity_unit;      /* > 0: opacity correction (R24) to this sample distance, mm; 0: none */
} orc_params;

/* ---- step 1: the ray path ------------------------------------------------ */
int orc_camera_frame(const orc_camera* cam, double w[3], double u[3], double v[3]);
int orc_pixel_ray(const orc_camera* cam, int W, int H, int i, int j, double o[3], double d[3]);
/* Returns 1 and the parameter interval [t_near, t_far] if the ray meets the
 * closed box [0,hi], else 0. */
int orc_box_clip(const double o[3], const double d[3], const double hi[3],
                 double* t_near, double* t_far);
/* Sample lattice of an interval of length L: m full segments and a remainder
 * r in [0, dt).  Returns the number of samples (m, plus 1 if r > 0). */
int64_t orc_lattice(double L, double dt, int64_t* m, double* r);

/* ---- step 2: the values along the ray ------------------------------------ */
double orc_trilinear(const orc_volume* vol, const double q[3]);
void orc_classify(const orc_tf* tf, double value, double rgba[4]);
/* As orc_classify, with the opacity entries corrected to the sample spacing
 * first (R24): a' = 1 - (1 - a)^r, r = dt / unit distance; r = 0 leaves the
 * table as it is. */
void orc_classify_corrected(const orc_tf* tf, double value, double r, double rgba[4]);

/* ---- step 3: the ray function, whole images ------------------------------ */
/* Render the listed pixels (pixel id = j*W + i; NULL = all W*H in order).
 * out: n*4 RGBA.  counts (nullable): samples processed per pixel.
 * band_lo/band_hi (nullable, both or neither): per-channel range of the
 * output over the early-termination tie band.  tie (nullable): bit 0 = the
 * pixel lies in an early-termination tie band, bit 1 = its last segment is
 * within 1e-6 of empty or full (sample count may differ by one), bit 2 = the
 * ray grazes the box (hit/miss decided by rounding), bit 3 = a value-window or
 * iso-value decision is decided by rounding.  For the iso-surface the band
 * spans the shade over the rounding of the hit refinement and the normal.
 * nthreads <= 0 uses all OpenMP threads. */
int orc_render(const orc_volume* vol, const orc_tf* tf, const orc_camera* cam,
               const orc_params* prm, const int64_t* pixels, int64_t n,
               double* out, int64_t* counts, double* band_lo, double* band_hi,
               uint8_t* tie, int nthreads);

/* Per-sample trace of one pixel's ray, for tests.  Each record holds 16
 * doubles: s, weight, q[3], value, rgba[4], alpha_used, C[3], T, count.
 * Returns the number of records (<= max_rec), or -1 on invalid input. */
int64_t orc_trace_ray(const orc_volume* vol, const orc_tf* tf, const orc_camera* cam,
                      const orc_params* prm, int i, int j, double* rec, int64_t max_rec);

/* ---- 8-bit per-brick scaled storage --------------------------------------- */
/* Bricks of B^3 cells; brick b covers cells [b*B, b*B+B-1] and nodes
 * [b*B, min(b*B+B, n-1)] per axis.  lo/hi = min/max node value over the
 * brick's nodes, scale = (hi-lo)/255 and code = rint((v-lo)/scale) clamped to
 * [0,255], all in binary32 (scale 1, codes 0 when hi == lo).  A sample is
 * decoded from the brick that owns its (clamped) cell. */
int64_t orc_u8_brick_count(const int64_t dims[3], int B, int64_t nb[3]);
int orc_encode_u8_bricks(const double* field, const int64_t dims[3], int B,
                         float* brick_lo, float* brick_scale, uint8_t* codes);

int orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
