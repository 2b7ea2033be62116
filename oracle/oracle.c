/*
 * oracle.c -- plain FP64 CPU reference raycaster (TEST INFRASTRUCTURE ONLY).
 *
 * Only the test-suite, the package smoke check and the benchmark's CPU
 * baseline load this library.  It is deliberately slow and literal: one ray
 * per pixel, scalar binary64 code, OpenMP over pixels and nothing else.
 *
 * Paper: Adeshina et al., "Hardware-Accelerated Raycasting: Towards an
 * Effective Brain MRI Visualization", arXiv:1211.5595.  Section 4.1 splits
 * ray casting into three steps; the code below is organised the same way:
 *   step 1  the path of the ray          (camera frame, pixel ray, box clip,
 *                                         evenly spaced sample lattice)
 *   step 2  the values along the ray     (trilinear resampling, Section 3.2;
 *                                         transfer-function classification,
 *                                         Sections 2.6 and 6)
 *   step 3  the ray function             (compositing, Section 4.2 eqs. 1-5;
 *                                         maximum-intensity, X-ray and
 *                                         average-intensity projection,
 *                                         Sections 2.4 and 4.1)
 *
 * Readings of points the paper leaves open (each is listed, with its reason,
 * in the project's design notes):
 *   R1  node-centred grid; the volume is the closed box [0,(n-1)s] per axis;
 *   R2  sample spacing dt = step_vox * min(spacing), in mm along a unit ray;
 *   R3  samples at the midpoints of the dt-segments of [t_near, t_far], plus
 *       one sample at the midpoint of the last, partial segment of length r,
 *       whose opacity is corrected to 1-(1-a)^(r/dt);
 *   R4  no opacity correction for full samples by default (the table alpha
 *       is the per-sample alpha); R24: on request, the table's opacities are
 *       per unit distance u and are corrected to the sample spacing,
 *       a' = 1-(1-a)^(dt/u), entry by entry before interpolation;
 *   R5  trilinear interpolation with clamp-to-edge, i0 = min(floor(q), n-2);
 *   R6  post-classification: interpolate the scalar, then look it up;
 *   R7  linear interpolation between the K table entries over [vmin, vmax];
 *   R8  colours are non-premultiplied, multiplied by alpha when composited;
 *   R9  front-to-back accumulation (equal to the paper's back-to-front sum,
 *       eq. (4), because "over" is associative);
 *   R10 early termination after the first sample whose accumulated opacity
 *       reaches the cutoff (not in the paper);
 *   R11 premultiplied background behind the volume;
 *   R12 look-at camera, pixel centres, row 0 at the top, aspect W/H;
 *   R13 projections reduce every lattice sample (no early termination): the
 *       maximum, dt times the weighted sum, or the weighted mean of the
 *       values; the scalar is classified once and laid over the background
 *       with the table's opacity;
 *   R14 thresholding composites as R9 with the samples outside the value
 *       window [iso_value, iso_high] transparent;
 *   R15 the iso-surface is hit at the first sample reaching the iso-value,
 *       refined linearly from the sample before, shaded by a headlight on
 *       the central-difference normal (ambient 0.2, diffuse 0.8), opaque.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ========================================================================= */
/* small vector helpers                                                       */
/* ========================================================================= */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
static int finite3(const double a[3]) { return isfinite(a[0]) && isfinite(a[1]) && isfinite(a[2]); }

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ========================================================================= */
/* step 1: the path of the ray (Section 4.1; camera settings, Section 6)      */
/* ========================================================================= */

/* Look-at frame (R12): w points from the eye to the centre, u to the right of
 * the image, v up in the image.  Invalid when eye == centre or up is parallel
 * to the viewing direction. */
int orc_camera_frame(const orc_camera* cam, double w[3], double u[3], double v[3]) {
    if (!cam || !finite3(cam->eye) || !finite3(cam->center) || !finite3(cam->up)) return ORC_EINVAL;
    double f[3] = {cam->center[0] - cam->eye[0], cam->center[1] - cam->eye[1], cam->center[2] - cam->eye[2]};
    double fl = norm3(f);
    if (!(fl > 0.0)) return ORC_EINVAL;
    for (int a = 0; a < 3; ++a) w[a] = f[a] / fl;
    double s[3];
    cross3(w, cam->up, s);
    double sl = norm3(s);
    if (!(sl >= 1e-12 * norm3(cam->up)) || !(sl > 0.0)) return ORC_EINVAL;
    for (int a = 0; a < 3; ++a) u[a] = s[a] / sl;
    cross3(u, w, v);
    return ORC_OK;
}

/* The viewing ray through the centre of pixel (i, j) (Section 4.1: a ray from
 * each pixel of the image plane).  Normalised image coordinates:
 *   xn = (2(i+1/2)/W - 1) * W/H,   yn = 1 - 2(j+1/2)/H.
 * Pinhole: origin at the eye, direction w + h*xn*u + h*yn*v normalised,
 * h = tan(fovy/2).  Orthographic: origin eye + hh*(xn*u + yn*v), direction w. */
int orc_pixel_ray(const orc_camera* cam, int W, int H, int i, int j, double o[3], double d[3]) {
    double w[3], u[3], v[3];
    if (W < 1 || H < 1) return ORC_EINVAL;
    if (orc_camera_frame(cam, w, u, v) != ORC_OK) return ORC_EINVAL;
    double xn = (2.0 * (i + 0.5) / W - 1.0) * ((double)W / (double)H);
    double yn = 1.0 - 2.0 * (j + 0.5) / H;
    if (cam->perspective) {
        if (!(cam->fovy_deg > 0.0 && cam->fovy_deg < 180.0)) return ORC_EINVAL;
        double h = tan(0.5 * cam->fovy_deg * M_PI / 180.0);
        double r[3];
        for (int a = 0; a < 3; ++a) r[a] = w[a] + h * xn * u[a] + h * yn * v[a];
        double rl = norm3(r);
        for (int a = 0; a < 3; ++a) {
            o[a] = cam->eye[a];
            d[a] = r[a] / rl;
        }
    } else {
        double hh = cam->ortho_half_height;
        if (!(hh > 0.0) || !isfinite(hh)) return ORC_EINVAL;
        for (int a = 0; a < 3; ++a) {
            o[a] = cam->eye[a] + hh * (xn * u[a] + yn * v[a]);
            d[a] = w[a];
        }
    }
    return ORC_OK;
}

/* Where the ray meets the volume (Section 4.1): slab test against the closed
 * box [0, hi] (R1).  For a direction component of zero the ray is inside that
 * slab for all t if lo <= o <= hi, else it misses.  The ray starts at t = 0
 * (an eye inside the volume starts sampling at the eye). */
int orc_box_clip(const double o[3], const double d[3], const double hi[3], double* t_near, double* t_far) {
    double t_in = -INFINITY, t_out = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            double t0 = (0.0 - o[a]) / d[a];
            double t1 = (hi[a] - o[a]) / d[a];
            if (t0 > t1) {
                double x = t0;
                t0 = t1;
                t1 = x;
            }
            if (t0 > t_in) t_in = t0;
            if (t1 < t_out) t_out = t1;
        } else if (o[a] < 0.0 || o[a] > hi[a]) {
            return 0;
        }
    }
    double tn = t_in > 0.0 ? t_in : 0.0;
    *t_near = tn;
    *t_far = t_out;
    return t_out > tn;
}

/* Evenly spaced samples along the ray (Section 4.1) (R3): the interval of
 * length L is cut into m segments of length dt and a remainder r in [0, dt). */
int64_t orc_lattice(double L, double dt, int64_t* m_out, double* r_out) {
    double mf = floor(L / dt);
    int64_t m = (int64_t)mf;
    double r = L - (double)m * dt;
    if (r < 0.0) {
        m -= 1;
        r += dt;
    }
    if (r >= dt) {
        m += 1;
        r -= dt;
    }
    if (m < 0) { /* L < 0 cannot happen for a hit; keep the lattice empty */
        m = 0;
        r = 0.0;
    }
    *m_out = m;
    *r_out = r;
    return m + (r > 0.0 ? 1 : 0);
}

/* ========================================================================= */
/* step 2: the values along the ray                                            */
/* ========================================================================= */

static int64_t clampi(int64_t x, int64_t lo, int64_t hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* Node value of the plain field. */
static double field_at(const orc_volume* vol, int64_t i, int64_t j, int64_t k) {
    return vol->field[(k * vol->dims[1] + j) * vol->dims[0] + i];
}

/* Decoded node value (a, b, c) of brick (bx, by, bz), 8-bit coded form. */
static double brick_node(const orc_volume* vol, const int64_t nb[3], int64_t bx, int64_t by, int64_t bz,
                         int64_t a, int64_t b, int64_t c) {
    const int64_t B1 = vol->brick + 1;
    int64_t brick_id = (bz * nb[1] + by) * nb[0] + bx;
    uint8_t code = vol->codes[brick_id * B1 * B1 * B1 + (c * B1 + b) * B1 + a];
    return (double)vol->brick_lo[brick_id] + (double)code * (double)vol->brick_scale[brick_id];
}

/* Trilinear resampling (Section 3.2) at index-space position q (R5): q is
 * clamped to the box, the cell is i0 = min(floor(q), n-2) with fraction
 * f = q - i0, and the value is the weighted sum of the cell's 8 corners with
 * weights prod_a (f_a or 1-f_a).  In the coded form all 8 corners are decoded
 * with the parameters of the brick that owns the cell. */
double orc_trilinear(const orc_volume* vol, const double q_in[3]) {
    int64_t c0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double hi = (double)(vol->dims[a] - 1);
        double q = q_in[a] < 0.0 ? 0.0 : (q_in[a] > hi ? hi : q_in[a]);
        int64_t i0 = clampi((int64_t)floor(q), 0, vol->dims[a] - 2);
        c0[a] = i0;
        f[a] = q - (double)i0;
    }
    double val = 0.0;
    if (vol->field) {
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    double wgt = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
                    val += wgt * field_at(vol, c0[0] + dx, c0[1] + dy, c0[2] + dz);
                }
    } else {
        int64_t nb[3];
        orc_u8_brick_count(vol->dims, vol->brick, nb);
        const int64_t B = vol->brick;
        int64_t bx = c0[0] / B, by = c0[1] / B, bz = c0[2] / B;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    double wgt = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
                    val += wgt * brick_node(vol, nb, bx, by, bz, c0[0] - bx * B + dx, c0[1] - by * B + dy,
                                            c0[2] - bz * B + dz);
                }
    }
    return val;
}

/* Largest magnitude among the 8 corner values that orc_trilinear blends at
 * q.  The binary32 interpolation on a device errs by a few units in the last
 * place of this magnitude; decisions taken on an interpolated value (a value
 * window, an iso-value) are flagged as rounding-decided within
 * 2^-20 of it (R21, R22). */
static double cell_corner_max(const orc_volume* vol, const double q_in[3]) {
    int64_t c0[3];
    for (int a = 0; a < 3; ++a) {
        double hi = (double)(vol->dims[a] - 1);
        double q = q_in[a] < 0.0 ? 0.0 : (q_in[a] > hi ? hi : q_in[a]);
        c0[a] = clampi((int64_t)floor(q), 0, vol->dims[a] - 2);
    }
    double mx = 0.0;
    int64_t nb[3] = {0, 0, 0};
    if (!vol->field) orc_u8_brick_count(vol->dims, vol->brick, nb);
    const int64_t B = vol->brick > 0 ? vol->brick : 1;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double v;
                if (vol->field) {
                    v = field_at(vol, c0[0] + dx, c0[1] + dy, c0[2] + dz);
                } else {
                    int64_t bx = c0[0] / B, by = c0[1] / B, bz = c0[2] / B;
                    v = brick_node(vol, nb, bx, by, bz, c0[0] - bx * B + dx, c0[1] - by * B + dy, c0[2] - bz * B + dz);
                }
                if (fabs(v) > mx) mx = fabs(v);
            }
    return mx;
}

static double decision_slack(const orc_volume* vol, const double q[3]) {
    return ldexp(cell_corner_max(vol, q), -20) + ldexp(1.0, -40);
}

/* Classification (Sections 2.6 and 6; post-classification, R6, R7): the value
 * is mapped to x = clamp((value-vmin)/(vmax-vmin), 0, 1) * (K-1) and the
 * colour and opacity are linearly interpolated between entries j0 and j0+1,
 * j0 = min(floor(x), K-2). */
void orc_classify(const orc_tf* tf, double value, double rgba[4]) {
    double x = (value - tf->vmin) / (tf->vmax - tf->vmin);
    x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
    x *= (double)(tf->K - 1);
    int64_t j0 = clampi((int64_t)floor(x), 0, tf->K - 2);
    double g = x - (double)j0;
    for (int c = 0; c < 4; ++c)
        rgba[c] = (1.0 - g) * (double)tf->rgba[4 * j0 + c] + g * (double)tf->rgba[4 * (j0 + 1) + c];
}

/* Opacity correction (R24): the table's opacities are per unit distance u;
 * a sample that stands for dt of ray gets a' = 1 - (1 - a)^(dt/u), applied to
 * the two table entries before they are interpolated, so the correction is a
 * transformation of the table (one table serves every sample of a render). */
void orc_classify_corrected(const orc_tf* tf, double value, double r, double rgba[4]) {
    orc_classify(tf, value, rgba);
    if (!(r > 0.0)) return;
    double x = (value - tf->vmin) / (tf->vmax - tf->vmin);
    x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
    x *= (double)(tf->K - 1);
    int64_t j0 = clampi((int64_t)floor(x), 0, tf->K - 2);
    double g = x - (double)j0;
    const double a0 = 1.0 - pow(1.0 - (double)tf->rgba[4 * j0 + 3], r);
    const double a1 = 1.0 - pow(1.0 - (double)tf->rgba[4 * (j0 + 1) + 3], r);
    rgba[3] = (1.0 - g) * a0 + g * a1;
}

/* ========================================================================= */
/* step 3: the ray function                                                    */
/* ========================================================================= */

typedef struct {
    double out[4], lo[4], hi[4];
    int64_t count;
    uint8_t tie;
} ray_result;

typedef struct {
    double o[3], d[3];
    double t_near, t_far, dt;
    int64_t m;
    double r;
    int hit;
    int graze;
} ray_path;

static double min3(const double s[3]) {
    double m = s[0] < s[1] ? s[0] : s[1];
    return m < s[2] ? m : s[2];
}

static int make_path(const orc_volume* vol, const orc_camera* cam, const orc_params* prm, int i, int j,
                     ray_path* rp) {
    if (orc_pixel_ray(cam, prm->width, prm->height, i, j, rp->o, rp->d) != ORC_OK) return ORC_EINVAL;
    double hi[3];
    for (int a = 0; a < 3; ++a) hi[a] = (double)(vol->dims[a] - 1) * vol->spacing[a];
    rp->dt = prm->step_vox * min3(vol->spacing);
    rp->hit = orc_box_clip(rp->o, rp->d, hi, &rp->t_near, &rp->t_far);
    rp->graze = 0;
    rp->m = 0;
    rp->r = 0.0;
    if (rp->hit) {
        orc_lattice(rp->t_far - rp->t_near, rp->dt, &rp->m, &rp->r);
        if (rp->m == 0 && rp->r == 0.0) rp->hit = 0;
    }
    /* A chord shorter than a micrometre means hit or miss is decided by rounding. */
    if (rp->hit && rp->t_far - rp->t_near < 1e-6) rp->graze = 1;
    return ORC_OK;
}

/* Position of sample k (k < m: midpoint of segment k; k == m: midpoint of the
 * remainder) and its weight (1, or r/dt for the remainder). */
static void sample_at(const ray_path* rp, int64_t k, double* s, double* weight) {
    if (k < rp->m) {
        *s = rp->t_near + ((double)k + 0.5) * rp->dt;
        *weight = 1.0;
    } else {
        *s = rp->t_near + (double)rp->m * rp->dt + 0.5 * rp->r;
        *weight = rp->r / rp->dt;
    }
}

static double value_at(const orc_volume* vol, const ray_path* rp, double s, double q[3]) {
    for (int a = 0; a < 3; ++a) q[a] = (rp->o[a] + s * rp->d[a]) / vol->spacing[a];
    return orc_trilinear(vol, q);
}

static void bg_out(const orc_params* prm, double out[4]) {
    for (int c = 0; c < 4; ++c) out[c] = prm->bg[c];
}

/* Pixel colour from the accumulated (C, T): the volume's premultiplied colour
 * C with transmittance T over the premultiplied background (R11). */
static void composite_out(const double C[3], double T, const orc_params* prm, double out[4]) {
    for (int c = 0; c < 3; ++c) out[c] = C[c] + T * prm->bg[c];
    out[3] = (1.0 - T) + T * prm->bg[3];
}

/* Compositing (Section 4.2).  Eq. (4) writes the intensity at the eye as the
 * sum of the emissions I(S_k) of the sample points, each attenuated by
 * exp(-tau(S_k, S_eye)), the optical depth between the point and the eye;
 * eq. (5) is its continuous form.  With per-sample opacity alpha_k =
 * 1 - exp(-kappa_k * dt) and emission c_k * alpha_k, the attenuation of
 * sample k is the product of (1 - alpha_j) over the samples j between it and
 * the eye, so walking from the eye into the volume:
 *     C += T * alpha_k * c_k,   T *= (1 - alpha_k),   T starts at 1.
 * The remainder sample's opacity is 1-(1-alpha)^(r/dt) (R3).  Early
 * termination (R10): stop after the first sample with 1 - T >= cutoff.
 * Tie band: states from the first sample with 1-T >= cutoff-delta to the
 * first with 1-T >= cutoff+delta (or the last sample) are all acceptable
 * stopping points for an implementation whose accumulated opacity differs by
 * less than delta; their per-channel range is reported. */
/* Projection ray functions (Section 2.4 and the Section 4.1 list): instead of
 * compositing, each ray reduces the interpolated values of all its lattice
 * samples to one scalar (no early termination; R-f1):
 *   maximum intensity projection  s = max_k v_k (the remainder sample
 *                                  included whatever its weight),
 *   X-ray projection              s = dt * sum_k w_k v_k, the Riemann sum of
 *                                  the line integral of f over the chord,
 *   average intensity projection  s = sum_k w_k v_k / sum_k w_k,
 * with w_k = 1 for full samples and r/dt for the remainder.  The scalar is
 * classified once and laid over the background with the table's opacity:
 * out.rgb = a c + (1 - a) bg.rgb, out.a = a + (1 - a) bg.a. */
static void ray_project(const orc_volume* vol, const orc_tf* tf, const orc_params* prm, const ray_path* rp,
                        ray_result* res) {
    const int64_t n = rp->m + (rp->r > 0.0 ? 1 : 0);
    double vmax = -INFINITY, sum = 0.0, wsum = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double s, weight, q[3];
        sample_at(rp, k, &s, &weight);
        const double val = value_at(vol, rp, s, q);
        if (val > vmax) vmax = val;
        sum += weight * val;
        wsum += weight;
    }
    double scalar;
    switch (prm->ray_function) {
        case ORC_MIP: scalar = vmax; break;
        case ORC_XRAY: scalar = rp->dt * sum; break;
        default: scalar = sum / wsum; break;
    }
    double rgba[4];
    orc_classify(tf, scalar, rgba);
    const double a = rgba[3];
    for (int c = 0; c < 3; ++c) res->out[c] = a * rgba[c] + (1.0 - a) * prm->bg[c];
    res->out[3] = a + (1.0 - a) * prm->bg[3];
    res->count = n;
    memcpy(res->lo, res->out, sizeof(res->out));
    memcpy(res->hi, res->out, sizeof(res->out));
}

/* Iso-surface (Section 4.1 list; R22).  The surface is hit at the first
 * lattice sample whose value reaches the iso-value; the hit point is refined
 * by linear interpolation between that sample and the one before it (none
 * when it is the first sample).  The normal is the direction of steepest
 * descent of the trilinear field, from central differences over +-1/2 voxel
 * per axis in index space scaled to millimetres; with a headlight the shade
 * is c * (0.2 + 0.8 |n.d|), c the table colour at the iso-value, and the
 * surface is opaque.  A miss shows the background. */
static void iso_shade(const orc_volume* vol, const orc_tf* tf, const orc_params* prm, const ray_path* rp, double s_hit,
                      const double dg[6], const double* pert, double out[4]) {
    /* dg (nullable): perturbations of the 6 central-difference samples */
    double p[3], q[3], g[3];
    for (int a = 0; a < 3; ++a) p[a] = rp->o[a] + s_hit * rp->d[a];
    double gg = 0.0, gd = 0.0;
    for (int a = 0; a < 3; ++a) {
        double fp, fm;
        for (int b = 0; b < 3; ++b) q[b] = p[b] / vol->spacing[b];
        q[a] += 0.5;
        fp = orc_trilinear(vol, q);
        q[a] -= 1.0;
        fm = orc_trilinear(vol, q);
        if (dg) {
            fp += pert[2 * a] * dg[2 * a];
            fm += pert[2 * a + 1] * dg[2 * a + 1];
        }
        g[a] = (fp - fm) / vol->spacing[a];
        gg += g[a] * g[a];
        gd += g[a] * rp->d[a];
    }
    const double cosang = gg > 0.0 ? fabs(gd) / sqrt(gg) : 1.0;
    double rgba[4];
    orc_classify(tf, prm->iso_value, rgba);
    const double shade = 0.2 + 0.8 * cosang;
    for (int c = 0; c < 3; ++c) out[c] = rgba[c] * shade;
    out[3] = 1.0;
}

static void ray_iso(const orc_volume* vol, const orc_tf* tf, const orc_params* prm, const ray_path* rp,
                    ray_result* res) {
    const int64_t n = rp->m + (rp->r > 0.0 ? 1 : 0);
    double s_prev = 0.0, v_prev = 0.0, e_prev = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double s, weight, q[3];
        sample_at(rp, k, &s, &weight);
        const double val = value_at(vol, rp, s, q);
        const double e = decision_slack(vol, q);
        if (fabs(val - prm->iso_value) <= e) res->tie |= 8;
        if (val >= prm->iso_value) {
            double s_hit = s, lam = 1.0, dl = 0.0;
            if (k > 0) {
                lam = (prm->iso_value - v_prev) / (val - v_prev);
                s_hit = s_prev + lam * (s - s_prev);
                /* how far the refinement may move under the values' rounding */
                dl = (e_prev * (1.0 - lam) + e * lam) / (val - v_prev);
            }
            res->count = k + 1;
            iso_shade(vol, tf, prm, rp, s_hit, NULL, NULL, res->out);
            /* band: the shade over the hit point moved by +-dl of a step and over
             * each central-difference value moved by its own rounding slack */
            double dg[6], pq[3];
            double spread[4] = {0, 0, 0, 0};
            for (int a = 0; a < 3; ++a) {
                for (int b = 0; b < 3; ++b) pq[b] = (rp->o[b] + s_hit * rp->d[b]) / vol->spacing[b];
                pq[a] += 0.5;
                dg[2 * a] = decision_slack(vol, pq);
                pq[a] -= 1.0;
                dg[2 * a + 1] = decision_slack(vol, pq);
            }
            for (int j = 0; j < 8; ++j) {
                double worst[4] = {0, 0, 0, 0};
                for (int sg = -1; sg <= 1; sg += 2) {
                    double o2[4];
                    if (j < 6) {
                        double pert[6] = {0, 0, 0, 0, 0, 0};
                        pert[j] = (double)sg;
                        iso_shade(vol, tf, prm, rp, s_hit, dg, pert, o2);
                    } else if (k > 0) {
                        const double s2 = s_prev + (lam + sg * dl) * (s - s_prev);
                        iso_shade(vol, tf, prm, rp, s2, NULL, NULL, o2);
                    } else {
                        continue;
                    }
                    for (int c = 0; c < 4; ++c)
                        if (fabs(o2[c] - res->out[c]) > worst[c]) worst[c] = fabs(o2[c] - res->out[c]);
                }
                for (int c = 0; c < 4; ++c) spread[c] += worst[c];
            }
            for (int c = 0; c < 4; ++c) {
                res->lo[c] = res->out[c] - spread[c];
                res->hi[c] = res->out[c] + spread[c];
            }
            return;
        }
        s_prev = s;
        v_prev = val;
        e_prev = e;
    }
    bg_out(prm, res->out);
    res->count = n;
    memcpy(res->lo, res->out, sizeof(res->out));
    memcpy(res->hi, res->out, sizeof(res->out));
}

static void ray_composite(const orc_volume* vol, const orc_tf* tf, const orc_params* prm, const ray_path* rp,
                          ray_result* res) {
    double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
    int64_t n = rp->m + (rp->r > 0.0 ? 1 : 0);
    const double lo_thr = prm->cutoff - prm->tie_delta, hi_thr = prm->cutoff + prm->tie_delta;
    int stopped = 0, in_band = 0;
    double state[4];
    const int window = prm->ray_function == ORC_THRESHOLD;
    const double r_corr = prm->opacity_unit > 0.0 ? rp->dt / prm->opacity_unit : 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double s, weight, q[3], rgba[4];
        sample_at(rp, k, &s, &weight);
        double val = value_at(vol, rp, s, q);
        orc_classify_corrected(tf, val, r_corr, rgba);
        double alpha = rgba[3];
        if (window) {
            /* thresholding (R21): samples outside [iso_value, iso_high] are transparent */
            const double e = decision_slack(vol, q);
            if (alpha > 0.0 && (fabs(val - prm->iso_value) <= e || fabs(val - prm->iso_high) <= e)) res->tie |= 8;
            if (val < prm->iso_value || val > prm->iso_high) alpha = 0.0;
        }
        if (k == rp->m) alpha = 1.0 - pow(1.0 - alpha, weight);
        for (int c = 0; c < 3; ++c) C[c] += T * alpha * rgba[c];
        T *= (1.0 - alpha);
        double A = 1.0 - T;
        composite_out(C, T, prm, state);
        if (!stopped) {
            res->count = k + 1;
            memcpy(res->out, state, sizeof(state));
        }
        if (A >= lo_thr && !in_band) {
            in_band = 1;
            memcpy(res->lo, state, sizeof(state));
            memcpy(res->hi, state, sizeof(state));
            if (A < hi_thr && k + 1 < n) res->tie |= 1;
        } else if (in_band) {
            for (int c = 0; c < 4; ++c) {
                if (state[c] < res->lo[c]) res->lo[c] = state[c];
                if (state[c] > res->hi[c]) res->hi[c] = state[c];
            }
        }
        if (A >= prm->cutoff) stopped = 1;
        if (stopped && (!in_band || A >= hi_thr)) break;
    }
    if (!in_band) {
        memcpy(res->lo, res->out, sizeof(res->out));
        memcpy(res->hi, res->out, sizeof(res->out));
    }
}

static int march_pixel(const orc_volume* vol, const orc_tf* tf, const orc_camera* cam, const orc_params* prm,
                       int i, int j, ray_result* res) {
    ray_path rp;
    memset(res, 0, sizeof(*res));
    if (make_path(vol, cam, prm, i, j, &rp) != ORC_OK) return ORC_EINVAL;
    if (!rp.hit) {
        bg_out(prm, res->out);
        memcpy(res->lo, res->out, sizeof(res->out));
        memcpy(res->hi, res->out, sizeof(res->out));
        res->count = 0;
        return ORC_OK;
    }
    double w = rp.r / rp.dt;
    if (rp.r > 0.0 && (w < 1e-6 || w > 1.0 - 1e-6)) res->tie |= 2;
    if (rp.r == 0.0) res->tie |= 2;
    if (rp.graze) res->tie |= 4;
    switch (prm->ray_function) {
        case ORC_COMPOSITE:
            ray_composite(vol, tf, prm, &rp, res);
            break;
        case ORC_MIP:
        case ORC_XRAY:
        case ORC_AVERAGE:
            ray_project(vol, tf, prm, &rp, res);
            break;
        case ORC_THRESHOLD:
            if (!(prm->iso_value <= prm->iso_high)) return ORC_EINVAL;
            ray_composite(vol, tf, prm, &rp, res);
            break;
        case ORC_ISO:
            ray_iso(vol, tf, prm, &rp, res);
            break;
        default:
            return ORC_EINVAL;
    }
    return ORC_OK;
}

static int check_inputs(const orc_volume* vol, const orc_tf* tf, const orc_camera* cam, const orc_params* prm) {
    if (!vol || !tf || !cam || !prm) return ORC_EINVAL;
    for (int a = 0; a < 3; ++a) {
        if (vol->dims[a] < 2) return ORC_EINVAL;
        if (!(vol->spacing[a] > 0.0) || !isfinite(vol->spacing[a])) return ORC_EINVAL;
    }
    if (!vol->field && !(vol->codes && vol->brick_lo && vol->brick_scale && vol->brick >= 1)) return ORC_EINVAL;
    if (!tf->rgba || tf->K < 2 || !(tf->vmax > tf->vmin)) return ORC_EINVAL;
    if (prm->width < 1 || prm->height < 1) return ORC_EINVAL;
    if (!(prm->step_vox > 0.0) || !isfinite(prm->step_vox)) return ORC_EINVAL;
    if (!(prm->cutoff > 0.0 && prm->cutoff <= 1.0)) return ORC_EINVAL;
    if (!(prm->tie_delta >= 0.0)) return ORC_EINVAL;
    if (!(prm->opacity_unit >= 0.0) || !isfinite(prm->opacity_unit)) return ORC_EINVAL;
    double w[3], u[3], v[3];
    if (orc_camera_frame(cam, w, u, v) != ORC_OK) return ORC_EINVAL;
    double o[3], d[3];
    if (orc_pixel_ray(cam, prm->width, prm->height, 0, 0, o, d) != ORC_OK) return ORC_EINVAL;
    return ORC_OK;
}

int orc_render(const orc_volume* vol, const orc_tf* tf, const orc_camera* cam, const orc_params* prm,
               const int64_t* pixels, int64_t n, double* out, int64_t* counts, double* band_lo, double* band_hi,
               uint8_t* tie, int nthreads) {
    if (check_inputs(vol, tf, cam, prm) != ORC_OK || !out) return ORC_EINVAL;
    const int64_t npix = (int64_t)prm->width * prm->height;
    if (!pixels) n = npix;
    if (n < 0) return ORC_EINVAL;
    if (pixels)
        for (int64_t p = 0; p < n; ++p)
            if (pixels[p] < 0 || pixels[p] >= npix) return ORC_EINVAL;
    int err = 0;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt) reduction(| : err)
#endif
    for (int64_t p = 0; p < n; ++p) {
        int64_t id = pixels ? pixels[p] : p;
        int i = (int)(id % prm->width), j = (int)(id / prm->width);
        ray_result res;
        if (march_pixel(vol, tf, cam, prm, i, j, &res) != ORC_OK) {
            err |= 1;
            continue;
        }
        for (int c = 0; c < 4; ++c) out[4 * p + c] = res.out[c];
        if (counts) counts[p] = res.count;
        if (band_lo && band_hi)
            for (int c = 0; c < 4; ++c) {
                band_lo[4 * p + c] = res.lo[c];
                band_hi[4 * p + c] = res.hi[c];
            }
        if (tie) tie[p] = res.tie;
    }
    (void)nthreads;
    return err ? ORC_EINVAL : ORC_OK;
}

int64_t orc_trace_ray(const orc_volume* vol, const orc_tf* tf, const orc_camera* cam, const orc_params* prm, int i,
                      int j, double* rec, int64_t max_rec) {
    if (check_inputs(vol, tf, cam, prm) != ORC_OK || !rec || max_rec < 0) return -1;
    if (prm->ray_function != ORC_COMPOSITE) return -1;
    ray_path rp;
    if (make_path(vol, cam, prm, i, j, &rp) != ORC_OK) return -1;
    if (!rp.hit) return 0;
    int64_t n = rp.m + (rp.r > 0.0 ? 1 : 0), nrec = 0;
    double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
    const double r_corr = prm->opacity_unit > 0.0 ? rp.dt / prm->opacity_unit : 0.0;
    for (int64_t k = 0; k < n && nrec < max_rec; ++k) {
        double s, weight, q[3], rgba[4];
        sample_at(&rp, k, &s, &weight);
        double val = value_at(vol, &rp, s, q);
        orc_classify_corrected(tf, val, r_corr, rgba);
        double alpha = rgba[3];
        if (k == rp.m) alpha = 1.0 - pow(1.0 - alpha, weight);
        for (int c = 0; c < 3; ++c) C[c] += T * alpha * rgba[c];
        T *= (1.0 - alpha);
        double* r = rec + 16 * nrec++;
        r[0] = s;
        r[1] = weight;
        r[2] = q[0];
        r[3] = q[1];
        r[4] = q[2];
        r[5] = val;
        for (int c = 0; c < 4; ++c) r[6 + c] = rgba[c];
        r[10] = alpha;
        r[11] = C[0];
        r[12] = C[1];
        r[13] = C[2];
        r[14] = T;
        r[15] = (double)(k + 1);
        if (1.0 - T >= prm->cutoff) break;
    }
    return nrec;
}

/* ========================================================================= */
/* 8-bit per-brick scaled storage (an encoding of the volume, not in the      */
/* paper: the scalar field of Section 2.1 stored with 8 bits per node).       */
/* ========================================================================= */
int64_t orc_u8_brick_count(const int64_t dims[3], int B, int64_t nb[3]) {
    int64_t total = 1;
    for (int a = 0; a < 3; ++a) {
        int64_t cells = dims[a] - 1;
        nb[a] = (cells + B - 1) / B;
        total *= nb[a];
    }
    return total;
}

int orc_encode_u8_bricks(const double* field, const int64_t dims[3], int B, float* brick_lo, float* brick_scale,
                         uint8_t* codes) {
    if (!field || !brick_lo || !brick_scale || !codes || B < 1) return ORC_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 2) return ORC_EINVAL;
    int64_t nb[3];
    orc_u8_brick_count(dims, B, nb);
    const int64_t B1 = B + 1;
    for (int64_t bz = 0; bz < nb[2]; ++bz)
        for (int64_t by = 0; by < nb[1]; ++by)
            for (int64_t bx = 0; bx < nb[0]; ++bx) {
                int64_t id = (bz * nb[1] + by) * nb[0] + bx;
                int64_t lo_n[3] = {bx * B, by * B, bz * B};
                int64_t hi_n[3];
                for (int a = 0; a < 3; ++a) {
                    hi_n[a] = lo_n[a] + B;
                    if (hi_n[a] > dims[a] - 1) hi_n[a] = dims[a] - 1;
                }
                double vmin = INFINITY, vmax = -INFINITY;
                for (int64_t k = lo_n[2]; k <= hi_n[2]; ++k)
                    for (int64_t j = lo_n[1]; j <= hi_n[1]; ++j)
                        for (int64_t i = lo_n[0]; i <= hi_n[0]; ++i) {
                            double x = field[(k * dims[1] + j) * dims[0] + i];
                            if (x < vmin) vmin = x;
                            if (x > vmax) vmax = x;
                        }
                float lo = (float)vmin, hi = (float)vmax;
                float scale = (hi > lo) ? (hi - lo) / 255.0f : 1.0f;
                brick_lo[id] = lo;
                brick_scale[id] = scale;
                uint8_t* cb = codes + id * B1 * B1 * B1;
                memset(cb, 0, (size_t)(B1 * B1 * B1));
                if (!(hi > lo)) continue;
                for (int64_t k = lo_n[2]; k <= hi_n[2]; ++k)
                    for (int64_t j = lo_n[1]; j <= hi_n[1]; ++j)
                        for (int64_t i = lo_n[0]; i <= hi_n[0]; ++i) {
                            float x = (float)field[(k * dims[1] + j) * dims[0] + i];
                            float qf = rintf((x - lo) / scale);
                            if (qf < 0.0f) qf = 0.0f;
                            if (qf > 255.0f) qf = 255.0f;
                            cb[((k - lo_n[2]) * B1 + (j - lo_n[1])) * B1 + (i - lo_n[0])] = (uint8_t)qf;
                        }
            }
    return ORC_OK;
}
