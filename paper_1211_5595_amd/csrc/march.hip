// march.hip -- the ray marcher for gfx950.
//
// One ray per lane, one ray tile (64 pixels) per wavefront, tiles grouped
// into workgroup blocks.  Per ray (arXiv:1211.5595, Section 4.1, three steps):
//   1. ray path: pixel ray from the camera (Section 6 camera settings),
//      clipped to the volume box, cut into evenly spaced samples;
//   2. values along the ray: trilinear resampling of the stored grid
//      (Section 3.2) and classification by the RGBA transfer function
//      (Sections 2.6 and 6) held in LDS;
//   3. ray function (the Section 4.1 list): front-to-back compositing of the
//      emission-absorption sum (Section 4.2, eqs. (4)-(5)) with early ray
//      termination; thresholding (compositing of a value window); maximum-,
//      X-ray and average-intensity projection (Section 2.4); iso-surface.
// Compositing can step over empty space: bricks whose samples all have zero
// opacity for the table are skipped a whole brick at a time, which leaves
// the result unchanged bit for bit.
//
// Precision: the ray set-up (direction, box entry/exit, sample lattice) runs
// in float-float; sample positions then advance as exact 32.32 fixed-point
// integers in padded index space, so the cell index is the high word and the
// trilinear fraction the low word.  Interpolation, classification and
// compositing run in binary32.  No binary64 on the device.
//
// Memory: the volume is read through buffer resources (out-of-range reads
// return zero, never fault).  In the cell-packed layouts a sample's 8 corners
// are one vector load; in the linear layout they are one vector offset plus
// 8 wave-uniform scalar offsets.
#include "ff_math.h"
#include "rt_internal.h"

namespace rtv {

namespace {

constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRsrcWord3);
}

// The volume's buffer descriptor: raw (byte offsets, byte bound) for the
// linear and brick layouts; structured with the cell as the record for the
// cell-packed layouts (8 bytes for 8-bit codes, 32 for binary32 and
// polynomial cells, 16 otherwise).
template <int KIND, int LAYOUT>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_vol_rsrc(const void* p, uint32_t bytes) {
    if constexpr (LAYOUT == LAYOUT_CELLS || LAYOUT == LAYOUT_POLY) {
        constexpr int shift = LAYOUT == LAYOUT_POLY || KIND == ST_F32 ? 5 : (KIND == ST_U8 || KIND == ST_U8B) ? 3 : 4;
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)(1 << shift), (int)(bytes >> shift),
                                                 kRsrcWord3);
    } else {
        return make_rsrc(p, bytes);
    }
}

// Member-wise copy of a volume description from any address space (the
// fields that are not used afterwards cost nothing).
template <class T>
__device__ __forceinline__ VolDev copy_vol(const T& v) {
    VolDev o;
    o.data = v.data;
    o.brick_par = v.brick_par;
    o.data_bytes = v.data_bytes;
    o.sy = v.sy;
    o.sz = v.sz;
    o.brick_bytes = v.brick_bytes;
    for (int a = 0; a < 3; ++a) {
        o.n[a] = v.n[a];
        o.nb[a] = v.nb[a];
        o.enb[a] = v.enb[a];
        o.snb[a] = v.snb[a];
    }
    o.bshift = v.bshift;
    o.kind = v.kind;
    o.layout = v.layout;
    o.ess_range = v.ess_range;
    o.eshift = v.eshift;
    o.esy = v.esy;
    o.esz = v.esz;
    o.ess_super = v.ess_super;
    o.ssy = v.ssy;
    o.ssz = v.ssz;
    return o;
}

// Per-lane state after the ray set-up.// Per-lane state after the ray set-up.
struct Ray {
    long long Q[3];   // padded index-space position of the next full sample, 32.32 fixed point
    long long dQ[3];  // increment per sample
    long long Qp[3];  // position of the remainder sample
    int m;            // number of full samples
    float wp;         // remainder weight r/dt, 0 when there is no remainder
};

// Step 1 of the ray-casting process: the ray path.  Returns false for a ray
// that misses the box [0, box_hi].
// Member-wise copy of a float-float value from any address space.
template <class T>
__device__ __forceinline__ ff ldff(const T& x) {
    return ff{x.hi, x.lo};
}

template <class VD>
__device__ __forceinline__ bool setup_ray(const VD& V, int i, int j, Ray& R) {
    const float a = (float)(2 * i + 1 - V.W);
    const float b = (float)(V.H - 2 * j - 1);
    // The ray in padded index space: origin oq and direction dq per mm of
    // the ray parameter t (the world ray divided by the spacing, plus 1 on
    // the origin), so sample positions are oq + t dq with no further scaling.
    ff oq[3], dq[3], lo[3], hi[3];
    if (V.perspective) {
        ff r[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) r[ax] = ff_add(ff_add(ldff(V.w[ax]), ff_mul_f(ldff(V.U[ax]), a)), ff_mul_f(ldff(V.V[ax]), b));
        ff n2 = ff_add(ff_add(ff_mul(r[0], r[0]), ff_mul(r[1], r[1])), ff_mul(r[2], r[2]));
        ff inv = ff_rsqrt(n2);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            oq[ax] = ldff(V.eye_q[ax]);
            dq[ax] = ff_mul(r[ax], ff_mul(inv, ldff(V.inv_sp[ax])));
            lo[ax] = ldff(V.face_lo_q[ax]);
            hi[ax] = ldff(V.face_hi_q[ax]);
        }
    } else {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            oq[ax] = ff_add(ff_add(ldff(V.eye_q[ax]), ff_mul_f(ldff(V.U_q[ax]), a)), ff_mul_f(ldff(V.V_q[ax]), b));
            dq[ax] = ldff(V.w_q[ax]);
            lo[ax] = ff_sub(ff_make(1.0f), oq[ax]);
            hi[ax] = ff_sub(ff_make((float)V.vol.n[ax]), oq[ax]);
        }
    }
    // Slab test against the closed box [1, n] (lo and hi are its faces
    // relative to the origin).  An axis the ray runs parallel to is tested in
    // world units, as the box [0, (n-1) s] against the origin.
    ff tin = ff_make(-INFINITY), tout = ff_make(INFINITY);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (dq[ax].hi == 0.0f) {
            ff o = ldff(V.eye[ax]);
            if (!V.perspective) o = ff_add(ff_add(o, ff_mul_f(ldff(V.U[ax]), a)), ff_mul_f(ldff(V.V[ax]), b));
            if (ff_lt(o, ff_make(0.0f)) || ff_lt(ldff(V.box_hi[ax]), o)) return false;
            continue;
        }
        const ff rd = ff_rcp(dq[ax]);
        ff t0 = ff_mul(lo[ax], rd);
        ff t1 = ff_mul(hi[ax], rd);
        if (ff_lt(t1, t0)) {
            ff x = t0;
            t0 = t1;
            t1 = x;
        }
        tin = ff_max(tin, t0);
        tout = ff_min(tout, t1);
    }
    const ff tnear = ff_max(tin, ff_make(0.0f));
    if (!ff_lt(tnear, tout)) return false;
    // Evenly spaced samples: m segments of dt and a remainder r in [0, dt)
    // (the quotient's floor from the reciprocal, then made exact against the
    // float-float remainder).
    const ff L = ff_sub(tout, tnear);
    int m = ff_floor_int(ff_mul(L, ldff(V.inv_dt)));
    ff r = ff_sub(L, ff_mul_f(ldff(V.dt), (float)m));
    if (r.hi < 0.0f) {
        m -= 1;
        r = ff_add(r, ldff(V.dt));
    }
    if (!ff_lt(r, ldff(V.dt))) {
        m += 1;
        r = ff_sub(r, ldff(V.dt));
    }
    if (m < 0) {
        m = 0;
        r = ff_make(0.0f);
    }
    R.m = m;
    // First sample at tnear + dt/2.
    const ff dt = ldff(V.dt);
    const ff s0 = ff_add(tnear, ff{0.5f * dt.hi, 0.5f * dt.lo});
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        R.Q[ax] = ff_to_fixed32(ff_add(oq[ax], ff_mul(s0, dq[ax])));
        R.dQ[ax] = ff_to_fixed32(ff_mul(dt, dq[ax]));
    }
    R.wp = 0.0f;
    if (r.hi > 0.0f) {
        const ff sp = ff_add(ff_add(tnear, ff_mul_f(dt, (float)m)), ff{0.5f * r.hi, 0.5f * r.lo});
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) R.Qp[ax] = ff_to_fixed32(ff_add(oq[ax], ff_mul(sp, dq[ax])));
        R.wp = r.hi * __builtin_amdgcn_rcpf(dt.hi);
    }
    return true;
}

__device__ __forceinline__ float lerp(float a, float b, float t) { return fmaf(t, b - a, a); }

// a * b + c on 24-bit unsigned operands in one instruction (the compiler
// otherwise splits the multiply-adds of a cell address into multiplies and
// three-way adds, two instructions more per sample).  b is wave-uniform.
__device__ __forceinline__ uint32_t mad24_s(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t d;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "s"(b), "v"(c));
    return d;
}
__device__ __forceinline__ uint32_t mad24_imm6(uint32_t a, uint32_t c) {
    uint32_t d;
    asm("v_mad_u32_u24 %0, %1, 6, %2" : "=v"(d) : "v"(a), "v"(c));
    return d;
}
// (a << S) + c in one instruction
template <int S>
__device__ __forceinline__ uint32_t lshl_add_(uint32_t a, uint32_t c) {
    uint32_t d;
    asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "n"(S), "v"(c));
    return d;
}
#define lshl_add(a, s, c) lshl_add_<s>((a), (c))

__device__ __forceinline__ uint32_t hiword(long long Q) { return (uint32_t)((unsigned long long)Q >> 32); }
__device__ __forceinline__ float frac32(long long Q) { return (float)(uint32_t)Q * 0x1p-32f; }

// Trilinear blend of the 8 corners c[dz*4+dy*2+dx] (Section 3.2): along x,
// then y, then z.
__device__ __forceinline__ float trilinear8(const float c[8], float fx, float fy, float fz) {
    const float x00 = lerp(c[0], c[1], fx), x10 = lerp(c[2], c[3], fx);
    const float x01 = lerp(c[4], c[5], fx), x11 = lerp(c[6], c[7], fx);
    return lerp(lerp(x00, x10, fy), lerp(x01, x11, fy), fz);
}

template <int KIND>
struct Elem;
template <>
struct Elem<ST_U8> {
    static constexpr uint32_t bytes = 1;
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t off, int soff) {
        return (float)__builtin_amdgcn_raw_buffer_load_b8(r, off, soff, 0);
    }
};
template <>
struct Elem<ST_U8B> : Elem<ST_U8> {};
template <>
struct Elem<ST_U15> {
    static constexpr uint32_t bytes = 2;  // only the cell-packed layout exists for this type
};
template <>
struct Elem<ST_U12> {
    static constexpr uint32_t bytes = 2;  // only the cell-packed layout exists for this type
};
template <>
struct Elem<ST_U16> {
    static constexpr uint32_t bytes = 2;
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t off, int soff) {
        return (float)__builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0);
    }
};
template <>
struct Elem<ST_F16> {
    static constexpr uint32_t bytes = 2;
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t off, int soff) {
        unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0);
        return (float)__builtin_bit_cast(_Float16, h);
    }
};
template <>
struct Elem<ST_F32> {
    static constexpr uint32_t bytes = 4;
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t off, int soff) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
    }
};

// Wave-uniform corner offsets of a cell in the linear and brick layouts, in bytes.
struct Corners {
    int c1, c2, c3, c4, c5, c6, c7;
};

__device__ __forceinline__ Corners corners_of(uint32_t e, uint32_t sy, uint32_t sz) {
    return Corners{(int)e, (int)sy, (int)(sy + e), (int)sz, (int)(sz + e), (int)(sz + sy), (int)(sz + sy + e)};
}

// Step 2 of the ray-casting process, split in two so the next sample's
// memory request can be issued before the current sample is processed:
// load() fetches what the sample's cell needs, value() interpolates.
template <int KIND, int LAYOUT>
struct Sampler;

// Linear padded grid: 8 scalar gathers at wave-uniform corner offsets.
template <int KIND>
struct Sampler<KIND, LAYOUT_LINEAR> {
    struct Raw {
        float c[8];
    };
    template <class VOL>
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, const VOL& vol, const Corners& cn,
                                               const long long Q[3]) {
        using E = Elem<KIND>;
        // the corner offsets ride in the scalar offset, which the buffer's bounds
        // check does not cover: a position past the padded grid (the request for
        // the sample after a ray's last, at steps above two voxels) is clamped so
        // that every corner stays inside the buffer; no cell of the grid moves
        const uint32_t off = min(__umul24(hiword(Q[2]), vol.sz) + __umul24(hiword(Q[1]), vol.sy) + hiword(Q[0]) * E::bytes,
                                 vol.data_bytes - (vol.sz + vol.sy + 2u * E::bytes));
        Raw w;
        w.c[0] = E::load(r, off, 0);
        w.c[1] = E::load(r, off, cn.c1);
        w.c[2] = E::load(r, off, cn.c2);
        w.c[3] = E::load(r, off, cn.c3);
        w.c[4] = E::load(r, off, cn.c4);
        w.c[5] = E::load(r, off, cn.c5);
        w.c[6] = E::load(r, off, cn.c6);
        w.c[7] = E::load(r, off, cn.c7);
        return w;
    }
    static __device__ __forceinline__ float value(const Raw& w, float fx, float fy, float fz) {
        return trilinear8(w.c, fx, fy, fz);
    }
};

// Cell-packed grid: one 8/16/32-byte vector load per sample.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Structured-buffer loads of the cell-packed layouts: the descriptor's record
// size is the cell's, the hardware scales the record index (no byte-offset
// shift per sample), and the bounds check counts records -- an index past the
// last cell reads zero, as an offset past the end of a raw buffer does.
__device__ u32x4 struct_load_b128(__amdgpu_buffer_rsrc_t r, uint32_t index, uint32_t voffset, uint32_t soffset,
                                  int aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.v4i32");
__device__ u32x2 struct_load_b64(__amdgpu_buffer_rsrc_t r, uint32_t index, uint32_t voffset, uint32_t soffset,
                                 int aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.v2i32");

template <int KIND>
struct CellBits;
template <>
struct CellBits<ST_U8> {
    using Raw = u32x2;
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, uint32_t cell) {
        return struct_load_b64(r, cell, 0, 0, 0);
    }
    static __device__ __forceinline__ void unpack(const Raw& w, float c[8]) {
#pragma unroll
        for (int k = 0; k < 8; ++k) c[k] = (float)((w[k >> 2] >> (8 * (k & 3))) & 0xffu);
    }
};
template <>
struct CellBits<ST_U16> {
    using Raw = u32x4;
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, uint32_t cell) {
        return struct_load_b128(r, cell, 0, 0, 0);
    }
    static __device__ __forceinline__ void unpack(const Raw& w, float c[8]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            c[2 * k] = (float)(w[k] & 0xffffu);
            c[2 * k + 1] = (float)(w[k] >> 16);
        }
    }
};
template <>
struct CellBits<ST_F16> {
    using Raw = u32x4;
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, uint32_t cell) {
        return struct_load_b128(r, cell, 0, 0, 0);
    }
    static __device__ __forceinline__ void unpack(const Raw& w, float c[8]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            c[2 * k] = (float)__builtin_bit_cast(_Float16, (unsigned short)(w[k] & 0xffffu));
            c[2 * k + 1] = (float)__builtin_bit_cast(_Float16, (unsigned short)(w[k] >> 16));
        }
    }
};
template <>
struct CellBits<ST_F32> {
    struct Raw {
        u32x4 a;
        u32x4 b;
    };
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, uint32_t cell) {
        Raw w;
        w.a = struct_load_b128(r, cell, 0, 0, 0);
        w.b = struct_load_b128(r, cell, 16, 0, 0);
        return w;
    }
    static __device__ __forceinline__ void unpack(const Raw& w, float c[8]) {
        // whole-vector casts: a bit cast of a single vector element lvalue
        // reads element 0 with this compiler
        const f32x4 fa = __builtin_bit_cast(f32x4, w.a), fb = __builtin_bit_cast(f32x4, w.b);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            c[k] = fa[k];
            c[4 + k] = fb[k];
        }
    }
};

// Storage index of padded cell (ix, iy, iz) in the 2x2x2-blocked cell order:
// 8 * block + within, block = (bz * nby + by) * nbx + bx with b = i >> 1 and
// within = (ix & 1) | (iy & 1) << 1 | (iz & 1) << 2.  Since i = 2b + (i & 1),
//   8 bx + (ix & 1) = ix + 6 bx,  8 nbx by + 2 (iy & 1) = 2 iy + (8 nbx - 4) by,
//   8 nbx nby bz + 4 (iz & 1) = 4 iz + (8 nbx nby - 8) bz,
// a sum of 24-bit multiply-adds (the strides sy = 8 nbx - 4 and
// sz = 8 nbx nby - 8 are precomputed, both below 2^24).
template <class VOL>
__device__ __forceinline__ uint32_t cell_index(const VOL& vol, const long long Q[3]) {
    const uint32_t ix = hiword(Q[0]), iy = hiword(Q[1]), iz = hiword(Q[2]);
    uint32_t c = lshl_add(iz, 2, lshl_add(iy, 1, ix));
    c = mad24_imm6(ix >> 1, c);
    c = mad24_s(iy >> 1, vol.sy, c);
    return mad24_s(iz >> 1, vol.sz, c);
}

// 15-bit difference cells: the x-lerp of a pair (c0, d = c1 - c0) is
// fma(fx, d, c0) -- exactly what trilinear8 computes from (c0, c1), so the
// images equal those of 16-bit cells bit for bit, with one conversion less
// per pair.
template <>
struct Sampler<ST_U15, LAYOUT_CELLS> {
    using Raw = u32x4;
    template <class VOL>
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, const VOL& vol, const Corners&,
                                               const long long Q[3]) {
        return struct_load_b128(r, cell_index(vol, Q), 0, 0, 0);
    }
    static __device__ __forceinline__ float value(const Raw& w, float fx, float fy, float fz) {
        float x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            x[k] = fmaf(fx, (float)(int)(short)(w[k] >> 16), (float)(w[k] & 0xffffu));
        return lerp(lerp(x[0], x[1], fy), lerp(x[2], x[3], fy), fz);
    }
};

// 12-bit half cells: each corner is the binary16 of (value - 2048), exact for
// values 0..4096.  A mixed-precision fused multiply-add reads binary16 halves
// of a register directly: one forms c1 - c0 exactly, one the x-lerp
// fma(fx, c1 - c0, c0) -- the operations of 16-bit cells on values shifted by
// 2048, with no conversions.  stored() is the interpolated value in the
// shifted units; value() adds the 2048 back.
__device__ __forceinline__ float half_pair_diff(uint32_t w) {  // hi half - lo half, exact
    float d;
    asm("v_fma_mix_f32 %0, %1, 1.0, -%1 op_sel:[1,0,0] op_sel_hi:[1,0,1]" : "=v"(d) : "v"(w));
    return d;
}
__device__ __forceinline__ float lo_half(uint32_t w) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
}

template <>
struct Sampler<ST_U12, LAYOUT_CELLS> {
    using Raw = u32x4;
    static constexpr float bias = 2048.0f;
    template <class VOL>
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, const VOL& vol, const Corners&,
                                               const long long Q[3]) {
        return struct_load_b128(r, cell_index(vol, Q), 0, 0, 0);
    }
    static __device__ __forceinline__ float stored(const Raw& w, float fx, float fy, float fz) {
        float x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = fmaf(fx, half_pair_diff(w[k]), lo_half(w[k]));
        return lerp(lerp(x[0], x[1], fy), lerp(x[2], x[3], fy), fz);
    }
    static __device__ __forceinline__ float value(const Raw& w, float fx, float fy, float fz) {
        return stored(w, fx, fy, fz) + bias;
    }
};

// Quad bricks: the quads of the sample's cell's two layers are 16
// consecutive bytes, one load from a raw buffer (whose bounds check covers
// the whole vector offset).  In 8-byte units the cell's offset is
// 4x + 8y + z + 8 (x>>1) + sy (y>>1) + sz (z/3), with z/3 as
// (z * 43691) >> 17 (exact for z < 2^17; the layout keeps z below 2^16).
// The four words are those of a 16-byte cell, so the interpolation is the
// cell samplers' own and images equal the cell layout's bit for bit.
__device__ __forceinline__ uint32_t div3(uint32_t z) {
    uint32_t d;
    asm("v_mul_u32_u24 %0, 0xaaab, %1" : "=v"(d) : "v"(z));
    return d >> 17;
}
__device__ __forceinline__ uint32_t mad24_imm8(uint32_t a, uint32_t c) {
    uint32_t d;
    asm("v_mad_u32_u24 %0, %1, 8, %2" : "=v"(d) : "v"(a), "v"(c));
    return d;
}
struct QuadsLoad {
    using Raw = u32x4;
    template <class VOL>
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, const VOL& vol, const Corners&,
                                               const long long Q[3]) {
        const uint32_t ix = hiword(Q[0]), iy = hiword(Q[1]), iz = hiword(Q[2]);
        uint32_t c = lshl_add(lshl_add(iy, 1, ix), 2, iz);
        c = mad24_imm8(ix >> 1, c);
        c = mad24_s(iy >> 1, vol.sy, c);
        c = mad24_s(div3(iz), vol.sz, c);
        return __builtin_amdgcn_raw_buffer_load_b128(r, c << 3, 0, 0);
    }
};
template <>
struct Sampler<ST_U12, LAYOUT_QUADS> : QuadsLoad {
    static constexpr float bias = Sampler<ST_U12, LAYOUT_CELLS>::bias;
    static __device__ __forceinline__ float stored(const Raw& w, float fx, float fy, float fz) {
        return Sampler<ST_U12, LAYOUT_CELLS>::stored(w, fx, fy, fz);
    }
    static __device__ __forceinline__ float value(const Raw& w, float fx, float fy, float fz) {
        return Sampler<ST_U12, LAYOUT_CELLS>::value(w, fx, fy, fz);
    }
};
template <>
struct Sampler<ST_U16, LAYOUT_QUADS> : QuadsLoad {
    static __device__ __forceinline__ float value(const Raw& w, float fx, float fy, float fz) {
        float c[8];
        CellBits<ST_U16>::unpack(w, c);
        return trilinear8(c, fx, fy, fz);
    }
};

// Cells in flight per ray in the single-view kernel's compositing loop: six
// when a sample's cell fits 16 bytes, four for the larger ones (six of those
// would exceed the kernel's registers).
template <class S>
constexpr int ring_depth() {
    return sizeof(typename S::Raw) <= 16 ? 6 : 4;
}

// An empty use of the first word of a loaded cell: pins the load ahead of a
// branch after which only one side needs it.
template <class Raw>
__device__ __forceinline__ void keep_issued(const Raw& w) {
    uint32_t first;
    __builtin_memcpy(&first, &w, sizeof(first));
    asm volatile("" ::"v"(first));
}

// Samplers whose stored values are shifted (bias != 0) give the compositing
// loop the shifted value, with the shift folded into the table mapping.
template <class...>
using void_t_ = void;
template <class S, class = void>
struct StoredBias {
    static constexpr float v = 0.0f;
};
template <class S>
struct StoredBias<S, void_t_<decltype(S::bias)>> {
    static constexpr float v = S::bias;
};
template <class S>
__device__ __forceinline__ float stored_value(const typename S::Raw& w, float fx, float fy, float fz) {
    if constexpr (StoredBias<S>::v != 0.0f)
        return S::stored(w, fx, fy, fz);
    else
        return S::value(w, fx, fy, fz);
}

template <int KIND>
struct Sampler<KIND, LAYOUT_CELLS> {
    using B = CellBits<KIND>;
    using Raw = typename B::Raw;
    template <class VOL>
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, const VOL& vol, const Corners&,
                                               const long long Q[3]) {
        return B::load(r, cell_index(vol, Q));
    }
    static __device__ __forceinline__ float value(const Raw& w, float fx, float fy, float fz) {
        float c[8];
        B::unpack(w, c);
        return trilinear8(c, fx, fy, fz);
    }
};

// Polynomial cells (integer data): 8 binary32 coefficients per cell; the
// trilinear value is the polynomial evaluated with 7 fused multiply-adds.
template <int KIND>
struct Sampler<KIND, LAYOUT_POLY> {
    using B = CellBits<ST_F32>;
    using Raw = typename B::Raw;
    template <class VOL>
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, const VOL& vol, const Corners&,
                                               const long long Q[3]) {
        return B::load(r, cell_index(vol, Q));
    }
    static __device__ __forceinline__ float value(const Raw& w, float fx, float fy, float fz) {
        const f32x4 a = __builtin_bit_cast(f32x4, w.a), b = __builtin_bit_cast(f32x4, w.b);
        // a = (p0, px, py, pz), b = (pxy, pxz, pyz, pxyz)
        const float cx = fmaf(fmaf(b[3], fz, b[0]), fy, fmaf(b[1], fz, a[1]));  // coefficient of fx
        const float c0 = fmaf(fmaf(b[2], fz, a[2]), fy, fmaf(a[3], fz, a[0]));  // value at fx = 0
        return fmaf(cx, fx, c0);
    }
};

// Cell-packed brick-scaled 8-bit codes: cell blocks shifted by one cell so
// each lies inside one brick; 8 codes per cell plus the block's (lo, scale).
template <>
struct Sampler<ST_U8B, LAYOUT_CELLS> {
    struct Raw {
        u32x2 w;
        float2 par;
    };
    template <class VOL>
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, const VOL& vol, const Corners&,
                                               const long long Q[3]) {
        const uint32_t ix = hiword(Q[0]) + 1u, iy = hiword(Q[1]) + 1u, iz = hiword(Q[2]) + 1u;
        const uint32_t blk = __umul24(__umul24(iz >> 1, (uint32_t)vol.nb[1]) + (iy >> 1), (uint32_t)vol.nb[0]) + (ix >> 1);
        const uint32_t w = (ix & 1u) | ((iy & 1u) << 1) | ((iz & 1u) << 2);
        Raw o;
        o.w = struct_load_b64(r, (blk << 3) | w, 0, 0, 0);
        // the codes come through the bounds-checked buffer; the parameters are a
        // plain load, so a request for a position past the grid (the next sample
        // after a ray's last, at a large step) is clamped to the last block
        const uint32_t last = (uint32_t)vol.nb[0] * (uint32_t)vol.nb[1] * (uint32_t)vol.nb[2] - 1u;
        o.par = vol.brick_par[min(blk, last)];
        return o;
    }
    static __device__ __forceinline__ float value(const Raw& o, float fx, float fy, float fz) {
        float c[8];
        CellBits<ST_U8>::unpack(o.w, c);
        return fmaf(o.par.y, trilinear8(c, fx, fy, fz), o.par.x);
    }
};

// Brick-scaled 8-bit codes: the brick owning the (clamped) cell supplies all
// 8 corners and the (lo, scale) that decodes their blend.
template <>
struct Sampler<ST_U8B, LAYOUT_BRICKS> {
    struct Raw {
        float c[8];
        float2 par;
    };
    template <class VOL>
    static __device__ __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, const VOL& vol, const Corners& cn,
                                               const long long Q[3]) {
        const uint32_t ix = hiword(Q[0]), iy = hiword(Q[1]), iz = hiword(Q[2]);
        const int cx = min(max((int)ix - 1, 0), vol.n[0] - 2) >> vol.bshift;
        const int cy = min(max((int)iy - 1, 0), vol.n[1] - 2) >> vol.bshift;
        const int cz = min(max((int)iz - 1, 0), vol.n[2] - 2) >> vol.bshift;
        const uint32_t lx = ix - ((uint32_t)cx << vol.bshift);
        const uint32_t ly = iy - ((uint32_t)cy << vol.bshift);
        const uint32_t lz = iz - ((uint32_t)cz << vol.bshift);
        const uint32_t bid =
            __umul24(__umul24((uint32_t)cz, (uint32_t)vol.nb[1]) + (uint32_t)cy, (uint32_t)vol.nb[0]) + (uint32_t)cx;
        // as for the linear grid: keep every corner (scalar offsets) inside the buffer
        const uint32_t off = min(__umul24(bid, vol.brick_bytes) + __umul24(lz, vol.sz) + __umul24(ly, vol.sy) + lx,
                                 vol.data_bytes - (vol.sz + vol.sy + 2u));
        using E = Elem<ST_U8>;
        Raw w;
        w.c[0] = E::load(r, off, 0);
        w.c[1] = E::load(r, off, cn.c1);
        w.c[2] = E::load(r, off, cn.c2);
        w.c[3] = E::load(r, off, cn.c3);
        w.c[4] = E::load(r, off, cn.c4);
        w.c[5] = E::load(r, off, cn.c5);
        w.c[6] = E::load(r, off, cn.c6);
        w.c[7] = E::load(r, off, cn.c7);
        w.par = vol.brick_par[bid];
        return w;
    }
    static __device__ __forceinline__ float value(const Raw& w, float fx, float fy, float fz) {
        return fmaf(w.par.y, trilinear8(w.c, fx, fy, fz), w.par.x);
    }
};

// Classification: post-classified RGBA by linear interpolation between
// table entries (entry K duplicates entry K-1 so x = K-1 needs no clamp).
__device__ __forceinline__ float4 classify(const float4* __restrict__ s_tf, float val, float ta, float tb,
                                           float Km1) {
    const float x = __builtin_amdgcn_fmed3f(fmaf(val, ta, tb), 0.0f, Km1);
    const uint32_t j0 = (uint32_t)x;
    const float g = __builtin_amdgcn_fractf(x);  // x >= 0: exactly x - j0
    const float4 t0 = s_tf[j0], t1 = s_tf[j0 + 1];
    return make_float4(lerp(t0.x, t1.x, g), lerp(t0.y, t1.y, g), lerp(t0.z, t1.z, g), lerp(t0.w, t1.w, g));
}

// One sample composited front to back (Section 4.2, eq. (4)).  `take` is
// false for a lane whose sample must count as transparent (a stopped ray in
// the ring, a value outside the threshold window).
//
// VOTE: the table's opacity is interpolated first, and colour and
// transmittance are updated only when some lane of the wavefront takes
// opacity.  A sample of opacity 0 leaves both unchanged bit for bit (T * 0 = 0
// is added, fma(-T, 0, T) = T), so skipping the update when no active lane
// has opacity changes nothing; on a typical orbit three of four wavefront
// steps are such, and their colour lerps and compositing are not issued.  The
// batched loop, with many wavefronts per SIMD to cover the latency the branch
// exposes, gains 7 %; the single-view ring and the skipping loop, whose
// unrolled bodies the branch would cut into blocks the scheduler cannot
// interleave, lose 10-25 % with it and keep the branch-free form.
template <bool VOTE>
__device__ __forceinline__ void composite_sample(const float4* __restrict__ s_tf, float val, float ta, float tb,
                                                 float Km1, bool take, float& Cr, float& Cg, float& Cb,
                                                 float& T) {
    const float x = __builtin_amdgcn_fmed3f(fmaf(val, ta, tb), 0.0f, Km1);
    const uint32_t j0 = (uint32_t)x;
    const float g = __builtin_amdgcn_fractf(x);  // x >= 0: exactly x - j0
    const float4 t0 = s_tf[j0], t1 = s_tf[j0 + 1];
    if constexpr (VOTE) {
        const float a = take ? lerp(t0.w, t1.w, g) : 0.0f;
        if (__builtin_amdgcn_ballot_w64(a != 0.0f) != 0) {
            const float Ta = T * a;
            asm volatile("" ::"v"(Ta));  // formed before T is overwritten: no copy of T
            Cr = fmaf(Ta, lerp(t0.x, t1.x, g), Cr);
            Cg = fmaf(Ta, lerp(t0.y, t1.y, g), Cg);
            Cb = fmaf(Ta, lerp(t0.z, t1.z, g), Cb);
            T = fmaf(-T, a, T);
        }
    } else {
        // all four channels interpolated together: both entries are read whole
        const float4 c = make_float4(lerp(t0.x, t1.x, g), lerp(t0.y, t1.y, g), lerp(t0.z, t1.z, g),
                                     lerp(t0.w, t1.w, g));
        const float a = take ? c.w : 0.0f;
        const float Ta = T * a;
        asm volatile("" ::"v"(Ta));
        Cr = fmaf(Ta, c.x, Cr);
        Cg = fmaf(Ta, c.y, Cg);
        Cb = fmaf(Ta, c.z, Cb);
        T = fmaf(-T, a, T);
    }
}

// Step 3: compositing one pixel's ray.  Lanes whose rays have stopped are
// masked off; the wavefront leaves the loop when no lane is left.
// Empty-space skipping.  A skip brick is empty for a table when every entry
// that a sample in it can reach has zero opacity; such samples change neither
// the colour nor the transmittance (T * 0 = 0 and fma(-T, 0, T) = T exactly),
// so stepping over them leaves the result unchanged bit for bit.  The value
// range is widened by 2^-18 of its magnitude (fp32 interpolation error is a
// few units in the last place) and by one table entry on each side.
template <class VD>
__device__ __forceinline__ bool range_is_empty(const VD& V, float2 r) {
    if (!(r.x <= r.y)) return false;  // NaN corners: never skipped
    const float slack = (fabsf(r.x) + fabsf(r.y)) * 0x1p-18f;
    const float Km1 = (float)(V.K - 1);
    const float x0 = __builtin_amdgcn_fmed3f(fmaf(r.x - slack, V.tf_a, V.tf_b), 0.0f, Km1);
    const float x1 = __builtin_amdgcn_fmed3f(fmaf(r.y + slack, V.tf_a, V.tf_b), 0.0f, Km1);
    const int j0 = max((int)x0 - 1, 0), j1 = min((int)x1 + 2, V.K);
    return V.tf_nz[j1 + 1] == V.tf_nz[j0];
}

// One bit per range (empty or not for the view's table) into LDS: one range
// per lane, four per lane in flight, words assembled by ballot.
template <class VD>
__device__ __forceinline__ void build_bits(uint32_t* dst, const float2* ranges, int count, const VD& V) {
    const int words = (count + 31) >> 5;
    const int lane = threadIdx.x & 63, step = (int)blockDim.x;
    for (int base = (int)(threadIdx.x & ~63u); base < count; base += 4 * step) {
        float2 r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = base + u * step + lane;
            r[u] = b < count ? ranges[b] : make_float2(1.0f, 0.0f);  // past the end: not empty
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const unsigned long long m = __builtin_amdgcn_ballot_w64(range_is_empty(V, r[u]));
            const int w = ((base + u * step) >> 5) + (lane >> 5);
            if ((lane & 31) == 0 && w < words) dst[w] = lane ? (uint32_t)(m >> 32) : (uint32_t)m;
        }
    }
}

// The view's skip bricks and super-bricks (4x4x4 skip bricks, with the union
// of their bricks' ranges), one bit each, in LDS.
template <class VD>
__device__ __forceinline__ void build_skip_mask(uint32_t* s_mask, const VD& V) {
    build_bits(s_mask, V.vol.ess_range, V.vol.enb[0] * V.vol.enb[1] * V.vol.enb[2], V);
    build_bits(s_mask + kSkipWords, V.vol.ess_super, V.vol.snb[0] * V.vol.snb[1] * V.vol.snb[2], V);
}

// Is the skip brick of the cell at Q empty?
template <class VOL>
__device__ __forceinline__ bool in_empty_brick(const uint32_t* s_mask, const VOL& vol, const long long Q[3]) {
    const uint32_t es = (uint32_t)vol.eshift;
    const uint32_t b = (hiword(Q[0]) >> es) + __umul24(hiword(Q[1]) >> es, vol.esy) +
                       __umul24(hiword(Q[2]) >> es, vol.esz);
    return (s_mask[b >> 5] >> (b & 31)) & 1u;
}

// A lower bound (at least 1) on the number of consecutive samples, from the
// one at Q on, whose cells lie in Q's block of 2^sh cells per axis.  Per axis
// the exact count is ceil(t) moving up (or not moving) and floor(t) + 1
// moving down, t = distance to the block face in cells over the step in
// cells.  Both are formed in binary32 and pushed down past their rounding
// (an absolute 2^-22 cells and a relative 2^-18), so t is never overstated.
__device__ __forceinline__ int samples_in_block(const long long Q[3], const long long dQ[3], uint32_t sh) {
    float n = 3.0e38f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long d = dQ[a];
        const bool down = d < 0;
        const uint32_t c = hiword(Q[a]);
        const uint32_t face = ((c >> sh) + (down ? 0u : 1u)) << sh;
        const float whole = (float)(down ? c - face : face - c);
        const float dist = fmaf((float)(uint32_t)Q[a], down ? 0x1p-32f : -0x1p-32f, whole);
        const unsigned long long ad = (unsigned long long)(down ? -d : d);
        const float step = fmaf((float)(uint32_t)ad, 0x1p-32f, (float)(uint32_t)(ad >> 32));
        const float t = fmaf(dist, 1.0f - 0x1p-20f, -0x1p-22f) * (__builtin_amdgcn_rcpf(step) * (1.0f - 0x1p-18f));
        n = fminf(n, floorf(t) + (down ? 1.0f : 0.0f));
    }
    return (int)fmaxf(fminf(n, 1.0e9f), 1.0f);
}

// Advance Q past the samples that lie in its (empty) skip brick, or in its
// super-brick when that is empty too; at most `left` samples.  Returns the
// number of samples stepped over.
template <class VOL>
__device__ __forceinline__ int leap(const uint32_t* s_mask, const VOL& vol, long long Q[3], const long long dQ[3],
                                    int left) {
    const uint32_t es = (uint32_t)vol.eshift, sh = es + 2u;
    const uint32_t q = (hiword(Q[0]) >> sh) + __umul24(hiword(Q[1]) >> sh, vol.ssy) + __umul24(hiword(Q[2]) >> sh, vol.ssz);
    const bool super_empty = (s_mask[kSkipWords + (q >> 5)] >> (q & 31)) & 1u;
    const uint32_t n = (uint32_t)min(samples_in_block(Q, dQ, super_empty ? sh : es), left);
#pragma unroll
    for (int a = 0; a < 3; ++a)
        Q[a] = (long long)((unsigned long long)Q[a] + (unsigned long long)n * (unsigned long long)dQ[a]);
    return (int)n;
}

template <class VD>
__device__ __forceinline__ bool in_window(float val, const VD& V) {
    return val >= V.iso_lo && val <= V.iso_hi;
}

// WINDOW: thresholding -- samples whose value lies outside [iso_lo, iso_hi]
// are transparent (their opacity is taken as 0).  COUNT: report the number of
// samples taken (without it the loop keeps no per-ray copy of its counter).
template <int KIND, int LAYOUT, bool SKIP, bool WINDOW, bool COUNT, bool PREFETCH, class VD>
__device__ __forceinline__ void march_pixel(const VD& V, const float4* __restrict__ s_tf,
                                            const uint32_t* __restrict__ s_mask, __amdgpu_buffer_rsrc_t rs,
                                            const Corners& cn, int i, int j, float4& px, int& count) {
    using S = Sampler<KIND, LAYOUT>;
    Ray R;
    float Cr = 0.0f, Cg = 0.0f, Cb = 0.0f, T = 1.0f;
    int k = 0;
    if (setup_ray(V, i, j, R)) {
        const float Km1 = (float)(V.K - 1);
        constexpr float bias = StoredBias<S>::v;
        const float ta = V.tf_a, thr = V.thr;
        float tb = bias != 0.0f ? fmaf(bias, ta, V.tf_b) : V.tf_b;
        asm("" : "+v"(tb));  // held in a vector register: fma(val, ta, tb) may read one scalar only
        // The cell strides and the buffer bound pinned in scalar registers:
        // left to the compiler they are reloaded from the view description in
        // every iteration (a scalar load the next cell request waits for), or
        // kept from the kernel's start and spilled.
        VolDev vol = copy_vol(V.vol);
        asm volatile("" : "+s"(vol.sy), "+s"(vol.sz));
        __amdgpu_buffer_rsrc_t rsp = rs;
        asm volatile("" : "+s"(rsp));
        if (R.m > 0) {
            typename S::Raw cur = S::load(rsp, vol, cn, R.Q);
            // wavefront-uniform: the bricks are looked at every 4th sample and
            // after each leap; a leap leaves `cur` stale (reloaded only when a
            // sample is taken, so a run of leaps never waits on memory)
            int it = 0;
            bool stale = false;
            if constexpr (PREFETCH) {
                // The cells of the next depth samples are in flight while this
                // sample is processed: a ring of registers, unrolled so every
                // buffer keeps its own registers (no copies), each refilled with
                // the cell depth samples ahead once it has been used.  A lone
                // view leaves most SIMDs with few wavefronts, where a sample
                // costs the memory latency unless loads overlap.
                // Qf is the position of sample kf, the next one to request; it
                // stops at the ray's last full sample (m - 1), so every request
                // is for a cell the ray itself samples -- the same cells, with
                // the same bounds, as the loop without a ring.  (A ray that has
                // stopped keeps requesting that last cell.)
                constexpr int depth = ring_depth<S>();
                typename S::Raw ring[depth];
                ring[0] = cur;
                long long Qf[3] = {R.Q[0], R.Q[1], R.Q[2]};
                int kf = 0;
                auto advance_request = [&]() {
                    if (kf < R.m - 1) {
                        ++kf;
#pragma unroll
                        for (int a = 0; a < 3; ++a) Qf[a] += R.dQ[a];
                    }
                };
#pragma unroll
                for (int b = 1; b < depth; ++b) {
                    advance_request();
                    ring[b] = S::load(rsp, vol, cn, Qf);
                }
                // Straight-line steps (no per-ray exit inside the ring): a ray
                // that has stopped keeps stepping with its opacity forced to 0,
                // which leaves its colour and transmittance unchanged bit for
                // bit (T * 0 = 0, fma(-T, 0, T) = T), so every refill is issued
                // unconditionally and each step waits only for its own cell.
                bool live = true;  // k < m and T above the cutoff
                for (;;) {
                    if constexpr (SKIP) {
                        // at the start of each round: when no live ray of the wavefront
                        // sits in an occupied brick, each live ray leaps to its first
                        // sample outside its brick (or super-brick, or to its end); the
                        // ring is refilled only when samples are taken again, so a run of
                        // leaps never waits on memory.  Stopped rays take no part (their
                        // position runs on past their ray and is never looked up).
                        if (V.skip_empty) {
                            bool occupied = false;
                            if (live) occupied = !in_empty_brick(s_mask, V.vol, R.Q);
                            if (__builtin_amdgcn_ballot_w64(occupied) == 0) {
                                if (live) {
                                    k += leap(s_mask, V.vol, R.Q, R.dQ, R.m - k);
                                    live = k < R.m;
                                }
                                if (__builtin_amdgcn_ballot_w64(live) == 0) break;
                                stale = true;
                                continue;
                            }
                            if (stale) {
                                stale = false;
                                if (live) {  // ring[b] = sample k + b, clamped to the ray's last
#pragma unroll
                                    for (int a = 0; a < 3; ++a) Qf[a] = R.Q[a];
                                    kf = k;
                                    ring[0] = S::load(rsp, vol, cn, Qf);
#pragma unroll
                                    for (int b = 1; b < depth; ++b) {
                                        advance_request();
                                        ring[b] = S::load(rsp, vol, cn, Qf);
                                    }
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int b = 0; b < depth; ++b) {
                        const float val = stored_value<S>(ring[b], frac32(R.Q[0]), frac32(R.Q[1]), frac32(R.Q[2]));
                        composite_sample<false>(s_tf, val, ta, tb, Km1,
                                                live && (!WINDOW || in_window(val + bias, V)), Cr, Cg, Cb, T);
                        k += live ? 1 : 0;
                        live = live && k < R.m && T > thr;
                        advance_request();
                        ring[b] = S::load(rsp, vol, cn, Qf);
#pragma unroll
                        for (int q = 0; q < 3; ++q) R.Q[q] += R.dQ[q];
                        // keep the steps in order: interleaving them would make the
                        // first step wait for every cell of the ring
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    if (__builtin_amdgcn_ballot_w64(live) == 0) break;
                }
            }
            if constexpr (!PREFETCH && !SKIP) {
                // Fixed steps in the batched kernel.  The cell of the next
                // sample is requested before the current one is processed, so
                // each load has a whole sample's work to arrive.  Samples go in
                // pairs: the loop body processes sample A (cell wa) and then,
                // unless A stopped the ray, sample B (cell wb), with one exit
                // test per pair; an odd count starts with one sample alone.  With
                // no exit between A and B, every register keeps one role and the
                // loop carries its state without copies.  The request after a
                // ray's last sample reads a cell one step past it, through the
                // same bounded reads as every other cell, and is never used.
                // Scheduling barriers keep each request where it is written (left
                // to the scheduler, the request for sample B sank below sample A's
                // work and B waited for its whole latency).
                long long P[3] = {R.Q[0], R.Q[1], R.Q[2]};
                typename S::Raw wa = cur, wb;
                int r = R.m;  // full samples not yet composited
                bool go = true;
                auto composite = [&](const typename S::Raw& w, const long long* at) {
                    const float val = stored_value<S>(w, frac32(at[0]), frac32(at[1]), frac32(at[2]));
                    composite_sample<true>(s_tf, val, ta, tb, Km1, !WINDOW || in_window(val + bias, V), Cr, Cg, Cb, T);
                };
                if (r & 1) {
                    long long Pn[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) Pn[q] = P[q] + R.dQ[q];
                    wb = S::load(rsp, vol, cn, Pn);
                    composite(wa, P);
                    r -= 1;
                    go = r > 0 && T > thr;
#pragma unroll
                    for (int q = 0; q < 3; ++q) P[q] = Pn[q];
                    wa = wb;
                }
                bool liveA = true;
                if (go) {
                    for (;;) {
                        // each position passes through an empty asm: the loop
                        // then keeps one 64-bit induction variable per axis
                        // (left alone, strength reduction split some layouts'
                        // positions into a base and an offset, adding several
                        // adds per sample)
                        long long P1[3];
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            P1[q] = P[q] + R.dQ[q];
                            asm("" : "+v"(P1[q]));
                        }
                        wb = S::load(rsp, vol, cn, P1);
                        __builtin_amdgcn_sched_barrier(0);
                        composite(wa, P);
                        liveA = T > thr;  // r >= 2 here: sample B exists
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            P[q] = P1[q] + R.dQ[q];
                            asm("" : "+v"(P[q]));
                        }
                        wa = S::load(rsp, vol, cn, P);
                        __builtin_amdgcn_sched_barrier(0);
                        if (liveA) composite(wb, P1);
                        r -= 2;
                        if (!(liveA && r > 0 && T > thr)) break;
                    }
                }
                k = R.m - r - (liveA ? 0 : 1);
            }
            for (; !PREFETCH && SKIP;) {
                if constexpr (SKIP) {
                    // all live rays of the wavefront in empty bricks: each leaps to
                    // its first sample outside its brick (or to the end of its ray)
                    if (V.skip_empty && (it++ & 3) == 0 &&
                        __builtin_amdgcn_ballot_w64(!in_empty_brick(s_mask, V.vol, R.Q)) == 0) {
                        it = 0;
                        k += leap(s_mask, V.vol, R.Q, R.dQ, R.m - k);
                        if (k >= R.m) break;
                        stale = true;
                        continue;
                    }
                    if (stale) {
                        cur = S::load(rsp, vol, cn, R.Q);
                        stale = false;
                    }
                }
                const float val = stored_value<S>(cur, frac32(R.Q[0]), frac32(R.Q[1]), frac32(R.Q[2]));
                composite_sample<false>(s_tf, val, ta, tb, Km1, !WINDOW || in_window(val + bias, V), Cr, Cg, Cb, T);
                ++k;
                if (k >= R.m || T <= thr) break;
                R.Q[0] += R.dQ[0];
                R.Q[1] += R.dQ[1];
                R.Q[2] += R.dQ[2];
                cur = S::load(rsp, vol, cn, R.Q);
            }
        }
        if (R.wp > 0.0f && T > thr) {
            const typename S::Raw w = S::load(rsp, vol, cn, R.Qp);
            const float val = stored_value<S>(w, frac32(R.Qp[0]), frac32(R.Qp[1]), frac32(R.Qp[2]));
            float4 c = classify(s_tf, val, ta, tb, Km1);
            if (WINDOW && !in_window(val + bias, V)) c.w = 0.0f;
            const float a = 1.0f - exp2f(R.wp * log2f(1.0f - c.w));
            const float Ta = T * a;
            Cr = fmaf(Ta, c.x, Cr);
            Cg = fmaf(Ta, c.y, Cg);
            Cb = fmaf(Ta, c.z, Cb);
            T = fmaf(-T, a, T);
            if constexpr (COUNT) ++k;
        }
    }
    px = make_float4(fmaf(T, V.bg[0], Cr), fmaf(T, V.bg[1], Cg), fmaf(T, V.bg[2], Cb), fmaf(T, V.bg[3], 1.0f - T));
    count = COUNT ? k : 0;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Stage the table in LDS.  alpha_exp > 0: opacity correction to the sample
// spacing, a' = 1 - (1 - a)^alpha_exp per entry (a = 0 stays exactly 0 and a = 1
// stays 1, so empty-space skipping's opacity counts still hold).
// Eight entries per lane are requested before any is stored, so a small
// workgroup (one wavefront staging 4097 entries) waits for memory 8 times, not 64.
__device__ __forceinline__ void load_tf(float4* s_tf, const float4* __restrict__ tf, int K, float alpha_exp) {
    constexpr int U = 8;
    const int step = (int)blockDim.x;
    for (int e0 = threadIdx.x; e0 <= K; e0 += U * step) {
        float4 t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = tf[min(e0 + u * step, K - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * step;
            if (e <= K) {
                if (alpha_exp > 0.0f) t[u].w = 1.0f - exp2f(alpha_exp * log2f(1.0f - t[u].w));
                s_tf[e] = t[u];
            }
        }
    }
}

// One workgroup block of a view: wave w renders tile (w % bw, w / bw) of the block.
// Step 3 for the projection ray functions: every sample of the lattice is
// visited (no early termination) and reduced to one scalar: the maximum, or
// the weighted sum (X-ray: times dt; average: over the summed weights).  The
// sum is compensated (Kahan), so its rounding error stays at a few units of
// the last place whatever the ray length.  The scalar is classified once and
// laid over the background with the table's opacity.
enum { RF_MAX = 0, RF_SUM = 1 };

template <int KIND, int LAYOUT, int RED, class VD>
__device__ __forceinline__ void project_pixel(const VD& V, const float4* __restrict__ s_tf,
                                              __amdgpu_buffer_rsrc_t rs, const Corners& cn, int i, int j,
                                              float4& px, int& count) {
    using S = Sampler<KIND, LAYOUT>;
    Ray R;
    float acc = RED == RF_MAX ? -INFINITY : 0.0f, comp = 0.0f;
    int k = 0;
    px = make_float4(V.bg[0], V.bg[1], V.bg[2], V.bg[3]);
    if (!setup_ray(V, i, j, R)) {
        count = 0;
        return;
    }
    if (R.m > 0) {
        VolDev vol = copy_vol(V.vol);  // strides and bound pinned, as in march_pixel
        asm volatile("" : "+s"(vol.sy), "+s"(vol.sz));
        __amdgpu_buffer_rsrc_t rsp = rs;
        asm volatile("" : "+s"(rsp));
        typename S::Raw cur = S::load(rsp, vol, cn, R.Q);
        for (;;) {
            const long long Qn[3] = {R.Q[0] + R.dQ[0], R.Q[1] + R.dQ[1], R.Q[2] + R.dQ[2]};
            const typename S::Raw nxt = S::load(rsp, vol, cn, Qn);
            const float val = S::value(cur, frac32(R.Q[0]), frac32(R.Q[1]), frac32(R.Q[2]));
            if (RED == RF_MAX) {
                acc = fmaxf(acc, val);
            } else {
                const float y = val - comp, t = acc + y;
                comp = (t - acc) - y;
                acc = t;
            }
            if (++k >= R.m) break;
            cur = nxt;
            R.Q[0] = Qn[0];
            R.Q[1] = Qn[1];
            R.Q[2] = Qn[2];
        }
    }
    if (R.wp > 0.0f) {
        const typename S::Raw w = S::load(rs, V.vol, cn, R.Qp);
        const float val = S::value(w, frac32(R.Qp[0]), frac32(R.Qp[1]), frac32(R.Qp[2]));
        if (RED == RF_MAX) {
            acc = fmaxf(acc, val);
        } else {
            const float y = val * R.wp - comp, t = acc + y;
            acc = t;
        }
        ++k;
    }
    count = k;
    float scalar = acc;
    if (RED == RF_SUM)
        scalar = V.ray_function == RT_FN_XRAY ? acc * V.dt.hi : acc / ((float)R.m + R.wp);
    const float4 c = classify(s_tf, scalar, V.tf_a, V.tf_b, (float)(V.K - 1));
    const float ia = 1.0f - c.w;
    px = make_float4(fmaf(c.w, c.x, ia * V.bg[0]), fmaf(c.w, c.y, ia * V.bg[1]), fmaf(c.w, c.z, ia * V.bg[2]),
                     fmaf(ia, V.bg[3], c.w));
}

// Step 3 for the iso-surface: the first lattice sample whose value reaches
// the iso-value is the hit; the hit point is refined linearly from the sample
// before (unless it is the first); the surface normal is the descent
// direction of the trilinear field from central differences over +-1/2 cell
// per axis, and the opaque surface is shaded by a headlight,
// c * (0.2 + 0.8 |n.d|), c the table colour at the iso-value.
template <int KIND, int LAYOUT, class VD>
__device__ __forceinline__ void iso_pixel(const VD& V, const float4* __restrict__ s_tf, __amdgpu_buffer_rsrc_t rs,
                                          const Corners& cn, int i, int j, float4& px, int& count) {
    using S = Sampler<KIND, LAYOUT>;
    Ray R;
    px = make_float4(V.bg[0], V.bg[1], V.bg[2], V.bg[3]);
    count = 0;
    if (!setup_ray(V, i, j, R)) return;
    const float iso = V.iso_lo;
    bool hit = false, refine = false;
    float v_prev = 0.0f, v_hit = 0.0f;
    int k = 0;
    long long P1[3] = {R.Q[0], R.Q[1], R.Q[2]};  // hit sample
    long long P0[3] = {0, 0, 0};                 // the sample before it
    if (R.m > 0) {
        VolDev vol = copy_vol(V.vol);  // strides and bound pinned, as in march_pixel
        asm volatile("" : "+s"(vol.sy), "+s"(vol.sz));
        __amdgpu_buffer_rsrc_t rsp = rs;
        asm volatile("" : "+s"(rsp));
        typename S::Raw cur = S::load(rsp, vol, cn, R.Q);
        for (;;) {
            const long long Qn[3] = {R.Q[0] + R.dQ[0], R.Q[1] + R.dQ[1], R.Q[2] + R.dQ[2]};
            const typename S::Raw nxt = S::load(rsp, vol, cn, Qn);
            const float val = S::value(cur, frac32(R.Q[0]), frac32(R.Q[1]), frac32(R.Q[2]));
            if (val >= iso) {
                hit = true;
                v_hit = val;
                break;
            }
            v_prev = val;
            if (++k >= R.m) break;
            cur = nxt;
            R.Q[0] = Qn[0];
            R.Q[1] = Qn[1];
            R.Q[2] = Qn[2];
        }
        // hit: sample k at R.Q; otherwise k == m and R.Q is the last full sample
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            P1[a] = R.Q[a];
            P0[a] = R.Q[a] - R.dQ[a];
        }
        refine = hit && k > 0;
    }
    if (!hit && R.wp > 0.0f) {
        const typename S::Raw w = S::load(rs, V.vol, cn, R.Qp);
        const float val = S::value(w, frac32(R.Qp[0]), frac32(R.Qp[1]), frac32(R.Qp[2]));
        if (val >= iso) {
            hit = true;
            v_hit = val;
            refine = R.m > 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                P0[a] = R.Q[a];
                P1[a] = R.Qp[a];
            }
        }
        k = R.m;
    }
    if (!hit) {
        count = R.m + (R.wp > 0.0f ? 1 : 0);
        return;
    }
    count = k + 1;
    long long P[3] = {P1[0], P1[1], P1[2]};
    if (refine) {
        const float lam = (iso - v_prev) / (v_hit - v_prev);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const long long D = P1[a] - P0[a];
            P[a] = P0[a] + (long long)rintf(lam * (float)D);
        }
    }
    // central differences over +-1/2 cell (2^31 in 32.32 fixed point) per axis
    float df[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        long long Pp[3] = {P[0], P[1], P[2]}, Pm[3] = {P[0], P[1], P[2]};
        Pp[a] += 0x80000000LL;
        Pm[a] -= 0x80000000LL;
        const float fp = S::value(S::load(rs, V.vol, cn, Pp), frac32(Pp[0]), frac32(Pp[1]), frac32(Pp[2]));
        const float fm = S::value(S::load(rs, V.vol, cn, Pm), frac32(Pm[0]), frac32(Pm[1]), frac32(Pm[2]));
        df[a] = fp - fm;
    }
    // n.d with g_a = df_a / s_a and d_a proportional to dQ_a * s_a: the spacing cancels in g.d
    float gd = 0.0f, gg = 0.0f, dd = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float isp = V.inv_sp[a].hi, dq = (float)R.dQ[a];
        gd = fmaf(df[a], dq, gd);
        gg = fmaf(df[a] * isp, df[a] * isp, gg);
        dd = fmaf(dq / isp, dq / isp, dd);
    }
    const float cosang = gg > 0.0f ? fabsf(gd) * __frsqrt_rn(gg) * __frsqrt_rn(dd) : 1.0f;
    const float4 c = classify(s_tf, iso, V.tf_a, V.tf_b, (float)(V.K - 1));
    const float shade = fmaf(0.8f, cosang, 0.2f);
    px = make_float4(c.x * shade, c.y * shade, c.z * shade, 1.0f);
}

// PREFETCH: the compositing loop requests the next cell before processing the
// current sample (the single-view kernel; see march_pixel).  COMP_ONLY: the
// view is known to composite, so only that path is compiled (the single-view
// kernel of a compositing view: one ray function keeps its view parameters out
// of spilled scalar registers).
template <int KIND, int LAYOUT, bool SKIP, bool PREFETCH, class VD, bool COMP_ONLY = false>
__device__ __forceinline__ void render_block(const VD& V, const float4* __restrict__ s_tf,
                                             const uint32_t* __restrict__ s_mask, int blk, const LaunchShape& ls,
                                             int tw_shift, unsigned long long* __restrict__ counter) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int tx, ty;
    if (ls.order == 0) {  // compact: the workgroup's tiles form a bw x bh block
        const int by = blk / V.blocks_x, bx = blk - by * V.blocks_x;
        tx = bx * ls.bw + wave % ls.bw;
        ty = by * ls.bh + wave / ls.bw;
        if (tx >= V.tiles_x || ty >= V.tiles_y) return;
    } else {  // spread: tile blk + nblocks * wave in row-major tile order
        const int t = blk + V.nblocks * wave;
        if (t >= V.tiles_x * V.tiles_y) return;
        ty = t / V.tiles_x;
        tx = t - ty * V.tiles_x;
    }
    const int i = tx * ls.tile_w + (lane & (ls.tile_w - 1)), j = ty * ls.tile_h + (lane >> tw_shift);
    const __amdgpu_buffer_rsrc_t rs = make_vol_rsrc<KIND, LAYOUT>(V.vol.data, V.vol.data_bytes);
    const Corners cn = corners_of(LAYOUT == LAYOUT_BRICKS ? 1u : Elem<KIND>::bytes, V.vol.sy, V.vol.sz);
    int count = 0;
    if (i < V.W && j < V.H) {
        float4 px;
        const int fn = V.ray_function;  // uniform over the view
        // the skipping loop keeps a per-ray counter anyway (leaps differ per ray)
        const bool want_count = SKIP || V.counts != nullptr || counter != nullptr;
        if (COMP_ONLY || fn == RT_FN_COMPOSITE) {
            if (want_count)
                march_pixel<KIND, LAYOUT, SKIP, false, true, PREFETCH, VD>(V, s_tf, s_mask, rs, cn, i, j, px, count);
            else
                march_pixel<KIND, LAYOUT, SKIP, false, SKIP, PREFETCH, VD>(V, s_tf, s_mask, rs, cn, i, j, px, count);
        } else if (fn == RT_FN_THRESHOLD) {
            march_pixel<KIND, LAYOUT, SKIP, true, true, PREFETCH, VD>(V, s_tf, s_mask, rs, cn, i, j, px, count);
        }
        else if (fn == RT_FN_ISO)
            iso_pixel<KIND, LAYOUT, VD>(V, s_tf, rs, cn, i, j, px, count);
        else if (fn == RT_FN_MIP)
            project_pixel<KIND, LAYOUT, RF_MAX, VD>(V, s_tf, rs, cn, i, j, px, count);
        else
            project_pixel<KIND, LAYOUT, RF_SUM, VD>(V, s_tf, rs, cn, i, j, px, count);
        const size_t p = (size_t)j * V.W + i;
        reinterpret_cast<float4*>(V.out)[p] = px;
        if (V.counts) V.counts[p] = count;
    }
    if (counter) {
        const int tot = wave_sum(count);
        if (lane == 0 && tot) atomicAdd(counter, (unsigned long long)tot);
    }
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of blocks (a compact band of the image) for L2 locality.
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int x = b & 7, idx = b >> 3;
    const int per = n >> 3, rem = n & 7;
    return x * per + min(x, rem) + idx;
}

// Occupancy of the batched kernels.  Fixed-step marching: 12-wavefront
// workgroups, two per CU (6 waves per SIMD, up to 80 VGPRs), which leaves the
// registers to keep the next sample's cell in flight while the current one is
// processed.  With empty-space skipping: 16-wavefront workgroups, two per CU
// (8 waves per SIMD, 64 VGPRs).  Either way two workgroups share a CU's LDS.
#define RT_BATCH_ATTRS __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(6)))
#define RT_BATCH_SKIP_ATTRS __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
// The single-view kernel: one view of up to a few thousand wavefronts never
// fills 8 per SIMD, so it may use the registers of 4 (its loads in flight).
#define RT_PLAIN_ATTRS __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4)))

// SKIP selects the compositing loop with empty-space skipping (a separate
// kernel, so the plain loop keeps its registers).
template <int KIND, int LAYOUT, bool SKIP, bool COMP_ONLY>
__global__ void RT_PLAIN_ATTRS march_plain_kernel(const ViewDesc V, const LaunchShape ls, int tw_shift,
                                                   unsigned long long* __restrict__ counter) {
    extern __shared__ float4 s_tf[];
    uint32_t* s_mask = reinterpret_cast<uint32_t*>(s_tf + V.K + 1);
    load_tf(s_tf, V.tf, V.K, V.alpha_exp);
    if (SKIP) build_skip_mask(s_mask, V);
    __syncthreads();
    render_block<KIND, LAYOUT, SKIP, true, ViewDesc, COMP_ONLY>(V, s_tf, s_mask, xcd_remap(blockIdx.x, gridDim.x), ls,
                                                               tw_shift,
                                               counter);
}

// Persistent batched marcher: workgroups claim blocks from a queue in the
// workspace until it runs dry; the view of a block is found by binary search
// over the per-view block prefix.  The transfer function in LDS is reloaded
// only when the claimed view uses a different table.
// The job table, block prefix and header do not change while a batch kernel
// runs (only the queue word is written, and never read through these
// pointers), so they are read through the constant address space: scalar
// loads, and descriptors the compiler knows to be wave-uniform.
typedef __attribute__((address_space(4))) const ViewDesc CViewDesc;
typedef __attribute__((address_space(4))) const int CInt;
typedef __attribute__((address_space(4))) const BatchHeader CBatchHeader;

template <int KIND, int LAYOUT, bool SKIP>
__device__ __forceinline__ void batch_body(char* __restrict__ ws, const LaunchShape& ls, int tw_shift,
                                           int tf_entries) {
    extern __shared__ float4 s_tf[];
    uint32_t* s_mask = reinterpret_cast<uint32_t*>(s_tf + tf_entries);
    int* s_claim = reinterpret_cast<int*>(s_mask + kSkipMaskBytes / 4);
    unsigned int* queue = &reinterpret_cast<BatchHeader*>(ws)->queue;
    const CBatchHeader* hdr = (const CBatchHeader*)(ws);
    const CInt* prefix = (const CInt*)(ws + kBatchHeaderBytes);
    const CViewDesc* jobs = (const CViewDesc*)(ws + kBatchHeaderBytes + kBatchPrefixBytes);
    const int n_jobs = (int)hdr->n_jobs;
    unsigned long long* counter = hdr->counter;
    const int total = prefix[n_jobs];
    // the table in LDS and the (volume, table) pair the mask was built for live
    // in LDS, not in scalar registers that would stay live across the marcher
    __shared__ const void* s_have[3];
    __shared__ float s_have_exp;  // the opacity correction of the staged table
    if (threadIdx.x == 0) {
        s_have[0] = s_have[1] = s_have[2] = nullptr;
        s_have_exp = 0.0f;
    }
    for (;;) {
        if (threadIdx.x == 0) s_claim[0] = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int g = __builtin_amdgcn_readfirstlane(s_claim[0]);
        if (g >= total) break;
        int lo = 0, hi = n_jobs;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (prefix[mid] <= g) lo = mid;
            else hi = mid;
        }
        const CViewDesc& V = jobs[lo];
        const bool new_tf = (const void*)V.tf != s_have[0] || V.alpha_exp != s_have_exp;
        const bool new_mask = SKIP && V.skip_empty && ((const void*)V.vol.ess_range != s_have[1] ||
                                                       (const void*)V.tf != s_have[2]);
        if (new_tf || new_mask) {
            __syncthreads();  // every lane has read s_have
            if (new_tf) load_tf(s_tf, V.tf, V.K, V.alpha_exp);
            if (new_mask) build_skip_mask(s_mask, V);
            if (threadIdx.x == 0) {
                s_have[0] = V.tf;
                s_have_exp = V.alpha_exp;
                if (new_mask) {
                    s_have[1] = V.vol.ess_range;
                    s_have[2] = V.tf;
                }
            }
            __syncthreads();
        }
        render_block<KIND, LAYOUT, SKIP, false, CViewDesc>(V, s_tf, s_mask, g - prefix[lo], ls, tw_shift, counter);
        __syncthreads();
    }
}

template <int KIND, int LAYOUT>
__global__ void RT_BATCH_ATTRS march_batch_kernel(char* __restrict__ ws, const LaunchShape ls, int tw_shift,
                                                  int tf_entries) {
    batch_body<KIND, LAYOUT, false>(ws, ls, tw_shift, tf_entries);
}

template <int KIND, int LAYOUT>
__global__ void RT_BATCH_SKIP_ATTRS march_batch_skip_kernel(char* __restrict__ ws, const LaunchShape ls,
                                                            int tw_shift, int tf_entries) {
    batch_body<KIND, LAYOUT, true>(ws, ls, tw_shift, tf_entries);
}

// Latency form of the batched launch: one workgroup per block of tiles, no
// queue, with the single-view kernel's occupancy and cell ring.  A batch
// smaller than the GPU then spreads over every compute unit in workgroups
// sized to it, as a lone view does, instead of filling a few 16-wavefront
// workgroups of the persistent kernel.  Each workgroup stages its own view's
// table (and skip mask) and renders one block.
template <int KIND, int LAYOUT, bool SKIP>
__global__ void RT_PLAIN_ATTRS march_views_kernel(char* __restrict__ ws, const LaunchShape ls, int tw_shift) {
    extern __shared__ float4 s_tf[];
    const CBatchHeader* hdr = (const CBatchHeader*)(ws);
    const CInt* prefix = (const CInt*)(ws + kBatchHeaderBytes);
    const CViewDesc* jobs = (const CViewDesc*)(ws + kBatchHeaderBytes + kBatchPrefixBytes);
    const int n_jobs = (int)hdr->n_jobs;
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid;
    }
    const CViewDesc& V = jobs[lo];
    uint32_t* s_mask = reinterpret_cast<uint32_t*>(s_tf + hdr->tf_lds_entries);
    load_tf(s_tf, V.tf, V.K, V.alpha_exp);
    if (SKIP && V.skip_empty) build_skip_mask(s_mask, V);
    __syncthreads();
    render_block<KIND, LAYOUT, SKIP, true, CViewDesc>(V, s_tf, s_mask, g - prefix[lo], ls, tw_shift, hdr->counter);
}

// The same for a batch carried in the kernel arguments.  The batch is the
// first argument, at offset 0 of the kernel-argument segment, and is read
// through that segment's constant address: scalar loads of the view at its
// index, as from the workspace (indexing the by-value argument itself would
// copy it to private memory).
typedef __attribute__((address_space(4))) const SmallBatch CSmallBatch;
template <int KIND, int LAYOUT, bool SKIP>
__global__ void RT_PLAIN_ATTRS march_views_args_kernel(const SmallBatch B, const LaunchShape ls, int tw_shift) {
    extern __shared__ float4 s_tf[];
    (void)B;
    const CSmallBatch* b = (const CSmallBatch*)__builtin_amdgcn_kernarg_segment_ptr();
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    const int n = b->n;
    int lo = 0;
#pragma unroll
    for (int i = 1; i < kSmallBatchJobs; ++i) lo += (i < n && b->prefix[i] <= g) ? 1 : 0;
    const CViewDesc& V = b->v[lo];
    uint32_t* s_mask = reinterpret_cast<uint32_t*>(s_tf + b->tf_lds_entries);
    load_tf(s_tf, V.tf, V.K, V.alpha_exp);
    if (SKIP && V.skip_empty) build_skip_mask(s_mask, V);
    __syncthreads();
    render_block<KIND, LAYOUT, SKIP, true, CViewDesc>(V, s_tf, s_mask, g - b->prefix[lo], ls, tw_shift, b->counter);
}

// Value range of every skip brick, one workgroup per brick: each of its
// padded cells is sampled by the marcher's own sampler at the cell's 8
// corners, so the range bounds what a sample in the brick can read (up to
// the rounding of the interpolation, which the emptiness test allows for).
template <int KIND, int LAYOUT>
__global__ void __launch_bounds__(256) skip_range_kernel(const VolDev vol) {
    using S = Sampler<KIND, LAYOUT>;
    __shared__ float s_lo[256], s_hi[256];
    const int b = blockIdx.x;
    const int bx = b % vol.enb[0], by = (b / vol.enb[0]) % vol.enb[1], bz = b / (vol.enb[0] * vol.enb[1]);
    const int E = 1 << vol.eshift;
    const int x0 = bx * E, y0 = by * E, z0 = bz * E;
    const int ex = min(E, vol.n[0] + 1 - x0), ey = min(E, vol.n[1] + 1 - y0), ez = min(E, vol.n[2] + 1 - z0);
    const __amdgpu_buffer_rsrc_t rs = make_vol_rsrc<KIND, LAYOUT>(vol.data, vol.data_bytes);
    const Corners cn = corners_of(LAYOUT == LAYOUT_BRICKS ? 1u : Elem<KIND>::bytes, vol.sy, vol.sz);
    float lo = INFINITY, hi = -INFINITY;
    int nan = 0;
    for (int c = threadIdx.x; c < ex * ey * ez; c += blockDim.x) {
        const long long Q[3] = {(long long)(x0 + c % ex) << 32, (long long)(y0 + (c / ex) % ey) << 32,
                                (long long)(z0 + c / (ex * ey)) << 32};
        const typename S::Raw raw = S::load(rs, vol, cn, Q);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float v = S::value(raw, (float)(k & 1), (float)((k >> 1) & 1), (float)(k >> 2));
            nan |= v != v;
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
    }
    nan = __syncthreads_or(nan);
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            s_lo[threadIdx.x] = fminf(s_lo[threadIdx.x], s_lo[threadIdx.x + st]);
            s_hi[threadIdx.x] = fmaxf(s_hi[threadIdx.x], s_hi[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        const_cast<float2*>(vol.ess_range)[b] = nan ? make_float2(NAN, NAN) : make_float2(s_lo[0], s_hi[0]);
}

// Super-brick ranges: the union of the ranges of its (up to 64) skip bricks,
// NaN when any of them is NaN.
__global__ void __launch_bounds__(256) super_range_kernel(const VolDev vol) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= vol.snb[0] * vol.snb[1] * vol.snb[2]) return;
    const int qx = q % vol.snb[0], qy = (q / vol.snb[0]) % vol.snb[1], qz = q / (vol.snb[0] * vol.snb[1]);
    float lo = INFINITY, hi = -INFINITY;
    bool nan = false;
    for (int bz = 4 * qz; bz < min(4 * qz + 4, vol.enb[2]); ++bz)
        for (int by = 4 * qy; by < min(4 * qy + 4, vol.enb[1]); ++by)
            for (int bx = 4 * qx; bx < min(4 * qx + 4, vol.enb[0]); ++bx) {
                const float2 r = vol.ess_range[bx + vol.enb[0] * (by + vol.enb[1] * bz)];
                nan = nan || !(r.x <= r.y);
                lo = fminf(lo, r.x);
                hi = fmaxf(hi, r.y);
            }
    const_cast<float2*>(vol.ess_super)[q] = nan ? make_float2(NAN, NAN) : make_float2(lo, hi);
}

template <int KIND, int LAYOUT>
hipError_t skip_range_launch(const VolDev& vol, hipStream_t s) {
    const int nb = vol.enb[0] * vol.enb[1] * vol.enb[2];
    hipLaunchKernelGGL((skip_range_kernel<KIND, LAYOUT>), dim3(nb), dim3(256), 0, s, vol);
    const int ns = vol.snb[0] * vol.snb[1] * vol.snb[2];
    hipLaunchKernelGGL(super_range_kernel, dim3((ns + 255) / 256), dim3(256), 0, s, vol);
    return hipGetLastError();
}

int log2i(int x) {
    int s = 0;
    while ((1 << s) < x) ++s;
    return s;
}

template <int KIND, int LAYOUT, bool SKIP, bool COMP_ONLY>
hipError_t plain_launch_k(const ViewDesc& v, const LaunchShape& ls, unsigned long long* counter, hipStream_t s) {
    const int nblk = v.nblocks;
    if (nblk <= 0) return hipSuccess;
    const size_t lds = (size_t)(v.K + 1) * sizeof(float4) + (v.skip_empty ? (size_t)kSkipMaskBytes : 0);
    // once per kernel, thread-safe (function-local static initialisation)
    static const hipError_t attr =
        hipFuncSetAttribute((const void*)march_plain_kernel<KIND, LAYOUT, SKIP, COMP_ONLY>,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)((kMaxK + 1) * sizeof(float4) + kSkipMaskBytes));
    (void)attr;
    hipLaunchKernelGGL((march_plain_kernel<KIND, LAYOUT, SKIP, COMP_ONLY>), dim3(nblk), dim3(64 * ls.waves), lds, s,
                       v, ls, log2i(ls.tile_w), counter);
    return hipGetLastError();
}

template <int KIND, int LAYOUT>
hipError_t plain_launch(const ViewDesc& v, const LaunchShape& ls, unsigned long long* counter, hipStream_t s) {
    const bool comp = v.ray_function == RT_FN_COMPOSITE;
    if (v.skip_empty)
        return comp ? plain_launch_k<KIND, LAYOUT, true, true>(v, ls, counter, s)
                    : plain_launch_k<KIND, LAYOUT, true, false>(v, ls, counter, s);
    return comp ? plain_launch_k<KIND, LAYOUT, false, true>(v, ls, counter, s)
                : plain_launch_k<KIND, LAYOUT, false, false>(v, ls, counter, s);
}

template <int KIND, int LAYOUT, bool SKIP>
hipError_t batch_launch_k(void* ws, int grid, const LaunchShape& ls, int max_k, hipStream_t s) {
    const int tf_entries = max_k + 1;
    const size_t lds = (size_t)tf_entries * sizeof(float4) + kSkipMaskBytes + 16;
    const void* fn = SKIP ? (const void*)march_batch_skip_kernel<KIND, LAYOUT>
                          : (const void*)march_batch_kernel<KIND, LAYOUT>;
    static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)((kMaxK + 1) * sizeof(float4) + kSkipMaskBytes + 16));
    (void)attr;
    if (ls.waves > (SKIP ? 16 : 12)) return hipErrorInvalidConfiguration;  // the shape checks refuse this first
    if constexpr (SKIP)
        hipLaunchKernelGGL((march_batch_skip_kernel<KIND, LAYOUT>), dim3(grid), dim3(64 * ls.waves), lds, s,
                           static_cast<char*>(ws), ls, log2i(ls.tile_w), tf_entries);
    else
        hipLaunchKernelGGL((march_batch_kernel<KIND, LAYOUT>), dim3(grid), dim3(64 * ls.waves), lds, s,
                           static_cast<char*>(ws), ls, log2i(ls.tile_w), tf_entries);
    return hipGetLastError();
}

template <int KIND, int LAYOUT>
hipError_t batch_launch(void* ws, int grid, const LaunchShape& ls, int max_k, bool skip, hipStream_t s) {
    return skip ? batch_launch_k<KIND, LAYOUT, true>(ws, grid, ls, max_k, s)
                : batch_launch_k<KIND, LAYOUT, false>(ws, grid, ls, max_k, s);
}

template <int KIND, int LAYOUT, bool SKIP>
hipError_t views_launch_k(void* ws, int blocks, const LaunchShape& ls, int max_k, hipStream_t s) {
    const size_t lds = (size_t)(max_k + 1) * sizeof(float4) + (SKIP ? (size_t)kSkipMaskBytes : 0);
    static const hipError_t attr =
        hipFuncSetAttribute((const void*)march_views_kernel<KIND, LAYOUT, SKIP>,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)((kMaxK + 1) * sizeof(float4) + kSkipMaskBytes));
    (void)attr;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((march_views_kernel<KIND, LAYOUT, SKIP>), dim3(blocks), dim3(64 * ls.waves), lds, s,
                       static_cast<char*>(ws), ls, log2i(ls.tile_w));
    return hipGetLastError();
}

template <int KIND, int LAYOUT>
hipError_t views_launch(void* ws, int blocks, const LaunchShape& ls, int max_k, bool skip, hipStream_t s) {
    return skip ? views_launch_k<KIND, LAYOUT, true>(ws, blocks, ls, max_k, s)
                : views_launch_k<KIND, LAYOUT, false>(ws, blocks, ls, max_k, s);
}

template <int KIND, int LAYOUT, bool SKIP>
hipError_t views_args_launch_k(const SmallBatch& b, const LaunchShape& ls, hipStream_t s) {
    const size_t lds = (size_t)b.tf_lds_entries * sizeof(float4) + (SKIP ? (size_t)kSkipMaskBytes : 0);
    static const hipError_t attr =
        hipFuncSetAttribute((const void*)march_views_args_kernel<KIND, LAYOUT, SKIP>,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)((kMaxK + 1) * sizeof(float4) + kSkipMaskBytes));
    (void)attr;
    const int blocks = b.prefix[b.n];
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((march_views_args_kernel<KIND, LAYOUT, SKIP>), dim3(blocks), dim3(64 * ls.waves), lds, s, b,
                       ls, log2i(ls.tile_w));
    return hipGetLastError();
}

template <int KIND, int LAYOUT>
hipError_t views_args_launch(const SmallBatch& b, const LaunchShape& ls, bool skip, hipStream_t s) {
    return skip ? views_args_launch_k<KIND, LAYOUT, true>(b, ls, s) : views_args_launch_k<KIND, LAYOUT, false>(b, ls, s);
}

}  // namespace

hipError_t launch_march_plain(const ViewDesc& v, const LaunchShape& ls, unsigned long long* counter,
                              hipStream_t s) {
    const int L = v.vol.layout;
    switch (v.vol.kind) {
        case ST_U8:
            return L == LAYOUT_CELLS  ? plain_launch<ST_U8, LAYOUT_CELLS>(v, ls, counter, s)
                   : L == LAYOUT_POLY ? plain_launch<ST_U8, LAYOUT_POLY>(v, ls, counter, s)
                                      : plain_launch<ST_U8, LAYOUT_LINEAR>(v, ls, counter, s);
        case ST_U16:
            return L == LAYOUT_CELLS    ? plain_launch<ST_U16, LAYOUT_CELLS>(v, ls, counter, s)
                   : L == LAYOUT_POLY   ? plain_launch<ST_U16, LAYOUT_POLY>(v, ls, counter, s)
                   : L == LAYOUT_QUADS ? plain_launch<ST_U16, LAYOUT_QUADS>(v, ls, counter, s)
                                        : plain_launch<ST_U16, LAYOUT_LINEAR>(v, ls, counter, s);
        case ST_F16:
            return L == LAYOUT_CELLS ? plain_launch<ST_F16, LAYOUT_CELLS>(v, ls, counter, s)
                                     : plain_launch<ST_F16, LAYOUT_LINEAR>(v, ls, counter, s);
        case ST_F32:
            return L == LAYOUT_CELLS ? plain_launch<ST_F32, LAYOUT_CELLS>(v, ls, counter, s)
                                     : plain_launch<ST_F32, LAYOUT_LINEAR>(v, ls, counter, s);
        case ST_U8B:
            return L == LAYOUT_CELLS ? plain_launch<ST_U8B, LAYOUT_CELLS>(v, ls, counter, s)
                                     : plain_launch<ST_U8B, LAYOUT_BRICKS>(v, ls, counter, s);
        case ST_U15:
            return L == LAYOUT_CELLS ? plain_launch<ST_U15, LAYOUT_CELLS>(v, ls, counter, s) : hipErrorInvalidValue;
        case ST_U12:
            return L == LAYOUT_CELLS    ? plain_launch<ST_U12, LAYOUT_CELLS>(v, ls, counter, s)
                   : L == LAYOUT_QUADS ? plain_launch<ST_U12, LAYOUT_QUADS>(v, ls, counter, s)
                                        : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_skip_ranges(const VolDev& v, hipStream_t s) {
    const int L = v.layout;
    switch (v.kind) {
        case ST_U8:
            return L == LAYOUT_CELLS  ? skip_range_launch<ST_U8, LAYOUT_CELLS>(v, s)
                   : L == LAYOUT_POLY ? skip_range_launch<ST_U8, LAYOUT_POLY>(v, s)
                                      : skip_range_launch<ST_U8, LAYOUT_LINEAR>(v, s);
        case ST_U16:
            return L == LAYOUT_CELLS    ? skip_range_launch<ST_U16, LAYOUT_CELLS>(v, s)
                   : L == LAYOUT_POLY   ? skip_range_launch<ST_U16, LAYOUT_POLY>(v, s)
                   : L == LAYOUT_QUADS ? skip_range_launch<ST_U16, LAYOUT_QUADS>(v, s)
                                        : skip_range_launch<ST_U16, LAYOUT_LINEAR>(v, s);
        case ST_F16:
            return L == LAYOUT_CELLS ? skip_range_launch<ST_F16, LAYOUT_CELLS>(v, s)
                                     : skip_range_launch<ST_F16, LAYOUT_LINEAR>(v, s);
        case ST_F32:
            return L == LAYOUT_CELLS ? skip_range_launch<ST_F32, LAYOUT_CELLS>(v, s)
                                     : skip_range_launch<ST_F32, LAYOUT_LINEAR>(v, s);
        case ST_U8B:
            return L == LAYOUT_CELLS ? skip_range_launch<ST_U8B, LAYOUT_CELLS>(v, s)
                                     : skip_range_launch<ST_U8B, LAYOUT_BRICKS>(v, s);
        case ST_U15:
            return L == LAYOUT_CELLS ? skip_range_launch<ST_U15, LAYOUT_CELLS>(v, s) : hipErrorInvalidValue;
        case ST_U12:
            return L == LAYOUT_CELLS    ? skip_range_launch<ST_U12, LAYOUT_CELLS>(v, s)
                   : L == LAYOUT_QUADS ? skip_range_launch<ST_U12, LAYOUT_QUADS>(v, s)
                                        : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_march_batch(int kind, int layout, void* workspace, int grid, const LaunchShape& ls, int max_k,
                              bool skip, hipStream_t s) {
    const bool C = layout == LAYOUT_CELLS, P = layout == LAYOUT_POLY, X = layout == LAYOUT_QUADS;
    switch (kind) {
        case ST_U8:
            return C   ? batch_launch<ST_U8, LAYOUT_CELLS>(workspace, grid, ls, max_k, skip, s)
                   : P ? batch_launch<ST_U8, LAYOUT_POLY>(workspace, grid, ls, max_k, skip, s)
                       : batch_launch<ST_U8, LAYOUT_LINEAR>(workspace, grid, ls, max_k, skip, s);
        case ST_U16:
            return C   ? batch_launch<ST_U16, LAYOUT_CELLS>(workspace, grid, ls, max_k, skip, s)
                   : P ? batch_launch<ST_U16, LAYOUT_POLY>(workspace, grid, ls, max_k, skip, s)
                   : X ? batch_launch<ST_U16, LAYOUT_QUADS>(workspace, grid, ls, max_k, skip, s)
                       : batch_launch<ST_U16, LAYOUT_LINEAR>(workspace, grid, ls, max_k, skip, s);
        case ST_F16:
            return C ? batch_launch<ST_F16, LAYOUT_CELLS>(workspace, grid, ls, max_k, skip, s)
                     : batch_launch<ST_F16, LAYOUT_LINEAR>(workspace, grid, ls, max_k, skip, s);
        case ST_F32:
            return C ? batch_launch<ST_F32, LAYOUT_CELLS>(workspace, grid, ls, max_k, skip, s)
                     : batch_launch<ST_F32, LAYOUT_LINEAR>(workspace, grid, ls, max_k, skip, s);
        case ST_U8B:
            return C ? batch_launch<ST_U8B, LAYOUT_CELLS>(workspace, grid, ls, max_k, skip, s)
                     : batch_launch<ST_U8B, LAYOUT_BRICKS>(workspace, grid, ls, max_k, skip, s);
        case ST_U15:
            return C ? batch_launch<ST_U15, LAYOUT_CELLS>(workspace, grid, ls, max_k, skip, s) : hipErrorInvalidValue;
        case ST_U12:
            return C   ? batch_launch<ST_U12, LAYOUT_CELLS>(workspace, grid, ls, max_k, skip, s)
                   : X ? batch_launch<ST_U12, LAYOUT_QUADS>(workspace, grid, ls, max_k, skip, s)
                       : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_march_views(int kind, int layout, void* workspace, int blocks, const LaunchShape& ls, int max_k,
                              bool skip, hipStream_t s) {
    const bool C = layout == LAYOUT_CELLS, P = layout == LAYOUT_POLY, X = layout == LAYOUT_QUADS;
    switch (kind) {
        case ST_U8:
            return C   ? views_launch<ST_U8, LAYOUT_CELLS>(workspace, blocks, ls, max_k, skip, s)
                   : P ? views_launch<ST_U8, LAYOUT_POLY>(workspace, blocks, ls, max_k, skip, s)
                       : views_launch<ST_U8, LAYOUT_LINEAR>(workspace, blocks, ls, max_k, skip, s);
        case ST_U16:
            return C   ? views_launch<ST_U16, LAYOUT_CELLS>(workspace, blocks, ls, max_k, skip, s)
                   : P ? views_launch<ST_U16, LAYOUT_POLY>(workspace, blocks, ls, max_k, skip, s)
                   : X ? views_launch<ST_U16, LAYOUT_QUADS>(workspace, blocks, ls, max_k, skip, s)
                       : views_launch<ST_U16, LAYOUT_LINEAR>(workspace, blocks, ls, max_k, skip, s);
        case ST_F16:
            return C ? views_launch<ST_F16, LAYOUT_CELLS>(workspace, blocks, ls, max_k, skip, s)
                     : views_launch<ST_F16, LAYOUT_LINEAR>(workspace, blocks, ls, max_k, skip, s);
        case ST_F32:
            return C ? views_launch<ST_F32, LAYOUT_CELLS>(workspace, blocks, ls, max_k, skip, s)
                     : views_launch<ST_F32, LAYOUT_LINEAR>(workspace, blocks, ls, max_k, skip, s);
        case ST_U8B:
            return C ? views_launch<ST_U8B, LAYOUT_CELLS>(workspace, blocks, ls, max_k, skip, s)
                     : views_launch<ST_U8B, LAYOUT_BRICKS>(workspace, blocks, ls, max_k, skip, s);
        case ST_U15:
            return C ? views_launch<ST_U15, LAYOUT_CELLS>(workspace, blocks, ls, max_k, skip, s) : hipErrorInvalidValue;
        case ST_U12:
            return C   ? views_launch<ST_U12, LAYOUT_CELLS>(workspace, blocks, ls, max_k, skip, s)
                   : X ? views_launch<ST_U12, LAYOUT_QUADS>(workspace, blocks, ls, max_k, skip, s)
                       : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_march_views_args(int kind, int layout, const SmallBatch& b, const LaunchShape& ls, bool skip,
                                   hipStream_t s) {
    const bool C = layout == LAYOUT_CELLS, P = layout == LAYOUT_POLY, X = layout == LAYOUT_QUADS;
    switch (kind) {
        case ST_U8:
            return C   ? views_args_launch<ST_U8, LAYOUT_CELLS>(b, ls, skip, s)
                   : P ? views_args_launch<ST_U8, LAYOUT_POLY>(b, ls, skip, s)
                       : views_args_launch<ST_U8, LAYOUT_LINEAR>(b, ls, skip, s);
        case ST_U16:
            return C   ? views_args_launch<ST_U16, LAYOUT_CELLS>(b, ls, skip, s)
                   : P ? views_args_launch<ST_U16, LAYOUT_POLY>(b, ls, skip, s)
                   : X ? views_args_launch<ST_U16, LAYOUT_QUADS>(b, ls, skip, s)
                       : views_args_launch<ST_U16, LAYOUT_LINEAR>(b, ls, skip, s);
        case ST_F16:
            return C ? views_args_launch<ST_F16, LAYOUT_CELLS>(b, ls, skip, s)
                     : views_args_launch<ST_F16, LAYOUT_LINEAR>(b, ls, skip, s);
        case ST_F32:
            return C ? views_args_launch<ST_F32, LAYOUT_CELLS>(b, ls, skip, s)
                     : views_args_launch<ST_F32, LAYOUT_LINEAR>(b, ls, skip, s);
        case ST_U8B:
            return C ? views_args_launch<ST_U8B, LAYOUT_CELLS>(b, ls, skip, s)
                     : views_args_launch<ST_U8B, LAYOUT_BRICKS>(b, ls, skip, s);
        case ST_U15:
            return C ? views_args_launch<ST_U15, LAYOUT_CELLS>(b, ls, skip, s) : hipErrorInvalidValue;
        case ST_U12:
            return C   ? views_args_launch<ST_U12, LAYOUT_CELLS>(b, ls, skip, s)
                   : X ? views_args_launch<ST_U12, LAYOUT_QUADS>(b, ls, skip, s)
                       : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

int batch_persistent_grid(const LaunchShape& ls, int max_k, bool skip) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const size_t lds = (size_t)(max_k + 1) * sizeof(float4) + kSkipMaskBytes + 16;
    const void* fn = skip ? (const void*)march_batch_skip_kernel<ST_U16, LAYOUT_CELLS>
                          : (const void*)march_batch_kernel<ST_U16, LAYOUT_CELLS>;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)((kMaxK + 1) * sizeof(float4) + kSkipMaskBytes + 16));
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * ls.waves, lds) != hipSuccess)
        per_cu = 1;
    if (per_cu < 1) per_cu = 1;
    return cus * per_cu;
}

}  // namespace rtv
