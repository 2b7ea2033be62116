// relayout.hip -- volume creation: source grid -> storage layout.
//
// The scalar field f(x,y,z) on a Cartesian grid (arXiv:1211.5595, Section
// 2.1) arrives as a C-order [z][y][x] array.  The marcher reads
//   - cell-packed and linear layouts of the grid with a one-node replicated
//     border on every face, so a sample that rounding places a hair outside
//     the box still has 8 valid corners and reproduces clamp-to-edge exactly;
//   - brick-scaled 8-bit: per brick of B^3 cells a (lo, scale) and 8-bit
//     codes for local nodes -1..B+1 (B+3 per axis), lo = min and
//     scale = (max-lo)/255 over the brick's nodes, code = rint((v-lo)/scale)
//     in binary32.  Every cell's 8 corners come from the brick owning it.
#include <hip/hip_fp16.h>

#include "rt_internal.h"

namespace rtv {

namespace {

template <int KIND>
struct Src;
template <>
struct Src<ST_U8> {
    using T = unsigned char;
    static __device__ __forceinline__ float f(T x) { return (float)x; }
};
template <>
struct Src<ST_U16> {
    using T = unsigned short;
    static __device__ __forceinline__ float f(T x) { return (float)x; }
};
template <>
struct Src<ST_F16> {
    using T = unsigned short;
    static __device__ __forceinline__ float f(T x) { return (float)__builtin_bit_cast(_Float16, x); }
};
template <>
struct Src<ST_F32> {
    using T = float;
    static __device__ __forceinline__ float f(T x) { return x; }
};

template <int SRC, int DST>
__device__ __forceinline__ void store_elem(void* dst, size_t e, typename Src<SRC>::T x) {
    if constexpr (DST == ST_U8) {
        static_cast<unsigned char*>(dst)[e] = (unsigned char)x;
    } else if constexpr (DST == ST_U16) {
        static_cast<unsigned short*>(dst)[e] = (unsigned short)x;
    } else if constexpr (DST == ST_F16) {
        if constexpr (SRC == ST_F16) {
            static_cast<unsigned short*>(dst)[e] = x;
        } else {
            // integers up to 2^24 and binary32 values are exact in float; one RNE rounding to half
            _Float16 h = (_Float16)Src<SRC>::f(x);
            static_cast<unsigned short*>(dst)[e] = __builtin_bit_cast(unsigned short, h);
        }
    } else {
        static_cast<float*>(dst)[e] = Src<SRC>::f(x);
    }
}

template <int SRC, int DST>
__global__ void __launch_bounds__(256) relayout_linear_kernel(const typename Src<SRC>::T* __restrict__ src,
                                                               void* __restrict__ dst, int nx, int ny, int nz) {
    const int px = nx + 2, py = ny + 2, pz = nz + 2;
    const size_t total = (size_t)px * py * pz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int pi = (int)(e % px);
        const size_t t = e / px;
        const int pj = (int)(t % py), pk = (int)(t / py);
        const int i = min(max(pi - 1, 0), nx - 1), j = min(max(pj - 1, 0), ny - 1), k = min(max(pk - 1, 0), nz - 1);
        store_elem<SRC, DST>(dst, e, src[((size_t)k * ny + j) * nx + i]);
    }
}

// Cell-packed layout: one thread per padded cell (cx, cy, cz) of the
// block-rounded cell grid; it writes the cell's 8 corners (padded nodes
// c..c+1 per axis, i.e. volume nodes clamp(c-1 .. c)) contiguously at
// ((block * 8) + within) * 8 elements, block = x-fastest index of
// (cx/2, cy/2, cz/2) and within = (cx&1) | (cy&1)<<1 | (cz&1)<<2.
template <int SRC, int DST>
__global__ void __launch_bounds__(256) relayout_cells_kernel(const typename Src<SRC>::T* __restrict__ src,
                                                              void* __restrict__ dst, int nx, int ny, int nz, int nbx,
                                                              int nby, int nbz) {
    const int cxn = 2 * nbx, cyn = 2 * nby, czn = 2 * nbz;
    const size_t total = (size_t)cxn * cyn * czn;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        // e enumerates cells in storage order: block-major, then within-block
        const int within = (int)(e & 7);
        const size_t blk = e >> 3;
        const int bx = (int)(blk % nbx);
        const size_t t = blk / nbx;
        const int by = (int)(t % nby), bz = (int)(t / nby);
        const int cx = 2 * bx + (within & 1), cy = 2 * by + ((within >> 1) & 1), cz = 2 * bz + (within >> 2);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int i = min(max(cx + (c & 1) - 1, 0), nx - 1);
            const int j = min(max(cy + ((c >> 1) & 1) - 1, 0), ny - 1);
            const int k = min(max(cz + (c >> 2) - 1, 0), nz - 1);
            store_elem<SRC, DST>(dst, e * 8 + c, src[((size_t)k * ny + j) * nx + i]);
        }
    }
}

// 15-bit difference cells: as relayout_cells_kernel (same block order), with
// each x-pair of corners stored as (c0, c1 - c0) in 16-bit words, the values
// clamped to 0..32767 first so that the difference fits a signed word.
template <int SRC>
__global__ void __launch_bounds__(256) relayout_cells_dx_kernel(const typename Src<SRC>::T* __restrict__ src,
                                                                 unsigned short* __restrict__ dst, int nx, int ny,
                                                                 int nz, int nbx, int nby, int nbz) {
    const int cxn = 2 * nbx, cyn = 2 * nby, czn = 2 * nbz;
    const size_t total = (size_t)cxn * cyn * czn;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int within = (int)(e & 7);
        const size_t blk = e >> 3;
        const int bx = (int)(blk % nbx);
        const size_t t = blk / nbx;
        const int by = (int)(t % nby), bz = (int)(t / nby);
        const int cx = 2 * bx + (within & 1), cy = 2 * by + ((within >> 1) & 1), cz = 2 * bz + (within >> 2);
#pragma unroll
        for (int c = 0; c < 8; c += 2) {
            const int j = min(max(cy + ((c >> 1) & 1) - 1, 0), ny - 1);
            const int k = min(max(cz + (c >> 2) - 1, 0), nz - 1);
            const int i0 = min(max(cx - 1, 0), nx - 1), i1 = min(max(cx, 0), nx - 1);
            const int v0 = min((int)src[((size_t)k * ny + j) * nx + i0], 32767);
            const int v1 = min((int)src[((size_t)k * ny + j) * nx + i1], 32767);
            dst[e * 8 + c] = (unsigned short)v0;
            dst[e * 8 + c + 1] = (unsigned short)(short)(v1 - v0);
        }
    }
}

// 12-bit half cells: as relayout_cells_kernel, each value clamped to 0..4096
// and stored as the binary16 of (value - 2048), which is exact on that range
// (every integer of magnitude up to 2048 is a binary16 value).
template <int SRC>
__global__ void __launch_bounds__(256) relayout_cells_h12_kernel(const typename Src<SRC>::T* __restrict__ src,
                                                                  _Float16* __restrict__ dst, int nx, int ny, int nz,
                                                                  int nbx, int nby, int nbz) {
    const size_t total = (size_t)8 * nbx * nby * nbz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int within = (int)(e & 7);
        const size_t blk = e >> 3;
        const int bx = (int)(blk % nbx);
        const size_t t = blk / nbx;
        const int by = (int)(t % nby), bz = (int)(t / nby);
        const int cx = 2 * bx + (within & 1), cy = 2 * by + ((within >> 1) & 1), cz = 2 * bz + (within >> 2);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int i = min(max(cx + (c & 1) - 1, 0), nx - 1);
            const int j = min(max(cy + ((c >> 1) & 1) - 1, 0), ny - 1);
            const int k = min(max(cz + (c >> 2) - 1, 0), nz - 1);
            const int v = min((int)src[((size_t)k * ny + j) * nx + i], 4096);
            dst[e * 8 + c] = (_Float16)(v - 2048);
        }
    }
}

// Quad bricks: one thread per 8-byte quad slot.  Slot e: brick e / 16
// (x-fastest over nbx, nby, nbz), column c = (e / 4) % 4 of the brick
// (x = 2 bx + (c & 1), y = 2 by + (c >> 1)), layer l = e % 4 (z = 3 bz + l);
// the quad holds volume nodes clamp(x-1..x, y-1..y) of slice clamp(z-1),
// x fastest: 16-bit integers, or (H12) the binary16 halves of
// (value - 2048) with the value clamped to 0..4096 as in the 12-bit cells.
template <int SRC, bool H12>
__global__ void __launch_bounds__(256) relayout_quads_kernel(const typename Src<SRC>::T* __restrict__ src,
                                                              uint2* __restrict__ dst, int nx, int ny, int nz,
                                                              int nbx, int nby, int nbz) {
    const size_t total = (size_t)16 * nbx * nby * nbz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int l = (int)(e & 3), c = (int)((e >> 2) & 3);
        const size_t blk = e >> 4;
        const int bx = (int)(blk % nbx);
        const size_t t = blk / nbx;
        const int by = (int)(t % nby), bz = (int)(t / nby);
        const int cx = 2 * bx + (c & 1), cy = 2 * by + (c >> 1), lz = 3 * bz + l;
        const int i0 = min(max(cx - 1, 0), nx - 1), i1 = min(cx, nx - 1);
        const int j0 = min(max(cy - 1, 0), ny - 1), j1 = min(cy, ny - 1);
        const int k = min(max(lz - 1, 0), nz - 1);
        const size_t r0 = ((size_t)k * ny + j0) * nx, r1 = ((size_t)k * ny + j1) * nx;
        const int v[4] = {(int)src[r0 + i0], (int)src[r0 + i1], (int)src[r1 + i0], (int)src[r1 + i1]};
        unsigned int w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if constexpr (H12) {
                const _Float16 h = (_Float16)(min(v[q], 4096) - 2048);
                w[q] = __builtin_bit_cast(unsigned short, h);
            } else {
                w[q] = (unsigned int)(v[q] & 0xffff);
            }
        }
        dst[e] = make_uint2(w[0] | (w[1] << 16), w[2] | (w[3] << 16));
    }
}

// Polynomial cells: as relayout_cells_kernel, but the 8 stored values are the
// coefficients of the cell's trilinear polynomial, formed in integer
// arithmetic from integer corners and stored as exact binary32 values.
template <int SRC>
__global__ void __launch_bounds__(256) relayout_poly_kernel(const typename Src<SRC>::T* __restrict__ src,
                                                             float4* __restrict__ dst, int nx, int ny, int nz, int nbx,
                                                             int nby, int nbz) {
    const size_t total = (size_t)8 * nbx * nby * nbz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int within = (int)(e & 7);
        const size_t blk = e >> 3;
        const int bx = (int)(blk % nbx);
        const size_t t = blk / nbx;
        const int by = (int)(t % nby), bz = (int)(t / nby);
        const int cx = 2 * bx + (within & 1), cy = 2 * by + ((within >> 1) & 1), cz = 2 * bz + (within >> 2);
        int c[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = min(max(cx + (k & 1) - 1, 0), nx - 1);
            const int j = min(max(cy + ((k >> 1) & 1) - 1, 0), ny - 1);
            const int l = min(max(cz + (k >> 2) - 1, 0), nz - 1);
            c[k] = (int)src[((size_t)l * ny + j) * nx + i];
        }
        const int p0 = c[0], px = c[1] - c[0], py = c[2] - c[0], pz = c[4] - c[0];
        const int pxy = c[3] - c[1] - c[2] + c[0], pxz = c[5] - c[1] - c[4] + c[0];
        const int pyz = c[6] - c[2] - c[4] + c[0];
        const int pxyz = c[7] - c[3] - c[5] - c[6] + c[1] + c[2] + c[4] - c[0];
        dst[2 * e] = make_float4((float)p0, (float)px, (float)py, (float)pz);
        dst[2 * e + 1] = make_float4((float)pxy, (float)pxz, (float)pyz, (float)pxyz);
    }
}

// One workgroup per brick: min and max over nodes [b*B, min(b*B+B, n-1)].
template <int SRC>
__global__ void __launch_bounds__(256) brick_minmax_kernel(const typename Src<SRC>::T* __restrict__ src, int nx,
                                                            int ny, int nz, int B, int nbx, int nby,
                                                            float2* __restrict__ par) {
    __shared__ float s_lo[256], s_hi[256];
    const int bid = blockIdx.x;
    const int bx = bid % nbx, by = (bid / nbx) % nby, bz = bid / (nbx * nby);
    const int x0 = bx * B, y0 = by * B, z0 = bz * B;
    const int ex = min(x0 + B, nx - 1) - x0 + 1, ey = min(y0 + B, ny - 1) - y0 + 1, ez = min(z0 + B, nz - 1) - z0 + 1;
    const int cnt = ex * ey * ez;
    float lo = INFINITY, hi = -INFINITY;
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        const int i = e % ex, j = (e / ex) % ey, k = e / (ex * ey);
        const float v = Src<SRC>::f(src[((size_t)(z0 + k) * ny + (y0 + j)) * nx + (x0 + i)]);
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
    }
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s_lo[threadIdx.x] = fminf(s_lo[threadIdx.x], s_lo[threadIdx.x + s]);
            s_hi[threadIdx.x] = fmaxf(s_hi[threadIdx.x], s_hi[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float l = s_lo[0], h = s_hi[0];
        par[bid] = make_float2(l, h > l ? (h - l) / 255.0f : 1.0f);
    }
}

// One thread per stored code; local node l in [0, B+2] is global node b*B+l-1,
// clamped into the volume.
template <int SRC>
__global__ void __launch_bounds__(256) brick_encode_kernel(const typename Src<SRC>::T* __restrict__ src, int nx,
                                                            int ny, int nz, int B, int nbx, int nby, int nbz,
                                                            const float2* __restrict__ par,
                                                            unsigned char* __restrict__ codes) {
    const int S = B + 3;
    const size_t per = (size_t)S * S * S;
    const size_t total = per * nbx * nby * nbz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int bid = (int)(e / per);
        const int l = (int)(e - (size_t)bid * per);
        const int lx = l % S, ly = (l / S) % S, lz = l / (S * S);
        const int bx = bid % nbx, by = (bid / nbx) % nby, bz = bid / (nbx * nby);
        const int i = min(max(bx * B + lx - 1, 0), nx - 1);
        const int j = min(max(by * B + ly - 1, 0), ny - 1);
        const int k = min(max(bz * B + lz - 1, 0), nz - 1);
        const float v = Src<SRC>::f(src[((size_t)k * ny + j) * nx + i]);
        const float2 p = par[bid];
        const float q = rintf((v - p.x) / p.y);
        codes[e] = (unsigned char)fminf(fmaxf(q, 0.0f), 255.0f);
    }
}

// Cell-packed 8-bit codes: one thread per cell of the shifted block grid
// (block b holds padded cells C with C+1 in {2b, 2b+1}); the owner brick of
// unpadded cell c = C-1 is clamp(c, 0, n-2)/B, the same for all 8 cells of a
// block.  Each cell gets its 8 corner codes (nodes clamp(c..c+1)) quantised
// with the owner's (lo, scale); the block's first cell also stores that pair.
template <int SRC>
__global__ void __launch_bounds__(256) brick_cells_kernel(const typename Src<SRC>::T* __restrict__ src, int nx,
                                                           int ny, int nz, int B, int nbx, int nby,
                                                           const float2* __restrict__ par, int cbx, int cby, int cbz,
                                                           float2* __restrict__ block_par,
                                                           unsigned char* __restrict__ codes) {
    const size_t total = (size_t)8 * cbx * cby * cbz;
    const int n[3] = {nx, ny, nz};
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int within = (int)(e & 7);
        const size_t blk = e >> 3;
        const int b[3] = {(int)(blk % cbx), (int)((blk / cbx) % cby), (int)(blk / ((size_t)cbx * cby))};
        int c[3], owner[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c[a] = 2 * b[a] + ((within >> a) & 1) - 2;  // unpadded cell index, -2..n
            owner[a] = min(max(c[a], 0), n[a] - 2) / B;
        }
        const float2 p = par[(owner[2] * nby + owner[1]) * nbx + owner[0]];
        unsigned long long word = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = min(max(c[0] + (k & 1), 0), nx - 1);
            const int j = min(max(c[1] + ((k >> 1) & 1), 0), ny - 1);
            const int l = min(max(c[2] + (k >> 2), 0), nz - 1);
            const float v = Src<SRC>::f(src[((size_t)l * ny + j) * nx + i]);
            const float q = fminf(fmaxf(rintf((v - p.x) / p.y), 0.0f), 255.0f);
            word |= (unsigned long long)(unsigned int)q << (8 * k);
        }
        reinterpret_cast<unsigned long long*>(codes)[e] = word;
        if (within == 0) block_par[blk] = p;
    }
}

int grid_for(size_t total, int block) {
    size_t g = (total + block - 1) / block;
    if (g > (size_t)1 << 20) g = (size_t)1 << 20;
    return (int)(g ? g : 1);
}

template <int SRC>
hipError_t linear_dispatch(const void* src, int dst_kind, const int32_t n[3], void* dst, hipStream_t s) {
    using T = typename Src<SRC>::T;
    const T* p = static_cast<const T*>(src);
    const size_t total = (size_t)(n[0] + 2) * (n[1] + 2) * (n[2] + 2);
    const int g = grid_for(total, 256);
    switch (dst_kind) {
        case ST_U8:
            if constexpr (SRC == ST_U8)
                hipLaunchKernelGGL((relayout_linear_kernel<SRC, ST_U8>), dim3(g), dim3(256), 0, s, p, dst, n[0], n[1],
                                   n[2]);
            else
                return hipErrorInvalidValue;
            break;
        case ST_U16:
            if constexpr (SRC == ST_U8 || SRC == ST_U16)
                hipLaunchKernelGGL((relayout_linear_kernel<SRC, ST_U16>), dim3(g), dim3(256), 0, s, p, dst, n[0],
                                   n[1], n[2]);
            else
                return hipErrorInvalidValue;
            break;
        case ST_F16:
            hipLaunchKernelGGL((relayout_linear_kernel<SRC, ST_F16>), dim3(g), dim3(256), 0, s, p, dst, n[0], n[1],
                               n[2]);
            break;
        case ST_F32:
            hipLaunchKernelGGL((relayout_linear_kernel<SRC, ST_F32>), dim3(g), dim3(256), 0, s, p, dst, n[0], n[1],
                               n[2]);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int SRC>
hipError_t cells_dispatch(const void* src, int dst_kind, const int32_t n[3], const int32_t nb[3], void* dst,
                          hipStream_t s) {
    using T = typename Src<SRC>::T;
    const T* p = static_cast<const T*>(src);
    const size_t total = (size_t)8 * nb[0] * nb[1] * nb[2];
    const int g = grid_for(total, 256);
    switch (dst_kind) {
        case ST_U8:
            if constexpr (SRC == ST_U8)
                hipLaunchKernelGGL((relayout_cells_kernel<SRC, ST_U8>), dim3(g), dim3(256), 0, s, p, dst, n[0], n[1],
                                   n[2], nb[0], nb[1], nb[2]);
            else
                return hipErrorInvalidValue;
            break;
        case ST_U16:
            if constexpr (SRC == ST_U8 || SRC == ST_U16)
                hipLaunchKernelGGL((relayout_cells_kernel<SRC, ST_U16>), dim3(g), dim3(256), 0, s, p, dst, n[0],
                                   n[1], n[2], nb[0], nb[1], nb[2]);
            else
                return hipErrorInvalidValue;
            break;
        case ST_F16:
            hipLaunchKernelGGL((relayout_cells_kernel<SRC, ST_F16>), dim3(g), dim3(256), 0, s, p, dst, n[0], n[1],
                               n[2], nb[0], nb[1], nb[2]);
            break;
        case ST_U15:
            if constexpr (SRC == ST_U8 || SRC == ST_U16)
                hipLaunchKernelGGL((relayout_cells_dx_kernel<SRC>), dim3(g), dim3(256), 0, s, p,
                                   static_cast<unsigned short*>(dst), n[0], n[1], n[2], nb[0], nb[1], nb[2]);
            else
                return hipErrorInvalidValue;
            break;
        case ST_U12:
            if constexpr (SRC == ST_U8 || SRC == ST_U16)
                hipLaunchKernelGGL((relayout_cells_h12_kernel<SRC>), dim3(g), dim3(256), 0, s, p,
                                   static_cast<_Float16*>(dst), n[0], n[1], n[2], nb[0], nb[1], nb[2]);
            else
                return hipErrorInvalidValue;
            break;
        case ST_F32:
            hipLaunchKernelGGL((relayout_cells_kernel<SRC, ST_F32>), dim3(g), dim3(256), 0, s, p, dst, n[0], n[1],
                               n[2], nb[0], nb[1], nb[2]);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int SRC>
hipError_t u8b_dispatch(const void* src, const int32_t n[3], int B, const int32_t nb[3], float2* par,
                        unsigned char* codes, hipStream_t s) {
    using T = typename Src<SRC>::T;
    const T* p = static_cast<const T*>(src);
    const int nbt = nb[0] * nb[1] * nb[2];
    hipLaunchKernelGGL(brick_minmax_kernel<SRC>, dim3(nbt), dim3(256), 0, s, p, n[0], n[1], n[2], B, nb[0], nb[1],
                       par);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t total = (size_t)nbt * (B + 3) * (B + 3) * (B + 3);
    hipLaunchKernelGGL(brick_encode_kernel<SRC>, dim3(grid_for(total, 256)), dim3(256), 0, s, p, n[0], n[1], n[2], B,
                       nb[0], nb[1], nb[2], par, codes);
    return hipGetLastError();
}

template <int SRC>
hipError_t u8b_cells_dispatch(const void* src, const int32_t n[3], int B, const int32_t nb[3], float2* par,
                              const int32_t ncb[3], float2* block_par, unsigned char* codes, hipStream_t s) {
    using T = typename Src<SRC>::T;
    const T* p = static_cast<const T*>(src);
    const int nbt = nb[0] * nb[1] * nb[2];
    hipLaunchKernelGGL(brick_minmax_kernel<SRC>, dim3(nbt), dim3(256), 0, s, p, n[0], n[1], n[2], B, nb[0], nb[1],
                       par);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t total = (size_t)8 * ncb[0] * ncb[1] * ncb[2];
    hipLaunchKernelGGL(brick_cells_kernel<SRC>, dim3(grid_for(total, 256)), dim3(256), 0, s, p, n[0], n[1], n[2], B,
                       nb[0], nb[1], par, ncb[0], ncb[1], ncb[2], block_par, codes);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_relayout_poly(const void* src, int src_kind, const int32_t n[3], const int32_t nb[3], void* dst,
                                hipStream_t s) {
    const size_t total = (size_t)8 * nb[0] * nb[1] * nb[2];
    float4* d = static_cast<float4*>(dst);
    switch (src_kind) {
        case ST_U8:
            hipLaunchKernelGGL(relayout_poly_kernel<ST_U8>, dim3(grid_for(total, 256)), dim3(256), 0, s,
                               static_cast<const unsigned char*>(src), d, n[0], n[1], n[2], nb[0], nb[1], nb[2]);
            break;
        case ST_U16:
            hipLaunchKernelGGL(relayout_poly_kernel<ST_U16>, dim3(grid_for(total, 256)), dim3(256), 0, s,
                               static_cast<const unsigned short*>(src), d, n[0], n[1], n[2], nb[0], nb[1], nb[2]);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_relayout_quads(const void* src, int src_kind, int dst_kind, const int32_t n[3],
                                 const int32_t nb[3], void* dst, hipStream_t s) {
    const size_t total = (size_t)16 * nb[0] * nb[1] * nb[2];
    uint2* d = static_cast<uint2*>(dst);
    const int g = grid_for(total, 256);
    if (dst_kind != ST_U16 && dst_kind != ST_U12) return hipErrorInvalidValue;
    const bool h12 = dst_kind == ST_U12;
    switch (src_kind) {
        case ST_U8: {
            const unsigned char* p = static_cast<const unsigned char*>(src);
            if (h12)
                hipLaunchKernelGGL((relayout_quads_kernel<ST_U8, true>), dim3(g), dim3(256), 0, s, p, d, n[0], n[1],
                                   n[2], nb[0], nb[1], nb[2]);
            else
                hipLaunchKernelGGL((relayout_quads_kernel<ST_U8, false>), dim3(g), dim3(256), 0, s, p, d, n[0], n[1],
                                   n[2], nb[0], nb[1], nb[2]);
            break;
        }
        case ST_U16: {
            const unsigned short* p = static_cast<const unsigned short*>(src);
            if (h12)
                hipLaunchKernelGGL((relayout_quads_kernel<ST_U16, true>), dim3(g), dim3(256), 0, s, p, d, n[0], n[1],
                                   n[2], nb[0], nb[1], nb[2]);
            else
                hipLaunchKernelGGL((relayout_quads_kernel<ST_U16, false>), dim3(g), dim3(256), 0, s, p, d, n[0],
                                   n[1], n[2], nb[0], nb[1], nb[2]);
            break;
        }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_relayout_u8b_cells(const void* src, int src_kind, const int32_t n[3], int B, const int32_t nb[3],
                                     float2* brick_par, const int32_t ncb[3], float2* block_par,
                                     unsigned char* codes, hipStream_t s) {
    switch (src_kind) {
        case ST_U8: return u8b_cells_dispatch<ST_U8>(src, n, B, nb, brick_par, ncb, block_par, codes, s);
        case ST_U16: return u8b_cells_dispatch<ST_U16>(src, n, B, nb, brick_par, ncb, block_par, codes, s);
        case ST_F16: return u8b_cells_dispatch<ST_F16>(src, n, B, nb, brick_par, ncb, block_par, codes, s);
        case ST_F32: return u8b_cells_dispatch<ST_F32>(src, n, B, nb, brick_par, ncb, block_par, codes, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_relayout_linear(const void* src, int src_kind, int dst_kind, const int32_t n[3], void* dst,
                                  hipStream_t s) {
    switch (src_kind) {
        case ST_U8: return linear_dispatch<ST_U8>(src, dst_kind, n, dst, s);
        case ST_U16: return linear_dispatch<ST_U16>(src, dst_kind, n, dst, s);
        case ST_F16: return linear_dispatch<ST_F16>(src, dst_kind, n, dst, s);
        case ST_F32: return linear_dispatch<ST_F32>(src, dst_kind, n, dst, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_relayout_cells(const void* src, int src_kind, int dst_kind, const int32_t n[3],
                                 const int32_t nb[3], void* dst, hipStream_t s) {
    switch (src_kind) {
        case ST_U8: return cells_dispatch<ST_U8>(src, dst_kind, n, nb, dst, s);
        case ST_U16: return cells_dispatch<ST_U16>(src, dst_kind, n, nb, dst, s);
        case ST_F16: return cells_dispatch<ST_F16>(src, dst_kind, n, nb, dst, s);
        case ST_F32: return cells_dispatch<ST_F32>(src, dst_kind, n, nb, dst, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_relayout_u8b(const void* src, int src_kind, const int32_t n[3], int B, const int32_t nb[3],
                               float2* brick_par, unsigned char* codes, hipStream_t s) {
    switch (src_kind) {
        case ST_U8: return u8b_dispatch<ST_U8>(src, n, B, nb, brick_par, codes, s);
        case ST_U16: return u8b_dispatch<ST_U16>(src, n, B, nb, brick_par, codes, s);
        case ST_F16: return u8b_dispatch<ST_F16>(src, n, B, nb, brick_par, codes, s);
        case ST_F32: return u8b_dispatch<ST_F32>(src, n, B, nb, brick_par, codes, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rtv
