// valu_probe.hip -- issue cost of single vector-ALU instruction kinds on one
// gfx950 SIMD, to read the marcher's instruction mix against.
//
// Each kernel runs one instruction kind in 8 independent dependency chains
// per lane, 8 wavefronts per SIMD on every compute unit, and is timed with
// events; the output is the time per wave64 instruction per SIMD, in cycles
// of the 2.4 GHz peak clock.  Nothing is read from memory; each lane stores
// one word.  Build and run:
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops valu_probe.hip -o valu_probe
//   ./valu_probe
#include <hip/hip_runtime.h>

#include <cstdio>

#define CH 8
#define BODY(INS) \
    _Pragma("unroll") for (int c = 0; c < CH; ++c) asm volatile(INS : "+v"(a[c]) : "v"(b), "v"(d));

template <int K>
__global__ void __launch_bounds__(256) probe(unsigned* out, int iters, unsigned b, unsigned d) {
    unsigned a[CH];
    unsigned long long w[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        a[c] = threadIdx.x * 7u + c;
        w[c] = threadIdx.x + c;
    }
    for (int i = 0; i < iters; ++i) {
        if constexpr (K == 0) { BODY("v_fma_f32 %0, %0, %1, %2") }
        if constexpr (K == 1) { BODY("v_fmac_f32 %0, %1, %2") }
        if constexpr (K == 2) { BODY("v_mul_f32 %0, %0, %1") }
        if constexpr (K == 3) { BODY("v_add_f32 %0, %0, %1") }
        if constexpr (K == 4) { BODY("v_sub_f32 %0, %0, %1") }
        if constexpr (K == 5) { BODY("v_add_u32 %0, %0, %1") }
        if constexpr (K == 6) { BODY("v_and_b32 %0, %0, %1") }
        if constexpr (K == 7) { BODY("v_mov_b32 %0, %1") }
        if constexpr (K == 8) { BODY("v_lshrrev_b32 %0, 1, %0") }
        if constexpr (K == 9) { BODY("v_lshlrev_b32 %0, 1, %0") }
        if constexpr (K == 10) { BODY("v_lshl_add_u32 %0, %0, 1, %1") }
        if constexpr (K == 11) { BODY("v_mad_u32_u24 %0, %0, %1, %2") }
        if constexpr (K == 12) { BODY("v_cvt_f32_u32 %0, %0") }
        if constexpr (K == 13) { BODY("v_cvt_u32_f32 %0, %0") }
        if constexpr (K == 14) { BODY("v_fract_f32 %0, %0") }
        if constexpr (K == 15) { BODY("v_med3_f32 %0, %0, %1, %2") }
        if constexpr (K == 16) { BODY("v_max_f32 %0, %0, %1") }
        if constexpr (K == 17) { BODY("v_fma_mix_f32 %0, %0, %1, %2 op_sel_hi:[0,0,1]") }
        if constexpr (K == 18) { BODY("v_cvt_f32_f16 %0, %0") }
        if constexpr (K == 19) {
#pragma unroll
            for (int c = 0; c < CH; ++c) asm volatile("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(w[c]) : "v"(w[(c + 1) % CH]));
        }
        if constexpr (K == 20) {
#pragma unroll
            for (int c = 0; c < CH; ++c) asm volatile("v_mov_b64 %0, %1" : "=v"(w[c]) : "v"(w[(c + 1) % CH]));
        }
        if constexpr (K == 21) {  // one carry-chained 64-bit add: two instructions
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                unsigned long long cc;
                unsigned hi = (unsigned)(w[c] >> 32);
                asm volatile("v_add_co_u32_e64 %0, %1, %0, %3\n\tv_addc_co_u32_e64 %2, %1, %2, %4, %1"
                             : "+v"(a[c]), "=&s"(cc), "+v"(hi) : "v"(b), "v"(d));
                w[c] = ((unsigned long long)hi << 32) | (unsigned)w[c];
            }
        }
    }
    unsigned s = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) s += a[c] + (unsigned)w[c] + (unsigned)(w[c] >> 32);
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

typedef void (*kfn)(unsigned*, int, unsigned, unsigned);

#define CK(x)                                                                                 \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);        \
            return 1;                                                                         \
        }                                                                                     \
    } while (0)

int main() {
    int cus = 0;
    CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    const int block = 256, grid = cus * 4 * 8 * 64 / block;  // 8 wavefronts per SIMD
    unsigned* out = nullptr;
    CK(hipMalloc(&out, (size_t)grid * block * sizeof(unsigned)));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    const int iters = 20000;
    const kfn fns[] = {probe<0>,  probe<1>,  probe<2>,  probe<3>,  probe<4>,  probe<5>,  probe<6>,  probe<7>,
                       probe<8>,  probe<9>,  probe<10>, probe<11>, probe<12>, probe<13>, probe<14>, probe<15>,
                       probe<16>, probe<17>, probe<18>, probe<19>, probe<20>, probe<21>};
    const char* names[] = {"v_fma_f32",      "v_fmac_f32",    "v_mul_f32",      "v_add_f32",     "v_sub_f32",
                           "v_add_u32",      "v_and_b32",     "v_mov_b32",      "v_lshrrev_b32", "v_lshlrev_b32",
                           "v_lshl_add_u32", "v_mad_u32_u24", "v_cvt_f32_u32",  "v_cvt_u32_f32", "v_fract_f32",
                           "v_med3_f32",     "v_max_f32",     "v_fma_mix_f32",  "v_cvt_f32_f16", "v_lshl_add_u64",
                           "v_mov_b64",      "v_add_co_u32+v_addc_co_u32"};
    const int n = sizeof(fns) / sizeof(fns[0]);
    for (int k = 0; k < n; ++k) {
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            CK(hipEventRecord(e0, 0));
            hipLaunchKernelGGL(fns[k], dim3(grid), dim3(block), 0, 0, out, iters, 3u, 5u);
            CK(hipGetLastError());
            CK(hipEventRecord(e1, 0));
            CK(hipEventSynchronize(e1));
            float ms = 0.0f;
            CK(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0 && ms < best) best = ms;
        }
        const double steps = (double)grid * (block / 64) * iters * CH;  // chain steps, wave64 granularity
        std::printf("{\"instruction\": \"%s\", \"ms\": %.4f, \"cycles_per_wave64_at_2.4GHz\": %.3f}\n", names[k], best,
                    (double)cus * 4 * 2.4e9 * best * 1e-3 / steps);
    }
    std::fflush(stdout);
    CK(hipFree(out));
    return 0;
}
