// VALU issue rates of single instruction forms on gfx950 (measurement tool, not
// part of the library).  Every lane runs eight independent register chains of
// one instruction; the rate is reported in wave-instructions per second and as a
// multiple of one wave64 instruction per SIMD every 4 cycles (1,024 SIMDs at
// 2.4 GHz).  The ALU rooflines of the alignment kernels are costed with these
// rates.  Build and run on one MI355X:
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       valu_rates.hip -o valu_rates && ./valu_rates
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>

#define CHAIN8(OP)                                                                    \
    asm volatile(OP : "+v"(x0) : "v"(y)); asm volatile(OP : "+v"(x1) : "v"(y));       \
    asm volatile(OP : "+v"(x2) : "v"(y)); asm volatile(OP : "+v"(x3) : "v"(y));       \
    asm volatile(OP : "+v"(x4) : "v"(y)); asm volatile(OP : "+v"(x5) : "v"(y));       \
    asm volatile(OP : "+v"(x6) : "v"(y)); asm volatile(OP : "+v"(x7) : "v"(y));

#define RATE_KERNEL(NAME, OP)                                                         \
    __global__ void __launch_bounds__(256) NAME(uint32_t *out, int iters, uint32_t seed) \
    {                                                                                 \
        uint32_t x0 = seed + threadIdx.x, x1 = x0 * 3u, x2 = x0 * 5u, x3 = x0 * 7u;   \
        uint32_t x4 = x0 * 11u, x5 = x0 * 13u, x6 = x0 * 17u, x7 = x0 * 19u;          \
        const uint32_t y = seed * 0x9E37u + 1u;                                       \
        for (int it = 0; it < iters; ++it) {                                          \
            _Pragma("unroll") for (int r = 0; r < 16; ++r) { CHAIN8(OP) }             \
        }                                                                             \
        out[blockIdx.x * blockDim.x + threadIdx.x] = x0 ^ x1 ^ x2 ^ x3 ^ x4 ^ x5 ^ x6 ^ x7; \
    }

RATE_KERNEL(k_add_u32, "v_add_u32 %0, %0, %1")
RATE_KERNEL(k_sub_u32, "v_sub_u32 %0, %0, %1")
RATE_KERNEL(k_and_b32, "v_and_b32 %0, %0, %1")
RATE_KERNEL(k_or_b32, "v_or_b32 %0, %0, %1")
RATE_KERNEL(k_xor_b32, "v_xor_b32 %0, %0, %1")
RATE_KERNEL(k_mov_b32, "v_mov_b32 %0, %1")
RATE_KERNEL(k_add_f32, "v_add_f32 %0, %0, %1")
RATE_KERNEL(k_mul_f32, "v_mul_f32 %0, %0, %1")
RATE_KERNEL(k_fma_f32, "v_fma_f32 %0, %0, %1, %0")
RATE_KERNEL(k_max_i16, "v_max_i16 %0, %0, %1")
RATE_KERNEL(k_max_i32, "v_max_i32 %0, %0, %1")
RATE_KERNEL(k_max_u32, "v_max_u32 %0, %0, %1")
RATE_KERNEL(k_max_f32, "v_max_f32 %0, %0, %1")
RATE_KERNEL(k_max3_i32, "v_max3_i32 %0, %0, %1, %0")
RATE_KERNEL(k_med3_f32, "v_med3_f32 %0, %0, %1, %0")
RATE_KERNEL(k_add3_u32, "v_add3_u32 %0, %0, %1, %0")
RATE_KERNEL(k_xad_u32, "v_xad_u32 %0, %0, %1, %0")
RATE_KERNEL(k_alignbit, "v_alignbit_b32 %0, %0, %1, 31")
RATE_KERNEL(k_bfe_i32, "v_bfe_i32 %0, %0, %1, 8")
RATE_KERNEL(k_perm_b32, "v_perm_b32 %0, %0, %1, %1")
RATE_KERNEL(k_lshlrev, "v_lshlrev_b32 %0, 1, %0")
RATE_KERNEL(k_lshl_or, "v_lshl_or_b32 %0, %0, 1, %1")
RATE_KERNEL(k_or3_b32, "v_or3_b32 %0, %0, %1, %0")
RATE_KERNEL(k_bitop3_b32, "v_bitop3_b32 %0, %0, %1, %0 bitop3:0x1e")
RATE_KERNEL(k_pk_add_u16, "v_pk_add_u16 %0, %0, %1")
RATE_KERNEL(k_pk_max_i16, "v_pk_max_i16 %0, %0, %1")
RATE_KERNEL(k_cvt_f32_i32, "v_cvt_f32_i32 %0, %0")
RATE_KERNEL(k_mov_dpp, "v_mov_b32_dpp %0, %1 row_shr:1 row_mask:0xf bank_mask:0xf")

typedef void (*rate_fn)(uint32_t *, int, uint32_t);

static void run(const char *name, rate_fn k, uint32_t *d, int blocks, int iters)
{
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        printf("event creation failed\n");
        return;
    }
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, 0, d, iters, 1u);   // warm-up
    (void)hipEventRecord(a);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, 0, d, iters, 2u);
    (void)hipEventRecord(b);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    const double instr = blocks * 4.0 * iters * 16.0 * 8.0;      // waves x instructions per lane
    const double rate = instr / (ms * 1e-3);
    printf("| `%s` | %.3f | %.1f | %.2f |\n", name + 2, ms, rate / 1e9, rate / (1024.0 * 2.4e9 / 4.0));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
}

int main()
{
    const int blocks = 2048, iters = 2000;   // 8 waves per SIMD
    uint32_t *d = nullptr;
    if (hipMalloc(&d, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) {
        printf("hipMalloc failed\n");
        return 1;
    }
    printf("| instruction | ms | G wave-instr/s | x (one per SIMD per 4 cycles) |\n|---|---|---|---|\n");
#define RUN(K) run(#K, K, d, blocks, iters)
    RUN(k_add_u32); RUN(k_sub_u32); RUN(k_and_b32); RUN(k_or_b32); RUN(k_xor_b32); RUN(k_mov_b32);
    RUN(k_add_f32); RUN(k_mul_f32); RUN(k_fma_f32); RUN(k_max_i16); RUN(k_max_i32); RUN(k_max_u32);
    RUN(k_max_f32); RUN(k_max3_i32); RUN(k_med3_f32); RUN(k_add3_u32); RUN(k_xad_u32); RUN(k_alignbit);
    RUN(k_bfe_i32); RUN(k_perm_b32); RUN(k_lshlrev); RUN(k_lshl_or); RUN(k_or3_b32); RUN(k_bitop3_b32); RUN(k_pk_add_u16);
    RUN(k_pk_max_i16); RUN(k_cvt_f32_i32); RUN(k_mov_dpp);
    (void)hipFree(d);
    return 0;
}
