// Encode step: ASCII bases -> 2-bit codes, 16 bases per 32-bit word.
//
// HBM-bound streaming: each thread reads 16 bytes (one 128-bit load when the
// source is aligned) and writes one word, so a wave moves 1 KiB in and 256 B
// out per instruction pair.
#include "internal.h"

namespace hpgsw {

__device__ __forceinline__ uint32_t base_code(uint32_t c, uint32_t &bad)
{
    // A=0x41 C=0x43 G=0x47 T=0x54 map to 0,1,2,3 through ((c>>1) ^ (c>>2)) & 3
    bool ok = (c == 'A') | (c == 'C') | (c == 'G') | (c == 'T');
    bad += ok ? 0u : 1u;
    return ok ? (((c >> 1) ^ (c >> 2)) & 3u) : 0u;
}

__device__ __forceinline__ uint32_t pack_dword(uint32_t x, uint32_t &bad)
{
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w |= base_code((x >> (8 * k)) & 0xFFu, bad) << (2 * k);
    return w;
}

__global__ void __launch_bounds__(256) k_pack2b(const uint8_t *__restrict__ ascii, uint64_t n,
                                                uint32_t *__restrict__ out, uint32_t *bad_count)
{
    const uint64_t nwords = (n + 15) >> 4;
    uint32_t bad = 0;
    const bool aligned = (reinterpret_cast<uintptr_t>(ascii) & 15u) == 0;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords;
         w += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t base = w << 4;
        uint32_t word = 0;
        if (aligned && base + 16 <= n) {
            uint4 v = *reinterpret_cast<const uint4 *>(ascii + base);
            word = pack_dword(v.x, bad) | (pack_dword(v.y, bad) << 8) |
                   (pack_dword(v.z, bad) << 16) | (pack_dword(v.w, bad) << 24);
        } else {
            for (int k = 0; k < 16; ++k)
                if (base + k < n)
                    word |= base_code(ascii[base + k], bad) << (2 * k);
        }
        out[w] = word;
    }
    if (bad_count) {
        // wave-level sum, one atomic per wave
        for (int off = 32; off > 0; off >>= 1)
            bad += __shfl_xor(bad, off);
        if ((threadIdx.x & 63) == 0 && bad)
            atomicAdd(bad_count, bad);
    }
}

hipError_t launch_pack2b(const uint8_t *ascii, uint64_t n, uint32_t *out, uint32_t *bad,
                         hipStream_t st)
{
    const uint64_t nwords = (n + 15) >> 4;
    if (nwords == 0)
        return hipSuccess;
    uint64_t blocks = (nwords + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    hipLaunchKernelGGL(k_pack2b, dim3((unsigned)blocks), dim3(256), 0, st, ascii, n, out, bad);
    return hipGetLastError();
}

}  // namespace hpgsw
