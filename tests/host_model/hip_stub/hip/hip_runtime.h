// Host stand-in for the few HIP runtime declarations the kernels' sources use,
// so that the unmodified kernel files compile as plain C++ for the CPU models
// (tests/host_model/score_model.cpp, splice_model.cpp, seeker_model.cpp and
// traceback_model.cpp).  Kernel launches compile to nothing; the models call
// the kernel functions themselves, one thread (or one loop step) per lane.
// Cross-lane operations, barriers and the AMDGPU builtins the kernels use are
// declared here and defined by the models.
#pragma once

#include <stdint.h>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...)
// one block runs at a time in the models, so a block's shared arrays can be
// function statics
#define __shared__ static

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };
typedef struct ihipStream_t *hipStream_t;

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
#define hipLaunchKernelGGL(...) ((void)0)
inline hipError_t hipGetLastError() { return hipSuccess; }

struct int2 {
    int x, y;
};
inline int2 make_int2(int x, int y) { return int2{x, y}; }

struct ModelIdx {
    unsigned x, y, z;
};
extern thread_local ModelIdx threadIdx, blockIdx, gridDim, blockDim;

inline int max(int a, int b) { return a > b ? a : b; }
inline int min(int a, int b) { return a < b ? a : b; }
inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline uint64_t min(uint64_t a, uint64_t b) { return a < b ? a : b; }
inline uint64_t max(uint64_t a, uint64_t b) { return a > b ? a : b; }

int model_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl);
int __shfl(int v, int src, int width = 64);
int __shfl_xor(int v, int mask, int width = 64);
uint64_t __shfl_xor(uint64_t v, int mask, int width = 64);
int __shfl_up(int v, unsigned delta, int width = 64);
uint32_t atomicAdd(uint32_t *p, uint32_t v);
uint32_t atomicSub(uint32_t *p, uint32_t v);
unsigned long long atomicCAS(unsigned long long *p, unsigned long long cmp, unsigned long long v);
uint32_t model_perm(uint32_t hi, uint32_t lo, uint32_t sel);
uint32_t model_alignbit(uint32_t hi, uint32_t lo, uint32_t shift);
int model_sbfe(int src, int offset, int width);
#ifdef MODEL_FENCE_HOOK
void __threadfence_block();     // defined by the model (it marks phases of the kernel)
#else
inline void __threadfence_block() {}
#endif
void __syncthreads();
void model_wave_barrier();
uint64_t __ballot(int pred);
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __ffsll(long long x) { return __builtin_ffsll(x); }
inline int __clzll(long long x) { return x ? __builtin_clzll((unsigned long long)x) : 64; }
#define __builtin_amdgcn_wave_barrier model_wave_barrier
#define __builtin_amdgcn_fence(...) __atomic_thread_fence(__ATOMIC_SEQ_CST)

#define __builtin_amdgcn_update_dpp model_update_dpp
#define __builtin_amdgcn_perm model_perm
#define __builtin_amdgcn_alignbit model_alignbit
#define __builtin_amdgcn_sbfe model_sbfe
// v_bitop3_b32: bit k of the result is bit (a_k << 2 | b_k << 1 | c_k) of the table
uint32_t model_bitop3(uint32_t a, uint32_t b, uint32_t c, uint32_t table);
#define __builtin_amdgcn_bitop3_b32 model_bitop3
