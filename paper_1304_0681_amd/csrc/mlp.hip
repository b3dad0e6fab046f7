// Candidate-filter MLP: 64 -> 128 (ReLU) -> 128 (ReLU) -> 1 (logit).
//
// bfloat16 operands, float32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16).  Operand layout of that instruction, per lane l
// of the wave: A[i][k] with i = l % 16, k = 8 * (l / 16) + e (e = 0..7, one
// 8 x bf16 register group); B[k][j] with j = l % 16, k = 8 * (l / 16) + e;
// result D[i][j] in element r of lane l for i = 4 * (l / 16) + r, j = l % 16.
//
// Inference (k_mlp_infer) is one fused kernel: every wave holds both weight
// matrices as MFMA B-fragments in registers for its whole life, streams 16
// candidates per tile, re-lays the hidden activations through a 4 KiB LDS
// tile, and reduces the last layer with lane shuffles.
//
// Training runs on the same matrix instructions through a generic tiled GEMM
// (k_gemm_bf16, one 16 x 16 output tile per wave, fixed-order K loop) plus
// small elementwise kernels; every reduction has a fixed order, so a training
// step is bitwise reproducible.  Rounding points match the reference: weights,
// inputs, hidden activations and the back-propagated dz2/dz1 are bfloat16
// when they enter a product.
#include "internal.h"
#include "mlp_internal.h"

namespace hpgsw {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x)
{
    // round to nearest even (inputs are finite)
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h)
{
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero8()
{
    return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Fused inference.
// ---------------------------------------------------------------------------
constexpr int kInferWaves = 4;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// two floats -> packed bfloat16 pair (round to nearest even, one instruction)
__device__ __forceinline__ uint32_t pk_bf16(float lo, float hi)
{
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// sum over the 16 lanes of a row, left in the row's last lane
__device__ __forceinline__ float row_sum16(float v)
{
    v += __builtin_amdgcn_update_dpp(0.f, v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0.f, v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0.f, v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0.f, v, 0x118, 0xf, 0xf, true);   // row_shr:8
    return v;
}

__global__ void __launch_bounds__(64 * kInferWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_mlp_infer(const MlpDev W, const uint16_t *__restrict__ X, uint32_t n, const uint32_t *d_n,
            float *__restrict__ logits)
{
    __shared__ __attribute__((aligned(16))) uint16_t h1s[kInferWaves][16][kHidden + 8];   // +8: spread LDS banks
    __shared__ float b1s[kHidden], b2s[kHidden], w3s[kHidden];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int li = lane & 15;      // row of A / column of B and D
    const int lk = lane >> 4;      // k group (8 wide) / row group of D
    if (d_n)
        n = min(n, *d_n);
    for (int i = threadIdx.x; i < kHidden; i += 64 * kInferWaves) {
        b1s[i] = W.b1[i];
        b2s[i] = W.b2[i];
        w3s[i] = bf2f(W.w3b[i]);
    }
    __syncthreads();
    // weight fragments: W1T is [128 out][64 in], W2T is [128 out][128 in]
    bf16x8 w1[8][2], w2[8][4];
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
            w1[nt][kk] = load8(W.w1t + (nt * 16 + li) * kIn + kk * 32 + lk * 8);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            w2[nt][kk] = load8(W.w2t + (nt * 16 + li) * kHidden + kk * 32 + lk * 8);
    }
    const float b3 = W.b3[0];
    const uint32_t n_tiles = (n + 15) / 16;
    const uint32_t stride = gridDim.x * kInferWaves;
    uint32_t tile = blockIdx.x * kInferWaves + wv;
    // inputs are loaded two tiles ahead: two register sets take turns
    auto load_x = [&](bf16x8 (&x)[2], uint32_t t) {
        const uint32_t row = t * 16 + li;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
            x[kk] = row < n ? load8(X + (uint64_t)row * kIn + kk * 32 + lk * 8) : zero8();
    };
    auto process = [&](bf16x8 (&xn)[2], uint32_t tile) {
        // layer 1, transposed: D(unit nt*16 + lk*4 + r, sample li) = W1 x^T (the
        // weight fragments serve as the A operand unchanged: same lanes, same
        // k), so each lane holds four consecutive units of one sample and
        // writes them to the sample's LDS row in one 8-byte store
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) {
            const int u0 = nt * 16 + lk * 4;
            f32x4 acc = {b1s[u0], b1s[u0 + 1], b1s[u0 + 2], b1s[u0 + 3]};
            acc = mfma(w1[nt][0], xn[0], acc);
            acc = mfma(w1[nt][1], xn[1], acc);
            const uint32_t h01 = pk_bf16(fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f));
            const uint32_t h23 = pk_bf16(fmaxf(acc[2], 0.f), fmaxf(acc[3], 0.f));
            *reinterpret_cast<uint2 *>(&h1s[wv][li][u0]) = make_uint2(h01, h23);
        }
        // the inputs are consumed: this register set takes the tile two ahead
        if (tile + 2 * stride < n_tiles)
            load_x(xn, tile + 2 * stride);
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): LDS writes done (same wave)
        __builtin_amdgcn_wave_barrier();
        bf16x8 ha[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            ha[kk] = load8(&h1s[wv][li][kk * 32 + lk * 8]);
        // layer 2 and the output unit
        float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) {
            const float b2 = b2s[nt * 16 + li], w3 = w3s[nt * 16 + li];
            f32x4 acc = {b2, b2, b2, b2};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                acc = mfma(ha[kk], w2[nt][kk], acc);
            const uint32_t h01 = pk_bf16(fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f));
            const uint32_t h23 = pk_bf16(fmaxf(acc[2], 0.f), fmaxf(acc[3], 0.f));
            part[0] += __builtin_bit_cast(float, h01 << 16) * w3;
            part[1] += __builtin_bit_cast(float, h01 & 0xFFFF0000u) * w3;
            part[2] += __builtin_bit_cast(float, h23 << 16) * w3;
            part[3] += __builtin_bit_cast(float, h23 & 0xFFFF0000u) * w3;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            part[r] = row_sum16(part[r]);
        if (li == 15) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t rr = tile * 16 + lk * 4 + r;
                if (rr < n)
                    logits[rr] = part[r] + b3;
            }
        }
        __builtin_amdgcn_wave_barrier();   // LDS tile reused by the next tile
    };
    bf16x8 xa[2], xb[2];
    if (tile < n_tiles)
        load_x(xa, tile);
    if (tile + stride < n_tiles)
        load_x(xb, tile + stride);
    for (; tile < n_tiles; tile += 2 * stride) {
        process(xa, tile);
        if (tile + stride < n_tiles)
            process(xb, tile + stride);
    }
}

// ---------------------------------------------------------------------------
// Training building blocks.
// ---------------------------------------------------------------------------

// C[M x N] (f32, row stride ldc) = A[M x K] * B[K x N]; A(i, k) = A[i*lda + k],
// B(k, j) = B[j*ldb + k] (both K-contiguous bf16, 16-byte aligned rows,
// K a multiple of 8).  One wave per 16 x 16 tile.
__global__ void __launch_bounds__(256) k_gemm_bf16(const uint16_t *A, uint32_t lda, const uint16_t *B,
                                                   uint32_t ldb, float *C, uint32_t ldc, uint32_t M,
                                                   uint32_t N, uint32_t K)
{
    const int lane = threadIdx.x & 63;
    const uint32_t tiles_n = (N + 15) / 16;
    const uint32_t tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= tiles_n * ((M + 15) / 16))
        return;
    const uint32_t tm = tile / tiles_n, tn = tile % tiles_n;
    const int li = lane & 15, lk = lane >> 4;
    const uint32_t i = tm * 16 + li, j = tn * 16 + li;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (uint32_t k0 = 0; k0 < K; k0 += 32) {
        const uint32_t k = k0 + lk * 8;
        const bf16x8 a = (i < M && k < K) ? load8(A + (uint64_t)i * lda + k) : zero8();
        const bf16x8 b = (j < N && k < K) ? load8(B + (uint64_t)j * ldb + k) : zero8();
        acc = mfma(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t ii = tm * 16 + lk * 4 + r;
        if (ii < M && j < N)
            C[(uint64_t)ii * ldc + j] = acc[r];
    }
}

// Z (f32 [B x H]) += bias; A = bf16(relu(Z)) row-major and transposed.
__global__ void __launch_bounds__(256) k_bias_relu(float *Z, const float *bias, uint32_t rows,
                                                   uint32_t cols, uint16_t *A, uint16_t *AT,
                                                   uint32_t ldt)
{
    const uint64_t idx = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (uint64_t)rows * cols)
        return;
    const uint32_t r = idx / cols, c = idx % cols;
    const float z = Z[idx] + bias[c];
    Z[idx] = z;
    const uint16_t a = f2bf(fmaxf(z, 0.f));
    A[idx] = a;
    AT[(uint64_t)c * ldt + r] = a;
}

// Output unit and loss: z = a2 . w3 + b3 (fixed order), dz = (sigmoid(z) - y)/B,
// dz2 = bf16(dz * w3 * [z2 > 0]) row-major and transposed; loss terms.
__global__ void __launch_bounds__(256) k_head(const MlpDev W, const uint16_t *A2, const float *Z2,
                                              const float *y, uint32_t B, float *zout, float *dz,
                                              uint16_t *DZ2, uint16_t *DZ2T, uint32_t ldt,
                                              float *lossterm)
{
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B)
        return;
    float z = 0.f;
    for (int j = 0; j < kHidden; ++j)
        z += bf2f(A2[(uint64_t)b * kHidden + j]) * bf2f(W.w3b[j]);
    z += W.b3[0];
    zout[b] = z;
    const float p = 1.f / (1.f + __expf(-z));
    const float d = (p - y[b]) / (float)B;
    dz[b] = d;
    lossterm[b] = fmaxf(z, 0.f) - z * y[b] + log1pf(__expf(-fabsf(z)));
    for (int j = 0; j < kHidden; ++j) {
        const float v = Z2[(uint64_t)b * kHidden + j] > 0.f ? d * bf2f(W.w3b[j]) : 0.f;
        const uint16_t h = f2bf(v);
        DZ2[(uint64_t)b * kHidden + j] = h;
        DZ2T[(uint64_t)j * ldt + b] = h;
    }
}

// dz1 = bf16(da1 * [z1 > 0]) row-major (unused) and transposed.
__global__ void __launch_bounds__(256) k_relu_back(const float *DA, const float *Z, uint32_t rows,
                                                   uint32_t cols, uint16_t *DT, uint32_t ldt)
{
    const uint64_t idx = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (uint64_t)rows * cols)
        return;
    const uint32_t r = idx / cols, c = idx % cols;
    DT[(uint64_t)c * ldt + r] = f2bf(Z[idx] > 0.f ? DA[idx] : 0.f);
}

// Column sums of a transposed bf16 matrix DT [cols][ldt] over its first `rows`
// entries, times w[r] when w is given (bias gradients; dw3 = a2^T dz).  One wave
// per column: lane l adds rows l, l + 64, ... in order, then an xor butterfly
// combines the lanes.  The order of every addition depends only on `rows`, so
// the result is reproducible bit for bit.
__global__ void __launch_bounds__(256) k_colsum_t(const uint16_t *DT, uint32_t ldt, uint32_t rows,
                                                  uint32_t cols, const float *w, float *out)
{
    const uint32_t c = blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    if (c >= cols)      // wave-uniform
        return;
    const uint16_t *col = DT + (uint64_t)c * ldt;
    float s = 0.f;
    for (uint32_t r = lane; r < rows; r += 64)
        s += bf2f(col[r]) * (w ? w[r] : 1.f);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_xor(s, off);
    if (lane == 0)
        out[c] = s;
}

// out[0] = (sum of x[0..n)) / div, one wave, in the same fixed order
__global__ void __launch_bounds__(64) k_sum_div(const float *x, uint32_t n, float div, float *out)
{
    const uint32_t lane = threadIdx.x & 63;
    float s = 0.f;
    for (uint32_t r = lane; r < n; r += 64)
        s += x[r];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_xor(s, off);
    if (lane == 0)
        out[0] = s / div;
}

// X (bf16 [B x 64]) -> XT [64 x ldt]
__global__ void __launch_bounds__(256) k_transpose_x(const uint16_t *X, uint32_t B, uint16_t *XT,
                                                     uint32_t ldt)
{
    const uint64_t idx = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (uint64_t)B * kIn)
        return;
    const uint32_t r = idx / kIn, c = idx % kIn;
    XT[(uint64_t)c * ldt + r] = X[idx];
}

// gradient matrices from GEMM outputs [out-major] into the parameter layout
// (W1 [in][out], W2 [in][out]): g[i*H + o] = G[o*ld + i]
__global__ void __launch_bounds__(256) k_scatter_grad(const float *G, uint32_t ld, uint32_t n_in,
                                                      float *g)
{
    const uint32_t idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= n_in * kHidden)
        return;
    const uint32_t i = idx / kHidden, o = idx % kHidden;
    g[idx] = G[(uint64_t)o * ld + i];
}

__global__ void __launch_bounds__(256) k_adam(float *theta, float *m, float *v, const float *g,
                                              uint32_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// float32 master parameters -> bf16 operand copies (W1T, W2T, W2, w3)
__global__ void __launch_bounds__(256) k_cast_params(const float *theta, MlpDev W)
{
    const uint32_t idx = blockIdx.x * 256 + threadIdx.x;
    if (idx < kIn * kHidden) {
        const uint32_t i = idx / kHidden, o = idx % kHidden;
        W.w1t[o * kIn + i] = f2bf(theta[kOffW1 + idx]);
    }
    if (idx < kHidden * kHidden) {
        const uint32_t i = idx / kHidden, o = idx % kHidden;
        const uint16_t h = f2bf(theta[kOffW2 + idx]);
        W.w2t[o * kHidden + i] = h;
        W.w2[idx] = h;
    }
    if (idx < kHidden)
        W.w3b[idx] = f2bf(theta[kOffW3 + idx]);
}

// ---------------------------------------------------------------------------
// Labels, read segments, filter decision, compaction.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_labels(uint32_t n_pairs, const sw_window *win,
                                                uint32_t n_reads, const sw_hit *hits,
                                                const int32_t *best, int32_t margin,
                                                int32_t min_best, float *y)
{
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n_pairs)
        return;
    const int s = hits[p].score;
    const uint32_t r = win[p].read_id;
    // a pair of no read scores -1 and is labelled 0 without a best score
    const int bs = r < n_reads ? best[r] : 0;
    y[p] = (r < n_reads && s >= 0 && s >= bs - margin && bs >= min_best) ? 1.f : 0.f;
}

__global__ void __launch_bounds__(256) k_seg_init(uint32_t n_reads, uint32_t *first, uint32_t *last,
                                                  uint32_t *count)
{
    const uint32_t r = blockIdx.x * 256 + threadIdx.x;
    if (r < n_reads) {
        first[r] = 0xFFFFFFFFu;
        last[r] = 0;
        count[r] = 0;
    }
}

// Runs of equal read ids: a read's first pair (min over its run starts), last
// pair (max over run ends) and number of runs; atomics only at run boundaries.
__global__ void __launch_bounds__(256) k_seg(uint32_t n_pairs, const uint32_t *d_n, const sw_window *win,
                                             uint32_t n_reads, uint32_t *first, uint32_t *last,
                                             uint32_t *runs)
{
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    if (d_n)
        n_pairs = min(n_pairs, *d_n);
    if (p >= n_pairs)
        return;
    const uint32_t r = win[p].read_id;
    if (r >= n_reads)
        return;
    if (p == 0 || win[p - 1].read_id != r) {
        atomicMin(first + r, p);
        atomicAdd(runs + r, 1u);
    }
    if (p + 1 == n_pairs || win[p + 1].read_id != r)
        atomicMax(last + r, p);
}

// count = pairs of a read stored in one run; a read split over several runs gets
// 0xFFFFFFFF, which fails every contiguity test (its pairs are all kept)
__global__ void __launch_bounds__(256) k_seg_final(uint32_t n_reads, const uint32_t *first,
                                                   const uint32_t *last, uint32_t *count)
{
    const uint32_t r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n_reads)
        return;
    const uint32_t runs = count[r];
    count[r] = runs == 0 ? 0u : (runs == 1 ? last[r] - first[r] + 1 : 0xFFFFFFFFu);
}

// Per read: keep all candidates when unsure (best logit below hi, or any
// logit in [lo, hi)), else the candidates with logit >= hi.  Reads whose
// pairs are not contiguous, or that have more than kMaxCand candidates, keep
// everything.
__global__ void __launch_bounds__(256) k_decide(uint32_t n_reads, const uint32_t *first,
                                                const uint32_t *last, const uint32_t *count,
                                                const float *logits, float lo, float hi,
                                                float drop, uint8_t *keep, uint32_t *n_unsure)
{
    const uint32_t r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n_reads || count[r] == 0)
        return;
    const uint32_t a = first[r], k = count[r];
    const bool contiguous = last[r] - a + 1 == k;
    bool unsure = !contiguous || k > kMaxCand;
    float mx = -INFINITY;
    if (!unsure) {
        for (uint32_t c = 0; c < k; ++c) {
            const float z = logits[a + c];
            mx = fmaxf(mx, z);
            unsure |= (z >= lo && z < hi);
        }
        if (mx < drop) {       // predicted unmapped: no candidate is aligned
            for (uint32_t c = 0; c < k; ++c)
                keep[a + c] = 0;
            return;
        }
        unsure |= mx < hi;
    }
    if (unsure) {
        if (contiguous)
            for (uint32_t c = 0; c < k; ++c)
                keep[a + c] = 1;
        atomicAdd(n_unsure, 1u);
        return;
    }
    for (uint32_t c = 0; c < k; ++c)
        keep[a + c] = logits[a + c] >= hi ? 1 : 0;
}

__global__ void k_zero_count(uint32_t *p)
{
    if (threadIdx.x == 0)
        *p = 0;
}

// non-contiguous reads: keep every pair of those reads
__global__ void __launch_bounds__(256) k_keep_noncontig(uint32_t n_pairs, const sw_window *win,
                                                        uint32_t n_reads, const uint32_t *first,
                                                        const uint32_t *last, const uint32_t *count,
                                                        uint8_t *keep)
{
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n_pairs)
        return;
    const uint32_t r = win[p].read_id;
    if (r >= n_reads)
        keep[p] = 0;
    else if (last[r] - first[r] + 1 != count[r])
        keep[p] = 1;
}

constexpr int kScanItems = 4096;   // pairs per block of the compaction scan

__global__ void __launch_bounds__(256) k_block_count(uint32_t n, const uint8_t *keep, uint32_t *bcount)
{
    __shared__ uint32_t part[256];
    const uint64_t base = (uint64_t)blockIdx.x * kScanItems;
    uint32_t s = 0;
    for (int k = threadIdx.x; k < kScanItems; k += 256)
        if (base + k < n)
            s += keep[base + k];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        bcount[blockIdx.x] = part[0];
}

__global__ void __launch_bounds__(1024) k_scan_blocks(uint32_t nb, uint32_t *bcount, uint32_t *total)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const uint32_t per = (nb + 1023) / 1024;
    uint32_t s = 0;
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t i = t * per + k;
        if (i < nb)
            s += bcount[i];
    }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t i = t * per + k;
        if (i < nb) {
            const uint32_t c = bcount[i];
            bcount[i] = run;
            run += c;
        }
    }
    if (t == 1023)
        total[0] = part[1023];
}

// stable compaction: kept pairs in input order
__global__ void __launch_bounds__(256) k_compact(uint32_t n, const uint8_t *keep, const uint32_t *boff,
                                                 const sw_window *win, sw_window *wout,
                                                 uint32_t *ids_out)
{
    __shared__ uint32_t part[256];
    const uint64_t base = (uint64_t)blockIdx.x * kScanItems;
    constexpr int PER = kScanItems / 256;   // 16 consecutive items per thread
    const uint64_t my = base + (uint64_t)threadIdx.x * PER;
    uint32_t s = 0;
    for (int k = 0; k < PER; ++k)
        if (my + k < n)
            s += keep[my + k];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t pos = boff[blockIdx.x] + part[threadIdx.x] - s;
    for (int k = 0; k < PER; ++k) {
        const uint64_t p = my + k;
        if (p < n && keep[p]) {
            wout[pos] = win[p];
            ids_out[pos] = (uint32_t)p;
            ++pos;
        }
    }
}

// Columns [B, ldt) of row blockIdx.x of a transposed operand (the K padding).
__global__ void __launch_bounds__(64) k_zero_pad(uint16_t *T, uint32_t B, uint32_t ldt)
{
    for (uint32_t c = B + threadIdx.x; c < ldt; c += 64)
        T[(uint64_t)blockIdx.x * ldt + c] = 0;
}

unsigned blocks_for(uint64_t n)
{
    const uint64_t b = (n + 255) / 256;
    return (unsigned)(b ? b : 1);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers.
// ---------------------------------------------------------------------------
hipError_t mlp_cast_params(const float *theta, const MlpDev &W, hipStream_t st)
{
    hipLaunchKernelGGL(k_cast_params, dim3(blocks_for(kHidden * kHidden)), dim3(256), 0, st, theta, W);
    return hipGetLastError();
}

hipError_t mlp_infer(const MlpDev &W, const uint16_t *X, uint32_t n, const uint32_t *d_n,
                     float *logits, int n_cu, hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    const uint32_t tiles = (n + 15) / 16;
    uint32_t blocks = (tiles + kInferWaves - 1) / kInferWaves;
    const uint32_t cap = (uint32_t)n_cu * 2;   // two waves per SIMD fit the register file
    if (blocks > cap)
        blocks = cap;
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks), dim3(64 * kInferWaves), 0, st, W, X, n, d_n, logits);
    return hipGetLastError();
}

hipError_t mlp_gemm(const uint16_t *A, uint32_t lda, const uint16_t *B, uint32_t ldb, float *C,
                    uint32_t ldc, uint32_t M, uint32_t N, uint32_t K, hipStream_t st)
{
    const uint32_t tiles = ((M + 15) / 16) * ((N + 15) / 16);
    hipLaunchKernelGGL(k_gemm_bf16, dim3((tiles + 3) / 4), dim3(256), 0, st, A, lda, B, ldb, C, ldc,
                       M, N, K);
    return hipGetLastError();
}

// One forward/backward pass of a minibatch; fills grad (parameter layout) and
// loss (device scalars).  ws: workspace laid out by mlp_workspace_bytes.
hipError_t mlp_backprop(const MlpDev &W, const uint16_t *X, const float *y, uint32_t B, float *grad,
                        float *loss, void *ws, hipStream_t st)
{
    const uint32_t ldt = (B + 31) / 32 * 32;    // transposed leading dimension, K padding
    char *p = static_cast<char *>(ws);
    auto take = [&](size_t bytes) { void *r = p; p += (bytes + 255) & ~size_t(255); return r; };
    float *Z1 = (float *)take(4ull * B * kHidden);
    float *Z2 = (float *)take(4ull * B * kHidden);
    float *DA1 = (float *)take(4ull * B * kHidden);
    uint16_t *A1 = (uint16_t *)take(2ull * B * kHidden);
    uint16_t *A2 = (uint16_t *)take(2ull * B * kHidden);
    uint16_t *A1T = (uint16_t *)take(2ull * kHidden * ldt);
    uint16_t *A2T = (uint16_t *)take(2ull * kHidden * ldt);
    uint16_t *DZ2 = (uint16_t *)take(2ull * B * kHidden);
    uint16_t *DZ2T = (uint16_t *)take(2ull * kHidden * ldt);
    uint16_t *DZ1T = (uint16_t *)take(2ull * kHidden * ldt);
    uint16_t *XT = (uint16_t *)take(2ull * kIn * ldt);
    float *z = (float *)take(4ull * B);
    float *dz = (float *)take(4ull * B);
    float *terms = (float *)take(4ull * B);
    float *GW = (float *)take(4ull * kHidden * kHidden);
    // zero the K padding of the transposed operands (a kernel, not memset nodes)
    hipError_t e;
    if (ldt != B) {
        for (uint16_t *q : {A1T, A2T, DZ2T, DZ1T})
            hipLaunchKernelGGL(k_zero_pad, dim3(kHidden), dim3(64), 0, st, q, B, ldt);
        hipLaunchKernelGGL(k_zero_pad, dim3(kIn), dim3(64), 0, st, XT, B, ldt);
    }
    const uint64_t bh = (uint64_t)B * kHidden;
    // forward
    hipLaunchKernelGGL(k_transpose_x, dim3(blocks_for((uint64_t)B * kIn)), dim3(256), 0, st, X, B, XT, ldt);
    if ((e = mlp_gemm(X, kIn, W.w1t, kIn, Z1, kHidden, B, kHidden, kIn, st))) return e;
    hipLaunchKernelGGL(k_bias_relu, dim3(blocks_for(bh)), dim3(256), 0, st, Z1, W.b1, B, kHidden, A1, A1T, ldt);
    if ((e = mlp_gemm(A1, kHidden, W.w2t, kHidden, Z2, kHidden, B, kHidden, kHidden, st))) return e;
    hipLaunchKernelGGL(k_bias_relu, dim3(blocks_for(bh)), dim3(256), 0, st, Z2, W.b2, B, kHidden, A2, A2T, ldt);
    hipLaunchKernelGGL(k_head, dim3(blocks_for(B)), dim3(256), 0, st, W, A2, Z2, y, B, z, dz, DZ2, DZ2T, ldt, terms);
    hipLaunchKernelGGL(k_sum_div, dim3(1), dim3(64), 0, st, terms, B, (float)B, loss);
    // backward
    hipLaunchKernelGGL(k_colsum_t, dim3(kHidden / 4), dim3(256), 0, st, A2T, ldt, B, kHidden, dz,
                       grad + kOffW3);
    hipLaunchKernelGGL(k_sum_div, dim3(1), dim3(64), 0, st, dz, B, 1.f, grad + kOffB3);
    hipLaunchKernelGGL(k_colsum_t, dim3(kHidden / 4), dim3(256), 0, st, DZ2T, ldt, B, kHidden,
                       (const float *)nullptr, grad + kOffB2);
    // dW2^T[o][i] = sum_b dz2[b][o] a1[b][i]
    if ((e = mlp_gemm(DZ2T, ldt, A1T, ldt, GW, kHidden, kHidden, kHidden, ldt, st))) return e;
    hipLaunchKernelGGL(k_scatter_grad, dim3(blocks_for(kHidden * kHidden)), dim3(256), 0, st, GW, kHidden, kHidden, grad + kOffW2);
    // da1[b][i] = sum_o dz2[b][o] W2[i][o]
    if ((e = mlp_gemm(DZ2, kHidden, W.w2, kHidden, DA1, kHidden, B, kHidden, kHidden, st))) return e;
    hipLaunchKernelGGL(k_relu_back, dim3(blocks_for(bh)), dim3(256), 0, st, DA1, Z1, B, kHidden, DZ1T, ldt);
    hipLaunchKernelGGL(k_colsum_t, dim3(kHidden / 4), dim3(256), 0, st, DZ1T, ldt, B, kHidden,
                       (const float *)nullptr, grad + kOffB1);
    // dW1^T[o][i] = sum_b dz1[b][o] x[b][i]
    if ((e = mlp_gemm(DZ1T, ldt, XT, ldt, GW, kIn, kHidden, kIn, ldt, st))) return e;
    hipLaunchKernelGGL(k_scatter_grad, dim3(blocks_for(kIn * kHidden)), dim3(256), 0, st, GW, kIn, kIn, grad + kOffW1);
    return hipGetLastError();
}

size_t mlp_workspace_bytes(uint32_t B)
{
    const size_t ldt = (B + 31) / 32 * 32;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    return 3 * al(4ull * B * kHidden) + 2 * al(2ull * B * kHidden) + 2 * al(2ull * kHidden * ldt) +
           al(2ull * B * kHidden) + 2 * al(2ull * kHidden * ldt) + al(2ull * kIn * ldt) +
           3 * al(4ull * B) + al(4ull * kHidden * kHidden);
}

hipError_t mlp_adam(float *theta, float *m, float *v, const float *g, float lr, int step,
                    hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(kParams)), dim3(256), 0, st, theta, m, v, g,
                       (uint32_t)kParams, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_labels(uint32_t n_pairs, const sw_window *win, uint32_t n_reads, const sw_hit *hits,
                      const int32_t *best, int32_t margin, int32_t min_best, float *y, hipStream_t st)
{
    if (n_pairs)
        hipLaunchKernelGGL(k_labels, dim3(blocks_for(n_pairs)), dim3(256), 0, st, n_pairs, win,
                           n_reads, hits, best, margin, min_best, y);
    return hipGetLastError();
}

hipError_t read_segments(uint32_t n_pairs, const uint32_t *d_n, const sw_window *win,
                         uint32_t n_reads, uint32_t *first, uint32_t *last, uint32_t *count,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_seg_init, dim3(blocks_for(n_reads)), dim3(256), 0, st, n_reads, first, last, count);
    if (n_pairs)
        hipLaunchKernelGGL(k_seg, dim3(blocks_for(n_pairs)), dim3(256), 0, st, n_pairs, d_n, win,
                           n_reads, first, last, count);
    hipLaunchKernelGGL(k_seg_final, dim3(blocks_for(n_reads)), dim3(256), 0, st, n_reads, first, last, count);
    return hipGetLastError();
}

hipError_t filter_decide(uint32_t n_pairs, const sw_window *win, uint32_t n_reads,
                         const uint32_t *first, const uint32_t *last, const uint32_t *count,
                         const float *logits, float lo, float hi, float drop, uint8_t *keep,
                         uint32_t *n_unsure, hipStream_t st)
{
    hipLaunchKernelGGL(k_decide, dim3(blocks_for(n_reads)), dim3(256), 0, st, n_reads, first, last,
                       count, logits, lo, hi, drop, keep, n_unsure);
    hipLaunchKernelGGL(k_keep_noncontig, dim3(blocks_for(n_pairs)), dim3(256), 0, st, n_pairs, win,
                       n_reads, first, last, count, keep);
    return hipGetLastError();
}

size_t compact_scratch_words(uint32_t n) { return (n + kScanItems - 1) / kScanItems + 1; }

hipError_t compact_pairs(uint32_t n, const uint8_t *keep, const sw_window *win, sw_window *wout,
                         uint32_t *ids_out, uint32_t *d_n_out, uint32_t *scratch, hipStream_t st)
{
    const uint32_t nb = (n + kScanItems - 1) / kScanItems;
    if (nb == 0) {      // a kernel, not a memset node, so that the call can be captured
        hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, st, d_n_out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_block_count, dim3(nb), dim3(256), 0, st, n, keep, scratch);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, nb, scratch, d_n_out);
    hipLaunchKernelGGL(k_compact, dim3(nb), dim3(256), 0, st, n, keep, scratch, win, wout, ids_out);
    return hipGetLastError();
}

}  // namespace hpgsw
