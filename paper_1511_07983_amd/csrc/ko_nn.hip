// libko_nn: the learned launch-order surrogate (include/ko_nn.h) on gfx950.
//
// One generic BF16 MFMA GEMM (v_mfma_f32_16x16x32_bf16, float32 accumulate)
// with strided operands and fused epilogues carries every product of the
// forward and backward passes; small kernels do pooling, the output layer,
// the loss, column sums and Adam.  All reductions are deterministic (no
// floating-point atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "ko_nn.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kHid = KO_NN_HID;
constexpr int kIn = KO_NN_IN;

// flat parameter offsets
constexpr size_t kW1 = 0;
constexpr size_t kB1 = kW1 + (size_t)kHid * kIn;
constexpr size_t kW2 = kB1 + kHid;
constexpr size_t kB2 = kW2 + (size_t)kHid * kHid;
constexpr size_t kW3 = kB2 + kHid;
constexpr size_t kB3 = kW3 + (size_t)kHid * kHid;
constexpr size_t kW4 = kB3 + kHid;
constexpr size_t kB4 = kW4 + kHid;
constexpr size_t kNP = kB4 + 1;                  // 140289
static_assert(kB4 == kW4 + kHid, "db4 follows dw4");
constexpr size_t kNPad = (kNP + 63) / 64 * 64;   // 140352

struct State {
    float *master, *grad, *m, *v;
    uint16_t *wb;
};

State state_of(void *p)
{
    State s;
    char *c = (char *)p;
    s.master = (float *)c;
    s.grad = s.master + kNPad;
    s.m = s.grad + kNPad;
    s.v = s.m + kNPad;
    s.wb = (uint16_t *)(s.v + kNPad);
    return s;
}

__host__ __device__ inline uint16_t to_bf16(float f)
{
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Two floats to BF16 (round to nearest even, as to_bf16 for every finite
// value) in one conversion instruction; lo in bits 0..15.
__device__ inline uint32_t pack_bf16x2(float lo, float hi)
{
    const bf16x2 h = __builtin_convertvector(f32x2{lo, hi}, bf16x2);
    uint32_t u;
    __builtin_memcpy(&u, &h, 4);
    return u;
}

__device__ inline float from_bf16(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// ------------------------------------------------------------------ GEMM
//
// C[m][n] = sum_k A(m,k) B(k,n) with A(m,k) = A[m*sam + k*sak] and
// B(k,n) = B[k*sbk + n*sbn] (BF16), a 64x64 tile per workgroup of 4 waves,
// each wave a 32x32 block of 2x2 MFMA 16x16x32 tiles, K in steps of 32
// staged through LDS (rows padded to 40 elements).
enum { kEpiNone = 0, kEpiRelu = 1, kEpiMask = 2 };

struct GemmArgs {
    const uint16_t *A;
    int64_t sam, sak;
    const uint16_t *B;
    int64_t sbk, sbn;
    int32_t M, N, K;
    int32_t epi;
    const float *bias;   // [N] or null
    const float *zref;   // kEpiMask: mask source, row-major with ldz
    int64_t ldz;
    float *C;            // fp32 result, row-major with ldc (or null)
    int64_t ldc;
    uint16_t *Cb;        // bf16 result (relu(C) for kEpiRelu), row-major with ldcb (or null)
    int64_t ldcb;
    // split-K: workgroup z sums k in [z*kchunk, (z+1)*kchunk) and stores its raw
    // partial product to P + z*M*N (row-major, N columns); a second kernel adds
    // the partials in z order, so the result does not depend on scheduling
    float *P;            // null = no split
    int64_t kchunk;
};

constexpr int kTile = 64;
constexpr int kKStep = 32;
constexpr int kPad = 40;

__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kTile][kPad];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kTile][kPad];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.x * kTile;
    const int64_t n0 = (int64_t)blockIdx.y * kTile;
    const int64_t kb = a.P ? (int64_t)blockIdx.z * a.kchunk : 0;
    const int64_t ke = a.P ? min((int64_t)a.K, kb + a.kchunk) : (int64_t)a.K;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++)
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int lr = tid >> 2;         // tile row (A) / tile column (B) loaded by this thread
    const int lk = (tid & 3) * 8;    // first of its 8 k values
    for (int64_t k0 = kb; k0 < ke; k0 += kKStep) {
        {
            const int64_t m = m0 + lr;
            for (int e = 0; e < 8; e++) {
                const int64_t k = k0 + lk + e;
                As[lr][lk + e] = (m < a.M && k < ke) ? a.A[m * a.sam + k * a.sak] : (uint16_t)0;
            }
            const int64_t n = n0 + lr;
            for (int e = 0; e < 8; e++) {
                const int64_t k = k0 + lk + e;
                Bs[lr][lk + e] = (n < a.N && k < ke) ? a.B[k * a.sbk + n * a.sbn] : (uint16_t)0;
            }
        }
        __syncthreads();
        const int kk = (lane >> 4) * 8;
        bf16x8 af[2], bfr[2];
        for (int i = 0; i < 2; i++)
            af[i] = *reinterpret_cast<const bf16x8 *>(&As[wm * 32 + i * 16 + (lane & 15)][kk]);
        for (int j = 0; j < 2; j++)
            bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wn * 32 + j * 16 + (lane & 15)][kk]);
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++)
            for (int e = 0; e < 4; e++) {
                const int64_t row = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + e;
                const int64_t col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row >= a.M || col >= a.N)
                    continue;
                float v = acc[i][j][e];
                if (a.P) {
                    a.P[(int64_t)blockIdx.z * a.M * a.N + row * a.N + col] = v;
                    continue;
                }
                if (a.epi == kEpiMask) {
                    v = (a.zref[row * a.ldz + col] > 0.f) ? v : 0.f;
                } else if (a.bias) {
                    v += a.bias[col];
                }
                if (a.C)
                    a.C[row * a.ldc + col] = v;
                if (a.Cb)
                    a.Cb[row * a.ldcb + col] = to_bf16(a.epi == kEpiRelu ? fmaxf(v, 0.f) : v);
            }
}

// The product of every forward and scoring layer, C = A W^T with A [M][K]
// and W [N][K] both contiguous along K (sak = sbk = 1): 128 x 128 tiles of 4
// waves, each wave a 64 x 64 block of 4 x 4 MFMA 16x16x32 tiles, K in steps of
// 32 staged through LDS with 16-byte loads (rows padded to 40 elements).
// Needs K % 32 == 0, N % 128 == 0, row pitches and base addresses aligned to
// 16 bytes; gemm() checks this and uses gemm_bf16_kernel otherwise.
constexpr int kNtTile = 128;

__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kNtTile][kPad];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kNtTile][kPad];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.x * kNtTile;
    const int64_t n0 = (int64_t)blockIdx.y * kNtTile;
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++)
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t k0 = 0; k0 < a.K; k0 += kKStep) {
        // 128 rows x 4 chunks of 8 elements per operand: two chunks per thread
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int idx = tid + h * 256;
            const int r = idx >> 2, c = (idx & 3) * 8;
            const int64_t m = m0 + r;
            uint4 va = make_uint4(0u, 0u, 0u, 0u);
            if (m < a.M)
                va = *reinterpret_cast<const uint4 *>(a.A + m * a.sam + k0 + c);
            *reinterpret_cast<uint4 *>(&As[r][c]) = va;
            const int64_t n = n0 + r;
            uint4 vb = make_uint4(0u, 0u, 0u, 0u);
            if (n < a.N)
                vb = *reinterpret_cast<const uint4 *>(a.B + n * a.sbn + k0 + c);
            *reinterpret_cast<uint4 *>(&Bs[r][c]) = vb;
        }
        __syncthreads();
        const int kk = (lane >> 4) * 8;
        bf16x8 af[4], bfr[4];
#pragma unroll
        for (int i = 0; i < 4; i++)
            af[i] = *reinterpret_cast<const bf16x8 *>(&As[wm * 64 + i * 16 + (lane & 15)][kk]);
#pragma unroll
        for (int j = 0; j < 4; j++)
            bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wn * 64 + j * 16 + (lane & 15)][kk]);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int64_t row = m0 + wm * 64 + i * 16 + (lane >> 4) * 4 + e;
                const int64_t col = n0 + wn * 64 + j * 16 + (lane & 15);
                if (row >= a.M || col >= a.N)
                    continue;
                float v = acc[i][j][e];
                if (a.epi == kEpiMask) {
                    v = (a.zref[row * a.ldz + col] > 0.f) ? v : 0.f;
                } else if (a.bias) {
                    v += a.bias[col];
                }
                if (a.C)
                    a.C[row * a.ldc + col] = v;
                if (a.Cb)
                    a.Cb[row * a.ldcb + col] = to_bf16(a.epi == kEpiRelu ? fmaxf(v, 0.f) : v);
            }
}

// The products of a training step, whose reductions are short: the whole K
// range of a workgroup (at most 256, a split-K chunk or a layer's width) is
// staged into LDS in one load phase, with every global load of the panel in
// flight at once, and then consumed by the MFMAs without further global
// round trips.  64 x 64 output tiles of 4 waves (each 32 x 32, 2 x 2 MFMA
// 16x16x32 tiles), so a 4096 x 256 product runs on 256 workgroups.
//
// An operand is k-contiguous (KC: element (r, k) at P[r * sr + k], 16-byte
// loads along k stored as they are) or r-contiguous (element (r, k) at
// P[k * sk + r]: 16-byte loads of 8 rows at one k, written transposed into
// the LDS tile, where the 64 lanes of a wave take 64 consecutive k so that
// their 2-byte writes fall into distinct dwords).  Either way every element
// of the 64 x 256 tile is written, zero outside the operand and past kw, so
// the MFMAs of a partial last k step add zeros.  The MFMA operands, the
// k order of the accumulation and the epilogue are those of gemm_bf16_kernel,
// so every output equals that kernel's bit for bit.
constexpr int kPanelK = 256;
constexpr int kPanelPitch = kPanelK + 8;   // elements; 132 dwords per row

template <bool KC>
__device__ __forceinline__ void load_panel(const uint16_t *P, int64_t sr, int64_t sk, int64_t r0, int32_t R,
                                           int64_t k0, int32_t kw, uint16_t (*S)[kPanelPitch])
{
    const int tid = threadIdx.x;
    uint4 v[8];
    if (KC) {
        // 64 rows x 32 chunks of 8 k: chunk c = tid + 256 i is row c / 32, k (c % 32) * 8
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int c = tid + 256 * i;
            const int r = c >> 5, kc = (c & 31) * 8;
            v[i] = make_uint4(0u, 0u, 0u, 0u);
            if (r0 + r < R && kc < kw)
                v[i] = *reinterpret_cast<const uint4 *>(P + (r0 + r) * sr + k0 + kc);
        }
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int c = tid + 256 * i;
            *reinterpret_cast<uint4 *>(&S[c >> 5][(c & 31) * 8]) = v[i];
        }
    } else {
        // thread t takes k = t and the 8 chunks of 8 rows at that k
#pragma unroll
        for (int i = 0; i < 8; i++) {
            v[i] = make_uint4(0u, 0u, 0u, 0u);
            if (tid < kw && r0 + 8 * i < R)
                v[i] = *reinterpret_cast<const uint4 *>(P + (k0 + tid) * sk + r0 + 8 * i);
        }
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint32_t w[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
            for (int e = 0; e < 8; e++)
                S[8 * i + e][tid] = (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
        }
    }
}

template <bool AK, bool BK>
__global__ __launch_bounds__(256) void panel_gemm_kernel(GemmArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kTile][kPanelPitch];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kTile][kPanelPitch];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.x * kTile;
    const int64_t n0 = (int64_t)blockIdx.y * kTile;
    const int64_t kb = a.P ? (int64_t)blockIdx.z * a.kchunk : 0;
    const int64_t ke = a.P ? min((int64_t)a.K, kb + a.kchunk) : (int64_t)a.K;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kk = (lane >> 4) * 8;
    for (int64_t p0 = kb; p0 < ke; p0 += kPanelK) {
        const int kw = (int)min((int64_t)kPanelK, ke - p0);
        const int ksteps = (kw + kKStep - 1) / kKStep;
        // A(m, k): k-contiguous rows of pitch sam, or m-contiguous rows of pitch sak
        load_panel<AK>(a.A, a.sam, a.sak, m0, a.M, p0, kw, As);
        load_panel<BK>(a.B, a.sbn, a.sbk, n0, a.N, p0, kw, Bs);
        __syncthreads();
        for (int ks = 0; ks < ksteps; ks++) {
            bf16x8 af[2], bfr[2];
#pragma unroll
            for (int i = 0; i < 2; i++)
                af[i] = *reinterpret_cast<const bf16x8 *>(&As[wm * 32 + i * 16 + (lane & 15)][ks * kKStep + kk]);
#pragma unroll
            for (int j = 0; j < 2; j++)
                bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wn * 32 + j * 16 + (lane & 15)][ks * kKStep + kk]);
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int64_t row = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + e;
                const int64_t col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row >= a.M || col >= a.N)
                    continue;
                float v = acc[i][j][e];
                if (a.P) {
                    a.P[(int64_t)blockIdx.z * a.M * a.N + row * a.N + col] = v;
                    continue;
                }
                if (a.epi == kEpiMask) {
                    v = (a.zref[row * a.ldz + col] > 0.f) ? v : 0.f;
                } else if (a.bias) {
                    v += a.bias[col];
                }
                if (a.C)
                    a.C[row * a.ldc + col] = v;
                if (a.Cb)
                    a.Cb[row * a.ldcb + col] = to_bf16(a.epi == kEpiRelu ? fmaxf(v, 0.f) : v);
            }
}

// ------------------------------------------------------------------ small kernels

// S[b][c] = sum_j relu(Z1[b*n+j][c]); also its BF16 copy, and the count of
// the sample's tokens with Z1 > 0 in column c (the bias gradient db1 is the
// column sum of dS times that count).
__global__ void pool_kernel(const float *Z1, int32_t B, int32_t n, float *S, uint16_t *Sb, uint8_t *cnt)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * kHid)
        return;
    const int64_t b = idx / kHid, c = idx % kHid;
    float s = 0.f;
    int k = 0;
    for (int j = 0; j < n; j++) {
        const float z = Z1[(b * n + j) * kHid + c];
        s += fmaxf(z, 0.f);
        k += z > 0.f;
    }
    S[idx] = s;
    Sb[idx] = to_bf16(s);
    cnt[idx] = (uint8_t)k;
}

__device__ inline float wave_sum(float v)
{
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

// Deterministic block sum (256 threads) of v; valid in thread 0.
__device__ inline float block_sum(float v, float *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        red[wave] = v;
    __syncthreads();
    float t = 0.f;
    if (threadIdx.x == 0)
        t = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return t;
}

// y[b] = A3b[b] . w4b + b4 (one wave per sample).
__global__ __launch_bounds__(256) void out_forward_kernel(const uint16_t *A3b, const uint16_t *wb,
                                                          const float *master, int32_t B, float *y)
{
    // the wave index is uniform across the wave: the early return stays a
    // scalar branch and the shuffles of wave_sum run with all lanes active
    const int64_t b = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= B)
        return;
    float s = 0.f;
    for (int c = lane; c < kHid; c += 64)
        s += from_bf16(A3b[b * kHid + c]) * from_bf16(wb[kW4 + c]);
    s = wave_sum(s);
    if (lane == 0)
        y[b] = s + master[kB4];
}

// The output layer, forward and backward, one wave per sample: y = A3b . w4b
// + b4 (the sum of out_forward_kernel), d = y - t, dy = 2 d / B, the squared
// error d^2 (the loss is their column sum), and dZ3 = dy w4b [Z3 > 0] in
// float32 and BF16.  With `sched` set, the first thread advances the step
// counter: the step's later kernels (the Adam update) read the new value and
// the step's earlier ones (minibatch selection) have read the old one.
__global__ __launch_bounds__(256) void head_kernel(const uint16_t *A3b, const uint16_t *wb, const float *master,
                                                   const float *Z3, const float *t, int32_t B, float *y,
                                                   float *dy, float *sq, float *dZ3, uint16_t *dZ3b,
                                                   ko_nn_sched *sched)
{
    if (sched && blockIdx.x == 0 && threadIdx.x == 0)
        sched->step += 1;
    // the wave index is uniform across the wave (see out_forward_kernel)
    const int64_t b = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= B)
        return;
    float s = 0.f;
    for (int c = lane; c < kHid; c += 64)
        s += from_bf16(A3b[b * kHid + c]) * from_bf16(wb[kW4 + c]);
    // the xor butterfly leaves the same sum, bit for bit, in every lane
    s = wave_sum(s);
    const float yb = s + master[kB4];
    const float d = yb - t[b];
    const float g = 2.f * d / (float)B;
    if (lane == 0) {
        y[b] = yb;
        dy[b] = g;
        sq[b] = d * d;
    }
    for (int c = lane; c < kHid; c += 64) {
        const float v = (Z3[b * kHid + c] > 0.f) ? g * from_bf16(wb[kW4 + c]) : 0.f;
        dZ3[b * kHid + c] = v;
        dZ3b[b * kHid + c] = to_bf16(v);
    }
}

// dZ1[r][c] = dS[r / n][c] [Z1[r][c] > 0], stored as BF16 (the token rows'
// only use): one wave per token row, four columns per lane.
__global__ __launch_bounds__(256) void dz1_kernel(const float *dS, const float *Z1, int64_t T, int32_t n,
                                                  uint16_t *dZ1b)
{
    // the row is uniform across the wave, so the bounds check is a scalar branch
    const int64_t r = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (r >= T)
        return;
    const int c = (threadIdx.x & 63) * 4;
    const float4 z = *reinterpret_cast<const float4 *>(Z1 + r * kHid + c);
    const float4 d = *reinterpret_cast<const float4 *>(dS + (r / n) * kHid + c);
    uint2 o;
    o.x = (uint32_t)to_bf16(z.x > 0.f ? d.x : 0.f) | ((uint32_t)to_bf16(z.y > 0.f ? d.y : 0.f) << 16);
    o.y = (uint32_t)to_bf16(z.z > 0.f ? d.z : 0.f) | ((uint32_t)to_bf16(z.w > 0.f ? d.w : 0.f) << 16);
    *reinterpret_cast<uint2 *>(dZ1b + r * kHid + c) = o;
}

// Column sums of up to five row-major matrices in one launch, stage 1 of 2:
// workgroup g of problem q covers rows [g chunk, (g + 1) chunk) and thread c
// adds w(r) X(r, c) down column c in row order (w(r) = wrow[r] or 1; X float32
// or BF16 with row pitch ld, times the count Xm(r, c) when Xm is set); with
// `with_w` thread `cols` adds w(r) alone.  The partials go to
// part[g][cols + with_w]; the finish kernel adds them.
struct ColProblem {
    const float *Xf;
    const uint16_t *Xb;
    const uint8_t *Xm;
    const float *wrow;
    float *part;
    int64_t ld, rows, chunk;
    int32_t cols, with_w, first;   // first: this problem's first workgroup
    int32_t pad;
};
constexpr int kColProblems = 5;
struct ColMulti {
    ColProblem p[kColProblems];
    int32_t count;
};

__global__ __launch_bounds__(320) void colsum_multi_kernel(ColMulti a)
{
    int q = 0;
    for (int i = 1; i < a.count; i++)
        q = ((int)blockIdx.x >= a.p[i].first) ? i : q;
    const ColProblem &p = a.p[q];
    const int c = threadIdx.x;
    const int width = p.cols + p.with_w;
    if (c >= width)
        return;
    const int64_t g = (int64_t)blockIdx.x - p.first;
    const int64_t r0 = g * p.chunk;
    const int64_t r1 = min(p.rows, r0 + p.chunk);
    float s = 0.f;
#pragma unroll 8
    for (int64_t r = r0; r < r1; r++) {
        const float w = p.wrow ? p.wrow[r] : 1.f;
        if (c < p.cols) {
            float x = p.Xf ? p.Xf[r * p.ld + c] : from_bf16(p.Xb[r * p.ld + c]);
            if (p.Xm)
                x *= (float)p.Xm[r * p.ld + c];
            s += w * x;
        } else {
            s += w;
        }
    }
    p.part[g * width + c] = s;
}

// Adam on one parameter: float32 master weight, moments and BF16 copy, with
// the bias corrections c1 = 1 - beta1^s and c2 = 1 - beta2^s of step s.
struct AdamArgs {
    float *master, *m, *v;
    uint16_t *wb;
    float lr, b1, b2, eps, c1, c2;
};

__device__ inline void adam_update(int64_t i, float gi, const AdamArgs &a)
{
    const float mi = a.b1 * a.m[i] + (1.f - a.b1) * gi;
    const float vi = a.b2 * a.v[i] + (1.f - a.b2) * gi * gi;
    a.m[i] = mi;
    a.v[i] = vi;
    const float wi = a.master[i] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
    a.master[i] = wi;
    a.wb[i] = to_bf16(wi);
}

// A float every lane holds, made explicitly wave-uniform.
__device__ inline float uniform_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// The step-dependent values of an update, evaluated once per thread at kernel
// entry while every lane is active (they are uniform: step and rate come from
// the caller or the schedule).
__device__ inline void adam_prepare(AdamArgs &a, int32_t step)
{
    a.c1 = uniform_f32(1.f - powf(a.b1, (float)step));
    a.c2 = uniform_f32(1.f - powf(a.b2, (float)step));
}

// The rate of step s: linear warm-up over `warmup` steps to lr, then half a
// cosine from lr down to lr * lr_final at step `total`.
__device__ inline float sched_rate(const ko_nn_sched &h, int32_t s)
{
    if (s <= h.warmup)
        return h.lr * (float)s / (float)max(1, h.warmup);
    const float p = (float)(s - h.warmup) / (float)max(1, h.total - h.warmup);
    return h.lr * (h.lr_final + (1.f - h.lr_final) * 0.5f * (1.f + cosf(3.14159265358979f * p)));
}

__global__ void adam_kernel(const float *g, int64_t count, AdamArgs a, int32_t step)
{
    adam_prepare(a, step);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        adam_update(i, g[i], a);
}

// Stage 2 of every reduction of a step, in one launch: the weight gradients
// from their split-K partials and the bias, output-layer and loss sums from
// their column partials.  A reduction is a segment: `count` outputs, each the
// sum of `rows` partials at stride `stride`.  A workgroup takes 32
// consecutive outputs of one segment; its 8 thread groups add 8 consecutive
// ranges of the partials, each in order, and the first group adds the 8
// range sums in order (a fixed order: deterministic).  Writes the gradients
// (and the loss, which is the sum over B); with `sched` set it then applies
// Adam to each parameter with step sched->step and its rate.  A segment with
// few partials (at most kFinShort) uses one group: 256 outputs per workgroup.
struct Segment {
    const float *P;
    int64_t stride;
    int32_t rows, count;
    int32_t param;   // the gradient of output o is parameter param + o; -1: the loss
    int32_t first;   // first workgroup
    int32_t groups;  // 1 or kFinGroups
    int32_t pad;
};
constexpr int kSegments = 8;
constexpr int kFinGroups = 8, kFinShort = 32;
struct FinishArgs {
    Segment seg[kSegments];
    int32_t count;
    int32_t B;
    float *grad, *loss_out;
    const ko_nn_sched *sched;
    AdamArgs adam;
};

__global__ __launch_bounds__(256) void finish_kernel(FinishArgs a)
{
    __shared__ float part[kFinGroups][256 / kFinGroups];
    AdamArgs ad = a.adam;
    if (a.sched) {
        const ko_nn_sched h = *a.sched;
        ad.lr = uniform_f32(sched_rate(h, h.step));
        ad.b1 = h.beta1, ad.b2 = h.beta2, ad.eps = h.eps;
        adam_prepare(ad, h.step);
    }
    int q = 0;
    for (int i = 1; i < a.count; i++)
        q = ((int)blockIdx.x >= a.seg[i].first) ? i : q;
    const Segment &sg = a.seg[q];
    // (shifts, not divisions: the group count is 1 or 8)
    const bool wide = sg.groups > 1;
    const int per = wide ? 256 / kFinGroups : 256;   // outputs per workgroup
    const int ol = wide ? (int)threadIdx.x % per : (int)threadIdx.x;
    const int grp = wide ? (int)threadIdx.x / per : 0;
    const int32_t lo = wide ? (sg.rows * grp) / kFinGroups : 0;
    const int32_t hi = wide ? (sg.rows * (grp + 1)) / kFinGroups : sg.rows;
    const int64_t o = (int64_t)(blockIdx.x - sg.first) * per + ol;
    float g = 0.f;
    if (o < sg.count) {
#pragma unroll 8
        for (int32_t z = lo; z < hi; z++)
            g += sg.P[z * sg.stride + o];
    }
    if (wide) {
        part[grp][ol] = g;
        __syncthreads();
        if (grp != 0)
            return;
#pragma unroll
        for (int i = 1; i < kFinGroups; i++)
            g += part[i][ol];
    }
    if (o >= sg.count)
        return;
    if (sg.param < 0) {
        if (a.loss_out)
            *a.loss_out = g / (float)a.B;
        return;
    }
    const int64_t param = sg.param + o;
    a.grad[param] = g;
    if (a.sched)
        adam_update(param, g, ad);
}

__global__ void refresh_kernel(const float *w, uint16_t *wb, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        wb[i] = to_bf16(w[i]);
}

__global__ void zero_f32_kernel(float *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = 0.f;
}

// x[b][i][0..7] = bf16(feat[set][i][.]); x[b][i][8 + pos] = 1; rest 0: input
// f of token i of sample row r.
__device__ inline uint16_t token_value(const float *feat, const int32_t *set_of, const uint8_t *pos, int64_t r,
                                       int64_t i, int f, int32_t n)
{
    const int64_t s = set_of ? set_of[r] : 0;
    if (f < KO_NN_FEAT)
        return to_bf16(feat[(s * n + i) * KO_NN_FEAT + f]);
    if (f < KO_NN_FEAT + KO_NN_POS)
        return (pos[r * n + i] == (uint8_t)(f - KO_NN_FEAT)) ? (uint16_t)0x3F80 : (uint16_t)0;
    return 0;
}

// (makespan[r] - center[s]) / scale[s] for sample row r of set s = set_of[r]
__device__ inline float target_value(const int64_t *makespans, const int32_t *set_of, const int64_t *center,
                                     const int64_t *scale, int64_t r)
{
    const int64_t s = set_of ? set_of[r] : 0;
    return (float)((double)(makespans[r] - center[s]) / (double)scale[s]);
}

__global__ void tokens_kernel(const float *feat, const int32_t *set_of, const uint8_t *pos,
                              const int64_t *rows, int32_t B, int32_t n, uint16_t *x)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * n * kIn)
        return;
    const int64_t t = idx / kIn;
    const int64_t b = t / n;
    x[idx] = token_value(feat, set_of, pos, rows ? rows[b] : b, t % n, (int)(idx % kIn), n);
}

// t[b] = (makespan[r] - center[s]) / scale[s] with r = rows[b] (or b), s = set_of[r]
__global__ void targets_kernel(const int64_t *makespans, const int32_t *set_of, const int64_t *center,
                               const int64_t *scale, const int64_t *rows, int32_t B, float *t)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B)
        return;
    t[b] = target_value(makespans, set_of, center, scale, rows ? rows[b] : b);
}

// A training step's minibatch, chosen on the device: sample b is row
// perm[(step mod per_epoch) B + b] with step = sched->step, the steps taken so
// far; its tokens and target are those of tokens_kernel and targets_kernel.
__global__ void batch_kernel(const float *feat, const int32_t *set_of, const uint8_t *pos, const int64_t *makespans,
                             const int64_t *center, const int64_t *scale, const int64_t *perm,
                             const ko_nn_sched *sched, int32_t B, int32_t n, uint16_t *x, float *t)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // a count below 1 is taken as 1 and the step as unsigned, so the slice
    // always starts inside the first per_epoch B entries of perm
    const uint32_t pe = (uint32_t)max(1, sched->per_epoch);
    const int64_t *rows = perm + (int64_t)((uint32_t)sched->step % pe) * B;
    if (idx < B)
        t[idx] = target_value(makespans, set_of, center, scale, rows[idx]);
    if (idx >= (int64_t)B * n * kIn)
        return;
    const int64_t tk = idx / kIn;
    x[idx] = token_value(feat, set_of, pos, rows[tk / n], tk % n, (int)(idx % kIn), n);
}

// Within-set ranks: ranks[s * per + i] = position of sample i of set s when
// the set's values are sorted by (value, i).  One workgroup per set sorts the
// keys (value - min) << 13 | i in LDS with a bitonic network (per <= 8192,
// padded to a power of two with the largest key); values of a set must span
// less than 2^51.
constexpr int kRankMax = 8192;

__global__ __launch_bounds__(1024) void within_set_rank_kernel(const int64_t *values, int32_t per, int32_t p2,
                                                               int64_t *ranks)
{
    __shared__ uint64_t key[kRankMax];
    __shared__ int64_t vmin[32];
    const int64_t s = blockIdx.x;
    const int64_t *v = values + s * per;
    // minimum of the set (keys are offsets from it)
    int64_t m = INT64_MAX;
    for (int i = threadIdx.x; i < per; i += blockDim.x)
        m = min(m, v[i]);
    for (int o = 32; o >= 1; o >>= 1)
        m = min(m, (int64_t)__shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0)
        vmin[threadIdx.x >> 6] = m;
    __syncthreads();
    m = vmin[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); w++)
        m = min(m, vmin[w]);
    for (int i = threadIdx.x; i < p2; i += blockDim.x)
        key[i] = (i < per) ? (((uint64_t)(v[i] - m) << 13) | (uint64_t)i) : ~0ull;
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < p2; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t a = key[i], b = key[l];
                    const bool up = (i & k) == 0;
                    if (up ? (a > b) : (a < b)) {
                        key[i] = b;
                        key[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int p = threadIdx.x; p < per; p += blockDim.x)
        ranks[s * per + (int64_t)(key[p] & 8191u)] = p;
}

// The feature part of layer 1 plus its bias, for kernel i and hidden unit j:
// g(i, j) = (sum_{k<8} W1[j][k] f_i[k]) + b1[j], summed in k order in
// float32 over the BF16 operands the token path multiplies.  w1r holds the 8
// BF16 weights W1[j][0..7].
__device__ __forceinline__ float layer1_base(const uint4 w1r, const float *fi, float b1)
{
    const uint32_t w[4] = {w1r.x, w1r.y, w1r.z, w1r.w};
    float z = 0.f;
#pragma unroll
    for (int k = 0; k < KO_NN_FEAT; k++) {
        const uint16_t h = (uint16_t)(w[k >> 1] >> (16 * (k & 1)));
        z += from_bf16(h) * from_bf16(to_bf16(fi[k]));
    }
    return z + b1;
}

// Layer 1 for one set, tabulated over launch positions: a token is its
// kernel's features plus a one-hot position, so its first-layer output is
//   T[i][p][j] = relu(g(i, j) + W1[j][8+p])
// for kernel i at position p (17 positions: 16 launch slots and "unplaced"),
// with g as in layer1_base.  Operands are the BF16 values the token path
// multiplies; sums are float32 (the token path adds the bias last, an
// association that differs only in float32 rounding).
__global__ void table_kernel(const uint16_t *wb, const float *master, const float *feat, int32_t n,
                             float *T)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * KO_NN_POS * kHid)
        return;
    const int j = (int)(idx % kHid);
    const int p = (int)((idx / kHid) % KO_NN_POS);
    const int64_t i = idx / ((int64_t)kHid * KO_NN_POS);
    const uint4 w1r = *reinterpret_cast<const uint4 *>(wb + kW1 + (size_t)j * kIn);
    const float g = layer1_base(w1r, feat + i * KO_NN_FEAT, master[kB1 + j]);
    T[idx] = fmaxf(g + from_bf16(wb[kW1 + (size_t)j * kIn + KO_NN_FEAT + p]), 0.f);
}

// Sum pooling from the table: S[b][j] = sum_i T[i][pos[b][i]][j] (kernel order,
// as the token path sums), stored as BF16.  One workgroup per sample; a
// position above 16 counts as "unplaced".
__global__ __launch_bounds__(256) void gather_pool_kernel(const float *T, const uint8_t *pos, int32_t n,
                                                          uint16_t *Sb)
{
    const int64_t b = blockIdx.x;
    const int j = threadIdx.x;
    float s = 0.f;
    for (int i = 0; i < n; i++) {
        const int p = min((int)pos[b * n + i], KO_NN_UNPLACED);
        s += T[((int64_t)i * KO_NN_POS + p) * kHid + j];
    }
    Sb[b * kHid + j] = to_bf16(s);
}

// Layers 2 and 3 and the output layer of a scoring tile: the 64 x 256 BF16
// activations in LDS (At, row pitch P) become relu(A W^T + b) twice, wave w
// computing columns [64w, 64w + 64) as 4 x 4 MFMA 16x16x32 tiles with W's
// 16-byte fragments read from memory (the fragments and k order of
// gemm_nt_kernel) and writing its BF16 result back over the tile once every
// wave has read it; then y for the tile's `rows` rows, one wave per row, as
// out_forward_kernel.  Called by all 256 threads after a barrier that
// published the tile.
template <int P>
__device__ __forceinline__ void score_layers(uint16_t (*At)[P], const uint16_t *wb, const float *master, int wave,
                                             int lane, int rows, int64_t b0, float *y)
{
    const int kk = (lane >> 4) * 8;
#pragma unroll
    for (int layer = 0; layer < 2; layer++) {
        const uint16_t *W = wb + (layer == 0 ? kW2 : kW3);
        const float *bias = master + (layer == 0 ? kB2 : kB3);
        f32x4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++)
                acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < kHid; k0 += kKStep) {
            bf16x8 af[4], bfr[4];
#pragma unroll
            for (int j = 0; j < 4; j++)
                bfr[j] = *reinterpret_cast<const bf16x8 *>(W + (size_t)(wave * 64 + j * 16 + (lane & 15)) * kHid +
                                                           k0 + kk);
#pragma unroll
            for (int i = 0; i < 4; i++)
                af[i] = *reinterpret_cast<const bf16x8 *>(&At[i * 16 + (lane & 15)][k0 + kk]);
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();  // every wave has read the tile
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int col = wave * 64 + j * 16 + (lane & 15);
            const float bc = bias[col];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int e = 0; e < 4; e += 2) {
                    const int row = i * 16 + (lane >> 4) * 4 + e;
                    const uint32_t h = pack_bf16x2(fmaxf(acc[i][j][e] + bc, 0.f), fmaxf(acc[i][j][e + 1] + bc, 0.f));
                    At[row][col] = (uint16_t)h;
                    At[row + 1][col] = (uint16_t)(h >> 16);
                }
        }
        __syncthreads();
    }
    for (int r = wave; r < rows; r += 4) {
        float s = 0.f;
        for (int c = lane; c < kHid; c += 64)
            s += from_bf16(At[r][c]) * from_bf16(wb[kW4 + c]);
        s = wave_sum(s);
        if (lane == 0)
            y[b0 + r] = s + master[kB4];
    }
}

// Scoring in one kernel, for a tile of 64 orders of one set per workgroup:
// the same values as table_kernel + gather_pool_kernel + the two hidden
// layers (gemm_nt_kernel) + out_forward_kernel, bit for bit, with nothing
// written to memory but y.
//   1. layer 1 and pooling: a token's first-layer output is
//      relu(g(i, j) + W1[j][8 + p]) (table_kernel); each thread keeps g for
//      its two columns and every kernel in registers and reads the position
//      weights from LDS, so the table (n x 17 x 256 floats) is never built.
//      A row's positions come in one 16-byte LDS read; S is summed in kernel
//      order and rounded to BF16 into an LDS tile [64][256];
//   2. layers 2 and 3: wave w computes columns [64w, 64w + 64) of
//      relu(A W^T + b) for the 64 rows as 4 x 4 MFMA 16x16x32 tiles, A from
//      the LDS tile, W's 16-byte fragments straight from memory (the same
//      fragments and k order as gemm_nt_kernel), and writes the BF16 result
//      back over the tile once every wave has read it;
//   3. the output layer: one wave per row, the same sum as out_forward_kernel.
constexpr int kScTile = 64;                // orders per workgroup
constexpr int kScPitch = kHid + 8;         // LDS row pitch (elements): 132 dwords, 4 mod 32 banks

template <int N>
__global__ __launch_bounds__(256) void score_kernel(const uint16_t *wb, const float *master, const float *feat,
                                                    const uint8_t *pos, int32_t B, float *y)
{
    __shared__ __attribute__((aligned(16))) uint16_t At[kScTile][kScPitch];
    __shared__ __attribute__((aligned(16))) float w1p[KO_NN_POS][kHid];
    // per row and kernel: the byte offset of the position's row of w1p
    __shared__ __attribute__((aligned(16))) uint16_t ps[kScTile][16];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // the wave index is uniform across the wave (see out_forward_kernel)
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t b0 = (int64_t)blockIdx.x * kScTile;
    const int rows = (int)min((int64_t)kScTile, (int64_t)B - b0);

    for (int idx = tid; idx < KO_NN_POS * kHid; idx += 256) {
        const int q = idx / kHid, j = idx % kHid;
        w1p[q][j] = from_bf16(wb[kW1 + (size_t)j * kIn + KO_NN_FEAT + q]);
    }
    for (int idx = tid; idx < kScTile * 16; idx += 256) {
        const int r = idx >> 4, i = idx & 15;
        const int p = (r < rows && i < N) ? min((int)pos[(b0 + r) * N + i], KO_NN_UNPLACED) : KO_NN_UNPLACED;
        ps[r][i] = (uint16_t)(p * kHid * (int)sizeof(float));
    }
    // thread t: columns c0 = 2 (t % 128) and c0 + 1, rows [32 (t / 128), +32)
    const int c0 = 2 * (tid & 127);
    const int r0 = (tid >> 7) * (kScTile / 2);
    const uint4 w1a = *reinterpret_cast<const uint4 *>(wb + kW1 + (size_t)c0 * kIn);
    const uint4 w1b = *reinterpret_cast<const uint4 *>(wb + kW1 + (size_t)(c0 + 1) * kIn);
    const float bias0 = master[kB1 + c0], bias1 = master[kB1 + c0 + 1];
    float g0[N], g1[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
        g0[i] = layer1_base(w1a, feat + i * KO_NN_FEAT, bias0);
        g1[i] = layer1_base(w1b, feat + i * KO_NN_FEAT, bias1);
    }
    __syncthreads();
    const char *wcol = reinterpret_cast<const char *>(&w1p[0][c0]);
    for (int r = r0; r < r0 + kScTile / 2; r++) {
        uint32_t pw[8];
        const uint4 q0 = *reinterpret_cast<const uint4 *>(&ps[r][0]);
        pw[0] = q0.x, pw[1] = q0.y, pw[2] = q0.z, pw[3] = q0.w;
        if (N > 8) {
            const uint4 q1 = *reinterpret_cast<const uint4 *>(&ps[r][8]);
            pw[4] = q1.x, pw[5] = q1.y, pw[6] = q1.z, pw[7] = q1.w;
        }
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int i = 0; i < N; i++) {
            const uint32_t off = (i & 1) ? (pw[i >> 1] >> 16) : (pw[i >> 1] & 0xFFFFu);
            const float2 w = *reinterpret_cast<const float2 *>(wcol + off);
            s0 += fmaxf(g0[i] + w.x, 0.f);
            s1 += fmaxf(g1[i] + w.y, 0.f);
        }
        *reinterpret_cast<uint32_t *>(&At[r][c0]) = pack_bf16x2(s0, s1);
    }
    __syncthreads();

    score_layers<kScPitch>(At, wb, master, wave, lane, rows, b0, y);
}

template <int N>
void launch_score_n(unsigned grid, hipStream_t st, const uint16_t *wb, const float *master, const float *feat,
                    const uint8_t *pos, int32_t B, float *y)
{
    hipLaunchKernelGGL(score_kernel<N>, dim3(grid), dim3(256), 0, st, wb, master, feat, pos, B, y);
}

template <int... Ns>
bool launch_score(int n, unsigned grid, hipStream_t st, const uint16_t *wb, const float *master, const float *feat,
                  const uint8_t *pos, int32_t B, float *y, std::integer_sequence<int, Ns...>)
{
    return ((n == Ns + 1 ? (launch_score_n<Ns + 1>(grid, st, wb, master, feat, pos, B, y), true) : false) || ...);
}

// ------------------------------------------------------------------ scoring, pooling on the matrix cores
//
// S = sum_i T[i][pos_i] is the product of an order's one-hot row with the
// set's layer-1 table viewed as a matrix with one row per (kernel, slot).  An
// order of an n-kernel set puts each kernel at a launch position 0..n-1 or
// leaves it unplaced (16), so a kernel needs n + 1 slots: slot p for position
// p < n and slot n for "unplaced".  With the table carried as two BF16
// matrices, hi = bf16(T) and lo = bf16(T - hi) (together 16 significant bits
// of T, a relative error below 2^-17), the pooling is a BF16 MFMA product
// with float32 accumulation like the layers after it, instead of 3 n float32
// instructions per hidden unit.  The one-hot entries are exact, so the result
// differs from the table path only by that representation and the order of
// the float32 additions; S is then rounded to BF16 as on every path.

constexpr int kSplitK(int n) { return (n * (n + 1) + kKStep - 1) / kKStep * kKStep; }

// Fragment order of a [256][32 KS] BF16 matrix (hidden unit h, k): the 512
// values of the MFMA operand fragment of unit block h / 16 at k step k / 32
// (64 lanes x 8 values: lane 16 (k % 32 / 8) + h % 16 holds k % 8 = 0..7) are
// contiguous, the blocks in (unit block, k step) order.
constexpr int kFragElems = 512;

constexpr int64_t frag_index(int h, int k, int KS)
{
    return ((int64_t)(h >> 4) * KS + (k >> 5)) * kFragElems + ((((k & 31) >> 3) << 4) | (h & 15)) * 8 + (k & 7);
}

// the kernels below write fragment (unit block rb, k step ks) with thread t
// holding unit 16 rb + (t / 8) % 16 and k = 32 ks + 8 (t / 128) + t % 8; the
// scoring kernel's lane l reads values [8 l, 8 l + 8) of a fragment as the
// MFMA operand of unit 16 rb + l % 16, k = 32 ks + 8 (l / 16) + 0..7
constexpr bool frag_order_consistent()
{
    for (int t = 0; t < kFragElems; t++) {
        const int lane = t >> 3;
        if (frag_index(16 + (lane & 15), 2 * kKStep + (lane >> 4) * 8 + (t & 7), 5) != (1 * 5 + 2) * kFragElems + t)
            return false;
    }
    return true;
}
static_assert(frag_order_consistent(), "fragment order and the threads' mapping agree");

// The scoring operand pack of one set, BF16 in fragment order: the split
// table's high part [256][KP] (hidden unit j, k = (n + 1) i + slot for kernel
// i, zero from n (n + 1) up to KP = kSplitK(n)), its low part, then W2 and W3
// [256][256] (the BF16 copies).  The table's T is computed exactly as
// table_kernel does for the slot's position.  One workgroup of 512 threads
// per fragment, grid (KP / 32, 16): thread t = 8 lane + e writes value e of
// the fragment's lane, so the writes are contiguous.
__global__ __launch_bounds__(512) void split_table_kernel(const uint16_t *wb, const float *master, const float *feat,
                                                          int32_t n, int32_t KP, uint16_t *split)
{
    const int ks = blockIdx.x, rb = blockIdx.y, t = threadIdx.x;
    const int lane = t >> 3;
    const int j = rb * 16 + (lane & 15), k = ks * kKStep + (lane >> 4) * 8 + (t & 7);
    const int64_t idx = ((int64_t)rb * (KP / kKStep) + ks) * kFragElems + t;
    uint16_t hi = 0, lo = 0;
    if (k < n * (n + 1)) {
        const int i = k / (n + 1), slot = k % (n + 1);
        const int p = slot < n ? slot : KO_NN_UNPLACED;
        const uint4 w1r = *reinterpret_cast<const uint4 *>(wb + kW1 + (size_t)j * kIn);
        const float g = layer1_base(w1r, feat + i * KO_NN_FEAT, master[kB1 + j]);
        const float T = fmaxf(g + from_bf16(wb[kW1 + (size_t)j * kIn + KO_NN_FEAT + p]), 0.f);
        hi = to_bf16(T);
        lo = to_bf16(T - from_bf16(hi));
    }
    split[idx] = hi;
    split[(int64_t)kHid * KP + idx] = lo;
}

// W2 (blockIdx.z = 0) and W3 (1) in fragment order into out[2][256 x 256];
// grid (8, 16, 2) of 512 threads, one fragment each
__global__ __launch_bounds__(512) void frag_weights_kernel(const uint16_t *wb, uint16_t *out)
{
    const int ks = blockIdx.x, rb = blockIdx.y, m = blockIdx.z, t = threadIdx.x;
    const int lane = t >> 3;
    const int h = rb * 16 + (lane & 15), k = ks * kKStep + (lane >> 4) * 8 + (t & 7);
    const size_t src = (m == 0 ? kW2 : kW3) + (size_t)h * kHid + k;
    out[(size_t)m * kHid * kHid + ((size_t)rb * (kHid / kKStep) + ks) * kFragElems + t] = wb[src];
}

// One product of the split scoring kernel for a wave, computed transposed:
// acc[i][j] (hidden units [64 w + 16 j, +16) x the tile's orders [16 i, +16))
// = init[j] + B A^T over K = 32 KS, where B (the weights or the split table in
// fragment order; with TWO a second matrix of the same shape, accumulated
// after the first in each k step) is the MFMA's first operand and A (the
// tile in LDS, in the same fragment order with orders as the units, so a
// wave's read is 1 KB contiguous) its second.  A lane so holds 4
// consecutive hidden units of one order.  The first k step takes init[j]
// (the bias of the lane's 4 units, or zero) as its addend, so nothing is
// cleared or added afterwards.
//
// B's fragments come from memory D k steps ahead of the MFMAs that use them,
// through D + 1 fragment sets in turn; the caller loads the first D
// (split_prefetch) before the barrier and epilogue that precede the product,
// so their latency hides behind them.  Each prefetch is fenced off from the
// scheduler (sched_barrier), which would otherwise sink the loads towards
// their first use; the k loop is unrolled in full, so every fragment set is
// a fixed set of registers.
typedef short s16x2 __attribute__((ext_vector_type(2)));

template <bool TWO>
struct SplitFrag {
    bf16x8 b[4], b2[4];
};

// The lane's fragment pointers of B (and B2) in fragment order (frag_index):
// the fragments of unit block 4 w + j at k step ks are 1 KB contiguous, lane l
// reading bytes [16 l, 16 l + 16), so a fragment load touches 8 whole cache
// lines instead of 16 half lines.
struct SplitB {
    const uint16_t *p, *p2;
    int ks_total;
    template <bool TWO>
    __device__ __forceinline__ void load(SplitFrag<TWO> &f, int ks) const
    {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            f.b[j] = *reinterpret_cast<const bf16x8 *>(p + (size_t)(j * ks_total + ks) * kFragElems);
            if (TWO)
                f.b2[j] = *reinterpret_cast<const bf16x8 *>(p2 + (size_t)(j * ks_total + ks) * kFragElems);
        }
    }
};

__device__ __forceinline__ SplitB split_b(const uint16_t *Bm, const uint16_t *Bm2, int ks_total, int wave, int lane)
{
    const size_t off = (size_t)(wave * 4) * ks_total * kFragElems + lane * 8;
    return SplitB{Bm + off, Bm2 ? Bm2 + off : nullptr, ks_total};
}

// k steps 0 .. D-1 of B into f[0 .. D-1]
template <int KS, int D, bool TWO>
__device__ __forceinline__ void split_prefetch(const SplitB &bm, SplitFrag<TWO> (&f)[D + 1])
{
#pragma unroll
    for (int s = 0; s < D && s < KS; s++)
        bm.load(f[s], s);
}

template <int KS, int D, bool TWO>
__device__ __forceinline__ void split_product(f32x4 (&acc)[8][4], const uint16_t *At, const SplitB &bm,
                                              SplitFrag<TWO> (&f)[D + 1], const f32x4 (&init)[4], int lane)
{
    static_assert(KS >= 1 && D >= 1, "at least one k step, prefetched at least one ahead");
#pragma clang loop unroll(full)
    for (int ks = 0; ks < KS; ks++) {
        if (ks + D < KS)
            bm.load(f[(ks + D) % (D + 1)], ks + D);
        __builtin_amdgcn_sched_barrier(0);
        const SplitFrag<TWO> &g = f[ks % (D + 1)];
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const bf16x8 af = *reinterpret_cast<const bf16x8 *>(At + ((size_t)i * KS + ks) * kFragElems + lane * 8);
#pragma unroll
            for (int j = 0; j < 4; j++) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g.b[j], af, ks == 0 ? init[j] : acc[i][j], 0, 0, 0);
                if (TWO)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g.b2[j], af, acc[i][j], 0, 0, 0);
            }
        }
    }
}

// BF16 of acc's 4 values (round to nearest even), with relu applied to the
// rounded values (a BF16 value below zero, -0 included, has its sign bit set:
// as a 16-bit integer it is negative, and the integer maximum with 0 gives
// +0; rounding and relu commute for every number that is not NaN).
template <bool RELU>
__device__ __forceinline__ uint2 bf16x4_of(const f32x4 &a)
{
    uint2 u{pack_bf16x2(a[0], a[1]), pack_bf16x2(a[2], a[3])};
    if (RELU) {
        s16x2 x, y;
        const s16x2 z = {0, 0};
        __builtin_memcpy(&x, &u.x, 4);
        __builtin_memcpy(&y, &u.y, 4);
        x = __builtin_elementwise_max(x, z);
        y = __builtin_elementwise_max(y, z);
        __builtin_memcpy(&u.x, &x, 4);
        __builtin_memcpy(&u.y, &y, 4);
    }
    return u;
}

// Scoring of a tile of 128 orders per workgroup (4 waves; wave w owns hidden
// units [64 w, 64 w + 64) of every product, for all 128 orders, so each
// fragment of the table or of W feeds 8 MFMAs):
//   1. the one-hot tile in LDS (row r: a 1 at (n + 1) i + slot for kernel
//      i, the slot being its position, or n when unplaced);
//   2. S = onehot (hi + lo), the hi then the lo product of each k step into
//      one float32 accumulator; S as BF16 over the tile once every wave has
//      read the one-hot rows (8 bytes per lane and tile: an order's 4
//      consecutive hidden units);
//   3. A2 = relu(b2 + S W2^T) as BF16 over the tile, likewise;
//   4. A3 = relu(b3 + A2 W3^T) rounded to BF16 stays in registers: each lane
//      multiplies its 16 A3 values of an order by w4, the 4 lanes that hold
//      the order's other units of this wave add theirs (two xor shuffles),
//      and the 4 waves' sums of a row are added in wave order with b4: y.
// Every sum has a fixed order, so y does not depend on scheduling.
constexpr int kSpRows = 128;
// prefetch distances (k steps) of the pooling product (fragment sets of 32
// VGPRs, 64 MFMAs a step) and of the layer products (16 VGPRs, 32 MFMAs)
constexpr int kPoolAhead = 1;
constexpr int kLayerAhead = 2;
static_assert(kB2 % 4 == 0 && kB3 % 4 == 0 && kW4 % 4 == 0, "16-byte bias and 8-byte w4 loads");

template <int N>
__global__ __launch_bounds__(256, 2) void score_split_kernel(const uint16_t *wb, const float *master,
                                                          const uint16_t *split, const uint8_t *pos, int32_t B,
                                                          float scale, int32_t accumulate, float *y)
{
    constexpr int KP = kSplitK(N);
    // the tile [128 orders][K] in fragment order (frag_index, orders as the
    // units): the one-hot rows (K = KP), then S and A2 (K = 256)
    __shared__ __attribute__((aligned(16))) uint16_t At[kSpRows * kSplitK(KO_NN_MAX_TOKENS)];
    __shared__ float yp[4][kSpRows];
    __shared__ uint8_t bad[kSpRows];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // the wave index is uniform across the wave (see out_forward_kernel)
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t b0 = (int64_t)blockIdx.x * kSpRows;
    const int rows = (int)min((int64_t)kSpRows, (int64_t)B - b0);
    // the table's first fragments and the tile's positions (every load
    // issued before any is waited for) arrive while the tile is cleared
    const SplitB tb = split_b(split, split + (size_t)kHid * KP, KP / kKStep, wave, lane);
    SplitFrag<true> tf[kPoolAhead + 1];
    split_prefetch<KP / kKStep, kPoolAhead>(tb, tf);
    constexpr int kPosPer = (kSpRows * N + 255) / 256;
    int pv[kPosPer];
#pragma unroll
    for (int q = 0; q < kPosPer; q++) {
        const int idx = tid + q * 256;
        pv[q] = idx < rows * N ? pos[b0 * N + idx] : 0;
    }

    for (int idx = tid; idx < kSpRows * KP / 8; idx += 256)
        *reinterpret_cast<uint4 *>(At + (size_t)idx * 8) = make_uint4(0u, 0u, 0u, 0u);
    if (tid < kSpRows)
        bad[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPosPer; q++) {
        const int idx = tid + q * 256;
        if (idx < rows * N) {
            const int r = idx / N, i = idx % N, p = pv[q];
            if (p < N || p >= KO_NN_UNPLACED)
                At[frag_index(r, i * (N + 1) + (p < N ? p : N), KP / kKStep)] = 0x3F80;   // BF16 1.0
            else
                bad[r] = 1;   // not a launch position of an N-kernel order
        }
    }
    __syncthreads();

    f32x4 acc[8][4];
    // the tile row (order) of acc[i][.] and the first of the 4 hidden units of acc[.][j]
    const int rl = lane & 15;
    auto unit_of = [&](int j) { return wave * 64 + j * 16 + (lane >> 4) * 4; };
    auto bias_of = [&](const float *b, f32x4 (&init)[4]) {
#pragma unroll
        for (int j = 0; j < 4; j++)
            init[j] = *reinterpret_cast<const f32x4 *>(b + unit_of(j));
    };
    // BF16 of acc (relu for RELU) over the tile
    auto store_tile = [&](auto relu) {
#pragma unroll
        for (int i = 0; i < 8; i++)
#pragma unroll
            for (int j = 0; j < 4; j++)
                *reinterpret_cast<uint2 *>(At + frag_index(i * 16 + rl, unit_of(j), kHid / kKStep)) =
                    bf16x4_of<decltype(relu)::value>(acc[i][j]);
    };

    f32x4 init[4];
#pragma unroll
    for (int j = 0; j < 4; j++)
        init[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    split_product<KP / kKStep, kPoolAhead, true>(acc, At, tb, tf, init, lane);
    const uint16_t *wfrag = split + (size_t)2 * kHid * KP;   // W2 and W3 in fragment order
    const SplitB w2 = split_b(wfrag, nullptr, kHid / kKStep, wave, lane);
    SplitFrag<false> wf[kLayerAhead + 1];
    split_prefetch<kHid / kKStep, kLayerAhead>(w2, wf);
    bias_of(master + kB2, init);
    __syncthreads();   // every wave has read the one-hot tile
    store_tile(std::false_type{});
    __syncthreads();
    split_product<kHid / kKStep, kLayerAhead, false>(acc, At, w2, wf, init, lane);
    const SplitB w3 = split_b(wfrag + (size_t)kHid * kHid, nullptr, kHid / kKStep, wave, lane);
    split_prefetch<kHid / kKStep, kLayerAhead>(w3, wf);
    bias_of(master + kB3, init);
    __syncthreads();   // every wave has read S
    store_tile(std::true_type{});
    __syncthreads();
    split_product<kHid / kKStep, kLayerAhead, false>(acc, At, w3, wf, init, lane);

    // output layer from the registers: w4 of the lane's 16 hidden units
    float w4[4][4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint2 h = *reinterpret_cast<const uint2 *>(wb + kW4 + unit_of(j));
        w4[j][0] = __uint_as_float(h.x << 16);
        w4[j][1] = __uint_as_float(h.x & 0xFFFF0000u);
        w4[j][2] = __uint_as_float(h.y << 16);
        w4[j][3] = __uint_as_float(h.y & 0xFFFF0000u);
    }
#pragma unroll
    for (int i = 0; i < 8; i++) {
        float part = 0.f;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint2 h = bf16x4_of<true>(acc[i][j]);
            part += __uint_as_float(h.x << 16) * w4[j][0];
            part += __uint_as_float(h.x & 0xFFFF0000u) * w4[j][1];
            part += __uint_as_float(h.y << 16) * w4[j][2];
            part += __uint_as_float(h.y & 0xFFFF0000u) * w4[j][3];
        }
        // the 4 lanes rl, rl + 16, rl + 32, rl + 48 hold the row's 64 units of this wave
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (lane < 16)
            yp[wave][i * 16 + rl] = part;
    }
    __syncthreads();
    if (tid < rows) {
        const float v = bad[tid] ? __builtin_nanf("")
                                 : (((yp[0][tid] + yp[1][tid]) + yp[2][tid]) + yp[3][tid]) + master[kB4];
        y[b0 + tid] = accumulate ? y[b0 + tid] + scale * v : scale * v;
    }
}

template <int N>
void launch_score_split_n(unsigned grid, hipStream_t st, const uint16_t *wb, const float *master,
                          const uint16_t *split, const uint8_t *pos, int32_t B, float scale, int32_t accumulate,
                          float *y)
{
    hipLaunchKernelGGL(score_split_kernel<N>, dim3(grid), dim3(256), 0, st, wb, master, split, pos, B, scale,
                       accumulate, y);
}

template <int... Ns>
bool launch_score_split(int n, unsigned grid, hipStream_t st, const uint16_t *wb, const float *master,
                        const uint16_t *split, const uint8_t *pos, int32_t B, float scale, int32_t accumulate,
                        float *y, std::integer_sequence<int, Ns...>)
{
    return ((n == Ns + 1 ? (launch_score_split_n<Ns + 1>(grid, st, wb, master, split, pos, B, scale, accumulate, y),
                            true)
                         : false) ||
            ...);
}

// ------------------------------------------------------------------ beam search

// Candidates of one beam step: prefix w (kernel indices of positions 0..d-1)
// grows by each of its m = n - d unused kernels, in increasing kernel order.
// Candidate c = w * m + t: pos[c][i] = position of kernel i (the prefix's, d
// for the new kernel, 16 = unplaced for the rest); cand[c] = w << 8 | kernel.
__global__ void beam_expand_kernel(const uint8_t *prefix, int32_t W, int32_t d, int32_t n, uint8_t *pos,
                                   int32_t *cand)
{
    const int m = n - d;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)W * m)
        return;
    const int64_t w = c / m;
    const int t = (int)(c % m);
    uint32_t used = 0;
    uint8_t p[KO_NN_MAX_TOKENS];
    for (int i = 0; i < n; i++)
        p[i] = KO_NN_UNPLACED;
    for (int j = 0; j < d; j++) {
        const int k = prefix[w * d + j];
        used |= 1u << k;
        p[k] = (uint8_t)j;
    }
    // the t-th unused kernel
    int k = 0, seen = 0;
    for (int i = 0; i < n; i++) {
        if (!((used >> i) & 1u)) {
            if (seen == t)
                k = i;
            seen++;
        }
    }
    p[k] = (uint8_t)d;
    for (int i = 0; i < n; i++)
        pos[c * n + i] = p[i];
    cand[c] = (int32_t)((w << 8) | k);
}

// Diversity rules on the scores of one step, in place (m candidates per
// prefix, W prefixes): with temperature > 0 every score first gets
// temperature * G added, G a standard Gumbel variate from the counter-based
// generator (seed, candidate index); then, with cap > 0, only the cap best
// scores of each prefix's children stay (ties by candidate order) and the
// others become +inf.  One thread per prefix.
__global__ void beam_cap_kernel(float *score, int32_t W, int32_t m, int32_t cap, float temperature, uint64_t seed)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W)
        return;
    float v[KO_NN_MAX_TOKENS];
    for (int t = 0; t < m; t++) {
        float x = score[w * m + t];
        if (temperature > 0.f) {
            // SplitMix64 (Steele, Lea & Flood 2014) of seed + (c + 1) * golden gamma
            uint64_t z = seed + (uint64_t)(w * m + t + 1) * 0x9E3779B97F4A7C15ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            const float u = ((float)(z >> 40) + 0.5f) * (1.0f / 16777216.0f);  // (0, 1)
            x += temperature * -logf(-logf(u));
        }
        v[t] = x;
    }
    if (cap > 0 && cap < m) {
        for (int t = 0; t < m; t++) {
            int better = 0;
            for (int u = 0; u < m; u++)
                better += (v[u] < v[t] || (v[u] == v[t] && u < t)) ? 1 : 0;
            if (better >= cap)
                v[t] = INFINITY;
        }
    }
    for (int t = 0; t < m; t++)
        score[w * m + t] = v[t];
}

// New prefixes: out[r] = prefix[parent] followed by the candidate's kernel,
// for the chosen candidates idx[0..keep).
__global__ void beam_gather_kernel(const uint8_t *prefix, int32_t d, const int32_t *cand, const int64_t *idx,
                                   int32_t keep, uint8_t *out)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= keep)
        return;
    const int32_t cw = cand[idx[r]];
    const int64_t w = cw >> 8;
    for (int j = 0; j < d; j++)
        out[r * (d + 1) + j] = prefix[w * d + j];
    out[r * (d + 1) + d] = (uint8_t)(cw & 0xFF);
}

// ------------------------------------------------------------------ host side

thread_local std::string g_err = "no error";

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define NN_HIP(call)                                                            \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess)                                                   \
            return fail(KO_EHIP, "%s: %s", #call, hipGetErrorString(e_));       \
    } while (0)

#define NN_LAUNCHED()                                                           \
    do {                                                                        \
        hipError_t e_ = hipGetLastError();                                      \
        if (e_ != hipSuccess)                                                   \
            return fail(KO_EHIP, "kernel launch: %s", hipGetErrorString(e_));   \
    } while (0)

unsigned grid1(int64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

struct ko_nn_graph {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

struct Work {
    float *P1, *P2, *P3;                    // split-K partials of dW1, dW2, dW3
    float *Pb1, *Pout, *Pb3, *Pb2, *Ploss;  // column-sum partials
    float *Z1, *S, *Z2, *Z3, *y, *dy, *sq, *dZ3, *dZ2, *dS;
    uint16_t *Sb, *A2b, *A3b, *dZ3b, *dZ2b, *dZ1b;
    uint8_t *cnt;   // tokens of a sample with Z1 > 0, per column
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// split count for a reduction over K rows: chunks of at least 256, at most `cap`
int64_t split_count(int64_t K, int64_t cap)
{
    int64_t s = K / 256;
    return s < 1 ? 1 : (s > cap ? cap : s);
}

// split counts: enough workgroups to fill the chip, few enough partials that
// the ordered reduction stays short; column sums use chunks of >= 16 rows
constexpr int64_t kSplitCapW1 = 256, kSplitCapW = 32, kColChunks = 4096, kColRows = 16;

// rows per chunk and chunk count of a column sum over `rows` rows
int64_t col_chunk(int64_t rows) { return std::max<int64_t>(kColRows, (rows + kColChunks - 1) / kColChunks); }
int64_t col_chunks(int64_t rows) { return (rows + col_chunk(rows) - 1) / col_chunk(rows); }

// K per split-K workgroup (a multiple of the MFMA k step) and the splits used
int64_t split_chunk(int64_t K, int64_t cap)
{
    const int64_t splits = split_count(K, cap);
    return ((K + splits - 1) / splits + kKStep - 1) / kKStep * kKStep;
}
int64_t splits_used(int64_t K, int64_t cap) { return (K + split_chunk(K, cap) - 1) / split_chunk(K, cap); }

Work work_of(void *p, int64_t B, int64_t n, size_t *total)
{
    char *c = (char *)p;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *r = c ? c + off : nullptr;
        off += align256(bytes);
        return r;
    };
    const int64_t T = B * n, BH = B * kHid, TH = T * kHid;
    Work w;
    w.P1 = (float *)take((size_t)splits_used(T, kSplitCapW1) * kHid * kIn * 4);
    w.P2 = (float *)take((size_t)splits_used(B, kSplitCapW) * kHid * kHid * 4);
    w.P3 = (float *)take((size_t)splits_used(B, kSplitCapW) * kHid * kHid * 4);
    w.Pb1 = (float *)take((size_t)col_chunks(B) * kHid * 4);
    w.Pout = (float *)take((size_t)col_chunks(B) * (kHid + 1) * 4);
    w.Pb3 = (float *)take((size_t)col_chunks(B) * kHid * 4);
    w.Pb2 = (float *)take((size_t)col_chunks(B) * kHid * 4);
    w.Ploss = (float *)take((size_t)col_chunks(B) * 4);
    w.Z1 = (float *)take(TH * 4);
    w.dZ1b = (uint16_t *)take(TH * 2);
    w.S = (float *)take(BH * 4);
    w.Sb = (uint16_t *)take(BH * 2);
    w.Z2 = (float *)take(BH * 4);
    w.A2b = (uint16_t *)take(BH * 2);
    w.Z3 = (float *)take(BH * 4);
    w.A3b = (uint16_t *)take(BH * 2);
    w.dZ3 = (float *)take(BH * 4);
    w.dZ3b = (uint16_t *)take(BH * 2);
    w.dZ2 = (float *)take(BH * 4);
    w.dZ2b = (uint16_t *)take(BH * 2);
    w.dS = (float *)take(BH * 4);
    w.y = (float *)take(B * 4);
    w.dy = (float *)take(B * 4);
    w.sq = (float *)take(B * 4);
    w.cnt = (uint8_t *)take(BH);
    *total = off;
    return w;
}

bool nt_eligible(const GemmArgs &a)
{
    auto aligned = [](const void *p) { return ((uintptr_t)p & 15u) == 0; };
    return !a.P && a.sak == 1 && a.sbk == 1 && a.K % kKStep == 0 && a.N % kNtTile == 0 && a.sam % 8 == 0 &&
           a.sbn % 8 == 0 && aligned(a.A) && aligned(a.B);
}

// The panel kernel takes each operand k-contiguous (K % 8 == 0) or
// r-contiguous (rows M or N % 8 == 0), with 16-byte aligned bases and pitches.
bool panel_operand_ok(const void *p, int64_t sr, int64_t sk, int32_t R, int32_t K)
{
    if (((uintptr_t)p & 15u) != 0)
        return false;
    if (sk == 1)
        return sr % 8 == 0 && K % 8 == 0;
    return sr == 1 && sk % 8 == 0 && R % 8 == 0;
}

bool panel_eligible(const GemmArgs &a)
{
    return panel_operand_ok(a.A, a.sam, a.sak, a.M, a.K) && panel_operand_ok(a.B, a.sbn, a.sbk, a.N, a.K);
}

void launch_panel(const GemmArgs &a, dim3 grid, hipStream_t st)
{
    const bool ak = a.sak == 1, bk = a.sbk == 1;
    if (ak && bk)
        hipLaunchKernelGGL((panel_gemm_kernel<true, true>), grid, dim3(256), 0, st, a);
    else if (ak)
        hipLaunchKernelGGL((panel_gemm_kernel<true, false>), grid, dim3(256), 0, st, a);
    else if (bk)
        hipLaunchKernelGGL((panel_gemm_kernel<false, true>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((panel_gemm_kernel<false, false>), grid, dim3(256), 0, st, a);
}

// Above this many 128 x 128 tiles the NT kernel's larger tiles read the
// operands fewer times than 64 x 64 panels; below it they leave CUs idle.
constexpr int64_t kNtMinTiles = 1024;

int gemm(const GemmArgs &a, hipStream_t st)
{
    if (a.M <= 0 || a.N <= 0 || a.K <= 0)
        return KO_OK;
    const int64_t nt_tiles = (a.M + kNtTile - 1) / kNtTile * (a.N / kNtTile);
    // (a product with K = 32 is one k step: the NT kernel's smaller LDS
    // footprint keeps more workgroups resident for its output-bound work)
    const bool nt_better = nt_eligible(a) && (nt_tiles >= kNtMinTiles || a.K <= kKStep);
    if (panel_eligible(a) && !nt_better) {
        dim3 g((unsigned)((a.M + kTile - 1) / kTile), (unsigned)((a.N + kTile - 1) / kTile));
        launch_panel(a, g, st);
        NN_LAUNCHED();
        return KO_OK;
    }
    if (nt_eligible(a)) {
        dim3 g((unsigned)((a.M + kNtTile - 1) / kNtTile), (unsigned)(a.N / kNtTile));
        hipLaunchKernelGGL(gemm_nt_kernel, g, dim3(256), 0, st, a);
        NN_LAUNCHED();
        return KO_OK;
    }
    dim3 grid((unsigned)((a.M + kTile - 1) / kTile), (unsigned)((a.N + kTile - 1) / kTile));
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, st, a);
    NN_LAUNCHED();
    return KO_OK;
}

// Split-K partial products of a weight gradient: workgroup z of the grid
// stores sum over its K chunk of A(m,k) B(k,n) to P + z M N; the finish
// kernel adds the splits_used(K, cap) partials in order.
int gemm_partials(GemmArgs a, float *P, int64_t cap, hipStream_t st)
{
    if (a.M <= 0 || a.N <= 0 || a.K <= 0)
        return KO_OK;
    a.kchunk = split_chunk(a.K, cap);
    a.P = P;
    a.C = nullptr;
    a.Cb = nullptr;
    dim3 grid((unsigned)((a.M + kTile - 1) / kTile), (unsigned)((a.N + kTile - 1) / kTile),
              (unsigned)splits_used(a.K, cap));
    if (panel_eligible(a))
        launch_panel(a, grid, st);
    else
        hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, st, a);
    NN_LAUNCHED();
    return KO_OK;
}

GemmArgs gemm_args(const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B, int64_t sbk,
                   int64_t sbn, int32_t M, int32_t N, int32_t K)
{
    GemmArgs a;
    std::memset(&a, 0, sizeof a);
    a.A = A;
    a.sam = sam;
    a.sak = sak;
    a.B = B;
    a.sbk = sbk;
    a.sbn = sbn;
    a.M = M;
    a.N = N;
    a.K = K;
    a.epi = kEpiNone;
    return a;
}

int check_batch(const void *state, const void *x, int32_t B, int32_t n, const void *work)
{
    if (!state || !x || !work)
        return fail(KO_EINVAL, "state, tokens and workspace must not be NULL");
    if (B < 1 || n < 1 || n > KO_NN_MAX_TOKENS)
        return fail(KO_EINVAL, "B must be >= 1 and n in 1..%d", KO_NN_MAX_TOKENS);
    if ((int64_t)B * n * kHid > (int64_t)1 << 31)
        return fail(KO_EINVAL, "batch too large");
    return KO_OK;
}

int forward_impl(const State &s, const uint16_t *x, int32_t B, int32_t n, float *y, Work &w,
                 hipStream_t st)
{
    int rc;
    const int32_t T = B * n;
    // Z1 = X W1^T + b1
    GemmArgs a = gemm_args(x, kIn, 1, s.wb + kW1, 1, kIn, T, kHid, kIn);
    a.bias = s.master + kB1;
    a.C = w.Z1;
    a.ldc = kHid;
    if ((rc = gemm(a, st)))
        return rc;
    hipLaunchKernelGGL(pool_kernel, dim3(grid1((int64_t)B * kHid)), dim3(256), 0, st, w.Z1, B, n, w.S,
                       w.Sb, w.cnt);
    NN_LAUNCHED();
    // A2 = relu(S W2^T + b2)
    a = gemm_args(w.Sb, kHid, 1, s.wb + kW2, 1, kHid, B, kHid, kHid);
    a.bias = s.master + kB2;
    a.epi = kEpiRelu;
    a.C = w.Z2;
    a.ldc = kHid;
    a.Cb = w.A2b;
    a.ldcb = kHid;
    if ((rc = gemm(a, st)))
        return rc;
    // A3 = relu(A2 W3^T + b3)
    a = gemm_args(w.A2b, kHid, 1, s.wb + kW3, 1, kHid, B, kHid, kHid);
    a.bias = s.master + kB3;
    a.epi = kEpiRelu;
    a.C = w.Z3;
    a.ldc = kHid;
    a.Cb = w.A3b;
    a.ldcb = kHid;
    if ((rc = gemm(a, st)))
        return rc;
    if (!y)
        return KO_OK;   // the training step's head kernel computes y
    hipLaunchKernelGGL(out_forward_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, st, w.A3b,
                       s.wb, s.master, B, y);
    NN_LAUNCHED();
    return KO_OK;
}

// Scoring forward from positions: S from the layer-1 table, then the two
// hidden layers (BF16 outputs only) and the output layer.
int forward_positions_impl(const State &s, const float *T, const uint8_t *pos, int32_t B, int32_t n,
                           float *y, uint16_t *Sb, uint16_t *A2b, uint16_t *A3b, hipStream_t st)
{
    int rc;
    hipLaunchKernelGGL(gather_pool_kernel, dim3((unsigned)B), dim3(kHid), 0, st, T, pos, n, Sb);
    NN_LAUNCHED();
    GemmArgs a = gemm_args(Sb, kHid, 1, s.wb + kW2, 1, kHid, B, kHid, kHid);
    a.bias = s.master + kB2;
    a.epi = kEpiRelu;
    a.Cb = A2b;
    a.ldcb = kHid;
    if ((rc = gemm(a, st)))
        return rc;
    a = gemm_args(A2b, kHid, 1, s.wb + kW3, 1, kHid, B, kHid, kHid);
    a.bias = s.master + kB3;
    a.epi = kEpiRelu;
    a.Cb = A3b;
    a.ldcb = kHid;
    if ((rc = gemm(a, st)))
        return rc;
    hipLaunchKernelGGL(out_forward_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, st, A3b, s.wb,
                       s.master, B, y);
    NN_LAUNCHED();
    return KO_OK;
}

// Forward, loss and every gradient of a minibatch (13 launches, no host
// synchronisation, nothing allocated); with `sched` set the step counter
// advances and the finish kernel applies Adam, which makes this one training
// step that a HIP graph can capture.
int backward_impl(const State &s, const uint16_t *x, const float *t, int32_t B, int32_t n, float *loss, Work &w,
                  ko_nn_sched *sched, hipStream_t st)
{
    int rc;
    const int64_t T = (int64_t)B * n;
    if ((rc = forward_impl(s, x, B, n, nullptr, w, st)))
        return rc;
    hipLaunchKernelGGL(head_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, st, w.A3b, s.wb, s.master, w.Z3,
                       t, B, w.y, w.dy, w.sq, w.dZ3, w.dZ3b, sched);
    NN_LAUNCHED();
    // layer 3: dZ2 = (dZ3b W3b) [Z2 > 0]; dW3 = dZ3b^T A2b (split-K partials)
    GemmArgs a = gemm_args(w.dZ3b, kHid, 1, s.wb + kW3, kHid, 1, B, kHid, kHid);
    a.epi = kEpiMask;
    a.zref = w.Z2;
    a.ldz = kHid;
    a.C = w.dZ2;
    a.ldc = kHid;
    a.Cb = w.dZ2b;
    a.ldcb = kHid;
    if ((rc = gemm(a, st)))
        return rc;
    if ((rc = gemm_partials(gemm_args(w.dZ3b, 1, kHid, w.A2b, kHid, 1, kHid, kHid, B), w.P3, kSplitCapW, st)))
        return rc;
    // layer 2: dS = dZ2b W2b; dW2 = dZ2b^T Sb
    a = gemm_args(w.dZ2b, kHid, 1, s.wb + kW2, kHid, 1, B, kHid, kHid);
    a.C = w.dS;
    a.ldc = kHid;
    if ((rc = gemm(a, st)))
        return rc;
    if ((rc = gemm_partials(gemm_args(w.dZ2b, 1, kHid, w.Sb, kHid, 1, kHid, kHid, B), w.P2, kSplitCapW, st)))
        return rc;
    // layer 1: dZ1 = dS (per token) [Z1 > 0]; dW1 = dZ1b^T X
    hipLaunchKernelGGL(dz1_kernel, dim3((unsigned)((T + 3) / 4)), dim3(256), 0, st, w.dS, w.Z1, T, n, w.dZ1b);
    NN_LAUNCHED();
    if ((rc = gemm_partials(gemm_args(w.dZ1b, 1, kHid, x, kIn, 1, kHid, kIn, (int32_t)T), w.P1, kSplitCapW1,
                            st)))
        return rc;
    // column sums over the samples: dw4 = sum dy A3b and db4 = sum dy; db3; db2;
    // db1 = sum dS cnt (dZ1 summed over a sample's tokens); the loss
    ColMulti cm;
    std::memset(&cm, 0, sizeof cm);
    const int64_t chB = col_chunk(B), nB = col_chunks(B);
    auto prob = [&](int q, const float *Xf, const uint16_t *Xb, int64_t ld, int32_t cols, const float *wrow,
                    int32_t with_w, float *part, const uint8_t *Xm = nullptr) {
        ColProblem &p = cm.p[q];
        p.Xf = Xf, p.Xb = Xb, p.Xm = Xm, p.wrow = wrow, p.part = part;
        p.ld = ld, p.rows = B, p.chunk = chB;
        p.cols = cols, p.with_w = with_w, p.first = (int32_t)(q * nB);
    };
    prob(0, nullptr, w.A3b, kHid, kHid, w.dy, 1, w.Pout);
    prob(1, w.dZ3, nullptr, kHid, kHid, nullptr, 0, w.Pb3);
    prob(2, w.dZ2, nullptr, kHid, kHid, nullptr, 0, w.Pb2);
    prob(3, w.sq, nullptr, 1, 1, nullptr, 0, w.Ploss);
    prob(4, w.dS, nullptr, kHid, kHid, nullptr, 0, w.Pb1, w.cnt);
    cm.count = kColProblems;
    hipLaunchKernelGGL(colsum_multi_kernel, dim3((unsigned)(kColProblems * nB)), dim3(320), 0, st, cm);
    NN_LAUNCHED();
    FinishArgs f;
    std::memset(&f, 0, sizeof f);
    int32_t blocks = 0;
    auto seg = [&](const float *P, int64_t stride, int64_t rows, int32_t count, int32_t param) {
        Segment &g = f.seg[f.count++];
        g.P = P, g.stride = stride, g.rows = (int32_t)rows, g.count = count, g.param = param, g.first = blocks;
        g.groups = rows <= kFinShort ? 1 : kFinGroups;
        const int32_t per = 256 / g.groups;
        blocks += (count + per - 1) / per;
    };
    seg(w.P1, (int64_t)kHid * kIn, splits_used(T, kSplitCapW1), kHid * kIn, (int32_t)kW1);
    seg(w.P2, (int64_t)kHid * kHid, splits_used(B, kSplitCapW), kHid * kHid, (int32_t)kW2);
    seg(w.P3, (int64_t)kHid * kHid, splits_used(B, kSplitCapW), kHid * kHid, (int32_t)kW3);
    seg(w.Pb1, kHid, nB, kHid, (int32_t)kB1);
    seg(w.Pout, kHid + 1, nB, kHid + 1, (int32_t)kW4);   // dw4 then db4 (kB4 = kW4 + 256)
    seg(w.Pb3, kHid, nB, kHid, (int32_t)kB3);
    seg(w.Pb2, kHid, nB, kHid, (int32_t)kB2);
    seg(w.Ploss, 1, nB, 1, -1);
    f.B = B;
    f.grad = s.grad;
    f.loss_out = loss;
    f.sched = sched;
    f.adam = AdamArgs{s.master, s.m, s.v, s.wb, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};   // the rest comes from sched
    hipLaunchKernelGGL(finish_kernel, dim3((unsigned)blocks), dim3(256), 0, st, f);
    NN_LAUNCHED();
    return KO_OK;
}

}  // namespace

extern "C" {

size_t ko_nn_num_params(void) { return kNP; }

size_t ko_nn_state_bytes(void) { return kNPad * 4 * 4 + kNPad * 2; }

size_t ko_nn_work_bytes(int32_t B, int32_t n)
{
    if (B < 1 || n < 1)
        return 0;
    size_t total = 0;
    (void)work_of(nullptr, B, n, &total);
    return total;
}

int ko_nn_load(void *state_dev, const float *params_host, void *hip_stream)
{
    if (!state_dev || !params_host)
        return fail(KO_EINVAL, "state and params must not be NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    State s = state_of(state_dev);
    std::vector<float> buf(kNPad, 0.f);
    std::memcpy(buf.data(), params_host, kNP * sizeof(float));
    NN_HIP(hipMemcpyAsync(s.master, buf.data(), kNPad * 4, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(zero_f32_kernel, dim3(grid1(3 * (int64_t)kNPad)), dim3(256), 0, st, s.grad,
                       3 * (int64_t)kNPad);
    NN_LAUNCHED();
    hipLaunchKernelGGL(refresh_kernel, dim3(grid1(kNPad)), dim3(256), 0, st, s.master, s.wb,
                       (int64_t)kNPad);
    NN_LAUNCHED();
    NN_HIP(hipStreamSynchronize(st));
    return KO_OK;
}

int ko_nn_read(const void *state_dev, int32_t which, float *out_host, void *hip_stream)
{
    if (!state_dev || !out_host || which < 0 || which > 3)
        return fail(KO_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    State s = state_of(const_cast<void *>(state_dev));
    const float *src[4] = {s.master, s.grad, s.m, s.v};
    NN_HIP(hipMemcpyAsync(out_host, src[which], kNP * 4, hipMemcpyDeviceToHost, st));
    NN_HIP(hipStreamSynchronize(st));
    return KO_OK;
}

int ko_nn_features(const ko_gpu_model *g, const ko_kernel *k, int32_t n, float *out)
{
    if (!g || !k || !out || n < 1)
        return fail(KO_EINVAL, "bad arguments");
    if (g->n_cu < 1 || g->reg_cu < 1 || g->lds_cu < 1 || g->wave_cu < 1 || g->blk_cu < 1 ||
        g->rb_milli < 1 || g->wave_size < 1)
        return fail(KO_EINVAL, "invalid gpu model");
    for (int32_t i = 0; i < n; i++) {
        const ko_kernel &q = k[i];
        if (q.n_tblk < 1 || q.n_inst < 1 || q.lds_blk < 0 || q.waves_blk < 1 || q.regs_thr < 1 ||
            q.r_milli < 1)
            return fail(KO_EINVAL, "kernel %d: invalid descriptor", i);
        const double ureg = (double)q.regs_thr * q.waves_blk * g->wave_size;
        const double ulds = (double)q.lds_blk;
        const double uwave = (double)q.waves_blk;
        if (ureg > (double)g->reg_cu || ulds > (double)g->lds_cu || uwave > (double)g->wave_cu)
            return fail(KO_EINVAL, "kernel %d: block exceeds an empty CU", i);
        const int64_t hi = q.r_milli > g->rb_milli ? q.r_milli : g->rb_milli;
        const double dur = (double)((q.n_inst * hi + q.r_milli - 1) / q.r_milli);
        int64_t occ = g->blk_cu;
        occ = std::min<int64_t>(occ, g->reg_cu / (int64_t)ureg);
        occ = std::min<int64_t>(occ, g->wave_cu / q.waves_blk);
        if (q.lds_blk > 0)
            occ = std::min<int64_t>(occ, g->lds_cu / q.lds_blk);
        float *f = out + (size_t)i * KO_NN_FEAT;
        f[0] = (float)(std::log2((double)q.n_tblk) / 16.0);
        f[1] = (float)(uwave / (double)g->wave_cu);
        f[2] = (float)(ureg / (double)g->reg_cu);
        f[3] = (float)(ulds / (double)g->lds_cu);
        f[4] = (float)(std::log2(dur) / 32.0);
        f[5] = (float)(std::log2((double)q.r_milli / (double)g->rb_milli) / 8.0);
        f[6] = (float)((double)occ / (double)g->blk_cu);
        f[7] = (float)(std::log2(1.0 + (double)q.n_tblk / ((double)occ * (double)g->n_cu)) / 8.0);
    }
    return KO_OK;
}

int ko_nn_lower_bound(const ko_gpu_model *g, const ko_kernel *k, int32_t n, int64_t *lb_out)
{
    if (!g || !k || !lb_out || n < 1)
        return fail(KO_EINVAL, "bad arguments");
    const int64_t cap[4] = {g->reg_cu, g->lds_cu, g->wave_cu, g->blk_cu};
    __int128 area[4] = {0, 0, 0, 0};
    int64_t lb = 0;
    for (int32_t i = 0; i < n; i++) {
        const ko_kernel &q = k[i];
        if (q.n_tblk < 1 || q.n_inst < 1 || q.r_milli < 1 || q.waves_blk < 1 || q.regs_thr < 1)
            return fail(KO_EINVAL, "kernel %d: invalid descriptor", i);
        const int64_t hi = q.r_milli > g->rb_milli ? q.r_milli : g->rb_milli;
        const int64_t d = (q.n_inst * hi + q.r_milli - 1) / q.r_milli;
        lb = std::max(lb, d);
        const int64_t u[4] = {(int64_t)q.regs_thr * q.waves_blk * g->wave_size, q.lds_blk,
                              q.waves_blk, 1};
        for (int x = 0; x < 4; x++)
            area[x] += (__int128)q.n_tblk * d * u[x];
    }
    for (int x = 0; x < 4; x++) {
        const __int128 den = (__int128)g->n_cu * cap[x];
        const __int128 v = (area[x] + den - 1) / den;
        lb = std::max<int64_t>(lb, (int64_t)v);
    }
    *lb_out = lb;
    return KO_OK;
}

int ko_nn_tokens(const float *feat_dev, const int32_t *set_of_dev, const uint8_t *pos_dev,
                 const int64_t *rows_dev, int32_t B, int32_t n, uint16_t *x_dev, void *hip_stream)
{
    if (!feat_dev || !pos_dev || !x_dev || B < 1 || n < 1 || n > KO_NN_MAX_TOKENS)
        return fail(KO_EINVAL, "bad arguments");
    hipLaunchKernelGGL(tokens_kernel, dim3(grid1((int64_t)B * n * kIn)), dim3(256), 0,
                       (hipStream_t)hip_stream, feat_dev, set_of_dev, pos_dev, rows_dev, B, n, x_dev);
    NN_LAUNCHED();
    return KO_OK;
}

int ko_nn_targets(const int64_t *makespans_dev, const int32_t *set_of_dev, const int64_t *center_dev,
                  const int64_t *scale_dev, const int64_t *rows_dev, int32_t B, float *t_dev,
                  void *hip_stream)
{
    if (!makespans_dev || !center_dev || !scale_dev || !t_dev || B < 1)
        return fail(KO_EINVAL, "bad arguments");
    hipLaunchKernelGGL(targets_kernel, dim3(grid1(B)), dim3(256), 0, (hipStream_t)hip_stream,
                       makespans_dev, set_of_dev, center_dev, scale_dev, rows_dev, B, t_dev);
    NN_LAUNCHED();
    return KO_OK;
}

int ko_nn_within_set_ranks(const int64_t *values_dev, int32_t n_sets, int32_t per_set, int64_t *ranks_dev,
                           void *hip_stream)
{
    if (!values_dev || !ranks_dev || n_sets < 1 || per_set < 1 || per_set > kRankMax)
        return fail(KO_EINVAL, "need values, ranks, n_sets >= 1 and 1 <= per_set <= %d", kRankMax);
    int32_t p2 = 1;
    while (p2 < per_set)
        p2 <<= 1;
    hipLaunchKernelGGL(within_set_rank_kernel, dim3((unsigned)n_sets), dim3(1024), 0, (hipStream_t)hip_stream,
                       values_dev, per_set, p2, ranks_dev);
    NN_LAUNCHED();
    return KO_OK;
}

int ko_nn_forward(const void *state_dev, const uint16_t *x_dev, int32_t B, int32_t n, float *y_dev,
                  void *work_dev, void *hip_stream)
{
    int rc = check_batch(state_dev, x_dev, B, n, work_dev);
    if (rc)
        return rc;
    if (!y_dev)
        return fail(KO_EINVAL, "y must not be NULL");
    size_t total;
    Work w = work_of(work_dev, B, n, &total);
    return forward_impl(state_of(const_cast<void *>(state_dev)), x_dev, B, n, y_dev, w,
                        (hipStream_t)hip_stream);
}

int ko_nn_backward(void *state_dev, const uint16_t *x_dev, const float *t_dev, int32_t B, int32_t n,
                   float *loss_dev, void *work_dev, void *hip_stream)
{
    int rc = check_batch(state_dev, x_dev, B, n, work_dev);
    if (rc)
        return rc;
    if (!t_dev)
        return fail(KO_EINVAL, "targets must not be NULL");
    size_t total;
    Work w = work_of(work_dev, B, n, &total);
    return backward_impl(state_of(state_dev), x_dev, t_dev, B, n, loss_dev, w, nullptr, (hipStream_t)hip_stream);
}

int ko_nn_train_step(void *state_dev, const uint16_t *x_dev, const float *t_dev, int32_t B, int32_t n,
                     ko_nn_sched *sched_dev, float *loss_dev, void *work_dev, void *hip_stream)
{
    int rc = check_batch(state_dev, x_dev, B, n, work_dev);
    if (rc)
        return rc;
    if (!t_dev || !sched_dev)
        return fail(KO_EINVAL, "targets and schedule must not be NULL");
    size_t total;
    Work w = work_of(work_dev, B, n, &total);
    return backward_impl(state_of(state_dev), x_dev, t_dev, B, n, loss_dev, w, sched_dev, (hipStream_t)hip_stream);
}

int ko_nn_batch(const float *feat_dev, const int32_t *set_of_dev, const uint8_t *pos_dev,
                const int64_t *makespans_dev, const int64_t *center_dev, const int64_t *scale_dev,
                const int64_t *perm_dev, const ko_nn_sched *sched_dev, int32_t B, int32_t n, uint16_t *x_dev,
                float *t_dev, void *hip_stream)
{
    if (!feat_dev || !pos_dev || !makespans_dev || !center_dev || !scale_dev || !perm_dev || !sched_dev || !x_dev ||
        !t_dev)
        return fail(KO_EINVAL, "only set_of may be NULL");
    if (B < 1 || n < 1 || n > KO_NN_MAX_TOKENS)
        return fail(KO_EINVAL, "B must be >= 1 and n in 1..%d", KO_NN_MAX_TOKENS);
    hipLaunchKernelGGL(batch_kernel, dim3(grid1((int64_t)B * n * kIn)), dim3(256), 0, (hipStream_t)hip_stream,
                       feat_dev, set_of_dev, pos_dev, makespans_dev, center_dev, scale_dev, perm_dev, sched_dev, B, n,
                       x_dev, t_dev);
    NN_LAUNCHED();
    return KO_OK;
}

int ko_nn_step_capture(void *state_dev, const float *feat_dev, const int32_t *set_of_dev, const uint8_t *pos_dev,
                       const int64_t *makespans_dev, const int64_t *center_dev, const int64_t *scale_dev,
                       const int64_t *perm_dev, ko_nn_sched *sched_dev, int32_t B, int32_t n, uint16_t *x_dev,
                       float *t_dev, float *loss_dev, void *work_dev, void *hip_stream, ko_nn_graph **out)
{
    if (!out)
        return fail(KO_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!hip_stream)
        return fail(KO_EINVAL, "capture needs a created stream, not the null stream");
    int rc = check_batch(state_dev, x_dev, B, n, work_dev);
    if (rc)
        return rc;
    if (!feat_dev || !pos_dev || !makespans_dev || !center_dev || !scale_dev || !perm_dev || !sched_dev || !t_dev)
        return fail(KO_EINVAL, "only set_of and loss may be NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    NN_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(batch_kernel, dim3(grid1((int64_t)B * n * kIn)), dim3(256), 0, st, feat_dev, set_of_dev,
                       pos_dev, makespans_dev, center_dev, scale_dev, perm_dev, sched_dev, B, n, x_dev, t_dev);
    rc = KO_OK;
    if (hipGetLastError() != hipSuccess)
        rc = fail(KO_EHIP, "batch kernel launch failed during capture");
    size_t total;
    Work w = work_of(work_dev, B, n, &total);
    if (!rc)
        rc = backward_impl(state_of(state_dev), x_dev, t_dev, B, n, loss_dev, w, sched_dev, st);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc || e != hipSuccess) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return rc ? rc : fail(KO_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(KO_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    }
    int device = 0;
    (void)hipGetDevice(&device);
    ko_nn_graph *g = new ko_nn_graph();
    g->device = device;
    g->graph = graph;
    g->exec = exec;
    *out = g;
    return KO_OK;
}

int ko_nn_graph_launch(ko_nn_graph *graph, void *hip_stream)
{
    if (!graph)
        return fail(KO_EINVAL, "graph must not be NULL");
    NN_HIP(hipGraphLaunch(graph->exec, (hipStream_t)hip_stream));
    return KO_OK;
}

int ko_nn_graph_destroy(ko_nn_graph *graph)
{
    if (!graph)
        return KO_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(graph->device);
    (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    (void)hipSetDevice(prev);
    delete graph;
    return KO_OK;
}

int ko_nn_adam(void *state_dev, int32_t step, float lr, float beta1, float beta2, float eps,
               void *hip_stream)
{
    if (!state_dev || step < 1)
        return fail(KO_EINVAL, "bad arguments");
    State s = state_of(state_dev);
    const AdamArgs a{s.master, s.m, s.v, s.wb, lr, beta1, beta2, eps, 0.f, 0.f};
    hipLaunchKernelGGL(adam_kernel, dim3(grid1(kNP)), dim3(256), 0, (hipStream_t)hip_stream, s.grad,
                       (int64_t)kNP, a, step);
    NN_LAUNCHED();
    return KO_OK;
}

int ko_nn_layer1_table(const void *state_dev, const float *feat_dev, int32_t n, float *table_dev,
                       void *hip_stream)
{
    if (!state_dev || !feat_dev || !table_dev)
        return fail(KO_EINVAL, "state, features and table must not be NULL");
    if (n < 1 || n > KO_NN_MAX_TOKENS)
        return fail(KO_EINVAL, "n must be in 1..%d", KO_NN_MAX_TOKENS);
    State s = state_of(const_cast<void *>(state_dev));
    hipLaunchKernelGGL(table_kernel, dim3(grid1((int64_t)n * KO_NN_POS * kHid)), dim3(256), 0,
                       (hipStream_t)hip_stream, s.wb, s.master, feat_dev, n, table_dev);
    NN_LAUNCHED();
    return KO_OK;
}

size_t ko_nn_score_work_bytes(int32_t B)
{
    if (B < 1)
        return 0;
    return 3 * align256((size_t)B * kHid * 2);
}

int ko_nn_forward_positions(const void *state_dev, const float *table_dev, const uint8_t *pos_dev,
                            int32_t B, int32_t n, float *y_dev, void *work_dev, void *hip_stream)
{
    if (!state_dev || !table_dev || !pos_dev || !y_dev || !work_dev)
        return fail(KO_EINVAL, "state, table, positions, y and workspace must not be NULL");
    if (B < 1 || n < 1 || n > KO_NN_MAX_TOKENS)
        return fail(KO_EINVAL, "B must be >= 1 and n in 1..%d", KO_NN_MAX_TOKENS);
    const size_t part = align256((size_t)B * kHid * 2);
    char *c = (char *)work_dev;
    return forward_positions_impl(state_of(const_cast<void *>(state_dev)), table_dev, pos_dev, B, n,
                                  y_dev, (uint16_t *)c, (uint16_t *)(c + part),
                                  (uint16_t *)(c + 2 * part), (hipStream_t)hip_stream);
}

int ko_nn_score(const void *state_dev, const float *feat_dev, const uint8_t *pos_dev, int32_t B, int32_t n,
                float *y_dev, void *hip_stream)
{
    if (!state_dev || !feat_dev || !pos_dev || !y_dev)
        return fail(KO_EINVAL, "state, features, positions and y must not be NULL");
    if (B < 1 || n < 1 || n > KO_NN_MAX_TOKENS)
        return fail(KO_EINVAL, "B must be >= 1 and n in 1..%d", KO_NN_MAX_TOKENS);
    const State s = state_of(const_cast<void *>(state_dev));
    const unsigned grid = (unsigned)(((int64_t)B + kScTile - 1) / kScTile);
    // one instantiation per set size: the kernel loop is unrolled over the tokens
    launch_score(n, grid, (hipStream_t)hip_stream, s.wb, s.master, feat_dev, pos_dev, B, y_dev,
                 std::make_integer_sequence<int, KO_NN_MAX_TOKENS>{});
    NN_LAUNCHED();
    return KO_OK;
}

size_t ko_nn_split_table_bytes(int32_t n)
{
    if (n < 1 || n > KO_NN_MAX_TOKENS)
        return 0;
    return ((size_t)2 * kHid * kSplitK(n) + (size_t)2 * kHid * kHid) * sizeof(uint16_t);
}

int ko_nn_split_table(const void *state_dev, const float *feat_dev, int32_t n, uint16_t *split_dev,
                      void *hip_stream)
{
    if (!state_dev || !feat_dev || !split_dev)
        return fail(KO_EINVAL, "state, features and table must not be NULL");
    if (n < 1 || n > KO_NN_MAX_TOKENS)
        return fail(KO_EINVAL, "n must be in 1..%d", KO_NN_MAX_TOKENS);
    if (((uintptr_t)split_dev & 15u) != 0)
        return fail(KO_EINVAL, "the table must be 16-byte aligned");
    State s = state_of(const_cast<void *>(state_dev));
    const int32_t KP = kSplitK(n);
    hipLaunchKernelGGL(split_table_kernel, dim3((unsigned)(KP / kKStep), kHid / 16), dim3(kFragElems), 0,
                       (hipStream_t)hip_stream, s.wb, s.master, feat_dev, n, KP, split_dev);
    NN_LAUNCHED();
    hipLaunchKernelGGL(frag_weights_kernel, dim3(kHid / kKStep, kHid / 16, 2), dim3(kFragElems), 0,
                       (hipStream_t)hip_stream, s.wb, split_dev + (size_t)2 * kHid * KP);
    NN_LAUNCHED();
    return KO_OK;
}

int ko_nn_score_split_acc(const void *state_dev, const uint16_t *split_dev, const uint8_t *pos_dev, int32_t B,
                          int32_t n, float scale, int32_t accumulate, float *y_dev, void *hip_stream)
{
    if (!state_dev || !split_dev || !pos_dev || !y_dev)
        return fail(KO_EINVAL, "state, table, positions and y must not be NULL");
    if (B < 1 || n < 1 || n > KO_NN_MAX_TOKENS)
        return fail(KO_EINVAL, "B must be >= 1 and n in 1..%d", KO_NN_MAX_TOKENS);
    if (((uintptr_t)split_dev & 15u) != 0)
        return fail(KO_EINVAL, "the table must be 16-byte aligned");
    const State s = state_of(const_cast<void *>(state_dev));
    const unsigned grid = (unsigned)(((int64_t)B + kSpRows - 1) / kSpRows);
    launch_score_split(n, grid, (hipStream_t)hip_stream, s.wb, s.master, split_dev, pos_dev, B, scale,
                       accumulate ? 1 : 0, y_dev, std::make_integer_sequence<int, KO_NN_MAX_TOKENS>{});
    NN_LAUNCHED();
    return KO_OK;
}

int ko_nn_score_split(const void *state_dev, const uint16_t *split_dev, const uint8_t *pos_dev, int32_t B,
                      int32_t n, float *y_dev, void *hip_stream)
{
    return ko_nn_score_split_acc(state_dev, split_dev, pos_dev, B, n, 1.f, 0, y_dev, hip_stream);
}

int ko_nn_beam_expand(const uint8_t *prefix_dev, int32_t W, int32_t d, int32_t n, uint8_t *pos_dev,
                      int32_t *cand_dev, void *hip_stream)
{
    if (n < 1 || n > KO_NN_MAX_TOKENS || d < 0 || d >= n || W < 1 || (int64_t)W * (n - d) > INT32_MAX)
        return fail(KO_EINVAL, "need 1 <= n <= %d, 0 <= d < n, W >= 1 and W * (n - d) < 2^31", KO_NN_MAX_TOKENS);
    if ((d > 0 && !prefix_dev) || !pos_dev || !cand_dev)
        return fail(KO_EINVAL, "prefixes (when d > 0), positions and candidates must not be NULL");
    const int64_t count = (int64_t)W * (n - d);
    hipLaunchKernelGGL(beam_expand_kernel, dim3(grid1(count)), dim3(256), 0, (hipStream_t)hip_stream, prefix_dev,
                       W, d, n, pos_dev, cand_dev);
    NN_LAUNCHED();
    return KO_OK;
}

int ko_nn_beam_cap(float *score_dev, int32_t W, int32_t m, int32_t cap, float temperature, uint64_t seed,
                   void *hip_stream)
{
    if (!score_dev || W < 1 || m < 1 || m > KO_NN_MAX_TOKENS || cap < 0 || !(temperature >= 0.f))
        return fail(KO_EINVAL, "need scores, W >= 1, 1 <= m <= %d, cap >= 0, temperature >= 0", KO_NN_MAX_TOKENS);
    hipLaunchKernelGGL(beam_cap_kernel, dim3(grid1(W)), dim3(256), 0, (hipStream_t)hip_stream, score_dev, W, m,
                       cap, temperature, seed);
    NN_LAUNCHED();
    return KO_OK;
}

int ko_nn_beam_gather(const uint8_t *prefix_dev, int32_t d, const int32_t *cand_dev, const int64_t *idx_dev,
                      int32_t keep, uint8_t *out_dev, void *hip_stream)
{
    if (d < 0 || d >= KO_NN_MAX_TOKENS || keep < 1 || (d > 0 && !prefix_dev) || !cand_dev || !idx_dev || !out_dev)
        return fail(KO_EINVAL, "need 0 <= d < %d, keep >= 1 and non-NULL buffers", KO_NN_MAX_TOKENS);
    hipLaunchKernelGGL(beam_gather_kernel, dim3(grid1(keep)), dim3(256), 0, (hipStream_t)hip_stream, prefix_dev, d,
                       cand_dev, idx_dev, keep, out_dev);
    NN_LAUNCHED();
    return KO_OK;
}

const char *ko_nn_last_error(void) { return g_err.c_str(); }

}  // extern "C"
