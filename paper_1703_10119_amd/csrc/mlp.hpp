// mlp.hpp -- kernels of the surface-flux surrogate: BF16 MFMA GEMMs with
// FP32 accumulation and fused epilogues, reductions, loss, AdamW and the
// feature builder (gfx950).
//
// The network maps a 48 h outdoor history and wall parameters to the next
// 10-min mean interior surface fluxes; it is not part of the paper.  All
// matrices are row-major; BF16 values are stored as uint16 (round to nearest
// even from FP32).
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dfhm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// FP32 -> BF16, round to nearest even (gfx950 converts in hardware:
// v_cvt_pk_bf16_f32, two values per instruction)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint32_t f2bf2(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// GELU z Phi(z), Phi the standard normal CDF, with Phi(-|z|) = erfc(|z|/sqrt 2) / 2
// from the rational-exponential approximation of Abramowitz & Stegun 7.1.26
// (Hastings): erfc(x) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2),
// t = 1 / (1 + p x), x >= 0, absolute error below 1.5e-7.  So the GELU
// error is below 7.5e-8 |z| plus FP32 rounding, at one reciprocal and one
// base-2 exponential (the library erff costs about three times as many
// instructions in the GEMM epilogues).
__device__ __forceinline__ float gelu(float z)
{
    // with w = z / 2: z Phi(z) = w + |z| (1/2 - Phi(-|z|)) for either sign,
    // and t = 1 / (1 + p |z| / sqrt 2) = 1 / (1 + 2 p |w| / sqrt 2)
    const float w = 0.5f * z;
    const float t = __builtin_amdgcn_rcpf(fmaf(2.0f * (0.3275911f * 0.70710678f), fabsf(w), 1.0f));
    // Phi(-|z|) = p e: the coefficients are a_i / 2, and exp(-z^2 / 2) = 2^(-2 w^2 / ln 2)
    const float p = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 0.5307027145f, -0.7265760135f), 0.7107068705f),
                                     -0.142248368f), 0.127414796f);
    const float e = __builtin_amdgcn_exp2f((-4.0f * 0.72134752f * w) * w);
    return fmaf(fabsf(z), fmaf(-p, e, 0.5f), w);
}
// The same GELU on four values, written step by step across them so that
// four independent chains interleave (same operations per value, so the
// results equal gelu()'s bit for bit).
__device__ __forceinline__ f32x4 gelu4(f32x4 z)
{
    f32x4 w, t, p, e, r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        w[q] = 0.5f * z[q];
        t[q] = fmaf(2.0f * (0.3275911f * 0.70710678f), fabsf(w[q]), 1.0f);
        e[q] = (-4.0f * 0.72134752f * w[q]) * w[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        t[q] = __builtin_amdgcn_rcpf(t[q]);
        e[q] = __builtin_amdgcn_exp2f(e[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = fmaf(t[q], 0.5307027145f, -0.7265760135f);
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = fmaf(t[q], p[q], 0.7107068705f);
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = fmaf(t[q], p[q], -0.142248368f);
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = fmaf(t[q], p[q], 0.127414796f);
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = fmaf(fabsf(z[q]), fmaf(-(t[q] * p[q]), e[q], 0.5f), w[q]);
    return r;
}
// Its derivative (erf form, library erff).
__device__ __forceinline__ float gelu_d(float z)
{
    const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * __expf(-0.5f * z * z);
    return cdf + z * pdf;
}

// Operand layouts.  For C[m][n] = sum_k A(m,k) B(k,n):
//   A: OP_K  -> A[m * lda + k] (reduction index contiguous)
//      OP_MN -> A[k * lda + m]
//   B: OP_K  -> B[n * ldb + k]
//      OP_MN -> B[k * ldb + n]
enum { OP_K = 0, OP_MN = 1 };
// Epilogues.
enum {
    EPI_F32 = 0,        // Cf[z][m][n] = acc (split-K partials when gridDim.z > 1)
    EPI_BIAS_F32 = 1,   // Cf[m][n] = bias[n] + acc (the sum starts at the bias)
    EPI_BIAS_GELU = 2,  // z = bias[n] + acc: Cb[m][n] = bf16(gelu(z)) and, when pre
                        // is not null, pre[m][n] = bf16(z) (kept for the backward pass)
    EPI_GELU_BWD = 3    // Cb[m][n] = bf16(acc * gelu'(aux[m][n]))
};

constexpr int GB_M = 128, GB_N = 128, GB_K = 32, G_PAD = 8;

// A 128 x 32 operand tile moves global -> registers (fetch) -> LDS (put),
// stored in LDS as [row][k] (k contiguous).  rows = M or N index, K multiple
// of 8, rows multiple of 8 (zero outside).  Each of the 256 lanes holds 32 B.
struct TileRegs { uint4 v[2]; };

template <int LAYOUT>
__device__ __forceinline__ TileRegs fetch_tile(const uint16_t *__restrict__ g, int ld, int row0,
                                               int nrows, int k0, int kend, int tid)
{
    TileRegs r;
    if (LAYOUT == OP_K) {
        const int rr = tid >> 1;                 // 128 rows, 2 lanes per row
        const int kk = (tid & 1) * 16;
        const int gr = row0 + rr;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int gk = k0 + kk + 8 * h;
            r.v[h] = make_uint4(0, 0, 0, 0);
            if (gr < nrows && gk < kend) r.v[h] = *(const uint4 *)(g + (int64_t)gr * ld + gk);
        }
    } else {
        const int kk = tid >> 3;                 // 32 k, 8 lanes per k
        const int rb = (tid & 7) * 16;
        const int gk = k0 + kk;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int gr = row0 + rb + 8 * h;
            r.v[h] = make_uint4(0, 0, 0, 0);
            if (gr < nrows && gk < kend) r.v[h] = *(const uint4 *)(g + (int64_t)gk * ld + gr);
        }
    }
    return r;
}

template <int LAYOUT>
__device__ __forceinline__ void put_tile(uint16_t (*s)[GB_K + G_PAD], const TileRegs &r, int tid)
{
    if (LAYOUT == OP_K) {
        const int rr = tid >> 1;
        const int kk = (tid & 1) * 16;
        *(uint4 *)&s[rr][kk] = r.v[0];
        *(uint4 *)&s[rr][kk + 8] = r.v[1];
    } else {
        const int kk = tid >> 3;
        const int rb = (tid & 7) * 16;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint16_t *e = (const uint16_t *)&r.v[h];
#pragma unroll
            for (int q = 0; q < 8; ++q) s[rb + 8 * h + q][kk] = e[q];
        }
    }
}

// One 128 x 128 output tile per workgroup of 256 lanes (2 x 2 waves of
// 64 x 64, each a 4 x 4 grid of 16 x 16 MFMA tiles, K step 32).  The K loop
// is software-pipelined: the next K tile is fetched into registers while the
// MFMAs consume the current one from LDS, and LDS is double-buffered, so a
// K step needs one barrier.  Split-K: blockIdx.z covers K range
// [z * kchunk, (z+1) * kchunk).
template <int LA, int LB, int EPI>
__global__ void __launch_bounds__(256)
k_gemm_bf16(int M, int N, int K, const uint16_t *__restrict__ A, int lda,
            const uint16_t *__restrict__ B, int ldb, float *__restrict__ Cf,
            uint16_t *__restrict__ Cb, int ldc, const float *__restrict__ bias,
            const uint16_t *__restrict__ aux, uint16_t *__restrict__ pre, int kchunk)
{
    __shared__ __align__(16) uint16_t sA[2][GB_M][GB_K + G_PAD];
    __shared__ __align__(16) uint16_t sB[2][GB_N][GB_K + G_PAD];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * GB_M, n0 = blockIdx.x * GB_N;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);

    const int fr = lane & 15;          // row (A) / column (B) inside a 16 x 16 tile
    const int fk = (lane >> 4) * 8;    // this lane's 8 reduction indices

    // the bias epilogues start the sums at the bias (the fused inference
    // kernel does the same, so both round alike)
    f32x4 acc[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = n0 + wn * 64 + j * 16 + fr;
        const float b0 = ((EPI == EPI_BIAS_F32 || EPI == EPI_BIAS_GELU) && col < N) ? bias[col] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][j] = (f32x4){b0, b0, b0, b0};
    }
    if (kbeg < kend) {
        TileRegs ra = fetch_tile<LA>(A, lda, m0, M, kbeg, kend, tid);
        TileRegs rb = fetch_tile<LB>(B, ldb, n0, N, kbeg, kend, tid);
        put_tile<LA>(sA[0], ra, tid);
        put_tile<LB>(sB[0], rb, tid);
        __syncthreads();
        int buf = 0;
        for (int k0 = kbeg; k0 < kend; k0 += GB_K) {
            const bool more = k0 + GB_K < kend;
            if (more) {
                ra = fetch_tile<LA>(A, lda, m0, M, k0 + GB_K, kend, tid);
                rb = fetch_tile<LB>(B, ldb, n0, N, k0 + GB_K, kend, tid);
            }
            bf16x8 af[4], bfr[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = *(const bf16x8 *)&sA[buf][wm * 64 + i * 16 + fr][fk];
#pragma unroll
            for (int j = 0; j < 4; ++j) bfr[j] = *(const bf16x8 *)&sB[buf][wn * 64 + j * 16 + fr][fk];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
            if (more) {
                // the other buffer was last read before the previous barrier
                put_tile<LA>(sA[buf ^ 1], ra, tid);
                put_tile<LB>(sB[buf ^ 1], rb, tid);
            }
            __syncthreads();
            buf ^= 1;
        }
    }
    // accumulator layout: lane holds rows 4*(lane/16)+r, column lane%16
    const int rbase = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 64 + i * 16 + rbase + r;
                const int col = n0 + wn * 64 + j * 16 + fr;
                if (row >= M || col >= N) continue;
                const float v = acc[i][j][r];
                const int64_t o = (int64_t)row * ldc + col;
                if (EPI == EPI_F32) {
                    Cf[(int64_t)blockIdx.z * M * ldc + o] = v;
                } else if (EPI == EPI_BIAS_F32) {
                    Cf[o] = v;
                } else if (EPI == EPI_BIAS_GELU) {
                    const float z = v;
                    if (pre) pre[(int64_t)row * N + col] = f2bf(z);
                    Cb[o] = f2bf(gelu(z));   // the fused inference kernel's arithmetic
                } else {
                    Cb[o] = f2bf(v * gelu_d(bf2f(aux[o])));
                }
            }
}

// ---------------------------------------------------------------- inference
// Weights in MFMA fragment order, for the inference kernel: a layer W[N][K]
// (N a multiple of 16) becomes tiles of 16 outputs x 32 inputs, each 1 KB
// in the order the 64 lanes of a wave read it as the A operand of
// v_mfma_f32_16x16x32_bf16 -- lane l takes outputs n = 16 nt + (l & 15) and
// inputs 32 ks + 8 (l >> 4) .. +7 -- so that a wave loads a fragment as one
// contiguous, fully used kilobyte:
//   ws[((nt KS + ks) 64 + l) 8 + e] = bf16(W[16 nt + (l & 15)][32 ks + 8 (l >> 4) + e]),
// KS = ceil(K / 32), zero for inputs at or beyond K and outputs at or
// beyond N (the copy holds ceil(N / 16) tiles).
__global__ void k_pack_swizzled(const float *__restrict__ w, uint16_t *__restrict__ ws, int N, int K)
{
    const int KS = (K + 31) / 32, NT = (N + 15) / 16;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)NT * KS * 512) return;
    const int e = (int)(i & 7), l = (int)((i >> 3) & 63);
    const int64_t t = i >> 9;
    const int ks = (int)(t % KS), nt = (int)(t / KS);
    const int n = nt * 16 + (l & 15), k = ks * 32 + (l >> 4) * 8 + e;
    ws[i] = (k < K && n < N) ? f2bf(w[(int64_t)n * K + k]) : (uint16_t)0;
}

// The whole forward pass of a block of 128 samples in one workgroup of 8
// waves: the hidden activations stay in LDS from layer to layer (BF16,
// [128][width + FI_PAD]), the weights stream from L2 into registers as MFMA
// operands (fragment order, above), and only the input rows and the output
// layer touch memory.  Each layer computes out^T = W act^T, so that a lane's
// four accumulators are four consecutive outputs of one sample (one 8-byte
// LDS store of BF16 GELU values, or one 16-byte store of FP32 outputs).
// Wave w owns output columns [16 NJ w, 16 NJ (w+1)) of every hidden layer
// (width = 128 NJ) for all 128 samples, and samples [16 w, 16 w + 16) of
// the output layer.  The arithmetic per element is that of the
// layer-by-layer path (k_gemm_bf16): the sum starts at the bias, FP32 MFMA
// accumulation over K in steps of 32 in ascending order, GELU, BF16
// rounding -- so the two paths agree bit for bit.
constexpr int FI_M = 128, FI_NW = 8, FI_PAD = 8, FI_KC = 64;
constexpr int FI_PF = 2;   // weight ring depth (K steps read ahead); divides 4 = K steps per 128 of width

// Layer operands by base and stride (no per-layer pointer table, which the
// kernel would have to copy to scratch memory to index), weights in
// fragment order: layer 0 W0 (K = n_in), b0; hidden layer l = 1 .. depth-1
// at Wh + (l-1) wh_stride, bh + (l-1) bh_stride; the output layer Wo
// (n_outp outputs), bo.
struct FusedNet {
    const uint16_t *W0, *Wh, *Wo;
    const float *b0, *bh, *bo;
    int64_t wh_stride, bh_stride;
    int depth;       // hidden layers
    int n_in;        // inputs (multiple of 8), x row stride ldx >= n_in
    int n_outp;      // output columns written (multiple of 16, <= 32)
};

template <int NJ>
__host__ __device__ constexpr size_t fused_lds_bytes()
{
    const size_t act = (size_t)FI_M * (128 * NJ + FI_PAD) * 2;
    const size_t stage = 2 * (size_t)FI_M * (FI_KC + FI_PAD) * 2;
    return act > stage ? act : stage;
}

template <int NJ>
__global__ void __launch_bounds__(64 * FI_NW) __attribute__((amdgpu_waves_per_eu(2)))
k_mlp_infer_fused(FusedNet net, const uint16_t *__restrict__ x, int ldx, int64_t batch,
                  float *__restrict__ y, int ldy)
{
    extern __shared__ __align__(16) uint16_t lds_act[];
    constexpr int W = 128 * NJ;                    // width
    constexpr int KSW = W / 32;                    // K steps of a hidden layer
    constexpr int LDA = W + FI_PAD;
    constexpr int LDS_ = FI_KC + FI_PAD;           // staging row stride
    constexpr int NT = 64 * FI_NW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * FI_M;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    const int nw0 = wave * NJ * 16;                // first output column of this wave
    const int nl = (lane >> 4) * 4;                // lane's first column in a 16-column tile
    const uint4 z4 = make_uint4(0, 0, 0, 0);

    f32x4 acc[8][NJ];
    // sums start at the bias of the lane's four columns
    auto init = [&](const float *__restrict__ bias) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const float4 bb = *(const float4 *)(bias + nw0 + j * 16 + nl);
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i][j] = (f32x4){bb.x, bb.y, bb.z, bb.w};
        }
    };
    // fragment (wave's column tile j, K step ks) of a layer with KS K steps
    auto wfrag = [&](const uint16_t *__restrict__ Wl, int KS, int j, int ks) {
        return __builtin_bit_cast(
            bf16x8, *(const uint4 *)(Wl + (((size_t)(nw0 / 16 + j) * KS + ks) * 64 + lane) * 8));
    };
    // GELU and BF16 of the accumulators into the activation block
    auto hidden_out = [&]() {
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const f32x4 g = gelu4(acc[i][j]);
                uint2 v;
                v.x = f2bf2(g[0], g[1]);
                v.y = f2bf2(g[2], g[3]);
                *(uint2 *)&lds_act[(i * 16 + fr) * LDA + nw0 + j * 16 + nl] = v;
            }
    };

    // ---- layer 0: input rows from x, staged through LDS in chunks of FI_KC
    // (128 rows x 8 pieces of 16 B per chunk, two per lane)
    {
        const int K = net.n_in, KS = (K + 31) / 32;
        const uint16_t *__restrict__ Wl = net.W0;
        uint16_t *stage = lds_act;
        auto fetch = [&](int k0, uint4 (&r)[2]) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int pc = tid + q * NT, row = pc >> 3, kc = (pc & 7) * 8;
                const int64_t g = m0 + row;
                r[q] = z4;
                if (g < batch && k0 + kc < K) r[q] = *(const uint4 *)(x + g * ldx + k0 + kc);
            }
        };
        auto put = [&](int buf, const uint4 (&r)[2]) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int pc = tid + q * NT, row = pc >> 3, kc = (pc & 7) * 8;
                *(uint4 *)(stage + (size_t)buf * FI_M * LDS_ + row * LDS_ + kc) = r[q];
            }
        };
        init(net.b0);
        uint4 rg[2];
        fetch(0, rg);
        put(0, rg);
        __syncthreads();
        int buf = 0;
        for (int k0 = 0; k0 < K; k0 += FI_KC) {
            const bool more = k0 + FI_KC < K;
            if (more) fetch(k0 + FI_KC, rg);
#pragma unroll
            for (int kk = 0; kk < FI_KC; kk += 32) {
                const int ks = (k0 + kk) / 32;
                if (ks < KS) {
                    bf16x8 wf[NJ];
#pragma unroll
                    for (int j = 0; j < NJ; ++j) wf[j] = wfrag(Wl, KS, j, ks);
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const bf16x8 af = *(const bf16x8 *)(stage + (size_t)buf * FI_M * LDS_ +
                                                            (i * 16 + fr) * LDS_ + kk + fk);
#pragma unroll
                        for (int j = 0; j < NJ; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[j], af, acc[i][j], 0, 0, 0);
                    }
                }
            }
            if (more) put(buf ^ 1, rg);   // last read before the previous barrier
            __syncthreads();
            buf ^= 1;
        }
        hidden_out();
        __syncthreads();
    }
    // ---- hidden layers 1 .. depth-1: B operand from the activation block
    for (int l = 1; l < net.depth; ++l) {
        const uint16_t *__restrict__ Wl = net.Wh + (l - 1) * net.wh_stride;
        init(net.bh + (l - 1) * net.bh_stride);
        // the weights of K steps ks .. ks + FI_PF - 1 in a ring of FI_PF
        // slots: step ks reads slot ks % FI_PF (a compile-time index in the
        // unrolled block) and refills it with step ks + FI_PF (clamped), so
        // the wait for a fragment covers only reads issued FI_PF steps before
        bf16x8 wr[FI_PF][NJ];
#pragma unroll
        for (int p = 0; p < FI_PF; ++p)
#pragma unroll
            for (int j = 0; j < NJ; ++j) wr[p][j] = wfrag(Wl, KSW, j, p);
        for (int ks0 = 0; ks0 < KSW; ks0 += FI_PF) {
#pragma unroll
            for (int p = 0; p < FI_PF; ++p) {
                const int ks = ks0 + p;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const bf16x8 af = *(const bf16x8 *)(lds_act + (i * 16 + fr) * LDA + ks * 32 + fk);
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[p][j], af, acc[i][j], 0, 0, 0);
                }
                const int kn = min(ks + FI_PF, KSW - 1);
#pragma unroll
                for (int j = 0; j < NJ; ++j) wr[p][j] = wfrag(Wl, KSW, j, kn);
                // keep the next step's LDS reads below this step's MFMAs (hoisted,
                // they took the registers of a deeper schedule and spilled)
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();          // every wave has read the layer's input
        hidden_out();
        __syncthreads();
    }
    // ---- output layer: wave w takes samples [16 w, 16 w + 16), all outputs
    {
        const int no = net.n_outp >> 4;
        f32x4 o[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const float4 bb = j < no ? *(const float4 *)(net.bo + j * 16 + nl) : make_float4(0.f, 0.f, 0.f, 0.f);
            o[j] = (f32x4){bb.x, bb.y, bb.z, bb.w};
        }
        // the same weight ring as the hidden layers, for one or two tiles
        auto out_tiles = [&](auto no_c) {
            constexpr int NO = decltype(no_c)::value;
            auto ofrag = [&](int j, int ks) {
                return __builtin_bit_cast(bf16x8, *(const uint4 *)(net.Wo + (((size_t)j * KSW + ks) * 64 + lane) * 8));
            };
            bf16x8 wr[FI_PF][NO];
#pragma unroll
            for (int p = 0; p < FI_PF; ++p)
#pragma unroll
                for (int j = 0; j < NO; ++j) wr[p][j] = ofrag(j, p);
            for (int ks0 = 0; ks0 < KSW; ks0 += FI_PF) {
#pragma unroll
                for (int p = 0; p < FI_PF; ++p) {
                    const int ks = ks0 + p;
                    const bf16x8 af = *(const bf16x8 *)(lds_act + (wave * 16 + fr) * LDA + ks * 32 + fk);
#pragma unroll
                    for (int j = 0; j < NO; ++j) o[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[p][j], af, o[j], 0, 0, 0);
                    const int kn = min(ks + FI_PF, KSW - 1);
#pragma unroll
                    for (int j = 0; j < NO; ++j) wr[p][j] = ofrag(j, kn);
                }
            }
        };
        if (no == 2) out_tiles(std::integral_constant<int, 2>{});
        else out_tiles(std::integral_constant<int, 1>{});
        const int64_t row = m0 + wave * 16 + fr;
        if (row < batch) {
#pragma unroll
            for (int j = 0; j < 2; ++j)
                if (j < no) *(float4 *)(y + row * ldy + j * 16 + nl) = make_float4(o[j][0], o[j][1], o[j][2], o[j][3]);
        }
    }
}

// Sum of split-K partials: out[i] = sum_z part[z][i] (+ out[i] if accumulate).
__global__ void k_sum_partials(const float *__restrict__ part, int nsplit, int64_t n, float *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * n + i];
    out[i] = s;
}

// Column sums of a BF16 matrix [rows][cols] (cols a multiple of 8) into FP32
// partials part[blockIdx.y][col] over the row range [blockIdx.y * rchunk,
// + rchunk): 256 lanes, lane (g, c) sums columns 8 c .. 8 c + 7 of block
// column group blockIdx.x over the rows g, g + 4, ... of the range with one
// 16-byte read per row, and the four row groups meet in LDS.
__global__ void __launch_bounds__(256) k_colsum_bf16(const uint16_t *__restrict__ x, int rows, int cols,
                                                     int rchunk, float *__restrict__ part)
{
    __shared__ float red[4][64][9];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int col0 = (blockIdx.x * 64 + c) * 8;
    const int r0 = blockIdx.y * rchunk, r1 = min(rows, r0 + rchunk);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (col0 < cols) {
        for (int r = r0 + g; r < r1; r += 4) {
            const uint4 v = *(const uint4 *)(x + (int64_t)r * cols + col0);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                s[2 * h] += __uint_as_float(w[h] << 16);
                s[2 * h + 1] += __uint_as_float(w[h] & 0xffff0000u);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[g][c][e] = s[e];
    __syncthreads();
    if (g == 0 && col0 < cols) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
            part[(int64_t)blockIdx.y * cols + col0 + e] =
                (red[0][c][e] + red[1][c][e]) + (red[2][c][e] + red[3][c][e]);
    }
}

// Loss of a head with F = n_out / 2 targets: outputs z[b][0..F) are the
// means, z[b][F..2F) the log variances, targets y[b][0..F) (normalised).
// Mean squared error on the means plus a Gaussian log-likelihood term for
// the log variances with the residual held fixed:
//   L = (1/B) sum_b sum_f [ r^2 + sg(r^2) exp(-s) + s ],  r = y - mu.
// Writes dZ[b][0..ldz) as BF16 (zeros beyond the 2F outputs) and per-block
// partial losses.
__global__ void k_loss(const float *__restrict__ z, int ldz, const float *__restrict__ y, int B,
                       int F, uint16_t *__restrict__ dz, float *__restrict__ part)
{
    __shared__ float red[256];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (b < B) {
        const float invB = 1.0f / (float)B;
        for (int f = 0; f < F; ++f) {
            const float mu = z[(int64_t)b * ldz + f];
            const float s = z[(int64_t)b * ldz + F + f];
            const float r = y[(int64_t)F * b + f] - mu;
            const float e = __expf(-s);
            l += r * r + r * r * e + s;
            dz[(int64_t)b * ldz + f] = f2bf(-2.0f * r * invB);
            dz[(int64_t)b * ldz + F + f] = f2bf((1.0f - r * r * e) * invB);
        }
        for (int f = 2 * F; f < ldz; ++f) dz[(int64_t)b * ldz + f] = 0;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Zero columns [c0, c1) of a BF16 matrix [rows][ld].
__global__ void k_zero_cols(uint16_t *__restrict__ x, int rows, int ld, int c0, int c1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int w = c1 - c0;
    if (i >= (int64_t)rows * w) return;
    x[(i / w) * ld + c0 + i % w] = 0;
}

// AdamW on FP32 master weights (the BF16 copies are packed afterwards).
// mask[i] = 0 keeps a padding weight at zero.
__global__ void k_adamw(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                        const float *__restrict__ g, const uint8_t *__restrict__ mask, int64_t n,
                        float lr, float b1, float b2, float eps, float wd, float c1, float c2)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mask && !mask[i]) { w[i] = 0.f; return; }
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi * c1, vh = vi * c2;     // bias corrections 1/(1 - b^t)
    float wi = w[i];
    wi -= lr * (mh / (sqrtf(vh) + eps) + wd * wi);
    w[i] = wi;
}

// BF16 copy of a weight matrix w[N][K] (FP32) as wb[N][ld].
__global__ void k_pack_weights(const float *__restrict__ w, uint16_t *__restrict__ wb, int N, int K,
                               int ld)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * K) return;
    const int64_t n = i / K, k = i % K;
    wb[n * ld + k] = f2bf(w[i]);
}

// Features of one sample: the outdoor temperature and humidity of side 0
// sampled every `dt_hist` seconds over the n_hist samples ending at time t
// (oldest first), z-scored, then 8 parameters, z-scored -- 5 per wall
// (params[w][0..4]) and 3 of the time (t / 1 day, sin and cos of the time of
// day) -- then zeros up to the row stride.  Inputs per sample: wall, time.
struct FeatDesc {
    int n_hist, stride;
    float dt_hist, T_mean, T_scale, RH_mean, RH_scale;
    float p_mean[8], p_scale[8];
};

__global__ void k_features(const int32_t *__restrict__ wall_of, const double *__restrict__ t_of,
                           const double *__restrict__ sines /* [W][8]: T mean, amp, period, phase, RH ... */,
                           const float *__restrict__ params /* [W][5] */, int nsamp, FeatDesc fd,
                           uint16_t *__restrict__ x)
{
    const int s = blockIdx.x;
    if (s >= nsamp) return;
    const int w = wall_of[s];
    const double t = t_of[s];
    const double *S = sines + (int64_t)w * 8;
    uint16_t *row = x + (int64_t)s * fd.stride;
    for (int i = threadIdx.x; i < fd.stride; i += blockDim.x) {
        float v = 0.f;
        if (i < 2 * fd.n_hist) {
            const int h = i < fd.n_hist ? i : i - fd.n_hist;
            const double *q = i < fd.n_hist ? S : S + 4;
            const double ts = t - (double)(fd.n_hist - 1 - h) * (double)fd.dt_hist;
            double ph = fmod(2.0 * 3.14159265358979323846 * ts / q[2] + q[3], 2.0 * 3.14159265358979323846);
            const float val = (float)(q[0] + q[1] * sin(ph));
            v = i < fd.n_hist ? (val - fd.T_mean) / fd.T_scale : (val - fd.RH_mean) / fd.RH_scale;
        } else if (i < 2 * fd.n_hist + 8) {
            const int p = i - 2 * fd.n_hist;
            float raw;
            if (p < 5) raw = params[(int64_t)w * 5 + p];
            else if (p == 5) raw = (float)(t / 86400.0);
            else {
                const double ph = 2.0 * 3.14159265358979323846 * fmod(t, 86400.0) / 86400.0;
                raw = (float)(p == 6 ? sin(ph) : cos(ph));
            }
            v = (raw - fd.p_mean[p]) / fd.p_scale[p];
        }
        row[i] = f2bf(v);
    }
}

// Decode the flux head.  Per field f (heat, vapour) the network predicts
// the flux relative to the wall's RMS flux, u_f, and the log of that RMS,
// l_f, each normalised (value = mean + std * output); outputs
// y[b] = (u_q, u_g, l_q, l_g, s_uq, s_ug, s_lq, s_lg), s = log variance.
// flux_f = u_f exp(l_f).  The predicted error relative to the RMS flux is
// e_f = sd(u_f) + |u_f| sd(l_f) to first order, sd = std * exp(s / 2);
// fallback when the estimate exceeds tau for either field.  scale[8] =
// (mean, std) of u_q, u_g, l_q, l_g.  With several networks (an ensemble
// trained on the same targets) flux_f is the members' mean, and the estimate
// adds their disagreement to their mean predicted error in quadrature:
// sqrt(E_f^2 + D_f^2), E_f = mean_k e_fk,
// D_f = (population) std_k of flux_fk over exp(mean_k l_fk), the members'
// spread relative to their mean predicted RMS; one network gives e_f itself.
// Outputs (each optional): flux[b][2], err[b] = max_f estimate, fallback[b].
// A member's outputs of sample b start at y[k] + ld * b.
struct DecodeScale { float m[4], s[4]; };
constexpr int kMaxEnsemble = 4;
struct DecodeNets {
    const float *y[kMaxEnsemble];
    int n, ld;
};

__global__ void k_decode(DecodeNets nets, int64_t batch, DecodeScale sc, float tau,
                         float *__restrict__ flux, float *__restrict__ err,
                         uint8_t *__restrict__ fallback)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const float inv = 1.0f / (float)nets.n;
    float emax = 0.f;
    bool fb = false;
    for (int f = 0; f < 2; ++f) {
        float fk[kMaxEnsemble];
        float fl = 0.f, e = 0.f, lm = 0.f;
#pragma unroll
        for (int k = 0; k < kMaxEnsemble; ++k) {
            fk[k] = 0.f;
            if (k < nets.n) {
                const float *o = nets.y[k] + (int64_t)nets.ld * b;
                const float u = o[f] * sc.s[f] + sc.m[f];
                const float lg = o[2 + f] * sc.s[2 + f] + sc.m[2 + f];
                fk[k] = u * __expf(lg);
                fl += fk[k];
                lm += lg;
                e += sc.s[f] * __expf(0.5f * o[4 + f]) + fabsf(u) * sc.s[2 + f] * __expf(0.5f * o[6 + f]);
            }
        }
        fl *= inv;
        if (flux) flux[2 * b + f] = fl;
        e *= inv;
        if (nets.n > 1) {
            float v = 0.f;
#pragma unroll
            for (int k = 0; k < kMaxEnsemble; ++k)
                if (k < nets.n) v += (fk[k] - fl) * (fk[k] - fl);
            const float d = sqrtf(v * inv) * __expf(-lm * inv);
            e = sqrtf(e * e + d * d);
        }
        fb = fb || !(e <= tau);
        emax = (f == 0 || !(e <= emax)) ? e : emax;   // a NaN estimate propagates
    }
    if (err) err[b] = emax;
    if (fallback) fallback[b] = (uint8_t)fb;
}

} // namespace dfhm
