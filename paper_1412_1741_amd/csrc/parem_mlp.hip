// Learned speculation proposal: a small MLP that scores the DFA states at a
// chunk boundary from the 32 bytes before it (not part of the paper; it
// replaces the full speculated set R_c by its m best-scored members, and the
// verify-and-re-run step keeps the match exact).
//
//   x  = concat(emb[w_0..w_31])          512   (a pad byte embeds as 0)
//   h1 = gelu(W1 x + b1)                  256
//   h2 = gelu(W2 h1 + b2)                 256
//   z  = W3 h2 + b3                       one logit per state (S = Q rows)
//   loss = masked softmax cross-entropy over the states of R_c
//
// Dense layers run on MFMA: bf16 operands, fp32 accumulation, fp32 master
// weights updated by AdamW, a bf16 copy feeding the next forward pass. The
// forward layers (training and inference alike) use v_mfma_f32_32x32x16_bf16,
// which on gfx950 does twice the work of the 32x32x8 form in about the same
// time; both forward paths sum k in the same order, so they give the same
// logits. The backward GEMMs use the 32x32x8 form. GELU is the erf form.
#include "parem_internal.h"

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

namespace parem {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// bf16 conversions: v_cvt_pk_bf16_f32, round to nearest even
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi) {
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ uint16_t f2bf(float f) { return (uint16_t)f2bf2(f, 0.0f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// erf by the rational approximation of Abramowitz & Stegun 7.1.26 (after
// Hastings): |error| <= 1.5e-7 in exact arithmetic, under 5e-7 in fp32 with
// the hardware reciprocal and exp2. That is far below the bf16 rounding the
// hidden activations receive, and it has no branches (the library erff
// evaluates two polynomial branches under divergence).
__device__ __forceinline__ float erf_fast(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float p = fmaf(1.061405429f, t, -1.453152027f);
    p = fmaf(p, t, 1.421413741f);
    p = fmaf(p, t, -0.284496736f);
    p = fmaf(p, t, 0.254829592f);
    p *= t;
    const float e = __builtin_amdgcn_exp2f(-(ax * ax) * 1.44269504088896341f);  // exp(-x^2)
    return copysignf(fmaf(-p, e, 1.0f), x);
}
// gelu(u) = u Phi(u) = max(u, 0) - |u| Phi(-|u|), with Phi(-|u|) = erfc(|u| / sqrt 2) / 2
// from the same approximation (erfc(x) = t P(t) exp(-x^2), t = 1 / (1 + p x))
__device__ __forceinline__ float gelu(float u) {
    const float au = fabsf(u);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, au, 1.0f));
    float p = fmaf(0.5f * 1.061405429f, t, 0.5f * -1.453152027f);
    p = fmaf(p, t, 0.5f * 1.421413741f);
    p = fmaf(p, t, 0.5f * -0.284496736f);
    p = fmaf(p, t, 0.5f * 0.254829592f);
    p *= t;
    const float q = p * __builtin_amdgcn_exp2f((u * u) * (-0.5f * 1.44269504088896341f));
    return fmaf(-au, q, fmaxf(u, 0.0f));
}
__device__ __forceinline__ float gelu_grad(float u) {
    return 0.5f * (1.0f + erf_fast(u * 0.70710678118654752f)) +
           u * 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.5f * u * u * 1.44269504088896341f);
}

// ---------------------------------------------------------------------------
// GEMM: C[M,N] = sum_k A[M,K] B[K,N], bf16 operands, fp32 accumulation.
// A is stored [M][K] (TA = false) or [K][M] (TA = true); B is stored [N][K]
// (TB = true) or [K][N] (TB = false). 64 x 64 output tile per workgroup of
// four waves (each a 32 x 32 MFMA block), K consumed 32 at a time through
// LDS tiles kept k-contiguous for both operands. With split > 0 (EPI_F32
// only), workgroup z takes k in [z split, (z + 1) split) and writes its
// partial sums at out32 + z M ldc; k_splitk_sum adds them in order.
// ---------------------------------------------------------------------------

enum Epi : int {
    EPI_F32 = 0,        // out32[m*ldc+n] = acc
    EPI_BIAS_GELU = 1,  // pre = acc + bias[n]; out32 = pre; out16 = bf16(gelu(pre))
    EPI_BIAS_F32 = 2,   // out32 = acc + bias[n]
    EPI_GELU_BWD = 3,   // d = acc * gelu'(aux32[m*ldc+n]); out32 = d; out16 = bf16(d)
    EPI_BIAS_BF16 = 4   // out16 = bf16(gelu(acc + bias[n])) (inference, no pre-activation kept)
};

constexpr int kGemmT = 256;
constexpr int kKT = 32;
constexpr int kLdsK = kKT + 8;  // padded row (elements) against bank conflicts

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(kGemmT) void k_gemm(const uint16_t *__restrict__ A, int lda,
                                                 const uint16_t *__restrict__ B, int ldb, int M, int N, int K,
                                                 const float *__restrict__ bias, const float *__restrict__ aux,
                                                 float *__restrict__ out32, uint16_t *__restrict__ out16,
                                                 int ldc, int split) {
    __shared__ __align__(16) uint16_t As[64][kLdsK];
    __shared__ __align__(16) uint16_t Bs[64][kLdsK];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    const int kb = split ? (int)blockIdx.z * split : 0;
    const int ke = split ? min(K, kb + split) : K;
    if (split) out32 += (size_t)blockIdx.z * M * ldc;

    for (int k0 = kb; k0 < ke; k0 += kKT) {
        // each thread stages 8 elements of each operand
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + u * kGemmT;  // 0..2047 over a 64 x 32 tile
            int r, kk;
            if (TA) { r = e & 63; kk = e >> 6; }   // consecutive threads walk m (contiguous when TA)
            else { r = e >> 5; kk = e & 31; }      // consecutive threads walk k
            const int gm = m0 + r, gk = k0 + kk;
            uint16_t v = 0;
            if (gm < M && gk < ke) v = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
            As[r][kk] = v;
            int rn, kn;
            if (TB) { rn = e >> 5; kn = e & 31; }  // B stored [N][K]: walk k
            else { rn = e & 63; kn = e >> 6; }     // B stored [K][N]: walk n
            const int gn = n0 + rn, gk2 = k0 + kn;
            uint16_t w = 0;
            if (gn < N && gk2 < ke) w = TB ? B[(size_t)gn * ldb + gk2] : B[(size_t)gk2 * ldb + gn];
            Bs[rn][kn] = w;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kKT; ks += 8) {
            // lane l holds A[m = l % 32][k = 4 (l / 32) + i] and B[k = 4 (l / 32) + i][n = l % 32]
            const int kk = ks + 4 * (lane >> 5);
            const bf16x4 a = *reinterpret_cast<const bf16x4 *>(&As[wm + (lane & 31)][kk]);
            const bf16x4 b = *reinterpret_cast<const bf16x4 *>(&Bs[wn + (lane & 31)][kk]);
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // lane l, register r holds C[m = 8 (r / 4) + 4 (l / 32) + r % 4][n = l % 32]
    const int n = n0 + wn + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (m >= M || n >= N) continue;
        const size_t o = (size_t)m * ldc + n;
        const float v = acc[r];
        if constexpr (EPI == EPI_F32) {
            out32[o] = v;
        } else if constexpr (EPI == EPI_BIAS_GELU) {
            const float pre = v + bias[n];
            out32[o] = pre;
            out16[o] = f2bf(gelu(pre));
        } else if constexpr (EPI == EPI_BIAS_F32) {
            out32[o] = v + bias[n];
        } else if constexpr (EPI == EPI_GELU_BWD) {
            const float d = v * gelu_grad(aux[o]);
            out32[o] = d;
            out16[o] = f2bf(d);
        } else {
            out16[o] = f2bf(gelu(v + bias[n]));
        }
    }
}

// Forward-layer GEMM, both operands K-contiguous: C[M,N] = A[M,K] B[N,K]^T.
// 128 x 128 output tile per workgroup; each wave computes a 64 x 64 block as
// 2 x 2 MFMA 32 x 32 tiles (32x32x16: lane l holds A[m = l % 32][k = 8 (l / 32)
// + i] and B[k = 8 (l / 32) + i][n = l % 32], i < 8). K advances 32 per stage through double-buffered
// LDS tiles filled with 16-byte loads (rows padded to 40 elements). K must be
// a multiple of 32 and lda/ldb multiples of 8.
constexpr int kNtRow = 40;

template <int EPI>
__global__ __launch_bounds__(kGemmT) void k_gemm_nt(const uint16_t *__restrict__ A, int lda,
                                                    const uint16_t *__restrict__ B, int ldb, int M, int N, int K,
                                                    const float *__restrict__ bias, const float *__restrict__ aux,
                                                    float *__restrict__ out32, uint16_t *__restrict__ out16,
                                                    int ldc) {
    __shared__ __align__(16) uint16_t As[2][128][kNtRow];
    __shared__ __align__(16) uint16_t Bs[2][128][kNtRow];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * 128, n0 = blockIdx.x * 128;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    // staging: thread loads rows r and r + 64 (r = tid / 4) at k offset 8 (tid % 4)
    const int lr = tid >> 2, lk = (tid & 3) * 8;
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    auto load = [&](int k0, uint4 (&ra)[2], uint4 (&rb)[2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int gm = m0 + lr + 64 * h, gn = n0 + lr + 64 * h;
            ra[h] = gm < M ? *reinterpret_cast<const uint4 *>(A + (size_t)gm * lda + k0 + lk) : make_uint4(0, 0, 0, 0);
            rb[h] = gn < N ? *reinterpret_cast<const uint4 *>(B + (size_t)gn * ldb + k0 + lk) : make_uint4(0, 0, 0, 0);
        }
    };
    auto store = [&](int buf, const uint4 (&ra)[2], const uint4 (&rb)[2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            *reinterpret_cast<uint4 *>(&As[buf][lr + 64 * h][lk]) = ra[h];
            *reinterpret_cast<uint4 *>(&Bs[buf][lr + 64 * h][lk]) = rb[h];
        }
    };
    uint4 ra[2], rb[2];
    load(0, ra, rb);
    store(0, ra, rb);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += kKT) {
        const bool more = k0 + kKT < K;
        if (more) load(k0 + kKT, ra, rb);
#pragma unroll
        for (int ks = 0; ks < kKT; ks += 16) {
            const int kk = ks + 8 * (lane >> 5);
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *reinterpret_cast<const bf16x8 *>(&As[buf][wm + 32 * i + (lane & 31)][kk]);
                b[i] = *reinterpret_cast<const bf16x8 *>(&Bs[buf][wn + 32 * i + (lane & 31)][kk]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) store(buf ^ 1, ra, rb);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + 32 * j + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (m >= M || n >= N) continue;
                const size_t o = (size_t)m * ldc + n;
                const float v = acc[i][j][r];
                if constexpr (EPI == EPI_F32) {
                    out32[o] = v;
                } else if constexpr (EPI == EPI_BIAS_GELU) {
                    const float pre = v + bias[n];
                    out32[o] = pre;
                    out16[o] = f2bf(gelu(pre));
                } else if constexpr (EPI == EPI_BIAS_F32) {
                    out32[o] = v + bias[n];
                } else if constexpr (EPI == EPI_GELU_BWD) {
                    const float d = v * gelu_grad(aux[o]);
                    out32[o] = d;
                    out16[o] = f2bf(d);
                } else {
                    out16[o] = f2bf(gelu(v + bias[n]));
                }
            }
        }
    }
}

// k-splits of a weight-gradient GEMM (K = batch rows): enough workgroups to
// fill the chip, at least 256 rows of K each
static int splitk_of(int M, int N, int K) {
    const int tiles = ((N + 63) / 64) * ((M + 63) / 64);
    int s = 1;
    while (s < 16 && tiles * s < 256 && K / (2 * s) >= 256) s *= 2;
    return s;
}

__global__ void k_splitk_sum(const float *__restrict__ part, int S, int M, int N, int ldc, float *__restrict__ out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)M * N) return;
    const size_t o = (i / N) * ldc + i % N;
    float v = 0.0f;
    for (int z = 0; z < S; ++z) v += part[(size_t)z * M * ldc + o];
    out[o] = v;
}

template <bool TA, bool TB, int EPI>
static void gemm(hipStream_t s, const uint16_t *A, int lda, const uint16_t *B, int ldb, int M, int N, int K,
                 const float *bias, const float *aux, float *out32, uint16_t *out16, int ldc,
                 float *part = nullptr) {
    if (!TA && TB && K % kKT == 0 && lda % 8 == 0 && ldb % 8 == 0 &&
        (reinterpret_cast<uintptr_t>(A) & 15u) == 0 && (reinterpret_cast<uintptr_t>(B) & 15u) == 0) {
        dim3 grid((N + 127) / 128, (M + 127) / 128);
        hipLaunchKernelGGL((k_gemm_nt<EPI>), grid, dim3(kGemmT), 0, s, A, lda, B, ldb, M, N, K, bias, aux, out32,
                           out16, ldc);
        return;
    }
    const int S = (EPI == EPI_F32 && part) ? splitk_of(M, N, K) : 1;
    if (S > 1) {
        // split-K: partial sums per k range, then their sum in a fixed order
        const int split = (K / S + kKT - 1) / kKT * kKT;
        const int nz = (K + split - 1) / split;
        dim3 grid((N + 63) / 64, (M + 63) / 64, nz);
        hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(kGemmT), 0, s, A, lda, B, ldb, M, N, K, bias, aux, part,
                           out16, ldc, split);
        const size_t n = (size_t)M * N;
        hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, nz, M, N, ldc,
                           out32);
        return;
    }
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(kGemmT), 0, s, A, lda, B, ldb, M, N, K, bias, aux, out32,
                       out16, ldc, 0);
}

// ---------------------------------------------------------------------------
// elementwise / reduction kernels
// ---------------------------------------------------------------------------

// window of the 32 bytes before each position (256 = pad before the text
// start) and the class of the byte just before it. A position beyond the
// text (p > len) reads nothing: its window is all pad and its class
// kRowInvalid, which the loss kernel skips.
constexpr uint16_t kRowInvalid = 0xffffu;

__global__ void k_windows(const uint8_t *__restrict__ text, uint64_t len, const uint64_t *__restrict__ pos,
                          uint32_t B, const uint8_t *__restrict__ cls, uint32_t start_class,
                          uint16_t *__restrict__ win, uint16_t *__restrict__ wcls) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kMlpWindow) return;
    const uint32_t b = i / kMlpWindow, k = i % kMlpWindow;
    const uint64_t p = pos[b];
    if (p > len) {
        win[i] = 256;
        if (k == 0) wcls[b] = kRowInvalid;
        return;
    }
    const int64_t q = (int64_t)p - (int64_t)kMlpWindow + (int64_t)k;
    win[i] = q < 0 ? (uint16_t)256 : (uint16_t)text[q];
    if (k == 0) wcls[b] = p == 0 ? (uint16_t)start_class : (uint16_t)cls[text[p - 1]];
}

// windows of chunk boundaries c * L (c = 0..chunks-1)
__global__ void k_windows_chunks(const uint8_t *__restrict__ text, uint64_t L, uint32_t chunks,
                                 const uint8_t *__restrict__ cls, uint32_t start_class, uint16_t *__restrict__ win,
                                 uint16_t *__restrict__ wcls) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= chunks * kMlpWindow) return;
    const uint32_t b = i / kMlpWindow, k = i % kMlpWindow;
    const uint64_t p = (uint64_t)b * L;
    const int64_t q = (int64_t)p - (int64_t)kMlpWindow + (int64_t)k;
    win[i] = q < 0 ? (uint16_t)256 : (uint16_t)text[q];
    if (k == 0) wcls[b] = p == 0 ? (uint16_t)start_class : (uint16_t)cls[text[p - 1]];
}

__global__ void k_embed(const uint16_t *__restrict__ win, uint32_t B, const uint16_t *__restrict__ emb16,
                        uint16_t *__restrict__ X) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;  // over B * 512
    if (i >= B * kMlpIn) return;
    const uint32_t b = i / kMlpIn, r = i % kMlpIn;
    const uint32_t w = win[b * kMlpWindow + r / kMlpEmb];
    X[i] = w >= 256 ? (uint16_t)0 : emb16[w * kMlpEmb + r % kMlpEmb];
}

// one wave per row: masked softmax cross-entropy; writes dZ = (p - onehot) / B
// (fp32 and bf16) and accumulates the mean loss. A state is allowed when it
// belongs to the speculated list of the row's class (inverse index hit). A
// row whose position lay beyond the text, or whose label is not an allowed
// state (e.g. 0xffffffff, the boundary state after a byte outside the
// alphabet), takes no part: its dZ row is zero and it adds no loss (the mean
// still divides by B).
__global__ __launch_bounds__(256) void k_softmax_ce(const float *__restrict__ Z, uint32_t B, uint32_t S,
                                                    const uint32_t *__restrict__ label,
                                                    const uint16_t *__restrict__ wcls,
                                                    const uint16_t *__restrict__ inv, uint32_t Q1,
                                                    float *__restrict__ dZ32, uint16_t *__restrict__ dZ16,
                                                    float *__restrict__ loss) {
    // one wave per row, rows strided over the grid; the loss is summed per
    // workgroup and added once (same-address atomics serialise)
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float invB = 1.0f / (float)B;
    float part = 0.0f;
    for (uint32_t row = blockIdx.x * 4 + wave; row < B; row += gridDim.x * 4) {
        const float *z = Z + (size_t)row * S;
        const uint32_t lab = label[row];
        const uint16_t rc = wcls[row];
        const uint16_t *iv = inv + (size_t)(rc == kRowInvalid ? 0 : rc) * Q1;
        if (rc == kRowInvalid || lab >= S || iv[lab] == 0xffffu) {
            for (uint32_t s = lane; s < S; s += 64) {
                dZ32[(size_t)row * S + s] = 0.0f;
                dZ16[(size_t)row * S + s] = 0;
            }
            continue;
        }
        float mx = -INFINITY;
        for (uint32_t s = lane; s < S; s += 64)
            if (iv[s] != 0xffffu) mx = fmaxf(mx, z[s]);
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        float sum = 0.0f;
        for (uint32_t s = lane; s < S; s += 64)
            if (iv[s] != 0xffffu) sum += expf(z[s] - mx);
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        for (uint32_t s = lane; s < S; s += 64) {
            float g = 0.0f;
            if (iv[s] != 0xffffu) g = expf(z[s] - mx) / sum;
            if (s == lab) g -= 1.0f;
            g *= invB;
            dZ32[(size_t)row * S + s] = g;
            dZ16[(size_t)row * S + s] = f2bf(g);
        }
        part += (logf(sum) + mx - z[lab]) * invB;
    }
    __shared__ float red[4];
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, red[0] + red[1] + red[2] + red[3]);
}
__global__ void k_colsum(const float *__restrict__ A, uint32_t B, uint32_t N, float *__restrict__ out) {
    const uint32_t n = blockIdx.x;
    float s = 0.0f;
    for (uint32_t b = threadIdx.x; b < B; b += blockDim.x) s += A[(size_t)b * N + n];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = red[0];
}

__global__ void k_zero(float *__restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// embedding gradient: scatter-add the input gradient rows by byte value.
// Each workgroup accumulates its rows into an LDS copy of the table, then
// adds the non-zero entries to the global gradient. 16 rows per workgroup:
// the loop is latency-bound, so the batch is spread over many workgroups.
constexpr uint32_t kEmbRowsPerBlock = 16;

__global__ __launch_bounds__(256) void k_embed_bwd(const uint16_t *__restrict__ win, uint32_t B,
                                                   const float *__restrict__ dX, float *__restrict__ demb) {
    __shared__ float acc[256 * kMlpEmb];
    for (uint32_t i = threadIdx.x; i < 256 * kMlpEmb; i += blockDim.x) acc[i] = 0.0f;
    __syncthreads();
    const uint32_t r0 = blockIdx.x * kEmbRowsPerBlock;
    const uint32_t r1 = min(B, r0 + kEmbRowsPerBlock);
    for (uint32_t i = r0 * kMlpIn + threadIdx.x; i < r1 * kMlpIn; i += blockDim.x) {
        const uint32_t b = i / kMlpIn, r = i % kMlpIn;
        const uint32_t w = win[b * kMlpWindow + r / kMlpEmb];
        if (w < 256) atomicAdd(&acc[w * kMlpEmb + r % kMlpEmb], dX[i]);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < 256 * kMlpEmb; i += blockDim.x)
        if (acc[i] != 0.0f) atomicAdd(&demb[i], acc[i]);
}

__global__ void k_zero_u32(uint32_t *__restrict__ p, uint32_t n) {
    if (threadIdx.x < n) p[threadIdx.x] = 0u;
}

__global__ void k_adamw(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                        float *__restrict__ v, uint16_t *__restrict__ w16, size_t n, float lr, float b1, float b2,
                        float eps, float wd, float bc1, float bc2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    const float wi = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
    w[i] = wi;
    w16[i] = f2bf(wi);
}

__global__ void k_to_bf16(const float *__restrict__ w, uint16_t *__restrict__ w16, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w16[i] = f2bf(w[i]);
}

// Top-m of each row's logits among the states of its class list (ties: the
// lower state id). Writes the chosen states' positions in the class list,
// ascending, and their number. The first chunk (start class) keeps {q0}.
// One wave per row: pass t takes the best item strictly after pass t-1's
// pick in the order (logit descending, position ascending), each lane over
// positions lane, lane + 64, ... and the wave joining the lanes' bests; lists
// are sorted by state id, so position order is state-id order.
__global__ __launch_bounds__(256) void k_topm(const float *__restrict__ Z, uint32_t rows, uint32_t S,
                                              const uint16_t *__restrict__ wcls, const uint32_t *__restrict__ loff,
                                              const uint32_t *__restrict__ llist, uint32_t m, uint32_t RM,
                                              uint16_t *__restrict__ sel, uint8_t *__restrict__ nsel) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (row >= rows) return;  // whole waves
    const uint32_t c = wcls[row];
    const uint32_t lo = loff[c], sz = loff[c + 1] - lo;
    uint16_t *out = sel + (size_t)row * RM;
    if (sz <= m) {
        for (uint32_t j = lane; j < sz; j += 64) out[j] = (uint16_t)j;
        if (lane == 0) nsel[row] = (uint8_t)sz;
        return;
    }
    const float *z = Z + (size_t)row * S;
    uint32_t picked[16];
    float last_v = INFINITY;
    uint32_t last_j = 0xffffffffu;
    for (uint32_t t = 0; t < m; ++t) {
        float best = -INFINITY;
        uint32_t bj = 0xffffffffu;
        for (uint32_t j = lane; j < sz; j += 64) {
            const uint32_t s = llist[lo + j];
            const float v = s < S ? z[s] : -INFINITY;
            const bool after = t == 0 || v < last_v || (v == last_v && j > last_j);
            if (!after) continue;
            if (bj == 0xffffffffu || v > best) {  // strict: the lower position wins ties
                best = v;
                bj = j;
            }
        }
        // join: larger logit, then lower position; lanes without a candidate
        // carry position 0xffffffff and lose every comparison
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const float ov = __shfl_xor(best, o, 64);
            const uint32_t oj = (uint32_t)__shfl_xor((int)bj, o, 64);
            const bool take = oj != 0xffffffffu && (bj == 0xffffffffu || ov > best || (ov == best && oj < bj));
            best = take ? ov : best;
            bj = take ? oj : bj;
        }
        picked[t] = bj;
        last_v = best;
        last_j = bj;
    }
    if (lane == 0) {
        for (uint32_t a = 1; a < m; ++a)
            for (uint32_t b = a; b > 0 && picked[b - 1] > picked[b]; --b) {
                const uint32_t x = picked[b];
                picked[b] = picked[b - 1];
                picked[b - 1] = x;
            }
        for (uint32_t t = 0; t < m; ++t) out[t] = (uint16_t)picked[t];
        nsel[row] = (uint8_t)m;
    }
}

// ---------------------------------------------------------------------------
// fused inference: windows -> embeddings -> two GELU layers -> head -> top-m
// for 128 chunk boundaries per workgroup, intermediates in LDS (heads of at
// most 64 states). The arithmetic is that of forward_rows: bf16 operands,
// MFMA fp32 accumulation in the same k order, bf16(gelu(acc + b)) hidden
// activations, fp32 logits acc + b3, so the logits are the same numbers.
// ---------------------------------------------------------------------------

constexpr int kFuseRows = 128;            // chunk boundaries per workgroup
constexpr int kFuseThreads = 512;         // 8 waves, each a 64 x 64 output block
constexpr int kFuseHeadMax = 64;          // head rows the fused kernel handles
constexpr int kFuseHRow = kMlpHid + 8;    // LDS row of hidden activations (elements)
constexpr int kFuseKT = 64;               // weight k-slice per stage (elements)
constexpr int kFuseBRow = kFuseKT + 8;    // LDS row of a staged weight k-slice (elements)

struct FuseLds {
    static constexpr size_t kB = 2 * (size_t)kMlpHid * kFuseBRow * 2;     // double-buffered weight slices
    static constexpr size_t kH = (size_t)kFuseRows * kFuseHRow * 2;        // hidden activations / logits
    static constexpr size_t kE = 256 * kMlpEmb * 2;                        // embedding table (bf16)
    static constexpr size_t kW = (size_t)kFuseRows * kMlpWindow;           // window bytes
    static constexpr size_t kC = (size_t)kFuseRows * 8;                    // class list (offset, size) per row
    static constexpr size_t kBytes = kB + kH + kE + kW + kC;
};
// after the head, the weight slices' space holds each row's logits in class
// list order (padded row against bank conflicts)
constexpr int kFuseKeyRow = kFuseHeadMax + 1;
static_assert((size_t)kFuseRows * kFuseKeyRow * 4 <= FuseLds::kB, "list logits fit the weight slices");

// weight rows [0, R) of W (row length K, bf16) at k-slice k0 .. k0+63 into Bs;
// rows >= valid are zero. Thread t stages 32 elements of row t / 2.
__device__ __forceinline__ void fuse_load_w(const uint16_t *__restrict__ W, int K, int R, int valid, int k0,
                                            uint4 (&r)[4]) {
    const int t = threadIdx.x;
    const int row = t >> 1, kof = (t & 1) * 32;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        r[h] = make_uint4(0, 0, 0, 0);
        if (row < R && row < valid) r[h] = *reinterpret_cast<const uint4 *>(W + (size_t)row * K + k0 + kof + 8 * h);
    }
}
__device__ __forceinline__ void fuse_store_w(uint16_t *Bs, int R, const uint4 (&r)[4]) {
    const int t = threadIdx.x;
    const int row = t >> 1, kof = (t & 1) * 32;
    if (row < R) {
#pragma unroll
        for (int h = 0; h < 4; ++h) *reinterpret_cast<uint4 *>(Bs + row * kFuseBRow + kof + 8 * h) = r[h];
    }
}

// One dense layer over the workgroup's 128 rows: acc[i][j] (row tile i, col
// tile j of this wave's block) = sum_k A[row][k] W[col][k]; A from `a_of`
// (8 consecutive k per lane, the 32x32x16 operand layout of k_gemm_nt).
template <int TI, int TJ, typename AOf>
__device__ __forceinline__ void fuse_layer(const uint16_t *__restrict__ W, int K, int R, int valid, uint16_t *Bs,
                                           int wm, int wn, AOf a_of, f32x16 (&acc)[TI][TJ]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    uint4 rb[4];
    fuse_load_w(W, K, R, valid, 0, rb);
    fuse_store_w(Bs, R, rb);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += kFuseKT) {
        const bool more = k0 + kFuseKT < K;
        if (more) fuse_load_w(W, K, R, valid, k0 + kFuseKT, rb);
        const uint16_t *B = Bs + buf * kMlpHid * kFuseBRow;
#pragma unroll
        for (int ks = 0; ks < kFuseKT; ks += 16) {
            const int kk = ks + 8 * (lane >> 5);
            bf16x8 a[TI], b[TJ];
#pragma unroll
            for (int i = 0; i < TI; ++i) a[i] = a_of(wm + 32 * i + (lane & 31), k0 + kk);
#pragma unroll
            for (int j = 0; j < TJ; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(B + (wn + 32 * j + (lane & 31)) * kFuseBRow + kk);
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) fuse_store_w(Bs + (buf ^ 1) * kMlpHid * kFuseBRow, R, rb);
        __syncthreads();
        buf ^= 1;
    }
}

__global__ __launch_bounds__(kFuseThreads) void k_mlp_select(const uint8_t *__restrict__ text, uint64_t L,
                                                            uint32_t chunks, const uint8_t *__restrict__ cls,
                                                            uint32_t start_class, const uint16_t *__restrict__ w16,
                                                            const float *__restrict__ w32, size_t o_emb, size_t o_W1,
                                                            size_t o_b1, size_t o_W2, size_t o_b2, size_t o_W3,
                                                            size_t o_b3, uint32_t S, const uint32_t *__restrict__ loff,
                                                            const uint32_t *__restrict__ llist, uint32_t m,
                                                            uint32_t RM, uint16_t *__restrict__ sel,
                                                            uint8_t *__restrict__ nsel, uint32_t *__restrict__ zero,
                                                            uint32_t nzero) {
    extern __shared__ __align__(16) uint8_t smem[];
    if (blockIdx.x == 0 && threadIdx.x < nzero) zero[threadIdx.x] = 0u;
    uint16_t *Bs = reinterpret_cast<uint16_t *>(smem);
    uint16_t *H = reinterpret_cast<uint16_t *>(smem + FuseLds::kB);
    uint16_t *E = reinterpret_cast<uint16_t *>(smem + FuseLds::kB + FuseLds::kH);
    uint8_t *Wn = smem + FuseLds::kB + FuseLds::kH + FuseLds::kE;
    uint32_t *Cl = reinterpret_cast<uint32_t *>(Wn + FuseLds::kW);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t r0 = (uint64_t)blockIdx.x * kFuseRows;

    // windows (chunk 0 has none: its selection is {q0}) and the embedding
    // table, every load issued before the first wait. Row r's window is
    // text[c L - 32, c L) with c = r0 + r; thread 2r + h holds its half h.
    // The class of the byte before the boundary (the window's last byte) is
    // looked up by thread 2r + 1 and used only at the end.
    uint32_t cls_row = start_class;
    if (tid < 2 * kFuseRows) {
        const int r = tid >> 1, h = tid & 1;
        const uint64_t c = r0 + r;
        const bool live = c > 0 && c < chunks;
        const uint8_t *src = text + c * L - kMlpWindow + 16 * h;
        uint32_t last = 0;
        if (((reinterpret_cast<uintptr_t>(text) | L) & 15) == 0) {
            uint4 v = make_uint4(0, 0, 0, 0);
            if (live) v = *reinterpret_cast<const uint4 *>(src);
            reinterpret_cast<uint4 *>(Wn)[tid] = v;
            last = v.w >> 24;
        } else {
            uint8_t v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = live ? src[k] : (uint8_t)0;
#pragma unroll
            for (int k = 0; k < 16; ++k) Wn[16 * tid + k] = v[k];
            last = v[15];
        }
        if (h == 1 && live) cls_row = cls[last];
    }
    reinterpret_cast<uint4 *>(E)[tid] = reinterpret_cast<const uint4 *>(w16 + o_emb)[tid];
    static_assert(256 * kMlpEmb / 8 == kFuseThreads, "one 16-byte piece of the embedding table per thread");
    __syncthreads();

    const int wm = (wave >> 2) * 64, wn = (wave & 3) * 64;
    f32x16 acc[2][2];
    // layer 1: A[row][k] = emb[window byte k / 16][k % 16]
    auto a_emb = [&](int row, int k) {
        const uint32_t byte = Wn[row * kMlpWindow + (k >> 4)];
        return *reinterpret_cast<const bf16x8 *>(E + byte * kMlpEmb + (k & 15));
    };
    fuse_layer<2, 2>(w16 + o_W1, kMlpIn, kMlpHid, kMlpHid, Bs, wm, wn, a_emb, acc);
    // h1 = bf16(gelu(acc + b1)) into H
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = wn + 32 * j + (lane & 31);
            const float bn = w32[o_b1 + n];
            uint16_t *hp = H + (wm + 32 * i + 4 * (lane >> 5)) * kFuseHRow + n;
#pragma unroll
            for (int r = 0; r < 16; r += 2) {
                const uint32_t pk = f2bf2(gelu(acc[i][j][r] + bn), gelu(acc[i][j][r + 1] + bn));
                hp[(8 * (r >> 2) + (r & 3)) * kFuseHRow] = (uint16_t)pk;
                hp[(8 * (r >> 2) + (r & 3) + 1) * kFuseHRow] = (uint16_t)(pk >> 16);
            }
        }
    __syncthreads();
    // layer 2: A = h1
    auto a_h = [&](int row, int k) { return *reinterpret_cast<const bf16x8 *>(H + row * kFuseHRow + k); };
    fuse_layer<2, 2>(w16 + o_W2, kMlpHid, kMlpHid, kMlpHid, Bs, wm, wn, a_h, acc);
    // every wave has read h1 (the layer ends with a barrier): overwrite with h2
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = wn + 32 * j + (lane & 31);
            const float bn = w32[o_b2 + n];
            uint16_t *hp = H + (wm + 32 * i + 4 * (lane >> 5)) * kFuseHRow + n;
#pragma unroll
            for (int r = 0; r < 16; r += 2) {
                const uint32_t pk = f2bf2(gelu(acc[i][j][r] + bn), gelu(acc[i][j][r + 1] + bn));
                hp[(8 * (r >> 2) + (r & 3)) * kFuseHRow] = (uint16_t)pk;
                hp[(8 * (r >> 2) + (r & 3) + 1) * kFuseHRow] = (uint16_t)(pk >> 16);
            }
        }
    __syncthreads();
    // head: 128 rows x 64 columns (states >= S are zero rows); wave: one 32 x 32 tile
    f32x16 zacc[1][1];
    fuse_layer<1, 1>(w16 + o_W3, kMlpHid, kFuseHeadMax, (int)S, Bs, (wave >> 1) * 32, (wave & 1) * 32, a_h, zacc);
    // the layer ended with a barrier: logits (fp32) over h2
    float *Z = reinterpret_cast<float *>(H);
    {
        const int n = (wave & 1) * 32 + (lane & 31);
        const float bn = n < (int)S ? w32[o_b3 + n] : 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = (wave >> 1) * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            Z[row * kFuseHeadMax + n] = zacc[0][0][r] + bn;
        }
    }
    // each row's class list: (offset, size)
    if (tid < 2 * kFuseRows && (tid & 1)) {
        const uint32_t lo = loff[cls_row];
        Cl[2 * (tid >> 1)] = lo;
        Cl[2 * (tid >> 1) + 1] = loff[cls_row + 1] - lo;
    }
    __syncthreads();
    // logits in list order into the weight slices' space (free after the head)
    // (every list load is issued before the first is used)
    float *Key = reinterpret_cast<float *>(Bs);
    constexpr int kKeyIters = kFuseRows * kFuseHeadMax / kFuseThreads;
    uint32_t stv[kKeyIters];
#pragma unroll
    for (int q = 0; q < kKeyIters; ++q) {
        const int i = tid + q * kFuseThreads, r = i / kFuseHeadMax, j = i % kFuseHeadMax;
        stv[q] = j < (int)Cl[2 * r + 1] ? llist[Cl[2 * r] + j] : 0xffffffffu;
    }
#pragma unroll
    for (int q = 0; q < kKeyIters; ++q) {
        const int i = tid + q * kFuseThreads, r = i / kFuseHeadMax, j = i % kFuseHeadMax;
        if (stv[q] != 0xffffffffu) Key[r * kFuseKeyRow + j] = Z[r * kFuseHeadMax + stv[q]];
    }
    __syncthreads();
    // top-m within each row's class list (at most 64 positions), in the order
    // (logit descending, position ascending) as k_topm: min(m, sz - m) passes,
    // each taking the best remaining position or dropping the worst kept one
    // (the last of the order). Four lanes per row (one workgroup of 512 holds
    // the 128 rows): each scans the positions j = q (mod 4), two quad shuffles
    // pick the pass's winner; the kept positions are written ascending.
    static_assert(kFuseThreads == 4 * kFuseRows, "four lanes per row");
    {
        const uint32_t r = tid >> 2, q = tid & 3;
        const uint64_t row = r0 + r;
        if (row < chunks) {
            const uint32_t sz = Cl[2 * r + 1];
            const float *z = Key + r * kFuseKeyRow;
            const uint32_t take = sz < m ? sz : m;
            uint64_t keep = sz >= 64 ? ~0ull : (1ull << sz) - 1;
            // (v, j) of two lanes of the quad: the one first in the pass's order
            auto pick = [&](float &v, int &j, bool best) {
#pragma unroll
                for (int o = 1; o <= 2; o <<= 1) {
                    const float ov = __shfl_xor(v, o, 64);
                    const int oj = __shfl_xor(j, o, 64);
                    const bool take_o = oj >= 0 && (j < 0 || (best ? (ov > v || (ov == v && oj < j))
                                                                   : (ov < v || (ov == v && oj > j))));
                    if (take_o) {
                        v = ov;
                        j = oj;
                    }
                }
            };
            if (take < sz && take <= sz - take) {
                keep = 0;
                for (uint32_t t = 0; t < take; ++t) {
                    float best = 0.0f;
                    int bj = -1;
                    for (uint32_t j = q; j < sz; j += 4) {
                        const float v = z[j];
                        if (!((keep >> j) & 1ull) && (bj < 0 || v > best)) {
                            best = v;
                            bj = (int)j;
                        }
                    }
                    pick(best, bj, true);
                    keep |= 1ull << bj;
                }
            } else if (take < sz) {
                for (uint32_t t = 0; t < sz - take; ++t) {
                    float worst = 0.0f;
                    int wj = -1;
                    for (uint32_t j = q; j < sz; j += 4) {
                        const float v = z[j];
                        if (((keep >> j) & 1ull) && (wj < 0 || v <= worst)) {
                            worst = v;
                            wj = (int)j;
                        }
                    }
                    // (a lane's candidates come in ascending j: on a tie the
                    // later one is the one to drop)
                    pick(worst, wj, false);
                    keep &= ~(1ull << wj);
                }
            }
            uint16_t *out = sel + row * RM;
            for (uint32_t j = q; j < sz; j += 4)
                if ((keep >> j) & 1ull) out[__popcll(keep & ((1ull << j) - 1))] = (uint16_t)j;
            if (q == 0) nsel[row] = (uint8_t)take;
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

void proposal_layout(Proposal &p) {
    size_t k = 0;
    p.o_emb = k; k += 256 * kMlpEmb;
    p.o_W1 = k; k += (size_t)kMlpHid * kMlpIn;
    p.o_b1 = k; k += kMlpHid;
    p.o_W2 = k; k += (size_t)kMlpHid * kMlpHid;
    p.o_b2 = k; k += kMlpHid;
    p.o_W3 = k; k += (size_t)p.S * kMlpHid;
    p.o_b3 = k; k += p.S;
    p.nparams = k;
}

static parem_status ensure_train(Proposal &p, uint32_t B) {
    if (p.cap_batch >= B) return PAREM_OK;
    hipFree(p.t_buf);
    p.t_buf = nullptr;
    const size_t S = p.S;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = round_up(off + bytes, 256); return o; };
    p.t_pos = take((size_t)B * 8);
    p.t_lab = take((size_t)B * 4);
    p.t_win = take((size_t)B * kMlpWindow * 2);
    p.t_cls = take((size_t)B * 2);
    p.t_X = take((size_t)B * kMlpIn * 2);
    p.t_pre1 = take((size_t)B * kMlpHid * 4);
    p.t_H1 = take((size_t)B * kMlpHid * 2);
    p.t_pre2 = take((size_t)B * kMlpHid * 4);
    p.t_H2 = take((size_t)B * kMlpHid * 2);
    p.t_Z = take((size_t)B * S * 4);
    p.t_dZ32 = take((size_t)B * S * 4);
    p.t_dZ16 = take((size_t)B * S * 2);
    p.t_dA2_32 = take((size_t)B * kMlpHid * 4);
    p.t_dA2_16 = take((size_t)B * kMlpHid * 2);
    p.t_dA1_32 = take((size_t)B * kMlpHid * 4);
    p.t_dA1_16 = take((size_t)B * kMlpHid * 2);
    p.t_dX = take((size_t)B * kMlpIn * 4);
    p.t_loss = take(256);
    // split-K partials of the three weight-gradient GEMMs (K = B), laid out
    // as the dispatcher writes them
    size_t part = 0;
    const int shapes[3][2] = {{(int)S, (int)kMlpHid}, {(int)kMlpHid, (int)kMlpHid}, {(int)kMlpHid, (int)kMlpIn}};
    for (const auto &mn : shapes) {
        const int sk = splitk_of(mn[0], mn[1], (int)B);
        if (sk <= 1) continue;
        const size_t split = ((size_t)B / sk + kKT - 1) / kKT * kKT;
        const size_t nz = (B + split - 1) / split;
        part = std::max(part, nz * mn[0] * mn[1] * 4);
    }
    p.t_part = take(part ? part : 4);
    if (hipMalloc(&p.t_buf, off) != hipSuccess) {
        p.t_buf = nullptr;
        p.cap_batch = 0;
        return PAREM_ENOMEM;
    }
    p.cap_batch = B;
    return PAREM_OK;
}

template <typename T>
static T *at(void *base, size_t off) {
    return reinterpret_cast<T *>(reinterpret_cast<uint8_t *>(base) + off);
}

// forward over B rows whose windows/classes are already in place; fills Z
static void forward_rows(const Proposal &p, hipStream_t s, const uint16_t *win, uint32_t B, uint16_t *X,
                         float *pre1, uint16_t *H1, float *pre2, uint16_t *H2, float *Z) {
    const uint16_t *w16 = p.d_params16;
    const float *w32 = p.d_params;
    const uint32_t nb = (B * kMlpIn + 255) / 256;
    hipLaunchKernelGGL(k_embed, dim3(nb), dim3(256), 0, s, win, B, w16 + p.o_emb, X);
    if (pre1) {
        gemm<false, true, EPI_BIAS_GELU>(s, X, kMlpIn, w16 + p.o_W1, kMlpIn, B, kMlpHid, kMlpIn, w32 + p.o_b1,
                                         nullptr, pre1, H1, kMlpHid);
        gemm<false, true, EPI_BIAS_GELU>(s, H1, kMlpHid, w16 + p.o_W2, kMlpHid, B, kMlpHid, kMlpHid, w32 + p.o_b2,
                                         nullptr, pre2, H2, kMlpHid);
    } else {
        gemm<false, true, EPI_BIAS_BF16>(s, X, kMlpIn, w16 + p.o_W1, kMlpIn, B, kMlpHid, kMlpIn, w32 + p.o_b1,
                                         nullptr, nullptr, H1, kMlpHid);
        gemm<false, true, EPI_BIAS_BF16>(s, H1, kMlpHid, w16 + p.o_W2, kMlpHid, B, kMlpHid, kMlpHid,
                                         w32 + p.o_b2, nullptr, nullptr, H2, kMlpHid);
    }
    gemm<false, true, EPI_BIAS_F32>(s, H2, kMlpHid, w16 + p.o_W3, kMlpHid, B, (int)p.S, kMlpHid, w32 + p.o_b3,
                                    nullptr, Z, nullptr, (int)p.S);
}

parem_status proposal_train_step(Proposal &p, const uint8_t *d_text, uint64_t len, const uint64_t *d_pos,
                                 const uint32_t *d_labels, uint32_t B, float lr, float wd, hipStream_t s,
                                 float *d_loss_out) {
    if (B == 0) return PAREM_EINVAL;
    parem_status st = ensure_train(p, B);
    if (st != PAREM_OK) return st;
    const DeviceDfa &d = *p.dfa;
    void *T = p.t_buf;
    uint16_t *win = at<uint16_t>(T, p.t_win), *wcls = at<uint16_t>(T, p.t_cls);
    const uint32_t S = p.S;
    const uint32_t nw = (B * kMlpWindow + 255) / 256;
    hipLaunchKernelGGL(k_windows, dim3(nw), dim3(256), 0, s, d_text, len, d_pos, B, d.d_cls, d.A + 1, win, wcls);
    float *loss = d_loss_out ? d_loss_out : at<float>(T, p.t_loss);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, loss, (size_t)1);
    uint16_t *X = at<uint16_t>(T, p.t_X), *H1 = at<uint16_t>(T, p.t_H1), *H2 = at<uint16_t>(T, p.t_H2);
    float *pre1 = at<float>(T, p.t_pre1), *pre2 = at<float>(T, p.t_pre2), *Z = at<float>(T, p.t_Z);
    forward_rows(p, s, win, B, X, pre1, H1, pre2, H2, Z);
    float *dZ32 = at<float>(T, p.t_dZ32);
    uint16_t *dZ16 = at<uint16_t>(T, p.t_dZ16);
    hipLaunchKernelGGL(k_softmax_ce, dim3(std::min<uint32_t>((B + 3) / 4, 256)), dim3(256), 0, s, Z, B, S, d_labels,
                       wcls, d.d_inv, d.Q + 1, dZ32, dZ16, loss);
    // backward
    float *g = p.d_grad;
    const uint16_t *w16 = p.d_params16;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((256 * kMlpEmb + 255) / 256)), dim3(256), 0, s, g + p.o_emb,
                       (size_t)256 * kMlpEmb);
    // head: dW3 = dZ^T H2, db3 = colsum dZ, dA2 = (dZ W3) * gelu'(pre2)
    float *part = at<float>(T, p.t_part);
    gemm<true, false, EPI_F32>(s, dZ16, (int)S, H2, kMlpHid, (int)S, kMlpHid, (int)B, nullptr, nullptr, g + p.o_W3,
                               nullptr, kMlpHid, part);
    hipLaunchKernelGGL(k_colsum, dim3(S), dim3(256), 0, s, dZ32, B, S, g + p.o_b3);
    float *dA2_32 = at<float>(T, p.t_dA2_32), *dA1_32 = at<float>(T, p.t_dA1_32);
    uint16_t *dA2_16 = at<uint16_t>(T, p.t_dA2_16), *dA1_16 = at<uint16_t>(T, p.t_dA1_16);
    gemm<false, false, EPI_GELU_BWD>(s, dZ16, (int)S, w16 + p.o_W3, kMlpHid, (int)B, kMlpHid, (int)S, nullptr, pre2,
                                     dA2_32, dA2_16, kMlpHid);
    // layer 2
    gemm<true, false, EPI_F32>(s, dA2_16, kMlpHid, H1, kMlpHid, kMlpHid, kMlpHid, (int)B, nullptr, nullptr,
                               g + p.o_W2, nullptr, kMlpHid, part);
    hipLaunchKernelGGL(k_colsum, dim3(kMlpHid), dim3(256), 0, s, dA2_32, B, kMlpHid, g + p.o_b2);
    gemm<false, false, EPI_GELU_BWD>(s, dA2_16, kMlpHid, w16 + p.o_W2, kMlpHid, (int)B, kMlpHid, kMlpHid, nullptr,
                                     pre1, dA1_32, dA1_16, kMlpHid);
    // layer 1
    gemm<true, false, EPI_F32>(s, dA1_16, kMlpHid, X, kMlpIn, kMlpHid, kMlpIn, (int)B, nullptr, nullptr,
                               g + p.o_W1, nullptr, kMlpIn, part);
    hipLaunchKernelGGL(k_colsum, dim3(kMlpHid), dim3(256), 0, s, dA1_32, B, kMlpHid, g + p.o_b1);
    float *dX = at<float>(T, p.t_dX);
    gemm<false, false, EPI_F32>(s, dA1_16, kMlpHid, w16 + p.o_W1, kMlpIn, (int)B, kMlpIn, kMlpHid, nullptr, nullptr,
                                dX, nullptr, kMlpIn);
    hipLaunchKernelGGL(k_embed_bwd, dim3((B + kEmbRowsPerBlock - 1) / kEmbRowsPerBlock), dim3(256), 0, s, win, B, dX,
                       g + p.o_emb);
    if (lr > 0.0f || wd > 0.0f) return proposal_adamw(p, g, lr, wd, s);
    return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
}

// One AdamW step on the master weights with gradient g (device, nparams).
// The bias corrections 1 - beta^t are formed in double on the host: in fp32,
// 1 - 0.999^t loses most of its digits for small t.
parem_status proposal_adamw(Proposal &p, const float *g, float lr, float wd, hipStream_t s) {
    p.step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = (float)(1.0 - std::pow((double)b1, (double)p.step));
    const float bc2 = (float)(1.0 - std::pow((double)b2, (double)p.step));
    hipLaunchKernelGGL(k_adamw, dim3((unsigned)((p.nparams + 255) / 256)), dim3(256), 0, s, p.d_params, g, p.d_m,
                       p.d_v, p.d_params16, p.nparams, lr, b1, b2, 1e-8f, wd, bc1, bc2);
    return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
}

size_t proposal_infer_bytes(const Proposal &p, uint64_t rows) {
    size_t b = 0;
    b += round_up(rows * kMlpWindow * 2, 256);
    b += round_up(rows * 2, 256);
    b += round_up(rows * kMlpIn * 2, 256);
    b += 2 * round_up(rows * kMlpHid * 2, 256);
    b += round_up(rows * p.S * 4, 256);
    return b;
}

// logits of the chunk boundaries c * L and the top-m selection per chunk
parem_status proposal_select(const Proposal &p, const uint8_t *d_text, uint64_t L, uint32_t chunks, uint32_t m,
                             uint32_t RM, void *scratch, hipStream_t s, uint16_t *sel, uint8_t *nsel, uint32_t *zero,
                             uint32_t nzero) {
    const DeviceDfa &d = *p.dfa;
    if (p.S <= (uint32_t)kFuseHeadMax && L >= 2 * kMlpWindow) {
        // fused path: no intermediates in memory
        static std::once_flag lds_once;
        static hipError_t lds_err = hipSuccess;
        std::call_once(lds_once, [] {
            lds_err = hipFuncSetAttribute(reinterpret_cast<const void *>(k_mlp_select),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)FuseLds::kBytes);
        });
        if (lds_err != hipSuccess) return PAREM_EDEVICE;
        hipLaunchKernelGGL(k_mlp_select, dim3((chunks + kFuseRows - 1) / kFuseRows), dim3(kFuseThreads),
                           FuseLds::kBytes, s, d_text, L, chunks, d.d_cls, d.A + 1, p.d_params16, p.d_params,
                           p.o_emb, p.o_W1, p.o_b1, p.o_W2, p.o_b2, p.o_W3, p.o_b3, p.S, d.d_loff, d.d_llist, m, RM,
                           sel, nsel, zero, nzero);
        return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = round_up(off + bytes, 256); return o; };
    uint16_t *win = at<uint16_t>(scratch, take((size_t)chunks * kMlpWindow * 2));
    uint16_t *wcls = at<uint16_t>(scratch, take((size_t)chunks * 2));
    uint16_t *X = at<uint16_t>(scratch, take((size_t)chunks * kMlpIn * 2));
    uint16_t *H1 = at<uint16_t>(scratch, take((size_t)chunks * kMlpHid * 2));
    uint16_t *H2 = at<uint16_t>(scratch, take((size_t)chunks * kMlpHid * 2));
    float *Z = at<float>(scratch, take((size_t)chunks * p.S * 4));
    hipLaunchKernelGGL(k_windows_chunks, dim3((chunks * kMlpWindow + 255) / 256), dim3(256), 0, s, d_text, L, chunks,
                       d.d_cls, d.A + 1, win, wcls);
    forward_rows(p, s, win, chunks, X, nullptr, H1, nullptr, H2, Z);
    hipLaunchKernelGGL(k_topm, dim3((chunks + 3) / 4), dim3(256), 0, s, Z, chunks, p.S, wcls, d.d_loff,
                       d.d_llist, m, RM, sel, nsel);
    if (nzero) hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, zero, nzero);
    return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
}

parem_status proposal_logits(const Proposal &p, const uint8_t *d_text, uint64_t len, const uint64_t *d_pos,
                             uint32_t B, float *d_logits, hipStream_t s) {
    Proposal &q = const_cast<Proposal &>(p);
    parem_status st = ensure_train(q, B);
    if (st != PAREM_OK) return st;
    const DeviceDfa &d = *p.dfa;
    void *T = q.t_buf;
    uint16_t *win = at<uint16_t>(T, q.t_win), *wcls = at<uint16_t>(T, q.t_cls);
    hipLaunchKernelGGL(k_windows, dim3((B * kMlpWindow + 255) / 256), dim3(256), 0, s, d_text, len, d_pos, B, d.d_cls,
                       d.A + 1, win, wcls);
    forward_rows(p, s, win, B, at<uint16_t>(T, q.t_X), at<float>(T, q.t_pre1), at<uint16_t>(T, q.t_H1),
                 at<float>(T, q.t_pre2), at<uint16_t>(T, q.t_H2), d_logits);
    return hipGetLastError() == hipSuccess ? PAREM_OK : PAREM_EDEVICE;
}

}  // namespace parem

using parem::Proposal;

extern "C" {

parem_status parem_proposal_create(parem_handle h, const float *params, uint64_t nparams, parem_proposal *out) {
    if (!h || !out || !params) return PAREM_EINVAL;
    *out = nullptr;
    if (h->dev.dead != 0xffffffffu) return PAREM_EUNSUPPORTED;  // no proposals for partial tables
    parem_proposal_s *p = new (std::nothrow) parem_proposal_s();
    if (!p) return PAREM_ENOMEM;
    p->dfa = &h->dev;
    p->S = h->dev.Q;
    parem::proposal_layout(*p);
    if (nparams != p->nparams) {
        delete p;
        return PAREM_EINVAL;
    }
    if (!h->dev.d_inv) {
        delete p;
        return PAREM_EUNSUPPORTED;
    }
    const size_t n = p->nparams;
    bool ok = hipMalloc(&p->d_params, n * 4) == hipSuccess && hipMalloc(&p->d_params16, n * 2) == hipSuccess &&
              hipMalloc(&p->d_grad, n * 4) == hipSuccess && hipMalloc(&p->d_m, n * 4) == hipSuccess &&
              hipMalloc(&p->d_v, n * 4) == hipSuccess;
    ok = ok && hipMemcpy(p->d_params, params, n * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(p->d_m, 0, n * 4) == hipSuccess && hipMemset(p->d_v, 0, n * 4) == hipSuccess &&
         hipMemset(p->d_grad, 0, n * 4) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(parem::k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, p->d_params,
                           p->d_params16, n);
        ok = hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        parem_proposal_free(p);
        return PAREM_ENOMEM;
    }
    *out = p;
    return PAREM_OK;
}

void parem_proposal_free(parem_proposal p) {
    if (!p) return;
    hipFree(p->d_params);
    hipFree(p->d_params16);
    hipFree(p->d_grad);
    hipFree(p->d_m);
    hipFree(p->d_v);
    hipFree(p->t_buf);
    delete p;
}

parem_status parem_proposal_params(parem_proposal p, float *params_out, float *grad_out, uint64_t nparams) {
    if (!p || nparams != p->nparams) return PAREM_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return PAREM_EDEVICE;
    if (params_out && hipMemcpy(params_out, p->d_params, nparams * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return PAREM_EDEVICE;
    if (grad_out && hipMemcpy(grad_out, p->d_grad, nparams * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return PAREM_EDEVICE;
    return PAREM_OK;
}

parem_status parem_proposal_train_step(parem_proposal p, const uint8_t *d_text, uint64_t len,
                                       const uint64_t *d_positions, const uint32_t *d_labels, uint32_t batch,
                                       float lr, float weight_decay, void *stream, float *d_loss) {
    if (!p || !d_text || !d_positions || !d_labels || batch == 0) return PAREM_EINVAL;
    return parem::proposal_train_step(*p, d_text, len, d_positions, d_labels, batch, lr, weight_decay,
                                      reinterpret_cast<hipStream_t>(stream), d_loss);
}

parem_status parem_proposal_select_size(parem_proposal p, uint64_t len, uint32_t chunk_len, uint64_t *bytes) {
    if (!p || !bytes || chunk_len == 0) return PAREM_EINVAL;
    const uint64_t chunks = (len + chunk_len - 1) / chunk_len;
    *bytes = parem::proposal_infer_bytes(*p, chunks ? chunks : 1);
    return PAREM_OK;
}

parem_status parem_proposal_select(parem_proposal p, const uint8_t *d_text, uint64_t len, uint32_t chunk_len,
                                   uint32_t m, uint16_t *d_sel, uint8_t *d_nsel, void *d_workspace,
                                   uint64_t workspace_bytes, void *stream) {
    if (!p || !d_text || !d_sel || !d_nsel || chunk_len == 0 || m == 0 || m > 16) return PAREM_EINVAL;
    const uint64_t chunks = (len + chunk_len - 1) / chunk_len;
    if (chunks == 0 || chunks > 0xffffffffull) return PAREM_EINVAL;
    if (!d_workspace || workspace_bytes < parem::proposal_infer_bytes(*p, chunks)) return PAREM_EINVAL;
    return parem::proposal_select(*p, d_text, chunk_len, (uint32_t)chunks, m, m, d_workspace,
                                  reinterpret_cast<hipStream_t>(stream), d_sel, d_nsel);
}

parem_status parem_proposal_logits(parem_proposal p, const uint8_t *d_text, uint64_t len,
                                   const uint64_t *d_positions, uint32_t batch, float *d_logits, void *stream) {
    if (!p || !d_text || !d_positions || !d_logits || batch == 0) return PAREM_EINVAL;
    return parem::proposal_logits(*p, d_text, len, d_positions, batch, d_logits,
                                  reinterpret_cast<hipStream_t>(stream));
}

parem_status parem_proposal_apply_grad(parem_proposal p, const float *d_grad, uint64_t nparams, float lr,
                                       float weight_decay, void *stream) {
    if (!p || !d_grad || nparams != p->nparams) return PAREM_EINVAL;
    return parem::proposal_adamw(*p, d_grad, lr, weight_decay, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
