// The depth-order network on gfx950: x -> [Linear -> GELU] x depth -> Linear -> softmax over T-counts,
// cross-entropy loss, Adam on FP32 master weights.  Every product is a BF16 x BF16 -> FP32 MFMA GEMM
// (v_mfma_f32_16x16x32_bf16) with operands in either orientation, so forward, dX and dW use one kernel:
//   forward:  Z = H W + b            (A = H, B = W)
//   dW:       dW = H^T G             (A = H transposed in memory, B = G)
//   dX:       G' = (G W^T) * gelu'(Z) (A = G, B = W transposed in memory)
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "common.h"

namespace tcw {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int TM = 64, TN = 64, TK = 32, LDS_K = 40;  // LDS rows padded to 80 bytes

enum Epi : int {
    EPI_STORE = 0,        // C = acc
    EPI_BIAS_GELU = 1,    // Z = acc + bias (fp32), H = gelu(Z) (bf16)
    EPI_BIAS = 2,         // C = acc + bias (fp32)
    EPI_GELU_GRAD = 3,    // G = acc * gelu'(Z) (fp32 and bf16)
};

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// C[M x N] = op(A)[M x K] op(B)[K x N].  TA: A element (m, k) at A[k * lda + m], else A[m * lda + k].
// TB: B element (k, n) at B[n * ldb + k], else B[k * ldb + n].  256 threads, 64 x 64 tile, 4 waves of 32 x 32.
// blockIdx.z = z takes the products k in [z kchunk, (z + 1) kchunk) (kchunk a multiple of TK) and, for
// EPI_STORE, writes its partial tile to C + z M ldc; with gridDim.z = 1 it is the whole product.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const __bf16* __restrict__ A, const __bf16* __restrict__ B, int M, int N,
                                              int K, int lda, int ldb, float* __restrict__ C, int ldc,
                                              const float* __restrict__ bias, const float* __restrict__ Zin,
                                              __bf16* __restrict__ Hout, int kchunk) {
    __shared__ __attribute__((aligned(16))) __bf16 As[TM][LDS_K];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[TN][LDS_K];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const __bf16 zero = (__bf16)0.0f;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    C += (size_t)blockIdx.z * M * ldc;
    for (int k0 = kb; k0 < ke; k0 += TK) {
        // A tile -> As[m][k]
        if (!TA) {
            const int m = t >> 2, kk = (t & 3) * 8;
            const int gm = m0 + m;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gk = k0 + kk + e;
                As[m][kk + e] = (gm < M && gk < K) ? A[(size_t)gm * lda + gk] : zero;
            }
        } else {
            const int kk = t >> 3, mm = (t & 7) * 8;
            const int gk = k0 + kk;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gm = m0 + mm + e;
                As[mm + e][kk] = (gm < M && gk < K) ? A[(size_t)gk * lda + gm] : zero;
            }
        }
        // B tile -> Bs[n][k]
        if (!TB) {
            const int kk = t >> 3, nn = (t & 7) * 8;
            const int gk = k0 + kk;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gn = n0 + nn + e;
                Bs[nn + e][kk] = (gn < N && gk < K) ? B[(size_t)gk * ldb + gn] : zero;
            }
        } else {
            const int n = t >> 2, kk = (t & 3) * 8;
            const int gn = n0 + n;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gk = k0 + kk + e;
                Bs[n][kk + e] = (gn < N && gk < K) ? B[(size_t)gn * ldb + gk] : zero;
            }
        }
        __syncthreads();
        bf16x8 a[2], b[2];
        const int r16 = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * i + r16][kq]);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * j + r16][kq]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // D layout: lane holds rows 4 (lane / 16) + r, column lane % 16 of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int gn = n0 + wn + 16 * j + (lane & 15);
                if (gm >= M || gn >= N) continue;
                float v = acc[i][j][r];
                const size_t o = (size_t)gm * ldc + gn;
                if (EPI == EPI_STORE) {
                    C[o] = v;
                } else if (EPI == EPI_BIAS) {
                    C[o] = v + bias[gn];
                } else if (EPI == EPI_BIAS_GELU) {
                    v += bias[gn];
                    C[o] = v;
                    Hout[o] = (__bf16)gelu_f(v);
                } else {
                    v *= gelu_grad_f(Zin[o]);
                    C[o] = v;
                    Hout[o] = (__bf16)v;
                }
            }
}

// softmax over `classes` logits per row, loss sum, G = (p - onehot) / batch (fp32 and bf16)
__global__ void k_softmax_ce(const float* logits, const int32_t* labels, int batch, int classes, float* probs,
                             float* g, __bf16* gb, float* loss_sum) {
    const int i = threadIdx.x + blockIdx.x * blockDim.x;
    if (i >= batch) return;
    const float* z = logits + (size_t)i * classes;
    float m = z[0];
    for (int c = 1; c < classes; ++c) m = fmaxf(m, z[c]);
    float s = 0.f;
    for (int c = 0; c < classes; ++c) s += expf(z[c] - m);
    const int y = labels ? labels[i] : -1;
    for (int c = 0; c < classes; ++c) {
        const float p = expf(z[c] - m) / s;
        if (probs) probs[(size_t)i * classes + c] = p;
        if (g) {
            const float gv = (p - (c == y ? 1.f : 0.f)) / (float)batch;
            g[(size_t)i * classes + c] = gv;
            gb[(size_t)i * classes + c] = (__bf16)gv;
        }
    }
    if (loss_sum && y >= 0 && y < classes) atomicAdd(loss_sum, -(z[y] - m - logf(s)));
}

// column sums: db[n] = sum_i G[i][n]
__global__ void k_colsum(const float* g, int rows, int cols, float* out) {
    const int n = blockIdx.x;
    float s = 0.f;
    for (int i = threadIdx.x; i < rows; i += blockDim.x) s += g[(size_t)i * cols + n];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = red[0];
}

__global__ void k_to_bf16(const float* x, __bf16* y, int64_t count) {
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; i < count; i += (int64_t)blockDim.x * gridDim.x)
        y[i] = (__bf16)x[i];
}

// Adam (Kingma & Ba 2015) on the FP32 master copy
__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; i < count; i += (int64_t)blockDim.x * gridDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// seeded initialisation: W uniform in [-1/sqrt(fan_in), 1/sqrt(fan_in)] from SplitMix64 outputs of
// the running index (u = (r >> 40) / 2^24), biases zero
__global__ void k_init(float* w, int64_t count, int64_t index0, int fan_in, uint64_t seed) {
    const double bound = 1.0 / sqrt((double)fan_in);
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; i < count; i += (int64_t)blockDim.x * gridDim.x) {
        const uint64_t r = sm64(seed, (uint64_t)(index0 + i));
        const double u = (double)(r >> 40) / 16777216.0;
        w[i] = (float)__dmul_rn(__dsub_rn(__dmul_rn(2.0, u), 1.0), bound);
    }
}

template <bool TA, bool TB, int EPI>
hipError_t gemm_t(const __bf16* A, const __bf16* B, int M, int N, int K, int lda, int ldb, float* C, int ldc,
                  const float* bias, const float* Z, __bf16* H, hipStream_t s, int splits = 1) {
    dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM, splits);
    const int kchunk = ((K + splits - 1) / splits + TK - 1) / TK * TK;
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, A, B, M, N, K, lda, ldb, C, ldc, bias, Z, H,
                       kchunk);
    return hipGetLastError();
}

// out[i] = sum over z of part[z * mn + i], in the order z = 0, 1, ... (the same sum on every run)
__global__ void k_sum_parts(const float* __restrict__ part, int splits, int64_t mn, float* __restrict__ out) {
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; i < mn; i += (int64_t)blockDim.x * gridDim.x) {
        float v = 0.f;
        for (int z = 0; z < splits; ++z) v += part[(size_t)z * mn + i];
        out[i] = v;
    }
}

// The weight gradient dW = H^T G (M x N) reduces over the batch K.  With few output tiles one tile
// per workgroup leaves most of the GPU idle while each runs the whole batch, so the batch is split
// over up to 16 workgroups per tile (at least 256 samples each) until about 4096 workgroups run.
int dw_splits(int M, int N, int K) {
    const int tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
    int splits = 1;
    while (splits < 16 && tiles * splits < 4096 && K / (2 * splits) >= 256) splits *= 2;
    return splits;
}

}  // namespace

hipError_t mlp_gemm(int mode, const void* A, const void* B, int M, int N, int K, int lda, int ldb, float* C, int ldc,
                    const float* bias, const float* Z, void* H, hipStream_t s) {
    const __bf16* a = (const __bf16*)A;
    const __bf16* b = (const __bf16*)B;
    __bf16* h = (__bf16*)H;
    switch (mode) {
        case 0: return gemm_t<false, false, EPI_STORE>(a, b, M, N, K, lda, ldb, C, ldc, bias, Z, h, s);
        case 1: return gemm_t<false, false, EPI_BIAS_GELU>(a, b, M, N, K, lda, ldb, C, ldc, bias, Z, h, s);
        case 2: return gemm_t<false, false, EPI_BIAS>(a, b, M, N, K, lda, ldb, C, ldc, bias, Z, h, s);
        case 3: return gemm_t<true, false, EPI_STORE>(a, b, M, N, K, lda, ldb, C, ldc, bias, Z, h, s);
        case 4: return gemm_t<false, true, EPI_GELU_GRAD>(a, b, M, N, K, lda, ldb, C, ldc, bias, Z, h, s);
        case 5: return gemm_t<false, true, EPI_STORE>(a, b, M, N, K, lda, ldb, C, ldc, bias, Z, h, s);
        case 6: return gemm_t<true, true, EPI_STORE>(a, b, M, N, K, lda, ldb, C, ldc, bias, Z, h, s);
        default: return hipErrorInvalidValue;
    }
}

size_t mlp_dw_part_floats(int M, int N, int K) {
    const int splits = dw_splits(M, N, K);
    return splits > 1 ? (size_t)splits * M * N : 0;
}

hipError_t mlp_gemm_dw(const void* H, const void* G, int M, int N, int K, float* dW, float* part, size_t part_floats,
                       hipStream_t s) {
    const __bf16* a = (const __bf16*)H;
    const __bf16* b = (const __bf16*)G;
    const int splits = dw_splits(M, N, K);
    if (splits == 1 || part == nullptr || part_floats < (size_t)splits * M * N)
        return gemm_t<true, false, EPI_STORE>(a, b, M, N, K, M, N, dW, N, nullptr, nullptr, nullptr, s);
    hipError_t e = gemm_t<true, false, EPI_STORE>(a, b, M, N, K, M, N, part, N, nullptr, nullptr, nullptr, s, splits);
    if (e != hipSuccess) return e;
    const int64_t mn = (int64_t)M * N;
    int64_t blocks = (mn + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)blocks), dim3(256), 0, s, part, splits, mn, dW);
    return hipGetLastError();
}

hipError_t mlp_softmax_ce(const float* logits, const int32_t* labels, int batch, int classes, float* probs, float* g,
                          void* gb, float* loss_sum, hipStream_t s) {
    hipLaunchKernelGGL(k_softmax_ce, dim3((batch + 255) / 256), dim3(256), 0, s, logits, labels, batch, classes, probs,
                       g, (__bf16*)gb, loss_sum);
    return hipGetLastError();
}

hipError_t mlp_colsum(const float* g, int rows, int cols, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3(cols), dim3(256), 0, s, g, rows, cols, out);
    return hipGetLastError();
}

hipError_t mlp_to_bf16(const float* x, void* y, int64_t count, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)blocks), dim3(256), 0, s, x, (__bf16*)y, count);
    return hipGetLastError();
}

hipError_t mlp_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1, float b2,
                    float eps, int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, s, p, g, m, v, count, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_init(float* w, int64_t count, int64_t index0, int fan_in, uint64_t seed, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(256), 0, s, w, count, index0, fan_in, seed);
    return hipGetLastError();
}

}  // namespace tcw
