// The depth-order network on gfx950: x -> [Linear -> GELU] x depth -> Linear -> softmax over T-counts,
// cross-entropy loss, Adam on FP32 master weights.  Every product is one BF16 x BF16 -> FP32 MFMA
// GEMM of the form C = A B^T with both operands stored K-contiguous (each row of A and of B holds
// consecutive k), so every operand fragment is one 16-byte load:
//   forward:  Z = H W + b              A = H (batch x in),      B = W^T (out x in)
//   dX:       G' = (G W^T) * gelu'(Z)  A = G (batch x out),     B = W (in x out)
//   dW:       dW = H^T G               A = H^T (in x batch),    B = G^T (out x batch)
// The epilogues write the transposed BF16 copies (H^T, G^T) the weight-gradient products read, so no
// product ever reads a strided operand.  Leading dimensions of BF16 buffers are multiples of 8.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "common.h"

namespace tcw {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

enum Epi : int {
    EPI_STORE = 0,      // C = acc
    EPI_BIAS = 1,       // C = acc + bias
    EPI_BIAS_GELU = 2,  // C = Z = acc + bias (fp32), H = gelu(Z) (bf16), T = H^T (bf16, optional)
    EPI_GELU_GRAD = 3,  // C = G = acc * gelu'(Zin) (fp32), H = G (bf16), T = G^T (bf16, optional)
};

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

constexpr int BN = 128, BK = 64, LDK = BK + 8;  // LDS rows of 64 k values padded to 144 bytes

// 8 consecutive k of row r of a K-contiguous operand (leading dimension ld, a multiple of 8), zero
// outside rows < rows and k < kend.
__device__ inline bf16x8 load8(const __bf16* __restrict__ p, int ld, int r, int k, int rows, int kend) {
    if (r < rows && k + 8 <= kend) return *reinterpret_cast<const bf16x8*>(p + (size_t)r * ld + k);
    bf16x8 v;
    const __bf16 zero = (__bf16)0.0f;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (r < rows && k + e < kend) ? p[(size_t)r * ld + k + e] : zero;
    return v;
}

// The epilogue of one output element v at (gm, gn); tv receives the BF16 value that also goes to the
// transposed copy.
template <int EPI>
__device__ inline void epilogue(float v, int gm, int gn, float* __restrict__ C, int ldc,
                                const float* __restrict__ bias, const float* __restrict__ Zin, int ldz,
                                __bf16* __restrict__ Hout, int ldh, __bf16& tv) {
    const size_t o = (size_t)gm * ldc + gn;
    if (EPI == EPI_STORE) {
        C[o] = v;
    } else if (EPI == EPI_BIAS) {
        C[o] = v + bias[gn];
    } else if (EPI == EPI_BIAS_GELU) {
        v += bias[gn];
        C[o] = v;
        tv = (__bf16)gelu_f(v);
        Hout[(size_t)gm * ldh + gn] = tv;
    } else {
        v *= gelu_grad_f(Zin[(size_t)gm * ldz + gn]);
        C[o] = v;
        tv = (__bf16)v;
        Hout[(size_t)gm * ldh + gn] = tv;
    }
}

// C[M x N] = A[M x K] B[N x K]^T.  (BM / WM) x (BN / WN) waves of 64 lanes, each computing a WM x WN
// tile of 32 x 32 MFMA tiles (v_mfma_f32_32x32x16_bf16); K in steps of BK = 64 staged through
// double-buffered LDS, the next step's 16-byte global loads held in registers while the current step
// computes.
// K split: blockIdx.z = z takes k in [z kchunk, (z + 1) kchunk).  With a workspace `part` every block
// writes its FP32 partial tile to part[z] and k_splitk_epilogue adds the partials and applies the
// epilogue; without one (only when gridDim.z = 1) the block applies the epilogue itself.
template <int BM, int BN_, int WM, int WN, int EPI>
__global__ __launch_bounds__((BM / WM) * (BN_ / WN) * 64) void k_gemm_nt(
    const __bf16* __restrict__ A, int lda, const __bf16* __restrict__ B, int ldb, int M, int N, int K,
    float* __restrict__ C, int ldc, const float* __restrict__ bias, const float* __restrict__ Zin, int ldz,
    __bf16* __restrict__ Hout, int ldh, __bf16* __restrict__ Tout, int ldt, int kchunk, float* __restrict__ part) {
    constexpr int WAVES_N = BN_ / WN, NT = (BM / WM) * WAVES_N * 64;
    constexpr int FM = WM / 32, FN = WN / 32;
    constexpr int RSTEP = NT / 8;                      // rows covered by one vector per thread
    constexpr int AV = BM / RSTEP, BV = BN_ / RSTEP;  // 16-byte vectors per thread per step
    static_assert(BM % RSTEP == 0 && BN_ % RSTEP == 0, "tile rows must be a multiple of threads / 8");
    __shared__ __attribute__((aligned(16))) __bf16 As[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BN_ * LDK];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    // Workgroups go to the 8 XCDs in turn (linear id mod 8), each XCD with its own L2.  With the grid's
    // row panels a multiple of 8, ids are remapped so that every tile of one row panel (one slice of A)
    // runs on the same XCD, which then fetches that slice once.
    int bx = blockIdx.x, by = blockIdx.y;
    if ((gridDim.y & 7) == 0) {
        const int id = blockIdx.x + gridDim.x * blockIdx.y, local = id >> 3;
        bx = local % gridDim.x;
        by = (local / gridDim.x) * 8 + (id & 7);
    }
    const int m0 = by * BM, n0 = bx * BN_;
    const int wm = (wave / WAVES_N) * WM, wn = (wave % WAVES_N) * WN;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    const int kv = (t & 7) * 8, r0 = t >> 3;  // this thread's vectors: rows r0 + RSTEP i, k offset kv
    const bool inner_rows = m0 + BM <= M && n0 + BN_ <= N;  // uniform over the block
    bf16x8 ra[AV], rb[BV];
    auto gload = [&](int k0) {
        if (inner_rows && k0 + BK <= ke) {
            // the whole step lies inside both operands: plain 16-byte loads
#pragma unroll
            for (int i = 0; i < AV; ++i)
                ra[i] = *reinterpret_cast<const bf16x8*>(A + (size_t)(m0 + r0 + RSTEP * i) * lda + k0 + kv);
#pragma unroll
            for (int i = 0; i < BV; ++i)
                rb[i] = *reinterpret_cast<const bf16x8*>(B + (size_t)(n0 + r0 + RSTEP * i) * ldb + k0 + kv);
        } else {
#pragma unroll
            for (int i = 0; i < AV; ++i) ra[i] = load8(A, lda, m0 + r0 + RSTEP * i, k0 + kv, M, ke);
#pragma unroll
            for (int i = 0; i < BV; ++i) rb[i] = load8(B, ldb, n0 + r0 + RSTEP * i, k0 + kv, N, ke);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < AV; ++i) *reinterpret_cast<bf16x8*>(&As[buf][(r0 + RSTEP * i) * LDK + kv]) = ra[i];
#pragma unroll
        for (int i = 0; i < BV; ++i) *reinterpret_cast<bf16x8*>(&Bs[buf][(r0 + RSTEP * i) * LDK + kv]) = rb[i];
    };
    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    // operand fragments: lane l holds row l % 32 of its 32-row tile, k = 8 (l / 32) .. + 7 of each 16
    const int fr = lane & 31, fk = 8 * (lane >> 5);
    const int steps = ke > kb ? (ke - kb + BK - 1) / BK : 0;
    if (steps > 0) {
        gload(kb);
        sstore(0);
    }
    __syncthreads();
    for (int s = 0; s < steps; ++s) {
        const int buf = s & 1;
        const bool more = s + 1 < steps;
        if (more) gload(kb + (s + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            bf16x8 a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[i] = *reinterpret_cast<const bf16x8*>(&As[buf][(wm + 32 * i + fr) * LDK + ks + fk]);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][(wn + 32 * j + fr) * LDK + ks + fk]);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) sstore(buf ^ 1);
        __syncthreads();
    }
    // D layout of a 32 x 32 tile: lane l holds column l % 32 and, in value r, row
    // 8 (r / 4) + 4 (l / 32) + r % 4
    if (part == nullptr) {
        // no workspace: the epilogue here (the host passes one whenever K is split)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int gn = n0 + wn + 32 * j + fr;
                if (gn >= N) continue;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int gm4 = m0 + wm + 32 * i + 8 * q + 4 * (lane >> 5);
                    __bf16 tv[4] = {(__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f};
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (gm4 + r < M)
                            epilogue<EPI>(acc[i][j][4 * q + r], gm4 + r, gn, C, ldc, bias, Zin, ldz, Hout, ldh, tv[r]);
                    if ((EPI == EPI_BIAS_GELU || EPI == EPI_GELU_GRAD) && Tout != nullptr) {
                        // four consecutive rows of column gn: four consecutive entries of row gn of the transpose
                        __bf16* tp = Tout + (size_t)gn * ldt + gm4;
                        if (gm4 + 4 <= M) {
                            bf16x4 w;
                            w[0] = tv[0];
                            w[1] = tv[1];
                            w[2] = tv[2];
                            w[3] = tv[3];
                            *reinterpret_cast<bf16x4*>(tp) = w;
                        } else {
                            for (int r = 0; r < 4 && gm4 + r < M; ++r) tp[r] = tv[r];
                        }
                    }
                }
            }
        return;
    }
    // split K: this block's partial tile
    float* mine = part + (size_t)blockIdx.z * M * N;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int gn = n0 + wn + 32 * j + fr;
            if (gn >= N) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int gm = m0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (gm < M) mine[(size_t)gm * N + gn] = acc[i][j][r];
            }
        }
}

// The split products' sum and epilogue: out(m, n) = sum over z = 0, 1, ... of part[z](m, n) (a fixed order,
// so the same sum on every run), then the epilogue.  32 x 32 tiles, 256 threads: coalesced reads and
// writes, the BF16 values staged in LDS for the transposed copy.
template <int EPI>
__global__ __launch_bounds__(256) void k_splitk_epilogue(const float* __restrict__ part, int splits, int M, int N,
                                                         float* __restrict__ C, int ldc, const float* __restrict__ bias,
                                                         const float* __restrict__ Zin, int ldz,
                                                         __bf16* __restrict__ Hout, int ldh, __bf16* __restrict__ Tout,
                                                         int ldt) {
    __shared__ __bf16 tile[32][33];
    const int n0 = blockIdx.x * 32, m0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const size_t mn = (size_t)M * N;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = ty + 8 * i, gm = m0 + rr, gn = n0 + tx;
        __bf16 tv = (__bf16)0.0f;
        if (gm < M && gn < N) {
            const float* p = part + (size_t)gm * N + gn;
            // left to right over z, four partials loaded ahead of their adds
            float v = 0.f;
            int z = 0;
            for (; z + 4 <= splits; z += 4) {
                const float a0 = p[(size_t)z * mn], a1 = p[(size_t)(z + 1) * mn], a2 = p[(size_t)(z + 2) * mn],
                            a3 = p[(size_t)(z + 3) * mn];
                v += a0;
                v += a1;
                v += a2;
                v += a3;
            }
            for (; z < splits; ++z) v += p[(size_t)z * mn];
            epilogue<EPI>(v, gm, gn, C, ldc, bias, Zin, ldz, Hout, ldh, tv);
        }
        tile[rr][tx] = tv;
    }
    if ((EPI == EPI_BIAS_GELU || EPI == EPI_GELU_GRAD) && Tout != nullptr) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int cc = ty + 8 * i, gn = n0 + cc, gm = m0 + tx;
            if (gn < N && gm < M) Tout[(size_t)gn * ldt + gm] = tile[tx][cc];
        }
    }
}

// softmax over `classes` logits per row, loss sum, G = (p - onehot) / batch as fp32 (g, ld classes),
// bf16 (gb, ld ldgb) and transposed bf16 (gt: classes x batch, ld ldgt, optional)
__global__ void k_softmax_ce(const float* logits, const int32_t* labels, int batch, int classes, float* probs,
                             float* g, __bf16* gb, int ldgb, __bf16* gt, int ldgt, float* loss_sum) {
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
            gb[(size_t)i * ldgb + c] = (__bf16)gv;
            if (gt) gt[(size_t)c * ldgt + i] = (__bf16)gv;
        }
    }
    if (loss_sum && y >= 0 && y < classes) atomicAdd(loss_sum, -(z[y] - m - logf(s)));
}

// column sums: db[n] = sum_i G[i][n]
// Column sums of g (rows x cols, row-major) in a fixed order.  k_colsum_part: a block covers 64
// columns x a slab of COLSUM_SLAB = 64 rows; its four groups of 64 threads each load 16 consecutive
// rows of one column at once (coalesced across the columns), sum them in row order, and the four
// group sums are added in group order.  k_colsum_fin adds the slab sums the same way (four groups
// of consecutive slabs, then the groups in order).
constexpr int COLSUM_SLAB = 64;

__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ g, int rows, int cols,
                                                     float* __restrict__ part) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + lane, r0 = blockIdx.y * COLSUM_SLAB + grp * 16;
    float a[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = (col < cols && r0 + i < rows) ? g[(size_t)(r0 + i) * cols + col] : 0.f;
    float sum = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) sum += a[i];
    red[grp][lane] = sum;
    __syncthreads();
    if (grp == 0 && col < cols)
        part[(size_t)blockIdx.y * cols + col] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

__global__ __launch_bounds__(256) void k_colsum_fin(const float* __restrict__ part, int slabs, int cols,
                                                    float* __restrict__ out) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + lane;
    const int per = (slabs + 3) / 4, z0 = grp * per, z1 = min(slabs, z0 + per);
    float sum = 0.f;
    if (col < cols) {
        int z = z0;
        for (; z + 8 <= z1; z += 8) {
            float a[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = part[(size_t)(z + i) * cols + col];
#pragma unroll
            for (int i = 0; i < 8; ++i) sum += a[i];
        }
        for (; z < z1; ++z) sum += part[(size_t)z * cols + col];
    }
    red[grp][lane] = sum;
    __syncthreads();
    if (grp == 0 && col < cols) out[col] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// x (rows x cols fp32, ld cols) -> y (bf16, ld ldy) and, if t != null, its transpose (cols x rows, ld
// ldt).  64 x 64 tiles through LDS, each thread 4 consecutive values per row: 16-byte loads, 8-byte
// stores in both directions (a row of 64 halves padded to 66 spreads a column read over the banks).
__global__ __launch_bounds__(256) void k_to_bf16_t(const float* __restrict__ x, int rows, int cols,
                                                   __bf16* __restrict__ y, int ldy, __bf16* __restrict__ t, int ldt) {
    __shared__ __bf16 tile[64][66];
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int q = (threadIdx.x & 15) * 4, tr = threadIdx.x >> 4;  // 16 groups of 4 columns x 16 rows
    const bool vec = (cols & 3) == 0 && (ldy & 3) == 0;
    for (int rr = tr; rr < 64; rr += 16) {
        const int r = r0 + rr, c = c0 + q;
        bf16x4 v;
        if (r < rows && vec && c + 4 <= cols) {
            const float4 f = *reinterpret_cast<const float4*>(x + (size_t)r * cols + c);
            v[0] = (__bf16)f.x;
            v[1] = (__bf16)f.y;
            v[2] = (__bf16)f.z;
            v[3] = (__bf16)f.w;
            *reinterpret_cast<bf16x4*>(y + (size_t)r * ldy + c) = v;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                v[e] = (__bf16)0.0f;
                if (r < rows && c + e < cols) {
                    v[e] = (__bf16)x[(size_t)r * cols + c + e];
                    y[(size_t)r * ldy + c + e] = v[e];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) tile[rr][q + e] = v[e];
    }
    if (!t) return;
    __syncthreads();
    const bool tvec = (ldt & 3) == 0;
    for (int cc = tr; cc < 64; cc += 16) {
        const int c = c0 + cc, r = r0 + q;
        if (c >= cols) continue;
        bf16x4 w;
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = tile[q + e][cc];
        if (tvec && r + 4 <= rows) {
            *reinterpret_cast<bf16x4*>(t + (size_t)c * ldt + r) = w;
        } else {
            for (int e = 0; e < 4 && r + e < rows; ++e) t[(size_t)c * ldt + r + e] = w[e];
        }
    }
}

// W (rows x cols fp32, ld cols) -> Wb (bf16, ld ldb) and W^T (bf16, cols x rows, ld ldt)
__global__ __launch_bounds__(256) void k_weights_bf16(const float* __restrict__ w, int rows, int cols,
                                                      __bf16* __restrict__ wb, int ldb, __bf16* __restrict__ wt,
                                                      int ldt) {
    __shared__ __bf16 tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int rr = ty; rr < 32; rr += 8) {
        const int r = r0 + rr, c = c0 + tx;
        __bf16 v = (__bf16)0.0f;
        if (r < rows && c < cols) {
            v = (__bf16)w[(size_t)r * cols + c];
            wb[(size_t)r * ldb + c] = v;
        }
        tile[rr][tx] = v;
    }
    __syncthreads();
    for (int cc = ty; cc < 32; cc += 8) {
        const int c = c0 + cc, r = r0 + tx;
        if (c < cols && r < rows) wt[(size_t)c * ldt + r] = tile[tx][cc];
    }
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

int cu_count() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}

// Tiles of 128 x 128 (four waves of 64 x 64) for the long products with many rows (M and K at least
// 2048), where the larger tile's operand reuse pays; else 64 x 128.  With fewer rows or a short K the
// 128 x 128 grid needs a deeper K split to fill the CUs, and its partials (written, then read back by
// the split sum) cost more than the smaller tile loses: on MI355X the 4096 x 512 x 512 products and the
// 512 x 512 x 4096 weight gradients take 4.7 us less, split sums included, on 64 x 128 tiles.
bool big_tiles(int M, int N, int K) { return M >= 2048 && N >= 128 && K >= 2048; }

int64_t tiles_of(int M, int N, int K) {
    const int bm = big_tiles(M, N, K) ? 128 : 64;
    return (int64_t)((M + bm - 1) / bm) * ((N + BN - 1) / BN);
}

// K is split until the grid holds about two workgroups per CU with 128 x 128 tiles (two fit in LDS and
// registers) or one with 64 x 128 tiles, with at least four K steps (256 k) per workgroup and at most
// 16 splits.
int splits_of(int M, int N, int K) {
    const int64_t tiles = tiles_of(M, N, K);
    const int64_t target = (big_tiles(M, N, K) ? 2 : 1) * (int64_t)cu_count();
    int splits = 1;
    while (splits < 16 && tiles * splits < target && K / (2 * splits) >= 4 * BK) splits *= 2;
    return splits;
}

template <int EPI>
hipError_t gemm_nt_t(const __bf16* A, int lda, const __bf16* B, int ldb, int M, int N, int K, float* C, int ldc,
                     const float* bias, const float* Z, int ldz, __bf16* H, int ldh, __bf16* T, int ldt, float* part,
                     size_t part_floats, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    int splits = splits_of(M, N, K);
    // an epilogue with a transposed BF16 copy always goes through the partial-sum kernel, which
    // transposes through LDS (stored from the MFMA layout, each lane would write its own row of T)
    const bool transposed = (EPI == EPI_BIAS_GELU || EPI == EPI_GELU_GRAD) && T != nullptr;
    bool via_part = splits > 1 || transposed;
    if (via_part && (part == nullptr || part_floats < (size_t)splits * M * N)) {
        splits = 1;  // no workspace: one workgroup per tile, epilogue in the GEMM
        via_part = false;
    }
    const int kchunk = ((K + splits - 1) / splits + BK - 1) / BK * BK;
    if (big_tiles(M, N, K)) {
        dim3 grid((N + BN - 1) / BN, (M + 127) / 128, splits);
        hipLaunchKernelGGL((k_gemm_nt<128, BN, 64, 64, EPI>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, C, ldc,
                           bias, Z, ldz, H, ldh, T, ldt, kchunk, via_part ? part : nullptr);
    } else {
        dim3 grid((N + BN - 1) / BN, (M + 63) / 64, splits);
        hipLaunchKernelGGL((k_gemm_nt<64, BN, 32, 64, EPI>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, C, ldc,
                           bias, Z, ldz, H, ldh, T, ldt, kchunk, via_part ? part : nullptr);
    }
    if (via_part) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        dim3 grid((N + 31) / 32, (M + 31) / 32);
        hipLaunchKernelGGL((k_splitk_epilogue<EPI>), grid, dim3(256), 0, s, part, splits, M, N, C, ldc, bias, Z, ldz,
                           H, ldh, T, ldt);
    }
    return hipGetLastError();
}

}  // namespace

size_t mlp_gemm_part_floats(int M, int N, int K) {
    // splits x M x N partials; M x N when unsplit (epilogues with a transposed copy)
    return (size_t)splits_of(M, N, K) * M * N;
}

size_t mlp_colsum_part_floats(int rows, int cols) {
    return (size_t)((rows + COLSUM_SLAB - 1) / COLSUM_SLAB) * cols;
}

hipError_t mlp_gemm_nt(int epi, const void* A, int lda, const void* B, int ldb, int M, int N, int K, float* C, int ldc,
                       const float* bias, const float* Z, int ldz, void* H, int ldh, void* T, int ldt, float* part,
                       size_t part_floats, hipStream_t s) {
    const __bf16* a = (const __bf16*)A;
    const __bf16* b = (const __bf16*)B;
    __bf16* h = (__bf16*)H;
    __bf16* t = (__bf16*)T;
    switch (epi) {
        case EPI_STORE:
            return gemm_nt_t<EPI_STORE>(a, lda, b, ldb, M, N, K, C, ldc, bias, Z, ldz, h, ldh, t, ldt, part,
                                        part_floats, s);
        case EPI_BIAS:
            return gemm_nt_t<EPI_BIAS>(a, lda, b, ldb, M, N, K, C, ldc, bias, Z, ldz, h, ldh, t, ldt, part,
                                       part_floats, s);
        case EPI_BIAS_GELU:
            return gemm_nt_t<EPI_BIAS_GELU>(a, lda, b, ldb, M, N, K, C, ldc, bias, Z, ldz, h, ldh, t, ldt, part,
                                            part_floats, s);
        case EPI_GELU_GRAD:
            return gemm_nt_t<EPI_GELU_GRAD>(a, lda, b, ldb, M, N, K, C, ldc, bias, Z, ldz, h, ldh, t, ldt, part,
                                            part_floats, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t mlp_softmax_ce(const float* logits, const int32_t* labels, int batch, int classes, float* probs, float* g,
                          void* gb, int ldgb, void* gt, int ldgt, float* loss_sum, hipStream_t s) {
    hipLaunchKernelGGL(k_softmax_ce, dim3((batch + 255) / 256), dim3(256), 0, s, logits, labels, batch, classes, probs,
                       g, (__bf16*)gb, ldgb, (__bf16*)gt, ldgt, loss_sum);
    return hipGetLastError();
}

hipError_t mlp_colsum(const float* g, int rows, int cols, float* out, float* part, size_t part_floats,
                      hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const int slabs = (rows + COLSUM_SLAB - 1) / COLSUM_SLAB;
    if (part == nullptr || part_floats < (size_t)slabs * cols) return hipErrorInvalidValue;
    const unsigned strips = (unsigned)((cols + 63) / 64);
    hipLaunchKernelGGL(k_colsum_part, dim3(strips, (unsigned)slabs), dim3(256), 0, s, g, rows, cols, part);
    hipLaunchKernelGGL(k_colsum_fin, dim3(strips), dim3(256), 0, s, part, slabs, cols, out);
    return hipGetLastError();
}

hipError_t mlp_input_bf16(const float* x, int rows, int cols, void* y, int ldy, void* t, int ldt, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    dim3 grid((cols + 63) / 64, (rows + 63) / 64);
    hipLaunchKernelGGL(k_to_bf16_t, grid, dim3(256), 0, s, x, rows, cols, (__bf16*)y, ldy, (__bf16*)t, ldt);
    return hipGetLastError();
}

hipError_t mlp_weights_bf16(const float* w, int rows, int cols, void* wb, int ldb, void* wt, int ldt, hipStream_t s) {
    dim3 grid((cols + 31) / 32, (rows + 31) / 32);
    hipLaunchKernelGGL(k_weights_bf16, grid, dim3(256), 0, s, w, rows, cols, (__bf16*)wb, ldb, (__bf16*)wt, ldt);
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
