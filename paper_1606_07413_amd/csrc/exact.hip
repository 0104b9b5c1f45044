// Exact channel-representation arithmetic over Z[1/sqrt2] (Sec. 4.1) on the GPU.
//
// A matrix is M = (A + B sqrt2) / sqrt2^e with integer A, B (int64 for n <= 2, int32 for n >= 3)
// and minimal e.  Right multiplication by the channel rep of R(P_p) follows its sparse column
// rule: column q is e_q when <p, q> = 0, else (e_q + s(p, q) e_{p^q}) / sqrt2, so
//   (M R)[:, q] = (M[:, q] + s M[:, p^q]) / sqrt2        (anticommuting q)
//   (M R)[:, q] = (sqrt2 M[:, q]) / sqrt2, (a, b) -> (2b, a)   (commuting q)
// and R^T flips s.  Every kernel here is single-block per matrix: these are set-up and
// verification paths (target preparation, chunk matrices S_c, claw checks), not the walk loop.
#include "common.h"
#include "internal.h"

namespace tcw {

namespace {

template <int NQ>
struct EGeo {
    static constexpr int R = 1 << (2 * NQ);
};

template <typename T>
__device__ inline T lim_of();
template <>
__device__ inline int32_t lim_of<int32_t>() { return (int32_t)1 << 29; }
template <>
__device__ inline int64_t lim_of<int64_t>() { return (int64_t)1 << 60; }

// (A, B, e) <- product with R(seq[0])^(T?) ... ; result left in (a, b).  Whole block cooperates.
template <int NQ, typename T>
__device__ void block_apply(T* a, T* b, T* ta, T* tb, int& e, const uint16_t* seq, const uint8_t* tr, int nseq,
                            int* flag) {
    constexpr int R = EGeo<NQ>::R;
    const T lim = lim_of<T>();
    T *ca = a, *cb = b, *na = ta, *nb = tb;
    for (int s = 0; s < nseq; ++s) {
        const uint32_t p = seq[s];
        const bool t = tr != nullptr && tr[s] != 0;
        for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
            const uint32_t q = idx & (R - 1);
            const int row = idx - (int)q;
            T va, vb;
            if (anticommutes<NQ>(p, q)) {
                int sg = rotation_sign<NQ>(p, q);
                if (t) sg = -sg;
                const int j = row + (int)(q ^ p);
                va = sg > 0 ? ca[idx] + ca[j] : ca[idx] - ca[j];
                vb = sg > 0 ? cb[idx] + cb[j] : cb[idx] - cb[j];
            } else {
                va = cb[idx] * 2;
                vb = ca[idx];
            }
            if (va > lim || va < -lim || vb > lim || vb < -lim) atomicOr(flag, 4);
            na[idx] = va;
            nb[idx] = vb;
        }
        __syncthreads();
        T* x = ca; ca = na; na = x;
        x = cb; cb = nb; nb = x;
        e += 1;
        // reduce: while every a is even, (a + b sqrt2)/sqrt2 = b + (a/2) sqrt2
        while (e > 0) {
            int odd = 0;
            for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) odd |= (int)(ca[idx] & 1);
            if (__syncthreads_or(odd)) break;
            for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
                const T va = ca[idx], vb = cb[idx];
                ca[idx] = vb;
                cb[idx] = va / 2;
            }
            e -= 1;
            __syncthreads();
        }
    }
    if (ca != a) {
        for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
            a[idx] = ca[idx];
            b[idx] = cb[idx];
        }
        __syncthreads();
    }
}

template <int NQ, typename T>
__device__ void block_reduce(T* a, T* b, int& e) {
    constexpr int R = EGeo<NQ>::R;
    while (e > 0) {
        int odd = 0;
        for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) odd |= (int)(a[idx] & 1);
        if (__syncthreads_or(odd)) break;
        for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
            const T va = a[idx], vb = b[idx];
            a[idx] = vb;
            b[idx] = va / 2;
        }
        e -= 1;
        __syncthreads();
    }
}

template <int NQ, typename T>
__global__ __launch_bounds__(1024) void k_identity(T* a, T* b, int32_t* e) {
    constexpr int R = EGeo<NQ>::R;
    for (int idx = threadIdx.x + blockIdx.x * blockDim.x; idx < R * R; idx += blockDim.x * gridDim.x) {
        const int r = idx / R, q = idx % R;
        a[idx] = (r == q) ? 1 : 0;
        b[idx] = 0;
    }
    if (threadIdx.x == 0 && blockIdx.x == 0) *e = 0;
}

template <int NQ, typename T>
__global__ __launch_bounds__(1024) void k_apply(T* a, T* b, T* ta, T* tb, int32_t* e_io, const T* sa, const T* sb,
                                                const int32_t* se, const uint16_t* seq, const uint8_t* tr, int nseq,
                                                int* flag) {
    constexpr int R = EGeo<NQ>::R;
    if (sa != a) {
        for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
            a[idx] = sa[idx];
            b[idx] = sb[idx];
        }
    }
    __syncthreads();
    int e = *se;
    __syncthreads();
    block_apply<NQ, T>(a, b, ta, tb, e, seq, tr, nseq, flag);
    if (threadIdx.x == 0) *e_io = e;
}

template <int NQ, typename T>
__global__ __launch_bounds__(1024) void k_from_i32(T* a, T* b, int32_t* e_io, const int32_t* ia, const int32_t* ib,
                                                   int32_t e0) {
    constexpr int R = EGeo<NQ>::R;
    for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
        a[idx] = (T)ia[idx];
        b[idx] = (T)ib[idx];
    }
    __syncthreads();
    int e = e0;
    block_reduce<NQ, T>(a, b, e);
    if (threadIdx.x == 0) *e_io = e;
}

template <int NQ, typename T>
__global__ void k_to_i32(const T* a, const T* b, int32_t* oa, int32_t* ob, int* flag) {
    constexpr int R = EGeo<NQ>::R;
    for (int idx = threadIdx.x + blockIdx.x * blockDim.x; idx < R * R; idx += blockDim.x * gridDim.x) {
        const T va = a[idx], vb = b[idx];
        if (va > (T)INT32_MAX || va < (T)INT32_MIN || vb > (T)INT32_MAX || vb < (T)INT32_MIN) atomicOr(flag, 4);
        oa[idx] = (int32_t)va;
        ob[idx] = (int32_t)vb;
    }
}

// X X^T = 2^e I with X = A + B sqrt2:  A A^T + 2 B B^T = 2^e I  and  A B^T + B A^T = 0.
template <int NQ, typename T>
__global__ void k_orthogonal(const T* a, const T* b, const int32_t* e_p, int* flag) {
    constexpr int R = EGeo<NQ>::R;
    const int idx = threadIdx.x + blockIdx.x * blockDim.x;
    if (idx >= R * R) return;
    const int i = idx / R, j = idx % R;
    const int e = *e_p;
    int64_t rat = 0, irr = 0;
    for (int k = 0; k < R; ++k) {
        const int64_t ai = a[i * R + k], bi = b[i * R + k], aj = a[j * R + k], bj = b[j * R + k];
        if (ai > (1 << 24) || ai < -(1 << 24) || bi > (1 << 24) || bi < -(1 << 24)) {
            atomicOr(flag, 4);
            return;
        }
        rat += ai * aj + 2 * bi * bj;
        irr += ai * bj + bi * aj;
    }
    const int64_t want = (i == j) ? ((e < 62) ? ((int64_t)1 << e) : -1) : 0;
    if (rat != want || irr != 0) atomicOr(flag, 1);
}

// ---- channel rep of an exact unitary (Sec. 4.1: U_hat_ij = 2^-n Tr(P_i U P_j U^dag)) ----
//
// U = V / sqrt2^e with V over Z[w], w = e^{i pi/4}, each entry four int64 coefficients of
// w^0..w^3 (w^4 = -1).  On the basis |c> (qubit 0 = most significant bit of c), the Pauli
// P_q = (x) sigma(x_j, z_j), sigma(x, z) = i^{xz} X^x Z^z, acts as
//   P_q |c> = i^{|x & z|} (-1)^{|z' & c|} |c ^ x'>,
// with x', z' the bit-reversed masks (qubit j on bit n-1-j).  Hence
//   Tr(P_i V P_j V^dag) = sum_{r,t} w^{k(r,t)} V[r ^ x_i'][t] conj(V[r][t ^ x_j'])
// with k = 2|x_i & z_i| + 4|z_i' & (r ^ x_i')| + 2|x_j & z_j| + 4|z_j' & (t ^ x_j')| (mod 8).
// The trace is real, t0 + t1 w + t2 w^2 + t3 w^3 with t2 = 0 and t3 = -t1, i.e. t0 + t1 sqrt2,
// and U_hat_ij = (t0 + t1 sqrt2) / sqrt2^(2(n + e)).

struct Zw {
    int64_t c[4];
};

__device__ inline Zw zw_load(const int64_t* p) { return Zw{{p[0], p[1], p[2], p[3]}}; }

__device__ inline Zw zw_mul_conj(const Zw& x, const Zw& y) {
    // x * conj(y), conj(y) = y0 - y3 w - y2 w^2 - y1 w^3
    const int64_t yc[4] = {y.c[0], -y.c[3], -y.c[2], -y.c[1]};
    Zw r{{0, 0, 0, 0}};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t v = x.c[i] * yc[j];
            if (i + j < 4) r.c[i + j] += v;
            else r.c[i + j - 4] -= v;
        }
    return r;
}

// acc += w^k x, k in 0..7
__device__ inline void zw_acc_rot(Zw& acc, const Zw& x, int k) {
    const int64_t sg = k >= 4 ? -1 : 1;
    const int kk = k & 3;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = i + kk;
        if (j < 4) acc.c[j] += sg * x.c[i];
        else acc.c[j - 4] -= sg * x.c[i];
    }
}

template <int NQ>
__device__ inline uint32_t bit_reverse_n(uint32_t v) {
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < NQ; ++j) r |= ((v >> j) & 1u) << (NQ - 1 - j);
    return r;
}

// One thread per channel-rep entry (i, j).  flag |= 1 if an entry is not real, 4 if t0 or t1 leaves int32.
template <int NQ>
__global__ __launch_bounds__(256) void k_unitary_channel(const int64_t* v, int32_t* oa, int32_t* ob, int* flag) {
    constexpr int D = 1 << NQ;
    constexpr int R = D * D;
    __shared__ int64_t sv[D * D * 4];
    for (int x = threadIdx.x; x < D * D * 4; x += blockDim.x) sv[x] = v[x];
    __syncthreads();
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= R * R) return;
    const uint32_t i = (uint32_t)idx / R, j = (uint32_t)idx % R;
    const uint32_t xi = i & (D - 1), zi = i >> NQ, xj = j & (D - 1), zj = j >> NQ;
    const uint32_t xir = bit_reverse_n<NQ>(xi), zir = bit_reverse_n<NQ>(zi);
    const uint32_t xjr = bit_reverse_n<NQ>(xj), zjr = bit_reverse_n<NQ>(zj);
    const int k0 = 2 * __builtin_popcount(xi & zi) + 2 * __builtin_popcount(xj & zj);
    Zw acc{{0, 0, 0, 0}};
    for (uint32_t r = 0; r < (uint32_t)D; ++r) {
        const uint32_t s = r ^ xir;
        const int ks = k0 + 4 * __builtin_popcount(zir & s);
        for (uint32_t t = 0; t < (uint32_t)D; ++t) {
            const uint32_t u = t ^ xjr;
            const int k = (ks + 4 * __builtin_popcount(zjr & u)) & 7;
            const Zw prod = zw_mul_conj(zw_load(&sv[(s * D + t) * 4]), zw_load(&sv[(r * D + u) * 4]));
            zw_acc_rot(acc, prod, k);
        }
    }
    if (acc.c[2] != 0 || acc.c[3] != -acc.c[1]) atomicOr(flag, 1);
    if (acc.c[0] > INT32_MAX || acc.c[0] < INT32_MIN || acc.c[1] > INT32_MAX || acc.c[1] < INT32_MIN)
        atomicOr(flag, 4);
    oa[idx] = (int32_t)acc.c[0];
    ob[idx] = (int32_t)acc.c[1];
}

// V V^dag = 2^e I over Z[w], one thread per entry (r, c); flag |= 8 otherwise.
template <int NQ>
__global__ __launch_bounds__(256) void k_unitary_check(const int64_t* v, int32_t e, int* flag) {
    constexpr int D = 1 << NQ;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= D * D) return;
    const int r = idx / D, c = idx % D;
    Zw acc{{0, 0, 0, 0}};
    for (int t = 0; t < D; ++t) {
        const Zw prod = zw_mul_conj(zw_load(&v[(r * D + t) * 4]), zw_load(&v[(c * D + t) * 4]));
        zw_acc_rot(acc, prod, 0);
    }
    const int64_t want = r == c ? ((int64_t)1 << e) : 0;
    if (acc.c[0] != want || acc.c[1] != 0 || acc.c[2] != 0 || acc.c[3] != 0) atomicOr(flag, 8);
}

// Signed permutation test on a reduced matrix: e = 0, B = 0, each column one +-1.
template <int NQ, typename T>
__global__ __launch_bounds__(256) void k_signed_perm(const T* a, const T* b, const int32_t* e_p, int32_t* ok,
                                                     int32_t* perm, int8_t* sign) {
    constexpr int R = EGeo<NQ>::R;
    __shared__ int bad;
    if (threadIdx.x == 0) bad = (*e_p != 0);
    __syncthreads();
    for (int q = threadIdx.x; q < R; q += blockDim.x) {
        int cnt = 0, row = -1, sg = 0;
        for (int i = 0; i < R; ++i) {
            const T va = a[i * R + q], vb = b[i * R + q];
            if (vb != 0) cnt += 2;
            if (va != 0) {
                cnt += 1;
                row = i;
                sg = (va == 1) ? 1 : (va == -1 ? -1 : 0);
            }
        }
        if (cnt != 1 || sg == 0) atomicOr(&bad, 1);
        perm[q] = row;
        sign[q] = (int8_t)sg;
    }
    __syncthreads();
    if (threadIdx.x == 0) *ok = bad ? 0 : 1;
}

// int8 packing of S for the walk kernels: phi[q4 * R + r] = bytes A[r][4 q4 .. 4 q4 + 3] (then B).
// n >= 3 uses the MFMA fragment layout instead: with KK = 2R / 64 K steps and NT = R / 16 tiles,
// dword idx = ((nt * KK + kk) * 64 + l) * 4 + w holds the bytes S''[nt*16 + l%16][kk*64 + (l/16)*16 +
// 4w + c], c = 0..3, with S'' = [A | B] (R x 2R).
template <int NQ, typename T>
__global__ void k_pack_phi(const T* a, const T* b, uint32_t* phi, int* flag) {
    constexpr int R = EGeo<NQ>::R;
    constexpr int Q4 = R / 4;
    const int idx = threadIdx.x + blockIdx.x * blockDim.x;
    if constexpr (NQ >= 3) {
        constexpr int KK = 2 * R / 64;
        if (idx >= 2 * Q4 * R) return;
        const int fi = idx >> 2, w = idx & 3;
        const int l = fi & 63, fk = fi >> 6;
        const int nt = fk / KK, kk = fk % KK;
        const int r = nt * 16 + (l & 15);
        uint32_t word = 0;
        for (int c = 0; c < 4; ++c) {
            const int qq = kk * 64 + (l >> 4) * 16 + 4 * w + c;
            const T v = qq < R ? a[r * R + qq] : b[r * R + qq - R];
            if (v > 127 || v < -127) atomicOr(flag, 2);
            word |= ((uint32_t)(uint8_t)(int8_t)v) << (8 * c);
        }
        phi[idx] = word;
        return;
    }
    if (idx >= Q4 * R) return;
    const int q4 = idx / R, r = idx % R;
    uint32_t wa = 0, wb = 0;
    for (int c = 0; c < 4; ++c) {
        const T va = a[r * R + 4 * q4 + c], vb = b[r * R + 4 * q4 + c];
        if (va > 127 || va < -127 || vb > 127 || vb < -127) atomicOr(flag, 2);
        wa |= ((uint32_t)(uint8_t)(int8_t)va) << (8 * c);
        wb |= ((uint32_t)(uint8_t)(int8_t)vb) << (8 * c);
    }
    phi[idx] = wa;
    phi[Q4 * R + idx] = wb;
}

// Claw check of (u0, u1): V = R(p_0)...R(p_{h-1}) from the side-0 point, W = S R(q_0)^T ... from
// the side-1 point, D = W V^T must be a signed permutation (Sec. 3, last merge case).
template <int NQ, typename T>
__global__ __launch_bounds__(1024) void k_claw(const T* sa, const T* sb, const int32_t* se, int k, const uint64_t* u0,
                                               const uint64_t* u1, int64_t count, T* scratch, int32_t* ok,
                                               int32_t* perm, int8_t* sign) {
    constexpr int R = EGeo<NQ>::R;
    constexpr uint32_t XI = R - 1;
    __shared__ uint16_t seq[64];
    __shared__ uint8_t trs[64];
    __shared__ int cnt[R];
    __shared__ int rowof[R];
    __shared__ int sgn[R];
    __shared__ int bad;
    __shared__ int oflow;
    T* va = scratch + (size_t)blockIdx.x * 6 * R * R;
    T* vb = va + R * R;
    T* wa = vb + R * R;
    T* wb = wa + R * R;
    T* ta = wb + R * R;
    T* tb = ta + R * R;
    const int h = k / 2;
    for (int64_t pi = blockIdx.x; pi < count; pi += gridDim.x) {
        uint64_t p0 = u0[pi], p1 = u1[pi];
        if ((p0 >> 32) & 1) {
            const uint64_t x = p0; p0 = p1; p1 = x;
        }
        const bool sides_ok = (((p0 >> 32) & 1) == 0) && (((p1 >> 32) & 1) == 1);
        // V from the identity
        for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
            va[idx] = ((idx / R) == (idx % R)) ? 1 : 0;
            vb[idx] = 0;
            wa[idx] = sa[idx];
            wb[idx] = sb[idx];
        }
        if (threadIdx.x == 0) {
            uint32_t x = (uint32_t)p0;
            for (int t = 0; t < h; ++t) {
                seq[t] = (uint16_t)(x % XI + 1);
                trs[t] = 0;
                x /= XI;
            }
            bad = sides_ok ? 0 : 1;
            oflow = 0;
        }
        __syncthreads();
        int ev = 0;
        block_apply<NQ, T>(va, vb, ta, tb, ev, seq, trs, h, &oflow);
        if (threadIdx.x == 0) {
            uint32_t x = (uint32_t)p1;
            for (int t = 0; t < h; ++t) {
                seq[t] = (uint16_t)(x % XI + 1);
                trs[t] = 1;
                x /= XI;
            }
        }
        __syncthreads();
        int ew = *se;
        block_apply<NQ, T>(wa, wb, ta, tb, ew, seq, trs, h, &oflow);
        for (int q = threadIdx.x; q < R; q += blockDim.x) {
            cnt[q] = 0;
            rowof[q] = -1;
            sgn[q] = 0;
        }
        __syncthreads();
        // D_iq = sum_k W_ik V_qk with exponent E = ew + ev; a unit entry is +-sqrt2^E
        const int E = ew + ev;
        const int64_t unit = (int64_t)1 << (E / 2);
        for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
            const int i = idx / R, q = idx % R;
            int64_t da = 0, db = 0;
            for (int kk = 0; kk < R; ++kk) {
                const int64_t xa = wa[i * R + kk], xb = wb[i * R + kk];
                const int64_t ya = va[q * R + kk], yb = vb[q * R + kk];
                da += xa * ya + 2 * xb * yb;
                db += xa * yb + xb * ya;
            }
            if (da != 0 || db != 0) {
                atomicAdd(&cnt[q], 1);
                int s = 0;
                if (E % 2 == 0) {
                    if (db == 0 && (da == unit || da == -unit)) s = da > 0 ? 1 : -1;
                } else {
                    if (da == 0 && (db == unit || db == -unit)) s = db > 0 ? 1 : -1;
                }
                if (s == 0) atomicOr(&bad, 1);
                rowof[q] = i;
                sgn[q] = s;
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < R; q += blockDim.x) {
            if (cnt[q] != 1) atomicOr(&bad, 1);
        }
        __syncthreads();
        const int good = (bad == 0 && oflow == 0) ? 1 : 0;
        for (int q = threadIdx.x; q < R; q += blockDim.x) {
            perm[pi * R + q] = good ? rowof[q] : -1;
            sign[pi * R + q] = (int8_t)(good ? sgn[q] : 0);
        }
        if (threadIdx.x == 0) ok[pi] = good;
        __syncthreads();
    }
}

// Canonical FP32 features of the exact matrix (a, b, e) held by the block (n <= 3): rows
// sign-normalised (first nonzero entry positive, decided exactly), sorted lexicographically as the
// integer sequences (a_0, b_0, a_1, b_1, ...), each entry (a + b sqrt2) 2^(-e/2) formed in double as
// t = a + b * SQRT2, t *= SQRT1_2 for odd e, t *= 2^(-floor(e/2)), rounded to float.
template <int NQ, typename T>
__device__ void block_features(const T* a, const T* b, int e, int32_t* rows /* R x 2R shared */,
                               int32_t* idx /* R shared */, float* out) {
    constexpr int R = EGeo<NQ>::R;
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        int sg = 0;
        for (int q = 0; q < R && sg == 0; ++q) {
            const int64_t va = a[r * R + q], vb = b[r * R + q];
            if (va == 0 && vb == 0) continue;
            if (va >= 0 && vb >= 0) sg = 1;
            else if (va <= 0 && vb <= 0) sg = -1;
            else if (va > 0) sg = (va * va > 2 * vb * vb) ? 1 : -1;
            else sg = (2 * vb * vb > va * va) ? 1 : -1;
        }
        if (sg == 0) sg = 1;
        for (int q = 0; q < R; ++q) {
            rows[r * 2 * R + 2 * q] = (int32_t)(sg * a[r * R + q]);
            rows[r * 2 * R + 2 * q + 1] = (int32_t)(sg * b[r * R + q]);
        }
        idx[r] = r;
    }
    __syncthreads();
    // bitonic sort of the row indices by lexicographic row order
    for (int k = 2; k <= R; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < R; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const int ri = idx[i], rl = idx[l];
                    int cmp = 0;
                    for (int c = 0; c < 2 * R && cmp == 0; ++c) {
                        const int32_t x = rows[ri * 2 * R + c], y = rows[rl * 2 * R + c];
                        cmp = (x < y) ? -1 : (x > y ? 1 : 0);
                    }
                    const bool asc = (i & k) == 0;
                    if ((asc && cmp > 0) || (!asc && cmp < 0)) {
                        idx[i] = rl;
                        idx[l] = ri;
                    }
                }
            }
            __syncthreads();
        }
    }
    const double sqrt2 = 1.4142135623730951, sqrt1_2 = 0.7071067811865476;
    const double scale = ldexp(1.0, -(e / 2));
    for (int t = threadIdx.x; t < R * R; t += blockDim.x) {
        const int i = t / R, q = t % R;
        const int r = idx[i];
        double v = __dadd_rn((double)rows[r * 2 * R + 2 * q], __dmul_rn((double)rows[r * 2 * R + 2 * q + 1], sqrt2));
        if (e & 1) v = __dmul_rn(v, sqrt1_2);
        out[t] = (float)__dmul_rn(v, scale);
    }
    __syncthreads();
}

template <int NQ, typename T>
__global__ __launch_bounds__(256) void k_features(const T* a, const T* b, const int32_t* e, float* out) {
    constexpr int R = EGeo<NQ>::R;
    __shared__ int32_t rows[R * 2 * R];
    __shared__ int32_t idx[R];
    block_features<NQ, T>(a, b, *e, rows, idx, out);
}

// Network data: targets built exactly from their words (Clifford word then rotations), packed as
// int8 for the walk step (n <= 3 layout) and turned into canonical features.  One block per target.
template <int NQ, typename T>
__global__ __launch_bounds__(1024) void k_build_batch(const uint16_t* words, const int32_t* offsets,
                                                      const int32_t* kof, int count, T* scratch, uint32_t* phi_out,
                                                      int32_t* rot_e_out, float* feat_out, int* flag) {
    constexpr int R = EGeo<NQ>::R;
    constexpr int Q4 = R / 4;
    __shared__ uint16_t seq[256];
    __shared__ int32_t rows[R * 2 * R];
    __shared__ int32_t idx[R];
    T* a = scratch + (size_t)blockIdx.x * 4 * R * R;
    T* b = a + R * R;
    T* ta = b + R * R;
    T* tb = ta + R * R;
    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        const int w0 = offsets[t], w1 = offsets[t + 1], k = kof[t];
        const int m = w1 - w0 - k;
        int nseq = 2 * m + k;
        if (nseq > 256) {
            if (threadIdx.x == 0) atomicOr(flag, 8);
            nseq = 0;
        }
        if (threadIdx.x == 0 && nseq > 0) {
            int s = 0;
            for (int j = 0; j < m; ++j) {
                seq[s++] = words[w0 + k + j];
                seq[s++] = words[w0 + k + j];
            }
            for (int j = k - 1; j >= 0; --j) seq[s++] = words[w0 + j];
        }
        for (int i = threadIdx.x; i < R * R; i += blockDim.x) {
            a[i] = (i / R == i % R) ? 1 : 0;
            b[i] = 0;
        }
        __syncthreads();
        int e = 0;
        block_apply<NQ, T>(a, b, ta, tb, e, seq, nullptr, nseq, flag);
        if constexpr (NQ == 3) {
            // MFMA fragment layout (as k_pack_phi for n >= 3)
            constexpr int KK = 2 * R / 64;
            for (int i = threadIdx.x; i < 2 * Q4 * R; i += blockDim.x) {
                const int fi = i >> 2, w = i & 3;
                const int l = fi & 63, fk = fi >> 6;
                const int nt = fk / KK, kk = fk % KK;
                const int r = nt * 16 + (l & 15);
                uint32_t word = 0;
                for (int c = 0; c < 4; ++c) {
                    const int qq = kk * 64 + (l >> 4) * 16 + 4 * w + c;
                    const T v = qq < R ? a[r * R + qq] : b[r * R + qq - R];
                    if (v > 127 || v < -127) atomicOr(flag, 2);
                    word |= ((uint32_t)(uint8_t)(int8_t)v) << (8 * c);
                }
                phi_out[(size_t)t * 2 * Q4 * R + i] = word;
            }
        } else {
            for (int i = threadIdx.x; i < Q4 * R; i += blockDim.x) {
                const int q4 = i / R, r = i % R;
                uint32_t wa = 0, wb = 0;
                for (int c = 0; c < 4; ++c) {
                    const T va = a[r * R + 4 * q4 + c], vb = b[r * R + 4 * q4 + c];
                    if (va > 127 || va < -127 || vb > 127 || vb < -127) atomicOr(flag, 2);
                    wa |= ((uint32_t)(uint8_t)(int8_t)va) << (8 * c);
                    wb |= ((uint32_t)(uint8_t)(int8_t)vb) << (8 * c);
                }
                phi_out[(size_t)t * 2 * Q4 * R + i] = wa;
                phi_out[(size_t)t * 2 * Q4 * R + Q4 * R + i] = wb;
            }
        }
        if (threadIdx.x == 0) rot_e_out[t] = (int32_t)((30ll * e) % 61);
        block_features<NQ, T>(a, b, e, rows, idx, feat_out + (size_t)t * R * R);
    }
}

template <typename F>
hipError_t dispatch_exact(int n, F&& f) {
    switch (n) {
        case 1: return f.template operator()<1, int64_t>();
        case 2: return f.template operator()<2, int64_t>();
        case 3: return f.template operator()<3, int32_t>();
        case 4: return f.template operator()<4, int32_t>();
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t exact_alloc(ExactDev& m, int n) {
    m.n = n;
    m.r = 1 << (2 * n);
    m.elem = n <= 2 ? 8 : 4;
    const size_t bytes = (size_t)m.r * m.r * m.elem;
    hipError_t err = hipMalloc(&m.a, bytes);
    if (err == hipSuccess) err = hipMalloc(&m.b, bytes);
    if (err == hipSuccess) err = hipMalloc(&m.e, sizeof(int32_t));
    return err;
}

void exact_free(ExactDev& m) {
    if (m.a) (void)hipFree(m.a);
    if (m.b) (void)hipFree(m.b);
    if (m.e) (void)hipFree(m.e);
    m.a = m.b = nullptr;
    m.e = nullptr;
}

namespace {
struct ScratchPair {
    void* ta = nullptr;
    void* tb = nullptr;
};
hipError_t scratch_pair(const ExactDev& m, ScratchPair& sp) {
    const size_t bytes = (size_t)m.r * m.r * m.elem;
    hipError_t err = hipMalloc(&sp.ta, bytes);
    if (err == hipSuccess) err = hipMalloc(&sp.tb, bytes);
    return err;
}
void scratch_free(ScratchPair& sp) {
    if (sp.ta) (void)hipFree(sp.ta);
    if (sp.tb) (void)hipFree(sp.tb);
}
}  // namespace

hipError_t exact_apply_ws(ExactDev& dst, const ExactDev& src, const uint16_t* seq, const uint8_t* tr, int nseq,
                          void* ta, void* tb, int* flag, hipStream_t s) {
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        hipLaunchKernelGGL((k_apply<NQ, T>), dim3(1), dim3(1024), 0, s, (T*)dst.a, (T*)dst.b, (T*)ta, (T*)tb, dst.e,
                           (const T*)src.a, (const T*)src.b, src.e, seq, tr, nseq, flag);
        return hipGetLastError();
    };
    return dispatch_exact(dst.n, f);
}

hipError_t exact_apply(ExactDev& dst, const ExactDev& src, const uint16_t* seq, const uint8_t* tr, int nseq,
                       int* flag, hipStream_t s) {
    ScratchPair sp;
    hipError_t err = scratch_pair(dst, sp);
    if (err != hipSuccess) {
        scratch_free(sp);
        return err;
    }
    err = exact_apply_ws(dst, src, seq, tr, nseq, sp.ta, sp.tb, flag, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    scratch_free(sp);
    return err;
}

namespace {
// One rotation on many blocks (the chunk matrix S_c = U R(c)^T), in two passes with no work matrices.
// Pass 1 writes (A', B') = the rotated columns of (src.A, src.B) into dst and folds into *m_min the
// number of reduction steps each entry allows: a step (a, b) -> (b, a / 2) needs a even, so from
// (a, b) the steps alternate the conditions 2 | a, 2 | b, 4 | a, 4 | b, ... and entry (a, b) allows
// min(2 v2(a), 2 v2(b) + 1) of them (v2 = 2-adic valuation, unbounded for 0).  Pass 2 takes
// m = min(*m_min, e + 1) steps in closed form, as block_apply's loop would: after 2j steps
// (a, b) / 2^j, after 2j + 1 steps (b / 2^j, a / 2^(j + 1)).
template <typename T>
__device__ inline int v2_of(T v) {
    if (v == 0) return 1 << 20;
    return (int)__builtin_ctzll((unsigned long long)v);
}

template <int NQ, typename T>
__global__ __launch_bounds__(256) void k_rotate1(T* a, T* b, const T* sa, const T* sb, uint32_t p, int transposed,
                                                int* flag, int32_t* m_min) {
    constexpr int R = EGeo<NQ>::R;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    int m = 1 << 30;
    if (idx < R * R) {
        const uint32_t q = idx & (R - 1);
        const int row = idx - (int)q;
        T va, vb;
        if (anticommutes<NQ>(p, q)) {
            int sg = rotation_sign<NQ>(p, q);
            if (transposed) sg = -sg;
            const int j = row + (int)(q ^ p);
            va = sg > 0 ? sa[idx] + sa[j] : sa[idx] - sa[j];
            vb = sg > 0 ? sb[idx] + sb[j] : sb[idx] - sb[j];
        } else {
            va = sb[idx] * 2;
            vb = sa[idx];
        }
        const T lim = lim_of<T>();
        if (va > lim || va < -lim || vb > lim || vb < -lim) atomicOr(flag, 4);
        a[idx] = va;
        b[idx] = vb;
        const int ma = 2 * v2_of(va), mb = 2 * v2_of(vb) + 1;
        m = ma < mb ? ma : mb;
    }
    // the wavefront's least, then one atomic per wavefront
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(m, off);
        m = o < m ? o : m;
    }
    if ((threadIdx.x & 63) == 0 && m < (1 << 30)) atomicMin(m_min, m);
}

template <int NQ, typename T>
__global__ __launch_bounds__(256) void k_rotate1_reduce(T* a, T* b, int32_t* e_io, const int32_t* se,
                                                       const int32_t* m_min) {
    constexpr int R = EGeo<NQ>::R;
    const int e1 = *se + 1;
    const int m = *m_min < e1 ? *m_min : e1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < R * R && m > 0) {
        const T va = a[idx], vb = b[idx];
        const int j = m >> 1;
        if (m & 1) {
            a[idx] = vb / ((T)1 << j);
            b[idx] = va / ((T)1 << (j + 1));
        } else {
            a[idx] = va / ((T)1 << j);
            b[idx] = vb / ((T)1 << j);
        }
    }
    if (idx == 0) *e_io = e1 - m;
}

__global__ void k_seq_one(uint16_t* seq, uint8_t* tr, uint16_t p, uint8_t t) {
    if (threadIdx.x == 0) {
        seq[0] = p;
        tr[0] = t;
    }
}
__global__ void k_fill_i32(int* dst, int v, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = v;
}
}  // namespace

hipError_t exact_rotate1(ExactDev& dst, const ExactDev& src, uint32_t p, int transposed, int32_t* m_tmp, int* flag,
                         hipStream_t s) {
    if (dst.a == src.a || dst.b == src.b) return hipErrorInvalidValue;
    hipError_t err = fill_i32(m_tmp, 1 << 30, 1, s);
    if (err != hipSuccess) return err;
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        constexpr int R = EGeo<NQ>::R;
        const int blocks = (R * R + 255) / 256;
        hipLaunchKernelGGL((k_rotate1<NQ, T>), dim3(blocks), dim3(256), 0, s, (T*)dst.a, (T*)dst.b, (const T*)src.a,
                           (const T*)src.b, p, transposed, flag, m_tmp);
        hipLaunchKernelGGL((k_rotate1_reduce<NQ, T>), dim3(blocks), dim3(256), 0, s, (T*)dst.a, (T*)dst.b, dst.e,
                           src.e, m_tmp);
        return hipGetLastError();
    };
    return dispatch_exact(dst.n, f);
}

hipError_t exact_seq_one(uint16_t* seq, uint8_t* tr, uint16_t p, uint8_t transpose, hipStream_t s) {
    hipLaunchKernelGGL(k_seq_one, dim3(1), dim3(64), 0, s, seq, tr, p, transpose);
    return hipGetLastError();
}

hipError_t fill_i32(int* dst, int v, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, dst, v, count);
    return hipGetLastError();
}

hipError_t exact_build(ExactDev& m, const uint16_t* seq, const uint8_t* tr, int nseq, int* flag, hipStream_t s) {
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        hipLaunchKernelGGL((k_identity<NQ, T>), dim3(64), dim3(1024), 0, s, (T*)m.a, (T*)m.b, m.e);
        return hipGetLastError();
    };
    hipError_t err = dispatch_exact(m.n, f);
    if (err != hipSuccess) return err;
    return exact_apply(m, m, seq, tr, nseq, flag, s);
}

hipError_t exact_from_i32(ExactDev& m, const int32_t* a, const int32_t* b, int32_t e, int* flag, hipStream_t s) {
    (void)flag;
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        hipLaunchKernelGGL((k_from_i32<NQ, T>), dim3(1), dim3(1024), 0, s, (T*)m.a, (T*)m.b, m.e, a, b, e);
        return hipGetLastError();
    };
    return dispatch_exact(m.n, f);
}

hipError_t exact_from_unitary(ExactDev& m, const int64_t* v, int32_t e, int32_t* a_tmp, int32_t* b_tmp, int* flag,
                              hipStream_t s) {
    const int n = m.n;
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        constexpr int D = 1 << NQ;
        constexpr int R = D * D;
        hipLaunchKernelGGL((k_unitary_check<NQ>), dim3((D * D + 255) / 256), dim3(256), 0, s, v, e, flag);
        hipLaunchKernelGGL((k_unitary_channel<NQ>), dim3((R * R + 255) / 256), dim3(256), 0, s, v, a_tmp, b_tmp,
                           flag);
        return hipGetLastError();
    };
    hipError_t err = dispatch_exact(n, f);
    if (err != hipSuccess) return err;
    return exact_from_i32(m, a_tmp, b_tmp, 2 * (n + e), flag, s);
}

hipError_t exact_to_i32(const ExactDev& m, int32_t* a, int32_t* b, int* flag, hipStream_t s) {
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        hipLaunchKernelGGL((k_to_i32<NQ, T>), dim3(64), dim3(1024), 0, s, (const T*)m.a, (const T*)m.b, a, b,
                           flag);
        return hipGetLastError();
    };
    return dispatch_exact(m.n, f);
}

hipError_t exact_check_orthogonal(const ExactDev& m, int* flag, hipStream_t s) {
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        constexpr int R = 1 << (2 * NQ);
        hipLaunchKernelGGL((k_orthogonal<NQ, T>), dim3((R * R + 255) / 256), dim3(256), 0, s, (const T*)m.a,
                           (const T*)m.b, m.e, flag);
        return hipGetLastError();
    };
    return dispatch_exact(m.n, f);
}

hipError_t exact_signed_perm(const ExactDev& m, int32_t* ok, int32_t* perm, int8_t* sign, hipStream_t s) {
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        hipLaunchKernelGGL((k_signed_perm<NQ, T>), dim3(1), dim3(256), 0, s, (const T*)m.a, (const T*)m.b, m.e,
                           ok, perm, sign);
        return hipGetLastError();
    };
    return dispatch_exact(m.n, f);
}

hipError_t exact_pack_phi(const ExactDev& m, uint32_t* phi, int* flag, hipStream_t s) {
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        constexpr int R = 1 << (2 * NQ);
        const int nthr = NQ >= 3 ? R / 2 * R : R / 4 * R;
        hipLaunchKernelGGL((k_pack_phi<NQ, T>), dim3((nthr + 255) / 256), dim3(256), 0, s, (const T*)m.a,
                           (const T*)m.b, phi, flag);
        return hipGetLastError();
    };
    return dispatch_exact(m.n, f);
}

size_t exact_claw_scratch_bytes(int n) {
    const size_t r = (size_t)1 << (2 * n);
    const size_t elem = n <= 2 ? 8 : 4;
    return 16 * 6 * r * r * elem;  // 16 blocks, 6 matrices of R x R each
}

hipError_t exact_claw_check(const ExactDev& S, int k, const uint64_t* u0, const uint64_t* u1, int64_t count,
                            void* scratch, size_t scratch_bytes, int32_t* ok, int32_t* perm, int8_t* sign,
                            hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (scratch_bytes < exact_claw_scratch_bytes(S.n)) return hipErrorInvalidValue;
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        const int blocks = (int)(count < 16 ? count : 16);
        hipLaunchKernelGGL((k_claw<NQ, T>), dim3(blocks), dim3(1024), 0, s, (const T*)S.a, (const T*)S.b, S.e, k,
                           u0, u1, count, (T*)scratch, ok, perm, sign);
        return hipGetLastError();
    };
    return dispatch_exact(S.n, f);
}

}  // namespace tcw

namespace tcw {

hipError_t exact_features(const ExactDev& m, float* out, hipStream_t s) {
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        if constexpr (NQ <= 3) {
            hipLaunchKernelGGL((k_features<NQ, T>), dim3(1), dim3(256), 0, s, (const T*)m.a, (const T*)m.b, m.e, out);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    };
    return dispatch_exact(m.n, f);
}

size_t build_batch_scratch_bytes(int n, int blocks) {
    const size_t r = (size_t)1 << (2 * n);
    return (size_t)blocks * 4 * r * r * (n <= 2 ? 8 : 4);
}

hipError_t build_batch(int n, const uint16_t* words, const int32_t* offsets, const int32_t* kof, int count,
                       void* scratch, int blocks, uint32_t* phi_out, int32_t* rot_e_out, float* feat_out, int* flag,
                       hipStream_t s) {
    auto f = [&]<int NQ, typename T>() -> hipError_t {
        if constexpr (NQ <= 3) {
            hipLaunchKernelGGL((k_build_batch<NQ, T>), dim3(blocks), dim3(1024), 0, s, words, offsets, kof, count,
                               (T*)scratch, phi_out, rot_e_out, feat_out, flag);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    };
    return dispatch_exact(n, f);
}

}  // namespace tcw
