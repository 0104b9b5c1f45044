// The walk step of the deterministic-walk claw search (Sec. 2 and Sec. 3) on gfx950.
//
// One walk is owned by a group of G = min(4^n, 64) lanes of one wavefront; lane gl holds the
// RPL = 4^n / G consecutive rows r = gl * RPL + j.  A step f(x, b) computes the matrix hash of
//   side 0: M = R(p_0) ... R(p_{h-1}),   side 1: M = S_c R(p_0)^T ... R(p_{h-1})^T
// (channel representations; p_j = base-xi digit j of x, plus one).  The hash needs only the row
// digests S_r = sum_q K[q] phi(M_rq) in Z/p, p = 2^61 - 1, phi(sqrt2) = 2^31, i.e. the vector
// phi(M) K.  By associativity that vector is computed without forming M:
//   side 0: S = R(p_0) (R(p_1) ( ... (R(p_{h-1}) K)))
//   side 1: S = phi(S_c) u,  u = R(p_0)^T ( ... (R(p_{h-1})^T K))
// Each factor touches the vector by the channel rep's column rule (one butterfly per
// anticommuting row; the 1/sqrt2 is a 61-bit rotation by 30); at n = 4 the first two factors
// applied to K come from a table of rotated keys built once per search seed (2 x 256^2 vectors of
// 256 values), so a step reads one row of it and applies the remaining h - 2.  The side-1 product
// with the fixed chunk matrix S_c = (A + B sqrt2)/sqrt2^e runs on int8 MFMA for n >= 3 (A and B in
// LDS as B-operand fragments, against signed base-256 digits of u and 2^31 u) and on int8 dot
// products (v_dot4_i32_i8) against 7-bit limbs of u for n <= 2.  At n = 4 a wavefront runs two
// walks, and when both next points are on side 1 one pass of the MFMAs serves both steps.  Then (nu + h of Sec. 2):
//   D_r = min(S_r, p - S_r)   (sign-normalised row: negating a row negates S_r)
//   H = mix64(sum_r g(D_r))   (mod 2^64: an additive multiset hash, so the order of the rows -- a
//                               left signed permutation -- drops out), with the element map
//   g(D) = ((D mod 2^32 + a) mod 2^32) ((D div 2^32 + b) mod 2^32),  a, b the halves of salt_h
//   (NH of Black, Halevi, Krawczyk, Krovetz and Rogaway, UMAC, CRYPTO 1999, on the digest's two
//   32-bit words: one 32 x 32 -> 64-bit product per row)
//   f(x, b) = (floor(H * xi^h / 2^64), H mod 2)                    (reduction back to a point)
#include "common.h"
#include "internal.h"

namespace tcw {

namespace {

template <int NQ>
struct Geo {
    static constexpr int R = 1 << (2 * NQ);
    static constexpr uint32_t XI = (uint32_t)R - 1;
    static constexpr int G = R < 64 ? R : 64;       // lanes per walk
    static constexpr int RPL = R / G;               // rows per lane (1 or 4)
    static constexpr int LRPL = RPL == 4 ? 2 : 0;
    static constexpr int WPW = 64 / G;              // walks per wavefront
    static constexpr int Q4 = R / 4;                // 4-column groups
    // most rotations per half with xi^h < 2^32
    static constexpr int HMAX = NQ == 1 ? 20 : (NQ == 2 ? 8 : (NQ == 3 ? 5 : 4));
};

typedef int v4i __attribute__((ext_vector_type(4)));

// n <= 2: S_c as int8 dwords [q/4][r] for v_dot4; per-walk limb buffer [q/4][limb].
template <int NQ, int WAVES>
struct Lds {
    uint32_t phiA[Geo<NQ>::Q4 * Geo<NQ>::R];
    uint32_t phiB[Geo<NQ>::Q4 * Geo<NQ>::R];
    uint64_t K[Geo<NQ>::R];
    uint32_t limbs[WAVES * Geo<NQ>::WPW][Geo<NQ>::Q4 * LIMB_STRIDE];
};

// n = 4: S_c as MFMA B-operand fragments.  With K stacked as [A | B] (512 columns), fragment
// (nt, kk) holds, for lane l, the 16 bytes S''[nt*16 + l%16][kk*64 + (l/16)*16 + 0..15] where
// S''[r][q] = A[r][q] for q < 256 and B[r][q - 256] otherwise; one ds_read_b128 per lane per MFMA.
// Per walk: digit rows [8][68] (signed base-256 digits of the rotated key vector, 4 columns per
// dword; the row stride of 68 dwords keeps the MFMA A-operand reads free of bank conflicts).
constexpr int N4_NT = 16, N4_KK = 8, N4_ROW = 68;
constexpr int N4_DIG = 8;  // signed base-256 digits of a residue below 2^62
template <int WAVES>
struct Lds<4, WAVES> {
    v4i frag[N4_NT * N4_KK * 64];
    uint64_t K[256];
    uint32_t limbs[WAVES][N4_DIG * N4_ROW];
    alignas(16) uint32_t zero_row[N4_ROW];  // A-operand rows 8..15 (no digit) read this
};

// n = 3: S_c as MFMA B-operand fragments in the same layout with KK = 2 K steps and NT = 4 tiles;
// per walk (one per wavefront, lane l holds row l): digit rows [8][20] (64 bytes, one per column,
// plus padding).
constexpr int N3_NT = 4, N3_KK = 2, N3_ROW = 20;
template <int WAVES>
struct Lds<3, WAVES> {
    v4i frag[N3_NT * N3_KK * 64];
    uint64_t K[64];
    uint32_t limbs[WAVES][N4_DIG * N3_ROW];
    alignas(16) uint32_t zero_row[N3_ROW];
};

// A value every lane of the wavefront holds (the walk of a whole wavefront), made explicitly uniform.
__device__ inline uint64_t uniform64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint32_t uniform32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NQ, int WAVES>
__device__ void load_lds(Lds<NQ, WAVES>& L, const SpaceDev& sp) {
    using Gm = Geo<NQ>;
    constexpr int NPHI = Gm::Q4 * Gm::R;
    if constexpr (NQ == 4) {
        const v4i* src = reinterpret_cast<const v4i*>(sp.phi);
        for (int i = threadIdx.x; i < N4_NT * N4_KK * 64; i += blockDim.x) L.frag[i] = src[i];
        for (int i = threadIdx.x; i < N4_ROW; i += blockDim.x) L.zero_row[i] = 0;
    } else if constexpr (NQ == 3) {
        const v4i* src = reinterpret_cast<const v4i*>(sp.phi);
        for (int i = threadIdx.x; i < N3_NT * N3_KK * 64; i += blockDim.x) L.frag[i] = src[i];
        for (int i = threadIdx.x; i < N3_ROW; i += blockDim.x) L.zero_row[i] = 0;
    } else {
        for (int i = threadIdx.x; i < NPHI; i += blockDim.x) {
            L.phiA[i] = sp.phi[i];
            L.phiB[i] = sp.phi[NPHI + i];
        }
    }
    for (int i = threadIdx.x; i < Gm::R; i += blockDim.x) L.K[i] = sp.keys[i];
}

// a 64-bit value moved by one DPP pattern (every source lane inside the wave: quad permutes, row
// rotations)
template <int CTRL>
__device__ inline uint64_t dpp64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, true);
    return ((uint64_t)hi << 32) | lo;
}

// x * 2^s mod p for a lane-dependent 0 <= s < 61 (x in [0, p])
__device__ inline uint64_t m61_rotv(uint64_t x, uint32_t s) {
    return ((x << s) | (x >> (61 - s))) & P61;
}

// sum_i acc_i 2^(7 i) mod p for nine signed limb sums |acc_i| < 2^24, exactly: the low five and
// the high four limbs are combined in 64-bit integers, then reduced.
__device__ inline uint64_t limbs_to_m61(const int32_t* acc) {
    uint64_t lo = 0, hi = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) lo += (uint64_t)(int64_t)acc[i] << (7 * i);
#pragma unroll
    for (int i = 5; i < NLIMB; ++i) hi += (uint64_t)(int64_t)acc[i] << (7 * (i - 5));
    // |lo| < 2^53, |hi| < 2^46: adding 4p keeps the exact value positive and below 2^64
    const uint64_t l = m61_fold(lo + 4 * P61), hh = m61_fold(hi + 4 * P61);
    return m61_add(l, m61_rot(hh, 35));
}

// Cross-half exchanges without LDS (gfx950 v_permlane32_swap / v_permlane16_swap).  permlane32_swap
// exchanges lanes 32..63 of its first operand with lanes 0..31 of its second; permlane16_swap the
// odd 16-lane rows of the first with the even rows of the second.  So half_add32(x, y) leaves lanes
// 0..31 with x + x(lane + 32) and lanes 32..63 with y(lane - 32) + y; half_add16 likewise within
// each 32-lane half (rows 0, 2 get x + x(lane + 16), rows 1, 3 get y(lane - 16) + y).
// half_addNN(v, v) is v + v(lane ^ NN) in every lane.
// The halves are joined into a register pair before the add (an empty asm the compiler cannot see
// through), so the sum is one 64-bit add rather than a split low add, carry and high add.
__device__ inline uint64_t join64(uint32_t lo, uint32_t hi) {
    uint64_t v = ((uint64_t)hi << 32) | lo;
    asm("" : "+v"(v));
    return v;
}
__device__ inline uint64_t half_add32(uint64_t x, uint64_t y) {
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)x, (uint32_t)y, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(x >> 32), (uint32_t)(y >> 32), false, false);
    return join64(lo[0], hi[0]) + join64(lo[1], hi[1]);
}
__device__ inline uint64_t half_add16(uint64_t x, uint64_t y) {
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)x, (uint32_t)y, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(x >> 32), (uint32_t)(y >> 32), false, false);
    return join64(lo[0], hi[0]) + join64(lo[1], hi[1]);
}
// 32-bit version: x + x(lane + 32) in lanes 0..31, y(lane - 32) + y in lanes 32..63.
__device__ inline int32_t half_add32_i32(int32_t x, int32_t y) {
    const auto v = __builtin_amdgcn_permlane32_swap((uint32_t)x, (uint32_t)y, false, false);
    return (int32_t)(v[0] + v[1]);
}

// n <= 2: phi(S_c) u with v_dot4_i32_i8 on A, B (int8, LDS) and 7-bit limbs of u.
template <int NQ, int WAVES>
__device__ inline void side1_dot4(const Lds<NQ, WAVES>& L, uint32_t* limbs, const uint64_t* u, int gl, int rot_e,
                                  uint64_t* S) {
    using Gm = Geo<NQ>;
    constexpr int R = Gm::R, RPL = Gm::RPL, Q4 = Gm::Q4;
    // 7-bit limbs of u, four columns per dword, into this group's LDS slot
    if constexpr (RPL == 4) {
#pragma unroll
        for (int i = 0; i < NLIMB; ++i) {
            uint32_t dw = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) dw |= (uint32_t)((u[j] >> (7 * i)) & 127) << (8 * j);
            limbs[gl * LIMB_STRIDE + i] = dw;
        }
    } else {
        uint8_t* lb = reinterpret_cast<uint8_t*>(limbs);
#pragma unroll
        for (int i = 0; i < NLIMB; ++i)
            lb[((gl >> 2) * LIMB_STRIDE + i) * 4 + (gl & 3)] = (uint8_t)((u[0] >> (7 * i)) & 127);
    }
    wave_sync();
    int32_t accA[RPL][NLIMB], accB[RPL][NLIMB];
#pragma unroll
    for (int j = 0; j < RPL; ++j)
#pragma unroll
        for (int i = 0; i < NLIMB; ++i) accA[j][i] = accB[j][i] = 0;
#pragma unroll 2
    for (int q4 = 0; q4 < Q4; ++q4) {
        uint32_t U[NLIMB];
#pragma unroll
        for (int i = 0; i < NLIMB; ++i) U[i] = limbs[q4 * LIMB_STRIDE + i];
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            const int a = (int)L.phiA[q4 * R + gl * RPL + j];
            const int b = (int)L.phiB[q4 * R + gl * RPL + j];
#pragma unroll
            for (int i = 0; i < NLIMB; ++i) {
                accA[j][i] = __builtin_amdgcn_sdot4(a, (int)U[i], accA[j][i], false);
                accB[j][i] = __builtin_amdgcn_sdot4(b, (int)U[i], accB[j][i], false);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
        // phi(S_c) u = 2^(30 e) (A u + 2^31 B u)
        const uint64_t al = limbs_to_m61(accA[j]), be = limbs_to_m61(accB[j]);
        S[j] = m61_rot(m61_add(al, m61_rot(be, 31)), rot_e);
    }
    wave_sync();
}

// n = 4: phi(S_c) u on MFMA (v_mfma_i32_16x16x64_i8; N = 16 matrix rows per tile, 16 tiles; K = 512
// = [A | B] in 8 steps).  A-operand row m < 8 is digit m of u on the A half of K, row 8 + m digit m
// of 2^31 u on the B half, so sum_m 256^m (D[m][r] + D[8 + m][r]) = A u + 2^31 B u = 2^(-30 e) S_r
// (mod p).  Lane l holds rows 4g..4g+3 (g = l/16) of column l%16 of every tile; the four lane groups
// are combined by a reduce-scatter over lanes l^32, l^16, leaving each lane four finished rows.
// out[m] = bytes m of x[0..3] (byte j of out[m] = byte m of x[j]): two rounds of v_perm_b32.
__device__ inline void transpose_bytes4(const uint32_t* x, uint32_t* out) {
    const uint32_t t0 = __builtin_amdgcn_perm(x[1], x[0], 0x05010400u);
    const uint32_t t1 = __builtin_amdgcn_perm(x[1], x[0], 0x07030602u);
    const uint32_t t2 = __builtin_amdgcn_perm(x[3], x[2], 0x05010400u);
    const uint32_t t3 = __builtin_amdgcn_perm(x[3], x[2], 0x07030602u);
    out[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
    out[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
    out[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
    out[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

template <int WAVES>
__device__ inline void side1_mfma(const Lds<4, WAVES>& L, uint32_t* limbs, const uint64_t* u, int lane, int rot_e,
                                  uint64_t* S) {
    const int g = lane >> 4, n16 = lane & 15;
    // A operand (16 rows x K = 512): rows 0..7 hold the digits of u on the A half of K (columns
    // q < 256) and are zero on the B half; rows 8..15 hold the digits of 2^31 u on the B half and
    // are zero on the A half.  Both sets go through the same 8-row LDS buffer, one after the other.
    const uint32_t* arow0 = n16 < N4_DIG ? limbs + n16 * N4_ROW : L.zero_row;
    const uint32_t* arow1 = n16 >= N4_DIG ? limbs + (n16 - N4_DIG) * N4_ROW : L.zero_row;
    v4i afr[N4_KK];
#pragma unroll
    for (int set = 0; set < 2; ++set) {
        // Signed base-256 digits: for v < 2^62, b = v + C0 with C0 = 0x8080808080808080 stays below
        // 2^64 and v = sum_m (byte_m(b) - 128) 256^m, each digit in [-128, 127]; as an int8 the digit
        // is byte_m(b) xor 0x80.  u is lazily reduced (< 2^61 + 2^32), and so is its image
        // 2^31 u = (u >> 30) + (u mod 2^30) 2^31 (mod p).
        uint32_t lo[4], hi[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t w = set ? (u[j] >> 30) + ((u[j] & 0x3fffffffull) << 31) : u[j];
            const uint64_t b = w + 0x8080808080808080ull;
            lo[j] = (uint32_t)b;
            hi[j] = (uint32_t)(b >> 32);
        }
        // 4 x 4 byte transposes: digit row m gets byte m of the lane's four values (columns 4 lane + j)
        uint32_t dg[N4_DIG];
        transpose_bytes4(lo, dg);
        transpose_bytes4(hi, dg + 4);
#pragma unroll
        for (int m = 0; m < N4_DIG; ++m) limbs[m * N4_ROW + lane] = dg[m] ^ 0x80808080u;
        wave_sync();
        const uint32_t* arow = set ? arow1 : arow0;
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) afr[set * 4 + kq] = *reinterpret_cast<const v4i*>(&arow[kq * 16 + g * 4]);
        wave_sync();
    }
    // N tiles in groups of NG: NG independent accumulation chains over the 8 K steps, then each
    // finished tile is combined at once, so only NG accumulators and 2 NG fragments (the current
    // and the next K step's) are live.
    // Accumulator row m = 4g + j of this lane is digit m % 8 of set g >> 1 (u, or 2^31 u), weight
    // 2^(8 (m % 8)) = 2^(32 (g & 1)) 2^(8j).  Each row sums 256 products, |acc| <= 256 * 128 * 127
    // < 2^22, so x = acc_0 + 2^8 acc_1 + 2^16 acc_2 + 2^24 acc_3 lies in (-2^45, 2^45) and the sum of
    // two such in (-2^46, 2^46).  Its weighted residue, kept lazily in [0, 2^62): with
    // s = 61 - 32 (g & 1),
    //   2^(61 - s) x = (x >> s) 2^61 + (x mod 2^s) 2^(61 - s) = (x >> s) + (x mod 2^s) 2^(61 - s)  (mod p)
    // and y = p + (x >> s) + (x mod 2^s) 2^(61 - s).  Four such values sum below 2^64.
    constexpr int NG = 2;
    const uint32_t s_g = 61 - 32 * (uint32_t)(g & 1);
    const uint64_t m_g = (1ull << s_g) - 1;
    // Fragments of tiles 8..15 lie beyond the 64 KiB reach of a DS immediate offset: they are read
    // through a second base address (kept opaque, so it is formed once instead of per read).
    uint32_t hi_base = 8 * N4_KK * 64;
    asm("" : "+v"(hi_base));
    const v4i* frag_hi = L.frag + hi_base;
    // Per tile, the two 32-bit halves of the raw sum: lo = acc_0 + 2^8 acc_1, hi = acc_2 + 2^8 acc_3,
    // |lo|, |hi| <= 257 * 256 * 128 * 127 < 2^30.
    int32_t lo[N4_NT], hi[N4_NT];
    uint64_t Q[8];
    // tile groups in the order 0..1, 8..9, 2..3, 10..11, ...: after every second group the tile
    // pairs (i, 8 + i) are complete and reduce at once, which keeps few halves live
#pragma unroll
    for (int gi = 0; gi < N4_NT / NG; ++gi) {
        const int n0 = (gi & 1) * 8 + (gi >> 1) * NG;
        v4i acc[NG];
#pragma unroll
        for (int i = 0; i < NG; ++i) acc[i] = v4i{0, 0, 0, 0};
        // B fragments double-buffered: the next K step's NG fragments are read while this step's MFMAs
        // run, so each read has a whole step of MFMAs to cover its LDS latency
        auto frag = [&](int t, int kk) -> v4i {
            return t < 8 ? L.frag[(t * N4_KK + kk) * 64 + lane] : frag_hi[((t - 8) * N4_KK + kk) * 64 + lane];
        };
        v4i bf[2][NG];
#pragma unroll
        for (int i = 0; i < NG; ++i) bf[0][i] = frag(n0 + i, 0);
#pragma unroll
        for (int kk = 0; kk < N4_KK; ++kk) {
            if (kk + 1 < N4_KK) {
#pragma unroll
                for (int i = 0; i < NG; ++i) bf[(kk + 1) & 1][i] = frag(n0 + i, kk + 1);
            }
            // the reads above are issued before this step's MFMAs (nothing moves across)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < NG; ++i)
                acc[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(afr[kk], bf[kk & 1][i], acc[i], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            lo[n0 + i] = acc[i][0] + acc[i][1] * 256;
            hi[n0 + i] = acc[i][2] + acc[i][3] * 256;
        }
        // reduce-scatter over the four lane groups.  Groups g and g ^ 2 carry the same digit weights,
        // so their halves add exactly first, still in 32 bits (|lo + lo'| < 2^31): lanes g < 2 keep
        // tiles 0..7 plus their l^32 partner's, lanes g >= 2 keep tiles 8..15.  The raw sum
        // x = lo + 2^16 hi (|x| < 2^47) then becomes its lazy weighted residue.
        if (gi & 1) {
#pragma unroll
            for (int i = n0 - 8; i < n0 - 8 + NG; ++i) {
                const int64_t x =
                    (int64_t)half_add32_i32(lo[i], lo[8 + i]) + (int64_t)half_add32_i32(hi[i], hi[8 + i]) * 65536;
                Q[i] = P61 + (uint64_t)(x >> s_g) + (((uint64_t)x & m_g) << (61 - s_g));
            }
        }
    }
    // within each half the even groups keep Q[0..3], the odd groups Q[4..7], adding the l^16
    // partner's: plain 64-bit sums below 2^63, one fold at the end.
#pragma unroll
    for (int i = 0; i < 4; ++i) S[i] = m61_rot(m61_fold(half_add16(Q[i], Q[4 + i])), rot_e);
}

// n = 4, two walks of one wavefront on side 1 together: walk w's digit rows become A-operand rows
// 8w .. 8w + 7, each over the whole K = [u | 2^31 u] (digit m of u on the A half, digit m of 2^31 u
// on the B half), so no A row is zero and one pass of the 128 MFMAs serves both walks.  Walk w's
// u goes through the wavefront's 8-row digit buffer one digit set at a time; only the lanes that
// hold rows of walk w (n16 / 8 == w) take fragments from it.
__device__ inline void digits_pair(uint32_t* limbs, const uint64_t* u, int lane, int w, v4i* afr) {
    const int g = lane >> 4, n16 = lane & 15;
    const bool mine = (n16 >> 3) == w;
    const uint32_t* arow = limbs + (n16 & 7) * N4_ROW;
#pragma unroll
    for (int set = 0; set < 2; ++set) {
        // signed base-256 digits of u (set 0) or of 2^31 u (set 1), as in side1_mfma
        uint32_t lo[4], hi[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t v = set ? (u[j] >> 30) + ((u[j] & 0x3fffffffull) << 31) : u[j];
            const uint64_t b = v + 0x8080808080808080ull;
            lo[j] = (uint32_t)b;
            hi[j] = (uint32_t)(b >> 32);
        }
        uint32_t dg[N4_DIG];
        transpose_bytes4(lo, dg);
        transpose_bytes4(hi, dg + 4);
#pragma unroll
        for (int m = 0; m < N4_DIG; ++m) limbs[m * N4_ROW + lane] = dg[m] ^ 0x80808080u;
        wave_sync();
        if (mine) {
#pragma unroll
            for (int kq = 0; kq < 4; ++kq) afr[set * 4 + kq] = *reinterpret_cast<const v4i*>(&arow[kq * 16 + g * 4]);
        }
        wave_sync();
    }
}

// The product of both walks on the shared A operand.  Accumulator row m = 4g + j of lane l is
// digit 4 (g & 1) + j of walk g >> 1 summed over both digit sets: 512 products of at most
// 128 x 127, |acc| < 2^23, so lo = acc_0 + 2^8 acc_1 and hi = acc_2 + 2^8 acc_3 stay within
// 257 x 512 x 128 x 127 < 2^31.  Each tile's raw sum x = lo + 2^16 hi becomes its lazy weighted
// residue (weight 2^(32 (g & 1)), as in side1_mfma); the two digit halves of a row sit in lanes l
// and l ^ 16 and are added by one cross-row swap per tile pair (i, 8 + i).  R[i] is then, in lanes
// of even g, row 16 i + n16 and, in lanes of odd g, row 16 (8 + i) + n16 of walk g >> 1.
template <int WAVES>
__device__ inline void side1_mfma_pair(const Lds<4, WAVES>& L, const v4i* afr, int lane, int rot_e, uint64_t* R) {
    const int g = lane >> 4;
    constexpr int NG = 2;
    const uint32_t s_g = 61 - 32 * (uint32_t)(g & 1);
    const uint64_t m_g = (1ull << s_g) - 1;
    uint32_t hi_base = 8 * N4_KK * 64;
    asm("" : "+v"(hi_base));
    const v4i* frag_hi = L.frag + hi_base;
    uint64_t Q[8];
#pragma unroll
    for (int gi = 0; gi < N4_NT / NG; ++gi) {
        const int n0 = (gi & 1) * 8 + (gi >> 1) * NG;
        v4i acc[NG];
#pragma unroll
        for (int i = 0; i < NG; ++i) acc[i] = v4i{0, 0, 0, 0};
        auto frag = [&](int t, int kk) -> v4i {
            return t < 8 ? L.frag[(t * N4_KK + kk) * 64 + lane] : frag_hi[((t - 8) * N4_KK + kk) * 64 + lane];
        };
        v4i bf[2][NG];
#pragma unroll
        for (int i = 0; i < NG; ++i) bf[0][i] = frag(n0 + i, 0);
#pragma unroll
        for (int kk = 0; kk < N4_KK; ++kk) {
            if (kk + 1 < N4_KK) {
#pragma unroll
                for (int i = 0; i < NG; ++i) bf[(kk + 1) & 1][i] = frag(n0 + i, kk + 1);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < NG; ++i)
                acc[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(afr[kk], bf[kk & 1][i], acc[i], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            const int64_t x = (int64_t)(acc[i][0] + acc[i][1] * 256) + (int64_t)(acc[i][2] + acc[i][3] * 256) * 65536;
            const uint64_t q = P61 + (uint64_t)(x >> s_g) + (((uint64_t)x & m_g) << (61 - s_g));
            if (gi & 1)
                R[n0 - 8 + i] = half_add16(Q[n0 - 8 + i], q);
            else
                Q[n0 + i] = q;
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) R[i] = m61_rot(m61_fold(R[i]), rot_e);
}

// n = 3: phi(S_c) u on MFMA, the n = 4 scheme at R = 64 with one row per lane: A-operand rows 0..7
// are the signed base-256 digits of u on the A half of K = 128, rows 8..15 those of 2^31 u on the
// B half; 4 N tiles x 2 K steps.  Lane l holds accumulator rows 4g..4g+3 (g = l/16) of column l%16
// of each tile; groups g and g ^ 2 have equal digit weights, so their raw sums add first (l^32),
// then as lazy weighted residues within each half (l^16), leaving each lane one finished row.
template <int WAVES>
__device__ inline void side1_mfma3(const Lds<3, WAVES>& L, uint32_t* limbs, const uint64_t* u, int lane, int rot_e,
                                   uint64_t* S) {
    const int g = lane >> 4, n16 = lane & 15;
    const uint32_t* arow0 = n16 < N4_DIG ? limbs + n16 * N3_ROW : L.zero_row;
    const uint32_t* arow1 = n16 >= N4_DIG ? limbs + (n16 - N4_DIG) * N3_ROW : L.zero_row;
    uint8_t* lb = reinterpret_cast<uint8_t*>(limbs);
    v4i afr[N3_KK];
#pragma unroll
    for (int set = 0; set < 2; ++set) {
        // digits as for n = 4 (bytes of v + 0x8080808080808080, each minus 128); column = lane
        const uint64_t w = set ? (u[0] >> 30) + ((u[0] & 0x3fffffffull) << 31) : u[0];
        const uint64_t b = w + 0x8080808080808080ull;
#pragma unroll
        for (int m = 0; m < N4_DIG; ++m) lb[m * N3_ROW * 4 + lane] = (uint8_t)((b >> (8 * m)) ^ 0x80);
        wave_sync();
        const uint32_t* arow = set ? arow1 : arow0;
        afr[set] = *reinterpret_cast<const v4i*>(&arow[g * 4]);
        wave_sync();
    }
    const uint32_t s_g = 61 - 32 * (uint32_t)(g & 1);
    const uint64_t m_g = (1ull << s_g) - 1;
    uint64_t P[N3_NT];
#pragma unroll
    for (int nt = 0; nt < N3_NT; ++nt) {
        v4i acc = v4i{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < N3_KK; ++kk)
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(afr[kk], L.frag[(nt * N3_KK + kk) * 64 + lane], acc, 0, 0, 0);
        // |acc| <= 64 * 128 * 127 < 2^20
        const int32_t lo = acc[0] + acc[1] * 256;
        const int32_t hi = acc[2] + acc[3] * 256;
        P[nt] = (uint64_t)((int64_t)lo + (int64_t)hi * 65536);
    }
    uint64_t Q[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int64_t x = (int64_t)half_add32(P[i], P[2 + i]);
        Q[i] = P61 + (uint64_t)(x >> s_g) + (((uint64_t)x & m_g) << (61 - s_g));
    }
    S[0] = m61_rot(m61_fold(half_add16(Q[0], Q[1])), rot_e);
}

// n = 3: for each (p, row r) bit 0 = P_p and P_r anticommute, bit 1 = their product's phase c is 3
// (the butterfly of R adds the partner), one byte each, computed at compile time.
struct Rot3Tab {
    uint8_t v[64 * 64];
};
constexpr Rot3Tab make_rot3_tab() {
    Rot3Tab t{};
    for (uint32_t p = 1; p < 64; ++p) {
        const uint32_t xp = p & 7, zp = p >> 3;
        for (uint32_t r = 0; r < 64; ++r) {
            const uint32_t xr = r & 7, zr = r >> 3;
            const uint32_t anti = (uint32_t)(__builtin_popcount(xp & zr) + __builtin_popcount(zp & xr)) & 1;
            const uint32_t c = (uint32_t)(__builtin_popcount(xp & zp) + __builtin_popcount(xr & zr) + 4 -
                                          __builtin_popcount((xp ^ xr) & (zp ^ zr)) + 2 * __builtin_popcount(zp & xr)) &
                               3;
            t.v[p * 64 + r] = (uint8_t)(anti | ((uint32_t)(c == 3) << 1));
        }
    }
    return t;
}
__device__ constexpr Rot3Tab ROT3_TAB = make_rot3_tab();

// n <= 3 (one row per lane, r = gl): the h rotations with the same lazy reduction as rotate4.
template <int NQ>
__device__ inline void rotate1(uint64_t& u, const uint32_t* dig, int h, int side, int gl, int gbase) {
    const uint32_t r = (uint32_t)gl;
    uint32_t tb[Geo<NQ>::HMAX];
    if constexpr (NQ == 3) {
        // every digit slot holds a valid code, so all loads stay in the table
#pragma unroll
        for (int t = 0; t < Geo<NQ>::HMAX; ++t) tb[t] = ROT3_TAB.v[dig[t] * 64 + r];
    }
#pragma unroll
    for (int t = Geo<NQ>::HMAX - 1; t >= 0; --t) {
        if (t >= h) continue;
        const uint32_t p = dig[t];
        const uint64_t part = shfl64(u, gbase + (gl ^ (int)p));
        // side 0 (R u): (u_r - s u_{r^p}) / sqrt2;  side 1 (R^T u): (u_r + s u_{r^p}) / sqrt2
        bool plus, anti;
        if constexpr (NQ == 3) {
            plus = (((tb[t] >> 1) ^ (uint32_t)side) & 1) != 0;
            anti = (tb[t] & 1) != 0;
        } else {
            plus = (side == 1) == (rotation_sign<NQ>(p, r) > 0);
            anti = anticommutes<NQ>(p, r) != 0;
        }
        const uint64_t q = plus ? part : (2 * P61 - part);
        const uint64_t sum = u + q;
        const uint64_t rot = (sum >> 31) + ((sum & 0x7fffffffull) << 30);
        u = anti ? rot : u;
    }
}

// n = 4: the h rotations applied to the key vector.  Lane l holds rows r_j = 4 l + j (j = 0..3).
// Rotation p touches row r when P_p and P_r anticommute (<p, r> = |x_p & z_r| + |z_p & x_r| odd);
// with P_p P_r = i^c P_{p^r}, c = |x_p & z_p| + |x_r & z_r| - |(x_p ^ x_r) & (z_p ^ z_r)| +
// 2 |z_p & x_r| (mod 4), the butterfly of R (side 0) adds the partner value u_{r^p} when c = 3
// and subtracts it when c = 1; R^T (side 1) the other way round.  Both bits depend only on (p, l, j)
// and sit in a compile-time table, one byte per (p, lane): bit j = anticommutes, bit 4 + j = c is 3.
struct Rot4Tab {
    uint8_t v[256 * 64];
};
constexpr Rot4Tab make_rot4_tab() {
    Rot4Tab t{};
    for (uint32_t p = 1; p < 256; ++p) {
        const uint32_t xp = p & 15, zp = p >> 4;
        for (uint32_t l = 0; l < 64; ++l) {
            uint32_t b = 0;
            for (uint32_t j = 0; j < 4; ++j) {
                const uint32_t r = 4 * l + j, xr = r & 15, zr = r >> 4;
                const uint32_t anti = (uint32_t)(__builtin_popcount(xp & zr) + __builtin_popcount(zp & xr)) & 1;
                const uint32_t c = (uint32_t)(__builtin_popcount(xp & zp) + __builtin_popcount(xr & zr) + 4 -
                                              __builtin_popcount((xp ^ xr) & (zp ^ zr)) +
                                              2 * __builtin_popcount(zp & xr)) & 3;
                b |= (anti << j) | ((uint32_t)(c == 3) << (4 + j));
            }
            t.v[p * 64 + l] = (uint8_t)b;
        }
    }
    return t;
}
__device__ constexpr Rot4Tab ROT4_TAB = make_rot4_tab();

// Values stay lazily reduced below 2^61 + 2^32: u + (2p - part) < 2^63, and for s = a 2^31 + b,
// s 2^30 = a 2^61 + b 2^30 = a + b 2^30 (mod p).
// part[j] = u[j ^ C] of lane src (C a compile-time register permutation).
template <int C>
__device__ inline void fetch4(const uint64_t* u, int src, uint64_t* part) {
#pragma unroll
    for (int j = 0; j < 4; ++j) part[j] = shfl64(u[j ^ C], src);
}

__device__ inline void rotate4(uint64_t* u, const uint32_t* dig, int h, int side, int gl, int gbase) {
    // the table bytes of the rotations to apply, first, so their latency overlaps the partner fetches
    uint32_t tb[Geo<4>::HMAX];
#pragma unroll
    for (int t = 0; t < Geo<4>::HMAX; ++t) tb[t] = t < h ? ROT4_TAB.v[dig[t] * 64 + gl] : 0u;
    const uint32_t side_b = side ? 0xf0u : 0u;
#pragma unroll
    for (int t = Geo<4>::HMAX - 1; t >= 0; --t) {
        if (t >= h) continue;
        const uint32_t p = dig[t];
        // partner rows r ^ p: lane l ^ (p >> 2), register j ^ (p & 3).  p is wave-uniform, so the
        // register order is a uniform branch and all eight partner fetches are issued together.
        const int src = gbase + (gl ^ (int)(p >> 2));
        uint64_t part[4];
        switch (p & 3) {
            case 0: fetch4<0>(u, src, part); break;
            case 1: fetch4<1>(u, src, part); break;
            case 2: fetch4<2>(u, src, part); break;
            default: fetch4<3>(u, src, part); break;
        }
        // bit j: anticommutes; bit 4 + j: the butterfly adds the partner (side 0: c = 3, side 1: c = 1)
        const uint32_t b = tb[t] ^ side_b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t q = ((b >> (4 + j)) & 1) ? part[j] : (2 * P61 - part[j]);
            const uint64_t sum = u[j] + q;
            const uint64_t r = (sum >> 31) + ((sum & 0x7fffffffull) << 30);
            u[j] = ((b >> j) & 1) ? r : u[j];
        }
    }
}

// n = 4: the key vector with the first rotations already applied -- R(p_{h-2}) R(p_{h-1}) K or the
// transposes' from the two-rotation table, one rotation from the one-rotation table, or K itself --
// into u (lane gl's four rows); returns how many rotations are left to apply.
template <int WAVES>
__device__ inline int key_row4(const SpaceDev& sp, const Lds<4, WAVES>& L, const uint32_t* dig, int side, int gl,
                               uint64_t* u) {
    const int h = sp.h;
    if (sp.rkeys2 != nullptr && h >= 2) {
        const uint64_t* tp =
            sp.rkeys2 + ((((uint32_t)side * 256u + dig[h - 1]) * 256u + dig[h - 2]) * 256u + 4u * (uint32_t)gl);
#pragma unroll
        for (int j = 0; j < 4; ++j) u[j] = tp[j];
        return h - 2;
    }
    if (sp.rkeys != nullptr && h >= 1) {
        const uint64_t* tp = sp.rkeys + ((uint32_t)side * 256u + dig[h - 1]) * 256u + 4u * (uint32_t)gl;
#pragma unroll
        for (int j = 0; j < 4; ++j) u[j] = tp[j];
        return h - 1;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) u[j] = L.K[gl * 4 + j];
    return h;
}

// One evaluation of f on `pt` by the walk group; every lane of the group returns the same values.
template <int NQ, int WAVES>
__device__ void walk_step(const SpaceDev& sp, const Lds<NQ, WAVES>& L, uint32_t* limbs, uint64_t pt, int gl,
                          int gbase, uint64_t& out_pt, uint64_t& out_h) {
    using Gm = Geo<NQ>;
    constexpr int R = Gm::R, RPL = Gm::RPL, Q4 = Gm::Q4, HMAX = Gm::HMAX;
    if constexpr (Gm::G == 64) pt = uniform64(pt);  // one walk per wavefront: decode on the scalar unit
    const uint32_t x = (uint32_t)pt;
    const int side = (int)((pt >> 32) & 1);
    const int h = sp.h;

    // mu: base-xi digits, least significant first; Pauli p_t = d_t + 1
    uint32_t dig[HMAX];
    {
        uint32_t xx = x;
#pragma unroll
        for (int t = 0; t < HMAX; ++t) {
            dig[t] = xx % Gm::XI + 1;
            xx /= Gm::XI;
        }
    }

    // key vector through the rotations, p_{h-1} first
    uint64_t u[RPL];
    if constexpr (NQ == 4) {
        // the first two rotations, R(p_{h-2}) R(p_{h-1}) K or the transposes', come precomputed for
        // every pair of Paulis (a 256 MiB table in HBM, 2 KiB per step in 32 contiguous bytes per
        // lane); with one rotation only, from a 1 MiB table; the others are applied here
        const int h_left = key_row4(sp, L, dig, side, gl, u);
        rotate4(u, dig, h_left, side, gl, gbase);
    } else {
        u[0] = L.K[gl];
        rotate1<NQ>(u[0], dig, h, side, gl, gbase);
    }

    uint64_t S[RPL];
    if (side) {
        if constexpr (NQ == 4) {
            side1_mfma<WAVES>(L, limbs, u, gl, sp.rot_e, S);
        } else if constexpr (NQ == 3) {
            side1_mfma3<WAVES>(L, limbs, u, gl, sp.rot_e, S);
        } else {
            side1_dot4<NQ, WAVES>(L, limbs, u, gl, sp.rot_e, S);
        }
    } else {
#pragma unroll
        for (int j = 0; j < RPL; ++j) S[j] = m61_fold(u[j]);  // n = 4 keeps u lazily reduced
    }

    // sign-normalised row digests and the multiset hash of the walk group's rows.  For c in
    // [0, p]: p - c = c ^ p, and of c and p - c the smaller is the one with bit 60 clear, so
    // min(c mod p, p - c mod p) = c ^ (bit 60 of c ? p : 0) (which also sends p to 0).
    uint64_t acc = 0;
    const uint32_t ka = (uint32_t)sp.salt_h, kb = (uint32_t)(sp.salt_h >> 32);
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
        const uint64_t c = S[j];
        const uint64_t d = c ^ (P61 & (0ull - ((c >> 60) & 1)));
        acc += (uint64_t)((uint32_t)d + ka) * (uint64_t)((uint32_t)(d >> 32) + kb);
    }
    if constexpr (Gm::G == 64) {
        // within each 16-lane row by DPP (quad permutes, then row rotations by 4 and 8, which add the
        // other quads' sums), then across rows by the cross-half swaps: no LDS round trip
        acc += dpp64<0xB1>(acc);   // quad_perm [1,0,3,2]
        acc += dpp64<0x4E>(acc);   // quad_perm [2,3,0,1]
        acc += dpp64<0x124>(acc);  // row_ror:4
        acc += dpp64<0x128>(acc);  // row_ror:8
        acc = half_add16(acc, acc);
        acc = half_add32(acc, acc);
        // one walk per wavefront: the sum is the same in every lane; finish on the scalar unit
        acc = uniform64(acc);
    } else {
        // a walk group is a quad (n = 1) or a 16-lane row (n = 2): DPP within it, no LDS round trip
        static_assert(Gm::G == 4 || Gm::G == 16, "walk groups below 64 lanes are quads or rows");
        acc += dpp64<0xB1>(acc);  // quad_perm [1,0,3,2]
        acc += dpp64<0x4E>(acc);  // quad_perm [2,3,0,1]
        if constexpr (Gm::G == 16) {
            acc += dpp64<0x124>(acc);  // row_ror:4
            acc += dpp64<0x128>(acc);  // row_ror:8
        }
    }
    const uint64_t H = mix64(acc);
    out_h = H;
    out_pt = mulhi64(H, sp.n_half) | ((H & 1) << 32);
}

// n = 4: one evaluation of f for each of the wavefront's two walks, both points on side 1 (pa, pb
// uniform).  Each walk's key row, rotations and digits in turn, then the shared MFMA product, and each 32-lane half of the wavefront hashes its walk's
// 256 rows (eight per lane).  The values equal those of two walk_step calls.
template <int WAVES>
__device__ void walk_step_pair4(const SpaceDev& sp, const Lds<4, WAVES>& L, uint32_t* limbs, uint64_t pa,
                                uint64_t pb, int lane, uint64_t& out_a, uint64_t& h_a, uint64_t& out_b,
                                uint64_t& h_b) {
    constexpr int HMAX = Geo<4>::HMAX;
    // the points are the same in every lane: decode on the scalar unit (uniform branches below)
    pa = uniform64(pa);
    pb = uniform64(pb);
    v4i afr[N4_KK];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        uint32_t dig[HMAX];
        uint32_t xx = (uint32_t)(w ? pb : pa);
#pragma unroll
        for (int t = 0; t < HMAX; ++t) {
            dig[t] = xx % Geo<4>::XI + 1;
            xx /= Geo<4>::XI;
        }
        uint64_t u[4];
        const int h_left = key_row4(sp, L, dig, 1, lane, u);
        rotate4(u, dig, h_left, 1, lane, 0);
        digits_pair(limbs, u, lane, w, afr);
    }
    uint64_t R[8];
    side1_mfma_pair<WAVES>(L, afr, lane, sp.rot_e, R);
    uint64_t acc = 0;
    const uint32_t ka = (uint32_t)sp.salt_h, kb = (uint32_t)(sp.salt_h >> 32);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint64_t c = R[i];
        const uint64_t d = c ^ (P61 & (0ull - ((c >> 60) & 1)));
        acc += (uint64_t)((uint32_t)d + ka) * (uint64_t)((uint32_t)(d >> 32) + kb);
    }
    acc += dpp64<0xB1>(acc);   // quad_perm [1,0,3,2]
    acc += dpp64<0x4E>(acc);   // quad_perm [2,3,0,1]
    acc += dpp64<0x124>(acc);  // row_ror:4
    acc += dpp64<0x128>(acc);  // row_ror:8
    acc = half_add16(acc, acc);
    // lanes 0..31 now hold walk a's sum, lanes 32..63 walk b's
    auto lane64 = [&](int l) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)acc, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(acc >> 32), l);
        return ((uint64_t)hi << 32) | lo;
    };
    const uint64_t sa = lane64(0), sb = lane64(32);
    h_a = mix64(sa);
    h_b = mix64(sb);
    out_a = mulhi64(h_a, sp.n_half) | ((h_a & 1) << 32);
    out_b = mulhi64(h_b, sp.n_half) | ((h_b & 1) << 32);
}

__device__ inline bool is_dist(const SpaceDev& sp, uint64_t pt) {
    if (sp.delta == 0) return true;
    const uint64_t x = pt & 0xffffffffull, b = (pt >> 32) & 1;
    return (mix64(((x << 1) | b) ^ sp.salt_d) >> (64 - sp.delta)) == 0;
}

__device__ inline uint64_t start_point(const SpaceDev& sp, uint64_t w, uint32_t j) {
    const uint64_t g = sm64(sp.salt_s, (w << 32) | j);
    return mulhi64(g, sp.n_half) | ((g & 1) << 32);
}

constexpr int WAVES_SMALL = 4;
template <int NQ>
struct WalkWaves {
    static constexpr int value = NQ == 4 ? 12 : WAVES_SMALL;
};

// ---- parity kernels ----
template <int NQ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_step(SpaceDev sp, const uint64_t* in, uint64_t* out,
                                                     uint64_t* hash, int64_t count) {
    using Gm = Geo<NQ>;
    __shared__ Lds<NQ, WAVES> L;
    load_lds(L, sp);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gi = lane / Gm::G, gl = lane % Gm::G, gbase = gi * Gm::G;
    uint32_t* limbs = L.limbs[wave * Gm::WPW + gi];
    const int64_t stride = (int64_t)gridDim.x * WAVES * Gm::WPW;
    for (int64_t base = ((int64_t)blockIdx.x * WAVES + wave) * Gm::WPW; base < count; base += stride) {
        const int64_t i = base + gi;
        if (i < count) {
            uint64_t o, hh;
            walk_step<NQ, WAVES>(sp, L, limbs, in[i], gl, gbase, o, hh);
            if (gl == 0) {
                out[i] = o;
                if (hash) hash[i] = hh;
            }
        }
    }
}

template <int NQ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_trails(SpaceDev sp, const uint64_t* starts, int64_t count,
                                                       uint32_t cap, uint64_t* dp, uint32_t* len) {
    using Gm = Geo<NQ>;
    __shared__ Lds<NQ, WAVES> L;
    load_lds(L, sp);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gi = lane / Gm::G, gl = lane % Gm::G, gbase = gi * Gm::G;
    uint32_t* limbs = L.limbs[wave * Gm::WPW + gi];
    const int64_t stride = (int64_t)gridDim.x * WAVES * Gm::WPW;
    for (int64_t base = ((int64_t)blockIdx.x * WAVES + wave) * Gm::WPW; base < count; base += stride) {
        const int64_t i = base + gi;
        if (i < count) {
            uint64_t pt = starts[i];
            uint32_t d = 0, found = 0;
            for (uint32_t t = 1; t <= cap; ++t) {
                uint64_t nx, hh;
                walk_step<NQ, WAVES>(sp, L, limbs, pt, gl, gbase, nx, hh);
                pt = nx;
                if (is_dist(sp, pt)) {
                    d = t;
                    found = 1;
                    break;
                }
            }
            if (gl == 0) {
                dp[i] = found ? pt : 0;
                len[i] = found ? d : 0;
            }
        }
    }
}

// Canonical hash of explicit matrices: the side-1 product with u = K (no rotations).
template <int NQ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_canon(SpaceDev sp, const uint32_t* phi_all, const int32_t* e,
                                                      int64_t count, uint64_t* out) {
    using Gm = Geo<NQ>;
    constexpr int NPHI = Gm::Q4 * Gm::R;
    __shared__ Lds<NQ, WAVES> L;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gi = lane / Gm::G, gl = lane % Gm::G, gbase = gi * Gm::G;
    uint32_t* limbs = L.limbs[wave * Gm::WPW + gi];
    for (int64_t m = blockIdx.x; m < count; m += gridDim.x) {
        SpaceDev s2 = sp;
        s2.phi = phi_all + (size_t)m * 2 * NPHI;
        s2.h = 0;
        s2.rot_e = (int32_t)(((30ll * e[m]) % 61 + 61) % 61);
        s2.n_half = 1;
        __syncthreads();
        load_lds(L, s2);
        __syncthreads();
        if (wave == 0 && gi == 0) {
            uint64_t o, hh;
            walk_step<NQ, WAVES>(s2, L, limbs, 1ull << 32, gl, gbase, o, hh);
            if (gl == 0) out[m] = hh;
        }
    }
}

// x y mod p for x, y < 2^61: x y = hi 2^64 + lo = 8 hi + lo (mod p), lo split at bit 61.
__device__ inline uint64_t m61_mul(uint64_t x, uint64_t y) {
    const uint64_t lo = x * y, hi = __umul64hi(x, y);
    return m61_fold((lo & P61) + (lo >> 61) + (hi << 3));
}

// Canonical hash of explicit matrices whose entries do not fit int8: the row digests
// S_r = sum_q phi(M_rq) K[q] by 64-bit modular products (one matrix per 64-lane block, rows over
// lanes), then the same sign fold, element map and sum as walk_step.  Exact for any int32 entries.
template <int NQ>
__global__ __launch_bounds__(64) void k_canon_wide(SpaceDev sp, const int32_t* a, const int32_t* b,
                                                   const int32_t* e, int64_t count, uint64_t* out) {
    constexpr int R = Geo<NQ>::R;
    const int lane = threadIdx.x;
    const uint32_t ka = (uint32_t)sp.salt_h, kb = (uint32_t)(sp.salt_h >> 32);
    for (int64_t m = blockIdx.x; m < count; m += gridDim.x) {
        // (a + b sqrt2) / sqrt2^e: phi(1/sqrt2) = 2^30, so the scale is a rotation by 30 e mod 61
        const int rot = (int)(((30ll * e[m]) % 61 + 61) % 61);
        uint64_t acc = 0;
        for (int r = lane; r < R; r += 64) {
            const int32_t* ar = a + ((size_t)m * R + r) * R;
            const int32_t* br = b + ((size_t)m * R + r) * R;
            uint64_t sum = 0;
            for (int q = 0; q < R; ++q) {
                const uint64_t v = m61_add(m61_from_i32(ar[q]), m61_rot(m61_from_i32(br[q]), 31));
                sum = m61_add(sum, m61_mul(v, sp.keys[q]));
            }
            const uint64_t c = m61_rot(sum, rot);
            const uint64_t d = c ^ (P61 & (0ull - ((c >> 60) & 1)));
            acc += (uint64_t)((uint32_t)d + ka) * (uint64_t)((uint32_t)(d >> 32) + kb);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc += shfl64(acc, lane ^ off);
        if (lane == 0) out[m] = mix64(acc);
    }
}

template <int NQ>
__global__ void k_pack_i32(const int32_t* a, const int32_t* b, int64_t count, uint32_t* phi, int* flag) {
    constexpr int R = Geo<NQ>::R, Q4 = Geo<NQ>::Q4;
    if constexpr (NQ >= 3) {
        // MFMA fragment layout (see Lds<4>, Lds<3>): 2 * Q4 * R dwords per matrix, KK = 2R / 64 K steps
        constexpr int KK = 2 * R / 64;
        const int64_t total4 = count * 2 * Q4 * R;
        for (int64_t idx = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; idx < total4;
             idx += (int64_t)blockDim.x * gridDim.x) {
            const int64_t m = idx / (2 * Q4 * R);
            const int rem = (int)(idx % (2 * Q4 * R));
            const int fi = rem >> 2, w = rem & 3;
            const int l = fi & 63, fk = fi >> 6;
            const int nt = fk / KK, kk = fk % KK;
            const int r = nt * 16 + (l & 15);
            const int32_t* am = a + m * R * R;
            const int32_t* bm = b + m * R * R;
            uint32_t word = 0;
            for (int c = 0; c < 4; ++c) {
                const int qq = kk * 64 + (l >> 4) * 16 + 4 * w + c;
                const int32_t v = qq < R ? am[r * R + qq] : bm[r * R + qq - R];
                if (v > 127 || v < -127) atomicOr(flag, 2);
                word |= ((uint32_t)(uint8_t)(int8_t)v) << (8 * c);
            }
            phi[m * 2 * Q4 * R + rem] = word;
        }
        return;
    }
    const int64_t total = count * Q4 * R;
    for (int64_t idx = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; idx < total;
         idx += (int64_t)blockDim.x * gridDim.x) {
        const int64_t m = idx / (Q4 * R);
        const int rem = (int)(idx % (Q4 * R));
        const int q4 = rem / R, r = rem % R;
        const int32_t* am = a + m * R * R;
        const int32_t* bm = b + m * R * R;
        uint32_t wa = 0, wb = 0;
        for (int c = 0; c < 4; ++c) {
            const int32_t va = am[r * R + 4 * q4 + c], vb = bm[r * R + 4 * q4 + c];
            if (va > 127 || va < -127 || vb > 127 || vb < -127) atomicOr(flag, 2);
            wa |= ((uint32_t)(uint8_t)(int8_t)va) << (8 * c);
            wb |= ((uint32_t)(uint8_t)(int8_t)vb) << (8 * c);
        }
        phi[m * 2 * Q4 * R + rem] = wa;
        phi[m * 2 * Q4 * R + Q4 * R + rem] = wb;
    }
}

__global__ void k_starts(SpaceDev sp, int64_t w0, uint32_t j, int64_t count, uint64_t* out) {
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; i < count; i += (int64_t)blockDim.x * gridDim.x)
        out[i] = start_point(sp, (uint64_t)(w0 + i), j);
}

// n = 4: out[side][p][q] = the first rotation of the walk step applied to K, by rotate4's butterfly
// (so the values are the ones the step would compute): side 0 R(p) K, side 1 R(p)^T K.  One block
// per (side, p), one thread per row q; p = 0 (no rotation) copies K.
__global__ void k_rot_keys(const uint64_t* keys, uint64_t* out) {
    const uint32_t q = threadIdx.x, p = blockIdx.x & 255u, side = blockIdx.x >> 8;
    uint64_t v = keys[q];
    if (p != 0) {
        const uint32_t b = ROT4_TAB.v[p * 64 + (q >> 2)], j = q & 3;
        if ((b >> j) & 1) {
            const uint64_t part = keys[q ^ p];
            const uint64_t w = (((b >> (4 + j)) ^ side) & 1) ? part : (2 * P61 - part);
            const uint64_t sum = v + w;
            v = (sum >> 31) + ((sum & 0x7fffffffull) << 30);
        }
    }
    out[(size_t)blockIdx.x * 256 + q] = v;
}

// n = 4: out[side][p][p'][q] = rotation p' (rotate4's butterfly) applied to rkeys[side][p]; one block
// per (side, p, p'), one thread per row q; p' = 0 copies.
__global__ void k_rot_keys2(const uint64_t* rkeys, uint64_t* out) {
    const uint32_t q = threadIdx.x, p2 = blockIdx.x & 255u, sp1 = blockIdx.x >> 8, side = sp1 >> 8;
    const uint64_t* in = rkeys + (size_t)sp1 * 256;
    uint64_t v = in[q];
    if (p2 != 0) {
        const uint32_t b = ROT4_TAB.v[p2 * 64 + (q >> 2)], j = q & 3;
        if ((b >> j) & 1) {
            const uint64_t part = in[q ^ p2];
            const uint64_t w = (((b >> (4 + j)) ^ side) & 1) ? part : (2 * P61 - part);
            const uint64_t sum = v + w;
            v = (sum >> 31) + ((sum & 0x7fffffffull) << 30);
        }
    }
    out[(size_t)blockIdx.x * 256 + q] = v;
}

// K[q] = (sm64(s_0, q) >> 3) mod p, s_0 = sm64(seed, 0)
__global__ void k_keys(int r, uint64_t seed, uint64_t* keys) {
    const int i = threadIdx.x + blockIdx.x * blockDim.x;
    if (i >= r) return;
    const uint64_t s0 = sm64(seed, 0);
    uint64_t k = sm64(s0, (uint64_t)i) >> 3;
    if (k >= P61) k -= P61;
    keys[i] = k;
}

// ---- the walk kernel: trails, distinguished-point table, backtracking (Sec. 3) ----

// Claim a slot for `dp` (linear probing).  Returns 1 = new (claimed), 2 = key present, 3 = full.
__device__ inline int table_claim(const WalkDev& wd, uint64_t dp, uint64_t& slot) {
    const uint64_t mask = (1ull << wd.log2_table) - 1;
    uint64_t s = mix64(dp ^ 0x5bd1e9955bd1e995ull) & mask;
    for (int probe = 0; probe < 64; ++probe) {
        uint64_t expected = EMPTY_KEY;
        const bool won = __hip_atomic_compare_exchange_strong(&wd.table[2 * s], &expected, dp, __ATOMIC_RELAXED,
                                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (won) {
            slot = s;
            return 1;
        }
        if (expected == dp) {
            slot = s;
            return 2;
        }
        s = (s + 1) & mask;
    }
    return 3;
}

__device__ inline uint64_t pack_value(uint64_t start, uint32_t len) {
    return (start & 0x1ffffffffull) | ((uint64_t)(len & 0x3fffffffu) << 33) | (1ull << 63);
}

// The walks of one block: walk slots first_block * WAVES * WPW + ... strided by nblocks blocks.
// A walk group's event counts, added to the member's statistics by its leader lane (flush_counts).
struct WalkCounts {
    uint64_t steps = 0, dps = 0, ins = 0, ab = 0, rh = 0, same = 0, red = 0, claw = 0, full = 0, spin = 0,
             active = 0;
};

__device__ inline void flush_counts(const WalkDev& wd, WalkCounts& c, bool leader) {
    if (leader) {
        atomicAdd(&wd.stats[ST_STEPS], (unsigned long long)c.steps);
        atomicAdd(&wd.stats[ST_DPS], (unsigned long long)c.dps);
        atomicAdd(&wd.stats[ST_INSERTS], (unsigned long long)c.ins);
        atomicAdd(&wd.stats[ST_ABANDONED], (unsigned long long)c.ab);
        atomicAdd(&wd.stats[ST_ROBIN], (unsigned long long)c.rh);
        atomicAdd(&wd.stats[ST_SAME], (unsigned long long)c.same);
        atomicAdd(&wd.stats[ST_REDUCTION], (unsigned long long)c.red);
        atomicAdd(&wd.stats[ST_CLAWS], (unsigned long long)c.claw);
        atomicAdd(&wd.stats[ST_FULL], (unsigned long long)c.full);
        atomicAdd(&wd.stats[ST_SPIN], (unsigned long long)c.spin);
        atomicAdd(&wd.stats[ST_ACTIVE], (unsigned long long)c.active);
        c = WalkCounts{};
    }
}

// Events of one evaluation, as bits: advance_walk returns them and the walk group's leader adds
// them to the group's counts in LDS, so no count is held in registers through the step.
enum : uint32_t {
    EV_DP = 1, EV_INS = 2, EV_AB = 4, EV_RH = 8, EV_SAME = 16, EV_RED = 32, EV_CLAW = 64, EV_FULL = 128, EV_SPIN = 256
};

__device__ inline void count_events(WalkCounts& c, uint32_t ev) {
    if (ev & EV_DP) c.dps++;
    if (ev & EV_INS) c.ins++;
    if (ev & EV_AB) c.ab++;
    if (ev & EV_RH) c.rh++;
    if (ev & EV_SAME) c.same++;
    if (ev & EV_RED) c.red++;
    if (ev & EV_CLAW) c.claw++;
    if (ev & EV_FULL) c.full++;
    if (ev & EV_SPIN) c.spin++;
}

__device__ inline WalkState load_state(const WalkDev& wd, int64_t w, bool uniform) {
    WalkState st = wd.states[w];
    if (uniform) {
        st.start = uniform64(st.start);
        st.cur = uniform64(st.cur);
        st.pa = uniform64(st.pa);
        st.pb = uniform64(st.pb);
        st.na = uniform64(st.na);
        st.ha = uniform64(st.ha);
        st.len = uniform32(st.len);
        st.trail = uniform32(st.trail);
        st.mode = uniform32(st.mode);
        st.rem = uniform32(st.rem);
    }
    return st;
}

// The point a walk evaluates f on next: its current point while walking, else the backtracking
// point that ALIGN / LOCK advances.
__device__ inline uint64_t step_arg(const WalkState& st) {
    // as masks rather than a choice of field, so the states stay in registers
    const uint64_t walk = 0ull - (uint64_t)((st.mode & 0xff) == MODE_WALK);
    const uint64_t second = 0ull - (uint64_t)((st.mode >> 8) & 1);
    return (st.cur & walk) | (((st.pb & second) | (st.pa & ~second)) & ~walk);
}

// Walk w's state after one evaluation f(arg) = (nxt, H): distinguished points into the table,
// backtracking of two trails that met (Sec. 3, Fig. 2), claws recorded, trails restarted.  WHOLE:
// the walk occupies the whole wavefront (its leader is lane 0).
template <bool WHOLE>
__device__ inline uint32_t advance_walk(const SpaceDev& sp, const WalkDev& wd, WalkState& st, int64_t w,
                                        uint64_t arg, uint64_t nxt, uint64_t H, bool leader, int gbase) {
    uint32_t ev = 0;
    const uint32_t mode = st.mode & 0xff;
    const uint32_t which = (st.mode >> 8) & 1;
    bool restart = false;
    if (mode == MODE_WALK && wd.enumerate) {
        // exhaustive mode: every point once, the table keyed by its full matrix hash and holding,
        // in the two 32-bit halves of the value, the least x of each side that reached the key (a
        // 32-bit atomic minimum, so no ordering between writers is needed).  The pairs are read
        // out after the last point (k_enum_pairs): which pairs are reported does not depend on
        // the order in which walks arrive.
        ev |= EV_DP;
        const uint64_t key = H == EMPTY_KEY ? (H ^ 1) : H;
        int kind = 0;
        if (leader) {
            uint64_t slot = 0;
            kind = table_claim(wd, key, slot);
            if (kind != 3) {
                uint32_t* half = reinterpret_cast<uint32_t*>(&wd.table[2 * slot + 1]) + ((arg >> 32) & 1);
                atomicMin(half, (uint32_t)arg);
            }
        }
        if constexpr (WHOLE)
            kind = (int)uniform32((uint32_t)kind);
        else
            kind = (int)shfl32((uint32_t)kind, gbase);
        if (kind == 3)
            ev |= EV_FULL;
        else if (kind == 1)
            ev |= EV_INS;
        restart = true;
    } else if (mode == MODE_WALK) {
        st.len++;
        if (is_dist(sp, nxt)) {
            ev |= EV_DP;
            int kind = 0;
            uint64_t slot = 0, other = 0;
            if (leader) kind = table_claim(wd, nxt, slot);
            // The slot's writer publishes its value right after its claim.  The value word is
            // all a reader uses (start, length and a ready bit), so relaxed device-scope atomics
            // suffice; release and acquire would write back and invalidate the L2 of the
            // wavefront's XCD at every distinguished point.
            if (leader && kind == 1)
                __hip_atomic_store(&wd.table[2 * slot + 1], pack_value(st.start, st.len), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            if (leader && kind == 2) {
                int spin = 0;
                do {
                    other = __hip_atomic_load(&wd.table[2 * slot + 1], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                } while (other == 0 && ++spin < (1 << 20));
                if (other == 0) kind = 4;
            }
            if constexpr (WHOLE) {
                // the walk is the whole wavefront and its leader is lane 0: the answer stays scalar
                kind = (int)uniform32((uint32_t)kind);
                other = uniform64(other);
            } else {
                kind = (int)shfl32((uint32_t)kind, gbase);
                other = shfl64(other, gbase);
            }
            restart = true;
            if (kind == 1) {
                ev |= EV_INS;
            } else if (kind == 3) {
                ev |= EV_FULL;
            } else if (kind == 4) {
                ev |= EV_SPIN;
            } else if (kind == 2) {
                const uint64_t ostart = other & 0x1ffffffffull;
                const uint32_t olen = (uint32_t)((other >> 33) & 0x3fffffffu);
                if (ostart != st.start) {
                    // backtrack the two trails (Sec. 3, Fig. 2)
                    restart = false;
                    st.pa = st.start;
                    st.pb = ostart;
                    const uint32_t la = st.len, lb = olen;
                    if (la > lb) {
                        st.mode = MODE_ALIGN;
                        st.rem = la - lb;
                        st.len = lb;
                    } else if (lb > la) {
                        st.mode = MODE_ALIGN | (1u << 8);
                        st.rem = lb - la;
                        st.len = la;
                    } else {
                        st.mode = MODE_LOCK;
                        st.rem = la;
                    }
                }
            }
        } else if (st.len >= wd.cap) {
            ev |= EV_AB;
            restart = true;
        } else {
            st.cur = nxt;
        }
    } else if (mode == MODE_ALIGN) {
        if (which) st.pb = nxt; else st.pa = nxt;
        if (--st.rem == 0) {
            if (st.pa == st.pb) {
                ev |= EV_RH;  // one trail started on the other
                restart = true;
            } else {
                st.mode = MODE_LOCK;
                st.rem = st.len;
            }
        }
    } else {  // MODE_LOCK
        if (!which) {
            st.na = nxt;
            st.ha = H;
            st.mode = MODE_LOCK | (1u << 8);
        } else {
            if (st.na == nxt) {
                // f(pa) = f(pb) with pa != pb: the merge
                const uint64_t sa = (st.pa >> 32) & 1, sb = (st.pb >> 32) & 1;
                if (sa == sb) {
                    ev |= EV_SAME;
                } else if (st.ha != H) {
                    ev |= EV_RED;
                } else {
                    ev |= EV_CLAW;
                    if (leader) {
                        const unsigned long long idx = atomicAdd(wd.claw_count, 1ull);
                        if (idx < wd.claw_cap) {
                            wd.claws[2 * idx] = st.pa;
                            wd.claws[2 * idx + 1] = st.pb;
                        }
                    }
                }
                restart = true;
            } else {
                st.pa = st.na;
                st.pb = nxt;
                st.mode = MODE_LOCK;
                if (--st.rem == 0) restart = true;  // cannot happen for two trails with one end
            }
        }
    }
    if (restart) {
        st.trail++;
        st.len = 0;
        st.mode = MODE_WALK;
        if (wd.enumerate) {
            const uint64_t idx = (uint64_t)w + (uint64_t)wd.walks * st.trail;
            if (idx >= wd.n_points) {
                st.mode = MODE_DONE;
            } else {
                st.start = (idx % sp.n_half) | ((idx / sp.n_half) << 32);
            }
        } else {
            st.start = start_point(sp, (uint64_t)w, st.trail);
        }
        st.cur = st.start;
    }
    return ev;
}

// `iters` evaluations of f for every walk of slice `block` of `nblocks` (walks (block * WAVES + wave)
// * WPW + group, then every nblocks * WAVES * WPW further).  cnt is the walk group's counts in LDS;
// only the group's leader lane writes it.
template <int NQ, int WAVES>
__device__ void walk_block_single(const SpaceDev& sp, const WalkDev& wd, int iters, Lds<NQ, WAVES>& L, int64_t block,
                                  int64_t nblocks, WalkCounts& cnt) {
    using Gm = Geo<NQ>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gi = lane / Gm::G, gl = lane % Gm::G, gbase = gi * Gm::G;
    const bool leader = gl == 0;
    uint32_t* limbs = L.limbs[wave * Gm::WPW + gi];
    // the frequent events (every distinguished point, most of them inserts) are counted in registers
    // and added to cnt once; the rest go to cnt as they happen
    uint32_t steps = 0, active = 0, dps = 0, ins = 0;
    const int64_t stride = nblocks * WAVES * Gm::WPW;
    for (int64_t base = (block * WAVES + wave) * Gm::WPW; base < wd.walks; base += stride) {
        const int64_t w = base + gi;
        if (w >= wd.walks) continue;
        WalkState st = load_state(wd, w, Gm::G == 64);
        for (int it = 0; it < iters; ++it) {
            if ((st.mode & 0xff) == MODE_DONE) break;
            const uint64_t arg = step_arg(st);
            uint64_t nxt, H;
            walk_step<NQ, WAVES>(sp, L, limbs, arg, gl, gbase, nxt, H);
            steps++;
            const uint32_t ev = advance_walk<Gm::G == 64>(sp, wd, st, w, arg, nxt, H, leader, gbase);
            dps += ev & EV_DP;
            ins += (ev >> 1) & 1;
            const uint32_t rare = ev & ~(uint32_t)(EV_DP | EV_INS);
            if (rare && leader) count_events(cnt, rare);
        }
        if ((st.mode & 0xff) != MODE_DONE) active++;
        if (leader) wd.states[w] = st;
    }
    if (leader) {
        cnt.steps += steps;
        cnt.active += active;
        cnt.dps += dps;
        cnt.ins += ins;
    }
}

// n = 4: each wavefront runs two walks, 2q and 2q + 1 for q = block * WAVES + wave, then every
// nblocks * WAVES further, and gives the pair 2 iters evaluations of f (a walk without a partner
// gets iters); cnt as in walk_block_single.  A walk whose next point is on side 0 steps alone; when both next points are on side
// 1 the two steps share one MFMA product (walk_step_pair4).  So the pair's steps add up to 2 iters
// while each walk's share varies with its sides: a launch's total is walks x iters as before.
template <int WAVES>
__device__ void walk_block_pairs(const SpaceDev& sp, const WalkDev& wd, int iters, Lds<4, WAVES>& L, int64_t block,
                                 int64_t nblocks, WalkCounts& cnt) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool leader = lane == 0;
    uint32_t* limbs = L.limbs[wave];
    uint32_t steps = 0, active = 0, dps = 0, ins = 0;  // frequent events in registers, as in walk_block_single
    const int64_t pairs = (wd.walks + 1) / 2;
    for (int64_t q = block * WAVES + wave; q < pairs; q += nblocks * WAVES) {
        const int64_t w0 = 2 * q, w1 = 2 * q + 1;
        const bool has_b = w1 < wd.walks;
        WalkState sa = load_state(wd, w0, true);
        WalkState sb = has_b ? load_state(wd, w1, true) : sa;
        const int total = has_b ? 2 * iters : iters;
        int left = total;
        while (left > 0) {
            const bool act_a = (sa.mode & 0xff) != MODE_DONE;
            const bool act_b = has_b && (sb.mode & 0xff) != MODE_DONE;
            if (!act_a && !act_b) break;
            const uint64_t arg_a = step_arg(sa), arg_b = step_arg(sb);
            const bool s1a = (arg_a >> 32) & 1, s1b = (arg_b >> 32) & 1;
            uint64_t na = 0, ha = 0, nb = 0, hb = 0;
            bool do_a, do_b;
            if (act_a && act_b && s1a && s1b && left >= 2) {
                walk_step_pair4<WAVES>(sp, L, limbs, arg_a, arg_b, lane, na, ha, nb, hb);
                do_a = do_b = true;
                left -= 2;
            } else {
                // a side-0 step first; otherwise the one walk still stepping (or walk a, on the last step)
                const bool pick_b = !act_a || (act_b && s1a && !s1b);
                uint64_t nx, hh;
                walk_step<4, WAVES>(sp, L, limbs, pick_b ? arg_b : arg_a, lane, 0, nx, hh);
                na = nb = nx;
                ha = hb = hh;
                do_a = !pick_b;
                do_b = pick_b;
                left -= 1;
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (!(k ? do_b : do_a)) continue;
                WalkState st = k ? sb : sa;
                const uint32_t ev =
                    advance_walk<true>(sp, wd, st, k ? w1 : w0, k ? arg_b : arg_a, k ? nb : na, k ? hb : ha, leader, 0);
                dps += ev & EV_DP;
                ins += (ev >> 1) & 1;
                const uint32_t rare = ev & ~(uint32_t)(EV_DP | EV_INS);
                if (rare && leader) count_events(cnt, rare);
                if (k)
                    sb = st;
                else
                    sa = st;
            }
        }
        steps += (uint32_t)(total - left);
        if ((sa.mode & 0xff) != MODE_DONE) active++;
        if (has_b && (sb.mode & 0xff) != MODE_DONE) active++;
        if (leader) {
            wd.states[w0] = sa;
            if (has_b) wd.states[w1] = sb;
        }
    }
    if (leader) {
        cnt.steps += steps;
        cnt.active += active;
        cnt.dps += dps;
        cnt.ins += ins;
    }
}

// The walks of one slice: paired on side 1 at n = 4, one walk group at a time otherwise.
template <int NQ, int WAVES>
__device__ void walk_block(const SpaceDev& sp, const WalkDev& wd, int iters, Lds<NQ, WAVES>& L, int64_t block,
                           int64_t nblocks, WalkCounts& cnt) {
    if constexpr (NQ == 4)
        walk_block_pairs<WAVES>(sp, wd, iters, L, block, nblocks, cnt);
    else
        walk_block_single<NQ, WAVES>(sp, wd, iters, L, block, nblocks, cnt);
}

template <int NQ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_walk(SpaceDev sp, WalkDev wd, int iters) {
    __shared__ Lds<NQ, WAVES> L;
    // one count slot per walk group (raw storage: a __shared__ object cannot have initialisers)
    __shared__ __attribute__((aligned(8))) unsigned char s_cnt[WAVES * Geo<NQ>::WPW * sizeof(WalkCounts)];
    const int lane = threadIdx.x & 63;
    const bool leader = lane % Geo<NQ>::G == 0;
    WalkCounts& mine = reinterpret_cast<WalkCounts*>(s_cnt)[(threadIdx.x >> 6) * Geo<NQ>::WPW + lane / Geo<NQ>::G];
    if (leader) mine = WalkCounts{};
    load_lds(L, sp);
    __syncthreads();
    walk_block<NQ, WAVES>(sp, wd, iters, L, blockIdx.x, gridDim.x, mine);
    flush_counts(wd, mine, leader);
}

// Many members in one persistent launch per qubit count, fed from a device queue: each block takes
// the next item (a slice of one member's walks for that member's number of evaluations) until the
// queue is empty, and reloads the member's S_c and keys into LDS only when the member changes.
// head[0] is the queue position (zeroed by a kernel before the launch); count[0] items are queued.
// Every block leaves once the position passes the count, so the grid always drains.
template <int NQ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_walk_queue(const SpaceDev* __restrict__ sps, const WalkDev* __restrict__ wds,
                                                           const WorkItem* __restrict__ items, const int32_t* count,
                                                           uint32_t* head) {
    __shared__ Lds<NQ, WAVES> L;
    __shared__ int32_t s_next;
    // the loaded member's event counts so far, one slot per walk group, written by the group's leader
    // as events happen (in registers they would hold 22 more VGPRs through the step and spill)
    __shared__ __attribute__((aligned(8))) unsigned char s_cnt[WAVES * Geo<NQ>::WPW * sizeof(WalkCounts)];
    const int32_t n_items = *count;
    const int lane = threadIdx.x & 63;
    const bool leader = lane % Geo<NQ>::G == 0;
    WalkCounts& mine = reinterpret_cast<WalkCounts*>(s_cnt)[(threadIdx.x >> 6) * Geo<NQ>::WPW + lane / Geo<NQ>::G];
    if (leader) mine = WalkCounts{};
    int32_t loaded = -1;
    for (;;) {
        if (threadIdx.x == 0) s_next = (int32_t)atomicAdd(head, 1u);
        __syncthreads();
        // the same value in every thread of the block; read from the first lane so that the item and
        // the member's descriptors are scalar loads
        const int32_t i = __builtin_amdgcn_readfirstlane(s_next);
        if (i >= n_items) break;
        const WorkItem it = items[i];
        // read through the pointer where used (scalar loads; the descriptors are never written during
        // the launch, which __restrict__ tells the compiler, so it may keep or reload them freely)
        const SpaceDev& sp = sps[it.slot];
        if (it.slot != loaded) {
            if (loaded >= 0) flush_counts(wds[loaded], mine, leader);
            load_lds(L, sp);
            loaded = it.slot;
        }
        __syncthreads();
        walk_block<NQ, WAVES>(sp, wds[it.slot], it.iters, L, it.unit, it.units, mine);
        __syncthreads();  // s_next and, for the next member, the LDS are rewritten after this
    }
    if (loaded >= 0) flush_counts(wds[loaded], mine, leader);
}

__global__ void k_walk_init(SpaceDev sp, WalkDev wd) {
    for (int64_t w = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; w < wd.walks;
         w += (int64_t)blockDim.x * gridDim.x) {
        WalkState st;
        st.trail = 0;
        st.len = 0;
        st.mode = MODE_WALK;
        st.rem = 0;
        st.pa = st.pb = st.na = st.ha = 0;
        if (wd.enumerate) {
            const uint64_t idx = (uint64_t)w;
            if (idx >= wd.n_points) {
                st.mode = MODE_DONE;
                st.start = 0;
            } else {
                st.start = (idx % sp.n_half) | ((idx / sp.n_half) << 32);
            }
        } else {
            st.start = start_point(sp, (uint64_t)w, 0);
        }
        st.cur = st.start;
        wd.states[w] = st;
    }
}

// Several batch members restarted in one launch: for member slots[blockIdx.x / RESTART_PER], its
// table cleared (EMPTY_KEY keys; values 0, or ENUM_TABLE_INIT in enumeration mode), its statistics
// and candidate count zeroed and its walk states set as k_walk_init sets them; RESTART_PER blocks
// share each member's work.
constexpr int RESTART_PER = 32;
__global__ __launch_bounds__(256) void k_member_restart(const SpaceDev* sps, const WalkDev* wds,
                                                        const int32_t* slots) {
    const int32_t slot = slots[blockIdx.x / RESTART_PER];
    const SpaceDev sp = sps[slot];
    const WalkDev wd = wds[slot];
    const uint64_t stride = (uint64_t)RESTART_PER * blockDim.x;
    const uint64_t first = (uint64_t)(blockIdx.x % RESTART_PER) * blockDim.x + threadIdx.x;
    const uint64_t value = wd.enumerate ? ENUM_TABLE_INIT : 0;
    const uint64_t nslots = 1ull << wd.log2_table;
    for (uint64_t i = first; i < nslots; i += stride) {
        wd.table[2 * i] = EMPTY_KEY;
        wd.table[2 * i + 1] = value;
    }
    for (uint64_t w = first; w < (uint64_t)wd.walks; w += stride) {
        WalkState st;
        st.trail = 0;
        st.len = 0;
        st.mode = MODE_WALK;
        st.rem = 0;
        st.pa = st.pb = st.na = st.ha = 0;
        if (wd.enumerate) {
            if (w >= wd.n_points) {
                st.mode = MODE_DONE;
                st.start = 0;
            } else {
                st.start = (w % sp.n_half) | ((w / sp.n_half) << 32);
            }
        } else {
            st.start = start_point(sp, w, 0);
        }
        st.cur = st.start;
        wd.states[w] = st;
    }
    if (first < ST_COUNT) wd.stats[first] = 0;
    if (first == 0) *wd.claw_count = 0;
}

__global__ void k_table_clear(uint64_t* table, uint64_t slots, uint64_t value) {
    for (uint64_t i = threadIdx.x + (uint64_t)blockIdx.x * blockDim.x; i < slots;
         i += (uint64_t)blockDim.x * gridDim.x) {
        table[2 * i] = EMPTY_KEY;
        table[2 * i + 1] = value;
    }
}

// After an exhaustive pass (enumeration mode): every key reached from both sides gives one
// candidate, the least x of side 0 against the least x of side 1.
__global__ void k_enum_pairs(WalkDev wd) {
    const uint64_t slots = 1ull << wd.log2_table;
    unsigned long long found = 0;
    for (uint64_t i = threadIdx.x + (uint64_t)blockIdx.x * blockDim.x; i < slots;
         i += (uint64_t)blockDim.x * gridDim.x) {
        if (wd.table[2 * i] == EMPTY_KEY) continue;
        const uint64_t v = wd.table[2 * i + 1];
        const uint32_t x0 = (uint32_t)v, x1 = (uint32_t)(v >> 32);
        if (x0 == ENUM_NONE || x1 == ENUM_NONE) continue;
        ++found;
        const unsigned long long idx = atomicAdd(wd.claw_count, 1ull);
        if (idx < wd.claw_cap) {
            wd.claws[2 * idx] = (uint64_t)x0;
            wd.claws[2 * idx + 1] = (uint64_t)x1 | (1ull << 32);
        }
    }
    if (found) atomicAdd(&wd.stats[ST_CLAWS], found);
}

// ---- meet-in-the-middle labels for the depth-order network ----
// Level table: key = matrix hash H (one salt for every h), value = 255 - (least h that reaches it).
__device__ inline int level_lookup(const uint64_t* table, int log2_table, uint64_t key) {
    const uint64_t mask = (1ull << log2_table) - 1;
    uint64_t s = mix64(key ^ 0x5bd1e9955bd1e995ull) & mask;
    for (int probe = 0; probe < 64; ++probe) {
        const uint64_t k = __hip_atomic_load(&table[2 * s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == key) {
            const uint64_t v = __hip_atomic_load(&table[2 * s + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return v ? 255 - (int)v : -1;
        }
        if (k == EMPTY_KEY) return -1;
        s = (s + 1) & mask;
    }
    return -1;
}

template <int NQ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_mitm_levels(SpaceDev sp, int h, uint64_t* table, int log2_table) {
    using Gm = Geo<NQ>;
    __shared__ Lds<NQ, WAVES> L;
    load_lds(L, sp);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gi = lane / Gm::G, gl = lane % Gm::G, gbase = gi * Gm::G;
    uint32_t* limbs = L.limbs[wave * Gm::WPW + gi];
    sp.h = h;
    const int64_t stride = (int64_t)gridDim.x * WAVES * Gm::WPW;
    for (int64_t base = ((int64_t)blockIdx.x * WAVES + wave) * Gm::WPW; base < (int64_t)sp.n_half; base += stride) {
        const int64_t x = base + gi;
        if (x >= (int64_t)sp.n_half) continue;
        uint64_t o, H;
        walk_step<NQ, WAVES>(sp, L, limbs, (uint64_t)x, gl, gbase, o, H);
        if (gl == 0) {
            const uint64_t key = H == EMPTY_KEY ? (H ^ 1) : H;
            uint64_t slot = 0;
            WalkDev wd{};
            wd.table = table;
            wd.log2_table = log2_table;
            if (table_claim(wd, key, slot) != 3) atomicMax(&table[2 * slot + 1], (uint64_t)(255 - h));
        }
    }
}

// Per target (block): least i + j over side-1 products of j <= h_max rotations from U whose hash is
// in the level table at level i; stops once j reaches the best total.  best_out = -1 if none.
template <int NQ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_mitm_probe(SpaceDev sp0, const uint32_t* phi_all,
                                                           const int32_t* rot_e_all, int count, int h_max,
                                                           const uint64_t* table, int log2_table, int32_t* best_out) {
    using Gm = Geo<NQ>;
    constexpr int NPHI = Gm::Q4 * Gm::R;
    __shared__ Lds<NQ, WAVES> L;
    __shared__ int best;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gi = lane / Gm::G, gl = lane % Gm::G, gbase = gi * Gm::G;
    uint32_t* limbs = L.limbs[wave * Gm::WPW + gi];
    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        SpaceDev sp = sp0;
        sp.phi = phi_all + (size_t)t * 2 * NPHI;
        sp.rot_e = rot_e_all[t];
        __syncthreads();
        load_lds(L, sp);
        if (threadIdx.x == 0) best = 1 << 20;
        __syncthreads();
        uint32_t nh = 1;
        for (int j = 0; j <= h_max; ++j) {
            if (j >= best) break;
            sp.h = j;
            sp.n_half = nh;
            for (int64_t base = (int64_t)wave * Gm::WPW; base < (int64_t)nh; base += WAVES * Gm::WPW) {
                const int64_t x = base + gi;
                if (x >= (int64_t)nh) continue;
                uint64_t o, H;
                walk_step<NQ, WAVES>(sp, L, limbs, (uint64_t)x | (1ull << 32), gl, gbase, o, H);
                if (gl == 0) {
                    const int lvl = level_lookup(table, log2_table, H == EMPTY_KEY ? (H ^ 1) : H);
                    if (lvl >= 0) atomicMin(&best, j + lvl);
                }
            }
            nh *= Gm::XI;
            __syncthreads();
        }
        if (threadIdx.x == 0) best_out[t] = best < (1 << 20) ? best : -1;
    }
}

template <typename F>
hipError_t dispatch_n(int n, F&& f) {
    switch (n) {
        case 1: return f.template operator()<1>();
        case 2: return f.template operator()<2>();
        case 3: return f.template operator()<3>();
        case 4: return f.template operator()<4>();
        default: return hipErrorInvalidValue;
    }
}

int cu_count(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

}  // namespace

int walk_grid_blocks(int n, int device, bool queue, int64_t walks) {
    // one persistent block per CU for n = 4 (the int8 S_c fills most of the 160 KiB LDS); at n = 3 the
    // walk kernel's 71 VGPRs leave room for six 4-wave blocks per CU, which pays with many walks
    // (2^20 walks: 13.8 ms per 3.4e7 steps against 14.4 ms with five) but not with a search's usual
    // 2^16 (the Toffoli search at theta = 1/2: 0.140 s with five, 0.151 s with six); the queue
    // kernel's 88 VGPRs leave room for five
    const int cus = cu_count(device);
    if (n == 3) return cus * (!queue && walks >= (1 << 19) ? 6 : 5);
    return n == 4 ? cus : cus * 4;
}

hipError_t keys_fill(int n, uint64_t seed, uint64_t* keys, hipStream_t s) {
    const int r = 1 << (2 * n);
    hipLaunchKernelGGL(k_keys, dim3((r + 255) / 256), dim3(256), 0, s, r, seed, keys);
    return hipGetLastError();
}

hipError_t rot_keys_fill(const uint64_t* keys, uint64_t* rkeys, hipStream_t s) {
    hipLaunchKernelGGL(k_rot_keys, dim3(512), dim3(256), 0, s, keys, rkeys);
    return hipGetLastError();
}

hipError_t rot_keys2_fill(const uint64_t* rkeys, uint64_t* rkeys2, hipStream_t s) {
    hipLaunchKernelGGL(k_rot_keys2, dim3(2 * 256 * 256), dim3(256), 0, s, rkeys, rkeys2);
    return hipGetLastError();
}

hipError_t launch_step(int n, const SpaceDev& sp, const uint64_t* in, uint64_t* out, uint64_t* hash, int64_t count,
                       hipStream_t s) {
    if (count <= 0) return hipSuccess;
    auto f = [&]<int NQ>() -> hipError_t {
        constexpr int W = WalkWaves<NQ>::value;
        const int64_t per_block = (int64_t)W * Geo<NQ>::WPW;
        int64_t blocks = (count + per_block - 1) / per_block;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL((k_step<NQ, W>), dim3((unsigned)blocks), dim3(W * 64), 0, s, sp, in, out, hash, count);
        return hipGetLastError();
    };
    return dispatch_n(n, f);
}

hipError_t launch_trails(int n, const SpaceDev& sp, const uint64_t* starts, int64_t count, uint32_t cap, uint64_t* dp,
                         uint32_t* len, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    auto f = [&]<int NQ>() -> hipError_t {
        constexpr int W = WalkWaves<NQ>::value;
        const int64_t per_block = (int64_t)W * Geo<NQ>::WPW;
        int64_t blocks = (count + per_block - 1) / per_block;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL((k_trails<NQ, W>), dim3((unsigned)blocks), dim3(W * 64), 0, s, sp, starts, count, cap,
                           dp, len);
        return hipGetLastError();
    };
    return dispatch_n(n, f);
}

hipError_t launch_starts(const SpaceDev& sp, int64_t w0, uint32_t j, int64_t count, uint64_t* out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_starts, dim3((unsigned)blocks), dim3(256), 0, s, sp, w0, j, count, out);
    return hipGetLastError();
}

hipError_t pack_phi_i32(int n, const int32_t* a, const int32_t* b, int64_t count, uint32_t* phi, int* flag,
                        hipStream_t s) {
    auto f = [&]<int NQ>() -> hipError_t {
        hipLaunchKernelGGL((k_pack_i32<NQ>), dim3(1024), dim3(256), 0, s, a, b, count, phi, flag);
        return hipGetLastError();
    };
    return dispatch_n(n, f);
}

hipError_t launch_canon_hash(int n, const SpaceDev& sp, const uint32_t* phi_all, const int32_t* e, int64_t count,
                             uint64_t* out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    auto f = [&]<int NQ>() -> hipError_t {
        constexpr int W = WalkWaves<NQ>::value;
        const int64_t blocks = count < 1024 ? count : 1024;
        hipLaunchKernelGGL((k_canon<NQ, W>), dim3((unsigned)blocks), dim3(W * 64), 0, s, sp, phi_all, e, count,
                           out);
        return hipGetLastError();
    };
    return dispatch_n(n, f);
}

hipError_t launch_canon_wide(int n, const SpaceDev& sp, const int32_t* a, const int32_t* b, const int32_t* e,
                             int64_t count, uint64_t* out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    auto f = [&]<int NQ>() -> hipError_t {
        const int64_t blocks = count < 4096 ? count : 4096;
        hipLaunchKernelGGL((k_canon_wide<NQ>), dim3((unsigned)blocks), dim3(64), 0, s, sp, a, b, e, count, out);
        return hipGetLastError();
    };
    return dispatch_n(n, f);
}

hipError_t launch_walk(int n, const SpaceDev& sp, const WalkDev& wd, int iters, int grid_blocks, hipStream_t s) {
    auto f = [&]<int NQ>() -> hipError_t {
        constexpr int W = WalkWaves<NQ>::value;
        const int64_t per_block = (int64_t)W * Geo<NQ>::WPW;
        int64_t blocks = (wd.walks + per_block - 1) / per_block;
        if (blocks > grid_blocks) blocks = grid_blocks;
        hipLaunchKernelGGL((k_walk<NQ, W>), dim3((unsigned)blocks), dim3(W * 64), 0, s, sp, wd, iters);
        return hipGetLastError();
    };
    return dispatch_n(n, f);
}

hipError_t launch_walk_queue(int n, const SpaceDev* sps, const WalkDev* wds, const WorkItem* items,
                             const int32_t* count, uint32_t* head, int blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    auto f = [&]<int NQ>() -> hipError_t {
        constexpr int W = WalkWaves<NQ>::value;
        hipLaunchKernelGGL((k_walk_queue<NQ, W>), dim3((unsigned)blocks), dim3(W * 64), 0, s, sps, wds, items, count,
                           head);
        return hipGetLastError();
    };
    return dispatch_n(n, f);
}

int walks_per_block(int n) {
    switch (n) {
        case 1: return WalkWaves<1>::value * Geo<1>::WPW;
        case 2: return WalkWaves<2>::value * Geo<2>::WPW;
        case 3: return WalkWaves<3>::value * Geo<3>::WPW;
        default: return WalkWaves<4>::value * Geo<4>::WPW;
    }
}

hipError_t launch_walk_init(const SpaceDev& sp, const WalkDev& wd, hipStream_t s) {
    int64_t blocks = (wd.walks + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_walk_init, dim3((unsigned)blocks), dim3(256), 0, s, sp, wd);
    return hipGetLastError();
}

hipError_t launch_member_restart(const SpaceDev* sps, const WalkDev* wds, const int32_t* slots, int count,
                                 hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_member_restart, dim3((unsigned)(count * RESTART_PER)), dim3(256), 0, s, sps, wds, slots);
    return hipGetLastError();
}

hipError_t launch_table_clear(uint64_t* table, int log2_table, uint64_t value, hipStream_t s) {
    const uint64_t slots = 1ull << log2_table;
    uint64_t blocks = (slots + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_table_clear, dim3((unsigned)blocks), dim3(256), 0, s, table, slots, value);
    return hipGetLastError();
}

hipError_t launch_enum_pairs(const WalkDev& wd, hipStream_t s) {
    const uint64_t slots = 1ull << wd.log2_table;
    uint64_t blocks = (slots + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_enum_pairs, dim3((unsigned)blocks), dim3(256), 0, s, wd);
    return hipGetLastError();
}

}  // namespace tcw

namespace tcw {

hipError_t mitm_levels(int n, const SpaceDev& sp, int h, uint64_t* table, int log2_table, hipStream_t s) {
    auto f = [&]<int NQ>() -> hipError_t {
        constexpr int W = WalkWaves<NQ>::value;
        if constexpr (NQ <= 3) {
            int64_t blocks = ((int64_t)sp.n_half + W * Geo<NQ>::WPW - 1) / (W * Geo<NQ>::WPW);
            if (blocks > 4096) blocks = 4096;
            if (blocks < 1) blocks = 1;
            hipLaunchKernelGGL((k_mitm_levels<NQ, W>), dim3((unsigned)blocks), dim3(W * 64), 0, s, sp, h, table,
                               log2_table);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    };
    return dispatch_n(n, f);
}

hipError_t mitm_probe(int n, const SpaceDev& sp, const uint32_t* phi_all, const int32_t* rot_e_all, int count,
                      int h_max, const uint64_t* table, int log2_table, int32_t* best_out, hipStream_t s) {
    auto f = [&]<int NQ>() -> hipError_t {
        constexpr int W = WalkWaves<NQ>::value;
        if constexpr (NQ <= 3) {
            const int blocks = count < 4096 ? count : 4096;
            hipLaunchKernelGGL((k_mitm_probe<NQ, W>), dim3(blocks), dim3(W * 64), 0, s, sp, phi_all, rot_e_all, count,
                               h_max, table, log2_table, best_out);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    };
    return dispatch_n(n, f);
}

}  // namespace tcw
