// Device-side arithmetic shared by the walk and exact kernels (gfx950, wave64).
//
// * SplitMix64 (Steele, Lea, Flood 2014) in counter form: sm64(s, i) = mix64(s + (i+1) GAMMA).
// * Z/p with p = 2^61 - 1 (a Mersenne prime): the row digest of the walk hash lives here.
//   2 is a square mod p: (2^31)^2 = 2^62 = 2 (mod p), so phi(sqrt2) = 2^31 and phi(1/sqrt2) = 2^30,
//   and multiplying by a power of two is a 61-bit rotation.
// * Pauli codes: x = q & (2^n - 1), z = q >> n (Sec. 4.1, binary symplectic form).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tcw {

constexpr uint64_t P61 = (1ull << 61) - 1;
constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;
constexpr uint64_t EMPTY_KEY = ~0ull;
constexpr int NLIMB = 9;      // 7-bit limbs of a 61-bit residue for the int8 dot products
constexpr int LIMB_STRIDE = 12;  // dwords per 4-column group in the limb buffer (16-byte aligned)

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t sm64(uint64_t seed, uint64_t i) { return mix64(seed + (i + 1) * GAMMA); }

__device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// ---- Z/(2^61 - 1); operands in [0, P61] (P61 itself stands for zero) ----
__device__ inline uint64_t m61_fold(uint64_t s) {
    s = (s & P61) + (s >> 61);
    return (s & P61) + (s >> 61);
}
__device__ inline uint64_t m61_add(uint64_t a, uint64_t b) { return m61_fold(a + b); }
__device__ inline uint64_t m61_sub(uint64_t a, uint64_t b) { return m61_fold(a + (P61 - b)); }
// x * 2^s mod p for 0 <= s < 61
__device__ inline uint64_t m61_rot(uint64_t x, int s) {
    return s == 0 ? x : (((x << s) | (x >> (61 - s))) & P61);
}
__device__ inline uint64_t m61_canon(uint64_t x) { return x == P61 ? 0 : x; }
// signed 32-bit integer to Z/p
__device__ inline uint64_t m61_from_i32(int32_t v) {
    return v >= 0 ? (uint64_t)v : P61 - (uint64_t)(-(int64_t)v);
}

// ---- Paulis ----
template <int NQ>
__host__ __device__ inline int anticommutes(uint32_t p, uint32_t q) {
    constexpr uint32_t M = (1u << NQ) - 1;
    const uint32_t xp = p & M, zp = p >> NQ, xq = q & M, zq = q >> NQ;
    return (__builtin_popcount(xp & zq) + __builtin_popcount(zp & xq)) & 1;
}

// c mod 4 with P_p P_q = i^c P_{p^q}
template <int NQ>
__host__ __device__ inline int product_phase(uint32_t p, uint32_t q) {
    constexpr uint32_t M = (1u << NQ) - 1;
    const uint32_t xp = p & M, zp = p >> NQ, xq = q & M, zq = q >> NQ;
    const int c = __builtin_popcount(xp & zp) + __builtin_popcount(xq & zq) -
                  __builtin_popcount((xp ^ xq) & (zp ^ zq)) + 2 * __builtin_popcount(zp & xq);
    return c & 3;
}

// s(p, q) = +1 if c = 1, -1 if c = 3: the column rule of the channel rep of R(P_p)
// (R(P) P_q R(P)^dag = (P_q + s P_{p^q}) / sqrt2 for anticommuting p, q).
template <int NQ>
__host__ __device__ inline int rotation_sign(uint32_t p, uint32_t q) {
    return product_phase<NQ>(p, q) == 1 ? 1 : -1;
}

// ---- wave-level exchange (ds_bpermute; src lane index in the wave) ----
__device__ inline uint32_t shfl32(uint32_t v, int src_lane) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)v);
}
__device__ inline uint64_t shfl64(uint64_t v, int src_lane) {
    const uint32_t lo = shfl32((uint32_t)v, src_lane);
    const uint32_t hi = shfl32((uint32_t)(v >> 32), src_lane);
    return ((uint64_t)hi << 32) | lo;
}

}  // namespace tcw
