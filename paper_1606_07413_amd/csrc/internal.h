// Internal structures shared by the host driver (api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace tcw {

// One search space (target x depth k x chunk x function version), as the walk kernels see it.
struct SpaceDev {
    uint32_t n_half;    // xi^h, points per side
    int32_t h;          // rotations per half
    int32_t delta;      // theta = 2^-delta
    int32_t rot_e;      // (30 * e_S) mod 61: multiplication by phi(1/sqrt2)^e_S in Z/p
    uint64_t salt_h;    // matrix-hash salt
    uint64_t salt_d;    // distinguished-point salt
    uint64_t salt_s;    // trail-start salt
    const uint32_t* phi;   // S_c as int8: A packed [q4][r] dwords, then B packed the same way
    const uint64_t* keys;  // K[R] (row-digest keys, < p)
    const uint64_t* rkeys; // n = 4, or null: the first rotation of a step applied to K for every Pauli,
                           // [side][p][q] = (R(p) K)_q (side 0), (R(p)^T K)_q (side 1); 2 x 256 x 256
    const uint64_t* rkeys2;  // n = 4, or null: the first two, [side][p][p'][q] = (R(p') R(p) K)_q
                             // (side 0; transposes for side 1), p applied first; 2 x 256^3 values
};

enum : uint32_t { MODE_WALK = 0, MODE_ALIGN = 1, MODE_LOCK = 2, MODE_DONE = 3 };

// Enumeration tables keep, per key, the least x of side 0 and of side 1 in the low and high halves of
// the value; ENUM_NONE marks a side that has not reached the key (x < xi^h < 2^32 - 1).
constexpr uint32_t ENUM_NONE = 0xffffffffu;
constexpr uint64_t ENUM_TABLE_INIT = ~0ull;

// 64-byte walk state, kept in HBM between launches.
struct WalkState {
    uint64_t start;  // start point of the current trail
    uint64_t cur;    // WALK: current point
    uint64_t pa;     // backtracking: point on the own trail
    uint64_t pb;     // backtracking: point on the stored trail
    uint64_t na;     // LOCK phase 1: f(pa)
    uint64_t ha;     // LOCK phase 1: matrix hash of pa
    uint32_t len;    // WALK: steps in the trail; backtracking: common remaining length
    uint32_t trail;  // trail index j
    uint32_t mode;   // MODE_*; bit 8: which point ALIGN advances / LOCK phase
    uint32_t rem;    // ALIGN / LOCK: steps left
};
static_assert(sizeof(WalkState) == 64, "walk state is 64 bytes");

enum StatIdx {
    ST_STEPS = 0, ST_DPS, ST_INSERTS, ST_ABANDONED, ST_ROBIN, ST_SAME, ST_REDUCTION, ST_CLAWS,
    ST_FULL, ST_SPIN, ST_ACTIVE, ST_COUNT
};

struct WalkDev {
    WalkState* states;
    int64_t walks;
    uint64_t* table;            // 2^log2_table slots of (key, value) u64 pairs
    int32_t log2_table;
    uint32_t cap;               // trail cap
    int32_t enumerate;          // 1: trail j of walk w starts at point w + walks * j
    uint64_t n_points;          // 2 * n_half
    unsigned long long* stats;  // ST_COUNT counters
    uint64_t* claws;            // claw candidate pairs (u0, u1)
    unsigned long long* claw_count;
    uint32_t claw_cap;
};

// ---- launchers (exact.hip) ----
// Exact matrices live on the device as int32 pairs (int64 for n <= 2) with exponent e.
struct ExactDev {
    int n = 0;
    int r = 0;
    void* a = nullptr;   // R*R elements of int32 (n >= 3) or int64 (n <= 2)
    void* b = nullptr;
    int32_t* e = nullptr;  // device scalar exponent
    size_t elem = 0;       // element size in bytes
};

hipError_t exact_alloc(ExactDev& m, int n);
void exact_free(ExactDev& m);
// m = prod_j R(C_j)^2 * R(P_k) ... R(P_1) (seq given as right-multiplications), reduced.
hipError_t exact_build(ExactDev& m, const uint16_t* seq_dev, const uint8_t* transpose_dev, int nseq,
                       int* flag_dev, hipStream_t s);
// dst = src * R(seq[0])^(T?) * ... , reduced; dst and src may alias.
hipError_t exact_apply(ExactDev& dst, const ExactDev& src, const uint16_t* seq_dev, const uint8_t* transpose_dev,
                       int nseq, int* flag_dev, hipStream_t s);
// as exact_apply, with the two R x R work matrices given (ta, tb) instead of allocated, and no
// synchronisation
hipError_t exact_apply_ws(ExactDev& dst, const ExactDev& src, const uint16_t* seq, const uint8_t* tr, int nseq,
                          void* ta, void* tb, int* flag, hipStream_t s);
// dst = src * R(p)^(T if transposed), reduced, for dst distinct from src: the result of exact_apply
// with a one-rotation word, on many blocks and without work matrices; m_tmp is one device int32 of
// scratch.  No synchronisation.
hipError_t exact_rotate1(ExactDev& dst, const ExactDev& src, uint32_t p, int transposed, int32_t* m_tmp, int* flag,
                         hipStream_t s);
// seq[0] = p, tr[0] = transpose (a one-rotation word on the device, written by a kernel)
hipError_t exact_seq_one(uint16_t* seq, uint8_t* tr, uint16_t p, uint8_t transpose, hipStream_t s);
// dst[0..count) = v by a kernel (no memset node, so it may sit in captured work)
hipError_t fill_i32(int* dst, int v, int count, hipStream_t s);
// load int32 host-provided values already on the device
hipError_t exact_from_i32(ExactDev& m, const int32_t* a_dev, const int32_t* b_dev, int32_t e, int* flag_dev,
                          hipStream_t s);
hipError_t exact_to_i32(const ExactDev& m, int32_t* a_dev, int32_t* b_dev, int* flag_dev, hipStream_t s);
// m = channel rep of U = V / sqrt2^e (V: d x d entries of Z[w], 4 int64 coefficients each, device),
// reduced.  a_tmp, b_tmp: R*R int32 each.  flag bits: 8 V V^dag != 2^e I, 1 an entry not real,
// 4 an entry out of range.  Needs n + e <= 29 and |coefficients| <= 2^20 (checked by the caller).
hipError_t exact_from_unitary(ExactDev& m, const int64_t* v_dev, int32_t e, int32_t* a_tmp, int32_t* b_tmp,
                              int* flag_dev, hipStream_t s);
// flag |= 1 if X X^T != 2^e I
hipError_t exact_check_orthogonal(const ExactDev& m, int* flag_dev, hipStream_t s);
// ok/perm/sign of a reduced matrix being a signed permutation
hipError_t exact_signed_perm(const ExactDev& m, int32_t* ok_dev, int32_t* perm_dev, int8_t* sign_dev, hipStream_t s);
// int8 packing of S for the walk kernels; flag |= 2 if a value is outside [-127, 127]
hipError_t exact_pack_phi(const ExactDev& m, uint32_t* phi_dev, int* flag_dev, hipStream_t s);
// claw checks: for each pair (u0, u1) compute V, W exactly and D = W V^T
hipError_t exact_claw_check(const ExactDev& S, int k, const uint64_t* u0, const uint64_t* u1, int64_t count,
                            void* scratch, size_t scratch_bytes, int32_t* ok, int32_t* perm, int8_t* sign,
                            hipStream_t s);
size_t exact_claw_scratch_bytes(int n);
// canonical FP32 features (n <= 3)
hipError_t exact_features(const ExactDev& m, float* out_dev, hipStream_t s);
// many targets from words: phi (n <= 3 int8 layout), rot_e, features; flag |= 2 / 4 / 8 on range errors
size_t build_batch_scratch_bytes(int n, int blocks);
hipError_t build_batch(int n, const uint16_t* words, const int32_t* offsets, const int32_t* kof, int count,
                       void* scratch, int blocks, uint32_t* phi_out, int32_t* rot_e_out, float* feat_out, int* flag,
                       hipStream_t s);
// meet-in-the-middle level table and probes (walk.hip)
hipError_t mitm_levels(int n, const SpaceDev& sp, int h, uint64_t* table, int log2_table, hipStream_t s);
hipError_t mitm_probe(int n, const SpaceDev& sp, const uint32_t* phi_all, const int32_t* rot_e_all, int count,
                      int h_max, const uint64_t* table, int log2_table, int32_t* best_out, hipStream_t s);

// ---- launchers (walk.hip) ----
hipError_t keys_fill(int n, uint64_t seed, uint64_t* keys_dev, hipStream_t s);
// n = 4: the rotated keys of SpaceDev::rkeys (2 x 256 x 256 values) from K.
hipError_t rot_keys_fill(const uint64_t* keys, uint64_t* rkeys, hipStream_t s);
// n = 4: SpaceDev::rkeys2 (2 x 256^3 values) from SpaceDev::rkeys.
hipError_t rot_keys2_fill(const uint64_t* rkeys, uint64_t* rkeys2, hipStream_t s);
hipError_t launch_step(int n, const SpaceDev& sp, const uint64_t* in, uint64_t* out, uint64_t* hash, int64_t count,
                       hipStream_t s);
hipError_t launch_trails(int n, const SpaceDev& sp, const uint64_t* starts, int64_t count, uint32_t cap,
                         uint64_t* dp, uint32_t* len, hipStream_t s);
hipError_t launch_starts(const SpaceDev& sp, int64_t w0, uint32_t j, int64_t count, uint64_t* out, hipStream_t s);
hipError_t launch_canon_hash(int n, const SpaceDev& sp, const uint32_t* phi_all, const int32_t* e, int64_t count,
                             uint64_t* out, hipStream_t s);
// canonical hash of matrices with entries of any int32 value (64-bit modular row digests)
hipError_t launch_canon_wide(int n, const SpaceDev& sp, const int32_t* a, const int32_t* b, const int32_t* e,
                             int64_t count, uint64_t* out, hipStream_t s);
hipError_t launch_walk(int n, const SpaceDev& sp, const WalkDev& wd, int iters, int grid_blocks, hipStream_t s);
hipError_t launch_walk_init(const SpaceDev& sp, const WalkDev& wd, hipStream_t s);
// One item of the batch work queue: `iters` evaluations of f for slice `unit` of `units` of the walks
// of member `slot` (the slice of walk_block(..., unit, units)).
struct WorkItem {
    int32_t slot, unit, units, iters;
};
// persistent queue kernel of qubit count n over `blocks` blocks (see k_walk_queue)
hipError_t launch_walk_queue(int n, const SpaceDev* sps, const WalkDev* wds, const WorkItem* items,
                             const int32_t* count, uint32_t* head, int blocks, hipStream_t s);
int walks_per_block(int n);
// value: what every slot's value word starts at (0 for walk tables: "not ready"; ENUM_TABLE_INIT for
// enumeration tables: no x on either side)
hipError_t launch_table_clear(uint64_t* table, int log2_table, uint64_t value, hipStream_t s);
// restart batch members slots[0..count) in one launch (descriptors already on the device): each
// member's table cleared, statistics and candidate count zeroed, walk states initialised
hipError_t launch_member_restart(const SpaceDev* sps, const WalkDev* wds, const int32_t* slots, int count,
                                 hipStream_t s);
// enumeration mode, after the last point: one claw candidate per key reached from both sides
hipError_t launch_enum_pairs(const WalkDev& wd, hipStream_t s);
int walk_grid_blocks(int n, int device, bool queue, int64_t walks);
hipError_t pack_phi_i32(int n, const int32_t* a, const int32_t* b, int64_t count, uint32_t* phi_out,
                        int* flag_dev, hipStream_t s);

// ---- depth-order network (mlp.hip) ----
// C = A B^T: A (M x K) and B (N x K) bf16 with K-contiguous rows (leading dimensions multiples of 8),
// FP32 accumulation.  epi 0: C = acc; 1: C = acc + bias; 2: C = Z = acc + bias, H = gelu(Z) (bf16, ld
// ldh) and, if T != null, T = H^T (bf16, ld ldt); 3: C = acc * gelu'(Z) (Z fp32, ld ldz), H = C (bf16),
// T = H^T if T != null.  C is fp32 with leading dimension ldc.  When the output has few tiles, K is
// split over workgroups and part (mlp_gemm_part_floats(M, N, K) floats) holds the partial products,
// summed in a fixed order; with a smaller workspace one workgroup takes each tile.  Products on one
// stream may share the workspace.
size_t mlp_gemm_part_floats(int M, int N, int K);
// workspace floats of mlp_colsum over a rows x cols matrix
size_t mlp_colsum_part_floats(int rows, int cols);
hipError_t mlp_gemm_nt(int epi, const void* A, int lda, const void* B, int ldb, int M, int N, int K, float* C, int ldc,
                       const float* bias, const float* Z, int ldz, void* H, int ldh, void* T, int ldt, float* part,
                       size_t part_floats, hipStream_t s);
// probabilities, loss sum and G = (p - onehot) / batch (fp32; bf16 with ld ldgb; transposed bf16 if gt)
hipError_t mlp_softmax_ce(const float* logits, const int32_t* labels, int batch, int classes, float* probs, float* g,
                          void* gb, int ldgb, void* gt, int ldgt, float* loss_sum, hipStream_t s);
// out[c] = sum over rows of g[r][c], in a fixed order; part: mlp_colsum_part_floats(rows, cols) floats
hipError_t mlp_colsum(const float* g, int rows, int cols, float* out, float* part, size_t part_floats,
                      hipStream_t s);
// x (rows x cols fp32) -> bf16 (ld ldy) and, if t != null, its transpose (ld ldt)
hipError_t mlp_input_bf16(const float* x, int rows, int cols, void* y, int ldy, void* t, int ldt, hipStream_t s);
// W (rows x cols fp32) -> bf16 W (ld ldb) and bf16 W^T (ld ldt)
hipError_t mlp_weights_bf16(const float* w, int rows, int cols, void* wb, int ldb, void* wt, int ldt, hipStream_t s);
hipError_t mlp_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1, float b2,
                    float eps, int step, hipStream_t s);
hipError_t mlp_init(float* w, int64_t count, int64_t index0, int fan_in, uint64_t seed, hipStream_t s);

}  // namespace tcw
