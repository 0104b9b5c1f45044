/*
 * tcw.h -- C ABI of the deterministic-walk T-count synthesis library for MI355X (gfx950).
 *
 * Method: Di Matteo & Mosca, "Parallelizing quantum circuit synthesis" (arXiv:1606.07413).
 * Problem (Sec. 4.1, the T-count decomposition): given the channel representation U_hat of an
 * n-qubit Clifford+T unitary U, find Paulis P_1..P_t and a Clifford D with
 *     U = e^{i phi} D R(P_t) ... R(P_1),   R(P) = (1 + w)/2 I + (1 - w)/2 P,  w = e^{i pi/4},
 * t (the T-count) as small as the depth order allows.  (The paper writes the Clifford on the right;
 * the left form used here is equivalent: conjugating D through R(P) gives R(+-P') and
 * R(-Q) = (Clifford commuting with R(Q)) R(Q).)
 * The search is the parallel claw search of Sec. 3: meet-in-the-middle halves of floor(k/2)
 * rotations, a walk function f(x, b) = z_b(x), distinguished points with fraction
 * theta = 2^-delta, a shared table of trail end points and backtracking of merged trails.
 *
 * Conventions shared by every call
 *  - Pauli code q in [0, 4^n): x = q mod 2^n, z = q >> n, qubit j carries bit j of x and z, qubit 0
 *    is the leftmost Kronecker factor.  Channel-rep rows and columns are indexed by this code
 *    (U_hat_ij = 2^-n Tr(P_i U P_j U^dag), Sec. 4.1).
 *  - Exact matrices: M = (A + B sqrt2) / sqrt2^e, A and B int32 row-major 4^n x 4^n, e >= 0.
 *  - Walk points (uint64): x in bits 0..31 (x < xi^h, xi = 4^n - 1, h = floor(k/2)), side b in bit 32
 *    (0: half-circuits from the identity, the paper's V side; 1: from the target, the W side).
 *  - Every pointer named *_dev is device memory (e.g. a torch CUDA tensor's data_ptr) borrowed for
 *    the call; work is enqueued on the context's stream and is asynchronous unless stated.  Host
 *    pointers are read or written before the call returns.
 *  - Return codes: TCW_OK or a negative TCW_E*; tcw_last_error() then describes the failure.  No
 *    C++ exception crosses this boundary.  One context per host thread.
 */
#ifndef TCW_H
#define TCW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TCW_OK 0
#define TCW_EINVAL (-1)    /* bad argument: n, k, chunk, sizes, a matrix that is not orthogonal */
#define TCW_ENOMEM (-2)    /* device or host allocation failed */
#define TCW_EDEVICE (-3)   /* a HIP runtime error (message in tcw_last_error) */
#define TCW_EOVERFLOW (-4) /* an exact value outside the proven int32/int8 range of the kernels */
#define TCW_ESTATE (-5)    /* call out of order (e.g. a finished walk session) */

#define TCW_MAX_T 64
#define TCW_MAX_R 256

typedef struct tcw_ctx tcw_ctx;
typedef struct tcw_target tcw_target;
typedef struct tcw_walk tcw_walk;

/* ---- context ------------------------------------------------------------------------------
 * tcw_create: bind to HIP device `device`; `hip_stream` (a hipStream_t, may be NULL for the null
 * stream) is borrowed, e.g. torch.cuda.current_stream().cuda_stream.  The context owns the device
 * buffers it allocates; among them, for n = 4, the rotated-key tables of up to 32 search seeds
 * (257 MiB each), kept for later searches with the same seed and released by tcw_destroy.  It also
 * keeps the device buffers of finished batch members and concurrently searched chunks (S_c, keys,
 * walk states, tables; at most 40 GiB) for later members of the same sizes, also until tcw_destroy.
 * tcw_last_error's string is owned by the context and valid until the next call on it. */
int tcw_create(tcw_ctx** out, int device, void* hip_stream);
int tcw_destroy(tcw_ctx* ctx);
const char* tcw_last_error(const tcw_ctx* ctx);
int tcw_set_stream(tcw_ctx* ctx, void* hip_stream);

/* ---- targets (Sec. 4.1, channel representation) ------------------------------------------
 * tcw_target_from_words: U_hat = D_hat R_hat(P_k) ... R_hat(P_1) with D_hat = prod_j R_hat(C_j)^2,
 * built exactly on the GPU.  paulis = [P_1..P_k] (host, each in 1..4^n-1), clifford = [C_1..C_m].
 * tcw_target_from_channel: A, B host arrays (R x R, R = 4^n) and e; validated on the GPU
 * (X X^T = 2^e I exactly with X = A + B sqrt2), TCW_EINVAL if not orthogonal.
 * The target owns a device copy; it must be freed with tcw_target_free before its context. */
int tcw_target_from_words(tcw_ctx* ctx, int n, const uint16_t* paulis, int k, const uint16_t* clifford,
                          int m, tcw_target** out);
int tcw_target_from_channel(tcw_ctx* ctx, int n, const int32_t* a, const int32_t* b, int32_t e,
                            tcw_target** out);
/* tcw_target_from_unitary: the target given as a unitary U = V / sqrt2^e (Sec. 4.1), V a d x d
 * host array (d = 2^n, row-major) of elements of Z[w], w = e^{i pi/4}, each as four int64
 * coefficients (c0, c1, c2, c3) = c0 + c1 w + c2 w^2 + c3 w^3, so v[(r d + c) 4 + j] = c_j of U's
 * entry (r, c); qubit 0 is the most significant bit of a basis index.  The channel rep
 * U_hat_ij = 2^-n Tr(P_i U P_j U^dag) (Sec. 4.1) is evaluated on the GPU entry by entry, exactly.
 * TCW_EINVAL if n is not in 1..4, e < 0 or n + e > 29, a coefficient lies outside [-2^20, 2^20],
 * or V V^dag != 2^e I; the input is copied. */
int tcw_target_from_unitary(tcw_ctx* ctx, int n, const int64_t* v, int32_t e, tcw_target** out);
/* tcw_target_random: a seeded synthetic target U_hat = D_hat R_hat(P_k) ... R_hat(P_1), D_hat =
 * prod_{j=1}^{16 n} R_hat(C_j)^2 (R(C)^2 is a Clifford, Sec. 4.1), built exactly on the GPU.  The
 * Paulis come from SplitMix64 (Steele, Lea and Flood, 2014) in counter form, r_i = mix64(seed +
 * (i + 1) 0x9E3779B97F4A7C15): P_j = floor(r_{j-1} xi / 2^64) + 1 for j = 1..k, then C_j the same from
 * r_{k + j - 1}, xi = 4^n - 1.  gen_paulis (host, k entries, may be NULL) receives P_1..P_k;
 * gen_perm and gen_sign (host, 4^n entries each, may be NULL) receive D: D P_q D^dag =
 * gen_sign[q] P_{gen_perm[q]}.  TCW_EINVAL if n is not in 1..4 or k is not in 0..TCW_MAX_T. */
int tcw_target_random(tcw_ctx* ctx, int n, int k, uint64_t seed, tcw_target** out, uint16_t* gen_paulis,
                      int32_t* gen_perm, int8_t* gen_sign);
int tcw_target_free(tcw_target* t);
/* Copy the reduced exact channel rep to host arrays a, b (R*R each) and *e.  Blocking. */
int tcw_target_channel(tcw_ctx* ctx, const tcw_target* t, int32_t* a, int32_t* b, int32_t* e);
int tcw_target_n(const tcw_target* t);

/* ---- one search space: target x depth k x chunk (Sec. 3) ---------------------------------
 * k >= 1; chunk = 0 for even k, 1..xi for odd k (S_c = U_hat R_hat(c)^T fixes P_1 = c).
 * seed: search seed (hash keys, salts, trail starts); version: function version (re-salting);
 * delta: theta = 2^-delta (0 marks every point distinguished). */
typedef struct tcw_space {
    int32_t k;
    int32_t chunk;
    uint64_t seed;
    uint32_t version;
    int32_t delta;
} tcw_space;

/* The per-point calls below (tcw_step, tcw_trails, tcw_start_points, tcw_canon_hash,
 * tcw_claw_check) take count = 0 as a no-op that still validates the space; their arrays may then
 * be NULL.  Otherwise every array pointer must be valid for `count` entries (NULL: TCW_EINVAL). */

/* tcw_step (parity): pts_out[i] = f(pts_in[i]) and, if hash_out_dev != NULL, the matrix hash H of
 * pts_in[i] (Sec. 3, f(x, b) = z_b(x); Sec. 2, h o nu o mu).  Device arrays of `count` entries. */
int tcw_step(tcw_ctx* ctx, const tcw_target* t, const tcw_space* sp, const uint64_t* pts_in_dev,
             uint64_t* pts_out_dev, uint64_t* hash_out_dev, int64_t count);

/* tcw_step_noalloc: for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  The same outputs as tcw_step, bit for bit, from
 * the same arguments, with every per-call buffer (the chunk matrix S_c and the two work matrices of
 * its construction, its int8 packing, the keys) in one fixed device array of
 * TCW_STEP_NOALLOC_SCRATCH bytes that the library holds on each device it runs on until the process
 * ends; it calls no allocating routine.  At n = 4 its steps apply every rotation themselves instead
 * of reading the context's rotated-key tables.  Calls that overlap on one device share that array and
 * race: serialise them (one call at a time per device, across contexts and threads).  Blocking (it
 * reads S_c's exponent and the range flag back).  Errors as for tcw_step; TCW_EINVAL for a space
 * whose buffers exceed the array (none with n <= 4 does); TCW_EDEVICE if the array's device address
 * could not be obtained when the context was created. */
#define TCW_STEP_NOALLOC_SCRATCH 1182464
int tcw_step_noalloc(tcw_ctx* ctx, const tcw_target* t, const tcw_space* sp, const uint64_t* pts_in_dev,
                     uint64_t* pts_out_dev, uint64_t* hash_out_dev, int64_t count);

/* tcw_trails (parity): from each start, apply f until the next point is distinguished (Sec. 3).
 * dp_out_dev[i] = that point, len_out_dev[i] = steps taken (>= 1); len 0 = no distinguished point
 * within `cap` steps (trail abandoned; dp_out undefined). */
int tcw_trails(tcw_ctx* ctx, const tcw_target* t, const tcw_space* sp, const uint64_t* starts_dev,
               int64_t count, uint32_t cap, uint64_t* dp_out_dev, uint32_t* len_out_dev);

/* tcw_start_points: start of trail j for walk w (Sec. 3, random starting pairs), for
 * w = w0 .. w0+count-1 at fixed j, into pts_out_dev. */
int tcw_start_points(tcw_ctx* ctx, const tcw_target* t, const tcw_space* sp, int64_t w0, uint32_t j,
                     int64_t count, uint64_t* pts_out_dev);

/* tcw_canon_hash (parity): matrix hash H of `count` exact matrices (the nu + h part of the walk
 * step): a_dev, b_dev are count x R x R int32 (any values), e_dev count int32 (any sign); keys from
 * (n, sp).  When every entry fits int8 (|a|, |b| <= 127) the digests come from the walk's own
 * side-1 product (int8 MFMA at n >= 3), otherwise from 64-bit modular products; the hash is the same
 * function either way.  count above 2^31: TCW_EINVAL. */
int tcw_canon_hash(tcw_ctx* ctx, int n, const tcw_space* sp, const int32_t* a_dev, const int32_t* b_dev,
                   const int32_t* e_dev, int64_t count, uint64_t* h_out_dev);

/* tcw_claw_check (exact, Sec. 3 last merge case): for point pairs (u0, u1) on opposite sides,
 * D = W V^T computed exactly; ok_out_dev[i] = 1 iff D is a signed permutation (a Clifford), and
 * then perm_out_dev[i*R + q], sign_out_dev[i*R + q] give D P_q D^dag = sign P_perm. */
int tcw_claw_check(tcw_ctx* ctx, const tcw_target* t, const tcw_space* sp, const uint64_t* u0_dev,
                   const uint64_t* u1_dev, int64_t count, int32_t* ok_out_dev, int32_t* perm_out_dev,
                   int8_t* sign_out_dev);

/* ---- walk sessions: many concurrent walks with a device distinguished-point table ----------
 * A session owns `walks` walk states (64 B each) and a table of 2^log2_table slots (16 B each).
 * tcw_walk_run enqueues one launch of walks x iters evaluations of f (walking, inserting
 * distinguished points, backtracking merged trails): every walk performs `iters` of them, except at
 * n = 4, where the two walks a wavefront runs (2q, 2q + 1) share 2 iters between them (a side-0 step
 * runs alone, two side-1 steps share one MFMA pass), so each one's share varies with its sides.  Claw candidates (equal
 * matrix hash, opposite sides) are queued on the device.  enumerate != 0 is the exhaustive mode for
 * small spaces: walk w takes the points w, w + walks, w + 2 walks, ... of the space once each and the
 * table is keyed by each point's full 64-bit matrix hash, keeping per side the least x that reached
 * the key; once every point is done (active_walks = 0), tcw_walk_claws reads out one candidate per
 * key reached from both sides (least side-0 x, least side-1 x), so the candidates do not depend on
 * the order in which walks arrive. */
typedef struct tcw_walk_stats {
    int64_t steps;          /* f evaluations, including backtracking */
    int64_t dps;            /* distinguished points reached */
    int64_t inserts;        /* new table entries */
    int64_t abandoned;      /* trails that hit the cap */
    int64_t robin_hood;     /* merges where one trail started on the other */
    int64_t same_side;      /* collisions of f within one side */
    int64_t reduction;      /* cross-side collisions of f with different matrix hashes */
    int64_t claws;          /* cross-side collisions with equal matrix hash (candidates) */
    int64_t table_full;     /* inserts dropped for lack of a free slot */
    int64_t spin_timeouts;  /* table readers that gave up waiting for a slot's value */
    int64_t active_walks;   /* walks not yet finished (enumeration mode) */
    int64_t claws_dropped;  /* claw candidates beyond the candidate buffer (4096 pairs per session, 1024 per
                               batch member), counted but not checked */
} tcw_walk_stats;

int tcw_walk_begin(tcw_ctx* ctx, const tcw_target* t, const tcw_space* sp, int64_t walks, int log2_table,
                   uint32_t cap, int enumerate, tcw_walk** out);
int tcw_walk_run(tcw_walk* w, int iters);
/* Blocking: synchronise the stream and read counters. */
int tcw_walk_stats_get(tcw_walk* w, tcw_walk_stats* out);
/* Blocking: copy up to max_pairs claw candidates (u0, u1) to host arrays; returns the count found
 * so far in *total.  Enumeration mode: the candidates are formed by this call once every point is
 * done (before that *total is 0), the first call after that forms them, later calls re-read them. */
int tcw_walk_claws(tcw_walk* w, uint64_t* u0, uint64_t* u1, int64_t max_pairs, int64_t* total);
/* Re-salt: switch to function version `version`, clear the table, restart every walk. */
int tcw_walk_reset(tcw_walk* w, uint32_t version);
/* Time of the last tcw_walk_run launch in milliseconds, from HIP events on the context stream
 * (blocking). */
int tcw_walk_last_ms(tcw_walk* w, float* ms);
/* Checkpoint / inspection: copy walk states [first, first + count) (64-byte records: start, cur,
 * pa, pb, na, ha as uint64; len, trail, mode, rem as uint32) to or from host memory, and the
 * table (2^log2_table slots of (key, value) uint64 pairs; key ~0 = empty; value = start |
 * len << 33 | 1 << 63).  A session resumed from both continues its trails exactly.  Blocking. */
int tcw_walk_read_states(tcw_walk* w, int64_t first, int64_t count, void* host_out);
int tcw_walk_write_states(tcw_walk* w, int64_t first, int64_t count, const void* host_in);
int tcw_walk_read_table(tcw_walk* w, void* host_out);
int tcw_walk_write_table(tcw_walk* w, const void* host_in);
int tcw_walk_end(tcw_walk* w);

/* ---- search driver (depth loop, chunk loop, budgets; Sec. 3 and Appendix) ------------------ */
#define TCW_ORDER_PLAIN 0       /* depths 0, 1, ..., k_max */
#define TCW_ORDER_GIVEN 1       /* depth_order first, then the remaining depths in increasing order; after a verified
                                   decomposition at depth k, every depth below k not yet searched is searched in
                                   increasing order and the lowest verified decomposition is returned */
#define TCW_ORDER_GIVEN_FIRST 2 /* as TCW_ORDER_GIVEN, but the first verified decomposition is returned: its T-count may
                                   exceed the minimum (tcw_result.minimal says whether the depths below were searched) */

#define TCW_STATUS_NOT_FOUND 0  /* no decomposition within the budgets or the wall-clock cap */
#define TCW_STATUS_FOUND 1      /* a decomposition was found and verified exactly */
#define TCW_STATUS_STOPPED 2    /* the call ended at a launch boundary on tcw_search_stop or launch_limit */

#define TCW_MAX_TRAIL_CAP ((1u << 30) - 1) /* longest trail a table entry can record */

typedef struct tcw_walk_params {
    int32_t k_max;            /* deepest depth searched (plain order 0..k_max) */
    int32_t delta;            /* theta = 2^-delta for walk spaces; < 0 (default): per space, the largest theta
                                 (delta >= 1) whose 2 N theta distinguished points per version fill at most a
                                 quarter of the table (Sec. 5.1: larger theta is faster while memory holds them) */
    int64_t walks;            /* concurrent walks */
    int32_t log2_table;       /* table slots 2^log2_table */
    uint64_t seed;            /* search seed */
    uint32_t version;         /* first function version */
    int32_t trail_cap_factor; /* cap = factor * 2^delta (default 20) */
    int32_t budget_beta;      /* steps per (k, chunk) = beta * N * 2^delta, N = 2 xi^h (default 16) */
    int32_t version_factor;   /* steps per function version = max(factor * N, 2 walks 2^delta) (default 2) */
    int64_t enum_max;         /* enumerate spaces with N <= enum_max (default 65536) */
    int32_t iters_per_launch; /* f evaluations per walk per launch, on average at n = 4 (default by n) */
    int32_t depth_order_kind; /* TCW_ORDER_PLAIN or TCW_ORDER_GIVEN */
    int32_t depth_order_len;
    int32_t depth_order[16];  /* depths to try in this order (GIVEN) */
    int32_t chunk_first;      /* odd k: first chunk tried (default 1) */
    int32_t chunk_last;       /* odd k: last chunk tried (default xi) */
    double max_seconds;       /* wall-clock cap for the whole search (0: none) */
    int32_t chunk_parallel;   /* odd k: chunks searched concurrently, each with walks / G walks and its
                                 own table; small (enumerated) chunks too while their tables fit 32 GiB
                                 (1, the default: one at a time in ascending order; 0: all) */
    int64_t launch_limit;     /* tcw_search / tcw_resume: end the call with TCW_STATUS_STOPPED after this many walk
                                 launches in the call (0, the default: no limit); the stopped search can be
                                 checkpointed */
} tcw_walk_params;
/* Ranges (else TCW_EINVAL, before any device work): delta <= 32; walks in 1..2^31 and log2_table in
 * 4..32 (in a batch, <= 0 takes the autotuner's choice); trail_cap_factor, budget_beta and
 * version_factor >= 1; enum_max >= 0; chunk_first, chunk_last in 0..xi; max_seconds >= 0;
 * k_max in 0..64; depth_order_kind one of TCW_ORDER_*; a given depth order of at most 16 depths in
 * 0..k_max; launch_limit >= 0.  The trail cap trail_cap_factor * 2^delta must not exceed
 * TCW_MAX_TRAIL_CAP: checked up front for delta >= 0 and, for an automatic delta, when a walk space
 * picks its delta (TCW_EINVAL then, before that space's first launch). */

typedef struct tcw_result {
    int32_t status;                 /* TCW_STATUS_*: 1 found and verified exactly, 0 not found, 2 stopped */
    int32_t t;                      /* its T-count (the depth k it was found at) */
    int32_t n;
    int32_t chunk;
    uint16_t paulis[TCW_MAX_T];     /* P_t, ..., P_1 */
    int32_t clifford_perm[TCW_MAX_R];
    int8_t clifford_sign[TCW_MAX_R]; /* D P_q D^dag = sign[q] P_perm[q] */
    tcw_walk_stats stats;           /* summed over every space searched */
    int64_t spaces;                 /* (k, chunk) spaces searched */
    int64_t versions;               /* function versions used */
    int64_t launches;
    int64_t false_claws;            /* candidates rejected by the exact check */
    double seconds;
    uint64_t failed_depths;         /* bit k: depth k was searched to its full budget (every chunk; small spaces
                                       exhaustively) without a verified decomposition */
    int32_t minimal;                /* 1: found, and every depth below t is in failed_depths, so t is minimal up to
                                       the per-depth budgets (exactly minimal where those depths were enumerated) */
    int32_t reserved;
} tcw_result;

void tcw_default_params(tcw_walk_params* p, int n);
/* Blocking.  Results written to *res (caller-allocated).  The search runs one launch at a time: between
 * launches it checks claw candidates exactly, switches function versions, chunks and depths, and ends
 * early on a stop request or after launch_limit launches (status TCW_STATUS_STOPPED); the stopped
 * search stays in the context for tcw_checkpoint until the next tcw_search / tcw_resume on it. */
int tcw_search(tcw_ctx* ctx, const tcw_target* t, const tcw_walk_params* p, tcw_result* res);

/* ---- stopping and resuming a search (a trail is fully described by its start, its current point
 * and its length, Sec. 3, so a search resumes from its walk states and its table) ---------------
 * tcw_search_stop: ask the search running on ctx (from another host thread) to stop at its next
 * launch boundary; it then returns TCW_STATUS_STOPPED.  A request made while no search runs applies
 * to the next one.  Thread-safe; the only call that may overlap another call on the same context.
 * tcw_checkpoint: serialise the stopped search of ctx (parameters, depth-loop position, counters, the
 * current space's walk states, its table and its counters) into host_buf.  *len is the buffer size on
 * entry and the bytes written (or needed) on return; host_buf = NULL only reports the size.
 * TCW_ESTATE if no stopped search is held (none stopped, or it stopped inside a group of concurrently
 * searched chunks, chunk_parallel != 1, whose members are not serialised); TCW_EINVAL if *len is too
 * small.  Blocking.
 * tcw_resume: continue a checkpointed search of the same target t (checked by a fingerprint of its
 * exact channel rep; TCW_EINVAL on a mismatch or a malformed buffer) in any context on any device of
 * the same kind, with the checkpoint's parameters except launch_limit (this call's limit, 0: none).
 * Walks continue their trails exactly: states, table, counters and the function version are restored.
 * *res as for tcw_search, its counters and seconds including the work before the stop.  Blocking. */
int tcw_search_stop(tcw_ctx* ctx);
int tcw_checkpoint(tcw_ctx* ctx, void* host_buf, size_t* len);
int tcw_resume(tcw_ctx* ctx, const tcw_target* t, const void* host_buf, size_t len, int64_t launch_limit,
               tcw_result* res);

/* ---- batching: many targets of mixed n and k, one graph replay per round ------------------------
 * tcw_search_batch: targets[i] is searched with params[i] (its own k_max, seed, budgets, wall-clock
 * cap max_seconds); walks <= 0, log2_table <= 0 or iters_per_launch <= 0 take the autotuner's
 * choice for that (n, k).  Depth 0 is checked on the spot; every other space (walked, or enumerated
 * when small) is a batch member, and all members advance together in rounds: each round replays one
 * hipGraph, captured once per call, whose parallel branches run one persistent queue kernel per qubit
 * count; its blocks take (member, slice of walks) items from a device queue until it is empty (each
 * member with its own S_c, keys, walk states and table; about four items per block, shared out by
 * walks).  Between rounds the host rewrites the queues and the member descriptors, switches function
 * versions, chunks and depths; claw candidates read after a round are checked exactly while the
 * next round runs, and a member whose space ends with unchecked candidates waits for them.
 * results[i] as for tcw_search (status 0: not found within budget or cap).
 * *aggregate_steps_per_s (may be NULL): walk steps of all targets per second of round time (graph
 * execution and the checks beside it).  Blocking.
 * tcw_autotune: times short walk launches of (n, k) over walk counts 64, 256, ... up to min(N/4, 2^20)
 * and returns the smallest count within 85% of the best rate, launch iterations for ~4 ms launches
 * and a table size holding a version's distinguished points with 4x headroom.  Results are cached
 * in the context per (n, k, delta).  Blocking. */
int tcw_search_batch(tcw_ctx* ctx, const tcw_target* const* targets, int count, const tcw_walk_params* params,
                     tcw_result* results, double* aggregate_steps_per_s);
int tcw_autotune(tcw_ctx* ctx, const tcw_target* t, int k, int chunk, int delta, uint64_t seed, int64_t* walks,
                 int* iters, int* log2_table, double* steps_per_s);

/* tcw_min_tcount: minimal T-count of a target (n <= 3) by meet in the middle (Sec. 3, the split
 * of the synthesis equation into two halves): every left-Clifford coset of T-count <= h_id
 * reached from the identity is tabled by its matrix hash (keyed by seed), then every product
 * U R(P_1)^T ... R(P_j)^T, j <= 2 h_max - h_id, is looked up.  The split h_id is chosen on the host to
 * minimise table plus probe steps (h_max itself for one target; the table holds at most 2^25 entries
 * unless the balanced split needs more); every split covers the same T-counts.  *t_out is the least
 * i + j over matches, which is the T-count whenever that is at most 2 h_max, else -1 (no
 * decomposition with T-count <= 2 h_max exists).  A 64-bit hash collision could only lower the
 * answer, never hide a match.  TCW_EOVERFLOW if U's entries do not fit int8 at its exponent.
 * Blocking. */
int tcw_min_tcount(tcw_ctx* ctx, const tcw_target* t, int h_max, uint64_t seed, int32_t* t_out);
/* ---- a decomposition as gates (Sec. 5.3: the rotations as Clifford-conjugated T gates, the
 * Clifford D from its action on Paulis by a stabilizer-tableau reduction) ---------------------
 * tcw_circuit: gates (application order, first gate applied first) whose product is U =
 * D R(P_t) ... R(P_1) of a verified result, up to global phase.  R(P) = C^dag T C (or T^dag) with C
 * mapping P to +-Z on one qubit; D = the inverse of the H / S / CNOT / Pauli sequence that reduces
 * D's images of X_j and Z_j to the identity.  Adjacent inverse pairs are cancelled.  The T and
 * T^dag gates number exactly res->t.  Qubit indices as in the Pauli codes (qubit 0 is the leftmost
 * Kronecker factor).  *count = gates needed; TCW_EOVERFLOW if that exceeds cap (nothing past cap is
 * written); TCW_EINVAL if res is not a verified decomposition.  Of clifford_perm / clifford_sign only
 * the entries of the generators (codes 1 << j, j < 2n) are read: non-identity codes below 4^n with
 * signs +-1 whose images reduce to the identity, else TCW_EINVAL.  Host only: needs no context or GPU. */
enum {
    TCW_GATE_H = 1,
    TCW_GATE_S = 2,
    TCW_GATE_SDG = 3,
    TCW_GATE_CNOT = 4, /* q0 control, q1 target */
    TCW_GATE_T = 5,
    TCW_GATE_TDG = 6,
    TCW_GATE_X = 7,
    TCW_GATE_Y = 8,
    TCW_GATE_Z = 9
};
typedef struct tcw_gate {
    int32_t kind;
    int32_t q0;
    int32_t q1; /* CNOT target, else -1 */
} tcw_gate;
int tcw_circuit(const tcw_result* res, tcw_gate* gates, int32_t cap, int32_t* count);

/* ---- learned depth order (the network that orders which depths k are searched first) ---------
 * Input: the target's canonical channel rep (rows sign-normalised by their first nonzero entry,
 * sorted lexicographically as integer sequences, minimal exponent e), entries
 * (a + b sqrt2) 2^(-e/2) as FP32 (n <= 3, so 4^n x 4^n features).  Network: depth hidden layers of
 * width `hidden` with GELU (erf form), a linear layer to `classes` T-counts 0..classes-1, softmax,
 * cross-entropy; BF16 weights and activations on MFMA with FP32 accumulation, FP32 master weights,
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * tcw_features: features of one target into out_dev (4^n * 4^n floats, device).
 * tcw_label_batch: `count` targets given as words (words[offsets[i] .. offsets[i+1]) = P_1..P_k then
 * C_1..C_m, k = kof[i]) are built exactly on the GPU; features_dev[i] gets their features and
 * labels_dev[i] their minimal T-count when it is at most 2 h_max (meet in the middle as in
 * tcw_min_tcount, with the split chosen for `count` targets: the table is built once per call, so a
 * large batch tables deeper identity-side levels and probes fewer rotations per target), else -1.
 * Host arrays: offsets[0] = 0 and non-decreasing,
 * 0 <= kof[i] <= word length, 2 m + k <= 256 rotations per word, codes in 1..4^n - 1, else
 * TCW_EINVAL before any device work.
 * tcw_mlp_create: parameters are W_0, b_0, W_1, b_1, ... (W_l row-major in x out); init (host,
 * optional) gives them, else W_l uniform in [-1/sqrt(in), 1/sqrt(in)] from SplitMix64(seed) of the
 * running weight index (u = (r >> 40) / 2^24) and b_l = 0.
 * tcw_mlp_forward: probs_dev[batch x classes] from x_dev[batch x in].  tcw_mlp_gradients: gradients
 * of the mean cross-entropy (host array of param_count floats) and the loss, no update.  A label
 * outside 0..classes-1 adds no loss term and no one-hot target (its probabilities are pushed down).
 * tcw_mlp_train_step: one Adam step on a batch.  tcw_mlp_depth_order: order_out[0..k_max] = depths
 * 0..k_max by descending key, ties smaller first: with params NULL the key is the predicted
 * probability p_k; with search parameters it is p_k / c_k, c_k as tcw_depth_costs gives it (the
 * expected-cost order for one hidden answer: a depth that probably holds it and costs little goes
 * first); probs_out (host, may be NULL) receives every class probability.  k_max <= 63.
 * tcw_depth_costs: cost_out[0..k_max] (host) = the walk steps the search driver spends on depth k
 * under params when that depth holds no decomposition (Sec. 3, eq:runtime, and the appendix law:
 * each chunk's budget beta N / theta, or N points when the space is enumerated, with theta resolved
 * as the driver resolves an open delta), plus 2^20 steps of fixed cost per depth; HUGE_VAL for a
 * depth whose spaces exceed 32-bit points.  Parameters checked as for tcw_search_batch (walks,
 * log2_table 0: the autotuned defaults).
 * All blocking except where noted; device pointers as elsewhere. */
typedef struct tcw_mlp tcw_mlp;
int tcw_features(tcw_ctx* ctx, const tcw_target* t, float* out_dev);
int tcw_label_batch(tcw_ctx* ctx, int n, int count, const uint16_t* words, const int32_t* offsets, const int32_t* kof,
                    int h_max, uint64_t seed, float* features_dev, int32_t* labels_dev);
int tcw_mlp_create(tcw_ctx* ctx, int inp, int hidden, int depth, int classes, const float* init, uint64_t seed,
                   tcw_mlp** out);
int tcw_mlp_free(tcw_mlp* m);
int tcw_mlp_param_count(const tcw_mlp* m, int64_t* count);
int tcw_mlp_get_params(tcw_mlp* m, float* host_out);
int tcw_mlp_set_params(tcw_mlp* m, const float* host_in);
int tcw_mlp_forward(tcw_mlp* m, const float* x_dev, int batch, float* probs_dev);
int tcw_mlp_gradients(tcw_mlp* m, const float* x_dev, const int32_t* labels_dev, int batch, float* grads_host,
                      float* loss);
int tcw_mlp_train_step(tcw_mlp* m, const float* x_dev, const int32_t* labels_dev, int batch, float lr, float* loss);
int tcw_mlp_depth_order(tcw_mlp* m, const tcw_target* t, int k_max, const tcw_walk_params* params,
                        int32_t* order_out, float* probs_out);
int tcw_depth_costs(tcw_ctx* ctx, const tcw_target* t, const tcw_walk_params* params, int k_max, double* cost_out);
/* tcw_mlp_train: `epochs` passes over count samples (x_dev count x in, labels_dev count) in fixed
 * consecutive batches of `batch` (the last one ragged), one Adam step each; *last_epoch_loss = mean
 * loss over the final pass. */
int tcw_mlp_train(tcw_mlp* m, const float* x_dev, const int32_t* labels_dev, int64_t count, int batch, int epochs,
                  float lr, float* last_epoch_loss);

#ifdef __cplusplus
}
#endif
#endif /* TCW_H */
