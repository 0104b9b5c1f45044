// C ABI and host-side search driver.  Every arithmetic step of the method runs in the kernels of
// exact.hip and walk.hip; this file validates arguments, owns device buffers, launches kernels on
// the caller's stream and sequences the search (Sec. 3: depth loop, chunk loop, function
// versions, budgets from the Appendix's runtime law).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tcw.h"
#include "common.h"
#include "internal.h"


struct TunedCfg {
    int64_t walks = 0;
    int iters = 0;
    int log2_table = 0;
    double rate = 0;
};

namespace tcw {
// n = 4: rotated key vectors (SpaceDev::rkeys, rkeys2), shared by the spaces of one search seed.
struct RotKeys {
    uint64_t* t1 = nullptr;  // 1 MiB
    uint64_t* t2 = nullptr;  // 256 MiB, or null when the allocation failed
    ~RotKeys() {
        if (t1) (void)hipFree(t1);
        if (t2) (void)hipFree(t2);
    }
};
}  // namespace tcw

constexpr size_t ROT_KEYS_KEEP = 32;  // seeds whose n = 4 rotated keys (257 MiB each) a context keeps

struct SearchRun;
void free_search_run(SearchRun* r);

struct tcw_ctx {
    std::map<uint64_t, TunedCfg> tuned;  // autotuner results by (n, k, delta)
    // n = 4 rotated keys by search seed, kept for later spaces of the same seed: freeing device
    // memory waits for the device, so a table lives until the context ends or until more than
    // ROT_KEYS_KEEP seeds are cached and it is the least recently used one no space holds
    struct RotEntry {
        std::shared_ptr<tcw::RotKeys> rk;
        uint64_t last = 0;
    };
    std::map<uint64_t, RotEntry> rot_keys;
    uint64_t rot_clock = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int* flag = nullptr;          // device scratch flag
    int32_t* rot_min = nullptr;   // device scratch of exact_rotate1 (the least reduction count)
    void* claw_scratch = nullptr;
    size_t claw_scratch_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    void* noalloc = nullptr;        // this device's copy of the tcw_step_noalloc scratch array
    hipError_t noalloc_err = hipSuccess;
    std::atomic<int> stop_req{0};   // tcw_search_stop: end the running search at its next launch boundary
    SearchRun* stopped = nullptr;   // the last search that ended on a stop, for tcw_checkpoint
    // device buffers of finished batch members, by exact size, for later batches (pool_alloc / pool_put)
    std::multimap<size_t, void*> pool;
    size_t pool_bytes = 0;
};

struct tcw_target {
    tcw_ctx* ctx = nullptr;
    int n = 0;
    tcw::ExactDev U;
};

namespace {

using tcw::ExactDev;
using tcw::SpaceDev;

int fail(tcw_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(tcw_ctx* c, hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(c, e == hipErrorOutOfMemory ? TCW_ENOMEM : TCW_EDEVICE, m);
}

// A search at n = 4 opens hundreds of chunk spaces as batch members, and allocating and freeing
// their buffers costs more than the kernels that fill them.  A finished batch returns its members'
// buffers here (after its streams are synchronised, so no work on them is pending) and later members
// take buffers of exactly the size they need; beyond POOL_MAX bytes they are freed.  tcw_destroy
// frees the rest.
constexpr size_t POOL_MAX = (size_t)40 << 30;

hipError_t pool_alloc(tcw_ctx* c, void** p, size_t bytes) {
    auto it = c->pool.find(bytes);
    if (it != c->pool.end()) {
        *p = it->second;
        c->pool.erase(it);
        c->pool_bytes -= bytes;
        return hipSuccess;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipErrorOutOfMemory && !c->pool.empty()) {
        // pooled buffers of other sizes hold the memory: free them (nothing is pending on them) and
        // try once more; the failed call's error is cleared so that later launch checks do not see it
        (void)hipGetLastError();
        for (auto& kv : c->pool) (void)hipFree(kv.second);
        c->pool.clear();
        c->pool_bytes = 0;
        e = hipMalloc(p, bytes);
    }
    return e;
}

void pool_put(tcw_ctx* c, void* p, size_t bytes) {
    if (!p) return;
    if (c->pool_bytes + bytes > POOL_MAX) {
        (void)hipFree(p);
        return;
    }
    c->pool.emplace(bytes, p);
    c->pool_bytes += bytes;
}

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
    } while (0)

// Device buffers local to one call, freed when the call returns on any path (an early HIP_TRY
// return included).
class DevScope {
   public:
    DevScope() = default;
    DevScope(const DevScope&) = delete;
    DevScope& operator=(const DevScope&) = delete;
    ~DevScope() {
        for (void* q : bufs_) (void)hipFree(q);
    }
    template <typename T>
    hipError_t alloc(T** p, size_t bytes) {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) return e;
        bufs_.push_back(q);
        *p = static_cast<T*>(q);
        return hipSuccess;
    }

   private:
    std::vector<void*> bufs_;
};

uint32_t xi_of(int n) { return (1u << (2 * n)) - 1; }

// xi^h, or 0 if it does not fit in 32 bits
uint64_t n_half_of(int n, int h) {
    uint64_t v = 1;
    for (int i = 0; i < h; ++i) {
        v *= xi_of(n);
        if (v >= (1ull << 32)) return 0;
    }
    return v;
}

int clear_flag(tcw_ctx* c) {
    HIP_TRY(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    return TCW_OK;
}

int read_flag(tcw_ctx* c, int* out) {
    HIP_TRY(c, hipMemcpyAsync(out, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

// Salts of the matrix hash, the distinguished-point test and the trail starts of a space.
void space_salts(tcw::SpaceDev& dev, uint64_t seed, uint32_t version, int k, int chunk) {
    const uint64_t ctxi = ((uint64_t)version << 16) | ((uint64_t)k << 8) | (uint64_t)chunk;
    dev.salt_h = tcw::sm64(tcw::sm64(seed, 2), ctxi);
    dev.salt_d = tcw::sm64(tcw::sm64(seed, 3), ctxi);
    dev.salt_s = tcw::sm64(tcw::sm64(seed, 4), ctxi);
}

// A prepared search space: S_c on the device (exact and int8-packed), keys, salts.
struct Space {
    tcw_ctx* ctx = nullptr;
    int n = 0, k = 0, chunk = 0, delta = 0;
    uint64_t seed = 0;
    uint32_t version = 0;
    ExactDev S;
    int32_t e_s = 0;
    uint32_t* phi = nullptr;
    uint64_t* keys = nullptr;
    std::shared_ptr<tcw::RotKeys> rk;  // n = 4: rotated keys (SpaceDev::rkeys, rkeys2)
    SpaceDev dev{};
    bool pooled = false;  // a batch member's space: buffers from and back to the context's pool

    size_t mat_bytes() const { return (size_t)S.r * S.r * S.elem; }
    size_t phi_bytes() const { return (size_t)S.r * S.r / 2 * sizeof(uint32_t) + 16; }
    size_t key_bytes() const { return (size_t)S.r * sizeof(uint64_t); }

    void release() {
        if (pooled && ctx) {
            pool_put(ctx, S.a, mat_bytes());
            pool_put(ctx, S.b, mat_bytes());
            pool_put(ctx, S.e, sizeof(int32_t));
            pool_put(ctx, phi, phi_bytes());
            pool_put(ctx, keys, key_bytes());
            S.a = S.b = nullptr;
            S.e = nullptr;
        } else {
            tcw::exact_free(S);
            if (phi) (void)hipFree(phi);
            if (keys) (void)hipFree(keys);
        }
        phi = nullptr;
        keys = nullptr;
    }

    ~Space() { release(); }

    void set_version(uint32_t v) {
        version = v;
        space_salts(dev, seed, v, k, chunk);
    }
};

int check_space(tcw_ctx* c, int n, const tcw_space* sp) {
    if (!sp) return fail(c, TCW_EINVAL, "space is NULL");
    if (sp->k < 1 || sp->k > TCW_MAX_T) return fail(c, TCW_EINVAL, "k must be in 1..64");
    if (sp->k % 2 == 1) {
        if (sp->chunk < 1 || (uint32_t)sp->chunk > xi_of(n)) return fail(c, TCW_EINVAL, "odd k needs chunk in 1..xi");
    } else if (sp->chunk != 0) {
        return fail(c, TCW_EINVAL, "even k needs chunk 0");
    }
    if (sp->delta < 0 || sp->delta > 32) return fail(c, TCW_EINVAL, "delta must be in 0..32");
    if (n_half_of(n, sp->k / 2) == 0) return fail(c, TCW_EINVAL, "xi^h must be below 2^32");
    if (sp->k > 255) return fail(c, TCW_EINVAL, "k too large");
    return TCW_OK;
}

int prepare_space(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, Space& out) {
    int rc = check_space(c, t->n, sp);
    if (rc) return rc;
    const int n = t->n;
    const int R = 1 << (2 * n);
    out.ctx = c;
    out.n = n;
    out.k = sp->k;
    out.chunk = sp->chunk;
    out.delta = sp->delta;
    out.seed = sp->seed;
    // a Space prepared before for the same qubit count keeps its buffers (a batch member's next chunk)
    if (out.S.a == nullptr || out.S.n != n || !out.phi || !out.keys) {
        out.release();
        if (out.pooled) {
            out.S.n = n;
            out.S.r = R;
            out.S.elem = n <= 2 ? 8 : 4;
            HIP_TRY(c, pool_alloc(c, &out.S.a, out.mat_bytes()));
            HIP_TRY(c, pool_alloc(c, &out.S.b, out.mat_bytes()));
            HIP_TRY(c, pool_alloc(c, reinterpret_cast<void**>(&out.S.e), sizeof(int32_t)));
            HIP_TRY(c, pool_alloc(c, reinterpret_cast<void**>(&out.phi), out.phi_bytes()));
            HIP_TRY(c, pool_alloc(c, reinterpret_cast<void**>(&out.keys), out.key_bytes()));
        } else {
            HIP_TRY(c, tcw::exact_alloc(out.S, n));
            HIP_TRY(c, hipMalloc(&out.phi, (size_t)R * R / 2 * sizeof(uint32_t) + 16));
            HIP_TRY(c, hipMalloc(&out.keys, (size_t)R * sizeof(uint64_t)));
        }
    }
    if ((rc = clear_flag(c))) return rc;
    // S_c = U R(c)^T for odd k, U for even k
    hipError_t e = hipSuccess;
    if (sp->k % 2 == 1) {
        e = tcw::exact_rotate1(out.S, t->U, (uint32_t)sp->chunk, 1, c->rot_min, c->flag, c->stream);
    } else {
        const size_t bytes = (size_t)out.S.r * out.S.r * out.S.elem;
        e = hipMemcpyAsync(out.S.a, t->U.a, bytes, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(out.S.b, t->U.b, bytes, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(out.S.e, t->U.e, sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "chunk matrix");
    HIP_TRY(c, tcw::exact_pack_phi(out.S, out.phi, c->flag, c->stream));
    HIP_TRY(c, tcw::keys_fill(n, sp->seed, out.keys, c->stream));
    if (n == 4) {
        // the keys depend on the seed only: one set of rotated keys per seed, cached in the context
        auto it = c->rot_keys.find(sp->seed);
        if (it == c->rot_keys.end()) {
            while (c->rot_keys.size() >= ROT_KEYS_KEEP) {
                auto victim = c->rot_keys.end();
                for (auto e = c->rot_keys.begin(); e != c->rot_keys.end(); ++e) {
                    const bool unused = e->second.rk.use_count() == 1;
                    if (unused && (victim == c->rot_keys.end() || e->second.last < victim->second.last)) victim = e;
                }
                if (victim == c->rot_keys.end()) break;  // every cached table is in use
                c->rot_keys.erase(victim);
            }
            auto rk = std::make_shared<tcw::RotKeys>();
            HIP_TRY(c, hipMalloc(&rk->t1, (size_t)2 * 256 * 256 * sizeof(uint64_t)));
            HIP_TRY(c, tcw::rot_keys_fill(out.keys, rk->t1, c->stream));
            if (hipMalloc(&rk->t2, (size_t)2 * 256 * 256 * 256 * sizeof(uint64_t)) == hipSuccess) {
                HIP_TRY(c, tcw::rot_keys2_fill(rk->t1, rk->t2, c->stream));
            } else {
                rk->t2 = nullptr;  // without the 256 MiB table the step applies one more rotation
                (void)hipGetLastError();
            }
            it = c->rot_keys.emplace(sp->seed, tcw_ctx::RotEntry{rk, 0}).first;
        }
        it->second.last = ++c->rot_clock;
        out.rk = it->second.rk;
    }
    HIP_TRY(c, hipMemcpyAsync(&out.e_s, out.S.e, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    int flag = 0;
    if ((rc = read_flag(c, &flag))) return rc;
    if (flag & 4) return fail(c, TCW_EOVERFLOW, "exact value out of range while forming S_c");
    if (flag & 2) return fail(c, TCW_EOVERFLOW, "S_c entry outside int8 range (exponent too large)");
    const int h = sp->k / 2;
    out.dev.n_half = (uint32_t)n_half_of(n, h);
    out.dev.h = h;
    out.dev.delta = sp->delta;
    out.dev.rot_e = (int32_t)((30ll * out.e_s) % 61);
    out.dev.phi = out.phi;
    out.dev.keys = out.keys;
    out.dev.rkeys = out.rk ? out.rk->t1 : nullptr;
    out.dev.rkeys2 = out.rk ? out.rk->t2 : nullptr;
    out.set_version(sp->version);
    return TCW_OK;
}

int default_log2_table(int n) { return n <= 2 ? 12 : (n == 3 ? 20 : 26); }

// theta of a walk space when the caller leaves it open.  The time to a golden collision falls as
// theta rises for as long as memory holds the distinguished points (Sec. 5.1), so take the largest
// theta = 2^-delta, delta >= 1, whose 2 N theta distinguished points per function version fill at
// most a quarter of the table: 8 N <= 2^(log2_table + delta).
int auto_delta(uint64_t npts, int log2_table) {
    int d = 1;
    while (d < 30 && (npts << 3) > (1ull << (log2_table + d))) ++d;
    return d;
}
int default_iters(int n) { return n <= 2 ? 64 : (n == 3 ? 32 : 8); }

// Walks of a walked space: at most a quarter of its points.  With more walks than that, a function
// version (at most the table's half load of steps) ends before the walks' trails and their
// backtracking do, and the search stops reporting claws (measured on Toffoli: 2^20 walks in depth-7
// chunks of 5e5 points never finish, 2^18 do).
int64_t walks_for(int64_t walks, uint64_t npts) {
    return std::min<int64_t>(walks, std::max<int64_t>(64, (int64_t)(npts / 4)));
}

}  // namespace

// ---------------------------------------------------------------------------------------------
struct tcw_walk {
    tcw_ctx* ctx = nullptr;
    Space space;
    tcw::WalkDev wd{};
    bool ended = false;
    bool pairs_formed = false;  // enumeration mode: candidates read out of the table
    int64_t launches = 0;

    ~tcw_walk() {
        if (wd.states) (void)hipFree(wd.states);
        if (wd.table) (void)hipFree(wd.table);
        if (wd.stats) (void)hipFree(wd.stats);
        if (wd.claws) (void)hipFree(wd.claws);
        if (wd.claw_count) (void)hipFree(wd.claw_count);
    }
};

namespace {

int walk_restart(tcw_walk* w) {
    tcw_ctx* c = w->ctx;
    w->pairs_formed = false;
    w->launches = 0;
    HIP_TRY(c, tcw::launch_table_clear(w->wd.table, w->wd.log2_table, w->wd.enumerate ? tcw::ENUM_TABLE_INIT : 0,
                                       c->stream));
    HIP_TRY(c, hipMemsetAsync(w->wd.stats, 0, tcw::ST_COUNT * sizeof(unsigned long long), c->stream));
    HIP_TRY(c, hipMemsetAsync(w->wd.claw_count, 0, sizeof(unsigned long long), c->stream));
    HIP_TRY(c, tcw::launch_walk_init(w->space.dev, w->wd, c->stream));
    return TCW_OK;
}

}  // namespace

// ---- device memory of tcw_step_noalloc ----
// One fixed array per device holds every per-call buffer of the step: the chunk matrix S_c (A and B,
// R x R of int32 at n >= 3, of int64 at n <= 2: at most 256 KiB each), the two work matrices of its
// construction, its exponent, the one-rotation word that forms it, its int8 packing and the keys.
namespace {
constexpr size_t NA_MAT = (size_t)256 * 256 * 4;
constexpr size_t NA_OFF_SA = 0, NA_OFF_SB = NA_MAT, NA_OFF_TA = 2 * NA_MAT, NA_OFF_TB = 3 * NA_MAT;
constexpr size_t NA_OFF_E = 4 * NA_MAT;          // S_c's exponent (int32)
constexpr size_t NA_OFF_SEQ = NA_OFF_E + 256;     // the rotation code (uint16) at +0, its transpose flag at +16
constexpr size_t NA_OFF_PHI = NA_OFF_SEQ + 256;   // int8 packing of S_c
constexpr size_t NA_PHI = (size_t)256 * 256 / 2 * 4 + 256;
constexpr size_t NA_OFF_KEYS = NA_OFF_PHI + NA_PHI;  // R keys (uint64)
constexpr size_t NA_BYTES = NA_OFF_KEYS + 256 * 8;
static_assert(NA_BYTES == TCW_STEP_NOALLOC_SCRATCH, "scratch size stated in tcw.h");
static_assert(NA_OFF_PHI % 256 == 0 && NA_OFF_KEYS % 256 == 0, "aligned parts");
}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {
constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mutex;
void* na_ptr[NA_MAX_DEVICES] = {};

// With the context's device current: this device's address of `scratch` (taken once per device).  The
// array's name in host code is a host-side stand-in, never a device address.
void noalloc_setup(tcw_ctx* c) {
    std::lock_guard<std::mutex> lock(na_mutex);
    if (c->device < 0 || c->device >= NA_MAX_DEVICES) {
        c->noalloc_err = hipErrorInvalidDevice;
        return;
    }
    if (!na_ptr[c->device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            c->noalloc_err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            (void)hipGetLastError();
            return;
        }
        na_ptr[c->device] = p;
    }
    c->noalloc = na_ptr[c->device];
}
}  // namespace

extern "C" {

int tcw_create(tcw_ctx** out, int device, void* stream) {
    if (!out) return TCW_EINVAL;
    *out = nullptr;
    tcw_ctx* c = new (std::nothrow) tcw_ctx();
    if (!c) return TCW_ENOMEM;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        delete c;
        return TCW_EDEVICE;
    }
    c->device = device;
    c->stream = (hipStream_t)stream;
    if (hipSetDevice(device) != hipSuccess || hipMalloc(&c->flag, sizeof(int)) != hipSuccess ||
        hipMalloc(&c->rot_min, sizeof(int32_t)) != hipSuccess || hipEventCreate(&c->ev0) != hipSuccess ||
        hipEventCreate(&c->ev1) != hipSuccess) {
        delete c;
        return TCW_EDEVICE;
    }
    noalloc_setup(c);
    *out = c;
    return TCW_OK;
}

int tcw_destroy(tcw_ctx* c) {
    if (!c) return TCW_EINVAL;
    if (c->stopped) free_search_run(c->stopped);
    c->stopped = nullptr;
    if (c->flag) (void)hipFree(c->flag);
    if (c->rot_min) (void)hipFree(c->rot_min);
    for (auto& e : c->pool) (void)hipFree(e.second);
    c->pool.clear();
    if (c->claw_scratch) (void)hipFree(c->claw_scratch);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
    return TCW_OK;
}

const char* tcw_last_error(const tcw_ctx* c) { return c ? c->err.c_str() : "no context"; }

int tcw_set_stream(tcw_ctx* c, void* stream) {
    if (!c) return TCW_EINVAL;
    c->stream = (hipStream_t)stream;
    return TCW_OK;
}

int tcw_target_n(const tcw_target* t) { return t ? t->n : 0; }

int tcw_target_from_words(tcw_ctx* c, int n, const uint16_t* paulis, int k, const uint16_t* clifford, int m,
                          tcw_target** out) {
    if (!c || !out) return TCW_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 4) return fail(c, TCW_EINVAL, "n must be in 1..4");
    if (k < 0 || m < 0 || (k > 0 && !paulis) || (m > 0 && !clifford)) return fail(c, TCW_EINVAL, "bad word arrays");
    const uint32_t xi = xi_of(n);
    // right-multiplication sequence: C_1 C_1 C_2 C_2 ... C_m C_m P_k ... P_1
    std::vector<uint16_t> seq;
    seq.reserve(2 * m + k);
    for (int j = 0; j < m; ++j) {
        if (clifford[j] < 1 || clifford[j] > xi) return fail(c, TCW_EINVAL, "Clifford Pauli out of range");
        seq.push_back(clifford[j]);
        seq.push_back(clifford[j]);
    }
    for (int j = k - 1; j >= 0; --j) {
        if (paulis[j] < 1 || paulis[j] > xi) return fail(c, TCW_EINVAL, "Pauli out of range");
        seq.push_back(paulis[j]);
    }
    tcw_target* t = new (std::nothrow) tcw_target();
    if (!t) return TCW_ENOMEM;
    t->ctx = c;
    t->n = n;
    hipError_t e = tcw::exact_alloc(t->U, n);
    uint16_t* seq_dev = nullptr;
    if (e == hipSuccess && !seq.empty()) e = hipMalloc(&seq_dev, seq.size() * sizeof(uint16_t));
    if (e == hipSuccess && !seq.empty())
        e = hipMemcpyAsync(seq_dev, seq.data(), seq.size() * sizeof(uint16_t), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
    if (e == hipSuccess) e = tcw::exact_build(t->U, seq_dev, nullptr, (int)seq.size(), c->flag, c->stream);
    if (seq_dev) (void)hipFree(seq_dev);
    if (e != hipSuccess) {
        tcw::exact_free(t->U);
        delete t;
        return hip_fail(c, e, "target build");
    }
    int flag = 0;
    int rc = read_flag(c, &flag);
    if (rc == TCW_OK && flag) rc = fail(c, TCW_EOVERFLOW, "exact value out of range while building the target");
    if (rc) {
        tcw::exact_free(t->U);
        delete t;
        return rc;
    }
    *out = t;
    return TCW_OK;
}

int tcw_target_from_channel(tcw_ctx* c, int n, const int32_t* a, const int32_t* b, int32_t e0, tcw_target** out) {
    if (!c || !out || !a || !b) return TCW_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 4) return fail(c, TCW_EINVAL, "n must be in 1..4");
    if (e0 < 0 || e0 > 60) return fail(c, TCW_EINVAL, "exponent must be in 0..60");
    const size_t rr = (size_t)1 << (4 * n);
    tcw_target* t = new (std::nothrow) tcw_target();
    if (!t) return TCW_ENOMEM;
    t->ctx = c;
    t->n = n;
    int32_t *da = nullptr, *db = nullptr;
    hipError_t e = tcw::exact_alloc(t->U, n);
    if (e == hipSuccess) e = hipMalloc(&da, rr * 4);
    if (e == hipSuccess) e = hipMalloc(&db, rr * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(da, a, rr * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(db, b, rr * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
    if (e == hipSuccess) e = tcw::exact_from_i32(t->U, da, db, e0, c->flag, c->stream);
    if (e == hipSuccess) e = tcw::exact_check_orthogonal(t->U, c->flag, c->stream);
    int flag = 0;
    int rc = TCW_OK;
    if (e == hipSuccess) {
        rc = read_flag(c, &flag);
    } else {
        rc = hip_fail(c, e, "target upload");
    }
    if (da) (void)hipFree(da);
    if (db) (void)hipFree(db);
    if (rc == TCW_OK && (flag & 4)) rc = fail(c, TCW_EOVERFLOW, "entries too large");
    if (rc == TCW_OK && (flag & 1)) rc = fail(c, TCW_EINVAL, "matrix is not orthogonal (X X^T != 2^e I)");
    if (rc) {
        tcw::exact_free(t->U);
        delete t;
        return rc;
    }
    *out = t;
    return TCW_OK;
}

int tcw_target_from_unitary(tcw_ctx* c, int n, const int64_t* v, int32_t e, tcw_target** out) {
    if (!c || !out || !v) return TCW_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 4) return fail(c, TCW_EINVAL, "n must be in 1..4");
    if (e < 0 || n + e > 29) return fail(c, TCW_EINVAL, "need 0 <= e and n + e <= 29");
    const size_t d = (size_t)1 << n, rr = (size_t)1 << (4 * n);
    for (size_t x = 0; x < d * d * 4; ++x)
        if (v[x] > (1 << 20) || v[x] < -(1 << 20)) return fail(c, TCW_EINVAL, "coefficients must lie in [-2^20, 2^20]");
    tcw_target* t = new (std::nothrow) tcw_target();
    if (!t) return TCW_ENOMEM;
    t->ctx = c;
    t->n = n;
    int64_t* dv = nullptr;
    int32_t *da = nullptr, *db = nullptr;
    hipError_t err = tcw::exact_alloc(t->U, n);
    if (err == hipSuccess) err = hipMalloc(&dv, d * d * 4 * sizeof(int64_t));
    if (err == hipSuccess) err = hipMalloc(&da, rr * 4);
    if (err == hipSuccess) err = hipMalloc(&db, rr * 4);
    if (err == hipSuccess) err = hipMemcpyAsync(dv, v, d * d * 4 * sizeof(int64_t), hipMemcpyHostToDevice, c->stream);
    if (err == hipSuccess) err = hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
    if (err == hipSuccess) err = tcw::exact_from_unitary(t->U, dv, e, da, db, c->flag, c->stream);
    int flag = 0;
    int rc = TCW_OK;
    // the orthogonality check only runs on values that passed the unitary and range checks
    if (err == hipSuccess) rc = read_flag(c, &flag);
    else rc = hip_fail(c, err, "unitary upload");
    if (rc == TCW_OK && flag == 0) {
        err = tcw::exact_check_orthogonal(t->U, c->flag, c->stream);
        if (err == hipSuccess) rc = read_flag(c, &flag);
        else rc = hip_fail(c, err, "orthogonality check");
    }
    if (dv) (void)hipFree(dv);
    if (da) (void)hipFree(da);
    if (db) (void)hipFree(db);
    if (rc == TCW_OK && (flag & 8)) rc = fail(c, TCW_EINVAL, "U is not unitary (V V^dag != 2^e I)");
    if (rc == TCW_OK && (flag & 1)) rc = fail(c, TCW_EINVAL, "channel rep is not real orthogonal");
    if (rc == TCW_OK && (flag & 4)) rc = fail(c, TCW_EOVERFLOW, "channel rep entry out of range");
    if (rc) {
        tcw::exact_free(t->U);
        delete t;
        return rc;
    }
    *out = t;
    return TCW_OK;
}

int tcw_target_random(tcw_ctx* c, int n, int k, uint64_t seed, tcw_target** out, uint16_t* gen_paulis,
                      int32_t* gen_perm, int8_t* gen_sign) {
    if (!c || !out) return TCW_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 4) return fail(c, TCW_EINVAL, "n must be in 1..4");
    if (k < 0 || k > TCW_MAX_T) return fail(c, TCW_EINVAL, "k must be in 0..TCW_MAX_T");
    // SplitMix64 in counter form; each draw maps to a non-identity Pauli by a multiply-high by xi
    const uint64_t xi = xi_of(n);
    const int m = 16 * n;
    auto draw = [&](int i) {
        return (uint16_t)((uint64_t)(((unsigned __int128)tcw::sm64(seed, (uint64_t)i) * xi) >> 64) + 1);
    };
    std::vector<uint16_t> ps(k > 0 ? k : 1), cl(m);
    for (int i = 0; i < k; ++i) ps[i] = draw(i);
    for (int j = 0; j < m; ++j) cl[j] = draw(k + j);
    if (gen_perm || gen_sign) {
        // D alone, as the signed permutation of its channel rep
        tcw_target* d = nullptr;
        int rc = tcw_target_from_words(c, n, nullptr, 0, cl.data(), m, &d);
        if (rc) return rc;
        const int R = 1 << (2 * n);
        int32_t *dok = nullptr, *dperm = nullptr;
        int8_t* dsign = nullptr;
        int32_t ok = 0;
        std::vector<int32_t> perm(R);
        std::vector<int8_t> sign(R);
        {
            DevScope scope;
            hipError_t e = scope.alloc(&dok, 4);
            if (e == hipSuccess) e = scope.alloc(&dperm, R * 4);
            if (e == hipSuccess) e = scope.alloc(&dsign, R);
            if (e == hipSuccess) e = tcw::exact_signed_perm(d->U, dok, dperm, dsign, c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(&ok, dok, 4, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(perm.data(), dperm, R * 4, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(sign.data(), dsign, R, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) rc = hip_fail(c, e, "Clifford of a random target");
        }
        tcw_target_free(d);
        if (rc) return rc;
        if (!ok) return fail(c, TCW_EOVERFLOW, "the Clifford word did not give a signed permutation");
        for (int q = 0; q < R; ++q) {
            if (gen_perm) gen_perm[q] = perm[q];
            if (gen_sign) gen_sign[q] = sign[q];
        }
    }
    int rc = tcw_target_from_words(c, n, ps.data(), k, cl.data(), m, out);
    if (rc) return rc;
    if (gen_paulis)
        for (int i = 0; i < k; ++i) gen_paulis[i] = ps[i];
    return TCW_OK;
}

int tcw_target_free(tcw_target* t) {
    if (!t) return TCW_EINVAL;
    tcw::exact_free(t->U);
    delete t;
    return TCW_OK;
}

int tcw_target_channel(tcw_ctx* c, const tcw_target* t, int32_t* a, int32_t* b, int32_t* e) {
    if (!c || !t || !a || !b || !e) return TCW_EINVAL;
    const size_t rr = (size_t)1 << (4 * t->n);
    int32_t *da = nullptr, *db = nullptr;
    DevScope scope;
    HIP_TRY(c, scope.alloc(&da, rr * 4));
    HIP_TRY(c, scope.alloc(&db, rr * 4));
    int rc = clear_flag(c);
    if (!rc) {
        hipError_t err = tcw::exact_to_i32(t->U, da, db, c->flag, c->stream);
        if (err == hipSuccess) err = hipMemcpyAsync(a, da, rr * 4, hipMemcpyDeviceToHost, c->stream);
        if (err == hipSuccess) err = hipMemcpyAsync(b, db, rr * 4, hipMemcpyDeviceToHost, c->stream);
        if (err == hipSuccess) err = hipMemcpyAsync(e, t->U.e, 4, hipMemcpyDeviceToHost, c->stream);
        if (err != hipSuccess) rc = hip_fail(c, err, "target copy");
    }
    int flag = 0;
    if (!rc) rc = read_flag(c, &flag);
    if (!rc && flag) rc = fail(c, TCW_EOVERFLOW, "entry does not fit int32");
    return rc;
}

int tcw_step(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, const uint64_t* in, uint64_t* out, uint64_t* hash,
             int64_t count) {
    if (!c || !t || count < 0 || (count > 0 && (!in || !out))) return TCW_EINVAL;
    if (count == 0) return check_space(c, t->n, sp);
    Space s;
    int rc = prepare_space(c, t, sp, s);
    if (rc) return rc;
    HIP_TRY(c, tcw::launch_step(t->n, s.dev, in, out, hash, count, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_step_noalloc(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, const uint64_t* in, uint64_t* out,
                     uint64_t* hash, int64_t count) {
    if (!c || !t || count < 0 || (count > 0 && (!in || !out))) return TCW_EINVAL;
    int rc = check_space(c, t->n, sp);
    if (rc || count == 0) return rc;
    const int n = t->n;
    const int R = 1 << (2 * n);
    const size_t elem = n <= 2 ? 8 : 4;
    if ((size_t)R * R * elem > NA_MAT || (size_t)R * R / 2 * 4 + 16 > NA_PHI || (size_t)R * 8 > NA_BYTES - NA_OFF_KEYS)
        return fail(c, TCW_EINVAL, "space larger than the no-allocation scratch (TCW_STEP_NOALLOC_SCRATCH bytes)");
    if (!c->noalloc)
        return fail(c, TCW_EDEVICE, std::string("no-allocation scratch unavailable on this device: ") +
                                        hipGetErrorString(c->noalloc_err));
    uint8_t* base = static_cast<uint8_t*>(c->noalloc);
    ExactDev S;
    S.n = n;
    S.r = R;
    S.elem = elem;
    S.a = base + NA_OFF_SA;
    S.b = base + NA_OFF_SB;
    S.e = reinterpret_cast<int32_t*>(base + NA_OFF_E);
    uint16_t* seq = reinterpret_cast<uint16_t*>(base + NA_OFF_SEQ);
    uint8_t* tr = base + NA_OFF_SEQ + 16;
    uint32_t* phi = reinterpret_cast<uint32_t*>(base + NA_OFF_PHI);
    uint64_t* keys = reinterpret_cast<uint64_t*>(base + NA_OFF_KEYS);
    // S_c = U R(c)^T for odd k, U for even k, built in the scratch array; range flags cleared by a kernel
    HIP_TRY(c, tcw::fill_i32(c->flag, 0, 1, c->stream));
    int nseq = 0;
    if (sp->k % 2 == 1) {
        HIP_TRY(c, tcw::exact_seq_one(seq, tr, (uint16_t)sp->chunk, 1, c->stream));
        nseq = 1;
    }
    HIP_TRY(c, tcw::exact_apply_ws(S, t->U, seq, tr, nseq, base + NA_OFF_TA, base + NA_OFF_TB, c->flag, c->stream));
    HIP_TRY(c, tcw::exact_pack_phi(S, phi, c->flag, c->stream));
    HIP_TRY(c, tcw::keys_fill(n, sp->seed, keys, c->stream));
    int32_t e_s = 0;
    int flag = 0;
    HIP_TRY(c, hipMemcpyAsync(&e_s, S.e, sizeof(e_s), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(&flag, c->flag, sizeof(flag), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (flag & 4) return fail(c, TCW_EOVERFLOW, "exact value out of range while forming S_c");
    if (flag & 2) return fail(c, TCW_EOVERFLOW, "S_c entry outside int8 range (exponent too large)");
    tcw::SpaceDev dev{};
    const int h = sp->k / 2;
    dev.n_half = (uint32_t)n_half_of(n, h);
    dev.h = h;
    dev.delta = sp->delta;
    dev.rot_e = (int32_t)((30ll * e_s) % 61);
    dev.phi = phi;
    dev.keys = keys;
    dev.rkeys = nullptr;   // every rotation of the step is applied (no rotated-key tables)
    dev.rkeys2 = nullptr;
    space_salts(dev, sp->seed, sp->version, sp->k, sp->chunk);
    HIP_TRY(c, tcw::launch_step(n, dev, in, out, hash, count, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_trails(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, const uint64_t* starts, int64_t count,
               uint32_t cap, uint64_t* dp, uint32_t* len) {
    if (!c || !t || count < 0 || cap == 0 || (count > 0 && (!starts || !dp || !len))) return TCW_EINVAL;
    if (count == 0) return check_space(c, t->n, sp);
    Space s;
    int rc = prepare_space(c, t, sp, s);
    if (rc) return rc;
    HIP_TRY(c, tcw::launch_trails(t->n, s.dev, starts, count, cap, dp, len, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_start_points(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, int64_t w0, uint32_t j, int64_t count,
                     uint64_t* out) {
    if (!c || !t || count < 0 || (count > 0 && !out) || w0 < 0 || w0 + count > (1ll << 32)) return TCW_EINVAL;
    int rc = check_space(c, t->n, sp);
    if (rc || count == 0) return rc;
    Space s;
    s.k = sp->k;
    s.chunk = sp->chunk;
    s.seed = sp->seed;
    s.dev.n_half = (uint32_t)n_half_of(t->n, sp->k / 2);
    s.set_version(sp->version);
    HIP_TRY(c, tcw::launch_starts(s.dev, w0, j, count, out, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_canon_hash(tcw_ctx* c, int n, const tcw_space* sp, const int32_t* a, const int32_t* b, const int32_t* e,
                   int64_t count, uint64_t* h_out) {
    if (!c || !sp || count < 0 || (count > 0 && (!a || !b || !e || !h_out))) return TCW_EINVAL;
    if (n < 1 || n > 4) return fail(c, TCW_EINVAL, "n must be in 1..4");
    if (count == 0) return TCW_OK;
    const int R = 1 << (2 * n);
    if (count > (int64_t)1 << 31) return fail(c, TCW_EINVAL, "count above 2^31");  // keeps the byte count exact
    uint32_t* phi = nullptr;
    uint64_t* keys = nullptr;
    DevScope scope;
    HIP_TRY(c, scope.alloc(&phi, (size_t)count * R * R / 2 * sizeof(uint32_t)));
    HIP_TRY(c, scope.alloc(&keys, (size_t)R * sizeof(uint64_t)));
    int rc = clear_flag(c);
    Space s;
    s.k = sp->k;
    s.chunk = sp->chunk;
    s.seed = sp->seed;
    s.dev.keys = keys;
    s.dev.delta = sp->delta;
    s.set_version(sp->version);
    hipError_t err = hipSuccess;
    if (!rc) err = tcw::pack_phi_i32(n, a, b, count, phi, c->flag, c->stream);
    if (!rc && err == hipSuccess) err = tcw::keys_fill(n, sp->seed, keys, c->stream);
    int flag = 0;
    if (!rc && err == hipSuccess) rc = read_flag(c, &flag);
    // entries that fit int8 go through the walk's own side-1 product; others through 64-bit products
    if (!rc && err == hipSuccess)
        err = flag ? tcw::launch_canon_wide(n, s.dev, a, b, e, count, h_out, c->stream)
                   : tcw::launch_canon_hash(n, s.dev, phi, e, count, h_out, c->stream);
    if (!rc && err == hipSuccess) err = hipStreamSynchronize(c->stream);
    if (!rc && err != hipSuccess) rc = hip_fail(c, err, "canon hash");
    return rc;
}

int tcw_claw_check(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, const uint64_t* u0, const uint64_t* u1,
                   int64_t count, int32_t* ok, int32_t* perm, int8_t* sign) {
    if (!c || !t || count < 0 || (count > 0 && (!u0 || !u1 || !ok || !perm || !sign))) return TCW_EINVAL;
    if (count == 0) return check_space(c, t->n, sp);
    Space s;
    int rc = prepare_space(c, t, sp, s);
    if (rc) return rc;
    const size_t need = tcw::exact_claw_scratch_bytes(t->n);
    if (c->claw_scratch_bytes < need) {
        if (c->claw_scratch) (void)hipFree(c->claw_scratch);
        c->claw_scratch = nullptr;
        c->claw_scratch_bytes = 0;
        HIP_TRY(c, hipMalloc(&c->claw_scratch, need));
        c->claw_scratch_bytes = need;
    }
    HIP_TRY(c, tcw::exact_claw_check(s.S, sp->k, u0, u1, count, c->claw_scratch, c->claw_scratch_bytes, ok, perm,
                                     sign, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

// ---- walk sessions ----
int tcw_walk_begin(tcw_ctx* c, const tcw_target* t, const tcw_space* sp, int64_t walks, int log2_table, uint32_t cap,
                   int enumerate, tcw_walk** out) {
    if (!c || !t || !out) return TCW_EINVAL;
    *out = nullptr;
    if (walks < 1 || walks > (1ll << 31)) return fail(c, TCW_EINVAL, "walks must be in 1..2^31");
    if (log2_table < 4 || log2_table > 32) return fail(c, TCW_EINVAL, "log2_table must be in 4..32");
    if (cap == 0 || cap > TCW_MAX_TRAIL_CAP) return fail(c, TCW_EINVAL, "cap must be in 1..TCW_MAX_TRAIL_CAP");
    tcw_walk* w = new (std::nothrow) tcw_walk();
    if (!w) return TCW_ENOMEM;
    w->ctx = c;
    int rc = prepare_space(c, t, sp, w->space);
    if (rc) {
        delete w;
        return rc;
    }
    tcw::WalkDev& wd = w->wd;
    wd.walks = walks;
    wd.log2_table = log2_table;
    wd.cap = cap;
    wd.enumerate = enumerate ? 1 : 0;
    wd.n_points = 2ull * w->space.dev.n_half;
    wd.claw_cap = 4096;
    hipError_t e = hipMalloc(&wd.states, (size_t)walks * sizeof(tcw::WalkState));
    if (e == hipSuccess) e = hipMalloc(&wd.table, ((size_t)1 << log2_table) * 16);
    if (e == hipSuccess) e = hipMalloc(&wd.stats, tcw::ST_COUNT * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&wd.claws, (size_t)wd.claw_cap * 16);
    if (e == hipSuccess) e = hipMalloc(&wd.claw_count, sizeof(unsigned long long));
    if (e != hipSuccess) {
        delete w;
        return hip_fail(c, e, "walk session allocation");
    }
    rc = walk_restart(w);
    if (rc) {
        delete w;
        return rc;
    }
    *out = w;
    return TCW_OK;
}

int tcw_walk_run(tcw_walk* w, int iters) {
    if (!w || iters < 1) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    if (w->ended) return fail(c, TCW_ESTATE, "walk session ended");
    HIP_TRY(c, hipMemsetAsync(&w->wd.stats[tcw::ST_ACTIVE], 0, sizeof(unsigned long long), c->stream));
    HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
    HIP_TRY(c, tcw::launch_walk(w->space.n, w->space.dev, w->wd, iters,
                                tcw::walk_grid_blocks(w->space.n, c->device, false, w->wd.walks), c->stream));
    HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
    w->launches++;
    return TCW_OK;
}

int tcw_walk_stats_get(tcw_walk* w, tcw_walk_stats* out) {
    if (!w || !out) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    unsigned long long v[tcw::ST_COUNT];
    unsigned long long cc = 0;
    HIP_TRY(c, hipMemcpyAsync(v, w->wd.stats, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(&cc, w->wd.claw_count, sizeof(cc), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    out->claws_dropped = cc > w->wd.claw_cap ? (int64_t)(cc - w->wd.claw_cap) : 0;
    out->steps = (int64_t)v[tcw::ST_STEPS];
    out->dps = (int64_t)v[tcw::ST_DPS];
    out->inserts = (int64_t)v[tcw::ST_INSERTS];
    out->abandoned = (int64_t)v[tcw::ST_ABANDONED];
    out->robin_hood = (int64_t)v[tcw::ST_ROBIN];
    out->same_side = (int64_t)v[tcw::ST_SAME];
    out->reduction = (int64_t)v[tcw::ST_REDUCTION];
    out->claws = (int64_t)v[tcw::ST_CLAWS];
    out->table_full = (int64_t)v[tcw::ST_FULL];
    out->spin_timeouts = (int64_t)v[tcw::ST_SPIN];
    out->active_walks = (int64_t)v[tcw::ST_ACTIVE];
    return TCW_OK;
}

int tcw_walk_claws(tcw_walk* w, uint64_t* u0, uint64_t* u1, int64_t max_pairs, int64_t* total) {
    if (!w || !total || max_pairs < 0 || (max_pairs > 0 && (!u0 || !u1))) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    if (w->wd.enumerate && !w->pairs_formed) {
        // the candidates exist once every point is done
        unsigned long long active = 1;
        if (w->launches > 0) {
            HIP_TRY(c, hipMemcpyAsync(&active, &w->wd.stats[tcw::ST_ACTIVE], sizeof(active), hipMemcpyDeviceToHost,
                                      c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
        }
        if (active != 0) {
            *total = 0;
            return TCW_OK;
        }
        HIP_TRY(c, tcw::launch_enum_pairs(w->wd, c->stream));
        w->pairs_formed = true;
    }
    unsigned long long cnt = 0;
    HIP_TRY(c, hipMemcpyAsync(&cnt, w->wd.claw_count, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *total = (int64_t)cnt;
    int64_t avail = (int64_t)(cnt < w->wd.claw_cap ? cnt : w->wd.claw_cap);
    int64_t m = avail < max_pairs ? avail : max_pairs;
    if (m > 0) {
        std::vector<uint64_t> buf(2 * m);
        HIP_TRY(c, hipMemcpyAsync(buf.data(), w->wd.claws, 16 * m, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int64_t i = 0; i < m; ++i) {
            u0[i] = buf[2 * i];
            u1[i] = buf[2 * i + 1];
        }
    }
    return TCW_OK;
}

int tcw_walk_reset(tcw_walk* w, uint32_t version) {
    if (!w) return TCW_EINVAL;
    w->space.set_version(version);
    return walk_restart(w);
}

int tcw_walk_last_ms(tcw_walk* w, float* ms) {
    if (!w || !ms) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    HIP_TRY(c, hipEventSynchronize(c->ev1));
    HIP_TRY(c, hipEventElapsedTime(ms, c->ev0, c->ev1));
    return TCW_OK;
}

int tcw_walk_read_states(tcw_walk* w, int64_t first, int64_t count, void* host_out) {
    if (!w || !host_out || first < 0 || count < 0 || first + count > w->wd.walks) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    HIP_TRY(c, hipMemcpyAsync(host_out, w->wd.states + first, (size_t)count * sizeof(tcw::WalkState),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_walk_write_states(tcw_walk* w, int64_t first, int64_t count, const void* host_in) {
    if (!w || !host_in || first < 0 || count < 0 || first + count > w->wd.walks) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    HIP_TRY(c, hipMemcpyAsync(w->wd.states + first, host_in, (size_t)count * sizeof(tcw::WalkState),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_walk_read_table(tcw_walk* w, void* host_out) {
    if (!w || !host_out) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    HIP_TRY(c, hipMemcpyAsync(host_out, w->wd.table, ((size_t)1 << w->wd.log2_table) * 16, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_walk_write_table(tcw_walk* w, const void* host_in) {
    if (!w || !host_in) return TCW_EINVAL;
    tcw_ctx* c = w->ctx;
    HIP_TRY(c, hipMemcpyAsync(w->wd.table, host_in, ((size_t)1 << w->wd.log2_table) * 16, hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

int tcw_walk_end(tcw_walk* w) {
    if (!w) return TCW_EINVAL;
    (void)hipStreamSynchronize(w->ctx->stream);
    delete w;
    return TCW_OK;
}

// ---- search driver ----
void tcw_default_params(tcw_walk_params* p, int n) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->k_max = 7;
    p->delta = -1;
    p->walks = n <= 2 ? 64 : (n == 3 ? (1 << 16) : (1 << 20));
    p->log2_table = default_log2_table(n);
    p->seed = 1;
    p->version = 0;
    p->trail_cap_factor = 20;
    p->budget_beta = 16;
    p->version_factor = 2;
    p->enum_max = 1 << 16;
    p->iters_per_launch = 0;
    p->depth_order_kind = TCW_ORDER_PLAIN;
    p->chunk_first = 0;
    p->chunk_last = 0;
    p->max_seconds = 0.0;
    p->chunk_parallel = 1;
    p->launch_limit = 0;
}

}  // extern "C"

namespace {

void decode_desc(uint64_t pt, int n, int h, std::vector<uint16_t>& out) {
    uint32_t x = (uint32_t)pt;
    const uint32_t xi = xi_of(n);
    for (int t = 0; t < h; ++t) {
        out.push_back((uint16_t)(x % xi + 1));
        x /= xi;
    }
}

void add_stats(tcw_walk_stats& a, const tcw_walk_stats& b) {
    a.steps += b.steps;
    a.dps += b.dps;
    a.inserts += b.inserts;
    a.abandoned += b.abandoned;
    a.robin_hood += b.robin_hood;
    a.same_side += b.same_side;
    a.reduction += b.reduction;
    a.claws += b.claws;
    a.table_full += b.table_full;
    a.spin_timeouts += b.spin_timeouts;
    a.claws_dropped += b.claws_dropped;
}

// Exact check of claw candidate pairs (host arrays) of a space: the first that passes, in the order
// given, fills res.
// Device buffers of the exact claw check for up to `cap` candidate pairs of targets with up to r rows.
struct ClawWs {
    uint64_t *d0 = nullptr, *d1 = nullptr;
    int32_t *ok = nullptr, *perm = nullptr;
    int8_t* sign = nullptr;
    int64_t cap = 0;
    int r = 0;
    ClawWs() = default;
    ClawWs(const ClawWs&) = delete;
    ClawWs& operator=(const ClawWs&) = delete;
    ~ClawWs() { release(); }
    void release() {
        for (void* q : {(void*)d0, (void*)d1, (void*)ok, (void*)perm, (void*)sign})
            if (q) (void)hipFree(q);
        d0 = d1 = nullptr;
        ok = perm = nullptr;
        sign = nullptr;
        cap = 0;
        r = 0;
    }
    hipError_t reserve(int64_t m, int rows) {
        if (m <= cap && rows <= r) return hipSuccess;
        release();
        hipError_t e;
        if ((e = hipMalloc(&d0, m * 8)) != hipSuccess || (e = hipMalloc(&d1, m * 8)) != hipSuccess ||
            (e = hipMalloc(&ok, m * 4)) != hipSuccess || (e = hipMalloc(&perm, m * rows * 4)) != hipSuccess ||
            (e = hipMalloc(&sign, m * rows)) != hipSuccess) {
            release();
            return e;
        }
        cap = m;
        r = rows;
        return hipSuccess;
    }
};

// The context's scratch for exact claw checks of n-qubit spaces, grown when too small.
int ensure_claw_scratch(tcw_ctx* c, int n) {
    const size_t need = tcw::exact_claw_scratch_bytes(n);
    if (c->claw_scratch_bytes < need) {
        if (c->claw_scratch) (void)hipFree(c->claw_scratch);
        c->claw_scratch = nullptr;
        c->claw_scratch_bytes = 0;
        HIP_TRY(c, hipMalloc(&c->claw_scratch, need));
        c->claw_scratch_bytes = need;
    }
    return TCW_OK;
}

// Exact check of candidate pairs (u0[i], u1[i]) on the context's stream, in the given order; the first
// verified one fills res.  With ws and the claw scratch already large enough, it allocates nothing (so
// it can run beside other device work).
int check_pairs_ws(tcw_ctx* c, const Space& sp, const uint64_t* u0, const uint64_t* u1, int64_t m, tcw_result* res,
                   int* found, ClawWs& ws) {
    *found = 0;
    if (m <= 0) return TCW_OK;
    const int n = sp.n;
    const int R = 1 << (2 * n);
    HIP_TRY(c, ws.reserve(m, R));
    HIP_TRY(c, hipMemcpyAsync(ws.d0, u0, m * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(ws.d1, u1, m * 8, hipMemcpyHostToDevice, c->stream));
    if (int rc = ensure_claw_scratch(c, n)) return rc;
    HIP_TRY(c, tcw::exact_claw_check(sp.S, sp.k, ws.d0, ws.d1, m, c->claw_scratch, c->claw_scratch_bytes, ws.ok,
                                     ws.perm, ws.sign, c->stream));
    std::vector<int32_t> ok(m), perm(m * R);
    std::vector<int8_t> sign(m * R);
    HIP_TRY(c, hipMemcpyAsync(ok.data(), ws.ok, m * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(perm.data(), ws.perm, m * R * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(sign.data(), ws.sign, m * R, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < m; ++i) {
        if (!ok[i]) {
            res->false_claws++;
            continue;
        }
        uint64_t pv = u0[i], pw = u1[i];
        if ((pv >> 32) & 1) std::swap(pv, pw);
        const int h = sp.k / 2;
        std::vector<uint16_t> dv, dw, desc;
        decode_desc(pv, n, h, dv);
        decode_desc(pw, n, h, dw);
        desc = dv;
        for (int t = h - 1; t >= 0; --t) desc.push_back(dw[t]);
        if (sp.k % 2) desc.push_back((uint16_t)sp.chunk);
        res->status = TCW_STATUS_FOUND;
        res->t = sp.k;
        res->chunk = sp.chunk;
        std::memset(res->paulis, 0, sizeof(res->paulis));
        for (size_t j = 0; j < desc.size() && j < TCW_MAX_T; ++j) res->paulis[j] = desc[j];
        for (int q = 0; q < R; ++q) {
            res->clifford_perm[q] = perm[i * R + q];
            res->clifford_sign[q] = sign[i * R + q];
        }
        *found = 1;
        break;
    }
    return TCW_OK;
}

int check_pairs(tcw_ctx* c, const Space& sp, const uint64_t* u0, const uint64_t* u1, int64_t m, tcw_result* res,
                int* found) {
    ClawWs ws;
    return check_pairs_ws(c, sp, u0, u1, m, res, found, ws);
}

// Candidates of an enumerated space are checked in increasing (u0, u1) order, so the decomposition
// returned does not depend on the order in which the candidates were written.
void sort_pairs(uint64_t* u0, uint64_t* u1, int64_t m) {
    std::vector<std::pair<uint64_t, uint64_t>> v(m);
    for (int64_t i = 0; i < m; ++i) v[i] = {u0[i], u1[i]};
    std::sort(v.begin(), v.end());
    for (int64_t i = 0; i < m; ++i) {
        u0[i] = v[i].first;
        u1[i] = v[i].second;
    }
}

// New claw candidates of a walk session; `seen` counts those already checked.
int check_claws(tcw_ctx* c, tcw_walk* w, int64_t& seen, tcw_result* res, int* found) {
    *found = 0;
    int64_t total = 0;
    std::vector<uint64_t> u0(4096), u1(4096);
    int rc = tcw_walk_claws(w, u0.data(), u1.data(), 4096, &total);
    if (rc) return rc;
    const int64_t avail = total < 4096 ? total : 4096;
    if (avail <= seen) return TCW_OK;
    if (w->wd.enumerate) sort_pairs(u0.data() + seen, u1.data() + seen, avail - seen);
    rc = check_pairs(c, w->space, u0.data() + seen, u1.data() + seen, avail - seen, res, found);
    seen = avail;
    return rc;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int depth_order_of(tcw_ctx* c, const tcw_walk_params* p, std::vector<int>& order) {
    order.clear();
    if (p->k_max < 0 || p->k_max > TCW_MAX_T) return fail(c, TCW_EINVAL, "k_max out of range");
    if (p->depth_order_kind == TCW_ORDER_GIVEN || p->depth_order_kind == TCW_ORDER_GIVEN_FIRST) {
        if (p->depth_order_len < 0 || p->depth_order_len > 16) return fail(c, TCW_EINVAL, "bad depth order");
        for (int i = 0; i < p->depth_order_len; ++i) {
            const int k = p->depth_order[i];
            if (k < 0 || k > p->k_max) return fail(c, TCW_EINVAL, "depth order entry out of range");
            bool dup = false;
            for (int o : order) dup |= (o == k);
            if (!dup) order.push_back(k);
        }
    } else if (p->depth_order_kind != TCW_ORDER_PLAIN) {
        return fail(c, TCW_EINVAL, "depth_order_kind must be one of TCW_ORDER_*");
    }
    // the plain increasing order is the fallback for depths the given order left out
    for (int k = 0; k <= p->k_max; ++k) {
        bool have = false;
        for (int o : order) have |= (o == k);
        if (!have) order.push_back(k);
    }
    return TCW_OK;
}

// Depth 0: is U_hat itself a signed permutation (a Clifford)?
int search_k0(tcw_ctx* c, const tcw_target* t, tcw_result* res, int* found) {
    const int R = 1 << (2 * t->n);
    *found = 0;
    int32_t *dok = nullptr, *dperm = nullptr;
    int8_t* dsign = nullptr;
    DevScope scope;
    HIP_TRY(c, scope.alloc(&dok, 4));
    HIP_TRY(c, scope.alloc(&dperm, R * 4));
    HIP_TRY(c, scope.alloc(&dsign, R));
    HIP_TRY(c, tcw::exact_signed_perm(t->U, dok, dperm, dsign, c->stream));
    int32_t ok = 0;
    std::vector<int32_t> perm(R);
    std::vector<int8_t> sign(R);
    HIP_TRY(c, hipMemcpyAsync(&ok, dok, 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(perm.data(), dperm, R * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(sign.data(), dsign, R, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    res->spaces++;
    if (ok) {
        res->status = TCW_STATUS_FOUND;
        res->t = 0;
        res->chunk = 0;
        std::memset(res->paulis, 0, sizeof(res->paulis));
        for (int q = 0; q < R; ++q) {
            res->clifford_perm[q] = perm[q];
            res->clifford_sign[q] = sign[q];
        }
        *found = 1;
    }
    return TCW_OK;
}

// Ranges of the search parameters, checked before any of them enters a shift or a launch.  In a
// batch, walks and log2_table <= 0 take the autotuner's choice.
int check_params(tcw_ctx* c, const tcw_walk_params* p, int n, bool batch) {
    if (p->delta > 32) return fail(c, TCW_EINVAL, "delta must be at most 32 (negative: automatic)");
    if ((!batch && p->walks < 1) || p->walks > (1ll << 31)) return fail(c, TCW_EINVAL, "walks must be in 1..2^31");
    if ((!batch || p->log2_table > 0) && (p->log2_table < 4 || p->log2_table > 32))
        return fail(c, TCW_EINVAL, "log2_table must be in 4..32");
    if (p->trail_cap_factor < 1 || p->budget_beta < 1 || p->version_factor < 1)
        return fail(c, TCW_EINVAL, "trail_cap_factor, budget_beta and version_factor must be positive");
    if (p->delta >= 0 && ((uint64_t)p->trail_cap_factor << p->delta) > TCW_MAX_TRAIL_CAP)
        return fail(c, TCW_EINVAL, "trail_cap_factor * 2^delta exceeds TCW_MAX_TRAIL_CAP");
    if (p->enum_max < 0) return fail(c, TCW_EINVAL, "enum_max must be non-negative");
    const int32_t xi = (int32_t)xi_of(n);
    if (p->chunk_first < 0 || p->chunk_first > xi || p->chunk_last < 0 || p->chunk_last > xi)
        return fail(c, TCW_EINVAL, "chunk_first and chunk_last must lie in 1..xi (0: default)");
    if (!(p->max_seconds >= 0)) return fail(c, TCW_EINVAL, "max_seconds must be non-negative");
    if (p->launch_limit < 0) return fail(c, TCW_EINVAL, "launch_limit must be non-negative");
    return TCW_OK;
}

// Trail cap of a walk space: trail_cap_factor * 2^delta, at most TCW_MAX_TRAIL_CAP (a table value
// keeps 30 bits of trail length).
int trail_cap_of(tcw_ctx* c, const tcw_walk_params* p, int delta, uint32_t* cap) {
    const uint64_t v = (uint64_t)p->trail_cap_factor << delta;
    if (delta > 32 || v > TCW_MAX_TRAIL_CAP)
        return fail(c, TCW_EINVAL, "trail_cap_factor * 2^delta exceeds TCW_MAX_TRAIL_CAP for this space");
    *cap = (uint32_t)v;
    return TCW_OK;
}

// Steps per function version: max(factor * N, 2 walks / theta), but no more than the table holds
// at half load (slots / 2 distinguished points, i.e. slots / (2 theta) steps).
uint64_t version_steps(const tcw_walk_params* p, uint64_t npts, int delta, int64_t walks, int log2_table) {
    uint64_t per_version = (uint64_t)p->version_factor * npts;
    const uint64_t floor_v = 2ull * (uint64_t)walks << delta;
    if (per_version < floor_v) per_version = floor_v;
    const uint64_t table_v = (1ull << (log2_table - 1)) << delta;
    return per_version < table_v ? per_version : table_v;
}

// The least table size, at most 2^lg slots, that keeps the function version as long as 2^lg slots
// would (version_steps) with the table at most a quarter full when the version ends: the stored
// distinguished points, and so the walks, are the same, and a larger table would only cost memory,
// allocation and clears.
int version_table_log2(const tcw_walk_params* p, uint64_t npts, int delta, int64_t walks, int lg) {
    const uint64_t dps = version_steps(p, npts, delta, walks, lg) >> delta;
    int fit = 10;
    while (fit < lg && (1ull << (fit - 2)) < dps) ++fit;
    return fit < lg ? fit : lg;
}

// the tables of one group of concurrently searched chunks stay within 2^35 bytes (32 GiB)
constexpr int CHUNK_TABLE_POOL_LOG2 = 35;

// What may end a batched run early: a stop request on the context, or a launch limit.
struct StopCtl {
    std::atomic<int>* flag = nullptr;
    int64_t* launches = nullptr;  // launches so far in the calling search
    int64_t limit = 0;            // 0: none
    bool stopped = false;
    bool due() const {
        return (flag && flag->load(std::memory_order_relaxed) != 0) || (limit > 0 && launches && *launches >= limit);
    }
};

struct BatchTarget;
int search_chunks_concurrent(tcw_ctx* c, const tcw_target* t, const tcw_walk_params* p, int k, int c_first,
                             int c_last, int delta, tcw_result* res, int* found, bool* cut, StopCtl* stop, double t0);

}  // namespace

// One tcw_search as a state machine that advances by one launch (or one set-up step) at a time, so
// that a stop request or a launch limit can end the call at a launch boundary and a stopped search
// can be serialised and resumed.
struct SearchRun {
    const tcw_target* t = nullptr;
    tcw_walk_params p{};
    tcw_result res{};
    std::vector<int32_t> order;   // depths in search order (a given order, then the plain fallback)
    int32_t oi = 0;               // next entry of order
    std::vector<int32_t> refine;  // TCW_ORDER_GIVEN after a hit: the depths below it not yet searched
    int32_t ri = 0;
    int32_t refining = 0;
    int32_t finished = 0;
    uint64_t searched = 0;        // bit k: depth k was started
    // current depth
    int32_t in_depth = 0, k = -1, cf = 0, cl = 0, chunk = 0, delta = 0, enumerate = 0, iters = 0;
    int32_t depth_cut = 0;        // the depth was cut short by the wall-clock cap
    uint64_t npts = 0;
    // current space: a walk session
    tcw_walk* w = nullptr;
    uint64_t budget = 0, per_version = 0, used = 0, used_v = 0;
    uint32_t version = 0;
    int64_t seen = 0;
    double elapsed = 0;           // seconds spent in earlier calls (before a stop)
    bool checkpointable = true;   // false after a stop inside a group of concurrent chunks
    ~SearchRun() {
        if (w) tcw_walk_end(w);
    }
};

void free_search_run(SearchRun* r) { delete r; }

namespace {

bool over_time(const SearchRun& s, double t0) {
    return s.p.max_seconds > 0 && s.elapsed + (now_s() - t0) > s.p.max_seconds;
}

void close_space(SearchRun& s) {
    if (s.w) {
        tcw_walk_end(s.w);
        s.w = nullptr;
    }
}

// A verified decomposition at depth s.k (already in s.res).  With TCW_ORDER_GIVEN the depths below it
// that have not been searched are searched next, in increasing order; the first of them to yield a
// decomposition is the lowest, and ends the search.
void on_hit(SearchRun& s) {
    close_space(s);
    s.in_depth = 0;
    if (s.p.depth_order_kind == TCW_ORDER_GIVEN && !s.refining) {
        s.refining = 1;
        s.refine.clear();
        for (int d = 0; d < s.res.t; ++d)
            if (!(s.searched >> d & 1)) s.refine.push_back(d);
        s.ri = 0;
        if (!s.refine.empty()) return;
    }
    s.finished = 1;
}

// Open the walk session of chunk s.chunk of the current depth.
int open_space(tcw_ctx* c, SearchRun& s) {
    const tcw_target* t = s.t;
    const tcw_walk_params* p = &s.p;
    tcw_space sp{s.k, s.chunk, p->seed, p->version, s.enumerate ? 0 : s.delta};
    s.res.spaces++;
    s.res.versions++;
    s.version = p->version;
    s.used = s.used_v = 0;
    s.seen = 0;
    int rc = TCW_OK;
    if (s.enumerate) {
        int64_t walks = (int64_t)s.npts < p->walks ? (int64_t)s.npts : p->walks;
        if (walks < 64) walks = (int64_t)s.npts < 64 ? (int64_t)s.npts : 64;
        int lg = 4;
        while ((1ull << lg) < 4 * s.npts && lg < 30) ++lg;
        s.budget = s.npts;
        s.per_version = ~0ull;
        rc = tcw_walk_begin(c, t, &sp, walks, lg, 2, 1, &s.w);
    } else {
        uint32_t cap = 0;
        if ((rc = trail_cap_of(c, p, s.delta, &cap))) return rc;
        const int64_t walks = walks_for(p->walks, s.npts);
        const int lg = version_table_log2(p, s.npts, s.delta, walks, p->log2_table);
        s.budget = (uint64_t)p->budget_beta * s.npts << s.delta;
        s.per_version = version_steps(p, s.npts, s.delta, walks, lg);
        // a launch must not overrun a function version
        const uint64_t fit = s.per_version / (uint64_t)walks;
        if ((uint64_t)s.iters > fit) s.iters = fit > 0 ? (int)fit : 1;
        rc = tcw_walk_begin(c, t, &sp, walks, lg, cap, 0, &s.w);
    }
    return rc;
}

// Start the next depth of the order (or of the refinement list); sets s.finished when none is left.
int next_depth(tcw_ctx* c, SearchRun& s, StopCtl* stop, double t0) {
    const tcw_target* t = s.t;
    const tcw_walk_params* p = &s.p;
    const int n = t->n;
    int k = -1;
    for (;;) {
        if (s.refining) {
            if (s.ri >= (int32_t)s.refine.size()) break;
            k = s.refine[s.ri++];
        } else {
            if (s.oi >= (int32_t)s.order.size()) break;
            k = s.order[s.oi++];
        }
        if (!(s.searched >> k & 1)) break;
        k = -1;
    }
    if (k < 0) {
        s.finished = 1;
        return TCW_OK;
    }
    s.searched |= 1ull << k;
    s.k = k;
    s.depth_cut = 0;
    int found = 0, rc = TCW_OK;
    if (k == 0) {
        if ((rc = search_k0(c, t, &s.res, &found))) return rc;
        if (found) on_hit(s);
        else s.res.failed_depths |= 1ull;
        return TCW_OK;
    }
    const uint64_t nh = n_half_of(n, k / 2);
    if (nh == 0) return TCW_OK;  // space beyond 32-bit points: not searchable here (not a failed depth)
    s.npts = 2 * nh;
    s.cf = s.cl = 0;
    if (k % 2) {
        s.cf = p->chunk_first > 0 ? p->chunk_first : 1;
        s.cl = p->chunk_last > 0 ? std::min<int>(p->chunk_last, (int)xi_of(n)) : (int)xi_of(n);
    }
    s.enumerate = (int64_t)s.npts <= p->enum_max;
    s.delta = p->delta >= 0 ? p->delta : auto_delta(s.npts, p->log2_table);
    s.iters = p->iters_per_launch > 0 ? p->iters_per_launch : default_iters(n);
    // odd depths with chunk_parallel != 1 run their chunks as concurrent batch members; enumerated
    // chunks only while their tables (4 npts slots of 16 B each) fit the chunk pool
    const uint64_t n_chunks = (uint64_t)(s.cl - s.cf + 1);
    const bool concurrent = k % 2 && p->chunk_parallel != 1 &&
                            (!s.enumerate || n_chunks * 64 * s.npts <= (1ull << CHUNK_TABLE_POOL_LOG2));
    if (concurrent) {
        if (!s.enumerate) {
            uint32_t cap = 0;
            if ((rc = trail_cap_of(c, p, s.delta, &cap))) return rc;
        }
        const int G = p->chunk_parallel <= 0 ? s.cl - s.cf + 1 : p->chunk_parallel;
        bool cut = false;
        for (int first = s.cf; first <= s.cl && !found; first += G) {
            if (over_time(s, t0)) {
                cut = true;
                break;
            }
            // each member resolves an open delta against its own (smaller) table
            rc = search_chunks_concurrent(c, t, p, k, first, std::min(s.cl, first + G - 1), p->delta, &s.res, &found,
                                          &cut, stop, t0 - s.elapsed);
            if (rc) return rc;
            if (stop && stop->stopped) {
                // stopped inside a group: the members are not serialised, so this search cannot be
                // checkpointed; a later call would repeat the depth
                s.checkpointable = false;
                return TCW_OK;
            }
        }
        if (found) on_hit(s);
        else if (!cut) s.res.failed_depths |= 1ull << k;
        return TCW_OK;
    }
    s.in_depth = 1;
    s.chunk = s.cf;
    return open_space(c, s);
}

// One launch of the current space, then the exact check of its new claw candidates and the
// bookkeeping of budgets, function versions and chunks.
int space_launch(tcw_ctx* c, SearchRun& s, int64_t* launches, double t0) {
    tcw_walk* w = s.w;
    int rc = tcw_walk_run(w, s.iters);
    s.res.launches++;
    (*launches)++;
    tcw_walk_stats st{};
    if (!rc) rc = tcw_walk_stats_get(w, &st);
    int found = 0;
    if (!rc && (!s.enumerate || st.active_walks == 0)) rc = check_claws(c, w, s.seen, &s.res, &found);
    if (rc) return rc;
    s.used = s.used - s.used_v + (uint64_t)st.steps;
    s.used_v = (uint64_t)st.steps;
    const bool space_done = s.enumerate ? st.active_walks == 0 : s.used >= s.budget;
    if (found || space_done) {
        add_stats(s.res.stats, st);
        close_space(s);
        if (found) {
            on_hit(s);
            return TCW_OK;
        }
        if (s.k % 2 && s.chunk < s.cl) {
            s.chunk++;
            return open_space(c, s);
        }
        s.in_depth = 0;
        if (!s.depth_cut) s.res.failed_depths |= 1ull << s.k;
        return TCW_OK;
    }
    if (over_time(s, t0)) {
        add_stats(s.res.stats, st);
        close_space(s);
        s.in_depth = 0;
        s.depth_cut = 1;
        s.finished = 1;
        return TCW_OK;
    }
    if (!s.enumerate && s.used_v >= s.per_version) {
        add_stats(s.res.stats, st);
        s.used_v = 0;
        s.seen = 0;
        ++s.version;
        s.res.versions++;
        return tcw_walk_reset(w, s.version);
    }
    return TCW_OK;
}

void finish_result(SearchRun& s, double t0) {
    tcw_result& r = s.res;
    r.seconds = s.elapsed + (now_s() - t0);
    if (r.status != TCW_STATUS_FOUND) {
        r.status = TCW_STATUS_NOT_FOUND;
        r.minimal = 0;
        return;
    }
    const uint64_t below = r.t >= 64 ? ~0ull : ((1ull << r.t) - 1);
    r.minimal = (r.failed_depths & below) == below ? 1 : 0;
}

// Runs s until it finishes, fails, or a stop request or the launch limit ends the call.  A stopped
// search moves into the context (c->stopped) with status TCW_STATUS_STOPPED in *res.
int run_search(tcw_ctx* c, SearchRun* s, tcw_result* res) {
    const double t0 = now_s();
    int64_t launches = 0;
    StopCtl stop;
    stop.flag = &c->stop_req;
    stop.launches = &launches;
    stop.limit = s->p.launch_limit;
    int rc = TCW_OK;
    while (!s->finished) {
        if (stop.due()) {
            c->stop_req.store(0);
            stop.stopped = true;
        }
        if (stop.stopped) break;
        if (s->in_depth) rc = space_launch(c, *s, &launches, t0);
        else if (over_time(*s, t0)) s->finished = 1;
        else rc = next_depth(c, *s, &stop, t0);
        if (rc) break;
    }
    if (rc) {
        delete s;
        return rc;
    }
    if (stop.stopped && !s->finished) {
        s->elapsed += now_s() - t0;
        *res = s->res;
        if (s->w) {
            // the open space's counters so far (kept out of s->res, which adds them when the space ends)
            tcw_walk_stats st{};
            if ((rc = tcw_walk_stats_get(s->w, &st))) {
                delete s;
                return rc;
            }
            add_stats(res->stats, st);
        }
        res->status = TCW_STATUS_STOPPED;
        res->minimal = 0;
        res->seconds = s->elapsed;
        if (s->res.status == TCW_STATUS_FOUND) res->t = s->res.t;  // a hit awaiting the depths below it
        if (c->stopped) free_search_run(c->stopped);
        c->stopped = s;
        return TCW_OK;
    }
    finish_result(*s, t0);
    *res = s->res;
    delete s;
    return TCW_OK;
}

}  // namespace

extern "C" int tcw_search(tcw_ctx* c, const tcw_target* t, const tcw_walk_params* p, tcw_result* res) {
    if (!c || !t || !p || !res) return TCW_EINVAL;
    std::memset(res, 0, sizeof(*res));
    if (c->stopped) {
        free_search_run(c->stopped);
        c->stopped = nullptr;
    }
    const int n = t->n;
    res->n = n;
    int rc = check_params(c, p, n, false);
    if (rc) return rc;
    std::vector<int> order;
    rc = depth_order_of(c, p, order);
    if (rc) return rc;
    SearchRun* s = new (std::nothrow) SearchRun();
    if (!s) return TCW_ENOMEM;
    s->t = t;
    s->p = *p;
    s->res.n = n;
    s->order.assign(order.begin(), order.end());
    return run_search(c, s, res);
}

extern "C" int tcw_search_stop(tcw_ctx* c) {
    if (!c) return TCW_EINVAL;
    c->stop_req.store(1);
    return TCW_OK;
}

// ---- checkpoints of a stopped search ----
namespace {

constexpr uint64_t CKPT_MAGIC = 0x3154504B43574354ull;  // "TCWCKPT1"

struct Writer {
    std::vector<uint8_t> buf;
    template <typename T>
    void put(const T& v) {
        const uint8_t* q = reinterpret_cast<const uint8_t*>(&v);
        buf.insert(buf.end(), q, q + sizeof(T));
    }
    void bytes(const void* q, size_t len) {
        const uint8_t* b = static_cast<const uint8_t*>(q);
        buf.insert(buf.end(), b, b + len);
    }
    template <typename T>
    void vec(const std::vector<T>& v) {
        put<uint64_t>(v.size());
        if (!v.empty()) bytes(v.data(), v.size() * sizeof(T));
    }
};

struct Reader {
    const uint8_t* p;
    size_t len, at = 0;
    bool ok = true;
    template <typename T>
    T get() {
        T v{};
        if (at + sizeof(T) > len) {
            ok = false;
            return v;
        }
        std::memcpy(&v, p + at, sizeof(T));
        at += sizeof(T);
        return v;
    }
    const uint8_t* take(size_t n) {
        if (!ok || at + n > len || at + n < at) {
            ok = false;
            return nullptr;
        }
        const uint8_t* q = p + at;
        at += n;
        return q;
    }
    template <typename T>
    void vec(std::vector<T>& v, size_t max_count) {
        const uint64_t cnt = get<uint64_t>();
        if (!ok || cnt > max_count) {
            ok = false;
            return;
        }
        const uint8_t* q = take(cnt * sizeof(T));
        if (!q) return;
        v.resize(cnt);
        if (cnt) std::memcpy(v.data(), q, cnt * sizeof(T));
    }
};

// A fingerprint of the target's exact channel rep (reduced form), to refuse a resume on another target.
int target_fingerprint(tcw_ctx* c, const tcw_target* t, uint64_t* fp) {
    const size_t rr = (size_t)1 << (4 * t->n);
    std::vector<int32_t> a(rr), b(rr);
    int32_t e = 0;
    int rc = tcw_target_channel(c, t, a.data(), b.data(), &e);
    if (rc) return rc;
    uint64_t h = tcw::mix64(0x5450524e54ull ^ (uint64_t)t->n);
    h = tcw::mix64(h ^ (uint64_t)(uint32_t)e);
    for (size_t i = 0; i < rr; ++i) h = tcw::mix64(h ^ (((uint64_t)(uint32_t)a[i] << 32) | (uint32_t)b[i]));
    *fp = h;
    return TCW_OK;
}

int serialise(tcw_ctx* c, const SearchRun& s, std::vector<uint8_t>& out) {
    Writer w;
    uint64_t fp = 0;
    int rc = target_fingerprint(c, s.t, &fp);
    if (rc) return rc;
    w.put(CKPT_MAGIC);
    w.put<uint32_t>(sizeof(tcw_walk_params));
    w.put<uint32_t>(sizeof(tcw_result));
    w.put<int32_t>(s.t->n);
    w.put(fp);
    w.put(s.p);
    w.put(s.res);
    w.vec(s.order);
    w.put(s.oi);
    w.vec(s.refine);
    w.put(s.ri);
    w.put(s.refining);
    w.put(s.searched);
    w.put(s.in_depth);
    w.put(s.k);
    w.put(s.cf);
    w.put(s.cl);
    w.put(s.chunk);
    w.put(s.delta);
    w.put(s.enumerate);
    w.put(s.iters);
    w.put(s.depth_cut);
    w.put(s.npts);
    w.put(s.elapsed);
    const int32_t has_space = s.w ? 1 : 0;
    w.put(has_space);
    if (has_space) {
        const tcw::WalkDev& wd = s.w->wd;
        w.put(s.budget);
        w.put(s.per_version);
        w.put(s.used);
        w.put(s.used_v);
        w.put(s.version);
        w.put(s.seen);
        w.put<int64_t>(wd.walks);
        w.put<int32_t>(wd.log2_table);
        w.put<uint32_t>(wd.cap);
        w.put<int32_t>(wd.enumerate);
        w.put<int64_t>(s.w->launches);
        unsigned long long st[tcw::ST_COUNT];
        unsigned long long cc = 0;
        HIP_TRY(c, hipMemcpyAsync(st, wd.stats, sizeof(st), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(&cc, wd.claw_count, sizeof(cc), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        w.bytes(st, sizeof(st));
        w.put<uint64_t>(cc);
        const size_t sbytes = (size_t)wd.walks * sizeof(tcw::WalkState);
        const size_t tbytes = ((size_t)1 << wd.log2_table) * 16;
        const size_t at = w.buf.size();
        w.buf.resize(at + sbytes + tbytes);
        HIP_TRY(c, hipMemcpyAsync(w.buf.data() + at, wd.states, sbytes, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(w.buf.data() + at + sbytes, wd.table, tbytes, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    out.swap(w.buf);
    return TCW_OK;
}

}  // namespace

extern "C" int tcw_checkpoint(tcw_ctx* c, void* host_buf, size_t* len) {
    if (!c || !len) return TCW_EINVAL;
    if (!c->stopped) return fail(c, TCW_ESTATE, "no stopped search in this context");
    if (!c->stopped->checkpointable)
        return fail(c, TCW_ESTATE, "the search stopped inside a group of concurrent chunks (chunk_parallel != 1)");
    std::vector<uint8_t> buf;
    int rc = serialise(c, *c->stopped, buf);
    if (rc) return rc;
    const size_t have = *len;
    *len = buf.size();
    if (!host_buf) return TCW_OK;
    if (have < buf.size()) return fail(c, TCW_EINVAL, "checkpoint buffer too small");
    std::memcpy(host_buf, buf.data(), buf.size());
    return TCW_OK;
}

extern "C" int tcw_resume(tcw_ctx* c, const tcw_target* t, const void* host_buf, size_t len, int64_t launch_limit,
                          tcw_result* res) {
    if (!c || !t || !host_buf || !res || launch_limit < 0) return TCW_EINVAL;
    std::memset(res, 0, sizeof(*res));
    if (c->stopped) {
        free_search_run(c->stopped);
        c->stopped = nullptr;
    }
    Reader r{static_cast<const uint8_t*>(host_buf), len};
    auto bad = [&](const char* what) { return fail(c, TCW_EINVAL, std::string("checkpoint: ") + what); };
    if (r.get<uint64_t>() != CKPT_MAGIC) return bad("not a search checkpoint");
    if (r.get<uint32_t>() != sizeof(tcw_walk_params) || r.get<uint32_t>() != sizeof(tcw_result))
        return bad("written by another version of the library");
    const int32_t n = r.get<int32_t>();
    const uint64_t fp = r.get<uint64_t>();
    if (!r.ok || n != t->n) return bad("target has another qubit count");
    uint64_t fp_t = 0;
    int rc = target_fingerprint(c, t, &fp_t);
    if (rc) return rc;
    if (fp != fp_t) return bad("taken on another target");
    std::unique_ptr<SearchRun> s(new (std::nothrow) SearchRun());
    if (!s) return TCW_ENOMEM;
    s->t = t;
    s->p = r.get<tcw_walk_params>();
    s->res = r.get<tcw_result>();
    r.vec(s->order, 65);
    s->oi = r.get<int32_t>();
    r.vec(s->refine, 65);
    s->ri = r.get<int32_t>();
    s->refining = r.get<int32_t>();
    s->searched = r.get<uint64_t>();
    s->in_depth = r.get<int32_t>();
    s->k = r.get<int32_t>();
    s->cf = r.get<int32_t>();
    s->cl = r.get<int32_t>();
    s->chunk = r.get<int32_t>();
    s->delta = r.get<int32_t>();
    s->enumerate = r.get<int32_t>();
    s->iters = r.get<int32_t>();
    s->depth_cut = r.get<int32_t>();
    s->npts = r.get<uint64_t>();
    s->elapsed = r.get<double>();
    const int32_t has_space = r.get<int32_t>();
    if (!r.ok) return bad("truncated");
    s->p.launch_limit = launch_limit;
    if ((rc = check_params(c, &s->p, n, false))) return rc;
    if (s->oi < 0 || s->oi > (int32_t)s->order.size() || s->ri < 0 || s->ri > (int32_t)s->refine.size())
        return bad("depth-loop position out of range");
    for (int32_t k : s->order)
        if (k < 0 || k > TCW_MAX_T) return bad("depth out of range");
    for (int32_t k : s->refine)
        if (k < 0 || k > TCW_MAX_T) return bad("depth out of range");
    if (s->in_depth != (has_space ? 1 : 0)) return bad("inconsistent space state");
    if (has_space) {
        s->budget = r.get<uint64_t>();
        s->per_version = r.get<uint64_t>();
        s->used = r.get<uint64_t>();
        s->used_v = r.get<uint64_t>();
        s->version = r.get<uint32_t>();
        s->seen = r.get<int64_t>();
        const int64_t walks = r.get<int64_t>();
        const int32_t lg = r.get<int32_t>();
        const uint32_t cap = r.get<uint32_t>();
        const int32_t en = r.get<int32_t>();
        const int64_t wl = r.get<int64_t>();
        unsigned long long st[tcw::ST_COUNT];
        const uint8_t* stq = r.take(sizeof(st));
        const uint64_t cc = r.get<uint64_t>();
        if (!r.ok || walks < 1 || walks > (1ll << 31) || lg < 4 || lg > 32 || en != s->enumerate)
            return bad("malformed walk session");
        const size_t sbytes = (size_t)walks * sizeof(tcw::WalkState);
        const size_t tbytes = ((size_t)1 << lg) * 16;
        const uint8_t* sq = r.take(sbytes);
        const uint8_t* tq = r.take(tbytes);
        if (!r.ok || !sq || !tq) return bad("truncated walk session");
        std::memcpy(st, stq, sizeof(st));
        tcw_space sp{s->k, s->chunk, s->p.seed, s->version, s->enumerate ? 0 : s->delta};
        if ((rc = tcw_walk_begin(c, t, &sp, walks, lg, cap, en, &s->w))) return rc;
        tcw::WalkDev& wd = s->w->wd;
        s->w->launches = wl;
        HIP_TRY(c, hipMemcpyAsync(wd.states, sq, sbytes, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(wd.table, tq, tbytes, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(wd.stats, st, sizeof(st), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(wd.claw_count, &cc, sizeof(cc), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    if (r.at != len) return bad("trailing bytes");
    return run_search(c, s.release(), res);
}

// ---------------------------------------------------------------------------------------------
// Autotuner and batched search (many targets of mixed n and k)
namespace {

int64_t floor_pow2(uint64_t v) {
    int64_t p = 1;
    while ((uint64_t)(p * 2) <= v) p *= 2;
    return p;
}

int autotune(tcw_ctx* c, const tcw_target* t, int k, int chunk, int delta, uint64_t seed, TunedCfg* out) {
    const int n = t->n;
    const uint64_t key = ((uint64_t)n << 40) | ((uint64_t)k << 20) | (uint64_t)delta;
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) {
        *out = it->second;
        return TCW_OK;
    }
    const uint64_t npts = 2 * n_half_of(n, k / 2);
    if (npts == 0) return fail(c, TCW_EINVAL, "space too large");
    // walks beyond N/4 only add warm-up (m / theta steps before the first distinguished points)
    const int64_t wmax = std::min<int64_t>(1 << 20, std::max<int64_t>(64, floor_pow2(npts / 4)));
    std::vector<int64_t> cands;
    for (int64_t w = 64; w < wmax; w *= 4) cands.push_back(w);
    cands.push_back(wmax);
    tcw_space sp{k, chunk, seed, 0xFFFFu, delta};
    std::vector<double> rates;
    for (int64_t w : cands) {
        tcw_walk* ws = nullptr;
        const uint64_t acap = std::min<uint64_t>((uint64_t)20 << delta, TCW_MAX_TRAIL_CAP);
        int rc = tcw_walk_begin(c, t, &sp, w, 16, (uint32_t)acap, 0, &ws);
        if (rc) return rc;
        const int iters = (int)std::max<int64_t>(1, std::min<int64_t>(64, (1 << 21) / w));
        float ms = 0, tot = 0;
        rc = tcw_walk_run(ws, iters);
        if (!rc) rc = tcw_walk_last_ms(ws, &ms);
        for (int r = 0; r < 2 && !rc; ++r) {
            rc = tcw_walk_run(ws, iters);
            if (!rc) rc = tcw_walk_last_ms(ws, &ms);
            tot += ms;
        }
        tcw_walk_end(ws);
        if (rc) return rc;
        rates.push_back((double)w * iters * 2 / (tot * 1e-3));
    }
    double best = 0;
    for (double r : rates) best = std::max(best, r);
    size_t pick = cands.size() - 1;
    for (size_t i = 0; i < cands.size(); ++i)
        if (rates[i] >= 0.85 * best) {
            pick = i;
            break;
        }
    TunedCfg cfg;
    cfg.walks = cands[pick];
    cfg.rate = rates[pick];
    // launches of about 4 ms between host checks
    cfg.iters = (int)std::max(1.0, std::min(64.0, cfg.rate * 4e-3 / (double)cfg.walks));
    // the table holds every distinguished point of a version: max(2 N theta, 2 m) of them, 4x headroom
    const double dps = std::max(2.0 * (double)npts / (double)(1ull << delta), 2.0 * (double)cfg.walks);
    int lg = 10;
    while ((double)(1ull << lg) < 4 * dps && lg < 26) ++lg;
    cfg.log2_table = lg;
    c->tuned[key] = cfg;
    *out = cfg;
    return TCW_OK;
}

constexpr uint32_t BATCH_CLAW_CAP = 1024;

struct BatchTarget {
    const tcw_target* t = nullptr;
    tcw_walk_params p{};
    tcw_result* res = nullptr;
    std::vector<int> order;
    size_t oi = 0;
    std::vector<int> refine;  // TCW_ORDER_GIVEN after a hit: unsearched depths below it, ascending
    size_t ri = 0;
    bool refining = false;
    uint64_t searched = 0;    // bit k: depth k was started
    int k = -1, chunk = 0, cl = 0;
    bool walking = false, done = false, cut = false;
    // held: the space is at its budget or version end but claw candidates of its last round are still
    // being checked; the member sits out the rounds until they are
    bool held = false;
    std::vector<uint64_t> pu0, pu1;  // candidates read after the last round, checked during the next
    std::unique_ptr<Space> space;
    tcw::WalkDev wd{};
    int64_t walks = 0;
    int iters = 0, log2 = 0;
    uint64_t budget = 0, per_version = 0, used = 0, used_v = 0;
    uint32_t version = 0;
    int64_t seen = 0;
    size_t states_cap = 0;
    int table_cap = 0;
};

struct BatchBuffers {
    unsigned long long* stats = nullptr;   // count x ST_COUNT
    unsigned long long* claw_count = nullptr;
    uint64_t* claws = nullptr;             // count x BATCH_CLAW_CAP x 2
    tcw::SpaceDev* sps = nullptr;          // count
    tcw::WalkDev* wds = nullptr;           // count
    tcw::WorkItem* items[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // work queue per qubit count
    int64_t items_cap[5] = {0, 0, 0, 0, 0};
    int32_t* counts = nullptr;             // 5: items queued per qubit count
    int32_t* heads = nullptr;              // 5: queue positions (zeroed by a kernel at the start of a round)
    int32_t* restart = nullptr;            // count: slots restarted before the next round
    std::vector<int32_t> pending;          // host: members whose restart waits for the next round
    ~BatchBuffers() {
        for (void* q : {(void*)stats, (void*)claw_count, (void*)claws, (void*)sps, (void*)wds, (void*)counts,
                        (void*)heads, (void*)restart})
            if (q) (void)hipFree(q);
        for (auto* q : items)
            if (q) (void)hipFree(q);
    }
};

// back to the context's pool: the caller has synchronised every stream that used them
void free_walk_buffers(tcw_ctx* c, BatchTarget& b) {
    pool_put(c, b.wd.states, b.states_cap);
    if (b.wd.table) pool_put(c, b.wd.table, ((size_t)1 << b.table_cap) * 16);
    b.wd.states = nullptr;
    b.wd.table = nullptr;
    b.states_cap = 0;
    b.table_cap = 0;
}

// (Re)start the walks of a target's current space: table cleared, counters zeroed, walks initialised.
// Queued and done for every pending member in one launch on the batch stream before the next round
// (k_member_restart), after that round's descriptors are on the device.
void batch_restart(BatchBuffers& bb, int slot) { bb.pending.push_back(slot); }

// A verified decomposition of member b (in b.res).  TCW_ORDER_GIVEN then searches the depths below it
// not yet searched, in increasing order (the first further hit is the lowest); otherwise b is done.
void batch_on_hit(BatchTarget& b) {
    if (b.p.depth_order_kind == TCW_ORDER_GIVEN && !b.refining) {
        b.refining = true;
        b.refine.clear();
        for (int d = 0; d < b.res->t; ++d)
            if (!(b.searched >> d & 1)) b.refine.push_back(d);
        b.ri = 0;
        b.chunk = b.cl = 0;  // the next space starts a new depth
        if (!b.refine.empty()) return;
    }
    b.done = true;
}

// Move a target to its next space: depth 0 is checked on the spot; the next space of a positive
// depth, enumerated when small and walked otherwise, leaves the target `walking`.  prev_done: the
// current space ran to its budget without a verified decomposition (so its depth is failed once its
// last chunk is done).
int batch_advance(tcw_ctx* c, BatchTarget& b, int slot, BatchBuffers& bb, double t0, bool prev_done) {
    const int n = b.t->n;
    const uint32_t xi = xi_of(n);
    while (!b.done) {
        if (b.p.max_seconds > 0 && now_s() - t0 > b.p.max_seconds) {
            b.done = true;
            b.cut = true;
            break;
        }
        // next (k, chunk)
        if (prev_done && b.k >= 0 && b.k % 2 == 1 && b.chunk < b.cl) {
            b.chunk++;
        } else {
            if (prev_done && b.k >= 1) b.res->failed_depths |= 1ull << b.k;
            prev_done = false;
            int k = -1;
            for (;;) {
                if (b.refining) {
                    if (b.ri >= b.refine.size()) break;
                    k = b.refine[b.ri++];
                } else {
                    if (b.oi >= b.order.size()) break;
                    k = b.order[b.oi++];
                }
                if (!(b.searched >> k & 1)) break;
                k = -1;
            }
            if (k < 0) {
                b.done = true;
                break;
            }
            b.searched |= 1ull << k;
            b.k = k;
            b.chunk = 0;
            b.cl = 0;
            if (b.k % 2) {
                b.chunk = b.p.chunk_first > 0 ? b.p.chunk_first : 1;
                b.cl = b.p.chunk_last > 0 ? std::min<int>(b.p.chunk_last, (int)xi) : (int)xi;
            }
        }
        int found = 0, rc = 0;
        if (b.k == 0) {
            if ((rc = search_k0(c, b.t, b.res, &found))) return rc;
            if (found) {
                batch_on_hit(b);
            } else {
                b.res->failed_depths |= 1ull;
            }
            continue;
        }
        const uint64_t nh = n_half_of(n, b.k / 2);
        if (nh == 0) {
            b.chunk = b.cl;
            continue;
        }
        const uint64_t npts = 2 * nh;
        // A small space is enumerated: every point evaluated once, keyed in the table by its full
        // matrix hash, as one more member of the batch; it is done after npts steps.  Larger
        // spaces are walked.
        const bool enumerate = (int64_t)npts <= b.p.enum_max;
        int delta = 0;
        uint32_t cap = 2;
        if (enumerate) {
            const int64_t wmax = std::max<int64_t>(64, b.p.walks);
            b.walks = (int64_t)npts < wmax ? (int64_t)npts : wmax;
            int lg = 4;
            while ((1ull << lg) < 4 * npts && lg < 30) ++lg;
            b.log2 = lg;
            b.iters = default_iters(n);
        } else {
            delta = b.p.delta >= 0 ? b.p.delta
                                   : auto_delta(npts, b.p.log2_table > 0 ? b.p.log2_table : default_log2_table(n));
            if ((rc = trail_cap_of(c, &b.p, delta, &cap))) return rc;
            TunedCfg cfg;
            if (b.p.walks <= 0 || b.p.log2_table <= 0 || b.p.iters_per_launch <= 0) {
                if ((rc = autotune(c, b.t, b.k, b.chunk, delta, b.p.seed, &cfg))) return rc;
            }
            b.walks = walks_for(b.p.walks > 0 ? b.p.walks : cfg.walks, npts);
            b.log2 = version_table_log2(&b.p, npts, delta, b.walks,
                                        b.p.log2_table > 0 ? b.p.log2_table : cfg.log2_table);
            b.iters = b.p.iters_per_launch > 0 ? b.p.iters_per_launch : cfg.iters;
        }
        // the member's previous space is finished (its candidates were checked and the round that
        // used it has completed), so its buffers serve the next one
        if (!b.space) {
            b.space.reset(new Space());
            b.space->pooled = true;
        }
        tcw_space sp{b.k, b.chunk, b.p.seed, b.p.version, delta};
        if ((rc = prepare_space(c, b.t, &sp, *b.space))) return rc;
        b.res->spaces++;
        b.res->versions++;
        b.version = b.p.version;
        if (enumerate) {
            b.budget = npts;
            b.per_version = ~0ull;  // no function versions: the enumeration is exhaustive
        } else {
            b.budget = (uint64_t)b.p.budget_beta * npts << delta;
            b.per_version = version_steps(&b.p, npts, delta, b.walks, b.log2);
            const uint64_t fit = b.per_version / (uint64_t)b.walks;
            if ((uint64_t)b.iters > fit) b.iters = fit > 0 ? (int)fit : 1;
        }
        b.used = b.used_v = 0;
        b.seen = 0;
        // walk buffers (kept across spaces when large enough)
        const size_t sbytes = (size_t)b.walks * sizeof(tcw::WalkState);
        if (b.states_cap < sbytes) {
            pool_put(c, b.wd.states, b.states_cap);  // no round is in flight here
            b.wd.states = nullptr;
            b.states_cap = 0;
            HIP_TRY(c, pool_alloc(c, reinterpret_cast<void**>(&b.wd.states), sbytes));
            b.states_cap = sbytes;
        }
        if (b.table_cap < b.log2) {
            if (b.wd.table) pool_put(c, b.wd.table, ((size_t)1 << b.table_cap) * 16);
            b.wd.table = nullptr;
            b.table_cap = 0;
            HIP_TRY(c, pool_alloc(c, reinterpret_cast<void**>(&b.wd.table), ((size_t)1 << b.log2) * 16));
            b.table_cap = b.log2;
        }
        b.wd.walks = b.walks;
        b.wd.log2_table = b.log2;
        b.wd.cap = cap;
        b.wd.enumerate = enumerate ? 1 : 0;
        b.wd.n_points = npts;
        b.wd.stats = bb.stats + (size_t)slot * tcw::ST_COUNT;
        b.wd.claws = bb.claws + (size_t)slot * BATCH_CLAW_CAP * 2;
        b.wd.claw_count = bb.claw_count + slot;
        b.wd.claw_cap = BATCH_CLAW_CAP;
        batch_restart(bb, slot);
        b.walking = true;
        return TCW_OK;
    }
    b.walking = false;
    free_walk_buffers(c, b);  // between rounds: its last round has completed
    return TCW_OK;
}

}  // namespace

extern "C" int tcw_autotune(tcw_ctx* c, const tcw_target* t, int k, int chunk, int delta, uint64_t seed,
                            int64_t* walks, int* iters, int* log2_table, double* steps_per_s) {
    if (!c || !t || !walks || !iters || !log2_table || !steps_per_s) return TCW_EINVAL;
    tcw_space sp{k, chunk, seed, 0, delta};
    int rc = check_space(c, t->n, &sp);
    if (rc) return rc;
    if (((uint64_t)20 << delta) > TCW_MAX_TRAIL_CAP) return fail(c, TCW_EINVAL, "delta too large for a trail cap");
    TunedCfg cfg;
    rc = autotune(c, t, k, chunk, delta, seed, &cfg);
    if (rc) return rc;
    *walks = cfg.walks;
    *iters = cfg.iters;
    *log2_table = cfg.log2_table;
    *steps_per_s = cfg.rate;
    return TCW_OK;
}

namespace {

tcw_walk_stats stats_of(const unsigned long long* st, unsigned long long claw_count, uint32_t claw_cap) {
    tcw_walk_stats ws{};
    ws.steps = (int64_t)st[tcw::ST_STEPS];
    ws.dps = (int64_t)st[tcw::ST_DPS];
    ws.inserts = (int64_t)st[tcw::ST_INSERTS];
    ws.abandoned = (int64_t)st[tcw::ST_ABANDONED];
    ws.robin_hood = (int64_t)st[tcw::ST_ROBIN];
    ws.same_side = (int64_t)st[tcw::ST_SAME];
    ws.reduction = (int64_t)st[tcw::ST_REDUCTION];
    ws.claws = (int64_t)st[tcw::ST_CLAWS];
    ws.table_full = (int64_t)st[tcw::ST_FULL];
    ws.spin_timeouts = (int64_t)st[tcw::ST_SPIN];
    ws.claws_dropped = claw_count > claw_cap ? (int64_t)(claw_count - claw_cap) : 0;
    return ws;
}

void set_minimal(tcw_result* r) {
    if (r->status != TCW_STATUS_FOUND) {
        r->minimal = 0;
        return;
    }
    const uint64_t below = r->t >= 64 ? ~0ull : ((1ull << r->t) - 1);
    r->minimal = (r->failed_depths & below) == below ? 1 : 0;
}

// Runs every member search of bt (each with its own depth order, chunk range, walks and table) in
// rounds until all are done, or, with stop_on_first, until one member holds a verified decomposition,
// or until `stop` is due (members still running then end with TCW_STATUS_STOPPED).  A round is one
// replay of a graph captured once: a kernel zeroes the queue positions, then one persistent queue
// kernel per qubit count takes (member, slice of walks) items until its queue is empty.  Between
// rounds the host refreshes the queues and the members' descriptors; claw candidates read after a
// round are checked exactly while the next round runs.  *agg: walk steps per second of round time.
int batch_run(tcw_ctx* c, std::vector<BatchTarget>& bt, bool stop_on_first, double t0, double* agg, StopCtl* stop) {
    const int count = (int)bt.size();
    BatchBuffers bb;
    HIP_TRY(c, hipMalloc(&bb.stats, (size_t)count * tcw::ST_COUNT * 8));
    HIP_TRY(c, hipMalloc(&bb.claw_count, (size_t)count * 8));
    HIP_TRY(c, hipMalloc(&bb.claws, (size_t)count * BATCH_CLAW_CAP * 16));
    HIP_TRY(c, hipMalloc(&bb.sps, (size_t)count * sizeof(tcw::SpaceDev)));
    HIP_TRY(c, hipMalloc(&bb.wds, (size_t)count * sizeof(tcw::WalkDev)));
    HIP_TRY(c, hipMalloc(&bb.counts, 5 * 4));
    HIP_TRY(c, hipMalloc(&bb.heads, 5 * 4));
    HIP_TRY(c, hipMalloc(&bb.restart, (size_t)count * 4));
    HIP_TRY(c, hipMemsetAsync(bb.stats, 0, (size_t)count * tcw::ST_COUNT * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(bb.claw_count, 0, (size_t)count * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(bb.counts, 0, 5 * 4, c->stream));
    // claw-check buffers sized once, so the checks that run beside a round allocate nothing
    int nmax = 1;
    bool has_n[5] = {false, false, false, false, false};
    for (auto& b : bt) {
        nmax = std::max(nmax, b.t->n);
        has_n[b.t->n] = true;
    }
    ClawWs cws;
    HIP_TRY(c, cws.reserve(BATCH_CLAW_CAP, 1 << (2 * nmax)));
    if (int e = ensure_claw_scratch(c, nmax)) return e;
    int rc = TCW_OK;
    for (int i = 0; i < count && !rc; ++i) {
        rc = batch_advance(c, bt[i], i, bb, t0, false);
        if (bt[i].done) bt[i].res->seconds = now_s() - t0;
    }
    if (rc) {
        (void)hipStreamSynchronize(c->stream);
        for (auto& b : bt) free_walk_buffers(c, b);
        return rc;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));

    // streams for the graph: one branch per qubit count (default priority)
    hipStream_t gs[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    auto cleanup = [&]() {
        // nothing may still use the members' buffers when they go back to the pool
        if (gs[0]) (void)hipStreamSynchronize(gs[0]);
        (void)hipStreamSynchronize(c->stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (int n = 0; n <= 4; ++n) {
            if (gs[n]) (void)hipStreamDestroy(gs[n]);
            if (join[n]) (void)hipEventDestroy(join[n]);
        }
        if (fork) (void)hipEventDestroy(fork);
        for (auto& b : bt) free_walk_buffers(c, b);
    };
#define BATCH_TRY(expr)                      \
    do {                                     \
        hipError_t _e = (expr);              \
        if (_e != hipSuccess) {              \
            cleanup();                       \
            return hip_fail(c, _e, #expr);   \
        }                                    \
    } while (0)
#define BATCH_RC(expr)     \
    do {                   \
        rc = (expr);       \
        if (rc) {          \
            cleanup();     \
            return rc;     \
        }                  \
    } while (0)
    BATCH_TRY(hipStreamCreateWithFlags(&gs[0], hipStreamNonBlocking));
    for (int n = 1; n <= 4; ++n) {
        BATCH_TRY(hipStreamCreateWithFlags(&gs[n], hipStreamNonBlocking));
        BATCH_TRY(hipEventCreateWithFlags(&join[n], hipEventDisableTiming));
    }
    BATCH_TRY(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    int grid[5] = {0, 0, 0, 0, 0};
    for (int n = 1; n <= 4; ++n) grid[n] = has_n[n] ? tcw::walk_grid_blocks(n, c->device, true, 0) : 0;
    bool dirty = true, recapture = true;
    int64_t total_steps = 0;
    double walk_seconds = 0;
    std::vector<unsigned long long> stats((size_t)count * tcw::ST_COUNT), ccount(count);
    std::vector<tcw::SpaceDev> h_sps(count);
    std::vector<tcw::WalkDev> h_wds(count);
    std::vector<tcw::WorkItem> h_items[5];
    int32_t h_counts[5] = {0, 0, 0, 0, 0};
    std::vector<char> queued(count, 0), hit(count, 0);
    bool stop_first = false;

    // the member's space ended (budget, version, time) or a check found a decomposition: act on it
    auto settle = [&](int i, bool found) -> int {
        BatchTarget& b = bt[i];
        const tcw_walk_stats ws = stats_of(&stats[(size_t)i * tcw::ST_COUNT], ccount[i], b.wd.claw_cap);
        const bool over_time = b.p.max_seconds > 0 && now_s() - t0 > b.p.max_seconds;
        if (found || over_time || b.used >= b.budget) {
            add_stats(b.res->stats, ws);
            b.walking = false;
            b.held = false;
            dirty = true;
            if (found) batch_on_hit(b);
            if (over_time && !b.done) {
                b.done = true;
                b.cut = true;
            }
            if (b.done) {
                b.res->seconds = now_s() - t0;
                free_walk_buffers(c, b);
            } else {
                int e = batch_advance(c, b, i, bb, t0, !found);
                if (e) return e;
                if (b.done) b.res->seconds = now_s() - t0;
            }
        } else if (b.used_v >= b.per_version) {
            add_stats(b.res->stats, ws);
            b.version++;
            b.res->versions++;
            b.space->set_version(b.version);
            b.used_v = 0;
            b.seen = 0;
            b.held = false;
            dirty = true;
            batch_restart(bb, i);
        }
        return TCW_OK;
    };

    for (;;) {
        bool any = false;
        for (auto& b : bt) any |= b.walking || !b.pu0.empty();
        if (!any) break;
        if (stop && stop->due()) {
            stop->stopped = true;
            break;
        }
        if (dirty) {
            // the queues: every walking member that is not held, in slices of its walks.  A qubit count's
            // queue holds about four items per block of its grid, shared out by walks, so an item spans
            // many walks per wavefront: the block's wavefronts meet at a barrier and reload the member's
            // LDS state only between items (one walk per wavefront per item ran four times slower)
            for (int n = 1; n <= 4; ++n) h_items[n].clear();
            int64_t walks_n[5] = {0, 0, 0, 0, 0};
            for (int i = 0; i < count; ++i) {
                BatchTarget& b = bt[i];
                queued[i] = b.walking && !b.held;
                if (queued[i]) walks_n[b.t->n] += b.walks;
            }
            for (int i = 0; i < count; ++i) {
                BatchTarget& b = bt[i];
                if (!queued[i]) continue;
                const int n = b.t->n;
                const int wpb = tcw::walks_per_block(n);
                const double share = 4.0 * grid[n] * (double)b.walks / (double)walks_n[n];
                const int64_t most = (b.walks + wpb - 1) / wpb;
                const int32_t units = (int32_t)std::max<int64_t>(1, std::min<int64_t>(most, std::llround(share)));
                for (int32_t u = 0; u < units; ++u) h_items[n].push_back(tcw::WorkItem{i, u, units, b.iters});
            }
            for (int n = 1; n <= 4; ++n) {
                const int64_t m = (int64_t)h_items[n].size();
                h_counts[n] = (int32_t)m;
                if (m > bb.items_cap[n]) {
                    // a larger queue buffer: its address is a kernel argument, so the graph is captured again
                    const int64_t cap = std::max<int64_t>(m, 2 * bb.items_cap[n]);
                    if (bb.items[n]) (void)hipFree(bb.items[n]);
                    bb.items[n] = nullptr;
                    bb.items_cap[n] = 0;
                    BATCH_TRY(hipMalloc(&bb.items[n], (size_t)cap * sizeof(tcw::WorkItem)));
                    bb.items_cap[n] = cap;
                    recapture = true;
                }
                if (m > 0)
                    BATCH_TRY(hipMemcpy(bb.items[n], h_items[n].data(), (size_t)m * sizeof(tcw::WorkItem),
                                        hipMemcpyHostToDevice));
            }
            BATCH_TRY(hipMemcpy(bb.counts, h_counts, 5 * 4, hipMemcpyHostToDevice));
            dirty = false;
        }
        if (recapture) {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            exec = nullptr;
            graph = nullptr;
            // capture: zero the queue positions (a kernel, not a memset node), fork one branch per qubit
            // count present in the batch, join
            BATCH_TRY(hipStreamBeginCapture(gs[0], hipStreamCaptureModeThreadLocal));
            BATCH_TRY(tcw::fill_i32(bb.heads, 0, 5, gs[0]));
            BATCH_TRY(hipEventRecord(fork, gs[0]));
            for (int n = 1; n <= 4; ++n) {
                if (!grid[n] || !bb.items[n]) continue;
                BATCH_TRY(hipStreamWaitEvent(gs[n], fork, 0));
                BATCH_TRY(tcw::launch_walk_queue(n, bb.sps, bb.wds, bb.items[n], bb.counts + n,
                                                 reinterpret_cast<uint32_t*>(bb.heads + n), grid[n], gs[n]));
                BATCH_TRY(hipEventRecord(join[n], gs[n]));
                BATCH_TRY(hipStreamWaitEvent(gs[0], join[n], 0));
            }
            BATCH_TRY(hipStreamEndCapture(gs[0], &graph));
            BATCH_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            recapture = false;
        }
        bool round = false;
        for (int i = 0; i < count; ++i) {
            if (!queued[i]) continue;
            round = true;
            h_sps[i] = bt[i].space->dev;
            h_wds[i] = bt[i].wd;
        }
        for (const int32_t i : bb.pending) {
            h_sps[i] = bt[i].space->dev;
            h_wds[i] = bt[i].wd;
        }
        const double tl = now_s();
        if (round || !bb.pending.empty()) {
            // descriptors for this replay (salts change with versions), the restarts of members that
            // begin a space or a version, then the round itself
            BATCH_TRY(hipMemcpyAsync(bb.sps, h_sps.data(), count * sizeof(tcw::SpaceDev), hipMemcpyHostToDevice,
                                     gs[0]));
            BATCH_TRY(hipMemcpyAsync(bb.wds, h_wds.data(), count * sizeof(tcw::WalkDev), hipMemcpyHostToDevice,
                                     gs[0]));
            if (!bb.pending.empty()) {
                BATCH_TRY(hipMemcpyAsync(bb.restart, bb.pending.data(), bb.pending.size() * 4, hipMemcpyHostToDevice,
                                         gs[0]));
                BATCH_TRY(tcw::launch_member_restart(bb.sps, bb.wds, bb.restart, (int)bb.pending.size(), gs[0]));
                BATCH_TRY(hipStreamSynchronize(gs[0]));  // the host may refill the list before the copy ran
                bb.pending.clear();
            }
            if (round) BATCH_TRY(hipGraphLaunch(exec, gs[0]));
        }
        // the last round's claw candidates, checked exactly while this round runs
        for (int i = 0; i < count; ++i) {
            BatchTarget& b = bt[i];
            hit[i] = 0;
            if (b.pu0.empty()) continue;
            int found = 0;
            BATCH_RC(check_pairs_ws(c, *b.space, b.pu0.data(), b.pu1.data(), (int64_t)b.pu0.size(), b.res, &found,
                                    cws));
            b.pu0.clear();
            b.pu1.clear();
            hit[i] = (char)found;
        }
        if (round) {
            BATCH_TRY(hipMemcpyAsync(stats.data(), bb.stats, stats.size() * 8, hipMemcpyDeviceToHost, gs[0]));
            BATCH_TRY(hipStreamSynchronize(gs[0]));
            walk_seconds += now_s() - tl;
            if (stop && stop->launches) (*stop->launches)++;
            // enumerated members whose last point is done: read out their candidates
            bool formed = false;
            for (int i = 0; i < count; ++i) {
                BatchTarget& b = bt[i];
                if (!queued[i] || !b.wd.enumerate) continue;
                if (stats[(size_t)i * tcw::ST_COUNT + tcw::ST_STEPS] >= b.budget) {
                    BATCH_TRY(tcw::launch_enum_pairs(b.wd, gs[0]));
                    formed = true;
                }
            }
            if (formed)
                BATCH_TRY(hipMemcpyAsync(stats.data(), bb.stats, stats.size() * 8, hipMemcpyDeviceToHost, gs[0]));
            BATCH_TRY(hipMemcpyAsync(ccount.data(), bb.claw_count, count * 8, hipMemcpyDeviceToHost, gs[0]));
            BATCH_TRY(hipStreamSynchronize(gs[0]));
        }
        for (int i = 0; i < count; ++i) {
            BatchTarget& b = bt[i];
            if (!b.walking) continue;
            if (queued[i]) {
                b.res->launches++;
                const uint64_t steps_now = stats[(size_t)i * tcw::ST_COUNT + tcw::ST_STEPS];
                total_steps += (int64_t)(steps_now - b.used_v);
                b.used += steps_now - b.used_v;
                b.used_v = steps_now;
            }
            if (hit[i]) {
                BATCH_RC(settle(i, true));
            } else {
                if (queued[i]) {
                    // new candidates of this round: checked during the next round
                    const int64_t avail = (int64_t)std::min<unsigned long long>(ccount[i], BATCH_CLAW_CAP);
                    if (avail > b.seen) {
                        const int64_t m = avail - b.seen;
                        std::vector<uint64_t> pairs(2 * m);
                        BATCH_TRY(hipMemcpy(pairs.data(), b.wd.claws + 2 * b.seen, 16 * m, hipMemcpyDeviceToHost));
                        b.pu0.resize(m);
                        b.pu1.resize(m);
                        for (int64_t j = 0; j < m; ++j) {
                            b.pu0[j] = pairs[2 * j];
                            b.pu1[j] = pairs[2 * j + 1];
                        }
                        if (b.wd.enumerate) sort_pairs(b.pu0.data(), b.pu1.data(), m);
                        b.seen = avail;
                    }
                }
                const bool over_time = b.p.max_seconds > 0 && now_s() - t0 > b.p.max_seconds;
                const bool ends = over_time || b.used >= b.budget || b.used_v >= b.per_version;
                if (ends && !b.pu0.empty() && !over_time) {
                    // the space ends, but its last candidates are not checked yet: sit out until they are
                    if (!b.held) {
                        b.held = true;
                        dirty = true;
                    }
                } else if (ends) {
                    if (!b.pu0.empty()) {
                        // out of time: check what is pending now rather than lose it
                        int found = 0;
                        BATCH_RC(check_pairs_ws(c, *b.space, b.pu0.data(), b.pu1.data(), (int64_t)b.pu0.size(), b.res,
                                                &found, cws));
                        b.pu0.clear();
                        b.pu1.clear();
                        hit[i] = (char)found;
                    }
                    BATCH_RC(settle(i, hit[i] != 0));
                }
            }
            if (stop_on_first && b.res->status == TCW_STATUS_FOUND && b.done) stop_first = true;
        }
        BATCH_TRY(hipStreamSynchronize(gs[0]));
        if (stop_first) break;
    }
    if (stop_first || (stop && stop->stopped)) {
        // end the members still running with their counts so far
        for (int i = 0; i < count; ++i) {
            BatchTarget& b = bt[i];
            if (!b.walking) continue;
            add_stats(b.res->stats, stats_of(&stats[(size_t)i * tcw::ST_COUNT], ccount[i], b.wd.claw_cap));
            b.walking = false;
            b.held = false;
            b.pu0.clear();
            b.pu1.clear();
            b.done = true;
            b.res->seconds = now_s() - t0;
            if (stop && stop->stopped) b.res->status = TCW_STATUS_STOPPED;
        }
    }
#undef BATCH_TRY
#undef BATCH_RC
    cleanup();
    for (auto& b : bt) {
        if (b.res->seconds == 0) b.res->seconds = now_s() - t0;
        set_minimal(b.res);
    }
    if (agg) *agg = walk_seconds > 0 ? (double)total_steps / walk_seconds : 0.0;
    return TCW_OK;
}

}  // namespace

namespace {

int search_chunks_concurrent(tcw_ctx* c, const tcw_target* t, const tcw_walk_params* p, int k, int c_first,
                             int c_last, int delta, tcw_result* res, int* found, bool* cut, StopCtl* stop, double t0) {
    const int n = t->n;
    const int G = c_last - c_first + 1;
    int lg_g = 0;
    while ((1 << lg_g) < G) ++lg_g;
    const int64_t walks_c = std::max<int64_t>(64, p->walks / G);
    const int log2_c = std::max(10, std::min(p->log2_table, CHUNK_TABLE_POOL_LOG2 - 4 - lg_g));
    const int iters = p->iters_per_launch > 0 ? p->iters_per_launch : default_iters(n);
    std::vector<BatchTarget> bt(G);
    std::vector<tcw_result> rs(G);
    for (int i = 0; i < G; ++i) {
        BatchTarget& b = bt[i];
        b.t = t;
        b.p = *p;
        b.p.walks = walks_c;
        b.p.log2_table = log2_c;
        b.p.iters_per_launch = iters;
        b.p.delta = delta;
        b.p.depth_order_kind = TCW_ORDER_PLAIN;
        b.p.chunk_first = b.p.chunk_last = c_first + i;
        b.order.assign(1, k);
        std::memset(&rs[i], 0, sizeof(tcw_result));
        rs[i].n = n;
        b.res = &rs[i];
    }
    const int rc = batch_run(c, bt, true, t0, nullptr, stop);
    if (rc) return rc;
    int64_t launches = 0;
    for (int i = 0; i < G; ++i) {
        const tcw_result& r = rs[i];
        add_stats(res->stats, r.stats);
        res->spaces += r.spaces;
        res->versions += r.versions;
        res->false_claws += r.false_claws;
        launches = std::max(launches, r.launches);
        *cut = *cut || bt[i].cut;
        if (r.status == TCW_STATUS_FOUND && !*found) {
            *found = 1;
            res->status = TCW_STATUS_FOUND;
            res->t = r.t;
            res->chunk = r.chunk;
            std::memcpy(res->paulis, r.paulis, sizeof(res->paulis));
            std::memcpy(res->clifford_perm, r.clifford_perm, sizeof(res->clifford_perm));
            std::memcpy(res->clifford_sign, r.clifford_sign, sizeof(res->clifford_sign));
        }
    }
    res->launches += launches;
    return TCW_OK;
}

}  // namespace

extern "C" int tcw_search_batch(tcw_ctx* c, const tcw_target* const* targets, int count, const tcw_walk_params* params,
                                tcw_result* results, double* aggregate_steps_per_s) {
    if (!c || !targets || !params || !results || count < 1) return TCW_EINVAL;
    for (int i = 0; i < count; ++i)
        if (!targets[i]) return fail(c, TCW_EINVAL, "NULL target in batch");
    const double t0 = now_s();
    std::vector<BatchTarget> bt(count);
    int rc = TCW_OK;
    for (int i = 0; i < count && !rc; ++i) {
        BatchTarget& b = bt[i];
        b.t = targets[i];
        b.p = params[i];
        b.res = &results[i];
        std::memset(b.res, 0, sizeof(tcw_result));
        b.res->n = b.t->n;
        rc = check_params(c, &b.p, b.t->n, true);
        if (!rc) rc = depth_order_of(c, &b.p, b.order);
    }
    if (rc) return rc;
    StopCtl stop;
    stop.flag = &c->stop_req;
    rc = batch_run(c, bt, false, t0, aggregate_steps_per_s, &stop);
    if (stop.stopped) c->stop_req.store(0);
    return rc;
}

// ---------------------------------------------------------------------------------------------
// Depth-order network: canonical features, exact labels by meet in the middle, BF16 MFMA training.
struct tcw_mlp {
    tcw_ctx* ctx = nullptr;
    int inp = 0, hidden = 0, depth = 0, classes = 0, L = 0;
    std::vector<int> sz;
    std::vector<int64_t> w_off, b_off;
    int64_t count = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
    std::vector<void*> Wb, Wt;  // bf16 weights: W_l (in x out) and W_l^T (out x in)
    int step = 0;
    int cap_b = 0;
    void *Xb = nullptr, *Xt = nullptr;
    std::vector<float*> Z, Gf;
    std::vector<void*> Hb, Ht, Gb, Gt;
    float *logits = nullptr, *probs = nullptr, *loss = nullptr, *xdev = nullptr;
    float* part = nullptr;  // partial products of the GEMMs whose K is split over workgroups
    size_t part_floats = 0;

    void free_batch() {
        for (void* q : {Xb, Xt, (void*)logits, (void*)probs, (void*)part})
            if (q) (void)hipFree(q);
        Xb = Xt = nullptr;
        part = nullptr;
        part_floats = 0;
        for (auto* v : {&Hb, &Ht, &Gb, &Gt}) {
            for (void* q : *v)
                if (q) (void)hipFree(q);
            v->clear();
        }
        for (auto* v : {&Z, &Gf}) {
            for (float* q : *v)
                if (q) (void)hipFree(q);
            v->clear();
        }
        logits = probs = nullptr;
        cap_b = 0;
    }
    ~tcw_mlp() {
        free_batch();
        for (void* q : {(void*)P, (void*)G, (void*)M, (void*)V, (void*)loss, (void*)xdev})
            if (q) (void)hipFree(q);
        for (auto* v : {&Wb, &Wt})
            for (void* q : *v)
                if (q) (void)hipFree(q);
    }
};

namespace {

// leading dimension of a bf16 buffer: a multiple of 8 elements, so every row starts 16-byte aligned
int ld8(int cols) { return (cols + 7) / 8 * 8; }

int mlp_ensure_batch(tcw_mlp* m, int b) {
    tcw_ctx* c = m->ctx;
    if (b <= m->cap_b) return TCW_OK;
    m->free_batch();
    const size_t b8 = (size_t)ld8(b);
    HIP_TRY(c, hipMalloc(&m->Xb, (size_t)b * ld8(m->inp) * 2));
    HIP_TRY(c, hipMalloc(&m->Xt, (size_t)m->inp * b8 * 2));
    m->Z.assign(m->depth, nullptr);
    m->Hb.assign(m->depth, nullptr);
    m->Ht.assign(m->depth, nullptr);
    m->Gf.assign(m->L, nullptr);
    m->Gb.assign(m->L, nullptr);
    m->Gt.assign(m->L, nullptr);
    for (int l = 0; l < m->depth; ++l) {
        HIP_TRY(c, hipMalloc(&m->Z[l], (size_t)b * m->hidden * 4));
        HIP_TRY(c, hipMalloc(&m->Hb[l], (size_t)b * ld8(m->hidden) * 2));
        HIP_TRY(c, hipMalloc(&m->Ht[l], (size_t)m->hidden * b8 * 2));
    }
    for (int l = 0; l < m->L; ++l) {
        const int out = m->sz[l + 1];
        HIP_TRY(c, hipMalloc(&m->Gf[l], (size_t)b * out * 4));
        HIP_TRY(c, hipMalloc(&m->Gb[l], (size_t)b * ld8(out) * 2));
        HIP_TRY(c, hipMalloc(&m->Gt[l], (size_t)out * b8 * 2));
    }
    HIP_TRY(c, hipMalloc(&m->logits, (size_t)b * m->classes * 4));
    HIP_TRY(c, hipMalloc(&m->probs, (size_t)b * m->classes * 4));
    // workspace of the split products (forward b x out, K = in; dX b x in, K = out; dW in x out, K = b) and
    // of the bias gradients' column sums
    size_t part = 0;
    for (int l = 0; l < m->L; ++l) {
        const int in = m->sz[l], out = m->sz[l + 1];
        part = std::max({part, tcw::mlp_gemm_part_floats(b, out, in), tcw::mlp_gemm_part_floats(b, in, out),
                         tcw::mlp_gemm_part_floats(in, out, b), tcw::mlp_colsum_part_floats(b, out)});
    }
    if (part > 0) {
        HIP_TRY(c, hipMalloc(&m->part, part * 4));
        m->part_floats = part;
    }
    m->cap_b = b;
    return TCW_OK;
}

// bf16 copies of the weights in both orientations, from the FP32 masters
int mlp_sync_bf16(tcw_mlp* m) {
    for (int l = 0; l < m->L; ++l)
        HIP_TRY(m->ctx, tcw::mlp_weights_bf16(m->P + m->w_off[l], m->sz[l], m->sz[l + 1], m->Wb[l], ld8(m->sz[l + 1]),
                                              m->Wt[l], ld8(m->sz[l]), m->ctx->stream));
    return TCW_OK;
}

// forward over a batch; with labels (training) also the transposed activations, the loss sum and the
// output-layer gradient
int mlp_forward(tcw_mlp* m, const float* x, int b, const int32_t* labels) {
    tcw_ctx* c = m->ctx;
    int rc = mlp_ensure_batch(m, b);
    if (rc) return rc;
    const bool train = labels != nullptr;
    const int b8 = ld8(b);
    HIP_TRY(c, tcw::mlp_input_bf16(x, b, m->inp, m->Xb, ld8(m->inp), train ? m->Xt : nullptr, b8, c->stream));
    for (int l = 0; l < m->L; ++l) {
        const void* A = l == 0 ? m->Xb : m->Hb[l - 1];
        const int K = m->sz[l], N = m->sz[l + 1];
        if (l < m->L - 1) {
            HIP_TRY(c, tcw::mlp_gemm_nt(2, A, ld8(K), m->Wt[l], ld8(K), b, N, K, m->Z[l], N, m->P + m->b_off[l], nullptr,
                                        0, m->Hb[l], ld8(N), train ? m->Ht[l] : nullptr, b8, m->part, m->part_floats,
                                        c->stream));
        } else {
            HIP_TRY(c, tcw::mlp_gemm_nt(1, A, ld8(K), m->Wt[l], ld8(K), b, N, K, m->logits, N, m->P + m->b_off[l],
                                        nullptr, 0, nullptr, 0, nullptr, 0, m->part, m->part_floats, c->stream));
        }
    }
    if (train) HIP_TRY(c, hipMemsetAsync(m->loss, 0, 4, c->stream));
    const int lo = m->L - 1;
    HIP_TRY(c, tcw::mlp_softmax_ce(m->logits, labels, b, m->classes, m->probs, train ? m->Gf[lo] : nullptr,
                                   train ? m->Gb[lo] : nullptr, ld8(m->classes), train ? m->Gt[lo] : nullptr, b8,
                                   train ? m->loss : nullptr, c->stream));
    return TCW_OK;
}

int mlp_backward(tcw_mlp* m, int b) {
    tcw_ctx* c = m->ctx;
    const int b8 = ld8(b);
    for (int l = m->L - 1; l >= 0; --l) {
        const void* Hin_t = l == 0 ? m->Xt : m->Ht[l - 1];
        const int in = m->sz[l], out = m->sz[l + 1];
        // dW_l = H_in^T G_l: rows of H_in^T and of G_l^T run over the batch
        HIP_TRY(c, tcw::mlp_gemm_nt(0, Hin_t, b8, m->Gt[l], b8, in, out, b, m->G + m->w_off[l], out, nullptr, nullptr,
                                    0, nullptr, 0, nullptr, 0, m->part, m->part_floats, c->stream));
        HIP_TRY(c, tcw::mlp_colsum(m->Gf[l], b, out, m->G + m->b_off[l], m->part, m->part_floats, c->stream));
        if (l > 0) {
            // G_{l-1} = (G_l W_l^T) * gelu'(Z_{l-1}): B = W_l (in x out), rows over out
            HIP_TRY(c, tcw::mlp_gemm_nt(3, m->Gb[l], ld8(out), m->Wb[l], ld8(out), b, in, out, m->Gf[l - 1], in,
                                        nullptr, m->Z[l - 1], in, m->Gb[l - 1], ld8(in), m->Gt[l - 1], b8, m->part,
                                        m->part_floats, c->stream));
        }
    }
    return TCW_OK;
}

}  // namespace

extern "C" int tcw_mlp_create(tcw_ctx* c, int inp, int hidden, int depth, int classes, const float* init, uint64_t seed,
                              tcw_mlp** out) {
    if (!c || !out || inp < 1 || hidden < 1 || depth < 0 || depth > 16 || classes < 2) return TCW_EINVAL;
    *out = nullptr;
    tcw_mlp* m = new (std::nothrow) tcw_mlp();
    if (!m) return TCW_ENOMEM;
    m->ctx = c;
    m->inp = inp;
    m->hidden = hidden;
    m->depth = depth;
    m->classes = classes;
    m->L = depth + 1;
    m->sz.push_back(inp);
    for (int l = 0; l < depth; ++l) m->sz.push_back(hidden);
    m->sz.push_back(classes);
    int64_t off = 0;
    for (int l = 0; l < m->L; ++l) {
        m->w_off.push_back(off);
        off += (int64_t)m->sz[l] * m->sz[l + 1];
        m->b_off.push_back(off);
        off += m->sz[l + 1];
    }
    m->count = off;
    auto bail = [&](hipError_t e) {
        delete m;
        return hip_fail(c, e, "network allocation");
    };
    hipError_t e = hipMalloc(&m->P, off * 4);
    if (e == hipSuccess) e = hipMalloc(&m->G, off * 4);
    if (e == hipSuccess) e = hipMalloc(&m->M, off * 4);
    if (e == hipSuccess) e = hipMalloc(&m->V, off * 4);
    if (e == hipSuccess) e = hipMalloc(&m->loss, 4);
    if (e != hipSuccess) return bail(e);
    m->Wb.assign(m->L, nullptr);
    m->Wt.assign(m->L, nullptr);
    for (int l = 0; l < m->L && e == hipSuccess; ++l) {
        e = hipMalloc(&m->Wb[l], (size_t)m->sz[l] * ld8(m->sz[l + 1]) * 2);
        if (e == hipSuccess) e = hipMalloc(&m->Wt[l], (size_t)m->sz[l + 1] * ld8(m->sz[l]) * 2);
    }
    if (e == hipSuccess) e = hipMemsetAsync(m->M, 0, off * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->V, 0, off * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->P, 0, off * 4, c->stream);
    if (e != hipSuccess) return bail(e);
    if (init) {
        e = hipMemcpyAsync(m->P, init, off * 4, hipMemcpyHostToDevice, c->stream);
    } else {
        int64_t idx = 0;
        for (int l = 0; l < m->L && e == hipSuccess; ++l) {
            const int64_t cnt = (int64_t)m->sz[l] * m->sz[l + 1];
            e = tcw::mlp_init(m->P + m->w_off[l], cnt, idx, m->sz[l], seed, c->stream);
            idx += cnt;
        }
    }
    if (e != hipSuccess) return bail(e);
    int rc = mlp_sync_bf16(m);
    if (!rc) {
        hipError_t se = hipStreamSynchronize(c->stream);
        if (se != hipSuccess) rc = hip_fail(c, se, "network init");
    }
    if (rc) {
        delete m;
        return rc;
    }
    *out = m;
    return TCW_OK;
}

extern "C" int tcw_mlp_free(tcw_mlp* m) {
    if (!m) return TCW_EINVAL;
    (void)hipStreamSynchronize(m->ctx->stream);
    delete m;
    return TCW_OK;
}

extern "C" int tcw_mlp_param_count(const tcw_mlp* m, int64_t* count) {
    if (!m || !count) return TCW_EINVAL;
    *count = m->count;
    return TCW_OK;
}

extern "C" int tcw_mlp_get_params(tcw_mlp* m, float* host) {
    if (!m || !host) return TCW_EINVAL;
    HIP_TRY(m->ctx, hipMemcpyAsync(host, m->P, m->count * 4, hipMemcpyDeviceToHost, m->ctx->stream));
    HIP_TRY(m->ctx, hipStreamSynchronize(m->ctx->stream));
    return TCW_OK;
}

extern "C" int tcw_mlp_set_params(tcw_mlp* m, const float* host) {
    if (!m || !host) return TCW_EINVAL;
    HIP_TRY(m->ctx, hipMemcpyAsync(m->P, host, m->count * 4, hipMemcpyHostToDevice, m->ctx->stream));
    int rc = mlp_sync_bf16(m);
    if (rc) return rc;
    HIP_TRY(m->ctx, hipStreamSynchronize(m->ctx->stream));
    return TCW_OK;
}

extern "C" int tcw_mlp_forward(tcw_mlp* m, const float* x, int batch, float* probs) {
    if (!m || !x || !probs || batch < 1) return TCW_EINVAL;
    int rc = mlp_forward(m, x, batch, nullptr);
    if (rc) return rc;
    HIP_TRY(m->ctx, hipMemcpyAsync(probs, m->probs, (size_t)batch * m->classes * 4, hipMemcpyDeviceToDevice,
                                   m->ctx->stream));
    HIP_TRY(m->ctx, hipStreamSynchronize(m->ctx->stream));
    return TCW_OK;
}

extern "C" int tcw_mlp_gradients(tcw_mlp* m, const float* x, const int32_t* labels, int batch, float* grads_host,
                                 float* loss) {
    if (!m || !x || !labels || batch < 1) return TCW_EINVAL;
    int rc = mlp_forward(m, x, batch, labels);
    if (!rc) rc = mlp_backward(m, batch);
    if (rc) return rc;
    float ls = 0;
    HIP_TRY(m->ctx, hipMemcpyAsync(&ls, m->loss, 4, hipMemcpyDeviceToHost, m->ctx->stream));
    if (grads_host) HIP_TRY(m->ctx, hipMemcpyAsync(grads_host, m->G, m->count * 4, hipMemcpyDeviceToHost, m->ctx->stream));
    HIP_TRY(m->ctx, hipStreamSynchronize(m->ctx->stream));
    if (loss) *loss = ls / (float)batch;
    return TCW_OK;
}

extern "C" int tcw_mlp_train_step(tcw_mlp* m, const float* x, const int32_t* labels, int batch, float lr, float* loss) {
    if (!m || !x || !labels || batch < 1 || !(lr > 0)) return TCW_EINVAL;
    int rc = mlp_forward(m, x, batch, labels);
    if (!rc) rc = mlp_backward(m, batch);
    if (rc) return rc;
    m->step++;
    HIP_TRY(m->ctx, tcw::mlp_adam(m->P, m->G, m->M, m->V, m->count, lr, 0.9f, 0.999f, 1e-8f, m->step, m->ctx->stream));
    rc = mlp_sync_bf16(m);
    if (rc) return rc;
    if (loss) {
        float ls = 0;
        HIP_TRY(m->ctx, hipMemcpyAsync(&ls, m->loss, 4, hipMemcpyDeviceToHost, m->ctx->stream));
        HIP_TRY(m->ctx, hipStreamSynchronize(m->ctx->stream));
        *loss = ls / (float)batch;
    }
    return TCW_OK;
}

extern "C" int tcw_features(tcw_ctx* c, const tcw_target* t, float* out_dev) {
    if (!c || !t || !out_dev) return TCW_EINVAL;
    if (t->n > 3) return fail(c, TCW_EINVAL, "features are defined for n <= 3");
    HIP_TRY(c, tcw::exact_features(t->U, out_dev, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TCW_OK;
}

namespace {

// Steps that depth k costs under p when it holds no decomposition of an n-qubit target (eq:runtime
// and the appendix law give the walks' cost of a space as its budget beta N / theta): every chunk
// runs its whole space, one step per point when enumerated, else its walk budget, with theta
// resolved as the driver resolves an open delta (concurrent chunks against their share of the chunk
// table pool); plus 2^20 steps per depth for set-up, launches and read-backs.  Infinite for a
// depth whose spaces are beyond 32-bit points.
double depth_cost_steps(int n, const tcw_walk_params* p, int k) {
    const double fixed = 1048576.0;
    if (k == 0) return fixed;
    const uint64_t nh = n_half_of(n, k / 2);
    if (nh == 0) return HUGE_VAL;
    const uint64_t npts = 2 * nh;
    double chunks = 1;
    if (k % 2) {
        const int cf = p->chunk_first > 0 ? p->chunk_first : 1;
        const int cl = p->chunk_last > 0 ? std::min<int>(p->chunk_last, (int)xi_of(n)) : (int)xi_of(n);
        chunks = cl >= cf ? cl - cf + 1 : 0;
    }
    if ((int64_t)npts <= p->enum_max) return fixed + chunks * (double)npts;
    int lg = p->log2_table > 0 ? p->log2_table : default_log2_table(n);
    if (k % 2 && p->chunk_parallel != 1) {
        const int G = p->chunk_parallel <= 0 ? (int)chunks : p->chunk_parallel;
        int lg_g = 0;
        while ((1 << lg_g) < G) ++lg_g;
        lg = std::max(10, std::min(lg, CHUNK_TABLE_POOL_LOG2 - 4 - lg_g));
    }
    const int delta = p->delta >= 0 ? p->delta : auto_delta(npts, lg);
    return fixed + chunks * (double)p->budget_beta * (double)npts * std::ldexp(1.0, delta);
}

}  // namespace

extern "C" int tcw_depth_costs(tcw_ctx* c, const tcw_target* t, const tcw_walk_params* p, int k_max,
                               double* cost_out) {
    if (!c || !t || !p || !cost_out || k_max < 0 || k_max > 63) return TCW_EINVAL;
    if (int rc = check_params(c, p, t->n, true)) return rc;
    for (int k = 0; k <= k_max; ++k) cost_out[k] = depth_cost_steps(t->n, p, k);
    return TCW_OK;
}

extern "C" int tcw_mlp_depth_order(tcw_mlp* m, const tcw_target* t, int k_max, const tcw_walk_params* sp,
                                   int32_t* order_out, float* probs_out) {
    if (!m || !t || !order_out || k_max < 0 || k_max > 63) return TCW_EINVAL;
    tcw_ctx* c = m->ctx;
    if (sp)
        if (int rc = check_params(c, sp, t->n, true)) return rc;
    const int R = 1 << (2 * t->n);
    if (R * R != m->inp) return fail(c, TCW_EINVAL, "network input size does not match the target");
    if (!m->xdev) HIP_TRY(c, hipMalloc(&m->xdev, (size_t)m->inp * 4));
    int rc = tcw_features(c, t, m->xdev);
    if (!rc) rc = mlp_forward(m, m->xdev, 1, nullptr);
    if (rc) return rc;
    std::vector<float> p(m->classes);
    HIP_TRY(c, hipMemcpyAsync(p.data(), m->probs, m->classes * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (probs_out)
        for (int i = 0; i < m->classes; ++i) probs_out[i] = p[i];
    // depths 0..k_max by descending key (ties: smaller depth first); the key is the predicted
    // probability, or with search parameters the probability per step of the depth's cost
    std::vector<int> ks;
    std::vector<double> key(k_max + 1);
    for (int k = 0; k <= k_max; ++k) {
        ks.push_back(k);
        const double pk = k < m->classes ? (double)p[k] : 0.0;
        key[k] = sp ? pk / depth_cost_steps(t->n, sp, k) : pk;
    }
    std::stable_sort(ks.begin(), ks.end(), [&](int a, int b) { return key[a] > key[b]; });
    for (int i = 0; i <= k_max; ++i) order_out[i] = ks[i];
    return TCW_OK;
}

namespace {

// Hash table of every left-Clifford coset reached by <= h rotations from the identity, keyed by
// matrix hash, value 255 - (least number of rotations); shared by the labelling and certificate calls.
struct LevelTable {
    uint64_t* table = nullptr;
    uint64_t* keys = nullptr;
    uint32_t* zero_phi = nullptr;
    int lg = 0;
    tcw::SpaceDev sp{};
    ~LevelTable() {
        for (void* q : {(void*)table, (void*)keys, (void*)zero_phi})
            if (q) (void)hipFree(q);
    }
};

int build_level_table(tcw_ctx* c, int n, int h_levels, uint64_t seed, LevelTable& lt) {
    const int R = 1 << (2 * n);
    HIP_TRY(c, hipMalloc(&lt.zero_phi, (size_t)R * R / 2 * 4));
    HIP_TRY(c, hipMemsetAsync(lt.zero_phi, 0, (size_t)R * R / 2 * 4, c->stream));
    HIP_TRY(c, hipMalloc(&lt.keys, (size_t)R * 8));
    HIP_TRY(c, tcw::keys_fill(n, seed, lt.keys, c->stream));
    uint64_t entries = 0;
    for (int h = 0; h <= h_levels; ++h) entries += n_half_of(n, h);
    lt.lg = 10;
    while ((1ull << lt.lg) < 4 * entries && lt.lg < 30) ++lt.lg;
    HIP_TRY(c, hipMalloc(&lt.table, ((size_t)1 << lt.lg) * 16));
    HIP_TRY(c, tcw::launch_table_clear(lt.table, lt.lg, 0, c->stream));
    lt.sp.delta = 0;
    lt.sp.salt_h = tcw::sm64(tcw::sm64(seed, 2), 0x4C4142454Cull);
    lt.sp.keys = lt.keys;
    lt.sp.phi = lt.zero_phi;
    for (int h = 0; h <= h_levels; ++h) {
        lt.sp.h = h;
        lt.sp.n_half = (uint32_t)n_half_of(n, h);
        HIP_TRY(c, tcw::mitm_levels(n, lt.sp, h, lt.table, lt.lg, c->stream));
    }
    return TCW_OK;
}

uint64_t level_entries(int n, int h) {
    uint64_t e = 0;
    for (int i = 0; i <= h; ++i) e += n_half_of(n, i);
    return e;
}

// Identity-side depth h_id of the meet-in-the-middle split for `count` targets.  The table holds every
// coset reached by <= h_id rotations and each target probes its products with <= 2 h_max - h_id
// rotations, so any split finds every T-count up to 2 h_max.  The one chosen minimises the table's
// steps plus the targets' worst-case probe steps, with the table at most 2^25 entries (or the
// balanced split's size, if larger): one target keeps the balanced split, a large batch moves
// work into the table it builds once.
int mitm_split(int n, int h_max, int64_t count) {
    const uint64_t cap = std::max<uint64_t>(1ull << 25, level_entries(n, h_max));
    auto cost = [&](int h) {
        return (double)level_entries(n, h) + (double)count * (double)level_entries(n, 2 * h_max - h);
    };
    int best = h_max;
    for (int h = 0; h <= 2 * h_max; ++h) {
        if (n_half_of(n, h) == 0 || n_half_of(n, 2 * h_max - h) == 0 || level_entries(n, h) > cap) continue;
        if (cost(h) < cost(best)) best = h;
    }
    return best;
}

int check_mitm_args(tcw_ctx* c, int n, int h_max) {
    if (n < 1 || n > 3) return fail(c, TCW_EINVAL, "meet in the middle runs for n <= 3");
    if (h_max < 0 || n_half_of(n, h_max) == 0) return fail(c, TCW_EINVAL, "h_max too large");
    uint64_t entries = 0;
    for (int h = 0; h <= h_max; ++h) entries += n_half_of(n, h);
    if (entries > (1ull << 28)) return fail(c, TCW_EINVAL, "h_max too large for the level table");
    return TCW_OK;
}

}  // namespace

extern "C" int tcw_label_batch(tcw_ctx* c, int n, int count, const uint16_t* words, const int32_t* offsets,
                               const int32_t* kof, int h_max, uint64_t seed, float* features_dev, int32_t* labels_dev) {
    if (!c || !words || !offsets || !kof || !features_dev || !labels_dev || count < 1) return TCW_EINVAL;
    int rc = check_mitm_args(c, n, h_max);
    if (rc) return rc;
    // the words are read on the device exactly as these arrays describe them: check them here
    if (offsets[0] != 0) return fail(c, TCW_EINVAL, "offsets[0] must be 0");
    const uint32_t xi = xi_of(n);
    for (int i = 0; i < count; ++i) {
        const int64_t len = (int64_t)offsets[i + 1] - offsets[i];
        if (len < 0 || kof[i] < 0 || kof[i] > len) return fail(c, TCW_EINVAL, "offsets must not decrease and kof[i] <= word length");
        if (2 * (len - kof[i]) + kof[i] > 256) return fail(c, TCW_EINVAL, "a word is longer than 256 rotations once expanded");
    }
    for (int64_t j = 0; j < offsets[count]; ++j)
        if (words[j] < 1 || words[j] > xi) return fail(c, TCW_EINVAL, "Pauli code out of range 1..4^n - 1");
    const int R = 1 << (2 * n);
    const int64_t nw = offsets[count];
    uint16_t* dwords = nullptr;
    int32_t *doff = nullptr, *dk = nullptr, *rot = nullptr;
    uint32_t* phi = nullptr;
    void* scratch = nullptr;
    const int chunk = 1024, blocks = 256;
    auto cleanup = [&]() {
        for (void* q : {(void*)dwords, (void*)doff, (void*)dk, (void*)rot, (void*)phi, scratch})
            if (q) (void)hipFree(q);
    };
#define LB_TRY(expr)                         \
    do {                                     \
        hipError_t _e = (expr);              \
        if (_e != hipSuccess) {              \
            cleanup();                       \
            return hip_fail(c, _e, #expr);   \
        }                                    \
    } while (0)
    LB_TRY(hipMalloc(&dwords, nw * 2 + 2));
    LB_TRY(hipMalloc(&doff, (count + 1) * 4));
    LB_TRY(hipMalloc(&dk, count * 4));
    LB_TRY(hipMemcpyAsync(dwords, words, nw * 2, hipMemcpyHostToDevice, c->stream));
    LB_TRY(hipMemcpyAsync(doff, offsets, (count + 1) * 4, hipMemcpyHostToDevice, c->stream));
    LB_TRY(hipMemcpyAsync(dk, kof, count * 4, hipMemcpyHostToDevice, c->stream));
    LB_TRY(hipMalloc(&rot, chunk * 4));
    LB_TRY(hipMalloc(&phi, (size_t)chunk * R * R / 2 * 4));
    LB_TRY(hipMalloc(&scratch, tcw::build_batch_scratch_bytes(n, blocks)));
    const int h_id = mitm_split(n, h_max, count);
    LevelTable lt;
    if ((rc = build_level_table(c, n, h_id, seed, lt)) || (rc = clear_flag(c))) {
        cleanup();
        return rc;
    }
    for (int first = 0; first < count; first += chunk) {
        const int cnt = std::min(chunk, count - first);
        LB_TRY(tcw::build_batch(n, dwords, doff + first, dk + first, cnt, scratch, blocks, phi, rot,
                                features_dev + (size_t)first * R * R, c->flag, c->stream));
        LB_TRY(tcw::mitm_probe(n, lt.sp, phi, rot, cnt, 2 * h_max - h_id, lt.table, lt.lg, labels_dev + first,
                               c->stream));
    }
    int flag = 0;
    rc = read_flag(c, &flag);
    cleanup();
#undef LB_TRY
    if (rc) return rc;
    if (flag) return fail(c, TCW_EOVERFLOW, "target outside the int8 / int32 range or word too long");
    return TCW_OK;
}

extern "C" int tcw_min_tcount(tcw_ctx* c, const tcw_target* t, int h_max, uint64_t seed, int32_t* t_out) {
    if (!c || !t || !t_out) return TCW_EINVAL;
    int rc = check_mitm_args(c, t->n, h_max);
    if (rc) return rc;
    const int n = t->n;
    const int R = 1 << (2 * n);
    uint32_t* phi = nullptr;
    int32_t* dev_i32 = nullptr;  // [0] rot_e, [1] result
    auto cleanup = [&]() {
        if (phi) (void)hipFree(phi);
        if (dev_i32) (void)hipFree(dev_i32);
    };
    LevelTable lt;
    int32_t e_u = 0;
    int flag = 0;
    hipError_t err = hipMalloc(&phi, (size_t)R * R / 2 * 4 + 16);
    if (err == hipSuccess) err = hipMalloc(&dev_i32, 2 * sizeof(int32_t));
    if (err == hipSuccess) err = hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
    if (err == hipSuccess) err = tcw::exact_pack_phi(t->U, phi, c->flag, c->stream);
    if (err == hipSuccess) err = hipMemcpyAsync(&e_u, t->U.e, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
    if (err != hipSuccess) {
        cleanup();
        return hip_fail(c, err, "target packing");
    }
    if ((rc = read_flag(c, &flag))) {
        cleanup();
        return rc;
    }
    if (flag) {
        cleanup();
        return fail(c, TCW_EOVERFLOW, "target entry outside the int8 range (exponent too large)");
    }
    const int32_t rot_e = (int32_t)((30ll * e_u) % 61);
    err = hipMemcpyAsync(dev_i32, &rot_e, sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
    if (err != hipSuccess) {
        cleanup();
        return hip_fail(c, err, "rot_e upload");
    }
    const int h_id = mitm_split(n, h_max, 1);
    if ((rc = build_level_table(c, n, h_id, seed, lt))) {
        cleanup();
        return rc;
    }
    err = tcw::mitm_probe(n, lt.sp, phi, dev_i32, 1, 2 * h_max - h_id, lt.table, lt.lg, dev_i32 + 1, c->stream);
    if (err == hipSuccess) err = hipMemcpyAsync(t_out, dev_i32 + 1, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
    cleanup();
    if (err != hipSuccess) return hip_fail(c, err, "meet-in-the-middle probe");
    return TCW_OK;
}

extern "C" int tcw_mlp_train(tcw_mlp* m, const float* x, const int32_t* labels, int64_t count, int batch, int epochs,
                             float lr, float* last_epoch_loss) {
    if (!m || !x || !labels || count < 1 || batch < 1 || epochs < 1 || !(lr > 0)) return TCW_EINVAL;
    double tot = 0;
    int64_t nb = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        tot = 0;
        nb = 0;
        for (int64_t first = 0; first < count; first += batch) {
            const int b = (int)std::min<int64_t>(batch, count - first);
            float ls = 0;
            int rc = tcw_mlp_train_step(m, x + first * m->inp, labels + first, b, lr, &ls);
            if (rc) return rc;
            tot += ls * b;
            nb += b;
        }
    }
    if (last_epoch_loss) *last_epoch_loss = (float)(tot / (double)nb);
    return TCW_OK;
}
